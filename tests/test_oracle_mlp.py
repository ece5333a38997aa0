"""Pins of the network oracle: gradients against central finite differences
(FP64), the BF16 rounding against an independent bit-level implementation,
and the features' invariances.  CPU only."""
import numpy as np
import pytest


def rand_params(seed, scale=0.4):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(size=1313) * scale


def test_gradient_matches_finite_differences(orc):
    P = rand_params(1)
    rng = np.random.Generator(np.random.PCG64(2))
    X = rng.normal(size=(12, 6))
    T = rng.normal(size=12)
    g, L = orc.mlp_loss_grad(P, X, T, emulate=False)
    eps = 1e-6
    idx = rng.choice(1313, size=200, replace=False).tolist() + [1312, 0, 192, 224, 1248, 1280]
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += eps
        Pm[i] -= eps
        _, Lp = orc.mlp_loss_grad(Pp, X, T, emulate=False)
        _, Lm = orc.mlp_loss_grad(Pm, X, T, emulate=False)
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(fd)), (i, fd, g[i])
    # the loss is the mean squared error of the forward outputs
    y = orc.mlp_forward(P, X, emulate=False)
    assert np.isclose(L, np.mean((y - T) ** 2), rtol=1e-14)


def _bf16_reference(v: float) -> float:
    # float32 bits, round the low 16 bits to nearest even, truncate
    b = int(np.float32(v).view(np.uint32))
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return float(np.uint32(b).view(np.float32))


def test_bf16_rounding():
    rng = np.random.Generator(np.random.PCG64(3))
    import oracle

    for v in np.concatenate([rng.normal(size=2000) * np.exp(rng.uniform(-20, 20, 2000)),
                             [1.0, -1.0, 1 + 2**-8, 1 + 2**-9, 1 + 3 * 2**-9, 255.5, 0.0]]):
        v32 = float(np.float32(v))  # the GPU rounds FP32 values
        assert oracle.mlp_bf16(v32) == _bf16_reference(v32), v


def test_features_invariances(orc):
    """Scale and Galilean invariance, and the target of identical states."""
    rng = np.random.Generator(np.random.PCG64(4))
    for _ in range(50):
        rL, rR, pL, pR = np.exp(rng.uniform(-2, 1, 4))
        uL, uR = rng.uniform(-1, 1, 2)
        ps = np.exp(rng.uniform(-2, 1))
        x, t = orc.mlp_features([rL, uL, pL, rR, uR, pR, ps])
        a, b, s = rng.uniform(0.1, 10, 3)
        vel = np.sqrt(b / a)  # velocity unit of the rescaled problem
        shift = rng.uniform(-5, 5)
        x2, t2 = orc.mlp_features([a * rL, vel * uL + shift, b * pL, a * rR, vel * uR + shift,
                                   b * pR, b * ps])
        np.testing.assert_allclose(x2, x, atol=1e-12)
        assert abs(t2 - t) < 1e-12
        np.testing.assert_allclose(x[3:], -x[:3], atol=1e-15)
    x, t = orc.mlp_features([1.3, 0.2, 0.7, 1.3, 0.2, 0.7, 0.7])
    np.testing.assert_allclose(x, 0, atol=1e-15)
    assert abs(t) < 1e-15


def test_emulated_forward_close_to_exact(orc):
    """BF16 rounding perturbs outputs by about its precision, not more."""
    P = rand_params(5, 0.2)
    X = np.random.Generator(np.random.PCG64(6)).normal(size=(200, 6))
    ye = orc.mlp_forward(P, X, emulate=True)
    y = orc.mlp_forward(P, X, emulate=False)
    assert np.max(np.abs(ye - y)) < 0.05 * (1 + np.max(np.abs(y)))
    assert np.max(np.abs(ye - y)) > 0  # rounding is applied
