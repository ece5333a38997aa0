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
        # the right state's slots are the left state's negated
        np.testing.assert_allclose(x[4:], -x[:2], atol=1e-15)
        # mirror image (left and right swapped, velocities negated): the same
        # problem reflected, so a, b change sign and w, q and the target stay
        xm, tm = orc.mlp_features([rR, -uR, pR, rL, -uL, pL, ps])
        np.testing.assert_allclose(xm, [-x[0], -x[1], x[2], x[3], -x[4], -x[5]], atol=1e-12)
        assert abs(tm - t) < 1e-12
    # identical states: every feature is 0, and the two-rarefaction guess is
    # the state's own pressure
    x, t = orc.mlp_features([1.3, 0.2, 0.7, 1.3, 0.2, 0.7, 0.7])
    np.testing.assert_allclose(x, 0, atol=1e-15)
    assert abs(t) < 1e-15


def test_feature_q_is_the_exact_star_pressure_of_two_rarefactions(orc):
    """q = ln(p_ptr / p_bar) with p_ptr the two-rarefaction guess: where both
    waves are rarefactions that guess is the exact star pressure, so q equals
    ln(p*/p_bar) of the independent bracketing solver (tests/exact_riemann.py);
    the target is the log of the record's p* over that guess."""
    import exact_riemann as ex

    rng = np.random.Generator(np.random.PCG64(17))
    n = 0
    while n < 200:
        rL, rR, pL, pR = np.exp(rng.uniform(-1.5, 1.5, 4))
        cL, cR = np.sqrt(1.4 * pL / rL), np.sqrt(1.4 * pR / rR)
        uL = rng.uniform(-0.5, 0.5)
        uR = uL + rng.uniform(0.0, 1.5) * (cL + cR)  # separating: two rarefactions
        ps, _ = ex.star((rL, uL, pL), (rR, uR, pR))
        if not (ps < min(pL, pR)) or ps < 1e-6 * max(pL, pR):
            continue
        x, t = orc.mlp_features([rL, uL, pL, rR, uR, pR, 2.0 * ps])
        pbar = np.sqrt(pL * pR)
        assert abs(x[3] - np.log(ps / pbar)) < 1e-11
        assert abs(t - np.log(2.0)) < 1e-11
        n += 1


def test_emulated_forward_close_to_exact(orc):
    """BF16 rounding perturbs outputs by about its precision, not more."""
    P = rand_params(5, 0.2)
    X = np.random.Generator(np.random.PCG64(6)).normal(size=(200, 6))
    ye = orc.mlp_forward(P, X, emulate=True)
    y = orc.mlp_forward(P, X, emulate=False)
    assert np.max(np.abs(ye - y)) < 0.05 * (1 + np.max(np.abs(y)))
    assert np.max(np.abs(ye - y)) > 0  # rounding is applied


def _routing_params():
    """Hand-built network whose output has a closed form: units 0-5 of layer 1
    pass x_k, units 6-11 pass -x_k; layer 2 permutes the units (unit i reads
    unit perm[i]); layer 3 weighs unit i by (i + 1) / 8."""
    P = np.zeros(1313)
    for k in range(6):
        P[0 + k * 6 + k] = 1.0          # W1[k][k]
        P[0 + (6 + k) * 6 + k] = -1.0   # W1[6+k][k]
    perm = [(5 * i + 3) % 32 for i in range(32)]
    for i in range(32):
        P[224 + i * 32 + perm[i]] = 1.0  # W2[i][perm[i]]
        P[1280 + i] = (i + 1) / 8.0      # W3[i]
    P[1312] = 0.25                       # b3
    return P, perm


def test_forward_closed_form(orc):
    """Routing network: y = b3 + sum_i w3_i relu(a1[perm[i]]) with
    a1 = (relu(x), relu(-x), 0, ...), evaluated unit by unit."""
    P, perm = _routing_params()
    rng = np.random.Generator(np.random.PCG64(7))
    X = np.round(rng.normal(size=(40, 6)) * 8) / 8  # exactly representable in BF16
    for emulate in (False, True):
        y = orc.mlp_forward(P, X, emulate=emulate)
        for x, yv in zip(X, y):
            a1 = [max(v, 0.0) for v in x] + [max(-v, 0.0) for v in x] + [0.0] * 20
            expect = 0.25 + sum((i + 1) / 8.0 * a1[perm[i]] for i in range(32))
            assert yv == expect, (x, yv, expect)


def test_emulated_gradient_exact_when_representable(orc):
    """With weights, inputs and residuals that BF16 holds exactly, the
    emulated gradient equals the exact one (itself pinned by finite
    differences), so the emulation only rounds, it does not reroute."""
    P, _ = _routing_params()
    P[192:224] = 0.125  # b1
    rng = np.random.Generator(np.random.PCG64(8))
    X = np.round(rng.normal(size=(4, 6)) * 4) / 4
    y = orc.mlp_forward(P, X, emulate=False)
    T = y - np.array([0.5, -0.25, 1.0, 0.125])  # residuals y - t
    ge, Le = orc.mlp_loss_grad(P, X, T, emulate=True)
    g, L = orc.mlp_loss_grad(P, X, T, emulate=False)
    assert Le == L
    np.testing.assert_array_equal(ge, g)
    assert np.count_nonzero(g[224:1248]) > 0 and np.count_nonzero(g[0:192]) > 0


def test_emulated_error_signals_are_bf16(orc):
    """In the emulated backward pass the error signals entering a matrix
    product are BF16 values: with x_0 = 1 and a layer-1 unit that passes x_0
    (so a1 = 1 there), the W2 column of that unit holds bf16(dL/dz2) and the
    first W1 column holds bf16(dL/dz1)."""
    import oracle

    P = rand_params(9, 0.4)
    P[0:6] = [1.0, 0, 0, 0, 0, 0]  # W1[0] passes x_0
    P[192] = 0.0                   # b1[0]
    rng = np.random.Generator(np.random.PCG64(10))
    for trial in range(20):
        X = np.concatenate([[1.0], np.round(rng.normal(size=5) * 16) / 16]).reshape(1, 6)
        T = rng.normal(size=1)
        g, _ = orc.mlp_loss_grad(P, X, T, emulate=True)
        col_w2 = g[224:1248].reshape(32, 32)[:, 0]  # dL/dW2[i][0] = bf16(gz2_i) * a1[0]
        col_w1 = g[0:192].reshape(32, 6)[:, 0]      # dL/dW1[k][0] = bf16(gz1_k) * 1
        for v in np.concatenate([col_w2, col_w1]):
            assert oracle.mlp_bf16(v) == v, (trial, v)
        assert np.count_nonzero(col_w2) > 0 and np.count_nonzero(col_w1) > 0
