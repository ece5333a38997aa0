"""The paper's OpenMP parallelisations of a time step (fine grain, coarse
grain with the neighbour busy-wait barrier, subdomain tasks with
interface-buffer dependencies) give the serial oracle step bitwise, for every
boundary type, ragged decompositions, thread counts that do not divide the
grid, and the other options.  CPU only."""
import numpy as np
import pytest

from paper_2106_13465_amd import inputs

SCHEMES = [0, 1, 2]


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("bc", [1, 2, 3])
def test_schemes_equal_serial_step(orc, scheme, bc):
    for nx, ny in [(37, 29), (17, 90), (64, 48)]:
        U = inputs.random_states(nx, ny, seed=60 + nx, rough=0.7)
        c = orc.cfg(bc=bc)
        ref = U.copy()
        for _ in range(2):
            orc.step(ref, c)
        for threads in (1, 2, 3, 4, 6):
            V = U.copy()
            for _ in range(2):
                orc.step_scheme(V, c, scheme, threads)
            assert np.array_equal(V, ref), (nx, ny, threads, orc.scheme_decomposition(threads, nx, ny))


@pytest.mark.parametrize("scheme", [1, 2])
def test_schemes_with_options_and_scalars(orc, scheme):
    U = inputs.random_states(41, 33, seed=70, rough=0.7)
    V0 = inputs.with_scalars(U, inputs.random_scalars(41, 33, seed=8))
    for opts in ({"riemann": 1, "limiter": 1}, {"riemann": 2, "limiter": 2}):
        c = orc.cfg(bc=3, nscalars=1, **opts)
        ref = V0.copy()
        orc.step(ref, c)
        V = V0.copy()
        orc.step_scheme(V, c, scheme, 4)
        assert np.array_equal(V, ref), opts


def test_decomposition(orc):
    assert orc.scheme_decomposition(16, 1000, 1000) == (4, 4)
    assert orc.scheme_decomposition(8, 1000, 500) in ((4, 2),)
    assert orc.scheme_decomposition(6, 2, 1000) == (1, 6)  # 2 x 167 cells beats 1 x 333
    px, py = orc.scheme_decomposition(7, 50, 50)
    assert px * py == 7
