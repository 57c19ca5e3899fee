"""Pins of the oracle's lattice geometry and initial configurations."""
import numpy as np
import pytest

from tests import inputs


def test_check_dims(orc):
    assert orc.check_dims((2, 2, 2, 2)) == 0
    assert orc.check_dims((8, 6, 4, 2)) == 0
    for bad in ((3, 4, 4, 4), (4, 4, 4, 1), (0, 4, 4, 4), (4, 4, 5, 4)):
        assert orc.check_dims(bad) == -1


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 6, 4), (6, 4, 2, 8)])
def test_neighbors_match_numpy_roll(orc, dims):
    # numpy's view: array indexed [t, z, y, x]; the neighbour of s along mu is
    # the site whose content np.roll(..., -1, axis) brings to s
    V = int(np.prod(dims))
    idx = np.arange(V).reshape(dims[::-1])
    for mu in range(4):
        axis = 3 - mu
        fwd = np.roll(idx, -1, axis=axis).ravel()
        bwd = np.roll(idx, +1, axis=axis).ravel()
        for s in range(V):
            assert orc.neighbor(dims, s, mu, +1) == fwd[s]
            assert orc.neighbor(dims, s, mu, -1) == bwd[s]
            # checkerboard: every nearest neighbour has the opposite parity
            assert orc.parity(dims, fwd[s]) != orc.parity(dims, s)


def test_cold_start(orc):
    dims = (4, 4, 4, 4)
    U = orc.cold(dims)
    assert np.array_equal(U[..., 0], np.ones((256, 4)))
    assert not U[..., 1:].any()
    assert orc.plaquette(dims, U) == (1.0, 1.0, 1.0)
    assert orc.polyakov(dims, U) == 1.0
    assert np.array_equal(orc.wilson(dims, U, 2, 3), np.ones((2, 3)))
    assert np.array_equal(orc.staple(dims, U, 17, 2), [6.0, 0, 0, 0])


def test_hot_start_is_haar(orc):
    # Haar measure (paper Sec. 2): uniform on S^3, so a0 has density
    # (2/pi) sqrt(1 - a0^2), <a0> = 0 and <a_i^2> = 1/4
    dims = (8, 8, 8, 8)
    U = orc.hot(dims, seed=2)
    a = U.reshape(-1, 4)
    N = a.shape[0]
    assert np.abs(np.linalg.norm(a, axis=1) - 1).max() < 1e-15
    assert abs(a[:, 0].mean()) < 5 * 0.5 / np.sqrt(N)
    for c in range(4):
        assert abs((a[:, c] ** 2).mean() - 0.25) < 5 * np.sqrt(1 / 8 - 1 / 16) / np.sqrt(N)
    edges = np.linspace(-1, 1, 41)
    cdf = lambda x: (x * np.sqrt(1 - x * x) + np.arcsin(x)) / np.pi + 0.5
    exp = N * np.diff(cdf(edges))
    hist = np.histogram(a[:, 0], edges)[0]
    assert ((hist - exp) ** 2 / exp).sum() < 80            # 39 dof
    # different seeds and lattice ids give different streams
    assert not np.array_equal(U, orc.hot(dims, seed=3))
    assert not np.array_equal(U, orc.hot(dims, seed=2, lat_id=1))
