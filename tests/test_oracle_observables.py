"""Pins of the oracle's measurements: plaquette, Polyakov loop, Wilson loops,
APE smearing.

Closed forms come from the abelian (U(1)) embedding U = exp(i theta sigma_3)
= (cos theta, 0, 0, sin theta): products of such links add angles, so every
loop trace is the cosine of its oriented angle sum, computed here with
numpy rolls.  Non-abelian ordering is pinned by gauge invariance, which a
transposed product or a wrong neighbour breaks.
"""
import numpy as np
import pytest

from tests import inputs

AX = {0: 3, 1: 2, 2: 1, 3: 0}   # direction -> numpy axis of a [t, z, y, x] array


def u1_config(dims, seed):
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    th = rng.uniform(-np.pi, np.pi, size=(V, 4))
    U = np.zeros((V, 4, 4))
    U[..., 0] = np.cos(th)
    U[..., 3] = np.sin(th)
    return U, th.reshape(tuple(dims[::-1]) + (4,))


def sh(a, mu, k=1):
    """a(s + k mu) as an array over s"""
    return np.roll(a, -k, axis=AX[mu])


DIMS = [(4, 4, 4, 4), (2, 4, 6, 4), (6, 2, 4, 8)]


@pytest.mark.parametrize("dims", DIMS)
def test_plaquette_u1_closed_form(orc, dims):
    U, th = u1_config(dims, 5)
    sp, tp = [], []
    for mu in range(4):
        for nu in range(mu + 1, 4):
            ang = th[..., mu] + sh(th[..., nu], mu) - sh(th[..., mu], nu) - th[..., nu]
            (tp if nu == 3 else sp).append(np.cos(ang).mean())
    tot, s, t = orc.plaquette(dims, U)
    assert abs(s - np.mean(sp)) < 1e-13 and abs(t - np.mean(tp)) < 1e-13
    assert abs(tot - (np.mean(sp) + np.mean(tp)) / 2) < 1e-13


@pytest.mark.parametrize("dims", DIMS)
def test_polyakov_u1_closed_form(orc, dims):
    U, th = u1_config(dims, 6)
    ref = np.cos(th[..., 3].sum(axis=0)).mean()
    assert abs(orc.polyakov(dims, U) - ref) < 1e-13


def u1_wilson(th, R, T):
    vals = []
    for mu in range(3):
        a = sum(sh(th[..., mu], mu, i) for i in range(R))
        b = sum(sh(sh(th[..., 3], mu, R), 3, j) for j in range(T))
        c = sum(sh(sh(th[..., mu], 3, T), mu, i) for i in range(R))
        d = sum(sh(th[..., 3], 3, j) for j in range(T))
        vals.append(np.cos(a + b - c - d).mean())
    return np.mean(vals)


@pytest.mark.parametrize("dims", [(4, 4, 4, 6), (6, 2, 4, 8)])
def test_wilson_u1_closed_form(orc, dims):
    U, th = u1_config(dims, 7)
    Rmax, Tmax = 3, 4
    W = orc.wilson(dims, U, Rmax, Tmax)
    for R in range(1, Rmax + 1):
        for T in range(1, Tmax + 1):
            assert abs(W[R - 1, T - 1] - u1_wilson(th, R, T)) < 1e-13


def test_wilson_11_is_temporal_plaquette(orc):
    dims = (4, 6, 4, 6)
    U = inputs.random_config(dims, 8)
    W = orc.wilson(dims, U, 1, 1)
    assert abs(W[0, 0] - orc.plaquette(dims, U)[2]) < 1e-14


@pytest.mark.parametrize("dims", [(4, 4, 4, 6), (2, 4, 2, 4)])
def test_ape_u1_closed_form(orc, dims):
    U, th = u1_config(dims, 9)
    alpha, n = 0.55, 3
    z = np.exp(1j * th[..., :3])
    for _ in range(n):
        new = np.empty_like(z)
        for mu in range(3):
            st = 0
            for nu in range(3):
                if nu == mu:
                    continue
                st = st + z[..., nu] * sh(z[..., mu], nu) * np.conj(sh(z[..., nu], mu))
                zb = sh(z[..., nu], nu, -1)
                st = st + np.conj(zb) * sh(z[..., mu], nu, -1) * sh(sh(z[..., nu], nu, -1), mu)
            w = (1 - alpha) * z[..., mu] + alpha / 4 * st
            new[..., mu] = w / np.abs(w)
        z = new
    S = orc.ape(dims, U, alpha, n)
    zz = z.reshape(-1, 3)
    assert np.abs(S[..., 0] - zz.real).max() < 1e-13
    assert np.abs(S[..., 3] - zz.imag).max() < 1e-13
    assert not S[..., 1:3].any()


def test_ape_special_cases(orc):
    dims = (4, 4, 4, 4)
    U = inputs.random_config(dims, 10)
    assert np.abs(orc.ape(dims, U, 0.0, 3) - U[:, :3, :]).max() < 1e-15   # alpha = 0
    assert np.array_equal(orc.ape(dims, orc.cold(dims), 0.7, 5), orc.cold(dims)[:, :3, :])
    S = orc.ape(dims, U, 0.7, 5)
    assert np.abs(np.linalg.norm(S, axis=2) - 1).max() < 1e-14


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 4)])
def test_gauge_invariance(orc, dims):
    U = inputs.random_config(dims, 11)
    G = U.copy()
    orc.gauge_transform(dims, G, seed=99)
    assert np.abs(G - U).max() > 0.1
    for a, b in zip(orc.plaquette(dims, U), orc.plaquette(dims, G)):
        assert abs(a - b) < 1e-14
    assert abs(orc.polyakov(dims, U) - orc.polyakov(dims, G)) < 1e-14
    Rm, Tm = min(dims[:3]), min(dims[3], 3)
    assert np.abs(orc.wilson(dims, U, Rm, Tm) - orc.wilson(dims, G, Rm, Tm)).max() < 1e-14
    # APE smearing is gauge covariant: smear(g U) = g smear(U), link by link
    S, SG = orc.ape(dims, U, 0.6, 4), orc.ape(dims, G, 0.6, 4)
    T = U.copy()
    T[:, :3, :] = S
    orc.gauge_transform(dims, T, seed=99)
    assert np.abs(T[:, :3, :] - SG).max() < 1e-13
    Ws = orc.wilson(dims, U, Rm, Tm, S)
    assert np.abs(Ws - orc.wilson(dims, G, Rm, Tm, SG)).max() < 1e-14


def test_polyakov_center_flip(orc):
    dims = (4, 4, 4, 6)
    U = inputs.random_config(dims, 12)
    F = U.copy()
    Ns = 64
    F[:Ns, 3, :] *= -1          # U_3(x, t=0) -> -U_3(x, t=0)
    assert orc.polyakov(dims, F) == -orc.polyakov(dims, U)
    assert abs(orc.plaquette(dims, F)[0] - orc.plaquette(dims, U)[0]) < 1e-15
