"""Brute-force pins of the oracle's measurements on tiny lattices (paper
Sec. 2: mean plaquette, Polyakov loop, APE smearing, W(R,T)), with
non-abelian random links.

Each observable is computed here straight from its definition with 2x2
complex matrices, U = a0 1 + i a.sigma, on a [t, z, y, x] grid shifted by
numpy rolls; nothing is shared with the oracle's C code but the link
array.  Products of non-commuting matrices make every ordering, dagger and
neighbour of the definitions visible, which the abelian closed forms
cannot; 2^4 exercises every periodic wrap (x + mu = x - mu), the uneven
lattices loops longer than the extents.
"""
import numpy as np
import pytest

from tests import inputs

SIG = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], complex)
AX = {0: 3, 1: 2, 2: 1, 3: 0}   # direction -> axis of a [t, z, y, x] grid
DIMS = [(2, 2, 2, 2), (2, 4, 6, 4), (4, 2, 2, 6)]


def matrices(dims, U):
    """[V, mu, 4] quaternions -> [t, z, y, x, mu, 2, 2] complex matrices."""
    a = U.reshape(tuple(dims[::-1]) + (U.shape[1], 4))
    return (a[..., 0, None, None] * np.eye(2)
            + 1j * np.einsum("...k,kij->...ij", a[..., 1:], SIG))


def sh(M, mu, k=1):
    """M(x + k mu) as a grid over x."""
    return np.roll(M, -k, axis=AX[mu])


def dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def half_tr(M):
    return 0.5 * np.trace(M, axis1=-2, axis2=-1).real


def line(M, mu, n):
    """Product M(x) M(x + mu) ... M(x + (n-1) mu) at every x."""
    out = np.broadcast_to(np.eye(2, dtype=complex), M.shape).copy()
    for i in range(n):
        out = out @ sh(M, mu, i)
    return out


def wilson_loop(Msp, Mt, R, T):
    """1/(3V) sum over x and spatial mu of 1/2 Re Tr of the R x T loop
    S_mu(x;R) T(x+R mu;T) S_mu(x+T t;R)^dag T(x;T)^dag."""
    Tl = line(Mt, 3, T)
    tot = 0.0
    for mu in range(3):
        S = line(Msp[..., mu, :, :], mu, R)
        tot += half_tr(S @ sh(Tl, mu, R) @ dag(sh(S, 3, T)) @ dag(Tl)).mean()
    return tot / 3


def ape_step(Msp, alpha):
    """One APE step of the spatial links from the previous ones: the four
    staples of the two other spatial directions, then the SU(2)
    projection of (1 - alpha) U + alpha/4 * sum (a real multiple of an
    SU(2) matrix: divide by the square root of its determinant)."""
    out = np.empty_like(Msp)
    for mu in range(3):
        U = Msp[..., mu, :, :]
        s = np.zeros_like(U)
        for nu in range(3):
            if nu == mu:
                continue
            N = Msp[..., nu, :, :]
            s += N @ sh(U, nu) @ dag(sh(N, mu))
            Nb = sh(N, nu, -1)
            s += dag(Nb) @ sh(U, nu, -1) @ sh(Nb, mu)
        w = (1 - alpha) * U + 0.25 * alpha * s
        out[..., mu, :, :] = w / np.sqrt(np.linalg.det(w).real)[..., None, None]
    return out


@pytest.mark.parametrize("dims", DIMS)
def test_plaquette_brute_force(orc, dims):
    U = inputs.random_config(dims, 31)
    M = matrices(dims, U)
    sp = tp = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Mu, Nu = M[..., mu, :, :], M[..., nu, :, :]
            p = half_tr(Mu @ sh(Nu, mu) @ dag(sh(Mu, nu)) @ dag(Nu)).mean()
            if nu == 3:
                tp += p / 3
            else:
                sp += p / 3
    tot, s, t = orc.plaquette(dims, U)
    assert abs(s - sp) < 1e-13 and abs(t - tp) < 1e-13
    assert abs(tot - 0.5 * (sp + tp)) < 1e-13


@pytest.mark.parametrize("dims", DIMS)
def test_polyakov_brute_force(orc, dims):
    U = inputs.random_config(dims, 32)
    Mt = matrices(dims, U)[..., 3, :, :]
    P = np.broadcast_to(np.eye(2, dtype=complex), Mt.shape[1:]).copy()
    for t in range(dims[3]):
        P = P @ Mt[t]
    assert abs(orc.polyakov(dims, U) - half_tr(P).mean()) < 1e-13


@pytest.mark.parametrize("dims", DIMS)
def test_wilson_loops_brute_force(orc, dims):
    U = inputs.random_config(dims, 33)
    M = matrices(dims, U)
    for R in range(1, dims[0] + 2):
        for T in range(1, dims[3] + 2):
            ref = wilson_loop(M[..., :3, :, :], M[..., 3, :, :], R, T)
            assert abs(orc.wilson_rt(dims, U, R, T) - ref) < 1e-13, (R, T)


@pytest.mark.parametrize("dims", DIMS)
def test_ape_and_smeared_wilson_loops_brute_force(orc, dims):
    U = inputs.random_config(dims, 34)
    M = matrices(dims, U)
    alpha, nsteps = 0.55, 3
    S = M[..., :3, :, :]
    for _ in range(nsteps):
        S = ape_step(S, alpha)
    So = orc.ape(dims, U, alpha, nsteps)
    assert np.abs(matrices(dims, So) - S).max() < 1e-13
    for R, T in ((1, 1), (2, 1), (1, dims[3]), (dims[0] + 1, 2)):
        ref = wilson_loop(S, M[..., 3, :, :], R, T)
        assert abs(orc.wilson_rt(dims, U, R, T, So) - ref) < 1e-13, (R, T)
