"""Pins of the oracle's heat bath (paper Sec. 2) and over-relaxation.

* staple: the change of the total Wilson action when one link is replaced
  equals -(beta/2) Re Tr[(W - U) V] (the definition of the staple V),
  checked with 2x2 complex matrices against the independently pinned
  plaquette, on lattices where every periodic wrap occurs (2^4 included);
* sampler: chi^2 of delta = 1 - a0 against the closed-form density
  sqrt(1 - a0^2) exp(alpha a0) (normaliser pi I1(alpha)/alpha) and the
  mean a0 = I2(alpha)/I1(alpha), for KP, Creutz and the hybrid;
* one link: X = U' W (W = V/k) has a0 from the same law and an isotropic
  vector part;
* checkerboard: the links of one (mu, parity) class are independent, so any
  visiting order gives bitwise the same sweep;
* strong coupling: <1/2 Tr U_P> = I2(beta)/I1(beta) + O(u^5);
* over-relaxation preserves the action exactly and is gauge covariant.
"""
import numpy as np
import pytest
from scipy import integrate, special, stats

from tests import inputs

SIG = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]], complex),
       np.array([[1, 0], [0, -1]], complex)]


def mat(a):
    return a[0] * np.eye(2) + 1j * (a[1] * SIG[0] + a[2] * SIG[1] + a[3] * SIG[2])


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 4, 6, 4), (4, 4, 4, 4)])
def test_staple_local_action_identity(orc, dims):
    V = int(np.prod(dims))
    U = inputs.random_config(dims, 21)
    rng = np.random.default_rng(22)
    P0 = orc.plaquette(dims, U)[0] * 6 * V
    for _ in range(12):
        s, mu = int(rng.integers(V)), int(rng.integers(4))
        St = orc.staple(dims, U, s, mu)
        W = rng.standard_normal(4)
        W /= np.linalg.norm(W)
        U2 = U.copy()
        U2[s, mu] = W
        dP = orc.plaquette(dims, U2)[0] * 6 * V - P0
        pred = 0.5 * np.trace((mat(W) - mat(U[s, mu])) @ mat(St)).real
        assert abs(dP - pred) < 1e-11


def target_pdf(delta, alpha):
    """density of delta = 1 - a0: sqrt(delta(2-delta)) exp(-alpha delta)/Z"""
    Z = np.pi * special.ive(1, alpha) / alpha
    return np.sqrt(np.clip(delta * (2 - delta), 0, None)) * np.exp(-alpha * delta) / Z


def test_normaliser_closed_form():
    for alpha in (0.25, 1.0, 6.0, 30.0):
        num = integrate.quad(lambda d: np.sqrt(d * (2 - d)) * np.exp(-alpha * d), 0, 2,
                             limit=200)[0]
        assert abs(num - np.pi * special.ive(1, alpha) / alpha) < 1e-10


def chi2_delta(delta, alpha, nbins=40):
    hi = min(2.0, 25.0 / alpha)
    edges = np.linspace(0, hi, nbins + 1)
    exp = np.array([integrate.quad(target_pdf, a, b, args=(alpha,))[0]
                    for a, b in zip(edges[:-1], edges[1:])])
    tail = 1 - exp.sum()
    obs = np.histogram(delta, edges)[0]
    exp = exp * delta.size
    obs = np.append(obs, (delta >= hi).sum())
    exp = np.append(exp, max(tail, 0) * delta.size)
    keep = exp > 5
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    return stats.chi2.sf(chi2, keep.sum() - 1)


@pytest.mark.parametrize("alpha", [0.25, 1.0, 2.0, 6.0, 15.0, 60.0])
@pytest.mark.parametrize("sampler", ["KP", "CREUTZ", "HYBRID"])
def test_sampler_distribution(orc, alpha, sampler):
    if sampler == "KP" and alpha < 1:
        n = 40000
    else:
        n = 100000
    d, tries = orc.sample_many(alpha, getattr(orc, sampler), 5, n)
    assert (d > 0).all() and (d < 2).all() and (tries >= 1).all()
    assert chi2_delta(d, alpha) > 1e-4
    a0 = 1 - d
    mean = special.ive(2, alpha) / special.ive(1, alpha)
    assert abs(a0.mean() - mean) < 5 * a0.std() / np.sqrt(n)


@pytest.mark.parametrize("alpha,sampler", [(0.5, "HYBRID"), (2.0, "HYBRID"), (3.0, "HYBRID"),
                                           (12.0, "HYBRID"), (12.0, "CREUTZ")])
def test_link_draw_direction(orc, alpha, sampler):
    """X = (a0, a): |X| = 1, a0 from the closed-form law, and a/|a| uniform
    on the sphere (cos theta and phi uniform) independently of a0."""
    n = 30000
    X = np.array([orc.sample_link(alpha, getattr(orc, sampler), 9, [i, 3, 5])[0]
                  for i in range(n)])
    assert np.abs(np.linalg.norm(X, axis=1) - 1).max() < 1e-14
    assert chi2_delta(1 - X[:, 0], alpha) > 1e-4
    y = X[:, 1:] / np.linalg.norm(X[:, 1:], axis=1, keepdims=True)
    edges = np.linspace(-1, 1, 21)
    for comp in range(3):       # each component of a uniform unit vector is uniform
        h = np.histogram(y[:, comp], edges)[0]
        assert stats.chisquare(h).pvalue > 1e-4, comp
    phi = np.arctan2(y[:, 1], y[:, 0])
    assert stats.chisquare(np.histogram(phi, np.linspace(-np.pi, np.pi, 21))[0]).pvalue > 1e-4
    q = np.quantile(X[:, 0], [0, 0.25, 0.5, 0.75, 1])
    for lo, hi in zip(q[:-1], q[1:]):
        sel = (X[:, 0] >= lo) & (X[:, 0] <= hi)
        for comp in range(3):
            m = (y[sel, comp] ** 2).mean()
            assert abs(m - 1 / 3) < 5 * np.sqrt(4 / 45 / sel.sum()), (lo, comp, m)
        assert abs((y[sel, 0] * y[sel, 2]).mean()) < 5 * np.sqrt(1 / 15 / sel.sum())


def test_sampler_fp32_uniforms(orc):
    d, _ = orc.sample_many(8.0, orc.HYBRID, 6, 100000, ubits=23)
    assert chi2_delta(d, 8.0) > 1e-4


def test_sampler_tiny_alpha_terminates(orc):
    # alpha -> 0 is Haar: a0 density (2/pi) sqrt(1 - a0^2)
    for alpha in (0.0, 1e-30, 1e-12):
        d, t = orc.sample_many(alpha, orc.HYBRID, 7, 20000)
        a0 = 1 - d
        assert abs(a0.mean()) < 0.02 and abs((a0 ** 2).mean() - 0.25) < 0.01
        assert t.mean() < 1.5


def test_acceptance_rates(orc):
    # KP is the efficient branch at large alpha, Creutz at small alpha
    _, t = orc.sample_many(6.0, orc.KP, 1, 50000)
    assert 1 / t.mean() > 0.9
    _, t = orc.sample_many(0.25, orc.CREUTZ, 1, 50000)
    assert 1 / t.mean() > 0.7


def test_single_link_update_distribution(orc):
    dims = (4, 4, 4, 4)
    U = inputs.random_config(dims, 23)
    s, mu, beta = 77, 2, 2.4
    St = orc.staple(dims, U, s, mu)
    k = np.linalg.norm(St)
    Wt = St / k
    M = 30000
    X = np.zeros((M, 4))
    for sweep in range(M):
        U2 = U.copy()
        orc.heatbath_link(dims, U2, s, mu, beta, seed=1, sweep=sweep)
        u = U2[s, mu]
        assert abs(np.linalg.norm(u) - 1) < 1e-15
        X[sweep] = orc.qmul(u, Wt)
    alpha = beta * k
    assert chi2_delta(1 - X[:, 0], alpha) > 1e-4
    mean = special.ive(2, alpha) / special.ive(1, alpha)
    assert abs(X[:, 0].mean() - mean) < 5 * X[:, 0].std() / np.sqrt(M)
    r2 = (1 - (X[:, 0] ** 2).mean()) / 3
    for c in (1, 2, 3):
        assert abs(X[:, c].mean()) < 5 * np.sqrt(r2 / M)
        assert abs((X[:, c] ** 2).mean() - r2) < 0.02 * r2 + 5 * r2 * np.sqrt(2 / M)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 6, 4)])
def test_checkerboard_order_independence(orc, dims):
    V = int(np.prod(dims))
    U = inputs.random_config(dims, 24)
    A, B = U.copy(), U.copy()
    ta = np.zeros(4 * V, np.uint32)
    tb = np.zeros(4 * V, np.uint32)
    orc.heatbath_sweep(dims, A, 2.3, seed=3, sweep=0, trace=ta)
    orc.heatbath_sweep(dims, B, 2.3, seed=3, sweep=0, trace=tb,
                       order=inputs.permutation(V, 25))
    assert np.array_equal(A, B) and np.array_equal(ta, tb)
    # every link changed, and each was accepted after >= 1 try
    assert (A != U).any(axis=2).all() and ((ta & 0x7FFFFFFF) >= 1).all()


def test_unitarity_after_sweeps(orc):
    dims = (4, 4, 4, 4)
    U = orc.hot(dims, 1)
    for sw in range(5):
        orc.heatbath_sweep(dims, U, 2.5, seed=1, sweep=sw)
    assert orc.max_unit_defect(dims, U) < 1e-14


def jackknife_mean(series, bin_size=10):
    nb = len(series) // bin_size
    b = np.asarray(series[: nb * bin_size]).reshape(nb, bin_size).mean(axis=1)
    m = b.mean()
    jk = (b.sum() - b) / (nb - 1)
    return m, np.sqrt((nb - 1) / nb * ((jk - m) ** 2).sum())


@pytest.mark.parametrize("beta", [0.3, 0.6])
def test_strong_coupling(orc, beta):
    dims = (4, 4, 4, 4)
    U = orc.hot(dims, 3)
    P = []
    for sw in range(1500):
        orc.heatbath_sweep(dims, U, beta, seed=4, sweep=sw)
        if sw >= 50:
            P.append(orc.plaquette(dims, U)[0])
    m, e = jackknife_mean(P)
    u = special.ive(2, beta) / special.ive(1, beta)
    assert abs(m - u) < 4 * e + 6 * u ** 5, (m, e, u)


def test_weak_coupling_loose(orc):
    dims = (4, 4, 4, 4)
    U = orc.cold(dims)
    beta = 8.0
    P = []
    for sw in range(300):
        orc.heatbath_sweep(dims, U, beta, seed=5, sweep=sw)
        if sw >= 50:
            P.append(orc.plaquette(dims, U)[0])
    assert abs(np.mean(P) - (1 - 3 / (4 * beta))) < 0.01


def test_overrelaxation_preserves_action(orc):
    dims = (4, 4, 2, 6)
    U = orc.hot(dims, 8)
    for sw in range(3):
        orc.heatbath_sweep(dims, U, 2.3, seed=8, sweep=sw)
    p0 = orc.plaquette(dims, U)[0]
    R = U.copy()
    orc.overrelax_sweep(dims, R)
    assert np.abs(R - U).max() > 0.1
    assert abs(orc.plaquette(dims, R)[0] - p0) < 1e-13
    # gauge covariance, link by link
    G = U.copy()
    orc.gauge_transform(dims, G, 31)
    orc.overrelax_sweep(dims, G)
    orc.gauge_transform(dims, R, 31)
    assert np.abs(G - R).max() < 1e-13
