"""CPU check of the FP32 parity helper: the 18 staple links it lists for
(s, mu) are exactly the links the oracle's staple depends on."""
import numpy as np

from tests import inputs, parity_util


def test_staple_links_match_oracle(orc):
    dims = (4, 2, 6, 4)
    V = int(np.prod(dims))
    U = inputs.random_config(dims, 51)
    rng = np.random.default_rng(52)
    for mu in range(4):
        S, D = parity_util.staple_links(dims, mu)
        for s in rng.integers(0, V, 6):
            listed = set(zip(S[:, s].tolist(), D.tolist()))
            assert len(listed) == 18 or dims[1] == 2   # extent 2 repeats sites
            base = orc.staple(dims, U, s, mu)
            for site in range(V):
                for nu in range(4):
                    W = U.copy()
                    W[site, nu] = [0.0, 1.0, 0.0, 0.0]
                    changed = np.abs(orc.staple(dims, W, s, mu) - base).max() > 1e-12
                    assert changed == ((site, nu) in listed), (mu, s, site, nu)


def test_downstream_matches_brute_force(orc):
    dims = (2, 4, 2, 4)
    V = int(np.prod(dims))
    rng = np.random.default_rng(53)
    flips = np.zeros((V, 4), bool)
    flips[rng.integers(0, V, 3), rng.integers(0, 4, 3)] = True
    par = parity_util.parity_array(dims)
    fast = parity_util.downstream_of_flips(dims, flips, par)
    taint = flips.copy()
    for mu in range(4):
        S, D = parity_util.staple_links(dims, mu)
        for p in (0, 1):
            for s in range(V):
                if par[s] != p:
                    continue
                if any(taint[S[k, s], D[k]] for k in range(18)):
                    taint[s, mu] = True
    assert np.array_equal(fast, taint)
    assert taint.sum() > flips.sum()


def test_staple_link_ids_and_update_order(orc):
    """The per-link staple list equals the vectorised one, and the links a
    sweep updates before class (mu, p) are exactly the earlier classes."""
    dims = (4, 2, 6, 4)
    par = parity_util.parity_array(dims)
    for mu in range(4):
        S, D = parity_util.staple_links(dims, mu)
        for s in (0, 7, 33, 190):
            assert sorted(parity_util.staple_link_ids(orc, dims, s, mu)) == sorted(zip(S[:, s].tolist(), D.tolist()))
        for p in (0, 1):
            m = parity_util.link_before_mask(par, mu, p)
            for nu in range(4):
                for q in (0, 1):
                    assert m[par == q, nu].all() == (2 * nu + q < 2 * mu + p)
                    assert m[par == q, nu].any() == (2 * nu + q < 2 * mu + p)


def test_fp32_bound_closed_form(orc):
    """Cold 2^4 lattice: every staple is six identity products (k = 6); for a
    new link with a0 = cos(0.3), delta = 1 - cos 0.3 and |a| = sin 0.3, so the
    bound is E_V/6 + 4u + d_delta (1 + 1/sin 0.3) + 18u with
    d_delta = delta (8u + 2 eps_k) + 4u/alpha, eps_k = E_V/6 + 2u; an input
    difference on a staple link updated earlier in the sweep adds its norm
    to E_V, one updated later does not."""
    u = parity_util.U32
    dims, beta = (2, 2, 2, 2), 2.0
    par = parity_util.parity_array(dims)
    U0 = orc.cold(dims)
    s, mu = 5, 2                      # parity 0 site, class (2, even)
    O = U0.copy()
    O[s, mu] = [np.cos(0.3), 0.0, np.sin(0.3), 0.0]

    def closed(E_V):
        eps_k = E_V / 6 + 2 * u
        delta = 1 - np.cos(0.3)
        dd = delta * (8 * u + 2 * eps_k) + 4 * u / (6 * beta)
        return E_V / 6 + 4 * u + dd * (1 + 1 / np.sin(0.3)) + 18 * u

    b0 = parity_util.fp32_update_bound(orc, dims, beta, U0, O, O.copy(), par, s, mu)
    assert abs(b0 - closed(parity_util.STAPLE_ROUNDING)) < 1e-18
    ids = parity_util.staple_link_ids(orc, dims, s, mu)
    early = [(j, nu) for j, nu in ids if nu < mu]        # directions 0, 1: updated earlier
    late = [(j, nu) for j, nu in ids if nu > mu]         # direction 3: updated later
    G = O.copy()
    G[early[0][0], early[0][1]] += np.array([0.0, 3e-6, 0.0, 4e-6])
    assert abs(parity_util.fp32_update_bound(orc, dims, beta, U0, O, G, par, s, mu)
               - closed(parity_util.STAPLE_ROUNDING + 5e-6 * ids.count(early[0]))) < 1e-15
    G = O.copy()
    G[late[0][0], late[0][1]] += np.array([0.0, 3e-6, 0.0, 4e-6])
    assert parity_util.fp32_update_bound(orc, dims, beta, U0, O, G, par, s, mu) == b0
