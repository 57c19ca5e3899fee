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


def test_update_condition_closed_form(orc):
    """Cold 2^4 lattice: every staple is 6 (six identity products), so
    6/k = 1; for a new link with a0 = cos(0.3) the vector part is sin(0.3)."""
    dims = (2, 2, 2, 2)
    U0 = orc.cold(dims)
    new = U0.copy()
    new[5, 2] = [np.cos(0.3), 0.0, np.sin(0.3), 0.0]
    c = parity_util.update_condition(orc, dims, U0, new, 5, 2)
    assert abs(c - (1.0 + 1.0 / np.sin(0.3))) < 1e-12
    assert parity_util.update_condition(orc, dims, U0, U0, 5, 2) == float("inf")
