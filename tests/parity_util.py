"""Helpers of the GPU parity tests: which links an FP32 accept/reject flip can
reach within one sweep (its downstream set), and link-error summaries."""
import numpy as np


def _shift(idx, mu, k):
    # idx: [t, z, y, x] site-index grid; value at s of the site s + k mu
    return np.roll(idx, -k, axis=3 - mu)


def staple_links(dims, mu):
    """For every site s, the (site, direction) pairs of the 18 links in the
    staple of link (s, mu): arrays of shape [18, V] (sites) and [18] (dirs)."""
    V = int(np.prod(dims))
    idx = np.arange(V).reshape(dims[::-1])
    sites, dirs = [], []
    for nu in range(4):
        if nu == mu:
            continue
        xp = _shift(idx, mu, 1)
        for g, d in ((xp, nu), (_shift(idx, nu, 1), mu), (idx, nu),
                     (_shift(xp, nu, -1), nu), (_shift(idx, nu, -1), mu),
                     (_shift(idx, nu, -1), nu)):
            sites.append(g.ravel())
            dirs.append(d)
    return np.array(sites), np.array(dirs)


def downstream_of_flips(dims, flips, parity):
    """flips: [V, 4] bool (links whose try record differs).  Returns [V, 4]
    bool: the flipped links and every link updated later in the same sweep
    whose staple contains a marked link (mu = 0..3, even then odd)."""
    taint = flips.copy()
    for mu in range(4):
        S, D = staple_links(dims, mu)
        for p in (0, 1):
            cls = parity == p
            hit = taint[S, D[:, None]].any(axis=0)
            taint[cls, mu] |= hit[cls]
    return taint


def parity_array(dims):
    V = int(np.prod(dims))
    s = np.arange(V)
    x = s % dims[0]
    y = (s // dims[0]) % dims[1]
    z = (s // (dims[0] * dims[1])) % dims[2]
    t = s // (dims[0] * dims[1] * dims[2])
    return (x + y + z + t) & 1


def update_condition(orc, dims, before, U_new, s, mu):
    """First-order sensitivity of a heat-bath update to rounding: the link is
    U' = X W^dag with W = V/k, so a staple error dV moves U' by ~dV/k (V is a
    sum of six unit-size products, hence 6/k), and X has vector part
    |a| = sqrt(delta (2 - delta)), so an error in delta moves it by
    ~d(delta)/|a| as a0 -> -1.  Returns 6/k + 1/|a|, from the oracle's
    configuration `before` the substep and its new link."""
    V = orc.staple(dims, before, s, mu)
    k = float(np.linalg.norm(V))
    if k == 0.0:
        return float("inf")
    a0 = float(orc.qmul(U_new[s, mu], V)[0]) / k
    a = float(np.sqrt(max(0.0, 1.0 - a0 * a0)))
    return 6.0 / k + (1.0 / a if a > 0 else float("inf"))
