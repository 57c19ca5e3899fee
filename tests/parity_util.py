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


# ---- binary32 sweep against the binary64 oracle ---------------------------
# Unit roundoff of binary32.
U32 = 2.0 ** -24
# Bound on the rounding error of the staple V computed in binary32 from
# exact unit links (2-norm over the four components): each of the six
# terms is a product of three unit quaternions; the first product rounds
# four times per component (<= 4u, every partial sum bounded by 1 by
# Cauchy-Schwarz), its error reaches the second product scaled by at most
# |x|_1 <= 2 (8u), and the second product is accumulated into V by four
# fused multiply-adds whose partial sums are bounded by 6 (24u): 36u per
# component and term, 6 terms, 2-norm <= 2 x the component bound.
STAPLE_ROUNDING = 2 * 6 * 36 * U32


def link_before_mask(parity, mu, par):
    """[V, 4] bool: the links a sweep updates before class (mu, par)
    (mu = 0..3, even then odd)."""
    V = parity.size
    m = np.zeros((V, 4), bool)
    for nu in range(4):
        for p in (0, 1):
            if 2 * nu + p < 2 * mu + par:
                m[parity == p, nu] = True
    return m


def staple_link_ids(orc, dims, s, mu):
    """The 18 (site, direction) links of the staple of link (s, mu)."""
    out = []
    for nu in range(4):
        if nu == mu:
            continue
        sm = orc.neighbor(dims, s, mu, 1)
        sn = orc.neighbor(dims, s, nu, 1)
        smn = orc.neighbor(dims, sm, nu, -1)
        snb = orc.neighbor(dims, s, nu, -1)
        out += [(sm, nu), (sn, mu), (s, nu), (smn, nu), (snb, mu), (snb, nu)]
    return out


def fp32_update_bound(orc, dims, beta, U0, O, G, parity, s, mu):
    """First-order bound on |U'_32 - U'_64| (2-norm) for the binary32 heat-bath
    update of link (s, mu) in one sweep that started from the identical
    configuration U0 (binary32 values) on both sides with identical uniforms,
    O / G the oracle's and the GPU's links after the sweep.

    Inputs: the staple links updated earlier in the sweep carry their own
    difference |G - O| (the rest are U0 on both sides), so
        E_V = STAPLE_ROUNDING + sum of those differences.
    Then k = |V| and alpha = beta k carry the relative error
    eps_k = E_V / k + 2u; delta = 1 - a0 from either sampler carries
    |d delta| <= delta (8u + 2 eps_k) + 4u / alpha (logarithms and
    reciprocals to a few ulp, with an absolute floor of the hardware
    logarithm near 1); |a| = sqrt(delta (2 - delta)) adds |d delta| / |a|;
    the direction n (two sines, a square root) 8u; W = V/k carries
    E_V / k + 4u; the product X W^dag 8u; the binary64 norm and the final
    rounding 2u.  Sum:
        E_V/k + 4u + |d delta| (1 + 1/|a|) + 8u + 10u.
    k and a0 come from the oracle's configuration before the substep (its
    links updated earlier in the sweep, U0 elsewhere)."""
    par = int(parity[s])
    before = np.where(link_before_mask(parity, mu, par)[..., None], O, U0)
    V = orc.staple(dims, before, s, mu)
    k = float(np.linalg.norm(V))
    if k == 0.0:
        return float("inf")
    earlier = link_before_mask(parity, mu, par)
    ein = sum(float(np.linalg.norm(G[j, nu] - O[j, nu])) for j, nu in staple_link_ids(orc, dims, s, mu)
              if earlier[j, nu])
    E_V = STAPLE_ROUNDING + ein
    a0 = float(orc.qmul(O[s, mu], V)[0]) / k      # 1/2 Tr(U' V) / k
    delta = 1.0 - a0
    a = float(np.sqrt(max(0.0, delta * (2.0 - delta))))
    if a == 0.0:
        return float("inf")
    eps_k = E_V / k + 2 * U32
    alpha = beta * k
    if alpha == 0.0:
        return float("inf")
    d_delta = delta * (8 * U32 + 2 * eps_k) + 4 * U32 / alpha
    return E_V / k + 4 * U32 + d_delta * (1 + 1 / a) + 18 * U32


def check_fp32_sweep(orc, dims, beta, U0, G, O, tg, to, tol=1e-5, label=""):
    """Binary32 links G against the binary64 oracle O after one sweep from the
    identical binary32 configuration U0, with the per-link try records tg / to.

    Per link |G - O| <= tol, with the exceptions counted and reported:
      flips        updates whose try count or sampler branch differ;
      downstream   links over tol updated later in the sweep with a flipped
                   link in their staple (chaotic, any size);
      conditioned  links over tol elsewhere, each within its first-order
                   rounding bound (fp32_update_bound); at most one link in
                   10^5 plus five may need it.
    Any other link over tol fails.  Returns the counts."""
    par = parity_array(dims)
    flips = (tg != to).reshape(-1, 4)
    down = downstream_of_flips(dims, flips, par)
    err = np.abs(G - O).max(axis=2)
    bad = err > tol
    clean = err[~down]
    cond = []
    for s, mu in zip(*np.nonzero(bad & ~down)):
        b = fp32_update_bound(orc, dims, beta, U0, O, G, par, int(s), int(mu))
        cond.append((float(err[s, mu]), b))
    n = err.size
    q = float(np.quantile(clean, 0.99999)) if clean.size else 0.0
    print(f"FP32 {label}{tuple(dims)} beta {beta:g}: {int(flips.sum())} flips, {int(bad.sum())} links > {tol:g} "
          f"({int((bad & down).sum())} downstream of flips, {len(cond)} within their rounding bound); "
          f"max clean |dU| {float(clean.max()) if clean.size else 0.0:.2e}, 99.999% {q:.2e}"
          + "".join(f"; |dU| {e:.2e} <= bound {b:.2e}" for e, b in cond), flush=True)
    for e, b in cond:
        assert e <= b, (label, e, b)
    assert len(cond) <= n * 1e-5 + 5, (label, len(cond))
    return {"flips": int(flips.sum()), "over_tol": int(bad.sum()), "downstream": int((bad & down).sum()),
            "conditioned": len(cond)}
