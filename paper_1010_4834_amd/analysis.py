"""Analysis of measured series: binned jackknife errors and the static
quark potential from Wilson loops.

Paper Sec. 5 (static potential): the potential between static sources
follows from the decay of W(R,T) in T, aV(R) = lim_T ln[W(R,T)/W(R,T+1)],
and is fitted with the Cornell form aV(R) = A + B/R + sigma a^2 R, whose
slope is the string tension (the paper's table gives sigma a^2 at
beta = 2.5).  These are host-side numerics on a few hundred numbers per
configuration; the measurements themselves come from the library.
"""
import numpy as np


def bin_series(x, nbins):
    """Average consecutive blocks of a series (axis 0) into `nbins` bins;
    the tail that does not fill a bin is dropped."""
    x = np.asarray(x, dtype=np.float64)
    if nbins < 2 or nbins > x.shape[0]:
        raise ValueError("need 2 <= nbins <= number of samples")
    b = x.shape[0] // nbins
    return x[: b * nbins].reshape((nbins, b) + x.shape[1:]).mean(axis=1)


def jackknife(bins, f=None):
    """Jackknife estimate of f(mean of bins) and its error.

    bins: array [nbins, ...]; f maps a mean (shape bins.shape[1:]) to a
    scalar or array (default: the mean itself).  Returns (estimate, error,
    leave-one-out values)."""
    bins = np.asarray(bins, dtype=np.float64)
    n = bins.shape[0]
    if n < 2:
        raise ValueError("jackknife needs at least two bins")
    f = f or (lambda m: m)
    full = np.asarray(f(bins.mean(axis=0)))
    tot = bins.sum(axis=0)
    loo = np.stack([np.asarray(f((tot - bins[i]) / (n - 1))) for i in range(n)])
    mean_loo = loo.mean(axis=0)
    err = np.sqrt((n - 1) / n * ((loo - mean_loo) ** 2).sum(axis=0))
    return full, err, loo


def effective_potential(W):
    """aV(R, T) = ln[W(R,T) / W(R,T+1)] of mean loops W[R-1, T-1];
    shape [Rmax, Tmax-1] (NaN where a ratio is not positive)."""
    W = np.asarray(W, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = W[:, :-1] / W[:, 1:]
        return np.where(r > 0, np.log(np.where(r > 0, r, 1.0)), np.nan)


def cornell_fit(R, V, dV=None):
    """Weighted least squares of V(R) = A + B/R + sigma R; returns
    (A, B, sigma).  dV: errors (None = equal weights)."""
    R = np.asarray(R, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    w = np.ones_like(V) if dV is None else 1.0 / np.asarray(dV, dtype=np.float64)
    X = np.stack([np.ones_like(R), 1.0 / R, R], axis=1)
    coef, *_ = np.linalg.lstsq(X * w[:, None], V * w, rcond=None)
    return coef


def static_potential(Wcfg, t0, rmin, rmax, nbins):
    """String tension from a series of Wilson-loop measurements.

    Wcfg: [nconf, Rmax, Tmax] per configuration (W[R-1, T-1]).  The
    potential is read at T = t0 (aV = ln W(R,t0)/W(R,t0+1)); the Cornell
    form is fitted for rmin <= R <= rmax with the jackknife errors of V as
    weights.  Returns a dict with V, dV (R = 1..Rmax), the fit (A, B, sigma)
    and its jackknife errors."""
    Wcfg = np.asarray(Wcfg, dtype=np.float64)
    Rmax, Tmax = Wcfg.shape[1], Wcfg.shape[2]
    if not (1 <= t0 < Tmax and 1 <= rmin < rmax <= Rmax):
        raise ValueError("t0 / R range outside the measured loops")
    bins = bin_series(Wcfg, nbins)
    pot = lambda Wm: effective_potential(Wm)[:, t0 - 1]
    V, dV, _ = jackknife(bins, pot)
    R = np.arange(1, Rmax + 1, dtype=np.float64)
    sel = slice(rmin - 1, rmax)
    Rs, dVs = R[sel], dV[sel]
    fit = lambda Wm: cornell_fit(Rs, pot(Wm)[sel], dVs)
    coef, dcoef, _ = jackknife(bins, fit)
    return {"R": R, "V": V, "dV": dV, "A": coef[0], "B": coef[1], "sigma": coef[2],
            "dA": dcoef[0], "dB": dcoef[1], "dsigma": dcoef[2], "t0": t0, "rmin": rmin, "rmax": rmax,
            "nbins": nbins}


def stable_t0(Wcfg, rmin, rmax, nbins, tmin=2):
    """Plateau choice for static_potential: the smallest t0 >= tmin whose
    fitted sigma a^2 agrees with the t0 + 1 fit within the t0 + 1 fit's
    jackknife error (excited states have decayed to within the noise).
    None if no t0 qualifies."""
    Wcfg = np.asarray(Wcfg, dtype=np.float64)
    prev = None
    for t0 in range(tmin, Wcfg.shape[2]):
        res = static_potential(Wcfg, t0, rmin, rmax, nbins)
        if prev is not None and abs(res["sigma"] - prev["sigma"]) <= res["dsigma"]:
            return prev["t0"]
        prev = res
    return None

