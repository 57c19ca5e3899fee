"""Long-run agreement: beyond a few sweeps the chain is chaotic, so GPU and
oracle runs are compared statistically.  Independent chains (different
seeds) of the GPU path (binary32 and binary64 links) and of the oracle give
the same mean plaquette and mean |Polyakov loop| within three standard
deviations of the combined binned jackknife errors.

Sizes are reduced stand-ins for the production workloads so that the
serial oracle finishes in about a minute: 10^4 at beta = 2.3 (plaquette),
8^3 x 4 at beta = 2.2 and 2.45 (either side of the Nt = 4 transition) for
the Polyakov loop, and a four-lattice 16^3 x 4 beta scan across the
transition advanced as one ensemble (the C3 form)."""
import sys
import time

import numpy as np
import pytest

from paper_1010_4834_amd import analysis as an

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def su2():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1010_4834_amd import su2 as s
    return s


def oracle_series(orc, dims, beta, seed, nsweeps):
    U = orc.hot(dims, seed)
    P = np.empty(nsweeps)
    L = np.empty(nsweeps)
    for sw in range(nsweeps):
        orc.heatbath_sweep(dims, U, beta, seed, sw)
        P[sw] = orc.plaquette(dims, U)[0]
        L[sw] = orc.polyakov(dims, U)
    return P, L


def gpu_series(su2, dims, beta, seed, nsweeps, prec):
    ens = su2.Ensemble([dims], [beta], start=su2.HOT, seed=seed, prec=prec)
    P, L = ens.run(nsweeps, seed)
    ens.close()
    return P[0], L[0]


def mean_err(x, discard, nbins):
    est, err, _ = an.jackknife(an.bin_series(np.asarray(x)[discard:], nbins))
    return float(est), float(err)


def agree(name, a, b):
    (m1, e1), (m2, e2) = a, b
    z = abs(m1 - m2) / np.hypot(e1, e2)
    print(f"{name}: {m1:.6f}({e1:.6f}) vs {m2:.6f}({e2:.6f}), {z:.2f} sigma", flush=True)
    assert z <= 3.0, name


P10 = dict(dims=(10, 10, 10, 10), beta=2.3, n=420, discard=60, nbins=12)


@pytest.fixture(scope="module")
def p10_ref(orc):
    """<P> of a serial oracle heat-bath chain on 10^4 at beta = 2.3."""
    t0 = time.perf_counter()
    Po, _ = oracle_series(orc, P10["dims"], P10["beta"], 101, P10["n"])
    print(f"oracle {P10['n']} sweeps of {P10['dims']}: {time.perf_counter() - t0:.1f} s", flush=True)
    return mean_err(Po, P10["discard"], P10["nbins"])


def test_plaquette_long_run(su2, p10_ref):
    dims, beta, n, discard, nbins = P10["dims"], P10["beta"], P10["n"], P10["discard"], P10["nbins"]
    ref = p10_ref
    for prec, seed in (("F32", 202), ("F64", 303)):
        Pg, _ = gpu_series(su2, dims, beta, seed, n, getattr(su2, prec))
        agree(f"<P> {prec} GPU vs oracle", mean_err(Pg, discard, nbins), ref)
    # a cross-check that the test can see a difference: a 0.5% shift of the
    # coupling moves <P> by many sigma
    Pb, _ = gpu_series(su2, dims, beta * 1.005, 404, n, su2.F32)
    m, e = mean_err(Pb, discard, nbins)
    assert abs(m - ref[0]) / np.hypot(e, ref[1]) > 3.0


def test_overrelaxation_mix_long_run(su2, p10_ref):
    """A chain of one heat-bath sweep and two over-relaxation sweeps per step
    (binary32) reaches the equilibrium <P> of the oracle's pure heat-bath
    chain: over-relaxation keeps the action and so the Boltzmann
    distribution, and the mix is ergodic through the heat bath."""
    dims, beta, n, discard, nbins = P10["dims"], P10["beta"], P10["n"], P10["discard"], P10["nbins"]
    lat = su2.Lattice(dims, start=su2.HOT, seed=505, prec=su2.F32)
    P = np.empty(n)
    for k in range(n):
        lat.heatbath(beta, 1, 505)
        lat.overrelax(2)
        P[k] = lat.plaquette()[0]
    tries, updates, defect = lat.stats()
    lat.close()
    assert defect < 1e-5
    agree("<P> F32 GPU 1 HB + 2 OR vs oracle HB", mean_err(P, discard, nbins), p10_ref)


@pytest.mark.parametrize("beta", [2.2, 2.45])
def test_polyakov_long_run(su2, orc, beta):
    # near the transition |L| decorrelates slowly: long runs, long bins
    dims, n, discard, nbins = (8, 8, 8, 4), 4000, 200, 16
    t0 = time.perf_counter()
    Po, Lo = oracle_series(orc, dims, beta, 111, n)
    print(f"oracle {n} sweeps of {dims} at beta {beta}: {time.perf_counter() - t0:.1f} s", flush=True)
    refP, refL = mean_err(Po, discard, nbins), mean_err(np.abs(Lo), discard, nbins)
    Pg, Lg = gpu_series(su2, dims, beta, 222, n, su2.F32)
    agree(f"<P> beta {beta}", mean_err(Pg, discard, nbins), refP)
    agree(f"<|L|> beta {beta}", mean_err(np.abs(Lg), discard, nbins), refL)
    sys.stdout.flush()


def test_beta_scan_across_the_transition(su2, orc):
    """A reduced C3-like scan: four 16^3 x 4 lattices at beta = 2.2, 2.3, 2.4,
    2.5 (either side of the Nt = 4 deconfinement point) advanced together as
    one binary32 ensemble, against four independent serial oracle chains run
    on host threads at once (the oracle is a C library called through ctypes,
    which releases the interpreter lock).  <P> and <|L|> agree within three
    combined binned-jackknife errors at every beta; the Polyakov loop
    decorrelates slowly near the transition, hence long bins."""
    from concurrent.futures import ThreadPoolExecutor
    dims, betas = (16, 16, 16, 4), (2.2, 2.3, 2.4, 2.5)
    n, discard, nbins = 2000, 200, 12

    def oracle_chain(k):
        t0 = time.perf_counter()
        P, L = oracle_series(orc, dims, betas[k], 131 + k, n)
        print(f"oracle chain beta {betas[k]}: {n} sweeps in {time.perf_counter() - t0:.1f} s", flush=True)
        return P, L

    with ThreadPoolExecutor(len(betas)) as ex:
        fut = [ex.submit(oracle_chain, k) for k in range(len(betas))]
        ens = su2.Ensemble([dims] * len(betas), list(betas), start=su2.HOT, seed=231, prec=su2.F32)
        Pg, Lg = ens.run(n, 231)
        ens.close()
        ref = [f.result() for f in fut]
    for k, b in enumerate(betas):
        Po, Lo = ref[k]
        agree(f"scan <P> beta {b}", mean_err(Pg[k], discard, nbins), mean_err(Po, discard, nbins))
        agree(f"scan <|L|> beta {b}", mean_err(np.abs(Lg[k]), discard, nbins),
              mean_err(np.abs(Lo), discard, nbins))
