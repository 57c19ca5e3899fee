"""GPU parity of the batched path: independent lattices of uneven sizes and
couplings advanced by the same launches (captured in a HIP graph), each
checked against the oracle run with its own lattice id and beta."""
import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def su2():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1010_4834_amd import su2 as s
    return s


def test_ensemble_fp64_parity(su2, orc):
    # the last lattice is the smallest allowed (every neighbour pair wraps
    # onto one site) at beta = 0 (the alpha = 0 branch for every link)
    dims = [(4, 4, 4, 4), (6, 6, 6, 4), (8, 8, 8, 6), (4, 4, 4, 8), (6, 4, 2, 10), (2, 2, 2, 2)]
    betas = [2.2, 2.35, 2.5, 2.65, 2.8, 0.0]
    ens = su2.Ensemble(dims, betas, start=su2.HOT, seed=5, prec=su2.F64)
    P, L = ens.run(3, 5)
    for i, (d, b) in enumerate(zip(dims, betas)):
        U = orc.hot(d, 5, lat_id=i)
        for sw in range(3):
            orc.heatbath_sweep(d, U, b, 5, sw, lat_id=i)
            assert abs(P[i, sw] - orc.plaquette(d, U)[0]) < 1e-12, (i, sw)
            assert abs(L[i, sw] - orc.polyakov(d, U)) < 1e-12, (i, sw)
        assert np.abs(ens.get_links(i) - U).max() < 1e-11
    tries, updates = ens.stats()
    assert updates == 3 * sum(4 * int(np.prod(d)) for d in dims) and tries >= updates
    ens.close()


def fp32_ensemble_sweep_parity(su2, orc, ens, dims, betas, seed, sample, label):
    """One binary32 sweep of the whole ensemble under its current launch
    shape; each sampled lattice against the binary64 oracle run from the
    library's own starting links with its lattice id and coupling, link by
    link (parity_util.check_fp32_sweep: 1e-5, flips and conditioned links
    counted), and the fused plaquette and Polyakov series against the oracle
    on the GPU's binary32 links."""
    from tests import parity_util
    U0 = {i: ens.get_links(i) for i in sample}
    ens.trace_tries(True)
    P, L = ens.run(1, seed)
    tot = {"flips": 0, "over_tol": 0, "downstream": 0, "conditioned": 0}
    for i in sample:
        d = dims[i]
        O = U0[i].copy()
        to = np.zeros(4 * O.shape[0], np.uint32)
        orc.heatbath_sweep(d, O, betas[i], seed, 0, lat_id=i, ubits=23, trace=to)
        G = ens.get_links(i)
        r = parity_util.check_fp32_sweep(orc, d, betas[i], U0[i], G, O, ens.get_tries(i), to,
                                         label=f"{label} lattice {i} ")
        for k in tot:
            tot[k] += r[k]
        assert abs(P[i, 0] - orc.plaquette(d, G)[0]) < 1e-6, i
        assert abs(L[i, 0] - orc.polyakov(d, G)) < 1e-6, i
    print(f"{label} FP32 totals over {len(sample)} lattices: {tot}", flush=True)
    ens.trace_tries(False)
    return tot


def test_ensemble_fp32_c5_link_parity(su2, orc):
    """The 64-lattice uneven ensemble (L in {8,12,16,24}, Nt in {4,6,8,L}),
    binary32 links, one sweep under the autotuned launch shape: one lattice
    of each of the 16 extent classes (spread over the lattice ids and
    couplings) link by link against the binary64 oracle."""
    dims, betas = inputs.c5_shapes()
    ens = su2.Ensemble(dims, betas, start=su2.HOT, seed=5, prec=su2.F32)
    su2.su2_ensemble_autotune(ens.h)
    print("launch", su2.su2_ensemble_get_launch(ens.h))
    sample = [c + 16 * (c % 4) for c in range(16)]
    assert sorted({dims[i] for i in sample}) == sorted(set(dims))
    fp32_ensemble_sweep_parity(su2, orc, ens, dims, betas, 5, sample, "C5")
    ens.close()


def test_ensemble_fp32_c3_link_parity(su2, orc):
    """The C3 beta scan at full size (16 x 32^3 x 4, beta in [2.1, 2.5], hot
    start seed 3), binary32, one sweep under the autotuned launch shape:
    lattices 0, 7 and 15 link by link against the binary64 oracle."""
    dims = [(32, 32, 32, 4)] * 16
    betas = inputs.c3_betas()
    ens = su2.Ensemble(dims, betas, start=su2.HOT, seed=3, prec=su2.F32)
    su2.su2_ensemble_autotune(ens.h)
    print("launch", su2.su2_ensemble_get_launch(ens.h))
    fp32_ensemble_sweep_parity(su2, orc, ens, dims, betas, 3, (0, 7, 15), "C3")
    ens.close()


def test_ensemble_fp64_c5_shapes(su2, orc):
    """The 64-lattice uneven ensemble in binary64 under the autotuned launch
    shape, one sweep: lattices of every extent class (8^3x4 up to 24^4)
    against the oracle link by link, with their plaquette and Polyakov
    values."""
    dims, betas = inputs.c5_shapes()
    ens = su2.Ensemble(dims, betas, start=su2.HOT, seed=5, prec=su2.F64)
    su2.su2_ensemble_autotune(ens.h)
    print("launch", su2.su2_ensemble_get_launch(ens.h))
    P, L = ens.run(1, 5)
    for i in (0, 9, 15, 18, 27, 36, 45, 54, 63):
        U = orc.hot(dims[i], 5, lat_id=i)
        orc.heatbath_sweep(dims[i], U, betas[i], 5, 0, lat_id=i)
        assert np.abs(ens.get_links(i) - U).max() < 1e-12, i
        assert abs(P[i, 0] - orc.plaquette(dims[i], U)[0]) < 1e-12, i
        assert abs(L[i, 0] - orc.polyakov(dims[i], U)) < 1e-12, i
    ens.close()


@pytest.mark.parametrize("prec,tol", [("F64", 1e-13), ("F32", 2e-7)])
def test_fused_plaquette_matches_standalone(su2, prec, tol):
    """The plaquette series summed inside the odd heat-bath substeps equals
    the standalone plaquette kernel on the configuration after each sweep."""
    dims = [(8, 6, 4, 10), (6, 6, 6, 6)]
    p = getattr(su2, prec)
    ens = su2.Ensemble(dims, [2.4, 2.7], start=su2.HOT, seed=7, prec=p)
    for launch in ((256, 0, 1, 1), (64, 16, 0, 2), (128, 0, 1, 4), (128, 0, 2, 1), (64, 0, 3, 1)):
        su2.su2_ensemble_set_launch(ens.h, *launch)
        P, _ = ens.run(1, 7, plaq=True, poly=False)
        for i, d in enumerate(dims):
            lat = su2.Lattice(d, start=su2.COLD, prec=p)
            lat.set_links(ens.get_links(i))
            assert abs(P[i, 0] - lat.plaquette()[0]) < tol, (launch, i)
            lat.close()
    ens.close()


def test_series_across_batches(su2):
    """A run longer than the series slots of a large lattice (64^4: about
    21 sweeps of partials) is reduced in several batches; every series value
    equals the standalone plaquette of an identical lattice advanced one
    sweep at a time."""
    dims, beta, seed, n = (64, 64, 64, 64), 2.5, 9, 25
    ens = su2.Ensemble([dims], [beta], start=su2.HOT, seed=seed, prec=su2.F32)
    P, _ = ens.run(n, seed, plaq=True, poly=False)
    ens.close()
    lat = su2.Lattice(dims, start=su2.HOT, seed=seed, prec=su2.F32)
    worst = 0.0
    for k in range(n):
        lat.heatbath(beta, 1, seed)
        worst = max(worst, abs(P[0, k] - lat.plaquette()[0]))
    lat.close()
    print(f"64^4 series over batches: worst |dP| {worst:.2e}")
    # same chain bit for bit; the two plaquette sums differ only in the
    # binary32 rounding of ~1e8 terms of random sign
    assert worst < 1e-9


@pytest.mark.parametrize("prec", ["F32", "F64"])
def test_measuring_does_not_change_the_chain(su2, prec):
    """Sweeps with the fused plaquette and Polyakov series leave the same
    links, bit for bit, as sweeps without measurements."""
    dims, beta, seed = (8, 6, 4, 10), 2.4, 13
    p = getattr(su2, prec)
    a = su2.Ensemble([dims], [beta], start=su2.HOT, seed=seed, prec=p)
    a.run(6, seed, plaq=True, poly=True)
    b = su2.Lattice(dims, start=su2.HOT, seed=seed, prec=p)
    b.heatbath(beta, 6, seed)
    assert np.array_equal(a.get_links(0), b.get_links())
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_multi_sweep_graphs_match_direct_launches(su2, prec):
    """Runs of 21 sweeps, 5 sweeps, 37 sweeps measured every second sweep
    (18 two-sweep units and one unmeasured sweep) and 9 sweeps with another
    seed, each replayed as one captured run graph; links, plaquette and
    Polyakov series are bit for bit those of the same sweeps launched one
    kernel at a time (SU2_NO_GRAPH)."""
    import os
    dims, betas = [(6, 4, 10, 6), (4, 4, 4, 8)], [2.3, 2.6]
    out = []
    for direct in (False, True):
        if direct:
            os.environ["SU2_NO_GRAPH"] = "1"
        try:
            ens = su2.Ensemble(dims, betas, start=su2.HOT, seed=9, prec=getattr(su2, prec))
            P, L = ens.run(21, 9)
            P2, L2 = ens.run(5, 9)     # the counter continues across runs
            P3, L3 = ens.run(37, 9, measure_every=2)
            P4, L4 = ens.run(9, 12)    # a new seed: the library uploads it before the run
            out.append((P, L, P2, L2, P3, L3, P4, L4, [ens.get_links(i) for i in range(len(dims))]))
            ens.close()
        finally:
            os.environ.pop("SU2_NO_GRAPH", None)
    (a, b) = out
    for x, y in zip(a[:8], b[:8]):
        assert np.array_equal(x, y)
    for x, y in zip(a[8], b[8]):
        assert np.array_equal(x, y)


def test_series_batches_and_long_runs_match_direct_launches(su2):
    """Graph forms that the short runs above do not reach, against direct
    launches, bit for bit: a 32^4 binary32 run of 200 sweeps measured after
    every sweep under block 64 (8192 plaquette tiles, so the per-sweep
    partial slots, about 64 MiB at most, hold 84 sweeps: one run
    graph with three series batches), and a 300-sweep run of two small
    lattices measured every third sweep (longer than one run graph: graphs
    of 16 sweeps and the binary remainder)."""
    import os
    cases = (([(32, 32, 32, 32)], [2.6], su2.F32, (64, 0, 3, 1), 200, 1),
             ([(6, 4, 10, 6), (4, 4, 4, 8)], [2.3, 2.6], su2.F64, None, 300, 3))
    for dims, betas, prec, launch, nsw, every in cases:
        out = []
        for direct in (False, True):
            if direct:
                os.environ["SU2_NO_GRAPH"] = "1"
            try:
                ens = su2.Ensemble(dims, betas, start=su2.HOT, seed=17, prec=prec)
                if launch:
                    su2.su2_ensemble_set_launch(ens.h, *launch)
                P, L = ens.run(nsw, 17, measure_every=every)
                out.append((P, L, [ens.get_links(i) for i in range(len(dims))]))
                ens.close()
            finally:
                os.environ.pop("SU2_NO_GRAPH", None)
        (a, b) = out
        print(dims[0], nsw, "sweeps:", a[0].shape, "measurements", flush=True)
        assert a[0].shape == (len(dims), nsw // every)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        for x, y in zip(a[2], b[2]):
            assert np.array_equal(x, y)


def test_ensemble_launch_shapes_bitwise_c5(su2):
    """The 64 uneven lattices of C5 in binary32, two sweeps from the hot
    start under launch shapes of every tile mode, links per lane 1, 2 and 4
    and a persistent grid: every lattice's links agree bit for bit (lattice
    boundaries fall inside workgroups and tiles differently in each)."""
    dims, betas = inputs.c5_shapes()
    ref = None
    for launch in ((128, 0, 2, 1), (256, 0, 1, 1), (64, 0, 3, 2), (128, 0, 0, 4), (64, 2048, 1, 1)):
        ens = su2.Ensemble(dims, betas, start=su2.HOT, seed=5, prec=su2.F32)
        su2.su2_ensemble_set_launch(ens.h, *launch)
        ens.run(2, 5, plaq=False, poly=False)
        G = [ens.get_links(i) for i in range(len(dims))]
        ens.close()
        if ref is None:
            ref = G
        else:
            for i in range(len(dims)):
                assert np.array_equal(G[i], ref[i]), (launch, i)


@pytest.mark.parametrize("launch", [None, (128, 0, 2, 1)])
def test_ensemble_fp64_c3_shapes(su2, orc, launch):
    """The C3 beta scan at full size (16 x 32^3 x 4, beta in [2.1, 2.5], hot
    start seed 3), binary64, one sweep under the autotuned launch shape and
    under tile mode 2: sampled lattices against the oracle link by link, and
    their plaquette and Polyakov series."""
    dims = [(32, 32, 32, 4)] * 16
    betas = [2.1 + 0.4 * i / 15 for i in range(16)]
    ens = su2.Ensemble(dims, betas, start=su2.HOT, seed=3, prec=su2.F64)
    if launch is None:
        su2.su2_ensemble_autotune(ens.h)
    else:
        su2.su2_ensemble_set_launch(ens.h, *launch)
    print("launch", su2.su2_ensemble_get_launch(ens.h))
    P, L = ens.run(1, 3)
    for i in (0, 7, 15):
        U = orc.hot(dims[i], 3, lat_id=i)
        orc.heatbath_sweep(dims[i], U, betas[i], 3, 0, lat_id=i)
        assert np.abs(ens.get_links(i) - U).max() < 1e-12, i
        assert abs(P[i, 0] - orc.plaquette(dims[i], U)[0]) < 1e-12, i
        assert abs(L[i, 0] - orc.polyakov(dims[i], U)) < 1e-12, i
    ens.close()


def test_handles_run_concurrently(su2):
    """Separate handles are independent: two ensembles driven from two host
    threads, each on its own stream, autotuning and sweeping at the same
    time, end with the links and series of the same runs made one after the
    other."""
    import threading
    import torch
    jobs = [([(8, 6, 4, 10), (6, 6, 6, 4)], [2.4, 2.7], 21), ([(4, 4, 4, 8)] * 3, [2.2, 2.5, 2.8], 22)]

    def run(dims, betas, seed, stream, out):
        ens = su2.Ensemble(dims, betas, start=su2.HOT, seed=seed, prec=su2.F32,
                           stream=None if stream is None else stream.cuda_stream)
        su2.su2_ensemble_set_launch(ens.h, 128, 0, 1, 1)
        P, L = ens.run(12, seed)
        out.append((P, L, [ens.get_links(i) for i in range(len(dims))]))
        ens.close()

    seq = []
    for dims, betas, seed in jobs:
        out = []
        run(dims, betas, seed, None, out)
        seq.append(out[0])
    streams = [torch.cuda.Stream() for _ in jobs]
    outs = [[] for _ in jobs]
    threads = [threading.Thread(target=run, args=(d, b, s, st, o))
               for (d, b, s), st, o in zip(jobs, streams, outs)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert all(not t.is_alive() for t in threads) and all(len(o) == 1 for o in outs)
    for (P, L, U), o in zip(seq, outs):
        P2, L2, U2 = o[0]
        assert np.array_equal(P, P2) and np.array_equal(L, L2)
        for a, b in zip(U, U2):
            assert np.array_equal(a, b)
