"""Benchmark: SU(2) checkerboard heat-bath link updates/s on one MI355X.

Default workload (32^4 lattice, beta = 2.6, hot start from Philox seed 2,
binary32 links with binary64 reductions and reunitarisation norm): one step
is one heat-bath sweep (8 checkerboard substeps over all 4V links) followed
by the mean plaquette, run through the batched path (the sweep and its
measurement captured once in a HIP graph and replayed; batch of one).

Prints ONE JSON line: value = link updates/s of the timed region (the
median of --reps repetitions of K steps), the roofline of the dominant kernel
(the heat-bath substep; algorithmic traffic 8 link transfers = 128 B per
update, timed per launch with HIP events stamped by the launch on the stream
it runs on, in an eager pass after the timed region), the 64^4 control that
exceeds the Infinity Cache, the plain FP64 single-lattice form on the same
GPU and schedule for comparison, and the serial FP64 oracle timed on the
host cores on a bounded sample.

  python bench.py [--steps K] [--warmup W] [--config c1|c2|c2x2|c2x4|c3|c4|c5|control64]

The other configurations are side measurements of the same library: control64
(a lattice larger than the Infinity Cache), c2x2 and c2x4 (independent replica
chains of the 32^4 lattice batched in one launch), c3 and c5 (ensembles; c3
and c5 also time the plain FP64 single-lattice form looped over their
lattices), c1 (8^4, binary64, launch-bound) and c4 (24^3x48: heat bath, APE
smearing and Wilson loops per configuration).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_BYTES = 256 << 20

# Bytes one heat-bath substep moves at 32^4 FP32 (and at 64^4 for the
# control), from rocprofv3 --pmc runs of FETCH_SIZE and WRITE_SIZE (KiB per
# dispatch, mean over the eight substeps of a sweep), scaled by 2.0 and 1.0:
# the factors that make a 1 GiB device copy read back its own size; bytes
# per launch for each launch shape measured (block, grid, tile mode, links
# per lane; a grid of 0 counts as its effective size, one workgroup per
# tile).  Valid only for the sources whose code (comments and layout aside)
# has this hash: the kernels and the host code that orders their tiles.
HB_TRAFFIC = {"sources_sha256": "f3d9d7bd90f0ae9b097c8e2a2b0890fce0f860495d8cef363ed0e4064d967e98",
              "by_launch": {(128, 4096, 3, 1): 74249104, (64, 8192, 3, 1): 74273863,
                            (256, 2048, 3, 1): 74094736, (64, 8192, 1, 1): 78245785,
                            (64, 7168, 3, 1): 76533206, (128, 3584, 3, 1): 77228460,
                            (256, 1792, 3, 1): 76072259, (64, 4096, 3, 1): 74261637,
                            (128, 2048, 3, 1): 74268106, (256, 1024, 3, 1): 74100859,
                            (64, 4096, 3, 2): 75724088, (128, 2048, 3, 2): 75571729},
              # the 64^4 control: 1 GiB algorithmic per launch
              "control64": {(256, 32768, 0, 1): 1267011584}}
KERNEL_SOURCES = ("su2_kernels.hip", "su2_device.hpp", "su2_internal.hpp", "su2_api.hip")


def effective_grid(grid, tiles):
    """Workgroups of a heat-bath launch that take tiles: grid 0 is one
    workgroup per tile (the tile count rounded up to a multiple of 8); a
    persistent grid beyond that count leaves the extra workgroups idle and
    hands out the tiles exactly as the rounded count does."""
    full = max(8, -(-tiles // 8) * 8)
    return full if grid <= 0 else min(grid, full)


def code_only(text):
    """C++ source text without its comments, whitespace runs collapsed to
    one space (string and character literals kept as written)."""
    import re
    tok = re.compile(r'//[^\n]*|/\*.*?\*/|"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'', re.S)
    text = tok.sub(lambda m: " " if m.group(0)[0] == "/" else m.group(0), text)
    return " ".join(text.split())


def kernel_sources_sha256():
    """SHA-256 of the code of the kernel sources (comments and layout
    aside), or None where they are not shipped."""
    import hashlib
    h = hashlib.sha256()
    try:
        for f in KERNEL_SOURCES:
            with open(os.path.join(ROOT, "paper_1010_4834_amd", "csrc", f), encoding="utf-8") as fh:
                h.update(code_only(fh.read()).encode())
                h.update(b"\0")
    except OSError:
        return None
    return h.hexdigest()


def configs():
    c3 = [(32, 32, 32, 4)] * 16, [2.1 + 0.4 * i / 15 for i in range(16)]
    combos = [(L, L, L, Nt) for L in (8, 12, 16, 24) for Nt in (4, 6, 8, L)]
    c5 = [combos[i % 16] for i in range(64)], [2.2 + 0.6 * i / 63 for i in range(64)]
    return {
        "c2": dict(dims=[(32, 32, 32, 32)], betas=[2.6], seed=2, poly=False,
                   desc="32^4 SU(2) heat bath, beta=2.6, hot start, 1 sweep + plaquette per step"),
        "c2x2": dict(dims=[(32, 32, 32, 32)] * 2, betas=[2.6] * 2, seed=2, poly=False,
                     desc="2 independent replica chains of the 32^4 lattice (beta=2.6, hot start, "
                          "own lattice ids in the Philox counter) in one launch, 1 sweep + "
                          "plaquette per step"),
        "c2x4": dict(dims=[(32, 32, 32, 32)] * 4, betas=[2.6] * 4, seed=2, poly=False,
                     desc="4 independent replica chains of the 32^4 lattice (256 MiB of links, "
                          "the Infinity Cache's size) in one launch, 1 sweep + plaquette per step"),
        # one GPU's share of the 32^4 lattice split into t-slabs over 2, 4 and
        # 8 GPUs; a periodic 32^3 x Nt/g lattice stands in for the slab and its
        # two ghost slices (same updates and reads per link, no exchange)
        **{"slab%d" % g: dict(dims=[(32, 32, 32, 32 // g)], betas=[2.6], seed=2, poly=False,
                              desc="32^3x%d SU(2) heat bath, beta=2.6, hot start, 1 sweep + plaquette "
                                   "per step: one GPU's t-slab of the 32^4 lattice on %d GPUs" % (32 // g, g))
           for g in (2, 4, 8)},
        "control64": dict(dims=[(64, 64, 64, 64)], betas=[2.6], seed=2, poly=False,
                          desc="64^4 SU(2) heat bath (1 GiB of links, beyond the 256 MB "
                               "Infinity Cache), beta=2.6, 1 sweep + plaquette per step"),
        "c3": dict(dims=c3[0], betas=c3[1], seed=3, poly=True,
                   desc="16 x 32^3x4 beta scan [2.1,2.5] in one launch, 1 sweep + plaquette "
                        "+ Polyakov per step"),
        "c5": dict(dims=c5[0], betas=c5[1], seed=5, poly=True,
                   desc="64 uneven lattices L^3xNt, L in {8,12,16,24}, Nt in {4,6,8,L}, "
                        "beta in [2.2,2.8], 1 sweep + plaquette + Polyakov per step"),
        "c1": dict(dims=[(8, 8, 8, 8)], betas=[2.3], seed=1, poly=False,
                   desc="8^4 SU(2) heat bath, beta=2.3, cold start, binary64, 20 sweeps with the "
                        "plaquette after each (launch-bound; context)"),
        "c4": dict(dims=[(24, 24, 24, 48)], betas=[2.5], seed=4, poly=False,
                   desc="24^3x48, beta=2.5: per configuration 5 heat-bath sweeps, APE smearing "
                        "(alpha 0.7, 25 steps) of the spatial links and on-axis Wilson loops "
                        "W(R<=12, T<=16)"),
    }


def cpu_baseline(dims, beta, seed, nsweeps):
    """The serial FP64 oracle on the host: nsweeps sweeps + plaquettes."""
    from oracle import oracle as orc
    U = orc.hot(dims, seed)
    t0 = time.perf_counter()
    for sw in range(nsweeps):
        orc.heatbath_sweep(dims, U, beta, seed, sw)
        orc.plaquette(dims, U)
    dt = time.perf_counter() - t0
    V = 1
    for d in dims:
        V *= d
    return 4 * V * nsweeps / dt, dt


def copy_probe(torch):
    """Device-to-device copy of 1 GiB: the achievable streaming bandwidth."""
    x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        y.copy_(x)
    c1.record()
    torch.cuda.synchronize()
    gbs = 2 * (1 << 30) * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del x, y
    return gbs


def host_info():
    """CPU model and thread count of the host that timed the oracle."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from oracle import build as ob
        flags = "gcc " + " ".join(ob.FLAGS)
    except Exception:
        flags = None
    return {"cpu": model, "threads": os.cpu_count(), "oracle_build": flags}


def cpu_all_cores(dims, beta, nsweeps, nthreads):
    """The same oracle on nthreads host threads at once, each on its own
    lattice (seeds 2, 3, ...).  The oracle is a C library called through
    ctypes, which releases the interpreter lock for each call, so the threads
    run in parallel; no process is started.  Aggregate link updates/s over
    the slowest thread."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(nthreads) as ex:
        res = list(ex.map(lambda i: cpu_baseline(dims, beta, 2 + i, nsweeps), range(nthreads)))
    V = 1
    for d in dims:
        V *= d
    slowest = max(dt for _, dt in res)
    return 4 * V * nsweeps * nthreads / slowest, slowest


def bench_c1(su2, args, cfg, stream):
    """8^4 binary64 from a cold start: 20 sweeps, plaquette after each, as
    plain per-call API use (one sweep call and one synchronising plaquette
    call per sweep) and as one graph-replayed ensemble series."""
    import numpy as np
    import torch
    dims, beta, seed = cfg["dims"][0], cfg["betas"][0], cfg["seed"]
    nsw = 20
    updates = 4 * int(np.prod(dims)) * nsw

    def plain():
        lat = su2.su2_create(*dims, su2.COLD, seed, su2.F64)
        su2.su2_set_stream(lat, stream.cuda_stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = []
        for _ in range(nsw):
            su2.su2_heatbath(lat, beta, 1, seed)
            P.append(su2.su2_plaquette(lat)[0])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        su2.su2_set_timing(lat, 1)
        su2.su2_heatbath(lat, beta, nsw, seed)
        hb_ms, hb_n = su2.su2_get_timing(lat, su2.K_HEATBATH)
        su2.su2_destroy(lat)
        return P, dt, 1e3 * hb_ms / hb_n

    def graph():
        # the first run (graph capture included) gives the cold-start series;
        # the second, continuing the chain, is timed
        ens = su2.su2_ensemble_create([dims], [beta], su2.COLD, seed, su2.F64)
        su2.su2_ensemble_set_stream(ens, stream.cuda_stream)
        P, _ = su2.su2_ensemble_run(ens, 1, nsw, seed, True, False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        su2.su2_ensemble_run(ens, 1, nsw, seed, True, False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        su2.su2_ensemble_destroy(ens)
        return P[0], dt

    for _ in range(max(args.warmup, 1)):   # warm-up on throwaway lattices
        plain()
        graph()
    P, t_plain, hb_us = plain()
    Pg, t_graph = graph()
    return {
        "metric": "heat-bath link updates/s, 8^4 binary64 (launch-bound context)",
        "value": updates / t_graph, "unit": "link updates/s", "n_gpus": 1, "steps": nsw,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_graph / nsw, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (cold start)",
        "config": {"workload": cfg["desc"], "sites": int(np.prod(dims))},
        "plain_calls": {"value": updates / t_plain, "ms_per_step": 1e3 * t_plain / nsw,
                        "form": "su2_heatbath + su2_plaquette per sweep (synchronising)"},
        "hb_avg_launch_us": hb_us,
        "plaquettes": P,
        "graph_vs_plain_max_abs_dP": float(np.abs(np.asarray(Pg) - np.asarray(P)).max()),
    }


def bench_c4(su2, args, cfg, stream):
    """Per configuration: 5 heat-bath sweeps, APE smearing, Wilson loops."""
    import numpy as np
    import torch
    dims, beta, seed = cfg["dims"][0], cfg["betas"][0], cfg["seed"]
    V = int(np.prod(dims))
    nconf = max(2, args.steps // 20)
    lat = su2.Lattice(dims, start=su2.HOT, seed=seed, prec=su2.F32, stream=stream.cuda_stream)
    if args.launch:
        su2.su2_set_launch(lat.h, *[int(x) for x in args.launch.split(",")])
    elif not args.no_tune:
        su2.su2_autotune(lat.h, beta)
    lat.heatbath(beta, args.warmup, seed)

    def one_config():
        lat.heatbath(beta, 5, seed)
        lat.ape_smear(0.7, 25)
        return lat.wilson_loops(12, 16)

    one_config()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nconf):
        W = one_config()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    W = np.asarray(W).ravel()
    if not (np.isfinite(W).all() and W[0] > 0):
        raise RuntimeError("Wilson loops invalid")
    su2.su2_set_timing(lat.h, 1)
    for _ in range(nconf):
        one_config()
    t = {k: su2.su2_get_timing(lat.h, getattr(su2, k)) for k in ("K_HEATBATH", "K_APE", "K_WILSON")}
    su2.su2_set_timing(lat.h, 0)
    # binary32 error of APE + Wilson loops: the same configuration (its
    # binary32 link values) smeared and measured in binary64
    U = lat.get_links()
    W32 = np.asarray(lat.wilson_loops(12, 16)).reshape(12, 16)
    lat.close()
    lat64 = su2.Lattice(dims, start=su2.COLD, prec=su2.F64, stream=stream.cuda_stream)
    lat64.set_links(U)
    lat64.ape_smear(0.7, 25)
    W64 = np.asarray(lat64.wilson_loops(12, 16)).reshape(12, 16)
    lat64.close()
    err = np.abs(W32 - W64)
    ms = {k: v[0] / nconf for k, v in t.items()}
    ape_step_us = 1e3 * t["K_APE"][0] / max(t["K_APE"][1], 1)
    ape_bytes = 6 * V * 16   # 3V spatial links read, 3V written per step
    return {
        "metric": "APE smearing + Wilson loops time per configuration, 24^3x48",
        "value": ms["K_APE"] + ms["K_WILSON"], "unit": "ms per configuration", "n_gpus": 1,
        "steps": nconf, "warmup": args.warmup, "ms_per_step": 1e3 * secs / nconf,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (Philox hot start)",
        "config": {"workload": cfg["desc"], "lattices": 1, "sites": V},
        "kernel_ms_per_config": {"heatbath_5_sweeps": ms["K_HEATBATH"], "ape_25_steps": ms["K_APE"],
                                 "wilson_R12_T16": ms["K_WILSON"]},
        "ape_step": {"avg_launch_us": ape_step_us, "bytes_per_launch": ape_bytes,
                     "GBs": ape_bytes / (ape_step_us * 1e-6) / 1e9},
        "W_1_1": float(W[0]),
        "fp32_error": {"max_abs": float(err.max()),
                       "max_rel": float((err / np.abs(W64)).max()),
                       "abs_by_T_at_R12": err[11].tolist(),
                       "form": "binary32 APE + Wilson loops vs binary64 on the same configuration"},
    }


def fp64_loop(su2, dims_list, betas, seed, nsteps):
    """The plain FP64 single-lattice form looped over the lattices: per step
    one heat-bath sweep + plaquette of each lattice in turn."""
    import numpy as np
    import torch
    lats = [su2.Lattice(d, start=su2.HOT, seed=seed, prec=su2.F64) for d in dims_list]
    for lat, b in zip(lats, betas):
        lat.heatbath(b, 2, seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        for lat, b in zip(lats, betas):
            lat.heatbath(b, 1, seed)
            lat.plaquette()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    for lat in lats:
        lat.close()
    upd = 4 * sum(int(np.prod(d)) for d in dims_list) * nsteps
    return upd / secs, secs / nsteps


def timed_runs(su2, torch, stream, ens, n, steps, seed, poly, reps, every=1):
    """reps runs of `steps` sweeps with the series, each bracketed by device
    synchronisation.  Returns the median repetition's seconds (the larger of
    its wall and stream-event time), that repetition's event milliseconds and
    the seconds of every repetition."""
    res = []
    for _ in range(max(1, reps)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        su2.su2_ensemble_run(ens, n, steps, seed, True, poly, every)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gms = e0.elapsed_time(e1)
        res.append((max(wall, gms * 1e-3), gms))
    every = [r[0] for r in res]
    res.sort()
    return res[len(res) // 2] + (every,)


def eager_event_pass(su2, ens, n, steps, seed, poly):
    """K steps with graph replay off and every kernel timed with HIP events
    (heat-bath launches stamp their own start and end)."""
    import time as _t
    su2.su2_ensemble_set_timing(ens, 1)
    t0 = _t.perf_counter()
    su2.su2_ensemble_run(ens, n, steps, seed, True, poly)
    dt = _t.perf_counter() - t0
    hb_ms, hb_n = su2.su2_ensemble_get_timing(ens, su2.K_HEATBATH)
    po_ms, po_n = su2.su2_ensemble_get_timing(ens, su2.K_POLYAKOV)
    rd_ms, rd_n = su2.su2_ensemble_get_timing(ens, su2.K_REDUCE)
    su2.su2_ensemble_set_timing(ens, 0)
    return {"hb_avg_us": 1e3 * hb_ms / hb_n, "poly_avg_us": 1e3 * po_ms / max(po_n, 1),
            "reduce_avg_us": 1e3 * rd_ms / max(rd_n, 1), "reduce_n": rd_n, "ms_per_step": 1e3 * dt / steps}


def fp64_form(su2, torch, stream, dims, beta, seed, args, value32):
    """The plain FP64 single-lattice form: the same kernels instantiated for
    binary64, one lattice, the library's default launch shape, on the same
    schedule as the timed region (K steps of one sweep + plaquette, median
    of the repetitions); the autotuned binary64 shape as a side figure."""
    import numpy as np
    V = int(np.prod(dims))
    out = {}
    for label, tune in (("default", False), ("autotuned", not args.no_tune)):
        if label == "autotuned" and not tune:
            continue
        ens = su2.su2_ensemble_create([dims], [beta], su2.HOT, seed, su2.F64)
        su2.su2_ensemble_set_stream(ens, stream.cuda_stream)
        if tune:
            su2.su2_ensemble_autotune(ens)
        launch = su2.su2_ensemble_get_launch(ens)
        su2.su2_ensemble_run(ens, 1, 5, seed, True, False)
        k64 = max(10, args.steps)
        secs, _, _ = timed_runs(su2, torch, stream, ens, 1, k64, seed, False, 3)
        ev = eager_event_pass(su2, ens, 1, max(5, k64 // 4), seed, False)
        su2.su2_ensemble_destroy(ens)
        v64 = 4 * V * k64 / secs
        out[label] = {"value": v64, "ms_per_step": 1e3 * secs / k64, "steps": k64,
                      "hb_avg_launch_us": ev["hb_avg_us"],
                      "hb_GBs": (V // 2) * 256 / (ev["hb_avg_us"] * 1e-6) / 1e9,
                      "launch": dict(zip(("block", "grid", "xcd_remap", "links_per_lane"), launch)),
                      "speedup_fp32_batched": value32 / v64}
    out["form"] = ("same kernels in binary64, one lattice, same schedule (one sweep + plaquette per step, "
                   "graph replay), median of 3 repetitions")
    return out


def control64(su2, torch, stream, launch, seed, args):
    """The 64^4 binary32 lattice (1 GiB of links, four times the 256 MB
    Infinity Cache) under its own autotuned launch shape (the 32^4 shape with
    --no-tune or --launch): steps of one sweep + plaquette and the heat-bath
    launch time, the HBM-bound figure."""
    dims, beta = (64, 64, 64, 64), 2.6
    V = 64 ** 4
    ens = su2.su2_ensemble_create([dims], [beta], su2.HOT, seed, su2.F32)
    su2.su2_ensemble_set_stream(ens, stream.cuda_stream)
    if args.no_tune or args.launch:
        su2.su2_ensemble_set_launch(ens, *launch)
    else:
        su2.su2_ensemble_autotune(ens)
    launch = su2.su2_ensemble_get_launch(ens)
    su2.su2_ensemble_run(ens, 1, 2, seed, True, False)
    k = max(4, args.steps // 4)
    secs, gms, _ = timed_runs(su2, torch, stream, ens, 1, k, seed, False, 3)
    ev = eager_event_pass(su2, ens, 1, 3, seed, False)
    su2.su2_ensemble_destroy(ens)
    hb_bytes = (V // 2) * 128
    hb_us = 1e3 * gms / (8 * k)     # timed region, as the 32^4 roofline
    ach = hb_bytes / (hb_us * 1e-6) / 1e9
    traffic = None
    eff = (launch[0], effective_grid(launch[1], -(-(V // 2) // (launch[0] * launch[3]))), launch[2], launch[3])
    if kernel_sources_sha256() == HB_TRAFFIC["sources_sha256"]:
        traffic = HB_TRAFFIC["control64"].get(eff)
    return {"workload": "64^4, beta=2.6, hot start, binary32, 1 sweep + plaquette per step",
            "launch": dict(zip(("block", "grid", "xcd_remap", "links_per_lane"), launch)),
            "value": 4 * V * k / secs, "ms_per_step": 1e3 * secs / k, "steps": k,
            "step_frac": 4 * V * 128 / (secs / k) / 1e9 / HBM_PEAK_GBS,
            "avg_launch_us": hb_us, "bytes_per_launch": hb_bytes, "achieved": ach,
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
            "kernel_only": {"avg_launch_us": ev["hb_avg_us"],
                            "frac": hb_bytes / (ev["hb_avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c2", choices=sorted(configs()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run the 1 GiB device copy also for configurations other than c2")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=8)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads for the all-core oracle figure (0: min(16, cores))")
    ap.add_argument("--launch", default=None,
                    help="block,grid,xcd_remap,links_per_lane (skips tuning)")
    ap.add_argument("--reps", type=int, default=11,
                    help="timed repetitions of K steps; value is the median repetition")
    ap.add_argument("--no-control", action="store_true", help="skip the 64^4 control in the c2 line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is designed, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1010_4834_amd import su2

    cfg = configs()[args.config]
    dims, betas, seed = cfg["dims"], cfg["betas"], cfg["seed"]
    n = len(dims)
    V_tot = sum(int(np.prod(d)) for d in dims)
    updates_per_step = 4 * V_tot
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if args.config == "c4":
        print(json.dumps(bench_c4(su2, args, cfg, stream)), flush=True)
        return
    if args.config == "c1":
        print(json.dumps(bench_c1(su2, args, cfg, stream)), flush=True)
        return

    ens = su2.su2_ensemble_create(dims, betas, su2.HOT, seed, su2.F32)
    su2.su2_ensemble_set_stream(ens, stream.cuda_stream)
    if args.launch:
        su2.su2_ensemble_set_launch(ens, *[int(x) for x in args.launch.split(",")])
    elif not args.no_tune:
        su2.su2_ensemble_autotune(ens)
    block, grid, remap, nl = su2.su2_ensemble_get_launch(ens)
    su2.su2_ensemble_run(ens, n, args.warmup, seed, True, cfg["poly"])

    # ---- timed region: reps x K steps (graph replay, the series stay on the
    # device until the end of each run); value from the median repetition ----
    secs, gpu_ms, rep_secs = timed_runs(su2, torch, stream, ens, n, args.steps, seed, cfg["poly"], args.reps)
    value = updates_per_step * args.steps / secs
    P, _ = su2.su2_ensemble_run(ens, n, 1, seed, True, cfg["poly"])
    if not (np.isfinite(P).all() and (P > 0).all() and (P < 1).all()):
        raise RuntimeError("plaquette series invalid")

    # ---- dominant kernel: the timed region's GPU time (events on the
    # library's stream around the median repetition) over its 8 K heat-bath
    # launches, every per-run fixed cost charged to them; and, kernel only,
    # an eager pass of K steps whose heat-bath launches stamp HIP events ----
    ev = eager_event_pass(su2, ens, n, args.steps, seed, cfg["poly"])
    hb_avg_us = 1e3 * gpu_ms / (8 * args.steps)
    traffic = None
    eff_grid = effective_grid(grid, -(-(updates_per_step // 8) // (block * nl)))
    if args.config == "c2" and kernel_sources_sha256() == HB_TRAFFIC["sources_sha256"]:
        traffic = HB_TRAFFIC["by_launch"].get((block, eff_grid, remap, nl))
    link_b = 16
    hb_bytes = (updates_per_step // 8) * 8 * link_b   # per substep: V/2 updates x 128 B
    achieved = hb_bytes / (hb_avg_us * 1e-6) / 1e9
    step_GBs = updates_per_step * 8 * link_b / (secs / args.steps) / 1e9
    tries, updates = su2.su2_ensemble_stats(ens)
    fp32_err = None
    if n == 1:
        # binary32 error of the measurements: the final configuration (its
        # binary32 link values) measured by a binary32 and a binary64 lattice
        U = su2.su2_ensemble_get_links(ens, 0, V_tot)
        meas = {}
        for prec in (su2.F32, su2.F64):
            lat = su2.su2_create(*dims[0], su2.COLD, seed, prec)
            su2.su2_set_stream(lat, stream.cuda_stream)
            su2.su2_set_links(lat, U)
            meas[prec] = (su2.su2_plaquette(lat), su2.su2_polyakov(lat))
            su2.su2_destroy(lat)
        (p32, l32), (p64, l64) = meas[su2.F32], meas[su2.F64]
        fp32_err = {"plaquette": max(abs(a - b) for a, b in zip(p32, p64)), "polyakov": abs(l32 - l64),
                    "form": "binary32 kernels (binary64 sums) vs binary64 on the same configuration"}
    # over-relaxation sweeps (paper Sec. 2, over-relaxation equation) of the
    # same final configuration at the same launch shape: 7 staple links and
    # the old link read, the new one written, 144 B per update in binary32
    overrelax = None
    if n == 1:
        lat = su2.su2_create(*dims[0], su2.COLD, seed, su2.F32)
        su2.su2_set_stream(lat, stream.cuda_stream)
        su2.su2_set_links(lat, U)
        su2.su2_set_launch(lat, block, grid, remap, 1)
        su2.su2_overrelax(lat, 2)
        su2.su2_set_timing(lat, 1)
        su2.su2_overrelax(lat, max(5, args.steps // 4))
        or_ms, or_n = su2.su2_get_timing(lat, su2.K_OVERRELAX)
        su2.su2_destroy(lat)
        or_us = 1e3 * or_ms / or_n
        or_bytes = (updates_per_step // 8) * 9 * link_b
        overrelax = {"kernel": "k_overrelax<float> (one checkerboard substep)", "avg_launch_us": or_us,
                     "bytes_per_launch": or_bytes, "GBs": or_bytes / (or_us * 1e-6) / 1e9,
                     "frac": or_bytes / (or_us * 1e-6) / 1e9 / HBM_PEAK_GBS}
    su2.su2_ensemble_destroy(ens)

    resident = updates_per_step * link_b <= INFINITY_CACHE_BYTES
    out = {
        "metric": "heat-bath link updates/s + HBM GB/s fraction, FP32 batched vs FP64 at 32^4",
        "value": value,
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * secs / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (Philox hot start)",
        "config": {"workload": cfg["desc"], "lattices": n, "sites": V_tot,
                   "links": "binary32, binary64 reductions and norm", "sweeps_per_step": 1,
                   "sampler": "Kennedy-Pendleton (alpha>=2) / Creutz",
                   "launch": {"block": block, "grid": grid, "xcd_remap": remap,
                              "links_per_lane": nl}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_heatbath<float> (one checkerboard substep)",
                     "bytes_per_launch": hb_bytes, "avg_launch_us": hb_avg_us,
                     "avg_launch_source": "timed region: HIP events on the library's stream around the "
                                          "median repetition, divided by its 8 K heat-bath launches "
                                          "(the per-run state, series-reduction and error-word kernels "
                                          "and every gap charged to them)",
                     "kernel_only": {"avg_launch_us": ev["hb_avg_us"],
                                     "frac": hb_bytes / (ev["hb_avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                     "source": "eager pass of K steps after the timed region, each "
                                               "heat-bath launch stamping HIP events with its own start "
                                               "and end (graph replay off)"},
                     "step_frac": step_GBs / HBM_PEAK_GBS,
                     "links_in_infinity_cache": resident},
        "timing": {"reps": args.reps, "rep_ms_per_step": [1e3 * t / args.steps for t in rep_secs],
                   "gpu_event_ms_median_rep": gpu_ms,
                   "eager_pass_ms_per_step": ev["ms_per_step"]},
        "other_kernels_us": {"polyakov": ev["poly_avg_us"], "series_reduction_per_batch": ev["reduce_avg_us"],
                             "series_reduction_batches": ev["reduce_n"]},
        "plaquette": "summed inside the odd heat-bath substeps (no separate pass)",
        "step_GBs": step_GBs,
        "tries_per_update": tries / max(updates, 1),
        "fp32_error": fp32_err,
    }
    if overrelax:
        out["overrelax"] = overrelax

    # ---- the plain FP64 single-lattice form on the same GPU and schedule ----
    if not args.no_fp64 and n == 1:
        out["fp64_plain"] = fp64_form(su2, torch, stream, dims[0], betas[0], seed, args, value)

    if not args.no_fp64 and n > 1:
        v64, s64 = fp64_loop(su2, dims, betas, seed, max(5, args.steps // 20))
        out["fp64_plain_loop"] = {"value": v64, "ms_per_step": 1e3 * s64,
                                  "form": "plain FP64 single-lattice calls looped over the lattices",
                                  "speedup_fp32_batched": value / v64}

    # ---- the HBM-bound control: 64^4 (1 GiB of links, beyond the cache) ----
    if args.config == "c2" and not args.no_control:
        out["control64"] = control64(su2, torch, stream, (block, grid, remap, nl), seed, args)

    if (args.config == "c2" or args.copy_probe) and not args.no_copy_probe:
        out["copy_probe_GBs"] = copy_probe(torch)

    if not args.no_cpu_baseline and args.config == "c2":
        rate, dt = cpu_baseline(dims[0], betas[0], seed, args.cpu_sweeps)
        out["cpu_baseline"] = {"value": rate, "unit": "link updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"{args.cpu_sweeps} heat-bath sweeps + plaquette of the "
                                         f"32^4 beta=2.6 hot-start lattice, serial FP64 oracle, "
                                         f"{dt:.1f} s"}
        out["host"] = host_info()
        nthr = args.cpu_threads or min(16, os.cpu_count() or 1)
        if nthr > 1:
            agg, dt = cpu_all_cores(dims[0], betas[0], 2, nthr)
            out["cpu_all_cores"] = {"value": agg, "unit": "link updates/s", "cores": nthr, "kind": "oracle",
                                    "sample": f"{nthr} host threads at once, each 2 sweeps + plaquette of "
                                              f"its own 32^4 lattice, serial FP64 oracle, {dt:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
