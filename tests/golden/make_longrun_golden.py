"""Writes longrun_oracle.json: the expected values of the long-run GPU tests,
from long serial-oracle heat-bath chains at the full workload shapes --
bin means of the mean plaquette and |Polyakov loop| at 32^4 (beta = 2.6)
and for the 64 uneven lattices, and smeared Wilson loops of configurations
5 sweeps apart at 24^3 x 48 (beta = 2.5).  Calls only the oracle (and the
workload shapes of tests/inputs.py); runs for about an hour on 8 host
threads.  Parts already in the file are kept unless named.

    python tests/golden/make_longrun_golden.py [--threads 8] [--parts c5,c2,c4]

Every plaquette/Polyakov chain starts hot, runs `discard` sweeps, then
`nbins * per_bin` sweeps measured after each sweep; a bin mean is the
plain average of its per_bin measurements (plaquette: (1/6V) sum of 1/2 Re
Tr U_P; Polyakov: the signed loop, averaged as |L|).  A Wilson-loop chain
starts hot, runs `ntherm` sweeps, then per configuration `nsep` sweeps,
APE smearing (alpha, nape steps) of the spatial links and W(R, T) at the
listed (R, T)."""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from tests import inputs  # noqa: E402

# 32^4 at beta = 2.6: eight independent chains
C2_RUN = dict(dims=(32, 32, 32, 32), beta=2.6, seeds=[9001 + k for k in range(8)],
              discard=100, nbins=10, per_bin=50)
# the 64 uneven lattices, one chain each
C5_RUN = dict(seed=9101, discard=200, nbins=20, per_bin=100)
# 24^3 x 48 at beta = 2.5: seven chains of 15 configurations
C4_RUN = dict(dims=(24, 24, 24, 48), beta=2.5, seeds=[9201 + k for k in range(7)], ntherm=100, nconf=15,
              nsep=5, alpha=0.7, nape=25, RT=[[1, 1], [2, 2], [4, 4], [2, 4], [4, 2], [6, 6], [8, 8]])


def chain(dims, beta, seed, discard, nbins, per_bin, lat_id=0):
    U = orc.hot(dims, seed, lat_id)
    P = np.empty(nbins * per_bin)
    L = np.empty(nbins * per_bin)
    for sw in range(discard + nbins * per_bin):
        orc.heatbath_sweep(dims, U, beta, seed, sw, lat_id)
        k = sw - discard
        if k >= 0:
            P[k] = orc.plaquette(dims, U)[0]
            L[k] = abs(orc.polyakov(dims, U))
    return (P.reshape(nbins, per_bin).mean(axis=1).tolist(),
            L.reshape(nbins, per_bin).mean(axis=1).tolist())


def wilson_chain(r, seed):
    dims = r["dims"]
    U = orc.hot(dims, seed)
    sw = 0
    for _ in range(r["ntherm"]):
        orc.heatbath_sweep(dims, U, r["beta"], seed, sw)
        sw += 1
    out = []
    for _ in range(r["nconf"]):
        for _ in range(r["nsep"]):
            orc.heatbath_sweep(dims, U, r["beta"], seed, sw)
            sw += 1
        S = orc.ape(dims, U, r["alpha"], r["nape"])
        out.append([orc.wilson_rt(dims, U, R, T, S) for R, T in r["RT"]])
    return out


def run_c4(pool):
    r = C4_RUN
    t0 = time.perf_counter()
    fut = [pool.submit(wilson_chain, r, s) for s in r["seeds"]]
    out = dict(r, chains=[dict(seed=s, W=f.result()) for s, f in zip(r["seeds"], fut)])
    print(f"C4: {len(r['seeds'])} chains in {time.perf_counter() - t0:.0f} s", flush=True)
    return out


def run_c2(pool):
    r = C2_RUN
    t0 = time.perf_counter()
    fut = [pool.submit(chain, r["dims"], r["beta"], s, r["discard"], r["nbins"], r["per_bin"]) for s in r["seeds"]]
    out = dict(r, chains=[dict(seed=s, P_bins=f.result()[0], L_bins=f.result()[1]) for s, f in zip(r["seeds"], fut)])
    print(f"32^4: {len(r['seeds'])} chains in {time.perf_counter() - t0:.0f} s", flush=True)
    return out


def run_c5(pool):
    r = C5_RUN
    dims, betas = inputs.c5_shapes()
    t0 = time.perf_counter()
    order = sorted(range(len(dims)), key=lambda i: -int(np.prod(dims[i])))   # largest first
    fut = {i: pool.submit(chain, dims[i], betas[i], r["seed"], r["discard"], r["nbins"], r["per_bin"], i)
           for i in order}
    lat = []
    for i in range(len(dims)):
        P, L = fut[i].result()
        lat.append(dict(dims=list(dims[i]), beta=betas[i], lat_id=i, P_bins=P, L_bins=L))
    print(f"C5: {len(dims)} chains in {time.perf_counter() - t0:.0f} s", flush=True)
    return dict(r, lattices=lat)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--parts", default="c5,c2,c4")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "longrun_oracle.json"))
    args = ap.parse_args()
    orc.lib()
    doc = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            doc = json.load(f)
    doc.update({"what": "long serial FP64 oracle heat-bath chains (hot start): bin means of <P> and <|L|>; "
                        "smeared Wilson loops per configuration",
                "script": "tests/golden/make_longrun_golden.py"})
    runs = {"c5": run_c5, "c2": run_c2, "c4": run_c4}
    with ThreadPoolExecutor(args.threads) as pool:
        for part in args.parts.split(","):
            doc[part] = runs[part](pool)
            with open(args.out, "w") as f:
                json.dump(doc, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
