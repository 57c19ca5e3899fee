"""The stored long-run oracle expectations match the workload shapes and
the schedule the GPU long-run tests assume (no GPU needed)."""
import json
import os

import numpy as np

from tests import inputs

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "longrun_oracle.json")


def test_longrun_golden_layout():
    with open(GOLD) as f:
        g = json.load(f)
    c2 = g["c2"]
    assert tuple(c2["dims"]) == inputs.C2["dims"] and c2["beta"] == inputs.C2["beta"]
    assert len({c["seed"] for c in c2["chains"]}) == len(c2["chains"]) == 8
    for c in c2["chains"]:
        assert len(c["P_bins"]) == len(c["L_bins"]) == c2["nbins"]
    dims, betas = inputs.c5_shapes()
    lats = g["c5"]["lattices"]
    assert [tuple(l["dims"]) for l in lats] == list(dims)
    assert np.allclose([l["beta"] for l in lats], betas, rtol=0, atol=0)
    assert [l["lat_id"] for l in lats] == list(range(64))
    for l in lats:
        assert len(l["P_bins"]) == len(l["L_bins"]) == g["c5"]["nbins"]
        # plaquette averages lie in (0, 1), |L| in [0, 1]
        assert all(0 < p < 1 for p in l["P_bins"]) and all(0 <= q <= 1 for q in l["L_bins"])
    c4 = g["c4"]
    assert tuple(c4["dims"]) == inputs.C4["dims"] and c4["beta"] == inputs.C4["beta"]
    for c in c4["chains"]:
        assert np.asarray(c["W"]).shape == (c4["nconf"], len(c4["RT"]))


def test_longrun_golden_physics():
    """Coarse physics checks of the stored chains: on every (L, Nt) class of
    the uneven lattices the plaquette rises with beta, and the square Wilson
    loops fall with their size."""
    with open(GOLD) as f:
        g = json.load(f)
    by_class = {}
    for l in g["c5"]["lattices"]:
        by_class.setdefault(tuple(l["dims"]), []).append((l["beta"], np.mean(l["P_bins"])))
    for pts in by_class.values():
        pts.sort()
        assert all(b[1] > a[1] for a, b in zip(pts, pts[1:]))
    W = np.mean([np.mean(c["W"], axis=0) for c in g["c4"]["chains"]], axis=0)
    sq = [k for k, (r, t) in enumerate(g["c4"]["RT"]) if r == t]
    assert np.all(np.diff(W[sq]) < 0) and 0 < W[sq][-1]
