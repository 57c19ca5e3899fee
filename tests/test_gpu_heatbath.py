"""GPU parity of the heat-bath path against the serial FP64 oracle, through
the C ABI (libsu2.so).

FP64: one substep / one sweep from an identical configuration agrees link by
link to 1e-12 with identical per-link try counts.  FP32 (links rounded to
binary32, 23-bit uniforms on both sides): links agree to 1e-5 except
downstream of accept/reject flips and within the first-order binary32
rounding bound of an ill-conditioned update, each class counted and
reported (tests/parity_util.check_fp32_sweep).
"""
import numpy as np
import pytest

from tests import inputs, parity_util

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def su2():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1010_4834_amd import su2 as s
    return s


def as_f32(U):
    return U.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 10, 6)])
def test_hot_start(su2, orc, dims):
    for prec, tol in ((su2.F64, 1e-14), (su2.F32, 6e-8)):
        lat = su2.Lattice(dims, start=su2.HOT, seed=2, prec=prec)
        G = lat.get_links()
        O = orc.hot(dims, 2)
        assert np.abs(G - O).max() < tol
        lat.close()
    lat = su2.Lattice(dims, start=su2.COLD, seed=2, prec=su2.F32)
    assert lat.plaquette() == (1.0, 1.0, 1.0)
    assert lat.polyakov() == 1.0
    lat.close()


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 10, 6), (2, 2, 2, 2)])
def test_substeps_fp64(su2, orc, dims):
    V = int(np.prod(dims))
    U = inputs.random_config(dims, 31)
    lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F64)
    lat.set_links(U)
    lat.trace_tries(True)
    lat.sweep = 5
    tr = np.zeros(4 * V, np.uint32)
    for mu in range(4):
        for p in range(2):
            lat.substep(2.3, 11, mu, p)
            orc.heatbath_substep(dims, U, 2.3, 11, 5, mu, p, trace=tr)
            G = lat.get_links()
            assert np.abs(G - U).max() < 1e-12, (mu, p)
    assert np.array_equal(lat.get_tries(), tr)
    lat.close()


@pytest.mark.parametrize("dims,beta,seed", [((8, 8, 8, 8), 2.3, 1), ((6, 4, 10, 6), 2.6, 3),
                                            ((4, 6, 2, 8), 0.4, 9), ((4, 4, 6, 4), 0.0, 11),
                                            ((4, 4, 4, 6), 12.0, 5)])
def test_sweep_fp64(su2, orc, dims, beta, seed):
    """One binary64 sweep from a random configuration: links within 1e-12 of
    the oracle and identical per-link try counts and sampler branches; beta = 0
    is the alpha = 0 branch (a0 uniform on [-1, 1]), beta = 12 the deep
    Kennedy-Pendleton regime (a0 near 1)."""
    V = int(np.prod(dims))
    U = inputs.random_config(dims, 32)
    lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F64)
    lat.set_links(U)
    lat.trace_tries(True)
    lat.heatbath(beta, 1, seed)
    tr = np.zeros(4 * V, np.uint32)
    orc.heatbath_sweep(dims, U, beta, seed, 0, trace=tr)
    assert np.array_equal(lat.get_tries(), tr)
    assert np.abs(lat.get_links() - U).max() < 1e-12
    tries, updates, defect = lat.stats()
    assert updates == 4 * V and tries == int((tr & 0x7FFFFFFF).sum())
    assert defect < 1e-14
    lat.close()


def test_creutz_sampler_fp64(su2, orc):
    dims = (4, 4, 6, 4)
    V = int(np.prod(dims))
    U = inputs.random_config(dims, 33)
    lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F64)
    su2.su2_set_sampler(lat.h, su2.CREUTZ)
    lat.set_links(U)
    lat.trace_tries(True)
    lat.heatbath(2.5, 1, 4)
    tr = np.zeros(4 * V, np.uint32)
    orc.heatbath_sweep(dims, U, 2.5, 4, 0, sampler=orc.CREUTZ, trace=tr)
    assert np.array_equal(lat.get_tries(), tr)
    assert np.abs(lat.get_links() - U).max() < 1e-12
    lat.close()


def test_c1_series_fp64(su2, orc):
    """8^4, beta = 2.3, cold start, 20 sweeps, Philox seed 1, plaquette after
    each sweep.  Beyond one sweep link-by-link agreement is not guaranteed in
    principle (a flip would decorrelate); in practice the FP64 maps stay
    within rounding, which is asserted loosely and printed."""
    dims = (8, 8, 8, 8)
    lat = su2.Lattice(dims, start=su2.COLD, seed=1, prec=su2.F64)
    U = orc.cold(dims)
    dp = []
    for sw in range(20):
        lat.heatbath(2.3, 1, 1)
        orc.heatbath_sweep(dims, U, 2.3, 1, sw)
        dp.append(abs(lat.plaquette()[0] - orc.plaquette(dims, U)[0]))
    print("C1 |dP| per sweep:", " ".join(f"{x:.1e}" for x in dp))
    assert max(dp) < 1e-10
    assert np.abs(lat.get_links() - U).max() < 1e-9
    lat.close()


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 10, 6)])
def test_sweep_fp32(su2, orc, dims):
    V = int(np.prod(dims))
    U0 = as_f32(inputs.random_config(dims, 34))
    U = U0.copy()
    lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F32)
    lat.set_links(U)
    lat.trace_tries(True)
    lat.heatbath(2.3, 1, 5)
    tr = np.zeros(4 * V, np.uint32)
    orc.heatbath_sweep(dims, U, 2.3, 5, 0, ubits=23, trace=tr)
    r = parity_util.check_fp32_sweep(orc, dims, 2.3, U0, lat.get_links(), U, lat.get_tries(), tr)
    assert r["flips"] <= max(2, V // 1000)
    lat.close()


@pytest.mark.parametrize("beta", [0.0, 0.4, 1.0, 12.0])
def test_sweep_fp32_coupling_range(su2, orc, beta):
    """Binary32 sweeps across the sampler's regimes, from a random
    configuration on the ragged lattice: beta = 0 (the uniform alpha = 0
    draw), 0.4 and 1.0 (mostly Creutz, alpha < 2), 12 (Kennedy-Pendleton
    far out in alpha, delta = 1 - a0 small)."""
    dims = (6, 4, 10, 6)
    V = int(np.prod(dims))
    U0 = as_f32(inputs.random_config(dims, 36))
    U = U0.copy()
    lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F32)
    lat.set_links(U)
    lat.trace_tries(True)
    lat.heatbath(beta, 1, 8)
    tr = np.zeros(4 * V, np.uint32)
    orc.heatbath_sweep(dims, U, beta, 8, 0, ubits=23, trace=tr)
    r = parity_util.check_fp32_sweep(orc, dims, beta, U0, lat.get_links(), U, lat.get_tries(), tr,
                                     label=f"beta {beta:g} ")
    assert r["flips"] <= max(2, V // 1000)
    lat.close()


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_full_size_c2_one_sweep(su2, orc, prec):
    """32^4, beta = 2.6, hot start seed 2: one sweep at the benchmark shape."""
    dims = (32, 32, 32, 32)
    p = getattr(su2, prec)
    lat = su2.Lattice(dims, start=su2.HOT, seed=2, prec=p)
    su2.su2_autotune(lat.h, 2.6)
    print("launch", su2.su2_get_launch(lat.h))
    # the oracle starts from the library's own hot start (its binary32 values
    # in FP32), checked against the oracle's hot start first
    U0 = lat.get_links()
    assert np.abs(U0 - orc.hot(dims, 2)).max() < (1e-14 if prec == "F64" else 6e-8)
    U = U0.copy()
    lat.trace_tries(True)
    lat.heatbath(2.6, 1, 2)
    V = U.shape[0]
    tr = np.zeros(4 * V, np.uint32)
    orc.heatbath_sweep(dims, U, 2.6, 2, 0, ubits=23 if prec == "F32" else 32, trace=tr)
    G = lat.get_links()
    if prec == "F64":
        assert np.array_equal(lat.get_tries(), tr)
        assert np.abs(G - U).max() < 1e-12
    else:
        parity_util.check_fp32_sweep(orc, dims, 2.6, U0, G, U, lat.get_tries(), tr, label="C2 ")
    P = lat.plaquette()
    Po = orc.plaquette(dims, U)
    assert abs(P[0] - Po[0]) < (1e-13 if prec == "F64" else 1e-6)
    lat.close()


@pytest.mark.parametrize("prec", ["F32", "F64"])
def test_try_recording_changes_nothing(su2, prec):
    """The parity tests compare the kernels that record per-link try counts;
    production runs use the forms without the record.  Both give bit for bit
    the same links and series: 32^4 at beta = 2.6 under the benchmark's
    autotuned shape, two measured sweeps (the fused-plaquette forms, and the
    Polyakov kernel) and one unmeasured sweep."""
    dims = (32, 32, 32, 32)
    p = getattr(su2, prec)
    shape, out = None, []
    for record in (False, True):
        ens = su2.Ensemble([dims], [2.6], start=su2.HOT, seed=2, prec=p)
        if shape is None:
            su2.su2_ensemble_autotune(ens.h)
            shape = su2.su2_ensemble_get_launch(ens.h)
            print("launch", shape, flush=True)
        else:
            su2.su2_ensemble_set_launch(ens.h, *shape)
        ens.trace_tries(record)
        P, L = ens.run(2, 2)
        ens.run(1, 2, plaq=False, poly=False)
        out.append((P, L, ens.get_links(0)))
        ens.close()
    (a, b) = out
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


def test_launch_shapes_bitwise(su2, orc):
    """FP64 links do not depend on the launch shape, the tile mode (all four)
    or graph replay."""
    import os
    dims = (6, 4, 10, 6)
    U = inputs.random_config(dims, 35)
    ref = None
    for block, grid, remap, nl in ((256, 0, 1, 1), (64, 0, 0, 2), (128, 16, 1, 4), (192, 8, 0, 1),
                                   (64, 24, 1, 4), (256, 0, 0, 2), (128, 0, 2, 1), (64, 16, 2, 2),
                                   (64, 0, 3, 1), (128, 16, 3, 2)):
        lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F64)
        su2.su2_set_launch(lat.h, block, grid, remap, nl)
        lat.set_links(U)
        lat.heatbath(2.4, 3, 6)
        G = lat.get_links()
        if ref is None:
            ref = G
        assert np.array_equal(G, ref), (block, grid, remap, nl)
        lat.close()
    os.environ["SU2_NO_GRAPH"] = "1"
    try:
        lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F64)
        lat.set_links(U)
        lat.heatbath(2.4, 3, 6)
        assert np.array_equal(lat.get_links(), ref)
        lat.close()
    finally:
        del os.environ["SU2_NO_GRAPH"]


def test_launch_shapes_bitwise_fp32(su2):
    """Binary32 links do not depend on the launch shape either."""
    dims = (8, 6, 4, 10)
    U = inputs.random_config(dims, 37).astype(np.float32).astype(np.float64)
    out = []
    for launch in ((256, 0, 1, 1), (128, 0, 1, 2), (64, 16, 0, 4), (192, 8, 1, 2), (128, 0, 2, 1), (64, 0, 3, 1)):
        lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F32)
        su2.su2_set_launch(lat.h, *launch)
        assert su2.su2_get_launch(lat.h) == launch
        lat.set_links(U)
        lat.heatbath(2.5, 2, 3)
        out.append(lat.get_links())
        lat.close()
    for G in out[1:]:
        assert np.array_equal(G, out[0])


def test_launch_shapes_bitwise_full_size(su2):
    """At 32^4 (4096 tiles of 128 half-sites) the benchmark's autotuner
    candidates agree bit for bit: one link per lane in every tile mode, two
    and four links per lane, two tiles per workgroup and the
    occupancy-exact persistent grid; two sweeps from the binary32 hot
    start."""
    dims = (32, 32, 32, 32)
    ref = None
    for launch in ((128, 0, 3, 1), (64, 0, 1, 1), (256, 0, 2, 1), (128, 0, 0, 2), (64, 0, 3, 4),
                   (128, 2048, 3, 1), (128, 3584, 3, 1)):
        lat = su2.Lattice(dims, start=su2.HOT, seed=2, prec=su2.F32)
        su2.su2_set_launch(lat.h, *launch)
        lat.heatbath(2.6, 2, 2)
        G = lat.get_links()
        lat.close()
        if ref is None:
            ref = G
        else:
            assert np.array_equal(G, ref), launch


def test_overrelax_fp64(su2, orc):
    dims = (6, 4, 4, 8)
    U = inputs.random_config(dims, 36)
    lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F64)
    lat.set_links(U)
    p0 = lat.plaquette()[0]
    lat.overrelax(2)
    orc.overrelax_sweep(dims, U)
    orc.overrelax_sweep(dims, U)
    assert np.abs(lat.get_links() - U).max() < 1e-12
    assert abs(lat.plaquette()[0] - p0) < 1e-13
    lat.close()


def test_overrelax_fp32(su2, orc):
    """One binary32 over-relaxation sweep against the binary64 oracle from the
    same binary32 links: U' = W^dag U^dag W^dag carries the staple error
    twice through W = V/k, so each link stays within
    2 E_V / k + 16u, E_V the staple rounding bound plus the differences of
    its links updated earlier in the sweep (tests/parity_util)."""
    dims = (8, 6, 4, 10)
    U0 = as_f32(inputs.random_config(dims, 38))
    O = U0.copy()
    lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F32)
    lat.set_links(U0)
    lat.overrelax(1)
    orc.overrelax_sweep(dims, O)
    check_overrelax_fp32(orc, dims, U0, lat.get_links(), O)
    lat.close()


def check_overrelax_fp32(orc, dims, U0, G, O):
    """Binary32 over-relaxed links G against the binary64 oracle's O, both
    from U0: every link within 1e-5 or within its bound 2 E_V / k + 16u,
    and at most one link in 10^5 plus five needing the bound."""
    err = np.abs(G - O).max(axis=2)
    par = parity_util.parity_array(dims)
    over = list(zip(*np.nonzero(err > 1e-5)))
    masks = {}
    for s, mu in over:
        s, mu = int(s), int(mu)
        key = (mu, int(par[s]))
        if key not in masks:
            earlier = parity_util.link_before_mask(par, mu, key[1])
            masks[key] = (earlier, np.where(earlier[..., None], O, U0))
        earlier, before = masks[key]
        k = float(np.linalg.norm(orc.staple(dims, before, s, mu)))
        ein = sum(float(np.linalg.norm(G[j, nu] - O[j, nu]))
                  for j, nu in parity_util.staple_link_ids(orc, dims, s, mu) if earlier[j, nu])
        bound = 2 * (parity_util.STAPLE_ROUNDING + ein) / k + 16 * parity_util.U32
        assert err[s, mu] <= bound, (s, mu, err[s, mu], bound)
    print(f"FP32 over-relaxation {dims}: max |dU| {err.max():.2e}, {len(over)} links > 1e-5 within their bound")
    assert len(over) <= err.size * 1e-5 + 5


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_overrelax_full_size(su2, orc, prec):
    """One over-relaxation sweep at 32^4 under the benchmark's autotuned
    launch shape against the oracle, from the configuration the benchmark
    over-relaxes: the hot start (seed 2) after heat-bath sweeps at beta =
    2.6 (on the GPU; both sides then start from its links).  Binary64 to
    1e-12 per link with the plaquette unchanged; binary32 by the bound
    above.  (From the Haar-random hot start itself about 0.08% of the
    staples are small enough to need the bound.)"""
    dims = (32, 32, 32, 32)
    lat = su2.Lattice(dims, start=su2.HOT, seed=2, prec=getattr(su2, prec))
    su2.su2_autotune(lat.h, 2.6)
    print("launch", su2.su2_get_launch(lat.h), flush=True)
    lat.heatbath(2.6, 5, 2)
    U0 = lat.get_links()
    O = U0.copy()
    p0 = lat.plaquette()[0]
    lat.overrelax(1)
    orc.overrelax_sweep(dims, O)
    G = lat.get_links()
    if prec == "F64":
        assert np.abs(G - O).max() < 1e-12
        assert abs(lat.plaquette()[0] - p0) < 1e-13
    else:
        check_overrelax_fp32(orc, dims, U0, G, O)
    lat.close()


def test_resume_bitwise(su2, tmp_path):
    dims = (4, 6, 4, 6)
    for prec in (su2.F64, su2.F32):
        a = su2.Lattice(dims, start=su2.HOT, seed=8, prec=prec)
        a.heatbath(2.5, 4, 8)
        b = su2.Lattice(dims, start=su2.HOT, seed=8, prec=prec)
        b.heatbath(2.5, 2, 8)
        path = str(tmp_path / "ck.su2")
        su2.su2_save(b.h, path)
        b.close()
        h = su2.su2_load(path)
        assert su2.su2_get_sweep(h) == 2
        su2.su2_heatbath(h, 2.5, 2, 8)
        assert np.array_equal(su2.su2_get_links(h, a.volume), a.get_links())
        su2.su2_destroy(h)
        a.close()


def test_errors(su2):
    dims = (4, 4, 4, 4)
    lat = su2.Lattice(dims, start=su2.COLD, prec=su2.F32)
    bad = np.zeros((256, 4, 4))
    with pytest.raises(su2.SU2Error) as e:
        lat.set_links(bad)
    assert e.value.status == su2.EINVAL
    for args in ((-1.0, 1, 1), (float("nan"), 1, 1), (2.0, -1, 1)):
        with pytest.raises(su2.SU2Error) as e:
            lat.heatbath(*args)
        assert e.value.status == su2.EINVAL
    with pytest.raises(su2.SU2Error):
        lat.wilson_loops(5, 2)
    with pytest.raises(su2.SU2Error):
        su2.su2_set_launch(lat.h, 100, 0, 1)
    for bad in ((128, 0, 4, 1), (128, 0, -1, 1), (128, 12, 1, 1), (128, 0, 1, 3)):
        with pytest.raises(su2.SU2Error) as e:
            su2.su2_set_launch(lat.h, *bad)
        assert e.value.status == su2.EINVAL, bad
    with pytest.raises(su2.SU2Error) as e:
        lat.get_smeared()
    assert e.value.status == su2.ESTATE
    lat.heatbath(0.0, 2, 3)           # beta = 0: Haar draws, no hang
    assert lat.stats()[2] < 1e-6
    lat.close()


def test_extents_and_host_sizes(su2):
    """The extent queries return what the handles were created with, and the
    binding refuses a host array or volume that disagrees with them (the
    library itself reads and writes whole lattices through bare pointers)."""
    lat = su2.Lattice((4, 6, 2, 8), start=su2.COLD, prec=su2.F32)
    assert su2.su2_get_dims(lat.h) == (4, 6, 2, 8)
    with pytest.raises(ValueError):
        su2.su2_get_links(lat.h, 100)
    with pytest.raises(ValueError):
        lat.set_links(np.zeros((10, 4, 4)))
    with pytest.raises(ValueError):
        su2.su2_get_tries(lat.h, 5)
    assert su2.su2_get_links(lat.h).shape == (384, 4, 4)
    lat.close()
    ens = su2.Ensemble([(4, 4, 4, 4), (6, 4, 2, 8)], [2.0, 2.5], prec=su2.F32)
    assert su2.su2_ensemble_count(ens.h) == 2
    assert su2.su2_ensemble_get_dims(ens.h, 1) == (6, 4, 2, 8)
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_ensemble_get_dims(ens.h, 2)
    assert e.value.status == su2.EINVAL
    with pytest.raises(ValueError):
        su2.su2_ensemble_run(ens.h, 1, 2, 3)
    with pytest.raises(ValueError):
        su2.su2_ensemble_get_links(ens.h, 0, 384)
    with pytest.raises(ValueError):
        ens.set_links(1, np.zeros((256, 4, 4)))
    P, L = su2.su2_ensemble_run(ens.h, None, 2, 3)
    assert P.shape == (2, 2) and L.shape == (2, 2) and np.isfinite(P).all()
    assert ens.get_links(1).shape == (384, 4, 4)
    ens.close()
