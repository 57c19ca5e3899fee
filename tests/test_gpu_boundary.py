"""GPU tests of the C-ABI contract beyond the sweep itself: measurements every
k-th sweep inside the captured graphs, numeric failures reported by the call
that caused them, and configuration files written and read outside the
library."""
import struct

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


def test_measure_every_fp64(su2, orc):
    """Runs that measure every 5th and every 3rd sweep: the series hold the
    oracle's plaquette and Polyakov loop after exactly those sweeps, the
    trailing sweeps measure nothing, and the chain continues across runs."""
    dims = [(4, 4, 4, 4), (6, 4, 2, 8)]
    betas = [2.3, 2.6]
    ens = su2.Ensemble(dims, betas, start=su2.HOT, seed=5, prec=su2.F64)
    P1, L1 = ens.run(12, 5, measure_every=5)   # after sweeps 5, 10; 11, 12 plain
    P2, L2 = ens.run(7, 5, measure_every=3)    # after sweeps 15, 18; 19 plain
    assert P1.shape == (2, 2) and P2.shape == (2, 2)
    for i, (d, b) in enumerate(zip(dims, betas)):
        U = orc.hot(d, 5, lat_id=i)
        ref = {}
        for sw in range(19):
            orc.heatbath_sweep(d, U, b, 5, sw, lat_id=i)
            ref[sw + 1] = (orc.plaquette(d, U)[0], orc.polyakov(d, U))
        got = {5: (P1[i, 0], L1[i, 0]), 10: (P1[i, 1], L1[i, 1]), 15: (P2[i, 0], L2[i, 0]),
               18: (P2[i, 1], L2[i, 1])}
        for sw, (p, l) in got.items():
            assert abs(p - ref[sw][0]) < 1e-12 and abs(l - ref[sw][1]) < 1e-12, (i, sw)
        assert np.abs(ens.get_links(i) - U).max() < 1e-11
    P3, L3 = ens.run(2, 5, measure_every=3)        # fewer sweeps than one measurement
    assert P3.shape == (2, 0) and L3.shape == (2, 0)
    with pytest.raises(su2.SU2Error) as e:
        su2._chk(su2._lib.su2_ensemble_run(ens.h, 4, 0, 5, None, None), "measure_every 0")
    assert e.value.status == su2.EINVAL
    ens.close()


def _poison(lat, torch):
    """Write a NaN into the temporal link of site 0 in the native buffer (a
    torch tensor owned by the Python lattice): block (mu = 3, even) starts at
    link 6 V/2, 16 bytes per binary32 link.  Temporal links are updated last
    in a sweep, so the earlier substeps read the NaN in their staples."""
    torch.cuda.synchronize()
    off = 6 * (lat.volume // 2) * 16
    lat._buf[off:off + 16].view(torch.float32)[0] = float("nan")
    torch.cuda.synchronize()


@pytest.mark.parametrize("kind", ["heatbath", "overrelax"])
def test_nonfinite_link_reported_once(su2, kind):
    """A NaN link makes its neighbours' staples non-finite: the sweep that
    meets them returns ENUMERIC (the affected links are NaN, not redrawn), the
    error is cleared once reported, and a valid configuration then sweeps
    cleanly."""
    import torch
    dims = (4, 4, 4, 4)
    lat = su2.Lattice(dims, start=su2.HOT, seed=3, prec=su2.F32)
    _poison(lat, torch)
    with pytest.raises(su2.SU2Error) as e:
        lat.heatbath(2.3, 1, 3) if kind == "heatbath" else lat.overrelax(1)
    assert e.value.status == su2.ENUMERIC
    assert np.isnan(lat.get_links()).any()
    lat.set_links(inputs.random_config(dims, 61))
    lat.heatbath(2.3, 1, 3)                       # no stale error
    lat.overrelax(1)
    P = lat.plaquette()
    assert np.isfinite(P).all()
    lat.close()


def test_configuration_files(su2, orc, tmp_path):
    """A configuration written with numpy from the documented layout (magic,
    four int32 extents, 16 V float64 links) loads with su2_load as a binary64
    lattice holding exactly those links; su2_save_config writes the same
    bytes back; a checkpoint written by su2_save reads back with numpy."""
    dims = (4, 6, 2, 8)
    U = orc.hot(dims, 17)
    p = tmp_path / "conf.su2"
    p.write_bytes(b"SU2CONF1" + np.asarray(dims, "<i4").tobytes() + U.astype("<f8").tobytes())
    h = su2.su2_load(str(p))
    assert su2.su2_get_dims(h) == dims and su2.su2_get_sweep(h) == 0
    G = su2.su2_get_links(h)
    assert np.array_equal(G, U)
    assert abs(su2.su2_plaquette(h)[0] - orc.plaquette(dims, U)[0]) < 1e-13
    q = tmp_path / "again.su2"
    su2.su2_save_config(h, str(q))
    assert q.read_bytes() == p.read_bytes()
    su2.su2_heatbath(h, 2.4, 3, 5)
    c = tmp_path / "ck.su2"
    su2.su2_save(h, str(c))
    raw = c.read_bytes()
    magic, (version, nx, ny, nz, nt, prec, sweep, seed) = raw[:8], struct.unpack("<I5iIQ", raw[8:44])
    assert magic == b"SU2CKPT1" and version == 1 and (nx, ny, nz, nt) == dims
    assert prec == su2.F64 and sweep == 3 and seed == 5
    links = np.frombuffer(raw[44:], "<f8").reshape(-1, 4, 4)
    assert np.array_equal(links, su2.su2_get_links(h))
    U2 = U.copy()
    for sw in range(3):
        orc.heatbath_sweep(dims, U2, 2.4, 5, sw)
    assert np.abs(links - U2).max() < 1e-12
    su2.su2_destroy(h)
    # a configuration with a non-unit link is refused
    bad = U.copy()
    bad[3, 1] *= 1.01
    p.write_bytes(b"SU2CONF1" + np.asarray(dims, "<i4").tobytes() + bad.astype("<f8").tobytes())
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_load(str(p))
    assert e.value.status == su2.EIO


@pytest.mark.parametrize("prec", ["F32", "F64"])
def test_maximum_volume_top_of_the_offset_range(su2, orc, prec):
    """A lattice at the volume cap (2^29 sites in binary32, 2^28 in
    binary64: 32 GiB of links either way), where a link's byte offset inside
    its (mu, parity) block reaches 2^32 - 16.  From a cold start every
    staple is exactly 6 x 1, so after one substep of the last block in
    memory (mu = 3, odd sites) each link is the normalised draw of the
    oracle's single-link sampler with alpha = 6 beta and that link's
    counter.  Sampled links (the first, the last 24, 32 random) are read
    from device memory and compared; the other blocks stay cold."""
    import torch
    P = getattr(su2, prec)
    dims = (64, 128, 128, 512) if prec == "F32" else (64, 128, 128, 256)
    V = int(np.prod(dims))
    vh = V // 2
    assert V == (1 << 29 if prec == "F32" else 1 << 28)
    beta, seed, mu, par = 2.3, 17, 3, 1
    print(f"maximum volume {prec}: dims {dims}, {su2.su2_link_bytes(*dims, P) >> 30} GiB of links", flush=True)
    lat = su2.Lattice(dims, start=su2.COLD, prec=P)
    try:
        lat.substep(beta, seed, mu, par)
        torch.cuda.synchronize()
        rng = np.random.default_rng(5)
        cbs = np.unique(np.concatenate([[0, 1, 2, 3], np.arange(vh - 24, vh), rng.integers(0, vh, 32)]))
        blk = 2 * mu + par
        if prec == "F32":
            f = lat._buf.view(torch.float32)
            idx = torch.as_tensor((blk * vh + cbs)[:, None] * 4 + np.arange(4), device="cuda")
            got = f[idx].double().cpu().numpy()
            # a0 of the first link of block (0, even) and of the last link of block (0, odd)
            cold = f[torch.as_tensor(np.array([0, 4 * (2 * vh - 1)]), device="cuda")].cpu().numpy()
        else:
            f = lat._buf.view(torch.float64)
            base = blk * vh * 4
            lo = base + 2 * cbs[:, None] + np.arange(2)
            hi = base + 2 * vh + 2 * cbs[:, None] + np.arange(2)
            idx = torch.as_tensor(np.concatenate([lo, hi], axis=1), device="cuda")
            got = f[idx].cpu().numpy()
            # a0 (low plane) of the first link of block (0, even) and of the last link of block (0, odd)
            cold = f[torch.as_tensor(np.array([0, 4 * vh + 2 * (vh - 1)]), device="cuda")].cpu().numpy()
        assert np.all(cold == 1.0), cold
        tag = (0 << 8) | (0 << 4) | (mu << 1) | par       # lattice 0, heat bath, (mu, parity)
        nx = dims[0]
        err = []
        for k, cb in enumerate(cbs):
            row = (2 * int(cb)) // nx
            y, z, t = row % dims[1], (row // dims[1]) % dims[2], row // (dims[1] * dims[2])
            s = 2 * int(cb) + ((par + y + z + t) & 1)
            X, _ = orc.sample_link(6.0 * beta, orc.HYBRID, seed, [s, 0, tag], ubits=23 if prec == "F32" else 32)
            err.append(float(np.abs(got[k] - X / np.linalg.norm(X)).max()))
        err = np.array(err)
        tol = 1e-5 if prec == "F32" else 1e-12
        top = int(cbs.max()) * 16 + (0 if prec == "F32" else vh * 16)   # binary64: the high plane's offset
        print(f"  {len(cbs)} sampled links up to cb {int(cbs.max())} (lane byte offset {top}): "
              f"max |dU| {err.max():.2e}, {int((err > tol).sum())} beyond {tol:g}", flush=True)
        assert (err > tol).sum() <= (1 if prec == "F32" else 0), err
        # unit links, and no link of the updated block left cold
        assert np.all(np.abs(np.linalg.norm(got, axis=1) - 1) < 1e-6) and np.all(got[:, 0] < 1.0)
    finally:
        lat.close()
        del lat
        torch.cuda.empty_cache()


def test_zero_sweeps_change_nothing(su2):
    """Empty work: zero heat-bath or over-relaxation sweeps and an ensemble
    run of zero sweeps leave links, sweep counter and try counts as they
    were, and return empty series."""
    lat = su2.Lattice((4, 4, 4, 6), start=su2.HOT, seed=3, prec=su2.F32)
    U = lat.get_links()
    lat.heatbath(2.3, 0, 3)
    lat.overrelax(0)
    assert lat.sweep == 0 and np.array_equal(lat.get_links(), U)
    lat.close()
    ens = su2.Ensemble([(4, 4, 4, 4), (6, 4, 4, 2)], [2.0, 2.4], start=su2.HOT, seed=4, prec=su2.F64)
    links = [ens.get_links(i) for i in range(2)]
    P, L = ens.run(0, 4)
    assert P.shape == (2, 0) and L.shape == (2, 0)
    P, L = ens.run(3, 4, measure_every=5)          # fewer sweeps than one measurement unit
    assert P.shape == (2, 0) and L.shape == (2, 0)
    assert not np.array_equal(ens.get_links(0), links[0])   # the three sweeps did run
    ens.close()

