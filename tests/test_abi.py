"""Host-side checks of the C ABI (no GPU needed): every entry point declared
in include/su2.h is exported by libsu2.so and bound in Python; argument
validation and the no-device path."""
import os
import re
import subprocess

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "su2.h")).read()
    return set(re.findall(r"^(?:su2_status|size_t|const char \*)\s*(su2_\w+)\(", text, re.M))


def test_header_symbols_exported():
    from paper_1010_4834_amd import su2
    names = declared()
    assert len(names) >= 40
    out = subprocess.run(["nm", "-D", "--defined-only", su2.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (su2_\w+)$", out, re.M))
    assert names <= exported, names - exported
    assert names == set(su2.EXPORTED), names ^ set(su2.EXPORTED)


def test_host_validation():
    from paper_1010_4834_amd import su2
    assert su2.su2_link_bytes(8, 8, 8, 8, su2.F32) == 4 * 8**4 * 16
    assert su2.su2_link_bytes(8, 8, 8, 8, su2.F64) == 4 * 8**4 * 32
    for bad in ((7, 8, 8, 8), (8, 8, 8, 0), (8, 1, 8, 8), (2, 256, 256, 256), (1 << 24, 2, 2, 2)):
        assert su2.su2_link_bytes(*bad, su2.F32) == 0
        with pytest.raises(su2.SU2Error) as e:
            su2.su2_create(*bad, su2.COLD, 1, su2.F32)
        assert e.value.status == su2.EINVAL
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_create(8, 8, 8, 8, 5, 1, su2.F32)
    assert e.value.status == su2.EINVAL
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_ensemble_create([(8, 8, 8, 8)], [-1.0], su2.HOT, 1, su2.F32)
    assert e.value.status == su2.EINVAL
    with pytest.raises(su2.SU2Error) as e:           # an empty ensemble
        su2.su2_ensemble_create(np.zeros((0, 4), dtype=np.int32), [], su2.HOT, 1, su2.F32)
    assert e.value.status == su2.EINVAL
    assert su2._lib.su2_status_str(-7).decode().startswith("non-finite")


def test_volume_cap_per_precision():
    """Link offsets inside a (mu, parity) block are 32-bit byte offsets, so a
    lattice holds at most 2^29 sites in binary32 and 2^28 in binary64; larger
    extents are refused before anything is allocated."""
    from paper_1010_4834_amd import su2
    V29 = (64, 128, 128, 512)          # 2^29 sites
    assert su2.su2_link_bytes(*V29, su2.F32) == 4 * (1 << 29) * 16
    assert su2.su2_link_bytes(*V29, su2.F64) == 0
    assert su2.su2_link_bytes(64, 128, 128, 256, su2.F64) == 4 * (1 << 28) * 32
    assert su2.su2_link_bytes(128, 128, 128, 512, su2.F32) == 0   # 2^30 sites
    for dims, prec in ((V29, su2.F64), ((128, 128, 128, 512), su2.F32)):
        with pytest.raises(su2.SU2Error) as e:
            su2.su2_create(*dims, su2.COLD, 1, prec)
        assert e.value.status == su2.EINVAL
        with pytest.raises(su2.SU2Error) as e:
            su2.su2_ensemble_create([dims], [2.0], su2.HOT, 1, prec)
        assert e.value.status == su2.EINVAL


def test_noalloc_argument_checks():
    """The allocation-free heat bath refuses bad arguments and lattices beyond
    its fixed scratch (2^27 sites) before any device call."""
    from paper_1010_4834_amd import su2
    fake = 1 << 20        # never dereferenced: every case fails validation first
    for args in (((256, 256, 256, 16), su2.F32, 2.3, 1),     # 2^28 sites
                 ((8, 8, 8, 7), su2.F32, 2.3, 1), ((8, 8, 8, 8), 5, 2.3, 1),
                 ((8, 8, 8, 8), su2.F32, -1.0, 1), ((8, 8, 8, 8), su2.F32, 2.3, -1)):
        with pytest.raises(su2.SU2Error) as e:
            su2.su2_heatbath_noalloc(fake, *args, 1)
        assert e.value.status == su2.EINVAL, args
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_heatbath_noalloc(None, (8, 8, 8, 8), su2.F32, 2.3, 1, 1)
    assert e.value.status == su2.EINVAL


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-GPU path")
def test_no_device():
    from paper_1010_4834_amd import su2
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_create(8, 8, 8, 8, su2.COLD, 1, su2.F32)
    assert e.value.status == su2.ENODEV


def test_single_hip_runtime():
    """Importing the binding before torch still leaves one HIP runtime in the
    process (torch's): two runtimes cannot share devices or pointers."""
    import sys
    code = ("from paper_1010_4834_amd import su2\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"


def test_host_arrays_are_sized_by_the_binding():
    """The library reads and writes whole lattices through bare pointers, so
    the binding refuses a host array of any other size, and a null handle is
    EINVAL for the extent queries (no GPU needed)."""
    from paper_1010_4834_amd import su2
    assert su2._f64(np.zeros((2, 4, 4)), 32, "t").dtype == np.float64
    for bad in (np.zeros((2, 4, 4)), np.zeros(31)):
        with pytest.raises(ValueError):
            su2._f64(bad, 16 * 3, "t")
    with pytest.raises(ValueError):
        su2.su2_ensemble_create([(4, 4, 4, 4), (4, 4, 4, 6)], [2.0], su2.HOT, 1, su2.F32)
    for call in (lambda: su2.su2_get_dims(None), lambda: su2.su2_ensemble_count(None),
                 lambda: su2.su2_ensemble_get_dims(None, 0)):
        with pytest.raises(su2.SU2Error) as e:
            call()
        assert e.value.status == su2.EINVAL


def _checkpoint(path, dims, prec, payload, magic=b"SU2CKPT1", version=1):
    import struct
    with open(path, "wb") as f:
        f.write(magic + struct.pack("<I5iIQ", version, *dims, prec, 0, 1) + payload)


def test_load_refuses_malformed_checkpoints(tmp_path):
    """su2_load checks the header and that the payload is exactly 16 V
    float64 before it allocates or reads it; all of this runs before any GPU
    call, so it is tested here."""
    from paper_1010_4834_amd import su2
    cold = np.tile(np.array([1.0, 0.0, 0.0, 0.0]), 256 * 4).tobytes()   # 4^4 sites, 4 links each
    cases = {
        "missing": None,
        "magic": (b"SU2CKPT0", 1, (4, 4, 4, 4), su2.F32, cold),
        "version": (b"SU2CKPT1", 2, (4, 4, 4, 4), su2.F32, cold),
        "odd extent": (b"SU2CKPT1", 1, (4, 4, 5, 4), su2.F32, cold),
        "precision": (b"SU2CKPT1", 1, (4, 4, 4, 4), 7, cold),
        "short payload": (b"SU2CKPT1", 1, (4, 4, 4, 4), su2.F32, cold[:-8]),
        "trailing bytes": (b"SU2CKPT1", 1, (4, 4, 4, 4), su2.F32, cold + b"\0"),
        # 2^30 sites announce a 128 GiB payload that the file does not hold
        "huge header": (b"SU2CKPT1", 1, (1024, 1024, 512, 2), su2.F32, b""),
    }
    for name, c in cases.items():
        p = tmp_path / name.replace(" ", "_")
        if c is not None:
            magic, version, dims, prec, payload = c
            _checkpoint(p, dims, prec, payload, magic, version)
        with pytest.raises(su2.SU2Error) as e:
            su2.su2_load(str(p))
        assert e.value.status == su2.EIO, name
    # the well-formed file passes every check; without a GPU the lattice
    # cannot be created
    p = tmp_path / "good"
    _checkpoint(p, (4, 4, 4, 4), su2.F32, cold)
    try:
        h = su2.su2_load(str(p))
    except su2.SU2Error as e:
        assert e.status == su2.ENODEV and not torch.cuda.is_available()
    else:
        su2.su2_destroy(h)
