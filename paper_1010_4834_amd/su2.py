"""Python binding of the gfx950 SU(2) library (libsu2.so, C ABI in include/su2.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI.  Functions keep the C names (su2_create,
su2_heatbath, ...) and raise SU2Error on a non-zero status.  PyTorch supplies
device memory (the link buffer can be a torch tensor) and streams.

There is no fallback: if libsu2.so is missing, importing this module raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsu2.so")

OK, EINVAL, ENOMEM, ENODEV, EDEVICE, ESTATE, EIO, ENUMERIC = 0, -1, -2, -3, -4, -5, -6, -7
COLD, HOT = 0, 1
F64, F32 = 0, 1
HYBRID, CREUTZ = 0, 1
K_HEATBATH, K_OVERRELAX, K_PLAQUETTE, K_POLYAKOV, K_REDUCE, K_APE, K_WILSON = range(7)
KERNEL_KINDS = 7


class SU2Error(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {_lib.su2_status_str(status).decode()} ({status})")


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(python -c 'import __graft_entry__ as g; g.build()')")

# torch ships its own HIP runtime under the same SONAME as the system one
# libsu2.so is linked against.  Loading torch first makes libsu2.so bind to
# that runtime, so the process holds a single HIP runtime whatever the
# caller imports first (with two, the second one sees no device and device
# pointers could not be shared with torch tensors).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)
_P, _I, _D = C.c_void_p, C.c_int, C.c_double
_U64, _U32, _SZ, _I64 = C.c_uint64, C.c_uint32, C.c_size_t, C.c_int64
_PP = C.POINTER(C.c_void_p)

_SIGS = {
    "su2_status_str": (C.c_char_p, [_I]),
    "su2_link_bytes": (_SZ, [_I, _I, _I, _I, _I]),
    "su2_create": (_I, [_I, _I, _I, _I, _I, _U64, _I, _P, _SZ, _PP]),
    "su2_destroy": (_I, [_P]),
    "su2_set_stream": (_I, [_P, _P]),
    "su2_set_sampler": (_I, [_P, _I]),
    "su2_heatbath": (_I, [_P, _D, _I, _U64]),
    "su2_heatbath_substep": (_I, [_P, _D, _U64, _I, _I]),
    "su2_overrelax": (_I, [_P, _I]),
    "su2_plaquette": (_I, [_P, _P, _P, _P]),
    "su2_polyakov": (_I, [_P, _P]),
    "su2_ape_smear": (_I, [_P, _D, _I]),
    "su2_wilson_loops": (_I, [_P, _I, _I, _P]),
    "su2_release_buffers": (_I, [_P]),
    "su2_get_links": (_I, [_P, _P]),
    "su2_set_links": (_I, [_P, _P]),
    "su2_get_smeared": (_I, [_P, _P]),
    "su2_device_links": (_I, [_P, _PP, _P]),
    "su2_get_dims": (_I, [_P, _P]),
    "su2_get_sweep": (_I, [_P, _P]),
    "su2_set_sweep": (_I, [_P, _U32]),
    "su2_stats": (_I, [_P, _P, _P, _P]),
    "su2_trace_tries": (_I, [_P, _I]),
    "su2_get_tries": (_I, [_P, _P]),
    "su2_save": (_I, [_P, C.c_char_p]),
    "su2_save_config": (_I, [_P, C.c_char_p]),
    "su2_load": (_I, [C.c_char_p, _PP]),
    "su2_set_launch": (_I, [_P, _I, _I, _I, _I]),
    "su2_get_launch": (_I, [_P, _P, _P, _P, _P]),
    "su2_autotune": (_I, [_P, _D]),
    "su2_set_timing": (_I, [_P, _I]),
    "su2_get_timing": (_I, [_P, _I, _P, _P]),
    "su2_heatbath_noalloc": (_I, [_P, _I, _I, _I, _I, _I, _D, _I, _U64, _U32, _P, _P]),
    "su2_ensemble_create": (_I, [_I, _P, _P, _I, _U64, _I, _P, _SZ, _PP]),
    "su2_ensemble_destroy": (_I, [_P]),
    "su2_ensemble_set_stream": (_I, [_P, _P]),
    "su2_ensemble_set_sampler": (_I, [_P, _I]),
    "su2_ensemble_run": (_I, [_P, _I, _I, _U64, _P, _P]),
    "su2_ensemble_count": (_I, [_P, _P]),
    "su2_ensemble_get_dims": (_I, [_P, _I, _P]),
    "su2_ensemble_get_links": (_I, [_P, _I, _P]),
    "su2_ensemble_set_links": (_I, [_P, _I, _P]),
    "su2_ensemble_stats": (_I, [_P, _P, _P]),
    "su2_ensemble_trace_tries": (_I, [_P, _I]),
    "su2_ensemble_get_tries": (_I, [_P, _I, _P]),
    "su2_ensemble_set_launch": (_I, [_P, _I, _I, _I, _I]),
    "su2_ensemble_get_launch": (_I, [_P, _P, _P, _P, _P]),
    "su2_ensemble_autotune": (_I, [_P]),
    "su2_ensemble_set_timing": (_I, [_P, _I]),
    "su2_ensemble_get_timing": (_I, [_P, _I, _P, _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


def _chk(status, where):
    if status != OK:
        raise SU2Error(status, where)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, n, where):
    """A C-contiguous float64 copy or view of exactly n values: the library
    reads n values from the pointer, so any other size is refused here."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != n:
        raise ValueError(f"{where}: {a.size} values given, the lattice needs {n}")
    return a


def _sites(h, volume, where, i=None):
    """Site count of the handle's lattice (lattice i of an ensemble), from the
    library; a caller-supplied volume must agree with it."""
    d = su2_get_dims(h) if i is None else su2_ensemble_get_dims(h, i)
    V = d[0] * d[1] * d[2] * d[3]
    if volume is not None and int(volume) != V:
        raise ValueError(f"{where}: volume {volume} given, the lattice has {V} sites")
    return V


# ---- C names -----------------------------------------------------------------
def su2_link_bytes(nx, ny, nz, nt, prec):
    return _lib.su2_link_bytes(nx, ny, nz, nt, prec)


def su2_create(nx, ny, nz, nt, start, seed, prec, device_links=None, device_bytes=0):
    h = C.c_void_p()
    _chk(_lib.su2_create(nx, ny, nz, nt, start, seed, prec, device_links, device_bytes,
                         C.byref(h)), "su2_create")
    return h


def su2_destroy(h):
    _chk(_lib.su2_destroy(h), "su2_destroy")


def su2_set_stream(h, stream):
    _chk(_lib.su2_set_stream(h, stream), "su2_set_stream")


def su2_set_sampler(h, sampler):
    _chk(_lib.su2_set_sampler(h, sampler), "su2_set_sampler")


def su2_heatbath(h, beta, nsweeps, seed):
    _chk(_lib.su2_heatbath(h, beta, nsweeps, seed), "su2_heatbath")


def su2_heatbath_substep(h, beta, seed, mu, parity):
    _chk(_lib.su2_heatbath_substep(h, beta, seed, mu, parity), "su2_heatbath_substep")


def su2_overrelax(h, nsweeps):
    _chk(_lib.su2_overrelax(h, nsweeps), "su2_overrelax")


def su2_plaquette(h):
    r = np.zeros(3)
    _chk(_lib.su2_plaquette(h, _ptr(r[0:]), _ptr(r[1:]), _ptr(r[2:])), "su2_plaquette")
    return float(r[0]), float(r[1]), float(r[2])


def su2_polyakov(h):
    r = np.zeros(1)
    _chk(_lib.su2_polyakov(h, _ptr(r)), "su2_polyakov")
    return float(r[0])


def su2_ape_smear(h, alpha, nsteps):
    _chk(_lib.su2_ape_smear(h, alpha, nsteps), "su2_ape_smear")


def su2_wilson_loops(h, rmax, tmax):
    out = np.zeros((rmax, tmax))
    _chk(_lib.su2_wilson_loops(h, rmax, tmax, _ptr(out)), "su2_wilson_loops")
    return out


def su2_release_buffers(h):
    _chk(_lib.su2_release_buffers(h), "su2_release_buffers")


def su2_get_links(h, volume=None):
    out = np.zeros((_sites(h, volume, "su2_get_links"), 4, 4))
    _chk(_lib.su2_get_links(h, _ptr(out)), "su2_get_links")
    return out


def su2_set_links(h, links):
    a = _f64(links, 16 * _sites(h, None, "su2_set_links"), "su2_set_links")
    _chk(_lib.su2_set_links(h, _ptr(a)), "su2_set_links")


def su2_get_smeared(h, volume=None):
    out = np.zeros((_sites(h, volume, "su2_get_smeared"), 3, 4))
    _chk(_lib.su2_get_smeared(h, _ptr(out)), "su2_get_smeared")
    return out


def su2_device_links(h):
    p, n = C.c_void_p(), C.c_size_t()
    _chk(_lib.su2_device_links(h, C.byref(p), C.byref(n)), "su2_device_links")
    return p.value, n.value


def su2_get_dims(h):
    d = np.zeros(4, dtype=np.int32)
    _chk(_lib.su2_get_dims(h, _ptr(d)), "su2_get_dims")
    return tuple(int(x) for x in d)


def su2_get_sweep(h):
    v = C.c_uint32()
    _chk(_lib.su2_get_sweep(h, C.byref(v)), "su2_get_sweep")
    return v.value


def su2_set_sweep(h, sweep):
    _chk(_lib.su2_set_sweep(h, sweep), "su2_set_sweep")


def su2_stats(h):
    t, u, d = C.c_uint64(), C.c_uint64(), C.c_double()
    _chk(_lib.su2_stats(h, C.byref(t), C.byref(u), C.byref(d)), "su2_stats")
    return t.value, u.value, d.value


def su2_trace_tries(h, enable):
    _chk(_lib.su2_trace_tries(h, int(enable)), "su2_trace_tries")


def su2_get_tries(h, volume=None):
    out = np.zeros(_sites(h, volume, "su2_get_tries") * 4, dtype=np.uint32)
    _chk(_lib.su2_get_tries(h, _ptr(out)), "su2_get_tries")
    return out


def su2_save(h, path):
    _chk(_lib.su2_save(h, os.fsencode(path)), "su2_save")


def su2_save_config(h, path):
    _chk(_lib.su2_save_config(h, os.fsencode(path)), "su2_save_config")


def su2_load(path):
    h = C.c_void_p()
    _chk(_lib.su2_load(os.fsencode(path), C.byref(h)), "su2_load")
    return h


def su2_set_launch(h, block, grid, remap, links_per_lane=1):
    _chk(_lib.su2_set_launch(h, block, grid, remap, links_per_lane), "su2_set_launch")


def su2_get_launch(h):
    v = [C.c_int() for _ in range(4)]
    _chk(_lib.su2_get_launch(h, *[C.byref(x) for x in v]), "su2_get_launch")
    return tuple(x.value for x in v)


def su2_autotune(h, beta):
    _chk(_lib.su2_autotune(h, beta), "su2_autotune")


def su2_set_timing(h, enable):
    _chk(_lib.su2_set_timing(h, int(enable)), "su2_set_timing")


def su2_get_timing(h, kind):
    ms, n = C.c_double(), C.c_int64()
    _chk(_lib.su2_get_timing(h, kind, C.byref(ms), C.byref(n)), "su2_get_timing")
    return ms.value, n.value


def su2_heatbath_noalloc(device_links, dims, prec, beta, nsweeps, seed, sweep=0, device_err=None, stream=None):
    """Heat-bath sweeps of a caller-owned native link buffer (device pointer)
    that allocate nothing and do not synchronise."""
    nx, ny, nz, nt = (int(d) for d in dims)
    _chk(_lib.su2_heatbath_noalloc(device_links, nx, ny, nz, nt, prec, beta, nsweeps, seed, sweep,
                                   device_err, stream), "su2_heatbath_noalloc")


def su2_ensemble_create(dims, betas, start, seed, prec, device_links=None, device_bytes=0):
    d = np.ascontiguousarray(dims, dtype=np.int32).reshape(-1, 4)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    if b.size != d.shape[0]:
        raise ValueError(f"su2_ensemble_create: {d.shape[0]} lattices but {b.size} couplings")
    h = C.c_void_p()
    _chk(_lib.su2_ensemble_create(d.shape[0], _ptr(d), _ptr(b), start, seed, prec, device_links,
                                  device_bytes, C.byref(h)), "su2_ensemble_create")
    return h


def su2_ensemble_destroy(h):
    _chk(_lib.su2_ensemble_destroy(h), "su2_ensemble_destroy")


def su2_ensemble_set_stream(h, stream):
    _chk(_lib.su2_ensemble_set_stream(h, stream), "su2_ensemble_set_stream")


def su2_ensemble_set_sampler(h, sampler):
    _chk(_lib.su2_ensemble_set_sampler(h, sampler), "su2_ensemble_set_sampler")


def su2_ensemble_count(h):
    n = C.c_int()
    _chk(_lib.su2_ensemble_count(h, C.byref(n)), "su2_ensemble_count")
    return n.value


def su2_ensemble_get_dims(h, i):
    d = np.zeros(4, dtype=np.int32)
    _chk(_lib.su2_ensemble_get_dims(h, i, _ptr(d)), "su2_ensemble_get_dims")
    return tuple(int(x) for x in d)


def su2_ensemble_run(h, n, nsweeps, seed, plaq=True, poly=True, measure_every=1):
    # the library writes count * (nsweeps // measure_every) values per series
    if n is None:
        n = su2_ensemble_count(h)
    elif int(n) != su2_ensemble_count(h):
        raise ValueError(f"su2_ensemble_run: n = {n} given, the ensemble has {su2_ensemble_count(h)} lattices")
    if nsweeps < 0 or measure_every < 1:
        raise ValueError("su2_ensemble_run: nsweeps < 0 or measure_every < 1")
    m = nsweeps // measure_every
    P = np.zeros((n, m)) if plaq else None
    L = np.zeros((n, m)) if poly else None
    _chk(_lib.su2_ensemble_run(h, nsweeps, measure_every, seed, _ptr(P) if plaq else None,
                               _ptr(L) if poly else None), "su2_ensemble_run")
    return P, L


def su2_ensemble_get_links(h, i, volume=None):
    out = np.zeros((_sites(h, volume, "su2_ensemble_get_links", i), 4, 4))
    _chk(_lib.su2_ensemble_get_links(h, i, _ptr(out)), "su2_ensemble_get_links")
    return out


def su2_ensemble_set_links(h, i, links):
    a = _f64(links, 16 * _sites(h, None, "su2_ensemble_set_links", i), "su2_ensemble_set_links")
    _chk(_lib.su2_ensemble_set_links(h, i, _ptr(a)), "su2_ensemble_set_links")


def su2_ensemble_stats(h):
    t, u = C.c_uint64(), C.c_uint64()
    _chk(_lib.su2_ensemble_stats(h, C.byref(t), C.byref(u)), "su2_ensemble_stats")
    return t.value, u.value


def su2_ensemble_trace_tries(h, enable):
    _chk(_lib.su2_ensemble_trace_tries(h, int(enable)), "su2_ensemble_trace_tries")


def su2_ensemble_get_tries(h, i, volume=None):
    out = np.zeros(_sites(h, volume, "su2_ensemble_get_tries", i) * 4, dtype=np.uint32)
    _chk(_lib.su2_ensemble_get_tries(h, i, _ptr(out)), "su2_ensemble_get_tries")
    return out


def su2_ensemble_set_launch(h, block, grid, remap, links_per_lane=1):
    _chk(_lib.su2_ensemble_set_launch(h, block, grid, remap, links_per_lane), "su2_ensemble_set_launch")


def su2_ensemble_get_launch(h):
    v = [C.c_int() for _ in range(4)]
    _chk(_lib.su2_ensemble_get_launch(h, *[C.byref(x) for x in v]), "su2_ensemble_get_launch")
    return tuple(x.value for x in v)


def su2_ensemble_autotune(h):
    _chk(_lib.su2_ensemble_autotune(h), "su2_ensemble_autotune")


def su2_ensemble_set_timing(h, enable):
    _chk(_lib.su2_ensemble_set_timing(h, int(enable)), "su2_ensemble_set_timing")


def su2_ensemble_get_timing(h, kind):
    ms, n = C.c_double(), C.c_int64()
    _chk(_lib.su2_ensemble_get_timing(h, kind, C.byref(ms), C.byref(n)), "su2_ensemble_get_timing")
    return ms.value, n.value


# ---- convenience wrappers ----------------------------------------------------------
def _torch_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Lattice:
    """One lattice; the link buffer is a torch uint8 tensor on the current
    device when torch_buffer is set (torch's allocator owns it)."""

    def __init__(self, dims, start=HOT, seed=1, prec=F32, torch_buffer=True, stream=None):
        self.dims = tuple(int(d) for d in dims)
        self.volume = int(np.prod(self.dims))
        self.prec = prec
        self._buf = None
        ptr, nbytes = None, 0
        if torch_buffer:
            import torch
            nbytes = su2_link_bytes(*self.dims, prec)
            if nbytes == 0:
                raise SU2Error(EINVAL, "Lattice")
            self._buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            ptr = self._buf.data_ptr()
        self.h = su2_create(*self.dims, start, seed, prec, ptr, nbytes)
        if stream is not None:
            su2_set_stream(self.h, stream)

    def close(self):
        if self.h:
            su2_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def heatbath(self, beta, nsweeps, seed):
        su2_heatbath(self.h, beta, nsweeps, seed)

    def substep(self, beta, seed, mu, parity):
        su2_heatbath_substep(self.h, beta, seed, mu, parity)

    def overrelax(self, nsweeps):
        su2_overrelax(self.h, nsweeps)

    def plaquette(self):
        return su2_plaquette(self.h)

    def polyakov(self):
        return su2_polyakov(self.h)

    def ape_smear(self, alpha, nsteps):
        su2_ape_smear(self.h, alpha, nsteps)

    def wilson_loops(self, rmax, tmax):
        return su2_wilson_loops(self.h, rmax, tmax)

    def get_links(self):
        return su2_get_links(self.h, self.volume)

    def set_links(self, links):
        su2_set_links(self.h, links)

    def get_smeared(self):
        return su2_get_smeared(self.h, self.volume)

    @property
    def sweep(self):
        return su2_get_sweep(self.h)

    @sweep.setter
    def sweep(self, v):
        su2_set_sweep(self.h, v)

    def stats(self):
        return su2_stats(self.h)

    def trace_tries(self, enable=True):
        su2_trace_tries(self.h, enable)

    def get_tries(self):
        return su2_get_tries(self.h, self.volume)


class Ensemble:
    """Independent lattices advanced by the same kernel launches."""

    def __init__(self, dims, betas, start=HOT, seed=1, prec=F32, stream=None):
        self.dims = [tuple(int(x) for x in d) for d in dims]
        self.n = len(self.dims)
        self.h = su2_ensemble_create(self.dims, betas, start, seed, prec)
        if stream is not None:
            su2_ensemble_set_stream(self.h, stream)

    def close(self):
        if self.h:
            su2_ensemble_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, nsweeps, seed, plaq=True, poly=True, measure_every=1):
        return su2_ensemble_run(self.h, self.n, nsweeps, seed, plaq, poly, measure_every)

    def trace_tries(self, enable=True):
        su2_ensemble_trace_tries(self.h, enable)

    def get_tries(self, i):
        return su2_ensemble_get_tries(self.h, i, int(np.prod(self.dims[i])))

    def get_links(self, i):
        return su2_ensemble_get_links(self.h, i, int(np.prod(self.dims[i])))

    def set_links(self, i, links):
        su2_ensemble_set_links(self.h, i, links)

    def stats(self):
        return su2_ensemble_stats(self.h)
