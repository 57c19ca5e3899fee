"""ctypes wrapper of the serial FP64 oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg to check the GPU library.  It shares no code with the GPU
path.  Arrays use the canonical layout U[s, mu, c] with
s = x + Nx*(y + Ny*(z + Nz*t)), c = (a0, a1, a2, a3).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

HYBRID, CREUTZ, KP = 0, 1, 2
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        I64, U64, U32, D = C.c_int64, C.c_uint64, C.c_uint32, C.c_double
        sig = {
            "or_philox4x32_10": (None, [P, P, P]),
            "or_uniform": (D, [U32, C.c_int]),
            "or_qmul": (None, [P, P, P]),
            "or_check_dims": (C.c_int, [P]),
            "or_volume": (I64, [P]),
            "or_parity": (C.c_int, [P, I64]),
            "or_neighbor": (I64, [P, I64, C.c_int, C.c_int]),
            "or_cold": (None, [P, P]),
            "or_hot": (None, [P, P, U64, U32]),
            "or_staple": (None, [P, P, I64, C.c_int, P]),
            "or_sample_delta": (U32, [D, C.c_int, U64, P, C.c_int, P, P]),
            "or_sample_link": (U32, [D, C.c_int, U64, P, C.c_int, P, P]),
            "or_sample_many": (None, [D, C.c_int, U64, I64, C.c_int, P, P]),
            "or_heatbath_link": (U32, [P, P, I64, C.c_int, D, U64, U32, U32, C.c_int, C.c_int]),
            "or_heatbath_substep": (U64, [P, P, D, U64, U32, U32, C.c_int, C.c_int,
                                          C.c_int, C.c_int, P, P]),
            "or_heatbath_sweep": (U64, [P, P, D, U64, U32, U32, C.c_int, C.c_int, P, P]),
            "or_overrelax_sweep": (None, [P, P]),
            "or_plaquette": (None, [P, P, P, P, P]),
            "or_polyakov": (D, [P, P]),
            "or_ape": (None, [P, P, D, C.c_int, P]),
            "or_wilson": (None, [P, P, P, C.c_int, C.c_int, P]),
            "or_wilson_rt": (D, [P, P, P, C.c_int, C.c_int]),
            "or_gauge_transform": (None, [P, P, U64]),
            "or_max_unit_defect": (D, [P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _dims(n):
    return np.ascontiguousarray(n, dtype=np.int32)


def _links(U):
    assert U.dtype == np.float64 and U.flags.c_contiguous
    return U


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def uniform(w, bits=32):
    return lib().or_uniform(int(w), int(bits))


def qmul(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.zeros(4)
    lib().or_qmul(_p(a), _p(b), _p(c))
    return c


def check_dims(n):
    return lib().or_check_dims(_p(_dims(n)))


def volume(n):
    return int(np.prod(n))


def neighbor(n, s, mu, step):
    return lib().or_neighbor(_p(_dims(n)), int(s), int(mu), int(step))


def parity(n, s):
    return lib().or_parity(_p(_dims(n)), int(s))


def cold(n):
    U = np.zeros((volume(n), 4, 4))
    lib().or_cold(_p(_dims(n)), _p(U))
    return U


def hot(n, seed, lat_id=0):
    U = np.zeros((volume(n), 4, 4))
    lib().or_hot(_p(_dims(n)), _p(U), int(seed), int(lat_id))
    return U


def staple(n, U, s, mu):
    V = np.zeros(4)
    lib().or_staple(_p(_dims(n)), _p(_links(U)), int(s), int(mu), _p(V))
    return V


def sample_delta(alpha, sampler, seed, ctr3, ubits=32):
    c = np.ascontiguousarray(ctr3, dtype=np.uint32)
    d = np.zeros(1)
    cr = np.zeros(1, dtype=np.int32)
    tries = lib().or_sample_delta(float(alpha), int(sampler), int(seed), _p(c),
                                  int(ubits), _p(d), _p(cr))
    return float(d[0]), int(tries), bool(cr[0])


def sample_link(alpha, sampler, seed, ctr3, ubits=32):
    c = np.ascontiguousarray(ctr3, dtype=np.uint32)
    X = np.zeros(4)
    tries = lib().or_sample_link(float(alpha), int(sampler), int(seed), _p(c), int(ubits),
                                 _p(X), None)
    return X, int(tries)


def sample_many(alpha, sampler, seed, nsamp, ubits=32):
    d = np.zeros(nsamp)
    t = np.zeros(nsamp, dtype=np.uint32)
    lib().or_sample_many(float(alpha), int(sampler), int(seed), int(nsamp), int(ubits),
                         _p(d), _p(t))
    return d, t


def heatbath_link(n, U, s, mu, beta, seed, sweep, lat_id=0, sampler=HYBRID, ubits=32):
    return lib().or_heatbath_link(_p(_dims(n)), _p(_links(U)), int(s), int(mu), float(beta),
                                  int(seed), int(sweep), int(lat_id), int(sampler), int(ubits))


def heatbath_substep(n, U, beta, seed, sweep, mu, parity, lat_id=0,
                     sampler=HYBRID, ubits=32, trace=None, order=None):
    if order is not None:
        order = np.ascontiguousarray(order, dtype=np.int64)
    return lib().or_heatbath_substep(_p(_dims(n)), _p(_links(U)), float(beta), int(seed),
                                     int(sweep), int(lat_id), int(sampler), int(ubits),
                                     int(mu), int(parity), _p(trace), _p(order))


def heatbath_sweep(n, U, beta, seed, sweep, lat_id=0, sampler=HYBRID, ubits=32,
                   trace=None, order=None):
    if order is not None:
        order = np.ascontiguousarray(order, dtype=np.int64)
    if trace is not None:
        assert trace.dtype == np.uint32 and trace.size == 4 * volume(n)
    return lib().or_heatbath_sweep(_p(_dims(n)), _p(_links(U)), float(beta), int(seed),
                                   int(sweep), int(lat_id), int(sampler), int(ubits),
                                   _p(trace), _p(order))


def overrelax_sweep(n, U):
    lib().or_overrelax_sweep(_p(_dims(n)), _p(_links(U)))


def plaquette(n, U):
    r = np.zeros(3)
    lib().or_plaquette(_p(_dims(n)), _p(_links(U)), _p(r[0:]), _p(r[1:]), _p(r[2:]))
    return float(r[0]), float(r[1]), float(r[2])


def polyakov(n, U):
    return lib().or_polyakov(_p(_dims(n)), _p(_links(U)))


def ape(n, U, alpha, nsteps):
    S = np.zeros((volume(n), 3, 4))
    lib().or_ape(_p(_dims(n)), _p(_links(U)), float(alpha), int(nsteps), _p(S))
    return S


def wilson(n, U, Rmax, Tmax, S=None):
    W = np.zeros((Rmax, Tmax))
    if S is not None:
        S = np.ascontiguousarray(S, dtype=np.float64)
    lib().or_wilson(_p(_dims(n)), _p(_links(U)), _p(S), int(Rmax), int(Tmax), _p(W))
    return W


def wilson_rt(n, U, R, T, S=None):
    if S is not None:
        S = np.ascontiguousarray(S, dtype=np.float64)
    return lib().or_wilson_rt(_p(_dims(n)), _p(_links(U)), _p(S), int(R), int(T))


def gauge_transform(n, U, seed):
    lib().or_gauge_transform(_p(_dims(n)), _p(_links(U)), int(seed))


def max_unit_defect(n, U):
    return lib().or_max_unit_defect(_p(_dims(n)), _p(_links(U)))
