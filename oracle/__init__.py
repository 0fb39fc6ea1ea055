"""FP64 CPU oracle for the SU(Nc) Wilson-action checkerboard sweep.

TEST INFRASTRUCTURE ONLY.  Plain, slow reference written from Cardoso &
Bicudo (arXiv:1112.4533), Sec. 2 (action, staple, heatbath, Cabibbo-Marinari,
overrelaxation, re-unitarization) and Sec. 3 (chessboard kernels).  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It shares no code with the HIP library.

Fields are numpy complex128 arrays of shape (4, V, Nc, Nc), indexed
[mu, s, i, j] with s = x + Lx*(y + Ly*(z + Lz*t)).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L4 = ctypes.c_int * 4
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = ctypes.c_int
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_uniform.argtypes = [ctypes.c_uint32]
        L.orc_uniform.restype = ctypes.c_double
        L.orc_check.argtypes = [ctypes.c_int, L4]
        L.orc_init.argtypes = [ctypes.c_int, L4, dp, ctypes.c_int, ctypes.c_uint64]
        L.orc_phase.argtypes = [ctypes.c_int, L4, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, dp, ip, dp]
        L.orc_sweep.argtypes = [ctypes.c_int, L4, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        L.orc_reunitarize.argtypes = [ctypes.c_int, L4, dp]
        L.orc_plaquette.argtypes = [ctypes.c_int, L4, dp, dp]
        L.orc_polyakov.argtypes = [ctypes.c_int, L4, dp, dp]
        L.orc_unitarity.argtypes = [ctypes.c_int, L4, dp, dp]
        L.orc_action.argtypes = [ctypes.c_int, L4, dp, ctypes.c_double, dp]
        L.orc_staple.argtypes = [ctypes.c_int, L4, dp, ctypes.c_int64, ctypes.c_int, dp]
        L.orc_heatbath_link.argtypes = [ctypes.c_int, L4, dp, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_overrelax_link.argtypes = [ctypes.c_int, L4, dp, ctypes.c_int64, ctypes.c_int,
                                         ctypes.c_int]
        L.orc_reunit_matrix.argtypes = [ctypes.c_int, dp]
        L.orc_phase_access_check.argtypes = [ctypes.c_int, L4, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                             ctypes.POINTER(ctypes.c_int64)]
        L.orc_sample_su2.argtypes = [dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_uint32, dp, ip, dp]
        _lib = L
    return _lib


def _L4(L):
    L = tuple(int(v) for v in L)
    assert len(L) == 4
    return (ctypes.c_int * 4)(*L)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle: {what} rejected its arguments")


def volume(L):
    return int(np.prod([int(v) for v in L]))


def _field(U, nc, L):
    assert U.dtype == np.complex128 and U.flags.c_contiguous
    assert U.shape == (4, volume(L), nc, nc), U.shape
    return U


def valid(nc, L):
    return lib().orc_check(int(nc), _L4(L)) == 0


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """Threads of later lattice-wide calls (results do not depend on it)."""
    _check(lib().orc_set_num_threads(int(n)), "set_num_threads")


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(w):
    return lib().orc_uniform(int(w) & 0xFFFFFFFF)


def new_field(nc, L, hot=False, seed=0):
    U = np.zeros((4, volume(L), nc, nc), dtype=np.complex128)
    _check(lib().orc_init(nc, _L4(L), _dp(U), int(bool(hot)), int(seed)), "init")
    return U


def phase(U, nc, L, kind, mu, parity, beta, seed, step, want_margin=False):
    """One checkerboard phase in place; kind 0 = heatbath, 1 = overrelaxation.
    With want_margin, returns per-site (decision margin, attempts, conditioning
    |A|_F / k_min); sites not updated get -1."""
    _field(U, nc, L)
    V = volume(L)
    margin = np.empty(V) if want_margin else None
    attempts = np.empty(V, dtype=np.int32) if want_margin else None
    cond = np.empty(V) if want_margin else None
    rc = lib().orc_phase(nc, _L4(L), _dp(U), int(kind), int(mu), int(parity), float(beta),
                         int(seed), int(step),
                         _dp(margin) if margin is not None else None,
                         attempts.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
                         if attempts is not None else None,
                         _dp(cond) if cond is not None else None)
    _check(rc, "phase")
    return (margin, attempts, cond) if want_margin else None


def phase_access_check(U, nc, L, kind, mu, parity, beta=1.0, seed=0, step=0):
    """Runs one phase serially with the oracle's access log (race check of
    the chessboard, Sec. 3): returns (links written by more than one update,
    links written by one update and read by another, links written).
    parity 2 updates both parities in one pass, a deliberately broken
    schedule."""
    _field(U, nc, L)
    out = (ctypes.c_int64 * 3)()
    _check(lib().orc_phase_access_check(nc, _L4(L), _dp(U), int(kind), int(mu), int(parity), float(beta),
                                        int(seed), int(step), out), "phase_access_check")
    return int(out[0]), int(out[1]), int(out[2])


def sweep(U, nc, L, beta, n_hb, n_or, seed, step0, reunit=True):
    _field(U, nc, L)
    _check(lib().orc_sweep(nc, _L4(L), _dp(U), float(beta), int(n_hb), int(n_or), int(seed),
                           int(step0), int(bool(reunit))), "sweep")


def reunitarize(U, nc, L):
    _field(U, nc, L)
    _check(lib().orc_reunitarize(nc, _L4(L), _dp(U)), "reunitarize")


def plaquette(U, nc, L):
    _field(U, nc, L)
    out = np.zeros(3)
    _check(lib().orc_plaquette(nc, _L4(L), _dp(U), _dp(out)), "plaquette")
    return out


def polyakov(U, nc, L):
    _field(U, nc, L)
    out = np.zeros(2)
    _check(lib().orc_polyakov(nc, _L4(L), _dp(U), _dp(out)), "polyakov")
    return complex(out[0], out[1])


def unitarity(U, nc, L):
    _field(U, nc, L)
    out = np.zeros(2)
    _check(lib().orc_unitarity(nc, _L4(L), _dp(U), _dp(out)), "unitarity")
    return out


def action(U, nc, L, beta):
    _field(U, nc, L)
    out = np.zeros(1)
    _check(lib().orc_action(nc, _L4(L), _dp(U), float(beta), _dp(out)), "action")
    return float(out[0])


def staple(U, nc, L, s, mu):
    _field(U, nc, L)
    A = np.zeros((nc, nc), dtype=np.complex128)
    _check(lib().orc_staple(nc, _L4(L), _dp(U), int(s), int(mu), _dp(A)), "staple")
    return A


def heatbath_link(U, nc, L, s, mu, beta, seed, step):
    _field(U, nc, L)
    _check(lib().orc_heatbath_link(nc, _L4(L), _dp(U), int(s), int(mu), float(beta), int(seed),
                                   int(step)), "heatbath_link")


def overrelax_link(U, nc, L, s, mu, reverse=False):
    _field(U, nc, L)
    _check(lib().orc_overrelax_link(nc, _L4(L), _dp(U), int(s), int(mu), int(bool(reverse))),
           "overrelax_link")


def reunit_matrix(M):
    M = np.ascontiguousarray(M, dtype=np.complex128).copy()
    nc = M.shape[0]
    assert M.shape == (nc, nc)
    _check(lib().orc_reunit_matrix(nc, _dp(M)), "reunit_matrix")
    return M


def sample_su2(alpha, seed, step=0, mu_sg=0):
    """Draws x in SU(2) ~ exp(alpha x0) dHaar for each alpha (counter site = index)."""
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    n = alpha.size
    x = np.zeros((n, 4))
    att = np.zeros(n, dtype=np.int32)
    margin = np.zeros(n)
    _check(lib().orc_sample_su2(_dp(alpha), n, int(seed), int(step), int(mu_sg), _dp(x),
                                att.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(margin)),
           "sample_su2")
    return x, att, margin
