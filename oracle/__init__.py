"""ORACLE — test infrastructure only.

Plain CPU definition of the modulo-primes cuboid sieve of Gallyamov et al.,
arXiv:1601.00636, used to check the GPU library.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import this package; the
product library never imports, links or calls it.

Pieces:
  cuboid_oracle.c  Q_pq(t) mod r (eq. 1.1/2.2), the unsolvability tables
                   (Def. 1.1, eq. 2.3), the byte packing (eq. 2.6), the sieve
                   over rectangles and over region (1.2); plain C + OpenMP.
  poly.py          Q_pq with Python integers (eq. 1.1), Theorem 1.1 flags.
  roots.py         exact integer-root search by real-root isolation.
"""
import ctypes
import os
import subprocess

import numpy as np

from .poly import q_coeffs, q_value, theorem_1_1_flags  # noqa: F401
from .roots import integer_roots, positive_t_roots, root_check  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cuboid_oracle.c")
_LIB = os.path.join(_HERE, "_cuboid_oracle.so")
_lib = None


def build(force=True):
    """Compile the C oracle (gcc, OpenMP) next to its source."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-Wall", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    P = ctypes.POINTER
    lib.oracle_q_mod_r.argtypes = [u64, u64, u64, u32]
    lib.oracle_q_mod_r.restype = u32
    lib.oracle_coeffs_mod_r.argtypes = [u64, u64, u32, P(u32)]
    lib.oracle_coeffs_mod_r.restype = None
    lib.oracle_table.argtypes = [u32, P(ctypes.c_uint8)]
    lib.oracle_table.restype = i32
    lib.oracle_u_entry.argtypes = [u32, u32, u32]
    lib.oracle_u_entry.restype = i32
    lib.oracle_pack.argtypes = [u32, P(ctypes.c_uint8), P(ctypes.c_uint8)]
    lib.oracle_pack.restype = u64
    lib.oracle_sieve.argtypes = [u32, u32, u32, u32, P(u32), u32, P(P(ctypes.c_uint8)),
                                 P(u64), P(u64), P(u64), u64, P(u64), i32]
    lib.oracle_sieve.restype = i32
    lib.oracle_region_qmin.argtypes = [u64]
    lib.oracle_region_qmin.restype = u64
    lib.oracle_sieve_region.argtypes = [u32, u32, P(u32), u32, P(P(ctypes.c_uint8)),
                                        P(u64), P(u64), P(u64), u64, P(u64), P(u32), i32]
    lib.oracle_sieve_region.restype = i32
    _lib = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def q_mod_r(p, q, t, r):
    """Q_pq(t) mod r, eq. (1.1) reduced as in eq. (2.2)."""
    return int(_load().oracle_q_mod_r(int(p), int(q), int(t), int(r)))


def coeffs_mod_r(p, q, r):
    """[c0, c2, c4, c6, c8, 1] of eq. (1.1) reduced modulo r."""
    out = (ctypes.c_uint32 * 6)()
    _load().oracle_coeffs_mod_r(int(p), int(q), int(r), out)
    return list(out)


_table_cache = {}


def table(r):
    """u_r of eq. (2.3) as an (r, r) uint8 array indexed [p~, q~]."""
    r = int(r)
    if r not in _table_cache:
        u = np.zeros(r * r, dtype=np.uint8)
        rc = _load().oracle_table(r, _ptr(u, ctypes.c_uint8))
        if rc != 0:
            raise ValueError("oracle_table(%d) failed: %d" % (r, rc))
        _table_cache[r] = u.reshape(r, r)
    return _table_cache[r]


def pack(r, u=None):
    """Bytes of u_r packed as in eq. (2.6)."""
    r = int(r)
    if u is None:
        u = table(r)
    u = np.ascontiguousarray(u, dtype=np.uint8).reshape(-1)
    out = np.zeros((r * r + 7) // 8, dtype=np.uint8)
    n = _load().oracle_pack(r, _ptr(u, ctypes.c_uint8), _ptr(out, ctypes.c_uint8))
    return bytes(out[:n])


def _tables_arg(primes):
    tabs = [np.ascontiguousarray(table(r)).reshape(-1) for r in primes]
    arr = (ctypes.POINTER(ctypes.c_uint8) * max(1, len(tabs)))()
    for i, t in enumerate(tabs):
        arr[i] = _ptr(t, ctypes.c_uint8)
    return arr, tabs


def sieve(p0, p1, q0, q1, primes, cap=1 << 20, threads=0, direct=False):
    """The sieve over p0..p1 x q0..q1 (inclusive) with the given primes.

    Returns dict(counts (in the order `primes` was given), survivors (sorted
    uint64 pair indices, at most `cap`), n_survivors, n_pairs).  Primes are
    tested in ascending order, so each count is the number of pairs whose first
    rejecting prime is that one.  direct=True builds no tables: each bit the
    walk needs is evaluated from Definition 1.1 (for large primes).
    """
    primes = [int(r) for r in primes]
    order = sorted(range(len(primes)), key=lambda i: primes[i])
    asc = np.array([primes[i] for i in order], dtype=np.uint32)
    if direct:
        tabs_arr, _keep = None, None
    else:
        tabs_arr, _keep = _tables_arg(asc)
    counts = np.zeros(max(1, len(asc)), dtype=np.uint64)
    surv = np.zeros(max(1, cap), dtype=np.uint64)
    n_pairs = ctypes.c_uint64(0)
    n_surv = ctypes.c_uint64(0)
    rc = _load().oracle_sieve(int(p0), int(p1), int(q0), int(q1), _ptr(asc, ctypes.c_uint32),
                              len(asc), tabs_arr, _ptr(counts, ctypes.c_uint64),
                              ctypes.byref(n_pairs), _ptr(surv, ctypes.c_uint64), cap,
                              ctypes.byref(n_surv), int(threads))
    if rc != 0:
        raise ValueError("oracle_sieve failed: %d" % rc)
    out_counts = np.zeros(len(primes), dtype=np.uint64)
    for k, i in enumerate(order):
        out_counts[i] = counts[k]
    ns = n_surv.value
    return dict(counts=out_counts, survivors=surv[:min(ns, cap)].copy(),
                n_survivors=ns, n_pairs=n_pairs.value)


def u_entry(a, b, r):
    """u_r(a, b) from Definition 1.1 (r evaluations of Q mod r)."""
    return int(_load().oracle_u_entry(int(a), int(b), int(r)))


def region_qmin(p):
    """Least q allowed by the lower bound of region (1.2)."""
    return int(_load().oracle_region_qmin(int(p)))


def sieve_region(p0, p1, primes, cap=1 << 16, threads=0):
    """The sieve over region (1.2) for p0 <= p <= p1 (section 5).

    Returns dict(counts, n_pairs, survivors (list of (p, q)), n_survivors,
    max_depth (1-based position in ascending `primes` of the deepest first
    rejecting prime)).
    """
    asc = np.array(sorted(int(r) for r in primes), dtype=np.uint32)
    tabs_arr, _keep = _tables_arg(asc)
    counts = np.zeros(max(1, len(asc)), dtype=np.uint64)
    surv = np.zeros(2 * max(1, cap), dtype=np.uint64)
    n_pairs = ctypes.c_uint64(0)
    n_surv = ctypes.c_uint64(0)
    depth = ctypes.c_uint32(0)
    rc = _load().oracle_sieve_region(int(p0), int(p1), _ptr(asc, ctypes.c_uint32), len(asc),
                                     tabs_arr, _ptr(counts, ctypes.c_uint64),
                                     ctypes.byref(n_pairs), _ptr(surv, ctypes.c_uint64), cap,
                                     ctypes.byref(n_surv), ctypes.byref(depth), int(threads))
    if rc != 0:
        raise ValueError("oracle_sieve_region failed: %d" % rc)
    ns = n_surv.value
    pairs = [(int(surv[2 * k]), int(surv[2 * k + 1])) for k in range(min(ns, cap))]
    return dict(counts=counts[:len(asc)].copy(), primes=asc.tolist(), n_pairs=n_pairs.value,
                survivors=pairs, n_survivors=ns, max_depth=depth.value)
