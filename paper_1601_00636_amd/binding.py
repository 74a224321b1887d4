"""Thin ctypes binding over libcuboid.so with the C interface's names
(include/cuboid.h).  Argument marshalling only: every step of the sieve runs in
the library's HIP kernels.  Raises CuboidError for non-zero status codes.

One HIP runtime per process: PyTorch wheels ship a HIP runtime of their own
(torch/lib/libamdhip64.so, with the same soname libamdhip64.so.7 as
/opt/rocm's).  The library is loaded after torch whenever torch is importable,
so its libamdhip64.so.7 dependency is satisfied by the copy torch has already
mapped and the two share devices, streams and memory; loading fails if two
HIP runtimes are mapped anyway.  Without torch the library uses /opt/rocm's.

Streams: None (the context's own stream), a raw hipStream_t integer, or a
torch.cuda.Stream (its handle).  Device buffers: integer addresses, or torch
device tensors passed by data_ptr() (TensorBatch).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CUBOID_LIB selects another build of the library (e.g. the host-sanitized one)
LIB_PATH = os.environ.get("CUBOID_LIB") or os.path.join(_HERE, "libcuboid.so")

(OK, E_BUSY, E_RANGE, E_LIMIT, E_PRIMES, E_CAPACITY, E_NOT_LOADED, E_DEVICE, E_ARG, E_IO,
 E_DATA) = range(11)

u8, u32, u64, i32 = ctypes.c_uint8, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
P = ctypes.POINTER


class cuboid_root(ctypes.Structure):
    _fields_ = [("p", u32), ("q", u32), ("t", u64), ("t_hi", u64), ("flags", u32),
                ("input_index", u32)]


class cuboid_request(ctypes.Structure):
    _fields_ = [("p0", u32), ("p1", u32), ("q0", u32), ("q1", u32)]


class cuboid_result(ctypes.Structure):
    _fields_ = [("survivors", P(u64)), ("cap", u64), ("n_survivors", u64), ("counts", P(u64)),
                ("n_pairs", u64), ("status", ctypes.c_int32), ("reserved", u32)]


class cuboid_tuning(ctypes.Structure):
    _fields_ = [("dense_primes", u32), ("workgroups", u32), ("lds_budget", u32), ("schedule", u32),
                ("piece_units", u32)]


class cuboid_timing(ctypes.Structure):
    _fields_ = [("sweep_ms", ctypes.c_double), ("total_gpu_ms", ctypes.c_double), ("units", u64),
                ("dense_primes", u32), ("workgroups", u32), ("graph", u32), ("reserved", u32)]


class cuboid_search_report(ctypes.Structure):
    _fields_ = [("p", u32), ("q", u32), ("p_hundred", u32), ("r_max", u32), ("pairs", u64),
                ("survivors", u64), ("unix_time", ctypes.c_int64), ("running", i32),
                ("status", i32)]


def _report(r):
    return {k: getattr(r, k) for k, _ in cuboid_search_report._fields_}


class cuboid_server_config(ctypes.Structure):
    _fields_ = [("streams", u32), ("max_slots", u32), ("max_launch_units", u64),
                ("hbm_budget_bytes", u64)]


class cuboid_server_stats(ctypes.Structure):
    _fields_ = [("submitted", u64), ("completed", u64), ("launches", u64), ("units", u64),
                ("max_admitted", u32), ("resweeps", u32)]


class cuboid_request_timing(ctypes.Structure):
    _fields_ = [("submit_ns", u64), ("admit_ns", u64), ("done_ns", u64)]


class CuboidError(RuntimeError):
    def __init__(self, status, what="", needed=None):
        self.status = status
        self.needed = needed
        text = _lib.cuboid_status_string(status).decode() if _lib else str(status)
        super().__init__("%s: status %d (%s)" % (what, status, text))


_lib = None


def hip_runtimes():
    """Paths of the HIP runtime libraries (libamdhip64) mapped into this process."""
    found = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                path = line.split()[-1] if line.count("/") else ""
                if os.path.basename(path).startswith("libamdhip64"):
                    found.add(os.path.realpath(path))
    except OSError:
        pass
    return sorted(found)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcuboid.so is not built (run paper_1601_00636_amd.build.build())")
    try:
        import torch  # noqa: F401  (maps torch's HIP runtime before the library's dependency)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are mapped (%s): load libcuboid after torch, or "
                          "without it" % ", ".join(runtimes))
    vp = ctypes.c_void_p
    sigs = {
        "cuboid_status_string": ([i32], ctypes.c_char_p),
        "cuboid_version": ([], ctypes.c_char_p),
        "cuboid_create": ([P(vp), i32], i32),
        "cuboid_destroy": ([vp], i32),
        "cuboid_q_mod_prime": ([vp, P(u32), P(u32), P(u32), P(u32), u64, P(u32)], i32),
        "cuboid_table_bytes": ([vp, u32, P(u8), ctypes.c_size_t, P(ctypes.c_size_t)], i32),
        "cuboid_sieve_range": ([vp, u32, u32, u32, u32, P(u32), u32, P(u64), u64, P(u64), P(u64),
                                P(u64), vp], i32),
        "cuboid_sieve_region": ([vp, u32, u32, u32, P(u32), u32, P(u64), u64, P(u64), P(u64),
                                 P(u64), P(u32), vp], i32),
        "cuboid_root_check": ([vp, P(u32), P(u32), u64, P(cuboid_root), u64, P(u64)], i32),
        "cuboid_exact_check": ([u32, u32, u64, u64, P(i32), P(u32)], i32),
        "cuboid_exact_value": ([u32, u32, u64, u64, ctypes.c_char_p, ctypes.c_size_t], i32),
        "cuboid_canonical_primes": ([P(u32), u32, P(u32), P(u8)], i32),
        "cuboid_sieve_batch": ([vp, P(cuboid_request), u32, P(u32), u32, P(cuboid_result), vp], i32),
        "cuboid_sieve_batch_dev": ([vp, P(cuboid_request), u32, P(u32), u32, vp, vp, vp, u64,
                                    P(u64), vp], i32),
        "cuboid_sieve_batch_dev_noalloc": ([vp, P(cuboid_request), u32, P(u32), u32, vp, vp, vp,
                                            u64, P(u64), vp], i32),
        "cuboid_device_alloc": ([vp, ctypes.c_size_t, P(vp)], i32),
        "cuboid_probe_peaks": ([vp, P(ctypes.c_double), P(ctypes.c_double)], i32),
        "cuboid_device_free": ([vp, vp], i32),
        "cuboid_device_read": ([vp, vp, vp, ctypes.c_size_t, vp], i32),
        "cuboid_autotune": ([vp, P(u32), u32, ctypes.c_char_p, P(cuboid_tuning)], i32),
        "cuboid_autotune_for": ([vp, P(u32), u32, P(cuboid_request), u32, ctypes.c_char_p,
                                 P(cuboid_tuning)], i32),
        "cuboid_set_tuning": ([vp, P(u32), u32, P(cuboid_tuning)], i32),
        "cuboid_get_tuning": ([vp, P(u32), u32, P(cuboid_tuning)], i32),
        "cuboid_enable_timing": ([vp, i32], i32),
        "cuboid_last_timing": ([vp, P(cuboid_timing)], i32),
        "cuboid_enable_graphs": ([vp, i32], i32),
        "cuboid_write_table_files": ([vp, P(u32), u32, ctypes.c_char_p, ctypes.c_char_p,
                                      ctypes.c_char_p], i32),
        "cuboid_check_table_files": ([vp, ctypes.c_char_p, ctypes.c_char_p, P(u32), u32, P(u32)],
                                     i32),
        "cuboid_search_start": ([vp, P(u32), u32, u32, u32, u32, ctypes.c_char_p, P(vp)], i32),
        "cuboid_search_current": ([vp, P(cuboid_search_report)], i32),
        "cuboid_search_survivors": ([vp, P(u64), u64, P(u64)], i32),
        "cuboid_search_stop": ([vp, P(cuboid_search_report)], i32),
        "cuboid_server_start": ([vp, P(u32), u32, P(cuboid_server_config), P(vp)], i32),
        "cuboid_server_submit": ([vp, P(cuboid_request), P(u64)], i32),
        "cuboid_server_submit_many": ([vp, P(cuboid_request), u32, P(u64), P(u32)], i32),
        "cuboid_server_poll": ([vp, u64, P(cuboid_result), i32, P(cuboid_request_timing)], i32),
        "cuboid_server_stats_get": ([vp, P(cuboid_server_stats)], i32),
        "cuboid_server_stop": ([vp], i32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def lib():
    return _load()


def exported_symbols():
    """Names of the C entry points this binding knows."""
    _load()
    return [n for n in dir(_lib) if n.startswith("cuboid_")]


def _arr(a, dtype):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    return a


def _p(a, ct):
    return a.ctypes.data_as(P(ct))


def _stream(stream):
    """None (the context's stream), a raw hipStream_t, or a torch stream, whose
    handle is a stream of the same HIP runtime (see the module docstring).
    torch's default stream is the null stream, handle 0, which the C interface
    reads as the context's own stream: work already queued on it is waited
    for first, so the call still comes after it (every call returns
    synchronised)."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream) if stream else None
    handle = int(stream.cuda_stream)
    if not handle:
        stream.synchronize()
        return None
    return ctypes.c_void_p(handle)


def _check(st, what, needed=None):
    if st != OK:
        raise CuboidError(st, what, needed)


# ---------------------------------------------------------------- functions

def cuboid_status_string(status):
    return _load().cuboid_status_string(int(status)).decode()


def cuboid_version():
    return _load().cuboid_version().decode()


def cuboid_create(device=0):
    h = ctypes.c_void_p()
    _check(_load().cuboid_create(ctypes.byref(h), int(device)), "cuboid_create")
    return h


def cuboid_destroy(ctx):
    return _load().cuboid_destroy(ctx)


def cuboid_q_mod_prime(ctx, p, q, t, r):
    p, q, t, r = (_arr(x, np.uint32) for x in (p, q, t, r))
    n = len(p)
    out = np.zeros(n, dtype=np.uint32)
    _check(_load().cuboid_q_mod_prime(ctx, _p(p, u32), _p(q, u32), _p(t, u32), _p(r, u32), n,
                                      _p(out, u32)), "cuboid_q_mod_prime")
    return out


def cuboid_table_bytes(ctx, r):
    written = ctypes.c_size_t(0)
    st = _load().cuboid_table_bytes(ctx, int(r), None, 0, ctypes.byref(written))
    if st not in (OK, E_CAPACITY):
        _check(st, "cuboid_table_bytes")
    buf = np.zeros(max(1, written.value), dtype=np.uint8)
    _check(_load().cuboid_table_bytes(ctx, int(r), _p(buf, u8), buf.size, ctypes.byref(written)),
           "cuboid_table_bytes")
    return bytes(buf[:written.value])


def cuboid_sieve_range(ctx, p0, p1, q0, q1, primes, cap=1 << 20, stream=None):
    """dict(counts, n_pairs, survivors, n_survivors); raises CuboidError."""
    pr = _arr(primes, np.uint32)
    counts = np.zeros(max(1, len(pr)), dtype=np.uint64)
    surv = np.empty(max(1, cap), dtype=np.uint64)   # first n_survivors written
    ns, npairs = ctypes.c_uint64(0), ctypes.c_uint64(0)
    st = _load().cuboid_sieve_range(ctx, int(p0), int(p1), int(q0), int(q1), _p(pr, u32), len(pr),
                                    _p(surv, u64), int(cap), ctypes.byref(ns), _p(counts, u64),
                                    ctypes.byref(npairs), _stream(stream))
    _check(st, "cuboid_sieve_range", needed=ns.value if st == E_CAPACITY else None)
    return dict(counts=counts[:len(pr)], n_pairs=npairs.value, n_survivors=ns.value,
                survivors=surv[:ns.value].copy())


def cuboid_sieve_region(ctx, p0, p1, primes, band_rows=100, cap=1 << 16, stream=None):
    """Region (1.2) for p0 <= p <= p1: dict(counts, n_pairs, n_survivors,
    survivors as (p, q) pairs, r_max per band of band_rows rows)."""
    pr = _arr(primes, np.uint32)
    counts = np.zeros(max(1, len(pr)), dtype=np.uint64)
    surv = np.empty(max(1, cap), dtype=np.uint64)
    n_bands = (int(p1) - int(p0) + band_rows) // band_rows if p1 >= p0 and band_rows else 1
    rmax = np.zeros(max(1, n_bands), dtype=np.uint32)
    ns, npairs = ctypes.c_uint64(0), ctypes.c_uint64(0)
    st = _load().cuboid_sieve_region(ctx, int(p0), int(p1), int(band_rows), _p(pr, u32), len(pr),
                                     _p(surv, u64), int(cap), ctypes.byref(ns), _p(counts, u64),
                                     ctypes.byref(npairs), _p(rmax, u32), _stream(stream))
    _check(st, "cuboid_sieve_region", needed=ns.value if st == E_CAPACITY else None)
    sv = surv[:ns.value]
    return dict(counts=counts[:len(pr)], n_pairs=npairs.value, n_survivors=ns.value,
                survivors=[(int(x >> np.uint64(32)), int(x & np.uint64(0xffffffff))) for x in sv],
                r_max=rmax[:n_bands].copy())


def cuboid_write_table_files(ctx, primes, tables_path, primes_path, text_path=None):
    pr = _arr(primes, np.uint32)
    enc = lambda x: x.encode() if x else None
    _check(_load().cuboid_write_table_files(ctx, _p(pr, u32), len(pr), enc(tables_path),
                                            enc(primes_path), enc(text_path)),
           "cuboid_write_table_files")


def cuboid_check_table_files(ctx, tables_path, primes_path, cap=6542):
    """Checks the files against the device's tables; returns their prime list."""
    out = np.zeros(max(1, cap), dtype=np.uint32)
    n = u32(0)
    st = _load().cuboid_check_table_files(ctx, tables_path.encode(), primes_path.encode(),
                                          _p(out, u32), int(cap), ctypes.byref(n))
    _check(st, "cuboid_check_table_files", needed=n.value if st == E_CAPACITY else None)
    return [int(x) for x in out[:n.value]]


def cuboid_search_start(ctx, primes, p=152, q=3, p_end=0, report_path=None):
    """Starts the background region search; returns its handle."""
    pr = _arr(primes, np.uint32)
    h = ctypes.c_void_p()
    rp = report_path.encode() if report_path else None
    _check(_load().cuboid_search_start(ctx, _p(pr, u32), len(pr), int(p), int(q), int(p_end), rp,
                                       ctypes.byref(h)), "cuboid_search_start")
    return h


def cuboid_search_current(h):
    r = cuboid_search_report()
    _check(_load().cuboid_search_current(h, ctypes.byref(r)), "cuboid_search_current")
    return _report(r)


def cuboid_search_survivors(h, cap=1 << 16):
    buf = np.empty(max(1, cap), dtype=np.uint64)
    n = ctypes.c_uint64(0)
    st = _load().cuboid_search_survivors(h, _p(buf, u64), int(cap), ctypes.byref(n))
    _check(st, "cuboid_search_survivors", needed=n.value if st == E_CAPACITY else None)
    return [(int(x >> np.uint64(32)), int(x & np.uint64(0xffffffff))) for x in buf[:n.value]]


def cuboid_search_stop(h):
    """Stops the search; returns its final report (raises if it ended in error)."""
    r = cuboid_search_report()
    st = _load().cuboid_search_stop(h, ctypes.byref(r))
    rep = _report(r)
    _check(st, "cuboid_search_stop")
    return rep


def cuboid_root_check(ctx, p, q, cap=1 << 16):
    """List of (p, q, t, flags, input_index) for every positive integer root."""
    p, q = _arr(p, np.uint32), _arr(q, np.uint32)
    roots = (cuboid_root * max(1, cap))()
    n = ctypes.c_uint64(0)
    st = _load().cuboid_root_check(ctx, _p(p, u32), _p(q, u32), len(p), roots, int(cap),
                                   ctypes.byref(n))
    _check(st, "cuboid_root_check", needed=n.value if st == E_CAPACITY else None)
    return [(r.p, r.q, r.t | r.t_hi << 64, r.flags, r.input_index) for r in roots[:n.value]]


def _t_halves(t):
    t = int(t)
    if t < 0 or t >= 1 << 128:
        raise ValueError("t must be in [0, 2^128)")
    return t & ((1 << 64) - 1), t >> 64


def cuboid_exact_check(p, q, t):
    z, f = i32(0), u32(0)
    lo, hi = _t_halves(t)
    _check(_load().cuboid_exact_check(int(p), int(q), lo, hi, ctypes.byref(z), ctypes.byref(f)),
           "cuboid_exact_check")
    return bool(z.value), f.value


def cuboid_exact_value(p, q, t):
    buf = ctypes.create_string_buffer(1024)
    lo, hi = _t_halves(t)
    _check(_load().cuboid_exact_value(int(p), int(q), lo, hi, buf, 1024), "cuboid_exact_value")
    return int(buf.value.decode())


def cuboid_canonical_primes(primes):
    pr = _arr(primes, np.uint32)
    out = np.zeros(max(1, len(pr)), dtype=np.uint32)
    triv = np.zeros(max(1, len(pr)), dtype=np.uint8)
    _check(_load().cuboid_canonical_primes(_p(pr, u32), len(pr), _p(out, u32), _p(triv, u8)),
           "cuboid_canonical_primes")
    return out[:len(pr)], triv[:len(pr)].astype(bool)


_RESULT_DTYPE = np.dtype([("survivors", "<u8"), ("cap", "<u8"), ("n_survivors", "<u8"),
                          ("counts", "<u8"), ("n_pairs", "<u8"), ("status", "<i4"),
                          ("reserved", "<u4")])
assert _RESULT_DTYPE.itemsize == ctypes.sizeof(cuboid_result)


class BatchResult:
    """Per-request results of cuboid_sieve_batch as arrays: status[n],
    counts[n, n_primes], n_pairs[n], n_survivors[n]; survivors of request i
    are survivors_flat[offsets[i] : offsets[i] + n_survivors[i]] when
    status[i] == OK.  Indexing gives one request as a dict."""

    def __init__(self, status, counts, n_pairs, n_survivors, flat, offsets):
        self.status, self.counts, self.n_pairs = status, counts, n_pairs
        self.n_survivors, self.survivors_flat, self.offsets = n_survivors, flat, offsets

    _res = None
    _caps = None

    def fits(self, n, n_primes, caps):
        """Whether a call with n requests, n_primes primes and these caps can
        reuse this result's arrays."""
        return (self._res is not None and len(self.status) == n and self.counts.shape[1] == n_primes
                and np.array_equal(self._caps, caps))

    def __len__(self):
        return len(self.status)

    def survivors(self, i):
        if self.status[i] != OK:
            return None
        a = int(self.offsets[i])
        return self.survivors_flat[a:a + int(self.n_survivors[i])]

    def __getitem__(self, i):
        return dict(status=int(self.status[i]), counts=self.counts[i], n_pairs=int(self.n_pairs[i]),
                    n_survivors=int(self.n_survivors[i]), survivors=self.survivors(i))

    def __iter__(self):
        return (self[i] for i in range(len(self)))


def cuboid_device_alloc(ctx, nbytes):
    """Device memory on the context's GPU (an int address)."""
    ptr = ctypes.c_void_p()
    _check(_load().cuboid_device_alloc(ctx, int(nbytes), ctypes.byref(ptr)), "cuboid_device_alloc")
    return int(ptr.value)


def cuboid_probe_peaks(ctx):
    """Measured (v_bcnt lane-ops/s, conflict-free LDS read bytes/s) of the context's GPU."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(_load().cuboid_probe_peaks(ctx, ctypes.byref(a), ctypes.byref(b)), "cuboid_probe_peaks")
    return {"valu_lane_ops_per_s": a.value, "lds_bytes_per_s": b.value}


def cuboid_device_free(ctx, ptr):
    _check(_load().cuboid_device_free(ctx, ctypes.c_void_p(int(ptr)) if ptr else None),
           "cuboid_device_free")


def cuboid_device_read(ctx, ptr, out, stream=None):
    """Copy len(out) elements' bytes from device address ptr into the numpy array out."""
    out = np.ascontiguousarray(out)
    _check(_load().cuboid_device_read(ctx, out.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.c_void_p(int(ptr)), out.nbytes, _stream(stream)),
           "cuboid_device_read")
    return out


_SURV_DEV_DTYPE = np.dtype([("idx", "<u8"), ("req", "<u4"), ("pad", "<u4")])


class DeviceBatch:
    """Device buffers for cuboid_sieve_batch_dev: counts [n_req][n_primes],
    pairs [n_req], surv_cap survivor entries.  read() brings them back."""

    def __init__(self, ctx, n_req, n_primes, surv_cap=0):
        self.ctx, self.n_req, self.n_primes, self.surv_cap = ctx, int(n_req), int(n_primes), int(surv_cap)
        self.counts = cuboid_device_alloc(ctx, max(1, self.n_req * self.n_primes) * 8)
        self.pairs = cuboid_device_alloc(ctx, max(1, self.n_req) * 8)
        self.surv = cuboid_device_alloc(ctx, self.surv_cap * 16) if self.surv_cap else 0
        self.n_survivors = 0

    def read(self):
        counts = cuboid_device_read(self.ctx, self.counts,
                                    np.empty((self.n_req, self.n_primes), dtype=np.uint64))
        pairs = cuboid_device_read(self.ctx, self.pairs, np.empty(self.n_req, dtype=np.uint64))
        k = min(self.n_survivors, self.surv_cap)
        surv = (cuboid_device_read(self.ctx, self.surv, np.empty(k, dtype=_SURV_DEV_DTYPE))
                if k else np.empty(0, dtype=_SURV_DEV_DTYPE))
        return counts, pairs, surv

    def free(self):
        for a in ("counts", "pairs", "surv"):
            if getattr(self, a):
                cuboid_device_free(self.ctx, getattr(self, a))
                setattr(self, a, 0)


class TensorBatch:
    """cuboid_sieve_batch_dev's outputs in caller-owned torch device tensors,
    passed by data_ptr(): counts [n_req, n_primes] and pairs [n_req], int64 or
    uint64; survivors int64 or uint64 [surv_cap, 2] (row k: the pair index and
    the request number), or None.  read() returns numpy copies as
    DeviceBatch.read() does."""

    def __init__(self, counts, pairs, survivors=None):
        def check(t, name, ndim):
            if not t.is_cuda or not t.is_contiguous() or t.element_size() != 8 or t.dim() != ndim:
                raise ValueError("%s: a contiguous 64-bit integer device tensor of %d dims"
                                 % (name, ndim))
        check(counts, "counts", 2)
        check(pairs, "pairs", 1)
        if counts.shape[0] != pairs.shape[0]:
            raise ValueError("counts and pairs disagree on the number of requests")
        self.n_req, self.n_primes = int(counts.shape[0]), int(counts.shape[1])
        self.tensors = (counts, pairs, survivors)
        self.counts, self.pairs = counts.data_ptr(), pairs.data_ptr()
        self.surv, self.surv_cap = 0, 0
        if survivors is not None:
            check(survivors, "survivors", 2)
            if survivors.shape[1] != 2:
                raise ValueError("survivors: shape [surv_cap, 2]")
            self.surv, self.surv_cap = survivors.data_ptr(), int(survivors.shape[0])
        self.n_survivors = 0

    def read(self):
        counts, pairs, survivors = self.tensors
        c = counts.cpu().numpy().view(np.uint64)
        p = pairs.cpu().numpy().view(np.uint64)
        k = min(self.n_survivors, self.surv_cap)
        if k:
            raw = survivors[:k].cpu().numpy()
            surv = np.ascontiguousarray(raw).view(_SURV_DEV_DTYPE).reshape(k)
        else:
            surv = np.empty(0, dtype=_SURV_DEV_DTYPE)
        return c, p, surv


def cuboid_sieve_batch_dev(ctx, requests, primes, dev, stream=None):
    """requests: (n, 4) array-like of (p0, p1, q0, q1); dev: a DeviceBatch or
    TensorBatch of the same n and prime count.  Returns the status;
    dev.n_survivors is set."""
    pr = _arr(primes, np.uint32)
    reqa = np.ascontiguousarray(np.asarray(requests, dtype=np.uint32).reshape(-1, 4))
    n = reqa.shape[0]
    if n != dev.n_req or len(pr) != dev.n_primes:
        raise ValueError("device buffers are for %d requests x %d primes" % (dev.n_req, dev.n_primes))
    ns = ctypes.c_uint64(0)
    st = _load().cuboid_sieve_batch_dev(ctx, reqa.ctypes.data_as(P(cuboid_request)), n, _p(pr, u32),
                                        len(pr), ctypes.c_void_p(dev.counts),
                                        ctypes.c_void_p(dev.pairs),
                                        ctypes.c_void_p(dev.surv) if dev.surv else None,
                                        dev.surv_cap, ctypes.byref(ns), _stream(stream))
    dev.n_survivors = int(ns.value)
    if st not in (OK, E_CAPACITY, E_LIMIT):
        _check(st, "cuboid_sieve_batch_dev")
    return st


def cuboid_sieve_batch_dev_noalloc(ctx, requests, primes, dev, stream=None):
    """cuboid_sieve_batch_dev without any device allocation: scratch comes from
    the library's fixed per-GPU array; the prime list's tables and rows up to
    the largest p must be resident from an earlier call.  Same arguments and
    results as cuboid_sieve_batch_dev."""
    pr = _arr(primes, np.uint32)
    reqa = np.ascontiguousarray(np.asarray(requests, dtype=np.uint32).reshape(-1, 4))
    n = reqa.shape[0]
    if n != dev.n_req or len(pr) != dev.n_primes:
        raise ValueError("device buffers are for %d requests x %d primes" % (dev.n_req, dev.n_primes))
    ns = ctypes.c_uint64(0)
    st = _load().cuboid_sieve_batch_dev_noalloc(
        ctx, reqa.ctypes.data_as(P(cuboid_request)), n, _p(pr, u32), len(pr),
        ctypes.c_void_p(dev.counts), ctypes.c_void_p(dev.pairs),
        ctypes.c_void_p(dev.surv) if dev.surv else None, dev.surv_cap, ctypes.byref(ns),
        _stream(stream))
    dev.n_survivors = int(ns.value)
    if st not in (OK, E_CAPACITY, E_LIMIT):
        _check(st, "cuboid_sieve_batch_dev_noalloc")
    return st


def cuboid_sieve_batch(ctx, requests, primes, caps=1024, stream=None, out=None):
    """requests: (n, 4) array-like of (p0, p1, q0, q1).  Returns (status, BatchResult).

    out: a BatchResult of an earlier call with the same number of requests,
    primes and caps; its arrays are overwritten instead of allocating new ones."""
    pr = _arr(primes, np.uint32)
    reqa = np.ascontiguousarray(np.asarray(requests, dtype=np.uint32).reshape(-1, 4))
    n = reqa.shape[0]
    caps = np.full(n, caps, dtype=np.uint64) if np.isscalar(caps) else _arr(caps, np.uint64)
    if out is not None and out.fits(n, len(pr), caps):
        res, counts, flat, offsets = out._res, out.counts, out.survivors_flat, out.offsets
    else:
        offsets = np.zeros(n + 1, dtype=np.uint64)
        np.cumsum(caps, out=offsets[1:])
        flat = np.empty(max(1, int(offsets[-1])), dtype=np.uint64)
        counts = np.zeros((n, max(1, len(pr))), dtype=np.uint64)[:, :len(pr)]
        res = np.zeros(max(1, n), dtype=_RESULT_DTYPE)
        res["survivors"][:n] = flat.ctypes.data + offsets[:-1] * 8
        res["cap"][:n] = caps
        res["counts"][:n] = counts.ctypes.data + np.arange(n, dtype=np.uint64) * (counts.strides[0])
    st = _load().cuboid_sieve_batch(ctx, reqa.ctypes.data_as(P(cuboid_request)), n, _p(pr, u32),
                                    len(pr), res.ctypes.data_as(P(cuboid_result)),
                                    _stream(stream))
    if st not in (OK, E_CAPACITY, E_LIMIT):
        _check(st, "cuboid_sieve_batch")
    if out is not None and out._res is res:
        return st, out
    r = BatchResult(res["status"][:n], counts, res["n_pairs"][:n], res["n_survivors"][:n], flat,
                    offsets)
    r._res, r._caps = res, caps.copy()
    return st, r


def cuboid_enable_timing(ctx, on=True):
    _check(_load().cuboid_enable_timing(ctx, 1 if on else 0), "cuboid_enable_timing")


def cuboid_last_timing(ctx):
    t = cuboid_timing()
    _check(_load().cuboid_last_timing(ctx, ctypes.byref(t)), "cuboid_last_timing")
    return dict(sweep_ms=t.sweep_ms, total_gpu_ms=t.total_gpu_ms, units=t.units,
                dense_primes=t.dense_primes, workgroups=t.workgroups, graph=t.graph)


def cuboid_enable_graphs(ctx, on=True):
    _check(_load().cuboid_enable_graphs(ctx, 1 if on else 0), "cuboid_enable_graphs")


def _tuning(t):
    return {k: getattr(t, k) for k, _ in cuboid_tuning._fields_}


def cuboid_set_tuning(ctx, primes, dense_primes=None, workgroups=0, lds_budget=0, schedule=0,
                      piece_units=0):
    """No keyword arguments: back to the defaults.  schedule: 0 or 3 workgroup
    pieces, 1 round-robin pieces per wave, 2 shared counter; piece_units: units
    per piece (0: chosen by launch size)."""
    pr = _arr(primes, np.uint32)
    if (dense_primes is None and not workgroups and not lds_budget and not schedule
            and not piece_units):
        _check(_load().cuboid_set_tuning(ctx, _p(pr, u32), len(pr), None), "cuboid_set_tuning")
        return
    t = cuboid_tuning(0xffffffff if dense_primes is None else int(dense_primes), int(workgroups),
                      int(lds_budget), int(schedule), int(piece_units))
    _check(_load().cuboid_set_tuning(ctx, _p(pr, u32), len(pr), ctypes.byref(t)),
           "cuboid_set_tuning")


def cuboid_get_tuning(ctx, primes):
    pr = _arr(primes, np.uint32)
    t = cuboid_tuning()
    _check(_load().cuboid_get_tuning(ctx, _p(pr, u32), len(pr), ctypes.byref(t)),
           "cuboid_get_tuning")
    return _tuning(t)


def cuboid_autotune(ctx, primes, cache_path=None):
    pr = _arr(primes, np.uint32)
    t = cuboid_tuning()
    cp = cache_path.encode() if cache_path else None
    _check(_load().cuboid_autotune(ctx, _p(pr, u32), len(pr), cp, ctypes.byref(t)),
           "cuboid_autotune")
    return _tuning(t)


def cuboid_autotune_for(ctx, primes, sample, cache_path=None):
    """sample: (n, 4) array-like of (p0, p1, q0, q1), requests standing for the workload."""
    pr = _arr(primes, np.uint32)
    reqa = np.ascontiguousarray(np.asarray(sample, dtype=np.uint32).reshape(-1, 4))
    t = cuboid_tuning()
    cp = cache_path.encode() if cache_path else None
    _check(_load().cuboid_autotune_for(ctx, _p(pr, u32), len(pr),
                                       reqa.ctypes.data_as(P(cuboid_request)), reqa.shape[0], cp,
                                       ctypes.byref(t)), "cuboid_autotune_for")
    return _tuning(t)


def cuboid_server_start(ctx, primes, streams=0, max_slots=0, max_launch_units=0,
                        hbm_budget_bytes=0):
    pr = _arr(primes, np.uint32)
    cfg = cuboid_server_config(int(streams), int(max_slots), int(max_launch_units),
                               int(hbm_budget_bytes))
    h = ctypes.c_void_p()
    _check(_load().cuboid_server_start(ctx, _p(pr, u32), len(pr), ctypes.byref(cfg),
                                       ctypes.byref(h)), "cuboid_server_start")
    return h


def cuboid_server_submit(srv, rect):
    r = cuboid_request(*[int(x) for x in rect])
    t = ctypes.c_uint64(0)
    _check(_load().cuboid_server_submit(srv, ctypes.byref(r), ctypes.byref(t)),
           "cuboid_server_submit")
    return t.value


def cuboid_server_submit_many(srv, rects):
    """Queue many rectangles in one call; returns their tickets (numpy uint64).
    An invalid rectangle queues none: CuboidError E_RANGE, with .needed set to
    its index."""
    reqa = np.ascontiguousarray(np.asarray(rects, dtype=np.uint32).reshape(-1, 4))
    tickets = np.zeros(max(1, reqa.shape[0]), dtype=np.uint64)
    bad = ctypes.c_uint32(0)
    st = _load().cuboid_server_submit_many(srv, reqa.ctypes.data_as(P(cuboid_request)),
                                           reqa.shape[0], _p(tickets, u64), ctypes.byref(bad))
    _check(st, "cuboid_server_submit_many", needed=bad.value if st == E_RANGE else None)
    return tickets[:reqa.shape[0]]


def cuboid_server_poll(srv, ticket, n_primes, cap=1024, wait=True):
    """dict(status, counts, n_pairs, n_survivors, survivors, latency_ns, ...) or
    None when wait is False and the ticket is not finished."""
    counts = np.zeros(max(1, n_primes), dtype=np.uint64)
    surv = np.empty(max(1, cap), dtype=np.uint64)
    res = cuboid_result()
    res.survivors = _p(surv, u64)
    res.cap = int(cap)
    res.counts = _p(counts, u64)
    tim = cuboid_request_timing()
    st = _load().cuboid_server_poll(srv, int(ticket), ctypes.byref(res), 1 if wait else 0,
                                    ctypes.byref(tim))
    if st == E_BUSY and not wait:
        return None
    if st not in (OK,):
        raise CuboidError(st, "cuboid_server_poll",
                          needed=res.n_survivors if st == E_CAPACITY else None)
    return dict(status=res.status, counts=counts[:n_primes], n_pairs=res.n_pairs,
                n_survivors=res.n_survivors, survivors=surv[:res.n_survivors].copy(),
                submit_ns=tim.submit_ns, admit_ns=tim.admit_ns, done_ns=tim.done_ns,
                latency_ns=tim.done_ns - tim.submit_ns)


def cuboid_server_stats_get(srv):
    st = cuboid_server_stats()
    _check(_load().cuboid_server_stats_get(srv, ctypes.byref(st)), "cuboid_server_stats_get")
    return dict(submitted=st.submitted, completed=st.completed, launches=st.launches,
                units=st.units, max_admitted=st.max_admitted, resweeps=st.resweeps)


def cuboid_server_stop(srv):
    _check(_load().cuboid_server_stop(srv), "cuboid_server_stop")


class Context:
    """Owns one cuboid_ctx; methods are the functions above without `ctx`."""

    def __init__(self, device=0):
        self.handle = cuboid_create(device)

    def close(self):
        if self.handle is not None:
            st = cuboid_destroy(self.handle)
            _check(st, "cuboid_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __getattr__(self, name):
        fn = globals().get("cuboid_" + name)
        if fn is None:
            raise AttributeError(name)
        return lambda *a, **k: fn(self.handle, *a, **k)
