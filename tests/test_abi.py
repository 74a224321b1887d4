"""The C-ABI library on the CPU: it loads, exports every entry point the
header declares, and its host-only functions behave (no GPU calls here)."""
import random
import re

import pytest

from oracle import poly
from paper_1601_00636_amd import binding as cb
from tests.conftest import ROOT


def _declared():
    txt = open(ROOT + "/include/cuboid.h").read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cuboid_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = cb.lib()
    names = _declared()
    assert "cuboid_sieve_range" in names and "cuboid_root_check" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_status_strings_and_version():
    assert cb.cuboid_version().endswith("gfx950")
    for s in range(11):
        assert cb.cuboid_status_string(s) and "unknown" not in cb.cuboid_status_string(s)
    assert "unknown" in cb.cuboid_status_string(99)


def test_canonical_primes():
    s, triv = cb.cuboid_canonical_primes([31, 2, 11, 7, 5, 3, 13])
    assert s.tolist() == [2, 3, 5, 7, 11, 13, 31]
    assert triv.tolist() == [True, True, True, True, False, False, False]
    for bad in ([], [4], [11, 11], [65537], [1], [65536]):
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_canonical_primes(bad)
        assert e.value.status == cb.E_PRIMES
    s, _ = cb.cuboid_canonical_primes([65521, 2])
    assert s.tolist() == [2, 65521]


def test_exact_value_matches_python_ints():
    # the whole coordinate range p, q < 2^32 and t up to 2^70 (the root bound
    # of eq. 1.1 reaches about 2^66.5 there)
    rng = random.Random(17)
    for k in range(3000):
        hi = 2**31 if k % 2 else 2**32
        p, q = rng.randrange(0, hi), rng.randrange(0, hi)
        t = rng.randrange(0, 2**64) if k % 3 else rng.randrange(0, 2**70)
        assert cb.cuboid_exact_value(p, q, t) == poly.q_value(p, q, t)
    for p, q, t in [(0, 0, 0), (1, 2, 0), (2**31 - 1, 2**31 - 1, 2**64 - 1), (5, 0, 25),
                    (2**32 - 1, 2**32 - 1, 2**70 - 1), (2**32 - 1, 0, 2**64), (2**32 - 1, 1, 2**67)]:
        assert cb.cuboid_exact_value(p, q, t) == poly.q_value(p, q, t)
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_exact_value(3, 5, 2**70)
    assert e.value.status == cb.E_LIMIT


def test_exact_check_roots_and_flags():
    for p in (1, 2, 12, 1000, 2**31 - 1, 2**31, 3000000019, 2**32 - 1):
        z, f = cb.cuboid_exact_check(p, p, p * p)
        assert z and f == poly.theorem_1_1_flags(p, p, p * p)
        assert not cb.cuboid_exact_check(p, p, p * p + 1)[0]
        z, _ = cb.cuboid_exact_check(p, 0, p * p)
        assert z
    rng = random.Random(3)
    for k in range(2000):
        hi = 2**32 if k % 2 else 2**31
        p, q = rng.randrange(0, hi), rng.randrange(0, hi)
        t = rng.randrange(0, 2**64) if k % 3 else rng.randrange(0, 2**70)
        assert cb.cuboid_exact_check(p, q, t)[1] == poly.theorem_1_1_flags(p, q, t)
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_exact_check(2**31, 1, 2**70)
    assert e.value.status == cb.E_LIMIT


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_create(0)
    assert e.value.status == cb.E_DEVICE


def test_calls_on_null_context_are_refused():
    import ctypes
    h = ctypes.c_void_p(0)
    assert cb.cuboid_destroy(h) == cb.E_NOT_LOADED
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_sieve_range(h, 1, 5, 1, 5, [11])
    assert e.value.status == cb.E_NOT_LOADED
    bogus = ctypes.c_void_p(0x1234560)
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_root_check(bogus, [1], [2])
    assert e.value.status == cb.E_NOT_LOADED
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_sieve_region(h, 1, 10, [11])
    assert e.value.status == cb.E_NOT_LOADED
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_search_start(bogus, [11], 152, 3)
    assert e.value.status == cb.E_NOT_LOADED
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_enable_graphs(h, True)
    assert e.value.status == cb.E_NOT_LOADED
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_write_table_files(h, [11], "/nonexistent/t.bin", "/nonexistent/p.bin")
    assert e.value.status == cb.E_NOT_LOADED
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_device_alloc(h, 64)
    assert e.value.status == cb.E_NOT_LOADED
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_autotune_for(bogus, [11], [(1, 2, 1, 2)])
    assert e.value.status == cb.E_NOT_LOADED
    lib = cb.lib()
    n = ctypes.c_uint64(7)
    req = (ctypes.c_uint32 * 4)(1, 5, 1, 5)
    pr = (ctypes.c_uint32 * 1)(11)
    assert lib.cuboid_sieve_batch_dev(h, ctypes.cast(req, ctypes.POINTER(cb.cuboid_request)), 1,
                                      pr, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), None, 0,
                                      ctypes.byref(n), None) == cb.E_NOT_LOADED
    assert lib.cuboid_device_read(h, None, None, 0, None) == cb.E_NOT_LOADED
    a, b = ctypes.c_double(), ctypes.c_double()
    assert lib.cuboid_probe_peaks(h, ctypes.byref(a), ctypes.byref(b)) == cb.E_NOT_LOADED


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, ROOT + "/bench.py", "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_stream_arguments():
    # torch and the library share one HIP runtime, so a torch stream's handle
    # is passed as is; the default (null) stream is waited for, then the
    # context's own stream runs the call
    class TorchStream:
        cuda_stream = 0x1234
    class DefaultTorchStream:
        cuda_stream = 0
        waited = False
        def synchronize(self):
            self.waited = True
    assert cb._stream(None) is None and cb._stream(0) is None
    d = DefaultTorchStream()
    assert cb._stream(d) is None and d.waited
    assert cb._stream(0x5000).value == 0x5000
    assert cb._stream(TorchStream()).value == 0x1234


def test_one_hip_runtime_after_load():
    # torch is mapped before the library, so at most one libamdhip64 is mapped
    cb.lib()
    assert len(cb.hip_runtimes()) <= 1
