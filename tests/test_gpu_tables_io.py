"""The paper's binary table files (section 2, eq. 2.7): written from the
device's tables, checked against the paper's printed u_11 (eqs. 2.5, 2.6) and
the oracle, read back with every table compared bit for bit.
"""
import json
import struct

import numpy as np
import pytest

import oracle
from paper_1601_00636_amd import binding as cb
from paper_1601_00636_amd import workloads as wl
from tests.conftest import golden_path

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    h = cb.cuboid_create(0)
    yield h
    assert cb.cuboid_destroy(h) == cb.OK


@pytest.fixture(scope="module")
def files(ctx, tmp_path_factory):
    d = tmp_path_factory.mktemp("tables")
    t, p, x = str(d / "Cuboid_pq_bit_tables.bin"), str(d / "Cuboid_primes.bin"), str(d / "tables.txt")
    cb.cuboid_write_table_files(ctx, wl.PRIMES_PAPER, t, p, x)
    return t, p, x


def _items(path):
    raw = open(path, "rb").read()
    assert len(raw) % 8 == 0
    return [struct.unpack_from("<hHI", raw, 8 * i) for i in range(len(raw) // 8)]


def test_layout_of_both_files(files):
    t, p, _ = files
    items = _items(p)
    primes = wl.PRIMES_PAPER
    assert [it[0] for it in items] == primes and all(it[1] == 0 for it in items)
    sizes = [(r * r + 7) // 8 for r in primes]
    assert [it[2] for it in items] == list(np.cumsum([0] + sizes[:-1]))
    assert len(open(t, "rb").read()) == sum(sizes)
    # the paper's "1.5 Mb" is an upper bound on these 96 tables
    assert sum(sizes) < 1.5 * 2**20


def test_tables_match_paper_and_oracle(files):
    t, p, _ = files
    raw = open(t, "rb").read()
    items = _items(p)
    with open(golden_path("u11_packed.json")) as f:
        u11 = json.load(f)
    off11 = items[0][2]
    assert items[1][2] - off11 == u11["n_bytes"]
    for idx, bits in u11["shown_msb_first"].items():
        assert format(raw[off11 + int(idx)], "08b") == bits, idx
    for r, _, off in items:
        if r <= 101 or r == 541:
            ref = bytes(oracle.pack(r))
            assert raw[off:off + len(ref)] == ref, r


def test_text_dump_starts_with_the_printed_table(files):
    _, _, x = files
    lines = open(x).read().split("\n")
    assert lines[0] == "r = 11"
    printed = [ln.strip() for ln in open(golden_path("u11_table.txt")) if ln.strip() and not ln.startswith("#")]
    assert lines[1:12] == printed
    assert lines[12] == "" and lines[13] == "r = 13"


def test_check_round_trip_and_damage(ctx, files, tmp_path):
    t, p, _ = files
    assert cb.cuboid_check_table_files(ctx, t, p) == wl.PRIMES_PAPER
    raw = bytearray(open(t, "rb").read())
    raw[5000] ^= 0x10
    bad = tmp_path / "bad.bin"
    bad.write_bytes(bytes(raw))
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_check_table_files(ctx, str(bad), p)
    assert e.value.status == cb.E_DATA
    short = tmp_path / "short.bin"
    short.write_bytes(open(t, "rb").read()[:-3])
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_check_table_files(ctx, str(short), p)
    assert e.value.status == cb.E_IO
    items = bytearray(open(p, "rb").read())
    items[2] = 1                        # padding of the first item
    badp = tmp_path / "badp.bin"
    badp.write_bytes(bytes(items))
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_check_table_files(ctx, t, str(badp))
    assert e.value.status == cb.E_DATA
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_check_table_files(ctx, t, str(tmp_path / "missing.bin"))
    assert e.value.status == cb.E_IO
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_check_table_files(ctx, t, p, cap=10)
    assert e.value.status == cb.E_CAPACITY and e.value.needed == 96
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_write_table_files(ctx, [11, 32771], str(tmp_path / "a"), str(tmp_path / "b"))
    assert e.value.status == cb.E_LIMIT
