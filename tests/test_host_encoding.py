"""Host logic of libpmscan (no GPU needed): the exported ABI, Table 2 codes,
the prime-derived Table 3 dictionary, the pattern image and the index formula
of Sect. 2.3, pinned to the values the paper prints."""
import os
import random
import re

import numpy as np
import pytest

from conftest import ROOT, golden_dict, golden_lines

scan = pytest.importorskip("paper_1611_06115_amd.scan")


@pytest.fixture(scope="module", autouse=True)
def built_library():
    if not os.path.exists(scan.LIB_PATH):
        from paper_1611_06115_amd import _build

        _build.build()
    scan.lib()


def header_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pm_[a-z_0-9]+)\s*\(", src, re.M)
    return sorted(set(names))


def test_library_exports_every_header_symbol():
    names = header_functions()
    assert "pm_scan" in names and "pm_encode_text" in names
    import ctypes

    lib = ctypes.CDLL(scan.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_table2_codes():
    for cls, sym, binary, dec in golden_lines("table2_pattern_codes.txt"):
        codes = scan.encode_pattern(sym)
        assert codes.tolist() == [int(dec)] and format(int(dec), "04b") == binary
        if cls != "-":
            # the class written as a bracket gives the same code
            assert scan.encode_pattern("[" + cls + "]").tolist() == [int(dec)]
    assert scan.encode_pattern("acgtmrwsykvhdbn-").tolist() == list(range(16))


def test_table3_pair_dictionary_from_primes():
    table = scan.pair_table()
    rows = golden_lines("table3_pair_values.txt")
    for p, row in enumerate(rows):
        vals = [int(x) for x in row[1:5]]
        idx = [int(x) for x in row[5:9]]
        code = scan.encode_pattern(row[0]).tolist()[0]
        assert code == p
        for t in range(4):
            assert idx[t] == (code << 2) | t
            assert table[idx[t]] == vals[t]


def test_sect2_3_index_example():
    g = golden_dict("example_sect2_3.txt")
    t_code = {r[0]: int(r[2]) for r in golden_lines("table1_text_codes.txt")}[g["text_symbol"][0][0]]
    p_code = scan.encode_pattern(g["pattern_symbol"][0][0])[0]
    idx = (int(p_code) << 2) | t_code
    assert idx == int(g["index"][0][0])
    assert scan.pair_table()[idx] == int(g["value"][0][0])


def test_sect2_5_steps_and_table4_indices():
    """STEP 2 p(10), STEP 3 r(2) = p << 2, and Table 4's l(10) = r OR t with the
    dictionary values of the 'match' rows."""
    g = golden_dict("example_sect2_5.txt")
    p = scan.encode_pattern(g["pattern"][0][0])
    assert p.tolist() == [int(x) for x in g["p10"][0]]
    assert [format(int(x) << 2, "06b") for x in p] == g["r2"][0]
    t1 = {r[0]: int(r[2]) for r in golden_lines("table1_text_codes.txt")}
    t10 = [t1[c] for c in g["text"][0][0]]
    assert t10 == [int(x) for x in g["t10"][0]]
    table = scan.pair_table()
    for row in g["table4"]:
        loc = int(row[0])
        vi = row.index("value")
        ls = [int(x) for x in row[2:vi]]
        vals = [int(x) for x in row[vi + 1:]]
        mine = [(int(p[j]) << 2) | t10[loc - 1 + j] for j in range(len(ls))]
        assert mine == ls
        assert [int(table[x]) for x in mine] == vals


def test_pattern_image_bits_are_table3():
    rnd = random.Random(1)
    table = scan.pair_table()
    for m in (1, 5, 31, 32, 33, 64, 100, 257):
        pat = "".join(rnd.choice("ACGTMRWSYKVHDBN-") for _ in range(m))
        codes = scan.encode_pattern(pat)
        img = scan.pattern_image(codes)
        assert img.size == 4 * ((m + 31) // 32)
        for j in range(m):
            for t in range(4):
                bit = int(img[4 * (j // 32) + t]) >> (j % 32) & 1
                assert bit == table[(int(codes[j]) << 2) | t]
        # bits past m are zero
        last = m % 32
        if last:
            for t in range(4):
                assert int(img[4 * (m // 32) + t]) >> last == 0


def test_pattern_errors():
    for bad in ("AZ", "A[]C", "A[C", "[A-]", "X", "[AC[G]]"):
        with pytest.raises(scan.PMError) as e:
            scan.encode_pattern(bad)
        assert e.value.status == -2
    assert scan.encode_pattern("[ca][GCT]").tolist() == scan.encode_pattern("MB").tolist()


def test_sizes():
    assert scan.text_bytes(0) >= 0
    for n in (1, 31, 32, 33, 10 ** 6, 3_100_000_000):
        assert scan.text_bytes(n) >= 8 * ((n + 31) // 32) + 16
        assert scan.text_bytes(n) % 16 == 0
        assert scan.workspace_bytes(n) > 0
    assert scan.lib().pm_pattern_bytes(33) == 32


def test_host_scan_chunk_bounds():
    """The host-memory scan's workspace grows with the chunk and is 0 for a
    chunk outside 1..2^48 (whose sizes would overflow); such a chunk is
    refused before any device work."""
    ws = scan.scan_host_workspace_bytes
    assert ws(0, 10) == 0 and ws(1000, 0) == 0
    assert 0 < ws(1000, 10) < ws(10 ** 6, 10) < ws(1 << 48, 10)
    assert ws((1 << 48) + 1, 10) == 0 and ws((1 << 64) - 1, 10) == 0
    import ctypes

    dummy = ctypes.c_void_p(256)  # never dereferenced: the argument check fails first
    codes = scan.encode_pattern("ACGT")
    for chunk in (0, (1 << 48) + 1, (1 << 64) - 1):
        st = scan.lib().pm_scan_host(dummy, 10 ** 6, codes.ctypes.data, 4, 0, dummy, chunk, None, None, 0,
                                     dummy, dummy, 1 << 30, None, None)
        assert st == -1, chunk


def test_expected_hits_closed_forms():
    """The output-sizing estimate: (n-m+1) * P(count <= k) for uniform bases,
    checked against closed forms (exact match probability prod |S_j|/4, and
    k >= m giving every window)."""
    P = lambda s: scan.Pattern(s)
    n = 10 ** 6
    assert scan.expected_hits(P("ACGT"), 0, n) == pytest.approx((n - 3) / 256)
    assert scan.expected_hits(P("MRN-"), 1, n) == pytest.approx((n - 3) * (0.5 * 0.5 * 1.0))
    assert scan.expected_hits(P("GATTACA"), 7, n) == pytest.approx(n - 6)
    # one mismatch allowed over 4 singletons: (1/4)^4 + 4 * (3/4) (1/4)^3
    assert scan.expected_hits(P("ACGT"), 1, n) == pytest.approx((n - 3) * (1 / 256 + 4 * 0.75 / 64))
    assert scan.expected_hits(P("ACGT"), 0, 3) == 0.0


def test_batch_workspace_grows_with_capacity():
    b1 = scan.Batch(["ACGT" * 10, "GATTACA"], [2, 1], 10 ** 6, capacities=[100, 100])
    b2 = scan.Batch(["ACGT" * 10, "GATTACA"], [2, 1], 10 ** 6, capacities=[100000, 100])
    assert scan.batch_workspace_bytes(10 ** 6, b2) > scan.batch_workspace_bytes(10 ** 6, b1) > 0
    assert b2.out_off.tolist() == [0, 100000]


def test_crt_route_workspace_and_arguments():
    """The transform route's workspace: 0 for m = 0 or m above 2^22, grows
    with the block (whose length is a power of two of at least 2m); bad
    arguments are refused before device work."""
    import ctypes

    ws = scan.crt_counts_workspace_bytes
    assert ws(1000, 0) == 0 and ws(10 ** 6, (1 << 22) + 1) == 0
    assert 0 < ws(1000, 10) <= ws(10 ** 6, 10) <= ws(10 ** 9, 10) < ws(10 ** 9, 1 << 21)
    assert ws(10 ** 9, 1 << 22) >= 40 * (1 << 23)
    dummy = ctypes.c_void_p(256)  # never dereferenced: the argument check fails first
    codes = scan.encode_pattern("ACGT")
    assert scan.lib().pm_crt_counts(dummy, 100, codes.ctypes.data, 0, dummy, dummy, 1 << 30, None) == -1
    assert scan.lib().pm_crt_counts(dummy, 100, codes.ctypes.data, (1 << 22) + 1, dummy, dummy, 1 << 30, None) == -5
    bad = np.array([16, 1], dtype=np.uint8)
    assert scan.lib().pm_crt_counts(dummy, 100, bad.ctypes.data, 2, dummy, dummy, 1 << 30, None) == -2
    small = scan.lib().pm_crt_counts(dummy, 100, codes.ctypes.data, 4, dummy, dummy, 16, None)
    assert small == -4


def test_batch_capacities_are_bounded():
    """Capacities summing past 2^44 hits (whose staging sizes would
    overflow 64 bits) get workspace 0 and are refused before device work."""
    import ctypes

    pats, ks, n = ["ACGT" * 10, "GATTACA"], [2, 1], 10 ** 6
    ok = scan.Batch(pats, ks, n, capacities=[1 << 43, 1 << 43])
    assert scan.batch_workspace_bytes(n, ok) > 0
    dummy = ctypes.c_void_p(256)  # never dereferenced: the argument check fails first
    for caps in ([(1 << 44), 1], [(1 << 63), 0], [(1 << 64) - 1, (1 << 64) - 1]):
        b = scan.Batch(pats, ks, n, capacities=caps)
        assert scan.batch_workspace_bytes(n, b) == 0, caps
        st = scan.lib().pm_scan_batch(dummy, n, len(b), b.codes.ctypes.data, b.m.ctypes.data, b.ks.ctypes.data,
                                      b.out_off.ctypes.data, b.capacity.ctypes.data, 0, n, dummy, dummy, dummy,
                                      dummy, dummy, 1 << 62, None, None)
        assert st == -1, caps


def test_noalloc_rejects_a_range_beyond_its_scratch_without_a_device():
    """pm_scan_noalloc checks the window range against its static scratch
    before it touches any device: a 3e9-window range is PM_ERR_WORKSPACE
    (the pointers here are never dereferenced)."""
    import ctypes

    limit = scan.noalloc_max_windows()
    assert 1 << 29 <= limit < 3_000_000_000
    codes = scan.encode_pattern("ACGTACGT")
    fake = ctypes.c_void_p(1 << 12)
    st = scan.lib().pm_scan_noalloc(fake, 3_000_000_000, codes.ctypes.data, codes.size, 2, fake, 0,
                                    scan.UINT64_MAX, fake, fake, 16, fake, None)
    assert st == -4  # PM_ERR_WORKSPACE
    assert "static scratch" in scan.lib().pm_last_error_detail().decode()
