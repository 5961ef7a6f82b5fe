"""GPU parity: libpmscan's scan against the oracle, bit-exact.

Every comparison is equality of the (position, count) lists; the path is pure
integer work, so the tolerance is zero.
"""
import random
import sys

import numpy as np
import pytest

import oracle
from conftest import golden_dict, golden_lines

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SYMBOLS = "ACGTMRWSYKVHDBN-"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_06115_amd import scan

    scan.lib()
    return scan


def gpu_hits(pm, text, pattern, k, **kw):
    say(f"  gpu scan n={text.n} m={pattern.m if hasattr(pattern, 'm') else len(pattern)} k={k} {kw}")
    pos, cnt = pm.scan(text, pattern, k, **kw)
    return pos.cpu().numpy(), cnt.cpu().numpy().astype(np.uint16)


def oracle_hits(ascii_np, pattern_str, k, threads=16, **kw):
    pos, cnt, total = oracle.scan(ascii_np, oracle.parse(pattern_str), k, threads=threads, **kw)
    assert total == pos.size
    return pos, cnt


def assert_same(got, want, label=""):
    gp, gc = got
    wp, wc = want
    if gp.size != wp.size or not np.array_equal(gp, wp) or not np.array_equal(gc, wc):
        gs = dict(zip(gp.tolist(), gc.tolist()))
        ws = dict(zip(wp.tolist(), wc.tolist()))
        only_g = sorted(set(gs) - set(ws))[:5]
        only_w = sorted(set(ws) - set(gs))[:5]
        diff = [(p, gs[p], ws[p]) for p in sorted(set(gs) & set(ws)) if gs[p] != ws[p]][:5]
        raise AssertionError(f"{label}: gpu {gp.size} hits, oracle {wp.size}; only gpu {only_g}; "
                             f"only oracle {only_w}; count diffs {diff}")


def random_text(rnd, n):
    return np.frombuffer(bytes(rnd.choice(b"ACGT") for _ in range(n)), dtype=np.uint8).copy()


def rand_pattern(rnd, m, class_frac=0.25, symbols=SYMBOLS):
    return "".join(rnd.choice("ACGT") if rnd.random() > class_frac else rnd.choice(symbols)
                   for _ in range(m))


def plant_copies(rnd, text, pattern, count, max_d):
    from oracle import reference as ref

    sets = ref.parse(pattern)
    m = len(sets)
    for _ in range(count):
        if text.size < m:
            return
        p = rnd.randrange(0, text.size - m + 1)
        for j, s in enumerate(sets):
            text[p + j] = ord(rnd.choice(sorted(s) or "ACGT"))
        for j in rnd.sample(range(m), min(m, rnd.randint(0, max_d))):
            text[p + j] = ord(rnd.choice("ACGT"))


# --- encoding -----------------------------------------------------------------

def decode_planar(buf: np.ndarray, n: int) -> np.ndarray:
    words = buf.view(np.uint32)
    hi = words[0::2]
    lo = words[1::2]
    idx = np.arange(n)
    b, i = idx // 32, idx % 32
    return (((hi[b] >> i) & 1) << 1 | ((lo[b] >> i) & 1)).astype(np.uint8)


def test_encode_text_table1(pm):
    codes = {r[0]: int(r[2]) for r in golden_lines("table1_text_codes.txt")}
    rnd = random.Random(2)
    for n in (1, 5, 31, 32, 33, 64, 1000, 4097, 100_003):
        say(f"encode n={n}")
        s = "".join(rnd.choice("ACGTacgt") for _ in range(n))
        t = pm.encode_text(np.frombuffer(s.encode(), dtype=np.uint8))
        torch.cuda.synchronize()
        t.check()
        buf = t.data.cpu().numpy()
        assert buf.size == pm.text_bytes(n)
        want = np.array([codes[c.upper()] for c in s], dtype=np.uint8)
        assert np.array_equal(decode_planar(buf, n), want)
        # everything past the text is zero
        words = buf.view(np.uint32)
        nb = (n + 31) // 32
        if n % 32:
            assert (words[2 * (nb - 1)] >> (n % 32)) == 0 and (words[2 * nb - 1] >> (n % 32)) == 0
        assert not words[2 * nb:].any()


def test_encode_text_bad_symbols(pm):
    for n, bad in ((100, [37, 80]), (5000, [4999]), (64, [0, 63]), (33, [32])):
        arr = np.frombuffer(b"A" * n, dtype=np.uint8).copy()
        for b in bad:
            arr[b] = ord("N")
        t = pm.encode_text(arr)
        torch.cuda.synchronize()
        assert int(t.bad.item()) == min(bad)
        with pytest.raises(pm.PMError):
            t.check()
    # unaligned source pointer takes the byte-wise path
    base = torch.from_numpy(np.frombuffer(b"xACGTNACGT" * 10, dtype=np.uint8).copy()).cuda()
    t = pm.encode_text(base[1:])
    torch.cuda.synchronize()
    assert int(t.bad.item()) == 4


# --- worked examples ------------------------------------------------------------

@pytest.mark.parametrize("fx", ["example_sect1_1.txt", "example_sect2_5.txt"])
def test_worked_examples(pm, fx):
    g = golden_dict(fx)
    text = np.frombuffer(g["text"][0][0].encode(), dtype=np.uint8)
    t = pm.encode_text(text)
    pat = pm.Pattern(g["pattern"][0][0])
    for k, key in ((0, "locations_k0"), (2, "locations_k2")):
        pos, cnt = gpu_hits(pm, t, pat, k)
        assert pos.tolist() == [int(x) - 1 for x in g[key][0]]
        assert_same((pos, cnt), oracle_hits(text, g["pattern"][0][0], k), fx)


# --- random parity ------------------------------------------------------------------

CASES = [
    # (m, n, k, class fraction)
    (1, 1000, 0, 0.5), (2, 5000, 1, 0.5), (5, 20000, 0, 0.3), (5, 20000, 2, 0.3),
    (17, 70001, 3, 0.25), (31, 65536, 4, 0.25), (32, 65537, 0, 0.1), (33, 100000, 5, 0.25),
    (48, 131072, 8, 0.3), (63, 99999, 6, 0.2), (64, 200000, 10, 0.2), (65, 200001, 7, 0.2),
    (100, 300000, 12, 0.2), (128, 262145, 16, 0.2), (257, 300000, 20, 0.15),
    (500, 400000, 30, 0.1), (1000, 500000, 40, 0.1), (1024, 600000, 63, 0.1),
    (2000, 700000, 64, 0.1), (300, 300000, 100, 0.1), (16, 500000, 8, 0.3), (20, 500000, 10, 0.3),
]


@pytest.mark.parametrize("m,n,k,cf", CASES)
def test_random_patterns(pm, m, n, k, cf):
    rnd = random.Random(m * 7919 + n + k)
    text = random_text(rnd, n)
    pat = rand_pattern(rnd, m, cf)
    plant_copies(rnd, text, pat, 40, k + 2)
    t = pm.encode_text(text)
    got = gpu_hits(pm, t, pm.Pattern(pat), k)
    want = oracle_hits(text, pat, k)
    assert_same(got, want, f"m={m} n={n} k={k} pattern={pat[:40]}")


def test_many_short_patterns_all_symbols(pm):
    rnd = random.Random(99)
    text = random_text(rnd, 20000)
    t = pm.encode_text(text)
    ws = pm.Workspace(t.data.device, t.n, 1 << 15)
    for trial in range(120):
        m = rnd.randint(1, 80)
        pat = rand_pattern(rnd, m, rnd.random())
        k = rnd.randint(0, m)
        plant_copies(rnd, text, pat, 0, 0)
        got = pm.scan(t, pm.Pattern(pat), k, ws=ws)
        got = (got[0].cpu().numpy(), got[1].cpu().numpy())
        assert_same(got, oracle_hits(text, pat, k), f"trial {trial} m={m} k={k} {pat}")


# --- ranges, capacity, edge cases ---------------------------------------------------

def test_window_ranges(pm):
    rnd = random.Random(5)
    text = random_text(rnd, 300000)
    pat = rand_pattern(rnd, 40, 0.3)
    plant_copies(rnd, text, pat, 200, 6)
    t = pm.encode_text(text)
    P = pm.Pattern(pat)
    for b, e in ((0, 1), (1, 2), (31, 33), (100, 70000), (65535, 65537), (131000, 10 ** 9),
                 (299960, 299961), (299961, 10 ** 9), (5, 5)):
        got = gpu_hits(pm, t, P, 6, win_begin=b, win_end=e)
        assert_same(got, oracle_hits(text, pat, 6, win_begin=b, win_end=e), f"range {b},{e}")


def test_capacity_protocol(pm):
    text = np.frombuffer(b"ACGT" * 25000, dtype=np.uint8)
    t = pm.encode_text(text)
    P = pm.Pattern("NNN")
    ws = pm.Workspace(t.data.device, t.n, 1000)
    pm.scan_async(t, P, 0, ws)
    torch.cuda.synchronize()
    assert int(ws.n_hits.item()) == 100000 - 2
    assert ws.pos[:1000].cpu().tolist() == list(range(1000))
    assert not ws.cnt[:1000].cpu().numpy().any()
    pos, cnt = pm.scan(t, P, 0, capacity=10)
    assert pos.numel() == 100000 - 2 and pos.cpu().tolist() == list(range(100000 - 2))


def test_edge_cases(pm):
    rnd = random.Random(8)
    text = random_text(rnd, 5000)
    t = pm.encode_text(text)
    small = pm.encode_text(text[:40])
    cases = [
        (small, text[:40], "ACGT" * 11, 3),                 # m > n
        (small, text[:40], "N" * 40, 0),                    # m == n
        (small, text[:40], "ACGTACGT" * 5, 40),             # m == n, k == m
        (t, text, "GATTACA", 7),                            # k == m: every window
        (t, text, "GATTACAGATTACA", 30),                    # k > m
        (t, text, "N" * 70, 0),                             # all N
        (t, text, "-" * 10, 9),                             # all '-', k < m: nothing
        (t, text, "-" * 10, 10),                            # all '-', k == m
        (t, text, "AC-GT-NN", 1),                           # dashes eat the budget
        (t, text, "AC-GT-NN", 2),
        (t, text, "A" + "N" * 200 + "C", 1),                # countable positions far apart
        (t, text, "N" * 100 + "ACGTTGCA" + "N" * 100, 2),   # filter window not at 0
        (t, text, "ACGTTGCAAC" * 10, 64),                   # k >= 64: no filter
        (t, text, "ACGTTGCAAC" * 10, 90),
        (t, text, "[AC][GT]" * 40, 20),
    ]
    for tt, raw, pat, k in cases:
        got = gpu_hits(pm, tt, pm.Pattern(pat), k)
        assert_same(got, oracle_hits(raw, pat, k), f"{pat[:30]} k={k}")


def test_errors(pm):
    t = pm.encode_text(np.frombuffer(b"ACGT" * 10, dtype=np.uint8))
    with pytest.raises(pm.PMError):
        pm.scan(t, pm.Pattern("ACGT"), 70000)
    with pytest.raises(pm.PMError):
        pm.Pattern("")


def test_workspace_reuse_across_texts(pm):
    """One workspace, consecutive scans of different lengths and ranges: the
    launch counter it carries keeps every call's output exact."""
    rnd = random.Random(21)
    big = random_text(rnd, 900000)
    pat = rand_pattern(rnd, 30, 0.3)
    plant_copies(rnd, big, pat, 300, 6)
    tb = pm.encode_text(big)
    ts = pm.encode_text(big[:50000])
    P = pm.Pattern(pat)
    ws = pm.Workspace(tb.data.device, tb.n, 1 << 12)
    for it in range(12):
        t, raw = (tb, big) if it % 3 else (ts, big[:50000])
        b = rnd.randint(0, raw.size // 2) if it % 4 == 3 else 0
        got = pm.scan(t, P, 6, win_begin=b, ws=ws)
        got = (got[0].cpu().numpy(), got[1].cpu().numpy())
        assert_same(got, oracle_hits(raw, pat, 6, win_begin=b), f"reuse {it}")


def test_deterministic_repeat(pm):
    rnd = random.Random(12)
    text = random_text(rnd, 400000)
    pat = rand_pattern(rnd, 24, 0.3)
    plant_copies(rnd, text, pat, 500, 5)
    t = pm.encode_text(text)
    a = gpu_hits(pm, t, pm.Pattern(pat), 5)
    b = gpu_hits(pm, t, pm.Pattern(pat), 5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[0].size > 100


def _periodic(rnd, n, unit, start, length):
    """A random text with `unit` repeated over [start, start + length)."""
    text = random_text(rnd, n)
    reps = np.frombuffer((unit * (length // len(unit) + 1)).encode(), dtype=np.uint8)[:length]
    text[start:start + length] = reps
    return text


@pytest.mark.parametrize("unit_len,reps,k,region", [
    (300, 2, 0, 20_000),     # m = 600: ~27 hits per tile, several lanes, wave-counted staging
    (300, 2, 5, 20_000),
    (40, 15, 2, 20_000),     # m = 600, a hit every 40 windows: > 32 per tile, the place kernel's re-scan
    (1000, 5, 3, 30_000),    # m = 5000 (157 chunks)
    (520, 1, 0, 600),        # m = 520 (17 chunks): one hit, verified by the whole wave
    (16, 32, 1, 10_000),     # m = 512 (16 chunks): verified lane by lane
])
def test_long_pattern_hit_density(pm, unit_len, reps, k, region):
    """Long patterns (the whole-wave exact counts) at controlled hit
    densities, from one hit to more than a tile can stage: periodic text
    regions make every window at a multiple of the period an exact copy."""
    rnd = random.Random(unit_len * 1000 + reps * 10 + k)
    unit = "".join(rnd.choice("ACGT") for _ in range(unit_len))
    pat = list(unit * reps)
    for j in rnd.sample(range(len(pat)), len(pat) // 10):  # classes that contain the base, and some Ns
        pat[j] = {"A": "R", "G": "R", "C": "Y", "T": "Y"}[pat[j]] if rnd.random() < 0.7 else "N"
    pat = "".join(pat)
    text = _periodic(rnd, 200_000, unit, 50_000, region + len(pat))
    t = pm.encode_text(text)
    got = gpu_hits(pm, t, pm.Pattern(pat), k)
    want = oracle_hits(text, pat, k)
    assert want[0].size >= 1
    assert_same(got, want, f"long pattern m={len(pat)} k={k}")


def test_long_pattern_weak_filter(pm):
    """A long pattern with few single-base positions and a large k: many
    survivors in many lanes, so lanes verify their own (not the whole wave)."""
    rnd = random.Random(99)
    text = random_text(rnd, 300_000)
    pat = "".join(rnd.choice("ACGT") if rnd.random() < 0.15 else rnd.choice("MRWSYKVHDBN") for _ in range(900))
    for k in (40, 120):
        plant_copies(rnd, text, pat, 5, k // 2)
        t = pm.encode_text(text)
        assert_same(gpu_hits(pm, t, pm.Pattern(pat), k), oracle_hits(text, pat, k), f"weak filter k={k}")


# --- configured workloads -------------------------------------------------------------

def test_small_workload(pm):
    """1e6 uniform bases, m = 32 (8 multi-base classes), 64 plants, k in {0, 2}."""
    from paper_1611_06115_amd import synth

    w = synth.small()
    t = pm.encode_text(w.text)
    P = pm.Pattern(w.patterns[0])
    for k in w.ks:
        got = gpu_hits(pm, t, P, k)
        assert_same(got, oracle_hits(w.text, w.patterns[0], k), f"small k={k}")
        found = dict(zip(got[0].tolist(), got[1].tolist()))
        for _, p, d in w.plants:
            if d <= k:
                assert found.get(p) == d


def test_long_m_workload(pm):
    """64e6 i.i.d. bases at GC 41%, m = 1024 and 4096, k in {0, 4, 16}."""
    from paper_1611_06115_amd import synth

    w = synth.long_m()
    t = pm.encode_text(w.text)
    for pi, pat in enumerate(w.patterns):
        P = pm.Pattern(pat)
        for k in w.ks:
            got = gpu_hits(pm, t, P, k)
            want = oracle_hits(w.text, pat, k)
            assert_same(got, want, f"long_m m={len(pat)} k={k}")
            planted = {p for q, p, d in w.plants if q == pi and d <= k}
            assert planted <= set(got[0].tolist())


def test_genome_workload_full(pm):
    """Full genome-scale scan (3.1e9 bases, m = 256, k = 4) in the launch
    configuration the benchmark times: the whole hit list equals a full
    oracle pass over every window (a few seconds on the host's cores), and
    every planted copy within the budget is reported with its distance."""
    from paper_1611_06115_amd import synth

    w = synth.genome()
    pat, k = w.patterns[0], w.ks[0]
    say(f"genome: n={w.n} m={len(pat)} k={k}")
    ascii_dev = torch.from_numpy(w.text).cuda()
    t = pm.encode_text(ascii_dev)
    torch.cuda.synchronize()
    t.check()
    del ascii_dev
    torch.cuda.empty_cache()
    pos, cnt = gpu_hits(pm, t, pm.Pattern(pat), k)
    found = dict(zip(pos.tolist(), cnt.tolist()))
    for _, p, d in w.plants:
        if d <= k:
            assert found.get(p) == d, (p, d)
    import os

    want = oracle_hits(w.text, pat, k, threads=len(os.sched_getaffinity(0)))
    assert_same((pos, cnt), want, "genome, every window")


def test_mscale_workload(pm):
    """The m-scaling workload at full size (a chromosome-2-sized Markov text,
    exact copies of m = 500, 10 000 and 100 000 cut at the sites of the
    paper's Tables 5-7): every pattern's list equals a full oracle scan and
    contains its cut site with count 0."""
    from paper_1611_06115_amd import synth

    w = synth.mscale()
    say(f"mscale: n={w.n}, {len(w.patterns)} patterns")
    t = pm.encode_text(w.text)
    for (pi, site, _), pat in zip(w.plants, w.patterns):
        got = gpu_hits(pm, t, pm.Pattern(pat), 0)
        assert_same(got, oracle_hits(w.text, pat, 0), f"mscale pattern {pi} m={len(pat)}")
        assert site in set(got[0].tolist()) and dict(zip(got[0].tolist(), got[1].tolist()))[site] == 0


def test_long_pattern_plan_reuse(pm):
    """Long patterns' plans are kept between calls: the same pattern at
    another k, and a pattern that differs only in its last position, must
    not reuse a plan built for something else."""
    rnd = random.Random(4096)
    text = random_text(rnd, 400_000)
    a = rand_pattern(rnd, 5000, 0.1, "ACGTRYN")
    b = a[:-1] + ("A" if a[-1] != "A" else "C")
    plant_copies(rnd, text, a, 3, 2)
    plant_copies(rnd, text, b, 3, 0)
    t = pm.encode_text(text)
    for pat, k in ((a, 0), (b, 0), (a, 2), (b, 3), (a, 0), (b, 0)):
        assert_same(gpu_hits(pm, t, pm.Pattern(pat), k), oracle_hits(text, pat, k), f"reuse k={k} {pat == a}")


def test_text_beyond_2_32_bases(pm):
    """A 4.4e9-base text: windows past 2^32 (one straddling it, one just after
    it, the very last one) are found with their counts by the plain and the
    batched scan, and both equal the oracle on ranges around them."""
    from paper_1611_06115_amd import synth

    n = 4_400_000_000
    rnd = random.Random(2 ** 32)
    text = synth.iid_text(n, seed=synth.SEED0 + 90)
    pat = rand_pattern(rnd, 100, 0.2, "ACGTRYN")
    sites = [(1 << 32) - 50, (1 << 32) + 12_345, n - 100]
    from oracle import reference as ref

    for p0 in sites:
        for j, cls in enumerate(ref.parse(pat)):
            text[p0 + j] = ord(rnd.choice(sorted(cls)))
    say(f"text of {n} bases, plants at {sites}")
    ascii_dev = torch.from_numpy(text).cuda()
    t = pm.encode_text(ascii_dev)
    torch.cuda.synchronize()
    t.check()
    del ascii_dev
    torch.cuda.empty_cache()
    k = 3
    plain = gpu_hits(pm, t, pm.Pattern(pat), k)
    batch = pm.scan_batch(t, [pat, "ACGTACGTACGTACGTACGTACGT"], [k, 2])[0]
    batch = (batch[0].cpu().numpy(), batch[1].cpu().numpy())
    assert_same(batch, plain, "batched vs plain")
    found = dict(zip(plain[0].tolist(), plain[1].tolist()))
    for p0 in sites:
        assert found.get(p0) == 0, p0
        b, e = max(0, p0 - 1_000_000), min(n - len(pat) + 1, p0 + 1_000_000)
        sel = (plain[0] >= b) & (plain[0] < e)
        assert_same((plain[0][sel], plain[1][sel]), oracle_hits(text, pat, k, win_begin=b, win_end=e),
                    f"range around {p0}")


def test_text_past_32_bit_offsets(pm):
    """A 17.6e9-base text, whose encoding (4.4 GB) is larger than 32-bit byte
    offsets reach: the fixed count kernel, which addresses the text that way,
    is not taken, and the genome-shaped pattern (whose plan it would take on
    a smaller text) runs through the generic kernel.  Copies planted past
    2^32 and 2^34 windows and at the end are found with count 0, the plain
    and the batched lists agree, and both equal the oracle on ranges around
    the copies."""
    from paper_1611_06115_amd import synth
    from oracle import reference as ref

    n = 17_600_000_000
    assert pm.lib().pm_text_bytes(n) > (1 << 32)
    dev = torch.device("cuda")
    say(f"text of {n} bases generated on the device")
    ascii_dev = torch.empty(n, dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.SEED0 + 91)
    lut = torch.tensor(list(b"ACGT"), dtype=torch.uint8, device=dev)
    chunk = 1 << 28
    for b in range(0, n, chunk):
        e = min(n, b + chunk)
        x = torch.randint(0, 4, (e - b,), dtype=torch.int64, device=dev, generator=gen)
        ascii_dev[b:e] = lut[x]
        del x
    pat = synth.genome_pattern()
    m, k = len(pat), 4
    rnd = random.Random(2 ** 34)
    sites = [(1 << 32) + 7, (1 << 34) + 1000, n - m - 3]
    for p0 in sites:
        copy = bytes(ord(rnd.choice(sorted(cls))) for cls in ref.parse(pat))
        ascii_dev[p0:p0 + m] = torch.frombuffer(bytearray(copy), dtype=torch.uint8).to(dev)
    t = pm.encode_text(ascii_dev)
    torch.cuda.synchronize()
    t.check()
    plain = gpu_hits(pm, t, pm.Pattern(pat), k)
    batch = pm.scan_batch(t, [pat, "ACGTACGTACGTACGTACGTACGTACGTACGT"], [k, 1])[0]
    batch = (batch[0].cpu().numpy(), batch[1].cpu().numpy())
    assert_same(batch, plain, "batched vs plain")
    found = dict(zip(plain[0].tolist(), plain[1].tolist()))
    nw = n - m + 1
    for p0 in sites:
        assert found.get(p0) == 0, p0
        b, e = max(0, p0 - 500_000), min(nw, p0 + 500_000)
        host = ascii_dev[b:e + m - 1].cpu().numpy()
        wp, wc = oracle_hits(host, pat, k)
        sel = (plain[0] >= b) & (plain[0] < e)
        assert_same((plain[0][sel], plain[1][sel]), (wp + b, wc), f"range around {p0}")
