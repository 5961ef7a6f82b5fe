"""GPU tests of the Linhart-Shamir transform route (Sect. 1.3, eqs. 1-3):
every window's mismatch count equals the oracle's full count, bit for bit,
across one-block and many-block texts (windows on both sides of every block
boundary), m from 1 to 5000, classes of every kind, '-' and 'N'; and the
windows it counts at most k are exactly the hits of the early-stop scan."""
import random
import sys

import numpy as np
import pytest

from test_gpu_parity import oracle_hits, plant_copies, rand_pattern, random_text

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SYM = "ACGTMRWSYKVHDBN-"


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


def oracle_counts(text, pattern, lo=0, hi=None):
    """The oracle's full counts of windows [lo, hi)."""
    import oracle

    sets = oracle.parse(pattern)
    m = len(sets)
    hi = text.size - m + 1 if hi is None else hi
    return oracle.counts(text[lo:hi + m - 1], sets).astype(np.int64)


def test_crt_worked_example(pm):
    """The Sect. 1.1 example (a, b, c relabelled A, C, G): counts of the six
    windows, exact at the paper's location 5 (position 4)."""
    text = np.frombuffer(b"AGGACCGGCA", dtype=np.uint8).copy()
    got = pm.crt_counts(pm.encode_text(text), "C[ACG]GG[CG]").cpu().numpy()
    assert got.tolist() == oracle_counts(text, "C[ACG]GG[CG]").tolist()
    assert got.tolist()[4] == 0 and sorted(np.flatnonzero(got <= 2).tolist()) == [0, 3, 4, 5]


@pytest.mark.parametrize("n,m,density,seed", [
    (1, 1, 0.0, 1), (7, 7, 0.5, 2), (1000, 33, 0.3, 3), (70_000, 500, 0.2, 4),
    (50_000, 3000, 0.25, 5), (20_000, 1, 0.5, 6), (5_000, 6000, 0.1, 7)])
def test_crt_counts_equal_oracle(pm, n, m, density, seed):
    rnd = random.Random(seed)
    text = random_text(rnd, n)
    pat = rand_pattern(rnd, m, density, SYM)
    say(f"crt counts n={n} m={m}")
    got = pm.crt_counts(pm.encode_text(text), pat).cpu().numpy().astype(np.int64)
    want = oracle_counts(text, pat) if m <= n else np.zeros(0, dtype=np.int64)
    assert got.shape == want.shape and np.array_equal(got, want)


@pytest.mark.parametrize("m", [64, 2500])
def test_crt_counts_across_blocks(pm, m):
    """A text of several transform blocks (2^20 bases each, overlapping by
    m-1): the windows on both sides of every boundary and a seeded sample
    equal the oracle's; all-'N' and all-'-' patterns give 0 and m."""
    rnd = random.Random(m)
    n = 3_300_000
    text = random_text(rnd, n)
    pat = rand_pattern(rnd, m, 0.3, SYM)
    t = pm.encode_text(text)
    say(f"crt blocks n={n} m={m}")
    got = pm.crt_counts(t, pat).cpu().numpy().astype(np.int64)
    nw = n - m + 1
    assert got.size == nw
    per = (1 << 20) - m + 1  # windows per block
    for b in range(1, nw // per + 1):
        lo, hi = max(0, b * per - 300), min(nw, b * per + 300)
        assert np.array_equal(got[lo:hi], oracle_counts(text, pat, lo, hi)), f"boundary {b}"
    for lo in rnd.sample(range(nw - 200), 5):
        assert np.array_equal(got[lo:lo + 200], oracle_counts(text, pat, lo, lo + 200)), f"sample {lo}"
    assert np.array_equal(got[-200:], oracle_counts(text, pat, nw - 200, nw))
    assert not pm.crt_counts(t, "N" * m).cpu().numpy().any()
    assert (pm.crt_counts(t, "-" * m).cpu().numpy() == m).all()


@pytest.mark.parametrize("m,k", [(40, 3), (700, 30)])
def test_crt_hits_equal_scan(pm, m, k):
    """Windows counted at most k by the transform route are the early-stop
    scan's hits, with the same counts (and the oracle's)."""
    rnd = random.Random(m * 7 + k)
    text = random_text(rnd, 400_000)
    pat = rand_pattern(rnd, m, 0.3, SYM)
    plant_copies(rnd, text, pat, 40, k)
    t = pm.encode_text(text)
    c = pm.crt_counts(t, pat).cpu().numpy()
    sel = np.flatnonzero(c <= k)
    pos, cnt = pm.scan(t, pm.Pattern(pat), k)
    assert sel.size >= 20
    assert np.array_equal(sel, pos.cpu().numpy()) and np.array_equal(c[sel], cnt.cpu().numpy())
    wp, wc = oracle_hits(text, pat, k)
    assert np.array_equal(sel, wp) and np.array_equal(c[sel], wc)


def test_crt_beyond_2_32_windows(pm):
    """A 4.4e9-base text (windows past 2^31 and 2^32): the route's counts at
    most k are the early-stop scan's hits with the same counts, found chunk
    by chunk (no single selection over more than 2^28 windows), and its
    counts on ranges straddling 2^31, 2^32, the transform blocks next to
    them and the text's end equal the oracle's."""
    from oracle import reference as ref

    from paper_1611_06115_amd import synth

    n = 4_400_000_000
    rnd = random.Random(2 ** 31)
    text = synth.iid_text(n, seed=synth.SEED0 + 91)
    pat = rand_pattern(rnd, 100, 0.2, "ACGTRYN")
    m, k = len(pat), 3
    sites = [(1 << 31) - 40, (1 << 32) - 60, (1 << 32) + 50, n - m - 5]  # disjoint copies
    for p0 in sites:
        for j, cls in enumerate(ref.parse(pat)):
            text[p0 + j] = ord(rnd.choice(sorted(cls)))
    say(f"crt beyond 2^32: n={n} m={m} k={k} plants {sites}")
    ascii_dev = torch.from_numpy(text).cuda()
    t = pm.encode_text(ascii_dev)
    torch.cuda.synchronize()
    t.check()
    del ascii_dev
    torch.cuda.empty_cache()
    c = pm.crt_counts(t, pat)
    nw = n - m + 1
    assert c.numel() == nw
    chunk = 1 << 28
    sel = torch.cat([torch.nonzero(c[lo:min(nw, lo + chunk)] <= k).flatten() + lo for lo in range(0, nw, chunk)])
    pos, cnt = pm.scan(t, pm.Pattern(pat), k)
    say(f"  {sel.numel()} windows at most {k}, scan {pos.numel()} hits")
    assert torch.equal(sel, pos) and torch.equal(c[sel], cnt.to(torch.int32))
    found = dict(zip(pos.cpu().tolist(), cnt.cpu().tolist()))
    assert all(found.get(p0) == 0 for p0 in sites)
    per = (1 << 20) - m + 1  # windows per transform block
    ranges = [((1 << 31) - 500, (1 << 31) + 500), ((1 << 32) - 500, (1 << 32) + 500), (nw - 300, nw)]
    for x in (1 << 31, 1 << 32):
        b = x // per
        ranges += [(b * per - 300, b * per + 300), ((b + 1) * per - 300, (b + 1) * per + 300)]
    for lo, hi in ranges:
        got = c[lo:hi].cpu().numpy().astype(np.int64)
        assert np.array_equal(got, oracle_counts(text, pat, lo, hi)), (lo, hi)
