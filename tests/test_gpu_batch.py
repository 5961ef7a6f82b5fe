"""GPU parity of the batched scan: every pattern's list equals the oracle's and
the plain single-pattern kernel's, bit for bit."""
import random
import sys

import numpy as np
import pytest

import oracle
from test_gpu_parity import assert_same, oracle_hits, plant_copies, rand_pattern, random_text

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def make_batch(rnd, text, count, m_lo, m_hi, k_hi, plant=True):
    pats, ks = [], []
    for _ in range(count):
        m = rnd.randint(m_lo, m_hi)
        pat = rand_pattern(rnd, m, rnd.random() * 0.4)
        k = rnd.randint(0, min(k_hi, m))
        if plant:
            plant_copies(rnd, text, pat, 3, k + 1)
        pats.append(pat)
        ks.append(k)
    return pats, ks


def check_batch(pm, t, text, pats, ks, res, label):
    for i, (pat, k) in enumerate(zip(pats, ks)):
        got = (res[i][0].cpu().numpy(), res[i][1].cpu().numpy())
        assert_same(got, oracle_hits(text, pat, k), f"{label} pattern {i} m={len(pat)} k={k}")


@pytest.mark.parametrize("group,sub,lane_words", [(4, 0, 6), (1, 3, 4), (3, 7, 6), (16, 1, 4), (5, 40, 6)])
def test_batch_matches_oracle(pm, group, sub, lane_words):
    rnd = random.Random(group * 100 + sub)
    text = random_text(rnd, 400_003)
    pats, ks = make_batch(rnd, text, 40, 1, 300, 12)
    t = pm.encode_text(text)
    cfg = pm.BatchConfig(group, sub, lane_words, 0)
    say(f"batch group={group} sub={sub} R={lane_words}")
    res = pm.scan_batch(t, pats, ks, config=cfg)
    check_batch(pm, t, text, pats, ks, res, f"g{group} s{sub}")


@pytest.mark.parametrize("group,sub,lane_words", [(8, 0, 4), (1, 4096, 6)])
def test_batch_many_sub_ranges(pm, group, sub, lane_words):
    """A few patterns over a 40e6-base text: the automatic choice (and an
    explicit 4096) cuts every group into 4096 sub-ranges, which the gather
    step's offset scan concatenates; lists equal the plain kernel's, and
    every planted copy is found."""
    from paper_1611_06115_amd import synth

    rnd = random.Random(4096 + group)
    text = synth.iid_text(40_000_000, seed=synth.SEED0 + 80 + group)
    no_gap = "ACGTMRWSYKVHDBN"  # every position of these patterns has a base that matches it
    pats = [rand_pattern(rnd, 24, 0.1, no_gap), "GATTACAGATTACA", rand_pattern(rnd, 200, 0.2, no_gap), "ACGTNNACGT"]
    ks = [1, 2, 12, 0]
    from oracle import reference as ref

    # exact copies (a base of each position's class), one per disjoint
    # 250 kb slot so that no copy overwrites another
    planted = []
    slot = len(text) // (40 * len(pats))
    for i, p in enumerate(pats):
        sets = ref.parse(p)
        for c in range(40):
            p0 = (i * 40 + c) * slot + rnd.randrange(0, slot - len(sets))
            for j, s in enumerate(sets):
                text[p0 + j] = ord(rnd.choice(sorted(s)))
            planted.append((i, p0))
    t = pm.encode_text(text)
    cfg = pm.BatchConfig(group, sub, lane_words, 0)
    say(f"batch many sub-ranges group={group} sub={sub} R={lane_words} n={t.n}")
    res = pm.scan_batch(t, pats, ks, config=cfg, rerun=False)
    for i, (p, k) in enumerate(zip(pats, ks)):
        assert res[i] is not None, f"pattern {i} overflowed its staging"
        got = (res[i][0].cpu().numpy(), res[i][1].cpu().numpy())
        plain = pm.scan(t, pm.Pattern(p), k)
        assert_same(got, (plain[0].cpu().numpy(), plain[1].cpu().numpy()), f"sub-ranges pattern {i}")
    found = {(i, int(x)) for i, r in enumerate(res) for x in r[0].cpu().numpy().tolist()}
    for i, p0 in planted:
        assert (i, p0) in found


def test_batch_deep_counters_and_edge_patterns(pm):
    """k up to 60 (5 and 6 counter levels, the second kernel), no-filter
    patterns (k >= 64), patterns longer than the text, all N / all '-'."""
    rnd = random.Random(77)
    text = random_text(rnd, 200_000)
    pats = ["ACGTACGTAC" * 3, "N" * 40, "-" * 5, "ACGT" * 60, "A" * 300_000, "GATTACA",
            rand_pattern(rnd, 120, 0.2), rand_pattern(rnd, 90, 0.1), rand_pattern(rnd, 200, 0.1)]
    ks = [3, 0, 5, 30, 2, 7, 20, 40, 64]
    for p, k in zip(pats, ks):
        plant_copies(rnd, text, p, 2, k)
    t = pm.encode_text(text)
    res = pm.scan_batch(t, pats, ks)
    check_batch(pm, t, text, pats, ks, res, "edge")


def test_batch_overflow_rerun(pm):
    """Capacities far too small: statuses flag the patterns and the wrapper
    re-scans them alone; results are still exact."""
    rnd = random.Random(5)
    text = random_text(rnd, 300_000)
    pats = ["NNNN", "AC", rand_pattern(rnd, 12, 0.5), rand_pattern(rnd, 40, 0.2)]
    ks = [0, 1, 4, 6]
    t = pm.encode_text(text)
    batch = pm.Batch(pats, ks, t.n, capacities=[10, 10, 10, 10])
    dev = t.data.device
    pos = torch.empty(40, dtype=torch.int64, device=dev)
    cnt = torch.empty(40, dtype=torch.uint16, device=dev)
    n_hits = torch.zeros(4, dtype=torch.int64, device=dev)
    status = torch.zeros(4, dtype=torch.int32, device=dev)
    ws = torch.empty(pm.batch_workspace_bytes(t.n, batch), dtype=torch.uint8, device=dev)
    pm.scan_batch_async(t, batch, pos, cnt, n_hits, status, ws)
    torch.cuda.synchronize()
    totals = [oracle_hits(text, p, k)[0].size for p, k in zip(pats, ks)]
    assert n_hits.cpu().tolist() == totals
    assert status.cpu().tolist() == [1 if c > 10 else 0 for c in totals]
    res = pm.scan_batch(t, batch, None)
    check_batch(pm, t, text, pats, ks, res, "overflow")


def test_batch_window_range_and_plain_kernel(pm):
    """A window sub-range of the batch equals the plain kernel on that range."""
    rnd = random.Random(6)
    text = random_text(rnd, 500_000)
    pats, ks = make_batch(rnd, text, 24, 10, 200, 8)
    t = pm.encode_text(text)
    batch = pm.Batch(pats, ks, t.n)
    dev = t.data.device
    pos = torch.empty(batch.total_capacity, dtype=torch.int64, device=dev)
    cnt = torch.empty(batch.total_capacity, dtype=torch.uint16, device=dev)
    n_hits = torch.zeros(len(batch), dtype=torch.int64, device=dev)
    status = torch.zeros(len(batch), dtype=torch.int32, device=dev)
    ws = torch.empty(pm.batch_workspace_bytes(t.n, batch), dtype=torch.uint8, device=dev)
    for b, e in ((0, 250_000), (123_457, 400_001), (499_000, 10 ** 9)):
        pm.scan_batch_async(t, batch, pos, cnt, n_hits, status, ws, win_begin=b, win_end=e)
        torch.cuda.synchronize()
        nh, st = n_hits.cpu().tolist(), status.cpu().tolist()
        for i, (pat, k) in enumerate(zip(pats, ks)):
            assert st[i] == 0
            o = int(batch.out_off[i])
            got = (pos[o:o + nh[i]].cpu().numpy(), cnt[o:o + nh[i]].cpu().numpy())
            plain = pm.scan(t, pm.Pattern(pat), k, win_begin=b, win_end=e)
            assert_same(got, (plain[0].cpu().numpy(), plain[1].cpu().numpy()), f"range {b},{e} plain {i}")
            assert_same(got, oracle_hits(text, pat, k, win_begin=b, win_end=e), f"range {b},{e} oracle {i}")


def test_batched_workload_sample(pm):
    """The batched workload's shape (m ~ U{16..2048}, class density up to 30%,
    k ~ U{0..8}, two planted copies per pattern) on a 16e6-base text with 256
    patterns: every list equals the oracle's."""
    from paper_1611_06115_amd import synth

    w = synth.batched(n=16_000_000, count=256)
    t = pm.encode_text(w.text)
    res = pm.scan_batch(t, w.patterns, w.ks)
    for i, (pat, k) in enumerate(zip(w.patterns, w.ks)):
        got = (res[i][0].cpu().numpy(), res[i][1].cpu().numpy())
        assert_same(got, oracle_hits(w.text, pat, k), f"batched sample pattern {i}")
    found = {(i, int(p)) for i, r in enumerate(res) for p in r[0].cpu().tolist()}
    for pi, p, d in w.plants:
        assert (pi, p) in found


def test_batched_workload_full(pm):
    """The batched workload at full size (256e6 bases, 4096 patterns) in the
    launch shape of the committed counter run the benchmark times (group 8,
    64 sub-ranges, 4 lane words) and in the automatic shape: every planted
    copy is found, 48 seeded patterns' lists equal the plain kernel's, and
    on a seeded window range of each the oracle's."""
    from paper_1611_06115_amd import synth

    w = synth.batched()
    say(f"batched full: n={w.n} patterns={len(w.patterns)}")
    ascii_dev = torch.from_numpy(w.text).cuda()
    t = pm.encode_text(ascii_dev)
    torch.cuda.synchronize()
    t.check()
    del ascii_dev
    torch.cuda.empty_cache()
    batch = pm.Batch(w.patterns, w.ks, t.n)
    rnd = random.Random(48)
    sample = sorted(rnd.sample(range(len(w.patterns)), 48))
    ranges = {i: rnd.randrange(0, t.n - len(w.patterns[i]) + 1 - 500_000) for i in sample}
    plants = {}
    for pi, p, d in w.plants:
        plants.setdefault(pi, []).append(p)
    for cfg in (pm.BatchConfig(8, 64, 4, 0), pm.BatchConfig(0, 0, 0, 0)):
        say(f"  shape group={cfg.group_size} sub={cfg.sub_ranges} R={cfg.lane_words}")
        res = pm.scan_batch(t, batch, None, config=cfg)
        for pi, ps in plants.items():
            got = res[pi][0].cpu().numpy()
            assert np.isin(np.array(ps, dtype=np.int64), got).all(), f"pattern {pi} plants {ps}"
        for i in sample:
            pat, k = w.patterns[i], w.ks[i]
            got = (res[i][0].cpu().numpy(), res[i][1].cpu().numpy())
            plain = pm.scan(t, pm.Pattern(pat), k)
            assert_same(got, (plain[0].cpu().numpy(), plain[1].cpu().numpy()), f"full batch pattern {i} vs plain")
            b = ranges[i]
            want = oracle_hits(w.text, pat, k, win_begin=b, win_end=b + 500_000)
            sel = (got[0] >= b) & (got[0] < b + 500_000)
            assert_same((got[0][sel], got[1][sel]), want, f"full batch pattern {i} range {b} vs oracle")
        say(f"  {len(sample)} sampled patterns equal to the plain kernel and the oracle")
