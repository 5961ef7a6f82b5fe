"""pm_scan_noalloc (the entry point with the library's static scratch instead
of a caller workspace) against pm_scan, bit-exact, through the C ABI.

Two calls in a row on the same device, the second on a smaller input, so
that the second runs over scratch that still holds the first call's
contents.
"""
import sys

import numpy as np
import pytest

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


def noalloc_hits(pm, text, pat, k, capacity, win_begin=0, win_end=None):
    dev = text.data.device
    pos = torch.full((capacity,), -7, dtype=torch.int64, device=dev)
    cnt = torch.zeros(capacity, dtype=torch.uint16, device=dev)
    n_hits = torch.full((1,), -7, dtype=torch.int64, device=dev)
    pm.scan_noalloc_async(text, pat, k, pos, cnt, n_hits, win_begin, win_end)
    torch.cuda.synchronize(dev)
    total = int(n_hits.item())
    kept = min(total, capacity)
    return total, pos[:kept].cpu().numpy(), cnt[:kept].cpu().numpy()


def workspace_hits(pm, text, pat, k, win_begin=0, win_end=None):
    pos, cnt = pm.scan(text, pat, k, win_begin=win_begin, win_end=win_end)
    return pos.cpu().numpy(), cnt.cpu().numpy()


def test_noalloc_equals_workspace_scan_on_two_calls(pm):
    from paper_1611_06115_amd import synth

    dev = torch.device("cuda:0")
    big = synth.small(n=3_000_000, n_plants=64)
    small = synth.small(n=120_000, n_plants=8)
    cases = [(big, 2, None), (small, 2, None), (big, 0, (1_000_003, 2_500_017)), (small, 3, (5, 70_001))]
    for w, k, rng in cases:
        text = pm.encode_text(w.text, device=dev)
        torch.cuda.synchronize(dev)
        text.check()
        pat = pm.Pattern(w.patterns[0])
        wb, we = rng if rng else (0, None)
        say(f"  noalloc n={w.n} m={pat.m} k={k} range={rng}")
        want_pos, want_cnt = workspace_hits(pm, text, pat, k, wb, we)
        total, pos, cnt = noalloc_hits(pm, text, pat, k, max(want_pos.size, 1) + 16, wb, we)
        assert total == want_pos.size
        assert np.array_equal(pos, want_pos) and np.array_equal(cnt, want_cnt)
        assert want_pos.size > 0
        # a capacity below the total: the lowest positions, and the true total
        if want_pos.size > 2:
            cap = want_pos.size // 2
            total2, pos2, cnt2 = noalloc_hits(pm, text, pat, k, cap, wb, we)
            assert total2 == want_pos.size
            assert np.array_equal(pos2, want_pos[:cap]) and np.array_equal(cnt2, want_cnt[:cap])


def test_noalloc_genome_range_equals_workspace_scan(pm):
    """The genome workload's pattern (m = 256, k = 4) over a range of the
    largest size one call takes, on a 40e6-base slice of the Markov text."""
    from paper_1611_06115_amd import synth

    dev = torch.device("cuda:0")
    w = synth.genome(n=40_000_000)
    text = pm.encode_text(torch.from_numpy(w.text).to(dev))
    torch.cuda.synchronize(dev)
    text.check()
    pat = pm.Pattern(w.patterns[0])
    k = w.ks[0]
    say(f"  noalloc genome slice n={w.n} m={pat.m} k={k}")
    want_pos, want_cnt = workspace_hits(pm, text, pat, k)
    total, pos, cnt = noalloc_hits(pm, text, pat, k, max(want_pos.size, 1) + 16)
    assert total == want_pos.size and want_pos.size > 0
    assert np.array_equal(pos, want_pos) and np.array_equal(cnt, want_cnt)


def test_noalloc_limit_and_a_tiny_text(pm):
    """The per-call window limit is the documented one, and a 256-base text
    (a single, partial tile) is scanned exactly."""
    limit = pm.noalloc_max_windows()
    assert limit >= 1 << 29
    dev = torch.device("cuda:0")
    w_text = np.frombuffer(b"ACGT" * 64, dtype=np.uint8)
    text = pm.encode_text(w_text, device=dev)
    torch.cuda.synchronize(dev)
    pat = pm.Pattern("ACGTACGT")
    # a range within the text is fine; the limit is checked on the clipped range
    total, pos, cnt = noalloc_hits(pm, text, pat, 0, 128)
    assert total == 63 and np.array_equal(pos, np.arange(0, 256 - 7, 4))
