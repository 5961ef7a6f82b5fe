"""GPU tests of the scan of a text kept in host memory (chunks with an m-1
overlap, Sect. 2.6): its lists equal the resident scan's and the oracle's,
bit for bit, whatever the chunk size, including hits that straddle chunk
boundaries."""
import random
import sys

import numpy as np
import pytest

from test_gpu_parity import assert_same, oracle_hits, rand_pattern, random_text

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


def plant_at(rnd, text, pattern, p0):
    from oracle import reference as ref

    for j, s in enumerate(ref.parse(pattern)):
        text[p0 + j] = ord(rnd.choice(sorted(s) or "ACGT"))


def as_np(res):
    return res[0].cpu().numpy(), res[1].cpu().numpy()


@pytest.mark.parametrize("m,k", [(33, 0), (300, 3), (2000, 8)])
def test_host_scan_equals_resident_and_oracle(pm, m, k):
    rnd = random.Random(m * 31 + k)
    n = 3_000_000
    text = random_text(rnd, n)
    pat = rand_pattern(rnd, m, 0.2, "ACGTRYSWN")
    chunk = 400_000
    # copies straddling chunk boundaries, starting on them, and ending on them
    for c in range(1, n // chunk):
        for p0 in (c * chunk - m // 2, c * chunk, c * chunk - m + 1):
            if 0 <= p0 <= n - m:
                plant_at(rnd, text, pat, p0)
    t = pm.encode_text(text)
    resident = as_np(pm.scan(t, pm.Pattern(pat), k))
    assert_same(resident, oracle_hits(text, pat, k), f"resident m={m} k={k}")
    assert resident[0].size >= 3
    for cb in (chunk, 999_983, 1_000, 10 ** 9):
        if cb < m // 4:
            continue
        say(f"host scan m={m} k={k} chunk={cb}")
        got = as_np(pm.scan_host(text, pm.Pattern(pat), k, chunk_bases=cb))
        assert_same(got, resident, f"host chunk={cb} m={m} k={k}")


def test_host_scan_pinned_capacity_and_small_chunks(pm):
    """Pinned host memory, an output buffer far too small (the re-run), and
    chunks shorter than the pattern."""
    rnd = random.Random(7)
    n = 1_000_000
    arr = random_text(rnd, n)
    pat = "ACGTNNACGT"
    for p0 in rnd.sample(range(n - 10), 300):
        plant_at(rnd, arr, pat, p0)
    pinned = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    pinned.numpy()[:] = arr
    t = pm.encode_text(arr)
    resident = as_np(pm.scan(t, pm.Pattern(pat), 1))
    assert resident[0].size > 300
    got = as_np(pm.scan_host(pinned, pm.Pattern(pat), 1, chunk_bases=65_536, capacity=5))
    assert_same(got, resident, "pinned, capacity 5")
    long_pat = rand_pattern(rnd, 3000, 0.1, "ACGTN")
    plant_at(rnd, arr, long_pat, 500_000)
    pinned.numpy()[:] = arr
    t = pm.encode_text(arr)
    got = as_np(pm.scan_host(pinned, pm.Pattern(long_pat), 2, chunk_bases=1_000))
    assert_same(got, as_np(pm.scan(t, pm.Pattern(long_pat), 2)), "chunks of 1000 windows, m = 3000")
    assert 500_000 in set(got[0].tolist())


def test_host_scan_errors_and_degenerate(pm):
    rnd = random.Random(8)
    text = random_text(rnd, 200_000)
    text[150_001] = ord("N")  # in the second chunk of 100 000 windows
    with pytest.raises(pm.PMError) as e:
        pm.scan_host(text, pm.Pattern("ACGT"), 0, chunk_bases=100_000)
    assert e.value.status == -2 and "150001" in str(e.value)
    ok = random_text(rnd, 1000)
    pos, cnt = pm.scan_host(ok, pm.Pattern("A" * 2000), 0)  # m > n: no windows
    assert pos.numel() == 0
    pos, cnt = pm.scan_host(ok, pm.Pattern("N" * 1000), 0, chunk_bases=7)  # m = n: one window
    assert pos.cpu().tolist() == [0] and cnt.cpu().tolist() == [0]
