"""FASTA input on the GPU: pm_scan_fasta equals the oracle's FASTA reading
(records separate, lower case folded, a window covering an unknown base or
crossing records has no count), hit for hit, on the hand-worked fixture and
on synthetic assemblies whose N runs and record boundaries straddle the
scan's tiles (8192 windows)."""
import random
import sys

import numpy as np
import pytest

import oracle
from test_host_fasta import golden_fasta

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


def assembly(seed, n_records, rec_len, n_runs, width=60):
    """Records of i.i.d. bases (GC 41%), a quarter soft-masked (lower case),
    with runs of N of 1 to 20 000 placed at seeded offsets, some across tile
    boundaries (multiples of 8192), and a few other IUPAC letters."""
    rnd = random.Random(seed)
    rng = np.random.default_rng(seed)
    lines = []
    for r in range(n_records):
        n = rec_len if r % 2 == 0 else rec_len // 3 + r
        seq = np.array(list(b"ACGT"), dtype=np.uint8)[rng.choice(4, size=n, p=[.295, .205, .205, .295])]
        for _ in range(n_runs):
            if rnd.random() < 0.5:
                start = max(0, (rnd.randrange(1, max(2, n // 8192 + 1)) * 8192) - rnd.randint(0, 300))
            else:
                start = rnd.randrange(0, max(1, n))
            seq[start:start + rnd.choice([1, 2, 5, 37, 300, 20_000])] = ord("N")
        for _ in range(3):
            seq[rnd.randrange(0, max(1, n))] = ord(rnd.choice("RYKMSW"))
        for _ in range(n // 4000 + 1):  # soft-masked stretches
            s = rnd.randrange(0, max(1, n))
            seq[s:s + 1000] = np.char.lower(seq[s:s + 1000].view("S1")).view(np.uint8)
        text = seq.tobytes().decode()
        lines.append(f">chr{r} synthetic record {r}")
        lines += [text[i:i + width] for i in range(0, len(text), width)]
    return "\n".join(lines) + "\n"


def gpu_fasta_hits(pm, fa_text, pattern, k, capacity=1 << 16):
    fa = pm.Fasta(fa_text)
    t = fa.encode(device=torch.device("cuda:0"))
    torch.cuda.synchronize()
    t.check()
    pos, cnt = pm.scan_fasta(fa, t, pattern, k, capacity=capacity)
    return pos.cpu().numpy(), cnt.cpu().numpy()


def test_fasta_golden_fixture_on_gpu(pm):
    fa_text, queries = golden_fasta()
    for p, k, want in queries:
        pos, cnt = gpu_fasta_hits(pm, fa_text, p, k)
        assert list(zip(pos.tolist(), cnt.tolist())) == want, p


@pytest.mark.parametrize("seed,m,k", [(1, 12, 2), (2, 40, 4), (3, 300, 20), (4, 3, 1)])
def test_fasta_assembly_equals_oracle(pm, seed, m, k):
    fa_text = assembly(seed, n_records=5, rec_len=200_000, n_runs=12)
    rnd = random.Random(seed)
    # a pattern cut from one record (so that it occurs), with classes
    from oracle import reference as ref

    recs = [seq for _, seq in ref.fasta_records(fa_text) if len(seq) > m]
    while True:
        seq = rnd.choice(recs)
        s = rnd.randrange(0, len(seq) - m)
        if all(c in "ACGT" for c in seq[s:s + m]):
            break
    # a fifth of the positions become a class holding the base
    holding = {b: sorted(x for x, mem in ref.IUPAC.items() if b in mem and len(mem) > 1) for b in "ACGT"}
    pat = "".join(c if rnd.random() > 0.2 else rnd.choice(holding[c]) for c in seq[s:s + m])
    say(f"  fasta assembly seed={seed} m={m} k={k}")
    got = gpu_fasta_hits(pm, fa_text, pat, k)
    want = oracle.fasta_scan(fa_text.encode(), pat, k, threads=8)
    assert want[0].size > 0
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_fasta_capacity_rerun_and_short_records(pm):
    """More hits than the first buffer (the binding re-runs with an exact
    one), and records shorter than the pattern."""
    fa_text = ">a\nAC\n>b\n" + "ACGT" * 5000 + "\n>c\nNNNN\n>d\nacgtacgtNacgt\n"
    pos, cnt = gpu_fasta_hits(pm, fa_text, "ACGT", 1, capacity=7)
    want = oracle.fasta_scan(fa_text.encode(), "ACGT", 1)
    assert np.array_equal(pos, want[0]) and np.array_equal(cnt, want[1]) and pos.size > 5000
