"""Exhaustive GPU parity: every pattern of length 1 to 3 over the 16 symbols
of Table 2 (4368 patterns) against the de Bruijn text B(4, 7) (every 7-mer
once), with every budget k from 0 to m -- through pm_scan one at a time and
through one pm_scan_batch of all of them -- equal to the oracle, hit for hit."""
import itertools
import sys

import numpy as np
import pytest

import oracle
from oracle import reference as ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SYMBOLS = "ACGTMRWSYKVHDBN-"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_06115_amd import scan

    text = np.frombuffer(ref.de_bruijn(7).encode(), dtype=np.uint8).copy()
    assert text.size == 4 ** 7 + 6
    t = scan.encode_text(text, device=torch.device("cuda:0"))
    torch.cuda.synchronize()
    t.check()
    items = [("".join(p), k) for m in (1, 2, 3) for p in itertools.product(SYMBOLS, repeat=m) for k in range(m + 1)]
    assert len({p for p, _ in items}) == 4368
    want = {}
    for p, k in items:
        pos, cnt, total = oracle.scan(text, oracle.parse(p), k, threads=4)
        want[(p, k)] = (pos, cnt)
    return scan, t, items, want


def test_exhaustive_short_patterns_plain(setup):
    scan, t, items, want = setup
    say(f"  {len(items)} (pattern, k) scans over {t.n} bases")
    ws = scan.Workspace(t.data.device, t.n, capacity=t.n)
    for p, k in items:
        pos, cnt = scan.scan(t, scan.Pattern(p), k, ws=ws)
        wp, wc = want[(p, k)]
        assert np.array_equal(pos.cpu().numpy(), wp) and np.array_equal(cnt.cpu().numpy(), wc), (p, k)


def test_exhaustive_short_patterns_one_batch(setup):
    scan, t, items, want = setup
    say(f"  one batch of {len(items)} (pattern, k)")
    got = scan.scan_batch(t, [p for p, _ in items], [k for _, k in items])
    for (p, k), g in zip(items, got):
        wp, wc = want[(p, k)]
        assert np.array_equal(g[0].cpu().numpy(), wp) and np.array_equal(g[1].cpu().numpy(), wc), (p, k)
