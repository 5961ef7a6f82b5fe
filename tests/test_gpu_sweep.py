"""A seeded random sweep over every entry point: the plain scan (whole text
and a random window range), the scan from host memory (random chunk size),
the batched scan (random launch shape) and the query server (random chunk
count) all equal the oracle, bit for bit, on random texts, pattern lengths
from 1 to 6000, class densities up to 50% (all symbols, '-' included) and k
from 0 to 70."""
import os
import random
import sys

import numpy as np
import pytest

from test_gpu_parity import assert_same, oracle_hits, plant_copies, rand_pattern, random_text

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
    from paper_1611_06115_amd import scan, server

    scan.lib()
    return scan, server


def as_np(r):
    return r[0].cpu().numpy(), r[1].cpu().numpy()


# PM_SWEEP_CASES widens the sweep (a longer run of 400 cases passed as well)
@pytest.mark.parametrize("case", range(int(os.environ.get("PM_SWEEP_CASES", "40"))))
def test_random_sweep(pm, case):
    scan, server = pm
    rnd = random.Random(1_000_003 * (case + 1))
    n = rnd.choice([1000, 20_000, 120_000, 300_000])
    text = random_text(rnd, n)
    pats, ks = [], []
    for _ in range(rnd.randint(1, 8)):
        m = rnd.choice([rnd.randint(1, 40), rnd.randint(40, 700), rnd.randint(500, 6000)])
        pat = rand_pattern(rnd, m, rnd.random() * 0.5, SYM)
        k = rnd.choice([0, rnd.randint(0, 8), rnd.randint(0, 70)])
        plant_copies(rnd, text, pat, rnd.randint(0, 20), rnd.randint(0, k + 2))
        pats.append(pat)
        ks.append(k)
    say(f"sweep case {case}: n={n} patterns {[(len(p), k) for p, k in zip(pats, ks)]}")
    t = scan.encode_text(text)
    want = [oracle_hits(text, p, k) for p, k in zip(pats, ks)]
    for i, (p, k) in enumerate(zip(pats, ks)):
        assert_same(as_np(scan.scan(t, scan.Pattern(p), k)), want[i], f"plain {i}")
        b, e = sorted(rnd.randrange(0, n + 5) for _ in range(2))
        assert_same(as_np(scan.scan(t, scan.Pattern(p), k, win_begin=b, win_end=e)),
                    oracle_hits(text, p, k, win_begin=b, win_end=e), f"range {i} [{b},{e})")
        cb = max(rnd.choice([1, 7, 1000, 65_536, 10 ** 9]), n // 500 + 1)
        assert_same(as_np(scan.scan_host(text, scan.Pattern(p), k, chunk_bases=cb)), want[i], f"host {i} chunk {cb}")
    cfg = scan.BatchConfig(rnd.choice([0, 1, 3, 8, 16]), rnd.choice([0, 1, 5, 64, 4096]), rnd.choice([0, 4, 6]), 0)
    res = scan.scan_batch(t, pats, ks, config=cfg)
    for i in range(len(pats)):
        assert_same(as_np(res[i]), want[i], f"batch {i} shape {cfg.group_size}/{cfg.sub_ranges}/{cfg.lane_words}")
    if n >= 20_000:
        with server.Server(t, 64 << 20, server.ServerConfig(chunks=rnd.choice([1, 2, 5, 8]))) as srv:
            ids = [srv.submit(p, k) for p, k in zip(pats, ks)]
            for i, q in enumerate(ids):
                info = srv.wait(q, 60_000)
                if info.state == server.FAILED:  # a result that can never fit this arena
                    assert info.error == -4
                    srv.release(q)
                    continue
                assert_same(as_np(srv.result(q)), want[i], f"served {i}")
