"""The batch-shape autotuner on the GPU: tune() over a small batch with a
temporary cache times every candidate shape, keeps the fastest, and a second
call is served from the cache; every candidate shape's lists equal the
oracle's."""
import sys

import numpy as np
import pytest

import oracle

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


def test_autotune_times_candidates_caches_and_every_shape_is_exact(pm, tmp_path):
    from paper_1611_06115_amd import autotune, synth

    w = synth.batched(n=8_000_000, count=64)
    t = pm.encode_text(w.text, device=torch.device("cuda:0"))
    torch.cuda.synchronize()
    t.check()
    batch = pm.Batch(w.patterns, w.ks, t.n)
    cache = autotune.Cache(str(tmp_path / "tune.json"))
    say(f"  tune: {len(batch)} patterns over {t.n} bases, {len(autotune.DEFAULT_CANDIDATES)} shapes")
    r = autotune.tune(t, batch, cache=cache, sample_windows=t.n)
    assert not r.cached and len(r.timings) == len(autotune.DEFAULT_CANDIDATES)
    chosen = "g%d s%d r%d" % (r.config.group_size, r.config.sub_ranges, r.config.lane_words)
    assert r.timings[chosen] == min(r.timings.values())
    assert round(r.ms, 4) == r.timings[chosen]
    # a second call: the cached choice, no timing
    r2 = autotune.tune(t, batch, cache=autotune.Cache(str(tmp_path / "tune.json")))
    assert r2.cached and not r2.timings
    assert (r2.config.group_size, r2.config.sub_ranges, r2.config.lane_words) == \
        (r.config.group_size, r.config.sub_ranges, r.config.lane_words)
    # every candidate shape's lists are the oracle's
    want = []
    for p, k in zip(w.patterns, w.ks):
        pos, cnt, total = oracle.scan(w.text, oracle.parse(p), k, threads=16)
        want.append((pos, cnt))
    for cand in autotune.DEFAULT_CANDIDATES:
        cfg = pm.BatchConfig(int(cand[0]), int(cand[1]), int(cand[2]), 0)
        say(f"  shape {cand}")
        got = pm.scan_batch(t, batch, None, config=cfg)
        for i, (g, (wp, wc)) in enumerate(zip(got, want)):
            gp, gc = g[0].cpu().numpy(), g[1].cpu().numpy()
            assert np.array_equal(gp, wp) and np.array_equal(gc, wc), (cand, i)
