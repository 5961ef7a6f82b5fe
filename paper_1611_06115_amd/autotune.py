"""Autotuner of the batched scan's launch shape.

The batched kernel has three shape parameters (pm_batch_config): patterns
that share one text tile (group size), text sub-ranges per pattern group
(work items), and 32-window words per lane (4 or 6).  The best choice
depends on the batch: many short patterns with small k favour large groups
(the text tile and its planes are shared by more patterns), few long or
high-k patterns favour smaller groups and more sub-ranges (balance).

`tune` times candidate shapes on a window sample of the real text with the
real patterns (every candidate computes the same result) and keeps the
fastest.  Choices are cached in a JSON file keyed by the GPU architecture and
driver and by a bucketed signature of the batch (number of patterns, text
length, histograms of pattern length and k), so a batch of the same kind on
the same machine reuses the choice without timing.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass

import numpy as np

from .scan import Batch, BatchConfig, Text, batch_workspace_bytes, scan_batch_async

# (group size, sub-ranges (0 = the library's choice), lane words)
DEFAULT_CANDIDATES = [
    (4, 0, 4), (8, 0, 4), (16, 0, 4),
    (4, 0, 6), (8, 0, 6), (16, 0, 6),
    (8, 64, 4), (8, 512, 4),
]


def _cache_path() -> str:
    return os.environ.get("PMSCAN_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pmscan", "autotune.json"))


def device_key() -> str:
    """GPU architecture and HIP runtime of the current device."""
    import torch

    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", props.name)
    return f"{arch}|hip-{torch.version.hip}"


def _bucket_log2(x: float) -> int:
    return int(math.floor(math.log2(max(x, 1.0))))


def signature(m, ks, n: int) -> str:
    """Bucketed description of a batch: log2 of the pattern count and of the
    text length, and the share of patterns in each (log2 m, k range) bucket,
    rounded to tenths."""
    m = np.asarray(m, dtype=np.float64)
    ks = np.asarray(ks, dtype=np.int64)
    k_edges = [0, 1, 3, 6, 11, 1 << 30]
    kb = np.searchsorted(k_edges, ks, side="right") - 1
    mb = np.floor(np.log2(np.maximum(m, 1.0))).astype(np.int64)
    hist = {}
    for a, b in zip(mb.tolist(), kb.tolist()):
        hist[(a, b)] = hist.get((a, b), 0) + 1
    parts = [f"c{_bucket_log2(len(m))}", f"n{_bucket_log2(n)}"]
    for key in sorted(hist):
        share = round(hist[key] / len(m), 1)
        if share > 0:
            parts.append(f"m{key[0]}k{key[1]}:{share:g}")
    return ",".join(parts)


@dataclass
class TuneResult:
    config: BatchConfig
    ms: float                 # time of the chosen shape on the sample
    timings: dict             # candidate -> ms on the sample
    cached: bool
    sample_windows: int


class Cache:
    """JSON file {device key: {signature: {group_size, sub_ranges, lane_words, ms}}}."""

    def __init__(self, path: str | None = None):
        self.path = path or _cache_path()
        self.data = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    def get(self, dev: str, sig: str):
        return self.data.get(dev, {}).get(sig)

    def put(self, dev: str, sig: str, entry: dict) -> None:
        self.data.setdefault(dev, {})[sig] = entry
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def tune(text: Text, batch: Batch, candidates=None, sample_windows: int | None = None, reps: int = 2,
         cache: Cache | None = None, use_cache: bool = True, stream=None) -> TuneResult:
    """Choose the batched launch shape for `batch` over `text` (see module doc)."""
    import torch

    dev_key = device_key()
    sig = signature(batch.m, batch.ks, text.n)
    cache = cache if cache is not None else Cache()
    if use_cache:
        hit = cache.get(dev_key, sig)
        if hit is not None:
            cfg = BatchConfig(int(hit["group_size"]), int(hit["sub_ranges"]), int(hit["lane_words"]), 0)
            return TuneResult(cfg, float(hit.get("ms", 0.0)), {}, True, int(hit.get("sample_windows", 0)))
    candidates = list(candidates or DEFAULT_CANDIDATES)
    if sample_windows is None:
        sample_windows = int(min(text.n, max(1 << 24, text.n // 8)))
    dev = text.data.device
    stream = stream or torch.cuda.current_stream()
    pos = torch.empty(max(batch.total_capacity, 1), dtype=torch.int64, device=dev)
    cnt = torch.empty(max(batch.total_capacity, 1), dtype=torch.uint16, device=dev)
    n_hits = torch.zeros(len(batch), dtype=torch.int64, device=dev)
    status = torch.zeros(len(batch), dtype=torch.int32, device=dev)
    timings = {}
    reference = None
    for cand in candidates:
        cfg = BatchConfig(int(cand[0]), int(cand[1]), int(cand[2]), 0)
        ws = torch.empty(batch_workspace_bytes(text.n, batch, cfg), dtype=torch.uint8, device=dev)
        run = lambda: scan_batch_async(text, batch, pos, cnt, n_hits, status, ws,  # noqa: E731
                                       win_begin=0, win_end=sample_windows, config=cfg, stream=stream)
        run()
        stream.synchronize()
        # every shape must give the same lists: totals, completion, and each
        # complete pattern's positions and counts
        totals = n_hits.cpu().numpy().copy()
        done = status.cpu().numpy() == 0
        lists = [(pos[int(o):int(o) + int(h)].cpu().numpy(), cnt[int(o):int(o) + int(h)].cpu().numpy())
                 if d else None for o, h, d in zip(batch.out_off, totals, done)]
        if reference is None:
            reference = (totals, lists)
        else:
            same = np.array_equal(reference[0], totals) and all(
                (a is None or b is None) or (np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]))
                for a, b in zip(reference[1], lists))
            if not same:
                raise RuntimeError(f"batch shape {cand} changed the hit lists")
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        e1.synchronize()
        timings[tuple(cand)] = e0.elapsed_time(e1) / reps
        del ws
    best = min(timings, key=timings.get)
    cfg = BatchConfig(int(best[0]), int(best[1]), int(best[2]), 0)
    cache.put(dev_key, sig, {"group_size": cfg.group_size, "sub_ranges": cfg.sub_ranges,
                             "lane_words": cfg.lane_words, "ms": round(timings[best], 4),
                             "sample_windows": sample_windows, "tuned_at": time.strftime("%Y-%m-%dT%H:%M:%S")})
    return TuneResult(cfg, timings[best], {"g%d s%d r%d" % k: round(v, 4) for k, v in timings.items()},
                      False, sample_windows)
