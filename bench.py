"""Benchmark of the k-mismatch character-class scan on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload genome]

A step is one pass of the hot path over the resident text: the pattern is
encoded on the host and the scan (filter, verification, ordered hit output)
runs as one kernel launch over every window.  The text is generated, planted
with copies of the pattern and encoded into device memory before timing
(one-time setup, reported separately as `encode_ms`).  K steps are timed with
HIP events on the stream the kernels run on.

Prints one JSON line: the metric (logical base-pattern comparisons per
second, (n - m + 1) * m per pattern and pass), the roofline of the scan
kernel, and the oracle timed on the host cores over a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# nominal int32 VALU lane-ops/s: CUs x lanes per clock (two instructions
# issued per SIMD per 4-clock cycle) x clock; used only when no calibration
# run has been committed
VALU_NOMINAL_TOPS = 256 * 128 * 2.4e9 / 1e12


def valu_peak() -> dict:
    """The VALU ceilings measured on the box by bench.py --valu-calibration
    (committed as profiles/valu_calibration.json): "peak" is the highest
    issue rate measured for any instruction (independent chains, full
    occupancy), "mix" the rate of the filter's 1:2 mix of alignbit and
    three-input LUT operations.  Falls back to the nominal figure."""
    path = os.path.join(PROFILE_DIR, "valu_calibration.json")
    if os.path.exists(path):
        with open(path) as f:
            c = json.load(f)["ceilings_T"]
        return {"peak": c["full_rate_max"], "mix": c["filter_mix_1_alignbit_2_bitop3"],
                "alignbit": c["v_alignbit_b32"], "source": "profiles/valu_calibration.json"}
    return {"peak": round(VALU_NOMINAL_TOPS, 1), "mix": None, "alignbit": None, "source": "nominal"}


# The sources that define each workload's kernels: a committed counter run
# applies only while these are unchanged.
KERNEL_SOURCES = {
    "genome": ("scan_kernels.hpp", "plan.cpp", "plan.hpp", "scan_core.hpp"),
    "batched": ("batch.hip", "batch.hpp", "plan.cpp", "plan.hpp", "scan_core.hpp"),
}


def kernel_source_sha(workload: str = "genome") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[workload]:
        with open(os.path.join(ROOT, "paper_1611_06115_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None when
    absent or taken on a different kernel source."""
    path = os.path.join(PROFILE_DIR, f"scan_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_sha(workload):
        return None
    return t.get("hbm_bytes_per_launch")


def measured_count_valu(workload: str):
    """VALU lane-ops per count-kernel launch from the committed counter run
    (SQ_INSTS_VALU x 64), or None when absent or taken on a different kernel
    source."""
    path = os.path.join(PROFILE_DIR, f"scan_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_sha(workload):
        return None
    return t.get("count_kernel_valu_lane_ops")


def valu_profile(workload: str):
    """The committed VALU counter run of a workload ({"config": launch shape,
    "valu_lane_ops_per_launch": ...}), or None when absent or taken on a
    different kernel source."""
    path = os.path.join(PROFILE_DIR, f"scan_{workload}_valu.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_sha(workload):
        return None
    return t


def settle(fn, stream, seconds: float, block: int = 20) -> dict:
    """Back-to-back steps for `seconds` of GPU time, before the warm-up.
    From an idle GPU the first ~200 genome scans run at a transient low
    shader clock (the power management overshoots, then settles: their mean
    is ~14% above the sustained step, single steps up to 35%), and the rate
    then holds for seconds; timing from idle would measure that transient.
    Returns the steps run and the mean ms per step of the first block (the
    from-idle figure)."""
    import torch

    if seconds <= 0:
        return {"seconds": 0, "steps": 0}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    first, steps, spent = None, 0, 0.0
    while spent < seconds * 1e3:
        e0.record(stream)
        for _ in range(block):
            fn()
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        if first is None:
            first = ms / block
        spent += ms
        steps += block
    return {"seconds": seconds, "steps": steps, "first_block_ms_per_step": round(first, 5)}


def time_steps(fn, steps: int, warmup: int, stream, kernel: bool = False, samples: list | None = None):
    """Mean ms per step over `steps` timed steps (HIP events on `stream`).
    With kernel=True also the mean duration of the scan's main kernel, from
    a pair of events the library records around that launch; those events
    go into a second timed loop of the same steps, so that they do not
    perturb the step time.  `samples`, if given, receives each step's kernel
    duration (ms)."""
    import torch

    from paper_1611_06115_amd import scan

    for _ in range(warmup):
        fn()
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    e1.synchronize()
    step_ms = e0.elapsed_time(e1) / steps
    if not kernel:
        return step_ms
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in pairs:  # creates the events
        a.record(stream)
        b.record(stream)
    stream.synchronize()
    for i in range(steps):
        scan.time_next_scan(*pairs[i])
        fn()
    stream.synchronize()
    each = [a.elapsed_time(b) for a, b in pairs]
    if samples is not None:
        samples.extend(each)
    return step_ms, sum(each) / steps


def time_steps_cold(fn, steps: int, warmup: int, stream, flush_bytes: int = 512 << 20, samples: list | None = None):
    """Like time_steps(kernel=True), but every step (timed on its own) comes
    after a write of flush_bytes to a scratch buffer, larger than the
    256 MB Infinity Cache, so that the text is read from HBM rather than from
    a cache that still holds it from the previous step."""
    import torch

    from paper_1611_06115_amd import scan

    scratch = torch.empty(flush_bytes, dtype=torch.uint8, device=stream.device)
    for _ in range(warmup):
        fn()
    stream.synchronize()
    step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    kern_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in kern_ev:  # creates the events
        a.record(stream)
        b.record(stream)
    stream.synchronize()
    for i in range(steps):
        scratch.fill_(i & 0xFF)
        a, b = step_ev[i]
        a.record(stream)
        scan.time_next_scan(*kern_ev[i])
        fn()
        b.record(stream)
    stream.synchronize()
    del scratch
    each = [a.elapsed_time(b) for a, b in kern_ev]
    if samples is not None:
        samples.extend(each)
    return sum(a.elapsed_time(b) for a, b in step_ev) / steps, sum(each) / steps


def host_cpu_model() -> str:
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads the oracle baseline uses: every core this process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


def cpu_baseline(text, pattern: str, k: int, m: int, target_s: float = 10.0, lists: bool = False):
    """The oracle (plain brute force with early stop, on every core the
    process may use) on a prefix of the windows, sized to about target_s
    seconds.  With lists=True also returns the oracle's (positions, counts)
    for that prefix and its end."""
    import oracle

    threads = host_threads()
    sets = oracle.parse(pattern)
    nw = text.size - m + 1
    sample = min(nw, 5_000_000)
    while True:  # grow the sample until one run takes about target_s
        t0 = time.perf_counter()
        pos, cnt, hits = oracle.scan(text, sets, k, threads=threads, win_end=sample, capacity=1 << 20)
        dt = time.perf_counter() - t0
        if dt >= 0.6 * target_s or sample >= nw:
            break
        sample = int(min(nw, sample * min(8.0, max(1.5, target_s / max(dt, 1e-3)))))
    res = {
        "value": round(sample * m / dt / 1e9, 3),
        "unit": "G comparisons/s",
        "cores": threads, "cpu_count": os.cpu_count(),
        "kind": "oracle", "cpu": host_cpu_model(),
        "sample": f"windows [0, {sample}) of the same text ({sample / nw:.1%} of the pass), "
                  f"k={k}, {dt:.1f} s wall, {hits} hits",
    }
    if lists:
        return res, (pos, cnt, hits, sample)
    return res


def run_plain(args):
    import numpy as np
    import torch

    from paper_1611_06115_amd import scan, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    pi = 0  # which of the workload's patterns is scanned
    if args.workload == "genome":
        w = synth.genome(n=args.n or 3_100_000_000)
        pattern, k = w.patterns[0], w.ks[0]
        desc = (f"genome: n={w.n} order-3 Markov GC 0.41, m={len(pattern)} "
                f"(20% 2-3-base classes), k={k}, 64 planted copies")
    elif args.workload == "small":
        w = synth.small(n=args.n or 1_000_000)
        pattern, k = w.patterns[0], args.k if args.k is not None else 2
        desc = f"small: n={w.n} uniform i.i.d., m={len(pattern)} (8 multi-base classes), k={k}"
    elif args.workload == "long_m":
        w = synth.long_m(n=args.n or 64_000_000)
        pi = 1 if args.m == 4096 else 0
        pattern, k = w.patterns[pi], args.k if args.k is not None else 16
        desc = f"long_m: n={w.n} i.i.d. GC 0.41, m={len(pattern)} (10% 2-3-base classes), k={k}"
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    log(f"[bench] generated {w.n} bases in {time.perf_counter() - t0:.1f}s")

    stream = torch.cuda.current_stream()
    ascii_dev = torch.from_numpy(w.text).to(dev)
    t0 = time.perf_counter()
    text = scan.encode_text(ascii_dev)
    stream.synchronize()
    encode_ms = (time.perf_counter() - t0) * 1e3
    text.check()
    # encode throughput, timed on its own (1 B in + 0.25 B out per base)
    enc_ms = time_steps(lambda: scan.encode_text(ascii_dev), 3, 1, stream)
    del ascii_dev
    torch.cuda.empty_cache()
    log(f"[bench] encoded in {encode_ms:.1f} ms (kernel {enc_ms:.3f} ms)")

    pat = scan.Pattern(pattern)
    m = pat.m
    ws = scan.Workspace(dev, text.n, capacity=1 << 20)
    step = lambda: scan.scan_async(text, pat, k, ws)  # noqa: E731
    kern_each = []
    if args.flush:
        settled = {"seconds": 0, "steps": 0}
        ms, kern_ms = time_steps_cold(step, args.steps, args.warmup, stream, samples=kern_each)
    else:
        settled = settle(step, stream, args.settle)
        log(f"[bench] settled: {settled}")
        ms, kern_ms = time_steps(step, args.steps, args.warmup, stream, kernel=True, samples=kern_each)
    hits = int(ws.n_hits.item())
    log(f"[bench] {args.steps} steps, {ms:.4f} ms/step (count kernel {kern_ms:.4f} ms), {hits} hits")

    # planted copies within the budget must all be reported
    pos = ws.pos[:min(hits, ws.capacity)].cpu().numpy()
    cnt = ws.cnt[:min(hits, ws.capacity)].cpu().numpy()
    found = dict(zip(pos.tolist(), cnt.tolist()))
    missed = [(p, d) for q, p, d in w.plants if q == pi and d <= k and found.get(p) != d]
    if missed:
        raise SystemExit(f"planted sites missed or miscounted: {missed[:5]}")

    nw = text.n - m + 1
    comps = nw * m
    sec = ms / 1e3
    # algorithmic bytes of the count kernel (one launch): the encoded text once,
    # the staged hits, the pattern image
    algo_bytes = 0.25 * text.n + 8.0 * hits + pat.image(dev).numel() * 4
    achieved = algo_bytes / (kern_ms / 1e3) / 1e9
    traffic = measured_traffic(args.workload)
    valu_ops = measured_count_valu(args.workload)
    result = {
        "metric": "G base-pattern comparisons/sec",
        "value": round(comps / sec / 1e9, 2),
        "unit": "G comparisons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 bitwise (exact integer counts)",
        "data": "synthetic",
        "config": {"workload": desc, "n": text.n, "m": m, "k": k, "windows": nw, "hits": hits,
                   "cache": ("cold: 512 MB written before each timed step" if args.flush
                             else "warm: steps back to back"),
                   # steps run back to back before the warm-up, so that the
                   # timed steps see the sustained clock (the first block's
                   # rate is the from-idle transient)
                   "settle": settled,
                   "count_kernel_ms": {"mean": round(kern_ms, 5), "sd": round(float(np.std(kern_each)), 5),
                                       "runs": len(kern_each)},
                   "windows_per_s": round(nw / sec, 1), "encode_kernel_ms": round(enc_ms, 4),
                   # the same kernel against the int32 VALU peak (its lane-ops
                   # per launch from the committed counter run)
                   "count_kernel_valu": None if valu_ops is None else {
                       "achieved": round(valu_ops / (kern_ms / 1e3) / 1e12, 2), "peak": valu_peak()["peak"],
                       "unit": "T int32 VALU lane-ops/s",
                       "frac": round(valu_ops / (kern_ms / 1e3) / 1e12 / valu_peak()["peak"], 4),
                       "mix_ceiling": valu_peak()["mix"], "peak_source": valu_peak()["source"]},
                   # context, not a target: the paper's CPU rate, (n - m + 1) m logical
                   # comparisons over its mean runtime for m = 500 on chromosome 2
                   # (243 199 373 bases, 6.595 s; Sect. 3, Table 5; hardware not stated)
                   "paper_cpu_context": {"value": round((243_199_373 - 499) * 500 / 6.595 / 1e9, 1),
                                         "unit": "G comparisons/s", "hardware": "not stated"}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on a bounded sample")
        result["cpu_baseline"], (opos, ocnt, ohits, osample) = cpu_baseline(w.text, pattern, k, m, lists=True)
        # the GPU list over the oracle's windows must equal the oracle's, hit for hit
        gpos = ws.pos[:min(hits, ws.capacity)].cpu().numpy()
        gcnt = ws.cnt[:min(hits, ws.capacity)].cpu().numpy()
        sel = gpos < osample
        if hits > ws.capacity or ohits != int(sel.sum()) or not (
                np.array_equal(gpos[sel], opos) and np.array_equal(gcnt[sel], ocnt)):
            raise SystemExit(f"GPU hits differ from the oracle's over windows [0, {osample})")
        result["config"]["oracle_check"] = (f"the GPU list equals the oracle's over windows [0, {osample}) "
                                            f"({osample / nw:.1%} of the pass, {ohits} hits)")
        log(f"[bench] GPU list equals the oracle's over [0, {osample})")
    if args.workload == "genome" and not args.no_served:
        # the served form on the same resident text: Poisson arrivals at
        # 1000 queries/s for 3 s from the served workload's query pool
        from paper_1611_06115_amd import server

        log("[bench] served latency on the resident text (1000 queries/s, 3 s)")
        pats, kq = synth.query_pool(count=4000)
        res = serve(text, [scan.Pattern(x) for x in pats], kq, 1000.0, 3.0,
                    server.ServerConfig(chunks=0, max_active=0, batch=scan.BatchConfig(0, 0, 0, 0)), 64.0)
        result["latency_ms"] = res["latency_ms"]
        result["config"]["served"] = {"workload": "served form on this text: Poisson arrivals at 1000/s for 3 s "
                                                  "from the served query pool (m log-uniform 20..5000, "
                                                  "k ~ U{0..10}, class density ~ U[0,0.3]), not planted",
                                      "queries": res["queries"], "qps_achieved": res["qps_achieved"],
                                      "hits": res["hits"], "queue_ms": res["queue_ms"],
                                      "value": res["value"], "unit": "G comparisons/s",
                                      "checked": res["checked"]}
    return result


def copy_calibration(gib: float = 1.0, reps: int = 3):
    """A plain device-to-device copy of a known size, for scaling the HBM
    byte counters (FETCH_SIZE / WRITE_SIZE) read in counter runs."""
    import torch

    nbytes = int(gib * (1 << 30))
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def valu_calibration(target_ms: float = 3.0):
    """Issue rates of the VALU instructions the scan kernels use, measured by
    the probe library (csrc/calib.hip): lane-operations per second of
    independent chains of one instruction (or the filter's 1:2 mix of
    alignbit and three-input LUT operations) at 1-8 waves per SIMD.  Prints
    one JSON object; the ceilings it reports are what the "alu" rooflines
    are set against."""
    import ctypes

    from paper_1611_06115_amd import _build

    if not os.path.exists(_build.CALIB_LIB):
        raise SystemExit(f"{_build.CALIB_LIB} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(_build.CALIB_LIB)
    L.pmc_kind_name.restype = ctypes.c_char_p
    L.pmc_valu_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    cus = L.pmc_compute_units()

    def probe(kind, chains, waves):
        ms, ops = ctypes.c_double(), ctypes.c_double()
        iters = 256
        for _ in range(2):  # size the loop to about target_ms per launch
            rc = L.pmc_valu_probe(kind, chains, waves, iters, 1, ctypes.byref(ms), ctypes.byref(ops))
            if rc:
                raise SystemExit(f"probe {kind} failed: hip error {rc}")
            iters = max(64, int(iters * target_ms / max(ms.value, 1e-3)))
        rc = L.pmc_valu_probe(kind, chains, waves, iters, 3, ctypes.byref(ms), ctypes.byref(ops))
        if rc:
            raise SystemExit(f"probe {kind} failed: hip error {rc}")
        return ops.value / (ms.value / 1e3) / 1e12

    rows = []
    for kind in range(L.pmc_kind_count()):
        name = L.pmc_kind_name(kind).decode()
        waves_list = (1, 2, 4, 5, 8) if kind in (0, 1, 3, 8) else (4, 8)
        for waves in waves_list:
            for chains in ((1, 2, 4, 8) if kind in (0, 1, 8) and waves in (4, 5) else (8,)):
                t = probe(kind, chains, waves)
                rows.append({"kind": name, "waves_per_simd": waves, "chains": chains, "T_lane_ops_s": round(t, 2)})
                log(f"[valu] {name:32s} waves {waves} chains {chains}: {t:6.2f} T lane-ops/s")
    best = lambda name: max(r["T_lane_ops_s"] for r in rows if r["kind"] == name)  # noqa: E731
    out = {
        "compute_units": cus,
        "nominal_single_issue_T": round(cus * 64 * 2.4e9 / 1e12, 2),
        "ceilings_T": {
            "full_rate_max": max(r["T_lane_ops_s"] for r in rows),
            "v_bitop3_b32": best("v_bitop3_b32 xor3"),
            "v_alignbit_b32": best("v_alignbit_b32 (sgpr shift)"),
            "filter_mix_1_alignbit_2_bitop3": best("alignbit:bitop3 1:2"),
        },
        "rows": rows,
    }
    print(json.dumps(out), flush=True)


def run_sustained(args):
    """The genome scan run back to back from an idle GPU for --duration
    seconds, its step time taken in blocks of 20 steps: the power transient
    of the first scans and the rate that holds after it (what the settle
    phase of the default line waits out)."""
    import numpy as np
    import torch

    from paper_1611_06115_amd import scan, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.genome(n=args.n or 3_100_000_000)
    pattern, k = w.patterns[0], w.ks[0]
    text = scan.encode_text(torch.from_numpy(w.text).to(dev))
    stream = torch.cuda.current_stream()
    stream.synchronize()
    text.check()
    pat = scan.Pattern(pattern)
    ws = scan.Workspace(dev, text.n, capacity=1 << 20)
    block = 20
    # enough blocks for the duration at the sustained rate (~0.15 ms a step)
    n_blocks = max(10, int(args.duration / (block * 0.15e-3)))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_blocks + 1)]
    for e in ev:  # creates the events
        e.record(stream)
    stream.synchronize()
    time.sleep(2.0)  # an idle GPU first
    ev[0].record(stream)
    for b in range(n_blocks):
        for _ in range(block):
            scan.scan_async(text, pat, k, ws)
        ev[b + 1].record(stream)
        if b % 50 == 49:
            ev[b + 1].synchronize()
            log(f"[bench] {(b + 1) * block} steps")
    stream.synchronize()
    per = np.array([ev[b].elapsed_time(ev[b + 1]) / block for b in range(n_blocks)])
    first = per[:10]  # steps 1-200
    rest = per[10:]
    nw = text.n - pat.m + 1
    steady = float(rest.mean())
    hits = int(ws.n_hits.item())
    return {
        "metric": "G base-pattern comparisons/sec", "value": round(nw * pat.m / (steady / 1e3) / 1e9, 2),
        "unit": "G comparisons/s", "n_gpus": 1, "steps": int(n_blocks * block), "warmup": 0,
        "ms_per_step": round(steady, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 bitwise (exact integer counts)", "data": "synthetic",
        "config": {"workload": f"sustained: the genome scan (n={text.n}, m={pat.m}, k={k}) back to back from "
                               f"an idle GPU, {n_blocks * block} steps timed in blocks of {block}",
                   "hits": hits,
                   "steps_1_200_ms_per_step": {"mean": round(float(first.mean()), 5),
                                               "max_block": round(float(first.max()), 5)},
                   "after_200_ms_per_step": {"mean": round(steady, 5), "min_block": round(float(rest.min()), 5),
                                             "max_block": round(float(rest.max()), 5),
                                             "sd_block": round(float(rest.std()), 5)},
                   "blocks_of_200_steps_ms": [round(float(per[i:i + 10].mean()), 4)
                                              for i in range(0, n_blocks, 10)]},
        "roofline": {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                     "traffic": None},
    }


def run_mscale(args):
    """The shape of the paper's m-scaling experiment (Sect. 3, Tables 5-7)
    on a synthetic text of chromosome 2's length: exact copies of m = 500,
    10 000 and 100 000 cut at the tables' five sites per length, each
    scanned in 5 timed runs (k = 0 unless --k).  Reports the mean and spread
    per site and per length, and the slowest length's mean over the
    fastest's."""
    import numpy as np
    import torch

    from paper_1611_06115_amd import scan, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    w = synth.mscale(n=args.n or synth.CHR2_LEN)
    k = args.k if args.k is not None else 0
    log(f"[bench] generated {w.n} bases and {len(w.patterns)} cut patterns in {time.perf_counter() - t0:.1f}s")
    stream = torch.cuda.current_stream()
    text = scan.encode_text(torch.from_numpy(w.text).to(dev))
    stream.synchronize()
    text.check()
    ws = scan.Workspace(dev, text.n, capacity=1 << 16)
    runs = 5
    rows = []
    for pi, pat_s in enumerate(w.patterns):
        pat = scan.Pattern(pat_s)
        step = lambda: scan.scan_async(text, pat, k, ws)  # noqa: E731
        for _ in range(max(1, args.warmup)):
            step()
        stream.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(runs)]
        for a, b in ev:
            a.record(stream)
            step()
            b.record(stream)
        stream.synchronize()
        t = np.array([a.elapsed_time(b) for a, b in ev])
        _, kern = time_steps(step, 3, 0, stream, kernel=True)
        hits = int(ws.n_hits.item())
        pos = ws.pos[:min(hits, ws.capacity)].cpu().numpy()
        site = w.plants[pi][1]
        if not (pos == site).any():
            raise SystemExit(f"cut site {site} of pattern {pi} (m={len(pat_s)}) not reported")
        rows.append({"m": len(pat_s), "location": site + 1, "ms": round(float(t.mean()), 4),
                     "sd": round(float(t.std()), 4), "kernel_ms": round(kern, 4), "hits": hits})
        log(f"[bench] m={len(pat_s)} at {site + 1}: {t.mean():.4f} +- {t.std():.4f} ms, {hits} hits")
    per_m = {}
    for r in rows:
        per_m.setdefault(r["m"], []).append(r["ms"])
    per_m = {m: round(float(np.mean(v)), 4) for m, v in per_m.items()}
    total_ms = sum(r["ms"] for r in rows)
    kern_ms = sum(r["kernel_ms"] for r in rows)
    comps = float(sum((text.n - r["m"] + 1) * r["m"] for r in rows))
    achieved = 0.25 * text.n * len(rows) / (kern_ms / 1e3) / 1e9
    result = {
        "metric": "G base-pattern comparisons/sec",
        "value": round(comps / (total_ms / 1e3) / 1e9, 1),
        "unit": "G comparisons/s",
        "n_gpus": 1, "steps": runs * len(rows), "warmup": args.warmup,
        "ms_per_step": round(total_ms / len(rows), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 bitwise (exact integer counts)", "data": "synthetic",
        "config": {"workload": f"mscale: n={text.n} order-3 Markov GC 0.41 (chromosome 2's length), exact "
                               f"copies of m = 500 / 10000 / 100000 at the 5 sites per length of Tables 5-7, k={k}",
                   "per_m_ms": per_m,
                   "slowest_over_fastest": round(max(per_m.values()) / min(per_m.values()), 4),
                   "rows": rows,
                   # context, not a target: the paper's mean CPU runtimes on the real
                   # chromosome 2 (Sect. 3, Tables 5-7; its hardware is not stated)
                   "paper_cpu_s": {"500": 6.595, "10000": 6.882, "100000": 6.980,
                                   "slowest_over_fastest": 1.0584, "hardware": "not stated"}},
        # the count kernel over all runs: the text once per scan
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(achieved / 8000.0, 4), "traffic": None},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w.text, w.patterns[0], k, len(w.patterns[0]))
    return result


def ls_direct_uint64_max_m(limit: int = 4000) -> int:
    """Largest m for which the Linhart-Shamir correlation, computed directly
    (no residues), stays below 2^64: m terms of n_S < M times the largest
    text code M / k_1, with k_1 < ... < k_4 the four smallest primes above m
    and M their product (the limit of Sect. 1.3.5)."""
    def is_prime(x):
        return x > 1 and all(x % d for d in range(2, int(x ** 0.5) + 1))

    best = 0
    for m in range(1, limit):
        ks, x = [], m + 1
        while len(ks) < 4:
            if is_prime(x):
                ks.append(x)
            x += 1
        big_m = ks[0] * ks[1] * ks[2] * ks[3]
        if m * (big_m - 1) * (big_m // ks[0]) < 1 << 64:
            best = m
    return best


def run_crt(args):
    """The Linhart-Shamir transform route (pm_crt_counts, Sect. 1.3): every
    window's mismatch count of one pattern over the long-pattern text, timed
    beside the early-stop scan of the same pattern.  The counts at or below
    k must equal the scan's hits."""
    import numpy as np
    import torch

    from paper_1611_06115_amd import scan, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.long_m(n=args.n or 64_000_000)
    pi = 1 if args.m == 4096 else 0
    pattern, k = w.patterns[pi], args.k if args.k is not None else 16
    stream = torch.cuda.current_stream()
    text = scan.encode_text(torch.from_numpy(w.text).to(dev))
    stream.synchronize()
    text.check()
    pat = scan.Pattern(pattern)
    m = pat.m
    nw = text.n - m + 1
    out = torch.empty(nw, dtype=torch.int32, device=dev)
    ws = torch.empty(scan.crt_counts_workspace_bytes(text.n, m), dtype=torch.uint8, device=dev)
    ms = time_steps(lambda: scan.crt_counts_into(text, pat, out, ws), args.steps, args.warmup, stream)
    sws = scan.Workspace(dev, text.n, capacity=1 << 20)
    scan_ms = time_steps(lambda: scan.scan_async(text, pat, k, sws), args.steps, args.warmup, stream)
    sel = torch.nonzero(out <= k).flatten()
    hits = int(sws.n_hits.item())
    if not (sel.numel() == hits and torch.equal(sel, sws.pos[:hits])
            and torch.equal(out[sel], sws.cnt[:hits].to(torch.int32))):
        raise SystemExit("transform-route counts at or below k differ from the scan's hits")
    log(f"[bench] crt route {ms:.3f} ms per pass over {text.n} bases (scan {scan_ms:.4f} ms), {hits} hits agree")
    sec = ms / 1e3
    algo_bytes = 0.25 * text.n + 4.0 * nw  # the text once and every window's count
    result = {
        "metric": "G base-pattern comparisons/sec",
        "value": round(nw * m / sec / 1e9, 2),
        "unit": "G comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 modular (exact integer counts)", "data": "synthetic",
        "config": {"workload": f"crt: n={text.n} i.i.d. GC 0.41, m={m}, every window's count by the "
                               f"Linhart-Shamir route (number-theoretic transforms, blocks of 2^20)",
                   "windows": nw, "k_checked": k, "hits": hits, "scan_ms": round(scan_ms, 4),
                   "ls_direct_uint64_max_m": ls_direct_uint64_max_m()},
        # the route's own bytes are the text and the counts; its transforms
        # pass each block's working set through the caches 2 log2(L) times
        "roofline": {"bound": "hbm", "achieved": round(algo_bytes / sec / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(algo_bytes / sec / 1e9 / HBM_PEAK_GBS, 4), "traffic": None},
    }
    if not args.no_cpu_baseline:
        import oracle

        sets = oracle.parse(pattern)
        sample = 20_000
        while True:
            t0 = time.perf_counter()
            oracle.counts(w.text[:sample + m - 1], sets)
            dt = time.perf_counter() - t0
            if dt >= 5.0 or sample >= nw:
                break
            sample = min(nw, sample * 4)
        result["cpu_baseline"] = {"value": round(sample * m / dt / 1e9, 3), "unit": "G comparisons/s",
                                  "cores": 1, "kind": "oracle", "cpu": host_cpu_model(),
                                  "sample": f"full counts (no early stop) of windows [0, {sample}), {dt:.1f} s"}
    return result


def run_outofcore(args):
    """The genome workload with the text kept in pinned host memory and
    scanned by streaming it through the device in chunks with an m-1 overlap
    (copies on a second stream overlapping the scans).  The link sets the
    pace, so the line reports the end-to-end rate next to one plain pinned
    host-to-device copy of the whole text."""
    import numpy as np
    import torch

    from paper_1611_06115_amd import scan, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n or 3_100_000_000
    chunk = args.chunk or (1 << 27)
    t0 = time.perf_counter()
    host = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    w = synth.genome(n=n, text=host.numpy())
    pattern, k = w.patterns[0], w.ks[0]
    log(f"[bench] generated {n} bases into pinned host memory in {time.perf_counter() - t0:.1f}s")
    pat = scan.Pattern(pattern)
    stream = torch.cuda.current_stream()
    copy_stream = torch.cuda.Stream(dev)
    reps = max(1, min(args.steps, 5))
    res = scan.scan_host(host, pat, k, chunk_bases=chunk, stream=stream, copy_stream=copy_stream)  # warm-up
    times = []
    for _ in range(reps):
        t1 = time.perf_counter()
        pos, cnt = scan.scan_host(host, pat, k, chunk_bases=chunk, stream=stream, copy_stream=copy_stream)
        times.append(time.perf_counter() - t1)
    sec = float(np.mean(times))
    # the link alone: one host-to-device copy of the whole text (after a
    # warm-up copy), the rate the chunks cannot beat
    whole = torch.empty(n, dtype=torch.uint8, device=dev)
    copy_times = []
    for rep in range(reps + 1):
        stream.synchronize()
        t1 = time.perf_counter()
        whole.copy_(host, non_blocking=True)
        stream.synchronize()
        if rep > 0:
            copy_times.append(time.perf_counter() - t1)
    del whole
    copy_sec = float(np.mean(copy_times))
    # the count kernel of the first chunk, timed by the library's hook (it
    # brackets the next pm_scan call made by this thread)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    e1.record(stream)
    stream.synchronize()
    scan.time_next_scan(e0, e1)
    scan.scan_host(host, pat, k, chunk_bases=chunk, stream=stream, copy_stream=copy_stream)
    kern_ms = e0.elapsed_time(e1)
    chunk_len = min(n, chunk + len(pattern) - 1)
    achieved = 0.25 * chunk_len / (kern_ms / 1e3) / 1e9
    hits = int(pos.numel())
    found = dict(zip(pos.cpu().tolist(), cnt.cpu().tolist()))
    missed = [(p, d) for q, p, d in w.plants if d <= k and found.get(p) != d]
    if missed:
        raise SystemExit(f"planted sites missed or miscounted: {missed[:5]}")
    m = len(pattern)
    comps = float(n - m + 1) * m
    moved = float(n + (len(range(0, n - m + 1, chunk)) - 1) * (m - 1))
    log(f"[bench] {reps} runs, {sec * 1e3:.1f} ms per scan from host memory, the text copied alone {copy_sec * 1e3:.1f} ms, "
        f"{hits} hits; a chunk's count kernel {kern_ms:.3f} ms")
    result = {
        "metric": "G base-pattern comparisons/sec",
        "value": round(comps / sec / 1e9, 1),
        "unit": "G comparisons/s",
        "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": round(sec * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 bitwise (exact integer counts)", "data": "synthetic",
        "config": {"workload": f"outofcore: the genome workload (n={n}, m={m}, k={k}) with the ASCII text in "
                               f"pinned host memory, streamed in chunks of {chunk} windows",
                   "hits": hits, "chunk_bases": chunk,
                   # the pace is the host-to-device link: the chunks with
                   # their overlaps over the scan's time, against the same
                   # copies alone
                   "link": {"achieved": round(moved / sec / 1e9, 2), "copy_alone": round(n / copy_sec / 1e9, 2),
                            "unit": "GB/s", "frac": round((moved / sec) / (n / copy_sec), 4),
                            "copy_alone_ms": round(copy_sec * 1e3, 3)}},
        # the dominant kernel: the count kernel of one chunk
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w.text, pattern, k, m)
    return result


def run_batched(args):
    import numpy as np
    import torch

    from paper_1611_06115_amd import scan, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    count = args.count or 4096
    w = synth.batched(n=args.n or 256_000_000, count=count)
    log(f"[bench] generated {w.n} bases and {count} patterns in {time.perf_counter() - t0:.1f}s")
    stream = torch.cuda.current_stream()
    text = scan.encode_text(torch.from_numpy(w.text).to(dev))
    stream.synchronize()
    text.check()
    batch = scan.Batch(w.patterns, w.ks, text.n)
    tuned = None
    prof = valu_profile("batched")
    explicit = not (args.group is None and args.sub is None and args.lane_words is None)
    if not explicit and not args.autotune and prof is not None:
        # the shape the committed counter run was taken with (chosen by the
        # autotuner when it was made), so that its VALU count applies
        c = prof["config"]
        cfg = scan.BatchConfig(c["group_size"], c["sub_ranges"], c["lane_words"], 0)
        log(f"[bench] batch shape of the committed counter run: {c}")
    elif not explicit:
        from paper_1611_06115_amd import autotune

        t0 = time.perf_counter()
        tr = autotune.tune(text, batch)
        cfg = tr.config
        tuned = {"group_size": cfg.group_size, "sub_ranges": cfg.sub_ranges, "lane_words": cfg.lane_words,
                 "cached": tr.cached, "sample_windows": tr.sample_windows, "sample_ms": tr.timings,
                 "seconds": round(time.perf_counter() - t0, 2)}
        log(f"[bench] autotuned batch shape {tuned}")
    else:
        cfg = scan.BatchConfig(args.group or 0, args.sub or 0, args.lane_words or 0, 0)
    pos = torch.empty(batch.total_capacity, dtype=torch.int64, device=dev)
    cnt = torch.empty(batch.total_capacity, dtype=torch.uint16, device=dev)
    n_hits = torch.zeros(count, dtype=torch.int64, device=dev)
    status = torch.zeros(count, dtype=torch.int32, device=dev)
    ws = torch.empty(scan.batch_workspace_bytes(text.n, batch, cfg), dtype=torch.uint8, device=dev)
    step = lambda: scan.scan_batch_async(text, batch, pos, cnt, n_hits, status, ws, config=cfg)  # noqa
    ms, kern_ms = time_steps(step, args.steps, args.warmup, stream, kernel=True)
    nh = n_hits.cpu().numpy()
    st = status.cpu().numpy()
    log(f"[bench] {args.steps} steps, {ms:.3f} ms/step (batch kernels {kern_ms:.3f} ms), {int(nh.sum())} hits, "
        f"{int(st.sum())} incomplete")
    # planted copies must be found
    found = {}
    for i in range(count):
        if st[i] == 0:
            o = int(batch.out_off[i])
            found[i] = set(pos[o:o + int(nh[i])].cpu().tolist())
    missed = [(pi, p) for pi, p, d in w.plants if pi in found and p not in found[pi]]
    if missed:
        raise SystemExit(f"planted sites missed: {missed[:5]}")
    m = batch.m.astype(np.float64)
    comps = float(((text.n - m + 1).clip(min=0) * m).sum())
    sec = ms / 1e3
    valu = None
    if prof is not None and prof["config"] == {"group_size": cfg.group_size, "sub_ranges": cfg.sub_ranges,
                                               "lane_words": cfg.lane_words}:
        valu = prof["valu_lane_ops_per_launch"]
    result = {
        "metric": "G base-pattern comparisons/sec",
        "value": round(comps / sec / 1e9, 1),
        "unit": "G comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 bitwise (exact integer counts)", "data": "synthetic",
        "config": {"workload": f"batched: n={text.n} i.i.d. GC 0.41, {count} patterns, m ~ U{{16..2048}}, "
                               f"class density ~ U[0,0.3], k ~ U{{0..8}}, 2 plants each",
                   "hits": int(nh.sum()), "incomplete": int(st.sum()),
                   "group_size": cfg.group_size, "sub_ranges": cfg.sub_ranges, "lane_words": cfg.lane_words,
                   "autotune": tuned},
        # VALU lane-ops of the batch kernels per launch (committed counter run)
        # over their live duration
        "roofline": {"bound": "alu",
                     "achieved": None if valu is None else round(valu / (kern_ms / 1e3) / 1e12, 2),
                     "peak": valu_peak()["peak"], "unit": "T int32 VALU lane-ops/s",
                     "frac": None if valu is None else round(valu / (kern_ms / 1e3) / 1e12 / valu_peak()["peak"], 4),
                     "mix_ceiling": valu_peak()["mix"], "peak_source": valu_peak()["source"],
                     "traffic": None},
    }
    if not args.no_cpu_baseline:
        import oracle

        threads = host_threads()
        t0 = time.perf_counter()
        done = 0
        comps_cpu = 0.0
        win = 4_000_000
        for i in range(count):   # patterns in order, one window prefix each, ~10 s in all
            sets = oracle.parse(w.patterns[i])
            oracle.scan(w.text, sets, w.ks[i], threads=threads, win_end=win, capacity=1 << 16)
            comps_cpu += min(win, text.n - len(sets) + 1) * len(sets)
            done += 1
            if time.perf_counter() - t0 > 10.0:
                break
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(comps_cpu / dt / 1e9, 3), "unit": "G comparisons/s",
                                  "cores": threads, "cpu_count": os.cpu_count(), "kind": "oracle",
                                  "cpu": host_cpu_model(),
                                  "sample": f"first {done} patterns, windows [0, {win}) each, {dt:.1f} s"}
    return result


def serve(text, pats, ks, rate: float, duration: float, cfg, arena_gib: float, check_every: int = 32):
    """Serve queries from the pool (pats, ks; cycled) arriving as a Poisson
    process at `rate` per second for `duration` seconds through the native
    engine (continuous batching over revolving text chunks).  Returns the
    throughput over the whole run, the latency percentiles (completion minus
    scheduled arrival) and the queueing delay; every check_every-th query's
    result is compared with the plain kernel run alone on the same text."""
    import threading

    import numpy as np

    from paper_1611_06115_amd import scan, server, synth

    n = text.n
    arrivals = synth.poisson_arrivals(rate, duration)
    srv = server.Server(text, int(arena_gib * (1 << 30)), cfg)
    for i in range(4):  # warm-up through the whole path (not timed)
        srv.result(srv.submit(pats[i], ks[i]))
    st0 = srv.stats()
    nq = int(arrivals.size)
    npool = len(pats)
    ids = [0] * nq
    submitted = threading.Semaphore(0)
    start = server.now_ns() + 20_000_000

    def client():
        for i in range(nq):
            due = start + int(arrivals[i] * 1e9)
            while True:
                d = due - server.now_ns()
                if d <= 0:
                    break
                time.sleep(d / 1e9 - 1e-4 if d > 300_000 else 0)
            ids[i] = srv.submit(pats[i % npool], ks[i % npool], arrival_ns=due)
            submitted.release()

    th = threading.Thread(target=client, daemon=True)
    th.start()
    lat = np.zeros(nq)
    queue = np.zeros(nq)
    hits = np.zeros(nq, dtype=np.int64)
    last = start
    every = max(1, check_every)
    kept = {}
    done_log = time.perf_counter()
    for i in range(nq):
        submitted.acquire()
        info = srv.wait(ids[i])
        if info.state != server.DONE:
            raise SystemExit(f"query {i} failed with status {info.error}: {srv.error_detail()}")
        lat[i] = (info.complete_ns - info.arrival_ns) / 1e6
        queue[i] = (info.admit_ns - info.arrival_ns) / 1e6
        hits[i] = info.n_hits
        last = max(last, info.complete_ns)
        if i % every == 0:
            kept[i] = srv.result(ids[i])
        else:
            srv.release(ids[i])
        if time.perf_counter() - done_log > 5:
            log(f"[bench] {i + 1}/{nq} queries done")
            done_log = time.perf_counter()
    th.join()
    st = srv.stats()
    elapsed = (last - start) / 1e9
    ms_arr = np.array([p.m for p in pats], dtype=np.float64)
    idx = np.arange(nq) % npool
    comps = float(((n - ms_arr[idx] + 1).clip(min=0) * ms_arr[idx]).sum())
    log(f"[bench] {nq} queries in {elapsed:.2f}s, p50 {np.percentile(lat, 50):.1f} ms, "
        f"p99 {np.percentile(lat, 99):.1f} ms, {int(hits.sum())} hits, stats {st}")
    srv.close()
    # sampled queries: the result equals the plain kernel run alone, bit for bit
    for i, (pos, cnt) in kept.items():
        qi = i % npool
        a_pos, a_cnt = scan.scan(text, pats[qi], ks[qi])
        if not (torch_equal(a_pos, pos) and torch_equal(a_cnt, cnt)):
            raise SystemExit(f"query {i}: served result differs from the plain kernel alone")
    log(f"[bench] {len(kept)} sampled queries equal to the plain kernel alone")
    return {
        "value": round(comps / elapsed / 1e9, 1), "elapsed_s": round(elapsed, 3),
        "queries": nq, "qps_achieved": round(nq / elapsed, 1), "hits": int(hits.sum()),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2),
                       "p99": round(float(np.percentile(lat, 99)), 2),
                       "mean": round(float(lat.mean()), 2), "max": round(float(lat.max()), 2)},
        "queue_ms": {"p50": round(float(np.percentile(queue, 50)), 2),
                     "p99": round(float(np.percentile(queue, 99)), 2)},
        "stats": st, "stats0": st0, "kept": kept,
        "checked": f"{len(kept)} sampled queries equal to the plain kernel run alone",
    }


def torch_equal(a, b) -> bool:
    import torch

    return bool(torch.equal(a, b))


def run_served(args):
    """Queries from the pool arrive as a Poisson process at --qps for
    --duration seconds and are served by the native engine (continuous
    batching over revolving text chunks).  Reports the throughput in
    comparisons/s over the whole run and the latency percentiles of the
    queries (completion minus scheduled arrival)."""
    import torch

    from paper_1611_06115_amd import scan, server, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n or 3_100_000_000
    rate = float(args.qps)
    t0 = time.perf_counter()
    w = synth.served(n=n, count=args.count or 20000)
    pats = [scan.Pattern(p) for p in w.patterns]
    log(f"[bench] generated {n} bases and {len(pats)} pool queries in {time.perf_counter() - t0:.1f}s")
    text = scan.encode_text(torch.from_numpy(w.text).to(dev))
    torch.cuda.synchronize()
    text.check()
    cfg = server.ServerConfig(chunks=args.chunks or 0, max_active=args.slots or 0,
                              batch=scan.BatchConfig(args.group or 0, args.sub or 0, args.lane_words or 0, 0))
    res = serve(text, pats, w.ks, rate, args.duration, cfg, args.arena_gib)
    npool = len(pats)
    # the sampled queries' planted sites are found
    plant_of = {pi: (pos, d) for pi, pos, d in w.plants}
    for i, (pos, cnt) in res["kept"].items():
        ppos, _ = plant_of[i % npool]
        if not bool((pos == ppos).any()):
            raise SystemExit(f"query {i}: planted site {ppos} missed")
    st, st0 = res["stats"], res["stats0"]
    steps = st["steps"] - st0["steps"]
    result = {
        "metric": "G base-pattern comparisons/sec",
        "value": res["value"],
        "unit": "G comparisons/s",
        "n_gpus": 1, "steps": steps, "warmup": 4, "ms_per_step": round(res["elapsed_s"] * 1e3 / max(steps, 1), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 bitwise (exact integer counts)", "data": "synthetic",
        "latency_ms": res["latency_ms"],
        "queue_ms": res["queue_ms"],
        "config": {"workload": f"served: n={n} order-3 Markov GC 0.41 resident, Poisson arrivals at {rate:g}/s "
                               f"for {args.duration:g} s from a {npool}-query pool (m log-uniform 20..5000, "
                               f"k ~ U{{0..10}}, class density ~ U[0,0.3], one plant each)",
                   "queries": res["queries"], "qps_achieved": res["qps_achieved"], "elapsed_s": res["elapsed_s"],
                   "hits": res["hits"], "chunks": st["chunks"], "slots": cfg.max_active or 1024,
                   "arena_gib": args.arena_gib, "peak_active": st["peak_active"],
                   "reruns": st["reruns"] - st0["reruns"], "hit_slots_peak": st["hit_slots_peak"],
                   "checked": res["checked"]},
        "roofline": {"bound": "alu", "achieved": None, "peak": valu_peak()["peak"],
                     "unit": "T int32 VALU lane-ops/s", "frac": None, "traffic": None},
    }
    if not args.no_cpu_baseline:
        import oracle

        threads = host_threads()
        t0 = time.perf_counter()
        done = 0
        comps_cpu = 0.0
        win = 4_000_000
        for i in range(npool):   # pool queries in order, one window prefix each, ~10 s in all
            sets = oracle.parse(w.patterns[i])
            oracle.scan(w.text, sets, w.ks[i], threads=threads, win_end=win, capacity=1 << 16)
            comps_cpu += min(win, n - len(sets) + 1) * len(sets)
            done += 1
            if time.perf_counter() - t0 > 10.0:
                break
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(comps_cpu / dt / 1e9, 3), "unit": "G comparisons/s",
                                  "cores": threads, "cpu_count": os.cpu_count(), "kind": "oracle",
                                  "cpu": host_cpu_model(),
                                  "sample": f"first {done} pool queries, windows [0, {win}) each, {dt:.1f} s"}
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="genome", choices=["genome", "small", "long_m", "batched", "served", "mscale", "outofcore", "crt",
                             "sustained"])
    ap.add_argument("--count", type=int, default=None, help="batched: number of patterns")
    ap.add_argument("--group", type=int, default=None, help="batched, served: patterns per text tile")
    ap.add_argument("--sub", type=int, default=None, help="batched: text sub-ranges")
    ap.add_argument("--lane-words", type=int, default=None, help="batched: 4 or 6")
    ap.add_argument("--autotune", action="store_true", help="batched: tune the launch shape now")
    ap.add_argument("--n", type=int, default=None, help="override the text length")
    ap.add_argument("--qps", type=float, default=1000.0, help="served: arrival rate")
    ap.add_argument("--duration", type=float, default=10.0,
                    help="served: seconds of arrivals; sustained: seconds of back-to-back scans")
    ap.add_argument("--chunks", type=int, default=None, help="served: text chunks per revolution")
    ap.add_argument("--slots", type=int, default=None, help="served: queries scanned together")
    ap.add_argument("--arena-gib", type=float, default=64.0, help="served: device memory of the server")
    ap.add_argument("--chunk", type=int, default=None, help="outofcore: windows per chunk")
    ap.add_argument("--flush", action="store_true",
                    help="genome/small/long_m: write 512 MB before each timed step (cold Infinity Cache)")
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--settle", type=float, default=0.25,
                    help="genome/small/long_m: seconds of back-to-back steps before the warm-up (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", action="store_true", help="genome: skip the served-latency leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter scaling)")
    ap.add_argument("--valu-calibration", action="store_true",
                    help="only measure the VALU issue rates of the kernels' instructions (alu peaks)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.valu_calibration:
        valu_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the scan shards "
              "by text range with an m-1 overlap and no exchange, see the design notes", flush=True)
        raise SystemExit(2)
    run = {"batched": run_batched, "served": run_served, "mscale": run_mscale, "sustained": run_sustained,
           "outofcore": run_outofcore, "crt": run_crt}.get(args.workload, run_plain)
    res = run(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
