"""The benchmark's output contract on the GPU (small sizes), and the
kernel-timing hook it relies on."""
import json
import os
import subprocess
import sys

import pytest

from conftest import ROOT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run_bench(*args, timeout=240):
    out = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                         capture_output=True, text=True, timeout=timeout)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [l for l in out.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1, out.stdout
    return json.loads(lines[0])


def check_contract(r):
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in r, key
    assert r["n_gpus"] == 1 and r["value"] > 0 and r["ms_per_step"] > 0
    assert "workload" in r["config"]
    rl = r["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in rl, key
    assert rl["bound"] in ("hbm", "mfma", "alu")


def test_bench_plain_contract():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = run_bench("--workload", "small", "--steps", "3", "--warmup", "1")
    check_contract(r)
    assert r["roofline"]["bound"] == "hbm" and 0 < r["roofline"]["frac"] < 1.5
    cb = r["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0


def test_bench_genome_line_carries_latency_and_the_oracle_check():
    """The default workload's line: the scan's roofline, the oracle on every
    host core with its list compared to the GPU's, and the served form's
    p50/p99 on the same resident text."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = run_bench("--workload", "genome", "--n", "20000000", "--steps", "3", "--warmup", "1", timeout=400)
    check_contract(r)
    assert r["roofline"]["bound"] == "hbm"
    cb = r["cpu_baseline"]
    assert cb["cores"] == len(os.sched_getaffinity(0)) and cb["cpu_count"] >= cb["cores"]
    assert "equals the oracle's" in r["config"]["oracle_check"]
    st = r["config"]["settle"]
    assert st["steps"] > 0 and st["first_block_ms_per_step"] > 0
    lat = r["latency_ms"]
    assert 0 < lat["p50"] <= lat["p99"] <= lat["max"]
    assert r["config"]["served"]["queries"] > 1000


def test_bench_served_contract():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = run_bench("--workload", "served", "--n", "30000000", "--count", "500", "--qps", "200", "--duration", "1",
                  "--arena-gib", "4", "--no-cpu-baseline")
    check_contract(r)
    lat = r["latency_ms"]
    assert 0 < lat["p50"] <= lat["p99"] <= lat["max"]
    assert r["config"]["queries"] > 50


def test_bench_mscale_and_outofcore_contract():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = run_bench("--workload", "mscale", "--n", "2000000", "--warmup", "1", "--no-cpu-baseline")
    check_contract(r)
    assert set(r["config"]["per_m_ms"]) == {"500", "10000", "100000"} and len(r["config"]["rows"]) == 15
    r = run_bench("--workload", "outofcore", "--n", "40000000", "--chunk", "5000000", "--steps", "2")
    check_contract(r)
    link = r["config"]["link"]
    assert link["achieved"] > 0 and link["copy_alone"] > 0 and 0 < link["frac"] <= 1.5
    assert r["cpu_baseline"]["kind"] == "oracle"


def test_bench_crt_contract():
    """The transform-route line (its counts at or below k are checked
    against the scan's hits inside the bench)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = run_bench("--workload", "crt", "--n", "3000000", "--steps", "2", "--warmup", "1", "--no-cpu-baseline")
    check_contract(r)
    c = r["config"]
    assert c["ls_direct_uint64_max_m"] == 240 and c["windows"] == 3_000_000 - 1024 + 1 and c["scan_ms"] > 0


def test_time_next_scan_brackets_the_count_kernel():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1611_06115_amd import scan, synth

    w = synth.small(n=2_000_000)
    t = scan.encode_text(w.text)
    pat = scan.Pattern(w.patterns[0])
    ws = scan.Workspace(t.data.device, t.n, 1 << 16)
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    b.record(s)
    e0.record(s)
    scan.time_next_scan(a, b)
    scan.scan_async(t, pat, 2, ws)
    e1.record(s)
    e1.synchronize()
    k_ms, step_ms = a.elapsed_time(b), e0.elapsed_time(e1)
    assert 0 < k_ms <= step_ms
    import ctypes

    with pytest.raises(scan.PMError):  # both events or neither
        scan.check(scan.lib().pm_time_next_scan(None, ctypes.c_void_p(b.cuda_event)))


def test_bench_sustained_run():
    """The from-idle run behind the settle phase: per-block step times, the
    first 200 steps apart from the rest."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = run_bench("--workload", "sustained", "--n", "20000000", "--duration", "0.05")
    check_contract(r)
    c = r["config"]
    assert c["steps_1_200_ms_per_step"]["mean"] > 0 and c["after_200_ms_per_step"]["mean"] > 0
    assert len(c["blocks_of_200_steps_ms"]) >= 1 and r["steps"] >= 200
