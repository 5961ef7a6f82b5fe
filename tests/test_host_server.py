"""Host side of the query server ABI (no GPU): struct layouts shared with the
Python binding, argument checks and arena sizing."""
import ctypes
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

scan = pytest.importorskip("paper_1611_06115_amd.scan")
server = pytest.importorskip("paper_1611_06115_amd.server")


@pytest.fixture(scope="module", autouse=True)
def built_library():
    if not os.path.exists(scan.LIB_PATH):
        from paper_1611_06115_amd import _build

        _build.build()
    scan.lib()


C_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "pmscan.h"
#define F(T, f) printf("%s.%s %zu\n", #T, #f, offsetof(T, f))
int main(void) {
    printf("pm_batch_config %zu\n", sizeof(pm_batch_config));
    printf("pm_server_config %zu\n", sizeof(pm_server_config));
    printf("pm_query_info %zu\n", sizeof(pm_query_info));
    printf("pm_server_stats %zu\n", sizeof(pm_server_stats));
    F(pm_server_config, workspace_bytes); F(pm_server_config, batch);
    F(pm_query_info, n_hits); F(pm_query_info, pos_dev); F(pm_query_info, cnt_dev);
    F(pm_query_info, arrival_ns); F(pm_query_info, complete_ns); F(pm_query_info, reruns);
    F(pm_server_stats, comparisons); F(pm_server_stats, active); F(pm_server_stats, chunks);
    F(pm_server_stats, hit_slots); F(pm_server_stats, workspace_bytes);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(C_PROBE)
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    types = {"pm_batch_config": scan.BatchConfig, "pm_server_config": server.ServerConfig,
             "pm_query_info": server.QueryInfo, "pm_server_stats": server.ServerStats}
    for key, value in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(types[t], f).offset == int(value), key
        else:
            assert ctypes.sizeof(types[key]) == int(value), key


def test_create_rejects_bad_arguments():
    L = scan.lib()
    h = ctypes.c_void_p()
    # null pointers
    assert L.pm_server_create(None, 1000, ctypes.c_void_p(256), 1 << 20, None, None, ctypes.byref(h)) == -1
    # misaligned arena
    assert L.pm_server_create(ctypes.c_void_p(256), 1000, ctypes.c_void_p(300), 1 << 20, None, None,
                              ctypes.byref(h)) == -1
    # arena below the minimum (checked before any device call)
    small = server.min_arena_bytes(10 ** 6) - 256
    assert L.pm_server_create(ctypes.c_void_p(256), 10 ** 6, ctypes.c_void_p(4096), small, None, None,
                              ctypes.byref(h)) == -4
    assert b"arena too small" in L.pm_last_error_detail()
    assert not h.value


def test_min_arena_grows_with_text_and_chunks():
    a = server.min_arena_bytes(10 ** 6)
    b = server.min_arena_bytes(10 ** 8)
    c = server.min_arena_bytes(10 ** 8, server.ServerConfig(chunks=64))
    d = server.min_arena_bytes(10 ** 8, server.ServerConfig(max_active=4096))
    assert 0 < a < b < c and b < d
    # the plain-kernel re-scan workspace of the whole text is part of it
    assert b > scan.workspace_bytes(10 ** 8)


def test_server_clock_is_monotonic():
    t = [server.now_ns() for _ in range(100)]
    assert all(x <= y for x, y in zip(t, t[1:])) and t[0] > 0


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys

    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stdout


def test_bench_run_time_inputs_match_the_kernels():
    """The committed counter runs that bench.py reads at run time (traffic
    and VALU figures) exist and were taken on the current kernel sources."""
    import json
    import sys

    sys.path.insert(0, ROOT)
    import bench

    for rel, wl in (("profiles/scan_genome_traffic.json", "genome"), ("profiles/scan_batched_valu.json", "batched")):
        with open(os.path.join(ROOT, rel)) as f:
            assert json.load(f)["kernel_source_sha"] == bench.kernel_source_sha(wl), rel
