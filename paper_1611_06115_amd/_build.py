"""Build libpmscan.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpmscan.so")
SOURCES = ["pmscan.hip", "plan.cpp", "batch.hip", "server.hip", "hostscan.hip", "ntt.hip", "fasta.cpp", "fasta_scan.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
]


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(extra: list[str] | None = None, out: str = LIB) -> str:
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *(extra or []), "-I", os.path.join(HERE, "..", "include"),
           *sources(), "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


CALIB_LIB = os.path.join(HERE, "libpmcalib.so")


def build_calib() -> str:
    """The VALU issue-rate probe (csrc/calib.hip) used by
    bench.py --valu-calibration; not part of the scan library."""
    tmp = CALIB_LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, os.path.join(CSRC, "calib.hip"), "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, CALIB_LIB)
    return CALIB_LIB


def build_c_client() -> str:
    """The test client that uses only the C ABI (tests/c_client), linked to
    the library in place."""
    src = os.path.join(HERE, "..", "tests", "c_client", "pm_client.cpp")
    out = os.path.join(HERE, "..", "tests", "c_client", "pm_client")
    if not os.path.exists(src):
        return ""
    cmd = [HIPCC, "-O2", "-std=c++17", "-Wall", "-I", os.path.join(HERE, "..", "include"), src,
           "-L", HERE, "-lpmscan", "-Wl,-rpath,$ORIGIN/../../paper_1611_06115_amd", "-o", out + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1:]))
