"""A client that uses only the C ABI and the HIP runtime (no Python, no
PyTorch: tests/c_client/pm_client.cpp) gets the oracle's hit lists."""
import os
import random
import subprocess

import numpy as np
import pytest

from conftest import ROOT
from test_gpu_parity import oracle_hits, plant_copies, rand_pattern, random_text

torch = pytest.importorskip("torch")

CLIENT = os.path.join(ROOT, "tests", "c_client", "pm_client")


def run_client(path, pattern, k):
    out = subprocess.run([CLIENT, path, pattern, str(k)], capture_output=True, text=True, timeout=120)
    return out.returncode, out.stdout, out.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("m,k,cf", [(12, 0, 0.2), (90, 4, 0.25), (700, 20, 0.1), (6, 0, 1.0)])
def test_c_client_matches_oracle(tmp_path, m, k, cf):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(CLIENT):
        pytest.fail("tests/c_client/pm_client is not built (run __graft_entry__.build())")
    rnd = random.Random(m * 17 + k)
    text = random_text(rnd, 200_003)
    pat = rand_pattern(rnd, m, cf, "ACGTMRWSYKVHDBN") if cf < 1.0 else "N" * m  # the last: every window
    plant_copies(rnd, text, pat, 30, k)
    path = tmp_path / "text.txt"
    path.write_bytes(text.tobytes())
    print(f"c client m={m} k={k}", flush=True)
    rc, out, err = run_client(str(path), pat, k)
    assert rc == 0, err
    rows = [tuple(int(x) for x in line.split()) for line in out.splitlines()]
    pos = np.array([r[0] for r in rows], dtype=np.int64)
    cnt = np.array([r[1] for r in rows], dtype=np.uint16)
    wp, wc = oracle_hits(text, pat, k)
    assert np.array_equal(pos, wp) and np.array_equal(cnt, wc)
    if cf == 1.0:
        assert pos.size == text.size - m + 1 > 1024  # the re-run with an exact buffer


def test_c_client_host_errors(tmp_path):
    """Errors found on the host come back as status codes, before any device
    call (this runs without a GPU)."""
    if not os.path.exists(CLIENT):
        pytest.skip("client not built")
    out = subprocess.run([CLIENT], capture_output=True, text=True, timeout=60)
    assert out.returncode == 2 and "usage" in out.stderr
    path = tmp_path / "t.txt"
    path.write_bytes(b"ACGT" * 10)
    rc, _, err = run_client(str(path), "AC[GT", 0)
    assert rc == 1 and "pm_encode_pattern" in err
