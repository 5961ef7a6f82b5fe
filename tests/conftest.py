import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def golden_lines(name):
    """Non-comment lines of a golden fixture, split into fields."""
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


def golden_dict(name):
    d = {}
    for fields in golden_lines(name):
        d.setdefault(fields[0], []).append(fields[1:])
    return d


@pytest.fixture(scope="session", autouse=True)
def _native_helpers_built():
    import oracle
    from paper_1611_06115_amd import synth

    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    if not os.path.exists(os.path.join(ROOT, "paper_1611_06115_amd", "libpmsynth.so")):
        synth.build()
