import os
import sys

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if REPO not in sys.path:
    sys.path.insert(0, REPO)
GOLDEN = os.path.join(REPO, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running (full-size workloads)")


def _ensure_built():
    """Build what is missing (and only that); __graft_entry__.build() compiles everything."""
    if not os.path.exists(os.path.join(REPO, "oracle", "liboracle.so")):
        from oracle import build as ob
        ob.build()
    if not os.path.exists(os.path.join(REPO, "paper_1208_5542_amd", "librmat.so")):
        from paper_1208_5542_amd import _build
        _build.build_rmat()


_ensure_built()


@pytest.fixture(scope="session")
def golden():
    import json

    def load(name):
        with open(os.path.join(GOLDEN, name)) as f:
            return json.load(f)
    return load
