import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_sessionstart(session):
    """Build the libraries once if this checkout has none yet (a fresh clone):
    the tests load what is built and never rebuild what exists."""
    libs = [os.path.join(ROOT, "paper_2505_20911_amd", "libtgv.so"),
            os.path.join(ROOT, "paper_2505_20911_amd", "libtgv_probe.so"),
            os.path.join(ROOT, "oracle", "libtgv_oracle.so")]
    if not all(os.path.exists(p) for p in libs):
        import __graft_entry__
        __graft_entry__.build()
