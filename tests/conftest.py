import os
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Host set-up tables are cached on disk between the plans of one test run
# (the same nside is planned many times; nside 2048 takes about a minute to
# build).  A library rebuild invalidates the files.
if "HP2SPH_TABLE_CACHE" not in os.environ:
    _cache = os.path.join(tempfile.gettempdir(), f"hp2sph_tables_{os.getuid()}")
    os.makedirs(_cache, exist_ok=True)
    os.environ["HP2SPH_TABLE_CACHE"] = _cache


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
