import os
import shutil
import sys
import tempfile


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_CACHE_DIR = None


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
    # the library's disk caches (code objects and autotuned geometries) live in
    # a directory of this session, so no state left by an earlier process can
    # change what a test runs
    global _CACHE_DIR
    _CACHE_DIR = tempfile.mkdtemp(prefix="hipmr_test_cache_")
    os.environ["HIPMR_CACHE_DIR"] = _CACHE_DIR


def pytest_unconfigure(config):
    if _CACHE_DIR:
        shutil.rmtree(_CACHE_DIR, ignore_errors=True)
