import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_sessionstart(session):
    # the host-sanitizer run (tests/test_host_sanitizers.py) points the
    # binding at the instrumented build of the library
    lib = os.environ.get("MAM_TEST_LIBRARY")
    if lib:
        from paper_2309_05315_amd import mam
        mam.LIB_PATH = lib
