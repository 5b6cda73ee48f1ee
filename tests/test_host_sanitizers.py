"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The CPU tests of the C ABI (argument validation, workspace sizing, path
selection: everything that runs without a GPU) are run again in a child
process against the host-instrumented build of the library, with the
sanitizer runtime preloaded; any report ends that process with an error.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def hostsan():
    from paper_2309_05315_amd import build
    try:
        build.hipcc()
    except RuntimeError:
        pytest.skip("no HIP compiler")
    lib = build.hostsan_library()
    env = dict(os.environ, LD_PRELOAD=build.asan_runtime(), MAM_TEST_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return lib, env


def test_instrumented_library_is_the_one_loaded(hostsan):
    lib, env = hostsan
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2309_05315_amd import mam\n"
            "mam.LIB_PATH = %r\n"
            "L = mam.lib()\n"
            "maps = open('/proc/self/maps').read()\n"
            "assert %r in maps and 'libclang_rt.asan' in maps\n"
            "assert L.mam_abi_version() == 1\n"
            "print('ok')\n") % (ROOT, lib, os.path.basename(lib))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def test_abi_tests_pass_under_host_sanitizers(hostsan):
    _, env = hostsan
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert " passed" in r.stdout
