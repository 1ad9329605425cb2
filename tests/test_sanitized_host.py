"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

build.py's sanitizer build compiles the planner, the taper and the C ABI's
host code with clang's -fsanitize=address,undefined (no recovery); a child
process preloads clang's ASan runtime, loads that library through
IDG_LIBRARY and runs the host tests of the planner (integer parity with the
oracle's planner), the ABI's argument validation and the taper routines.  A
sanitizer report ends the child with a non-zero status.  No device call is
made.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

build = pytest.importorskip("paper_1909_07226_amd.build")


def _toolchain_or_skip():
    try:
        build._hipcc()
        build._clang()
        build.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    for src in ("kernels.hip", "image.hip", "calib.hip"):
        if not os.path.exists(os.path.join(build.BUILD, src.replace(".", "_") + ".o")):
            pytest.skip("plain build objects missing (run the plain build first)")


@pytest.fixture(scope="module")
def sanitized_lib():
    _toolchain_or_skip()
    return build.build_sanitized()


def _run_child(args, timeout):
    env = build.sanitizer_env()
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    return subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=timeout)


def test_sanitized_library_is_the_one_loaded(sanitized_lib):
    code = ("import paper_1909_07226_amd as idg, os\n"
            "assert idg._lib.LIB_PATH == os.environ['IDG_LIBRARY'], idg._lib.LIB_PATH\n"
            "idg._lib.lib()\n"
            "maps = open('/proc/self/maps').read()\n"
            "assert 'libclang_rt.asan' in maps and os.environ['IDG_LIBRARY'] in maps\n"
            "print('ok', idg.version())\n")
    res = _run_child(["-c", code], timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok")


def test_host_tests_pass_under_the_sanitizers(sanitized_lib):
    res = _run_child(["-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                      "tests/test_abi_host.py", "tests/test_taper_host.py", "-k", "not lofar_full"], timeout=900)
    out = res.stdout + res.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
