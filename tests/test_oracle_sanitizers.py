"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code; the oracle has no GPU code): the library is rebuilt with both
sanitizers, undefined behaviour made fatal, and a representative set of the
oracle's own pin tests runs against it in a child process with the ASan
runtime preloaded.  Out-of-bounds or use-after-free accesses and undefined
behaviour (signed overflow, bad shifts, misaligned or null accesses) abort
the child and fail this test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# every oracle code path: the 2-D schemes and options, sides, multi-block
# grids, 3-D, the forward/reverse modes and the operation count
SUBSET = [
    "tests/test_oracle_schemes.py",
    "tests/test_oracle_euler.py::test_sod_matches_exact_riemann_solution",
    "tests/test_oracle_cfl.py",
    "tests/test_oracle_adjoint.py",
    "tests/test_oracle_boundaries.py",
    "tests/test_oracle_multiblock.py",
    "tests/test_oracle_3d.py::test_free_stream_preserved",
    "tests/test_oracle_3d.py::test_z_independent_data_reduce_to_the_2d_scheme",
    "tests/test_oracle_variants.py",
    "tests/test_oracle_seventh.py",
]


def test_oracle_tests_pass_under_asan_and_ubsan(tmp_path):
    from oracle import build
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime")
    lib = build.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ)
    env.update(ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="8")
    tests = [t for t in SUBSET if os.path.exists(os.path.join(ROOT, t.split("::")[0]))]
    # the long refinement studies (Shu-Osher, Table 3) are left to the
    # regular run: their code paths are the ones the other tests exercise
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        "-k", "not shu_osher and not table3", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=3000)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
