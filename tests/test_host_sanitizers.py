"""Host AddressSanitizer / UndefinedBehaviorSanitizer runs (CPU only).

The C oracle and the host side of libmdx (argument validation, size queries,
workspace plans) are rebuilt with ASan and UBSan, the device code unchanged
and never launched, and the host-only tests run against those builds in a
child process that preloads clang's ASan runtime.  Both libraries use the
same clang runtime, so one process holds them together.

The child runs in a copy of the tree whose libmdx.so and liboracle.so are the
sanitized builds; the working tree's libraries are left alone.  A planted
out-of-bounds read in a throwaway C file shows that the setup reports errors
rather than passing silently.
"""

import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
_RT = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
ASAN_RT = _RT[-1] if _RT else None

# host-side instrumentation only: each sanitizer flag is scoped to the host pass
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-shared-libasan"]
C_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
         "-shared-libasan"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

pytestmark = pytest.mark.skipif(
    not (ASAN_RT and os.path.exists(CLANG) and os.path.exists(HIPCC)),
    reason="clang ASan runtime or hipcc not installed")


def _env():
    env = dict(os.environ)
    env.update(SAN_ENV)
    env["LD_PRELOAD"] = ASAN_RT
    env.pop("PYTHONPATH", None)
    return env


def _build_mdx(out):
    sys.path.insert(0, ROOT)
    from paper_2101_08878_amd import build as B
    sys.path.pop(0)
    flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"] + HOST_SAN
    cmd = [HIPCC, *flags, "-I", os.path.join(ROOT, "include"), "-I", B.CSRC, "-x", "hip",
           *[os.path.join(B.CSRC, s) for s in B.SOURCES], "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)


def _build_oracle(out):
    cmd = [CLANG, "-std=c11", "-O1", "-g", "-fPIC", "-shared", "-pthread", *C_SAN,
           "-o", out, os.path.join(ROOT, "oracle", "oracle.c")]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)


@pytest.fixture(scope="module")
def san_tree(tmp_path_factory):
    """A copy of the sources and host tests with sanitized libraries in place."""
    t = tmp_path_factory.mktemp("san")
    pkg = t / "paper_2101_08878_amd"
    pkg.mkdir()
    for f in glob.glob(os.path.join(ROOT, "paper_2101_08878_amd", "*.py")):
        shutil.copy(f, pkg)
    (t / "oracle").mkdir()
    for f in ["__init__.py", "build.py", "oracle.c"]:
        shutil.copy(os.path.join(ROOT, "oracle", f), t / "oracle")
    shutil.copytree(os.path.join(ROOT, "include"), t / "include")
    shutil.copytree(os.path.join(ROOT, "workloads"), t / "workloads",
                    ignore=shutil.ignore_patterns("__pycache__"))
    (t / "tests").mkdir()
    for f in ["conftest.py", "helpers.py", "test_abi_cpu.py", "test_oracle_pins.py"]:
        shutil.copy(os.path.join(ROOT, "tests", f), t / "tests")
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), t / "tests" / "golden")
    _build_mdx(str(pkg / "libmdx.so"))
    _build_oracle(str(t / "oracle" / "liboracle.so"))
    return t


def test_sanitizer_setup_reports_a_planted_overflow(tmp_path):
    src = tmp_path / "oob.c"
    src.write_text(
        "#include <stdlib.h>\n"
        "int oob_read(int n) { int *a = malloc(n * sizeof(int)); int v; a[0] = 1; v = a[n]; free(a);"
        " return v; }\n")
    lib = tmp_path / "liboob.so"
    subprocess.run([CLANG, "-O0", "-g", "-fPIC", "-shared", *C_SAN, "-o", str(lib), str(src)],
                   check=True, capture_output=True, timeout=120)
    code = f"import ctypes; ctypes.CDLL({str(lib)!r}).oob_read(4)"
    r = subprocess.run([sys.executable, "-c", code], env=_env(), capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr


def test_host_tests_pass_under_asan_and_ubsan(san_tree):
    r = subprocess.run(
        [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
         "tests/test_abi_cpu.py", "tests/test_oracle_pins.py"],
        cwd=str(san_tree), env=_env(), capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr, tail
    assert "runtime error" not in r.stderr, tail
