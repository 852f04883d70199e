"""CPU-only sanitizer runs: the oracle and the library's host code built with
AddressSanitizer and UndefinedBehaviorSanitizer (the library's device code is
built as usual and never launched here), then the oracle's pin tests and the
C-ABI host checks (configuration validation, workspace sizing, argument and
state errors, the seeded config fuzz) run against those builds in a child
process with the sanitizer runtime preloaded.  Any report ends the child and
fails the test.

A first test plants a heap overflow and a signed overflow in a small C
library and checks that this set-up reports both, so a silent pass means the
runtime was really there.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LLVM = "/opt/rocm/llvm"
HIPCC = "/opt/rocm/bin/hipcc"


def _runtime():
    hits = sorted(glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    return hits[-1] if hits else None


RT = _runtime()
pytestmark = pytest.mark.skipif(RT is None or not os.path.exists(HIPCC), reason="clang sanitizer runtime or hipcc missing")

SAN_C = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libsan"]
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-shared-libsan"]


def _env(logdir):
    env = dict(os.environ)
    env["LD_PRELOAD"] = RT
    env["ASAN_OPTIONS"] = f"detect_leaks=0:halt_on_error=1:log_path={logdir}/asan"
    env["UBSAN_OPTIONS"] = f"halt_on_error=1:print_stacktrace=1:log_path={logdir}/ubsan"
    return env


def _reports(logdir):
    out = []
    for p in sorted(glob.glob(os.path.join(logdir, "*san.*"))):
        out.append(open(p).read())
    return "\n".join(out)


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    oracle_so = str(d / "liboracle_san.so")
    subprocess.check_call([os.path.join(LLVM, "bin", "clang"), "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer",
                           "-ffp-contract=off", "-fPIC", "-shared"] + SAN_C +
                          ["-o", oracle_so, os.path.join(ROOT, "oracle", "avl_oracle.c"), "-lm"])
    from paper_1804_03901_amd import build as avl_build
    lib_so = str(d / "libavl_san.so")
    csrc = os.path.join(ROOT, "paper_1804_03901_amd", "csrc")
    subprocess.check_call([HIPCC, f"--offload-arch={avl_build.ARCH}", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                           "-fvisibility=hidden", "-ffp-contract=off", "-fno-omit-frame-pointer",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SAN_HOST +
                          ["-I", os.path.join(ROOT, "include")] +
                          [os.path.join(csrc, s) for s in avl_build.SOURCES] + ["-o", lib_so],
                          stderr=subprocess.DEVNULL)
    return d, oracle_so, lib_so


def test_planted_errors_are_reported(builds):
    d = builds[0]
    src = d / "planted.c"
    src.write_text(textwrap.dedent("""
        #include <stdlib.h>
        int heap_over(int n) { int* p = malloc(sizeof(int) * n); p[n] = 1; int r = p[0]; free(p); return r; }
        int int_over(int a) { return a * a * a; }
    """))
    so = str(d / "libplanted.so")
    subprocess.check_call([os.path.join(LLVM, "bin", "clang"), "-O0", "-g", "-fPIC", "-shared"] + SAN_C +
                          ["-o", so, str(src)])
    for fn, arg, word in (("heap_over", 4, "heap-buffer-overflow"), ("int_over", 1 << 20, "signed integer overflow")):
        logdir = d / f"log_{fn}"
        logdir.mkdir()
        code = f"import ctypes; ctypes.CDLL({so!r}).{fn}({arg})"
        r = subprocess.run([sys.executable, "-c", code], env=_env(logdir), capture_output=True, text=True)
        assert r.returncode != 0, fn
        assert word in _reports(logdir) + r.stderr, fn


def test_oracle_pins_and_host_checks_under_sanitizers(builds):
    d, oracle_so, lib_so = builds
    logdir = d / "log_suite"
    logdir.mkdir()
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py"))) + [os.path.join(ROOT, "tests", "test_abi.py")]
    code = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        import pytest
        import oracle
        oracle._LIB = {oracle_so!r}
        from paper_1804_03901_amd import avl
        avl.load.__defaults__ = ({lib_so!r},)
        rc = pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + {files!r})
        maps = open("/proc/self/maps").read()
        assert {oracle_so!r} in maps and {lib_so!r} in maps, "sanitized builds not loaded"
        sys.exit(int(rc))
    """)
    r = subprocess.run([sys.executable, "-c", code], env=_env(logdir), capture_output=True, text=True, cwd=ROOT)
    rep = _reports(logdir)
    assert r.returncode == 0 and not rep, (r.stdout[-3000:], r.stderr[-3000:], rep[-3000:])
    assert " passed" in r.stdout
