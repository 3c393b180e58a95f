"""Host sanitizer runs (CPU only).

The FP64 oracles are rebuilt with gcc's AddressSanitizer and
UndefinedBehaviorSanitizer (every UB report fatal) and their pin suites run
against those copies; the C-ABI library is rebuilt with both sanitizers on
its host code and the ABI tests (argument checks, error codes, messages,
workspace sizing) run against it.  Each suite runs in a child process with
the matching sanitizer runtime preloaded (gcc's for the oracles, clang's for
the hipcc build); a sanitizer report fails the child and this test.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_MARKERS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _gcc_runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"gcc has no {name}")
    return path


def _clang_asan_runtime():
    c = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not c:
        pytest.skip("no clang ASan runtime under /opt/rocm/llvm")
    return c[-1]


def _run(env_extra, args, probe):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    # the child really maps the sanitised library and the ASan runtime
    p = subprocess.run([sys.executable, "-c", probe + "; m = open('/proc/self/maps').read(); "
                        "print(sum(x in m for x in ('libasan', 'libclang_rt.asan')), lib)"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout + p.stderr
    n, lib = p.stdout.split()[-2:]
    assert int(n) >= 1 and lib in env_extra.values(), p.stdout
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *args], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for m in SAN_MARKERS:
        assert m not in out, out[-4000:]
    return out


@pytest.mark.slow
def test_oracles_under_asan_ubsan(tmp_path):
    import oracle.oracle as OO
    from oracle import variants as OV
    lib = OO.build_oracle(force=True, sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    vlib = OV.build_var_oracle(force=True, sanitize=True, out=str(tmp_path / "liboracle_var_san.so"))
    pre = _gcc_runtime("libasan.so") + ":" + _gcc_runtime("libubsan.so")
    out = _run({"LD_PRELOAD": pre, "EFUNC_ORACLE_LIB": lib, "EFUNC_ORACLE_VAR_LIB": vlib},
               ["tests/test_oracle_pins.py", "tests/test_oracle_var_pins.py"],
               "import oracle.oracle as O; O.load(); lib = O._lib._name")
    assert " passed" in out


@pytest.mark.slow
def test_c_abi_host_code_under_asan_ubsan(tmp_path):
    from paper_2505_21319_amd import build as B
    lib = B.build(sanitize=True, out=str(tmp_path / "libefunc_san.so"))
    out = _run({"LD_PRELOAD": _clang_asan_runtime(), "EFUNC_LIBRARY": lib}, ["tests/test_abi.py"],
               "from paper_2505_21319_amd import efunc as E; lib = E.lib()._name")
    assert " passed" in out
