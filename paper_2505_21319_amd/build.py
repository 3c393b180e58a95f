"""Build libefunc.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libefunc.so")
SOURCES = [os.path.join(HERE, "csrc", "efunc_kernels.hip"),
           os.path.join(HERE, "csrc", "efunc_capi.hip"),
           os.path.join(HERE, "csrc", "efunc_batch.hip"),
           os.path.join(HERE, "csrc", "initnet.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


# Host-code AddressSanitizer + UndefinedBehaviorSanitizer for the C ABI; the
# device code is built as usual (-Xarch_host keeps the sanitizers off it).
# Load the result with clang's ASan runtime preloaded.
SANITIZE_FLAGS = ["-O1", "-g", "-Xarch_host", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def build(verbose: bool = False, sanitize: bool = False, out: str = None) -> str:
    out = out or LIB
    tmp = out + ".tmp"
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + SANITIZE_FLAGS if sanitize else HIPCC_FLAGS
    cmd = [hipcc(), *flags, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(HERE, "csrc"), "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
