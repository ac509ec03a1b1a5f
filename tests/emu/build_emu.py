"""Build liblks_emu.so: the library's own sources compiled for the host against the HIP stand-in in
this folder, with AddressSanitizer.  TEST INFRASTRUCTURE ONLY (CPU; never loaded on a GPU).

The sources are compiled unchanged except for one mechanical rewrite: a dynamic LDS declaration
`extern __shared__ ... NAME[];` becomes a pointer to the launch's guarded LDS allocation.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2506_23895_amd", "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liblks_emu.so")
SOURCES = ["lks_api.hip", "lks_kernels2d.hip", "lks_kernels3d.hip", "lks_kernels_common.hip",
           "lks_kernels2d_paper.hip"]
FLAGS = ["-std=c++20", "-O1", "-g", "-fPIC", "-fno-omit-frame-pointer", "-fsanitize=address",
         "-Wno-attributes", "-Wno-ignored-attributes", "-I", HERE, "-I", os.path.join(ROOT, "include"),
         "-I", CSRC]

_DYN_LDS = re.compile(r"extern\s+__shared__\s+(?:__align__\(\d+\)\s+)?unsigned\s+char\s+(\w+)\[\];")


def rewrite(src: str) -> str:
    return _DYN_LDS.sub(r"unsigned char *\1 = emu::dyn_lds();", src)


def _stale(out: str, deps) -> bool:
    return not os.path.exists(out) or any(os.path.getmtime(d) > os.path.getmtime(out) for d in deps)


def build(force: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    headers += [os.path.join(HERE, "hip", "hip_runtime.h"), os.path.join(ROOT, "include", "lks.h")]
    objs, procs = [], []
    for s in SOURCES + ["emu_runtime.cpp"]:
        src = os.path.join(CSRC, s) if s.endswith(".hip") else os.path.join(HERE, s)
        cpp = os.path.join(OUT_DIR, os.path.splitext(s)[0] + ".cpp")
        obj = os.path.join(OUT_DIR, os.path.splitext(s)[0] + ".o")
        with open(src) as f:
            text = rewrite(f.read())
        if not os.path.exists(cpp) or open(cpp).read() != text:
            with open(cpp, "w") as f:
                f.write(text)
        objs.append(obj)
        if force or _stale(obj, [cpp] + headers):
            procs.append(subprocess.Popen(["g++", *FLAGS, "-c", cpp, "-o", obj]))
    if any(p.wait() != 0 for p in procs):
        raise RuntimeError("emulator build failed")
    if force or _stale(LIB, objs):
        subprocess.check_call(["g++", "-shared", "-fsanitize=address", "-o", LIB, *objs])
    return LIB


def asan_env() -> dict:
    env = dict(os.environ)
    env["LD_PRELOAD"] = subprocess.check_output(["gcc", "-print-file-name=libasan.so"]).decode().strip()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:detect_stack_use_after_return=0:verify_asan_link_order=0"
    return env


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
