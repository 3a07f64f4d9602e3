"""Build a copy of libpilot.so whose host runtime is compiled with
AddressSanitizer and UndefinedBehaviorSanitizer.

The host runtime (csrc/pilot_runtime.cpp: argument validation, planning,
workspace layout, the graph cache, the serving slots) is compiled by g++ with
the sanitizers and linked with the normal build's HIP objects (kernels and
their launchers, unchanged).  The copy is for host-side checks only: load it
through PILOT_LIB_OVERRIDE with gcc's libasan and libstdc++ preloaded, e.g.

    python -m paper_2606_31098_amd.build_host_sanitized /tmp/san
    LD_PRELOAD="$(gcc -print-file-name=libasan.so) $(gcc -print-file-name=libstdc++.so.6)" \\
    ASAN_OPTIONS=detect_leaks=0:verify_asan_link_order=0 UBSAN_OPTIONS=halt_on_error=1 \\
    PILOT_LIB_OVERRIDE=/tmp/san/libpilot.so python -m pytest tests -m gpu

(libstdc++ is preloaded so that the sanitizer finds the C++ runtime's throw
routine; torch's own library folder must be on LD_LIBRARY_PATH, because a
library opened through the sanitizer's dlopen no longer sees its caller's
runpath.)  The normal build must exist first (its objects are reused).
"""
from __future__ import annotations

import os
import subprocess
import sys

from . import build as B

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def build_host_sanitized(out_dir: str, runtime_src: str | None = None) -> str:
    """Build out_dir/libpilot.so; runtime_src replaces csrc/pilot_runtime.cpp
    (a modified copy, for the test that plants a mistake)."""
    hip_objs = [os.path.join(B.OBJ, os.path.basename(s) + ".o") for s in B.sources() if s.endswith(".hip")]
    missing = [o for o in hip_objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"build the library first (python -m paper_2606_31098_amd.build): missing {missing}")
    os.makedirs(out_dir, exist_ok=True)
    rt = runtime_src or os.path.join(B.CSRC, "pilot_runtime.cpp")
    rt_obj = os.path.join(out_dir, "pilot_runtime_san.o")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include",
                    f"-I{B.CSRC}", "-Wno-unused-result", *SAN, "-c", rt, "-o", rt_obj], check=True)
    so = os.path.join(out_dir, "libpilot.so")
    lib = os.path.realpath(os.path.join(rocm, "lib"))
    subprocess.run(["g++", "-shared", "-fPIC", *SAN, "-o", so, *hip_objs, rt_obj, f"-L{lib}", f"-Wl,-rpath,{lib}",
                    "-lamdhip64"], check=True)
    return so


if __name__ == "__main__":
    print(build_host_sanitized(sys.argv[1] if len(sys.argv) > 1 else os.path.join(B.HERE, "_build", "san")))
