"""Builds libtucker_als.so for gfx950 with hipcc (in-tree).

Every source is compiled to an object of its own, in parallel, and the objects
are linked into the shared library.

``--sanitize`` builds ``libtucker_als_san.so`` instead (objects in
``_build_san``): the host code compiled with AddressSanitizer and
UndefinedBehaviorSanitizer (``-Xarch_host`` before each ``-fsanitize=``, so the
device code is built as usual), for running the argument-validation tests on
the CPU with the sanitizer runtime preloaded (``SANITIZER_RUNTIME`` names it).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtucker_als.so")
OBJ_SAN = os.path.join(HERE, "_build_san")
LIB_SAN = os.path.join(HERE, "libtucker_als_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
SANITIZER_RUNTIME = "/opt/rocm/lib/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"
SOURCES = ["tk_api.hip", "k_small_la.hip", "k_mode_step.hip", "k_stream.hip", "k_fused.hip",
           "k_fused_bf16.hip", "k_fused_big.hip", "k_fused_bf16_big.hip", "k_batched.hip",
           "k_svec.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = ["--offload-arch=gfx950"]
COMPILE = ARCH + [
    "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions (a device
    # feature; the host pass does not know it and prints one line per source
    # saying it ignores it, which _quiet drops)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
]
HOST_IGNORED = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"


def _quiet(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if l.strip() != HOST_IGNORED)


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = _quiet(r.stdout + r.stderr)
    return r.returncode, out


def _stale(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(HERE, "..", "include", "tucker_als.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False,
          sanitize: bool = False) -> str:
    """Compiles every source (only the out-of-date ones with ``incremental``)
    and links the library (the sanitizer build with ``sanitize``)."""
    obj_dir, lib = (OBJ_SAN, LIB_SAN) if sanitize else (OBJ, LIB)
    extra = SAN_FLAGS if sanitize else []
    os.makedirs(obj_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    objs = [os.path.join(obj_dir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[HIPCC] + COMPILE + extra + ["-c", os.path.join(CSRC, s), "-o", o]
            for s, o in zip(SOURCES, objs)
            if not incremental or _stale(os.path.join(CSRC, s), o)]
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        results = list(ex.map(lambda c: _run(c, verbose), cmds))
    failed = False
    for (rc, out), cmd in zip(results, cmds):
        if out.strip():
            sys.stderr.write(f"--- {os.path.basename(cmd[-3])}\n{out}\n")
        failed |= rc != 0
    if failed:
        raise RuntimeError("hipcc failed compiling libtucker_als.so")
    tmp = lib + ".tmp"
    link_extra = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-shared-libsan"] if sanitize else []
    rc, out = _run([HIPCC] + ARCH + ["-shared", "-fPIC"] + link_extra + objs + ["-o", tmp], verbose)
    if out.strip():
        sys.stderr.write(out + "\n")
    if rc != 0:
        raise RuntimeError(f"hipcc failed linking {os.path.basename(lib)}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv,
                sanitize="--sanitize" in sys.argv))
