"""Build libpt_hip.so (the gfx950 HIP library behind include/pt.h) in-tree.

    python -m paper_2307_15255_amd.build [-v] [-j JOBS]

Each translation unit under csrc/ is compiled on its own (in parallel, one
hipcc per unit) into paper_2307_15255_amd/_build/, then linked. hipcc
cross-compiles for gfx950 without a GPU present.

`build()` always recompiles everything. `ensure_built()` is what the
binding calls on import: it builds only when the library is missing or was
built from other sources (a content hash of the sources and flags sits next
to the library), and holds a file lock meanwhile so that concurrent
processes build once.
"""
from __future__ import annotations

import concurrent.futures as cf
import fcntl
import glob
import hashlib
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpt_hip.so")
# A build whose host code carries AddressSanitizer and UBSan (the device code
# is built as usual); only the CPU tests load it, under the sanitizer runtime.
SAN_OBJ = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(HERE, "libpt_hip_san.so")
SAN_FLAGS = [
    "-Xarch_host", "-fsanitize=address,undefined",
    "-Xarch_host", "-fno-sanitize-recover=all",
    "-Xarch_host", "-fno-omit-frame-pointer",
    "-g",
]
HASH = LIB + ".srchash"
HEADER = os.path.join(ROOT, "include", "pt.h")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # packed fp32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def source_hash() -> str:
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*"))) + [HEADER]:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    h.update(" ".join([HIPCC] + FLAGS).encode())
    return h.hexdigest()


def _jobs(jobs: int | None) -> int:
    if jobs:
        return jobs
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(16, n))


def _compile(src: str, verbose: bool, sanitize: bool = False) -> tuple[str, float]:
    obj = os.path.join(SAN_OBJ if sanitize else OBJ, os.path.basename(src) + ".o")
    flags = [f for f in FLAGS if not (sanitize and f == "-O3")] + (["-O1", *SAN_FLAGS] if sanitize else [])
    cmd = [HIPCC, *flags, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    t = time.time()
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(line for line in r.stdout.splitlines() if "packed-fp32-ops" not in line)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{out}")
    if out.strip() and verbose:
        print(out, flush=True)
    return obj, time.time() - t


def build(verbose: bool = False, jobs: int | None = None, sanitize: bool = False) -> str:
    """Compile every unit (in parallel) and link libpt_hip.so (sanitize:
    libpt_hip_san.so, host code under AddressSanitizer and UBSan)."""
    os.makedirs(SAN_OBJ if sanitize else OBJ, exist_ok=True)
    digest = source_hash()
    srcs = sources()
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=_jobs(jobs)) as ex:
        results = list(ex.map(lambda s: _compile(s, verbose, sanitize), srcs))
    objs = [o for o, _ in results]
    lib = SAN_LIB if sanitize else LIB
    tmp = lib + f".tmp{os.getpid()}"
    link_flags = ["-Xarch_host", "-fsanitize=address,undefined"] if sanitize else []
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, *link_flags, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    if sanitize:
        return lib
    with open(HASH + ".tmp", "w") as f:
        f.write(digest + "\n")
    os.replace(HASH + ".tmp", HASH)
    if verbose:
        slow = max(results, key=lambda r: r[1])
        print(f"built {LIB} in {time.time() - t0:.1f} s (slowest unit {os.path.basename(slow[0])}: "
              f"{slow[1]:.1f} s)", flush=True)
    return LIB


def is_current() -> bool:
    if not os.path.exists(LIB) or not os.path.exists(HASH):
        return False
    with open(HASH) as f:
        return f.read().strip() == source_hash()


def ensure_built(verbose: bool = True) -> str:
    """Build the library unless the one on disk matches the sources."""
    if is_current():
        return LIB
    os.makedirs(OBJ, exist_ok=True)
    with open(os.path.join(OBJ, ".lock"), "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        try:
            if not is_current():
                if verbose:
                    print(f"building {os.path.basename(LIB)} for gfx950 ({len(sources())} units) ...",
                          file=sys.stderr, flush=True)
                build(verbose=False)
        finally:
            fcntl.flock(lock, fcntl.LOCK_UN)
    return LIB


if __name__ == "__main__":
    jobs = None
    if "-j" in sys.argv:
        jobs = int(sys.argv[sys.argv.index("-j") + 1])
    print(build(verbose="-v" in sys.argv, jobs=jobs))
