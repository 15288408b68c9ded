"""Build the HIP library libpswa.so in-tree with hipcc for gfx950.

Usage: python paper_2605_20977_amd/build.py [--incremental] [--only P_D_R,...]
(or __graft_entry__.build(), which always compiles every object).
--incremental recompiles only objects older than their source or any header
under csrc/ and include/. --only (development builds) compiles just the
listed persistent-kernel instances (arithmetic_headsize_rowtile) and stubs
the others out. It does not import the package, so it works with no library
built.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpswa.so")
OBJ = os.path.join(PKG, "_build")

SOURCES = ["kernels_f32.hip", "persistent.hip", "train.hip", "pswa_capi.cpp", "batch.cpp",
           "coder.cpp", "profile.cpp", "noalloc.hip"]
# persistent_kernel.hip is compiled once per (arithmetic, head size, row tile)
PERSISTENT_INSTANCES = [(0, d, 32) for d in (16, 32, 48, 64)] + [
    (p, d, r) for p in (1, 2) for r in (16, 32) for d in (16, 32, 48, 64)]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no implicit multiply-add contraction: identical source gives identical
    # arithmetic in every kernel and translation unit
    "-ffp-contract=off",
    # packed FP32 instructions stay off: plain scalar FP32 only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    # host-pass notes about the packed-fp32 feature are expected
    err = "\n".join(ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln)
    return r.returncode, err


def _headers_digest() -> str:
    h = hashlib.sha256()
    for d in (CSRC, os.path.join(ROOT, "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith(".h"):
                h.update(f.encode())
                h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def _unit_digest(cmd, hdr: str) -> str:
    """Digest of what an object is built from: the command, its source and
    every header (taken before the compile starts)."""
    h = hashlib.sha256(hdr.encode())
    h.update(" ".join(cmd[:-1]).encode())
    h.update(open(cmd[-3], "rb").read())
    return h.hexdigest()


def _stale(cmd, digest: str) -> bool:
    obj = cmd[-1]
    stamp = obj + ".stamp"
    if not (os.path.exists(obj) and os.path.exists(stamp)):
        return True
    return open(stamp).read().strip() != digest


def build(verbose: bool = True, jobs: int | None = None, incremental: bool = False,
          only: list | None = None) -> str:
    """Compile every object (in parallel; only the stale ones when
    incremental; `only` persistent instances, the rest as stubs) and link
    libpswa.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    units = []  # the long persistent instances first
    for p, d, r in PERSISTENT_INSTANCES:
        stub = only is not None and (p, d, r) not in only
        obj = os.path.join(OBJ, f"persistent_kernel_{p}_{d}_{r}{'_stub' if stub else ''}.o")
        units.append([hipcc, *HIPCC_FLAGS, *inc, f"-DPSWA_PREC={p}", f"-DPSWA_DH={d}",
                      f"-DPSWA_R={r}", *(["-DPSWA_STUB_INSTANCE"] if stub else []), "-c",
                      os.path.join(CSRC, "persistent_kernel.hip"), "-o", obj])
    for src in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        units.append([hipcc, *HIPCC_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj])
    objs = [u[-1] for u in units]
    hdr = _headers_digest()
    digests = {u[-1]: _unit_digest(u, hdr) for u in units}
    if incremental:
        units = [u for u in units if _stale(u, digests[u[-1]])]
    jobs = jobs or min(16, os.cpu_count() or 1)
    if verbose:
        print(f"compiling {len(units)} objects with {jobs} jobs", flush=True)
    with ThreadPoolExecutor(max(1, jobs)) as ex:
        results = list(ex.map(_run, units))
    failed = False
    for cmd, (rc, err) in zip(units, results):
        if rc != 0:
            failed = True
            sys.stderr.write(" ".join(cmd) + "\n" + err + "\n")
        else:
            with open(cmd[-1] + ".stamp", "w") as f:
                f.write(digests[cmd[-1]] + "\n")
            if verbose and err.strip():
                sys.stderr.write(err + "\n")
    if failed:
        raise RuntimeError("hipcc failed building libpswa.so")
    tmp = LIB + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    rc, err = _run(link)
    if rc != 0:
        sys.stderr.write(" ".join(link) + "\n" + err + "\n")
        raise RuntimeError("linking libpswa.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", flush=True)
    return LIB


if __name__ == "__main__":
    argv = sys.argv[1:]
    sel = None
    if "--only" in argv:
        sel = [tuple(int(v) for v in spec.split("_"))
               for spec in argv[argv.index("--only") + 1].split(",")]
    build(incremental="--incremental" in argv, only=sel)
