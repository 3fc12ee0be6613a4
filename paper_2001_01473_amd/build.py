"""Build libstencil5d.so for MI355X (gfx950) with hipcc.

The sweep kernels are C++ templates (``csrc/sweep2d.h``).  This script fixes
the set of compiled variants -- dtype, shape, radius, cells per lane, fused
depth b_T, prefetch depth -- writes one small instantiation unit per variant
plus a registry table into ``_build/``, compiles them in parallel and links
everything with the host code into ``libstencil5d.so`` next to this file.

Variant pruning follows the spirit of AN5D's register pruning ("Tuning"):
a variant is built only if its register window fits in the 256 architected
VGPRs of a gfx950 lane and its compute region keeps at least a quarter of the
tile width.

Usage: ``python -m paper_2001_01473_amd.build [--jobs N] [--incremental]``.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libstencil5d.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-I" + CSRC, "-I" + INCLUDE]

HOST_SOURCES = ["abi.cpp", "halo.hip"]
HEADERS = ["s5d_internal.h", "sweep2d.h"]

DTYPES = {0: ("f32", "float", 1), 1: ("f64", "double", 2)}
MAX_BT = 10


def est_vgprs_2d(words, box, r, cpl, bt, pfk):
    """Register window estimate of one 2D variant, in 32-bit VGPRs."""
    u = 2 * r + 1
    nx = 2 * r if box else 0
    stage = u * pfk * cpl
    return words * (bt * u * (cpl + nx) + stage + cpl + 2 * r) + 24


def variants_2d():
    """(dtype, box, r, cpl, bt, pfk) tuples that get compiled."""
    out = []
    for dtype, (_, _, words) in DTYPES.items():
        cpls = (4,) if dtype == 0 else (2, 4)
        for box, rmax in ((0, 4), (1, 2)):
            for r in range(1, rmax + 1):
                for cpl in cpls:
                    if r > cpl:
                        continue
                    for bt in range(1, MAX_BT + 1):
                        if 64 * cpl - 2 * bt * r < 16 * cpl:
                            continue
                        pfk = 1 if r <= 2 else 0
                        if est_vgprs_2d(words, box, r, cpl, bt, pfk) > 256:
                            pfk = 0
                        if est_vgprs_2d(words, box, r, cpl, bt, pfk) > 256:
                            continue
                        out.append((dtype, box, r, cpl, bt, pfk))
    return out


def _vname(v):
    dtype, box, r, cpl, bt, pfk = v
    return "k2d_%s_%s_r%d_c%d_b%d_p%d" % (DTYPES[dtype][0], "box" if box else "star",
                                          r, cpl, bt, pfk)


def _write_if_changed(path, text):
    if os.path.exists(path):
        with open(path) as f:
            if f.read() == text:
                return
    with open(path, "w") as f:
        f.write(text)


def _generate(variants):
    inst = os.path.join(BUILD, "inst")
    os.makedirs(inst, exist_ok=True)
    units = []
    for v in variants:
        dtype, box, r, cpl, bt, pfk = v
        name = _vname(v)
        text = ('#include "sweep2d.h"\nnamespace s5d {\nKernel2D %s() {\n'
                '  return make_kernel2d<%s, %d, %s, %d, %d, %d>();\n}\n}  // namespace s5d\n'
                % (name, DTYPES[dtype][1], r, "true" if box else "false", bt, cpl, pfk))
        path = os.path.join(inst, name + ".hip")
        _write_if_changed(path, text)
        units.append(path)
    lines = ['#include "s5d_internal.h"', "namespace s5d {"]
    lines += ["Kernel2D %s();" % _vname(v) for v in variants]
    lines.append("const Entry2D kRegistry2D[] = {")
    for v in variants:
        dtype, box, r, cpl, bt, pfk = v
        lines.append("  {%d, %d, %d, %d, %d, &%s}," % (dtype, box, r, cpl, bt, _vname(v)))
    lines.append("};")
    lines.append("const int kRegistry2DSize = %d;" % len(variants))
    lines.append("}  // namespace s5d")
    reg = os.path.join(BUILD, "registry.cpp")
    _write_if_changed(reg, "\n".join(lines) + "\n")
    return units, reg


def _digest(paths, extra):
    h = hashlib.sha1()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    h.update(" ".join(extra).encode())
    return h.hexdigest()[:16]


def _compile(src, header_digest, incremental):
    base = os.path.splitext(os.path.basename(src))[0]
    key = _digest([src], DEVICE_FLAGS + [header_digest, "v2"])
    obj = os.path.join(BUILD, "obj", "%s.%s.o" % (base, key))
    if incremental and os.path.exists(obj):
        return obj, 0.0
    os.makedirs(os.path.dirname(obj), exist_ok=True)
    tmp = obj + ".tmp%d" % os.getpid()
    t0 = time.time()
    host_only = src.endswith(".cpp")  # plain host code: no device pass
    cmd = [HIPCC, *DEVICE_FLAGS, *(["--offload-host-only"] if host_only else []),
           "-c", src, "-o", tmp]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, res.stdout))
    os.replace(tmp, obj)
    return obj, time.time() - t0


def build(jobs: int | None = None, incremental: bool = False, verbose: bool = False) -> str:
    """Compile every kernel variant and link libstencil5d.so; returns its path."""
    if not incremental and os.path.isdir(os.path.join(BUILD, "obj")):
        shutil.rmtree(os.path.join(BUILD, "obj"))
    variants = variants_2d()
    units, reg = _generate(variants)
    hdr = _digest([os.path.join(CSRC, h) for h in HEADERS] +
                  [os.path.join(INCLUDE, "stencil5d.h")], [])
    sources = [os.path.join(CSRC, s) for s in HOST_SOURCES] + [reg] + units
    # longest first: the box and deep variants dominate the build time
    sources.sort(key=lambda p: (("box" not in p), -len(p)))
    jobs = jobs or max(1, min(32, os.cpu_count() or 1))
    t0 = time.time()
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, s, hdr, incremental): s for s in sources}
        for fut in cf.as_completed(futs):
            obj, dt = fut.result()
            objs.append(obj)
            if verbose and dt > 0:
                print("  %-60s %6.1f s" % (os.path.basename(futs[fut]), dt), flush=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *sorted(objs)]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout)
    os.replace(tmp, LIB)
    if verbose:
        print("built %s: %d kernel variants in %.0f s" % (LIB, len(variants), time.time() - t0))
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true",
                    help="reuse object files whose sources and flags are unchanged")
    ap.add_argument("--list", action="store_true", help="print the variant set and exit")
    args = ap.parse_args(argv)
    if args.list:
        for v in variants_2d():
            print(_vname(v))
        return 0
    build(jobs=args.jobs, incremental=args.incremental, verbose=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
