"""Build libstencil5d.so for MI355X (gfx950) with hipcc.

The sweep kernels are C++ templates (``csrc/sweep2d.h``).  This script fixes
the set of compiled variants -- dtype, shape, radius, cells per lane, fused
depth b_T, prefetch depth -- writes one small instantiation unit per variant
plus a registry table into ``_build/``, compiles them in parallel and links
everything with the host code into ``libstencil5d.so`` next to this file.

Variant pruning follows the spirit of AN5D's register pruning ("Tuning"):
candidates whose compute region keeps at least a quarter of the tile width and
whose register state plausibly fits are compiled, and only those that the
compiler fits into the 256 architected VGPRs of a gfx950 lane without scratch
memory (at most 128 accumulation registers used as spill space) enter the
library.  Each variant's
resource report (VGPRs, occupancy, LDS) is kept in kernel_resources.json.

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

HOST_SOURCES = ["abi.cpp", "batch.cpp", "server.cpp", "tune.cpp", "halo.hip", "norms.hip", "direct.hip"]
HEADERS = ["s5d_internal.h", "kcommon.h", "sweep2d.h", "sweep3d.h", "sweepw2d.h", "sweepp2d.h", "persist2d.h",
           "persist_schedule.h"]
HOST_HEADERS = ["host.h", "batch.h", "norms.h", "direct.h", "stream2d.h", "stream3d.h"]  # not included by the variant units

# Kernel kinds: (name, C++ type, 32-bit words per element, accumulation
# policy).  Kind 2 is float32 with compensated (Dot2) accumulation.
DTYPES = {0: ("f32", "float", 1, 0), 1: ("f64", "double", 2, 0), 2: ("f32c", "float", 1, 1)}
MAX_BT = 10
# Compensated accumulation costs about nine VALU operations per term instead of
# one FMA, so these kernels are bound by arithmetic already at small depth.
MAX_BT_COMP = 4

# Expressions (s5d_desc.expr): 0 the weighted sum, 1 the weighted sum divided
# by c0, 2 gradient2d, 3 per-cell weights.  Expressions 2 and 3 run on the
# window kernels (sweepw2d.h).
EXPR_TAG = {0: "", 1: "div_", 2: "grad_", 3: "varc_"}
# The expression stencils of the paper's general benchmarks (Table 3) that get
# kernels: (expr, box, radius) -- j2d5pt, j2d9pt, j2d9pt-gol, gradient2d --
# and the variable-coefficient stars and 3x3 box.
EXPR_2D = [(1, 0, 1), (1, 0, 2), (1, 1, 1), (2, 0, 1), (3, 0, 1), (3, 0, 2), (3, 1, 1)]
# Deepest fused depth compiled per expression (window kernels keep 2r+1 rows
# per level; per-cell weights add n loads per cell and level).
MAX_BT_EXPR = {1: 10, 2: 10, 3: 4}


# Persistent batched launches (sweepp2d.h): the 2D families that get one
# kernel each, as (kind, box, r, cells per lane, deepest depth).  A family's
# kernel holds every depth 1..deepest and takes the registers of the deepest,
# so the deepest depth kept is the one whose own kernel still runs at the
# occupancy of the family's default depth.
PERSIST_2D = [(0, 0, 1, 4, 10), (0, 0, 2, 4, 7), (0, 1, 1, 4, 7), (1, 0, 1, 2, 10), (1, 0, 2, 2, 6)]
# waves per SIMD asked of each family's kernel: that of its deepest depth alone
PERSIST_WPE = {(0, 0, 1, 4, 10): 3, (0, 0, 2, 4, 7): 2, (0, 1, 1, 4, 7): 3, (1, 0, 1, 2, 10): 2, (1, 0, 2, 2, 6): 2}


def _pname(f):
    dtype, box, r, cpl, mx = f
    return "kp2d_%s_%s_r%d_c%d_b%d" % (DTYPES[dtype][0], "box" if box else "star", r, cpl, mx)


def est_vgprs_2d(words, box, r, cpl, bt, nr, accw=1):
    """Lower bound of the register state of one 2D variant, in 32-bit VGPRs:
    2r accumulator rows per level (accw values per accumulator), the load
    ring, the extended row."""
    return words * (bt * 2 * r * cpl * accw + nr * cpl + cpl + 2 * r) + 16


def ring_depth(r, bt, words):
    """Rows in the load ring (NR - 1 in flight): 4 for deep kernels, 8 when the
    kernel is shallow (b_T <= 2) and therefore bound by memory latency; a
    divisor or multiple of 2r so the unrolled loop stays lcm(2r, NR) <= 8."""
    if r == 3:
        return 6 if bt <= 2 and words == 1 else 3
    if bt <= 2 and not (words == 2 and r >= 3):
        return 8
    return 4


def candidates_2d():
    """(dtype, expr, box, r, cpl, bt, nr) tuples worth compiling."""
    out = []
    for dtype, (_, _, words, acc) in DTYPES.items():
        cpls = (2, 4) if dtype == 1 else (4,)
        # boxes of radius 3 and 4 (49 and 81 points) with plain accumulation
        for box, rmax in ((0, 4), (1, 2 if acc else 4)):
            for r in range(1, rmax + 1):
                for cpl in cpls:
                    if r > cpl:
                        continue
                    for bt in range(1, (MAX_BT_COMP if acc else MAX_BT) + 1):
                        if 64 * cpl - 2 * bt * r < 16 * cpl:
                            continue
                        nr = ring_depth(r, bt, words)
                        if est_vgprs_2d(words, box, r, cpl, bt, nr, 1 + acc) > 224:
                            continue
                        out.append((dtype, 0, box, r, cpl, bt, nr))
    # expression stencils: plain float32 (4 cells per lane) and float64 (2)
    for dtype in (0, 1):
        words = DTYPES[dtype][2]
        cpl = 4 if dtype == 0 else 2
        for expr, box, r in EXPR_2D:
            for bt in range(1, MAX_BT_EXPR[expr] + 1):
                if 64 * cpl - 2 * bt * r < 16 * cpl:
                    continue
                nr = ring_depth(r, bt, words) if expr == 1 else window_ring(r)
                rows = 2 * r + (1 if expr >= 2 else 0)
                if words * (bt * rows * cpl + nr * cpl + cpl + 2 * r) + 16 > 224:
                    continue
                out.append((dtype, expr, box, r, cpl, bt, nr))
    return out


def window_ring(r):
    """Load ring of the window kernels: a divisor or multiple of the 2r+1-row
    window, so the unrolled loop stays short (lcm(2r+1, NR) steps)."""
    return 3 if r == 1 else 5


def variants_2d():
    """Variants in the built library: the candidates the compiler fitted into
    registers without scratch spills (read from the last build's resource
    record), or all candidates if there is no record yet."""
    rec = _load_resources()
    if not rec:
        return candidates_2d()
    return [v for v in candidates_2d() if _vname(v) in rec and rec[_vname(v)]["ok"]]


# 3D tile shapes per dtype: (cells per lane along axis 2, rows per wave along
# axis 1, waves per workgroup); the tile is nw*m rows by 64*cpl columns.
TILES_3D = {0: [(2, 4, 8), (2, 2, 16)], 1: [(2, 2, 8), (2, 4, 8)], 2: [(2, 2, 8), (2, 4, 8)]}
MAX_BT_3D = {1: 5, 2: 3}


def est_vgprs_3d(words, box, r, cpl, m, bt, nr, accw=1):
    """Register state of one 3D variant: 2r accumulator (accw values each) and
    r delay planes per level, the load ring and the extended plane, in 32-bit
    VGPRs."""
    cells = m * cpl
    return words * (bt * (2 * accw + 1) * r * cells + nr * cells + (m + 2 * r) * (cpl + 2 * r)) + 24


def candidates_3d():
    """(dtype, expr, box, r, cpl, m, nw, bt, nr) tuples worth compiling."""
    out = []
    for dtype, (_, _, words, acc) in DTYPES.items():
        for box in (0, 1):
            for r in (1, 2):
                for cpl, m, nw in TILES_3D[dtype]:
                    if r > cpl or r > m:
                        continue
                    # VGPR cap per lane: a workgroup of nw waves keeps ceil(nw/4)
                    # waves on each SIMD of its CU
                    cap = min(256, 512 // max(1, (nw + 3) // 4))
                    for bt in range(1, min(MAX_BT_3D[r], 2 if acc else 99) + 1):
                        c1, c2 = nw * m - 2 * bt * r, 64 * cpl - 2 * bt * r
                        if c1 < (nw * m) // 3 or c2 < 16:
                            continue
                        if box and r == 2 and (bt > 2 or acc):
                            continue
                        if est_vgprs_3d(words, box, r, cpl, m, bt, 2, 1 + acc) > 0.85 * cap:
                            continue
                        out.append((dtype, 0, box, r, cpl, m, nw, bt, 2))
                        # j3d27pt: the 27-point box divided by c0, plain float32 and float64
                        if box and r == 1 and not acc and (cpl, m, nw) == TILES_3D[dtype][0 if dtype else 0]:
                            out.append((dtype, 1, box, r, cpl, m, nw, bt, 2))
    return out


def variants_3d():
    rec = _load_resources()
    if not rec:
        return candidates_3d()
    return [v for v in candidates_3d() if _vname3(v) in rec and rec[_vname3(v)]["ok"]]


def linear_variants_2d():
    """Built variants of the weighted-sum stencils: (dtype, box, r, cpl, bt, nr)."""
    return [(v[0],) + v[2:] for v in variants_2d() if v[1] == 0]


def linear_variants_3d():
    """Built 3D variants of the weighted-sum stencils: (dtype, box, r, cpl, m, nw, bt, nr)."""
    return [(v[0],) + v[2:] for v in variants_3d() if v[1] == 0]


def _vname3(v):
    dtype, expr, box, r, cpl, m, nw, bt, nr = v
    return "k3d_%s_%s%s_r%d_c%d_m%d_w%d_b%d_n%d" % (DTYPES[dtype][0], EXPR_TAG[expr], "box" if box else "star",
                                                    r, cpl, m, nw, bt, nr)


RESOURCES = os.path.join(HERE, "kernel_resources.json")


def _load_resources():
    if not os.path.exists(RESOURCES):
        return {}
    import json
    with open(RESOURCES) as f:
        return json.load(f)


_RES_KEYS = {"VGPRs": "vgprs", "AGPRs": "agprs", "ScratchSize [bytes/lane]": "scratch",
             "Occupancy [waves/SIMD]": "occupancy", "LDS Size [bytes/block]": "lds",
             "SGPRs": "sgprs"}


def _parse_resources(text):
    """Kernel resource remarks of one compile.  A unit holds a variant's
    single-grid and batched kernels; the worse value of the two is kept
    (the largest register, scratch and LDS use, the lowest occupancy)."""
    import re
    out = {}
    for line in text.splitlines():
        m = re.search(r"remark:.*?\s(VGPRs|AGPRs|SGPRs|ScratchSize \[bytes/lane\]|"
                      r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]): (\d+) \[-Rpass-analysis",
                      line)
        if m:
            key, val = _RES_KEYS[m.group(1)], int(m.group(2))
            if key not in out:
                out[key] = val
            else:
                out[key] = min(out[key], val) if key == "occupancy" else max(out[key], val)
    return out


def _vname(v):
    dtype, expr, box, r, cpl, bt, nr = v
    return "k2d_%s_%s%s_r%d_c%d_b%d_n%d" % (DTYPES[dtype][0], EXPR_TAG[expr], "box" if box else "star",
                                            r, cpl, bt, nr)


def _write_if_changed(path, text):
    if os.path.exists(path):
        with open(path) as f:
            if f.read() == text:
                return
    with open(path, "w") as f:
        f.write(text)


def _generate(variants, variants3=(), families=()):
    inst = os.path.join(BUILD, "inst")
    os.makedirs(inst, exist_ok=True)
    units = []
    for f in families:
        dtype, box, r, cpl, mx = f
        depths = ", ".join("Depth<%d, %d>" % (bt, ring_depth(r, bt, DTYPES[dtype][2]))
                           for bt in range(mx, 0, -1))
        text = ('#include "sweepp2d.h"\nnamespace s5d {\nPersist2D %s() {\n'
                '  return make_persist2d<%s, %d, 0, %d, %s, %d, %d, %s>();\n}\n}  // namespace s5d\n'
                % (_pname(f), DTYPES[dtype][1], DTYPES[dtype][3], r, "true" if box else "false", cpl,
                   PERSIST_WPE[f], depths))
        path = os.path.join(inst, _pname(f) + ".hip")
        _write_if_changed(path, text)
        units.append(path)
    for v in variants3:
        dtype, expr, box, r, cpl, m, nw, bt, nr = v
        name = _vname3(v)
        text = ('#include "sweep3d.h"\nnamespace s5d {\nKernel3D %s() {\n'
                '  return make_kernel3d<%s, %d, %d, %d, %s, %d, %d, %d, %d, %d>();\n}\n}  // namespace s5d\n'
                % (name, DTYPES[dtype][1], DTYPES[dtype][3], expr, r, "true" if box else "false", bt, cpl,
                   m, nw, nr))
        path = os.path.join(inst, name + ".hip")
        _write_if_changed(path, text)
        units.append(path)
    for v in variants:
        dtype, expr, box, r, cpl, bt, nr = v
        name = _vname(v)
        if expr >= 2:
            text = ('#include "sweepw2d.h"\nnamespace s5d {\nKernel2D %s() {\n'
                    '  return make_kernelw2d<%s, %s, %d, %s, %d, %d, %d>();\n}\n}  // namespace s5d\n'
                    % (name, DTYPES[dtype][1], "OP_GRADIENT" if expr == 2 else "OP_VARCOEF", r,
                       "true" if box else "false", bt, cpl, nr))
        else:
            text = ('#include "sweep2d.h"\nnamespace s5d {\nKernel2D %s() {\n'
                    '  return make_kernel2d<%s, %d, %d, %d, %s, %d, %d, %d>();\n}\n}  // namespace s5d\n'
                    % (name, DTYPES[dtype][1], DTYPES[dtype][3], expr, r, "true" if box else "false", bt,
                       cpl, nr))
        path = os.path.join(inst, name + ".hip")
        _write_if_changed(path, text)
        units.append(path)
    lines = ['#include "s5d_internal.h"', '#include "persist2d.h"', "namespace s5d {"]
    lines += ["Kernel2D %s();" % _vname(v) for v in variants]
    lines.append("const Entry2D kRegistry2D[] = {")
    for v in variants:
        dtype, expr, box, r, cpl, bt, nr = v
        lines.append("  {%d, %d, %d, %d, %d, %d, &%s}," % (dtype, expr, box, r, cpl, bt, _vname(v)))
    lines.append("};")
    lines.append("const int kRegistry2DSize = %d;" % len(variants))
    lines += ["Kernel3D %s();" % _vname3(v) for v in variants3]
    lines.append("const Entry3D kRegistry3D[] = {")
    for v in variants3:
        dtype, expr, box, r, cpl, m, nw, bt, nr = v
        lines.append("  {%d, %d, %d, %d, %d, %d, %d, %d, &%s}," % (dtype, expr, box, r, cpl, m, nw, bt,
                                                                 _vname3(v)))
    if not variants3:
        lines.append("  {0, 0, 0, 0, 0, 0, 0, 0, nullptr},")
    lines.append("};")
    lines.append("const int kRegistry3DSize = %d;" % len(variants3))
    lines += ["Persist2D %s();" % _pname(f) for f in families]
    lines.append("const EntryP2D kRegistryP2D[] = {")
    for f in families:
        dtype, box, r, cpl, mx = f
        lines.append("  {%d, 0, %d, %d, %d, %d, &%s}," % (dtype, box, r, cpl, mx, _pname(f)))
    if not families:
        lines.append("  {0, 0, 0, 0, 0, 0, nullptr},")
    lines.append("};")
    lines.append("const int kRegistryP2DSize = %d;" % len(families))
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
    """Compile one unit; returns (object path, seconds, kernel resources)."""
    import json
    base = os.path.splitext(os.path.basename(src))[0]
    key = _digest([src], DEVICE_FLAGS + [header_digest, "v7"])
    obj = os.path.join(BUILD, "obj", "%s.%s.o" % (base, key))
    meta = obj + ".res.json"
    if incremental and os.path.exists(obj) and os.path.exists(meta):
        with open(meta) as f:
            return obj, 0.0, json.load(f)
    os.makedirs(os.path.dirname(obj), exist_ok=True)
    tmp = obj + ".tmp%d" % os.getpid()
    t0 = time.time()
    host_only = src.endswith(".cpp")  # plain host code: no device pass
    cmd = [HIPCC, *DEVICE_FLAGS, *(["--offload-host-only"] if host_only
                                   else ["-Rpass-analysis=kernel-resource-usage"]),
           "-c", src, "-o", tmp]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, res.stdout))
    os.replace(tmp, obj)
    resources = _parse_resources(res.stdout)
    with open(meta, "w") as f:
        json.dump(resources, f)
    return obj, time.time() - t0, resources


def build(jobs: int | None = None, incremental: bool = False, verbose: bool = False,
          only: str | None = None) -> str:
    """Compile every candidate kernel variant, keep those without register
    spills, write the registry and link libstencil5d.so; returns its path.
    `only` (a regular expression over variant names) builds a subset, for
    kernel development."""
    import json
    import re
    if not incremental and os.path.isdir(os.path.join(BUILD, "obj")):
        shutil.rmtree(os.path.join(BUILD, "obj"))
    cands = [v for v in candidates_2d() if only is None or re.search(only, _vname(v))]
    cands3 = [v for v in candidates_3d() if only is None or re.search(only, _vname3(v))]
    fams = [f for f in PERSIST_2D if only is None or re.search(only, _pname(f))]
    units, _ = _generate(cands, cands3, fams)
    # kernel units include only the device headers they use (a 3D unit does
    # not see the 2D sweep, and so on); host sources also the public header and
    # the host-side internal headers
    hdr = _digest([os.path.join(CSRC, h) for h in HEADERS], [])
    base_hdr = ["s5d_internal.h", "kcommon.h"]
    unit_hdr = {
        "2d": _digest([os.path.join(CSRC, h) for h in base_hdr + ["sweep2d.h"]], []),
        "w2d": _digest([os.path.join(CSRC, h) for h in base_hdr + ["sweep2d.h", "sweepw2d.h"]], []),
        "3d": _digest([os.path.join(CSRC, h) for h in base_hdr + ["sweep3d.h"]], []),
        "p2d": _digest([os.path.join(CSRC, h) for h in base_hdr + ["sweep2d.h", "sweepp2d.h", "persist2d.h",
                                                                     "persist_schedule.h"]], []),
    }

    def key_of_unit(path):
        name = os.path.basename(path)
        if name.startswith("k3d_"):
            return unit_hdr["3d"]
        if name.startswith("kp2d_"):
            return unit_hdr["p2d"]
        if "_grad_" in name or "_varc_" in name:
            return unit_hdr["w2d"]
        return unit_hdr["2d"]
    jobs = jobs or max(1, min(32, os.cpu_count() or 1))
    t0 = time.time()
    objs, res_by_unit = {}, {}
    host = [os.path.join(CSRC, s) for s in HOST_SOURCES]
    host_hdr = hdr + _digest([os.path.join(CSRC, h) for h in HOST_HEADERS] +
                             [os.path.join(INCLUDE, "stencil5d.h")], [])
    # longest first: the box and deep variants dominate the build time
    order = sorted(units, key=lambda p: ("kp2d_" not in p, "box" not in p, -len(p))) + host
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, s, host_hdr if s in host else key_of_unit(s), incremental): s
                for s in order}
        for fut in cf.as_completed(futs):
            obj, dt, resources = fut.result()
            src = futs[fut]
            objs[src] = obj
            res_by_unit[os.path.splitext(os.path.basename(src))[0]] = resources
            if verbose and dt > 0:
                print("  %-44s %6.1f s  %s" % (os.path.basename(src), dt, resources), flush=True)
    record = {}
    for v in cands:
        r = dict(res_by_unit.get(_vname(v), {}))
        # no scratch memory; accumulation registers used as spill space are
        # tolerated (they cost register copies, not memory traffic)
        r["ok"] = r.get("scratch", 1) == 0 and r.get("vgprs", 999) <= 256 and r.get("agprs", 0) <= 128
        record[_vname(v)] = r
    for v in cands3:
        r = dict(res_by_unit.get(_vname3(v), {}))
        r["ok"] = r.get("scratch", 1) == 0 and r.get("vgprs", 999) <= 256 and r.get("agprs", 0) <= 128
        record[_vname3(v)] = r
    for f in fams:
        r = dict(res_by_unit.get(_pname(f), {}))
        r["ok"] = r.get("scratch", 1) == 0 and r.get("vgprs", 999) <= 256 and r.get("agprs", 0) <= 128
        record[_pname(f)] = r
    kept = [v for v in cands if record[_vname(v)]["ok"]]
    kept3 = [v for v in cands3 if record[_vname3(v)]["ok"]]
    keptp = [f for f in fams if record[_pname(f)]["ok"]]
    _, reg = _generate(kept, kept3, keptp)
    reg_obj, _, _ = _compile(reg, hdr, False)
    with open(RESOURCES, "w") as f:
        json.dump(record, f, indent=1, sort_keys=True)
    link = [objs[s] for s in host] + [reg_obj] + \
        [objs[os.path.join(BUILD, "inst", _vname(v) + ".hip")] for v in kept] + \
        [objs[os.path.join(BUILD, "inst", _vname3(v) + ".hip")] for v in kept3] + \
        [objs[os.path.join(BUILD, "inst", _pname(f) + ".hip")] for f in keptp]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *link]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout)
    os.replace(tmp, LIB)
    if verbose:
        print("built %s: %d of %d 2D and %d of %d 3D candidate variants and %d of %d persistent families fit "
              "in registers, %.0f s" % (LIB, len(kept), len(cands), len(kept3), len(cands3), len(keptp),
                                        len(fams), time.time() - t0))
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true",
                    help="reuse object files whose sources and flags are unchanged")
    ap.add_argument("--list", action="store_true", help="print the variant set and exit")
    ap.add_argument("--only", default=None, help="regular expression: build matching variants only")
    args = ap.parse_args(argv)
    if args.list:
        rec = _load_resources()
        for v in candidates_2d():
            print(_vname(v), rec.get(_vname(v), {}))
        for v in candidates_3d():
            print(_vname3(v), rec.get(_vname3(v), {}))
        return 0
    build(jobs=args.jobs, incremental=args.incremental, verbose=True, only=args.only)
    return 0


if __name__ == "__main__":
    sys.exit(main())
