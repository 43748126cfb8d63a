"""Benchmark: solves per second at relative residual 1e-10 on one MI355X.

Default workload (large512; one step = one whole solve, plan cached): the
512^3 grid, periodic in x and y, Dirichlet in z; eta = 10^6 unit point
charges of random sign at uniformly drawn cells plus N(0, 1e-3) noise, minus
its mean (seed 5); FP64 vectors (1 GiB each), tol 1e-10.  The headline line is
the preconditioner on the int8 matrix cores with FP64 accuracy (I8X6: exact
products of six balanced base-256 digits, FP64 recombination); the same
right-hand side is then solved with the FP64, FP32, BF16 (flexible beta),
split-BF16 (BF16X6) and seven-digit int8 (I8X7) preconditioners for the
mixed-versus-FP64 comparison, and the CPU oracle
computes the minimum-norm solution of the same input on the host cores, which
every precision's result is compared with (norm-wise and element-wise).

Other workloads (--workload):
  single256  256 x 256 x 128, (P, P, DN), 10^4 charges (seed 2), FP32
             preconditioner, tol 1e-10
  latency2d  2D 64 x 64, Dirichlet on every edge, 16 Gaussian blobs (seed 1), FP64
             preconditioner, tol 1e-12 (latency-bound)
  batch64    64 right-hand sides on 128^3, Neumann on every face (singular),
             the same charge generator with seeds 3000 + b, BF16 preconditioner
             with the flexible beta, tol 1e-10; one step = one batched solve of 64
  serving    the request stream of the serving layer (see serving_bench)

    python bench.py [--workload large512] [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "3D solves/s at rel-res 1e-10, mixed vs FP64 PCG; p50/p99 latency"
COPY_CAL_BYTES = 256 << 20     # bytes read (and written) by the calibration copy
COPY_CAL_RUNS = 3               # times it runs, first of the run's device copies
# TFLOP/s; bf16x6 counts the FP32-equivalent flops of a product, whose
# emulation issues six BF16 matrix-core products: its ceiling is 2500 / 6;
# i8x7 and i8x6 count the FP64-equivalent flops, each of which costs 28 or
# 21 int8 matrix-core operations (5000 TOP/s dense): their ceilings are
# 5000 / 28 and 5000 / 21
INT8_PRODUCTS = {"i8x7": 28, "i8x6": 21}
PEAK = {"hbm_GBs": 8000.0, "f64": 78.6, "f32": 157.3, "bf16": 2500.0, "bf16x6": 2500.0 / 6,
        "i8x7": 5000.0 / 28, "i8x6": 5000.0 / 21}
DTYPE = {"f32": "f64+f32", "f64": "f64", "bf16": "f64+bf16", "bf16x6": "f64+bf16x6",
         "i8x7": "f64+i8x7", "i8x6": "f64+i8x6"}
PRECS = ("f64", "f32", "bf16", "bf16x6", "i8x7", "i8x6")
FP64_ACCURATE = ("f64", "i8x7", "i8x6")
MODEPROD = ("modeprod_z_fwd", "modeprod_y_fwd", "modeprod_x_fwd", "modeprod_x_bwd",
            "modeprod_y_bwd", "modeprod_z_bwd")

WORKLOADS = {
    "single256": dict(grid=(256, 256, 128), bcs=("P", "P", "DN"), batch=1, prec="f32", tol=1e-10,
                 steps=40, field="charges", ncharges=10_000, seed=2,
                 desc="3D 256x256x128, BC (P,P,DN), 1e4 random-sign unit charges + "
                      "N(0,1e-3) noise, zero mean, seed 2; one solve per step"),
    "latency2d": dict(grid=(64, 64, 1), bcs=("D", "D"), batch=1, prec="f64", tol=1e-12,
                 steps=200, field="blobs", seed=1,
                 desc="2D 64x64, BC (D,D), 16 Gaussian blobs (sigma 2, seed 1); "
                      "one solve per step"),
    "batch64": dict(grid=(128, 128, 128), bcs=("N", "N", "N"), batch=64, prec="bf16", tol=1e-10,
                 steps=10, field="charges", ncharges=10_000, seed=3000,
                 desc="64 RHS on 3D 128^3, BC (N,N,N) singular, 1e4 charges + N(0,1e-3) "
                      "noise per RHS (seed 3000+b), zero mean; one batched solve per step"),
    "large512": dict(grid=(512, 512, 512), bcs=("P", "P", "D"), batch=1, prec="i8x6", tol=1e-10,
                 steps=10, field="charges", ncharges=1_000_000, seed=5,
                 desc="3D 512^3, BC (P,P,D), 1e6 random-sign unit charges + N(0,1e-3) "
                      "noise, zero mean, seed 5; one solve per step"),
}


# ------------------------------------------------------- HBM traffic record ----
# Measured HBM bytes per launch come from two rocprofv3 counter runs of this
# script (FETCH_SIZE, then WRITE_SIZE, with --copy-calibration), turned into a
# record under profiles/ by --ingest-traffic.  Both counters are scaled by
# what they read for the calibration copy of known size.  The record carries
# a digest of the kernel sources; once a kernel has changed, traffic is null.
KERNEL_SOURCES = ("kp_modeprod.hip", "kp_vector.hip", "kp_common.h", "kp_internal.h", "kp_state.h")
VEC_KERNELS = {"stencil_dot": "kp::k_zm<0>", "update_ur": "kp::k_zm<1>",
               "dot_rz": "kp::k_dot_rz", "update_p": "kp::k_update_p"}
PRODUCT_ORDER = {3: ("modeprod_x_fwd", "modeprod_y_fwd", "modeprod_z_fwd", "modeprod_x_bwd",
                     "modeprod_y_bwd", "modeprod_z_bwd"),
                 2: ("modeprod_x_fwd", "modeprod_y_fwd", "modeprod_x_bwd", "modeprod_y_bwd")}


def traffic_path(workload):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2501_03377_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(src, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def int8_fits(grid):
    """The int8 split preconditioners need every axis a multiple of 16 and at
    most 512."""
    return all(n % 16 == 0 and n <= 512 for n in grid if n > 1)


def pid_of(prec):
    return {"f64": 0, "f32": 1, "bf16": 2, "bf16x6": 3, "i8x7": 4, "i8x6": 5}[prec]


def launch_identity(cls, prec, grid, batch, tuning):
    """The profiler's name (and, for mode products, total threads) of the
    kernel that a class launches with the given tile choices."""
    if cls in VEC_KERNELS:
        return VEC_KERNELS[cls]
    if cls == "small_solve":
        return "kp::(anonymous namespace)::k_small_solve"
    from paper_2501_03377_amd.kpcg import kp_tile_shape, PREC
    nx, ny, nz = grid
    dim = 3 if nz > 1 else 2
    if cls not in PRODUCT_ORDER[dim]:
        return None
    q = PRODUCT_ORDER[dim].index(cls)
    K = grid["xyz".index(cls.split("_")[1])]
    rows = nx * ny * nz // K
    if prec in INT8_PRODUCTS:
        # k-blocks of 64 per wave; up to 256 one block of 4 waves per 64 rows,
        # above it split over two waves per row group, one block of 4 waves
        # per 32 rows, the epilogue kind (1: the Hadamard factor) and the
        # digit count parameters
        nkb, S = -(-K // 64), 7 if prec == "i8x7" else 6
        epi = 1 if q == dim - 1 else 0
        nrb = -(-rows // 128)
        if K <= 128 and nrb * 8 <= 8192:
            # operator-resident: persistent blocks of 8 waves, one or two per CU
            lds = nkb * 4 * nkb * S * 64 * 16 + 64 * nkb * 12
            per_cu = 2 if 2 * lds <= 160 * 1024 else 1
            blocks = max(1, min(nrb, -(-256 * per_cu // batch))) * batch
            return f"kp::mp_ozr<{nkb}, {epi}, {S}>|{blocks * 512}"
        if K <= 256:
            return f"kp::mp_oz<{nkb}, 1, {S}>|{-(-rows // 64) * batch * 256}"
        return f"kp::mp_ozh<{-(-nkb // 2)}, {epi}, {S}>|{-(-rows // 32) * batch * 256}"
    tc = {"f64": "double", "f32": "float", "bf16": "__bf16", "bf16x6": "float"}[prec]
    ti = "double" if q == 0 else tc
    to = "double" if q == 2 * dim - 1 else tc
    vec = K % (8 if prec in ("bf16", "bf16x6") else 4) == 0
    if vec and tuning[q] in (20, 21) and K <= 128:
        # operator-resident tiles: persistent blocks, as many per right-hand
        # side as fill the chip once
        wn, wc = (8, 1) if tuning[q] == 20 else (4, 2)
        res_lds = {"f64": 131072, "f32": 65536, "bf16": 32768, "bf16x6": 98304}[prec]
        if to == "__bf16":
            res_lds += 128 * (64 + 8) * 2       # the staged output tile
        per_cu = max(1, min(4, 160 * 1024 // res_lds))
        nrb = -(-rows // 64)
        blocks = max(1, min(nrb, -(-256 * per_cu // batch))) * batch
        return (f"kp::mp_res<{pid_of(prec)}, {ti}, {to}, {wn}, {wc}>"
                f"|{blocks * 256 * wc}")
    if vec:
        rc, (wn, wm, wc) = kp_tile_shape(tuning[q], PREC[prec])
        if rc != 0:
            return None
    else:
        wn, wm, wc = 4, 2, 2
    blocks = -(-rows // (64 * wm)) * -(-K // (16 * wn * wc)) * batch
    pid = pid_of(prec)
    return (f"kp::mp_kernel<{pid}, {ti}, {to}, {wn}, {wm}, {wc}, {'true' if vec else 'false'}>"
            f"|{blocks * 256 * wc}")


def ingest_traffic(workload, fetch_dir, write_dir, command):
    """Averages FETCH_SIZE and WRITE_SIZE per kernel over the dispatches of two
    counter runs and writes the traffic record of the workload."""
    import csv
    import glob

    def read(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        acc, copies = {}, []
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").strip()
            v = float(r["Counter_Value"])
            if "copyBuffer" in name:
                copies.append((int(r["Dispatch_Id"]), v))
                continue
            name = profiler_kernel_name(name)
            # mode products by name and total threads, as launch_identity names them
            key = f"{name}|{r['Grid_Size']}" if name.startswith("kp::mp_") else name
            t = acc.setdefault(key, [0.0, 0])
            t[0] += v
            t[1] += 1
        # the calibration copies are the run's first device copies (issued
        # before anything else is copied); later copies move the workload's
        # own data and have other sizes
        cal = [v for _, v in sorted(copies)[:COPY_CAL_RUNS]]
        return {k: t[0] / t[1] for k, t in acc.items()}, (sum(cal) / len(cal) if cal else 0.0)

    fetch, copy_fetch = read(fetch_dir, "FETCH_SIZE")
    write, copy_write = read(write_dir, "WRITE_SIZE")
    rec = {"workload": workload, "digest": kernel_digest(), "command": command,
           "copy_bytes": COPY_CAL_BYTES, "copy_fetch_kib": copy_fetch, "copy_write_kib": copy_write,
           "kernels": {k: {"fetch_kib": fetch[k], "write_kib": write.get(k)} for k in sorted(fetch)}}
    with open(traffic_path(workload), "w") as f:
        json.dump(rec, f, indent=1)
    return rec


# matrix-core rates per CU per cycle by operand type (dense, the published
# MI355X peaks at 2.4 GHz over 256 CUs): ops counted as the profiler's
# SQ_INSTS_VALU_MFMA_MOPS_* (units of 512 operations)
MFMA_OPS_PER_CU_CYCLE = {"F64": 128.0, "F32": 256.0, "BF16": 4096.0, "I8": 8192.0}
NUM_XCD, NUM_CU, SIMD_PER_CU = 8, 256, 4


def profiler_kernel_name(name):
    """The profiler's kernel name in the form launch_identity uses.  rocprofv3
    leaves most templates with __bf16 arguments mangled, and demangles the
    operand pair (__bf16, double) as 'bool _Accum'; both are rewritten."""
    import re
    m = re.match(r"_ZN2kp(\d+)(mp_kernel|mp_res)I(.*?E)EEv", name)
    if m:
        args, rest = [], m.group(3)
        while rest:
            t = re.match(r"Li(\d+)E|Lb([01])E|DF16b|d|f", rest)
            if not t:
                return name
            tok = t.group(0)
            args.append(t.group(1) if t.group(1) else ("true" if t.group(2) == "1" else "false")
                        if t.group(2) else {"DF16b": "__bf16", "d": "double", "f": "float"}[tok])
            rest = rest[len(tok):]
        return f"kp::{m.group(2)}<{', '.join(args)}>"
    name = re.sub(r"^kp::(mp_kernel|mp_res)<(\d+), bool _Accum, ", r"kp::\1<\2, __bf16, double, ",
                  name.replace("void ", "").strip())
    return name


def ingest_mfma(counter_dir, bench_log, workload, prec):
    """Per mode-product kernel of one counter run: dispatches, duration, the
    clock GRBM_GUI_ACTIVE implies, the matrix-core busy fraction
    (SQ_VALU_MFMA_BUSY_CYCLES over SIMD-cycles) and the operations per
    CU-cycle of each operand type against its peak; as markdown rows.  The
    products a kernel served come from the tile choices in the JSON line of
    the profiled bench run (bench_log)."""
    import csv
    import glob
    f = glob.glob(os.path.join(counter_dir, "**", "*counter_collection.csv"), recursive=True)[0]
    disp = {}
    for r in csv.DictReader(open(f)):
        name = profiler_kernel_name(r["Kernel_Name"].split("(")[0].replace("void ", "").strip())
        if not any(t in name for t in ("mp_kernel", "mp_res", "mp_oz")):
            continue
        d = disp.setdefault(r["Dispatch_Id"], {"key": f"{name}|{r['Grid_Size']}", "c": {},
                                               "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
        d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    wl = WORKLOADS[workload]
    line = [ln for ln in open(bench_log) if ln.startswith("{")][-1]
    tiles = json.loads(line)["config"]["tile_configs"]
    names = {}
    for cls in PRODUCT_ORDER[3 if wl["grid"][2] > 1 else 2]:
        ident = launch_identity(cls, prec, wl["grid"], wl["batch"], tiles)
        names.setdefault(ident, []).append(cls.replace("modeprod_", ""))
    agg = {}
    for d in disp.values():
        a = agg.setdefault(d["key"], {"n": 0, "ns": 0.0, "c": {}})
        a["n"] += 1
        a["ns"] += d["ns"]
        for k, v in d["c"].items():
            a["c"][k] = a["c"].get(k, 0.0) + v
    rows = []
    for key, a in sorted(agg.items(), key=lambda t: -t[1]["ns"]):
        n, c = a["n"], a["c"]
        gui = c.get("GRBM_GUI_ACTIVE", 0.0) / n / NUM_XCD          # cycles of one XCD
        if gui <= 0:
            continue
        us = a["ns"] / n / 1e3
        busy = c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / n / (gui * NUM_CU * SIMD_PER_CU)
        parts = []
        for t, peak in MFMA_OPS_PER_CU_CYCLE.items():
            ops = c.get(f"SQ_INSTS_VALU_MFMA_MOPS_{t}", 0.0) / n * 512.0
            if ops > 0:
                parts.append(f"{t} {ops / (gui * NUM_CU):.1f} ops/CU-cycle = {ops / (gui * NUM_CU) / peak:.3f} of peak")
        cls = names.get(key)
        hbm = "-"
        if cls:
            by = product_bytes("modeprod_" + cls[0], prec, wl["grid"]) * wl["batch"]
            hbm = f"{by / (us * 1e-6) / 1e9:.0f} GB/s = {by / (us * 1e-6) / 1e9 / PEAK['hbm_GBs']:.3f}"
        kname, grid = key.rsplit("|", 1)
        rows.append(f"| `{kname}` ({grid} threads) | {', '.join(cls or ['(tuning trial)'])} | {n} | {us:.1f} | "
                    f"{gui / us / 1e3:.2f} | {busy:.3f} | {'; '.join(parts) or '-'} | {hbm} |")
    return rows


def measured_traffic(workload, identity):
    """HBM bytes per launch of a kernel from the workload's traffic record, or
    None when there is no record, the kernel is not in it or has changed."""
    try:
        with open(traffic_path(workload)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    k = rec["kernels"].get(identity) if identity else None
    if k is None or rec.get("digest") != kernel_digest() or k.get("write_kib") is None:
        return None
    if not rec["copy_fetch_kib"] or not rec["copy_write_kib"]:
        return None
    return (k["fetch_kib"] * rec["copy_bytes"] / rec["copy_fetch_kib"]
            + k["write_kib"] * rec["copy_bytes"] / rec["copy_write_kib"])


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def make_eta(wl):
    import synth
    nx, ny, nz = wl["grid"]
    shape = (nz, ny, nx) if nz > 1 else (ny, nx)
    if wl["field"] == "blobs":
        one = lambda b: synth.gaussian_blobs_2d(nx, ny, 16, 2.0, seed=wl["seed"] + b)
    else:
        one = lambda b: synth.charge_field(shape, ncharges=wl["ncharges"], noise_std=1e-3,
                                           seed=wl["seed"] + b)
    if wl["batch"] == 1:
        return one(0)
    return np.stack([one(b) for b in range(wl["batch"])])


def solve_work(name, grid, results, flex=False, spectral=True):
    """Algorithmic work of one kernel class over one whole (batched) solve,
    summed over the right-hand sides that are still active in each launch
    (a converged RHS skips its blocks).  Returns ('flop', F) for a mode
    product: 2 N n_axis per application, plus N for the Hadamard factor on
    the last forward product (z in 3D, y in 2D), so that the six add up to
    Table 2's 4N(nx+ny+nz) + N; or ('byte', B) for an HBM-bound vector
    kernel, FP64 words moved per unknown times 8 N.  A RHS that converged
    after s iterations used p pinv applications (one at start, one per
    iteration, except a last iteration that stopped on the residual test
    and error bound) and s stencil and U/R updates; when the last
    application was followed by the stop, its P update is skipped.  The
    timed back-to-back launches of the roofline move the full 5 words of a
    later U/R update (launch_work)."""
    nx, ny, nz = grid
    N = nx * ny * nz
    tot = 0.0
    for r in results:
        s, p = r["iterations"], r["pinv_applications"]
        if name in MODEPROD:
            n_axis = {"x": nx, "y": ny, "z": nz}[name.split("_")[1]]
            last_fwd = "modeprod_z_fwd" if nz > 1 else "modeprod_y_fwd"
            tot += p * (2.0 * N * n_axis + (N if name == last_fwd else 0.0))
        elif name == "stencil_dot":      # reads P (W = L P stored for the flexible beta)
            tot += s * (1 + flex) * 8.0 * N
        elif name == "update_ur":        # reads P, R, U, writes R, U (L P recomputed)
            # (the first iteration takes U_0 = 0 without reading it)
            tot += (5 * s - (1 if s >= 1 else 0)) * 8.0 * N
        elif name == "dot_rz":           # reads R, Z (and W for the flexible beta)
            tot += p * (2 + flex) * 8.0 * N
        elif name == "update_p":         # P_0 = Z_0: 2 words; P = Z + beta P: 3 words
            # one P update per application, except after the last when the
            # solve stopped on the error estimate that followed it; P_0 = Z_0
            # is a launch of its own only off the spectral path (FP32 and BF16
            # products, the flexible beta): otherwise the first application
            # writes P_0 itself
            nu = p - (1 if p > s else 0)
            if not spectral:
                tot += (2 + 3 * (nu - 1)) * 8.0 * N if nu >= 1 else 0.0
            else:
                tot += 3 * (nu - 1) * 8.0 * N if nu >= 2 else 0.0
        elif name == "small_solve":      # the whole solve in one kernel: its mode products
            tot += p * (4.0 * N * (nx + ny) + N)
        else:
            return None, 0.0
    return ("flop" if name in MODEPROD or name == "small_solve" else "byte"), tot


def launch_work(name, grid, batch, flex=False):
    """Algorithmic work of one launch of a kernel class with every one of
    `batch` right-hand sides active, as the library's kernel timing call
    launches it: ('flop', F) or ('byte', B), per unit as in solve_work (an
    update_p launch after the first iteration moves 3 words per unknown)."""
    nx, ny, nz = grid
    N = nx * ny * nz
    if name in MODEPROD:
        n_axis = {"x": nx, "y": ny, "z": nz}[name.split("_")[1]]
        last_fwd = "modeprod_z_fwd" if nz > 1 else "modeprod_y_fwd"
        return "flop", batch * (2.0 * N * n_axis + (N if name == last_fwd else 0.0))
    words = {"stencil_dot": 1 + flex, "update_ur": 5, "dot_rz": 2 + flex, "update_p": 3}
    if name not in words:
        return None, 0.0
    return "byte", batch * words[name] * 8.0 * N


ELEM_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "bf16x6": 4, "i8x7": 8, "i8x6": 8}


def product_bytes(name, prec, grid):
    """Algorithmic HBM bytes of one mode product per right-hand side: its
    input read once and its output written once.  The first product reads the
    FP64 residual and the last writes the FP64 preconditioned residual; the
    intermediates are in the compute type (FP64 for the int8 split)."""
    nx, ny, nz = grid
    dim = 3 if nz > 1 else 2
    order = PRODUCT_ORDER[dim]
    e = ELEM_BYTES[prec]
    bin_ = 8 if name == order[0] else e
    bout = 8 if name == order[-1] else e
    return nx * ny * nz * (bin_ + bout)


def run_solves(plan, eta_d, u, steps, tol, flags=0, max_iter=60):
    """steps solves back to back; Python's cyclic garbage collector runs
    before them and not during them (as timeit does)."""
    import gc
    import torch
    lat, res = [], None
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            t = time.perf_counter()
            _, res, _, rc = plan.solve(eta_d, tol=tol, max_iter=max_iter, flags=flags, out=u)
            lat.append(time.perf_counter() - t)
            if rc != 0:
                raise RuntimeError(f"solve failed with status {rc}: {res}")
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
    finally:
        gc.enable()
    return T, np.array(lat), res


def cpu_baseline(wl, eta, budget_s=25.0):
    """The FP64 oracle on the host cores: the minimum-norm solution L^+ eta_c
    written out from the eigen-expansion of the operator (LAPACK eigenbases
    of the 1D matrices, each axis contracted into the eigenbasis and back,
    numpy), over the workload's right-hand sides in turn while the time
    budget lasts (at least one solve).  Returns the oracle solutions by RHS
    index and the timing record."""
    import oracle
    from threadpoolctl import threadpool_info
    bcs = wl["bcs"]
    etas = eta if wl["batch"] > 1 else eta[None]
    sols, runs, t_solve = {}, 0, 0.0
    t_all = time.perf_counter()
    while runs == 0 or (time.perf_counter() - t_all) < budget_s * 0.5:
        b = runs % len(etas)
        t = time.perf_counter()
        u, _ = oracle.min_norm_solution(etas[b].T, bcs)
        t_solve += time.perf_counter() - t
        sols.setdefault(b, u.T)
        runs += 1
        if runs == len(etas):
            break
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    nx, ny, nz = wl["grid"]
    gtxt = f"{nx}x{ny}" + (f"x{nz}" if nz > 1 else "")
    return sols, {
        "value": runs / t_solve,
        "unit": "solves/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{runs} oracle solve(s) of {len(sols)} of the workload's {len(etas)} "
                  f"{gtxt} right-hand side(s): the minimum-norm solution from the "
                  "eigen-expansion (LAPACK eigh bases, FP64 numpy)",
        "solve_s": t_solve / runs,
        "host_cpus": os.cpu_count(),
    }


def stream_ceiling():
    """Streaming rates this GPU reaches with torch's own kernels over 1 GiB
    FP64 tensors: a device copy (16 B per element moved) and a sum (8 B read
    per element).  A practical ceiling for the HBM-bound passes, beside the
    published 8 TB/s peak that the roofline fraction is taken against."""
    import torch
    n = 1 << 27
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    rates = {}
    for name, fn, bytes_per in (("copy", lambda: y.copy_(x), 16), ("read", lambda: x.sum(), 8)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        e1.synchronize()
        rates[name] = bytes_per * n / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return {"copy_GBs": round(rates["copy"], 1), "read_GBs": round(rates["read"], 1),
            "copy_frac_of_peak": round(rates["copy"] / PEAK["hbm_GBs"], 4),
            "read_frac_of_peak": round(rates["read"] / PEAK["hbm_GBs"], 4),
            "how": "torch copy_ and sum over 1 GiB FP64 tensors, 10 launches between HIP events"}


def rel_errors(u, ref):
    """(||u - ref||_2 / ||ref||_2, max|u - ref| / max|ref|)."""
    d = u - ref
    n2, ninf = np.linalg.norm(ref), np.max(np.abs(ref))
    return (float(np.linalg.norm(d) / (n2 if n2 > 0 else 1.0)),
            float(np.max(np.abs(d)) / (ninf if ninf > 0 else 1.0)))


def serving_bench(args):
    """Request-stream benchmark of the server (one JSON line).

    2000 seeded requests (synth.serving_requests): grid uniform from five
    sizes, one boundary condition per axis from {P, D, N, DN}, tol from
    {1e-8, 1e-10}, inter-arrival gaps exponential.  Each request's field is
    one of 8 charge fields per grid size held in HBM before timing (10^4
    charges + N(0, 1e-3) noise, zero mean).  HBM budget 200 GB for plans,
    workspaces and staging.  Phases: closed loop (every request queued at
    once) gives the saturated throughput mu; open loop at 0.8 mu (Poisson
    arrivals, latency = completion - arrival on the server clock) gives
    p50 / p99, also at 0.5, 1.0 and 1.2 mu; 50 sampled requests are replayed
    one at a time (alone) and compared with their in-mix results and
    latencies; the same closed loop with the FP64 preconditioner; the oracle
    checks a seeded sample of 20 requests from each (grid, singular) stratum
    of the stream against the results the 0.8 mu run gave."""
    import threading
    import torch
    import synth
    from paper_2501_03377_amd import Server, KP_FLAG_FLEX_BETA

    prec = args.prec or "f32"
    count = args.requests
    reqs = synth.serving_requests(count=count, seed=4)
    grids = synth.SERVING_GRIDS
    torch.cuda.set_device(0)
    log(f"serving: {count} requests, generating 8 fields per grid size")
    pools = {}
    for gi, (nx, ny, nz) in enumerate(grids):
        pools[(nx, ny, nz)] = [
            torch.from_numpy(synth.charge_field((nz, ny, nx), ncharges=10_000, noise_std=1e-3,
                                                seed=40_000 + 8 * gi + k)).cuda()
            for k in range(8)]
    rng = np.random.default_rng(44)
    sample = sorted(rng.choice(count, size=min(50, count), replace=False).tolist())
    # the oracle's check: a seeded sample stratified by (grid, singular), up to
    # 20 requests of every stratum the stream holds
    import oracle
    stratum = lambda i: (tuple(reqs[i]["grid"]), oracle.is_singular(reqs[i]["bcs"]))
    strata = {}
    for i in range(count):
        strata.setdefault(stratum(i), []).append(i)
    rng_c = np.random.default_rng(45)
    check = sorted(j for key in sorted(strata) for j in
                   rng_c.choice(strata[key], size=min(20, len(strata[key])), replace=False).tolist())
    kept = sorted(set(sample) | set(check))
    flags = KP_FLAG_FLEX_BETA if prec == "bf16" else 0
    budget = int(200e9)

    def eta_of(r):
        return pools[tuple(r["grid"])][r["field_seed"] % 8]

    def drain(srv, n):
        done = {}
        while len(done) < n:
            for c in srv.poll(max_n=512, timeout=1.0):
                done[c["id"]] = c
        return done

    def closed_loop(srv, p, outs=None):
        t0 = srv.now()
        for r in reqs:
            srv.submit(r["id"], eta_of(r), r["bcs"], tol=r["tol"], prec=p, flags=flags,
                       u=(outs or {}).get(r["id"]))
        done = drain(srv, len(reqs))
        t1 = max(c["t_end"] for c in done.values())
        return done, len(reqs) / (t1 - t0)

    def open_loop(srv, p, rate, outs=None):
        arrivals = np.cumsum([r["gap"] for r in reqs]) / rate
        t0 = srv.now() + 0.05

        def submitter():
            for r, ta in zip(reqs, arrivals):
                delay = t0 + ta - srv.now()
                if delay > 0:
                    time.sleep(delay)
                srv.submit(r["id"], eta_of(r), r["bcs"], tol=r["tol"], prec=p, flags=flags,
                           u=(outs or {}).get(r["id"]))

        th = threading.Thread(target=submitter)
        th.start()
        done = drain(srv, len(reqs))
        th.join()
        lat = np.array([c["t_end"] - c["t_submit"] for c in done.values()])
        t_first = min(c["t_submit"] for c in done.values())
        t_last = max(c["t_end"] for c in done.values())
        return done, {"rate_offered": rate, "solves_per_s": len(reqs) / (t_last - t_first),
                      "p50_ms": float(np.percentile(lat, 50) * 1e3),
                      "p99_ms": float(np.percentile(lat, 99) * 1e3),
                      "mean_batch": float(np.mean([c["batch"] for c in done.values()]))}

    srv = Server(hbm_budget=budget, workers=args.workers, max_batch=args.max_batch)
    try:
        log("closed loop (cold plan cache)")
        done_cold, mu_cold = closed_loop(srv, prec)
        log("closed loop (warm plan cache)")
        done_mu, mu = closed_loop(srv, prec)
        bad = [c for c in done_mu.values() if c["status"] != 0]
        if bad:
            raise RuntimeError(f"{len(bad)} requests failed, first: {bad[0]}; "
                               f"server: {srv.last_error()}")
        outs = {i: torch.empty_like(eta_of(reqs[i])) for i in kept}
        levels = {}
        for frac in ([0.8] + ([0.5, 1.0, 1.2] if args.sweep else [])):
            log(f"open loop at {frac} mu")
            d, lv = open_loop(srv, prec, frac * mu, outs if frac == 0.8 else None)
            levels[str(frac)] = lv
            if frac == 0.8:
                mix = d
        mix_u = {i: outs[i].cpu().numpy() for i in kept}
        del outs
        log("alone replay of the sampled requests")
        alone_lat, same = [], 0
        for i in sample:
            r = reqs[i]
            u = torch.empty_like(eta_of(r))
            srv.submit(i, eta_of(r), r["bcs"], tol=r["tol"], prec=prec, flags=flags, u=u)
            c = drain(srv, 1)[i]
            alone_lat.append(c["t_end"] - c["t_submit"])
            same += int(np.array_equal(u.cpu().numpy(), mix_u[i]))
        mix_lat = [mix[i]["t_end"] - mix[i]["t_submit"] for i in sample]
        st = srv.stats()
    finally:
        srv.close()

    comp = {}
    if not args.no_compare:
        # the same stream with the FP64 preconditioner, and with its int8
        # split where every grid allows it
        for p in ("f64", "i8x7", "i8x6"):
            if p == prec or (p in INT8_PRODUCTS and not all(int8_fits(g) for g in grids)):
                continue
            log(f"closed loop, {'FP64' if p == 'f64' else p.upper()} preconditioner")
            srv = Server(hbm_budget=budget, workers=args.workers, max_batch=args.max_batch)
            try:
                closed_loop(srv, p)
                _, mu_p = closed_loop(srv, p)
                comp[p] = {"solves_per_s": mu_p}
            finally:
                srv.close()

    lv = levels["0.8"]
    out = {
        "metric": METRIC, "value": mu, "unit": "solves/s", "n_gpus": 1,
        "steps": count, "warmup": count, "ms_per_step": 1e3 / mu, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": f"serving: {count} requests, grids {list(map(list, grids))}, "
                               "BC per axis from P/D/N/DN, tol 1e-8 or 1e-10, Poisson arrivals, "
                               f"HBM budget 200 GB, {prec.upper()} preconditioner; value = "
                               "saturated closed-loop throughput (warm plan cache)",
                   "workers": args.workers, "max_batch": args.max_batch},
        "p50_ms": lv["p50_ms"], "p99_ms": lv["p99_ms"],
        "serving": {"mu_cold": mu_cold, "mu": mu, "open_loop": levels,
                    "hbm_high_water_GB": st["hbm_high_water"] / 1e9,
                    "plans_created": st["plans_created"], "plans_evicted": st["plans_evicted"],
                    "batches": st["batches"], "rejected": st["rejected"],
                    "alone_vs_mix": {"requests": len(sample), "bitwise_equal": same,
                                     "alone_p50_ms": float(np.median(alone_lat) * 1e3),
                                     "mix_p50_ms": float(np.median(mix_lat) * 1e3)}},
        "compare": comp,
    }
    if "f64" in comp:
        out["speedup_vs_fp64"] = mu / comp["f64"]["solves_per_s"]
        for p, c in comp.items():
            if p != "f64":
                c["speedup_vs_fp64"] = c["solves_per_s"] / comp["f64"]["solves_per_s"]
    if not args.no_cpu_baseline:
        # the oracle on the stratified check sample (every stratum, up to 20
        # requests each), in stratum order; its rate is the CPU baseline
        from threadpoolctl import threadpool_info
        log(f"oracle on {len(check)} requests, {len(strata)} (grid, singular) strata")
        t_all, errs = time.perf_counter(), []
        for i in check:
            r = reqs[i]
            H = eta_of(r).cpu().numpy().T
            sol = oracle.min_norm_solution(H, r["bcs"])[0].T
            errs.append(float(np.linalg.norm(mix_u[i] - sol) / np.linalg.norm(sol)))
        dt = time.perf_counter() - t_all
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
        out["cpu_baseline"] = {"value": len(check) / dt, "unit": "solves/s", "cores": int(threads),
                               "kind": "oracle",
                               "sample": f"{len(check)} requests of the stream, a seeded sample "
                                         f"stratified by (grid, singular): up to 20 of each of the "
                                         f"{len(strata)} strata (the minimum-norm solution from "
                                         "the eigen-expansion, LAPACK eigh bases, FP64 numpy)"}
        out["rel_err_vs_oracle"] = max(errs)
        out["rel_err_over_tol"] = max(e / reqs[i]["tol"] for e, i in zip(errs, check))
        out["oracle_checked"] = len(check)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="large512", choices=sorted(WORKLOADS) + ["serving"])
    ap.add_argument("--requests", type=int, default=2000, help="serving: stream length")
    ap.add_argument("--workers", type=int, default=4, help="serving: worker threads")
    ap.add_argument("--max-batch", type=int, default=4, help="serving: largest batch")
    ap.add_argument("--sweep", action="store_true", help="serving: also 0.5, 1.0, 1.2 mu")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", default=None, choices=list(PRECS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shapes")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison runs in the other precisions (for profiler runs)")
    ap.add_argument("--ingest-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE) of this "
                         "workload into its traffic record under profiles/, then exit")
    ap.add_argument("--ingest-command", default="", help="the profiler command, for the record")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain device copy of 256 MiB three times, the reference "
                         "that scales the FETCH_SIZE / WRITE_SIZE counters of a profiler run")
    ap.add_argument("--ingest-mfma", nargs=2, metavar=("COUNTER_DIR", "BENCH_LOG"),
                    help="print the matrix-core counters of a rocprofv3 run of this workload "
                         "and --prec per mode-product kernel (markdown rows), then exit")
    args = ap.parse_args()
    if args.ingest_mfma:
        prec = args.prec or WORKLOADS[args.workload]["prec"]
        print("| kernel | products | dispatches | avg us | GRBM cycles/ns | MFMA busy | "
              "ops per CU-cycle (of peak) | algorithmic HBM (of 8 TB/s) |")
        print("|---|---|---|---|---|---|---|---|")
        print("\n".join(ingest_mfma(*args.ingest_mfma, args.workload, prec)))
        return
    if args.ingest_traffic:
        rec = ingest_traffic(args.workload, *args.ingest_traffic, args.ingest_command)
        print(f"wrote {traffic_path(args.workload)}: {len(rec['kernels'])} kernels")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent solves shard across GPUs without communication).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "serving":
        serving_bench(args)
        return

    import torch
    from paper_2501_03377_amd import Plan, KP_FLAG_FLEX_BETA

    wl = WORKLOADS[args.workload]
    prec = args.prec or wl["prec"]
    steps = args.steps or wl["steps"]
    tol, batch, bcs = wl["tol"], wl["batch"], wl["bcs"]
    nx, ny, nz = wl["grid"]
    N = nx * ny * nz

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(COPY_CAL_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(COPY_CAL_RUNS):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"workload {args.workload}: generating input")
    eta = make_eta(wl)
    eta_d = torch.from_numpy(eta).cuda()
    flex = lambda p: KP_FLAG_FLEX_BETA if p == "bf16" else 0

    def kernel_table(prof, p, results, nsolves):
        table = {}
        for name, (ms, cnt) in prof.items():
            if cnt == 0:
                continue
            avg_us = 1000.0 * ms / cnt
            kind, work = solve_work(name, wl["grid"], results, p == "bf16",
                                    p in FP64_ACCURATE)
            units = work * nsolves / cnt            # algorithmic work per launch
            entry = {"avg_us": round(avg_us, 2), "launches": cnt, "total_ms": round(ms, 3)}
            if kind == "flop":
                tf = units / (avg_us * 1e-6) / 1e12
                entry.update({"TFLOPs": round(tf, 2), "frac_peak": round(tf / PEAK[p], 4)})
                if name in MODEPROD:
                    # the same launches against the HBM roof (the one that
                    # binds BF16 products): algorithmic bytes of the
                    # applications that ran, over the traced time
                    apps = sum(r["pinv_applications"] for r in results) * nsolves
                    gbs = product_bytes(name, p, wl["grid"]) * apps / cnt / (avg_us * 1e-6) / 1e9
                    entry.update({"GBs_alg": round(gbs, 1),
                                  "hbm_frac": round(gbs / PEAK["hbm_GBs"], 4)})
            elif kind == "byte":
                gbs = units / (avg_us * 1e-6) / 1e9
                entry.update({"GBs": round(gbs, 1), "frac_peak": round(gbs / PEAK["hbm_GBs"], 4)})
            table[name] = entry
        return table

    def measure(p, k, time_dominant=False):
        """Tuned plan, warmup, k timed solves (graphs, no timing events), then
        k profiled solves (per-launch HIP events, direct launches)."""
        log(f"{p}: plan + autotune")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = Plan(nx, ny, nz, bcs, prec=p, max_batch=batch)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tuning = plan.autotune(batch=batch, reps=3) if not args.no_tune else plan.tuning
        torch.cuda.synchronize()
        plan_ms, tune_ms = (t1 - t0) * 1e3, (time.perf_counter() - t1) * 1e3
        uu = torch.empty_like(eta_d)
        run_solves(plan, eta_d, uu, args.warmup, tol, flex(p))
        log(f"{p}: {k} timed solves")
        T, lat, res = run_solves(plan, eta_d, uu, k, tol, flex(p))
        uh = uu.cpu().numpy()
        fresh = None
        if time_dominant:
            # the same solves alternating between two (eta, u) buffer pairs, as
            # a caller that switches buffers: no call repeats the previous
            # one's pointers, so the whole-solve graph is not replayed (the
            # start is launched directly, the iterations replay a graph
            # captured per pair)
            log(f"{p}: {k} solves alternating two buffer pairs")
            pairs = [(eta_d, uu), (eta_d.clone(), torch.empty_like(eta_d))]
            flat = []
            for i in range(k + 2):
                e_, u_ = pairs[i % 2]
                _, fl, _ = run_solves(plan, e_, u_, 1, tol, flex(p))
                if i >= 2:                 # the first use of each pair captures its graph
                    flat.append(fl[0])
            flat = np.array(flat)
            fresh = {"p50_ms": round(float(np.percentile(flat, 50)) * 1e3, 4),
                     "p99_ms": round(float(np.percentile(flat, 99)) * 1e3, 4),
                     "solves": int(flat.size),
                     "note": "solves alternating between two (eta, u) buffer pairs: each "
                             "solve's start launched directly, its iterations replaying a graph "
                             "captured per pair (the timed region repeats one pair and replays "
                             "the whole-solve graph)"}
            del pairs
        log(f"{p}: {k} profiled solves")
        plan.set_profiling(True)
        plan.profile_reset()
        Tp, _, _ = run_solves(plan, eta_d, uu, k, tol, flex(p))
        prof = plan.profile()
        kernels = kernel_table(prof, p, res, k)
        dom = None
        if time_dominant:
            # the roofline's kernel: the most expensive class with a defined
            # algorithmic work (the scalar finalize kernels are latency, not
            # work), timed back to back so that its average is the kernel's
            # own duration (the traced averages above include launch gaps)
            # (small 2D problems: the whole solve is one kernel, timed on
            # the last solve's arguments)
            timed = [c for c in kernels
                     if launch_work(c, wl["grid"], 1)[0] is not None or c == "small_solve"]
            cls = max(timed, key=lambda c: kernels[c]["total_ms"])
            reps = int(min(2000, max(20, 0.2e6 / max(kernels[cls]["avg_us"], 1.0))))
            log(f"{p}: {reps} back-to-back launches of {cls}")
            dom = (cls, plan.time_kernel(cls, batch=batch, flags=flex(p), reps=reps), reps)
        plan.close()
        return dict(T=T, lat=lat, res=res, u=uh, tuning=tuning, Tp=Tp, kernels=kernels, dom=dom,
                    plan_ms=plan_ms, tune_ms=tune_ms, fresh=fresh)

    m = measure(prec, steps, time_dominant=True)
    kernels, res = m["kernels"], m["res"]
    dom, dom_ms, dom_reps = m["dom"]
    kind, units = launch_work(dom, wl["grid"], batch, prec == "bf16")
    if kind is None:            # one launch per solve: the solve's work
        kind, units = solve_work(dom, wl["grid"], res, prec == "bf16", prec in FP64_ACCURATE)
    rate = units / (dom_ms * 1e-3)
    ident = launch_identity(dom, prec, wl["grid"], batch, m["tuning"])
    traffic = measured_traffic(args.workload, ident)
    if kind == "flop" and prec in INT8_PRODUCTS:
        # the int8 split issues 28 (i8x7) or 21 (i8x6) exact int8 digit
        # products for every FP64 multiply-add of the contraction: its
        # matrix-core work is that many times the algorithmic flops, priced
        # against the published dense int8 peak
        ops = INT8_PRODUCTS[prec] * rate
        roof = {"bound": "mfma", "achieved": round(ops / 1e12, 1), "peak": 5000.0,
                "unit": "TOP/s", "frac": round(ops / 1e12 / 5000.0, 4),
                "mfma_dtype": "int8",
                "fp64_equivalent_TFLOPs": round(rate / 1e12, 2)}
    elif kind == "flop":
        roof = {"bound": "mfma", "achieved": round(rate / 1e12, 2), "peak": PEAK[prec],
                "unit": "TFLOP/s", "frac": round(rate / 1e12 / PEAK[prec], 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(rate / 1e9, 1), "peak": PEAK["hbm_GBs"],
                "unit": "GB/s", "frac": round(rate / 1e9 / PEAK["hbm_GBs"], 4)}
    if dom in MODEPROD:
        roof["hbm_frac_alg"] = round(product_bytes(dom, prec, wl["grid"]) * batch
                                     / (dom_ms * 1e-3) / 1e9 / PEAK["hbm_GBs"], 4)
    # working set of the solve (the FP64 vectors eta, u, R, P, W, Z and the two
    # product buffers): below about 1 GB part of it can stay in the 256 MB
    # Infinity Cache, and a rate against the HBM peak then overstates HBM use
    ws = batch * N * (6 * 8 + 2 * ELEM_BYTES[prec])
    roof["working_set_bytes"] = ws
    if ws < 1 << 30:
        roof["cache_caveat"] = ("working set below 1 GB: partly resident in the 256 MB "
                                "Infinity Cache, so HBM fractions are upper bounds")
    roof.update({"traffic": traffic, "kernel": dom, "launch": ident,
                 "avg_us": round(dom_ms * 1e3, 2), "launches_timed": dom_reps,
                 "algorithmic_per_launch": units})
    if traffic is not None and kind == "byte":
        roof["traffic_over_algorithmic"] = round(traffic / units, 3)
    elif traffic is not None and dom in MODEPROD:
        roof["traffic_over_algorithmic_bytes"] = round(
            traffic / (product_bytes(dom, prec, wl["grid"]) * batch), 3)
    ceiling = stream_ceiling()
    if dom == "small_solve":
        # one workgroup, hence one of the 256 compute units, per right-hand side
        cus = min(batch, 256)
        roof["frac_of_used_cus"] = round(roof["frac"] * 256 / cus, 4)

    its = [r["iterations"] for r in res]
    out = {
        "metric": METRIC,
        "value": batch * steps / m["T"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * m["T"] / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {wl['desc']}; to rel. residual {tol:g} with the "
                        f"{prec.upper()} pseudoinverse preconditioner",
            "grid": list(wl["grid"]), "bcs": list(bcs), "pinv_precision": prec, "tol": tol,
            "batch": batch, "tile_configs": m["tuning"],
        },
        "p50_ms": float(np.percentile(m["lat"], 50) * 1000.0),
        "p99_ms": float(np.percentile(m["lat"], 99) * 1000.0),
        "fresh_buffers": m["fresh"],
        "iterations": max(its),
        "iterations_min": min(its),
        "pinv_applications": max(r["pinv_applications"] for r in res),
        "rel_res": max(r["rel_res"] for r in res),
        "true_rel_res": max(r["true_rel_res"] for r in res),
        "unknowns_iterations_per_s": N * sum(its) * steps / m["T"],
        # once per plan, outside the timed solves: closed-form bases and
        # their upload, then the tile autotuner
        "plan_ms": round(m["plan_ms"], 3), "autotune_ms": round(m["tune_ms"], 1),
        "ms_per_step_profiled": 1000.0 * m["Tp"] / steps,
        "roofline": roof,
        "stream_ceiling": ceiling,
        "kernels": kernels,
    }

    if not args.no_compare:
        comp = {}
        for p in PRECS:
            if p == prec or (p in INT8_PRODUCTS and not int8_fits(wl["grid"])):
                continue
            c = measure(p, max(3, steps // 4))
            comp[p] = {"solves_per_s": batch * len(c["lat"]) / c["T"],
                       "p50_ms": float(np.percentile(c["lat"], 50) * 1000.0),
                       "iterations": max(r["iterations"] for r in c["res"]),
                       "pinv_applications": max(r["pinv_applications"] for r in c["res"]),
                       "kernels": c["kernels"], "u": c["u"]}
        out["compare"] = comp

    if not args.no_cpu_baseline:
        log("oracle on the host cores")
        sols, cpu = cpu_baseline(wl, eta)
        out["cpu_baseline"] = cpu

        def err(uh):
            uh = uh if batch > 1 else uh[None]
            e = [rel_errors(uh[b], s) for b, s in sols.items()]
            return max(x[0] for x in e), max(x[1] for x in e)
        out["rel_err_vs_oracle"], out["max_err_vs_oracle"] = err(m["u"])
        out["rel_err_sample"] = (f"max over RHS {sorted(sols)}; rel_err = ||u - u_o||_2 / "
                                 "||u_o||_2, max_err = max|u - u_o| / max|u_o|")
        for c in out.get("compare", {}).values():
            c["rel_err_vs_oracle"], c["max_err_vs_oracle"] = err(c["u"])
    for c in out.get("compare", {}).values():
        c.pop("u", None)
    if "f64" in out.get("compare", {}):
        f64 = out["compare"]["f64"]["solves_per_s"]
        out["speedup_vs_fp64"] = out["value"] / f64
        for p, c in out["compare"].items():
            if p != "f64":
                c["speedup_vs_fp64"] = c["solves_per_s"] / f64
    print(json.dumps(out))


if __name__ == "__main__":
    main()
