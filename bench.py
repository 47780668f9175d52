"""Benchmark of the sparse leaf path on one MI355X.

Workload: the power-law CSR matrix of 2,000,000 x 2,000,000 with Pareto
(alpha = 2) row degrees, 32,000,000 nonzeros and a degree cap of 50,000,
uniform distinct columns, values uniform[-1, 1]; a dense vector of 2,000,000
and a dense 2,000,000 x 32 row-major operand.  Inputs are generated on the
GPU and resident in HBM before timing starts.

One step is the whole hot path on that batch in FP32: the tile partition of
the matrix, the SpMV leaf a = B c, the SpMM leaf A = B C and their carry
fix-ups, each with the schedule the exhaustive autotuner picked (untimed,
before warm-up).  `value` is GFLOP/s of the step (2 nnz + 2 nnz N flops).

Besides the headline line it reports, from the same run:
 - roofline: the dominant leaf kernel (SpMM) against the 8 TB/s HBM peak,
   with its duration taken from HIP events the library records around that
   kernel on its own stream during the timed steps, and its HBM-side
   traffic from hardware counters when they were taken on these sources;
 - leaf_spread: min / median / max per-launch time of the SpMV and SpMM
   leaves, back to back (warm) and after a 1 GiB write that flushes the
   256 MB MALL (cold);
 - variants: FP64 SpMV/SpMM and BF16 SpMM (FP32 accumulation) with the same
   schedules, and the row / non-zero / merge schedules compared;
 - ops: every other leaf at its full workload, and the SpMV of the paper's
   weak-scaling study at one GPU's share (banded, 7e8 nonzeros, FP64),
   each warm (median, min, max) and with the MALL flushed (cold_ms);
 - cpu_baseline: the CPU oracle timed on the host on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 10]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_COLS = 32
# HBM traffic of the SpMM leaf measured with hardware counters (FETCH_SIZE,
# WRITE_SIZE, each scaled against a plain 1 GiB device copy); used only while
# the kernel sources are the ones the counters were taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmm_leaf_traffic_powerlaw2M.txt")
SPMM_SOURCES = [os.path.join(ROOT, "paper_2207_13901_amd", "csrc", f)
                for f in ("spmm.hip", "device.hpp")]


def sources_digest(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counted_traffic(schedule):
    """Counter-measured HBM bytes per SpMM leaf launch, or None when the
    record is missing, was taken on other kernel sources or with another
    leaf kernel (kind, col_tile, items_per_lane, variant; the merge tile only
    sets how many chunks a workgroup walks, so it changes the carries, a few
    KB, not the leaf's traffic)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    try:
        if rec.get("sources_digest") != sources_digest(SPMM_SOURCES):
            return None
        keys = ("kind", "col_tile", "items_per_lane", "variant")
        rs = json.loads(rec["schedule"])
        if any(rs.get(k, 0) != schedule.get(k, 0) for k in keys):
            return None
        return int(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def spmm_kernel_name(sched):
    """Leaf kernel a SpMM schedule dispatches for the FP32 N=32 operands."""
    kind = sched.get("kind", "merge")
    if kind == "row":
        return "k_spmm_row"
    if kind == "nnz":
        return "k_spmm_tiles"
    vec = (sched.get("variant", 0) == 0 and sched.get("items_per_lane", 16) <= 16 and
           sched.get("col_tile", 32) >= 32)
    return "k_spmm_pipe, 4 columns per lane" if vec else "k_spmm_pipe"


def algorithmic_bytes(n, m, nnz, N, vbytes, dbytes, obytes):
    """Compulsory bytes of one leaf launch: pos, crd, vals read once, each
    dense input row read once and each output row written once."""
    spmv = 4 * (n + 1) + (4 + vbytes) * nnz + dbytes * m + obytes * n
    spmm = 4 * (n + 1) + (4 + vbytes) * nnz + dbytes * m * N + obytes * n * N
    return spmv, spmm


def tuning_median(fn, reps, warmup):
    from paper_2207_13901_amd import tuning
    return tuning.time_call(fn, reps=reps, warmup=warmup)


def _rate(ms, nbytes, flops, spread=None):
    out = {"ms": round(ms, 5), "GB_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
           "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "GFLOP_s": round(flops / (ms * 1e-3) / 1e9, 2), "algorithmic_bytes": int(nbytes)}
    if spread:
        out.update(spread)
        out["cold_frac_hbm"] = round(nbytes / (spread["cold_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


_FLUSH = []
_COLD = [True]  # --no-cold clears it


def _time_ops(fn, reps=10, warmup=3):
    """Median milliseconds of fn() back to back (warm), plus min / max and the
    median with the 256 MB MALL flushed by a 1 GiB write before each call
    (cold; the write itself is not timed)."""
    import torch
    if not _COLD[0]:
        return tuning_median(fn, reps, warmup), None
    if not _FLUSH:
        _FLUSH.append(torch.empty(1 << 28, dtype=torch.float32, device="cuda"))
    flush = _FLUSH[0]

    def once(cold):
        if cold:
            flush.fill_(1.0)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b)

    for _ in range(warmup):
        fn()
    warm = sorted(once(False) for _ in range(reps))
    cold = sorted(once(True) for _ in range(reps))
    return warm[len(warm) // 2], {"min_ms": round(warm[0], 5), "max_ms": round(warm[-1], 5),
                                  "cold_ms": round(cold[len(cold) // 2], 5)}


def measure_banded(dev, spl, tuning, torch):
    """One GPU's share of the paper's weak-scaling SpMV: the banded CSR of
    20,000,000 rows with 35 nonzeros per interior row (699,999,694), FP64
    values and vector; the fastest of a few schedules, median of 10 calls."""
    from workloads import configs
    print("[bench] generating the 7e8-nonzero banded matrix", file=sys.stderr, flush=True)
    c = configs.banded(device=dev)
    n = c["n"]
    nnz = int(c["crd"].numel())
    B = spl.CSR(c["pos"], c["crd"], c["vals"], (n, n))
    x = c["x"]
    y = torch.empty(n, dtype=torch.float64, device=dev)
    cands = ([dict(kind="row", lanes_per_row=L) for L in (8, 16, 32, 64)] +
             [dict(kind="merge", tile=T, items_per_lane=4) for T in (4096, 16384)] +
             [dict(kind="merge", tile=T, items_per_lane=8) for T in (8192, 32768)] +
             [dict(kind="merge", tile=4096, items_per_lane=4, variant=1),
              dict(kind="nnz", tile=4096, items_per_lane=8)])
    best, res = tuning.search(lambda s: (lambda: spl.spmv(B, x, y, sched=s)), cands, reps=3)
    ms, ms_spread = _time_ops(lambda: spl.spmv(B, x, y, sched=spl.schedule(**best)))
    out = _rate(ms, 4 * (n + 1) + 12 * nnz + 8 * n + 8 * n, 2 * nnz, ms_spread)
    out.update(schedule=best, n=n, nnz=nnz,
               schedules_ms={json.dumps(c, sort_keys=True): round(t, 4) for c, t in res})
    del B, c, x, y
    torch.cuda.empty_cache()
    return out


def measure_banded64(dev, spl, tuning, torch, n=62_000_000):
    """The banded matrix at 62,000,000 rows (2,169,999,694 nonzeros, 26 GB in
    FP64): positions pass 2^31, so pos is int64; merge schedules only."""
    from workloads import configs
    print("[bench] generating the 2.17e9-nonzero banded matrix", file=sys.stderr, flush=True)
    c = configs.banded(device=dev, n=n, pos_dtype=torch.int64)
    nnz = int(c["crd"].numel())
    B = spl.CSR(c["pos"], c["crd"], c["vals"], (n, n))
    x = c["x"]
    y = torch.empty(n, dtype=torch.float64, device=dev)
    cands = ([dict(kind="merge", tile=T, items_per_lane=4) for T in (4096, 16384)] +
             [dict(kind="merge", tile=T, items_per_lane=8) for T in (8192, 32768)])
    best, res = tuning.search(lambda s: (lambda: spl.spmv(B, x, y, sched=s)), cands, reps=3)
    ms, ms_spread = _time_ops(lambda: spl.spmv(B, x, y, sched=spl.schedule(**best)))
    out = _rate(ms, 8 * (n + 1) + 12 * nnz + 8 * n + 8 * n, 2 * nnz, ms_spread)
    out.update(schedule=best, n=n, nnz=nnz, pos="int64",
               schedules_ms={json.dumps(c, sort_keys=True): round(t, 4) for c, t in res})
    del B, c, x, y
    torch.cuda.empty_cache()
    return out


def measure_coord_partition(dev, spl, tuning, torch, ncolors=8):
    """The value-range partition of the power-law matrix's columns into
    eight equal blocks (one kernel), and the SpMV as the sum of the eight
    column blocks' windowed products (FP64), against the whole SpMV."""
    import numpy as np
    from workloads import configs
    c = configs.config2(device=dev, with_dense=False)
    n = c["n"]
    nnz = int(c["crd"].numel())
    B = spl.CSR(c["pos"], c["crd"], c["vals"], (n, n))
    x = c["x"]
    bounds = torch.as_tensor(np.linspace(0, n, ncolors + 1).astype(np.int32), device=dev)
    out = torch.empty(ncolors + 1, n, dtype=torch.int32, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    ms_p, ms_p_spread = _time_ops(lambda: spl.coord_partition(B, bounds, out))
    spl.coord_partition(B, bounds, out)
    lanes = [dict(kind="row", lanes_per_row=L) for L in (1, 2, 4, 8)] + \
        [dict(kind="merge", tile=T, items_per_lane=it)
         for T, it in ((1024, 4), (4096, 4), (2048, 8), (8192, 8))]

    def windows(sc):
        for col in range(ncolors):
            spl.spmv_window(B, out[col], out[col + 1], x, y, sched=sc)

    best, _ = tuning.search(lambda sc: (lambda: windows(sc)), lanes, reps=3)
    sb = spl.schedule(**best)
    ms_w, ms_w_spread = _time_ops(lambda: windows(sb))
    res = {"partition": _rate(ms_p, 4 * (n + 1) + 4 * nnz + 4 * (ncolors + 1) * n, 0,
                              ms_p_spread),
           "windows_spmv_f64": _rate(ms_w, ncolors * 8 * n + 12 * nnz + 8 * n + ncolors * 8 * n,
                                     2 * nnz, ms_w_spread)}
    res["windows_spmv_f64"]["schedule"] = best
    res["workload"] = (f"power-law CSR {n}^2, {nnz} nnz, FP64; {ncolors} equal column blocks, "
                       f"the SpMV as the {ncolors} blocks' windowed products")
    del B, c, x, out, y
    torch.cuda.empty_cache()
    return res


# SpTTV runs the SpMV leaf on the fiber level: the SpMV candidates plus
# longer merge tiles (several chunks per workgroup), which short fibers favour
def _ttv_candidates():
    from paper_2207_13901_amd import tuning
    return tuning.SPMV_CANDIDATES + [dict(kind="merge", tile=T, items_per_lane=it, variant=v)
                                     for T, it in ((4096, 4), (16384, 4), (8192, 8), (32768, 8))
                                     for v in (0, 2)]


TTV_CANDIDATES = _ttv_candidates()


def measure_ddc(dev, spl, tuning, torch):
    """SpTTV and SpMTTKRP (FP32) on the (Dense, Dense, Compressed) tensor
    shaped like the paper's "patents": 46 x 239,172 x 239,172 with 1e8
    values over 11,001,912 fibers; autotuned schedule, median of 10 calls.
    The MTTKRP time includes writing out the Dense middle level."""
    from workloads import configs
    print("[bench] generating the (Dense, Dense, Compressed) tensor", file=sys.stderr, flush=True)
    c = configs.ddc(device=dev)
    I, J, Kd = c["I"], c["J"], c["K"]
    F = I * J
    nnz = int(c["crd2"].numel())
    R = c["C"].shape[1]
    B = spl.DDC(c["pos2"], c["crd2"], c["vals"].to(torch.float32), (I, J, Kd))
    cv = c["c"].to(torch.float32)
    A = torch.empty(F, dtype=torch.float32, device=dev)
    out = {}
    best, _ = tuning.search(lambda s: (lambda: spl.spttv(B, cv, A, sched=s)),
                            TTV_CANDIDATES, reps=5)
    st = spl.schedule(**best)
    ms, ms_spread = _time_ops(lambda: spl.spttv(B, cv, A, sched=st))
    out["spttv_f32"] = _rate(ms, 4 * (F + 1) + 8 * nnz + 4 * Kd + 4 * F, 2 * nnz, ms_spread)
    out["spttv_f32"]["schedule"] = best
    del A
    C = c["C"].to(torch.float32)
    D = c["D"].to(torch.float32)
    M = torch.empty(I, R, dtype=torch.float32, device=dev)
    best, _ = tuning.search(lambda s: (lambda: spl.mttkrp(B, C, D, M, sched=s)),
                            tuning.MTTKRP_CANDIDATES, reps=3)
    sk = spl.schedule(**best)
    ws = spl.workspace(spl.N.OP_MTTKRP, B, R, sk)  # holds the expanded Dense level too
    ms, ms_spread = _time_ops(lambda: spl.mttkrp(B, C, D, M, sched=sk, ws=ws))
    nbytes = 4 * (F + 1) + 8 * nnz + 4 * (J + Kd) * R + 4 * I * R
    out["mttkrp_f32"] = _rate(ms, nbytes, 2 * R * (nnz + F), ms_spread)
    out["mttkrp_f32"]["schedule"] = best
    out["workload"] = f"(Dense, Dense, Compressed) {I}x{J}x{Kd}, {nnz} nnz, {F} fibers, R={R}"
    del B, C, D, M, c, cv, ws
    torch.cuda.empty_cache()
    return out


OPS = ("sddmm", "spadd3", "spttv", "mttkrp", "inner", "banded", "ddc", "coord", "banded64")


def measure_other_ops(dev, spl, tuning, torch, fixed=None, next_rows=True, only=None):
    """Every other leaf at its full workload: SDDMM and SpAdd3 on the three
    1,000,000-row CSR matrices, SpTTV, SpMTTKRP and the inner product on the
    200,000^3 CSF tensor with 1e8 nonzeros.  SpTTV and SpMTTKRP run with the
    autotuned schedule unless `fixed` gives one ({"spttv": {...},
    "mttkrp": {...}}).  Median (and min, max) of 10 timed calls after
    3 warm-up calls, inputs resident in HBM, and the median of 10 calls
    each after a 1 GiB write that flushes the MALL (cold_ms, cold_frac_hbm).
    `only`: a subset of OPS."""
    from workloads import configs
    want = set(only) if only else set(OPS if next_rows else OPS[:5])
    res = {}
    if want & {"sddmm", "spadd3"}:
        _ops_config3(dev, spl, tuning, torch, configs, want, res)
    if want & {"spttv", "mttkrp", "inner"}:
        _ops_config4(dev, spl, tuning, torch, configs, want, res, fixed or {})
    if "banded" in want:
        res["spmv_banded_f64"] = measure_banded(dev, spl, tuning, torch)
    if "ddc" in want:
        res["ddc"] = measure_ddc(dev, spl, tuning, torch)
    if "coord" in want:
        res["coord_partition"] = measure_coord_partition(dev, spl, tuning, torch)
    if "banded64" in want:
        res["spmv_banded_int64_f64"] = measure_banded64(dev, spl, tuning, torch)
    res["workloads"] = {
        "spadd3_sddmm": "3 CSR 1000000x1000000, Poisson(8) rows, 30% shared rows, K=128",
        "csf": "CSF 200000^3, 100000000 nnz, power-law slices, R=32",
        "banded": "CSR 20000000^2, rows i-17..i+17 (699999694 nnz), FP64",
    }
    return res


def _ops_config3(dev, spl, tuning, torch, configs, want, res):
    """SDDMM (FP32, BF16 on the vector ALUs, BF16 on the matrix cores) and
    SpAdd3 on the three 1,000,000-row CSR matrices."""
    print("[bench] generating the 1e6-row SpAdd3/SDDMM operands", file=sys.stderr, flush=True)
    c3 = configs.config3(device=dev)
    n = c3["n"]
    K = c3["Cd"].shape[1]
    ops = [spl.CSR(c3[k]["pos"], c3[k]["crd"], c3[k]["vals"].to(torch.float32), (n, n))
           for k in "BCD"]
    B = ops[0]
    nnzB = B.crd.numel()
    sddmm_forms = (("sddmm_f32", torch.float32, 0), ("sddmm_bf16_valu", torch.bfloat16, 0),
                   ("sddmm_bf16_mfma", torch.bfloat16, 1))
    for name, fdt, variant in sddmm_forms if "sddmm" in want else ():
        C = c3["Cd"].to(torch.float32).to(fdt)
        D = c3["Dd"].to(torch.float32).to(fdt)
        A = torch.empty(nnzB, dtype=torch.float32, device=dev)
        s = spl.schedule(variant=variant)
        ms, ms_spread = _time_ops(lambda: spl.sddmm(B, C, D, A, sched=s))
        esz = 2 if fdt == torch.bfloat16 else 4
        nbytes = 4 * (n + 1) + 8 * nnzB + K * n * esz * 2 + 4 * nnzB
        res[name] = _rate(ms, nbytes, nnzB * (2 * K + 1), ms_spread)
        del C, D, A
    if "spadd3" in want:
        # the forms (whole calls, both phases): merges a lane per row with 1 the
        # inputs read directly, 2 coordinates in LDS, 3 coordinates and values
        # in LDS; 4 ranks, a lane per input entry
        var_ms = {v: tuning.time_call(
            lambda v=v: spl.spadd3(*ops, sched=spl.schedule("row", variant=v)), reps=10, warmup=3)
            for v in (1, 2, 3, 4)}
        ms, ms_spread = _time_ops(lambda: spl.spadd3(*ops))
        out = spl.spadd3(*ops)
        nnzA = out.crd.numel()
        nnzs = sum(o.crd.numel() for o in ops)
        nbytes = (3 * 4 * (n + 1) + 4 * nnzs + 4 * (n + 1)) + \
                 (3 * 4 * (n + 1) + 8 * nnzs + 4 * (n + 1) + 8 * nnzA)
        res["spadd3_f32"] = _rate(ms, nbytes, nnzs - nnzA, ms_spread)
        res["spadd3_f32"]["nnz_out"] = nnzA
        res["spadd3_f32"]["variants_ms"] = {str(v): round(t, 5) for v, t in var_ms.items()}
        del out
    del ops, B, c3
    torch.cuda.empty_cache()


def _ops_config4(dev, spl, tuning, torch, configs, want, res, fixed):
    """SpTTV, SpMTTKRP (FP32 and BF16) and the inner products on the CSF
    tensor of 200,000^3 with 1e8 nonzeros."""
    print("[bench] generating the 1e8-nonzero CSF tensor", file=sys.stderr, flush=True)
    c4 = configs.config4(device=dev)
    I, J, Kd = c4["I"], c4["J"], c4["K"]
    F = c4["crd1"].numel()
    nnz = c4["crd2"].numel()
    R = c4["C"].shape[1]
    B32 = spl.CSF(c4["pos1"], c4["crd1"], c4["pos2"], c4["crd2"], c4["vals"].to(torch.float32),
                  (I, J, Kd))
    cv = c4["c"].to(torch.float32)
    if "spttv" in want:
        At = torch.empty(F, dtype=torch.float32, device=dev)
        # SpTTV is the SpMV leaf on the fiber level: the same candidate schedules
        if "spttv" in fixed:
            best_t = fixed["spttv"]
        else:
            best_t, _ = tuning.search(lambda s: (lambda: spl.spttv(B32, cv, At, sched=s)),
                                        TTV_CANDIDATES, reps=5)
        st = spl.schedule(**best_t)
        ms, ms_spread = _time_ops(lambda: spl.spttv(B32, cv, At, sched=st))
        res["spttv_f32"] = _rate(ms, 4 * (F + 1) + 8 * nnz + 4 * Kd + 4 * F, 2 * nnz, ms_spread)
        res["spttv_f32"]["schedule"] = best_t
        del At
    mttkrp_forms = (("mttkrp_f32", torch.float32), ("mttkrp_bf16_f32acc", torch.bfloat16))
    for name, dt in mttkrp_forms if "mttkrp" in want else ():
        Bt = B32.with_vals(B32.vals.to(dt))
        C = c4["C"].to(torch.float32).to(dt)
        D = c4["D"].to(torch.float32).to(dt)
        M = torch.empty(I, R, dtype=torch.float32, device=dev)
        if "mttkrp" in fixed:
            best_k = fixed["mttkrp"]
        else:
            best_k, _ = tuning.search(lambda s: (lambda: spl.mttkrp(Bt, C, D, M, sched=s)),
                                        tuning.MTTKRP_CANDIDATES, reps=3)
        sk = spl.schedule(**best_k)
        ms, ms_spread = _time_ops(lambda: spl.mttkrp(Bt, C, D, M, sched=sk))
        esz = 2 if dt == torch.bfloat16 else 4
        nbytes = 4 * (I + 1) + 4 * F + 4 * (F + 1) + (4 + esz) * nnz + esz * (J + Kd) * R + 4 * I * R
        res[name] = _rate(ms, nbytes, 2 * R * (nnz + F), ms_spread)
        res[name]["schedule"] = best_k
        del Bt, C, D, M
    if "inner" in want:
        B64 = B32.with_vals(c4["vals"])
        C64 = B32.with_vals(c4["vals2"])
        a = torch.empty(1, dtype=torch.float64, device=dev)
        ms, ms_spread = _time_ops(lambda: spl.inner(B64, C64, a))
        res["inner_f64"] = _rate(ms, 16 * nnz, 2 * nnz, ms_spread)
        # the co-iteration of two patterns: the same coordinates in other
        # arrays, so every fiber is looked up and every position matched
        Cg = spl.CSF(c4["pos1"].clone(), c4["crd1"].clone(), c4["pos2"].clone(),
                     c4["crd2"].clone(), c4["vals2"], (I, J, Kd))
        ms, ms_spread = _time_ops(lambda: spl.inner(B64, Cg, a))
        res["inner_general_f64"] = _rate(
            ms, 2 * (4 * (I + 1) + 4 * F + 4 * (F + 1) + 12 * nnz), 2 * nnz, ms_spread)
        del B64, C64, Cg
    del B32, c4
    torch.cuda.empty_cache()


def measure_live_regret(dev, spl, tuning, torch, count=40, max_nnz=1e7):
    """The learned selectors against the exhaustive autotuner, measured in
    this run: the first `count` held-out matrices of the 2,000-matrix corpus
    (seeded; the training set never saw them) with at most `max_nnz`
    nonzeros; every candidate schedule timed (median of 5), the selector's
    choice from the matrix's features on the GPU.  Regret = t(choice) /
    t(fastest) - 1 per matrix, for the learned choice, the library default
    and the paper's fixed rule (SpMV row split, SpMM non-zero split; the
    best of that kind on these matrices)."""
    import numpy as np
    from paper_2207_13901_amd import learned
    from workloads import corpus
    _, test_ids = corpus.split(2000, 400)
    ids = [i for i in test_ids if corpus.spec(i)["nnz_target"] <= max_nnz][:count]
    sels = {}
    for op in ("spmv", "spmm"):
        path = os.path.join(learned.DATA_DIR, f"selector_{op}.json")
        if os.path.exists(path):
            sels[op] = learned.Selector.from_json(json.load(open(path)))
    if not sels:
        return None
    times = {op: [] for op in sels}
    chosen = {op: [] for op in sels}
    for i in ids:
        s, pos, crd, vals = corpus.generate(i, dev)
        n = s["n"]
        B = spl.CSR(pos, crd, vals, (n, n))
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty(n, dtype=torch.float32, device=dev)
        D = torch.ones(n, learned.SPMM_COLS, dtype=torch.float32, device=dev)
        A = torch.empty(n, learned.SPMM_COLS, dtype=torch.float32, device=dev)
        for op, sel in sels.items():
            call = (lambda sc: spl.spmv(B, x, y, sched=sc)) if op == "spmv" else \
                (lambda sc: spl.spmm(B, D, A, sched=sc))
            cands = learned.candidates(op)
            times[op].append([tuning.time_call(lambda c=c: call(spl.schedule(**c)), reps=5)
                              for c in cands])
            chosen[op].append(cands.index(sel.choose(B)))
        del B, pos, crd, vals, x, y, D, A
    torch.cuda.empty_cache()
    out = {"matrices": len(ids), "max_nnz": max_nnz,
           "families": {f: sum(1 for i in ids if corpus.spec(i)["family"] == f)
                        for f in corpus.FAMILIES}}
    for op in sels:
        T = np.asarray(times[op])
        cands = learned.candidates(op)
        default = cands.index(learned.LIBRARY_DEFAULT[op])
        kind = "row" if op == "spmv" else "nnz"
        rule = min((k for k, c in enumerate(cands) if c["kind"] == kind),
                   key=lambda k: float(np.mean(T[:, k] / T.min(1))))
        out[op] = {"learned": learned.regret(T, np.asarray(chosen[op])),
                   "library_default": learned.regret(T, np.full(len(T), default)),
                   "paper_rule": learned.regret(T, np.full(len(T), rule))}
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_openmp(oracle, pos, crd, c2, N, torch):
    """The CPU comparison of the whole step: double-precision SpMV and SpMM
    loops with OpenMP over rows (dynamic, 1,024 rows a chunk) on every core
    OpenMP is given, over the full matrix (FP64 values and operands); one
    warm-up, median of 5."""
    import numpy as np
    base = oracle.CpuBaseline()
    vals = np.ascontiguousarray(c2["vals"].cpu().numpy())
    x = np.ascontiguousarray(c2["x"].cpu().numpy())
    D = np.ascontiguousarray(c2["B"].cpu().numpy())
    n = len(pos) - 1
    y = np.empty(n)
    A = np.empty((n, N))
    times = []
    for rep in range(6):
        t0 = time.perf_counter()
        base.spmv(pos, crd, vals, x, y)
        base.spmm(pos, crd, vals, D, A)
        if rep:
            times.append(time.perf_counter() - t0)
    t = sorted(times)[len(times) // 2]
    nnz = int(pos[-1])
    return {"value": round((2.0 * nnz + 2.0 * nnz * N) / t / 1e9, 3), "unit": "GFLOP/s",
            "ms_per_step": round(1e3 * t, 2), "cores": base.threads(), "kind": "openmp_fp64",
            "cpu_model": cpu_model(),
            "sample": "the whole step (SpMV + SpMM N=32) over all rows, FP64, 1 warm-up, "
                      "median of 5"}


def precision_statement(dev, spl, torch, oracle, c2, B32, B16, D32, D16):
    """Error of each BF16 result (FP32 accumulation) against the oracle on
    (i) the BF16-rounded inputs and (ii) the original FP32 inputs, and of
    the FP32 form against the oracle on its inputs, on sampled output rows
    of the full workloads: SpMM on the power-law matrix, SDDMM (vector ALUs
    and matrix cores) on the 1,000,000-row matrix, SpMTTKRP on the CSF
    tensor.  Statistics: max and median |err| / S, ||err||_2 / ||ref||_2."""
    import numpy as np
    from workloads import configs

    def h64(t):
        return t.detach().to("cpu").to(torch.float64).numpy()

    def sample(pos, k, heavy, seed):
        deg = np.diff(pos)
        rs = np.random.RandomState(seed)
        return np.unique(np.concatenate([rs.choice(len(deg), k, replace=False),
                                         np.argsort(deg)[-heavy:], [0, len(deg) - 1]]))

    res = {}
    pos, crd = c2["pos"].cpu().numpy(), c2["crd"].cpu().numpy()
    rows = sample(pos, 400, 20, 1)
    rt = torch.as_tensor(rows, device=dev)
    ref32, S32 = oracle.spmm(pos, crd, h64(B32.vals), h64(D32), rows=rows)
    ref16, S16 = oracle.spmm(pos, crd, h64(B16.vals), h64(D16), rows=rows)
    got32 = h64(spl.spmm(B32, D32)[rt])
    got16 = h64(spl.spmm(B16, D16)[rt])
    res["spmm"] = {"fp32": oracle.error_statement(got32, ref32, S32),
                   "bf16_vs_bf16_inputs": oracle.error_statement(got16, ref16, S16),
                   "bf16_vs_fp32_inputs": oracle.error_statement(got16, ref32, S32),
                   "rows_sampled": int(rows.size)}

    c3 = configs.config3(device=dev)
    n = c3["n"]
    Bm = c3["B"]
    hpos, hcrd = Bm["pos"].cpu().numpy(), Bm["crd"].cpu().numpy()
    B = spl.CSR(Bm["pos"], Bm["crd"], Bm["vals"].to(torch.float32), (n, n))
    rows = sample(hpos, 3000, 20, 2)
    sub_pos = np.concatenate([[0], np.cumsum(np.diff(hpos)[rows])]).astype(np.int32)
    sel = np.concatenate([np.arange(hpos[r], hpos[r + 1]) for r in rows])
    rt = torch.as_tensor(rows, device=dev)
    C32, Dd32 = c3["Cd"].to(torch.float32), c3["Dd"].to(torch.float32)
    C16, Dd16 = C32.to(torch.bfloat16), Dd32.to(torch.bfloat16)
    bv = h64(B.vals)[sel]
    ref32, S32 = oracle.sddmm(sub_pos, hcrd[sel], bv, h64(C32[rt]), h64(Dd32))
    ref16, S16 = oracle.sddmm(sub_pos, hcrd[sel], bv, h64(C16[rt]), h64(Dd16))
    res["sddmm"] = {"fp32": oracle.error_statement(h64(spl.sddmm(B, C32, Dd32))[sel], ref32, S32),
                    "positions_sampled": int(sel.size)}
    for name, variant in (("bf16_valu", 0), ("bf16_mfma", 1)):
        got = h64(spl.sddmm(B, C16, Dd16, sched=spl.schedule(variant=variant)))[sel]
        res["sddmm"][name + "_vs_bf16_inputs"] = oracle.error_statement(got, ref16, S16)
        res["sddmm"][name + "_vs_fp32_inputs"] = oracle.error_statement(got, ref32, S32)
    del B, C32, Dd32, C16, Dd16, c3
    torch.cuda.empty_cache()

    c4 = configs.config4(device=dev)
    h = {k: c4[k].cpu().numpy() for k in ("pos1", "crd1", "pos2", "crd2")}
    I, J, Kd = c4["I"], c4["J"], c4["K"]
    v32 = c4["vals"].to(torch.float32)
    T32 = spl.CSF(c4["pos1"], c4["crd1"], c4["pos2"], c4["crd2"], v32, (I, J, Kd))
    T16 = T32.with_vals(v32.to(torch.bfloat16))
    F32, G32 = c4["C"].to(torch.float32), c4["D"].to(torch.float32)
    F16, G16 = F32.to(torch.bfloat16), G32.to(torch.bfloat16)
    rows = sample(h["pos1"], 200, 10, 3)
    rt = torch.as_tensor(rows, device=dev)
    ref32, S32 = oracle.mttkrp(h["pos1"], h["crd1"], h["pos2"], h["crd2"], h64(v32), h64(F32),
                               h64(G32), rows=rows)
    ref16, S16 = oracle.mttkrp(h["pos1"], h["crd1"], h["pos2"], h["crd2"], h64(T16.vals),
                               h64(F16), h64(G16), rows=rows)
    got32 = h64(spl.mttkrp(T32, F32, G32)[rt])
    got16 = h64(spl.mttkrp(T16, F16, G16)[rt])
    res["mttkrp"] = {"fp32": oracle.error_statement(got32, ref32, S32),
                     "bf16_vs_bf16_inputs": oracle.error_statement(got16, ref16, S16),
                     "bf16_vs_fp32_inputs": oracle.error_statement(got16, ref32, S32),
                     "slices_sampled": int(rows.size)}
    del T32, T16, F32, G32, F16, G16, c4
    torch.cuda.empty_cache()
    res["note"] = ("BF16 operands: SpMM vals and C; SDDMM C and D; MTTKRP vals, C and D; "
                   "round to nearest even from FP32; default schedules")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="shrink the workload (testing only; the headline uses 1.0)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-variants", action="store_true", help="skip variant measurements")
    ap.add_argument("--no-ops", action="store_true",
                    help="skip the SDDMM/SpAdd3/SpTTV/SpMTTKRP/inner-product measurements")
    ap.add_argument("--profile", action="store_true",
                    help="only the timed steps (for rocprofv3 runs)")
    ap.add_argument("--sched-spmv", type=str, default=None,
                    help="JSON schedule for SpMV instead of autotuning")
    ap.add_argument("--sched-spmm", type=str, default=None,
                    help="JSON schedule for SpMM instead of autotuning")
    ap.add_argument("--sched", action="append", default=[], metavar="OP=JSON",
                    help="fixed schedule for spttv or mttkrp (repeatable)")
    ap.add_argument("--no-next", action="store_true",
                    help="leave out the banded and (Dense, Dense, Compressed) workloads")
    ap.add_argument("--ops-only", action="store_true",
                    help="only the SDDMM/SpAdd3/SpTTV/SpMTTKRP/inner-product measurements")
    ap.add_argument("--only", type=str, default=None,
                    help="with --ops-only: comma-separated subset of " + ",".join(OPS))
    ap.add_argument("--calibrate", action="store_true",
                    help="run a 1 GiB device copy first (counter scale reference)")
    ap.add_argument("--no-cold", action="store_true",
                    help="time the other leaves back to back only, without the MALL-flushed "
                         "trials (for rocprofv3 runs whose kernel averages are the warm ones)")
    args = ap.parse_args()
    _COLD[0] = not args.no_cold
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2207_13901_amd as spl
    from paper_2207_13901_amd import tuning
    from paper_2207_13901_amd import _native as N
    from workloads import configs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.calibrate:
        # plain copy of 1 GiB: 1 GiB read + 1 GiB written per dispatch
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    fixed = {}
    for item in args.sched:
        op, js = item.split("=", 1)
        fixed[op] = json.loads(js)
    if args.ops_only:
        only = args.only.split(",") if args.only else None
        if only and not set(only) <= set(OPS):
            ap.error(f"--only takes names from {','.join(OPS)}")
        print(json.dumps({"ops": measure_other_ops(dev, spl, tuning, torch, fixed,
                                                   not args.no_next, only)}),
              flush=True)
        return
    t0 = time.time()
    c2 = configs.config2(device=dev, scale=args.scale, N=N_COLS)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    n = c2["n"]
    nnz = int(c2["crd"].numel())
    print(f"[bench] generated n={n} nnz={nnz} in {gen_s:.1f}s", file=sys.stderr, flush=True)

    def csr(dtype):
        return spl.CSR(c2["pos"], c2["crd"], c2["vals"].to(dtype), (n, n))

    B32, B64, B16 = csr(torch.float32), csr(torch.float64), csr(torch.bfloat16)
    x32, x64 = c2["x"].to(torch.float32), c2["x"]
    D32, D64, D16 = c2["B"].to(torch.float32), c2["B"], c2["B"].to(torch.float32).to(torch.bfloat16)
    y32, y64 = torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float64, device=dev)
    A32 = torch.empty(n, N_COLS, dtype=torch.float32, device=dev)
    A64 = torch.empty(n, N_COLS, dtype=torch.float64, device=dev)

    # -- exhaustive schedule search (untimed) ---------------------------------
    reps = 3 if args.profile else 5
    if args.sched_spmv:
        best_v, res_v = json.loads(args.sched_spmv), []
    else:
        best_v, res_v = tuning.search(lambda s: (lambda: spl.spmv(B32, x32, y32, sched=s)),
                                        tuning.SPMV_CANDIDATES, reps=reps)
    if args.sched_spmm:
        best_m, res_m = json.loads(args.sched_spmm), []
    else:
        best_m, res_m = tuning.search(lambda s: (lambda: spl.spmm(B32, D32, A32, sched=s)),
                                        tuning.SPMM_CANDIDATES, reps=reps)
    sv, sm = spl.schedule(**best_v), spl.schedule(**best_m)
    ws_v = spl.workspace(N.OP_SPMV, B32, 1, sv)
    ws_m = spl.workspace(N.OP_SPMM, B32, N_COLS, sm)
    print(f"[bench] schedules spmv={best_v} spmm={best_m}", file=sys.stderr, flush=True)

    # the learned selector's choice for this matrix (features and network on
    # the GPU), timed against the exhaustive autotuner's choice
    learned_out = None
    if not args.profile and res_v and res_m:
        from paper_2207_13901_amd import learned
        learned_out = {}
        for op, best, res, call in (
                ("spmv", best_v, res_v, lambda s: spl.spmv(B32, x32, y32, sched=s)),
                ("spmm", best_m, res_m, lambda s: spl.spmm(B32, D32, A32, sched=s))):
            path = os.path.join(learned.DATA_DIR, f"selector_{op}.json")
            if not os.path.exists(path):
                continue
            sel = learned.Selector.from_json(json.load(open(path)))
            choice = sel.choose(B32)
            sc = spl.schedule(**choice)
            t_learned = tuning.time_call(lambda: call(sc), reps=10, warmup=3)
            t_best = tuning.time_call(lambda: call(spl.schedule(**best)), reps=10, warmup=3)
            learned_out[op] = {"learned_choice": choice, "autotuned_choice": best,
                               "learned_ms": round(t_learned, 5), "autotuned_ms": round(t_best, 5),
                               "regret": round(t_learned / t_best - 1.0, 4)}
        print("[bench] live held-out regret", file=sys.stderr, flush=True)
        learned_out["held_out_live"] = measure_live_regret(dev, spl, tuning, torch)
        regret_path = os.path.join(learned.DATA_DIR, "regret.json")
        if os.path.exists(regret_path):
            rep = json.load(open(regret_path))
            learned_out["held_out_corpus"] = {
                op: {"learned_mean_regret": round(rep[op]["learned"]["mean"], 4),
                     "library_default_mean_regret": round(rep[op]["library_default"]["mean"], 4),
                     "best_fixed_mean_regret": round(rep[op]["best_fixed_on_train"]["mean"], 4),
                     "paper_rule_mean_regret": round(rep[op]["paper_rule"]["mean"], 4),
                     "matrices": rep[op]["held_out_matrices"]} for op in ("spmv", "spmm")}

    def step():
        spl.spmv(B32, x32, y32, sched=sv, ws=ws_v)
        spl.spmm(B32, D32, A32, sched=sm, ws=ws_m)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    spl.timing_read(N.OP_SPMV)
    spl.timing_read(N.OP_SPMM)
    spl.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    spl.timing_enable(False)
    lv, msv = spl.timing_read(N.OP_SPMV)
    lm, msm = spl.timing_read(N.OP_SPMM)
    ms_per_step = 1e3 * elapsed / args.steps
    flops = 2.0 * nnz + 2.0 * nnz * N_COLS
    gflops = flops / (ms_per_step * 1e-3) / 1e9

    # the same step in FP64 (the only precision the paper's example states),
    # with its own autotuned schedules, under the same protocol
    fp64_step = None
    if not args.profile and not args.no_variants:
        bv, _ = tuning.search(lambda s: (lambda: spl.spmv(B64, x64, y64, sched=s)),
                              tuning.SPMV_CANDIDATES, reps=reps)
        bm, _ = tuning.search(lambda s: (lambda: spl.spmm(B64, D64, A64, sched=s)),
                              tuning.SPMM_CANDIDATES, reps=reps)
        sv64, sm64 = spl.schedule(**bv), spl.schedule(**bm)
        wv64 = spl.workspace(N.OP_SPMV, B64, 1, sv64)
        wm64 = spl.workspace(N.OP_SPMM, B64, N_COLS, sm64)

        def step64():
            spl.spmv(B64, x64, y64, sched=sv64, ws=wv64)
            spl.spmm(B64, D64, A64, sched=sm64, ws=wm64)

        for _ in range(args.warmup):
            step64()
        torch.cuda.synchronize()
        t64 = time.perf_counter()
        for _ in range(args.steps):
            step64()
        torch.cuda.synchronize()
        ms64 = 1e3 * (time.perf_counter() - t64) / args.steps
        fp64_step = {"ms_per_step": round(ms64, 4),
                     "GFLOP_s": round((2.0 * nnz + 2.0 * nnz * N_COLS) / (ms64 * 1e-3) / 1e9, 2),
                     "schedule_spmv": bv, "schedule_spmm": bm,
                     "protocol": f"{args.warmup} warm-up then {args.steps} timed steps"}
        del wv64, wm64

    # per-launch spread of the two leaf kernels (untimed loop after the
    # timed steps, one read-back per step), warm and with the 256 MB MALL
    # flushed by a 1 GiB write before each step
    spread = {}
    if not args.profile:
        flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        for mode in ("warm", "cold"):
            per = {"spmv": [], "spmm": []}
            for _ in range(10):
                if mode == "cold":
                    flush.fill_(1.0)
                torch.cuda.synchronize()
                spl.timing_enable(True)
                step()
                spl.timing_enable(False)
                per["spmv"].append(spl.timing_read(N.OP_SPMV)[1])
                per["spmm"].append(spl.timing_read(N.OP_SPMM)[1])
            for op, v in per.items():
                v = sorted(v)
                spread.setdefault(op, {})[mode] = {"min_ms": round(v[0], 5),
                                                   "median_ms": round(v[len(v) // 2], 5),
                                                   "max_ms": round(v[-1], 5)}
        del flush

    bytes_v32, bytes_m32 = algorithmic_bytes(n, n, nnz, N_COLS, 4, 4, 4)
    spmm_ms = msm / max(lm, 1)
    spmv_ms = msv / max(lv, 1)
    achieved = bytes_m32 / (spmm_ms * 1e-3) / 1e9
    out = {
        "metric": "GFLOP/s + % HBM roofline (SpMV/SpMM/MTTKRP); BF16 & learned vs FP32 autotuned",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("CSR 2,000,000 x 2,000,000 power-law rows (Pareto alpha=2, "
                         "32,000,000 nnz, cap 50,000), SpMV + SpMM with N=32, FP32, "
                         "autotuned schedules") if args.scale == 1.0 else
                        f"scaled power-law CSR n={n} nnz={nnz}",
            "n": n, "nnz": nnz, "N": N_COLS,
            "schedule_spmv": best_v, "schedule_spmm": best_m,
        },
        "roofline": {
            "kernel": f"SpMM leaf ({spmm_kernel_name(best_m)}), FP32",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": counted_traffic(best_m),
            "algorithmic_bytes_per_launch": bytes_m32,
            "avg_launch_ms": round(spmm_ms, 5),
            "launches": lm,
        },
        "fp64_step": fp64_step,
        "kernels": {
            "spmv_f32": {"avg_ms": round(spmv_ms, 5), "launches": lv,
                         "GB_s": round(bytes_v32 / (spmv_ms * 1e-3) / 1e9, 1),
                         "frac_hbm": round(bytes_v32 / (spmv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "GFLOP_s": round(2 * nnz / (spmv_ms * 1e-3) / 1e9, 2)},
            "spmm_f32": {"avg_ms": round(spmm_ms, 5), "launches": lm,
                         "GB_s": round(achieved, 1),
                         "frac_hbm": round(achieved / HBM_PEAK_GBS, 4),
                         "GFLOP_s": round(2 * nnz * N_COLS / (spmm_ms * 1e-3) / 1e9, 2)},
        },
        "leaf_spread": spread,
        "autotune": {
            "spmv_ms": {json.dumps(c, sort_keys=True): round(t, 4) for c, t in res_v},
            "spmm_ms": {json.dumps(c, sort_keys=True): round(t, 4) for c, t in res_m},
        },
    }

    if spread:
        # the same kernel with the 256 MB MALL flushed before each launch
        cold = spread["spmm"]["cold"]["median_ms"]
        ach = bytes_m32 / (cold * 1e-3) / 1e9
        out["roofline"]["mall_flushed"] = {"median_launch_ms": cold, "achieved": round(ach, 1),
                                           "frac": round(ach / HBM_PEAK_GBS, 4)}

    if learned_out is not None:
        out["learned"] = learned_out

    if not args.profile and not args.no_variants and res_v and res_m:
        var = {}
        bv64, bm64 = algorithmic_bytes(n, n, nnz, N_COLS, 8, 8, 8)
        _, bm16 = algorithmic_bytes(n, n, nnz, N_COLS, 2, 2, 4)
        # BF16 values and dense rows (FP32 accumulation and output) with
        # their own autotuned schedule
        best16, res16 = tuning.search(lambda s: (lambda: spl.spmm(B16, D16, A32, sched=s)),
                                      tuning.SPMM_BF16_CANDIDATES, reps=reps)
        sm16 = spl.schedule(**best16)
        for name, fn, nbytes, fl in (
            ("spmv_f64", lambda: spl.spmv(B64, x64, y64, sched=sv), bv64, 2 * nnz),
            ("spmm_f64", lambda: spl.spmm(B64, D64, A64, sched=sm), bm64, 2 * nnz * N_COLS),
            ("spmm_bf16_f32acc", lambda: spl.spmm(B16, D16, A32, sched=sm16), bm16,
             2 * nnz * N_COLS),
        ):
            ms = tuning.time_call(fn, reps=10, warmup=3)
            var[name] = {"ms": round(ms, 5), "GFLOP_s": round(fl / (ms * 1e-3) / 1e9, 2),
                         "GB_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                         "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        # wide columns (N = 128): the dense operand that an MFMA form of SpMM
        # would contract; timed on the vector-lane leaf
        D128 = torch.empty(n, 128, dtype=torch.float32, device=dev).uniform_(-1, 1)
        A128 = torch.empty(n, 128, dtype=torch.float32, device=dev)
        ms = tuning.time_call(lambda: spl.spmm(B32, D128, A128), reps=10, warmup=3)
        _, b128 = algorithmic_bytes(n, n, nnz, 128, 4, 4, 4)
        var["spmm_f32_N128"] = {"ms": round(ms, 5),
                                "GFLOP_s": round(2 * nnz * 128 / (ms * 1e-3) / 1e9, 2),
                                "GB_s": round(b128 / (ms * 1e-3) / 1e9, 1),
                                "frac_hbm": round(b128 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                "gathered_row_GB_s": round(nnz * 512 / (ms * 1e-3) / 1e9, 1)}
        del D128, A128
        var["spmm_bf16_f32acc"]["schedule"] = best16
        var["spmm_bf16_f32acc"]["schedules_ms"] = {json.dumps(c, sort_keys=True): round(t, 4)
                                                   for c, t in res16}
        var["spmm_bf16_f32acc"]["vs_fp32_autotuned"] = round(
            min(t for _, t in res_m) / var["spmm_bf16_f32acc"]["ms"], 3)
        # the paper's fixed rules: SpMV row split, SpMM non-zero split
        rule_v = min((t for c, t in res_v if c["kind"] == "row"))
        rule_m = min((t for c, t in res_m if c["kind"] == "nnz"))
        var["fixed_rules_vs_autotuned"] = {
            "spmv_row_best_ms": round(rule_v, 5), "spmm_nnz_best_ms": round(rule_m, 5),
            "spmv_autotuned_ms": round(min(t for _, t in res_v), 5),
            "spmm_autotuned_ms": round(min(t for _, t in res_m), 5)}
        out["variants"] = var

    if not args.profile and not args.no_variants:
        # memory-system ceilings the leaves run against
        big = torch.ones(1 << 29, dtype=torch.float32, device=dev)  # 2 GiB
        ms = tuning.time_call(lambda: spl.probe(0, big), reps=5, warmup=2)
        ceil = {"stream_read_GB_s": round(big.numel() * 4 / (ms * 1e-3) / 1e9, 1)}
        # nnz random row reads, the gather pattern of one SpMV / SpMM call,
        # from tables of growing size (L2 = 4 MB per XCD, MALL = 256 MB)
        for row_bytes, mbs in ((4, (2, 8, 64)), (8, (16,)), (128, (8, 64, 128, 256, 1024)),
                               (256, (512,))):
            for mb in mbs:
                table = big[: mb * (1 << 18)]
                ms = tuning.time_call(
                    lambda: spl.probe(1, table, row_bytes=row_bytes, count=nnz), reps=5, warmup=2)
                ceil[f"gather_{row_bytes}B_rows_from_{mb}MB"] = {
                    "ms_per_nnz_gathers": round(ms, 5),
                    "Grows_per_s": round(nnz / (ms * 1e-3) / 1e9, 2)}
        # the same gathers with 16-byte lanes (a quarter of the load instructions)
        for row_bytes, mb in ((64, 128), (128, 256)):
            table = big[: mb * (1 << 18)]
            ms = tuning.time_call(
                lambda: spl.probe(2, table, row_bytes=row_bytes, count=nnz), reps=5, warmup=2)
            ceil[f"gather_{row_bytes}B_rows_16B_lanes_from_{mb}MB"] = {
                "ms_per_nnz_gathers": round(ms, 5),
                "Grows_per_s": round(nnz / (ms * 1e-3) / 1e9, 2)}
        del big
        out["ceilings"] = ceil

    if not args.profile and not args.no_ops:
        del B64, B16, D64, D16, A64
        torch.cuda.empty_cache()
        out["ops"] = measure_other_ops(dev, spl, tuning, torch, fixed, not args.no_next)

    if not args.profile and not args.no_cpu:
        import oracle
        pos = c2["pos"].cpu().numpy()
        crd = c2["crd"].cpu().numpy()
        vals = c2["vals"].to(torch.float32).to(torch.float64).cpu().numpy()
        xh = x32.to(torch.float64).cpu().numpy()
        Dh = D32.to(torch.float64).cpu().numpy()
        # sample: every row for SpMV, a contiguous row block for SpMM sized
        # to about a quarter of the nonzeros
        rows_m = int(np.searchsorted(pos, nnz // 4))
        t1 = time.perf_counter()
        oracle.spmv(pos, crd, vals, xh)
        t2 = time.perf_counter()
        oracle.spmm(pos[:rows_m + 1], crd[:pos[rows_m]], vals[:pos[rows_m]], Dh)
        t3 = time.perf_counter()
        flops_sample = 2.0 * nnz + 2.0 * int(pos[rows_m]) * N_COLS
        out["cpu_baseline"] = {
            "value": round(flops_sample / (t3 - t1) / 1e9, 4),
            "unit": "GFLOP/s",
            "cores": 1,
            "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"SpMV over all {n} rows ({nnz} nnz, {t2 - t1:.2f}s) + SpMM N=32 over "
                       f"rows 0..{rows_m} ({int(pos[rows_m])} nnz, {t3 - t2:.2f}s); "
                       "single-threaded long-double C loops"),
        }
        out["cpu_openmp_fp64"] = cpu_openmp(oracle, pos, crd, c2, N_COLS, torch)
        print("[bench] precision statement", file=sys.stderr, flush=True)
        out["precision"] = precision_statement(dev, spl, torch, oracle, c2, B32,
                                               csr(torch.bfloat16), D32,
                                               D32.to(torch.bfloat16))
    if args.profile:
        out["sources_digest"] = sources_digest(SPMM_SOURCES)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
