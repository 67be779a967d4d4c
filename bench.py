"""Benchmark of the near-field P2P operator on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: 2M points uniform on the unit sphere, leaf boxes sized for ~32 points
per non-empty box, k = 2 pi * 64, complex64 strengths ~ N(0,1), one right-hand
side (seeded, synthetic).  One step is one pass of the whole path on that input,
already resident in HBM: the plan build with the leaf-box ids computed from the
positions inside it (Morton keys, sort, box table, neighbour lists; replicated
source lists for the tiles layout), the FP32 apply y = A_near q, and the plan's
release.  The step uses the
non-redundant CSR layout unless --layout tiles is given; the other layout is
timed beside it.

Printed: one JSON line.  value = near-field interactions (ordered pairs with
r != 0) per second of the whole step.  Besides it: the apply alone, the FP64 path
and the non-redundant layout on the same input, the relative L2 error of the
FP32 and FP64 results against the FP64 oracle, the roofline of the dominant
kernel (the FP32 sweep) and the oracle's own rate on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU issue model of the MI355X, in issue slots of 128 FP32 lanes per clock per
# CU (the published 157.3 TFLOP/s FP32 vector rate at 256 CUs and 2.4 GHz; plain,
# unpacked v_fma_f32 reaches it, measured by the issue-rate microbenchmark at
# about 100 lanes per clock per CU counted at 2.4 GHz).  Measured costs, in such
# slots: FP32 FMA, multiply, add and integer operations 1, conversions 2,
# transcendentals 4 (quarter rate), and a transcendental does not issue beside
# the other VALU work: the microbenchmark's pair stream (15 FMAs, rsq, sin, cos)
# takes the sum of its parts' times.
CUS, LANES_PER_CLK, CLOCK_HZ = 256, 128, 2.4e9
PEAK_SLOTS = CUS * LANES_PER_CLK * CLOCK_HZ            # 7.86e13 issue slots / s

# Algorithmic work per pair of the FP32 Helmholtz sweep: 3 coordinate differences,
# 3 operations for r^2, r = r^2 / r, the phase in turns and its range reduction
# (2), G = (cos, sin) / r (2) and the complex multiply-add (4): 15 VALU operations,
# plus the transcendentals rsq, sin and cos at 4 slots each: 27 slots per pair.
SLOTS_PER_PAIR = 15 + 4 * 3
PEAK_GPAIRS = PEAK_SLOTS / SLOTS_PER_PAIR / 1e9        # 2913 Gpair/s
ISSUE_LIB = os.path.join(ROOT, "paper_2403_01596_amd", "libp2p_issue.so")
ISSUE_MIXES = ["fma", "trans", "pair", "issued", "int", "cvt"]

# Reverse pass (dq and dx together, FP32 Helmholtz), per pair: the geometry above
# (3 differences, 3 for r^2, r, phase and reduction: 9 VALU + rsq, sin, cos), G =
# (c + is)/r (2), dq's conj(G) g (4), u = conj(g_i) q_j + conj(g_j) q_i (8), the two
# parts of (c + is)(ik - 1/r) (2), Re(G' u) (2), 1/r^2 and its product (2) and the
# three dx multiply-adds (3): 32 VALU operations plus 3 transcendentals = 44 slots.
BWD_SLOTS_PER_PAIR = 32 + 4 * 3
PEAK_BWD_GPAIRS = PEAK_SLOTS / BWD_SLOTS_PER_PAIR / 1e9   # 1787 Gpair/s

# FP64 sweep, per pair: 3 differences, 3 for r^2, the 1/r refinement (5), r and the
# phase in turns (2), the half-turn reduction (3), x^2, x^4, x^8 (3), the sine and
# cosine polynomials (20) and the sine's factor x (1), the sign of an odd half
# turn (4) and its application (2), G (2) and the complex multiply-add (4): 52 FP64
# VALU operations at 64 lanes per clock per CU (the published 78.6 TFLOP/s FP64
# vector rate: 2 of the slots above each) plus v_rsq_f64 at a quarter of that (8):
# 112 slots.
F64_SLOTS_PER_PAIR = 2 * 52 + 8
PEAK_F64_GPAIRS = PEAK_SLOTS / F64_SLOTS_PER_PAIR / 1e9   # 702 Gpair/s

# Multi-RHS product: one complex multiply-add per (pair, right-hand side) = 8 real
# flops on the FP32 matrix cores (dense FP32 MFMA peak 157.3 TFLOP/s).
FLOPS_PER_PAIR_RHS = 8
PEAK_MFMA_F32 = 157.3e12

# Untimed steps run for this long before the warm-up steps: the GPU leaves idle on
# a lower clock and takes tens of milliseconds to reach its steady one.
SPIN_UP_S = 0.25

COUNTERS_FILE = os.path.join(ROOT, "profiles", "sweep_f32_csr_sphere2M_counters.md")
VALU_COUNTERS_FILE = os.path.join(ROOT, "profiles", "sweep_f32_csr_sphere2M_valu_counters.md")
KERNEL_SOURCES = ["paper_2403_01596_amd/csrc/sweep.h", "paper_2403_01596_amd/csrc/apply.hip",
                  "paper_2403_01596_amd/csrc/common.h"]
MRHS_COUNTERS_FILE = os.path.join(ROOT, "profiles", "mrhs_f32_csr_batch17_counters.md")
MRHS_SOURCES = ["paper_2403_01596_amd/csrc/mrhs.hip", "paper_2403_01596_amd/csrc/mrhs.h",
                "paper_2403_01596_amd/csrc/sweep.h", "paper_2403_01596_amd/csrc/common.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def single_core_oracle(W, oracle):
    """The oracle on one thread: the 8192-point cube (every row) and a bounded
    sample of rows of the 500k-point cube."""
    out = {}
    c1 = W.plain_f64_cube()
    orc = oracle.Plan(c1.ids)
    pairs = orc.stats(c1.xyz)["n_pairs"]
    t0 = time.perf_counter()
    orc.apply(c1.xyz, c1.k, c1.q, threads=1)
    out["cube8192_g8"] = {"gpairs_s": round(pairs / (time.perf_counter() - t0) / 1e9, 5), "rows": c1.n,
                          "pairs": pairs}
    c5 = W.grad_cube_500k()
    orc = oracle.Plan(c5.ids)
    rows = np.arange(0, c5.n, 50)
    tb = orc.tables()
    sizes = np.diff(tb["box_start"]).astype(np.int64)
    nsrc = np.array([sizes[tb["nbr_idx"][tb["nbr_start"][T]:tb["nbr_start"][T + 1]]].sum()
                     for T in range(sizes.size)])
    pos = np.empty(c5.n, np.int64)
    pos[tb["perm"]] = np.arange(c5.n)
    box = np.searchsorted(tb["box_start"], pos[rows], side="right") - 1
    pairs = int(nsrc[box].sum() - rows.size)  # distinct points: each row skips its self pair
    t0 = time.perf_counter()
    orc.apply_rows(c5.xyz, c5.k, c5.q, rows, threads=1)
    out["cube500k_g25_every_50th_row"] = {"gpairs_s": round(pairs / (time.perf_counter() - t0) / 1e9, 5),
                                          "rows": int(rows.size), "pairs": pairs}
    return out


def spin_up(fn, torch):
    """Untimed calls of fn for SPIN_UP_S seconds: after an idle spell (plan builds,
    host work) the clock takes tens of milliseconds to climb back to its steady
    value, and a short timed loop would otherwise run on that ramp."""
    end = time.perf_counter() + SPIN_UP_S
    while time.perf_counter() < end:
        fn()
        torch.cuda.synchronize()


def kernel_source_digest(sources=None) -> str:
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_value(path, key, sources=None):
    """A figure (`key: value`) from a committed counter summary, if the summary was
    taken on the current kernel sources (else None)."""
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    b = re.search(key + r":\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != kernel_source_digest(sources):
        return None
    return float(b.group(1))


def stored_traffic(path=None, sources=None):
    """HBM bytes per launch of a kernel from its committed counter summary, if the
    summary was taken on the current kernel sources (else None)."""
    try:
        text = open(path or COUNTERS_FILE).read()
    except OSError:
        return None
    m = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != kernel_source_digest(sources):
        return None
    return float(b.group(1))


def measure_issue_rates(torch, iters=4000, blocks=8 * CUS):
    """VALU issue rates of six instruction mixes (libp2p_issue.so): FMA, the three
    transcendentals, the FP32 sweep's algorithmic stream per pair (15 FMAs + rsq,
    sin, cos), the mix the sweep issues per pair (its counters), integer
    subtractions and conversions; 8 workgroups of 4 wavefronts per CU, every chain
    independent.  Per mix: lane-operations per second, the lanes per clock per CU
    that rate means at the published 2.4 GHz (a lower bound of the per-clock rate,
    since the clock runs at most that fast), and the mix's time per operation in
    FMA issue slots (FMA mix = 1)."""
    import ctypes
    L = ctypes.CDLL(ISSUE_LIB)
    L.p2p_issue_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_float)]
    L.p2p_issue_counts.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    lanes = blocks * 256.0 * iters  # loop trips of all lanes
    out = {}
    ms = ctypes.c_float()
    fma_slot_ms = None
    for mix, name in enumerate(ISSUE_MIXES):
        valu, trans = ctypes.c_int(), ctypes.c_int()
        L.p2p_issue_counts(mix, ctypes.byref(valu), ctypes.byref(trans))
        end = time.perf_counter() + SPIN_UP_S  # the clock out of idle first
        while time.perf_counter() < end:
            rc = L.p2p_issue_run(mix, blocks, iters, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError("issue-rate kernel %s failed (%d)" % (name, rc))
        times = []
        for _ in range(5):
            rc = L.p2p_issue_run(mix, blocks, iters, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError("issue-rate kernel %s failed (%d)" % (name, rc))
            times.append(ms.value)
        t_ms = min(times)
        ops = lanes * valu.value
        if fma_slot_ms is None:
            fma_slot_ms = t_ms / valu.value  # the FMA mix comes first: its time per FMA per lane-trip
        r = {"valu_per_trip": valu.value, "trans_per_trip": trans.value, "ms": round(t_ms, 4),
             "lane_ops_per_s": float("%.4g" % (ops / (t_ms * 1e-3))),
             "lanes_per_clk_cu_at_2_4ghz": round(ops / (t_ms * 1e-3) / CUS / CLOCK_HZ, 2),
             "fma_slots_per_trip": round(t_ms / fma_slot_ms, 2)}
        if name == "pair":
            r["gpairs_s"] = round(lanes / (t_ms * 1e-3) / 1e9, 1)
        out[name] = r
        log("issue %-6s %2d VALU/trip (%2d transcendental): %.3f ms, %6.2f lanes/clk/CU at 2.4 GHz, "
            "%5.2f FMA slots per trip" % (name, valu.value, trans.value, t_ms, r["lanes_per_clk_cu_at_2_4ghz"],
                                          r["fma_slots_per_trip"]))
    return out


def measure_mrhs(p2p, W, torch, reps, with_oracle):
    """1M sphere points at ~32 per box (k = 2 pi 32) plus 16 uneven sphere instances of
    10k..200k points, 64 complex64 right-hand sides each, all in one captured launch."""
    m = 64
    insts = [W.multi_rhs_main(m)] + W.multi_rhs_batch(m)
    log("multi-RHS batch: %d instances, %d points" % (len(insts), sum(i.n for i in insts)))
    plans, qs = [], []
    for inst in insts:
        xyz = torch.from_numpy(inst.xyz).cuda()
        ids = torch.from_numpy(inst.ids).cuda()
        plans.append(p2p.Plan(xyz, ids, inst.k, dtype=torch.complex64, layout="csr", max_rhs=m))
        qs.append(torch.from_numpy(inst.q).cuda())
    ys = [torch.empty_like(q) for q in qs]
    batch = p2p.Batch(plans, m)
    shape = batch.tune(qs, ys)
    n_pairs = sum(pl.info()["n_pairs"] for pl in plans)
    for _ in range(5):  # untimed: the clock ramps up over the first calls after a pause
        batch.apply_into(qs, ys)
    torch.cuda.synchronize()
    # kernel time: events around the product kernel (eager calls)
    batch.timing(True)
    for _ in range(reps):
        batch.apply_into(qs, ys)
    torch.cuda.synchronize()
    kern_ms, calls = batch.timing_read()
    batch.timing(False)
    kern_ms /= calls
    # one captured launch (gather + product), replayed
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.apply_into(qs, ys)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        batch.apply_into(qs, ys)
    for _ in range(5):  # untimed, as for the eager calls
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / reps
    out = {"workload": "sphere1M_D32_k64pi + 16 uneven sphere instances (10k..200k), 64 complex64 RHS",
           "instances": len(insts), "points": sum(i.n for i in insts), "rhs": m, "n_pairs": n_pairs,
           "launch_shape": {"rhs_per_item": shape[0], "waves_per_block": shape[1]},
           "graph_ms": round(graph_ms, 4), "kernel_ms": round(kern_ms, 4),
           "pair_rhs_per_s": round(n_pairs * m / (graph_ms * 1e-3), 1),
           "roofline": {"bound": "mfma", "achieved": round(FLOPS_PER_PAIR_RHS * n_pairs * m / (kern_ms * 1e-3) / 1e12, 2),
                        "peak": PEAK_MFMA_F32 / 1e12, "unit": "TFLOP/s",
                        "frac": round(FLOPS_PER_PAIR_RHS * n_pairs * m / (kern_ms * 1e-3) / PEAK_MFMA_F32, 4),
                        "traffic": stored_traffic(MRHS_COUNTERS_FILE, MRHS_SOURCES),
                        "kernel": "k_mrhs (FP32 MFMA 16x16x4, CSR)"}}
    if with_oracle:
        import oracle
        from scipy.spatial import cKDTree
        per = []
        for j, (inst, y) in enumerate(zip(insts, ys)):
            got = y.cpu().numpy()
            if j == 0:  # the 1M instance: every row
                ref = oracle.Plan(inst.ids).apply(inst.xyz, inst.k, inst.q)
                out["rel_err_main_all_rows"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
                continue
            # the small instances: 400 random rows plus the rows of the 20 closest pairs
            dist, nb = cKDTree(inst.xyz).query(inst.xyz, k=2)
            close = np.argsort(dist[:, 1])[:20]
            rows = np.unique(np.concatenate([np.random.default_rng(1).choice(inst.n, min(inst.n, 400), replace=False),
                                             close, nb[close, 1]]))
            ref = oracle.Plan(inst.ids).apply_rows(inst.xyz, inst.k, inst.q, rows)
            per.append(float(np.linalg.norm(got[rows] - ref) / np.linalg.norm(ref)))
        out["rel_err_small_instances_max"] = max(per)
        out["rel_err_small_instances_sample"] = "400 random rows + the rows of the 20 closest pairs, per instance"
    log("multi-RHS: graph %.3f ms, kernel %.3f ms, %.3g pair-RHS/s, %.1f%% of FP32 MFMA peak" % (
        graph_ms, kern_ms, out["pair_rhs_per_s"], 100 * out["roofline"]["frac"]))
    batch.close()
    for pl in plans:
        pl.close()
    return out


def measure_backward(p2p, W, torch, reps, with_oracle):
    """Reverse pass (dq and dx in one sweep) on 500k uniform points in a 25^3 grid,
    k = 2 pi * 16, FP32 and FP64, CSR layout; sweep kernel time from the library's
    events; relative L2 errors of dq and dx over every row against the oracle's
    reverse pass."""
    inst = W.grad_cube_500k()
    xyz = torch.from_numpy(inst.xyz).cuda()
    ids = torch.from_numpy(inst.ids).cuda()
    g64 = W.strengths(inst.n, 1, np.random.default_rng(5), np.complex128)
    out = {"workload": "cube500k_g25 (500k uniform points, 25^3 boxes, k = 2 pi 16), dq and dx"}
    orc = None
    if with_oracle:
        import oracle
        orc = oracle.Plan(inst.ids)
    for dt, name in ((torch.complex64, "f32"), (torch.complex128, "f64")):
        npd = np.complex64 if name == "f32" else np.complex128
        q = torch.from_numpy(inst.q.astype(npd)).cuda()
        g = torch.from_numpy(g64.astype(npd)).cuda()
        plan = p2p.Plan(xyz, ids, inst.k, dtype=dt, layout="csr")
        n_pairs = plan.info()["n_pairs"]
        dq, dx = plan.backward(q, g)
        errs = None
        if orc is not None:
            dq_ref, dx_ref = orc.backward(inst.xyz, inst.k, inst.q.astype(npd), g64.astype(npd))
            errs = {"dq": float(np.linalg.norm(dq.cpu().numpy() - dq_ref) / np.linalg.norm(dq_ref)),
                    "dx": float(np.linalg.norm(dx.cpu().numpy() - dx_ref) / np.linalg.norm(dx_ref))}
        spin_up(lambda: plan.backward(q, g), torch)
        plan.timing(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.backward(q, g)
        e1.record()
        torch.cuda.synchronize()
        kern_ms, calls = plan.timing_read()
        plan.timing(False)
        kern_ms /= calls
        call_ms = e0.elapsed_time(e1) / reps
        out[name] = {"n_pairs": n_pairs, "call_ms": round(call_ms, 4), "kernel_ms": round(kern_ms, 4),
                     "gpairs_s": round(n_pairs / kern_ms / 1e6, 2), "rel_err": errs}
        plan.close()
    out["roofline_f32"] = {"bound": "alu", "achieved": out["f32"]["gpairs_s"], "peak": round(PEAK_BWD_GPAIRS, 1),
                           "unit": "Gpair/s", "frac": round(out["f32"]["gpairs_s"] / PEAK_BWD_GPAIRS, 4),
                           "work_per_pair": "32 VALU + 3 transcendental (4 slots each) = %d issue slots"
                                            % BWD_SLOTS_PER_PAIR}
    log("backward: f32 %.3f ms (%.1f Gpair/s, %.1f%% of its ALU roofline), f64 %.3f ms" % (
        out["f32"]["kernel_ms"], out["f32"]["gpairs_s"], 100 * out["roofline_f32"]["frac"], out["f64"]["kernel_ms"]))
    return out


def measure_layouts(p2p, W, torch, reps, with_oracle):
    """The two source layouts on 4M points of the (1, 0.5, 0.25) ellipsoid at 16, 32
    and 64 points per box (k = pi / (2h)), FP32: plan build and sweep kernel, and the
    relative L2 error of every output row against the oracle."""
    out = {"workload": "ellipsoid4M at D = 16, 32, 64, k = pi / (2h), FP32"}
    for d in (16, 32, 64):
        inst = W.ellipsoid_4m(d)
        xyz = torch.from_numpy(inst.xyz).cuda()
        ids = torch.from_numpy(inst.ids).cuda()
        q = torch.from_numpy(inst.q[:, 0].copy()).cuda()
        ref = None
        if with_oracle:
            import oracle
            ref = oracle.Plan(inst.ids).apply(inst.xyz, inst.k, inst.q)[:, 0]
        row = {}
        for layout in ("tiles", "csr"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = p2p.Plan(xyz, ids, inst.k, dtype=torch.complex64, layout=layout)
            torch.cuda.synchronize()  # the build returns before its last kernels end
            plan_ms = (time.perf_counter() - t0) * 1e3
            info = plan.info()
            n_pairs = info["n_pairs"]
            y = plan.apply(q)
            err = None
            if ref is not None:
                err = float(np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref))
            spin_up(lambda: plan.apply(q), torch)
            plan.timing(True)
            for _ in range(reps):
                plan.apply(q)
            torch.cuda.synchronize()
            kern_ms, calls = plan.timing_read()
            plan.timing(False)
            kern_ms /= calls
            row[layout] = {"plan_ms": round(plan_ms, 3), "sweep_ms": round(kern_ms, 4),
                           "gpairs_s": round(n_pairs / kern_ms / 1e6, 2), "rel_err": err,
                           "close_pairs": info["n_close_pairs"], "near_boxes": info["n_near_boxes"],
                           "boxes": info["n_boxes"], "device_bytes": info["device_bytes"]}
            plan.close()
        row["n_pairs"] = n_pairs
        out["D%d" % d] = row
        log("ellipsoid D=%d: %d pairs; tiles %.1f Gpair/s (plan %.2f ms, err %s), csr %.1f Gpair/s (plan %.2f ms, "
            "err %s)" % (d, n_pairs, row["tiles"]["gpairs_s"], row["tiles"]["plan_ms"], row["tiles"]["rel_err"],
                         row["csr"]["gpairs_s"], row["csr"]["plan_ms"], row["csr"]["rel_err"]))
    return out


def measure_paper_2d(p2p, torch, reps, with_oracle, max_layout_bytes=4e9, max_boxes=4 ** 12):
    """The paper's own grid (section 4.6, eq. 38): N = 4^L points uniform on the unit
    square, L = 4..11, quadtree height L + i, i = -3..3 (D = 4^(1-i) points per box,
    empty boxes included), CT = 15, one real potential per point, the 2-D log kernel.
    Per cell: the Indexing and Repetition layouts' host collection, host-to-device
    transfer and kernel (section 3.2, 3.3), the library's own plan and sweep of the
    same points, and, for N <= 65536, the oracle on one core (the paper's CPU
    baseline).  Cells whose Repetition layout would exceed max_layout_bytes, or whose
    tree has more than max_boxes leaves, are left out (as the paper left out cells
    beyond its resources).  Then the paper's model (section 3.4) re-fitted on these
    measurements: lambda_RAM from eq. 16, lambda_GPU from eq. 28, and alpha, beta,
    gamma of eq. 36 by non-negative least squares."""
    import numpy as np
    CT = 15
    rows = []
    dev = torch.device("cuda:0")

    def kernel_ms(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    for L in range(4, 12):
        N = 4 ** L
        rng = np.random.default_rng(L)
        xy = rng.random((N, 2))
        q = rng.standard_normal(N)
        xyz = np.zeros((N, 3))
        xyz[:, :2] = xy
        ref = None
        for i in range(-3, 4):
            level = L + i
            boxes = 4 ** (level - 1)
            D = N / boxes
            row = {"L": L, "i": i, "N": N, "level": level, "boxes": boxes, "D": D}
            # Repetition record: 3 + 27 CT doubles, or 3 + 3 x the largest neighbourhood
            est = N * 8 * (3 + 3 * 9 * max(CT, int(np.ceil(2.5 * D))))
            if boxes > max_boxes or est > max_layout_bytes:
                row["skipped"] = "Repetition layout ~%.1f GB or %d boxes" % (est / 1e9, boxes)
                rows.append(row)
                continue
            if with_oracle and N <= 65536:
                import oracle
                t0 = time.perf_counter()
                ref = oracle.apply2d(xy, q, level, threads=1)
                row["baseline_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
            else:
                ref = None
            for method in ("indexing", "repetition"):
                Q = p2p.Quad2D(method, xy, q, level, CT)
                inf = Q.info()
                trs = []
                for _ in range(3):
                    Q.transfer()
                    trs.append(Q.info()["transfer_ms"])
                y = torch.empty(N, dtype=torch.float64, device=dev)
                k_ms = kernel_ms(lambda: Q.run(y))
                m = {"collect_ms": round(inf["collect_ms"], 3), "transfer_ms": round(float(np.median(trs)), 3),
                     "kernel_ms": round(k_ms, 4), "layout_bytes": inf["layout_bytes"], "t_max": inf["t_max"]}
                if ref is not None:
                    yy = y.cpu().numpy()
                    m["rel_err"] = float(np.linalg.norm(yy - ref) / np.linalg.norm(ref))
                row[method] = m
                row["t"] = inf["t_max"]
                Q.close()
            # the library's own route: device plan of (x, y, 0), FP64 sweep with the 2-D kernel
            xd = torch.from_numpy(xyz).to(dev)
            qd = torch.from_numpy(q).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P = p2p.Plan.from_grid(xd, (0.0, 0.0, 0.0), 2.0 ** (1 - level), 0.0, dtype=torch.complex128, layout="csr")
            torch.cuda.synchronize()
            plan_ms = (time.perf_counter() - t0) * 1e3
            yo = torch.empty(N, dtype=torch.float64, device=dev)
            a_ms = kernel_ms(lambda: P.apply_log2d(qd, yo))
            row["library"] = {"plan_ms": round(plan_ms, 3), "apply_ms": round(a_ms, 4)}
            if ref is not None:
                yy = yo.cpu().numpy()
                row["library"]["rel_err"] = float(np.linalg.norm(yy - ref) / np.linalg.norm(ref))
            P.close()
            ind, rep = row["indexing"], row["repetition"]
            tot = lambda m: m["collect_ms"] + m["transfer_ms"] + m["kernel_ms"]
            row["X_total"] = tot(ind) / tot(rep)
            row["X_collect"] = ind["collect_ms"] / rep["collect_ms"]
            row["X_transfer"] = ind["transfer_ms"] / rep["transfer_ms"]
            row["X_kernel"] = ind["kernel_ms"] / rep["kernel_ms"]
            row["library_vs_repetition"] = tot(rep) / (row["library"]["plan_ms"] + row["library"]["apply_ms"])
            rows.append(row)
            log("paper 2-D L=%d i=%+d N=%d D=%.4g t=%d: collect %.1f / %.1f ms, transfer %.2f / %.2f, kernel %.3f / "
                "%.3f (Indexing / Repetition), Repetition %.2fx; library plan %.2f + sweep %.3f ms" % (
                    L, i, N, D, row["t"], ind["collect_ms"], rep["collect_ms"], ind["transfer_ms"],
                    rep["transfer_ms"], ind["kernel_ms"], rep["kernel_ms"], row["X_total"],
                    row["library"]["plan_ms"], row["library"]["apply_ms"]))
    fit = paper_model_fit(rows)
    done = [r for r in rows if "X_total" in r]
    best = max((r for r in done if r["N"] >= 16384), key=lambda r: r["X_total"])
    return {"workload": "unit square, N = 4^L (L = 4..11), height L + i (i = -3..3), CT = 15, 2-D log kernel, FP64",
            "cells": rows, "fit": fit,
            "repetition_over_indexing_max_N_ge_16384": {"X_total": round(best["X_total"], 3), "L": best["L"],
                                                        "i": best["i"]},
            "paper_repetition_over_indexing": "7-13x for N >= 16,000 and i >= 2 (context only: other hardware)"}


def measure_overlap(p2p, W, torch, reps):
    """The near field beside a far-field stand-in (paper, section 1: the P2P operator
    does not depend on the far field and takes about 30% of the MLFMA product's
    time).  The FP32 apply of the 2M-point sphere runs on a stream of its own; the
    stand-in -- batched FP32 matrix products, sized to take about 70 / 30 of the
    apply's time -- on a second stream (both at
    the default priority).  Two stand-ins: large products that fill the device by
    themselves, and many small launches that do not (as a far field's per-level
    translations may).  Reported: each alone, both started together (median of
    reps), the time saved against running them one after the other, and whether
    the apply's output is bitwise the same."""
    import numpy as np
    dev = torch.device("cuda:0")
    inst = W.sphere_2m()
    xyz = torch.from_numpy(inst.xyz).to(dev)
    q = torch.from_numpy(inst.q[:, 0].copy()).to(dev)
    plan = p2p.Plan.from_grid(xyz, [float(v) for v in inst.origin], inst.h, inst.k, dtype=torch.complex64,
                              layout="csr")
    s_near, s_far = torch.cuda.Stream(), torch.cuda.Stream()
    y_ref = torch.empty_like(q)
    y = torch.empty_like(q)

    def near(out):
        with torch.cuda.stream(s_near):
            plan.apply(q, out)

    def timed(fns):
        e0 = torch.cuda.Event(enable_timing=True)
        e0.record(torch.cuda.current_stream())
        ends = []
        for st, fn in fns:
            st.wait_event(e0)
            fn()
            e = torch.cuda.Event(enable_timing=True)
            e.record(st)
            ends.append(e)
        torch.cuda.synchronize()
        return max(e0.elapsed_time(e) for e in ends)

    for _ in range(5):
        near(y_ref)
    torch.cuda.synchronize()
    t_near = float(np.median([timed([(s_near, lambda: near(y_ref))]) for _ in range(reps)]))
    out = {"near_ms": round(t_near, 4), "stand_ins": {}}
    # two stand-ins, each sized to about 70 / 30 of the apply's time: large batched
    # products that fill the device on their own, and many small launches that do
    # not.  Each is captured once into a HIP graph and replayed, so that host launch
    # costs do not decide the result; the near field is enqueued first.
    for name, batch, dim in (("large", 512, 64), ("small", 8, 32)):
        a = torch.randn(batch, dim, dim, device=dev)
        b = torch.randn(batch, dim, dim, device=dev)
        c = torch.empty(batch, dim, dim, device=dev)

        def captured(count):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(s_far):
                torch.bmm(a, b, out=c)  # warm the library's handles before capture
                s_far.synchronize()
                with torch.cuda.graph(g, stream=s_far):
                    for _ in range(count):
                        torch.bmm(a, b, out=c)

            def run():
                with torch.cuda.stream(s_far):
                    g.replay()
            return run, g

        run10, g10 = captured(10)
        for _ in range(3):
            run10()
        torch.cuda.synchronize()
        t10 = float(np.median([timed([(s_far, run10)]) for _ in range(5)]))
        count = max(1, int(round(10 * t_near * 7.0 / 3.0 / t10)))
        far, g = captured(count)
        far()
        torch.cuda.synchronize()
        t_far = float(np.median([timed([(s_far, far)]) for _ in range(reps)]))
        both, same = [], True
        for _ in range(reps):
            both.append(timed([(s_near, lambda: near(y)), (s_far, far)]))
            same = same and bool(torch.equal(y, y_ref))
        t_both = float(np.median(both))
        out["stand_ins"][name] = {
            "launches": "%d x batched %d x (%d x %d) FP32 products, one captured graph" % (count, batch, dim, dim),
            "far_ms": round(t_far, 4), "concurrent_ms": round(t_both, 4), "serial_ms": round(t_near + t_far, 4),
            "saved_fraction_of_near": round((t_near + t_far - t_both) / t_near, 4),
            "near_output_bitwise_equal": same}
        del g, g10
    plan.close()
    out["workload"] = "sphere2M_D32_k128pi FP32 apply (CSR) on its own stream beside a far-field stand-in"
    return out


def paper_model_fit(rows, n_min=4096):
    """The paper's speedup model (section 3.4) against the measured cells with
    N >= n_min (smaller cells take microseconds, where launch and timer overheads
    dominate).  Eq. 36 models X_total = alpha X_collect + gamma X_transfer + beta
    X_kernel with constant coefficients: fitted here by non-negative least squares,
    as the paper does.  Exactly, X_total = sum over phases of (Repetition's time in
    the phase / its total) x X_phase, so each cell's own time shares are the
    coefficients that make eq. 36 exact; their means are reported beside the fit.
    lambda_RAM (eq. 16) and lambda_GPU (eq. 28) per cell, by density D."""
    import numpy as np
    from scipy.optimize import nnls
    done = [r for r in rows if "X_total" in r and r["N"] >= n_min]
    A = np.array([[r["X_collect"], r["X_kernel"], r["X_transfer"]] for r in done])
    b = np.array([r["X_total"] for r in done])
    coef, _ = nnls(A, b)
    pred = A @ coef
    tot = lambda m: m["collect_ms"] + m["transfer_ms"] + m["kernel_ms"]
    shares = np.array([[r["repetition"]["collect_ms"] / tot(r["repetition"]),
                        r["repetition"]["kernel_ms"] / tot(r["repetition"]),
                        r["repetition"]["transfer_ms"] / tot(r["repetition"])] for r in done])
    by_d = {}
    for r in done:
        d = by_d.setdefault("%g" % r["D"], {"lambda_RAM": [], "lambda_GPU": [], "X_total": []})
        d["lambda_RAM"].append(r["X_collect"] * 21.6 * r["t"] * r["D"])
        d["lambda_GPU"].append(r["X_kernel"] * r["N"] * r["D"] / (55.3 * r["t"]))
        d["X_total"].append(r["X_total"])
    med = lambda v: round(float(np.median(v)), 4)
    return {"cells": len(done), "N_min": n_min,
            "nnls": {"alpha": round(float(coef[0]), 4), "beta": round(float(coef[1]), 4),
                     "gamma": round(float(coef[2]), 4),
                     "rel_residual": round(float(np.linalg.norm(pred - b) / np.linalg.norm(b)), 4)},
            "time_shares_mean": {"alpha": round(float(shares[:, 0].mean()), 4),
                                 "beta": round(float(shares[:, 1].mean()), 4),
                                 "gamma": round(float(shares[:, 2].mean()), 4)},
            "by_density": {k: {"lambda_RAM_median": med(v["lambda_RAM"]), "lambda_GPU_median": med(v["lambda_GPU"]),
                               "X_total_median": med(v["X_total"]), "cells": len(v["X_total"])}
                           for k, v in sorted(by_d.items(), key=lambda kv: -float(kv[0]))},
            "paper": {"alpha": 0.82, "beta": 0.09, "gamma": 0.18, "lambda_RAM": "75-180, mean 108",
                      "lambda_GPU": "about 640", "hardware": "Core i7 7th gen + GeForce GTX 1050"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--no-mrhs", action="store_true", help="skip the multi-right-hand-side batch")
    ap.add_argument("--mrhs-only", action="store_true", help="only the multi-right-hand-side batch")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the reverse-pass and layout measurements on their own workloads")
    ap.add_argument("--layout", choices=["csr", "tiles"], default="csr",
                    help="source layout of the timed step and of the roofline kernel")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only build the plan and run the apply --apply-reps times (for counter runs)")
    ap.add_argument("--sweep-precision", choices=["f32", "f64"], default="f32",
                    help="precision of the plan that --sweep-only runs")
    ap.add_argument("--sweep-workload", choices=["sphere2M", "ellipsoid4M_D16", "ellipsoid4M_D32", "ellipsoid4M_D64"],
                    default="sphere2M", help="input of --sweep-only")
    ap.add_argument("--paper-2d", action="store_true",
                    help="only the paper's 2-D experiment grid (Indexing vs Repetition) and the model re-fit")
    ap.add_argument("--paper-2d-cell", default=None, metavar="L,i",
                    help="only the two 2-D layouts' kernels on one cell of that grid, 5 runs each "
                         "(for counter runs)")
    ap.add_argument("--issue-rates", action="store_true",
                    help="only the VALU issue-rate microbenchmark (one JSON line)")
    ap.add_argument("--overlap", action="store_true",
                    help="only the near field beside a far-field stand-in on a second stream")
    ap.add_argument("--backward-only", action="store_true",
                    help="only run the reverse pass on its 500k-point cube, FP32 then FP64, "
                         "--apply-reps times each (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the operator is built and measured on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import torch
    import paper_2403_01596_amd as p2p
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copied 3 x %d bytes" % (a.numel() * 4))
        return 0

    if args.overlap:
        print(json.dumps(measure_overlap(p2p, W, torch, 20)))
        return 0

    if args.issue_rates:
        print(json.dumps(measure_issue_rates(torch)))
        return 0

    if args.paper_2d_cell:
        L, i = (int(v) for v in args.paper_2d_cell.split(","))
        rng = np.random.default_rng(L)
        xy, q = rng.random((4 ** L, 2)), rng.standard_normal(4 ** L)
        for method in ("indexing", "repetition"):
            Q = p2p.Quad2D(method, xy, q, L + i, 15)
            Q.transfer()
            y = torch.empty(4 ** L, dtype=torch.float64, device="cuda")
            for _ in range(5):
                Q.run(y)
            torch.cuda.synchronize()
            log("paper 2-D cell L=%d i=%d: %s kernel run 5 times" % (L, i, method))
            Q.close()
        return 0

    if args.paper_2d:
        print(json.dumps(measure_paper_2d(p2p, torch, 5, not args.no_cpu)))
        return 0

    if args.mrhs_only:
        print(json.dumps(measure_mrhs(p2p, W, torch, args.apply_reps, not args.no_cpu)))
        return 0

    if args.backward_only:
        g = W.grad_cube_500k()
        gx = torch.from_numpy(g.xyz).to(dev)
        gi = torch.from_numpy(g.ids).to(dev)
        for dt in (torch.complex64, torch.complex128):
            q = torch.from_numpy(g.q[:, 0].copy()).to(dev).to(dt)
            plan = p2p.Plan(gx, gi, g.k, dtype=dt, layout="csr")
            spin_up(lambda: plan.backward(q, q), torch)
            plan.timing(True)
            for _ in range(args.apply_reps):
                plan.backward(q, q)
            torch.cuda.synchronize()
            kern_ms, calls = plan.timing_read()
            plan.timing(False)
            log("backward-only: %s, %d timed passes, %d pairs each, sweep kernel %.4f ms (HIP events)" % (
                dt, args.apply_reps, plan.info()["n_pairs"], kern_ms / calls))
            plan.close()
        return 0

    if args.sweep_only and args.sweep_workload != "sphere2M":
        inst = W.ellipsoid_4m(int(args.sweep_workload.split("_D")[1]))
    else:
        inst = W.sphere_2m()
    log("workload %s: n=%d h=%.6g D=%.2f k=%.4f" % (inst.name, inst.n, inst.h, inst.d_mean, inst.k))
    xyz = torch.from_numpy(inst.xyz).to(dev)
    q32 = torch.from_numpy(inst.q[:, 0].copy()).to(dev)
    q64 = q32.to(torch.complex128)
    origin = [float(v) for v in inst.origin]

    if args.sweep_only:
        ids = p2p.box_ids(xyz, origin, inst.h)
        f64 = args.sweep_precision == "f64"
        plan = p2p.Plan(xyz, ids, inst.k, dtype=torch.complex128 if f64 else torch.complex64, layout=args.layout)
        for _ in range(args.apply_reps):
            plan.apply(q64 if f64 else q32)
        torch.cuda.synchronize()
        log("sweep-only: %d applies, %d pairs each" % (args.apply_reps, plan.info()["n_pairs"]))
        plan.close()
        return 0

    def step():
        plan = p2p.Plan.from_grid(xyz, origin, inst.h, inst.k, dtype=torch.complex64, layout=args.layout)
        y = plan.apply(q32)
        plan.close()
        return y

    # ---- the step: box ids + plan + FP32 apply + release.  Untimed steps for a
    # fixed spell first, so that the timed ones run at the steady clock rather than
    # on the ramp out of idle, then the W warm-up steps.
    spin_end = time.perf_counter() + SPIN_UP_S
    while time.perf_counter() < spin_end:
        step()
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the timed region: K steps back to back, bracketed by a synchronisation and a
    # HIP event on the stream the steps run on at each end (the plan build's host
    # waits show up as idle time inside it); the headline is the region over K
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r0.record()
    for _ in range(args.steps):
        y32 = step()
    r1.record()
    torch.cuda.synchronize()
    wall_s = (time.perf_counter() - t0) / args.steps
    step_s = r0.elapsed_time(r1) * 1e-3 / args.steps
    # the spread of single steps: K more, an event pair around each.  Every event
    # recorded behind the sweep costs GPU time of its own (measured: the idle spell
    # between a sweep and the next build's first kernel grows from about 6 us to
    # 40-60 us with the two per-step events), so these run above the region's mean.
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    step_ms = np.array([a.elapsed_time(b) for a, b in evs])
    log("step: %.3f ms (timed region / %d), %.3f ms (host clock); per-step events: median %.3f, min %.3f" % (
        step_s * 1e3, args.steps, wall_s * 1e3, float(np.median(step_ms)), float(step_ms.min())))

    # ---- where the step's time goes: one step at a time from an idle GPU, an event
    # before the build, between build and apply, and after the apply (the build
    # returns before its last kernels end, so the GPU's clock divides the phases);
    # the release on the host clock
    phases = {"plan_create": 0.0, "apply": 0.0, "release": 0.0}
    for _ in range(args.steps):
        ea, eb, ec = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        ea.record()
        pl = p2p.Plan.from_grid(xyz, origin, inst.h, inst.k, dtype=torch.complex64, layout=args.layout)
        eb.record()
        pl.apply(q32)
        ec.record()
        t3 = time.perf_counter()
        pl.close()
        t4 = time.perf_counter()
        torch.cuda.synchronize()
        for key, dt in zip(phases, (ea.elapsed_time(eb), eb.elapsed_time(ec), (t4 - t3) * 1e3)):
            phases[key] += dt / args.steps
    log("phases (ms): " + ", ".join("%s %.3f" % kv for kv in phases.items()))
    # the box ids on their own (p2p_box_ids, one synchronisation), for comparison
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        p2p.box_ids(xyz, origin, inst.h)
    box_ids_ms = (time.perf_counter() - t0) * 1e3 / args.steps

    # ---- pieces of the step, on resident plans
    ids = p2p.box_ids(xyz, origin, inst.h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan32 = p2p.Plan(xyz, ids, inst.k, dtype=torch.complex64, layout=args.layout)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan32.info()
    n_pairs = info["n_pairs"]
    # the plan build against the HBM roofline: the bytes it must move at least
    # (positions read once; permutation, FP64 and fixed-point sorted coordinates,
    # box tables and neighbour lists written once), over the measured build of the
    # timed step (ids computed inside the build, so no id array is read)
    plan_bytes = (inst.n * (24 + 4 + 24 + 12) + info["n_boxes"] * (8 + 4 * 4) + info["n_nbr"] * 4
                  + info["tile_entries"] * (4 + 12))

    def time_apply(plan, q, reps):
        spin_up(lambda: plan.apply(q), torch)
        plan.timing(True)
        plan.apply(q)
        torch.cuda.synchronize()
        plan.timing_read()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = plan.apply(q)
        e1.record()
        torch.cuda.synchronize()
        sweep_ms, calls = plan.timing_read()
        plan.timing(False)
        return out, e0.elapsed_time(e1) / reps, sweep_ms / calls

    other = "tiles" if args.layout == "csr" else "csr"
    y32, apply32_ms, sweep32_ms = time_apply(plan32, q32, args.apply_reps)
    log("f32 %s: apply %.3f ms, sweep kernel %.3f ms" % (args.layout, apply32_ms, sweep32_ms))
    plan_o = p2p.Plan(xyz, ids, inst.k, dtype=torch.complex64, layout=other)
    _, apply_o_ms, sweep_o_ms = time_apply(plan_o, q32, max(3, args.apply_reps // 4))
    plan_o.close()
    log("f32 %s: apply %.3f ms, sweep kernel %.3f ms" % (other, apply_o_ms, sweep_o_ms))
    plan64 = p2p.Plan(xyz, ids, inst.k, dtype=torch.complex128, layout=args.layout)
    y64, apply64_ms, sweep64_ms = time_apply(plan64, q64, max(3, args.apply_reps // 4))
    plan64.close()
    log("f64 %s: apply %.3f ms, sweep kernel %.3f ms" % (args.layout, apply64_ms, sweep64_ms))

    achieved = n_pairs / (sweep32_ms * 1e-3) / 1e9
    traffic = stored_traffic() if args.layout == "csr" else None
    issue = measure_issue_rates(torch)
    issued = stored_value(VALU_COUNTERS_FILE, "issued_slots_per_pair") if args.layout == "csr" else None
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(PEAK_GPAIRS, 1), "unit": "Gpair/s",
                "frac": round(achieved / PEAK_GPAIRS, 4), "traffic": traffic,
                "kernel": "sweep FP32 %s (k_apply<F32,helmholtz,%s>)" % (args.layout, args.layout),
                "work_per_pair": "15 VALU (1 slot) + 3 transcendental (4 slots) = %d issue slots of 128 lanes/clk/CU"
                                 % SLOTS_PER_PAIR,
                "pair_stream_measured": {"gpairs_s": issue["pair"]["gpairs_s"],
                                         "fma_slots_per_pair": issue["pair"]["fma_slots_per_trip"],
                                         "fma_lanes_per_clk_cu_at_2_4ghz":
                                             issue["fma"]["lanes_per_clk_cu_at_2_4ghz"]},
                "algorithmic_slots_per_pair": SLOTS_PER_PAIR, "issued_slots_per_pair": issued,
                "pairs_per_launch": n_pairs, "kernel_ms": round(sweep32_ms, 4)}

    # ---- oracle on the host cores: every target row of the same input
    cpu = None
    errs = {}
    if not args.no_cpu:
        import oracle
        orc = oracle.Plan(inst.ids)
        tb = orc.tables()
        rows = np.arange(inst.n)
        sizes = np.diff(tb["box_start"]).astype(np.int64)
        nbr_src = np.array([sizes[tb["nbr_idx"][tb["nbr_start"][T]:tb["nbr_start"][T + 1]]].sum()
                            for T in range(len(sizes))], dtype=np.int64)
        pos = np.empty(inst.n, np.int64)
        pos[tb["perm"]] = np.arange(inst.n)
        box_of_row = np.searchsorted(tb["box_start"], pos[rows], side="right") - 1
        # the points are distinct, so each row skips exactly its self pair
        assert np.unique(inst.xyz, axis=0).shape[0] == inst.n
        pairs_sample = int(nbr_src[box_of_row].sum() - rows.size)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        t0 = time.perf_counter()
        yref = orc.apply_rows(inst.xyz, inst.k, inst.q, rows, threads=threads)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": round(pairs_sample / cpu_s / 1e9, 5), "unit": "Gpair/s", "cores": threads,
               "kind": "oracle", "seconds": round(cpu_s, 2), "cpu_model": cpu_model(),
               "host_threads": os.cpu_count(),
               "sample": "every target row of the same 2M-point input (%d rows, %d pairs), "
                         "FP64, OpenMP over rows" % (rows.size, pairs_sample),
               "single_core": single_core_oracle(W, oracle)}
        y32h = y32.cpu().numpy()[rows]
        y64h = y64.cpu().numpy()[rows]
        ref = yref[:, 0]
        errs = {"f32": float(np.linalg.norm(y32h - ref) / np.linalg.norm(ref)),
                "f64": float(np.linalg.norm(y64h - ref) / np.linalg.norm(ref))}
        log("oracle %.1f s on %d threads; rel L2 f32 %.3e f64 %.3e" % (cpu_s, threads, errs["f32"], errs["f64"]))
    plan32.close()
    mrhs = None if args.no_mrhs else measure_mrhs(p2p, W, torch, max(3, args.apply_reps // 4), not args.no_cpu)
    backward = None if args.no_extra else measure_backward(p2p, W, torch, max(3, args.apply_reps // 4),
                                                           not args.no_cpu)
    layouts = None if args.no_extra else measure_layouts(p2p, W, torch, max(3, args.apply_reps // 4),
                                                         not args.no_cpu)

    value = n_pairs / step_s / 1e9
    line = {
        "metric": "near-field interactions/s (G-pairs/s) at stated rel-err; % of VALU/HBM roofline",
        "value": round(value, 3), "unit": "Gpair/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "step_timing": {"statistic": "HIP events bracketing %d back-to-back steps, over %d" % (args.steps, args.steps),
                        "host_clock_mean_ms": round(wall_s * 1e3, 4),
                        "per_step_events": {"median_ms": round(float(np.median(step_ms)), 4),
                                            "min_ms": round(float(step_ms.min()), 4),
                                            "max_ms": round(float(step_ms.max()), 4),
                                            "note": "an event pair around each of %d further steps; the events "
                                                    "themselves add GPU time to each step" % args.steps}},
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": inst.name, "n_points": inst.n, "k": inst.k, "leaf_h": inst.h,
                   "d_mean": round(inst.d_mean, 3), "rhs": 1, "precision": "f32", "layout": args.layout,
                   "step": "plan build with the leaf-box ids from (origin, h) + FP32 apply + release"},
        "rel_err": errs or None,
        "n_pairs": n_pairs,
        "apply": {"f32_%s_gpairs_s" % args.layout: round(n_pairs / apply32_ms / 1e6, 2),
                  "f32_%s_gpairs_s" % other: round(n_pairs / apply_o_ms / 1e6, 2),
                  "f64_%s_gpairs_s" % args.layout: round(n_pairs / apply64_ms / 1e6, 2),
                  "f32_%s_ms" % args.layout: round(apply32_ms, 4), "f32_%s_ms" % other: round(apply_o_ms, 4),
                  "f64_%s_ms" % args.layout: round(apply64_ms, 4),
                  "sweep_ms": {"f32_" + args.layout: round(sweep32_ms, 4), "f32_" + other: round(sweep_o_ms, 4),
                               "f64_" + args.layout: round(sweep64_ms, 4)},
                  "roofline_f64": {"bound": "alu", "achieved": round(n_pairs / sweep64_ms / 1e6, 2),
                                   "peak": round(PEAK_F64_GPAIRS, 1), "unit": "Gpair/s",
                                   "frac": round(n_pairs / sweep64_ms / 1e6 / PEAK_F64_GPAIRS, 4),
                                   "work_per_pair": "52 FP64 VALU (2 slots) + v_rsq_f64 (8) = %d issue slots"
                                                    % F64_SLOTS_PER_PAIR}},
        "plan_ms": round(plan_s * 1e3, 3),
        "step_phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "plan_roofline": {"bound": "hbm", "algorithmic_bytes": plan_bytes,
                          "achieved": round(plan_bytes / (phases["plan_create"] * 1e-3) / 1e9, 1),
                          "peak": 8000.0, "unit": "GB/s",
                          "frac": round(plan_bytes / (phases["plan_create"] * 1e-3) / 8e12, 4),
                          "bytes_per_point": "24 read (positions) + 40 written (permutation, FP64 and fixed-point "
                                             "coordinates) + 24 per box + 4 per neighbour-list entry"},
        "box_ids_call_ms": round(box_ids_ms, 4),
        "plan": {"n_boxes": info["n_boxes"], "t_max": info["t_max"], "device_bytes": info["device_bytes"],
                 "near_boxes": info["n_near_boxes"], "close_pairs": info["n_close_pairs"]},
        "roofline": roofline,
        "issue_rates": issue,
        "cpu_baseline": cpu,
        "multi_rhs": mrhs,
        "backward": backward,
        "layouts": layouts,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
