"""Benchmark: grid-point RK4 stage updates per second of the generating-function
stencil on one MI355X, with the HBM roofline of the stage kernel and the CPU
oracle timed beside it.

Workload (default): 10 Kerr modes at cutoff 6 (6^10 = 60,466,176 grid points
in the diagonal occupation-difference sector), seeded parameters, observable
prod_j (|0><0| - |1><1|), merged layout, mixed precision (complex64 stage
grids with FP32 stencil arithmetic, complex128 state, FP64 expectation),
dt = 0.05 ns.  One benchmark step is one RK4 time step (four fused stage
launches over the whole grid); the timed region is K steps through
hgf_evolve followed by one hgf_expectation.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point RK stage updates/s + % HBM peak; time-to-1e-5 vs FP64 plain"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per grid point of one stage launch, averaged over the
# four stages of one RK4 step.  With s = size of a stage-grid element and
# w = size of a state element (y), the stages move
#   stage 1: read yf (s) + write X1 (s)                        = 2s
#   stage 2: read X1 (s) + write V1 (s)                        = 2s
#   stage 3: read V1, X1 (2s) + write V2 (s)                   = 3s
#   stage 4: read V2, X1 (2s) + read/write y (2w) + write yf (s) = 3s + 2w
# in mixed precision (yf is the stage-1 stencil input, a copy of y in the
# stage precision); in FP64 the stencil input of stage 1 is y itself and
# there is no yf:  stage 1 = 2s, stage 4 = 2s + 2w.
#   complex64 stages, complex128 state (mixed):  s = 8,  w = 16 -> 112 / 4 = 28
#   real float stages, real double state (mixed): s = 4, w = 8  ->  56 / 4 = 14
#   complex128 (fp64): s = w = 16 -> 176 / 4 = 44;   real double (fp64): 22
def bytes_per_point_stage(precision: str, real: bool) -> float:
    s = (4 if precision == "mixed" else 8) * (1 if real else 2)
    w = 8 * (1 if real else 2)
    if precision == "mixed":
        return (2 * s + 2 * s + 3 * s + 3 * s + 2 * w) / 4.0
    return (2 * s + 2 * s + 3 * s + 2 * s + 2 * w) / 4.0
STAGE_KERNEL = "k_rk4_tiled"
KERNEL_SOURCE = os.path.join(ROOT, "paper_2203_05526_amd", "csrc", "hgf_tiled.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_rk4_tiled_10mode_mixed_traffic.json")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def stored_traffic(shape: dict, real: bool = True, precision: str = "mixed"):
    """HBM bytes per stage launch from committed rocprofv3 counter runs, or
    None when the kernel source changed since, or no run used this launch
    shape (with these element types)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    want = [shape[k] for k in ("nfast", "threads", "xblock", "pipe", "wgs_per_cu", "walk_block")]
    kind = f":{precision}:{'real' if real else 'complex'}:"
    for entry in t.get("shapes", []):
        if kind in entry["tune_cache_line"] and [int(x) for x in entry["tune_cache_line"].split()[1:7]] == want:
            return entry["traffic_bytes_per_launch"]
    return None


def cpu_baseline(w, steps: int):
    """The CPU oracle (number-basis adjoint master equation, classical RK4) on
    the same grid for a few steps, all host threads."""
    import oracle
    ops = oracle.product_sectors(w.factors)
    cores = oracle.max_threads()  # before the one-thread run below sets the count to 1
    t0 = time.perf_counter()
    oracle.evolve_steps(w.system, ops, steps, w.dt)
    el = time.perf_counter() - t0
    pts = int(np.prod(w.system.cutoff))
    # one host thread: the same ten modes at cutoff 4 (4^10 points; the same
    # per-point work, a grid small enough for a few steps in seconds)
    s1 = w.system.copy()
    s1.cutoff = (4,) * s1.n_modes
    f1 = [f[:4, :4] for f in w.factors]
    t1 = time.perf_counter()
    oracle.evolve_steps(s1, oracle.product_sectors(f1), 3, w.dt, nthreads=1)
    el1 = time.perf_counter() - t1
    return {"value": pts * 4 * steps / el, "unit": "point-stage updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} RK4 steps over all {pts} points of the same 10-mode grid ({el:.1f} s)",
            "single_thread": {"value": 4 ** s1.n_modes * 4 * 3 / el1, "unit": "point-stage updates/s",
                              "sample": f"3 RK4 steps of the same 10 modes at cutoff 4 on one thread ({el1:.1f} s)"}}


def golden(name: str):
    """Stored FP64 oracle values (written by tests/golden/make_golden.py, which
    calls only the oracle)."""
    with open(os.path.join(ROOT, "tests", "golden", f"{name}.json")) as fh:
        return json.load(fh)


def ten_mode_full_horizon(hgf, torch, w, S, tune_cache=None):
    """The 10-mode workload over its full horizon (T = 2 us, 4e4 steps) in
    mixed precision and in FP64, each in its tuned launch shape: wall time of
    hgf_evolve + hgf_expectation and the relative error of the expectation
    value against the stored FP64 oracle value (a product of single-mode
    oracle runs, exact on the diagonal sector)."""
    ref = complex(*golden("workloads")["ten_mode"]["value"])
    out = {"workload": "10 Kerr modes, cutoff 6, parity-weighted projector, T = 2 us, dt = 0.05 ns (4e4 steps)",
           "oracle_value": [ref.real, ref.imag]}
    for prec in ("mixed", "fp64"):
        op = hgf.map_operator(S, factors=w.factors, precision=prec)
        hgf.autotune([op], w.dt, cache=tune_cache)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hgf.evolve(op, w.t_total, w.dt)
        J = hgf.expectation(op, w.states[0])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[prec] = {"seconds": el, "steps": op.info()["steps_done"], "rel_err_vs_oracle": abs(J - ref) / abs(ref)}
        log(f"10-mode full horizon {prec}: {el:.1f} s, error {out[prec]['rel_err_vs_oracle']:.2e}")
        del op
    out["mixed_within_1e-5"] = out["mixed"]["rel_err_vs_oracle"] <= 1e-5
    out["fp64_within_1e-10"] = out["fp64"]["rel_err_vs_oracle"] <= 1e-10
    return out


def time_to_tolerance(hgf, torch):
    """Wall time of the full 3-mode horizon (1e5 steps) in mixed precision and
    in FP64, each with its error against the FP64 oracle's stored value."""
    import synth
    gold = golden("three_mode")
    w = synth.three_mode_c1()
    S = hgf.define_system(w.system)
    ref = complex(*gold["values"][0])
    out = {"workload": "3 Kerr modes, cutoff 12, bitstring projector, T = 10 us, dt = 0.1 ns (1e5 steps)"}
    for prec in ("mixed", "fp64"):
        op = hgf.map_operator(S, factors=w.factors, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hgf.evolve(op, w.t_total, w.dt)
        J = hgf.expectation(op, w.states[0])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"{prec}_s"] = el
        out[f"{prec}_rel_err"] = abs(J - ref) / abs(ref)
    out["mixed_within_1e-5"] = out["mixed_rel_err"] <= 1e-5
    out["off_diagonal"] = stiff_time_to_tolerance(hgf, torch)
    return out


def stiff_time_to_tolerance(hgf, torch):
    """Wall time and error against the FP64 oracle's stored value on the
    product-of-quadratures workload (4 modes, cutoff 8, 16 off-diagonal
    sectors with Kerr phases of ~1.5e3 rad/us, T = 0.02 us): classical RK4 at
    dt = 1 ps (2e4 steps) against the integrating-factor RK4 at dt = 1 ns (20
    steps), in FP64 and mixed precision."""
    import synth
    with open(os.path.join(ROOT, "tests", "golden", "quadratures.json")) as fh:
        gold = json.load(fh)
    ref = complex(*gold["value"])
    w = synth.grad_c3b()
    S = hgf.define_system(w.system)
    for prec in ("fp64", "mixed"):  # load the kernels once (the calls below, on copies)
        warm = hgf.map_operator(S, factors=w.factors, precision=prec)
        hgf.evolve(warm, 4 * w.dt, w.dt)
        hgf.expectation(warm, w.states[0])
        warm = hgf.map_operator(S, factors=w.factors, precision=prec)
        hgf.evolve(warm, w.t_total, 1e-3, scheme="lawson")
        hgf.expectation(warm, w.states[0])
    del warm
    out = {"workload": "4 Kerr modes, cutoff 8, product of quadratures, T = 0.02 us (16 sectors of 7^4 points)"}
    for scheme, dt in (("rk4", w.dt), ("lawson", 1e-3)):
        for prec in ("fp64", "mixed"):
            op = hgf.map_operator(S, factors=w.factors, precision=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hgf.evolve(op, w.t_total, dt, scheme=scheme)
            J = hgf.expectation(op, w.states[0])
            torch.cuda.synchronize()
            out[f"{scheme}_{prec}"] = {"dt_us": dt, "steps": int(round(w.t_total / dt)),
                                       "seconds": time.perf_counter() - t0, "rel_err": abs(J - ref) / abs(ref)}
    return out


def batch_throughput(hgf, torch, seq_steps: int, steps=None, tune_cache=None):
    """One grouped, graph-captured hgf_evolve_batch over the batch workload:
    64 systems of 6 modes at cutoff 8 plus 32 systems of 2-5 modes with
    cutoffs 6-20 (seeded), mixed precision, dt = 0.1 ns, over the full horizon
    T = 1 us (1e4 steps), with every member's expectation value against the
    stored FP64 oracle value; the same members evolved one call at a time
    over `seq_steps` steps for comparison.  With `steps` set, only that many
    steps are run (for profiling) and no error is reported.  The roofline
    entry is the whole batch's algorithmic bytes (every member's bytes per
    point-stage, as for the single grid, times its points, times 4 stages per
    step) over the evolve time from HIP events on the launching stream."""
    import synth
    ws = synth.batch_c2()
    ops = [hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision="mixed") for w in ws]
    pts = sum(op.info()["total_points"] for op in ops)
    dt = ws[0].dt
    import tempfile
    tmp = tempfile.TemporaryDirectory()
    batch_cache = tune_cache or os.path.join(tmp.name, "batch.txt")
    t0 = time.perf_counter()
    hgf.autotune(ops, dt, cache=batch_cache)  # grid shapes, and the grouped launches of the batch as a whole
    tune_s = time.perf_counter() - t0
    # sequential reference: the same members evolved one hgf_evolve call at a
    # time, each with the launch shape tuned for its grid alone
    ops2 = [hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision="mixed")
            for w in (ws if seq_steps else [])]
    for op in ops2:
        hgf.autotune([op], dt, cache=os.path.join(tmp.name, "shapes.txt"))
    # warm-up (plan, graph) on fresh copies, so that the timed run starts at t = 0
    warm = [hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision="mixed") for w in ws[:1]]
    hgf.evolve_batch(warm + ops[1:], [2 * dt] * len(ops), [dt] * len(ops))
    del warm
    ops = [hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision="mixed") for w in ws]
    hgf.autotune(ops, dt, cache=batch_cache)  # applies the shapes found above without measuring
    full = steps is None
    if full:
        steps = ws[0].n_steps
    step_bytes = 0.0
    for op in ops:
        info = op.info()
        if info["real_functions"] not in (0, info["n_functions"]):
            raise RuntimeError("batch member with both real and complex grids")
        step_bytes += 4 * bytes_per_point_stage("mixed", info["real_functions"] > 0) * info["total_points"]
    hgf.evolve_batch(ops, [0.0] * len(ops), [dt] * len(ops))
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    hgf.evolve_batch(ops, [w.t_total if full else steps * w.dt for w in ws], [w.dt for w in ws])
    ev1.record()
    Js = [hgf.expectation(op, w.states[0]) for op, w in zip(ops, ws)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ev_s = ev0.elapsed_time(ev1) * 1e-3
    achieved = step_bytes * steps / ev_s / 1e9
    errs = None
    if full:
        refs = [complex(*m["value"]) for m in golden("workloads")["batch"]]
        errs = [abs(J - r) / abs(r) for J, r in zip(Js, refs)]
    for op in ops2:
        hgf.evolve(op, 2 * dt, dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for op in ops2:
        hgf.evolve(op, seq_steps * dt, dt)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t1 if seq_steps else None
    tmp.cleanup()
    return {"workload": "96 systems: 64 x (6 modes, cutoff 8) + 32 x (2-5 modes, cutoffs 6-20), mixed, "
                        "T = 1 us, dt = 0.1 ns",
            "members": len(ops), "grid_points": pts, "steps": steps,
            "value": pts * 4 * steps / el, "unit": "point-stage updates/s", "seconds": el,
            "rel_err_vs_oracle": None if errs is None else max(errs),
            "within_1e-5": None if errs is None else max(errs) <= 1e-5,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_step": step_bytes,
                         "evolve_seconds_events": ev_s},
            "sequential": None if not seq_steps else
            {"steps": seq_steps, "seconds": el_seq, "value": pts * 4 * seq_steps / el_seq},
            "autotune_seconds": tune_s}


def axis_count_comparison(hgf, torch):
    """The stage kernel (mixed, real diagonal sector, autotuned shape) on grids
    of tens of millions of points with 10, 8, 7 and 5 axes: 6^10, 9^8, 13^7
    and 32^5.  With more axes more of them are slow (outside the LDS tile),
    and more neighbour tiles must be reused from one XCD's L2; the algorithmic
    bandwidth (14 B per point-stage) over the stage time from HIP events."""
    import synth
    out = []
    for cut in ((6,) * 10, (9,) * 8, (13,) * 7, (32,) * 5):
        s, _, _ = synth.seeded_system(cut, 4, alpha_range=(0.3, 1.0))
        op = hgf.map_operator(hgf.define_system(s), factors=synth.parity_factors(cut), precision="mixed")
        pts = op.info()["total_points"]
        dt = 5e-5
        hgf.autotune([op], dt)
        cfg = op.tile_config(0)
        hgf.evolve(op, 2 * dt, dt)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n = 50
        e0.record()
        hgf.evolve(op, n * dt, dt)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / (4 * n)
        gbs = bytes_per_point_stage("mixed", True) * pts / us / 1e3
        out.append({"grid": "x".join(map(str, cut)), "points": pts, "slow_axes": len(cut) - cfg["nfast"],
                    "tile_shape": cfg, "us_per_stage": us, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS})
        del op
    return out


def network_timing(hgf, torch, five_only: bool = False):
    """The driven, exchange-coupled network of the paper's example (Table I
    parameters, secular dissipator at zero temperature, observable prod_j a_j,
    horizon w_q t / pi = 10, 100 RK4 steps) for 1 to 5 modes at cutoff 6, FP64,
    on the full (k, l) grid; the operator error on the three-level truncation
    against the paper's reference recipe (cutoff 7, half the step) for up to 4
    modes.  Five modes are also run in mixed precision, and on the untiled
    stage kernel in both precisions; per stage: the wall time of the 400
    stages over 4, and the algorithmic bandwidth (44 B per point-stage in
    FP64, 28 B in mixed: the stage grids once, the state twice in stage 4)."""
    import synth
    runs = []

    def timed(op, w):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hgf.evolve(op, w.t_total, w.dt)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for n in () if five_only else (1, 2, 3, 4, 5):
        w = synth.table1_network(n, 6)
        op = hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision="fp64")
        pts = op.info()["total_points"]
        el = timed(op, w)
        rec = {"modes": n, "cutoff": 6, "grid_points": pts, "steps": w.n_steps, "seconds": el,
               "value": pts * 4 * w.n_steps / el, "unit": "point-stage updates/s",
               "kernel": ("tiled" if op.tile_config(0)["nfast"] else
                          "resident" if op.tile_config(0)["resident"] else "untiled")}
        if n <= 4:
            wr = synth.table1_network(n, 7)
            ref = hgf.map_operator(hgf.define_system(wr.system), factors=wr.factors, precision="fp64")
            hgf.evolve(ref, wr.t_total, wr.dt / 2)
            M, Mr = hgf.reconstruct(op, 3), hgf.reconstruct(ref, 3)
            rec["eps_r_3_levels"] = float(np.linalg.norm(M - Mr) / np.linalg.norm(Mr))
            del ref
        del op
        runs.append(rec)
        log(f"network {n} modes: {el:.3f} s")
    five = []
    w = synth.table1_network(5, 6)
    ref3 = None
    for prec, nbytes in (("fp64", 44), ("mixed", 28)):
        for kernel in ("tiled", "untiled"):
            op = hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision=prec)
            if kernel == "untiled":
                op.set_tile_config(0, 0)
            hgf.evolve(op, 2 * w.dt, w.dt)  # warm-up (graph capture)
            el = timed(op, w)
            pts = op.info()["total_points"]
            stage_s = el / (4 * w.n_steps)
            rec = {"precision": prec, "kernel": kernel, "stage_us": 1e6 * stage_s,
                   "value": pts / stage_s, "unit": "point-stage updates/s",
                   "algorithmic_GBps": nbytes * pts / stage_s / 1e9,
                   "hbm_frac": nbytes * pts / stage_s / 1e9 / HBM_PEAK_GBS}
            # the three-level operator after the 2 + 100 steps, against the FP64 tiled run
            M3 = hgf.reconstruct(op, 3)
            if ref3 is None:
                ref3 = M3
            else:
                rec["rel_diff_vs_fp64_3_levels"] = float(np.linalg.norm(M3 - ref3) / np.linalg.norm(ref3))
            five.append(rec)
            del op
            log(f"network 5 modes {prec} {kernel}: {1e6 * stage_s:.0f} us per stage, "
                f"{rec.get('rel_diff_vs_fp64_3_levels', 0.0):.2e} from FP64")
    return {"workload": "Table I network (chain, drive on mode 1), cutoff 6, T = 1/700 us, dt = T/100, FP64",
            "runs": runs, "five_modes": five}


def network_storage(hgf, torch, max_modes: int = 4):
    """The paper's memory comparison on the network example (Table I chain,
    operator prod_j a_j, w_q t / pi = 10 in 100 RK4 steps, cutoff 6, FP64):
    the conventional representation (one grid over all (k, l)) against the
    separated form G = Gx Gy + R of Eqs. (9a)-(9c) with R approximated on the
    diagonal k = l (the paper's approximation by a function of x_j y_j), both
    with the thresholded representation (coefficients with |g| <= threshold
    dropped after every step).  Per mode count and method: the operator error
    on the three lowest levels against the paper's reference recipe (the
    conventional method at cutoff 7 and half the step, untruncated), without
    truncation and at the largest threshold (from a geometric sweep) whose
    error stays within the common target max(100 ppm, 1.25 x the larger
    untruncated error); the peak number of coefficients kept (the stored
    elements of a sparse store) and the dense grid points, and the same at
    the granularity of tiles (the stage kernel's tile on the full grid, one
    grid of a monomial in the separated form); the wall time.
    The separated form with R on the whole box (exact) is also run untruncated
    up to three modes, and the separated form at cutoff 5 (untruncated, and
    thresholded where its untruncated error meets the target).  For one and
    two modes also the running peak against the simulated time (the paper's
    figure of stored elements against w_q t / pi)."""
    import synth

    def run(w, layout, thr):
        op = hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision="fp64", layout=layout)
        if thr > 0:
            hgf.set_threshold(op, thr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hgf.evolve(op, w.t_total, w.dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        info = op.info()
        return op, el, info

    out = []
    for n in range(1, max_modes + 1):
        w = synth.table1_network(n, 6)
        wr = synth.table1_network(n, 7)
        ref_op = hgf.map_operator(hgf.define_system(wr.system), factors=wr.factors, precision="fp64")
        hgf.evolve(ref_op, wr.t_total, wr.dt / 2)
        Mr = hgf.reconstruct(ref_op, 3)
        del ref_op

        def eps(op):
            M = hgf.reconstruct(op, 3)
            return float(np.linalg.norm(M - Mr) / np.linalg.norm(Mr))

        rec = {"modes": n, "cutoff": 6}
        base = {}
        for name, layout in (("conventional", "merged"), ("separated", "separated")):
            op, el, info = run(w, layout, 0.0)
            base[name] = {"eps_r_untruncated": eps(op), "dense_points": info["total_points"], "seconds": el,
                          "functions": info["n_functions"]}
            del op
        if n <= 3:
            op, el, info = run(w, "separated_exact", 0.0)
            rec["separated_exact"] = {"eps_r_untruncated": eps(op), "dense_points": info["total_points"],
                                      "seconds": el}
            del op
        target = max(1e-4, 1.25 * max(base["conventional"]["eps_r_untruncated"],
                                      base["separated"]["eps_r_untruncated"]))
        rec["eps_r_target"] = target
        def sweep(wl, layout):
            for k in range(0, 25):
                thr = 10.0 ** (-1.0 - 0.5 * k)
                op, el, info = run(wl, layout, thr)
                e = eps(op)
                del op
                if e <= target:
                    return {"threshold": thr, "eps_r": e, "stored_peak": info["stored_peak"], "seconds": el,
                            "stored_tiles_peak": info["stored_tiles_peak"], "tile_points": info["tile_points"],
                            "tiles": info["total_points"] // max(1, info["tile_points"])}
            return None

        for name, layout in (("conventional", "merged"), ("separated", "separated")):
            base[name]["truncated"] = sweep(w, layout)
            rec[name] = base[name]
        # the separated form one level lower (its truncation error at cutoff 6 is below the target)
        w5 = synth.table1_network(n, 5)
        op, el, info = run(w5, "separated", 0.0)
        e5 = eps(op)
        del op
        rec["separated_cutoff5"] = {"eps_r_untruncated": e5, "dense_points": info["total_points"], "seconds": el,
                                    "truncated": sweep(w5, "separated") if e5 <= target else None}
        if n <= 2:  # the running peak against the simulated time (w_q t / pi = 1 .. 10), at the chosen thresholds
            rec["peak_vs_time"] = {}
            for name, layout in (("conventional", "merged"), ("separated", "separated")):
                best = rec[name]["truncated"]
                if best is None:
                    continue
                op = hgf.map_operator(hgf.define_system(w.system), factors=w.factors, precision="fp64",
                                      layout=layout)
                hgf.set_threshold(op, best["threshold"])
                peaks = []
                for _ in range(10):
                    hgf.evolve(op, w.t_total / 10, w.dt)
                    peaks.append(op.info()["stored_peak"])
                rec["peak_vs_time"][name] = {"wq_t_over_pi": list(range(1, 11)), "stored_peak": peaks}
                del op
        out.append(rec)
        log(f"network storage {n} modes: conventional {rec['conventional']['truncated']}, "
            f"separated {rec['separated']['truncated']}, separated at cutoff 5 {rec['separated_cutoff5']}")
    return {"workload": "Table I network (chain, drive on mode 1), operator prod_j a_j, cutoff 6, "
                        "T = 1/700 us in 100 RK4 steps, FP64; reference: conventional at cutoff 7, half step",
            "runs": out}


def gradient_timing(hgf, torch, t_total: float):
    """hgf_grad on the 4-mode, cutoff-16 workload (bitstring projector,
    coherent state, 22 parameters, checkpoints every 100 steps)."""
    import synth
    w = synth.grad_c3()
    S = hgf.define_system(w.system)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    val, g = hgf.grad(S, w.states[0], t_total, w.dt, factors=w.factors, checkpoint_every=100)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    steps = int(round(t_total / w.dt))
    out = {"workload": f"4 Kerr modes, cutoff 16, bitstring projector, T = {t_total} us, dt = 0.1 ns",
           "steps": steps, "params": len(g), "seconds": el, "value": val.real,
           "max_abs_grad": float(np.max(np.abs(g)))}
    ref = golden("workloads")["gradient"]
    if steps == ref["steps"]:
        rv = complex(*ref["value"])
        rg = np.array([complex(*x) for x in ref["grad"]])
        out["rel_err_vs_oracle"] = {"value": abs(val - rv) / abs(rv),
                                    "grad": float(np.max(np.abs(g - rg)) / np.max(np.abs(rg)))}
    return out


def small_gradient_timing(hgf, torch):
    """hgf_grad on a small off-diagonal workload (4 Kerr modes, cutoff 5,
    product of quadratures: 16 sectors of 256 points; T = 0.02 us, dt = 0.01
    ns, 2,000 steps, checkpoints every 100): on chip (every sector within the
    resident integrator's size) and on the stage launches (HGF_RESIDENT=0),
    each with its errors against the stored oracle value and sensitivities."""
    import synth
    w = synth.grad_c3b(cutoff=5, t_total=0.02, dt=1e-5)
    ref = golden("small_gradient")
    rv = complex(*ref["value"])
    rg = np.array([complex(*x) for x in ref["grad"]])
    S = hgf.define_system(w.system)
    out = {"workload": f"{w.name}, 16 sectors of 256 points, T = 0.02 us, dt = 0.01 ns", "steps": w.n_steps,
           "params": len(rg)}
    prev = os.environ.get("HGF_RESIDENT")
    try:
        for name, res in (("on_chip", None), ("stage_launches", "0")):
            if res is None:
                os.environ.pop("HGF_RESIDENT", None)
            else:
                os.environ["HGF_RESIDENT"] = res
            hgf.grad(S, w.states[0], 10 * w.dt, w.dt, factors=w.factors, checkpoint_every=100)  # loads the kernels
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            val, g = hgf.grad(S, w.states[0], w.t_total, w.dt, factors=w.factors, checkpoint_every=100)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            out[name] = {"seconds": el, "us_per_step": el / w.n_steps * 1e6,
                         "rel_err_vs_oracle": {"value": abs(val - rv) / abs(rv),
                                               "grad": float(np.max(np.abs(g - rg)) / np.max(np.abs(rg)))}}
    finally:
        if prev is None:
            os.environ.pop("HGF_RESIDENT", None)
        else:
            os.environ["HGF_RESIDENT"] = prev
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64 and time-to-1e-5 comparisons")
    ap.add_argument("--no-full-horizon", action="store_true",
                    help="skip the full-horizon runs of the 10-mode workload (4e4 steps, mixed and FP64)")
    ap.add_argument("--tune-cache", default=None,
                    help="launch-shape cache file: shapes found there are applied without measuring")
    ap.add_argument("--only", choices=["network", "network5", "gradient", "storage", "batch", "axes"], default=None,
                    help="run one section alone and print its JSON (for profiling it): network = the Table I "
                         "network for 1 to 5 modes, network5 = its five-mode runs alone, gradient = the gradient "
                         "workload over 0.5 us (5,000 steps), storage = the conventional and separated "
                         "network forms with thresholds, batch = the batch workload over --steps steps, "
                         "axes = the stage kernel on grids of 10, 8, 7 and 5 axes")
    ap.add_argument("--complex-grids", action="store_true",
                    help="time the general complex form of the grid (real-grid form off) as the main run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (a function is never "
              "split; the functions of a batch would be placed whole on separate GPUs).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2203_05526_amd as hgf
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    hgf.load_library()
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 2.0, out=b)  # one elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        log("copy calibration: 5 elementwise passes reading and writing 1 GiB")
        del a, b
    if args.only == "axes":
        print(json.dumps({"axis_count": axis_count_comparison(hgf, torch)}))
        return
    if args.only == "batch":
        print(json.dumps({"batch": batch_throughput(hgf, torch, 0, steps=args.steps, tune_cache=args.tune_cache)}))
        return
    if args.only == "storage":
        print(json.dumps({"network_storage": network_storage(hgf, torch)}))
        return
    if args.only in ("network", "network5"):
        print(json.dumps({"network": network_timing(hgf, torch, five_only=args.only == "network5")}))
        return
    if args.only == "gradient":
        gradient_timing(hgf, torch, 0.01)  # first call: loads the kernels, captures the graphs
        print(json.dumps({"gradient": gradient_timing(hgf, torch, 0.5),
                          "gradient_small": small_gradient_timing(hgf, torch)}))
        return
    w = synth.large_c4()
    pts = int(np.prod(w.system.cutoff))
    S = hgf.define_system(w.system)

    def run(precision, steps, warmup, real_grids=True):
        tm = time.perf_counter()
        if not real_grids:
            os.environ["HGF_REAL_GRIDS"] = "0"  # the general complex form of the same grid
        try:
            op = hgf.map_operator(S, factors=w.factors, precision=precision)  # step (i): host build and upload
        finally:
            os.environ.pop("HGF_REAL_GRIDS", None)
        torch.cuda.synchronize()
        log(f"map_operator: {time.perf_counter() - tm:.3f} s")
        real = op.info()["real_functions"] == 1
        t0 = time.perf_counter()
        hgf.autotune([op], w.dt, cache=args.tune_cache)  # stage-kernel launch shape, measured on this GPU
        tune = dict(op.tile_config(0), seconds=time.perf_counter() - t0)
        log(f"autotuned shape {tune}")
        if warmup:
            hgf.evolve(op, warmup * w.dt, w.dt)
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record()
        hgf.evolve(op, steps * w.dt, w.dt)
        end.record()
        J = hgf.expectation(op, w.states[0])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        launch_s = start.elapsed_time(end) * 1e-3 / (4 * steps)
        del op
        return el, launch_s, J, real, tune

    log(f"timing {args.steps} steps ({args.precision}) over {pts} points")
    el, launch_s, J, real, tune = run(args.precision, args.steps, args.warmup, real_grids=not args.complex_grids)
    log(f"done: {el:.3f} s, stage launch {launch_s * 1e6:.1f} us")
    value = pts * 4 * args.steps / el
    bytes_launch = bytes_per_point_stage(args.precision, real) * pts
    achieved = bytes_launch / launch_s / 1e9
    traffic = stored_traffic(tune, real, args.precision)
    # the same operands streamed once per point with no neighbour reads
    ceil_us = hgf.stream_ceiling(args.precision, real, pts, 10)
    ceil_s = sum(ceil_us) / 4 * 1e-6
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "point-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ({"mixed": "f32 stencil, f64 state", "fp64": "f64"}[args.precision]
                  + (" (real grids: real generator and data on the diagonal sector)" if real else " (complex)")),
        "data": "synthetic (seeded parameters, no dataset)",
        "config": {"workload": "10 Kerr modes, cutoff 6 (6^10 grid points), parity-weighted projector, "
                               "dt = 0.05 ns, merged layout",
                   "precision": args.precision, "grid_points": pts, "seed": 4, "real_grids": real,
                   "tile_shape": tune},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": STAGE_KERNEL, "avg_launch_us": launch_s * 1e6,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     # the counted HBM bytes per launch over the launch time
                     "traffic_GBps": None if traffic is None else traffic / launch_s / 1e9,
                     # streaming ceiling: the stage operands read and written once per point
                     # (hgf_stream_ceiling), per stage and averaged; the kernel's time over it
                     "stream_ceiling": {"us_per_stage": ceil_us, "avg_launch_us": ceil_s * 1e6,
                                        "GBps": bytes_launch / ceil_s / 1e9,
                                        "kernel_time_over_ceiling": launch_s / ceil_s}},
        "expectation": [J.real, J.imag],
    }
    if not args.no_extras:
        log("fp64 comparison")
        n64 = max(10, args.steps // 4)
        el64, launch64, J64, real64, _ = run("fp64", n64, 2)
        line["fp64_plain"] = {"value": pts * 4 * n64 / el64, "steps": n64, "real_grids": real64,
                              "achieved_GBs": bytes_per_point_stage("fp64", real64) * pts / launch64 / 1e9}
        log("complex grid (real-grid form off)")
        line["complex_grid"] = {}
        # the same steps as the real-grid run of that precision, whose J it is compared with
        same = {args.precision: (args.steps, args.warmup, J), "fp64": (n64, 2, J64)}
        for prec in ("mixed", "fp64"):
            nc, wc, Jr = same.get(prec, (n64, 2, None))
            elc, launchc, Jc, realc, tunec = run(prec, nc, wc, real_grids=False)
            bc = bytes_per_point_stage(prec, realc) * pts
            line["complex_grid"][prec] = {
                "value": pts * 4 * nc / elc, "steps": nc, "real_grids": realc, "avg_launch_us": launchc * 1e6,
                "algorithmic_bytes_per_launch": bc, "achieved_GBs": bc / launchc / 1e9,
                "frac": bc / launchc / 1e9 / HBM_PEAK_GBS, "tile_shape": tunec,
                "rel_diff_from_real_grid_J": None if Jr is None else abs(Jc - Jr) / abs(Jr)}
        log("time-to-1e-5 on the 3-mode workload")
        line["time_to_1e-5"] = time_to_tolerance(hgf, torch)
        if not args.no_full_horizon:
            log("10-mode workload over the full horizon")
            line["time_to_1e-5"]["ten_mode"] = ten_mode_full_horizon(hgf, torch, w, S, args.tune_cache)
        log("batched evolve")
        line["batch"] = batch_throughput(hgf, torch, 500)
        log("gradient")
        line["gradient"] = gradient_timing(hgf, torch, 5.0)
        line["gradient_small"] = small_gradient_timing(hgf, torch)
        log("network")
        line["network"] = network_timing(hgf, torch)
        log("network storage (thresholded, conventional vs separated)")
        line["network"]["storage"] = network_storage(hgf, torch)
    if not args.no_cpu_baseline:
        log("cpu oracle baseline")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
