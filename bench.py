#!/usr/bin/env python
"""Benchmark of the amortized interval subdivision path on one MI355X.

One step = one full run of Algorithm 3 with the interval exclusion criterion
(Moroz, arXiv 2406.09857) on the two-surface curve workload: two random
trivariate polynomials of total degree 100 (N(0,1) coefficients, seed 3),
domain [-1,1]^3, levels 0..10.  Every level evaluates both polynomials on the
level's CSF (interval_eval_level), filters and bisects (filter_subdivide).
The inputs are resident in HBM before the timed region.

Prints one JSON line: throughput in interval box evaluations per second
(sum over levels and polynomials of |S_level|, divided by the step time),
the FP64 roofline of the dominant kernel (HIP events around each of its
launches in the last timed step), and the CPU oracle timed on a bounded
sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "interval box-evals/sec per level + % FP64-VALU peak; batched & adjoint vs plain"
# MI355X published FP64 vector peak (an FMA counts as two operations).
FP64_PEAK = 78.6e12
# FP64 VALU instruction issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz =
# 39.3e12 lane-instructions/s (every wave64 FP64 instruction, FMA and max
# alike, holds its SIMD for 4 clocks); the published 78.6 TFLOP/s is this rate
# with every instruction an FMA counted as two operations.
FP64_ISSUE_PEAK = 256 * 64 * 2.4e9
OPS_PER_STEP = 4      # algorithmic: the lower and upper multiply-add (product and sum) of one interval Horner step
EVAL_KERNELS = ("k_stage1", "k_narrow", "k_leaf")


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="curve", choices=["curve", "surface", "tiny"])
    ap.add_argument("--cpu-depth", type=int, default=9, help="oracle sample: levels 0..cpu-depth of the workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched, adjoint, variable-order, Taylor-test, early-exit, inclusion and Newton legs")
    ap.add_argument("--batched-eager", action="store_true",
                    help="only the batched workload: autotune, then one eager run with the chosen launch shapes "
                         "(for counter collection); prints its per-level counts and steps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (reference for the HBM byte counters)")
    return ap.parse_args()


def workload(name):
    from paper_2406_09857_amd import synth
    if name == "curve":
        return synth.curve(), "two trivariate polynomials, total degree 100, N(0,1) coefficients, domain [-1,1]^3, levels 0..10"
    if name == "surface":
        return synth.surface(), "one trivariate polynomial, total degree 40, N(0,1) coefficients, domain [-1,1]^3, levels 0..9"
    return synth.tiny(), "one bivariate polynomial, total degree 20, integer coefficients in [-100,100], domain [-1,1]^2, levels 0..8"


def cpu_baseline(w, depth):
    from oracle import core as orc
    nth = orc.max_threads()
    t0 = time.perf_counter()
    recs = orc.subdivide(w.polys, w.k, depth, dom=w.domain(), nthreads=nth)
    dt = time.perf_counter() - t0
    evals = sum(len(w.polys) * len(r["S"]["boxes"]) for r in recs)
    return {"value": evals / dt, "unit": "box-evals/s", "cores": nth, "kind": "oracle",
            "sample": f"oracle subdivision of the same workload, levels 0..{depth} ({evals} box evaluations, "
                      f"{dt:.2f} s, OpenMP over x1 fibres)"}


def _evt_ms(fn, reps=1):
    """Time `fn` on torch's current stream with HIP events (ms per call)."""
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def bench_batched(vx, reps):
    """64 independent systems (degrees 10..60, depth 8): one graph-replayed
    batched run against 64 sequential plain runs of the same systems."""
    import torch
    from paper_2406_09857_amd import synth
    w = synth.batch()
    dom = w.domain()
    b, r = vx.run_subdivision_batch(w.systems, dom, w.depth, graph=False)
    cap = [max(int(n), 1) for n in r["need"]]
    b.close()
    del b
    b = vx.Batch(w.systems, dom, w.depth, cap=cap, graph=True)
    chosen, _ = b.autotune(reps=1)
    b.run()
    torch.cuda.synchronize()
    ms = _evt_ms(b.run, reps)
    r = b.result(want_last=False, want_kept=False)
    b.close()
    del b
    evals = int(r["stats"][:, 0, 3].sum())
    steps = int(sum(r["steps"]))
    ws = torch.empty(6 << 30, dtype=torch.uint8, device="cuda")
    for sysp in w.systems[:4]:
        vx.run_subdivision(sysp, dom, w.depth, ws=ws, want_kept=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sysp in w.systems:
        vx.run_subdivision(sysp, dom, w.depth, ws=ws, want_kept=False)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3
    del ws
    return {"workload": f"{w.name}: {len(w.systems)} single-polynomial trivariate systems, degrees uniform in "
                        f"[10, 60], N(0,1) coefficients, domain [-1,1]^3, levels 0..{w.depth}",
            "ms_per_run": ms, "box_evals_per_s": evals / (ms * 1e-3), "interval_steps": steps,
            "fp64_flop_frac": OPS_PER_STEP * steps / (ms * 1e-3) / FP64_PEAK,
            "plain_64_runs_ms": plain_ms, "speedup_vs_plain": plain_ms / ms,
            "mode": "hipGraph replay, per-level autotuned launch shapes",
            "tune": chosen, "node_capacity": cap,
            "parity": "bit-identical to the plain runs (tests/test_gpu_batch.py)"}


def bench_adjoint(vx, polys, dom, depth, kept):
    """Point evaluation on the final kept-box centres: the forward on the CSF
    grid of centres (amortized) and per point, forward + hand-written backward
    (Jacobian, dF/dx and dF/dcoef on the grid), 3 Newton steps from the
    centres (the first evaluation on the grid, the later ones per point: the
    steps move the points off the grid), and the same steps all per point."""
    import torch
    csf = vx.CSF.from_arrays(3, depth, kept["idx"], kept["ptr"])
    x = vx.csf_centres(csf, dom)
    n = int(x.shape[0])
    gbar = torch.ones((len(polys), n), dtype=torch.float64, device="cuda")
    fwd = lambda: vx.eval_grad(polys, None, want_jac=False, grid=csf, dom=dom)
    fwd_jac = lambda: vx.eval_grad(polys, None, want_jac=True, grid=csf, dom=dom)
    fwd_pt = lambda: vx.eval_grad(polys, x, want_jac=False)
    fb = lambda: vx.eval_grad(polys, None, want_jac=True, gbar=gbar, want_xbar=True, want_dcoef=True, grid=csf,
                              dom=dom)
    fwd(); fwd_jac(); fwd_pt(); fb()
    torch.cuda.synchronize()
    f_ms = min(_evt_ms(fwd) for _ in range(3))
    fj_ms = min(_evt_ms(fwd_jac) for _ in range(3))
    fpt_ms = _evt_ms(fwd_pt)
    fb_ms = _evt_ms(fb)
    f0 = fwd()[0].abs().amax(dim=0)
    xp = x.clone()
    newton_pt_ms = _evt_ms(lambda: vx.newton_project(polys, xp, steps=3))
    xn = x.clone()
    newton_ms = _evt_ms(lambda: vx.newton_project(polys, xn, steps=3, grid=(csf, dom)))
    assert torch.equal(xn, xp)
    f3 = vx.eval_grad(polys, xn, want_jac=False)[0].abs().amax(dim=0)
    return {"points": n, "forward_ms": f_ms, "forward_with_jacobian_ms": fj_ms,
            "forward_per_point_ms": fpt_ms, "grid_speedup_vs_per_point": fpt_ms / f_ms,
            "forward_backward_ms": fb_ms, "backward_over_forward": fb_ms / fj_ms,
            "newton3_ms": newton_ms, "newton3_per_point_ms": newton_pt_ms,
            "median_residual_before": float(torch.median(f0)),
            "median_residual_after_3_newton": float(torch.median(f3)),
            "parity": "values bit-identical to the oracle and to the per-point path, Jacobian vs derivative "
                      "polynomials and central differences, dcoef vs long-double sums over the whole grid, "
                      "Newton vs CPU steps (tests/test_gpu_grad.py, tests/test_gpu_grad_fullsize.py)"}


def bench_mean_value(vx, polys, dom, depth, plain_stats, plain_ms):
    """The curve run with C0 and the mean-value test together against C0 alone."""
    import torch
    vx.run_subdivision(polys, dom, depth, want_kept=False, mean_value=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, _ = vx.run_subdivision(polys, dom, depth, want_kept=False, mean_value=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    return {"ms_per_run": ms, "plain_ms_per_run": plain_ms,
            "kept_per_level": [s["kept"][2] for s in stats],
            "plain_kept_per_level": [s["kept"][2] for s in plain_stats],
            "parity": "enclosures bit-identical to the oracle (tests/test_gpu_meanvalue.py)"}


def bench_taylor2(vx, polys, dom, depth, plain_stats, plain_ms, mv_stats):
    """The curve run with C0 and the order-2 Taylor test together, against C0
    alone and against C0 with the mean-value test."""
    import torch
    vx.run_subdivision(polys, dom, depth, want_kept=False, taylor2=True)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        stats, _ = vx.run_subdivision(polys, dom, depth, want_kept=False, taylor2=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    return {"ms_per_run": ms, "plain_ms_per_run": plain_ms,
            "kept_per_level": [s["kept"][2] for s in stats],
            "mean_value_kept_per_level": mv_stats,
            "plain_kept_per_level": [s["kept"][2] for s in plain_stats],
            "parity": "enclosures bit-identical to the oracle (tests/test_gpu_taylor2.py)"}


def bench_taylor_m(vx, polys, dom, depth, plain_stats, plain_ms, t2_stats, m=3):
    """The curve run with C0 and the Taylor test of order m >= 3 (the
    multinomial terms of orders below m at the centres, those of order m on
    the boxes), against C0 alone and against C0 with the order-2 test."""
    import torch
    vx.run_subdivision(polys, dom, depth, want_kept=False, taylor_order=m)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        stats, _ = vx.run_subdivision(polys, dom, depth, want_kept=False, taylor_order=m)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    return {"order": m, "ms_per_run": ms, "plain_ms_per_run": plain_ms,
            "kept_per_level": [s["kept"][2] for s in stats],
            "taylor2_kept_per_level": t2_stats,
            "plain_kept_per_level": [s["kept"][2] for s in plain_stats],
            "parity": "enclosures bit-identical to the oracle (tests/test_gpu_taylor_m.py)"}


def bench_early_exit(vx, polys, dom, depth, plain_stats, plain_ms):
    """Early exit for systems: each polynomial evaluated only on the boxes the
    earlier ones kept (same kept sets), on the curve and on the points system
    (three trivariate degree-20 polynomials, levels 0..9)."""
    import torch
    from paper_2406_09857_amd import synth

    def timed(ps, dm, dp, **kw):
        vx.run_subdivision(ps, dm, dp, want_kept=False, level_times=False, **kw)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            st, _ = vx.run_subdivision(ps, dm, dp, want_kept=False, level_times=False, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps, st

    out = {}
    for tag, kw in (("curve", {}), ("curve_from_level_9", {"early_exit_from": 9})):
        ms, st = timed(polys, dom, depth, early_exit=True, **kw)
        out[tag] = {"ms_per_run": ms, "plain_ms_per_run": plain_ms, "vs_plain": plain_ms / ms,
                    "steps": sum(s["steps"] for s in st), "plain_steps": sum(s["steps"] for s in plain_stats),
                    "same_kept_counts": [s["kept"] for s in st] == [s["kept"] for s in plain_stats]}
    w = synth.points()
    pp = vx.as_polys(w.polys)
    ms_p, st_p = timed(pp, w.domain(), w.depth)
    ms_e, st_e = timed(pp, w.domain(), w.depth, early_exit=True)
    out["points"] = {"workload": "points_k3_d20, levels 0..9", "ms_per_run": ms_e, "plain_ms_per_run": ms_p,
                     "vs_plain": ms_p / ms_e, "steps": sum(s["steps"] for s in st_e),
                     "plain_steps": sum(s["steps"] for s in st_p),
                     "same_kept_counts": [s["kept"] for s in st_e] == [s["kept"] for s in st_p]}
    out["parity"] = "kept sets equal to the oracle's, steps equal to Theorem 1 on the survivors (tests/test_gpu_early_exit.py)"
    return out


def bench_order(vx, polys, kept):
    """Theorem 1's cost of the curve's final kept set (level 10) under each of
    the six orders of the variables, from CSFs built on the device."""
    import torch
    K = vx.CSF.from_arrays(kept["k"], kept["level"], kept["idx"], kept["ptr"])
    vx.variable_order_costs(polys, K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    costs = vx.variable_order_costs(polys, K)
    ms = (time.perf_counter() - t0) * 1e3
    return {"boxes": int(K.nboxes), "ms_all_orders": ms,
            "orders": [{"order": list(o), "N": c, "steps": st} for o, c, st in costs],
            "cheapest": list(min(costs, key=lambda c: c[2])[0]),
            "parity": "node counts and steps equal to the oracle's (tests/test_gpu_order.py)"}


def bench_inclusion(vx):
    """The inclusion criterion C1 on the surface's final kept set (levels 0..9
    of one trivariate degree-40 polynomial): certified boxes and time."""
    import torch
    from paper_2406_09857_amd import synth
    w = synth.surface()
    dom = w.domain()
    _, kept = vx.run_subdivision(w.polys, dom, w.depth)
    K = vx.CSF.from_arrays(3, w.depth, kept["idx"], kept["ptr"])
    out = {"workload": "surface_k3_d40: one trivariate polynomial, total degree 40, N(0,1) coefficients, "
                       "domain [-1,1]^3, kept boxes of level 9",
           "boxes": K.nboxes,
           "parity": "flags equal to the oracle's (tests/test_gpu_inclusion.py)"}
    for name, taylor in (("vertices", False), ("taylor2", True)):
        vx.inclusion_test(w.polys, K, dom, taylor=taylor)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            incl = vx.inclusion_test(w.polys, K, dom, taylor=taylor)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        out[name] = {"certified": int(incl.sum()), "ms": ms, "boxes_per_s": K.nboxes / (ms * 1e-3)}
    # Algorithm 3 with both criteria: C1 from level 7 on (boxes narrower than
    # 2^-5 on [-1,1]), certified boxes leave the loop
    plain_ms = None
    for name in ("plain", "vertices", "taylor"):
        kw = {} if name == "plain" else {"inclusion": name, "inclusion_from": 7}
        vx.run_subdivision(w.polys, dom, w.depth, want_kept=False, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, _ = vx.run_subdivision(w.polys, dom, w.depth, want_kept=False, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if name == "plain":
            plain_ms = ms
            out["loop_plain"] = {"ms_per_run": ms, "kept_last_level": stats[-1]["kept"][2]}
        else:
            out["loop_c1_" + name] = {"ms_per_run": ms, "c1_from_level": 7,
                                      "certified_per_level": [s["certified"] for s in stats],
                                      "continuing_last_level": stats[-1]["kept"][2],
                                      "vs_plain": ms / plain_ms}
    return out


def bench_newton(vx):
    """The Newton interval test on the final kept set of the points workload
    (three trivariate polynomials of degree 20, levels 0..9)."""
    import torch
    from paper_2406_09857_amd import synth
    w = synth.points()
    dom = w.domain()
    t0 = time.perf_counter()
    _, kept = vx.run_subdivision(w.polys, dom, w.depth, want_kept=True)
    torch.cuda.synchronize()
    run_ms = (time.perf_counter() - t0) * 1e3
    K = vx.CSF.from_arrays(3, w.depth, kept["idx"], kept["ptr"])
    vx.newton_test(w.polys, K, dom)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        incl = vx.newton_test(w.polys, K, dom)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    out = {"workload": "points_k3_d20: three trivariate polynomials, total degree 20, coefficients uniform in "
                       "[-10, 10], domain [-1,1]^3, kept boxes of level 9",
           "run_ms_with_kept_copy": run_ms, "boxes": K.nboxes, "certified": int(incl.sum()), "ms": ms,
           "parity": "flags and Krawczyk enclosures equal to the oracle's (tests/test_gpu_newton.py)"}
    # Algorithm 3 with C1 = the Newton test from level 6 on
    for name, kw in (("loop_plain", {}), ("loop_newton", {"inclusion": "vertices", "inclusion_from": 6})):
        vx.run_subdivision(w.polys, dom, w.depth, want_kept=False, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, _ = vx.run_subdivision(w.polys, dom, w.depth, want_kept=False, **kw)
        torch.cuda.synchronize()
        out[name] = {"ms_per_run": (time.perf_counter() - t0) * 1e3,
                     "certified_per_level": [s_["certified"] for s_ in stats],
                     "continuing_last_level": stats[-1]["kept"][2]}
    # fewer equations than variables: the circle of a sphere and a plane,
    # C1 = the Newton test on the span of the gradients from level 5 on
    c1 = synth.monomial_poly(3, 2, {(2, 0, 0): 1.0, (0, 2, 0): 1.0, (0, 0, 2): 1.0, (0, 0, 0): -0.5})
    c2 = synth.monomial_poly(3, 1, {(0, 0, 1): 1.0, (0, 0, 0): -0.3})
    cdom = [-1.0, 1.0] * 3
    span = {"workload": "circle_k3: x^2 + y^2 + z^2 = 0.5 and z = 0.3 (two equations, three variables), "
                        "domain [-1,1]^3, levels 0..9"}
    for name, kw in (("loop_plain", {}), ("loop_newton_span", {"inclusion": "vertices", "inclusion_from": 5})):
        vx.run_subdivision([c1, c2], cdom, 9, want_kept=False, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, _ = vx.run_subdivision([c1, c2], cdom, 9, want_kept=False, **kw)
        torch.cuda.synchronize()
        span[name] = {"ms_per_run": (time.perf_counter() - t0) * 1e3,
                      "certified_per_level": [s_["certified"] for s_ in stats],
                      "continuing_last_level": stats[-1]["kept"][2]}
    span["parity"] = "flags, K and the loop's sets equal to the oracle's (tests/test_gpu_newton.py)"
    out["span"] = span
    return out


COPY_BYTES = 1 << 31  # bytes read (and written) by the calibration copy


def copy_calibration():
    """One elementwise copy of COPY_BYTES: its FETCH_SIZE / WRITE_SIZE
    readings convert the counters of the measured kernels to bytes."""
    import torch
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES}))


# The sources compiled into the evaluation kernels (eval.hip and what it includes).
EVAL_SOURCES = ("eval.hip", "eval.hpp", "batch.inc", "common.hpp", "fill.hpp", "interval.hpp", "profile.hpp",
                "scan.hpp", "xcd.hpp")


def source_digest() -> str:
    """Digest of the evaluation kernels' sources: a counter or traffic figure
    measured on other sources is stale."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2406_09857_amd", "csrc")
    for name in sorted(EVAL_SOURCES):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def _profile_fields(path: str):
    """key: value lines of a committed counter summary, or None when it is
    missing or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != source_digest():
        return None
    return fields


def measured_inst_per_step(workload: str):
    """VALU instructions (all of them: the FP64 products, sums and max of the
    interval steps and everything else the kernels issue) per interval step
    of each evaluation kernel and over all three, counted by rocprofv3
    (SQ_INSTS_VALU, one count per wave instruction, times 64 lanes) and
    divided by Theorem 1's steps of the counted launches; from the committed
    summary profiles/eval_kernels_<workload>_counters.txt, or None when it is
    missing or was taken on other sources."""
    f = _profile_fields(os.path.join(ROOT, "profiles", f"eval_kernels_{workload}_counters.txt"))
    if f is None:
        return None
    out = {}
    for name in EVAL_KERNELS + ("all",):
        try:
            out[name] = float(f[f"{name}.valu_inst_per_step"])
        except (KeyError, ValueError):
            return None
    return out


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/<kernel>_<workload>_traffic.txt), or None when there is none
    or the kernel sources changed since it was taken."""
    fields = _profile_fields(os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt"))
    if fields is None:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def batched_eager():
    """The batched workload run once eagerly (no graph) with autotuned launch
    shapes, so that a counter collector sees each level's kernels."""
    import torch
    from paper_2406_09857_amd import binding as vx, synth
    w = synth.batch()
    dom = w.domain()
    b, r = vx.run_subdivision_batch(w.systems, dom, w.depth, graph=False)
    cap = [max(int(n), 1) for n in r["need"]]
    chosen, level_ms = b.autotune(reps=1)
    b.close()
    del b
    e = vx.Batch(w.systems, dom, w.depth, cap=cap, tune=chosen, graph=False)
    e.run()
    r = e.result(want_last=False, want_kept=False)
    torch.cuda.synchronize()
    print(json.dumps({"workload": w.name, "tune": chosen, "level_ms": level_ms,
                      "n": r["stats"][:, 0, : w.k + 1].tolist(), "steps_depth": r["steps_depth"].tolist()}))


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.batched_eager:
        batched_eager()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding by x1 fibres over several GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)
    w, desc = workload(args.workload)
    # The CPU baseline runs first, before this process touches the GPU, so
    # that no runtime thread of the GPU legs shares the host cores with it.
    cpu = cpu_baseline(w, min(args.cpu_depth, w.depth)) if not args.no_cpu_baseline else None

    import torch
    from paper_2406_09857_amd import binding as vx

    polys = vx.as_polys(w.polys)
    dom = w.domain()
    ws = torch.empty(6 << 30, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        vx.run_subdivision(polys, dom, w.depth, ws=ws, want_kept=False, level_times=False)
    torch.cuda.synchronize()
    # Every kernel timed over one untimed step (event records between all
    # launches slow the level loop down); it picks the dominant kernel, whose
    # launches alone are then timed with events inside the timed region.
    prof_all, dom_name = {}, None
    if not args.no_profile:
        vx.profile_begin()
        vx.run_subdivision(polys, dom, w.depth, ws=ws, want_kept=False)
        prof_all = vx.profile_end()
        evk = {n: r for n, r in prof_all.items() if n.startswith("k_") and r["ms"] > 0}
        dom_name = max(evk, key=lambda n: evk[n]["ms"]) if evk else None
    torch.cuda.synchronize()
    # The timed steps record no per-level events (each one is a packet the
    # stream passes between kernels); one more run, untimed, records them for
    # the per-level table.  The dominant kernel's launches are event-timed in
    # the last timed step (its launches repeat every step; events around the
    # launches of every step slow each step by about 1 %).
    t0 = time.perf_counter()
    for i in range(args.steps):
        if dom_name and i == args.steps - 1:
            vx.profile_begin(only=dom_name)
        vx.run_subdivision(polys, dom, w.depth, ws=ws, want_kept=False, level_times=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = vx.profile_end() if dom_name else {}
    ms_step = (t1 - t0) * 1e3 / args.steps
    stats, _ = vx.run_subdivision(polys, dom, w.depth, ws=ws, want_kept=False)
    torch.cuda.synchronize()

    evals = sum(len(polys) * s["n"][w.k - 1] for s in stats)
    steps_total = sum(s["steps"] for s in stats)
    eval_ms = sum(s["eval_ms"] for s in stats)
    ips = measured_inst_per_step(args.workload)  # counted FP64 instructions per step, or None

    def fracs(steps, ms, inst=None):
        """Algorithmic FP64 FLOP rate over the published peak, and (with a
        counted instruction rate) the FP64 VALU issue fraction."""
        if ms <= 0:
            return None, None
        flop = OPS_PER_STEP * steps / (ms * 1e-3) / FP64_PEAK
        issue = inst * steps / (ms * 1e-3) / FP64_ISSUE_PEAK if inst else None
        return flop, issue

    levels = []
    for s in stats:
        fl, iss = fracs(s["steps"], s["eval_ms"], ips["all"] if ips else None)
        levels.append({"level": s["level"], "boxes": s["n"][w.k - 1], "N": s["n"], "kept": s["kept"][w.k - 1],
                       "eval_ms": round(s["eval_ms"], 4), "filter_ms": round(s["filter_ms"], 4),
                       "box_evals_per_s": (len(polys) * s["n"][w.k - 1] / (s["eval_ms"] * 1e-3))
                       if s["eval_ms"] > 0 else None,
                       "fp64_flop_frac": fl, "fp64_issue_frac": iss})

    roof = None
    kernels = {}
    for name, r in prof_all.items():
        if r["ms"] <= 0:
            continue
        kernels[name] = {"launches": r["launches"], "avg_ms": r["ms"] / r["launches"], "total_ms": r["ms"],
                         "units_per_launch": r["units"] / r["launches"]}
    if dom_name and prof.get(dom_name, {}).get("ms", 0) > 0:
        r = prof[dom_name]
        avg_s = r["ms"] * 1e-3 / r["launches"]
        steps_per_launch = r["units"] / r["launches"]
        ops_per_launch = OPS_PER_STEP * steps_per_launch
        achieved = ops_per_launch / avg_s / 1e12
        inst = ips.get(dom_name) if ips else None
        roof = {"bound": "alu", "kernel": dom_name, "achieved": achieved, "peak": FP64_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": achieved / (FP64_PEAK / 1e12),
                "traffic": measured_traffic(dom_name, args.workload),
                "avg_launch_ms": avg_s * 1e3, "ops_per_launch": ops_per_launch,
                "steps_per_launch": steps_per_launch,
                "issue": {"note": "VALU instruction issue (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: a wave64 "
                                  "FP64 instruction, FMA or max, every 4 clocks per SIMD); VALU instructions per "
                                  "step counted by rocprofv3 "
                                  f"(profiles/eval_kernels_{args.workload}_counters.txt), null if that "
                                  "summary is missing or was taken on other sources",
                          "peak_lane_inst_per_s": FP64_ISSUE_PEAK,
                          "algorithmic_ops_frac": ops_per_launch / avg_s / FP64_ISSUE_PEAK,
                          "valu_inst_per_step": inst,
                          "valu_inst_frac": inst * steps_per_launch / avg_s / FP64_ISSUE_PEAK if inst else None}}

    out = {
        "metric": METRIC,
        "value": evals / (ms_step * 1e-3),
        "unit": "box-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {desc}", "polynomials": len(polys), "depth": w.depth,
                   "box_evals_per_step": evals, "interval_steps_per_step": steps_total},
        "eval_only": {"box_evals_per_s": evals / (eval_ms * 1e-3) if eval_ms > 0 else None,
                      "fp64_flop_frac": fracs(steps_total, eval_ms)[0],
                      "fp64_issue_frac": fracs(steps_total, eval_ms, ips["all"] if ips else None)[1],
                      "ms": eval_ms},
        "roofline": roof,
        "kernels_note": "every kernel, HIP-event timed over one untimed step before the timed region",
        "kernels": kernels,
        "levels_note": "per-level eval/filter times from one untimed run with level timing events; "
                       "the timed steps record none",
        "levels": levels,
    }
    if not args.no_extras and args.workload == "curve":
        del ws
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(vx, reps=5)
        _, kept = vx.run_subdivision(polys, dom, w.depth, want_kept=True)
        out["adjoint"] = bench_adjoint(vx, polys, dom, w.depth, kept)
        out["variable_order"] = bench_order(vx, polys, kept)
        out["mean_value"] = bench_mean_value(vx, polys, dom, w.depth, stats, ms_step)
        out["taylor2"] = bench_taylor2(vx, polys, dom, w.depth, stats, ms_step,
                                       out["mean_value"]["kept_per_level"])
        out["taylor3"] = bench_taylor_m(vx, polys, dom, w.depth, stats, ms_step,
                                        out["taylor2"]["kept_per_level"], m=3)
        out["early_exit"] = bench_early_exit(vx, polys, dom, w.depth, stats, ms_step)
        out["inclusion"] = bench_inclusion(vx)
        out["newton"] = bench_newton(vx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
