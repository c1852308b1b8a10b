#!/usr/bin/env python3
"""Time-to-solve and H2 matvec bandwidth of the isogeometric single-layer BEM on one MI355X.

Workload (the metric's configuration): interior Laplace Dirichlet problem on the unit sphere given
as 6 exact rational NURBS patches, spline degree p=3, 32x32 elements per patch (m=5; dim S = 7,350,
dim S* = 98,304), H2 compression with q=8 Chebyshev nodes per parametric direction and eta=1.6,
Gauss order 6; Dirichlet data from 4 seeded exterior point charges; Jacobi-preconditioned GMRES(100) to
true relative residual 1e-8; potential at 100 seeded interior points.

One step = operator assembly (Bezier extraction, partition, near-field quadrature, coupling blocks,
Jacobi diagonal) + right-hand side + solve + potential: the whole hot path once.  Inputs (the NURBS
control nets, 24 KB) are host data handed to the library; everything after that runs on the GPU.

Prints one JSON line.  Extra keys: h2_matvec_GBps (algorithmic bytes of one matvec / median time of
igb_matvec), per-stage matvec times, roofline of the dominant matvec kernel, and the CPU oracle
baseline projected from a timed sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-solve (rel res 1e-8) + H2 matvec GB/s; mixed/learned vs plain FP64"
HBM_PEAK_GBPS = 8000.0
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s
FP64_VECTOR_PEAK_TFLOPS = 78.6
# flop model of one Laplace kernel evaluation in the far field: 3 differences, 5 for |d|^2,
# 2 for the reciprocal square root, 2 for the accumulation
FLOP_PER_EVAL_LAPLACE = 12
# one evaluation applied both ways (mirrored blocks): 3 differences, 5 for |d|^2,
# 2 for the reciprocal square root, 4 for the two accumulations
FLOP_PER_EVAL_SYM = 14
WORKLOAD = "laplace_sphere_p3_m5_q8"
PRM = dict(p=3, m=5, q=8, eta=1.6, gauss_regular=6)
MODES = {"onthefly": 2, "stored": 1}
TOL = 1e-8
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1708_09162_amd", "csrc", "igabem.hip")


def source_sha() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def read_traffic(stage: str):
    """HBM bytes per launch of a kernel from committed rocprofv3 counter summaries, or None when
    missing or taken on a different kernel source."""
    path = os.path.join(PROFILE_DIR, f"{stage}_{WORKLOAD}_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for ln in fh:
            if ":" in ln and not ln.startswith("#"):
                k, v = ln.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != source_sha():
        return None
    try:
        fetch = float(vals["FETCH_SIZE_KiB_per_dispatch"]) * float(vals.get("fetch_scale", "1.0"))
        write = float(vals["WRITE_SIZE_KiB_per_dispatch"]) * float(vals.get("write_scale", "1.0"))
        return int(round((fetch + write) * 1024.0))
    except (KeyError, ValueError):
        return None


def calibrate_copy():
    """A plain device copy of known size (1 GiB read + 1 GiB written per launch) for scaling
    the HBM byte counters."""
    import torch

    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 5}), flush=True)


def charge_field(torch, pts, pos, q):
    g = torch.zeros(pts.shape[0], dtype=torch.float64, device=pts.device)
    for x0, c in zip(pos, q):
        d = torch.linalg.norm(pts - torch.tensor(x0, dtype=torch.float64, device=pts.device), dim=1)
        g += float(c) / (4.0 * math.pi * d)
    return g


RESTART = 100


def one_step(torch, igb, geo, cfg, ev_dev, mode, far_precision=0, solver="gmres"):
    """The whole path once; returns (operator, density, solve info, potential, timings).  solver "gmres":
    Jacobi-preconditioned GMRES(100) (igb_solve_fgmres without a network); "cg": Jacobi CG (igb_solve)."""
    t = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = igb.Operator(geo, device="cuda:0", mode=MODES[mode], far_precision=far_precision, **PRM)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pts = op.rhs_points()
    b = op.rhs(charge_field(torch, pts, *cfg["charges"]))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if solver == "gmres":
        w, info = op.solve_fgmres(b, None, tol=TOL, max_iter=20000, restart=RESTART)
    else:
        w, info = op.solve(b, tol=TOL, max_iter=20000)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    u = op.potential(w, ev_dev)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    t.update(assembly_s=t1 - t0, rhs_s=t2 - t1, solve_s=t3 - t2, potential_s=t4 - t3, total_s=t4 - t0)
    return op, w, info, u, t


def mixed_leg(torch, igb, geo, cfg, ev_dev, fp64_ms, exact, steps: int = 2):
    """The same step with the single-precision far field (far_precision IGB_FP32) and CG refined to the FP64
    tolerance with FP64 residuals: time-to-solve beside the plain FP64 CG step and the headline step."""
    def timed(fp, solver):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = one_step(torch, igb, geo, cfg, ev_dev, "onthefly", fp, solver)
            if _ + 1 < steps:
                del res
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / steps, res

    one_step(torch, igb, geo, cfg, ev_dev, "onthefly", 0, "cg")  # warmup
    cg_ms, (op, w, info_cg, u, t) = timed(0, "cg")
    del op
    op, w, info, u, t = one_step(torch, igb, geo, cfg, ev_dev, "onthefly", igb.IGB_FP32, "cg")  # warmup
    del op
    ms, (op, w, info, u, t) = timed(igb.IGB_FP32, "cg")
    st = op.profile(reps=20)
    print(f"[bench] single-precision far field: {ms / 1e3:.4f} s per step, {info.iterations} it", file=sys.stderr,
          flush=True)
    return {"far_precision": "fp32 (kernel values from the hardware reciprocal square root, FP64 sums)",
            "solver": "jacobi_cg_reliable_updates",
            "value": round(ms / 1e3, 5), "ms_per_step": round(ms, 3), "vs_fp64_cg": round(ms / cg_ms, 4),
            "fp64_cg_ms_per_step": round(cg_ms, 3), "fp64_cg_iterations": int(info_cg.iterations),
            "vs_fp64": round(ms / fp64_ms, 4),
            "iterations": int(info.iterations), "rel_residual": float(info.rel_residual),
            "potential_max_err": float(np.abs(u.cpu().numpy() - exact).max()),
            "breakdown_s": {k: round(v, 4) for k, v in t.items()},
            "coupling_ms": round(st["coupling"], 4)}


def learned_leg(torch, igb, epochs: int = 4, seeds=(5, 6, 7, 8)):
    """The learned preconditioner on its own workload: Laplace on the perturbed sphere (p=2, 128x128 elements
    per patch, q=8), 2000 seeded training vectors, the linear network trained on the GPU (loss on x) from four
    seeded initial weights, each then used in flexible GMRES to 1e-8 (at most 300 steps), beside the plain FP64
    solve (Jacobi CG) and Jacobi FGMRES, all from w = 0.  Every seed is reported: the network's effect depends
    on its initial weights.  "selected": the seed with the fewest steps on a validation right-hand side (other
    point charges), or Jacobi when none beats it there, then timed on the real right-hand side."""
    from paper_1708_09162_amd import workloads as W

    c5 = W.config_learned_preconditioner()
    prm = dict(p=c5["p"], m=c5["m"], q=c5["q"], eta=c5["eta"], gauss_regular=c5["gauss_regular"])
    geo = igb.Geometry(c5["patches"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = igb.Operator(geo, device="cuda:0", mode=igb.IGB_H2_ONTHEFLY, **prm)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    b = op.rhs(charge_field(torch, op.rhs_points(), *W.point_charges(*c5["charges"])))
    npatch, side = op.grid
    res = {"workload": c5["name"], "n_dof": int(op.info.n_dof), "n_pairs": c5["n_pairs"], "epochs": epochs,
           "activation": "linear", "assembly_s": round(t_asm, 3)}

    def timed_solve(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        w, info = fn()
        torch.cuda.synchronize()
        return w, info, time.perf_counter() - t

    _, i_cg, t_cg = timed_solve(lambda: op.solve(b, tol=TOL, max_iter=20000))
    _, i_j, t_j = timed_solve(lambda: op.solve_fgmres(b, None, tol=TOL, max_iter=5000, restart=100))
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(c5["pair_seed"])
    x = torch.randn((c5["n_pairs"], op.info.n_dof), dtype=torch.float64, device="cuda:0", generator=gen)
    torch.cuda.synchronize()
    t = time.perf_counter()
    y32, x32 = op.training_pairs(x)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t
    del x
    # validation right-hand side: other point charges (seed 3), used only to choose among the seeds
    b_val = op.rhs(charge_field(torch, op.rhs_points(), *W.point_charges(4, 3)))
    _, iv_j, _ = timed_solve(lambda: op.solve_fgmres(b_val, None, tol=TOL, max_iter=300, restart=100))
    runs, nets = [], {}
    for seed in seeds:
        net = igb.CNN(W.cnn_initial_weights(seed), igb.IGB_CNN_LINEAR, device="cuda:0")
        torch.cuda.synchronize()
        t = time.perf_counter()
        losses = net.train(y32, x32, npatch, side, side, epochs=epochs, batch=16, lr=1e-3)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t
        _, i_v, _ = timed_solve(lambda: op.solve_fgmres(b_val, net, tol=TOL, max_iter=300, restart=100))
        w, i_n, t_n = timed_solve(lambda: op.solve_fgmres(b, net, tol=TOL, max_iter=300, restart=100))
        r = b - op.matvec(w)
        runs.append({"init_seed": seed, "train_s": round(t_train, 3),
                     "loss_per_epoch": [round(float(v), 5) for v in losses],
                     "validation_iterations": int(i_v.iterations) if i_v.converged else None,
                     "iterations": int(i_n.iterations), "converged": int(i_n.converged), "solve_s": round(t_n, 4),
                     "true_rel_residual": float(torch.linalg.norm(r) / torch.linalg.norm(b))})
        nets[seed] = net
    conv = [rr for rr in runs if rr["converged"]]
    # selection on the validation right-hand side alone; Jacobi when no seed beats it there
    cand = [rr for rr in runs if rr["validation_iterations"] is not None
            and rr["validation_iterations"] < iv_j.iterations]
    chosen = min(cand, key=lambda rr: rr["validation_iterations"]) if cand else None
    sel_net = nets[chosen["init_seed"]] if chosen else None
    w, i_s, t_s = timed_solve(lambda: op.solve_fgmres(b, sel_net, tol=TOL, max_iter=5000, restart=100))
    res["selected"] = {"preconditioner": f"network seed {chosen['init_seed']}" if chosen else "jacobi",
                       "validation_iterations_jacobi": int(iv_j.iterations),
                       "iterations": int(i_s.iterations), "converged": int(i_s.converged), "solve_s": round(t_s, 4),
                       "solve_vs_plain_fp64": round(t_s / t_cg, 4),
                       "train_s_all_seeds": round(sum(rr["train_s"] for rr in runs), 3)}
    del nets, sel_net
    res.update({
        "plain_fp64_cg": {"iterations": int(i_cg.iterations), "solve_s": round(t_cg, 4)},
        "jacobi_fgmres": {"iterations": int(i_j.iterations), "solve_s": round(t_j, 4)},
        "network_fgmres_per_seed": runs,
        "network_converged_within_300": f"{len(conv)}/{len(runs)}",
        "network_median_iterations": float(np.median([rr["iterations"] for rr in runs])),
        "network_best_solve_vs_plain_fp64": round(min(rr["solve_s"] for rr in conv) / t_cg, 4) if conv else None,
        "pairs_s": round(t_pairs, 3),
    })
    print(f"[bench] learned preconditioner: CG {i_cg.iterations} it {t_cg:.3f} s, Jacobi FGMRES {i_j.iterations} it "
          f"{t_j:.3f} s, network FGMRES per seed {[(rr['iterations'], rr['converged']) for rr in runs]}, "
          f"selected {res['selected']['preconditioner']}: {i_s.iterations} it {t_s:.3f} s", file=sys.stderr, flush=True)
    return res


def batched_leg(torch, igb, n: int = 128, max_iter: int = 3000, restart: int = 1000):
    """Many independent instances (sphere/torus, m 2-5, p 1-3, Laplace or Helmholtz, one right-hand side each),
    every operator on its own stream: one-at-a-time solves against igb_solve_many (solves overlapping on the
    GPU), same tolerance and step limit (GMRES restart 1000 for Helmholtz: shorter cycles stall at high kappa)."""
    from paper_1708_09162_amd import workloads as W

    cfg = W.config_batched(n)
    inst = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, d in enumerate(cfg):
        patches = W.torus_patches() if d["geometry"] == "torus" else W.sphere_patches()
        op = igb.Operator(igb.Geometry(patches), mode=igb.IGB_H2_ONTHEFLY, kernel=d["kernel"],
                          wavenumber=d["wavenumber"], p=d["p"], m=d["m"], q=d["q"], eta=d["eta"],
                          gauss_regular=d["gauss_regular"], device="cuda:0", stream=torch.cuda.Stream())
        pts = op.rhs_points()
        torch.cuda.synchronize()
        pn = pts.cpu().numpy()
        g = (W.helmholtz_point_source(pn, d["source"], d["wavenumber"]) if d["kernel"] == 1
             else W.laplace_charge_field(pn, *d["charges"]))
        inst.append((op, op.rhs(torch.tensor(g, device="cuda:0"))))
        torch.cuda.synchronize()
        if i % 32 == 31:
            print(f"[bench] batched: {i + 1} instances assembled", file=sys.stderr, flush=True)
    t_asm = time.perf_counter() - t0
    t0 = time.perf_counter()
    seq = [op.solve(b, tol=TOL, max_iter=max_iter, restart=restart)[1] for op, b in inst]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    print(f"[bench] batched: one-at-a-time solves {t_seq:.2f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    _, infos = igb.solve_many([op for op, _ in inst], [b for _, b in inst], tol=TOL, max_iter=max_iter,
                              restart=restart)
    torch.cuda.synchronize()
    t_many = time.perf_counter() - t0
    print(f"[bench] batched: solve_many {t_many:.2f} s", file=sys.stderr, flush=True)
    return {"instances": n, "max_iter": max_iter, "restart": restart, "assembly_s": round(t_asm, 3),
            "sequential_solve_s": round(t_seq, 3), "solve_many_s": round(t_many, 3),
            "speedup": round(t_seq / t_many, 3), "instances_per_s": round(n / t_many, 2),
            "converged": f"{sum(i.converged for i in infos)}/{n}",
            "converged_one_at_a_time": f"{sum(i.converged for i in seq)}/{n}",
            "total_dofs": int(sum(op.info.n_dof for op, _ in inst))}


def cpu_baseline(cfg, iterations: int, seed: int = 7):
    """Oracle time-to-solve projected from a timed stratified sample of the same workload:
    near-field pair quadrature (per class) and coupling-block evaluation (the oracle evaluates
    coupling blocks inside every matvec)."""
    import oracle

    P = oracle.Problem(cfg["patches"], **PRM)
    threads = oracle.num_threads()
    classes = P.near_pair_classes()
    _, far = P.partition()
    rng = np.random.default_rng(seed)
    t_asm, parts = 0.0, []
    for c in range(4):
        rows = classes[classes[:, 2] == c]
        k = max(32, len(rows) // 100)
        pick = rows[rng.choice(len(rows), min(k, len(rows)), replace=False)]
        t0 = time.perf_counter()
        P.pair_blocks(pick[:, :2])
        dt = time.perf_counter() - t0
        t_asm += dt / len(pick) * len(rows)
        parts.append(f"{len(pick)}/{len(rows)} class-{c} pairs")
    kf = max(200, len(far) // 100)
    pick = far[rng.choice(len(far), min(kf, len(far)), replace=False)]
    t0 = time.perf_counter()
    P.coupling_blocks(pick)
    dt = time.perf_counter() - t0
    t_far = dt / len(pick) * len(far)
    parts.append(f"{len(pick)}/{len(far)} coupling blocks")
    value = t_asm + (iterations + 2) * t_far
    return {"value": value, "unit": "s", "cores": threads, "kind": "oracle",
            "sample": "projected from a timed random sample of the full workload: " + ", ".join(parts)
                      + f"; time = near quadrature + (solver iterations + 2) x coupling evaluation per matvec",
            "assembly_s": t_asm, "matvec_s": t_far}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--matvec-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=sorted(MODES), default="onthefly",
                    help="far field: coupling blocks generated in every matvec (default) or stored in HBM")
    ap.add_argument("--calibrate-copy", action="store_true", help="only run a plain 1 GiB device copy")
    ap.add_argument("--no-mixed", action="store_true", help="skip the single-precision far-field leg")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner leg")
    ap.add_argument("--batched", action="store_true",
                    help="also run the 128-instance batched-solve leg (about 90 s)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the whole path runs on one GPU; multi-GPU runs (--gpus > 1) are not supported. "
              "The path would shard by target clusters, with one all-gather of cluster moments per product.",
              file=sys.stderr, flush=True)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import torch

    from paper_1708_09162_amd import igabem as igb
    from paper_1708_09162_amd import workloads as W

    cfg = W.config_sphere_h2()
    geo = igb.Geometry(cfg["patches"])
    ev = cfg["eval_points"]
    ev_dev = torch.tensor(ev, dtype=torch.float64, device="cuda:0")
    print(f"[bench] workload {WORKLOAD}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    op = None
    for i in range(args.warmup):
        if op is not None:
            del op
        op, w, info, u, t = one_step(torch, igb, geo, cfg, ev_dev, args.mode)
        print(f"[bench] warmup {i}: {t['total_s']:.3f} s, {info.iterations} it", file=sys.stderr, flush=True)
    times = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        if op is not None:
            del op
        op, w, info, u, t = one_step(torch, igb, geo, cfg, ev_dev, args.mode)
        times.append(t)
        print(f"[bench] step {i}: {t['total_s']:.3f} s (assembly {t['assembly_s']:.3f}, solve {t['solve_s']:.3f},"
              f" {info.iterations} it, relres {info.rel_residual:.2e})", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / max(1, args.steps)

    # accuracy of the last step against the exact interior potential
    exact = W.laplace_charge_field(ev, *cfg["charges"])
    pot_err = float(np.abs(u.cpu().numpy() - exact).max())

    # H2 matvec bandwidth: algorithmic bytes / median time of igb_matvec
    x = torch.randn(op.info.n_dof, dtype=torch.float64, device="cuda:0")
    for _ in range(3):
        op.matvec(x)
    mv = []
    for _ in range(args.matvec_reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        op.matvec(x)
        e1.record()
        e1.synchronize()
        mv.append(e0.elapsed_time(e1))
    mv_ms = float(np.median(mv))
    gbps = op.info.matvec_bytes / (mv_ms * 1e-3) / 1e9

    # per-stage durations (HIP events on the operator's stream) and the rooflines of the two
    # dominant matvec kernels: near-field block GEMV (HBM) and far field (HBM when coupling
    # blocks are stored, FP64 ALU when they are generated on the fly)
    stages = op.profile(reps=args.matvec_reps)  # launched as in igb_matvec
    sep = op.profile(reps=args.matvec_reps, separate=True)  # one kernel per stage
    near, far = op.partition()
    q2 = PRM["q"] ** 2
    npatch = len(cfg["patches"])
    off = np.concatenate([[0], np.cumsum([npatch << (2 * l) for l in range(op.info.leaf_level + 1)])])
    rows = len(np.unique(off[far[:, 0]] + far[:, 1]))  # clusters with far blocks (rows written)
    srcs = len(np.unique(off[far[:, 0]] + far[:, 2]))  # distinct source moment vectors read
    roofs = {}
    # symmetric near storage: blocks (t, s) with t <= s, column stride nl rounded up to 8; the
    # kernel reads them and the S* vector once and writes one partial row per block side
    flags = int(op.info.layout_flags)
    fused = bool(flags & 4)  # near blocks ride along in the far-field launch
    nleaf = npatch << (2 * op.info.leaf_level)
    nl = op.info.n_dof_super // nleaf
    ld = (nl + 7) // 8 * 8 if flags & 1 else nl
    nsb = int(np.sum(near[:, 0] <= near[:, 1])) if flags & 1 else len(near)
    ndiag = int(np.sum(near[:, 0] == near[:, 1])) if flags & 1 else 0
    near_bytes = op.info.near_bytes + 8 * op.info.n_dof_super + 8 * ld * (2 * nsb - ndiag)
    tt = (q2 + 7) // 8
    a = near_bytes / (sep["near_gemv"] * 1e-3) / 1e9
    roofs["near_gemv"] = {"bound": "hbm", "kernel": "k_near_sym<double>" if flags & 1 else "k_bsr_gemv<double, 0>",
                          "achieved": round(a, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                          "frac": round(a / HBM_PEAK_GBPS, 4), "traffic": read_traffic("near_gemv"),
                          "algorithmic_bytes": int(near_bytes), "avg_ms": round(sep["near_gemv"], 4),
                          "launched_alone": True}
    if args.mode == "stored":
        cb = op.info.coupling_bytes + 8 * q2 * (rows + srcs)
        a = cb / (stages["coupling"] * 1e-3) / 1e9
        roofs["coupling"] = {"bound": "hbm", "kernel": "k_bsr_gemv<double, 1>", "achieved": round(a, 1),
                             "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(a / HBM_PEAK_GBPS, 4),
                             "traffic": read_traffic("coupling_stored"), "algorithmic_bytes": int(cb),
                             "avg_ms": round(stages["coupling"], 4)}
    else:
        # mirrored pairs: each pair of blocks is generated once and applied both ways
        sym = bool(flags & 2)
        evals = (len(far) // 2 if sym else len(far)) * q2 * q2
        fpe = FLOP_PER_EVAL_SYM if sym else FLOP_PER_EVAL_LAPLACE
        flops = fpe * evals

        def alu_roof(kname, ms, traffic):
            a = flops / (ms * 1e-3) / 1e12
            return {"bound": "alu", "kernel": kname, "achieved": round(a, 2), "peak": FP64_VECTOR_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(a / FP64_VECTOR_PEAK_TFLOPS, 4), "traffic": traffic,
                    "algorithmic_flops": int(flops), "kernel_evaluations": int(evals),
                    "block_entries_applied": int(len(far) * q2 * q2), "flop_per_evaluation": fpe,
                    "avg_ms": round(ms, 4)}
        kfar = f"k_far_sym<double, {tt}, false>" if sym else "k_far_onthefly<double>"
        roofs["far_field"] = alu_roof(kfar, sep["coupling"], read_traffic("coupling") if sym else None)
        roofs["far_field"]["launched_alone"] = True
        if fused:
            # as launched in the solver: the near blocks ride along with the far-field pairs
            roofs["coupling"] = alu_roof(f"k_sym_products<double, {tt}, false>", stages["coupling"],
                                         read_traffic("coupling_fused"))
            roofs["coupling"]["hbm_bytes_alongside"] = int(near_bytes)
            roofs["coupling"]["hbm_GBps_alongside"] = round(near_bytes / (stages["coupling"] * 1e-3) / 1e9, 1)
        else:
            roofs["coupling"] = dict(roofs["far_field"])
    # the dominant kernel of the product as launched in the solver
    roofline = roofs["coupling"] if stages["coupling"] >= stages["near_gemv"] else roofs["near_gemv"]

    mean = {k: float(np.mean([t[k] for t in times])) for k in times[0]} if times else {}
    out = {
        "metric": METRIC,
        "value": round(ms_per_step / 1e3, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "geometry": "unit sphere, 6 rational NURBS patches of bidegree 4",
                   "kernel": "laplace", "p": PRM["p"], "m": PRM["m"], "q": PRM["q"], "eta": PRM["eta"],
                   "gauss_regular": PRM["gauss_regular"], "n_dof": int(op.info.n_dof),
                   "n_dof_super": int(op.info.n_dof_super), "rel_tol": TOL, "mode": "h2_" + args.mode,
                   "solver": f"jacobi_gmres_{RESTART}"},
        "h2_matvec_GBps": round(gbps, 1),
        "h2_matvec_ms": round(mv_ms, 4),
        "matvec_bytes": int(op.info.matvec_bytes),
        "stage_ms": {k: round(v, 4) for k, v in stages.items()},
        "stage_ms_separate": {k: round(v, 4) for k, v in sep.items()},
        "breakdown_s": {k: round(v, 4) for k, v in mean.items()},
        "host_setup_s": round(float(op.info.setup_seconds), 4),
        "iterations": int(info.iterations),
        "rel_residual": float(info.rel_residual),
        "potential_max_err": pot_err,
        "near_blocks": int(op.info.n_near_blocks),
        "far_blocks": int(op.info.n_far_blocks),
        "roofline": roofline,
        "roofline_stages": roofs,
        "cpu_baseline": None,
    }
    if args.mode == "onthefly" and not args.no_mixed:
        out["mixed_fp32_far"] = mixed_leg(torch, igb, geo, cfg, ev_dev, ms_per_step, exact)
    if not args.no_learned:
        out["learned_preconditioner"] = learned_leg(torch, igb)
    if args.batched:
        out["batched"] = batched_leg(torch, igb)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, int(info.iterations))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
