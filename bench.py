#!/usr/bin/env python3
"""Benchmark of the MS-GFEM local spectral stage on one MI355X.

One step = the whole hot path for one batch: assembly of every oversampled
box (materials, partition of unity, block-27 stencils, banded factors) and the
A-harmonic local GEVPs to rho <= 1e-6, with eigenvalues, eigenvectors and
residuals resident in HBM at the end.  The mesh, materials and decomposition
are resident on the device before timing starts.

Workload (default): the uniform batch of 64 interior 14^3-element oversampled
boxes (10125 DoF each) of a ply/resin laminate, n_ev = 16, block 32, FP64.

Prints one JSON line: GEVPs/s (boxes whose n_ev pairs all reach
rho <= 1e-6, per second) of the FP64 path, the roofline of its dominant
kernel (HIP events around each launch on its stream, algorithmic
bytes/flops from the library), the same workload on the two mixed-precision
paths (an FP32 copy of the preconditioner's factor; FP32 operator copies
first with an FP64 finish; both return FP64 residuals) with their ratio to
the FP64 path, the FP64 path started from the learned warm
start (network trained before timing; its inference is inside the step), the
uneven batch (168 boxes of 4.6k-25k DoF, bands up to 48 tiles) as a second
workload, and the FP64 CPU oracle timed on a bounded sample of the same boxes.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "local GEVPs/sec (n_ev pairs, resid≤1e-6), mixed vs FP64 path; SpMM HBM GB/s"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
# rocprofv3 summary of the FP64 path on this workload (kernel times and the
# FETCH_SIZE / WRITE_SIZE traffic of its kernels)
PROFILE = "local_stage_uniform_batch64_fp64.md"
# the same for the mixed path on the uneven batch
PROFILE_C3 = "local_stage_uneven_batch168_mixed.md"


def cpu_baseline(prob, n_sample: int):
    """The FP64 oracle on n_sample boxes of the same batch (dense assembly + Schur + eigh)."""
    import numpy as np
    from oracle import fem, gevp
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    kec = fem.KeCache(prob)
    t0 = time.perf_counter()
    for j in list(prob.batch)[:n_sample]:
        ops = gevp.local_ops(prob, int(j), kec)
        gevp.schur_gevp(ops, int(prob.n_ev[int(j)]))
    dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "GEVP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n_sample} of {len(prob.batch)} boxes of the same batch, FP64 dense "
                      f"assembly + Schur reduction + scipy eigh, {dt:.1f} s"}


def roofline(stats, profile_name):
    """Roofline of the dominant kernel of a profiled run: algorithmic bytes
    (or flops) per launch over the average launch duration (HIP events on the
    launch stream); a block solve's launch is one solve operation (its three
    phase kernels when the matrices are split).  traffic: FETCH_SIZE +
    WRITE_SIZE per launch from the committed profile, while its sources are
    unchanged."""
    from paper_2211_13893_amd import profiling
    dom = max(stats, key=lambda n: stats[n]["ms"])
    d = stats[dom]
    avg_s = d["ms"] / d["launches"] / 1e3
    per_launch_bytes = d["bytes"] / d["launches"]
    per_launch_flops = d["flops"] / d["launches"]
    ai = per_launch_flops / per_launch_bytes if per_launch_bytes else float("inf")
    if ai > PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9):
        achieved = per_launch_flops / avg_s / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None}
    else:
        achieved = per_launch_bytes / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None}
    roof.update(kernel=dom, avg_launch_ms=avg_s * 1e3, algorithmic_bytes_per_launch=per_launch_bytes,
                algorithmic_flops_per_launch=per_launch_flops,
                fp64_tflops=per_launch_flops / avg_s / 1e12)
    lib_kernel = {"band_solve": "k_band_solve", "spmm": "k_spmm"}.get(dom)
    if lib_kernel and profile_name:
        t = profiling.recorded_traffic(os.path.join(ROOT, "profiles", profile_name), lib_kernel)
        roof["traffic"] = t
        if t:
            roof["traffic_vs_algorithmic"] = t / per_launch_bytes
    return roof


def kernel_table(stats, steps):
    tot_ms = sum(v["ms"] for v in stats.values()) or 1.0
    out = {}
    for n, v in stats.items():
        sec = v["ms"] / 1e3
        out[n] = {"launches": v["launches"], "ms_per_step": v["ms"] / steps, "share": v["ms"] / tot_ms,
                  "GB/s": (v["bytes"] / sec / 1e9) if sec > 0 else None,
                  "TFLOP/s": (v["flops"] / sec / 1e12) if sec > 0 else None}
    return out


def c3_leg(run, args):
    """The uneven batch (168 boxes of 4.6k-25k DoF, one plan) with the plan
    options of its size class: FP64, and the mixed path (FP32 copy of the
    preconditioner's factor; SpMM, interior solves, Gram, FP64 Rayleigh-Ritz
    and residuals in FP64) with LOBPCG iterations replayed from HIP graphs
    against the eager loop (both without per-kernel events), and a profiled
    run of the mixed path for its roofline."""
    import numpy as np
    from paper_2211_13893_amd import synth
    import gc
    import torch
    up = synth.uneven_laminate()
    steps = max(5, args.steps)

    def one(*a, **kw):
        # each plan of this batch holds about 100 GB: release it before the next
        r = run(*a, **kw)
        r["dofs"] = [b.n_dof for b in r["stage"].boxes]
        r["k"] = int(r["stage"].k)
        del r["stage"]
        gc.collect()
        torch.cuda.empty_cache()
        return r

    fp = one(0, problem=up, steps=steps, warmup=1)
    mixed = one(1, problem=up, steps=steps, warmup=1)
    graph = one(1, problem=up, steps=steps, warmup=1, profile=False, graph=True)
    eager = one(1, problem=up, steps=steps, warmup=1, profile=False, graph=False)
    dofs = fp["dofs"]
    dnu = np.abs(1.0 / (mixed["nu"] + 1.0) - 1.0 / (fp["nu"] + 1.0)) * (fp["nu"] + 1.0)
    out = {"workload": "uneven_laminate",
           "description": "all 168 oversampled boxes of a wrinkled 256x32x24-element laminate (24 plies of "
                          "random angle) cut at random tensor positions (6-16 elements), overlap 1, "
                          "oversampling 1-3, n_ev 8-32, rho <= 1e-6, one plan",
           "box_dof": [int(min(dofs)), int(max(dofs))], "block": fp["k"], "steps": steps, "warmup": 1,
           "size_class": fp["size_class"], "plan_options": fp["plan_options"],
           "fp64": {"value": fp["value"], "unit": "GEVP/s", "ms_per_step": fp["ms_step"],
                    "converged": f"{fp['conv']}/{len(dofs)}", "lobpcg_iters_mean": float(fp["iters"].mean()),
                    "roofline": roofline(fp["stats"], None), "kernels": kernel_table(fp["stats"], steps)},
           "mixed_fp32_preconditioner": {
               "value": mixed["value"], "unit": "GEVP/s", "ms_per_step": mixed["ms_step"],
               "converged": f"{mixed['conv']}/{len(dofs)}", "lobpcg_iters_mean": float(mixed["iters"].mean()),
               "max_nu_rel_diff_vs_fp64_path": float(dnu.max()),
               "roofline": roofline(mixed["stats"], PROFILE_C3), "kernels": kernel_table(mixed["stats"], steps)},
           "graph_vs_eager": {"graph": {"value": graph["value"], "ms_per_step": graph["ms_step"],
                                        "graph_launches_last_step": graph["graph_launches"]},
                              "eager": {"value": eager["value"], "ms_per_step": eager["ms_step"]},
                              "ratio": graph["value"] / eager["value"] if eager["value"] > 0 else None,
                              "path": "mixed (FP32 preconditioner factor), no per-kernel events"}}
    del fp, mixed, graph, eager
    return out


def c4_leg(n_train_seeds=79, n_held_seeds=16, n_boxes=256, steps=2000):
    """The learned warm start at scale: a 48-mode basis (the 48 lowest
    A-harmonic modes of the homogeneous reference box, two deflated rounds),
    labels from the FP64 path on n_train_seeds x n_boxes training boxes
    (seeds 0 ..), Adam on 64-box minibatches, then LOBPCG iterations and time
    from the random and the learned start on n_held_seeds x n_boxes held-out
    boxes (seeds 10^6 ..).  The best start each basis span allows (the label
    projector's leading vectors, so the network's ceiling) is measured for
    the 32- and 48-mode bases on the first held-out batch."""
    import gc
    import numpy as np
    import torch
    from paper_2211_13893_amd import msgfem, synth, warm
    t0 = time.perf_counter()
    G48, st_ref, _ = warm.reference_basis(ng=48)
    del st_ref
    G32, st_ref, _ = warm.reference_basis(ng=32)
    del st_ref
    _log("[C4] reference bases of 48 and 32 modes done")
    feats, labels = warm.dataset(G48, range(n_train_seeds), n_boxes=n_boxes, log=_log)
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    net, losses = warm.fit_dataset(G48, feats, labels, steps=steps, log=_log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_train = sum(f.shape[0] for f in feats)
    del feats, labels
    gc.collect()
    torch.cuda.empty_cache()
    held = [10**6 + i for i in range(n_held_seeds)]
    ev = warm.evaluate(net, G48, held, n_boxes=n_boxes, log=_log)
    _log("[C4] basis ceilings")
    # ceilings of the two bases on the first held-out batch
    p = synth.warm_start_batch(n_boxes=n_boxes, seed=held[0])
    st = msgfem.LocalStage(p, tuned=True)
    st.msgfem_assemble_local()
    out = st.msgfem_local_eigs()
    ceil = {}
    for name, G in (("basis32", G32), ("basis48", G48)):
        P = st.msgfem_warm_labels(out, G, 16).double().cpu().numpy()
        _, V = np.linalg.eigh(P)
        coef = torch.as_tensor(np.ascontiguousarray(V[:, :, -16:]).reshape(P.shape[0], -1), dtype=torch.float32,
                               device="cuda:0")
        o2 = st.msgfem_local_eigs(x0=st.msgfem_warm_start(coef, G, 16, 0))
        ceil[name] = float(o2["iters"].float().mean().item())
    it_rand_first = float(out["iters"].float().mean().item())
    del st, out
    gc.collect()
    torch.cuda.empty_cache()
    ir, iw = ev["iters_random"], ev["iters_warm"]
    return {"workload": "warm_start_batch",
            "description": "14^3-element boxes of wrinkled ply/resin laminates (wrinkle amplitude U[0, 0.8] ply, "
                           "layer moduli log-U scaled by 1/1.2 .. 1.2), n_ev 16, FP64 path, rho <= 1e-6",
            "training_boxes": int(n_train), "held_out_boxes": int(ir.size), "basis_modes": 48,
            "adam_steps": steps, "minibatch": 64, "final_loss": float(np.mean(losses[-50:])),
            "data_seconds": t_data, "train_seconds": t_train,
            "iters_mean_random": float(ir.mean()), "iters_mean_learned": float(iw.mean()),
            "iteration_reduction": float(1.0 - iw.mean() / ir.mean()),
            "seconds_per_box_random": float(ev["seconds_random"].sum() / ir.size),
            "seconds_per_box_learned": float(ev["seconds_warm"].sum() / iw.size),
            "time_reduction": float(1.0 - ev["seconds_warm"].sum() / ev["seconds_random"].sum()),
            "max_nu_rel_diff": ev["max_nu_rel_diff"], "all_converged": ev["all_converged"],
            "ceiling_first_held_batch": {"iters_random": it_rand_first, **{f"iters_{k}": v for k, v in ceil.items()}},
            "network": "4 conv3d 3^3 (6->32->32->32->32, strides 1,1,2,2, ReLU), mean pool, affine 32 -> 48*16; "
                       "BF16 storage, FP32 sums; forward convolutions on the BF16 matrix cores, backward on "
                       "FP32 FMA kernels"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--boxes", type=int, default=64)
    ap.add_argument("--cpu-sample", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision path")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm-start path")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch workload")
    ap.add_argument("--block", type=int, default=0, help="LOBPCG block width (0: the library's rule)")
    ap.add_argument("--no-c5", action="store_true", help="skip the full-laminate pipeline")
    ap.add_argument("--no-f1", action="store_true", help="skip the GenEO vs MS-GFEM comparison")
    ap.add_argument("--no-c4", action="store_true", help="skip the learned warm start at scale")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the local GEVPs of a batch "
                                   "are independent and would be sharded by subdomain across GPUs"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2211_13893_amd import msgfem, synth

    prob = synth.uniform_batch(n_boxes=args.boxes)

    def run(precision: int, net=None, G=None, problem=None, steps=None, warmup=None, profile=True, **stage_kw):
        """Time `steps` full local stages (assembly + factorisation + LOBPCG; with
        a warm-start network also its features, inference and start block).
        With profile, HIP events bracket every kernel launch in the timed
        region (the per-kernel times and the roofline come from them; the
        LOBPCG iterations are then launched eagerly, not from graphs)."""
        stage_kw.setdefault("tuned", True)
        stage = msgfem.LocalStage(problem or prob, tol=1e-6, precision=precision, block=args.block, **stage_kw)
        steps = args.steps if steps is None else steps
        warmup = args.warmup if warmup is None else warmup

        def step():
            stage.msgfem_assemble_local()
            x0 = net.start_block(stage, G) if net is not None else None
            return stage.msgfem_local_eigs(x0=x0)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        if profile:
            stage.msgfem_profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stats = {}
        if profile:
            stage.msgfem_profile(False)
            stats = stage.msgfem_profile_stats()
        ms_step = (t1 - t0) / steps * 1e3
        status = out["status"].cpu().numpy()
        iters = out["iters"].cpu().numpy()
        conv = 0
        for b in range(len(stage.batch)):
            r = stage.resid(out, b).cpu().numpy()
            conv += int(np.all(r <= 1e-6) and status[b] == 0)
        res = {"stage": stage, "stats": stats, "ms_step": ms_step, "conv": conv, "iters": iters,
               "value": conv / (ms_step / 1e3), "nu": out["evals"].cpu().numpy(),
               "graph_launches": stage.get_option(msgfem.INFO_GRAPH_LAUNCHES),
               "plan_options": dict(getattr(stage, "plan_options", {})),
               "size_class": getattr(stage, "size_class", None)}
        return res

    fp = run(0)
    stage, stats, ms_step, conv, iters, value = (fp["stage"], fp["stats"], fp["ms_step"], fp["conv"],
                                                 fp["iters"], fp["value"])
    mixed = None
    if not args.no_mixed:
        mixed = {}
        for prec, name, what in ((1, "fp32_preconditioner", "FP32 copy of the preconditioner's factor "
                                  "(A + s DAD)^{-1}; SpMM, extension/adjoint solves, Gram, Rayleigh-Ritz "
                                  "and residuals FP64"),
                                 (2, "fp32_operators_first", "FP32 stencil and factor copies until rho <= 1e-4, "
                                  "then FP64 re-imaging and finish")):
            mx = run(prec)
            lam64, lam32 = fp["nu"], mx["nu"]
            dnu = np.abs(1.0 / (lam32 + 1.0) - 1.0 / (lam64 + 1.0)) * (lam64 + 1.0)
            mixed[name] = {"precision": prec, "description": what,
                           "value": mx["value"], "unit": "GEVP/s", "ms_per_step": mx["ms_step"],
                           "converged": f"{mx['conv']}/{len(stage.batch)}",
                           "lobpcg_iters_mean": float(mx["iters"].mean()),
                           "vs_fp64_path": mx["value"] / value if value > 0 else None,
                           "max_nu_rel_diff_vs_fp64_path": float(dnu.max()),
                           "kernels_ms_per_step": {n: v["ms"] / args.steps for n, v in mx["stats"].items()}}
            del mx
    uneven = None
    if not args.no_uneven:
        uneven = c3_leg(run, args)
    warm_res = None
    if not args.no_warm:
        from paper_2211_13893_amd import warm
        t0 = time.perf_counter()
        G, _, _ = warm.reference_basis(ng=32)
        net, losses = warm.fit(G, seeds=range(4), steps=300)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        wr = run(0, net, G)
        dnu = np.abs(1.0 / (wr["nu"] + 1.0) - 1.0 / (fp["nu"] + 1.0)) * (fp["nu"] + 1.0)
        warm_res = {"value": wr["value"], "unit": "GEVP/s", "ms_per_step": wr["ms_step"],
                    "converged": f"{wr['conv']}/{len(stage.batch)}",
                    "lobpcg_iters_mean": float(wr["iters"].mean()),
                    "vs_fp64_path": wr["value"] / value if value > 0 else None,
                    "max_nu_rel_diff_vs_fp64_path": float(dnu.max()),
                    "training": f"basis of 32 reference modes; 300 BF16 Adam steps on 4 x 64 "
                                f"warm-start boxes (seeds 0-3), FP64-path labels; final loss "
                                f"{losses[-1]:.3f}; {t_train:.1f} s, outside the timed steps",
                    "kernels_ms_per_step": {n: v["ms"] / args.steps for n, v in wr["stats"].items()}}
        del wr

    # dominant kernel and its roofline
    tot_ms = sum(v["ms"] for v in stats.values()) or 1.0
    roof = roofline(stats, PROFILE)
    kernels = kernel_table(stats, args.steps)
    spmm = stats.get("spmm")
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "GEVP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "uniform_batch",
                   "description": f"{args.boxes} interior oversampled boxes of 14^3 Q1 elements "
                                  "(10125 DoF), 0.25 mm plies / 0.05 mm resin, core 8^3, overlap 1, "
                                  f"oversampling 2, n_ev 16, LOBPCG block {int(stage.k)}, rho <= 1e-6, FP64 path",
                   "boxes": args.boxes, "n_ev": 16, "block": int(stage.k), "tol": 1e-6,
                   "path": "fp64", "parallelism": "subdomain batch on one GPU",
                   "size_class": fp["size_class"], "plan_options": fp["plan_options"],
                   "lobpcg_launch": "eager (per-kernel HIP events in the timed region)"},
        "converged": f"{conv}/{len(stage.batch)}",
        "lobpcg_iters_mean": float(iters.mean()),
        "spmm_hbm_GBs": (spmm["bytes"] / (spmm["ms"] / 1e3) / 1e9) if spmm else None,
        "roofline": roof,
        "kernels": kernels,
        "mixed_path": mixed,
        "warm_start_path": warm_res,
        "uneven_batch": uneven,
        "cpu_baseline": None,
    }
    # the remaining legs need the GPU's memory: release the uniform-batch plans
    del fp, stage
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    if not args.no_c5:
        line["full_pipeline"] = full_pipeline_leg()
        gc.collect()
        torch.cuda.empty_cache()
    if not args.no_f1:
        line["geneo_vs_msgfem"] = f1_leg()
        gc.collect()
        torch.cuda.empty_cache()
    if not args.no_c4:
        line["learned_warm_start_at_scale"] = c4_leg()
        gc.collect()
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline and args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_sample)
    print(json.dumps(line), flush=True)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def full_pipeline_leg():
    """The whole pipeline on the 512x64x48-element ply/resin laminate (4.9M DoF,
    384 subdomains of 16^3-element cores, overlap 2, oversampling 2, n_ev 20):
    the A-harmonic local stage streamed through plans sized to HBM, coarse
    assembly (N_H = 7680) and FP64 coarse solve, then the GenEO local stage,
    its coarse matrix and the two-level CG to 1e-8 as the fine reference."""
    import numpy as np
    from paper_2211_13893_amd import pipeline, synth
    prob = synth.full_laminate()
    t0 = time.perf_counter()
    res = pipeline.run(prob, tol=1e-6, log=_log)
    wall = time.perf_counter() - t0
    loc = res["local"]
    conv = int(np.sum((loc.status == 0) & (loc.max_rho <= 1e-6)))
    en = pipeline.error_norms(prob, res["u_pcg"], res["uG"])
    gl = res["geneo_local"]
    out = {"workload": "full_laminate",
           "description": "512x64x48-element wrinkled ply/resin laminate (0.25 mm plies, 0.05 mm resin), "
                          "384 subdomains of 16^3-element cores, overlap 2, oversampling 2, n_ev 20, rho <= 1e-6, "
                          "FP64; clamped at x = 0, -10 MPa on x = max",
           "n_dof": int(prob.n_dofs), "subdomains": int(prob.nsd), "n_coarse": int(res["store"].NH),
           "local_plans": len(loc.chunks), "local_converged": f"{conv}/{prob.nsd}",
           "local_gevp_per_s": conv / loc.seconds, "lobpcg_iters_mean": float(loc.iters.mean()),
           "stage_seconds": res["times"], "pipeline_wall_seconds": wall,
           "geneo_local_plans": len(gl.chunks), "geneo_local_converged": int(np.sum(gl.status == 0)),
           "pcg_iters": res["pcg_iters"], "pcg_relres": res["pcg_relres"],
           "e_a_vs_pcg": res["e_a"], "e_d_vs_pcg": float(en[4]), "e_eps_vs_pcg": float(en[5])}
    del res
    return out


def f1_leg():
    """Classic GenEO against A-harmonic MS-GFEM as coarse approximations (Sec.
    5.4) on the uneven laminate (636k DoF): e_a, e_d, e_eps against the GenEO
    two-level CG solution for n_ev = 8, 16, 24 per subdomain."""
    import numpy as np
    import torch
    from paper_2211_13893_amd import pipeline, synth
    prob = synth.uneven_laminate()
    ref = pipeline.run(prob, tol=1e-6, log=_log)
    uh, gs = ref["u_pcg"], ref["geneo_store"]
    rows = []
    for n in (8, 16, 24):
        row = {"n_ev": n}
        for geneo, name in ((False, "msgfem"), (True, "geneo")):
            uG, loc, dt = pipeline.coarse_approximation(prob, geneo, n, log=_log)
            en = gs.energy(uh, uG).cpu().numpy()
            nm = pipeline.error_norms(prob, uh, uG)
            row[name] = {"e_a": float(np.sqrt(en[0] / en[1])), "e_d": float(nm[4]), "e_eps": float(nm[5]),
                         "seconds": dt, "converged": int(np.sum(loc.status == 0))}
            del uG
            torch.cuda.empty_cache()
        rows.append(row)
    out = {"workload": "uneven_laminate", "reference": f"GenEO two-level CG, relres {ref['pcg_relres']:.1e}, "
                                                      f"{ref['pcg_iters']} iterations",
           "rows": rows}
    del ref
    return out


if __name__ == "__main__":
    main()
