"""Autotuner of the block-solve options per size class (writes tuning.json).

Times one full local stage (assembly, factorisation, LOBPCG to rho <= 1e-6)
of each workload below under every combination of

    split in {0, 1}        MSGFEM_OPT_SPLIT (nested dissection)
    solve in {1, 2, 3}     MSGFEM_OPT_SOLVE (vector / matrix cores x 8 / x 16)
    graph in {0, 1}        MSGFEM_OPT_GRAPH

(combinations whose solve family falls back to one already timed are
skipped), checks that every box converged, and stores for each workload's
size class (tuning.size_class) the fastest combination together with all
timings.  Run on the GPU:

    python -m paper_2211_13893_amd.autotune [--out paper_2211_13893_amd/tuning.json]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import msgfem, synth, tuning


def workloads():
    lam = synth.full_laminate(nx=96, ny=64, nz=48)
    return [
        ("beam (4 subdomains)", synth.laminated_beam(), None, 5),
        ("uniform batch, 16 boxes", synth.uniform_batch(n_boxes=16), None, 3),
        ("uniform batch, 64 boxes", synth.uniform_batch(n_boxes=64), None, 3),
        ("uneven batch, 168 boxes", synth.uneven_laminate(), None, 2),
        ("laminate chunk, 24 boxes of up to 24^3 nodes", lam, list(range(24)), 1),
    ]


def time_stage(prob, batch, steps, split, solve, graph):
    import torch
    st = msgfem.LocalStage(prob, batch=batch, tol=1e-6, split=split, solve=solve, graph=graph)
    fam = st.get_option(msgfem.INFO_SOLVE_FAMILY)

    def step():
        st.msgfem_assemble_local()
        return st.msgfem_local_eigs()

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    ok = bool(np.all(out["status"].cpu().numpy() == 0))
    bt = st.get_option(msgfem.INFO_MAX_BT_AHAT)
    cls = tuning.size_class(bt, len(st.batch), st.k)
    del st, out
    torch.cuda.empty_cache()
    return ms, ok, fam, cls


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=tuning.TABLE)
    a = ap.parse_args(argv)
    classes = {}
    for name, prob, batch, steps in workloads():
        seen = {}
        results = []
        cls = None
        for split in (0, 1):
            for solve in (3, 2, 1):
                for graph in (0, 1):
                    ms, ok, fam, cls = time_stage(prob, batch, steps, split, solve, graph)
                    key = (split, fam, graph)
                    if key in seen:
                        continue
                    seen[key] = ms
                    results.append(dict(split=split, solve=solve, family=fam, graph=graph, ms=round(ms, 2), ok=ok))
                    print(f"{name}: split {split} solve {solve} (families {fam}) graph {graph}: {ms:.1f} ms"
                          f"{'' if ok else '  NOT CONVERGED'}", flush=True)
        good = [r for r in results if r["ok"]]
        best = min(good, key=lambda r: r["ms"])
        entry = dict(split=best["split"], solve=best["solve"], graph=best["graph"], ms=best["ms"], workload=name,
                     timings=results)
        # a class measured on several workloads keeps the larger one's choice
        if cls not in classes or classes[cls]["ms"] < entry["ms"]:
            classes[cls] = entry
        print(f"  -> class {cls}: split {best['split']} solve {best['solve']} graph {best['graph']}", flush=True)
    table = {"device": "MI355X (gfx950)",
             "measured": "one local stage per timing (assembly + factorisation + LOBPCG to rho <= 1e-6), FP64",
             "classes": classes}
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
