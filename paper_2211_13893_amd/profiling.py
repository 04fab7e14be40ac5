"""Kernel-time and HBM-traffic summaries of the local stage from rocprofv3 output.

    python -m paper_2211_13893_amd.profiling run [--boxes 64] [--steps 1] [--workload uniform|uneven]
                                                 [--precision 0|1]
        the profiled workload: one 256 MiB device-to-device copy (the
        calibration of the traffic counters), then `steps` local stages
        (assembly + factorisation + LOBPCG) of the uniform batch or the
        uneven batch, with the plan options of their size class and eager
        LOBPCG launches (as the timed steps of bench.py);
    python -m paper_2211_13893_amd.profiling summarize --trace D --fetch D --write D --out F.md
        a markdown summary of the kernel statistics of a `--kernel-trace
        --stats` run (directory D) and, per kernel, the HBM bytes per launch
        from a `--pmc FETCH_SIZE` and a `--pmc WRITE_SIZE` run of the same
        workload.  Each counter is scaled by the factor that makes it read
        256 MiB for the calibration copy (read 256 MiB, written 256 MiB).
        --solve-phases P: the block solve of a split plan is P dispatches
        (chains forward, separators, chains backward) per solve operation;
        its time and traffic are also given per operation, the unit of the
        roofline in bench.py.

The summary records a SHA-256 of the kernel sources; bench.py reports the
measured traffic only while those sources are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys
import time
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 256 * 1024 * 1024
# kernel (name prefix in the trace) -> sources it is built from
KERNEL_SOURCES = {
    "k_band_solve": ["csrc/solve.hip", "csrc/band_view.hpp", "csrc/internal.hpp"],
    "k_spmm": ["csrc/spmm.hip", "csrc/internal.hpp"],
}


def sources_sha256(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    n = re.sub(r"\(.*$", "", name.strip().strip('"'))
    n = re.sub(r"^void ", "", n)
    return n.replace("msg::", "")


def _csv(d: str, suffix: str):
    files = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    with open(files[0], newline="") as f:
        return list(csv.DictReader(f))


def counter_per_dispatch(d: str, counter: str):
    """{dispatch id: (kernel name, grid size, summed counter value in KiB)}."""
    out = {}
    for r in _csv(d, "counter_collection.csv"):
        if not r["Counter_Name"].startswith(counter):
            continue
        k = int(r["Dispatch_Id"])
        name, grid, v = out.get(k, (r["Kernel_Name"], int(r["Grid_Size"]), 0.0))
        out[k] = (name, grid, v + float(r["Counter_Value"]))
    return out


def calibration(per_dispatch) -> float:
    """Bytes per counter unit: the 256 MiB copy is the copy dispatch with the largest value."""
    copies = [v for (n, g, v) in per_dispatch.values() if "copyBuffer" in n or "copy" in n.lower()]
    if not copies:
        raise RuntimeError("no copy kernel in the counter run")
    return COPY_BYTES / max(copies)


def traffic_per_launch(fetch_dir: str, write_dir: str):
    """{kernel: (launches, mean HBM bytes read, mean bytes written)} and the two factors."""
    f = counter_per_dispatch(fetch_dir, "FETCH_SIZE")
    w = counter_per_dispatch(write_dir, "WRITE_SIZE")
    cf, cw = calibration(f), calibration(w)
    acc = defaultdict(lambda: [0, 0.0, 0.0])
    for k, (n, g, v) in f.items():
        a = acc[short_name(n)]
        a[0] += 1
        a[1] += v * cf
    for k, (n, g, v) in w.items():
        acc[short_name(n)][2] += v * cw
    return {n: (a[0], a[1] / a[0], a[2] / a[0]) for n, a in acc.items() if a[0]}, cf, cw


def summarize(trace: str, fetch: str, write: str, out: str, title: str, commands: str, solve_phases: int = 1):
    stats = _csv(trace, "kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in stats)
    rows = sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))
    traffic, cf, cw = traffic_per_launch(fetch, write) if fetch and write else ({}, None, None)
    lines = [f"# {title}", "", "Commands (from the repository root, one MI355X):", "", "```", commands.strip(),
             "```", "", "## Kernel time (`--kernel-trace --stats`)", "",
             "| kernel | calls | total ms | avg us | min us | max us | share % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:20]:
        lines.append(f"| {short_name(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {100 * float(r['TotalDurationNs']) / tot:.2f} |")
    solve = [r for r in stats if short_name(r["Name"]).startswith("k_band_solve")]
    if solve:
        calls = sum(int(r["Calls"]) for r in solve)
        tns = sum(float(r["TotalDurationNs"]) for r in solve)
        ops = calls / solve_phases
        lines += ["", f"Block solve per operation ({solve_phases} dispatch(es) per solve): {ops:.0f} operations, "
                      f"{tns / ops / 1e3:.1f} us per operation."]
    if traffic:
        lines += ["", "## HBM traffic per launch (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`)", "",
                  f"Calibration on the 256 MiB copy: bytes = FETCH_SIZE x {cf / 1024:.3f} KiB, "
                  f"WRITE_SIZE x {cw / 1024:.3f} KiB.", "",
                  "| kernel | launches | read MB/launch | written MB/launch |", "|---|---:|---:|---:|"]
        for n, (c, r_, w_) in sorted(traffic.items(), key=lambda t: -(t[1][1] + t[1][2]) * t[1][0])[:12]:
            lines.append(f"| {n} | {c} | {r_ / 1e6:.3f} | {w_ / 1e6:.3f} |")
        lines += ["", "Machine-readable (bench.py reads these while the sources are unchanged):", ""]
        for kern in KERNEL_SOURCES:
            hit = [(n, v) for n, v in traffic.items() if n.startswith(kern)]
            if not hit:
                continue
            c = sum(v[0] for _, v in hit)
            per = solve_phases if kern == "k_band_solve" else 1
            b = sum(v[0] * (v[1] + v[2]) for _, v in hit) / (c / per)
            lines.append(f"    traffic_bytes_per_launch {kern} {b:.0f} sources_sha256 {sources_sha256(kern)}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


def recorded_traffic(md_path: str, kernel: str):
    """HBM bytes per launch of `kernel` recorded in a summary, or None when
    the file is absent or the kernel's sources changed since."""
    if not os.path.exists(md_path):
        return None
    pat = re.compile(rf"traffic_bytes_per_launch {re.escape(kernel)} ([0-9.e+]+) sources_sha256 ([0-9a-f]+)")
    with open(md_path) as f:
        for line in f:
            m = pat.search(line)
            if m:
                return float(m.group(1)) if m.group(2) == sources_sha256(kernel) else None
    return None


def run_workload(boxes: int, steps: int, workload: str = "uniform", precision: int = 0):
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2211_13893_amd import msgfem, synth
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print("calibration copy done", flush=True)
    del a, b
    prob = synth.uniform_batch(n_boxes=boxes) if workload == "uniform" else synth.uneven_laminate()
    # eager LOBPCG launches, as in the timed steps of bench.py (which bracket
    # every launch with HIP events): graph replays would add the empty
    # iterations of a replay after convergence to the dispatch counts
    st = msgfem.LocalStage(prob, tol=1e-6, precision=precision, tuned=True, graph=False)
    print(f"plan options {st.plan_options} (class {st.size_class})", flush=True)
    for i in range(steps):
        st.msgfem_assemble_local()
        out = st.msgfem_local_eigs()
        torch.cuda.synchronize()
        print(f"step {i} done, iterations {out['iters'].cpu().numpy().mean():.2f}", flush=True)


def run_reuse(boxes: int, changed: int, layout: str = "contiguous"):
    """Offline/online reuse on the uniform batch: solve all boxes, change the
    ply material in the middle 2^3 elements of `changed` cores (a run of
    neighbouring cores, or every (boxes // changed)-th core; elements that no
    other oversampled box holds), then time a full
    recompute against the online path (assemble, digest, solve only the boxes
    whose digest changed, merge)."""
    import dataclasses
    import json
    import numpy as np
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2211_13893_amd import msgfem, synth
    p0 = synth.uniform_batch(n_boxes=boxes)
    if layout == "strided":     # every (boxes // changed)-th core
        picked = [int(p0.batch[i]) for i in range(0, boxes, max(1, boxes // changed))][:changed]
    else:                       # a run of neighbouring cores in the middle of the column
        first = max(0, boxes // 2 - changed // 2)
        picked = [int(p0.batch[i]) for i in range(first, min(boxes, first + changed))]
    em = p0.elem_mat.copy().reshape(p0.nz, p0.ny, p0.nx)
    for sd in picked:
        x, y, z = (int(c) + 3 for c in p0.cores[sd, :3])
        em[z:z + 2, y:y + 2, x:x + 2] = (em[z:z + 2, y:y + 2, x:x + 2] + 1) % p0.materials.shape[0]
    p1 = dataclasses.replace(p0, elem_mat=em.ravel())
    st0 = msgfem.LocalStage(p0, tol=1e-6)
    st0.msgfem_assemble_local()
    d0 = st0.msgfem_box_digest()
    out0 = st0.msgfem_local_eigs()
    st1 = msgfem.LocalStage(p1, tol=1e-6)
    torch.cuda.synchronize()
    print("offline solve done", flush=True)
    ms = {}

    def timed(name, fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        ms[name] = (time.perf_counter() - t) * 1e3
        return r

    timed("assemble_all", st1.msgfem_assemble_local)
    timed("eigs_all", st1.msgfem_local_eigs)
    print("full recompute done", flush=True)
    timed("assemble_all", st1.msgfem_assemble_local)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    d1 = timed("digest", st1.msgfem_box_digest)
    e1.record()
    found = [int(st1.batch[b]) for b in np.flatnonzero((d0 != d1).cpu().numpy())]
    stc = timed("plan_changed", lambda: msgfem.LocalStage(p1, batch=found, tol=1e-6))
    timed("assemble_changed", stc.msgfem_assemble_local)
    outc = timed("eigs_changed", stc.msgfem_local_eigs)
    timed("merge", lambda: st1.msgfem_merge_eigs(out0, stc, outc))
    # the in-place variant on the full plan: no second plan, assembly or merge
    mask = [1 if int(j) in found else 0 for j in st1.batch]
    stored = {k: v.clone() for k, v in out0.items() if k != "status"}
    timed("eigs_subset_inplace", lambda: st1.msgfem_local_eigs_subset(mask, stored))
    torch.cuda.synchronize()
    digest_ms = e0.elapsed_time(e1)
    nbytes = sum(243 * 8 * b.n_nodes + 9 * b.n_dof for b in st1.boxes)
    full = ms["assemble_all"] + ms["eigs_all"]
    online = sum(ms[k] for k in ("assemble_all", "digest", "plan_changed", "assemble_changed", "eigs_changed",
                                 "merge"))
    online_inplace = ms["assemble_all"] + ms["digest"] + ms["eigs_subset_inplace"]
    print(json.dumps({"reuse": {"boxes": boxes, "layout": layout, "changed": picked, "found": found, "ms": ms,
                                "full_ms": full, "online_ms": online, "online_inplace_ms": online_inplace, "digest_event_ms": digest_ms,
                                "digest_bytes": nbytes, "digest_GBps": nbytes / digest_ms / 1e6}}), flush=True)
    if found != picked:
        raise SystemExit("digest found other boxes than the changed ones")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--boxes", type=int, default=64)
    r.add_argument("--steps", type=int, default=1)
    r.add_argument("--workload", choices=["uniform", "uneven"], default="uniform")
    r.add_argument("--precision", type=int, default=0)
    u = sub.add_parser("reuse")
    u.add_argument("--boxes", type=int, default=64)
    u.add_argument("--changed", type=int, default=8)
    u.add_argument("--layout", choices=["contiguous", "strided"], default="contiguous")
    s = sub.add_parser("summarize")
    s.add_argument("--trace", required=True)
    s.add_argument("--fetch")
    s.add_argument("--write")
    s.add_argument("--out", required=True)
    s.add_argument("--title", default="Kernel trace")
    s.add_argument("--commands", default="")
    s.add_argument("--solve-phases", type=int, default=1)
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run_workload(a.boxes, a.steps, a.workload, a.precision)
    elif a.cmd == "reuse":
        run_reuse(a.boxes, a.changed, a.layout)
    else:
        summarize(a.trace, a.fetch, a.write, a.out, a.title, a.commands, a.solve_phases)


if __name__ == "__main__":
    main()
