"""The MS-GFEM pipeline on one GPU with the local stage streamed through plans.

A decomposition whose oversampled boxes do not fit in one plan (a 24^3-element
box holds about 4 GB of operators and banded factors) is solved chunk by
chunk: each chunk is one plan over some subdomains, assembled and eigensolved,
and its share of the coarse problem goes into a coarse store
(``msgfem.CoarseStore``, the library's msgfem_coarse_* calls) before the plan
is freed.  Then the Galerkin system and the coarse solve give the MS-GFEM
solution u^G (Sec. 3.3, 4.4).  For comparison, and as the fine reference
where a direct solve is out of reach, the GenEO local eigenproblems (Sec. 3.2)
are streamed the same way into a GenEO store, which also keeps every
subdomain's interior factor (FP32) for the two-level additive Schwarz CG.

Every array operation runs in the library; this module only chooses chunks,
allocates through the bindings and times the stages.
"""
from __future__ import annotations

import ctypes
import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import msgfem


@dataclasses.dataclass
class LocalResult:
    iters: np.ndarray            # [nsd] LOBPCG iterations per subdomain
    status: np.ndarray           # [nsd] status bits
    max_rho: np.ndarray          # [nsd] largest residual of the subdomain's pairs
    evals: Dict[int, np.ndarray]  # subdomain -> eigenvalues
    kept: Dict[int, dict]        # subdomains whose eigenvectors were kept (host copies)
    chunks: List[List[int]]
    seconds: float


def box_bytes(problem, sd: int, geneo: bool = False, precision: int = 0, device: int = 0) -> int:
    """Device bytes (operators + workspace) a plan needs for subdomain sd alone (host-side query)."""
    lib = msgfem.load()
    p = problem
    mesh = msgfem.msgfem_mesh(p.nx, p.ny, p.nz, p.materials.shape[0], 1, 1, 1, 1)
    cores = np.ascontiguousarray(p.cores, np.int32)
    ovs = np.ascontiguousarray(p.ovs, np.int32)
    dec = msgfem.msgfem_decomp(p.nsd, cores.ctypes.data, p.overlap, ovs.ctypes.data)
    b = np.asarray([sd], np.int32)
    nev = np.asarray([p.n_ev[sd]], np.int32)
    opts = msgfem.msgfem_eig_opts(1.0, 1e-6, 200, 0, precision, 1 if geneo else 0, 1)
    plan = ctypes.c_void_p()
    rc = lib.msgfem_plan_create(ctypes.byref(plan), device, ctypes.byref(mesh), ctypes.byref(dec), b.ctypes.data,
                                nev.ctypes.data, 1, ctypes.byref(opts))
    try:
        msgfem._check(rc, plan, "msgfem_plan_create")
        s = msgfem.msgfem_sizes()
        msgfem._check(lib.msgfem_plan_sizes(plan, ctypes.byref(s)), plan, "msgfem_plan_sizes")
        return int(s.ops_bytes + s.work_bytes)
    finally:
        lib.msgfem_plan_destroy(plan)


def make_chunks(problem, budget_bytes: int, geneo: bool = False, subdomains: Optional[Sequence[int]] = None,
                max_chunk: Optional[int] = None) -> List[List[int]]:
    """Chunks of subdomains whose plans fit in budget_bytes.  Boxes sorted by
    size are dealt round-robin, so every chunk holds one of the largest boxes
    (its band width decides the block-solve layout, which a GenEO store needs
    to be the same for every chunk)."""
    sds = list(range(problem.nsd)) if subdomains is None else list(subdomains)
    sizes = {j: box_bytes(problem, j, geneo) for j in sds}
    order = sorted(sds, key=lambda j: -sizes[j])
    per = max(1, int(budget_bytes // max(sizes.values())))
    if max_chunk:
        per = min(per, max_chunk)
    n = (len(order) + per - 1) // per
    return [order[c::n] for c in range(n)]


def local_stage_streamed(problem, store: "msgfem.CoarseStore", chunks: List[List[int]], geneo: bool = False,
                         tol: float = 1e-6, precision: int = 0, keep: Sequence[int] = (), device: str = "cuda:0",
                         log=None) -> LocalResult:
    """Assemble and eigensolve every chunk, add it to the store, keep per-box results."""
    import torch
    nsd = problem.nsd
    iters = np.zeros(nsd, np.int32)
    status = np.zeros(nsd, np.int32)
    max_rho = np.full(nsd, np.nan)
    evals: Dict[int, np.ndarray] = {}
    kept: Dict[int, dict] = {}
    keep = set(int(j) for j in keep)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ci, chunk in enumerate(chunks):
        st = msgfem.LocalStage(problem, batch=chunk, tol=tol, geneo=geneo, precision=precision, device=device,
                               tuned=True)
        st.msgfem_assemble_local()
        out = st.msgfem_local_eigs()
        store.add(st, out)
        it = out["iters"].cpu().numpy()
        stat = out["status"].cpu().numpy()
        for b, j in enumerate(chunk):
            iters[j] = it[b]
            status[j] = stat[b]
            max_rho[j] = float(st.resid(out, b).max())
            evals[j] = st.eigvals(out, b).cpu().numpy()
            if j in keep:
                kept[j] = dict(evals=evals[j], evecs=st.eigvecs(out, b).cpu().numpy(),
                               resid=st.resid(out, b).cpu().numpy())
        if log:
            log(f"  chunk {ci + 1}/{len(chunks)}: {len(chunk)} boxes, iterations {it.min()}-{it.max()}, "
                f"status {sorted(set(stat.tolist()))}")
        # the chunks' plans have nearly the same sizes (boxes dealt round-robin
        # by size), so the caching allocator serves each plan from the blocks
        # the previous one freed; returning them to the driver made every
        # chunk's first solve map its buffers afresh (about 4 s per chunk of
        # the full laminate).  An allocation that does not fit makes torch
        # release the cache and retry by itself.
        del st, out
        torch.cuda.synchronize()
    torch.cuda.synchronize()
    return LocalResult(iters, status, max_rho, evals, kept, chunks, time.perf_counter() - t0)


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0


def run(problem, tol: float = 1e-6, budget_fraction: float = 0.7, with_geneo_pcg: bool = True,
        pcg_rtol: float = 1e-8, pcg_maxit: int = 2000, keep: Sequence[int] = (), max_chunk: Optional[int] = None,
        device: str = "cuda:0", log=None) -> dict:
    """The whole pipeline; returns the solutions (device tensors), per-box results and stage times (s)."""
    import torch
    times = {}
    free, _ = torch.cuda.mem_get_info()
    ms = msgfem.CoarseStore(problem, geneo=False, device=device)
    free, _ = torch.cuda.mem_get_info()
    chunks = make_chunks(problem, int(free * budget_fraction), max_chunk=max_chunk)
    if log:
        log(f"[pipeline] {problem.name}: {problem.nsd} subdomains, {problem.n_dofs} DoF, N_H {ms.NH}; "
            f"A-harmonic stage in {len(chunks)} chunks")
    loc = local_stage_streamed(problem, ms, chunks, tol=tol, keep=keep, device=device, log=log)
    times["local"] = loc.seconds
    (AH, bH), times["coarse_assembly"] = _timed(ms.galerkin)
    sol, times["coarse_solve"] = _timed(lambda: ms.solve(AH, bH))
    res = dict(problem=problem, local=loc, store=ms, AH=AH, bH=bH, uG=sol["uG"], up=sol["up"], c=sol["c"],
               coarse_status=int(sol["status"].item()), times=times)
    if not with_geneo_pcg:
        return res
    del AH
    torch.cuda.empty_cache()
    gs = msgfem.CoarseStore(problem, geneo=True, device=device)
    free, _ = torch.cuda.mem_get_info()
    gchunks = make_chunks(problem, int(free * budget_fraction * 0.8), geneo=True, max_chunk=max_chunk)
    if log:
        log(f"[pipeline] GenEO stage in {len(gchunks)} chunks")
    gloc = local_stage_streamed(problem, gs, gchunks, geneo=True, tol=tol, device=device, log=log)
    times["geneo_local"] = gloc.seconds
    (A0, _), times["geneo_coarse_assembly"] = _timed(gs.galerkin)
    pcg, times["pcg"] = _timed(lambda: gs.pcg(A0, rtol=pcg_rtol, maxit=pcg_maxit))
    en = gs.energy(pcg["u"], sol["uG"]).cpu().numpy()
    res.update(geneo_local=gloc, geneo_store=gs, A0=A0, u_pcg=pcg["u"], pcg_iters=pcg["iters"],
               pcg_relres=pcg["relres"], pcg_status=int(pcg["status"].item()),
               e_a=float(np.sqrt(en[0] / en[1])) if en[1] > 0 else float("nan"))
    if log:
        log(f"[pipeline] PCG {pcg['iters']} iterations, relres {pcg['relres']:.2e}; e_a(u^G vs PCG) {res['e_a']:.4e}")
    return res


def error_norms(problem, u_ref, u, device: str = "cuda:0"):
    """e_d, e_eps of Sec. 5.3 (msgfem_error_norms through a one-box plan of the same mesh)."""
    st = msgfem.LocalStage(problem, batch=[0], device=device)
    return st.msgfem_error_norms(u_ref, u).cpu().numpy()


def coarse_approximation(problem, geneo: bool, n_ev: int, tol: float = 1e-6, budget_fraction: float = 0.6,
                         device: str = "cuda:0", log=None):
    """u^G of one coarse space with n_ev functions per subdomain: the A-harmonic
    MS-GFEM space (geneo False) or the classic GenEO space (geneo True, local
    spaces and particular functions on Omega_j), streamed through plans.
    Returns (uG, local result, seconds)."""
    import torch
    p = dataclasses.replace(problem, n_ev=np.full(problem.nsd, int(n_ev), np.int32))
    store = msgfem.CoarseStore(p, geneo=geneo, device=device)
    free, _ = torch.cuda.mem_get_info()
    chunks = make_chunks(p, int(free * budget_fraction), geneo=geneo)
    t0 = time.perf_counter()
    loc = local_stage_streamed(p, store, chunks, geneo=geneo, tol=tol, device=device)
    AH, bH = store.galerkin()
    sol = store.solve(AH, bH)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    uG = sol["uG"].clone()
    del store, AH, bH, sol
    torch.cuda.empty_cache()
    if log:
        log(f"  {'GenEO' if geneo else 'MS-GFEM'} n_ev {n_ev}: {len(chunks)} plans, {dt:.2f} s")
    return uG, loc, dt
