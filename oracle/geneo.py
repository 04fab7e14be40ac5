"""Classic GenEO local eigenproblem and two-level additive Schwarz CG (oracle).

Test infrastructure.  Sec. 3.2: on each overlapping Omega_j (no
oversampling, no A-harmonic constraint), a_{Omega_j}(phi, v) =
lambda a_{Omega_j}(Xi phi, Xi v) for all v in V_h(Omega_j), the m_j smallest
eigenpairs spanning the coarse space R_j^T Xi_j(phi_{j,k}).  Used as the
coarse level of a two-level additive Schwarz preconditioner
M^{-1} = R_0^T A_0^{-1} R_0 + sum_j R_j^T A_j^{-1} R_j (Sec. 3.2), with
A_j the Dirichlet matrix of Omega_j (DoFs supported inside Omega_j) and
A_0 = Z^T A Z, Z the GenEO coarse basis.  Sec. 5.3 uses the resulting CG to
produce the fine reference solution.  The solution of that CG is pinned by
the sparse direct solve; its iteration count has no pin (the condition bound
of Sec. 3.2 has an unknown constant).

Pins of the local GenEO pencil (tests/test_oracle_geneo.py): the literal
pencil (A, D A D) by QZ on a tiny box; exactly 3 |P| eigenvalues equal to 1,
P the nodes whose 27-point neighbourhood has mu = 1 (there D phi = phi and
A phi = D A D phi); Courant-Fischer against the separately pinned A-harmonic
oracle with no oversampling (V_A is a subspace of V_h(Omega_j), so every
A-harmonic lambda_k is at least the GenEO lambda_k); independence of the
oversampling; six rigid-body zeros on a floating subdomain and none on a
clamped one.  The GenEO coarse approximation (geneo_msgfem) is pinned by
recovering the fine solution when every GenEO eigenvector is kept (the
partition-of-unity-weighted local spaces then span all of V_h), by Galerkin
orthogonality and by nested spaces (e_a non-increasing in n_ev).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import coarse, decomp, fem


def omega_dofs(prob, j: int):
    """(global DoFs of the closed Omega_j box, interior-node mask, mu per DoF)."""
    elo, ehi = prob.omega_box(j)
    nlo, nhi = decomp.node_box(elo, ehi)
    I, J, K = decomp.local_node_grid(nlo, nhi)
    g = I + (prob.nx + 1) * (J + (prob.ny + 1) * K)
    gd = (3 * g[:, None] + np.arange(3)[None, :]).ravel()
    bnd = decomp.interior_boundary_mask(prob, nlo, nhi, I, J, K)
    mu = decomp.pou_global(prob, j)[g]
    return gd, np.repeat(~bnd, 3), np.repeat(mu, 3)


def geneo_local(prob, j: int, n_ev: int, s: float = 1.0, kecache=None):
    """n_ev smallest eigenpairs of the GenEO pencil on Omega_j (Neumann matrix, B3 removed)."""
    elo, ehi = prob.omega_box(j)
    A = fem.assemble_box_dense(prob, elo, ehi, kecache)
    gd, _, mu = omega_dofs(prob, j)
    keep = np.flatnonzero(prob.dirichlet[gd] == 0)
    Ak = A[np.ix_(keep, keep)]
    d = mu[keep]
    B = d[:, None] * Ak * d[None, :]
    nu, X = sla.eigh(B, Ak + s * B)
    order = np.argsort(-nu)[:n_ev]
    nu, X = nu[order], X[:, order]
    phi = np.zeros((gd.size, n_ev))
    phi[keep] = X
    return 1.0 / nu - s, phi, gd, mu


def geneo_locals(prob, n_ev, kecache=None, load=None, s: float = 1.0):
    """Per subdomain (phi, psi, mu, dofs, lambda) of the GenEO local space used as
    a stand-alone coarse approximation (Sec. 5.4 compares it with the
    A-harmonic space): phi the n_ev lowest GenEO eigenvectors on Omega_j, psi
    the particular function on Omega_j itself (A psi = b on the DoFs that are
    neither on the interior boundary of Omega_j nor clamped, psi = 0 there),
    the same construction as the A-harmonic case with Omega_j^* = Omega_j.
    The tuple matches the ``locals_`` argument of ``coarse.msgfem``."""
    if load is None:
        load = fem.traction_load(prob)
    out = []
    for j in range(prob.nsd):
        k = int(prob.n_ev[j]) if n_ev is None else (n_ev[j] if hasattr(n_ev, "__len__") else int(n_ev))
        lam, phi, gd, mu = geneo_local(prob, j, k, s=s, kecache=kecache)
        _, inner, _ = omega_dofs(prob, j)
        i1 = np.flatnonzero(inner & (prob.dirichlet[gd] == 0))
        psi = np.zeros(gd.size)
        bj = load[gd]
        if np.any(bj[i1] != 0.0):
            elo, ehi = prob.omega_box(j)
            A = fem.assemble_box_dense(prob, elo, ehi, kecache)
            psi[i1] = sla.cho_solve(sla.cho_factor(A[np.ix_(i1, i1)], lower=True), bj[i1])
        out.append((phi, psi, mu, gd, lam))
    return out


def geneo_msgfem(prob, n_ev=None, A=None, b=None, s: float = 1.0):
    """The coarse approximation u^G in the GenEO space (Galerkin with the
    particular functions of ``geneo_locals``), for comparison with the
    A-harmonic MS-GFEM space of ``coarse.msgfem``."""
    kec = fem.KeCache(prob)
    A = fem.assemble_global_sparse(prob, kec) if A is None else A
    b = fem.traction_load(prob) if b is None else b
    return coarse.msgfem(prob, n_ev, A, b, s, locals_=geneo_locals(prob, n_ev, kec, b, s))


def geneo_coarse_basis(prob, n_ev, kecache=None) -> np.ndarray:
    cols = []
    for j in range(prob.nsd):
        k = int(prob.n_ev[j]) if n_ev is None else int(n_ev)
        lam, phi, gd, mu = geneo_local(prob, j, k, kecache=kecache)
        Vj = coarse.mgs_twice(mu[:, None] * phi)
        G = np.zeros((prob.n_dofs, Vj.shape[1]))
        G[gd] = Vj
        cols.append(G)
    return np.concatenate(cols, axis=1)


def two_level_pcg(prob, A, b, n_ev=None, rtol: float = 1e-8, maxit: int = 2000):
    """Plain preconditioned CG with the two-level GenEO additive Schwarz preconditioner."""
    F = coarse.free_dofs(prob)
    pos = -np.ones(prob.n_dofs, dtype=np.int64)
    pos[F] = np.arange(F.size)
    AF = A[F][:, F].tocsr()
    bF = b[F]
    Z = geneo_coarse_basis(prob, n_ev)[F]
    A0 = Z.T @ (AF @ Z)
    c0 = sla.cho_factor(0.5 * (A0 + A0.T), lower=True)
    locs = []
    for j in range(prob.nsd):
        gd, inner, _ = omega_dofs(prob, j)
        idx = pos[gd[inner]]
        idx = idx[idx >= 0]
        Aj = AF[idx][:, idx].toarray()
        locs.append((idx, sla.cho_factor(Aj, lower=True)))

    def prec(r):
        z = Z @ sla.cho_solve(c0, Z.T @ r)
        for idx, cf in locs:
            z[idx] += sla.cho_solve(cf, r[idx])
        return z

    x = np.zeros(F.size)
    r = bF.copy()
    z = prec(r)
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(bF)
    it = 0
    while np.linalg.norm(r) > rtol * nb and it < maxit:
        q = AF @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    u = np.zeros(prob.n_dofs)
    u[F] = x
    return u, it, float(np.linalg.norm(r) / nb)
