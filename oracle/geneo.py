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
clamped one.
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
