"""Particular functions, the MS-GFEM coarse problem and the fine solve (oracle).

Test infrastructure.  Sec. 3.3: the coarse space V_H is spanned by the
partition-of-unity-weighted local eigenvectors R_j^T Xi_j(phi_{j,k}|Omega_j);
the local particular function u^p_j = psi^r + psi^d solves
a(psi^r, v) = b_{Omega*}(v) for v in V_{h,DI} (so psi^r vanishes on B2 and B3)
and psi^d carries the Dirichlet data A-harmonically; the global particular
function is u^p = sum_j R_j^T Xi_j(u^p_j|Omega_j); and the MS-GFEM solution
u^G = u^p + u_H, u_H in V_H, satisfies a(u^G, v) = b(v) for all v in V_H.
Sec. 4.3 multiplies the eigenvectors by the partition of unity and
re-orthogonalises them by Gram-Schmidt before the coarse matrix is formed.

Readings: Gram-Schmidt is Euclidean modified Gram-Schmidt applied twice,
dropping vectors whose norm falls below 1e-12 of the largest; the particular
function is lifted to the right-hand side (the Galerkin statement above)
instead of being appended with a Dirichlet row (Sec. 4.4), which gives the
same u^G and keeps the coarse matrix symmetric positive definite.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import decomp, fem, gevp


def free_dofs(prob) -> np.ndarray:
    return np.flatnonzero(prob.dirichlet == 0)


def fine_solve(prob, A=None, b=None) -> np.ndarray:
    """u_h: the fine FE solution with zero Dirichlet data (sparse direct)."""
    A = fem.assemble_global_sparse(prob) if A is None else A
    b = fem.traction_load(prob) if b is None else b
    F = free_dofs(prob)
    u = np.zeros(prob.n_dofs)
    u[F] = spla.spsolve(A[F][:, F].tocsc(), b[F])
    return u


def particular_local(ops: gevp.LocalOps) -> np.ndarray:
    """psi^r on Omega^*: A11 psi1 = b1, psi = 0 on B2 and B3 (zero Dirichlet data)."""
    i1 = ops.i1
    psi = np.zeros(ops.A.shape[0])
    if np.any(ops.b[i1] != 0.0):
        A11 = ops.A[np.ix_(i1, i1)]
        psi[i1] = sla.cho_solve(sla.cho_factor(A11, lower=True), ops.b[i1])
    return psi


def mgs_twice(V: np.ndarray, drop: float = 1e-12) -> np.ndarray:
    """Euclidean modified Gram-Schmidt, two passes, dropping near-dependent columns."""
    if V.shape[1] == 0:
        return V
    ref = np.max(np.linalg.norm(V, axis=0))
    Q = []
    for c in range(V.shape[1]):
        v = V[:, c].copy()
        for _ in range(2):
            for q in Q:
                v -= (q @ v) * q
        nv = np.linalg.norm(v)
        if nv > drop * ref:
            Q.append(v / nv)
    return np.stack(Q, axis=1) if Q else V[:, :0]


@dataclasses.dataclass
class CoarseResult:
    V: np.ndarray           # [n_dofs, N_H] global coarse basis
    up: np.ndarray          # global particular function
    AH: np.ndarray
    bH: np.ndarray
    c: np.ndarray
    uG: np.ndarray
    lam: list               # per subdomain eigenvalues used


def local_basis(prob, j: int, n_ev: int, kecache=None, load=None, s: float = 1.0):
    """(Phi_j, psi_j, mu_j, star dofs, eigenvalues) of subdomain j."""
    ops = gevp.local_ops(prob, j, kecache, load)
    res = gevp.schur_gevp(ops, n_ev, s)
    psi = particular_local(ops)
    return res.phi, psi, ops.mu, decomp.star_global_dofs(prob, j), res.lam


def msgfem(prob, n_ev=None, A=None, b=None, s: float = 1.0, locals_=None) -> CoarseResult:
    """The MS-GFEM coarse approximation u^G (Sec. 3.3) with the coarse basis of Sec. 4.3."""
    kec = fem.KeCache(prob)
    A = fem.assemble_global_sparse(prob, kec) if A is None else A
    b = fem.traction_load(prob) if b is None else b
    cols, up, lams = [], np.zeros(prob.n_dofs), []
    for j in range(prob.nsd):
        k = int(prob.n_ev[j]) if n_ev is None else (n_ev[j] if hasattr(n_ev, "__len__") else n_ev)
        if locals_ is not None:
            phi, psi, mu, gd, lam = locals_[j]
        else:
            phi, psi, mu, gd, lam = local_basis(prob, j, k, kec, b, s)
        lams.append(lam)
        Vj = mu[:, None] * phi            # Xi_j applied to phi restricted to Omega_j
        Vj = mgs_twice(Vj)
        G = np.zeros((prob.n_dofs, Vj.shape[1]))
        G[gd] = Vj
        cols.append(G)
        up[gd] += mu * psi
    V = np.concatenate(cols, axis=1)
    F = free_dofs(prob)
    AF = A[F][:, F]
    VF = V[F]
    AH = VF.T @ (AF @ VF)
    AH = 0.5 * (AH + AH.T)
    bH = VF.T @ (b[F] - AF @ up[F])
    c = spd_solve(AH, bH)
    uG = up + V @ c
    return CoarseResult(V, up, AH, bH, c, uG, lams)


def spd_solve(AH: np.ndarray, bH: np.ndarray, rtol: float = 1e-13) -> np.ndarray:
    """Cholesky solve; eigen-truncated pseudo-solve when A^H is numerically singular."""
    try:
        return sla.cho_solve(sla.cho_factor(AH, lower=True), bH)
    except np.linalg.LinAlgError:
        w, U = np.linalg.eigh(AH)
        keep = w > rtol * w.max()
        return U[:, keep] @ ((U[:, keep].T @ bH) / w[keep])


def energy_error(prob, A, uh: np.ndarray, uG: np.ndarray) -> float:
    """e_a = ||u_h - u^G||_A / ||u_h||_A over the free DoFs."""
    F = free_dofs(prob)
    AF = A[F][:, F]
    e = (uh - uG)[F]
    return float(np.sqrt(e @ (AF @ e)) / np.sqrt(uh[F] @ (AF @ uh[F])))


def select_modes(lam, t: float) -> int:
    """m_j for the threshold t on reciprocal local eigenvalues (Sec. 1, Sec. 5).

    The local space keeps the eigenvectors whose eigenvalue is below 1/t, so
    that the smallest excluded eigenvalue lambda^{j,m_j+1} of the error bound
    of Sec. 3.3 is at least 1/t.  The zero eigenvalues of a floating box (an
    infinite reciprocal) count as long as their rounding stays below 1/t.
    """
    if not t > 0:
        raise ValueError("threshold t must be positive")
    return int(np.count_nonzero(np.asarray(lam, dtype=np.float64) < 1.0 / t))


def error_norms(prob, uh: np.ndarray, u: np.ndarray) -> dict:
    """e_d and e_eps of Sec. 5.3: relative L2 errors of displacement and strain.

    Both are integrals over the mesh of the trilinear fields, by the 2x2x2
    Gauss rule of the element stiffness; the strain is the symmetric gradient
    with its Frobenius norm.  Returns the four integrals and the two ratios.
    """
    pts, wts = fem.gauss_rule(2)
    sums = np.zeros(4)
    for i, j, k in fem.box_elements((0, 0, 0), (prob.nx, prob.ny, prob.nz)):
        ids = fem.element_nodes(prob, i, j, k)
        X = prob.xyz[ids]
        R = uh.reshape(-1, 3)[ids]
        D = R - u.reshape(-1, 3)[ids]
        for xi, w in zip(pts, wts):
            N = np.prod(1.0 + fem.REF * xi, axis=1) / 8.0
            dN = fem.shape_grad_ref(xi)
            J = dN.T @ X
            dNdx = np.linalg.solve(J, dN.T).T
            wd = w * abs(np.linalg.det(J))
            for q, F in ((0, D), (1, R)):
                v = N @ F
                G = F.T @ dNdx                      # G[c, e] = d u_c / d x_e
                E = 0.5 * (G + G.T)
                sums[q] += wd * (v @ v)
                sums[2 + q] += wd * np.sum(E * E)
    e_d = np.sqrt(sums[0] / sums[1])
    e_eps = np.sqrt(sums[2] / sums[3])
    return {"sums": sums, "e_d": float(e_d), "e_eps": float(e_eps)}
