"""The A-harmonic local generalized eigenproblem (oracle; test infrastructure).

Sec. 3.3 defines, on each oversampling domain Omega_j^*, the GEVP
a_{Omega*}(phi, v) = lambda a_{Omega*}(Xi phi, Xi v) for phi, v in the
A-harmonic space V_A (functions of V_{h,D} whose energy is orthogonal to
V_{h,DI}); eigenvalues ascending, the m_j smallest kept.  Sec. 3.3 (mixed
form) and Sec. 4.3 (its matrix form) impose A-harmonicity with a Lagrange
multiplier: the (2 n1 + n2) pencil
    [[A11, A12, A11], [A21, A22, A21], [A11, A12, 0]] (phi1, phi2, p)
        = lambda diag(B11, 0, 0) (phi1, phi2, p),
with A the Omega^*-stiffness with B3 rows/columns removed and
B11 = a(Xi phi_k, Xi phi_l) over B1, i.e. D A D on B1 with D = diag(mu).

Exact reduction (used by ``schur_gevp``): the third block row gives
phi1 = E phi2 with E = -A11^{-1} A12 (the A-harmonic extension), the first
gives p = lambda A11^{-1} B11 phi1, and the second then reads
S phi2 = lambda M phi2 with S = A22 - A21 A11^{-1} A12 (interior Schur
complement) and M = E^T B11 E.  Both S and M may be singular (rigid modes,
vanishing partition of unity), so the oracle solves the equivalent definite
pencil M x = nu T x, T = S + s M (s > 0), nu = 1 / (lambda + s), keeping the
n_ev largest nu.  ``augmented_gevp`` solves the literal pencil by QZ and pins
the reduction on tiny boxes.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import decomp, fem


@dataclasses.dataclass
class LocalOps:
    A: np.ndarray       # dense Omega^* stiffness, all DoFs of the node box
    cls: np.ndarray     # 1/2/3 per DoF
    mu: np.ndarray      # PoU per DoF
    b: np.ndarray       # restriction of the load to Omega^* (per DoF of the box)

    @property
    def i1(self):
        return np.flatnonzero(self.cls == 1)

    @property
    def i2(self):
        return np.flatnonzero(self.cls == 2)


def local_ops(prob, j: int, kecache=None, load=None) -> LocalOps:
    """Dense a_{Omega_j^*}, DoF classes, PoU and restricted load of subdomain j."""
    elo, ehi = prob.omega_star_box(j)
    A = fem.assemble_box_dense(prob, elo, ehi, kecache)
    cls = decomp.dof_classes(prob, j)
    mu = decomp.pou_dofs(prob, j)
    if load is None:
        load = fem.traction_load(prob)
    b = load[decomp.star_global_dofs(prob, j)]
    return LocalOps(A, cls, mu, b)


@dataclasses.dataclass
class GevpResult:
    lam: np.ndarray        # ascending eigenvalues (n_ev)
    nu: np.ndarray         # 1 / (lam + s), descending
    phi: np.ndarray        # [n, n_ev] eigenvectors on all DoFs of Omega^* (0 on B3)
    x: np.ndarray          # [n2, n_ev] boundary coordinates (T-orthonormal)
    S: np.ndarray
    M: np.ndarray
    E: np.ndarray
    s: float


def reduce_schur(ops: LocalOps):
    """E = -A11^{-1} A12, S = A22 + A21 E, M = E^T B11 E (dense, FP64)."""
    i1, i2 = ops.i1, ops.i2
    A11 = ops.A[np.ix_(i1, i1)]
    A12 = ops.A[np.ix_(i1, i2)]
    A22 = ops.A[np.ix_(i2, i2)]
    c = sla.cho_factor(A11, lower=True)
    E = -sla.cho_solve(c, A12)
    S = A22 + A12.T @ E
    d1 = ops.mu[i1]
    B11 = d1[:, None] * A11 * d1[None, :]
    M = E.T @ B11 @ E
    S = 0.5 * (S + S.T)
    M = 0.5 * (M + M.T)
    return E, S, M


def normalise_sign(phi: np.ndarray) -> np.ndarray:
    """Unit 2-norm columns whose entry of largest magnitude is positive."""
    phi = phi / np.linalg.norm(phi, axis=0, keepdims=True)
    idx = np.argmax(np.abs(phi), axis=0)
    sg = np.sign(phi[idx, np.arange(phi.shape[1])])
    sg[sg == 0] = 1.0
    return phi * sg


def schur_gevp(ops: LocalOps, n_ev: int | None, s: float = 1.0) -> GevpResult:
    """The n_ev smallest eigenpairs of S x = lambda M x via M x = nu (S + s M) x."""
    i1, i2 = ops.i1, ops.i2
    E, S, M = reduce_schur(ops)
    T = S + s * M
    nu, X = sla.eigh(M, T)                 # ascending nu, X^T T X = I
    order = np.argsort(-nu)
    nu, X = nu[order], X[:, order]
    if n_ev is not None:
        nu, X = nu[:n_ev], X[:, :n_ev]
    lam = 1.0 / nu - s
    n = ops.A.shape[0]
    phi = np.zeros((n, X.shape[1]))
    phi[i1] = E @ X
    phi[i2] = X
    return GevpResult(lam, nu, normalise_sign(phi), X, S, M, E, s)


def augmented_gevp(ops: LocalOps):
    """Finite eigenvalues of the literal (2 n1 + n2) mixed pencil, by QZ (tiny boxes only)."""
    i1, i2 = ops.i1, ops.i2
    n1, n2 = i1.size, i2.size
    A11 = ops.A[np.ix_(i1, i1)]
    A12 = ops.A[np.ix_(i1, i2)]
    A21 = ops.A[np.ix_(i2, i1)]
    A22 = ops.A[np.ix_(i2, i2)]
    d1 = ops.mu[i1]
    B11 = d1[:, None] * A11 * d1[None, :]
    N = 2 * n1 + n2
    K = np.zeros((N, N))
    K[:n1, :n1] = A11
    K[:n1, n1:n1 + n2] = A12
    K[:n1, n1 + n2:] = A11
    K[n1:n1 + n2, :n1] = A21
    K[n1:n1 + n2, n1:n1 + n2] = A22
    K[n1:n1 + n2, n1 + n2:] = A21
    K[n1 + n2:, :n1] = A11
    K[n1 + n2:, n1:n1 + n2] = A12
    Bf = np.zeros((N, N))
    Bf[:n1, :n1] = B11
    w = sla.eig(K, Bf, right=False, homogeneous_eigvals=True)
    alpha, beta = w[0], w[1]
    scale = np.abs(alpha) + np.abs(beta)
    finite = np.abs(beta) > 1e-9 * scale
    lam = (alpha[finite] / beta[finite])
    return np.sort(lam.real), lam


def nu_residual(M: np.ndarray, T: np.ndarray, nu: float, x: np.ndarray) -> float:
    """rho = ||M x - nu T x|| / (||M x|| + nu ||T x||) (scale-free, defined for rigid modes)."""
    Mx, Tx = M @ x, T @ x
    return float(np.linalg.norm(Mx - nu * Tx) / (np.linalg.norm(Mx) + nu * np.linalg.norm(Tx)))


def harmonic_residual(ops: LocalOps, phi: np.ndarray) -> float:
    """||(A phi)_{B1}|| / ||(|A| |phi|)_{B1}||: A-harmonicity of a full-box vector."""
    i1 = ops.i1
    r = (ops.A @ phi)[i1]
    d = (np.abs(ops.A) @ np.abs(phi))[i1]
    return float(np.linalg.norm(r) / np.linalg.norm(d))


def subspace_angle(P: np.ndarray, Q: np.ndarray) -> float:
    """Largest principal angle (radians) between span P and span Q."""
    return float(np.max(sla.subspace_angles(P, Q)))
