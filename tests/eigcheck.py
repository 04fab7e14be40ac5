"""Checks of GPU eigenpairs against the oracle's matrices (test-side helpers).

The library reports, per pair, a residual rho that it computes itself.  These
helpers recompute everything a GPU pair claims from the oracle's dense
Schur matrices of the same subdomain (Sec. 3.3; its matrix form Sec. 4.3):
M = E^T B11 E and T = S + s M on B2, taking only the B2 block x of each GPU
eigenvector phi = (E x, x, 0) (rho is scale-free, so the normalisation of phi
does not matter):

* ``oracle_rho``: rho = |M x - nu T x| / (|M x| + nu |T x|) with nu = 1/(lambda + s)
  the GPU's eigenvalue;
* ``davis_kahan``: the largest principal angle, in the T inner product,
  between the span of the GPU's first q vectors and the oracle's invariant
  subspace of the q largest nu, against the sin-theta bound of Davis and
  Kahan.  In the standard form C = L^{-1} M L^{-T} (T = L L^T) the GPU block
  becomes Y = L^T X_T (X_T the T-orthonormalised block), its Rayleigh
  quotient H = X_T^T M X_T and its residual R = L^{-1} (M X_T - T X_T H);
  with delta = (smallest eigenvalue of H) - nu_{q+1} > 0,
  |sin Theta|_2 <= |sin Theta|_F <= |R|_F / delta.  Everything in the bound
  comes from the oracle's matrices, nothing from the library's residuals.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from oracle import gevp


def oracle_rho(ref: "gevp.GevpResult", i2: np.ndarray, lam: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """rho of every GPU pair (lam[c], phi[:, c]) from the oracle's M and T."""
    T = ref.S + ref.s * ref.M
    nu = 1.0 / (lam + ref.s)
    X = phi[i2]
    return np.array([gevp.nu_residual(ref.M, T, float(nu[c]), X[:, c]) for c in range(lam.size)])


def check_rho(ref, i2, lam, phi, rho_gpu, tol=1e-6):
    """Asserts oracle rho <= tol for every pair and agreement with the reported rho.

    Both sides evaluate the same quantity in FP64 on the same vector; they
    differ by the rounding of M x and T x (about 1e-15 of |M x| + nu |T x|,
    times the growth of the dense products), so the reported rho must match
    to 1e-3 of its size plus 1e-11."""
    r = oracle_rho(ref, i2, lam, phi)
    assert np.all(r <= tol), r
    assert np.all(np.abs(r - rho_gpu) <= 1e-3 * np.maximum(r, rho_gpu) + 1e-11), (r, rho_gpu)
    return r


def davis_kahan_mt(M, T, X, Xref, nu_next: float):
    """(angle, bound) for a block X against the T-orthonormal block Xref of the
    pencil M x = nu T x; see the module docstring."""
    L = sla.cholesky(T, lower=True)
    G = X.T @ T @ X
    Rg = sla.cholesky(0.5 * (G + G.T), lower=False)
    Xt = sla.solve_triangular(Rg, X.T, trans="T", lower=False).T        # X Rg^{-1}: T-orthonormal
    H = Xt.T @ M @ Xt
    H = 0.5 * (H + H.T)
    theta = np.linalg.eigvalsh(H)
    R = sla.solve_triangular(L, M @ Xt - T @ Xt @ H, lower=True)
    delta = theta.min() - nu_next
    ang = float(np.max(sla.subspace_angles(L.T @ Xt, L.T @ Xref)))
    bound = np.linalg.norm(R) / delta if delta > 0 else np.inf
    return ang, bound


def davis_kahan(ref, i2: np.ndarray, phi: np.ndarray, q: int, nu_next: float):
    """(angle, bound) for the first q GPU vectors of the A-harmonic pencil."""
    return davis_kahan_mt(ref.M, ref.S + ref.s * ref.M, phi[i2][:, :q], ref.x[:, :q], nu_next)


def check_subspaces(ref, i2, phi, n_ev, min_gap=1e-3, say=print):
    """Davis-Kahan at every cut q <= n_ev where the oracle's relative gap exceeds
    min_gap (ref must hold at least n_ev + 1 pairs).  The angle's own rounding
    (about 1e-12 for these sizes) is allowed on top of the bound."""
    nu = ref.nu
    gaps = (nu[:n_ev] - nu[1:n_ev + 1]) / nu[:n_ev]
    cuts = [c + 1 for c in range(n_ev) if gaps[c] > min_gap]
    out = []
    for q in cuts:
        ang, bound = davis_kahan(ref, i2, phi, q, float(nu[q]))
        out.append((q, ang, bound))
        assert np.sin(ang) <= bound + 1e-10, (q, ang, bound)
    if out:
        q, ang, bound = out[-1]
        say(f"    T-angle of the first {q}: {ang:.2e} (Davis-Kahan bound {bound:.1e}; {len(out)} cuts checked)")
    return out
