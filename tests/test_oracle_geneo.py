"""Pins of the oracle's classic GenEO eigenproblem (Sec. 3.2), CPU only.

The GenEO pencil on Omega_j is a(phi, v) = lambda a(Xi phi, Xi v) over the
non-Dirichlet DoFs of the closed Omega_j box, with Xi = diag(mu_j).  The
oracle solves it as B x = nu (A + s B) x, B = D A D.  These tests fix that
answer without re-deriving it from the same code:

* the literal pencil (A, D A D) solved by QZ on a tiny box has the same finite
  eigenvalues (pins the shift trick and the ordering);
* exactly 3 |P| eigenvalues equal 1, P = the nodes whose whole 27-point
  neighbourhood carries mu_j = 1: a vector supported on P has D phi = phi and
  A phi supported where mu = 1, so A phi = D A D phi (the lambda = 1 cluster
  that Sec. 3.2 names as the limit of lambda^{j, m_j + 1}); a wrong D, a
  wrong partition of unity or a wrong box changes the count;
* Courant-Fischer: with no oversampling (Omega_j^* = Omega_j) the A-harmonic
  space is a subspace of V_h(Omega_j) and both pencils share both forms, so
  every A-harmonic lambda_k is at least the GenEO lambda_k;
* the result does not depend on the oversampling (GenEO lives on Omega_j);
* a floating subdomain has exactly the six rigid-body zeros, a clamped one
  none (Dirichlet DoFs removed).
"""
import numpy as np
import scipy.linalg as sla

from oracle import decomp, fem, geneo, gevp
from paper_2211_13893_amd import synth


def _full_geneo_spectrum(prob, j, s=1.0):
    """Every eigenvalue of the GenEO pencil of subdomain j (lambda = 1/nu - s), ascending."""
    elo, ehi = prob.omega_box(j)
    A = fem.assemble_box_dense(prob, elo, ehi)
    gd, _, mu = geneo.omega_dofs(prob, j)
    keep = np.flatnonzero(prob.dirichlet[gd] == 0)
    Ak = A[np.ix_(keep, keep)]
    d = mu[keep]
    B = d[:, None] * Ak * d[None, :]
    nu = sla.eigh(B, Ak + s * B, eigvals_only=True)
    with np.errstate(divide="ignore"):
        lam = 1.0 / nu - s
    return np.sort(lam), A, gd, mu, keep


def test_geneo_matches_literal_pencil_qz():
    p = synth.small_box(n=4, core=2, overlap=1, ovs=1, n_ev=8, seed=2)
    j = 3
    lam, *_ = geneo.geneo_local(p, j, 12)
    elo, ehi = p.omega_box(j)
    A = fem.assemble_box_dense(p, elo, ehi)
    gd, _, mu = geneo.omega_dofs(p, j)
    keep = np.flatnonzero(p.dirichlet[gd] == 0)
    Ak = A[np.ix_(keep, keep)]
    d = mu[keep]
    alpha, beta = sla.eig(Ak, d[:, None] * Ak * d[None, :], right=False, homogeneous_eigvals=True)
    fin = np.abs(beta) > 1e-9 * (np.abs(alpha) + np.abs(beta))
    lq = np.sort((alpha[fin] / beta[fin]).real)
    # the six rigid-body zeros are ill-conditioned in the literal pencil (0/0
    # is avoided by the shift); compare them in absolute terms
    assert np.all(np.abs(lq[:6]) <= 1e-8) and np.all(np.abs(lam[:6]) <= 1e-8)
    rel = np.abs(lq[6:12] - lam[6:12]) / lam[6:12]
    assert rel.max() <= 1e-9, rel


def _mu_one_neighbourhood_nodes(prob, j, mu):
    elo, ehi = prob.omega_box(j)
    nlo, nhi = decomp.node_box(elo, ehi)
    mx, my, mz = decomp.box_shape(nlo, nhi)
    m = mu[::3].reshape(mz, my, mx) == 1.0
    cnt = 0
    for k in range(mz):
        for jj in range(my):
            for i in range(mx):
                if m[max(k - 1, 0):k + 2, max(jj - 1, 0):jj + 2, max(i - 1, 0):i + 2].all():
                    cnt += 1
    return cnt


def test_geneo_lambda_one_cluster():
    # 12^3 mesh, 6^3 cores, overlap 2: each Omega_j holds a block of nodes with
    # mu = 1 whose neighbours also have mu = 1
    p = synth.small_box(n=12, core=6, overlap=2, ovs=1, n_ev=8, seed=1)
    for j in (0, 5):
        lam, _, _, mu, _ = _full_geneo_spectrum(p, j)
        n_p = _mu_one_neighbourhood_nodes(p, j, mu)
        n_one = int(np.sum(np.abs(lam - 1.0) <= 1e-8))
        assert n_p > 0
        assert n_one == 3 * n_p, (j, n_one, n_p)


def test_courant_fischer_aharmonic_above_geneo():
    # ovs = 0: Omega_j^* = Omega_j, V_A is a subspace of V_h(Omega_j)
    for n, core, ov, clamp in ((6, 2, 1, False), (8, 4, 1, False), (8, 4, 2, False), (8, 4, 1, True)):
        p = synth.small_box(n=n, core=core, overlap=ov, ovs=0, n_ev=12, seed=3, clamp=clamp)
        for j in range(min(p.nsd, 4)):
            ref = gevp.schur_gevp(gevp.local_ops(p, j), 12)
            lg, *_ = geneo.geneo_local(p, j, 12)
            assert np.all(ref.lam >= lg - 1e-9 * np.maximum(1.0, np.abs(lg))), (n, core, ov, j)


def test_geneo_independent_of_oversampling():
    a = synth.small_box(n=8, core=4, overlap=1, ovs=0, n_ev=8, seed=4)
    b = synth.small_box(n=8, core=4, overlap=1, ovs=2, n_ev=8, seed=4)
    for j in (0, 7):
        la, pa, *_ = geneo.geneo_local(a, j, 10)
        lb, pb, *_ = geneo.geneo_local(b, j, 10)
        assert np.array_equal(la, lb) and np.array_equal(pa, pb)


def test_geneo_rigid_modes_floating_and_clamped():
    fl = synth.small_box(n=8, core=4, overlap=1, ovs=1, n_ev=8, seed=5)
    lam, *_ = geneo.geneo_local(fl, 0, 10)
    assert np.sum(np.abs(lam) <= 1e-8) == 6 and lam[6] > 1e-3
    cl = synth.small_box(n=8, core=4, overlap=1, ovs=1, n_ev=8, seed=5, clamp=True)
    lam, *_ = geneo.geneo_local(cl, 0, 10)      # core 0 touches the clamped face x = 0
    assert lam[0] > 1e-3


def test_geneo_coarse_approximation_all_modes_recovers_fine_solution():
    # every GenEO eigenvector kept: sum_j R_j^T Xi_j V_h(Omega_j) = V_h, so u^G = u_h
    from oracle import coarse
    p = synth.small_box(n=4, core=2, overlap=1, ovs=1, n_ev=8, seed=3, clamp=True)
    A = fem.assemble_global_sparse(p)
    b = fem.traction_load(p)
    uh = coarse.fine_solve(p, A, b)
    n_all = []
    for j in range(p.nsd):
        gd, _, _ = geneo.omega_dofs(p, j)
        n_all.append(int(np.sum(p.dirichlet[gd] == 0)))
    res = geneo.geneo_msgfem(p, n_all, A, b)
    assert coarse.energy_error(p, A, uh, res.uG) <= 1e-8


def test_geneo_coarse_approximation_galerkin_and_nested():
    from oracle import coarse
    p = synth.laminated_beam()
    A = fem.assemble_global_sparse(p)
    b = fem.traction_load(p)
    uh = coarse.fine_solve(p, A, b)
    F = coarse.free_dofs(p)
    AF = A[F][:, F]
    prev = np.inf
    for n in (4, 8, 12):
        res = geneo.geneo_msgfem(p, n, A, b)
        g = res.V[F].T @ (AF @ (uh - res.uG)[F])
        assert np.abs(g).max() <= 1e-9 * np.abs(res.V[F].T @ (AF @ uh[F])).max()
        ea = coarse.energy_error(p, A, uh, res.uG)
        assert ea <= prev * (1 + 1e-12)
        prev = ea
