"""Pins of the oracle's subdomains, partition of unity and local GEVP (CPU).

Sec. 3.1 / 4.2 / 4.3 fix the DoF classes and the partition of unity; Sec. 3.3
and 4.3 fix the eigenproblem.  The reduction to the interior Schur complement
is pinned by the literal mixed (2 n1 + n2) pencil solved by QZ and by a
30-digit mpmath solve; Sec. 5.2 states that subdomains away from the
Dirichlet boundary have exactly six zero eigenvalues (rigid-body modes).
"""
import os

import numpy as np
import pytest

from oracle import decomp, fem, gevp
from paper_2211_13893_amd import synth


def test_beam_dof_classes_exact():
    p = synth.laminated_beam()
    counts = [[int((decomp.dof_classes(p, j) == c).sum()) for c in (1, 2, 3)] for j in range(4)]
    # Omega^* x-ranges [0,16], [8,28], [20,40], [32,48] of a 7x7 node cross-section
    assert counts == [[2205, 147, 147], [2793, 294, 0], [2793, 294, 0], [2352, 147, 0]]


def test_uniform_batch_box_sizes():
    p = synth.uniform_batch(n_boxes=2)
    for j in p.batch:
        cls = decomp.dof_classes(p, int(j))
        assert cls.size == 10125
        assert int((cls == 1).sum()) == 3 * 13 ** 3 == 6591
        assert int((cls == 2).sum()) == 3534
        assert int((cls == 3).sum()) == 0


def test_beam_pou_ramp_closed_form():
    """o=2: mu_0 falls linearly from 1 at x=10 to 0 at x=14 (2o = 4 element overlap)."""
    p = synth.laminated_beam()
    mu = decomp.pou_nodes(p, 0)
    nlo, nhi = decomp.node_box(*p.omega_star_box(0))
    I, J, K = decomp.local_node_grid(nlo, nhi)
    for x in range(17):
        vals = mu[I == x]
        expect = 1.0 if x <= 10 else max(0.0, (14 - x) / 4.0)
        assert np.allclose(vals, expect, atol=1e-15)


@pytest.mark.parametrize("maker", [lambda: synth.laminated_beam(),
                                   lambda: synth.small_box(n=7, core=2, overlap=1, ovs=1),
                                   lambda: synth.small_box(n=9, core=3, overlap=2, ovs=1),
                                   lambda: synth.uneven_laminate(nx=30, ny=14, nz=12)])
def test_pou_sums_to_one(maker):
    p = maker()
    total = np.zeros(p.n_nodes)
    for j in range(p.nsd):
        mu = decomp.pou_global(p, j)
        assert mu.min() >= 0.0 and mu.max() <= 1.0
        total += mu
        # zero outside Omega_j
        elo, ehi = p.omega_box(j)
        nn = (p.nx + 1, p.ny + 1)
        idx = np.arange(p.n_nodes)
        I, J, K = idx % nn[0], (idx // nn[0]) % nn[1], idx // (nn[0] * nn[1])
        out = (I < elo[0]) | (I > ehi[0]) | (J < elo[1]) | (J > ehi[1]) | (K < elo[2]) | (K > ehi[2])
        assert np.all(mu[out] == 0.0)
    assert np.abs(total - 1.0).max() <= 1e-15


def test_pou_weights_are_capped_chebyshev_distance():
    """The sweeps of Sec. 4.2 converge to min(2o, Chebyshev hops to the interior boundary)."""
    p = synth.small_box(n=12, core=4, overlap=2, ovs=1)
    for j in range(p.nsd):
        elo, ehi = p.omega_box(j)
        nlo, nhi = decomp.node_box(*p.omega_star_box(j))
        w = decomp.pou_weights_on_box(p, j, nlo, nhi)
        I, J, K = decomp.local_node_grid(nlo, nhi)
        N = (p.nx, p.ny, p.nz)
        d = np.full(I.shape, 2 * p.overlap, dtype=float)
        inside = np.ones(I.shape, bool)
        for ax, idx in enumerate((I, J, K)):
            inside &= (idx >= elo[ax]) & (idx <= ehi[ax])
            if elo[ax] > 0:
                d = np.minimum(d, idx - elo[ax])
            if ehi[ax] < N[ax]:
                d = np.minimum(d, ehi[ax] - idx)
        d = np.where(inside, d, 0.0)
        assert np.array_equal(w, d)


FLOAT_TILE = 2 + 5 * (2 + 5 * 2)   # tile (2,2,2) of a 10^3 mesh with 2^3 cores: interior box


@pytest.fixture(scope="module")
def tiny_floating():
    p = synth.small_box(n=10, core=2, overlap=1, ovs=1)
    return p, gevp.local_ops(p, FLOAT_TILE)


def test_schur_reduction_matches_literal_mixed_pencil(tiny_floating):
    p, ops = tiny_floating
    res = gevp.schur_gevp(ops, None)
    lam_aug, _ = gevp.augmented_gevp(ops)
    good = np.sort(res.lam[res.nu > 1e-12 * res.nu.max()])
    rank_m = np.linalg.matrix_rank(res.M, tol=1e-10 * np.abs(res.M).max())
    assert lam_aug.size == rank_m == good.size
    scale = np.maximum(1.0, np.abs(lam_aug))
    assert np.max(np.abs(good - lam_aug) / scale) <= 1e-10


def test_clamped_subdomain_matches_mixed_pencil():
    p = synth.small_box(n=8, core=2, overlap=1, ovs=1, clamp=True)
    j = 0 + 4 * (1 + 4 * 1)
    ops = gevp.local_ops(p, j)
    assert (ops.cls == 3).sum() > 0
    res = gevp.schur_gevp(ops, None)
    lam_aug, _ = gevp.augmented_gevp(ops)
    good = np.sort(res.lam[res.nu > 1e-12 * res.nu.max()])
    n = min(40, lam_aug.size)
    assert np.max(np.abs(good[:n] - lam_aug[:n]) / np.maximum(1.0, np.abs(lam_aug[:n]))) <= 1e-10
    # touching the clamp: no rigid-body zero modes
    assert good[0] > 1e-3


def test_six_rigid_modes_and_harmonicity(tiny_floating):
    p, ops = tiny_floating
    res = gevp.schur_gevp(ops, 12)
    assert np.all(np.abs(res.lam[:6]) <= 1e-8)
    assert res.lam[6] > 1e-3
    for k in range(12):
        assert gevp.harmonic_residual(ops, res.phi[:, k]) <= 1e-10
        assert gevp.nu_residual(res.M, res.S + res.s * res.M, res.nu[k], res.x[:, k]) <= 1e-12


def _golden(name):
    """key -> value table of a fixture under tests/golden/ ('#' lines are comments)."""
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    out = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = v
    return out


def test_beam_eigenvalues_rigid_modes_only_when_floating():
    # Sec. 5.2: six zero eigenvalues exactly when the box is floating
    g = _golden("rigid_modes.txt")
    p = synth.laminated_beam()
    kec = fem.KeCache(p)
    for j in range(4):
        res = gevp.schur_gevp(gevp.local_ops(p, j, kec), 10)
        nzero = int(np.sum(np.abs(res.lam) <= 1e-8))
        want = g["zero_eigenvalues_clamped"] if j == 0 else g["zero_eigenvalues_floating"]
        assert nzero == int(want)
        assert np.all(np.diff(res.lam) >= -1e-9)


def test_eigenvalues_invariant_under_scaling_and_shift(tiny_floating):
    p, ops = tiny_floating
    ref = gevp.schur_gevp(ops, 14)
    scaled = gevp.LocalOps(7.5 * ops.A, ops.cls, ops.mu, ops.b)
    r2 = gevp.schur_gevp(scaled, 14, s=0.3)
    assert np.allclose(r2.lam[6:], ref.lam[6:], rtol=1e-9)
    assert np.abs(r2.lam[:6]).max() <= 1e-7


def test_more_oversampling_raises_eigenvalues():
    """Sec. 5.2 / Thm. 3.2: larger oversampling -> faster growth of lambda_k."""
    lams = []
    for ovs in (0, 1, 2):
        p = synth.small_box(n=10, core=2, overlap=1, ovs=ovs, material="iso")
        j = 2 + 5 * (2 + 5 * 2)
        lams.append(gevp.schur_gevp(gevp.local_ops(p, j), 20).lam)
    for k in range(8, 20):
        assert lams[0][k] < lams[1][k] < lams[2][k]


@pytest.mark.slow
def test_fp64_eigenvalues_against_mpmath():
    """30-digit solve of the same pencil (nonzero nu via the 24x24 compressed form)."""
    mp = pytest.importorskip("mpmath")
    p = synth.small_box(n=5, core=1, overlap=1, ovs=0)
    j = 2 + 5 * (2 + 5 * 2)
    ops = gevp.local_ops(p, j)
    ref = gevp.schur_gevp(ops, None)
    mp.mp.dps = 30
    i1, i2 = ops.i1, ops.i2
    A = ops.A

    def mat(X):
        return mp.matrix(X.tolist())

    def msolve(Am, Bm):
        LU, piv = mp.mp.LU_decomp(Am.copy())
        out = mp.matrix(Bm.rows, Bm.cols)
        for c in range(Bm.cols):
            x = mp.mp.U_solve(LU, mp.mp.L_solve(LU, mp.matrix([Bm[r, c] for r in range(Bm.rows)]), piv))
            for r in range(Bm.rows):
                out[r, c] = x[r]
        return out

    A11, A12, A22 = mat(A[np.ix_(i1, i1)]), mat(A[np.ix_(i1, i2)]), mat(A[np.ix_(i2, i2)])
    E = -msolve(A11, A12)
    S = A22 + A12.T * E
    d = ops.mu[i1]
    B11 = mat(d[:, None] * A[np.ix_(i1, i1)] * d[None, :])
    M = E.T * B11 * E
    T = S + M
    w, U = mp.eigsy(B11)
    Bh = U * mp.diag([mp.sqrt(max(x, 0)) for x in w]) * U.T
    F = Bh * E
    G = F * msolve(T, F.T)
    nu = sorted([float(x) for x in mp.eigsy(G, eigvals_only=True)], reverse=True)
    k = 20
    assert np.max(np.abs(np.array(nu[:k]) - ref.nu[:k]) / ref.nu[:k]) <= 1e-11
