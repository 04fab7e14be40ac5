"""CPU checks of the eigenpair checks the GPU tests use (tests/eigcheck.py)."""
import numpy as np
import pytest

from oracle import gevp
from paper_2211_13893_amd import synth

import eigcheck


@pytest.fixture(scope="module")
def case():
    p = synth.small_box(n=8, core=2, overlap=1, ovs=1, n_ev=8, seed=6)
    ops = gevp.local_ops(p, 21)   # core (1, 1, 1): a floating interior box
    ref = gevp.schur_gevp(ops, 12)
    return ops, ref


def _phi_from_x(ref, ops, X):
    phi = np.zeros((ops.A.shape[0], X.shape[1]))
    phi[ops.i1] = ref.E @ X
    phi[ops.i2] = X
    return phi


def test_rho_of_exact_pairs(case):
    ops, ref = case
    r = eigcheck.oracle_rho(ref, ops.i2, ref.lam, ref.phi)
    assert r.max() <= 1e-12


def test_rho_detects_a_wrong_eigenvalue(case):
    ops, ref = case
    lam = ref.lam.copy()
    lam[7] *= 1.0 + 1e-3
    r = eigcheck.oracle_rho(ref, ops.i2, lam, ref.phi)
    assert r[7] > 1e-6 and np.delete(r, 7).max() <= 1e-12


def test_davis_kahan_holds_for_perturbed_vectors(case):
    ops, ref = case
    rng = np.random.default_rng(1)
    for eps in (1e-9, 1e-7, 1e-5):
        X = ref.x[:, :10] + eps * rng.standard_normal(ref.x[:, :10].shape) * np.abs(ref.x).max()
        phi = _phi_from_x(ref, ops, X)
        for q in (6, 8):
            ang, bound = eigcheck.davis_kahan(ref, ops.i2, phi, q, float(ref.nu[q]))
            assert 0.0 < np.sin(ang) <= bound
            assert bound < 1e3 * np.sin(ang)     # and not vacuous


def test_davis_kahan_flags_a_swapped_vector(case):
    ops, ref = case
    X = ref.x[:, :10].copy()
    X[:, 7] = ref.x[:, 11]          # an eigenvector outside the leading eight
    phi = _phi_from_x(ref, ops, X)
    ang, bound = eigcheck.davis_kahan(ref, ops.i2, phi, 8, float(ref.nu[8]))
    assert ang > 1.0                 # the subspaces differ by a whole direction
    assert not np.isfinite(bound) or np.sin(ang) <= bound
