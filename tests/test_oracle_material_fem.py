"""Pins of the oracle's material tensors, element matrices and assembly (CPU).

Every check here is fixed by mathematics independent of the oracle's own
code: lamina closed forms, Lame's isotropic tensor, rigid-body null spaces,
exact energies of linear fields, exact symbolic integration, the patch test
and the closed-form solution of a bar under uniform traction (Sec. 2, 5.1).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import coarse, fem, material
from paper_2211_13893_amd import synth

PLY = list(synth.PLY_CONSTANTS)


def _ex_closed(theta_deg, E1=162000.0, E2=10000.0, G12=5200.0, n12=0.35):
    """Standard lamina transformation: 1/E_x(t) = c^4/E1 + (1/G12 - 2 n12/E1) s^2 c^2 + s^4/E2."""
    t = np.deg2rad(theta_deg)
    c, s = np.cos(t), np.sin(t)
    return 1.0 / (c ** 4 / E1 + (1.0 / G12 - 2.0 * n12 / E1) * s * s * c * c + s ** 4 / E2)


@pytest.mark.parametrize("theta", [0.0, 30.0, 45.0, -45.0, 90.0, 17.5])
def test_rotated_ply_axial_modulus_closed_form(theta):
    C = material.material_C(PLY + [theta])
    Sg = np.linalg.inv(C)
    assert abs(1.0 / Sg[0, 0] - _ex_closed(theta)) <= 1e-10 * _ex_closed(theta)


def test_ply_tensor_spd_and_symmetries():
    C0 = material.material_C(PLY + [0.0])
    assert np.allclose(C0, C0.T, rtol=0, atol=1e-9)
    w = np.linalg.eigvalsh(C0)
    assert w.min() > 0
    # smallest eigenvalue of the unrotated ply is the transverse shear modulus G23
    assert abs(w.min() - 3500.0) < 1e-8
    # 90 degrees equals 0 degrees with axes 1 and 2 swapped (Voigt 11<->22, 23<->13)
    C90 = material.material_C(PLY + [90.0])
    perm = [1, 0, 2, 4, 3, 5]
    assert np.allclose(C90, C0[np.ix_(perm, perm)], rtol=1e-12, atol=1e-7)
    for t in (0.0, 30.0, 45.0, -60.0):
        Ct = material.material_C(PLY + [t])
        assert np.allclose(Ct, material.material_C(PLY + [t + 180.0]), rtol=1e-12, atol=1e-7)
        # Mandel-form eigenvalues are rotation invariant
        m = np.array([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
        # engineering-shear Voigt stiffness -> Mandel: C_M = diag(m) C diag(m) / ... for stiffness:
        CM = Ct * np.outer(m, m)
        CM0 = C0 * np.outer(m, m)
        assert np.allclose(np.linalg.eigvalsh(CM), np.linalg.eigvalsh(CM0), rtol=1e-11)


def test_isotropic_matches_lame():
    E, nu = 3000.0, 0.35
    C = material.material_C(list(synth.isotropic_constants(E, nu)) + [0.0])
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    ref = np.zeros((6, 6))
    ref[:3, :3] = lam
    ref[[0, 1, 2], [0, 1, 2]] += 2 * mu
    ref[[3, 4, 5], [3, 4, 5]] = mu
    assert np.allclose(C, ref, rtol=1e-12, atol=1e-9)


def _rigid_modes(X):
    R = np.zeros((24, 6))
    for a in range(8):
        x, y, z = X[a]
        R[3 * a:3 * a + 3, 0:3] = np.eye(3)
        R[3 * a:3 * a + 3, 3] = [-y, x, 0]
        R[3 * a:3 * a + 3, 4] = [z, 0, -x]
        R[3 * a:3 * a + 3, 5] = [0, -z, y]
    return R


def _distorted_hex(rng):
    X = (fem.REF + 1.0) / 2.0 * np.array([1.3, 0.8, 0.25])
    return X + 0.06 * rng.standard_normal(X.shape)


def test_element_stiffness_null_space_and_spectrum():
    rng = np.random.default_rng(1)
    X = _distorted_hex(rng)
    C = material.material_C(PLY + [30.0])
    Ke = fem.element_stiffness(X, C)
    assert np.abs(Ke - Ke.T).max() <= 1e-15 * np.abs(Ke).max() * 24
    w = np.linalg.eigvalsh(Ke)
    assert np.all(np.abs(w[:6]) <= 1e-12 * w[-1])
    assert w[6] > 1e-6 * w[-1]
    R = _rigid_modes(X)
    assert np.abs(Ke @ R).max() <= 1e-12 * np.abs(Ke).max() * np.abs(R).max()
    # homogeneity: Ke(alpha x) = alpha Ke(x) in 3D
    assert np.allclose(fem.element_stiffness(2.5 * X, C), 2.5 * Ke, rtol=1e-12, atol=1e-9)


def test_linear_field_energy_is_exact():
    """0.5 u^T Ke u = 0.5 eps:C:eps |e| for u = G x (Lame tensor, parallelepiped volume)."""
    rng = np.random.default_rng(2)
    E, nu = 3000.0, 0.35
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    C = material.material_C(list(synth.isotropic_constants(E, nu)) + [0.0])
    Aff = np.array([[1.2, 0.1, 0.05], [0.2, 0.9, -0.1], [0.0, 0.15, 0.4]])
    X = ((fem.REF + 1.0) / 2.0) @ Aff.T + np.array([3.0, -1.0, 2.0])
    vol = abs(np.linalg.det(Aff))
    Ke = fem.element_stiffness(X, C)
    for _ in range(5):
        G = rng.standard_normal((3, 3))
        u = (X @ G.T).ravel()
        eps = 0.5 * (G + G.T)
        energy = 0.5 * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps)) * vol
        assert abs(0.5 * u @ Ke @ u - energy) <= 1e-11 * energy


def test_element_stiffness_matches_exact_symbolic_integral():
    """Affine element: exact sympy integration of B^T C B det J over the reference cube."""
    sympy = pytest.importorskip("sympy")
    xi, eta, zeta = sympy.symbols("xi eta zeta")
    Aff = sympy.Matrix([[sympy.Rational(3, 2), 0, sympy.Rational(1, 5)],
                        [0, 1, 0], [sympy.Rational(1, 10), 0, sympy.Rational(1, 2)]])
    E, nu = sympy.Integer(3000), sympy.Rational(7, 20)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    Cs = sympy.zeros(6, 6)
    for i in range(3):
        for j in range(3):
            Cs[i, j] = lam
        Cs[i, i] += 2 * mu
        Cs[i + 3, i + 3] = mu
    # x = Aff (xi+1)/2 ; grad_x N = (dxi/dx)^T grad_xi N, dxi/dx = 2 Aff^{-1}
    Jinv = 2 * Aff.inv()
    detJ = Aff.det() / 8
    N = []
    for a in range(8):
        r = [2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
        N.append((1 + r[0] * xi) * (1 + r[1] * eta) * (1 + r[2] * zeta) / 8)
    B = sympy.zeros(6, 24)
    for a in range(8):
        g_ref = sympy.Matrix([sympy.diff(N[a], v) for v in (xi, eta, zeta)])
        gx, gy, gz = list(Jinv.T * g_ref)
        c = 3 * a
        B[0, c], B[1, c + 1], B[2, c + 2] = gx, gy, gz
        B[3, c + 1], B[3, c + 2] = gz, gy
        B[4, c], B[4, c + 2] = gz, gx
        B[5, c], B[5, c + 1] = gy, gx
    integrand = (B.T * Cs * B) * detJ
    rows = [0, 4, 13, 23]
    X = ((fem.REF + 1.0) / 2.0) @ np.array(Aff.tolist(), dtype=float).T
    Ke = fem.element_stiffness(X, material.material_C([3000.0, 3000.0, 3000.0, 3000 / 2.7, 3000 / 2.7,
                                                        3000 / 2.7, 0.35, 0.35, 0.35, 0.0]))
    for r in rows:
        for c in range(24):
            ex = sympy.integrate(sympy.expand(integrand[r, c]), (xi, -1, 1), (eta, -1, 1), (zeta, -1, 1))
            assert abs(float(ex) - Ke[r, c]) <= 1e-10 * np.abs(Ke).max()


def test_patch_test_wrinkled_mesh():
    """Homogeneous material, u = G x + c on the boundary: the interior reproduces it exactly."""
    p = synth.small_box(n=5, core=5, material="iso", wrinkle=0.7)
    A = fem.assemble_global_sparse(p).tocsr()
    rng = np.random.default_rng(3)
    G = rng.standard_normal((3, 3))
    c = rng.standard_normal(3)
    u_ex = (p.xyz @ G.T + c).ravel()
    nn = p.nx + 1
    I = np.arange(p.n_nodes) % nn
    J = (np.arange(p.n_nodes) // nn) % nn
    K = np.arange(p.n_nodes) // (nn * nn)
    bnd = (I == 0) | (I == p.nx) | (J == 0) | (J == p.ny) | (K == 0) | (K == p.nz)
    bd = np.repeat(bnd, 3)
    F, D = np.flatnonzero(~bd), np.flatnonzero(bd)
    u = u_ex.copy()
    u[F] = spla.spsolve(A[F][:, F].tocsc(), -A[F][:, D] @ u_ex[D])
    assert np.abs(u[F] - u_ex[F]).max() <= 1e-10 * np.abs(u_ex).max()


def test_traction_load_total_force():
    p = synth.laminated_beam()
    b = fem.traction_load(p)
    assert np.allclose(b.reshape(-1, 3).sum(0), [-10.0 * 36.0, 0.0, 0.0], rtol=1e-13, atol=1e-9)


@pytest.mark.parametrize("theta", [0.0, 30.0])
def test_bar_under_uniform_traction_closed_form(theta):
    """Roller-supported homogeneous ply bar, -10 MPa on x=48: sigma_xx uniform, u linear.

    Delta u_x over the length equals -10 * 48 / E_x(theta) (lamina closed form).
    """
    p = synth.laminated_beam(material="ply", theta=theta, roller=True)
    u = coarse.fine_solve(p)
    U = u.reshape(-1, 3)
    nn = p.nx + 1
    I = np.arange(p.n_nodes) % nn
    du = U[I == p.nx, 0] - U[I == 0, 0]
    expect = -10.0 * 48.0 / _ex_closed(theta)
    assert np.abs(du - expect).max() <= 1e-9 * abs(expect)
    # the whole field is linear in x: fit and check the residual
    Xh = np.hstack([p.xyz, np.ones((p.n_nodes, 1))])
    coef, *_ = np.linalg.lstsq(Xh, U, rcond=None)
    assert np.abs(Xh @ coef - U).max() <= 1e-9 * np.abs(U).max()
