"""Material tensors of the plies and the resin (oracle; test infrastructure).

Sec. 2 (generalized Hooke's law) takes a symmetric positive definite
fourth-order tensor C_ijkl per point; Sec. 5.1 models every ply as a
homogeneous orthotropic material given by nine engineering constants and
orients it in the global frame by a standard tensor rotation about the
laminate normal.  Voigt order (11, 22, 33, 23, 13, 12) with engineering shear
strains; the rotation is applied to the full fourth-order tensor, not to the
6x6 matrix.
"""
from __future__ import annotations

import numpy as np

VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def _voigt_index(i: int, j: int) -> int:
    return VOIGT.index((min(i, j), max(i, j)))


def compliance(consts) -> np.ndarray:
    """Orthotropic compliance (material frame) from E1..E3, G12, G13, G23, nu12, nu13, nu23."""
    E1, E2, E3, G12, G13, G23, n12, n13, n23 = [float(c) for c in consts[:9]]
    S = np.zeros((6, 6))
    S[0, 0], S[1, 1], S[2, 2] = 1.0 / E1, 1.0 / E2, 1.0 / E3
    S[0, 1] = S[1, 0] = -n12 / E1
    S[0, 2] = S[2, 0] = -n13 / E1
    S[1, 2] = S[2, 1] = -n23 / E2
    S[3, 3], S[4, 4], S[5, 5] = 1.0 / G23, 1.0 / G13, 1.0 / G12
    return S


def voigt_to_tensor(C6: np.ndarray) -> np.ndarray:
    """Stiffness 6x6 (engineering shear) -> C_ijkl (all minor/major symmetries)."""
    C = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    C[i, j, k, l] = C6[_voigt_index(i, j), _voigt_index(k, l)]
    return C


def tensor_to_voigt(C: np.ndarray) -> np.ndarray:
    C6 = np.zeros((6, 6))
    for I, (i, j) in enumerate(VOIGT):
        for J, (k, l) in enumerate(VOIGT):
            C6[I, J] = C[i, j, k, l]
    return C6


def rotation_z(theta_deg: float) -> np.ndarray:
    """Q maps material axes to global axes: fibre axis e1 -> (cos t, sin t, 0)."""
    t = np.deg2rad(theta_deg)
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rotate_tensor(C: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """C'_ijkl = Q_ip Q_jq Q_kr Q_ls C_pqrs."""
    return np.einsum("ip,jq,kr,ls,pqrs->ijkl", Q, Q, Q, Q, C)


def material_C(row) -> np.ndarray:
    """Global 6x6 stiffness of one material row (9 constants + ply angle in degrees)."""
    C6_mat = np.linalg.inv(compliance(row))
    C6_mat = 0.5 * (C6_mat + C6_mat.T)
    Ct = rotate_tensor(voigt_to_tensor(C6_mat), rotation_z(float(row[9])))
    return tensor_to_voigt(Ct)


def material_table(materials: np.ndarray) -> np.ndarray:
    """[n_mat, 6, 6] global stiffness matrices."""
    return np.stack([material_C(r) for r in materials])
