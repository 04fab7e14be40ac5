"""Q1 hexahedral linear elasticity (oracle; test infrastructure).

Sec. 2: strain eps = sym(grad u), stress sigma = C : eps, bilinear form
a(u, v) = integral of sigma(u) : eps(v), load b(v) = integral over Gamma_N of
g . v (f = 0 in every workload), assembled element by element, a = sum_e a_e,
and restricted to a mesh-resolved region D as a_D = sum over e in D of a_e.
Sec. 5.1 uses piecewise-(tri)linear hexahedra with one element per layer.
The element integral here uses the full 2x2x2 Gauss-Legendre rule (the
reduced rule mentioned in Sec. 5.1 would add hourglass zero modes and leave
the interior block of a floating subdomain singular).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import material

# reference coordinates of the 8 local nodes, a = di + 2 dj + 4 dk
REF = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
                for a in range(8)], dtype=np.float64)


def gauss_rule(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    pts, wts = [], []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                pts.append([x[i], x[j], x[k]])
                wts.append(w[i] * w[j] * w[k])
    return np.array(pts), np.array(wts)


def shape_grad_ref(xi: np.ndarray) -> np.ndarray:
    """dN_a/dxi_d at one reference point, [8, 3]."""
    g = np.zeros((8, 3))
    for a in range(8):
        r = REF[a]
        f = [(1 + r[d] * xi[d]) for d in range(3)]
        g[a, 0] = r[0] * f[1] * f[2] / 8.0
        g[a, 1] = f[0] * r[1] * f[2] / 8.0
        g[a, 2] = f[0] * f[1] * r[2] / 8.0
    return g


def strain_matrix(dNdx: np.ndarray) -> np.ndarray:
    """B [6, 24]: Voigt strain (11,22,33,23,13,12; engineering shear) of the 24 local DoFs."""
    B = np.zeros((6, 24))
    for a in range(8):
        gx, gy, gz = dNdx[a]
        c = 3 * a
        B[0, c + 0] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c + 1], B[3, c + 2] = gz, gy
        B[4, c + 0], B[4, c + 2] = gz, gx
        B[5, c + 0], B[5, c + 1] = gy, gx
    return B


def element_stiffness(X: np.ndarray, C6: np.ndarray, ngauss: int = 2) -> np.ndarray:
    """Ke = sum over Gauss points of B^T C B det(J) w for nodes X [8, 3]."""
    pts, wts = gauss_rule(ngauss)
    Ke = np.zeros((24, 24))
    for xi, w in zip(pts, wts):
        dN = shape_grad_ref(xi)
        J = dN.T @ X                      # J[d, e] = d x_e / d xi_d
        detJ = np.linalg.det(J)
        dNdx = np.linalg.solve(J, dN.T).T  # rows: grad_x N_a
        B = strain_matrix(dNdx)
        Ke += B.T @ C6 @ B * detJ * w
    return Ke


def element_nodes(prob, e_i: int, e_j: int, e_k: int) -> np.ndarray:
    """Global node ids of element (i, j, k) in local order a = di + 2 dj + 4 dk."""
    nx1, ny1 = prob.nx + 1, prob.ny + 1
    ids = []
    for a in range(8):
        i, j, k = e_i + (a & 1), e_j + ((a >> 1) & 1), e_k + ((a >> 2) & 1)
        ids.append(i + nx1 * (j + ny1 * k))
    return np.array(ids)


def box_elements(lo, hi):
    for k in range(int(lo[2]), int(hi[2])):
        for j in range(int(lo[1]), int(hi[1])):
            for i in range(int(lo[0]), int(hi[0])):
                yield i, j, k


class KeCache:
    """Element matrices of a problem, memoised by element id."""

    def __init__(self, prob):
        self.prob = prob
        self.C = material.material_table(prob.materials)
        self.cache = {}

    def __call__(self, i, j, k) -> np.ndarray:
        p = self.prob
        eid = i + p.nx * (j + p.ny * k)
        Ke = self.cache.get(eid)
        if Ke is None:
            nodes = element_nodes(p, i, j, k)
            Ke = element_stiffness(p.xyz[nodes], self.C[p.elem_mat[eid]])
            self.cache[eid] = Ke
        return Ke


def box_node_ids(prob, nlo, nhi) -> np.ndarray:
    """Global node ids of the node box [nlo, nhi] (inclusive), x fastest."""
    nx1, ny1 = prob.nx + 1, prob.ny + 1
    ii = np.arange(nlo[0], nhi[0] + 1)
    jj = np.arange(nlo[1], nhi[1] + 1)
    kk = np.arange(nlo[2], nhi[2] + 1)
    K, J, I = np.meshgrid(kk, jj, ii, indexing="ij")
    return (I + nx1 * (J + ny1 * K)).ravel()


def assemble_box_dense(prob, elo, ehi, kecache: KeCache | None = None) -> np.ndarray:
    """Dense a_D on the element box D = [elo, ehi) over the nodes of D (Sec. 2).

    Rows/columns are the DoFs of the node box [elo, ehi], node-major with the
    nodes ordered x fastest, 3 components per node.
    """
    kec = kecache or KeCache(prob)
    mx, my, mz = (int(ehi[d] - elo[d]) + 1 for d in range(3))
    n = 3 * mx * my * mz
    A = np.zeros((n, n))
    for (i, j, k) in box_elements(elo, ehi):
        Ke = kec(i, j, k)
        loc = []
        for a in range(8):
            li = (i - elo[0]) + (a & 1)
            lj = (j - elo[1]) + ((a >> 1) & 1)
            lk = (k - elo[2]) + ((a >> 2) & 1)
            node = li + mx * (lj + my * lk)
            loc.extend([3 * node, 3 * node + 1, 3 * node + 2])
        loc = np.array(loc)
        A[np.ix_(loc, loc)] += Ke
    return A


def assemble_global_sparse(prob, kecache: KeCache | None = None) -> sp.csr_matrix:
    """Global stiffness (all DoFs, Dirichlet rows not yet removed)."""
    kec = kecache or KeCache(prob)
    rows, cols, vals = [], [], []
    for (i, j, k) in box_elements((0, 0, 0), (prob.nx, prob.ny, prob.nz)):
        Ke = kec(i, j, k)
        nodes = element_nodes(prob, i, j, k)
        dofs = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
        rows.append(np.repeat(dofs, 24))
        cols.append(np.tile(dofs, 24))
        vals.append(Ke.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(prob.n_dofs, prob.n_dofs)).tocsr()
    return A


def _face_elements(prob, face):
    """Elements with a face on the given boundary side and that face's local nodes."""
    axis = "xyz".index(face[0])
    side = 1 if face[1] == "+" else 0
    n = (prob.nx, prob.ny, prob.nz)
    for (i, j, k) in box_elements((0, 0, 0), n):
        idx = (i, j, k)
        if (side == 0 and idx[axis] == 0) or (side == 1 and idx[axis] == n[axis] - 1):
            locs = [a for a in range(8) if ((a >> axis) & 1) == side]
            yield (i, j, k), locs


def traction_load(prob, ngauss: int = 2) -> np.ndarray:
    """Consistent nodal loads b_i = integral over Gamma_N of g . phi_i (Sec. 2)."""
    b = np.zeros(prob.n_dofs)
    x, w = np.polynomial.legendre.leggauss(ngauss)
    for face, g in prob.tractions:
        axis = "xyz".index(face[0])
        other = [d for d in range(3) if d != axis]
        for (i, j, k), locs in _face_elements(prob, face):
            nodes = element_nodes(prob, i, j, k)
            # bilinear face map over the two in-face reference coordinates
            F = np.array([prob.xyz[nodes[a]] for a in locs])        # 4 nodes
            rf = np.array([[REF[a][other[0]], REF[a][other[1]]] for a in locs])
            for q1, w1 in zip(x, w):
                for q2, w2 in zip(x, w):
                    N = (1 + rf[:, 0] * q1) * (1 + rf[:, 1] * q2) / 4.0
                    dN1 = rf[:, 0] * (1 + rf[:, 1] * q2) / 4.0
                    dN2 = (1 + rf[:, 0] * q1) * rf[:, 1] / 4.0
                    t1 = dN1 @ F
                    t2 = dN2 @ F
                    dA = np.linalg.norm(np.cross(t1, t2))
                    for a_i, a in enumerate(locs):
                        dof = 3 * nodes[a]
                        b[dof:dof + 3] += N[a_i] * np.asarray(g) * dA * w1 * w2
    return b
