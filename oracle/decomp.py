"""Subdomains, DoF classes and the partition of unity (oracle; test infrastructure).

Sec. 3.1: cores are grown by o element layers into the overlapping Omega_j and
(Sec. 3.3) further into the oversampling domain Omega_j^*.  Sec. 4.2: the
smooth partition of unity starts from weights 0 on the boundary of Omega_j
(and on the oversampling layers outside Omega_j) and 2o elsewhere, lowers
them by the neighbour rule w_p = min(w_p, w_q + 1) for 2o - 1 sweeps, caps at
2o, and normalises mu_{j,p} = w_{j,p} / sum_i w_{i,p}.  Sec. 4.3: the DoFs of
Omega_j^* split into B1 (interior plus Neumann boundary), B2 (interior
boundary of Omega_j^*, neither Dirichlet nor Neumann) and B3 (Dirichlet).

Readings (the paper leaves these open): "boundary of Omega_j" in the
partition of unity is its interior boundary (the part not on the boundary of
Omega); the graph is the extended connectivity graph of the mesh, i.e. nodes
sharing an element; a node of the interior boundary of Omega_j^* that also
lies on a Neumann face is in B2 (it belongs to an element outside Omega_j^*).
"""
from __future__ import annotations

import numpy as np


def node_box(elo, ehi):
    """Node index box [elo, ehi] (inclusive) of the element box [elo, ehi)."""
    return np.asarray(elo, dtype=np.int64), np.asarray(ehi, dtype=np.int64)


def box_shape(nlo, nhi):
    return tuple(int(nhi[d] - nlo[d]) + 1 for d in range(3))


def local_node_grid(nlo, nhi):
    """Global (i, j, k) index arrays of the node box, flattened x fastest."""
    mx, my, mz = box_shape(nlo, nhi)
    K, J, I = np.meshgrid(np.arange(mz), np.arange(my), np.arange(mx), indexing="ij")
    return (I.ravel() + nlo[0], J.ravel() + nlo[1], K.ravel() + nlo[2])


def interior_boundary_mask(prob, nlo, nhi, I, J, K):
    """Nodes of the box on a face of the box that is not part of the mesh boundary."""
    N = (prob.nx, prob.ny, prob.nz)
    on = np.zeros(I.shape, dtype=bool)
    for d, idx in enumerate((I, J, K)):
        if nlo[d] > 0:
            on |= idx == nlo[d]
        if nhi[d] < N[d]:
            on |= idx == nhi[d]
    return on


def dof_classes(prob, j: int) -> np.ndarray:
    """Class 1/2/3 of every DoF of Omega_j^* (node-major, 3 per node)."""
    nlo, nhi = node_box(*prob.omega_star_box(j))
    I, J, K = local_node_grid(nlo, nhi)
    gnode = I + (prob.nx + 1) * (J + (prob.ny + 1) * K)
    bnd = interior_boundary_mask(prob, nlo, nhi, I, J, K)
    cls = np.ones((gnode.size, 3), dtype=np.int64)
    cls[bnd, :] = 2
    dir_ = prob.dirichlet.reshape(-1, 3)[gnode].astype(bool)
    cls[dir_] = 3
    return cls.ravel()


def pou_weights_on_box(prob, i: int, nlo, nhi) -> np.ndarray:
    """Weights w_{i,p} of subdomain i at the nodes of the node box [nlo, nhi].

    Follows Sec. 4.2 literally on the node box: w = 0 outside the closed
    Omega_i and on its interior boundary, 2o inside; then 2o - 1 Jacobi sweeps
    of w_p = min(w_p, min over graph neighbours q of w_q + 1), capped at 2o.
    Nodes of the box outside Omega_i keep w = 0.
    """
    o = prob.overlap
    elo, ehi = prob.omega_box(i)
    # work on the union box of [nlo, nhi] and Omega_i's nodes so that sweeps see all neighbours
    ulo = np.minimum(nlo, elo)
    uhi = np.maximum(nhi, ehi)
    mx, my, mz = box_shape(ulo, uhi)
    I, J, K = local_node_grid(ulo, uhi)
    inside = ((I >= elo[0]) & (I <= ehi[0]) & (J >= elo[1]) & (J <= ehi[1])
              & (K >= elo[2]) & (K <= ehi[2]))
    bnd = interior_boundary_mask(prob, elo, ehi, I, J, K) & inside
    w = np.where(inside & ~bnd, 2.0 * o, 0.0).reshape(mz, my, mx)
    fixed = (~inside | bnd).reshape(mz, my, mx)
    for _ in range(2 * o - 1):
        big = np.full((mz + 2, my + 2, mx + 2), np.inf)
        big[1:-1, 1:-1, 1:-1] = w
        nb = np.full_like(w, np.inf)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dx == dy == dz == 0:
                        continue
                    nb = np.minimum(nb, big[1 + dz:1 + dz + mz, 1 + dy:1 + dy + my, 1 + dx:1 + dx + mx])
        w = np.where(fixed, 0.0, np.minimum(np.minimum(w, nb + 1.0), 2.0 * o))
    w = w.ravel()
    # extract the requested box
    sel = ((I >= nlo[0]) & (I <= nhi[0]) & (J >= nlo[1]) & (J <= nhi[1])
           & (K >= nlo[2]) & (K <= nhi[2]))
    return w[sel]


def _boxes_intersect(alo, ahi, blo, bhi) -> bool:
    return all(alo[d] <= bhi[d] and blo[d] <= ahi[d] for d in range(3))


def pou_nodes(prob, j: int) -> np.ndarray:
    """mu_{j,p} at every node of Omega_j^* (zero outside Omega_j)."""
    nlo, nhi = node_box(*prob.omega_star_box(j))
    wj = pou_weights_on_box(prob, j, nlo, nhi)
    total = np.zeros_like(wj)
    for i in range(prob.nsd):
        ilo, ihi = prob.omega_box(i)
        if not _boxes_intersect(nlo, nhi, ilo, ihi):
            continue
        total += pou_weights_on_box(prob, i, nlo, nhi)
    mu = np.zeros_like(wj)
    nz = wj > 0
    mu[nz] = wj[nz] / total[nz]
    return mu


def pou_dofs(prob, j: int) -> np.ndarray:
    """mu per DoF of Omega_j^* (the three components of a node share its weight)."""
    return np.repeat(pou_nodes(prob, j), 3)


def pou_global(prob, j: int) -> np.ndarray:
    """mu_j as a global node vector (zero outside Omega_j)."""
    nlo, nhi = node_box(*prob.omega_star_box(j))
    I, J, K = local_node_grid(nlo, nhi)
    g = I + (prob.nx + 1) * (J + (prob.ny + 1) * K)
    out = np.zeros(prob.n_nodes)
    out[g] = pou_nodes(prob, j)
    return out


def star_global_dofs(prob, j: int) -> np.ndarray:
    """Global DoF ids of Omega_j^* in the local (node-major, x fastest) order."""
    nlo, nhi = node_box(*prob.omega_star_box(j))
    I, J, K = local_node_grid(nlo, nhi)
    g = I + (prob.nx + 1) * (J + (prob.ny + 1) * K)
    return (3 * g[:, None] + np.arange(3)[None, :]).ravel()
