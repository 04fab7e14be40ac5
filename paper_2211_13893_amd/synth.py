"""Seeded synthetic laminate problems (inputs only).

This module produces the *inputs* of the local spectral stage of MS-GFEM
(Benezech et al., "Scalable multiscale-spectral GFEM with an application to
composite aero-structures"): a structured hexahedral mesh of a laminated
composite, the engineering constants and ply angle of every element, the
boundary conditions and the overlapping domain decomposition.  It performs
none of the method's arithmetic (no material tensors, no element matrices, no
partition of unity, no eigenproblems): both the FP64 CPU oracle and the HIP
library read exactly these arrays and do all of that themselves.

Conventions shared by every consumer (Sec. 2, "Problem formulation"):

* Mesh: ``nx*ny*nz`` hexahedra on a node grid ``(nx+1)*(ny+1)*(nz+1)``.
  Node id ``i + (nx+1)*(j + (ny+1)*k)``; element id ``i + nx*(j + ny*k)``;
  the 8 local nodes of an element are ordered lexicographically,
  ``a = di + 2*dj + 4*dk``.  DoF id ``3*node + component`` (node-blocked
  vectors, one 3-vector per Lagrange basis function, Sec. 2).
* Units mm, N, MPa.
* ``materials[m] = (E1, E2, E3, G12, G13, G23, nu12, nu13, nu23, theta_deg)``:
  orthotropic engineering constants in the material frame plus the ply angle,
  a rotation about +z (fibre axis ``(cos t, sin t, 0)``).  An isotropic
  material has ``E1=E2=E3``, ``G=E/(2(1+nu))`` and ``theta=0``.
* Boundary: ``dirichlet[dof] = 1`` on the clamped DoFs (zero displacement,
  h = 0 in every workload here) and a list of uniform tractions
  ``(face, g)`` with ``face`` in ``{"x-","x+","y-","y+","z-","z+"}``.
* Decomposition (Sec. 3.1): non-overlapping element boxes ("cores")
  ``[lo, hi)`` per axis, a global overlap ``o`` (layers of elements added to a
  core to form Omega_j) and a per-subdomain oversampling ``ovs`` (further
  layers forming Omega_j^*; the paper's o^* equals ``o + ovs``).  Both
  extensions are clipped to the mesh.  ``batch`` lists the subdomains whose
  local eigenproblems are solved.

Random draws use ``numpy.random.Generator(PCG64(SeedSequence([cfg, item])))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Carbon/epoxy ply constants of the laminated-beam workload (MPa).
PLY_CONSTANTS = (162000.0, 10000.0, 10000.0, 5200.0, 5200.0, 3500.0, 0.35, 0.35, 0.5)
# Isotropic resin interlayer (MPa).
RESIN_E, RESIN_NU = 3000.0, 0.35

FACES = ("x-", "x+", "y-", "y+", "z-", "z+")


def isotropic_constants(E: float, nu: float) -> Tuple[float, ...]:
    G = E / (2.0 * (1.0 + nu))
    return (E, E, E, G, G, G, nu, nu, nu)


@dataclasses.dataclass
class Problem:
    """One synthetic workload: mesh, materials, boundary data, decomposition."""

    name: str
    nx: int
    ny: int
    nz: int
    xyz: np.ndarray            # float64 [n_nodes, 3]
    elem_mat: np.ndarray       # int32 [n_elems]
    materials: np.ndarray      # float64 [n_mat, 10]
    dirichlet: np.ndarray      # uint8 [n_dofs]
    tractions: List[Tuple[str, Tuple[float, float, float]]]
    cores: np.ndarray          # int32 [nsd, 6]: lo_x, lo_y, lo_z, hi_x, hi_y, hi_z
    overlap: int
    ovs: np.ndarray            # int32 [nsd]
    n_ev: np.ndarray           # int32 [nsd]
    batch: np.ndarray          # int32 [nb] subdomains whose GEVPs are solved

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def n_elems(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_dofs(self) -> int:
        return 3 * self.n_nodes

    @property
    def nsd(self) -> int:
        return int(self.cores.shape[0])

    def omega_box(self, j: int) -> Tuple[np.ndarray, np.ndarray]:
        """Element box [lo, hi) of Omega_j: the core grown by ``overlap`` layers."""
        lo = np.maximum(self.cores[j, :3] - self.overlap, 0)
        hi = np.minimum(self.cores[j, 3:] + self.overlap, [self.nx, self.ny, self.nz])
        return lo.astype(np.int64), hi.astype(np.int64)

    def omega_star_box(self, j: int) -> Tuple[np.ndarray, np.ndarray]:
        """Element box [lo, hi) of Omega_j^*: Omega_j grown by ``ovs[j]`` layers."""
        g = self.overlap + int(self.ovs[j])
        lo = np.maximum(self.cores[j, :3] - g, 0)
        hi = np.minimum(self.cores[j, 3:] + g, [self.nx, self.ny, self.nz])
        return lo.astype(np.int64), hi.astype(np.int64)


def _rng(cfg: int, item: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg, item])))


def _grid_xyz(xs: np.ndarray, ys: np.ndarray, zs: np.ndarray) -> np.ndarray:
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    # node id i + (nx+1)*(j + (ny+1)*k): x fastest
    return np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(),
                     Z.transpose(2, 1, 0).ravel()], axis=1).astype(np.float64)


def _apply_wrinkle(xyz: np.ndarray, amp: float, sigma: float, xc: float, yc: float) -> None:
    """Gaussian out-of-plane ply wrinkle, uniform through the thickness."""
    if amp == 0.0:
        return
    dx = xyz[:, 0] - xc
    dy = xyz[:, 1] - yc
    xyz[:, 2] += amp * np.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma))


def _clamp_x0(nx: int, ny: int, nz: int) -> np.ndarray:
    d = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1), dtype=np.uint8)
    for k in range(nz + 1):
        for j in range(ny + 1):
            node = (nx + 1) * (j + (ny + 1) * k)
            d[3 * node: 3 * node + 3] = 1
    return d


def _layered_materials(layer_kind: Sequence[str], layer_angle: Sequence[float],
                       scale: Optional[Sequence[float]] = None):
    """One material row per element layer (ply constants rotated by its angle)."""
    rows = []
    for li, (kind, ang) in enumerate(zip(layer_kind, layer_angle)):
        f = 1.0 if scale is None else float(scale[li])
        if kind == "ply":
            c = PLY_CONSTANTS
            row = [c[0] * f, c[1] * f, c[2] * f, c[3] * f, c[4] * f, c[5] * f,
                   c[6], c[7], c[8], float(ang)]
        else:
            c = isotropic_constants(RESIN_E * f, RESIN_NU)
            row = list(c) + [0.0]
        rows.append(row)
    return np.asarray(rows, dtype=np.float64)


def _elem_mat_by_layer(nx: int, ny: int, nz: int) -> np.ndarray:
    k = np.repeat(np.arange(nz, dtype=np.int32), nx * ny)
    return k


def _tiles(nx: int, ny: int, nz: int, t: Tuple[int, int, int]) -> np.ndarray:
    cores = []
    for kz in range(0, nz, t[2]):
        for ky in range(0, ny, t[1]):
            for kx in range(0, nx, t[0]):
                cores.append([kx, ky, kz, min(kx + t[0], nx), min(ky + t[1], ny), min(kz + t[2], nz)])
    return np.asarray(cores, dtype=np.int32)


def laminated_beam(n_ev: int = 10, overlap: int = 2, ovs: int = 2,
                   material: str = "laminate", theta: float = 0.0,
                   roller: bool = False, n_sub: int = 4,
                   shape: Tuple[int, int, int] = (48, 6, 6)) -> Problem:
    """Laminated beam, 48x6x6 unit hexahedra over [0,48]x[0,6]x[0,6] mm.

    (``shape`` shrinks the beam for small tests; the stacking then repeats.)

    Six 1 mm plies stacked [0/90/45/-45/90/0] from z=0 upward, clamped at
    x=0, uniform compressive traction 10 MPa on x=48, four cores of 12x6x6
    along x.  ``material="ply"`` gives every layer the same ply angle
    ``theta``; ``"iso"`` makes the beam homogeneous resin.  ``roller=True``
    replaces the clamp by a roller face plus the minimal point supports that
    admit the uniform-stress solution (u_x=0 on x=0; u_y=u_z=0 at (0,0,0);
    u_z=0 at (0,6,0)).
    """
    nx, ny, nz = shape
    xyz = _grid_xyz(np.arange(nx + 1, dtype=float), np.arange(ny + 1, dtype=float),
                    np.arange(nz + 1, dtype=float))
    if material == "laminate":
        stack = [0.0, 90.0, 45.0, -45.0, 90.0, 0.0]
        angles = [stack[l % 6] for l in range(nz)]
        mats = _layered_materials(["ply"] * nz, angles)
    elif material == "ply":
        mats = _layered_materials(["ply"] * nz, [theta] * nz)
    elif material == "iso":
        mats = _layered_materials(["resin"] * nz, [0.0] * nz)
    else:
        raise ValueError(material)
    elem_mat = _elem_mat_by_layer(nx, ny, nz)
    if roller:
        d = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1), dtype=np.uint8)
        for k in range(nz + 1):
            for j in range(ny + 1):
                d[3 * ((nx + 1) * (j + (ny + 1) * k))] = 1
        d[3 * 0 + 1] = d[3 * 0 + 2] = 1
        d[3 * ((nx + 1) * ny) + 2] = 1   # node (0, ny, 0)
    else:
        d = _clamp_x0(nx, ny, nz)
    w = nx // n_sub
    cores = np.asarray([[w * s, 0, 0, w * (s + 1) if s < n_sub - 1 else nx, ny, nz]
                        for s in range(n_sub)], dtype=np.int32)
    return Problem("beam", nx, ny, nz, xyz, elem_mat, mats, d, [("x+", (-10.0, 0.0, 0.0))],
                   cores, overlap, np.full(n_sub, ovs, np.int32), np.full(n_sub, n_ev, np.int32),
                   np.arange(n_sub, dtype=np.int32))


def _ply_resin_stack(rng: np.random.Generator, n_layers: int, t_ply: float, t_resin: float):
    """Alternating ply / resin element layers, phase and ply angles from ``rng``."""
    phase = int(rng.integers(0, 2))
    kinds, angles, thick = [], [], []
    for l in range(n_layers):
        ply = ((l + phase) % 2) == 0
        kinds.append("ply" if ply else "resin")
        angles.append(float(rng.choice([0.0, 45.0, -45.0, 90.0])) if ply else 0.0)
        thick.append(t_ply if ply else t_resin)
    z = np.concatenate([[0.0], np.cumsum(thick)])
    return kinds, angles, z


def uniform_batch(n_boxes: int = 64, core: int = 8, overlap: int = 1, ovs: int = 2,
                  n_ev: int = 16, seed: int = 0, h_xy: float = 0.25) -> Problem:
    """Uniform batch of interior oversampled boxes of a thick ply/resin laminate.

    A column of ``3 x 3 x (n_boxes + 2)`` cubic cores (``core`` elements per
    side) tiles a laminate of alternating 0.25 mm plies and 0.05 mm resin
    interlayers (one element per layer, h_xy = 0.25 mm in-plane).  The batch
    is the ``n_boxes`` cores of the central column that have a neighbour on
    every side, so every oversampled box lies in the interior of the mesh:
    its whole boundary is interior boundary and no box touches the boundary
    data.  Each box sees a different window of the random ply sequence.
    """
    rng = _rng(2, seed)
    nx = ny = 3 * core
    nz = (n_boxes + 2) * core
    kinds, angles, zs = _ply_resin_stack(rng, nz, 0.25, 0.05)
    xyz = _grid_xyz(h_xy * np.arange(nx + 1), h_xy * np.arange(ny + 1), zs)
    mats = _layered_materials(kinds, angles)
    elem_mat = _elem_mat_by_layer(nx, ny, nz)
    cores = _tiles(nx, ny, nz, (core, core, core))
    # tile (1, 1, t) has index 1 + 3*(1 + 3*t)
    batch = np.asarray([1 + 3 * (1 + 3 * t) for t in range(1, n_boxes + 1)], dtype=np.int32)
    nsd = cores.shape[0]
    return Problem("uniform_batch", nx, ny, nz, xyz, elem_mat, mats,
                   np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1), np.uint8), [],
                   cores, overlap, np.full(nsd, ovs, np.int32), np.full(nsd, n_ev, np.int32), batch)


def warm_start_batch(n_boxes: int = 64, seed: int = 0, wrinkle_max: float = 0.8,
                     modulus_spread: float = 0.2, homogeneous: bool = False, core: int = 8,
                     overlap: int = 1, ovs: int = 2, n_ev: int = 16, h_xy: float = 0.25) -> Problem:
    """Training / held-out boxes of the learned warm start: the uniform batch's
    14^3 interior boxes of a ply/resin laminate, plus a Gaussian ply wrinkle of
    amplitude U[0, wrinkle_max] ply thicknesses (sigma 8 elements, random
    centre) and one log-uniform modulus factor in [1/(1+spread), 1+spread] per
    layer.  With ``homogeneous`` every element is one isotropic material on
    the same node grid (the reference box of the coefficient basis)."""
    rng = _rng(4, seed)
    nx = ny = 3 * core
    nz = (n_boxes + 2) * core
    kinds, angles, zs = _ply_resin_stack(rng, nz, 0.25, 0.05)
    xyz = _grid_xyz(h_xy * np.arange(nx + 1), h_xy * np.arange(ny + 1), zs)
    lo, hi = np.log(1.0 / (1.0 + modulus_spread)), np.log(1.0 + modulus_spread)
    scale = np.exp(rng.uniform(lo, hi, size=nz))
    amp = float(rng.uniform(0.0, wrinkle_max)) * 0.25
    xc, yc = rng.uniform(0.0, nx * h_xy), rng.uniform(0.0, ny * h_xy)
    _apply_wrinkle(xyz, amp, 8.0 * h_xy, xc, yc)
    if homogeneous:
        mats = np.asarray([list(isotropic_constants(10000.0, 0.3)) + [0.0]], dtype=np.float64)
        elem_mat = np.zeros(nx * ny * nz, dtype=np.int32)
    else:
        mats = _layered_materials(kinds, angles, scale)
        elem_mat = _elem_mat_by_layer(nx, ny, nz)
    cores = _tiles(nx, ny, nz, (core, core, core))
    batch = np.asarray([1 + 3 * (1 + 3 * t) for t in range(1, n_boxes + 1)], dtype=np.int32)
    nsd = cores.shape[0]
    return Problem("warm_start_batch", nx, ny, nz, xyz, elem_mat, mats,
                   np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1), np.uint8), [],
                   cores, overlap, np.full(nsd, ovs, np.int32), np.full(nsd, n_ev, np.int32), batch)


def _random_cuts(rng: np.random.Generator, n: int, lo: int, hi: int) -> List[int]:
    cuts = [0]
    while cuts[-1] < n:
        w = int(rng.integers(lo, hi + 1))
        cuts.append(min(cuts[-1] + w, n))
    if len(cuts) > 2 and cuts[-1] - cuts[-2] < lo:
        cuts.pop(-2)
    return cuts


def uneven_laminate(seed: int = 0, nx: int = 256, ny: int = 32, nz: int = 24) -> Problem:
    """Uneven batch: wrinkled 1 mm-ply laminate with random tensor-product cuts.

    ``nx x ny x nz`` unit elements, 24 plies of random angle, a Gaussian ply
    wrinkle (amplitude 0.6 mm, sigma 8 mm, centred in x-y), core widths drawn
    from U{6..16} per axis, overlap 1, oversampling U{1..3}, n_ev U{8..32};
    clamped at x=0 and compressed by 10 MPa on x=nx.
    """
    rng = _rng(3, seed)
    angles = [float(rng.choice([0.0, 45.0, -45.0, 90.0])) for _ in range(nz)]
    xyz = _grid_xyz(np.arange(nx + 1, dtype=float), np.arange(ny + 1, dtype=float),
                    np.arange(nz + 1, dtype=float))
    _apply_wrinkle(xyz, 0.6, 8.0, nx / 2.0, ny / 2.0)
    mats = _layered_materials(["ply"] * nz, angles)
    elem_mat = _elem_mat_by_layer(nx, ny, nz)
    cx, cy, cz = (_random_cuts(rng, n, 6, 16) for n in (nx, ny, nz))
    cores = []
    for k in range(len(cz) - 1):
        for j in range(len(cy) - 1):
            for i in range(len(cx) - 1):
                cores.append([cx[i], cy[j], cz[k], cx[i + 1], cy[j + 1], cz[k + 1]])
    cores = np.asarray(cores, dtype=np.int32)
    nsd = cores.shape[0]
    ovs = rng.integers(1, 4, size=nsd).astype(np.int32)
    n_ev = rng.integers(8, 33, size=nsd).astype(np.int32)
    return Problem("uneven", nx, ny, nz, xyz, elem_mat, mats, _clamp_x0(nx, ny, nz),
                   [("x+", (-10.0, 0.0, 0.0))], cores, 1, ovs, n_ev,
                   np.arange(nsd, dtype=np.int32))


def full_laminate(seed: int = 0, nx: int = 512, ny: int = 64, nz: int = 48, core: int = 16,
                  n_ev: int = 20) -> Problem:
    """Large wrinkled ply/resin laminate with cubic cores (overlap 2, ovs 2)."""
    rng = _rng(5, seed)
    kinds, angles, zs = _ply_resin_stack(rng, nz, 0.25, 0.05)
    xyz = _grid_xyz(0.25 * np.arange(nx + 1), 0.25 * np.arange(ny + 1), zs)
    _apply_wrinkle(xyz, 0.6 * 0.25, 8 * 0.25, 0.25 * nx / 2.0, 0.25 * ny / 2.0)
    mats = _layered_materials(kinds, angles)
    elem_mat = _elem_mat_by_layer(nx, ny, nz)
    cores = _tiles(nx, ny, nz, (core, core, core))
    nsd = cores.shape[0]
    return Problem("full", nx, ny, nz, xyz, elem_mat, mats, _clamp_x0(nx, ny, nz),
                   [("x+", (-10.0, 0.0, 0.0))], cores, 2, np.full(nsd, 2, np.int32),
                   np.full(nsd, n_ev, np.int32), np.arange(nsd, dtype=np.int32))


def small_box(n: int = 4, core: int = 2, overlap: int = 1, ovs: int = 1, n_ev: int = 8,
              seed: int = 0, material: str = "laminate", wrinkle: float = 0.0,
              clamp: bool = False) -> Problem:
    """Small test problem: an ``n^3``-element cube of unit elements tiled by
    ``core^3`` cores, random ply angles per element layer (or one isotropic
    material), optional wrinkle and clamp at x=0.  Every core is in the batch.
    """
    rng = _rng(7, seed)
    nx = ny = nz = n
    xyz = _grid_xyz(np.arange(nx + 1, dtype=float), np.arange(ny + 1, dtype=float),
                    np.arange(nz + 1, dtype=float))
    _apply_wrinkle(xyz, wrinkle, n / 3.0, n / 2.0, n / 2.0)
    if material == "iso":
        mats = _layered_materials(["resin"] * nz, [0.0] * nz)
    else:
        kinds = ["ply" if rng.random() < 0.7 else "resin" for _ in range(nz)]
        angles = [float(rng.choice([0.0, 45.0, -45.0, 90.0, 30.0])) for _ in range(nz)]
        mats = _layered_materials(kinds, angles)
    elem_mat = _elem_mat_by_layer(nx, ny, nz)
    cores = _tiles(nx, ny, nz, (core, core, core))
    nsd = cores.shape[0]
    d = _clamp_x0(nx, ny, nz) if clamp else np.zeros(3 * (nx + 1) ** 3, np.uint8)
    tr = [("x+", (-10.0, 0.0, 0.0))] if clamp else []
    return Problem("small", nx, ny, nz, xyz, elem_mat, mats, d, tr, cores, overlap,
                   np.full(nsd, ovs, np.int32), np.full(nsd, n_ev, np.int32),
                   np.arange(nsd, dtype=np.int32))


def slab(nxy: int = 40, nz: int = 4, core: int = 20, overlap: int = 1, ovs: int = 1, n_ev: int = 8,
         seed: int = 0, clamp: bool = False) -> Problem:
    """Thin laminate slab of unit elements (``nxy x nxy x nz``, one random ply
    angle per element layer) tiled by ``core x core x nz`` cores.  Its
    oversampled boxes have wide node planes (about ``(core+3)^2`` nodes), so
    their banded matrices span more than 33 tiles of 32 rows: the wide-band
    test problem.  Every core is in the batch.  ``clamp`` fixes the x = 0
    face and compresses the x = nxy face by 10 MPa (a well-posed global
    problem for the fine solve)."""
    rng = _rng(8, seed)
    nx = ny = nxy
    xyz = _grid_xyz(np.arange(nx + 1, dtype=float), np.arange(ny + 1, dtype=float),
                    np.arange(nz + 1, dtype=float))
    kinds = ["ply" if rng.random() < 0.75 else "resin" for _ in range(nz)]
    angles = [float(rng.choice([0.0, 45.0, -45.0, 90.0])) for _ in range(nz)]
    mats = _layered_materials(kinds, angles)
    elem_mat = _elem_mat_by_layer(nx, ny, nz)
    cores = _tiles(nx, ny, nz, (core, core, nz))
    nsd = cores.shape[0]
    d = _clamp_x0(nx, ny, nz) if clamp else np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1), np.uint8)
    tr = [("x+", (-10.0, 0.0, 0.0))] if clamp else []
    return Problem("slab", nx, ny, nz, xyz, elem_mat, mats, d, tr, cores, overlap,
                   np.full(nsd, ovs, np.int32), np.full(nsd, n_ev, np.int32), np.arange(nsd, dtype=np.int32))


def start_block(n2: int, k: int, seed: int, item: int) -> np.ndarray:
    """Seeded Gaussian start block ``[n2, k]`` for iterative eigensolvers."""
    return _rng(11, seed * 1000003 + item).standard_normal((n2, k))
