// Internal definitions shared by the HIP translation units of libmsgfem.
//
// Data layout in HBM (one "plan" = one mesh, one decomposition, one batch of
// oversampled subdomains):
//   * every oversampled box Omega_j^* is a node grid mx*my*mz, nodes x fastest,
//     DoF = 3*node + component;
//   * the box stiffness is a block-27 stencil stored structure-of-arrays:
//     stencil[(nb*9 + 3*cr + cc) * n_nodes + node], nb = (dx+1)+3(dy+1)+9(dz+1);
//   * block vectors are row-major [n_dof][k] (k columns contiguous per DoF);
//   * banded SPD factors are 32x32 tiles: tile (I, I-s) at
//     ((I*BT + s) * 1024), row-major inside the tile, s = 0 the diagonal tile;
//     the inverses of the diagonal tiles follow in a separate NT*1024 array;
//   * after factorisation the unit-lower band (Lu, D^{-1}) of every box matrix
//     is written twice more, once per sweep direction of the block solve, in
//     the order the solve reads it (for bands of at most 65 tiles straight
//     from L, the band then keeping L off the diagonal and D^{-1} on it), so that a wavefront's load instruction reads 1 KB of
//     consecutive memory.  Matrix-core solve (bands of at most 65 tiles):
//     1 + 8 nslot slots of 8 KB per tile row (slot 0 = D^{-1} in the forward
//     copy, slot s = tile s), double2 pp of lane l at ((I*S + slot)*8 + pp)*64
//     + l (see k_band_relayout4).  Wider bands (vector-FMA solve): fragment
//     double2 j (0..31) of solve thread t (0..nthr-1) for tile set p (tiles
//     1+32p .. 32+32p) of tile row I at (((I*nsets + p)*32 + j) * nthr + t) * 2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MSG_TILE 32
#define MSG_TILE2 1024
#define SOLVE_TILES 32      // off-diagonal band tiles covered by the solve's thread layout
#define UPD_THREADS 512     // k_update workgroup: 8 wavefronts x 4 row blocks of 16
#define UPD_ROWS (UPD_THREADS)

namespace msg {

// One banded SPD matrix of a box in 32x32 tile-band storage.  A box matrix
// (A11 or Ahat) is either one band over the node order (one part), or split
// by one layer of nodes across the slowest order axis (nested dissection,
// three parts): chain 0 = the layers before the separator, chain 1 = the
// layers after it taken from the far end, each followed by the separator
// rows, and the separator block S itself (dense, BT == NT).  The chains are
// factored on their own rows (NTf tile rows; their separator rows get the
// off-diagonal factor tiles L_sc only) and S holds the Cholesky factor of the
// Schur complement A_ss - sum_c L_sc L_sc^T.
struct BandPart {
  int32_t NT, BT;       // tile rows, band tiles
  int32_t NTf;          // tile rows factored (chain rows; NT for a whole band and for S)
  int32_t pad;          // leading identity rows (a chain's last row ends tile row NTf - 1)
  int32_t nc, nsep;     // rows of the order after the padding, then separator rows
  int32_t mirror;       // the rows run over the layers from the far end (chain 1)
  int32_t pad_;
  int64_t off, ioff;    // band tiles, inverse diagonal tiles (doubles)
  int64_t fw, bw;       // solve-ordered copies (forward / backward sweep)
};

// Per-box metadata, uploaded once per plan.
struct BoxMeta {
  int32_t sd;                 // subdomain id in the decomposition
  int32_t mx, my, mz;         // box node dims
  int32_t g0[3];              // global node index of box node (0,0,0)
  int32_t olo[3], ohi[3];     // Omega_j node box (global, inclusive)
  int32_t iface_lo[3];        // 1 if the low face of the box on this axis is interior boundary
  int32_t iface_hi[3];
  int32_t olo_int[3];         // 1 if the low face of Omega_j is interior (not on the mesh boundary)
  int32_t ohi_int[3];
  int32_t sub_lo[3], sub_hi[3];  // node sub-box (box-relative, inclusive) holding B1 (and B3)
  int32_t n_nodes, n_dof;
  int32_t n_ev;
  // whole-band geometry (tiles of 32) of A11 on the sub-box and Ahat on the full box
  int32_t nt11, bt11, n11;    // tile rows, band tiles, matrix order (unpadded)
  int32_t nth, bth, nh;
  int32_t flags;              // BOX_COMPACT_DINV: D^{-1} tiles compact at each part's ioff (coarse store)
  int32_t ord[2];             // node order of the A11 / Ahat bands: box axis of the fastest, middle and
                              // slowest order index in bits 0-1, 2-3, 4-5 (the longest axis slowest)
  int32_t nd[2];              // 1: the matrix is split into two chains and a separator (three parts)
  int32_t zs[2];              // separator layer (slowest order index) of a split matrix
  int32_t pad0_;
  int64_t node_off;           // offset into per-node arrays of the batch
  int64_t dof_off;            // offset into per-dof arrays
  int64_t vec_off;            // offset (doubles) of this box inside one block-vector array
  int64_t evec_off;           // offset (doubles) into the eigenvector output
  int64_t eval_off;           // offset into eigenvalue output
  BandPart part[2][3];        // [kind][part]: part 0 alone for a whole band
};

// BoxMeta.flags: the D^{-1} tiles of the factors are stored compactly, tile
// I of a part at its ioff + I*1024, instead of on the band's diagonal (a
// coarse store keeps only what the block solves read)
#define BOX_COMPACT_DINV 1

// solve threads that hold a band fragment: 16 per off-diagonal tile of a set
__host__ __device__ inline int solve_nthr(int BT) {
  int t = BT - 1 < SOLVE_TILES ? BT - 1 : SOLVE_TILES;
  return 16 * (t > 0 ? t : 0);
}
// tile sets of SOLVE_TILES off-diagonal tiles the solve walks per step (1 or 2;
// bands up to 2*SOLVE_TILES + 1 tiles)
#define SOLVE_MAX_BT (2 * SOLVE_TILES + 1)
__host__ __device__ inline int solve_sets(int BT) { return BT - 1 > SOLVE_TILES ? 2 : 1; }
// jobs (wavefronts) of one step of the tile Cholesky with panels of P
// columns: the step's chain and P diagonal tiles, padded to whole workgroups
// of four (so that a workgroup holds whole rows), then (BT - 2) rows x P / 2
// column pairs
#define CHOL_ROW0(P) ((((P) + 1) + 3) / 4 * 4)
__host__ __device__ inline int chol_jobs(int P, int max_bt) {
  return CHOL_ROW0(P) + (max_bt > 2 ? max_bt - 2 : 0) * (P / 2);
}
// workgroups of one step: the diagonal and row workgroups of every matrix,
// the matrix count padded to a multiple of 8 (one XCD per matrix)
__host__ __device__ inline int chol_grid(int P, int nmat, int max_bt) {
  return (chol_jobs(P, max_bt) + 3) / 4 * ((nmat + 7) / 8 * 8);
}

// the matrix-core block solve (k_band_solve4) takes bands of at most
// 1 + 8 * SOLVE4_MAX_SLOTS tiles with 8 columns per workgroup (up to 5 slots
// in registers, 6-8 as two sets of four); the 16-column solve's LDS ring
// limits it to 31 tiles, 4 slots.  Its copies hold 1 + 8 nslot tiles per row
#define SOLVE4_MAX_SLOTS 8
__host__ __device__ inline int solve4_nslot(int BT) { return (BT - 1 + 7) / 8; }
__host__ __device__ inline int solve4_slots(int BT) { return 1 + 8 * solve4_nslot(BT); }
// doubles of one solve-ordered copy of a band (room for either layout)
__host__ __device__ inline int64_t solve_copy_doubles(int NT, int BT) {
  const int64_t a = (int64_t)NT * solve_sets(BT) * 64 * solve_nthr(BT);
  const int64_t b = (int64_t)NT * solve4_slots(BT) * MSG_TILE2;
  return a > b ? a : b;
}

// One SPD matrix in 32x32 tile-band storage (tiles at fac + off, inverse
// diagonal tiles at fac + ioff); BT == NT is a dense matrix.
struct MatDesc {
  int32_t NT, BT;
  int32_t status_idx;   // index into the status array for pivot failures
  int32_t NTf;          // columns factored (a chain stops before its separator rows; 0 = NT)
  int64_t off, ioff;
};

// The separator Schur complement of a split matrix: the two chains' bands
// (off0, off1, factored on NTf0, NTf1 tile rows, band BT) and S (offS, NTs x
// NTs tiles, dense lower in band storage with BT = NTs).
struct SepDesc {
  int32_t NTs, BT, NTf0, NTf1;
  int64_t off0, off1, offS;
};

struct MeshDev {
  int32_t nx, ny, nz;
  int32_t n_mat;
  const double* xyz;
  const int32_t* elem_mat;
  const double* materials;
  const uint8_t* dirichlet;
};

// Where the LOBPCG block X of a box lives.  The iteration keeps its blocks
// (four image kinds x five slots) in 20 buffers of the workspace, buffer
// (kind * 5 + id) at vec + (kind * 5 + id) * VT; the host rotates the slot ->
// buffer map every iteration without moving data, and a box retired as
// converged is left in the buffer it was in (xbuf[box] = its id, -1 while it
// is still iterated, when X is in buffer cur).
struct XLoc {
  const double* vec;
  int64_t VT;
  int32_t cur;
  const int32_t* xbuf;
  __device__ const double* at(int kind, int box) const {
    const int id = xbuf[box] >= 0 ? xbuf[box] : cur;
    return vec + (int64_t)(kind * 5 + id) * VT;
  }
};

__host__ __device__ inline int nb_index(int dx, int dy, int dz) {
  return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
}

}  // namespace msg
