// Block SpMM with the block-27 box stencil (Sec. 2: a_{Omega*} assembled).
//
//   Y  = scale * A X       on the DoFs whose class bit is set in y_classes
//                          (0 on the others)
//   Y2 = D A D X           (optional) with D = diag(mu_j on B1, 0 elsewhere):
//                          the partition-of-unity form B of Sec. 4.3.
// B3 rows and columns are removed from A (Sec. 4.3): the output is masked by
// class, and X must be zero on B3 (every block the library forms is; the
// C entry point masks a caller's block first, k_mask_b3).
//
// One thread per (node, CW consecutive columns): the 243 stencil values of a
// node are read once per CW columns (structure of arrays, coalesced across
// nodes), the rows of X in 16-byte pieces.  With Y2, mu of the neighbour DoF
// is folded into the stencil value.  ST is the stencil's storage precision
// (double, or float in the mixed path); arithmetic is FP64.  Blocks are ordered box-major per XCD
// (block x runs on XCD x mod 8): XCD c takes every block of box c, then of
// box c + 8, ..., so the 27-point neighbourhoods of a box come from that
// XCD's L2 while it works on the box.
// grid.x = 8 * ceil(n_box/8) * blocks_per_box (n_box = 1: blocks_per_box).
#include "internal.hpp"

namespace msg {

// CW columns of row d starting at c0 (zero beyond k); pairs when k is even
template <int CW>
__device__ inline void load_cols(const double* __restrict__ x, int64_t d, int k, int c0, double (&v)[CW]) {
  const double* p = x + d * k + c0;
  if ((k & 1) == 0) {
#pragma unroll
    for (int j = 0; j < CW; j += 2) {
      if (c0 + j < k) {
        const double2 a = *(const double2*)(p + j);
        v[j] = a.x;
        v[j + 1] = a.y;
      } else {
        v[j] = 0.0;
        v[j + 1] = 0.0;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < CW; ++j) v[j] = (c0 + j < k) ? p[j] : 0.0;
  }
}

template <bool TWO, int CW, typename ST>
__global__ __launch_bounds__(256) void k_spmm(const BoxMeta* __restrict__ meta, int n_box,
                                              int blocks_per_box,
                                              const ST* __restrict__ stencil,
                                              const uint8_t* __restrict__ cls,
                                              const double* __restrict__ mu1,
                                              const double* __restrict__ X, double* Y,
                                              double* Y2, int k, int y_classes,
                                              double scale, const int32_t* __restrict__ active) {
  // a single box (the whole-mesh operator) is spread over all XCDs instead
  const int xb = blockIdx.x, r = xb >> 3;
  const int box = n_box == 1 ? 0 : (r / blocks_per_box) * 8 + (xb & 7);
  const int blk = n_box == 1 ? xb : r % blocks_per_box;
  if (box >= n_box) return;
  if (active && !active[box]) return;
  const BoxMeta& bm = meta[box];
  const int nq = (k + CW - 1) / CW;
  const int64_t t = (int64_t)blk * blockDim.x + threadIdx.x;
  if (t >= (int64_t)bm.n_nodes * nq) return;
  const int node = (int)(t / nq), q = (int)(t % nq);
  const int c0 = CW * q;
  const int li = node % bm.mx, lj = (node / bm.mx) % bm.my, lk = node / (bm.mx * bm.my);
  const ST* st = stencil + bm.node_off * 243 + node;
  const uint8_t* cl = cls + bm.dof_off;
  const double* m1 = mu1 + bm.dof_off;
  const double* x = X + (bm.dof_off * k);
  double acc[3][CW], acc2[3][CW];
#pragma unroll
  for (int cr = 0; cr < 3; ++cr)
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      acc[cr][j] = 0.0;
      acc2[cr][j] = 0.0;
    }
  // Neighbours outside the box have zero stencil blocks (the assembly writes
  // all 27 blocks of every node), so their index is clamped into the box and
  // the 27-point loop runs without branches.  With the second output the x
  // loop stays rolled: its registers then allow 4 wavefronts per SIMD.
  constexpr int kUnrollX = TWO ? 1 : 3;
#pragma unroll 1
  for (int dz = -1; dz <= 1; ++dz) {
    const int kk = min(max(lk + dz, 0), bm.mz - 1);
#pragma unroll 1
    for (int dy = -1; dy <= 1; ++dy) {
      const int jj = min(max(lj + dy, 0), bm.my - 1);
#pragma unroll kUnrollX
      for (int dx = -1; dx <= 1; ++dx) {
        const int ii = min(max(li + dx, 0), bm.mx - 1);
        const int nn = ii + bm.mx * (jj + bm.my * kk);
        const int nb = nb_index(dx, dy, dz);
        double xv[3][CW];
        double mu[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          load_cols<CW>(x, 3 * nn + cc, k, c0, xv[cc]);
          mu[cc] = TWO ? m1[3 * nn + cc] : 0.0;
        }
#pragma unroll
        for (int cr = 0; cr < 3; ++cr)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            const double a = (double)st[(int64_t)(nb * 9 + 3 * cr + cc) * bm.n_nodes];
            const double am = a * mu[cc];
#pragma unroll
            for (int j = 0; j < CW; ++j) {
              acc[cr][j] += a * xv[cc][j];
              if (TWO) acc2[cr][j] += am * xv[cc][j];
            }
          }
      }
    }
  }
  double* y = Y ? Y + (bm.dof_off * k) : nullptr;
  double* y2 = TWO ? Y2 + (bm.dof_off * k) : nullptr;
#pragma unroll
  for (int cr = 0; cr < 3; ++cr) {
    const int d = 3 * node + cr;
    const bool w = (y_classes >> cl[d]) & 1;
    const double mo = TWO ? m1[d] : 0.0;
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      if (c0 + j < k) {
        if (y) y[(int64_t)d * k + c0 + j] = w ? scale * acc[cr][j] : 0.0;
        if (TWO) y2[(int64_t)d * k + c0 + j] = mo * acc2[cr][j];
      }
    }
  }
}

template __global__ void k_spmm<false, 8, double>(const BoxMeta*, int, int, const double*, const uint8_t*,
                                                   const double*, const double*, double*, double*, int, int, double,
                                                   const int32_t*);
template __global__ void k_spmm<false, 8, float>(const BoxMeta*, int, int, const float*, const uint8_t*,
                                                   const double*, const double*, double*, double*, int, int, double,
                                                   const int32_t*);
template __global__ void k_spmm<false, 1, double>(const BoxMeta*, int, int, const double*, const uint8_t*,
                                                   const double*, const double*, double*, double*, int, int, double,
                                                   const int32_t*);
template __global__ void k_spmm<false, 1, float>(const BoxMeta*, int, int, const float*, const uint8_t*,
                                                   const double*, const double*, double*, double*, int, int, double,
                                                   const int32_t*);
template __global__ void k_spmm<true, 4, double>(const BoxMeta*, int, int, const double*, const uint8_t*,
                                                   const double*, const double*, double*, double*, int, int, double,
                                                   const int32_t*);
template __global__ void k_spmm<true, 4, float>(const BoxMeta*, int, int, const float*, const uint8_t*,
                                                   const double*, const double*, double*, double*, int, int, double,
                                                   const int32_t*);

// out = X with the rows of B3 DoFs cleared (flat over all boxes' [n_dof][k] blocks)
__global__ void k_mask_b3(const uint8_t* __restrict__ cls, const double* __restrict__ X, int k, int64_t n,
                          double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = cls[e / k] == 3 ? 0.0 : X[e];
}

}  // namespace msg
