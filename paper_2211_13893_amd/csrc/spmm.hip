// Block SpMM with the block-27 box stencil (Sec. 2: a_{Omega*} assembled).
//
//   Y  = scale * A X       on the DoFs whose class bit is set in y_classes
//                          (0 on the others); B3 inputs are ignored (B3
//                          rows/columns are removed from A, Sec. 4.3)
//   Y2 = D A D X           (optional) with D = diag(mu_j on B1, 0 elsewhere):
//                          the partition-of-unity form B of Sec. 4.3.
// One thread per (node, group of 4 columns); grid.y = box.  The stencil is
// read once per node (structure of arrays, coalesced across nodes); the
// column groups of a node share it through the cache.
#include "internal.hpp"

namespace msg {

__global__ __launch_bounds__(256) void k_spmm(const BoxMeta* __restrict__ meta,
                                              const double* __restrict__ stencil,
                                              const uint8_t* __restrict__ cls,
                                              const double* __restrict__ mu1,
                                              const double* __restrict__ X, double* Y,
                                              double* Y2, int k, int y_classes,
                                              double scale, const int32_t* __restrict__ active) {
  int box = blockIdx.y;
  if (active && !active[box]) return;
  const BoxMeta& bm = meta[box];
  int nq = (k + 3) >> 2;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)bm.n_nodes * nq) return;
  int node = (int)(t / nq), q = (int)(t % nq);
  int c0 = 4 * q;
  int li = node % bm.mx, lj = (node / bm.mx) % bm.my, lk = node / (bm.mx * bm.my);
  const double* st = stencil + bm.node_off * 243;
  const uint8_t* cl = cls + bm.dof_off;
  const double* m1 = mu1 + bm.dof_off;
  const double* x = X + (bm.dof_off * k);
  double acc[3][4] = {}, acc2[3][4] = {};
  const bool two = Y2 != nullptr;
  for (int dz = -1; dz <= 1; ++dz) {
    int kk = lk + dz;
    if (kk < 0 || kk >= bm.mz) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      int jj = lj + dy;
      if (jj < 0 || jj >= bm.my) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        int ii = li + dx;
        if (ii < 0 || ii >= bm.mx) continue;
        int nn = ii + bm.mx * (jj + bm.my * kk);
        int nb = nb_index(dx, dy, dz);
        double xv[3][4], xm[3][4];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          int d = 3 * nn + cc;
          bool ok = cl[d] != 3;
          double mu = m1[d];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            double v = (ok && c0 + j < k) ? x[(int64_t)d * k + c0 + j] : 0.0;
            xv[cc][j] = v;
            xm[cc][j] = mu * v;
          }
        }
#pragma unroll
        for (int cr = 0; cr < 3; ++cr)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            double a = st[(int64_t)(nb * 9 + 3 * cr + cc) * bm.n_nodes + node];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              acc[cr][j] += a * xv[cc][j];
              if (two) acc2[cr][j] += a * xm[cc][j];
            }
          }
      }
    }
  }
  double* y = Y ? Y + (bm.dof_off * k) : nullptr;
  double* y2 = two ? Y2 + (bm.dof_off * k) : nullptr;
#pragma unroll
  for (int cr = 0; cr < 3; ++cr) {
    int d = 3 * node + cr;
    uint8_t kc = cl[d];
    bool w = (y_classes >> kc) & 1;
    double mu = m1[d];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (c0 + j < k) {
        if (y) y[(int64_t)d * k + c0 + j] = w ? scale * acc[cr][j] : 0.0;
        if (two) y2[(int64_t)d * k + c0 + j] = mu * acc2[cr][j];
      }
    }
  }
}

}  // namespace msg
