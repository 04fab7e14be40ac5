// Two-level additive Schwarz preconditioned CG with the GenEO coarse space
// (Sec. 3.2; the fine reference solve of Sec. 5.3):
//   M^{-1} r = R_0^T A_0^{-1} R_0 r + sum_j R_j^T A_j^{-1} R_j r,
// A_j the Dirichlet matrix of Omega_j (its interior block, factored by the
// local stage of a GenEO plan), R_0^T the PoU-weighted GenEO basis and
// A_0 = R_0 A R_0^T its Galerkin matrix (the coarse problem of that plan).
// The global operator is a block-27 stencil of the whole mesh assembled by the
// same element kernel.  Dot products are reduced in a fixed order.
#include "internal.hpp"

namespace msg {

// global vector -> box vectors (1 column) on the class-1 DoFs of every box
__global__ void k_gather_boxes(const BoxMeta* __restrict__ meta, MeshDev mesh,
                               const uint8_t* __restrict__ cls, const double* __restrict__ g,
                               double* __restrict__ xb) {
  const BoxMeta& bm = meta[blockIdx.y];
  int dof = blockIdx.x * blockDim.x + threadIdx.x;
  if (dof >= bm.n_dof) return;
  int node = dof / 3, comp = dof % 3;
  int gi = bm.g0[0] + node % bm.mx, gj = bm.g0[1] + (node / bm.mx) % bm.my,
      gk = bm.g0[2] + node / (bm.mx * bm.my);
  int64_t gd = 3 * (gi + (int64_t)(mesh.nx + 1) * (gj + (int64_t)(mesh.ny + 1) * gk)) + comp;
  xb[bm.dof_off + dof] = (cls[bm.dof_off + dof] == 1) ? g[gd] : 0.0;
}

// z[global] += zb on the class-1 DoFs of every box
__global__ void k_scatter_boxes(const BoxMeta* __restrict__ meta, MeshDev mesh,
                                const uint8_t* __restrict__ cls, const double* __restrict__ zb,
                                double* __restrict__ z) {
  const BoxMeta& bm = meta[blockIdx.y];
  int dof = blockIdx.x * blockDim.x + threadIdx.x;
  if (dof >= bm.n_dof) return;
  if (cls[bm.dof_off + dof] != 1) return;
  int node = dof / 3, comp = dof % 3;
  int gi = bm.g0[0] + node % bm.mx, gj = bm.g0[1] + (node / bm.mx) % bm.my,
      gk = bm.g0[2] + node / (bm.mx * bm.my);
  int64_t gd = 3 * (gi + (int64_t)(mesh.nx + 1) * (gj + (int64_t)(mesh.ny + 1) * gk)) + comp;
  double v = zb[bm.dof_off + dof];
  if (v != 0.0) atomicAdd(&z[gd], v);
}

// rc[row_off + a] = V_j[:, a]^T rb_j, one workgroup per box
__global__ __launch_bounds__(256) void k_coarse_restrict(const BoxMeta* __restrict__ meta, int k,
                                                         const double* __restrict__ V,
                                                         const double* __restrict__ rb,
                                                         const int32_t* __restrict__ row_off,
                                                         double* __restrict__ rc) {
  __shared__ double red[256];
  const BoxMeta& bm = meta[blockIdx.x];
  const double* Vb = V + bm.dof_off * k;
  const double* r = rb + bm.dof_off;
  for (int a = 0; a < bm.n_ev; ++a) {
    double s = 0.0;
    for (int d = threadIdx.x; d < bm.n_dof; d += 256) s += Vb[(int64_t)d * k + a] * r[d];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) rc[row_off[blockIdx.x] + a] = red[0];
    __syncthreads();
  }
}

// partial dot products of (a, b) over the rows with cls == 1, per block
__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     const uint8_t* __restrict__ cls, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    if (cls[t] == 1) s += a[t] * b[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_dot_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// sc: [0] r.z, [1] p.q, [2] r.z new, [3] r.r, [4] alpha, [5] beta
__global__ void k_pcg_alpha(double* sc) { sc[4] = sc[0] / sc[1]; }
__global__ void k_pcg_beta(double* sc) {
  sc[5] = sc[2] / sc[0];
  sc[0] = sc[2];
}

// x += alpha p, r -= alpha q (free DoFs)
__global__ void k_pcg_xr(const uint8_t* __restrict__ cls, int64_t n, const double* __restrict__ sc,
                         const double* __restrict__ p, const double* __restrict__ q,
                         double* __restrict__ x, double* __restrict__ r) {
  const double al = sc[4];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    if (cls[t] != 1) continue;
    x[t] += al * p[t];
    r[t] -= al * q[t];
  }
}

// p = z + beta p (beta = 0 on the first iteration: sc == nullptr)
__global__ void k_pcg_p(const uint8_t* __restrict__ cls, int64_t n, const double* __restrict__ sc,
                        const double* __restrict__ z, double* __restrict__ p) {
  const double be = sc ? sc[5] : 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = (cls[t] == 1) ? z[t] + be * p[t] : 0.0;
}

// r = b - q on free DoFs, 0 on Dirichlet DoFs
__global__ void k_sub(const uint8_t* __restrict__ cls, int64_t n, const double* __restrict__ b,
                      const double* __restrict__ q, double* __restrict__ r) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    r[t] = (cls[t] == 1) ? b[t] - q[t] : 0.0;
}

}  // namespace msg
