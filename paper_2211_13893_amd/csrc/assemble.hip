// Assembly of the local operators on every oversampled box (Sec. 2, 4.2, 4.3).
//
//  k_materials      : ply stiffness from engineering constants, rotated about z
//                     by the 6x6 Bond matrix (the oracle rotates the 4th-order
//                     tensor instead).
//  k_pou_total      : sum over all subdomains of the capped hop distances
//                     w_{i,p} (Sec. 4.2) at every mesh node (integer atomics,
//                     hence exact and order independent).
//  k_assemble       : one wavefront per box node; lane (e, b) integrates the
//                     3x3 block (a, b) of the element stiffness of the e-th
//                     element around the node with the 2x2x2 Gauss rule and the
//                     lanes are summed in a fixed order into the node's 27
//                     stencil blocks (a_{Omega*} = sum of a_e over e in Omega*).
//  k_classes_mu     : DoF classes B1/B2/B3 (Sec. 4.3) and mu_j restricted to B1.
#include "internal.hpp"

namespace msg {

__global__ void k_materials(const double* __restrict__ mat, int n_mat, double* __restrict__ ctab) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_mat) return;
  const double* p = mat + 10 * m;
  double E1 = p[0], E2 = p[1], E3 = p[2], G12 = p[3], G13 = p[4], G23 = p[5];
  double n12 = p[6], n13 = p[7], n23 = p[8], th = p[9] * (M_PI / 180.0);
  // normal compliance block and its inverse by cofactors
  double s11 = 1.0 / E1, s22 = 1.0 / E2, s33 = 1.0 / E3;
  double s12 = -n12 / E1, s13 = -n13 / E1, s23 = -n23 / E2;
  double c11 = s22 * s33 - s23 * s23, c12 = s13 * s23 - s12 * s33, c13 = s12 * s23 - s13 * s22;
  double c22 = s11 * s33 - s13 * s13, c23 = s12 * s13 - s11 * s23, c33 = s11 * s22 - s12 * s12;
  double det = s11 * c11 + s12 * c12 + s13 * c13;
  double C[6][6] = {};
  C[0][0] = c11 / det; C[0][1] = C[1][0] = c12 / det; C[0][2] = C[2][0] = c13 / det;
  C[1][1] = c22 / det; C[1][2] = C[2][1] = c23 / det; C[2][2] = c33 / det;
  C[3][3] = G23; C[4][4] = G13; C[5][5] = G12;
  // Bond stress matrix of the rotation a = R_z(th) (material -> global)
  double cs = cos(th), sn = sin(th);
  double a[3][3] = {{cs, -sn, 0.0}, {sn, cs, 0.0}, {0.0, 0.0, 1.0}};
  const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
  double K[6][6];
  for (int I = 0; I < 6; ++I) {
    int i = vi[I], j = vj[I];
    for (int J = 0; J < 6; ++J) {
      int k = vi[J], l = vj[J];
      if (J < 3) K[I][J] = a[i][k] * a[j][l];
      else K[I][J] = a[i][k] * a[j][l] + a[i][l] * a[j][k];
    }
  }
  double T[6][6];
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      double s = 0.0;
      for (int L = 0; L < 6; ++L) s += K[I][L] * C[L][J];
      T[I][J] = s;
    }
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      double s = 0.0;
      for (int L = 0; L < 6; ++L) s += T[I][L] * K[J][L];
      ctab[36 * m + 6 * I + J] = s;
    }
}

// capped Chebyshev distance of node (i,j,k) to the interior faces of the
// Omega box [lo, hi] (inclusive), 0 outside the box and on interior faces.
__device__ inline int pou_weight(int i, int j, int k, const int* lo, const int* hi,
                                 const int* lo_int, const int* hi_int, int cap) {
  int idx[3] = {i, j, k};
  int w = cap;
  for (int d = 0; d < 3; ++d) {
    if (idx[d] < lo[d] || idx[d] > hi[d]) return 0;
    if (lo_int[d]) w = min(w, idx[d] - lo[d]);
    if (hi_int[d]) w = min(w, hi[d] - idx[d]);
  }
  return w;
}

// omega: [nsd][6] node boxes (lo_x,lo_y,lo_z,hi_x,hi_y,hi_z, inclusive)
__global__ void k_pou_total(const int32_t* __restrict__ omega, int nsd, int nx, int ny, int nz,
                            int cap, int32_t* __restrict__ wtot) {
  int sd = blockIdx.y;
  if (sd >= nsd) return;
  const int32_t* ob = omega + 6 * sd;
  int lo[3] = {ob[0], ob[1], ob[2]}, hi[3] = {ob[3], ob[4], ob[5]};
  int N[3] = {nx, ny, nz};
  int lo_int[3], hi_int[3];
  for (int d = 0; d < 3; ++d) { lo_int[d] = lo[d] > 0; hi_int[d] = hi[d] < N[d]; }
  int sx = hi[0] - lo[0] + 1, sy = hi[1] - lo[1] + 1, sz = hi[2] - lo[2] + 1;
  int64_t cnt = (int64_t)sx * sy * sz;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < cnt;
       t += (int64_t)gridDim.x * blockDim.x) {
    int i = lo[0] + (int)(t % sx);
    int j = lo[1] + (int)((t / sx) % sy);
    int k = lo[2] + (int)(t / ((int64_t)sx * sy));
    int w = pou_weight(i, j, k, lo, hi, lo_int, hi_int, cap);
    if (w > 0) {
      int64_t g = i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k);
      atomicAdd(&wtot[g], w);
    }
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

// One wavefront per node of a box.  blockDim = 256 (4 nodes per block);
// grid.x covers the nodes of the largest box, grid.y = box.
__global__ __launch_bounds__(256) void k_assemble(const BoxMeta* __restrict__ meta, MeshDev mesh,
                                                  const double* __restrict__ ctab,
                                                  double* __restrict__ stencil) {
  __shared__ double acc[4][243];
  const BoxMeta& bm = meta[blockIdx.y];
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int node = blockIdx.x * 4 + wave;
  for (int t = lane; t < 243; t += 64) acc[wave][t] = 0.0;
  bool valid = node < bm.n_nodes;
  int li = 0, lj = 0, lk = 0;
  if (valid) {
    li = node % bm.mx;
    lj = (node / bm.mx) % bm.my;
    lk = node / (bm.mx * bm.my);
  }
  int e = lane >> 3, b = lane & 7;
  int bx = e & 1, by = (e >> 1) & 1, bz = (e >> 2) & 1;
  // element lower corner (box-relative node coords)
  int ex = li + bx - 1, ey = lj + by - 1, ez = lk + bz - 1;
  bool inbox = valid && ex >= 0 && ey >= 0 && ez >= 0 && ex < bm.mx - 1 && ey < bm.my - 1 &&
               ez < bm.mz - 1;
  int a = (1 - bx) + 2 * (1 - by) + 4 * (1 - bz);
  int dx = (b & 1) - (a & 1), dy = ((b >> 1) & 1) - ((a >> 1) & 1), dz = ((b >> 2) & 1) - ((a >> 2) & 1);
  double blk[3][3] = {};
  if (inbox) {
    int gx = bm.g0[0] + ex, gy = bm.g0[1] + ey, gz = bm.g0[2] + ez;
    int64_t eid = gx + (int64_t)mesh.nx * (gy + (int64_t)mesh.ny * gz);
    const double* C = ctab + 36 * mesh.elem_mat[eid];
    double X[8][3];
    for (int q = 0; q < 8; ++q) {
      int64_t gn = (gx + (q & 1)) + (int64_t)(mesh.nx + 1) *
                   ((gy + ((q >> 1) & 1)) + (int64_t)(mesh.ny + 1) * (gz + ((q >> 2) & 1)));
      X[q][0] = mesh.xyz[3 * gn + 0];
      X[q][1] = mesh.xyz[3 * gn + 1];
      X[q][2] = mesh.xyz[3 * gn + 2];
    }
    double Cl[36];
    for (int q = 0; q < 36; ++q) Cl[q] = C[q];
    const double gp = 0.57735026918962576451;  // 1/sqrt(3)
    double ra[3] = {(double)(2 * (a & 1) - 1), (double)(2 * ((a >> 1) & 1) - 1), (double)(2 * ((a >> 2) & 1) - 1)};
    double rb[3] = {(double)(2 * (b & 1) - 1), (double)(2 * ((b >> 1) & 1) - 1), (double)(2 * ((b >> 2) & 1) - 1)};
    for (int g = 0; g < 8; ++g) {
      double xi[3] = {(g & 1) ? gp : -gp, ((g >> 1) & 1) ? gp : -gp, ((g >> 2) & 1) ? gp : -gp};
      // Jacobian J[d][c] = sum_q dN_q/dxi_d * x_q[c]
      double J[3][3] = {};
      for (int q = 0; q < 8; ++q) {
        double r0 = 2 * (q & 1) - 1, r1 = 2 * ((q >> 1) & 1) - 1, r2 = 2 * ((q >> 2) & 1) - 1;
        double f0 = 1 + r0 * xi[0], f1 = 1 + r1 * xi[1], f2 = 1 + r2 * xi[2];
        double d0 = 0.125 * r0 * f1 * f2, d1 = 0.125 * f0 * r1 * f2, d2 = 0.125 * f0 * f1 * r2;
        for (int c = 0; c < 3; ++c) {
          J[0][c] += d0 * X[q][c];
          J[1][c] += d1 * X[q][c];
          J[2][c] += d2 * X[q][c];
        }
      }
      double i00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      double i01 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
      double i02 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
      double i10 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      double i11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
      double i12 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
      double i20 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      double i21 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
      double i22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      double detJ = J[0][0] * i00 + J[0][1] * i10 + J[0][2] * i20;
      double inv = 1.0 / detJ;
      // grad_x N = J^{-1} grad_xi N
      double da[3] = {0.125 * ra[0] * (1 + ra[1] * xi[1]) * (1 + ra[2] * xi[2]),
                      0.125 * (1 + ra[0] * xi[0]) * ra[1] * (1 + ra[2] * xi[2]),
                      0.125 * (1 + ra[0] * xi[0]) * (1 + ra[1] * xi[1]) * ra[2]};
      double db[3] = {0.125 * rb[0] * (1 + rb[1] * xi[1]) * (1 + rb[2] * xi[2]),
                      0.125 * (1 + rb[0] * xi[0]) * rb[1] * (1 + rb[2] * xi[2]),
                      0.125 * (1 + rb[0] * xi[0]) * (1 + rb[1] * xi[1]) * rb[2]};
      double ga[3], gb[3];
      ga[0] = inv * (i00 * da[0] + i01 * da[1] + i02 * da[2]);
      ga[1] = inv * (i10 * da[0] + i11 * da[1] + i12 * da[2]);
      ga[2] = inv * (i20 * da[0] + i21 * da[1] + i22 * da[2]);
      gb[0] = inv * (i00 * db[0] + i01 * db[1] + i02 * db[2]);
      gb[1] = inv * (i10 * db[0] + i11 * db[1] + i12 * db[2]);
      gb[2] = inv * (i20 * db[0] + i21 * db[1] + i22 * db[2]);
      // B columns (Voigt 11,22,33,23,13,12; engineering shear)
      double Ba[3][6] = {{ga[0], 0, 0, 0, ga[2], ga[1]},
                         {0, ga[1], 0, ga[2], 0, ga[0]},
                         {0, 0, ga[2], ga[1], ga[0], 0}};
      double Bb[3][6] = {{gb[0], 0, 0, 0, gb[2], gb[1]},
                         {0, gb[1], 0, gb[2], 0, gb[0]},
                         {0, 0, gb[2], gb[1], gb[0], 0}};
      double wd = detJ;  // Gauss weights are 1
      for (int j = 0; j < 3; ++j) {
        double CB[6];
        for (int I = 0; I < 6; ++I) {
          double s = 0.0;
          for (int L = 0; L < 6; ++L) s += Cl[6 * I + L] * Bb[j][L];
          CB[I] = s;
        }
        for (int i = 0; i < 3; ++i) {
          double s = 0.0;
          for (int I = 0; I < 6; ++I) s += Ba[i][I] * CB[I];
          blk[i][j] += wd * s;
        }
      }
    }
  }
  __syncthreads();
  int nb = nb_index(dx, dy, dz);
  for (int pass = 0; pass < 8; ++pass) {
    if (e == pass && inbox) {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) acc[wave][nb * 9 + 3 * i + j] += blk[i][j];
    }
    __syncthreads();
  }
  if (valid) {
    double* out = stencil + bm.node_off * 243;
    for (int t = lane; t < 243; t += 64) out[(int64_t)t * bm.n_nodes + node] = acc[wave][t];
  }
}

// DoF classes (1: B1, 2: B2, 3: B3) and mu1 = mu_j on B1 DoFs, 0 elsewhere.
__global__ void k_classes_mu(const BoxMeta* __restrict__ meta, MeshDev mesh, int cap,
                             const int32_t* __restrict__ wtot, uint8_t* __restrict__ cls,
                             double* __restrict__ mu1) {
  const BoxMeta& bm = meta[blockIdx.y];
  int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= bm.n_nodes) return;
  int li = node % bm.mx, lj = (node / bm.mx) % bm.my, lk = node / (bm.mx * bm.my);
  int l[3] = {li, lj, lk}, m[3] = {bm.mx, bm.my, bm.mz};
  bool b2 = false;
  for (int d = 0; d < 3; ++d) {
    if (bm.iface_lo[d] && l[d] == 0) b2 = true;
    if (bm.iface_hi[d] && l[d] == m[d] - 1) b2 = true;
  }
  int gi = bm.g0[0] + li, gj = bm.g0[1] + lj, gk = bm.g0[2] + lk;
  int64_t gn = gi + (int64_t)(mesh.nx + 1) * (gj + (int64_t)(mesh.ny + 1) * gk);
  int w = pou_weight(gi, gj, gk, bm.olo, bm.ohi, bm.olo_int, bm.ohi_int, cap);
  double mu = (w > 0) ? (double)w / (double)wtot[gn] : 0.0;
  for (int c = 0; c < 3; ++c) {
    int64_t d = bm.dof_off + 3 * node + c;
    uint8_t k = mesh.dirichlet[3 * gn + c] ? 3 : (b2 ? 2 : 1);
    cls[d] = k;
    mu1[d] = (k == 1) ? mu : 0.0;
  }
}

}  // namespace msg
