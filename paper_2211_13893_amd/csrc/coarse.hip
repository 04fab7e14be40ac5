// The MS-GFEM coarse problem from the local spectral stage (Sec. 3.3, 4.3, 4.4).
//
//  k_box_load      : consistent nodal loads b_{Omega*}(phi_i) of the uniform
//                    tractions on the mesh faces that lie in the box (2x2 Gauss on
//                    the bilinear face quads).
//  k_coarse_basis  : V_j = Xi_j(phi_{j,k}) = mu_j phi_{j,k} and the weighted
//                    particular function mu_j psi_j on the box grid.
//  k_cholqr_coef   : Cholesky of V_j^T V_j with dropping of columns whose
//                    orthogonal part is below 1e-12 of the largest column norm,
//                    and the coefficients R^{-1} of the orthonormalised basis
//                    (applied twice: CholQR2, the Gram-Schmidt step of Sec. 4.3).
//  k_coarse_pairs  : Galerkin blocks A^H_{ij} = V_i^T (A V_j) over the node
//                    intersection of Omega_i with the box of Omega_j^*, and
//                    V_i^T A (mu_j psi_j) for the right-hand side.
//  k_coarse_rhs    : b^H_i = V_i^T b - sum_j V_i^T A (mu_j psi_j).
//  k_dense_tiles / k_trsv_* : the coarse matrix in dense tile form for the
//                    tile Cholesky, and the single-RHS solve by column launches.
//  k_store_box / k_store_local32 : a plan's coarse data (and, for GenEO, its
//                    local Dirichlet solve data in FP32) into a coarse store
//                    that gathers every subdomain across plans.
//  k_prolong       : u^G = sum_j R_j^T (mu_j psi_j + V_j c_j).
//  k_error_norms   : the relative L2 errors e_d and e_eps of Sec. 5.3.
#include "internal.hpp"

namespace msg {

// face descriptor: axis (0..2), side (0: low, 1: high), traction g (3)
struct FaceLoad {
  int32_t axis, side;
  double g[3];
};

// Coarse pair: rows of box i, columns of box j, over the global node range [lo, hi]
struct CoarsePair {
  int32_t i, j;
  int32_t lo[3], hi[3];
  int32_t row_off, col_off;   // offsets in the coarse numbering
};

// Adaptive local spaces (Sec. 1 and Sec. 5: a threshold t on the reciprocals
// of the local eigenvalues decides which eigenvectors enter a local space).
// Box j keeps its m_j leading eigenpairs, m_j = #{k < n_ev_j : lambda_k <
// 1/t} (lambda ascending, so 1/lambda_{m_j+1} <= t; the zero eigenvalues of
// floating boxes, at rounding level either side of 0, count while that
// rounding stays below 1/t), and the
// other columns of its eigenvectors are written as zero, which the coarse
// basis then drops.  Status bit 16 when all n_ev_j pass (the threshold may
// need more eigenpairs than were computed).  One workgroup per box.
__global__ __launch_bounds__(256) void k_select_modes(const BoxMeta* __restrict__ meta,
                                                      const double* __restrict__ evals, double inv_t,
                                                      const double* evecs, double* out,
                                                      int32_t* __restrict__ m,
                                                      int32_t* __restrict__ status) {
  __shared__ int keep;
  const BoxMeta& bm = meta[blockIdx.x];
  const int nev = bm.n_ev;
  if (threadIdx.x == 0) {
    int c = 0;
    while (c < nev && evals[bm.eval_off + c] < inv_t) ++c;
    keep = c;
    m[blockIdx.x] = c;
    if (c == nev) status[blockIdx.x] |= 16;
  }
  __syncthreads();
  const int kp = keep;
  const int64_t n = (int64_t)bm.n_dof * nev;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int c = (int)(e % nev);
    out[bm.evec_off + e] = c < kp ? evecs[bm.evec_off + e] : 0.0;
  }
}

__global__ void k_box_load(const BoxMeta* __restrict__ meta, MeshDev mesh,
                           const FaceLoad* __restrict__ faces, int n_faces,
                           double* __restrict__ b) {
  const BoxMeta& bm = meta[blockIdx.y];
  int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= bm.n_nodes) return;
  int l[3] = {node % bm.mx, (node / bm.mx) % bm.my, node / (bm.mx * bm.my)};
  int gidx[3] = {bm.g0[0] + l[0], bm.g0[1] + l[1], bm.g0[2] + l[2]};
  int m[3] = {bm.mx, bm.my, bm.mz};
  int N[3] = {mesh.nx, mesh.ny, mesh.nz};
  double acc[3] = {0.0, 0.0, 0.0};
  const double gp = 0.57735026918962576451;
  for (int f = 0; f < n_faces; ++f) {
    const int ax = faces[f].axis, side = faces[f].side;
    if (gidx[ax] != (side ? N[ax] : 0)) continue;
    const int e1 = (ax + 1) % 3, e2 = (ax + 2) % 3;
    // quads with lower in-face corner (u0, v0), u0 in {l-1, l}, inside the box
    for (int du = -1; du <= 0; ++du)
      for (int dv = -1; dv <= 0; ++dv) {
        int u0 = l[e1] + du, v0 = l[e2] + dv;
        if (u0 < 0 || v0 < 0 || u0 >= m[e1] - 1 || v0 >= m[e2] - 1) continue;
        // corner coordinates of the quad (global nodes)
        double X[2][2][3];
        for (int a1 = 0; a1 < 2; ++a1)
          for (int a2 = 0; a2 < 2; ++a2) {
            int gi[3];
            gi[ax] = gidx[ax];
            gi[e1] = bm.g0[e1] + u0 + a1;
            gi[e2] = bm.g0[e2] + v0 + a2;
            int64_t gn = gi[0] + (int64_t)(mesh.nx + 1) * (gi[1] + (int64_t)(mesh.ny + 1) * gi[2]);
            for (int c = 0; c < 3; ++c) X[a1][a2][c] = mesh.xyz[3 * gn + c];
          }
        const int c1 = l[e1] - u0, c2 = l[e2] - v0;  // this node's corner
        const double r1 = 2 * c1 - 1, r2 = 2 * c2 - 1;
        for (int q1 = 0; q1 < 2; ++q1)
          for (int q2 = 0; q2 < 2; ++q2) {
            double s1 = q1 ? gp : -gp, s2 = q2 ? gp : -gp;
            double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
            for (int a1 = 0; a1 < 2; ++a1)
              for (int a2 = 0; a2 < 2; ++a2) {
                double p1 = 2 * a1 - 1, p2 = 2 * a2 - 1;
                double d1 = 0.25 * p1 * (1 + p2 * s2), d2 = 0.25 * (1 + p1 * s1) * p2;
                for (int c = 0; c < 3; ++c) {
                  t1[c] += d1 * X[a1][a2][c];
                  t2[c] += d2 * X[a1][a2][c];
                }
              }
            double nx_ = t1[1] * t2[2] - t1[2] * t2[1];
            double ny_ = t1[2] * t2[0] - t1[0] * t2[2];
            double nz_ = t1[0] * t2[1] - t1[1] * t2[0];
            double dA = sqrt(nx_ * nx_ + ny_ * ny_ + nz_ * nz_);
            double Nn = 0.25 * (1 + r1 * s1) * (1 + r2 * s2);
            for (int c = 0; c < 3; ++c) acc[c] += Nn * faces[f].g[c] * dA;
          }
      }
  }
  for (int c = 0; c < 3; ++c) b[bm.dof_off + 3 * node + c] = acc[c];
}

// V[dof][c] = mu1[dof] * phi[dof][c] (c < n_ev, 0 above), pv[dof] = mu1[dof] * psi[dof]
__global__ void k_coarse_basis(const BoxMeta* __restrict__ meta, int k, const double* __restrict__ mu1,
                               const double* __restrict__ evecs, const double* __restrict__ psi,
                               double* __restrict__ V, double* __restrict__ pv) {
  const BoxMeta& bm = meta[blockIdx.y];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)bm.n_dof * k) return;
  int dof = (int)(t / k), c = (int)(t % k);
  double mu = mu1[bm.dof_off + dof];
  V[bm.dof_off * k + t] = (c < bm.n_ev) ? mu * evecs[bm.evec_off + (int64_t)dof * bm.n_ev + c] : 0.0;
  if (c == 0) pv[bm.dof_off + dof] = mu * psi[bm.dof_off + dof];
}

// One workgroup per box: Y = R^{-1} of the Cholesky factor R^T R = V^T V with
// dropped columns zeroed.  G is [box][2][k][k] (the first copy is used).
__global__ __launch_bounds__(256) void k_cholqr_coef(int k, const double* __restrict__ G,
                                                     double* __restrict__ Y) {
  extern __shared__ double sm[];
  const int box = blockIdx.x, ld = k + 1, tid = threadIdx.x;
  double* C = sm;            // k x (k+1)
  int* drop = (int*)(C + k * ld);
  const double* g = G + (int64_t)box * 2 * k * k;
  double gmax = 0.0;
  for (int i = 0; i < k; ++i) gmax = fmax(gmax, g[i * k + i]);
  const double thr = 1e-24 * gmax;   // (1e-12 of the largest column norm)^2
  for (int t = tid; t < k * k; t += 256) {
    int i = t / k, j = t % k;
    C[i * ld + j] = 0.5 * (g[i * k + j] + g[j * k + i]);
  }
  for (int t = tid; t < k; t += 256) drop[t] = 0;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    double piv = C[j * ld + j];
    bool dj = !(piv > thr) || gmax == 0.0;
    if (dj) {
      for (int t = tid; t < k; t += 256) {
        if (t > j) C[t * ld + j] = 0.0;
        if (t < j) C[j * ld + t] = 0.0;
      }
      if (tid == 0) { C[j * ld + j] = 1.0; drop[j] = 1; }
      __syncthreads();
      continue;
    }
    double sd = sqrt(piv);
    for (int t = tid; t < k; t += 256)
      if (t > j) C[t * ld + j] /= sd;
    __syncthreads();
    if (tid == 0) C[j * ld + j] = sd;
    for (int t = tid; t < k * k; t += 256) {
      int i = t / k, c = t % k;
      if (i > j && c > j && c <= i) C[i * ld + c] -= C[i * ld + j] * C[c * ld + j];
    }
    __syncthreads();
  }
  // Y = L^{-T} (upper triangular), column c by back substitution: L^T y = e_c
  double* Yb = Y + (int64_t)box * k * k;
  for (int c = tid; c < k; c += 256) {
    for (int i = k - 1; i >= 0; --i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int q = i + 1; q < k; ++q) s -= C[q * ld + i] * Yb[q * k + c];
      Yb[i * k + c] = s / C[i * ld + i];
    }
  }
  __syncthreads();
  for (int t = tid; t < k * k; t += 256) {
    int i = t / k, c = t % k;
    if (drop[i] || drop[c]) Yb[t] = 0.0;
  }
}

// One workgroup per pair.  outputs (a, b), a < n_ev(i), b <= n_ev(j) (b = n_ev(j)
// is the particular column); AH row-major NH x NH; rpart[pair][rstride]
// (rstride >= every n_ev).
__global__ __launch_bounds__(256) void k_coarse_pairs(const BoxMeta* __restrict__ meta,
                                                      const CoarsePair* __restrict__ pairs, int k,
                                                      const double* __restrict__ V,
                                                      const double* __restrict__ AV,
                                                      const double* __restrict__ Ap, int NH, int rstride,
                                                      double* __restrict__ AH,
                                                      double* __restrict__ rpart) {
  const CoarsePair pr = pairs[blockIdx.x];
  const BoxMeta& bi = meta[pr.i];
  const BoxMeta& bj = meta[pr.j];
  const int na = bi.n_ev, nbc = bj.n_ev + 1;
  const int sx = pr.hi[0] - pr.lo[0] + 1, sy = pr.hi[1] - pr.lo[1] + 1, sz = pr.hi[2] - pr.lo[2] + 1;
  const int64_t nn = (int64_t)sx * sy * sz;
  const double* Vi = V + bi.dof_off * k;
  const double* AVj = AV + bj.dof_off * k;
  const double* Apj = Ap + bj.dof_off;
  for (int o = threadIdx.x; o < na * nbc; o += 256) {
    const int a = o / nbc, b = o % nbc;
    double acc = 0.0;
    for (int64_t t = 0; t < nn; ++t) {
      int gx = pr.lo[0] + (int)(t % sx), gy = pr.lo[1] + (int)((t / sx) % sy), gz = pr.lo[2] + (int)(t / ((int64_t)sx * sy));
      int ni = (gx - bi.g0[0]) + bi.mx * ((gy - bi.g0[1]) + bi.my * (gz - bi.g0[2]));
      int nj = (gx - bj.g0[0]) + bj.mx * ((gy - bj.g0[1]) + bj.my * (gz - bj.g0[2]));
      for (int c = 0; c < 3; ++c) {
        double vi = Vi[(int64_t)(3 * ni + c) * k + a];
        double w = (b < bj.n_ev) ? AVj[(int64_t)(3 * nj + c) * k + b] : Apj[3 * nj + c];
        acc += vi * w;
      }
    }
    if (b < bj.n_ev) AH[(int64_t)(pr.row_off + a) * NH + pr.col_off + b] = acc;
    else rpart[(int64_t)blockIdx.x * rstride + a] = acc;
  }
}

// b^H_i[a] = V_i[:,a]^T b_i - sum over the pairs of row box i of rpart; a unit
// diagonal for dropped (zero) coarse functions.  One workgroup per box.
__global__ __launch_bounds__(256) void k_coarse_rhs(const BoxMeta* __restrict__ meta, int k,
                                                    const double* __restrict__ V,
                                                    const double* __restrict__ bload,
                                                    const int32_t* __restrict__ pair_start,
                                                    const int32_t* __restrict__ row_off, int NH, int rstride,
                                                    const double* __restrict__ rpart,
                                                    double* __restrict__ AH,
                                                    double* __restrict__ bH) {
  __shared__ double red[256];
  const int box = blockIdx.x;
  const BoxMeta& bm = meta[box];
  const double* Vb = V + bm.dof_off * k;
  const double* bb = bload + bm.dof_off;
  for (int a = 0; a < bm.n_ev; ++a) {
    double s = 0.0;
    for (int d = threadIdx.x; d < bm.n_dof; d += 256) s += Vb[(int64_t)d * k + a] * bb[d];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double r = red[0];
      for (int p = pair_start[box]; p < pair_start[box + 1]; ++p) r -= rpart[(int64_t)p * rstride + a];
      const int64_t l = row_off[box] + a;
      bH[l] = r;
      if (AH[l * NH + l] == 0.0) AH[l * NH + l] = 1.0;
    }
    __syncthreads();
  }
}

// dense NH x NH (row-major) -> tile-band storage with BT = NT (lower tiles, identity padding)
__global__ void k_dense_tiles(const double* __restrict__ AH, int NH, int NT, double* __restrict__ T) {
  int64_t total = (int64_t)NT * NT * MSG_TILE2;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int e = (int)(t & 1023);
    int64_t tile = t >> 10;
    int I = (int)(tile / NT), s = (int)(tile % NT);
    int row = I * 32 + (e >> 5), col = (I - s) * 32 + (e & 31);
    double v = 0.0;
    if (col >= 0 && col <= row) {
      if (row < NH && col < NH) v = AH[(int64_t)row * NH + col];
      else v = (row == col) ? 1.0 : 0.0;
    }
    T[t] = v;
  }
}

// Multi-workgroup single-RHS solve with the unit-lower tile factor A = Lu D Lu^T
// of a dense matrix (BT = NT, D^{-1} in the diagonal tile slot), in three
// phases of launches: forward columns J = 0..NT-2 (y_I -= Lu(I,J) y_J for
// every I > J, one workgroup per I; y_J is final once launch J-1 is done),
// w = D^{-1} y, then backward columns J = NT-1..1 (x_I -= Lu(J,I)^T x_J for
// every I < J).  y starts as b (zero past NH).
__global__ void k_trsv_init(const double* __restrict__ b, int NH, int n, double* __restrict__ y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) y[i] = i < NH ? b[i] : 0.0;
}

// 256 threads per target tile: thread t takes row t >> 3 and inner indices
// 4 (t & 7) .. +3 (32 contiguous bytes per thread, a tile row per 8 lanes)
__global__ __launch_bounds__(256) void k_trsv_fwd(const double* __restrict__ T, int NT, int J, double* __restrict__ y) {
  const int I = J + 1 + blockIdx.x;
  if (I >= NT) return;
  const int t = threadIdx.x, r = t >> 3, q0 = 4 * (t & 7);
  const double* L = T + ((int64_t)I * NT + (I - J)) * MSG_TILE2 + r * 32 + q0;
  const double* yj = y + (int64_t)J * 32 + q0;
  double acc = L[0] * yj[0] + L[1] * yj[1] + L[2] * yj[2] + L[3] * yj[3];
  acc += __shfl_xor(acc, 1);
  acc += __shfl_xor(acc, 2);
  acc += __shfl_xor(acc, 4);
  if ((t & 7) == 0) y[(int64_t)I * 32 + r] -= acc;
}

// w_I = D^{-1}_I y_I into x, one workgroup per tile row
__global__ __launch_bounds__(256) void k_trsv_diag(const double* __restrict__ T, int NT, const double* __restrict__ y,
                                                   double* __restrict__ x) {
  const int I = blockIdx.x, t = threadIdx.x, r = t >> 3, q0 = 4 * (t & 7);
  const double* D = T + ((int64_t)I * NT) * MSG_TILE2 + r * 32 + q0;
  const double* yi = y + (int64_t)I * 32 + q0;
  double acc = D[0] * yi[0] + D[1] * yi[1] + D[2] * yi[2] + D[3] * yi[3];
  acc += __shfl_xor(acc, 1);
  acc += __shfl_xor(acc, 2);
  acc += __shfl_xor(acc, 4);
  if ((t & 7) == 0) x[(int64_t)I * 32 + r] = acc;
}

// 256 threads per target: thread t takes output row r = t & 31 and inner
// indices 4 (t >> 5) .. +3 (a column of Lu(J,I) read across the lanes), the
// eight partial sums added in LDS in a fixed order
__global__ __launch_bounds__(256) void k_trsv_bwd(const double* __restrict__ T, int NT, int J, double* __restrict__ x) {
  __shared__ double part[8][32];
  const int I = blockIdx.x;
  if (I >= J) return;
  const int t = threadIdx.x, r = t & 31, g = t >> 5;
  const double* L = T + ((int64_t)J * NT + (J - I)) * MSG_TILE2;
  const double* xj = x + (int64_t)J * 32;
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) acc += L[(4 * g + u) * 32 + r] * xj[4 * g + u];
  part[g][r] = acc;
  __syncthreads();
  if (t < 32) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += part[q][t];
    x[(int64_t)I * 32 + t] -= s;
  }
}

// Export of one plan's coarse data into a coarse store: box b of the plan is
// subdomain pm.sd, whose slot in the store is described by smeta[pm.sd].
// V, AV: plan block layout [n_dof][kp]; the store keeps kc columns.
__global__ void k_store_box(const BoxMeta* __restrict__ pmeta, const BoxMeta* __restrict__ smeta, int kp, int kc,
                            const double* __restrict__ V, const double* __restrict__ AV, const double* __restrict__ pv,
                            const double* __restrict__ Ap, const double* __restrict__ bload,
                            const uint8_t* __restrict__ cls, double* __restrict__ sV, double* __restrict__ sAV,
                            double* __restrict__ spv, double* __restrict__ sAp, double* __restrict__ sbload,
                            uint8_t* __restrict__ scls) {
  const BoxMeta& pm = pmeta[blockIdx.y];
  const BoxMeta& sm = smeta[pm.sd];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)pm.n_dof * kc) return;
  const int dof = (int)(t / kc), c = (int)(t % kc);
  const int64_t pr = pm.dof_off + dof, sr = sm.dof_off + dof;
  sV[sr * kc + c] = c < kp ? V[pr * kp + c] : 0.0;
  sAV[sr * kc + c] = c < kp ? AV[pr * kp + c] : 0.0;
  if (c == 0) {
    spv[sr] = pv[pr];
    sAp[sr] = Ap[pr];
    sbload[sr] = bload[pr];
    scls[sr] = cls[pr];
  }
}

// FP32 copies of the two solve-ordered copies of every part of a plan box's
// A11 factor and of its D^{-1} tiles into the store's local-solve area
// (element offsets fw / bw / ioff of smeta[sd].part[0][*], the last compact:
// BOX_COMPACT_DINV)
__global__ void k_store_local32(const BoxMeta* __restrict__ pmeta, const BoxMeta* __restrict__ smeta,
                                const double* __restrict__ fac, float* __restrict__ loc) {
  const BoxMeta& pm = pmeta[blockIdx.y];
  const BoxMeta& sm = smeta[pm.sd];
  for (int pi = 0; pi < (pm.nd[0] ? 3 : 1); ++pi) {
    const BandPart& q = pm.part[0][pi];
    const BandPart& t = sm.part[0][pi];
    const int64_t n = solve_copy_doubles(q.NT, q.BT);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
      loc[t.fw + e] = (float)fac[q.fw + e];
      loc[t.bw + e] = (float)fac[q.bw + e];
    }
    // the D^{-1} tiles the vector-FMA solve reads from the band's diagonal slot
    // (the matrix-core layout keeps them in its forward copy), compactly
    const int64_t nd = (int64_t)q.NT * MSG_TILE2;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nd; e += (int64_t)gridDim.x * blockDim.x)
      loc[t.ioff + e] = (float)fac[q.off + (e >> 10) * q.BT * MSG_TILE2 + (e & 1023)];
  }
}

// u^G[global dof] += mu_j psi_j + V_j c_j (atomic over the boxes sharing a node)
__global__ void k_prolong(const BoxMeta* __restrict__ meta, MeshDev mesh, int k,
                          const double* __restrict__ V, const double* __restrict__ pv,
                          const double* __restrict__ c, const int32_t* __restrict__ row_off,
                          double* __restrict__ uG, double* __restrict__ up) {
  const int box = blockIdx.y;
  const BoxMeta& bm = meta[box];
  int dof = blockIdx.x * blockDim.x + threadIdx.x;
  if (dof >= bm.n_dof) return;
  int node = dof / 3, comp = dof % 3;
  int gi = bm.g0[0] + node % bm.mx, gj = bm.g0[1] + (node / bm.mx) % bm.my,
      gk = bm.g0[2] + node / (bm.mx * bm.my);
  int64_t gd = 3 * (gi + (int64_t)(mesh.nx + 1) * (gj + (int64_t)(mesh.ny + 1) * gk)) + comp;
  const double* Vr = V + (bm.dof_off + dof) * k;
  const double* cb = c + row_off[box];
  double p = pv[bm.dof_off + dof];
  double s = p;
  for (int a = 0; a < bm.n_ev; ++a) s += Vr[a] * cb[a];
  if (s != 0.0) atomicAdd(&uG[gd], s);
  if (up && p != 0.0) atomicAdd(&up[gd], p);
}

// Error metrics of Sec. 5.3: relative L2 errors of the displacement and of the
// strain between a reference field u_h and an approximation u, as integrals
// over the whole mesh by the 2x2x2 Gauss rule of the element stiffness (exact
// for trilinear fields on parallelepiped elements).  The strain is the
// symmetric gradient, measured by its Frobenius norm (each shear component
// counted twice).  out = [int |u_h - u|^2, int |u_h|^2, int |eps(u_h - u)|^2,
// int |eps(u_h)|^2, e_d, e_eps].  One workgroup with a fixed summation order,
// so repeated calls give identical bits; the nodal values are re-read per
// Gauss point from the caches rather than held in registers.
#define ERR_THREADS 1024
__global__ __launch_bounds__(ERR_THREADS) void k_error_norms(MeshDev mesh, const double* __restrict__ uref,
                                                             const double* __restrict__ u,
                                                             double* __restrict__ out) {
  __shared__ double red[4][ERR_THREADS];
  const int tid = threadIdx.x;
  const int nx1 = mesh.nx + 1, ny1 = mesh.ny + 1;
  const int64_t ne = (int64_t)mesh.nx * mesh.ny * mesh.nz;
  const double gq = 0.57735026918962576451;   // 1/sqrt(3): 2-point Gauss abscissa, weight 1
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t e = tid; e < ne; e += ERR_THREADS) {
    const int ei = (int)(e % mesh.nx);
    const int ej = (int)((e / mesh.nx) % mesh.ny);
    const int ek = (int)(e / ((int64_t)mesh.nx * mesh.ny));
    int64_t nd[8];
    for (int a = 0; a < 8; ++a)
      nd[a] = (ei + (a & 1)) + (int64_t)nx1 * ((ej + ((a >> 1) & 1)) + (int64_t)ny1 * (ek + ((a >> 2) & 1)));
    for (int g = 0; g < 8; ++g) {
      const double xi[3] = {(g & 1) ? gq : -gq, (g & 2) ? gq : -gq, (g & 4) ? gq : -gq};
      // J[d][c] = d x_c / d xi_d
      double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      for (int a = 0; a < 8; ++a) {
        const double r0 = (a & 1) ? 1.0 : -1.0, r1 = (a & 2) ? 1.0 : -1.0, r2 = (a & 4) ? 1.0 : -1.0;
        const double f0 = 1.0 + r0 * xi[0], f1 = 1.0 + r1 * xi[1], f2 = 1.0 + r2 * xi[2];
        const double dn[3] = {0.125 * r0 * f1 * f2, 0.125 * f0 * r1 * f2, 0.125 * f0 * f1 * r2};
        for (int c = 0; c < 3; ++c) {
          const double x = mesh.xyz[3 * nd[a] + c];
          for (int d = 0; d < 3; ++d) J[d][c] += dn[d] * x;
        }
      }
      const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
      const double id = 1.0 / det;
      // Ji = J^{-1}: grad_x N = Ji grad_xi N
      const double Ji[3][3] = {
          {c00 * id, (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id, (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id},
          {c01 * id, (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id, (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id},
          {c02 * id, (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id, (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id}};
      double vr[3] = {0, 0, 0}, vd[3] = {0, 0, 0};
      double Gr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Gd[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      for (int a = 0; a < 8; ++a) {
        const double r0 = (a & 1) ? 1.0 : -1.0, r1 = (a & 2) ? 1.0 : -1.0, r2 = (a & 4) ? 1.0 : -1.0;
        const double f0 = 1.0 + r0 * xi[0], f1 = 1.0 + r1 * xi[1], f2 = 1.0 + r2 * xi[2];
        const double n = 0.125 * f0 * f1 * f2;
        const double dn[3] = {0.125 * r0 * f1 * f2, 0.125 * f0 * r1 * f2, 0.125 * f0 * f1 * r2};
        double dx[3];
        for (int c = 0; c < 3; ++c) dx[c] = Ji[c][0] * dn[0] + Ji[c][1] * dn[1] + Ji[c][2] * dn[2];
        for (int c = 0; c < 3; ++c) {
          const double ra = uref[3 * nd[a] + c];
          const double da = ra - u[3 * nd[a] + c];
          vr[c] += n * ra;
          vd[c] += n * da;
          for (int q = 0; q < 3; ++q) {
            Gr[c][q] += ra * dx[q];
            Gd[c][q] += da * dx[q];
          }
        }
      }
      double sr = 0.0, sd = 0.0, er = 0.0, ed = 0.0;
      for (int c = 0; c < 3; ++c) {
        sr += vr[c] * vr[c];
        sd += vd[c] * vd[c];
        for (int q = 0; q < 3; ++q) {
          const double tr = 0.5 * (Gr[c][q] + Gr[q][c]), td = 0.5 * (Gd[c][q] + Gd[q][c]);
          er += tr * tr;
          ed += td * td;
        }
      }
      const double w = fabs(det);
      acc[0] += w * sd;
      acc[1] += w * sr;
      acc[2] += w * ed;
      acc[3] += w * er;
    }
  }
  for (int q = 0; q < 4; ++q) red[q][tid] = acc[q];
  __syncthreads();
  for (int h = ERR_THREADS / 2; h > 0; h >>= 1) {
    if (tid < h)
      for (int q = 0; q < 4; ++q) red[q][tid] += red[q][tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    for (int q = 0; q < 4; ++q) out[q] = red[q][0];
    for (int q = 0; q < 2; ++q) {
      const double num = red[2 * q][0], den = red[2 * q + 1][0];
      out[4 + q] = den > 0.0 ? sqrt(num / den) : (num == 0.0 ? 0.0 : INFINITY);
    }
  }
}

}  // namespace msg
