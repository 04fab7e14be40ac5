// Banded SPD factorisations on the oversampled boxes (the block solves that
// use them are in solve.hip).
//
// Two matrices per box are factorised once and reused by every eigensolver
// iteration:
//   kind 0: A11, the Omega^*-stiffness on the B1 DoFs (interior solve defining
//           the A-harmonic extension E = -A11^{-1} A12 and its adjoint),
//           ordered over the node sub-box that holds B1;
//   kind 1: Ahat = A + s*D A D on B1 u B2 (B3 removed), whose B2 trace is the
//           preconditioner of the shifted Schur pencil.
// DoFs of the (sub-)box that do not belong to the matrix become identity rows,
// so the band structure of the lexicographic node order is kept.  Storage is
// 32x32 tiles in band form (see internal.hpp); the Cholesky factor overwrites
// the tiles and the inverses of the diagonal tiles are kept for the solves.
#include "band_view.hpp"

namespace msg {

// One thread per 8 consecutive entries of a tile row; grid.x strides over
// NT*BT*128 of the largest part, grid.y = box, grid.z = part.  Entries of
// padding rows are identity rows, entries between inactive DoFs identity or
// zero, the rest the stencil value (times 1 + s mu_r mu_c for Ahat).  In a
// chain of a split matrix the separator x separator block is left zero (it
// belongs to S alone).
__global__ void k_band_build(const BoxMeta* __restrict__ meta, int kind,
                             const double* __restrict__ stencil, const uint8_t* __restrict__ cls,
                             const double* __restrict__ mu1, double shift, double* __restrict__ fac) {
  const BoxMeta& bm = meta[blockIdx.y];
  const int part = blockIdx.z;
  if (part > 0 && !bm.nd[kind]) return;
  BandView v = band_view(bm, kind, part);
  const bool chain = bm.nd[kind] && part < 2;
  const int sep0 = chain ? v.NTf * MSG_TILE : 0x7fffffff;   // first separator row of a chain
  const int64_t total = (int64_t)v.NT * v.BT * (MSG_TILE2 / 8);
  const double* st = stencil + bm.node_off * 243;
  const uint8_t* cl = cls + bm.dof_off;
  const double* m1 = mu1 + bm.dof_off;
  double* out = fac + v.off;
  const int sxy = v.sx * v.sy;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(t & 127);               // 8-entry group of the tile: row g/4, columns 8(g%4) ..
    const int64_t tile = t >> 7;
    const int I = (int)(tile / v.BT), s = (int)(tile % v.BT);
    const int row = I * MSG_TILE + (g >> 2), col0 = (I - s) * MSG_TILE + 8 * (g & 3);
    double val[8];
    // row: order coordinates, component, DoF, class
    const int rq = band_to_order(v, row);
    const bool rin = rq >= 0;
    const int rnode = rin ? rq / 3 : 0, rc = rin ? rq - 3 * (rq / 3) : 0;
    const int ri = rnode % v.sx, rj = (rnode / v.sx) % v.sy, rk = rnode / sxy;
    const int dr = 3 * (v.base + ri * v.st0 + rj * v.st1 + rk * v.st2) + rc;
    const bool ar = rin && dof_active(kind, cl[dr]);
    const double mr = (kind == 1 && rin) ? m1[dr] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int col = col0 + q;
      double x = 0.0;
      if (col >= 0 && col <= row && !(row >= sep0 && col >= sep0)) {
        const int cq = band_to_order(v, col);
        if (!rin || cq < 0) {
          x = (row == col) ? 1.0 : 0.0;
        } else {
          const int cnode = cq / 3, cc = cq - 3 * cnode;
          const int ci = cnode % v.sx, cj = (cnode / v.sx) % v.sy, ck = cnode / sxy;
          const int di = ci - ri, dj = cj - rj, dk = ck - rk;
          // outside the 27-point neighbourhood the entry is zero whatever the
          // classes (the diagonal is inside): the class byte is read only there
          if (di >= -1 && di <= 1 && dj >= -1 && dj <= 1 && dk >= -1 && dk <= 1) {
            const int dc = 3 * (v.base + ci * v.st0 + cj * v.st1 + ck * v.st2) + cc;
            const bool ac = dof_active(kind, cl[dc]);
            if (!ar || !ac) {
              x = (row == col) ? 1.0 : 0.0;
            } else {
              const int nr = dr / 3;
              const int nbi = 13 + di * v.w0 + dj * v.w1 + dk * v.w2;   // 27-point index of the box offset
              const double a = st[(int64_t)(nbi * 9 + 3 * rc + cc) * bm.n_nodes + nr];
              x = (kind == 1) ? a * (1.0 + shift * mr * m1[dc]) : a;
            }
          }
        }
      }
      val[q] = x;
    }
    double2* o = (double2*)(out + (tile << 10) + (g >> 2) * 32 + 8 * (g & 3));
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = make_double2(val[2 * q], val[2 * q + 1]);
  }
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// 32x32 tile product on one wavefront with the FP64 matrix cores:
// acc (2x2 blocks of 16x16) += sa * A B^T for row-major 32x32 tiles A, B.
// v_mfma_f64_16x16x4f64 lane layout: A operand A[l&15][l>>4], B operand
// B[l>>4][l&15], accumulator item v of lane l = D[(l>>4) + 4v][l&15].
__device__ inline void tile_mfma_abt(const double* __restrict__ A, const double* __restrict__ B,
                                     double sa, dbl4 acc[2][2], int lane) {
  const int i = lane & 15, k = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    double a0 = sa * A[i * 32 + 4 * kk + k];
    double a1 = sa * A[(16 + i) * 32 + 4 * kk + k];
    double b0 = B[i * 32 + 4 * kk + k];
    double b1 = B[(16 + i) * 32 + 4 * kk + k];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// acc += A B for row-major 32x32 tiles (B operand B[k][j] read along rows).
__device__ inline void tile_mfma_ab(const double* __restrict__ A, const double* __restrict__ B,
                                    dbl4 acc[2][2], int lane) {
  const int i = lane & 15, k = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    double a0 = A[i * 32 + 4 * kk + k];
    double a1 = A[(16 + i) * 32 + 4 * kk + k];
    double b0 = B[(4 * kk + k) * 32 + i];
    double b1 = B[(4 * kk + k) * 32 + 16 + i];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// acc += A^T B for row-major 32x32 tiles.
__device__ inline void tile_mfma_atb(const double* __restrict__ A, const double* __restrict__ B,
                                     dbl4 acc[2][2], int lane) {
  const int i = lane & 15, k = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    double a0 = A[(4 * kk + k) * 32 + i];
    double a1 = A[(4 * kk + k) * 32 + 16 + i];
    double b0 = B[(4 * kk + k) * 32 + i];
    double b1 = B[(4 * kk + k) * 32 + 16 + i];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

__device__ inline void tile_load_acc(const double* __restrict__ C, dbl4 acc[2][2], int lane) {
  const int j = lane & 15, r = lane >> 4;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[bi][bj][v] = C[(16 * bi + r + 4 * v) * 32 + 16 * bj + j];
}

__device__ inline void tile_store_acc(double* __restrict__ C, const dbl4 acc[2][2], int lane) {
  const int j = lane & 15, r = lane >> 4;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) C[(16 * bi + r + 4 * v) * 32 + 16 * bj + j] = acc[bi][bj][v];
}

// Value of v in lane j of the wavefront (j uniform).
__device__ inline double lane_value(double v, int j) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cholesky of the diagonal tile T (in place, lower) and the inverse of its
// factor into Ti, by one wavefront without barriers: lane i (mod 32) keeps row
// i of the tile in registers and takes the entries of other rows from their
// lanes (readlane with a compile-time lane index).  Left-looking:
//   L[i][j] = (A[i][j] - sum_{q<j} L[i][q] L[j][q]) / L[j][j];
// then lane c forms column c of L^{-1} by forward substitution.  Returns 1
// if a pivot was not positive (it is replaced by 1).
__device__ int diag_tile_factor(double* __restrict__ T, double* __restrict__ Ti) {
  const int lane = threadIdx.x & 63, i = lane & 31;
  double r[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) r[q] = T[i * 32 + q];
  int bad = 0;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    double s = r[j];
#pragma unroll
    for (int q = 0; q < j; ++q) s -= r[q] * lane_value(r[q], j);
    double d = lane_value(s, j);
    if (!(d > 0.0)) {
      d = 1.0;
      bad = 1;
    }
    const double sd = sqrt(d);
    r[j] = (i == j) ? sd : (i > j ? s / sd : 0.0);
  }
  double x[32];
#pragma unroll
  for (int ii = 0; ii < 32; ++ii) {
    double s = (ii == i) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < ii; ++q) s -= lane_value(r[q], ii) * x[q];
    x[ii] = s / lane_value(r[ii], ii);
  }
  if (lane < 32) {
#pragma unroll
    for (int q = 0; q < 32; ++q) T[i * 32 + q] = r[q];
#pragma unroll
    for (int ii = 0; ii < 32; ++ii) Ti[ii * 32 + i] = x[ii];
  }
  return bad;
}

// Right-looking tile Cholesky, one launch per tile column K (K = -1 first):
// the trailing update with panel K, A(K+sI, K+sJ) -= L(K+sI,K) L(K+sJ,K)^T
// for 1 <= sJ <= sI <= m, one tile per wavefront on the matrix cores, spread
// over workgroups; workgroup 0 also owns pair (1,1), whose target is the next
// diagonal tile, and factors that tile (and inverts it) right after its update.
// grid (n_wg, n_mat), 256 threads.
__global__ __launch_bounds__(256) void k_chol_update(const MatDesc* __restrict__ mats, int K,
                                                     double* __restrict__ fac,
                                                     int32_t* __restrict__ status) {
  const MatDesc v = mats[blockIdx.y];
  if (K >= v.NT - 1) return;
  const int m = (K < 0) ? 0 : min(v.BT - 1, v.NT - 1 - K);
  const int npairs = m * (m + 1) / 2;
  const bool owner = blockIdx.x == 0;
  if (!owner && (int)blockIdx.x * 4 >= npairs) return;
  double* L = fac + v.off;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int p = blockIdx.x * 4 + wave;
  if (p < npairs) {
    int sI = 1;
    while ((sI * (sI + 1)) / 2 <= p) ++sI;
    int sJ = p - (sI - 1) * sI / 2 + 1;
    const double* Ta = L + ((int64_t)(K + sI) * v.BT + sI) * MSG_TILE2;
    const double* Tb = L + ((int64_t)(K + sJ) * v.BT + sJ) * MSG_TILE2;
    double* Tc = L + ((int64_t)(K + sI) * v.BT + (sI - sJ)) * MSG_TILE2;
    dbl4 acc[2][2];
    tile_load_acc(Tc, acc, lane);
    tile_mfma_abt(Ta, Tb, -1.0, acc, lane);
    tile_store_acc(Tc, acc, lane);
  }
  if (owner) {
    // the next diagonal tile was updated above by wavefront 0 (pair 0); the
    // same wavefront factors it
    if (wave == 0) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wavefront's tile stores are complete
      double* T = L + (int64_t)(K + 1) * v.BT * MSG_TILE2;
      const int bad = diag_tile_factor(T, fac + v.ioff + (int64_t)(K + 1) * MSG_TILE2);
      if (lane == 0 && bad) atomicOr(&status[v.status_idx], 4);
    }
  }
}

// Panel of column K: L(K+s, K) = A(K+s, K) L_KK^{-T} = A Linv_KK^T, one tile per
// wavefront on the matrix cores.  grid (ceil(max(BT-1)/4), n_mat).
__global__ __launch_bounds__(256) void k_chol_panel(const MatDesc* __restrict__ mats, int K,
                                                    double* __restrict__ fac) {
  const MatDesc v = mats[blockIdx.y];
  if (K >= v.NT) return;
  const int m = min(v.BT - 1, v.NT - 1 - K);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + wave + 1;
  if (s > m) return;
  double* T = fac + v.off + ((int64_t)(K + s) * v.BT + s) * MSG_TILE2;
  const double* Ti = fac + v.ioff + (int64_t)K * MSG_TILE2;
  dbl4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
  tile_mfma_abt(T, Ti, 1.0, acc, lane);
  tile_store_acc(T, acc, lane);
}

// Left-looking tile Cholesky of banded matrices, one launch per step J
// (J = -1 .. NT-2).  Invariant before step J: every tile of the columns
// K <= J-1 is final; the diagonal tile J is factored and its inverse stored;
// the tiles (I, J), I > J, hold A minus the products that earlier steps took.
// Step J completes column J (L(I,J) = X L_JJ^{-T} from the remaining products
// of row I) and factors the diagonal tile J+1 (its chain job), so the
// diagonal factor of a column is computed by the launch before the one that
// needs it, next to the bulk of the tile products; the products that read
// only final tiles are gathered into panels (k_chol_step below).  A wavefront
// owns whole 32x32 target tiles (each loaded operand feeds two or four
// MFMAs) on the FP64 matrix cores; no job shares data with another wavefront.
#define CH_LD 34   // LDS row stride (doubles) of staged tiles

// A 32x32 row-major tile in the MFMA operand layout: lane (i = l&15, k = l>>4)
// holds, for row block b (rows 16b + i) and step 2m + e, inner index
// 8m + 2k + e (16 contiguous bytes per load).  The same registers serve as
// the A operand of A B^T and as the B operand (rows of B).
struct TileOps {
  double2 v[2][4];
};

__device__ inline void tops_load(const double* __restrict__ T, int lane, TileOps& o) {
  const int i = lane & 15, k = lane >> 4;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const double2* p = reinterpret_cast<const double2*>(T + (16 * b + i) * 32 + 2 * k);
#pragma unroll
    for (int m = 0; m < 4; ++m) o.v[b][m] = p[4 * m];
  }
}

// acc[bi][bj] += A[bi] B[bj]^T; lower = blocks with bi >= bj only
template <bool LOWER = false>
__device__ inline void tops_abt(const TileOps& A, const TileOps& B, dbl4 acc[2][2]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        if (LOWER && bi < bj) continue;
        acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v[bi][m].x, B.v[bj][m].x, acc[bi][bj], 0, 0, 0);
      }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        if (LOWER && bi < bj) continue;
        acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v[bi][m].y, B.v[bj][m].y, acc[bi][bj], 0, 0, 0);
      }
  }
}

// Accumulator layout of a 16x16 block (item v of lane l = row (l>>4) + 4v,
// column l&15): block (bi, bj) of a tile with leading dimension ld, or of its
// transpose (quadT_*: item v of lane l = C[16bj + (l&15)][16bi + (l>>4) + 4v]).
__device__ inline dbl4 quad_get(const double* __restrict__ C, int ld, int bi, int bj, int lane) {
  const double* p = C + (16 * bi + (lane >> 4)) * ld + 16 * bj + (lane & 15);
  return dbl4{p[0], p[4 * ld], p[8 * ld], p[12 * ld]};
}

__device__ inline void quad_put(double* __restrict__ C, int ld, int bi, int bj, int lane, dbl4 x) {
  double* p = C + (16 * bi + (lane >> 4)) * ld + 16 * bj + (lane & 15);
  p[0] = x[0];
  p[4 * ld] = x[1];
  p[8 * ld] = x[2];
  p[12 * ld] = x[3];
}

__device__ inline dbl4 quadT_get(const double* __restrict__ C, int bi, int bj, int lane) {
  const double* p = C + (16 * bj + (lane & 15)) * 32 + 16 * bi + (lane >> 4);
  return dbl4{p[0], p[4], p[8], p[12]};
}

__device__ inline void quadT_put(double* __restrict__ C, int bi, int bj, int lane, dbl4 x) {
  double* p = C + (16 * bj + (lane & 15)) * 32 + 16 * bi + (lane >> 4);
  p[0] = x[0];
  p[4] = x[1];
  p[8] = x[2];
  p[12] = x[3];
}

// L(I,J) = X L_JJ^{-T} from X^T in accumulator layout (XT[bk][bb] = block of
// X^T): L^T = L_JJ^{-1} X^T on the matrix cores, the accumulators of X^T used
// directly as B operands (item v of block bk is inner index 16bk + (l>>4) + 4v).
// Stores L(I,J) (row-major) and returns L^T in accumulator layout.
__device__ inline void trsm_from_xt(const double* __restrict__ Linv, const dbl4 XT[2][2], double* __restrict__ out,
                                    dbl4 LT[2][2], int lane) {
  const int i = lane & 15, k = lane >> 4;
  const dbl4 zero = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ba = 0; ba < 2; ++ba)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) LT[ba][bb] = zero;
#pragma unroll
  for (int bk = 0; bk < 2; ++bk)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int ba = 0; ba < 2; ++ba) {
        const double a = Linv[(16 * ba + i) * 32 + 16 * bk + k + 4 * v];
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
          LT[ba][bb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, XT[bk][bb][v], LT[ba][bb], 0, 0, 0);
      }
#pragma unroll
  for (int ba = 0; ba < 2; ++ba)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) quadT_put(out, ba, bb, lane, LT[ba][bb]);
}

// One wavefront: C = L L^T for the 32x32 SPD tile C in LDS (stride CH_LD,
// lower triangle read).  Writes L to Lg (row-major, zero above the diagonal)
// and L^{-1} to Ig (row-major).  Lane (i, h) = (l&31, l>>5) holds columns
// 16h .. 16h+15 of row i.  Right-looking: at step j the lanes holding column
// j scale it, publish it in LDS (vec) and every lane updates its trailing
// entries with its own row's multiplier and the broadcast column.  The
// inverse is then formed by forward substitution, lane (c, h) holding rows
// 16h .. 16h+15 of column c, the columns of L read from Lt (LDS, L^T).
// dinv (32), vec (32), Lt (32 x CH_LD) are LDS scratch.  Returns 1 if a
// pivot was not positive (it is replaced by 1).
__device__ int factor_tile32(const double* __restrict__ C, double* __restrict__ Lt, double* __restrict__ dinv,
                             double* __restrict__ vec, double* __restrict__ Lg, double* __restrict__ Ig) {
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
  double a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) a[c] = (16 * h + c <= i) ? C[i * CH_LD + 16 * h + c] : 0.0;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const int jh = j >> 4, jc = j & 15;
    asm volatile("" ::: "memory");   // keep each step's LDS reads in their step (register pressure)
    double d = lane_value(a[jc], j + 32 * jh);
    if (!(d > 0.0)) {
      d = 1.0;
      bad = 1;
    }
    const double sd = sqrt(d), inv = 1.0 / sd;
    if (h == jh) {
      const double l = (i == j) ? sd : (i > j ? a[jc] * inv : 0.0);
      a[jc] = l;
      vec[i] = l;
    }
    if (lane == 0) dinv[j] = inv;
    // the other half's lanes read what these lanes wrote: no load may move above
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    const double li = vec[i];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const double m = vec[16 * h + c];
      // column j itself is final; earlier columns see m = 0
      if (c != jc || h != jh) a[c] -= li * m;
    }
    // keep the update in its step (deferring it keeps every multiplier live)
#pragma unroll
    for (int c = 0; c < 16; ++c) asm volatile("" : "+v"(a[c]));
  }
  // rows of L to global memory, columns to Lt
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int q = 16 * h + c;
    const double w = (q <= i) ? a[c] : 0.0;
    Lg[i * 32 + q] = w;
    Lt[q * CH_LD + i] = w;
  }
  double x[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = (16 * h + r == i) ? 1.0 : 0.0;
#pragma unroll
  for (int jj = 0; jj < 32; ++jj) {
    const int jh = jj >> 4, jr = jj & 15;
    asm volatile("" ::: "memory");
    if (h == jh) {
      x[jr] *= dinv[jj];
      vec[i] = x[jr];
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    const double xj = vec[i];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const double m = Lt[jj * CH_LD + 16 * h + r];   // L(16h+r, jj): zero above the diagonal
      if (r != jr || h != jh) x[r] -= m * xj;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) asm volatile("" : "+v"(x[r]));
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) Ig[(16 * h + r) * 32 + i] = x[r];
  return bad;
}

// One step J of the left-looking tile Cholesky, with the products that read
// only final tiles gathered into panels of P columns.  Step J completes
// column J (L(I,J) for the band rows I > J) and factors the diagonal tile
// J+1.  At a panel step (J + 1 divisible by P, J = -1 included) the products
// L(I,K) L(c,K)^T with K <= J-1 are subtracted from the next P columns
// c = J+1 .. J+P in one pass over the band window (each tile L(I,K) read
// once for P columns): for the diagonal tiles J+2 .. J+P+1 and for the rows'
// tiles (I, c), c < I.  The products with K between the last panel step and
// J-1 (at most P) are taken where column J or the diagonal tile J+1 is
// formed.  Jobs (one wavefront each): 0, the chain of the step (X^T of
// L(J+1,J), its triangular solve, the diagonal tile J+1's remaining products
// and its one-wavefront Cholesky and inverse); 1 .. P, the panel products of
// the diagonal tiles (then empty jobs up to the next multiple of four, so
// that a workgroup holds whole rows); then per band row I = J + s (s >= 2)
// and pair g of panel columns, the triangular solve for L(I,J) (g = 0) and
// the panel products of columns J+1+2g, J+2+2g.
// grid chol_grid(P, n_mat, max BT), 256 threads: workgroup y of a matrix
// holds jobs 4y .. 4y+3 (one per wavefront); the order in which the
// (matrix, y) workgroups are dispatched is set by `group` (below).

// One job of step J on matrix *mat, run by one wavefront (job 0 uses the LDS
// scratch X, Y (32 x CH_LD each), dinv and vec).  The descriptor is read here,
// so that a loop over jobs keeps nothing of it live between them.
template <int P>
__device__ __forceinline__ void chol_job(const MatDesc* __restrict__ mat, int J, int job, double* __restrict__ fac,
                                         int32_t* __restrict__ status, double* __restrict__ X,
                                         double* __restrict__ Y, double* __restrict__ dinv,
                                         double* __restrict__ vec) {
  static_assert(P >= 2 && P % 2 == 0, "panel columns come in pairs");
  constexpr int G = P / 2;
  const MatDesc v = *mat;
  const int lane = threadIdx.x & 63;
  const int BT = v.BT, NT = v.NT;
  // a chain of a split matrix factors its first NF columns only: its
  // separator rows get L(I, J) for J < NF, no tile of a column >= NF changes
  const int NF = v.NTf > 0 ? v.NTf : NT;
  if (J >= NF) return;
  double* L = fac + v.off;
  auto tile = [&](int I, int K) { return L + ((int64_t)I * BT + (I - K)) * MSG_TILE2; };
  const double* LinvJ = fac + v.ioff + (int64_t)(J < 0 ? 0 : J) * MSG_TILE2;
  const dbl4 zero = {0.0, 0.0, 0.0, 0.0};
  const bool panel = ((J + 1) % P) == 0;
  // the last panel step before J (its products reached column J)
  const int Jb = J >= 0 ? (J / P) * P - 1 : -1;
  dbl4 acc[2][2], xt[2][2], lt[2][2];
  auto zero4 = [&](dbl4 (&a)[2][2]) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) a[bi][bj] = zero;
  };
  // X^T = A(I,J)^T - sum_{K = max(Jb, kb) .. J-1} L(J,K) L(I,K)^T, then
  // L(I,J) = X L_JJ^{-T} stored, L(I,J)^T returned in lt
  auto column_tile = [&](int I, int kb) {
    zero4(xt);
    for (int K = max(Jb, kb); K <= J - 1; ++K) {
      TileOps a, b;
      tops_load(tile(J, K), lane, a);
      tops_load(tile(I, K), lane, b);
      tops_abt(a, b, xt);
    }
    double* T = tile(I, J);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) xt[bi][bj] = quadT_get(T, bi, bj, lane) - xt[bi][bj];
    trsm_from_xt(LinvJ, xt, T, lt, lane);
  };

  if (job == 0) {
    const int R = J + 1;
    if (R > NT - 1) return;
    const bool diag = R < NF;                // the diagonal tile R is factored here
    const int kbR = max(0, R - (BT - 1));
    const bool has_x = J >= 0 && BT >= 2;   // tile (R, J) exists
    if (has_x) column_tile(R, kbR);
    if (!diag) return;
    zero4(acc);
    if (has_x) {
      // + L(R,J) L(R,J)^T: the accumulators of L^T serve as both operands
#pragma unroll
      for (int bk = 0; bk < 2; ++bk)
#pragma unroll
        for (int w = 0; w < 4; ++w)
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
              acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(lt[bk][bi][w], lt[bk][bj][w], acc[bi][bj], 0, 0, 0);
    }
    // the diagonal tile R received the products K <= Jb - 1 at step Jb
    for (int K = max(kbR, Jb); K <= J - 1; ++K) {
      TileOps a;
      tops_load(tile(R, K), lane, a);
      tops_abt<true>(a, a, acc);
    }
    double* T = tile(R, R);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        if (bi >= bj) quad_put(X, CH_LD, bi, bj, lane, quad_get(T, 32, bi, bj, lane) - acc[bi][bj]);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // the tile is read by other lanes below
    const int bad = factor_tile32(X, Y, dinv, vec, T, fac + v.ioff + (int64_t)R * MSG_TILE2);
    if (lane == 0 && bad) atomicOr(&status[v.status_idx], 4);
    return;
  }
  if (job <= P) {
    // panel products of the diagonal tiles J+2 .. J+P+1
    const int R = J + 1 + job;
    if (!panel || R > NT - 1 || R >= NF) return;
    const int k0 = max(0, R - (BT - 1)), k1 = J - 1;
    if (k0 > k1) return;
    zero4(acc);
    for (int K = k1; K >= k0; --K) {
      TileOps a;
      tops_load(tile(R, K), lane, a);
      tops_abt<true>(a, a, acc);   // the upper block of a diagonal tile is not read
    }
    double* T = tile(R, R);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        if (bi >= bj) quad_put(T, 32, bi, bj, lane, quad_get(T, 32, bi, bj, lane) - acc[bi][bj]);
    return;
  }
  if (job < CHOL_ROW0(P)) return;   // padding of the diagonal jobs
  const int r = job - CHOL_ROW0(P);
  const int s = 2 + r / G, g = r % G, I = J + s;
  if (J < 0 || s > BT - 1 || I > NT - 1) return;
  const int kb = max(0, I - (BT - 1));   // K range of row I's band tiles: [kb, I]
  if (g == 0) column_tile(I, kb);
  if (!panel) return;
  // panel products of columns c0 = J+1+2g and c0+1 (those before row I)
  const int c0 = J + 1 + 2 * g;
  const int k1 = J - 1;
  if (kb > k1 || c0 >= NF || c0 >= I) return;
  const bool two = c0 + 1 < NF && c0 + 1 < I;
  dbl4 acc2[2][2];
  zero4(acc);
  zero4(acc2);
  if (two) {
    for (int K = k1; K >= kb; --K) {
      TileOps a, b, c;
      tops_load(tile(I, K), lane, a);
      tops_load(tile(c0, K), lane, b);
      tops_load(tile(c0 + 1, K), lane, c);
      tops_abt(a, b, acc);
      tops_abt(a, c, acc2);
    }
    double* T2 = tile(I, c0 + 1);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) quad_put(T2, 32, bi, bj, lane, quad_get(T2, 32, bi, bj, lane) - acc2[bi][bj]);
  } else {
    for (int K = k1; K >= kb; --K) {
      TileOps a, b;
      tops_load(tile(I, K), lane, a);
      tops_load(tile(c0, K), lane, b);
      tops_abt(a, b, acc);
    }
  }
  double* T1 = tile(I, c0);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) quad_put(T1, 32, bi, bj, lane, quad_get(T1, 32, bi, bj, lane) - acc[bi][bj]);
}

template <int P>
__global__ __launch_bounds__(256, 3) void k_chol_step(const MatDesc* __restrict__ mats, int nmat, int max_bt, int group, int J,
                                                      double* __restrict__ fac, int32_t* __restrict__ status) {
  __shared__ __align__(16) double X[32 * CH_LD];
  __shared__ __align__(16) double Y[32 * CH_LD];
  __shared__ double dinv[32], vec[32];
  // dispatch order (block id): the diagonal workgroups of every matrix first
  // (each step's chain starts at once), then the row workgroups, row group
  // by row group within groups of `group` matrices (a multiple of 8 that
  // divides the matrix count padded to a multiple of 8, so that the grid
  // covers every (matrix, y); the padded count: the longest rows of every
  // matrix first; 8: matrix by matrix, so that a matrix's rows read the
  // tiles they share while they are in L2).
  // Matrix m always runs on XCD m mod 8 (block id mod 8).
  const int nyb = (chol_jobs(P, max_bt) + 3) / 4, ndb = CHOL_ROW0(P) / 4, nrb = nyb - ndb;
  const int nm8 = (nmat + 7) / 8 * 8, L8 = (int)blockIdx.x;
  int mat, yb;
  if (L8 < ndb * nm8) {
    yb = L8 / nm8;
    mat = L8 - yb * nm8;
  } else {
    const int R = L8 - ndb * nm8, grp = R / (group * nrb), r8 = R - grp * group * nrb;
    mat = grp * group + r8 % group;
    yb = ndb + r8 / group;
  }
  if (mat >= nmat) return;
  chol_job<P>(mats + mat, J, yb * 4 + (threadIdx.x >> 6), fac, status, X, Y, dinv, vec);
}
template __global__ void k_chol_step<4>(const MatDesc*, int, int, int, int, double*, int32_t*);

// The steps J = -1 .. last_J of one matrix per workgroup of 8 wavefronts: the
// jobs of k_chol_step, taken by the wavefronts in job order from a counter in
// LDS, with a workgroup barrier between steps in place of a launch per step
// (the step's global writes are visible to the whole workgroup after it).
// Matrices proceed independently, each on one CU, so one matrix's chain
// overlaps the products of others and a matrix's tiles are read on one CU.
// Pays when the matrices fill the chip about once and their bands are narrow
// (few jobs per step).  grid (n_mat), 512 threads.
template <int P>
__global__ __launch_bounds__(512) void k_chol_matrix(const MatDesc* __restrict__ mats, int last_J,
                                                     double* __restrict__ fac, int32_t* __restrict__ status) {
  __shared__ __align__(16) double X[32 * CH_LD];
  __shared__ __align__(16) double Y[32 * CH_LD];
  __shared__ double dinv[32], vec[32];
  __shared__ int next[2];   // job counters of even and odd steps
  constexpr int W = 8;      // wavefronts
  const MatDesc* mat = mats + blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int NF = mat->NTf > 0 ? mat->NTf : mat->NT;
  const int lastJ = min(last_J, NF - 1);
  const int njobs = chol_jobs(P, mat->BT);
  if (threadIdx.x == 0) next[0] = W;
  for (int J = -1; J <= lastJ; ++J) {
    __syncthreads();
    // every wavefront has left step J-1, whose counter is readied here for
    // step J+1 (published by the next barrier); wavefront w starts with job w
    // (job 0, the chain, on wavefront 0: the only user of X, Y, dinv, vec)
    if (threadIdx.x == 0) next[(J + 2) & 1] = W;
    int job = __builtin_amdgcn_readfirstlane(wave);
    while (job < njobs) {
      chol_job<P>(mat, J, job, fac, status, X, Y, dinv, vec);
      int nj = 0;
      if (lane == 0) nj = atomicAdd(&next[(J + 1) & 1], 1);
      job = __builtin_amdgcn_readfirstlane(nj);
    }
  }
}
template __global__ void k_chol_matrix<4>(const MatDesc*, int, double*, int32_t*);

// The separator's Schur complement of a split matrix, once both chains are
// factored on their own columns:
//   S(I,J) -= sum_{c = 0,1} sum_K Lc(NFc + I, K) Lc(NFc + J, K)^T,  I >= J,
// K over chain c's columns in band of row NFc + I (the chain's separator
// rows hold L_sc = A_sc L_cc^{-T}).  S then holds A_ss - sum_c L_sc L_sc^T
// and is factored as a dense band.  One target tile per wavefront, ntg
// workgroups of four per separator.  The workgroups of separator n run one
// after another on XCD n mod 8 (block id mod 8), so the separator rows that
// all its target tiles read are fetched from HBM about once;
// grid 8 * ntg * ceil(n_sep / 8), 256 threads.
__global__ __launch_bounds__(256) void k_sep_syrk(const SepDesc* __restrict__ seps, int n_sep, int ntg,
                                                  double* __restrict__ fac) {
  const int L8 = (int)blockIdx.x, sep = (L8 / (8 * ntg)) * 8 + (L8 & 7), tg = (L8 >> 3) % ntg;
  if (sep >= n_sep) return;
  const SepDesc d = seps[sep];
  const int lane = threadIdx.x & 63;
  const int t = tg * 4 + (threadIdx.x >> 6);
  const int NTs = d.NTs;
  if (t >= NTs * (NTs + 1) / 2) return;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (I > 0 && I * (I + 1) / 2 > t) --I;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  const int J = t - I * (I + 1) / 2;
  const dbl4 zero = {0.0, 0.0, 0.0, 0.0};
  dbl4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = zero;
  for (int c = 0; c < 2; ++c) {
    const int NF = c ? d.NTf1 : d.NTf0;
    const double* L = fac + (c ? d.off1 : d.off0);
    auto tile = [&](int R, int K) { return L + ((int64_t)R * d.BT + (R - K)) * MSG_TILE2; };
    for (int K = max(0, NF + I - (d.BT - 1)); K < NF; ++K) {
      TileOps a, b;
      tops_load(tile(NF + I, K), lane, a);
      if (I == J) {
        tops_abt<true>(a, a, acc);
      } else {
        tops_load(tile(NF + J, K), lane, b);
        tops_abt(a, b, acc);
      }
    }
  }
  double* T = fac + d.offS + ((int64_t)I * NTs + (I - J)) * MSG_TILE2;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
      if (I != J || bi >= bj) quad_put(T, 32, bi, bj, lane, quad_get(T, 32, bi, bj, lane) - acc[bi][bj]);
}

// After the factorisation A = L L^T: rewrite the factor in block unit-lower
// form A = Lu D Lu^T with Lu(I,J) = L(I,J) L_JJ^{-1} (off-diagonal tiles, in
// place) and D^{-1}_II = L_II^{-T} L_II^{-1} stored in the diagonal tile slot,
// so that the block triangular sweeps need no diagonal solve.
// grid (ceil(max NT*BT / 4), n_mat), one tile per wavefront.
__global__ __launch_bounds__(256) void k_chol_unit(const MatDesc* __restrict__ mats,
                                                   double* __restrict__ fac) {
  const MatDesc v = mats[blockIdx.y];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + wave;
  if (t >= (int64_t)v.NT * v.BT) return;
  const int I = (int)(t / v.BT), s = (int)(t % v.BT);
  if (s > I) return;
  if (v.NTf > 0 && I - s >= v.NTf) return;   // a chain's separator block stays zero
  double* T = fac + v.off + ((int64_t)I * v.BT + s) * MSG_TILE2;
  const double* Ti = fac + v.ioff + (int64_t)(I - s) * MSG_TILE2;
  dbl4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
  if (s == 0) tile_mfma_atb(Ti, Ti, acc, lane);
  else tile_mfma_ab(T, Ti, acc, lane);
  tile_store_acc(T, acc, lane);
}

// Copies of the unit-lower band in the order the block solve reads it.  Solve
// thread t (tile s = 1 + 32p + t/16 of set p, row quad rq = (t/2)%8, half
// h = t%2) of tile row I holds 64 factor values as 32 double2 j:
//   forward  (tile (I, I-s)):     j = 8i + q2 -> Lu[4rq+i][16h+2q2 .. +1]
//   backward (tile (I+s, I)^T):   j = 2q + e  -> Lu[16h+q][4rq+2e .. +1]
// stored at (((I*nsets + p)*32 + j) * nthr + t); tiles outside the matrix or
// the band are zero.  One workgroup per (tile slot s, tile row I, box): it
// stages the forward source tile (I, s) and the backward source tile
// (I+s, s) in LDS with coalesced loads and writes the 16 threads' pieces of
// each, 256 contiguous bytes per j.  A chain of a split matrix has no tiles
// in its separator columns.  grid (32*max nsets, max NT, 3 n_box): z = 3 box + part.
__global__ __launch_bounds__(256) void k_band_relayout(const BoxMeta* __restrict__ meta, int kind,
                                                       double* __restrict__ fac) {
  __shared__ double Tf[MSG_TILE2], Tb[MSG_TILE2];
  const BoxMeta& bm = meta[blockIdx.z / 3];
  const int part = blockIdx.z % 3;
  if (part > 0 && !bm.nd[kind]) return;
  BandView v = band_view(bm, kind, part);
  const int nthr = solve_nthr(v.BT), nsets = solve_sets(v.BT);
  const int s = 1 + blockIdx.x, I = blockIdx.y;
  if (I >= v.NT || s > SOLVE_TILES * nsets || (nsets == 1 && s > v.BT - 1)) return;
  const int p = (s - 1) / SOLVE_TILES, tbase = 16 * ((s - 1) % SOLVE_TILES);
  const double* L = fac + v.off;
  const bool fok = s < v.BT && s <= I && I - s < v.NTf, bok = s < v.BT && I + s < v.NT && I < v.NTf;
  const int u = threadIdx.x;
  {
    const double2* src = (const double2*)(L + ((int64_t)I * v.BT + (fok ? s : 0)) * MSG_TILE2);
    const double2* srb = (const double2*)(L + ((int64_t)(bok ? I + s : I) * v.BT + (bok ? s : 0)) * MSG_TILE2);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const double2 a = fok ? src[u + 256 * r] : make_double2(0.0, 0.0);
      const double2 b = bok ? srb[u + 256 * r] : make_double2(0.0, 0.0);
      Tf[2 * (u + 256 * r)] = a.x;
      Tf[2 * (u + 256 * r) + 1] = a.y;
      Tb[2 * (u + 256 * r)] = b.x;
      Tb[2 * (u + 256 * r) + 1] = b.y;
    }
  }
  __syncthreads();
  double2* fw = (double2*)(fac + v.fw);
  double2* bw = (double2*)(fac + v.bw);
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int q = u + 256 * r;                 // piece: j = q / 16, thread slot tbase + q % 16
    const int j = q >> 4, tl = q & 15;
    const int rq = (tl >> 1) & 7, h = tl & 1;
    const int64_t e = ((int64_t)(I * nsets + p) * 32 + j) * nthr + tbase + tl;
    const int i = j >> 3, q2 = j & 7;
    fw[e] = make_double2(Tf[(4 * rq + i) * 32 + 16 * h + 2 * q2], Tf[(4 * rq + i) * 32 + 16 * h + 2 * q2 + 1]);
    const int qq = j >> 1, c = j & 1;
    bw[e] = make_double2(Tb[(16 * h + qq) * 32 + 4 * rq + 2 * c], Tb[(16 * h + qq) * 32 + 4 * rq + 2 * c + 1]);
  }
}




// Entry (row, inner index c0 of e = 0; e = 1 is c0 + 4) of a 32x32 tile held
// by lane l in double2 piece pp of the matrix-core solve copies.  wide = 0:
// the A operand of v_mfma_f64_4x4x4f64 (k_band_solve4), lane l = 16 kk + 4 o
// + i -> row 16 (pp >> 2) + 4 o + i, c0 = 8 (pp & 3) + kk; wide = 1: the A
// operand of v_mfma_f64_16x16x4f64 (k_band_solve16), lane l = 16 k + i ->
// row 16 (pp >> 2) + i, c0 = 8 (pp & 3) + k.
__device__ inline void solve_piece_entry(int wide, int pp, int l, int* row, int* c0) {
  if (wide) {
    *row = 16 * (pp >> 2) + (l & 15);
    *c0 = 8 * (pp & 3) + (l >> 4);
  } else {
    *row = 16 * (pp >> 2) + 4 * ((l >> 2) & 3) + (l & 3);
    *c0 = 8 * (pp & 3) + (l >> 4);
  }
}

// Copies of the unit-lower band in the operand order of the matrix-core block
// solves (k_band_solve4; bands of at most 65 tiles).  Tile row I has 1 + 8
// nslot slots of 8 KB: slot 0 of the forward copy is D^{-1}_I, slot s >= 1 the
// tile (I, I-s) (forward) or (I+s, I)^T (backward); tiles outside the matrix
// or the band are zero.  Inside a slot, double2 pp (0..7) of lane l = 16 kk +
// 4 o + i holds A[16 rh + 4 o + i][4 ss + kk] for rh = pp >> 2 and ss = 2 (pp
// & 3) + e, e = 0, 1 (the A operand of v_mfma_f64_4x4x4f64 for 4x4 blocks o),
// at ((I S + slot) 8 + pp) 64 + l, S = solve4_slots(BT).  One workgroup per
// (slot, tile row, box part) stages the source tiles in LDS and writes 1 KB
// per pp.  grid (1 + 8 max nslot, max NT, 3 n_box): z = 3 box + part.
__global__ __launch_bounds__(256) void k_band_relayout4(const BoxMeta* __restrict__ meta, int kind,
                                                        double* __restrict__ fac, int wide) {
  __shared__ double Tf[MSG_TILE2], Tb[MSG_TILE2];
  const BoxMeta& bm = meta[blockIdx.z / 3];
  const int part = blockIdx.z % 3;
  if (part > 0 && !bm.nd[kind]) return;
  BandView v = band_view(bm, kind, part);
  const int S = solve4_slots(v.BT);
  const int slot = blockIdx.x, I = blockIdx.y;
  if (I >= v.NT || slot >= S) return;
  const double* L = fac + v.off;
  // forward source: D^{-1}_I (the diagonal slot after the unit-lower rewrite) or tile (I, I-s)
  const bool fok = slot == 0 ? I < v.NTf : (slot < v.BT && slot <= I && I - slot < v.NTf);
  const bool bok = slot >= 1 && slot < v.BT && I + slot < v.NT && I < v.NTf;
  const int u = threadIdx.x;
  {
    const double2* src = (const double2*)(L + ((int64_t)I * v.BT + (fok ? slot : 0)) * MSG_TILE2);
    const double2* srb = (const double2*)(L + ((int64_t)(bok ? I + slot : I) * v.BT + (bok ? slot : 0)) * MSG_TILE2);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const double2 a = fok ? src[u + 256 * r] : make_double2(0.0, 0.0);
      const double2 b = bok ? srb[u + 256 * r] : make_double2(0.0, 0.0);
      Tf[2 * (u + 256 * r)] = a.x;
      Tf[2 * (u + 256 * r) + 1] = a.y;
      Tb[2 * (u + 256 * r)] = b.x;
      Tb[2 * (u + 256 * r) + 1] = b.y;
    }
  }
  __syncthreads();
  double2* fw = (double2*)(fac + v.fw) + ((int64_t)I * S + slot) * 8 * 64;
  double2* bw = (double2*)(fac + v.bw) + ((int64_t)I * S + slot) * 8 * 64;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int q = u + 256 * r;                 // (pp, lane)
    const int pp = q >> 6, l = q & 63;
    int row, c0;   // entry of e = 0 (e = 1 adds 4 to the inner index)
    solve_piece_entry(wide, pp, l, &row, &c0);
    fw[q] = make_double2(Tf[row * 32 + c0], Tf[row * 32 + c0 + 4]);
    bw[q] = make_double2(Tb[c0 * 32 + row], Tb[(c0 + 4) * 32 + row]);
  }
}

// The block unit-lower rewrite (as k_chol_unit) fused with the copies of
// k_band_relayout4, for batches whose bands all fit the matrix-core solve:
// each tile Lu(I, I-s) = L(I, I-s) L_{I-s}^{-1}, and D^{-1}_I = L_I^{-T} L_I^{-1},
// is formed once and written straight into the forward copy (row I, slot s)
// and the backward copy (row I-s, slot s, transposed); D^{-1}_I also replaces
// the band's diagonal tile, while the off-diagonal tiles of the band keep L
// (only the copies are read afterwards).  The band is read once and the
// copies written once, instead of reading the band, rewriting it and reading
// it again.  Slots outside the matrix or the band are zero: a forward slot
// with s > I or s >= BT, a backward slot with s = 0, s >= BT or I + s >= NT.
// A chain of a split matrix has no D^{-1} on its separator rows and no
// tiles in its separator columns.  One wavefront per slot s = 4 blockIdx.x +
// wave of tile row I = blockIdx.y; grid (ceil(S / 4), max NT, 3 n_box): z = 3
// box + part, 256 threads.
__global__ __launch_bounds__(256) void k_band_unit_relayout4(const BoxMeta* __restrict__ meta, int kind,
                                                             double* __restrict__ fac, int wide) {
  __shared__ double Tl[4][MSG_TILE2];
  const BoxMeta& bm = meta[blockIdx.z / 3];
  const int part = blockIdx.z % 3;
  if (part > 0 && !bm.nd[kind]) return;
  BandView v = band_view(bm, kind, part);
  const int S = solve4_slots(v.BT);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = 4 * blockIdx.x + wave, I = blockIdx.y;
  if (I >= v.NT || s >= S) return;
  double* L = fac + v.off;
  const double* Linv = fac + v.ioff;
  double2* fw = (double2*)(fac + v.fw) + ((int64_t)I * S + s) * 8 * 64;

  if (s == 0 ? I < v.NTf : (s < v.BT && s <= I && I - s < v.NTf)) {
    double* T = Tl[wave];
    dbl4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
    if (s == 0) tile_mfma_atb(Linv + (int64_t)I * MSG_TILE2, Linv + (int64_t)I * MSG_TILE2, acc, lane);
    else tile_mfma_ab(L + ((int64_t)I * v.BT + s) * MSG_TILE2, Linv + (int64_t)(I - s) * MSG_TILE2, acc, lane);
    tile_store_acc(T, acc, lane);
    if (s == 0) tile_store_acc(L + (int64_t)I * v.BT * MSG_TILE2, acc, lane);
    // other lanes' entries of T are read next
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    double2* bw = (double2*)(fac + v.bw) + ((int64_t)(I - s) * S + s) * 8 * 64;
#pragma unroll
    for (int pp = 0; pp < 8; ++pp) {
      // operand order of the lane (see k_band_relayout4): row and inner index of e = 0
      int row, c0;
      solve_piece_entry(wide, pp, lane, &row, &c0);
      fw[pp * 64 + lane] = make_double2(T[row * 32 + c0], T[row * 32 + c0 + 4]);
      if (s >= 1) bw[pp * 64 + lane] = make_double2(T[c0 * 32 + row], T[(c0 + 4) * 32 + row]);
    }
  } else {
#pragma unroll
    for (int pp = 0; pp < 8; ++pp) fw[pp * 64 + lane] = make_double2(0.0, 0.0);
  }
  if (s == 0 || s >= v.BT || I + s >= v.NT || I >= v.NTf) {
    double2* bz = (double2*)(fac + v.bw) + ((int64_t)I * S + s) * 8 * 64;
#pragma unroll
    for (int pp = 0; pp < 8; ++pp) bz[pp * 64 + lane] = make_double2(0.0, 0.0);
  }
}


// FP32 copies for the mixed path (same element offsets as the FP64 arrays):
// the two solve-ordered band copies and the D^{-1} diagonal tiles of every
// part of both box matrices (grid.y = box, grid.z = matrix kind), and the
// stencil (grid.z = 2).
__global__ void k_mixed_copies(const BoxMeta* __restrict__ meta, int zbase, const double* __restrict__ fac,
                               float* __restrict__ fac32, const double* __restrict__ stencil,
                               float* __restrict__ stencil32) {
  const BoxMeta& bm = meta[blockIdx.y];
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, st = (int64_t)gridDim.x * blockDim.x;
  const int z = zbase + blockIdx.z;   // 0: A11 factor data, 1: Ahat factor data, 2: stencil
  if (z == 2) {
    const int64_t o = bm.node_off * 243, n = (int64_t)bm.n_nodes * 243;
    for (int64_t e = t0; e < n; e += st) stencil32[o + e] = (float)stencil[o + e];
    return;
  }
  for (int part = 0; part < (bm.nd[z] ? 3 : 1); ++part) {
    BandView v = band_view(bm, z, part);
    const int64_t nb = solve_copy_doubles(v.NT, v.BT);
    for (int64_t e = t0; e < nb; e += st) {
      fac32[v.fw + e] = (float)fac[v.fw + e];
      fac32[v.bw + e] = (float)fac[v.bw + e];
    }
    const int64_t nd = (int64_t)v.NT * MSG_TILE2;
    for (int64_t e = t0; e < nd; e += st) {
      const int64_t o = v.off + (e >> 10) * v.BT * MSG_TILE2 + (e & 1023);
      fac32[o] = (float)fac[o];
    }
  }
}

}  // namespace msg
