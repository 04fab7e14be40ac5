// Banded SPD factorisations and block solves on the oversampled boxes.
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
#include "internal.hpp"

namespace msg {

struct BandView {
  int NT, BT, n;
  int64_t off, ioff;
  int sx, sy, sz;   // (sub-)box node dims of the ordering
  int ox, oy, oz;   // offset of the ordering's node (0,0,0) inside the box
};

__device__ inline BandView band_view(const BoxMeta& bm, int kind) {
  BandView v;
  if (kind == 0) {
    v.NT = bm.nt11; v.BT = bm.bt11; v.n = bm.n11; v.off = bm.f11_off; v.ioff = bm.f11i_off;
    v.sx = bm.sub_hi[0] - bm.sub_lo[0] + 1;
    v.sy = bm.sub_hi[1] - bm.sub_lo[1] + 1;
    v.sz = bm.sub_hi[2] - bm.sub_lo[2] + 1;
    v.ox = bm.sub_lo[0]; v.oy = bm.sub_lo[1]; v.oz = bm.sub_lo[2];
  } else {
    v.NT = bm.nth; v.BT = bm.bth; v.n = bm.nh; v.off = bm.fh_off; v.ioff = bm.fhi_off;
    v.sx = bm.mx; v.sy = bm.my; v.sz = bm.mz;
    v.ox = v.oy = v.oz = 0;
  }
  return v;
}

// band row -> box DoF (or -1 for padding rows)
__device__ inline int band_to_dof(const BandView& v, const BoxMeta& bm, int r) {
  if (r >= v.n) return -1;
  int node = r / 3, c = r - 3 * node;
  int i = node % v.sx, j = (node / v.sx) % v.sy, k = node / (v.sx * v.sy);
  int bn = (i + v.ox) + bm.mx * ((j + v.oy) + bm.my * (k + v.oz));
  return 3 * bn + c;
}

__device__ inline bool dof_active(int kind, uint8_t c) {
  return kind == 0 ? (c == 1) : (c == 1 || c == 2);
}

// One thread per tile entry; grid.x over NT*BT*1024 of the largest box, grid.y = box.
__global__ void k_band_build(const BoxMeta* __restrict__ meta, int kind,
                             const double* __restrict__ stencil, const uint8_t* __restrict__ cls,
                             const double* __restrict__ mu1, double shift, double* __restrict__ fac) {
  const BoxMeta& bm = meta[blockIdx.y];
  BandView v = band_view(bm, kind);
  int64_t total = (int64_t)v.NT * v.BT * MSG_TILE2;
  const double* st = stencil + bm.node_off * 243;
  const uint8_t* cl = cls + bm.dof_off;
  const double* m1 = mu1 + bm.dof_off;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int e = (int)(t & 1023);
    int64_t tile = t >> 10;
    int I = (int)(tile / v.BT), s = (int)(tile % v.BT);
    int r = e >> 5, c = e & 31;
    int row = I * MSG_TILE + r, col = (I - s) * MSG_TILE + c;
    double val = 0.0;
    if (col < 0 || col > row) {
      val = 0.0;
    } else if (row >= v.n) {
      val = (row == col) ? 1.0 : 0.0;
    } else {
      int dr = band_to_dof(v, bm, row), dc = band_to_dof(v, bm, col);
      bool ar = dof_active(kind, cl[dr]), ac = dof_active(kind, cl[dc]);
      if (!ar || !ac) {
        val = (row == col) ? 1.0 : 0.0;
      } else {
        int nr = dr / 3, nc = dc / 3;
        int ir = nr % bm.mx, jr = (nr / bm.mx) % bm.my, kr = nr / (bm.mx * bm.my);
        int ic = nc % bm.mx, jc = (nc / bm.mx) % bm.my, kc = nc / (bm.mx * bm.my);
        int dx = ic - ir, dy = jc - jr, dz = kc - kr;
        if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) {
          int nb = nb_index(dx, dy, dz);
          double a = st[(int64_t)(nb * 9 + 3 * (dr % 3) + (dc % 3)) * bm.n_nodes + nr];
          val = (kind == 1) ? a * (1.0 + shift * m1[dr] * m1[dc]) : a;
        }
      }
    }
    fac[(kind == 0 ? bm.f11_off : bm.fh_off) + t] = val;
  }
}

// Right-looking tile Cholesky, one workgroup (256 threads) per (box, kind).
// grid.x = box.  status[box] gets bit 2 set if a pivot is not positive.
__global__ __launch_bounds__(256) void k_band_potrf(const BoxMeta* __restrict__ meta, int kind,
                                                    double* __restrict__ fac,
                                                    int32_t* __restrict__ status) {
  __shared__ double D[32][33];
  __shared__ double Di[32][33];
  __shared__ double Pa[4][32][33];
  __shared__ double Pb[4][32][33];
  __shared__ int bad;
  const BoxMeta& bm = meta[blockIdx.x];
  BandView v = band_view(bm, kind);
  double* L = fac + v.off;
  double* Li = fac + v.ioff;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid == 0) bad = 0;
  for (int K = 0; K < v.NT; ++K) {
    double* TKK = L + (int64_t)K * v.BT * MSG_TILE2;
    for (int t = tid; t < 1024; t += 256) D[t >> 5][t & 31] = TKK[t];
    __syncthreads();
    // unblocked Cholesky of the diagonal tile
    for (int j = 0; j < 32; ++j) {
      if (tid >= j && tid < 32) {
        double d = D[j][j];
        if (!(d > 0.0)) {
          d = 1.0;
          bad = 1;
        }
        double sd = sqrt(d);
        if (tid == j) D[j][j] = sd;
        else D[tid][j] = D[tid][j] / sd;
      }
      __syncthreads();
      for (int t = tid; t < 1024; t += 256) {
        int i = t >> 5, c = t & 31;
        if (i > j && c > j && c <= i) D[i][c] -= D[i][j] * D[c][j];
      }
      __syncthreads();
    }
    // inverse of the lower-triangular diagonal tile, column by column
    if (tid < 32) {
      int c = tid;
      for (int i = 0; i < 32; ++i) {
        if (i < c) { Di[i][c] = 0.0; continue; }
        double s = (i == c) ? 1.0 : 0.0;
        for (int q = c; q < i; ++q) s -= D[i][q] * Di[q][c];
        Di[i][c] = s / D[i][i];
      }
    }
    __syncthreads();
    for (int t = tid; t < 1024; t += 256) {
      int i = t >> 5, c = t & 31;
      TKK[t] = (c <= i) ? D[i][c] : 0.0;
      Li[(int64_t)K * 1024 + t] = Di[i][c];
    }
    // panel: L(I,K) = A(I,K) * L_KK^{-T}, tile by tile through LDS:
    // x[r][c] = sum_{q<=c} a[r][q] Di[c][q]
    int m = min(v.BT - 1, v.NT - 1 - K);
    for (int s = 1; s <= m; ++s) {
      double* T = L + ((int64_t)(K + s) * v.BT + s) * MSG_TILE2;
      for (int t = tid; t < 1024; t += 256) Pa[0][t >> 5][t & 31] = T[t];
      __syncthreads();
      for (int t = tid; t < 1024; t += 256) {
        int r = t >> 5, c = t & 31;
        double x = 0.0;
        for (int q = 0; q <= c; ++q) x += Pa[0][r][q] * Di[c][q];
        T[t] = x;
      }
      __syncthreads();
    }
    // trailing update A(I,J) -= L(I,K) L(J,K)^T, K < J <= I < K+BT
    int npairs = m * (m + 1) / 2;
    int rounds = (npairs + 3) / 4;
    for (int rd = 0; rd < rounds; ++rd) {
      int p = rd * 4 + wave;
      int sI = 0, sJ = 0;
      bool act = p < npairs;
      if (act) {
        // invert p -> (sI, sJ) with 1 <= sJ <= sI <= m, p = (sI-1)sI/2 + (sJ-1)
        sI = 1;
        while ((sI * (sI + 1)) / 2 <= p) ++sI;
        sJ = p - (sI - 1) * sI / 2 + 1;
        const double* A1 = L + ((int64_t)(K + sI) * v.BT + sI) * MSG_TILE2;
        const double* B1 = L + ((int64_t)(K + sJ) * v.BT + sJ) * MSG_TILE2;
        for (int t = lane; t < 1024; t += 64) {
          Pa[wave][t >> 5][t & 31] = A1[t];
          Pb[wave][t >> 5][t & 31] = B1[t];
        }
      }
      __syncthreads();
      if (act) {
        int r0 = (lane >> 3) * 4, c0 = (lane & 7) * 4;
        double acc[4][4] = {};
        for (int q = 0; q < 32; ++q) {
          double av[4], bv[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) av[i] = Pa[wave][r0 + i][q];
#pragma unroll
          for (int j = 0; j < 4; ++j) bv[j] = Pb[wave][c0 + j][q];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
        }
        double* Tt = L + ((int64_t)(K + sI) * v.BT + (sI - sJ)) * MSG_TILE2;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) Tt[(r0 + i) * 32 + c0 + j] -= acc[i][j];
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (tid == 0 && bad) atomicOr(&status[blockIdx.x], 4);
}

// Block solve (L L^T) x = f for KC columns [c0, c0+KC) of a box block vector.
// Reads `in` (box layout [n_dof][ldk]) on the matrix's DoFs, writes `out` on
// the DoFs whose class bit is set in out_classes (bit c for class c); with
// zero_rest, every other DoF of the box gets 0 in these columns.  Scratch
// holds the forward result, NT*32*KC doubles per (box, chunk).
// grid.x = n_chunks * n_boxes (chunk fastest inside an XCD-friendly order),
// dynamic LDS = BT*32*KC doubles.
template <int KC>
__global__ __launch_bounds__(256) void k_band_solve(const BoxMeta* __restrict__ meta, int n_box,
                                                    int n_chunk, int kind,
                                                    const double* __restrict__ fac,
                                                    const uint8_t* __restrict__ cls,
                                                    const double* in, double* out, int ldk,
                                                    int out_classes, int zero_rest,
                                                    double* __restrict__ scratch,
                                                    int64_t scratch_stride,
                                                    const int32_t* __restrict__ active) {
  extern __shared__ double ring[];   // [BT][32][KC]
  __shared__ double T[32][KC + 1];
  int chunk = blockIdx.x % n_chunk;
  int box = blockIdx.x / n_chunk;
  if (box >= n_box) return;
  if (active && !active[box]) return;
  const BoxMeta& bm = meta[box];
  BandView v = band_view(bm, kind);
  const double* L = fac + v.off;
  const double* Li = fac + v.ioff;
  const uint8_t* cl = cls + bm.dof_off;
  const int tid = threadIdx.x;
  const int r = tid / KC, c = tid % KC;   // 32 x KC outputs per tile row (256 = 32*8)
  const int col = chunk * KC + c;
  const bool colok = col < ldk;
  const double* vin = in + bm.vec_off;
  double* vout = out + bm.vec_off;
  double* y = scratch + (int64_t)(box * n_chunk + chunk) * scratch_stride;
  // forward: L y = f
  for (int I = 0; I < v.NT; ++I) {
    int row = I * 32 + r;
    int dof = band_to_dof(v, bm, row);
    double acc = 0.0;
    if (dof >= 0 && colok && dof_active(kind, cl[dof])) acc = vin[(int64_t)dof * ldk + col];
    int smax = min(v.BT - 1, I);
    for (int s = 1; s <= smax; ++s) {
      const double* Lt = L + ((int64_t)I * v.BT + s) * MSG_TILE2 + r * 32;
      const double* yp = ring + (int64_t)((I - s) % v.BT) * 32 * KC;
#pragma unroll 8
      for (int q = 0; q < 32; ++q) acc -= Lt[q] * yp[q * KC + c];
    }
    T[r][c] = acc;
    __syncthreads();
    const double* Di = Li + (int64_t)I * MSG_TILE2 + r * 32;
    double yv = 0.0;
    for (int q = 0; q <= r; ++q) yv += Di[q] * T[q][c];
    ring[(int64_t)(I % v.BT) * 32 * KC + r * KC + c] = yv;
    y[(int64_t)row * KC + c] = yv;
    __syncthreads();
  }
  // backward: L^T x = y
  for (int I = v.NT - 1; I >= 0; --I) {
    int row = I * 32 + r;
    double acc = y[(int64_t)row * KC + c];
    int smax = min(v.BT - 1, v.NT - 1 - I);
    for (int s = 1; s <= smax; ++s) {
      const double* Lt = L + ((int64_t)(I + s) * v.BT + s) * MSG_TILE2 + r;
      const double* xp = ring + (int64_t)((I + s) % v.BT) * 32 * KC;
#pragma unroll 8
      for (int q = 0; q < 32; ++q) acc -= Lt[q * 32] * xp[q * KC + c];
    }
    T[r][c] = acc;
    __syncthreads();
    const double* Di = Li + (int64_t)I * MSG_TILE2 + r;
    double xv = 0.0;
    for (int q = r; q < 32; ++q) xv += Di[q * 32] * T[q][c];
    ring[(int64_t)(I % v.BT) * 32 * KC + r * KC + c] = xv;
    int dof = band_to_dof(v, bm, row);
    if (dof >= 0 && colok) {
      uint8_t k = cl[dof];
      if (dof_active(kind, k) && ((out_classes >> k) & 1)) vout[(int64_t)dof * ldk + col] = xv;
    }
    __syncthreads();
  }
  if (zero_rest && colok) {
    // zero the DoFs of this box (this chunk's columns) that were not written
    for (int d = tid / KC; d < bm.n_dof; d += 256 / KC) {
      uint8_t k = cl[d];
      bool written = false;
      if (dof_active(kind, k) && ((out_classes >> k) & 1)) {
        // A11 orders only the sub-box: B1 DoFs always lie in it
        written = true;
      }
      if (!written) vout[(int64_t)d * ldk + col] = 0.0;
    }
  }
}

template __global__ void k_band_solve<8>(const BoxMeta*, int, int, int, const double*, const uint8_t*,
                                         const double*, double*, int, int, int, double*, int64_t,
                                         const int32_t*);

}  // namespace msg
