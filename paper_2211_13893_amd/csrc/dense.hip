// Dense block kernels of the locally optimal block preconditioned conjugate
// gradient (LOBPCG) iteration on the shifted A-harmonic pencil
//      M x = nu T x,   T = S + s M,   nu = 1/(lambda + s)
// (Sec. 3.3 and 4.3: S x = lambda M x is the mixed GEVP after eliminating the
// Lagrange multiplier and the B1 unknowns).  Basis blocks are stored as
// full-box vectors Z~ = [E Z; Z] together with A Z~, D A D Z~ and M Z, so the
// Gram matrices of the Rayleigh-Ritz step are Z~^T A Z~ = Z^T S Z and
// Z~^T (D A D) Z~ = Z^T M Z.
//
//  k_gram_partial / k_gram_reduce : Gram matrices over row chunks, summed in a
//                                   fixed order (bitwise reproducible).
//  k_rayleigh_ritz                : one workgroup per box: scaled Cholesky of
//                                   the T-Gram with dropping of near-dependent
//                                   columns, congruence of the M-Gram, cyclic
//                                   parallel Jacobi, top-k Ritz coefficients.
//  k_update                       : X <- Z Y, P <- Z Yp for the four kinds.
//  k_residual / k_converge        : R = M X - nu T X on B2, the scale-free
//                                   residual rho = |R| / (|MX| + nu |TX|),
//                                   convergence and iteration bookkeeping.
#include <cfloat>

#include "internal.hpp"

namespace msg {

struct Blk3 {
  const double* p[3];
};

#define UPD_DEPTH 2    // MFMA step pairs (8 inner indices each) whose A operands are requested ahead

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Partial Gram matrices of one row chunk of one box:
//   part[box][chunk][0] = Z^T (A Z),  part[box][chunk][1] = Z^T (B Z)
// (upper 16x16 blocks only), Z = [Z_0 .. Z_{nblk-1}] of m = nblk*k <= 16 NB
// columns, with the FP64 matrix cores (16x16x4: one group of 4 rows is one
// inner step).  The workgroup stages the chunk GRAM_SLAB rows at a time: the
// rows of Z, A Z and B Z with 16-byte loads into LDS (two buffers; the next
// slab is requested while this one is used), laid out so that the operand of
// one (16-column slice, group of 4 rows) is 64 consecutive doubles in lane
// order.  Wavefront w of the NB takes product p = w / (NB/2) and the block
// rows a = w % (NB/2) and NB-1-a: NB+1 blocks for every wavefront, each a sum
// over the chunk's rows in order.  The chunks are added by k_gram_reduce.
#define GRAM_SLAB 16
#define GRAM_PIECES 6   // 16-byte pieces per thread and slab: 3 * GRAM_SLAB * m/2 <= 6 * 64 NB

template <int NB, int A>
__device__ __forceinline__ void gram_chunk(double* __restrict__ sh, int m, int k, int64_t base, int r_begin,
                                           int r_end, int which, const Blk3& Z, const Blk3& AZ, const Blk3& BZ,
                                           double* __restrict__ out) {
  constexpr int R0 = A, R1 = NB - 1 - A;   // the two block rows
  constexpr int NW = NB - A;               // product slices A .. NB-1
  constexpr int N1 = A + 1;                // blocks of row R1: columns R1 .. NB-1
  constexpr int KIND = 4 * NB * 64;        // doubles of one kind in a buffer
  constexpr int BUF = 3 * KIND;
  const int t = threadIdx.x, lane = t & 63;
  // this thread's pieces: kind, slab row, column pair -> source and LDS slot
  const int half = m / 2, per_kind = GRAM_SLAB * half;
  const double* src[GRAM_PIECES];
  int dst[GRAM_PIECES], prow[GRAM_PIECES];
#pragma unroll
  for (int i = 0; i < GRAM_PIECES; ++i) {
    const int e = t + i * 64 * NB;
    prow[i] = -1;
    src[i] = nullptr;
    dst[i] = 0;
    if (e < 3 * per_kind) {
      const int kq = e / per_kind, rem = e - kq * per_kind;
      const int rr = rem / half, c = 2 * (rem - rr * half);
      const Blk3& X = kq == 0 ? Z : (kq == 1 ? AZ : BZ);
      const int cb = c / k;
      const double* x = cb == 0 ? X.p[0] : (cb == 1 ? X.p[1] : X.p[2]);
      src[i] = x + base + (c - cb * k);
      prow[i] = rr;
      dst[i] = kq * KIND + ((rr >> 2) * NB + (c >> 4)) * 64 + (rr & 3) * 16 + (c & 15);
    }
  }
  const int n_slab = (r_end - r_begin + GRAM_SLAB - 1) / GRAM_SLAB;
  double2 v[GRAM_PIECES];
  auto fetch = [&](int slab) {
#pragma unroll
    for (int i = 0; i < GRAM_PIECES; ++i) {
      const int row = r_begin + slab * GRAM_SLAB + prow[i];
      v[i] = (prow[i] >= 0 && row < r_end) ? *reinterpret_cast<const double2*>(src[i] + (int64_t)row * k)
                                           : make_double2(0.0, 0.0);
    }
  };
  // slots of columns past m are never staged: zero both buffers once
  for (int e = t; e < 2 * BUF; e += 64 * NB) sh[e] = 0.0;
  dbl4 acc0[NW], acc1[N1];
#pragma unroll
  for (int j = 0; j < NW; ++j) acc0[j] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < N1; ++j) acc1[j] = dbl4{0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  if (n_slab > 0) fetch(0);
  for (int slab = 0; slab < n_slab; ++slab) {
    double* B = sh + (slab & 1) * BUF;
#pragma unroll
    for (int i = 0; i < GRAM_PIECES; ++i)
      if (prow[i] >= 0) *reinterpret_cast<double2*>(B + dst[i]) = v[i];
    // one barrier per slab: a buffer is rewritten two slabs later, after
    // every wavefront has passed the barrier that follows its last reads
    __syncthreads();
    if (slab + 1 < n_slab) fetch(slab + 1);
    const double* Zs = B;
    const double* Ws = B + (1 + which) * KIND;
#pragma unroll
    for (int g = 0; g < GRAM_SLAB / 4; ++g) {
      const double z0 = Zs[(g * NB + R0) * 64 + lane], z1 = Zs[(g * NB + R1) * 64 + lane];
      double w[NW];
#pragma unroll
      for (int j = 0; j < NW; ++j) w[j] = Ws[(g * NB + A + j) * 64 + lane];
#pragma unroll
      for (int j = 0; j < NW; ++j) acc0[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(z0, w[j], acc0[j], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < N1; ++j)
        acc1[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(z1, w[R1 - A + j], acc1[j], 0, 0, 0);
    }
  }
  // item q of lane l is entry (16 bi + (l>>4) + 4q, 16 bj + (l&15)) of the block
  const int lc = lane & 15, lr = lane >> 4;
#pragma unroll
  for (int j = 0; j < NW; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * R0 + lr + 4 * q, c = 16 * (A + j) + lc;
      if (i < m && c < m) out[i * m + c] = acc0[j][q];
    }
#pragma unroll
  for (int j = 0; j < N1; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * R1 + lr + 4 * q, c = 16 * (R1 + j) + lc;
      if (i < m && c < m) out[i * m + c] = acc1[j][q];
    }
}

template <int NB>
__global__ __launch_bounds__(64 * NB) void k_gram_partial(const BoxMeta* __restrict__ meta, int nblk,
                                                          Blk3 Z, Blk3 AZ, Blk3 BZ, int k,
                                                          int rows_per_chunk, int n_chunk,
                                                          double* __restrict__ part,
                                                          const int32_t* __restrict__ active) {
  static_assert(NB == 2 || NB == 4 || NB == 6, "2, 4 or 6 blocks of 16 columns");
  __shared__ __align__(16) double sh[2 * 3 * 4 * NB * 64];
  const int box = blockIdx.y, chunk = blockIdx.x;
  if (active && !active[box]) return;
  const BoxMeta& bm = meta[box];
  const int m = nblk * k;
  const int wave = threadIdx.x >> 6;
  const int which = wave / (NB / 2), a = wave % (NB / 2);
  const int r_begin = chunk * rows_per_chunk;
  const int r_end = min(bm.n_dof, r_begin + rows_per_chunk);
  const int64_t base = bm.dof_off * k;
  double* out = part + (((int64_t)box * n_chunk + chunk) * 2 + which) * m * m;
  // every wavefront passes the same barriers whichever block rows it holds
  if (a == 0) gram_chunk<NB, 0>(sh, m, k, base, r_begin, r_end, which, Z, AZ, BZ, out);
  if constexpr (NB >= 4) {
    if (a == 1) gram_chunk<NB, 1>(sh, m, k, base, r_begin, r_end, which, Z, AZ, BZ, out);
  }
  if constexpr (NB >= 6) {
    if (a == 2) gram_chunk<NB, 2>(sh, m, k, base, r_begin, r_end, which, Z, AZ, BZ, out);
  }
}

// G[box][2][m][m] = sum over chunks (fixed order); lower 16-blocks mirrored.

template __global__ void k_gram_partial<2>(const BoxMeta*, int, Blk3, Blk3, Blk3, int, int, int, double*,
                                           const int32_t*);
template __global__ void k_gram_partial<4>(const BoxMeta*, int, Blk3, Blk3, Blk3, int, int, int, double*,
                                           const int32_t*);
template __global__ void k_gram_partial<6>(const BoxMeta*, int, Blk3, Blk3, Blk3, int, int, int, double*,
                                           const int32_t*);

__global__ void k_gram_reduce(int m, int n_chunk, const double* __restrict__ part,
                              double* __restrict__ G, const int32_t* __restrict__ active) {
  int box = blockIdx.y;
  if (active && !active[box]) return;
  const int mm = m * m, mm2 = 2 * mm;
  int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= mm2) return;
  int which = o / mm, e = o % mm, i = e / m, j = e % m;
  int src = ((i >> 4) <= (j >> 4)) ? e : j * m + i;
  const double* p = part + (int64_t)box * n_chunk * mm2 + which * mm + src;
  double s = 0.0;
  for (int c = 0; c < n_chunk; ++c) s += p[(int64_t)c * mm2];
  G[(int64_t)box * mm2 + o] = s;
}

// One workgroup per box.  dynamic LDS: C[m][m+1], V[m][m+1] + small arrays.
// Lg: global scratch m*m per box for the Cholesky factor.
#define RR_THREADS 1024

// In-place triangular solve with the lower-triangular Lm (LDS, leading
// dimension ld) for one right-hand side x_i = X[base + i*stride] by a group of
// 8 consecutive lanes (gl = lane in the group): forward L x = b, or backward
// L^T x = b.  Each dot product is split over the 8 lanes and summed with lane
// shuffles; the group's first lane writes x_i.
__device__ inline void tri_solve_group(const double* Lm, int ld, int m, double* X, int base, int stride,
                                       bool backward, int gl) {
  for (int step = 0; step < m; ++step) {
    const int i = backward ? m - 1 - step : step;
    double s = 0.0;
    if (!backward) {
      for (int q = gl; q < i; q += 8) s += Lm[i * ld + q] * X[base + q * stride];
    } else {
      for (int q = i + 1 + gl; q < m; q += 8) s += Lm[q * ld + i] * X[base + q * stride];
    }
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 4);
    if (gl == 0) X[base + i * stride] = (X[base + i * stride] - s) / Lm[i * ld + i];
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  }
}

__global__ __launch_bounds__(1024) void k_rayleigh_ritz(int m, int k, int nblk_x, double shift,
                                                       const double* __restrict__ G,
                                                       double* __restrict__ Lg,
                                                       double* __restrict__ Y,
                                                       double* __restrict__ Yp,
                                                       double* __restrict__ nu,
                                                       const int32_t* __restrict__ active) {
  extern __shared__ double sm[];
  int box = blockIdx.x;
  if (active && !active[box]) return;
  const int ld = m + 1;
  double* C = sm;
  double* V = C + m * ld;
  double* dsc = V + m * ld;          // m scale factors
  double* ev = dsc + m;              // m eigenvalues
  double* rcb = ev + m;              // 2 x m/2 rotation cos (two rounds: even, odd)
  double* rsb = rcb + m;             // 2 x m/2 rotation sin
  double* red = rsb + m;             // 256 reduction slots
  int* drop = (int*)(red + 256);     // m
  int* order = drop + m;             // m
  int* ppb = order + m;              // 2 x m/2: rotation pairs of the two rounds
  int* qqb = ppb + m;                // 2 x m/2
  int* perm = qqb + m;               // m: active directions first (Jacobi on those only)
  int* nj = perm + m;                // 1: size of the Jacobi block
  const int tid = threadIdx.x;
  const double* GA = G + (int64_t)box * 2 * m * m;
  const double* GB = GA + m * m;
  double* L = Lg + (int64_t)box * m * m;
  // 1. scaled T-Gram
  for (int i = tid; i < m; i += RR_THREADS) {
    double t = GA[i * m + i] + shift * GB[i * m + i];
    dsc[i] = (t > 0.0) ? 1.0 / sqrt(t) : 0.0;
    drop[i] = (t > 0.0) ? 0 : 1;
  }
  __syncthreads();
  for (int t = tid; t < m * m; t += RR_THREADS) {
    int i = t / m, j = t % m;
    double a = 0.5 * ((GA[i * m + j] + shift * GB[i * m + j]) + (GA[j * m + i] + shift * GB[j * m + i]));
    C[i * ld + j] = a * dsc[i] * dsc[j];
  }
  __syncthreads();
  // 2. Cholesky with dropping of near-dependent columns (pivot <= tau: the
  //    column becomes e_j and row j of L is cleared), left-looking on one
  //    wavefront: L[i][j] = (C[i][j] - sum_{q<j} L[i][q] L[j][q]) / L[j][j]
  const double tau = 1e-12;
  if (tid < 64) {
    const int ln = tid;
    for (int j = 0; j < m; ++j) {
      double pp = 0.0;
      for (int q = ln; q < j; q += 64) pp += C[j * ld + q] * C[j * ld + q];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) pp += __shfl_xor(pp, o);
      const double piv = C[j * ld + j] - pp;
      const bool dj = drop[j] || !(piv > tau);
      if (dj) {
        for (int t = ln; t < m; t += 64) {
          if (t > j) C[t * ld + j] = 0.0;
          if (t < j) C[j * ld + t] = 0.0;
        }
        if (ln == 0) {
          C[j * ld + j] = 1.0;
          drop[j] = 1;
        }
      } else {
        const double sd = sqrt(piv);
        for (int i = j + 1 + ln; i < m; i += 64) {
          double t = C[i * ld + j];
          for (int q = 0; q < j; ++q) t -= C[i * ld + q] * C[j * ld + q];
          C[i * ld + j] = t / sd;
        }
        if (ln == 0) C[j * ld + j] = sd;
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
  }
  __syncthreads();
  // keep L in LDS (V's space, free until the Jacobi sweeps) and in global
  for (int t = tid; t < m * m; t += RR_THREADS) {
    int i = t / m, c = t % m;
    double l = (c <= i) ? C[i * ld + c] : 0.0;
    L[t] = l;
    V[i * ld + c] = l;
  }
  __syncthreads();
  // 3. scaled M-Gram, dropped rows/columns removed
  for (int t = tid; t < m * m; t += RR_THREADS) {
    int i = t / m, j = t % m;
    double b = 0.5 * (GB[i * m + j] + GB[j * m + i]) * dsc[i] * dsc[j];
    C[i * ld + j] = (drop[i] || drop[j]) ? 0.0 : b;
  }
  __syncthreads();
  // 4. C <- L^{-1} C (columns as right-hand sides), then C <- C L^{-T} (rows)
  {
    const int grp = tid >> 3, gl = tid & 7;
    if (grp < m) tri_solve_group(V, ld, m, C, grp, ld, false, gl);
    __syncthreads();
    if (grp < m) tri_solve_group(V, ld, m, C, grp * ld, 1, false, gl);
    __syncthreads();
  }
  for (int t = tid; t < m * m; t += RR_THREADS) {
    int i = t / m, j = t % m;
    if (i < j) {
      double a = 0.5 * (C[i * ld + j] + C[j * ld + i]);
      C[i * ld + j] = a;
      C[j * ld + i] = a;
    }
  }
  __syncthreads();
  // 4b. Directions dropped by the Cholesky (zero rows and columns of C, e.g.
  //     the W and P columns of converged pairs) need no rotations: C is
  //     permuted to P C P^T with the active directions first, and Jacobi runs
  //     on the leading mj x mj block (mj = their count, made even with one
  //     dropped direction if needed).
  if (tid == 0) {
    int a = 0;
    for (int i = 0; i < m; ++i)
      if (!drop[i]) perm[a++] = i;
    const int na = a;
    for (int i = 0; i < m; ++i)
      if (drop[i]) perm[a++] = i;
    nj[0] = min(m, max(2, na + (na & 1)));
  }
  __syncthreads();
  for (int t = tid; t < m * m; t += RR_THREADS) {
    const int i = t / m, j = t % m;
    V[i * ld + j] = C[perm[i] * ld + perm[j]];
  }
  __syncthreads();
  for (int t = tid; t < m * m; t += RR_THREADS) {
    const int i = t / m, j = t % m;
    C[i * ld + j] = V[i * ld + j];
    V[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int mj = nj[0];
  // 5. cyclic parallel Jacobi (round-robin pairing, mj even).  Round r pairs
  //    (0, 1 + r mod (m-1)) and (1 + (r+i) mod (m-1), 1 + (r-i) mod (m-1)),
  //    i = 1..m/2-1; all m/2 rotations of a round commute.  A round computes
  //    the rotations, then applies them to C from both sides in one pass over
  //    the 2x2 blocks C[{p_a,q_a},{p_b,q_b}] <- R_a B R_b^T, R = [[c,-s],[s,c]],
  //    and to the columns of V (V <- V R^T); the next round's rotations are
//    computed while V is updated.  Only the upper triangle of C is
  //    kept (entry (x, y) at C[min][max]), so a round updates the blocks with
  //    a <= b; a thread applies one rotation to several rows of V.  Both halve
  //    the LDS traffic of a round, which bounds it.
  const int h = mj / 2, m1 = mj - 1;
  auto cix = [&](int x, int y) { return x < y ? x * ld + y : y * ld + x; };
  auto pair_of = [&](int r, int i, int& p, int& q) {
    if (i == 0) {
      p = 0;
      q = 1 + (r % m1);
    } else {
      int a1 = r + i;
      if (a1 >= m1) a1 -= m1;
      int a2 = r + m1 - i;
      if (a2 >= m1) a2 -= m1;
      if (a2 >= m1) a2 -= m1;
      p = 1 + a1;
      q = 1 + a2;
    }
  };
  int* zero_pq = order;   // 2 x m/2 flags per pair (reused: order is set in step 6)
  // A thread's share of a round is the same in every round: the 2x2 blocks
  // (a, b), a <= b, numbered e = tid and tid + RR_THREADS along the rows of the
  // triangle (row a holds h - a blocks; h (h + 1) / 2 <= 2 RR_THREADS for
  // m <= 126), and the rows g, g + G, ... of V for rotation i.
  int blk_a[2], blk_b[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    int e = tid + u * RR_THREADS, a = 0;
    while (a < h && e >= h - a) {
      e -= h - a;
      ++a;
    }
    blk_a[u] = a < h ? a : -1;
    blk_b[u] = a < h ? a + e : -1;
  }
  // V is updated by the threads below RR_THREADS - 64 while the last wavefront
  // computes the next round's rotations (they depend on C only)
  const int vG = (RR_THREADS - 64) / h, vi = tid % h, vg = tid / h;
  // rotation i of round r into buffer b (of two, by round parity)
  auto rotation = [&](int r, int b, int i) {
    int p, q;
    pair_of(r, i, p, q);
    ppb[b * (m / 2) + i] = p;
    qqb[b * (m / 2) + i] = q;
    const double apq = C[cix(p, q)];
    const double app = C[p * ld + p], aqq = C[q * ld + q];
    double c = 1.0, sn = 0.0;
    int z = 0;
    // (|apq| > 1e-18 sqrt|app aqq| compared squared: one square root less on
    // the round's serial path)
    if (fabs(apq) > 1e-300 && apq * apq > 1e-36 * fabs(app * aqq)) {
      const double th = (aqq - app) / (2.0 * apq);
      const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
      c = rsqrt(1.0 + t * t);
      sn = t * c;
      z = 1;
    } else if (fabs(apq) > 0.0) {
      z = 1;
    }
    rcb[b * (m / 2) + i] = c;
    rsb[b * (m / 2) + i] = sn;
    zero_pq[b * (m / 2) + i] = z;
  };
  for (int sweep = 0; sweep < 30; ++sweep) {
    // convergence test: off-diagonal mass vs. total (one barrier)
    double off = 0.0, tot = 0.0;
    for (int t = tid; t < mj * mj; t += RR_THREADS) {
      const int i = t / mj, j = t - (t / mj) * mj;
      if (i > j) continue;
      const double a = C[i * ld + j];
      if (i == j) {
        tot += a * a;
      } else {
        off += 2.0 * a * a;
        tot += 2.0 * a * a;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      tot += __shfl_xor(tot, o);
    }
    if ((tid & 63) == 0) {
      red[tid >> 6] = off;
      red[16 + (tid >> 6)] = tot;
    }
    __syncthreads();
    double offs = 0.0, tots = 0.0;
    for (int w = 0; w < RR_THREADS / 64; ++w) {
      offs += red[w];
      tots += red[16 + w];
    }
    __syncthreads();
    // relative off-diagonal norm 1e-12: Ritz values then carry errors ~1e-24
    if (offs <= 1e-24 * tots || tots == 0.0) break;
    for (int i = tid; i < h; i += RR_THREADS) rotation(0, 0, i);
    __syncthreads();
    for (int r = 0; r < m1; ++r) {
      const int bo = (r & 1) * (m / 2);
      const int* pp = ppb + bo;
      const int* qq = qqb + bo;
      const double* rc = rcb + bo;
      const double* rs = rsb + bo;
      const int* zq = zero_pq + bo;
      // C <- R C R^T over the 2x2 blocks (a <= b) of the upper triangle
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int ia = blk_a[u], ib = blk_b[u];
        if (ia < 0) continue;
        const int pa = pp[ia], qa = qq[ia], pb = pp[ib], qb = qq[ib];
        const double ca = rc[ia], sa = rs[ia], cb = rc[ib], sb = rs[ib];
        if (ia == ib) {
          const int e01 = cix(pa, qa);
          const double b00 = C[pa * ld + pa], b01 = C[e01], b11 = C[qa * ld + qa];
          const double r00 = ca * b00 - sa * b01, r01 = ca * b01 - sa * b11;
          const double r10 = sa * b00 + ca * b01, r11 = sa * b01 + ca * b11;
          const double n00 = ca * r00 - sa * r01, n11 = sa * r10 + ca * r11;
          // (pa, qa) is the entry the rotation annihilates
          const double n01 = zq[ia] ? 0.0 : sa * r00 + ca * r01;
          C[pa * ld + pa] = n00;
          C[e01] = (pa < qa) ? n01 : (zq[ia] ? 0.0 : ca * r10 - sa * r11);
          C[qa * ld + qa] = n11;
        } else {
          const int e00 = cix(pa, pb), e01 = cix(pa, qb), e10 = cix(qa, pb), e11 = cix(qa, qb);
          const double b00 = C[e00], b01 = C[e01], b10 = C[e10], b11 = C[e11];
          // rows: R_a B
          const double r00 = ca * b00 - sa * b10, r01 = ca * b01 - sa * b11;
          const double r10 = sa * b00 + ca * b10, r11 = sa * b01 + ca * b11;
          // columns: (R_a B) R_b^T
          C[e00] = cb * r00 - sb * r01;
          C[e01] = sb * r00 + cb * r01;
          C[e10] = cb * r10 - sb * r11;
          C[e11] = sb * r10 + cb * r11;
        }
      }
      __syncthreads();
      if (tid >= RR_THREADS - 64) {
        // the next round's rotations, from the updated C
        const int i = tid - (RR_THREADS - 64);
        if (r + 1 < m1 && i < h) rotation(r + 1, (r + 1) & 1, i);
      } else {
        // V <- V R^T: thread (pair i, row group g) takes rows g, g + G, ...
        const int G = vG, i = vi, g = vg;
        if (g < G) {
          const int p = pp[i], q = qq[i];
          const double c = rc[i], sn = rs[i];
          for (int row = g; row < mj; row += G) {
            const double vp = V[row * ld + p], vq = V[row * ld + q];
            V[row * ld + p] = c * vp - sn * vq;
            V[row * ld + q] = sn * vp + c * vq;
          }
        }
      }
      __syncthreads();
    }
  }
  // 6. sort eigenvalues descending (dropped directions have eigenvalue 0);
  //    eigenvector c is column c of V, its rows back in the original order
  for (int i = tid; i < m; i += RR_THREADS) {
    double e = C[i * ld + i];
    ev[i] = (e == e) ? e : -1.0e300;   // NaN ranks last
    order[i] = i;
  }
  __syncthreads();
  for (int t = tid; t < m * m; t += RR_THREADS) {
    const int i = t / m, c = t % m;
    C[perm[i] * ld + c] = V[i * ld + c];
  }
  __syncthreads();
  for (int t = tid; t < m * m; t += RR_THREADS) {
    const int i = t / m, c = t % m;
    V[i * ld + c] = C[i * ld + c];
  }
  __syncthreads();
  for (int i = tid; i < m; i += RR_THREADS) {
    double e = ev[i];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      double f = ev[j];
      if (f > e || (f == e && j < i)) ++rank;
    }
    order[rank] = i;
  }
  __syncthreads();
  // 7. Ritz coefficients Y[:, c] = D L^{-T} V[:, order[c]] (L back in LDS, C's space;
  //    the back substitution runs in place in the column of V owned by c)
  for (int t = tid; t < m * m; t += RR_THREADS) {
    int i = t / m, q = t % m;
    C[i * ld + q] = L[t];
  }
  __syncthreads();
  double* Yb = Y + (int64_t)box * m * k;
  double* Ypb = Yp + (int64_t)box * m * k;
  {
    const int grp = tid >> 3, gl = tid & 7;
    if (grp < k) tri_solve_group(C, ld, m, V, order[grp], ld, true, gl);
  }
  __syncthreads();
  for (int t = tid; t < m * k; t += RR_THREADS) {
    const int i = t / k, c = t - (t / k) * k;
    Yb[t] = V[i * ld + order[c]];
  }
  for (int c = tid; c < k; c += RR_THREADS) nu[(int64_t)box * k + c] = ev[order[c]];
  __syncthreads();
  for (int t = tid; t < m * k; t += RR_THREADS) {
    int i = t / k;
    double v = Yb[t] * dsc[i];
    v = drop[i] ? 0.0 : v;
    Yb[t] = v;
    Ypb[t] = (i < nblk_x * k) ? 0.0 : v;
  }
}

struct Blk4x3 {
  const double* p[4][3];
};
struct Out4 {
  double* p[4];
};

// X_new = Z Y, P_new = Z Yp for kind = blockIdx.z (0: Z~, 1: A Z~, 2: DAD Z~, 3: M Z),
// Z = [Z_0 .. Z_{nblk-1}] of m = nblk*k columns, Y and Yp m x k per box.
// FP64 matrix cores (16x16x4): a wavefront takes 16 rows at a time (4 blocks
// of 16 rows per wavefront, UPD_ROWS rows per workgroup); the inner index
// runs over the m columns of Z, 8 per pair of MFMA steps: lane (row li,
// lk) loads Z[row][8t + 2lk .. +1] as one 16-byte piece and uses its halves
// in steps 2t and 2t+1 (inner index 8t + 2lk + e), and the B operand is
// read to match.  Output columns in CB blocks of 16 (k <= 16 CB: 2 for the
// LOBPCG block, 6 for a coarse basis of up to 96 columns); Y and Yp are
// staged in LDS once per workgroup in operand order: the B operand of step
// 2t + e and column block cb is 64 consecutive doubles in lane order (lane
// (lk, li) holds Y[8t + 2lk + e][16 cb + li], zero outside m x k), so every
// operand read is one conflict-free ds_read_b64 with a constant offset.
// grid (ceil(max n_dof / UPD_ROWS), n_box, kinds);
// dynamic LDS = 2 * ceil(m/8) * 2 * CB * 64 doubles
template <int CB>
__global__ __launch_bounds__(UPD_THREADS, CB == 2 ? 3 : 1) void k_update(const BoxMeta* __restrict__ meta, int nblk, int k,
                                                Blk4x3 Z, Out4 OX, Out4 OP,
                                                const double* __restrict__ Y,
                                                const double* __restrict__ Yp,
                                                const int32_t* __restrict__ active) {
  extern __shared__ double sm[];
  int box = blockIdx.y, kind = blockIdx.z;
  const BoxMeta& bm = meta[box];
  // a converged box's block stays in the buffer it was retired in (XLoc)
  if (active && !active[box]) return;
  const int r_wg = blockIdx.x * UPD_ROWS;
  if (r_wg >= bm.n_dof) return;
  const int m = nblk * k;
  const int npairs = (m + 7) >> 3;
  const int ystride = npairs * 2 * CB * 64;   // doubles of one staged matrix
  double* ys = sm;
  double* yps = sm + ystride;
  const bool wantP = OP.p[kind] != nullptr;
  for (int t = threadIdx.x; t < ystride; t += UPD_THREADS) {
    // slot t: operand group g = (2 tp + e) CB + cb, lane l
    const int l = t & 63, g = t >> 6;
    const int cb = g % CB, te = g / CB, tp = te >> 1, e = te & 1;
    const int i = 8 * tp + 2 * (l >> 4) + e, c = 16 * cb + (l & 15);
    const bool ok = i < m && c < k;
    const int64_t src = (int64_t)box * m * k + (ok ? i * k + c : 0);
    ys[t] = ok ? Y[src] : 0.0;
    yps[t] = (ok && wantP) ? Yp[src] : 0.0;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t base = bm.dof_off * k;
  for (int rb = 0; rb < 4; ++rb) {
    const int r0 = r_wg + (wave * 4 + rb) * 16;
    if (r0 >= bm.n_dof) break;
    const int row = r0 + li;
    const bool rok = row < bm.n_dof;
    dbl4 ax[CB], ap[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      ax[cb] = dbl4{0.0, 0.0, 0.0, 0.0};
      ap[cb] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
    // A operands of step pair t (inner indices 8t + 2lk, +1: one block, k
    // being a multiple of 8).  Two register sets of UPD_DEPTH pairs: the
    // next set is requested before the current one is multiplied.
    auto load_a = [&](int t) {
      const int i = 8 * t + 2 * lk;
      double2 a = double2{0.0, 0.0};
      if (t < npairs && rok && i < m) {
        const int b = i / k;
        a = *(const double2*)(Z.p[kind][b] + base + (int64_t)row * k + (i - b * k));
      }
      return a;
    };
    auto mma = [&](int t, double2 a) {
      if (t < npairs) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const double av = e ? a.y : a.x;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            const int o = ((2 * t + e) * CB + cb) * 64 + lane;
            ax[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, ys[o], ax[cb], 0, 0, 0);
            if (wantP) ap[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, yps[o], ap[cb], 0, 0, 0);
          }
        }
      }
    };
    double2 pa[UPD_DEPTH], pb[UPD_DEPTH];
#pragma unroll
    for (int j = 0; j < UPD_DEPTH; ++j) pa[j] = load_a(j);
    for (int t = 0; t < npairs; t += 2 * UPD_DEPTH) {
#pragma unroll
      for (int j = 0; j < UPD_DEPTH; ++j) pb[j] = load_a(t + UPD_DEPTH + j);
#pragma unroll
      for (int j = 0; j < UPD_DEPTH; ++j) mma(t + j, pa[j]);
#pragma unroll
      for (int j = 0; j < UPD_DEPTH; ++j) pa[j] = load_a(t + 2 * UPD_DEPTH + j);
#pragma unroll
      for (int j = 0; j < UPD_DEPTH; ++j) mma(t + UPD_DEPTH + j, pb[j]);
    }
    // accumulator item v of lane l: row r0 + (l >> 4) + 4 v, column 16 cb + (l & 15)
    double* ox = OX.p[kind] + base;
    double* op = wantP ? OP.p[kind] + base : nullptr;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int col = 16 * cb + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ro = r0 + lk + 4 * v;
        if (ro < bm.n_dof && col < k) {
          ox[(int64_t)ro * k + col] = ax[cb][v];
          if (wantP) op[(int64_t)ro * k + col] = ap[cb][v];
        }
      }
    }
  }
}

template __global__ void k_update<2>(const BoxMeta*, int, int, Blk4x3, Out4, Out4, const double*, const double*,
                                     const int32_t*);
template __global__ void k_update<6>(const BoxMeta*, int, int, Blk4x3, Out4, Out4, const double*, const double*,
                                     const int32_t*);

// Deflation against the converged block Yq of an earlier round (Z = [W, Yq]):
// Yc = [I; -C] with C = (T Yq)^T W, the cross block of the T-Gram matrix
// G_S + s G_M of [W, Yq] (m = 2k; Yq is T-orthonormal with zero guard
// columns), so that k_update forms W - Yq C for every image kind.
__global__ void k_proj_coef(int k, double shift, const double* __restrict__ G, double* __restrict__ Yc,
                            const int32_t* __restrict__ active) {
  const int box = blockIdx.x;
  if (active && !active[box]) return;
  const int m = 2 * k, mm = m * m;
  const double* GS = G + (int64_t)box * 2 * mm;
  const double* GM = GS + mm;
  double* Y = Yc + (int64_t)box * m * k;
  for (int t = threadIdx.x; t < m * k; t += blockDim.x) {
    const int i = t / k, c = t % k;
    double v;
    if (i < k) {
      v = (i == c) ? 1.0 : 0.0;
    } else {
      const int e = i * m + c;   // row k + q (Yq column q), column c (W column c)
      v = -(GS[e] + shift * GM[e]);
    }
    Y[t] = v;
  }
}

// dst = X (image kind `kind`, located by xl) on the first cnt columns of
// every box, 0 on the others, cnt = min(nround, n_ev - col0): a round's
// converged block with its guard columns cleared (grid (rows, n_box))
__global__ void k_keep_cols(const BoxMeta* __restrict__ meta, int k, int col0, int nround, XLoc xl, int kind,
                            double* __restrict__ dst) {
  const BoxMeta& bm = meta[blockIdx.y];
  const double* __restrict__ src = xl.at(kind, blockIdx.y);
  const int cnt = min(nround, bm.n_ev - col0);
  const int64_t n = (int64_t)bm.n_dof * k;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % k);
    dst[bm.dof_off * k + t] = c < cnt ? src[bm.dof_off * k + t] : 0.0;
  }
}

// R = MX - nu (SX + s MX) on the rows whose class bit is set in rcls (B2 for
// the A-harmonic GEVP, where SX = (A X~) on B2; B1 u B2 for GenEO), written
// into R (zero elsewhere); partial column sums of |R|^2, |MX|^2, |TX|^2.
// grid (n_chunk, n_box), RES_THREADS threads; thread = (row slot tid/32, column tid%32); k <= 32
#define RES_THREADS 1024   // k_residual: 32 columns x 32 row slots
__global__ __launch_bounds__(RES_THREADS) void k_residual(const BoxMeta* __restrict__ meta,
                                                  const uint8_t* __restrict__ cls, int rcls, int k,
                                                  double shift, const double* __restrict__ AX,
                                                  const double* __restrict__ MX,
                                                  const double* __restrict__ nu,
                                                  double* __restrict__ R, int rows_per_chunk,
                                                  int n_chunk, double* __restrict__ part,
                                                  const int32_t* __restrict__ active) {
  __shared__ double red[3][RES_THREADS];
  int box = blockIdx.y, chunk = blockIdx.x;
  if (active && !active[box]) return;
  const BoxMeta& bm = meta[box];
  const int tid = threadIdx.x, col = tid & 31, slot = tid >> 5;
  double sr = 0.0, sm_ = 0.0, st = 0.0;
  if (col < k) {
    double v = nu[(int64_t)box * k + col];
    int r_begin = chunk * rows_per_chunk;
    int r_end = min(bm.n_dof, r_begin + rows_per_chunk);
    for (int row = r_begin + slot; row < r_end; row += RES_THREADS / 32) {
      int64_t o = (bm.dof_off * k) + (int64_t)row * k + col;
      double r = 0.0;
      if ((rcls >> cls[bm.dof_off + row]) & 1) {
        double mx = MX[o], sx = AX[o];
        double tx = sx + shift * mx;
        r = mx - v * tx;
        sr += r * r;
        sm_ += mx * mx;
        st += tx * tx;
      }
      R[o] = r;
    }
  }
  red[0][tid] = sr;
  red[1][tid] = sm_;
  red[2][tid] = st;
  __syncthreads();
  if (tid < 32) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int s = 0; s < RES_THREADS / 32; ++s) {
      a += red[0][s * 32 + tid];
      b += red[1][s * 32 + tid];
      c += red[2][s * 32 + tid];
    }
    double* out = part + (((int64_t)box * n_chunk + chunk) * 3) * 32;
    out[tid] = a;
    out[32 + tid] = b;
    out[64 + tid] = c;
  }
}

// Per box: rho from the partial sums of this round's pairs (nev = min(nround,
// n_ev - col0) of them, the box's pairs col0 ..).  On the box's last round
// the pairs are converged at rho <= tol.  On a round that later rounds deflate
// against, the target is tol_defl (< tol): an error e in those vectors limits
// the later pairs' residuals to about (nu_earlier / nu_later) |e|; a box that
// meets tol but stalls short of tol_defl (near the rounding floor of its
// images) is retired STALL_ITERS iterations after it met tol (reached[box] =
// that iteration, -1 before).
// A column whose rho is not a finite number (a zero or non-finite
// denominator, or a non-finite residual) sets status bit 8; a box with bit 4
// (a non-positive pivot in its factors) or bit 8 is retired at once as failed,
// so it does not hold the batch loop.  On the last iteration (last != 0) a box
// still active whose pairs miss tol gets bit 1.  Updates active/iters and the
// count of boxes still active; a retired box's xbuf entry records x_id, the
// buffer that holds the current block X (no kernel moves it afterwards).
#define STALL_ITERS 6
__global__ void k_converge(const BoxMeta* __restrict__ meta, int n_box, int k, int n_chunk,
                           const double* __restrict__ part, const double* __restrict__ nu,
                           double tol, double tol_defl, double* __restrict__ rho, int32_t* __restrict__ active,
                           int32_t* __restrict__ iters, int32_t* __restrict__ n_active,
                           int last, int32_t* __restrict__ status, int col0, int nround,
                           const int32_t* __restrict__ it_dev, int32_t* __restrict__ reached, int x_id,
                           int32_t* __restrict__ xbuf) {
  const int it = *it_dev;   // the iteration index (device-side, so a captured graph can advance it)
  // one wavefront per box, lane c < k takes column c (chunks summed in order)
  const int box = blockIdx.x, c = threadIdx.x;
  if (box >= n_box || !active[box]) return;
  const int nev = min(nround, meta[box].n_ev - col0);
  const bool last_round = meta[box].n_ev - col0 <= nround;
  const double tol_eff = last_round ? tol : tol_defl;
  bool ok = true, ok_user = true, fin = true;
  if (c < k) {
    double a = 0.0, b = 0.0, d = 0.0;
    for (int ch = 0; ch < n_chunk; ++ch) {
      const double* p = part + (((int64_t)box * n_chunk + ch) * 3) * 32;
      a += p[c];
      b += p[32 + c];
      d += p[64 + c];
    }
    const double v = nu[(int64_t)box * k + c];
    // |nu|: a Ritz value at rounding level may come out slightly negative
    const double den = sqrt(b) + fabs(v) * sqrt(d);
    // rho is defined for a positive finite denominator only (a zero column, or
    // one with M x = T x = 0, has no eigenvalue)
    const double r = (den > 0.0 && den <= DBL_MAX) ? sqrt(a) / den : __builtin_nan("");
    rho[(int64_t)box * k + c] = r;
    if (c < nev) {
      fin = r <= DBL_MAX;          // false for NaN and inf
      ok = r <= tol_eff;
      ok_user = r <= tol;
    }
  }
  const bool all_ok = __all(ok);
  const bool all_user = __all(ok_user);
  const bool all_fin = __all(fin);
  if (c == 0) {
    int32_t st = status[box];
    if (!all_fin) st |= 8;
    bool retire = false;
    if (st & (4 | 8)) {
      retire = true;             // failed: retired, not converged
    } else if (all_ok) {
      retire = true;
    } else if (all_user && !last_round) {
      if (reached[box] < 0) reached[box] = it;
      retire = it - reached[box] >= STALL_ITERS;
    }
    if (retire) {
      active[box] = 0;
      xbuf[box] = x_id;          // its block X stays in buffer x_id from now on
    } else {
      if (last && !all_user) st |= 1;
      iters[box] += last ? 0 : 1;
      atomicAdd(n_active, 1);
    }
    status[box] = st;
  }
}

// Clears the status bits a local eigensolve sets (1 not converged, 8
// non-finite, 16 threshold) on the boxes it is about to solve (all boxes, or
// those with mask[b] != 0), keeping bit 4 of the assembly.
__global__ void k_status_clear(int n_box, const int32_t* __restrict__ mask, int32_t* __restrict__ status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n_box && (!mask || mask[b])) status[b] &= ~(1 | 8 | 16);
}

// *x += d (the iteration counter of a captured LOBPCG iteration)
__global__ void k_add_i32(int32_t* __restrict__ x, int32_t d) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *x += d;
}

// status[i] |= bits for i < n
__global__ void k_status_or(int32_t* __restrict__ status, int n, int32_t bits) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) status[i] |= bits;
}

// dst[b] = src[b] where mask[b] != 0 (the iteration counts of a masked solve)
__global__ void k_copy_masked_i32(int n, const int32_t* __restrict__ mask, const int32_t* __restrict__ src,
                                  int32_t* __restrict__ dst) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n && mask[b]) dst[b] = src[b];
}

// Soft locking: a column whose residual is below lock_tol gets no new search
// direction (its W and P columns are zeroed, so the Rayleigh-Ritz step drops
// them); it stays in X and keeps being improved by the projection.  Without
// it, the preconditioned residuals of columns converged to rounding level are
// pure noise that corrupts the Gram matrices.  grid (rows, n_box).
__global__ void k_lock(const BoxMeta* __restrict__ meta, int k, const double* __restrict__ rho,
                       double lock_tol, double* __restrict__ W, double* P0, double* P1, double* P2,
                       double* P3, const int32_t* __restrict__ active) {
  int box = blockIdx.y;
  if (active && !active[box]) return;
  const BoxMeta& bm = meta[box];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)bm.n_dof * k) return;
  int c = (int)(t % k);
  if (!(rho[(int64_t)box * k + c] <= lock_tol)) return;
  int64_t o = bm.dof_off * k + t;
  W[o] = 0.0;
  if (P0) P0[o] = 0.0;
  if (P1) P1[o] = 0.0;
  if (P2) P2[o] = 0.0;
  if (P3) P3[o] = 0.0;
}

// random start block on the classes in vcls (counter-based hash, uniform in [-1, 1)), zero elsewhere
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_random_start(const BoxMeta* __restrict__ meta, const uint8_t* __restrict__ cls,
                               int k, int vcls, uint64_t seed, double* __restrict__ X) {
  int box = blockIdx.y;
  const BoxMeta& bm = meta[box];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)bm.n_dof * k) return;
  int row = (int)(t / k), col = (int)(t % k);
  double v = 0.0;
  if ((vcls >> cls[bm.dof_off + row]) & 1) {
    uint64_t h = mix64(seed ^ mix64(((uint64_t)bm.sd << 40) ^ ((uint64_t)row << 8) ^ (uint64_t)col));
    v = (double)(h >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  }
  X[(bm.dof_off * k) + t] = v;
}

// copy a caller start block (values on the classes in vcls, box layout [n_dof][k]) into X
__global__ void k_copy_start(const BoxMeta* __restrict__ meta, const uint8_t* __restrict__ cls,
                             int k, int vcls, const double* __restrict__ X0, double* __restrict__ X) {
  int box = blockIdx.y;
  const BoxMeta& bm = meta[box];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)bm.n_dof * k) return;
  int row = (int)(t / k);
  X[(bm.dof_off * k) + t] = ((vcls >> cls[bm.dof_off + row]) & 1) ? X0[(bm.dof_off * k) + t] : 0.0;
}

// Output: lambda ascending, unit 2-norm eigenvectors on all box DoFs (0 on B3)
// with the entry of largest magnitude positive, rho per pair.  One workgroup per box.
#define OUT_THREADS 1024   // k_output: 32 columns x 32 row slots

__global__ __launch_bounds__(OUT_THREADS) void k_output(const BoxMeta* __restrict__ meta, int k,
                                                double shift, XLoc xl,
                                                const double* __restrict__ nu,
                                                const double* __restrict__ rho,
                                                double* __restrict__ evals,
                                                double* __restrict__ evecs,
                                                double* __restrict__ resid,
                                                const int32_t* __restrict__ mask, int col0, int nround) {
  __shared__ double sn[OUT_THREADS];
  __shared__ double sa[OUT_THREADS];
  __shared__ int si[OUT_THREADS];
  __shared__ double scale[32];
  int box = blockIdx.x;
  if (mask && !mask[box]) return;   // a box the caller did not select keeps its output
  const BoxMeta& bm = meta[box];
  const double* __restrict__ X = xl.at(0, box);
  const int tid = threadIdx.x, col = tid & 31, slot = tid >> 5;
  // this round writes pairs col0 .. col0 + nev - 1 of the box (columns of X
  // 0 .. nev - 1); the rows of evecs hold all n_ev pairs
  const int nev = min(nround, bm.n_ev - col0);
  if (nev <= 0) return;
  const int ld = bm.n_ev;
  double s2 = 0.0, amax = -1.0;
  int imax = 0x7fffffff;
  if (col < nev) {
    for (int row = slot; row < bm.n_dof; row += OUT_THREADS / 32) {
      double v = X[(bm.dof_off * k) + (int64_t)row * k + col];
      s2 += v * v;
      double a = fabs(v);
      if (a > amax) { amax = a; imax = row; }
    }
  }
  sn[tid] = s2;
  sa[tid] = amax;
  si[tid] = imax;
  __syncthreads();
  if (tid < 32 && col < nev) {
    double n2 = 0.0, am = -1.0;
    int im = 0x7fffffff;
    for (int s = 0; s < OUT_THREADS / 32; ++s) {
      n2 += sn[s * 32 + tid];
      double a = sa[s * 32 + tid];
      int ii = si[s * 32 + tid];
      if (a > am || (a == am && ii < im)) { am = a; im = ii; }
    }
    if (im < 0 || im >= bm.n_dof) im = 0;   // all-NaN column: keep the read in bounds
    double v = X[(bm.dof_off * k) + (int64_t)im * k + tid];
    double sg = (v < 0.0) ? -1.0 : 1.0;
    scale[tid] = sg / sqrt(n2);
    double nv = nu[(int64_t)box * k + tid];
    evals[bm.eval_off + col0 + tid] = 1.0 / nv - shift;
    resid[bm.eval_off + col0 + tid] = rho[(int64_t)box * k + tid];
  }
  __syncthreads();
  for (int64_t t = tid; t < (int64_t)bm.n_dof * nev; t += OUT_THREADS) {
    int row = (int)(t / nev), c = (int)(t % nev);
    evecs[bm.evec_off + (int64_t)row * ld + col0 + c] = X[(bm.dof_off * k) + (int64_t)row * k + c] * scale[c];
  }
}

// X <- X on the DoFs whose class bit is set in classes, 0 elsewhere
// (flat over all boxes' [n_dof][k] blocks)
__global__ void k_keep_classes(const uint8_t* __restrict__ cls, int classes, int k, int64_t n,
                               double* __restrict__ X) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    if (!((classes >> cls[e / k]) & 1)) X[e] = 0.0;
}

}  // namespace msg
