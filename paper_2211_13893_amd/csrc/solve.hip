// Block triangular solves with the banded box factors A = Lu D Lu^T
// (factorised by band.hip), reading the solve-ordered band copies.
#include "band_view.hpp"

namespace msg {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Block solve A x = f with A = Lu D Lu^T for KC columns [chunk*KC, +KC) of a
// box block vector.  Reads `in` (box layout [n_dof][ldk]) on the matrix's
// DoFs, writes `out` on the DoFs whose class bit is set in out_classes (bit c
// for class c); with zero_rest, every other DoF of the box gets 0 in these
// columns.  Scratch holds w = D^{-1} y of the forward sweep, NT*32*KC doubles
// per (box, chunk), and one more row (index NT) that takes stores without a
// target; scratch_stride >= (NT + 1)*32*KC.
//
// Forward sweep  y_I = f_I - sum_s Lu(I,I-s) y_{I-s}; backward sweep
// x_I = w_I - sum_s Lu(I+s,I)^T x_{I+s}.  A step's work items are
// (band tile s, row quad, half of the inner index): thread t handles tile
// s = 1 + 32p + (t >> 4) of tile set p (NS sets, bands up to 32*NS + 1
// tiles), rows 4*((t >> 1) & 7) .. +3 and inner indices 16*(t & 1) .. +15,
// for all KC columns, so every solution row read from the LDS ring feeds four
// factor rows.  The partial sums of a wavefront's 4 tile groups and 2 halves
// are combined in registers by a reduce-scatter over lane ^ 1 (DPP), lane ^ 16
// and lane ^ 32 (permlane swaps), leaving 4 of the 32 x KC sums per lane; the
// 8 wavefronts' sums go through LDS and are added in a fixed order by the
// first 32*KC threads.  The product w = D^{-1} y of the previous forward step
// is formed by the last two wavefronts.
//
// Latency: the factor fragment of the next tile set or step is requested
// piece by piece while the current one is used, so the loads stream during
// the arithmetic, and stays in flight across the LDS-only barriers while the
// step is reduced.  For the compiler to wait for each global load only where
// its own value is needed, every global load and store of a step is issued by
// every thread of a wavefront that holds tiles, unconditionally and in the
// same order: out-of-range work items read a valid address and discard the
// value, and stores without a target write the spare scratch row.
//
// A matrix split by a separator layer (BoxMeta.nd) is solved in three
// launches over the block A = [A_00 . A_0s; . A_11 A_1s; A_s0 A_s1 A_ss]:
//   phase 1, per chain c: y_c = Lu_cc^{-1} f_c and, continuing over the
//            chain's separator rows, t_c = -Lu_sc y_c (the chain's band with
//            zero tiles in its separator columns), w_c = D_c^{-1} y_c;
//   phase 2, per box: the separator block S = Lu_ss D_s Lu_ss^T on
//            f_s + t_0 + t_1 (forward, D^{-1}, backward) gives x_s;
//   phase 3, per chain: x_c = Lu_cc^{-T} (w_c - Lu_sc^T x_s), the backward
//            sweep from the chain's last row with x_s in the ring.
// The two chains of a box are independent work units, so each box streams
// its factor on two CUs at once, each over half of the rows.  A whole band
// takes phases 1 and 3 as one chain (or phase 0, both sweeps in one launch,
// when no box of the plan is split).
//
// The column chunks of one box share an XCD (block id mod 8) so the factor
// they stream is read from HBM once and then hit in that XCD's L2.  With an
// order array (box indices by decreasing sweep length) the longest sweeps are
// dispatched first, so on a batch of unequal boxes that needs more than one
// wave of workgroups the largest boxes do not start last.
// grid.x = 8 * n_chunk * ceil(n_unit/8) (n_unit = 2 n_box in phases 1 and 3,
// n_box otherwise), 512 threads; dynamic LDS = BT*32*KC doubles.  Scratch:
// w of unit (box, chain) at (2 box + chain) * n_chunk + chunk; the separator
// exchange of (box, chunk) at sep + (box * n_chunk + chunk) * 4 sep_q: t_0,
// t_1, w of S and x_s, sep_q doubles each ((NTs + 1) * 32 * KC).
#define SOLVE_THREADS 512
#define SOLVE_WAVES (SOLVE_THREADS / 64)
// Barrier for LDS traffic only (__syncthreads would also wait for every
// global load).  Inside the sweeps no thread reads global memory that
// another thread of the block wrote, so they need no global-memory barrier.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// value of the partner lane (lane ^ 1) through a DPP quad permutation
__device__ inline double dpp_xor1(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// a + a(lane ^ 16) on lanes with bit 4 clear, b + b(lane ^ 16) on the others
__device__ inline double swap16_sum(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
// a + a(lane ^ 32) on lanes 0..31, b + b(lane ^ 32) on lanes 32..63
__device__ inline double swap32_sum(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// f[i][q]: forward  = Lu[4rq+i][16h+q] of tile (I, I-s);
//          backward = Lu[16h+q][4rq+i] of tile (I+s, I)  (row i of its transpose)
// read from the solve-ordered copy (fw or bw) of the band; consecutive
// threads read consecutive 16-byte pieces.  P points at piece 0 of this
// thread's slot of one (row, set); piece j is at P + j*nthr.
template <typename T> struct vec2_of;
template <> struct vec2_of<double> { typedef double2 type; };
template <> struct vec2_of<float> { typedef float2 type; };

template <typename T>
__device__ inline void frag_load(const typename vec2_of<T>::type* __restrict__ P, int nthr, int dir,
                                 double (&f)[4][16]) {
  if (dir < 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const auto a = P[(int64_t)(8 * i + q) * nthr];
        f[i][2 * q] = a.x;
        f[i][2 * q + 1] = a.y;
      }
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const auto a = P[(int64_t)(2 * q) * nthr];
      const auto b = P[(int64_t)(2 * q + 1) * nthr];
      f[0][q] = a.x;
      f[1][q] = a.y;
      f[2][q] = b.x;
      f[3][q] = b.y;
    }
  }
}

// T: precision of the factor copies read by the sweeps (double, or float in
// the mixed path; ft = the factor array in that precision, same offsets as
// fac).  Arithmetic, right-hand sides and solutions are FP64 in both cases.
template <int KC, int NS, typename T>
__global__ __launch_bounds__(SOLVE_THREADS) void k_band_solve(
    const BoxMeta* __restrict__ meta, int n_box, int n_chunk, int kind,
    const T* __restrict__ ft, const uint8_t* __restrict__ cls,
    const double* in, double* out,
    int ldk, int out_classes, int zero_rest, double* __restrict__ scratch, int64_t scratch_stride,
    const int32_t* __restrict__ active, int phase, double* __restrict__ sep, int64_t sep_q,
    const int32_t* __restrict__ order) {
  static_assert(32 * KC == 256, "reduction threads = the first 256, w threads = the last 128");
  static_assert(KC == 8, "the register reduce-scatter splits 8 columns over 4 tile groups");
  static_assert(SOLVE_THREADS / 16 == SOLVE_TILES, "one tile group of 16 threads per tile of a set");
  extern __shared__ double ring[];   // [BT][32][KC]
  __shared__ double part[SOLVE_WAVES][32][KC + 1];
  __shared__ double Dl[32][33];      // D^{-1} tile of the current forward step
  __shared__ double Wl[32 * KC];     // w of the previous forward step
  const int x = blockIdx.x;
  const int xcd = x & 7, rest = x >> 3;
  const int chunk = rest % n_chunk;
  const int nun = (phase == 1 || phase == 3) ? 2 : 1;
  const int unit = (rest / n_chunk) * 8 + xcd;
  const int bslot = unit / nun, chain = unit - bslot * nun;
  if (bslot >= n_box) return;
  const int box = order ? order[bslot] : bslot;   // boxes with the longest sweeps first
  if (active && !active[box]) return;
  const BoxMeta& bm = meta[box];
  const bool split = bm.nd[kind] != 0;
  if ((phase == 2 && !split) || (chain == 1 && !split)) return;
  BandView v = band_view(bm, kind, phase == 2 ? 2 : chain);
  const uint8_t* cl = cls + bm.dof_off;
  const int tid = threadIdx.x;
  const int h = tid & 1, rq = (tid >> 1) & 7, sg = tid >> 4;  // item of the thread
  const int g = sg & 3, wave = tid >> 6;                      // tile group inside the wavefront
  const bool red = tid < 32 * KC;
  const int t8 = tid & (32 * KC - 1);                         // reduction slot (duplicated above 256)
  const int rr = t8 / KC, cc = t8 % KC;
  const int col = chunk * KC + cc;
  const bool colok = col < ldk;
  const int colc = colok ? col : ldk - 1;
  const bool wthr = tid >= SOLVE_THREADS - 128;               // forms w = D^{-1} y
  const double* vin = in + bm.dof_off * ldk;
  double* vout = out + bm.dof_off * ldk;
  double* sb = split ? sep + ((int64_t)box * n_chunk + chunk) * 4 * sep_q : nullptr;
  double* w = phase == 2 ? sb + 2 * sep_q : scratch + ((int64_t)(2 * box + chain) * n_chunk + chunk) * scratch_stride;
  const int BT = v.BT, NT = v.NT, NF = v.NTf;
  const bool do_fwd = phase <= 2, do_bwd = phase != 1;
  const int nthr = solve_nthr(BT);
  const int nsets = NS == 1 ? 1 : solve_sets(BT);
  const int tc = nthr ? min(tid, nthr - 1) : 0;
  // wavefronts that hold band tiles (in set 0, which is full when set 1 is used)
  const bool wave_tiles = __builtin_amdgcn_readfirstlane(tid) < nthr;
  typedef typename vec2_of<T>::type V2;
  const V2* Ffw = nthr ? (const V2*)(ft + v.fw) + tc : (const V2*)(ft + v.off);
  const V2* Fbw = nthr ? (const V2*)(ft + v.bw) + tc : (const V2*)(ft + v.off);
  auto slot = [&](const V2* F, int I, int p) { return F + (int64_t)(I * nsets + p) * 32 * nthr; };
  double f[4][16];

  // partial sums of this thread's item over its half of the inner index,
  // with the next fragment (Fn) requested piece by piece as the current
  // pieces are used (the loads are issued whether or not the thread has a
  // tile, so every step issues the same loads)
  auto accumulate = [&](bool has, const double* yp, double (&acc)[4][KC], const V2* Fn, int dir) {
    if (!wave_tiles) return;
#pragma unroll
    for (int qq = 0; qq < 8; ++qq) {
      if (has) {
#pragma unroll
        for (int q = 2 * qq; q < 2 * qq + 2; ++q) {
          const double* y0 = yp + (16 * h + q) * KC;
#pragma unroll
          for (int c = 0; c < KC; ++c) {
            const double a = y0[c];
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i][c] += f[i][q] * a;
          }
        }
      }
      if (dir < 0) {
        // pieces 8i + qq hold f[i][2qq], f[i][2qq+1]
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const V2 a = Fn[(int64_t)(8 * i + qq) * nthr];
          f[i][2 * qq] = a.x;
          f[i][2 * qq + 1] = a.y;
        }
      } else {
        // pieces 2q, 2q+1 hold f[0..3][q]
#pragma unroll
        for (int q = 2 * qq; q < 2 * qq + 2; ++q) {
          const V2 a = Fn[(int64_t)(2 * q) * nthr];
          const V2 b = Fn[(int64_t)(2 * q + 1) * nthr];
          f[0][q] = a.x;
          f[1][q] = a.y;
          f[2][q] = b.x;
          f[3][q] = b.y;
        }
      }
    }
  };
  // reduce-scatter of the wavefront's partial sums: after the three exchanges
  // lane (g, rq, h) holds the wavefront total of rows 4rq+2h+i2 (i2 = 0, 1)
  // and columns c + 2(g>>1) + 4(g&1) (c = 0, 1); every slot is written each step
  auto store_part = [&](double (&acc)[4][KC]) {
    double v1[2][KC];
#pragma unroll
    for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const double keep = h ? acc[2 + i2][c] : acc[i2][c];
        const double send = h ? acc[i2][c] : acc[2 + i2][c];
        v1[i2][c] = keep + dpp_xor1(send);
      }
    double v2[2][4];
#pragma unroll
    for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
      for (int c = 0; c < 4; ++c) v2[i2][c] = swap16_sum(v1[i2][c], v1[i2][c + 4]);
#pragma unroll
    for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        part[wave][4 * rq + 2 * h + i2][c + 2 * (g >> 1) + 4 * (g & 1)] = swap32_sum(v2[i2][c], v2[i2][c + 2]);
  };
  // sum over the wavefronts in a fixed order
  auto part_sum = [&]() {
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int q = 0; q < SOLVE_WAVES; q += 2) {
      a0 += part[q][rr][cc];
      a1 += part[q + 1][rr][cc];
    }
    return a0 + a1;
  };
  // Wl = D^{-1}_J y_J (D^{-1}_J in Dl, y_J in its ring slot), by the w threads
  auto form_w = [&](int J) {
    const int u = tid - (SOLVE_THREADS - 128);
    const double* yp = ring + (int64_t)(J % BT) * 32 * KC;
#pragma unroll
    for (int o = u; o < 32 * KC; o += 128) {
      const int r = o / KC, c = o % KC;
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int q = 0; q < 32; q += 2) {
        a0 += Dl[r][q] * yp[q * KC + c];
        a1 += Dl[r][q + 1] * yp[(q + 1) * KC + c];
      }
      Wl[o] = a0 + a1;
    }
  };
  auto zero_acc = [&](double (&acc)[4][KC]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < KC; ++c) acc[i][c] = 0.0;
  };

  // ---- forward: Lu y = f
  if (do_fwd) {
  if (wave_tiles) frag_load<T>(slot(Ffw, 0, 0), nthr, -1, f);
  for (int I = 0; I < NT; ++I) {
    const int smax = min(BT - 1, I);
    // right-hand side and D^{-1} tile of this step (used after the first
    // barrier; the class byte is tested there too, so no wait is forced here)
    const int dof = band_to_dof(v, bm, I * 32 + rr);
    const int dofc = dof >= 0 ? dof : 0;
    const double fraw = vin[(int64_t)dofc * ldk + colc];
    const uint8_t cb = cl[dofc];
    const V2* dp = (const V2*)(ft + v.doff + (int64_t)I * v.dstride) + 2 * t8;
    const V2 da = dp[0], db = dp[1];
    // w_{I-1} (Dl and its ring slot were completed last step)
    if (wthr && I >= 1) form_w(I - 1);
    double acc[4][KC];
    zero_acc(acc);
    const int In = min(I + 1, NT - 1);
    const int s0 = 1 + sg;
    const bool has0 = s0 <= smax;
    const bool two = NS == 2 && nsets == 2;
    accumulate(has0, ring + (int64_t)((has0 ? I - s0 : 0) % BT) * 32 * KC, acc,
               two ? slot(Ffw, I, 1) : slot(Ffw, In, 0), -1);
    if (two) {
      const int s1 = 1 + SOLVE_TILES + sg;
      const bool has1 = s1 <= smax;
      accumulate(has1, ring + (int64_t)((has1 ? I - s1 : 0) % BT) * 32 * KC, acc, slot(Ffw, In, 0), -1);
    }
    store_part(acc);
    lds_barrier();
    w[(int64_t)((I >= 1 ? I - 1 : NT) * 32 + rr) * KC + cc] = Wl[t8];
    if (red) {
      const int e = 4 * tid;
      Dl[e >> 5][e & 31] = da.x;
      Dl[(e + 1) >> 5][(e + 1) & 31] = da.y;
      Dl[(e + 2) >> 5][(e + 2) & 31] = db.x;
      Dl[(e + 3) >> 5][(e + 3) & 31] = db.y;
      // a chain's separator rows (I >= NF) collect t_c = -Lu_sc y_c; S adds both
      const bool fok = (dof >= 0) & colok & dof_active(kind, cb) & (I < NF);
      double rhs = fok ? fraw : 0.0;
      if (phase == 2) {
        const int64_t o = (int64_t)(I * 32 + rr) * KC + cc;
        rhs += sb[o] + sb[sep_q + o];
      }
      const double yv = rhs - part_sum();
      ring[(int64_t)(I % BT) * 32 * KC + rr * KC + cc] = yv;
      if (phase == 1 && I >= NF) sb[chain * sep_q + (int64_t)((I - NF) * 32 + rr) * KC + cc] = yv;
    }
    lds_barrier();
  }
  if (wthr) form_w(NT - 1);
  lds_barrier();
  w[(int64_t)((NT - 1) * 32 + rr) * KC + cc] = Wl[t8];
  __syncthreads();
  }
  if (!do_bwd) return;

  // ---- backward: Lu^T x = w, from the last own row (a chain: with x_s of
  // the separator rows in the ring)
  if (phase == 3 && split) {
    if (red)
      for (int i = 0; i < NT - NF; ++i)
        ring[(int64_t)((NF + i) % BT) * 32 * KC + rr * KC + cc] = sb[3 * sep_q + (int64_t)(i * 32 + rr) * KC + cc];
    __syncthreads();
  }
  if (wave_tiles) frag_load<T>(slot(Fbw, NF - 1, 0), nthr, +1, f);
  for (int I = NF - 1; I >= 0; --I) {
    const int smax = min(BT - 1, NT - 1 - I);
    const int row = I * 32 + rr;
    const double fv = w[(int64_t)row * KC + cc];
    const int dof = band_to_dof(v, bm, row);
    const uint8_t cb = cl[dof >= 0 ? dof : 0];
    double acc[4][KC];
    zero_acc(acc);
    const int In = max(I - 1, 0);
    const int s0 = 1 + sg;
    const bool has0 = s0 <= smax;
    const bool two = NS == 2 && nsets == 2;
    accumulate(has0, ring + (int64_t)((has0 ? I + s0 : 0) % BT) * 32 * KC, acc,
               two ? slot(Fbw, I, 1) : slot(Fbw, In, 0), +1);
    if (two) {
      const int s1 = 1 + SOLVE_TILES + sg;
      const bool has1 = s1 <= smax;
      accumulate(has1, ring + (int64_t)((has1 ? I + s1 : 0) % BT) * 32 * KC, acc, slot(Fbw, In, 0), +1);
    }
    store_part(acc);
    lds_barrier();
    double xv = 0.0;
    if (red) {
      xv = fv - part_sum();
      ring[(int64_t)(I % BT) * 32 * KC + rr * KC + cc] = xv;
      if (phase == 2) sb[3 * sep_q + (int64_t)(I * 32 + rr) * KC + cc] = xv;
    }
    // the solution goes to `out` where it belongs, else to the spare row
    const bool wr = red & (dof >= 0) & colok & dof_active(kind, cb) & (((out_classes >> cb) & 1) != 0);
    *(wr ? vout + (int64_t)dof * ldk + col : w + (int64_t)(NT * 32 + rr) * KC + cc) = xv;
    lds_barrier();
  }
  if (zero_rest && colok && red && (phase == 0 || (phase == 3 && chain == 0))) {
    // zero the DoFs of this box (this chunk's columns) that were not written
    for (int d = rr; d < bm.n_dof; d += 32) {
      uint8_t k = cl[d];
      bool written = dof_active(kind, k) && ((out_classes >> k) & 1);
      if (!written) vout[(int64_t)d * ldk + col] = 0.0;
    }
  }
}

#define SOLVE_INST(NS, T)                                                                                     \
  template __global__ void k_band_solve<8, NS, T>(const BoxMeta*, int, int, int, const T*, const uint8_t*,   \
                                                  const double*, double*, int, int, int, double*, int64_t,     \
                                                  const int32_t*, int, double*, int64_t, const int32_t*);
SOLVE_INST(1, double)
SOLVE_INST(2, double)
SOLVE_INST(1, float)
SOLVE_INST(2, float)


// The same block solve on the FP64 matrix cores, for bands of at most
// 1 + 8 NSLOT tiles (NSLOT = 8: two sets of four slots, each wavefront
// streaming the second set's pieces of a row while it multiplies the first
// set, and the first set's pieces of the next row during the second) (k_band_relayout4 writes the operand copies).  One step
// y_I = f_I - sum_s Lu(I,I-s) y_{I-s} (backward: x_I = w_I - sum_s
// Lu(I+s,I)^T x_{I+s}) is a 32 x 8 block product per tile, done as
// v_mfma_f64_4x4x4f64: lane l = 16 kk + 4 o + i supplies A[16 rh + 4 o + i][4 ss + kk]
// (the factor, streamed from the copy) and B[4 ss + kk][4 ch + j] (j = l & 3,
// the solution row from the LDS ring), and accumulates C[16 rh + 4 o + i][4 ch + j]
// at lane 16 i + 4 o + j, four 4x4 blocks o per instruction, 8 instructions
// (ss) per (rh, ch) and tile.  Wavefront w takes tiles s = 1 + w + 8u,
// s <= BT-1 (a wavefront skips its slots past the band: loads and products);
// all tiles of a wavefront add into the same 4 accumulators, so
// the wavefront's partial sum of the step leaves in 4 LDS stores.  The
// wavefront of 4x4x4 products is FP64-FMA work that the matrix cores run at
// close to their rate with two wavefronts per SIMD (the vector unit does not),
// and a ring value read from LDS feeds four factor rows.  Wavefront 7 also
// forms w_{I-1} = D^{-1}_{I-1} y_{I-1} (slot 0 of the forward copy) and
// stores it.  The factor pieces of the next row are requested one by one as
// the current ones are used.  The ring is cleared before each sweep, so rows outside
// the matrix read zeros.  Scratch as for k_band_solve.
// grid.x = 8 * n_chunk * ceil(n_box/8), 512 threads; dynamic LDS = BT*32*KC doubles.
template <bool WIDE> struct McAcc;
template <> struct McAcc<false> { double a[2][2]; };   // 4x4x4: (row half, column half)
template <> struct McAcc<true> { dbl4 a[2]; };         // 16x16x4: row half
template <int NSLOT, bool WIDE, typename T>
__global__ __launch_bounds__(SOLVE_THREADS) void k_band_solve4(
    const BoxMeta* __restrict__ meta, int n_box, int n_chunk, int kind,
    const T* __restrict__ ft, const uint8_t* __restrict__ cls,
    const double* in, double* out,
    int ldk, int out_classes, int zero_rest, double* __restrict__ scratch, int64_t scratch_stride,
    const int32_t* __restrict__ active, int phase, double* __restrict__ sep, int64_t sep_q,
    const int32_t* __restrict__ order) {
  constexpr int KC = WIDE ? 16 : 8;
  // NSLOT 8: two sets of four register slots (tiles 1 + w + 8u, then 33 + w + 8u)
  constexpr bool TWOSET = NSLOT > 5;
  constexpr int NR = TWOSET ? 4 : NSLOT;
  static_assert(!TWOSET || (NSLOT == 8 && !WIDE), "two sets: 8 slots, 8 columns (the LDS ring of 65 rows)");
  static_assert(SOLVE_THREADS == 512, "8 wavefronts: tiles 1 + w + 8u");
  static_assert(32 * KC <= SOLVE_THREADS, "one reduction thread per entry of a 32 x KC step");
  extern __shared__ double ring[];   // [BT][32][KC]
  __shared__ double part[SOLVE_WAVES][32][KC + 1];
  const int x = blockIdx.x;
  const int xcd = x & 7, rest = x >> 3;
  const int chunk = rest % n_chunk;
  const int nun = (phase == 1 || phase == 3) ? 2 : 1;
  const int unit = (rest / n_chunk) * 8 + xcd;
  const int bslot = unit / nun, chain = unit - bslot * nun;
  if (bslot >= n_box) return;
  const int box = order ? order[bslot] : bslot;   // boxes with the longest sweeps first
  if (active && !active[box]) return;
  const BoxMeta& bm = meta[box];
  const bool split = bm.nd[kind] != 0;
  if ((phase == 2 && !split) || (chain == 1 && !split)) return;
  BandView v = band_view(bm, kind, phase == 2 ? 2 : chain);
  const uint8_t* cl = cls + bm.dof_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kk = lane >> 4, ob = (lane >> 2) & 3, jl = lane & 3;   // operand roles of the lane (4x4x4)
  const int oi = lane >> 4;                                        // accumulator row i of the lane
  const int li = lane & 15;                                        // 16x16x4: row / column, inner index kk
  const bool red = tid < 32 * KC;
  const int t8 = tid & (32 * KC - 1);
  const int rr = t8 / KC, cc = t8 % KC;
  const int col = chunk * KC + cc;
  const bool colok = col < ldk;
  const int colc = colok ? col : ldk - 1;
  const double* vin = in + bm.dof_off * ldk;
  double* vout = out + bm.dof_off * ldk;
  double* sb = split ? sep + ((int64_t)box * n_chunk + chunk) * 4 * sep_q : nullptr;
  double* w = phase == 2 ? sb + 2 * sep_q : scratch + ((int64_t)(2 * box + chain) * n_chunk + chunk) * scratch_stride;
  const int BT = v.BT, NT = v.NT, NF = v.NTf;
  const bool do_fwd = phase <= 2, do_bwd = phase != 1;
  const int S = solve4_slots(BT);
  typedef typename vec2_of<T>::type V2;
  // piece pair pp of slot `sl` of row I, this lane
  auto piece = [&](const T* base, int I, int sl, int pp) {
    return (const V2*)(base) + (((int64_t)I * S + sl) * 8 + pp) * 64 + lane;
  };
  const T* Ffw = ft + v.fw;
  const T* Fbw = ft + v.bw;
  const bool wforms = wave == SOLVE_WAVES - 1;
  // factor pieces of this wavefront's slots (and of D^{-1} for wavefront 7)
  double A[NR][16], Aw[16];
  auto load_slot = [&](double (&a)[16], const T* base, int I, int sl) {
#pragma unroll
    for (int pp = 0; pp < 8; ++pp) {
      const V2 t = *piece(base, I, sl, pp);
      a[2 * pp] = (double)t.x;
      a[2 * pp + 1] = (double)t.y;
    }
  };
  // acc += the tile's 32 x KC product with the ring row yp; the next row's
  // pieces of the slot are requested as the current ones are used.  4x4x4:
  // per inner step ss the two ring values of the lane feed both row halves,
  // so the four accumulators are updated in turn (independent MFMA chains);
  // 16x16x4: one ring value per step feeds both row halves (two chains).
  auto tile_step = [&](double (&a)[16], const double* yp, McAcc<WIDE>& acc, const T* base, int In, int sl) {
#pragma unroll
    for (int ss2 = 0; ss2 < 4; ++ss2) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int ss = 2 * ss2 + e;
        if constexpr (WIDE) {
          const double bv = yp[(4 * ss + kk) * KC + li];
#pragma unroll
          for (int rh = 0; rh < 2; ++rh)
            acc.a[rh] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2 * (4 * rh + ss2) + e], bv, acc.a[rh], 0, 0, 0);
        } else {
          const double b0 = yp[(4 * ss + kk) * KC + jl];
          const double b1 = yp[(4 * ss + kk) * KC + 4 + jl];
#pragma unroll
          for (int rh = 0; rh < 2; ++rh) {
            const double av = a[2 * (4 * rh + ss2) + e];
            acc.a[rh][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, b0, acc.a[rh][0], 0, 0, 0);
            acc.a[rh][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, b1, acc.a[rh][1], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int rh = 0; rh < 2; ++rh) {
        const int pp = 4 * rh + ss2;
        const V2 t = *piece(base, In, sl, pp);
        a[2 * pp] = (double)t.x;
        a[2 * pp + 1] = (double)t.y;
      }
    }
  };
  auto zero_acc = [&](McAcc<WIDE>& acc) {
    if constexpr (WIDE) {
      acc.a[0] = dbl4{0.0, 0.0, 0.0, 0.0};
      acc.a[1] = dbl4{0.0, 0.0, 0.0, 0.0};
    } else {
      acc.a[0][0] = acc.a[0][1] = acc.a[1][0] = acc.a[1][1] = 0.0;
    }
  };
  auto store_part = [&](const McAcc<WIDE>& acc) {
    if constexpr (WIDE) {
#pragma unroll
      for (int rh = 0; rh < 2; ++rh)
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4) part[wave][16 * rh + kk + 4 * v4][li] = acc.a[rh][v4];
    } else {
#pragma unroll
      for (int rh = 0; rh < 2; ++rh)
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) part[wave][16 * rh + 4 * ob + oi][4 * ch + jl] = acc.a[rh][ch];
    }
  };
  auto part_sum = [&]() {
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int q = 0; q < SOLVE_WAVES; q += 2) {
      a0 += part[q][rr][cc];
      a1 += part[q + 1][rr][cc];
    }
    return a0 + a1;
  };
  auto clear_ring = [&]() {
    for (int e = tid; e < BT * 32 * KC; e += SOLVE_THREADS) ring[e] = 0.0;
  };
  // w_J = D^{-1}_J y_J by wavefront 7 into row `dst` of the scratch (the spare row NT when J < 0)
  auto form_w = [&](int J, int dst) {
    const double* yp = ring + (int64_t)((J < 0 ? 0 : J) % BT) * 32 * KC;
    if constexpr (WIDE) {
      dbl4 accw[2] = {dbl4{0.0, 0.0, 0.0, 0.0}, dbl4{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
      for (int ss = 0; ss < 8; ++ss) {
        const double bv = yp[(4 * ss + kk) * KC + li];
#pragma unroll
        for (int rh = 0; rh < 2; ++rh)
          accw[rh] = __builtin_amdgcn_mfma_f64_16x16x4f64(Aw[2 * (4 * rh + (ss >> 1)) + (ss & 1)], bv, accw[rh], 0, 0, 0);
      }
#pragma unroll
      for (int rh = 0; rh < 2; ++rh)
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4) w[(int64_t)(dst * 32 + 16 * rh + kk + 4 * v4) * KC + li] = accw[rh][v4];
    } else {
      double accw[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
      for (int ss = 0; ss < 8; ++ss) {
        const double b0 = yp[(4 * ss + kk) * KC + jl];
        const double b1 = yp[(4 * ss + kk) * KC + 4 + jl];
#pragma unroll
        for (int rh = 0; rh < 2; ++rh) {
          const double av = Aw[2 * (4 * rh + (ss >> 1)) + (ss & 1)];
          accw[rh][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, b0, accw[rh][0], 0, 0, 0);
          accw[rh][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, b1, accw[rh][1], 0, 0, 0);
        }
      }
#pragma unroll
      for (int rh = 0; rh < 2; ++rh)
#pragma unroll
        for (int ch = 0; ch < 2; ++ch)
          w[(int64_t)(dst * 32 + 16 * rh + 4 * ob + oi) * KC + 4 * ch + jl] = accw[rh][ch];
    }
  };

  // ---- forward: Lu y = f
  if (do_fwd) {
  clear_ring();
#pragma unroll
  for (int u = 0; u < NR; ++u)
    if (1 + wave + 8 * u <= BT - 1) load_slot(A[u], Ffw, 0, 1 + wave + 8 * u);
  if (wforms) load_slot(Aw, Ffw, 0, 0);
  lds_barrier();
  for (int I = 0; I < NT; ++I) {
    const int dof = band_to_dof(v, bm, I * 32 + rr);
    const int dofc = dof >= 0 ? dof : 0;
    const double fraw = vin[(int64_t)dofc * ldk + colc];
    const uint8_t cb = cl[dofc];
    const int In = min(I + 1, NT - 1);
    McAcc<WIDE> acc;
    zero_acc(acc);
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int s = 1 + wave + 8 * u;
      // row I-s (zero before row 0); tiles past the band are skipped (wave-uniform)
      const double* yp = ring + (int64_t)(((I - s) % BT + BT) % BT) * 32 * KC;
      if (s <= BT - 1) {
        // two sets: the first streams the second set's pieces of row I (when
        // the wavefront has that slot), the second the first set's of row In
        const bool has1 = TWOSET && s + 32 <= BT - 1;
        tile_step(A[u], yp, acc, Ffw, has1 ? I : In, has1 ? s + 32 : s);
      }
    }
    if constexpr (TWOSET) {
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int s = 33 + wave + 8 * u;
        const double* yp = ring + (int64_t)(((I - s) % BT + BT) % BT) * 32 * KC;
        if (s <= BT - 1) tile_step(A[u], yp, acc, Ffw, In, s - 32);
      }
    }
    store_part(acc);
    // w_{I-1} (its ring row was completed last step); D^{-1} of row I next
    if (wforms) {
      form_w(I - 1, I >= 1 ? I - 1 : NT);
      load_slot(Aw, Ffw, I, 0);
    }
    lds_barrier();
    if (red) {
      // a chain's separator rows (I >= NF) collect t_c = -Lu_sc y_c; S adds both
      const bool fok = (dof >= 0) & colok & dof_active(kind, cb) & (I < NF);
      double rhs = fok ? fraw : 0.0;
      if (phase == 2) {
        const int64_t o = (int64_t)(I * 32 + rr) * KC + cc;
        rhs += sb[o] + sb[sep_q + o];
      }
      const double yv = rhs - part_sum();
      ring[(int64_t)(I % BT) * 32 * KC + rr * KC + cc] = yv;
      if (phase == 1 && I >= NF) sb[chain * sep_q + (int64_t)((I - NF) * 32 + rr) * KC + cc] = yv;
    }
    lds_barrier();
  }
  if (wforms) form_w(NT - 1, NT - 1);
  __syncthreads();
  }
  if (!do_bwd) return;
  clear_ring();

  // ---- backward: Lu^T x = w, from the last own row (a chain: with x_s of
  // the separator rows in the ring)
  __syncthreads();
  if (phase == 3 && split) {
    if (red)
      for (int i = 0; i < NT - NF; ++i)
        ring[(int64_t)((NF + i) % BT) * 32 * KC + rr * KC + cc] = sb[3 * sep_q + (int64_t)(i * 32 + rr) * KC + cc];
  }
#pragma unroll
  for (int u = 0; u < NR; ++u)
    if (1 + wave + 8 * u <= BT - 1) load_slot(A[u], Fbw, NF - 1, 1 + wave + 8 * u);
  __syncthreads();
  for (int I = NF - 1; I >= 0; --I) {
    const int row = I * 32 + rr;
    const double fv = w[(int64_t)row * KC + cc];
    const int dof = band_to_dof(v, bm, row);
    const uint8_t cb = cl[dof >= 0 ? dof : 0];
    const int In = max(I - 1, 0);
    McAcc<WIDE> acc;
    zero_acc(acc);
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int s = 1 + wave + 8 * u;
      const double* yp = ring + (int64_t)((I + s) % BT) * 32 * KC;   // zero beyond row NT-1
      if (s <= BT - 1) {
        const bool has1 = TWOSET && s + 32 <= BT - 1;
        tile_step(A[u], yp, acc, Fbw, has1 ? I : In, has1 ? s + 32 : s);
      }
    }
    if constexpr (TWOSET) {
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int s = 33 + wave + 8 * u;
        const double* yp = ring + (int64_t)((I + s) % BT) * 32 * KC;
        if (s <= BT - 1) tile_step(A[u], yp, acc, Fbw, In, s - 32);
      }
    }
    store_part(acc);
    lds_barrier();
    double xv = 0.0;
    if (red) {
      xv = fv - part_sum();
      ring[(int64_t)(I % BT) * 32 * KC + rr * KC + cc] = xv;
      if (phase == 2) sb[3 * sep_q + (int64_t)(I * 32 + rr) * KC + cc] = xv;
    }
    const bool wr = red & (dof >= 0) & colok & dof_active(kind, cb) & (((out_classes >> cb) & 1) != 0);
    *(wr ? vout + (int64_t)dof * ldk + col : w + (int64_t)(NT * 32 + rr) * KC + cc) = xv;
    lds_barrier();
  }
  if (zero_rest && colok && red && (phase == 0 || (phase == 3 && chain == 0))) {
    for (int d = rr; d < bm.n_dof; d += 32) {
      uint8_t k = cl[d];
      bool written = dof_active(kind, k) && ((out_classes >> k) & 1);
      if (!written) vout[(int64_t)d * ldk + col] = 0.0;
    }
  }
}

#define SOLVE4_INST(NSL, W, T)                                                                                  \
  template __global__ void k_band_solve4<NSL, W, T>(const BoxMeta*, int, int, int, const T*, const uint8_t*,   \
                                                    const double*, double*, int, int, int, double*, int64_t,    \
                                                    const int32_t*, int, double*, int64_t, const int32_t*);
#define SOLVE4_INST_ALL(W, T) SOLVE4_INST(1, W, T) SOLVE4_INST(2, W, T) SOLVE4_INST(3, W, T) SOLVE4_INST(4, W, T)
SOLVE4_INST_ALL(false, double)
SOLVE4_INST_ALL(false, float)
SOLVE4_INST(5, false, double)
SOLVE4_INST(5, false, float)
SOLVE4_INST(8, false, double)
SOLVE4_INST(8, false, float)
SOLVE4_INST_ALL(true, double)
SOLVE4_INST_ALL(true, float)

}  // namespace msg
