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

// The same products for a batch of boxes and a block of width k (a multiple
// of 8), staged through LDS.  A workgroup takes 8 columns of one box (or of
// an x-tile of it when a node plane holds more than SP_PLANE nodes) and
// marches through the box's node planes (z, the slowest node index): the
// rows of X (and mu) of planes z-1, z, z+1 sit in LDS and the 27 neighbours
// of a node are read there, so the stencil is the only stream (read once
// per node and column group, 16 nodes per load).  Four threads per node,
// two columns each (16 wavefronts per CU hide the stencil's latency).  Plane
// z+2 is requested into registers while plane z is computed and stored into
// the slot plane z-1 leaves.  The 8-column groups of a box run on one XCD
// (block x on XCD x mod 8), so the box's stencil is read from HBM about
// once.  LDS: 3 slots of [3 DoFs][SP_PLANE nodes][4 column pairs] double2
// (the 4 threads of a node read consecutive 16-byte pieces), plus [3][SP_PLANE]
// mu with the second product.
// grid.x = 8 * n_group * ceil(n_unit / 8), units = n_box * max_tiles
// (unit = box * max_tiles + tile); 1024 threads.
#define SP_PLANE 240
#define SP_THREADS 1024

// x-tile width of a box: the whole plane when it fits, else the widest tile
// whose plane with one halo column on each side fits (0: does not fit)
__host__ __device__ inline int sp_tile_x(int mx, int my) {
  if (mx * my <= SP_PLANE) return mx;
  const int t = SP_PLANE / my - 2;
  return t >= 1 ? t : 0;
}

// value of lane (lane & ~3) + o of the quad (DPP quad_perm broadcast, o a constant)
__device__ inline double quad_bcast(double v, int o) {
  const int ctrl = o == 0 ? 0x00 : o == 1 ? 0x55 : o == 2 ? 0xAA : 0xFF;
  int lo, hi;
  switch (ctrl) {
    case 0x00:
      lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x00, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x00, 0xF, 0xF, false);
      break;
    case 0x55:
      lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x55, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x55, 0xF, 0xF, false);
      break;
    case 0xAA:
      lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xAA, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xAA, 0xF, 0xF, false);
      break;
    default:
      lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xFF, 0xF, 0xF, false);
      hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xFF, 0xF, 0xF, false);
      break;
  }
  return __hiloint2double(hi, lo);
}

template <bool TWO, typename ST>
__global__ __launch_bounds__(SP_THREADS) void k_spmm_planes(const BoxMeta* __restrict__ meta, int n_box,
                                                            int max_tiles, int n_group,
                                                            const ST* __restrict__ stencil,
                                                            const uint8_t* __restrict__ cls,
                                                            const double* __restrict__ mu1,
                                                            const double* __restrict__ X, double* Y, double* Y2,
                                                            int k, int y_classes, double scale,
                                                            const int32_t* __restrict__ active) {
  extern __shared__ double2 spl[];   // [3 slots][3 DoFs][SP_PLANE][4] double2, then (TWO) [3][3][SP_PLANE] double
  double* smu = (double*)(spl + 3 * 3 * SP_PLANE * 4);
  const int xb = blockIdx.x, xcd = xb & 7, rest = xb >> 3;
  const int g = rest % n_group;
  const int unit = (rest / n_group) * 8 + xcd;
  const int box = unit / max_tiles, tile = unit - box * max_tiles;
  if (box >= n_box) return;
  if (active && !active[box]) return;
  const BoxMeta& bm = meta[box];
  const int mx = bm.mx, my = bm.my, mz = bm.mz;
  const int TX = sp_tile_x(mx, my);
  const int x0 = tile * TX;
  if (TX == 0 || x0 >= mx) return;
  const int xs = max(x0 - 1, 0), xe = min(x0 + TX + 1, mx), TXh = xe - xs;   // staged columns
  const int TXa = min(TX, mx - x0);                                           // own columns
  const int tid = threadIdx.x, tn = tid >> 2, q = tid & 3;
  const bool own = tn < TXa * my;
  const int ly = own ? tn / TXa : 0, lx = own ? tn - ly * TXa : 0;
  const int nx = x0 + lx;
  const int c0 = 8 * g;
  const double* x = X + bm.dof_off * k + c0;
  const uint8_t* cl = cls + bm.dof_off;
  const double* m1 = mu1 + bm.dof_off;
  const int nunits = TXh * my * 12;   // double2 pieces of a staged plane
  constexpr int MAXU = (SP_PLANE * 12 + SP_THREADS - 1) / SP_THREADS;
  constexpr int MAXM = (SP_PLANE * 3 + SP_THREADS - 1) / SP_THREADS;
  double2 buf[MAXU];
  double bmu[MAXM];
  // plane z into registers: piece u = (staged node h, DoF c, column pair pc)
  auto fetch = [&](int z) {
#pragma unroll
    for (int r = 0; r < MAXU; ++r) {
      const int u = tid + SP_THREADS * r;
      buf[r] = double2{0.0, 0.0};
      if (u < nunits) {
        const int h = u / 12, e = u - 12 * h;
        const int hy = h / TXh, hx = h - hy * TXh;
        const int node = (xs + hx) + mx * (hy + my * z);
        buf[r] = *(const double2*)(x + (int64_t)(3 * node + (e >> 2)) * k + 2 * (e & 3));
      }
    }
    if (TWO) {
#pragma unroll
      for (int r = 0; r < MAXM; ++r) {
        const int u = tid + SP_THREADS * r;
        bmu[r] = 0.0;
        if (u < TXh * my * 3) {
          const int h = u / 3, c = u - 3 * h;
          const int hy = h / TXh, hx = h - hy * TXh;
          bmu[r] = m1[3 * ((xs + hx) + mx * (hy + my * z)) + c];
        }
      }
    }
  };
  auto stash = [&](int slot) {
#pragma unroll
    for (int r = 0; r < MAXU; ++r) {
      const int u = tid + SP_THREADS * r;
      if (u < nunits) {
        const int h = u / 12, e = u - 12 * h;
        spl[((slot * 3 + (e >> 2)) * SP_PLANE + h) * 4 + (e & 3)] = buf[r];
      }
    }
    if (TWO) {
#pragma unroll
      for (int r = 0; r < MAXM; ++r) {
        const int u = tid + SP_THREADS * r;
        if (u < TXh * my * 3) {
          const int h = u / 3, c = u - 3 * h;
          smu[(slot * 3 + c) * SP_PLANE + h] = bmu[r];
        }
      }
    }
  };
  fetch(0);
  stash(0);
  if (mz > 1) {
    fetch(1);
    stash(1);
  }
  __syncthreads();
  if (mz > 2) fetch(2);
  const ST* stb = stencil + bm.node_off * 243;
  double* y = Y ? Y + bm.dof_off * k + c0 + 2 * q : nullptr;
  double* y2 = TWO ? Y2 + bm.dof_off * k + c0 + 2 * q : nullptr;
  for (int z = 0; z < mz; ++z) {
    if (own) {
      const int node = nx + mx * (ly + my * z);
      const ST* st = stb + node;
      double acc[3][2], acc2[3][2];
#pragma unroll
      for (int cr = 0; cr < 3; ++cr) {
        acc[cr][0] = acc[cr][1] = 0.0;
        acc2[cr][0] = acc2[cr][1] = 0.0;
      }
      // neighbours outside the box have zero stencil blocks: their index is
      // clamped into the box (the staged tile includes the clamped node).
      // Per layer dz, the 4 threads of the node split the 81 coefficients of
      // its 9 neighbours (coefficient v = 9 nbl + e to lane v % 4), request
      // them together, and pass each one round the quad.
#pragma unroll 1
      for (int dz = -1; dz <= 1; ++dz) {
        const int zz = min(max(z + dz, 0), mz - 1);
        const int slot = zz % 3;
        // coefficient v of the layer is stencil row 81 (dz + 1) + v of the node
        // (nb * 9 + e with nb = nbl + 9 (dz + 1)); lane v % 4 reads it.  With
        // the second product the layer goes in two parts (neighbours 0-4,
        // 5-8) to hold fewer coefficients at a time.
        constexpr int NH = TWO ? 2 : 1;
        constexpr int NR = TWO ? 12 : 21;
#pragma unroll
        for (int hh = 0; hh < NH; ++hh) {
          asm volatile("" ::: "memory");   // each part's loads after the previous part
          const int vlo = hh == 0 ? 0 : 45, vhi = NH == 1 ? 81 : (hh == 0 ? 45 : 81);
          const int qq = (q - vlo) & 3;   // this lane's first coefficient: vlo + qq
          double sv[NR];
          const ST* sq = st + (int64_t)(81 * (dz + 1) + vlo + qq) * bm.n_nodes;
          const int64_t s4 = 4 * (int64_t)bm.n_nodes;
#pragma unroll
          for (int r = 0; r < NR; ++r) sv[r] = (vlo + qq + 4 * r < vhi) ? (double)sq[r * s4] : 0.0;
#pragma unroll
          for (int nbl = 0; nbl < 9; ++nbl) {
            if (9 * nbl < vlo || 9 * nbl >= vhi) continue;
            asm volatile("" ::: "memory");   // one neighbour's LDS reads at a time (register pressure)
            const int dy = nbl / 3 - 1, dx = nbl % 3 - 1;
            const int yy = min(max(ly + dy, 0), my - 1);
            const int xx = min(max(nx + dx, 0), mx - 1);
            const int h = (xx - xs) + TXh * yy;
            double2 xv[3];
            double mu[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
              xv[cc] = spl[((slot * 3 + cc) * SP_PLANE + h) * 4 + q];
              mu[cc] = TWO ? smu[(slot * 3 + cc) * SP_PLANE + h] : 0.0;
            }
#pragma unroll
            for (int e = 0; e < 9; ++e) {
              const int v = 9 * nbl + e, cr = e / 3, cc = e % 3;
              const double a = quad_bcast(sv[(v - vlo) >> 2], v & 3);
              acc[cr][0] += a * xv[cc].x;
              acc[cr][1] += a * xv[cc].y;
              if (TWO) {
                const double am = a * mu[cc];
                acc2[cr][0] += am * xv[cc].x;
                acc2[cr][1] += am * xv[cc].y;
              }
            }
          }
        }
      }
#pragma unroll
      for (int cr = 0; cr < 3; ++cr) {
        const int d = 3 * node + cr;
        const bool w = (y_classes >> cl[d]) & 1;
        if (y) *(double2*)(y + (int64_t)d * k) = w ? double2{scale * acc[cr][0], scale * acc[cr][1]} : double2{0.0, 0.0};
        if (TWO) {
          const double mo = m1[d];
          *(double2*)(y2 + (int64_t)d * k) = double2{mo * acc2[cr][0], mo * acc2[cr][1]};
        }
      }
    }
    // slot (z+2) % 3 held plane z-1, which no thread reads any more
    __syncthreads();
    if (z + 2 < mz) stash((z + 2) % 3);
    __syncthreads();
    if (z + 3 < mz) fetch(z + 3);
  }
}

#define SPP_INST(TW, ST)                                                                                        \
  template __global__ void k_spmm_planes<TW, ST>(const BoxMeta*, int, int, int, const ST*, const uint8_t*,      \
                                                 const double*, const double*, double*, double*, int, int, double, \
                                                 const int32_t*);
SPP_INST(false, double)
SPP_INST(true, double)
SPP_INST(false, float)
SPP_INST(true, float)

// out = X with the rows of B3 DoFs cleared (flat over all boxes' [n_dof][k] blocks)
__global__ void k_mask_b3(const uint8_t* __restrict__ cls, const double* __restrict__ X, int k, int64_t n,
                          double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = cls[e / k] == 3 ? 0.0 : X[e];
}

}  // namespace msg
