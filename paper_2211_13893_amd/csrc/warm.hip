// Learned warm start of the local eigensolver (not in the paper; a start
// block for the LOBPCG iteration of Sec. 3.3 / 4.3 local GEVPs).
//
// A small 3D CNN maps the per-element field of an oversampled box to
// coefficients C (ng x ne) of its first ne start vectors in a fixed basis G
// of ng smooth boundary functions (the lowest A-harmonic eigenvectors of a
// homogeneous isotropic reference box, orthonormal on B2):
//     X0[:, e] = G C[:, e] on B2 (e < ne), seeded random columns e >= ne.
// Network: four 3x3x3 convolutions (zero padding 1, strides 1, 1, 2, 2,
// ReLU), global average, one affine map.  Activations and convolution
// weights are stored in BF16 (or FP32 for checking) with FP32 accumulation;
// master weights, gradients and the Adam state are FP32.
//
// Layouts: activations [B][C][D][D][D]; conv weights [C_out][C_in][27]
// (tap = 9p + 3q + r for offsets (p-1, q-1, r-1) along z, y, x); linear
// weights [n_out][width].  Parameter vector: w0 b0 w1 b1 w2 b2 w3 b3 wl bl.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.hpp"
#include "msgfem.h"

namespace msg {

// ---------------------------------------------------------------- storage
// BF16 = the upper 16 bits of an IEEE single, rounded to nearest even
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline float ldv(const float* p, int64_t i) { return p[i]; }
__device__ inline float ldv(const uint16_t* p, int64_t i) { return bf2f(p[i]); }
__device__ inline void stv(float* p, int64_t i, float v) { p[i] = v; }
__device__ inline void stv(uint16_t* p, int64_t i, float v) { p[i] = f2bf(v); }

__host__ __device__ inline int cnn_out(int d, int s) { return (d - 1) / s + 1; }

// ---------------------------------------------------------------- kernels
template <typename T>
__global__ void k_cnn_store(const float* __restrict__ src, T* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    stv(dst, i, src[i]);
}

// y = ReLU(conv(x) + b), one thread per output value
template <typename T>
__global__ void k_conv_fwd(const T* __restrict__ x, const T* __restrict__ w, const float* __restrict__ bias,
                           T* __restrict__ y, int B, int ci_n, int co_n, int d, int s) {
  const int od = cnn_out(d, s), ov = od * od * od, iv = d * d * d;
  const int64_t n = (int64_t)B * co_n * ov;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(t % ov);
    const int co = (int)((t / ov) % co_n);
    const int b = (int)(t / ((int64_t)ov * co_n));
    const int k = o % od, j = (o / od) % od, i = o / (od * od);
    float acc = bias[co];
    for (int ci = 0; ci < ci_n; ++ci) {
      const T* xp = x + ((int64_t)b * ci_n + ci) * iv;
      const T* wp = w + ((int64_t)co * ci_n + ci) * 27;
      for (int p = 0; p < 3; ++p) {
        const int zi = s * i + p - 1;
        if (zi < 0 || zi >= d) continue;
        for (int q = 0; q < 3; ++q) {
          const int zj = s * j + q - 1;
          if (zj < 0 || zj >= d) continue;
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const int zk = s * k + r - 1;
            if (zk < 0 || zk >= d) continue;
            acc += ldv(wp, 9 * p + 3 * q + r) * ldv(xp, ((int64_t)zi * d + zj) * d + zk);
          }
        }
      }
    }
    stv(y, t, acc > 0.0f ? acc : 0.0f);
  }
}

// The same layer for BF16 storage on the matrix cores, as an implicit GEMM
//     Y[co][v] = sum_k W[co][k] X[k][v],
// X[k][v] the input value of channel ci(k) under tap tap(k) of output voxel v
// (zero outside the grid), with v_mfma_f32_16x16x16bf16_1k: BF16 products,
// FP32 sums.  The K order is ci-major (k = 27 ci + tap) in general and
// tap-major (k = ci_n tap + ci) when ci_n is a multiple of 16, so that a
// chunk of 16 k shares one tap and its bounds test.  W comes packed in that
// order by k_pack_conv_w: 32 rows (zero past co_n) of kp = 27 ci_n rounded up
// to 16 (zero past 27 ci_n).  A wavefront owns 16 output voxels of one sample
// and every output channel (co_n <= 32, two 16-row blocks).
// Lane layout (l = lane): A operand A[l&15][4(l>>4) + e], B operand
// B[4(l>>4) + e][l&15], accumulator item e = D[4(l>>4) + e][l&15], e < 4.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void k_pack_conv_w(const float* __restrict__ w, uint16_t* __restrict__ wp, int ci_n, int co_n, int kp,
                              int tap_major) {
  const int K = 27 * ci_n;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < 32 * kp; t += gridDim.x * blockDim.x) {
    const int co = t / kp, k = t % kp;
    float v = 0.0f;
    if (co < co_n && k < K) {
      const int ci = tap_major ? k % ci_n : k / 27, tap = tap_major ? k / ci_n : k % 27;
      v = w[((int64_t)co * ci_n + ci) * 27 + tap];
    }
    wp[t] = f2bf(v);
  }
}

template <bool TAP_MAJOR>
__global__ __launch_bounds__(256) void k_conv_fwd_mfma(const uint16_t* __restrict__ x,
                                                       const uint16_t* __restrict__ wp,
                                                       const float* __restrict__ bias, uint16_t* __restrict__ y,
                                                       int B, int ci_n, int co_n, int kp, int d, int s) {
  const int od = cnn_out(d, s), ov = od * od * od, iv = d * d * d;
  const int nt = (ov + 15) / 16;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wave >= (int64_t)B * nt) return;
  const int b = (int)(wave / nt), o = (int)(wave % nt) * 16 + (lane & 15), g = lane >> 4;
  const bool vox = o < ov;
  const int oc = vox ? o : 0;
  const int i = oc / (od * od), j = (oc / od) % od, k = oc % od;
  const int z0 = s * i - 1, y0 = s * j - 1, x0 = s * k - 1;
  const int K = 27 * ci_n;
  const uint16_t* xb = x + (int64_t)b * ci_n * iv;
  const uint16_t* w0p = wp + (int64_t)(lane & 15) * kp + 4 * g;
  const uint16_t* w1p = w0p + (int64_t)16 * kp;
  f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  // ci-major order: (ci, tap) of this lane's 4 k values in the current chunk
  int ci[4], tap[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    ci[e] = (4 * g + e) / 27;
    tap[e] = (4 * g + e) % 27;
  }
  const int nblk_ci = ci_n / 16;
  for (int kc = 0, c = 0; kc < K; kc += 16, ++c) {
    bf16x4 bv;
    if (TAP_MAJOR) {
      const int t = c / nblk_ci, cb = c % nblk_ci;
      const int zi = z0 + t / 9, zj = y0 + (t / 3) % 3, zk = x0 + t % 3;
      const bool in = vox && zi >= 0 && zi < d && zj >= 0 && zj < d && zk >= 0 && zk < d;
      const uint16_t* xp = xb + (int64_t)(cb * 16 + 4 * g) * iv + (in ? (zi * d + zj) * d + zk : 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) bv[e] = in ? (short)xp[(int64_t)e * iv] : (short)0;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uint16_t xv = 0;
        if (kc + 4 * g + e < K) {
          const int zi = z0 + tap[e] / 9, zj = y0 + (tap[e] / 3) % 3, zk = x0 + tap[e] % 3;
          if (vox && zi >= 0 && zi < d && zj >= 0 && zj < d && zk >= 0 && zk < d)
            xv = xb[(int64_t)ci[e] * iv + (zi * d + zj) * d + zk];
        }
        bv[e] = (short)xv;
        tap[e] += 16;
        if (tap[e] >= 27) {
          tap[e] -= 27;
          ++ci[e];
        }
      }
    }
    const bf16x4 a0 = *(const bf16x4*)(w0p + kc);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, bv, acc0, 0, 0, 0);
    if (co_n > 16) {
      const bf16x4 a1 = *(const bf16x4*)(w1p + kc);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, bv, acc1, 0, 0, 0);
    }
  }
  if (!vox) return;
  uint16_t* yb = y + (int64_t)b * co_n * ov;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c0 = 4 * g + e, c1 = 16 + 4 * g + e;
    if (c0 < co_n) {
      const float v = acc0[e] + bias[c0];
      stv(yb, (int64_t)c0 * ov + o, v > 0.0f ? v : 0.0f);
    }
    if (c1 < co_n) {
      const float v = acc1[e] + bias[c1];
      stv(yb, (int64_t)c1 * ov + o, v > 0.0f ? v : 0.0f);
    }
  }
}

// g[b][c] = mean over the grid of a[b][c]
template <typename T>
__global__ void k_pool_fwd(const T* __restrict__ a, float* __restrict__ g, int B, int C, int vol) {
  __shared__ float red[256];
  const int bc = blockIdx.x;
  float s = 0.0f;
  for (int v = threadIdx.x; v < vol; v += 256) s += ldv(a, (int64_t)bc * vol + v);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[bc] = red[0] / (float)vol;
}

__global__ void k_linear_fwd(const float* __restrict__ g, const float* __restrict__ wl,
                             const float* __restrict__ bl, float* __restrict__ out, int B, int C, int NO) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * NO) return;
  const int b = t / NO, o = t % NO;
  float s = bl[o];
  for (int c = 0; c < C; ++c) s += wl[o * C + c] * g[b * C + c];
  out[t] = s;
}

// Subspace loss per sample: E = c c^T - P (c = out[b] as [ng][ne], P the
// label projector [ng][ng]); loss[b] = |E|_F^2, gout[b] = gscale 4 E c.
__global__ void k_cnn_loss(const float* __restrict__ out, const float* __restrict__ P, int ng, int ne,
                           float gscale, float* __restrict__ loss, float* __restrict__ gout) {
  extern __shared__ float sm[];
  float* c = sm;                 // ng*ne
  float* E = c + ng * ne;        // ng*ng
  float* red = E + ng * ng;      // 256
  const int b = blockIdx.x;
  const float* cb = out + (int64_t)b * ng * ne;
  const float* Pb = P + (int64_t)b * ng * ng;
  for (int t = threadIdx.x; t < ng * ne; t += 256) c[t] = cb[t];
  __syncthreads();
  float l = 0.0f;
  for (int t = threadIdx.x; t < ng * ng; t += 256) {
    const int i = t / ng, j = t % ng;
    float s = -Pb[t];
    for (int e = 0; e < ne; ++e) s += c[i * ne + e] * c[j * ne + e];
    E[t] = s;
    l += s * s;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[b] = red[0];
  for (int t = threadIdx.x; t < ng * ne; t += 256) {
    const int i = t / ne, e = t % ne;
    float s = 0.0f;
    for (int h = 0; h < ng; ++h) s += E[i * ng + h] * c[h * ne + e];
    gout[(int64_t)b * ng * ne + t] = gscale * 4.0f * s;
  }
}

// gwl[o][c] = sum_b gout[b][o] g[b][c];  gbl[o] = sum_b gout[b][o]
__global__ void k_linear_bwd_w(const float* __restrict__ gout, const float* __restrict__ g,
                               float* __restrict__ gwl, float* __restrict__ gbl, int B, int C, int NO) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NO * (C + 1)) return;
  const int o = t / (C + 1), c = t % (C + 1);
  float s = 0.0f;
  for (int b = 0; b < B; ++b) s += gout[b * NO + o] * (c < C ? g[b * C + c] : 1.0f);
  if (c < C) gwl[o * C + c] = s;
  else gbl[o] = s;
}

// gg[b][c] = sum_o gout[b][o] wl[o][c]
__global__ void k_linear_bwd_x(const float* __restrict__ gout, const float* __restrict__ wl,
                               float* __restrict__ gg, int B, int C, int NO) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * C) return;
  const int b = t / C, c = t % C;
  float s = 0.0f;
  for (int o = 0; o < NO; ++o) s += gout[b * NO + o] * wl[o * C + c];
  gg[t] = s;
}

// gradient of the pooled, ReLU-activated last map: gy = gg / vol where a > 0
template <typename T>
__global__ void k_pool_bwd(const float* __restrict__ gg, const T* __restrict__ a, float* __restrict__ gy,
                           int64_t n, int vol) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    gy[t] = ldv(a, t) > 0.0f ? gg[t / vol] / (float)vol : 0.0f;
}

// gx[b][ci][v] = sum_{co, taps} w[co][ci][tap] gy[b][co][o(v, tap)], times
// the ReLU mask of the layer input a (if given); one thread per input value
template <typename T>
__global__ void k_conv_bwd_data(const float* __restrict__ gy, const T* __restrict__ w, const T* __restrict__ a,
                                float* __restrict__ gx, int B, int ci_n, int co_n, int d, int s) {
  const int od = cnn_out(d, s), ov = od * od * od, iv = d * d * d;
  const int64_t n = (int64_t)B * ci_n * iv;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    if (a && !(ldv(a, t) > 0.0f)) {
      gx[t] = 0.0f;
      continue;
    }
    const int v = (int)(t % iv);
    const int ci = (int)((t / iv) % ci_n);
    const int b = (int)(t / ((int64_t)iv * ci_n));
    const int zk = v % d, zj = (v / d) % d, zi = v / (d * d);
    float acc = 0.0f;
    for (int p = 0; p < 3; ++p) {
      const int ni = zi + 1 - p;            // = s * i
      if (ni < 0 || ni % s) continue;
      const int i = ni / s;
      if (i >= od) continue;
      for (int q = 0; q < 3; ++q) {
        const int nj = zj + 1 - q;
        if (nj < 0 || nj % s) continue;
        const int j = nj / s;
        if (j >= od) continue;
        for (int r = 0; r < 3; ++r) {
          const int nk = zk + 1 - r;
          if (nk < 0 || nk % s) continue;
          const int k = nk / s;
          if (k >= od) continue;
          const int o = (i * od + j) * od + k, tap = 9 * p + 3 * q + r;
          for (int co = 0; co < co_n; ++co)
            acc += ldv(w, ((int64_t)co * ci_n + ci) * 27 + tap) * gy[((int64_t)b * co_n + co) * ov + o];
        }
      }
    }
    gx[t] = acc;
  }
}

// gw[co][ci][tap] = sum_{b, o} gy[b][co][o] x[b][ci][pos(o, tap)]; one
// workgroup per (co, ci); blockIdx.y == 1 forms gb[co] (ci = 0 only).
// Fixed-order reduction.
template <typename T>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const float* __restrict__ gy, const T* __restrict__ x,
                                                    float* __restrict__ gw, float* __restrict__ gb, int B,
                                                    int ci_n, int co_n, int d, int s) {
  __shared__ float red[27][257];
  const int co = blockIdx.x / ci_n, ci = blockIdx.x % ci_n;
  const int od = cnn_out(d, s), ov = od * od * od, iv = d * d * d;
  const int64_t n = (int64_t)B * ov;
  if (blockIdx.y == 1) {
    if (ci != 0) return;
    float sb = 0.0f;
    for (int64_t t = threadIdx.x; t < n; t += 256) {
      const int b = (int)(t / ov), o = (int)(t % ov);
      sb += gy[((int64_t)b * co_n + co) * ov + o];
    }
    red[0][threadIdx.x] = sb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[0][threadIdx.x] += red[0][threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) gb[co] = red[0][0];
    return;
  }
  float acc[27];
#pragma unroll
  for (int tp = 0; tp < 27; ++tp) acc[tp] = 0.0f;
  for (int64_t t = threadIdx.x; t < n; t += 256) {
    const int b = (int)(t / ov), o = (int)(t % ov);
    const float g = gy[((int64_t)b * co_n + co) * ov + o];
    if (g == 0.0f) continue;
    const int k = o % od, j = (o / od) % od, i = o / (od * od);
    const T* xp = x + ((int64_t)b * ci_n + ci) * iv;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const int zi = s * i + p - 1, zj = s * j + q - 1, zk = s * k + r - 1;
          if (zi >= 0 && zi < d && zj >= 0 && zj < d && zk >= 0 && zk < d)
            acc[9 * p + 3 * q + r] += g * ldv(xp, ((int64_t)zi * d + zj) * d + zk);
        }
  }
#pragma unroll
  for (int tp = 0; tp < 27; ++tp) red[tp][threadIdx.x] = acc[tp];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int tp = 0; tp < 27; ++tp) red[tp][threadIdx.x] += red[tp][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 27) gw[((int64_t)co * ci_n + ci) * 27 + threadIdx.x] = red[threadIdx.x][0];
}

// Adam step t (1-based) on every parameter
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, int t) {
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---------------------------------------------------------- warm start
// features of every box: [box][6][ez][ey][ex], per element of the
// oversampled box (cos 2 theta, sin 2 theta, ply flag, (ln E1 - ln 1e4)/2.5,
// 10 dz/dx, 10 dz/dy) with the slopes averaged over the element's four edges
// along that axis (a ply wrinkle shows in them).
__global__ void k_warm_features(const BoxMeta* __restrict__ meta, MeshDev mesh, float* __restrict__ feat) {
  const BoxMeta& bm = meta[blockIdx.y];
  const int ex = bm.mx - 1, ey = bm.my - 1, ez = bm.mz - 1, ne = ex * ey * ez;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int i = e % ex, j = (e / ex) % ey, k = e / (ex * ey);
  const int gi = bm.g0[0] + i, gj = bm.g0[1] + j, gk = bm.g0[2] + k;
  const int ge = gi + mesh.nx * (gj + mesh.ny * gk);
  const double* m = mesh.materials + (int64_t)mesh.elem_mat[ge] * 10;
  const double th = m[9] * (M_PI / 180.0);
  const bool ply = m[0] != m[1];
  auto node = [&](int a, int b, int c) {
    return (int64_t)(gi + a) + (int64_t)(mesh.nx + 1) * ((gj + b) + (int64_t)(mesh.ny + 1) * (gk + c));
  };
  double sx = 0.0, sy = 0.0;
  for (int u = 0; u < 2; ++u)
    for (int w = 0; w < 2; ++w) {
      const double* a0 = mesh.xyz + 3 * node(0, u, w);
      const double* a1 = mesh.xyz + 3 * node(1, u, w);
      sx += (a1[2] - a0[2]) / (a1[0] - a0[0]);
      const double* b0 = mesh.xyz + 3 * node(u, 0, w);
      const double* b1 = mesh.xyz + 3 * node(u, 1, w);
      sy += (b1[2] - b0[2]) / (b1[1] - b0[1]);
    }
  float* f = feat + (int64_t)blockIdx.y * 6 * ne;
  f[e] = (float)cos(2.0 * th);
  f[ne + e] = (float)sin(2.0 * th);
  f[2 * ne + e] = ply ? 1.0f : 0.0f;
  f[3 * ne + e] = (float)((log(m[0]) - log(1.0e4)) / 2.5);
  f[4 * ne + e] = (float)(2.5 * sx);
  f[5 * ne + e] = (float)(2.5 * sy);
}

// G = the B2 parts of ng vectors (box 0 layout [n_dof][nv]) orthonormalised
// by modified Gram-Schmidt (twice) over B2; one workgroup.  G [n_dof][ng].
__global__ __launch_bounds__(1024) void k_warm_basis(const BoxMeta* __restrict__ meta,
                                                     const uint8_t* __restrict__ cls,
                                                     const double* __restrict__ V, int nv, int ng,
                                                     double* __restrict__ G) {
  __shared__ double red[1024];
  const BoxMeta& bm = meta[0];
  const int n = bm.n_dof, tid = threadIdx.x;
  const uint8_t* cl = cls + bm.dof_off;
  for (int64_t t = tid; t < (int64_t)n * ng; t += 1024) {
    const int d = (int)(t / ng), g = (int)(t % ng);
    G[t] = cl[d] == 2 ? V[(int64_t)d * nv + g] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < ng; ++c) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = 0; q < c; ++q) {
        double s = 0.0;
        for (int d = tid; d < n; d += 1024) s += G[(int64_t)d * ng + q] * G[(int64_t)d * ng + c];
        red[tid] = s;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
          if (tid < w) red[tid] += red[tid + w];
          __syncthreads();
        }
        const double pr = red[0];
        __syncthreads();
        for (int d = tid; d < n; d += 1024) G[(int64_t)d * ng + c] -= pr * G[(int64_t)d * ng + q];
        __syncthreads();
      }
    }
    double s = 0.0;
    for (int d = tid; d < n; d += 1024) s += G[(int64_t)d * ng + c] * G[(int64_t)d * ng + c];
    red[tid] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double nrm = sqrt(red[0]);
    __syncthreads();
    for (int d = tid; d < n; d += 1024) G[(int64_t)d * ng + c] = nrm > 0.0 ? G[(int64_t)d * ng + c] / nrm : 0.0;
    __syncthreads();
  }
}

// labels: P = Q Q^T (ng x ng) with Q an orthonormal basis of G^T X_B2,
// X the first ne eigenvectors of the box; one workgroup per box
__global__ __launch_bounds__(256) void k_warm_labels(const BoxMeta* __restrict__ meta,
                                                     const uint8_t* __restrict__ cls,
                                                     const double* __restrict__ evecs,
                                                     const double* __restrict__ G, int ng, int ne,
                                                     float* __restrict__ P) {
  extern __shared__ double q[];    // [ng][ne]
  const BoxMeta& bm = meta[blockIdx.x];
  const int n = bm.n_dof, nev = bm.n_ev;
  const uint8_t* cl = cls + bm.dof_off;
  const double* X = evecs + bm.evec_off;
  for (int t = threadIdx.x; t < ng * ne; t += 256) {
    const int g = t / ne, e = t % ne;
    double s = 0.0;
    for (int d = 0; d < n; ++d)
      if (cl[d] == 2) s += G[(int64_t)d * ng + g] * X[(int64_t)d * nev + e];
    q[t] = s;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    // modified Gram-Schmidt (twice) of the ne columns, one wavefront
    const int ln = threadIdx.x;
    for (int c = 0; c < ne; ++c) {
      for (int pass = 0; pass < 2; ++pass)
        for (int p = 0; p < c; ++p) {
          double s = 0.0;
          for (int g = ln; g < ng; g += 64) s += q[g * ne + p] * q[g * ne + c];
          for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
          for (int g = ln; g < ng; g += 64) q[g * ne + c] -= s * q[g * ne + p];
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        }
      double s = 0.0;
      for (int g = ln; g < ng; g += 64) s += q[g * ne + c] * q[g * ne + c];
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      const double nrm = sqrt(s);
      for (int g = ln; g < ng; g += 64) q[g * ne + c] = nrm > 0.0 ? q[g * ne + c] / nrm : 0.0;
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
  }
  __syncthreads();
  float* Pb = P + (int64_t)blockIdx.x * ng * ng;
  for (int t = threadIdx.x; t < ng * ng; t += 256) {
    const int i = t / ng, j = t % ng;
    double s = 0.0;
    for (int e = 0; e < ne; ++e) s += q[i * ne + e] * q[j * ne + e];
    Pb[t] = (float)s;
  }
}

// 64-bit mix of (seed, box, dof, column) into a standard normal value
__device__ inline double warm_gauss(uint64_t seed, uint64_t a, uint64_t b, uint64_t c) {
  auto mix = [](uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  };
  const uint64_t h1 = mix(seed ^ mix(a ^ mix(b ^ mix(c))));
  const uint64_t h2 = mix(h1 + 0x632be59bd9b4e019ull);
  const double u1 = ((h1 >> 11) + 1) * (1.0 / 9007199254740993.0);
  const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// x0 of every box on B2: column e < ne = G C[:, e], the other columns seeded
// Gaussian; 0 off B2.  A predicted column that is not finite or is zero falls
// back to a Gaussian column too.  Box block layout [n_dof][k].  One thread
// per DoF row: the box's C and its column checks sit in LDS, the row's G
// entries are read once per 8 columns, and the row of x0 is written whole.
__global__ __launch_bounds__(256) void k_warm_start(const BoxMeta* __restrict__ meta,
                                                    const uint8_t* __restrict__ cls,
                                                    const float* __restrict__ coef, const double* __restrict__ G,
                                                    int ng, int ne, int k, uint64_t seed, double* __restrict__ x0) {
  extern __shared__ float wsh[];          // C of this box [ng][ne], then one flag per column
  int* okc = (int*)(wsh + ng * ne);
  const int box = blockIdx.y;
  const BoxMeta& bm = meta[box];
  const float* cb = coef + (int64_t)box * ng * ne;
  for (int i = threadIdx.x; i < ng * ne; i += blockDim.x) wsh[i] = cb[i];
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    double nrm = 0.0;
    for (int g = 0; g < ng; ++g) {
      const double cg = (double)cb[g * ne + e];
      nrm += cg * cg;
    }
    okc[e] = (nrm > 0.0 && isfinite(nrm)) ? 1 : 0;
  }
  __syncthreads();
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= bm.n_dof) return;
  double* xr = x0 + ((int64_t)bm.dof_off + d) * k;
  if (cls[bm.dof_off + d] != 2) {
    for (int e = 0; e < k; ++e) xr[e] = 0.0;
    return;
  }
  const double* gr = G + (int64_t)d * ng;
  for (int e0 = 0; e0 < ne; e0 += 8) {
    double acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0.0;
    for (int g = 0; g < ng; ++g) {
      const double gv = gr[g];
      const float* cr = wsh + g * ne + e0;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (e0 + j < ne) acc[j] += gv * (double)cr[j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = e0 + j;
      if (e < ne) xr[e] = okc[e] ? acc[j] : warm_gauss(seed, box, d, e);
    }
  }
  for (int e = ne; e < k; ++e) xr[e] = warm_gauss(seed, box, d, e);
}

// ------------------------------------------------------------- C ABI
namespace {
struct CnnDims {
  int cin, width, n_out, d0, d[5];
  int64_t woff[4], boff[4], wl, bl, n_params;
  int kp[4];                 // packed K per layer (27 ci_n rounded up to 16)
  int64_t wpoff[4], n_wp;    // packed BF16 weights of the matrix-core layers: 32 x kp each
};
CnnDims cnn_dims(int cin, int width, int n_out, int d0) {
  CnnDims c;
  c.cin = cin;
  c.width = width;
  c.n_out = n_out;
  c.d0 = d0;
  const int st[4] = {1, 1, 2, 2};
  c.d[0] = d0;
  for (int l = 0; l < 4; ++l) c.d[l + 1] = cnn_out(c.d[l], st[l]);
  int64_t off = 0;
  for (int l = 0; l < 4; ++l) {
    c.woff[l] = off;
    off += (int64_t)width * (l == 0 ? cin : width) * 27;
    c.boff[l] = off;
    off += width;
  }
  c.wl = off;
  off += (int64_t)n_out * width;
  c.bl = off;
  off += n_out;
  c.n_params = off;
  c.n_wp = 0;
  for (int l = 0; l < 4; ++l) {
    c.kp[l] = (27 * (l == 0 ? cin : width) + 15) / 16 * 16;
    c.wpoff[l] = c.n_wp;
    c.n_wp += 32 * (int64_t)c.kp[l];
  }
  return c;
}
struct CnnWork {
  char* act;        // storage-type activations: x, a1..a4
  int64_t aoff[5];
  char* wT;         // storage-type conv weights
  uint16_t* wP;     // packed BF16 conv weights (matrix-core layers)
  float* g;         // pooled [B][width]
  float* gg;        // [B][width]
  float* gA;        // gradient ping-pong buffers
  float* gB;
  int64_t bytes;
};
CnnWork cnn_work(const CnnDims& c, int B, int esz, void* base) {
  CnnWork w;
  char* b = (char*)base;
  int64_t off = 0;
  auto al = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
  int64_t maxv = 0;
  for (int l = 0; l <= 4; ++l) {
    const int ch = l == 0 ? c.cin : c.width;
    const int64_t v = (int64_t)B * ch * c.d[l] * c.d[l] * c.d[l];
    w.aoff[l] = off;
    off = al(off + v * esz);
    maxv = v > maxv ? v : maxv;
  }
  w.act = b;
  w.wT = b + off;
  off = al(off + c.n_params * esz);
  w.wP = (uint16_t*)(b + off);
  off = al(off + c.n_wp * 2);
  w.g = (float*)(b + off);
  off = al(off + (int64_t)B * c.width * 4);
  w.gg = (float*)(b + off);
  off = al(off + (int64_t)B * c.width * 4);
  w.gA = (float*)(b + off);
  off = al(off + maxv * 4);
  w.gB = (float*)(b + off);
  off = al(off + maxv * 4);
  w.bytes = off;
  return w;
}
inline unsigned nblk(int64_t n) { return (unsigned)(n <= 0 ? 1 : (n + 255) / 256 < 65535 ? (n + 255) / 256 : 65535); }

template <typename T>
int cnn_forward_t(const CnnDims& c, const float* params, int B, const float* x, float* out, void* work,
                  hipStream_t s) {
  CnnWork w = cnn_work(c, B, sizeof(T), work);
  T* wT = (T*)w.wT;
  k_cnn_store<T><<<nblk(c.n_params), 256, 0, s>>>(params, wT, c.n_params);
  const int64_t nx = (int64_t)B * c.cin * c.d0 * c.d0 * c.d0;
  k_cnn_store<T><<<nblk(nx), 256, 0, s>>>(x, (T*)(w.act + w.aoff[0]), nx);
  const int st[4] = {1, 1, 2, 2};
  for (int l = 0; l < 4; ++l) {
    const int ci = l == 0 ? c.cin : c.width;
    const int64_t n = (int64_t)B * c.width * c.d[l + 1] * c.d[l + 1] * c.d[l + 1];
    if (sizeof(T) == 2 && c.width <= 32) {
      const int ov = c.d[l + 1] * c.d[l + 1] * c.d[l + 1];
      const int64_t waves = (int64_t)B * ((ov + 15) / 16);
      const bool tap_major = ci % 16 == 0;
      uint16_t* wp = w.wP + c.wpoff[l];
      k_pack_conv_w<<<nblk(32 * (int64_t)c.kp[l]), 256, 0, s>>>(params + c.woff[l], wp, ci, c.width, c.kp[l],
                                                                tap_major ? 1 : 0);
      const unsigned grid = (unsigned)((waves + 3) / 4);
      const uint16_t* xin = (const uint16_t*)(w.act + w.aoff[l]);
      uint16_t* yout = (uint16_t*)(w.act + w.aoff[l + 1]);
      if (tap_major)
        k_conv_fwd_mfma<true><<<grid, 256, 0, s>>>(xin, wp, params + c.boff[l], yout, B, ci, c.width, c.kp[l],
                                                   c.d[l], st[l]);
      else
        k_conv_fwd_mfma<false><<<grid, 256, 0, s>>>(xin, wp, params + c.boff[l], yout, B, ci, c.width, c.kp[l],
                                                    c.d[l], st[l]);
    } else {
      k_conv_fwd<T><<<nblk(n), 256, 0, s>>>((const T*)(w.act + w.aoff[l]), wT + c.woff[l], params + c.boff[l],
                                             (T*)(w.act + w.aoff[l + 1]), B, ci, c.width, c.d[l], st[l]);
    }
  }
  const int vol = c.d[4] * c.d[4] * c.d[4];
  k_pool_fwd<T><<<B * c.width, 256, 0, s>>>((const T*)(w.act + w.aoff[4]), w.g, B, c.width, vol);
  k_linear_fwd<<<nblk((int64_t)B * c.n_out), 256, 0, s>>>(w.g, params + c.wl, params + c.bl, out, B, c.width,
                                                           c.n_out);
  return hipGetLastError() == hipSuccess ? MSGFEM_OK : MSGFEM_EHIP;
}

template <typename T>
int cnn_backward_t(const CnnDims& c, const float* params, int B, const float* gout, float* grads, void* work,
                   hipStream_t s) {
  CnnWork w = cnn_work(c, B, sizeof(T), work);
  const T* wT = (const T*)w.wT;
  k_linear_bwd_w<<<nblk((int64_t)c.n_out * (c.width + 1)), 256, 0, s>>>(gout, w.g, grads + c.wl, grads + c.bl, B,
                                                                         c.width, c.n_out);
  k_linear_bwd_x<<<nblk((int64_t)B * c.width), 256, 0, s>>>(gout, params + c.wl, w.gg, B, c.width, c.n_out);
  const int vol = c.d[4] * c.d[4] * c.d[4];
  const int64_t n4 = (int64_t)B * c.width * vol;
  k_pool_bwd<T><<<nblk(n4), 256, 0, s>>>(w.gg, (const T*)(w.act + w.aoff[4]), w.gA, n4, vol);
  const int st[4] = {1, 1, 2, 2};
  float* gy = w.gA;
  float* gx = w.gB;
  for (int l = 3; l >= 0; --l) {
    const int ci = l == 0 ? c.cin : c.width;
    k_conv_bwd_w<T><<<dim3(c.width * ci, 2), 256, 0, s>>>(gy, (const T*)(w.act + w.aoff[l]), grads + c.woff[l],
                                                           grads + c.boff[l], B, ci, c.width, c.d[l], st[l]);
    if (l > 0) {
      const int64_t n = (int64_t)B * ci * c.d[l] * c.d[l] * c.d[l];
      k_conv_bwd_data<T><<<nblk(n), 256, 0, s>>>(gy, wT + c.woff[l], (const T*)(w.act + w.aoff[l]), gx, B, ci,
                                                  c.width, c.d[l], st[l]);
      float* tmp = gy;
      gy = gx;
      gx = tmp;
    }
  }
  return hipGetLastError() == hipSuccess ? MSGFEM_OK : MSGFEM_EHIP;
}
}  // namespace

}  // namespace msg

using namespace msg;

extern "C" int msgfem_cnn_sizes(int32_t cin, int32_t width, int32_t n_out, int32_t d, int32_t batch,
                                int64_t* n_params, int64_t* work_bytes) {
  if (cin < 1 || width < 1 || n_out < 1 || d < 1 || batch < 1 || !n_params || !work_bytes) return MSGFEM_EARG;
  CnnDims c = cnn_dims(cin, width, n_out, d);
  *n_params = c.n_params;
  *work_bytes = cnn_work(c, batch, 4, nullptr).bytes;   // FP32 storage is the larger
  return MSGFEM_OK;
}

extern "C" int msgfem_cnn_forward(const float* params, int32_t cin, int32_t width, int32_t n_out, int32_t d,
                                  int32_t batch, int32_t bf16, const float* x, float* out, void* work,
                                  void* stream) {
  if (!params || !x || !out || !work || cin < 1 || width < 1 || n_out < 1 || d < 1 || batch < 1)
    return MSGFEM_EARG;
  CnnDims c = cnn_dims(cin, width, n_out, d);
  hipStream_t s = (hipStream_t)stream;
  return bf16 ? cnn_forward_t<uint16_t>(c, params, batch, x, out, work, s)
              : cnn_forward_t<float>(c, params, batch, x, out, work, s);
}

extern "C" int msgfem_cnn_backward(const float* params, int32_t cin, int32_t width, int32_t n_out, int32_t d,
                                   int32_t batch, int32_t bf16, const float* gout, float* grads, void* work,
                                   void* stream) {
  if (!params || !gout || !grads || !work || cin < 1 || width < 1 || n_out < 1 || d < 1 || batch < 1)
    return MSGFEM_EARG;
  CnnDims c = cnn_dims(cin, width, n_out, d);
  hipStream_t s = (hipStream_t)stream;
  return bf16 ? cnn_backward_t<uint16_t>(c, params, batch, gout, grads, work, s)
              : cnn_backward_t<float>(c, params, batch, gout, grads, work, s);
}

extern "C" int msgfem_cnn_loss(const float* out, const float* labels, int32_t ng, int32_t ne, int32_t batch,
                               float gscale, float* loss, float* gout, void* stream) {
  if (!out || !labels || !loss || !gout || ng < 1 || ne < 1 || batch < 1) return MSGFEM_EARG;
  const size_t lds = (size_t)(ng * ne + ng * ng + 256) * 4;
  if (lds > 64 * 1024) return MSGFEM_ESIZE;
  k_cnn_loss<<<batch, 256, lds, (hipStream_t)stream>>>(out, labels, ng, ne, gscale, loss, gout);
  return hipGetLastError() == hipSuccess ? MSGFEM_OK : MSGFEM_EHIP;
}

extern "C" int msgfem_cnn_adam(float* params, const float* grads, float* m, float* v, int64_t n, int32_t step,
                               float lr, void* stream) {
  if (!params || !grads || !m || !v || n < 1 || step < 1) return MSGFEM_EARG;
  k_adam<<<nblk(n), 256, 0, (hipStream_t)stream>>>(params, grads, m, v, n, lr, 0.9f, 0.999f, 1e-8f, step);
  return hipGetLastError() == hipSuccess ? MSGFEM_OK : MSGFEM_EHIP;
}
