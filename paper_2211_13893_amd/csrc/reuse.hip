// Offline/online reuse of local spaces (Sec. 1 and Sec. 6: the local spaces of
// subdomains whose data did not change can be kept, and only the changed ones
// recomputed).
//
//  k_box_digest + k_box_digest_finish : a 64-bit digest per batch box of everything its local
//                 eigenproblem reads once assembled: the block-27 stencil of
//                 a_{Omega*}, the DoF classes B1/B2/B3 and the partition of
//                 unity mu_j, plus the box geometry, n_ev and a salt with the
//                 eigensolver options.  Each value is mixed with its position
//                 by the splitmix64 finaliser (Steele, Lea and Flood, 2014) and
//                 the mixed words are summed modulo 2^64, which makes the
//                 digest independent of the order of the partial sums, so it
//                 is the same bits on every run.
//  k_copy_eigs  : copies one box's eigenpairs, residuals and iteration count
//                 between two eigen outputs of plans with the same box
//                 geometry.

#include "internal.hpp"

namespace msg {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// position-tagged word: distinct streams (stencil, classes, mu) use distinct tags
__device__ __forceinline__ uint64_t tagged(uint64_t v, uint64_t tag, int64_t i) {
  return mix64(v ^ mix64(tag + 0x9e3779b97f4a7c15ull * (uint64_t)(i + 1)));
}

#define DIGEST_THREADS 256
// grid (chunks, nb): workgroup c of box b sums its slice of the box's words
// and adds the sum into acc[b] (unsigned 64-bit atomics; integer addition is
// exact and commutative, so the result does not depend on their order).  acc
// must be zero beforehand; k_box_digest_finish then mixes in the geometry
// and the salt.
__global__ __launch_bounds__(DIGEST_THREADS) void k_box_digest(const BoxMeta* __restrict__ meta,
                                                               const double* __restrict__ stencil,
                                                               const double* __restrict__ mu1,
                                                               const uint8_t* __restrict__ cls,
                                                               unsigned long long* __restrict__ acc) {
  __shared__ uint64_t red[DIGEST_THREADS];
  const BoxMeta& bm = meta[blockIdx.y];
  const int tid = threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * DIGEST_THREADS;
  const int64_t first = (int64_t)blockIdx.x * DIGEST_THREADS + tid;
  uint64_t h = 0;
  const double* st = stencil + bm.node_off * 243;
  const int64_t ns = (int64_t)bm.n_nodes * 243;
  for (int64_t i = first; i < ns; i += stride) h += tagged((uint64_t)__double_as_longlong(st[i]), 1, i);
  for (int64_t i = first; i < bm.n_dof; i += stride) {
    h += tagged((uint64_t)__double_as_longlong(mu1[bm.dof_off + i]), 2, i);
    h += tagged((uint64_t)cls[bm.dof_off + i], 3, i);
  }
  red[tid] = h;
  __syncthreads();
  for (int s = DIGEST_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) atomicAdd(&acc[blockIdx.y], (unsigned long long)red[0]);
}

__global__ void k_box_digest_finish(const BoxMeta* __restrict__ meta, int nb, uint64_t salt,
                                    unsigned long long* __restrict__ acc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const BoxMeta& bm = meta[b];
  uint64_t g = acc[b];
  const int32_t geo[7] = {bm.mx, bm.my, bm.mz, bm.g0[0], bm.g0[1], bm.g0[2], bm.n_ev};
  for (int q = 0; q < 7; ++q) g += tagged((uint64_t)(uint32_t)geo[q], 4, q);
  acc[b] = mix64(g ^ salt);
}

__global__ void k_copy_eigs(int n_ev, int64_t n_vec, const double* __restrict__ sval,
                            const double* __restrict__ svec, const double* __restrict__ sres,
                            const int32_t* __restrict__ sit, double* __restrict__ dval,
                            double* __restrict__ dvec, double* __restrict__ dres, int32_t* __restrict__ dit) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_vec) dvec[i] = svec[i];
  if (i < n_ev) {
    dval[i] = sval[i];
    dres[i] = sres[i];
  }
  if (i == 0) dit[0] = sit[0];
}

}  // namespace msg
