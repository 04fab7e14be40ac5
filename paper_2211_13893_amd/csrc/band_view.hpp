// Band matrices of the oversampled boxes: which DoFs a tile row maps to,
// shared by the band build, the relayout and the block solve.
#pragma once
#include "internal.hpp"

namespace msg {

struct BandView {
  int NT, BT, NTf;
  int64_t off, ioff;
  int64_t doff, dstride;   // D^{-1} tile I of the unit-lower factor at doff + I*dstride
  int64_t fw, bw;   // solve-ordered band copies (forward / backward sweep)
  int sx, sy, sz;   // node dims of the ordering, fastest to slowest index
  int base;         // box node of the ordering's node (0,0,0)
  int st0, st1, st2;   // box node strides of the three order indices
  int w0, w1, w2;      // their weights in the 27-point neighbour index (1, 3 or 9)
  // rows of the part: pad identity rows, nc rows of the order (layers from
  // the far end when mirror), nsep rows of the separator layer zs
  int pad, nc, nsep, mirror, L, zs;
};

// the ordering of a (sub-)box with node dims d[3] (box axes) starting at box
// node (o[0], o[1], o[2]); ord encodes the box axis of each order index
__device__ inline void band_order(BandView& v, const BoxMeta& bm, int ord, const int d[3], const int o[3]) {
  const int a0 = ord & 3, a1 = (ord >> 2) & 3, a2 = (ord >> 4) & 3;
  const int st[3] = {1, bm.mx, bm.mx * bm.my};
  const int w[3] = {1, 3, 9};
  v.sx = d[a0]; v.sy = d[a1]; v.sz = d[a2];
  v.st0 = st[a0]; v.st1 = st[a1]; v.st2 = st[a2];
  v.w0 = w[a0]; v.w1 = w[a1]; v.w2 = w[a2];
  v.base = o[0] + bm.mx * (o[1] + bm.my * o[2]);
}

// part 0..2 of the A11 (kind 0) or Ahat (kind 1) factorisation of a box
__device__ inline BandView band_view(const BoxMeta& bm, int kind, int part = 0) {
  BandView v;
  const BandPart& q = bm.part[kind][part];
  v.NT = q.NT; v.BT = q.BT; v.NTf = q.NTf;
  v.off = q.off; v.ioff = q.ioff; v.fw = q.fw; v.bw = q.bw;
  v.pad = q.pad; v.nc = q.nc; v.nsep = q.nsep; v.mirror = q.mirror;
  if (kind == 0) {
    const int d[3] = {bm.sub_hi[0] - bm.sub_lo[0] + 1, bm.sub_hi[1] - bm.sub_lo[1] + 1,
                      bm.sub_hi[2] - bm.sub_lo[2] + 1};
    band_order(v, bm, bm.ord[0], d, bm.sub_lo);
  } else {
    const int d[3] = {bm.mx, bm.my, bm.mz}, o[3] = {0, 0, 0};
    band_order(v, bm, bm.ord[1], d, o);
  }
  v.L = 3 * v.sx * v.sy;
  v.zs = bm.zs[kind];
  const bool compact = bm.flags & BOX_COMPACT_DINV;
  v.doff = compact ? q.ioff : q.off;
  v.dstride = compact ? (int64_t)MSG_TILE2 : (int64_t)q.BT * MSG_TILE2;
  return v;
}

// band row of the part -> row of the whole (sub-)box order (3 node + component), or -1
__device__ inline int band_to_order(const BandView& v, int r) {
  r -= v.pad;
  if (r < 0) return -1;
  if (r < v.nc) {
    if (!v.mirror) return r;
    const int l = r / v.L;
    return (v.sz - 1 - l) * v.L + (r - l * v.L);
  }
  r -= v.nc;
  return r < v.nsep ? v.zs * v.L + r : -1;
}

// row of the whole order -> box DoF
__device__ inline int order_to_dof(const BandView& v, int q) {
  int node = q / 3, c = q - 3 * node;
  int i = node % v.sx, j = (node / v.sx) % v.sy, k = node / (v.sx * v.sy);
  return 3 * (v.base + i * v.st0 + j * v.st1 + k * v.st2) + c;
}

// band row -> box DoF (or -1 for padding rows)
__device__ inline int band_to_dof(const BandView& v, const BoxMeta& bm, int r) {
  (void)bm;
  const int q = band_to_order(v, r);
  return q < 0 ? -1 : order_to_dof(v, q);
}

__device__ inline bool dof_active(int kind, uint8_t c) {
  return kind == 0 ? (c == 1) : (c == 1 || c == 2);
}

}  // namespace msg
