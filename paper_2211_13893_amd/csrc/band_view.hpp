// Band matrices of the oversampled boxes: which DoFs a tile row maps to,
// shared by the band build, the relayout and the block solve.
#pragma once
#include "internal.hpp"

namespace msg {

struct BandView {
  int NT, BT, n;
  int64_t off, ioff;
  int64_t doff, dstride;   // D^{-1} tile I of the unit-lower factor at doff + I*dstride
  int64_t fw, bw;   // solve-ordered band copies (forward / backward sweep)
  int sx, sy, sz;   // (sub-)box node dims of the ordering
  int ox, oy, oz;   // offset of the ordering's node (0,0,0) inside the box
};

__device__ inline BandView band_view(const BoxMeta& bm, int kind) {
  BandView v;
  if (kind == 0) {
    v.NT = bm.nt11; v.BT = bm.bt11; v.n = bm.n11; v.off = bm.f11_off; v.ioff = bm.f11i_off;
    v.fw = bm.f11_fw; v.bw = bm.f11_bw;
    v.sx = bm.sub_hi[0] - bm.sub_lo[0] + 1;
    v.sy = bm.sub_hi[1] - bm.sub_lo[1] + 1;
    v.sz = bm.sub_hi[2] - bm.sub_lo[2] + 1;
    v.ox = bm.sub_lo[0]; v.oy = bm.sub_lo[1]; v.oz = bm.sub_lo[2];
    const bool compact = bm.flags & BOX_COMPACT_DINV;
    v.doff = compact ? bm.f11i_off : bm.f11_off;
    v.dstride = compact ? (int64_t)MSG_TILE2 : (int64_t)bm.bt11 * MSG_TILE2;
  } else {
    v.NT = bm.nth; v.BT = bm.bth; v.n = bm.nh; v.off = bm.fh_off; v.ioff = bm.fhi_off;
    v.fw = bm.fh_fw; v.bw = bm.fh_bw;
    v.sx = bm.mx; v.sy = bm.my; v.sz = bm.mz;
    v.ox = v.oy = v.oz = 0;
    v.doff = bm.fh_off;
    v.dstride = (int64_t)bm.bth * MSG_TILE2;
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

}  // namespace msg
