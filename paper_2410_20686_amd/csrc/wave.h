// Cross-lane helpers of the compositing kernels (64-wide CDNA wavefronts, gfx950 DPP and
// row-swap permutes) and the thread-to-pixel map of a tile.
#pragma once

#include "common.h"

namespace odgs {

template <int CTRL>
__device__ inline float dpp_read(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Exchange step of a multi-value butterfly: the lane keeps `lo` or `hi` (by `bit`) and adds the
// partner's copy of the same slot; the partner (reached with DPP control CTRL) has the opposite
// `bit` and holds the same slot meanings.
template <int CTRL>
__device__ inline float bfly(float lo, float hi, bool bit) {
  return (bit ? hi : lo) + dpp_read<CTRL>(bit ? lo : hi);
}

// Sum of a value over the four 16-lane rows of the wavefront, returned in every row: the gfx950
// row-swap permutes (lanes 32-63 <-> 0-31, then odd <-> even rows) need no LDS traffic.
__device__ inline float sum_rows(float x) {
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  const float y = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(y), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Pixel of a thread inside a TILE x TILE tile: wavefront w owns quadrant w (row-major over the
// TILE/8 x TILE/8 quadrants), lane l the pixel (l % 8, l / 8) inside it.
template <int TILE>
__device__ inline void local_pixel(int t, int& lx, int& ly) {
  constexpr int QPR = TILE / 8;
  const int w = t >> 6, l = t & 63;
  lx = (w % QPR) * 8 + (l & 7);
  ly = (w / QPR) * 8 + (l >> 3);
}

}  // namespace odgs
