// Window test of a control point (Section III-G, Eq. 3): the template box of
// side N at (x, y) - floor(N/2) must lie inside A and the search box of side
// N + 2r at (bx, by) - floor(N/2) - r inside B.  Shared by every matcher
// kernel and by the server's host-side check of submitted points, and built
// for the host by a sanitizer test.
//
// Every sum is formed in 64 bits from 32-bit operands, so no control point,
// template side or radius that fits an int32 can wrap past the test: a point
// near INT_MIN or INT_MAX is simply outside.
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#define CFOG_HD __host__ __device__
#else
#define CFOG_HD
#endif

namespace cfog {

// Whether [lo, lo + n) lies inside [0, size).
CFOG_HD inline bool span_inside(int64_t lo, int64_t n, int64_t size) { return lo >= 0 && n >= 0 && lo + n <= size; }

// Top-left corners of a control point's template box in A (tx0, ty0) and
// search box in B (sx0, sy0), and whether both boxes lie inside their images.
// The corners are only meaningful when `inside` is true; they then fit an int.
struct CpBoxes {
  int tx0, ty0, sx0, sy0;
  bool inside;
};

CFOG_HD inline CpBoxes cp_boxes(int32_t x, int32_t y, int32_t bx, int32_t by, int32_t N, int32_t r, int32_t hA,
                                int32_t wA, int32_t hB, int32_t wB) {
  const int64_t h = (int64_t)(N / 2), rr = r, n = N, ws = (int64_t)N + 2 * rr;
  const int64_t tx0 = (int64_t)x - h, ty0 = (int64_t)y - h;
  const int64_t sx0 = (int64_t)bx - h - rr, sy0 = (int64_t)by - h - rr;
  CpBoxes b;
  b.inside = N >= 1 && r >= 0 && span_inside(tx0, n, wA) && span_inside(ty0, n, hA) && span_inside(sx0, ws, wB) &&
             span_inside(sy0, ws, hB);
  b.tx0 = b.inside ? (int)tx0 : 0;
  b.ty0 = b.inside ? (int)ty0 : 0;
  b.sx0 = b.inside ? (int)sx0 : 0;
  b.sy0 = b.inside ? (int)sy0 : 0;
  return b;
}

}  // namespace cfog
