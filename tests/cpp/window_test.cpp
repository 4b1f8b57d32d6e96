// Host test of the control-point window rule (window.hpp), built with
// -fsanitize=address,undefined: any signed overflow in the rule aborts.
//
// The reference is the rule of Eq. 3 written out over the box's pixels:
// a box is inside when its first and last pixel are valid indices of the
// image, evaluated in 128-bit arithmetic; on small images it is also
// checked against enumerating every pixel of the box.
#include <limits.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <random>
#include <vector>
#include "window.hpp"

static int failures = 0;

#define CHECK(cond, ...)                                 \
  do {                                                   \
    if (!(cond)) {                                       \
      ++failures;                                        \
      if (failures < 20) {                               \
        printf("FAIL %s:%d: ", __FILE__, __LINE__);      \
        printf(__VA_ARGS__);                             \
        printf("\n");                                    \
      }                                                  \
    }                                                    \
  } while (0)

typedef __int128 i128;

// box [lo, lo + n) inside [0, size): first pixel >= 0 and last pixel < size
static bool ref_span(i128 lo, i128 n, i128 size) { return n >= 1 && lo >= 0 && lo + n - 1 <= size - 1; }

static bool ref_inside(int32_t x, int32_t y, int32_t bx, int32_t by, int32_t N, int32_t r, int32_t hA, int32_t wA,
                       int32_t hB, int32_t wB) {
  if (N < 1 || r < 0) return false;
  const i128 h = N / 2;
  return ref_span((i128)x - h, N, wA) && ref_span((i128)y - h, N, hA) && ref_span((i128)bx - h - r, (i128)N + 2 * (i128)r, wB) &&
         ref_span((i128)by - h - r, (i128)N + 2 * (i128)r, hB);
}

// every pixel of the box is an index of the image (small sizes only)
static bool enum_span(int64_t lo, int64_t n, int64_t size) {
  if (n < 1) return false;
  for (int64_t i = lo; i < lo + n; ++i)
    if (i < 0 || i >= size) return false;
  return true;
}

static void check(int32_t x, int32_t y, int32_t bx, int32_t by, int32_t N, int32_t r, int32_t hA, int32_t wA,
                  int32_t hB, int32_t wB) {
  const cfog::CpBoxes b = cfog::cp_boxes(x, y, bx, by, N, r, hA, wA, hB, wB);
  const bool ref = ref_inside(x, y, bx, by, N, r, hA, wA, hB, wB);
  CHECK(b.inside == ref, "cp (%d,%d,%d,%d) N=%d r=%d A=%dx%d B=%dx%d: got %d want %d", x, y, bx, by, N, r, hA, wA,
        hB, wB, (int)b.inside, (int)ref);
  if (b.inside) {
    const int h = N / 2;
    CHECK(b.tx0 == x - h && b.ty0 == y - h && b.sx0 == bx - h - r && b.sy0 == by - h - r, "corners");
    CHECK(b.tx0 >= 0 && b.tx0 + N <= wA && b.sy0 >= 0 && (int64_t)b.sy0 + N + 2 * (int64_t)r <= hB, "corner range");
  }
}

int main() {
  const int32_t ext[] = {INT_MIN, INT_MIN + 1, INT_MIN / 2, -65536, -1000, -1, 0, 1, 2, 1000, 65536,
                         INT_MAX / 2, INT_MAX - 1, INT_MAX};
  // extreme coordinates against images of several sizes, with every
  // combination of extreme values in one coordinate and sane ones elsewhere
  const int32_t Ns[] = {1, 2, 7, 8, 48, 100, 128, 65536};
  const int32_t rs[] = {0, 1, 10, 32, 65536};
  const int32_t sizes[] = {1, 64, 2048, INT_MAX};
  for (int32_t N : Ns)
    for (int32_t r : rs)
      for (int32_t S : sizes) {
        const int32_t mid = S / 2;
        for (int32_t v : ext) {
          check(v, mid, mid, mid, N, r, S, S, S, S);
          check(mid, v, mid, mid, N, r, S, S, S, S);
          check(mid, mid, v, mid, N, r, S, S, S, S);
          check(mid, mid, mid, v, N, r, S, S, S, S);
          check(v, v, v, v, N, r, S, S, S, S);
        }
        // +-h and +-r around the flush positions of every edge
        const int32_t h = N / 2;
        const int64_t cand[] = {h - 1, h, h + 1, (int64_t)h + r - 1, (int64_t)h + r, (int64_t)h + r + 1,
                                (int64_t)S - N + h - 1, (int64_t)S - N + h, (int64_t)S - N + h + 1,
                                (int64_t)S - N + h - r - 1, (int64_t)S - N + h - r, (int64_t)S - N + h - r + 1,
                                -(int64_t)h, -(int64_t)r};
        for (int64_t c : cand) {
          if (c < INT_MIN || c > INT_MAX) continue;
          const int32_t v = (int32_t)c;
          check(v, mid, mid, mid, N, r, S, S, S, S);
          check(mid, v, mid, mid, N, r, S, S, S, S);
          check(mid, mid, v, mid, N, r, S, S, S, S);
          check(mid, mid, mid, v, N, r, S, S, S, S);
        }
      }
  // invalid template sides and radii are never inside
  check(10, 10, 10, 10, 0, 1, 64, 64, 64, 64);
  check(10, 10, 10, 10, -5, 1, 64, 64, 64, 64);
  check(10, 10, 10, 10, 4, -1, 64, 64, 64, 64);
  check(10, 10, 10, 10, INT_MIN, INT_MAX, 64, 64, 64, 64);
  check(10, 10, 10, 10, INT_MAX, INT_MAX, INT_MAX, INT_MAX, INT_MAX, INT_MAX);

  // small images: every position of both boxes against pixel enumeration,
  // for even and odd N, with A and B of different sizes
  for (int32_t N = 1; N <= 6; ++N)
    for (int32_t r = 0; r <= 3; ++r)
      for (int32_t x = -4; x <= 16; ++x)
        for (int32_t bx = -6; bx <= 18; ++bx) {
          const int32_t hA = 9, wA = 11, hB = 13, wB = 12;
          const int32_t y = 5, by = 6;
          const cfog::CpBoxes b = cfog::cp_boxes(x, y, bx, by, N, r, hA, wA, hB, wB);
          const int64_t h = N / 2;
          const bool e = enum_span(x - h, N, wA) && enum_span(y - h, N, hA) && enum_span(bx - h - r, N + 2 * r, wB) &&
                         enum_span(by - h - r, N + 2 * r, hB);
          CHECK(b.inside == e, "enum N=%d r=%d x=%d bx=%d: got %d want %d", N, r, x, bx, (int)b.inside, (int)e);
          // the transposed case exercises the row tests
          const cfog::CpBoxes t = cfog::cp_boxes(y, x, by, bx, N, r, wA, hA, wB, hB);
          const bool et = enum_span(x - h, N, wA) && enum_span(y - h, N, hA) &&
                          enum_span(bx - h - r, N + 2 * r, wB) && enum_span(by - h - r, N + 2 * r, hB);
          CHECK(t.inside == et, "enum transposed N=%d r=%d", N, r);
        }

  // random int32 values
  std::mt19937_64 rng(12345);
  std::uniform_int_distribution<int64_t> any(INT_MIN, INT_MAX), small(-300, 300), side(1, 300), rad(0, 40);
  for (int i = 0; i < 2000000; ++i) {
    const bool wild = (i & 3) == 0;
    auto pick = [&]() { return (int32_t)(wild ? any(rng) : small(rng)); };
    check(pick(), pick(), pick(), pick(), (int32_t)side(rng), (int32_t)rad(rng), (int32_t)side(rng),
          (int32_t)side(rng), (int32_t)side(rng), (int32_t)side(rng));
  }
  if (failures) {
    printf("%d failures\n", failures);
    return 1;
  }
  printf("ALL OK\n");
  return 0;
}
