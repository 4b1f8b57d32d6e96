// Host test of the channel-split planner (split_plan.hpp).
#include <stdio.h>
#include <stdlib.h>
#include "split_plan.hpp"

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);          \
      ++failures;                                                  \
    }                                                              \
  } while (0)

int main() {
  using cfog::plan_split_choice;
  // 400 points on 256 slots (P = 144, N = 100, r = 20): the 144 points of
  // the last round run as 3 channel groups each (432 items, two half-filled
  // rounds of short items instead of one round of whole points)
  auto a = plan_split_choice(144, 400, 256, 9, 100, 140, 41);
  CHECK(a.n_whole == 256 && a.G == 3);
  CHECK(a.slot == (41 * 41 + 63) / 64 * 64 && a.slot % 64 == 0 && a.slot >= 41 * 41);
  CHECK(a.bytes == (4u * 144 * 3 * a.slot + 255) / 256 * 256);
  // a multiple of the slots: no last round to fill
  auto b = plan_split_choice(144, 512, 256, 9, 100, 140, 41);
  CHECK(b.G == 1 && b.n_whole == 512 && b.bytes == 0);
  // fewer points than slots: every point splits, up to one group per channel
  auto c = plan_split_choice(72, 16, 512, 9, 48, 68, 21);
  CHECK(c.n_whole == 0 && c.G == 9);
  // one channel cannot split; nor can an empty launch
  CHECK(plan_split_choice(144, 10, 256, 1, 100, 140, 41).G == 1);
  CHECK(plan_split_choice(144, 0, 256, 9, 100, 140, 41).G == 1);
  // the split items stay within two rounds of slots, and a split never
  // models slower than the whole last round
  for (int n = 1; n <= 2000; n += 7) {
    for (int m : {2, 3, 9, 16, 36}) {
      auto s = plan_split_choice(144, n, 256, m, 100, 140, 41);
      CHECK(s.G >= 1 && s.G <= (m < 16 ? m : 16));
      CHECK(s.n_whole >= 0 && s.n_whole <= n);
      if (s.G > 1) {
        CHECK(s.n_whole == n - n % 256);
        CHECK((long)(n - s.n_whole) * s.G <= 512);
        CHECK(s.bytes >= 4u * (size_t)(n - s.n_whole) * s.G * 41 * 41);
      } else {
        CHECK(s.n_whole == n && s.bytes == 0);
      }
    }
  }
  if (failures) return 1;
  printf("ALL OK\n");
  return 0;
}
