// Host-side choice of the channel split of a matcher launch's last round
// (see SplitArgs in kernels.hpp).  Host-only and free of HIP types, so that
// it can be tested on the CPU.
#pragma once
#include <stddef.h>
#include <algorithm>

namespace cfog {

struct SplitChoice {
  int n_whole;  // tasks [0, n_whole) run whole
  int G;        // channel groups of each later task (1: no split)
  int slot;     // floats per partial surface (K^2 rounded up to 64)
  size_t bytes; // workspace bytes of the partial surfaces (256-byte multiple)
};

// n tasks on S workgroup slots with m channels and an FFT side P; (Nmax,
// Wsmax, Kmax) bound the tasks' template, window and surface sides.  The
// last round of a launch leaves S - (n mod S) slots idle; its tasks may each
// run as G items over the channel groups [g m / G, (g+1) m / G).  G minimises
// a cost counted in 1-D FFTs of length P: per channel the row FFTs of
// template and window (two rows per FFT) and the column FFTs of both
// half-spectra; per item the inverse and the epilogue; a split pays a fixed
// 5% of a whole task for the reduce launch.  Split items are kept within two
// rounds of slots.
inline SplitChoice plan_split_choice(int P, int n, int S, int m, int Nmax, int Wsmax, int Kmax) {
  SplitChoice sp{n, 1, 0, 0};
  if (m < 2 || n <= 0 || S <= 0) return sp;
  const int q = n / S, rem = n % S;
  if (rem == 0) return sp;
  const int PH = P / 2 + 1;
  const double cf = (Nmax + 1) / 2 + (Wsmax + 1) / 2 + 2.0 * PH;
  const double ci = PH + (Kmax + 1) / 2;
  auto cost = [&](int G) { return ((m + G - 1) / G) * cf + ci; };
  double best = (q + 1) * cost(1);
  int bestG = 1;
  for (int G = 2; G <= std::min(m, 16) && (long)rem * G <= 2L * S; ++G) {
    const double t = q * cost(1) + ((rem * G + S - 1) / S) * cost(G) + 0.05 * cost(1);
    if (t < best) {
      best = t;
      bestG = G;
    }
  }
  if (bestG == 1) return sp;
  sp.n_whole = n - rem;
  sp.G = bestG;
  sp.slot = (Kmax * Kmax + 63) / 64 * 64;
  sp.bytes = (sizeof(float) * (size_t)rem * bestG * sp.slot + 255) / 256 * 256;
  return sp;
}

}  // namespace cfog
