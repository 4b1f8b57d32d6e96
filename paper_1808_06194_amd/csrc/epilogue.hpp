// SSD assembly (Eq. 5 of Ye et al.) from a correlation surface held in LDS,
// with the energy terms from FP64 summed-area tables, optional surface output
// and the lexicographic argmin / second-best of Eq. 4 (or, for the objective
// of Eq. 7, of the negated correlation), plus the optional sub-pixel
// refinement of the best offset.  Shared by the FFT and the direct (MFMA)
// matchers.
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>
#include "kernels.hpp"

namespace cfog {

// Loads and stores through global-address-space pointers.  Device pointers
// that reach a kernel inside job records have no known address space, so the
// compiler would issue flat accesses, which also count as LDS operations:
// every wait on LDS traffic would then wait for them too (the matchers'
// prefetched volume rows, the energies, the surface stores).
__device__ __forceinline__ float ldg(const float* p) {
  return *(const __attribute__((address_space(1))) float*)p;
}
__device__ __forceinline__ double ldg(const double* p) {
  return *(const __attribute__((address_space(1))) double*)p;
}
__device__ __forceinline__ void stg(float* p, float v) { *(__attribute__((address_space(1))) float*)p = v; }

struct ArgminState {
  float bv;  // best value
  int bi;    // its row-major index (u_y * K + u_x)
  float sv;  // smallest value among all other indices
  int bad;   // a non-finite value was seen
};

__device__ __forceinline__ void am_push(ArgminState& s, float v, int i) {
  if (!(v == v) || fabsf(v) == INFINITY) { s.bad = 1; return; }
  if (v < s.bv || (v == s.bv && i < s.bi)) {
    s.sv = fminf(s.sv, s.bv);
    s.bv = v;
    s.bi = i;
  } else {
    s.sv = fminf(s.sv, v);
  }
}

__device__ __forceinline__ void am_merge(ArgminState& s, const ArgminState& o) {
  s.bad |= o.bad;
  if (o.bv < s.bv || (o.bv == s.bv && o.bi < s.bi)) {
    s.sv = fminf(fminf(s.sv, s.bv), o.sv);
    s.bv = o.bv;
    s.bi = o.bi;
  } else {
    s.sv = fminf(s.sv, fminf(o.bv, o.sv));
  }
}

// Sum of Q over an n x n box with top-left (y0, x0) from its SAT (row stride ld).
__device__ __forceinline__ double box_sum(const double* sat, int ld, int y0, int x0, int n) {
  const double* a = sat + (size_t)y0 * ld + x0;
  const double* b = a + (size_t)n * ld;
  return (ldg(b + n) - ldg(a + n)) - (ldg(b) - ldg(a));
}

// Abscissa, relative to the middle sample, of the vertex of the parabola
// through (-1, a), (0, b), (1, c); 0 unless the samples are convex.
__device__ __forceinline__ double parabola_vertex(double a, double b, double c) {
  const double den = a - 2.0 * b + c;
  return den > 0.0 ? 0.5 * (a - c) / den : 0.0;
}

// Writes the result of control point cpi of job jd from the correlation
// Cs[u_y * K + u_x] (LDS, all K*K values visible to the workgroup):
//   SSD(u) = E1 + E2(u) - 2 C(u), summed in FP64 and rounded to FP32
//   (objective of Eq. 7: -C(u) instead, without the energies),
// surfaces (if requested), argmin (ties to the smallest index), the smallest
// other value and (if requested) the best offset refined per axis by the
// parabola through the best value and its axis neighbours.  (tx0, ty0):
// template top-left in A; (sx0, sy0): search-window top-left in B.
// red: NT/64 ArgminState of LDS scratch.
template <int NT>
__device__ __forceinline__ void ssd_epilogue(const MatchJob& jd, int cpi, int tx0, int ty0, int sx0, int sy0,
                                             const float* Cs, ArgminState* red) {
  const int N = jd.N, r = jd.r, K = 2 * r + 1;
  const bool corr = jd.obj != 0;
  ArgminState st{INFINITY, INT_MAX, INFINITY, 0};
  const double E1 = corr ? 0.0 : box_sum(jd.satA, jd.wA + 1, ty0, tx0, N);
  const int ldB = jd.wB + 1;
  auto value = [&](int idx) -> float {
    if (corr) return -Cs[idx];
    const int uy = idx / K, ux = idx - uy * K;
    const double E2 = box_sum(jd.satB, ldB, sy0 + uy, sx0 + ux, N);
    return (float)(E1 + E2 - 2.0 * (double)Cs[idx]);
  };
  float* surf = jd.surfaces ? jd.surfaces + (size_t)cpi * K * K : nullptr;
  for (int idx = threadIdx.x; idx < K * K; idx += NT) {
    const float s = value(idx);
    am_push(st, s, idx);
    if (surf) stg(surf + idx, s);
  }
  // wave reduction then across waves
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ArgminState t;
    t.bv = __shfl_xor(st.bv, o, 64);
    t.bi = __shfl_xor(st.bi, o, 64);
    t.sv = __shfl_xor(st.sv, o, 64);
    t.bad = __shfl_xor(st.bad, o, 64);
    am_merge(st, t);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = st;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < NT / 64; ++i) am_merge(st, red[i]);
    Result* res = jd.out + cpi;
    if (st.bad) {
      *res = Result{0, 0, NAN, NAN, kCpNonFinite, 0};
      if (jd.subpix) jd.subpix[cpi] = make_float2(NAN, NAN);
    } else {
      const int uy = st.bi / K, ux = st.bi - uy * K;
      *res = Result{ux - r, uy - r, st.bv, st.sv, kCpOk, 0};
      if (jd.subpix) {
        // the same FP32 values as the surface output
        float fx = (float)(ux - r), fy = (float)(uy - r);
        if (ux > 0 && ux < K - 1)
          fx += (float)parabola_vertex(value(st.bi - 1), st.bv, value(st.bi + 1));
        if (uy > 0 && uy < K - 1)
          fy += (float)parabola_vertex(value(st.bi - K), st.bv, value(st.bi + K));
        jd.subpix[cpi] = make_float2(fx, fy);
      }
    }
  }
}

// Out-of-bounds control point: status, NaN surface.
template <int NT>
__device__ __forceinline__ void oob_result(const MatchJob& jd, int cpi) {
  const int K = 2 * jd.r + 1;
  if (threadIdx.x == 0) {
    jd.out[cpi] = Result{0, 0, NAN, NAN, kCpOutOfBounds, 0};
    if (jd.subpix) jd.subpix[cpi] = make_float2(NAN, NAN);
  }
  if (jd.surfaces) {
    float* s = jd.surfaces + (size_t)cpi * K * K;
    for (int i = threadIdx.x; i < K * K; i += NT) s[i] = NAN;
  }
}

}  // namespace cfog
