// SSD template matching of control points in the frequency domain
// (Section III-G of Ye et al.: Eqs. 3-6 and 8-9), one workgroup per control
// point, everything on chip.
//
// For control point (x, y) in A with search centre (bx, by) in B, template side
// N, radius r, h = N/2, K = 2r+1, Ws = N + 2r:
//   T_c  = D_A[c][y-h .. y-h+N)[x-h .. x-h+N)               (template)
//   S_c  = D_B[c][by-h-r .. +Ws)[bx-h-r .. +Ws)              (search window)
//   C(u) = sum_c sum_q T_c(q) S_c(q+u),  u in [0, 2r]^2        (correlation)
//   SSD(d) = E1 + E2(d) - 2 C(d + r)                          (Eq. 5)
// with E1, E2 from the FP64 summed-area tables and d = u - r the returned
// offset of B's window relative to the search centre.
//
// The orientation axis of Eq. 9's 3-D transform is only ever read back at
// zero orientation shift, where the orientation DFT / inverse DFT pair reduces
// (Parseval) to a plain sum over channels of 2-D spectral products.  So each
// channel goes through real 2-D FFTs of size P x P (P >= Ws):
//   x-pass: rows of T_c (or S_c), two real rows packed per complex FFT;
//   y-pass: complex column FFTs of the half-spectrum kx in [0, P/2], with the
//           two packed rows separated on load via Z(k) / conj Z(-k);
//   ACC(ky, kx) += conj(T^_c) * S^_c  (registers; T^_c is parked in registers
//           between the T and S passes of the channel);
// then one inverse: column IFFTs (kept rows u_y < K) and a C2R row IFFT with
// two output rows packed per complex FFT (kept columns u_x < K), the SSD
// assembly in FP64, and a lexicographic argmin + second-best over (SSD, index).
//
// 1-D FFTs of length P = R1 * R2 are two radix stages in LDS:
//   stage 1: t[b R1 + k1] = sum_a x[b + R2 a] W_R1^{a k1}         (b < R2)
//   stage 2: X[k1 + R1 k2] = sum_b W_P^{k1 b} t[b R1 + k1] W_R2^{b k2}
// with the small DFTs as unrolled register codelets (dft.hpp).
#include <hip/hip_runtime.h>
#include <float.h>
#include <limits.h>
#include "dft.hpp"
#include "kernels.hpp"

namespace cfog {

template <int P_, int R1_, int R2_, int NT_>
struct FftCfg {
  static constexpr int P = P_, R1 = R1_, R2 = R2_, NT = NT_;
  static_assert(P == R1 * R2, "P must equal R1 * R2");
  static constexpr int PH = P / 2 + 1;
  static constexpr int NB_Y1 = PH * R2;  // column-FFT stage-1 butterflies (radix R1)
  static constexpr int NB_Y2 = PH * R1;  // column-FFT stage-2 butterflies (radix R2)
  static constexpr int KS1 = (NB_Y1 + NT - 1) / NT;
  static constexpr int KF = (NB_Y2 + NT - 1) / NT;
  static constexpr int NW = NT / 64;
  static constexpr size_t LDS = sizeof(float2) * ((size_t)P * PH + P) + NW * 16;
};

struct ArgminState {
  float bv;
  int bi;
  float sv;
  int bad;
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

__device__ __forceinline__ double box_sum(const double* sat, int ld, int y0, int x0, int n) {
  const double* a = sat + (size_t)y0 * ld + x0;
  const double* b = a + (size_t)n * ld;
  return (b[n] - a[n]) - (b[0] - a[0]);
}

// x-pass: forward FFT of nrows x ncols real rows (src, leading dim ld),
// zero-padded to P, two rows per complex FFT.  Row pair q's spectrum Z_q(k),
// k in [0, P), is left at X[2q*PH + k].
template <class C>
__device__ __forceinline__ void xpass_fwd(const float* __restrict__ src, int64_t ld, int nrows, int ncols,
                                          float2* X, const float2* tw) {
  constexpr int P = C::P, R1 = C::R1, R2 = C::R2, PH = C::PH, NT = C::NT;
  const int nrp = (nrows + 1) >> 1;
  for (int b = threadIdx.x; b < nrp * R2; b += NT) {
    const int q = b / R2, j = b - q * R2;
    const float* r0 = src + (int64_t)(2 * q) * ld;
    const bool has1 = (2 * q + 1) < nrows;
    float2 v[R1];
#pragma unroll
    for (int a = 0; a < R1; ++a) {
      const int xx = j + R2 * a;
      float re = 0.f, im = 0.f;
      if (xx < ncols) {
        re = r0[xx];
        if (has1) im = r0[ld + xx];
      }
      v[a] = make_float2(re, im);
    }
    dft<R1, -1>(v);
    float2* dst = X + 2 * q * PH + j * R1;
#pragma unroll
    for (int k = 0; k < R1; ++k) dst[k] = v[k];
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nrp * R1; b += NT) {
    const int q = b / R1, k1 = b - q * R1;
    float2* base = X + 2 * q * PH + k1;
    float2 v[R2];
    v[0] = base[0];
#pragma unroll
    for (int bb = 1; bb < R2; ++bb) v[bb] = cmul(base[R1 * bb], tw[k1 * bb]);
    dft<R2, -1>(v);
#pragma unroll
    for (int k = 0; k < R2; ++k) base[R1 * k] = v[k];
  }
  __syncthreads();
}

// y-pass: forward column FFTs of the half-spectrum (kx in [0, P/2]) of the rows
// left by xpass_fwd; rows >= nrows are zero.  Output ownership: butterfly
// b = threadIdx.x + k*NT owns ky = k1 + R1*k2 of column kx = b % PH,
// k1 = b / PH; each value is handed to sink(k, k2, value).
template <class C, class Sink>
__device__ __forceinline__ void ypass_fwd(int nrows, float2* X, const float2* tw, Sink&& sink) {
  constexpr int P = C::P, R1 = C::R1, R2 = C::R2, PH = C::PH, NT = C::NT;
  float2 v[C::KS1][R1];
#pragma unroll
  for (int k = 0; k < C::KS1; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < C::NB_Y1) {
      const int kx = b % PH, j = b / PH;
      const int km = (kx == 0) ? 0 : P - kx;
#pragma unroll
      for (int a = 0; a < R1; ++a) {
        const int y = j + R2 * a;
        float2 val = make_float2(0.f, 0.f);
        if (y < nrows) {
          const float2* zq = X + (y & ~1) * PH;
          const float2 z1 = zq[kx], z2 = zq[km];
          // A(k) = (Z(k) + conj Z(-k)) / 2 ;  B(k) = (Z(k) - conj Z(-k)) / 2i
          val = (y & 1) ? make_float2(0.5f * (z1.y + z2.y), 0.5f * (z2.x - z1.x))
                        : make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
        }
        v[k][a] = val;
      }
      dft<R1, -1>(v[k]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < C::KS1; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < C::NB_Y1) {
      const int kx = b % PH, j = b / PH;
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) X[(j * R1 + k1) * PH + kx] = v[k][k1];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < C::KF; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < C::NB_Y2) {
      const int kx = b % PH, k1 = b / PH;
      float2 w[R2];
      w[0] = X[k1 * PH + kx];
#pragma unroll
      for (int bb = 1; bb < R2; ++bb) w[bb] = cmul(X[(k1 + R1 * bb) * PH + kx], tw[k1 * bb]);
      dft<R2, -1>(w);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) sink(k, k2, w[k2]);
    }
  }
}

template <class C>
__device__ void match_one(const MatchJob& jd, int cpi, float2* X, float2* tw, ArgminState* red) {
  constexpr int P = C::P, R1 = C::R1, R2 = C::R2, PH = C::PH, NT = C::NT, KF = C::KF;
  const int4 cp = jd.cps[cpi];
  const int N = jd.N, r = jd.r, K = 2 * r + 1, h = N / 2, Ws = N + 2 * r;
  const int tx0 = cp.x - h, ty0 = cp.y - h;
  const int sx0 = cp.z - h - r, sy0 = cp.w - h - r;
  Result* res = jd.out + cpi;
  const bool inA = tx0 >= 0 && ty0 >= 0 && tx0 + N <= jd.wA && ty0 + N <= jd.hA;
  const bool inB = sx0 >= 0 && sy0 >= 0 && sx0 + Ws <= jd.wB && sy0 + Ws <= jd.hB;
  if (!(inA && inB)) {
    if (threadIdx.x == 0) *res = Result{0, 0, NAN, NAN, kCpOutOfBounds, 0};
    if (jd.surfaces) {
      float* s = jd.surfaces + (size_t)cpi * K * K;
      for (int i = threadIdx.x; i < K * K; i += NT) s[i] = NAN;
    }
    return;
  }

  float2 acc[KF][R2];
#pragma unroll
  for (int k = 0; k < KF; ++k)
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) acc[k][k2] = make_float2(0.f, 0.f);

  const size_t planeA = (size_t)jd.hA * jd.wA, planeB = (size_t)jd.hB * jd.wB;
  for (int c = 0; c < jd.m; ++c) {
    float2 th[KF][R2];
    __syncthreads();
    xpass_fwd<C>(jd.volA + c * planeA + (size_t)ty0 * jd.wA + tx0, jd.wA, N, N, X, tw);
    ypass_fwd<C>(N, X, tw, [&](int k, int k2, float2 v) { th[k][k2] = v; });
    __syncthreads();
    xpass_fwd<C>(jd.volB + c * planeB + (size_t)sy0 * jd.wB + sx0, jd.wB, Ws, Ws, X, tw);
    ypass_fwd<C>(Ws, X, tw, [&](int k, int k2, float2 v) { acc[k][k2] = cmac_conj(acc[k][k2], th[k][k2], v); });
  }

  // ---- inverse: columns (ky -> u_y), keep rows u_y < K
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KF; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < C::NB_Y2) {
      const int kx = b % PH, k1 = b / PH;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) X[(k1 + R1 * k2) * PH + kx] = acc[k][k2];
    }
  }
  __syncthreads();
  {
    float2 v[C::KS1][R1];
#pragma unroll
    for (int k = 0; k < C::KS1; ++k) {
      const int b = threadIdx.x + k * NT;
      if (b < C::NB_Y1) {
        const int kx = b % PH, j = b / PH;
#pragma unroll
        for (int a = 0; a < R1; ++a) v[k][a] = X[(j + R2 * a) * PH + kx];
        dft<R1, +1>(v[k]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < C::KS1; ++k) {
      const int b = threadIdx.x + k * NT;
      if (b < C::NB_Y1) {
        const int kx = b % PH, j = b / PH;
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) X[(j * R1 + k1) * PH + kx] = v[k][k1];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < KF; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < C::NB_Y2) {
      const int kx = b % PH, k1 = b / PH;
      float2 w[R2];
      w[0] = X[k1 * PH + kx];
#pragma unroll
      for (int bb = 1; bb < R2; ++bb) {
        const float2 t = tw[k1 * bb];
        w[bb] = cmul(X[(k1 + R1 * bb) * PH + kx], make_float2(t.x, -t.y));
      }
      dft<R2, +1>(w);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int uy = k1 + R1 * k2;
        if (uy < K) X[uy * PH + kx] = w[k2];
      }
    }
  }
  __syncthreads();

  // ---- inverse: rows (kx -> u_x), two real output rows per complex FFT
  const int npair = (K + 1) >> 1;
  float2* SC = X + K * PH;
  for (int b = threadIdx.x; b < npair * R2; b += NT) {
    const int p = b / R2, j = b - p * R2;
    const float2* v1r = X + (2 * p) * PH;
    const bool has2 = 2 * p + 1 < K;
    float2 v[R1];
#pragma unroll
    for (int a = 0; a < R1; ++a) {
      const int kx = j + R2 * a;
      const bool lo = kx <= P / 2;
      const int kk = lo ? kx : P - kx;
      const float2 v1 = v1r[kk];
      const float2 v2 = has2 ? v1r[PH + kk] : make_float2(0.f, 0.f);
      v[a] = lo ? make_float2(v1.x - v2.y, v1.y + v2.x) : make_float2(v1.x + v2.y, v2.x - v1.y);
    }
    dft<R1, +1>(v);
    float2* dst = SC + p * P + j * R1;
#pragma unroll
    for (int k = 0; k < R1; ++k) dst[k] = v[k];
  }
  __syncthreads();

  ArgminState st{INFINITY, INT_MAX, INFINITY, 0};
  const double E1 = box_sum(jd.satA, jd.wA + 1, ty0, tx0, N);
  const int ldB = jd.wB + 1;
  const double inv = 1.0 / ((double)P * (double)P);
  float* surf = jd.surfaces ? jd.surfaces + (size_t)cpi * K * K : nullptr;
  for (int b = threadIdx.x; b < npair * R1; b += NT) {
    const int p = b / R1, k1 = b - p * R1;
    const float2* base = SC + p * P + k1;
    float2 w[R2];
    w[0] = base[0];
#pragma unroll
    for (int bb = 1; bb < R2; ++bb) {
      const float2 t = tw[k1 * bb];
      w[bb] = cmul(base[R1 * bb], make_float2(t.x, -t.y));
    }
    dft<R2, +1>(w);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      const int ux = k1 + R1 * k2;
      if (ux < K) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int uy = 2 * p + e;
          if (uy < K) {
            const double cval = (double)(e ? w[k2].y : w[k2].x) * inv;
            const double E2 = box_sum(jd.satB, ldB, sy0 + uy, sx0 + ux, N);
            const float s = (float)(E1 + E2 - 2.0 * cval);
            const int idx = uy * K + ux;
            am_push(st, s, idx);
            if (surf) surf[idx] = s;
          }
        }
      }
    }
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
    for (int i = 1; i < C::NW; ++i) am_merge(st, red[i]);
    if (st.bad) {
      *res = Result{0, 0, NAN, NAN, kCpNonFinite, 0};
    } else {
      const int uy = st.bi / K, ux = st.bi - uy * K;
      *res = Result{ux - r, uy - r, st.bv, st.sv, kCpOk, 0};
    }
  }
}

template <class C>
__device__ __forceinline__ void init_twiddles(float2* tw) {
  for (int k = threadIdx.x; k < C::P; k += C::NT) {
    double s, c;
    sincospi(2.0 * k / C::P, &s, &c);
    tw[k] = make_float2((float)c, (float)-s);
  }
}

template <class C>
__global__ __launch_bounds__(C::NT) void match_fft_plain_kernel(MatchJob jd) {
  extern __shared__ float2 smem[];
  float2* X = smem;
  float2* tw = X + C::P * C::PH;
  ArgminState* red = reinterpret_cast<ArgminState*>(tw + C::P);
  init_twiddles<C>(tw);
  __syncthreads();
  match_one<C>(jd, blockIdx.x, X, tw, red);
}

template <class C>
__global__ __launch_bounds__(C::NT) void match_fft_tasks_kernel(const MatchJob* __restrict__ jobs,
                                                                const int2* __restrict__ tasks, int n_tasks) {
  extern __shared__ float2 smem[];
  float2* X = smem;
  float2* tw = X + C::P * C::PH;
  ArgminState* red = reinterpret_cast<ArgminState*>(tw + C::P);
  init_twiddles<C>(tw);
  __syncthreads();
  for (int t = blockIdx.x; t < n_tasks; t += gridDim.x) {
    const int2 tk = tasks[t];
    const MatchJob jd = jobs[tk.x];
    match_one<C>(jd, tk.y, X, tw, red);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ plans
#define CFOG_PLANS(X)  \
  X(16, 4, 4, 64)      \
  X(24, 4, 6, 128)     \
  X(32, 4, 8, 128)     \
  X(40, 5, 8, 256)     \
  X(48, 6, 8, 256)     \
  X(64, 8, 8, 256)     \
  X(72, 8, 9, 256)     \
  X(80, 8, 10, 512)    \
  X(96, 8, 12, 512)    \
  X(100, 10, 10, 512)  \
  X(120, 10, 12, 1024) \
  X(128, 8, 16, 1024)  \
  X(144, 12, 12, 1024) \
  X(160, 10, 16, 1024)

static const FftPlan kPlans[] = {
#define CFOG_PLAN_ENTRY(P, R1, R2, NT) {P, R1, R2, NT, FftCfg<P, R1, R2, NT>::LDS},
    CFOG_PLANS(CFOG_PLAN_ENTRY)
#undef CFOG_PLAN_ENTRY
};

const FftPlan* fft_plans(int* count) {
  *count = (int)(sizeof(kPlans) / sizeof(kPlans[0]));
  return kPlans;
}

const FftPlan* choose_fft_plan(int N, int r) {
  const int Ws = N + 2 * r, K = 2 * r + 1;
  for (const FftPlan& p : kPlans) {
    if (p.P < Ws) continue;
    const int PH = p.P / 2 + 1;
    if ((long)((K + 1) / 2) * p.P > (long)(p.P - K) * PH) continue;  // inverse row scratch
    return &p;
  }
  return nullptr;
}

template <class C>
static int launch_plain_t(const MatchJob& job, hipStream_t st) {
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)match_fft_plain_kernel<C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)C::LDS) != hipSuccess)
      return -2;
    attr_set = true;
  }
  hipLaunchKernelGGL(match_fft_plain_kernel<C>, dim3(job.n_cps), dim3(C::NT), C::LDS, st, job);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <class C>
static int launch_tasks_t(const MatchJob* jobs, const int2* tasks, int n_tasks, int n_blocks, hipStream_t st) {
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)match_fft_tasks_kernel<C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)C::LDS) != hipSuccess)
      return -2;
    attr_set = true;
  }
  hipLaunchKernelGGL(match_fft_tasks_kernel<C>, dim3(n_blocks), dim3(C::NT), C::LDS, st, jobs, tasks, n_tasks);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_match_fft_plain(const FftPlan* plan, const MatchJob& job, hipStream_t st) {
  if (job.n_cps <= 0) return 0;
#define CFOG_PLAN_CASE(P_, R1_, R2_, NT_) \
  if (plan->P == P_) return launch_plain_t<FftCfg<P_, R1_, R2_, NT_>>(job, st);
  CFOG_PLANS(CFOG_PLAN_CASE)
#undef CFOG_PLAN_CASE
  return -1;
}

int launch_match_fft_tasks(const FftPlan* plan, const MatchJob* d_jobs, const int2* d_tasks, int n_tasks,
                           int n_blocks, hipStream_t st) {
  if (n_tasks <= 0) return 0;
#define CFOG_PLAN_CASE(P_, R1_, R2_, NT_) \
  if (plan->P == P_) return launch_tasks_t<FftCfg<P_, R1_, R2_, NT_>>(d_jobs, d_tasks, n_tasks, n_blocks, st);
  CFOG_PLANS(CFOG_PLAN_CASE)
#undef CFOG_PLAN_CASE
  return -1;
}

}  // namespace cfog
