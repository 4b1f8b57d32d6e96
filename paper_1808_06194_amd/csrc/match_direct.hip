// Direct (spatial) evaluation of the correlation term of Eq. 5 (Ye et al.,
// Section III-G) as BF16 MFMA GEMMs with FP32 accumulation: the precision
// alternative to the FP32 FFT path.  The energies and the SSD assembly are the
// same FP64 summed-area-table epilogue as the FFT path.
//
// With T_c the template and S_c the search window of channel c,
//   C(u_y, u_x) = sum_c sum_s sum_tx  S_c(s, tx + u_x) * T_c(s - u_y, tx)
// is one GEMM per control point with
//   M = u_x  (rows of a Hankel matrix built from search row s),
//   N = u_y  (template row s - u_y, zero outside the template),
//   K = (c, s, tx)  (all channels, all search rows, the template columns),
// so every output tile of C accumulates in MFMA registers with no scatter.
// v_mfma_f32_16x16x32_bf16 tiles: M and N are padded to 16, the template
// width to 32.  Per channel the template (bf16, with 15 zero rows above and
// below) and the search window (bf16) are staged in LDS.  Every wave keeps
// all (2r+1)^2 outputs in registers (up to 5 x 5 tiles) and takes every 8th
// search row s, so per (s, 32-column chunk) it reads 5 A and at most 5 B
// fragments for up to 25 MFMAs; the waves' partial sums are added in wave
// order at the end (deterministic).  Operand fragments:
//   A (lane l, u_x block m): 8 bf16 of search row s from column
//      32kc + 8(l/16) + 16m + l%16, read as 5 aligned dwords and realigned by a
//      byte shift;
//   B (lane l, u_y block n): 8 bf16 of template row s - 16n - l%16, columns
//      32kc + 8(l/16) .. +7, one aligned 16-byte LDS read.
// Precision: inputs are rounded to BF16 (round to nearest, 8 significant bits,
// unit roundoff u = 2^-8), products are exact in FP32, so
//   |C_bf16 - C| <= [(2u + u^2) + gamma_L (1 + u)^2] sum |T S|,
// with gamma_L = L 2^-24 / (1 - L 2^-24) for the longest chain of L FP32
// additions into one output: m channels x ceil(Ws / 8) search rows of a wave x
// ceil(N / 32) chunks of MFMAs of 32 products each, plus the 8 wave partials.
// As sum |T S| <= sqrt(E1 E2) <= (E1 + E2) / 2 and SSD = E1 + E2 - 2C, the
// SSD surface is within [(2u + u^2) + gamma_L (1 + u)^2 + 2^-23] (E1 + E2(d))
// of the exact one (the last term is its own FP32 rounding): about 2^-7, or
// 0.0095 at N = 128, r = 32, m = 9, against ~1e-6 for the FP32 FFT path.
#include <hip/hip_runtime.h>
#include <algorithm>
#include "cfog.h"
#include "epilogue.hpp"
#include "kernels.hpp"
#include "window.hpp"

namespace cfog {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int D_NB = 5;            // max 16-wide blocks of u_x (and u_y): 2r+1 <= 80
constexpr int D_NW = 8;            // waves per workgroup
constexpr int D_NT = 64 * D_NW;
constexpr int D_TPAD = 15;         // zero template rows above and below
constexpr int D_RB = 8;            // rows staged per batch of loads
constexpr int D_PW = 4;            // waves whose partial correlations are summed together

struct DirectGeom {
  int N, r, K, nblk, NP, Ws;
  int TROWS;  // template rows staged: N + 2 * D_TPAD (row tr holds template row tr - D_TPAD)
  int TLD;    // template row stride in dwords, NP/2 + 4: an odd multiple of 4, so the
              // 16 rows one B fragment reads start in 16 different 4-bank groups
  int SLD;    // search row stride in dwords (NP + 16 nblk + 2 bf16: the fragment over-read)
  size_t t_bytes, lds;
};

static DirectGeom direct_geom(int N, int r) {
  DirectGeom g;
  g.N = N;
  g.r = r;
  g.K = 2 * r + 1;
  g.nblk = (g.K + 15) / 16;
  g.NP = (N + 31) / 32 * 32;
  g.Ws = N + 2 * r;
  g.TROWS = N + 2 * D_TPAD;
  g.TLD = g.NP / 2 + 4;
  g.SLD = (g.NP + 16 * g.nblk + 2) / 2;
  g.t_bytes = (size_t)g.TROWS * g.TLD * 4;
  const size_t sb = (size_t)g.Ws * g.SLD * 4;
  // after the channels: Cs (K x K) and D_PW partial surfaces; the epilogue's
  // argmin scratch sits behind Cs once the partials are summed
  const size_t c = (size_t)g.K * g.K * 4 * (1 + D_PW) + 16 * D_NW;
  g.lds = std::max(g.t_bytes + sb, c);
  return g;
}

__device__ __forceinline__ unsigned pack_bf16x2(float lo, float hi) {
  const __bf16 a = (__bf16)lo, b = (__bf16)hi;
  return (unsigned)__builtin_bit_cast(unsigned short, a) | ((unsigned)__builtin_bit_cast(unsigned short, b) << 16);
}

// Stage `nrows` rows of `ncols` valid fp32 values (row r at src + r * ld when
// valid(r), zeros otherwise) as packed bf16 pairs, `width` bf16 per row, into
// dst with a row stride of `ldd` dwords.  Rows r = wv, wv + NW, ...; the
// loads of D_RB rows are issued before their conversions.
template <class Valid>
__device__ __forceinline__ void stage_rows(unsigned* dst, int ldd, int nrows, int width, const float* src,
                                           size_t ld, int ncols, Valid valid, int wv, int lane) {
  for (int r0 = wv; r0 < nrows; r0 += D_NW * D_RB) {
    for (int x = 2 * lane; x < width; x += 128) {
      float a[D_RB], b[D_RB];
#pragma unroll
      for (int u = 0; u < D_RB; ++u) {
        const int r = r0 + u * D_NW;
        a[u] = b[u] = 0.f;
        if (r < nrows && valid(r)) {
          const float* p = src + (size_t)r * ld;
          if (x < ncols) a[u] = p[x];
          if (x + 1 < ncols) b[u] = p[x + 1];
        }
      }
#pragma unroll
      for (int u = 0; u < D_RB; ++u) {
        const int r = r0 + u * D_NW;
        if (r < nrows) dst[(size_t)r * ldd + x / 2] = pack_bf16x2(a[u], b[u]);
      }
    }
  }
}

template <int NB>
__global__ __launch_bounds__(D_NT) void match_direct_kernel(MatchJob jd, DirectGeom g) {
  extern __shared__ unsigned char dsm[];
  unsigned* Tl = reinterpret_cast<unsigned*>(dsm);                             // TROWS x TLD dwords
  unsigned* Sl = reinterpret_cast<unsigned*>(dsm + g.t_bytes);                 // Ws x SLD dwords
  float* Cs = reinterpret_cast<float*>(dsm);                                    // K x K, after the channels
  ArgminState* red = reinterpret_cast<ArgminState*>(dsm + (size_t)g.K * g.K * 4);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar loop control
  const int l16 = lane & 15, kg = lane >> 4;
  const int N = g.N, r = g.r, K = g.K, NP = g.NP, Ws = g.Ws;
  const size_t planeA = (size_t)jd.hA * jd.wA, planeB = (size_t)jd.hB * jd.wB;

  for (int cpi = blockIdx.x; cpi < jd.n_cps; cpi += gridDim.x) {
    const int4 cp = jd.cps[cpi];
    const CpBoxes bx = cp_boxes(cp.x, cp.y, cp.z, cp.w, N, r, jd.hA, jd.wA, jd.hB, jd.wB);
    __syncthreads();  // the previous point's epilogue is done with LDS
    if (!bx.inside) {
      oob_result<D_NT>(jd, cpi);
      continue;
    }
    const int tx0 = bx.tx0, ty0 = bx.ty0, sx0 = bx.sx0, sy0 = bx.sy0;
    // acc[m][n]: u_x block m, u_y block n; lane element q is
    // u_x = 16 m + 4 (lane / 16) + q, u_y = 16 n + lane % 16
    f32x4 acc[NB][NB];
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
      for (int n = 0; n < NB; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int c = 0; c < jd.m; ++c) {
      __syncthreads();  // MFMA reads of the previous channel are done
      stage_rows(Tl, g.TLD, g.TROWS, NP, jd.volA + c * planeA + (ptrdiff_t)(ty0 - D_TPAD) * jd.wA + tx0, jd.wA, N,
                 [&](int tr) { return tr >= D_TPAD && tr < D_TPAD + N; }, wv, lane);
      stage_rows(Sl, g.SLD, Ws, 2 * g.SLD, jd.volB + c * planeB + (size_t)sy0 * jd.wB + sx0, jd.wB, Ws,
                 [](int) { return true; }, wv, lane);
      __syncthreads();
      // this wave's search rows; for row s the u_y blocks n whose template
      // rows s - u_y meet [0, N) are those with 0 <= s - 16 n <= N + 14
      for (int s = wv; s < Ws; s += D_NW) {
        const int nhi = min(NB - 1, s >> 4);
        const int nlo = max(0, (s - N + 1) >> 4);
        const unsigned* srow = Sl + (size_t)s * g.SLD;
        for (int kc = 0; kc < NP / 32; ++kc) {
          // issue every operand read of this chunk before the first use
          unsigned raw[NB][5];
#pragma unroll
          for (int m = 0; m < NB; ++m) {
            // 8 bf16 of search row s from column 32 kc + 8 kg + 16 m + lane % 16
            const unsigned* sp = srow + ((32 * kc + 8 * kg + 16 * m + l16) >> 1);
#pragma unroll
            for (int i = 0; i < 5; ++i) raw[m][i] = sp[i];
          }
          uint4 bw[NB];
#pragma unroll
          for (int n = 0; n < NB; ++n) {
            // template row s - 16 n - lane % 16, columns 32 kc + 8 kg .. + 7
            // (rows of blocks outside [nlo, nhi] are clamped and not used)
            const int tr = min(max(s - 16 * n - l16 + D_TPAD, 0), g.TROWS - 1);
            bw[n] = *reinterpret_cast<const uint4*>(Tl + (size_t)tr * g.TLD + 16 * kc + 4 * kg);
          }
          const unsigned sh = (l16 & 1) * 2;  // e & 1 for every m
          bf16x8 A[NB];
#pragma unroll
          for (int m = 0; m < NB; ++m) {
            unsigned av[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = __builtin_amdgcn_alignbyte(raw[m][i + 1], raw[m][i], sh);
            A[m] = __builtin_bit_cast(bf16x8, av);
          }
#pragma unroll
          for (int n = 0; n < NB; ++n) {
            if (n >= nlo && n <= nhi) {
              const bf16x8 B = __builtin_bit_cast(bf16x8, bw[n]);
#pragma unroll
              for (int m = 0; m < NB; ++m) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[m], B, acc[m][n], 0, 0, 0);
            }
          }
        }
      }
    }
    __syncthreads();  // all MFMA reads of T/S are done: Cs and the partials may overwrite them
    // sum the waves' partial correlations in wave order (deterministic): D_PW
    // waves at a time store theirs side by side behind Cs, then every thread
    // adds the D_PW values of its elements into Cs.  (Adding wave by wave into
    // Cs serialised each wave's read-modify-writes: about 8% of a point's
    // time at K = 65.)
    const int KK = K * K;
    float* part = Cs + KK;
    for (int w0 = 0; w0 < D_NW; w0 += D_PW) {
      if (wv >= w0 && wv < w0 + D_PW) {
        float* mine = part + (size_t)(wv - w0) * KK;
#pragma unroll
        for (int m = 0; m < NB; ++m)
#pragma unroll
          for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int ux = 16 * m + 4 * kg + q, uy = 16 * n + l16;
              if (ux < K && uy < K) mine[uy * K + ux] = acc[m][n][q];
            }
      }
      __syncthreads();
      for (int i = threadIdx.x; i < KK; i += D_NT) {
        float s = w0 == 0 ? 0.f : Cs[i];
#pragma unroll
        for (int w = 0; w < D_PW; ++w) s += part[(size_t)w * KK + i];
        Cs[i] = s;
      }
      __syncthreads();
    }
    ssd_epilogue<D_NT>(jd, cpi, tx0, ty0, sx0, sy0, Cs, red);
  }
}

size_t direct_workspace_bytes(const cfog_job*, int, int, int) { return 0; }

template <int NB>
static void launch_nb(const MatchJob& d, const DirectGeom& g, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(match_direct_kernel<NB>, dim3(blocks), dim3(D_NT), g.lds, st, d, g);
}

int init_direct_attributes() {
  const void* k[D_NB] = {(const void*)match_direct_kernel<1>, (const void*)match_direct_kernel<2>,
                         (const void*)match_direct_kernel<3>, (const void*)match_direct_kernel<4>,
                         (const void*)match_direct_kernel<5>};
  for (int i = 0; i < D_NB; ++i)
    if (hipFuncSetAttribute(k[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds) != hipSuccess) return -2;
  return 0;
}

int launch_match_direct(const cfog_job* jobs, int n_jobs, int m, int obj, void*, int num_cus, hipStream_t st) {
  for (int i = 0; i < n_jobs; ++i)
    if (!direct_supported(jobs[i].N, jobs[i].r)) return -1;
  for (int i = 0; i < n_jobs; ++i) {
    const cfog_job& j = jobs[i];
    if (j.n_cps == 0) continue;
    const DirectGeom g = direct_geom(j.N, j.r);
    MatchJob d{};
    d.volA = j.volA; d.satA = j.satA; d.hA = j.hA; d.wA = j.wA;
    d.volB = j.volB; d.satB = j.satB; d.hB = j.hB; d.wB = j.wB;
    d.cps = reinterpret_cast<const int4*>(j.cps);
    d.n_cps = j.n_cps; d.N = j.N; d.r = j.r; d.m = m;
    d.out = reinterpret_cast<Result*>(j.out);
    d.surfaces = j.surfaces;
    d.subpix = reinterpret_cast<float2*>(j.subpix);
    d.obj = obj;
    const int per_cu = std::max(1, (int)(kMaxLds / g.lds));
    const int blocks = std::min(j.n_cps, num_cus * per_cu);
    switch (g.nblk) {
      case 1: launch_nb<1>(d, g, blocks, st); break;
      case 2: launch_nb<2>(d, g, blocks, st); break;
      case 3: launch_nb<3>(d, g, blocks, st); break;
      case 4: launch_nb<4>(d, g, blocks, st); break;
      default: launch_nb<5>(d, g, blocks, st); break;
    }
    if (hipGetLastError() != hipSuccess) return -2;
  }
  return 0;
}

bool direct_supported(int N, int r) {
  if (N < 1 || r < 0 || N > kMaxSide || r > kMaxSide) return false;
  const DirectGeom g = direct_geom(N, r);
  return g.nblk <= D_NB && g.lds <= kMaxLds;
}

}  // namespace cfog
