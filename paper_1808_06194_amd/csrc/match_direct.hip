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
// width to 32.  Per channel the template (bf16, with zero rows above and below
// so that s - u_y never leaves it) and the search window (bf16) are staged in
// LDS; wave w owns the u_x block w and all u_y blocks.  Operand fragments:
//   A (lane l): 8 bf16 of search row s from column 32kc + 8(l/16) + u_x,
//      read as 5 aligned dwords and realigned by a byte shift;
//   B (lane l): 8 bf16 of template row s - u_y, columns 32kc + 8(l/16) .. +7,
//      one aligned 16-byte LDS read.
// Inputs are rounded to BF16 (relative error 2^-9 each), so |C_bf16 - C| <=
// 2^-8 sum |T S| <= 2^-9 (E1 + E2): the SSD surface is within 2^-8 (E1 + E2)
// of the exact one, against ~1e-6 for the FP32 FFT path.
#include <hip/hip_runtime.h>
#include <algorithm>
#include "cfog.h"
#include "epilogue.hpp"
#include "kernels.hpp"

namespace cfog {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int D_NB = 5;            // max 16-wide blocks of u_x (and u_y): 2r+1 <= 80
constexpr int D_NT = 64 * D_NB;    // one wave per u_x block

struct DirectGeom {
  int N, r, K, nblk, NP, Ws, OFF, TROWS, SW;
  int TLD;  // template row stride in dwords: NP/2 + 4, so that the 16 rows a
            // B fragment reads start in different LDS banks
  size_t lds;
};

static DirectGeom direct_geom(int N, int r) {
  DirectGeom g;
  g.N = N;
  g.r = r;
  g.K = 2 * r + 1;
  g.nblk = (g.K + 15) / 16;
  g.NP = (N + 31) / 32 * 32;
  g.Ws = N + 2 * r;
  g.OFF = 16 * g.nblk;               // template rows start here in LDS
  g.TROWS = g.Ws + g.OFF;            // rows s - u_y + OFF, s < Ws, u_y < 16 nblk
  g.SW = g.NP + 16 * g.nblk + 2;     // search row width incl. the fragment over-read
  g.TLD = g.NP / 2 + 4;
  const size_t t = (size_t)g.TROWS * g.TLD * 4, sb = (size_t)g.Ws * g.SW * 2;
  const size_t c = (size_t)g.K * g.K * 4;
  g.lds = std::max(t + sb, c) + 16 * D_NB;
  return g;
}

__device__ __forceinline__ unsigned pack_bf16x2(float lo, float hi) {
  const __bf16 a = (__bf16)lo, b = (__bf16)hi;
  return (unsigned)__builtin_bit_cast(unsigned short, a) | ((unsigned)__builtin_bit_cast(unsigned short, b) << 16);
}

__global__ __launch_bounds__(D_NT) void match_direct_kernel(MatchJob jd, DirectGeom g) {
  extern __shared__ unsigned char dsm[];
  unsigned* Tl = reinterpret_cast<unsigned*>(dsm);                                  // TROWS x TLD dwords
  unsigned* Sl = Tl + (size_t)g.TROWS * g.TLD;                                       // Ws x SW/2 dwords
  float* Cs = reinterpret_cast<float*>(dsm);                                         // aliases T after the loop
  ArgminState* red = reinterpret_cast<ArgminState*>(dsm + g.lds - 16 * D_NB);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int N = g.N, r = g.r, K = g.K, NP = g.NP, Ws = g.Ws, SW = g.SW;
  const size_t planeA = (size_t)jd.hA * jd.wA, planeB = (size_t)jd.hB * jd.wB;

  for (int cpi = blockIdx.x; cpi < jd.n_cps; cpi += gridDim.x) {
    const int4 cp = jd.cps[cpi];
    const int h = N / 2;
    const int tx0 = cp.x - h, ty0 = cp.y - h, sx0 = cp.z - h - r, sy0 = cp.w - h - r;
    __syncthreads();  // previous task's epilogue is done with LDS
    const bool inA = tx0 >= 0 && ty0 >= 0 && tx0 + N <= jd.wA && ty0 + N <= jd.hA;
    const bool inB = sx0 >= 0 && sy0 >= 0 && sx0 + Ws <= jd.wB && sy0 + Ws <= jd.hB;
    if (!(inA && inB)) {
      oob_result<D_NT>(jd, cpi);
      continue;
    }
    f32x4 acc[D_NB];
#pragma unroll
    for (int n = 0; n < D_NB; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int c = 0; c < jd.m; ++c) {
      __syncthreads();  // MFMA reads of the previous channel are done
      const float* TA = jd.volA + c * planeA + (size_t)ty0 * jd.wA + tx0;
      const float* SB = jd.volB + c * planeB + (size_t)sy0 * jd.wB + sx0;
      for (int t = wv; t < g.TROWS; t += D_NB) {
        const int ty = t - g.OFF;
        const bool row_ok = ty >= 0 && ty < N;
        for (int x = 2 * lane; x < NP; x += 128) {
          float a = 0.f, b = 0.f;
          if (row_ok) {
            if (x < N) a = TA[(size_t)ty * jd.wA + x];
            if (x + 1 < N) b = TA[(size_t)ty * jd.wA + x + 1];
          }
          Tl[(size_t)t * g.TLD + x / 2] = pack_bf16x2(a, b);
        }
      }
      for (int y = wv; y < Ws; y += D_NB) {
        for (int x = 2 * lane; x < SW; x += 128) {
          const float a = x < Ws ? SB[(size_t)y * jd.wB + x] : 0.f;
          const float b = x + 1 < Ws ? SB[(size_t)y * jd.wB + x + 1] : 0.f;
          Sl[(size_t)y * (SW / 2) + x / 2] = pack_bf16x2(a, b);
        }
      }
      __syncthreads();
      if (wv < g.nblk) {
        const int ux = 16 * wv + (lane & 15), kg = lane >> 4;
        const int uyl = lane & 15;
        for (int s = 0; s < Ws; ++s) {
          // u_y blocks with some template row s - u_y inside [0, N)
          const int nhi = min(g.nblk - 1, s >> 4);
          const int nlo = max(0, (s - N - 14 + 15) >> 4);
          const unsigned* srow = Sl + (size_t)s * (SW / 2);
          for (int kc = 0; kc < NP / 32; ++kc) {
            const int e = 32 * kc + 8 * kg + ux;  // first search column of this lane's fragment
            const unsigned* sp = srow + (e >> 1);
            const unsigned w0 = sp[0], w1 = sp[1], w2 = sp[2], w3 = sp[3], w4 = sp[4];
            const unsigned sh = (e & 1) * 2;
            unsigned av[4];
            av[0] = __builtin_amdgcn_alignbyte(w1, w0, sh);
            av[1] = __builtin_amdgcn_alignbyte(w2, w1, sh);
            av[2] = __builtin_amdgcn_alignbyte(w3, w2, sh);
            av[3] = __builtin_amdgcn_alignbyte(w4, w3, sh);
            const bf16x8 A = __builtin_bit_cast(bf16x8, av);
#pragma unroll
            for (int n = 0; n < D_NB; ++n) {
              if (n >= nlo && n <= nhi) {
                const int t = s - (16 * n + uyl) + g.OFF;
                const uint4 bw = *reinterpret_cast<const uint4*>(Tl + (size_t)t * g.TLD + (32 * kc + 8 * kg) / 2);
                const bf16x8 B = __builtin_bit_cast(bf16x8, bw);
                acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[n], 0, 0, 0);
              }
            }
          }
        }
      }
    }
    __syncthreads();  // all MFMA reads of T/S are done: Cs may overwrite them
    if (wv < g.nblk) {
#pragma unroll
      for (int n = 0; n < D_NB; ++n) {
        const int uy = 16 * n + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ux = 16 * wv + 4 * (lane >> 4) + q;
          if (n < g.nblk && uy < K && ux < K) Cs[uy * K + ux] = acc[n][q];
        }
      }
    }
    __syncthreads();
    ssd_epilogue<D_NT>(jd, cpi, tx0, ty0, sx0, sy0, Cs, red);
  }
}

static int g_direct_attr = 1;

size_t direct_workspace_bytes(const cfog_job*, int, int, int) { return 0; }

int launch_match_direct(const cfog_job* jobs, int n_jobs, int m, void*, int num_cus, hipStream_t st) {
  if (g_direct_attr == 1) {
    g_direct_attr = hipFuncSetAttribute((const void*)match_direct_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kMaxLds) == hipSuccess
                        ? 0
                        : -2;
  }
  if (g_direct_attr != 0) return -2;
  for (int i = 0; i < n_jobs; ++i) {
    const cfog_job& j = jobs[i];
    const DirectGeom g = direct_geom(j.N, j.r);
    if (g.nblk > D_NB || g.lds > kMaxLds) return -1;
  }
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
    const int per_cu = std::max(1, (int)(kMaxLds / g.lds));
    const int blocks = std::min(j.n_cps, num_cus * per_cu);
    hipLaunchKernelGGL(match_direct_kernel, dim3(blocks), dim3(D_NT), g.lds, st, d, g);
    if (hipGetLastError() != hipSuccess) return -2;
  }
  return 0;
}

bool direct_supported(int N, int r) {
  const DirectGeom g = direct_geom(N, r);
  return g.nblk <= D_NB && g.lds <= kMaxLds;
}

}  // namespace cfog
