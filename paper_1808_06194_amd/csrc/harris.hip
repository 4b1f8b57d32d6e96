// Block-based Harris feature points (Section IV of Ye et al.): the reference
// image is divided into n x n cells; the chip (up to 64 x 64 pixels) centred
// on each cell is read and its k pixels with the largest Harris response
// become feature points, which are the control points the matcher takes.
//
// One workgroup per chip, everything in LDS (two chips per CU); lanes map to
// chip columns and the four waves take every fourth row, so no index is
// divided; the Gaussian radius is a template parameter (unrolled taps):
//   1. the chip (clipped to the image);
//   2. gradients by [-1, 0, 1] with the chip's borders replicated;
//   3. the structure tensor products gx^2, gx gy, gy^2 (formed on the fly)
//      smoothed by a normalised Gaussian (horizontal then vertical pass,
//      chip borders replicated) and the response R = det - kappa trace^2;
//   4. k rounds of a workgroup argmax (largest R, ties to the smallest
//      row-major index), each marking its winner as taken.
#include <hip/hip_runtime.h>
#include <math.h>
#include <limits.h>
#include <algorithm>
#include "cfog.h"
#include "kernels.hpp"

namespace cfog {

constexpr int HR_NT = 256;
constexpr int HR_MAX_CHIP = 64;
constexpr int HR_MAX_K = 64;

struct HarrisArgs {
  const float* img;
  int64_t stride;
  int H, W, n, k, chip;
  float kappa;
  float w[kMaxGaussRadius + 1];  // w[|j|], j in [-R, R]
  cfog_cp* cps;
  float* resp;
};

constexpr int HR_LD = HR_MAX_CHIP;  // LDS row stride of every chip array
constexpr int HR_NW = HR_NT / 64;

// Dynamic LDS: five 64 x 64 arrays (80 KB, so two chips share a CU; the
// argmax scratch lives in a dead array, as any static LDS would push a
// workgroup past half of the CU's 160 KB).  The chip is dead once the
// gradients exist and shares storage with the first smoothed product; the
// response reuses gx.
static size_t harris_lds_bytes() { return (size_t)5 * HR_LD * HR_LD * sizeof(float); }

template <int R>
__global__ __launch_bounds__(HR_NT) void harris_grid_kernel(HarrisArgs a) {
  extern __shared__ float hsm[];
  constexpr int CC = HR_LD * HR_LD;
  float* gx = hsm;
  float* gy = gx + CC;
  float* ta = gy + CC;
  float* tb = ta + CC;
  float* tc = tb + CC;
  float* img = ta;  // read only by the gradient pass
  float* Rv = gx;   // written by the vertical pass, after the last gx read
  float* bestv = tb;                                 // HR_NW values, after the vertical pass
  int* besti = reinterpret_cast<int*>(tb + HR_NW);   // their indices
  const int cell = blockIdx.x, ci = cell / a.n, cj = cell - ci * a.n;
  // chip of cell (ci, cj): centred at ((2 cj + 1) W / 2n, (2 ci + 1) H / 2n), clipped
  const int cy = (int)(((int64_t)(2 * ci + 1) * a.H) / (2 * a.n));
  const int cx = (int)(((int64_t)(2 * cj + 1) * a.W) / (2 * a.n));
  const int y0 = max(0, cy - a.chip / 2), x0 = max(0, cx - a.chip / 2);
  const int h = min(a.H, cy - a.chip / 2 + a.chip) - y0, w = min(a.W, cx - a.chip / 2 + a.chip) - x0;
  const int x = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool col = x < w;
  float wt[R + 1];
#pragma unroll
  for (int j = 0; j <= R; ++j) wt[j] = a.w[j];

  constexpr int RPW = HR_LD / HR_NW;  // rows per wave (the row loops below are unrolled over them)
  {
    // all loads of the chip issued before the first LDS store
    float v[RPW];
    const float* src = a.img + (int64_t)y0 * a.stride + x0 + x;
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
      const int y = wv + HR_NW * t;
      if (col && y < h) v[t] = src[(int64_t)y * a.stride];
    }
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
      const int y = wv + HR_NW * t;
      if (col && y < h) img[y * HR_LD + x] = v[t];
    }
  }
  __syncthreads();
  const int xp = min(x + 1, w - 1), xm = max(x - 1, 0);
#pragma unroll
  for (int t = 0; t < RPW; ++t) {
    const int y = wv + HR_NW * t;
    if (col && y < h) {
      const float* row = img + y * HR_LD;
      gx[y * HR_LD + x] = row[xp] - row[xm];
      gy[y * HR_LD + x] = img[min(y + 1, h - 1) * HR_LD + x] - img[max(y - 1, 0) * HR_LD + x];
    }
  }
  __syncthreads();
  // horizontal pass of the three products (columns clamped to the chip)
  int xs[2 * R + 1];
#pragma unroll
  for (int j = -R; j <= R; ++j) xs[j + R] = min(max(x + j, 0), w - 1);
#pragma unroll
  for (int t = 0; t < RPW; ++t) {
    const int y = wv + HR_NW * t;
    if (col && y < h) {
      const float* rx = gx + y * HR_LD;
      const float* ry = gy + y * HR_LD;
      float sa = 0.f, sb = 0.f, sc = 0.f;
#pragma unroll
      for (int j = -R; j <= R; ++j) {
        const float u = rx[xs[j + R]], v = ry[xs[j + R]], wj = wt[j < 0 ? -j : j];
        sa = fmaf(wj, u * u, sa);
        sb = fmaf(wj, u * v, sb);
        sc = fmaf(wj, v * v, sc);
      }
      ta[y * HR_LD + x] = sa;
      tb[y * HR_LD + x] = sb;
      tc[y * HR_LD + x] = sc;
    }
  }
  __syncthreads();
  // vertical pass (rows clamped to the chip) and the response
#pragma unroll
  for (int t = 0; t < RPW; ++t) {
    const int y = wv + HR_NW * t;
    if (col && y < h) {
      float sa = 0.f, sb = 0.f, sc = 0.f;
#pragma unroll
      for (int j = -R; j <= R; ++j) {
        const int q = min(max(y + j, 0), h - 1) * HR_LD + x;
        const float wj = wt[j < 0 ? -j : j];
        sa = fmaf(wj, ta[q], sa);
        sb = fmaf(wj, tb[q], sb);
        sc = fmaf(wj, tc[q], sc);
      }
      const float tr = sa + sc;
      Rv[y * HR_LD + x] = sa * sc - sb * sb - a.kappa * tr * tr;
    }
  }
  __syncthreads();

  const int lane = x;
  for (int q = 0; q < a.k; ++q) {
    float bv = -INFINITY;
    int bi = INT_MAX;
#pragma unroll
    for (int t = 0; t < RPW; ++t) {  // increasing row-major index per thread
      const int y = wv + HR_NW * t;
      if (col && y < h) {
        const float v = Rv[y * HR_LD + x];
        if (v > bv) {  // taken pixels hold NaN and never win
          bv = v;
          bi = y * w + x;
        }
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      bestv[wv] = bv;
      besti[wv] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int u = 1; u < HR_NW; ++u)
        if (bestv[u] > bv || (bestv[u] == bv && besti[u] < bi)) {
          bv = bestv[u];
          bi = besti[u];
        }
      const int o = cell * a.k + q;
      if (bi != INT_MAX) {
        const int yy = bi / w, xx = bi - yy * w;
        a.cps[o] = cfog_cp{x0 + xx, y0 + yy, x0 + xx, y0 + yy};
        if (a.resp) a.resp[o] = bv;
        Rv[yy * HR_LD + xx] = NAN;
      } else {  // no finite response left (a non-finite chip)
        a.cps[o] = cfog_cp{-1, -1, -1, -1};
        if (a.resp) a.resp[o] = NAN;
      }
    }
    __syncthreads();
  }
}

template <int R>
static int set_harris_attr() {
  return hipFuncSetAttribute((const void*)harris_grid_kernel<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)harris_lds_bytes()) == hipSuccess
             ? 0
             : -2;
}

int init_harris_attributes() {
  if (set_harris_attr<0>() || set_harris_attr<1>() || set_harris_attr<2>() || set_harris_attr<3>() ||
      set_harris_attr<4>() || set_harris_attr<5>() || set_harris_attr<6>() || set_harris_attr<7>() ||
      set_harris_attr<8>())
    return -2;
  return 0;
}

template <int R>
static int launch_harris(const HarrisArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(harris_grid_kernel<R>, dim3(a.n * a.n), dim3(HR_NT), harris_lds_bytes(), st, a);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace cfog

extern "C" int cfog_harris_grid(cfog_ctx* ctx, const float* d_img, int32_t H, int32_t W, int64_t row_stride,
                                int32_t n, int32_t k, int32_t chip, float sigma, float kappa, cfog_cp* d_cps,
                                float* d_response, void* stream) {
  if (!ctx || !d_img || !d_cps || H < 1 || W < 1 || row_stride < W || n < 1 || k < 1 ||
      k > cfog::HR_MAX_K || chip < 1 || chip > cfog::HR_MAX_CHIP || !(sigma > 0.f) || !isfinite(sigma) ||
      !isfinite(kappa) || ((uintptr_t)d_cps % 16) != 0 || ((uintptr_t)d_response % 4) != 0)
    return CFOG_EINVAL;
  if ((int64_t)n * n > INT_MAX / k) return CFOG_EINVAL;
  const int R = (int)(4.0 * sigma + 0.5);
  if (R > cfog::kMaxGaussRadius) return CFOG_EUNSUPPORTED;
  // every chip must hold at least k pixels
  for (int i = 0; i < n; ++i) {
    const int cy = (int)(((int64_t)(2 * i + 1) * H) / (2 * n));
    const int h = std::min(H, cy - chip / 2 + chip) - std::max(0, cy - chip / 2);
    for (int j = 0; j < n; ++j) {
      const int cx = (int)(((int64_t)(2 * j + 1) * W) / (2 * n));
      const int w = std::min(W, cx - chip / 2 + chip) - std::max(0, cx - chip / 2);
      if (h < 1 || w < 1 || h * w < k) return CFOG_EINVAL;
    }
  }
  cfog::HarrisArgs a{};
  a.img = d_img;
  a.stride = row_stride;
  a.H = H;
  a.W = W;
  a.n = n;
  a.k = k;
  a.chip = chip;
  a.kappa = kappa;
  double ws[cfog::kMaxGaussRadius + 1], tot = 0.0;
  for (int j = 0; j <= R; ++j) {
    ws[j] = exp(-(double)j * j / (2.0 * (double)sigma * sigma));
    tot += (j ? 2.0 : 1.0) * ws[j];
  }
  for (int j = 0; j <= R; ++j) a.w[j] = (float)(ws[j] / tot);
  a.cps = d_cps;
  a.resp = d_response;
  hipStream_t st = (hipStream_t)stream;
  int rc = -2;
  switch (R) {
    case 0: rc = cfog::launch_harris<0>(a, st); break;
    case 1: rc = cfog::launch_harris<1>(a, st); break;
    case 2: rc = cfog::launch_harris<2>(a, st); break;
    case 3: rc = cfog::launch_harris<3>(a, st); break;
    case 4: rc = cfog::launch_harris<4>(a, st); break;
    case 5: rc = cfog::launch_harris<5>(a, st); break;
    case 6: rc = cfog::launch_harris<6>(a, st); break;
    case 7: rc = cfog::launch_harris<7>(a, st); break;
    case 8: rc = cfog::launch_harris<8>(a, st); break;
    default: return CFOG_EUNSUPPORTED;
  }
  return rc == 0 ? CFOG_OK : CFOG_EHIP;
}
