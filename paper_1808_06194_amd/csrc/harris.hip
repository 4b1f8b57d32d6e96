// Block-based Harris feature points (Section IV of Ye et al.): the reference
// image is divided into n x n cells; the chip (up to 64 x 64 pixels) centred
// on each cell is read and its k pixels with the largest Harris response
// become feature points, which are the control points the matcher takes.
//
// One workgroup per chip, everything in LDS (two chips per CU):
//   1. the chip (clipped to the image);
//   2. gradients by [-1, 0, 1] with the chip's borders replicated;
//   3. the structure tensor products gx^2, gx gy, gy^2 smoothed by a
//      normalised Gaussian (horizontal then vertical pass, chip borders
//      replicated) and the response R = det - kappa trace^2;
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
  int H, W, n, k, chip, R;
  float kappa;
  float w[kMaxGaussRadius + 1];  // w[|j|], j in [-R, R]
  cfog_cp* cps;
  float* resp;
};

__device__ __forceinline__ int hclamp(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// Dynamic LDS: five chip-sized arrays (at most 80 KB, so two chips share a
// CU).  The chip is dead once the gradients exist and shares storage with the
// first smoothed product; the response reuses gx.
static size_t harris_lds_bytes(int chip) { return (size_t)5 * chip * chip * sizeof(float); }

__global__ __launch_bounds__(HR_NT) void harris_grid_kernel(HarrisArgs a) {
  extern __shared__ float hsm[];
  const int cc = a.chip * a.chip;
  float* gx = hsm;
  float* gy = gx + cc;
  float* ta = gy + cc;
  float* tb = ta + cc;
  float* tc = tb + cc;
  float* img = ta;  // read only by the gradient pass
  float* Rv = gx;   // written by the vertical pass, after the last gx read
  __shared__ float bestv[HR_NT / 64];
  __shared__ int besti[HR_NT / 64];
  const int cell = blockIdx.x, ci = cell / a.n, cj = cell - ci * a.n;
  // chip of cell (ci, cj): centred at ((2 cj + 1) W / 2n, (2 ci + 1) H / 2n), clipped
  const int cy = (int)(((int64_t)(2 * ci + 1) * a.H) / (2 * a.n));
  const int cx = (int)(((int64_t)(2 * cj + 1) * a.W) / (2 * a.n));
  const int y0 = max(0, cy - a.chip / 2), x0 = max(0, cx - a.chip / 2);
  const int h = min(a.H, cy - a.chip / 2 + a.chip) - y0, w = min(a.W, cx - a.chip / 2 + a.chip) - x0;
  const int np = h * w;
  const int tid = threadIdx.x;

  for (int i = tid; i < np; i += HR_NT) {
    const int y = i / w, x = i - y * w;
    img[i] = a.img[(int64_t)(y0 + y) * a.stride + x0 + x];
  }
  __syncthreads();
  for (int i = tid; i < np; i += HR_NT) {
    const int y = i / w, x = i - y * w;
    const float* row = img + y * w;
    gx[i] = row[hclamp(x + 1, w - 1)] - row[hclamp(x - 1, w - 1)];
    gy[i] = img[hclamp(y + 1, h - 1) * w + x] - img[hclamp(y - 1, h - 1) * w + x];
  }
  __syncthreads();
  const int R = a.R;
  for (int i = tid; i < np; i += HR_NT) {
    const int y = i / w, x = i - y * w;
    float sa = 0.f, sb = 0.f, sc = 0.f;
    for (int j = -R; j <= R; ++j) {
      const int q = y * w + hclamp(x + j, w - 1);
      const float wj = a.w[j < 0 ? -j : j];
      sa = fmaf(wj, gx[q] * gx[q], sa);
      sb = fmaf(wj, gx[q] * gy[q], sb);
      sc = fmaf(wj, gy[q] * gy[q], sc);
    }
    ta[i] = sa;
    tb[i] = sb;
    tc[i] = sc;
  }
  __syncthreads();
  for (int i = tid; i < np; i += HR_NT) {
    const int y = i / w, x = i - y * w;
    float sa = 0.f, sb = 0.f, sc = 0.f;
    for (int j = -R; j <= R; ++j) {
      const int q = hclamp(y + j, h - 1) * w + x;
      const float wj = a.w[j < 0 ? -j : j];
      sa = fmaf(wj, ta[q], sa);
      sb = fmaf(wj, tb[q], sb);
      sc = fmaf(wj, tc[q], sc);
    }
    const float tr = sa + sc;
    Rv[i] = sa * sc - sb * sb - a.kappa * tr * tr;
  }
  __syncthreads();

  const int lane = tid & 63, wv = tid >> 6;
  for (int q = 0; q < a.k; ++q) {
    float bv = -INFINITY;
    int bi = INT_MAX;
    for (int i = tid; i < np; i += HR_NT) {
      const float v = Rv[i];
      if (v > bv || (v == bv && i < bi)) {  // taken pixels hold NaN and never win
        bv = v;
        bi = i;
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
    if (tid == 0) {
      for (int u = 1; u < HR_NT / 64; ++u)
        if (bestv[u] > bv || (bestv[u] == bv && besti[u] < bi)) {
          bv = bestv[u];
          bi = besti[u];
        }
      const int o = cell * a.k + q;
      if (bi != INT_MAX) {
        const int y = bi / w, x = bi - y * w;
        a.cps[o] = cfog_cp{x0 + x, y0 + y, x0 + x, y0 + y};
        if (a.resp) a.resp[o] = bv;
        Rv[bi] = NAN;
      } else {  // no finite response left (a non-finite chip)
        a.cps[o] = cfog_cp{-1, -1, -1, -1};
        if (a.resp) a.resp[o] = NAN;
      }
    }
    __syncthreads();
  }
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
  a.R = R;
  a.kappa = kappa;
  double ws[cfog::kMaxGaussRadius + 1], tot = 0.0;
  for (int j = 0; j <= R; ++j) {
    ws[j] = exp(-(double)j * j / (2.0 * (double)sigma * sigma));
    tot += (j ? 2.0 : 1.0) * ws[j];
  }
  for (int j = 0; j <= R; ++j) a.w[j] = (float)(ws[j] / tot);
  a.cps = d_cps;
  a.resp = d_response;
  static int attr = 1;
  if (attr == 1)
    attr = hipFuncSetAttribute((const void*)cfog::harris_grid_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)cfog::harris_lds_bytes(cfog::HR_MAX_CHIP)) == hipSuccess
               ? 0
               : -1;
  if (attr != 0) return CFOG_EHIP;
  hipLaunchKernelGGL(cfog::harris_grid_kernel, dim3(n * n), dim3(cfog::HR_NT), cfog::harris_lds_bytes(chip),
                     (hipStream_t)stream, a);
  if (hipGetLastError() != hipSuccess) return CFOG_EHIP;
  return CFOG_OK;
}
