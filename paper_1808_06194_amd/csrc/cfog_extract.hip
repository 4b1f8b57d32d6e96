// CFOG extraction (Section III-F of Ye et al.) and FP64 summed-area tables of
// the per-pixel energy Q = sum_k D_k^2 (the energy terms of Eq. 5).
//
// Layout: image [H][row_stride] fp32; volume D [m][H][W] fp32 (planar, one
// contiguous H*W plane per orientation); SAT [(H+1)][(W+1)] fp64 with a zero
// first row and column, SAT(y, x) = sum_{y'<y, x'<x} Q.
//
// One workgroup produces a TX x TY output tile for all m channels:
//   A. stage the image tile plus a (R+1)-pixel halo in LDS (clamp-to-edge);
//   B. per pixel of the tile + R halo: gx, gy by [-1,0,1] (Eq. 2's filters),
//      g_k = |cos(theta_k) gx + sin(theta_k) gy| for theta_k = k pi / m, and the
//      circular [1,2,1]/4 orientation smoothing, all in registers; result -> LDS;
//   C. per channel: horizontal then vertical Gaussian pass (radius R, clamp-to-
//      edge; the halo values of B were computed at clamped positions), output
//      written straight to HBM; Q accumulated in FP64 from the FP32 outputs.
// The Gaussian and the [1,2,1] kernel are linear and act on different axes, so
// applying the orientation smoothing before the spatial one gives the same
// volume as the order the paper describes (up to FP32 rounding).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "kernels.hpp"

namespace cfog {

constexpr int EX_TX = 64;
constexpr int EX_TY = 16;
constexpr int EX_NT = 256;

struct ExtractArgs {
  const float* img;
  int64_t stride;
  int H, W, m, R;
  float* vol;
  double* sat;  // nullable
  float cs[kMaxOrient];
  float sn[kMaxOrient];
  float w[kMaxGaussRadius + 1];  // w[|j|], j in [-R, R]
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__global__ __launch_bounds__(EX_NT) void cfog_extract_kernel(ExtractArgs a) {
  extern __shared__ float lds[];
  const int R = a.R, m = a.m;
  const int IW = EX_TX + 2 * R + 2, IH = EX_TY + 2 * R + 2;  // image tile
  const int GW = EX_TX + 2 * R, GH = EX_TY + 2 * R;          // channel tile
  float* img = lds;                                          // IH * IW
  float* G = img + IH * IW;                                  // m * GH * GW
  float* Hb = G + m * GH * GW;                               // 2 * GH * EX_TX
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * EX_TX, y0 = blockIdx.y * EX_TY;
  const int H = a.H, W = a.W;

  // A. image tile, rows y0-R-1 .. y0+TY+R, clamped
  for (int i = tid; i < IH * IW; i += EX_NT) {
    int r = i / IW, c = i - r * IW;
    int gy = clampi(y0 - R - 1 + r, 0, H - 1), gx = clampi(x0 - R - 1 + c, 0, W - 1);
    img[i] = a.img[(int64_t)gy * a.stride + gx];
  }
  __syncthreads();

  // B. oriented channels + Z smoothing at clamped positions of the halo tile
  const int oy = y0 - R - 1, ox = x0 - R - 1;  // global coords of img[0][0]
  for (int i = tid; i < GH * GW; i += EX_NT) {
    int r = i / GW, c = i - r * GW;
    int Yc = clampi(y0 - R + r, 0, H - 1), Xc = clampi(x0 - R + c, 0, W - 1);
    int yl = Yc - oy, xl = Xc - ox;
    int xp = clampi(Xc + 1, 0, W - 1) - ox, xm = clampi(Xc - 1, 0, W - 1) - ox;
    int yp = clampi(Yc + 1, 0, H - 1) - oy, ym = clampi(Yc - 1, 0, H - 1) - oy;
    float gx = img[yl * IW + xp] - img[yl * IW + xm];
    float gy = img[yp * IW + xl] - img[ym * IW + xl];
    float g0 = fabsf(fmaf(a.cs[0], gx, a.sn[0] * gy));
    float prev = fabsf(fmaf(a.cs[m - 1], gx, a.sn[m - 1] * gy));
    float cur = g0;
    for (int k = 0; k < m; ++k) {
      float nxt = (k + 1 < m) ? fabsf(fmaf(a.cs[k + 1], gx, a.sn[k + 1] * gy)) : g0;
      G[(k * GH + r) * GW + c] = fmaf(0.25f, prev + nxt, 0.5f * cur);
      prev = cur;
      cur = nxt;
    }
  }
  __syncthreads();

  // C. separable Gaussian per channel; each thread owns 4 output pixels
  constexpr int PPT = EX_TX * EX_TY / EX_NT;
  double q[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) q[p] = 0.0;
  const size_t plane = (size_t)H * W;
  for (int k = 0; k < m; ++k) {
    float* hb = Hb + (k & 1) * GH * EX_TX;
    const float* gk = G + k * GH * GW;
    for (int i = tid; i < GH * EX_TX; i += EX_NT) {
      int r = i / EX_TX, c = i - r * EX_TX;
      const float* row = gk + r * GW + c + R;
      float s = a.w[0] * row[0];
      for (int j = 1; j <= R; ++j) s = fmaf(a.w[j], row[-j] + row[j], s);
      hb[i] = s;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      int i = tid + p * EX_NT;
      int r = i / EX_TX, c = i - r * EX_TX;
      const float* col = hb + (r + R) * EX_TX + c;
      float s = a.w[0] * col[0];
      for (int j = 1; j <= R; ++j) s = fmaf(a.w[j], col[-j * EX_TX] + col[j * EX_TX], s);
      int gyy = y0 + r, gxx = x0 + c;
      if (gyy < H && gxx < W) {
        a.vol[k * plane + (size_t)gyy * W + gxx] = s;
        q[p] = fma((double)s, (double)s, q[p]);
      }
    }
    // the next channel writes the other half of Hb; the one after this
    // overwrites this half only after the next barrier
  }
  if (a.sat) {
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      int i = tid + p * EX_NT;
      int r = i / EX_TX, c = i - r * EX_TX;
      int gyy = y0 + r, gxx = x0 + c;
      if (gyy < H && gxx < W) a.sat[(size_t)(gyy + 1) * (W + 1) + gxx + 1] = q[p];
    }
  }
}

// ---------------------------------------------------------------- FP64 SAT
// Pass 1: zero row 0 and column 0, inclusive scan of every row in place.
constexpr int SAT_NT = 256;

__device__ __forceinline__ double wave_incl_scan(double v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    double t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__global__ __launch_bounds__(SAT_NT) void sat_rows_kernel(double* sat, int H, int W) {
  __shared__ double wsum[SAT_NT / 64];
  const int row = blockIdx.x;  // 0..H
  double* p = sat + (size_t)row * (W + 1);
  if (row == 0) {
    for (int x = threadIdx.x; x <= W; x += SAT_NT) p[x] = 0.0;
    return;
  }
  if (threadIdx.x == 0) p[0] = 0.0;
  double carry = 0.0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int base = 1; base <= W; base += SAT_NT) {
    int x = base + threadIdx.x;
    double v = (x <= W) ? p[x] : 0.0;
    v = wave_incl_scan(v);
    if (lane == 63) wsum[wv] = v;
    __syncthreads();
    double off = carry;
    for (int i = 0; i < wv; ++i) off += wsum[i];
    double tot = 0.0;
    for (int i = 0; i < SAT_NT / 64; ++i) tot += wsum[i];
    if (x <= W) p[x] = v + off;
    carry += tot;
    __syncthreads();
  }
}

// Pass 2: column scan over row blocks.  Block b covers rows [1 + b*SB, ...).
constexpr int SAT_SB = 64;

__global__ __launch_bounds__(SAT_NT) void sat_cols_local_kernel(double* sat, int H, int W) {
  const int x = blockIdx.x * SAT_NT + threadIdx.x;
  if (x > W) return;
  const int r0 = 1 + blockIdx.y * SAT_SB, r1 = min(H + 1, r0 + SAT_SB);
  double s = 0.0;
  for (int y = r0; y < r1; ++y) {
    double* q = sat + (size_t)y * (W + 1) + x;
    s += *q;
    *q = s;
  }
}

// Pass 3: carry block totals down each column (last row of every block ends
// up holding the global prefix), one thread per column.
__global__ __launch_bounds__(SAT_NT) void sat_cols_carry_kernel(double* sat, int H, int W, int nblk) {
  const int x = blockIdx.x * SAT_NT + threadIdx.x;
  if (x > W) return;
  double run = 0.0;
  for (int b = 0; b < nblk; ++b) {
    int last = min(H, b * SAT_SB + SAT_SB);  // last row index of block b
    double* q = sat + (size_t)last * (W + 1) + x;
    run += *q;
    *q = run;
  }
}

// Pass 4: add the previous block's global prefix to the other rows of a block.
__global__ __launch_bounds__(SAT_NT) void sat_cols_fix_kernel(double* sat, int H, int W) {
  const int x = blockIdx.x * SAT_NT + threadIdx.x;
  const int b = blockIdx.y + 1;
  if (x > W) return;
  const int prev_last = b * SAT_SB;  // last row of block b-1
  const double off = sat[(size_t)prev_last * (W + 1) + x];
  const int r0 = 1 + b * SAT_SB, r1 = min(H, r0 + SAT_SB - 1);  // excludes own last row
  for (int y = r0; y < r1; ++y) sat[(size_t)y * (W + 1) + x] += off;
}

int launch_extract(const float* img, int64_t stride, int H, int W, int m, float sigma, int R,
                   float* vol, double* sat, hipStream_t st) {
  ExtractArgs a{};
  a.img = img; a.stride = stride; a.H = H; a.W = W; a.m = m; a.R = R; a.vol = vol; a.sat = sat;
  for (int k = 0; k < m; ++k) {
    double th = k * 3.14159265358979323846 / m;
    a.cs[k] = (float)cos(th);
    a.sn[k] = (float)sin(th);
  }
  double ws[kMaxGaussRadius + 1], tot = 0.0;
  for (int j = 0; j <= R; ++j) { ws[j] = exp(-(double)j * j / (2.0 * sigma * sigma)); tot += (j ? 2 : 1) * ws[j]; }
  for (int j = 0; j <= R; ++j) a.w[j] = (float)(ws[j] / tot);
  const int IW = EX_TX + 2 * R + 2, IH = EX_TY + 2 * R + 2;
  const int GW = EX_TX + 2 * R, GH = EX_TY + 2 * R;
  size_t lds = sizeof(float) * ((size_t)IH * IW + (size_t)m * GH * GW + 2 * (size_t)GH * EX_TX);
  if (lds > kMaxLds) return -1;
  dim3 grid((W + EX_TX - 1) / EX_TX, (H + EX_TY - 1) / EX_TY);
  hipLaunchKernelGGL(cfog_extract_kernel, grid, dim3(EX_NT), lds, st, a);
  if (hipGetLastError() != hipSuccess) return -2;
  if (sat) {
    hipLaunchKernelGGL(sat_rows_kernel, dim3(H + 1), dim3(SAT_NT), 0, st, sat, H, W);
    const int nblk = (H + SAT_SB - 1) / SAT_SB;
    dim3 g2((W + 1 + SAT_NT - 1) / SAT_NT, nblk);
    hipLaunchKernelGGL(sat_cols_local_kernel, g2, dim3(SAT_NT), 0, st, sat, H, W);
    hipLaunchKernelGGL(sat_cols_carry_kernel, dim3((W + 1 + SAT_NT - 1) / SAT_NT), dim3(SAT_NT), 0, st,
                       sat, H, W, nblk);
    if (nblk > 1) {
      dim3 g3((W + 1 + SAT_NT - 1) / SAT_NT, nblk - 1);
      hipLaunchKernelGGL(sat_cols_fix_kernel, g3, dim3(SAT_NT), 0, st, sat, H, W);
    }
    if (hipGetLastError() != hipSuccess) return -2;
  }
  return 0;
}

size_t extract_lds_bytes(int m, int R) {
  const int IW = EX_TX + 2 * R + 2, IH = EX_TY + 2 * R + 2;
  const int GW = EX_TX + 2 * R, GH = EX_TY + 2 * R;
  return sizeof(float) * ((size_t)IH * IW + (size_t)m * GH * GW + 2 * (size_t)GH * EX_TX);
}

}  // namespace cfog
