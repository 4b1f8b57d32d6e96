// Iterative outlier rejection of control points with a cubic polynomial
// mapping model (Section IV of Ye et al.): fit the model to all kept points by
// least squares, remove the point with the largest residual, and repeat until
// the RMSE falls below a threshold (or ten points, the model's size, remain).
//
// One workgroup per point set; sets of up to 8192 points are held in LDS for
// the whole loop (coordinates and keep flags), larger ones are read from
// global memory.  In FP64:
//   1. once, the 55 + 20 entries of the normal equations (ten monomials of
//      the normalised source coordinates; both target coordinates) summed
//      over all points (per-thread partials, wave shuffles, LDS);
//   per iteration:
//   2. a Cholesky solve of the 10 x 10 system for both right-hand sides;
//   3. residuals |model(p) - q| of the kept points, their squared sum and the
//      largest one (ties to the smaller index);
//   4. removal of that point, whose products are subtracted from the normal
//      equations (a rank-one downdate, so the sums need not be formed again).
#include <hip/hip_runtime.h>
#include <math.h>
#include <limits.h>
#include "cfog.h"

namespace cfog {

constexpr int RJ_NT = 512;
constexpr int RJ_NW = RJ_NT / 64;
constexpr int RJ_T = 10;                   // monomials of a bivariate cubic
constexpr int RJ_G = RJ_T * (RJ_T + 1) / 2;  // unique entries of the normal matrix
constexpr int RJ_V = RJ_G + 2 * RJ_T;      // plus the two right-hand sides
constexpr int RJ_LDS_POINTS = 8192;        // sets up to this size live in LDS

// Dynamic LDS of a set of n points: both coordinate arrays and the flags.
static size_t reject_lds_bytes(int n) {
  return n <= RJ_LDS_POINTS ? (size_t)n * (2 * sizeof(float2) + 1) : 0;
}

__device__ __forceinline__ void cubic_terms(double u, double v, double (&t)[RJ_T]) {
  t[0] = 1.0;
  t[1] = u;
  t[2] = v;
  t[3] = u * u;
  t[4] = u * v;
  t[5] = v * v;
  t[6] = u * u * u;
  t[7] = u * u * v;
  t[8] = u * v * v;
  t[9] = v * v * v;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// RES: the set lives in LDS (n <= RJ_LDS_POINTS).  A compile-time choice, so
// that every point access has a known address space (LDS or global) instead
// of going through flat instructions.
template <bool RES>
__global__ __launch_bounds__(RJ_NT) void reject_kernel(const float2* __restrict__ src, const float2* __restrict__ dst,
                                                       int n, float thr, unsigned char* keep, cfog_reject_result* out) {
  extern __shared__ float2 rj_pts[];
  __shared__ double part[RJ_NW][RJ_V];
  __shared__ double sys[RJ_V];
  __shared__ double coef[RJ_T][2];
  __shared__ double rd[RJ_NW];
  __shared__ int ri[RJ_NW];
  __shared__ double ext[4];
  __shared__ int done, active, removed;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const float2* ps = RES ? rj_pts : src;
  const float2* pd = RES ? rj_pts + n : dst;
  unsigned char* pk = RES ? reinterpret_cast<unsigned char*>(rj_pts + 2 * n) : keep;

  // points into LDS (resident sets); bounding box -> centre and half-extent per axis
  {
    double mn[2] = {INFINITY, INFINITY}, mx[2] = {-INFINITY, -INFINITY};
    for (int i = tid; i < n; i += RJ_NT) {
      const float2 p = src[i];
      if (RES) {
        rj_pts[i] = p;
        rj_pts[n + i] = dst[i];
      }
      mn[0] = fmin(mn[0], (double)p.x);
      mn[1] = fmin(mn[1], (double)p.y);
      mx[0] = fmax(mx[0], (double)p.x);
      mx[1] = fmax(mx[1], (double)p.y);
      pk[i] = 1;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      mn[0] = fmin(mn[0], __shfl_xor(mn[0], o, 64));
      mn[1] = fmin(mn[1], __shfl_xor(mn[1], o, 64));
      mx[0] = fmax(mx[0], __shfl_xor(mx[0], o, 64));
      mx[1] = fmax(mx[1], __shfl_xor(mx[1], o, 64));
    }
    if (lane == 0) {
      part[wv][0] = mn[0];
      part[wv][1] = mn[1];
      part[wv][2] = mx[0];
      part[wv][3] = mx[1];
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < RJ_NW; ++w) {
        mn[0] = fmin(mn[0], part[w][0]);
        mn[1] = fmin(mn[1], part[w][1]);
        mx[0] = fmax(mx[0], part[w][2]);
        mx[1] = fmax(mx[1], part[w][3]);
      }
      for (int a = 0; a < 2; ++a) {
        const double half = 0.5 * (mx[a] - mn[a]);
        ext[a] = 0.5 * (mn[a] + mx[a]);
        ext[2 + a] = half > 0.0 ? half : 1.0;
      }
      done = 0;
      active = n;
      removed = 0;
    }
    __syncthreads();
  }
  const double cx = ext[0], cy = ext[1], sx = ext[2], sy = ext[3];

  // 1. normal equations over all points (every point starts kept)
  {
    double acc[RJ_V];
#pragma unroll
    for (int e = 0; e < RJ_V; ++e) acc[e] = 0.0;
    for (int i = tid; i < n; i += RJ_NT) {
      const float2 p = ps[i], q = pd[i];
      double t[RJ_T];
      cubic_terms(((double)p.x - cx) / sx, ((double)p.y - cy) / sy, t);
      int e = 0;
#pragma unroll
      for (int a = 0; a < RJ_T; ++a)
#pragma unroll
        for (int b = a; b < RJ_T; ++b) acc[e++] += t[a] * t[b];
#pragma unroll
      for (int a = 0; a < RJ_T; ++a) {
        acc[RJ_G + 2 * a] += t[a] * (double)q.x;
        acc[RJ_G + 2 * a + 1] += t[a] * (double)q.y;
      }
    }
#pragma unroll
    for (int e = 0; e < RJ_V; ++e) {
      const double v = wave_sum(acc[e]);
      if (lane == 0) part[wv][e] = v;
    }
    __syncthreads();
    if (tid < RJ_V) {
      double v = 0.0;
      for (int w = 0; w < RJ_NW; ++w) v += part[w][tid];
      sys[tid] = v;
    }
    __syncthreads();
  }

  for (;;) {
    // 2. Cholesky solve (one thread: 10 x 10, every index fixed at compile
    // time so that the factor stays in registers)
    if (tid == 0) {
      // entry (a, b), a >= b, of the symmetric matrix held as the packed upper triangle
      auto A = [&](int a, int b) { return sys[b * RJ_T - b * (b - 1) / 2 + (a - b)]; };
      double L[RJ_T][RJ_T];
      bool ok = true;
#pragma unroll
      for (int j = 0; j < RJ_T; ++j) {
        double d = A(j, j);
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        ok = ok && d > 0.0;
        const double ljj = sqrt(d > 0.0 ? d : 1.0);
        L[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < RJ_T; ++i) {
          double t = A(i, j);
#pragma unroll
          for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
          L[i][j] = t / ljj;
        }
      }
      if (!ok) {
        done = 2;  // singular normal matrix (degenerate point layout)
      } else {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          double y[RJ_T], x[RJ_T];
#pragma unroll
          for (int i = 0; i < RJ_T; ++i) {
            double t = sys[RJ_G + 2 * i + c];
#pragma unroll
            for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
            y[i] = t / L[i][i];
          }
#pragma unroll
          for (int i = RJ_T - 1; i >= 0; --i) {
            double t = y[i];
#pragma unroll
            for (int k = i + 1; k < RJ_T; ++k) t -= L[k][i] * x[k];
            x[i] = t / L[i][i];
            coef[i][c] = x[i];
          }
        }
      }
    }
    __syncthreads();
    if (done == 2) break;
    // 3. residuals, RMSE, largest residual
    double ss = 0.0, best = -1.0;
    int bi = INT_MAX;
    for (int i = tid; i < n; i += RJ_NT) {
      if (!pk[i]) continue;
      const float2 p = ps[i], q = pd[i];
      double t[RJ_T];
      cubic_terms(((double)p.x - cx) / sx, ((double)p.y - cy) / sy, t);
      double mxv = 0.0, myv = 0.0;
#pragma unroll
      for (int a = 0; a < RJ_T; ++a) {
        mxv += t[a] * coef[a][0];
        myv += t[a] * coef[a][1];
      }
      const double ex = mxv - (double)q.x, ey = myv - (double)q.y;
      const double r2 = ex * ex + ey * ey;
      ss += r2;
      const double rr = sqrt(r2);
      if (rr > best || (rr == best && i < bi)) {
        best = rr;
        bi = i;
      }
    }
    ss = wave_sum(ss);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      part[wv][0] = ss;
      rd[wv] = best;
      ri[wv] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < RJ_NW; ++w) {
        s += part[w][0];
        if (rd[w] > best || (rd[w] == best && ri[w] < bi)) {
          best = rd[w];
          bi = ri[w];
        }
      }
      const double rmse = sqrt(s / active);
      if (bi == INT_MAX || !(rmse == rmse)) {
        done = 2;  // a non-finite residual: no point can be chosen
      } else if (rmse < (double)thr || active <= RJ_T) {
        done = 1;
        out->rmse = rmse;
      } else {
        // 4. remove the point and downdate the normal equations
        pk[bi] = 0;
        --active;
        ++removed;
        const float2 p = ps[bi], q = pd[bi];
        double t[RJ_T];
        cubic_terms(((double)p.x - cx) / sx, ((double)p.y - cy) / sy, t);
        int e = 0;
        for (int a = 0; a < RJ_T; ++a)
          for (int b = a; b < RJ_T; ++b) sys[e++] -= t[a] * t[b];
        for (int a = 0; a < RJ_T; ++a) {
          sys[RJ_G + 2 * a] -= t[a] * (double)q.x;
          sys[RJ_G + 2 * a + 1] -= t[a] * (double)q.y;
        }
      }
    }
    __syncthreads();
    if (done) break;
  }
  if (RES)
    for (int i = tid; i < n; i += RJ_NT) keep[i] = pk[i];
  if (tid == 0) {
    out->status = done == 1 ? 0 : 1;
    out->removed = removed;
    out->n_kept = active;
    if (done != 1) out->rmse = NAN;
    for (int a = 0; a < RJ_T; ++a) {
      out->coef[a][0] = done == 1 ? coef[a][0] : NAN;
      out->coef[a][1] = done == 1 ? coef[a][1] : NAN;
    }
    out->centre[0] = cx;
    out->centre[1] = cy;
    out->half_extent[0] = sx;
    out->half_extent[1] = sy;
  }
}

int init_outlier_attributes() {
  return hipFuncSetAttribute((const void*)reject_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)reject_lds_bytes(RJ_LDS_POINTS)) == hipSuccess
             ? 0
             : -2;
}

}  // namespace cfog

extern "C" int cfog_reject_outliers(cfog_ctx* ctx, const float* d_src, const float* d_dst, int32_t n, float threshold,
                                    unsigned char* d_keep, cfog_reject_result* d_result, void* stream) {
  if (!ctx || !d_src || !d_dst || !d_keep || !d_result || n < 10 || n > (1 << 20) || !(threshold >= 0.f) ||
      ((uintptr_t)d_src % 8) != 0 || ((uintptr_t)d_dst % 8) != 0 || ((uintptr_t)d_result % 8) != 0)
    return CFOG_EINVAL;
  const float2* src = reinterpret_cast<const float2*>(d_src);
  const float2* dst = reinterpret_cast<const float2*>(d_dst);
  if (n <= cfog::RJ_LDS_POINTS)
    hipLaunchKernelGGL(cfog::reject_kernel<true>, dim3(1), dim3(cfog::RJ_NT), cfog::reject_lds_bytes(n),
                       (hipStream_t)stream, src, dst, n, threshold, d_keep, d_result);
  else
    hipLaunchKernelGGL(cfog::reject_kernel<false>, dim3(1), dim3(cfog::RJ_NT), 0, (hipStream_t)stream, src, dst, n,
                       threshold, d_keep, d_result);
  return hipGetLastError() == hipSuccess ? CFOG_OK : CFOG_EHIP;
}
