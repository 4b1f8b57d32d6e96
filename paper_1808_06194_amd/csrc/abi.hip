// C-ABI entry points of libcfog: argument validation, plan selection,
// workspace layout and launch sequencing.  All compute runs in the HIP
// kernels of cfog_extract.hip and match_fft.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <algorithm>
#include <vector>
#include "cfog.h"
#include "kernels.hpp"

struct cfog_ctx {
  int device = 0;
  int last_error = 0;
  int num_cus = 0;
};

namespace {

int record(cfog_ctx* ctx, hipError_t e) {
  if (e != hipSuccess) {
    if (ctx) ctx->last_error = (int)e;
    return CFOG_EHIP;
  }
  return CFOG_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

int validate_job(const cfog_job& j, int m) {
  if (!j.volA || !j.satA || !j.volB || !j.satB) return CFOG_EINVAL;
  if (j.n_cps < 0 || (j.n_cps > 0 && (!j.cps || !j.out))) return CFOG_EINVAL;
  if (j.hA < 1 || j.wA < 1 || j.hB < 1 || j.wB < 1) return CFOG_EINVAL;
  if (j.N < 1 || j.r < 0 || m < 1 || m > cfog::kMaxOrient) return CFOG_EINVAL;
  if (!aligned(j.cps, 16) || !aligned(j.out, 8) || !aligned(j.satA, 8) || !aligned(j.satB, 8) ||
      !aligned(j.volA, 4) || !aligned(j.volB, 4) || !aligned(j.surfaces, 4))
    return CFOG_EINVAL;
  return CFOG_OK;
}

cfog::MatchJob to_device_job(const cfog_job& j, int m) {
  cfog::MatchJob d{};
  d.volA = j.volA; d.satA = j.satA; d.hA = j.hA; d.wA = j.wA;
  d.volB = j.volB; d.satB = j.satB; d.hB = j.hB; d.wB = j.wB;
  d.cps = reinterpret_cast<const int4*>(j.cps);
  d.n_cps = j.n_cps; d.N = j.N; d.r = j.r; d.m = m;
  d.out = reinterpret_cast<cfog::Result*>(j.out);
  d.surfaces = j.surfaces;
  return d;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Batched path workspace: [MatchJob x n_jobs][int2 x total CPs]
size_t batched_ws_bytes(const cfog_job* jobs, int n_jobs) {
  size_t n = 0;
  for (int i = 0; i < n_jobs; ++i) n += (size_t)std::max(0, jobs[i].n_cps);
  return align_up(sizeof(cfog::MatchJob) * (size_t)n_jobs, 256) + sizeof(int2) * n;
}

}  // namespace

extern "C" {

int cfog_ctx_create(int device, cfog_ctx** out) {
  if (!out) return CFOG_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return CFOG_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return CFOG_EHIP;
  cfog_ctx* c = new cfog_ctx();
  c->device = device;
  if (hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    c->num_cus = 256;
  *out = c;
  return CFOG_OK;
}

int cfog_ctx_destroy(cfog_ctx* ctx) {
  delete ctx;
  return CFOG_OK;
}

int cfog_ctx_last_error(cfog_ctx* ctx) {
  if (!ctx) return CFOG_EINVAL;
  int e = ctx->last_error;
  ctx->last_error = 0;
  return e;
}

const char* cfog_status_str(int s) {
  switch (s) {
    case CFOG_OK: return "ok";
    case CFOG_EINVAL: return "invalid argument";
    case CFOG_EUNSUPPORTED: return "unsupported configuration";
    case CFOG_ENOMEM: return "workspace too small or allocation failed";
    case CFOG_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int32_t cfog_max_window(void) {
  int n = 0;
  const cfog::FftPlan* p = cfog::fft_plans(&n);
  return p[n - 1].P;
}

int32_t cfog_fft_size(int32_t N, int32_t r) {
  if (N < 1 || r < 0) return 0;
  const cfog::FftPlan* p = cfog::choose_fft_plan(N, r);
  return p ? p->P : 0;
}

int cfog_extract(cfog_ctx* ctx, const float* d_img, int32_t H, int32_t W, int64_t row_stride, int32_t m,
                 float sigma, int32_t gauss_radius, float* d_vol, double* d_sat, void* stream) {
  if (!ctx || !d_img || !d_vol) return CFOG_EINVAL;
  if (H < 1 || W < 1 || row_stride < W || m < 1 || m > cfog::kMaxOrient) return CFOG_EINVAL;
  if (!(sigma > 0.f) || !isfinite(sigma)) return CFOG_EINVAL;
  int R = gauss_radius < 0 ? (int)(4.0 * sigma + 0.5) : gauss_radius;
  if (R > cfog::kMaxGaussRadius) return CFOG_EUNSUPPORTED;
  if (!aligned(d_sat, 8)) return CFOG_EINVAL;
  if (cfog::extract_lds_bytes(m, R) > cfog::kMaxLds) return CFOG_EUNSUPPORTED;
  int rc = cfog::launch_extract(d_img, row_stride, H, W, m, sigma, R, d_vol, d_sat, (hipStream_t)stream);
  if (rc == -1) return CFOG_EUNSUPPORTED;
  if (rc != 0) return record(ctx, hipGetLastError());
  return CFOG_OK;
}

size_t match_batch_workspace_size(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m,
                                  int32_t flags) {
  if (!ctx || n_jobs < 0 || (n_jobs > 0 && !jobs)) return (size_t)-1;
  for (int i = 0; i < n_jobs; ++i)
    if (validate_job(jobs[i], m) != CFOG_OK) return (size_t)-1;
  if (flags == CFOG_PATH_BATCHED_FFT) return batched_ws_bytes(jobs, n_jobs);
  return 0;
}

int match_batch(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m, int32_t flags, void* d_ws,
                size_t ws_bytes, void* stream) {
  if (!ctx || n_jobs < 0 || (n_jobs > 0 && !jobs)) return CFOG_EINVAL;
  if (flags != CFOG_PATH_PLAIN_FFT && flags != CFOG_PATH_BATCHED_FFT && flags != CFOG_PATH_MFMA_BF16)
    return CFOG_EINVAL;
  std::vector<const cfog::FftPlan*> plans(n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    int rc = validate_job(jobs[i], m);
    if (rc != CFOG_OK) return rc;
    plans[i] = cfog::choose_fft_plan(jobs[i].N, jobs[i].r);
    if (!plans[i]) return CFOG_EUNSUPPORTED;
  }
  hipStream_t st = (hipStream_t)stream;
  if (flags == CFOG_PATH_MFMA_BF16) return CFOG_EUNSUPPORTED;
  if (flags == CFOG_PATH_PLAIN_FFT) {
    for (int i = 0; i < n_jobs; ++i) {
      if (jobs[i].n_cps == 0) continue;
      if (cfog::launch_match_fft_plain(plans[i], to_device_job(jobs[i], m), st) != 0)
        return record(ctx, hipGetLastError());
    }
    return CFOG_OK;
  }
  // batched: one persistent launch per FFT plan over a (job, cp) task table
  const size_t need = batched_ws_bytes(jobs, n_jobs);
  if (need > 0 && (!d_ws || ws_bytes < need)) return CFOG_ENOMEM;
  if (!aligned(d_ws, 256)) return CFOG_EINVAL;
  std::vector<cfog::MatchJob> hj(n_jobs);
  for (int i = 0; i < n_jobs; ++i) hj[i] = to_device_job(jobs[i], m);
  int nplans = 0;
  const cfog::FftPlan* all = cfog::fft_plans(&nplans);
  std::vector<int2> tasks;
  std::vector<int> bucket_begin(nplans + 1, 0);
  for (int p = 0; p < nplans; ++p) {
    bucket_begin[p] = (int)tasks.size();
    for (int i = 0; i < n_jobs; ++i)
      if (plans[i] == &all[p])
        for (int c = 0; c < jobs[i].n_cps; ++c) tasks.push_back(make_int2(i, c));
  }
  bucket_begin[nplans] = (int)tasks.size();
  if (tasks.empty()) return CFOG_OK;
  char* ws = (char*)d_ws;
  cfog::MatchJob* d_jobs = (cfog::MatchJob*)ws;
  int2* d_tasks = (int2*)(ws + align_up(sizeof(cfog::MatchJob) * (size_t)n_jobs, 256));
  if (hipMemcpyAsync(d_jobs, hj.data(), sizeof(cfog::MatchJob) * n_jobs, hipMemcpyHostToDevice, st) != hipSuccess)
    return record(ctx, hipGetLastError());
  if (hipMemcpyAsync(d_tasks, tasks.data(), sizeof(int2) * tasks.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return record(ctx, hipGetLastError());
  for (int p = 0; p < nplans; ++p) {
    int n = bucket_begin[p + 1] - bucket_begin[p];
    if (n == 0) continue;
    int per_cu = std::max<int>(1, (int)(cfog::kMaxLds / all[p].lds));
    per_cu = std::min(per_cu, std::max(1, 2048 / all[p].NT));
    int blocks = std::min(n, ctx->num_cus * per_cu);
    if (cfog::launch_match_fft_tasks(&all[p], d_jobs, d_tasks + bucket_begin[p], n, blocks, st) != 0)
      return record(ctx, hipGetLastError());
  }
  // the host task table must outlive the asynchronous copy
  if (hipStreamSynchronize(st) != hipSuccess) return record(ctx, hipGetLastError());
  return CFOG_OK;
}

}  // extern "C"
