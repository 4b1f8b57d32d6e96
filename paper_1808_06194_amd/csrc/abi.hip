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
  void* ext_ws = nullptr;  // context-owned extraction workspace
  size_t ext_ws_bytes = 0;
  void* stage = nullptr;   // pinned host staging for task tables
  size_t stage_bytes = 0;
  hipEvent_t stage_done = nullptr;  // recorded after the last copy out of `stage`
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

// Workspace of match_batch: [template-spectrum buffers of the large-P plans]
// [batched path: MatchJob x n_jobs | int2 x total CPs]
struct WsLayout {
  size_t tg = 0;       // bytes of the template-spectrum region
  size_t jobs_off = 0, tasks_off = 0, total = 0;
};

WsLayout ws_layout(cfog_ctx* ctx, const cfog_job* jobs, int n_jobs, int flags,
                   const std::vector<const cfog::FftPlan*>& plans) {
  WsLayout L;
  size_t ncp = 0;
  for (int i = 0; i < n_jobs; ++i) {
    ncp += (size_t)std::max(0, jobs[i].n_cps);
    const cfog::FftPlan* p = plans[i];
    if (p && p->tg_bytes && jobs[i].n_cps > 0) {
      // plain path: one launch per job; batched path: one per plan over all jobs
      const int blocks = flags == CFOG_PATH_PLAIN_FFT ? std::min(jobs[i].n_cps, cfog::plan_slots(p, ctx->num_cus))
                                                      : cfog::plan_slots(p, ctx->num_cus);
      L.tg = std::max(L.tg, (size_t)blocks * p->tg_bytes);
    }
  }
  L.tg = align_up(L.tg, 256);
  L.total = L.tg;
  if (flags == CFOG_PATH_BATCHED_FFT && ncp > 0) {
    L.jobs_off = L.total;
    L.tasks_off = align_up(L.jobs_off + sizeof(cfog::MatchJob) * (size_t)n_jobs, 256);
    L.total = L.tasks_off + sizeof(int2) * ncp;
  }
  return L;
}

int ensure_stage(cfog_ctx* ctx, size_t bytes) {
  if (!ctx->stage_done && hipEventCreateWithFlags(&ctx->stage_done, hipEventDisableTiming) != hipSuccess)
    return record(ctx, hipGetLastError());
  // wait until the previous copy out of the staging buffer has completed
  if (hipEventSynchronize(ctx->stage_done) != hipSuccess) return record(ctx, hipGetLastError());
  if (ctx->stage_bytes >= bytes) return CFOG_OK;
  if (ctx->stage) (void)hipHostFree(ctx->stage);
  ctx->stage = nullptr;
  ctx->stage_bytes = 0;
  const size_t nb = std::max<size_t>(bytes, 1 << 20);
  if (hipHostMalloc(&ctx->stage, nb, hipHostMallocDefault) != hipSuccess) return CFOG_ENOMEM;
  ctx->stage_bytes = nb;
  return CFOG_OK;
}

int resolve_plans(const cfog_job* jobs, int n_jobs, int m, std::vector<const cfog::FftPlan*>& plans) {
  plans.assign(n_jobs, nullptr);
  for (int i = 0; i < n_jobs; ++i) {
    int rc = validate_job(jobs[i], m);
    if (rc != CFOG_OK) return rc;
    plans[i] = cfog::choose_fft_plan(jobs[i].N, jobs[i].r);
    if (!plans[i]) return CFOG_EUNSUPPORTED;
  }
  return CFOG_OK;
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
  if (!ctx) return CFOG_OK;
  if (ctx->ext_ws) (void)hipFree(ctx->ext_ws);
  if (ctx->stage_done) {
    (void)hipEventSynchronize(ctx->stage_done);
    (void)hipEventDestroy(ctx->stage_done);
  }
  if (ctx->stage) (void)hipHostFree(ctx->stage);
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

size_t cfog_extract_workspace_size(int32_t H, int32_t W) {
  if (H < 1 || W < 1) return 0;
  return cfog::extract_workspace_bytes(H, W);
}

int cfog_extract(cfog_ctx* ctx, const float* d_img, int32_t H, int32_t W, int64_t row_stride, int32_t m,
                 float sigma, int32_t gauss_radius, float* d_vol, double* d_sat, void* d_ws, size_t ws_bytes,
                 void* stream) {
  if (!ctx || !d_img || !d_vol) return CFOG_EINVAL;
  if (H < 1 || W < 1 || row_stride < W || m < 1 || m > cfog::kMaxOrient) return CFOG_EINVAL;
  if (!(sigma > 0.f) || !isfinite(sigma)) return CFOG_EINVAL;
  int R = gauss_radius < 0 ? (int)(4.0 * sigma + 0.5) : gauss_radius;
  if (R > cfog::kMaxGaussRadius) return CFOG_EUNSUPPORTED;
  if (!aligned(d_sat, 8)) return CFOG_EINVAL;
  if (cfog::extract_lds_bytes(m, R) > cfog::kMaxLds) return CFOG_EUNSUPPORTED;
  const size_t need = d_sat ? cfog::extract_workspace_bytes(H, W) : 0;
  if (need && d_ws && ws_bytes < need) return CFOG_ENOMEM;
  if (!aligned(d_ws, 8)) return CFOG_EINVAL;
  if (need && !d_ws) {
    if (ctx->ext_ws_bytes < need) {
      if (ctx->ext_ws) {
        // the old workspace may still be in use by queued work on any stream
        if (hipDeviceSynchronize() != hipSuccess) return record(ctx, hipGetLastError());
        (void)hipFree(ctx->ext_ws);
        ctx->ext_ws = nullptr;
        ctx->ext_ws_bytes = 0;
      }
      if (hipMalloc(&ctx->ext_ws, need) != hipSuccess) {
        ctx->ext_ws = nullptr;
        return CFOG_ENOMEM;
      }
      ctx->ext_ws_bytes = need;
    }
    d_ws = ctx->ext_ws;
  }
  int rc = cfog::launch_extract(d_img, row_stride, H, W, m, sigma, R, d_vol, d_sat, d_ws, (hipStream_t)stream);
  if (rc == -1) return CFOG_EUNSUPPORTED;
  if (rc != 0) return record(ctx, hipGetLastError());
  return CFOG_OK;
}

size_t match_batch_workspace_size(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m,
                                  int32_t flags) {
  if (!ctx || n_jobs < 0 || (n_jobs > 0 && !jobs)) return (size_t)-1;
  std::vector<const cfog::FftPlan*> plans;
  if (resolve_plans(jobs, n_jobs, m, plans) == CFOG_EINVAL) return (size_t)-1;
  return ws_layout(ctx, jobs, n_jobs, flags, plans).total;
}

int match_batch(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m, int32_t flags, void* d_ws,
                size_t ws_bytes, void* stream) {
  if (!ctx || n_jobs < 0 || (n_jobs > 0 && !jobs)) return CFOG_EINVAL;
  if (flags != CFOG_PATH_PLAIN_FFT && flags != CFOG_PATH_BATCHED_FFT && flags != CFOG_PATH_MFMA_BF16)
    return CFOG_EINVAL;
  std::vector<const cfog::FftPlan*> plans;
  int rc = resolve_plans(jobs, n_jobs, m, plans);
  if (rc != CFOG_OK) return rc;
  if (flags == CFOG_PATH_MFMA_BF16) return CFOG_EUNSUPPORTED;
  const WsLayout W = ws_layout(ctx, jobs, n_jobs, flags, plans);
  if (W.total > 0 && (!d_ws || ws_bytes < W.total)) return CFOG_ENOMEM;
  if (!aligned(d_ws, 256)) return CFOG_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)d_ws;
  void* tg_ws = W.tg ? ws : nullptr;
  if (flags == CFOG_PATH_PLAIN_FFT) {
    for (int i = 0; i < n_jobs; ++i) {
      if (jobs[i].n_cps == 0) continue;
      const cfog::FftPlan* p = plans[i];
      const int blocks = p->tg_bytes ? std::min(jobs[i].n_cps, cfog::plan_slots(p, ctx->num_cus)) : jobs[i].n_cps;
      if (cfog::launch_match_fft(p, to_device_job(jobs[i], m), nullptr, nullptr, jobs[i].n_cps, blocks, tg_ws, st) !=
          0)
        return record(ctx, hipGetLastError());
    }
    return CFOG_OK;
  }
  // batched: one persistent launch per FFT plan over a (job, cp) task table
  int nplans = 0;
  const cfog::FftPlan* all = cfog::fft_plans(&nplans);
  size_t ncp = 0;
  for (int i = 0; i < n_jobs; ++i) ncp += jobs[i].n_cps;
  if (ncp == 0) return CFOG_OK;
  const size_t table_bytes = W.total - W.jobs_off;
  rc = ensure_stage(ctx, table_bytes);
  if (rc != CFOG_OK) return rc;
  char* stage = (char*)ctx->stage;
  cfog::MatchJob* hj = (cfog::MatchJob*)stage;
  int2* ht = (int2*)(stage + (W.tasks_off - W.jobs_off));
  for (int i = 0; i < n_jobs; ++i) hj[i] = to_device_job(jobs[i], m);
  std::vector<int> bucket_begin(nplans + 1, 0);
  size_t nt = 0;
  for (int p = 0; p < nplans; ++p) {
    bucket_begin[p] = (int)nt;
    for (int i = 0; i < n_jobs; ++i)
      if (plans[i] == &all[p])
        for (int c = 0; c < jobs[i].n_cps; ++c) ht[nt++] = make_int2(i, c);
  }
  bucket_begin[nplans] = (int)nt;
  if (hipMemcpyAsync(ws + W.jobs_off, stage, table_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return record(ctx, hipGetLastError());
  if (hipEventRecord(ctx->stage_done, st) != hipSuccess) return record(ctx, hipGetLastError());
  const cfog::MatchJob* d_jobs = (const cfog::MatchJob*)(ws + W.jobs_off);
  const int2* d_tasks = (const int2*)(ws + W.tasks_off);
  for (int p = 0; p < nplans; ++p) {
    const int n = bucket_begin[p + 1] - bucket_begin[p];
    if (n == 0) continue;
    const int blocks = std::min(n, cfog::plan_slots(&all[p], ctx->num_cus));
    if (cfog::launch_match_fft(&all[p], cfog::MatchJob{}, d_jobs, d_tasks + bucket_begin[p], n, blocks, tg_ws, st) !=
        0)
      return record(ctx, hipGetLastError());
  }
  return CFOG_OK;
}

}  // extern "C"
