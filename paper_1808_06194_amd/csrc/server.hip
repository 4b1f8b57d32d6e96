// Matching server (the serving entry points of cfog.h): resident CFOG volumes,
// admission by device memory, continuous batching over several streams.
//
// One host worker thread owns all device work:
//   1. takes newly submitted requests into the scheduler (sched.hpp);
//   2. retires finished batches (event query), copies their results from the
//      slot's pinned staging into the callers' buffers and reports them;
//   3. for every idle slot, forms the next batch in arrival order and enqueues
//      it on the slot's stream: CFOG extraction of pairs that just became
//      resident, waits on the extraction events of the other pairs it reads,
//      the CP upload, one match_batch call, the result download, an event.
// Slots run concurrently, so batches formed while others execute overlap on
// the device.  Each slot has its own cfog_ctx (its streams and staging), its
// own match workspace and fixed device / pinned staging sized by the
// per-batch limits; the pair volumes live in one device region managed by
// the scheduler's arena.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <time.h>
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>
#include "cfog.h"
#include "kernels.hpp"
#include "sched.hpp"
#include "trace.hpp"
#include "window.hpp"

namespace {

using cfog::serve::round_up;

int64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000 + ts.tv_nsec;
}

struct PairImg {
  const float* img[2];
  int h[2], w[2];
  int64_t stride[2];
  size_t vol_off[2], sat_off[2], ws_off;  // offsets inside the pair's block
  size_t ws_bytes;
  hipEvent_t ready = nullptr;  // recorded after the pair's last extraction
};

struct Req {
  int64_t id;
  int pair;
  std::vector<cfog_cp> cps;  // the points inside both images (sent to the device)
  std::vector<int32_t> idx;  // their positions in the caller's list
  int n_all;                 // points of the request
  int N, r;
  cfog_result* h_out;
  float* h_surf;
  int64_t t_submit = 0, t_admit = 0, t_launch = 0;
};

struct Slot {
  cfog_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  void* ws = nullptr;            // match_batch workspace
  size_t ws_bytes = 0;
  cfog_cp* d_cps = nullptr;      // device staging
  cfog_result* d_out = nullptr;
  float* d_surf = nullptr;
  cfog_cp* h_cps = nullptr;      // pinned host staging
  cfog_result* h_out = nullptr;
  float* h_surf = nullptr;
  bool busy = false;
  cfog::serve::Batch batch;
  std::vector<Req*> reqs;
};

// Upper bound of match_batch's workspace for one batch of at most max_cps
// control points in max_jobs jobs: the job table and the task table (the
// server runs without channel splits).
size_t match_ws_bound(int path, int num_cus, int max_cps, int max_jobs) {
  (void)num_cus;
  if (path == CFOG_PATH_MFMA_BF16) return 0;
  return round_up(sizeof(cfog::MatchJob) * (size_t)max_jobs, 256) + sizeof(int2) * (size_t)max_cps + 256;
}

bool supported(int path, int N, int r) {
  if (path == CFOG_PATH_MFMA_BF16) return cfog::direct_supported(N, r);
  return cfog::choose_fft_plan(N, r) != nullptr;
}

}  // namespace

struct cfog_server {
  int device = 0;
  cfog_server_config cfg{};
  int num_cus = 0;
  char* arena = nullptr;
  size_t fixed_bytes = 0;
  std::unique_ptr<cfog::serve::Scheduler> sched;
  std::vector<PairImg> pairs;
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> incoming;
  std::unordered_map<int64_t, Req*> waiting;  // in the scheduler, not yet launched
  std::deque<cfog_request_info> done;
  std::thread worker;
  bool stop = false;
  int failed = 0;  // first device failure (a negative status); sticky
  int64_t next_id = 0, submitted = 0;
  int64_t done_at_submit = 0;  // requests with no point inside the images
  int in_flight = 0, max_in_flight = 0;
};

namespace {

void report(cfog_server* s, Req* r, int status, int batch_reqs) {
  cfog_request_info info{};
  info.id = r->id;
  info.status = status;
  info.n_cps = (int32_t)r->n_all;
  info.t_submit_ns = r->t_submit;
  info.t_admit_ns = r->t_admit;
  info.t_launch_ns = r->t_launch;
  info.t_done_ns = now_ns();
  info.batch_reqs = batch_reqs;
  s->done.push_back(info);
  delete r;
}

// Enqueue one batch on slot `sl`.  Called with the server lock held.
int launch(cfog_server* s, Slot& sl) {
  const int m = s->cfg.m;
  for (int pid : sl.batch.extract) {
    PairImg& p = s->pairs[pid];
    char* base = s->arena + s->sched->pair(pid).off;
    for (int k = 0; k < 2; ++k) {
      int rc = cfog_extract(sl.ctx, p.img[k], p.h[k], p.w[k], p.stride[k], m, s->cfg.sigma, -1,
                            (float*)(base + p.vol_off[k]), (double*)(base + p.sat_off[k]), base + p.ws_off,
                            p.ws_bytes, sl.st);
      if (rc != CFOG_OK) return rc;
    }
    if (hipEventRecord(p.ready, sl.st) != hipSuccess) return CFOG_EHIP;
  }
  std::vector<int> seen;
  for (const auto& q : sl.batch.reqs) {
    if (std::find(seen.begin(), seen.end(), q.pair) != seen.end()) continue;
    seen.push_back(q.pair);
    const PairImg& p = s->pairs[q.pair];
    if (hipStreamWaitEvent(sl.st, p.ready, 0) != hipSuccess) return CFOG_EHIP;
  }
  std::vector<cfog_job> jobs;
  jobs.reserve(sl.reqs.size());
  size_t cp_off = 0, sf_off = 0;
  for (Req* r : sl.reqs) {
    const PairImg& p = s->pairs[r->pair];
    const char* base = s->arena + s->sched->pair(r->pair).off;
    const size_t n = r->cps.size(), K = 2 * (size_t)r->r + 1;
    memcpy(sl.h_cps + cp_off, r->cps.data(), n * sizeof(cfog_cp));
    cfog_job j{};
    j.volA = (const float*)(base + p.vol_off[0]);
    j.satA = (const double*)(base + p.sat_off[0]);
    j.hA = p.h[0];
    j.wA = p.w[0];
    j.volB = (const float*)(base + p.vol_off[1]);
    j.satB = (const double*)(base + p.sat_off[1]);
    j.hB = p.h[1];
    j.wB = p.w[1];
    j.cps = sl.d_cps + cp_off;
    j.n_cps = (int32_t)n;
    j.N = r->N;
    j.r = r->r;
    j.out = sl.d_out + cp_off;
    j.surfaces = r->h_surf ? sl.d_surf + sf_off : nullptr;
    j.subpix = nullptr;
    jobs.push_back(j);
    cp_off += n;
    if (r->h_surf) sf_off += n * K * K;
  }
  if (hipMemcpyAsync(sl.d_cps, sl.h_cps, cp_off * sizeof(cfog_cp), hipMemcpyHostToDevice, sl.st) != hipSuccess)
    return CFOG_EHIP;
  // whole points: a request's results must not depend on its batch
  int rc = match_batch(sl.ctx, jobs.data(), (int32_t)jobs.size(), m, s->cfg.flags | CFOG_NO_SPLIT, sl.ws,
                       sl.ws_bytes, sl.st);
  if (rc != CFOG_OK) return rc;
  if (hipMemcpyAsync(sl.h_out, sl.d_out, cp_off * sizeof(cfog_result), hipMemcpyDeviceToHost, sl.st) != hipSuccess)
    return CFOG_EHIP;
  if (sf_off && hipMemcpyAsync(sl.h_surf, sl.d_surf, sf_off * sizeof(float), hipMemcpyDeviceToHost, sl.st) !=
                    hipSuccess)
    return CFOG_EHIP;
  if (hipEventRecord(sl.done, sl.st) != hipSuccess) return CFOG_EHIP;
  return CFOG_OK;
}

// Results of the points of request r that were sent to the device (res,
// surf: in the order of r->idx) into the caller's buffers; the other points
// are outside an image and get the out-of-bounds result.
void scatter_results(const Req* r, const cfog_result* res, const float* surf) {
  const size_t KK = (2 * (size_t)r->r + 1) * (2 * (size_t)r->r + 1);
  const cfog_result oob{0, 0, NAN, NAN, CFOG_CP_OUT_OF_BOUNDS, 0};
  size_t k = 0;
  for (int i = 0; i < r->n_all; ++i) {
    const bool sent = k < r->idx.size() && r->idx[k] == i;
    r->h_out[i] = sent ? res[k] : oob;
    if (r->h_surf) {
      float* dst = r->h_surf + (size_t)i * KK;
      if (sent)
        memcpy(dst, surf + k * KK, KK * sizeof(float));
      else
        std::fill(dst, dst + KK, NAN);
    }
    k += sent;
  }
}

// Retire the slot's batch: copy results out (status CFOG_OK) or fail it.
void retire(cfog_server* s, Slot& sl, int status) {
  size_t cp_off = 0, sf_off = 0;
  const int nb = (int)sl.reqs.size();
  for (Req* r : sl.reqs) {
    const size_t n = r->cps.size(), K = 2 * (size_t)r->r + 1;
    if (status == CFOG_OK) scatter_results(r, sl.h_out + cp_off, r->h_surf ? sl.h_surf + sf_off : nullptr);
    cp_off += n;
    if (r->h_surf) sf_off += n * K * K;
    report(s, r, status, nb);
  }
  sl.reqs.clear();
  s->sched->complete(sl.batch);
  sl.batch = cfog::serve::Batch{};
  sl.busy = false;
  --s->in_flight;
}

void fail_all_pending(cfog_server* s) {
  for (const auto& q : s->sched->drop_pending()) {
    auto it = s->waiting.find(q.id);
    if (it == s->waiting.end()) continue;
    Req* r = it->second;
    s->waiting.erase(it);
    report(s, r, s->failed, 0);
  }
}

void worker_main(cfog_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progressed = false;
    while (!s->incoming.empty()) {
      Req* r = s->incoming.front();
      s->incoming.pop_front();
      cfog::serve::Request q;
      q.id = r->id;
      q.pair = r->pair;
      q.n_cps = (int)r->cps.size();
      q.surf_values = r->h_surf ? r->cps.size() * (size_t)(2 * r->r + 1) * (2 * r->r + 1) : 0;
      s->waiting[r->id] = r;
      s->sched->submit(q);
    }
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t e = hipEventQuery(sl.done);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess && !s->failed) s->failed = CFOG_EHIP;
      retire(s, sl, e == hipSuccess ? CFOG_OK : CFOG_EHIP);
      progressed = true;
    }
    if (s->failed) fail_all_pending(s);
    for (Slot& sl : s->slots) {
      if (s->failed || sl.busy) continue;
      if (!s->sched->next_batch(&sl.batch)) break;
      const int64_t t = now_ns();
      for (const auto& q : sl.batch.reqs) {
        Req* r = s->waiting[q.id];
        s->waiting.erase(q.id);
        r->t_admit = t;
        sl.reqs.push_back(r);
      }
      sl.busy = true;
      s->max_in_flight = std::max(s->max_in_flight, ++s->in_flight);
      const int rc = launch(s, sl);
      const int64_t tl = now_ns();
      for (Req* r : sl.reqs) r->t_launch = tl;
      if (rc != CFOG_OK) {
        // the batch may be partly enqueued: wait for what was, then fail it
        // and drop the pairs it should have extracted
        (void)hipStreamSynchronize(sl.st);
        if (rc == CFOG_EHIP && !s->failed) s->failed = CFOG_EHIP;
        const std::vector<int> ext = sl.batch.extract;
        retire(s, sl, rc);
        for (int pid : ext) s->sched->forget(pid);
      }
      progressed = true;
    }
    if (progressed) s->cv_done.notify_all();
    const bool busy = s->in_flight > 0;
    if (!busy && s->incoming.empty() && s->sched->pending() == 0) {
      if (s->stop) break;
      s->cv_work.wait(lk, [&] { return s->stop || !s->incoming.empty(); });
      continue;
    }
    if (!progressed) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

void free_slot(Slot& sl) {
  if (sl.st) (void)hipStreamSynchronize(sl.st);
  if (sl.done) (void)hipEventDestroy(sl.done);
  if (sl.st) (void)hipStreamDestroy(sl.st);
  if (sl.ws) (void)hipFree(sl.ws);
  if (sl.d_cps) (void)hipFree(sl.d_cps);
  if (sl.d_out) (void)hipFree(sl.d_out);
  if (sl.d_surf) (void)hipFree(sl.d_surf);
  if (sl.h_cps) (void)hipHostFree(sl.h_cps);
  if (sl.h_out) (void)hipHostFree(sl.h_out);
  if (sl.h_surf) (void)hipHostFree(sl.h_surf);
  if (sl.ctx) (void)cfog_ctx_destroy(sl.ctx);
  sl = Slot{};
}

void free_server(cfog_server* s) {
  for (Slot& sl : s->slots) free_slot(sl);
  for (PairImg& p : s->pairs)
    if (p.ready) (void)hipEventDestroy(p.ready);
  if (s->arena) (void)hipFree(s->arena);
  delete s;
}

}  // namespace

extern "C" {

int cfog_server_create(int device, const cfog_server_config* cfg_in, cfog_server** out) {
  if (!out) return CFOG_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CFOG_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return CFOG_EHIP;
  cfog_server_config c{};
  if (cfg_in) {
    c = *cfg_in;
  } else {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return CFOG_EHIP;
    c.hbm_budget = fr / 10 * 8;
    c.n_slots = 4;
    c.max_batch_cps = 8192;
    c.max_batch_reqs = 256;
    c.m = 9;
    c.sigma = 0.8f;
    c.flags = CFOG_PATH_BATCHED_FFT;
    c.max_batch_surf = (size_t)1 << 22;
  }
  const int path = c.flags & CFOG_PATH_MASK;
  if (c.n_slots < 1 || c.n_slots > 16 || c.max_batch_cps < 1 || c.max_batch_reqs < 1 || c.m < 1 ||
      c.m > cfog::kMaxOrient || !(c.sigma > 0.f) || (int)(4.0 * c.sigma + 0.5) > cfog::kMaxGaussRadius ||
      (c.flags & ~(CFOG_PATH_MASK | CFOG_OBJ_CORR)) ||
      (path != CFOG_PATH_BATCHED_FFT && path != CFOG_PATH_PLAIN_FFT && path != CFOG_PATH_MFMA_BF16))
    return CFOG_EINVAL;
  std::unique_ptr<cfog_server> s(new cfog_server());
  s->device = device;
  s->cfg = c;
  if (hipDeviceGetAttribute(&s->num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    s->num_cus = 256;
  const size_t ws = match_ws_bound(path, s->num_cus, c.max_batch_cps, c.max_batch_reqs);
  const size_t per_slot = round_up(ws, 256) + round_up(sizeof(cfog_cp) * c.max_batch_cps, 256) +
                          round_up(sizeof(cfog_result) * c.max_batch_cps, 256) +
                          round_up(sizeof(float) * std::max<size_t>(c.max_batch_surf, 1), 256);
  s->fixed_bytes = per_slot * c.n_slots;
  if (c.hbm_budget <= s->fixed_bytes + (1 << 20)) return CFOG_ENOMEM;
  const size_t arena_bytes = (c.hbm_budget - s->fixed_bytes) / 256 * 256;
  cfog::serve::Limits lim;
  lim.max_batch_cps = c.max_batch_cps;
  lim.max_batch_reqs = c.max_batch_reqs;
  lim.max_batch_surf = c.max_batch_surf;
  s->sched.reset(new cfog::serve::Scheduler(arena_bytes, lim));
  cfog_server* raw = s.release();
  auto fail = [&](int rc) {
    free_server(raw);
    return rc;
  };
  if (hipMalloc(&raw->arena, arena_bytes) != hipSuccess) {
    raw->arena = nullptr;
    return fail(CFOG_ENOMEM);
  }
  raw->slots.resize(c.n_slots);
  for (Slot& sl : raw->slots) {
    int rc = cfog_ctx_create(device, &sl.ctx);
    if (rc != CFOG_OK) return fail(rc);
    if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess) return fail(CFOG_EHIP);
    if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) return fail(CFOG_EHIP);
    sl.ws_bytes = ws;
    if ((ws && hipMalloc(&sl.ws, ws) != hipSuccess) ||
        hipMalloc(&sl.d_cps, sizeof(cfog_cp) * c.max_batch_cps) != hipSuccess ||
        hipMalloc(&sl.d_out, sizeof(cfog_result) * c.max_batch_cps) != hipSuccess ||
        hipMalloc(&sl.d_surf, sizeof(float) * std::max<size_t>(c.max_batch_surf, 1)) != hipSuccess)
      return fail(CFOG_ENOMEM);
    if (hipHostMalloc(&sl.h_cps, sizeof(cfog_cp) * c.max_batch_cps, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&sl.h_out, sizeof(cfog_result) * c.max_batch_cps, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&sl.h_surf, sizeof(float) * std::max<size_t>(c.max_batch_surf, 1), hipHostMallocDefault) !=
            hipSuccess)
      return fail(CFOG_ENOMEM);
  }
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return CFOG_OK;
}

int cfog_server_destroy(cfog_server* s) {
  if (!s) return CFOG_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->waiting) delete kv.second;
  for (Req* r : s->incoming) delete r;
  (void)hipSetDevice(s->device);
  free_server(s);
  return CFOG_OK;
}

int cfog_server_add_pair(cfog_server* s, const float* d_imgA, int32_t hA, int32_t wA, int64_t strideA,
                         const float* d_imgB, int32_t hB, int32_t wB, int64_t strideB, int32_t* pair_id) {
  cfog::TraceRange trace("cfog_server_add_pair");
  if (!s || !d_imgA || !d_imgB || !pair_id || hA < 1 || wA < 1 || hB < 1 || wB < 1 || strideA < wA ||
      strideB < wB)
    return CFOG_EINVAL;
  PairImg p;
  p.img[0] = d_imgA;
  p.img[1] = d_imgB;
  p.h[0] = hA;
  p.w[0] = wA;
  p.h[1] = hB;
  p.w[1] = wB;
  p.stride[0] = strideA;
  p.stride[1] = strideB;
  size_t off = 0;
  for (int k = 0; k < 2; ++k) {
    p.vol_off[k] = off;
    off += round_up(sizeof(float) * (size_t)s->cfg.m * p.h[k] * p.w[k], 256);
    p.sat_off[k] = off;
    off += round_up(sizeof(double) * (size_t)(p.h[k] + 1) * (p.w[k] + 1), 256);
  }
  p.ws_off = off;
  p.ws_bytes = std::max(cfog_extract_workspace_size(hA, wA), cfog_extract_workspace_size(hB, wB));
  off += round_up(p.ws_bytes, 256);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed) return s->failed;
  if (round_up(off, 256) > s->sched->arena().size()) return CFOG_ENOMEM;
  (void)hipSetDevice(s->device);
  if (hipEventCreateWithFlags(&p.ready, hipEventDisableTiming) != hipSuccess) return CFOG_EHIP;
  s->pairs.push_back(p);
  *pair_id = s->sched->add_pair(off);
  return CFOG_OK;
}

int cfog_server_submit(cfog_server* s, int32_t pair_id, const cfog_cp* h_cps, int32_t n_cps, int32_t N, int32_t r,
                       cfog_result* h_out, float* h_surfaces, int64_t* req_id) {
  cfog::TraceRange trace("cfog_server_submit");
  if (!s || !req_id || n_cps < 1 || !h_cps || !h_out || N < 1 || r < 0) return CFOG_EINVAL;
  if (!supported(s->cfg.flags & CFOG_PATH_MASK, N, r)) return CFOG_EUNSUPPORTED;
  const size_t K = 2 * (size_t)r + 1;
  std::unique_ptr<Req> q(new Req());
  q->pair = pair_id;
  q->n_all = n_cps;
  q->N = N;
  q->r = r;
  q->h_out = h_out;
  q->h_surf = h_surfaces;
  bool immediate = false;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed) return s->failed;
    if (pair_id < 0 || pair_id >= s->sched->n_pairs()) return CFOG_EINVAL;
    // only points whose template and search boxes lie inside the images go to
    // the device (the kernels' own test, run here on the host)
    const PairImg& p = s->pairs[pair_id];
    for (int i = 0; i < n_cps; ++i) {
      const cfog_cp& c = h_cps[i];
      if (cfog::cp_boxes(c.x, c.y, c.bx, c.by, N, r, p.h[0], p.w[0], p.h[1], p.w[1]).inside) {
        q->cps.push_back(c);
        q->idx.push_back(i);
      }
    }
    const size_t surf = h_surfaces ? q->cps.size() * K * K : 0;
    if (!q->cps.empty() && !s->sched->feasible(pair_id, (int)q->cps.size(), surf)) return CFOG_ENOMEM;
    q->id = s->next_id++;
    q->t_submit = now_ns();
    *req_id = q->id;
    ++s->submitted;
    if (q->cps.empty()) {
      // nothing to match: every point is out of bounds; reported at once
      scatter_results(q.get(), nullptr, nullptr);
      q->t_admit = q->t_launch = q->t_submit;
      report(s, q.release(), CFOG_OK, 0);
      ++s->done_at_submit;
      immediate = true;
    } else {
      s->incoming.push_back(q.release());
    }
  }
  if (immediate)
    s->cv_done.notify_all();
  else
    s->cv_work.notify_one();
  return CFOG_OK;
}

int cfog_server_poll(cfog_server* s, cfog_request_info* infos, int32_t max, int64_t timeout_us, int32_t* n_done) {
  if (!s || !n_done || max < 0 || (max > 0 && !infos)) return CFOG_EINVAL;
  *n_done = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_us > 0 && max > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !s->done.empty(); });
  int n = 0;
  while (n < max && !s->done.empty()) {
    infos[n++] = s->done.front();
    s->done.pop_front();
  }
  *n_done = n;
  return CFOG_OK;
}

int cfog_server_get_stats(cfog_server* s, cfog_server_stats* o) {
  if (!s || !o) return CFOG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  const auto& st = s->sched->stats();
  *o = cfog_server_stats{};
  o->submitted = s->submitted;
  o->completed = st.completed + s->done_at_submit;
  o->batches = st.batches;
  o->evictions = st.evictions;
  o->extractions = st.extractions;
  o->blocked = st.blocked;
  o->arena_bytes = s->sched->arena().size();
  o->arena_used = s->sched->arena().used();
  o->arena_peak = s->sched->arena().peak();
  o->max_in_flight = s->max_in_flight;
  return CFOG_OK;
}

}  // extern "C"
