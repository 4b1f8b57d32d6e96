// C-ABI entry points of libcfog: argument validation, FFT-plan selection
// (pinned, autotuned or default), workspace layout, batched task tables,
// multi-stream bucket launches and the hipGraph cache.  All compute runs in
// the HIP kernels of cfog_extract.hip, match_fft.hip and match_direct.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>
#include "cfog.h"
#include "kernels.hpp"
#include "split_plan.hpp"
#include "trace.hpp"

namespace {

// Streams the FFT-size buckets of a batched call run on.  Every bucket's
// persistent grid fills the GPU by itself; two streams let one bucket's last
// round overlap the next bucket's first (measured on a 64-pair batch: 1, 2, 3
// and 4 streams took 9.72, 9.45, 10.03 and 9.86 ms per call).
constexpr int kBucketStreams = 2;

// Device scratch of match_batch_noalloc: one array per GPU, resident from the
// library's load until the process ends, shared by every call on that GPU.
// Host code never uses its name as an address: the device address of each
// GPU's copy comes from hipGetSymbolAddress (scratch_address below).
constexpr size_t kNoallocScratchBytes = (size_t)CFOG_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

// Device address of `scratch` on the current device (which must be `device`),
// looked up once per device; nullptr if the lookup failed.
void* scratch_address(int device) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) p = nullptr;
  addr[device] = p;
  return p;
}

struct GraphEntry {
  std::vector<unsigned char> key;  // exact call signature (jobs bytes + scalars)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* host_tables = nullptr;     // pinned copy of the task tables the graph uploads
  ~GraphEntry() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (host_tables) (void)hipHostFree(host_tables);
  }
};

uint64_t fnv1a(const unsigned char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

}  // namespace

struct cfog_ctx {
  int device = 0;
  int last_error = 0;
  int num_cus = 0;
  void* ext_ws = nullptr;  // context-owned extraction workspace
  size_t ext_ws_bytes = 0;
  void* stage = nullptr;   // pinned host staging for task tables (eager path)
  size_t stage_bytes = 0;
  hipEvent_t stage_done = nullptr;  // recorded after the last copy out of `stage`
  hipStream_t bucket[kBucketStreams] = {};
  hipEvent_t fork = nullptr, join[kBucketStreams] = {};
  hipStream_t capture = nullptr;
  std::map<long, int> pinned;   // (N, r) -> P chosen by the caller
  std::map<long, int> tuned;    // (N, r, m) -> P chosen by the autotuner
  std::string plan_cache_path;  // optional persistent autotuner cache
  std::unordered_map<uint64_t, std::unique_ptr<GraphEntry>> graphs;
  void* scratch = nullptr;      // this device's static scratch (match_batch_noalloc)
};

namespace {

long nr_key(int N, int r) { return (long)N * 4096 + r; }
long nrm_key(int N, int r, int m) { return ((long)N * 4096 + r) * 128 + m; }

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
  if (j.N < 1 || j.r < 0 || m < 1 || m > cfog::kMaxChannels) return CFOG_EINVAL;
  if (j.N > cfog::kMaxSide || j.r > cfog::kMaxSide) return CFOG_EUNSUPPORTED;
  if (!aligned(j.cps, 16) || !aligned(j.out, 8) || !aligned(j.satA, 8) || !aligned(j.satB, 8) ||
      !aligned(j.volA, 4) || !aligned(j.volB, 4) || !aligned(j.surfaces, 4) || !aligned(j.subpix, 8))
    return CFOG_EINVAL;
  return CFOG_OK;
}

cfog::MatchJob to_device_job(const cfog_job& j, int m, int obj) {
  cfog::MatchJob d{};
  d.volA = j.volA; d.satA = j.satA; d.hA = j.hA; d.wA = j.wA;
  d.volB = j.volB; d.satB = j.satB; d.hB = j.hB; d.wB = j.wB;
  d.cps = reinterpret_cast<const int4*>(j.cps);
  d.n_cps = j.n_cps; d.N = j.N; d.r = j.r; d.m = m;
  d.out = reinterpret_cast<cfog::Result*>(j.out);
  d.surfaces = j.surfaces;
  d.subpix = reinterpret_cast<float2*>(j.subpix);
  d.obj = obj;
  return d;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

const cfog::FftPlan* plan_by_P(int P) {
  int n = 0;
  const cfog::FftPlan* all = cfog::fft_plans(&n);
  for (int i = 0; i < n; ++i)
    if (all[i].P == P) return &all[i];
  return nullptr;
}

// The FFT plan used for (N, r, m): a caller pin, else the autotuner's pick,
// else the smallest fitting size.
const cfog::FftPlan* select_plan(cfog_ctx* ctx, int N, int r, int m) {
  auto it = ctx->pinned.find(nr_key(N, r));
  if (it != ctx->pinned.end()) return plan_by_P(it->second);
  auto jt = ctx->tuned.find(nrm_key(N, r, m));
  if (jt != ctx->tuned.end()) return plan_by_P(jt->second);
  return cfog::choose_fft_plan(N, r);
}

// ------------------------------------------------------------- batch plans

// Channel split of the last round of a launch (split_plan.hpp).
cfog::SplitArgs plan_split(const cfog::FftPlan* p, int n, int S, int m, int Nmax, int Wsmax, int Kmax,
                           size_t* bytes) {
  const cfog::SplitChoice c = cfog::plan_split_choice(p->P, n, S, m, Nmax, Wsmax, Kmax);
  *bytes = c.bytes;
  return cfog::SplitArgs{c.n_whole, c.G, c.slot, nullptr};
}

// Workspace layout of a plain-path launch of job j: the split partials (when
// split_ok), one workgroup per work item.
struct PlainLayout {
  const cfog::FftPlan* p = nullptr;
  cfog::SplitArgs sp{0, 1, 0, nullptr};
  int blocks = 0;
  size_t split_off = 0, total = 0;
};

PlainLayout plain_layout(cfog_ctx* ctx, const cfog_job& j, int m, bool split_ok) {
  PlainLayout L;
  L.p = select_plan(ctx, j.N, j.r, m);
  if (!L.p) return L;
  const int S = cfog::plan_slots(L.p, ctx->num_cus);
  size_t sb = 0;
  L.sp = split_ok ? plan_split(L.p, j.n_cps, S, m, j.N, j.N + 2 * j.r, 2 * j.r + 1, &sb)
                  : cfog::SplitArgs{j.n_cps, 1, 0, nullptr};
  const int items = cfog::split_items(j.n_cps, L.sp);
  L.blocks = items;
  L.split_off = 0;
  L.total = sb;
  return L;
}

struct Bucket {
  const cfog::FftPlan* plan;
  int begin, count, blocks;
  cfog::SplitArgs sp;
  size_t split_off;  // its split partials (sp.G > 1)
};

struct BatchPlan {
  std::vector<cfog::MatchJob> jobs;
  std::vector<int2> tasks;
  std::vector<Bucket> buckets;
  size_t jobs_off = 0, tasks_off = 0, table_bytes = 0, total = 0;
};

// split_budget: workspace bytes the split partials may take (buckets are
// split in order while they fit).
int build_batch(cfog_ctx* ctx, const cfog_job* jobs, int n_jobs, int m, int obj, BatchPlan& B,
                size_t split_budget) {
  std::vector<const cfog::FftPlan*> plans(n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    int rc = validate_job(jobs[i], m);
    if (rc != CFOG_OK) return rc;
    plans[i] = select_plan(ctx, jobs[i].N, jobs[i].r, m);
    if (!plans[i]) return CFOG_EUNSUPPORTED;
  }
  B.jobs.resize(n_jobs);
  for (int i = 0; i < n_jobs; ++i) B.jobs[i] = to_device_job(jobs[i], m, obj);
  int nplans = 0;
  const cfog::FftPlan* all = cfog::fft_plans(&nplans);
  std::vector<size_t> split_bytes;
  for (int p = 0; p < nplans; ++p) {
    Bucket b{&all[p], (int)B.tasks.size(), 0, 0, cfog::SplitArgs{0, 1, 0, nullptr}, 0};
    int Nmax = 0, Wmax = 0, Kmax = 0;
    for (int i = 0; i < n_jobs; ++i)
      if (plans[i] == &all[p] && jobs[i].n_cps > 0) {
        for (int c = 0; c < jobs[i].n_cps; ++c) B.tasks.push_back(make_int2(i, c));
        Nmax = std::max(Nmax, jobs[i].N);
        Wmax = std::max(Wmax, jobs[i].N + 2 * jobs[i].r);
        Kmax = std::max(Kmax, 2 * jobs[i].r + 1);
      }
    b.count = (int)B.tasks.size() - b.begin;
    if (b.count == 0) continue;
    const int S = cfog::plan_slots(b.plan, ctx->num_cus);
    size_t sb = 0;
    b.sp = plan_split(b.plan, b.count, S, m, Nmax, Wmax, Kmax, &sb);
    if (sb > split_budget) {
      b.sp = cfog::SplitArgs{b.count, 1, 0, nullptr};
      sb = 0;
    }
    split_budget -= sb;
    split_bytes.push_back(sb);
    b.blocks = std::min(cfog::split_items(b.count, b.sp), S);
    B.buckets.push_back(b);
  }
  B.jobs_off = 0;
  B.tasks_off = align_up(B.jobs_off + sizeof(cfog::MatchJob) * (size_t)n_jobs, 256);
  size_t end = align_up(B.tasks_off + sizeof(int2) * B.tasks.size(), 256);
  B.table_bytes = B.tasks_off + sizeof(int2) * B.tasks.size() - B.jobs_off;
  for (size_t k = 0; k < B.buckets.size(); ++k) {
    B.buckets[k].split_off = end;
    end += split_bytes[k];
  }
  B.total = end;
  return CFOG_OK;
}

void fill_tables(const BatchPlan& B, void* host) {
  char* h = (char*)host;
  memcpy(h, B.jobs.data(), sizeof(cfog::MatchJob) * B.jobs.size());
  memcpy(h + (B.tasks_off - B.jobs_off), B.tasks.data(), sizeof(int2) * B.tasks.size());
}

// Enqueue the upload of the tables from `host` and one persistent launch per
// bucket, the buckets on the context's streams forked from / joined to `st`.
int enqueue_batch(cfog_ctx* ctx, const BatchPlan& B, char* ws, const void* host, hipStream_t st) {
  if (hipMemcpyAsync(ws + B.jobs_off, host, B.table_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return record(ctx, hipGetLastError());
  const cfog::MatchJob* d_jobs = (const cfog::MatchJob*)(ws + B.jobs_off);
  const int2* d_tasks = (const int2*)(ws + B.tasks_off);
  auto launch_bucket = [&](const Bucket& b, hipStream_t s) {
    cfog::SplitArgs sp = b.sp;
    sp.part = sp.G > 1 ? (float*)(ws + b.split_off) : nullptr;
    return cfog::launch_match_fft(b.plan, cfog::MatchJob{}, d_jobs, d_tasks + b.begin, b.count, b.blocks, sp,
                                  s) == 0 &&
           cfog::launch_split_reduce(cfog::MatchJob{}, d_jobs, d_tasks + b.begin, b.count, sp, s) == 0;
  };
  if (B.buckets.size() == 1) {
    if (!launch_bucket(B.buckets[0], st)) return record(ctx, hipGetLastError());
    return CFOG_OK;
  }
  if (hipEventRecord(ctx->fork, st) != hipSuccess) return record(ctx, hipGetLastError());
  const int ns = std::min<int>(kBucketStreams, (int)B.buckets.size());
  for (int s = 0; s < ns; ++s)
    if (hipStreamWaitEvent(ctx->bucket[s], ctx->fork, 0) != hipSuccess) return record(ctx, hipGetLastError());
  // largest buckets first, round-robin over the streams
  std::vector<int> order(B.buckets.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return (long)B.buckets[a].count * B.buckets[a].plan->P * B.buckets[a].plan->P >
           (long)B.buckets[b].count * B.buckets[b].plan->P * B.buckets[b].plan->P;
  });
  for (size_t k = 0; k < order.size(); ++k) {
    if (!launch_bucket(B.buckets[order[k]], ctx->bucket[k % ns])) return record(ctx, hipGetLastError());
  }
  for (int s = 0; s < ns; ++s) {
    if (hipEventRecord(ctx->join[s], ctx->bucket[s]) != hipSuccess) return record(ctx, hipGetLastError());
    if (hipStreamWaitEvent(st, ctx->join[s], 0) != hipSuccess) return record(ctx, hipGetLastError());
  }
  return CFOG_OK;
}

int ensure_stage(cfog_ctx* ctx, size_t bytes) {
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

// ---------------------------------------------------------------- autotuner

void load_plan_cache(cfog_ctx* ctx) {
  if (ctx->plan_cache_path.empty()) return;
  FILE* f = fopen(ctx->plan_cache_path.c_str(), "r");
  if (!f) return;
  int N, r, m, P;
  while (fscanf(f, "%d %d %d %d", &N, &r, &m, &P) == 4) {
    const cfog::FftPlan* p = plan_by_P(P);
    if (p && N >= 1 && r >= 0 && m >= 1 && m <= cfog::kMaxChannels && cfog::plan_fits(p, N, r)) ctx->tuned[nrm_key(N, r, m)] = P;
  }
  fclose(f);
}

void save_plan_cache(cfog_ctx* ctx) {
  if (ctx->plan_cache_path.empty()) return;
  std::string tmp = ctx->plan_cache_path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  for (auto& kv : ctx->tuned) {
    const long nrm = kv.first;
    const int m = (int)(nrm % 128), nr = (int)(nrm / 128);
    fprintf(f, "%d %d %d %d\n", nr / 4096, nr % 4096, m, kv.second);
  }
  fclose(f);
  rename(tmp.c_str(), ctx->plan_cache_path.c_str());
}

// Time the candidate FFT sizes for (N, r) on up to 2 x #CU control points of
// job j and keep the fastest.  The trial launches write into the job's own
// result buffer; the real launch that follows on the same stream overwrites
// them.
int autotune(cfog_ctx* ctx, const cfog_job& j, int m, hipStream_t st) {
  const long key = nrm_key(j.N, j.r, m);
  if (ctx->pinned.count(nr_key(j.N, j.r)) || ctx->tuned.count(key) || j.n_cps == 0) return CFOG_OK;
  int nplans = 0;
  const cfog::FftPlan* all = cfog::fft_plans(&nplans);
  const cfog::FftPlan* first = cfog::choose_fft_plan(j.N, j.r);
  if (!first) return CFOG_EUNSUPPORTED;
  std::vector<const cfog::FftPlan*> cands;
  for (int p = 0; p < nplans && cands.size() < 3; ++p)
    if (all[p].P >= first->P && cfog::plan_fits(&all[p], j.N, j.r)) cands.push_back(&all[p]);
  if (cands.size() <= 1) {
    ctx->tuned[key] = first->P;
    return CFOG_OK;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return record(ctx, hipGetLastError());
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return record(ctx, hipGetLastError());
  }
  cfog::MatchJob dj = to_device_job(j, m, 0);
  dj.n_cps = std::min(j.n_cps, 2 * ctx->num_cus);
  dj.surfaces = nullptr;
  dj.subpix = nullptr;
  float best = 1e30f;
  int bestP = first->P;
  for (const cfog::FftPlan* p : cands) {
    const int blocks = dj.n_cps;
    float ms = 0.f;
    bool ok = true;
    for (int rep = 0; rep < 2 && ok; ++rep) {  // the first launch warms up
      ok = hipEventRecord(e0, st) == hipSuccess &&
           cfog::launch_match_fft(p, dj, nullptr, nullptr, dj.n_cps, blocks, cfog::SplitArgs{dj.n_cps, 1, 0, nullptr},
                                  st) == 0 &&
           hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    }
    if (!ok) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return record(ctx, hipGetLastError());
    }
    if (ms < best) {
      best = ms;
      bestP = p->P;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->tuned[key] = bestP;
  save_plan_cache(ctx);
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
  std::unique_ptr<cfog_ctx> c(new cfog_ctx());
  c->device = device;
  if (hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    c->num_cus = 256;
  if (hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming) != hipSuccess) return CFOG_EHIP;
  if (hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess) return CFOG_EHIP;
  for (int s = 0; s < kBucketStreams; ++s) {
    if (hipStreamCreateWithFlags(&c->bucket[s], hipStreamNonBlocking) != hipSuccess) return CFOG_EHIP;
    if (hipEventCreateWithFlags(&c->join[s], hipEventDisableTiming) != hipSuccess) return CFOG_EHIP;
  }
  if (hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) return CFOG_EHIP;
  if (cfog::init_kernel_attributes() != 0) return CFOG_EHIP;
  c->scratch = scratch_address(device);
  if (!c->scratch) return CFOG_EHIP;
  if (const char* p = getenv("CFOG_PLAN_CACHE")) c->plan_cache_path = p;
  load_plan_cache(c.get());
  *out = c.release();
  return CFOG_OK;
}

int cfog_ctx_destroy(cfog_ctx* ctx) {
  if (!ctx) return CFOG_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->graphs.clear();
  if (ctx->ext_ws) (void)hipFree(ctx->ext_ws);
  if (ctx->stage_done) (void)hipEventDestroy(ctx->stage_done);
  if (ctx->stage) (void)hipHostFree(ctx->stage);
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  for (int s = 0; s < kBucketStreams; ++s) {
    if (ctx->bucket[s]) (void)hipStreamDestroy(ctx->bucket[s]);
    if (ctx->join[s]) (void)hipEventDestroy(ctx->join[s]);
  }
  if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
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

int cfog_set_plan(cfog_ctx* ctx, int32_t N, int32_t r, int32_t P) {
  if (!ctx || N < 1 || r < 0 || P < 0) return CFOG_EINVAL;
  if (P == 0) {
    ctx->pinned.erase(nr_key(N, r));
  } else {
    const cfog::FftPlan* p = plan_by_P(P);
    if (!p || !cfog::plan_fits(p, N, r)) return CFOG_EUNSUPPORTED;
    ctx->pinned[nr_key(N, r)] = P;
  }
  ctx->graphs.clear();  // captured launches baked in the old choice
  return CFOG_OK;
}

int32_t cfog_plan_for(cfog_ctx* ctx, int32_t N, int32_t r, int32_t m) {
  if (!ctx || N < 1 || r < 0) return 0;
  const cfog::FftPlan* p = select_plan(ctx, N, r, m);
  return p ? p->P : 0;
}

size_t cfog_extract_workspace_size(int32_t H, int32_t W) {
  if (H < 1 || W < 1) return 0;
  return cfog::extract_workspace_bytes(H, W);
}

int cfog_extract(cfog_ctx* ctx, const float* d_img, int32_t H, int32_t W, int64_t row_stride, int32_t m,
                 float sigma, int32_t gauss_radius, float* d_vol, double* d_sat, void* d_ws, size_t ws_bytes,
                 void* stream) {
  return cfog_extract_scheme(ctx, d_img, H, W, row_stride, m, sigma, gauss_radius, 2, d_vol, d_sat, d_ws, ws_bytes,
                             stream);
}

// The context's extraction workspace, grown to `need` bytes.
static int context_extract_ws(cfog_ctx* ctx, size_t need, void** ws) {
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
  *ws = ctx->ext_ws;
  return CFOG_OK;
}

int cfog_extract_scheme(cfog_ctx* ctx, const float* d_img, int32_t H, int32_t W, int64_t row_stride, int32_t m,
                        float sigma, int32_t gauss_radius, int32_t scheme, float* d_vol, double* d_sat, void* d_ws,
                        size_t ws_bytes, void* stream) {
  cfog::TraceRange trace("cfog_extract");
  if (!ctx || !d_img || !d_vol || (scheme != 1 && scheme != 2)) return CFOG_EINVAL;
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
    const int rc = context_extract_ws(ctx, need, &d_ws);
    if (rc != CFOG_OK) return rc;
  }
  int rc = cfog::launch_extract(d_img, row_stride, H, W, m, sigma, R, d_vol, d_sat, d_ws, (hipStream_t)stream,
                                scheme);
  if (rc == -1) return CFOG_EUNSUPPORTED;
  if (rc != 0) return record(ctx, hipGetLastError());
  return CFOG_OK;
}

static std::vector<cfog::ExtractImage> batch_images(const cfog_image* imgs, int32_t n) {
  std::vector<cfog::ExtractImage> v((size_t)n);
  for (int i = 0; i < n; ++i) {
    const cfog_image& c = imgs[i];
    v[i] = cfog::ExtractImage{c.d_img, c.row_stride, c.H, c.W, c.d_vol, c.d_sat};
  }
  return v;
}

size_t cfog_extract_batch_workspace_size(const cfog_image* imgs, int32_t n) {
  if (!imgs || n <= 0) return 0;
  std::vector<int> H((size_t)n), W((size_t)n);
  std::unique_ptr<bool[]> with_sat(new bool[(size_t)n]);
  for (int i = 0; i < n; ++i) {
    if (imgs[i].H < 1 || imgs[i].W < 1) return 0;
    H[i] = imgs[i].H;
    W[i] = imgs[i].W;
    with_sat[i] = imgs[i].d_sat != nullptr;
  }
  return cfog::extract_batch_workspace_bytes(H.data(), W.data(), with_sat.get(), n);
}

int cfog_extract_batch(cfog_ctx* ctx, const cfog_image* imgs, int32_t n, int32_t m, float sigma,
                       int32_t gauss_radius, int32_t scheme, void* d_ws, size_t ws_bytes, void* stream) {
  cfog::TraceRange trace("cfog_extract_batch");
  if (!ctx || n < 0 || (n > 0 && !imgs) || (scheme != 1 && scheme != 2)) return CFOG_EINVAL;
  if (m < 1 || m > cfog::kMaxOrient || !(sigma > 0.f) || !isfinite(sigma)) return CFOG_EINVAL;
  if (n == 0) return CFOG_OK;
  for (int i = 0; i < n; ++i) {
    const cfog_image& c = imgs[i];
    if (!c.d_img || !c.d_vol || c.H < 1 || c.W < 1 || c.row_stride < c.W) return CFOG_EINVAL;
    if (!aligned(c.d_sat, 8)) return CFOG_EINVAL;
  }
  const int R = gauss_radius < 0 ? (int)(4.0 * sigma + 0.5) : gauss_radius;
  if (R > cfog::kMaxGaussRadius) return CFOG_EUNSUPPORTED;
  if (cfog::extract_lds_bytes(m, R) > cfog::kMaxLds) return CFOG_EUNSUPPORTED;
  if (!aligned(d_ws, 8)) return CFOG_EINVAL;
  const size_t need = cfog_extract_batch_workspace_size(imgs, n);
  if (need && d_ws && ws_bytes < need) return CFOG_ENOMEM;
  if (need && !d_ws) {
    const int rc = context_extract_ws(ctx, need, &d_ws);
    if (rc != CFOG_OK) return rc;
  }
  const std::vector<cfog::ExtractImage> v = batch_images(imgs, n);
  const int rc = cfog::launch_extract_batch(v.data(), n, m, sigma, R, d_ws, (hipStream_t)stream, scheme);
  if (rc == -1) return CFOG_EUNSUPPORTED;
  if (rc != 0) return record(ctx, hipGetLastError());
  return CFOG_OK;
}

int cfog_extract_fhog(cfog_ctx* ctx, const float* d_img, int32_t H, int32_t W, int64_t row_stride, int32_t cell,
                      float* d_vol, double* d_sat, void* d_ws, size_t ws_bytes, void* stream) {
  cfog::TraceRange trace("cfog_extract_fhog");
  if (!ctx || !d_img || !d_vol || H < 1 || W < 1 || row_stride < W || cell < 1) return CFOG_EINVAL;
  if (cell > 8) return CFOG_EUNSUPPORTED;
  if (!aligned(d_sat, 8) || !aligned(d_ws, 8)) return CFOG_EINVAL;
  const size_t need = d_sat ? cfog::extract_workspace_bytes(H, W) : 0;
  if (need && d_ws && ws_bytes < need) return CFOG_ENOMEM;
  if (need && !d_ws) {
    const int rc = context_extract_ws(ctx, need, &d_ws);
    if (rc != CFOG_OK) return rc;
  }
  const int rc = cfog::launch_fhog(d_img, row_stride, H, W, cell, d_vol, d_sat, d_ws, (hipStream_t)stream);
  if (rc == -1) return CFOG_EUNSUPPORTED;
  if (rc != 0) return record(ctx, hipGetLastError());
  return CFOG_OK;
}

// Workspace bytes of a match_batch call, with the channel splits (the
// recommended size) or without them (the minimum).
static size_t ws_need(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m, int32_t flags, bool split) {
  if (!ctx || n_jobs < 0 || (n_jobs > 0 && !jobs)) return (size_t)-1;
  const int path = flags & CFOG_PATH_MASK;
  for (int i = 0; i < n_jobs; ++i)
    if (validate_job(jobs[i], m) != CFOG_OK) return (size_t)-1;
  if (path == CFOG_PATH_MFMA_BF16) return cfog::direct_workspace_bytes(jobs, n_jobs, m, ctx->num_cus);
  if (path == CFOG_PATH_PLAIN_FFT) {
    size_t need = 0;  // the jobs run one after another on one stream
    for (int i = 0; i < n_jobs; ++i) {
      if (jobs[i].n_cps == 0) continue;
      const PlainLayout L = plain_layout(ctx, jobs[i], m, split);
      if (!L.p) return 0;  // match_batch reports CFOG_EUNSUPPORTED
      need = std::max(need, L.total);
    }
    return align_up(need, 256);
  }
  BatchPlan B;
  if (build_batch(ctx, jobs, n_jobs, m, 0, B, split ? SIZE_MAX : 0) != CFOG_OK) return 0;
  return B.total;
}

size_t match_batch_workspace_size(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m,
                                  int32_t flags) {
  return ws_need(ctx, jobs, n_jobs, m, flags, !(flags & CFOG_NO_SPLIT));
}

// match_batch without its trace range (match_batch_noalloc calls it too, and
// calls nothing that may allocate)
static int match_batch_run(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m, int32_t flags,
                           void* d_ws, size_t ws_bytes, void* stream) {
  if (!ctx || n_jobs < 0 || (n_jobs > 0 && !jobs)) return CFOG_EINVAL;
  const int path = flags & CFOG_PATH_MASK;
  if (flags & ~(CFOG_PATH_MASK | CFOG_AUTOTUNE | CFOG_USE_GRAPH | CFOG_OBJ_CORR | CFOG_NO_SPLIT)) return CFOG_EINVAL;
  const bool split_ok = !(flags & CFOG_NO_SPLIT);
  const int obj = (flags & CFOG_OBJ_CORR) ? 1 : 0;
  if (path != CFOG_PATH_PLAIN_FFT && path != CFOG_PATH_BATCHED_FFT && path != CFOG_PATH_MFMA_BF16)
    return CFOG_EINVAL;
  if ((flags & CFOG_USE_GRAPH) && path != CFOG_PATH_BATCHED_FFT) return CFOG_EINVAL;
  if ((flags & CFOG_AUTOTUNE) && path == CFOG_PATH_MFMA_BF16) return CFOG_EINVAL;
  for (int i = 0; i < n_jobs; ++i) {
    int rc = validate_job(jobs[i], m);
    if (rc != CFOG_OK) return rc;
  }
  if (!aligned(d_ws, 256)) return CFOG_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)d_ws;

  if (path == CFOG_PATH_MFMA_BF16) {
    const size_t need = cfog::direct_workspace_bytes(jobs, n_jobs, m, ctx->num_cus);
    if (need > 0 && (!d_ws || ws_bytes < need)) return CFOG_ENOMEM;
    int rc = cfog::launch_match_direct(jobs, n_jobs, m, obj, d_ws, ctx->num_cus, st);
    if (rc == -1) return CFOG_EUNSUPPORTED;
    return rc == 0 ? CFOG_OK : record(ctx, hipGetLastError());
  }

  for (int i = 0; i < n_jobs; ++i)
    if (!cfog::choose_fft_plan(jobs[i].N, jobs[i].r)) return CFOG_EUNSUPPORTED;
  const size_t need = ws_need(ctx, jobs, n_jobs, m, flags, false);  // the minimum
  if (need > 0 && (!d_ws || ws_bytes < need)) return CFOG_ENOMEM;
  if (flags & CFOG_AUTOTUNE) {
    // tune each distinct (N, r) on its first job
    std::map<long, int> seen;
    for (int i = 0; i < n_jobs; ++i) {
      if (seen.count(nr_key(jobs[i].N, jobs[i].r)) || jobs[i].n_cps == 0) continue;
      seen[nr_key(jobs[i].N, jobs[i].r)] = 1;
      int rc = autotune(ctx, jobs[i], m, st);
      if (rc != CFOG_OK) return rc;
    }
  }

  if (path == CFOG_PATH_PLAIN_FFT) {
    for (int i = 0; i < n_jobs; ++i) {
      if (jobs[i].n_cps == 0) continue;
      // the channel split only where the workspace holds its partials
      PlainLayout L = plain_layout(ctx, jobs[i], m, split_ok);
      if (L.total > (d_ws ? ws_bytes : 0)) L = plain_layout(ctx, jobs[i], m, false);
      if (L.total > (d_ws ? ws_bytes : 0)) return CFOG_ENOMEM;
      cfog::SplitArgs sp = L.sp;
      sp.part = sp.G > 1 ? (float*)(ws + L.split_off) : nullptr;
      const cfog::MatchJob dj = to_device_job(jobs[i], m, obj);
      if (cfog::launch_match_fft(L.p, dj, nullptr, nullptr, jobs[i].n_cps, L.blocks, sp, st) != 0 ||
          cfog::launch_split_reduce(dj, nullptr, nullptr, jobs[i].n_cps, sp, st) != 0)
        return record(ctx, hipGetLastError());
    }
    return CFOG_OK;
  }

  // ---- batched path
  uint64_t h = 0;
  std::vector<unsigned char> key;
  if (flags & CFOG_USE_GRAPH) {
    const size_t jb = sizeof(cfog_job) * (size_t)n_jobs;
    key.resize(jb + 4 * sizeof(uint64_t));
    if (jb) memcpy(key.data(), jobs, jb);
    uint64_t sc[4] = {(uint64_t)n_jobs, ((uint64_t)m << 32) | (uint32_t)flags, (uint64_t)(uintptr_t)d_ws,
                      (uint64_t)ws_bytes};
    memcpy(key.data() + jb, sc, sizeof(sc));
    h = fnv1a(key.data(), key.size());
    auto it = ctx->graphs.find(h);
    if (it != ctx->graphs.end() && it->second->key == key) {
      if (hipGraphLaunch(it->second->exec, st) != hipSuccess) return record(ctx, hipGetLastError());
      return CFOG_OK;
    }
  }
  BatchPlan B;
  int rc = build_batch(ctx, jobs, n_jobs, m, obj, B, 0);
  if (rc != CFOG_OK) return rc;
  if (B.tasks.empty()) return CFOG_OK;
  if (!d_ws || ws_bytes < B.total) return CFOG_ENOMEM;
  if (split_ok && ws_bytes > B.total) {  // room for channel splits
    BatchPlan Bs;
    rc = build_batch(ctx, jobs, n_jobs, m, obj, Bs, ws_bytes - B.total);
    if (rc != CFOG_OK) return rc;
    if (Bs.total <= ws_bytes) B = std::move(Bs);
  }

  if (!(flags & CFOG_USE_GRAPH)) {
    rc = ensure_stage(ctx, B.table_bytes);
    if (rc != CFOG_OK) return rc;
    fill_tables(B, ctx->stage);
    rc = enqueue_batch(ctx, B, ws, ctx->stage, st);
    if (rc != CFOG_OK) return rc;
    if (hipEventRecord(ctx->stage_done, st) != hipSuccess) return record(ctx, hipGetLastError());
    return CFOG_OK;
  }

  // capture the upload + bucket launches once on the context's capture stream
  std::unique_ptr<GraphEntry> g(new GraphEntry());
  g->key = key;
  if (hipHostMalloc(&g->host_tables, B.table_bytes, hipHostMallocDefault) != hipSuccess) return CFOG_ENOMEM;
  fill_tables(B, g->host_tables);
  if (hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return record(ctx, hipGetLastError());
  rc = enqueue_batch(ctx, B, ws, g->host_tables, ctx->capture);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(ctx->capture, &graph);
  if (rc != CFOG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess) return record(ctx, ec);
  g->graph = graph;
  if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) return record(ctx, hipGetLastError());
  if (hipGraphLaunch(g->exec, st) != hipSuccess) return record(ctx, hipGetLastError());
  if (ctx->graphs.size() >= 64) ctx->graphs.clear();
  ctx->graphs[h] = std::move(g);
  return CFOG_OK;
}

int match_batch(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m, int32_t flags, void* d_ws,
                size_t ws_bytes, void* stream) {
  cfog::TraceRange trace("match_batch");
  return match_batch_run(ctx, jobs, n_jobs, m, flags, d_ws, ws_bytes, stream);
}

size_t cfog_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

int match_batch_noalloc(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m, int32_t flags,
                        void* stream) {
  if (!ctx || n_jobs < 0 || (n_jobs > 0 && !jobs)) return CFOG_EINVAL;
  const int path = flags & CFOG_PATH_MASK;
  // the batched path stages its task tables in pinned host memory and the
  // autotuner creates events: neither runs here
  if (path != CFOG_PATH_PLAIN_FFT && path != CFOG_PATH_MFMA_BF16) return CFOG_EINVAL;
  if (flags & ~(CFOG_PATH_MASK | CFOG_OBJ_CORR | CFOG_NO_SPLIT)) return CFOG_EINVAL;
  if (!ctx->scratch) return CFOG_EHIP;
  const size_t need = ws_need(ctx, jobs, n_jobs, m, flags, false);  // without channel splits
  if (need == (size_t)-1) return CFOG_EINVAL;
  if (need > kNoallocScratchBytes) return CFOG_ENOMEM;
  // the channel splits are taken where their partials also fit, exactly as
  // match_batch does with a workspace of this size
  return match_batch_run(ctx, jobs, n_jobs, m, flags, ctx->scratch, kNoallocScratchBytes, stream);
}

}  // extern "C"
