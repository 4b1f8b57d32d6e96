// Internal declarations shared by the HIP translation units of libcfog.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cfog {

constexpr int kMaxOrient = 16;        // m <= 16 orientation channels (CFOG extraction)
constexpr int kMaxChannels = 64;      // channels of a volume the matcher takes (FHOG: 36)
constexpr int kMaxGaussRadius = 8;    // Gaussian radius R <= 8 taps each side
constexpr size_t kMaxLds = 160 * 1024;
constexpr int kMaxSide = 1 << 16;      // template sides and radii above this are rejected before any
                                       // arithmetic on them (no path supports them anyway)

// Per-control-point result, 24 bytes (mirrors cfog_result of the C-ABI).
struct Result {
  int dx, dy;
  float best, second;
  int status, pad;
};

// Device-side description of one matching job (mirrors cfog_job).
struct MatchJob {
  const float* volA; const double* satA; int hA, wA;
  const float* volB; const double* satB; int hB, wB;
  const int4* cps; int n_cps;
  int N, r, m;
  Result* out;
  float* surfaces;
  float2* subpix;  // nullable: refined offsets
  int obj;         // 0: SSD (Eq. 4), 1: correlation (Eq. 7)
};

enum : int { kCpOk = 0, kCpOutOfBounds = 1, kCpNonFinite = 2 };

// scheme 2: oriented channels of Eq. 2; scheme 1: binned orientation.
int launch_extract(const float* img, int64_t stride, int H, int W, int m, float sigma, int R,
                   float* vol, double* sat, void* ws, hipStream_t st, int scheme = 2);
// Several images with the same parameters, grouped largest first, up to 8 per
// launch (three launches per group with SATs).  The carry workspaces of the
// images with a SAT follow each other in ws in image order, each rounded up
// to 256 bytes.
struct ExtractImage {
  const float* img;
  int64_t stride;
  int H, W;
  float* vol;
  double* sat;  // nullable
};
int launch_extract_batch(const ExtractImage* ims, int n, int m, float sigma, int R, void* ws, hipStream_t st,
                         int scheme);
size_t extract_batch_workspace_bytes(const int* H, const int* W, const bool* with_sat, int n);
// Pixel-wise HOG (36 channels) with cells of `cell` pixels (1..8); the SAT as
// for the CFOG volume.  0 ok, -1 unsupported cell, -2 HIP error.
int launch_fhog(const float* img, int64_t stride, int H, int W, int cell, float* vol, double* sat, void* ws,
                hipStream_t st);
size_t extract_lds_bytes(int m, int R);
size_t extract_workspace_bytes(int H, int W);

// FFT matcher plans: FFT side P = R1 * R2, NT threads per workgroup, lds
// bytes of dynamic LDS, templates of up to t_rows rows.
struct FftPlan { int P, R1, R2, NT; size_t lds; int t_rows; };
const FftPlan* fft_plans(int* count);
// Smallest supported plan with P >= Ws whose LDS scratch also fits the
// inverse row pass for K = 2r + 1; nullptr if none.
const FftPlan* choose_fft_plan(int N, int r);
// Whether plan p can match template side N with radius r.
bool plan_fits(const FftPlan* p, int N, int r);
// Set the dynamic-LDS limits of every kernel of the library on the current
// device (once per device, from context creation, before any stream capture;
// safe to call from several host threads).  0 on success.
int init_kernel_attributes();
int init_direct_attributes();
int init_harris_attributes();
int init_outlier_attributes();
// Workgroups of this plan that fit the device at once.
int plan_slots(const FftPlan* p, int num_cus);
// Launch the FFT matcher.  d_jobs == nullptr: n_tasks control points of job0
// (plain path).  Otherwise n_tasks (job, cp) pairs from d_tasks over d_jobs.
// Channel split of a launch's last tasks: tasks [0, n_whole) run whole; every
// later task runs as G work items, item g taking the channels
// [g m / G, (g+1) m / G) and writing its correlation surface (K*K floats) to
// part[(task - n_whole) * G + g][slot]; the split-reduce kernel then adds the
// G surfaces in the order g = 0, 1, .. and finishes those tasks.  G = 1: no
// split.  Used when a launch leaves workgroup slots idle in its last round.
struct SplitArgs {
  int n_whole;
  int G;
  int slot;
  float* part;
};

// n_blocks: workgroups (a grid-stride loop covers the remaining items).
int launch_match_fft(const FftPlan* plan, const MatchJob& job0, const MatchJob* d_jobs, const int2* d_tasks,
                     int n_tasks, int n_blocks, const SplitArgs& sp, hipStream_t st);
// Finishes the split tasks [sp.n_whole, n_tasks) (no-op for G = 1).
int launch_split_reduce(const MatchJob& job0, const MatchJob* d_jobs, const int2* d_tasks, int n_tasks,
                        const SplitArgs& sp, hipStream_t st);
// Work items of a launch of n_tasks tasks under sp.
__host__ __device__ inline int split_items(int n_tasks, const SplitArgs& sp) {
  return sp.G > 1 ? sp.n_whole + (n_tasks - sp.n_whole) * sp.G : n_tasks;
}
int init_match_fft_attributes();
int init_extract_attributes();

}  // namespace cfog

#include "cfog.h"
namespace cfog {
// Direct correlation as BF16 MFMA GEMMs with FP32 accumulation (match_direct.hip).
size_t direct_workspace_bytes(const cfog_job* jobs, int n_jobs, int m, int num_cus);
// 0 on success, -1 unsupported configuration, -2 HIP error.
int launch_match_direct(const cfog_job* jobs, int n_jobs, int m, int obj, void* ws, int num_cus, hipStream_t st);
// Whether the direct path supports template side N with radius r.
bool direct_supported(int N, int r);

}  // namespace cfog
