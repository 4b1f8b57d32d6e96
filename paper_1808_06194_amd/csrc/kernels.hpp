// Internal declarations shared by the HIP translation units of libcfog.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cfog {

constexpr int kMaxOrient = 16;        // m <= 16 orientation channels
constexpr int kMaxGaussRadius = 8;    // Gaussian radius R <= 8 taps each side
constexpr size_t kMaxLds = 160 * 1024;

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
};

enum : int { kCpOk = 0, kCpOutOfBounds = 1, kCpNonFinite = 2 };

int launch_extract(const float* img, int64_t stride, int H, int W, int m, float sigma, int R,
                   float* vol, double* sat, hipStream_t st);
size_t extract_lds_bytes(int m, int R);

// FFT matcher plans: FFT side P = R1 * R2, NT threads per workgroup.
struct FftPlan { int P, R1, R2, NT; size_t lds; };
const FftPlan* fft_plans(int* count);
// Smallest supported plan with P >= Ws whose LDS scratch also fits the
// inverse row pass for K = 2r + 1; nullptr if none.
const FftPlan* choose_fft_plan(int N, int r);
// Launch the plain FFT matcher: one workgroup per control point of one job.
int launch_match_fft_plain(const FftPlan* plan, const MatchJob& job, hipStream_t st);
// Launch the FFT matcher over a device task table (job index, cp index) for
// jobs that share one plan; grid-stride persistent workgroups.
int launch_match_fft_tasks(const FftPlan* plan, const MatchJob* d_jobs, const int2* d_tasks, int n_tasks,
                           int n_blocks, hipStream_t st);

}  // namespace cfog
