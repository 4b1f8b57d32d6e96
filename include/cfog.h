/*
 * cfog.h - C-ABI of libcfog: CFOG extraction and SSD template matching by
 * 3-D FFT on AMD Instinct MI355X (gfx950).
 *
 * Method: Ye, Bruzzone, Shan, Bovolo, Zhu, "Fast and Robust Matching for
 * Multimodal Remote Sensing Image Registration".
 *   - cfog_extract: the pixel-wise CFOG feature representation (Section III-F:
 *     oriented gradient channels of Eq. 2 smoothed by a 2-D Gaussian in X/Y
 *     and a [1,2,1] kernel along the orientation axis), plus an FP64
 *     summed-area table of the per-pixel energy sum_k D_k^2 (the energy terms
 *     of Eq. 5).
 *   - match_batch: for every control point, the SSD similarity of Eq. 3 over a
 *     search window, evaluated as Eq. 5 with the correlation term by FFT
 *     (Eqs. 8-9), and the matching function of Eq. 4 (argmin).
 *
 * Conventions (apply to every entry point):
 *   - All image, volume, table, control-point and result buffers are DEVICE
 *     pointers owned by the caller; the library never frees them.  Job arrays
 *     (cfog_job) are HOST arrays.  `stream` is a hipStream_t passed as void*
 *     (NULL = the null stream).
 *   - Calls are stream-ordered and asynchronous: a return of CFOG_OK means the
 *     work was validated and enqueued.  Faults during execution surface at the
 *     caller's next synchronisation of that stream; cfog_ctx_last_error()
 *     reports the last HIP error the library saw.
 *   - Errors are negative return codes (never abort, never C++ exceptions).
 *   - A cfog_ctx is not thread-safe: use one per host thread.
 *   - Axes: x = column, y = row.  Layouts are row-major.
 */
#ifndef CFOG_H_
#define CFOG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define CFOG_OK 0
#define CFOG_EINVAL (-1)       /* invalid argument (null pointer, bad size, ...) */
#define CFOG_EUNSUPPORTED (-2) /* valid but not supported (e.g. window too large) */
#define CFOG_ENOMEM (-3)       /* workspace too small / allocation failed */
#define CFOG_EHIP (-4)         /* HIP runtime error at launch */

/* per-control-point status in cfog_result.status */
#define CFOG_CP_OK 0
#define CFOG_CP_OUT_OF_BOUNDS 1 /* template leaves A or search window leaves B */
#define CFOG_CP_NONFINITE 2     /* a similarity value was NaN or infinite */

/* match_batch flags: exactly one path ... */
#define CFOG_PATH_PLAIN_FFT 0x1   /* one FFT launch per job, one workgroup per CP */
#define CFOG_PATH_BATCHED_FFT 0x2 /* all jobs' CPs fused into persistent launches per FFT size */
#define CFOG_PATH_MFMA_BF16 0x4   /* direct correlation as BF16 MFMA GEMMs (FP32 accumulate) */
#define CFOG_PATH_MASK 0xF
/* ... plus optional modifiers */
#define CFOG_AUTOTUNE 0x100  /* FFT paths: time candidate FFT sizes per (N, r) on first use */
#define CFOG_USE_GRAPH 0x200 /* batched path: capture the launches once, replay on identical calls */
#define CFOG_OBJ_CORR 0x400  /* any path: the objective of Eq. 7 (maximise the correlation
                                C(d) = sum D1 * D2 over the window, no energy terms); every
                                similarity value (ssd_best, ssd_second, surfaces) is then -C(d) */
#define CFOG_NO_SPLIT 0x800  /* FFT paths: match every point whole (no channel split, see
                                match_batch), so that its result does not depend on the
                                other points of the call */

typedef struct cfog_ctx cfog_ctx;

/* Create a context bound to HIP device `device` (it becomes current).
 * Returns CFOG_OK and *out, or CFOG_EINVAL / CFOG_EHIP. */
int cfog_ctx_create(int device, cfog_ctx** out);

/* Destroy a context; NULL is accepted.  Frees only what the context owns. */
int cfog_ctx_destroy(cfog_ctx* ctx);

/* Last HIP error code (hipError_t as int) recorded by the context, 0 if none;
 * reading it clears it. */
int cfog_ctx_last_error(cfog_ctx* ctx);

/* Static description of a status code (never NULL). */
const char* cfog_status_str(int status);

/*
 * cfog_extract - CFOG volume of one image (Section III-F, Eq. 2).
 *
 *   d_img       [H][row_stride] fp32 image (row_stride >= W, in elements).
 *   m           number of orientation channels, 1..16 (paper default 9);
 *               theta_k = k*pi/m, k = 0..m-1.
 *   sigma       Gaussian std in pixels (paper default 0.8), > 0.
 *   gauss_radius taps each side, 0..8; -1 selects int(4*sigma + 0.5).
 *   d_vol       output [m][H][W] fp32, planar (plane stride H*W).
 *   d_sat       nullable output [(H+1)][(W+1)] fp64 summed-area table of
 *               Q = sum_k D_k^2 computed from the fp32 volume values:
 *               SAT(y, x) = sum_{y'<y, x'<x} Q(y', x'); row 0 and column 0 are 0.
 *   d_ws        device workspace of ws_bytes >= cfog_extract_workspace_size(H, W)
 *               when d_sat is not NULL; it must stay untouched until the call's
 *               work completes on `stream`.  NULL selects a workspace owned by
 *               the context (calls on several streams must then not overlap).
 *   Borders are replicated (clamp-to-edge) for the gradient and the Gaussian;
 *   gx, gy are central differences by [-1, 0, 1] without a 1/2 factor.
 *   Returns CFOG_EINVAL for null pointers, H or W < 1, m out of range, bad
 *   sigma/radius; CFOG_EUNSUPPORTED if the tile does not fit on chip;
 *   CFOG_ENOMEM if ws_bytes is too small or the context workspace cannot grow.
 */
int cfog_extract(cfog_ctx* ctx, const float* d_img, int32_t H, int32_t W, int64_t row_stride,
                 int32_t m, float sigma, int32_t gauss_radius, float* d_vol, double* d_sat,
                 void* d_ws, size_t ws_bytes, void* stream);

/* cfog_extract with a choice of the oriented-gradient scheme of Section III-F:
 * scheme 2 is Eq. 2 (what cfog_extract computes); scheme 1 bins the gradient
 * orientation, taken modulo 180 degrees, between the two nearest of the m bin
 * centres k*pi/m and splits the gradient magnitude between them with weights
 * falling linearly with the distance to each bin (circularly over the bins).
 * The smoothing, outputs and errors are those of cfog_extract; CFOG_EINVAL
 * for a scheme other than 1 or 2. */
int cfog_extract_scheme(cfog_ctx* ctx, const float* d_img, int32_t H, int32_t W, int64_t row_stride,
                        int32_t m, float sigma, int32_t gauss_radius, int32_t scheme, float* d_vol,
                        double* d_sat, void* d_ws, size_t ws_bytes, void* stream);

/* Pixel-wise HOG (Section III-C, the FHOG descriptor built pixel by pixel):
 * at every pixel the histogram of a block of 2 x 2 cells of `cell` pixels
 * centred on it.  Gradients as in cfog_extract; the unsigned orientation
 * (modulo 180 degrees) is split between the two nearest of 9 bins (centres
 * k*pi/9) linearly in the distance, circularly; a gradient at block offset
 * (dx, dy), |dx|, |dy| <= cell, adds to cell (a, b) with the weight
 * wa(dx) wb(dy), w0(d) = max(0, 1 - |d + cell/2| / cell),
 * w1(d) = max(0, 1 - |d - cell/2| / cell) (pixels beyond the image replicate
 * the border); the 36 values of a pixel are divided by
 * sqrt(sum of their squares + 1e-12).
 *   d_vol   DEVICE out, planar [36][H][W] float: channel (2a + b) * 9 + k is
 *           cell column a (0 left), cell row b (0 top), bin k.
 *   d_sat, d_ws, ws_bytes, stream, H, W, row_stride: as for cfog_extract.
 *   cell    1..8 (CFOG_EUNSUPPORTED above 8, CFOG_EINVAL below 1).
 * The volume is matched by match_batch with m = 36. */
int cfog_extract_fhog(cfog_ctx* ctx, const float* d_img, int32_t H, int32_t W, int64_t row_stride,
                      int32_t cell, float* d_vol, double* d_sat, void* d_ws, size_t ws_bytes,
                      void* stream);

/* Device workspace (bytes) cfog_extract (and cfog_extract_fhog) needs to
 * build the SAT of an H x W image: the larger of
 * 8 * (H * ceil(W/128) + ceil(H/16) * W) (CFOG tiles of 128 x 16) and
 * 8 * (H * ceil(W/64) + ceil(H/32) * W) (pixel-wise HOG tiles of 64 x 32). */
size_t cfog_extract_workspace_size(int32_t H, int32_t W);

/* One image of cfog_extract_batch: the arguments of cfog_extract that differ
 * between images (same meaning, layout and ownership). */
typedef struct cfog_image {
  const float* d_img;  /* DEVICE [H][row_stride] fp32 */
  int64_t row_stride;  /* >= W, in elements */
  int32_t H, W;
  float* d_vol;        /* DEVICE out [m][H][W] fp32 */
  double* d_sat;       /* DEVICE out [(H+1)][(W+1)] fp64, or NULL for no SAT */
} cfog_image;

/* cfog_extract_batch - cfog_extract_scheme (Section III-F, Eq. 2 or scheme 1)
 * of n images with the same m, sigma, radius and scheme, in one stream-ordered
 * call: up to 8 images share each launch, which saves the launch boundaries
 * of per-image calls.  Each image's outputs are bit-identical to those of
 * cfog_extract_scheme on it.
 *   imgs        HOST array of n images (read during the call only).
 *   d_ws        device workspace of ws_bytes >=
 *               cfog_extract_batch_workspace_size(imgs, n), or NULL for the
 *               context's (then calls on several streams must not overlap).
 * Errors as for cfog_extract_scheme, checked for every image before any work
 * is queued; CFOG_EINVAL also for n < 0, or imgs NULL with n > 0.  n = 0
 * queues nothing.  The workspace size is 0 for n <= 0 or imgs NULL. */
size_t cfog_extract_batch_workspace_size(const cfog_image* imgs, int32_t n);
int cfog_extract_batch(cfog_ctx* ctx, const cfog_image* imgs, int32_t n, int32_t m, float sigma,
                       int32_t gauss_radius, int32_t scheme, void* d_ws, size_t ws_bytes, void* stream);

/* One control point: template centre (x, y) in A; search centre (bx, by) in B
 * (a georeferenced prediction; bx = x, by = y when A and B are co-registered).
 * Any int32 values are accepted: a point whose template box
 * [y - N/2, y - N/2 + N) x [x - N/2, x - N/2 + N) leaves A, or whose search box
 * [by - N/2 - r, by - N/2 + N + r) x [bx - N/2 - r, bx - N/2 + N + r) leaves B,
 * gets CFOG_CP_OUT_OF_BOUNDS (the test is computed in 64 bits, so coordinates
 * near INT_MIN or INT_MAX cannot wrap into the image). */
typedef struct {
  int32_t x, y, bx, by;
} cfog_cp;

/* One result (24 bytes).  (dx, dy): A's template at (x, y) best matches B's
 * window centred at (bx + dx, by + dy) (this is -v of Eq. 3).  ssd_best is the
 * minimum SSD (Eq. 3), ssd_second the smallest SSD over all other offsets
 * (+inf when r = 0).
 * Ties go to the smallest row-major index (dy first, then dx).  For a status
 * other than CFOG_CP_OK: dx = dy = 0 and both SSDs are NaN. */
typedef struct {
  int32_t dx, dy;
  float ssd_best, ssd_second;
  int32_t status, pad;
} cfog_result;

/* One matching job: a pair of CFOG volumes (from cfog_extract, with SATs) and
 * a list of control points sharing template side N and search radius r.
 *   Template of CP p: rows [y - N/2, y - N/2 + N), cols [x - N/2, x - N/2 + N) of A.
 *   Offsets d = (dx, dy) in [-r, r]^2, i.e. (2r+1)^2 candidates.
 *   cps      device array of n_cps cfog_cp (16-byte aligned).
 *   out      device array of n_cps cfog_result.
 *   surfaces nullable device array [n_cps][2r+1][2r+1] fp32 of SSD(d),
 *            index [dy + r][dx + r]; NaN for points that are not CFOG_CP_OK.
 *   subpix   nullable device array [n_cps][2] fp32 (fdx, fdy): the best offset
 *            refined to sub-pixel precision (the quadratic fit of Section V-B,
 *            read as a three-point parabola per axis through the best value and
 *            its two axis neighbours: fdx = dx + (S(dx-1) - S(dx+1)) /
 *            (2 (S(dx-1) - 2 S(dx) + S(dx+1))), likewise fdy; an axis whose
 *            neighbour lies outside [-r, r], or whose three values are not
 *            convex, keeps its integer offset); NaN for points that are not
 *            CFOG_CP_OK.  8-byte aligned. */
typedef struct {
  const float* volA;
  const double* satA;
  int32_t hA, wA;
  const float* volB;
  const double* satB;
  int32_t hB, wB;
  const cfog_cp* cps;
  int32_t n_cps;
  int32_t N, r;
  int32_t pad_;
  cfog_result* out;
  float* surfaces;
  float* subpix;
} cfog_job;

/* Device workspace (bytes) recommended for match_batch with these jobs and
 * flags (it includes the channel-split partials described at match_batch);
 * may be 0.  Returns (size_t)-1 for invalid jobs. */
size_t match_batch_workspace_size(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m,
                                  int32_t flags);

/*
 * match_batch - SSD template matching of every control point of every job
 * (Eqs. 3-6, 8-9; Eq. 4 argmin).  Volumes have m channels (1..64: a CFOG volume
 * has 1..16, a pixel-wise HOG volume 36).
 *   jobs        host array of n_jobs jobs (n_jobs >= 0).
 *   flags       one CFOG_PATH_* value, optionally | CFOG_OBJ_CORR (Eq. 7
 *               objective), | CFOG_NO_SPLIT and | CFOG_AUTOTUNE (FFT paths:
 *               the first call for a given (N, r, m) times up to three FFT sizes
 *               on the job's own points and keeps the fastest; with the
 *               environment variable CFOG_PLAN_CACHE naming a file, choices
 *               persist across processes) and | CFOG_USE_GRAPH (batched path:
 *               the task-table upload and the bucket launches are captured into a
 *               hipGraph keyed by the exact jobs array, workspace pointer and size;
 *               identical later calls replay it).  Query the workspace size again
 *               after an autotuning call: a larger FFT size may need more.
 *   d_ws        device workspace of ws_bytes bytes, normally
 *               match_batch_workspace_size(); may be NULL when that size is 0.
 *               It must stay untouched until the work completes on `stream`.
 *               FFT paths: when a launch's control points would leave
 *               workgroup slots idle in its last round, the points of that
 *               round are split by channel groups over several workgroups and
 *               their partial correlations summed (in a fixed order) by a
 *               second kernel; this needs the extra workspace, and a smaller
 *               workspace (down to the minimum without splits) runs unsplit.
 *               Results are deterministic for a given call and workspace
 *               size; a split point differs from a whole one only by FP32
 *               rounding.  CFOG_NO_SPLIT turns splitting off (the plain and
 *               batched paths then return identical bits).
 *   Returns CFOG_EINVAL for invalid jobs, CFOG_EUNSUPPORTED when 2r+1 or
 *   N + 2r exceeds what the chosen path supports (always for N or r above
 *   65536), CFOG_ENOMEM when the
 *   workspace is too small.  Per-point failures are reported in out[].status.
 */
int match_batch(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m, int32_t flags, void* d_ws,
                size_t ws_bytes, void* stream);

/* match_batch_noalloc - match_batch for callers that cannot allocate memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  It allocates nothing, host or device: its workspace is a
 * device array of CFOG_NOALLOC_SCRATCH_MIB MiB that the library holds on each
 * GPU from its load until the process ends (its address is taken once per
 * device by cfog_ctx_create).  The caller still owns and passes the inputs
 * and outputs (the jobs, as for match_batch).
 *   flags   CFOG_PATH_PLAIN_FFT or CFOG_PATH_MFMA_BF16, optionally
 *           | CFOG_OBJ_CORR | CFOG_NO_SPLIT (CFOG_EINVAL for the batched path,
 *           CFOG_AUTOTUNE or CFOG_USE_GRAPH: they stage host tables or time
 *           trial launches).
 *   Results are bit-identical to match_batch with a workspace of
 *   cfog_noalloc_scratch_bytes() bytes (and so to match_batch with its
 *   recommended workspace whenever that is no larger).  The array needs no
 *   clearing between calls (every value read is written earlier in the same
 *   call).  All calls on one GPU share the one array: calls that overlap on
 *   the device (other streams, other threads, other contexts) race and give
 *   undefined results; order them on one stream or synchronise.
 *   Returns CFOG_ENOMEM when the call's workspace without channel splits
 *   exceeds the array, otherwise as match_batch. */
#define CFOG_NOALLOC_SCRATCH_MIB 48
int match_batch_noalloc(cfog_ctx* ctx, const cfog_job* jobs, int32_t n_jobs, int32_t m, int32_t flags,
                        void* stream);

/* Bytes of the device array match_batch_noalloc works in. */
size_t cfog_noalloc_scratch_bytes(void);

/* Largest N + 2r the FFT paths support. */
int32_t cfog_max_window(void);

/* Pin the FFT side P used for template side N and radius r on this context
 * (P = 0 removes the pin).  Returns CFOG_EUNSUPPORTED if no kernel of side P
 * fits (P < N + 2r or too little on-chip scratch).  Pins take precedence over
 * the autotuner; both only change the rounding of the FFT, not the method. */
int cfog_set_plan(cfog_ctx* ctx, int32_t N, int32_t r, int32_t P);

/* FFT side P this context uses for (N, r) with m channels (pin, autotuned
 * choice, or default); 0 if unsupported. */
int32_t cfog_plan_for(cfog_ctx* ctx, int32_t N, int32_t r, int32_t m);

/* FFT side P the FFT paths use for template side N and radius r (P >= N + 2r),
 * or 0 if unsupported. */
int32_t cfog_fft_size(int32_t N, int32_t r);

/* ------------------------------------------------------ feature points
 *
 * cfog_harris_grid - block-based Harris feature points in a reference image
 * (Section IV): the image is divided into n x n cells; for cell (i, j)
 * (row-major) the chip of `chip` x `chip` pixels centred at
 * (floor((2j+1) W / 2n), floor((2i+1) H / 2n)), clipped to the image, is read,
 * and its k pixels with the largest Harris response become feature points.
 * Details the paper leaves open, as implemented: gradients by [-1, 0, 1]
 * with the chip's borders replicated; the structure tensor of the gradients
 * smoothed by a normalised Gaussian of std `sigma` (radius int(4 sigma + 0.5),
 * chip borders replicated); response R = det - kappa trace^2 (kappa = 0.04 is
 * the usual choice); ties in R go to the smaller row-major index in the chip.
 *   d_img       DEVICE [H][row_stride] fp32 image.
 *   n, k        cells per axis (>= 1) and points per chip (1..64; every chip
 *               must hold at least k pixels).
 *   chip        chip side, 1..64 (the paper uses 60).
 *   d_cps       DEVICE output [n*n*k] cfog_cp, 16-byte aligned: for cell c and
 *               rank q (decreasing R) entry c*k + q holds (x, y, x, y), i.e. a
 *               control point whose search centre defaults to the same
 *               position; (-1, -1, -1, -1) if the chip has no finite response
 *               left.
 *   d_response  nullable DEVICE output [n*n*k] fp32: R of each point.
 * Asynchronous on `stream`.  CFOG_EINVAL for bad arguments, CFOG_EUNSUPPORTED
 * for a Gaussian radius above 8.
 */
int cfog_harris_grid(cfog_ctx* ctx, const float* d_img, int32_t H, int32_t W, int64_t row_stride, int32_t n,
                     int32_t k, int32_t chip, float sigma, float kappa, cfog_cp* d_cps, float* d_response,
                     void* stream);

/* ---------------------------------------------------- outlier rejection
 *
 * cfog_reject_outliers - iterative outlier rejection of control points with a
 * cubic polynomial mapping model (Section IV): fit the model to all kept
 * points by least squares, remove the point with the largest residual, repeat
 * until the RMSE is below `threshold` pixels (Table V uses 3.5) or ten points
 * (the model's size) remain.  Readings of what the paper leaves open: source
 * coordinates normalised by the centre and half-extent of their bounding box;
 * residual = Euclidean distance between the mapped source point and its match;
 * RMSE = sqrt(mean residual^2) over the kept points; ties in the largest
 * residual go to the smaller index.  FP64 normal equations (formed once,
 * then downdated by each removed point), Cholesky solve.
 *   d_src, d_dst  DEVICE [n][2] fp32 (x, y): points in A and their matches in
 *                 B (e.g. (x + fdx, y + fdy) from match results), 8-byte aligned.
 *   n             10 .. 2^20 points; the work grows as n * (points removed).
 *   d_keep        DEVICE output [n] bytes: 1 kept, 0 removed.
 *   d_result      DEVICE output, one cfog_reject_result, 8-byte aligned.
 * Asynchronous on `stream`; CFOG_EINVAL for bad arguments.
 */
typedef struct {
  double coef[10][2];    /* x' = sum_a coef[a][0] t_a, y' = sum_a coef[a][1] t_a with
                            t = (1, u, v, u^2, u v, v^2, u^3, u^2 v, u v^2, v^3) */
  double centre[2];      /* u = (x - centre[0]) / half_extent[0], v likewise with y */
  double half_extent[2];
  double rmse;           /* of the final fit (NaN if status != 0) */
  int32_t removed, n_kept;
  int32_t status;        /* 0 ok; 1 singular or non-finite fit (coef NaN) */
  int32_t pad;
} cfog_reject_result;

int cfog_reject_outliers(cfog_ctx* ctx, const float* d_src, const float* d_dst, int32_t n, float threshold,
                         unsigned char* d_keep, cfog_reject_result* d_result, void* stream);

/* ------------------------------------------------------------- serving
 *
 * A matching server: a request loop that keeps the CFOG volumes of
 * registered image pairs resident in device memory and matches the control
 * points of requests as they arrive (the same method as match_batch).
 *
 *   - Memory: the server allocates one device region of `hbm_budget` bytes.
 *     A pair's volumes and SATs (4*m + 8 bytes per pixel of each image, plus
 *     one SAT row and column) are computed by cfog_extract on first use and
 *     stay resident; each admitted request holds a block for its CP list,
 *     results and optional surfaces (16 + 24 + 4*(2r+1)^2 bytes per CP) until
 *     it completes.
 *   - Admission: strictly in arrival order, as soon as the request's pair is
 *     resident (or room for it can be made) and its own block fits.  Making
 *     room evicts the least recently used pairs that no admitted request uses;
 *     an evicted pair is recomputed when a later request needs it.
 *   - Continuous batching: consecutive admitted requests form one batch (up to
 *     max_batch_cps control points and max_batch_reqs requests) that runs as
 *     one match_batch call on one of n_slots streams; while batches run, new
 *     arrivals are admitted into the next free slot, so their work overlaps
 *     on the device.
 *   - A request's result does not depend on what it is batched with: every
 *     control point is matched by the same kernel and FFT size as alone.
 *   - Threads: the server runs one host worker thread.  Its entry points may
 *     be called from any host thread (they are serialised internally).
 *   - Timestamps are CLOCK_MONOTONIC nanoseconds.
 */
typedef struct cfog_server cfog_server;

typedef struct {
  size_t hbm_budget;       /* bytes of device memory for volumes and request buffers */
  int32_t n_slots;         /* batches in flight at once, 1..16 (streams) */
  int32_t max_batch_cps;   /* control points per batch, >= 1 (and per request) */
  int32_t max_batch_reqs;  /* requests per batch, >= 1 */
  int32_t m;               /* orientation channels, 1..16 */
  float sigma;             /* Gaussian std of the extraction, > 0 */
  int32_t flags;           /* match_batch path: CFOG_PATH_BATCHED_FFT, _PLAIN_FFT or _MFMA_BF16,
                              optionally | CFOG_OBJ_CORR */
  size_t max_batch_surf;   /* surface values per batch (and per request) staged for the host */
} cfog_server_config;

typedef struct {
  int64_t id;              /* request id returned by cfog_server_submit */
  int32_t status;          /* CFOG_OK, or a negative code if the request failed */
  int32_t n_cps;
  int64_t t_submit_ns;     /* cfog_server_submit called */
  int64_t t_admit_ns;      /* admitted into a batch (memory granted) */
  int64_t t_launch_ns;     /* its batch enqueued on the device */
  int64_t t_done_ns;       /* results copied into the caller's buffers */
  int32_t batch_reqs;      /* requests in its batch */
  int32_t pad;
} cfog_request_info;

typedef struct {
  int64_t submitted, completed, batches, evictions, extractions, blocked;
  size_t arena_bytes, arena_used, arena_peak;
  int32_t max_in_flight;   /* most batches seen on the device at once */
  int32_t pad;
} cfog_server_stats;

/* Create a server on HIP device `device`.  cfg may be NULL for defaults
 * (budget 80% of free device memory, 4 slots, 8192 CPs and 256 requests per
 * batch, m = 9, sigma = 0.8, batched FFT path, 2^22 surface values).
 * CFOG_EINVAL for out-of-range fields, CFOG_ENOMEM if the region cannot be
 * allocated. */
int cfog_server_create(int device, const cfog_server_config* cfg, cfog_server** out);

/* Finish every submitted request, then free what the server owns.  NULL is
 * accepted. */
int cfog_server_destroy(cfog_server* srv);

/* Register an image pair: A and B are DEVICE fp32 images [h][stride] owned by
 * the caller, which must keep them unchanged while the server lives.  *pair_id
 * receives the pair's id (0, 1, ...).  Volumes are computed on first use, on
 * the server's own streams, which do not wait for any stream of the caller:
 * the writes that fill the images must have completed on the device (e.g.
 * hipStreamSynchronize of the stream that wrote them) before the first
 * cfog_server_submit naming the pair.
 * CFOG_ENOMEM if the pair alone exceeds the budget. */
int cfog_server_add_pair(cfog_server* srv, const float* d_imgA, int32_t hA, int32_t wA, int64_t strideA,
                         const float* d_imgB, int32_t hB, int32_t wB, int64_t strideB, int32_t* pair_id);

/* Submit a request: match n_cps control points (HOST array, copied before the
 * call returns) of pair `pair_id` with template side N and radius r.  Results
 * are written to the caller's HOST buffers h_out[n_cps] and, if h_surfaces is
 * not NULL, h_surfaces[n_cps][2r+1][2r+1]; both must stay valid until the
 * request is reported by cfog_server_poll.  *req_id receives the id.
 * Every point is first tested on the host against the pair's image sizes with
 * the rule the kernels use (template box of Eq. 3 inside A, search box inside
 * B, computed in 64 bits so that any int32 coordinate is safe); points outside
 * never reach the device and get the CFOG_CP_OUT_OF_BOUNDS result (NaN
 * surface).  A request with no point inside is reported at once.
 * CFOG_EINVAL for bad arguments, CFOG_EUNSUPPORTED for (N, r) the path cannot
 * match, CFOG_ENOMEM for a request that could never fit the budget or the
 * per-batch limits, CFOG_EHIP after a device failure of the server. */
int cfog_server_submit(cfog_server* srv, int32_t pair_id, const cfog_cp* h_cps, int32_t n_cps, int32_t N,
                       int32_t r, cfog_result* h_out, float* h_surfaces, int64_t* req_id);

/* Report up to `max` completed requests (each exactly once) into infos[];
 * waits up to timeout_us microseconds for the first one (0: do not wait).
 * *n_done receives the count. */
int cfog_server_poll(cfog_server* srv, cfog_request_info* infos, int32_t max, int64_t timeout_us,
                     int32_t* n_done);

/* Counters since creation. */
int cfog_server_get_stats(cfog_server* srv, cfog_server_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* CFOG_H_ */
