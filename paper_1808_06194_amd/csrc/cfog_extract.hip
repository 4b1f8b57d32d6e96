// CFOG extraction (Section III-F of Ye et al.) and the FP64 summed-area table
// of the per-pixel energy Q = sum_k D_k^2 (the energy terms of Eq. 5).
//
// Layout: image [H][row_stride] fp32; volume D [m][H][W] fp32 (planar, one
// contiguous H*W plane per orientation); SAT [(H+1)][(W+1)] fp64 with a zero
// first row and column, SAT(y+1, x+1) = sum_{y'<=y, x'<=x} Q(y', x').
//
// The volume and table writes are nontemporal stores: they stream past the
// caches, which nothing reads again before the matcher (measured on the
// extraction's write pattern alone: 10-13% faster than cached stores).
//
// Kernel 1 (cfog_extract_kernel<R, M>) produces a 64 x 32 output tile for all
// m channels:
//   A. stage the image tile plus an (R+1)-pixel halo in LDS (clamp-to-edge);
//   B. gx, gy by [-1,0,1] (the filters given after Eq. 2) at every pixel of
//      the tile + R halo, at the clamped pixel (which is what clamp-to-edge
//      Gaussian borders read), kept in registers by the thread that owns the
//      pixel for the whole channel loop;
//   C. per channel k: each thread forms g_k = |cos(theta_k) gx + sin(theta_k) gy|
//      (Eq. 2, theta_k = k pi / m) once for its pixels into the LDS channel
//      plane (channel k + 1's while the vertical pass of channel k runs);
//      the horizontal Gaussian pass reads it by 16-byte pieces (four outputs
//      per thread, consecutive lanes on consecutive columns), then the
//      vertical pass (radius R, 4 outputs per thread from a sliding window
//      down a column); the circular [1,2,1]/4 orientation smoothing is
//      applied to the spatially smoothed channels with rolling registers,
//      and each finished channel goes straight to HBM; Q accumulated in FP64
//      from the FP32 outputs;
//   D. the tile-local 2-D inclusive prefix L of Q (row scan across the 64 lanes
//      of a wave, column scan down the tile), written into the SAT buffer,
//      plus the tile's right column and bottom row into a small workspace.
// LDS holds the channel plane and one row-pass buffer (the image tile shares
// its storage; the wave carries of D reuse the dead channel plane), about
// 22 KB at R = 3; four 512-thread workgroups (32 waves) share a CU; two
// barriers per channel.  (Measured on 2048^2 images: 64 x 16 tiles of 256
// threads, eight per CU, 4% slower; with two row-pass buffers, one barrier per
// channel and six per CU, 7-8% slower.  Forming g_k from two gradient planes
// inside the horizontal pass computed each value three times.)

// Global SAT from tile-local prefixes: for a tile (i, j) with origin (y0, x0),
//   SAT(y, x) = L(y, x) + sum_{j'<j} Rc_{i,j'}(y) + sum_{i'<i} Bt_{i',j}(x)
//             + sum_{i'<i, j'<j} total(i', j')
// where Rc is a tile's right column of L and Bt its bottom row.  Kernel 2
// turns Rc into exclusive prefixes along each image row and Bt into exclusive
// prefixes along each image column; kernel 3 adds the three terms in place.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <vector>
#include "kernels.hpp"

namespace cfog {

constexpr int EX_TX = 64;
constexpr int EX_TY = 32;
constexpr int EX_NT = 512;
constexpr int EX_RUN = 4;  // outputs per thread in the sliding Gaussian passes

// One image of an extraction launch (blockIdx.z selects it).
struct ExImage {
  const float* img;
  int64_t stride;
  float* vol;
  double* sat;  // nullable
  double* rc;   // [H][ntx] right columns of the tile-local prefixes
  double* bt;   // [nty][W] bottom rows
  int H, W, ntx, nty;
};

// Images per launch: their tile grids are overlaid (the launch spans the
// largest), and the tiles outside an image's own grid exit at once.
constexpr int kExBatch = 8;

struct ExtractArgs {
  ExImage im[kExBatch];
  int m;
  int scheme;                     // 2: Eq. 2; 1: binned orientation (scheme 1)
  float cs[kMaxOrient];           // cos(theta_k)
  float sn[kMaxOrient];           // sin(theta_k)
  float w[kMaxGaussRadius + 1];   // w[|j|], j in [-R, R]
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// The value of another lane by a DPP move of both halves (lanes without a
// source, or in rows outside ROW_MASK, read 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_take(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Inclusive prefix sum over the 64 lanes of a wave (all lanes active): shifts
// by 1, 2, 4, 8 within each row of 16 lanes, then row 0's total into row 1
// and row 2's into row 3, then lane 31's into rows 2 and 3.
__device__ __forceinline__ double wave_incl_scan(double v) {
  v += dpp_take<0x111, 0xf>(v);  // row_shr:1
  v += dpp_take<0x112, 0xf>(v);  // row_shr:2
  v += dpp_take<0x114, 0xf>(v);  // row_shr:4
  v += dpp_take<0x118, 0xf>(v);  // row_shr:8
  v += dpp_take<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_take<0x143, 0xc>(v);  // row_bcast:31
  return v;
}

// D. Tile-local 2-D inclusive prefix of the per-pixel energies q (rows
// [orow, orow + EX_RUN) of column oc of a TX x TY tile at row y0; a row of the
// tile spans TX / 64 waves, EX_NT / TX row groups of EX_RUN rows stack down),
// written into the SAT buffer, plus the tile's right column (rc) and bottom
// row (bt) for the carry kernels.  qx: (EX_NT / TX) TX + EX_NT / 64 EX_RUN
// doubles of LDS.
template <int TX, int TY>
__device__ __forceinline__ void tile_sat_prefix(double (&q)[EX_RUN], double* qx, double* sat, double* rc, double* bt,
                                                int H, int W, int ntx, int y0, int orow, int oc, int gxx) {
  constexpr int NWX = TX / 64, NRG = EX_NT / TX;
  static_assert(TX % 64 == 0 && NRG * EX_RUN == TY, "tile geometry");
  const int tid = threadIdx.x, lane = tid & 63, rg = tid / TX, hx = (tid >> 6) % NWX;
#pragma unroll
  for (int o = 0; o < EX_RUN; ++o) q[o] = wave_incl_scan(q[o]);  // along x within the wave's 64 columns
  if constexpr (NWX > 1) {
    // the row totals of the waves to the left in the same row group
    double* wt = qx + NRG * TX;  // [row group][wave][row]
    if (lane == 63) {
#pragma unroll
      for (int o = 0; o < EX_RUN; ++o) wt[(rg * NWX + hx) * EX_RUN + o] = q[o];
    }
    __syncthreads();
    for (int h = 0; h < hx; ++h) {
#pragma unroll
      for (int o = 0; o < EX_RUN; ++o) q[o] += wt[(rg * NWX + h) * EX_RUN + o];
    }
  }
#pragma unroll
  for (int o = 1; o < EX_RUN; ++o) q[o] += q[o - 1];              // along y within the thread
  qx[rg * TX + oc] = q[EX_RUN - 1];
  __syncthreads();
  double up = 0.0;
  for (int i = 0; i < rg; ++i) up += qx[i * TX + oc];
  const int W1 = W + 1;
#pragma unroll
  for (int o = 0; o < EX_RUN; ++o) {
    q[o] += up;
    const int gyy = y0 + orow + o;
    if (gyy < H && gxx < W) __builtin_nontemporal_store(q[o], sat + (size_t)(gyy + 1) * W1 + gxx + 1);
    if (oc == TX - 1 && gyy < H) rc[(size_t)gyy * ntx + blockIdx.x] = q[o];
  }
  if (rg == NRG - 1 && gxx < W) bt[(size_t)blockIdx.y * W + gxx] = q[EX_RUN - 1];
}

// The CFOG tile: 128 x 16 outputs, so that each row of a channel plane is
// written 512 contiguous bytes at a time (measured on the extraction's write
// pattern: 13-18% faster than 64 x 32 tiles, whose rows are 256 bytes).
constexpr int CF_TX = 128;
constexpr int CF_TY = 16;

// LDS geometry of the CFOG tile for Gaussian radius R.
template <int R>
struct ExTile {
  static constexpr int TX = CF_TX, TY = CF_TY;
  static constexpr int IW = TX + 2 * R + 2, IH = TY + 2 * R + 2;  // image tile (+1 for the gradient)
  static constexpr int GW = TX + 2 * R, GH = TY + 2 * R;          // gradient / channel tile
  static constexpr int NQ = (4 + 2 * R + 3) / 4;  // 16-byte reads per 4 horizontal outputs
  // channel row stride: a multiple of 4 floats covering the last quad's reads
  static constexpr int GWP = ((GW + 3) / 4 * 4) > (TX - 4 + 4 * NQ) ? ((GW + 3) / 4 * 4) : (TX - 4 + 4 * NQ);
  static constexpr int QPR = TX / 4;              // horizontal outputs four at a time, per row
  static constexpr int NQUAD = GH * QPR;
  static constexpr size_t IMG = ((size_t)IH * IW + 3) / 4 * 4;   // floats
  static constexpr size_t GP = (size_t)GH * GWP;                 // floats of the channel plane
  static constexpr size_t HB = (size_t)GH * TX;                   // floats: one channel's row pass
  // the spatially smoothed channels 0 and 1 of a thread's 4 outputs, needed
  // again by the circular orientation smoothing after the last channel
  static constexpr size_t KEEP = 2 * EX_RUN * EX_NT;  // floats, [value][thread]
  // LDS: [channel plane | KEEP] then HB; the image tile shares the first
  // region (it is dead once the gradients are in registers)
  static constexpr size_t A = (GP + KEEP) > IMG ? (GP + KEEP) : IMG;
  static constexpr size_t BYTES = 4 * (A + HB);
  // halo-tile pixels of a thread: thread t takes column t % TX of the rows
  // t / TX + RPP i (NROW of them), and the 2R columns right of the first TX
  // are spread over the threads (NEXTRA each)
  static constexpr int RPP = EX_NT / TX;
  static constexpr int NROW = (GH + RPP - 1) / RPP;
  static constexpr int NX = 2 * R;
  // where the last row slot is past the tile for some threads (GH not a
  // multiple of RPP), those threads take the extra columns in it if they fit
  static constexpr int LASTR = GH % RPP;  // threads with tid / TX >= LASTR have no row in the last slot
  static constexpr bool FOLD = LASTR != 0 && (RPP - LASTR) * TX >= NX * GH;
  static constexpr int NEXTRA = FOLD ? 0 : (NX * GH + EX_NT - 1) / EX_NT;
  static constexpr int NPX = NROW + NEXTRA;
  static_assert((EX_NT / TX) * EX_RUN == TY, "one EX_RUN-row piece of the tile per thread");
};

// M > 0: the channel count fixed at compile time (the channel loop unrolls
// and the orientation smoothing's register rotation disappears); M = 0 reads
// it from the arguments.  S1: scheme 1 instead of Eq. 2, fixed at compile
// time so that the per-pixel channel value carries no branch.
template <int R, int M, bool S1>
__global__ __launch_bounds__(EX_NT) __attribute__((amdgpu_waves_per_eu(M > 0 ? 8 : 1, 8))) void cfog_extract_kernel(ExtractArgs a) {
  using T = ExTile<R>;
  constexpr int TX = T::TX, TY = T::TY;
  constexpr int IW = T::IW, IH = T::IH, GW = T::GW, GH = T::GH, GWP = T::GWP;
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  const int m = M > 0 ? M : a.m;
  float* gk = lds;                                   // GH * GWP: one oriented-gradient channel
  float* keep = gk + T::GP;                          // KEEP: Gs_0, Gs_1 of this thread's outputs
  float* img = lds;                                  // IH * IW, read only by the gradient pass
  float* Hb = lds + T::A;                            // GH * TX row-pass outputs
  double* qx = reinterpret_cast<double*>(gk);        // the tile prefix's carries, after the last channel
  static_assert(T::GP * sizeof(float) >= ((EX_NT / TX) * TX + (EX_NT / 64) * EX_RUN) * sizeof(double),
                "tile prefix carries");
  const ExImage I = a.im[blockIdx.z];
  if ((int)blockIdx.x >= I.ntx || (int)blockIdx.y >= I.nty) return;  // beyond this image's tiles
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int H = I.H, W = I.W;
  float w[R + 1];
#pragma unroll
  for (int j = 0; j <= R; ++j) w[j] = a.w[j];

  // A. image tile, rows y0-R-1 .. y0+TY+R, clamped; all loads issued before
  // the LDS stores so their latencies overlap.  Ordinary (cached) loads: the
  // tile below is dispatched to the same XCD whenever the tile grid is a
  // multiple of 8 tiles wide, and reads these halo rows again from its L2.
  {
    constexpr int NIT = (IH * IW + EX_NT - 1) / EX_NT;
    float v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int i = tid + it * EX_NT;
      if (i < IH * IW) {
        const int r = i / IW, c = i - r * IW;
        const int gy = clampi(y0 - R - 1 + r, 0, H - 1), gx = clampi(x0 - R - 1 + c, 0, W - 1);
        v[it] = I.img[(int64_t)gy * I.stride + gx];
      }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int i = tid + it * EX_NT;
      if (i < IH * IW) img[i] = v[it];
    }
  }
  __syncthreads();

  // B. gradients of the halo tile.  Interior tiles read their neighbours
  // directly; tiles at the border take them at clamped positions, which is
  // what clamp-to-edge gradient and Gaussian borders read.
  const bool interior = x0 - R - 1 >= 0 && y0 - R - 1 >= 0 && x0 + TX + R <= W - 1 && y0 + TY + R <= H - 1;
  const int oy = y0 - R - 1, ox = x0 - R - 1;  // global coords of img[0][0]
  auto grad = [&](int r, int c) {              // (gx, gy) at halo-tile pixel (r, c)
    if (interior) {
      const float* p = img + (r + 1) * IW + c + 1;
      return make_float2(p[1] - p[-1], p[IW] - p[-IW]);
    }
    const int Yc = clampi(y0 - R + r, 0, H - 1), Xc = clampi(x0 - R + c, 0, W - 1);
    const int yl = Yc - oy, xl = Xc - ox;
    const int xp = clampi(Xc + 1, 0, W - 1) - ox, xm = clampi(Xc - 1, 0, W - 1) - ox;
    const int yp = clampi(Yc + 1, 0, H - 1) - oy, ym = clampi(Yc - 1, 0, H - 1) - oy;
    return make_float2(img[yl * IW + xp] - img[yl * IW + xm], img[yp * IW + xl] - img[ym * IW + xl]);
  };
  // this thread's pixels (the mapping of ExTile): row slots at column
  // tid % TX of the rows tid / TX + RPP it (rows beyond the tile are skipped,
  // uniformly per wave), extra slots in the columns right of the first TX
  const int pc = tid % TX, pr = tid / TX;
  // folded extra pixel of this thread (in its last row slot), if any
  const int fe = tid - T::LASTR * TX;
  const bool fold_px = T::FOLD && pr >= T::LASTR && fe < T::NX * GH;
  float2 gb[T::NPX];  // this thread's pixels, held through the channel loop
#pragma unroll
  for (int it = 0; it < T::NROW; ++it) {
    const int r = pr + it * T::RPP;
    if (T::FOLD && it == T::NROW - 1 && pr >= T::LASTR) {
      const int fr = fe / T::NX;
      gb[it] = fold_px ? grad(fr, TX + (fe - fr * T::NX)) : make_float2(0.f, 0.f);
    } else {
      gb[it] = r < GH ? grad(r, pc) : make_float2(0.f, 0.f);
    }
  }
#pragma unroll
  for (int e = 0; e < T::NEXTRA; ++e) {
    const int t = tid + e * EX_NT;
    const int r = t / T::NX, c = TX + (t - r * T::NX);
    gb[T::NROW + e] = t < T::NX * GH ? grad(r, c) : make_float2(0.f, 0.f);
  }
  // scheme 1 keeps (|g|, orientation bin position in [0, m)) instead of (gx, gy)
  if constexpr (S1) {
    const float bscale = (float)m / 3.14159265358979f;
#pragma unroll
    for (int it = 0; it < T::NPX; ++it) {
      const float2 g = gb[it];
      float phi = atan2f(g.y, g.x);
      if (phi < 0.f) phi += 3.14159265358979f;
      float b = phi * bscale;
      if (b >= (float)m) b -= (float)m;
      gb[it] = make_float2(sqrtf(g.x * g.x + g.y * g.y), b);
    }
  }
  // the padding columns of the channel plane feed only channel values that
  // no output reads
  const float mf = (float)m;
  // oriented gradient g_k of one pixel from its two gradient values:
  // |cos(theta_k) gx + sin(theta_k) gy| (Eq. 2), or for scheme 1
  // |g| max(0, 1 - circular distance of the bin position to k)
  auto form_channel = [&](int k) {
    const float ck = a.cs[k], sk = a.sn[k], kf = (float)k;
    auto g_of = [&](float2 uv) {
      if constexpr (S1) {
        const float d = fabsf(uv.y - kf);
        return uv.x * fmaxf(0.f, 1.f - fminf(d, mf - d));
      } else {
        return fabsf(fmaf(ck, uv.x, sk * uv.y));
      }
    };
#pragma unroll
    for (int it = 0; it < T::NROW; ++it) {
      if (T::FOLD && it == T::NROW - 1 && pr >= T::LASTR) {
        const int fr = fe / T::NX;
        if (fold_px) gk[fr * GWP + TX + (fe - fr * T::NX)] = g_of(gb[it]);
      } else if (pr + it * T::RPP < GH) {
        gk[(pr + it * T::RPP) * GWP + pc] = g_of(gb[it]);
      }
    }
#pragma unroll
    for (int e = 0; e < T::NEXTRA; ++e) {
      const int t = tid + e * EX_NT;
      const int r = t / T::NX;
      if (t < T::NX * GH) gk[r * GWP + TX + (t - r * T::NX)] = g_of(gb[T::NROW + e]);
    }
  };
  __syncthreads();  // every read of the image tile is done: the channel plane shares its storage
  form_channel(0);
  __syncthreads();

  // C. per channel: the horizontal Gaussian of the oriented gradient (the
  // channel values computed on the fly from the gradient planes), then the
  // vertical pass, which leaves the spatially smoothed channel Gs_k for the
  // rows [4 (tid/64), +4) of column tid % 64 in registers.  A barrier after
  // each pass: the next channel's row pass rewrites the buffer.
  const int oc = tid % TX, orow = (tid / TX) * EX_RUN;
  const int gxx = x0 + oc;
  double q[EX_RUN];
  float pm2[EX_RUN], pm1[EX_RUN];
#pragma unroll
  for (int p = 0; p < EX_RUN; ++p) { q[p] = 0.0; pm2[p] = pm1[p] = 0.f; }
  const size_t plane = (size_t)H * W;
  float* const vout = I.vol + (size_t)min(y0 + orow, H - 1) * W + min(gxx, W - 1);
  bool vok[EX_RUN];
#pragma unroll
  for (int o = 0; o < EX_RUN; ++o) vok[o] = y0 + orow + o < H && gxx < W;
  auto emit = [&](int k, const float (&d)[EX_RUN]) {
    float* p = vout + k * plane;
#pragma unroll
    for (int o = 0; o < EX_RUN; ++o) {
      if (vok[o]) {
        __builtin_nontemporal_store(d[o], p + (size_t)o * W);
        q[o] = fma((double)d[o], (double)d[o], q[o]);
      }
    }
  };
  auto channel = [&](int k) {
    float* hb = Hb;
    // horizontal pass: each thread four consecutive outputs of one row from
    // 16-byte reads of the channel plane (QPR threads cover a row)
#pragma unroll
    for (int it = 0; it < (T::NQUAD + EX_NT - 1) / EX_NT; ++it) {
      const int qd = tid + it * EX_NT;
      if (T::NQUAD % EX_NT == 0 || qd < T::NQUAD) {
        const int r = qd / T::QPR, c4 = (qd - r * T::QPR) * 4;
        const float4* sx = reinterpret_cast<const float4*>(gk + r * GWP + c4);
        float x[4 * T::NQ];
#pragma unroll
        for (int u = 0; u < T::NQ; ++u) {
          const float4 vx = sx[u];
          x[4 * u] = vx.x;
          x[4 * u + 1] = vx.y;
          x[4 * u + 2] = vx.z;
          x[4 * u + 3] = vx.w;
        }
        float o4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float s = w[0] * x[j + R];
#pragma unroll
          for (int t = 1; t <= R; ++t) s = fmaf(w[t], x[j + R - t] + x[j + R + t], s);
          o4[j] = s;
        }
        *reinterpret_cast<float4*>(hb + r * TX + c4) = make_float4(o4[0], o4[1], o4[2], o4[3]);
      }
    }
    __syncthreads();
    float cur[EX_RUN];
    {
      const float* col = hb + orow * TX + oc;  // col[t*TX] = row orow - R + t
      float v[EX_RUN + 2 * R];
#pragma unroll
      for (int t = 0; t < EX_RUN + 2 * R; ++t) v[t] = col[t * TX];
#pragma unroll
      for (int o = 0; o < EX_RUN; ++o) {
        float s = w[0] * v[o + R];
#pragma unroll
        for (int j = 1; j <= R; ++j) s = fmaf(w[j], v[o + R - j] + v[o + R + j], s);
        cur[o] = s;
      }
    }
  // circular [1,2,1]/4 along orientation: D_{k-1} = Gs_{k-2}/4 + Gs_{k-1}/2 + Gs_k/4
    if (k < 2) {
      // kept in this thread's LDS slots (registers are the occupancy limit)
#pragma unroll
      for (int o = 0; o < EX_RUN; ++o) keep[(k * EX_RUN + o) * EX_NT + tid] = cur[o];
    } else {
      float d[EX_RUN];
#pragma unroll
      for (int o = 0; o < EX_RUN; ++o) d[o] = fmaf(0.25f, pm2[o] + cur[o], 0.5f * pm1[o]);
      emit(k - 1, d);
    }
#pragma unroll
    for (int o = 0; o < EX_RUN; ++o) { pm2[o] = pm1[o]; pm1[o] = cur[o]; }
    // the next channel's values: the channel plane was last read by this
    // channel's row pass, which the barrier above has closed
    if (k + 1 < m) form_channel(k + 1);
    __syncthreads();  // every read of Hb is done and the next channel is formed
  };
  if constexpr (M > 0) {
#pragma unroll
    for (int k = 0; k < M; ++k) channel(k);
  } else {
    for (int k = 0; k < m; ++k) channel(k);
  }
  {
    float d[EX_RUN], g0[EX_RUN], g1[EX_RUN];
#pragma unroll
    for (int o = 0; o < EX_RUN; ++o) {
      g0[o] = keep[o * EX_NT + tid];
      g1[o] = m > 1 ? keep[(EX_RUN + o) * EX_NT + tid] : 0.f;
    }
    if (m == 1) {
      emit(0, g0);
    } else {
      // D_{m-1} = Gs_{m-2}/4 + Gs_{m-1}/2 + Gs_0/4 ;  D_0 = Gs_{m-1}/4 + Gs_0/2 + Gs_1/4
#pragma unroll
      for (int o = 0; o < EX_RUN; ++o) d[o] = fmaf(0.25f, pm2[o] + g0[o], 0.5f * pm1[o]);
      emit(m - 1, d);
#pragma unroll
      for (int o = 0; o < EX_RUN; ++o) d[o] = fmaf(0.25f, pm1[o] + g1[o], 0.5f * g0[o]);
      emit(0, d);
    }
  }
  if (!I.sat) return;
  tile_sat_prefix<TX, TY>(q, qx, I.sat, I.rc, I.bt, H, W, I.ntx, y0, orow, oc, gxx);
}

// ------------------------------------------------ pixel-wise HOG (FHOG)
// Section III-C: at every pixel, the histogram of a block of 2 x 2 cells of
// C pixels centred on it over 9 unsigned orientation bins (centres k pi / 9,
// linear split between the two nearest bins), each gradient spread over the
// cells with bilinear weights max(0, 1 - |d - o| / C) for cell centres
// o = -C/2, +C/2 at block offsets d in [-C, C] (clamp-to-edge borders), the
// 36 values normalised by sqrt(|v|^2 + 1e-12).  Channel (2 a + b) 9 + k is
// cell column a, cell row b, bin k.  Same tiles as the CFOG kernel: per bin,
// the bin's channel on the halo tile, both horizontal cell passes, both
// vertical cell passes into registers (9 x 4 values for each of the 4 pixels
// of a thread) until the norm is known; then the normalised values go out
// and their energies feed the tile-local SAT prefix.
constexpr int FH_BINS = 9;
constexpr int FH_MAX_CELL = 8;

struct FhogArgs {
  const float* img;
  int64_t stride;
  int H, W;
  float* vol;
  double* sat;  // nullable
  double* rc;
  double* bt;
  int ntx, nty;
};

template <int C>
struct FhTile {
  static constexpr int IW = EX_TX + 2 * C + 2, IH = EX_TY + 2 * C + 2;  // image tile (+1 for the gradient)
  static constexpr int GW = EX_TX + 2 * C, GH = EX_TY + 2 * C;          // gradient / channel tile
  static constexpr size_t IMG = ((size_t)IH * IW + 3) / 4 * 4;          // floats (keeps G 16-byte aligned)
  static constexpr size_t MB = (size_t)GH * GW;                         // float2 (|g|, bin position)
  static constexpr int NQ = (4 + 2 * C + 3) / 4;  // 16-byte reads per 4 horizontal outputs
  // channel row stride: a multiple of 4 floats covering the last quad's reads
  static constexpr int GWP = ((GW + 3) / 4 * 4) > (EX_TX - 4 + 4 * NQ) ? ((GW + 3) / 4 * 4) : (EX_TX - 4 + 4 * NQ);
  static constexpr int NQUAD = GH * EX_TX / 4;  // horizontal outputs four at a time
  static constexpr size_t G = (size_t)GH * GWP;                         // floats
  static constexpr size_t HX = 2 * (size_t)GH * EX_TX;                  // floats: both horizontal passes
  static constexpr size_t BYTES = 4 * IMG + 8 * MB + 4 * G + 4 * HX + 8 * (EX_NT / 64) * 64;
};

// Bilinear weight of block offset d for cell a (centre offset (a - 1/2) C).
template <int C>
__device__ __forceinline__ float fh_w(int d, int a) {
  const float o = (a == 0 ? -0.5f : 0.5f) * (float)C;
  return fmaxf(0.f, 1.f - fabsf((float)d - o) / (float)C);
}

template <int C>
__global__ __launch_bounds__(EX_NT) void fhog_kernel(FhogArgs a) {
  using T = FhTile<C>;
  constexpr int IW = T::IW, IH = T::IH, GW = T::GW, GH = T::GH;
  extern __shared__ float4 lds4[];
  float* img = reinterpret_cast<float*>(lds4);
  float2* mb = reinterpret_cast<float2*>(img + T::IMG);
  float* G = reinterpret_cast<float*>(mb + T::MB);
  float* hx = G + T::G;
  double* qx = reinterpret_cast<double*>(hx + T::HX);
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * EX_TX, y0 = blockIdx.y * EX_TY;
  const int H = a.H, W = a.W;

  // A. image tile, rows y0-C-1 .. y0+TY+C, clamped
  for (int i = tid; i < IH * IW; i += EX_NT) {
    const int r = i / IW, c = i - r * IW;
    const int gy = clampi(y0 - C - 1 + r, 0, H - 1), gx = clampi(x0 - C - 1 + c, 0, W - 1);
    img[i] = a.img[(int64_t)gy * a.stride + gx];
  }
  __syncthreads();
  // B. (|g|, orientation bin position) at the clamped positions of the halo tile
  {
    const int oy = y0 - C - 1, ox = x0 - C - 1;
    const float bscale = (float)FH_BINS / 3.14159265358979f;
    for (int i = tid; i < GH * GW; i += EX_NT) {
      const int r = i / GW, c = i - r * GW;
      const int Yc = clampi(y0 - C + r, 0, H - 1), Xc = clampi(x0 - C + c, 0, W - 1);
      const int yl = Yc - oy, xl = Xc - ox;
      const int xp = clampi(Xc + 1, 0, W - 1) - ox, xm = clampi(Xc - 1, 0, W - 1) - ox;
      const int yp = clampi(Yc + 1, 0, H - 1) - oy, ym = clampi(Yc - 1, 0, H - 1) - oy;
      const float gx = img[yl * IW + xp] - img[yl * IW + xm], gy = img[yp * IW + xl] - img[ym * IW + xl];
      float phi = atan2f(gy, gx);
      if (phi < 0.f) phi += 3.14159265358979f;
      float b = phi * bscale;
      if (b >= (float)FH_BINS) b -= (float)FH_BINS;
      mb[i] = make_float2(sqrtf(gx * gx + gy * gy), b);
    }
  }
  __syncthreads();

  // C. per bin: channel, horizontal cell passes, vertical cell passes
  const int oc = tid & 63, orow = (tid >> 6) * EX_RUN;
  const int gxx = x0 + oc;
  float v[FH_BINS][4][EX_RUN];
  float n2[EX_RUN];
#pragma unroll
  for (int o = 0; o < EX_RUN; ++o) n2[o] = 0.f;
#pragma unroll
  for (int k = 0; k < FH_BINS; ++k) {
    for (int i = tid; i < GH * GW; i += EX_NT) {
      const int r = i / GW, c = i - r * GW;
      const float2 g = mb[i];
      const float d = fabsf(g.y - (float)k);
      G[r * T::GWP + c] = g.x * fmaxf(0.f, 1.f - fminf(d, (float)FH_BINS - d));
    }
    __syncthreads();
    // both horizontal cell passes, four consecutive outputs per thread from
    // 16-byte reads (16 threads cover a row); the padding columns of G feed
    // no output
#pragma unroll
    for (int it = 0; it < (T::NQUAD + EX_NT - 1) / EX_NT; ++it) {
      const int qd = tid + it * EX_NT;
      if (T::NQUAD % EX_NT == 0 || qd < T::NQUAD) {
        const int r = qd >> 4, c4 = (qd & 15) * 4;
        const float4* src = reinterpret_cast<const float4*>(G + r * T::GWP + c4);
        float x[4 * T::NQ];
#pragma unroll
        for (int u = 0; u < T::NQ; ++u) {
          const float4 t = src[u];
          x[4 * u] = t.x;
          x[4 * u + 1] = t.y;
          x[4 * u + 2] = t.z;
          x[4 * u + 3] = t.w;
        }
        float o0[4], o1[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float s0 = 0.f, s1 = 0.f;
#pragma unroll
          for (int d = -C; d <= C; ++d) {
            s0 = fmaf(fh_w<C>(d, 0), x[j + C + d], s0);
            s1 = fmaf(fh_w<C>(d, 1), x[j + C + d], s1);
          }
          o0[j] = s0;
          o1[j] = s1;
        }
        *reinterpret_cast<float4*>(hx + r * EX_TX + c4) = make_float4(o0[0], o0[1], o0[2], o0[3]);
        *reinterpret_cast<float4*>(hx + GH * EX_TX + r * EX_TX + c4) = make_float4(o1[0], o1[1], o1[2], o1[3]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int ca = 0; ca < 2; ++ca) {
      const float* col = hx + ca * GH * EX_TX + (orow + C) * EX_TX + oc;  // col[t * TX] = output row orow + t
#pragma unroll
      for (int o = 0; o < EX_RUN; ++o) {
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int d = -C; d <= C; ++d) {
          const float x = col[(o + d) * EX_TX];
          s0 = fmaf(fh_w<C>(d, 0), x, s0);
          s1 = fmaf(fh_w<C>(d, 1), x, s1);
        }
        v[k][2 * ca][o] = s0;
        v[k][2 * ca + 1][o] = s1;
        n2[o] = fmaf(s0, s0, fmaf(s1, s1, n2[o]));
      }
    }
    // the next bin's channel pass writes G, which no thread still reads; its
    // barrier precedes the next writes of hx
  }

  // D. normalise, write the 36 channels, energies -> tile-local SAT prefix
  const size_t plane = (size_t)H * W;
  float* const vout = a.vol + (size_t)min(y0 + orow, H - 1) * W + min(gxx, W - 1);
  double q[EX_RUN];
#pragma unroll
  for (int o = 0; o < EX_RUN; ++o) {
    q[o] = 0.0;
    const bool ok = y0 + orow + o < H && gxx < W;
    const float inv = 1.0f / sqrtf(n2[o] + 1e-12f);
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll
      for (int k = 0; k < FH_BINS; ++k) {
        const float val = v[k][c4][o] * inv;
        if (ok) {
          __builtin_nontemporal_store(val, vout + (size_t)(c4 * FH_BINS + k) * plane + (size_t)o * W);
          q[o] = fma((double)val, (double)val, q[o]);
        }
      }
  }
  if (!a.sat) return;
  tile_sat_prefix<EX_TX, EX_TY>(q, qx, a.sat, a.rc, a.bt, H, W, a.ntx, y0, orow, oc, gxx);
}

// Kernel 2: exclusive prefixes of the right columns along each image row (one
// wave per row, lanes across tiles) and of the bottom rows along each image
// column (64 columns per workgroup, lanes across columns, the tile rows split
// between the 16 waves: each wave sums its rows, the partial sums are
// exchanged in LDS, then each wave writes its exclusive prefixes).  A wave's
// first 8 tile rows stay in registers between the two steps, which at up to
// 128 tile rows is all of them: one round of loads, one of stores.
constexpr int SAT_NT = 1024;
constexpr int SAT_WAVES = SAT_NT / 64;
constexpr int SAT_CH = 8;

// The SAT carries and fix-up of up to kExBatch images per launch (the last
// grid dimension selects the image; images without a SAT are skipped).
struct SatImage {
  double* sat;
  double* rc;
  double* bt;
  int H, W, ntx, nty;
};
struct SatBatch {
  SatImage im[kExBatch];
};

__device__ __forceinline__ double wave_excl_scan(double v, double& total) {
  const double inc = wave_incl_scan(v);
  total = __shfl(inc, 63, 64);
  return inc - v;
}

__global__ __launch_bounds__(SAT_NT) void sat_carry_kernel(SatBatch b) {
  const SatImage I = b.im[blockIdx.y];
  double* const rc = I.rc;
  double* const bt = I.bt;
  const int H = I.H, W = I.W, ntx = I.ntx, nty = I.nty;
  const int row_blocks = (H + SAT_WAVES - 1) / SAT_WAVES;
  if (!I.sat || (int)blockIdx.x >= row_blocks + (W + 63) / 64) return;  // beyond this image's blocks
  if ((int)blockIdx.x < row_blocks) {
    const int y = blockIdx.x * SAT_WAVES + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (y >= H) return;
    double* p = rc + (size_t)y * ntx;
    double carry = 0.0;
    for (int base = 0; base < ntx; base += 64) {
      const int j = base + lane;
      const double v = j < ntx ? p[j] : 0.0;
      double tot;
      const double ex = wave_excl_scan(v, tot);
      if (j < ntx) p[j] = ex + carry;
      carry += tot;
    }
    return;
  }
  __shared__ double part[SAT_WAVES][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = (blockIdx.x - row_blocks) * 64 + lane;
  const int per = (nty + SAT_WAVES - 1) / SAT_WAVES;
  const int i0 = wv * per, i1 = min(nty, i0 + per);
  const bool xok = x < W;
  double first[SAT_CH];
#pragma unroll
  for (int u = 0; u < SAT_CH; ++u) first[u] = (xok && i0 + u < i1) ? bt[(size_t)(i0 + u) * W + x] : 0.0;
  double sum = 0.0;
#pragma unroll
  for (int u = 0; u < SAT_CH; ++u) sum += first[u];
  if (xok) {
    for (int i = i0 + SAT_CH; i < i1; i += SAT_CH) {
      double v[SAT_CH];
#pragma unroll
      for (int u = 0; u < SAT_CH; ++u) v[u] = (i + u < i1) ? bt[(size_t)(i + u) * W + x] : 0.0;
#pragma unroll
      for (int u = 0; u < SAT_CH; ++u) sum += v[u];
    }
  }
  part[wv][lane] = sum;
  __syncthreads();
  if (!xok) return;
  double run = 0.0;
  for (int k = 0; k < wv; ++k) run += part[k][lane];
#pragma unroll
  for (int u = 0; u < SAT_CH; ++u) {
    if (i0 + u < i1) bt[(size_t)(i0 + u) * W + x] = run;
    run += first[u];
  }
  for (int i = i0 + SAT_CH; i < i1; i += SAT_CH) {
    double v[SAT_CH];
#pragma unroll
    for (int u = 0; u < SAT_CH; ++u) v[u] = (i + u < i1) ? bt[(size_t)(i + u) * W + x] : 0.0;
#pragma unroll
    for (int u = 0; u < SAT_CH; ++u) {
      if (i + u < i1) bt[(size_t)(i + u) * W + x] = run;
      run += v[u];
    }
  }
}

// Kernel 3: SAT = L + row carry + column carry + corner, in place; zero row 0
// and column 0.  One workgroup per TX x TY extraction tile, one thread per
// pixel column of a row group of EX_RUN rows (TX and TY as in the extraction
// kernel that wrote the tile-local prefixes).  The tile's values and carries
// are loaded first, so their latency overlaps the corner's reduction.
template <int TX, int TY>
__global__ __launch_bounds__(EX_NT) void sat_fix_kernel(SatBatch b) {
  static_assert((EX_NT / TX) * EX_RUN == TY, "tile geometry");
  __shared__ double corner_part[EX_NT / 64];
  const SatImage I = b.im[blockIdx.z];
  if (!I.sat || (int)blockIdx.x >= I.ntx || (int)blockIdx.y >= I.nty) return;  // beyond this image's tiles
  double* const sat = I.sat;
  const double* const rc = I.rc;
  const double* const bt = I.bt;
  const int H = I.H, W = I.W, ntx = I.ntx;
  const int tid = threadIdx.x, oc = tid % TX, rg = tid / TX, wv = tid >> 6;
  const int tx = blockIdx.x, ty = blockIdx.y;
  const int x0 = tx * TX, y0 = ty * TY;
  const int W1 = W + 1;
  const int gxx = x0 + oc;
  double* const p0 = sat + (size_t)(y0 + rg * EX_RUN + 1) * W1 + gxx + 1;
  bool ok[EX_RUN];
  double l[EX_RUN], r[EX_RUN];
  const double colc = gxx < W ? bt[(size_t)ty * W + gxx] : 0.0;
#pragma unroll
  for (int o = 0; o < EX_RUN; ++o) {
    const int gyy = y0 + rg * EX_RUN + o;
    ok[o] = gxx < W && gyy < H;
    l[o] = ok[o] ? p0[(size_t)o * W1] : 0.0;
    r[o] = ok[o] ? rc[(size_t)gyy * ntx + tx] : 0.0;
  }
  // corner = sum_{j' < tx} (column prefix of bottom rows at the last column of tile j')
  double cpart = 0.0;
  for (int j = tid; j < tx; j += EX_NT) {
    const int xl = min(W, (j + 1) * TX) - 1;
    cpart += bt[(size_t)ty * W + xl];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cpart += __shfl_xor(cpart, o, 64);
  if ((tid & 63) == 0) corner_part[wv] = cpart;
  __syncthreads();
  double corner = 0.0;
#pragma unroll
  for (int k = 0; k < EX_NT / 64; ++k) corner += corner_part[k];
#pragma unroll
  for (int o = 0; o < EX_RUN; ++o)
    if (ok[o]) __builtin_nontemporal_store(l[o] + r[o] + colc + corner, p0 + (size_t)o * W1);
  if (ty == 0) {
    for (int x = x0 + tid; x < min(W + 1, x0 + TX + 1); x += EX_NT) sat[x] = 0.0;
  }
  if (tx == 0) {
    for (int y = y0 + tid; y < min(H + 1, y0 + TY + 1); y += EX_NT) sat[(size_t)y * W1] = 0.0;
  }
}

static size_t lds_bytes(int m, int R) {
  (void)m;
  switch (R) {
    case 0: return ExTile<0>::BYTES;
    case 1: return ExTile<1>::BYTES;
    case 2: return ExTile<2>::BYTES;
    case 3: return ExTile<3>::BYTES;
    case 4: return ExTile<4>::BYTES;
    case 5: return ExTile<5>::BYTES;
    case 6: return ExTile<6>::BYTES;
    case 7: return ExTile<7>::BYTES;
    case 8: return ExTile<8>::BYTES;
    default: return (size_t)-1;
  }
}

size_t extract_lds_bytes(int m, int R) { return lds_bytes(m, R); }

// The carries of a TX x TY tiling: right columns [H][ntx], bottom rows [nty][W].
static size_t carry_bytes(int H, int W, int TX, int TY) {
  const size_t ntx = (W + TX - 1) / TX, nty = (H + TY - 1) / TY;
  return sizeof(double) * ((size_t)H * ntx + nty * (size_t)W);
}

// Enough for the CFOG tiling and the pixel-wise HOG tiling.
size_t extract_workspace_bytes(int H, int W) {
  return std::max(carry_bytes(H, W, CF_TX, CF_TY), carry_bytes(H, W, EX_TX, EX_TY));
}

template <int R, bool S1>
static int launch_rs(const ExtractArgs& a, dim3 grid, hipStream_t st) {
  const size_t lds = lds_bytes(a.m, R);
  if constexpr (R == 3) {
    if (a.m == 9) {  // the paper's parameters (sigma 0.8, nine orientations)
      hipLaunchKernelGGL((cfog_extract_kernel<R, 9, S1>), grid, dim3(EX_NT), lds, st, a);
      return hipGetLastError() == hipSuccess ? 0 : -2;
    }
  }
  hipLaunchKernelGGL((cfog_extract_kernel<R, 0, S1>), grid, dim3(EX_NT), lds, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <int R>
static int launch_r(const ExtractArgs& a, dim3 grid, hipStream_t st) {
  return a.scheme == 1 ? launch_rs<R, true>(a, grid, st) : launch_rs<R, false>(a, grid, st);
}

template <int R, bool S1>
static int set_attr_s() {
  if (hipFuncSetAttribute((const void*)cfog_extract_kernel<R, 0, S1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kMaxLds) != hipSuccess)
    return -2;
  if constexpr (R == 3) {
    if (hipFuncSetAttribute((const void*)cfog_extract_kernel<R, 9, S1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kMaxLds) != hipSuccess)
      return -2;
  }
  return 0;
}

template <int R>
static int set_attr() {
  return set_attr_s<R, false>() != 0 || set_attr_s<R, true>() != 0 ? -2 : 0;
}

template <int C>
static int set_fh_attr() {
  return hipFuncSetAttribute((const void*)fhog_kernel<C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)FhTile<C>::BYTES) == hipSuccess
             ? 0
             : -2;
}

int init_extract_attributes() {
  if (set_fh_attr<1>() || set_fh_attr<2>() || set_fh_attr<3>() || set_fh_attr<4>() || set_fh_attr<5>() ||
      set_fh_attr<6>() || set_fh_attr<7>() || set_fh_attr<8>())
    return -2;
  if (set_attr<0>() || set_attr<1>() || set_attr<2>() || set_attr<3>() || set_attr<4>() || set_attr<5>() ||
      set_attr<6>() || set_attr<7>() || set_attr<8>())
    return -2;
  return 0;
}

// The SAT carries and fix-up of the images of one launch (tiles of TX x TY).
template <int TX, int TY>
static int launch_sat(const SatBatch& b, int n, hipStream_t st) {
  int carry_blocks = 0, ntx = 0, nty = 0;
  for (int i = 0; i < n; ++i) {
    const SatImage& I = b.im[i];
    if (!I.sat) continue;
    carry_blocks = std::max(carry_blocks, (I.H + SAT_WAVES - 1) / SAT_WAVES + (I.W + 63) / 64);
    ntx = std::max(ntx, I.ntx);
    nty = std::max(nty, I.nty);
  }
  if (!carry_blocks) return 0;
  hipLaunchKernelGGL(sat_carry_kernel, dim3(carry_blocks, n), dim3(SAT_NT), 0, st, b);
  hipLaunchKernelGGL((sat_fix_kernel<TX, TY>), dim3(ntx, nty, n), dim3(EX_NT), 0, st, b);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

size_t extract_batch_workspace_bytes(const int* H, const int* W, const bool* with_sat, int n) {
  size_t off = 0;
  for (int i = 0; i < n; ++i)
    if (with_sat[i]) off += (extract_workspace_bytes(H[i], W[i]) + 255) / 256 * 256;
  return off;
}

int launch_extract_batch(const ExtractImage* ims, int n, int m, float sigma, int R, void* ws, hipStream_t st,
                         int scheme) {
  if (lds_bytes(m, R) > kMaxLds || R < 0 || R > kMaxGaussRadius) return -1;
  ExtractArgs a{};
  a.scheme = scheme;
  a.m = m;
  for (int k = 0; k < m; ++k) {
    double th = k * 3.14159265358979323846 / m;
    a.cs[k] = (float)cos(th);
    a.sn[k] = (float)sin(th);
  }
  double ws_[kMaxGaussRadius + 1], tot = 0.0;
  for (int j = 0; j <= R; ++j) { ws_[j] = exp(-(double)j * j / (2.0 * sigma * sigma)); tot += (j ? 2 : 1) * ws_[j]; }
  for (int j = 0; j <= R; ++j) a.w[j] = (float)(ws_[j] / tot);
  // the images' carry workspaces follow each other in image order
  std::vector<size_t> off((size_t)n);
  size_t o = 0;
  for (int i = 0; i < n; ++i) {
    off[i] = o;
    if (ims[i].sat) o += (extract_workspace_bytes(ims[i].H, ims[i].W) + 255) / 256 * 256;
  }
  // launch groups of images of similar size (largest first), so that few
  // workgroups of a group's overlaid grid fall outside their image
  std::vector<int> order((size_t)n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (int64_t)ims[x].H * ims[x].W > (int64_t)ims[y].H * ims[y].W;
  });
  for (int i0 = 0; i0 < n; i0 += kExBatch) {
    const int nb = std::min(kExBatch, n - i0);
    SatBatch sb{};
    int ntx = 0, nty = 0;
    for (int i = 0; i < nb; ++i) {
      const int j = order[i0 + i];
      const ExtractImage& src = ims[j];
      ExImage& I = a.im[i];
      I = ExImage{};
      I.img = src.img; I.stride = src.stride; I.vol = src.vol; I.sat = src.sat; I.H = src.H; I.W = src.W;
      I.ntx = (src.W + CF_TX - 1) / CF_TX;
      I.nty = (src.H + CF_TY - 1) / CF_TY;
      if (src.sat) {
        I.rc = (double*)((char*)ws + off[j]);
        I.bt = I.rc + (size_t)src.H * I.ntx;
      }
      sb.im[i] = SatImage{I.sat, I.rc, I.bt, I.H, I.W, I.ntx, I.nty};
      ntx = std::max(ntx, I.ntx);
      nty = std::max(nty, I.nty);
    }
    for (int i = nb; i < kExBatch; ++i) a.im[i] = ExImage{};
    const dim3 grid(ntx, nty, nb);
    int rc = -1;
    switch (R) {
      case 0: rc = launch_r<0>(a, grid, st); break;
      case 1: rc = launch_r<1>(a, grid, st); break;
      case 2: rc = launch_r<2>(a, grid, st); break;
      case 3: rc = launch_r<3>(a, grid, st); break;
      case 4: rc = launch_r<4>(a, grid, st); break;
      case 5: rc = launch_r<5>(a, grid, st); break;
      case 6: rc = launch_r<6>(a, grid, st); break;
      case 7: rc = launch_r<7>(a, grid, st); break;
      case 8: rc = launch_r<8>(a, grid, st); break;
      default: return -1;
    }
    if (rc != 0) return rc;
    rc = launch_sat<CF_TX, CF_TY>(sb, nb, st);
    if (rc != 0) return rc;
  }
  return 0;
}

int launch_extract(const float* img, int64_t stride, int H, int W, int m, float sigma, int R, float* vol,
                   double* sat, void* ws, hipStream_t st, int scheme) {
  const ExtractImage im{img, stride, H, W, vol, sat};
  return launch_extract_batch(&im, 1, m, sigma, R, ws, st, scheme);
}

}  // namespace cfog

namespace cfog {

template <int C>
static void launch_fh(const FhogArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(fhog_kernel<C>, dim3(a.ntx, a.nty), dim3(EX_NT), FhTile<C>::BYTES, st, a);
}

int launch_fhog(const float* img, int64_t stride, int H, int W, int cell, float* vol, double* sat, void* ws,
                hipStream_t st) {
  if (cell < 1 || cell > FH_MAX_CELL) return -1;
  FhogArgs a{};
  a.img = img; a.stride = stride; a.H = H; a.W = W; a.vol = vol; a.sat = sat;
  a.ntx = (W + EX_TX - 1) / EX_TX;
  a.nty = (H + EX_TY - 1) / EX_TY;
  a.rc = (double*)ws;
  a.bt = a.rc + (size_t)H * a.ntx;
  switch (cell) {
    case 1: launch_fh<1>(a, st); break;
    case 2: launch_fh<2>(a, st); break;
    case 3: launch_fh<3>(a, st); break;
    case 4: launch_fh<4>(a, st); break;
    case 5: launch_fh<5>(a, st); break;
    case 6: launch_fh<6>(a, st); break;
    case 7: launch_fh<7>(a, st); break;
    default: launch_fh<8>(a, st); break;
  }
  if (hipGetLastError() != hipSuccess) return -2;
  if (!sat) return 0;
  SatBatch sb{};
  sb.im[0] = SatImage{sat, a.rc, a.bt, H, W, a.ntx, a.nty};
  return launch_sat<EX_TX, EX_TY>(sb, 1, st);
}

}  // namespace cfog
