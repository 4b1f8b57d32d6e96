// SSD template matching of control points in the frequency domain
// (Section III-G of Ye et al.: Eqs. 3-6 and 8-9), one workgroup per control
// point at a time, everything on chip.
//
// For control point (x, y) in A with search centre (bx, by) in B, template side
// N, radius r, h = N/2, K = 2r+1, Ws = N + 2r:
//   T_c  = D_A[c][y-h .. y-h+N)[x-h .. x-h+N)               (template)
//   S_c  = D_B[c][by-h-r .. +Ws)[bx-h-r .. +Ws)              (search window)
//   C(u) = sum_c sum_q T_c(q) S_c(q+u),  u in [0, 2r]^2        (correlation)
//   SSD(d) = E1 + E2(d) - 2 C(d + r)                          (Eq. 5)
// with E1, E2 from the FP64 summed-area tables and d = u - r the returned
// offset of B's window relative to the search centre.
//
// The orientation axis of Eq. 9's 3-D transform is only ever read back at
// zero orientation shift, where the orientation DFT / inverse DFT pair reduces
// (Parseval) to a plain sum over channels of 2-D spectral products.  So each
// channel goes through real 2-D FFTs of size P x P (P >= Ws):
//   x-pass: rows of T_c (or S_c), two real rows packed per complex FFT, the
//           two half-spectra separated via Z(k) and conj Z(-k);
//   y-pass: complex column FFTs of the half-spectrum kx in [0, P/2];
//   ACC(ky, kx) += conj(T^_c) * S^_c  in registers.  Per plan layout: the
//           row spectra of T_c and S_c side by side in LDS, both x-passes in
//           one phase and each y-pass column transforming S then T (fused);
//           or T^_c parked in registers between the T and S passes of the
//           channel (the DC and Nyquist columns, both real, as one complex
//           column job where that saves a round);
// then one inverse: column IFFTs (kept rows u_y < K) and a C2R row IFFT with
// two output rows packed per complex FFT (kept columns u_x < K), the SSD
// assembly in FP64, and a lexicographic argmin + second-best over (SSD, index).
//
// Execution: every 1-D FFT of length P = R1 * R2 is owned by a group of
// G = max(R1, R2) lanes of one wave:
//   stage 1 (lane j < R2):  t[j R1 + k1] = sum_a x[j + R2 a] W_R1^{a k1}
//   stage 2 (lane k1 < R1): X[k1 + R1 k2] = sum_j W_P^{k1 j} t[j R1 + k1] W_R2^{j k2}
// with the small DFTs as unrolled register codelets (dft.hpp), the twiddles
// W_P^{k1 j} formed by recurrence from W_P^{k1}, and the exchange between
// stages through the FFT's own LDS row or column, with t at positions that
// keep a group's accesses in distinct banks (s1_pos, s1c).  Only the x -> y
// transposes need workgroup barriers (2 per channel in the fused layout, 4
// otherwise).
#include <hip/hip_runtime.h>
#include <limits.h>
#include <algorithm>
#include <mutex>
#include <vector>
#include "dft.hpp"
#include "epilogue.hpp"
#include "kernels.hpp"
#include "window.hpp"

namespace cfog {

// Orders the LDS accesses of one wave (the hardware keeps a wave's LDS
// operations in order; this stops the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// An integer the compiler must treat as computed here: addresses derived
// from it are rebuilt near their use instead of being hoisted out of the
// task loop and kept live (which costs registers).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Channel layouts of a plan: T^ parked in registers between the template's
// and the window's passes (LAY_REG), or both row spectra side by side in LDS
// (LAY_FUSED).
enum : int { LAY_REG = 0, LAY_FUSED = 1 };

template <int P_, int R1_, int R2_, int NT_, int LAY_>
struct FftCfg {
  static constexpr int P = P_, R1 = R1_, R2 = R2_, NT = NT_;
  static_assert(P == R1 * R2, "P must equal R1 * R2");
  static_assert(NT % 64 == 0 && NT <= 1024, "bad workgroup size");
  static constexpr int PH = P / 2 + 1;
  static constexpr int G = R1 > R2 ? R1 : R2;  // lanes per FFT group
  static constexpr int GPW = 64 / G;           // groups per wave
  static constexpr int NW = NT / 64;
  static constexpr int NG = NW * GPW;          // groups per workgroup
  // The DC and Nyquist columns of the x-pass half-spectra are real.  Where
  // P/2 is a multiple of NG, the P/2 + 1 columns would take a whole round
  // more than P/2 columns, so those two go through one complex column FFT as
  // its real and imaginary parts (the packed job, column index 0): P/2 column
  // jobs, a round and its accumulators fewer (P = 120 and 192).
  static constexpr bool PACK = (P / 2) % NG == 0;
  static constexpr int NCOL = PACK ? P / 2 : PH;   // column jobs of a y-pass
  static constexpr int KF = (NCOL + NG - 1) / NG;  // column rounds per group
  static constexpr size_t BASE = sizeof(float2) * ((size_t)P * PH + P) + NW * 16;
  // Fused layout (plans with one workgroup per CU): the row spectra of the
  // template (XT, up to XT_ROWS rows) and of the window (X, P rows) side by
  // side, so both x-passes share one phase and each y-pass column transforms
  // S then T: two barriers per channel instead of four, no T^ registers.
  // Templates of more rows than XT_ROWS take a larger plan.
  static constexpr bool FUSE = LAY_ == LAY_FUSED;
  static constexpr size_t XT_FIT = (kMaxLds - BASE) / (sizeof(float2) * PH) / 2 * 2;
  static constexpr int XT_ROWS = FUSE ? (int)(XT_FIT < (size_t)P ? XT_FIT : (size_t)P) : 0;
  static constexpr int T_ROWS = FUSE ? XT_ROWS : P;  // template rows the plan takes
  static constexpr size_t LDS = BASE + sizeof(float2) * (size_t)XT_ROWS * PH;
};

// Lane identity within the FFT group layout.
template <class C>
struct Lane {
  int g;   // group index in the workgroup (>= NG for idle lanes)
  int li;  // lane index in the group
  __device__ __forceinline__ Lane() {
    const int lane = threadIdx.x & 63, gi = lane / C::G;
    li = lane - gi * C::G;
    g = gi < C::GPW ? (int)(threadIdx.x >> 6) * C::GPW + gi : INT_MAX / 2;
  }
};

// The inputs of a stage-2 DFT of lane k1: w[b] = get(b) W_P^{-k1 b} (INV:
// W_P^{+k1 b}).  The twiddles come by recurrence from W_P^{k1}: one LDS read
// instead of R2 - 1 (measured 3% faster at P = 144, 15% at P = 192), at most
// R2 - 2 more FP32 roundings in each.
template <class C, bool INV, class Get>
__device__ __forceinline__ void stage2_inputs(float2 (&w)[C::R2], const float2* tw, int k1, Get&& get) {
  float2 t1 = tw[C::R1 + k1];
  if (INV) t1.y = -t1.y;
  float2 t = t1;
  w[0] = get(0);
#pragma unroll
  for (int b = 1; b < C::R2; ++b) {
    if (b > 1) t = cmul(t, t1);
    w[b] = cmul(get(b), t);
  }
}

// Where lane j of an x-pass group leaves stage-1 output k in its pair's row
// buffer (2 PH = P + 2 slots), chosen so that neither the group's writes
// (fixed k) nor its stage-2 reads (fixed j) share LDS banks: j R1 + k plus
// j / 4 (unpadded, the stride R1 puts lanes j and j + 8 in one bank at
// R1 = 12: 1% at P = 144, 12% at P = 192), and for R1 = 16 with R2 >= 10,
// where that still pairs lanes, k R2 + j plus k / 8 (a further 5% at P = 192).
template <class C>
__device__ __forceinline__ int s1_pos(int j, int k) {
  static_assert((C::R2 - 1) / 4 <= 2 && (C::R1 - 1) / 8 <= 1, "the stage-1 outputs must fit the pair's two rows");
  if constexpr (C::R1 == 16 && C::R2 >= 10) return k * C::R2 + j + (k >> 3);
  return j * C::R1 + k + (j >> 2);
}

// Where lane j of a column FFT leaves its stage-1 output k: row k R2 + j of
// the column, i.e. back in the rows it read (j + R2 a), so stage 1 is in place
// per lane and consecutive lanes write consecutive rows; stage 2 then reads
// rows k1 R2 + b.  (The natural order, row j R1 + k, puts a group's writes
// R1 rows apart, which at R1 = 16 lands 12 lanes in two LDS banks; measured:
// 2% faster at P = 144, 17% at P = 192.)
template <class C>
__device__ __forceinline__ int s1c(int j, int k) { return k * C::R2 + j; }

// One set of rows for the x-pass: nrows x ncols real values at src (leading
// dim ld), transformed into X (row stride PH).  zero_tail: rows
// [2 ceil(nrows/2), P) of X are zeroed (a y-pass that reads all P rows).
struct XRows {
  const float* src;
  int64_t ld;
  int nrows, ncols;
  float2* X;
  bool zero_tail;
};

// x-pass: forward FFTs of the rows of NS sets (the pairs of set 0, then those
// of set 1), zero-padded to P, two rows per complex FFT; leaves the
// half-spectra of the rows in each set's X as [row][kx], kx in [0, P/2].
template <class C, int NS>
__device__ __forceinline__ void xpass_fwd(const Lane<C>& L, const XRows (&S)[NS], const float2* tw) {
  constexpr int P = C::P, R1 = C::R1, R2 = C::R2, PH = C::PH;
  const int nrp0 = (S[0].nrows + 1) >> 1;
  const int total = NS > 1 ? nrp0 + ((S[NS - 1].nrows + 1) >> 1) : nrp0;
  // item i -> (set, pair)
  auto which = [&](int i, int& s, int& q) {
    s = (NS > 1 && i >= nrp0) ? 1 : 0;
    q = s ? i - nrp0 : i;
  };
  // the two rows of a pair, zero-padded, packed as one complex row
  auto load = [&](int i, float2 (&v)[R1]) {
    int s, q;
    which(i, s, q);
    const XRows& R = S[NS > 1 ? s : 0];
    const int j = L.li;
    const float* r0 = R.src + (int64_t)(2 * q) * R.ld;
    const bool has1 = (2 * q + 1) < R.nrows;
#pragma unroll
    for (int a = 0; a < R1; ++a) {
      const int xx = j + R2 * a;
      float re = 0.f, im = 0.f;
      if (xx < R.ncols) {
        re = ldg(r0 + xx);
        if (has1) im = ldg(r0 + R.ld + xx);
      }
      v[a] = make_float2(re, im);
    }
  };
  // each pair is loaded just before its transform: fetching the next pair
  // ahead lost on the plans that use this pass (P = 100 at 768 threads;
  // P = 160 and 192, whose registers spill, by 1%), unlike the prefetching
  // fused pass of P = 144
  for (int i = L.g; i < total; i += C::NG) {
    int s, q;
    which(i, s, q);
    const XRows& R = S[NS > 1 ? s : 0];
    float2* base = R.X + 2 * opaque(q) * PH;
    if (L.li < R2) {
      const int j = L.li;
      float2 v[R1];
      load(i, v);
      dft<R1, -1>(v);
#pragma unroll
      for (int k = 0; k < R1; ++k) base[s1_pos<C>(j, k)] = v[k];
    }
    wave_sync();
    xpass_stage2<C>(L, base, q, R.nrows, tw);
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) xpass_zero_tail<C>(S[s]);
}

// Stage 2 of the row FFT of pair q at base (stage 1 done), then the
// separation of the two packed rows into their half-spectra.
template <class C>
__device__ __forceinline__ void xpass_stage2(const Lane<C>& L, float2* base, int q, int nrows, const float2* tw) {
  constexpr int P = C::P, R1 = C::R1, R2 = C::R2, PH = C::PH;
  {
    // stage 2 on every lane of the group (idle lanes duplicate lane R1-1 so the
    // cross-lane fetch below runs with the whole wave active)
    const int k1 = L.li < R1 ? L.li : R1 - 1;
    float2 v[R2];
    stage2_inputs<C, false>(v, tw, k1, [&](int b) { return base[s1_pos<C>(b, k1)]; });
    dft<R2, -1>(v);
    // separate the packed rows: 2 A(k) = Z(k) + conj Z(-k), 2 B(k) = (Z(k) - conj Z(-k)) / i
    // (the factor 2 of both spectra, 4 in their product, is taken out by the
    // inverse's normalisation: exact, being a power of two).
    // Z(-k) for k = k1 + R1 k2 is Z((R1-k1) + R1 (R2-1-k2)), i.e. register R2-1-k2 of
    // lane R1-k1 of the group (k1 > 0), or this lane's register (R2-k2) mod R2 (k1 = 0).
    const int lane = threadIdx.x & 63;
    const int msrc = lane - L.li + (k1 == 0 ? 0 : R1 - k1);
    // the value of lane R1 - k1 of the group: where the group is a DPP row
    // (R1 = 16) or half row (R1 = 8), a mirror within it and a shift by one
    // lane (lane i then holds lane R1 - i's value; lane 0's is not used), on
    // the vector units; otherwise an LDS permute
    auto from_mirror = [&](float x) -> float {
      if constexpr (C::G == R1 && (R1 == 16 || R1 == 8)) {
        constexpr int MIRROR = R1 == 16 ? 0x140 : 0x141;  // row_mirror, row_half_mirror
        const int t = __builtin_amdgcn_update_dpp(0, __float_as_int(x), MIRROR, 0xf, 0xf, false);
        return __int_as_float(__builtin_amdgcn_update_dpp(0, t, 0x111, 0xf, 0xf, false));  // row_shr:1
      } else {
        return __shfl(x, msrc, 64);
      }
    };
    const bool odd_pad = (2 * q + 1) >= nrows;  // second row of the pair is padding
    static_for<0, R2>([&](auto k2I) {
      constexpr int k2 = decltype(k2I)::value;
      const float2 far = make_float2(from_mirror(v[R2 - 1 - k2].x), from_mirror(v[R2 - 1 - k2].y));
      const float2 zm = (k1 == 0) ? v[(R2 - k2) % R2] : far;
      const int k = k1 + R1 * k2;
      if (L.li < R1 && k <= P / 2) {
        const float2 z = v[k2];
        base[k] = make_float2(z.x + zm.x, z.y - zm.y);
        base[PH + k] = odd_pad ? make_float2(0.f, 0.f) : make_float2(z.y + zm.y, zm.x - z.x);
      }
    });
    wave_sync();
  }
}

// Rows [2 ceil(nrows/2), P) of a set's half-spectra are zero padding (an odd
// last row is zeroed by its pair); needed where a y-pass reads all P rows.
template <class C>
__device__ __forceinline__ void xpass_zero_tail(const XRows& R) {
  if (!R.zero_tail) return;
  const int r0 = 2 * ((R.nrows + 1) >> 1);
  for (int t = threadIdx.x; t < (C::P - r0) * C::PH; t += C::NT) R.X[r0 * C::PH + t] = make_float2(0.f, 0.f);
}

// The x-pass of the fused layout: as xpass_fwd over the template's rows then
// the window's, except that the first pair of this group (template pair L.g)
// was loaded into vn by the caller during the previous channel's y-pass,
// which hides its global-memory latency; vn then prefetches the next pair.
template <class C>
__device__ __forceinline__ void xpass_fused(const Lane<C>& L, const XRows (&S)[2], const float2* tw,
                                            float2 (&vn)[C::R1]) {
  constexpr int P = C::P, R1 = C::R1, R2 = C::R2, PH = C::PH;
  const int nrp0 = (S[0].nrows + 1) >> 1;
  const int total = nrp0 + ((S[1].nrows + 1) >> 1);
  auto load = [&](int i, float2 (&v)[R1]) {
    const bool s1 = i >= nrp0;
    const XRows& R = s1 ? S[1] : S[0];
    const int q = s1 ? i - nrp0 : i;
    const int j = L.li;
    const float* r0 = R.src + (int64_t)(2 * q) * R.ld;
    const bool has1 = (2 * q + 1) < R.nrows;
#pragma unroll
    for (int a = 0; a < R1; ++a) {
      const int xx = j + R2 * a;
      float re = 0.f, im = 0.f;
      if (xx < R.ncols) {
        re = ldg(r0 + xx);
        if (has1) im = ldg(r0 + R.ld + xx);
      }
      v[a] = make_float2(re, im);
    }
  };
  if (L.g >= nrp0 && L.g < total && L.li < R2) load(L.g, vn);  // not covered by the preload
  for (int i = L.g; i < total; i += C::NG) {
    const bool s1 = i >= nrp0;
    const XRows& R = s1 ? S[1] : S[0];
    const int q = s1 ? i - nrp0 : i;
    float2* base = R.X + 2 * opaque(q) * PH;
    if (L.li < R2) {
      const int j = L.li;
      float2 v[R1];
#pragma unroll
      for (int a = 0; a < R1; ++a) v[a] = vn[a];
      if (i + C::NG < total) load(i + C::NG, vn);
      dft<R1, -1>(v);
#pragma unroll
      for (int k = 0; k < R1; ++k) base[s1_pos<C>(j, k)] = v[k];
    }
    wave_sync();
    xpass_stage2<C>(L, base, q, R.nrows, tw);
  }
  xpass_zero_tail<C>(S[1]);
}

// Issues the loads of this group's first pair of the fused x-pass (template
// pair L.g) into vn.
template <class C>
__device__ __forceinline__ void xpass_fused_preload(const Lane<C>& L, const XRows& T, float2 (&vn)[C::R1]) {
  if (L.g < ((T.nrows + 1) >> 1) && L.li < C::R2) {
    const int j = L.li, q = L.g;
    const float* r0 = T.src + (int64_t)(2 * q) * T.ld;
    const bool has1 = (2 * q + 1) < T.nrows;
#pragma unroll
    for (int a = 0; a < C::R1; ++a) {
      const int xx = j + C::R2 * a;
      float re = 0.f, im = 0.f;
      if (xx < T.ncols) {
        re = ldg(r0 + xx);
        if (has1) im = ldg(r0 + T.ld + xx);
      }
      vn[a] = make_float2(re, im);
    }
  }
}

// Row `row` of a y-pass input column: col[row PH], or for the packed job
// (col = X, the DC column) the DC value plus i times the Nyquist value.
template <class C>
__device__ __forceinline__ float2 col_in(const float2* col, int row, bool pk) {
  const float2 v = col[row * C::PH];
  return pk ? make_float2(v.x, col[row * C::PH + C::P / 2].x) : v;
}

// The packed job's share of the spectral product, for lane k1 holding
// ky = k1 + R1 k2.  zs and zt are the column FFTs of (DC + i Nyquist) of the
// window and the template; with F(-ky) = F((P - ky) mod P),
//   T0 = (zt + conj zt(-ky)) / 2,  TN = (zt - conj zt(-ky)) / 2i  (S likewise),
// both Hermitian in ky, and acc += conj(T0) S0 + i conj(TN) SN, whose inverse
// column FFT is the DC column's correlation plus i times the Nyquist one's:
//   conj(T0) S0 + i conj(TN) SN = (u s + i v t) / 4,
//   u, v = conj zt +- zt(-ky),  s, t = zs +- conj zs(-ky).
// The values at -ky come through LDS: column 0 takes zs, column P/2 zt.
template <class C>
__device__ __forceinline__ void packed_mac(float2* col, int k1, const float2 (&zs)[C::R2], const float2 (&zt)[C::R2],
                                           float2 (&acc)[C::R2]) {
  constexpr int P = C::P, R1 = C::R1, R2 = C::R2, PH = C::PH;
  wave_sync();  // the stage-2 reads of the column are done
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    const int ky = k1 + R1 * k2;
    col[ky * PH] = zs[k2];
    col[ky * PH + P / 2] = zt[k2];
  }
  wave_sync();
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    const int ky = k1 + R1 * k2;
    const int km = ky == 0 ? 0 : P - ky;
    const float2 sm = col[km * PH], tm = col[km * PH + P / 2];
    const float2 ta = zt[k2], sc = zs[k2];
    const float2 u = make_float2(ta.x + tm.x, tm.y - ta.y);
    const float2 v = make_float2(ta.x - tm.x, -ta.y - tm.y);
    const float2 sp = make_float2(sc.x + sm.x, sc.y - sm.y);
    const float2 sq = make_float2(sc.x - sm.x, sc.y + sm.y);
    const float2 us = cmul(u, sp), vt = cmul(v, sq);
    acc[k2].x = fmaf(0.25f, us.x - vt.y, acc[k2].x);
    acc[k2].y = fmaf(0.25f, us.y + vt.x, acc[k2].y);
  }
}

// y-pass of the fused layout.  For each column kx of the group: the window's
// column FFT in place in X (all P rows), then the template's, whose first
// stage reads XT (rows < nT, zero beyond) and writes its intermediate into the
// X column the window's transform has just left; conj(T^) S^ is accumulated
// into acc[rnd][k2] for ky = k1 + R1 k2.
template <class C>
__device__ __forceinline__ void ypass_fused(const Lane<C>& L, const float2* XT, int nT, float2* X, const float2* tw,
                                            float2 (&acc)[C::KF][C::R2]) {
  constexpr int R1 = C::R1, R2 = C::R2, PH = C::PH;
  static_for<0, C::KF>([&](auto rndI) {
    constexpr int rnd = decltype(rndI)::value;
    const int kx = L.g + rnd * C::NG;
    if (kx < C::NCOL) {
      const bool pk = C::PACK && rnd == 0 && kx == 0;
      float2* col = X + opaque(kx);
      const float2* colT = XT + kx;
      float2 sh[R2];
      // window: stage 1 in place, stage 2 into registers
      if (L.li < R2) {
        const int j = L.li;
        float2 v[R1];
#pragma unroll
        for (int a = 0; a < R1; ++a) v[a] = col_in<C>(col, j + R2 * a, pk);
        dft<R1, -1>(v);
#pragma unroll
        for (int k = 0; k < R1; ++k) col[s1c<C>(j, k) * PH] = v[k];
      }
      wave_sync();
      if (L.li < R1) {
        const int k1 = L.li;
        stage2_inputs<C, false>(sh, tw, k1, [&](int b) { return col[s1c<C>(b, k1) * PH]; });
        dft<R2, -1>(sh);
      }
      wave_sync();
      // template: stage 1 from XT into the X column, stage 2 into registers
      if (L.li < R2) {
        const int j = L.li;
        float2 v[R1];
#pragma unroll
        for (int a = 0; a < R1; ++a) {
          const int row = j + R2 * a;
          v[a] = row < nT ? col_in<C>(colT, row, pk) : make_float2(0.f, 0.f);
        }
        dft<R1, -1>(v);
#pragma unroll
        for (int k = 0; k < R1; ++k) col[s1c<C>(j, k) * PH] = v[k];
      }
      wave_sync();
      if (L.li < R1) {
        const int k1 = L.li;
        float2 w[R2];
        stage2_inputs<C, false>(w, tw, k1, [&](int b) { return col[s1c<C>(b, k1) * PH]; });
        dft<R2, -1>(w);
        if (pk) {
          packed_mac<C>(col, k1, sh, w, acc[rnd]);
        } else {
#pragma unroll
          for (int k2 = 0; k2 < R2; ++k2) acc[rnd][k2] = cmac_conj(acc[rnd][k2], w[k2], sh[k2]);
        }
      }
    }
  });
}

// y-pass: forward column FFTs of the half-spectrum (rows >= nrows were zeroed
// by the x-pass).
// Column kx = g + rnd * NG; lane k1 < R1 of its group ends up with
// ky = k1 + R1 k2 and hands each value to sink(rnd, k2, kx, value), or for
// the packed job all of them to psink(rnd, k1, values, column).
template <class C, class Sink, class PSink>
__device__ __forceinline__ void ypass_fwd(const Lane<C>& L, float2* X, const float2* tw, Sink&& sink, PSink&& psink) {
  constexpr int R1 = C::R1, R2 = C::R2, PH = C::PH;
  static_for<0, C::KF>([&](auto rndI) {
    constexpr int rnd = decltype(rndI)::value;
    const int kx = L.g + rnd * C::NG;
    if (kx < C::NCOL) {
      const bool pk = C::PACK && rnd == 0 && kx == 0;
      float2* col = X + opaque(kx);
      if (L.li < R2) {
        const int j = L.li;
        float2 v[R1];
#pragma unroll
        for (int a = 0; a < R1; ++a) v[a] = col_in<C>(col, j + R2 * a, pk);
        dft<R1, -1>(v);
#pragma unroll
        for (int k = 0; k < R1; ++k) col[s1c<C>(j, k) * PH] = v[k];
      }
      wave_sync();
      if (L.li < R1) {
        const int k1 = L.li;
        float2 w[R2];
        stage2_inputs<C, false>(w, tw, k1, [&](int b) { return col[s1c<C>(b, k1) * PH]; });
        dft<R2, -1>(w);
        if (pk) {
          psink(rndI, k1, w, col);
        } else {
          static_for<0, R2>([&](auto k2I) {
            constexpr int k2 = decltype(k2I)::value;
            sink(rndI, k2I, kx, w[k2]);
          });
        }
      }
    }
  });
}

// Control point cpi of job jd over the channels [c0, c1).  part == nullptr:
// the whole sum, finished by the epilogue; otherwise the partial correlation
// surface goes to part (item g of a split task; item 0 reports an
// out-of-bounds point).
template <class C>
__device__ __forceinline__ void match_one(const Lane<C>& L, const MatchJob& jd, int cpi, float2* X, const float2* tw,
                          ArgminState* red, int c0, int c1, float* __restrict__ part, int g) {
  constexpr int P = C::P, R1 = C::R1, R2 = C::R2, PH = C::PH, NT = C::NT, KF = C::KF;
  const int4 cp = jd.cps[cpi];
  const int N = jd.N, r = jd.r, K = 2 * r + 1, Ws = N + 2 * r;
  const CpBoxes bx = cp_boxes(cp.x, cp.y, cp.z, cp.w, N, r, jd.hA, jd.wA, jd.hB, jd.wB);
  if (!bx.inside) {
    if (g == 0) oob_result<NT>(jd, cpi);
    return;
  }
  const int tx0 = bx.tx0, ty0 = bx.ty0, sx0 = bx.sx0, sy0 = bx.sy0;

  float2 acc[KF][R2];
#pragma unroll
  for (int k = 0; k < KF; ++k)
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) acc[k][k2] = make_float2(0.f, 0.f);

  const size_t planeA = (size_t)jd.hA * jd.wA, planeB = (size_t)jd.hB * jd.wB;
  const float* tA = jd.volA + (size_t)ty0 * jd.wA + tx0;
  const float* sB = jd.volB + (size_t)sy0 * jd.wB + sx0;
  // fused layout: both x-passes in one phase (template rows into XT, window
  // rows into X), then one y-pass phase; two barriers per channel
  auto fused_channels = [&]() {
    float2* XT = reinterpret_cast<float2*>(reinterpret_cast<char*>(X) + C::BASE);
    if constexpr (C::P >= 144) {
      // P = 144 loads the next channel's first template pair during this
      // channel's y-pass (measured: 1.4%).  At P = 120 (768 threads, 168
      // VGPRs) the pair held through the y-pass raised the spills from 6 to
      // 26 VGPRs and made the plan 7% slower.
      float2 vn[R1];
      xpass_fused_preload<C>(L, XRows{tA + c0 * planeA, jd.wA, N, N, XT, false}, vn);
      for (int c = c0; c < c1; ++c) {
        __syncthreads();  // previous readers of X and XT are done
        const XRows rows[2] = {{tA + c * planeA, jd.wA, N, N, XT, false}, {sB + c * planeB, jd.wB, Ws, Ws, X, true}};
        xpass_fused<C>(L, rows, tw, vn);
        __syncthreads();
        if (c + 1 < c1) xpass_fused_preload<C>(L, XRows{tA + (c + 1) * planeA, jd.wA, N, N, XT, false}, vn);
        ypass_fused<C>(L, XT, N, X, tw, acc);
      }
    } else {
      for (int c = c0; c < c1; ++c) {
        __syncthreads();  // previous readers of X and XT are done
        const XRows rows[2] = {{tA + c * planeA, jd.wA, N, N, XT, false}, {sB + c * planeB, jd.wB, Ws, Ws, X, true}};
        xpass_fwd<C, 2>(L, rows, tw);
        __syncthreads();
        ypass_fused<C>(L, XT, N, X, tw, acc);
      }
    }
  };
  // two-phase layout: T^ parked in registers between the template's and the
  // window's passes; four barriers per channel
  auto split_channels = [&]() {
    for (int c = c0; c < c1; ++c) {
      float2 th[KF][R2];
      __syncthreads();  // previous readers of X are done
      const XRows rt[1] = {{tA + c * planeA, jd.wA, N, N, X, true}};
      xpass_fwd<C, 1>(L, rt, tw);
      __syncthreads();
      auto park = [&](auto rndI, auto k2I, int, float2 v) {
        constexpr int rnd = decltype(rndI)::value, k2 = decltype(k2I)::value;
        th[rnd][k2] = v;
      };
      ypass_fwd<C>(L, X, tw, park, [&](auto rndI, int, const float2 (&w)[R2], float2*) {
        static_for<0, R2>([&](auto k2I) { park(rndI, k2I, 0, w[decltype(k2I)::value]); });
      });
      __syncthreads();
      const XRows rs[1] = {{sB + c * planeB, jd.wB, Ws, Ws, X, true}};
      xpass_fwd<C, 1>(L, rs, tw);
      __syncthreads();
      auto parked = [&](auto rndI, auto k2I, int) {
        constexpr int rnd = decltype(rndI)::value, k2 = decltype(k2I)::value;
        return th[rnd][k2];
      };
      ypass_fwd<C>(L, X, tw, [&](auto rndI, auto k2I, int kx, float2 v) {
        constexpr int rnd = decltype(rndI)::value, k2 = decltype(k2I)::value;
        acc[rnd][k2] = cmac_conj(acc[rnd][k2], parked(rndI, k2I, kx), v);
      }, [&](auto rndI, int k1, const float2 (&w)[R2], float2* col) {
        constexpr int rnd = decltype(rndI)::value;
        float2 zt[R2];
        static_for<0, R2>([&](auto k2I) { zt[decltype(k2I)::value] = parked(rndI, k2I, 0); });
        packed_mac<C>(col, k1, w, zt, acc[rnd]);
      });
    }
  };
  if constexpr (C::FUSE) fused_channels();  // N <= XT_ROWS (plan_fits)
  else split_channels();

  // ---- inverse along y: each group transforms its own columns in place and
  // keeps the rows u_y < K (no workgroup barrier: a column is group-private).
#pragma unroll
  for (int rnd = 0; rnd < KF; ++rnd) {
    const int kx = L.g + rnd * C::NG;
    if (kx < C::NCOL) {
      // the packed job's outputs: real part the DC column, imaginary the Nyquist
      const bool pk = C::PACK && rnd == 0 && kx == 0;
      float2* col = X + opaque(kx);
      if (L.li < R1) {
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) col[(L.li + R1 * k2) * PH] = acc[rnd][k2];
      }
      wave_sync();
      if (L.li < R2) {
        const int j = L.li;
        float2 v[R1];
#pragma unroll
        for (int a = 0; a < R1; ++a) v[a] = col[(j + R2 * a) * PH];
        dft<R1, +1>(v);
#pragma unroll
        for (int k = 0; k < R1; ++k) col[s1c<C>(j, k) * PH] = v[k];
      }
      wave_sync();
      if (L.li < R1) {
        const int k1 = L.li;
        float2 w[R2];
        stage2_inputs<C, true>(w, tw, k1, [&](int b) { return col[s1c<C>(b, k1) * PH]; });
        dft<R2, +1>(w);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
          const int uy = k1 + R1 * k2;
          if (uy < K) {
            if (pk) {
              col[uy * PH] = make_float2(w[k2].x, 0.f);
              col[uy * PH + P / 2] = make_float2(w[k2].y, 0.f);
            } else {
              col[uy * PH] = w[k2];
            }
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- inverse along x: C2R, two output rows per complex FFT, kept u_x < K.
  // A pair's stage-1 outputs overwrite its own two input rows (2 PH >= P
  // slots, read into registers by the same wave first); the correlation
  // C(u_y, u_x) goes to LDS behind all the pairs' rows.
  const int npair = (K + 1) >> 1;
  float* Cs = reinterpret_cast<float*>(X + 2 * npair * PH);
  // 1/P^2 of the inverse 2-D DFT and 1/4 for the doubled row spectra of T and S
  const float inv = 0.25f / ((float)P * (float)P);
  for (int p = L.g; p < npair; p += C::NG) {
    float2* sc = X + 2 * opaque(p) * PH;
    float2 v[R1];
    if (L.li < R2) {
      const int j = L.li;
      const float2* v1r = X + (2 * p) * PH;
      const bool has2 = 2 * p + 1 < K;
#pragma unroll
      for (int a = 0; a < R1; ++a) {
        const int kx = j + R2 * a;
        const bool lo = kx <= P / 2;
        const int kk = lo ? kx : P - kx;
        const float2 v1 = v1r[kk];
        const float2 v2 = has2 ? v1r[PH + kk] : make_float2(0.f, 0.f);
        v[a] = lo ? make_float2(v1.x - v2.y, v1.y + v2.x) : make_float2(v1.x + v2.y, v2.x - v1.y);
      }
    }
    wave_sync();  // every read of the pair's rows precedes the writes into them
    if (L.li < R2) {
      dft<R1, +1>(v);
#pragma unroll
      for (int k = 0; k < R1; ++k) sc[L.li * R1 + k] = v[k];
    }
    wave_sync();
    if (L.li < R1) {
      const int k1 = L.li;
      float2 w[R2];
      stage2_inputs<C, true>(w, tw, k1, [&](int b) { return sc[k1 + R1 * b]; });
      dft<R2, +1>(w);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int ux = k1 + R1 * k2;
        if (ux < K) {
          Cs[(2 * p) * K + ux] = w[k2].x * inv;
          if (2 * p + 1 < K) Cs[(2 * p + 1) * K + ux] = w[k2].y * inv;
        }
      }
    }
  }
  __syncthreads();

  if (part) {
    for (int i = threadIdx.x; i < K * K; i += NT) stg(part + i, Cs[i]);
    return;
  }
  ssd_epilogue<NT>(jd, cpi, tx0, ty0, sx0, sy0, Cs, red);
}

// One kernel for both paths: with jobs == nullptr every task t is control
// point t of job0 (plain path); otherwise task t = tasks[t] = (job, cp) over the
// device job table (batched path).  Workgroups loop over tasks with a grid
// stride.
template <class C>
__global__ __launch_bounds__(C::NT) void match_fft_kernel(MatchJob job0, const MatchJob* __restrict__ jobs,
                                                          const int2* __restrict__ tasks, int n_tasks,
                                                          SplitArgs sp) {
  extern __shared__ float2 smem[];
  float2* X = smem;
  float2* tw = X + C::P * C::PH;
  ArgminState* red = reinterpret_cast<ArgminState*>(tw + C::P);
  // stage-2 twiddles W_P^{k1 b} stored lane-major, tw[b * R1 + k1] (stage 2
  // reads row b = 1 and forms the other powers)
  for (int i = threadIdx.x; i < C::P; i += C::NT) {
    const int b = i / C::R1, k1 = i - b * C::R1;
    double s, c;
    sincospi(2.0 * (double)((k1 * b) % C::P) / C::P, &s, &c);
    tw[i] = make_float2((float)c, (float)-s);
  }
  const Lane<C> L;
  const int n_items = split_items(n_tasks, sp);
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    __syncthreads();  // twiddles ready / previous task's reduction done
    int t = it, g = 0, G = 1;
    if (sp.G > 1 && it >= sp.n_whole) {  // an item of a split task
      const int s = it - sp.n_whole;
      t = sp.n_whole + s / sp.G;
      g = s - (t - sp.n_whole) * sp.G;
      G = sp.G;
    }
    MatchJob jd = job0;
    int cpi = t;
    if (jobs) {
      const int2 tk = tasks[t];
      jd = jobs[tk.x];
      cpi = tk.y;
    }
    float* part = G > 1 ? sp.part + (size_t)(it - sp.n_whole) * sp.slot : nullptr;
    match_one<C>(L, jd, cpi, X, tw, red, g * jd.m / G, (g + 1) * jd.m / G, part, g);
  }
}

// ------------------------------------------------------------------ plans
//  P, R1, R2, NT, layout  (R1 >= R2 keeps the per-lane outputs of stage 2
//  small).  NT is set per size from measurement: as many waves as the
//  registers allow, in workgroups that fill a CU's wave slots (P = 32 and
//  40 at 256 threads instead of 192, 2% faster; P = 60 and 64 at 512
//  threads: 16 waves per CU where 384 and 320 threads left 12 and 15, 10%
//  and 15% faster; P = 80-120 at 768 threads, three waves per
//  SIMD: P = 80 and 90 6% and 5% faster than at 448 and 512, P = 96..108
//  take every column in one round, P = 120 is 19% faster than at 512;
//  P = 144 at 512 threads beats 256-384 and 768).  The layout too: the
//  fused one was 6-18% faster than parking T^ in registers for P = 80..144.
//  P = 160 and 192 park T^ in registers at 512 threads, where P = 192's
//  DC/Nyquist packing leaves three whole column rounds: 10% and 18% faster
//  than parking it in a global workspace at 768 threads, whose round trip
//  was most of their HBM traffic.
//  Sizes that lost to the next larger one on every measured (N, r) are left
//  out: P = 128 (T^ in registers, 256 VGPRs and spills: 25-35% slower than
//  P = 144), P = 150 (15 x 10, fused, 512 threads, spills: 1-11% slower than
//  P = 160 on the same windows since P = 160 keeps T^ in registers; its
//  registers layout spills 161 VGPRs) and P = 180 (15 x 12, several hundred
//  spilled registers at any workgroup size: twice the time of P = 192).
#define CFOG_PLANS(X)                  \
  X(16, 4, 4, 64, LAY_REG)             \
  X(24, 6, 4, 128, LAY_REG)            \
  X(32, 8, 4, 256, LAY_REG)            \
  X(40, 8, 5, 256, LAY_REG)            \
  X(48, 8, 6, 256, LAY_REG)            \
  X(60, 10, 6, 512, LAY_REG)           \
  X(64, 8, 8, 512, LAY_REG)            \
  X(72, 9, 8, 384, LAY_REG)            \
  X(80, 10, 8, 768, LAY_FUSED)         \
  X(90, 10, 9, 768, LAY_FUSED)         \
  X(96, 12, 8, 768, LAY_FUSED)         \
  X(100, 10, 10, 768, LAY_FUSED)       \
  X(108, 12, 9, 768, LAY_FUSED)        \
  X(120, 12, 10, 768, LAY_FUSED)       \
  X(144, 12, 12, 512, LAY_FUSED)       \
  X(160, 16, 10, 512, LAY_REG)         \
  X(192, 16, 12, 512, LAY_REG)

#define CFOG_CFG(P_, R1_, R2_, NT_, L_) FftCfg<P_, R1_, R2_, NT_, L_>

static const FftPlan kPlans[] = {
#define CFOG_PLAN_ENTRY(P_, R1_, R2_, NT_, L_) \
  {P_, R1_, R2_, NT_, CFOG_CFG(P_, R1_, R2_, NT_, L_)::LDS, CFOG_CFG(P_, R1_, R2_, NT_, L_)::T_ROWS},
    CFOG_PLANS(CFOG_PLAN_ENTRY)
#undef CFOG_PLAN_ENTRY
};

const FftPlan* fft_plans(int* count) {
  *count = (int)(sizeof(kPlans) / sizeof(kPlans[0]));
  return kPlans;
}

bool plan_fits(const FftPlan* p, int N, int r) {
  if (N < 1 || r < 0 || N > kMaxSide || r > kMaxSide) return false;
  const int Ws = N + 2 * r, K = 2 * r + 1;
  if (p->P < Ws || N > p->t_rows) return false;
  const int PH = p->P / 2 + 1;
  // the K x K correlation must fit behind the rows of the inverse's row pairs
  return (long)K * K <= 2L * (long)(p->P - 2 * ((K + 1) / 2)) * PH;
}

const FftPlan* choose_fft_plan(int N, int r) {
  for (const FftPlan& p : kPlans)
    if (plan_fits(&p, N, r)) return &p;
  return nullptr;
}

// Workgroups of each plan resident per CU, from the runtime's occupancy
// calculator (registers, LDS and waves); filled by init_match_fft_attributes.
static int g_plan_occupancy[64];

int plan_slots(const FftPlan* p, int num_cus) {
  const int i = (int)(p - kPlans);
  int per_cu = (i >= 0 && i < 64) ? g_plan_occupancy[i] : 0;
  if (per_cu <= 0) per_cu = std::max(1, std::min((int)(kMaxLds / p->lds), 32 / (p->NT / 64)));
  return num_cus * per_cu;
}

template <class C>
static int launch_t(const MatchJob& job0, const MatchJob* jobs, const int2* tasks, int n_tasks, int n_blocks,
                    const SplitArgs& sp, hipStream_t st) {
  hipLaunchKernelGGL(match_fft_kernel<C>, dim3(n_blocks), dim3(C::NT), C::LDS, st, job0, jobs, tasks, n_tasks, sp);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// One workgroup per split task: the sum of its G partial surfaces (in item
// order) into LDS, then the epilogue of the whole sum.
constexpr int SR_NT = 1024;
__global__ __launch_bounds__(SR_NT) void split_reduce_kernel(MatchJob job0, const MatchJob* __restrict__ jobs,
                                                            const int2* __restrict__ tasks, SplitArgs sp) {
  extern __shared__ float4 sr_lds[];
  ArgminState* red = reinterpret_cast<ArgminState*>(sr_lds);
  float* Cs = reinterpret_cast<float*>(red + SR_NT / 64);
  const int t = sp.n_whole + blockIdx.x;
  MatchJob jd = job0;
  int cpi = t;
  if (jobs) {
    const int2 tk = tasks[t];
    jd = jobs[tk.x];
    cpi = tk.y;
  }
  const int4 cp = jd.cps[cpi];
  const int K = 2 * jd.r + 1;
  const CpBoxes bx = cp_boxes(cp.x, cp.y, cp.z, cp.w, jd.N, jd.r, jd.hA, jd.wA, jd.hB, jd.wB);
  if (!bx.inside) return;  // reported by the task's first item
  const float* p = sp.part + (size_t)blockIdx.x * sp.G * sp.slot;
  for (int i = threadIdx.x; i < K * K; i += SR_NT) {
    float s = ldg(p + i);
    for (int g = 1; g < sp.G; ++g) s += ldg(p + (size_t)g * sp.slot + i);
    Cs[i] = s;
  }
  __syncthreads();
  ssd_epilogue<SR_NT>(jd, cpi, bx.tx0, bx.ty0, bx.sx0, bx.sy0, Cs, red);
}

int launch_split_reduce(const MatchJob& job0, const MatchJob* d_jobs, const int2* d_tasks, int n_tasks,
                        const SplitArgs& sp, hipStream_t st) {
  if (sp.G <= 1 || n_tasks <= sp.n_whole) return 0;
  const size_t lds = sizeof(ArgminState) * (SR_NT / 64) + sizeof(float) * (size_t)sp.slot;
  if (lds > kMaxLds) return -1;
  hipLaunchKernelGGL(split_reduce_kernel, dim3(n_tasks - sp.n_whole), dim3(SR_NT), lds, st, job0, d_jobs, d_tasks,
                     sp);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int init_match_fft_attributes() {
  int idx = 0;
#define CFOG_PLAN_ATTR(P_, R1_, R2_, NT_, L_)                                                               \
  {                                                                                                          \
    using Cfg = CFOG_CFG(P_, R1_, R2_, NT_, L_);                                                             \
    if (hipFuncSetAttribute((const void*)match_fft_kernel<Cfg>, hipFuncAttributeMaxDynamicSharedMemorySize,  \
                            (int)Cfg::LDS) != hipSuccess)                                                    \
      return -2;                                                                                             \
    int n = 0;                                                                                               \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, match_fft_kernel<Cfg>, Cfg::NT, Cfg::LDS) !=        \
        hipSuccess)                                                                                          \
      n = 0;                                                                                                 \
    g_plan_occupancy[idx++] = n;                                                                             \
  }
  CFOG_PLANS(CFOG_PLAN_ATTR)
#undef CFOG_PLAN_ATTR
  if (hipFuncSetAttribute((const void*)split_reduce_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kMaxLds) != hipSuccess)
    return -2;
  return 0;
}

int init_kernel_attributes() {
  static std::mutex mu;
  static std::vector<int> done;  // devices already set up
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -2;
  std::lock_guard<std::mutex> lock(mu);
  if (std::find(done.begin(), done.end(), dev) != done.end()) return 0;
  int rc = init_match_fft_attributes();
  if (rc == 0) rc = init_extract_attributes();
  if (rc == 0) rc = init_direct_attributes();
  if (rc == 0) rc = init_harris_attributes();
  if (rc == 0) rc = init_outlier_attributes();
  if (rc == 0) done.push_back(dev);
  return rc;
}

int launch_match_fft(const FftPlan* plan, const MatchJob& job0, const MatchJob* d_jobs, const int2* d_tasks,
                     int n_tasks, int n_blocks, const SplitArgs& sp, hipStream_t st) {
  if (n_tasks <= 0) return 0;
#define CFOG_PLAN_CASE(P_, R1_, R2_, NT_, L_) \
  if (plan->P == P_)                          \
    return launch_t<CFOG_CFG(P_, R1_, R2_, NT_, L_)>(job0, d_jobs, d_tasks, n_tasks, n_blocks, sp, st);
  CFOG_PLANS(CFOG_PLAN_CASE)
#undef CFOG_PLAN_CASE
  return -1;
}

}  // namespace cfog
