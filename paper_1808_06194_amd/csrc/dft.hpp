// Register-resident small DFT codelets for gfx950 (wave64).
//
// dft<R, DIR>(v) transforms R complex values held in registers:
//   X[k] = sum_n v[n] * exp(DIR * 2 pi i n k / R),   DIR = -1 forward, +1 inverse
// (unnormalised).  R in {2,3,4,5} are written out; composite R = A*B with
// coprime factors use the prime-factor mapping (no twiddles), the others a
// compile-time Cooley-Tukey split with constant-folded twiddles, so every
// loop below is fully unrolled and every twiddle is an immediate.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

#define CFOG_HD __host__ __device__ __forceinline__

namespace cfog {

// ------------------------------------------------------------ complex helpers
CFOG_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
CFOG_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
CFOG_HD float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// conj(a) * b
CFOG_HD float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -a.y * b.x));
}
// acc += conj(a) * b
CFOG_HD float2 cmac_conj(float2 acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, fmaf(a.y, b.y, acc.x));
  acc.y = fmaf(a.x, b.y, fmaf(-a.y, b.x, acc.y));
  return acc;
}
CFOG_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by DIR*i : (x + iy) * (DIR i)
template <int DIR>
CFOG_HD float2 mul_i(float2 a) {
  return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------- compile-time cos/sin (2 pi k / n)
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {  // |x| <= pi/4
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 14; ++i) { term *= -x2 / ((2 * i) * (2 * i + 1)); sum += term; }
  return sum;
}
constexpr double taylor_cos(double x) {  // |x| <= pi/4
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 14; ++i) { term *= -x2 / ((2 * i - 1) * (2 * i)); sum += term; }
  return sum;
}
// cos and sin of 2 pi k / n via octant reduction on the exact rational k/n.
constexpr double cos2pi(long k, long n) {
  k %= n; if (k < 0) k += n;
  // angle = 2 pi k / n = (pi/4) * (8k/n); octant o = floor(8k/n)
  long o = (8 * k) / n;
  double rem = (8.0 * k - o * n) / n;  // in [0,1)
  double x = rem * (kPi / 4);
  double c = taylor_cos(x), s = taylor_sin(x);
  double cp = taylor_cos(kPi / 4 - x), sp = taylor_sin(kPi / 4 - x);
  switch (o) {  // cos(o pi/4 + x)
    case 0: return c;
    case 1: return sp;          // cos(pi/4 + x) = sin(pi/4 - x)
    case 2: return -s;          // cos(pi/2 + x)
    case 3: return -cp;         // cos(3pi/4 + x) = -cos(pi/4 - x)
    case 4: return -c;
    case 5: return -sp;
    case 6: return s;
    default: return cp;
  }
}
// sin(2 pi k / n) = cos(2 pi (4k - n) / 4n)
constexpr double sin2pi(long k, long n) { return cos2pi(4 * k - n, 4 * n); }

template <int I, int N, class F>
CFOG_HD void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// v * exp(DIR * 2 pi i K / R) with K, R compile-time.
template <int K, int R, int DIR>
CFOG_HD float2 twiddle(float2 v) {
  constexpr int k = ((K % R) + R) % R;
  if constexpr (k == 0) {
    return v;
  } else if constexpr (4 * k == R) {
    return mul_i<DIR>(v);
  } else if constexpr (2 * k == R) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * k == 3 * R) {
    return mul_i<-DIR>(v);
  } else {
    constexpr float c = (float)cos2pi(k, R);
    constexpr float s = (float)(DIR * sin2pi(k, R));
    return make_float2(fmaf(v.x, c, -v.y * s), fmaf(v.x, s, v.y * c));
  }
}

template <int R, int DIR> struct Dft;

template <int DIR> struct Dft<1, DIR> {
  CFOG_HD static void run(float2*) {}
};

template <int DIR> struct Dft<2, DIR> {
  CFOG_HD static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int DIR> struct Dft<3, DIR> {
  CFOG_HD static void run(float2* v) {
    constexpr float s3 = 0.866025403784438646763723170752936183f;
    float2 a = v[0], b = v[1], c = v[2];
    float2 t = cadd(b, c);
    float2 m = make_float2(fmaf(-0.5f, t.x, a.x), fmaf(-0.5f, t.y, a.y));
    float2 d = csub(b, c);
    float2 n = mul_i<DIR>(cscale(d, s3));
    v[0] = cadd(a, t);
    v[1] = cadd(m, n);
    v[2] = csub(m, n);
  }
};

template <int DIR> struct Dft<4, DIR> {
  CFOG_HD static void run(float2* v) {
    float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    float2 s13 = cadd(v[1], v[3]), d13 = mul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  }
};

template <int DIR> struct Dft<5, DIR> {
  CFOG_HD static void run(float2* v) {
    constexpr float c1 = (float)cos2pi(1, 5), c2 = (float)cos2pi(2, 5);
    constexpr float s1 = (float)sin2pi(1, 5), s2 = (float)sin2pi(2, 5);
    float2 a = v[0];
    float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    float2 m1 = make_float2(a.x + c1 * t1.x + c2 * t2.x, a.y + c1 * t1.y + c2 * t2.y);
    float2 m2 = make_float2(a.x + c2 * t1.x + c1 * t2.x, a.y + c2 * t1.y + c1 * t2.y);
    float2 n1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    float2 n2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    n1 = mul_i<DIR>(n1);
    n2 = mul_i<DIR>(n2);
    v[0] = cadd(a, cadd(t1, t2));
    v[1] = cadd(m1, n1);
    v[4] = csub(m1, n1);
    v[2] = cadd(m2, n2);
    v[3] = csub(m2, n2);
  }
};

// Composite R = A * B:  n = B a + b,  k = k1 + A k2
//   X[k1 + A k2] = sum_b W_R^{b k1} W_B^{b k2} sum_a v[B a + b] W_A^{a k1}
template <int A, int B, int DIR>
struct DftSplit {
  CFOG_HD static void run(float2* v) {
    constexpr int R = A * B;
    float2 y[B][A];
    static_for<0, B>([&](auto bI) {
      constexpr int b = decltype(bI)::value;
      float2 t[A];
      static_for<0, A>([&](auto aI) { constexpr int a = decltype(aI)::value; t[a] = v[B * a + b]; });
      Dft<A, DIR>::run(t);
      static_for<0, A>([&](auto kI) {
        constexpr int k1 = decltype(kI)::value;
        y[b][k1] = twiddle<b * k1, R, DIR>(t[k1]);
      });
    });
    static_for<0, A>([&](auto kI) {
      constexpr int k1 = decltype(kI)::value;
      float2 t[B];
      static_for<0, B>([&](auto bI) { constexpr int b = decltype(bI)::value; t[b] = y[b][k1]; });
      Dft<B, DIR>::run(t);
      static_for<0, B>([&](auto k2I) { constexpr int k2 = decltype(k2I)::value; v[k1 + A * k2] = t[k2]; });
    });
  }
};

// Coprime R = A * B (Good-Thomas prime-factor algorithm): with the input map
// n = (B a + A b) mod R and the output map k = (B tA k1 + A tB k2) mod R,
// tA = B^-1 mod A, tB = A^-1 mod B, the exponent n k reduces mod R to
// B (B tA) a k1 + A (A tB) b k2, so
//   X[k(k1, k2)] = sum_b W_B^{b k2} sum_a W_A^{a k1} v[n(a, b)]
// with no twiddle factors between the two sets of small DFTs (the maps are
// compile-time register permutations).
constexpr int inv_mod(int x, int m) {
  for (int t = 1; t < m; ++t)
    if ((x * t) % m == 1) return t;
  return 1;  // m == 1
}

template <int A, int B, int DIR>
struct DftPfa {
  CFOG_HD static void run(float2* v) {
    constexpr int R = A * B;
    constexpr int tA = inv_mod(B % A, A), tB = inv_mod(A % B, B);
    float2 y[B][A];
    static_for<0, B>([&](auto bI) {
      constexpr int b = decltype(bI)::value;
      float2 t[A];
      static_for<0, A>([&](auto aI) { constexpr int a = decltype(aI)::value; t[a] = v[(B * a + A * b) % R]; });
      Dft<A, DIR>::run(t);
      static_for<0, A>([&](auto kI) { constexpr int k1 = decltype(kI)::value; y[b][k1] = t[k1]; });
    });
    float2 out[R];
    static_for<0, A>([&](auto kI) {
      constexpr int k1 = decltype(kI)::value;
      float2 t[B];
      static_for<0, B>([&](auto bI) { constexpr int b = decltype(bI)::value; t[b] = y[b][k1]; });
      Dft<B, DIR>::run(t);
      static_for<0, B>([&](auto k2I) {
        constexpr int k2 = decltype(k2I)::value;
        out[(B * tA * k1 + A * tB * k2) % R] = t[k2];
      });
    });
    static_for<0, R>([&](auto iI) { constexpr int i = decltype(iI)::value; v[i] = out[i]; });
  }
};

template <int DIR> struct Dft<6, DIR> : DftPfa<2, 3, DIR> {};
template <int DIR> struct Dft<8, DIR> : DftSplit<2, 4, DIR> {};
template <int DIR> struct Dft<9, DIR> : DftSplit<3, 3, DIR> {};
template <int DIR> struct Dft<10, DIR> : DftPfa<2, 5, DIR> {};
template <int DIR> struct Dft<12, DIR> : DftPfa<4, 3, DIR> {};
template <int DIR> struct Dft<15, DIR> : DftPfa<3, 5, DIR> {};
template <int DIR> struct Dft<16, DIR> : DftSplit<4, 4, DIR> {};
template <int DIR> struct Dft<18, DIR> : DftPfa<2, 9, DIR> {};
template <int DIR> struct Dft<20, DIR> : DftPfa<4, 5, DIR> {};
template <int DIR> struct Dft<24, DIR> : DftPfa<8, 3, DIR> {};

template <int R, int DIR>
CFOG_HD void dft(float2* v) { Dft<R, DIR>::run(v); }

}  // namespace cfog
