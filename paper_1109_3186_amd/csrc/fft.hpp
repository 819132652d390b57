// Register-resident, LDS-exchanged complex FFT for one workgroup (gfx950).
//
// One workgroup transforms one N-point sequence, N = 2^LOGN with 8 <= LOGN <= 15.
// Each of the T = N / P threads keeps P points in registers.  The transform is a
// Stockham auto-sort sequence of radix-R passes (R divides P): in a pass with
// current sub-transform length NS, butterfly j (0 <= j < N/R) reads the points
// j + r N/R, multiplies point r by exp(s 2 pi i r k / (NS R)) with k = j mod NS,
// does an R-point DFT in registers and writes output q to
// (j / NS) NS R + k + q NS.  Between passes the points travel through LDS, real
// parts then imaginary parts, so that N = 32768 fits the 160 KB of one CU.
//
// A launch provides Geo<PL>::LDS_TOTAL floats of dynamic LDS: the exchange area and,
// for the larger plans, the second pass's twiddle table after it.
//
// Load pattern of the first pass and store pattern of the last pass are both
// "point (t + u T) + r N / R", i.e. coalesced across threads (held in register
// u R + in_reg(r) before a pass's DFT, u R + out_reg(q) after it), and the output
// is in natural order.  The transform is unnormalised:
// sum_n x[n] exp(s 2 pi i k n / N) with s = -1 (forward) or +1 (inverse).
#pragma once
#include <hip/hip_runtime.h>

namespace ddx {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// sin(2 pi x) and cos(2 pi x) of an angle given in revolutions; the hardware
// transcendental unit takes revolutions directly (measured max abs error
// 1.24e-7 over [-1/2, 1/2)).
__device__ __forceinline__ float sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float cos_rev(float x) { return __builtin_amdgcn_cosf(x); }

// exp(S 2 pi i num / 2^LOGDEN) for 0 <= num < 2^LOGDEN, reduced exactly to [-1/2, 1/2).
template <int LOGDEN, int S>
__device__ __forceinline__ float2 twiddle(int num) {
  float x = (float)num * (1.0f / (float)(1 << LOGDEN));
  x = (x >= 0.5f) ? x - 1.0f : x;
  return make_float2(cos_rev(x), (float)S * sin_rev(x));
}

// cos and sin of 2 pi m / 32, m = 0..15 (constants of the in-register butterflies)
__device__ constexpr float kCos32[16] = {
    1.000000000e+00f, 9.807852804e-01f, 9.238795325e-01f, 8.314696123e-01f,
    7.071067812e-01f, 5.555702330e-01f, 3.826834324e-01f, 1.950903220e-01f,
    0.0f,             -1.950903220e-01f, -3.826834324e-01f, -5.555702330e-01f,
    -7.071067812e-01f, -8.314696123e-01f, -9.238795325e-01f, -9.807852804e-01f};
__device__ constexpr float kSin32[16] = {
    0.0f,             1.950903220e-01f, 3.826834324e-01f, 5.555702330e-01f,
    7.071067812e-01f, 8.314696123e-01f, 9.238795325e-01f, 9.807852804e-01f,
    1.000000000e+00f, 9.807852804e-01f, 9.238795325e-01f, 8.314696123e-01f,
    7.071067812e-01f, 5.555702330e-01f, 3.826834324e-01f, 1.950903220e-01f};

constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Multiply by exp(S 2 pi i m / 32) with m a compile-time constant after unrolling.
template <int S>
__device__ __forceinline__ float2 rot32(float2 a, int m) {
  if (m == 0) return a;
  if (m == 8) return S > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
  const float c = kCos32[m], s = (float)S * kSin32[m];
  return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// In-place R-point DFT of v[0..R-1] (R = 2..32) by decimation in time: input
// point r is held in register in_reg(r) = bitrev(r), output X[q] in register
// out_reg(q) = q.  Working in place keeps the register footprint at the R points
// themselves.  A butterfly of length 2h takes a and b w (w = W_{2h}^j):
//   a' = a + b w in four FMAs, b' = a - b w = 2 a - a' in two,
// instead of a + b, a - b and a complex product (eight instructions); w = 1 and
// w = +-i are additions only.
template <int R, int S>
__device__ __forceinline__ void dft_reg(float2* v) {
#pragma unroll
  for (int h = 1; h < R; h <<= 1) {  // butterflies of length 2h
#pragma unroll
    for (int i = 0; i < R; i += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const float2 a = v[i + j], b = v[i + j + h];
        const int m = j * (16 / h);  // W_{2h}^j = W_32^m
        if (m == 0 || m == 8) {
          const float2 t = rot32<S>(b, m);
          v[i + j] = cadd(a, t);
          v[i + j + h] = csub(a, t);
        } else {
          const float c = kCos32[m], s = (float)S * kSin32[m];
          const float2 o = make_float2(fmaf(b.x, c, fmaf(-b.y, s, a.x)), fmaf(b.x, s, fmaf(b.y, c, a.y)));
          v[i + j] = o;
          v[i + j + h] = make_float2(fmaf(2.f, a.x, -o.x), fmaf(2.f, a.y, -o.y));
        }
      }
    }
  }
}

// Register that holds DFT input point r before dft_reg<R>, and output q after it.
template <int R>
__device__ __forceinline__ constexpr int in_reg(int r) { return bitrev(r, ilog2(R)); }
template <int R>
__device__ __forceinline__ constexpr int out_reg(int q) { return q; }

// Radix plan per transform length: P points per thread, passes of radix R[i].
template <int LOGN_, int P_, int NP_, int R0, int R1, int R2, int R3 = 1>
struct PlanDef {
  static constexpr int LOGN = LOGN_, P = P_, NP = NP_;
  static constexpr int R[4] = {R0, R1, R2, R3};
};
template <int LOGN> struct Plan;
template <> struct Plan<8> : PlanDef<8, 16, 2, 16, 16, 1> {};
template <> struct Plan<9> : PlanDef<9, 16, 3, 16, 16, 2> {};
template <> struct Plan<10> : PlanDef<10, 16, 3, 16, 16, 4> {};
template <> struct Plan<11> : PlanDef<11, 16, 3, 16, 16, 8> {};
template <> struct Plan<12> : PlanDef<12, 16, 3, 16, 16, 16> {};
// 2^13 and 2^14 as three passes of 32 points per thread (256 and 512 threads):
// measured 7-10 % faster per point than four passes of 16 (two or more
// workgroups share a CU either way).
template <> struct Plan<13> : PlanDef<13, 32, 3, 32, 32, 8> {};
template <> struct Plan<14> : PlanDef<14, 32, 3, 32, 32, 16> {};
template <> struct Plan<15> : PlanDef<15, 64, 3, 32, 32, 32> {};
// 32768 points over 1024 threads of 32 points: four waves per SIMD at 128 VGPRs
// instead of two at ~205, for kernels whose register use allows it.
struct Plan15Wide : PlanDef<15, 32, 3, 32, 32, 32> {};

template <class PL> struct Geo {
  static constexpr int N = 1 << PL::LOGN;
  static constexpr int P = PL::P;
  static constexpr int T = N / P;  // threads per workgroup
  static constexpr int NP = PL::NP;
  static constexpr int R0 = PL::R[0];
  static constexpr int RL = PL::R[NP - 1];
  // LDS floats for one half-exchange (one pad word per 32 against bank conflicts)
  static constexpr int LDS_FLOATS = N + N / 32;
  // Twiddles of the second pass (stride R0, radix R1) from a table in LDS when it
  // costs at most two entries per thread to fill: TAB[r][k] = exp(S 2 pi i r k /
  // (R0 R1)), r < R1, k < R0, placed after the exchange area.
  static constexpr bool TABLE = NP >= 2 && PL::R[0] * PL::R[1] <= 2 * T;
  static constexpr int TAB_FLOATS = TABLE ? 2 * PL::R[0] * PL::R[1] : 0;
  static constexpr int LDS_TOTAL = LDS_FLOATS + TAB_FLOATS;  // floats a launch must provide
};

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 5); }

// Exchange through LDS between a pass of radix R at stride NS and the next of radix R2.
// Addresses are written as a per-thread base plus compile-time offsets, split into
// segments below 64 KB so that every access uses the instruction's immediate offset
// instead of a register of its own.
template <int STRIDE>  // offset r * STRIDE floats, segments of at most 16383 floats
__device__ __forceinline__ float* lds_seg(float* base, int r) {
  constexpr int SEG = STRIDE >= 16384 ? 1 : 16383 / STRIDE + 1;
  return base + (r / SEG) * SEG * STRIDE;
}

template <class PL, int R, int NS, int R2>
__device__ __forceinline__ void exchange(float2* v, float* lds, int t) {
  using G = Geo<PL>;
  // writes: output q of butterfly j goes to (j / NS) NS R + k + q NS
  constexpr bool WLIN = (NS % 32 == 0) || (NS * R <= 32 && 32 % (NS * R) == 0) || (NS == 1 && R % 32 == 0);
  // reads: point r of the next pass is t + u T + r N / R2
  constexpr int RSTR = G::N / R2;
  constexpr bool RLIN = RSTR % 32 == 0;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
#pragma unroll
    for (int u = 0; u < G::P / R; ++u) {
      const int j = t + u * G::T;
      const int k = j & (NS - 1);
      const int base = (j / NS) * NS * R + k;
      float* wb = lds + lds_pad(base);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const float2 o = v[u * R + out_reg<R>(q)];
        const float val = half ? o.y : o.x;
        if constexpr (WLIN) {
          constexpr int WSTR = NS + NS / 32;
          lds_seg<WSTR>(wb, q)[(q % (WSTR >= 16384 ? 1 : 16383 / WSTR + 1)) * WSTR] = val;
        } else {
          lds[lds_pad(base + q * NS)] = val;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < G::P / R2; ++u) {
      float* rb = lds + lds_pad(t + u * G::T);
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        float val;
        if constexpr (RLIN) {
          constexpr int STR = RSTR + RSTR / 32;
          val = lds_seg<STR>(rb, r)[(r % (STR >= 16384 ? 1 : 16383 / STR + 1)) * STR];
        } else {
          val = lds[lds_pad(t + u * G::T + r * RSTR)];
        }
        if (half) v[u * R2 + in_reg<R2>(r)].y = val; else v[u * R2 + in_reg<R2>(r)].x = val;
      }
    }
    __syncthreads();
  }
}

// A zero the compiler cannot see through, computed after `dep`: indices offset by
// it cannot be hoisted above the work that produced `dep` (empty asm, no code).
__device__ __forceinline__ int opaque_zero(float dep) {
  int z = 0;
  asm volatile("; opaque %1" : "+v"(z) : "v"(dep));
  return z;
}

// Force the R values of a butterfly group to be fully computed at this point
// (empty asm, no code), so that later work ordered after it does not overlap it.
template <int R>
__device__ __forceinline__ void pin_regs(float2* v) {
#pragma unroll
  for (int i = 0; i < R; ++i) asm volatile("; pin %0 %1" : "+v"(v[i].x), "+v"(v[i].y));
}

// Apply the twiddles exp(S 2 pi i r k / 2^LOGD), r = 1..R-1, to one butterfly group.
// Powers w^1..w^7 of w = exp(S 2 pi i k / 2^LOGD) come from products of the exact
// w^1 (depth <= 3); every eighth power w^{8a} is exact again and w^{8a+b} =
// w^{8a} w^b, so no twiddle is more than four roundings from exact while only
// R/8 of them need the transcendental unit.
template <int LOGD, int R, int S>
__device__ __forceinline__ void apply_twiddles(float2* v, int k) {
  const float2 w1 = twiddle<LOGD, S>(k);
  float2 wb[8];
  wb[1] = w1;
  if constexpr (R > 2) {
    wb[2] = cmul(w1, w1);
    wb[3] = cmul(wb[2], w1);
  }
  if constexpr (R > 4) {
    wb[4] = cmul(wb[2], wb[2]);
    wb[5] = cmul(wb[4], w1);
    wb[6] = cmul(wb[3], wb[3]);
    wb[7] = cmul(wb[6], w1);
  }
  constexpr int B = R < 8 ? R : 8;
#pragma unroll
  for (int b = 1; b < B; ++b) v[in_reg<R>(b)] = cmul(v[in_reg<R>(b)], wb[b]);
#pragma unroll
  for (int a = 1; a < R / 8; ++a) {
    // 8 a k < 2^LOGD (k < 2^LOGD / R): exact anchor
    const float2 wa = twiddle<LOGD, S>(8 * a * k);
    v[in_reg<R>(8 * a)] = cmul(v[in_reg<R>(8 * a)], wa);
#pragma unroll
    for (int b = 1; b < 8; ++b) v[in_reg<R>(8 * a + b)] = cmul(v[in_reg<R>(8 * a + b)], cmul(wa, wb[b]));
  }
}

template <class PL, int R, int NS, int S>
__device__ __forceinline__ void pass(float2* v, int t) {
  using G = Geo<PL>;
  constexpr int LOGD = ilog2(NS * R);
  int z = 0;
#pragma unroll
  for (int u = 0; u < G::P / R; ++u) {
    if (NS > 1) apply_twiddles<LOGD, R, S>(v + u * R, (t + z + u * G::T) & (NS - 1));
    dft_reg<R, S>(v + u * R);
    // the next group's twiddles wait for this group's butterflies (register pressure)
    if (u + 1 < G::P / R) {
      pin_regs<R>(v + u * R);
      z = opaque_zero(v[u * R].x);
    }
  }
}

// Fill the second pass's twiddle table (Geo::TABLE): entry r NS + k, NS = R0, is
// exp(S 2 pi i r k / (NS R)) from its exactly reduced angle, so every twiddle of
// that pass carries one rounding of the transcendental unit instead of up to four
// from products.  Made visible by the first exchange's barrier.
template <class PL, int S>
__device__ __forceinline__ void fill_twiddle_table(float* lds, int t) {
  using G = Geo<PL>;
  constexpr int NS = PL::R[0], R = PL::R[1], E = NS * R;
  float2* tab = reinterpret_cast<float2*>(lds + G::LDS_FLOATS);
#pragma unroll
  for (int e = 0; e < (E + G::T - 1) / G::T; ++e) {
    const int i = t + e * G::T;
    if (E % G::T == 0 || i < E) tab[i] = twiddle<ilog2(E), S>((i / NS) * (i % NS));
  }
}

// The second pass with its twiddles read from the table (stride NS = R0).
template <class PL, int R, int NS, int S>
__device__ __forceinline__ void pass_table(float2* v, const float* lds, int t) {
  using G = Geo<PL>;
  const float2* tab = reinterpret_cast<const float2*>(lds + G::LDS_FLOATS);
  int z = 0;
#pragma unroll
  for (int u = 0; u < G::P / R; ++u) {
    const float2* row = tab + ((t + z + u * G::T) & (NS - 1));
#pragma unroll
    for (int r = 1; r < R; ++r) v[u * R + in_reg<R>(r)] = cmul(v[u * R + in_reg<R>(r)], row[r * NS]);
    dft_reg<R, S>(v + u * R);
    if (u + 1 < G::P / R) {
      pin_regs<R>(v + u * R);
      z = opaque_zero(v[u * R].x);
    }
  }
}

// Passes 1.. of the transform (pass 0 is done by the caller, fused with its loads).
template <class PL, int S, int PASS, int NS>
struct Passes {
  __device__ __forceinline__ static void run(float2* v, float* lds, int t) {
    constexpr int RP = PL::R[PASS - 1];
    constexpr int R = PL::R[PASS];
    exchange<PL, RP, NS / RP, R>(v, lds, t);
    if constexpr (PASS == 1 && Geo<PL>::TABLE) pass_table<PL, R, NS, S>(v, lds, t);
    else pass<PL, R, NS, S>(v, t);
    if constexpr (PASS + 1 < PL::NP) Passes<PL, S, PASS + 1, NS * R>::run(v, lds, t);
  }
};

// Full transform.  load(i) supplies input point i; the first pass runs group by
// group as its points arrive.  On return output t + u T + q N / RL is in register
// u RL + out_reg<RL>(q).
template <class PL, int S, class Load>
__device__ __forceinline__ void fft_workgroup(float2* v, float* lds, int t, Load load) {
  using G = Geo<PL>;
  if constexpr (G::TABLE) fill_twiddle_table<PL, S>(lds, t);
  int z = 0;
#pragma unroll
  for (int u = 0; u < G::P / G::R0; ++u) {
#pragma unroll
    for (int r = 0; r < G::R0; ++r) v[u * G::R0 + in_reg<G::R0>(r)] = load(t + z + u * G::T + r * (G::N / G::R0));
    dft_reg<G::R0, S>(v + u * G::R0);
    // loads of the next group wait for this group's butterflies (register pressure)
    if (u + 1 < G::P / G::R0) {
      pin_regs<G::R0>(v + u * G::R0);
      z = opaque_zero(v[u * G::R0].x);
    }
  }
  if constexpr (G::NP > 1) Passes<PL, S, 1, G::R0>::run(v, lds, t);
}

}  // namespace ddx
