// Device-side arithmetic shared by the sweep, init and batch kernels (gfx950).
//
// Every floating-point step is spelled out (explicit fused multiply-adds, the
// library is built with -ffp-contract=off, division and square root correctly
// rounded), so that a site update is a fixed function of its inputs and random
// draws: the GPU result is reproducible bit for bit across launch shapes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsg {

// Philox stream tags: fourth word of the counter.
enum : uint32_t { kTagMetropolis = 0, kTagInitSpin = 1, kTagInitJ = 2, kTagSwap = 3,
                  kTagHeatBath = 5 };

struct Word4 {
  uint32_t w0, w1, w2, w3;
};

// a ^ b ^ c as one vector instruction (v_bitop3_b32 with the truth table of a
// three-way exclusive or).  Worth it only when two operands are per-lane values: a
// wave-uniform pair is folded on the scalar unit first, for one vector xor.
__device__ __forceinline__ uint32_t xor3_v(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon et al., SC'11).  Each round takes two 32x32->64 products
// of counter words 0 and 2 with the round multipliers and mixes their halves with
// words 1 and 3 and the key; the key advances by the Weyl constants between rounds.
// Callers put the only per-lane word (the site) in word 1 and wave-uniform values in
// words 0, 2, 3 and the key: the products of the first rounds then stay on the
// scalar unit, and the mixing xors of the first rounds have a uniform pair.  From
// round 3 (word 1's mix) and round 4 (word 3's) on, both non-key operands are per-lane.
__device__ __forceinline__ Word4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t a = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
    const uint32_t n0 = round >= 3 ? xor3_v((uint32_t)(b >> 32), c1, k0)
                                   : (uint32_t)(b >> 32) ^ c1 ^ k0;
    const uint32_t n2 = round >= 4 ? xor3_v((uint32_t)(a >> 32), c3, k1)
                                   : (uint32_t)(a >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)b;
    c3 = (uint32_t)a;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Word4{c0, c1, c2, c3};
}

// NB Philox4x32-10 blocks whose counters differ only in word 2, advanced round by round
// together: each block's arithmetic is philox10's, and the NB independent chains of
// dependent products are interleaved in the instruction stream (latency hiding for a
// wave that has few others beside it on its SIMD).
template <int NB>
__device__ __forceinline__ void philox10_n(uint32_t c0, uint32_t c1, const uint32_t (&c2)[NB],
                                           uint32_t c3, uint32_t k0, uint32_t k1,
                                           Word4 (&out)[NB]) {
  uint32_t w0[NB], w1[NB], w2[NB], w3[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    w0[i] = c0;
    w1[i] = c1;
    w2[i] = c2[i];
    w3[i] = c3;
  }
#pragma unroll
  for (int round = 0; round < 10; ++round) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const uint64_t a = (uint64_t)w0[i] * 0xD2511F53u;
      const uint64_t b = (uint64_t)w2[i] * 0xCD9E8D57u;
      const uint32_t n0 = round >= 3 ? xor3_v((uint32_t)(b >> 32), w1[i], k0)
                                     : (uint32_t)(b >> 32) ^ w1[i] ^ k0;
      const uint32_t n2 = round >= 4 ? xor3_v((uint32_t)(a >> 32), w3[i], k1)
                                     : (uint32_t)(a >> 32) ^ w3[i] ^ k1;
      w1[i] = (uint32_t)b;
      w3[i] = (uint32_t)a;
      w0[i] = n0;
      w2[i] = n2;
    }
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) out[i] = Word4{w0[i], w1[i], w2[i], w3[i]};
}

// Uniform in (0,1): the top 23 bits of w as an odd multiple of 2^-24.  Exact in
// binary32 and binary64 (the same value in both precisions).
template <typename R>
__device__ __forceinline__ R odd_part(uint32_t w) {
  return (R)(((w >> 9) << 1) | 1u);  // < 2^24, exactly representable
}
// f = 1 + m 2^-23 for the top 23 bits m of w: the exponent field of 1.0 funnel-shifted
// in above them, one v_alignbit_b32.  The binary32 forms below derive every uniform of
// a hit from f exactly; they give the same bits as the integer-conversion route.
__device__ __forceinline__ float one_plus_top23(uint32_t w) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9u));
}

template <typename R>
__device__ __forceinline__ R unit_uniform(uint32_t w) {
  return odd_part<R>(w) * (R)0x1p-24;
}
// u = (2m + 1) 2^-24 = f - (1 - 2^-24): both operands in [1/2, 2], so exact (Sterbenz).
template <>
__device__ __forceinline__ float unit_uniform<float>(uint32_t w) {
  return one_plus_top23(w) - 0x1.fffffep-1f;
}

template <typename R>
struct Trig;

// sin/cos(pi r / 2) on r in [-1/2, 1/2]: Taylor polynomials in r (correctly rounded
// coefficients (+-)(pi/2)^k / k!), Horner with fused multiply-adds.
template <>
struct Trig<float> {
  __device__ __forceinline__ static void eval(float r, float& s, float& c) {
    const float r2 = r * r;
    float p = 0x1.507834p-13f;          // r^9
    p = fmaf(p, r2, -0x1.32d2ccp-8f);   // r^7
    p = fmaf(p, r2, 0x1.466bc6p-4f);    // r^5
    p = fmaf(p, r2, -0x1.4abbcep-1f);   // r^3
    p = fmaf(p, r2, 0x1.921fb6p+0f);    // r^1
    s = p * r;
    float q = -0x1.a6d1f2p-16f;         // r^10
    q = fmaf(q, r2, 0x1.e1f506p-11f);   // r^8
    q = fmaf(q, r2, -0x1.55d3c8p-6f);   // r^6
    q = fmaf(q, r2, 0x1.03c1f0p-2f);    // r^4
    q = fmaf(q, r2, -0x1.3bd3ccp+0f);   // r^2
    c = fmaf(q, r2, 1.0f);              // r^0
  }
};

template <>
struct Trig<double> {
  __device__ __forceinline__ static void eval(double r, double& s, double& c) {
    const double r2 = r * r;
    double p = 0x1.aaec32af93359p-38;      // r^17
    p = fma(p, r2, -0x1.6fadb9f155744p-31);  // r^15
    p = fma(p, r2, 0x1.e8f434d018d63p-25);   // r^13
    p = fma(p, r2, -0x1.e3074fde8871fp-19);  // r^11
    p = fma(p, r2, 0x1.50783487ee782p-13);   // r^9
    p = fma(p, r2, -0x1.32d2cce62bd86p-8);   // r^7
    p = fma(p, r2, 0x1.466bc6775aae2p-4);    // r^5
    p = fma(p, r2, -0x1.4abbce625be53p-1);   // r^3
    p = fma(p, r2, 0x1.921fb54442d18p+0);    // r^1
    s = p * r;
    double q = 0x1.20c62c2f2d7f5p-34;       // r^16
    q = fma(q, r2, -0x1.b6e24f44b128fp-28);  // r^14
    q = fma(q, r2, 0x1.f9d38a3763cc3p-22);   // r^12
    q = fma(q, r2, -0x1.a6d1f2a204a8cp-16);  // r^10
    q = fma(q, r2, 0x1.e1f506891babbp-11);   // r^8
    q = fma(q, r2, -0x1.55d3c7e3cbffap-6);   // r^6
    q = fma(q, r2, 0x1.03c1f081b5ac4p-2);    // r^4
    q = fma(q, r2, -0x1.3bd3cc9be45dep+0);   // r^2
    c = fma(q, r2, 1.0);                     // r^0
  }
};

__device__ __forceinline__ float dev_fma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double dev_fma(double a, double b, double c) { return fma(a, b, c); }
// sqrtf is correctly rounded under -fhip-fp32-correctly-rounded-divide-sqrt (the
// residual-checked expansion around v_sqrt_f32); __fsqrt_rn is not on this toolchain.
__device__ __forceinline__ float dev_sqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double dev_sqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float dev_div(float a, float b) { return __fdiv_rn(a, b); }
__device__ __forceinline__ double dev_div(double a, double b) { return __ddiv_rn(a, b); }
__device__ __forceinline__ float dev_rint(float a) { return rintf(a); }
__device__ __forceinline__ double dev_rint(double a) { return rint(a); }

// Own exp, expm1, log and log1p for the heat-bath draw and the Gaussian couplings: a
// fixed sequence of correctly rounded operations, so that results do not depend on a
// math library's last bits.  Methods:
//  - exp, expm1 on [kXMin, 0]: Cody and Waite's reduction (Software Manual for the
//    Elementary Functions, 1980), x = k ln2 + r with |r| <= ln2/2 and ln 2 split into a
//    head (a multiple of 2^-16 in binary32, 2^-32 in binary64, so k * head is exact) and
//    a tail; expm1(r) = r + r^2 (1/2! + r (1/3! + ...)) (Taylor, to r^8 / r^13);
//    exp(x) = 2^k (1 + expm1(r)), expm1(x) = 2^k expm1(r) + (2^k - 1), one rounding
//    each.  Smaller inputs are raised to kXMin (the results stay normal).
//  - log on normal positive x: x = 2^e m, m in [sqrt(1/2), sqrt(2)),
//    log x = e ln2 + 2 atanh((m - 1) / (m + 1)); log1p on |x| <= 1/2: 2 atanh(x / (2 + x));
//    2 atanh(f) = 2f + 2f f^2 (1/3 + f^2 (1/5 + ...)) (Taylor, to f^15 / f^35).
// Coefficients: 1/n! and 1/(2j+1) correctly rounded.  Within 2 ulp of the true values.
template <typename R>
struct Elem;

template <>
struct Elem<float> {
  static constexpr float kXMin = -80.0f;
  static constexpr float kLn2Hi = 0x1.62e4p-1f, kLn2Lo = 0x1.7f7d1cp-20f;
  static constexpr float kLog2e = 0x1.715476p+0f, kSqrtHalf = 0x1.6a09e6p-1f;
  __device__ __forceinline__ static float expm1_poly(float r) {  // sum_{n>=2} r^(n-2)/n!
    float q = 0x1.a01a02p-16f;       // 1/8!
    q = fmaf(q, r, 0x1.a01a02p-13f);  // 1/7!
    q = fmaf(q, r, 0x1.6c16c2p-10f);  // 1/6!
    q = fmaf(q, r, 0x1.111112p-7f);   // 1/5!
    q = fmaf(q, r, 0x1.555556p-5f);   // 1/4!
    q = fmaf(q, r, 0x1.555556p-3f);   // 1/3!
    return fmaf(q, r, 0x1p-1f);       // 1/2!
  }
  __device__ __forceinline__ static float atanh_poly(float s) {  // sum_{j>=1} s^(j-1)/(2j+1)
    float q = 0x1.111112p-4f;         // 1/15
    q = fmaf(q, s, 0x1.3b13b2p-4f);   // 1/13
    q = fmaf(q, s, 0x1.745d18p-4f);   // 1/11
    q = fmaf(q, s, 0x1.c71c72p-4f);   // 1/9
    q = fmaf(q, s, 0x1.24924ap-3f);   // 1/7
    q = fmaf(q, s, 0x1.99999ap-3f);   // 1/5
    return fmaf(q, s, 0x1.555556p-2f);  // 1/3
  }
  __device__ __forceinline__ static float frexp_(float x, int& e) { return frexpf(x, &e); }
  __device__ __forceinline__ static float ldexp_(float x, int e) { return ldexpf(x, e); }
};

template <>
struct Elem<double> {
  static constexpr double kXMin = -700.0;
  static constexpr double kLn2Hi = 0x1.62e42ffp-1, kLn2Lo = -0x1.718432a1b0e26p-35;
  static constexpr double kLog2e = 0x1.71547652b82fep+0, kSqrtHalf = 0x1.6a09e667f3bcdp-1;
  __device__ __forceinline__ static double expm1_poly(double r) {
    double q = 0x1.6124613a86d09p-33;   // 1/13!
    q = fma(q, r, 0x1.1eed8eff8d898p-29);  // 1/12!
    q = fma(q, r, 0x1.ae64567f544e4p-26);  // 1/11!
    q = fma(q, r, 0x1.27e4fb7789f5cp-22);  // 1/10!
    q = fma(q, r, 0x1.71de3a556c734p-19);  // 1/9!
    q = fma(q, r, 0x1.a01a01a01a01ap-16);  // 1/8!
    q = fma(q, r, 0x1.a01a01a01a01ap-13);  // 1/7!
    q = fma(q, r, 0x1.6c16c16c16c17p-10);  // 1/6!
    q = fma(q, r, 0x1.1111111111111p-7);   // 1/5!
    q = fma(q, r, 0x1.5555555555555p-5);   // 1/4!
    q = fma(q, r, 0x1.5555555555555p-3);   // 1/3!
    return fma(q, r, 0x1p-1);              // 1/2!
  }
  __device__ __forceinline__ static double atanh_poly(double s) {
    double q = 0x1.d41d41d41d41dp-6;     // 1/35
    q = fma(q, s, 0x1.f07c1f07c1f08p-6);  // 1/33
    q = fma(q, s, 0x1.0842108421084p-5);  // 1/31
    q = fma(q, s, 0x1.1a7b9611a7b96p-5);  // 1/29
    q = fma(q, s, 0x1.2f684bda12f68p-5);  // 1/27
    q = fma(q, s, 0x1.47ae147ae147bp-5);  // 1/25
    q = fma(q, s, 0x1.642c8590b2164p-5);  // 1/23
    q = fma(q, s, 0x1.8618618618618p-5);  // 1/21
    q = fma(q, s, 0x1.af286bca1af28p-5);  // 1/19
    q = fma(q, s, 0x1.e1e1e1e1e1e1ep-5);  // 1/17
    q = fma(q, s, 0x1.1111111111111p-4);  // 1/15
    q = fma(q, s, 0x1.3b13b13b13b14p-4);  // 1/13
    q = fma(q, s, 0x1.745d1745d1746p-4);  // 1/11
    q = fma(q, s, 0x1.c71c71c71c71cp-4);  // 1/9
    q = fma(q, s, 0x1.2492492492492p-3);  // 1/7
    q = fma(q, s, 0x1.999999999999ap-3);  // 1/5
    return fma(q, s, 0x1.5555555555555p-2);  // 1/3
  }
  __device__ __forceinline__ static double frexp_(double x, int& e) { return frexp(x, &e); }
  __device__ __forceinline__ static double ldexp_(double x, int e) { return ldexp(x, e); }
};

// exp(x) = scale (1 + p), scale = 2^k, for x in [kXMin, 0] (smaller x raised to kXMin).
template <typename R>
__device__ __forceinline__ void own_exp_parts(R x, R& scale, R& p) {
  using E = Elem<R>;
  x = x < E::kXMin ? E::kXMin : x;
  const R k = dev_rint(x * E::kLog2e);
  R r = dev_fma(-k, E::kLn2Hi, x);
  r = dev_fma(-k, E::kLn2Lo, r);
  p = dev_fma(r * r, E::expm1_poly(r), r);
  scale = E::ldexp_((R)1, (int)k);
}
template <typename R>
__device__ __forceinline__ R own_exp(R x) {
  R scale, p;
  own_exp_parts(x, scale, p);
  return dev_fma(scale, p, scale);
}
template <typename R>
__device__ __forceinline__ R own_expm1(R x) {
  R scale, p;
  own_exp_parts(x, scale, p);
  return dev_fma(scale, p, scale - (R)1);
}
// 2 atanh(f), |f| <= 1/3.
template <typename R>
__device__ __forceinline__ R own_atanh2(R f) {
  const R s = f * f, t = f + f;
  return dev_fma(t * s, Elem<R>::atanh_poly(s), t);
}
template <typename R>
__device__ __forceinline__ R own_log1p(R x) {  // |x| <= 1/2
  return own_atanh2(dev_div(x, (R)2 + x));
}
template <typename R>
__device__ __forceinline__ R own_log(R x) {  // x positive and normal
  using E = Elem<R>;
  int e;
  R m = E::frexp_(x, e);  // m in [1/2, 1)
  if (m < E::kSqrtHalf) {
    m = m + m;
    e -= 1;
  }
  const R lm = own_atanh2(dev_div(m - (R)1, m + (R)1));
  const R ef = (R)e;
  return dev_fma(ef, E::kLn2Hi, dev_fma(ef, E::kLn2Lo, lm));
}

// Metropolis acceptance exp(x) for x = -beta dE.  Binary32 uses the hardware 2^y
// (v_exp_f32, within 1 ulp) at y = x log2(e): the result is within 2e-8 of exp(x)
// everywhere it can matter (y*2^y is at most 0.53 times the 4e-8 rounding of y), far
// inside the 1e-6 band in which decisions are flagged as too close to call.
__device__ __forceinline__ float accept_prob(float x) {
  return __builtin_amdgcn_exp2f(x * 0x1.715476p+0f);
}
__device__ __forceinline__ double accept_prob(double x) { return exp(x); }

// (sin, cos) of 2 pi u for an exact uniform u.  t = 4u splits exactly into its
// nearest integer q (t is never a half-integer) and r = t - q, 2 pi u = (pi/2)(q + r);
// the quadrant q mod 4 rotates (sin, cos) of (pi/2) r.
template <typename R>
__device__ __forceinline__ void sincos_2pi_t(R t, R& s_out, R& c_out);

template <typename R>
__device__ __forceinline__ void sincos_2pi(R u, R& s_out, R& c_out) {
  sincos_2pi_t(u * (R)4, s_out, c_out);
}

// Same, given t = 4u.
template <typename R>
__device__ __forceinline__ void sincos_2pi_t(R t, R& s_out, R& c_out) {
  const R q = dev_rint(t);
  const R r = t - q;
  R s, c;
  Trig<R>::eval(r, s, c);
  const int quadrant = ((int)q) & 3;
  const R cq = (quadrant & 1) ? s : c;  // quadrants 1, 3 exchange the pair
  const R sq = (quadrant & 1) ? c : s;
  c_out = (quadrant == 1 || quadrant == 2) ? -cq : cq;
  s_out = (quadrant >= 2) ? -sq : sq;
}

// Binary32: the quadrant rotation on the bit patterns, with three-input bitwise
// operations (v_bitop3_b32; the truth-table byte is the function applied to the
// operand masks 0xF0, 0xCC, 0xAA).  Bit 0 of q exchanges the pair (select on a
// 0 / all-ones mask, table 0xCA = a ? b : c); bit 1 of q flips the sign of sin and
// bit 1 of q + 1 the sign of cos (table 0x6A = (a & b) ^ c on the sign bit).
template <>
__device__ __forceinline__ void sincos_2pi_t<float>(float t, float& s_out, float& c_out) {
  const float q = rintf(t);
  const float r = t - q;
  float s, c;
  Trig<float>::eval(r, s, c);
  const int32_t qi = (int32_t)q;
  const uint32_t odd = (uint32_t)__builtin_amdgcn_sbfe(qi, 0, 1);  // 0 or ~0
  const uint32_t sb = __float_as_uint(s), cb = __float_as_uint(c);
  const uint32_t sq = __builtin_amdgcn_bitop3_b32(odd, cb, sb, 0xCA);  // odd: sin <- cos
  const uint32_t cq = __builtin_amdgcn_bitop3_b32(odd, sb, cb, 0xCA);
  s_out = __uint_as_float(__builtin_amdgcn_bitop3_b32((uint32_t)qi << 30, 0x80000000u, sq, 0x6A));
  c_out = __uint_as_float(
      __builtin_amdgcn_bitop3_b32((uint32_t)(qi + 1) << 30, 0x80000000u, cq, 0x6A));
}

template <typename R>
struct Vec3 {
  R x, y, z;
};

template <typename R>
__device__ __forceinline__ R dot3(const Vec3<R>& a, const Vec3<R>& b) {
  return dev_fma(a.z, b.z, dev_fma(a.y, b.y, a.x * b.x));
}

// Point uniform on the unit sphere: z = 2 u0 - 1 is uniform on [-1, 1] (exact),
// the azimuth 2 pi u1 is uniform and independent, rho = sqrt(1 - z^2) rounded once
// inside the root.
template <typename R>
__device__ __forceinline__ Vec3<R> sphere_point(R u0, R u1) {
  const R z = (R)2 * u0 - (R)1;
  const R rho = dev_sqrt(dev_fma(-z, z, (R)1));
  R s, c;
  sincos_2pi(u1, s, c);
  return Vec3<R>{rho * c, rho * s, z};
}

// The same point straight from two Philox words: with u = odd * 2^-24 exact, both
// 2u - 1 = odd * 2^-23 - 1 and 4u = odd * 2^-22 are exact, so folding the scale
// into one operation gives identical bits.
// Correctly rounded square root of a positive normal binary32 x: the hardware root
// (within 1 ulp) is moved to its neighbour when the residual x - r*r of the neighbour
// shows that neighbour is the nearer root.  sqrtf performs the same steps plus
// scaling for denormal and special inputs, which the sphere point never produces
// (there 1 - z^2 >= 2^-22).
__device__ __forceinline__ float sqrt_rn_normal(float x) {
  const float r = __builtin_amdgcn_sqrtf(x);
  const float down = __uint_as_float(__float_as_uint(r) - 1u);
  const float up = __uint_as_float(__float_as_uint(r) + 1u);
  float out = fmaf(-down, r, x) <= 0.0f ? down : r;
  out = fmaf(-up, r, x) > 0.0f ? up : out;
  return out;
}
__device__ __forceinline__ double sqrt_rn_normal(double x) { return sqrt(x); }

template <typename R>
__device__ __forceinline__ Vec3<R> sphere_point_words(uint32_t w0, uint32_t w1) {
  const R z = dev_fma(odd_part<R>(w0), (R)0x1p-23, (R)-1);
  const R rho = sqrt_rn_normal(dev_fma(-z, z, (R)1));
  R s, c;
  sincos_2pi_t(odd_part<R>(w1) * (R)0x1p-22, s, c);
  return Vec3<R>{rho * c, rho * s, z};
}
// Binary32: with f = 1 + m 2^-23 from each word, 2u - 1 = (2f - 2) - (1 - 2^-23) (the
// product-difference m 2^-22 is exact, and so is the difference, a multiple of 2^-23
// below 1 in magnitude) and 4u = 4f - (4 - 2^-22) in one exact fused multiply-add.
template <>
__device__ __forceinline__ Vec3<float> sphere_point_words<float>(uint32_t w0, uint32_t w1) {
  const float z = fmaf(one_plus_top23(w0), 2.0f, -2.0f) - 0x1.fffffcp-1f;
  const float rho = sqrt_rn_normal(fmaf(-z, z, 1.0f));
  float s, c;
  sincos_2pi_t(fmaf(one_plus_top23(w1), 4.0f, -0x1.fffffep+1f), s, c);
  return Vec3<float>{rho * c, rho * s, z};
}

// Exact draw from the conditional law exp(beta sigma.h) on the sphere.  With
// a = beta |h|, w = 1 - u0 and q = 1 - e^{-2a}, the cosine to the field is
// c = 1 + log(1 - w q)/a, evaluated as log1p(-w q) while w q <= 1/2 and as
// log(u0 + w e^{-2a}) (one fused multiply-add, no cancellation) above (the own exp,
// expm1, log and log1p above); c = 2 u0 - 1 for a = 0.  The azimuth is 2 pi u1, and the tangent frame about n = h/|h| is the
// branch-free orthonormal basis of Duff et al. (JCGT 2017).
template <typename R>
__device__ __forceinline__ Vec3<R> heat_bath_point(const Vec3<R>& h, R beta, R u0, R u1) {
  const R hh = dot3(h, h);
  const R hn = dev_sqrt(hh);
  const R a = beta * hn;
  R c;
  if (a > (R)0) {
    const R w = (R)1 - u0;
    const R wq = w * -own_expm1((R)-2 * a);
    const R lg = wq <= (R)0.5 ? own_log1p(-wq) : own_log(dev_fma(w, own_exp((R)-2 * a), u0));
    c = (R)1 + dev_div(lg, a);
  } else {
    c = (R)2 * u0 - (R)1;
  }
  c = c > (R)1 ? (R)1 : c;
  c = c < (R)-1 ? (R)-1 : c;
  const R rho = dev_sqrt(dev_fma(-c, c, (R)1));
  R sn, cs;
  sincos_2pi(u1, sn, cs);
  if (!(hh > (R)0)) return Vec3<R>{rho * cs, rho * sn, c};
  const Vec3<R> n{dev_div(h.x, hn), dev_div(h.y, hn), dev_div(h.z, hn)};
  const R sgn = n.z >= (R)0 ? (R)1 : (R)-1;
  const R ia = dev_div((R)-1, sgn + n.z);
  const R b = n.x * n.y * ia;
  const Vec3<R> e1{dev_fma(sgn * n.x * n.x, ia, (R)1), sgn * b, -sgn * n.x};
  const Vec3<R> e2{b, dev_fma(n.y * n.y, ia, sgn), -n.y};
  const R px = rho * cs, py = rho * sn;
  return Vec3<R>{dev_fma(c, n.x, dev_fma(px, e1.x, py * e2.x)),
                 dev_fma(c, n.y, dev_fma(px, e1.y, py * e2.y)),
                 dev_fma(c, n.z, dev_fma(px, e1.z, py * e2.z))};
}

// Reflection of s about the field direction (over-relaxation): the largest move
// that keeps -s.h; a zero field leaves s unchanged.
template <typename R>
__device__ __forceinline__ Vec3<R> reflect(const Vec3<R>& s, const Vec3<R>& h) {
  const R hh = dot3(h, h);
  const R sh = dot3(s, h);
  const R f = dev_div(sh + sh, hh);
  const bool ok = hh > (R)0;
  return Vec3<R>{ok ? dev_fma(f, h.x, -s.x) : s.x, ok ? dev_fma(f, h.y, -s.y) : s.y,
                 ok ? dev_fma(f, h.z, -s.z) : s.z};
}

// A double moved between lanes by one DPP control (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum of a double across the 64 lanes of a wavefront (every lane ends with the same
// value).  Within rows of 16 lanes the exchanges are DPP moves: quad_perm [1,0,3,2]
// (lane ^ 1) and [2,3,0,1] (lane ^ 2), after which the four lanes of a quad hold the
// same bits (addition commutes), so the row half-mirror (lane i with 7 - i) and the
// row mirror (i with 15 - i) bring in the neighbouring quad's and half-row's sums just
// as lane ^ 4 and lane ^ 8 would; across rows, lane shuffles (^ 16, ^ 32).  The result
// is the butterfly's, bit for bit.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD b % 8).
// Renumber them so that XCD x receives one contiguous range of tiles: tiles that
// share neighbour planes then meet in the same L2.  A bijection for any count.
__device__ __forceinline__ int32_t xcd_tile(int32_t b, int32_t n) {
  const int32_t q = n >> 3, r = n & 7;
  const int32_t xcd = b & 7, local = b >> 3;
  return xcd * q + min(xcd, r) + local;
}

// Sum of a double over the workgroup (blockDim.x a multiple of 64, at most 1024):
// wave sums, then wave 0's lane 0 adds them in wave order.  The result is valid in
// thread 0 only.  Every thread of the workgroup must call it (two barriers).
__device__ __forceinline__ double block_sum(double v, double* scratch16) {
  const double w = wave_sum(v);
  if ((threadIdx.x & 63) == 0) scratch16[threadIdx.x >> 6] = w;
  __syncthreads();
  double total = 0.0;
  if (threadIdx.x == 0) {
    for (unsigned i = 0; i < blockDim.x / 64; ++i) total += scratch16[i];
  }
  __syncthreads();
  return total;
}

}  // namespace hsg
