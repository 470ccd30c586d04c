// One colour-pass update of one site: gather the local field of eq. (2) from the six
// other-colour neighbours, then apply k Metropolis hits, k heat-bath draws or one
// over-relaxation step.  Shared by the single-lattice colour-pass kernel and the
// batched kernel, so a lattice gives the same bits alone or inside a batch.
#pragma once

#include "hsg_device.h"
#include "hsg_internal.h"

namespace hsg {

// Position of internal element e (0 <= e < N) of the colour-split layout.
struct SiteOf {
  int32_t c, xh, y, z, x;
  int64_t ic;         // index within the colour's planes
  uint32_t canon;     // x + L*y + L*L*z
};

__device__ __forceinline__ SiteOf site_of(int64_t e, int32_t L) {
  const int32_t Lh = L / 2;
  const int64_t Nh = (int64_t)Lh * L * L;
  SiteOf s;
  s.c = e >= Nh ? 1 : 0;
  s.ic = e - (int64_t)s.c * Nh;
  s.xh = (int32_t)(s.ic % Lh);
  const int64_t r = s.ic / Lh;
  s.y = (int32_t)(r % L);
  s.z = (int32_t)(r / L);
  s.x = 2 * s.xh + ((s.y + s.z + s.c) & 1);
  s.canon = (uint32_t)s.x + (uint32_t)L * ((uint32_t)s.y + (uint32_t)L * (uint32_t)s.z);
  return s;
}

// Random initial state of internal element e (0 <= e < N) of an L^3 lattice:
// spin uniform on the sphere from Philox tag 1; couplings (when J is not NULL) by
// Box-Muller from tag 2: (u0,u1) -> Jx, Jy; (u2,u3) -> Jz.  Counter (0, site, 0, tag).
template <typename R>
__device__ __forceinline__ void init_site(int32_t L, int64_t e, uint32_t k0, uint32_t k1,
                                          R* spins, R* J, uint32_t jk0, uint32_t jk1) {
  const int64_t Nh = (int64_t)L * L * L / 2;
  const SiteOf st = site_of(e, L);
  const Word4 ws = philox10(0u, st.canon, 0u, kTagInitSpin, k0, k1);
  const Vec3<R> s = sphere_point(unit_uniform<R>(ws.w0), unit_uniform<R>(ws.w1));
  const int64_t base = (int64_t)3 * st.c * Nh + st.ic;
  spins[base] = s.x;
  spins[base + Nh] = s.y;
  spins[base + 2 * Nh] = s.z;
  if (!J) return;
  const Word4 wj = philox10(0u, st.canon, 0u, kTagInitJ, jk0, jk1);
  R sn, cs;
  const R r01 = dev_sqrt((R)-2 * own_log(unit_uniform<R>(wj.w0)));
  sincos_2pi(unit_uniform<R>(wj.w1), sn, cs);
  J[base] = r01 * cs;
  J[base + Nh] = r01 * sn;
  const R r23 = dev_sqrt((R)-2 * own_log(unit_uniform<R>(wj.w2)));
  sincos_2pi(unit_uniform<R>(wj.w3), sn, cs);
  J[base + 2 * Nh] = r23 * cs;
}

// Where a site sits: colour c, column xh of its colour row, row y, plane z.
struct SitePos {
  int32_t L, Lh, c, xh, y, z;
};

// Monte Carlo stream of the site: Philox key and the uniform counter words.
template <typename R>
struct HitCtx {
  R beta;
  uint32_t sweep, phase;
  int32_t k_hits;
  uint32_t seed_lo, seed_hi;
};

// The update of one site given its spin s and local field h (eq. 2): reflection about
// h (over-relaxation), or k Metropolis hits / heat-bath draws with h fixed.  s is
// replaced in place; returns the sum of the accepted energy changes.
//
// Uniforms: the site's stream in a phase is the words of the Philox blocks b = 0, 1,
// ... with counter (sweep, site, phase << 16 | b, tag), in word order.  Metropolis hit
// j takes uniforms 3j, 3j+1, 3j+2 (polar, azimuth, acceptance), heat-bath draw j takes
// 2j, 2j+1: four hits share three blocks, two draws one block.  The hits are taken in
// such groups.  A hit's draws, trial spin and trial energy do not depend on earlier
// decisions, only its accept/reject step does; with G > 1 a group's trials are formed
// first (instruction-level parallelism for a wave with few neighbours on its SIMD),
// then its decisions in order.  Every operation and the order of the energy sum are
// the same for any G.  A heat-bath draw is always taken and does not depend on the spin
// it replaces, so of k draws only the last counts and only that one is computed.
template <typename R, PassMode MODE, int G = 1>
__device__ __forceinline__ double apply_update(Vec3<R>& s, const Vec3<R>& h, uint32_t site,
                                               const HitCtx<R>& hc) {
  double dE_sum = 0.0;
  if constexpr (MODE == PassMode::OverRelax) {
    s = reflect(s, h);
  } else if constexpr (MODE == PassMode::HeatBath) {
    const uint32_t j = (uint32_t)hc.k_hits - 1u;  // the last draw: uniforms 2j, 2j + 1
    const Word4 x = philox10(hc.sweep, site, (hc.phase << 16) | (j >> 1), kTagHeatBath,
                             hc.seed_lo, hc.seed_hi);
    const uint32_t w0 = (j & 1u) ? x.w2 : x.w0, w1 = (j & 1u) ? x.w3 : x.w1;
    const Vec3<R> t = heat_bath_point(h, hc.beta, unit_uniform<R>(w0), unit_uniform<R>(w1));
    const R dE = dot3(s, h) - dot3(t, h);
    s = t;
    dE_sum = (double)dE;
  } else {
    constexpr uint32_t tag = kTagMetropolis;
    constexpr int U = 3;             // uniforms per hit
    constexpr int H = 4;             // hits per group
    constexpr int NB = U * H / 4;    // Philox blocks per group
    // every group complete (k_hits a multiple of four): no per-group conditions
    constexpr bool kFull = MODE == PassMode::MetropolisFull;
    R sh = dot3(s, h);
    uint32_t b0 = 0;
    for (int32_t j0 = 0; j0 < hc.k_hits; j0 += H, b0 += NB) {
      const int32_t nh = hc.k_hits - j0;  // hits left (the group takes min(H, nh))
      uint32_t w[4 * NB];
      auto block = [&](int i) {
        const Word4 x = philox10(hc.sweep, site, (hc.phase << 16) | (b0 + (uint32_t)i), tag,
                                 hc.seed_lo, hc.seed_hi);
        w[4 * i] = x.w0;
        w[4 * i + 1] = x.w1;
        w[4 * i + 2] = x.w2;
        w[4 * i + 3] = x.w3;
      };
      if (kFull) {
        // a full group: its NB blocks advanced together (philox10_n)
        uint32_t c2[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) c2[i] = (hc.phase << 16) | (b0 + (uint32_t)i);
        Word4 x[NB];
        philox10_n<NB>(hc.sweep, site, c2, tag, hc.seed_lo, hc.seed_hi, x);
        // all words complete here (an empty statement that takes them as operands):
        // without it each block's rounds would be sunk to its first use, behind the
        // previous hit's decision, one chain at a time again
#pragma unroll
        for (int i = 0; i < NB; ++i)
          asm volatile("" : "+v"(x[i].w0), "+v"(x[i].w1), "+v"(x[i].w2), "+v"(x[i].w3));
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          w[4 * i] = x[i].w0;
          w[4 * i + 1] = x[i].w1;
          w[4 * i + 2] = x[i].w2;
          w[4 * i + 3] = x[i].w3;
        }
      } else {
#pragma unroll
        for (int i = 0; i < NB; ++i)
          if (i == 0 || 4 * i < U * nh) block(i);
      }
      (void)nh;
      Vec3<R> trial[H];
      R th[H], u2[H];
      auto draw = [&](int g) {
        trial[g] = sphere_point_words<R>(w[U * g], w[U * g + 1]);
        u2[g] = unit_uniform<R>(w[U * g + 2]);
        th[g] = dot3(trial[g], h);
      };
      auto decide = [&](int g) {
        const R dE = sh - th[g];
        const bool accept = (dE <= (R)0) || (u2[g] < accept_prob(-hc.beta * dE));
        if (accept) {
          s = trial[g];
          sh = th[g];
          dE_sum += (double)dE;
        }
      };
      if constexpr (G == 1) {
#pragma unroll
        for (int g = 0; g < H; ++g) {
          if (kFull || g < nh) {
            draw(g);
            decide(g);
          }
        }
      } else {
#pragma unroll
        for (int g = 0; g < H; ++g)
          if (kFull || g < nh) draw(g);
#pragma unroll
        for (int g = 0; g < H; ++g)
          if (kFull || g < nh) decide(g);
      }
    }
  }
  return dE_sum;
}

// Updates the site in place; returns the sum of the accepted energy changes.
// A load of data the pass only reads (couplings, the other colour's spins); with NT
// it carries the non-temporal cache hint.
template <bool NT, typename R>
__device__ __forceinline__ R read_only_ld(const R* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

template <typename R, PassMode MODE, bool NT = false>
__device__ __forceinline__ double update_site(const Planes<R>& S, const Planes<R>& J,
                                              const SitePos& q, const HitCtx<R>& hc) {
  const int32_t L = q.L, Lh = q.Lh, c = q.c, xh = q.xh, y = q.y, z = q.z;
  const int32_t p = (y + z + c) & 1;  // x = 2 xh + p
  const int32_t ym = y == 0 ? L - 1 : y - 1, yp = y == L - 1 ? 0 : y + 1;
  const int32_t zm = z == 0 ? L - 1 : z - 1, zp = z == L - 1 ? 0 : z + 1;
  const int32_t row = Lh * (y + L * z);
  const int32_t own = row + xh;
  // other-colour neighbours: x+1 and x-1 in the same row, y+-1 and z+-1 at the same xh
  const int32_t n_px = row + (p ? (xh + 1 == Lh ? 0 : xh + 1) : xh);
  const int32_t n_mx = row + (p ? xh : (xh == 0 ? Lh - 1 : xh - 1));
  const int32_t n_py = Lh * (yp + L * z) + xh, n_my = Lh * (ym + L * z) + xh;
  const int32_t n_pz = Lh * (y + L * zp) + xh, n_mz = Lh * (y + L * zm) + xh;
  const int oc = 3 * c, nc = 3 * (1 - c);

  // couplings of the six bonds: +x,+y,+z stored at the site, -x,-y,-z at the neighbour
  const R j_px = read_only_ld<NT>(J.p[oc + 0] + own), j_mx = read_only_ld<NT>(J.p[nc + 0] + n_mx);
  const R j_py = read_only_ld<NT>(J.p[oc + 1] + own), j_my = read_only_ld<NT>(J.p[nc + 1] + n_my);
  const R j_pz = read_only_ld<NT>(J.p[oc + 2] + own), j_mz = read_only_ld<NT>(J.p[nc + 2] + n_mz);
  R hcomp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R* sn = S.p[nc + k];
    R acc = j_px * read_only_ld<NT>(sn + n_px);
    acc = dev_fma(j_mx, read_only_ld<NT>(sn + n_mx), acc);
    acc = dev_fma(j_py, read_only_ld<NT>(sn + n_py), acc);
    acc = dev_fma(j_my, read_only_ld<NT>(sn + n_my), acc);
    acc = dev_fma(j_pz, read_only_ld<NT>(sn + n_pz), acc);
    acc = dev_fma(j_mz, read_only_ld<NT>(sn + n_mz), acc);
    hcomp[k] = acc;
  }
  const Vec3<R> h{hcomp[0], hcomp[1], hcomp[2]};
  Vec3<R> s{*(S.p[oc + 0] + own), *(S.p[oc + 1] + own),
            *(S.p[oc + 2] + own)};

  const uint32_t site = (uint32_t)(2 * xh + p) + (uint32_t)L * (uint32_t)(y + L * z);
  const double dE_sum = apply_update<R, MODE>(s, h, site, hc);
  S.p[oc + 0][own] = s.x;
  S.p[oc + 1][own] = s.y;
  S.p[oc + 2][own] = s.z;
  return dE_sum;
}

// Element at byte offset `off` of a plane whose base is wave-uniform: the access uses
// the scalar-base + 32-bit vector-offset addressing of global loads and stores, with no
// 64-bit address arithmetic per lane.  A binary32 plane of N/2 <= 2^30 values spans less
// than 2^32 bytes for every L the library accepts.
__device__ __forceinline__ float plane_ld(const float* base, uint32_t off) {
  return *(const float*)((const char*)base + off);
}
// The same for data the pass only reads; with NT the load carries the non-temporal hint.
template <bool NT>
__device__ __forceinline__ float plane_ld_ro(const float* base, uint32_t off) {
  const float* p = (const float*)((const char*)base + off);
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
__device__ __forceinline__ void plane_st(float* base, uint32_t off, float v) {
  *(float*)((char*)base + off) = v;
}

// The binary32 site update of the colour passes (single lattice, batched, served): the same field (eq. 2, same
// order of products and fused multiply-adds) and the same apply_update as update_site,
// with 32-bit byte offsets into the six planes.
template <PassMode MODE, bool NT>
__device__ __forceinline__ double update_site_b32(const Planes<float>& S, const Planes<float>& J,
                                                  const SitePos& q, const HitCtx<float>& hc) {
  const uint32_t L = (uint32_t)q.L, Lh = (uint32_t)q.Lh, xh = (uint32_t)q.xh;
  const uint32_t y = (uint32_t)q.y, z = (uint32_t)q.z;
  const int32_t c = q.c;
  const uint32_t p = (y + z + (uint32_t)c) & 1u;  // x = 2 xh + p
  const uint32_t ym = y == 0 ? L - 1 : y - 1, yp = y == L - 1 ? 0 : y + 1;
  const uint32_t zm = z == 0 ? L - 1 : z - 1, zp = z == L - 1 ? 0 : z + 1;
  const uint32_t row = Lh * (y + L * z);
  const uint32_t own = (row + xh) << 2;
  const uint32_t n_px = (row + (p ? (xh + 1 == Lh ? 0 : xh + 1) : xh)) << 2;
  const uint32_t n_mx = (row + (p ? xh : (xh == 0 ? Lh - 1 : xh - 1))) << 2;
  const uint32_t n_py = (Lh * (yp + L * z) + xh) << 2, n_my = (Lh * (ym + L * z) + xh) << 2;
  const uint32_t n_pz = (Lh * (y + L * zp) + xh) << 2, n_mz = (Lh * (y + L * zm) + xh) << 2;
  const int oc = 3 * c, nc = 3 * (1 - c);
  const float j_px = plane_ld_ro<NT>(J.p[oc + 0], own), j_mx = plane_ld_ro<NT>(J.p[nc + 0], n_mx);
  const float j_py = plane_ld_ro<NT>(J.p[oc + 1], own), j_my = plane_ld_ro<NT>(J.p[nc + 1], n_my);
  const float j_pz = plane_ld_ro<NT>(J.p[oc + 2], own), j_mz = plane_ld_ro<NT>(J.p[nc + 2], n_mz);
  float hcomp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float* sn = S.p[nc + k];
    float acc = j_px * plane_ld_ro<NT>(sn, n_px);
    acc = dev_fma(j_mx, plane_ld_ro<NT>(sn, n_mx), acc);
    acc = dev_fma(j_py, plane_ld_ro<NT>(sn, n_py), acc);
    acc = dev_fma(j_my, plane_ld_ro<NT>(sn, n_my), acc);
    acc = dev_fma(j_pz, plane_ld_ro<NT>(sn, n_pz), acc);
    acc = dev_fma(j_mz, plane_ld_ro<NT>(sn, n_mz), acc);
    hcomp[k] = acc;
  }
  const Vec3<float> h{hcomp[0], hcomp[1], hcomp[2]};
  Vec3<float> s{plane_ld(S.p[oc + 0], own), plane_ld(S.p[oc + 1], own), plane_ld(S.p[oc + 2], own)};
  const uint32_t site = (2 * xh + p) + L * (y + L * z);
  const double dE_sum = apply_update<float, MODE>(s, h, site, hc);
  plane_st(S.p[oc + 0], own, s.x);
  plane_st(S.p[oc + 1], own, s.y);
  plane_st(S.p[oc + 2], own, s.z);
  return dE_sum;
}

// s / |s| (length from a fused dot product, correctly rounded root and divisions).
template <typename R>
__device__ __forceinline__ Vec3<R> unit_vector(const Vec3<R>& s) {
  const R n = dev_sqrt(dot3(s, s));
  return Vec3<R>{dev_div(s.x, n), dev_div(s.y, n), dev_div(s.z, n)};
}

// sigma <- sigma / |sigma| for the spin at index e of colour c (N/2 = Nh per colour).
template <typename R>
__device__ __forceinline__ void renormalise_spin(const Planes<R>& S, int c, int64_t e) {
  const Vec3<R> s{S.p[3 * c][e], S.p[3 * c + 1][e], S.p[3 * c + 2][e]};
  const R n = dev_sqrt(dot3(s, s));
  S.p[3 * c][e] = dev_div(s.x, n);
  S.p[3 * c + 1][e] = dev_div(s.y, n);
  S.p[3 * c + 2][e] = dev_div(s.z, n);
}

// sigma_i . h_i of the colour-0 site (xh, y, z) in binary64.  Every bond has exactly
// one colour-0 end (L even), so H = -(sum of this over the colour-0 sites).
template <typename R>
__device__ __forceinline__ double colour0_bond_sum(const R* spins, const R* J, int64_t Nh,
                                                   int32_t L, int32_t Lh, int32_t xh, int32_t y,
                                                   int32_t z) {
  const int32_t p = (y + z) & 1;
  const int32_t ym = y == 0 ? L - 1 : y - 1, yp = y == L - 1 ? 0 : y + 1;
  const int32_t zm = z == 0 ? L - 1 : z - 1, zp = z == L - 1 ? 0 : z + 1;
  const int64_t row = (int64_t)Lh * (y + (int64_t)L * z);
  const int64_t own = row + xh;
  const int64_t nb[6] = {row + (p ? (xh + 1 == Lh ? 0 : xh + 1) : xh),
                         row + (p ? xh : (xh == 0 ? Lh - 1 : xh - 1)),
                         (int64_t)Lh * (yp + (int64_t)L * z) + xh,
                         (int64_t)Lh * (ym + (int64_t)L * z) + xh,
                         (int64_t)Lh * (y + (int64_t)L * zp) + xh,
                         (int64_t)Lh * (y + (int64_t)L * zm) + xh};
  const double jb[6] = {(double)J[own],      (double)J[3 * Nh + nb[1]], (double)J[Nh + own],
                        (double)J[4 * Nh + nb[3]], (double)J[2 * Nh + own],
                        (double)J[5 * Nh + nb[5]]};
  double e_site = 0.0;
  for (int k = 0; k < 3; ++k) {
    double hk = 0.0;
    for (int d = 0; d < 6; ++d) hk = fma(jb[d], (double)spins[(3 + k) * Nh + nb[d]], hk);
    e_site = fma((double)spins[k * Nh + own], hk, e_site);
  }
  return e_site;
}

}  // namespace hsg
