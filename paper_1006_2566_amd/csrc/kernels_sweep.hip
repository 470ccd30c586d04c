// Colour-pass kernels: one launch updates every site of one colour (§4's
// checkerboard: sites of one colour share no bond, so they are independent).
//
// Memory: spins and couplings are colour-split structure-of-arrays (six planes of
// N/2 values each), so a wavefront reads one contiguous row segment per plane and
// the six neighbours of a colour-c site are the same xh in the rows y+-1 and planes
// z+-1 of the other colour, plus xh and xh+-1 in its own row.  A pass therefore
// reads the own colour's spins and couplings, the other colour's spins and
// couplings, and writes the own colour's spins: 30 bytes per lattice site in
// binary32.  Neighbour rows shared by adjacent tiles are served from L2, which is
// why tiles are assigned to XCDs in contiguous z ranges (see xcd_tile).
#include <algorithm>

#include "hsg_device.h"
#include "hsg_internal.h"
#include "hsg_site.h"

namespace hsg {

static int ceil_log2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

Geometry pass_geometry(int32_t L) {
  Geometry g{};
  g.L = L;
  g.Lh = L / 2;
  g.bx_log = std::min(6, ceil_log2(g.Lh));
  g.by_log = std::min(8 - g.bx_log, ceil_log2(L));
  g.bz_log = std::min(8 - g.bx_log - g.by_log, ceil_log2(L));
  g.tiles_x = (g.Lh + (1 << g.bx_log) - 1) >> g.bx_log;
  g.tiles_y = (L + (1 << g.by_log) - 1) >> g.by_log;
  g.tiles_z = (L + (1 << g.bz_log) - 1) >> g.bz_log;
  g.n_blocks = g.tiles_x * g.tiles_y * g.tiles_z;
  g.threads = 1 << (g.bx_log + g.by_log + g.bz_log);
  return g;
}

size_t work_bytes_for(int32_t L) {
  return 256 + sizeof(double) * ((size_t)pass_geometry(L).n_blocks + (size_t)kReduceRegion);
}

size_t fused_offset(int32_t L) { return (work_bytes_for(L) + 255) & ~(size_t)255; }

size_t work_bytes_for(int32_t L, int32_t dtype_bytes) {
  if (!march_supported(L) && !phase_supported(L)) return work_bytes_for(L);
  return fused_offset(L) + (size_t)3 * L * L * L * (size_t)dtype_bytes;
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

// The binary32 site update of the single-lattice pass: the same field (eq. 2, same
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

// One tile of a colour pass (a BX x BY x BZ block of the colour's sites); Metropolis
// and heat-bath passes add the tile's accepted energy changes to partials[tile] in a
// fixed order (wave sums, then the waves in order).  `tile` must be wave-uniform.
template <typename R, PassMode MODE, bool NT>
__device__ __forceinline__ void pass_tile(const PassArgs<R>& a, int32_t tile) {
  const Geometry& g = a.g;
  const int32_t tx = tile % g.tiles_x;
  const int32_t rest = tile / g.tiles_x;
  const int32_t ty = rest % g.tiles_y;
  const int32_t tz = rest / g.tiles_y;
  const int32_t t = (int32_t)threadIdx.x;
  SitePos q;
  q.L = g.L;
  q.Lh = g.Lh;
  q.c = a.colour;
  q.xh = (tx << g.bx_log) + (t & ((1 << g.bx_log) - 1));
  q.y = (ty << g.by_log) + ((t >> g.bx_log) & ((1 << g.by_log) - 1));
  q.z = (tz << g.bz_log) + (t >> (g.bx_log + g.by_log));
  const bool active = t < g.threads && q.xh < g.Lh && q.y < g.L && q.z < g.L;
  const HitCtx<R> hc{a.beta, a.sweep, a.phase, a.k_hits, a.seed_lo, a.seed_hi};

  double dE_sum = 0.0;
  if (active) {
    if constexpr (sizeof(R) == 4)
      dE_sum = update_site_b32<MODE, NT>(a.spins, a.J, q, hc);
    else
      dE_sum = update_site<R, MODE, NT>(a.spins, a.J, q, hc);
  }

  if constexpr (MODE != PassMode::OverRelax) {
    __shared__ double wave_part[4];
    const double v = wave_sum(dE_sum);
    if ((t & 63) == 0) wave_part[t >> 6] = v;
    __syncthreads();
    if (t == 0) a.partials[tile] += ((wave_part[0] + wave_part[1]) + (wave_part[2] + wave_part[3]));
  }
}

// Workgroup b of the launch takes tile tile_base + xcd_tile(b) (mirrored when the pass
// walks z backwards); the grid is tile_count workgroups.
template <typename R, PassMode MODE, bool NT>
__global__ __launch_bounds__(256) void colour_pass_kernel(PassArgs<R> a) {
  int32_t tile = xcd_tile((int32_t)blockIdx.x, a.tile_count);
  if (a.reverse) tile = a.tile_count - 1 - tile;
  pass_tile<R, MODE, NT>(a, __builtin_amdgcn_readfirstlane(a.tile_base + tile));
}

template <typename R, bool NT>
void launch_pass_kind(PassMode mode, const PassArgs<R>& a, hipStream_t stream) {
  const dim3 grid((unsigned)a.tile_count), block(256);
  switch (mode) {
    case PassMode::Metropolis:
      hipLaunchKernelGGL((colour_pass_kernel<R, PassMode::Metropolis, NT>), grid, block, 0, stream,
                         a);
      break;
    case PassMode::OverRelax:
      hipLaunchKernelGGL((colour_pass_kernel<R, PassMode::OverRelax, NT>), grid, block, 0, stream,
                         a);
      break;
    case PassMode::HeatBath:
      hipLaunchKernelGGL((colour_pass_kernel<R, PassMode::HeatBath, NT>), grid, block, 0, stream,
                         a);
      break;
  }
}

template <typename R>
hipError_t launch_colour_pass(PassMode mode, const PassArgs<R>& a, hipStream_t stream) {
  if (a.tile_count < 1 || a.tile_base < 0 || a.tile_base + a.tile_count > a.g.n_blocks)
    return hipErrorInvalidValue;
  if (a.nt)
    launch_pass_kind<R, true>(mode, a, stream);
  else
    launch_pass_kind<R, false>(mode, a, stream);
  return hipGetLastError();
}

template hipError_t launch_colour_pass<float>(PassMode, const PassArgs<float>&, hipStream_t);
template hipError_t launch_colour_pass<double>(PassMode, const PassArgs<double>&, hipStream_t);

// *E += sum of the partials in a fixed order (strided per thread, then a fixed tree),
// and the partials are reset to zero for the next sweeps.
__global__ __launch_bounds__(1024) void fold_partials_kernel(double* partials, int32_t n,
                                                             double* E) {
  __shared__ double wave_part[16];
  double acc = 0.0;
  for (int32_t i = (int32_t)threadIdx.x; i < n; i += 1024) {
    acc += partials[i];
    partials[i] = 0.0;
  }
  const double v = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) wave_part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double total = 0.0;
    for (int w = 0; w < 16; ++w) total += wave_part[w];
    *E += total;
  }
}

hipError_t launch_fold_partials(double* partials, int32_t n, double* E, hipStream_t stream) {
  hipLaunchKernelGGL(fold_partials_kernel, dim3(1), dim3(1024), 0, stream, partials, n, E);
  return hipGetLastError();
}

}  // namespace hsg
