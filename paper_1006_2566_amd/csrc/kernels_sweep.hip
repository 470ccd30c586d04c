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
    case PassMode::MetropolisFull:
      if (metropolis_mode(a.k_hits) == PassMode::MetropolisFull)
        hipLaunchKernelGGL((colour_pass_kernel<R, PassMode::MetropolisFull, NT>), grid, block, 0,
                           stream, a);
      else
        hipLaunchKernelGGL((colour_pass_kernel<R, PassMode::Metropolis, NT>), grid, block, 0,
                           stream, a);
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
