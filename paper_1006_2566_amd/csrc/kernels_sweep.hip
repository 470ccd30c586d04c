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
  return 256 + sizeof(double) * ((size_t)pass_geometry(L).n_blocks +
                                 (size_t)kReduceBlocks * kReduceSlots);
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD b % 8).
// Renumber them so that XCD x receives one contiguous range of tiles: tiles that
// share neighbour planes then meet in the same L2.  A bijection for any count.
__device__ __forceinline__ int32_t xcd_tile(int32_t b, int32_t n) {
  const int32_t q = n >> 3, r = n & 7;
  const int32_t xcd = b & 7, local = b >> 3;
  return xcd * q + min(xcd, r) + local;
}

// Spin accesses, optionally with the non-temporal hint (streamed past the caches so
// that the couplings, reused by every pass, keep their place).
template <bool NT, typename R>
__device__ __forceinline__ R load_spin(const R* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool NT, typename R>
__device__ __forceinline__ void store_spin(R v, R* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <typename R, PassMode MODE, bool NT>
__global__ __launch_bounds__(256) void colour_pass_kernel(PassArgs<R> a) {
  const Geometry& g = a.g;
  int32_t tile = xcd_tile((int32_t)blockIdx.x, g.n_blocks);
  if (a.reverse) tile = g.n_blocks - 1 - tile;
  const int32_t tx = tile % g.tiles_x;
  const int32_t rest = tile / g.tiles_x;
  const int32_t ty = rest % g.tiles_y;
  const int32_t tz = rest / g.tiles_y;
  const int32_t t = (int32_t)threadIdx.x;
  const int32_t xh = (tx << g.bx_log) + (t & ((1 << g.bx_log) - 1));
  const int32_t y = (ty << g.by_log) + ((t >> g.bx_log) & ((1 << g.by_log) - 1));
  const int32_t z = (tz << g.bz_log) + (t >> (g.bx_log + g.by_log));
  const bool active = t < g.threads && xh < g.Lh && y < g.L && z < g.L;

  double dE_sum = 0.0;
  if (active) {
    const int32_t L = g.L, Lh = g.Lh, c = a.colour;
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
    const R j_px = a.J.p[oc + 0][own], j_mx = a.J.p[nc + 0][n_mx];
    const R j_py = a.J.p[oc + 1][own], j_my = a.J.p[nc + 1][n_my];
    const R j_pz = a.J.p[oc + 2][own], j_mz = a.J.p[nc + 2][n_mz];
    R hc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R* sn = a.spins.p[nc + k];
      R acc = j_px * load_spin<NT>(sn + n_px);
      acc = dev_fma(j_mx, load_spin<NT>(sn + n_mx), acc);
      acc = dev_fma(j_py, load_spin<NT>(sn + n_py), acc);
      acc = dev_fma(j_my, load_spin<NT>(sn + n_my), acc);
      acc = dev_fma(j_pz, load_spin<NT>(sn + n_pz), acc);
      acc = dev_fma(j_mz, load_spin<NT>(sn + n_mz), acc);
      hc[k] = acc;
    }
    const Vec3<R> h{hc[0], hc[1], hc[2]};
    Vec3<R> s{load_spin<NT>(a.spins.p[oc + 0] + own), load_spin<NT>(a.spins.p[oc + 1] + own),
              load_spin<NT>(a.spins.p[oc + 2] + own)};

    if constexpr (MODE == PassMode::OverRelax) {
      s = reflect(s, h);
    } else {
      const uint32_t site = (uint32_t)(2 * xh + p) + (uint32_t)L * (uint32_t)(y + L * z);
      const uint32_t tag = MODE == PassMode::Metropolis ? kTagMetropolis : kTagHeatBath;
      R sh = dot3(s, h);
      for (int32_t j = 0; j < a.k_hits; ++j) {
        const Word4 w = philox10(a.sweep, site, (a.phase << 16) | (uint32_t)j, tag, a.seed_lo,
                                 a.seed_hi);
        Vec3<R> trial;
        if constexpr (MODE == PassMode::Metropolis) {
          trial = sphere_point_words<R>(w.w0, w.w1);
        } else {
          trial = heat_bath_point(h, a.beta, unit_uniform<R>(w.w0), unit_uniform<R>(w.w1));
        }
        const R th = dot3(trial, h);
        const R dE = sh - th;
        bool accept = true;
        if constexpr (MODE == PassMode::Metropolis) {
          const R u2 = unit_uniform<R>(w.w2);
          accept = (dE <= (R)0) || (u2 < accept_prob(-a.beta * dE));
        }
        if (accept) {
          s = trial;
          sh = th;
          dE_sum += (double)dE;
        }
      }
    }
    store_spin<NT>(s.x, a.spins.p[oc + 0] + own);
    store_spin<NT>(s.y, a.spins.p[oc + 1] + own);
    store_spin<NT>(s.z, a.spins.p[oc + 2] + own);
  }

  if constexpr (MODE != PassMode::OverRelax) {
    __shared__ double wave_part[4];
    const double v = wave_sum(dE_sum);
    if ((t & 63) == 0) wave_part[t >> 6] = v;
    __syncthreads();
    if (t == 0) a.partials[tile] += ((wave_part[0] + wave_part[1]) + (wave_part[2] + wave_part[3]));
  }
}

template <typename R, bool NT>
static void launch_mode(PassMode mode, const PassArgs<R>& a, hipStream_t stream) {
  const dim3 grid((unsigned)a.g.n_blocks), block(256);
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
hipError_t launch_colour_pass(PassMode mode, bool stream_spins, const PassArgs<R>& a,
                              hipStream_t stream) {
  if (stream_spins)
    launch_mode<R, true>(mode, a, stream);
  else
    launch_mode<R, false>(mode, a, stream);
  return hipGetLastError();
}

template hipError_t launch_colour_pass<float>(PassMode, bool, const PassArgs<float>&, hipStream_t);
template hipError_t launch_colour_pass<double>(PassMode, bool, const PassArgs<double>&,
                                                hipStream_t);

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
