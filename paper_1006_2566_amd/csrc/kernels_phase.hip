// One over-relaxation phase of the checkerboard schedule (§4) -- the colour-0 pass and
// then the colour-1 pass -- in one launch, reading the spins once and writing them once.
//
// Each workgroup owns a tile of 64 x kPTY sites in (x, y) and kPZ planes in z, and
// marches through z holding, in LDS, three planes of each colour of its region (the
// tile widened by one colour site on each side in x and by two rows in y): colour 1 on
// planes a - 1 .. a + 1, colour 0 on planes a - 2 .. a.  At step t it
// updates the colour-0 sites of plane a = z0 - 1 + t over the tile and a ring of one
// site (stage A), then the colour-1 sites of plane a - 1 over the tile (stage B), whose
// colour-0 neighbours on planes a - 2, a - 1 and a are then all updated.  The ring
// and the planes z0 - 1 and z0 + kPZ belong to other workgroups, which compute them
// too, from the same inputs and the same Philox draws, hence to the same bits; so
// workgroups never communicate.  They read the spins before the phase from one
// buffer and write the tile after it to another.
//
// The site arithmetic (field of eq. 2 in the fixed order of the single-pass kernel,
// then the reflection of §4) is the single pass's, so results equal two colour passes
// bit for bit.
#include "hsg_device.h"
#include "hsg_internal.h"
#include "hsg_site.h"

namespace hsg {
namespace {

constexpr int kPTX = 32;                 // colour sites of a tile row (64 sites in x)
constexpr int kRegX = kPTX + 2;          // region row: xh0 - 1 .. xh0 + 32
constexpr int kRegY = kPTY + 4;          // region rows: y0 - 2 .. y0 + kPTY + 1
constexpr int kColour = kRegY * kRegX;   // one colour, one component, one plane
constexpr int kSlice = 3 * kColour;      // one colour, three components, one plane
constexpr int kRing = 3;                 // planes of each colour in LDS
constexpr int kLoadRounds = (kSlice + kPhaseThreads - 1) / kPhaseThreads;
constexpr int kASites = (kPTY + 2) * (kPTX + 1);  // colour-0 sites of stage A per plane
constexpr int kARounds = (kASites + kPhaseThreads - 1) / kPhaseThreads;
constexpr int kBSites = kPTY * kPTX;                // colour-1 sites of stage B per plane
constexpr int kBRounds = (kBSites + kPhaseThreads - 1) / kPhaseThreads;
constexpr int kStore = 2 * 3 * kPTY * kPTX;         // values of a plane's own tile
constexpr int kStoreRounds = (kStore + kPhaseThreads - 1) / kPhaseThreads;

struct PhaseCtx {
  int32_t L, Lh;
  uint32_t Nh, zstride;  // N/2 and L/2 * L
  int32_t xh0, y0, z0;   // tile origin (colour column, row, plane)
};

__device__ __forceinline__ int32_t wrap_to(int32_t v, int32_t n) {
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// One colour of a region plane in registers: element e (component, row, column) of
// the slice, its colour-0 global offset without the plane's z offset (colour 1 adds
// 3 N/2).
struct SliceOffsets {
  uint32_t off[kLoadRounds];
};

template <typename R>
struct SliceRegs {
  R v[kLoadRounds];
};

__device__ __forceinline__ void slice_offsets(SliceOffsets& so, const PhaseCtx& m) {
#pragma unroll
  for (int k = 0; k < kLoadRounds; ++k) {
    const int32_t e = (int32_t)threadIdx.x + k * kPhaseThreads;
    const int32_t comp = e / kColour;
    const int32_t r = e - comp * kColour;
    const int32_t ry = r / kRegX;
    const int32_t j = r - ry * kRegX;
    const int32_t y = wrap_to(m.y0 - 2 + ry, m.L);
    const int32_t xh = wrap_to(m.xh0 - 1 + j, m.Lh);
    so.off[k] = (uint32_t)comp * m.Nh + (uint32_t)xh + (uint32_t)m.Lh * (uint32_t)y;
  }
}

template <typename R>
__device__ __forceinline__ void fetch(SliceRegs<R>& sr, const SliceOffsets& so, const R* in,
                                      const PhaseCtx& m, int32_t c, int32_t q) {
  const uint32_t base = (uint32_t)(3 * c) * m.Nh + m.zstride * (uint32_t)wrap_to(q, m.L);
#pragma unroll
  for (int k = 0; k < kLoadRounds; ++k)
    if ((int32_t)threadIdx.x + k * kPhaseThreads < kSlice) sr.v[k] = in[so.off[k] + base];
}

// Slice of colour c, plane q (q >= -3) in the colour's ring.
template <typename R>
__device__ __forceinline__ R* slice(R* lds, int32_t c, int32_t q) {
  return lds + (c * kRing + (q + 3 * kRing) % kRing) * kSlice;
}

template <typename R>
__device__ __forceinline__ void put(R* lds, const SliceRegs<R>& sr, int32_t c, int32_t q) {
  R* dst = slice(lds, c, q);
#pragma unroll
  for (int k = 0; k < kLoadRounds; ++k) {
    const int32_t e = (int32_t)threadIdx.x + k * kPhaseThreads;
    if (e < kSlice) dst[e] = sr.v[k];
  }
}

// Update of the site of colour C in region row ry, column j, on plane q (z): the
// field from the window (neighbour colour 1 - C), the six couplings from global memory
// in the single pass's order, then apply_update; the result goes back to the window.
template <typename R, int C, PassMode MODE>
__device__ __forceinline__ double phase_site(R* lds, const R* J, const PhaseCtx& m,
                                             int32_t q, int32_t z, int32_t ry, int32_t j,
                                             const HitCtx<R>& hc) {
  const R* cur = slice(lds, 1 - C, q);
  const R* up = slice(lds, 1 - C, q + 1);
  const R* dn = slice(lds, 1 - C, q - 1);
  const int32_t y = wrap_to(m.y0 - 2 + ry, m.L);
  const int32_t p = (y + z + C) & 1;  // x parity of colour-C sites on this row
  const int32_t xh = wrap_to(m.xh0 - 1 + j, m.Lh);
  const int32_t row = ry * kRegX;
  const int32_t i_px = row + (p ? j + 1 : j), i_mx = row + (p ? j : j - 1);
  const int32_t i_py = row + kRegX + j, i_my = row - kRegX + j, i_z = row + j;
  // couplings: +x,+y,+z at the site (colour C planes), -x,-y,-z at the neighbours
  const int32_t ym = y == 0 ? m.L - 1 : y - 1, zm = z == 0 ? m.L - 1 : z - 1;
  const int32_t xhm = p ? xh : (xh == 0 ? m.Lh - 1 : xh - 1);
  const uint32_t zo = m.zstride * (uint32_t)z;
  const uint32_t own = zo + (uint32_t)m.Lh * (uint32_t)y + (uint32_t)xh;
  const R* Jo = J + (uint32_t)(3 * C) * m.Nh;
  const R* Jn = J + (uint32_t)(3 * (1 - C)) * m.Nh;
  const R j_px = Jo[own];
  const R j_mx = Jn[zo + (uint32_t)m.Lh * (uint32_t)y + (uint32_t)xhm];
  const R j_py = Jo[m.Nh + own];
  const R j_my = Jn[m.Nh + zo + (uint32_t)m.Lh * (uint32_t)ym + (uint32_t)xh];
  const R j_pz = Jo[2 * m.Nh + own];
  const R j_mz = Jn[2 * m.Nh + m.zstride * (uint32_t)zm + (uint32_t)m.Lh * (uint32_t)y +
                    (uint32_t)xh];
  R hcomp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int32_t kb = k * kColour;
    R acc = j_px * cur[kb + i_px];
    acc = dev_fma(j_mx, cur[kb + i_mx], acc);
    acc = dev_fma(j_py, cur[kb + i_py], acc);
    acc = dev_fma(j_my, cur[kb + i_my], acc);
    acc = dev_fma(j_pz, up[kb + i_z], acc);
    acc = dev_fma(j_mz, dn[kb + i_z], acc);
    hcomp[k] = acc;
  }
  const Vec3<R> h{hcomp[0], hcomp[1], hcomp[2]};
  R* mine = slice(lds, C, q);
  const int32_t io = ry * kRegX + j;
  Vec3<R> s{mine[io], mine[kColour + io], mine[2 * kColour + io]};
  const uint32_t site = (uint32_t)(2 * xh + p) + (uint32_t)m.L * (uint32_t)(y + m.L * z);
  const double d = apply_update<R, MODE>(s, h, site, hc);
  mine[io] = s.x;
  mine[kColour + io] = s.y;
  mine[2 * kColour + io] = s.z;
  return d;
}

// The over-relaxation phase (the one the schedule runs as one launch): no energy
// changes to record.
template <typename R>
__global__ __launch_bounds__(kPhaseThreads) void phase_kernel(PhaseArgs<R> a) {
  constexpr PassMode MODE = PassMode::OverRelax;
  __shared__ R lds[2 * kRing * kSlice];
  const int32_t tiles_x = a.L / 2 / kPTX, tiles_y = a.L / kPTY;
  const int32_t tile = xcd_tile((int32_t)blockIdx.x, (int32_t)gridDim.x);
  const int32_t tx = tile % tiles_x;
  const int32_t rest = tile / tiles_x;
  const int32_t ty = rest % tiles_y, tz = rest / tiles_y;
  PhaseCtx m;
  m.L = a.L;
  m.Lh = a.L / 2;
  m.zstride = (uint32_t)m.Lh * (uint32_t)a.L;
  m.Nh = m.zstride * (uint32_t)a.L;
  m.xh0 = tx * kPTX;
  m.y0 = ty * kPTY;
  m.z0 = tz * kPZ;
  const HitCtx<R> hc{a.beta, a.sweep, a.phase, a.k_hits, a.seed_lo, a.seed_hi};

  // before step 0 (stage A on plane z0 - 1): colour 1 of planes z0 - 2 .. z0, colour 0
  // of plane z0 - 1; in registers the slices the end of step 0 puts in place
  SliceOffsets so;
  slice_offsets(so, m);
  SliceRegs<R> r0, r1;
  for (int32_t q = m.z0 - 2; q <= m.z0; ++q) {
    fetch<R>(r1, so, a.in, m, 1, q);
    put<R>(lds, r1, 1, q);
  }
  fetch<R>(r0, so, a.in, m, 0, m.z0 - 1);
  put<R>(lds, r0, 0, m.z0 - 1);
  fetch<R>(r0, so, a.in, m, 0, m.z0);
  fetch<R>(r1, so, a.in, m, 1, m.z0 + 1);

  for (int32_t t = 0; t <= kPZ + 1; ++t) {
    const int32_t q = m.z0 - 1 + t;  // stage A plane; stage B works on q - 1
    __syncthreads();
    {
      const int32_t z = wrap_to(q, m.L);
#pragma unroll
      for (int r = 0; r < kARounds; ++r) {
        const int32_t i = (int32_t)threadIdx.x + r * kPhaseThreads;
        if (i < kASites) {
          const int32_t dr = i / (kPTX + 1);
          const int32_t ry = 1 + dr;
          const int32_t y = wrap_to(m.y0 - 2 + ry, m.L);
          const int32_t p0 = (y + z) & 1;
          const int32_t j = (i - dr * (kPTX + 1)) + (1 - p0);
          phase_site<R, 0, MODE>(lds, a.J, m, q, z, ry, j, hc);
        }
      }
    }
    __syncthreads();
    if (t >= 2) {
      const int32_t b = q - 1;
      const int32_t z = wrap_to(b, m.L);
#pragma unroll
      for (int r = 0; r < kBRounds; ++r) {
        const int32_t i = (int32_t)threadIdx.x + r * kPhaseThreads;
        if (i < kBSites) {
          const int32_t dr = i / kPTX;
          phase_site<R, 1, MODE>(lds, a.J, m, b, z, 2 + dr, 1 + (i - dr * kPTX), hc);
        }
      }
      __syncthreads();
    }
    // colour 0 of plane q + 1 replaces plane q - 2 (last read by stage B)
    if (t <= kPZ) put<R>(lds, r0, 0, q + 1);
    if (t >= 2) {
      // plane b = q - 1 is final: write the tile's sites of both colours
      const int32_t b = q - 1;
      const uint32_t zo = m.zstride * (uint32_t)wrap_to(b, m.L);
#pragma unroll
      for (int r = 0; r < kStoreRounds; ++r) {
        const int32_t e = (int32_t)threadIdx.x + r * kPhaseThreads;
        if (e < kStore) {
          const int32_t col = e % kPTX;
          const int32_t rest2 = e / kPTX;
          const int32_t iy = rest2 % kPTY;
          const int32_t cc = rest2 / kPTY;  // 3 * colour + component
          const int32_t c = cc / 3, comp = cc - 3 * c;
          const R v = slice(lds, c, b)[comp * kColour + (2 + iy) * kRegX + 1 + col];
          a.out[(uint32_t)cc * m.Nh + zo + (uint32_t)m.Lh * (uint32_t)(m.y0 + iy) +
                (uint32_t)(m.xh0 + col)] = v;
        }
      }
      __syncthreads();
    }
    // colour 1 of plane q + 2 replaces plane q - 1 (stored above)
    if (t <= kPZ) {
      put<R>(lds, r1, 1, q + 2);
      if (t + 1 <= kPZ) {
        fetch<R>(r0, so, a.in, m, 0, q + 2);
        fetch<R>(r1, so, a.in, m, 1, q + 3);
      }
    }
  }
}

}  // namespace

bool phase_supported(int32_t L) {
  return L >= kPhaseMinL && L % (2 * kPTX) == 0 && L % kPTY == 0 && L % kPZ == 0;
}

int32_t phase_blocks(int32_t L) { return (L / 2 / kPTX) * (L / kPTY) * (L / kPZ); }

template <typename R>
hipError_t launch_phase(const PhaseArgs<R>& a, hipStream_t st) {
  if (!phase_supported(a.L)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)phase_blocks(a.L)), block(kPhaseThreads);
  hipLaunchKernelGGL(phase_kernel<R>, grid, block, 0, st, a);
  return hipGetLastError();
}

template hipError_t launch_phase<float>(const PhaseArgs<float>&, hipStream_t);
template hipError_t launch_phase<double>(const PhaseArgs<double>&, hipStream_t);

}  // namespace hsg
