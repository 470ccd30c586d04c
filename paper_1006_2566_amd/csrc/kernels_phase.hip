// One over-relaxation phase of the checkerboard schedule (§4) -- the colour-0 pass and
// then the colour-1 pass -- in one launch, reading the spins once and writing them once;
// optionally followed, in the same launch, by the colour-0 pass of the next sweep's
// Monte Carlo phase.
//
// Each workgroup owns a tile of 64 x kPTY sites in (x, y) and a run of planes in z, and
// marches through z holding, in LDS, a few planes of each colour of its region.  With NS
// stages (2: the phase; 3: the phase and the Monte Carlo pass) stage s updates its
// colour on the tile and a ring of NS - 1 - s sites around it, so that the next stage
// finds every neighbour it reads already updated; the region is the tile widened on each
// side by NS - 1 colour columns in x and NS rows in y.  With a = z0 - (NS - 1) + t the
// plane of stage A at step t:
//
//   stage A   colour 0, over-relaxation, ring NS - 1, plane a
//   stage B   colour 1, over-relaxation, ring NS - 2, plane a - 1 (reads colour 0 on
//             a - 2 .. a)
//   stage C   colour 0, Monte Carlo, the tile only, plane a - 3 (reads colour 1 on
//             a - 4 .. a - 2, as stage B left them in earlier steps)
//
// The ring and the planes outside the tile's own belong to other workgroups, which
// compute them too, from the same inputs and the same Philox draws, hence to the same
// bits; so workgroups never communicate.  They read the spins before the launch from one
// buffer and write the tile after it to another, each site from registers after its
// last stage (colour 1 after stage B; colour 0 after stage A, or stage C when the launch
// carries the Monte Carlo pass).  Stage C runs on the tile only: the
// expensive Monte Carlo update is never recomputed, and the phase's spin traffic (the
// planes in LDS) serves the Monte Carlo pass too, as do the couplings stage A loads for
// the tile's sites: stage A takes those sites first, each thread the one it will update
// in stage C three steps later, and keeps its six couplings and its spin in registers.
//
// The site arithmetic (field of eq. 2 in the fixed order of the single-pass kernel, then
// the reflection of §4 or the k Metropolis hits / heat-bath draws) is the single pass's,
// so results equal the pass-by-pass schedule bit for bit; only the order in which the
// binary64 energy changes of stage C are summed differs.
#include <type_traits>

#include "hsg_device.h"
#include "hsg_internal.h"
#include "hsg_site.h"

namespace hsg {
namespace {

constexpr int kPTX = 32;      // colour sites of a tile row (64 sites in x)
constexpr int kHitGroup = 4;  // Monte Carlo hits whose draws are computed together

__device__ __forceinline__ int32_t wrap_to(int32_t v, int32_t n) {
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// The LDS window of a march with NS stages and THREADS threads.  Region column j holds
// colour column xh0 - OX + j, region row ry holds row y0 - OY + ry.  Colour 0 keeps K0
// planes, colour 1 K1 planes.
template <int NS, int K0_, int K1_, int THREADS_>
struct Win {
  static constexpr int OX = NS - 1;
  static constexpr int OY = NS;
  static constexpr int RX = kPTX + 2 * OX;
  static constexpr int RY = kPTY + 2 * OY;
  static constexpr int COLOUR = RY * RX;  // one colour, one component, one plane
  static constexpr int SLICE = 3 * COLOUR;  // one colour, three components, one plane
  static constexpr int K0 = K0_;
  static constexpr int K1 = K1_;
  static constexpr int THREADS = THREADS_;
  static constexpr int LOAD_ROUNDS = (SLICE + THREADS - 1) / THREADS;
};
using WinPhase = Win<2, 3, 3, kPhaseThreads>;  // the phase
using WinMc = Win<3, 3, 3, kPhaseThreads>;     // the phase and stage C

// The carried pass's colour-1 planes after stage B, three of them in a ring: the sites
// stage B updates (the tile widened by one row and one colour column on each side),
// the only ones stage C reads.
template <class W>
struct Compact {
  static constexpr int CX = kPTX + 2;
  static constexpr int CY = kPTY + 2;
  static constexpr int COLOUR = CX * CY;
  static constexpr int SLICE = 3 * COLOUR;
  static constexpr int X0 = W::OX - 1;  // region column of compact column 0
  static constexpr int Y0 = W::OY - 1;  // region row of compact row 0
};

template <typename R, class W>
__device__ __forceinline__ R* compact_slice(R* lds, int32_t q) {
  return lds + (W::K0 + W::K1) * W::SLICE + ((q + 9) % 3) * Compact<W>::SLICE;
}

// The sites a stage with ring H updates on one plane: rows OY - H .. OY + kPTY + H - 1,
// kPTX + H sites of the stage's colour in each.  On a row whose sites of that colour
// have x parity p, the first sits in region column OX - (H + p) / 2.
template <class W, int H>
struct StageShape {
  static constexpr int PER_ROW = kPTX + H;
  static constexpr int ROWS = kPTY + 2 * H;
  static constexpr int COUNT = PER_ROW * ROWS;
  static constexpr int RY0 = W::OY - H;
};

struct PhaseCtx {
  int32_t L, Lh;
  uint32_t Nh, zstride;  // N/2 and L/2 * L
  int32_t xh0, y0, z0;   // tile origin (colour column, row, plane)
};

// One colour of a region plane in registers: element e (component, row, column) of
// the slice, its colour-0 global offset without the plane's z offset (colour 1 adds
// 3 N/2).
template <class W>
struct SliceOffsets {
  uint32_t off[W::LOAD_ROUNDS];
};

template <typename R, class W>
struct SliceRegs {
  R v[W::LOAD_ROUNDS];
};

template <class W>
__device__ __forceinline__ void slice_offsets(SliceOffsets<W>& so, const PhaseCtx& m) {
#pragma unroll
  for (int k = 0; k < W::LOAD_ROUNDS; ++k) {
    const int32_t e = (int32_t)threadIdx.x + k * W::THREADS;
    const int32_t comp = e / W::COLOUR;
    const int32_t r = e - comp * W::COLOUR;
    const int32_t ry = r / W::RX;
    const int32_t j = r - ry * W::RX;
    const int32_t y = wrap_to(m.y0 - W::OY + ry, m.L);
    const int32_t xh = wrap_to(m.xh0 - W::OX + j, m.Lh);
    so.off[k] = (uint32_t)comp * m.Nh + (uint32_t)xh + (uint32_t)m.Lh * (uint32_t)y;
  }
}

template <typename R, class W>
__device__ __forceinline__ void fetch(SliceRegs<R, W>& sr, const SliceOffsets<W>& so,
                                      const R* in, const PhaseCtx& m, int32_t c, int32_t q) {
  const uint32_t base = (uint32_t)(3 * c) * m.Nh + m.zstride * (uint32_t)wrap_to(q, m.L);
#pragma unroll
  for (int k = 0; k < W::LOAD_ROUNDS; ++k)
    if ((int32_t)threadIdx.x + k * W::THREADS < W::SLICE) sr.v[k] = in[so.off[k] + base];
}

// Slice of colour c, plane q (q >= -8) in the colour's ring.
template <typename R, class W>
__device__ __forceinline__ R* slice(R* lds, int32_t c, int32_t q) {
  const int32_t slot = c == 0 ? (q + 8 * W::K0) % W::K0 : W::K0 + (q + 8 * W::K1) % W::K1;
  return lds + slot * W::SLICE;
}

template <typename R, class W>
__device__ __forceinline__ void put(R* lds, const SliceRegs<R, W>& sr, int32_t c, int32_t q) {
  R* dst = slice<R, W>(lds, c, q);
#pragma unroll
  for (int k = 0; k < W::LOAD_ROUNDS; ++k) {
    const int32_t e = (int32_t)threadIdx.x + k * W::THREADS;
    if (e < W::SLICE) dst[e] = sr.v[k];
  }
}

// Where site i of a stage with ring H (colour C) sits on plane q: region row and
// column, periodic z, y, colour column and the x parity of the row's colour-C sites.
struct SiteRef {
  int32_t z, ry, j, y, xh, p;
};

template <class W, int C, int H>
__device__ __forceinline__ SiteRef site_ref(const PhaseCtx& m, int32_t q, int32_t i) {
  using P = StageShape<W, H>;
  SiteRef r;
  r.z = wrap_to(q, m.L);
  const int32_t dr = i / P::PER_ROW;
  r.ry = P::RY0 + dr;
  r.y = wrap_to(m.y0 - W::OY + r.ry, m.L);
  r.p = (r.y + r.z + C) & 1;
  r.j = (i - dr * P::PER_ROW) + W::OX - ((H + r.p) >> 1);
  r.xh = wrap_to(m.xh0 - W::OX + r.j, m.Lh);
  return r;
}

// Site i of stage A with stage C behind it (NS = 3): the tile's sites first, in stage
// C's order (site i < kPTX * kPTY sits where stage C's site i does), then the ring of two
// sites: the two rows above and below the tile, then its first and last columns.
template <class W>
__device__ __forceinline__ SiteRef site_ref_a3(const PhaseCtx& m, int32_t q, int32_t i) {
  constexpr int PER = kPTX + 2;  // ring-2 row: 34 colour sites, columns 1 .. 34
  SiteRef r;
  r.z = wrap_to(q, m.L);
  if (i < kPTX * kPTY) {
    r.ry = W::OY + i / kPTX;
    r.j = W::OX + i % kPTX;
  } else {
    const int32_t k = i - kPTX * kPTY;
    if (k < 4 * PER) {
      const int32_t row = k / PER;  // 0, 1: above the tile; 2, 3: below it
      r.ry = row < 2 ? 1 + row : W::OY + kPTY + row - 2;
      r.j = 1 + (k - row * PER);
    } else {
      const int32_t e = k - 4 * PER;
      r.ry = W::OY + (e >> 1);
      r.j = (e & 1) ? PER : 1;
    }
  }
  r.y = wrap_to(m.y0 - W::OY + r.ry, m.L);
  r.p = (r.y + r.z) & 1;
  r.xh = wrap_to(m.xh0 - W::OX + r.j, m.Lh);
  return r;
}

// The six couplings of a site: +x,+y,+z bonds stored at the site (colour C planes),
// -x,-y,-z at its other-colour neighbours.
template <typename R>
struct Bonds {
  R px, mx, py, my, pz, mz;
};

template <typename R, int C>
__device__ __forceinline__ Bonds<R> site_bonds(const R* J, const PhaseCtx& m, const SiteRef& r) {
  const int32_t ym = r.y == 0 ? m.L - 1 : r.y - 1, zm = r.z == 0 ? m.L - 1 : r.z - 1;
  const int32_t xhm = r.p ? r.xh : (r.xh == 0 ? m.Lh - 1 : r.xh - 1);
  const uint32_t zo = m.zstride * (uint32_t)r.z;
  const uint32_t own = zo + (uint32_t)m.Lh * (uint32_t)r.y + (uint32_t)r.xh;
  const R* Jo = J + (uint32_t)(3 * C) * m.Nh;
  const R* Jn = J + (uint32_t)(3 * (1 - C)) * m.Nh;
  Bonds<R> b;
  b.px = Jo[own];
  b.mx = Jn[zo + (uint32_t)m.Lh * (uint32_t)r.y + (uint32_t)xhm];
  b.py = Jo[m.Nh + own];
  b.my = Jn[m.Nh + zo + (uint32_t)m.Lh * (uint32_t)ym + (uint32_t)r.xh];
  b.pz = Jo[2 * m.Nh + own];
  b.mz = Jn[2 * m.Nh + m.zstride * (uint32_t)zm + (uint32_t)m.Lh * (uint32_t)r.y +
            (uint32_t)r.xh];
  return b;
}

// Stage s (colour C = s & 1 for s < 2, colour 0 for s = 2; ring NS - 1 - s, none for
// s = 2) with a thread of the first T per site: thread threadIdx.x takes one site per
// round.  StageBonds holds the couplings of a thread's sites when they are loaded ahead
// of the stage.
template <class W, int S, int T>
struct Stage {
  static constexpr int C = S == 1 ? 1 : 0;
  static constexpr int H = S == 2 ? 0 : W::OX - S;
  static constexpr int COUNT = StageShape<W, H>::COUNT;
  static constexpr int ROUNDS = (COUNT + T - 1) / T;
  __device__ __forceinline__ static bool has(int r) {
    const int32_t i = (int32_t)threadIdx.x + r * T;
    return (int32_t)threadIdx.x < T && (COUNT % T == 0 || i < COUNT);
  }
};

template <typename R, class W, int S, int T>
struct StageBonds {
  Bonds<R> b[Stage<W, S, T>::ROUNDS];
};

template <typename R, class W, int S, int T>
__device__ __forceinline__ void fetch_bonds(StageBonds<R, W, S, T>& sb, const R* J,
                                            const PhaseCtx& m, int32_t q) {
  using St = Stage<W, S, T>;
#pragma unroll
  for (int r = 0; r < St::ROUNDS; ++r)
    if (St::has(r))
      sb.b[r] = site_bonds<R, St::C>(
          J, m, site_ref<W, St::C, St::H>(m, q, (int32_t)threadIdx.x + r * T));
}

// The local field of eq. 2 at a site from the spins of the other colour on three planes
// (components `cs` values apart, neighbours at the given offsets) and its couplings, in
// the fixed order of the single-pass kernel.
template <typename R>
__device__ __forceinline__ Vec3<R> plane_field(const R* cur, const R* up, const R* dn,
                                               int32_t cs, int32_t i_px, int32_t i_mx,
                                               int32_t i_py, int32_t i_my, int32_t i_z,
                                               const Bonds<R>& jb) {
  R hcomp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int32_t kb = k * cs;
    R acc = jb.px * cur[kb + i_px];
    acc = dev_fma(jb.mx, cur[kb + i_mx], acc);
    acc = dev_fma(jb.py, cur[kb + i_py], acc);
    acc = dev_fma(jb.my, cur[kb + i_my], acc);
    acc = dev_fma(jb.pz, up[kb + i_z], acc);
    acc = dev_fma(jb.mz, dn[kb + i_z], acc);
    hcomp[k] = acc;
  }
  return Vec3<R>{hcomp[0], hcomp[1], hcomp[2]};
}

__device__ __forceinline__ bool in_tile(int32_t ry, int32_t j, int32_t ox, int32_t oy) {
  return ry >= oy && ry < oy + kPTY && j >= ox && j < ox + kPTX;
}

template <typename R>
__device__ __forceinline__ void write_site(R* out, const PhaseCtx& m, int32_t c,
                                           const SiteRef& r, const Vec3<R>& s) {
  R* o = out + (uint32_t)(3 * c) * m.Nh + m.zstride * (uint32_t)r.z +
         (uint32_t)m.Lh * (uint32_t)r.y + (uint32_t)r.xh;
  o[0] = s.x;
  o[m.Nh] = s.y;
  o[2 * m.Nh] = s.z;
}

// Update of the site of colour C at r on plane q: the field of eq. 2 from the window
// (neighbour colour 1 - C) and the couplings jb, then (optionally renormalising before
// or after) apply_update.  The result goes back to the window when `keep` (with COMPACT,
// to the compact plane q instead); with `own_out` the tile's sites are also written to
// the output; with `spin_out` it is also returned there.
template <typename R, class W, int C, PassMode MODE, int G, bool COMPACT = false>
__device__ __forceinline__ double phase_site(R* lds, R* out, const PhaseCtx& m, int32_t q,
                                             const SiteRef& r, const Bonds<R>& jb,
                                             const HitCtx<R>& hc, bool renorm_before,
                                             bool renorm_after, bool keep, bool own_out,
                                             Vec3<R>* spin_out = nullptr) {
  const int32_t j = r.j;
  const int32_t row = r.ry * W::RX;
  const Vec3<R> h = plane_field<R>(
      slice<R, W>(lds, 1 - C, q), slice<R, W>(lds, 1 - C, q + 1), slice<R, W>(lds, 1 - C, q - 1),
      W::COLOUR, row + (r.p ? j + 1 : j), row + (r.p ? j : j - 1), row + W::RX + j,
      row - W::RX + j, row + j, jb);
  R* mine = slice<R, W>(lds, C, q);
  const int32_t io = row + j;
  Vec3<R> s{mine[io], mine[W::COLOUR + io], mine[2 * W::COLOUR + io]};
  if (renorm_before) s = unit_vector(s);
  const uint32_t site =
      (uint32_t)(2 * r.xh + r.p) + (uint32_t)m.L * (uint32_t)(r.y + m.L * r.z);
  const double d = apply_update<R, MODE, G>(s, h, site, hc);
  if (renorm_after) s = unit_vector(s);
  if (keep) {
    if constexpr (COMPACT) {
      using CP = Compact<W>;
      R* dst = compact_slice<R, W>(lds, q);
      const int32_t ic = (r.ry - CP::Y0) * CP::CX + (j - CP::X0);
      dst[ic] = s.x;
      dst[CP::COLOUR + ic] = s.y;
      dst[2 * CP::COLOUR + ic] = s.z;
    } else {
      mine[io] = s.x;
      mine[W::COLOUR + io] = s.y;
      mine[2 * W::COLOUR + io] = s.z;
    }
  }
  if (own_out && in_tile(r.ry, j, W::OX, W::OY)) write_site<R>(out, m, C, r, s);
  if (spin_out) *spin_out = s;
  return d;
}

// Stage C of the carried pass: the Monte Carlo update of colour-0 tile site r on plane q,
// its spin s (after the over-relaxation phase) and couplings jb kept in registers since
// stage A, the colour-1 neighbours from the compact planes q - 1 .. q + 1.  The result
// goes to the output.
template <typename R, class W, PassMode MODE, int G>
__device__ __forceinline__ double carried_site(R* lds, R* out, const PhaseCtx& m, int32_t q,
                                               const SiteRef& r, const Bonds<R>& jb, Vec3<R> s,
                                               const HitCtx<R>& hc, bool renorm_before) {
  using CP = Compact<W>;
  const int32_t j = r.j - CP::X0;
  const int32_t row = (r.ry - CP::Y0) * CP::CX;
  const Vec3<R> h = plane_field<R>(
      compact_slice<R, W>(lds, q), compact_slice<R, W>(lds, q + 1),
      compact_slice<R, W>(lds, q - 1), CP::COLOUR, row + (r.p ? j + 1 : j),
      row + (r.p ? j : j - 1), row + CP::CX + j, row - CP::CX + j, row + j, jb);
  if (renorm_before) s = unit_vector(s);
  const uint32_t site =
      (uint32_t)(2 * r.xh + r.p) + (uint32_t)m.L * (uint32_t)(r.y + m.L * r.z);
  const double d = apply_update<R, MODE, G>(s, h, site, hc);
  write_site<R>(out, m, 0, r, s);
  return d;
}

// Every site of stage s on plane q, with the couplings fetched for it (sb), or with
// PRE false loading each site's couplings just before its update (fewer registers).
template <typename R, class W, int S, PassMode MODE, int G, int T, bool PRE,
          bool COMPACT = false>
__device__ __forceinline__ double stage(R* lds, const R* J, R* out, const PhaseCtx& m,
                                        int32_t q, const StageBonds<R, W, S, T>& sb,
                                        const HitCtx<R>& hc, bool renorm_before,
                                        bool renorm_after, bool keep, bool own_out) {
  using St = Stage<W, S, T>;
  double d = 0.0;
#pragma unroll
  for (int r = 0; r < St::ROUNDS; ++r) {
    if (St::has(r)) {
      const SiteRef ref = site_ref<W, St::C, St::H>(m, q, (int32_t)threadIdx.x + r * T);
      const Bonds<R> jb = PRE ? sb.b[r] : site_bonds<R, St::C>(J, m, ref);
      d += phase_site<R, W, St::C, MODE, G, COMPACT>(lds, out, m, q, ref, jb, hc, renorm_before,
                                                     renorm_after, keep, own_out);
    }
  }
  return d;
}

__device__ __forceinline__ PhaseCtx phase_ctx(int32_t L, int32_t zp) {
  const int32_t tiles_x = L / 2 / kPTX, tiles_y = L / kPTY;
  const int32_t tile = xcd_tile((int32_t)blockIdx.x, (int32_t)gridDim.x);
  const int32_t tx = tile % tiles_x;
  const int32_t rest = tile / tiles_x;
  const int32_t ty = rest % tiles_y, tz = rest / tiles_y;
  PhaseCtx m;
  m.L = L;
  m.Lh = L / 2;
  m.zstride = (uint32_t)m.Lh * (uint32_t)L;
  m.Nh = m.zstride * (uint32_t)L;
  m.xh0 = tx * kPTX;
  m.y0 = ty * kPTY;
  m.z0 = tz * zp;
  return m;
}

// Before step 0 (stage A on plane z0 - NS + 1): colour 1 of planes z0 - NS .. z0 - NS
// + 2 and colour 0 of plane z0 - NS + 1 in LDS; in registers the slices the end of step
// 0 puts in place.
template <typename R, class W, int NS>
__device__ __forceinline__ void prologue(R* lds, SliceRegs<R, W>& r0, SliceRegs<R, W>& r1,
                                         const SliceOffsets<W>& so, const R* in,
                                         const PhaseCtx& m) {
  for (int32_t q = m.z0 - NS; q <= m.z0 - NS + 2; ++q) {
    fetch<R, W>(r1, so, in, m, 1, q);
    put<R, W>(lds, r1, 1, q);
  }
  fetch<R, W>(r0, so, in, m, 0, m.z0 - NS + 1);
  put<R, W>(lds, r0, 0, m.z0 - NS + 1);
  fetch<R, W>(r0, so, in, m, 0, m.z0 - NS + 2);
  fetch<R, W>(r1, so, in, m, 1, m.z0 - NS + 3);
}

// The over-relaxation phase alone (stages A and B): each step stage A on plane q, stage
// B on plane q - 1, then the next planes into the window.  The couplings of a stage's
// sites are loaded a step ahead (the loads stay in flight across the barriers).
template <typename R>
__global__ __launch_bounds__(kPhaseThreads) void phase_kernel(PhaseArgs<R> a) {
  using W = WinPhase;
  constexpr PassMode OR = PassMode::OverRelax;
  constexpr int T = kPhaseThreads;
  constexpr int STEPS = kPZ + 2;
  __shared__ R lds[(W::K0 + W::K1) * W::SLICE];
  const PhaseCtx m = phase_ctx(a.L, kPZ);
  const HitCtx<R> hc{a.beta, a.sweep, a.phase, a.k_hits, a.seed_lo, a.seed_hi};
  SliceOffsets<W> so;
  slice_offsets<W>(so, m);
  SliceRegs<R, W> r0, r1;
  prologue<R, W, 2>(lds, r0, r1, so, a.in, m);
  StageBonds<R, W, 0, T> bA;
  StageBonds<R, W, 1, T> bB;
  fetch_bonds<R, W, 0, T>(bA, a.J, m, m.z0 - 1);
  for (int32_t t = 0; t < STEPS; ++t) {
    const int32_t q = m.z0 - 1 + t;  // stage A's plane; stage B on q - 1
    __syncthreads();
    // colour 0 of plane q is final after stage A: its tile goes out from there
    const bool own_a = q >= m.z0 && q < m.z0 + kPZ;
    stage<R, W, 0, OR, 1, T, true>(lds, a.J, a.out, m, q, bA, hc, false, false, true, own_a);
    if (t + 1 < STEPS) fetch_bonds<R, W, 0, T>(bA, a.J, m, q + 1);
    if (t == 1) fetch_bonds<R, W, 1, T>(bB, a.J, m, q);
    __syncthreads();
    if (t >= 2) {
      // colour 1 of plane q - 1 is final after stage B and read by no later stage: its
      // tile goes out from there, nothing back to the window
      const bool own = q - 1 >= m.z0 && q - 1 < m.z0 + kPZ;
      stage<R, W, 1, OR, 1, T, true>(lds, a.J, a.out, m, q - 1, bB, hc, false, false, false,
                                     own);
      if (t + 1 < STEPS) fetch_bonds<R, W, 1, T>(bB, a.J, m, q);
    }
    __syncthreads();
    if (t < STEPS - 1) {
      // colour 0 of plane q + 1 replaces plane q - 2 (last read by stage B), colour 1 of
      // plane q + 2 replaces plane q - 1 (last read this step)
      put<R, W>(lds, r0, 0, q + 1);
      put<R, W>(lds, r1, 1, q + 2);
      if (t < STEPS - 2) {
        fetch<R, W>(r0, so, a.in, m, 0, q + 2);
        fetch<R, W>(r1, so, a.in, m, 1, q + 3);
      }
    }
  }
}

// The phase, then the colour-0 pass of the next sweep's Monte Carlo phase in mode MC
// (stage C), each step in three intervals between barriers:
//
//   1. stage C on plane q - 3, then stage A on plane q
//   2. stage B on plane q - 1, its results to the compact plane q - 1
//   3. the next planes into the window
//
// Stage C reads colour 1 only from the compact planes q - 4 .. q - 2, which stage B
// finished in earlier steps, so it shares an interval with stage A, and its own spins
// and couplings come from registers: this thread's tile site as stage A left it three
// steps earlier.  So the window keeps three planes of each colour.
template <typename R, PassMode MC>
__global__ __launch_bounds__(kPhaseThreads)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2))) void phase_mc_kernel(PhaseArgs<R> a) {
  using W = WinMc;
  using CP = Compact<W>;
  using StA = StageShape<W, 2>;
  constexpr PassMode OR = PassMode::OverRelax;
  constexpr int T = kPhaseThreads;
  constexpr int RA = (StA::COUNT + T - 1) / T;  // stage A rounds
  constexpr int LAST_A = kPZ + 3;                // stage A on planes z0 - 2 .. z0 + kPZ + 1
  constexpr int FIRST_C = 5;                     // stage C on planes z0 .. z0 + kPZ - 1
  constexpr int STEPS = kPZ + FIRST_C;
  // binary32 keeps stage C's couplings in registers from stage A; binary64 (one
  // workgroup per compute unit, twice the registers per value) loads them again
  constexpr bool KEEP_BONDS = sizeof(R) == 4;
  static_assert(T == kPTX * kPTY, "one stage-C site per thread");
  __shared__ R lds[(W::K0 + W::K1) * W::SLICE + 3 * CP::SLICE];
  const PhaseCtx m = phase_ctx(a.L, kPZ);
  const HitCtx<R> hc{a.beta, a.sweep, a.phase, a.k_hits, a.seed_lo, a.seed_hi};
  const HitCtx<R> hm{a.beta, a.mc_sweep, 0u, a.k_hits, a.seed_lo, a.seed_hi};
  const bool rn = a.renorm != 0;
  SliceOffsets<W> so;
  slice_offsets<W>(so, m);
  SliceRegs<R, W> r0, r1;
  prologue<R, W, 3>(lds, r0, r1, so, a.in, m);
  StageBonds<R, W, 1, T> unused;
  // this thread's tile site as stage A left it one, two and three steps ago
  Bonds<R> b1{}, b2{}, b3{};
  Vec3<R> s1{}, s2{}, s3{};
  double dE = 0.0;
  for (int32_t t = 0; t < STEPS; ++t) {
    const int32_t q = m.z0 - 2 + t;  // stage A's plane; stage B on q - 1, C on q - 3
    __syncthreads();
    // Interval 1: stage C, then stage A (stage C consumes the oldest registers before
    // stage A fills new ones).  Waves take a priority by stage (0 in stage C, 3 in stage
    // A and the plane loads, 2 in stage B), so that one of the two workgroups on a compute
    // unit issues first while they are in different stages.
    if (t >= FIRST_C) {
      __builtin_amdgcn_s_setprio(0);
      const SiteRef ref = site_ref<W, 0, 0>(m, q - 3, (int32_t)threadIdx.x);
      const Bonds<R> jb = KEEP_BONDS ? b3 : site_bonds<R, 0>(a.J, m, ref);
      dE += carried_site<R, W, MC, kHitGroup>(lds, a.out, m, q - 3, ref, jb, s3, hm, rn);
    }
    Bonds<R> b0 = b1;
    Vec3<R> s0 = s1;
    if (t <= LAST_A) {
      __builtin_amdgcn_s_setprio(3);
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        const int32_t i = (int32_t)threadIdx.x + r * T;
        if (i < StA::COUNT) {
          const SiteRef ref = site_ref_a3<W>(m, q, i);
          const Bonds<R> jb = site_bonds<R, 0>(a.J, m, ref);
          if (KEEP_BONDS && r == 0) b0 = jb;
          phase_site<R, W, 0, OR, 1>(lds, a.out, m, q, ref, jb, hc, false, false, true, false,
                                     r == 0 ? &s0 : nullptr);
        }
      }
    }
    b3 = b2;
    b2 = b1;
    b1 = b0;
    s3 = s2;
    s2 = s1;
    s1 = s0;
    __syncthreads();
    // Interval 2: stage B.  Colour 1 of plane q - 1 is final: its tile goes out from
    // there, the sites stage C reads to the compact plane.
    if (t >= 2 && t <= LAST_A) {
      __builtin_amdgcn_s_setprio(2);
      const bool own = q - 1 >= m.z0 && q - 1 < m.z0 + kPZ;
      stage<R, W, 1, OR, 1, T, false, true>(lds, a.J, a.out, m, q - 1, unused, hc, false, rn,
                                            true, own);
    }
    __syncthreads();
    // Interval 3: colour 0 of plane q + 1 replaces plane q - 2 and colour 1 of plane q + 2
    // replaces plane q - 1, both last read by stage B above; the planes of the next step's
    // end are loaded (in flight through the next step).
    __builtin_amdgcn_s_setprio(3);
    if (t < LAST_A) {
      put<R, W>(lds, r0, 0, q + 1);
      put<R, W>(lds, r1, 1, q + 2);
      if (t + 1 < LAST_A) {
        fetch<R, W>(r0, so, a.in, m, 0, q + 2);
        fetch<R, W>(r1, so, a.in, m, 1, q + 3);
      }
    }
  }
  __shared__ double s_red[16];
  const double total = block_sum(dE, s_red);
  if (threadIdx.x == 0) a.partials[blockIdx.x] += total;
}

template <typename R>
hipError_t launch_alone(const PhaseArgs<R>& a, hipStream_t st) {
  const dim3 grid((unsigned)phase_blocks(a.L)), block(kPhaseThreads);
  hipLaunchKernelGGL((phase_kernel<R>), grid, block, 0, st, a);
  return hipGetLastError();
}

template <typename R, PassMode MC>
hipError_t launch_mc(const PhaseArgs<R>& a, hipStream_t st) {
  const dim3 grid((unsigned)phase_blocks(a.L)), block(kPhaseThreads);
  hipLaunchKernelGGL((phase_mc_kernel<R, MC>), grid, block, 0, st, a);
  return hipGetLastError();
}

}  // namespace

bool phase_supported(int32_t L) {
  return L >= kPhaseMinL && L <= kPhaseMaxL && L % (2 * kPTX) == 0 && L % kPTY == 0 &&
         L % kPZ == 0;
}

int32_t phase_blocks(int32_t L) { return (L / 2 / kPTX) * (L / kPTY) * (L / kPZ); }

template <typename R>
hipError_t launch_phase(const PhaseArgs<R>& a, hipStream_t st) {
  if (!phase_supported(a.L)) return hipErrorInvalidValue;
  if (!a.then_mc) return launch_alone<R>(a, st);
  if (!a.partials) return hipErrorInvalidValue;
  const PassMode mc = (PassMode)a.mc_mode == PassMode::HeatBath ? PassMode::HeatBath
                       : metropolis_mode(a.k_hits);
  if ((PassMode)a.mc_mode == PassMode::OverRelax) return hipErrorInvalidValue;
  if (mc == PassMode::MetropolisFull) return launch_mc<R, PassMode::MetropolisFull>(a, st);
  if (mc == PassMode::Metropolis) return launch_mc<R, PassMode::Metropolis>(a, st);
  return launch_mc<R, PassMode::HeatBath>(a, st);
}

template hipError_t launch_phase<float>(const PhaseArgs<float>&, hipStream_t);
template hipError_t launch_phase<double>(const PhaseArgs<double>&, hipStream_t);

}  // namespace hsg
