// Fused colour passes: one launch runs up to four consecutive colour passes of the
// checkerboard schedule (§4) -- e.g. the two over-relaxation passes of sweep n and the
// two Metropolis passes of sweep n + 1 -- reading the spins from HBM once and writing
// them once, instead of once per pass.
//
// Each workgroup owns a TX x TY x ZC block of sites and marches through its planes in
// z, holding a window of S + 2 planes of its block, widened by S sites on each side in
// x and y, in LDS.  A pass only reads the other colour on planes z-1..z+1, so pass s
// can follow pass s-1 one plane behind: at march step t, pass s updates plane
// P(t) - s.  Pass s also updates a ring of S-1-s sites around the block (and as many
// extra planes in z), so that pass s+1 finds every neighbour it needs already updated:
// those halo sites belong to other workgroups, which compute them too, from the same
// inputs and the same Philox draws, hence to the same bits.  Workgroups therefore never
// communicate; they read the state before the launch from one buffer and write the
// block's final state to another.  The couplings are read from global memory by every
// pass; the workgroups of one XCD take neighbouring blocks of the same z range, so the
// couplings of the planes they are working on stay in that XCD's L2.
//
// The site update itself (field of eq. 2 in the fixed order, then apply_update) is the
// one the single-pass kernel uses, so results equal the pass-by-pass schedule bit for
// bit; only the order in which the binary64 energy changes are summed differs.
#include "hsg_device.h"
#include "hsg_internal.h"
#include "hsg_site.h"

namespace hsg {
namespace {

constexpr int kTX = 64;       // block extent in x (sites); 32 sites of each colour per row
constexpr int kTY = 16;       // block extent in y
constexpr int kThreads = 640;
constexpr int kHitGroup = 4;  // hits whose draws are computed together (see apply_update)

__device__ __forceinline__ int32_t wrap(int32_t v, int32_t n) {
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

template <typename R, int S>
struct Block {
  static constexpr int RX = kTX + 2 * S;  // region extent in x (sites)
  static constexpr int RXh = RX / 2;      // sites of one colour per region row
  static constexpr int RY = kTY + 2 * S;
  static constexpr int W = S + 2;         // planes in the window
  static constexpr int ROW = RXh;
  static constexpr int COLOUR = RY * RXh;
  static constexpr int COMP = 2 * COLOUR;
  static constexpr int PLANE = 3 * COMP;  // values of one plane of the region
};

// Offsets below are 32-bit element offsets from the array base: 6 N/2 < 2^32 for the
// lattices the fused passes accept (L <= 1024).
template <typename R>
struct MarchCtx {
  const R* in;
  R* out;
  const R* J;
  int32_t L, Lh;
  uint32_t Nh, zstride;    // N/2 and the sites of one colour per z plane (L/2 * L)
  int32_t x0, y0, z0, zc;  // region origin in x and y (may be negative), block's first plane
};


// Plane q of the region into registers (a thread's share: element threadIdx.x +
// k * kThreads of the slot), then from registers into the window slot: the load is
// issued a whole march step before the values are needed.  The in-plane part of each
// element's global offset is fixed for the launch.
template <typename R, int S>
struct PlaneRegs {
  static constexpr int N = (Block<R, S>::PLANE + kThreads - 1) / kThreads;
  uint32_t off[N];
  R v[N];
};

template <typename R, int S>
__device__ __forceinline__ void plane_offsets(PlaneRegs<R, S>& pr, const MarchCtx<R>& m) {
  using B = Block<R, S>;
  const int32_t xh0 = m.x0 >> 1;  // x0 is even
#pragma unroll
  for (int k = 0; k < PlaneRegs<R, S>::N; ++k) {
    const int32_t e = (int32_t)threadIdx.x + k * kThreads;
    const int32_t comp = e / B::COMP;
    const int32_t r1 = e - comp * B::COMP;
    const int32_t c = r1 / B::COLOUR;
    const int32_t r2 = r1 - c * B::COLOUR;
    const int32_t ry = r2 / B::ROW;
    const int32_t j = r2 - ry * B::ROW;
    const int32_t y = wrap(m.y0 + ry, m.L);
    const int32_t xh = wrap(xh0 + j, m.Lh);
    pr.off[k] = (uint32_t)(3 * c + comp) * m.Nh + (uint32_t)xh + (uint32_t)m.Lh * (uint32_t)y;
  }
}

template <typename R, int S>
__device__ __forceinline__ void fetch_plane(PlaneRegs<R, S>& pr, const MarchCtx<R>& m, int32_t q) {
  const int32_t z = q < 0 ? q + m.L : (q >= m.L ? q - m.L : q);  // q within S planes of [0, L)
  const uint32_t zo = m.zstride * (uint32_t)z;
#pragma unroll
  for (int k = 0; k < PlaneRegs<R, S>::N; ++k) {
    if ((int32_t)threadIdx.x + k * kThreads < Block<R, S>::PLANE) pr.v[k] = m.in[pr.off[k] + zo];
  }
}

template <typename R, int S>
__device__ __forceinline__ void put_plane(R* lds, const PlaneRegs<R, S>& pr, int32_t q) {
  using B = Block<R, S>;
  R* dst = lds + ((q + B::W * 64) % B::W) * B::PLANE;  // q >= -S
#pragma unroll
  for (int k = 0; k < PlaneRegs<R, S>::N; ++k) {
    const int32_t e = (int32_t)threadIdx.x + k * kThreads;
    if (e < B::PLANE) dst[e] = pr.v[k];
  }
}

// Writes the block's own sites (both colours) of plane q (inside [0, L)) to the output.
template <typename R, int S>
__device__ __forceinline__ void store_plane(const R* lds, const MarchCtx<R>& m, int32_t q) {
  using B = Block<R, S>;
  const R* src = lds + (q % B::W) * B::PLANE;
  constexpr int HALF = kTX / 2;
  constexpr int COUNT = 3 * 2 * kTY * HALF;
  const uint32_t base = (uint32_t)((m.x0 + S) >> 1) +
                        (uint32_t)m.Lh * (uint32_t)(m.y0 + S) + m.zstride * (uint32_t)q;
#pragma unroll
  for (int k = 0; k < (COUNT + kThreads - 1) / kThreads; ++k) {
    const int32_t e = (int32_t)threadIdx.x + k * kThreads;
    if (e < COUNT) {
      const int32_t row = e / HALF, j = e - row * HALF;
      const int32_t comp = row / (2 * kTY);
      const int32_t r1 = row - comp * 2 * kTY;
      const int32_t c = r1 / kTY, iy = r1 - c * kTY;
      const R v = src[comp * B::COMP + c * B::COLOUR + (S + iy) * B::ROW + (S / 2 + j)];
      m.out[(uint32_t)(3 * c + comp) * m.Nh + base + (uint32_t)j + (uint32_t)m.Lh * (uint32_t)iy] = v;
    }
  }
}

// The sites a pass with halo H updates on one plane: rows ry in [S-H, S+TY+H) of the
// region, in each the TX/2 + H sites of the pass's colour between columns S-H and
// S+TX+H.  Site i of the pass sits in row S-H + i / (TX/2 + H); on a plane where the
// row's sites of colour c have x parity b it is column rx = 2j + b.
template <int S, int H>
struct PassShape {
  static constexpr int PER_ROW = kTX / 2 + H;
  static constexpr int ROWS = kTY + 2 * H;
  static constexpr int COUNT = PER_ROW * ROWS;
  static constexpr int ROUNDS = (COUNT + kThreads - 1) / kThreads;
  static constexpr int R0 = S - H;
};

struct PassSite {
  int32_t ry, j, b, rx;
};

// The plane a pass works on in one march step, resolved once per step (uniform):
// periodic z and z-1, the window slots of planes q, q+1, q-1, and whether q is one of
// the block's own planes.
struct PlaneRef {
  int32_t z, zm;
  int32_t cur, up, dn;
  bool own;
};

template <int S>
__device__ __forceinline__ PlaneRef plane_ref(int32_t q, int32_t L, int32_t z0, int32_t zc) {
  constexpr int W = S + 2;
  PlaneRef r;
  r.z = q < 0 ? q + L : (q >= L ? q - L : q);  // q is within S planes of [0, L)
  r.zm = r.z == 0 ? L - 1 : r.z - 1;
  const int32_t sq = (q + W * 64) % W;  // q >= -S > -64 W
  r.cur = sq;
  r.up = sq + 1 == W ? 0 : sq + 1;
  r.dn = sq == 0 ? W - 1 : sq - 1;
  r.own = q >= z0 && q < z0 + zc;
  return r;
}

template <int S, int H>
__device__ __forceinline__ PassSite pass_site(int32_t i, int32_t c, int32_t parity) {
  using P = PassShape<S, H>;
  PassSite ps;
  const int32_t dr = i / P::PER_ROW;
  ps.ry = P::R0 + dr;
  ps.b = (c + ps.ry + parity) & 1;
  ps.j = ((P::R0 - ps.b + 1) >> 1) + (i - dr * P::PER_ROW);
  ps.rx = 2 * ps.j + ps.b;
  return ps;
}

// The six couplings of a site: +x,+y,+z bonds stored at the site, -x,-y,-z at its
// other-colour neighbours (read-only, from global memory).
template <typename R>
struct Bonds {
  R px, mx, py, my, pz, mz;
};

template <typename R, int S, int H, int C>
__device__ __forceinline__ Bonds<R> fetch_bonds(const MarchCtx<R>& m, int32_t i,
                                                const PlaneRef& pl) {
  Bonds<R> o{};
  if (i >= PassShape<S, H>::COUNT) return o;
  const int32_t z = pl.z, zm = pl.zm;
  const PassSite ps = pass_site<S, H>(i, C, z + m.x0 + m.y0);
  const int32_t x = wrap(m.x0 + ps.rx, m.L), y = wrap(m.y0 + ps.ry, m.L);
  const int32_t xm = x == 0 ? m.L - 1 : x - 1, ym = y == 0 ? m.L - 1 : y - 1;
  const uint32_t zo = m.zstride * (uint32_t)z, zmo = m.zstride * (uint32_t)zm;
  const uint32_t yo = (uint32_t)m.Lh * (uint32_t)y, ymo = (uint32_t)m.Lh * (uint32_t)ym;
  const uint32_t xo = (uint32_t)(x >> 1), xmo = (uint32_t)(xm >> 1);
  const R* Jo = m.J + (uint32_t)(3 * C) * m.Nh;        // this colour's bonds
  const R* Jn = m.J + (uint32_t)(3 * (1 - C)) * m.Nh;  // the other colour's
  const uint32_t own = zo + yo + xo;
  o.px = Jo[own];
  o.mx = Jn[zo + yo + xmo];
  o.py = Jo[m.Nh + own];
  o.my = Jn[m.Nh + zo + ymo + xo];
  o.pz = Jo[2 * m.Nh + own];
  o.mz = Jn[2 * m.Nh + zmo + yo + xo];
  return o;
}

// Site i of pass `st` (halo H, colour C) on plane q: local field from the window (eq.
// 2, the fixed order of the single-pass kernel), then the update.  Returns the energy
// change when the site is one of the block's own, else 0.
template <typename R, int S, int H, int C, PassMode MODE>
__device__ __forceinline__ double march_site(R* lds, const MarchCtx<R>& m, const MarchStage& st,
                                             const PlaneRef& pl, int32_t i, const Bonds<R>& jb,
                                             const HitCtx<R>& hc) {
  using B = Block<R, S>;
  if (i >= PassShape<S, H>::COUNT) return 0.0;
  const int32_t z = pl.z;
  const PassSite ps = pass_site<S, H>(i, C, z + m.x0 + m.y0);
  R* cur = lds + pl.cur * B::PLANE;
  const R* up = lds + pl.up * B::PLANE;
  const R* dn = lds + pl.dn * B::PLANE;
  constexpr int nc = (1 - C) * B::COLOUR;
  const int32_t row_o = nc + ps.ry * B::ROW;
  const int32_t i_px = row_o + ps.j + ps.b, i_mx = row_o + ps.j + ps.b - 1;
  const int32_t i_py = row_o + B::ROW + ps.j, i_my = row_o - B::ROW + ps.j;
  const int32_t i_z = row_o + ps.j;
  R hcomp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int32_t kb = k * B::COMP;
    R acc = jb.px * cur[kb + i_px];
    acc = dev_fma(jb.mx, cur[kb + i_mx], acc);
    acc = dev_fma(jb.py, cur[kb + i_py], acc);
    acc = dev_fma(jb.my, cur[kb + i_my], acc);
    acc = dev_fma(jb.pz, up[kb + i_z], acc);
    acc = dev_fma(jb.mz, dn[kb + i_z], acc);
    hcomp[k] = acc;
  }
  const Vec3<R> h{hcomp[0], hcomp[1], hcomp[2]};
  const int32_t io = C * B::COLOUR + ps.ry * B::ROW + ps.j;
  Vec3<R> s{cur[io], cur[B::COMP + io], cur[2 * B::COMP + io]};
  if (st.renorm_before) s = unit_vector(s);
  const int32_t x = wrap(m.x0 + ps.rx, m.L), y = wrap(m.y0 + ps.ry, m.L);
  const uint32_t site = (uint32_t)x + (uint32_t)m.L * (uint32_t)(y + m.L * z);
  const double d = apply_update<R, MODE, kHitGroup>(s, h, site, hc);
  if (st.renorm_after) s = unit_vector(s);
  cur[io] = s.x;
  cur[B::COMP + io] = s.y;
  cur[2 * B::COMP + io] = s.z;
  const bool own = pl.own && ps.ry >= S && ps.ry < S + kTY && ps.rx >= S && ps.rx < S + kTX;
  return own ? d : 0.0;
}

// Bonds of the (at most two) sites a thread handles in one pass.
template <typename R>
struct PassBonds {
  Bonds<R> v[2];
};

template <typename R, int S, int s>
__device__ __forceinline__ PassBonds<R> fetch_pass_bonds(const MarchCtx<R>& m,
                                                         const PlaneRef& pl) {
  constexpr int H = S - 1 - s;
  static_assert(PassShape<S, H>::ROUNDS <= 2, "too many sites per thread");
  PassBonds<R> pb;
#pragma unroll
  for (int r = 0; r < PassShape<S, H>::ROUNDS; ++r)
    pb.v[r] = fetch_bonds<R, S, H, s & 1>(m, (int32_t)threadIdx.x + r * kThreads, pl);
  return pb;
}

template <typename R, int S, int s, PassMode MODE>
__device__ __forceinline__ double march_pass(R* lds, const MarchCtx<R>& m, const MarchArgs<R>& a,
                                             const PassBonds<R>& pb, const PlaneRef& pl) {
  constexpr int H = S - 1 - s;
  const MarchStage& st = a.st[s];
  const HitCtx<R> hc{a.beta, st.sweep, st.phase, a.k_hits, a.seed_lo, a.seed_hi};
  double dE = 0.0;
#pragma unroll
  for (int r = 0; r < PassShape<S, H>::ROUNDS; ++r)
    dE += march_site<R, S, H, s & 1, MODE>(lds, m, st, pl, (int32_t)threadIdx.x + r * kThreads,
                                           pb.v[r], hc);
  return dE;
}

// S passes per launch; passes 0 and 1 run mode M0, passes 2 and 3 mode M1.  Pass s
// updates colour s & 1.
template <typename R, int S, PassMode M0, PassMode M1>
__global__ __launch_bounds__(kThreads) void march_kernel(MarchArgs<R> a) {
  using B = Block<R, S>;
  __shared__ R lds[B::W * B::PLANE];
  __shared__ double s_red[16];
  // blocks in (x, y, z-range) order, each XCD taking a contiguous range of them
  const int32_t tile = xcd_tile((int32_t)blockIdx.x, (int32_t)gridDim.x);
  const int32_t bx = tile % a.tiles_x;
  const int32_t rest = tile / a.tiles_x;
  const int32_t by = rest % a.tiles_y, bz = rest / a.tiles_y;
  MarchCtx<R> m;
  m.in = a.in;
  m.out = a.out;
  m.J = a.J;
  m.L = a.L;
  m.Lh = a.L / 2;
  m.zstride = (uint32_t)m.Lh * (uint32_t)a.L;
  m.Nh = m.zstride * (uint32_t)a.L;
  m.x0 = bx * kTX - S;
  m.y0 = by * kTY - S;
  m.zc = a.zc;
  m.z0 = bz * a.zc;

  // window: planes z0-S and z0-S+1 now; plane P+1 of step t is fetched into registers
  // during step t-1.  The bonds of each pass are fetched while the previous pass runs.
  PlaneRegs<R, S> pr;
  plane_offsets<R, S>(pr, m);
  fetch_plane<R, S>(pr, m, m.z0 - S);
  put_plane<R, S>(lds, pr, m.z0 - S);
  fetch_plane<R, S>(pr, m, m.z0 - S + 1);
  put_plane<R, S>(lds, pr, m.z0 - S + 1);
  fetch_plane<R, S>(pr, m, m.z0 - S + 2);
  auto ref = [&](int32_t q) { return plane_ref<S>(q, m.L, m.z0, m.zc); };
  PassBonds<R> bc = fetch_pass_bonds<R, S, 0>(m, ref(m.z0 - S + 1)), bn;

  double dE = 0.0;
  const int32_t n_steps = a.zc + 2 * S - 2;
  for (int32_t t = 0; t < n_steps; ++t) {
    const int32_t P = m.z0 - S + 1 + t;
    const PlaneRef p0 = ref(P), p1 = ref(P - 1);
    put_plane<R, S>(lds, pr, P + 1);
    if (t + 1 < n_steps) fetch_plane<R, S>(pr, m, P + 2);
    __syncthreads();
    bn = fetch_pass_bonds<R, S, 1>(m, p1);
    dE += march_pass<R, S, 0, M0>(lds, m, a, bc, p0);
    __syncthreads();
    bc = bn;
    if constexpr (S == 4) {
      const PlaneRef p2 = ref(P - 2), p3 = ref(P - 3);
      bn = fetch_pass_bonds<R, S, 2>(m, p2);
      if (t >= 2) dE += march_pass<R, S, 1, M0>(lds, m, a, bc, p1);
      __syncthreads();
      bc = bn;
      bn = fetch_pass_bonds<R, S, 3>(m, p3);
      if (t >= 4) dE += march_pass<R, S, 2, M1>(lds, m, a, bc, p2);
      __syncthreads();
      bc = bn;
      bn = fetch_pass_bonds<R, S, 0>(m, ref(P + 1));
      if (t >= 6) dE += march_pass<R, S, 3, M1>(lds, m, a, bc, p3);
      __syncthreads();
    } else {
      bn = fetch_pass_bonds<R, S, 0>(m, ref(P + 1));
      if (t >= 2) dE += march_pass<R, S, 1, M0>(lds, m, a, bc, p1);
      __syncthreads();
    }
    bc = bn;
    if (t >= 2 * S - 2) store_plane<R, S>(lds, m, P - (S - 1));
  }
  const double total = block_sum(dE, s_red);
  if (threadIdx.x == 0) a.partials[blockIdx.x] += total;
}

template <typename R, int S>
hipError_t launch_modes(const MarchArgs<R>& a, PassMode m0, PassMode m1, hipStream_t st) {
  const dim3 grid((unsigned)march_blocks(a.L)), block(kThreads);
  using PM = PassMode;
#define HSG_MARCH(M0, M1) hipLaunchKernelGGL((march_kernel<R, S, M0, M1>), grid, block, 0, st, a)
  if constexpr (S == 2) {
    (void)m1;
    if (m0 == PM::Metropolis) HSG_MARCH(PM::Metropolis, PM::Metropolis);
    else if (m0 == PM::HeatBath) HSG_MARCH(PM::HeatBath, PM::HeatBath);
    else HSG_MARCH(PM::OverRelax, PM::OverRelax);
  } else {
    if (m0 == PM::OverRelax && m1 == PM::OverRelax) HSG_MARCH(PM::OverRelax, PM::OverRelax);
    else if (m0 == PM::OverRelax && m1 == PM::Metropolis) HSG_MARCH(PM::OverRelax, PM::Metropolis);
    else if (m0 == PM::OverRelax && m1 == PM::HeatBath) HSG_MARCH(PM::OverRelax, PM::HeatBath);
    else if (m0 == PM::Metropolis && m1 == PM::OverRelax) HSG_MARCH(PM::Metropolis, PM::OverRelax);
    else if (m0 == PM::HeatBath && m1 == PM::OverRelax) HSG_MARCH(PM::HeatBath, PM::OverRelax);
    else if (m0 == PM::Metropolis && m1 == PM::Metropolis) HSG_MARCH(PM::Metropolis, PM::Metropolis);
    else if (m0 == PM::HeatBath && m1 == PM::HeatBath) HSG_MARCH(PM::HeatBath, PM::HeatBath);
    else return hipErrorInvalidValue;
  }
#undef HSG_MARCH
  return hipGetLastError();
}

}  // namespace

bool march_supported(int32_t L) {
  return L >= kMarchMinL && L <= kMarchMaxL && L % kTX == 0 && L % kTY == 0 && L % kMarchZ == 0;
}

int32_t march_blocks(int32_t L) { return (L / kTX) * (L / kTY) * (L / kMarchZ); }

template <typename R>
int32_t march_max_stages() {
  return sizeof(R) == 4 ? 4 : 2;
}

template <typename R>
hipError_t launch_march(const MarchArgs<R>& a0, int32_t n_stages, hipStream_t st) {
  MarchArgs<R> a = a0;
  a.tiles_x = a.L / kTX;
  a.tiles_y = a.L / kTY;
  a.zc = kMarchZ;
  const PassMode m0 = (PassMode)a.st[0].mode;
  const PassMode m1 = n_stages > 2 ? (PassMode)a.st[2].mode : m0;
  if (n_stages == 2) return launch_modes<R, 2>(a, m0, m1, st);
  if constexpr (sizeof(R) == 4) {
    if (n_stages == 4) return launch_modes<R, 4>(a, m0, m1, st);
  }
  return hipErrorInvalidValue;
}

template int32_t march_max_stages<float>();
template int32_t march_max_stages<double>();
template hipError_t launch_march<float>(const MarchArgs<float>&, int32_t, hipStream_t);
template hipError_t launch_march<double>(const MarchArgs<double>&, int32_t, hipStream_t);

}  // namespace hsg
