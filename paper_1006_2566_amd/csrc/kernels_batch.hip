// Batched form: many independent lattices ("chains") of mixed size advanced by one
// launch, plus replica exchange (parallel tempering) and pairwise overlaps over the
// chains of a batch.
//
// One workgroup owns one chain for the whole launch: it runs that chain's colour
// passes with a workgroup barrier between them, so a whole sweep -- and several
// sweeps -- happen inside the launch with no grid-wide synchronisation.  Workgroups
// are dispatched in the caller's order (largest lattices first), which balances
// lattices of uneven L; the launch has no state of its own, so it can be captured in
// a HIP graph and replayed.  The site update is the same function as in the
// single-lattice colour pass.
#include <algorithm>

#include "hsg.h"
#include "hsg_device.h"
#include "hsg_internal.h"
#include "hsg_site.h"

namespace hsg {

namespace {

// Quotient by a small divisor d: with m = ceil(2^32 / d) = (2^32 + e) / d, 0 <= e < d,
// n m / 2^32 = n/d + n e / (d 2^32), whose floor is floor(n/d) as long as n e < 2^32 --
// true for n < 2^24 and d <= 256.  Chains have L <= 256, so the divisors L/2 and L
// qualify and the colour index stays below 128 * 256 * 256 = 2^23.  d = 1 passes.
struct SmallDiv {
  uint32_t d, m;
  __device__ __forceinline__ explicit SmallDiv(uint32_t d_) : d(d_), m(d_ > 1 ? 0xFFFFFFFFu / d_ + 1u : 0u) {}
  __device__ __forceinline__ uint32_t div(uint32_t n) const { return d > 1 ? __umulhi(n, m) : n; }
};

// Workgroup size of the per-chain reductions (energy, overlaps): one workgroup
// reduces a whole chain, so large chains want the largest workgroup.
constexpr int kChainReduceThreads = 1024;

template <typename R>
struct ChainView {
  Planes<R> S, J;
  int32_t L, Lh;
  int64_t Nh;
};

template <typename R>
__device__ __forceinline__ ChainView<R> chain_view(const hsg_chain& ch, R* spins_base,
                                                   R* J_base) {
  ChainView<R> v;
  v.L = ch.L;
  v.Lh = ch.L / 2;
  v.Nh = (int64_t)v.Lh * v.L * v.L;
  v.S = planes_of<R>(spins_base + ch.spin_offset, v.Nh);
  v.J = planes_of<R>(J_base + ch.J_offset, v.Nh);
  return v;
}

template <typename R>
struct BatchArgs {
  const hsg_chain* chains;
  R* spins;
  R* J;
  const double* beta;
  double* E;
  uint32_t* sweep;
  int32_t* remaining;
  const int32_t* order;
  int32_t n_chains;
  int32_t n_sweeps;
};

// The site update of a chain's site: the binary32 form (scalar plane bases, 32-bit
// offsets) or the generic one.
template <typename R, PassMode MODE>
__device__ __forceinline__ double site_update(const ChainView<R>& v, const SitePos& q,
                                              const HitCtx<R>& hc) {
  if constexpr (sizeof(R) == 4)
    return update_site_b32<MODE, false>(v.S, v.J, q, hc);
  else
    return update_site<R, MODE>(v.S, v.J, q, hc);
}

// One colour pass of mode MODE over a chain, spread over the workgroup.  The colour
// is a compile-time constant, so the site update addresses its planes with constant
// indices (no pointer table in scratch memory, global rather than flat loads).
template <typename R, PassMode MODE, int COLOUR>
__device__ __forceinline__ double chain_pass(const ChainView<R>& v, const HitCtx<R>& hc,
                                             const SmallDiv& by_lh, const SmallDiv& by_l) {
  double dE = 0.0;
  SitePos q;
  q.L = v.L;
  q.Lh = v.Lh;
  q.c = COLOUR;
  for (uint32_t ic = threadIdx.x; ic < (uint32_t)v.Nh; ic += blockDim.x) {
    const uint32_t r = by_lh.div(ic);
    q.xh = (int32_t)(ic - r * (uint32_t)v.Lh);
    const uint32_t zq = by_l.div(r);
    q.y = (int32_t)(r - zq * (uint32_t)v.L);
    q.z = (int32_t)zq;
    if constexpr (sizeof(R) == 4)
      dE += update_site_b32<MODE, false>(v.S, v.J, q, hc);
    else
      dE += update_site<R, MODE>(v.S, v.J, q, hc);
  }
  return dE;
}

// Value every lane of the wave holds the same copy of, made visibly uniform (scalar)
// for the compiler: loop bounds and exits that contain workgroup barriers must be.
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)v);
}
__device__ __forceinline__ uint64_t uniform(uint64_t v) {
  return (uint64_t)uniform((uint32_t)v) | ((uint64_t)uniform((uint32_t)(v >> 32)) << 32);
}
__device__ __forceinline__ int64_t uniform(int64_t v) { return (int64_t)uniform((uint64_t)v); }

// The chain table entry, with every field made uniform (see uniform()).
__device__ __forceinline__ hsg_chain load_chain(const hsg_chain* chains, int32_t ci) {
  const hsg_chain c = chains[ci];
  hsg_chain u;
  u.spin_offset = uniform(c.spin_offset);
  u.J_offset = uniform(c.J_offset);
  u.seed = uniform(c.seed);
  u.J_seed = uniform(c.J_seed);
  u.L = uniform(c.L);
  u.k_hits = uniform(c.k_hits);
  u.n_or = uniform(c.n_or);
  u.renorm_every = uniform(c.renorm_every);
  u.flags = uniform(c.flags);
  u.reserved = 0;
  return u;
}

// One workgroup per chain: workgroup b advances chain order[b].  The hardware
// dispatcher hands workgroups to compute units as they free up, in order, so the
// caller's order (largest lattices first) balances chains of uneven size without a
// software queue, and every loop that contains a barrier has uniform bounds.
template <typename R>
__global__ __launch_bounds__(1024) void batch_sweep_kernel(BatchArgs<R> a) {
  __shared__ double s_red[16];
  const int32_t ci = uniform(a.order[blockIdx.x]);
  const hsg_chain ch = load_chain(a.chains, ci);
  const ChainView<R> v = chain_view<R>(ch, a.spins, a.J);
  const SmallDiv by_lh((uint32_t)v.Lh), by_l((uint32_t)v.L);
  int32_t n = a.n_sweeps;
  if (a.remaining) n = uniform(min(n, a.remaining[ci]));
  HitCtx<R> hc;
  hc.beta = (R)a.beta[ci];
  hc.k_hits = ch.k_hits;
  hc.seed_lo = (uint32_t)ch.seed;
  hc.seed_hi = (uint32_t)(ch.seed >> 32);
  const uint32_t sweep0 = uniform(a.sweep[ci]);
  const bool heat = (ch.flags & HSG_HEAT_BATH) != 0;
  double dE = 0.0;
  for (int32_t s = 0; s < n; ++s) {
    hc.sweep = sweep0 + (uint32_t)s;
    for (int32_t phase = 0; phase <= ch.n_or; ++phase) {
      if (phase == 0 && ch.k_hits == 0) continue;
      hc.phase = (uint32_t)phase;
      if (phase > 0) {
        chain_pass<R, PassMode::OverRelax, 0>(v, hc, by_lh, by_l);
        __syncthreads();
        chain_pass<R, PassMode::OverRelax, 1>(v, hc, by_lh, by_l);
      } else if (heat) {
        dE += chain_pass<R, PassMode::HeatBath, 0>(v, hc, by_lh, by_l);
        __syncthreads();
        dE += chain_pass<R, PassMode::HeatBath, 1>(v, hc, by_lh, by_l);
      } else if (ch.k_hits % 4 == 0) {  // every group of four hits complete
        dE += chain_pass<R, PassMode::MetropolisFull, 0>(v, hc, by_lh, by_l);
        __syncthreads();
        dE += chain_pass<R, PassMode::MetropolisFull, 1>(v, hc, by_lh, by_l);
      } else {
        dE += chain_pass<R, PassMode::Metropolis, 0>(v, hc, by_lh, by_l);
        __syncthreads();
        dE += chain_pass<R, PassMode::Metropolis, 1>(v, hc, by_lh, by_l);
      }
      __syncthreads();
    }
    if (ch.renorm_every > 0 && (hc.sweep + 1u) % (uint32_t)ch.renorm_every == 0u) {
      for (uint32_t e = threadIdx.x; e < 2u * (uint32_t)v.Nh; e += blockDim.x) {
        const int c = e >= (uint32_t)v.Nh ? 1 : 0;
        renormalise_spin(v.S, c, (int64_t)e - c * v.Nh);
      }
      __syncthreads();
    }
  }
  const double total = block_sum(dE, s_red);
  if (threadIdx.x == 0) {
    a.E[ci] += total;
    a.sweep[ci] = sweep0 + (uint32_t)n;
    if (a.remaining) a.remaining[ci] -= n;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void batch_init_kernel(const hsg_chain* chains, R* spins,
                                                         R* J) {
  const hsg_chain ch = chains[blockIdx.y];
  const int64_t N = (int64_t)ch.L * ch.L * ch.L;
  R* js = (ch.flags & HSG_CHAIN_INIT_J) ? J + ch.J_offset : nullptr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * blockDim.x)
    init_site<R>(ch.L, e, (uint32_t)ch.seed, (uint32_t)(ch.seed >> 32), spins + ch.spin_offset, js,
                 (uint32_t)ch.J_seed, (uint32_t)(ch.J_seed >> 32));
}

template <typename R>
__global__ __launch_bounds__(kChainReduceThreads) void batch_energy_kernel(
    const hsg_chain* chains, const R* spins, const R* J, double* out) {
  __shared__ double s_red[16];
  const hsg_chain ch = chains[blockIdx.x];
  const int32_t L = ch.L, Lh = L / 2;
  const int64_t Nh = (int64_t)Lh * L * L;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < Nh; e += blockDim.x) {
    const SiteOf st = site_of(e, L);
    acc += colour0_bond_sum(spins + ch.spin_offset, J + ch.J_offset, Nh, L, Lh, st.xh, st.y, st.z);
  }
  const double total = block_sum(acc, s_red);
  if (threadIdx.x == 0) out[blockIdx.x] = -total;
}

// Overlap of two chains of equal L, reduced by one workgroup.
template <typename R>
__device__ __forceinline__ void pair_overlap(const hsg_chain& ca, const hsg_chain& cb,
                                             const R* spins, double* out) {
  __shared__ double s_red[16];
  const int64_t N = (int64_t)ca.L * ca.L * ca.L, Nh = N / 2;
  const R* a = spins + ca.spin_offset;
  const R* b = spins + cb.spin_offset;
  double v[15] = {0.0};
  for (int64_t e = threadIdx.x; e < N; e += blockDim.x) {
    const int64_t c = e >= Nh ? 1 : 0;
    const int64_t base = 3 * c * Nh + (e - c * Nh);
    double av[3], bv[3];
    for (int k = 0; k < 3; ++k) {
      av[k] = (double)a[base + k * Nh];
      bv[k] = (double)b[base + k * Nh];
    }
    for (int m = 0; m < 3; ++m) {
      for (int n = 0; n < 3; ++n) v[3 * m + n] = fma(av[m], bv[n], v[3 * m + n]);
      v[9 + m] += av[m];
      v[12 + m] += bv[m];
    }
  }
  for (int k = 0; k < 15; ++k) {
    const double t = block_sum(v[k], s_red);
    if (threadIdx.x == 0) out[k] = t / (double)N;
  }
}

template <typename R>
__global__ __launch_bounds__(kChainReduceThreads) void chain_pairs_overlap_kernel(
    const hsg_chain* chains, const R* spins, const int32_t* pairs, double* out) {
  const int32_t p = blockIdx.x;
  pair_overlap<R>(chains[pairs[2 * p]], chains[pairs[2 * p + 1]], spins, out + 15 * (int64_t)p);
}

template <typename R>
__global__ __launch_bounds__(kChainReduceThreads) void ladder_pairs_overlap_kernel(
    const hsg_chain* chains, const R* spins, const int32_t* chain_at_slot, int32_t n_temps,
    const int32_t* ladder_pairs, double* out) {
  const int32_t p = blockIdx.x, t = blockIdx.y;
  const int32_t la = ladder_pairs[2 * p], lb = ladder_pairs[2 * p + 1];
  const int32_t a = chain_at_slot[(int64_t)la * n_temps + t];
  const int32_t b = chain_at_slot[(int64_t)lb * n_temps + t];
  pair_overlap<R>(chains[a], chains[b], spins, out + 15 * ((int64_t)p * n_temps + t));
}

// One exchange round per ladder (one thread per ladder; the ladders are short).
__global__ void pt_exchange_kernel(int32_t n_ladders, int32_t n_temps, int32_t* chain_at_slot,
                                   const double* beta_of_slot, int32_t* accepted,
                                   uint32_t seed_lo, uint32_t seed_hi, uint32_t* round_ctr,
                                   const double* E, double* beta) {
  const int32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t round = *round_ctr;  // advanced by bump_round_kernel afterwards
  if (l >= n_ladders) return;
  int32_t* slots = chain_at_slot + (int64_t)l * n_temps;
  for (int32_t t = (int32_t)(round & 1u); t + 1 < n_temps; t += 2) {
    const int32_t ca = slots[t], cb = slots[t + 1];
    const double delta = (beta_of_slot[t] - beta_of_slot[t + 1]) * (E[ca] - E[cb]);
    const Word4 w = philox10((uint32_t)t, round, (uint32_t)l, kTagSwap, seed_lo, seed_hi);
    const double u = unit_uniform<double>(w.w0);
    if (delta >= 0.0 || u < exp(delta)) {
      slots[t] = cb;
      slots[t + 1] = ca;
      if (accepted) accepted[(int64_t)l * n_temps + t] += 1;
    }
  }
  for (int32_t t = 0; t < n_temps; ++t) beta[slots[t]] = beta_of_slot[t];
}

__global__ void bump_round_kernel(uint32_t* round_ctr) { *round_ctr += 1u; }

// ------------------------------------------------------------------------------------
// Multi-lattice colour pass: one launch updates colour c of every listed chain.  Tile
// t covers blockDim.x consecutive colour sites of one chain; chains that have used up
// their budget, or do not have this phase, return at once.

template <typename R>
struct MultiPassArgs {
  const hsg_chain* chains;
  R* spins;
  R* J;
  const double* beta;
  double* E;
  const uint32_t* sweep;
  const int32_t* remaining;
  const int32_t* tiles;
  int32_t n_tiles;
  int32_t s;  // sweep offset within the call
  int32_t phase;
  int32_t colour;
  int32_t reverse;
};

template <typename R, int COLOUR>
__global__ __launch_bounds__(1024) void multi_pass_kernel(MultiPassArgs<R> a) {
  __shared__ double s_red[16];
  int32_t t = xcd_tile((int32_t)blockIdx.x, a.n_tiles);
  if (a.reverse) t = a.n_tiles - 1 - t;
  const int32_t ci = uniform(a.tiles[2 * t]), ic0 = uniform(a.tiles[2 * t + 1]);
  if (a.s >= uniform(a.remaining[ci])) return;
  const hsg_chain ch = load_chain(a.chains, ci);
  if ((a.phase == 0 && ch.k_hits == 0) || a.phase > ch.n_or) return;
  const ChainView<R> v = chain_view<R>(ch, a.spins, a.J);
  const uint32_t ic = (uint32_t)ic0 + threadIdx.x;
  HitCtx<R> hc;
  hc.beta = (R)a.beta[ci];
  hc.k_hits = ch.k_hits;
  hc.seed_lo = (uint32_t)ch.seed;
  hc.seed_hi = (uint32_t)(ch.seed >> 32);
  hc.sweep = a.sweep[ci] + (uint32_t)a.s;
  hc.phase = (uint32_t)a.phase;
  double dE = 0.0;
  if (ic < (uint32_t)v.Nh) {
    const SmallDiv by_lh((uint32_t)v.Lh), by_l((uint32_t)v.L);
    SitePos q;
    q.L = v.L;
    q.Lh = v.Lh;
    q.c = COLOUR;
    const uint32_t r = by_lh.div(ic);
    q.xh = (int32_t)(ic - r * (uint32_t)v.Lh);
    const uint32_t zq = by_l.div(r);
    q.y = (int32_t)(r - zq * (uint32_t)v.L);
    q.z = (int32_t)zq;
    if (a.phase > 0)
      site_update<R, PassMode::OverRelax>(v, q, hc);
    else if (ch.flags & HSG_HEAT_BATH)
      dE = site_update<R, PassMode::HeatBath>(v, q, hc);
    else if (ch.k_hits % 4 == 0)  // every group of four hits complete
      dE = site_update<R, PassMode::MetropolisFull>(v, q, hc);
    else
      dE = site_update<R, PassMode::Metropolis>(v, q, hc);
  }
  if (a.phase == 0) {
    const double total = block_sum(dE, s_red);
    if (threadIdx.x == 0 && total != 0.0) atomicAdd(&a.E[ci], total);
  }
}

// Renormalisation after sweep offset s for the chains whose schedule asks for it.
template <typename R>
__global__ __launch_bounds__(1024) void multi_renorm_kernel(const hsg_chain* chains, R* spins,
                                                            const uint32_t* sweep,
                                                            const int32_t* remaining,
                                                            const int32_t* tiles, int32_t s) {
  const int32_t t = blockIdx.x;
  const int32_t ci = tiles[2 * t], ic0 = tiles[2 * t + 1];
  if (s >= remaining[ci]) return;
  const hsg_chain ch = chains[ci];
  if (ch.renorm_every <= 0 || (sweep[ci] + (uint32_t)s + 1u) % (uint32_t)ch.renorm_every != 0u)
    return;
  const int64_t Nh = (int64_t)(ch.L / 2) * ch.L * ch.L;
  const Planes<R> S = planes_of<R>(spins + ch.spin_offset, Nh);
  const int64_t e = (int64_t)ic0 + threadIdx.x;
  if (e < Nh) {
    renormalise_spin(S, 0, e);
    renormalise_spin(S, 1, e);
  }
}

// Advances every chain's sweep counter and budget by the sweeps it ran.
__global__ void multi_finish_kernel(int32_t n_chains, uint32_t* sweep, int32_t* remaining,
                                    int32_t n_sweeps) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_chains) return;
  const int32_t n = min(n_sweeps, remaining[c]);
  if (n > 0) {
    sweep[c] += (uint32_t)n;
    remaining[c] -= n;
  }
}

}  // namespace

template <typename R>
hipError_t launch_batch_init(const hsg_batch* b, hipStream_t st) {
  hipLaunchKernelGGL(batch_init_kernel<R>, dim3(64, (unsigned)b->n_chains), dim3(256), 0, st,
                     b->chains, (R*)b->spins, (R*)b->J);
  hipLaunchKernelGGL(batch_energy_kernel<R>, dim3((unsigned)b->n_chains),
                     dim3(kChainReduceThreads), 0, st,
                     b->chains, (const R*)b->spins, (const R*)b->J, b->E);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_sweep(const hsg_batch* b, int32_t n_sweeps, hipStream_t st) {
  BatchArgs<R> a;
  a.chains = b->chains;
  a.spins = (R*)b->spins;
  a.J = (R*)b->J;
  a.beta = b->beta;
  a.E = b->E;
  a.sweep = b->sweep;
  a.remaining = b->remaining;
  a.order = b->order;
  a.n_chains = b->n_chains;
  a.n_sweeps = n_sweeps;
  const int threads = b->threads > 0 ? b->threads : 256;
  hipLaunchKernelGGL(batch_sweep_kernel<R>, dim3((unsigned)b->n_chains), dim3((unsigned)threads), 0, st,
                     a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_energy(const hsg_batch* b, double* out, hipStream_t st) {
  hipLaunchKernelGGL(batch_energy_kernel<R>, dim3((unsigned)b->n_chains),
                     dim3(kChainReduceThreads), 0, st,
                     b->chains, (const R*)b->spins, (const R*)b->J, out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_overlap(const hsg_batch* b, const int32_t* pairs, int32_t n_pairs,
                                double* out, hipStream_t st) {
  hipLaunchKernelGGL(chain_pairs_overlap_kernel<R>, dim3((unsigned)n_pairs),
                     dim3(kChainReduceThreads), 0, st,
                     b->chains, (const R*)b->spins, pairs, out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_pt_overlap(const hsg_pt* pt, const hsg_batch* b, const int32_t* ladder_pairs,
                             int32_t n_pairs, double* out, hipStream_t st) {
  hipLaunchKernelGGL(ladder_pairs_overlap_kernel<R>, dim3((unsigned)n_pairs, (unsigned)pt->n_temps),
                     dim3(kChainReduceThreads), 0, st, b->chains, (const R*)b->spins,
                     pt->chain_at_slot,
                     pt->n_temps, ladder_pairs, out);
  return hipGetLastError();
}

hipError_t launch_pt_exchange(const hsg_pt* pt, const hsg_batch* b, hipStream_t st) {
  const unsigned blocks = (unsigned)((pt->n_ladders + 63) / 64);
  hipLaunchKernelGGL(pt_exchange_kernel, dim3(blocks), dim3(64), 0, st, pt->n_ladders, pt->n_temps,
                     pt->chain_at_slot, pt->beta_of_slot, pt->accepted, (uint32_t)pt->seed,
                     (uint32_t)(pt->seed >> 32), pt->round, (const double*)b->E, b->beta);
  hipLaunchKernelGGL(bump_round_kernel, dim3(1), dim3(1), 0, st, pt->round);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_pass_sweep(const hsg_batch* b, const int32_t* tiles, int32_t n_tiles,
                                   int32_t tile_sites, int32_t max_n_or, int32_t renorm,
                                   int32_t n_sweeps, hipStream_t st) {
  MultiPassArgs<R> a;
  a.chains = b->chains;
  a.spins = (R*)b->spins;
  a.J = (R*)b->J;
  a.beta = b->beta;
  a.E = b->E;
  a.sweep = b->sweep;
  a.remaining = b->remaining;
  a.tiles = tiles;
  a.n_tiles = n_tiles;
  int32_t pass = 0;
  for (int32_t s = 0; s < n_sweeps; ++s) {
    a.s = s;
    for (int32_t phase = 0; phase <= max_n_or; ++phase) {
      a.phase = phase;
      for (int32_t colour = 0; colour < 2; ++colour) {
        a.colour = colour;
        a.reverse = pass++ & 1;
        if (colour == 0)
          hipLaunchKernelGGL((multi_pass_kernel<R, 0>), dim3((unsigned)n_tiles),
                             dim3((unsigned)tile_sites), 0, st, a);
        else
          hipLaunchKernelGGL((multi_pass_kernel<R, 1>), dim3((unsigned)n_tiles),
                             dim3((unsigned)tile_sites), 0, st, a);
      }
    }
    if (renorm)
      hipLaunchKernelGGL(multi_renorm_kernel<R>, dim3((unsigned)n_tiles), dim3((unsigned)tile_sites),
                         0, st, b->chains, (R*)b->spins, (const uint32_t*)b->sweep,
                         (const int32_t*)b->remaining, tiles, s);
  }
  hipLaunchKernelGGL(multi_finish_kernel, dim3((unsigned)((b->n_chains + 255) / 256)), dim3(256), 0,
                     st, b->n_chains, b->sweep, b->remaining, n_sweeps);
  return hipGetLastError();
}

#define HSG_BATCH_INSTANTIATE(R)                                                              \
  template hipError_t launch_batch_init<R>(const hsg_batch*, hipStream_t);                    \
  template hipError_t launch_batch_sweep<R>(const hsg_batch*, int32_t, hipStream_t); \
  template hipError_t launch_batch_energy<R>(const hsg_batch*, double*, hipStream_t);         \
  template hipError_t launch_batch_overlap<R>(const hsg_batch*, const int32_t*, int32_t,      \
                                              double*, hipStream_t);                          \
  template hipError_t launch_pt_overlap<R>(const hsg_pt*, const hsg_batch*, const int32_t*,   \
                                           int32_t, double*, hipStream_t);                     \
  template hipError_t launch_batch_pass_sweep<R>(const hsg_batch*, const int32_t*, int32_t,   \
                                                 int32_t, int32_t, int32_t, int32_t, hipStream_t);
HSG_BATCH_INSTANTIATE(float)
HSG_BATCH_INSTANTIATE(double)

}  // namespace hsg
