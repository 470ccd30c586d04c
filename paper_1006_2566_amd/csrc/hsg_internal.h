// Host-side internals of libhsg: launch geometry, kernel argument blocks and the
// launchers each kernel file exports to the C interface in api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hsg {

// A colour pass covers the N/2 sites of one colour, stored as L planes (z) of L rows
// (y) of L/2 sites (xh).  Each workgroup takes a BX x BY x BZ tile of (xh, y, z);
// BX is one wavefront wide when L/2 allows it, so a wave reads whole row segments.
struct Geometry {
  int32_t L, Lh;
  int32_t bx_log, by_log, bz_log;     // tile extents are 1 << *_log
  int32_t tiles_x, tiles_y, tiles_z;  // tiles along xh, y, z
  int32_t n_blocks;                   // tiles_x * tiles_y * tiles_z
  int32_t threads;                    // BX * BY * BZ (<= 256)
};

Geometry pass_geometry(int32_t L);

// Blocks of the fixed-size grid used by the energy and overlap reductions.
constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;
constexpr int kReduceSlots = 16;  // doubles per block partial (overlap needs 15)
// Blocks and doubles per block partial of the Fourier-overlap reduction.
constexpr int kFourierBlocks = 512;
constexpr int kFourierSlots = 64;
constexpr int kReduceRegion = kReduceBlocks * kFourierSlots;  // doubles, for either reduction
static_assert(kFourierBlocks <= kReduceBlocks && kReduceSlots <= kFourierSlots,
              "reduce region too small");

// Scratch layout of hsg_lattice.work (bytes):
//   [0, 256)                              reserved
//   [256, 256 + 8*n_blocks)               per-tile energy-change partials of the passes
//   [.., + 8*kReduceRegion)               per-block partials of energy / overlaps
//   [fused_offset(L), + 3*N*sizeof(R))    second spin array of fused and phase launches
//                                         (only for L that march_supported or
//                                         phase_supported accepts)
size_t work_bytes_for(int32_t L);  // without the second spin array
size_t fused_offset(int32_t L);    // 256-byte aligned end of the above
size_t work_bytes_for(int32_t L, int32_t dtype_bytes);  // with it where it applies
inline double* pass_partials(void* work) { return (double*)((char*)work + 256); }
inline double* reduce_partials(void* work, int32_t L) {
  return pass_partials(work) + pass_geometry(L).n_blocks;
}

// Pointers of the six planes (3 components x 2 colours) of a colour-split array.
template <typename R>
struct Planes {
  R* p[6];
};

template <typename R>
__host__ __device__ inline Planes<R> planes_of(void* base, int64_t half_sites) {
  Planes<R> out;
  for (int k = 0; k < 6; ++k) out.p[k] = (R*)base + (int64_t)k * half_sites;
  return out;
}

// MetropolisFull is Metropolis when k_hits is a multiple of four, so that every group of
// four hits is complete (the launchers choose it; the arithmetic is Metropolis's).
enum class PassMode : int { Metropolis = 0, OverRelax = 1, HeatBath = 2, MetropolisFull = 3 };
__host__ __device__ inline PassMode metropolis_mode(int32_t k_hits) {
  return k_hits % 4 == 0 ? PassMode::MetropolisFull : PassMode::Metropolis;
}

template <typename R>
struct PassArgs {
  Planes<R> spins;   // colour-split spins
  Planes<R> J;       // colour-split couplings
  double* partials;  // one double per tile (Metropolis / heat bath only)
  R beta;
  uint32_t seed_lo, seed_hi;
  uint32_t sweep;
  uint32_t phase;
  int32_t k_hits;
  int32_t colour;
  int32_t reverse;     // walk the tiles from the last z plane to the first
  int32_t tile_base;   // the launch covers tiles [tile_base, tile_base + tile_count)
  int32_t tile_count;  // (the whole pass, or one z slab of tiles)
  int32_t nt;          // read-only data through non-temporal loads
  Geometry g;
};

template <typename R>
hipError_t launch_colour_pass(PassMode mode, const PassArgs<R>& a, hipStream_t stream);

// A colour pass inside a fused launch.
struct MarchStage {
  int32_t mode;           // PassMode
  int32_t colour;         // colour updated
  uint32_t sweep, phase;  // Philox counter words
  int32_t renorm_before;  // divide each updated spin by its length before the update
  int32_t renorm_after;   // ... and after it
};
constexpr int kMarchMaxStages = 4;
constexpr int kMarchMinL = 256;   // smaller lattices give too few workgroups
constexpr int kMarchMaxL = 1024;  // element offsets stay below 2^32
constexpr int kMarchZ = 64;      // planes per workgroup

template <typename R>
struct MarchArgs {
  const R* in;       // colour-split spins before the launch's first pass
  R* out;            // colour-split spins after its last pass (distinct from in)
  const R* J;        // colour-split couplings
  double* partials;  // one per workgroup, energy changes of its own sites are added
  R beta;
  uint32_t seed_lo, seed_hi;
  int32_t k_hits;
  int32_t L;
  int32_t tiles_x, tiles_y, zc;  // set by launch_march
  MarchStage st[kMarchMaxStages];
};

// An over-relaxation phase (colour-0 pass then colour-1 pass) in one launch, optionally
// followed by the next sweep's colour-0 Monte Carlo pass (kernels_phase.hip).  Tile
// shape timed on MI355X at L = 256 against 128-1024 threads, 4-32 rows and 16-64 planes.
constexpr int kPhaseThreads = 512;
constexpr int kPTY = 16;  // tile rows
constexpr int kPZ = 32;   // planes per workgroup
constexpr int kPhaseMinL = 64;
// Element offsets of the phase launch reach 3 N (six planes of N/2 from one base) and are
// 32-bit: L = 1024 keeps them below 2^32.
constexpr int kPhaseMaxL = 1024;

template <typename R>
struct PhaseArgs {
  const R* in;  // colour-split spins before the phase
  R* out;       // after it (distinct from in)
  const R* J;   // colour-split couplings
  R beta;       // inverse temperature of the Monte Carlo pass
  uint32_t seed_lo, seed_hi;
  uint32_t sweep, phase;  // Philox counter words of the phase (over-relaxation draws none)
  int32_t k_hits;
  int32_t L;
  // With then_mc: after the phase, the colour-0 pass of the Monte Carlo phase of sweep
  // mc_sweep (mode mc_mode, a PassMode other than OverRelax).  With renorm, every spin
  // is divided by its length between the two (colour 1 right after its over-relaxation
  // step, colour 0 right before its Monte Carlo update).  The energy changes of a
  // workgroup's sites are added to partials[blockIdx.x].
  int32_t then_mc;
  int32_t mc_mode;
  uint32_t mc_sweep;
  int32_t renorm;
  double* partials;
};

bool phase_supported(int32_t L);
int32_t phase_blocks(int32_t L);
template <typename R>
hipError_t launch_phase(const PhaseArgs<R>& a, hipStream_t stream);

bool march_supported(int32_t L);
int32_t march_blocks(int32_t L);
template <typename R>
int32_t march_max_stages();
// n_stages consecutive passes (2, or 4 in binary32) described by a.st.
template <typename R>
hipError_t launch_march(const MarchArgs<R>& a, int32_t n_stages, hipStream_t stream);

// *E += sum of the n partials (fixed order); the partials are then zeroed.
hipError_t launch_fold_partials(double* partials, int32_t n, double* E, hipStream_t stream);

template <typename R>
hipError_t launch_init(int32_t L, uint64_t seed, void* spins, void* J, hipStream_t stream);
template <typename R>
hipError_t launch_import(int32_t L, const R* canon_spins, const R* canon_J, void* spins,
                         void* J, hipStream_t stream);
template <typename R>
hipError_t launch_export(int32_t L, const void* spins, const void* J, R* canon_spins,
                         R* canon_J, hipStream_t stream);
template <typename R>
hipError_t launch_renormalise(int32_t L, void* spins, int32_t colours, hipStream_t stream);
// out[0] = H (recomputed, binary64).
template <typename R>
hipError_t launch_energy(int32_t L, const void* spins, const void* J, double* partials,
                         double* out, hipStream_t stream);
template <typename R>
hipError_t launch_overlap(int32_t L, const void* a, const void* b, double* partials,
                          double* out, hipStream_t stream);
hipError_t launch_zero(double* p, int64_t n, hipStream_t stream);
template <typename R>
hipError_t launch_overlap_fourier(int32_t L, const void* a, const void* b, double* partials,
                                  double* out, hipStream_t stream);

}  // namespace hsg

struct hsg_batch;
struct hsg_pt;

namespace hsg {

template <typename R>
hipError_t launch_batch_init(const hsg_batch* b, hipStream_t st);
template <typename R>
hipError_t launch_batch_sweep(const hsg_batch* b, int32_t n_sweeps, hipStream_t st);
template <typename R>
hipError_t launch_batch_energy(const hsg_batch* b, double* out, hipStream_t st);
template <typename R>
hipError_t launch_batch_overlap(const hsg_batch* b, const int32_t* pairs, int32_t n_pairs,
                                double* out, hipStream_t st);
template <typename R>
hipError_t launch_pt_overlap(const hsg_pt* pt, const hsg_batch* b, const int32_t* ladder_pairs,
                             int32_t n_pairs, double* out, hipStream_t st);
hipError_t launch_pt_exchange(const hsg_pt* pt, const hsg_batch* b, hipStream_t st);
template <typename R>
hipError_t launch_batch_overlap_fourier(const hsg_batch* b, const int32_t* pairs, int32_t n_pairs,
                                        double* out, hipStream_t st);
template <typename R>
hipError_t launch_pt_overlap_fourier(const hsg_pt* pt, const hsg_batch* b,
                                     const int32_t* ladder_pairs, int32_t n_pairs, double* out,
                                     hipStream_t st);
template <typename R>
hipError_t launch_batch_pass_sweep(const hsg_batch* b, const int32_t* tiles, int32_t n_tiles,
                                   int32_t tile_sites, int32_t max_n_or, int32_t renorm,
                                   int32_t n_sweeps, hipStream_t st);
hipError_t launch_copy_double(const double* src, double* dst, hipStream_t stream);

}  // namespace hsg
