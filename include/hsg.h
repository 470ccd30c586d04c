/*
 * hsg.h -- C interface of libhsg, the MI355X (gfx950) library for the checkerboard
 * Monte Carlo sweep of the 3D Heisenberg spin glass of Bernaschi, Parisi & Parisi,
 * "The Heisenberg spin glass model on GPU: myths and actual facts" (arXiv:1006.2566).
 *
 * Model (§2): spins sigma_i are 3-component unit vectors on an L x L x L lattice,
 * periodic in x, y and z, site i = x + L*y + L*L*z; the couplings J_ij on the 3*L^3
 * nearest-neighbour bonds are Gaussian with mean 0 and variance 1; the energy is
 * H = -sum over bonds J_ij sigma_i . sigma_j (eq. 1, each bond once), and a site
 * interacts with its six neighbours through the local field of eq. (2),
 * h_i = sum_j J_ij sigma_j.  Dynamics (§4 and the methods §2 names): sites of one
 * colour c = (x+y+z) & 1 share no bond and are updated together (the checkerboard);
 * a sweep is a Monte Carlo phase (Metropolis with k hits per site, or heat bath),
 * then n_or over-relaxation phases (reflection of sigma about h, §4), each phase
 * being the colour-0 pass followed by the colour-1 pass.  Random numbers, which the
 * paper leaves aside, come from Philox4x32-10 keyed by the lattice seed with counter
 * (sweep, site, (phase << 16) | block, stream tag): a site's uniforms in a phase are the
 * words of its blocks 0, 1, ... in order, three per Metropolis hit (four hits per three
 * blocks) and two per heat-bath draw.
 *
 * Conventions for every function:
 *  - Return HSG_OK (0) or a negative HSG_E* code; never abort, never throw.  After an
 *    error, hsg_last_error() returns a message (per calling thread).
 *  - Buffers marked "device" are device memory the CALLER allocates and owns (the
 *    Python binding uses torch tensors); the library allocates nothing persistent.
 *  - Work is enqueued on the given HIP stream (hipStream_t passed as void*, NULL =
 *    the default stream) and returns before it completes; results written to device
 *    memory are valid once the stream has reached that point.
 *  - Calls that share buffers must be ordered by the caller (one stream, or events).
 *
 * Internal layout ("colour-split", both spins and J): 6 planes of N/2 elements,
 * plane (3*c + a) holds component (or bond direction) a of the colour-c sites, the
 * site (x, y, z) of colour c sitting at index xh + (L/2)*(y + L*z) with
 * x = 2*xh + ((y + z + c) & 1).  Use hsg_import / hsg_export to convert from / to
 * the canonical layout (3 planes of N elements, element [a*N + i]).
 */
#ifndef HSG_H
#define HSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HSG_OK 0
#define HSG_EINVAL (-1)      /* an argument is out of range or a required pointer is NULL */
#define HSG_EDEVICE (-3)     /* a HIP call or kernel launch failed */
#define HSG_EUNSUPPORTED (-4) /* valid request that the library does not implement */

#define HSG_F32 0 /* binary32 spins and couplings */
#define HSG_F64 1 /* binary64 spins and couplings */

#define HSG_L_MAX 1290 /* largest L: N = L^3 < 2^31 keeps every site index in 32 bits */

/* Sweep flags (hsg_sweep_params.flags).  HSG_SNAKE, HSG_FUSED and the variants below
 * change the order in which memory is touched, never a spin; with HSG_FUSED and
 * HSG_PHASE_MC the binary64 energy changes are summed in another (still fixed) order. */
#define HSG_HEAT_BATH 1 /* the Monte Carlo phase uses heat-bath draws instead of Metropolis */
#define HSG_SNAKE 2     /* successive colour passes walk the lattice in opposite z order */
#define HSG_FUSED 4     /* run up to four consecutive colour passes per launch (binary32;
                           two in binary64), each workgroup marching through z with its
                           block of the lattice in LDS: the lattice is read and written once
                           per launch instead of once per pass.  Needs L a multiple of 64
                           with HSG_FUSED_MIN_L <= L <= HSG_FUSED_MAX_L, else ignored;
                           overrides HSG_SNAKE.
                           Uses the second half of the work buffer as a second spin array */
#define HSG_FUSED_MIN_L 256
#define HSG_FUSED_MAX_L 1024
/* Variants of the memory schedule that reproduce the kernel designs the paper compares
 * (§4, Table 2: GM, TEXT, CA, SM, SM4P) on this GPU.  Each computes exactly what the
 * default schedule (the GM analogue: one launch per colour pass reading global memory)
 * computes, spin for spin; they exist to measure the paper's design question. */
#define HSG_MARCH_PHASE 16  /* with HSG_FUSED: one phase -- the colour-0 and colour-1
                               passes -- per launch of the LDS plane march (the SM
                               analogue: three planes on chip, both colours of a plane
                               before the next); HSG_FUSED alone, up to two phases per
                               march in binary32, is the SM4P analogue.  HSG_EINVAL
                               without HSG_FUSED */
#define HSG_PLANE_LAUNCH 32 /* one launch per z slab of tiles -- per z plane for L >= 64 --
                               instead of one per pass: 2L launches per phase, the CA
                               analogue's launch count.  Not with HSG_FUSED */
#define HSG_PHASE_LAUNCH 128 /* each over-relaxation phase -- its colour-0 and colour-1
                               passes -- runs as one launch that marches through z with a
                               window of planes in LDS, reading and writing the spins once
                               (L a multiple of 64, 64 <= L <= 1024; else ignored: the
                               launch indexes with 32-bit offsets up to 3 L^3).  Uses the second
                               spin array of the work buffer.  Not with HSG_FUSED */
#define HSG_PHASE_MC 256   /* as HSG_PHASE_LAUNCH, and when a sweep of the call is followed
                               by another (k_hits > 0), the launch of its last
                               over-relaxation phase also runs the next sweep's colour-0
                               Monte Carlo pass on each workgroup's own sites, after the
                               phase (renormalisation between them when due).  The Monte
                               Carlo arithmetic, which is never recomputed, hides the
                               phase's memory traffic.  Not with HSG_FUSED */
#define HSG_STREAM_LOADS 64 /* couplings and the other colour's spins, which a pass only
                               reads, are loaded with the non-temporal cache hint: the
                               nearest this GPU has to the texture path of the TEXT variant.
                               Not with HSG_FUSED */

typedef struct hsg_lattice {
  int32_t L;         /* even, 2 <= L <= HSG_L_MAX */
  int32_t dtype;     /* HSG_F32 or HSG_F64 */
  uint64_t seed;     /* Philox key of this lattice (init and Monte Carlo streams) */
  uint64_t sweep;    /* index of the next sweep (Philox counter word); hsg_sweep adds n */
  void *spins;       /* device, 3*L^3 elements of dtype, internal layout */
  void *J;           /* device, 3*L^3 elements of dtype, internal layout */
  double *E;         /* device, 1 double: the tracked energy H */
  void *work;        /* device scratch of at least work_bytes from hsg_lattice_bytes */
  size_t work_bytes; /* size of work in bytes */
} hsg_lattice;

typedef struct hsg_sweep_params {
  double T;             /* temperature, > 0; INFINITY means beta = 0 */
  int32_t k_hits;       /* Metropolis hits (or heat-bath draws) per site per sweep, >= 0 */
  int32_t n_or;         /* over-relaxation phases per sweep, >= 0; k_hits + n_or >= 1 */
  int32_t renorm_every; /* R > 0: after sweep s with (s+1) % R == 0 every spin is
                           divided by its length; 0 = never */
  int32_t flags;        /* OR of HSG_HEAT_BATH, HSG_SNAKE, HSG_FUSED, HSG_MARCH_PHASE,
                           HSG_PLANE_LAUNCH, HSG_STREAM_LOADS, HSG_PHASE_LAUNCH,
                           HSG_PHASE_MC */
} hsg_sweep_params;

/* Sizes of the three device buffers of an L^3 lattice of the given dtype.  Any
 * output pointer may be NULL.  HSG_EINVAL for odd L, L < 2, L > HSG_L_MAX or an
 * unknown dtype. */
int hsg_lattice_bytes(int32_t L, int32_t dtype, size_t *spin_bytes, size_t *J_bytes,
                      size_t *work_bytes);

/* Random initial state from lat->seed (§2 model): spins uniform on the sphere,
 * couplings N(0,1) by Box-Muller, both from Philox (stream tags 1 and 2, counter
 * (0, canonical site index, 0, tag)); then *lat->E = H and the scratch is cleared.
 * lat->sweep is left as it is. */
int hsg_init_lattice(hsg_lattice *lat, void *stream);

/* Load a state given in canonical layout: canon_spins and canon_J are device
 * arrays of 3*L^3 elements of lat->dtype ([a*N + i], J[d*N + i] = coupling of the
 * bond (i, i + e_d)).  canon_J may be NULL to keep the couplings.  Sets *lat->E = H
 * and clears the scratch.  Input and output must not overlap. */
int hsg_import(hsg_lattice *lat, const void *canon_spins, const void *canon_J, void *stream);

/* Write the state in canonical layout to device arrays of 3*L^3 elements;
 * either output may be NULL. */
int hsg_export(const hsg_lattice *lat, void *canon_spins, void *canon_J, void *stream);

/* n_sweeps >= 0 sweeps of the dynamics described at the top of this file, starting at
 * sweep index lat->sweep, which then advances by n_sweeps (the host-side field is
 * updated when the call returns; the work itself is only enqueued).  *lat->E is
 * advanced by the sum of accepted energy changes (binary64).  HSG_EINVAL also when
 * the sweep index would pass 2^32. */
int hsg_sweep(hsg_lattice *lat, const hsg_sweep_params *p, int32_t n_sweeps, void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation -- and so cannot provide a work buffer:
 * hsg_sweep with the same arguments and results, lat->work and lat->work_bytes ignored.
 * Its scratch (the per-tile energy partials) is a fixed array inside the library,
 * HSG_NOALLOC_SCRATCH_BYTES on every GPU the library runs on, held until the process
 * ends; the call allocates nothing and calls no allocating routine.  Limits: L <=
 * HSG_NOALLOC_L_MAX, and the pass-by-pass schedule only (HSG_SNAKE, HSG_PLANE_LAUNCH,
 * HSG_STREAM_LOADS, HSG_HEAT_BATH honoured; HSG_FUSED, HSG_MARCH_PHASE, HSG_PHASE_LAUNCH
 * and HSG_PHASE_MC, which need a second spin array, give HSG_EINVAL), as does any larger
 * L.  Every call on one GPU shares that GPU's array (cleared at the start of each call):
 * calls that overlap on one GPU -- on different streams, or from different threads --
 * race and must be ordered by the caller. */
#define HSG_NOALLOC_L_MAX 512
#define HSG_NOALLOC_SCRATCH_BYTES (2u << 20) /* 262144 partials: L = 512 */
int hsg_sweep_noalloc(hsg_lattice *lat, const hsg_sweep_params *p, int32_t n_sweeps,
                      void *stream);

/* Kinds of launch reported by hsg_sweep_timed. */
#define HSG_LAUNCH_OTHER 0        /* renormalisation, energy fold */
#define HSG_LAUNCH_MC_PASS 1      /* Metropolis or heat-bath colour pass */
#define HSG_LAUNCH_OR_PASS 2      /* over-relaxation colour pass */
#define HSG_LAUNCH_OR_PHASE 3     /* over-relaxation phase in one launch (HSG_PHASE_LAUNCH) */
#define HSG_LAUNCH_OR_PHASE_MC 4  /* the same carrying the next colour-0 Monte Carlo pass
                                     (HSG_PHASE_MC) */
#define HSG_LAUNCH_MARCH 5        /* fused passes (HSG_FUSED) */

/* Measurement form of hsg_sweep: the same sweeps (same arguments, same results), with a
 * pair of HIP events recorded on `stream` around each of the call's first `capacity`
 * kernel launches.  Synchronous: returns after the stream has passed the last
 * recorded launch, with kinds[i] (HSG_LAUNCH_*) and ms[i] (milliseconds between the
 * two events, the launch's duration in stream order) for launch i < *n_recorded.
 * kinds and ms are host arrays of capacity entries (NULL when capacity = 0).  The
 * events are created and destroyed inside the call.  HSG_EINVAL for capacity < 0,
 * missing outputs or a call nested inside another (per thread); HSG_EDEVICE if an
 * event cannot be created or read. */
int hsg_sweep_timed(hsg_lattice *lat, const hsg_sweep_params *p, int32_t n_sweeps, void *stream,
                    int32_t capacity, int32_t *kinds, float *ms, int32_t *n_recorded);

/* *out_dev = the energy H: the tracked value (recompute = 0) or a fresh binary64
 * sum over all bonds (recompute != 0; deterministic order).  out_dev is device
 * memory for one double. */
int hsg_energy(const hsg_lattice *lat, int32_t recompute, double *out_dev, void *stream);

/* Overlap between two configurations of the same L and dtype (binary64 sums):
 * out_dev[3*mu + nu] = (1/N) sum_i a_i^mu b_i^nu for mu, nu in {x,y,z}, then the
 * magnetisations out_dev[9..11] = (1/N) sum_i a_i, out_dev[12..14] = (1/N) sum_i b_i.
 * out_dev is device memory for 15 doubles.  a's work buffer is used as scratch. */
int hsg_overlap(const hsg_lattice *a, const hsg_lattice *b, double *out_dev, void *stream);

/* Spin-glass observables of two replicas a, b (same couplings, same L and dtype).
 * The paper defines no observable; these are the standard ones of vector spin
 * glasses, built on the local overlap tensor q_r^{mu nu} = a_r^mu b_r^nu of the
 * model of §2.  Its Fourier components
 *     Q^{mu nu}(k) = (1/N) sum_r q_r^{mu nu} exp(+i k.r),   r = (x, y, z),
 * are taken at k = 0 and at the three smallest non-zero wave-vectors
 * k_d = (2 pi / L) e_d, summed in binary64 in a fixed order (the same record on
 * every run).  One record is HSG_FOURIER_VALUES doubles:
 *     [0, 9)               Q^{mu nu}(0), row-major (= hsg_overlap's first 9 values)
 *     [9 + 18d, 18 + 18d)  Re Q^{mu nu}(k_d), d = 0, 1, 2 for x, y, z
 *     [18 + 18d, 27 + 18d) Im Q^{mu nu}(k_d)
 *     [63]                 q2(0) = sum_{mu nu} Q^{mu nu}(0)^2
 *     [64]                 q2(k_min) = (1/3) sum_d sum_{mu nu} |Q^{mu nu}(k_d)|^2
 * Over a series of records (thermal history, disorder samples), chi_SG(k) = N <q2(k)>,
 * the second-moment correlation length is sqrt(chi_SG(0)/chi_SG(k_min) - 1) /
 * (2 sin(pi/L)) and the Binder cumulant of the 9-component order parameter is
 * (11 - 9 <q2(0)^2> / <q2(0)>^2) / 2. */
#define HSG_FOURIER_VALUES 65

/* The record of lattices a and b into out_dev (device, HSG_FOURIER_VALUES doubles).
 * HSG_EINVAL if L or dtype differ or out_dev is NULL; a's work buffer is used as
 * scratch. */
int hsg_overlap_fourier(const hsg_lattice *a, const hsg_lattice *b, double *out_dev,
                        void *stream);

/* ======================================================================================
 * Batched form: many independent lattices ("chains") -- disorder samples, replicas and
 * temperatures -- advanced by one launch.  Each workgroup owns one chain and runs its
 * sweeps with workgroup barriers between colour passes; workgroups are dispatched in
 * the caller's order.  A chain computes exactly what hsg_sweep computes for the same
 * lattice.
 * ==================================================================================== */

#define HSG_BATCH_L_MAX 256 /* largest L of a chain in a batch */
#define HSG_CHAIN_INIT_J 8  /* chain flag: hsg_batch_init draws this chain's couplings */

typedef struct hsg_chain {
  int64_t spin_offset; /* element offset of the chain's spins (3*L^3 elements, internal
                          layout) in hsg_batch.spins */
  int64_t J_offset;    /* element offset of its couplings in hsg_batch.J (chains of one
                          disorder sample share them) */
  uint64_t seed;       /* Philox key of the chain's initial spins and Monte Carlo stream */
  uint64_t J_seed;     /* Philox key of the couplings (read with HSG_CHAIN_INIT_J) */
  int32_t L;           /* even, 2 <= L <= HSG_BATCH_L_MAX */
  int32_t k_hits;      /* as hsg_sweep_params */
  int32_t n_or;
  int32_t renorm_every;
  int32_t flags;       /* HSG_HEAT_BATH, HSG_CHAIN_INIT_J */
  int32_t reserved;    /* 0 */
} hsg_chain;           /* 56 bytes */

typedef struct hsg_batch {
  int32_t n_chains;
  int32_t dtype;           /* HSG_F32 or HSG_F64, for every chain */
  const hsg_chain *chains; /* device [n_chains] */
  void *spins;             /* device: base of all chains' spins */
  void *J;                 /* device: base of all couplings */
  double *beta;            /* device [n_chains]: inverse temperature of each chain */
  double *E;               /* device [n_chains]: tracked energy of each chain */
  uint32_t *sweep;         /* device [n_chains]: next sweep index of each chain */
  int32_t *remaining;      /* device [n_chains] or NULL: sweeps each chain still has to run;
                              a launch runs min(n_sweeps, remaining) and subtracts them */
  const int32_t *order;    /* device [n_chains]: a permutation, the order in which
                              workgroups are dispatched (largest L first balances load) */
  int32_t threads;         /* threads per workgroup: a multiple of 64 up to 1024 (0 = 256) */
  int32_t reserved;        /* must be 0 */
} hsg_batch;

/* Host-side check of a chain table before it is copied to the device: every chain
 * has an even 2 <= L <= HSG_BATCH_L_MAX, k_hits/n_or/renorm_every/flags as
 * hsg_sweep accepts them, and its spins (3*L^3 elements from spin_offset) and
 * couplings (from J_offset) inside buffers of spin_elems and J_elems elements; the
 * spin ranges of different chains do not overlap.  HSG_EINVAL names the first bad
 * chain.  The device entry points trust the table, so callers run this first. */
int hsg_batch_check(const hsg_chain *host_chains, int32_t n_chains, int64_t spin_elems,
                    int64_t J_elems);

/* Every chain: spins from its seed (as hsg_init_lattice); chains flagged
 * HSG_CHAIN_INIT_J also draw the couplings at their J_offset from J_seed (flag exactly
 * one chain per coupling block).  Then E = H for every chain and the work queue is
 * cleared.  beta, sweep and remaining are the caller's to set. */
int hsg_batch_init(const hsg_batch *b, void *stream);

/* Up to n_sweeps sweeps of every chain (fewer where remaining says so), each with its
 * own k_hits, n_or, renorm_every, flags, beta and sweep counter.  One launch; the
 * work queue resets itself at the end, so the call can be captured in a HIP graph and
 * replayed.  Chains must not overlap in memory except for shared couplings. */
int hsg_batch_sweep(const hsg_batch *b, int32_t n_sweeps, void *stream);

/* out_dev[c] = H of chain c, recomputed in binary64 (device array [n_chains]). */
int hsg_batch_energy(const hsg_batch *b, double *out_dev, void *stream);

/* Overlaps of chain pairs (same L): pairs_dev is a device array [n_pairs][2] of chain
 * indices; out_dev [n_pairs][15] receives Q (9, row-major), m_a (3), m_b (3) as
 * hsg_overlap does. */
int hsg_batch_overlap(const hsg_batch *b, const int32_t *pairs_dev, int32_t n_pairs,
                      double *out_dev, void *stream);

/* Records of hsg_overlap_fourier for chain pairs: pairs_dev [n_pairs][2] of chain
 * indices (device); out_dev [n_pairs][HSG_FOURIER_VALUES] (device).  A pair whose
 * indices are out of range or whose chains differ in L gets a record of NaNs. */
int hsg_batch_overlap_fourier(const hsg_batch *b, const int32_t *pairs_dev, int32_t n_pairs,
                              double *out_dev, void *stream);

/* Tiles for hsg_batch_pass_sweep: for each chain listed in active[0..n_active), its
 * colour-site range [0, L^3/2) split into runs of tile_sites (<= 1024) consecutive
 * colour sites; tiles_out[2*t] = chain, tiles_out[2*t+1] = first colour-site index.
 * Host memory.  *n_tiles receives the count; HSG_EINVAL if it would exceed capacity. */
int hsg_batch_tiles(const hsg_chain *host_chains, int32_t n_chains, const int32_t *active,
                    int32_t n_active, int32_t tile_sites, int32_t *tiles_out, int32_t capacity,
                    int32_t *n_tiles);

/* Up to n_sweeps sweeps of the chains that own tiles, as a sequence of launches: one
 * per colour pass, each covering the tiles of every listed chain (so lattices too large
 * for one workgroup still fill the GPU, and lattices of every size share launches),
 * then one per sweep for the renormalisation when renorm != 0, then a finishing launch
 * that advances b->sweep and b->remaining.  Chain c runs min(n_sweeps, remaining[c])
 * sweeps (b->remaining must be set).  All listed chains follow one pass schedule:
 * phases 0..max n_or, a chain skipping phases it does not have.  Energy changes are
 * added to b->E with device atomics (the order of the binary64 additions, and so the
 * last bits of E, may vary between runs; spins do not).  tiles_dev is a device copy
 * of the table from hsg_batch_tiles; tile_sites must match it. */
int hsg_batch_pass_sweep(const hsg_batch *b, const int32_t *tiles_dev, int32_t n_tiles,
                         int32_t tile_sites, int32_t max_n_or, int32_t renorm, int32_t n_sweeps,
                         void *stream);

/* Parallel tempering over temperature ladders of chains of a batch. */
typedef struct hsg_pt {
  int32_t n_ladders;
  int32_t n_temps;
  int32_t *chain_at_slot;     /* device [n_ladders][n_temps]: chain index in each slot */
  const double *beta_of_slot; /* device [n_temps]: inverse temperature of slot t */
  int32_t *accepted;          /* device [n_ladders][n_temps] or NULL: swaps accepted per pair */
  uint32_t *round;            /* device [1]: index n of the next exchange round */
  uint64_t seed;              /* Philox key of the exchange stream */
} hsg_pt;

/* One replica-exchange round on every ladder, n = *pt->round (then incremented on the
 * device, so the call can be captured in a HIP graph): round n proposes the slot
 * pairs (t, t+1) with t = n mod 2, t+2, ...; a pair with chains a, b is swapped with
 * probability min(1, exp((beta_t - beta_{t+1}) (E_a - E_b))) using the uniform of
 * Philox(key = seed, counter (t, n, ladder, 3)).  Swapped chains exchange slots; then
 * b->beta[chain] is set from its slot for every chain of every ladder. */
int hsg_pt_exchange(const hsg_pt *pt, const hsg_batch *b, void *stream);

/* Overlap, slot by slot, between ladders: ladder_pairs_dev [n_pairs][2] of ladder
 * indices; out_dev [n_pairs][n_temps][15] (as hsg_batch_overlap) for the chains that
 * occupy slot t of the two ladders. */
int hsg_pt_overlap(const hsg_pt *pt, const hsg_batch *b, const int32_t *ladder_pairs_dev,
                   int32_t n_pairs, double *out_dev, void *stream);

/* Records of hsg_overlap_fourier, slot by slot, between ladders: ladder_pairs_dev
 * [n_pairs][2] of ladder indices (device); out_dev [n_pairs][n_temps][HSG_FOURIER_VALUES]
 * (device) for the chains in slot t of the two ladders (records of NaNs for ladder
 * indices out of range or chains of different L).  Capturable in a HIP graph. */
int hsg_pt_overlap_fourier(const hsg_pt *pt, const hsg_batch *b,
                           const int32_t *ladder_pairs_dev, int32_t n_pairs, double *out_dev,
                           void *stream);

/* Message describing the last error returned to this thread ("" if none). */
const char *hsg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HSG_H */
