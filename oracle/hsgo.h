/*
 * hsgo -- plain CPU oracle for the checkerboard Monte Carlo sweep of the 3D
 * Heisenberg spin glass (Bernaschi, Parisi & Parisi, "The Heisenberg spin glass
 * model on GPU: myths and actual facts", arXiv:1006.2566).
 *
 * TEST INFRASTRUCTURE ONLY.  This library defines what the GPU library must
 * compute; it is slow on purpose (one site at a time, canonical layout, no
 * blocking or fusion).  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header or constant table
 * with the HIP library.
 *
 * Canonical layout (both precisions):
 *   site index i = x + L*y + L*L*z, 0 <= x,y,z < L, periodic in x, y, z (§2, eq. 2
 *   and the index formula beside it);
 *   spins: 3*N values, component-major: spins[a*N + i], a = 0,1,2 (x,y,z component);
 *   J:     3*N values, J[d*N + i] is the coupling on the bond (i, i + e_d), d = x,y,z,
 *          so every one of the 3N bonds is stored exactly once.
 * Colour of a site: c = (x + y + z) & 1; a colour pass updates all sites of one
 * colour, which share no bond (the checkerboard of §4).
 *
 * Functions with suffix _f32 compute in IEEE binary32, _f64 in binary64; all
 * energies, overlaps and accumulated energy changes are binary64.
 */
#ifndef HSGO_H
#define HSGO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox stream tags (fourth counter word). */
enum { HSGO_TAG_MH = 0, HSGO_TAG_INIT_SPIN = 1, HSGO_TAG_INIT_J = 2, HSGO_TAG_PT = 3,
       HSGO_TAG_HB = 5 };

/* One Philox4x32-10 block: out = philox(ctr, key). */
void hsgo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Uniform on (0,1) from a 32-bit word: ((w >> 9) + 1/2) * 2^-23, exact in binary32. */
double hsgo_u01(uint32_t w);
void hsgo_philox_many(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out);
/* The Monte Carlo uniforms of one site in one phase: uniform n is hsgo_u01 of word
   n % 4 of the Philox block with counter (sweep, site, (phase << 16) | n / 4, tag).
   A Metropolis hit j takes uniforms 3j, 3j+1, 3j+2; a heat-bath draw j takes 2j, 2j+1. */
typedef struct {
  uint32_t ctr[4];
  uint32_t key[2];
  int64_t block; /* block held in w, -1 before the first */
  uint32_t w[4];
} hsgo_ustream;
void hsgo_ustream_init(hsgo_ustream *us, uint64_t sweep, uint32_t site, uint32_t phase,
                       uint32_t tag, const uint32_t key[2]);
double hsgo_ustream_at(hsgo_ustream *us, int64_t n);
void hsgo_u01_many(int64_t n, const uint32_t *w, double *out);
/* Taylor coefficients of sin/cos(pi*r/2) in r: coef[k] = (-1)^floor(k/2) (pi/2)^k / k!,
   k = 0..17, correctly rounded from binary128 arithmetic. */
void hsgo_poly_coefs_f64(double out[18]);
void hsgo_poly_coefs_f32(float out[18]);
/* Constants of the own exp / log family: expm1[n] = 1/n!, atanh[j] = 1/(2j+1) for
   n, j < 18, ln2 = {head of ln 2 (a multiple of 2^-16 in binary32, 2^-32 in binary64),
   ln 2 - head, log2(e), sqrt(1/2)}; binary128 arithmetic rounded once. */
void hsgo_elem_consts_f32(float expm1[18], float atanh[18], float ln2[4]);
void hsgo_elem_consts_f64(double expm1[18], double atanh[18], double ln2[4]);

/* OpenMP threads of the parallel loops (results do not depend on the count). */
int hsgo_threads(void);
void hsgo_set_threads(int n);

/* Replica-exchange step over one temperature ladder (see hsgo_common.c). */
int hsgo_pt_swap(int32_t n_temps, const double *beta_of_slot, const double *E_of_chain,
                 int32_t *chain_at_slot, uint64_t seed, uint32_t stream_id, uint32_t round,
                 int32_t *accepted_pairs);

#define HSGO_DECLARE(R, SUF)                                                                  \
  void hsgo_sincos_2pi_##SUF(R u, R *sin_out, R *cos_out);                                    \
  void hsgo_trial_spin_##SUF(R u0, R u1, R s[3]);                                             \
  void hsgo_init_##SUF(int32_t L, uint64_t seed, R *spins, R *J);                             \
  void hsgo_field_##SUF(const R Jn[6], const R nbs[18], R h[3]);                             \
  void hsgo_local_field_##SUF(int32_t L, const R *spins, const R *J, int32_t x, int32_t y,    \
                              int32_t z, R h[3]);                                             \
  int64_t hsgo_site_update_##SUF(int32_t mode, const R h[3], R s[3], uint64_t seed,           \
                                 uint64_t sweep, uint32_t site, uint32_t phase,              \
                                 int32_t k_hits, double T, double margin_eps, double *dE,    \
                                 int64_t *accepted);                                          \
  void hsgo_overrelax_site_##SUF(const R h[3], R s[3]);                                       \
  R hsgo_exp_##SUF(R x);                                                                      \
  R hsgo_expm1_##SUF(R x);                                                                    \
  R hsgo_log_##SUF(R x);                                                                      \
  R hsgo_log1p_##SUF(R x);                                                                    \
  void hsgo_heat_bath_draw_##SUF(const R h[3], R beta, R u0, R u1, R s[3]);                  \
  void hsgo_elem_many_##SUF(int32_t which, int64_t n, const R *x, R *out);                   \
  int hsgo_sweep_##SUF(int32_t L, uint64_t seed, uint64_t sweep0, int32_t n_sweeps, double T, \
                       int32_t k_hits, int32_t n_or, int32_t renorm_every, int32_t heat_bath, \
                       R *spins, const R *J, double *E, double margin_eps, uint8_t *taint,    \
                       int64_t *n_flagged, int64_t *n_accepted);                              \
  double hsgo_energy_##SUF(int32_t L, const R *spins, const R *J);                            \
  void hsgo_overlap_##SUF(int32_t L, const R *a, const R *b, double out[15]);                 \
  void hsgo_renormalise_##SUF(int64_t n_sites, R *spins);

HSGO_DECLARE(float, f32)
HSGO_DECLARE(double, f64)

#ifdef __cplusplus
}
#endif
#endif
