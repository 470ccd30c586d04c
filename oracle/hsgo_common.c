/*
 * hsgo_common.c -- precision-independent parts of the CPU oracle.
 * TEST INFRASTRUCTURE ONLY (see hsgo.h).
 *
 * The paper leaves random numbers out on purpose (§1, end of §2); the counter-based
 * generator below is the standard Philox4x32-10 of Salmon, Moraes, Dror & Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC'11), written from its
 * definition there.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stddef.h>
#include "hsgo.h"

/* Threads the oracle's parallel loops use (OpenMP), and a way to set them: the sweep's
 * result does not depend on the count (sums are formed per plane, then in plane order). */
int hsgo_threads(void) { return omp_get_max_threads(); }
void hsgo_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* Philox4x32 with 10 rounds.  One round maps counter (c0,c1,c2,c3) and key
 * (k0,k1) through two 32x32->64 multiplications:
 *     (hi0,lo0) = 0xD2511F53 * c0,   (hi1,lo1) = 0xCD9E8D57 * c2,
 *     counter  <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
 * between rounds the key is advanced by the Weyl increments (0x9E3779B9, 0xBB67AE85). */
void hsgo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* The top 23 bits of w, centred in their cell: (2*(w>>9) + 1) * 2^-24.  The
 * result lies strictly inside (0,1) and is exact in binary32 and binary64, so the
 * two precisions see the same uniforms. */
double hsgo_u01(uint32_t w) {
  return ((double)(w >> 9) * 2.0 + 1.0) * 0x1p-24;
}

void hsgo_ustream_init(hsgo_ustream *us, uint64_t sweep, uint32_t site, uint32_t phase,
                       uint32_t tag, const uint32_t key[2]) {
  us->ctr[0] = (uint32_t)sweep;
  us->ctr[1] = site;
  us->ctr[2] = phase << 16;
  us->ctr[3] = tag;
  us->key[0] = key[0];
  us->key[1] = key[1];
  us->block = -1;
}

double hsgo_ustream_at(hsgo_ustream *us, int64_t n) {
  const int64_t b = n / 4;
  if (b != us->block) {
    uint32_t ctr[4] = {us->ctr[0], us->ctr[1], us->ctr[2] | (uint32_t)b, us->ctr[3]};
    hsgo_philox4x32_10(ctr, us->key, us->w);
    us->block = b;
  }
  return hsgo_u01(us->w[n % 4]);
}

/* coef[k] = (-1)^floor(k/2) * (pi/2)^k / k!: the Taylor coefficients, in the
 * reduced variable r, of cos(pi r / 2) (even k) and sin(pi r / 2) (odd k).
 * Evaluated in binary128 and rounded once to the target precision. */
static void poly_coefs_q(__float128 out[18]) {
  const __float128 half_pi = 3.14159265358979323846264338327950288419716939937510Q / 2;
  __float128 term = 1;
  for (int k = 0; k < 18; ++k) {
    if (k > 0) term = term * half_pi / k;
    out[k] = ((k / 2) % 2 == 0) ? term : -term;
  }
}

/* Constants of the own exp / log family, evaluated in binary128 and rounded once:
 * expm1[n] = 1/n! (n = 2..17), atanh[j] = 1/(2j+1) (j = 1..17), and ln2[] = {head of
 * ln 2 (ln 2 rounded to a multiple of 2^-split, so that e * head is exact for every
 * exponent e of the format), tail (ln 2 - head), log2(e), sqrt(1/2)}. */
static const __float128 LN2_Q = 0.693147180559945309417232121458176568075500134360255Q;
static const __float128 SQRT_HALF_Q = 0.707106781186547524400844362104849039284835937688474Q;

static void elem_consts_q(__float128 expm1[18], __float128 atanh[18]) {
  __float128 f = 1;
  for (int n = 0; n < 18; ++n) {
    if (n > 0) f = f * n;
    expm1[n] = 1 / f;
    atanh[n] = (__float128)1 / (2 * n + 1);
  }
}

void hsgo_elem_consts_f32(float expm1[18], float atanh[18], float ln2[4]) {
  __float128 e[18], a[18];
  elem_consts_q(e, a);
  for (int n = 0; n < 18; ++n) {
    expm1[n] = (float)e[n];
    atanh[n] = (float)a[n];
  }
  const __float128 head = (__float128)(int64_t)(LN2_Q * 65536 + 0.5Q) / 65536; /* 2^-16 */
  ln2[0] = (float)head;
  ln2[1] = (float)(LN2_Q - head);
  ln2[2] = (float)(1 / LN2_Q);
  ln2[3] = (float)SQRT_HALF_Q;
}

void hsgo_elem_consts_f64(double expm1[18], double atanh[18], double ln2[4]) {
  __float128 e[18], a[18];
  elem_consts_q(e, a);
  for (int n = 0; n < 18; ++n) {
    expm1[n] = (double)e[n];
    atanh[n] = (double)a[n];
  }
  const __float128 head = (__float128)(int64_t)(LN2_Q * 4294967296.0Q + 0.5Q) / 4294967296.0Q;
  ln2[0] = (double)head;
  ln2[1] = (double)(LN2_Q - head);
  ln2[2] = (double)(1 / LN2_Q);
  ln2[3] = (double)SQRT_HALF_Q;
}

void hsgo_poly_coefs_f64(double out[18]) {
  __float128 q[18];
  poly_coefs_q(q);
  for (int k = 0; k < 18; ++k) out[k] = (double)q[k];
}

void hsgo_poly_coefs_f32(float out[18]) {
  __float128 q[18];
  poly_coefs_q(q);
  for (int k = 0; k < 18; ++k) out[k] = (float)q[k];
}

/* Replica exchange (parallel tempering) over one ladder of n_temps temperature
 * slots.  Slot t holds chain chain_at_slot[t] at inverse temperature beta_of_slot[t].
 * Round n proposes the pairs (t, t+1) with t = n mod 2, t+2, ...; a pair is swapped
 * with probability min(1, exp((beta_t - beta_{t+1}) (E_a - E_b))), where a, b are
 * the chains in slots t, t+1.  The uniform comes from Philox with key = seed and
 * counter (t, round, stream_id, TAG_PT).  A swap exchanges the chains' slots
 * (their temperatures); spins never move.  The number of accepted swaps per
 * pair is added to accepted_pairs[t] when that array is given. */
int hsgo_pt_swap(int32_t n_temps, const double *beta_of_slot, const double *E_of_chain,
                 int32_t *chain_at_slot, uint64_t seed, uint32_t stream_id, uint32_t round,
                 int32_t *accepted_pairs) {
  if (n_temps < 1 || !beta_of_slot || !E_of_chain || !chain_at_slot) return -1;
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  int n_acc = 0;
  for (int32_t t = (int32_t)(round & 1u); t + 1 < n_temps; t += 2) {
    int32_t a = chain_at_slot[t], b = chain_at_slot[t + 1];
    double delta = (beta_of_slot[t] - beta_of_slot[t + 1]) * (E_of_chain[a] - E_of_chain[b]);
    uint32_t ctr[4] = {(uint32_t)t, round, stream_id, HSGO_TAG_PT}, w[4];
    hsgo_philox4x32_10(ctr, key, w);
    double u = hsgo_u01(w[0]);
    int accept = (delta >= 0.0) || (u < exp(delta));
    if (accept) {
      chain_at_slot[t] = b;
      chain_at_slot[t + 1] = a;
      ++n_acc;
      if (accepted_pairs) accepted_pairs[t] += 1;
    }
  }
  return n_acc;
}

/* Convenience loops for the Python shim: n Philox blocks and n uniforms. */
void hsgo_philox_many(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out) {
  for (int64_t i = 0; i < n; ++i) hsgo_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

void hsgo_u01_many(int64_t n, const uint32_t *w, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = hsgo_u01(w[i]);
}
