/* Drives every entry point of the CPU oracle at small sizes, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (the oracle keeps per-plane arrays
 * of length L on the stack and indexes neighbours with periodic wrap-around).
 * Exits 0 when every call returns normally and the results are finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include "hsgo.h"

#define RUN(R, SUF)                                                                          \
  static int run_##SUF(int32_t L) {                                                          \
    const int64_t N = (int64_t)L * L * L;                                                    \
    R *s = malloc(sizeof(R) * 3 * N), *J = malloc(sizeof(R) * 3 * N);                        \
    R *b = malloc(sizeof(R) * 3 * N);                                                        \
    uint8_t *taint = calloc((size_t)N, 1);                                                   \
    if (!s || !J || !b || !taint) return 1;                                                  \
    hsgo_init_##SUF(L, 7, s, J);                                                             \
    hsgo_init_##SUF(L, 8, b, J);                                                             \
    double E = hsgo_energy_##SUF(L, s, J);                                                   \
    int64_t fl = 0, ac = 0;                                                                  \
    int rc = hsgo_sweep_##SUF(L, 7, 0, 3, 0.5, 4, 2, 2, 0, s, J, &E, 1e-3, taint, &fl, &ac); \
    rc |= hsgo_sweep_##SUF(L, 7, 3, 2, 0.3, 3, 1, 1, 1, s, J, &E, 1e-6, taint, &fl, &ac);    \
    rc |= hsgo_sweep_##SUF(L, 7, 5, 1, INFINITY, 1, 0, 0, 0, s, J, NULL, 1e-6, NULL, NULL,   \
                           NULL);                                                            \
    R h[3];                                                                                  \
    hsgo_local_field_##SUF(L, s, J, L - 1, 0, L - 1, h);                                     \
    hsgo_overrelax_site_##SUF(h, s);                                                         \
    R t[3];                                                                                  \
    hsgo_heat_bath_draw_##SUF(h, (R)2, (R)0.25, (R)0.75, t);                                 \
    double ov[15];                                                                           \
    hsgo_overlap_##SUF(L, s, b, ov);                                                         \
    hsgo_renormalise_##SUF(N, s);                                                            \
    R x[4] = {(R)-3, (R)0.25, (R)1.5, (R)-0.5}, y[4];                                        \
    for (int w = 0; w < 4; ++w) hsgo_elem_many_##SUF(w, 4, x, y);                            \
    E += hsgo_energy_##SUF(L, s, J);                                                         \
    int bad = rc != 0 || !isfinite(E) || !isfinite(ov[0]) || !isfinite((double)t[0]);        \
    free(s);                                                                                 \
    free(J);                                                                                 \
    free(b);                                                                                 \
    free(taint);                                                                             \
    return bad;                                                                              \
  }
RUN(float, f32)
RUN(double, f64)

int main(void) {
  const int32_t sizes[] = {2, 4, 6, 8, 10};
  int bad = 0;
  for (int i = 0; i < 5; ++i) bad |= run_f32(sizes[i]) | run_f64(sizes[i]);
  double beta[4] = {2.0, 1.5, 1.0, 0.5}, E[4] = {-3.0, -1.0, -2.0, 0.5};
  int32_t slot[4] = {0, 1, 2, 3}, acc[4] = {0, 0, 0, 0};
  for (uint32_t r = 0; r < 6; ++r) hsgo_pt_swap(4, beta, E, slot, 11, 0, r, acc);
  uint32_t ctr[8] = {1, 2, 3, 4, 5, 6, 7, 8}, key[2] = {9, 10}, out[8];
  hsgo_philox_many(2, ctr, key, out);
  double u[8];
  hsgo_u01_many(8, out, u);
  printf("oracle sanitizer run: %s\n", bad ? "FAILED" : "ok");
  return bad;
}
