/* Binary32 instance of the CPU oracle.  TEST INFRASTRUCTURE ONLY (see hsgo.h). */
#include <math.h>
#include <stdint.h>
#include "hsgo.h"
#define R float
#define SUF f32
#define RSQRT sqrtf
#define REXP expf
#define RLOG logf
#define RLOG1P log1pf
#define REXPM1 expm1f
#define RFMA fmaf
#define RRINT rintf
#define RFABS fabs
#define N_SIN 5 /* sin terms r^1 .. r^9 */
#define N_COS 6 /* cos terms r^0 .. r^10 */
#define POLY_COEFS hsgo_poly_coefs_f32
#include "hsgo_real.inc"
