/* Binary32 instance of the CPU oracle.  TEST INFRASTRUCTURE ONLY (see hsgo.h). */
#include <math.h>
#include <stdint.h>
#include "hsgo.h"
#define R float
#define SUF f32
#define RSQRT sqrtf
#define REXP expf
#define RFMA fmaf
#define RRINT rintf
#define RFABS fabs
#define N_SIN 5 /* sin terms r^1 .. r^9 */
#define N_COS 6 /* cos terms r^0 .. r^10 */
#define POLY_COEFS hsgo_poly_coefs_f32
#define RFREXP frexpf
#define RLDEXP ldexpf
#define N_EXPM1 8
#define N_ATANH 7
#define EXP_XMIN -80.0f
#define CONSTS hsgo_elem_consts_f32
#include "hsgo_real.inc"
