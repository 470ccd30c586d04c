/* Binary64 instance of the CPU oracle.  TEST INFRASTRUCTURE ONLY (see hsgo.h). */
#include <math.h>
#include <stdint.h>
#include "hsgo.h"
#define R double
#define SUF f64
#define RSQRT sqrt
#define REXP exp
#define RLOG log
#define RLOG1P log1p
#define REXPM1 expm1
#define RFMA fma
#define RRINT rint
#define RFABS fabs
#define N_SIN 9 /* sin terms r^1 .. r^17 */
#define N_COS 9 /* cos terms r^0 .. r^16 */
#define POLY_COEFS hsgo_poly_coefs_f64
#include "hsgo_real.inc"
