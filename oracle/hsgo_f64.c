/* Binary64 instance of the CPU oracle.  TEST INFRASTRUCTURE ONLY (see hsgo.h). */
#include <math.h>
#include <stdint.h>
#include "hsgo.h"
#define R double
#define SUF f64
#define RSQRT sqrt
#define REXP exp
#define RFMA fma
#define RRINT rint
#define RFABS fabs
#define N_SIN 9 /* sin terms r^1 .. r^17 */
#define N_COS 9 /* cos terms r^0 .. r^16 */
#define POLY_COEFS hsgo_poly_coefs_f64
#define RFREXP frexp
#define RLDEXP ldexp
#define N_EXPM1 13
#define N_ATANH 17
#define EXP_XMIN -700.0
#define CONSTS hsgo_elem_consts_f64
#include "hsgo_real.inc"
