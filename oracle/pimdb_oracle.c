/*
 * CPU oracle for the bosonic PIMD exchange potential and forces
 * (Feldman & Hirshberg, "Quadratic Scaling Bosonic Path Integral Molecular
 * Dynamics").  TEST INFRASTRUCTURE: only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the GPU library.
 *
 * The body (oracle_body.h) is compiled twice:
 *   *_f64 : IEEE double, round to nearest, no fast-math;
 *   *_f80 : x87 long double (64-bit significand), the high-precision
 *           reference used to measure the rounding error of FP64 results.
 *
 * Build: gcc -O2 -fno-fast-math -std=c11 -shared -fPIC pimdb_oracle.c -lm
 */
#include <math.h>
#include <stdlib.h>
#include <stddef.h>

#define REAL double
#define SFX _f64
#define EXP exp
#define LOG log
#define EXPM1 expm1
#define RINT rint
#include "oracle_body.h"
#undef REAL
#undef SFX
#undef EXP
#undef LOG
#undef EXPM1
#undef RINT

#define REAL long double
#define SFX _f80
#define EXP expl
#define LOG logl
#define EXPM1 expm1l
#define RINT rintl
#include "oracle_body.h"
#undef REAL
#undef SFX
#undef EXP
#undef LOG
#undef EXPM1
#undef RINT

/* size of the significand of long double on this host (64 on x86-64) */
int orc_long_double_mant_dig(void) { return __LDBL_MANT_DIG__; }
