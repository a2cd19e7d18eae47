/*
 * AM-QFT ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, recursive CPU implementation of the eight AM-QFT variants of
 * L. Pasquini, "A class of AM-QFT algorithms for power-of-two FFT"
 * (arXiv:1404.1810), plus the direct O(N^2) definitions of the CDFT, DCT-0 and
 * DST-0.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this code; the GPU library never does, and the two share no
 * source.
 *
 * Conventions (the paper's own notation):
 *   - every signal of periodization L is held in a "full-index" array of
 *     length L/2+1 (L for the CDFT/RDFT), indexed by the time index n (for s)
 *     or the harmonic k (for S); only the entries in sto_n / sto_k of the
 *     signal type (Table "tab:notation") are read or written.
 *   - REAL is double for the truth build and float for the same-precision
 *     emulation build; trigonometric constants are always evaluated in double
 *     and rounded once to REAL.
 *   - The fixed-point build (ORACLE_FIXED; Sec. 7.2 binary translations,
 *     Sec. 7.4 fixed-point implementations) holds every value as a 32-bit
 *     two's-complement integer in units of the input's last bit, and each
 *     constant as round(f * 2^29) (Q2.29; f in (-2, 2): the 2cos / 2sin
 *     families of variants 1, 3, 5, 7 -- the 1/(2cos) / 1/(2sin) families of
 *     the other four are unbounded and have no such format).  Additions are
 *     exact; a product a * k is round((a k) / 2^29) and a halving is
 *     round(a / 2), both to nearest with ties away from zero (the binary
 *     translation of the magnitude, sign restored: rounding commutes with
 *     negation, so a sign flip anywhere in the data changes no rounding); a
 *     result outside int32 wraps and is counted.  Additions being exact, the
 *     result depends only on which values are rounded, not on the order of
 *     the sums.
 *   - Every real addition/subtraction, multiplication by a constant and
 *     halving (binary translation, Sec. 7.2) goes through add/sub/mul/half so
 *     that the counts can be compared with Tables "tab:costo_varianti" and
 *     "tab:compara_*".
 *
 * Parity pins (see tests/test_oracle*.py): brute force against the direct
 * DFT, closed forms, Parseval/linearity/shift, real-input symmetry, operation
 * counts equal to the paper's tables, constants touched, bitwise equality of
 * all variants for N <= 8, and every sub-function against its direct DCT-0 /
 * DST-0 definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_FIXED
typedef int32_t REAL;
#define Q_FRAC 29
static long long g_wraps; /* results that left the int32 range */
static REAL wrap32(long long v)
{
    if (v < INT32_MIN || v > INT32_MAX) g_wraps++;
    return (REAL)(int32_t)(uint32_t)(uint64_t)v;
}
#else
#ifndef ORACLE_REAL
#define ORACLE_REAL double
#endif
typedef ORACLE_REAL REAL;
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    long long adds;   /* real additions and subtractions                */
    long long mults;  /* real multiplications by a trigonometric constant */
    long long halves; /* real multiplications by 1/2 (binary translations) */
    long long base_const_uses; /* uses of cos(pi/4) = sin(pi/4) (base cases) */
} oracle_counts;

typedef struct {
    int variant;            /* 1..8                                       */
    long N;                 /* periodization of the outermost transform   */
    oracle_counts *cnt;     /* may be NULL                                */
    unsigned char *touched; /* N/4 flags, index p of theta_N * p; or NULL */
} ctx_t;

/* ------------------------------------------------------------------ */
/* counted arithmetic                                                   */
/* ------------------------------------------------------------------ */
#ifdef ORACLE_FIXED
static REAL add(ctx_t *c, REAL a, REAL b) { if (c->cnt) c->cnt->adds++; return wrap32((long long)a + b); }
static REAL sub(ctx_t *c, REAL a, REAL b) { if (c->cnt) c->cnt->adds++; return wrap32((long long)a - b); }
/* round(v / 2^s) to nearest, ties away from zero */
static long long round_shift(long long v, int s)
{
    const long long h = 1LL << (s - 1);
    return v >= 0 ? (v + h) >> s : -((-v + h) >> s);
}
static REAL mul(ctx_t *c, REAL a, REAL k)
{
    if (c->cnt) c->cnt->mults++;
    return wrap32(round_shift((long long)a * k, Q_FRAC));
}
static REAL half(ctx_t *c, REAL a) { if (c->cnt) c->cnt->halves++; return wrap32(round_shift(a, 1)); }
#else
static REAL add(ctx_t *c, REAL a, REAL b) { if (c->cnt) c->cnt->adds++; return a + b; }
static REAL sub(ctx_t *c, REAL a, REAL b) { if (c->cnt) c->cnt->adds++; return a - b; }
static REAL mul(ctx_t *c, REAL a, REAL k) { if (c->cnt) c->cnt->mults++; return a * k; }
static REAL half(ctx_t *c, REAL a) { if (c->cnt) c->cnt->halves++; return a * (REAL)0.5; }
#endif

/* families of stored constants, Sec. 7.1 */
enum { COS2 = 0, SIN2 = 1, SEC2 = 2, CSC2 = 3 };

/* The constant f(theta*j) with theta = 2*pi/L (the periodization of the
 * dct_oo/dst_oo call).  In terms of the outermost transform this is
 * f(theta_N * p) with p = j*N/L, 1 <= p <= N/4-1 (Sec. 7.1); p is recorded. */
static REAL konst(ctx_t *c, int fam, long j, long L)
{
    long p = j * (c->N / L);
    if (c->touched && p >= 0 && p < c->N / 4) c->touched[p] = 1;
#ifdef ORACLE_FIXED
    /* the exact f(2 pi j / L), in long double, rounded once to Q2.29 */
    const long double pi = 3.141592653589793238462643383279502884L;
    long double al = 2.0L * pi * (long double)j / (long double)L;
    long double f = fam == COS2 ? 2.0L * cosl(al) : 2.0L * sinl(al);
    return (REAL)llroundl(f * (long double)(1L << Q_FRAC));
#endif
    double a = 2.0 * M_PI * (double)j / (double)L;
    double v;
    switch (fam) {
    case COS2: v = 2.0 * cos(a); break;
    case SIN2: v = 2.0 * sin(a); break;
    case SEC2: v = 1.0 / (2.0 * cos(a)); break;
    default:   v = 1.0 / (2.0 * sin(a)); break;
    }
    return (REAL)v;
}

/* cos(pi/4) = sin(pi/4), the constant of the N = 8 base cases (Sec. 7.1) */
static REAL base_const(ctx_t *c)
{
    if (c->cnt) c->cnt->base_const_uses++;
#ifdef ORACLE_FIXED
    return (REAL)llroundl(cosl(3.141592653589793238462643383279502884L / 4.0L) * (long double)(1L << Q_FRAC));
#else
    return (REAL)cos(M_PI / 4.0);
#endif
}

static REAL *alloc(long n)
{
    REAL *p = (REAL *)calloc((size_t)(n > 0 ? n : 1), sizeof(REAL));
    return p;
}

static int skeleton_a(int v) { return v == 1 || v == 4 || v == 5 || v == 8; }

/* forward declarations of the recursive functions (Sec. 4 and 6) */
static void dct(ctx_t *c, long L, const REAL *s, REAL *S);
static void dst(ctx_t *c, long L, const REAL *s, REAL *S);
static void dct_ot(ctx_t *c, long L, const REAL *s, REAL *S);
static void dst_ot(ctx_t *c, long L, const REAL *s, REAL *S);
static void dct_to(ctx_t *c, long L, const REAL *s, REAL *S);
static void dst_to(ctx_t *c, long L, const REAL *s, REAL *S);
static void dct_oo(ctx_t *c, long L, const REAL *s, REAL *S);
static void dst_oo(ctx_t *c, long L, const REAL *s, REAL *S);

/* ------------------------------------------------------------------ */
/* dct[L]: DCT-0 of s_dc_tt, n,k in 0..L/2 (eq. qft_0B)                 */
/* ------------------------------------------------------------------ */
static void dct(ctx_t *c, long L, const REAL *s, REAL *S)
{
    if (L == 2) { /* direct definition: cos(0) = 1, cos(pi) = -1 */
        S[0] = add(c, s[0], s[1]);
        S[1] = sub(c, s[0], s[1]);
        return;
    }
    long q = L / 4;
    if (skeleton_a(c->variant)) {
        /* D_n (DCT context, Table tab:elabora_relations_B): even n -> s_dc_et,
         * halved by H_n into s_dc_tt[L/2]; odd n -> s_dc_ot[L]. */
        REAL *e = alloc(L / 4 + 1), *E = alloc(L / 4 + 1);
        REAL *o = alloc(L / 2 + 1), *O = alloc(L / 2 + 1);
        for (long nA = 0; nA <= L / 4; nA++) e[nA] = s[2 * nA];
        for (long n = 1; n < L / 2; n += 2) o[n] = s[n];
        dct(c, L / 2, e, E);
        dct_ot(c, L, o, O);
        for (long k = 0; k < q; k++) {
            S[k] = add(c, E[k], O[k]);
            S[L / 2 - k] = sub(c, E[k], O[k]);
        }
        S[q] = E[q];
        free(e); free(E); free(o); free(O);
    } else {
        /* D_k (DCT context): sums feed the even harmonics (s_dc_te, halved by
         * H_k into s_dc_tt[L/2]), differences the odd ones (s_dc_to[L]). */
        REAL *e = alloc(L / 4 + 1), *E = alloc(L / 4 + 1);
        REAL *o = alloc(L / 2 + 1), *O = alloc(L / 2 + 1);
        for (long n = 0; n < q; n++) {
            e[n] = add(c, s[n], s[L / 2 - n]);
            o[n] = sub(c, s[n], s[L / 2 - n]);
        }
        e[q] = s[q];
        dct(c, L / 2, e, E);
        dct_to(c, L, o, O);
        for (long kA = 0; kA <= q; kA++) S[2 * kA] = E[kA];
        for (long k = 1; k < L / 2; k += 2) S[k] = O[k];
        free(e); free(E); free(o); free(O);
    }
}

/* ------------------------------------------------------------------ */
/* dst[L]: DST-0 of s_ds_tt, n,k in 1..L/2-1 (eq. qft_0C)               */
/* ------------------------------------------------------------------ */
static void dst(ctx_t *c, long L, const REAL *s, REAL *S)
{
    if (L == 4) { /* direct definition: sin(pi/2) = 1 */
        S[1] = s[1];
        return;
    }
    long q = L / 4;
    if (skeleton_a(c->variant)) {
        /* D_n (DST context): even n -> s_ds_et -> H_n -> s_ds_tt[L/2];
         * odd n -> s_ds_ot[L]. */
        REAL *e = alloc(L / 4 + 1), *E = alloc(L / 4 + 1);
        REAL *o = alloc(L / 2 + 1), *O = alloc(L / 2 + 1);
        for (long nA = 1; nA < L / 4; nA++) e[nA] = s[2 * nA];
        for (long n = 1; n < L / 2; n += 2) o[n] = s[n];
        dst(c, L / 2, e, E);
        dst_ot(c, L, o, O);
        for (long k = 1; k < q; k++) {
            S[k] = add(c, O[k], E[k]);
            S[L / 2 - k] = sub(c, O[k], E[k]);
        }
        S[q] = O[q];
        free(e); free(E); free(o); free(O);
    } else {
        /* D_k (DST context): differences feed the even harmonics (s_ds_te ->
         * H_k -> s_ds_tt[L/2]), sums the odd ones (s_ds_to[L]). */
        REAL *e = alloc(L / 4 + 1), *E = alloc(L / 4 + 1);
        REAL *o = alloc(L / 2 + 1), *O = alloc(L / 2 + 1);
        for (long n = 1; n < q; n++) {
            e[n] = sub(c, s[n], s[L / 2 - n]);
            o[n] = add(c, s[n], s[L / 2 - n]);
        }
        o[q] = s[q];
        dst(c, L / 2, e, E);
        dst_to(c, L, o, O);
        for (long kA = 1; kA < q; kA++) S[2 * kA] = E[kA];
        for (long k = 1; k < L / 2; k += 2) S[k] = O[k];
        free(e); free(E); free(o); free(O);
    }
}

/* ------------------------------------------------------------------ */
/* dct_ot[L]: s_dc_ot, n odd < L/2, k = 0..L/4-1 (skeleton A)           */
/* ------------------------------------------------------------------ */
static void dct_ot(ctx_t *c, long L, const REAL *s, REAL *S)
{
    if (L == 4) { S[0] = s[1]; return; }
    long q = L / 4;
    REAL *e = alloc(L / 4 + 1), *F = alloc(L / 4 + 1);
    REAL *o = alloc(L / 2 + 1), *O = alloc(L / 2 + 1);
    /* D_k (DCT context): s_dc_ot -> (s_dc_oe, s_dc_oo) */
    for (long n = 1; n < q; n += 2) {
        e[n] = add(c, s[n], s[L / 2 - n]);
        o[n] = sub(c, s[n], s[L / 2 - n]);
    }
    /* H_k: s_dc_oe[L] -> s_dc_ot[L/2], same samples, S_oe(2kA) = S_ot(kA) */
    dct_ot(c, L / 2, e, F);
    dct_oo(c, L, o, O);
    for (long kA = 0; kA < L / 8; kA++) S[2 * kA] = F[kA];
    for (long k = 1; k < q; k += 2) S[k] = O[k];
    free(e); free(F); free(o); free(O);
}

/* ------------------------------------------------------------------ */
/* dst_ot[L]: s_ds_ot, n odd < L/2, k = 1..L/4 (skeleton A)             */
/* ------------------------------------------------------------------ */
static void dst_ot(ctx_t *c, long L, const REAL *s, REAL *S)
{
    if (L == 4) { S[1] = s[1]; return; }
    long q = L / 4;
    REAL *e = alloc(L / 4 + 1), *F = alloc(L / 4 + 1);
    REAL *o = alloc(L / 2 + 1), *O = alloc(L / 2 + 1);
    /* D_k (DST context): difference -> s_ds_oe (even k), sum -> s_ds_oo */
    for (long n = 1; n < q; n += 2) {
        e[n] = sub(c, s[n], s[L / 2 - n]);
        o[n] = add(c, s[n], s[L / 2 - n]);
    }
    dst_ot(c, L / 2, e, F); /* H_k: s_ds_oe[L] -> s_ds_ot[L/2] */
    dst_oo(c, L, o, O);
    for (long kA = 1; kA <= L / 8; kA++) S[2 * kA] = F[kA];
    for (long k = 1; k < q; k += 2) S[k] = O[k];
    free(e); free(F); free(o); free(O);
}

/* ------------------------------------------------------------------ */
/* dct_to[L]: s_dc_to, n = 0..L/4-1, k odd < L/2 (skeleton B)           */
/* ------------------------------------------------------------------ */
static void dct_to(ctx_t *c, long L, const REAL *s, REAL *S)
{
    if (L == 4) { S[1] = s[0]; return; }
    long q = L / 4;
    REAL *t = alloc(L / 4 + 1), *E = alloc(L / 4 + 1);
    REAL *o = alloc(L / 2 + 1), *O = alloc(L / 2 + 1);
    /* D_n (DCT context): even n -> s_dc_eo -> H_n -> s_dc_to[L/2];
     * odd n -> s_dc_oo[L] */
    for (long j = 0; j < q / 2; j++) t[j] = s[2 * j];
    for (long n = 1; n < q; n += 2) o[n] = s[n];
    dct_to(c, L / 2, t, E);
    dct_oo(c, L, o, O);
    for (long k = 1; k < q; k += 2) {
        S[k] = add(c, E[k], O[k]);
        S[L / 2 - k] = sub(c, E[k], O[k]);
    }
    free(t); free(E); free(o); free(O);
}

/* ------------------------------------------------------------------ */
/* dst_to[L]: s_ds_to, n = 1..L/4, k odd < L/2 (skeleton B)             */
/* ------------------------------------------------------------------ */
static void dst_to(ctx_t *c, long L, const REAL *s, REAL *S)
{
    if (L == 4) { S[1] = s[1]; return; }
    long q = L / 4;
    REAL *t = alloc(L / 4 + 1), *E = alloc(L / 4 + 1);
    REAL *o = alloc(L / 2 + 1), *O = alloc(L / 2 + 1);
    /* D_n (DST context): even n -> s_ds_eo -> H_n -> s_ds_to[L/2];
     * odd n -> s_ds_oo[L] */
    for (long j = 1; j <= q / 2; j++) t[j] = s[2 * j];
    for (long n = 1; n < q; n += 2) o[n] = s[n];
    dst_to(c, L / 2, t, E);
    dst_oo(c, L, o, O);
    for (long k = 1; k < q; k += 2) {
        S[k] = add(c, O[k], E[k]);
        S[L / 2 - k] = sub(c, O[k], E[k]);
    }
    free(t); free(E); free(o); free(O);
}

/* ------------------------------------------------------------------ */
/* dct_oo[L]: s_dc_oo, n and k odd < L/4 (Table tab:DCT_odd_transf.)    */
/* The M relations below are re-derived from the AM DSB-SC identity     */
/* (eqs. qft_36-38) where the printed table is garbled. */
/* ------------------------------------------------------------------ */
static void dct_oo(ctx_t *c, long L, const REAL *s, REAL *S)
{
    if (L == 8) { S[1] = mul(c, s[1], base_const(c)); return; }
    long q = L / 4;
    REAL *e = alloc(L / 2 + 1), *E = alloc(L / 2 + 1);
    REAL *t = alloc(L / 4 + 1), *F = alloc(L / 4 + 1);
    switch (c->variant) {
    case 1: /* M1: s_dc_oe(n) = 2cos(theta n) s(n); recurrence in frequency */
        for (long n = 1; n < q; n += 2) e[n] = mul(c, s[n], konst(c, COS2, n, L));
        dct_ot(c, L / 2, e, F);
        for (long kA = 0; kA < L / 8; kA++) E[2 * kA] = F[kA];
        S[1] = half(c, E[0]);
        for (long k = 2; k <= q - 2; k += 2) S[k + 1] = sub(c, E[k], S[k - 1]);
        break;
    case 4: /* M4 (improved QFT): s_dc_oe(n) = s(n) / (2cos(theta n)) */
        for (long n = 1; n < q; n += 2) e[n] = mul(c, s[n], konst(c, SEC2, n, L));
        dct_ot(c, L / 2, e, F);
        for (long kA = 0; kA < L / 8; kA++) E[2 * kA] = F[kA];
        for (long k = 1; k <= q - 3; k += 2) S[k] = add(c, E[k - 1], E[k + 1]);
        S[q - 1] = E[q - 2];
        break;
    case 5: /* M5: s_ds_oe(n) = 2sin(theta n) s(n); the child is a DST */
        for (long n = 1; n < q; n += 2) e[n] = mul(c, s[n], konst(c, SIN2, n, L));
        dst_ot(c, L / 2, e, F);
        for (long kA = 1; kA <= L / 8; kA++) E[2 * kA] = F[kA];
        S[q - 1] = half(c, E[q]);
        for (long k = q - 2; k >= 2; k -= 2) S[k - 1] = add(c, E[k], S[k + 1]);
        break;
    case 8: /* M8: s_ds_oe(n) = s(n) / (2sin(theta n)) */
        for (long n = 1; n < q; n += 2) e[n] = mul(c, s[n], konst(c, CSC2, n, L));
        dst_ot(c, L / 2, e, F);
        for (long kA = 1; kA <= L / 8; kA++) E[2 * kA] = F[kA];
        S[1] = E[2];
        for (long k = 3; k <= q - 1; k += 2) S[k] = sub(c, E[k + 1], E[k - 1]);
        break;
    case 2: /* M2: neighbour sums in time (s_dc_eo), 1/(2cos) in frequency */
        e[0] = s[1];
        for (long n = 2; n <= q - 2; n += 2) e[n] = add(c, s[n - 1], s[n + 1]);
        for (long j = 0; j < q / 2; j++) t[j] = e[2 * j]; /* H_n */
        dct_to(c, L / 2, t, F);
        for (long k = 1; k < q; k += 2) S[k] = mul(c, F[k], konst(c, SEC2, k, L));
        break;
    case 3: /* M3: recurrence in time (s_dc_eo), 2cos in frequency */
        e[q - 2] = s[q - 1];
        for (long n = q - 4; n >= 2; n -= 2) e[n] = sub(c, s[n + 1], e[n + 2]);
        e[0] = half(c, sub(c, s[1], e[2]));
        for (long j = 0; j < q / 2; j++) t[j] = e[2 * j];
        dct_to(c, L / 2, t, F);
        for (long k = 1; k < q; k += 2) S[k] = mul(c, F[k], konst(c, COS2, k, L));
        break;
    case 6: /* M6: neighbour differences in time (s_ds_eo), 1/(2sin) */
        e[q] = s[q - 1];
        for (long n = 2; n <= q - 2; n += 2) e[n] = sub(c, s[n - 1], s[n + 1]);
        for (long j = 1; j <= q / 2; j++) t[j] = e[2 * j];
        dst_to(c, L / 2, t, F);
        for (long k = 1; k < q; k += 2) S[k] = mul(c, F[k], konst(c, CSC2, k, L));
        break;
    case 7: /* M7: recurrence in time (s_ds_eo), 2sin in frequency */
        e[2] = s[1];
        for (long n = 4; n <= q - 2; n += 2) e[n] = add(c, s[n - 1], e[n - 2]);
        e[q] = half(c, add(c, s[q - 1], e[q - 2]));
        for (long j = 1; j <= q / 2; j++) t[j] = e[2 * j];
        dst_to(c, L / 2, t, F);
        for (long k = 1; k < q; k += 2) S[k] = mul(c, F[k], konst(c, SIN2, k, L));
        break;
    }
    free(e); free(E); free(t); free(F);
}

/* ------------------------------------------------------------------ */
/* dst_oo[L]: s_ds_oo, n and k odd < L/4 (Table tab:DST_odd_transf.)    */
/* ------------------------------------------------------------------ */
static void dst_oo(ctx_t *c, long L, const REAL *s, REAL *S)
{
    if (L == 8) { S[1] = mul(c, s[1], base_const(c)); return; }
    long q = L / 4;
    REAL *e = alloc(L / 2 + 1), *E = alloc(L / 2 + 1);
    REAL *t = alloc(L / 4 + 1), *F = alloc(L / 4 + 1);
    switch (c->variant) {
    case 1: /* M1: s_ds_oe(n) = 2cos(theta n) s(n); recurrence from k = q */
        for (long n = 1; n < q; n += 2) e[n] = mul(c, s[n], konst(c, COS2, n, L));
        dst_ot(c, L / 2, e, F);
        for (long kA = 1; kA <= L / 8; kA++) E[2 * kA] = F[kA];
        S[q - 1] = half(c, E[q]);
        for (long k = q - 2; k >= 2; k -= 2) S[k - 1] = sub(c, E[k], S[k + 1]);
        break;
    case 4: /* M4: s_ds_oe(n) = s(n) / (2cos(theta n)) */
        for (long n = 1; n < q; n += 2) e[n] = mul(c, s[n], konst(c, SEC2, n, L));
        dst_ot(c, L / 2, e, F);
        for (long kA = 1; kA <= L / 8; kA++) E[2 * kA] = F[kA];
        S[1] = E[2];
        for (long k = 3; k <= q - 1; k += 2) S[k] = add(c, E[k - 1], E[k + 1]);
        break;
    case 5: /* M5: s_dc_oe(n) = 2sin(theta n) s(n); the child is a DCT */
        for (long n = 1; n < q; n += 2) e[n] = mul(c, s[n], konst(c, SIN2, n, L));
        dct_ot(c, L / 2, e, F);
        for (long kA = 0; kA < L / 8; kA++) E[2 * kA] = F[kA];
        S[1] = half(c, E[0]);
        for (long k = 2; k <= q - 2; k += 2) S[k + 1] = add(c, E[k], S[k - 1]);
        break;
    case 8: /* M8: s_dc_oe(n) = s(n) / (2sin(theta n)) */
        for (long n = 1; n < q; n += 2) e[n] = mul(c, s[n], konst(c, CSC2, n, L));
        dct_ot(c, L / 2, e, F);
        for (long kA = 0; kA < L / 8; kA++) E[2 * kA] = F[kA];
        for (long k = 1; k <= q - 3; k += 2) S[k] = sub(c, E[k - 1], E[k + 1]);
        S[q - 1] = E[q - 2];
        break;
    case 2: /* M2: s_ds_eo neighbour sums, 1/(2cos) in frequency */
        e[q] = s[q - 1];
        for (long n = 2; n <= q - 2; n += 2) e[n] = add(c, s[n + 1], s[n - 1]);
        for (long j = 1; j <= q / 2; j++) t[j] = e[2 * j];
        dst_to(c, L / 2, t, F);
        for (long k = 1; k < q; k += 2) S[k] = mul(c, F[k], konst(c, SEC2, k, L));
        break;
    case 3: /* M3: s_ds_eo recurrence from n = 2, 2cos in frequency */
        e[2] = s[1];
        for (long n = 4; n <= q - 2; n += 2) e[n] = sub(c, s[n - 1], e[n - 2]);
        e[q] = half(c, sub(c, s[q - 1], e[q - 2]));
        for (long j = 1; j <= q / 2; j++) t[j] = e[2 * j];
        dst_to(c, L / 2, t, F);
        for (long k = 1; k < q; k += 2) S[k] = mul(c, F[k], konst(c, COS2, k, L));
        break;
    case 6: /* M6: s_dc_eo neighbour differences, 1/(2sin) in frequency */
        e[0] = s[1];
        for (long n = 2; n <= q - 2; n += 2) e[n] = sub(c, s[n + 1], s[n - 1]);
        for (long j = 0; j < q / 2; j++) t[j] = e[2 * j];
        dct_to(c, L / 2, t, F);
        for (long k = 1; k < q; k += 2) S[k] = mul(c, F[k], konst(c, CSC2, k, L));
        break;
    case 7: /* M7: s_dc_eo recurrence from n = q-2, 2sin in frequency */
        e[q - 2] = s[q - 1];
        for (long n = q - 4; n >= 2; n -= 2) e[n] = add(c, s[n + 1], e[n + 2]);
        e[0] = half(c, add(c, s[1], e[2]));
        for (long j = 0; j < q / 2; j++) t[j] = e[2 * j];
        dct_to(c, L / 2, t, F);
        for (long k = 1; k < q; k += 2) S[k] = mul(c, F[k], konst(c, SIN2, k, L));
        break;
    }
    free(e); free(E); free(t); free(F);
}

/* ------------------------------------------------------------------ */
/* rdft[N]: decomposition D_r (eqs. qft_22-25).                         */
/* Output: Re R(k) for k = 0..N/2 in Rr, Im R(k) for k = 0..N/2 in Ri.  */
/* ------------------------------------------------------------------ */
static void rdft(ctx_t *c, long N, const REAL *r, REAL *Rr, REAL *Ri)
{
    if (N == 1) { Rr[0] = r[0]; Ri[0] = 0; return; }
    if (N == 2) { /* direct definition */
        Rr[0] = add(c, r[0], r[1]);
        Rr[1] = sub(c, r[0], r[1]);
        Ri[0] = 0; Ri[1] = 0;
        return;
    }
    REAL *cc = alloc(N / 2 + 1), *C = alloc(N / 2 + 1);
    REAL *d = alloc(N / 2 + 1), *D = alloc(N / 2 + 1);
    cc[0] = r[0];
    cc[N / 2] = r[N / 2];
    for (long n = 1; n < N / 2; n++) {
        cc[n] = add(c, r[n], r[N - n]);   /* eq. qft_22 */
        d[n] = sub(c, r[n], r[N - n]);    /* eq. qft_23 */
    }
    dct(c, N, cc, C);
    dst(c, N, d, D);
    for (long k = 0; k <= N / 2; k++) Rr[k] = C[k];          /* eq. qft_24 */
    Ri[0] = 0; Ri[N / 2] = 0;
    for (long k = 1; k < N / 2; k++) Ri[k] = -D[k];          /* eq. qft_25 */
    free(cc); free(C); free(d); free(D);
}

/* ------------------------------------------------------------------ */
/* cdft[N]: decomposition D_c (eqs. qft_15-21) into two RDFTs.          */
/* eq. qft_19A is used with the sign of Re R2 corrected to "+" (from    */
/* X = R1 + i R2); eq. qft_20 is its mirror.                            */
/* ------------------------------------------------------------------ */
static void cdft(ctx_t *c, long N, const REAL *xr, const REAL *xi, REAL *Xr, REAL *Xi)
{
    if (N == 1) { Xr[0] = xr[0]; Xi[0] = xi[0]; return; }
    if (N == 2) { /* direct definition */
        Xr[0] = add(c, xr[0], xr[1]); Xi[0] = add(c, xi[0], xi[1]);
        Xr[1] = sub(c, xr[0], xr[1]); Xi[1] = sub(c, xi[0], xi[1]);
        return;
    }
    REAL *R1r = alloc(N / 2 + 1), *R1i = alloc(N / 2 + 1);
    REAL *R2r = alloc(N / 2 + 1), *R2i = alloc(N / 2 + 1);
    rdft(c, N, xr, R1r, R1i); /* s_1_re_tt = Re x, eq. qft_15 */
    rdft(c, N, xi, R2r, R2i); /* s_2_re_tt = Im x, eq. qft_16 */
    for (long k = 1; k < N / 2; k++) {
        Xr[k]     = sub(c, R1r[k], R2i[k]);   /* eq. qft_17  */
        Xr[N - k] = add(c, R1r[k], R2i[k]);   /* eq. qft_18  */
        Xi[k]     = add(c, R1i[k], R2r[k]);   /* eq. qft_19A (sign fixed) */
        Xi[N - k] = sub(c, R2r[k], R1i[k]);   /* eq. qft_20  */
    }
    Xr[0] = R1r[0];         Xi[0] = R2r[0];          /* eqs. qft_19, qft_21 */
    Xr[N / 2] = R1r[N / 2]; Xi[N / 2] = R2r[N / 2];
    free(R1r); free(R1i); free(R2r); free(R2i);
}

/* ================================================================== */
/* exported entry points                                                */
/* ================================================================== */
static int is_pow2(long n) { return n >= 1 && (n & (n - 1)) == 0; }

/* kinds for oracle_sub */
enum { K_DCT = 0, K_DST, K_DCT_OT, K_DST_OT, K_DCT_TO, K_DST_TO, K_DCT_OO, K_DST_OO };

/* CDFT of a batch: x and X are (batch, n) arrays of real and imaginary parts. */
int oracle_cdft(long n, long batch, int variant, const REAL *xr, const REAL *xi,
                REAL *Xr, REAL *Xi, oracle_counts *cnt, unsigned char *touched)
{
    if (!is_pow2(n) || variant < 1 || variant > 8 || batch < 0) return -1;
#ifdef ORACLE_FIXED
    if (variant % 2 == 0) return -2; /* unbounded constants: no Q2.29 form */
#endif
    ctx_t c = {variant, n, cnt, touched};
    for (long b = 0; b < batch; b++)
        cdft(&c, n, xr + b * n, xi + b * n, Xr + b * n, Xi + b * n);
    return 0;
}

/* RDFT: r is (n,), Rr/Ri receive k = 0..n/2 */
int oracle_rdft(long n, int variant, const REAL *r, REAL *Rr, REAL *Ri,
                oracle_counts *cnt, unsigned char *touched)
{
    if (!is_pow2(n) || variant < 1 || variant > 8) return -1;
#ifdef ORACLE_FIXED
    if (variant % 2 == 0) return -2;
#endif
    ctx_t c = {variant, n, cnt, touched};
    rdft(&c, n, r, Rr, Ri);
    return 0;
}

/* One recursive function on full-index arrays of length L/2+1.
 * ntop is the periodization whose constant table indexes are recorded. */
int oracle_sub(int kind, long L, long ntop, int variant, const REAL *s, REAL *S,
               oracle_counts *cnt, unsigned char *touched)
{
    if (!is_pow2(L) || variant < 1 || variant > 8 || ntop < L) return -1;
#ifdef ORACLE_FIXED
    if (variant % 2 == 0) return -2;
#endif
    ctx_t c = {variant, ntop, cnt, touched};
    switch (kind) {
    case K_DCT: if (L < 2) return -1; dct(&c, L, s, S); break;
    case K_DST: if (L < 4) return -1; dst(&c, L, s, S); break;
    case K_DCT_OT: if (L < 4) return -1; dct_ot(&c, L, s, S); break;
    case K_DST_OT: if (L < 4) return -1; dst_ot(&c, L, s, S); break;
    case K_DCT_TO: if (L < 4) return -1; dct_to(&c, L, s, S); break;
    case K_DST_TO: if (L < 4) return -1; dst_to(&c, L, s, S); break;
    case K_DCT_OO: if (L < 8) return -1; dct_oo(&c, L, s, S); break;
    case K_DST_OO: if (L < 8) return -1; dst_oo(&c, L, s, S); break;
    default: return -1;
    }
    return 0;
}

#ifndef ORACLE_FIXED
/* ------------------------------------------------------------------ */
/* Direct definitions (O(N^2)), evaluated in long double with the       */
/* product n*k reduced modulo the periodization before the trig call.   */
/* ------------------------------------------------------------------ */
#define TWO_PI_L 6.283185307179586476925286766559005768L

/* X(k) = sum_n x(n) exp(sign * i * 2 pi n k / N), eq. qft_0A (sign = -1) */
int oracle_dft_direct(long n, long batch, int sign, const REAL *xr, const REAL *xi,
                      REAL *Xr, REAL *Xi)
{
    if (n < 1 || batch < 0 || (sign != 1 && sign != -1)) return -1;
    for (long b = 0; b < batch; b++) {
        const REAL *ar = xr + b * n, *ai = xi + b * n;
        for (long k = 0; k < n; k++) {
            long double sr = 0, si = 0;
            for (long m = 0; m < n; m++) {
                long r = (long)(((__int128)m * k) % n);
                long double a = TWO_PI_L * (long double)r / (long double)n;
                long double cs = cosl(a), sn = sign * sinl(a);
                sr += (long double)ar[m] * cs - (long double)ai[m] * sn;
                si += (long double)ar[m] * sn + (long double)ai[m] * cs;
            }
            Xr[b * n + k] = (REAL)sr;
            Xi[b * n + k] = (REAL)si;
        }
    }
    return 0;
}

/* DCT-0 / DST-0 of a pruned signal (eqs. qft_0B, qft_0C), full-index
 * arrays of length L/2+1; mask_n / mask_k select sto_n / sto_k. */
int oracle_dcst_direct(int is_sine, long L, const REAL *s, const unsigned char *mask_n,
                       const unsigned char *mask_k, REAL *S)
{
    if (!is_pow2(L) || L < 2) return -1;
    for (long k = 0; k <= L / 2; k++) {
        if (!mask_k[k]) continue;
        long double acc = 0;
        for (long n = 0; n <= L / 2; n++) {
            if (!mask_n[n]) continue;
            long r = (long)(((__int128)n * k) % L);
            long double a = TWO_PI_L * (long double)r / (long double)L;
            acc += (long double)s[n] * (is_sine ? sinl(a) : cosl(a));
        }
        S[k] = (REAL)acc;
    }
    return 0;
}

#endif /* !ORACLE_FIXED */

/* size of REAL, so the loader can check which build it has */
int oracle_real_size(void) { return (int)sizeof(REAL); }

#ifdef ORACLE_FIXED
int oracle_is_fixed(void) { return 1; }
/* wrapped results since the last call (and reset) */
long long oracle_fixed_wraps(void) { long long w = g_wraps; g_wraps = 0; return w; }
/* the scalar rules, for the pins */
int oracle_fixed_mul(int a, int k) { ctx_t c = {1, 4, NULL, NULL}; return mul(&c, a, k); }
int oracle_fixed_half(int a) { ctx_t c = {1, 4, NULL, NULL}; return half(&c, a); }
int oracle_fixed_konst(int fam, long j, long L) { ctx_t c = {1, L, NULL, NULL}; return konst(&c, fam, j, L); }
int oracle_fixed_base_const(void) { ctx_t c = {1, 8, NULL, NULL}; return base_const(&c); }
#else
int oracle_is_fixed(void) { return 0; }
#endif
