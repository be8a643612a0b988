/*
 * rrs_oracle.c -- plain FP64 CPU oracle for Refined Random Search (RRS)
 * projection-based depths (Leone, Mozharovskyi, Bounie, "Massive
 * parallelization of projection-based depths", arXiv 2506.08262).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant generator with the GPU library;
 * both sides implement the same written recipe independently.
 *
 * Build: gcc -O3 -march=x86-64-v3 -ffp-contract=off -fopenmp -shared -fPIC
 * (no -ffast-math).
 * Every multiply-add that is meant to be fused is written as fma(); all other
 * arithmetic is single IEEE-754 binary64 operations in the order written.
 *
 * What each function follows in the paper:
 *   - philox4x64_10 ....... counter-based generator of Salmon et al. (SC'11);
 *                           the paper only asks for random directions, the
 *                           generator choice is this project's.
 *   - o_gauss_pair ........ N(0,1) variates for Alg. S1 (Box-Muller).
 *   - o_direction ......... Alg. S1 (randomSphere) for the first refinement,
 *                           Alg. S4 (randomSpherePole) for later ones.
 *   - o_area_cap_angle .... the polar angle of a point uniform in area on a
 *                           spherical cap (the cap law the main text states;
 *                           Alg. S4 draws the angle uniformly instead).
 *   - o_project ........... Alg. 2 (ProjParallel) inner loop, on the centred
 *                           point x - z.
 *   - o_uni_halfspace ..... Sec. 2, halfspace depth D_H.
 *   - o_uni_projection .... Sec. 2, projection depth D_P (median / MAD).
 *   - o_uni_apd ........... Sec. 2, asymmetric projection depth D_AP.
 *   - o_rrs_query ......... Alg. 1 (classical RRS) with the parallel
 *                           formulation of Alg. 4 / Alg. S5 and the
 *                           sequential tie rule of Alg. S3.
 *   - o_rrs_replay ........ Alg. 1 steps 3-5 along a given trajectory: the
 *                           exact univariate depths of each refinement's
 *                           directions when the poles follow another
 *                           implementation's choices (test protocol for an
 *                           approximate projection arithmetic).
 *
 * Parity status: Philox words, the special functions and the univariate
 * depths are pinned by independent checks in the test suite; the RRS driver
 * is pinned by brute-force exact depth, closed forms and invariants, and its
 * refinement chain (cap schedule, first-index argmin, strict pole update,
 * initial minimum) by closed forms on symmetric point sets, exact arc minima
 * in the plane and a replay of Alg. 1 from the pinned building blocks.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11).  Multipliers and Weyl key increments are the   */
/* published 4x64 constants.                                                */
/* ------------------------------------------------------------------------ */
#define PH_M0 0xD2E7470EE14C6C93ULL
#define PH_M1 0xCA5A826395121157ULL
#define PH_W0 0x9E3779B97F4A7C15ULL
#define PH_W1 0xBB67AE8584CAA73BULL

void o_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {            /* key schedule: bump before rounds 2..10 */
            k0 += PH_W0;
            k1 += PH_W1;
        }
        unsigned __int128 p0 = (unsigned __int128)PH_M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)PH_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Word k of the stream of direction (q, l, j): block k/4 of the counter
 * (k/4, j, l, q) under key (seed, 0), lane k%4. */
static uint64_t o_word(uint64_t seed, uint64_t q, uint64_t l, uint64_t j, uint64_t k)
{
    uint64_t ctr[4] = {k >> 2, j, l, q};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    o_philox4x64_10(ctr, key, out);
    return out[k & 3];
}

/* Uniform on the open interval (0,1): (2*(w>>12)+1) * 2^-53, exact. */
double o_uniform(uint64_t w)
{
    return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

/* ------------------------------------------------------------------------ */
/* Special functions written from their series (no libm transcendentals).   */
/* ------------------------------------------------------------------------ */
#define O_LN2       0x1.62e42fefa39efp-1   /* ln 2 rounded to binary64    */
#define O_SQRT_HALF 0x1.6a09e667f3bcdp-1   /* sqrt(1/2) rounded           */
#define O_PIO2      0x1.921fb54442d18p+0   /* pi/2 rounded                */

/* Natural log of x > 0: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
 * ln m = 2 atanh(s), s = (m-1)/(m+1), odd series through s^23. */
double o_log(double x)
{
    int e;
    double m = frexp(x, &e);            /* m in [0.5, 1) */
    if (m < O_SQRT_HALF) {
        m = m * 2.0;
        e = e - 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double s2 = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, s2, 1.0 / 21.0);
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    double at = fma(s * s2, p, s);      /* atanh(s) = s + s^3 (1/3 + s^2/5 + ...) */
    return fma((double)e, O_LN2, 2.0 * at);
}

/* sin and cos of (pi/2) f for f in [0,1]: reduce to g = min(f, 1-f) <= 1/2,
 * x = g * pi/2 <= pi/4, Taylor series through x^17 (sin) and x^16 (cos). */
void o_sincos_halfpi(double f, double *sn, double *cs)
{
    int swap = f > 0.5;
    double g = swap ? 1.0 - f : f;
    double x = g * O_PIO2;
    double z = x * x;
    double ps = 1.0 / 355687428096000.0;           /* +1/17! */
    ps = fma(ps, z, -1.0 / 1307674368000.0);       /* -1/15! */
    ps = fma(ps, z, 1.0 / 6227020800.0);           /* +1/13! */
    ps = fma(ps, z, -1.0 / 39916800.0);            /* -1/11! */
    ps = fma(ps, z, 1.0 / 362880.0);               /* +1/9!  */
    ps = fma(ps, z, -1.0 / 5040.0);                /* -1/7!  */
    ps = fma(ps, z, 1.0 / 120.0);                  /* +1/5!  */
    ps = fma(ps, z, -1.0 / 6.0);                   /* -1/3!  */
    double s = fma(x * z, ps, x);
    double pc = 1.0 / 20922789888000.0;            /* +1/16! */
    pc = fma(pc, z, -1.0 / 87178291200.0);         /* -1/14! */
    pc = fma(pc, z, 1.0 / 479001600.0);            /* +1/12! */
    pc = fma(pc, z, -1.0 / 3628800.0);             /* -1/10! */
    pc = fma(pc, z, 1.0 / 40320.0);                /* +1/8!  */
    pc = fma(pc, z, -1.0 / 720.0);                 /* -1/6!  */
    pc = fma(pc, z, 1.0 / 24.0);                   /* +1/4!  */
    pc = fma(pc, z, -1.0 / 2.0);                   /* -1/2!  */
    double c = fma(z, pc, 1.0);
    if (swap) { *sn = c; *cs = s; }
    else      { *sn = s; *cs = c; }
}

/* Box-Muller: two independent N(0,1) from two open uniforms.
 * R = sqrt(-2 ln u1), angle 2 pi u2 split into quadrant and (pi/2) f. */
void o_gauss_pair(double u1, double u2, double *g1, double *g2)
{
    double r = sqrt(-2.0 * o_log(u1));
    double v = 4.0 * u2;                /* exact */
    double qd = floor(v);
    double f = v - qd;                  /* exact, in [0,1) */
    double s, c;
    o_sincos_halfpi(f, &s, &c);
    double ct, st;
    int quad = (int)qd;
    if (quad == 0)      { ct = c;  st = s;  }
    else if (quad == 1) { ct = -s; st = c;  }
    else if (quad == 2) { ct = -c; st = -s; }
    else                { ct = s;  st = -c; }
    *g1 = r * ct;
    *g2 = r * st;
}

/* k Gaussians from words base, base+1, ... of the stream (pairs). */
static void o_gaussians(uint64_t seed, uint64_t q, uint64_t l, uint64_t j,
                        uint64_t base, int64_t k, double *g)
{
    for (int64_t i = 0; i < k; i += 2) {
        double u1 = o_uniform(o_word(seed, q, l, j, base + (uint64_t)i));
        double u2 = o_uniform(o_word(seed, q, l, j, base + (uint64_t)i + 1));
        double a, b;
        o_gauss_pair(u1, u2, &a, &b);
        g[i] = a;
        if (i + 1 < k) g[i + 1] = b;
    }
}

/*
 * Area-uniform polar angle in a cap (the RRS_FLAG_AREA_CAP reading of "uniform
 * on the cap"): on S^(d-1) the polar angle theta of a point uniform on the cap
 * {angle <= eps} has density proportional to sin(theta)^(d-2).  With
 * x = sin(theta) and the binomial series 1 / sqrt(1 - s^2) = sum_k c_k s^(2k),
 * c_0 = 1, c_(k+1) = c_k (2k+1) / (2k+2), the mass below theta is
 * J(x) = int_0^x s^(d-2) / sqrt(1 - s^2) ds = x^(d-1) T(x),
 * T(x) = sum_k c_k x^(2k) / (d - 1 + 2k).  Inverting J(x) = u J(x_e),
 * x_e = sin(eps), by Newton's method in y = x / x_e from y = 1 (the function
 * y^(d-1) T(x_e y) is increasing and convex, so the iterates decrease to the
 * root), gives sin(theta) = x_e y and cos(theta) = sqrt((1 - x)(1 + x)).
 * The series stops at the first term at most 2^-60 of the running sum (and
 * after 200000 terms; accurate to about 1e-10 for eps <= 0.99 pi/2).
 */
static void o_cap_series(double x, int64_t n1, double *T, double *R)
{
    double x2 = x * x, c = 1.0, p = 1.0, t_sum = 0.0, r_sum = 0.0;
    for (int64_t k = 0; k < 200000; ++k) {
        double t = (c * p) / (double)(n1 + 2 * k);
        t_sum = t_sum + t;
        r_sum = r_sum + (double)(2 * k) * t;   /* R = x T'(x) */
        if (t <= 0x1p-60 * t_sum) break;
        p = p * x2;
        c = (c * (double)(2 * k + 1)) / (double)(2 * k + 2);
    }
    *T = t_sum;
    *R = r_sum;
}

static double o_pow_int(double y, int64_t e)
{
    double r = 1.0, b = y;
    while (e > 0) {
        if (e & 1) r = r * b;
        e >>= 1;
        if (e > 0) b = b * b;
    }
    return r;
}

void o_area_cap_angle(double u, double phi, int64_t d, double *st, double *ct)
{
    int64_t n1 = d - 1;
    double xe, ce, Te, Re;
    o_sincos_halfpi(phi, &xe, &ce);
    o_cap_series(xe, n1, &Te, &Re);
    double target = u * Te, y = 1.0;
    for (int it = 0; it < 200; ++it) {
        double T, R;
        o_cap_series(xe * y, n1, &T, &R);
        double P = o_pow_int(y, n1);
        double g = P * T - target;
        double gp = (P / y) * ((double)n1 * T + R);   /* derivative in y */
        double yn = y - g / gp;
        if (!(yn < y)) break;
        y = yn;
    }
    double x = xe * y;
    *st = x;
    *ct = sqrt((1.0 - x) * (1.0 + x));
}

/*
 * Direction j of refinement l (1-based) for query q.  With first_cap, the
 * first refinement also takes the l >= 2 branch (phi = 1: angle-uniform in
 * the hemisphere around the initial pole e1), the literal reading of the
 * algorithms' initial cap of half-angle pi/2.
 *   l == 1 : Alg. S1 -- d Gaussians divided by their Euclidean norm, i.e.
 *            uniform on the whole sphere (the first refinement is a plain
 *            random search; the full sphere keeps D_AP correct because D_AP
 *            is not symmetric under u -> -u).
 *   l >= 2 : Alg. S4 -- a direction within angle (pi/2) phi of e1, where
 *            phi = alpha^(l-1):  v1 = cos(theta), v_{2..d} = sin(theta) w/|w|,
 *            theta = (pi/2) U phi, then the Householder reflection that swaps
 *            e1 and the pole p (Alg. S4's reflection step, read as
 *            u = v - beta w, w = e1 - p, beta = 2 (w.v) / (w.w)).
 * pole has d entries; u receives d entries.
 */
static void o_direction_mode(uint64_t seed, uint64_t q, uint64_t l, uint64_t j, int64_t d,
                             double phi, const double *pole, double *u, int first_cap,
                             int area_cap)
{
    if (l == 1 && !first_cap) {
        o_gaussians(seed, q, l, j, 0, d, u);
        double s = 0.0;
        for (int64_t c = 0; c < d; ++c) s = fma(u[c], u[c], s);
        double nrm = sqrt(s);
        for (int64_t c = 0; c < d; ++c) u[c] = u[c] / nrm;
        return;
    }
    double *v = (double *)malloc(sizeof(double) * (size_t)d);
    double st, ct;
    if (area_cap) {
        o_area_cap_angle(o_uniform(o_word(seed, q, l, j, 0)), phi, d, &st, &ct);
    } else {
        double f = o_uniform(o_word(seed, q, l, j, 0)) * phi;
        o_sincos_halfpi(f, &st, &ct);
    }
    o_gaussians(seed, q, l, j, 1, d - 1, v + 1);
    double s = 0.0;
    for (int64_t c = 1; c < d; ++c) s = fma(v[c], v[c], s);
    double nrm = sqrt(s);
    v[0] = ct;
    for (int64_t c = 1; c < d; ++c) v[c] = st * (v[c] / nrm);

    double a = 1.0 - pole[0];           /* w = e1 - p : w0 = a, wc = -p_c */
    double ww = a * a;
    for (int64_t c = 1; c < d; ++c) ww = fma(pole[c], pole[c], ww);
    if (ww == 0.0) {                    /* p == e1 : identity */
        memcpy(u, v, sizeof(double) * (size_t)d);
        free(v);
        return;
    }
    double wv = a * v[0];
    for (int64_t c = 1; c < d; ++c) wv = fma(-pole[c], v[c], wv);
    double beta = (2.0 * wv) / ww;
    u[0] = fma(-beta, a, v[0]);
    for (int64_t c = 1; c < d; ++c) u[c] = fma(beta, pole[c], v[c]);
    free(v);
}

/* Either first-refinement reading (exported for the pin tests). */
void o_direction_ex(uint64_t seed, uint64_t q, uint64_t l, uint64_t j, int64_t d, double phi,
                    const double *pole, double *u, int first_cap, int area_cap)
{
    o_direction_mode(seed, q, l, j, d, phi, pole, u, first_cap, area_cap);
}

/* The generator of the depth calls: refinement 1 on the whole sphere. */
void o_direction(uint64_t seed, uint64_t q, uint64_t l, uint64_t j, int64_t d,
                 double phi, const double *pole, double *u)
{
    o_direction_mode(seed, q, l, j, d, phi, pole, u, 0, 0);
}

/* Alg. 2 inner loop on the centred point: t = sum_c (x_c - z_c) u_c,
 * accumulated by fused multiply-add in coordinate order c = 0..d-1. */
void o_project(const double *X, int64_t n, int64_t d, const double *z,
               const double *u, double *t)
{
    for (int64_t i = 0; i < n; ++i) {
        const double *x = X + i * d;
        double a = 0.0;
        for (int64_t c = 0; c < d; ++c) a = fma(x[c] - z[c], u[c], a);
        t[i] = a;
    }
}

/* ------------------------------------------------------------------------ */
/* Univariate depths of y = z.u among y_i = x_i.u, written on t_i = y_i - y. */
/* ------------------------------------------------------------------------ */

/* Sec. 2, halfspace depth: min(#{y_i <= y}, #{y_i >= y}); returns the count,
 * the depth is count / n. */
int64_t o_uni_halfspace(const double *t, int64_t n)
{
    int64_t le = 0, ge = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (t[i] <= 0.0) ++le;
        if (t[i] >= 0.0) ++ge;
    }
    return le < ge ? le : ge;
}

static int o_cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

/* The usual median: middle order statistic, or the mean (a+b)*0.5 of the two
 * middle ones for even counts.  Sorts v in place. */
double o_median_inplace(double *v, int64_t n)
{
    qsort(v, (size_t)n, sizeof(double), o_cmp_double);
    if (n & 1) return v[n / 2];
    return (v[n / 2 - 1] + v[n / 2]) * 0.5;
}

/* Sec. 2, projection depth: 1 / (1 + |y - med| / MAD), MAD = med |y_i - med|.
 * On t: |y - med(y)| = |med(t)|.  MAD == 0 (not covered by the paper):
 * depth 1 if med == 0, else 0.  Outputs med and MAD when non-NULL. */
double o_uni_projection(const double *t, int64_t n, double *med_out, double *mad_out)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(w, t, sizeof(double) * (size_t)n);
    double med = o_median_inplace(w, n);
    for (int64_t i = 0; i < n; ++i) w[i] = fabs(t[i] - med);
    double mad = o_median_inplace(w, n);
    free(w);
    if (med_out) *med_out = med;
    if (mad_out) *mad_out = mad;
    if (mad == 0.0) return (med == 0.0) ? 1.0 : 0.0;
    return 1.0 / (1.0 + fabs(med) / mad);
}

/* Sec. 2, asymmetric projection depth: 1 / (1 + (y - med)_+ / MAD_+), where
 * MAD_+ is the median of the strictly positive deviations y_i - med.
 * On t: (y - med(y))_+ = max(-med(t), 0) and y_i - med(y) = t_i - med(t).
 * Empty positive set (not covered by the paper): depth 1 if the numerator is
 * 0, else 0. */
double o_uni_apd(const double *t, int64_t n, double *med_out, double *madp_out)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(w, t, sizeof(double) * (size_t)n);
    double med = o_median_inplace(w, n);
    int64_t np = 0;
    for (int64_t i = 0; i < n; ++i) {
        double dv = t[i] - med;
        if (dv > 0.0) w[np++] = dv;
    }
    double num = (med < 0.0) ? -med : 0.0;
    double madp = (np > 0) ? o_median_inplace(w, np) : 0.0;
    free(w);
    if (med_out) *med_out = med;
    if (madp_out) *madp_out = madp;
    if (np == 0) return (num == 0.0) ? 1.0 : 0.0;
    return 1.0 / (1.0 + num / madp);
}

/* ------------------------------------------------------------------------ */
/* RRS driver for one query.                                                */
/* ------------------------------------------------------------------------ */
enum { O_HALFSPACE = 0, O_PROJECTION = 1, O_APD = 2 };

/*
 * Alg. 1 / Alg. 4 / Alg. S5 for query index q (the query's position in the
 * caller's batch, which keys its random stream).  Per refinement l = 1..r:
 * generate m = ceil(K/r) directions, project, take the univariate depth of
 * each, find the first index attaining the minimum (Alg. S3 scans directions
 * in order with a strict '<'), and move the pole there only if that minimum
 * is strictly below the running minimum.  The cap scale phi starts at 1 and
 * is multiplied by alpha after every refinement (epsilon = (pi/2) phi).
 *
 * Halfspace depth compares integer counts; the depth is count / n.
 * Outputs: depth; count (halfspace only, may be NULL); pole_out (d, may be
 * NULL) = final pole; trace (may be NULL) = per refinement
 * {j*, improved, value-of-min as double bits}.
 */
static void o_rrs_query_mode(int notion, const double *X, int64_t n, int64_t d,
                             const double *z, uint64_t q, int64_t K, int32_t r, double alpha,
                             uint64_t seed, double *depth, int64_t *count, double *pole_out,
                             int64_t *trace, int first_cap, int area_cap)
{
    int64_t m = (K + r - 1) / r;
    double *pole = (double *)calloc((size_t)d, sizeof(double));
    double *U = (double *)malloc(sizeof(double) * (size_t)(m * d));
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    pole[0] = 1.0;
    double dmin = 1.0;
    int64_t cmin = n;
    double phi = 1.0;
    for (int32_t l = 1; l <= r; ++l) {
        int64_t jbest = -1;
        double vbest = 0.0;
        int64_t cbest = 0;
        for (int64_t j = 0; j < m; ++j) {
            double *u = U + j * d;
            o_direction_mode(seed, q, (uint64_t)l, (uint64_t)j, d, phi, pole, u, first_cap,
                             area_cap);
            o_project(X, n, d, z, u, t);
            if (notion == O_HALFSPACE) {
                int64_t c = o_uni_halfspace(t, n);
                if (jbest < 0 || c < cbest) { jbest = j; cbest = c; }
            } else {
                double v = (notion == O_PROJECTION) ? o_uni_projection(t, n, NULL, NULL)
                                                    : o_uni_apd(t, n, NULL, NULL);
                if (jbest < 0 || v < vbest) { jbest = j; vbest = v; }
            }
        }
        int improved;
        if (notion == O_HALFSPACE) {
            improved = cbest < cmin;
            if (improved) cmin = cbest;
            vbest = (double)cbest;
        } else {
            improved = vbest < dmin;
            if (improved) dmin = vbest;
        }
        if (improved) memcpy(pole, U + jbest * d, sizeof(double) * (size_t)d);
        if (trace) {
            trace[3 * (l - 1) + 0] = jbest;
            trace[3 * (l - 1) + 1] = improved;
            memcpy(&trace[3 * (l - 1) + 2], &vbest, sizeof(double));
        }
        phi = phi * alpha;
    }
    if (notion == O_HALFSPACE) {
        dmin = (double)cmin / (double)n;
        if (count) *count = cmin;
    }
    *depth = dmin;
    if (pole_out) memcpy(pole_out, pole, sizeof(double) * (size_t)d);
    free(pole);
    free(U);
    free(t);
}

void o_rrs_query(int notion, const double *X, int64_t n, int64_t d,
                 const double *z, uint64_t q, int64_t K, int32_t r, double alpha,
                 uint64_t seed, double *depth, int64_t *count, double *pole_out,
                 int64_t *trace)
{
    o_rrs_query_mode(notion, X, n, d, z, q, K, r, alpha, seed, depth, count, pole_out, trace, 0,
                     0);
}

/* Replay of one query along a trajectory chosen elsewhere (Alg. 1 steps 3-5
 * with someone else's step-4 decisions): refinement l generates its
 * directions around the pole the trajectory has reached (e1 at l = 1, then
 * u_{j*} of every refinement the trajectory marks improved), computes the
 * exact univariate depth of every direction and reports
 *   out[3 (l-1) + 0] = the smallest depth over the directions (exact minimum),
 *   out[3 (l-1) + 1] = the depth of the direction the trajectory chose,
 *   out[3 (l-1) + 2] = the first index attaining the minimum (as a double).
 * traj[3 (l-1) + 0] = chosen index j*, traj[3 (l-1) + 1] = improved (0/1).
 * Halfspace depths are reported as counts / n. */
void o_rrs_replay(int notion, const double *X, int64_t n, int64_t d, const double *z,
                  uint64_t q, int64_t K, int32_t r, double alpha, uint64_t seed,
                  const int64_t *traj, double *out)
{
    int64_t m = (K + r - 1) / r;
    double *pole = (double *)calloc((size_t)d, sizeof(double));
    double *U = (double *)malloc(sizeof(double) * (size_t)(m * d));
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    double *v = (double *)malloc(sizeof(double) * (size_t)m);
    pole[0] = 1.0;
    double phi = 1.0;
    for (int32_t l = 1; l <= r; ++l) {
        int64_t jmin = 0;
        for (int64_t j = 0; j < m; ++j) {
            double *u = U + j * d;
            o_direction(seed, q, (uint64_t)l, (uint64_t)j, d, phi, pole, u);
            o_project(X, n, d, z, u, t);
            if (notion == O_HALFSPACE)
                v[j] = (double)o_uni_halfspace(t, n) / (double)n;
            else if (notion == O_PROJECTION)
                v[j] = o_uni_projection(t, n, NULL, NULL);
            else
                v[j] = o_uni_apd(t, n, NULL, NULL);
            if (v[j] < v[jmin]) jmin = j;
        }
        const int64_t jg = traj[3 * (l - 1) + 0];
        out[3 * (l - 1) + 0] = v[jmin];
        out[3 * (l - 1) + 1] = (jg >= 0 && jg < m) ? v[jg] : NAN;
        out[3 * (l - 1) + 2] = (double)jmin;
        if (traj[3 * (l - 1) + 1] && jg >= 0 && jg < m)
            memcpy(pole, U + jg * d, sizeof(double) * (size_t)d);
        phi = phi * alpha;
    }
    free(pole);
    free(U);
    free(t);
    free(v);
}

/* All queries; queries are independent, spread over nthreads OpenMP threads
 * (nthreads <= 0: the runtime default).  Query i uses stream index q0 + i. */
void o_rrs_depth(int notion, const double *X, int64_t n, int64_t d,
                 const double *Z, int64_t nq, uint64_t q0, int64_t K, int32_t r,
                 double alpha, uint64_t seed, double *depth, int64_t *count,
                 double *poles, int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nq; ++i) {
        o_rrs_query(notion, X, n, d, Z + i * d, q0 + (uint64_t)i, K, r, alpha, seed,
                    &depth[i], count ? &count[i] : NULL,
                    poles ? poles + i * d : NULL, NULL);
    }
}

int32_t o_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Queries with explicit stream indices qidx[i] (row i of Z), in parallel;
 * first_cap selects the first-refinement cap reading (see o_direction_mode). */
void o_rrs_depth_idx_mode(int notion, const double *X, int64_t n, int64_t d,
                          const double *Z, int64_t nq, const uint64_t *qidx, int64_t K,
                          int32_t r, double alpha, uint64_t seed, double *depth,
                          int64_t *count, double *poles, int32_t nthreads, int first_cap,
                          int area_cap)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nq; ++i) {
        o_rrs_query_mode(notion, X, n, d, Z + i * d, qidx[i], K, r, alpha, seed,
                         &depth[i], count ? &count[i] : NULL,
                         poles ? poles + i * d : NULL, NULL, first_cap, area_cap);
    }
}

/* Queries with explicit stream indices qidx[i] (row i of Z), in parallel. */
void o_rrs_depth_idx(int notion, const double *X, int64_t n, int64_t d,
                     const double *Z, int64_t nq, const uint64_t *qidx, int64_t K,
                     int32_t r, double alpha, uint64_t seed, double *depth,
                     int64_t *count, double *poles, int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nq; ++i) {
        o_rrs_query(notion, X, n, d, Z + i * d, qidx[i], K, r, alpha, seed,
                    &depth[i], count ? &count[i] : NULL,
                    poles ? poles + i * d : NULL, NULL);
    }
}
