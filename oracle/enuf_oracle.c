/*
 * enuf_oracle.c -- plain, slow FP64 CPU oracle for ENUF-DPD electrostatics.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may load, link or
 * call this library: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or constant
 * generator with the HIP implementation.
 *
 * What it computes (Wang, Laaksonen & Lu, "Implementation of non-uniform FFT
 * based Ewald summation in Dissipative Particle Dynamics"):
 *
 *  * The Ewald split of the periodic Coulomb energy (Sec. 3.1, eq. 16) with
 *    the reciprocal sum truncated to the sphere 0 < |k| < Kc of integer
 *    wave vectors and evaluated DIRECTLY, i.e. without any NFFT (eq. 18-19 for
 *    the energy, eq. 22-24 for the force).  The NFFT only approximates this
 *    sum, so the direct sum is the exact target of the GPU path.
 *  * The real-space pair term q_i q_j erfc(alpha r)/r over minimum-image pairs
 *    with r < r_cut (eq. 31) and its exact negative gradient (the printed
 *    force expression, eq. 32, drops factors; the gradient is used instead).
 *  * The Slater charge-smearing correction (Sec. 4, eq. 27-28) in its
 *    additive reading: for the same pairs the point-charge 1/r is replaced by
 *    B1(r)/r, i.e. the pair energy gains -q_i q_j (1 + r/lambda) e^{-2r/lambda}/r.
 *  * The self term -(alpha/sqrt(pi)) sum q_j^2 (eq. 16).
 *  * One step of the modified velocity-Verlet DPD integrator (Table 2,
 *    steps 0-6) with conservative, dissipative and random pair forces
 *    (eq. 2-7), harmonic bonds (Sec. 2) and the electrostatic force above.
 *  * Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) for the random
 *    variable theta_ij of the random force (Philox4x64-10 is kept as well).
 *
 * Units: the Coulomb prefactor 1/(4 pi eps0 epsr) is 1; a driver scales
 * energies and forces by its coupling constant.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2
#define OR_ECOINCIDENT -7

/* ------------------------------------------------------------------ */
/* helpers                                                              */
/* ------------------------------------------------------------------ */

/* Periodic wrap into [0, L). */
static double wrap_coord(double x, double L)
{
    double y = x - L * floor(x / L);
    if (y >= L) y = 0.0;
    if (y < 0.0) y = 0.0;
    return y;
}

/* Minimum-image separation vector d = r_i - r_j. */
static void min_image(const double *ri, const double *rj, double L, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        double v = ri[a] - rj[a];
        v -= L * nearbyint(v / L);
        d[a] = v;
    }
}

/* ------------------------------------------------------------------ */
/* Real space: Ewald erfc term (eq. 31) + Slater correction (eq. 27)    */
/* ------------------------------------------------------------------ */

/*
 * Pair energy and force factor for one pair at distance r (r < r_cut), per
 * unit q_i q_j:
 *   e_short : erfc(alpha r)/r - (1 + r/lambda) e^{-2r/lambda}/r
 *             (the Slater term is absent when lambda == 0),
 *   e_slat  : the Slater term alone (diagnostic; not defined at r = 0),
 *   f       : force on i is q_i q_j * f * d, d = r_i - r_j, i.e.
 *             f = -(1/r) d/dr e_short.
 *
 * With lambda > 0, e_short = [B1(r) - erf(alpha r)]/r and
 * f = B2(r)/r^3 - [erf(alpha r)/r^3 - (2 alpha/sqrt(pi)) e^{-alpha^2 r^2}/r^2]
 * (B1, B2 of eq. 27-28).  The closed forms of both brackets cancel
 * catastrophically as r -> 0, so for x = r/lambda < 1/2 the oracle sums
 * their convergent, all-positive series instead:
 *   B1 = e^{-2x} [x + sum_{n>=2} (2x)^n/n!],  B2 = e^{-2x} sum_{n>=3} (2x)^n/n!
 *     (1 - e^{-y} sum_{n<m} y^n/n! = e^{-y} sum_{n>=m} y^n/n!, y = 2x),
 *   erf(z) = (2/sqrt(pi)) e^{-z^2} sum_{n>=0} 2^n z^{2n+1}/(2n+1)!!
 *     (Abramowitz & Stegun 7.1.6).
 * At r = 0 the pair contributes 1/lambda - 2 alpha/sqrt(pi) and no force.
 */
static int pair_terms(double r, double alpha, double lambda,
                      double *e_short, double *e_slat, double *f)
{
    const double two_over_sqrtpi = 2.0 / sqrt(M_PI);
    if (lambda > 0.0 && r < 0.5 * lambda) {
        double x = r / lambda, y = 2.0 * x, z = alpha * r, z2 = z * z;
        /* b1 = B1 e^{2x}/x = 1 + sum_{n>=2} 2^n x^{n-1}/n!,
         * b2 = B2 e^{2x}/x^3 = sum_{n>=3} 2^n x^{n-3}/n!  (no division by x) */
        double b2 = 8.0 / 6.0, term = b2, b1 = 1.0 + 2.0 * x + b2 * x * x;
        for (int n = 4; n < 40; ++n) {
            term *= y / n;                       /* 2^n x^{n-3}/n! */
            b2 += term;
            b1 += term * x * x;
        }
        /* g0 = sum_{n>=0} 2^n z^{2n}/(2n+1)!!,  g1 = sum_{n>=1} 2^n z^{2n-2}/(2n+1)!! */
        double t = 1.0, g0 = 1.0, g1 = 0.0;
        for (int n = 1; n < 40; ++n) {
            t *= 2.0 * z2 / (2.0 * n + 1.0);     /* 2^n z^{2n}/(2n+1)!! */
            g0 += t;
        }
        t = 2.0 / 3.0;                           /* n = 1 term of g1: 2 / 3!! */
        for (int n = 1; n < 40; ++n) {
            g1 += t;
            t *= 2.0 * z2 / (2.0 * n + 3.0);
        }
        double ex = exp(-y), ez = exp(-z2);
        double u = ex * b1 / lambda - two_over_sqrtpi * alpha * ez * g0;
        double l3 = lambda * lambda * lambda;
        double fr = ex * b2 / l3 - two_over_sqrtpi * alpha * alpha * alpha * ez * g1;
        *e_short = u;
        *e_slat = (r > 0.0) ? -(1.0 + x) * ex / r : 0.0;
        *f = (r > 0.0) ? fr : 0.0;   /* d = 0: the force vanishes */
        return OR_OK;
    }
    if (r == 0.0) return OR_ECOINCIDENT;
    double r2 = r * r;
    double ar = alpha * r;
    double erfc_ar = erfc(ar);
    double ee = erfc_ar / r;
    /* -dU/dr / r for U = erfc(alpha r)/r */
    double fr = (erfc_ar / r + two_over_sqrtpi * alpha * exp(-ar * ar)) / r2;
    double es = 0.0;
    if (lambda > 0.0) {
        double x = r / lambda;
        double ex = exp(-2.0 * x);
        es = -(1.0 + x) * ex / r;
        /* -dU/dr / r for U = -(1 + x) e^{-2x}/r  is  -(1 + 2x + 2x^2) e^{-2x}/r^3 */
        fr += -(1.0 + 2.0 * x + 2.0 * x * x) * ex / (r2 * r);
    }
    *e_short = ee + es;
    *e_slat = es;
    *f = fr;
    return OR_OK;
}

/*
 * Real-space energy and forces over all charged pairs with minimum-image
 * distance r < r_cut.
 *   sel == NULL: forces for every particle (zeros for neutral ones) and the
 *                energies E[0] = whole short-range sum (erfc term plus Slater
 *                correction, summed per pair so that close pairs keep their
 *                accuracy) and E[1] = the Slater correction alone, which is
 *                already contained in E[0].
 *   sel != NULL: forces only for the nsel listed particles (row k of F
 *                belongs to particle sel[k]); energies are not computed
 *                (E[0] = E[1] = NaN).
 */
int oracle_real(int64_t n, const double *pos, const double *q, double L,
                double alpha, double r_cut, double lambda,
                int64_t nsel, const int64_t *sel, double *F, double *E)
{
    if (n < 0 || !(L > 0.0) || !(alpha > 0.0) || !(r_cut > 0.0) || lambda < 0.0)
        return OR_EINVAL;
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!w) return OR_ENOMEM;
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) w[3 * i + a] = wrap_coord(pos[3 * i + a], L);

    int64_t nout = sel ? nsel : n;
    double *Ei = (double *)calloc((size_t)(nout > 0 ? nout : 1), 2 * sizeof(double));
    if (!Ei) { free(w); return OR_ENOMEM; }
    int status = OR_OK;
    const double rc2 = r_cut * r_cut;

#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nout; ++k) {
        int64_t i = sel ? sel[k] : k;
        double fx = 0.0, fy = 0.0, fz = 0.0, ee = 0.0, es = 0.0;
        if (q[i] != 0.0) {
            for (int64_t j = 0; j < n; ++j) {
                if (j == i || q[j] == 0.0) continue;
                double d[3];
                min_image(&w[3 * i], &w[3 * j], L, d);
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (!(r2 < rc2)) continue;
                double r = sqrt(r2), e1, e2, f;
                if (pair_terms(r, alpha, lambda, &e1, &e2, &f) != OR_OK) {
#pragma omp atomic write
                    status = OR_ECOINCIDENT;
                    continue;
                }
                double qq = q[i] * q[j];
                fx += qq * f * d[0];
                fy += qq * f * d[1];
                fz += qq * f * d[2];
                if (j > i) { ee += qq * e1; es += qq * e2; }
            }
        }
        F[3 * k + 0] = fx;
        F[3 * k + 1] = fy;
        F[3 * k + 2] = fz;
        Ei[2 * k + 0] = ee;
        Ei[2 * k + 1] = es;
    }
    if (sel) {
        E[0] = NAN;
        E[1] = NAN;
    } else {
        double s0 = 0.0, s1 = 0.0;
        for (int64_t k = 0; k < nout; ++k) { s0 += Ei[2 * k]; s1 += Ei[2 * k + 1]; }
        E[0] = s0;
        E[1] = s1;
    }
    free(Ei);
    free(w);
    return status;
}

/* ------------------------------------------------------------------ */
/* Reciprocal space: direct sum over 0 < |k| < Kc (eq. 18-24)           */
/* ------------------------------------------------------------------ */

typedef struct { double re, im; } cplx;

/* Integer wave vectors k != 0 with |k|^2 < Kc^2, in lexicographic order. */
static int64_t build_kvectors(int Kc, int **kv_out)
{
    int K1 = Kc - 1;
    int64_t cnt = 0;
    for (int a = -K1; a <= K1; ++a)
        for (int b = -K1; b <= K1; ++b)
            for (int c = -K1; c <= K1; ++c) {
                int k2 = a * a + b * b + c * c;
                if (k2 > 0 && k2 < Kc * Kc) ++cnt;
            }
    int *kv = (int *)malloc(sizeof(int) * 3 * (size_t)(cnt > 0 ? cnt : 1));
    if (!kv) return -1;
    int64_t m = 0;
    for (int a = -K1; a <= K1; ++a)
        for (int b = -K1; b <= K1; ++b)
            for (int c = -K1; c <= K1; ++c) {
                int k2 = a * a + b * b + c * c;
                if (k2 > 0 && k2 < Kc * Kc) {
                    kv[3 * m] = a; kv[3 * m + 1] = b; kv[3 * m + 2] = c;
                    ++m;
                }
            }
    *kv_out = kv;
    return cnt;
}

/* Per-axis phase factors e^{-2 pi i k x / L} for k = -K1..K1 (index k + K1). */
static void phase_rows(const double *r, double L, int K1, cplx *rows /* 3*(2K1+1) */)
{
    int nk = 2 * K1 + 1;
    for (int a = 0; a < 3; ++a)
        for (int k = -K1; k <= K1; ++k) {
            double th = 2.0 * M_PI * (double)k * r[a] / L;
            rows[a * nk + (k + K1)].re = cos(th);
            rows[a * nk + (k + K1)].im = -sin(th);
        }
}

/*
 * Direct reciprocal sum.  S(k) = sum_j q_j e^{-2 pi i k . r_j / L} over ALL
 * charged particles; E = (1/(2 pi L)) sum_k W(k) |S(k)|^2 with
 * W(k) = exp(-pi^2 |k|^2/(alpha L)^2)/|k|^2;
 * F_i = (2 q_i / L^2) sum_k W(k) k Im( e^{+2 pi i k . r_i / L} S(k) ).
 * sel/nsel as for oracle_real; E is always computed (it needs only S).
 * The particle loop for S is split into fixed blocks whose partial sums are
 * added in block order, so the result does not depend on the thread count.
 */
int oracle_recip(int64_t n, const double *pos, const double *q, double L,
                 double alpha, int Kc, int64_t nsel, const int64_t *sel,
                 double *F, double *E)
{
    if (n < 0 || !(L > 0.0) || !(alpha > 0.0) || Kc < 1) return OR_EINVAL;
    int *kv = NULL;
    int64_t nk = build_kvectors(Kc, &kv);
    if (nk < 0) return OR_ENOMEM;
    int K1 = Kc - 1, nrow = 2 * K1 + 1;
    double *Wk = (double *)malloc(sizeof(double) * (size_t)(nk > 0 ? nk : 1));
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!Wk || !w) { free(kv); free(Wk); free(w); return OR_ENOMEM; }
    const double aL = alpha * L;
    for (int64_t m = 0; m < nk; ++m) {
        double k2 = (double)(kv[3 * m] * kv[3 * m] + kv[3 * m + 1] * kv[3 * m + 1]
                             + kv[3 * m + 2] * kv[3 * m + 2]);
        Wk[m] = exp(-M_PI * M_PI * k2 / (aL * aL)) / k2;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) w[3 * i + a] = wrap_coord(pos[3 * i + a], L);

    /* fixed particle blocks (independent of the thread count) */
    int64_t bs = 512;
    if (n / 64 + 1 > bs) bs = n / 64 + 1;
    int64_t nb = (n + bs - 1) / bs;
    if (nb < 1) nb = 1;
    cplx *Sb = (cplx *)calloc((size_t)nb * (size_t)(nk > 0 ? nk : 1), sizeof(cplx));
    cplx *S = (cplx *)calloc((size_t)(nk > 0 ? nk : 1), sizeof(cplx));
    if (!Sb || !S) { free(kv); free(Wk); free(w); free(Sb); free(S); return OR_ENOMEM; }

#pragma omp parallel
    {
        cplx *rows = (cplx *)malloc(sizeof(cplx) * 3 * (size_t)nrow);
#pragma omp for schedule(static)
        for (int64_t b = 0; b < nb; ++b) {
            cplx *Sp = Sb + (size_t)b * (size_t)nk;
            int64_t j1 = (b + 1) * bs < n ? (b + 1) * bs : n;
            for (int64_t j = b * bs; j < j1; ++j) {
                if (q[j] == 0.0) continue;
                phase_rows(&w[3 * j], L, K1, rows);
                for (int64_t m = 0; m < nk; ++m) {
                    cplx ex = rows[kv[3 * m] + K1];
                    cplx ey = rows[nrow + kv[3 * m + 1] + K1];
                    cplx ez = rows[2 * nrow + kv[3 * m + 2] + K1];
                    double xyr = ex.re * ey.re - ex.im * ey.im;
                    double xyi = ex.re * ey.im + ex.im * ey.re;
                    double re = xyr * ez.re - xyi * ez.im;
                    double im = xyr * ez.im + xyi * ez.re;
                    Sp[m].re += q[j] * re;
                    Sp[m].im += q[j] * im;
                }
            }
        }
        free(rows);
    }
    for (int64_t b = 0; b < nb; ++b)
        for (int64_t m = 0; m < nk; ++m) {
            S[m].re += Sb[(size_t)b * nk + m].re;
            S[m].im += Sb[(size_t)b * nk + m].im;
        }
    free(Sb);

    double e = 0.0;
    for (int64_t m = 0; m < nk; ++m) e += Wk[m] * (S[m].re * S[m].re + S[m].im * S[m].im);
    *E = e / (2.0 * M_PI * L);

    int64_t nout = sel ? nsel : n;
#pragma omp parallel
    {
        cplx *rows = (cplx *)malloc(sizeof(cplx) * 3 * (size_t)nrow);
#pragma omp for schedule(static)
        for (int64_t k = 0; k < nout; ++k) {
            int64_t i = sel ? sel[k] : k;
            double fx = 0.0, fy = 0.0, fz = 0.0;
            if (q[i] != 0.0) {
                phase_rows(&w[3 * i], L, K1, rows);
                for (int64_t m = 0; m < nk; ++m) {
                    cplx ex = rows[kv[3 * m] + K1];
                    cplx ey = rows[nrow + kv[3 * m + 1] + K1];
                    cplx ez = rows[2 * nrow + kv[3 * m + 2] + K1];
                    double xyr = ex.re * ey.re - ex.im * ey.im;
                    double xyi = ex.re * ey.im + ex.im * ey.re;
                    double er = xyr * ez.re - xyi * ez.im;   /* e^{-i theta_i} */
                    double ei = xyr * ez.im + xyi * ez.re;
                    /* Im( conj(e) * S ) = er*S.im - (-ei)*S.re ... with conj(e) = er - i ei */
                    double imv = er * S[m].im - ei * S[m].re;
                    double c = Wk[m] * imv;
                    fx += c * kv[3 * m];
                    fy += c * kv[3 * m + 1];
                    fz += c * kv[3 * m + 2];
                }
            }
            double s = 2.0 * q[i] / (L * L);
            F[3 * k + 0] = s * fx;
            F[3 * k + 1] = s * fy;
            F[3 * k + 2] = s * fz;
        }
        free(rows);
    }
    free(S);
    free(kv);
    free(Wk);
    free(w);
    return OR_OK;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int oracle_num_threads(void) { return omp_get_max_threads(); }

/* Threads of the parallel loops that the calling host thread starts from now
 * on (n >= 1; timing of the oracle on one core or on all of them). */
void oracle_set_threads(int n) { if (n >= 1) omp_set_num_threads(n); }

/* Self term of eq. 16: -(alpha/sqrt(pi)) sum_j q_j^2. */
double oracle_self(int64_t n, const double *q, double alpha)
{
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += q[j] * q[j];
    return -alpha / sqrt(M_PI) * s;
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11)                                 */
/* ------------------------------------------------------------------ */

static inline uint64_t mulhilo64(uint64_t a, uint64_t b, uint64_t *hi)
{
    __uint128_t p = (__uint128_t)a * (__uint128_t)b;
    *hi = (uint64_t)(p >> 64);
    return (uint64_t)p;
}

void oracle_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, hi1;
        uint64_t lo0 = mulhilo64(M0, c0, &hi0);
        uint64_t lo1 = mulhilo64(M1, c2, &hi1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Philox4x32-10 (same paper): 32-bit words, multipliers 0xD2511F53 and
 * 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85. */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * theta_ij for the random force: zero mean, unit variance (eq. 5 text),
 * uniform on [-sqrt(3), sqrt(3)).  Philox4x32-10 with counter
 * (min(i,j), max(i,j), low and high word of the step) and key (low and high
 * word of the seed); 53 random bits from the first two output words.
 */
double oracle_theta(uint64_t seed, uint64_t step, int64_t i, int64_t j)
{
    uint32_t lo = (uint32_t)(i < j ? i : j), hi = (uint32_t)(i < j ? j : i);
    uint32_t ctr[4] = {lo, hi, (uint32_t)step, (uint32_t)(step >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    uint64_t bits = ((uint64_t)out[0] << 21) | (uint64_t)(out[1] >> 11);
    double u = (double)bits * (1.0 / 9007199254740992.0);
    return sqrt(3.0) * (2.0 * u - 1.0);
}

/* ------------------------------------------------------------------ */
/* DPD (Sec. 2, eq. 2-7; Table 2)                                       */
/* ------------------------------------------------------------------ */

typedef struct {
    double L;          /* box edge */
    double a;          /* conservative amplitude a_ij (one species) */
    double gamma;      /* dissipation strength */
    double sigma;      /* noise amplitude, sigma^2 = 2 gamma kT */
    double dt;         /* time step */
    double lam;        /* velocity-prediction parameter of the modified VV */
    double k_bond;     /* harmonic spring constant */
    double r0_bond;    /* bond rest length */
    double kappa;      /* electrostatic coupling (Coulomb prefactor) */
    double alpha;      /* Ewald parameters ... */
    double r_cut;
    double lambda_e;
    int Kc;
    int use_elec;      /* 0: no electrostatics */
    int nspec;         /* species (0 or 1: every pair uses a) */
    const int *species;/* [n] species of each particle, in [0, nspec) (nspec > 1) */
    double atab[16];   /* a_ij = atab[4 s_i + s_j], symmetric, nspec <= 4 (Sec. 2) */
} oracle_dpd_params;

/*
 * Total force on every particle at positions pos and (predicted) velocities
 * vel: DPD conservative + dissipative + random (R_c = 1, m = 1), harmonic
 * bonds, and kappa times the Ewald electrostatic force.  The random force is
 * returned divided by sqrt(dt), so that a velocity update v += f dt applies
 * sigma w^R theta rhat sqrt(dt) as in Table 2.  bonds holds nb index pairs.
 * E_elec (may be NULL) receives kappa * (real + Slater + recip + self).
 */
int oracle_dpd_forces(int64_t n, const double *pos, const double *vel, const double *q,
                      int64_t nb, const int64_t *bonds, const oracle_dpd_params *P,
                      uint64_t seed, uint64_t step, double *F, double *E_elec)
{
    if (n < 1 || !P || !(P->L > 0.0) || !(P->dt > 0.0)) return OR_EINVAL;
    const int typed = P->nspec > 1;
    if (typed) {
        if (P->nspec > 4 || !P->species) return OR_EINVAL;
        for (int64_t i = 0; i < n; ++i)
            if (P->species[i] < 0 || P->species[i] >= P->nspec) return OR_EINVAL;
    }
    const double L = P->L, isdt = 1.0 / sqrt(P->dt);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(&pos[3 * i], &pos[3 * j], L, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < 1.0) || r2 == 0.0) continue;
            double r = sqrt(r2);
            double e[3] = {d[0] / r, d[1] / r, d[2] / r};
            double wr = 1.0 - r;
            double vdot = (vel[3 * i] - vel[3 * j]) * e[0] + (vel[3 * i + 1] - vel[3 * j + 1]) * e[1]
                          + (vel[3 * i + 2] - vel[3 * j + 2]) * e[2];
            double th = oracle_theta(seed, step, i, j);
            /* eq. 3: the conservative amplitude of the pair's two species */
            double aij = typed ? P->atab[4 * P->species[i] + P->species[j]] : P->a;
            double mag = aij * wr - P->gamma * wr * wr * vdot + P->sigma * wr * th * isdt;
            fx += mag * e[0];
            fy += mag * e[1];
            fz += mag * e[2];
        }
        F[3 * i] = fx;
        F[3 * i + 1] = fy;
        F[3 * i + 2] = fz;
    }
    /* harmonic bonds: F_i = -K (r - r0) rhat_ij, F_j = -F_i (serial, fixed order) */
    for (int64_t b = 0; b < nb; ++b) {
        int64_t i = bonds[2 * b], j = bonds[2 * b + 1];
        if (i < 0 || j < 0 || i >= n || j >= n || i == j) return OR_EINVAL;
        double d[3];
        min_image(&pos[3 * i], &pos[3 * j], L, d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r == 0.0) continue;
        double mag = -P->k_bond * (r - P->r0_bond) / r;
        for (int a = 0; a < 3; ++a) {
            F[3 * i + a] += mag * d[a];
            F[3 * j + a] -= mag * d[a];
        }
    }
    if (E_elec) *E_elec = 0.0;
    if (P->use_elec) {
        double *Fr = (double *)malloc(sizeof(double) * 3 * (size_t)n);
        double *Fk = (double *)malloc(sizeof(double) * 3 * (size_t)n);
        if (!Fr || !Fk) { free(Fr); free(Fk); return OR_ENOMEM; }
        double Er[2], Ek;
        int st = oracle_real(n, pos, q, L, P->alpha, P->r_cut, P->lambda_e, 0, NULL, Fr, Er);
        if (st == OR_OK) st = oracle_recip(n, pos, q, L, P->alpha, P->Kc, 0, NULL, Fk, &Ek);
        if (st != OR_OK) { free(Fr); free(Fk); return st; }
        for (int64_t i = 0; i < 3 * n; ++i) F[i] += P->kappa * (Fr[i] + Fk[i]);
        if (E_elec) *E_elec = P->kappa * (Er[0] + Ek + oracle_self(n, q, P->alpha));
        free(Fr);
        free(Fk);
    }
    return OR_OK;
}

/*
 * One modified velocity-Verlet step (Table 2), in place:
 *   (0) v0 = v + lam dt f        (predicted velocity, f = force of the last step)
 *   (1) v  = v + dt f / 2
 *   (2) r  = r + dt v, wrapped into [0, L)
 *   (3)-(5) f = forces(r, v0) with the random numbers of step `step`
 *   (6) v  = v + dt f / 2
 * On entry F holds the forces of the previous step; on exit the new ones.
 */
int oracle_dpd_step(int64_t n, double *pos, double *vel, double *F, const double *q,
                    int64_t nb, const int64_t *bonds, const oracle_dpd_params *P,
                    uint64_t seed, uint64_t step, double *E_elec)
{
    if (n < 1 || !P) return OR_EINVAL;
    const double dt = P->dt;
    double *v0 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!v0) return OR_ENOMEM;
    for (int64_t i = 0; i < 3 * n; ++i) {
        v0[i] = vel[i] + P->lam * dt * F[i];
        vel[i] = vel[i] + 0.5 * dt * F[i];
        pos[i] = wrap_coord(pos[i] + dt * vel[i], P->L);
    }
    int st = oracle_dpd_forces(n, pos, v0, q, nb, bonds, P, seed, step, F, E_elec);
    if (st == OR_OK)
        for (int64_t i = 0; i < 3 * n; ++i) vel[i] += 0.5 * dt * F[i];
    free(v0);
    return st;
}

/* ------------------------------------------------------------------ */
/* Structure observables (Sec. 5: radial distribution functions;        */
/* Sec. 6: radius of gyration of a chain)                               */
/* ------------------------------------------------------------------ */

/*
 * Pair-distance histogram by class.  Every unordered pair {sel[a], sel[b]},
 * a < b, of the nsel selected particles is counted once, at the minimum-image
 * distance r, into hist[(c_lo * ncls + c_hi) * nbins + k] (c_lo <= c_hi the
 * pair's classes) for the bin k with (k w)^2 <= r^2 < ((k + 1) w)^2,
 * w = r_max / nbins; pairs beyond the last edge are not counted.  hist is
 * accumulated (not cleared).  The bin is decided on r^2 against the squared
 * edges (k w)(k w), so it does not depend on how a square root rounds.
 */
int oracle_pair_histogram(int64_t n, const double *pos, int64_t nsel, const int64_t *sel,
                          const int *cls, int ncls, double L, double r_max, int nbins,
                          uint64_t *hist)
{
    if (n < 0 || nsel < 0 || ncls < 1 || nbins < 1 || !(L > 0.0) || !(r_max > 0.0)) return OR_EINVAL;
    for (int64_t a = 0; a < nsel; ++a)
        if (sel[a] < 0 || sel[a] >= n || cls[a] < 0 || cls[a] >= ncls) return OR_EINVAL;
    const double w = r_max / nbins;
    double *edge = (double *)malloc(sizeof(double) * (size_t)(nbins + 1));
    if (!edge) return OR_ENOMEM;
    for (int k = 0; k <= nbins; ++k) {
        double e = (double)k * w;
        edge[k] = e * e;
    }
    for (int64_t a = 0; a < nsel; ++a) {
        for (int64_t b = a + 1; b < nsel; ++b) {
            double d[3];
            min_image(&pos[3 * sel[b]], &pos[3 * sel[a]], L, d);
            double r2 = d[0] * d[0] + d[1] * d[1];
            r2 = r2 + d[2] * d[2];
            if (!(r2 < edge[nbins])) continue;
            int k = (int)(sqrt(r2) / w);
            if (k > nbins - 1) k = nbins - 1;
            while (k > 0 && edge[k] > r2) --k;
            while (k < nbins - 1 && edge[k + 1] <= r2) ++k;
            int lo = cls[a] < cls[b] ? cls[a] : cls[b];
            int hi = cls[a] < cls[b] ? cls[b] : cls[a];
            hist[((size_t)lo * ncls + hi) * nbins + k] += 1;
        }
    }
    free(edge);
    return OR_OK;
}

/*
 * Squared radius of gyration of nchains chains of len beads each; chain c is
 * beads[c * len .. c * len + len - 1] in bond order.  The chain is unwrapped
 * by following the minimum image from each bead to the next (bonds shorter
 * than L / 2), then Rg^2 = (1/len) sum_k |u_k - u_cm|^2 with u_cm the mean of
 * the unwrapped beads.  out[c] receives Rg^2.
 */
int oracle_chain_rg2(int64_t n, const double *pos, int nchains, int len, const int64_t *beads,
                     double L, double *out)
{
    if (nchains < 0 || len < 1 || !(L > 0.0)) return OR_EINVAL;
    double *u = (double *)malloc(sizeof(double) * 3 * (size_t)len);
    if (!u) return OR_ENOMEM;
    for (int c = 0; c < nchains; ++c) {
        const int64_t *bd = beads + (size_t)c * len;
        for (int k = 0; k < len; ++k)
            if (bd[k] < 0 || bd[k] >= n) { free(u); return OR_EINVAL; }
        for (int a = 0; a < 3; ++a) u[a] = pos[3 * bd[0] + a];
        for (int k = 1; k < len; ++k) {
            double d[3];
            min_image(&pos[3 * bd[k]], &pos[3 * bd[k - 1]], L, d);
            for (int a = 0; a < 3; ++a) u[3 * k + a] = u[3 * (k - 1) + a] + d[a];
        }
        double cm[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < len; ++k)
            for (int a = 0; a < 3; ++a) cm[a] += u[3 * k + a];
        for (int a = 0; a < 3; ++a) cm[a] /= len;
        double s = 0.0;
        for (int k = 0; k < len; ++k)
            for (int a = 0; a < 3; ++a) {
                double v = u[3 * k + a] - cm[a];
                s += v * v;
            }
        out[c] = s / len;
    }
    free(u);
    return OR_OK;
}
