/*
 * sht_oracle.c -- TEST INFRASTRUCTURE ONLY (the CPU oracle).
 *
 * Plain, slow, CPU reference for the harmonic part of full-sky Taylor
 * lensing: for one colatitude theta it returns the per-m Fourier
 * coefficients of the theta-derivatives of a band-limited spin-0 field and
 * of the spin-2 field Q+iU,
 *
 *     F^{(j)}_m(theta) = sum_l a_lm d^j/dtheta^j lambda_lm(theta),
 *
 * for j = 0..nderiv and m = 0..lmax.  These are the "derivatives computed
 * from the harmonic coefficients" that the pixel-relative Taylor expansion
 * (eq. 4 and eq. 5 of the paper, Sec. II.B) needs at every pixel centre.
 * The paper obtained them with repeated healpy SHTs; here they come from the
 * definition: the normalized associated Legendre recursion in l, with every
 * recursion step differentiated by Leibniz' rule, and the spin-2 functions
 * from the three-term recursion of the Wigner d-functions.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this library.  It shares no code with the GPU library.
 *
 * Precision: all arithmetic is x87 80-bit long double (64-bit mantissa,
 * 15-bit exponent).  The wide exponent means that sin^m(theta) for m up to
 * several thousand does not underflow, so no rescaling logic is needed; the
 * results are rounded to double on output.
 *
 * Conventions
 *   lambda_lm(theta): orthonormal, Condon-Shortley phase, so that
 *     Y_lm = lambda_lm(theta) e^{i m phi} (equal to scipy's sph_harm_y).
 *   spin-s functions: sY_lm = sqrt((l-s)!/(l+s)!) eth^s Y_lm with
 *     eth f = -(sin t)^s (d_t + i csc t d_phi)(sin t)^{-s} f  (and the
 *     conjugate operator for negative s); sY_lm = s_lambda_lm(t) e^{i m phi}.
 *     In Wigner-d form s_lambda_lm(t) is proportional to d^l_{m,-s}(t), and
 *     it obeys, for fixed (m, s) and L >= l_min + 1 with l_min = max(|m|,|s|),
 *       lam_L = a_L (cos t + b_L) lam_{L-1} - c_L lam_{L-2},
 *       R_L = sqrt((L^2-m^2)(L^2-s^2)),
 *       a_L = sqrt((2L+1)(2L-1)) L / R_L,    b_L = m s / (L (L-1)),
 *       c_L = sqrt((2L+1)/(2L-3)) L R_{L-1} / ((L-1) R_L)   (c = 0 at l_min+1).
 *     For s = 0 this is the usual normalized Legendre recursion.
 *   E/B: Q+iU = sum 2a_lm 2Y_lm with 2a_lm = -(E_lm + i B_lm) and
 *     Q-iU = sum -2a_lm -2Y_lm with -2a_lm = -(E_lm - i B_lm).
 *     Per m >= 0 the Fourier coefficients of the real maps Q and U are
 *       Q_m = (P_m + M_m)/2,  U_m = (P_m - M_m)/(2i),
 *       P_m = -sum_l (E_lm + i B_lm) 2lambda_lm,
 *       M_m = -sum_l (E_lm - i B_lm) (-2)lambda_lm.
 *     Coefficients with l < 2 are ignored for E and B.
 *
 * a_lm layout: complex128 interleaved, index m*(2*lmax+1-m)/2 + l (m >= 0).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;

#define OR_MAXD 24 /* largest derivative order supported */

static const ld PI_L = 3.141592653589793238462643383279502884L;

static size_t idx_lm(int lmax, int l, int m)
{
    return (size_t)m * (size_t)(2 * lmax + 1 - m) / 2 + (size_t)l;
}

static ld binom_l(int n, int k)
{
    ld r = 1.0L;
    for (int i = 1; i <= k; ++i) r = r * (ld)(n - k + i) / (ld)i;
    return r;
}

/* d^i/dt^i cos(t) = cos(t + i pi/2), d^i/dt^i sin(t) = sin(t + i pi/2);
 * for argument k t the i-th derivative carries k^i. */
static ld cos_deriv(ld c, ld s, int i)
{
    switch (i & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
    }
}
static ld sin_deriv(ld c, ld s, int i)
{
    switch (i & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
    }
}

/* Start values lam^{(j)}_{l_min, m}(t) for spin s in {0, +2, -2}.
 *
 * s = 0: lambda_00 = 1/sqrt(4 pi); lambda_mm = -sqrt((2m+1)/(2m)) sin t
 *   lambda_{m-1,m-1}; derivatives of each step by Leibniz.
 * s = +-2, m >= 2: s_lambda_mm = (-1)^m sqrt((2m+1)/4pi)
 *   sqrt((2m)!/((m+s)!(m-s)!)) cos^{m-s}(t/2) sin^{m+s}(t/2), generated as
 *   s_lambda_22 = sqrt(5/4pi) g^2 with g = sin^2(t/2) (s=+2) or cos^2(t/2)
 *   (s=-2), and s_lambda_mm = -sqrt((2m+1) m / (2 (m^2 - s^2))) sin t
 *   s_lambda_{m-1,m-1}.
 * s = +-2, m in {0,1}: l_min = 2, closed forms
 *   m=0: sqrt(5/4pi) sqrt(6)/4 sin^2 t                 (both signs)
 *   m=1: -sqrt(5/4pi) sin t sin^2(t/2)  (s=+2),  +sqrt(5/4pi) sin t cos^2(t/2)  (s=-2).
 * Every start value is a product of sin t, sin^2(t/2), cos^2(t/2), so its
 * derivatives follow by Leibniz' rule from those of the factors without
 * cancellation near the poles (sin^2(t/2) = (1 - cos t)/2 is evaluated
 * directly, its derivatives are -cos^{(j)}(t)/2).
 * All three follow from the eth definition applied to lambda_2m / lambda_mm
 * (checked against it in the tests).
 *
 * table: [m][j], m = 0..lmax, j = 0..J.  Built by an m-recursion per theta.
 */
static void start_table(int lmax, int J, int s, ld t, ld *table)
{
    const ld c = cosl(t), sn = sinl(t);
    const ld k5 = sqrtl(5.0L / (4.0L * PI_L));
    ld sd[OR_MAXD + 1];
    for (int i = 0; i <= J; ++i) sd[i] = sin_deriv(c, sn, i);

    memset(table, 0, sizeof(ld) * (size_t)(lmax + 1) * (size_t)(J + 1));
    if (s == 0) {
        ld prev[OR_MAXD + 1], cur[OR_MAXD + 1];
        for (int j = 0; j <= J; ++j) prev[j] = 0.0L;
        prev[0] = 1.0L / sqrtl(4.0L * PI_L);
        for (int j = 0; j <= J; ++j) table[j] = prev[j];
        for (int m = 1; m <= lmax; ++m) {
            ld f = -sqrtl((ld)(2 * m + 1) / (ld)(2 * m));
            for (int j = 0; j <= J; ++j) {
                ld acc = 0.0L;
                for (int i = 0; i <= j; ++i)
                    acc += binom_l(j, i) * sd[i] * prev[j - i];
                cur[j] = f * acc;
            }
            for (int j = 0; j <= J; ++j) {
                prev[j] = cur[j];
                table[(size_t)m * (J + 1) + j] = cur[j];
            }
        }
        return;
    }
    /* spin +-2 */
    if (lmax < 2) return;
    const ld sh = sinl(0.5L * t), ch = cosl(0.5L * t);
    ld st[OR_MAXD + 1], g[OR_MAXD + 1];
    for (int i = 0; i <= J; ++i) {
        st[i] = sd[i];
        if (i == 0) g[i] = (s > 0) ? sh * sh : ch * ch;
        else g[i] = ((s > 0) ? -0.5L : 0.5L) * cos_deriv(c, sn, i);
    }
    /* m = 0, l_min = 2 : k5 sqrt(6)/4 (sin t)^2 */
    for (int j = 0; j <= J; ++j) {
        ld acc = 0.0L;
        for (int i = 0; i <= j; ++i) acc += binom_l(j, i) * st[i] * st[j - i];
        table[0 * (J + 1) + j] = k5 * sqrtl(6.0L) * 0.25L * acc;
    }
    /* m = 1, l_min = 2 : -+ k5 sin t g */
    for (int j = 0; j <= J; ++j) {
        ld acc = 0.0L;
        for (int i = 0; i <= j; ++i) acc += binom_l(j, i) * st[i] * g[j - i];
        table[1 * (J + 1) + j] = ((s > 0) ? -k5 : k5) * acc;
    }
    /* m = 2 : k5 g^2 */
    ld prev[OR_MAXD + 1], cur[OR_MAXD + 1];
    for (int j = 0; j <= J; ++j) {
        ld acc = 0.0L;
        for (int i = 0; i <= j; ++i) acc += binom_l(j, i) * g[i] * g[j - i];
        prev[j] = k5 * acc;
        table[2 * (J + 1) + j] = prev[j];
    }
    for (int m = 3; m <= lmax; ++m) {
        ld f = -sqrtl((ld)(2 * m + 1) * (ld)m / (2.0L * (ld)(m * m - 4)));
        for (int j = 0; j <= J; ++j) {
            ld acc = 0.0L;
            for (int i = 0; i <= j; ++i)
                acc += binom_l(j, i) * sd[i] * prev[j - i];
            cur[j] = f * acc;
        }
        for (int j = 0; j <= J; ++j) {
            prev[j] = cur[j];
            table[(size_t)m * (J + 1) + j] = cur[j];
        }
    }
}

/* Recursion coefficients of the spin-s three-term recursion (header). */
static void rec_coeffs(int L, int m, int s, int lmin, ld *a, ld *b, ld *cc)
{
    ld RL = sqrtl((ld)((long long)L * L - (long long)m * m) * (ld)((long long)L * L - (long long)s * s));
    *a = sqrtl((ld)(2 * L + 1) * (ld)(2 * L - 1)) * (ld)L / RL;
    *b = (m * s == 0) ? 0.0L : (ld)(m * s) / ((ld)L * (ld)(L - 1));
    if (L == lmin + 1) {
        *cc = 0.0L;
    } else {
        int K = L - 1;
        ld RK = sqrtl((ld)((long long)K * K - (long long)m * m) * (ld)((long long)K * K - (long long)s * s));
        *cc = sqrtl((ld)(2 * L + 1) / (ld)(2 * L - 3)) * (ld)L * RK / ((ld)(L - 1) * RL);
    }
}

/* For one (theta, m): run the recursion of spin s over l = l_min..lmax with
 * j = 0..J derivatives and accumulate sum_l coef_l * lam^{(j)}_l for up to
 * two complex coefficient arrays (cA, cB may be NULL).  Results in
 * outA/outB[j][2] (re, im), long double. */
static void accumulate_m(int lmax, int J, int s, int m, ld t,
                         const ld *start_row, const double *cA, const double *cB,
                         ld (*outA)[2], ld (*outB)[2])
{
    const int abs_s = s < 0 ? -s : s;
    const int lmin = m > abs_s ? m : abs_s;
    const ld c = cosl(t), sn = sinl(t);
    ld cd[OR_MAXD + 1];
    for (int i = 0; i <= J; ++i) cd[i] = cos_deriv(c, sn, i);
    ld w[OR_MAXD + 1][OR_MAXD + 1];
    for (int j = 0; j <= J; ++j)
        for (int i = 0; i <= j; ++i) w[j][i] = binom_l(j, i) * cd[i];

    ld p2[OR_MAXD + 1], p1[OR_MAXD + 1], cur[OR_MAXD + 1];
    for (int j = 0; j <= J; ++j) {
        outA[j][0] = outA[j][1] = 0.0L;
        if (outB) outB[j][0] = outB[j][1] = 0.0L;
        p2[j] = 0.0L;
        p1[j] = start_row[j];
    }
    if (lmin > lmax) return;
    for (int l = lmin; l <= lmax; ++l) {
        if (l > lmin) {
            ld a, b, cc;
            rec_coeffs(l, m, s, lmin, &a, &b, &cc);
            for (int j = 0; j <= J; ++j) {
                /* d^j[(cos t + b) p1] = b p1^{(j)} + sum_i C(j,i) cos^{(i)} p1^{(j-i)} */
                ld acc = b * p1[j];
                for (int i = 0; i <= j; ++i) acc += w[j][i] * p1[j - i];
                cur[j] = a * acc - cc * p2[j];
            }
            for (int j = 0; j <= J; ++j) {
                p2[j] = p1[j];
                p1[j] = cur[j];
            }
        }
        size_t k = idx_lm(lmax, l, m);
        if (cA) {
            ld re = cA[2 * k], im = cA[2 * k + 1];
            for (int j = 0; j <= J; ++j) {
                outA[j][0] += re * p1[j];
                outA[j][1] += im * p1[j];
            }
        }
        if (cB && outB) {
            ld re = cB[2 * k], im = cB[2 * k + 1];
            for (int j = 0; j <= J; ++j) {
                outB[j][0] += re * p1[j];
                outB[j][1] += im * p1[j];
            }
        }
    }
}

/*
 * oracle_synth_rings: per-ring Fourier coefficients of theta-derivatives.
 *
 *   lmax, nderiv (J), nring, theta[nring]
 *   alm_T / alm_E / alm_B: complex128 interleaved (may be NULL; E NULL means
 *     no polarization; B NULL means B = 0)
 *   outT / outQ / outU: double [nring][J+1][lmax+1][2] (skipped when NULL)
 *   nthreads: OpenMP threads (<= 0: library default)
 *
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_synth_rings(int lmax, int nderiv, int nring, const double *theta,
                       const double *alm_T, const double *alm_E, const double *alm_B,
                       double *outT, double *outQ, double *outU, int nthreads)
{
    if (lmax < 0 || nderiv < 0 || nderiv > OR_MAXD || nring < 0 || !theta) return -1;
    const int J = nderiv;
    const int pol = (alm_E != NULL) && outQ && outU;
    const int doT = (alm_T != NULL) && outT;
    const size_t tab = (size_t)(lmax + 1) * (J + 1);
    ld *t0 = (ld *)calloc((size_t)nring * tab, sizeof(ld));
    ld *tp = pol ? (ld *)calloc((size_t)nring * tab, sizeof(ld)) : NULL;
    ld *tm = pol ? (ld *)calloc((size_t)nring * tab, sizeof(ld)) : NULL;
    if (!t0 || (pol && (!tp || !tm))) {
        free(t0); free(tp); free(tm);
        return -1;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < nring; ++r) {
        ld t = (ld)theta[r];
        start_table(lmax, J, 0, t, t0 + (size_t)r * tab);
        if (pol) {
            start_table(lmax, J, 2, t, tp + (size_t)r * tab);
            start_table(lmax, J, -2, t, tm + (size_t)r * tab);
        }
    }

    const long long ntask = (long long)nring * (lmax + 1);
#pragma omp parallel for schedule(dynamic, 4)
    for (long long task = 0; task < ntask; ++task) {
        const int r = (int)(task / (lmax + 1));
        const int m = (int)(task % (lmax + 1));
        const ld t = (ld)theta[r];
        ld A[OR_MAXD + 1][2], B[OR_MAXD + 1][2];
        if (doT) {
            accumulate_m(lmax, J, 0, m, t, t0 + (size_t)r * tab + (size_t)m * (J + 1),
                         alm_T, NULL, A, NULL);
            for (int j = 0; j <= J; ++j) {
                size_t o = (((size_t)r * (J + 1) + j) * (lmax + 1) + m) * 2;
                outT[o] = (double)A[j][0];
                outT[o + 1] = (double)A[j][1];
            }
        }
        if (pol) {
            /* s = +2: sum E 2lam and sum B 2lam ; s = -2: same with -2lam */
            ld Ep[OR_MAXD + 1][2], Bp[OR_MAXD + 1][2], Em[OR_MAXD + 1][2], Bm[OR_MAXD + 1][2];
            accumulate_m(lmax, J, 2, m, t, tp + (size_t)r * tab + (size_t)m * (J + 1),
                         alm_E, alm_B, Ep, alm_B ? Bp : NULL);
            accumulate_m(lmax, J, -2, m, t, tm + (size_t)r * tab + (size_t)m * (J + 1),
                         alm_E, alm_B, Em, alm_B ? Bm : NULL);
            if (!alm_B)
                for (int j = 0; j <= J; ++j) Bp[j][0] = Bp[j][1] = Bm[j][0] = Bm[j][1] = 0.0L;
            for (int j = 0; j <= J; ++j) {
                /* P = -(E + iB).2lam ; M = -(E - iB).(-2)lam  (complex E, B) */
                ld Pr = -(Ep[j][0] - Bp[j][1]);
                ld Pi = -(Ep[j][1] + Bp[j][0]);
                ld Mr = -(Em[j][0] + Bm[j][1]);
                ld Mi = -(Em[j][1] - Bm[j][0]);
                /* Q = (P + M)/2 ; U = (P - M)/(2i) = -i (P - M)/2 */
                ld Qr = 0.5L * (Pr + Mr), Qi = 0.5L * (Pi + Mi);
                ld Dr = 0.5L * (Pr - Mr), Di = 0.5L * (Pi - Mi);
                ld Ur = Di, Ui = -Dr;
                size_t o = (((size_t)r * (J + 1) + j) * (lmax + 1) + m) * 2;
                outQ[o] = (double)Qr;
                outQ[o + 1] = (double)Qi;
                outU[o] = (double)Ur;
                outU[o + 1] = (double)Ui;
            }
        }
    }
    free(t0);
    free(tp);
    free(tm);
    return 0;
}

/*
 * oracle_spin_lambda: the functions themselves (for the pins), s in {0,2,-2}:
 * out[l][j] = d^j/dt^j s_lambda_lm(t) for l = 0..lmax at one (t, m).
 */
int oracle_spin_lambda(int lmax, int nderiv, int s, int m, double theta, double *out)
{
    if (lmax < 0 || nderiv < 0 || nderiv > OR_MAXD || m < 0 || m > lmax) return -1;
    if (!(s == 0 || s == 2 || s == -2)) return -1;
    const int J = nderiv;
    ld *tab = (ld *)calloc((size_t)(lmax + 1) * (J + 1), sizeof(ld));
    if (!tab) return -1;
    start_table(lmax, J, s, (ld)theta, tab);
    const int abs_s = s < 0 ? -s : s;
    const int lmin = m > abs_s ? m : abs_s;
    memset(out, 0, sizeof(double) * (size_t)(lmax + 1) * (J + 1));
    /* run the recursion and record every l (reuse accumulate_m by feeding a
     * unit coefficient at a single l would be quadratic; do it inline) */
    const ld t = (ld)theta, c = cosl(t), sn = sinl(t);
    ld cd[OR_MAXD + 1];
    for (int i = 0; i <= J; ++i) cd[i] = cos_deriv(c, sn, i);
    ld p2[OR_MAXD + 1], p1[OR_MAXD + 1], cur[OR_MAXD + 1];
    for (int j = 0; j <= J; ++j) {
        p2[j] = 0.0L;
        p1[j] = tab[(size_t)m * (J + 1) + j];
    }
    for (int l = lmin; l <= lmax; ++l) {
        if (l > lmin) {
            ld a, b, cc;
            rec_coeffs(l, m, s, lmin, &a, &b, &cc);
            for (int j = 0; j <= J; ++j) {
                ld acc = b * p1[j];
                for (int i = 0; i <= j; ++i) acc += binom_l(j, i) * cd[i] * p1[j - i];
                cur[j] = a * acc - cc * p2[j];
            }
            for (int j = 0; j <= J; ++j) {
                p2[j] = p1[j];
                p1[j] = cur[j];
            }
        }
        for (int j = 0; j <= J; ++j) out[(size_t)l * (J + 1) + j] = (double)p1[j];
    }
    free(tab);
    return 0;
}

int oracle_max_deriv(void) { return OR_MAXD; }
