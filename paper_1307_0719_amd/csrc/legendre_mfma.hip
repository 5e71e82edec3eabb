// Harmonic stage on the matrix cores: "L-power" form of the theta-derivatives.
//
// The normalized Legendre functions obey
//     lam'' = -cot t lam' + (m^2 csc^2 t - L) lam,      L = l(l+1),
// so every theta-derivative of lam, and (through the eth operator) of the
// spin-2 combinations W = (2lam + -2lam)/2 and X = (2lam - -2lam)/2, is a
// combination sum_p [alpha_p(t, m) L^p lam + beta_p(t, m) L^p lam'] whose
// coefficients do not depend on l:
//     W/N_l = -2 cot t lam' + (2 m^2 csc^2 t - L) lam,
//     X/N_l = -2 m csc t lam' + 2 m csc t cot t lam,     N_l = sqrt((l-2)!/(l+2)!),
// and d/dt maps (alpha_p, beta_p) -> (alpha_p' + m^2 csc^2 beta_p - beta_{p-1},
//                                      alpha_p + beta_p' - cot t beta_p).
// The sums over l therefore become, per m, one dense product
//     S[ring, {lam, lam'}][col] = sum_l A[ring, {lam, lam'}][l] * R[l][col],
//     R[l][.] = { L^p a^T_lm,  N_l L^p E_lm,  N_l L^p B_lm }   (re, im),
// run on MFMA (32 x 32 x 2 FP32), followed by a per-(ring, m) epilogue that
// applies the FP64 coefficients (obtained from Taylor jets of cot, csc in t)
// and forms T, Q = -(sum E W + i B X), U = i sum E X - sum B W and their
// theta-derivatives.
//
// The recursion of lam and lam' runs in FP64 registers (north/south by the
// parity of l+m), exponent-scaled as in the direct kernel.  A wave holds 32
// ring pairs; lanes r and r+32 run the same ring's recursion two l-steps apart,
// so a 32x32x2 MFMA takes its k = 0 / k = 1 operands (l and l+2, same parity)
// straight from the two half-waves.  The FP32 matrix accumulators are flushed
// into FP64 totals after every 64-l chunk: sequential FP32 accumulation over
// thousands of l would otherwise dominate the error.  Rings whose sin t is too
// small for the 1/sin t coefficients stay on the direct FP64 kernel.
#include "tl_internal.h"

namespace tl {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr double kHi = 0x1p256;
constexpr double kDown = 0x1p-512;

constexpr int KCH = 64;    // l values per LDS chunk
constexpr int NCOL = 32;   // GEMM columns (one MFMA block)
constexpr int MGRP = 8;    // consecutive m per workgroup
constexpr int WG = 256;    // 4 waves
constexpr int RPW = 32;    // ring pairs per wave
constexpr int RPB = 128;   // ring pairs per workgroup

struct Cols {
    int PT, PS, nT, nE, nB, ncol;
};
__host__ __device__ constexpr Cols cols_of(int N, bool hasb)
{
    Cols c{};
    c.PT = N / 2;
    c.PS = N / 2 + 1;
    c.nT = 2 * (c.PT + 1);
    c.nE = 2 * (c.PS + 1);
    c.nB = hasb ? 2 * (c.PS + 1) : 0;
    c.ncol = c.nT + c.nE + c.nB;
    return c;
}

// ----------------------------------------------------------- Taylor jets
// f(t + h) = sum_i f[i] h^i, truncated at order K.
template <int K>
struct Jet {
    double c[K + 1];
};

template <int K>
__device__ __forceinline__ Jet<K> jmul(const Jet<K> &a, const Jet<K> &b, int ord)
{
    Jet<K> r;
#pragma unroll
    for (int i = 0; i <= K; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k <= i; ++k) s = fma(a.c[k], b.c[i - k], s);
        r.c[i] = (i <= ord) ? s : 0.0;
    }
    return r;
}

// d/dt of a jet (order drops by one)
template <int K>
__device__ __forceinline__ Jet<K> jder(const Jet<K> &a)
{
    Jet<K> r;
#pragma unroll
    for (int i = 0; i < K; ++i) r.c[i] = (double)(i + 1) * a.c[i + 1];
    r.c[K] = 0.0;
    return r;
}

// Coefficients alpha_jp, beta_jp (j = 0..N, p = 0..P) of one family at one
// (theta, m), from the initial jets (al0, be0) by repeated application of d/dt.
template <int N, int P>
__device__ void family_coeffs(Jet<N> (&al)[P + 1], Jet<N> (&be)[P + 1], const Jet<N> &mcsc2,
                              const Jet<N> &cot, double (&ca)[N + 1][P + 1], double (&cb)[N + 1][P + 1])
{
#pragma unroll
    for (int j = 0; j <= N; ++j) {
#pragma unroll
        for (int p = 0; p <= P; ++p) {
            ca[j][p] = al[p].c[0];
            cb[j][p] = be[p].c[0];
        }
        if (j == N) break;
        const int ord = N - j - 1;
        Jet<N> nal[P + 1], nbe[P + 1];
#pragma unroll
        for (int p = 0; p <= P; ++p) {
            Jet<N> t1 = jder<N>(al[p]);
            Jet<N> t2 = jmul<N>(mcsc2, be[p], ord);
            Jet<N> t3 = jder<N>(be[p]);
            Jet<N> t4 = jmul<N>(cot, be[p], ord);
#pragma unroll
            for (int i = 0; i <= N; ++i) {
                double pm = (p > 0) ? be[p - 1].c[i] : 0.0;
                nal[p].c[i] = (i <= ord) ? t1.c[i] + t2.c[i] - pm : 0.0;
                nbe[p].c[i] = (i <= ord) ? al[p].c[i] + t3.c[i] - t4.c[i] : 0.0;
            }
        }
#pragma unroll
        for (int p = 0; p <= P; ++p) {
            al[p] = nal[p];
            be[p] = nbe[p];
        }
    }
}

// Epilogue for one (ring, m): S[type*2 + parity][col] are the FP64 column
// sums of lam (type 0) and lam' (type 1) over l+m even (parity 0) / odd (1).
// half 0 forms T, half 1 forms Q and U (north ring r and south ring rs).
template <int N, bool POL, bool HASB>
__device__ void epilogue(const double (*S)[cols_of(N, HASB).ncol], int half, int m, double th, int r, int rs,
                         int lmax, size_t plane, float2 *__restrict__ FT, float2 *__restrict__ FQ,
                         float2 *__restrict__ FU)
{
    constexpr Cols C = cols_of(N, HASB);
    constexpr int PT = C.PT, PS = C.PS;
    auto nsum = [&](int type, int c) { return S[type * 2][c] + S[type * 2 + 1][c]; };
    auto dsum = [&](int type, int c) { return S[type * 2][c] - S[type * 2 + 1][c]; };

    // Taylor jets of csc, cot at theta
    Jet<N> js, jc, csc, cot, jm2;
    {
        const double st = sin(th), ct = cos(th);
        double fac = 1.0;
#pragma unroll
        for (int i = 0; i <= N; ++i) {
            if (i > 0) fac *= (double)i;
            double sd, cd;
            switch (i & 3) {
            case 0: sd = st; cd = ct; break;
            case 1: sd = ct; cd = -st; break;
            case 2: sd = -st; cd = -ct; break;
            default: sd = -ct; cd = st; break;
            }
            js.c[i] = sd / fac;
            jc.c[i] = cd / fac;
        }
        csc.c[0] = 1.0 / js.c[0];
#pragma unroll
        for (int i = 1; i <= N; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = 1; k <= i; ++k) s = fma(js.c[k], csc.c[i - k], s);
            csc.c[i] = -s * csc.c[0];
        }
        cot = jmul<N>(jc, csc, N);
        Jet<N> csc2 = jmul<N>(csc, csc, N);
        const double mm = (double)m * (double)m;
#pragma unroll
        for (int i = 0; i <= N; ++i) jm2.c[i] = mm * csc2.c[i];
    }
    if (half == 0) {
        Jet<N> al[PT + 1], be[PT + 1];
#pragma unroll
        for (int p = 0; p <= PT; ++p)
#pragma unroll
            for (int i = 0; i <= N; ++i) al[p].c[i] = be[p].c[i] = 0.0;
        al[0].c[0] = 1.0;
        double ca[N + 1][PT + 1], cb[N + 1][PT + 1];
        family_coeffs<N, PT>(al, be, jm2, cot, ca, cb);
#pragma unroll
        for (int j = 0; j <= N; ++j) {
            double nre = 0, nim = 0, sre = 0, sim = 0;
#pragma unroll
            for (int p = 0; p <= PT; ++p) {
                nre += ca[j][p] * nsum(0, 2 * p) + cb[j][p] * nsum(1, 2 * p);
                nim += ca[j][p] * nsum(0, 2 * p + 1) + cb[j][p] * nsum(1, 2 * p + 1);
                sre += ca[j][p] * dsum(0, 2 * p) + cb[j][p] * dsum(1, 2 * p);
                sim += ca[j][p] * dsum(0, 2 * p + 1) + cb[j][p] * dsum(1, 2 * p + 1);
            }
            FT[j * plane + (size_t)r * (lmax + 1) + m] = make_float2((float)nre, (float)nim);
            if (rs != r) {
                const double sg = (j & 1) ? -1.0 : 1.0;
                FT[j * plane + (size_t)rs * (lmax + 1) + m] = make_float2((float)(sg * sre), (float)(sg * sim));
            }
        }
        return;
    }
    if constexpr (POL) {
        const double dm = (double)m;
        Jet<N> cscot = jmul<N>(csc, cot, N);
        double wa[N + 1][PS + 1], wb[N + 1][PS + 1], xa[N + 1][PS + 1], xb[N + 1][PS + 1];
        {
            Jet<N> al[PS + 1], be[PS + 1];
#pragma unroll
            for (int p = 0; p <= PS; ++p)
#pragma unroll
                for (int i = 0; i <= N; ++i) al[p].c[i] = be[p].c[i] = 0.0;
#pragma unroll
            for (int i = 0; i <= N; ++i) {
                al[0].c[i] = 2.0 * jm2.c[i];
                be[0].c[i] = -2.0 * cot.c[i];
            }
            al[1].c[0] = -1.0;
            family_coeffs<N, PS>(al, be, jm2, cot, wa, wb);
        }
        {
            Jet<N> al[PS + 1], be[PS + 1];
#pragma unroll
            for (int p = 0; p <= PS; ++p)
#pragma unroll
                for (int i = 0; i <= N; ++i) al[p].c[i] = be[p].c[i] = 0.0;
#pragma unroll
            for (int i = 0; i <= N; ++i) {
                al[0].c[i] = 2.0 * dm * cscot.c[i];
                be[0].c[i] = -2.0 * dm * csc.c[i];
            }
            family_coeffs<N, PS>(al, be, jm2, cot, xa, xb);
        }
#pragma unroll
        for (int j = 0; j <= N; ++j) {
            double ewn[2] = {0, 0}, exn[2] = {0, 0}, bwn[2] = {0, 0}, bxn[2] = {0, 0};
            double ews[2] = {0, 0}, exs[2] = {0, 0}, bws[2] = {0, 0}, bxs[2] = {0, 0};
#pragma unroll
            for (int p = 0; p <= PS; ++p) {
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) {
                    const int ce = C.nT + 2 * p + ri;
                    ewn[ri] += wa[j][p] * nsum(0, ce) + wb[j][p] * nsum(1, ce);
                    exn[ri] += xa[j][p] * nsum(0, ce) + xb[j][p] * nsum(1, ce);
                    ews[ri] += wa[j][p] * dsum(0, ce) + wb[j][p] * dsum(1, ce);
                    exs[ri] += xa[j][p] * dsum(0, ce) + xb[j][p] * dsum(1, ce);
                    if constexpr (HASB) {
                        const int cb_ = C.nT + C.nE + 2 * p + ri;
                        bwn[ri] += wa[j][p] * nsum(0, cb_) + wb[j][p] * nsum(1, cb_);
                        bxn[ri] += xa[j][p] * nsum(0, cb_) + xb[j][p] * nsum(1, cb_);
                        bws[ri] += wa[j][p] * dsum(0, cb_) + wb[j][p] * dsum(1, cb_);
                        bxs[ri] += xa[j][p] * dsum(0, cb_) + xb[j][p] * dsum(1, cb_);
                    }
                }
            }
            // south: W-type sums carry (-1)^j, X-type sums -(-1)^j
            const double sg = (j & 1) ? -1.0 : 1.0;
#pragma unroll
            for (int ri = 0; ri < 2; ++ri) {
                ews[ri] *= sg;
                bws[ri] *= sg;
                exs[ri] *= -sg;
                bxs[ri] *= -sg;
            }
            // Q = -(EW + i BX), U = i EX - BW  (complex sums)
            const size_t on = j * plane + (size_t)r * (lmax + 1) + m;
            FQ[on] = make_float2((float)(-(ewn[0] - bxn[1])), (float)(-(ewn[1] + bxn[0])));
            FU[on] = make_float2((float)(-exn[1] - bwn[0]), (float)(exn[0] - bwn[1]));
            if (rs != r) {
                const size_t os = j * plane + (size_t)rs * (lmax + 1) + m;
                FQ[os] = make_float2((float)(-(ews[0] - bxs[1])), (float)(-(ews[1] + bxs[0])));
                FU[os] = make_float2((float)(-exs[1] - bws[0]), (float)(exs[0] - bws[1]));
            }
        }
    }
}

// LDS of one workgroup: chunk operands during the l loop, epilogue buffer
// afterwards.
template <int NC>
struct MfmaSmem {
    struct Chunk {
        float rhs[KCH * NCOL];
        double2 cf[KCH + 2];
    };
    struct Epi {
        double tot[RPW][4][NC];  // [ring][type*2+parity][col]
    };
    union {
        Chunk ch;
        Epi ep;
    };
};

// One work item: ring block rblk (RPB ring pairs from j.rbeg), m-groups
// mg0 .. mg0 + nmg - 1 (MGRP consecutive m each) of one realization.
template <int N, bool POL, bool HASB>
__device__ void mfma_item(const MfmaJob &J, int rblk, int mg0, int nmg, MfmaSmem<cols_of(N, HASB).ncol> &sm)
{
    const int lmax = J.lmax, ntheta = J.ntheta, nrp = J.nrp, jtab = J.jtab;
    const double2 *__restrict__ trig = J.trig;
    const double *__restrict__ theta = J.theta;
    const double4 *__restrict__ coef0 = J.coef0;
    const double *__restrict__ start = J.start;
    const int *__restrict__ exps = J.exps;
    const int *__restrict__ mcut = J.mcut;
    const double2 *__restrict__ almT = J.almT;
    const double2 *__restrict__ almE = J.almE;
    const double2 *__restrict__ almB = J.almB;
    float2 *__restrict__ FT = J.FT;
    float2 *__restrict__ FQ = J.FQ;
    float2 *__restrict__ FU = J.FU;
    constexpr Cols C = cols_of(N, HASB);
    static_assert(C.ncol <= NCOL, "column block overflow");
    constexpr int NC = C.ncol;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int hi = lane >> 5;          // lanes 32..63 run two l-steps ahead
    const int rl = lane & 31;
    const int r = J.rbeg + rblk * RPB + wave * RPW + rl;
    const bool live = r < nrp;
    const double x = live ? trig[r].x : 0.0;
    const double sn = live ? trig[r].y : 1.0;
    const double th = live ? theta[r] : 1.5707963267948966;
    const int rs = ntheta - 1 - r;
    const size_t plane = (size_t)ntheta * (lmax + 1);
    const int mc = live ? mcut[r] + 2 : -1;  // spin-2 terms reach two past the scalar cut

    for (int mi = 0; mi < MGRP * nmg; ++mi) {
        const int m = mg0 * MGRP + mi;
        if (m > lmax) break;
        const size_t base = (size_t)m * (2 * lmax + 1 - m) / 2;
        if (!__syncthreads_or(m <= mc)) {  // evanescent for every ring of the block
            if (live && hi == 0) {
                for (int j = 0; j <= N; ++j) {
                    FT[j * plane + (size_t)r * (lmax + 1) + m] = make_float2(0.f, 0.f);
                    if (rs != r) FT[j * plane + (size_t)rs * (lmax + 1) + m] = make_float2(0.f, 0.f);
                    if (POL) {
                        FQ[j * plane + (size_t)r * (lmax + 1) + m] = make_float2(0.f, 0.f);
                        FU[j * plane + (size_t)r * (lmax + 1) + m] = make_float2(0.f, 0.f);
                        if (rs != r) {
                            FQ[j * plane + (size_t)rs * (lmax + 1) + m] = make_float2(0.f, 0.f);
                            FU[j * plane + (size_t)rs * (lmax + 1) + m] = make_float2(0.f, 0.f);
                        }
                    }
                }
            }
            continue;
        }

        double l1 = 0.0, l2 = 0.0, d1 = 0.0, d2 = 0.0;
        int e = 1;
        if (live) {
            const double *sb = start + (size_t)m * jtab * nrp;  // family 0, l = m
            l1 = sb[r];
            d1 = sb[(size_t)nrp + r];
            e = exps[(size_t)m * nrp + r];
        }
        auto step = [&](double a, double c) {
            const double nl1 = a * (x * l1) - c * l2;
            const double nd1 = a * fma(x, d1, -sn * l1) - c * d2;
            l2 = l1;
            l1 = nl1;
            d2 = d1;
            d1 = nd1;
        };
        if (hi) {  // the upper half-wave runs two l-steps ahead
            for (int s2 = 1; s2 <= 2; ++s2) {
                double a = 0.0, c = 0.0;
                if (m + s2 <= lmax) {
                    const double4 q4 = coef0[base + m + s2];
                    a = q4.x;
                    c = q4.z;
                }
                step(a, c);
            }
        }

        double tot[2][2][16];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int v = 0; v < 16; ++v) tot[t][p][v] = 0.0;

        for (int c0 = m; c0 <= lmax; c0 += KCH) {
            __syncthreads();
            {
                const int ll = tid >> 2, cq = tid & 3;
                const int l = c0 + ll;
                double2 aT = make_double2(0, 0), aE = make_double2(0, 0), aB = make_double2(0, 0);
                double L = (double)l * (double)(l + 1), nl = 0.0;
                if (l <= lmax) {
                    aT = almT[base + l];
                    if (POL) {
                        aE = almE[base + l];
                        if (HASB) aB = almB[base + l];
                        if (l >= 2) nl = 1.0 / sqrt((double)(l - 1) * l * (double)(l + 1) * (double)(l + 2));
                    }
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int c = cq * 8 + q;
                    double v = 0.0;
                    if (c < C.nT) {
                        const int p = c >> 1;
                        double w = 1.0;
                        for (int t = 0; t < p; ++t) w *= L;
                        v = w * ((c & 1) ? aT.y : aT.x);
                    } else if (POL && c < C.nT + C.nE) {
                        const int p = (c - C.nT) >> 1;
                        double w = nl;
                        for (int t = 0; t < p; ++t) w *= L;
                        v = w * (((c - C.nT) & 1) ? aE.y : aE.x);
                    } else if (POL && HASB && c < C.ncol) {
                        const int p = (c - C.nT - C.nE) >> 1;
                        double w = nl;
                        for (int t = 0; t < p; ++t) w *= L;
                        v = w * (((c - C.nT - C.nE) & 1) ? aB.y : aB.x);
                    }
                    sm.ch.rhs[ll * NCOL + c] = (float)v;
                }
                if (tid < KCH + 2) {
                    const int lc = c0 + tid;
                    double2 cf = make_double2(0, 0);
                    if (lc <= lmax) {
                        const double4 q4 = coef0[base + lc];
                        cf = make_double2(q4.x, q4.z);
                    }
                    sm.ch.cf[tid] = cf;
                }
            }
            __syncthreads();
            floatx16 acc[2][2];  // [type][parity]
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int v = 0; v < 16; ++v) acc[t][p][v] = 0.0f;
            const int ng = min(KCH, lmax - c0 + 1);
            for (int g = 0; g < ng; g += 4) {
                // lane value at q: l = c0 + g + q + 2 hi; the state already holds
                // that l at the very first group of this m (start value / prologue),
                // otherwise one recursion step per q (zero coefficients past lmax).
                const bool first = (c0 == m) && (g == 0);
                float v[2], w[2];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!(first && q == 0)) {
                        const double2 cf = sm.ch.cf[g + q + 2 * hi];
                        step(cf.x, cf.y);
                    }
                    if (q < 2) {
                        v[q] = (e == 0) ? (float)l1 : 0.0f;
                        w[q] = (e == 0) ? (float)d1 : 0.0f;
                    }
                }
                if (e > 0) {
                    const double mx = fmax(fmax(fabs(l1), fabs(l2)), fmax(fabs(d1), fabs(d2)));
                    if (mx > kHi) {
                        l1 *= kDown;
                        l2 *= kDown;
                        d1 *= kDown;
                        d2 *= kDown;
                        e -= 1;
                    }
                }
                const float bev = sm.ch.rhs[(g + 0 + 2 * hi) * NCOL + rl];
                const float bod = sm.ch.rhs[(g + 1 + 2 * hi) * NCOL + rl];
                acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(v[0], bev, acc[0][0], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[0], bev, acc[1][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(v[1], bod, acc[0][1], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[1], bod, acc[1][1], 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int vv = 0; vv < 16; ++vv) tot[t][p][vv] += (double)acc[t][p][vv];
        }

        // ---- epilogue: the waves take turns transposing their totals to one
        // lane per ring (lanes 0..31 then form T, lanes 32..63 form Q/U) ----
        for (int turn = 0; turn < WG / 64; ++turn) {
            __syncthreads();
            if (wave == turn && rl < NC) {
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int p = 0; p < 2; ++p)
#pragma unroll
                        for (int vv = 0; vv < 16; ++vv) {
                            const int row = 8 * (vv >> 2) + 4 * hi + (vv & 3);
                            sm.ep.tot[row][t * 2 + p][rl] = tot[t][p][vv];
                        }
            }
            __syncthreads();
            if (wave == turn && live) epilogue<N, POL, HASB>(sm.ep.tot[rl], hi, m, th, r, rs, lmax, plane, FT, FQ, FU);
        }
    }
}

template <int N, bool POL, bool HASB>
__global__ __launch_bounds__(WG) void k_legendre_mfma(const MfmaJob J)
{
    __shared__ MfmaSmem<cols_of(N, HASB).ncol> sm;
    mfma_item<N, POL, HASB>(J, blockIdx.x, blockIdx.y, 1, sm);
}

// Persistent form: workgroups pop work items (realization, ring block,
// first m-group, m-groups) from a queue ordered longest first until it is
// empty; every workgroup exits once the head passes the end.
template <int N, bool POL, bool HASB>
__global__ __launch_bounds__(WG) void k_legendre_mfma_queue(const MfmaJob *__restrict__ jobs,
                                                            const int4 *__restrict__ items, int nitems,
                                                            int *__restrict__ head)
{
    __shared__ MfmaSmem<cols_of(N, HASB).ncol> sm;
    __shared__ int s_it;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_it = atomicAdd(head, 1);
        __syncthreads();
        const int it = s_it;
        if (it >= nitems) break;
        const int4 w = items[it];
        mfma_item<N, POL, HASB>(jobs[w.x], w.y, w.z, w.w, sm);
    }
}

MfmaJob make_job(const Plan &p, const void *T, const void *E, const void *B, void *FT, void *FQ, void *FU)
{
    MfmaJob J{};
    J.lmax = p.lmax;
    J.ntheta = p.ntheta;
    J.nrp = p.nrp;
    J.rbeg = p.rpole;
    J.jtab = p.jtab;
    J.trig = (const double2 *)p.trig.ptr;
    J.theta = (const double *)p.theta.ptr;
    J.coef0 = (const double4 *)p.coef0.ptr;
    J.start = (const double *)p.start.ptr;
    J.exps = (const int *)p.exps.ptr;
    J.mcut = (const int *)p.mcut.ptr;
    J.almT = (const double2 *)T;
    J.almE = (const double2 *)E;
    J.almB = (const double2 *)B;
    J.FT = (float2 *)FT;
    J.FQ = (float2 *)FQ;
    J.FU = (float2 *)FU;
    return J;
}

template <int N, bool POL, bool HASB>
hipError_t launch_N(Plan &p, const void *T, const void *E, const void *B, void *FT, void *FQ, void *FU)
{
    if constexpr (cols_of(N, HASB).ncol > NCOL) {
        return hipErrorInvalidValue;
    } else {
        const int nr = p.nrp - p.rpole;
        if (nr <= 0) return hipSuccess;
        dim3 grid((nr + RPB - 1) / RPB, (p.lmax + 1 + MGRP - 1) / MGRP);
        hipLaunchKernelGGL((k_legendre_mfma<N, POL, HASB>), grid, dim3(WG), 0, p.stream,
                           make_job(p, T, E, B, FT, FQ, FU));
        return hipGetLastError();
    }
}

template <int N, bool POL, bool HASB>
hipError_t launch_queue_N(hipStream_t st, const MfmaJob *jobs, const int4 *items, int nitems, int *head, int ngroups)
{
    if constexpr (cols_of(N, HASB).ncol > NCOL) {
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_legendre_mfma_queue<N, POL, HASB>), dim3(ngroups), dim3(WG), 0, st, jobs, items, nitems,
                           head);
        return hipGetLastError();
    }
}

}  // namespace

bool mfma_supported(int order, bool hasb) { return cols_of(order, hasb).ncol <= NCOL; }

int mfma_ring_block() { return RPB; }
int mfma_m_group() { return MGRP; }

MfmaJob mfma_job(const Plan &p, const void *T, const void *E, const void *B, void *FT, void *FQ, void *FU)
{
    return make_job(p, T, E, B, FT, FQ, FU);
}

hipError_t launch_legendre_mfma_queue(int order, bool pol, bool hasb, hipStream_t st, const MfmaJob *jobs,
                                      const int4 *items, int nitems, int *head, int ngroups)
{
#define TL_CASE(NN)                                                                                    \
    case NN:                                                                                           \
        if (!pol) return launch_queue_N<NN, false, false>(st, jobs, items, nitems, head, ngroups);      \
        if (hasb) return launch_queue_N<NN, true, true>(st, jobs, items, nitems, head, ngroups);       \
        return launch_queue_N<NN, true, false>(st, jobs, items, nitems, head, ngroups);
    switch (order) {
        TL_CASE(0)
        TL_CASE(1)
        TL_CASE(2)
        TL_CASE(3)
        TL_CASE(4)
        TL_CASE(5)
        TL_CASE(6)
        TL_CASE(7)
        TL_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef TL_CASE
}

hipError_t launch_legendre_mfma(Plan &p, const void *T, const void *E, const void *B, void *FT, void *FQ, void *FU)
{
    const bool pol = p.pol, hasb = pol && B != nullptr;
#define TL_CASE(NN)                                                                                 \
    case NN:                                                                                        \
        if (!pol) return launch_N<NN, false, false>(p, T, E, B, FT, FQ, FU);                         \
        if (hasb) return launch_N<NN, true, true>(p, T, E, B, FT, FQ, FU);                          \
        return launch_N<NN, true, false>(p, T, E, B, FT, FQ, FU);
    switch (p.order) {
        TL_CASE(0)
        TL_CASE(1)
        TL_CASE(2)
        TL_CASE(3)
        TL_CASE(4)
        TL_CASE(5)
        TL_CASE(6)
        TL_CASE(7)
        TL_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef TL_CASE
}

}  // namespace tl
