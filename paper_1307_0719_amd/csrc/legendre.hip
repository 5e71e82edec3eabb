// Harmonic (Legendre) stage of Taylor lensing on gfx950.
//
// For every m and ring the stage forms the theta-derivatives of the per-m
// Fourier coefficients of the unlensed fields (the derivative inputs of the
// pixel-relative Taylor expansion, eqs. 4-5 of Naess & Louis 2013),
//
//     F^{(j)}_m(theta) = sum_{l>=m} a_lm d^j/dtheta^j s_lambda_lm(theta),  j = 0..J,
//
// for spin s = 0 (T) and s = +-2 (Q/U).  s_lambda_lm obeys, at fixed (m, s),
//     lam_L = a_L (cos t + b_L) lam_{L-1} - c_L lam_{L-2}
// with a_L = sqrt((2L+1)(2L-1)) L / R_L,  b_L = m s / (L(L-1)),
// c_L = sqrt((2L+1)/(2L-3)) L R_{L-1} / ((L-1) R_L), R_L = sqrt((L^2-m^2)(L^2-s^2)).
// Differentiating every step by Leibniz' rule gives the recursion of all
// derivative orders at once: d^j[(cos t + b) p] = b p^{(j)} + sum_i C(j,i) cos^{(i)} p^{(j-i)}.
//
// Design:
//  * one lane per ring pair (theta, pi - theta): the north/south values come
//    from the parity lam(pi - t) = (-1)^{l+m+j} lam(t) (spin: the opposite spin
//    family), so the recursion runs once per pair;
//  * one wave per m; eight waves (eight consecutive m) per workgroup so that
//    the F[.][ring][m] writes of a workgroup fill whole cache lines;
//  * all recursion arithmetic in FP64 registers; a_lm and the recursion
//    coefficients are wave-uniform (scalar loads);
//  * underflow of sin^m t for large m: values are kept as mantissa * 2^(-512 e)
//    with an integer e per lane and family; e > 0 means "below 2^-256, not
//    accumulated"; the start values at l = max(m, |s|) come from a plan-time
//    table built by an m-recursion with the same scaling.
#include <type_traits>

#include "tl_internal.h"

namespace tl {

namespace {

constexpr double kHi = 0x1p256;
constexpr double kLo = 0x1p-256;
constexpr double kUp = 0x1p512;
constexpr double kDown = 0x1p-512;

__host__ __device__ constexpr double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

// d^i/dt^i cos t  and  d^i/dt^i sin t
__device__ __forceinline__ double cosd(double c, double s, int i)
{
    switch (i & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
    }
}
__device__ __forceinline__ double sind(double c, double s, int i)
{
    switch (i & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
    }
}

// ------------------------------------------------------------ tables ----

// Recursion coefficients {a, b, c, 0} for spin 0 and spin +2 at every (l, m)
// of the triangular layout (entries with l <= l_min hold zeros; b of spin -2
// is -b of spin +2).
__global__ void k_coef(int lmax, double4 *__restrict__ coef0, double4 *__restrict__ coef2)
{
    const int m = blockIdx.y;
    const size_t base = (size_t)m * (2 * lmax + 1 - m) / 2;
    for (int L = m + threadIdx.x + blockIdx.x * blockDim.x; L <= lmax; L += blockDim.x * gridDim.x) {
        double4 c0 = make_double4(0, 0, 0, 0), c2 = make_double4(0, 0, 0, 0);
        const double dL = L, dm = m;
        if (L >= m + 1) {
            // spin 0: a = sqrt((4L^2-1)/(L^2-m^2)), c = sqrt((2L+1)/(2L-3) ((L-1)^2-m^2)/(L^2-m^2))
            const double q = dL * dL - dm * dm;
            c0.x = sqrt((4.0 * dL * dL - 1.0) / q);
            if (L >= m + 2) {
                const double K = L - 1;
                c0.z = sqrt((2.0 * dL + 1.0) / (2.0 * dL - 3.0) * ((K * K - dm * dm) / q));
            }
        }
        const int lmin2 = m > 2 ? m : 2;
        if (L >= lmin2 + 1) {
            const double qm = dL * dL - dm * dm, qs = dL * dL - 4.0;
            c2.x = sqrt((2.0 * dL + 1.0) * (2.0 * dL - 1.0) * dL * dL / (qm * qs));
            c2.y = (m == 0) ? 0.0 : 2.0 * dm / (dL * (dL - 1.0));
            if (L >= lmin2 + 2) {
                const double K = L - 1;
                c2.z = sqrt((2.0 * dL + 1.0) / (2.0 * dL - 3.0) * (dL * dL) / (K * K) *
                            ((K * K - dm * dm) / qm) * ((K * K - 4.0) / qs));
            }
        }
        coef0[base + L] = c0;
        coef2[base + L] = c2;
    }
}

// Start values lam^{(j)}_{l_min, m}(theta_r) for every m, as (mantissa, e):
// family 0: spin 0, l_min = m; family 1/2: spin +2/-2, l_min = max(m, 2).
//   lambda_00 = 1/sqrt(4 pi), lambda_mm = -sqrt((2m+1)/(2m)) sin t lambda_{m-1,m-1};
//   s = +-2: m = 0: sqrt(5/4pi) sqrt(6)/4 sin^2 t;  m = 1: -+ sqrt(5/4pi) sin t g;
//   m = 2: sqrt(5/4pi) g^2 with g = sin^2(t/2) (s=+2), cos^2(t/2) (s=-2);
//   m >= 3: -sqrt((2m+1) m / (2(m^2-4))) sin t lam_{m-1}.
// Products only, derivatives by Leibniz (no cancellation at small t).
template <int J>
__global__ void k_start(int lmax, int nrp, int jtab, const double2 *__restrict__ trig,
                        const double *__restrict__ theta, double *__restrict__ start,
                        int *__restrict__ exps)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int fam = blockIdx.y;
    if (r >= nrp) return;
    const double c = trig[r].x, s = trig[r].y;
    double sd[J + 1];
#pragma unroll
    for (int i = 0; i <= J; ++i) sd[i] = sind(c, s, i);

    double *st = start + (size_t)fam * (lmax + 1) * jtab * nrp;
    int *ex = exps + (size_t)fam * (lmax + 1) * nrp;
    auto put = [&](int m, const double(&v)[J + 1], int e) {
#pragma unroll
        for (int j = 0; j <= J; ++j) st[((size_t)m * jtab + j) * nrp + r] = v[j];
        ex[(size_t)m * nrp + r] = e;
    };
    auto leib = [&](const double(&a)[J + 1], const double(&b)[J + 1], double(&o)[J + 1]) {
#pragma unroll
        for (int j = 0; j <= J; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i <= j; ++i) acc = fma(binom(j, i) * a[i], b[j - i], acc);
            o[j] = acc;
        }
    };
    auto renorm_up = [&](double(&v)[J + 1], int &e) {
        double mx = 0.0;
#pragma unroll
        for (int j = 0; j <= J; ++j) mx = fmax(mx, fabs(v[j]));
        if (mx != 0.0 && mx < kLo) {
#pragma unroll
            for (int j = 0; j <= J; ++j) v[j] *= kUp;
            e += 1;
        }
    };

    const double k5 = sqrt(5.0 / (4.0 * M_PI));
    double prev[J + 1], cur[J + 1];
    int e = 0;
    int m0;
    if (fam == 0) {
#pragma unroll
        for (int j = 0; j <= J; ++j) prev[j] = 0.0;
        prev[0] = 1.0 / sqrt(4.0 * M_PI);
        put(0, prev, 0);
        m0 = 1;
    } else {
        if (lmax < 2) {
            // nothing: spin-2 functions need l >= 2
            return;
        }
        const double t = theta[r];
        const double sh = sin(0.5 * t), ch = cos(0.5 * t);
        double g[J + 1];
#pragma unroll
        for (int i = 0; i <= J; ++i)
            g[i] = (i == 0) ? ((fam == 1) ? sh * sh : ch * ch)
                            : ((fam == 1) ? -0.5 : 0.5) * cosd(c, s, i);
        double v[J + 1];
        leib(sd, sd, v);
#pragma unroll
        for (int j = 0; j <= J; ++j) v[j] *= k5 * sqrt(6.0) * 0.25;
        put(0, v, 0);
        leib(sd, g, v);
#pragma unroll
        for (int j = 0; j <= J; ++j) v[j] *= (fam == 1) ? -k5 : k5;
        put(1, v, 0);
        leib(g, g, prev);
#pragma unroll
        for (int j = 0; j <= J; ++j) prev[j] *= k5;
        put(2, prev, 0);
        m0 = 3;
    }
    for (int m = m0; m <= lmax; ++m) {
        const double dm = m;
        const double f = (fam == 0) ? -sqrt((2.0 * dm + 1.0) / (2.0 * dm))
                                    : -sqrt((2.0 * dm + 1.0) * dm / (2.0 * (dm * dm - 4.0)));
        leib(sd, prev, cur);
#pragma unroll
        for (int j = 0; j <= J; ++j) prev[j] = f * cur[j];
        renorm_up(prev, e);
        put(m, prev, e);
    }
}

// Evanescent cut: for ring pair r, the largest m whose lambda_lm(theta_r)
// (or, at l = m, one of its stored theta-derivatives) reaches 2^-200 for some
// l <= lmax.  Beyond it the derivative maps, scaled by dtheta^j / j!, get
// contributions below 2^-200 (m / r)^j: dropped.  One lane per (r, m): the
// j = 0 recursion with the same exponent scaling as the kernels, stopped at
// the first significant l.
__global__ void k_mcut(int lmax, int nrp, int jtab, const double2 *__restrict__ trig,
                       const double4 *__restrict__ coef0, const double *__restrict__ start,
                       const int *__restrict__ exps, int *__restrict__ mcut)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (r >= nrp || m > lmax) return;
    const double x = trig[r].x;
    double p1 = start[(size_t)m * jtab * nrp + r], p2 = 0.0;
    int e = exps[(size_t)m * nrp + r];
    const size_t base = (size_t)m * (2 * lmax + 1 - m) / 2;
    const double sig = 0x1p-200;
    // at the start also test the stored theta-derivatives: on the pole ring the
    // value vanishes for m >= 1 while derivatives of order >= m do not
    double s0 = 0.0;
    for (int j = 0; j < jtab; ++j) s0 = fmax(s0, fabs(start[((size_t)m * jtab + j) * nrp + r]));
    bool hit = (e == 0) && s0 >= sig;
    for (int l = m + 1; l <= lmax && !hit; ++l) {
        const double4 cf = coef0[base + l];
        const double nv = cf.x * (x * p1) - cf.z * p2;
        p2 = p1;
        p1 = nv;
        if (e > 0 && fmax(fabs(p1), fabs(p2)) > kHi) {
            p1 *= kDown;
            p2 *= kDown;
            e -= 1;
        }
        hit = (e == 0) && fabs(p1) >= sig;
    }
    if (hit) atomicMax(&mcut[r], m);
}

// ------------------------------------------------------------ recursion --

template <int J>
struct Rec {
    double p1[J + 1], p2[J + 1];
    int e;
};

template <int J>
__device__ __forceinline__ void rec_step(Rec<J> &st, double4 cf, double xb, const double (&w)[J + 1][J + 1])
{
    double cur[J + 1];
#pragma unroll
    for (int j = 0; j <= J; ++j) {
        double t = xb * st.p1[j];
#pragma unroll
        for (int i = 1; i <= j; ++i) t = fma(w[j][i], st.p1[j - i], t);
        cur[j] = fma(cf.x, t, -cf.z * st.p2[j]);
    }
#pragma unroll
    for (int j = 0; j <= J; ++j) {
        st.p2[j] = st.p1[j];
        st.p1[j] = cur[j];
    }
}

template <int J>
__device__ __forceinline__ void renorm_down(Rec<J> &st)
{
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j <= J; ++j) mx = fmax(mx, fmax(fabs(st.p1[j]), fabs(st.p2[j])));
    if (mx > kHi) {
#pragma unroll
        for (int j = 0; j <= J; ++j) {
            st.p1[j] *= kDown;
            st.p2[j] *= kDown;
        }
        st.e -= 1;
    }
}

template <int J, int NR>
__device__ __forceinline__ void accum(double2 (&acc)[NR][J + 1], const double2 (&a)[NR], const double (&p)[J + 1])
{
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
        for (int j = 0; j <= J; ++j) {
            acc[q][j].x = fma(a[q].x, p[j], acc[q][j].x);
            acc[q][j].y = fma(a[q].y, p[j], acc[q][j].y);
        }
}

// Per-wave LDS staging of the recursion coefficients and right-hand sides:
// chunk k holds l in [64k, 64k + 64); lane q loads entry q with a vector
// load, the recursion then reads the chunk by broadcast.  Only the owning
// wave touches its region, so wave-scope fences order the accesses.
template <int NR>
struct Stage {
    double4 cf[64];
    double2 a[NR][64];
};

template <int NR>
__device__ __forceinline__ void stage_fill(Stage<NR> &st, int cbase, int lmax, const double4 *__restrict__ coef,
                                           const double2 *const (&rr)[NR])
{
    const int q = threadIdx.x & 63;
    const int l = cbase + q;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (l <= lmax) {
        st.cf[q] = coef[l];
#pragma unroll
        for (int k = 0; k < NR; ++k) st.a[k][q] = rr[k][l];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Run one family over l = lmin..lmax, accumulating into accE (l even) and
// accO (l odd) for NR right-hand sides rr (realizations sharing the
// recursion).  rhs pointers and coef are based at (l = 0, m) of the
// triangular layout.  BSGN multiplies the table's b (spin 0: 0, spin +2: +1,
// spin -2: -1).  The loop walks 64-l chunks staged in LDS; a chunk in which
// every lane of the wave already has exponent 0 runs without the exponent
// logic (values stay O(1) from there on), two steps per iteration.
template <int J, int NR, int BSGN>
__device__ void run_family(int lmin, int lmax, double x, const double (&w)[J + 1][J + 1],
                           const double4 *__restrict__ coef, const double2 *const (&rr)[NR], Rec<J> &st,
                           double2 (&accE)[NR][J + 1], double2 (&accO)[NR][J + 1], Stage<NR> &sg)
{
    if (lmin > lmax) return;
    auto xb = [&](const double4 &cf) -> double {
        if constexpr (BSGN == 0) return x;
        else if constexpr (BSGN > 0) return x + cf.y;
        else return x - cf.y;
    };
    auto rhs = [&](double2 (&a)[NR], int q) {
#pragma unroll
        for (int k = 0; k < NR; ++k) a[k] = sg.a[k][q];
    };
    int cb = lmin & ~63;
    stage_fill<NR>(sg, cb, lmax, coef, rr);
    if constexpr (J >= 2) {
        // many derivative orders: the compact loop keeps the register count
        // (and occupancy) of the larger recursion state low
        double2 a[NR];
        auto fetch = [&](int l, double4 &cf) {
            if (l >= cb + 64) {
                cb = l & ~63;
                stage_fill<NR>(sg, cb, lmax, coef, rr);
            }
            cf = sg.cf[l - cb];
            rhs(a, l - cb);
        };
        double4 cf;
        if (st.e == 0) {
            fetch(lmin, cf);
            if (lmin & 1) accum<J, NR>(accO, a, st.p1);
            else accum<J, NR>(accE, a, st.p1);
        }
        int l = lmin + 1;
        if (l <= lmax && (l & 1)) {
            fetch(l, cf);
            rec_step<J>(st, cf, xb(cf), w);
            if (st.e > 0) renorm_down<J>(st);
            if (st.e == 0) accum<J, NR>(accO, a, st.p1);
            ++l;
        }
        for (; l + 1 <= lmax; l += 2) {
            fetch(l, cf);
            rec_step<J>(st, cf, xb(cf), w);
            if (st.e == 0) accum<J, NR>(accE, a, st.p1);
            fetch(l + 1, cf);
            rec_step<J>(st, cf, xb(cf), w);
            if (st.e == 0) accum<J, NR>(accO, a, st.p1);
            if (st.e > 0) renorm_down<J>(st);
        }
        if (l <= lmax) {
            fetch(l, cf);
            rec_step<J>(st, cf, xb(cf), w);
            if (st.e > 0) renorm_down<J>(st);
            if (st.e == 0) accum<J, NR>(accE, a, st.p1);
        }
        return;
    }
    {  // the start value itself (l = lmin)
        double2 a[NR];
        rhs(a, lmin - cb);
        if (st.e == 0) {
            if (lmin & 1) accum<J, NR>(accO, a, st.p1);
            else accum<J, NR>(accE, a, st.p1);
        }
    }
    int l = lmin + 1;
    while (l <= lmax) {
        if (l >= cb + 64) {
            cb += 64;
            stage_fill<NR>(sg, cb, lmax, coef, rr);
        }
        const int end = min(lmax, cb + 63);  // last l of this chunk
        if (__all(st.e == 0)) {
            // fast path: align l to even, then (even, odd) pairs
            auto one = [&](double2 (&A)[NR][J + 1]) {
                const int q = l - cb;
                double2 a[NR];
                const double4 c0 = sg.cf[q];
                rec_step<J>(st, c0, xb(c0), w);
                rhs(a, q);
                accum<J, NR>(A, a, st.p1);
                ++l;
            };
            if ((l & 1) && l <= end) one(accO);
#pragma unroll 1
            for (; l + 1 <= end; l += 2) {
                const int q = l - cb;
                double2 a[NR];
                const double4 c0 = sg.cf[q];
                rec_step<J>(st, c0, xb(c0), w);
                rhs(a, q);
                accum<J, NR>(accE, a, st.p1);
                const double4 c1 = sg.cf[q + 1];
                rec_step<J>(st, c1, xb(c1), w);
                rhs(a, q + 1);
                accum<J, NR>(accO, a, st.p1);
            }
            if (l <= end) one(accE);
        } else {
#pragma unroll 1
            for (; l <= end; ++l) {
                const int q = l - cb;
                const double4 c0 = sg.cf[q];
                rec_step<J>(st, c0, xb(c0), w);
                if (st.e > 0) renorm_down<J>(st);
                if (st.e == 0) {
                    double2 a[NR];
                    rhs(a, q);
                    if (l & 1) accum<J, NR>(accO, a, st.p1);
                    else accum<J, NR>(accE, a, st.p1);
                }
            }
        }
    }
}

template <int J>
__device__ __forceinline__ void leibniz_weights(double c, double s, double (&w)[J + 1][J + 1])
{
#pragma unroll
    for (int j = 0; j <= J; ++j)
#pragma unroll
        for (int i = 0; i <= J; ++i) w[j][i] = (i <= j) ? binom(j, i) * cosd(c, s, i) : 0.0;
}

template <int J>
__device__ __forceinline__ void load_start(Rec<J> &st, const double *__restrict__ start,
                                           const int *__restrict__ exps, int fam, int m, int lmax,
                                           int jtab, int nrp, int r)
{
    const double *sb = start + ((size_t)fam * (lmax + 1) + m) * jtab * nrp;
#pragma unroll
    for (int j = 0; j <= J; ++j) {
        st.p1[j] = sb[(size_t)j * nrp + r];
        st.p2[j] = 0.0;
    }
    st.e = exps[((size_t)fam * (lmax + 1) + m) * nrp + r];
}

template <typename FT>
__device__ __forceinline__ void store_c(FT *F, size_t idx, double2 v);
template <>
__device__ __forceinline__ void store_c<double>(double *F, size_t idx, double2 v)
{
    reinterpret_cast<double2 *>(F)[idx] = v;
}
template <>
__device__ __forceinline__ void store_c<float>(float *F, size_t idx, double2 v)
{
    reinterpret_cast<float2 *>(F)[idx] = make_float2((float)v.x, (float)v.y);
}

// Scalar field, NB realizations sharing the recursion:
//     F_q[j][ring][m] = sum_l a^q_lm d^j lambda_lm(theta_ring).
// One wave: 64 ring pairs at one m (outputs with a NULL F are skipped).
template <int J, int NB, typename FT>
__device__ __forceinline__ void body_scalar(int m, int r0, int lmax, int ntheta, int nrp, int rend, int jtab,
                                            const double2 *__restrict__ trig, const double4 *__restrict__ coef0,
                                            const double *__restrict__ start, const int *__restrict__ exps,
                                            const int *__restrict__ mcut, const DirectSet &set, Stage<NB> &sgw)
{
    if (m > lmax) return;  // whole wave
    const bool live = r0 < rend;
    const bool active = live && m <= mcut[r0];
    const int r = live ? r0 : 0;  // idle lanes still help fill the LDS chunks
    const size_t plane = (size_t)ntheta * (lmax + 1);
    const int rs = ntheta - 1 - r;
    if (!__any(active)) {          // evanescent for the whole wave: zeros
        if (live)
            for (int q = 0; q < NB; ++q) {
                FT *F = (FT *)set.F[q];
                if (!F) continue;
                for (int j = 0; j <= J; ++j) {
                    store_c<FT>(F, j * plane + (size_t)r * (lmax + 1) + m, make_double2(0, 0));
                    store_c<FT>(F, j * plane + (size_t)rs * (lmax + 1) + m, make_double2(0, 0));
                }
            }
        return;
    }
    const double c = trig[r].x, s = trig[r].y;
    double w[J + 1][J + 1];
    leibniz_weights<J>(c, s, w);
    const size_t base = (size_t)m * (2 * lmax + 1 - m) / 2;

    Rec<J> st;
    load_start<J>(st, start, exps, 0, m, lmax, jtab, nrp, r);
    double2 accE[NB][J + 1], accO[NB][J + 1];
    const double2 *rr[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        rr[q] = set.a[q] + base;
#pragma unroll
        for (int j = 0; j <= J; ++j) accE[q][j] = accO[q][j] = make_double2(0, 0);
    }
    run_family<J, NB, 0>(m, lmax, c, w, coef0 + base, rr, st, accE, accO, sgw);

    const bool modd = m & 1;
    if (!live) return;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        FT *F = (FT *)set.F[q];
        if (!F) continue;
#pragma unroll
        for (int j = 0; j <= J; ++j) {
            double2 ev = modd ? accO[q][j] : accE[q][j];  // l + m even
            double2 od = modd ? accE[q][j] : accO[q][j];
            if (!active) ev = od = make_double2(0, 0);
            store_c<FT>(F, j * plane + (size_t)r * (lmax + 1) + m, make_double2(ev.x + od.x, ev.y + od.y));
            if (rs != r) {
                const double sg = (j & 1) ? -1.0 : 1.0;
                store_c<FT>(F, j * plane + (size_t)rs * (lmax + 1) + m,
                            make_double2(sg * (ev.x - od.x), sg * (ev.y - od.y)));
            }
        }
    }
}

template <int J, int NB, typename FT>
__global__ __launch_bounds__(512) void k_legendre_scalar(
    int lmax, int ntheta, int nrp, int rend, int jtab, const double2 *__restrict__ trig,
    const double4 *__restrict__ coef0, const double *__restrict__ start, const int *__restrict__ exps,
    const int *__restrict__ mcut, const DirectSet set)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ Stage<NB> sgs[8];
    body_scalar<J, NB, FT>(blockIdx.y * 8 + wave, blockIdx.x * 64 + (threadIdx.x & 63), lmax, ntheta, nrp, rend,
                           jtab, trig, coef0, start, exps, mcut, set, sgs[wave]);
}

// i * z
__device__ __forceinline__ double2 mul_i(double2 z) { return make_double2(-z.y, z.x); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// Atomic add of a complex value (two independent real adds).
template <typename FT>
__device__ __forceinline__ void add_c(FT *F, size_t idx, double2 v)
{
    atomicAdd(F + 2 * idx, (FT)v.x);
    atomicAdd(F + 2 * idx + 1, (FT)v.y);
}

template <typename FT>
__device__ __forceinline__ double2 load_c(const FT *F, size_t idx);
template <>
__device__ __forceinline__ double2 load_c<double>(const double *F, size_t idx)
{
    return reinterpret_cast<const double2 *>(F)[idx];
}
template <>
__device__ __forceinline__ double2 load_c<float>(const float *F, size_t idx)
{
    const float2 v = reinterpret_cast<const float2 *>(F)[idx];
    return make_double2(v.x, v.y);
}

// Spin-2 field from E (and B), NB realizations sharing the recursion:
// FQ/FU[j][ring][m] = Fourier coefficients of d^j Q and d^j U with
//   P_m = -sum (E + iB) 2lam,  M_m = -sum (E - iB) (-2)lam,
//   Q_m = (P_m + M_m)/2,       U_m = (P_m - M_m)/(2i),
// and, at the south ring, 2lam^{(j)}(pi - t) = (-1)^{l+m+j} (-2)lam^{(j)}(t).
// The spin +2 family gives P north and M south, the spin -2 family M north
// and P south: the first family stores its halves of Q and U, the second
// adds its halves (the lane re-reads its own stores), so no realization's
// results wait in registers for the other family.
//
// SPLIT (the polar caps, where few waves run): the wave runs the one family
// fam0 and adds its halves of Q and U atomically into rows the caller has
// zeroed (a sum of two terms: the same in either order).
template <int J, bool HASB, int NB, typename FT, bool SPLIT>
__device__ __forceinline__ void body_spin(int m, int r0, int fam0, int lmax, int ntheta, int nrp, int rend, int jtab,
                                          const double2 *__restrict__ trig, const double4 *__restrict__ coef2,
                                          const double *__restrict__ start, const int *__restrict__ exps,
                                          const int *__restrict__ mcut, const DirectSet &set,
                                          Stage<NB *(HASB ? 2 : 1)> &sgw)
{
    constexpr int PER = HASB ? 2 : 1;  // right-hand sides per realization
    constexpr int NR = NB * PER;
    if (m > lmax) return;  // whole wave
    const bool live = r0 < rend;
    // spin-2 functions stay below the scalar cut plus 2 (|m - s| <= m + 2)
    const bool active = live && m <= mcut[r0] + 2;
    const int r = live ? r0 : 0;
    const size_t plane = (size_t)ntheta * (lmax + 1);
    const int rs = ntheta - 1 - r;
    const size_t on = (size_t)r * (lmax + 1) + m, os = (size_t)rs * (lmax + 1) + m;
    if (!__any(active)) {
        if (live && !SPLIT)  // (split: the rows are zero already)
            for (int q = 0; q < NB; ++q) {
                FT *FQ = (FT *)set.F[q], *FU = (FT *)set.G[q];
                if (!FQ) continue;
                for (int j = 0; j <= J; ++j) {
                    store_c<FT>(FQ, j * plane + on, make_double2(0, 0));
                    store_c<FT>(FQ, j * plane + os, make_double2(0, 0));
                    store_c<FT>(FU, j * plane + on, make_double2(0, 0));
                    store_c<FT>(FU, j * plane + os, make_double2(0, 0));
                }
            }
        return;
    }
    const double c = trig[r].x, s = trig[r].y;
    double w[J + 1][J + 1];
    leibniz_weights<J>(c, s, w);
    const size_t base = (size_t)m * (2 * lmax + 1 - m) / 2;
    const int lmin = m > 2 ? m : 2;
    const bool modd = m & 1;
    const double2 *rr[NR];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        rr[q * PER] = set.a[q] + base;
        if constexpr (HASB) rr[q * PER + 1] = set.b[q] + base;
    }

#pragma unroll
    for (int fam = 0; fam < 2; ++fam) {
        if (SPLIT && fam != fam0) continue;
        Rec<J> st;
        load_start<J>(st, start, exps, 1 + fam, m, lmax, jtab, nrp, r);
        double2 accE[NR][J + 1], accO[NR][J + 1];
#pragma unroll
        for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int j = 0; j <= J; ++j) accE[k][j] = accO[k][j] = make_double2(0, 0);
        if (fam == 0) run_family<J, NR, 1>(lmin, lmax, c, w, coef2 + base, rr, st, accE, accO, sgw);
        else run_family<J, NR, -1>(lmin, lmax, c, w, coef2 + base, rr, st, accE, accO, sgw);
        if (!live) continue;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            FT *FQ = (FT *)set.F[q], *FU = (FT *)set.G[q];
            if (!FQ) continue;
#pragma unroll
            for (int j = 0; j <= J; ++j) {
                const int kE = q * PER, kB = q * PER + PER - 1;
                const double2 Ee = modd ? accO[kE][j] : accE[kE][j], Eo = modd ? accE[kE][j] : accO[kE][j];
                double2 Be = make_double2(0, 0), Bo = make_double2(0, 0);
                if constexpr (HASB) {
                    Be = modd ? accO[kB][j] : accE[kB][j];
                    Bo = modd ? accE[kB][j] : accO[kB][j];
                }
                const double sg = (j & 1) ? -1.0 : 1.0;
                // family +2: P_N = -(SE + i SB), M_S = -(-1)^j [(Ee - Eo) - i (Be - Bo)]
                // family -2: M_N = -(SE - i SB), P_S = -(-1)^j [(Ee - Eo) + i (Be - Bo)]
                const double2 sumE = cadd(Ee, Eo), sumB = cadd(Be, Bo);
                const double2 difE = csub(Ee, Eo), difB = csub(Be, Bo);
                double2 Pn = make_double2(0, 0), Mn = Pn, Ps = Pn, Ms = Pn;
                if (fam == 0) {
                    Pn = cscale(cadd(sumE, mul_i(sumB)), -1.0);
                    Ms = cscale(csub(difE, mul_i(difB)), -sg);
                } else {
                    Mn = cscale(csub(sumE, mul_i(sumB)), -1.0);
                    Ps = cscale(cadd(difE, mul_i(difB)), -sg);
                }
                if (!active) Pn = Mn = Ps = Ms = make_double2(0, 0);
                // Q = (P + M)/2,  U = -i (P - M)/2
                double2 qn = cscale(cadd(Pn, Mn), 0.5), un = cscale(mul_i(csub(Pn, Mn)), -0.5);
                double2 qs = cscale(cadd(Ps, Ms), 0.5), us = cscale(mul_i(csub(Ps, Ms)), -0.5);
                if constexpr (SPLIT) {
                    add_c<FT>(FQ, j * plane + on, qn);
                    add_c<FT>(FU, j * plane + on, un);
                    if (rs != r) {
                        add_c<FT>(FQ, j * plane + os, qs);
                        add_c<FT>(FU, j * plane + os, us);
                    }
                    continue;
                }
                if (fam == 1) {
                    qn = cadd(qn, load_c<FT>(FQ, j * plane + on));
                    un = cadd(un, load_c<FT>(FU, j * plane + on));
                    if (rs != r) {
                        qs = cadd(qs, load_c<FT>(FQ, j * plane + os));
                        us = cadd(us, load_c<FT>(FU, j * plane + os));
                    }
                }
                store_c<FT>(FQ, j * plane + on, qn);
                store_c<FT>(FU, j * plane + on, un);
                if (rs != r) {
                    store_c<FT>(FQ, j * plane + os, qs);
                    store_c<FT>(FU, j * plane + os, us);
                }
            }
        }
    }
}

template <int J, bool HASB, int NB, typename FT>
__global__ __launch_bounds__(512) void k_legendre_spin(
    int lmax, int ntheta, int nrp, int rend, int jtab, const double2 *__restrict__ trig,
    const double4 *__restrict__ coef2, const double *__restrict__ start, const int *__restrict__ exps,
    const int *__restrict__ mcut, const DirectSet set)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ Stage<NB *(HASB ? 2 : 1)> sgs[8];
    body_spin<J, HASB, NB, FT, false>(blockIdx.y * 8 + wave, blockIdx.x * 64 + (threadIdx.x & 63), 0, lmax, ntheta,
                                      nrp, rend, jtab, trig, coef2, start, exps, mcut, set, sgs[wave]);
}

template <int J>
hipError_t start_tables_J(Plan &p)
{
    dim3 grid((p.nrp + 63) / 64, 3);
    hipLaunchKernelGGL((k_start<J>), grid, dim3(64), 0, p.stream, p.lmax, p.nrp, p.jtab,
                       (const double2 *)p.trig.ptr, (const double *)p.theta.ptr, (double *)p.start.ptr,
                       (int *)p.exps.ptr);
    return hipGetLastError();
}

// Right-hand sides one lane of the direct kernels carries (accumulators:
// 8 (J + 1) VGPRs each) within the 256-VGPR budget of 512-thread workgroups.
constexpr int rhs_max(int J) { return J == 0 ? 5 : J <= 2 ? 4 : J <= 4 ? 3 : J <= 6 ? 2 : 1; }

// The recursion tables a direct spin-0 launch walks: the plan's, or the
// lensing potential's own (band limit lmax_phi, derivative entries of J = 1).
struct RecTab {
    int lmax, jtab;
    const double4 *coef0;
    const double *start;
    const int *exps, *mcut;
};
RecTab rec_tab(const Plan &p, bool phi)
{
    if (phi && p.phi_tables())
        return RecTab{p.lmax_phi, 2, (const double4 *)p.coefP0.ptr, (const double *)p.startP.ptr,
                      (const int *)p.expsP.ptr, (const int *)p.mcutP.ptr};
    return RecTab{p.lmax, p.jtab, (const double4 *)p.coef0.ptr, (const double *)p.start.ptr, (const int *)p.exps.ptr,
                  (const int *)p.mcut.ptr};
}

template <int J, int NB, typename FT>
hipError_t scalar_JN(Plan &p, int rend, const DirectSet &set, const RecTab &t)
{
    dim3 grid((rend + 63) / 64, (t.lmax + 1 + 7) / 8);
    hipLaunchKernelGGL((k_legendre_scalar<J, NB, FT>), grid, dim3(512), 0, p.stream, t.lmax, p.ntheta, p.nrp, rend,
                       t.jtab, (const double2 *)p.trig.ptr, t.coef0, t.start, t.exps, t.mcut, set);
    return hipGetLastError();
}

template <int J, bool HASB, int NB, typename FT>
hipError_t spin_JN(Plan &p, int rend, const DirectSet &set)
{
    dim3 grid((rend + 63) / 64, (p.lmax + 1 + 7) / 8);
    hipLaunchKernelGGL((k_legendre_spin<J, HASB, NB, FT>), grid, dim3(512), 0, p.stream, p.lmax, p.ntheta, p.nrp,
                       rend, p.jtab, (const double2 *)p.trig.ptr, (const double4 *)p.coef2.ptr,
                       (const double *)p.start.ptr, (const int *)p.exps.ptr, (const int *)p.mcut.ptr, set);
    return hipGetLastError();
}

// Realizations per launch: FP32 outputs (the caps of the FP32 and
// tabulated forms) and the FP64 deflection (J = 1) take several, the FP64
// form one.
template <int J, typename FT>
constexpr int scalar_nb() { return (std::is_same<FT, float>::value || J == 1) ? rhs_max(J) : 1; }
template <int J, bool HASB, typename FT>
constexpr int spin_nb()
{
    if (!std::is_same<FT, float>::value) return 1;
    if (!HASB) return J == 1 ? 3 : rhs_max(J);
    return (rhs_max(J) - 1) / 2 > 1 ? (rhs_max(J) - 1) / 2 : 1;
}

// ---- polar caps in one launch ----
//
// The caps hold few ring pairs, so a launch per field and realization group
// leaves most SIMDs idle while each wave walks its l recursion; here every
// (task, m, ring block) is a wave of one launch: the deflection, T, and the
// two spin families of Q/U (split across waves, adding into zeroed rows) of
// every realization group run side by side.
template <int J, bool HASB>
constexpr int caps_nrmax()
{
    constexpr int a = scalar_nb<1, double>(), b = scalar_nb<J, float>(), c = spin_nb<J, HASB, float>() * (HASB ? 2 : 1);
    return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

template <int J, bool HASB>
__global__ __launch_bounds__(512) void k_legendre_caps(int lmax, int ntheta, int nrp, int rend, int jtab,
                                                       const double2 *__restrict__ trig,
                                                       const double4 *__restrict__ coef0,
                                                       const double4 *__restrict__ coef2,
                                                       const double *__restrict__ start, const int *__restrict__ exps,
                                                       const int *__restrict__ mcut, const CapsArgs args)
{
    constexpr int NBD = scalar_nb<1, double>(), NBT = scalar_nb<J, float>(), NBS = spin_nb<J, HASB, float>();
    constexpr int NRM = caps_nrmax<J, HASB>();
    __shared__ Stage<NRM> sgs[8];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m = blockIdx.y * 8 + wave;
    const int r0 = blockIdx.x * 64 + (threadIdx.x & 63);
    const int4 t = args.task[blockIdx.z];
    // members past the task's count repeat its last realization (valid
    // reads) and store nothing
    auto member = [&](int q) { return t.y + (q < t.z ? q : t.z - 1); };
    DirectSet set{};
    if (t.x == 0) {
#pragma unroll
        for (int q = 0; q < NBD; ++q) {
            set.a[q] = args.P[member(q)];
            set.F[q] = q < t.z ? args.FP[member(q)] : nullptr;
        }
        body_scalar<1, NBD, double>(m, r0, lmax, ntheta, nrp, rend, jtab, trig, coef0, start, exps, mcut, set,
                                    reinterpret_cast<Stage<NBD> &>(sgs[wave]));
    } else if (t.x == 1) {
#pragma unroll
        for (int q = 0; q < NBT; ++q) {
            set.a[q] = args.T[member(q)];
            set.F[q] = q < t.z ? args.FT[member(q)] : nullptr;
        }
        body_scalar<J, NBT, float>(m, r0, lmax, ntheta, nrp, rend, jtab, trig, coef0, start, exps, mcut, set,
                                   reinterpret_cast<Stage<NBT> &>(sgs[wave]));
    } else {
#pragma unroll
        for (int q = 0; q < NBS; ++q) {
            set.a[q] = args.E[member(q)];
            set.b[q] = HASB ? args.B[member(q)] : nullptr;
            set.F[q] = q < t.z ? args.FQ[member(q)] : nullptr;
            set.G[q] = q < t.z ? args.FU[member(q)] : nullptr;
        }
        body_spin<J, HASB, NBS, float, true>(m, r0, t.x - 2, lmax, ntheta, nrp, rend, jtab, trig, coef2, start, exps,
                                             mcut, set, reinterpret_cast<Stage<NBS *(HASB ? 2 : 1)> &>(sgs[wave]));
    }
}

// Zero the cap rows [0, rend) and [ntheta - rend, ntheta) of the J + 1
// derivative planes of FQ and FU (FP32 complex) of each realization:
// blockIdx.y = plane * 2 + side, blockIdx.z = realization * 2 + field.
__global__ void k_zero_cap_rows(const CapsArgs args, int ntheta, int lmax, int rend)
{
    const int rr = blockIdx.z >> 1, fld = blockIdx.z & 1;
    const int plane = blockIdx.y >> 1, side = blockIdx.y & 1;
    float *F = (float *)(fld ? args.FU[rr] : args.FQ[rr]);
    const size_t row = (size_t)(lmax + 1) * 2;  // floats per ring row
    const size_t seg = (size_t)rend * row;
    float *base = F + (size_t)plane * ntheta * row + (side ? (size_t)(ntheta - rend) * row : 0);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < seg; i += (size_t)gridDim.x * blockDim.x)
        base[i] = 0.f;
}

template <int J, bool HASB>
hipError_t caps_JH(Plan &p, int rend, const CapsArgs &a, int nreal, hipStream_t st)
{
    if (p.pol && nreal > 0) {
        hipLaunchKernelGGL(k_zero_cap_rows, dim3(256, 2 * (J + 1), 2 * nreal), dim3(256), 0, st, a, p.ntheta,
                           p.lmax, rend);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    dim3 grid((rend + 63) / 64, (p.lmax + 1 + 7) / 8, a.ntask);
    hipLaunchKernelGGL((k_legendre_caps<J, HASB>), grid, dim3(512), 0, st, p.lmax, p.ntheta, p.nrp, rend, p.jtab,
                       (const double2 *)p.trig.ptr, (const double4 *)p.coef0.ptr, (const double4 *)p.coef2.ptr,
                       (const double *)p.start.ptr, (const int *)p.exps.ptr, (const int *)p.mcut.ptr, a);
    return hipGetLastError();
}

template <int J, typename FT>
hipError_t scalar_J(Plan &p, int rend, const DirectSet &set, const RecTab &t)
{
    if (rend <= 0 || set.n <= 0) return hipSuccess;
    constexpr int MX = scalar_nb<J, FT>();
    switch (set.n) {
    case 1: return scalar_JN<J, 1, FT>(p, rend, set, t);
    case 2: if constexpr (MX >= 2) return scalar_JN<J, 2, FT>(p, rend, set, t); break;
    case 3: if constexpr (MX >= 3) return scalar_JN<J, 3, FT>(p, rend, set, t); break;
    case 4: if constexpr (MX >= 4) return scalar_JN<J, 4, FT>(p, rend, set, t); break;
    case 5: if constexpr (MX >= 5) return scalar_JN<J, 5, FT>(p, rend, set, t); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <int J, bool HASB, typename FT>
hipError_t spin_J(Plan &p, int rend, const DirectSet &set)
{
    if (rend <= 0 || set.n <= 0) return hipSuccess;
    constexpr int MX = spin_nb<J, HASB, FT>();
    switch (set.n) {
    case 1: return spin_JN<J, HASB, 1, FT>(p, rend, set);
    case 2: if constexpr (MX >= 2) return spin_JN<J, HASB, 2, FT>(p, rend, set); break;
    case 3: if constexpr (MX >= 3) return spin_JN<J, HASB, 3, FT>(p, rend, set); break;
    case 4: if constexpr (MX >= 4) return spin_JN<J, HASB, 4, FT>(p, rend, set); break;
    case 5: if constexpr (MX >= 5) return spin_JN<J, HASB, 5, FT>(p, rend, set); break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <int J>
int direct_max_J(bool spin, bool hasb, bool out64)
{
    if (!spin) return out64 ? scalar_nb<J, double>() : scalar_nb<J, float>();
    if (hasb) return out64 ? spin_nb<J, true, double>() : spin_nb<J, true, float>();
    return out64 ? spin_nb<J, false, double>() : spin_nb<J, false, float>();
}

}  // namespace

hipError_t launch_tables(Plan &p)
{
    {
        dim3 grid(((p.lmax + 1) + 255) / 256, p.lmax + 1);
        hipLaunchKernelGGL(k_coef, grid, dim3(256), 0, p.stream, p.lmax, (double4 *)p.coef0.ptr,
                           (double4 *)p.coef2.ptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipError_t e;
    switch (p.jtab - 1) {
    case 1: e = start_tables_J<1>(p); break;
    case 2: e = start_tables_J<2>(p); break;
    case 3: e = start_tables_J<3>(p); break;
    case 4: e = start_tables_J<4>(p); break;
    case 5: e = start_tables_J<5>(p); break;
    case 6: e = start_tables_J<6>(p); break;
    case 7: e = start_tables_J<7>(p); break;
    case 8: e = start_tables_J<8>(p); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(p.mcut.ptr, 0xff, p.mcut.bytes, p.stream);  // -1: nothing significant
    if (e != hipSuccess) return e;
    dim3 grid((p.nrp + 255) / 256, p.lmax + 1);
    hipLaunchKernelGGL(k_mcut, grid, dim3(256), 0, p.stream, p.lmax, p.nrp, p.jtab, (const double2 *)p.trig.ptr,
                       (const double4 *)p.coef0.ptr, (const double *)p.start.ptr, (const int *)p.exps.ptr,
                       (int *)p.mcut.ptr);
    e = hipGetLastError();
    if (e != hipSuccess || !p.phi_tables()) return e;
    // the lensing potential's tables at its own band limit (spin 0, J = 1)
    const int L = p.lmax_phi;
    hipLaunchKernelGGL(k_coef, dim3((L + 1 + 255) / 256, L + 1), dim3(256), 0, p.stream, L, (double4 *)p.coefP0.ptr,
                       (double4 *)p.coefP2.ptr);
    hipLaunchKernelGGL((k_start<1>), dim3((p.nrp + 63) / 64, 3), dim3(64), 0, p.stream, L, p.nrp, 2,
                       (const double2 *)p.trig.ptr, (const double *)p.theta.ptr, (double *)p.startP.ptr,
                       (int *)p.expsP.ptr);
    e = hipMemsetAsync(p.mcutP.ptr, 0xff, p.mcutP.bytes, p.stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mcut, dim3((p.nrp + 255) / 256, L + 1), dim3(256), 0, p.stream, L, p.nrp, 2,
                       (const double2 *)p.trig.ptr, (const double4 *)p.coefP0.ptr, (const double *)p.startP.ptr,
                       (const int *)p.expsP.ptr, (int *)p.mcutP.ptr);
    return hipGetLastError();
}

int direct_max(int J, bool spin, bool hasb, bool out64)
{
    switch (J) {
    case 0: return direct_max_J<0>(spin, hasb, out64);
    case 1: return direct_max_J<1>(spin, hasb, out64);
    case 2: return direct_max_J<2>(spin, hasb, out64);
    case 3: return direct_max_J<3>(spin, hasb, out64);
    case 4: return direct_max_J<4>(spin, hasb, out64);
    case 5: return direct_max_J<5>(spin, hasb, out64);
    case 6: return direct_max_J<6>(spin, hasb, out64);
    case 7: return direct_max_J<7>(spin, hasb, out64);
    case 8: return direct_max_J<8>(spin, hasb, out64);
    default: return 0;
    }
}

int caps_nb(int kind, int J, bool hasb)
{
#define TL_NB(JJ)                                                                                 \
    case JJ:                                                                                      \
        return kind == 0   ? scalar_nb<1, double>()                                               \
               : kind == 1 ? scalar_nb<JJ, float>()                                               \
                           : (hasb ? spin_nb<JJ, true, float>() : spin_nb<JJ, false, float>());
    switch (J) {
        TL_NB(0)
        TL_NB(1)
        TL_NB(2)
        TL_NB(3)
        TL_NB(4)
        TL_NB(5)
        TL_NB(6)
    default: return 0;
    }
#undef TL_NB
}

hipError_t launch_legendre_caps(Plan &p, int rend, const CapsArgs &a, int nreal, bool hasb, hipStream_t st)
{
    if (!st) st = p.stream;
    if (rend <= 0 || a.ntask <= 0) return hipSuccess;
    if (a.ntask > kCapsMaxTasks) return hipErrorInvalidValue;
#define TL_CAPS(JJ) \
    case JJ: return hasb ? caps_JH<JJ, true>(p, rend, a, nreal, st) : caps_JH<JJ, false>(p, rend, a, nreal, st);
    switch (p.order) {
        TL_CAPS(0)
        TL_CAPS(1)
        TL_CAPS(2)
        TL_CAPS(3)
        TL_CAPS(4)
        TL_CAPS(5)
        TL_CAPS(6)
    default: return hipErrorInvalidValue;
    }
#undef TL_CAPS
}

hipError_t launch_legendre_scalar_set(Plan &p, int J, int rend, const DirectSet &set, bool out64, bool phi)
{
    const RecTab t = rec_tab(p, phi);
    if (phi && p.phi_tables() && J > 1) return hipErrorInvalidValue;  // its tables hold J <= 1
#define TL_CASE(JJ) \
    case JJ: return out64 ? scalar_J<JJ, double>(p, rend, set, t) : scalar_J<JJ, float>(p, rend, set, t);
    switch (J) {
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

hipError_t launch_legendre_spin_set(Plan &p, int J, int rend, const DirectSet &set, bool out64)
{
    const bool hasb = set.b[0] != nullptr;
#define TL_CASE(JJ)                                                                                    \
    case JJ:                                                                                           \
        if (hasb) return out64 ? spin_J<JJ, true, double>(p, rend, set) : spin_J<JJ, true, float>(p, rend, set); \
        return out64 ? spin_J<JJ, false, double>(p, rend, set) : spin_J<JJ, false, float>(p, rend, set);
    switch (J) {
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

hipError_t launch_legendre_scalar(Plan &p, int J, int rend, const void *alm, void *F, bool out64)
{
    DirectSet set{};
    set.n = 1;
    set.a[0] = (const double2 *)alm;
    set.F[0] = F;
    return launch_legendre_scalar_set(p, J, rend, set, out64);
}

hipError_t launch_legendre_spin(Plan &p, int J, int rend, const void *almE, const void *almB, void *FQ, void *FU,
                                bool out64)
{
    DirectSet set{};
    set.n = 1;
    set.a[0] = (const double2 *)almE;
    set.b[0] = (const double2 *)almB;
    set.F[0] = FQ;
    set.G[0] = FU;
    return launch_legendre_spin_set(p, J, rend, set, out64);
}

}  // namespace tl
