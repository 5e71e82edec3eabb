// Shared device helpers of the L-power harmonic kernels (reduced-precision
// forms): column layout of the right-hand sides, Taylor jets of csc and cot
// and the per-(ring, m) coefficients that turn the lam / lam' sums into the
// theta-derivatives of T and of the spin-2 combinations (the associated
// Legendre equation gives lam'' in terms of lam and lam').
#pragma once

#include "tl_internal.h"

namespace tl {
namespace lp {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

// A float the optimizer cannot see through: without it, a double rounded to
// float and then to FP16/BF16 is folded into one double -> 16-bit conversion,
// which has no instruction and is emulated in integer code.
__device__ __forceinline__ float opaque(float x)
{
    asm volatile("" : "+v"(x));
    return x;
}

template <bool BF>
struct H;
template <>
struct H<true> {
    using T = __bf16;
    using V = bf16x8;
};
template <>
struct H<false> {
    using T = _Float16;
    using V = halfx8;
};

// Columns of one realization: T (L^p a^T, p <= PT), E and B (N_l L^p a, p <=
// PS), then, with def, the lensing potential (a^phi: its lam and lam' sums
// are the theta-derivatives of order 0 and 1 the deflection needs).  Real and
// imaginary parts in adjacent columns.
struct Cols {
    int PT, PS, nT, nE, nB, nP, n1;
};
__host__ __device__ constexpr Cols cols_of(int N, bool pol, bool hasb, bool def = false)
{
    Cols c{};
    c.PT = N / 2;
    c.PS = N / 2 + 1;
    c.nT = 2 * (c.PT + 1);
    c.nE = pol ? 2 * (c.PS + 1) : 0;
    c.nB = pol && hasb ? 2 * (c.PS + 1) : 0;
    c.nP = def ? 2 : 0;
    c.n1 = c.nT + c.nE + c.nB + c.nP;
    return c;
}

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
template <int K>
__device__ __forceinline__ Jet<K> jder(const Jet<K> &a)
{
    Jet<K> r;
#pragma unroll
    for (int i = 0; i < K; ++i) r.c[i] = (double)(i + 1) * a.c[i + 1];
    r.c[K] = 0.0;
    return r;
}
template <int N, int P>
__device__ inline void family_coeffs(Jet<N> (&al)[P + 1], Jet<N> (&be)[P + 1], const Jet<N> &mcsc2, const Jet<N> &cot,
                              double (&ca)[N + 1][P + 1], double (&cb)[N + 1][P + 1])
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

// L-power coefficients of one ring (theta) and m: T family (ta, tb) and the
// spin-2 combinations W (wa, wb) and X (xa, xb).  Built from the Taylor jets
// of sin and cos at theta (csc, cot and m^2 csc^2 by jet products).
template <int N>
struct Jets {
    Jet<N> csc, cot, jm2;
};
template <int N>
__device__ inline void base_jets(double th, int m, Jets<N> &J)
{
    Jet<N> js, jc;
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
    J.csc.c[0] = 1.0 / js.c[0];
#pragma unroll
    for (int i = 1; i <= N; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 1; k <= i; ++k) s = fma(js.c[k], J.csc.c[i - k], s);
        J.csc.c[i] = -s * J.csc.c[0];
    }
    J.cot = jmul<N>(jc, J.csc, N);
    Jet<N> csc2 = jmul<N>(J.csc, J.csc, N);
    const double mm = (double)m * (double)m;
#pragma unroll
    for (int i = 0; i <= N; ++i) J.jm2.c[i] = mm * csc2.c[i];
}

template <int N>
struct CoefT {
    static constexpr int PT = N / 2;
    double ta[N + 1][PT + 1], tb[N + 1][PT + 1];
};
template <int N>
__device__ inline void coefficients_T(double th, int m, CoefT<N> &C)
{
    constexpr int PT = N / 2;
    Jets<N> J;
    base_jets<N>(th, m, J);
    Jet<N> al[PT + 1], be[PT + 1];
#pragma unroll
    for (int p = 0; p <= PT; ++p)
#pragma unroll
        for (int i = 0; i <= N; ++i) al[p].c[i] = be[p].c[i] = 0.0;
    al[0].c[0] = 1.0;
    family_coeffs<N, PT>(al, be, J.jm2, J.cot, C.ta, C.tb);
}

template <int N>
struct CoefP {
    static constexpr int PS = N / 2 + 1;
    double wa[N + 1][PS + 1], wb[N + 1][PS + 1], xa[N + 1][PS + 1], xb[N + 1][PS + 1];
};
template <int N>
__device__ inline void coefficients_P(double th, int m, CoefP<N> &C)
{
    constexpr int PS = N / 2 + 1;
    Jets<N> J;
    base_jets<N>(th, m, J);
    Jet<N> cscot = jmul<N>(J.csc, J.cot, N);
    {
        Jet<N> al[PS + 1], be[PS + 1];
#pragma unroll
        for (int p = 0; p <= PS; ++p)
#pragma unroll
            for (int i = 0; i <= N; ++i) al[p].c[i] = be[p].c[i] = 0.0;
#pragma unroll
        for (int i = 0; i <= N; ++i) {
            al[0].c[i] = 2.0 * J.jm2.c[i];
            be[0].c[i] = -2.0 * J.cot.c[i];
        }
        al[1].c[0] = -1.0;
        family_coeffs<N, PS>(al, be, J.jm2, J.cot, C.wa, C.wb);
    }
    {
        const double dm = (double)m;
        Jet<N> al[PS + 1], be[PS + 1];
#pragma unroll
        for (int p = 0; p <= PS; ++p)
#pragma unroll
            for (int i = 0; i <= N; ++i) al[p].c[i] = be[p].c[i] = 0.0;
#pragma unroll
        for (int i = 0; i <= N; ++i) {
            al[0].c[i] = 2.0 * dm * cscot.c[i];
            be[0].c[i] = -2.0 * dm * J.csc.c[i];
        }
        family_coeffs<N, PS>(al, be, J.jm2, J.cot, C.xa, C.xb);
    }
}

// Right-hand side value of column c (realization c / n1, local column
// c % n1) at degree l: {L^p a^T} for T, {N_l L^p a^E}, {N_l L^p a^B} for the
// spin-2 families, a^phi with DEF, real and imaginary parts in adjacent
// columns.
template <int N, bool POL, bool HASB, int NBAT, bool DEF = false>
__device__ __forceinline__ double rhs_value(const TabBatch &batch, size_t base, int lmax, int l, int c)
{
    constexpr Cols C = cols_of(N, POL, HASB, DEF);
    const int b = c / C.n1, cc = c % C.n1;
    if (b >= NBAT || l > lmax) return 0.0;
    if (DEF && cc >= C.n1 - C.nP) {
        if (!batch.P[b]) return 0.0;
        const double2 a = batch.P[b][base + l];
        return (cc & 1) ? a.y : a.x;
    }
    const double L = (double)l * (double)(l + 1);
    if (cc < C.nT) {
        const double2 a = batch.T[b][base + l];
        double w = 1.0;
        for (int t = 0; t < (cc >> 1); ++t) w *= L;
        return w * ((cc & 1) ? a.y : a.x);
    }
    if (!POL || l < 2) return 0.0;
    const double nl = 1.0 / sqrt((double)(l - 1) * l * (double)(l + 1) * (double)(l + 2));
    int q = cc - C.nT;
    const double2 *src = batch.E[b];
    if (HASB && q >= C.nE) {
        q -= C.nE;
        src = batch.B[b];
    }
    const double2 a = src[base + l];
    double w = nl;
    for (int t = 0; t < (q >> 1); ++t) w *= L;
    return w * ((q & 1) ? a.y : a.x);
}

// Wave-local ordering of LDS accesses (each wave owns its region).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace lp
}  // namespace tl
