// In-place FP64 complex transforms of up to 8192 points in LDS for one
// workgroup of 512 threads (the theta-derivative FFTs along great circles
// and the forward ring transforms of the analysis).
#pragma once
#include "tl_internal.h"

namespace tl {
namespace {

constexpr int kTfThreads = 512;

__device__ inline int bitrev(int t, int lg) { return (int)(__brev((unsigned)t) >> (32 - lg)); }

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// r consecutive radix-2 decimation-in-time stages s .. s + r - 1 of an
// in-place transform, in registers: with half = 2^(s-1), block b holds the
// 2^r elements base + pos + t half (pos = b mod half), which those stages
// combine only among themselves; stage s + q pairs t with t + 2^q (t mod
// 2^(q+1) < 2^q) under the twiddle W_{2^(s+q)}^(pos + (t mod 2^q) half).
// The twiddle e^{-2 pi i e / P}, e < P / 2, is th[e / 64] tl[e % 64] from
// two tables in LDS; inverse: conjugate twiddles (no 1/P).  Ends with a
// barrier.
constexpr int kTwLo = 64;
constexpr int kTwHi = kThetaFftMaxP / 2 / kTwLo;

__device__ inline double2 twiddle(const double2 *th, const double2 *tl, int e)
{
    return cmul(th[e / kTwLo], tl[e % kTwLo]);
}

template <int r>
__device__ void fft_stages(double2 *x, int P, int s, const double2 *th, const double2 *tl, bool inverse)
{
    constexpr int R = 1 << r;
    const int half = 1 << (s - 1);
    for (int b = threadIdx.x; b < P / R; b += kTfThreads) {
        const int pos = b & (half - 1);
        double2 *xb = x + (b >> (s - 1)) * (R * half) + pos;
        double2 v[R];
#pragma unroll
        for (int t = 0; t < R; ++t) v[t] = xb[t * half];
#pragma unroll
        for (int q = 0; q < r; ++q) {
            const int hq = 1 << q;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if ((t & (2 * hq - 1)) < hq) {
                    double2 w = twiddle(th, tl, (pos + (t & (hq - 1)) * half) * (P >> (s + q)));
                    if (inverse) w.y = -w.y;
                    const double2 a = v[t], c = cmul(w, v[t + hq]);
                    v[t] = make_double2(a.x + c.x, a.y + c.y);
                    v[t + hq] = make_double2(a.x - c.x, a.y - c.y);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t) xb[t * half] = v[t];
    }
    __syncthreads();
}

// In-place transform of x[0..P) stored in bit-reversed order: the lg
// radix-2 stages three at a time (radix 8), the rest two or one at a time.
__device__ void lds_fft(double2 *x, int P, int lg, const double2 *th, const double2 *tl, bool inverse)
{
    int s = 1;
    for (; s + 2 <= lg; s += 3) fft_stages<3>(x, P, s, th, tl, inverse);
    if (s + 1 == lg) fft_stages<2>(x, P, s, th, tl, inverse);
    else if (s == lg) fft_stages<1>(x, P, s, th, tl, inverse);
}

// The LDS twiddle tables th (64 entries) and tl (64 entries) from a global
// table: e^{-2 pi i e / P} = tw[e] (conj = false) or conj(tw[e]) (conj =
// true, for a table of e^{+2 pi i e / P}), e < P / 2.  No barrier.
__device__ inline void load_twiddles(double2 *th, double2 *tl, const double2 *__restrict__ tw, int P, bool conj)
{
    for (int i = threadIdx.x; i < kTwHi + kTwLo; i += kTfThreads) {
        double2 v;
        bool ok;
        if (i < kTwHi) {
            ok = i * kTwLo < P / 2;
            if (ok) v = tw[i * kTwLo];
        } else {
            ok = i - kTwHi < P / 2;
            if (ok) v = tw[i - kTwHi];
        }
        if (ok) {
            if (conj) v.y = -v.y;
            (i < kTwHi ? th[i] : tl[i - kTwHi]) = v;
        }
    }
}

}  // namespace
}  // namespace tl
