// Theta-derivatives of maps on the equal-theta grid by FFT (the FFT route
// that the conclusion, Sec. IV, says the equirectangular pixelization opens):
// the samples of one meridian (ring i, column c) and of its opposite
// meridian (column c + nphi/2, read from the south pole back up) lie on one
// great circle through both poles, P = 2 (ntheta - 1) equally spaced points
// of it.  Along that circle T, and Q and U in the (e_theta, e_phi) basis
// (both basis vectors change sign across a pole, so the quadratic Q, U do
// not), are trigonometric polynomials of degree <= lmax in the circle angle,
// so for lmax < P / 2 the derivative d^j/dtheta^j is exact from the circle's
// DFT: multiply coefficient kappa by (i kappa)^j.  On the opposite meridian
// theta runs against the circle angle, which flips odd derivatives.
//
// One workgroup takes two circles (columns c, c + 1 and their opposites) as
// the real and imaginary parts of one complex transform in LDS (FP64, P <=
// 8192: 128 KiB; radix-8 steps, a barrier per three stages; twiddles as
// products of two 64-entry tables in LDS), keeps the
// spectrum in registers and runs one inverse transform per derivative
// order.  Workgroups are ordered so that each XCD
// takes a contiguous range of columns: the strided column loads of
// neighbouring workgroups then share the lines in that XCD's L2.
#include "lds_fft.h"

namespace tl {
namespace {

constexpr int kTfReg = kThetaFftMaxP / kTfThreads;  // spectrum entries per thread

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// Map i of the launch: input in + i istride, output of order j at
// out + i ostride + slot(j) pstride, slot(j) = sa j - sb j (j - 1) / 2 + sc,
// = dtheta^j / j! d^j/dtheta^j of the input, j = 1..jmax; every map is
// [nr][nphi].  Grid: (nphi / 4 rounded up) * nmaps workgroups, linear order.
template <typename T>
__global__ __launch_bounds__(kTfThreads) void k_theta_fft(const T *__restrict__ in, T *__restrict__ out,
                                                          const double2 *__restrict__ tw, int P, int lg, int nphi,
                                                          int npair, int nmaps, int jmax, ThetaFftLayout lay)
{
    using V = typename Vec2<T>::type;
    extern __shared__ unsigned char smem_raw[];
    double2 *x = reinterpret_cast<double2 *>(smem_raw);
    double2 *th = x + P;       // tw[64 a], a < P / 128 (at least one)
    double2 *tl = th + kTwHi;  // tw[b], b < min(64, P / 2)
    load_twiddles(th, tl, tw, P, false);

    // XCD-contiguous order: XCD w % 8 takes a contiguous run of the
    // (map, circle pair) items
    const int total = npair * nmaps;
    const int w = blockIdx.x;
    const int xcd = w & 7, base = total >> 3, rem = total & 7;
    const int item = xcd * base + min(xcd, rem) + (w >> 3);
    const int map = item / npair;
    const int c0 = 2 * (item - map * npair);
    const int hp = nphi / 2;
    const bool two = c0 + 1 < hp;
    const int nr = P / 2 + 1;
    const T *src = in + (size_t)map * lay.istride;

    // all loads of a thread in flight before the first LDS store
    V ld[kTfReg];
#pragma unroll
    for (int r = 0; r < kTfReg; ++r) {
        const int t = threadIdx.x + r * kTfThreads;
        if (t < P) {
            const bool north = t <= P / 2;
            const T *q = src + (size_t)(north ? t : P - t) * nphi + (north ? c0 : c0 + hp);
            if (two) {
                ld[r] = *reinterpret_cast<const V *>(q);
            } else {
                ld[r].x = q[0];
                ld[r].y = (T)0;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kTfReg; ++r) {
        const int t = threadIdx.x + r * kTfThreads;
        if (t < P) x[bitrev(t, lg)] = make_double2((double)ld[r].x, (double)ld[r].y);
    }
    __syncthreads();
    lds_fft(x, P, lg, th, tl, false);

    double2 X[kTfReg];
#pragma unroll
    for (int r = 0; r < kTfReg; ++r) {
        const int k = threadIdx.x + r * kTfThreads;
        X[r] = k < P ? x[k] : make_double2(0.0, 0.0);
    }

    const double dth = 2.0 * M_PI / (double)P;  // circle spacing = ring spacing
    double fact = 1.0;
    for (int j = 1; j <= jmax; ++j) {
        fact *= (double)j;
        __syncthreads();  // every read of the previous inverse is done
#pragma unroll
        for (int r = 0; r < kTfReg; ++r) {
            const int k = threadIdx.x + r * kTfThreads;
            if (k < P) {
                const int kap = k <= P / 2 ? k : k - P;
                const double u = (double)kap * dth;
                double mag = 1.0;
                for (int e = 0; e < j; ++e) mag *= u;
                mag /= fact * (double)P;
                // the Nyquist term's odd derivatives are not sampled
                if (2 * k == P && (j & 1)) mag = 0.0;
                const double2 v = X[r];
                double2 y;
                switch (j & 3) {  // (i)^j mag
                case 0: y = make_double2(mag * v.x, mag * v.y); break;
                case 1: y = make_double2(-mag * v.y, mag * v.x); break;
                case 2: y = make_double2(-mag * v.x, -mag * v.y); break;
                default: y = make_double2(mag * v.y, -mag * v.x); break;
                }
                x[bitrev(k, lg)] = y;
            }
        }
        __syncthreads();
        lds_fft(x, P, lg, th, tl, true);

        T *dst = out + (size_t)map * lay.ostride + (size_t)(lay.sa * j - lay.sb * j * (j - 1) / 2 + lay.sc) * lay.pstride;
        const double sg = (j & 1) ? -1.0 : 1.0;
        for (int t = threadIdx.x; t < nr; t += kTfThreads) {
            const double2 a = x[t];
            const double2 b = x[t == 0 ? 0 : P - t];
            T *qa = dst + (size_t)t * nphi + c0;
            T *qb = qa + hp;
            if (two) {
                V va, vb;
                va.x = (T)a.x;
                va.y = (T)a.y;
                vb.x = (T)(sg * b.x);
                vb.y = (T)(sg * b.y);
                *reinterpret_cast<V *>(qa) = va;
                *reinterpret_cast<V *>(qb) = vb;
            } else {
                qa[0] = (T)a.x;
                qb[0] = (T)(sg * b.x);
            }
        }
    }
}

}  // namespace

bool theta_fft_grid(int ntheta)
{
    const int h = ntheta - 1;
    return h >= 2 && h <= kThetaFftMaxP / 2 && (h & (h - 1)) == 0;
}

hipError_t launch_theta_fft(Plan &p, const void *in, void *out, int nmaps, int jmax, const ThetaFftLayout &lay)
{
    const int P = 2 * (p.ntheta - 1);
    int lg = 0;
    while ((1 << lg) < P) ++lg;
    const int npair = (p.nphi / 2 + 1) / 2;
    const int64_t nwg = (int64_t)npair * nmaps;
    const size_t smem = (size_t)(P + kTwHi + kTwLo) * sizeof(double2);
    hipError_t e;
    if (p.fp64()) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_theta_fft<double>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        k_theta_fft<double><<<dim3((unsigned)nwg), dim3(kTfThreads), smem, p.stream>>>(
            (const double *)in, (double *)out, (const double2 *)p.twT.ptr, P, lg, p.nphi, npair, nmaps, jmax, lay);
    } else {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_theta_fft<float>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        k_theta_fft<float><<<dim3((unsigned)nwg), dim3(kTfThreads), smem, p.stream>>>(
            (const float *)in, (float *)out, (const double2 *)p.twT.ptr, P, lg, p.nphi, npair, nmaps, jmax, lay);
    }
    return hipGetLastError();
}

}  // namespace tl
