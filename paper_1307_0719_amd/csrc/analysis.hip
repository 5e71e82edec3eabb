// Analysis of a temperature map on the equal-theta grid: the spherical-
// harmonic coefficients whose power spectra measure the accuracy of the
// lensed maps (Sec. III.A-B),
//   a_lm = sum_i w_i lambda_lm(theta_i) (2 pi / nphi) sum_k T(theta_i, phi_k) e^{-i m phi_k},
// w_i the Clenshaw-Curtis weights of the rings (exact for polynomials in
// cos theta of degree <= ntheta - 1).
//
// k_ring_analysis: one workgroup per pair of rings, both rings as the real
// and imaginary parts of one FP64 transform in LDS (rows read coalesced),
// the two spectra separated from X_m and conj X_{P-m}; the ring weights
// summed by the workgroup; G[ring][m] = (2 pi / P) w_i X_m.
// k_analysis_lm: one wave per (m, 64 ring pairs), a lane per ring pair
// (north and south ring share lambda up to (-1)^(l+m)); the normalized
// Legendre recursion over l in FP64 with a power-of-two scale for the start
// value sin^m theta (which underflows near the poles at high m); the sum
// over the wave's ring pairs by a butterfly of lane shuffles, kept by lane
// (l - m) mod 64 and added to a_lm atomically per 64 multipoles.
#include "lds_fft.h"

namespace tl {
namespace {

constexpr int kAnaWaves = 4;

__global__ __launch_bounds__(kTfThreads) void k_ring_analysis(const double *__restrict__ map,
                                                              double2 *__restrict__ G,
                                                              const double2 *__restrict__ twid, int ntheta, int P,
                                                              int lg, int lmax)
{
    extern __shared__ unsigned char smem_raw[];
    double2 *x = reinterpret_cast<double2 *>(smem_raw);
    double2 *th = x + P;
    double2 *tl = th + kTwHi;
    double *red = reinterpret_cast<double *>(tl + kTwLo);  // [2][kTfThreads]
    const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
    const bool two = r1 < ntheta;
    load_twiddles(th, tl, twid, P, true);
    for (int t = threadIdx.x; t < P; t += kTfThreads) {
        const double a = map[(size_t)r0 * P + t];
        const double b = two ? map[(size_t)r1 * P + t] : 0.0;
        x[bitrev(t, lg)] = make_double2(a, b);
    }
    // Clenshaw-Curtis weights: w_i = c_i (1 - sum_{j=1}^{N/2} b_j cos(2 pi i j / N) / (4 j^2 - 1)) / N
    const int N = ntheta - 1;
    double s0 = 0.0, s1 = 0.0;
    for (int j = threadIdx.x + 1; j <= N / 2; j += kTfThreads) {
        const double f = (2 * j == N ? 1.0 : 2.0) / (4.0 * (double)j * (double)j - 1.0);
        s0 += f * cospi(2.0 * (double)((int64_t)r0 * j % N) / (double)N);
        if (two) s1 += f * cospi(2.0 * (double)((int64_t)r1 * j % N) / (double)N);
    }
    red[threadIdx.x] = s0;
    red[kTfThreads + threadIdx.x] = s1;
    __syncthreads();
    for (int o = kTfThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[threadIdx.x] += red[threadIdx.x + o];
            red[kTfThreads + threadIdx.x] += red[kTfThreads + threadIdx.x + o];
        }
        __syncthreads();
    }
    lds_fft(x, P, lg, th, tl, false);
    const double dphi = 2.0 * M_PI / (double)P;
    const double w0 = (r0 == 0 || r0 == N ? 1.0 : 2.0) * (1.0 - red[0]) / (double)N;
    const double w1 = (r1 == N ? 1.0 : 2.0) * (1.0 - red[kTfThreads]) / (double)N;
    const double g0 = 0.5 * w0 * dphi, g1 = 0.5 * w1 * dphi;
    for (int m = threadIdx.x; m <= lmax; m += kTfThreads) {
        const double2 X = x[m];
        const double2 Y = x[(P - m) & (P - 1)];
        // ring r0: (X_m + conj Y) / 2; ring r1: (X_m - conj Y) / (2 i)
        G[(size_t)r0 * (lmax + 1) + m] = make_double2(g0 * (X.x + Y.x), g0 * (X.y - Y.y));
        if (two) G[(size_t)r1 * (lmax + 1) + m] = make_double2(g1 * (X.y + Y.y), -g1 * (X.x - Y.x));
    }
}

// norm[m] = (-1)^m sqrt((2m + 1) / (4 pi) prod_{k=1}^{m} (2k - 1) / (2k)): lambda_mm / sin^m
__global__ void k_lm_norm(double *__restrict__ norm, int lmax)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m > lmax) return;
    double p = 1.0;
    for (int k = 1; k <= m; ++k) p *= (double)(2 * k - 1) / (double)(2 * k);
    const double v = sqrt((2.0 * m + 1.0) / (4.0 * M_PI) * p);
    norm[m] = (m & 1) ? -v : v;
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(64 * kAnaWaves) void k_analysis_lm(const double2 *__restrict__ G,
                                                               const double *__restrict__ norm,
                                                               double *__restrict__ alm, int lmax, int ntheta,
                                                               int nrp)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = kAnaWaves * blockIdx.y + wave;
    if (m > lmax) return;  // whole waves only
    const int r = blockIdx.x * 64 + lane;
    double sn = 1.0, cs = 0.0;
    double2 ge = make_double2(0.0, 0.0), go = ge;
    if (r < nrp) {
        sincospi((double)r / (double)(ntheta - 1), &sn, &cs);
        const int rs = ntheta - 1 - r;
        const double2 gn = G[(size_t)r * (lmax + 1) + m];
        const double2 gs = rs != r ? G[(size_t)rs * (lmax + 1) + m] : make_double2(0.0, 0.0);
        ge = make_double2(gn.x + gs.x, gn.y + gs.y);
        go = make_double2(gn.x - gs.x, gn.y - gs.y);
    }
    // lambda_mm = norm[m] sin^m theta held as p1 2^E
    double p1 = norm[m], p2 = 0.0;
    int E = 0;
    for (int k = 0; k < m; ++k) {
        p1 *= sn;
        if (fabs(p1) < 0x1p-300) {
            p1 *= 0x1p300;
            E -= 300;
        }
    }
    const size_t row = (size_t)m * (2 * lmax + 1 - m) / 2;
    double2 keep = make_double2(0.0, 0.0);
    const double m2 = (double)m * (double)m;
    for (int l = m; l <= lmax; ++l) {
        if (l > m) {
            const double dl = (double)l;
            const double a = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - m2));
            const double b = sqrt(((dl - 1.0) * (dl - 1.0) - m2) / (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
            const double v = a * (cs * p1 - b * p2);
            p2 = p1;
            p1 = v;
            if (E < 0 && fabs(p1) > 0x1p300) {
                p1 *= 0x1p-300;
                p2 *= 0x1p-300;
                E += 300;
            }
        }
        const double lam = E == 0 ? p1 : ldexp(p1, E);
        const double2 g = ((l + m) & 1) ? go : ge;
        const double sx = wave_sum(lam * g.x);
        const double sy = wave_sum(lam * g.y);
        const int slot = (l - m) & 63;
        if (lane == slot) keep = make_double2(sx, sy);
        if (slot == 63 || l == lmax) {
            const int l0 = l - slot;
            if (lane <= slot) {
                double *dst = alm + 2 * (row + (size_t)(l0 + lane));
                atomicAdd(dst, keep.x);
                atomicAdd(dst + 1, keep.y);
            }
            keep = make_double2(0.0, 0.0);
        }
    }
}

}  // namespace

bool analysis_grid(int nphi) { return nphi >= 2 && nphi <= kThetaFftMaxP && (nphi & (nphi - 1)) == 0; }

size_t analysis_scratch_bytes(const Plan &p) { return (size_t)p.ntheta * (p.lmax + 1) * sizeof(double2); }

hipError_t launch_analysis_T(Plan &p, const double *map, void *alm)
{
    const int P = p.nphi;
    int lg = 0;
    while ((1 << lg) < P) ++lg;
    double2 *G = (double2 *)p.F.ptr;
    // the start-value norms in the deflection buffer (2 npix >= lmax + 1 values)
    double *norm = (double *)p.alpha.ptr;
    const size_t nalm = (size_t)(p.lmax + 1) * (p.lmax + 2) / 2;
    hipError_t e = hipMemsetAsync(alm, 0, nalm * sizeof(double2), p.stream);
    if (e != hipSuccess) return e;
    const size_t smem = (size_t)(P + kTwHi + kTwLo) * sizeof(double2) + 2 * kTfThreads * sizeof(double);
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ring_analysis),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ring_analysis, dim3((p.ntheta + 1) / 2), dim3(kTfThreads), smem, p.stream, map, G,
                       (const double2 *)p.twid64.ptr, p.ntheta, P, lg, p.lmax);
    hipLaunchKernelGGL(k_lm_norm, dim3((p.lmax + 1 + 255) / 256), dim3(256), 0, p.stream, norm, p.lmax);
    hipLaunchKernelGGL(k_analysis_lm, dim3((p.nrp + 63) / 64, (p.lmax + kAnaWaves) / kAnaWaves),
                       dim3(64 * kAnaWaves), 0, p.stream, (const double2 *)G, (const double *)norm, (double *)alm,
                       p.lmax, p.ntheta, p.nrp);
    return hipGetLastError();
}

}  // namespace tl
