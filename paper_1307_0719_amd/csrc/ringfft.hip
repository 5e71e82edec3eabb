// Ring FFT stage: per-m theta-derivative coefficients -> derivative maps.
//
// Each workgroup takes one job = one row of Fourier coefficients F_m
// (m = 0..L, complex) of one ring, and produces up to kMaxJobK real rings
//     out[n] = scale * sum_{m=-L}^{L} (i m)^k F_m e^{i m phi_n},  phi_n = 2 pi n / N,
// with F_{-m} = conj(F_m).  These are the phi-derivatives d^k_phi of the
// theta-derivative maps (the derivative inputs of eq. 5 of the paper); the
// (i m)^k factor is applied in Fourier space while the row is loaded.
//
// Real output from a Hermitian half spectrum: with X_0 = Re c_0,
// X_m = c_m (0 < m < N/2), X_{N/2} = 2 Re c_{N/2} (present iff L = N/2, the
// alias of +-N/2 at the pixel centres), M = N/2 and
//     Z_m = (X_m + conj X_{M-m}) + i e^{2 pi i m/N} (X_m - conj X_{M-m}),
// the length-M inverse DFT z = IDFT_M(Z) gives out[2n] = Re z_n, out[2n+1] = Im z_n.
// The length-M transform is a Stockham autosort FFT in LDS (ping-pong
// buffers, radices 8, 4, 2, 5, 3), twiddles from a table e^{2 pi i t/N}.
#include <hip/hip_fp16.h>

#include "tl_internal.h"

namespace tl {

namespace {

template <typename R>
struct C2;
template <>
struct C2<float> {
    using T = float2;
};
template <>
struct C2<double> {
    using T = double2;
};

template <typename V>
__device__ __forceinline__ V cmk(decltype(V().x) a, decltype(V().x) b)
{
    V v;
    v.x = a;
    v.y = b;
    return v;
}
template <typename V>
__device__ __forceinline__ V cadd(V a, V b) { return cmk<V>(a.x + b.x, a.y + b.y); }
template <typename V>
__device__ __forceinline__ V csub(V a, V b) { return cmk<V>(a.x - b.x, a.y - b.y); }
template <typename V>
__device__ __forceinline__ V cmul(V a, V b) { return cmk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <typename V>
__device__ __forceinline__ V cmuli(V a) { return cmk<V>(-a.y, a.x); }   // i a
template <typename V>
__device__ __forceinline__ V cconj(V a) { return cmk<V>(a.x, -a.y); }

// Store of one complex output: as it is, or rounded to FP16 (the mixed maps).
// Non-temporal: the maps are written once and read by the next kernel
// (measured 3 % faster ring FFTs than plain stores; non-temporal loads in the
// remap were slower).
template <typename V>
__device__ __forceinline__ void put(V *o, size_t i, V v)
{
    __builtin_nontemporal_store(v.x, &o[i].x);
    __builtin_nontemporal_store(v.y, &o[i].y);
}
template <typename V>
__device__ __forceinline__ void put(__half2 *o, size_t i, V v)
{
    const __half2 h = __floats2half2_rn((float)v.x, (float)v.y);
    __builtin_nontemporal_store(*reinterpret_cast<const unsigned *>(&h), reinterpret_cast<unsigned *>(&o[i]));
}

// Output q of a job: FP32/FP64 ring in Dbase, or (bit q of h16, FP32 kernels)
// an FP16 ring in D16.
template <typename R, typename F>
__device__ __forceinline__ void with_out(const FftJob &job, int q, R *Dbase, __half *D16, F &&f)
{
    if constexpr (sizeof(R) == 4) {
        if ((job.h16 >> q) & 1) {
            f(reinterpret_cast<__half2 *>(D16 + job.dst[q]));
            return;
        }
    }
    f(reinterpret_cast<typename C2<R>::T *>(Dbase + job.dst[q]));
}

// In-register inverse DFT of size r (sign +): y_s = sum_q v_q e^{+2 pi i q s / r}.
template <typename V>
__device__ __forceinline__ void dft2(V *v)
{
    V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}
template <typename V>
__device__ __forceinline__ void dft4(V *v)
{
    V a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    V b0 = cadd(v[1], v[3]), b1 = cmuli(csub(v[1], v[3]));
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
}
template <typename V>
__device__ __forceinline__ void dft8(V *v)
{
    using R = decltype(V().x);
    const R h = (R)0.70710678118654752440084436210484904;
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    dft4(e);
    dft4(o);
    // o_s *= e^{2 pi i s / 8}
    o[1] = cmk<V>(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y));
    o[2] = cmuli(o[2]);
    o[3] = cmk<V>(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y));
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        v[s] = cadd(e[s], o[s]);
        v[s + 4] = csub(e[s], o[s]);
    }
}
template <typename V>
__device__ __forceinline__ void dft3(V *v)
{
    using R = decltype(V().x);
    const R c = (R)-0.5, s = (R)0.86602540378443864676372317075293618;
    V t = cadd(v[1], v[2]);
    V d = csub(v[1], v[2]);
    V y0 = cadd(v[0], t);
    V m1 = cmk<V>(v[0].x + c * t.x, v[0].y + c * t.y);
    V m2 = cmk<V>(-s * d.y, s * d.x);  // i s d
    v[0] = y0;
    v[1] = cadd(m1, m2);
    v[2] = csub(m1, m2);
}
template <typename V>
__device__ __forceinline__ void dft5(V *v)
{
    using R = decltype(V().x);
    const R c1 = (R)0.30901699437494742410229341718281906;   // cos 2pi/5
    const R c2 = (R)-0.80901699437494742410229341718281906;  // cos 4pi/5
    const R s1 = (R)0.95105651629515357211643933337938214;   // sin 2pi/5
    const R s2 = (R)0.58778525229247312916870595463907277;   // sin 4pi/5
    V t1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
    V t2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
    V y0 = cadd(v[0], cadd(t1, t2));
    V a1 = cmk<V>(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    V a2 = cmk<V>(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    // b1 = i (s1 d1 + s2 d2), b2 = i (s2 d1 - s1 d2)
    V q1 = cmk<V>(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
    V q2 = cmk<V>(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
    V b1 = cmuli(q1), b2 = cmuli(q2);
    v[0] = y0;
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
}

// One radix-RX Stockham pass (inverse): for every butterfly b < M/RX,
// v_s = src[b + s M/RX] e^{2 pi i (b mod Ns) s / (Ns RX)}, v = IDFT_RX(v),
// dst[(b / Ns) Ns RX + b mod Ns + s Ns] = v_s.
template <int RX, typename V>
__device__ __forceinline__ void stockham_pass(const V *__restrict__ src, V *__restrict__ dst, int M, int Ns, int N,
                                              int tid, int T, const V *__restrict__ twN)
{
    const int nb = M / RX;
    const int tstride = N / (Ns * RX);
    for (int b = tid; b < nb; b += T) {
        V v[RX];
        const int kk = b % Ns;
#pragma unroll
        for (int s = 0; s < RX; ++s) {
            V x = src[b + s * nb];
            if (s > 0 && kk > 0) x = cmul(x, twN[kk * s * tstride]);
            v[s] = x;
        }
        if constexpr (RX == 2) dft2(v);
        else if constexpr (RX == 3) dft3(v);
        else if constexpr (RX == 4) dft4(v);
        else if constexpr (RX == 5) dft5(v);
        else dft8(v);
        const int base = (b / Ns) * Ns * RX + kk;
#pragma unroll
        for (int s = 0; s < RX; ++s) dst[base + s * Ns] = v[s];
    }
}

struct Radices {
    int n;
    int r[16];
};

template <typename R>
__global__ __launch_bounds__(256) void k_ring_fft(const FftJob *__restrict__ jobs,
                                                  const typename C2<R>::T *__restrict__ Fbase,
                                                  R *__restrict__ Dbase, __half *__restrict__ D16, int lmax, int M,
                                                  const typename C2<R>::T *__restrict__ twN, Radices rad)
{
    using V = typename C2<R>::T;
    extern __shared__ unsigned char smem_raw[];
    V *bufA = reinterpret_cast<V *>(smem_raw);
    V *bufB = bufA + M;
    const int tid = threadIdx.x;
    const int T = blockDim.x;
    const FftJob &job = jobs[blockIdx.x];
    const V *F = Fbase + job.src;
    const int N = 2 * M;
    const int L = lmax;

    for (int q = 0; q < job.nk; ++q) {
        const int k = job.k[q];
        const double scale = job.scale[q];
        // X(m) = scale (i m)^k F_m for 0 < m < M (0 beyond L); X(0), X(M) real.
        auto coefX = [&](int m) -> V {
            if (m > L) return cmk<V>(0, 0);
            const V f = F[m];
            double mk = 1.0;
            for (int t = 0; t < k; ++t) mk *= (double)m;
            const double s = scale * mk;
            double re = s * (double)f.x, im = s * (double)f.y;
            // multiply by i^k
            switch (k & 3) {
            case 1: { double t2 = re; re = -im; im = t2; } break;
            case 2: re = -re; im = -im; break;
            case 3: { double t2 = re; re = im; im = -t2; } break;
            default: break;
            }
            if (m == 0) return cmk<V>((R)re, 0);
            if (m == M) return cmk<V>((R)(2.0 * re), 0);
            return cmk<V>((R)re, (R)im);
        };
        for (int m = tid; m < M; m += T) {
            const V xm = coefX(m);
            const V xc = cconj(coefX(M - m));
            const V sum = cadd(xm, xc);
            const V dif = csub(xm, xc);
            const V tw = twN[m];  // e^{2 pi i m / N}
            bufA[m] = cadd(sum, cmuli(cmul(tw, dif)));
        }
        __syncthreads();
        // Stockham passes (inverse transform)
        V *src = bufA, *dst = bufB;
        int Ns = 1;
        for (int p = 0; p < rad.n; ++p) {
            const int r = rad.r[p];
            switch (r) {
            case 2: stockham_pass<2, V>(src, dst, M, Ns, N, tid, T, twN); break;
            case 3: stockham_pass<3, V>(src, dst, M, Ns, N, tid, T, twN); break;
            case 4: stockham_pass<4, V>(src, dst, M, Ns, N, tid, T, twN); break;
            case 5: stockham_pass<5, V>(src, dst, M, Ns, N, tid, T, twN); break;
            default: stockham_pass<8, V>(src, dst, M, Ns, N, tid, T, twN); break;
            }
            __syncthreads();
            V *t = src;
            src = dst;
            dst = t;
            Ns *= r;
        }
        with_out<R>(job, q, Dbase, D16, [&](auto *out) {
            for (int n = tid; n < M; n += T) put(out, n, src[n]);
        });
        __syncthreads();
    }
}

// ---- HEALPix rings: ring-dependent length and phase ----
//
// Ring r of a HEALPix grid has N = nphi_r pixels at phi_n = phi0_r + 2 pi n / N,
// and lmax may exceed N / 2 (the polar rings hold 4, 8, ... pixels), so the
// coefficients fold onto the N frequencies of the ring:
//     X_q = e^{i q phi0} sum_{m = q mod N, |m| <= lmax} sigma^{(m - q) / N} c_m,
// c_m = scale (i m)^k F_m, c_{-m} = conj c_m, c_0 = Re c_0, sigma = e^{i N phi0}
// = +-1.  X is Hermitian, so the half-length transform above applies (M = N/2),
// with a Stockham FFT over the radices of M = 2 i, any i: passes of radix 2, 3,
// 4, 5, 8 as above, other primes p by a direct p-point sum per output (M p
// operations per pass).  Twiddles e^{2 pi i t / N} of every length N = 4 i,
// i = 1..nside, at offset 2 i (i - 1) of one table.

// One Stockham pass of any radix RX, one output per thread and step.
template <typename V>
__device__ __forceinline__ void stockham_any(const V *__restrict__ src, V *__restrict__ dst, int M, int Ns, int N,
                                             int RX, int tid, int T, const V *__restrict__ twN)
{
    const int nb = M / RX;
    const int tstride = N / (Ns * RX);
    const int np = N / RX;
    for (int idx = tid; idx < M; idx += T) {
        const int b = idx / RX, t = idx - b * RX;
        const int kk = b % Ns;
        // exponent of output t: s (kk tstride + t N / RX) for the input s
        const int step = kk * tstride + t * np;  // < N
        V y = cmk<V>(0, 0);
        int e = 0;
        for (int s2 = 0; s2 < RX; ++s2) {
            y = cadd(y, cmul(src[b + s2 * nb], twN[e]));
            e += step;
            if (e >= N) e -= N;
        }
        dst[(b / Ns) * Ns * RX + kk + t * Ns] = y;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_ring_fft_hpx(const FftJob *__restrict__ jobs,
                                                      const typename C2<R>::T *__restrict__ Fbase,
                                                      R *__restrict__ Dbase, __half *__restrict__ D16, int lmax,
                                                      const HRing *__restrict__ hring,
                                                      const typename C2<R>::T *__restrict__ twAll)
{
    using V = typename C2<R>::T;
    extern __shared__ unsigned char smem_raw[];
    __shared__ int s_rad[24];
    __shared__ int s_nrad;
    const int tid = threadIdx.x, T = blockDim.x;
    const FftJob &job = jobs[blockIdx.x];
    const HRing hr = hring[job.pad];
    const int N = hr.nphi, M = N / 2, L = lmax;
    const int i4 = N / 4;
    const V *twN = twAll + (size_t)2 * i4 * (i4 - 1);
    V *bufA = reinterpret_cast<V *>(smem_raw);  // M entries
    V *bufB = bufA + M;                           // M + 1 entries (X_0 .. X_M)
    const V *F = Fbase + job.src;
    if (tid == 0) {
        // radices of M: 8, 4, 2, 5, 3, then the remaining primes ascending
        int n = M, c = 0;
        const int small[5] = {8, 4, 2, 5, 3};
        for (int a = 0; a < 5; ++a)
            while (n % small[a] == 0 && n > 1) {
                s_rad[c++] = small[a];
                n /= small[a];
            }
        for (int pr = 7; n > 1; pr += 2)
            while (n % pr == 0) {
                s_rad[c++] = pr;
                n /= pr;
            }
        s_nrad = c;
    }
    for (int q = 0; q < job.nk; ++q) {
        const int k = job.k[q];
        const double scale = job.scale[q];
        auto coef = [&](int m) -> double2 {  // scale (i m)^k F_m, m >= 0
            const V f = F[m];
            double mk = 1.0;
            for (int t = 0; t < k; ++t) mk *= (double)m;
            const double s = scale * mk;
            double re = s * (double)f.x, im = m == 0 ? 0.0 : s * (double)f.y;
            switch (k & 3) {
            case 1: { const double t2 = re; re = -im; im = t2; } break;
            case 2: re = -re; im = -im; break;
            case 3: { const double t2 = re; re = im; im = -t2; } break;
            default: break;
            }
            return make_double2(re, im);
        };
        // folded half spectrum X_0 .. X_M
        for (int qq = tid; qq <= M; qq += T) {
            double re = 0.0, im = 0.0, sg = 1.0;
            for (int m = qq; m <= L; m += N, sg *= hr.sigma) {
                const double2 c = coef(m);
                re += sg * c.x;
                im += sg * c.y;
            }
            sg = hr.sigma;
            for (int m = N - qq; m <= L; m += N, sg *= hr.sigma) {  // m = -(t N - qq), t >= 1
                const double2 c = coef(m);
                re += sg * c.x;
                im -= sg * c.y;
            }
            double sn = 0.0, cs = 1.0;  // e^{i qq phi0}, phi0 = pi shift / N
            if (hr.shift) sincospi((double)qq / (double)N, &sn, &cs);
            double xr = re * cs - im * sn, xi = re * sn + im * cs;
            if (qq == 0 || qq == M) xi = 0.0;  // real by Hermitian symmetry
            bufB[qq] = cmk<V>((R)xr, (R)xi);
        }
        __syncthreads();
        for (int m = tid; m < M; m += T) {
            const V xm = bufB[m];
            const V xc = cconj(bufB[M - m]);
            bufA[m] = cadd(cadd(xm, xc), cmuli(cmul(twN[m], csub(xm, xc))));
        }
        __syncthreads();
        V *src = bufA, *dst = bufB;
        int Ns = 1;
        for (int pi = 0; pi < s_nrad; ++pi) {
            const int r = s_rad[pi];
            switch (r) {
            case 2: stockham_pass<2, V>(src, dst, M, Ns, N, tid, T, twN); break;
            case 3: stockham_pass<3, V>(src, dst, M, Ns, N, tid, T, twN); break;
            case 4: stockham_pass<4, V>(src, dst, M, Ns, N, tid, T, twN); break;
            case 5: stockham_pass<5, V>(src, dst, M, Ns, N, tid, T, twN); break;
            case 8: stockham_pass<8, V>(src, dst, M, Ns, N, tid, T, twN); break;
            default: stockham_any<V>(src, dst, M, Ns, N, r, tid, T, twN); break;
            }
            __syncthreads();
            V *t2 = src;
            src = dst;
            dst = t2;
            Ns *= r;
        }
        with_out<R>(job, q, Dbase, D16, [&](auto *out) {
            for (int n = tid; n < M; n += T) put(out, n, src[n]);
        });
        __syncthreads();
    }
}

__global__ void k_fill_words(uint32_t *__restrict__ x, size_t n, uint32_t v)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// FP64 -> FP32 and FP32 -> FP64 copies of n values (grid-stride)
__global__ void k_to_f32(const double *__restrict__ x, float *__restrict__ y, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}
__global__ void k_to_f64(const float *__restrict__ x, double *__restrict__ y, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}


// ---- power-of-two lengths M = 512 .. 4096: radix-16 passes ----
//
// In-register inverse DFT of size 16 as 4 x 4: y[k1 + 4 k2] =
// sum_n2 e^{2 pi i n2 k2/4} [e^{2 pi i n2 k1/16} sum_n1 v[4 n1 + n2] e^{2 pi i n1 k1/4}].
template <typename V>
__device__ __forceinline__ void dft16(V *v)
{
    using R = decltype(V().x);
    V a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        V t[4] = {v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]};
        dft4(t);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = t[k1];
    }
    // e^{2 pi i j/16}, j = n2 k1
    const R c1 = (R)0.92387953251128675612818318939678829, s1 = (R)0.38268343236508977172845998403039887;
    const R h = (R)0.70710678118654752440084436210484904;
    auto tw = [&](V x, int j) -> V {
        switch (j) {
        case 0: return x;
        case 1: return cmul(x, cmk<V>(c1, s1));
        case 2: return cmk<V>(h * (x.x - x.y), h * (x.x + x.y));
        case 3: return cmul(x, cmk<V>(s1, c1));
        case 4: return cmuli(x);
        case 6: return cmk<V>(-h * (x.x + x.y), h * (x.x - x.y));
        case 9: return cmul(x, cmk<V>(-c1, -s1));
        default: return x;
        }
    };
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) a[n2][k1] = tw(a[n2][k1], n2 * k1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        V t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
        dft4(t);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
}

template <int RX, typename V>
__device__ __forceinline__ void dftR(V *v)
{
    if constexpr (RX == 2) dft2(v);
    else if constexpr (RX == 4) dft4(v);
    else if constexpr (RX == 8) dft8(v);
    else dft16(v);
}

// LDS index with one pad slot per 32 entries (breaks the power-of-two
// strides of the butterfly stores across banks).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }

// Multiply v[s] by e^{2 pi i kk s / (Ns RX)}, s = 1..RX-1: w = e^{2 pi i kk/(Ns RX)}
// and w^4 from the table, w^s as a product of at most three of w, w^2, w^3,
// w^4, w^8 (one rounding per product).
template <int RX, typename V>
__device__ __forceinline__ void apply_twiddles(V (&v)[RX], const V *__restrict__ twN, int kk, int tstride)
{
    const V w1 = twN[kk * tstride];
    const V w2 = cmul(w1, w1);
    const V w3 = cmul(w2, w1);
    V w4 = w2, w8 = w2;
    if constexpr (RX >= 8) w4 = twN[4 * kk * tstride];
    if constexpr (RX >= 16) w8 = cmul(w4, w4);
#pragma unroll
    for (int s = 1; s < RX; ++s) {
        const int lo = s & 3, b4 = (s >> 2) & 1, b8 = s >> 3;
        V w = lo == 1 ? w1 : (lo == 2 ? w2 : w3);
        if (lo == 0) w = b4 ? w4 : w8;
        else {
            if (b4) w = cmul(w, w4);
            if (b8) w = cmul(w, w8);
        }
        if (lo == 0 && b4 && b8) w = cmul(w4, w8);
        v[s] = cmul(v[s], w);
    }
}

// One in-place Stockham pass (radix RX, stride Ns, powers of two) over the
// padded LDS buffer: butterfly b, kk = b mod Ns reads buf[b + s M/RX], applies
// e^{2 pi i kk s/(Ns RX)}, transforms, and writes position
// (b / Ns) Ns RX + kk + s Ns -- into buf, or into the output ring.
template <int M, int RX, int Ns, bool TO_GLOBAL, typename V, typename O>
__device__ __forceinline__ void pass_p2(V *__restrict__ buf, O *__restrict__ out, int tid,
                                        const V *__restrict__ twN)
{
    constexpr int nb = M / RX;
    constexpr int N = 2 * M;
    constexpr int tstride = N / (Ns * RX);
    static_assert(nb <= 256, "one butterfly per thread");
    const bool act = tid < nb;
    const int b = act ? tid : 0;
    V v[RX];
#pragma unroll
    for (int s = 0; s < RX; ++s) v[s] = buf[lpad(b + s * nb)];
    if (!TO_GLOBAL) __syncthreads();  // every read before the in-place writes
    if (act) {
        const int kk = b & (Ns - 1);
        if constexpr (Ns > 1) apply_twiddles<RX>(v, twN, kk, tstride);
        dftR<RX>(v);
        const int base = (b / Ns) * Ns * RX + kk;
#pragma unroll
        for (int s = 0; s < RX; ++s) {
            if constexpr (TO_GLOBAL) put(out, base + s * Ns, v[s]);
            else buf[lpad(base + s * Ns)] = v[s];
        }
    }
}

// X(m) = scale (i m)^K F_m for 0 < m < M, X(0) = Re, X(M) = 2 Re, zero past
// the row end L (f holds F at the clamped index), for the phi-derivative order
// K, a compile-time constant.
template <int K, int M, typename R, typename V>
__device__ __forceinline__ V coef_x(V f, int m, int L, R scale)
{
    R sc = m <= L ? scale : (R)0;
    const R mf = (R)m;
#pragma unroll
    for (int t = 0; t < K; ++t) sc *= mf;
    R re = sc * f.x, im = sc * f.y;
    if constexpr ((K & 3) == 1) { const R t2 = re; re = -im; im = t2; }
    else if constexpr ((K & 3) == 2) { re = -re; im = -im; }
    else if constexpr ((K & 3) == 3) { const R t2 = re; re = im; im = -t2; }
    im = (m == 0 || m == M) ? (R)0 : im;
    re = (m == M) ? (R)2 * re : re;
    return cmk<V>(re, im);
}

// The row values a thread needs: F at m = t + 256 s and at M - m for s < RL/2
// (clamped to the row end), and F_{M/2}.
template <int M, typename V>
__device__ __forceinline__ void load_pairs(V (&f)[M / 256], V &fmid, const V *__restrict__ F, int L, int tid)
{
    constexpr int H = M / 512;
#pragma unroll
    for (int s = 0; s < H; ++s) {
        const int m = tid + 256 * s, mr = M - m;
        f[s] = F[m <= L ? m : L];
        f[H + s] = F[mr <= L ? mr : L];
    }
    fmid = F[M / 2 <= L ? M / 2 : L];
}

// Z(m) = (X(m) + conj X(M-m)) + i w^m (X(m) - conj X(M-m)), w = e^{2 pi i/N}:
// the thread of m < M/2 also writes Z(M - m) (from the same two coefficients,
// with w^{M-m} = -conj w^m), and thread 0 writes Z(M/2).  The row values come
// from registers loaded once per job (CACHE) or from the row itself.
template <int K, int M, bool CACHE, typename R, typename V>
__device__ __forceinline__ void build_z(V *__restrict__ buf, const V (&f)[M / 256], V fmid, const V *__restrict__ F,
                                        int L, R scale, V tb, const V *__restrict__ twN, int tid)
{
    constexpr int H = M / 512;
#pragma unroll(CACHE ? H : 2)
    for (int s = 0; s < H; ++s) {
        const int m = tid + 256 * s;
        const int mr = M - m;  // M/2 + 1 .. M
        const V fm = CACHE ? f[s] : F[m <= L ? m : L];
        const V fr = CACHE ? f[H + s] : F[mr <= L ? mr : L];
        const V xm = coef_x<K, M>(fm, m, L, scale);
        const V xr = coef_x<K, M>(fr, mr, L, scale);
        const V tw = cmul(tb, twN[256 * s]);  // e^{2 pi i m/N}
        const V xc = cconj(xr);
        buf[lpad(m)] = cadd(cadd(xm, xc), cmuli(cmul(tw, csub(xm, xc))));
        const V xc2 = cconj(xm);
        const V tw2 = cmk<V>(-tw.x, tw.y);  // e^{2 pi i (M-m)/N}
        if (m > 0) buf[lpad(mr)] = cadd(cadd(xr, xc2), cmuli(cmul(tw2, csub(xr, xc2))));
    }
    if (tid == 0) {
        const V xh = coef_x<K, M>(CACHE ? fmid : F[M / 2 <= L ? M / 2 : L], M / 2, L, scale);
        const V xc = cconj(xh);
        buf[lpad(M / 2)] = cadd(cadd(xh, xc), cmuli(cmul(twN[M / 2], csub(xh, xc))));
    }
}

// The last pass of pass_p2 (Ns = 256, RX = RL) kept in registers: v[s] holds
// the pair of output pixels tid + 256 s.
template <int M, typename V>
__device__ __forceinline__ void last_pass_regs(const V *__restrict__ buf, V (&v)[M / 256], int tid,
                                               const V *__restrict__ twN)
{
    constexpr int RL = M / 256;
#pragma unroll
    for (int s = 0; s < RL; ++s) v[s] = buf[lpad(tid + s * 256)];
    apply_twiddles<RL>(v, twN, tid, 2 * M / (256 * RL));
    dftR<RL>(v);
}

// Two FP16 outputs a, b of one job into their paired plane: pixel n of a at
// 2n, of b at 2n + 1; ha holds a's pixel pair i (rounded to FP16), y is b's.
// Written once, read by the remap: the stores bypass the caches.
__device__ __forceinline__ void put_pair(__half *o, size_t i, __half2 ha, float2 y)
{
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    const __half2 h0 = __halves2half2(__low2half(ha), __float2half_rn(y.x));
    const __half2 h1 = __halves2half2(__high2half(ha), __float2half_rn(y.y));
    const u2 w = {*reinterpret_cast<const unsigned *>(&h0), *reinterpret_cast<const unsigned *>(&h1)};
    __builtin_nontemporal_store(w, reinterpret_cast<u2 *>(o) + i);
}

// Length M = 256 RL (RL = 2, 4, 8, 16): 256 threads; passes 16, 16, RL.  The
// spectrum of each output is built by the code for its phi-derivative order.
// FP32 jobs may pair consecutive FP16 outputs (bit q of job.pair): the first
// one's last pass waits in LDS, in FP16, until the second one's is done.
// Two waves per SIMD: the register budget holds an FP32 row for the whole job
// (its re-reads, once per output, cost more than the lost occupancy).
template <typename R, int M>
__global__ __launch_bounds__(256, 2) void k_ring_fft_p2(
    const FftJob *__restrict__ jobs, const typename C2<R>::T *__restrict__ Fbase, R *__restrict__ Dbase, __half *__restrict__ D16, int lmax,
    const typename C2<R>::T *__restrict__ twN)
{
    using V = typename C2<R>::T;
    constexpr int RL = M / 256;
    static_assert(RL == 2 || RL == 4 || RL == 8 || RL == 16, "power-of-two length 512..4096");
    extern __shared__ unsigned char smem_raw[];
    V *buf = reinterpret_cast<V *>(smem_raw);
    const int tid = threadIdx.x;
    const FftJob &job = jobs[blockIdx.x];
    const V *F = Fbase + job.src;
    const int L = lmax;

    const V tb = twN[tid];
    // FP32: the row is read once per job and kept in registers for all of its
    // outputs; FP64 reads it again per output (register budget)
    constexpr bool CACHE = sizeof(R) == 4;
    V f[RL], fmid;
    if constexpr (CACHE) load_pairs<M>(f, fmid, F, L, tid);
    // the first output of a pair, after the FFT buffer (FP32 kernels)
    __half2 *held = reinterpret_cast<__half2 *>(smem_raw + (size_t)(M + M / 32) * sizeof(V));
    for (int q = 0; q < job.nk; ++q) {
        const R scale = (R)job.scale[q];
        switch (job.k[q]) {  // uniform
        case 0: build_z<0, M, CACHE>(buf, f, fmid, F, L, scale, tb, twN, tid); break;
        case 1: build_z<1, M, CACHE>(buf, f, fmid, F, L, scale, tb, twN, tid); break;
        case 2: build_z<2, M, CACHE>(buf, f, fmid, F, L, scale, tb, twN, tid); break;
        case 3: build_z<3, M, CACHE>(buf, f, fmid, F, L, scale, tb, twN, tid); break;
        case 4: build_z<4, M, CACHE>(buf, f, fmid, F, L, scale, tb, twN, tid); break;
        case 5: build_z<5, M, CACHE>(buf, f, fmid, F, L, scale, tb, twN, tid); break;
        case 6: build_z<6, M, CACHE>(buf, f, fmid, F, L, scale, tb, twN, tid); break;
        case 7: build_z<7, M, CACHE>(buf, f, fmid, F, L, scale, tb, twN, tid); break;
        default: build_z<8, M, CACHE>(buf, f, fmid, F, L, scale, tb, twN, tid); break;
        }
        __syncthreads();
        pass_p2<M, 16, 1, false>(buf, (V *)nullptr, tid, twN);
        __syncthreads();
        pass_p2<M, 16, 16, false>(buf, (V *)nullptr, tid, twN);
        __syncthreads();
        // last pass straight to the output ring: out[2n], out[2n+1] = Re, Im z_n
        if constexpr (sizeof(R) == 4) {
            if ((job.pair >> q) & 1) {
                V v[RL];
                last_pass_regs<M>(buf, v, tid, twN);
#pragma unroll
                for (int s = 0; s < RL; ++s) held[tid + 256 * s] = __floats2half2_rn(v[s].x, v[s].y);
            } else if (q > 0 && ((job.pair >> (q - 1)) & 1)) {
                V v[RL];
                last_pass_regs<M>(buf, v, tid, twN);
#pragma unroll
                for (int s = 0; s < RL; ++s) put_pair(D16 + job.dst[q - 1], tid + 256 * s, held[tid + 256 * s], v[s]);
            } else {
                with_out<R>(job, q, Dbase, D16, [&](auto *out) { pass_p2<M, RL, 256, true>(buf, out, tid, twN); });
            }
        } else {
            with_out<R>(job, q, Dbase, D16, [&](auto *out) { pass_p2<M, RL, 256, true>(buf, out, tid, twN); });
        }
        __syncthreads();
    }
}

// ---- HEALPix rings of power-of-two length N = 2 M, lmax < N ----
//
// The radix-16 kernel above with the ring's phase and one fold term: for
// 0 <= m <= M, X_m = e^{i pi m shift / N} (c_m + sigma conj c_{N - m}) (terms
// beyond lmax are zero; lmax < N leaves no other alias), X_0 and X_M real.
__device__ __forceinline__ void sc_pi(float x, float *sn, float *cs) { sincospif(x, sn, cs); }
__device__ __forceinline__ void sc_pi(double x, double *sn, double *cs) { sincospi(x, sn, cs); }

template <int K, typename R, typename V>
__device__ __forceinline__ V coef_h(V f, int m, int L, R scale)
{
    R sc = m <= L ? scale : (R)0;
    const R mf = (R)m;
#pragma unroll
    for (int t = 0; t < K; ++t) sc *= mf;
    R re = sc * f.x, im = m == 0 ? (R)0 : sc * f.y;
    if constexpr ((K & 3) == 1) { const R t2 = re; re = -im; im = t2; }
    else if constexpr ((K & 3) == 2) { re = -re; im = -im; }
    else if constexpr ((K & 3) == 3) { const R t2 = re; re = im; im = -t2; }
    return cmk<V>(re, im);
}

// X_m from the cached F_m, the mirror F_{N - m} read when N - m <= lmax, and
// the phase e^{i pi m shift / N}.
template <int K, int M, typename R, typename V>
__device__ __forceinline__ V xh(V f, int m, const V *__restrict__ F, int L, R scale, R sigma, V ph)
{
    constexpr int N = 2 * M;
    V x = coef_h<K, R, V>(f, m, L, scale);
    const int mm = N - m;
    if (mm <= L) {
        const V c = coef_h<K, R, V>(F[mm], mm, L, scale);
        x = cmk<V>(x.x + sigma * c.x, x.y - sigma * c.y);
    }
    x = cmul(x, ph);
    if (m == 0 || m == M) x.y = (R)0;
    return x;
}

template <int K, int M, bool CACHE, typename R, typename V>
__device__ __forceinline__ void build_z_h(V *__restrict__ buf, const V (&f)[M / 256], V fmid, const V (&ph)[M / 512],
                                          V phmid, bool shift, const V *__restrict__ F, int L, R scale, R sigma,
                                          V tb, const V *__restrict__ twN, int tid)
{
    constexpr int H = M / 512;
#pragma unroll(CACHE ? H : 2)
    for (int s = 0; s < H; ++s) {
        const int m = tid + 256 * s;
        const int mr = M - m;
        const V fm = CACHE ? f[s] : F[m <= L ? m : L];
        const V fr = CACHE ? f[H + s] : F[mr <= L ? mr : L];
        const V phr = shift ? cmk<V>(ph[s].y, ph[s].x) : ph[s];
        const V xm = xh<K, M>(fm, m, F, L, scale, sigma, ph[s]);
        const V xr = xh<K, M>(fr, mr, F, L, scale, sigma, phr);
        const V tw = cmul(tb, twN[256 * s]);  // e^{2 pi i m/N}
        const V xc = cconj(xr);
        buf[lpad(m)] = cadd(cadd(xm, xc), cmuli(cmul(tw, csub(xm, xc))));
        const V xc2 = cconj(xm);
        const V tw2 = cmk<V>(-tw.x, tw.y);  // e^{2 pi i (M-m)/N}
        if (m > 0) buf[lpad(mr)] = cadd(cadd(xr, xc2), cmuli(cmul(tw2, csub(xr, xc2))));
    }
    if (tid == 0) {
        const V xhm = xh<K, M>(CACHE ? fmid : F[M / 2 <= L ? M / 2 : L], M / 2, F, L, scale, sigma, phmid);
        const V xc = cconj(xhm);
        buf[lpad(M / 2)] = cadd(cadd(xhm, xc), cmuli(cmul(twN[M / 2], csub(xhm, xc))));
    }
}

template <typename R, int M>
__global__ __launch_bounds__(256, 2) void k_ring_fft_hpx_p2(
    const FftJob *__restrict__ jobs, const typename C2<R>::T *__restrict__ Fbase, R *__restrict__ Dbase, __half *__restrict__ D16, int lmax,
    const HRing *__restrict__ hring, const typename C2<R>::T *__restrict__ twAll)
{
    using V = typename C2<R>::T;
    constexpr int RL = M / 256;
    constexpr int H = M / 512;
    constexpr int N = 2 * M;
    extern __shared__ unsigned char smem_raw[];
    V *buf = reinterpret_cast<V *>(smem_raw);
    const int tid = threadIdx.x;
    const FftJob &job = jobs[blockIdx.x];
    const HRing hr = hring[job.pad];
    const V *twN = twAll + (size_t)2 * (M / 2) * (M / 2 - 1);  // N = 4 i, i = M / 2
    const V *F = Fbase + job.src;
    const int L = lmax;
    const R sigma = (R)hr.sigma;
    const V tb = twN[tid];
    // phases e^{i pi m shift / N} of the thread's m (that of M - m is
    // e^{i pi / 2} conj of it: swap the parts) and (thread 0) of M / 2
    V ph[H], phmid = cmk<V>((R)1, (R)0);
#pragma unroll
    for (int s = 0; s < H; ++s) {
        const int m = tid + 256 * s;
        ph[s] = cmk<V>((R)1, (R)0);
        if (hr.shift) {
            R sn, cs;
            sc_pi((R)m / (R)N, &sn, &cs);
            ph[s] = cmk<V>(cs, sn);
        }
    }
    if (hr.shift) {
        R sn, cs;
        sc_pi((R)(M / 2) / (R)N, &sn, &cs);
        phmid = cmk<V>(cs, sn);
    }
    constexpr bool CACHE = sizeof(R) == 4;
    const bool shift = hr.shift != 0;
    V f[RL], fmid;
    if constexpr (CACHE) load_pairs<M>(f, fmid, F, L, tid);
    for (int q = 0; q < job.nk; ++q) {
        const R scale = (R)job.scale[q];
        switch (job.k[q]) {  // uniform
        case 0: build_z_h<0, M, CACHE>(buf, f, fmid, ph, phmid, shift, F, L, scale, sigma, tb, twN, tid); break;
        case 1: build_z_h<1, M, CACHE>(buf, f, fmid, ph, phmid, shift, F, L, scale, sigma, tb, twN, tid); break;
        case 2: build_z_h<2, M, CACHE>(buf, f, fmid, ph, phmid, shift, F, L, scale, sigma, tb, twN, tid); break;
        case 3: build_z_h<3, M, CACHE>(buf, f, fmid, ph, phmid, shift, F, L, scale, sigma, tb, twN, tid); break;
        case 4: build_z_h<4, M, CACHE>(buf, f, fmid, ph, phmid, shift, F, L, scale, sigma, tb, twN, tid); break;
        case 5: build_z_h<5, M, CACHE>(buf, f, fmid, ph, phmid, shift, F, L, scale, sigma, tb, twN, tid); break;
        case 6: build_z_h<6, M, CACHE>(buf, f, fmid, ph, phmid, shift, F, L, scale, sigma, tb, twN, tid); break;
        case 7: build_z_h<7, M, CACHE>(buf, f, fmid, ph, phmid, shift, F, L, scale, sigma, tb, twN, tid); break;
        default: build_z_h<8, M, CACHE>(buf, f, fmid, ph, phmid, shift, F, L, scale, sigma, tb, twN, tid); break;
        }
        __syncthreads();
        pass_p2<M, 16, 1, false>(buf, (V *)nullptr, tid, twN);
        __syncthreads();
        pass_p2<M, 16, 16, false>(buf, (V *)nullptr, tid, twN);
        __syncthreads();
        with_out<R>(job, q, Dbase, D16, [&](auto *out) { pass_p2<M, RL, 256, true>(buf, out, tid, twN); });
        __syncthreads();
    }
}

// ---- HEALPix rings of awkward length: Bluestein's chirp transform ----
//
// A ring whose half length M has a prime factor above 13 takes the length-M
// inverse DFT z_n = sum_k Z_k e^{2 pi i n k / M} as a convolution: with
// w = e^{i pi / M} and n k = (n^2 + k^2 - (n - k)^2) / 2,
//     z_n = w^{n^2} sum_k (Z_k w^{k^2}) w^{-(n - k)^2},
// a circular convolution of length P (a power of two >= 2 M - 1, so the
// negative lags do not wrap onto positive ones): a_k = Z_k w^{k^2} padded with
// zeros, b_j = w^{-j^2} at j and P - j.  c = IDFT_P(DFT_P(a) DFT_P(b)) / P,
// with DFT_P(b) / P from the plan (b is even, so its forward and inverse
// sums agree), DFT_P(a) = conj(IDFT_P(conj a)).  w^t = e^{2 pi i t / N}
// (N = 2 M) comes from the ring's twiddle table at t = k^2 mod N.  The
// length-P transforms run in place in LDS (radix-16 Stockham passes, the
// last of radix P / 4096 .. 16, every value of a pass read into registers
// before any is written).  Every ring of half length M > 32 outside the
// power-of-two class takes this path: smooth lengths too (a generic
// mixed-radix pass with run-time radices and strides is slower than the two
// fixed power-of-two transforms).

// One in-place Stockham pass of radix RX (stride Ns) over P points, T
// threads: each thread reads all of its butterflies' inputs, the workgroup
// syncs, then transforms and writes.  Twiddles e^{2 pi i t / 8192} from twP.
template <int P, int RX, int Ns, int T, typename V>
__device__ __forceinline__ void ipass(V *__restrict__ buf, int tid, const V *__restrict__ twP)
{
    constexpr int nb = P / RX;
    constexpr int U = (nb + T - 1) / T;
    constexpr int tstride = 8192 / (Ns * RX);
    V v[U][RX];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + T * u;
        if (nb % T == 0 || b < nb) {
#pragma unroll
            for (int s = 0; s < RX; ++s) v[u][s] = buf[lpad(b + s * nb)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + T * u;
        if (nb % T == 0 || b < nb) {
            const int kk = b & (Ns - 1);
            if constexpr (Ns > 1) apply_twiddles<RX>(v[u], twP, kk, tstride);
            dftR<RX>(v[u]);
            const int base = (b / Ns) * Ns * RX + kk;
#pragma unroll
            for (int s = 0; s < RX; ++s) buf[lpad(base + s * Ns)] = v[u][s];
        }
    }
    __syncthreads();
}

// In-place inverse DFT of P = 256 .. 8192 points (sign +, unnormalized);
// the caller syncs before (inputs written) and the last pass syncs after.
template <int P, int T, typename V>
__device__ __forceinline__ void fft_inplace(V *__restrict__ buf, int tid, const V *__restrict__ twP)
{
    static_assert(P >= 256 && P <= 8192 && (P & (P - 1)) == 0, "power of two 256..8192");
    ipass<P, 16, 1, T>(buf, tid, twP);
    ipass<P, 16, 16, T>(buf, tid, twP);
    if constexpr (P > 256) {
        constexpr int R3 = P / 256 < 16 ? P / 256 : 16;
        ipass<P, R3, 256, T>(buf, tid, twP);
    }
    if constexpr (P == 8192) ipass<P, 2, 4096, T>(buf, tid, twP);
}

// Threads of the Bluestein kernels: 512 for P = 8192 (one radix-16
// butterfly per thread and pass), else 256.
template <int P>
constexpr int blue_threads() { return P == 8192 ? 512 : 256; }

// Chirp spectra of the plan (FP64, once per plan): one workgroup per ring
// length, item {M, P, boff, 0}; out[boff + k] = DFT_P(b)_k / P.
template <int P>
__global__ __launch_bounds__(blue_threads<P>()) void k_bluestein_table(const int4 *__restrict__ items, const double2 *__restrict__ twAll,
                                                         const double2 *__restrict__ twP, double2 *__restrict__ out64,
                                                         float2 *__restrict__ out32)
{
    using V = double2;
    extern __shared__ unsigned char smem_raw[];
    V *buf = reinterpret_cast<V *>(smem_raw);
    const int tid = threadIdx.x;
    const int4 it = items[blockIdx.x];
    const int M = it.x, N = 2 * M, i4 = N / 4;
    const int64_t boff = it.z;
    const V *twN = twAll + (size_t)2 * i4 * (i4 - 1);
    constexpr int T = blue_threads<P>();
    for (int j = tid; j < P; j += T) {
        V b = cmk<V>(0.0, 0.0);
        const int jj = j < M ? j : (j > P - M ? P - j : -1);
        if (jj >= 0) b = cconj(twN[(int)(((int64_t)jj * jj) % N)]);  // w^{-j^2}
        buf[lpad(j)] = b;
    }
    __syncthreads();
    fft_inplace<P, T>(buf, tid, twP);
    const double inv = 1.0 / (double)P;
    for (int k = tid; k < P; k += T) {
        const V x = buf[lpad(k)];
        out64[boff + k] = cmk<V>(x.x * inv, x.y * inv);
        out32[boff + k] = make_float2((float)(x.x * inv), (float)(x.y * inv));
    }
}

// Ring syntheses of the Bluestein rings (class P): per output, the folded
// half spectrum X_0 .. X_M into the upper half of the buffer (X_0 and X_M,
// both real, share slot M), Z_k as in the mixed-radix kernel, a_k = conj(Z_k
// w^{k^2}), the two transforms around the product with the chirp spectrum,
// and out[2n], out[2n + 1] = Re, Im (w^{n^2} c_n).
// FP32: at most 128 VGPRs (four waves per SIMD; a few spills cost less than
// the lost occupancy); FP64 keeps its registers.
template <typename R, int P>
__global__ __launch_bounds__(blue_threads<P>()) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
void k_ring_fft_blue(
    const FftJob *__restrict__ jobs, const typename C2<R>::T *__restrict__ Fbase, R *__restrict__ Dbase, __half *__restrict__ D16, int lmax,
    const HRing *__restrict__ hring, const typename C2<R>::T *__restrict__ twAll,
    const typename C2<R>::T *__restrict__ twP, const typename C2<R>::T *__restrict__ bhat)
{
    using V = typename C2<R>::T;
    constexpr int T = blue_threads<P>();
    extern __shared__ unsigned char smem_raw[];
    V *buf = reinterpret_cast<V *>(smem_raw);
    const int tid = threadIdx.x;
    const FftJob &job = jobs[blockIdx.x];
    const HRing hr = hring[job.pad];
    const int N = hr.nphi, M = N / 2, L = lmax, i4 = N / 4;
    const R sigma = (R)hr.sigma;
    const V *twN = twAll + (size_t)2 * i4 * (i4 - 1);
    const V *bh = bhat + hr.boff;
    const V *F = Fbase + job.src;
    for (int q = 0; q < job.nk; ++q) {
        const int k = job.k[q];
        const R scale = (R)job.scale[q];
        auto coef = [&](int m) -> V {  // scale (i m)^k F_m, m >= 0
            const V f = F[m];
            R mk = scale;
            for (int t = 0; t < k; ++t) mk *= (R)m;
            R re = mk * f.x, im = m == 0 ? (R)0 : mk * f.y;
            switch (k & 3) {
            case 1: { const R t2 = re; re = -im; im = t2; } break;
            case 2: re = -re; im = -im; break;
            case 3: { const R t2 = re; re = im; im = -t2; } break;
            default: break;
            }
            return cmk<V>(re, im);
        };
        // X_qq = e^{i qq phi0} sum over m = qq mod N (with sigma per wrap)
        auto fold = [&](int qq) -> V {
            R re = 0, im = 0, sg = 1;
            for (int m = qq; m <= L; m += N, sg *= sigma) {
                const V c = coef(m);
                re += sg * c.x;
                im += sg * c.y;
            }
            sg = sigma;
            for (int m = N - qq; m <= L; m += N, sg *= sigma) {
                const V c = coef(m);
                re += sg * c.x;
                im -= sg * c.y;
            }
            R sn = 0, cs = 1;
            if (hr.shift) sc_pi((R)qq / (R)N, &sn, &cs);
            return cmk<V>(re * cs - im * sn, re * sn + im * cs);
        };
        for (int t = tid; t < M; t += T) buf[lpad(M + t)] = t == 0 ? cmk<V>(fold(0).x, fold(M).x) : fold(t);
        __syncthreads();
        for (int t = tid; t < M; t += T) {
            const V s0 = buf[lpad(M)];
            const V xm = t == 0 ? cmk<V>(s0.x, (R)0) : buf[lpad(M + t)];
            const V xr = t == 0 ? cmk<V>(s0.y, (R)0) : buf[lpad(M + M - t)];
            const V xc = cconj(xr);
            const V z = cadd(cadd(xm, xc), cmuli(cmul(twN[t], csub(xm, xc))));
            buf[lpad(t)] = cconj(cmul(z, twN[(int)(((int64_t)t * t) % N)]));
        }
        __syncthreads();
        for (int t = M + tid; t < P; t += T) buf[lpad(t)] = cmk<V>((R)0, (R)0);
        __syncthreads();
        fft_inplace<P, T>(buf, tid, twP);
        for (int t = tid; t < P; t += T) buf[lpad(t)] = cmul(cconj(buf[lpad(t)]), bh[t]);
        __syncthreads();
        fft_inplace<P, T>(buf, tid, twP);
        with_out<R>(job, q, Dbase, D16, [&](auto *out) {
            for (int n = tid; n < M; n += T) put(out, n, cmul(buf[lpad(n)], twN[(int)(((int64_t)n * n) % N)]));
        });
        __syncthreads();
    }
}
}  // namespace

// Kernel fill of n 32-bit words (usable inside captured graphs, unlike a
// memset node).
// Deflection ring FFTs in FP32 for rings whose FP64 transform does not fit
// in LDS: the FP64 rows (2 x ntheta x (L + 1) complex) to FP32 in the
// scratch, the FP32 transform into the scratch after them, then the
// deflection back to FP64 in alpha.
hipError_t launch_defl_fft32(Plan &p, const void *rows64, void *alpha, int L)
{
    const size_t nrow = (size_t)2 * p.ntheta * (L + 1) * 2;  // real values of the rows
    const size_t na = (size_t)2 * p.npix();
    float *rows32 = (float *)p.dscratch.ptr, *a32 = rows32 + nrow;
    const unsigned nb = 2048;
    hipLaunchKernelGGL(k_to_f32, dim3(nb), dim3(256), 0, p.stream, (const double *)rows64, rows32, nrow);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = launch_fft_jobs(p, rows32, a32, (const FftJob *)p.jobsDefl.ptr, p.njobsDefl, false, 0, nullptr, L);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_to_f64, dim3(nb), dim3(256), 0, p.stream, a32, (double *)alpha, na);
    return hipGetLastError();
}

hipError_t fill_words(void *x, size_t n, uint32_t v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint32_t *)x, n, v);
    return hipGetLastError();
}

// Allow the ping-pong LDS buffers of this plan's FFT length beyond the
// default 64 KiB dynamic-LDS limit when the device has more.
// LDS of the radix-16 kernel: the padded buffer, and for FP32 the FP16
// first outputs of pairs
template <typename R>
constexpr size_t p2_lds(int M)
{
    return (size_t)(M + M / 32) * sizeof(typename C2<R>::T) + (sizeof(R) == 4 ? (size_t)M * sizeof(__half2) : 0);
}

template <typename R, int M>
hipError_t prep_p2()
{
    const size_t b = p2_lds<R>(M);
    if (b <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ring_fft_p2<R, M>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
}

// LDS of one Bluestein buffer of P points (padded)
template <typename V>
constexpr size_t blue_lds(int P) { return (size_t)(P + P / 32) * sizeof(V); }

template <typename R, int P>
hipError_t blue_attr()
{
    const size_t b = blue_lds<typename C2<R>::T>(P);
    if (b <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ring_fft_blue<R, P>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
}

template <typename R>
hipError_t blue_prepare()
{
    hipError_t e = blue_attr<R, 4096>();
    if (e == hipSuccess) e = blue_attr<R, 8192>();
    if (e == hipSuccess && sizeof(R) == 8) {
        const size_t b4 = blue_lds<double2>(4096), b8 = blue_lds<double2>(8192);
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bluestein_table<4096>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)b4);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bluestein_table<8192>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)b8);
    }
    return e;
}

template <int P>
void launch_blue_table(Plan &p, const int4 *items, int n)
{
    hipLaunchKernelGGL(k_bluestein_table<P>, dim3(n), dim3(blue_threads<P>()), blue_lds<double2>(P), p.stream, items,
                       (const double2 *)p.twid64.ptr, (const double2 *)p.twP64.ptr, (double2 *)p.bhat64.ptr,
                       (float2 *)p.bhat32.ptr);
}

hipError_t launch_bluestein_tables(Plan &p, const std::vector<int4> &items)
{
    if (items.empty()) return hipSuccess;
    hipError_t e = blue_prepare<double>();
    if (e != hipSuccess) return e;
    int4 *d = nullptr;
    e = hipMalloc(&d, items.size() * sizeof(int4));
    if (e != hipSuccess) return e;
    e = hipMemcpy(d, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice);
    // items come sorted by P: one launch per class
    size_t a = 0;
    while (e == hipSuccess && a < items.size()) {
        size_t b = a;
        while (b < items.size() && items[b].y == items[a].y) ++b;
        const int n = (int)(b - a);
        switch (items[a].y) {
        case 256: launch_blue_table<256>(p, d + a, n); break;
        case 512: launch_blue_table<512>(p, d + a, n); break;
        case 1024: launch_blue_table<1024>(p, d + a, n); break;
        case 2048: launch_blue_table<2048>(p, d + a, n); break;
        case 4096: launch_blue_table<4096>(p, d + a, n); break;
        case 8192: launch_blue_table<8192>(p, d + a, n); break;
        default: e = hipErrorInvalidValue; break;
        }
        if (e == hipSuccess) e = hipGetLastError();
        a = b;
    }
    const hipError_t e2 = hipStreamSynchronize(p.stream);
    (void)hipFree(d);
    return e != hipSuccess ? e : e2;
}

template <typename R, int P>
void launch_blue(Plan &p, const void *Fbase, void *Dbase, void *D16, const FftJob *jobs, int n)
{
    using V = typename C2<R>::T;
    const bool f64 = sizeof(R) == 8;
    hipLaunchKernelGGL((k_ring_fft_blue<R, P>), dim3(n), dim3(blue_threads<P>()), blue_lds<V>(P), p.stream, jobs,
                       (const V *)Fbase,
                       (R *)Dbase, (__half *)D16, p.lmax, (const HRing *)p.hring.ptr,
                       (const V *)(f64 ? p.twid64.ptr : p.twid32.ptr), (const V *)(f64 ? p.twP64.ptr : p.twP32.ptr),
                       (const V *)(f64 ? p.bhat64.ptr : p.bhat32.ptr));
}

template <typename R, int M>
void launch_hpx_p2(Plan &p, const void *Fbase, void *Dbase, void *D16, const FftJob *jobs, int n)
{
    using V = typename C2<R>::T;
    const bool f64 = sizeof(R) == 8;
    hipLaunchKernelGGL((k_ring_fft_hpx_p2<R, M>), dim3(n), dim3(256), (size_t)(M + M / 32) * sizeof(V), p.stream, jobs,
                       (const V *)Fbase, (R *)Dbase, (__half *)D16, p.lmax, (const HRing *)p.hring.ptr,
                       (const V *)(f64 ? p.twid64.ptr : p.twid32.ptr));
}

template <typename R, int M>
hipError_t hpx_p2_attr()
{
    using V = typename C2<R>::T;
    const size_t b = (size_t)(M + M / 32) * sizeof(V);
    if (b <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ring_fft_hpx_p2<R, M>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
}

// The job classes of one HEALPix list: mixed radix, Bluestein by P, then the
// power-of-two rings.
template <typename R>
hipError_t launch_hpx(Plan &p, const void *Fbase, void *Dbase, void *D16, const FftJob *jobs, int njobs, int list)
{
    using V = typename C2<R>::T;
    const int *cnt = p.hjobs[list];
    int a = 0;
    if (cnt[0] > 0) {
        const size_t M = (size_t)p.hmax_direct;
        hipLaunchKernelGGL(k_ring_fft_hpx<R>, dim3(cnt[0]), dim3(256), (2 * M + 1) * sizeof(V), p.stream, jobs,
                           (const V *)Fbase, (R *)Dbase, (__half *)D16, p.lmax, (const HRing *)p.hring.ptr,
                           (const V *)(sizeof(R) == 8 ? p.twid64.ptr : p.twid32.ptr));
        a = cnt[0];
    }
    for (int c = 1; c < kHpxClasses; ++c) {
        const int n = cnt[c];
        if (n <= 0) continue;
        if (c == kHpxPow2) {
            switch (p.hmax_pow2) {
            case 512: launch_hpx_p2<R, 512>(p, Fbase, Dbase, D16, jobs + a, n); break;
            case 1024: launch_hpx_p2<R, 1024>(p, Fbase, Dbase, D16, jobs + a, n); break;
            case 2048: launch_hpx_p2<R, 2048>(p, Fbase, Dbase, D16, jobs + a, n); break;
            case 4096: launch_hpx_p2<R, 4096>(p, Fbase, Dbase, D16, jobs + a, n); break;
            default: return hipErrorInvalidValue;
            }
            a += n;
            continue;
        }
        switch (c) {
        case 1: launch_blue<R, 256>(p, Fbase, Dbase, D16, jobs + a, n); break;
        case 2: launch_blue<R, 512>(p, Fbase, Dbase, D16, jobs + a, n); break;
        case 3: launch_blue<R, 1024>(p, Fbase, Dbase, D16, jobs + a, n); break;
        case 4: launch_blue<R, 2048>(p, Fbase, Dbase, D16, jobs + a, n); break;
        case 5: launch_blue<R, 4096>(p, Fbase, Dbase, D16, jobs + a, n); break;
        default: launch_blue<R, 8192>(p, Fbase, Dbase, D16, jobs + a, n); break;
        }
        a += n;
    }
    if (a != njobs) return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t fft_prepare(Plan &p)
{
    if (p.nside) {
        const size_t M = (size_t)p.hmax_direct;
        const size_t b64 = (2 * M + 1) * sizeof(double2), b32 = (2 * M + 1) * sizeof(float2);
        hipError_t e = hipSuccess;
        if (b64 > 65536)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ring_fft_hpx<double>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)b64);
        if (e == hipSuccess && b32 > 65536)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ring_fft_hpx<float>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)b32);
        if (e == hipSuccess) e = blue_prepare<double>();
        if (e == hipSuccess) e = blue_prepare<float>();
        if (e == hipSuccess && p.hmax_pow2 == 4096) e = hpx_p2_attr<double, 4096>();
        if (e == hipSuccess && p.hmax_pow2 == 4096) e = hpx_p2_attr<float, 4096>();
        if (e == hipSuccess && p.hmax_pow2 == 2048) e = hpx_p2_attr<double, 2048>();
        return e;
    }
    const size_t M = (size_t)p.nphi / 2;
    if (M == 4096) {
        hipError_t e = prep_p2<double, 4096>();
        if (e == hipSuccess) e = prep_p2<float, 4096>();
        if (e != hipSuccess) return e;
    } else if (M == 2048) {
        hipError_t e = prep_p2<double, 2048>();
        if (e != hipSuccess) return e;
    }
    const size_t b64 = 2 * M * sizeof(double2), b32 = 2 * M * sizeof(float2);
    if (b64 > 65536 && !p.defl32) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ring_fft<double>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)b64);
        if (e != hipSuccess) return e;
    }
    if (b32 > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ring_fft<float>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)b32);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename R, int M>
hipError_t launch_p2(Plan &p, const void *Fbase, void *Dbase, void *D16, const FftJob *jobs, int njobs, const void *tw,
                     int L)
{
    using V = typename C2<R>::T;
    const size_t shm = p2_lds<R>(M);
    hipLaunchKernelGGL((k_ring_fft_p2<R, M>), dim3(njobs), dim3(256), shm, p.stream, jobs, (const V *)Fbase,
                       (R *)Dbase, (__half *)D16, L, (const V *)tw);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_p2_R(Plan &p, const void *Fbase, void *Dbase, void *D16, const FftJob *jobs, int njobs, const void *tw,
                       int M, int L)
{
    switch (M) {
    case 512: return launch_p2<R, 512>(p, Fbase, Dbase, D16, jobs, njobs, tw, L);
    case 1024: return launch_p2<R, 1024>(p, Fbase, Dbase, D16, jobs, njobs, tw, L);
    case 2048: return launch_p2<R, 2048>(p, Fbase, Dbase, D16, jobs, njobs, tw, L);
    case 4096: return launch_p2<R, 4096>(p, Fbase, Dbase, D16, jobs, njobs, tw, L);
    default: return hipErrorInvalidValue;
    }
}

bool fft_p2(int M) { return M == 512 || M == 1024 || M == 2048 || M == 4096; }

hipError_t launch_fft_jobs(Plan &p, const void *Fbase, void *Dbase, const FftJob *jobs, int njobs, bool fp64,
                           int list, void *D16, int L)
{
    if (njobs <= 0) return hipSuccess;
    if (L < 0) L = p.lmax;
    if (p.nside) {
        if (list < 0 || list > 1) return hipErrorInvalidValue;
        return fp64 ? launch_hpx<double>(p, Fbase, Dbase, D16, jobs, njobs, list)
                    : launch_hpx<float>(p, Fbase, Dbase, D16, jobs, njobs, list);
    }
    const int M = p.nphi / 2;
    if (fft_p2(M)) {
        if (fp64) return launch_p2_R<double>(p, Fbase, Dbase, D16, jobs, njobs, p.twid64.ptr, M, L);
        return launch_p2_R<float>(p, Fbase, Dbase, D16, jobs, njobs, p.twid32.ptr, M, L);
    }
    Radices rad;
    rad.n = p.nradix;
    for (int i = 0; i < p.nradix; ++i) rad.r[i] = p.radix[i];
    if (fp64) {
        size_t shm = 2 * (size_t)M * sizeof(double2);
        hipLaunchKernelGGL(k_ring_fft<double>, dim3(njobs), dim3(256), shm, p.stream, jobs,
                           (const double2 *)Fbase, (double *)Dbase, (__half *)D16, L, M,
                           (const double2 *)p.twid64.ptr, rad);
    } else {
        size_t shm = 2 * (size_t)M * sizeof(float2);
        hipLaunchKernelGGL(k_ring_fft<float>, dim3(njobs), dim3(256), shm, p.stream, jobs,
                           (const float2 *)Fbase, (float *)Dbase, (__half *)D16, L, M, (const float2 *)p.twid32.ptr,
                           rad);
    }
    return hipGetLastError();
}

}  // namespace tl
