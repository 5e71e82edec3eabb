// Learned remainder of the order-2 Taylor sum: a small convolutional network
// on the 5 x 5 patch of order <= 2 derivative maps around each output
// pixel's nearest source pixel.  It predicts the terms of eq. 5 beyond
// order 2 (the remainder that higher orders would add), which is then added
// to the order-2 sum before the polarization rotation.
//
// Network (per output pixel): input 20 channels x 5 x 5 (the 18 pre-scaled
// maps Dt_jk, j + k <= 2, of T, Q, U, each field divided by its RMS over the
// patch, plus u and v), conv 3x3 valid 20 -> 32 + tanh, conv 3x3 valid
// 32 -> 32 + tanh, 1x1 32 -> 3; correction_f = sigma_f * scale_f * y_f.
//
// Forward: one wave per 32 pixels, all three layers on
// v_mfma_f32_32x32x16_bf16 in the transposed orientation out[channel][pixel]
// = W[channel][k] * x[k][pixel]: the accumulator of one layer (lane = pixel,
// 16 channels per lane) is directly the B operand of the next when the next
// layer's k index is ordered the way the accumulator holds the channels, so
// no transposition goes through LDS.  The weights are repacked once per
// update into those A-operand layouts (BF16), the patch is gathered into LDS
// (BF16, 24 channels per position), accumulation is FP32.
// Backward (training only): FP32 on the vector ALUs, one workgroup walking
// 32-pixel tiles staged in LDS; each thread owns fixed gradient entries and
// adds them to the global gradient once at the end.
#include "geom.h"
#include "tl_internal.h"

namespace tl {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int NIN = 20, NH = 32, NOUT = 3;
constexpr int CP = 24;   // channels per patch position in LDS (20 used)
constexpr int NPOS = 25;
constexpr int PU4 = NPOS * CP * 2 / 16;  // uint4 per pixel patch (75)
constexpr int K1S = 14;  // layer-1 k-steps: 27 blocks of 8 (9 taps x 3 channel blocks) + 1 empty
constexpr int K2S = 18;  // layer-2 k-steps: 9 positions x 2
constexpr int K3S = 2;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN * 9, OW2 = OB1 + NH, OB2 = OW2 + NH * NH * 9, OW3 = OB2 + NH,
              OB3 = OW3 + NOUT * NH, OSC = OB3 + NOUT;
static_assert(OSC == kCnnTrain, "parameter layout");

__device__ __forceinline__ uint4 pack8(const float (&f)[8])
{
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)f[e];
    uint4 w;
    __builtin_memcpy(&w, &v, 16);
    return w;
}

__device__ __forceinline__ bf16x8 as_bf(uint4 w)
{
    bf16x8 v;
    __builtin_memcpy(&v, &w, 16);
    return v;
}

// Channel held in accumulator slot v by lanes of half h (rows of the 32x32 D
// block: 8 (v / 4) + 4 h + v % 4).
__host__ __device__ constexpr int acc_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// ---------------------------------------------------------- weight packing --
// W1p[s][lane]: lane (o = lane % 32, h = lane / 32) holds W1[o][c][dy][dx] for
// k-block kb = 2 s + h, kb = 3 (3 dy + dx) + cb, c = 8 cb + e (e = 0..7);
// zero for c >= 20 and kb >= 27.
// W2p[t][lane]: t = 2 q + w (q = 3 qy + qx): W2[o][c][qy][qx] with
// c = acc_row(8 w + e, h).  W3p[t][lane]: W3[f][acc_row(8 t + e, h)], f < 3.
__global__ void k_cnn_pack(const float *__restrict__ P, uint4 *__restrict__ W1p, uint4 *__restrict__ W2p,
                           uint4 *__restrict__ W3p)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = g & 63, s = g >> 6;
    const int o = lane & 31, h = lane >> 5;
    float f[8];
    if (s < K1S) {
        const int kb = 2 * s + h;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            f[e] = 0.f;
            if (kb < 27) {
                const int tap = kb / 3, c = 8 * (kb % 3) + e;
                if (c < NIN) f[e] = P[OW1 + (o * NIN + c) * 9 + tap];
            }
        }
        W1p[s * 64 + lane] = pack8(f);
    } else if (s < K1S + K2S) {
        const int t = s - K1S, q = t >> 1, w = t & 1;
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] = P[OW2 + (o * NH + acc_row(8 * w + e, h)) * 9 + q];
        W2p[t * 64 + lane] = pack8(f);
    } else if (s < K1S + K2S + K3S) {
        const int t = s - K1S - K2S;
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] = o < NOUT ? P[OW3 + o * NH + acc_row(8 * t + e, h)] : 0.f;
        W3p[t * 64 + lane] = pack8(f);
    }
}

// ---------------------------------------------------------------- forward --
struct Grid {
    int ntheta, nphi;
    const double *theta;
    const double2 *trig, *phitrig;
    const double *phival;
    size_t ds;  // plane stride of the derivative maps (elements)
};

struct TrainBufs {
    uint4 *X;    // [n][PU4] normalized patch (BF16, as the forward used it)
    float *H1;   // [n][9][32] layer-1 activations
    float *H2;   // [n][32]
    float *Y;    // [n][3]
    float *S;    // [n][3] patch RMS per field
};

template <bool TRAIN>
__global__ __launch_bounds__(64) void k_cnn_forward(Grid G, const float *__restrict__ D,
                                                    const double *__restrict__ at, const double *__restrict__ ap,
                                                    const int64_t *__restrict__ pix, int64_t n,
                                                    const uint4 *__restrict__ W1p, const uint4 *__restrict__ W2p,
                                                    const uint4 *__restrict__ W3p, const float *__restrict__ P,
                                                    float *__restrict__ corr, TrainBufs tb)
{
    __shared__ uint4 s_patch[32][PU4];
    const int lane = threadIdx.x, p = lane & 31, h = lane >> 5;
    const int64_t e = (int64_t)blockIdx.x * 32 + p;
    const bool live = e < n;
    const int64_t px = live ? (pix ? pix[e] : e) : 0;
    const int nphi = G.nphi, ntheta = G.ntheta;
    const int i = (int)(px / nphi), k = (int)(px % nphi);
    const size_t npix = (size_t)ntheta * nphi;
    const PixLoc L = locate_pixel(i, k, ntheta, nphi, G.theta, G.trig, G.phitrig, G.phival, at[px], ap[px],
                                  nullptr, nullptr, (size_t)px, false, false);
    const double dth = M_PI / (double)(ntheta - 1), dph = 2.0 * M_PI / (double)nphi;
    const float u = (float)((L.thp - G.theta[L.i0]) / dth);
    const float v = (float)((L.php - G.phival[L.kh]) / dph);

    // patch positions of this lane half: [13 h, 13 h + 13) within 0..24
    const int pos0 = 13 * h, pos1 = h ? NPOS : 13;
    auto src = [&](int pos) -> size_t {
        int r = L.i0 + pos / 5 - 2;
        r = r < 0 ? 0 : (r > ntheta - 1 ? ntheta - 1 : r);
        int c = L.k0 + pos % 5 - 2;
        c = c < 0 ? c + nphi : (c >= nphi ? c - nphi : c);
        return (size_t)r * nphi + c;
    };
    float ss[3] = {0.f, 0.f, 0.f};
    for (int pos = pos0; pos < pos1; ++pos) {
        const size_t o = src(pos);
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const float x = D[(size_t)(6 * f + q) * G.ds + o];
                ss[f] = fmaf(x, x, ss[f]);
            }
    }
    float inv[3], sig[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const float t = ss[f] + __shfl_xor(ss[f], 32);
        sig[f] = sqrtf(t / 150.f);
        if (!(sig[f] > 0.f)) sig[f] = 1.f;
        inv[f] = 1.f / sig[f];
    }
    for (int pos = pos0; pos < pos1; ++pos) {
        const size_t o = src(pos);
        float c24[CP];
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int q = 0; q < 6; ++q) c24[6 * f + q] = D[(size_t)(6 * f + q) * G.ds + o] * inv[f];
        c24[18] = u;
        c24[19] = v;
#pragma unroll
        for (int c = 20; c < CP; ++c) c24[c] = 0.f;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            float f8[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) f8[q] = c24[8 * b + q];
            const uint4 w = pack8(f8);
            s_patch[p][pos * 3 + b] = w;
            if (TRAIN && live) tb.X[e * PU4 + pos * 3 + b] = w;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    uint4 w1[K1S];
#pragma unroll
    for (int s = 0; s < K1S; ++s) w1[s] = W1p[s * 64 + lane];
    float b1[16], b2[16];
#pragma unroll
    for (int vv = 0; vv < 16; ++vv) {
        b1[vv] = P[OB1 + acc_row(vv, h)];
        b2[vv] = P[OB2 + acc_row(vv, h)];
    }
    const uint4 zero = make_uint4(0, 0, 0, 0);
    floatx16 acc2;
#pragma unroll
    for (int vv = 0; vv < 16; ++vv) acc2[vv] = 0.f;
    for (int q = 0; q < 9; ++q) {
        const int qy = q / 3, qx = q % 3;
        floatx16 acc1;
#pragma unroll
        for (int vv = 0; vv < 16; ++vv) acc1[vv] = 0.f;
#pragma unroll
        for (int s = 0; s < K1S; ++s) {
            const int kb = 2 * s + h;
            uint4 bw = zero;
            if (kb < 27) {
                const int tap = kb / 3, cb = kb % 3;
                const int pos = (qy + tap / 3) * 5 + qx + tap % 3;
                bw = s_patch[p][pos * 3 + cb];
            }
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(w1[s]), as_bf(bw), acc1, 0, 0, 0);
        }
        float hv[16];
#pragma unroll
        for (int vv = 0; vv < 16; ++vv) hv[vv] = tanhf(acc1[vv] + b1[vv]);
        if (TRAIN && live)
#pragma unroll
            for (int vv = 0; vv < 16; ++vv) tb.H1[(e * 9 + q) * NH + acc_row(vv, h)] = hv[vv];
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            float f8[8];
#pragma unroll
            for (int q8 = 0; q8 < 8; ++q8) f8[q8] = hv[8 * w + q8];
            acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(W2p[(2 * q + w) * 64 + lane]), as_bf(pack8(f8)),
                                                           acc2, 0, 0, 0);
        }
    }
    float h2[16];
#pragma unroll
    for (int vv = 0; vv < 16; ++vv) h2[vv] = tanhf(acc2[vv] + b2[vv]);
    if (TRAIN && live)
#pragma unroll
        for (int vv = 0; vv < 16; ++vv) tb.H2[e * NH + acc_row(vv, h)] = h2[vv];
    floatx16 acc3;
#pragma unroll
    for (int vv = 0; vv < 16; ++vv) acc3[vv] = 0.f;
#pragma unroll
    for (int t = 0; t < K3S; ++t) {
        float f8[8];
#pragma unroll
        for (int q8 = 0; q8 < 8; ++q8) f8[q8] = h2[8 * t + q8];
        acc3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(W3p[t * 64 + lane]), as_bf(pack8(f8)), acc3, 0, 0, 0);
    }
    // rows 0..2 of the output block (slots 0..2 of lanes 0..31) are y_f
    if (live && h == 0) {
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float y = acc3[f] + P[OB3 + f];
            corr[(size_t)f * n + e] = sig[f] * P[OSC + f] * y;
            if (TRAIN) {
                tb.Y[e * 3 + f] = y;
                tb.S[e * 3 + f] = sig[f];
            }
        }
    }
}

// --------------------------------------------------------------- backward --
constexpr int BT = 1024;  // threads per backward workgroup
constexpr int NW1 = NH * NIN * 9, NW2 = NH * NH * 9;
constexpr int J1 = (NW1 + BT - 1) / BT, J2 = NW2 / BT;
static_assert(NW2 % BT == 0, "dW2 ownership");

__global__ __launch_bounds__(BT) void k_cnn_backward(int64_t n, TrainBufs tb, const float *__restrict__ target,
                                                     const float *__restrict__ P, float *__restrict__ grad,
                                                     float *__restrict__ loss)
{
    __shared__ uint4 sX[32][PU4];
    __shared__ float sH1[32][9][NH];   // h1, then the layer-1 pre-activation gradient
    __shared__ float sH2[32][NH];
    __shared__ float sG2[32][NH];      // layer-2 pre-activation gradient
    __shared__ float sG3[32][NOUT];
    __shared__ float sW2[NH][NH][9];
    __shared__ float sW3[NOUT][NH];
    const int tid = threadIdx.x;
    for (int x = tid; x < NW2; x += BT) (&sW2[0][0][0])[x] = P[OW2 + x];
    for (int x = tid; x < NOUT * NH; x += BT) (&sW3[0][0])[x] = P[OW3 + x];
    float gW1[J1], gW2[J2];
#pragma unroll
    for (int j = 0; j < J1; ++j) gW1[j] = 0.f;
#pragma unroll
    for (int j = 0; j < J2; ++j) gW2[j] = 0.f;
    float gB1 = 0.f, gB2 = 0.f, gW3 = 0.f, gB3 = 0.f, lsum = 0.f;
    const float inv3n = 1.f / (3.f * (float)n);
    const int64_t ntile = (n + 31) / 32;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t e0 = tile * 32;
        __syncthreads();
        for (int x = tid; x < 32 * PU4; x += BT) {
            const int pp = x / PU4, r = x % PU4;
            sX[pp][r] = (e0 + pp < n) ? tb.X[(e0 + pp) * PU4 + r] : make_uint4(0, 0, 0, 0);
        }
        for (int x = tid; x < 32 * 9 * NH; x += BT) {
            const int pp = x / (9 * NH);
            (&sH1[0][0][0])[x] = (e0 + pp < n) ? tb.H1[e0 * 9 * NH + x] : 0.f;
        }
        for (int x = tid; x < 32 * NH; x += BT) {
            const int pp = x / NH;
            (&sH2[0][0])[x] = (e0 + pp < n) ? tb.H2[e0 * NH + x] : 0.f;
        }
        if (tid < 32 * NOUT) {
            const int pp = tid / NOUT, f = tid % NOUT;
            float g = 0.f;
            if (e0 + pp < n) {
                const int64_t ee = e0 + pp;
                const float tn = target[(size_t)f * n + ee] / (tb.S[ee * 3 + f] * P[OSC + f]);
                const float d = tb.Y[ee * 3 + f] - tn;
                lsum += d * d;
                g = 2.f * d * inv3n;
            }
            sG3[pp][f] = g;
        }
        __syncthreads();
        // layer 3 and the layer-2 pre-activation gradient
        for (int x = tid; x < 32 * NH; x += BT) {
            const int pp = x / NH, o = x % NH;
            float s = 0.f;
#pragma unroll
            for (int f = 0; f < NOUT; ++f) s = fmaf(sW3[f][o], sG3[pp][f], s);
            const float hh = sH2[pp][o];
            sG2[pp][o] = s * (1.f - hh * hh);
        }
        __syncthreads();
        if (tid < NOUT * NH) {
            const int f = tid / NH, o = tid % NH;
            for (int pp = 0; pp < 32; ++pp) gW3 = fmaf(sG3[pp][f], sH2[pp][o], gW3);
        }
        if (tid < NOUT)
            for (int pp = 0; pp < 32; ++pp) gB3 += sG3[pp][tid];
        if (tid < NH)
            for (int pp = 0; pp < 32; ++pp) gB2 += sG2[pp][tid];
#pragma unroll
        for (int j = 0; j < J2; ++j) {
            const int idx = tid + BT * j;  // (o, c, q) of W2[o][c][q]
            const int o = idx / (NH * 9), c = (idx / 9) % NH, q = idx % 9;
            float s = 0.f;
#pragma unroll 4
            for (int pp = 0; pp < 32; ++pp) s = fmaf(sG2[pp][o], sH1[pp][q][c], s);
            gW2[j] += s;
        }
        __syncthreads();
        // layer-1 pre-activation gradient, in place of h1 (each entry is read
        // and written by its own thread only)
        for (int x = tid; x < 32 * 9 * NH; x += BT) {
            const int pp = x / (9 * NH), q = (x / NH) % 9, c = x % NH;
            float sacc = 0.f;
#pragma unroll 8
            for (int o = 0; o < NH; ++o) sacc = fmaf(sW2[o][c][q], sG2[pp][o], sacc);
            const float hh = sH1[pp][q][c];
            sH1[pp][q][c] = sacc * (1.f - hh * hh);
        }
        __syncthreads();
        if (tid < NH)
            for (int pp = 0; pp < 32; ++pp)
                for (int q = 0; q < 9; ++q) gB1 += sH1[pp][q][tid];
#pragma unroll
        for (int j = 0; j < J1; ++j) {
            const int idx = tid + BT * j;  // (o, c, tap) of W1[o][c][dy][dx]
            if (idx < NW1) {
                const int o = idx / (NIN * 9), c = (idx / 9) % NIN, tap = idx % 9;
                const int dy = tap / 3, dx = tap % 3;
                const int cb = c >> 3, ce = c & 7;
                float s = 0.f;
#pragma unroll 1
                for (int pp = 0; pp < 32; ++pp)
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        const int pos = (q / 3 + dy) * 5 + q % 3 + dx;
                        const uint4 w = sX[pp][pos * 3 + cb];
                        const unsigned word = (&w.x)[ce >> 1];
                        const float xv = __uint_as_float((ce & 1) ? (word & 0xffff0000u) : (word << 16));
                        s = fmaf(sH1[pp][q][o], xv, s);
                    }
                gW1[j] += s;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < J1; ++j)
        if (tid + BT * j < NW1) atomicAdd(&grad[OW1 + tid + BT * j], gW1[j]);
#pragma unroll
    for (int j = 0; j < J2; ++j) atomicAdd(&grad[OW2 + tid + BT * j], gW2[j]);
    if (tid < NH) {
        atomicAdd(&grad[OB1 + tid], gB1);
        atomicAdd(&grad[OB2 + tid], gB2);
    }
    if (tid < NOUT * NH) atomicAdd(&grad[OW3 + tid], gW3);
    if (tid < NOUT) atomicAdd(&grad[OB3 + tid], gB3);
    if (tid < 32 * NOUT) atomicAdd(loss, lsum * (1.f / (3.f * (float)n)));
}

__global__ void k_fill(float *__restrict__ x, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// Adam with bias correction (c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t)).
__global__ void k_cnn_adam(float *__restrict__ P, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace

hipError_t cnn_pack(const CnnBufs &c, hipStream_t st)
{
    const int nthreads = (K1S + K2S + K3S) * 64;
    hipLaunchKernelGGL(k_cnn_pack, dim3((nthreads + 255) / 256), dim3(256), 0, st, (const float *)c.params,
                       (uint4 *)c.W1p, (uint4 *)c.W2p, (uint4 *)c.W3p);
    return hipGetLastError();
}

size_t cnn_packed_bytes() { return (size_t)(K1S + K2S + K3S) * 64 * 16; }
size_t cnn_train_bytes_per_pixel() { return PU4 * 16 + (9 * NH + NH + 3 + 3) * sizeof(float); }

hipError_t cnn_forward(const Plan &p, const CnnBufs &c, const float *D, const double *at, const double *ap,
                       const int64_t *pix, int64_t n, float *corr, bool train, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    // the plan's own maps have padded planes; a caller's are [field][map][pixel]
    Grid G{p.ntheta, p.nphi, (const double *)p.theta.ptr, (const double2 *)p.trig.ptr,
           (const double2 *)p.phitab.ptr, (const double *)p.phival.ptr,
           D == (const float *)p.D.ptr ? p.dstride : p.npix()};
    TrainBufs tb{};
    if (train) {
        char *b = (char *)c.work;
        tb.X = (uint4 *)b;
        b += (size_t)n * PU4 * 16;
        tb.H1 = (float *)b;
        b += (size_t)n * 9 * NH * 4;
        tb.H2 = (float *)b;
        b += (size_t)n * NH * 4;
        tb.Y = (float *)b;
        b += (size_t)n * 3 * 4;
        tb.S = (float *)b;
    }
    const unsigned nb = (unsigned)((n + 31) / 32);
    if (train)
        hipLaunchKernelGGL(k_cnn_forward<true>, dim3(nb), dim3(64), 0, st, G, D, at, ap, pix, n,
                           (const uint4 *)c.W1p, (const uint4 *)c.W2p, (const uint4 *)c.W3p, (const float *)c.params,
                           corr, tb);
    else
        hipLaunchKernelGGL(k_cnn_forward<false>, dim3(nb), dim3(64), 0, st, G, D, at, ap, pix, n,
                           (const uint4 *)c.W1p, (const uint4 *)c.W2p, (const uint4 *)c.W3p, (const float *)c.params,
                           corr, tb);
    return hipGetLastError();
}

hipError_t cnn_backward(const CnnBufs &c, int64_t n, const float *target, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, dim3((kCnnTrain + 1 + 255) / 256), dim3(256), 0, st, (float *)c.grad,
                       (int64_t)kCnnTrain + 1, 0.f);  // gradient and the loss slot after it
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n <= 0) return e;
    TrainBufs tb{};
    char *b = (char *)c.work;
    tb.X = (uint4 *)b;
    b += (size_t)n * PU4 * 16;
    tb.H1 = (float *)b;
    b += (size_t)n * 9 * NH * 4;
    tb.H2 = (float *)b;
    b += (size_t)n * NH * 4;
    tb.Y = (float *)b;
    b += (size_t)n * 3 * 4;
    tb.S = (float *)b;
    const int64_t ntile = (n + 31) / 32;
    const unsigned nb = (unsigned)(ntile < 512 ? ntile : 512);
    hipLaunchKernelGGL(k_cnn_backward, dim3(nb), dim3(BT), 0, st, n, tb, target, (const float *)c.params,
                       (float *)c.grad, (float *)c.grad + kCnnTrain);
    return hipGetLastError();
}

hipError_t cnn_adam(const CnnBufs &c, int step, float lr, hipStream_t st)
{
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - pow(b1, step))), c2 = (float)(1.0 / (1.0 - pow(b2, step)));
    hipLaunchKernelGGL(k_cnn_adam, dim3((kCnnTrain + 255) / 256), dim3(256), 0, st, (float *)c.params,
                       (const float *)c.grad, (float *)c.m, (float *)c.v, kCnnTrain, lr, (float)b1, (float)b2, 1e-8f,
                       c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return cnn_pack(c, st);
}

hipError_t cnn_zero(float *x, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, 0.f);
    return hipGetLastError();
}

}  // namespace tl
