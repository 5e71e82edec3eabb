// Harmonic stage for the reduced-precision forms: lambda / lambda' tables at
// plan time, a streaming MFMA GEMM per call.
//
// The L-power form (legendre_mfma.hip) needs, per m, the product of the
// matrix A[ring, {lam, lam'}][l] with right-hand sides built from a_lm.  A
// depends only on the grid and lmax, so the reduced-precision forms compute
// it once, in FP64 (same recursion, same exponent scaling), round it to
// FP16/BF16 (optionally as hi + lo), and store it in HBM already arranged as
// v_mfma_f32_32x32x16 operands: per (m, 32-ring tile, 32-l chunk, type,
// parity) one 1 KiB block whose lane i holds the 8 values of ring i % 32 at
// l = l0 + par + 2 (8 (i / 32) + q), q = 0..7.  Each call then streams the
// blocks (coalesced 16-byte lane loads) against right-hand sides computed in
// LDS, for up to TL_TAB_MAXBATCH realizations at once -- the FP64 recursion is
// paid once per plan, the table once per batch.  The epilogue is the FP64
// L-power epilogue of the FP32 form.
//
// Precision forms: FP16 / BF16 store one table and take one MFMA per
// product; BF16X3 / FP16X2 store hi and lo tables and take hi*hi + hi*lo +
// lo*hi.  FP16 operands are scaled by powers of two: lam' by 2^-7 in the
// table, every right-hand-side column of a given m by the power of two that
// brings its largest entry to [2^13, 2^14).
#include "tl_internal.h"

namespace tl {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

constexpr double kHi = 0x1p256;
constexpr double kDown = 0x1p-512;
constexpr int KC = 32;          // l values per table chunk (16 per parity)
constexpr int TILE = 32;        // ring pairs per table tile
constexpr double kDerivScale = 0x1p-7;  // lam' scale in FP16 tables

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

// ------------------------------------------------------------ builder ----
// One lane per ring pair, 64 lanes = two 32-ring tiles of one m.  Writes, for
// every 32-l chunk, the blocks [type][parity] (and [hi/lo] when split), and
// the first chunk holding a non-zero value per (m, tile).
template <bool BF, bool SPLIT>
__global__ __launch_bounds__(64) void k_build_tab(int lmax, int nrp, int rbeg, int ntile, int jtab,
                                                  const double2 *__restrict__ trig, const double4 *__restrict__ coef0,
                                                  const double *__restrict__ start, const int *__restrict__ exps,
                                                  const int64_t *__restrict__ moff, uint4 *__restrict__ tab,
                                                  int *__restrict__ kstart)
{
    using T = typename H<BF>::T;
    const int m = blockIdx.y;
    const int lane = threadIdx.x;
    const int tile = blockIdx.x * 2 + (lane >> 5);
    const int rl = lane & 31;
    if (tile >= ntile) return;
    const int r = rbeg + tile * TILE + rl;
    const bool live = r < nrp;
    const double x = live ? trig[r].x : 0.0, sn = live ? trig[r].y : 1.0;
    const size_t base = (size_t)m * (2 * lmax + 1 - m) / 2;
    const int nk = (lmax - m + 1 + KC - 1) / KC;
    constexpr int NSPL = SPLIT ? 2 : 1;
    // block of (m, tile): nk chunks x NSPL x 2 types x 2 parities x 64 lanes x 16 B
    uint4 *blk = tab + (moff[m] + (int64_t)tile * nk * NSPL * 4 * 64);
    const double dscale = BF ? 1.0 : kDerivScale;

    double l1 = 0, l2 = 0, d1 = 0, d2 = 0;
    int e = 1;
    if (live) {
        const double *sb = start + (size_t)m * jtab * nrp;
        l1 = sb[r];
        d1 = sb[(size_t)nrp + r];
        e = exps[(size_t)m * nrp + r];
    }
    int first = nk;
    for (int kc = 0; kc < nk; ++kc) {
        float v[2][2][16];  // [type][parity][k]
        bool any = false;
#pragma unroll
        for (int s = 0; s < KC; ++s) {
            const int l = m + kc * KC + s;
            if (l > m && l <= lmax) {
                const double4 cf = coef0[base + l];
                const double nl1 = cf.x * (x * l1) - cf.z * l2;
                const double nd1 = cf.x * fma(x, d1, -sn * l1) - cf.z * d2;
                l2 = l1;
                l1 = nl1;
                d2 = d1;
                d1 = nd1;
            }
            if (e > 0 && fmax(fmax(fabs(l1), fabs(l2)), fmax(fabs(d1), fabs(d2))) > kHi) {
                l1 *= kDown;
                l2 *= kDown;
                d1 *= kDown;
                d2 *= kDown;
                e -= 1;
            }
            const bool use = (e == 0) && (l <= lmax);
            v[0][s & 1][s >> 1] = use ? (float)l1 : 0.0f;
            v[1][s & 1][s >> 1] = use ? (float)(d1 * dscale) : 0.0f;
            any |= use && (l1 != 0.0 || d1 != 0.0);
        }
        if (any && kc < first) first = kc;
        // write: lane slot rl gets k 0..7, slot rl + 32 gets k 8..15
        uint4 *cb = blk + (int64_t)kc * NSPL * 4 * 64;
#pragma unroll
        for (int sp = 0; sp < NSPL; ++sp)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        T q[8];
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const float f = v[t][p][h * 8 + k];
                            const T hiv = (T)f;
                            q[k] = (sp == 0) ? hiv : (T)(f - (float)hiv);
                        }
                        uint4 w;
                        __builtin_memcpy(&w, q, 16);
                        if (live) cb[((sp * 2 + t) * 2 + p) * 64 + h * 32 + rl] = w;
                    }
    }
    // first non-empty chunk of the tile (lanes of the tile agree by min)
    atomicMin(&kstart[(size_t)m * ntile + tile], first);
}

// ----------------------------------------------------------- the GEMM ----
struct Cols {
    int PT, PS, nT, nE, nB, n1;
};
__host__ __device__ constexpr Cols cols_of(int N, bool hasb)
{
    Cols c{};
    c.PT = N / 2;
    c.PS = N / 2 + 1;
    c.nT = 2 * (c.PT + 1);
    c.nE = 2 * (c.PS + 1);
    c.nB = hasb ? 2 * (c.PS + 1) : 0;
    c.n1 = c.nT + c.nE + c.nB;
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
__device__ void family_coeffs(Jet<N> (&al)[P + 1], Jet<N> (&be)[P + 1], const Jet<N> &mcsc2, const Jet<N> &cot,
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

// Coefficients of one ring (theta) and m for T (ct*), W (cw*), X (cx*).
template <int N>
struct Coef {
    static constexpr int PT = N / 2, PS = N / 2 + 1;
    double ta[N + 1][PT + 1], tb[N + 1][PT + 1];
    double wa[N + 1][PS + 1], wb[N + 1][PS + 1], xa[N + 1][PS + 1], xb[N + 1][PS + 1];
};
template <int N>
__device__ void coefficients(double th, int m, bool pol, Coef<N> &C)
{
    constexpr int PT = N / 2, PS = N / 2 + 1;
    Jet<N> js, jc, csc, cot, jm2;
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
    {
        Jet<N> al[PT + 1], be[PT + 1];
#pragma unroll
        for (int p = 0; p <= PT; ++p)
#pragma unroll
            for (int i = 0; i <= N; ++i) al[p].c[i] = be[p].c[i] = 0.0;
        al[0].c[0] = 1.0;
        family_coeffs<N, PT>(al, be, jm2, cot, C.ta, C.tb);
    }
    if (!pol) return;
    Jet<N> cscot = jmul<N>(csc, cot, N);
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
        family_coeffs<N, PS>(al, be, jm2, cot, C.wa, C.wb);
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
            be[0].c[i] = -2.0 * dm * csc.c[i];
        }
        family_coeffs<N, PS>(al, be, jm2, cot, C.xa, C.xb);
    }
}

// Batched GEMM: one workgroup = 4 waves = 4 tiles of 32 ring pairs at one m;
// NBAT realizations, NB = ceil(NBAT * n1 / 32) column blocks in one pass.
template <bool BF, bool SPLIT, int N, bool POL, bool HASB, int NBAT>
__global__ __launch_bounds__(256) void k_legendre_tab(
    int lmax, int ntheta, int nrp, int rbeg, int ntile, const double *__restrict__ theta,
    const int *__restrict__ mcut, const int64_t *__restrict__ moff, const uint4 *__restrict__ tab,
    const int *__restrict__ kstart, const TabBatch batch)
{
    using T = typename H<BF>::T;
    using V = typename H<BF>::V;
    constexpr Cols C = cols_of(N, HASB);
    constexpr int NCOLS = NBAT * C.n1;
    constexpr int NB = (NCOLS + 31) / 32;
    constexpr int NSPL = SPLIT ? 2 : 1;

    __shared__ uint4 s_b[NSPL][NB][2][32][2];  // [split][block][parity][col][k-half] (8 values each)
    __shared__ float s_scale[NB * 32];         // per column: value = stored * 2^-scale (log2 in float)
    __shared__ float s_tr[4][32][4][33];       // epilogue transposition, per wave [ring][type*2+par][col]
    __shared__ int s_ks;

    const int m = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = blockIdx.x * 4 + wave;
    const int rl = lane & 31, hl = lane >> 5;
    const int r = rbeg + tile * TILE + rl;
    const bool live = (tile < ntile) && (r < nrp);
    const size_t base = (size_t)m * (2 * lmax + 1 - m) / 2;
    const int nk = (lmax - m + 1 + KC - 1) / KC;
    const size_t plane = (size_t)ntheta * (lmax + 1);

    // evanescent for every ring of the block: zeros
    const int mc = live ? mcut[r] + 2 : -1;
    if (!__syncthreads_or(m <= mc)) {
        if (live && hl == 0)
            for (int b = 0; b < NBAT; ++b)
                for (int j = 0; j <= N; ++j) {
                    const int rs = ntheta - 1 - r;
                    float2 *F[3] = {batch.FT[b], batch.FQ[b], batch.FU[b]};
                    for (int f = 0; f < (POL ? 3 : 1); ++f) {
                        F[f][j * plane + (size_t)r * (lmax + 1) + m] = make_float2(0.f, 0.f);
                        if (rs != r) F[f][j * plane + (size_t)rs * (lmax + 1) + m] = make_float2(0.f, 0.f);
                    }
                }
        return;
    }
    // first chunk with a non-zero table value over the 4 tiles
    if (tid == 0) s_ks = nk;
    __syncthreads();
    if (lane == 0 && tile < ntile) atomicMin(&s_ks, kstart[(size_t)m * ntile + tile]);

    // right-hand-side value of column c (realization b, local column cc) at l
    auto rhs = [&](int l, int c) -> double {
        const int b = c / C.n1, cc = c % C.n1;
        if (b >= NBAT || l > lmax) return 0.0;
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
    };

    // per-column power-of-two scale (FP16 only): largest |value| over l
    if (!BF) {
        __shared__ float s_mx[NB * 32];
        for (int c = tid; c < NB * 32; c += 256) s_mx[c] = 0.f;
        __syncthreads();
        for (int idx = tid; idx < (lmax - m + 1) * NCOLS; idx += 256) {
            const int l = m + idx / NCOLS, c = idx % NCOLS;
            const float v = (float)fabs(rhs(l, c));
            atomicMax((unsigned *)&s_mx[c], __float_as_uint(v));  // non-negative floats order as uints
        }
        __syncthreads();
        for (int c = tid; c < NB * 32; c += 256) {
            const float mx = s_mx[c];
            int ex = 0;
            if (mx > 0.f) frexpf(mx, &ex);  // mx in [2^(ex-1), 2^ex)
            s_scale[c] = (float)(14 - ex);  // stored = value * 2^(14 - ex) < 2^14
        }
    } else {
        for (int c = tid; c < NB * 32; c += 256) s_scale[c] = 0.f;
    }
    __syncthreads();
    const int ks = s_ks;

    floatx16 acc[NB][2][2];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[b][t][p][v] = 0.f;

    const uint4 *blk = (tile < ntile) ? tab + (moff[m] + (int64_t)tile * nk * NSPL * 4 * 64) : nullptr;
    for (int kc = ks; kc < nk; ++kc) {
        __syncthreads();
        // right-hand sides of this chunk: 32 l (16 per parity) x NB*32 columns
        for (int idx = tid; idx < NB * 32 * 2 * 2; idx += 256) {
            const int hh = idx & 1, p = (idx >> 1) & 1, c = (idx >> 2) % 32, b = idx / 128;
            const int col = b * 32 + c;
            const float sc = exp2f(s_scale[col]);
            T hi8[8], lo8[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int kk = hh * 8 + k;
                const int l = m + kc * KC + p + 2 * kk;
                const float f = (float)(rhs(l, col) * (double)sc);
                hi8[k] = (T)f;
                lo8[k] = (T)(f - (float)hi8[k]);
            }
            uint4 w;
            __builtin_memcpy(&w, hi8, 16);
            s_b[0][b][p][c][hh] = w;
            if (SPLIT) {
                __builtin_memcpy(&w, lo8, 16);
                s_b[NSPL - 1][b][p][c][hh] = w;
            }
        }
        __syncthreads();
        if (tile < ntile) {
            const uint4 *cb = blk + (int64_t)kc * NSPL * 4 * 64;
            V A[NSPL][2][2];
#pragma unroll
            for (int sp = 0; sp < NSPL; ++sp)
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        const uint4 w = cb[((sp * 2 + t) * 2 + p) * 64 + lane];
                        __builtin_memcpy(&A[sp][t][p], &w, 16);
                    }
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    V Bh, Bl;
                    uint4 w = s_b[0][b][p][rl][hl];
                    __builtin_memcpy(&Bh, &w, 16);
                    if (SPLIT) {
                        w = s_b[NSPL - 1][b][p][rl][hl];
                        __builtin_memcpy(&Bl, &w, 16);
                    }
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        if constexpr (BF) {
                            acc[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][t][p], Bh, acc[b][t][p], 0, 0, 0);
                            if constexpr (SPLIT) {
                                acc[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][t][p], Bl, acc[b][t][p], 0, 0, 0);
                                acc[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[NSPL - 1][t][p], Bh, acc[b][t][p], 0, 0, 0);
                            }
                        } else {
                            acc[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[0][t][p], Bh, acc[b][t][p], 0, 0, 0);
                            if constexpr (SPLIT) {
                                acc[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[0][t][p], Bl, acc[b][t][p], 0, 0, 0);
                                acc[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[NSPL - 1][t][p], Bh, acc[b][t][p], 0, 0, 0);
                            }
                        }
                    }
                }
        }
    }

    // ---- epilogue: per wave, transpose one 32-column block at a time ----
    Coef<N> cf;
    if (live) coefficients<N>(theta[r], m, POL, cf);
    const int rs = ntheta - 1 - r;
    const double dsc = BF ? 1.0 : 1.0 / kDerivScale;
    // output accumulators for this lane's ring: lanes 0..31 T, lanes 32..63 Q/U
    for (int bb = 0; bb < NBAT; ++bb) {
        // sums S[type*2+par][cc] of realization bb, gathered block by block
        double S[4][C.n1];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < C.n1; ++c) S[q][c] = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int c0 = b * 32;
            if (c0 + 32 <= bb * C.n1 || c0 >= (bb + 1) * C.n1) continue;
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int vv = 0; vv < 16; ++vv) {
                        const int row = 8 * (vv >> 2) + 4 * hl + (vv & 3);
                        s_tr[wave][row][t * 2 + p][rl] = acc[b][t][p][vv];
                    }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < C.n1; ++c) {
                const int col = bb * C.n1 + c;
                if (col < c0 || col >= c0 + 32) continue;
                const double isc = exp2(-(double)s_scale[col]);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    S[q][c] = (double)s_tr[wave][rl][q][col - c0] * isc * ((q >> 1) ? dsc : 1.0);
            }
        }
        if (!live) continue;
        auto nsum = [&](int type, int c) { return S[type * 2][c] + S[type * 2 + 1][c]; };
        auto dsum = [&](int type, int c) { return S[type * 2][c] - S[type * 2 + 1][c]; };
        float2 *FT = batch.FT[bb];
        if (hl == 0) {
#pragma unroll
            for (int j = 0; j <= N; ++j) {
                double nre = 0, nim = 0, sre = 0, sim = 0;
#pragma unroll
                for (int p = 0; p <= C.PT; ++p) {
                    nre += cf.ta[j][p] * nsum(0, 2 * p) + cf.tb[j][p] * nsum(1, 2 * p);
                    nim += cf.ta[j][p] * nsum(0, 2 * p + 1) + cf.tb[j][p] * nsum(1, 2 * p + 1);
                    sre += cf.ta[j][p] * dsum(0, 2 * p) + cf.tb[j][p] * dsum(1, 2 * p);
                    sim += cf.ta[j][p] * dsum(0, 2 * p + 1) + cf.tb[j][p] * dsum(1, 2 * p + 1);
                }
                FT[j * plane + (size_t)r * (lmax + 1) + m] = make_float2((float)nre, (float)nim);
                if (rs != r) {
                    const double sg = (j & 1) ? -1.0 : 1.0;
                    FT[j * plane + (size_t)rs * (lmax + 1) + m] = make_float2((float)(sg * sre), (float)(sg * sim));
                }
            }
        } else if constexpr (POL) {
            float2 *FQ = batch.FQ[bb], *FU = batch.FU[bb];
#pragma unroll
            for (int j = 0; j <= N; ++j) {
                double ewn[2] = {0, 0}, exn[2] = {0, 0}, bwn[2] = {0, 0}, bxn[2] = {0, 0};
                double ews[2] = {0, 0}, exs[2] = {0, 0}, bws[2] = {0, 0}, bxs[2] = {0, 0};
#pragma unroll
                for (int p = 0; p <= C.PS; ++p)
#pragma unroll
                    for (int ri = 0; ri < 2; ++ri) {
                        const int ce = C.nT + 2 * p + ri;
                        ewn[ri] += cf.wa[j][p] * nsum(0, ce) + cf.wb[j][p] * nsum(1, ce);
                        exn[ri] += cf.xa[j][p] * nsum(0, ce) + cf.xb[j][p] * nsum(1, ce);
                        ews[ri] += cf.wa[j][p] * dsum(0, ce) + cf.wb[j][p] * dsum(1, ce);
                        exs[ri] += cf.xa[j][p] * dsum(0, ce) + cf.xb[j][p] * dsum(1, ce);
                        if constexpr (HASB) {
                            const int cb_ = C.nT + C.nE + 2 * p + ri;
                            bwn[ri] += cf.wa[j][p] * nsum(0, cb_) + cf.wb[j][p] * nsum(1, cb_);
                            bxn[ri] += cf.xa[j][p] * nsum(0, cb_) + cf.xb[j][p] * nsum(1, cb_);
                            bws[ri] += cf.wa[j][p] * dsum(0, cb_) + cf.wb[j][p] * dsum(1, cb_);
                            bxs[ri] += cf.xa[j][p] * dsum(0, cb_) + cf.xb[j][p] * dsum(1, cb_);
                        }
                    }
                const double sg = (j & 1) ? -1.0 : 1.0;
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) {
                    ews[ri] *= sg;
                    bws[ri] *= sg;
                    exs[ri] *= -sg;
                    bxs[ri] *= -sg;
                }
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
}

template <bool BF, bool SPLIT>
hipError_t build_BS(Plan &p)
{
    dim3 grid((p.ntile + 1) / 2, p.lmax + 1);
    hipLaunchKernelGGL((k_build_tab<BF, SPLIT>), grid, dim3(64), 0, p.stream, p.lmax, p.nrp, p.rpole, p.ntile, p.jtab,
                       (const double2 *)p.trig.ptr, (const double4 *)p.coef0.ptr, (const double *)p.start.ptr,
                       (const int *)p.exps.ptr, (const int64_t *)p.moff.ptr, (uint4 *)p.tab.ptr, (int *)p.kstart.ptr);
    return hipGetLastError();
}

template <bool BF, bool SPLIT, int N, bool POL, bool HASB, int NBAT>
hipError_t gemm_launch(Plan &p, const TabBatch &b)
{
    if constexpr ((NBAT * cols_of(N, HASB).n1 + 31) / 32 > 4) {
        return hipErrorInvalidValue;
    } else {
        dim3 grid((p.ntile + 3) / 4, p.lmax + 1);
        hipLaunchKernelGGL((k_legendre_tab<BF, SPLIT, N, POL, HASB, NBAT>), grid, dim3(256), 0, p.stream, p.lmax,
                           p.ntheta, p.nrp, p.rpole, p.ntile, (const double *)p.theta.ptr, (const int *)p.mcut.ptr,
                           (const int64_t *)p.moff.ptr, (const uint4 *)p.tab.ptr, (const int *)p.kstart.ptr, b);
        return hipGetLastError();
    }
}

template <bool BF, bool SPLIT, int N, bool POL, bool HASB>
hipError_t gemm_nbat(Plan &p, const TabBatch &b)
{
    switch (b.n) {
    case 1: return gemm_launch<BF, SPLIT, N, POL, HASB, 1>(p, b);
    case 2: return gemm_launch<BF, SPLIT, N, POL, HASB, 2>(p, b);
    case 3: return gemm_launch<BF, SPLIT, N, POL, HASB, 3>(p, b);
    case 4: return gemm_launch<BF, SPLIT, N, POL, HASB, 4>(p, b);
    case 5: return gemm_launch<BF, SPLIT, N, POL, HASB, 5>(p, b);
    default: return hipErrorInvalidValue;
    }
}

template <bool BF, bool SPLIT>
hipError_t gemm_form(Plan &p, const TabBatch &b)
{
    const bool hasb = p.pol && b.B[0] != nullptr;
#define TL_CASE(NN)                                                              \
    case NN:                                                                     \
        if (!p.pol) return gemm_nbat<BF, SPLIT, NN, false, false>(p, b);         \
        if (hasb) return gemm_nbat<BF, SPLIT, NN, true, true>(p, b);             \
        return gemm_nbat<BF, SPLIT, NN, true, false>(p, b);
    switch (p.order) {
        TL_CASE(0)
        TL_CASE(1)
        TL_CASE(2)
        TL_CASE(3)
        TL_CASE(4)
        TL_CASE(5)
        TL_CASE(6)
    default: return hipErrorInvalidValue;
    }
#undef TL_CASE
}

}  // namespace

int tab_max_batch(int order, bool pol, bool hasb)
{
    if (order > 6) return 0;
    const Cols c = cols_of(order, pol && hasb);
    const int n1 = pol ? c.n1 : c.nT;
    int nb = 0;
    while (nb < 5 && ((nb + 1) * n1 + 31) / 32 <= 4) ++nb;
    return nb;
}

size_t tab_bytes(int lmax, int ntile, bool split, std::vector<int64_t> &moff)
{
    moff.assign((size_t)lmax + 2, 0);
    int64_t off = 0;
    for (int m = 0; m <= lmax; ++m) {
        moff[m] = off;
        const int nk = (lmax - m + 1 + KC - 1) / KC;
        off += (int64_t)ntile * nk * (split ? 2 : 1) * 4 * 64;  // uint4 units
    }
    moff[lmax + 1] = off;
    return (size_t)off * 16;
}

hipError_t launch_build_tab(Plan &p)
{
    switch (p.precision) {
    case TL_BF16: return build_BS<true, false>(p);
    case TL_FP16: return build_BS<false, false>(p);
    case TL_BF16X3: return build_BS<true, true>(p);
    case TL_FP16X2: return build_BS<false, true>(p);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_legendre_tab(Plan &p, const TabBatch &b)
{
    switch (p.precision) {
    case TL_BF16: return gemm_form<true, false>(p, b);
    case TL_FP16: return gemm_form<false, false>(p, b);
    case TL_BF16X3: return gemm_form<true, true>(p, b);
    case TL_FP16X2: return gemm_form<false, true>(p, b);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tl
