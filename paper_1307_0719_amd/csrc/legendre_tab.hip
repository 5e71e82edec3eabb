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
// l = l0 + par + 2 (8 (i / 32) + q), q = 0..7.  Each call builds the
// right-hand sides of up to six realizations (k_tab_rhs), streams the blocks
// against them (k_legendre_tab, coalesced 16-byte lane loads; column sums to
// HBM) and turns the sums into rows with the FP64 L-power epilogue
// (k_tab_epi) -- the FP64 recursion is paid once per plan, the table once per
// batch.
//
// Precision forms: FP16 / BF16 store one table and take one MFMA per
// product; BF16X3 / FP16X2 store hi and lo tables and take hi*hi + hi*lo +
// lo*hi.  FP16 operands are scaled by powers of two: lam' by 2^-7 in the
// table, every right-hand-side column of a given m by the power of two that
// brings its largest entry to [2^13, 2^14); lam and lam' by the plan's powers
// of two 2^lam_e0, 2^lam_e1 (their bounds just below 2^15, so that the lo part
// of a split value stays a normal FP16 number).
#include <algorithm>

#include "lpower.h"
#include "tl_internal.h"

namespace tl {

namespace {

using namespace lp;

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr double kHi = 0x1p256;
constexpr double kDown = 0x1p-512;
constexpr int KC = 32;          // l values per table chunk (16 per parity)
constexpr int TILE = 32;        // ring pairs per table tile

// ------------------------------------------------------------ builder ----
// One lane per ring pair, 64 lanes = two 32-ring tiles of one m.  Writes, for
// every 32-l chunk, the blocks [type][parity] (and [hi/lo] when split), and
// the first chunk holding a non-zero value per (m, tile).
template <bool BF, bool SPLIT>
__global__ __launch_bounds__(64) void k_build_tab(int lmax, int nrp, int rbeg, int ntile, int jtab, int e0, int e1,
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
    const double lscale = ldexp(1.0, e0), dscale = ldexp(1.0, e1);

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
            v[0][s & 1][s >> 1] = use ? (float)(l1 * lscale) : 0.0f;
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
                            const float f = opaque(v[t][p][h * 8 + k]);
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

// All columns of realization b at degree l (layout of cols_of: T, E, B,
// the lensing potential), from the per-l factors L = l(l+1) and N_l.
template <int N, bool POL, bool HASB>
__device__ __forceinline__ void rhs_row(const TabBatch &batch, int b, size_t idx, double L, double nl,
                                        double (&v)[cols_of(N, POL, HASB, true).n1])
{
    constexpr Cols C = cols_of(N, POL, HASB, true);
    {
        const double2 a = batch.T[b][idx];
        double w = 1.0;
#pragma unroll
        for (int p = 0; p <= C.PT; ++p, w *= L) {
            v[2 * p] = w * a.x;
            v[2 * p + 1] = w * a.y;
        }
    }
    if constexpr (POL) {
        const double2 a = batch.E[b][idx];
        double w = nl;
#pragma unroll
        for (int p = 0; p <= C.PS; ++p, w *= L) {
            v[C.nT + 2 * p] = w * a.x;
            v[C.nT + 2 * p + 1] = w * a.y;
        }
        if constexpr (HASB) {
            const double2 e = batch.B[b][idx];
            double u = nl;
#pragma unroll
            for (int p = 0; p <= C.PS; ++p, u *= L) {
                v[C.nT + C.nE + 2 * p] = u * e.x;
                v[C.nT + C.nE + 2 * p + 1] = u * e.y;
            }
        }
    }
    const double2 f = batch.P[b] ? batch.P[b][idx] : make_double2(0.0, 0.0);
    v[C.n1 - 2] = f.x;
    v[C.n1 - 1] = f.y;
}

// Right-hand sides of one call, built once per m (one workgroup per m) in
// the B-operand layout of v_mfma_f32_32x32x16: per (m, 32-l chunk) the blocks
// [split][column block][parity][k-half][column] of 8 values, so that lane i of
// a wave loads entry i of a block.  A thread takes one l (the factors L and
// N_l once) for half of the realizations; 128-l slices pass through LDS to
// be regrouped into the 8-value entries.  FP16: every column of a given m is
// scaled by the power of two 2^e that brings its largest |value| to
// [2^13, 2^14); e goes to colexp[m][column].
template <bool BF, bool SPLIT, int N, bool POL, bool HASB, int NBMAX>
__global__ __launch_bounds__(256) void k_tab_rhs(int lmax, int ntile, int NBAT, const int64_t *__restrict__ moff,
                                                 const TabBatch batch, uint4 *__restrict__ rhs,
                                                 float *__restrict__ colexp)
{
    using T = typename H<BF>::T;
    constexpr Cols C = cols_of(N, POL, HASB, true);
    const int NCOLS = NBAT * C.n1;
    const int NB = (NCOLS + 31) / 32;
    constexpr int NSPL = SPLIT ? 2 : 1;
    const int RCH = NSPL * NB * 128;                // uint4 per chunk
    constexpr int LCH = NBMAX <= 4 ? 128 : 32;      // l per LDS slice
    constexpr int CW = NBMAX * 32 + 2;              // LDS row (columns, padded)
    __shared__ float s_ex[NBMAX * 32];
    __shared__ T s_v[NSPL][LCH][CW];
    const int m = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const size_t base = (size_t)m * (2 * lmax + 1 - m) / 2;
    const int nk = (lmax - m + 1 + KC - 1) / KC;
    const int64_t cum = moff[m] / ((int64_t)ntile * NSPL * 256);  // chunks of all m' < m
    uint4 *out = rhs + cum * RCH;
    auto factors = [&](int l, double &L, double &nl) {
        L = (double)l * (double)(l + 1);
        nl = (POL && l >= 2) ? 1.0 / sqrt((double)(l - 1) * l * (double)(l + 1) * (double)(l + 2)) : 0.0;
    };

    for (int c = tid; c < NB * 32; c += 256) s_ex[c] = 0.f;
    __syncthreads();
    if constexpr (!BF) {
        // column maxima: per-thread running maxima, wave reduction, LDS max
        for (int b0 = tid >> 7; b0 < NBAT; b0 += 2) {
            float mx[C.n1];
#pragma unroll
            for (int c = 0; c < C.n1; ++c) mx[c] = 0.f;
            for (int l = m + (tid & 127); l <= lmax; l += 128) {
                double L, nl, v[C.n1];
                factors(l, L, nl);
                rhs_row<N, POL, HASB>(batch, b0, base + l, L, nl, v);
#pragma unroll
                for (int c = 0; c < C.n1; ++c) mx[c] = fmaxf(mx[c], (float)fabs(v[c]));
            }
#pragma unroll
            for (int c = 0; c < C.n1; ++c) {
                float x = mx[c];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) x = fmaxf(x, __shfl_xor(x, off));
                if (lane == 0) atomicMax((unsigned *)&s_ex[b0 * C.n1 + c], __float_as_uint(x));  // x >= 0
            }
        }
        __syncthreads();
        for (int c = tid; c < NB * 32; c += 256) {
            const float mx = s_ex[c];
            int ex = 0;
            if (mx > 0.f) frexpf(mx, &ex);  // mx in [2^(ex-1), 2^ex)
            s_ex[c] = (float)(14 - ex);     // stored = value * 2^(14 - ex) < 2^14
        }
        __syncthreads();
    }
    for (int c = tid; c < NB * 32; c += 256) colexp[(size_t)m * NB * 32 + c] = s_ex[c];

    for (int l0 = m; l0 <= lmax; l0 += LCH) {
        __syncthreads();
        {
            const int li = tid & (LCH - 1), l = l0 + li;
            for (int b0 = tid / LCH; b0 < NBAT; b0 += 256 / LCH) {
                double v[C.n1];
                if (l <= lmax) {
                    double L, nl;
                    factors(l, L, nl);
                    rhs_row<N, POL, HASB>(batch, b0, base + l, L, nl, v);
                } else {
#pragma unroll
                    for (int c = 0; c < C.n1; ++c) v[c] = 0.0;
                }
#pragma unroll
                for (int c = 0; c < C.n1; ++c) {
                    const int col = b0 * C.n1 + c;
                    // the column's power of two, applied exactly (s_ex holds integers)
                    const float f = opaque((float)ldexp(v[c], (int)s_ex[col]));
                    const T hi = (T)f;
                    s_v[0][li][col] = hi;
                    if constexpr (SPLIT) s_v[1][li][col] = (T)(f - (float)hi);
                }
            }
            if (tid < LCH)
                for (int col = NCOLS; col < NB * 32; ++col)
#pragma unroll
                    for (int sp = 0; sp < NSPL; ++sp) s_v[sp][tid][col] = (T)0.f;
        }
        __syncthreads();
        const int kc0 = (l0 - m) / KC;
        const int PER = RCH;  // uint4 entries per chunk
        for (int idx = tid; idx < (LCH / KC) * PER; idx += 256) {
            const int q = idx / PER, w = idx % PER;
            const int kc = kc0 + q;
            if (kc >= nk) continue;
            const int c = w & 31, hh = (w >> 5) & 1, p = (w >> 6) & 1, rest = w >> 7;
            const int b = rest % NB, sp = rest / NB;
            T v8[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v8[k] = s_v[sp][q * KC + p + 2 * (hh * 8 + k)][b * 32 + c];
            uint4 wv;
            __builtin_memcpy(&wv, v8, 16);
            out[(int64_t)kc * RCH + w] = wv;
        }
    }
}

// Column sums of a table pass with nbat realizations, [m][ring pair - rbeg]
// [realization][type * 2 + parity][column of the realization]: the blocks a
// wave writes for one (m, ring pair) share cache lines.
__device__ __forceinline__ size_t colsum_offset(int bb, int rp, int m, int nrn, int nbat, int n1)
{
    return (((size_t)m * nrn + rp) * nbat + bb) * 4 * n1;
}

// Batched GEMM: one workgroup = 4 waves = 4 tiles of 32 ring pairs at one m;
// NBAT realizations, NB = ceil(NBAT * n1 / 32) column blocks in one pass.  The
// table streams from HBM once per pass; the right-hand sides of one m (built
// by k_tab_rhs) are shared by all its tiles, and the workgroups of one m run
// on one XCD (m = xcd + 8 i) so they are read from HBM once.  Each wave walks
// its own tile from its first non-empty chunk; nothing in the main loop
// synchronizes the workgroup.  The column sums, scaled back by the column
// powers of two, go to HBM straight from the accumulators (lanes hold
// consecutive columns): sums[m][ring pair - rbeg][realization][type*2 +
// parity][column of the realization]; k_tab_epi turns them into the rows.
template <bool BF, bool SPLIT, int NB>
__global__ __launch_bounds__(256) void k_legendre_tab(int lmax, int nrp, int rbeg, int ntile, int ngrp, int e0, int e1,
                                                      int n1, int NCOLS, const int *__restrict__ mcut,
                                                      const int64_t *__restrict__ moff, const uint4 *__restrict__ tab,
                                                      const int *__restrict__ kstart, const uint4 *__restrict__ rhs,
                                                      const float *__restrict__ colexp, float *__restrict__ sums)
{
    using V = typename H<BF>::V;
    constexpr int NSPL = SPLIT ? 2 : 1;
    constexpr int RCH = NSPL * NB * 128;

    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int m = xcd + 8 * (q / ngrp);
    if (m > lmax) return;  // whole workgroup
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = (q % ngrp) * 4 + wave;
    const int rl = lane & 31, hl = lane >> 5;
    const int r = rbeg + tile * TILE + rl;
    const bool live = (tile < ntile) && (r < nrp);
    const int nk = (lmax - m + 1 + KC - 1) / KC;

    // evanescent for every ring of the block: nothing to sum (the epilogue
    // writes zeros past each ring's cut)
    const int mc = live ? mcut[r] + 2 : -1;
    if (!__syncthreads_or(m <= mc)) return;

    floatx16 acc[NB][2][2];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[b][t][p][v] = 0.f;

    if (tile < ntile) {
        // The table and the right-hand sides stream with PF chunks in flight
        // per wave (the loop is bound by memory latency, not by the matrix
        // cores): loads retire in order, so the chunk consumed now must be
        // the oldest one in flight, for both operands.
        constexpr int PFA = SPLIT ? 2 : (NB >= 3 ? 3 : 4);  // table chunks in flight
        constexpr int PFB = SPLIT ? 1 : PFA;                 // right-hand-side chunks (from L2)
        constexpr int PG = PFA;  // PFB divides PFA
        constexpr int AW = NSPL * 4;  // uint4 per lane per chunk
        const int ks = __builtin_amdgcn_readfirstlane(kstart[(size_t)m * ntile + tile]);
        const uint4 *blk = tab + (moff[m] + (int64_t)tile * nk * AW * 64) + lane;
        const int64_t cum = moff[m] / ((int64_t)ntile * NSPL * 256);
        const uint4 *rb = rhs + cum * RCH + lane;
        uint4 Ab[PFA][AW];
        uint4 Bb[PFB][NSPL][NB][2];
        auto loadA = [&](uint4 (&dst)[AW], int kc) {
            const uint4 *cb = blk + (int64_t)kc * AW * 64;
#pragma unroll
            for (int u = 0; u < AW; ++u) {
                const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(cb + u * 64));
                __builtin_memcpy(&dst[u], &v, 16);
            }
        };
        auto loadB = [&](uint4 (&dst)[NSPL][NB][2], int kc) {
            const uint4 *rc = rb + (int64_t)kc * RCH;
#pragma unroll
            for (int sp = 0; sp < NSPL; ++sp)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int p = 0; p < 2; ++p) dst[sp][b][p] = rc[((sp * NB + b) * 2 + p) * 64];
        };
        // issue order B(k), A(k) for the first chunks, as in the loop
#pragma unroll
        for (int u = 0; u < PFA; ++u) {
            if (u < PFB && ks + u < nk) loadB(Bb[u], ks + u);
            if (ks + u < nk) loadA(Ab[u], ks + u);
        }
        // one chunk: operands from slot u, refill the slots PFB / PFA chunks ahead
        auto chunk = [&](const uint4 (&Au)[AW], const uint4 (&Bu)[NSPL][NB][2]) {
            V A[NSPL][2][2], Bv[NSPL][NB][2];
#pragma unroll
            for (int sp = 0; sp < NSPL; ++sp) {
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int p = 0; p < 2; ++p) __builtin_memcpy(&A[sp][t][p], &Au[(sp * 2 + t) * 2 + p], 16);
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int p = 0; p < 2; ++p) __builtin_memcpy(&Bv[sp][b][p], &Bu[sp][b][p], 16);
            }
            return [=](floatx16 (&ac)[NB][2][2]) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        const V Bh = Bv[0][b][p];
                        const V Bl = Bv[NSPL - 1][b][p];
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            if constexpr (BF) {
                                ac[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][t][p], Bh, ac[b][t][p], 0, 0, 0);
                                if constexpr (SPLIT) {
                                    ac[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][t][p], Bl, ac[b][t][p], 0, 0, 0);
                                    ac[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[NSPL - 1][t][p], Bh, ac[b][t][p], 0, 0, 0);
                                }
                            } else {
                                ac[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[0][t][p], Bh, ac[b][t][p], 0, 0, 0);
                                if constexpr (SPLIT) {
                                    ac[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[0][t][p], Bl, ac[b][t][p], 0, 0, 0);
                                    ac[b][t][p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A[NSPL - 1][t][p], Bh, ac[b][t][p], 0, 0, 0);
                                }
                            }
                        }
                    }
            };
        };
        // whole groups of PG chunks (one back edge), then the tail
        int k0 = ks;
        for (; k0 + PG <= nk; k0 += PG) {
#pragma unroll
            for (int u = 0; u < PG; ++u) {
                auto mm = chunk(Ab[u % PFA], Bb[u % PFB]);
                if (k0 + u + PFB < nk) loadB(Bb[u % PFB], k0 + u + PFB);
                if (k0 + u + PFA < nk) loadA(Ab[u % PFA], k0 + u + PFA);
                mm(acc);
            }
        }
#pragma unroll
        for (int u = 0; u < PG; ++u)
            if (k0 + u < nk) {
                auto mm = chunk(Ab[u % PFA], Bb[u % PFB]);
                if (k0 + u + PFB < nk) loadB(Bb[u % PFB], k0 + u + PFB);
                mm(acc);
            }
    }

    if (tile >= ntile) return;
    const int nrn = nrp - rbeg;
    const float usc[2] = {ldexpf(1.f, -e0), ldexpf(1.f, -e1)};  // exact: powers of two
    const float *cex = colexp + (size_t)m * NB * 32;
    const int rp0 = tile * TILE + 4 * hl;  // ring pair of accumulator slot 0
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int col = b * 32 + rl;
        if (col >= NCOLS) continue;
        const int bb = col / n1, c = col % n1;
        const float isc = ldexpf(1.f, -(int)cex[col]);  // exact: powers of two
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int rp = rp0 + 8 * (v >> 2) + (v & 3);
            if (rp >= nrn) continue;
            float *base = sums + colsum_offset(bb, rp, m, nrn, NCOLS / n1, n1) + c;
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int p = 0; p < 2; ++p)  // non-temporal: read once by the epilogue
                    __builtin_nontemporal_store(acc[b][t][p][v] * isc * usc[t], &base[(t * 2 + p) * n1]);
        }
    }
}

// Non-temporal store of a complex value: the epilogue's rows are written
// once and read by the ring FFTs (measured 1.6 ms less per headline step
// than plain stores).
template <typename T2>
__device__ __forceinline__ void nts(T2 *p, T2 v)
{
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

// Epilogue of the table GEMM: one thread per (m, ring pair), consecutive m
// across a wave (coalesced row writes).  The FP64 coefficients of a (ring,
// m) are formed once and applied to every realization's column sums: T and
// the lensing potential below the ring's cut, Q/U two past it (spin-2
// functions reach |m - 2|); zeros beyond.
template <int N, bool POL, bool HASB>
__global__ __launch_bounds__(256) void k_tab_epi(int lmax, int ntheta, int nrp, int rbeg, int NBAT,
                                                 const double *__restrict__ theta, const int *__restrict__ mcut,
                                                 const float *__restrict__ sums, const TabBatch batch)
{
    constexpr Cols C = cols_of(N, POL, HASB, true);
    const int m = blockIdx.x * 64 + (threadIdx.x & 63);
    const int r = rbeg + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (m > lmax || r >= nrp) return;
    const int nrn = nrp - rbeg;
    const size_t plane = (size_t)ntheta * (lmax + 1);
    const int rs = ntheta - 1 - r;
    // south ring row; on the equator ring (rs == r) the north value is
    // stored there again (a select, not a branch around the stores)
    const bool eq = rs == r;
    const size_t on = (size_t)r * (lmax + 1) + m, os = (size_t)rs * (lmax + 1) + m;
    const size_t sstride = (size_t)4 * C.n1;  // one realization's sums
    const float *S0 = sums + colsum_offset(0, r - rbeg, m, nrn, NBAT, C.n1);
    const int mc = mcut[r];
    const double th = theta[r];

    // A thread's column sums of one realization: [type*2+parity][column],
    // read as float2 (columns come in Re / Im pairs) for the columns a phase
    // needs: [c0, c0 + nc) and, with tail, the potential's last two.
    constexpr int NT2 = C.nT / 2, NQ2 = (C.nE + C.nB) / 2;
    auto load_cols = [&](const float *S, int c0, auto &dst, bool tail) {
        constexpr int W = sizeof(dst[0]) / sizeof(float2);
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
#pragma unroll
            for (int i = 0; i < W - (tail ? 1 : 0); ++i)
                dst[q4][i] = *reinterpret_cast<const float2 *>(S + q4 * C.n1 + c0 + 2 * i);
            if (tail) dst[q4][W - 1] = *reinterpret_cast<const float2 *>(S + q4 * C.n1 + C.n1 - 2);
        }
    };
    {   // T and the lensing potential
        const bool act = m <= mc;
        CoefT<N> cf;
        if (act) coefficients_T<N>(th, m, cf);
        for (int bb = 0; bb < NBAT; ++bb) {
            float2 R[4][NT2 + 1];  // T columns, then the potential's
            if (act) load_cols(S0 + (size_t)bb * sstride, 0, R, true);
            auto val = [&](int q4, int c) -> double {
                const int i = c < C.nT ? c >> 1 : NT2;
                return (c & 1) ? (double)R[q4][i].y : (double)R[q4][i].x;
            };
            auto nsum = [&](int type, int c) { return val(type * 2, c) + val(type * 2 + 1, c); };
            auto dsum = [&](int type, int c) { return val(type * 2, c) - val(type * 2 + 1, c); };
            float2 *FT = batch.FT[bb];
#pragma unroll
            for (int j = 0; j <= N; ++j) {
                double nre = 0, nim = 0, sre = 0, sim = 0;
                if (act) {
#pragma unroll
                    for (int p = 0; p <= C.PT; ++p) {
                        nre += cf.ta[j][p] * nsum(0, 2 * p) + cf.tb[j][p] * nsum(1, 2 * p);
                        nim += cf.ta[j][p] * nsum(0, 2 * p + 1) + cf.tb[j][p] * nsum(1, 2 * p + 1);
                        sre += cf.ta[j][p] * dsum(0, 2 * p) + cf.tb[j][p] * dsum(1, 2 * p);
                        sim += cf.ta[j][p] * dsum(0, 2 * p + 1) + cf.tb[j][p] * dsum(1, 2 * p + 1);
                    }
                }
                const float2 vn = make_float2((float)nre, (float)nim);
                const double sg = (j & 1) ? -1.0 : 1.0;
                nts(&FT[j * plane + on], vn);
                nts(&FT[j * plane + os], eq ? vn : make_float2((float)(sg * sre), (float)(sg * sim)));
            }
            // lensing potential: the lam sums (j = 0) and lam' sums (j = 1)
            // themselves, in the deflection's FP64 rows
            if (double2 *FP = batch.FP[bb]) {
                const int c = C.n1 - C.nP;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const double2 vn = act ? make_double2(nsum(j, c), nsum(j, c + 1)) : make_double2(0.0, 0.0);
                    const double sg = j ? -1.0 : 1.0;
                    const double2 vs =
                        act ? make_double2(sg * dsum(j, c), sg * dsum(j, c + 1)) : make_double2(0.0, 0.0);
                    nts(&FP[j * plane + on], vn);
                    nts(&FP[j * plane + os], eq ? vn : vs);
                }
            }
        }
    }
    if constexpr (POL) {
        const bool act = m <= mc + 2;
        CoefP<N> cf;
        if (act) coefficients_P<N>(th, m, cf);
        for (int bb = 0; bb < NBAT; ++bb) {
            float2 R[4][NQ2];  // E (and B) columns
            if (act) load_cols(S0 + (size_t)bb * sstride, C.nT, R, false);
            auto val = [&](int q4, int c) -> double {
                const int i = (c - C.nT) >> 1;
                return (c & 1) ? (double)R[q4][i].y : (double)R[q4][i].x;
            };
            auto nsum = [&](int type, int c) { return val(type * 2, c) + val(type * 2 + 1, c); };
            auto dsum = [&](int type, int c) { return val(type * 2, c) - val(type * 2 + 1, c); };
            float2 *FQ = batch.FQ[bb], *FU = batch.FU[bb];
#pragma unroll
            for (int j = 0; j <= N; ++j) {
                double ewn[2] = {0, 0}, exn[2] = {0, 0}, bwn[2] = {0, 0}, bxn[2] = {0, 0};
                double ews[2] = {0, 0}, exs[2] = {0, 0}, bws[2] = {0, 0}, bxs[2] = {0, 0};
                if (act) {
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
                }
                const double sg = (j & 1) ? -1.0 : 1.0;
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) {
                    ews[ri] *= sg;
                    bws[ri] *= sg;
                    exs[ri] *= -sg;
                    bxs[ri] *= -sg;
                }
                const float2 qn = make_float2((float)(-(ewn[0] - bxn[1])), (float)(-(ewn[1] + bxn[0])));
                const float2 un = make_float2((float)(-exn[1] - bwn[0]), (float)(exn[0] - bwn[1]));
                nts(&FQ[j * plane + on], qn);
                nts(&FU[j * plane + on], un);
                nts(&FQ[j * plane + os], eq ? qn : make_float2((float)(-(ews[0] - bxs[1])), (float)(-(ews[1] + bxs[0]))));
                nts(&FU[j * plane + os], eq ? un : make_float2((float)(-exs[1] - bws[0]), (float)(exs[0] - bws[1])));
            }
        }
    }
}

template <bool BF, bool SPLIT>
hipError_t build_BS(Plan &p)
{
    dim3 grid((p.ntile + 1) / 2, p.lmax + 1);
    hipLaunchKernelGGL((k_build_tab<BF, SPLIT>), grid, dim3(64), 0, p.stream, p.lmax, p.nrp, p.rpole, p.ntile, p.jtab,
                       p.lam_e0, p.lam_e1,
                       (const double2 *)p.trig.ptr, (const double4 *)p.coef0.ptr, (const double *)p.start.ptr,
                       (const int *)p.exps.ptr, (const int64_t *)p.moff.ptr, (uint4 *)p.tab.ptr, (int *)p.kstart.ptr);
    return hipGetLastError();
}

// The table pass over NB column blocks (ncols columns, n1 per realization).
template <bool BF, bool SPLIT, int NB>
hipError_t gemm_pass(Plan &p, int n1, int ncols)
{
    const int m8 = (p.lmax + 1 + 7) / 8;
    const int ngrp = (p.ntile + 3) / 4;
    hipLaunchKernelGGL((k_legendre_tab<BF, SPLIT, NB>), dim3(8 * m8 * ngrp), dim3(256), 0, p.stream, p.lmax, p.nrp,
                       p.rpole, p.ntile, ngrp, p.lam_e0, p.lam_e1, n1, ncols, (const int *)p.mcut.ptr,
                       (const int64_t *)p.moff.ptr, (const uint4 *)p.tab.ptr, (const int *)p.kstart.ptr,
                       (const uint4 *)p.rhs.ptr, (const float *)p.colexp.ptr, (float *)p.tabsum.ptr);
    return hipGetLastError();
}

template <bool BF, bool SPLIT, int N, bool POL, bool HASB>
hipError_t gemm_launch(Plan &p, const TabBatch &b, int part)
{
    constexpr int n1 = cols_of(N, POL, HASB, true).n1;
    const int nbat = b.n;
    const int ncols = nbat * n1;
    const int NB = (ncols + 31) / 32;
    if (nbat < 1 || nbat > kTabMaxBatch || NB > kTabMaxBlocks) return hipErrorInvalidValue;
    if ((size_t)NB > p.rhs_nb) return hipErrorInvalidValue;  // buffers sized at plan time
    if (part == 0) {
        hipLaunchKernelGGL((k_tab_rhs<BF, SPLIT, N, POL, HASB, kTabMaxBlocks>), dim3(p.lmax + 1), dim3(256), 0,
                           p.stream, p.lmax, p.ntile, nbat, (const int64_t *)p.moff.ptr, b, (uint4 *)p.rhs.ptr,
                           (float *)p.colexp.ptr);
        return hipGetLastError();
    }
    if (part == 1) {
        switch (NB) {
        case 1: return gemm_pass<BF, SPLIT, 1>(p, n1, ncols);
        case 2: return gemm_pass<BF, SPLIT, 2>(p, n1, ncols);
        case 3: return gemm_pass<BF, SPLIT, 3>(p, n1, ncols);
        case 4: return gemm_pass<BF, SPLIT, 4>(p, n1, ncols);
        default: return hipErrorInvalidValue;
        }
    }
    const int nrn = p.nrp - p.rpole;
    if ((size_t)(p.lmax + 1) * nrn * ncols * 4 * sizeof(float) > p.tabsum.bytes) return hipErrorInvalidValue;
    dim3 grid((p.lmax + 1 + 63) / 64, (nrn + 3) / 4);
    hipLaunchKernelGGL((k_tab_epi<N, POL, HASB>), grid, dim3(256), 0, p.stream, p.lmax, p.ntheta, p.nrp, p.rpole, nbat,
                       (const double *)p.theta.ptr, (const int *)p.mcut.ptr, (const float *)p.tabsum.ptr, b);
    return hipGetLastError();
}

template <bool BF, bool SPLIT>
hipError_t gemm_form(Plan &p, const TabBatch &b, int part)
{
    const bool hasb = p.pol && b.B[0] != nullptr;
#define TL_CASE(NN)                                                              \
    case NN:                                                                     \
        if (!p.pol) return gemm_launch<BF, SPLIT, NN, false, false>(p, b, part); \
        if (hasb) return gemm_launch<BF, SPLIT, NN, true, true>(p, b, part);     \
        return gemm_launch<BF, SPLIT, NN, true, false>(p, b, part);
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
    const int n1 = cols_of(order, pol, hasb, true).n1;
    int nb = 0;
    while (nb < kTabMaxBatch && ((nb + 1) * n1 + 31) / 32 <= kTabMaxBlocks) ++nb;
    return nb;
}

int tab_rhs_blocks(int order, bool pol, int batch)
{
    int nb = 1;
    for (int hb = 0; hb < 2; ++hb) {
        if (hb && !pol) break;
        const int n1 = cols_of(order, pol, hb != 0, true).n1;
        const int g = std::min(std::max(batch, 1), tab_max_batch(order, pol, hb != 0));
        nb = std::max(nb, (g * n1 + 31) / 32);
    }
    return nb;
}

size_t tab_sum_bytes(int lmax, int nrn, int order, bool pol, int batch)
{
    size_t cols = 0;
    for (int hb = 0; hb < 2; ++hb) {
        if (hb && !pol) break;
        const int g = std::min(std::max(batch, 1), tab_max_batch(order, pol, hb != 0));
        cols = std::max(cols, (size_t)g * cols_of(order, pol, hb != 0, true).n1);
    }
    return (size_t)(lmax + 1) * (size_t)(nrn > 0 ? nrn : 0) * 4 * cols * sizeof(float);
}

size_t tab_rhs_bytes(int lmax, bool split, int nblocks)
{
    size_t chunks = 0;
    for (int m = 0; m <= lmax; ++m) chunks += (lmax - m + 1 + KC - 1) / KC;
    return chunks * (split ? 2 : 1) * nblocks * 128 * 16;
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

hipError_t launch_legendre_tab(Plan &p, const TabBatch &b, int part)
{
    switch (p.precision) {
    case TL_BF16: return gemm_form<true, false>(p, b, part);
    case TL_FP16: return gemm_form<false, false>(p, b, part);
    case TL_BF16X3: return gemm_form<true, true>(p, b, part);
    case TL_FP16X2: return gemm_form<false, true>(p, b, part);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tl
