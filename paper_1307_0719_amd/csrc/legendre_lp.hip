// Harmonic stage of the reduced-precision forms, computed on the fly: the
// FP64 recursion of lam and lam' in registers feeds 16-bit matrix-core
// products against the right-hand sides of up to four realizations at once.
//
// The L-power form (see legendre_mfma.hip) reduces every theta-derivative to
// two sums per (ring, m): sum_l lam_lm R[l][c] and sum_l lam'_lm R[l][c], R the
// right-hand-side columns {L^p a^T, N_l L^p a^E, N_l L^p a^B} (re, im) of each
// realization.  Here a wave owns 64 ring pairs and walks l in groups of 16:
// every lane runs its own ring's recursion (no duplicated FP64 work) and packs
// the 8 values of each parity (l - m even / odd) into one
// v_mfma_f32_32x32x16 operand.  Lanes 0..31 (rings 0..31 of the wave) give
// k = 0..7, lanes 32..63 (rings 32..63) k = 8..15, so the B operand carries
// the right-hand sides twice -- k < 8 in columns 0..15, k >= 8 in columns
// 16..31, zero elsewhere -- and a 32x32 accumulator holds 16 columns for each
// of the 64 rings.  Products run in FP16 or BF16 (optionally hi + lo split,
// three products) with FP32 accumulation; FP16 values carry power-of-two
// scales (lam x 2^lam_e0, lam' x 2^lam_e1 from the plan, each column of an m
// scaled into [2^13, 2^14)).  The
// per-(ring, m) epilogue applies the FP64 L-power coefficients.  No tables:
// the recursion costs the same FP64 work per call as the FP32 form, while the
// matrix work grows with the number of realizations.
#include "lpower.h"
#include "tl_internal.h"

namespace tl {

namespace {

using namespace lp;

constexpr double kHi = 0x1p256;
constexpr double kDown = 0x1p-512;
constexpr int GL = 16;                  // l-steps per group (8 per parity)
constexpr int RPW = 64;                 // ring pairs per wave
constexpr int WPG = 4;                  // waves per workgroup
constexpr int RPG = RPW * WPG;          // ring pairs per workgroup

template <int N, bool POL, bool HASB, int NBAT>
struct LpShape {
    static constexpr Cols C = cols_of(N, POL, HASB);
    static constexpr int NCOL = NBAT * C.n1;
    static constexpr int NBLK = (NCOL + 15) / 16;  // 16-column blocks
};

__device__ __forceinline__ int ngroups(int lmax, int m) { return (lmax - m + 1 + GL - 1) / GL; }

// Right-hand sides of one call in B-operand layout, one workgroup per m: per
// (m, group g, split, parity, block) 64 lanes x 8 values; lane (h, c): values
// for l = m + 16 g + parity + 2 e (e = 0..7) of column 16 blk + (c mod 16)
// when h == (c >= 16), else zero.  FP16: colexp[m][column] as in the table
// forms.
template <bool BF, bool SPLIT, int N, bool POL, bool HASB, int NBAT>
__global__ __launch_bounds__(256) void k_lp_rhs(int lmax, const int64_t *__restrict__ goff, const TabBatch batch,
                                                uint4 *__restrict__ rhs, float *__restrict__ colexp)
{
    using T = typename H<BF>::T;
    using S = LpShape<N, POL, HASB, NBAT>;
    constexpr int NCOL = S::NCOL, NBLK = S::NBLK, NSPL = SPLIT ? 2 : 1;
    constexpr int RCH = NSPL * 2 * NBLK * 64;  // uint4 per group
    __shared__ float s_ex[NBLK * 16];
    const int m = blockIdx.x;
    const int tid = threadIdx.x;
    const size_t base = (size_t)m * (2 * lmax + 1 - m) / 2;
    if (!BF) {
        for (int c = tid; c < NBLK * 16; c += 256) s_ex[c] = 0.f;
        __syncthreads();
        for (int idx = tid; idx < (lmax - m + 1) * NCOL; idx += 256) {
            const int l = m + idx / NCOL, c = idx % NCOL;
            const float v = (float)fabs(rhs_value<N, POL, HASB, NBAT>(batch, base, lmax, l, c));
            atomicMax((unsigned *)&s_ex[c], __float_as_uint(v));  // non-negative floats order as uints
        }
        __syncthreads();
        for (int c = tid; c < NBLK * 16; c += 256) {
            const float mx = s_ex[c];
            int ex = 0;
            if (mx > 0.f) frexpf(mx, &ex);
            s_ex[c] = (float)(14 - ex);
        }
    } else {
        for (int c = tid; c < NBLK * 16; c += 256) s_ex[c] = 0.f;
    }
    __syncthreads();
    for (int c = tid; c < NBLK * 16; c += 256) colexp[(size_t)m * NBLK * 16 + c] = s_ex[c];
    const int ng = ngroups(lmax, m);
    uint4 *out = rhs + goff[m] * RCH;
    for (int idx = tid; idx < ng * 2 * NBLK * 64; idx += 256) {
        const int lane = idx & 63, blk = (idx >> 6) % NBLK, p = ((idx >> 6) / NBLK) & 1, g = idx / (128 * NBLK);
        const int h = lane >> 5, col = lane & 31;
        const int gc = blk * 16 + (col & 15);
        const bool on = (h == (col >= 16 ? 1 : 0)) && gc < NCOL;
        const double sc = on ? ldexp(1.0, (int)s_ex[gc]) : 0.0;
        T hi8[8], lo8[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int l = m + GL * g + p + 2 * e;
            const float f = opaque(on ? (float)(rhs_value<N, POL, HASB, NBAT>(batch, base, lmax, l, gc) * sc) : 0.f);
            hi8[e] = (T)f;
            lo8[e] = (T)(f - (float)hi8[e]);
        }
        uint4 w;
        uint4 *dst = out + (int64_t)g * RCH + (p * NBLK + blk) * 64 + lane;
        __builtin_memcpy(&w, hi8, 16);
        dst[0] = w;
        if constexpr (SPLIT) {
            __builtin_memcpy(&w, lo8, 16);
            dst[2 * NBLK * 64] = w;
        }
    }
}

template <bool BF>
__device__ __forceinline__ void pack_vals(const float (&v)[8], uint4 &hi, uint4 &lo)
{
    using T = typename H<BF>::T;
    T h8[8], l8[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float f = opaque(v[e]);
        h8[e] = (T)f;
        l8[e] = (T)(f - (float)h8[e]);
    }
    __builtin_memcpy(&hi, h8, 16);
    __builtin_memcpy(&lo, l8, 16);
}

template <bool BF>
__device__ __forceinline__ floatx16 mma(uint4 a, uint4 b, floatx16 c)
{
    using V = typename H<BF>::V;
    V av, bv;
    __builtin_memcpy(&av, &a, 16);
    __builtin_memcpy(&bv, &b, 16);
    if constexpr (BF) return __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, c, 0, 0, 0);
}

struct LpArgs {
    int lmax, ntheta, nrp, rbeg, nrb, jtab, e0, e1;
    const double2 *trig;
    const double *theta;
    const double4 *coef0;
    const double *start;
    const int *exps;
    const int *mcut;
    const int64_t *goff;
    const uint4 *rhs;
    const float *colexp;
};

// One workgroup = 4 waves x 64 ring pairs at one m; workgroups of one m run on
// one XCD (m = xcd + 8 i) so the right-hand sides of m are read from HBM once.
template <bool BF, bool SPLIT, int N, bool POL, bool HASB, int NBAT>
__global__ __launch_bounds__(256) void k_legendre_lp(const LpArgs A, const TabBatch batch)
{
    using S = LpShape<N, POL, HASB, NBAT>;
    constexpr Cols C = S::C;
    constexpr int NBLK = S::NBLK, NSPL = SPLIT ? 2 : 1;
    constexpr int RCH = NSPL * 2 * NBLK * 64;
    // LDS: one chunk (4 groups = 64 l) of B operands and recursion
    // coefficients shared by the 4 waves; the epilogue transposition reuses it
    constexpr int CHB = 4 * RCH;  // uint4 of B operands per chunk
    struct Stg {
        uint4 b[CHB];
        double2 cf[64];  // (a, c) stepping into l = m + 64 chunk + 1 .. + 64
    };
    __shared__ union {
        Stg st;
        float tr[WPG][RPW][4][17];  // [wave][ring][type*2+par][col]
    } sm;

    const int lmax = A.lmax, nrp = A.nrp;
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int m = xcd + 8 * (q / A.nrb);
    if (m > lmax) return;  // whole workgroup
    const int rb = q % A.nrb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = A.rbeg + rb * RPG + wave * RPW + lane;
    const bool live = r < nrp;
    const int rr = live ? r : nrp - 1;  // idle lanes recurse a valid ring, write nothing
    const size_t plane = (size_t)A.ntheta * (lmax + 1);
    const int rs = A.ntheta - 1 - r;

    // evanescent for every ring of the workgroup: zeros
    const int mc = live ? A.mcut[r] + 2 : -1;
    if (!__syncthreads_or(m <= mc)) {
        if (live)
            for (int b = 0; b < NBAT; ++b)
                for (int j = 0; j <= N; ++j) {
                    float2 *F[3] = {batch.FT[b], batch.FQ[b], batch.FU[b]};
                    for (int f = 0; f < (POL ? 3 : 1); ++f) {
                        F[f][j * plane + (size_t)r * (lmax + 1) + m] = make_float2(0.f, 0.f);
                        if (rs != r) F[f][j * plane + (size_t)rs * (lmax + 1) + m] = make_float2(0.f, 0.f);
                    }
                }
        return;
    }

    const double x = A.trig[rr].x, sn = A.trig[rr].y;
    double l1 = A.start[((size_t)m * A.jtab) * nrp + rr];
    double d1 = A.start[((size_t)m * A.jtab + 1) * nrp + rr];
    double l2 = 0.0, d2 = 0.0;
    int e = A.exps[(size_t)m * nrp + rr];
    const size_t base = (size_t)m * (2 * lmax + 1 - m) / 2;
    const double lscale = ldexp(1.0, A.e0), fscale = ldexp(1.0, A.e1);

    floatx16 acc[NBLK][2][2];
#pragma unroll
    for (int b = 0; b < NBLK; ++b)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[b][t][p][v] = 0.f;

    const uint4 *rp = A.rhs + A.goff[m] * RCH;
    const int ng = ngroups(lmax, m);
    const int nch = (ng + 3) / 4;
    // the next chunk travels through registers while the current one is used
    constexpr int PER = (CHB + 255) / 256;
    uint4 pre[PER];
    double2 pcf = make_double2(0.0, 0.0);
    auto issue = [&](int c) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + 256 * i;
            const int gg = 4 * c + idx / RCH;
            pre[i] = (idx < CHB && gg < ng) ? rp[(int64_t)4 * c * RCH + idx] : make_uint4(0, 0, 0, 0);
        }
        if (tid < 64) {
            const int l = m + 64 * c + tid + 1;
            pcf = make_double2(0.0, 0.0);
            if (l <= lmax) {
                const double4 q4 = A.coef0[base + l];
                pcf = make_double2(q4.x, q4.z);
            }
        }
    };
    auto commit = [&]() {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = tid + 256 * i;
            if (idx < CHB) sm.st.b[idx] = pre[i];
        }
        if (tid < 64) sm.st.cf[tid] = pcf;
    };
    issue(0);
    commit();
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        if (c + 1 < nch) issue(c + 1);
        for (int gi = 0; gi < 4; ++gi) {
            const int g = 4 * c + gi;
            if (g >= ng) break;
            double2 cfv[GL];
#pragma unroll
            for (int s = 0; s < GL; ++s) cfv[s] = sm.st.cf[gi * GL + s];
            float va[2][8], vd[2][8];
            // value at l = m + 16 g + s, then one step to l + 1
            if (__all(e == 0)) {
#pragma unroll
                for (int s = 0; s < GL; ++s) {
                    va[s & 1][s >> 1] = (float)(l1 * lscale);
                    vd[s & 1][s >> 1] = (float)(d1 * fscale);
                    const double nl1 = cfv[s].x * (x * l1) - cfv[s].y * l2;
                    const double nd1 = cfv[s].x * fma(x, d1, -sn * l1) - cfv[s].y * d2;
                    l2 = l1;
                    l1 = nl1;
                    d2 = d1;
                    d1 = nd1;
                }
            } else {
#pragma unroll
                for (int s = 0; s < GL; ++s) {
                    const bool use = e == 0;
                    va[s & 1][s >> 1] = use ? (float)(l1 * lscale) : 0.f;
                    vd[s & 1][s >> 1] = use ? (float)(d1 * fscale) : 0.f;
                    const double nl1 = cfv[s].x * (x * l1) - cfv[s].y * l2;
                    const double nd1 = cfv[s].x * fma(x, d1, -sn * l1) - cfv[s].y * d2;
                    l2 = l1;
                    l1 = nl1;
                    d2 = d1;
                    d1 = nd1;
                    if ((s & 1) && e > 0 && fmax(fmax(fabs(l1), fabs(l2)), fmax(fabs(d1), fabs(d2))) > kHi) {
                        l1 *= kDown;
                        l2 *= kDown;
                        d1 *= kDown;
                        d2 *= kDown;
                        e -= 1;
                    }
                }
            }
            // e only decreases: still > 0 on every lane means every value of
            // the group was below 2^-256 (stored as zero): no products
            if (__all(e > 0)) continue;
            const uint4 *bg = sm.st.b + gi * RCH + lane;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                uint4 ah[2], al[2];
                pack_vals<BF>(va[p], ah[0], al[0]);
                pack_vals<BF>(vd[p], ah[1], al[1]);
#pragma unroll
                for (int b = 0; b < NBLK; ++b) {
                    const uint4 bh = bg[(p * NBLK + b) * 64];
#pragma unroll
                    for (int t = 0; t < 2; ++t) acc[b][t][p] = mma<BF>(ah[t], bh, acc[b][t][p]);
                    if constexpr (SPLIT) {
                        const uint4 bl = bg[((2 + p) * NBLK + b) * 64];
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            acc[b][t][p] = mma<BF>(ah[t], bl, acc[b][t][p]);
                            acc[b][t][p] = mma<BF>(al[t], bh, acc[b][t][p]);
                        }
                    }
                }
            }
        }
        __syncthreads();  // every wave is done with chunk c
        if (c + 1 < nch) {
            commit();
            __syncthreads();
        }
    }

    // ---- epilogue: lane = ring; blocks transposed through wave-private LDS ----
    const float usc[2] = {ldexpf(1.f, -A.e0), ldexpf(1.f, -A.e1)};  // exact: powers of two
    const float *cex = A.colexp + (size_t)m * NBLK * 16;
    const double th = A.theta[rr];
    // sums S[type*2+par][c - c0] of global columns c0 .. c0 + NC - 1
    auto gather = [&](float (*Sv)[C.n1], int c0, int nc) {
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            if (b * 16 + 16 <= c0 || b * 16 >= c0 + nc) continue;
            wave_sync();
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int vv = 0; vv < 16; ++vv) {
                        const int row = 8 * (vv >> 2) + 4 * (lane >> 5) + (vv & 3);
                        const int col = lane & 31;
                        sm.tr[wave][row + (col >= 16 ? 32 : 0)][t * 2 + p][col & 15] = acc[b][t][p][vv];
                    }
            wave_sync();
#pragma unroll
            for (int c = 0; c < C.n1; ++c) {
                if (c >= nc) break;
                const int gc = c0 + c;
                if (gc < b * 16 || gc >= b * 16 + 16) continue;
                const float isc = ldexpf(1.f, -(int)cex[gc]);
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4)
                    Sv[q4][c] = sm.tr[wave][lane][q4][gc - b * 16] * isc * usc[q4 >> 1];
            }
        }
    };
    float Sv[4][C.n1];
    auto nsum = [&](int type, int c) { return (double)Sv[type * 2][c] + (double)Sv[type * 2 + 1][c]; };
    auto dsum = [&](int type, int c) { return (double)Sv[type * 2][c] - (double)Sv[type * 2 + 1][c]; };
    {
        CoefT<N> cf;
        coefficients_T<N>(th, m, cf);
        for (int bb = 0; bb < NBAT; ++bb) {
            gather(Sv, bb * C.n1, C.nT);
            if (!live) continue;
            float2 *FT = batch.FT[bb];
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
        }
    }
    if constexpr (POL) {
        CoefP<N> cf;
        coefficients_P<N>(th, m, cf);
        constexpr int NP = C.nE + C.nB;
        for (int bb = 0; bb < NBAT; ++bb) {
            // spin-2 columns of realization bb, stored from Sv[.][0]
            gather(Sv, bb * C.n1 + C.nT, NP);
            if (!live) continue;
            float2 *FQ = batch.FQ[bb], *FU = batch.FU[bb];
#pragma unroll
            for (int j = 0; j <= N; ++j) {
                double ewn[2] = {0, 0}, exn[2] = {0, 0}, bwn[2] = {0, 0}, bxn[2] = {0, 0};
                double ews[2] = {0, 0}, exs[2] = {0, 0}, bws[2] = {0, 0}, bxs[2] = {0, 0};
#pragma unroll
                for (int p = 0; p <= C.PS; ++p)
#pragma unroll
                    for (int ri = 0; ri < 2; ++ri) {
                        const int ce = 2 * p + ri;
                        ewn[ri] += cf.wa[j][p] * nsum(0, ce) + cf.wb[j][p] * nsum(1, ce);
                        exn[ri] += cf.xa[j][p] * nsum(0, ce) + cf.xb[j][p] * nsum(1, ce);
                        ews[ri] += cf.wa[j][p] * dsum(0, ce) + cf.wb[j][p] * dsum(1, ce);
                        exs[ri] += cf.xa[j][p] * dsum(0, ce) + cf.xb[j][p] * dsum(1, ce);
                        if constexpr (HASB) {
                            const int cb_ = C.nE + 2 * p + ri;
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

template <bool BF, bool SPLIT, int N, bool POL, bool HASB, int NBAT>
hipError_t lp_launch(Plan &p, const TabBatch &b, int part)
{
    using S = LpShape<N, POL, HASB, NBAT>;
    if constexpr (S::NBLK > 4) {
        return hipErrorInvalidValue;
    } else {
        if ((size_t)S::NBLK > p.rhs_nb) return hipErrorInvalidValue;  // buffers sized at plan time
        if (part == 0) {
            hipLaunchKernelGGL((k_lp_rhs<BF, SPLIT, N, POL, HASB, NBAT>), dim3(p.lmax + 1), dim3(256), 0, p.stream,
                               p.lmax, (const int64_t *)p.moff.ptr, b, (uint4 *)p.rhs.ptr, (float *)p.colexp.ptr);
            return hipGetLastError();
        }
        const int nr = p.nrp - p.rpole;
        if (nr <= 0) return hipSuccess;
        LpArgs A{};
        A.lmax = p.lmax;
        A.ntheta = p.ntheta;
        A.nrp = p.nrp;
        A.rbeg = p.rpole;
        A.nrb = (nr + RPG - 1) / RPG;
        A.jtab = p.jtab;
        A.e0 = p.lam_e0;
        A.e1 = p.lam_e1;
        A.trig = (const double2 *)p.trig.ptr;
        A.theta = (const double *)p.theta.ptr;
        A.coef0 = (const double4 *)p.coef0.ptr;
        A.start = (const double *)p.start.ptr;
        A.exps = (const int *)p.exps.ptr;
        A.mcut = (const int *)p.mcut.ptr;
        A.goff = (const int64_t *)p.moff.ptr;
        A.rhs = (const uint4 *)p.rhs.ptr;
        A.colexp = (const float *)p.colexp.ptr;
        const int m8 = (p.lmax + 1 + 7) / 8;
        hipLaunchKernelGGL((k_legendre_lp<BF, SPLIT, N, POL, HASB, NBAT>), dim3(8 * m8 * A.nrb), dim3(256), 0,
                           p.stream, A, b);
        return hipGetLastError();
    }
}

template <bool BF, bool SPLIT, int N, bool POL, bool HASB>
hipError_t lp_nbat(Plan &p, const TabBatch &b, int part)
{
    switch (b.n) {
    case 1: return lp_launch<BF, SPLIT, N, POL, HASB, 1>(p, b, part);
    case 2: return lp_launch<BF, SPLIT, N, POL, HASB, 2>(p, b, part);
    case 3: return lp_launch<BF, SPLIT, N, POL, HASB, 3>(p, b, part);
    case 4: return lp_launch<BF, SPLIT, N, POL, HASB, 4>(p, b, part);
    default: return hipErrorInvalidValue;
    }
}

template <bool BF, bool SPLIT>
hipError_t lp_form(Plan &p, const TabBatch &b, int part)
{
    const bool hasb = p.pol && b.B[0] != nullptr;
#define TL_CASE(NN)                                                              \
    case NN:                                                                     \
        if (!p.pol) return lp_nbat<BF, SPLIT, NN, false, false>(p, b, part);     \
        if (hasb) return lp_nbat<BF, SPLIT, NN, true, true>(p, b, part);         \
        return lp_nbat<BF, SPLIT, NN, true, false>(p, b, part);
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

int lp_max_batch(int order, bool pol, bool hasb)
{
    if (order > 6) return 0;
    const int n1 = cols_of(order, pol, hasb).n1;
    int nb = 0;
    while (nb < 4 && ((nb + 1) * n1 + 15) / 16 <= 4) ++nb;
    return nb;
}

int lp_rhs_blocks(int order, bool pol, int batch)
{
    int nb = 1;
    for (int hb = 0; hb < 2; ++hb) {
        if (hb && !pol) break;
        const int n1 = cols_of(order, pol, hb != 0).n1;
        const int g = std::min(std::max(batch, 1), lp_max_batch(order, pol, hb != 0));
        nb = std::max(nb, (g * n1 + 15) / 16);
    }
    return nb;
}

// group offsets: goff[m] = number of 16-l groups of all m' < m
size_t lp_groups(int lmax, std::vector<int64_t> &goff)
{
    goff.assign((size_t)lmax + 2, 0);
    int64_t off = 0;
    for (int m = 0; m <= lmax; ++m) {
        goff[m] = off;
        off += (lmax - m + 1 + GL - 1) / GL;
    }
    goff[lmax + 1] = off;
    return (size_t)off;
}

size_t lp_rhs_bytes(int lmax, bool split, int nblocks)
{
    std::vector<int64_t> g;
    return lp_groups(lmax, g) * (split ? 2 : 1) * 2 * nblocks * 64 * 16;
}

hipError_t launch_legendre_lp(Plan &p, const TabBatch &b, int part)
{
    switch (p.precision) {
    case TL_BF16: return lp_form<true, false>(p, b, part);
    case TL_FP16: return lp_form<false, false>(p, b, part);
    case TL_BF16X3: return lp_form<true, true>(p, b, part);
    case TL_FP16X2: return lp_form<false, true>(p, b, part);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tl
