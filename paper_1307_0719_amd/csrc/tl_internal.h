// Internal declarations of the taylens HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/taylens.h"

namespace tl {

constexpr int kMaxOrder = TL_MAX_ORDER;

// Per-thread last-error message (set by fail()).
void set_error(const std::string &msg);

// Device arrays owned by a plan.  Sizes in elements unless noted.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// One ring FFT job: one source row of per-m coefficients (complex, m = 0..lmax)
// and up to kMaxJobK outputs, each the real ring
//     out[n] = scale * sum_{m=-L}^{L} (i m)^k F_m e^{i m phi_n}.
constexpr int kMaxJobK = kMaxOrder + 1;
struct FftJob {
    int64_t src;                 // element offset (complex) of F_0 of the row
    int32_t nk;                  // number of outputs
    int32_t pad;                 // (HEALPix: the ring)
    int32_t k[kMaxJobK];         // phi-derivative order of each output
    int32_t h16;                 // bit q: output q is FP16, dst[q] counts from the FP16 maps
    int32_t pair;                // bit q: outputs q and q + 1 share a paired plane at dst[q]
                                 // (pixel n of output q at 2n, of output q + 1 at 2n + 1)
    int64_t dst[kMaxJobK];       // element offset (real) of each output ring
    double scale[kMaxJobK];      // multiplier of each output
};

// Mixed-precision derivative maps (FP32 forms' internal maps, order >= 3):
// D_jk with j + k < kMix16 in FP32, [field][6][pixel]; the higher orders,
// which the remap multiplies by |u|^j |v|^k <= 2^-(j+k), in FP16 after them,
// [field][ndmap - 6][pixel], both j-major.
constexpr int kMix16 = 3;
__host__ __device__ constexpr int mix_n32() { return 6; }
__host__ __device__ constexpr int mix_idx32(int j, int k) { return j == 0 ? k : (j == 1 ? 3 + k : 5); }
__host__ __device__ constexpr int mix_kmin16(int j) { return j >= kMix16 ? 0 : kMix16 - j; }
__host__ __device__ constexpr int mix_idx16(int N, int j, int k)
{
    int s = 0;
    for (int jj = 0; jj < j; ++jj) s += N - jj - mix_kmin16(jj) + 1;
    return s + k - mix_kmin16(j);
}

// Paired planes of the plan's own FP16 maps (mixed layout on equal-theta
// rings whose FFT runs in one workgroup): along each row j, FP16 maps k and
// k + 1 share one plane of two values per pixel, taken greedily from the
// first FP16 map, so a remap lane reads both with one load.  Returns 0 for a
// map on its own plane, 1 for the first of a pair, 2 for the second.
__host__ __device__ constexpr bool map_is16(bool mix, int j, int k) { return mix && j + k >= kMix16; }
__host__ __device__ constexpr int pair_pos(int N, bool mix, int j, int k)
{
    int kk = 0;
    while (kk <= N - j) {
        const bool pr = kk + 1 <= N - j && map_is16(mix, j, kk) && map_is16(mix, j, kk + 1);
        if (k == kk) return pr ? 1 : 0;
        if (pr && k == kk + 1) return 2;
        kk += pr ? 2 : 1;
    }
    return 0;
}

// Realizations handled by one pass of the table GEMM (reduced-precision forms).
constexpr int kTabMaxBatch = 6;   // realizations per table pass
constexpr int kTabMaxBlocks = 4;   // 32-column blocks per table pass
struct TabBatch {
    int n;
    const double2 *T[kTabMaxBatch];
    const double2 *E[kTabMaxBatch];
    const double2 *B[kTabMaxBatch];
    float2 *FT[kTabMaxBatch];
    float2 *FQ[kTabMaxBatch];
    float2 *FU[kTabMaxBatch];
    // lensing potential (table engine; NULL: none): a^phi and the FP64 rows
    // [2][ntheta][lmax+1] of its lam and lam' sums (the deflection's Fphi)
    const double2 *P[kTabMaxBatch];
    double2 *FP[kTabMaxBatch];
};

// One ring of a HEALPix grid (RING order): first pixel, pixel count, the
// phase e^{i nphi phi0} (+-1), phi of the first pixel (phi0 = pi shift / nphi,
// shift 0 or 1), and how its ring FFT runs: P = 0, mixed radix; else
// Bluestein's chirp transform of padded length P, with the spectrum of the
// chirp at element offset boff of the plan's chirp tables.
struct HRing {
    int64_t start;
    int32_t nphi;
    int32_t sigma;
    double phi0;
    int64_t boff;
    int32_t P;
    int32_t shift;
    int32_t cls;      // FFT job class (below)
    int32_t pad;
};

// HEALPix ring FFT job classes: 0 = mixed radix, 1..6 = Bluestein with
// P = 2^(c + 7) (256 .. 8192), 7 = power-of-two length 1024..8192 with
// lmax < N (the belt of nside 256..2048: the radix-16 kernel).
constexpr int kHpxClasses = 8;
constexpr int kHpxPow2 = 7;
inline int hpx_class_of_P(int P)
{
    int c = 0;
    while (P > 128) {
        P >>= 1;
        ++c;
    }
    return c;
}

struct Plan {
    int lmax = 0;
    int lmax_phi = 0;  // band limit of the lensing potential (>= lmax)
    int nside = 0;    // > 0: HEALPix rings (RING order) instead of the equal-theta grid
    int ntheta = 0, nphi = 0;
    int nrp = 0;      // ring pairs = ceil(ntheta/2)
    int order = 0;    // N
    int jtab = 0;     // derivative entries per start value (max(N,1)+1)
    int precision = TL_FP32;
    int pol = 0, rotate = 1, naive = 0;
    int rpole = 0;    // ring pairs kept on the direct FP64 kernel (the polar caps)
    int batch = 1;    // realizations per table-GEMM pass (reduced-precision forms)
    int ntile = 0;    // 32-ring-pair tiles outside the caps (table forms)
    bool tables = false;  // reduced forms: plan-time tables (else on-the-fly recursion)
    // FP16 operand scales of lambda and lambda' (powers of two, 2^lam_e0 and
    // 2^lam_e1; 0 for BF16): the largest value either can take at this lmax
    // stays below 2^15, so every value that matters keeps a normal lo part
    int lam_e0 = 0, lam_e1 = 0;
    int64_t cap = 0;
    hipStream_t stream = nullptr;
    int device = 0;

    // FFT length factorization (M = nphi/2 = prod radix)
    int nradix = 0;
    int radix[32];

    // tables
    DevBuf theta;     // double [ntheta]
    DevBuf trig;      // double2 {cos, sin} [nrp] (north rings)
    DevBuf phitab;    // double2 {cos phi_k, sin phi_k} [nphi] + double phi_k [nphi]
    DevBuf phival;    // double [nphi]
    DevBuf twid64;    // double2 [nphi]  e^{2 pi i t / nphi}
    DevBuf twid32;    // float2  [nphi]
    DevBuf coef0;     // double4 {a, b, c, 0} spin 0, triangular
    DevBuf coef2;     // double4 {a, b(+2), c, 0} spin 2, triangular
    DevBuf start;     // double [3][lmax+1][jtab][nrp]
    DevBuf exps;      // int    [3][lmax+1][nrp]
    DevBuf mcut;      // int    [nrp]  largest significant m per ring pair
    // the same recursion tables for the lensing potential when lmax_phi >
    // lmax (spin 0, derivative entries of J = 1: jtab 2)
    DevBuf coefP0, coefP2, startP, expsP, mcutP;
    bool phi_tables() const { return lmax_phi != lmax; }
    // deflection ring FFTs in FP32 (non-FP64 plans whose rings are too long
    // for the FP64 transform in LDS): FP32 rows and deflection in dscratch
    bool defl32 = false;
    DevBuf dscratch;
    DevBuf twT;       // double2 [ntheta - 1] e^{-2 pi i t / (2 (ntheta - 1))} (theta_fft_grid)
    // FP64 form: the harmonic stage synthesizes the rows j = 0 only and the
    // theta-derivatives come from FFTs along the great circles (opt.theta_fft)
    bool theta_fft = false;
    DevBuf hring;     // HRing [ntheta] (HEALPix plans)
    DevBuf twP64;     // double2 [8192] e^{2 pi i t / 8192} (HEALPix plans with Bluestein rings)
    DevBuf twP32;     // float2  [8192]
    DevBuf bhat64;    // double2 chirp spectra of the Bluestein ring lengths (HEALPix)
    DevBuf bhat32;    // float2 copy
    // HEALPix FFT jobs per class (deflection list, main list), in list order
    int hjobs[2][kHpxClasses] = {};
    int hmax_direct = 0;  // largest half length M of the mixed-radix rings
    int hmax_P = 0;       // largest Bluestein length
    int hmax_pow2 = 0;    // half length M of the power-of-two class (0: none)
    bool caps_defl_done = false;  // the last harmonic stage also ran the deflection's caps
    DevBuf tab;       // lambda / lambda' tables in MFMA operand layout (reduced-precision forms)
    DevBuf moff;      // int64 [lmax+2] offsets (16-byte units) of each m in tab
    DevBuf kstart;    // int [lmax+1][ntile] first non-empty 32-l chunk
    DevBuf rhs;       // table-GEMM right-hand sides of one call, B-operand layout
    DevBuf colexp;    // float [lmax+1][32 * rhs_nb] power-of-two column scales (FP16)
    DevBuf tabsum;    // float column sums of the table GEMM [lmax+1][nrp-rpole][batch][4][n1]
    size_t rhs_nb = 0;  // 32-column blocks the rhs buffer holds per chunk

    // work buffers
    DevBuf Fphi;      // complex128 [batch][2][ntheta][lmax+1]
    DevBuf alpha;     // double [2][ntheta][nphi]
    DevBuf F;         // complex (64 or 128) [nfield][N+1][ntheta][lmax+1]
    DevBuf D;         // real [nfield][ndmap][ntheta][nphi]
    DevBuf jobsDefl;  // FftJob [ntheta * 2]
    DevBuf jobsMain;  // FftJob [nfield * (N+1) * ntheta]
    DevBuf jobsInt;   // the same jobs into the plan's own maps D (padded planes, mix16)
    int njobsDefl = 0, njobsMain = 0;
    bool mix16 = false;  // the plan's own maps D are mixed precision
    // plane strides (elements) of the plan's own maps: the pixel count
    // rounded up to an odd multiple of 256 bytes, so that the maps a remap
    // lane gathers at one pixel do not all share their low address bits
    size_t dstride = 0, dstride16 = 0;
    // the plan's own FP16 maps use paired planes (pair_pos); slots s and
    // s + 1 of a pair together hold 2 dstride16 elements
    bool paired = false;
    // Tabulated plans of several realizations per pass: the realizations of
    // a pass alternate between two sets of maps and deflection fields (D,
    // alpha and D2, alpha2), so that the remap of one runs on a second
    // stream (side, default priority) while the ring FFTs of the next run
    // on the plan's stream; ev_fft[s] / ev_remap[s] order the uses of set s.
    DevBuf D2, alpha2;
    hipStream_t side = nullptr;
    hipEvent_t ev_fft[2] = {nullptr, nullptr}, ev_remap[2] = {nullptr, nullptr};
    // the polar caps of a tabulated pass run on the second stream beside the
    // table epilogue: ev_gemm (plan's stream, after the table GEMM) starts
    // them, ev_caps (second stream) holds back what follows the epilogue
    hipEvent_t ev_gemm = nullptr, ev_caps = nullptr;
    bool overlap() const { return side != nullptr && !profile; }

    size_t total_bytes = 0;
    // work counts (tl_plan_query)
    int64_t q_elems = 0, q_elems_caps = 0, q_tab_chunks = 0, q_tab_chunk_bytes = 0;

    // instrumentation: event pairs per timed stage launch
    struct ProfRec {
        int stage;
        hipEvent_t a, b;
    };
    bool profile = false;
    std::vector<ProfRec> prof;

    int nfield() const { return pol ? 3 : 1; }
    int ndmap() const { return (order + 1) * (order + 2) / 2; }
    // FP16 maps of the mixed layout start after the FP32 ones
    void *d16() const { return d16_of(D.ptr); }
    void *d16_of(const void *maps) const { return (char *)maps + (size_t)nfield() * mix_n32() * dstride * 4; }
    // the plan's own maps (either set)
    bool own(const void *maps) const { return maps && (maps == D.ptr || maps == D2.ptr); }
    bool fp64() const { return precision == TL_FP64; }
    bool tabform() const { return precision >= TL_BF16X3; }
    size_t npix() const { return nside ? (size_t)12 * nside * nside : (size_t)ntheta * (size_t)nphi; }
    size_t nalm() const { return (size_t)(lmax + 1) * (size_t)(lmax + 2) / 2; }
};

// Realizations of one launch of the direct FP64 kernels (they share the
// recursion): a = a_lm (spin: a^E), b = a^B (spin; all NULL or none), F =
// output rows (spin: FQ), G = FU.
constexpr int kDirectMax = 5;
struct DirectSet {
    int n;
    const double2 *a[kDirectMax];
    const double2 *b[kDirectMax];
    void *F[kDirectMax];
    void *G[kDirectMax];
};

// ---- kernel launchers (return hipError_t) ----
hipError_t launch_tables(Plan &p);
// most realizations one direct launch takes at derivative order J
int direct_max(int J, bool spin, bool hasb, bool out64);
// phi: the lensing potential's band limit and tables (Plan::phi_tables)
hipError_t launch_legendre_scalar_set(Plan &p, int J, int rend, const DirectSet &set, bool out64,
                                      bool phi = false);
hipError_t launch_legendre_spin_set(Plan &p, int J, int rend, const DirectSet &set, bool out64);
hipError_t launch_legendre_scalar(Plan &p, int J, int rend, const void *alm, void *F, bool out64);
hipError_t launch_legendre_spin(Plan &p, int J, int rend, const void *almE, const void *almB, void *FQ,
                                void *FU, bool out64);
bool mfma_supported(int order, bool hasb);
int tab_max_batch(int order, bool pol, bool hasb);
size_t tab_bytes(int lmax, int ntile, bool split, std::vector<int64_t> &moff);
int tab_rhs_blocks(int order, bool pol, int batch);
size_t tab_rhs_bytes(int lmax, bool split, int nblocks);
size_t tab_sum_bytes(int lmax, int nrn, int order, bool pol, int batch);
hipError_t launch_build_tab(Plan &p);
// part 0: right-hand sides of the batch (k_tab_rhs); part 1: the GEMM
// (column sums); part 2: its epilogue (rows of the theta-derivatives)
hipError_t launch_legendre_tab(Plan &p, const TabBatch &b, int part);
// on-the-fly reduced-precision harmonic kernel (legendre_lp.hip)
int lp_max_batch(int order, bool pol, bool hasb);
int lp_rhs_blocks(int order, bool pol, int batch);
size_t lp_groups(int lmax, std::vector<int64_t> &goff);
size_t lp_rhs_bytes(int lmax, bool split, int nblocks);
hipError_t launch_legendre_lp(Plan &p, const TabBatch &b, int part);
// Stage numbers of the per-kernel profile (one kernel per stage).
enum Stage {
    ST_DEFL_LEG = 0, ST_DEFL_FFT, ST_LEG_T, ST_LEG_QU, ST_LEG_MFMA, ST_TAB_RHS, ST_TAB_GEMM, ST_FFT, ST_REMAP, ST_CNN,
    ST_TAB_EPI, ST_CAPS
};

// Polar caps of the FP32 and tabulated forms in one launch (FP32 rows):
// task {kind, first realization, count, 0}, kind 0 = deflection (FP64 rows
// of the potential, J = 1), 1 = T, 2 = spin +2 family of Q/U, 3 = spin -2
// family; pointers per realization of the pass.
constexpr int kCapsMaxTasks = 32;
struct CapsArgs {
    int ntask;
    int4 task[kCapsMaxTasks];
    const double2 *T[kTabMaxBatch], *E[kTabMaxBatch], *B[kTabMaxBatch], *P[kTabMaxBatch];
    void *FT[kTabMaxBatch], *FQ[kTabMaxBatch], *FU[kTabMaxBatch], *FP[kTabMaxBatch];
};
// realizations one task of this kind takes (0: the combined launch does not
// cover this order)
int caps_nb(int kind, int J, bool hasb);
// zeroes the Q/U cap rows of realizations [0, nreal) (spin families add
// into them), then launches the tasks over ring pairs [0, rend)
hipError_t launch_legendre_caps(Plan &p, int rend, const CapsArgs &a, int nreal, bool hasb,
                                hipStream_t st = nullptr);  // st: default the plan's stream

// ---- learned remainder correction (cnn.hip) ----
constexpr int kCnnTrain = 32 * 20 * 9 + 32 + 32 * 32 * 9 + 32 + 3 * 32 + 3;  // trainable parameters
constexpr int kCnnParam = kCnnTrain + 3;                                     // + output scales
struct CnnBufs {
    void *params = nullptr;  // float [kCnnParam] (FP32 master)
    void *m = nullptr, *v = nullptr;  // float [kCnnTrain] Adam moments
    void *grad = nullptr;    // float [kCnnTrain + 1]: gradient, then the loss
    void *W1p = nullptr, *W2p = nullptr, *W3p = nullptr;  // BF16 MFMA operands
    void *work = nullptr;    // training activations (cnn_train_bytes_per_pixel each)
};
hipError_t cnn_pack(const CnnBufs &c, hipStream_t st);
size_t cnn_packed_bytes();
size_t cnn_train_bytes_per_pixel();
// corr: float [3][n]; train: also keep activations in c.work (n pixels)
hipError_t cnn_forward(const Plan &p, const CnnBufs &c, const float *D, const double *at, const double *ap,
                       const int64_t *pix, int64_t n, float *corr, bool train, hipStream_t st);
hipError_t cnn_backward(const CnnBufs &c, int64_t n, const float *target, hipStream_t st);
hipError_t cnn_adam(const CnnBufs &c, int step, float lr, hipStream_t st);
hipError_t cnn_zero(float *x, int64_t n, hipStream_t st);
hipError_t launch_legendre_mfma(Plan &p, const void *T, const void *E, const void *B, void *FT, void *FQ,
                                void *FU);
// One realization's arguments of the matrix-core harmonic kernel.
struct MfmaJob {
    int lmax, ntheta, nrp, rbeg, jtab;
    const double2 *trig;
    const double *theta;
    const double4 *coef0;
    const double *start;
    const int *exps;
    const int *mcut;
    const double2 *almT, *almE, *almB;
    float2 *FT, *FQ, *FU;
};
MfmaJob mfma_job(const Plan &p, const void *T, const void *E, const void *B, void *FT, void *FQ, void *FU);
int mfma_ring_block();  // ring pairs per work item
int mfma_m_group();     // consecutive m per m-group
// items[i] = {job, ring block, first m-group, m-groups}; head: queue counter (zero before the launch)
hipError_t launch_legendre_mfma_queue(int order, bool pol, bool hasb, hipStream_t st, const MfmaJob *jobs,
                                      const int4 *items, int nitems, int *head, int ngroups);
hipError_t fill_words(void *x, size_t n, uint32_t v, hipStream_t st);
// theta-derivatives by FFT along the great circles through both poles
// (thetafft.hip): grids with ntheta - 1 a power of two in [2, kThetaFftMaxP / 2]
constexpr int kThetaFftMaxP = 8192;
bool theta_fft_grid(int ntheta);
// Where the maps of one theta-FFT launch live (elements of the plan's real
// type): map i at in + i istride; its order-j output at out + i ostride +
// (sa j - sb j (j - 1) / 2 + sc) pstride.  Consecutive outputs [j - 1]:
// {plane, jmax plane, plane, 1, 0, -1}; the plan's j-major derivative maps
// of column k at order N: {ndmap ds, ndmap ds, ds, N + 1, 1, k}.
struct ThetaFftLayout {
    size_t istride, ostride, pstride;
    int sa, sb, sc;
};
// dtheta^j / j! d^j_theta of each input map, j = 1..jmax, maps [ntheta][nphi]
// in the plan's real type; on the plan's stream
hipError_t launch_theta_fft(Plan &p, const void *in, void *out, int nmaps, int jmax, const ThetaFftLayout &lay);
// analysis of an FP64 temperature map into a_lm (analysis.hip): rings of a
// power of two of pixels up to kThetaFftMaxP; scratch in the plan's F buffer
// (analysis_scratch_bytes of it) and its deflection buffer (lmax + 1 values)
bool analysis_grid(int nphi);
size_t analysis_scratch_bytes(const Plan &p);
hipError_t launch_analysis_T(Plan &p, const double *map, void *alm);
// the deflection's ring FFTs in FP32 (Plan::defl32) from the FP64 rows at
// band limit L into the FP64 deflection alpha
hipError_t launch_defl_fft32(Plan &p, const void *rows64, void *alpha, int L);
// list: 0 = the deflection jobs, 1 = the main jobs (HEALPix plans launch each
// job class of the list on its own)
bool fft_p2(int M);  // rings of 2 M points take the one-workgroup radix-16 kernel
// L: band limit of the rows (default the plan's lmax; the deflection's rows
// have lmax_phi + 1 entries); equal-theta plans
hipError_t launch_fft_jobs(Plan &p, const void *Fbase, void *Dbase, const FftJob *jobs, int njobs,
                           bool fp64, int list, void *D16 = nullptr, int L = -1);
// HEALPix: chirp spectra of the Bluestein ring lengths (items {M, class P, boff})
hipError_t launch_bluestein_tables(Plan &p, const std::vector<int4> &items);
// D: the plan's own maps (padded, maybe mixed) or a caller's ([field][map][pixel]);
// corr (optional, FP32 [3][ntheta][nphi]): added to the Taylor sums before the rotation;
// st: the stream (default: the plan's)
hipError_t launch_remap(Plan &p, const void *D, const double *at, const double *ap,
                        const double *thsrc, const double *phsrc, void *T, void *Q, void *U,
                        const float *corr = nullptr, hipStream_t st = nullptr);

}  // namespace tl
