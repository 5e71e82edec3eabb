// C ABI of the taylens library: plans, argument validation, stage sequencing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <vector>
#include <string>
#include <mutex>
#include <sys/stat.h>

#include "tl_internal.h"

namespace tl {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

hipError_t fft_prepare(Plan &p);

}  // namespace tl

using namespace tl;

#define TL_VERSION 10000

namespace {

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

int hipfail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return TL_ERR_HIP;
}

#define TL_HIP(call, what)                           \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return hipfail(e_, what); \
    } while (0)

// Records a HIP event pair around one stage when the plan is profiling.
struct StageScope {
    Plan &p;
    int stage;
    hipEvent_t a = nullptr, b = nullptr;
    StageScope(Plan &pl, int st) : p(pl), stage(st)
    {
        if (!p.profile) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, p.stream);
    }
    ~StageScope()
    {
        if (!a) return;
        (void)hipEventRecord(b, p.stream);
        p.prof.push_back({stage, a, b});
    }
};

void clear_prof(Plan &p)
{
    for (auto &r : p.prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    p.prof.clear();
}

bool factor_radices(int M, Plan &p)
{
    p.nradix = 0;
    int n = M;
    while (n % 8 == 0 && n > 1) {
        p.radix[p.nradix++] = 8;
        n /= 8;
    }
    while (n % 4 == 0 && n > 1) {
        p.radix[p.nradix++] = 4;
        n /= 4;
    }
    while (n % 2 == 0 && n > 1) {
        p.radix[p.nradix++] = 2;
        n /= 2;
    }
    while (n % 5 == 0 && n > 1) {
        p.radix[p.nradix++] = 5;
        n /= 5;
    }
    while (n % 3 == 0 && n > 1) {
        p.radix[p.nradix++] = 3;
        n /= 3;
    }
    return n == 1 && p.nradix <= 16;
}

void free_buf(DevBuf &b)
{
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
}

void free_plan_buffers(Plan &p)
{
    DevBuf *bufs[] = {&p.theta, &p.trig, &p.phitab, &p.phival, &p.twid64, &p.twid32, &p.coef0, &p.coef2,
                      &p.start, &p.exps, &p.mcut, &p.tab, &p.moff, &p.kstart, &p.rhs, &p.colexp, &p.tabsum, &p.Fphi, &p.alpha, &p.F, &p.D, &p.jobsDefl, &p.jobsMain, &p.jobsInt, &p.hring,
                      &p.twP64, &p.twP32, &p.bhat64, &p.bhat32, &p.D2, &p.alpha2, &p.coefP0, &p.coefP2,
                      &p.startP, &p.expsP, &p.mcutP, &p.dscratch, &p.twT};
    for (DevBuf *b : bufs) free_buf(*b);
    if (p.side) (void)hipStreamSynchronize(p.side);
    for (int i = 0; i < 2; ++i) {
        if (p.ev_fft[i]) (void)hipEventDestroy(p.ev_fft[i]);
        if (p.ev_remap[i]) (void)hipEventDestroy(p.ev_remap[i]);
        p.ev_fft[i] = p.ev_remap[i] = nullptr;
    }
    if (p.ev_gemm) (void)hipEventDestroy(p.ev_gemm);
    if (p.ev_caps) (void)hipEventDestroy(p.ev_caps);
    p.ev_gemm = p.ev_caps = nullptr;
    if (p.side) (void)hipStreamDestroy(p.side);
    p.side = nullptr;
}

int alloc(Plan &p, DevBuf &b, size_t bytes, const char *name)
{
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        (void)hipGetLastError();
        return fail(TL_ERR_NOMEM, std::string("hipMalloc failed for ") + name + " (" +
                                     std::to_string(bytes) + " bytes): " + hipGetErrorString(e));
    }
    b.bytes = bytes;
    p.total_bytes += bytes;
    return TL_OK;
}

int dmap_index(int N, int j, int k) { return j * (N + 1) - j * (j - 1) / 2 + k; }

double factorial(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

// HEALPix rings (RING order, the published geometry of Gorski et al. 2005):
// ring i = 1 .. 4 nside - 1 with colatitude from z = 1 - i^2/(3 nside^2) in
// the polar caps (through sin(theta/2), exact near the poles) and
// z = 4/3 - 2 i/(3 nside) in the belt, 4 i resp. 4 nside pixels, the first at
// phi0 = pi/(4 i) in the caps and pi s/(4 nside), s = (i - nside + 1) mod 2, in
// the belt; sigma = e^{i nphi phi0} = -1 for shifted rings, +1 otherwise.
// Ring FFT of half length M: 0 = mixed radix (M <= 32), else the Bluestein
// length P (power of two >= 2 M - 1, >= 256).
int healpix_blue_P(int M)
{
    if (M <= 32) return 0;
    int P = 256;
    while (P < 2 * M - 1) P <<= 1;
    return P;
}

// HEALPix rings (Gorski et al. 2005, RING order): colatitude, first pixel,
// pixel count, phase; the FFT class of each ring (power-of-two lengths 1024 ..
// 8192 with lmax < N take the radix-16 kernel), and (items) the distinct
// Bluestein lengths {M, P, offset, 0} sorted by P, with their chirp-table
// total (nbhat elements).
void healpix_rings(int nside, int lmax, std::vector<double> &th, std::vector<HRing> &hr,
                   std::vector<int4> *items = nullptr, size_t *nbhat = nullptr)
{
    const int nr = 4 * nside - 1;
    th.assign(nr, 0.0);
    hr.assign(nr, HRing{});
    int64_t start = 0;
    for (int r = 0; r < nr; ++r) {
        const int i = r + 1;
        const bool north = i <= 2 * nside;
        const int ii = north ? i : 4 * nside - i;
        double t, p0;
        int n, sig, sh;
        if (ii < nside) {
            t = 2.0 * std::asin((double)ii / (std::sqrt(6.0) * nside));
            if (!north) t = M_PI - t;
            n = 4 * ii;
            p0 = M_PI / (4.0 * ii);
            sig = -1;
            sh = 1;
        } else {
            t = std::acos(4.0 / 3.0 - 2.0 * i / (3.0 * nside));
            n = 4 * nside;
            sh = (i - nside + 1) % 2;
            p0 = M_PI * sh / (4.0 * nside);
            sig = sh ? -1 : 1;
        }
        th[r] = t;
        hr[r] = HRing{start, n, sig, p0, 0, 0, sh};
        start += n;
    }
    // distinct Bluestein half lengths M = 2 i (i = 1 .. nside), by P then M
    std::vector<int4> it;
    for (int i = 1; i <= nside; ++i) {
        const int P = healpix_blue_P(2 * i);
        if (P) it.push_back(make_int4(2 * i, P, 0, 0));
    }
    std::stable_sort(it.begin(), it.end(), [](const int4 &a, const int4 &b) { return a.y < b.y; });
    std::vector<int64_t> off((size_t)2 * nside + 1, -1);
    int64_t tot = 0;
    for (int4 &x : it) {
        x.z = (int)tot;
        off[x.x] = tot;
        tot += x.y;
    }
    for (HRing &h : hr) {
        const int M = h.nphi / 2;
        // belt rings only: the class runs one kernel instance, of one length
        const bool pow2 = h.nphi == 4 * nside && (M == 512 || M == 1024 || M == 2048 || M == 4096) && lmax < h.nphi;
        h.P = pow2 ? 0 : healpix_blue_P(M);
        h.boff = h.P ? off[M] : 0;
        h.cls = pow2 ? kHpxPow2 : (h.P ? hpx_class_of_P(h.P) : 0);
    }
    if (items) *items = it;
    if (nbhat) *nbhat = (size_t)tot;
}

struct Sizes {
    size_t theta, trig, phitab, phival, twid64, twid32, coef, start, exps, mcut, Fphi, alpha, F, D, jd, jm;
    size_t tab = 0, moff = 0, kstart = 0, rhs = 0, colexp = 0, tabsum = 0, hring = 0;
    size_t twP64 = 0, twP32 = 0, bhat64 = 0, bhat32 = 0, jx = 0, D2 = 0, alpha2 = 0;
    size_t coefP = 0, startP = 0, expsP = 0, mcutP = 0, dscratch = 0, twT = 0;
    size_t total() const
    {
        return theta + trig + phitab + phival + twid64 + twid32 + 2 * coef + start + exps + mcut + Fphi + alpha + F +
               D + jd + jm + tab + moff + kstart + rhs + colexp + tabsum + hring + twP64 + twP32 + bhat64 + bhat32 + jx +
               D2 + alpha2 + 2 * coefP + startP + expsP + mcutP + dscratch + twT;
    }
};

// Whether a plan's workspace holds the scratch of FP32 deflection FFTs:
// plans of FP32 maps on equal-theta rings whose FP64 transform (two buffers
// of nphi / 2 complex) exceeds the 160 KiB of LDS of a gfx950 workgroup.
bool defl32_sized(const Plan &p)
{
    return !p.nside && !p.fp64() && 2 * (size_t)(p.nphi / 2) * sizeof(double2) > (size_t)160 * 1024;
}

Sizes plan_sizes(const Plan &p)
{
    Sizes s;
    const size_t nalm = p.nalm();
    const size_t rowc = (size_t)p.ntheta * (p.lmax + 1);
    const size_t cbytes = p.fp64() ? 16 : 8;
    const size_t rbytes = p.fp64() ? 8 : 4;
    s.theta = p.ntheta * sizeof(double);
    s.trig = p.ntheta * sizeof(double2);
    s.phitab = p.nphi * sizeof(double2);
    s.phival = (p.nphi + 1) * sizeof(double);
    // twiddles e^{2 pi i t / N}: one length, or every HEALPix ring length 4 i
    const size_t ntw = p.nside ? (size_t)2 * p.nside * (p.nside + 1) : (size_t)p.nphi;
    s.twid64 = ntw * sizeof(double2);
    s.twid32 = ntw * sizeof(float2);
    s.hring = p.nside ? (size_t)p.ntheta * sizeof(HRing) : 0;
    if (p.nside && p.hmax_P > 0) {
        std::vector<double> th;
        std::vector<HRing> hr;
        size_t nb = 0;
        healpix_rings(p.nside, p.lmax, th, hr, nullptr, &nb);
        s.twP64 = 8192 * sizeof(double2);
        s.twP32 = 8192 * sizeof(float2);
        s.bhat64 = nb * sizeof(double2);
        s.bhat32 = nb * sizeof(float2);
    }
    s.coef = nalm * sizeof(double4);
    s.start = 3 * (size_t)(p.lmax + 1) * p.jtab * p.nrp * sizeof(double);
    s.exps = 3 * (size_t)(p.lmax + 1) * p.nrp * sizeof(int);
    s.mcut = (size_t)p.nrp * sizeof(int);
    s.Fphi = 2 * (size_t)p.ntheta * (p.lmax_phi + 1) * 16 * (p.tabform() ? p.batch : 1);
    if (p.phi_tables()) {  // the lensing potential's recursion tables (spin 0, J = 1)
        const size_t L = (size_t)p.lmax_phi;
        s.coefP = (L + 1) * (L + 2) / 2 * sizeof(double4);
        s.startP = 3 * (L + 1) * 2 * p.nrp * sizeof(double);
        s.expsP = 3 * (L + 1) * p.nrp * sizeof(int);
        s.mcutP = (size_t)p.nrp * sizeof(int);
    }
    s.alpha = 2 * p.npix() * sizeof(double);
    s.F = (size_t)p.nfield() * (p.order + 1) * rowc * cbytes * (p.tabform() ? p.batch : 1);
    if (p.tabform() && !p.tables) {
        const bool split = p.precision == TL_BF16X3 || p.precision == TL_FP16X2;
        s.moff = (p.lmax + 2) * sizeof(int64_t);
        s.rhs = lp_rhs_bytes(p.lmax, split, (int)p.rhs_nb);
        s.colexp = (size_t)(p.lmax + 1) * 16 * p.rhs_nb * sizeof(float);
    } else if (p.tabform()) {
        std::vector<int64_t> mo;
        s.tab = tab_bytes(p.lmax, p.ntile, p.precision == TL_BF16X3 || p.precision == TL_FP16X2, mo);
        s.moff = (p.lmax + 2) * sizeof(int64_t);
        s.kstart = (size_t)(p.lmax + 1) * (p.ntile > 0 ? p.ntile : 1) * sizeof(int);
        const int nb = tab_rhs_blocks(p.order, p.pol != 0, p.batch);
        s.rhs = tab_rhs_bytes(p.lmax, p.precision == TL_BF16X3 || p.precision == TL_FP16X2, nb);
        s.colexp = (size_t)(p.lmax + 1) * 32 * nb * sizeof(float);
        s.tabsum = tab_sum_bytes(p.lmax, p.nrp - p.rpole, p.order, p.pol != 0, p.batch);
    }
    s.D = p.mix16 ? (size_t)p.nfield() * (mix_n32() * p.dstride * 4 + (p.ndmap() - mix_n32()) * p.dstride16 * 2)
                  : (size_t)p.nfield() * p.ndmap() * p.dstride * rbytes;
    if (defl32_sized(p))  // FP32 rows and deflection of the FP32 deflection FFTs
        s.dscratch = (size_t)2 * p.ntheta * (p.lmax_phi + 1) * 2 * sizeof(float) + 2 * p.npix() * sizeof(float);
    if (!p.nside && theta_fft_grid(p.ntheta))  // twiddles of the theta-derivative FFTs
        s.twT = (size_t)(p.ntheta - 1) * sizeof(double2);
    if (p.tabform() && p.batch > 1) {  // the second set of maps and deflections
        s.D2 = s.D;
        s.alpha2 = s.alpha;
    }
    s.jd = 2 * (size_t)p.ntheta * sizeof(FftJob);
    s.jm = (size_t)p.nfield() * (p.order + 1) * p.ntheta * sizeof(FftJob);
    s.jx = s.jm;
    return s;
}

// Reduced-precision forms: plan-time lambda tables, unless the environment
// variable TAYLENS_ONTHEFLY=1 (read at plan creation) selects the on-the-fly
// recursion (no tables; faster plan creation, less memory, slower per call at
// lmax 4096).
bool use_tables()
{
    const char *e = getenv("TAYLENS_ONTHEFLY");
    return !(e && e[0] == '1');
}

int validate_options(int32_t lmax, tl_grid grid, const tl_options *opt)
{
    if (!opt) return fail(TL_ERR_INVALID, "options pointer is NULL");
    if (lmax < 0) return fail(TL_ERR_INVALID, "lmax must be >= 0");
    if (lmax > 16384) return fail(TL_ERR_UNSUPPORTED, "lmax above 16384 is not supported");
    if (grid.ntheta < 2) return fail(TL_ERR_INVALID, "ntheta must be >= 2");
    if (grid.nphi < 2 || (grid.nphi & 1)) return fail(TL_ERR_INVALID, "nphi must be even and >= 2");
    if ((int64_t)grid.nphi < 2 * (int64_t)lmax)
        return fail(TL_ERR_INVALID, "nphi must be >= 2*lmax (band limit of each ring)");
    if (opt->order < 0 || opt->order > TL_MAX_ORDER) return fail(TL_ERR_INVALID, "order must be in 0..8");
    if (opt->precision < TL_FP64 || opt->precision > TL_BF16) return fail(TL_ERR_INVALID, "unknown precision");
    const bool tab = opt->precision >= TL_BF16X3;
    if (tab && opt->order > 6) return fail(TL_ERR_UNSUPPORTED, "the tabulated precision forms support orders 0..6");
    if (opt->pol != 0 && opt->pol != 1) return fail(TL_ERR_INVALID, "pol must be 0 or 1");
    if (opt->rotate != 0 && opt->rotate != 1) return fail(TL_ERR_INVALID, "rotate must be 0 or 1");
    if (opt->naive_pos != 0 && opt->naive_pos != 1) return fail(TL_ERR_INVALID, "naive_pos must be 0 or 1");
    if (opt->maps16 != 0 && opt->maps16 != 1) return fail(TL_ERR_INVALID, "maps16 must be 0 or 1");
    if (opt->batch < 0 || (!tab && opt->batch > 1))
        return fail(TL_ERR_INVALID, "batch must be 0 or 1 for the FP64 / FP32 forms");
    const int bmax = use_tables() ? tab_max_batch(opt->order, opt->pol != 0, false)
                                  : lp_max_batch(opt->order, opt->pol != 0, false);
    if (tab && opt->batch > bmax)
        return fail(TL_ERR_INVALID, "batch too large for this order (at most " + std::to_string(bmax) + ")");
    if (opt->workspace_cap < 0) return fail(TL_ERR_INVALID, "workspace_cap must be >= 0");
    if (opt->lmax_phi != 0) {
        if (opt->lmax_phi < lmax) return fail(TL_ERR_INVALID, "lmax_phi must be 0 or >= lmax");
        if (opt->lmax_phi > 16384) return fail(TL_ERR_UNSUPPORTED, "lmax_phi above 16384 is not supported");
        if ((int64_t)grid.nphi < 2 * (int64_t)opt->lmax_phi)
            return fail(TL_ERR_INVALID, "nphi must be >= 2*lmax_phi (band limit of the deflection on each ring)");
    }
    if (opt->theta_fft != 0 && opt->theta_fft != 1) return fail(TL_ERR_INVALID, "theta_fft must be 0 or 1");
    if (opt->theta_fft) {
        if (opt->precision != TL_FP64) return fail(TL_ERR_UNSUPPORTED, "theta_fft is an option of the FP64 form");
        if (!theta_fft_grid(grid.ntheta) || (int64_t)lmax > (int64_t)grid.ntheta - 2)
            return fail(TL_ERR_UNSUPPORTED, "theta_fft needs ntheta - 1 a power of two in [2, 4096] and "
                                            "lmax <= ntheta - 2");
    }
    Plan tmp;
    if (!factor_radices(grid.nphi / 2, tmp))
        return fail(TL_ERR_UNSUPPORTED, "nphi/2 must be a product of 2, 3 and 5");
    return TL_OK;
}

// The job of field f, theta-derivative row j into the plan's own maps:
// planes of dstride elements, [field][ndmap][plane]; with mix16, outputs with
// j + k < kMix16 to the FP32 maps [field][6][plane], the others (bit set in
// h16) to the FP16 maps [field][ndmap - 6][plane of dstride16] after them,
// single or paired (Plan::paired, bit q of pair).  off = the ring's first
// pixel.
FftJob int_job(const Plan &p, FftJob a, int f, int j, int64_t off)
{
    const int N = p.order, n16 = p.ndmap() - mix_n32();
    const int64_t s32 = (int64_t)p.dstride, s16 = (int64_t)p.dstride16;
    a.h16 = 0;
    a.pair = 0;
    for (int q = 0; q < a.nk; ++q) {
        const int k = a.k[q];
        // paired planes: the pair's plane starts at the slot of its first map
        const int pos = p.paired ? pair_pos(N, p.mix16, j, k) : 0;
        const int k0 = pos == 2 ? k - 1 : k;
        const int64_t o = pos ? 2 * off : off;
        if (pos == 1) a.pair |= 1 << q;
        if (!p.mix16) {
            a.dst[q] = ((int64_t)f * p.ndmap() + dmap_index(N, j, k0)) * s32 + o;
        } else if (j + k >= kMix16) {
            a.h16 |= 1 << q;
            a.dst[q] = ((int64_t)f * n16 + mix_idx16(N, j, k0)) * s16 + o;
        } else {
            a.dst[q] = ((int64_t)f * mix_n32() + mix_idx32(j, k0)) * s32 + o;
        }
    }
    return a;
}

// FFT jobs of a HEALPix plan: rows to rings of their own length (pad = the
// ring), pixel offsets of RING order; derivative maps scaled by
// delta^(j+k) / (j! k!), delta = pi / (4 nside) (the remap's residual unit).
int build_jobs_healpix(Plan &p)
{
    const int N = p.order;
    const size_t row = (size_t)(p.lmax + 1);
    std::vector<double> th;
    std::vector<HRing> hr;
    healpix_rings(p.nside, p.lmax, th, hr);
    const size_t np = p.npix();
    std::vector<FftJob> jd(2 * (size_t)p.ntheta);
    for (int i = 0; i < p.ntheta; ++i) {
        FftJob a{};
        a.src = (int64_t)((size_t)(1 * p.ntheta + i) * row);  // d_theta phi
        a.nk = 1;
        a.pad = i;
        a.k[0] = 0;
        a.dst[0] = hr[i].start;
        a.scale[0] = 1.0;
        jd[2 * i] = a;
        FftJob b{};
        b.src = (int64_t)((size_t)i * row);                   // d_phi phi / sin theta
        b.nk = 1;
        b.pad = i;
        b.k[0] = 1;
        b.dst[0] = (int64_t)np + hr[i].start;
        b.scale[0] = 1.0 / std::sin(th[i]);
        jd[2 * i + 1] = b;
    }
    p.njobsDefl = (int)jd.size();
    const double del = M_PI / (4.0 * p.nside);
    std::vector<FftJob> jm((size_t)p.nfield() * (N + 1) * p.ntheta);
    std::vector<FftJob> jx(jm.size());
    size_t q = 0;
    for (int f = 0; f < p.nfield(); ++f)
        for (int j = 0; j <= N; ++j)
            for (int i = 0; i < p.ntheta; ++i) {
                FftJob a{};
                a.src = (int64_t)((((size_t)f * (N + 1) + j) * p.ntheta + i) * row);
                a.nk = N - j + 1;
                a.pad = i;
                for (int k = 0; k <= N - j; ++k) {
                    a.k[k] = k;
                    a.dst[k] = (int64_t)(((size_t)f * p.ndmap() + dmap_index(N, j, k)) * np + hr[i].start);
                    a.scale[k] = std::pow(del, j + k) / (factorial(j) * factorial(k));
                }
                jx[q] = int_job(p, a, f, j, hr[i].start);
                jm[q++] = a;
            }
    p.njobsMain = (int)jm.size();
    // each list by FFT class: mixed radix first, then Bluestein by P
    auto by_class = [&](std::vector<FftJob> &v, int *cnt) {
        auto cls = [&](const FftJob &j) { return (int)hr[j.pad].cls; };
        std::stable_sort(v.begin(), v.end(), [&](const FftJob &a, const FftJob &b) { return cls(a) < cls(b); });
        for (int c = 0; c < kHpxClasses; ++c) cnt[c] = 0;
        for (const FftJob &j : v) ++cnt[cls(j)];
    };
    by_class(jd, p.hjobs[0]);
    by_class(jm, p.hjobs[1]);
    {
        int cnt[kHpxClasses];
        by_class(jx, cnt);  // the same stable permutation as jm
    }
    TL_HIP(hipMemcpy(p.jobsDefl.ptr, jd.data(), jd.size() * sizeof(FftJob), hipMemcpyHostToDevice), "jobs copy");
    TL_HIP(hipMemcpy(p.jobsMain.ptr, jm.data(), jm.size() * sizeof(FftJob), hipMemcpyHostToDevice), "jobs copy");
    TL_HIP(hipMemcpy(p.jobsInt.ptr, jx.data(), jx.size() * sizeof(FftJob), hipMemcpyHostToDevice), "jobs copy");
    return TL_OK;
}

int build_jobs(Plan &p)
{
    if (p.nside) return build_jobs_healpix(p);
    const int N = p.order;
    const double dth = M_PI / (double)(p.ntheta - 1);
    const double dph = 2.0 * M_PI / (double)p.nphi;
    const size_t row = (size_t)(p.lmax + 1);
    const size_t rowp = (size_t)(p.lmax_phi + 1);  // the deflection's rows
    // deflection: alpha_theta = d_theta phi (j=1, k=0); alpha_phi = d_phi phi / sin theta
    // (j=0, k=1), on the pole rings +- d_theta d_phi phi (j=1, k=1).
    std::vector<FftJob> jd(2 * (size_t)p.ntheta);
    for (int i = 0; i < p.ntheta; ++i) {
        FftJob a{};
        a.src = (int64_t)((size_t)(1 * p.ntheta + i) * rowp);
        a.nk = 1;
        a.k[0] = 0;
        a.dst[0] = (int64_t)i * p.nphi;
        a.scale[0] = 1.0;
        jd[2 * i] = a;
        FftJob b{};
        b.nk = 1;
        b.k[0] = 1;
        b.dst[0] = (int64_t)((size_t)p.ntheta + i) * p.nphi;
        if (i == 0 || i == p.ntheta - 1) {
            b.src = (int64_t)((size_t)(1 * p.ntheta + i) * rowp);
            b.scale[0] = (i == 0) ? 1.0 : -1.0;
        } else {
            b.src = (int64_t)((size_t)(0 * p.ntheta + i) * rowp);
            b.scale[0] = 1.0 / std::sin(M_PI * (double)i / (double)(p.ntheta - 1));
        }
        jd[2 * i + 1] = b;
    }
    p.njobsDefl = (int)jd.size();
    std::vector<FftJob> jm((size_t)p.nfield() * (N + 1) * p.ntheta);
    std::vector<FftJob> jx(jm.size());
    size_t q = 0;
    for (int f = 0; f < p.nfield(); ++f)
        for (int j = 0; j <= N; ++j)
            for (int i = 0; i < p.ntheta; ++i) {
                FftJob a{};
                a.src = (int64_t)((((size_t)f * (N + 1) + j) * p.ntheta + i) * row);
                a.nk = N - j + 1;
                for (int k = 0; k <= N - j; ++k) {
                    a.k[k] = k;
                    a.dst[k] = (int64_t)((((size_t)f * p.ndmap() + dmap_index(N, j, k)) * p.ntheta + i) * p.nphi);
                    a.scale[k] = std::pow(dth, j) * std::pow(dph, k) / (factorial(j) * factorial(k));
                }
                jx[q] = int_job(p, a, f, j, (int64_t)i * p.nphi);
                jm[q++] = a;
            }
    p.njobsMain = (int)jm.size();
    TL_HIP(hipMemcpy(p.jobsDefl.ptr, jd.data(), jd.size() * sizeof(FftJob), hipMemcpyHostToDevice), "jobs copy");
    TL_HIP(hipMemcpy(p.jobsMain.ptr, jm.data(), jm.size() * sizeof(FftJob), hipMemcpyHostToDevice), "jobs copy");
    TL_HIP(hipMemcpy(p.jobsInt.ptr, jx.data(), jx.size() * sizeof(FftJob), hipMemcpyHostToDevice), "jobs copy");
    return TL_OK;
}

// Ring FFTs of the main rows F into the maps Dout: the plan's own maps
// (padded planes, mixed precision when mix16) or a caller's (plain layout).
hipError_t launch_main_fft(Plan &p, const void *F, void *Dout)
{
    if (p.own(Dout))
        return launch_fft_jobs(p, F, Dout, (const FftJob *)p.jobsInt.ptr, p.njobsMain, p.fp64(), 1,
                               p.mix16 ? p.d16_of(Dout) : nullptr);
    return launch_fft_jobs(p, F, Dout, (const FftJob *)p.jobsMain.ptr, p.njobsMain, p.fp64(), 1);
}

int upload_tables(Plan &p)
{
    std::vector<double> th(p.ntheta);
    std::vector<double2> tr(p.ntheta);
    std::vector<HRing> hr;
    if (p.nside) healpix_rings(p.nside, p.lmax, th, hr);
    for (int i = 0; i < p.ntheta; ++i) {
        if (!p.nside) th[i] = M_PI * (double)i / (double)(p.ntheta - 1);
        tr[i] = make_double2(std::cos(th[i]), std::sin(th[i]));
    }
    if (p.nside) {
        TL_HIP(hipMemcpy(p.hring.ptr, hr.data(), hr.size() * sizeof(HRing), hipMemcpyHostToDevice), "ring copy");
        // twiddles of every ring length N = 4 i at offset 2 i (i - 1)
        std::vector<double2> t64((size_t)2 * p.nside * (p.nside + 1));
        std::vector<float2> t32(t64.size());
        for (int i = 1; i <= p.nside; ++i) {
            const int N = 4 * i;
            const size_t off = (size_t)2 * i * (i - 1);
            for (int t = 0; t < N; ++t) {
                long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)t / (long double)N;
                t64[off + t] = make_double2((double)cosl(a), (double)sinl(a));
                t32[off + t] = make_float2((float)cosl(a), (float)sinl(a));
            }
        }
        TL_HIP(hipMemcpy(p.twid64.ptr, t64.data(), t64.size() * sizeof(double2), hipMemcpyHostToDevice), "tw");
        TL_HIP(hipMemcpy(p.twid32.ptr, t32.data(), t32.size() * sizeof(float2), hipMemcpyHostToDevice), "tw");
        if (p.hmax_P > 0) {
            // twiddles of the power-of-two Bluestein transforms, then the
            // chirp spectra of every Bluestein ring length
            std::vector<double2> w64(8192);
            std::vector<float2> w32(8192);
            for (int t = 0; t < 8192; ++t) {
                long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)t / 8192.0L;
                w64[t] = make_double2((double)cosl(a), (double)sinl(a));
                w32[t] = make_float2((float)cosl(a), (float)sinl(a));
            }
            TL_HIP(hipMemcpy(p.twP64.ptr, w64.data(), w64.size() * sizeof(double2), hipMemcpyHostToDevice), "tw");
            TL_HIP(hipMemcpy(p.twP32.ptr, w32.data(), w32.size() * sizeof(float2), hipMemcpyHostToDevice), "tw");
            std::vector<double> th2;
            std::vector<HRing> hr2;
            std::vector<int4> items;
            healpix_rings(p.nside, p.lmax, th2, hr2, &items);
            TL_HIP(launch_bluestein_tables(p, items), "chirp tables");
        }
    }
    std::vector<double2> pt(p.nphi);
    std::vector<double> pv(p.nphi + 1);
    for (int k = 0; k <= p.nphi; ++k) {
        pv[k] = 2.0 * M_PI * (double)k / (double)p.nphi;
        if (k < p.nphi) pt[k] = make_double2(std::cos(pv[k]), std::sin(pv[k]));
    }
    TL_HIP(hipMemcpy(p.theta.ptr, th.data(), th.size() * sizeof(double), hipMemcpyHostToDevice), "table copy");
    TL_HIP(hipMemcpy(p.trig.ptr, tr.data(), tr.size() * sizeof(double2), hipMemcpyHostToDevice), "table copy");
    TL_HIP(hipMemcpy(p.phitab.ptr, pt.data(), pt.size() * sizeof(double2), hipMemcpyHostToDevice), "table copy");
    TL_HIP(hipMemcpy(p.phival.ptr, pv.data(), pv.size() * sizeof(double), hipMemcpyHostToDevice), "table copy");
    if (p.nside) return TL_OK;
    const int N = p.nphi;  // FFT twiddles e^{2 pi i t / nphi}
    std::vector<double2> t64(N);
    std::vector<float2> t32(N);
    for (int t = 0; t < N; ++t) {
        long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)t / (long double)N;
        t64[t] = make_double2((double)cosl(a), (double)sinl(a));
        t32[t] = make_float2((float)cosl(a), (float)sinl(a));
    }
    TL_HIP(hipMemcpy(p.twid64.ptr, t64.data(), t64.size() * sizeof(double2), hipMemcpyHostToDevice), "table copy");
    TL_HIP(hipMemcpy(p.twid32.ptr, t32.data(), t32.size() * sizeof(float2), hipMemcpyHostToDevice), "table copy");
    if (p.twT.ptr) {  // e^{-2 pi i t / P}, t < P / 2, P = 2 (ntheta - 1)
        const int P = 2 * (p.ntheta - 1);
        std::vector<double2> tt(P / 2);
        for (int t = 0; t < P / 2; ++t) {
            long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)t / (long double)P;
            tt[t] = make_double2((double)cosl(a), -(double)sinl(a));
        }
        TL_HIP(hipMemcpy(p.twT.ptr, tt.data(), tt.size() * sizeof(double2), hipMemcpyHostToDevice), "table copy");
    }
    return TL_OK;
}

int check_plan(tl_plan plan)
{
    if (!plan) return fail(TL_ERR_INVALID, "plan is NULL");
    return TL_OK;
}

void *fphi_slot(Plan &p, int q) { return (char *)p.Fphi.ptr + (size_t)q * 2 * p.ntheta * (p.lmax_phi + 1) * 16; }

// lam / lam' sums of the lensing potentials P[0..n) (NULL entries skipped)
// into fphi_slot(q) by the direct FP64 kernel, realizations sharing the
// recursion, several per launch: every ring, or with caps_only the polar
// caps (the table pass has filled the other rings).
int defl_legendre(Plan &p, int n, const void *const *P, bool caps_only)
{
    const int rend = caps_only ? p.rpole : p.nrp;
    const int mx = direct_max(1, false, false, true);
    DirectSet set{};
    auto flush = [&]() -> int {
        if (!set.n) return TL_OK;
        StageScope sc(p, ST_DEFL_LEG);
        TL_HIP(launch_legendre_scalar_set(p, 1, rend, set, true, true), "deflection legendre");
        set = DirectSet{};
        return TL_OK;
    };
    for (int q = 0; q < n; ++q) {
        if (!P[q]) continue;
        set.a[set.n] = (const double2 *)P[q];
        set.F[set.n] = fphi_slot(p, q);
        if (++set.n == mx) {
            int rc = flush();
            if (rc) return rc;
        }
    }
    return flush();
}

// Deflection of realization q into alpha (default plan.alpha) from fphi_slot(q) (zeros when
// its alm_phi is NULL).
int defl_fft(Plan &p, const void *alm_phi, int q, void *alpha = nullptr)
{
    if (!alpha) alpha = p.alpha.ptr;
    if (!alm_phi) {
        TL_HIP(fill_words(alpha, p.alpha.bytes / 4, 0u, p.stream), "alpha clear");
        return TL_OK;
    }
    StageScope sc(p, ST_DEFL_FFT);
    if (p.defl32) {
        TL_HIP(launch_defl_fft32(p, fphi_slot(p, q), alpha, p.lmax_phi), "deflection fft");
        return TL_OK;
    }
    TL_HIP(launch_fft_jobs(p, fphi_slot(p, q), alpha, (const FftJob *)p.jobsDefl.ptr, p.njobsDefl, true, 0, nullptr,
                           p.lmax_phi),
           "deflection fft");
    return TL_OK;
}

// Deflection of one realization into plan.alpha (zeros when alm_phi is NULL).
int run_deflection(Plan &p, const void *alm_phi)
{
    const void *P[1] = {alm_phi};
    int rc = defl_legendre(p, 1, P, false);
    return rc ? rc : defl_fft(p, alm_phi, 0);
}

// The split table forms take the lensing potential into their pass (two
// more right-hand-side columns per realization) when every realization has
// one.  The single-table FP16 / BF16 forms keep the FP64 deflection: their
// 16-bit lam rounding (relative 2^-12 per term) would reach the positions,
// and a displacement of the order of a pixel turns it into map errors
// against the steep gradients of the band-limited fields.
bool fold_deflection(const Plan &p, int n, const void *const *P)
{
    if (!(p.tables && p.ntile > 0) || !P || p.phi_tables()) return false;
    if (p.precision != TL_BF16X3 && p.precision != TL_FP16X2) return false;
    for (int i = 0; i < n; ++i)
        if (!P[i]) return false;
    return true;
}

// Whether the polar caps of n realizations of this FP32-row plan take the
// one combined launch (orders up to 6; caps present).
bool caps_one_launch(const Plan &p, int n, bool hasb)
{
    return !p.fp64() && p.rpole > 0 && n >= 1 && n <= kTabMaxBatch && caps_nb(1, p.order, hasb) > 0;
}

// Polar caps (ring pairs below rpole) of n realizations in one launch: T,
// both spin families of Q/U and, with P, the lensing potential's FP64 rows
// (fphi_slot) -- FP32 rows Fout[q] laid out [field][N + 1][ring][m].
int run_caps(Plan &p, int n, const void *const *T, const void *const *E, const void *const *B, const void *const *P,
             void *const *Fout, bool hasb, hipStream_t st = nullptr)
{
    const size_t rowc = (size_t)p.ntheta * (p.lmax + 1) * (p.order + 1);
    CapsArgs a{};
    auto add = [&](int kind) {
        const int nb = caps_nb(kind, p.order, hasb);
        for (int i0 = 0; i0 < n; i0 += nb) a.task[a.ntask++] = make_int4(kind, i0, std::min(nb, n - i0), 0);
    };
    for (int q = 0; q < n; ++q) {
        char *F = (char *)Fout[q];
        a.T[q] = (const double2 *)T[q];
        a.E[q] = p.pol ? (const double2 *)E[q] : nullptr;
        a.B[q] = hasb ? (const double2 *)B[q] : nullptr;
        a.P[q] = P ? (const double2 *)P[q] : nullptr;
        a.FT[q] = F;
        a.FQ[q] = p.pol ? F + rowc * 8 : nullptr;
        a.FU[q] = p.pol ? F + 2 * rowc * 8 : nullptr;
        a.FP[q] = P ? fphi_slot(p, q) : nullptr;
    }
    if (P) add(0);
    add(1);
    if (p.pol) {
        add(2);
        add(3);
    }
    StageScope sc(p, ST_CAPS);
    TL_HIP(launch_legendre_caps(p, p.rpole, a, p.pol ? n : 0, hasb, st), "legendre caps");
    return TL_OK;
}

// Harmonic stage of n realizations (n <= plan batch for the table forms).
// P (optional): their lensing potentials; when fold_deflection() holds, the
// lam / lam' sums of phi outside the caps go to fphi_slot(q).
// j0: the direct kernels synthesize the rows j = 0 only (the FP64 form
// with theta_fft, whose maps then take their theta-derivatives by FFT)
int run_legendre_many(Plan &p, int n, const void *const *T, const void *const *E, const void *const *B,
                      void *const *Fout, const void *const *P = nullptr, bool j0 = false)
{
    const int J = j0 ? 0 : p.order;
    const size_t rowc = (size_t)p.ntheta * (p.lmax + 1) * (p.order + 1);
    const size_t cb = p.fp64() ? 16 : 8;
    const bool hasb = p.pol && B[0] != nullptr;
    // FP32 form: matrix-core contraction away from the polar caps; tabulated
    // forms: table GEMM away from the caps; caps and the FP64 form: direct
    // FP64 recursion.
    const bool mfma = p.precision == TL_FP32 && mfma_supported(p.order, hasb);
    const bool tab = p.tabform() && p.ntile > 0;
    const int rend = (mfma || tab) ? p.rpole : p.nrp;
    p.caps_defl_done = false;
    const bool caps1 = (mfma || tab) && caps_one_launch(p, n, hasb);
    // tabulated passes with a second stream: the caps run there, beside the
    // table epilogue (they write only the cap rings' rows)
    const bool side_caps = caps1 && tab && p.tables && p.overlap();
    bool caps_pending = side_caps;
    auto caps = [&](hipStream_t st) -> int {
        const bool defl = fold_deflection(p, n, P);
        int rc = run_caps(p, n, T, E, B, defl ? P : nullptr, Fout, hasb, st);
        if (!rc) p.caps_defl_done = defl;
        return rc;
    };
    if (caps1 && !side_caps) {
        int rc = caps(p.stream);
        if (rc) return rc;
    }
    // direct kernels: several realizations per launch share the recursion
    for (int i0 = 0, mx = direct_max(p.order, false, false, p.fp64()); !caps1 && i0 < n; i0 += mx) {
        DirectSet set{};
        set.n = std::min(mx, n - i0);
        for (int q = 0; q < set.n; ++q) {
            set.a[q] = (const double2 *)T[i0 + q];
            set.F[q] = Fout[i0 + q];
        }
        StageScope sc(p, ST_LEG_T);
        TL_HIP(launch_legendre_scalar_set(p, J, rend, set, p.fp64()), "legendre T");
    }
    for (int i0 = 0, mx = direct_max(p.order, true, hasb, p.fp64()); !caps1 && p.pol && i0 < n; i0 += mx) {
        DirectSet set{};
        set.n = std::min(mx, n - i0);
        for (int q = 0; q < set.n; ++q) {
            char *F = (char *)Fout[i0 + q];
            set.a[q] = (const double2 *)E[i0 + q];
            set.b[q] = hasb ? (const double2 *)B[i0 + q] : nullptr;
            set.F[q] = F + rowc * cb;
            set.G[q] = F + 2 * rowc * cb;
        }
        StageScope sc(p, ST_LEG_QU);
        TL_HIP(launch_legendre_spin_set(p, J, rend, set, p.fp64()), "legendre QU");
    }
    for (int i = 0; i < n; ++i) {
        char *F = (char *)Fout[i];
        if (mfma) {
            StageScope sc(p, ST_LEG_MFMA);
            TL_HIP(launch_legendre_mfma(p, T[i], E[i], B[i], F, p.pol ? F + rowc * cb : nullptr,
                                        p.pol ? F + 2 * rowc * cb : nullptr),
                   "legendre mfma");
        }
    }
    if (tab) {
        const int gmax = p.tables ? tab_max_batch(p.order, p.pol != 0, hasb) : lp_max_batch(p.order, p.pol != 0, hasb);
        for (int i0 = 0; i0 < n; i0 += gmax) {
            TabBatch b{};
            b.n = std::min(gmax, n - i0);
            for (int q = 0; q < b.n; ++q) {
                char *F = (char *)Fout[i0 + q];
                b.T[q] = (const double2 *)T[i0 + q];
                b.E[q] = (const double2 *)E[i0 + q];
                b.B[q] = (const double2 *)B[i0 + q];
                b.FT[q] = (float2 *)F;
                b.FQ[q] = (float2 *)(F + rowc * cb);
                b.FU[q] = (float2 *)(F + 2 * rowc * cb);
                if (fold_deflection(p, n, P)) {
                    b.P[q] = (const double2 *)P[i0 + q];
                    b.FP[q] = (double2 *)fphi_slot(p, i0 + q);
                }
            }
            {
                StageScope sc(p, ST_TAB_RHS);
                TL_HIP(p.tables ? launch_legendre_tab(p, b, 0) : launch_legendre_lp(p, b, 0),
                       "legendre right-hand sides");
            }
            {
                StageScope sc(p, ST_TAB_GEMM);
                TL_HIP(p.tables ? launch_legendre_tab(p, b, 1) : launch_legendre_lp(p, b, 1),
                       "legendre matrix-core stage");
            }
            if (caps_pending) {
                TL_HIP(hipEventRecord(p.ev_gemm, p.stream), "stream order");
                TL_HIP(hipStreamWaitEvent(p.side, p.ev_gemm, 0), "stream order");
                const int rc = caps(p.side);
                if (rc) return rc;
                TL_HIP(hipEventRecord(p.ev_caps, p.side), "stream order");
                caps_pending = false;
            }
            if (p.tables) {
                StageScope sc(p, ST_TAB_EPI);
                TL_HIP(launch_legendre_tab(p, b, 2), "legendre table epilogue");
            }
        }
    }
    if (side_caps) TL_HIP(hipStreamWaitEvent(p.stream, p.ev_caps, 0), "stream order");
    return TL_OK;
}

// all_j = false: only what the derivative maps need (rows j = 0 with theta_fft)
int run_legendre(Plan &p, const void *T, const void *E, const void *B, void *Fout, bool all_j = true)
{
    const void *Ts[1] = {T}, *Es[1] = {E}, *Bs[1] = {B};
    void *Fs[1] = {Fout};
    return run_legendre_many(p, 1, Ts, Es, Bs, Fs, nullptr, !all_j && p.theta_fft);
}

// Derivative maps from the harmonic rows: ring FFTs of every row j, or with
// theta_fft ring FFTs of the rows j = 0 (the maps D_0k) and the maps j >= 1
// by FFT along the great circles through both poles.
hipError_t maps_from_rows(Plan &p, const void *F, void *Dout)
{
    if (!p.theta_fft) return launch_main_fft(p, F, Dout);
    const int N = p.order, nf = p.nfield();
    const bool own = p.own(Dout);
    const FftJob *jobs = (const FftJob *)(own ? p.jobsInt.ptr : p.jobsMain.ptr);
    for (int f = 0; f < nf; ++f) {
        const hipError_t e =
            launch_fft_jobs(p, F, Dout, jobs + (size_t)f * (N + 1) * p.ntheta, p.ntheta, p.fp64(), 1);
        if (e != hipSuccess) return e;
    }
    const size_t ds = own ? p.dstride : (size_t)p.ntheta * p.nphi;
    const size_t rb = p.fp64() ? 8 : 4;
    for (int k = 0; k < N; ++k) {  // D_jk = dtheta^j / j! d^j_theta D_0k, j = 1..N-k
        const ThetaFftLayout lay{(size_t)p.ndmap() * ds, (size_t)p.ndmap() * ds, ds, N + 1, 1, k};
        const hipError_t e = launch_theta_fft(p, (const char *)Dout + (size_t)k * ds * rb, Dout, nf, N - k, lay);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int run_derivs(Plan &p, const void *T, const void *E, const void *B, void *Dout)
{
    int rc = run_legendre(p, T, E, B, p.F.ptr, false);
    if (rc) return rc;
    StageScope sc(p, ST_FFT);
    TL_HIP(maps_from_rows(p, p.F.ptr, Dout), "ring fft");
    return TL_OK;
}

int check_fields(const Plan &p, const void *T, const void *E)
{
    if (!T) return fail(TL_ERR_INVALID, "alm_T is NULL");
    if (p.pol && !E) return fail(TL_ERR_INVALID, "alm_E is NULL for a polarized plan");
    return TL_OK;
}

int check_outputs(const Plan &p, const void *T, const void *Q, const void *U)
{
    if (!T) return fail(TL_ERR_INVALID, "T_out is NULL");
    if (p.pol && (!Q || !U)) return fail(TL_ERR_INVALID, "Q_out/U_out are NULL for a polarized plan");
    return TL_OK;
}

int set_device_of(Plan &p)
{
    int cur = 0;
    TL_HIP(hipGetDevice(&cur), "hipGetDevice");
    if (cur != p.device) TL_HIP(hipSetDevice(p.device), "hipSetDevice");
    return TL_OK;
}

// Work counts for tl_plan_query, from the evanescent cut and the table's
// first non-empty chunks (mirrors which blocks the kernels visit).
hipError_t count_work(Plan &p)
{
    std::vector<int> mc(p.nrp);
    hipError_t e = hipMemcpy(mc.data(), p.mcut.ptr, p.nrp * sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    p.q_elems = p.q_elems_caps = 0;
    for (int r = 0; r < p.nrp; ++r) {
        const int64_t top = std::min(mc[r], p.lmax);
        // sum_{m=0}^{top} (lmax - m + 1)
        const int64_t n = top < 0 ? 0 : (top + 1) * (int64_t)(p.lmax + 1) - top * (top + 1) / 2;
        p.q_elems += n;
        if (r < p.rpole) p.q_elems_caps += n;
    }
    p.q_tab_chunks = p.q_tab_chunk_bytes = 0;
    if (p.tabform() && p.tables && p.ntile > 0) {
        const int nspl = (p.precision == TL_BF16X3 || p.precision == TL_FP16X2) ? 2 : 1;
        p.q_tab_chunk_bytes = (int64_t)nspl * 4 * 64 * 16;
        std::vector<int> ks((size_t)(p.lmax + 1) * p.ntile);
        e = hipMemcpy(ks.data(), p.kstart.ptr, ks.size() * sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
        for (int m = 0; m <= p.lmax; ++m) {
            const int nk = (p.lmax - m + 1 + 31) / 32;
            for (int g = 0; g * 4 < p.ntile; ++g) {
                bool any = false;  // some ring of the 4 tiles at or below its cut + 2
                for (int t = g * 4; t < std::min(p.ntile, g * 4 + 4) && !any; ++t)
                    for (int rl = 0; rl < 32 && !any; ++rl) {
                        const int r = p.rpole + t * 32 + rl;
                        if (r < p.nrp && m <= mc[r] + 2) any = true;
                    }
                if (!any) continue;
                for (int t = g * 4; t < std::min(p.ntile, g * 4 + 4); ++t)
                    p.q_tab_chunks += std::max(0, nk - ks[(size_t)m * p.ntile + t]);
            }
        }
    }
    return hipSuccess;
}

}  // namespace

struct tl_plan_s {
    Plan p;
};

struct tl_cnn_s {
    CnnBufs c;
    int device = 0;
    int step = 0;
    DevBuf params, m, v, grad, packed;
    DevBuf work;   // training activations
    DevBuf corr;   // float [3][n] scratch of the training calls / full-map correction
};

struct tl_batch_s {
    int n = 0;
    std::vector<tl_plan> plans;
    int order = 0, pol = 0, device = 0, ncu = 256;
    hipStream_t user = nullptr;     // the plans' stream
    hipStream_t bs = nullptr;       // the batch's own stream (capturable)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<DevBuf> F;          // harmonic-stage output per realization (complex64)
    DevBuf jobs, items, head;
    int nitems = 0;
    int m_groups = 1, gpc = 2;
    bool autotune = false, use_graph = false, tuned = false;
    double tuned_ms = 0.0;
    int64_t replays = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void *> cap_alms;
    std::vector<void *> cap_outs;
    std::string key;
};

namespace {

void free_cnn(tl_cnn_s *h)
{
    DevBuf *b[] = {&h->params, &h->m, &h->v, &h->grad, &h->packed, &h->work, &h->corr};
    for (DevBuf *x : b) free_buf(*x);
}

// Grow a scratch buffer of the network (synchronizes before a reallocation).
int cnn_reserve(tl_cnn_s *h, DevBuf &b, size_t bytes, hipStream_t st)
{
    if (b.bytes >= bytes) return TL_OK;
    TL_HIP(hipStreamSynchronize(st), "synchronize");
    free_buf(b);
    TL_HIP(hipMalloc(&b.ptr, bytes), "cnn scratch");
    b.bytes = bytes;
    if (&b == &h->work) h->c.work = b.ptr;
    return TL_OK;
}

int cnn_check_plan(tl_plan plan, tl_cnn net)
{
    if (!plan) return fail(TL_ERR_INVALID, "plan is NULL");
    if (!net) return fail(TL_ERR_INVALID, "network is NULL");
    const Plan &p = plan->p;
    if (p.order != 2 || !p.pol || p.fp64() || p.nside)
        return fail(TL_ERR_UNSUPPORTED,
                    "the correction network needs an order-2 polarized equal-theta plan with float maps");
    return TL_OK;
}

int cnn_check_pixels(const Plan &p, const float *D, const double *at, const double *ap, const int64_t *pix,
                     int64_t n)
{
    if (!D || !at || !ap) return fail(TL_ERR_INVALID, "NULL derivative maps or deflection");
    if (n < 0) return fail(TL_ERR_INVALID, "pixel count must be >= 0");
    if (!pix && (size_t)n > p.npix()) return fail(TL_ERR_INVALID, "n exceeds the map size with pix NULL");
    return TL_OK;
}

// forward (training mode) + backward into net->c.grad
int cnn_grad_run(tl_cnn net, Plan &p, const float *D, const double *at, const double *ap, const int64_t *pix,
                 int64_t n, const float *target)
{
    int rc;
    if ((rc = cnn_reserve(net, net->work, std::max<size_t>(1, (size_t)n) * cnn_train_bytes_per_pixel(), p.stream)))
        return rc;
    if ((rc = cnn_reserve(net, net->corr, std::max<size_t>(1, (size_t)n) * 3 * sizeof(float), p.stream))) return rc;
    TL_HIP(cnn_forward(p, net->c, D, at, ap, pix, n, (float *)net->corr.ptr, true, p.stream), "cnn forward");
    TL_HIP(cnn_backward(net->c, n, target, p.stream), "cnn backward");
    return TL_OK;
}

// ---------------------------------------------------------------- batch --

void batch_drop_graph(tl_batch_s *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->cap_alms.clear();
    b->cap_outs.clear();
}

void free_batch(tl_batch_s *b)
{
    batch_drop_graph(b);
    for (auto &f : b->F) free_buf(f);
    free_buf(b->jobs);
    free_buf(b->items);
    free_buf(b->head);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->bs) (void)hipStreamDestroy(b->bs);
}

size_t batch_rowc(const Plan &p) { return (size_t)p.ntheta * (p.lmax + 1) * (p.order + 1); }

// Work items (realization, ring block, first m-group, m-groups), longest first.
int batch_items(tl_batch_s *b, int nmg)
{
    const int RPB = mfma_ring_block(), MG = mfma_m_group();
    struct It {
        int4 w;
        double cost;
    };
    std::vector<It> v;
    for (int i = 0; i < b->n; ++i) {
        const Plan &p = b->plans[i]->p;
        const int nr = p.nrp - p.rpole;
        const int ngrp = (p.lmax + 1 + MG - 1) / MG;
        for (int rb = 0; rb * RPB < nr; ++rb) {
            const int rings = std::min(RPB, nr - rb * RPB);
            for (int g0 = 0; g0 < ngrp; g0 += nmg) {
                const int cnt = std::min(nmg, ngrp - g0);
                double c = 0.0;
                for (int m = g0 * MG; m < std::min((g0 + cnt) * MG, p.lmax + 1); ++m) c += (double)(p.lmax - m + 1);
                v.push_back({make_int4(i, rb, g0, cnt), c * rings});
            }
        }
    }
    std::stable_sort(v.begin(), v.end(), [](const It &a, const It &c) { return a.cost > c.cost; });
    std::vector<int4> w(v.size());
    for (size_t k = 0; k < v.size(); ++k) w[k] = v[k].w;
    free_buf(b->items);
    b->nitems = (int)w.size();
    if (w.empty()) return TL_OK;
    TL_HIP(hipMalloc(&b->items.ptr, w.size() * sizeof(int4)), "batch items");
    b->items.bytes = w.size() * sizeof(int4);
    TL_HIP(hipMemcpy(b->items.ptr, w.data(), b->items.bytes, hipMemcpyHostToDevice), "batch items");
    return TL_OK;
}

std::string tune_path()
{
    const char *e = getenv("TAYLENS_TUNE_CACHE");
    if (e && *e) return e;
    const char *h = getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/taylens_tune.txt";
}

bool tune_lookup(const std::string &key, int &nmg, int &gpc, double &ms)
{
    FILE *f = fopen(tune_path().c_str(), "r");
    if (!f) return false;
    char line[1024];
    bool hit = false;
    while (fgets(line, sizeof line, f)) {
        char k[900];
        int a = 0, c = 0;
        double t = 0;
        if (sscanf(line, "%899s %d %d %lf", k, &a, &c, &t) == 4 && key == k && a >= 1 && a <= 8 && c >= 1 &&
            c <= 8) {
            nmg = a;
            gpc = c;
            ms = t;
            hit = true;  // the last entry wins
        }
    }
    fclose(f);
    return hit;
}

void tune_store(const std::string &key, int nmg, int gpc, double ms)
{
    const std::string path = tune_path();
    const size_t sl = path.rfind('/');
    if (sl != std::string::npos) (void)mkdir(path.substr(0, sl).c_str(), 0755);
    FILE *f = fopen(path.c_str(), "a");
    if (!f) return;  // not cached
    fprintf(f, "%s %d %d %.6f\n", key.c_str(), nmg, gpc, ms);
    fclose(f);
}

int batch_queue_launch(tl_batch_s *b, bool hasb)
{
    TL_HIP(fill_words(b->head.ptr, 1, 0u, b->bs), "queue head");
    TL_HIP(launch_legendre_mfma_queue(b->order, b->pol != 0, hasb, b->bs, (const MfmaJob *)b->jobs.ptr,
                                      (const int4 *)b->items.ptr, b->nitems, (int *)b->head.ptr, b->gpc * b->ncu),
           "persistent harmonic kernel");
    return TL_OK;
}

// Time the candidate work-item shapes on this batch; keep the fastest.
int batch_tune(tl_batch_s *b, bool hasb)
{
    int nmg = 1, gpc = 2;
    double ms = 0.0;
    if (tune_lookup(b->key, nmg, gpc, ms)) {
        b->m_groups = nmg;
        b->gpc = gpc;
        b->tuned_ms = ms;
        b->tuned = true;
        return batch_items(b, nmg);
    }
    hipEvent_t e0, e1;
    TL_HIP(hipEventCreate(&e0), "event");
    TL_HIP(hipEventCreate(&e1), "event");
    double best = 1e300;
    int bn = 1, bg = 2;
    int rc = TL_OK;
    const int cand_m[] = {1, 2, 4}, cand_g[] = {1, 2, 4};
    for (int cm : cand_m) {
        if ((rc = batch_items(b, cm))) break;
        for (int cg : cand_g) {
            b->gpc = cg;
            if ((rc = batch_queue_launch(b, hasb))) break;  // warm-up
            hipError_t e = hipEventRecord(e0, b->bs);
            if (e == hipSuccess && (rc = batch_queue_launch(b, hasb))) break;
            if (e == hipSuccess) e = hipEventRecord(e1, b->bs);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) {
                rc = hipfail(e, "autotune timing");
                break;
            }
            if (t < best) {
                best = t;
                bn = cm;
                bg = cg;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    b->m_groups = bn;
    b->gpc = bg;
    b->tuned_ms = best;
    b->tuned = true;
    tune_store(b->key, bn, bg, best);
    return batch_items(b, bn);
}

int batch_enqueue(tl_batch_s *b, const void *const *alms, void *const *outs, bool hasb)
{
    // polar caps (direct FP64 kernels) of every realization
    for (int i = 0; i < b->n; ++i) {
        Plan &p = b->plans[i]->p;
        char *F = (char *)b->F[i].ptr;
        const size_t rc8 = batch_rowc(p) * 8;
        if (caps_one_launch(p, 1, hasb)) {  // as a single call of the plan does
            void *Fs[1] = {F};
            const int rc = run_caps(p, 1, &alms[4 * i], &alms[4 * i + 1], &alms[4 * i + 2], nullptr, Fs, hasb);
            if (rc) return rc;
            continue;
        }
        TL_HIP(launch_legendre_scalar(p, p.order, p.rpole, alms[4 * i], F, false), "legendre T");
        if (p.pol)
            TL_HIP(launch_legendre_spin(p, p.order, p.rpole, alms[4 * i + 1], alms[4 * i + 2], F + rc8, F + 2 * rc8,
                                        false),
                   "legendre QU");
    }
    int rc = batch_queue_launch(b, hasb);
    if (rc) return rc;
    for (int i = 0; i < b->n; ++i) {
        Plan &p = b->plans[i]->p;
        if ((rc = run_deflection(p, alms[4 * i + 3]))) return rc;
        TL_HIP(launch_main_fft(p, b->F[i].ptr, p.D.ptr),
               "ring fft");
        const double *at = (const double *)p.alpha.ptr;
        TL_HIP(launch_remap(p, p.D.ptr, at, at + p.npix(), nullptr, nullptr, outs[3 * i], outs[3 * i + 1],
                            outs[3 * i + 2]),
               "remap");
    }
    return TL_OK;
}

// Point every plan at the batch stream for the duration of a run.
struct BatchStreams {
    tl_batch_s *b;
    std::vector<hipStream_t> keep;
    explicit BatchStreams(tl_batch_s *bb) : b(bb)
    {
        for (auto pl : b->plans) {
            keep.push_back(pl->p.stream);
            pl->p.stream = b->bs;
        }
    }
    ~BatchStreams()
    {
        // reverse order: a plan listed twice gets its first-seen stream back
        for (size_t i = keep.size(); i-- > 0;) b->plans[i]->p.stream = keep[i];
    }
};

// Plan fields from validated options (no device work).
void plan_fields(Plan &p, int32_t lmax, tl_grid grid, const tl_options *opt, void *hip_stream, int nside = 0)
{
    p.lmax = lmax;
    p.lmax_phi = opt->lmax_phi > 0 ? opt->lmax_phi : lmax;
    p.theta_fft = opt->theta_fft == 1 && nside == 0;
    p.nside = nside;
    if (nside) {
        grid.ntheta = 4 * nside - 1;  // HEALPix rings; nphi = the longest ring
        grid.nphi = 4 * nside;
    }
    p.ntheta = grid.ntheta;
    p.nphi = grid.nphi;
    p.nrp = (grid.ntheta + 1) / 2;
    p.order = opt->order;
    p.jtab = (opt->order > 1 ? opt->order : 1) + 1;
    p.precision = opt->precision;
    p.pol = opt->pol;
    p.rotate = opt->rotate;
    p.naive = opt->naive_pos;
    p.cap = opt->workspace_cap;
    p.stream = (hipStream_t)hip_stream;
    factor_radices(p.nphi / 2, p);
    {
        // polar caps stay on the direct FP64 kernel: the csc and cot jets of
        // the L-power epilogue amplify the rounding of the contraction there.
        // sin theta < 0.15 in general; 0.05 for the split FP16 form, whose
        // scaled 22-bit operands keep the first ring outside its caps at
        // about 5e-6 of the map RMS at lmax 4096 (4e-6 at 0.08, 1.6e-6 at
        // 0.15, 1e-5 at 0.03)
        const double smin = p.precision == TL_FP16X2 ? 0.05 : 0.15;
        std::vector<double> th;
        std::vector<HRing> hr;
        if (p.nside) {
            healpix_rings(p.nside, lmax, th, hr);
            p.hmax_direct = 0;
            p.hmax_P = 0;
            p.hmax_pow2 = 0;
            for (const HRing &h : hr) {
                if (h.cls == kHpxPow2) p.hmax_pow2 = std::max(p.hmax_pow2, h.nphi / 2);
                else if (h.P) p.hmax_P = std::max(p.hmax_P, (int)h.P);
                else p.hmax_direct = std::max(p.hmax_direct, h.nphi / 2);
            }
        }
        auto sin_ring = [&](int r) {
            return p.nside ? std::sin(th[r]) : std::sin(M_PI * (double)r / (double)(p.ntheta - 1));
        };
        // the equal-theta grid's pole ring always stays direct (its deflection
        // is a limit); HEALPix has no pole ring
        int rp = p.nside ? 0 : 1;
        while (rp < p.nrp && sin_ring(rp) < smin) ++rp;
        // Large caps fill whole 64-lane waves of the direct kernels (a wave
        // walks the whole l recursion for its 64 ring pairs, however few are
        // live): down to a multiple of 64 when that gives up at most 1/16 of
        // the cap, else up (more rings on the direct FP64 kernels, in the
        // same wall time).
        if (rp >= 48) {
            const int dn = rp / 64 * 64;
            rp = (dn >= 64 && rp - dn <= rp / 16) ? dn : std::min(p.nrp, (rp + 63) / 64 * 64);
        }
        p.rpole = rp;
    }
    p.batch = opt->batch > 1 ? opt->batch : 1;
    // maps16: orders >= 3 of the FP32-map forms on the equal-theta grid keep
    // D_jk with j + k >= 3 in FP16 (the remap scales them by |u|^j |v|^k <=
    // 1/8: 6e-7 to 1.2e-6 of the map RMS for the lensed CMB at lmax 4096, up
    // to ~1e-4 for power at the band limit).  Not on HEALPix rings, whose
    // offsets in units of delta reach nside / i on polar ring i.
    p.mix16 = opt->maps16 == 1 && !p.fp64() && p.order >= kMix16 && p.nside == 0;
    // paired FP16 planes where the ring FFT runs in one workgroup (pow2 rings)
    p.paired = p.mix16 && grid.nphi % 2 == 0 && fft_p2(grid.nphi / 2);
    {
        auto padded = [](size_t n, size_t q) {
            const size_t b = (n + q - 1) / q;
            return (b | 1) * q;
        };
        const size_t np = nside ? (size_t)12 * nside * nside : (size_t)grid.ntheta * grid.nphi;
        p.dstride = padded(np, p.fp64() ? 32 : 64);  // 256-byte units
        p.dstride16 = padded(np, 128);
    }
    p.ntile = (p.nrp - p.rpole + 31) / 32;
    p.tables = p.tabform() && use_tables();
    if (p.precision == TL_FP16 || p.precision == TL_FP16X2) {
        // Addition theorem: sum_m |Y_lm|^2 = (2l+1)/4pi and, differentiated
        // twice at coincident points, sum_m |d_theta Y_lm|^2 = (2l+1)/4pi *
        // l(l+1)/2, so |lam_lm| and |lam'_lm| stay below these at every theta.
        // FP16 hi + lo holds 22 bits only while the lo part is normal, i.e.
        // for |value| >= 2^-3: scale both so their bound sits just below 2^15.
        const double L = (double)p.lmax;
        const double b0 = std::sqrt((2.0 * L + 1.0) / (4.0 * M_PI));
        const double b1 = std::sqrt((2.0 * L + 1.0) / (4.0 * M_PI) * L * (L + 1.0) * 0.5);
        p.lam_e0 = (int)std::floor(std::log2(32768.0 / b0));
        p.lam_e1 = b1 > 0.0 ? (int)std::floor(std::log2(32768.0 / b1)) : p.lam_e0;
    }
    if (p.tabform()) p.rhs_nb = p.tables ? tab_rhs_blocks(p.order, p.pol != 0, p.batch)
                                         : lp_rhs_blocks(p.order, p.pol != 0, p.batch);
}

// The current device, and whether the FP64 ring FFT of this nphi fits in LDS.
int plan_device_checks(Plan &p)
{
    TL_HIP(hipGetDevice(&p.device), "hipGetDevice");
    int smem = 0;
    TL_HIP(hipDeviceGetAttribute(&smem, hipDeviceAttributeMaxSharedMemoryPerBlock, p.device),
           "hipDeviceGetAttribute");
    // ring FFT buffers in LDS: 2 M (equal-theta); HEALPix: 2 M + 1 for the
    // mixed-radix rings, P + P / 32 for the Bluestein ones
    const size_t need64 = p.nside ? std::max({2 * (size_t)p.hmax_direct + 1, (size_t)(p.hmax_P + p.hmax_P / 32),
                                              (size_t)(p.hmax_pow2 + p.hmax_pow2 / 32)}) *
                                        sizeof(double2)
                                  : 2 * (size_t)(p.nphi / 2) * sizeof(double2);
    // equal-theta rings too long for the FP64 transform: plans of FP32 maps
    // take the deflection's ring FFTs in FP32 as well
    const size_t need32 = 2 * (size_t)(p.nphi / 2) * sizeof(float2);
    p.defl32 = defl32_sized(p) && need64 > (size_t)smem && need32 <= (size_t)smem;
    if (need64 > (size_t)smem && !p.defl32)
        return fail(TL_ERR_UNSUPPORTED, "nphi too large for the FP64 ring FFT in LDS on this device (" +
                                            std::to_string(need64) + " > " + std::to_string(smem) + " bytes)");
    return TL_OK;
}

struct BufItem {
    DevBuf *b;
    size_t n;
    const char *name;
};

std::vector<BufItem> plan_buffer_list(Plan &p, const Sizes &sz)
{
    return {{&p.theta, sz.theta, "theta"},   {&p.trig, sz.trig, "trig"},       {&p.phitab, sz.phitab, "phitab"},
            {&p.phival, sz.phival, "phival"}, {&p.twid64, sz.twid64, "twid64"}, {&p.twid32, sz.twid32, "twid32"},
            {&p.coef0, sz.coef, "coef0"},    {&p.coef2, sz.coef, "coef2"},     {&p.start, sz.start, "start"},
            {&p.exps, sz.exps, "exps"},      {&p.mcut, sz.mcut, "mcut"},       {&p.Fphi, sz.Fphi, "Fphi"},
            {&p.alpha, sz.alpha, "alpha"},   {&p.F, sz.F, "F"},                {&p.D, sz.D, "D"},
            {&p.jobsDefl, sz.jd, "jobsDefl"}, {&p.jobsMain, sz.jm, "jobsMain"}, {&p.jobsInt, sz.jx, "jobsInt"},
            {&p.tab, sz.tab, "tab"},
            {&p.moff, sz.moff, "moff"},      {&p.kstart, sz.kstart, "kstart"}, {&p.rhs, sz.rhs, "rhs"},
            {&p.colexp, sz.colexp, "colexp"}, {&p.tabsum, sz.tabsum, "tabsum"}, {&p.hring, sz.hring, "hring"},
            {&p.twP64, sz.twP64, "twP64"},   {&p.twP32, sz.twP32, "twP32"},   {&p.bhat64, sz.bhat64, "bhat64"},
            {&p.bhat32, sz.bhat32, "bhat32"}, {&p.D2, sz.D2, "D2"},       {&p.alpha2, sz.alpha2, "alpha2"},
            {&p.coefP0, sz.coefP, "coefP0"}, {&p.coefP2, sz.coefP, "coefP2"}, {&p.startP, sz.startP, "startP"},
            {&p.expsP, sz.expsP, "expsP"},   {&p.mcutP, sz.mcutP, "mcutP"},   {&p.dscratch, sz.dscratch, "dscratch"},
            {&p.twT, sz.twT, "twT"}};
}

// Everything a plan computes into its buffers once they exist: angle and
// twiddle tables, FFT jobs, recursion coefficients, start values and the
// evanescent cut, the lambda tables of the tabulated forms; waits for them
// and counts the work.
int plan_setup(Plan &p)
{
    int rc;
    if (p.D2.ptr) {  // the second stream of a tabulated batch (default priority)
        hipError_t e = hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking);
        for (int i = 0; i < 2 && e == hipSuccess; ++i) {
            e = hipEventCreateWithFlags(&p.ev_fft[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&p.ev_remap[i], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p.ev_gemm, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p.ev_caps, hipEventDisableTiming);
        if (e != hipSuccess) return hipfail(e, "second stream");
    }
    if ((rc = upload_tables(p))) return rc;
    if ((rc = build_jobs(p))) return rc;
    hipError_t e = hipMemsetAsync(p.start.ptr, 0, p.start.bytes, p.stream);
    if (e == hipSuccess) e = hipMemsetAsync(p.exps.ptr, 0, p.exps.bytes, p.stream);
    if (e == hipSuccess) e = launch_tables(p);
    if (e == hipSuccess && p.tabform() && !p.tables) {
        std::vector<int64_t> go;
        lp_groups(p.lmax, go);
        e = hipMemcpy(p.moff.ptr, go.data(), go.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && p.tabform() && p.tables && p.ntile > 0) {
        std::vector<int64_t> mo;
        tab_bytes(p.lmax, p.ntile, p.precision == TL_BF16X3 || p.precision == TL_FP16X2, mo);
        e = hipMemcpy(p.moff.ptr, mo.data(), mo.size() * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemsetAsync(p.kstart.ptr, 0x7f, p.kstart.bytes, p.stream);
        if (e == hipSuccess) e = launch_build_tab(p);
    }
    if (e == hipSuccess) e = fft_prepare(p);
    if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
    if (e == hipSuccess) e = count_work(p);
    if (e != hipSuccess) return hipfail(e, "plan tables");
    return TL_OK;
}

// The whole path for one realization on a plan whose arguments are checked.
int lens_map_core(Plan &p, const void *alm_T, const void *alm_E, const void *alm_B, const void *alm_phi,
                  void *T_out, void *Q_out, void *U_out)
{
    int rc;
    if (fold_deflection(p, 1, &alm_phi)) {
        const void *Ts[1] = {alm_T}, *Es[1] = {alm_E}, *Bs[1] = {alm_B}, *Ps[1] = {alm_phi};
        void *Fs[1] = {p.F.ptr};
        if ((rc = run_legendre_many(p, 1, Ts, Es, Bs, Fs, Ps))) return rc;
        if (!p.caps_defl_done && (rc = defl_legendre(p, 1, Ps, true))) return rc;
        if ((rc = defl_fft(p, alm_phi, 0))) return rc;
        StageScope sc(p, ST_FFT);
        TL_HIP(launch_main_fft(p, p.F.ptr, p.D.ptr),
               "ring fft");
    } else {
        if ((rc = run_deflection(p, alm_phi))) return rc;
        if ((rc = run_derivs(p, alm_T, alm_E, alm_B, p.D.ptr))) return rc;
    }
    const double *at = (const double *)p.alpha.ptr;
    StageScope sc(p, ST_REMAP);
    TL_HIP(launch_remap(p, p.D.ptr, at, at + p.npix(), nullptr, nullptr, T_out, Q_out, U_out), "remap");
    return TL_OK;
}

// ---- allocation-free lensing: the workspace in a static device array ----

// Largest workspace of tl_lens_map_simple_noalloc (128 MiB): T+Q/U at order 4
// up to lmax ~ 256 on the 513 x 1024 grid, T-only larger.  Each device the
// library runs on holds its own copy until the process ends.
constexpr size_t kScratchBytes = (size_t)128 << 20;

std::mutex g_scratch_mu;
constexpr int kScratchDevices = 64;
void *g_scratch_ptr[kScratchDevices] = {};

}  // namespace

// Device copy of the workspace.  Its name is only a host-side handle: host
// code uses the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Address of `scratch` on device dev (current), looked up once per device.
int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kScratchDevices) return fail(TL_ERR_UNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hipfail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(TL_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TL_OK;
}

}  // namespace

extern "C" {

int tl_version(void) { return TL_VERSION; }

const char *tl_last_error(void) { return g_err.c_str(); }

int tl_plan_create(tl_plan *out, int32_t lmax, tl_grid grid, const tl_options *opt, void *hip_stream)
{
    if (!out) return fail(TL_ERR_INVALID, "plan output pointer is NULL");
    *out = nullptr;
    int rc = validate_options(lmax, grid, opt);
    if (rc) return rc;

    tl_plan_s *h = new (std::nothrow) tl_plan_s();
    if (!h) return fail(TL_ERR_NOMEM, "host allocation failed");
    Plan &p = h->p;
    plan_fields(p, lmax, grid, opt, hip_stream);
    Sizes sz = plan_sizes(p);
    if (p.cap > 0 && sz.total() > (size_t)p.cap) {
        delete h;
        return fail(TL_ERR_NOMEM, "plan needs " + std::to_string(sz.total()) + " bytes, above workspace_cap " +
                                      std::to_string(p.cap));
    }
    if ((rc = plan_device_checks(p))) {
        delete h;
        return rc;
    }
    for (auto &it : plan_buffer_list(p, sz)) {
        if (it.n == 0) continue;
        rc = alloc(p, *it.b, it.n, it.name);
        if (rc) {
            free_plan_buffers(p);
            delete h;
            return rc;
        }
    }
    if ((rc = plan_setup(p))) {
        free_plan_buffers(p);
        delete h;
        return rc;
    }
    *out = h;
    return TL_OK;
}

int tl_plan_create_healpix(tl_plan *out, int32_t lmax, int32_t nside, const tl_options *opt, void *hip_stream)
{
    if (!out) return fail(TL_ERR_INVALID, "plan output pointer is NULL");
    *out = nullptr;
    if (nside < 1) return fail(TL_ERR_INVALID, "nside must be >= 1");
    if (nside > 2048) return fail(TL_ERR_UNSUPPORTED, "nside above 2048 is not supported (FP64 ring FFT in LDS)");
    // the options and lmax as for the equal-theta grid; the ring lengths of a
    // HEALPix grid need no relation to lmax (the ring synthesis folds m)
    int32_t n2 = 8;  // a power of two >= 2 lmax stands in for the ring length
    while (n2 < 2 * (int64_t)lmax && n2 < (1 << 30)) n2 *= 2;
    tl_grid g{3, n2};
    if (opt && opt->lmax_phi != 0 && opt->lmax_phi != lmax)
        return fail(TL_ERR_UNSUPPORTED, "a separate lmax_phi is not supported on HEALPix rings");
    if (opt && opt->theta_fft != 0)
        return fail(TL_ERR_UNSUPPORTED, "theta_fft needs the equal-theta grid");
    int rc = validate_options(lmax, g, opt);
    if (rc) return rc;
    tl_plan_s *h = new (std::nothrow) tl_plan_s();
    if (!h) return fail(TL_ERR_NOMEM, "host allocation failed");
    Plan &p = h->p;
    plan_fields(p, lmax, g, opt, hip_stream, nside);
    Sizes sz = plan_sizes(p);
    if (p.cap > 0 && sz.total() > (size_t)p.cap) {
        delete h;
        return fail(TL_ERR_NOMEM, "plan needs " + std::to_string(sz.total()) + " bytes, above workspace_cap " +
                                      std::to_string(p.cap));
    }
    if ((rc = plan_device_checks(p))) {
        delete h;
        return rc;
    }
    for (auto &it : plan_buffer_list(p, sz)) {
        if (it.n == 0) continue;
        rc = alloc(p, *it.b, it.n, it.name);
        if (rc) {
            free_plan_buffers(p);
            delete h;
            return rc;
        }
    }
    if ((rc = plan_setup(p))) {
        free_plan_buffers(p);
        delete h;
        return rc;
    }
    *out = h;
    return TL_OK;
}

int tl_plan_destroy(tl_plan plan)
{
    if (!plan) return TL_OK;
    Plan &p = plan->p;
    (void)set_device_of(p);
    (void)hipStreamSynchronize(p.stream);
    clear_prof(p);
    free_plan_buffers(p);
    delete plan;
    return TL_OK;
}

int tl_plan_profile(tl_plan plan, int32_t enable)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    Plan &p = plan->p;
    int rc = set_device_of(p);
    if (rc) return rc;
    TL_HIP(hipStreamSynchronize(p.stream), "synchronize");
    clear_prof(p);
    p.profile = enable != 0;
    return TL_OK;
}

int tl_plan_stage_times(tl_plan plan, double *ms, int64_t *calls)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    if (!ms) return fail(TL_ERR_INVALID, "ms is NULL");
    Plan &p = plan->p;
    int rc = set_device_of(p);
    if (rc) return rc;
    TL_HIP(hipStreamSynchronize(p.stream), "synchronize");
    for (int i = 0; i < TL_NSTAGE; ++i) {
        ms[i] = 0.0;
        if (calls) calls[i] = 0;
    }
    for (auto &r : p.prof) {
        float t = 0.f;
        TL_HIP(hipEventElapsedTime(&t, r.a, r.b), "event time");
        ms[r.stage] += t;
        if (calls) calls[r.stage] += 1;
    }
    return TL_OK;
}

int tl_plan_query(tl_plan plan, int32_t key, int64_t *value)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    if (!value) return fail(TL_ERR_INVALID, "value pointer is NULL");
    const Plan &p = plan->p;
    switch (key) {
    case TL_Q_RPOLE: *value = p.rpole; return TL_OK;
    case TL_Q_ELEMS: *value = p.q_elems; return TL_OK;
    case TL_Q_ELEMS_CAPS: *value = p.q_elems_caps; return TL_OK;
    case TL_Q_TAB_CHUNKS: *value = p.q_tab_chunks; return TL_OK;
    case TL_Q_TAB_CHUNK_BYTES: *value = p.q_tab_chunk_bytes; return TL_OK;
    case TL_Q_DEFL_FOLDED: {
        const void *one[1] = {&p};  // any non-NULL potential
        *value = fold_deflection(p, 1, one) ? 1 : 0;
        return TL_OK;
    }
    default: return fail(TL_ERR_INVALID, "unknown query key " + std::to_string(key));
    }
}

int tl_plan_workspace_bytes(tl_plan plan, int64_t *bytes)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    if (!bytes) return fail(TL_ERR_INVALID, "bytes pointer is NULL");
    *bytes = (int64_t)plan->p.total_bytes;
    return TL_OK;
}

int tl_deflection(tl_plan plan, const void *alm_phi, double *alpha_theta, double *alpha_phi)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    Plan &p = plan->p;
    if (!alm_phi || !alpha_theta || !alpha_phi) return fail(TL_ERR_INVALID, "NULL argument");
    int rc = set_device_of(p);
    if (rc) return rc;
    if ((rc = run_deflection(p, alm_phi))) return rc;
    const size_t bytes = p.npix() * sizeof(double);
    TL_HIP(hipMemcpyAsync(alpha_theta, p.alpha.ptr, bytes, hipMemcpyDeviceToDevice, p.stream), "copy");
    TL_HIP(hipMemcpyAsync(alpha_phi, (char *)p.alpha.ptr + bytes, bytes, hipMemcpyDeviceToDevice, p.stream), "copy");
    return TL_OK;
}

int tl_legendre(tl_plan plan, const void *alm_T, const void *alm_E, const void *alm_B, void *F_out)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    Plan &p = plan->p;
    int rc = check_fields(p, alm_T, alm_E);
    if (rc) return rc;
    if (!F_out) return fail(TL_ERR_INVALID, "F_out is NULL");
    if ((rc = set_device_of(p))) return rc;
    return run_legendre(p, alm_T, alm_E, alm_B, F_out);
}

int tl_synth_derivs(tl_plan plan, const void *alm_T, const void *alm_E, const void *alm_B, void *D_out)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    Plan &p = plan->p;
    int rc = check_fields(p, alm_T, alm_E);
    if (rc) return rc;
    if (!D_out) return fail(TL_ERR_INVALID, "D_out is NULL");
    if ((rc = set_device_of(p))) return rc;
    return run_derivs(p, alm_T, alm_E, alm_B, D_out);
}

int tl_remap(tl_plan plan, const void *D, const double *alpha_theta, const double *alpha_phi, void *T_out,
             void *Q_out, void *U_out)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    Plan &p = plan->p;
    if (!D || !alpha_theta || !alpha_phi) return fail(TL_ERR_INVALID, "NULL argument");
    int rc = check_outputs(p, T_out, Q_out, U_out);
    if (rc) return rc;
    if ((rc = set_device_of(p))) return rc;
    TL_HIP(launch_remap(p, D, alpha_theta, alpha_phi, nullptr, nullptr, T_out, Q_out, U_out), "remap");
    return TL_OK;
}

int tl_analysis_T(tl_plan plan, const double *map, void *alm_out)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    Plan &p = plan->p;
    if (!map || !alm_out) return fail(TL_ERR_INVALID, "NULL argument");
    if ((uintptr_t)map % 8 || (uintptr_t)alm_out % 16) return fail(TL_ERR_INVALID, "misaligned map or alm_out");
    if (p.nside) return fail(TL_ERR_UNSUPPORTED, "the analysis needs the equal-theta grid");
    if (!analysis_grid(p.nphi))
        return fail(TL_ERR_UNSUPPORTED, "the analysis needs nphi a power of two in [2, 8192]");
    if (p.F.bytes < analysis_scratch_bytes(p))
        return fail(TL_ERR_UNSUPPORTED, "the plan's harmonic-stage buffer is too small for the analysis "
                                        "(use order >= 1, a polarized plan or the FP64 form)");
    int rc = set_device_of(p);
    if (rc) return rc;
    TL_HIP(launch_analysis_T(p, map, alm_out), "analysis");
    return TL_OK;
}

int tl_theta_derivs(tl_plan plan, const void *maps, int32_t nmaps, int32_t jmax, void *out)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    Plan &p = plan->p;
    if (!maps || !out) return fail(TL_ERR_INVALID, "NULL argument");
    if (jmax < 1 || jmax > TL_MAX_ORDER) return fail(TL_ERR_INVALID, "jmax must be in 1..8");
    if (nmaps < 0) return fail(TL_ERR_INVALID, "nmaps must be >= 0");
    const size_t vec = p.fp64() ? 16 : 8;
    if ((uintptr_t)maps % vec || (uintptr_t)out % vec)
        return fail(TL_ERR_INVALID, "maps and out must be aligned to two values");
    if (p.nside || !p.twT.ptr)
        return fail(TL_ERR_UNSUPPORTED, "theta-derivative FFTs need an equal-theta plan with ntheta - 1 a power of "
                                        "two in [2, 4096]");
    if (p.lmax > p.ntheta - 2)
        return fail(TL_ERR_UNSUPPORTED, "theta-derivative FFTs need lmax <= ntheta - 2");
    // one workgroup of 512 threads per pair of circles and map; the grid's
    // work items must stay below 2^32
    const int64_t nwg = (int64_t)((p.nphi / 2 + 1) / 2) * nmaps;
    if (nwg * 512 > (int64_t)UINT32_MAX) return fail(TL_ERR_INVALID, "too many maps for one launch");
    if (nmaps == 0) return TL_OK;
    int rc = set_device_of(p);
    if (rc) return rc;
    const size_t plane = (size_t)p.ntheta * p.nphi;
    const ThetaFftLayout lay{plane, (size_t)jmax * plane, plane, 1, 0, -1};
    TL_HIP(launch_theta_fft(p, maps, out, nmaps, jmax, lay), "theta fft");
    return TL_OK;
}

int tl_lens_map(tl_plan plan, const void *alm_T, const void *alm_E, const void *alm_B, const void *alm_phi,
                void *T_out, void *Q_out, void *U_out)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    Plan &p = plan->p;
    int rc = check_fields(p, alm_T, alm_E);
    if (rc) return rc;
    if ((rc = check_outputs(p, T_out, Q_out, U_out))) return rc;
    if ((rc = set_device_of(p))) return rc;
    return lens_map_core(p, alm_T, alm_E, alm_B, alm_phi, T_out, Q_out, U_out);
}

int tl_lens_map_pos(tl_plan plan, const void *alm_T, const void *alm_E, const void *alm_B, const double *theta_src,
                    const double *phi_src, void *T_out, void *Q_out, void *U_out)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    Plan &p = plan->p;
    int rc = check_fields(p, alm_T, alm_E);
    if (rc) return rc;
    if (!theta_src || !phi_src) return fail(TL_ERR_INVALID, "position pointers are NULL");
    if ((rc = check_outputs(p, T_out, Q_out, U_out))) return rc;
    if ((rc = set_device_of(p))) return rc;
    if ((rc = run_derivs(p, alm_T, alm_E, alm_B, p.D.ptr))) return rc;
    TL_HIP(launch_remap(p, p.D.ptr, nullptr, nullptr, theta_src, phi_src, T_out, Q_out, U_out), "remap");
    return TL_OK;
}

int tl_lens_map_batch(int32_t n, const tl_plan *plans, const void *const *alms, void *const *outs)
{
    if (n < 0) return fail(TL_ERR_INVALID, "n must be >= 0");
    if (n == 0) return TL_OK;
    if (!plans || !alms || !outs) return fail(TL_ERR_INVALID, "NULL argument");
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return fail(TL_ERR_INVALID, "plan " + std::to_string(i) + " is NULL");
        int rc = check_fields(plans[i]->p, alms[4 * i], alms[4 * i + 1]);
        if (rc) return rc;
        if ((rc = check_outputs(plans[i]->p, outs[3 * i], outs[3 * i + 1], outs[3 * i + 2]))) return rc;
    }
    hipStream_t s0 = plans[0]->p.stream;
    // Every plan's workspace is used on s0 for this pass: s0 first waits for
    // the work already queued on each other plan stream, and afterwards each
    // of those streams waits for s0 (outputs and workspace reuse).
    std::vector<hipStream_t> others;
    for (int i = 0; i < n; ++i) {
        hipStream_t s = plans[i]->p.stream;
        if (s != s0 && std::find(others.begin(), others.end(), s) == others.end()) others.push_back(s);
    }
    int rc = set_device_of(plans[0]->p);
    if (rc) return rc;
    hipEvent_t ev = nullptr;
    if (!others.empty()) {
        TL_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
        for (hipStream_t s : others) {
            hipError_t e = hipEventRecord(ev, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(s0, ev, 0);
            if (e != hipSuccess) {
                (void)hipEventDestroy(ev);
                return hipfail(e, "stream ordering");
            }
        }
    }
    for (int i = 0; i < n && rc == TL_OK; ++i) {
        Plan &p = plans[i]->p;
        hipStream_t keep = p.stream;
        p.stream = s0;
        rc = tl_lens_map(plans[i], alms[4 * i], alms[4 * i + 1], alms[4 * i + 2], alms[4 * i + 3], outs[3 * i],
                         outs[3 * i + 1], outs[3 * i + 2]);
        p.stream = keep;
    }
    if (ev) {
        // also on failure: work queued before it must still order the streams
        hipError_t e = hipEventRecord(ev, s0);
        for (size_t k = 0; e == hipSuccess && k < others.size(); ++k) e = hipStreamWaitEvent(others[k], ev, 0);
        (void)hipEventDestroy(ev);
        if (e != hipSuccess && rc == TL_OK) return hipfail(e, "stream ordering");
    }
    return rc;
}

int tl_lens_map_many(tl_plan plan, int32_t n, const void *const *alms, void *const *outs)
{
    if (check_plan(plan)) return TL_ERR_INVALID;
    if (n < 0) return fail(TL_ERR_INVALID, "n must be >= 0");
    if (n == 0) return TL_OK;
    if (!alms || !outs) return fail(TL_ERR_INVALID, "NULL argument");
    Plan &p = plan->p;
    int rc;
    for (int i = 0; i < n; ++i) {
        if ((rc = check_fields(p, alms[4 * i], alms[4 * i + 1]))) return rc;
        if ((rc = check_outputs(p, outs[3 * i], outs[3 * i + 1], outs[3 * i + 2]))) return rc;
        if ((alms[4 * i + 2] == nullptr) != (alms[2] == nullptr))
            return fail(TL_ERR_INVALID, "alm_B must be given for all realizations or for none");
    }
    if ((rc = set_device_of(p))) return rc;
    const size_t rowbytes = (size_t)p.nfield() * (p.order + 1) * p.ntheta * (p.lmax + 1) * (p.fp64() ? 16 : 8);
    const int g = p.tabform() ? p.batch : 1;
    const bool ovl = p.overlap() && n > 1;
    int u = 0;  // realizations launched
    for (int i0 = 0; i0 < n; i0 += g) {
        const int k = std::min(g, n - i0);
        const void *T[kTabMaxBatch], *E[kTabMaxBatch], *B[kTabMaxBatch], *P[kTabMaxBatch];
        void *F[kTabMaxBatch];
        for (int q = 0; q < k; ++q) {
            T[q] = alms[4 * (i0 + q)];
            E[q] = alms[4 * (i0 + q) + 1];
            B[q] = alms[4 * (i0 + q) + 2];
            P[q] = alms[4 * (i0 + q) + 3];
            F[q] = (char *)p.F.ptr + q * rowbytes;
        }
        const bool fold = fold_deflection(p, k, P);
        if ((rc = run_legendre_many(p, k, T, E, B, F, P, p.theta_fft))) return rc;
        // deflection sums of the whole group (outside the caps from the
        // table pass when folded), then per realization: deflection FFT,
        // ring FFTs, remap
        if (!(fold && p.caps_defl_done) && (rc = defl_legendre(p, k, P, fold))) return rc;
        for (int q = 0; q < k; ++q, ++u) {
            // realization u uses set u % 2 of maps and deflections (overlap)
            const int st = ovl ? (u & 1) : 0;
            void *D = st ? p.D2.ptr : p.D.ptr, *alpha = st ? p.alpha2.ptr : p.alpha.ptr;
            if (ovl && u >= 2) TL_HIP(hipStreamWaitEvent(p.stream, p.ev_remap[st], 0), "stream order");
            if ((rc = defl_fft(p, P[q], q, alpha))) return rc;
            {
                StageScope sc(p, ST_FFT);
                TL_HIP(maps_from_rows(p, F[q], D), "ring fft");
            }
            const double *at = (const double *)alpha;
            void *To = outs[3 * (i0 + q)], *Qo = outs[3 * (i0 + q) + 1], *Uo = outs[3 * (i0 + q) + 2];
            if (ovl) {
                // the remap on the second stream, after this realization's FFTs
                TL_HIP(hipEventRecord(p.ev_fft[st], p.stream), "stream order");
                TL_HIP(hipStreamWaitEvent(p.side, p.ev_fft[st], 0), "stream order");
                TL_HIP(launch_remap(p, D, at, at + p.npix(), nullptr, nullptr, To, Qo, Uo, nullptr, p.side),
                       "remap");
                TL_HIP(hipEventRecord(p.ev_remap[st], p.side), "stream order");
            } else {
                StageScope sc(p, ST_REMAP);
                TL_HIP(launch_remap(p, D, at, at + p.npix(), nullptr, nullptr, To, Qo, Uo), "remap");
            }
        }
    }
    // the plan's stream waits for the last remap (the second stream runs in order)
    if (ovl && u > 0) TL_HIP(hipStreamWaitEvent(p.stream, p.ev_remap[(u - 1) & 1], 0), "stream order");
    return TL_OK;
}

int tl_batch_create(tl_batch *out, int32_t n, const tl_plan *plans, const tl_batch_options *opt)
{
    if (!out) return fail(TL_ERR_INVALID, "batch output pointer is NULL");
    *out = nullptr;
    if (n <= 0) return fail(TL_ERR_INVALID, "n must be >= 1");
    if (!plans || !opt) return fail(TL_ERR_INVALID, "NULL argument");
    if (opt->m_groups < 0 || opt->m_groups > 8 || opt->groups_per_cu < 0 || opt->groups_per_cu > 8)
        return fail(TL_ERR_INVALID, "m_groups and groups_per_cu must be in 0..8");
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return fail(TL_ERR_INVALID, "plan " + std::to_string(i) + " is NULL");
        const Plan &p = plans[i]->p;
        const Plan &p0 = plans[0]->p;
        if (p.precision != TL_FP32) return fail(TL_ERR_UNSUPPORTED, "a batch needs TL_FP32 plans");
        if (p.nside) return fail(TL_ERR_UNSUPPORTED, "a batch needs equal-theta plans");
        if (p.order != p0.order || p.pol != p0.pol) return fail(TL_ERR_INVALID, "plans differ in order or pol");
        if (p.stream != p0.stream || p.device != p0.device) return fail(TL_ERR_INVALID, "plans differ in stream");
        if (!mfma_supported(p.order, p.pol != 0)) return fail(TL_ERR_UNSUPPORTED, "order too high for the batch");
    }
    tl_batch_s *b = new (std::nothrow) tl_batch_s;
    if (!b) return fail(TL_ERR_NOMEM, "host allocation failed");
    auto bail = [&](int code) {
        free_batch(b);
        delete b;
        return code;
    };
    b->n = n;
    b->plans.assign(plans, plans + n);
    const Plan &p0 = plans[0]->p;
    b->order = p0.order;
    b->pol = p0.pol;
    b->device = p0.device;
    b->user = p0.stream;
    b->autotune = opt->autotune != 0;
    b->use_graph = opt->use_graph != 0;
    b->m_groups = opt->m_groups ? opt->m_groups : 1;
    b->gpc = opt->groups_per_cu ? opt->groups_per_cu : 2;
    int rc = set_device_of(plans[0]->p);
    if (rc) return bail(rc);
    hipError_t e = hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->bs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) return bail(hipfail(e, "batch stream"));
    b->F.resize(n);
    std::vector<std::pair<int, int>> shapes;
    for (int i = 0; i < n; ++i) {
        const Plan &p = plans[i]->p;
        const size_t bytes = (size_t)p.nfield() * batch_rowc(p) * 8;
        e = hipMalloc(&b->F[i].ptr, bytes);
        if (e != hipSuccess) return bail(fail(TL_ERR_NOMEM, "batch harmonic output: out of device memory"));
        b->F[i].bytes = bytes;
        shapes.push_back({p.lmax, p.ntheta});
    }
    e = hipMalloc(&b->jobs.ptr, n * sizeof(MfmaJob));
    if (e == hipSuccess) e = hipMalloc(&b->head.ptr, 256);
    if (e != hipSuccess) return bail(hipfail(e, "batch buffers"));
    b->jobs.bytes = n * sizeof(MfmaJob);
    b->head.bytes = 256;
    std::sort(shapes.begin(), shapes.end());
    b->key = "mfmaq-N" + std::to_string(b->order) + "-P" + std::to_string(b->pol) + "-cu" + std::to_string(b->ncu);
    for (size_t k = 0; k < shapes.size();) {
        size_t j = k;
        while (j < shapes.size() && shapes[j] == shapes[k]) ++j;
        b->key += "-" + std::to_string(shapes[k].first) + "x" + std::to_string(shapes[k].second) + "." +
                  std::to_string(j - k);
        k = j;
    }
    if ((rc = batch_items(b, b->m_groups))) return bail(rc);
    *out = b;
    return TL_OK;
}

int tl_batch_destroy(tl_batch b)
{
    if (!b) return TL_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->bs);
    free_batch(b);
    (void)hipSetDevice(cur);
    delete b;
    return TL_OK;
}

int tl_batch_run(tl_batch b, const void *const *alms, void *const *outs)
{
    if (!b) return fail(TL_ERR_INVALID, "batch is NULL");
    if (!alms || !outs) return fail(TL_ERR_INVALID, "NULL argument");
    int rc;
    const bool hasb = b->pol && alms[2] != nullptr;
    for (int i = 0; i < b->n; ++i) {
        const Plan &p = b->plans[i]->p;
        if ((rc = check_fields(p, alms[4 * i], alms[4 * i + 1]))) return rc;
        if ((rc = check_outputs(p, outs[3 * i], outs[3 * i + 1], outs[3 * i + 2]))) return rc;
        if (b->pol && ((alms[4 * i + 2] != nullptr) != hasb))
            return fail(TL_ERR_INVALID, "alm_B must be set for all realizations or for none");
    }
    if ((rc = set_device_of(b->plans[0]->p))) return rc;
    for (auto pl : b->plans)
        if (pl->p.stream != b->user) return fail(TL_ERR_INVALID, "a plan's stream changed since the batch was made");
    // order after the caller's earlier work, and the caller's later work after this
    TL_HIP(hipEventRecord(b->ev_in, b->user), "event");
    TL_HIP(hipStreamWaitEvent(b->bs, b->ev_in, 0), "event wait");
    BatchStreams guard(b);
    bool profiling = false;
    for (auto pl : b->plans) profiling |= pl->p.profile;
    const bool same = b->exec && !profiling && b->cap_alms.size() == (size_t)4 * b->n &&
                      std::equal(b->cap_alms.begin(), b->cap_alms.end(), alms) &&
                      std::equal(b->cap_outs.begin(), b->cap_outs.end(), outs);
    if (same) {
        TL_HIP(hipGraphLaunch(b->exec, b->bs), "graph launch");
        b->replays += 1;
    } else {
        // the captured graph's persistent kernel reads b->jobs, rewritten
        // below: it no longer describes these arguments
        batch_drop_graph(b);
        std::vector<MfmaJob> J(b->n);
        for (int i = 0; i < b->n; ++i) {
            const Plan &p = b->plans[i]->p;
            char *F = (char *)b->F[i].ptr;
            const size_t rc8 = batch_rowc(p) * 8;
            J[i] = mfma_job(p, alms[4 * i], alms[4 * i + 1], alms[4 * i + 2], F, p.pol ? F + rc8 : nullptr,
                            p.pol ? F + 2 * rc8 : nullptr);
        }
        TL_HIP(hipMemcpyAsync(b->jobs.ptr, J.data(), J.size() * sizeof(MfmaJob), hipMemcpyHostToDevice, b->bs),
               "batch jobs");
        TL_HIP(hipStreamSynchronize(b->bs), "synchronize");
        if (b->autotune && !b->tuned && (rc = batch_tune(b, hasb))) return rc;
        if (b->use_graph && !profiling) {
            batch_drop_graph(b);
            TL_HIP(hipStreamBeginCapture(b->bs, hipStreamCaptureModeThreadLocal), "begin capture");
            rc = batch_enqueue(b, alms, outs, hasb);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(b->bs, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return hipfail(e, "end capture");
            b->graph = g;
            TL_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
            TL_HIP(hipGraphLaunch(b->exec, b->bs), "graph launch");
            b->cap_alms.assign(alms, alms + 4 * b->n);
            b->cap_outs.assign(outs, outs + 3 * b->n);
        } else if ((rc = batch_enqueue(b, alms, outs, hasb))) {
            return rc;
        }
    }
    TL_HIP(hipEventRecord(b->ev_out, b->bs), "event");
    TL_HIP(hipStreamWaitEvent(b->user, b->ev_out, 0), "event wait");
    return TL_OK;
}

int tl_batch_info(tl_batch b, int32_t *m_groups, int32_t *groups_per_cu, double *tuned_ms, int64_t *graph_replays)
{
    if (!b) return fail(TL_ERR_INVALID, "batch is NULL");
    if (m_groups) *m_groups = b->m_groups;
    if (groups_per_cu) *groups_per_cu = b->gpc;
    if (tuned_ms) *tuned_ms = b->tuned ? b->tuned_ms : 0.0;
    if (graph_replays) *graph_replays = b->replays;
    return TL_OK;
}

int tl_cnn_create(tl_cnn *out, const float *params)
{
    if (!out) return fail(TL_ERR_INVALID, "network output pointer is NULL");
    *out = nullptr;
    if (!params) return fail(TL_ERR_INVALID, "params is NULL");
    tl_cnn_s *h = new (std::nothrow) tl_cnn_s;
    if (!h) return fail(TL_ERR_NOMEM, "host allocation failed");
    auto bail = [&](int code) {
        free_cnn(h);
        delete h;
        return code;
    };
    hipError_t e = hipGetDevice(&h->device);
    struct {
        DevBuf *b;
        size_t bytes;
    } list[] = {{&h->params, kCnnParam * sizeof(float)},
                {&h->m, kCnnTrain * sizeof(float)},
                {&h->v, kCnnTrain * sizeof(float)},
                {&h->grad, (kCnnTrain + 1) * sizeof(float)},
                {&h->packed, cnn_packed_bytes()}};
    for (auto &x : list) {
        if (e != hipSuccess) break;
        e = hipMalloc(&x.b->ptr, x.bytes);
        if (e == hipSuccess) x.b->bytes = x.bytes;
    }
    if (e != hipSuccess) return bail(hipfail(e, "cnn allocation"));
    h->c.params = h->params.ptr;
    h->c.m = h->m.ptr;
    h->c.v = h->v.ptr;
    h->c.grad = h->grad.ptr;
    // packed operands: layer 1 (14 steps), layer 2 (18), layer 3 (2), 64 x 16 B each
    h->c.W1p = h->packed.ptr;
    h->c.W2p = (char *)h->packed.ptr + 14 * 64 * 16;
    h->c.W3p = (char *)h->packed.ptr + (14 + 18) * 64 * 16;
    *out = h;
    const int rc = tl_cnn_set_params(h, params);
    if (rc) {
        *out = nullptr;
        return bail(rc);
    }
    return TL_OK;
}

int tl_cnn_destroy(tl_cnn net)
{
    if (!net) return TL_OK;
    (void)hipDeviceSynchronize();
    free_cnn(net);
    delete net;
    return TL_OK;
}

int tl_cnn_get_params(tl_cnn net, float *params_out)
{
    if (!net || !params_out) return fail(TL_ERR_INVALID, "NULL argument");
    TL_HIP(hipDeviceSynchronize(), "synchronize");
    TL_HIP(hipMemcpy(params_out, net->params.ptr, kCnnParam * sizeof(float), hipMemcpyDeviceToHost), "copy");
    return TL_OK;
}

int tl_cnn_set_params(tl_cnn net, const float *params)
{
    if (!net || !params) return fail(TL_ERR_INVALID, "NULL argument");
    for (int i = 0; i < kCnnParam; ++i)
        if (!std::isfinite(params[i])) return fail(TL_ERR_INVALID, "non-finite parameter");
    TL_HIP(hipDeviceSynchronize(), "synchronize");
    TL_HIP(hipMemcpy(net->params.ptr, params, kCnnParam * sizeof(float), hipMemcpyHostToDevice), "copy");
    TL_HIP(hipMemset(net->m.ptr, 0, net->m.bytes), "clear");
    TL_HIP(hipMemset(net->v.ptr, 0, net->v.bytes), "clear");
    net->step = 0;
    TL_HIP(cnn_pack(net->c, nullptr), "cnn pack");
    TL_HIP(hipDeviceSynchronize(), "synchronize");
    return TL_OK;
}

int tl_cnn_forward(tl_cnn net, tl_plan plan, const float *D, const double *alpha_theta, const double *alpha_phi,
                   const int64_t *pix, int64_t n, float *corr_out)
{
    int rc = cnn_check_plan(plan, net);
    if (rc) return rc;
    Plan &p = plan->p;
    if ((rc = cnn_check_pixels(p, D, alpha_theta, alpha_phi, pix, n))) return rc;
    if (!corr_out) return fail(TL_ERR_INVALID, "corr_out is NULL");
    if ((rc = set_device_of(p))) return rc;
    TL_HIP(cnn_forward(p, net->c, D, alpha_theta, alpha_phi, pix, n, corr_out, false, p.stream), "cnn forward");
    return TL_OK;
}

int tl_cnn_grad(tl_cnn net, tl_plan plan, const float *D, const double *alpha_theta, const double *alpha_phi,
                const int64_t *pix, int64_t n, const float *target, float *grad_out)
{
    int rc = cnn_check_plan(plan, net);
    if (rc) return rc;
    Plan &p = plan->p;
    if ((rc = cnn_check_pixels(p, D, alpha_theta, alpha_phi, pix, n))) return rc;
    if (!target || !grad_out) return fail(TL_ERR_INVALID, "target or grad_out is NULL");
    if (n == 0) return fail(TL_ERR_INVALID, "the loss of zero pixels is undefined");
    if ((rc = set_device_of(p))) return rc;
    if ((rc = cnn_grad_run(net, p, D, alpha_theta, alpha_phi, pix, n, target))) return rc;
    TL_HIP(hipMemcpyAsync(grad_out, net->grad.ptr, (kCnnTrain + 1) * sizeof(float), hipMemcpyDeviceToDevice,
                          p.stream),
           "copy");
    return TL_OK;
}

int tl_cnn_train_step(tl_cnn net, tl_plan plan, const float *D, const double *alpha_theta, const double *alpha_phi,
                      const int64_t *pix, int64_t n, const float *target, float lr, float *loss_out)
{
    int rc = cnn_check_plan(plan, net);
    if (rc) return rc;
    Plan &p = plan->p;
    if ((rc = cnn_check_pixels(p, D, alpha_theta, alpha_phi, pix, n))) return rc;
    if (!target) return fail(TL_ERR_INVALID, "target is NULL");
    if (n == 0) return fail(TL_ERR_INVALID, "the loss of zero pixels is undefined");
    if (!(lr > 0.f) || !std::isfinite(lr)) return fail(TL_ERR_INVALID, "lr must be positive");
    if ((rc = set_device_of(p))) return rc;
    if ((rc = cnn_grad_run(net, p, D, alpha_theta, alpha_phi, pix, n, target))) return rc;
    if (loss_out)
        TL_HIP(hipMemcpyAsync(loss_out, (float *)net->grad.ptr + kCnnTrain, sizeof(float), hipMemcpyDeviceToDevice,
                              p.stream),
               "copy");
    net->step += 1;
    TL_HIP(cnn_adam(net->c, net->step, lr, p.stream), "cnn adam");
    return TL_OK;
}

int tl_lens_map_cnn(tl_plan plan, tl_cnn net, const void *alm_T, const void *alm_E, const void *alm_B,
                    const void *alm_phi, void *T_out, void *Q_out, void *U_out)
{
    int rc = cnn_check_plan(plan, net);
    if (rc) return rc;
    Plan &p = plan->p;
    if ((rc = check_fields(p, alm_T, alm_E))) return rc;
    if ((rc = check_outputs(p, T_out, Q_out, U_out))) return rc;
    if ((rc = set_device_of(p))) return rc;
    if ((rc = cnn_reserve(net, net->corr, 3 * p.npix() * sizeof(float), p.stream))) return rc;
    if ((rc = run_deflection(p, alm_phi))) return rc;
    if ((rc = run_derivs(p, alm_T, alm_E, alm_B, p.D.ptr))) return rc;
    const double *at = (const double *)p.alpha.ptr;
    {
        StageScope sc(p, ST_CNN);
        TL_HIP(cnn_forward(p, net->c, (const float *)p.D.ptr, at, at + p.npix(), nullptr, (int64_t)p.npix(),
                           (float *)net->corr.ptr, false, p.stream),
               "cnn forward");
    }
    StageScope sc(p, ST_REMAP);
    TL_HIP(launch_remap(p, p.D.ptr, at, at + p.npix(), nullptr, nullptr, T_out, Q_out, U_out,
                        (const float *)net->corr.ptr),
           "remap");
    return TL_OK;
}

int tl_lens_map_simple(const void *alm_T, const void *alm_E, const void *alm_B, const void *alm_phi, int32_t lmax,
                       int32_t order, tl_grid grid, void *T_out, void *Q_out, void *U_out)
{
    tl_options o{};
    o.order = order;
    o.precision = TL_FP32;
    o.pol = alm_E != nullptr;
    o.rotate = 1;
    tl_plan plan = nullptr;
    int rc = tl_plan_create(&plan, lmax, grid, &o, nullptr);
    if (rc) return rc;
    rc = tl_lens_map(plan, alm_T, alm_E, alm_B, alm_phi, T_out, Q_out, U_out);
    if (rc == TL_OK) {
        hipError_t e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) rc = hipfail(e, "synchronize");
    }
    tl_plan_destroy(plan);
    return rc;
}

int tl_lens_map_simple_noalloc(const void *alm_T, const void *alm_E, const void *alm_B, const void *alm_phi,
                               int32_t lmax, int32_t order, tl_grid grid, void *T_out, void *Q_out, void *U_out)
{
    tl_options o{};
    o.order = order;
    o.precision = TL_FP32;
    o.pol = alm_E != nullptr;
    o.rotate = 1;
    int rc = validate_options(lmax, grid, &o);
    if (rc) return rc;
    Plan p;
    plan_fields(p, lmax, grid, &o, nullptr);
    if ((rc = check_fields(p, alm_T, alm_E))) return rc;
    if ((rc = check_outputs(p, T_out, Q_out, U_out))) return rc;
    // the plan's buffers, each 256-byte aligned, carved from the array
    const Sizes sz = plan_sizes(p);
    std::vector<BufItem> items = plan_buffer_list(p, sz);
    size_t need = 0;
    for (auto &it : items)
        if (it.n) need += (it.n + 255) & ~(size_t)255;
    if (need > kScratchBytes)
        return fail(TL_ERR_NOMEM, "tl_lens_map_simple_noalloc: this lmax, grid and order need " +
                                      std::to_string(need) + " bytes of workspace, above its static " +
                                      std::to_string(kScratchBytes) + "-byte array");
    if ((rc = plan_device_checks(p))) return rc;
    void *base = nullptr;
    if ((rc = scratch_address(p.device, &base))) return rc;
    size_t off = 0;
    for (auto &it : items) {
        if (!it.n) continue;
        it.b->ptr = (char *)base + off;
        it.b->bytes = it.n;
        off += (it.n + 255) & ~(size_t)255;
    }
    p.total_bytes = off;
    // tables and start values into the array, then the path; everything on
    // the null stream, which is synchronized before returning
    if ((rc = plan_setup(p))) return rc;
    rc = lens_map_core(p, alm_T, alm_E, alm_B, alm_phi, T_out, Q_out, U_out);
    if (rc == TL_OK) {
        const hipError_t e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) rc = hipfail(e, "synchronize");
    }
    return rc;
}

}  // extern "C"
