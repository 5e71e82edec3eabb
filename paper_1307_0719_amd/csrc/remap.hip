// Remap + Taylor sum + polarization rotation (Sec. II.B, eqs. 2, 4, 5).
//
// One lane per output pixel x = (theta_i, phi_k), lanes of a wave along phi:
//  1. displaced position x' from alpha by the geodesic of length |alpha| in the
//     direction (a_t e_theta + a_p e_phi)/|alpha| (parallel transport, Sec. II.A),
//     or by coordinate addition (naive rule), or given by the caller;
//  2. nearest grid point (i0, k0) by rounding half up in theta and phi, with
//     scaled residuals u = (theta' - theta_i0)/dtheta, v = (phi' - phi_k0)/dphi;
//  3. s' = sum_{j+k<=N} u^j v^k Dt_{jk}(i0, k0) for s in {T, Q, U}, Horner in v then
//     u, where Dt are the derivative maps pre-scaled by dtheta^j dphi^k/(j!k!);
//  4. Q' + iU' = e^{2 i gamma} (Q + iU), gamma the angle between the transported
//     e_theta(x') and e_theta(x): e^{i gamma} = e^{i psi} e^{-i psi'} with psi the
//     bearing of alpha at x and psi' the bearing of the geodesic's tangent at x'.
// Positions, residuals and the rotation angle are FP64; the sum uses R (FP32 or
// FP64).  Neighbouring lanes gather neighbouring source pixels, so the gathers
// from each derivative map are mostly coalesced.
#include <hip/hip_fp16.h>

#include "geom.h"
#include "tl_internal.h"

namespace tl {

namespace {

template <typename R, int N, bool POL, bool MIX, bool PAIRED>
__global__ __launch_bounds__(256) void k_remap(int ntheta, int nphi, const double *__restrict__ theta,
                                               const double2 *__restrict__ trig, const double2 *__restrict__ phitrig,
                                               const double *__restrict__ phival, const R *__restrict__ D,
                                               const __half *__restrict__ D16, size_t ds, size_t ds16,
                                               const double *__restrict__ at, const double *__restrict__ ap,
                                               const double *__restrict__ thsrc, const double *__restrict__ phsrc,
                                               int rotate, int naive, const float *__restrict__ corr,
                                               R *__restrict__ To, R *__restrict__ Qo, R *__restrict__ Uo)
{
    const int i = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nphi) return;
    const size_t idx = (size_t)i * nphi + k;
    const double TWO_PI = 6.283185307179586476925286766559;

    const PixLoc L = locate_pixel(i, k, ntheta, nphi, theta, trig, phitrig, phival, thsrc ? 0.0 : at[idx],
                                  thsrc ? 0.0 : ap[idx], thsrc, phsrc, idx, naive != 0, POL && rotate);
    const double cg = L.cg, sg = L.sg;
    const int i0 = L.i0, k0 = L.k0;
    const R u = (R)((L.thp - theta[i0]) * ((double)(ntheta - 1) / M_PI));
    const R v = (R)((L.php - phival[L.kh]) * ((double)nphi / TWO_PI));

    const size_t plane = (size_t)ntheta * nphi;
    const size_t pix0 = (size_t)i0 * nphi + k0;
    R res[POL ? 3 : 1];
#pragma unroll
    for (int f = 0; f < (POL ? 3 : 1); ++f) {
        // Horner in v then u over the maps at pix0: the plain layout
        // [field][ND][ds], or (MIX) FP32 maps of j + k < kMix16 then FP16 maps
        constexpr int ND = (N + 1) * (N + 2) / 2;
        const R *Df = D + (size_t)f * (MIX ? mix_n32() : ND) * ds + pix0;
        const __half *Hf = D16 + (MIX ? (size_t)f * (ND - mix_n32()) * ds16 + pix0 : 0);
        R acc = 0;
#pragma unroll
        for (int j = N; j >= 0; --j) {
            const int base = j * (N + 1) - j * (j - 1) / 2;  // index of (j, 0)
            R inner = 0;
            float2 pr = make_float2(0.f, 0.f);  // a paired plane's two values, read at its second map
#pragma unroll
            for (int kk = N - j; kk >= 0; --kk) {
                R d;
                const bool h = MIX && j + kk >= kMix16;
                const int pos = PAIRED ? pair_pos(N, MIX, j, kk) : 0;
                const size_t slot = h ? (size_t)mix_idx16(N, j, kk) : (size_t)(MIX ? mix_idx32(j, kk) : base + kk);
                if (pos == 2) {
                    // the plane of slot - 1 holds (D_{j,kk-1}, D_{j,kk}) at 2 pix0
                    if (h) pr = __half22float2(*reinterpret_cast<const __half2 *>(Hf + (slot - 1) * ds16 + pix0));
                    else pr = *reinterpret_cast<const float2 *>(Df + (slot - 1) * ds + pix0);
                    d = (R)pr.y;
                } else if (pos == 1) {
                    d = (R)pr.x;
                } else if (h) {
                    d = (R)__half2float(Hf[slot * ds16]);
                } else {
                    d = Df[slot * ds];
                }
                inner = inner * v + d;
            }
            acc = acc * u + inner;
        }
        res[f] = acc;
    }
    if (corr) {  // learned remainder of the order-N sum, added before the rotation
#pragma unroll
        for (int f = 0; f < (POL ? 3 : 1); ++f) res[f] += (R)corr[(size_t)f * plane + idx];
    }
    To[idx] = res[0];
    if constexpr (POL) {
        const R q = res[1], uu = res[2];
        Qo[idx] = (R)(cg * (double)q - sg * (double)uu);
        Uo[idx] = (R)(sg * (double)q + cg * (double)uu);
    }
}

// HEALPix output and source pixels (RING order; the paper's own grid, Sec.
// II.B): output pixel n of ring r at (theta_r, phi0_r + 2 pi n / nphi_r), its
// displaced position x', the pixel containing x' and that pixel's centre x0';
// the Taylor series about x0' in u = (theta' - theta0') / delta,
// v = (phi' - phi0') / delta (wrapped to (-pi, pi]), delta = pi / (4 nside),
// the scale of the derivative maps; then the rotation R.
template <typename R, int N, bool POL, bool MIX>
__global__ __launch_bounds__(256) void k_remap_hpx(int nside, const double *__restrict__ theta,
                                                   const double2 *__restrict__ trig, const HRing *__restrict__ hring,
                                                   size_t npix, const R *__restrict__ D,
                                                   const __half *__restrict__ D16, size_t ds, size_t ds16,
                                                   const double *__restrict__ at,
                                                   const double *__restrict__ ap, const double *__restrict__ thsrc,
                                                   const double *__restrict__ phsrc, int rotate, int naive,
                                                   R *__restrict__ To, R *__restrict__ Qo, R *__restrict__ Uo)
{
    const double TWO_PI = 6.283185307179586476925286766559;
    const int r = blockIdx.y;
    const HRing hr = hring[r];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= hr.nphi) return;
    const size_t idx = (size_t)hr.start + k;
    double thp, php, cg = 1.0, sg = 0.0;
    if (thsrc) {
        thp = thsrc[idx];
        php = phsrc[idx];
        php = php - floor(php / TWO_PI) * TWO_PI;
        thp = thp < 0.0 ? 0.0 : (thp > M_PI ? M_PI : thp);
    } else {
        const double ph = hr.phi0 + TWO_PI * (double)k / (double)hr.nphi;
        double sp, cp;
        sincos(ph, &sp, &cp);
        displace(theta[r], ph, trig[r].x, trig[r].y, cp, sp, at[idx], ap[idx], naive != 0, false,
                 POL && rotate, thp, php, cg, sg);
    }
    int r0, k0;
    healpix_locate(nside, thp, php, r0, k0);
    const HRing h0 = hring[r0];
    const double ph0 = h0.phi0 + TWO_PI * (double)k0 / (double)h0.nphi;
    double dph = php - ph0;
    dph -= TWO_PI * floor(dph / TWO_PI + 0.5);
    const double idel = 4.0 * nside / M_PI;
    const R u = (R)((thp - theta[r0]) * idel);
    const R v = (R)(dph * idel);
    const size_t pix0 = (size_t)h0.start + k0;
    R res[POL ? 3 : 1];
#pragma unroll
    for (int f = 0; f < (POL ? 3 : 1); ++f) {
        // Horner in v then u over the maps at pix0: the plain layout
        // [field][ND][ds], or (MIX) FP32 maps of j + k < kMix16 then FP16 maps
        constexpr int ND = (N + 1) * (N + 2) / 2;
        const R *Df = D + (size_t)f * (MIX ? mix_n32() : ND) * ds + pix0;
        const __half *Hf = D16 + (MIX ? (size_t)f * (ND - mix_n32()) * ds16 + pix0 : 0);
        R acc = 0;
#pragma unroll
        for (int j = N; j >= 0; --j) {
            const int base = j * (N + 1) - j * (j - 1) / 2;  // index of (j, 0)
            R inner = 0;
#pragma unroll
            for (int kk = N - j; kk >= 0; --kk) {
                R d;
                if (MIX && j + kk >= kMix16) d = (R)__half2float(Hf[(size_t)mix_idx16(N, j, kk) * ds16]);
                else d = Df[(size_t)(MIX ? mix_idx32(j, kk) : base + kk) * ds];
                inner = inner * v + d;
            }
            acc = acc * u + inner;
        }
        res[f] = acc;
    }
    To[idx] = res[0];
    if constexpr (POL) {
        const R q = res[1], uu = res[2];
        Qo[idx] = (R)(cg * (double)q - sg * (double)uu);
        Uo[idx] = (R)(sg * (double)q + cg * (double)uu);
    }
}

template <typename R, int N, bool MIX>
hipError_t remap_NM(Plan &p, const void *D, const double *at, const double *ap, const double *ths,
                    const double *phs, const float *corr, void *T, void *Q, void *U, hipStream_t st)
{
    dim3 grid((p.nphi + 255) / 256, p.ntheta);
    const __half *D16 = MIX ? (const __half *)p.d16_of(D) : nullptr;
    // the plan's own maps have padded planes; a caller's are [field][map][pixel]
    const bool own = p.own(D);
    const size_t ds = own ? p.dstride : p.npix(), ds16 = p.dstride16;
    if (p.nside) {
        if (corr) return hipErrorInvalidValue;
        if (p.pol)
            hipLaunchKernelGGL((k_remap_hpx<R, N, true, MIX>), grid, dim3(256), 0, st, p.nside,
                               (const double *)p.theta.ptr, (const double2 *)p.trig.ptr, (const HRing *)p.hring.ptr,
                               p.npix(), (const R *)D, D16, ds, ds16, at, ap, ths, phs, p.rotate, p.naive, (R *)T, (R *)Q,
                               (R *)U);
        else
            hipLaunchKernelGGL((k_remap_hpx<R, N, false, MIX>), grid, dim3(256), 0, st, p.nside,
                               (const double *)p.theta.ptr, (const double2 *)p.trig.ptr, (const HRing *)p.hring.ptr,
                               p.npix(), (const R *)D, D16, ds, ds16, at, ap, ths, phs, p.rotate, p.naive, (R *)T, (R *)Q,
                               (R *)U);
        return hipGetLastError();
    }
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, dim3(256), 0, st, p.ntheta, p.nphi, (const double *)p.theta.ptr,
                           (const double2 *)p.trig.ptr, (const double2 *)p.phitab.ptr, (const double *)p.phival.ptr,
                           (const R *)D, D16, ds, ds16, at, ap, ths, phs, p.rotate, p.naive, corr, (R *)T, (R *)Q,
                           (R *)U);
        return hipGetLastError();
    };
    if constexpr (sizeof(R) == 4) {
        if (own && p.paired)
            return p.pol ? launch(k_remap<R, N, true, MIX, true>) : launch(k_remap<R, N, false, MIX, true>);
    }
    return p.pol ? launch(k_remap<R, N, true, MIX, false>) : launch(k_remap<R, N, false, MIX, false>);
}

// The plan's own maps are mixed precision when mix16 (orders >= 3 of the
// FP32 forms); maps elsewhere are plain.
template <typename R, int N>
hipError_t remap_N(Plan &p, const void *D, const double *at, const double *ap, const double *ths,
                   const double *phs, const float *corr, void *T, void *Q, void *U, hipStream_t st)
{
    if constexpr (N >= kMix16 && sizeof(R) == 4) {
        if (p.mix16 && p.own(D)) return remap_NM<R, N, true>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
    }
    return remap_NM<R, N, false>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
}

template <typename R>
hipError_t remap_R(Plan &p, const void *D, const double *at, const double *ap, const double *ths,
                   const double *phs, const float *corr, void *T, void *Q, void *U, hipStream_t st)
{
    switch (p.order) {
    case 0: return remap_N<R, 0>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
    case 1: return remap_N<R, 1>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
    case 2: return remap_N<R, 2>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
    case 3: return remap_N<R, 3>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
    case 4: return remap_N<R, 4>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
    case 5: return remap_N<R, 5>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
    case 6: return remap_N<R, 6>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
    case 7: return remap_N<R, 7>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
    case 8: return remap_N<R, 8>(p, D, at, ap, ths, phs, corr, T, Q, U, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_remap(Plan &p, const void *D, const double *at, const double *ap, const double *thsrc,
                        const double *phsrc, void *T, void *Q, void *U, const float *corr, hipStream_t st)
{
    if (!st) st = p.stream;
    if (p.fp64()) return remap_R<double>(p, D, at, ap, thsrc, phsrc, corr, T, Q, U, st);
    return remap_R<float>(p, D, at, ap, thsrc, phsrc, corr, T, Q, U, st);
}

}  // namespace tl
