// Displaced position, nearest grid pixel and polarization rotation of one
// output pixel (Sec. II.A/II.B): shared by the remap and the learned
// correction so both see the same (i0, k0, u, v).
#pragma once

#include <hip/hip_runtime.h>

namespace tl {

struct PixLoc {
    int i0, k0, kh;      // nearest ring, pixel (k0 = kh mod nphi)
    double thp, php;     // displaced position
    double cg, sg;       // cos 2 gamma, sin 2 gamma of the rotation
};

// Grid tables: theta[ntheta], trig[ring] = {cos, sin} (north rings; the
// caller passes the ring's own values), phitrig[k] = {cos, sin} phi_k,
// phival[nphi + 1] = phi_k.  at, ap = alpha components at the pixel.  With
// thsrc the position is given (no rotation).  want_rot: compute cg, sg.
__device__ __forceinline__ PixLoc locate_pixel(int i, int k, int ntheta, int nphi, const double *__restrict__ theta,
                                               const double2 *__restrict__ trig,
                                               const double2 *__restrict__ phitrig,
                                               const double *__restrict__ phival, double a_t, double a_p,
                                               const double *thsrc, const double *phsrc, size_t idx, bool naive,
                                               bool want_rot)
{
    const double TWO_PI = 6.283185307179586476925286766559;
    const double dth_grid = M_PI / (double)(ntheta - 1);
    const double dph_grid = TWO_PI / (double)nphi;
    PixLoc L;
    L.cg = 1.0;
    L.sg = 0.0;
    double thp, php;
    if (thsrc) {
        thp = thsrc[idx];
        php = phsrc[idx];
        php = php - floor(php / TWO_PI) * TWO_PI;
    } else {
        const double d = sqrt(a_t * a_t + a_p * a_p);
        const bool pole = (i == 0) || (i == ntheta - 1);
        if (d == 0.0) {
            thp = theta[i];
            php = phival[k];
        } else if (naive && !pole) {
            const double st = trig[i].y;
            thp = theta[i] + a_t;
            php = phival[k] + a_p / st;
            if (thp < 0.0) {
                thp = -thp;
                php += M_PI;
            }
            if (thp > M_PI) {
                thp = TWO_PI - thp;
                php += M_PI;
            }
            php = php - floor(php / TWO_PI) * TWO_PI;
        } else {
            const double ct = trig[i].x, st = trig[i].y;
            const double cp = phitrig[k].x, sp = phitrig[k].y;
            const double x0 = st * cp, x1 = st * sp, x2 = ct;
            const double et0 = ct * cp, et1 = ct * sp, et2 = -st;
            const double ep0 = -sp, ep1 = cp;
            const double id = 1.0 / d;
            const double u0 = (a_t * et0 + a_p * ep0) * id;
            const double u1 = (a_t * et1 + a_p * ep1) * id;
            const double u2 = (a_t * et2) * id;
            double sd, cd;
            sincos(d, &sd, &cd);
            const double y0 = cd * x0 + sd * u0, y1 = cd * x1 + sd * u1, y2 = cd * x2 + sd * u2;
            const double rho = sqrt(y0 * y0 + y1 * y1);
            thp = atan2(rho, y2);
            php = atan2(y1, y0);
            if (php < 0.0) php += TWO_PI;
            if (want_rot && !naive) {
                // tangent of the geodesic at x'
                const double t0 = -sd * x0 + cd * u0, t1 = -sd * x1 + cd * u1, t2 = -sd * x2 + cd * u2;
                double cpp = 1.0, spp = 0.0;
                if (rho > 0.0) {
                    const double ir = 1.0 / rho;
                    cpp = y0 * ir;
                    spp = y1 * ir;
                }
                const double ctp = y2, stp = rho;
                const double tt = t0 * ctp * cpp + t1 * ctp * spp - t2 * stp;  // t . e_theta(x')
                const double tp = -t0 * spp + t1 * cpp;                       // t . e_phi(x')
                // e^{i gamma} = (a_t + i a_p)(tt - i tp) / (d |t|)
                const double gr = a_t * tt + a_p * tp;
                const double gi = a_p * tt - a_t * tp;
                const double inrm = 1.0 / (gr * gr + gi * gi);
                L.cg = (gr * gr - gi * gi) * inrm;
                L.sg = 2.0 * gr * gi * inrm;
            }
        }
    }
    // nearest pixel (round half up), residuals against the grid tables
    int i0 = (int)floor(thp / dth_grid + 0.5);
    i0 = i0 < 0 ? 0 : (i0 > ntheta - 1 ? ntheta - 1 : i0);
    int kh = (int)floor(php / dph_grid + 0.5);
    kh = kh < 0 ? 0 : (kh > nphi ? nphi : kh);
    L.i0 = i0;
    L.kh = kh;
    L.k0 = kh == nphi ? 0 : kh;
    L.thp = thp;
    L.php = php;
    return L;
}

}  // namespace tl
