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

// Displaced position x' of the point (theta, phi) with cos/sin (ct, st) and
// (cp, sp) by the deflection (a_t, a_p) (Sec. II.A): the geodesic of length
// |alpha| in the direction (a_t e_theta + a_p e_phi) / |alpha|, or with naive
// the coordinate sum theta + a_t, phi + a_p / sin theta reflected over the
// poles (not on a pole ring: pole).  With want_rot also cos and sin of 2 gamma,
// gamma the angle between the transported e_theta(x') and e_theta(x).
__device__ __forceinline__ void displace(double th, double ph, double ct, double st, double cp, double sp,
                                         double a_t, double a_p, bool naive, bool pole, bool want_rot,
                                         double &thp, double &php, double &cg, double &sg)
{
    const double TWO_PI = 6.283185307179586476925286766559;
    cg = 1.0;
    sg = 0.0;
    const double d = sqrt(a_t * a_t + a_p * a_p);
    if (d == 0.0) {
        thp = th;
        php = ph;
    } else if (naive && !pole) {
        thp = th + a_t;
        php = ph + a_p / st;
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
            cg = (gr * gr - gi * gi) * inrm;
            sg = 2.0 * gr * gi * inrm;
        }
    }
}

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
        const bool pole = (i == 0) || (i == ntheta - 1);
        displace(theta[i], phival[k], trig[i].x, trig[i].y, phitrig[k].x, phitrig[k].y, a_t, a_p, naive, pole,
                 want_rot, thp, php, L.cg, L.sg);
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

// HEALPix pixel containing the direction (thp, php in [0, 2 pi)), RING
// order: ring (0-based, 0 .. 4 nside - 2) and index in the ring.  The belt
// (|z| <= 2/3) is cut by the two families of pixel edge lines
// nside (1/2 + tt) -+ (3/4) nside z, tt = phi / (pi/2); the caps by the same
// lines in nside sqrt(3 (1 - |z|)) = nside sin theta sqrt(3 / (1 + |z|))
// (the published HEALPix construction).
__device__ __forceinline__ void healpix_locate(int nside, double thp, double php, int &ring, int &kin)
{
    double sn, z;
    sincos(thp, &sn, &z);
    const double za = fabs(z);
    double tt = php * 0.63661977236758134307553505349006;  // 2 / pi
    if (tt >= 4.0) tt -= 4.0;
    if (tt < 0.0) tt += 4.0;
    if (za <= 2.0 / 3.0) {
        const double t1 = nside * (0.5 + tt), t2 = nside * z * 0.75;
        const int jp = (int)floor(t1 - t2), jm = (int)floor(t1 + t2);
        const int ir = nside + 1 + jp - jm;  // 1 .. 2 nside + 1 from ring nside
        const int kshift = 1 - (ir & 1);
        const int num = jp + jm - nside + kshift + 1;
        int ip = num >= 0 ? num / 2 : -((1 - num) / 2);  // floor division
        const int n4 = 4 * nside;
        ip %= n4;
        if (ip < 0) ip += n4;
        ring = ir + nside - 2;
        kin = ip;
    } else {
        const double tp = tt - floor(tt);
        const double tmp = nside * sn * sqrt(3.0 / (1.0 + za));
        const int jp = (int)floor(tp * tmp), jm = (int)floor((1.0 - tp) * tmp);
        const int ir = jp + jm + 1;  // from the nearer pole
        int ip = (int)floor(tt * ir);
        if (ip >= 4 * ir) ip -= 4 * ir;
        ring = z > 0.0 ? ir - 1 : 4 * nside - 1 - ir;
        kin = ip;
    }
}

}  // namespace tl
