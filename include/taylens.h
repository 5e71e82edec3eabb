/*
 * taylens.h -- C ABI of the MI355X (gfx950) full-sky Taylor-lensing library.
 *
 * The library lenses band-limited CMB fields given as spherical-harmonic
 * coefficients: T'(x) = T(x + alpha), P'(x) = R P(x + alpha) with
 * alpha = grad phi (eqs. 1-2 of Naess & Louis 2013, "Lensing simulations by
 * Taylor expansion -- not so inefficient after all").  The value at the
 * displaced point is the Taylor series about the nearest pixel centre,
 * truncated at order N (eq. 4; per component eq. 5, Sec. II.B), so the
 * expansion variable is the sub-pixel residual, not the full deflection.
 *
 * Pixelization: equal-theta (Clenshaw-Curtis) ring grid with both poles,
 *     theta_i = pi * i / (ntheta - 1),  i = 0..ntheta-1   (ring 0 = north pole)
 *     phi_k   = 2 pi * k / nphi,        k = 0..nphi-1
 * Maps are row-major [ntheta][nphi].  Q/U are components in the local
 * (e_theta, e_phi) basis of each pixel (Q = P_tt, U = P_tp).
 *
 * Harmonic coefficients: complex128 (interleaved re, im), triangular
 * m-major layout, a_lm at index m*(2*lmax+1-m)/2 + l for 0 <= m <= l <= lmax;
 * negative m follow from a_{l,-m} = (-1)^m conj(a_lm) (real fields).  The
 * imaginary part of m = 0 entries is ignored.  Orthonormal Y_lm with the
 * Condon-Shortley phase; spin-2 harmonics sY_lm = sqrt((l-2)!/(l+2)!) eth^2 Y_lm,
 * with Q + iU = sum -(E_lm + i B_lm) 2Y_lm; E/B entries with l < 2 are ignored.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller.  A
 * plan owns only its workspace (allocated at tl_plan_create, released by
 * tl_plan_destroy).  All work is queued on the plan's HIP stream; no call
 * synchronizes the stream except tl_plan_create (which builds its tables).
 * Tabulated plans with opt.batch > 1 also own a second stream (default
 * priority) that runs part of a call's work; it is ordered after the plan's
 * stream by events, and the plan's stream waits for it before the call
 * returns, so the caller still orders everything through the plan's stream.
 * A plan is not thread-safe: use one plan per host thread / stream.
 *
 * Errors: every function returns TL_OK (0) or a negative code; arguments are
 * validated on the host before any HIP call, so invalid arguments never
 * launch work.  tl_last_error() gives a thread-local message for the last
 * failure on the calling thread.  The library never aborts or exits.
 */
#ifndef TAYLENS_H
#define TAYLENS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TL_OK 0
#define TL_ERR_INVALID (-1)     /* bad argument (null plan/pointer, sizes)       */
#define TL_ERR_UNSUPPORTED (-2) /* valid request this build does not provide     */
#define TL_ERR_HIP (-3)         /* a HIP runtime call failed (see tl_last_error)  */
#define TL_ERR_NOMEM (-4)       /* allocation failed or workspace_cap exceeded   */

#define TL_MAX_ORDER 8 /* largest Taylor order N */

/* Contraction precision of the harmonic (Legendre) stage.  The recursion of
 * the Legendre functions is always FP64, and so are the positions, the
 * rotation angle and the polar caps (sin theta < 0.15; < 0.05 for
 * TL_FP16X2).
 *   TL_FP64   FP64 throughout; maps are float64.
 *   TL_FP32   FP32 matrix-core contraction (L-power form), FP32 derivative maps
 *             and Taylor sum; float32 maps.
 *   TL_BF16X3, TL_FP16X2, TL_FP16, TL_BF16: the lambda / lambda' values are
 *             tabulated at plan creation (rounded to BF16 / FP16; the X3 / X2
 *             forms keep hi + lo parts and take hi*hi + hi*lo + lo*hi on the
 *             matrix cores), each call streams the table (up to opt.batch
 *             realizations per pass, tl_lens_map_many); float32 maps.
 *             Orders 0..6.  Tables: about 4 * nrp * lmax^2 bytes (x2 split).
 *             With the environment variable TAYLENS_ONTHEFLY=1 at plan
 *             creation the same forms run without tables: the FP64 recursion
 *             feeds the 16-bit matrix products directly (up to 4 realizations
 *             per pass at order 4 with T+E); results agree with the tabulated
 *             engine to rounding. */
enum {
    TL_FP64 = 0,
    TL_FP32 = 1,
    TL_BF16X3 = 2,
    TL_FP16X2 = 3,
    TL_FP16 = 4,
    TL_BF16 = 5
};

typedef struct {
    int32_t ntheta; /* rings, >= 2                        */
    int32_t nphi;   /* pixels per ring, even, >= 2*lmax, and nphi/2 a product of 2, 3, 5 */
} tl_grid;

typedef struct {
    int32_t order;         /* Taylor order N, 0..TL_MAX_ORDER (0 = nearest pixel)    */
    int32_t precision;     /* TL_FP64 / TL_FP32 / ...                                */
    int32_t pol;           /* 1: T and Q/U; 0: T only                                 */
    int32_t rotate;        /* 1: apply the parallel-transport rotation R to Q/U       */
    int32_t naive_pos;     /* 1: theta' = theta + a_t, phi' = phi + a_p / sin theta
                              (reflected over the poles; pole rings stay geodesic;
                              no rotation).  0: geodesic displacement.             */
    int32_t batch;         /* realizations per harmonic-stage pass for the tabulated
                              forms (tl_lens_map_many): 0 or 1 = one; at most 6
                              with tables (up to 128 right-hand-side columns: 6
                              at order 4 with T + E, fewer with B or at high
                              orders; error if too many), 4 on the fly.  Must be
                              0 or 1 for TL_FP64 / TL_FP32.                        */
    int64_t workspace_cap; /* bytes; 0 = no cap.  tl_plan_create fails with
                              TL_ERR_NOMEM if the plan would need more.            */
    int32_t maps16;        /* 1: the plan's internal derivative maps D_jk with
                              j + k >= 3 are FP16 (orders >= 3 of the non-FP64
                              forms on the equal-theta grid; ignored elsewhere):
                              30 % less map traffic at order 4.  The remap
                              multiplies them by |u|^j |v|^k <= 1/8 in pixel
                              units, so their rounding costs about 1e-6 of the
                              map RMS for skies whose power falls off well
                              before the band limit (the lensed CMB at lmax
                              4096), but up to ~1e-4 for power at the grid's
                              band limit.  0: FP32 maps.  tl_synth_derivs
                              always returns FP32 maps.                          */
    int32_t lmax_phi;      /* band limit of the lensing potential (Sec. II.A: the
                              deflection is synthesized to its own, higher band
                              limit than the fields): 0 = lmax; otherwise
                              lmax <= lmax_phi <= 16384 and nphi >= 2 lmax_phi,
                              equal-theta plans only (TL_ERR_UNSUPPORTED for
                              HEALPix rings unless 0 or lmax).  alm_phi then holds
                              (lmax_phi + 1)(lmax_phi + 2)/2 coefficients; the
                              deflection takes the direct FP64 recursion on
                              every ring (not the tables of the tabulated forms). */
    int32_t theta_fft;     /* 1: TL_FP64 plans synthesize only the rows j = 0 in the
                              harmonic stage (the ring FFTs give D_0k) and take the
                              theta-derivatives D_jk, j >= 1, by FFT along the great
                              circles through both poles (tl_theta_derivs; the FFT
                              route of Sec. IV), for tl_lens_map, tl_lens_map_many,
                              tl_lens_map_pos and tl_synth_derivs (tl_legendre still
                              returns every row).  Needs the equal-theta grid with
                              ntheta - 1 a power of two in [2, 4096] and
                              lmax <= ntheta - 2, and TL_FP64 (TL_ERR_UNSUPPORTED
                              otherwise); results equal the recursion's to FP64
                              rounding.  0: every row by the recursion.            */
} tl_options;

typedef struct tl_plan_s *tl_plan;

/* Create a plan for band limit lmax (>= 0) on the given grid.  hip_stream is a
 * hipStream_t (NULL = default stream).  Builds the recursion-coefficient and
 * start-value tables on the device and waits for them.  On failure *plan is
 * set to NULL. */
int tl_plan_create(tl_plan *plan, int32_t lmax, tl_grid grid, const tl_options *opt,
                   void *hip_stream);

/* Plan on HEALPix rings (RING order, npix = 12 nside^2; the pixelization of
 * the paper's simulations, Sec. II.A-B) instead of the equal-theta grid:
 * output pixels are the HEALPix centres, the derivative maps live on them, and
 * the remap expands about the centre of the pixel that CONTAINS the displaced
 * position (the paper's ang2pix / pix2ang step, Sec. II.B), in the offsets
 * (theta' - theta0, phi' - phi0) of eq. 5.  Ring syntheses fold the band
 * limit onto each ring's own pixel count and phase, so lmax is free.  Maps
 * (outputs of tl_lens_map, tl_lens_map_many; alpha of tl_deflection) are
 * [npix] in RING order; derivative maps (tl_synth_derivs, tl_remap) are
 * [field][jk][npix] scaled by delta^(j+k) / (j! k!), delta = pi / (4 nside);
 * positions for tl_lens_map_pos are [npix].  1 <= nside <= 2048.  Batches
 * (tl_batch_*), tl_lens_map_batch of mixed grids aside, and the correction
 * network take equal-theta plans only (TL_ERR_UNSUPPORTED). */
int tl_plan_create_healpix(tl_plan *plan, int32_t lmax, int32_t nside, const tl_options *opt,
                           void *hip_stream);

/* Release a plan and its workspace (NULL is accepted).  Waits for the plan's
 * stream first. */
int tl_plan_destroy(tl_plan plan);

/* Device bytes held by the plan. */
int tl_plan_workspace_bytes(tl_plan plan, int64_t *bytes);

/* Work counts of a plan, fixed at creation (for throughput accounting):
 *   TL_Q_RPOLE       ring pairs near the poles kept on the direct FP64 kernels
 *                    in the FP32 and tabulated forms
 *   TL_Q_ELEMS       (l, m, ring pair) elements of the harmonic stage at or
 *                    below the evanescent cut (all ring pairs)
 *   TL_Q_ELEMS_CAPS  the same, restricted to the pole-adjacent ring pairs
 *   TL_Q_TAB_CHUNKS  (m, 32-ring tile, 32-l chunk) table blocks the table
 *                    GEMM streams per pass (tabulated forms; 0 otherwise)
 *   TL_Q_TAB_CHUNK_BYTES  bytes of one such block (both tables, hi and lo)
 *   TL_Q_DEFL_FOLDED 1 when the table GEMM also carries the lensing
 *                    potential (tl_lens_map / tl_lens_map_many with alm_phi
 *                    given: the deflection's harmonic sums outside the caps
 *                    come from the same pass, the caps from the direct FP64
 *                    kernel), else 0
 * Returns TL_ERR_INVALID for an unknown key or a NULL value pointer. */
#define TL_Q_RPOLE 0
#define TL_Q_ELEMS 1
#define TL_Q_ELEMS_CAPS 2
#define TL_Q_TAB_CHUNKS 3
#define TL_Q_TAB_CHUNK_BYTES 4
#define TL_Q_DEFL_FOLDED 5
int tl_plan_query(tl_plan plan, int32_t key, int64_t *value);

/* Lens one realization (the full method, eqs. 1, 2, 5):
 *   alm_T (required), alm_E (required iff opt.pol), alm_B (NULL = 0),
 *   alm_phi (NULL = no deflection: the unlensed maps).
 *   T_out, Q_out, U_out: [ntheta][nphi] float64 (TL_FP64) or float32
 *   (other precisions); Q_out/U_out are ignored when opt.pol = 0. */
int tl_lens_map(tl_plan plan, const void *alm_T, const void *alm_E, const void *alm_B,
                const void *alm_phi, void *T_out, void *Q_out, void *U_out);

/* Same remap + Taylor sum at caller-given source positions theta_src,
 * phi_src ([ntheta][nphi] float64, theta in [0, pi], any real phi): output
 * pixel x takes the order-N Taylor series of eq. 5 about the pixel centre
 * nearest to its source position, in the residual (theta' - theta_i0,
 * phi' - phi_k0) (Sec. II.B; the nearest-pixel rule of Sec. II.A/B).  No
 * rotation is applied (the positions do not define a transport path).
 * Outputs as in tl_lens_map; the call fails with TL_ERR_INVALID before any
 * launch if a position pointer is NULL.  Positions outside [0, pi] are
 * clamped to the first / last ring; phi is wrapped. */
int tl_lens_map_pos(tl_plan plan, const void *alm_T, const void *alm_E, const void *alm_B,
                    const double *theta_src, const double *phi_src, void *T_out, void *Q_out,
                    void *U_out);

/* ---- stage entry points (the same kernels tl_lens_map runs) ---- */

/* Deflection alpha = grad phi on the grid (Sec. II.A):
 * alpha_theta = d_theta phi, alpha_phi = d_phi phi / sin theta, with the
 * limits +- d_theta d_phi phi on the pole rings.  float64 [ntheta][nphi];
 * direct FP64 recursion and contraction in every precision form. */
int tl_deflection(tl_plan plan, const void *alm_phi, double *alpha_theta, double *alpha_phi);

/* Harmonic stage: per-ring Fourier coefficients of the theta-derivatives
 * that the Taylor series of eq. 5 needs (its d^j_theta factors; Sec. II.B
 * obtains the same derivatives by repeated transforms),
 * F[field][j][ring][m] complex (complex128 for TL_FP64, complex64 otherwise),
 * field in (T) or (T, Q, U), j = 0..order, m = 0..lmax:
 *   F^{(j)}_m(theta_i) = sum_l a_lm d^j/dtheta^j lambda_lm(theta_i)   (T)
 * and the Fourier coefficients of the real Q and U maps likewise
 * (sum over m of F_m e^{i m phi}, m < 0 by the real-field symmetry).
 * F_out: caller-owned device buffer of nfield*(order+1)*ntheta*(lmax+1)
 * complex entries.  NULL alm_T (or alm_E on a polarized plan) or F_out:
 * TL_ERR_INVALID. */
int tl_legendre(tl_plan plan, const void *alm_T, const void *alm_E, const void *alm_B,
                void *F_out);

/* Derivative maps, the coefficients of the Taylor series of eq. 5 at every
 * pixel centre (Sec. II.B: derivatives of T, Q, U up to the chosen order):
 * D[field][jk][ring][pix] (float64 / float32), jk running
 * over (j, k) with j + k <= order, j-major (j = 0: k = 0..N; j = 1: k = 0..N-1;
 * ...), each map SCALED by dtheta^j dphi^k / (j! k!) with dtheta = pi/(ntheta-1),
 * dphi = 2 pi/nphi:  D = dtheta^j dphi^k/(j!k!) d^j_theta d^k_phi s.
 * D_out: caller-owned device buffer of nfield*ndmap*ntheta*nphi values,
 * ndmap = (order+1)(order+2)/2.  NULL inputs: TL_ERR_INVALID. */
int tl_synth_derivs(tl_plan plan, const void *alm_T, const void *alm_E, const void *alm_B,
                    void *D_out);

/* Remap + Taylor sum + rotation from given scaled derivative maps (layout of
 * tl_synth_derivs) and deflection maps (layout of tl_deflection): the source
 * position x' of each pixel (geodesic displacement by alpha, Sec. II.A, or
 * the naive rule), its nearest pixel centre and the order-N sum of eq. 5 in
 * the residual (Sec. II.B), then Q' + iU' = e^{2i gamma}(Q + iU), the
 * parallel-transport rotation R of eq. 2.  All pointers are caller-owned
 * device buffers; NULL: TL_ERR_INVALID. */
int tl_remap(tl_plan plan, const void *D, const double *alpha_theta, const double *alpha_phi,
             void *T_out, void *Q_out, void *U_out);

/* Theta-derivatives by FFT instead of the harmonic recursion: the route that
 * the conclusion (Sec. IV) opens by moving to equal-theta (equirectangular)
 * pixels.  Meridian phi_c and its opposite phi_c + pi form one great circle
 * through both poles, sampled at P = 2 (ntheta - 1) equal steps of
 * dtheta = pi / (ntheta - 1); along it T, Q and U (components in the
 * (e_theta, e_phi) basis) of fields of band limit lmax are trigonometric
 * polynomials of degree <= lmax, so for lmax < P / 2 their theta-derivatives
 * follow exactly from the circle's DFT (theta runs against the circle on the
 * opposite meridian: odd orders change sign there).
 *   maps: nmaps maps [ntheta][nphi] in the plan's real type (float64 for
 *         TL_FP64, float32 otherwise), e.g. the j = 0 maps D_0k of
 *         tl_synth_derivs (any k: d_phi commutes with d_theta);
 *   out:  nmaps * jmax maps, out[i][j - 1] = dtheta^j / j! d^j_theta maps[i]
 *         for j = 1..jmax (the scaling of tl_synth_derivs, so that D_0k in
 *         gives D_jk out).
 * Arithmetic FP64 (the transform of each pair of circles in LDS).  Input
 * content above degree P / 2 - 1 along the circle aliases; the Nyquist
 * degree keeps its even derivatives only.  Requirements: an equal-theta
 * plan with ntheta - 1 a power of two, 2 <= ntheta - 1 <= 4096, and
 * lmax <= ntheta - 2 (TL_ERR_UNSUPPORTED otherwise); 1 <= jmax <= 8,
 * nmaps >= 0, maps and out caller-owned device buffers aligned to two
 * values (TL_ERR_INVALID otherwise) that must not overlap (not checked: the
 * result is then undefined).  Queued on the plan's stream. */
int tl_theta_derivs(tl_plan plan, const void *maps, int32_t nmaps, int32_t jmax, void *out);

/* Spherical-harmonic analysis of a temperature map on the plan's equal-theta
 * grid, the transform behind the power spectra that measure the accuracy of
 * the lensed maps (Sec. III.A-B):
 *   a_lm = sum_i w_i lambda_lm(theta_i) (2 pi / nphi) sum_k T(theta_i, phi_k) e^{-i m phi_k},
 * 0 <= m <= l <= the plan's lmax, w_i the Clenshaw-Curtis weights of the
 * rings (exact for polynomials in cos theta of degree <= ntheta - 1), so the
 * result is exact to FP64 rounding for maps of band limit L with
 * L + lmax <= ntheta - 1 and L + lmax < nphi.
 *   map:     float64 [ntheta][nphi] device array (any plan precision);
 *   alm_out: complex128 device array in the triangular layout of the plan's
 *            lmax, overwritten (the m = 0 entries carry the rounding of a
 *            zero imaginary part; the order of the atomic sums over ring
 *            blocks is not fixed, so repeated calls agree to rounding).
 * The plan's harmonic-stage buffer (ntheta (lmax + 1) complex128 values)
 * and deflection buffer serve as scratch: requires an equal-theta plan with nphi a power of two, 2 <= nphi
 * <= 8192, whose buffer is large enough (FP64 plans; order >= 1 or
 * polarized plans of the other forms) -- TL_ERR_UNSUPPORTED otherwise;
 * NULL or misaligned pointers: TL_ERR_INVALID.  Queued on the plan's
 * stream. */
int tl_analysis_T(tl_plan plan, const double *map, void *alm_out);

/* Lens n realizations (each as tl_lens_map: eqs. 1, 2, 5), plans[i] with
 * coefficient pointers alms[4i..4i+3] (T, E, B, phi) and outputs
 * outs[3i..3i+2] (T, Q, U).  Plans may differ in lmax and grid.  Queued on
 * plans[0]'s stream in one pass; that stream first waits for the work
 * already queued on every other plan's stream, and each of those streams
 * then waits for the pass, so workspace and outputs stay ordered. */
int tl_lens_map_batch(int32_t n, const tl_plan *plans, const void *const *alms,
                      void *const *outs);

/* Lens n realizations on ONE plan (all share lmax, grid, order, precision):
 * alms[4i..4i+3] = (T, E, B, phi), outs[3i..3i+2] = (T, Q, U).  For the
 * tabulated forms the harmonic stage runs opt.batch realizations per pass over
 * the lambda tables; the other stages run per realization, alternating
 * between two sets of the plan's maps so that one realization's remap (and a
 * pass's polar caps) run on the plan's second stream beside the next
 * realization's ring FFTs (and the pass's table epilogue).  Results are
 * those of n single tl_lens_map calls, bit for bit. */
int tl_lens_map_many(tl_plan plan, int32_t n, const void *const *alms, void *const *outs);

/* Convenience form with the signature
 *   lens_map(alm_T, alm_E, alm_B, alm_phi, lmax, order, grid) -> T', Q', U'
 * (FP32, geodesic positions, rotation on, T+Q/U iff alm_E != NULL): creates a
 * plan on the default stream, lenses, synchronizes and destroys the plan. */
int tl_lens_map_simple(const void *alm_T, const void *alm_E, const void *alm_B,
                       const void *alm_phi, int32_t lmax, int32_t order, tl_grid grid,
                       void *T_out, void *Q_out, void *U_out);

/* Allocation-free form of tl_lens_map_simple, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, kernels and results, but
 * the plan's workspace (tables, start values, harmonic output, derivative
 * and deflection maps) lives in a static device array of 128 MiB that the
 * library holds on every device it runs on until the process ends; no
 * hipMalloc, hipFree or allocating library call is made.  The array's
 * address is looked up once per device (with that device current).  The
 * call works on the current device and the null stream, which it
 * synchronizes before returning.  A size whose workspace exceeds 128 MiB
 * (T+Q/U order 4 fits up to lmax ~ 256 on 513 x 1024 rings) fails with
 * TL_ERR_NOMEM before any device work.  Every call on one device uses the
 * same array: calls that overlap on one device (several host threads) race
 * and must be serialized by the caller. */
int tl_lens_map_simple_noalloc(const void *alm_T, const void *alm_E, const void *alm_B,
                               const void *alm_phi, int32_t lmax, int32_t order, tl_grid grid,
                               void *T_out, void *Q_out, void *U_out);

/* ---- batches of realizations with uneven lmax ----
 *
 * A batch lenses n realizations, each with its own plan (plans may repeat:
 * realizations of equal lmax can share one), in one pass: the polar-cap
 * kernels of every realization, then ONE persistent launch of the
 * matrix-core harmonic kernel whose workgroups pop work items (realization,
 * block of ring pairs, run of m) from a queue ordered by decreasing cost
 * (longest processing time first), then per realization the deflection,
 * ring FFTs and remap.  The whole sequence can be captured in a HIP graph
 * and replayed.  Work-item shape (m per item) and persistent grid size come
 * from an autotuner that times the candidates on the batch itself at the
 * first run and caches the choice on disk (TAYLENS_TUNE_CACHE, default
 * $HOME/.cache/taylens_tune.txt; unwritable: not cached).
 * Requirements: every plan TL_FP32 form, same order (<= 8), same pol, same
 * stream; a batch keeps its own harmonic-stage output per realization. */
typedef struct tl_batch_s *tl_batch;
typedef struct {
    int32_t autotune;       /* 1: tune at the first run (see above); 0: use the two fields below */
    int32_t use_graph;      /* 1: capture at the first run, replay while the argument pointers are unchanged */
    int32_t m_groups;       /* runs of 8 m per work item, 1..8 (0: 1) */
    int32_t groups_per_cu;  /* persistent workgroups per compute unit, 1..8 (0: 2) */
} tl_batch_options;

int tl_batch_create(tl_batch *out, int32_t n, const tl_plan *plans, const tl_batch_options *opt);
int tl_batch_destroy(tl_batch b);
/* alms: 4n device pointers (T, E, B, phi per realization; E/B/phi as in
 * tl_lens_map, B all NULL or all set); outs: 3n device pointers. */
int tl_batch_run(tl_batch b, const void *const *alms, void *const *outs);
/* The work-item shape in use and the tuned time of the harmonic launch (ms,
 * 0 if not tuned); graph_replays counts runs served by graph replay. */
int tl_batch_info(tl_batch b, int32_t *m_groups, int32_t *groups_per_cu, double *tuned_ms,
                  int64_t *graph_replays);

/* ---- learned remainder correction ----
 *
 * The Taylor series of eq. 5 is cut at order N; a small network predicts,
 * per output pixel, what the terms beyond order 2 add (the order-6 minus
 * order-2 sum), from the 5 x 5 patch of order <= 2 derivative maps around the
 * nearest source pixel (Sec. II.B gives the nearest-pixel expansion it
 * corrects).  The correction is added to the order-2 sum before the
 * polarization rotation R.  Network: input channels = the 18 pre-scaled maps
 * Dt_jk (j + k <= 2) of T, Q, U, each field divided by its RMS sigma_f over
 * the patch, plus the scaled residuals u, v; conv 3x3 valid 20 -> 32 + tanh,
 * conv 3x3 valid 32 -> 32 + tanh, 1x1 32 -> 3 = y; correction_f =
 * sigma_f * scale_f * y_f.  Forward on BF16 matrix cores with FP32
 * accumulation; FP32 master weights; training by Adam on the mean squared
 * error of y against target_f / (sigma_f scale_f).
 *
 * Parameter vector (host, float, TL_CNN_NPARAM): W1[32][20][3][3], b1[32],
 * W2[32][32][3][3], b2[32], W3[3][32], b3[3] (the TL_CNN_NTRAIN trained
 * values), then scale[3] (fixed).
 *
 * Every call that takes a plan needs an order-2, polarized plan whose form
 * is not TL_FP64 (its derivative maps are float); it runs on the plan's
 * stream.  D = that plan's derivative maps (tl_synth_derivs layout, float
 * [3][6][ntheta][nphi]), alpha_theta / alpha_phi its deflection
 * (tl_deflection, double [ntheta][nphi]); pix = n flat output-pixel indices
 * (ring-major, device int64) or NULL for pixels 0..n-1.  Device buffers are
 * the caller's.  A network object is not thread-safe. */
#define TL_CNN_NTRAIN 15139
#define TL_CNN_NPARAM 15142
typedef struct tl_cnn_s *tl_cnn;

/* Create from a host parameter vector; Adam state zero.  The weights are
 * uploaded on the null stream (synchronized before return). */
int tl_cnn_create(tl_cnn *out, const float *params);
int tl_cnn_destroy(tl_cnn net);
/* Copy the current parameters to host memory (synchronizes the device). */
int tl_cnn_get_params(tl_cnn net, float *params_out);
/* Replace the parameters (host vector) and reset the Adam state. */
int tl_cnn_set_params(tl_cnn net, const float *params);

/* corr_out (device float [3][n]): the correction of each selected pixel. */
int tl_cnn_forward(tl_cnn net, tl_plan plan, const float *D, const double *alpha_theta,
                   const double *alpha_phi, const int64_t *pix, int64_t n, float *corr_out);

/* Gradient of the training loss for target (device float [3][n], the
 * remainder to predict for each pixel, same layout as corr_out):
 * grad_out (device float [TL_CNN_NTRAIN + 1]) = d loss / d params in
 * parameter order, then the loss itself.  Parameters are not changed. */
int tl_cnn_grad(tl_cnn net, tl_plan plan, const float *D, const double *alpha_theta,
                const double *alpha_phi, const int64_t *pix, int64_t n, const float *target,
                float *grad_out);

/* One Adam step (beta 0.9, 0.999, eps 1e-8, bias-corrected) at learning rate
 * lr on the gradient for target; loss_out (device float, may be NULL) gets
 * the loss before the step. */
int tl_cnn_train_step(tl_cnn net, tl_plan plan, const float *D, const double *alpha_theta,
                      const double *alpha_phi, const int64_t *pix, int64_t n, const float *target,
                      float lr, float *loss_out);

/* tl_lens_map of an order-2 plan with the network's correction added before
 * the rotation. */
int tl_lens_map_cnn(tl_plan plan, tl_cnn net, const void *alm_T, const void *alm_E,
                    const void *alm_B, const void *alm_phi, void *T_out, void *Q_out, void *U_out);

/* ---- instrumentation ---- */

/* Stages timed by tl_plan_profile, one kernel launch each:
 * 0 harmonic kernel of the deflection (FP64; all rings, or the pole-adjacent
 * rings when the table GEMM carries the lensing potential), 1 its ring FFTs,
 * 2 direct FP64 harmonic kernel of T, 3 direct FP64 harmonic kernel of Q/U
 * (all rings in the FP64 form, the pole-adjacent rings in the others),
 * 4 matrix-core harmonic kernel of the FP32 form (T and Q/U, the remaining
 * rings), 5 right-hand sides of the tabulated forms, 6 their table GEMM
 * (column sums), 7 ring FFTs of the derivative maps, 8 remap + Taylor sum +
 * rotation, 9 the learned correction network (tl_lens_map_cnn), 10 the
 * epilogue of the table GEMM (theta-derivative rows from the column sums),
 * 11 the polar caps of the FP32 and tabulated forms in one launch: the
 * direct FP64 recursion for T, for each spin family of Q/U and (when the
 * table GEMM carries the lensing potential) for the deflection, every
 * realization of the pass (stages 0, 2 and 3 then cover only what this one
 * does not).  The direct kernels take several realizations per launch in
 * tl_lens_map_many. */
#define TL_NSTAGE 12

/* enable != 0: from now on record a HIP event pair on the plan's stream
 * around every stage of every call (no synchronization is added); 0: stop.
 * Either way the accumulated records are cleared. */
int tl_plan_profile(tl_plan plan, int32_t enable);

/* Synchronize the plan's stream and return, per stage, the summed elapsed
 * milliseconds (ms[TL_NSTAGE]) and the number of timed launches
 * (calls[TL_NSTAGE], may be NULL) since profiling was enabled. */
int tl_plan_stage_times(tl_plan plan, double *ms, int64_t *calls);

/* Thread-local message of the last failure on this thread ("" if none). */
const char *tl_last_error(void);

/* Library version: major*10000 + minor*100 + patch. */
int tl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TAYLENS_H */
