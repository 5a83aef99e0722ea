/*
 * apx.h — C ABI of the MI355X (gfx950) chi^2 forward-modelling library.
 *
 * The library renders images made of elliptical Sersic profiles, point sources and a
 * flat sky per image, integrates them over sub-pixel nodes, convolves them with a PSF,
 * and fits them by Levenberg-Marquardt.  It implements the hot path of image
 * modelling described in "AstroPhot: Fitting Everything Everywhere All at Once in
 * Astronomical Images" (Stone et al. 2023):
 *   - composite model, a sum of windowed components (§2.1, §2.1.1, §2.4 windows);
 *   - sub-pixel integration (§2.1.2) and direct-mode PSF convolution (§2.1.3);
 *   - chi^2 of data, model and inverse variance (§2.2, Eq. chi2);
 *   - exact derivatives (§2.3), Levenberg-Marquardt with damped Cholesky (§2.5);
 *   - many small fits batched together (§3.2), joint multi-image fits with shared
 *     parameters and per-image pixel->sky maps (§3.3).
 *
 * Conventions (identical to the Python spec that the binding marshals):
 *   - Pixel (i, j) of an H x W image has its centre at x = j, y = i.  Arrays are
 *     row-major.  Data, weight and model arrays of all images are concatenated in
 *     image order into one flat FP32 buffer ("pixel buffer", n_pix elements).
 *   - The PSF of image k is a P x P FP32 stamp (P odd, 1 <= P <= 63), used as given
 *     (callers normalise it); stamps are concatenated in image order.  The model is
 *     the true convolution M[i,j] = sum_{u,v} K[c+u][c+v] S[i-u][j-v], c = (P-1)/2,
 *     of the pre-convolution image S defined on the extended grid
 *     [-c, H+c) x [-c, W+c), plus the image's flat sky (not convolved).
 *   - affine[6] maps pixel to sky coordinates:
 *       u_x = a0 + a1 x + a2 y,  u_y = a3 + a4 x + a5 y;  pixel area = |a1 a5 - a2 a4|.
 *   - A Sersic component has local parameters (x0, y0, q, PA, n, Re, log10 Ie), centre
 *     in the sky frame, PA in radians counter-clockwise from +x;
 *     I(R) = Ie exp(-b_n ((R/Re)^(1/n) - 1)), R = sqrt(x'^2 + (y'/q)^2) floored at 1e-6,
 *     gamma(2n, b_n) = Gamma(2n)/2.  A pixel holds area * sum_k w_k I(node_k).
 *   - A point source has local parameters (x, y, log10 F) in the sky frame; its flux is
 *     splatted bilinearly onto the four surrounding pixel centres before convolution
 *     (the "psf star model", bilinear PSF interpolation).  Only log10 F may be free.
 *   - par[k] is the theta index of local parameter k, or -1 (value taken from
 *     fixed[k]).  Indices may repeat across components (tied parameters, whose
 *     derivatives add).  Every sub-problem owns one contiguous theta range
 *     (sub_par[2s], sub_par[2s+1]) and every parameter of its images lies inside it.
 *   - chi^2 = sum_i w_i (d_i - m_i)^2 (the paper's Eq. chi2 is half of this plus a
 *     constant); w = 1/sigma^2, w = 0 masks a pixel.
 *
 * Precision: theta, chi^2, J^T W J, J^T W r, gradients and LM state are FP64.  Images,
 * PSFs, weights, models and Jacobian entries are stored in FP32.  The Jacobian path
 * (derivative sampling, its convolutions) and the adjoint run in FP32 with FP64
 * pixel->centre offsets; the objective path (model for chi^2, residual and LM trials)
 * runs in FP64 unless APX_OBJECTIVE_FP32 is chosen.  Every reduction accumulates in
 * FP64 in a fixed order (results are bitwise reproducible).
 *
 * Ownership: every pointer argument of a hot-path call is a caller-owned DEVICE
 * pointer, except where marked "host".  The library copies descriptors at
 * apx_problem_create, borrows the PSF pointer for the life of the problem, and keeps
 * its scratch in one caller-provided device workspace (apx_problem_bind_workspace).
 * After binding, hot-path calls allocate nothing and do not synchronise the host;
 * they are enqueued on the context's stream.
 *
 * Errors: every call returns apx_status (0 = APX_OK).  Host-side validation failures
 * return APX_E_INVALID / APX_E_UNSUPPORTED / APX_E_WORKSPACE before anything is
 * enqueued; HIP runtime failures return APX_E_HIP.  apx_last_error() gives a message.
 * Conditions found on the device (parameters outside the model's domain, non-finite
 * values) set a sticky per-problem flag read by apx_problem_check(), which
 * synchronises the stream.  Nothing throws across the ABI.
 */
#ifndef APX_H
#define APX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t apx_status;

#define APX_OK              0
#define APX_E_INVALID      (-1)   /* bad descriptor, size, index or null pointer     */
#define APX_E_HIP          (-2)   /* HIP runtime error                               */
#define APX_E_NONFINITE    (-3)   /* NaN/Inf met on the device                       */
#define APX_E_WORKSPACE    (-4)   /* no workspace bound, or too small                */
#define APX_E_UNSUPPORTED  (-5)   /* e.g. P > 63, a free point-source position       */
#define APX_E_DOMAIN       (-6)   /* theta outside the model domain (render/chi2)    */

#define APX_SERSIC 0
#define APX_POINT  1

#define APX_RULE_MIDPOINT        0   /* offsets (k+1/2)/s - 1/2, weights 1/s^2       */
#define APX_RULE_GAUSS_LEGENDRE  1   /* s-point Gauss-Legendre per axis (§2.1.2)     */

#define APX_MODE_UNIFORM     0       /* s x s nodes in every pixel                   */
#define APX_MODE_WITHIN_K_RE 1       /* s x s nodes where the pixel-centre R < k Re,
                                        the pixel centre alone elsewhere (§2.1.2)     */
#define APX_MODE_ADAPTIVE    2       /* two-pass adaptive integration (§2.1.2), k_re is
                                        the relative tolerance tol > 0; s and rule are
                                        not used.  Per Sersic component: the pixel
                                        centres give the window flux F and the error
                                        budget e = tol F / N (N window pixels); a pixel
                                        keeps its centre value when the second-difference
                                        estimate of the midpoint error, area (|I(x+1) +
                                        I(x-1) - 2 I| + |I(y+1) + I(y-1) - 2 I|) / 24, is
                                        at most e, else takes 3 x 3 Gauss-Legendre when
                                        that moves it by at most e, else is cut into
                                        5 x 5 sub-pixels, each at 5 x 5 Gauss-Legendre
                                        when within e of its 3 x 3 value, else the mean
                                        of its 5 x 5 sub-sub-pixels at 7 x 7.  The choices
                                        are made in FP64 at each theta; the derivatives
                                        are those of the chosen rule (choices held
                                        fixed).                                         */

/* Precision of the objective path (render -> convolve -> chi^2 / residual).  The
 * Jacobian path (derivative images, their convolutions, J^T W J inputs) and the adjoint
 * contraction always run in FP32 with FP64 accumulation. */
#define APX_OBJECTIVE_FP64   0       /* default: FP64 profiles, convolution and chi^2;
                                        the LM gain ratio resolves chi^2 changes far
                                        below FP32 rounding (parameter rtol 1e-6)      */
#define APX_OBJECTIVE_FP32   1       /* FP32 profiles and convolution (fastest render) */

#define APX_MAX_PSF 63

/* Convolution mode (§2.1.3: direct convolution, efficient for small stamps, or FFT
 * convolution, efficient for large ones).  APX_CONV_FFT applies to images with P >=
 * APX_FFT_MIN_P: their Jacobian-column and adjoint convolutions, and the model convolution
 * when the objective is FP32, whose output box is at least 32 x 32 run as overlap-save
 * 128 x 128 FFTs in FP32 (two output blocks per complex transform); the rest stays direct,
 * as does the FP64 objective convolution.  Results equal the direct ones to FP32 rounding
 * relative to each tile's largest values. */
#define APX_CONV_DIRECT 0
#define APX_CONV_FFT    1
#define APX_FFT_MIN_P   15
/* APX_CONV_DIRECT also runs the Jacobian-column convolutions of an image whose stamp is
 * the outer product of two vectors (rank one to FP32 rounding: K_uv = a_u b_v, e.g. a
 * Gaussian) as two 1-D passes, 2 P multiply-adds per output per pass instead of P^2; the
 * result is the same convolution to FP32 rounding.  The stamp is read back when the problem
 * is created.  The objective (model) convolution stays 2-D.  APX_CONV_DIRECT_2D keeps
 * every convolution 2-D. */
#define APX_CONV_DIRECT_2D 2
/* APX_CONV_AUTO: as APX_CONV_DIRECT (rank-one stamps by two 1-D passes), and a job of the
 * FP32 kinds (Jacobian columns, adjoint, the FP32 objective's model) on an image with a
 * fixed stamp of P >= APX_FFT_MIN_P that is not rank one, no sub-pixel grid and an output
 * box of at least 32 x 32 runs as FFT tiles (as in APX_CONV_FFT) when an operation-count
 * model prices them below its direct tiles: with nch channels of an h x w output, blocks =
 * ceil(h / (129 - P)) ceil(w / (129 - P)), FFT cost = ceil(nch blocks / 2)
 * APX_AUTO_FFT_PAIR_COST, direct cost = nch min over the four tile shapes (TH x TW) of
 * ceil(h / TH) ceil(w / TW) (TH TW (P^2 + 10) + 8 (TH + P - 1)(TW + P - 1) + 3000); FFT
 * when strictly cheaper.  The choice depends on the geometry only, not on timings. */
#define APX_CONV_AUTO 3
#define APX_AUTO_FFT_PAIR_COST 1.0e6

/* Sub-pixel re-centring (§2.1.3).  With shift != APX_SHIFT_NONE every Sersic component
 * is sampled (and pixel-integrated) with its centre moved to the centre of the nearest
 * pixel of its image, n = floor(p + 1/2) for its pixel position p, and the convolved
 * image is moved back by delta = p - n (each axis in [-1/2, 1/2)) by interpolation:
 * m_c(i) = sum_t w_y(t_y) w_x(t_x) (K * S'_c)(i - t), |t| <= a per axis, with
 *   APX_SHIFT_BILINEAR: a = 1, the two nearest samples (1 - |delta|, |delta|);
 *   APX_SHIFT_LANCZOS:  a = shift_a in [2, APX_SHIFT_MAX_A], weights
 *                       sinc(t - delta) sinc((t - delta)/a), normalised to unit sum.
 * The derivatives in x0, y0 come through delta alone (d delta / d(x0, y0) is the inverse
 * of the image's linear map; the bilinear one is taken from the right at delta = 0).
 * Point sources (already bilinear splats) are not moved.  The library applies the shift
 * before the convolution (it commutes with it), so a component's support grows by a
 * pixels on every side (clipped to the extended grid).  Not with APX_MODE_ADAPTIVE, nor
 * with psf_up > 1 (a higher-resolution PSF is the alternative the paper gives). */
#define APX_SHIFT_NONE     0
#define APX_SHIFT_BILINEAR 1
#define APX_SHIFT_LANCZOS  2
#define APX_SHIFT_MAX_A    5

/* LM constants (§2.5 gives the method, not the constants; these are fixed here). */
#define APX_LM_LAMBDA0     1e-2
#define APX_LM_UP          11.0
#define APX_LM_DOWN        9.0
#define APX_LM_EPS4        0.1
#define APX_LM_LAMBDA_MIN  1e-9
#define APX_LM_LAMBDA_MAX  1e9
#define APX_LM_ATTEMPTS    4      /* Cholesky tries per iteration (lambda *= UP between) */
#define APX_LM_DAMP_FLOOR  1e-12  /* D_kk = max(A_kk, floor * max A_kk)                */

/* An image whose PSF has a higher resolution than its pixels (§2.1.3: sampling and
 * convolution then run at the PSF's resolution and the result is integrated onto the
 * image pixels) sets psf_up = U in {2, 4, 8}: its model is rendered on U x U sub-pixels
 * per pixel (sub-pixel (yf, xf) centred at pixel coordinates ((xf + 1/2)/U - 1/2,
 * (yf + 1/2)/U - 1/2)), convolved there with its stamp (P in sub-pixels) and summed over
 * each pixel's U x U sub-pixels.  Its components' windows are then in sub-pixels
 * (extended by c sub-pixels).  Such images always use direct convolution. */
typedef struct apx_image_desc {
    int32_t H, W;          /* output grid                                        */
    int32_t P;             /* PSF side, odd, 1..63                               */
    int32_t sub;           /* sub-problem this image belongs to                  */
    int32_t sky_par;       /* theta index of the flat sky, -1 = fixed            */
    int32_t psf_up;        /* PSF samples per pixel per axis: 0 or 1 (same
                              resolution), 2, 4 or 8                             */
    double  sky_fixed;     /* sky value when sky_par == -1                       */
    double  affine[6];     /* pixel -> sky map (see above)                       */
} apx_image_desc;

typedef struct apx_comp_desc {
    int32_t type;          /* APX_SERSIC or APX_POINT                            */
    int32_t image;         /* image index                                        */
    int32_t box[4];        /* window (y0, x0, y1, x1), half-open, extended-grid
                              coordinates of its image; clipped by the library     */
    int32_t par[7];        /* theta indices of the local parameters, -1 = fixed  */
    int32_t reserved;
    double  fixed[7];      /* values of fixed local parameters                   */
} apx_comp_desc;

/* Live PSF model of one image (§2.1.3: the PSF may itself be a model with parameters
 * optimised in the fit; §3.4).  APX_PSF_MOFFAT: f(r) = (1 + r^2 / R_d^2)^(-n) with power n
 * and scale R_d in pixels, point-sampled at the integer offsets of the image's P x P stamp
 * grid and normalised to unit sum before the convolution.  The image's stamp in `psf` only
 * fixes P.  Its parameters may be free theta indices of the image's sub-problem (they add
 * Jacobian columns (dK/dphi) * S, S the pre-convolution model) or fixed.  Domain, checked
 * like the Sersic one: n in [0.2, 20], R_d in [0.05, 1e3]. */
#define APX_PSF_MOFFAT 0
typedef struct apx_psf_model_desc {
    int32_t image;         /* image index (at most one model per image)          */
    int32_t type;          /* APX_PSF_MOFFAT                                     */
    int32_t par[2];        /* theta indices of (n, R_d), -1 = fixed              */
    double  fixed[2];      /* values of fixed parameters                         */
} apx_psf_model_desc;

typedef struct apx_problem_desc {
    int32_t n_images, n_comps, n_par, n_sub;
    const apx_image_desc* images;   /* host, [n_images]                            */
    const apx_comp_desc*  comps;    /* host, [n_comps]                             */
    const int32_t*        sub_par;  /* host, [2*n_sub]: first theta index, count   */
    const float*          psf;      /* device, concatenated P*P stamps (borrowed)  */
    int32_t s;                      /* nodes per axis, 1..8                        */
    int32_t rule;                   /* APX_RULE_*                                  */
    int32_t mode;                   /* APX_MODE_*                                  */
    int32_t objective;              /* APX_OBJECTIVE_* (precision of the model used
                                       for chi^2, residuals and LM trials)          */
    double  k_re;                   /* k of APX_MODE_WITHIN_K_RE; tol of
                                       APX_MODE_ADAPTIVE                             */
    int32_t n_psf_models;           /* live PSF models (0: every stamp is fixed)     */
    int32_t conv_mode;              /* APX_CONV_DIRECT (default), APX_CONV_FFT, APX_CONV_DIRECT_2D or APX_CONV_AUTO */
    const apx_psf_model_desc* psf_models;   /* host, [n_psf_models]                 */
    int32_t shift;                  /* APX_SHIFT_* sub-pixel re-centring (0 = none)   */
    int32_t shift_a;                /* Lanczos order a (APX_SHIFT_LANCZOS only)      */
} apx_problem_desc;

/* Per-sub-problem LM state, device memory, [n_sub] entries (apx_lm_init fills it). */
typedef struct apx_lm_state {
    double  lambda;        /* current damping                                     */
    double  chi2;          /* chi^2 at the current theta                          */
    double  chi2_trial;    /* chi^2 of the last trial (inf if out of domain)      */
    double  pred;          /* predicted decrease h^T (lambda D h + g) of the trial */
    double  rho;           /* gain ratio of the last trial                        */
    int32_t need_jac;      /* 1: J^T W J must be formed at theta before the solve */
    int32_t accepted;      /* last trial accepted                                 */
    int32_t n_accept, n_reject;
    int32_t n_chol_retry;  /* Cholesky failures so far (each raised lambda)       */
    int32_t status;        /* 0, or APX_E_* found on the device                   */
} apx_lm_state;

typedef struct apx_ctx apx_ctx;
typedef struct apx_problem apx_problem;

/* --------------------------------------------------------------- lifecycle ---- */
const char* apx_version(void);
const char* apx_status_string(apx_status s);

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t (NULL = the
 * default stream).  device = -1 creates a host-only context: problems can be created
 * (validated and planned) and sized, but not bound or run.  Errors: APX_E_INVALID
 * (null out), APX_E_HIP. */
apx_status apx_ctx_create(int device, void* hip_stream, apx_ctx** out);
apx_status apx_ctx_set_stream(apx_ctx* ctx, void* hip_stream);

/* Output tile shapes of the direct convolution (§2.1.3).  Every convolution job (an image,
 * or the Jacobian columns of one window) is cut into workgroup tiles of one of four shapes:
 * 0 = 32 x 64, 1 = 16 x 64, 2 = 32 x 32, 3 = 16 x 32 output pixels; the direct jobs of one
 * kind at one PSF size take the one shape of least estimated cost (tiles needed x cost of
 * one tile, summed over those jobs), so that each PSF size is one launch.  The policy
 * holds for problems created after the call:
 *   APX_TILES_AUTOTUNE (default): on a device context, the first problem that needs a
 *     convolution kernel at a PSF size times all four shapes of it on a synthetic
 *     256 x 256 job of 32 channels (a few ms, synchronous on the context stream, in scratch
 *     memory the context allocates once and frees in apx_ctx_destroy) and the context keeps
 *     the table; host-only contexts use the model;
 *   APX_TILES_MODEL: an operation-count model, no timing;
 *   APX_TILES_FIXED + s (s = 0..3): shape s for every job.
 * The shape changes nothing but the order in which the FP64 per-tile partial sums of chi^2,
 * J^T W r and the gradient are added.  APX_E_INVALID for an unknown policy. */
#define APX_TILES_AUTOTUNE  0
#define APX_TILES_MODEL     1
#define APX_TILES_FIXED     2
apx_status apx_ctx_set_tiles(apx_ctx* ctx, int32_t policy);

/* Measured cost of one tile, in microseconds, of each shape (us[4]) of convolution kernel
 * `kernel` (0 model FP32, 1 Jacobian columns, 2 adjoint, 3 model FP64) at PSF size P, as
 * timed by the autotuner; APX_E_INVALID when that pair has not been timed. */
apx_status apx_ctx_tile_cost(const apx_ctx* ctx, int32_t kernel, int32_t P, double* us);

/* Set that table entry (us[4], positive and finite) instead of timing it: under
 * APX_TILES_AUTOTUNE, problems created afterwards take their shapes from it.  Replays another
 * run's choices, e.g. under a profiler that perturbs the timings.  APX_E_INVALID for a bad
 * kernel, an even or out-of-range P, or a bad cost. */
apx_status apx_ctx_set_tile_cost(apx_ctx* ctx, int32_t kernel, int32_t P, const double* us);
apx_status apx_ctx_destroy(apx_ctx* ctx);
const char* apx_last_error(const apx_ctx* ctx);

/* Validate and copy the descriptor, build the launch plan (tiles, component lists,
 * Jacobian groups, pair lists).  Host-only; nothing is enqueued.  Errors:
 * APX_E_INVALID (inconsistent descriptor), APX_E_UNSUPPORTED. */
apx_status apx_problem_create(apx_ctx* ctx, const apx_problem_desc* desc, apx_problem** out);

/* Bytes of device workspace the problem needs (256-byte aligned base required). */
apx_status apx_problem_workspace_bytes(const apx_problem* p, uint64_t* bytes);

/* Hand the problem its workspace (caller-owned device memory, >= the queried size)
 * and upload the plan into it (asynchronously on the context stream).  Errors:
 * APX_E_WORKSPACE (null / too small / misaligned), APX_E_HIP. */
apx_status apx_problem_bind_workspace(apx_problem* p, void* dev, uint64_t bytes);

/* Sizes: total output pixels, total extended-grid pixels, stored Jacobian entries. */
apx_status apx_problem_sizes(const apx_problem* p, int64_t* n_pix, int64_t* n_ext, int64_t* n_jac);

/* Convolution jobs of `kind` (0 model, 1 Jacobian columns, 2 adjoint) per tile shape:
 * counts[s] for s = 0..3 (see apx_ctx_set_tiles), counts[4] = jobs in FFT mode, counts[5]
 * = jobs run as two 1-D passes (rank-one stamps).  counts must hold 6 entries. */
apx_status apx_problem_tile_shapes(const apx_problem* p, int32_t kind, int32_t* counts);

/* Synchronise the stream and return the sticky device flag, then clear it: APX_OK,
 * APX_E_DOMAIN, APX_E_NONFINITE, or APX_E_HIP when a substitution hand-off wait of the
 * damped solve ran out (that iteration's step was dropped). */
apx_status apx_problem_check(apx_problem* p);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): binds the problem to the library's own
 * scratch array on the context's device instead of a caller workspace -- 64 MiB per GPU,
 * a static device array that each GPU the library runs on holds until the process ends.
 * Afterwards every entry point behaves as after apx_problem_bind_workspace (same kernels,
 * same results) and allocates nothing.  This call allocates nothing either: it uploads
 * the plan tables and clears the flags that must start at zero, after a device-wide
 * synchronisation.  The scratch is shared: binding another problem on the same device
 * makes the earlier one refuse further calls with APX_E_WORKSPACE (bind it again to use
 * it), and calls on the scratch from several threads or streams at once race.
 * APX_E_WORKSPACE (with the sizes in apx_last_error) when apx_problem_workspace_bytes
 * exceeds 64 MiB; APX_E_INVALID for a host-only context; APX_E_HIP if the array's address
 * could not be looked up.  Note that apx_problem_create itself may allocate once per
 * context for the tile autotuner's timing buffer: use APX_TILES_MODEL or a fixed shape
 * (apx_ctx_set_tiles), or measured costs (apx_ctx_set_tile_cost), to avoid it. */
apx_status apx_problem_bind_scratch(apx_problem* p);

/* Bound of the damped solve's substitution hand-off waits (the blocked Cholesky path of
 * sub-problems with more than 64 parameters, §2.5).  Each wait polls a flag that an
 * earlier workgroup of the same launch raises; one that polls `polls` times without
 * seeing it gives up, raises the sticky flag reported as APX_E_HIP by apx_problem_check,
 * and that iteration's step is dropped (theta and lambda as after a failed factorisation).
 * polls > 0: the bound; 0: the default (2^22 polls); polls < 0: every wait takes its flag
 * as never raised and gives up after -polls polls -- a way to exercise the give-up path
 * from the host in which every kernel still ends normally.  Synchronises the stream and
 * drops a captured LM iteration graph.  APX_E_WORKSPACE before bind_workspace. */
apx_status apx_problem_set_wait_limit(apx_problem* p, int32_t polls);
apx_status apx_problem_destroy(apx_problem* p);

/* Kernel timing (tracing aid).  When enabled, every launch group of the hot path is
 * bracketed by HIP events recorded on the context stream; apx_problem_timing()
 * synchronises and returns the summed duration and launch count of one class since
 * the last enable.  With apx_lm_run(use_graph = 1) the events are captured into the
 * iteration's graph (a graph captured under another set of classes is captured again)
 * and every replay records into fresh events.  The classes cannot change during a
 * capture (APX_E_INVALID). */
#define APX_TIME_PREP       0
#define APX_TIME_RENDER     1     /* pre-convolution render (objective path)   */
#define APX_TIME_CONV_FWD   2     /* model convolution + chi^2 partials         */
#define APX_TIME_DERIV      3     /* derivative images                          */
#define APX_TIME_CONV_JCOL  4     /* Jacobian-column convolutions               */
#define APX_TIME_PAIRS      5     /* J^T W J tiles (MFMA)                       */
#define APX_TIME_REDUCE     6     /* ordered reductions and assembly            */
#define APX_TIME_SOLVE      7     /* damped Cholesky + substitution             */
#define APX_TIME_LM         8     /* trial, accept and state kernels            */
#define APX_TIME_CONV_ADJ   9     /* adjoint convolution                        */
#define APX_TIME_GRAD       10    /* adjoint contraction with recomputed samples */
#define APX_TIME_CONV_SEP   11    /* Jacobian-column convolutions as two 1-D passes (rank-one stamps) */
#define APX_TIME_CONV_FFT   12    /* convolutions on FFT tiles (any kind)        */
#define APX_TIME_CLASSES    13
/* Kernel timing with HIP events on the context stream: enabled != 0 records every class;
 * set_timing_classes records only the classes in mask (bit 1 << class), which keeps the
 * event overhead off the other launches.  Either call resets the records. */
apx_status apx_problem_set_timing(apx_problem* p, int32_t enabled);
apx_status apx_problem_set_timing_classes(apx_problem* p, uint32_t mask);
apx_status apx_problem_timing(apx_problem* p, int32_t klass, double* total_ms, int64_t* launches);

/* ------------------------------------------------------------------ hot path ---- */
/* model[n_pix] = PSF (x) sum of components + sky, for all images (§2.1, §2.1.2-3).
 * theta: device [n_par] FP64.  Out-of-domain theta -> APX_E_DOMAIN via check(). */
apx_status apx_render(apx_problem* p, const double* theta, float* model);

/* chi2[n_sub] = sum w (d - m)^2 per sub-problem (§2.2, Eq. chi2 without the 1/2).
 * data, weight: device [n_pix] FP32.  chi2: device FP64. */
apx_status apx_chi2(apx_problem* p, const double* theta, const float* data,
                    const float* weight, double* chi2);

/* Dense Jacobian dm/dtheta (§2.3): J[k * ldJ + i] for theta index k, pixel i
 * (ldJ >= n_pix), FP32, every entry written (zeros outside supports). */
apx_status apx_jacobian(apx_problem* p, const double* theta, float* J, int64_t ldJ);

/* Per sub-problem s (theta range [p0, p0+n)): JtWJ block n x n row-major at offset
 * sum_{t<s} n_t^2, JtWr[p0 + k], chi2[s] (§2.5 normal equations).  FP64, device. */
apx_status apx_jtwj(apx_problem* p, const double* theta, const float* data,
                    const float* weight, double* JtWJ, double* JtWr, double* chi2);

/* d chi2 / d theta [n_par] FP64 by the adjoint (reverse) pass: correlate -2 w r with
 * the PSF onto the extended grid, then contract with the recomputed sub-pixel
 * derivatives (§2.3 backpropagation); also writes chi2[n_sub]. */
apx_status apx_chi2_grad(apx_problem* p, const double* theta, const float* data,
                         const float* weight, double* grad, double* chi2);

/* Parameter covariance at theta (§2.5: the inverse of the Hessian the LM approximates
 * gives the uncertainties and the full covariance of the parameters): for each
 * sub-problem s, cov_s = (J^T W J)^{-1} in FP64, an n_s x n_s row-major block at offset
 * sum_{t<s} n_t^2 (the layout of apx_jtwj's JtWJ); also chi2[n_sub].  J^T W J is formed
 * as in apx_jtwj, factored by Cholesky without damping and inverted column block by
 * column block.  For chi^2 = sum w r^2 this is the usual 1-sigma covariance (the inverse
 * of half the chi^2 Hessian).  A block whose J^T W J is not positive definite is filled
 * with NaN.  cov: device FP64, overwritten; asynchronous on the context stream. */
apx_status apx_covariance(apx_problem* p, const double* theta, const float* data,
                          const float* weight, double* cov, double* chi2);

/* Factor of the parameter covariance, for use as the sampler's mass matrix: for each
 * sub-problem s, F_s = L^{-T} where J^T W J = L L^T (lower Cholesky factor, no damping),
 * so that F_s F_s^T = (J^T W J)^{-1} = cov_s of apx_covariance.  F_s is upper triangular,
 * written in full (zeros below the diagonal) as an n_s x n_s row-major block at offset
 * sum_{t<s} n_t^2; also chi2[n_sub].  A block whose J^T W J is not positive definite is
 * filled with NaN.  F: device FP64, overwritten; asynchronous on the context stream. */
apx_status apx_covariance_factor(apx_problem* p, const double* theta, const float* data,
                                 const float* weight, double* F, double* chi2);

/* Hamiltonian Monte Carlo (§2.5; §3.5 starts it at the LM fit with the LM covariance as the
 * inverse mass matrix; the method is the hybrid Monte Carlo of Duane et al. 1987).  Target
 * of each sub-problem s: U_s = chi2_s / 2 (flat priors), sampled as its own chain.
 * F: device FP64 per-sub blocks in the layout of apx_covariance with F_s F_s^T = Sigma_s,
 * the inverse mass matrix (apx_covariance_factor gives one; any factor is accepted).  The
 * momenta are whitened, r = F^T p ~ N(0, I), K = |r|^2 / 2, and a leapfrog step of size
 * `step` is r -= (step/2) F^T grad U; theta += step F r; r -= (step/2) F^T grad U.
 * Sample i: r = z[i * n_par + j] (j over the sub-problem's range), n_leapfrog steps
 * (n_leapfrog gradient passes; the gradient at the start of a trajectory is carried over),
 * then per sub-problem: accepted iff every leapfrog point stayed in the model domain and
 * log(u[i * n_sub + s]) < H0 - H1, H = U + K; a rejected sub-problem returns to its start.
 * theta: device [n_par] FP64, in: start, out: the chain's last state.  z: device FP64
 * [n_samples * n_par] standard normals; u: device FP64 [n_samples * n_sub] uniforms in
 * (0, 1] (the caller draws both).  samples: device FP64 [n_samples * n_par], theta after
 * each transition (entries outside every sub-problem copied).  stats: device FP64
 * [n_samples * n_sub * 3] = (accepted 0/1, H0, H1).  An out-of-domain start raises
 * APX_E_DOMAIN via apx_problem_check; out-of-domain points inside trajectories only reject.
 * n_leapfrog >= 1, step > 0 finite, n_samples >= 0, else APX_E_INVALID.  Uses the LM's
 * Cholesky scratch (do not interleave with apx_lm_* calls of the same problem).
 * Asynchronous on the context stream. */
apx_status apx_hmc_run(apx_problem* p, const float* data, const float* weight, double* theta,
                       const double* F, double step, int32_t n_leapfrog, int32_t n_samples,
                       const double* z, const double* u, double* samples, double* stats);

/* No-U-Turn sampling (§2.5; §3.5 runs NUTS from the LM fit with the LM covariance as the
 * inverse mass matrix): the slice-sampling NUTS of Hoffman & Gelman in the whitened
 * momenta of apx_hmc_run (same F, leapfrog and energy H = sum_s chi2_s / 2 + |r|^2 / 2),
 * one joint chain over all sub-problems.  Per transition i: r = z[i * n_par ...]; the
 * uniforms u[i * D ...], D = 1 + max_depth + 2^(max_depth + 1), are taken strictly in
 * the order the algorithm asks for them: the slice variable (log slice = log(u) - H0),
 * then per doubling a direction (-1 if < 1/2) and, as they occur, one per merge of a
 * subtree (the second half's proposal replaces the first's with probability
 * n'' / (n' + n'')) and one per doubling whose subtree continued (its proposal becomes the
 * sample with probability min(1, n' / n)).  A subtree stops when -H < log slice -
 * APX_NUTS_DELTA_MAX (divergent; also when a point leaves the model domain) or its ends
 * make a U-turn: (theta+ - theta-) . F r- < 0 or (theta+ - theta-) . F r+ < 0.  The tree
 * stops at max_depth doublings (1..APX_NUTS_MAX_DEPTH).  theta: device [n_par], in: start,
 * out: last sample.  samples: device FP64 [n_samples * n_par].  stats: device FP64
 * [n_samples * 4] = (depth, leapfrog steps, points in the slice, divergent).  The tree
 * state lives on the device: each doubling is issued as one fixed sequence of launches
 * (every leaf, merge and U-turn test of a tree of that depth, acting only while the tree has
 * not stopped; a leaf after a stop re-runs the gradient pass on the last point and changes
 * nothing), and the host reads the tree state once per doubling to decide whether to double
 * again.  u is read on the device and, for the directions, once on the host.  Returns after
 * the last transition.  Uses the LM's Cholesky scratch. */
#define APX_NUTS_MAX_DEPTH 10
#define APX_NUTS_DELTA_MAX 1000.0
apx_status apx_nuts_run(apx_problem* p, const float* data, const float* weight, double* theta,
                        const double* F, double step, int32_t max_depth, int32_t n_samples,
                        const double* z, const double* u, double* samples, double* stats);

/* Step-size warm-up of NUTS (§3.5: warm-up samples select the step before sampling):
 * n_warmup transitions of apx_nuts_run (same z, u layout; theta advances) while dual
 * averaging (Hoffman & Gelman) adapts the step on the acceptance statistic a_m = mean over
 * the leaves of transition m's last doubling of min(1, exp(H0 - H)): with mu = log(10 step0),
 * Hbar_m = (1 - 1/(m + t0)) Hbar_{m-1} + (target - a_m) / (m + t0), log step_m = mu -
 * sqrt(m) / gamma Hbar_m, log stepbar_m = m^-kappa log step_m + (1 - m^-kappa) log
 * stepbar_{m-1} (gamma, t0, kappa below).  step: HOST pointer, in: the first step, out:
 * stepbar after the last transition.  target_accept in (0, 1).  Synchronous. */
#define APX_NUTS_DA_GAMMA 0.05
#define APX_NUTS_DA_T0    10.0
#define APX_NUTS_DA_KAPPA 0.75
apx_status apx_nuts_warmup(apx_problem* p, const float* data, const float* weight, double* theta,
                           const double* F, double* step, int32_t max_depth, int32_t n_warmup,
                           double target_accept, const double* z, const double* u);

/* Vector-Jacobian product of the render (the reverse pass of the model of §2.3, the
 * same adjoint as apx_chi2_grad with the caller's seed in place of -2 w r):
 * grad_theta[k] = sum_i grad_model[i] * d model_i / d theta_k, i over every output pixel
 * of every image in apx_render's order.  grad_model: device FP32 [n_pix], read only;
 * grad_theta: device FP64 [n_par], overwritten.  Entries of theta that no component or
 * sky uses get 0.  Out-of-domain theta raises the sticky APX_E_DOMAIN flag as in
 * apx_render.  Asynchronous on the context stream. */
apx_status apx_render_vjp(apx_problem* p, const double* theta, const float* grad_model,
                          double* grad_theta);

/* Initialise the Levenberg-Marquardt state of every sub-problem at theta (§2.5: the fit
 * starts from the initial parameters with a small damping): lambda = 1e-2, chi2 and the
 * residual at theta (the objective path), need_jac = 1 so the first apx_lm_step forms the
 * normal equations, counters zeroed.  theta: device FP64 [n_par], read only (copy it into
 * the buffer the iterations update); data, weight: device FP32 [n_pix]; state: device,
 * [n_sub] apx_lm_state, overwritten.  Out-of-domain theta raises the sticky APX_E_DOMAIN
 * flag (apx_problem_check).  Asynchronous on the context stream. */
apx_status apx_lm_init(apx_problem* p, const double* theta, const float* data,
                       const float* weight, apx_lm_state* state);

/* One LM iteration on every sub-problem (§2.5): form J^T W J, J^T W r if the last
 * step was accepted; damped Cholesky with lambda retries; trial; gain ratio;
 * accept/reject.  theta (device, in/out) and state are updated on the device; the
 * host never waits.  Equivalent to fitting every sub-problem on its own. */
apx_status apx_lm_step(apx_problem* p, const float* data, const float* weight,
                       double* theta, apx_lm_state* state);

/* n_iter Levenberg-Marquardt iterations (§2.5), each exactly apx_lm_step, and for many
 * sub-problems the batching of many small models in one problem (§3.2).  use_graph != 0
 * captures one iteration into a HIP graph on first use (per data / weight / theta / state
 * pointer set and timing classes) and replays it n_iter times: no host work per iteration,
 * results bitwise those of eager iterations.  Buffers as in apx_lm_step (theta and state
 * updated in place on the device); n_iter >= 0, else APX_E_INVALID; a graph needs a
 * non-default context stream (APX_E_INVALID otherwise).  Asynchronous. */
apx_status apx_lm_run(apx_problem* p, int32_t n_iter, const float* data,
                      const float* weight, double* theta, apx_lm_state* state,
                      int32_t use_graph);

#ifdef __cplusplus
}
#endif

#endif /* APX_H */
