// Internal declarations of the apx library: device-side plan records, per-call
// constants and the launchers each kernel translation unit exports to the host API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/apx.h"

namespace apx {

// Tile shapes --------------------------------------------------------------------
constexpr int RT_Y = 8, RT_X = 32;            // render / derivative / gradient tiles (256 px)
// Convolution output tiles a workgroup can own (rows x cols).  Every lane computes CV_R
// consecutive outputs of one row, so shape s runs tile_th(s) * tile_tw(s) / CV_R threads.
// The tile shape of each convolution job is chosen per job (apx_ctx_set_tiles).
constexpr int N_TILE_SHAPES = 4;
__host__ __device__ constexpr int tile_th(int s) { return (s & 1) ? 16 : 32; }
__host__ __device__ constexpr int tile_tw(int s) { return s < 2 ? 64 : 32; }
constexpr int CV_R = 8;                       // consecutive outputs per lane (register window)
constexpr int PAIR_KC = 32;                   // pixels per LDS stage of the J^T W J kernel
constexpr int CHOL_NB = 64;                   // block size of the blocked Cholesky
constexpr int SMALL_N = 64;                   // sub-problems up to this size: one-wave solver
constexpr int MAX_NODES_1D = 8;
constexpr int N_XCD = 8;                       // accelerator dies, each with its own L2
// FFT-mode convolution: 128 x 128 transform tiles; a job in FFT mode has tile shape
// SHAPE_FFT, whose output blocks are (FFT_T - P + 1)^2
constexpr int FFT_T = 128;
constexpr int SHAPE_FFT = N_TILE_SHAPES;
// a Jacobian-column job on an image with a rank-one stamp: two 1-D passes over SEP_TH x
// SEP_TW output tiles
constexpr int SHAPE_SEP = N_TILE_SHAPES + 1;
constexpr int SEP_TH = 32, SEP_TW = 64;
__host__ __device__ constexpr int shape_th(int s, int P) {
    return s == SHAPE_FFT ? FFT_T - P + 1 : (s == SHAPE_SEP ? SEP_TH : tile_th(s));
}
__host__ __device__ constexpr int shape_tw(int s, int P) {
    return s == SHAPE_FFT ? FFT_T - P + 1 : (s == SHAPE_SEP ? SEP_TW : tile_tw(s));
}

// Workgroups of a launch are dealt to the XCDs round-robin (block b to XCD b % 8), each
// with its own L2.  Block b takes logical item xcd_chunk_item(b, n): runs of XCD_CHUNK
// consecutive items go to the XCDs in turn (run k to XCD k % 8), so a run's items (the
// columns of one group, the tile pairs of one pixel slice) share their global reads in one
// L2, while items that exit early (sub-problems that skip a phase) spread over the XCDs at
// the grain of one run.  (Giving each XCD one contiguous eighth of the items shares more,
// but left XCDs idle when the skipped sub-problems bunched up: 25 % slower LM iterations.)
// The last n mod (8 XCD_CHUNK) items keep their order.  A bijection on [0, n) for every n.
// xcd_item(b, n) gives each XCD one contiguous range of items instead, for launches where a
// group of items that must share an L2 is longer than a run and no item skips.
__device__ __forceinline__ int xcd_item(int b, int n) {
    const int x = b % N_XCD, q = n / N_XCD, r = n % N_XCD;
    return x * q + (x < r ? x : r) + b / N_XCD;
}
constexpr int XCD_CHUNK = 8;
__device__ __forceinline__ int xcd_chunk_item(int b, int n) {
    const int full = n / (N_XCD * XCD_CHUNK);
    if (b >= full * N_XCD * XCD_CHUNK) return b;
    const int x = b % N_XCD, s = b / N_XCD;
    return ((s / XCD_CHUNK) * N_XCD + x) * XCD_CHUNK + s % XCD_CHUNK;
}
// Sub-pixel re-centring taps per component (written by k_prep): wx, wy, dwx/d delta_x,
// dwy/d delta_y, each SHIFT_NT entries indexed by t + a (t = -a..a)
constexpr int SHIFT_NT = 2 * APX_SHIFT_MAX_A + 1;
constexpr int STAP_STRIDE = 4 * SHIFT_NT;
// b_n table: cubic Hermite nodes (b, db/dn) on [BN_N0, BN_N0 + (BN_COUNT-1)/BN_INV_H]
constexpr double BN_N0 = 0.35;
constexpr double BN_INV_H = 256.0;
constexpr int BN_COUNT = 2600;

// Plan records (uploaded once into the workspace) -------------------------------
struct DImage {
    int H, W, P, c;           // render grid (sub-pixels when up > 1), stamp, half-width
    int EH, EW;               // extended grid (H+2c) x (W+2c)
    int up, Hc, Wc, pad_up;   // sub-pixels per pixel per axis; the image's own pixel grid
    int sub, sky_par;
    double sky_fixed;
    long long pix_off;        // first element in the pixel buffers (Hc x Wc pixels)
    long long ext_off;        // first element in the extended-grid buffers
    long long psf_off;        // first element of the stamp
    double aff[6];            // render-grid pixel -> sky
    double inv[6];            // sky -> render-grid pixel
    double area;              // |det| of the linear part (render-grid pixel area)
    int live;                 // 1: the stamp is a live Moffat model rendered from theta
    int live_par[2];          // theta indices of (n, R_d), -1 = fixed
    int pad_live;
    double live_fixed[2];
    long long live_off;       // into psf_live: K, dK/dn, dK/dR_d (3 P^2 floats)
    long long fft_off;        // FFT mode: into fft_spec (2 slots of FFT_T^2), -1 = none
    long long sep_off;        // rank-one stamp K_uv = a_u b_v: into psf_sep (a, then b), -1 = none
};

struct DComp {
    int type, image;
    int box[4];               // clipped window y0, x0, y1, x1 (extended-grid coords); with
                              // re-centring, the support of the shifted component (sbox
                              // grown by the interpolation half-width, clipped)
    int sbox[4];              // where the component is sampled (the clipped window)
    int par[7];
    int group;                // Jacobian group, -1 when the component has no free parameter
    int col[7];               // column of local parameter k inside its group, -1 = fixed
    int sub, pad;
    long long aoff;           // adaptive mode: first entry of the window in the per-pixel arrays
    double fixed[7];
};

// Per-call component constants (written by k_prep from theta)
struct CompConst {
    double x0, y0;            // Sersic centre (sky frame); point: pixel position
    double cs_d, sn_d, q_d;   // FP64 copies for the within-k-Re test
    double iq_d;              // 1 / q (FP64 profile)
    double kre;               // k * Re
    double h_d, A_d, B_d;     // t = exp2(g log2 R^2 - h), I = exp2(A - B t)
    double g_d;               // 0.5 / n
    double F64;               // point-source flux (FP64)
    float cs, sn, iq;         // cos PA, sin PA, 1/q
    float g;                  // 0.5 / n
    float b, bp, n, re, q;    // b_n, db_n/dn and raw parameters (derivatives)
    float F;                  // point-source flux
    int valid;                // parameters inside the model domain
    int pad;
};

struct DGroup {               // columns sharing one window on one image
    int image, type, ncols, sub;
    int iy0, ix0, ih, iw;     // input box (window), extended render-grid coords
    int oy0, ox0, oh, ow;     // output box (window dilated by c, clipped to the image), in
                              // image pixels (render-grid box / up, rounded outward)
    int comp_begin, comp_end; // into group_comps
    int col_begin;            // global id of column 0
    int tile_begin, ntiles;   // RT tiles of the input box (deriv / grad)
    long long d_off, j_off;   // element offsets into the D and J buffers
    long long gp_off;         // offset of the gradient partials (ncols * ntiles)
};

struct DCol { int group, comp, local, par; };

struct RTile { int a, y0, x0, pad; };         // a = image (render) or group (deriv/grad)

struct ConvJob {
    long long in_off, out_off;                // element offsets of channel 0
    long long in_cs, out_cs;                  // channel strides
    int in_y0, in_x0, in_h, in_w;             // input rectangle (zero outside)
    int out_y0, out_x0, out_h, out_w;         // output rectangle
    int image, group, ntx, shape;             // shape: output tile shape (tile_th/tile_tw)
    int in_src;                               // input: 0 derivative images, 1 the model S
    int kslot[2];                             // stamp of channel 0 / 1 on live-PSF images:
                                              // 0 K, 1 dK/dn, 2 dK/dR_d
    int gram_part;                            // 1: the columns' sum w r J and sum w J come
                                              // from k_gram4; the epilogue skips them
};
struct ConvItem { int job, ch, ty, tx; };

struct DPair {
    int g, h, image, sub;
    int y0, x0, y1, x1;       // intersection of the two output boxes
};
// one tile pair over stages [s0, s1) of the pair's box (stage s: row y0 + s / nxs, pixels
// x0 + (s % nxs) KC ... of that row, nxs = ceil((x1 - x0) / KC))
struct PairItem { int pair, ta, tb, s0, s1, pad; long long out_off; };
// The J^T W J of a narrow group with itself (at most GRAM4_MAX_T tiles of 4 columns) over one
// K-slice, by 4 x 4 FP64 MFMA blocks: item.ta = the group's 4-column tiles; the partial is
// every tile pair (a <= b, row-major over the upper triangle) as a 4 x 4 block.
constexpr int GRAM4_MAX_T = 9;

// Adaptive integration: the Sersic windows cut into chunks of up to ADAPT_CHUNK pixels
// (row-major window order); a pixel that needs sub-pixels is appended to the refine list.
constexpr int ADAPT_CHUNK = 256;
struct AChunk { int comp, start; };
struct ARef { int comp, idx; };

struct DSub {
    int p0, n;
    long long a_off;
    int large, flag_off;      // flag_off: 2 x blocks of sflag
    int diag_idx, pad;        // large: slot in chol_diag (the latest factored diagonal block)
};

// Per-sub-problem LM scratch flags
struct LMFlags {
    int chol_done;            // factorisation succeeded this iteration
    int chol_fail;            // current attempt failed
    int trial_bad;            // trial parameters outside the domain
    int skip;                 // 1: sub-problem skips the current render/phase
    int subst_fail;           // a substitution hand-off wait ran out this iteration
    int rhs_folded;           // the forward substitution ran inside the first factorisation
    int adopted;              // this iteration's step is the one solved ahead (see LMSpec)
};

// Step solved ahead (large sub-problems): while an iteration factors A + lambda D, the same
// launches also factor A + lambda' D with lambda' = min(UP lambda, max), the damping the next
// iteration starts from if this trial is rejected (same A, same D).  The next iteration
// adopts that solution, with its retries, instead of solving again.
struct LMSpec {
    double lam_start;         // lambda' the solve started from
    double lam_final;         // lambda after its own retries
    double pred;              // h^T (lambda D h + g) of its step
    int valid, done, retries, pad;
};

// Launch-time views of the workspace ----------------------------------------------
struct Plan {
    int n_images, n_comps, n_par, n_sub, n_groups, n_cols;
    int s, rule, mode, objective;
    int shift, shift_a;       // re-centring: APX_SHIFT_*, interpolation half-width a (0: none)
    double k_re;
    float node_o[MAX_NODES_1D], node_w[MAX_NODES_1D];
    double node_od[MAX_NODES_1D], node_wd[MAX_NODES_1D];

    const DImage* images;
    const DComp* comps;
    const DGroup* groups;
    const DCol* cols;
    const DSub* subs;
    const int* group_comps;
    const float* psf;         // caller's stamps
    float* psf_flip;          // flipped stamps (adjoint)
    float* psf_live;          // live-PSF stamps and their derivatives (3 P^2 per live image)
    double* psf64;            // every stamp in FP64 (objective convolution)
    float2* fft_spec;         // FFT mode: stamp spectra (K, flipped K) per image
    const float2* fft_tw;     // [FFT_T]: exp(-2 pi i m / FFT_T)

    // render tiles with component CSR
    const RTile* rtiles; int n_rtiles;
    const int* rtile_off; const int* rtile_comps;
    // deriv/grad tiles
    const RTile* gtiles; int n_gtiles;

    // buffers
    CompConst* cc;
    double* stap;             // [n_comps * STAP_STRIDE] re-centring taps (shift != 0)
    float* S;                 // extended grid (render, FP32 objective)
    double* S64;              // extended grid (render, FP64 objective)
    float* Abar;              // extended grid adjoint
    float* rbuf;              // residual d - m (FP32)
    float* D;                 // derivative images
    float* J;                 // Jacobian blocks
    double* fwd_part;         // 3 per FWD conv item: sum w r^2, sum w r, sum w
    double* img_sum;          // 3 per image
    double* jcol_part;        // 2 per JCOL item: sum w r J, sum w J
    double* col_sum;          // 2 per column
    double* pair_part;        // pair tiles
    double* grad_part;        // gradient partials (per group: ncols x ntiles)
    double* grad_col;         // per column
    double* A;                // internal J^T W J blocks (per sub)
    double* gvec;             // internal J^T W r [n_par]
    double* M;                // Cholesky factor (per sub)
    double* Ddiag;            // damping diagonal [n_par]
    double* hvec;             // step [n_par]
    double* yvec;             // substitution right-hand side [n_par]
    double* theta_trial;      // [n_par]
    LMFlags* lmf;             // [n_sub]
    int* sflag;               // substitution hand-off flags (per large sub: forward, backward blocks)
    double* chol_diag;        // per large sub: a factored diagonal block on its way into M
    LMSpec* spec;             // [n_sub] the step solved ahead
    long long a_total;        // entries of M per copy (the solve-ahead copy follows)
    int n_sflag, n_large;     // per copy: substitution flags, large sub-problems
    int* sticky;              // device error flags
    double* sky_val;          // [n_images] sky of each image at the current theta
    const int* par_sub;       // [n_par] sub-problem of each theta index (-1: none)
    const double* bn_tab;     // [2 * BN_COUNT]: b_n, db_n/dn at the table nodes
    const double* ptab;       // [PTAB_N]: the FP64 render's 2^x / log2 table (sersic64.h)
    const float* psf_sep;     // factors of rank-one stamps (2 P per such image)

    // adaptive integration (mode APX_MODE_ADAPTIVE, tolerance k_re)
    const double* agl;        // Gauss-Legendre offsets / weights on [-1/2, 1/2]: o3 w3 o5 w5 o7 w7
    const AChunk* achunks; int n_achunks;
    const int* acomp_chunk;   // [n_comps + 1]: chunks of each component (CSR)
    double* apart;            // [n_achunks] window-flux partials
    double* ae;               // [n_comps] error budget e = tol F / N
    double* av0;              // [n_apix] profile at the pixel centre
    double* aval;             // [n_apix] pixel value (mean of the profile, before the area)
    int* aneed;               // [n_apix] per refine entry: mask of the sub-pixels taken at 7 x 7
    int* acode;               // [n_apix] 0 centre, 1 3 x 3, -1 - r: refine entry r
    ARef* aref;               // [n_apix] refine list
    float* adval;             // [7 n_apix] derivatives of refined pixels (before the area)
    int* acount;              // refine-list length
    long long n_apix;

    long long n_pix, n_ext;
    // bound of a substitution hand-off wait in polls; < 0: every wait takes its flag as never
    // raised and gives up after -wait_spin_max polls (forces the give-up path from the host)
    int wait_spin_max;
};

// entries of the FP64 render's 2^x / log2 table (layout in sersic64.h)
constexpr int PTAB_N = 192;

// default bound of a substitution hand-off wait (polls of ~64 cycles each)
constexpr int SUBST_SPIN_MAX = 1 << 22;

// Sticky flag bits
constexpr int FLAG_DOMAIN = 1, FLAG_NONFINITE = 2, FLAG_STALL = 4;
// live Moffat PSF domain
constexpr double PSF_N_MIN = 0.2, PSF_N_MAX = 20.0, PSF_RD_MIN = 0.05, PSF_RD_MAX = 1e3;
constexpr int GROUP_PSF = 2;                   // DGroup.type of the live-PSF columns of an image

// The buffers of the damped solve for copy `which` (0: this iteration's lambda, 1: the
// solve-ahead lambda'): M, yvec, hvec, the hand-off flags, the factorisation flags and the
// diagonal-block slots of copy 1 follow those of copy 0.
__device__ __forceinline__ Plan solve_view(const Plan& p, int which) {
    Plan q = p;
    if (which) {
        q.M += p.a_total;
        q.yvec += p.n_par;
        q.hvec += p.n_par;
        q.sflag += p.n_sflag;
        q.lmf += p.n_sub;
        q.chol_diag += (long long)p.n_large * CHOL_NB * CHOL_NB;
    }
    return q;
}

// skip_mode of the launchers: 0 none, 1 sub-problems without a valid trial (the trial
// render), 2 sub-problems that keep their Jacobian (lm[sub].need_jac == 0)
__device__ __forceinline__ bool sub_skipped(const Plan& p, int sub, int mode, const apx_lm_state* lm) {
    if (mode == 1) return p.lmf[sub].chol_done == 0 || p.lmf[sub].trial_bad != 0;
    if (mode == 2) return lm[sub].need_jac == 0;
    return false;
}

// Launchers (each returns hipGetLastError()) ----------------------------------------
// k_model.hip
hipError_t launch_prep(const Plan& p, const double* theta, int lm_trial, hipStream_t st);
// skip_mode: 0 none, 1 skip sub-problems without a valid trial, 2 skip those that keep J
hipError_t launch_render_mode(const Plan& p, int skip_mode, const apx_lm_state* lm, hipStream_t st);
hipError_t launch_render64(const Plan& p, int skip_mode, const apx_lm_state* lm, hipStream_t st);
hipError_t launch_deriv(const Plan& p, const apx_lm_state* lm, hipStream_t st);
hipError_t launch_grad_tiles(const Plan& p, hipStream_t st);
hipError_t launch_flip_psf(const Plan& p, hipStream_t st);

// k_adapt.hip: error budgets, choices and values of the adaptive integration at the
// current theta (after launch_prep); want_grad also forms the refined pixels' derivatives
hipError_t launch_adapt(const Plan& p, int skip_mode, const apx_lm_state* lm, int want_grad, hipStream_t st);
// per image: img_sum[3 k + 1] = -sum(seed) / 2, so that the image-sum terms of the gradient
// assembly (weight -2) give the seed's sum (the sky column of a vector-Jacobian product)
hipError_t launch_seed_sums(const Plan& p, const float* seed, double* part, hipStream_t st);

// k_conv_*.hip
enum ConvKind { CONV_FWD = 0, CONV_JCOL = 1, CONV_ADJ = 2, CONV_JCOL_PSF = 3 };   // PSF: live-PSF columns
struct ConvLaunch {
    const ConvJob* jobs;
    const ConvItem* items;
    int item_begin, item_count, P, shape;
    const int4* pairs;        // FFT mode: items sharing one transform (second -1 = none), their sub-problem
    int pair_begin, pair_count;
};
struct ConvIO {
    const float* in;          // input buffer base (FWD, JCOL)
    const float* in_s;        // JCOL jobs with in_src = 1: the pre-convolution model S
    const double* in64;       // input buffer base (FWD, FP64 objective)
    float* out;               // output buffer base (FWD: optional model)
    const float* data;        // FWD: data (null = no residual / partials)
    const float* weight;      // FWD, JCOL (null = no partials), ADJ
    const float* seed;        // ADJ: the seed itself (vector-Jacobian product) instead of -2 w r
    double* part;             // per-item partials
    int skip_mode;            // as launch_render_mode
    const apx_lm_state* lm;
};
hipError_t launch_conv_fwd(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st);
hipError_t launch_conv_fwd64(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st);
hipError_t launch_conv_jcol(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st);
hipError_t launch_conv_adj(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st);
// Jacobian-column convolution as two 1-D passes (jobs of shape SHAPE_SEP)
hipError_t launch_conv_sep(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st);
// k_conv_fft.hip: FFT mode (kinds FWD with the FP32 objective, JCOL, ADJ)
hipError_t launch_conv_fft(const Plan& p, int kind, const ConvLaunch& L, const ConvIO& io, hipStream_t st);
hipError_t launch_fft_stamps(const Plan& p, int live_only, hipStream_t st);

// k_jtwj.hip
struct PairLaunch { const DPair* pairs; const PairItem* items; int n_items; int tm; };
// Workgroups of k_pair<tm> resident per compute unit (0 if the runtime cannot say).
int pair_blocks_per_cu(int tm);
hipError_t launch_pairs(const Plan& p, const PairLaunch& L, const float* weight,
                        const apx_lm_state* lm, hipStream_t st);
// L.items: Gram items with L.tm = the number of 4-column tiles (1..GRAM4_MAX_T)
hipError_t launch_gram4(const Plan& p, const PairLaunch& L, const float* weight,
                        const apx_lm_state* lm, hipStream_t st);
struct SegSum {
    const double* src; int stride, comp;
    const int* seg; const int* idx; const double* wts;
    int n_seg;
    double* out; int ostride, ocomp;
    double scale;
    const int* seg_sub; const apx_lm_state* lm;
    int ncomp;                                // components comp .. comp + ncomp - 1 (0: one)
};
hipError_t launch_segsum(const SegSum& a, hipStream_t st);
struct AsmA {
    const long long* ent_off; const int* ent_sub; const int* ent_row; const int* ent_col;
    const long long* ent_src;
    long long n_ent;
    const double* src;
    const DSub* subs;
    double* out;
    const apx_lm_state* lm;
};
hipError_t launch_assemble_A(const AsmA& a, hipStream_t st);
hipError_t launch_fill(double* x, long long n, double v, hipStream_t st);
hipError_t launch_fill_f(float* x, long long n, float v, hipStream_t st);
hipError_t launch_jscatter(const Plan& p, const int* par_off, const int* par_cols,
                           const int* par_sky_off, const int* par_sky, float* Jd, long long ldJ,
                           hipStream_t st);
hipError_t launch_chi2_check(const double* chi2, int n, int* sticky, hipStream_t st);

// k_lm.hip
hipError_t launch_lm_begin(const Plan& p, apx_lm_state* lm, hipStream_t st);
// large sub-problems whose step was solved ahead take it (step, pred, lambda, retries)
hipError_t launch_lm_begin_adopt(const Plan& p, apx_lm_state* lm, hipStream_t st);
hipError_t launch_lm_init(const Plan& p, const double* chi2_sub, apx_lm_state* lm, hipStream_t st);
hipError_t launch_chol_small(const Plan& p, const int* small_subs, int n_small, int nmax,
                             apx_lm_state* lm, hipStream_t st);
hipError_t launch_chol_large(const Plan& p, int sub, int n, apx_lm_state* lm, hipStream_t st);
hipError_t launch_chol_reset(const Plan& p, int sub, hipStream_t st);
hipError_t launch_chol_blocks(const Plan& p, int sub, int n, hipStream_t st);
hipError_t launch_lm_trial(const Plan& p, const double* theta, apx_lm_state* lm, hipStream_t st);
hipError_t launch_lm_accept(const Plan& p, const double* chi2_trial, double* theta,
                            apx_lm_state* lm, hipStream_t st);

// k_cov.hip
// factor / forward_only: F = L^{-T} (A = L L^T) instead of A^{-1}, so that F F^T = A^{-1}
hipError_t launch_cov_small(const Plan& p, const int* small_subs, int n_small, int nmax, double* cov,
                            int factor, hipStream_t st);
hipError_t launch_cov_fill(const Plan& p, int sub, int n, hipStream_t st);
hipError_t launch_cov_cols(const Plan& p, int sub, int n, double* cov, int forward_only, hipStream_t st);
hipError_t launch_cov_transpose(const Plan& p, int sub, int n, double* X, hipStream_t st);

// k_hmc.hip: the vector steps of Hamiltonian Monte Carlo around the gradient passes
struct HmcIO {
    double* theta;            // [n_par] current point (in/out)
    double* theta0;           // [n_par] start of the trajectory
    double* r;                // [n_par] whitened momenta
    double* grad_cur;         // [n_par] d chi2 / d theta at theta0 (start of the next trajectory)
    double* grad_new;         // [n_par] d chi2 / d theta at the latest leapfrog point
    double* chi2_cur;         // [n_sub]
    double* chi2_new;         // [n_sub]
    double* H0;               // [n_sub]
    const double* z;          // [n_samples * n_par] standard normals
    const double* u;          // [n_samples * n_sub] uniforms
    double* samples;          // [n_samples * n_par]
    double* stats;            // [n_samples * n_sub * 3]: accepted, H0, H1
};
hipError_t launch_hmc_transpose(const Plan& p, const double* F, double* Ft, hipStream_t st);
// out[j] += coef * (M_s^T v_s)[j - p0_s] for every theta index j of sub-problem s; nothing
// when skip is given and *skip != 0
hipError_t launch_hmc_matvec(const Plan& p, const double* M, const double* v, double* out, double coef,
                             hipStream_t st, const int* skip = nullptr);
hipError_t launch_hmc_begin(const Plan& p, const HmcIO& h, long long i, hipStream_t st);
hipError_t launch_hmc_accept(const Plan& p, const HmcIO& h, long long i, hipStream_t st);
hipError_t launch_clear_trial_flags(const Plan& p, hipStream_t st);

// NUTS tree state of one transition on the device.  The host issues the launches of a whole
// doubling (every leaf, subtree merge and U-turn test of a tree of that depth) without
// waiting; the kernels act only where the tree in progress has not stopped, and the host
// reads this struct once per doubling to decide whether to double again.
struct NutsDev {
    double log_slice;                       // log u0 - H0
    double H0;                              // energy at the start of the transition
    double alpha;                           // sum of min(1, exp(H0 - H)) over the doubling's leaves
    long long cnt;                          // points in the slice, whole trajectory
    long long c[APX_NUTS_MAX_DEPTH + 1];    // points in the slice of the subtree in progress, by level
    int gate[APX_NUTS_MAX_DEPTH + 1];       // level j: its second half was built
    int stop;                               // the doubling in progress stopped (divergence or U-turn)
    int one;                                // 1: the entry flag of a doubling's tree
    int take;                               // the last merge took its second half's proposal
    int accept;                             // the last doubling's proposal became the sample
    int k;                                  // next uniform of the transition
    int steps, divergent, n_alpha;
};
// Up to 7 device vectors of n_par doubles copied dst[i] <- src[i] under one condition.
struct NutsCopy {
    double* dst[7];
    const double* src[7];
    int n;
};
// H0 and the slice from the start point (chi2 [n_sub], momenta r), k = 1, counters cleared
hipError_t launch_nuts_start(const Plan& p, NutsDev* d, const double* chi2, const double* r, const double* u,
                             hipStream_t st);
// a doubling begins: its direction draw is consumed, stop and the acceptance statistic cleared
hipError_t launch_nuts_doubling(NutsDev* d, hipStream_t st);
// the copies when *flag == want
hipError_t launch_nuts_copy(const int* flag, int want, const NutsCopy& c, long long n, hipStream_t st);
// a leaf's energy (clears the domain flags) and, unless stopped, its slice count and tests
hipError_t launch_nuts_leaf(const Plan& p, NutsDev* d, const double* chi2, const double* r, hipStream_t st);
// level j after its first half: when *entry, copies (inner, outer, proposal) and c[j] = c[j-1];
// gate[j] = !stop
hipError_t launch_nuts_level(NutsDev* d, int j, const int* entry, const NutsCopy& c, long long n, hipStream_t st);
// level j after its second half, when gate[j]: draw, proposal (copies `prop` when taken),
// c[j] += c[j-1], outer end (copies `outer`)
hipError_t launch_nuts_merge(NutsDev* d, int j, const double* u, const NutsCopy& prop, const NutsCopy& outer,
                             long long n, hipStream_t st);
// end of a doubling of depth `depth`: the trajectory's end (copies `edge`), and unless
// stopped the draw that may make the doubling's proposal the sample (copies `sample`);
// cnt += c[depth]
hipError_t launch_nuts_top(NutsDev* d, int depth, const double* u, const NutsCopy& edge, const NutsCopy& sample,
                           long long n, hipStream_t st);
// U-turn test of ends (tm, rm), (tp, rp) with velocities vm = F rm, vp = F rp: when
// *flag == want and (tp - tm) . vm < 0 or (tp - tm) . vp < 0, stop
hipError_t launch_nuts_uturn(const Plan& p, const double* tm, const double* tp, const double* vm,
                             const double* vp, NutsDev* d, const int* flag, int want, hipStream_t st);

}  // namespace apx
