// Host side of the apx C ABI: descriptor validation, launch-plan construction
// (tiles, component lists, Jacobian groups and pair lists, ordered-reduction tables),
// workspace layout and the launch sequences of the hot-path entry points.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "apx_internal.h"

using namespace apx;

struct apx_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int tiles = APX_TILES_AUTOTUNE;                     // tile-shape policy for new problems
    std::map<int, std::array<double, 4>> tile_us;       // (kernel, P) -> measured us per tile
    void* tune_mem = nullptr;                           // autotuner scratch (allocated once)
    size_t tune_bytes = 0;
    int pair_slots = 0;                                 // resident k_pair<64> workgroups
};

// ------------------------------------------------------------ library scratch
// Device memory for callers that cannot allocate (code under graph capture, serving loops,
// harnesses that forbid hipMalloc): one array per GPU the library runs on, held until the
// process ends.  A problem bound to it (apx_problem_bind_scratch) keeps its plan tables and
// every per-call buffer there, as it would in a caller workspace.  In host code the array's
// name is only a stand-in: its device address comes from hipGetSymbolAddress, looked up
// once per device when the first context of that device is created.
static constexpr size_t APX_SCRATCH_BYTES = size_t(64) << 20;
static constexpr int APX_SCRATCH_DEVICES = 64;
static __device__ __align__(256) char scratch[APX_SCRATCH_BYTES];

namespace {
struct ScratchSlot {
    bool looked_up = false;
    hipError_t status = hipSuccess;
    void* ptr = nullptr;          // device address of `scratch` on this device
    uint64_t generation = 0;      // bumped by every binding; a problem keeps the value it bound
};
std::mutex g_scratch_mu;
ScratchSlot g_scratch[APX_SCRATCH_DEVICES];

// with `device` current: look the array's address up once
void scratch_lookup(int device) {
    if (device < 0 || device >= APX_SCRATCH_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchSlot& sl = g_scratch[device];
    if (sl.looked_up) return;
    sl.looked_up = true;
    void* ptr = nullptr;
    sl.status = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    sl.ptr = sl.status == hipSuccess ? ptr : nullptr;
}
}  // namespace

namespace {

struct PRange { int P, shape, begin, count, pair_begin, pair_count; };

template <class T>
struct DevArr {
    const std::vector<T>* host = nullptr;
    size_t off = 0;   // byte offset in the workspace
};

struct Layout {
    size_t total = 0;
    size_t take(size_t bytes) {
        size_t o = (total + 255) & ~size_t(255);
        total = o + ((bytes + 255) & ~size_t(255));
        return o;
    }
};

}  // namespace

struct apx_problem {
    apx_ctx* ctx = nullptr;
    int n_images = 0, n_comps = 0, n_par = 0, n_sub = 0;
    int s = 3, rule = 0, mode = 0, objective = 0, conv_mode = 0;
    int shift = 0, shift_a = 0;                   // re-centring method, interpolation half-width
    double k_re = 0.0;
    const float* psf = nullptr;

    std::vector<DImage> images;
    std::vector<DComp> comps;
    std::vector<DGroup> groups;
    std::vector<DCol> cols;
    std::vector<DSub> subs;
    std::vector<int> group_comps;
    std::vector<RTile> rtiles, gtiles;
    std::vector<int> rtile_off, rtile_comps;
    std::vector<ConvJob> fwd_jobs, jcol_jobs, adj_jobs, psf_jobs;
    std::vector<ConvItem> fwd_items, jcol_items, adj_items, psf_items;
    std::vector<PRange> fwd_ranges, jcol_ranges, adj_ranges, psf_ranges;
    std::vector<int4> fwd_pairs, jcol_pairs, adj_pairs;    // FFT mode: items per transform (+ sub-problem)
    long long n_fft_spec = 0;                     // FFT mode: stamp spectra (complex entries)
    int n_fft_images = 0;
    bool fft_fixed_ready = false;                 // spectra of fixed stamps computed
    int fft_live = -1;                            // images with spectra of live stamps (-1: not counted yet)
    std::vector<float> fft_tw;                    // exp(-2 pi i m / FFT_T) as (re, im)
    long long n_live = 0;                         // floats of live-PSF stamps (3 P^2 each)
    bool has_live_cols = false;                   // some live PSF has a free parameter
    std::vector<DPair> pairs;
    std::vector<PairItem> pitems64, pitems16;
    std::vector<PairItem> gitems;                 // 4 x 4-block Gram items, sorted by tile count
    int gram_begin[GRAM4_MAX_T + 2] = {};         // items of tile count t: [gram_begin[t], gram_begin[t + 1])
    // reduction tables
    std::vector<int> img_seg, img_idx;            // FWD items of each image
    std::vector<int> col_seg, col_idx;            // JCOL items of each column
    std::vector<int> gcol_seg;                    // grad partials of each column (contiguous)
    std::vector<int> chi_seg, chi_idx;            // img_sum entries of each sub
    std::vector<int> g_seg, g_idx, g_sub;         // J^T W r sources per theta index
    std::vector<double> g_w;
    std::vector<int> gr_seg, gr_idx;              // gradient sources per theta index
    std::vector<double> gr_w;
    std::vector<long long> a_off_csr, a_src;      // A assembly
    std::vector<int> a_sub, a_row, a_col;
    std::vector<int> par_sub, par_off, par_cols, par_sky_off, par_sky;
    std::vector<int> small_subs, large_subs;
    int n_sflag = 0;                              // substitution hand-off flags
    std::vector<int> theta_subs;                  // sub of each theta-assembly segment
    int nmax_small = 0;
    std::vector<float> node_o, node_w;
    std::vector<double> node_od, node_wd;
    std::vector<double> bn_tab;
    std::vector<double> ptab;                     // FP64 render: 2^x / log2 table
    std::vector<float> psf_sep;                   // factors of rank-one stamps (a, then b)
    std::vector<double> agl;                      // adaptive: GL 3/5/7 offsets and weights
    std::vector<AChunk> achunks;
    std::vector<int> acomp_chunk;
    long long n_apix = 0;

    long long n_pix = 0, n_ext = 0, n_d = 0, n_j = 0, n_pairpart = 0, n_gradpart = 0, a_total = 0;
    long long n_psf = 0;

    // workspace
    char* ws = nullptr;
    uint64_t ws_bytes = 0;
    bool bound = false;
    bool on_scratch = false;         // bound to the library scratch of ctx->device
    uint64_t scratch_gen = 0;        // the scratch binding this problem made
    Layout L;
    std::map<std::string, size_t> off;
    Plan plan{};
    double* asrc = nullptr;          // [pair_part | col_sum | grad_col | img_sum]
    long long asrc_col = 0, asrc_gcol = 0, asrc_img = 0;
    double* chi2_sub = nullptr;      // [n_sub]
    double* chi2_trial = nullptr;    // [n_sub]

    // kernel timing
    bool timing = false;
    uint32_t timing_mask = 0;        // classes recorded while timing
    bool capturing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_recs;   // (class, index of start event)
    // timing inside a captured LM iteration: the events recorded during capture become
    // event-record nodes; each replay points them at fresh events of ev_pool
    struct CapMark { int klass; hipEvent_t ev[2]; hipGraphNode_t node[2]; };
    std::vector<CapMark> cap_marks;
    std::string cap_error;                       // first failure of a mark during capture

    // graph cache for apx_lm_run
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    const void* gkey[4] = {nullptr, nullptr, nullptr, nullptr};
    uint32_t gmask = 0;                          // timing classes captured into the graph
};

// ------------------------------------------------------------------------ helpers
static apx_status fail(apx_ctx* c, apx_status s, const std::string& m) {
    if (c) c->err = m;
    return s;
}

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            return fail(P->ctx, APX_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

static void gauss_legendre(int s, std::vector<double>& x, std::vector<double>& w) {
    x.assign(s, 0.0);
    w.assign(s, 0.0);
    for (int i = 0; i < s; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (s + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= s; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            double pp = s * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (std::fabs(z - z1) < 1e-16) {
                // recompute derivative at the converged node
                p1 = 1.0; p2 = 0.0;
                for (int j = 1; j <= s; ++j) {
                    double p3 = p2;
                    p2 = p1;
                    p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
                }
                pp = s * (z * p1 - p2) / (z * z - 1.0);
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
                break;
            }
        }
    }
    std::sort(x.begin(), x.end());
    // weights are symmetric; re-pair after sorting
    std::vector<double> w2(s);
    for (int i = 0; i < s; ++i) {
        double z = x[i], p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= s; ++j) {
            double p3 = p2;
            p2 = p1;
            p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        double pp = s * (z * p1 - p2) / (z * z - 1.0);
        w2[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
    w = w2;
}

static inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------- tile-shape choice
// Kernel keys of the cost table: the three convolution epilogues, FWD split by precision.
enum { TUNE_FWD32 = 0, TUNE_JCOL = 1, TUNE_ADJ = 2, TUNE_FWD64 = 3 };

// Operation-count model of one tile: P^2 FMAs and an epilogue per output, the staged input
// tile with its halo, and a fixed per-workgroup cost (in FMA-lane units).
static double tile_model(int P, int shape) {
    const double th = tile_th(shape), tw = tile_tw(shape);
    return th * tw * ((double)P * P + 10.0) + 8.0 * (th + P - 1) * (tw + P - 1) + 3000.0;
}

// The autotuner: time every tile shape of one convolution kernel at PSF size P on a
// synthetic 256 x 256 job of 32 channels (zero data, so timings do not depend on values),
// in scratch memory of the context, and keep microseconds per tile (best of 3 timed pairs
// of launches after 2 warm-up launches).  Synchronous on the context stream.
static constexpr int TUNE_H = 256, TUNE_CH = 32, TUNE_MAXP = 63;
static bool tune_kernel(apx_ctx* C, int key, int P, std::array<double, 4>& us) {
    const int c = (P - 1) / 2, EH = TUNE_H + 2 * c;
    const int EMAX = TUNE_H + TUNE_MAXP - 1;
    const long long npx = (long long)TUNE_H * TUNE_H, next = (long long)EMAX * EMAX;
    const int max_items = ceil_div(EMAX, 16) * ceil_div(EMAX, 32) * TUNE_CH;   // smallest tile, widest output
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
    const size_t o_img = take(sizeof(DImage)), o_job = take(sizeof(ConvJob));
    const size_t o_items = take(sizeof(ConvItem) * max_items), o_psf = take(sizeof(float) * TUNE_MAXP * TUNE_MAXP);
    const size_t o_psf64 = take(sizeof(double) * TUNE_MAXP * TUNE_MAXP);
    const size_t o_sky = take(sizeof(double)), o_r = take(sizeof(float) * npx), o_w = take(sizeof(float) * npx);
    const size_t o_d = take(sizeof(float) * npx), o_in = take(sizeof(float) * next * TUNE_CH);
    const size_t o_in64 = take(sizeof(double) * next), o_out = take(sizeof(float) * (size_t)TUNE_CH * next);
    const size_t o_part = take(sizeof(double) * 3 * max_items);
    if (!C->tune_mem) {
        if (hipMalloc(&C->tune_mem, off) != hipSuccess) { C->tune_mem = nullptr; return false; }
        C->tune_bytes = off;
        if (hipMemset(C->tune_mem, 0, off) != hipSuccess) return false;
    }
    char* base = (char*)C->tune_mem;
    hipStream_t st = C->stream;
    DImage im{};
    im.H = im.W = TUNE_H; im.P = P; im.c = c; im.EH = im.EW = EH;
    im.up = 1; im.Hc = im.Wc = TUNE_H;
    im.area = 1.0;
    if (hipMemcpy(base + o_img, &im, sizeof im, hipMemcpyHostToDevice) != hipSuccess) return false;
    Plan p{};
    p.n_images = 1;
    p.images = (const DImage*)(base + o_img);
    // every stamp pointer a kernel may read (FP32, flipped, FP64) points at zeroed scratch
    p.psf = (const float*)(base + o_psf);
    p.psf_flip = (float*)(base + o_psf);
    p.psf_live = (float*)(base + o_psf);
    p.psf64 = (double*)(base + o_psf64);
    p.sky_val = (double*)(base + o_sky);
    p.rbuf = (float*)(base + o_r);
    ConvIO io{};
    io.in = (const float*)(base + o_in);
    io.in64 = (const double*)(base + o_in64);
    io.out = (float*)(base + o_out);
    io.weight = (const float*)(base + o_w);
    io.part = (double*)(base + o_part);
    const bool fwd = key == TUNE_FWD32 || key == TUNE_FWD64;
    if (fwd) { io.data = (const float*)(base + o_d); io.out = nullptr; }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return false;
    bool ok = true;
    for (int shape = 0; shape < N_TILE_SHAPES && ok; ++shape) {
        ConvJob jb{};
        if (key == TUNE_ADJ) {
            jb.in_y0 = 0; jb.in_x0 = 0; jb.in_h = TUNE_H; jb.in_w = TUNE_H;
            jb.out_y0 = -c; jb.out_x0 = -c; jb.out_h = EH; jb.out_w = EH;
        } else {
            jb.in_y0 = -c; jb.in_x0 = -c; jb.in_h = EH; jb.in_w = EH;
            jb.out_y0 = 0; jb.out_x0 = 0; jb.out_h = TUNE_H; jb.out_w = TUNE_H;
            if (key == TUNE_JCOL) { jb.in_cs = next; jb.out_cs = npx; }
        }
        jb.shape = shape;
        std::vector<ConvItem> items;
        const int ny = ceil_div(jb.out_h, tile_th(shape)), nx = ceil_div(jb.out_w, tile_tw(shape));
        for (int ch = 0; ch < TUNE_CH; ++ch)
            for (int ty = 0; ty < ny; ++ty)
                for (int tx = 0; tx < nx; ++tx) items.push_back(ConvItem{0, ch, ty, tx});
        if ((int)items.size() > max_items ||
            hipMemcpy(base + o_job, &jb, sizeof jb, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(base + o_items, items.data(), sizeof(ConvItem) * items.size(), hipMemcpyHostToDevice) != hipSuccess) {
            ok = false;
            break;
        }
        ConvLaunch L{(const ConvJob*)(base + o_job), (const ConvItem*)(base + o_items), 0, (int)items.size(), P, shape};
        auto launch = [&]() {
            switch (key) {
                case TUNE_FWD32: return launch_conv_fwd(p, L, io, st);
                case TUNE_FWD64: return launch_conv_fwd64(p, L, io, st);
                case TUNE_JCOL: return launch_conv_jcol(p, L, io, st);
                default: return launch_conv_adj(p, L, io, st);
            }
        };
        double best = 1e300;
        for (int rep = 0; rep < 5 && ok; ++rep) {
            if (rep >= 2) ok = hipEventRecord(e0, st) == hipSuccess;
            ok = ok && launch() == hipSuccess && launch() == hipSuccess;
            if (rep >= 2 && ok) {
                float ms = 0.f;
                ok = hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                best = std::min(best, (double)ms * 1e3 / (2.0 * items.size()));
            }
        }
        us[shape] = best;
    }
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return ok;
}

// Cost of one tile of each shape for kernel `key` at PSF size P under the context's policy.
static std::array<double, 4> tile_costs(apx_ctx* C, int key, int P) {
    std::array<double, 4> cost;
    if (C->tiles == APX_TILES_AUTOTUNE && C->device >= 0) {
        const int k = key * 64 + P;
        auto it = C->tile_us.find(k);
        if (it != C->tile_us.end()) return it->second;
        if (tune_kernel(C, key, P, cost)) {
            C->tile_us[k] = cost;
            return cost;
        }
        (void)hipGetLastError();                        // fall back to the model
    }
    for (int s = 0; s < N_TILE_SHAPES; ++s) cost[s] = tile_model(P, s);
    return cost;
}

// Automatic mode: a job of nch channels with an out_h x out_w output takes FFT tiles when
// its pairs of 128 x 128 transforms (ceil(nch * blocks / 2), blocks of (129 - P)^2 outputs)
// cost less than its direct tiles of the cheapest shape, both by the operation-count model
// (tile_model) with one transform pair at APX_AUTO_FFT_PAIR_COST units.  Calibrated on
// MI355X: over a full Jacobian phase of 4096 cutouts a pair takes as long as 4.7e6 units of
// direct tiles on average, but the whole LM iteration is fastest near 1e6, where all but the
// smallest jobs take FFT tiles: the direct launches left behind are small and bound by their
// latency, not by their operation count.  The model, not the autotuner's timings, decides,
// so the choice and the results do not depend on timing noise.
static bool auto_fft(int P, int out_h, int out_w, int nch) {
    double direct = 1e300;
    for (int s = 0; s < N_TILE_SHAPES; ++s)
        direct = std::min(direct, (double)ceil_div(out_h, tile_th(s)) * ceil_div(out_w, tile_tw(s)) * tile_model(P, s));
    const int B = FFT_T - P + 1;
    const long long blocks = (long long)ceil_div(out_h, B) * ceil_div(out_w, B);
    const double fft = (double)((nch * blocks + 1) / 2) * APX_AUTO_FFT_PAIR_COST;
    return fft < direct * nch;
}

// Workgroups of the 64-wide J^T W J tile kernel resident on the whole device at once; a
// plan-only context takes gfx950's (256 compute units, 3 per unit at the kernel's 134
// registers per lane).
static int pair_slots(apx_ctx* C) {
    if (C->pair_slots > 0) return C->pair_slots;
    int per_cu = 3, n_cu = 256;
    if (C->device >= 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, C->device) == hipSuccess && v > 0)
            n_cu = v;
        else
            (void)hipGetLastError();
        const int b = pair_blocks_per_cu(64);
        if (b > 0) per_cu = b;
    }
    C->pair_slots = per_cu * n_cu;
    return C->pair_slots;
}

// Tile shape of least estimated cost (tiles needed x measured or modelled cost of one tile)
// summed over a group of jobs at one PSF size (outputs h[j] x w[j] with nch[j] channels
// each).  A shape must beat the best lower-indexed (larger) one by more than 3 % to be
// taken: measured costs of near-equal shapes wobble from run to run, and the larger tile
// re-reads less halo.  Every direct job of one kind and PSF size takes this one shape, so a
// phase launches once per PSF size: per-job shapes split a batch of small images into four
// launches per size, each ending in a partly filled round (on 4096 cutouts the FP64 model
// convolutions took 2.34 ms per iteration in 36 launches, 1.82 ms in 9).
static int choose_group_shape(apx_ctx* C, int key, int P, const std::vector<int>& h,
                              const std::vector<int>& w, const std::vector<int>& nch) {
    if (C->tiles >= APX_TILES_FIXED && C->tiles < APX_TILES_FIXED + N_TILE_SHAPES) return C->tiles - APX_TILES_FIXED;
    const std::array<double, 4> cost = tile_costs(C, key, P);
    int best = 0;
    double bc = 1e300;
    for (int s = 0; s < N_TILE_SHAPES; ++s) {
        double v = 0.0;
        for (size_t j = 0; j < h.size(); ++j)
            if (h[j] > 0 && w[j] > 0)
                v += (double)nch[j] * ceil_div(h[j], tile_th(s)) * ceil_div(w[j], tile_tw(s)) * cost[s];
        if (v < 0.97 * bc) { bc = v; best = s; }
    }
    return best;
}

// Regularised lower incomplete gamma P(a, x) by its power series (x < a + 1 here).
static double gammainc_lower_series_host(double a, double x) {
    if (x <= 0.0) return 0.0;
    double sum = 1.0, term = 1.0;
    for (int k = 1; k < 5000; ++k) {
        term *= x / (a + k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return std::exp(a * std::log(x) - x - std::lgamma(a + 1.0)) * sum;
}

// Sersic b_n: the root of P(2n, b) = 1/2, by bracketed Newton from the asymptotic guess.
static double sersic_bn_host(double n) {
    const double a = 2.0 * n;
    double lo = std::max(a - 1.0, 1e-12), hi = a + 0.5;
    double b = a - 1.0 / 3.0 + 4.0 / (405.0 * n) + 46.0 / (25515.0 * n * n);
    if (!(b > lo && b < hi)) b = 0.5 * (lo + hi);
    const double lga = std::lgamma(a);
    for (int it = 0; it < 100; ++it) {
        const double f = gammainc_lower_series_host(a, b) - 0.5;
        if (f > 0.0) hi = b; else lo = b;
        const double fp = std::exp((a - 1.0) * std::log(b) - b - lga);
        double bn = b - f / fp;
        if (!(bn > lo && bn < hi)) bn = 0.5 * (lo + hi);
        const double step = std::fabs(bn - b);
        b = bn;
        if (step <= 1e-15 * b) break;
    }
    return b;
}

// The FP64 render's 2^x / log2 table (layout in sersic64.h), in extended precision and
// rounded once.
static void build_pow2_table(std::vector<double>& tab) {
    tab.resize(PTAB_N);
    for (int j = 0; j < 64; ++j) {
        tab[j] = (double)exp2l((long double)j / 64.0L);
        const long double c = 0.5L + ((long double)j + 0.5L) / 128.0L;
        const double r = (double)(1.0L / c);
        tab[64 + j] = r;
        tab[128 + j] = (double)(-log2l((long double)r));
    }
}

static void build_bn_table(std::vector<double>& tab) {
    tab.resize(2 * BN_COUNT);
    const double hd = 1e-5;
    for (int k = 0; k < BN_COUNT; ++k) {
        const double n = BN_N0 + k / BN_INV_H;
        tab[2 * k] = sersic_bn_host(n);
        tab[2 * k + 1] = (sersic_bn_host(n + hd) - sersic_bn_host(n - hd)) / (2.0 * hd);
    }
}

// Event pair around a launch group when timing is on (never during capture).
struct TimeScope {
    apx_problem* P;
    int klass;
    size_t idx = (size_t)-1;
    TimeScope(apx_problem* P_, int k);
    ~TimeScope();
};

// During capture: an event-record node appended to the captured work by hand (a plain
// event record inside a capture is only a dependency marker); the node's event is a
// placeholder that every replay replaces.  Returns false (and notes why) on any failure.
static bool capture_mark(apx_problem* P, hipEvent_t ev, hipGraphNode_t* node) {
    hipStream_t st = P->ctx->stream;
    hipStreamCaptureStatus cs;
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t* deps = nullptr;
    size_t nd = 0;
    hipError_t e = hipStreamGetCaptureInfo_v2(st, &cs, &id, &g, &deps, &nd);
    if (e == hipSuccess && cs != hipStreamCaptureStatusActive) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = hipGraphAddEventRecordNode(node, g, deps, nd, ev);
    if (e == hipSuccess) e = hipStreamUpdateCaptureDependencies(st, node, 1, hipStreamSetCaptureDependencies);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (P->cap_error.empty()) P->cap_error = std::string("timing mark in capture: ") + hipGetErrorString(e);
        return false;
    }
    return true;
}

TimeScope::TimeScope(apx_problem* P_, int k) : P(P_), klass(k) {
    if (!P->timing || !((P->timing_mask >> k) & 1u)) return;
    if (P->capturing) {
        apx_problem::CapMark m{};
        m.klass = k;
        if (hipEventCreate(&m.ev[0]) != hipSuccess) { P->cap_error = "timing: event creation"; return; }
        if (hipEventCreate(&m.ev[1]) != hipSuccess) {
            hipEventDestroy(m.ev[0]);
            P->cap_error = "timing: event creation";
            return;
        }
        P->cap_marks.push_back(m);
        idx = P->cap_marks.size() - 1;
        capture_mark(P, m.ev[0], &P->cap_marks[idx].node[0]);
        return;
    }
    while (P->ev_pool.size() < P->ev_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        P->ev_pool.push_back(e);
    }
    idx = P->ev_used;
    P->ev_used += 2;
    hipEventRecord(P->ev_pool[idx], P->ctx->stream);
}
TimeScope::~TimeScope() {
    if (idx == (size_t)-1) return;
    if (P->capturing) {
        capture_mark(P, P->cap_marks[idx].ev[1], &P->cap_marks[idx].node[1]);
        return;
    }
    hipEventRecord(P->ev_pool[idx + 1], P->ctx->stream);
    P->ev_recs.emplace_back(klass, idx);
}

static void drop_graph(apx_problem* P) {
    if (P->gexec) { hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
    if (P->graph) { hipGraphDestroy(P->graph); P->graph = nullptr; }
    for (auto& m : P->cap_marks) {
        hipEventDestroy(m.ev[0]);
        hipEventDestroy(m.ev[1]);
    }
    P->cap_marks.clear();
    P->cap_error.clear();
}

// Before a replay: fresh events of the pool for every timing mark of the graph.
static apx_status arm_mark_nodes(apx_problem* P) {
    for (const auto& m : P->cap_marks) {
        while (P->ev_pool.size() < P->ev_used + 2) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            P->ev_pool.push_back(e);
        }
        const size_t idx = P->ev_used;
        P->ev_used += 2;
        HIPCHK(hipGraphExecEventRecordNodeSetEvent(P->gexec, m.node[0], P->ev_pool[idx]));
        HIPCHK(hipGraphExecEventRecordNodeSetEvent(P->gexec, m.node[1], P->ev_pool[idx + 1]));
        P->ev_recs.emplace_back(m.klass, idx);
    }
    return APX_OK;
}



// ------------------------------------------------------------------ plan build
static apx_status build_plan(apx_problem* P, const apx_problem_desc* d) {
    apx_ctx* C = P->ctx;
    P->n_images = d->n_images;
    P->n_comps = d->n_comps;
    P->n_par = d->n_par;
    P->n_sub = d->n_sub;
    P->s = d->s;
    P->rule = d->rule;
    P->mode = d->mode;
    P->k_re = d->k_re;
    P->objective = d->objective;
    P->conv_mode = d->conv_mode;
    P->psf = d->psf;
    if (d->n_images < 1 || d->n_comps < 0 || d->n_par < 0 || d->n_sub < 1)
        return fail(C, APX_E_INVALID, "counts: need n_images >= 1, n_sub >= 1, n_comps, n_par >= 0");
    if (!d->images || (d->n_comps > 0 && !d->comps) || !d->sub_par || (!d->psf && C->device >= 0))
        return fail(C, APX_E_INVALID, "null descriptor pointer");
    if (d->s < 1 || d->s > MAX_NODES_1D) return fail(C, APX_E_UNSUPPORTED, "s must be in 1..8");
    if (d->rule != APX_RULE_MIDPOINT && d->rule != APX_RULE_GAUSS_LEGENDRE)
        return fail(C, APX_E_INVALID, "unknown node rule");
    if (d->mode != APX_MODE_UNIFORM && d->mode != APX_MODE_WITHIN_K_RE && d->mode != APX_MODE_ADAPTIVE)
        return fail(C, APX_E_INVALID, "unknown sampling mode");
    if (d->mode == APX_MODE_WITHIN_K_RE && !(d->k_re > 0.0 && std::isfinite(d->k_re)))
        return fail(C, APX_E_INVALID, "k_re must be > 0");
    if (d->mode == APX_MODE_ADAPTIVE && !(d->k_re > 0.0 && std::isfinite(d->k_re)))
        return fail(C, APX_E_INVALID, "adaptive tolerance (k_re) must be > 0");
    if (d->objective != APX_OBJECTIVE_FP64 && d->objective != APX_OBJECTIVE_FP32)
        return fail(C, APX_E_INVALID, "unknown objective precision");
    if (d->conv_mode != APX_CONV_DIRECT && d->conv_mode != APX_CONV_FFT && d->conv_mode != APX_CONV_DIRECT_2D &&
        d->conv_mode != APX_CONV_AUTO)
        return fail(C, APX_E_INVALID, "unknown convolution mode");
    if (d->shift != APX_SHIFT_NONE && d->shift != APX_SHIFT_BILINEAR && d->shift != APX_SHIFT_LANCZOS)
        return fail(C, APX_E_INVALID, "unknown re-centring method");
    if (d->shift == APX_SHIFT_LANCZOS && (d->shift_a < 2 || d->shift_a > APX_SHIFT_MAX_A))
        return fail(C, APX_E_UNSUPPORTED, "Lanczos order must be in 2..5");
    if (d->shift != APX_SHIFT_NONE && d->mode == APX_MODE_ADAPTIVE)
        return fail(C, APX_E_UNSUPPORTED, "re-centring with adaptive integration");
    P->shift = d->shift;
    P->shift_a = d->shift == APX_SHIFT_NONE ? 0 : (d->shift == APX_SHIFT_BILINEAR ? 1 : d->shift_a);

    // nodes (adaptive mode: its 3 x 3 Gauss-Legendre level; the other levels use agl)
    if (d->mode == APX_MODE_ADAPTIVE) {
        P->s = 3;
        P->rule = APX_RULE_GAUSS_LEGENDRE;
        for (int order : {3, 5, 7}) {
            std::vector<double> x, w;
            gauss_legendre(order, x, w);
            for (int k = 0; k < order; ++k) P->agl.push_back(x[k] / 2.0);
            for (int k = 0; k < order; ++k) P->agl.push_back(w[k] / 2.0);
        }
    }
    const int s_nodes = P->s;
    if (d->mode == APX_MODE_ADAPTIVE) {
        std::vector<double> x, w;
        gauss_legendre(3, x, w);
        for (int k = 0; k < 3; ++k) {
            P->node_od.push_back(x[k] / 2.0);
            P->node_wd.push_back(w[k] / 2.0);
        }
    } else if (d->rule == APX_RULE_MIDPOINT) {
        for (int k = 0; k < d->s; ++k) {
            P->node_od.push_back((k + 0.5) / d->s - 0.5);
            P->node_wd.push_back(1.0 / d->s);
        }
    } else {
        std::vector<double> x, w;
        gauss_legendre(d->s, x, w);
        for (int k = 0; k < d->s; ++k) {
            P->node_od.push_back(x[k] / 2.0);
            P->node_wd.push_back(w[k] / 2.0);
        }
    }
    for (int k = 0; k < s_nodes; ++k) {
        P->node_o.push_back((float)P->node_od[k]);
        P->node_w.push_back((float)P->node_wd[k]);
    }

    build_bn_table(P->bn_tab);
    build_pow2_table(P->ptab);
    if (d->conv_mode == APX_CONV_FFT || d->conv_mode == APX_CONV_AUTO)
        for (int m = 0; m < FFT_T; ++m) {
            const double a = -2.0 * M_PI * m / FFT_T;
            P->fft_tw.push_back((float)std::cos(a));
            P->fft_tw.push_back((float)std::sin(a));
        }

    // sub-problems
    P->subs.resize(d->n_sub);
    P->par_sub.assign(d->n_par, -1);
    long long aoff = 0;
    for (int s = 0; s < d->n_sub; ++s) {
        int p0 = d->sub_par[2 * s], n = d->sub_par[2 * s + 1];
        if (p0 < 0 || n < 0 || (long long)p0 + n > d->n_par)
            return fail(C, APX_E_INVALID, "sub_par range out of theta");
        for (int k = p0; k < p0 + n; ++k) {
            if (P->par_sub[k] >= 0) return fail(C, APX_E_INVALID, "sub-problem theta ranges overlap");
            P->par_sub[k] = s;
        }
        DSub sb{};
        sb.p0 = p0;
        sb.n = n;
        sb.a_off = aoff;
        sb.large = n > SMALL_N ? 1 : 0;
        sb.flag_off = P->n_sflag;
        sb.diag_idx = sb.large ? (int)P->large_subs.size() : -1;
        if (sb.large) P->n_sflag += 2 * ((n + CHOL_NB - 1) / CHOL_NB);
        aoff += (long long)n * n;
        P->subs[s] = sb;
        if (sb.large) P->large_subs.push_back(s);
        else {
            P->small_subs.push_back(s);
            P->nmax_small = std::max(P->nmax_small, n);
        }
    }
    P->a_total = aoff;
    auto in_sub = [&](int par, int sub) { return par >= 0 && par < d->n_par && P->par_sub[par] == sub; };

    // images
    P->images.resize(d->n_images);
    long long pix = 0, ext = 0, psfo = 0;
    for (int k = 0; k < d->n_images; ++k) {
        const apx_image_desc& id = d->images[k];
        if (id.H < 1 || id.W < 1) return fail(C, APX_E_INVALID, "image " + std::to_string(k) + ": H, W >= 1");
        if (id.P < 1 || id.P % 2 == 0) return fail(C, APX_E_INVALID, "image " + std::to_string(k) + ": P must be odd");
        if (id.P > APX_MAX_PSF) return fail(C, APX_E_UNSUPPORTED, "image " + std::to_string(k) + ": P > 63");
        if (id.sub < 0 || id.sub >= d->n_sub) return fail(C, APX_E_INVALID, "image sub out of range");
        if (id.sky_par >= 0 && !in_sub(id.sky_par, id.sub))
            return fail(C, APX_E_INVALID, "image " + std::to_string(k) + ": sky_par outside its sub-problem");
        if (id.sky_par < -1) return fail(C, APX_E_INVALID, "sky_par < -1");
        const int U = id.psf_up <= 1 ? 1 : id.psf_up;
        if (U != 1 && U != 2 && U != 4 && U != 8)
            return fail(C, APX_E_UNSUPPORTED, "image " + std::to_string(k) + ": psf_up must be 1, 2, 4 or 8");
        if (U != 1 && d->shift != APX_SHIFT_NONE)
            return fail(C, APX_E_UNSUPPORTED, "re-centring with a higher-resolution PSF");
        if ((long long)U * id.H > (1 << 24) || (long long)U * id.W > (1 << 24))
            return fail(C, APX_E_UNSUPPORTED, "image " + std::to_string(k) + ": render grid too large");
        DImage im{};
        im.up = U;
        im.Hc = id.H;
        im.Wc = id.W;
        im.H = U * id.H;
        im.W = U * id.W;
        im.P = id.P;
        im.c = (id.P - 1) / 2;
        im.EH = im.H + 2 * im.c;
        im.EW = im.W + 2 * im.c;
        im.sub = id.sub;
        im.sky_par = id.sky_par;
        im.sky_fixed = id.sky_fixed;
        im.pix_off = pix;
        im.ext_off = ext;
        im.psf_off = psfo;
        im.fft_off = -1;
        if (d->conv_mode == APX_CONV_FFT && id.P >= APX_FFT_MIN_P && U == 1) {
            im.fft_off = P->n_fft_spec;
            P->n_fft_spec += 2LL * FFT_T * FFT_T;
            ++P->n_fft_images;
        }
        // render-grid pixel -> sky: the image's map after pixel = (sub-pixel + 1/2) / U - 1/2
        {
            const double* a = id.affine;
            const double o = (1.0 - U) / (2.0 * U);
            im.aff[0] = a[0] + (a[1] + a[2]) * o;
            im.aff[1] = a[1] / U;
            im.aff[2] = a[2] / U;
            im.aff[3] = a[3] + (a[4] + a[5]) * o;
            im.aff[4] = a[4] / U;
            im.aff[5] = a[5] / U;
        }
        const double det = im.aff[1] * im.aff[5] - im.aff[2] * im.aff[4];
        if (!std::isfinite(det) || det == 0.0) return fail(C, APX_E_INVALID, "singular affine map");
        im.area = std::fabs(det);
        // inverse: p = Ainv (u - t)
        const double i11 = im.aff[5] / det, i12 = -im.aff[2] / det;
        const double i21 = -im.aff[4] / det, i22 = im.aff[1] / det;
        im.inv[1] = i11;
        im.inv[2] = i12;
        im.inv[4] = i21;
        im.inv[5] = i22;
        im.inv[0] = -(i11 * im.aff[0] + i12 * im.aff[3]);
        im.inv[3] = -(i21 * im.aff[0] + i22 * im.aff[3]);
        P->images[k] = im;
        pix += (long long)id.H * id.W;
        ext += (long long)im.EH * im.EW;
        psfo += (long long)id.P * id.P;
    }
    P->n_pix = pix;
    P->n_ext = ext;
    P->n_psf = psfo;

    // live PSF models
    if (d->n_psf_models < 0 || (d->n_psf_models > 0 && !d->psf_models))
        return fail(C, APX_E_INVALID, "psf_models: bad count or null pointer");
    for (int m = 0; m < d->n_psf_models; ++m) {
        const apx_psf_model_desc& md = d->psf_models[m];
        if (md.type != APX_PSF_MOFFAT) return fail(C, APX_E_UNSUPPORTED, "unknown PSF model type");
        if (md.image < 0 || md.image >= d->n_images) return fail(C, APX_E_INVALID, "PSF model image out of range");
        DImage& im = P->images[md.image];
        if (im.live) return fail(C, APX_E_INVALID, "two PSF models for one image");
        for (int q = 0; q < 2; ++q) {
            if (md.par[q] < -1 || (md.par[q] >= 0 && !in_sub(md.par[q], im.sub)))
                return fail(C, APX_E_INVALID, "PSF model parameter outside its image's sub-problem");
            if (md.par[q] >= 0 && md.par[q] == im.sky_par)
                return fail(C, APX_E_INVALID, "PSF model parameter shares the sky index");
            if (md.par[q] < 0 && !std::isfinite(md.fixed[q]))
                return fail(C, APX_E_INVALID, "non-finite fixed PSF parameter");
            im.live_par[q] = md.par[q];
            im.live_fixed[q] = md.fixed[q];
        }
        im.live = 1;
        im.live_off = P->n_live;
        P->n_live += 3LL * im.P * im.P;
    }

    // rank-one stamps: K_uv = a_u b_v to FP32 rounding (a Gaussian, for one), whose
    // Jacobian-column convolutions run as two 1-D passes.  With the largest entry at
    // (u0, v0): a_u = K_u,v0 and b_v = K_u0,v / K_u0,v0; every entry must be reproduced to
    // 4e-7 of itself (three FP32 roundings of exact products) plus 1e-9 of the largest.
    for (int k = 0; k < d->n_images; ++k) P->images[k].sep_off = -1;
    P->psf_sep.clear();
    if ((d->conv_mode == APX_CONV_DIRECT || d->conv_mode == APX_CONV_AUTO) && C->device >= 0 && P->n_psf > 0) {
        std::vector<float> h((size_t)P->n_psf);
        if (hipMemcpy(h.data(), d->psf, (size_t)P->n_psf * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(C, APX_E_HIP, "reading the stamps back");
        for (int k = 0; k < d->n_images; ++k) {
            DImage& im = P->images[k];
            if (im.live || im.up != 1 || im.P < 3) continue;
            const int Pk = im.P;
            const float* K = h.data() + im.psf_off;
            int u0 = 0, v0 = 0;
            double kmax = 0.0;
            for (int u = 0; u < Pk; ++u)
                for (int v = 0; v < Pk; ++v)
                    if (std::fabs((double)K[u * Pk + v]) > kmax) { kmax = std::fabs((double)K[u * Pk + v]); u0 = u; v0 = v; }
            if (!(kmax > 0.0) || !std::isfinite(kmax)) continue;
            std::vector<double> a(Pk), b(Pk);
            for (int u = 0; u < Pk; ++u) a[u] = K[u * Pk + v0];
            for (int v = 0; v < Pk; ++v) b[v] = (double)K[u0 * Pk + v] / (double)K[u0 * Pk + v0];
            bool ok = true;
            for (int u = 0; u < Pk && ok; ++u)
                for (int v = 0; v < Pk && ok; ++v) {
                    const double kv = K[u * Pk + v];
                    ok = std::isfinite(kv) && std::fabs(kv - a[u] * b[v]) <= 4e-7 * std::fabs(kv) + 1e-9 * kmax;
                }
            if (!ok) continue;
            im.sep_off = (long long)P->psf_sep.size();
            for (int u = 0; u < Pk; ++u) P->psf_sep.push_back((float)a[u]);
            for (int v = 0; v < Pk; ++v) P->psf_sep.push_back((float)b[v]);
        }
    }

    // components
    P->comps.resize(d->n_comps);
    for (int i = 0; i < d->n_comps; ++i) {
        const apx_comp_desc& cd = d->comps[i];
        if (cd.type != APX_SERSIC && cd.type != APX_POINT) return fail(C, APX_E_INVALID, "unknown component type");
        if (cd.image < 0 || cd.image >= d->n_images) return fail(C, APX_E_INVALID, "component image out of range");
        const DImage& im = P->images[cd.image];
        DComp c{};
        c.type = cd.type;
        c.image = cd.image;
        c.sub = im.sub;
        c.group = -1;
        for (int k = 0; k < 7; ++k) {
            c.par[k] = cd.par[k];
            c.fixed[k] = cd.fixed[k];
            c.col[k] = -1;
            if (cd.par[k] < -1 || cd.par[k] >= d->n_par)
                return fail(C, APX_E_INVALID, "component " + std::to_string(i) + ": par index out of range");
            if (cd.par[k] >= 0 && !in_sub(cd.par[k], im.sub))
                return fail(C, APX_E_INVALID, "component " + std::to_string(i) + ": parameter outside its sub-problem");
            if (cd.par[k] >= 0 && cd.par[k] == im.sky_par)
                return fail(C, APX_E_INVALID, "component parameter shares the sky index");
            if (cd.par[k] < 0 && !std::isfinite(cd.fixed[k]) && (cd.type == APX_SERSIC || k < 3))
                return fail(C, APX_E_INVALID, "non-finite fixed parameter");
        }
        if (cd.type == APX_POINT) {
            if (cd.par[0] >= 0 || cd.par[1] >= 0)
                return fail(C, APX_E_UNSUPPORTED, "point-source positions must be fixed");
            for (int k = 3; k < 7; ++k)
                if (cd.par[k] >= 0) return fail(C, APX_E_INVALID, "point source has 3 local parameters");
        }
        // clip the window to the extended grid
        int y0 = std::max(cd.box[0], -im.c), x0 = std::max(cd.box[1], -im.c);
        int y1 = std::min(cd.box[2], im.H + im.c), x1 = std::min(cd.box[3], im.W + im.c);
        if (y1 <= y0 || x1 <= x0) { y0 = x0 = y1 = x1 = 0; }
        c.box[0] = c.sbox[0] = y0; c.box[1] = c.sbox[1] = x0;
        c.box[2] = c.sbox[2] = y1; c.box[3] = c.sbox[3] = x1;
        if (cd.type == APX_SERSIC && P->shift != APX_SHIFT_NONE && y1 > y0) {
            // the shifted component reaches shift_a pixels beyond where it is sampled
            const int a = P->shift_a;
            c.box[0] = std::max(y0 - a, -im.c);
            c.box[1] = std::max(x0 - a, -im.c);
            c.box[2] = std::min(y1 + a, im.H + im.c);
            c.box[3] = std::min(x1 + a, im.W + im.c);
        }
        P->comps[i] = c;
    }

    // adaptive integration: per-pixel arrays of the Sersic windows, cut into chunks
    if (d->mode == APX_MODE_ADAPTIVE) {
        P->acomp_chunk.assign(1, 0);
        for (int i = 0; i < d->n_comps; ++i) {
            DComp& c = P->comps[i];
            const long long npx = (long long)(c.box[2] - c.box[0]) * (c.box[3] - c.box[1]);
            c.aoff = P->n_apix;
            if (c.type == APX_SERSIC) {
                for (long long e = 0; e < npx; e += ADAPT_CHUNK) P->achunks.push_back(AChunk{i, (int)e});
                P->n_apix += npx;
            }
            P->acomp_chunk.push_back((int)P->achunks.size());
        }
        if (P->n_apix >= (1LL << 31) || P->achunks.size() >= (size_t)INT32_MAX)
            return fail(C, APX_E_UNSUPPORTED, "adaptive integration: too many window pixels");
    }

    // render tiles (extended grid) with component lists
    {
        std::vector<int> tile_base(d->n_images + 1, 0);
        for (int k = 0; k < d->n_images; ++k) {
            const DImage& im = P->images[k];
            const int ny = ceil_div(im.EH, RT_Y), nx = ceil_div(im.EW, RT_X);
            tile_base[k + 1] = tile_base[k] + ny * nx;
            for (int ty = 0; ty < ny; ++ty)
                for (int tx = 0; tx < nx; ++tx) P->rtiles.push_back(RTile{k, -im.c + ty * RT_Y, -im.c + tx * RT_X, 0});
        }
        const int nt = (int)P->rtiles.size();
        std::vector<int> cnt(nt + 1, 0);
        auto for_tiles = [&](int ci, auto&& fn) {
            const DComp& c = P->comps[ci];
            if (c.box[2] <= c.box[0]) return;
            const DImage& im = P->images[c.image];
            const int nx = ceil_div(im.EW, RT_X);
            const int ty0 = (c.box[0] + im.c) / RT_Y, ty1 = (c.box[2] - 1 + im.c) / RT_Y;
            const int tx0 = (c.box[1] + im.c) / RT_X, tx1 = (c.box[3] - 1 + im.c) / RT_X;
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) fn(tile_base[c.image] + ty * nx + tx);
        };
        for (int ci = 0; ci < d->n_comps; ++ci) for_tiles(ci, [&](int t) { cnt[t + 1]++; });
        for (int t = 0; t < nt; ++t) cnt[t + 1] += cnt[t];
        P->rtile_off = cnt;
        P->rtile_comps.assign(cnt[nt], 0);
        std::vector<int> fillp(cnt.begin(), cnt.end() - 1);
        for (int ci = 0; ci < d->n_comps; ++ci) for_tiles(ci, [&](int t) { P->rtile_comps[fillp[t]++] = ci; });
    }

    // Jacobian groups: Sersic components with a free parameter sharing image and window
    // merge into one group; each point source with a free flux is its own group.
    {
        std::map<std::tuple<int, int, int, int, int>, int> key2g;
        std::vector<std::vector<int>> gcomps;
        for (int ci = 0; ci < d->n_comps; ++ci) {
            DComp& c = P->comps[ci];
            bool anyfree = false;
            for (int k = 0; k < 7; ++k) anyfree = anyfree || c.par[k] >= 0;
            if (!anyfree || c.box[2] <= c.box[0]) continue;
            int g;
            if (c.type == APX_SERSIC) {
                auto key = std::make_tuple(c.image, c.box[0], c.box[1], c.box[2], c.box[3]);
                auto it = key2g.find(key);
                if (it == key2g.end()) {
                    g = (int)gcomps.size();
                    key2g[key] = g;
                    gcomps.emplace_back();
                } else g = it->second;
            } else {
                g = (int)gcomps.size();
                gcomps.emplace_back();
            }
            gcomps[g].push_back(ci);
            c.group = g;
        }
        long long doff = 0, joff = 0, gpoff = 0;
        for (size_t g = 0; g < gcomps.size(); ++g) {
            const DComp& c0 = P->comps[gcomps[g][0]];
            const DImage& im = P->images[c0.image];
            DGroup gr{};
            gr.image = c0.image;
            gr.type = c0.type;
            gr.sub = im.sub;
            gr.iy0 = c0.box[0];
            gr.ix0 = c0.box[1];
            gr.ih = c0.box[2] - c0.box[0];
            gr.iw = c0.box[3] - c0.box[1];
            // output box on the render grid, then in image pixels (rounded outward)
            const int oy0 = std::max(0, c0.box[0] - im.c), ox0 = std::max(0, c0.box[1] - im.c);
            const int oy1 = std::min(im.H, c0.box[2] + im.c), ox1 = std::min(im.W, c0.box[3] + im.c);
            gr.oy0 = oy0 / im.up;
            gr.ox0 = ox0 / im.up;
            gr.oh = oy1 > oy0 ? ceil_div(oy1, im.up) - gr.oy0 : 0;
            gr.ow = ox1 > ox0 ? ceil_div(ox1, im.up) - gr.ox0 : 0;
            gr.comp_begin = (int)P->group_comps.size();
            gr.col_begin = (int)P->cols.size();
            int nc = 0;
            for (int ci : gcomps[g]) {
                P->group_comps.push_back(ci);
                DComp& c = P->comps[ci];
                for (int k = 0; k < 7; ++k) {
                    if (c.par[k] < 0) continue;
                    c.col[k] = nc++;
                    P->cols.push_back(DCol{(int)g, ci, k, c.par[k]});
                }
            }
            gr.comp_end = (int)P->group_comps.size();
            gr.ncols = nc;
            gr.d_off = doff;
            gr.j_off = joff;
            doff += (long long)nc * gr.ih * gr.iw;
            joff += (long long)nc * gr.oh * gr.ow;
            gr.tile_begin = (int)P->gtiles.size();
            const int ny = ceil_div(gr.ih, RT_Y), nx = ceil_div(gr.iw, RT_X);
            for (int ty = 0; ty < ny; ++ty)
                for (int tx = 0; tx < nx; ++tx) P->gtiles.push_back(RTile{(int)g, ty * RT_Y, tx * RT_X, 0});
            gr.ntiles = ny * nx;
            gr.gp_off = gpoff;
            gpoff += (long long)nc * gr.ntiles;
            P->groups.push_back(gr);
        }
        // live-PSF columns of each image: input the pre-convolution model S on the
        // extended grid, output the whole image, no derivative images and no tiles
        for (int k = 0; k < d->n_images; ++k) {
            const DImage& im = P->images[k];
            if (!im.live || (im.live_par[0] < 0 && im.live_par[1] < 0)) continue;
            DGroup gr{};
            gr.image = k;
            gr.type = GROUP_PSF;
            gr.sub = im.sub;
            gr.iy0 = -im.c; gr.ix0 = -im.c; gr.ih = im.EH; gr.iw = im.EW;
            gr.oy0 = 0; gr.ox0 = 0; gr.oh = im.Hc; gr.ow = im.Wc;
            gr.comp_begin = gr.comp_end = (int)P->group_comps.size();
            gr.col_begin = (int)P->cols.size();
            int nc = 0;
            for (int q = 0; q < 2; ++q)
                if (im.live_par[q] >= 0) {
                    P->cols.push_back(DCol{(int)P->groups.size(), -1, q, im.live_par[q]});
                    ++nc;
                }
            gr.ncols = nc;
            gr.d_off = doff;
            gr.j_off = joff;
            joff += (long long)nc * gr.oh * gr.ow;
            gr.tile_begin = (int)P->gtiles.size();
            gr.ntiles = 0;
            gr.gp_off = gpoff;
            P->groups.push_back(gr);
            P->has_live_cols = true;
        }
        P->n_d = doff;
        P->n_j = joff;
        P->n_gradpart = gpoff;
    }
    const int n_cols = (int)P->cols.size();
    const int n_groups = (int)P->groups.size();
    // groups whose columns' J^T W r (sum w r J) and sum w J (the sky row of J^T W J) come from
    // the 4 x 4-block Gram kernel, which forms their self-pair and reads each pixel's weight
    // anyway, instead of from the convolution epilogues
    auto gram_part = [&](int g) {
        const DGroup& gr = P->groups[g];
        return gr.type != GROUP_PSF && gr.oh > 0 && gr.ow > 0 && gr.ncols > 0 && gr.ncols <= 4 * GRAM4_MAX_T;
    };

    // convolution jobs and items, sorted by (PSF size, tile shape): one launch per pair,
    // except that the FFT-tile items of every PSF size form one range and one launch (the
    // FFT kernel takes P at run time, so one grid keeps the chip full to its end instead of
    // leaving a partly filled last round per PSF size).
    // The direct jobs of one PSF size take the tile shape of least estimated cost over all of
    // them (choose_group_shape).
    // In FFT mode, jobs of the FP32 kinds on images with spectra and outputs of at least
    // 32 x 32 take the FFT shape; in automatic mode, such a job (on an image with a fixed,
    // not rank-one stamp at P >= APX_FFT_MIN_P) takes it when the cost model prices its
    // transforms below its direct tiles (auto_fft), and its image gets spectra.  The items
    // of each FFT range are paired (two per complex transform) when they share the image,
    // and so the stamp.
    auto add_items = [&](int kind, std::vector<ConvJob>& jobs, std::vector<ConvItem>& items,
                         std::vector<PRange>& ranges, const std::vector<int>& jobP,
                         const std::vector<int>& nch, std::vector<int>* job_item_begin,
                         std::vector<int4>* pairs) {
        const int key = kind == CONV_JCOL ? TUNE_JCOL : kind == CONV_ADJ ? TUNE_ADJ
                      : P->objective == APX_OBJECTIVE_FP64 ? TUNE_FWD64 : TUNE_FWD32;
        for (size_t j = 0; j < jobs.size(); ++j) {
            DImage& im = P->images[jobs[j].image];
            const bool big = jobs[j].out_h >= 32 && jobs[j].out_w >= 32;
            const bool sep = kind == CONV_JCOL && im.sep_off >= 0;
            bool fft = pairs && big && P->conv_mode == APX_CONV_FFT && im.fft_off >= 0;
            if (pairs && big && !sep && P->conv_mode == APX_CONV_AUTO && !im.live && im.up == 1 &&
                im.P >= APX_FFT_MIN_P && nch[j] > 0 && auto_fft(jobP[j], jobs[j].out_h, jobs[j].out_w, nch[j])) {
                fft = true;
                if (im.fft_off < 0) {
                    im.fft_off = P->n_fft_spec;
                    P->n_fft_spec += 2LL * FFT_T * FFT_T;
                    ++P->n_fft_images;
                }
            }
            jobs[j].shape = fft ? SHAPE_FFT : sep ? SHAPE_SEP : 0;
        }
        // the direct jobs of each PSF size: one shape for the group (choose_group_shape)
        {
            std::map<int, std::vector<int>> byP;
            for (size_t j = 0; j < jobs.size(); ++j)
                if (jobs[j].shape < N_TILE_SHAPES) byP[jobP[j]].push_back((int)j);
            for (const auto& kv : byP) {
                std::vector<int> h, w, nc;
                for (int j : kv.second) {
                    h.push_back(jobs[j].out_h);
                    w.push_back(jobs[j].out_w);
                    nc.push_back(nch[j]);
                }
                const int s = choose_group_shape(C, key, kv.first, h, w, nc);
                for (int j : kv.second) jobs[j].shape = s;
            }
        }
        std::vector<int> order(jobs.size());
        for (size_t i = 0; i < jobs.size(); ++i) order[i] = (int)i;
        // FFT jobs sort after every direct and two-pass job, by PSF size among themselves
        auto fft_key = [&](int a) { return jobs[a].shape == SHAPE_FFT ? 1 : 0; };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            if (fft_key(a) != fft_key(b)) return fft_key(a) < fft_key(b);
            return jobP[a] != jobP[b] ? jobP[a] < jobP[b] : jobs[a].shape < jobs[b].shape;
        });
        if (job_item_begin) job_item_begin->assign(jobs.size(), 0);
        for (int j : order) {
            const ConvJob& jb = jobs[j];
            const int ny = ceil_div(jb.out_h, shape_th(jb.shape, jobP[j]));
            const int nx = ceil_div(jb.out_w, shape_tw(jb.shape, jobP[j]));
            if (job_item_begin) (*job_item_begin)[j] = (int)items.size();
            const int b = (int)items.size();
            for (int ch = 0; ch < nch[j]; ++ch)
                for (int ty = 0; ty < ny; ++ty)
                    for (int tx = 0; tx < nx; ++tx) items.push_back(ConvItem{j, ch, ty, tx});
            const int cnt = (int)items.size() - b;
            if (cnt == 0) continue;
            const bool same = !ranges.empty() && ranges.back().shape == jb.shape &&
                              (jb.shape == SHAPE_FFT || ranges.back().P == jobP[j]);
            if (same)
                ranges.back().count += cnt;
            else
                ranges.push_back(PRange{jb.shape == SHAPE_FFT ? 0 : jobP[j], jb.shape, b, cnt, 0, 0});
        }
        if (!pairs) return;
        for (PRange& r : ranges) {
            if (r.shape != SHAPE_FFT) continue;
            r.pair_begin = (int)pairs->size();
            for (int i = r.begin; i < r.begin + r.count;) {
                const bool two = i + 1 < r.begin + r.count &&
                                 jobs[items[i].job].image == jobs[items[i + 1].job].image;
                pairs->push_back(make_int4(i, two ? i + 1 : -1, P->images[jobs[items[i].job].image].sub, 0));
                i += two ? 2 : 1;
            }
            r.pair_count = (int)pairs->size() - r.pair_begin;
        }
    };
    auto job_tiles = [&](const ConvJob& jb) {
        const int Pj = P->images[jb.image].P;
        return ceil_div(jb.out_h, shape_th(jb.shape, Pj)) * ceil_div(jb.out_w, shape_tw(jb.shape, Pj));
    };
    std::vector<int> fwd_item_begin, jcol_item_begin;
    {
        std::vector<int> jp, nch;
        for (int k = 0; k < d->n_images; ++k) {
            const DImage& im = P->images[k];
            ConvJob jb{};
            jb.in_off = im.ext_off;
            jb.out_off = im.pix_off;
            jb.in_y0 = -im.c; jb.in_x0 = -im.c; jb.in_h = im.EH; jb.in_w = im.EW;
            jb.out_y0 = 0; jb.out_x0 = 0; jb.out_h = im.H; jb.out_w = im.W;
            jb.image = k;
            jb.group = -1;
            P->fwd_jobs.push_back(jb);
            jp.push_back(im.P);
            nch.push_back(1);
            ConvJob ja = jb;
            ja.in_off = 0;                   // adjoint input is staged from the residual
            ja.in_y0 = 0; ja.in_x0 = 0; ja.in_h = im.H; ja.in_w = im.W;
            ja.out_off = im.ext_off;
            ja.out_y0 = -im.c; ja.out_x0 = -im.c; ja.out_h = im.EH; ja.out_w = im.EW;
            P->adj_jobs.push_back(ja);
        }
        add_items(CONV_FWD, P->fwd_jobs, P->fwd_items, P->fwd_ranges, jp, nch, &fwd_item_begin,
                  P->objective == APX_OBJECTIVE_FP32 ? &P->fwd_pairs : nullptr);
        add_items(CONV_ADJ, P->adj_jobs, P->adj_items, P->adj_ranges, jp, nch, nullptr, &P->adj_pairs);
    }
    std::vector<int> psf_job_of(n_groups, -1), psf_item_begin;
    {
        // one job per group (index = group); live-PSF groups get no items here and a job
        // of their own in the PSF list (input S, derivative stamps)
        std::vector<int> jp, nch, pjp, pnch;
        for (int g = 0; g < n_groups; ++g) {
            const DGroup& gr = P->groups[g];
            const DImage& im = P->images[gr.image];
            ConvJob jb{};
            jb.in_off = gr.d_off;
            jb.in_cs = (long long)gr.ih * gr.iw;
            jb.out_off = gr.j_off;
            jb.out_cs = (long long)gr.oh * gr.ow;
            jb.in_y0 = gr.iy0; jb.in_x0 = gr.ix0; jb.in_h = gr.ih; jb.in_w = gr.iw;
            // the job's output rectangle is on the render grid (whole pixels of sub-pixels)
            jb.out_y0 = im.up * gr.oy0; jb.out_x0 = im.up * gr.ox0;
            jb.out_h = im.up * gr.oh; jb.out_w = im.up * gr.ow;
            jb.image = gr.image;
            jb.group = g;
            jb.gram_part = gram_part(g) ? 1 : 0;
            const bool psfg = gr.type == GROUP_PSF;
            P->jcol_jobs.push_back(jb);
            jp.push_back(im.P);
            nch.push_back(!psfg && gr.oh > 0 && gr.ow > 0 ? gr.ncols : 0);
            if (psfg) {
                ConvJob pj = jb;
                pj.in_src = 1;
                pj.in_off = im.ext_off;
                pj.in_cs = 0;                      // every PSF column convolves the same S
                for (int ch = 0; ch < gr.ncols && ch < 2; ++ch) pj.kslot[ch] = 1 + P->cols[gr.col_begin + ch].local;
                psf_job_of[g] = (int)P->psf_jobs.size();
                P->psf_jobs.push_back(pj);
                pjp.push_back(im.P);
                pnch.push_back(gr.ncols);
            }
        }
        add_items(CONV_JCOL, P->jcol_jobs, P->jcol_items, P->jcol_ranges, jp, nch, &jcol_item_begin,
                  &P->jcol_pairs);
        add_items(CONV_JCOL, P->psf_jobs, P->psf_items, P->psf_ranges, pjp, pnch, &psf_item_begin, nullptr);
    }

    // reduction tables: FWD items per image, JCOL items per column, grad partials per column
    {
        P->img_seg.assign(1, 0);
        for (int k = 0; k < d->n_images; ++k) {
            const DImage& im = P->images[k];
            (void)im;
            const int n = job_tiles(P->fwd_jobs[k]);
            for (int q = 0; q < n; ++q) P->img_idx.push_back(fwd_item_begin[k] + q);
            P->img_seg.push_back((int)P->img_idx.size());
        }
        P->col_seg.assign(1, 0);
        P->gcol_seg.assign(1, 0);
        const int n_main_items = (int)P->jcol_items.size();
        for (int g = 0; g < n_groups; ++g) {
            const DGroup& gr = P->groups[g];
            const int pj = psf_job_of[g];
            const ConvJob& job = pj >= 0 ? P->psf_jobs[pj] : P->jcol_jobs[g];
            const int per = (gr.oh > 0 && gr.ow > 0) ? job_tiles(job) : 0;
            // partials of the PSF list follow those of the main list in jcol_part
            const int first = pj >= 0 ? n_main_items + psf_item_begin[pj] : jcol_item_begin[g];
            for (int ch = 0; ch < gr.ncols; ++ch) {
                if (!gram_part(g))        // (the others' partials come from k_gram4)
                    for (int q = 0; q < per; ++q) P->col_idx.push_back(first + ch * per + q);
                P->col_seg.push_back((int)P->col_idx.size());
                P->gcol_seg.push_back((int)(gr.gp_off + (long long)(ch + 1) * gr.ntiles));
            }
        }
    }

    // pairs of groups on one image whose output boxes intersect.  A pair's box is cut
    // into K-slices of whole LDS stages (KC pixels of one row).  Narrow pairs (16-wide
    // tiles) take slices of about 4096 pixels.  The 64-wide tile pairs share the grid in
    // proportion to their work, so their items fill the resident workgroups of the chip
    // about once (no second, partly empty wave of workgroups); each item still gets at
    // least 32 stages.
    {
        struct Wide { int pi, na, nb, tri, stages; };
        std::vector<Wide> wide;
        std::vector<std::vector<PairItem>> gram_items(GRAM4_MAX_T + 1);
        long long outoff = 0;
        auto tile_pairs = [](int na, int nb, int tri) { return tri ? na * (na + 1) / 2 : na * nb; };
        // K-slices outermost: the tile pairs that run together read the same rows of J
        auto add_pair_items = [&](int pi, int na, int nb, bool tri, int stages, int per, int tm) {
            for (int s0 = 0; s0 < stages; s0 += per)
                for (int ta = 0; ta < na; ++ta)
                    for (int tb = tri ? ta : 0; tb < nb; ++tb) {
                        PairItem it{};
                        it.pair = pi;
                        it.ta = ta;
                        it.tb = tb;
                        it.s0 = s0;
                        it.s1 = std::min(stages, s0 + per);
                        it.out_off = outoff;
                        outoff += (long long)tm * tm;
                        (tm == 64 ? P->pitems64 : P->pitems16).push_back(it);
                    }
        };
        std::vector<std::vector<int>> by_img(d->n_images);
        for (int g = 0; g < n_groups; ++g)
            if (P->groups[g].oh > 0 && P->groups[g].ow > 0) by_img[P->groups[g].image].push_back(g);
        for (int k = 0; k < d->n_images; ++k) {
            const auto& gl = by_img[k];
            for (size_t a = 0; a < gl.size(); ++a)
                for (size_t b = a; b < gl.size(); ++b) {
                    const DGroup& G = P->groups[gl[a]];
                    const DGroup& H = P->groups[gl[b]];
                    const int y0 = std::max(G.oy0, H.oy0), x0 = std::max(G.ox0, H.ox0);
                    const int y1 = std::min(G.oy0 + G.oh, H.oy0 + H.oh), x1 = std::min(G.ox0 + G.ow, H.ox0 + H.ow);
                    if (y1 <= y0 || x1 <= x0) continue;
                    DPair pr{gl[a], gl[b], k, G.sub, y0, x0, y1, x1};
                    const int pi = (int)P->pairs.size();
                    P->pairs.push_back(pr);
                    const int tm = (std::min(G.ncols, H.ncols) >= 48) ? 64 : 16;
                    const int na = ceil_div(G.ncols, tm), nb = ceil_div(H.ncols, tm);
                    const int stages = (y1 - y0) * ceil_div(x1 - x0, PAIR_KC);
                    const bool tri = gl[a] == gl[b];
                    if (tri && G.ncols <= 4 * GRAM4_MAX_T) {
                        // a narrow group with itself: 4 x 4 blocks (k_gram4), K-slices of ~4096 px
                        const int nt = ceil_div(G.ncols, 4);
                        const int per = std::max(1, 4096 / PAIR_KC);
                        for (int s0 = 0; s0 < stages; s0 += per) {
                            PairItem it{};
                            it.pair = pi;
                            it.ta = nt;
                            it.s0 = s0;
                            it.s1 = std::min(stages, s0 + per);
                            gram_items[nt].push_back(it);
                        }
                        continue;
                    }
                    if (tm == 64) {
                        wide.push_back({pi, na, nb, tri ? 1 : 0, stages});
                        continue;
                    }
                    add_pair_items(pi, na, nb, tri, stages, std::max(1, 4096 / PAIR_KC), 16);
                }
        }
        long long work = 0;
        for (const Wide& w : wide) work += (long long)tile_pairs(w.na, w.nb, w.tri) * w.stages;
        const long long slots = pair_slots(P->ctx);
        for (const Wide& w : wide) {
            const int tp = tile_pairs(w.na, w.nb, w.tri);
            const double share = (double)slots * tp * w.stages / (double)std::max(1LL, work);
            int slices = std::max(1, (int)(share / tp));
            slices = std::min(slices, std::max(1, w.stages / 32));
            add_pair_items(w.pi, w.na, w.nb, w.tri, w.stages, ceil_div(w.stages, slices), 64);
        }
        P->gitems.clear();
        for (int t = 0; t <= GRAM4_MAX_T; ++t) {
            P->gram_begin[t] = (int)P->gitems.size();
            for (PairItem it : gram_items[t]) {
                it.out_off = outoff;
                outoff += (long long)16 * (t * (t + 1) / 2 + t);     // tile pairs, then J^T W [r 1]
                P->gitems.push_back(it);
            }
        }
        P->gram_begin[GRAM4_MAX_T + 1] = (int)P->gitems.size();
        P->n_pairpart = outoff;
    }
    P->asrc_col = P->n_pairpart;
    P->asrc_gcol = P->asrc_col + 2LL * n_cols;
    P->asrc_img = P->asrc_gcol + n_cols;
    if (P->asrc_img + 3LL * d->n_images > (long long)INT32_MAX)   // J^T W r sources are 32-bit indices
        return fail(C, APX_E_INVALID, "problem too large: J^T W J partials exceed 2^31 entries");

    // the 4 x 4-block Gram items of each group, and where each holds a column's J^T W r
    // (comp 0) and sum w J (comp 1) over its K-slice: after the item's t (t + 1) / 2 tile-pair
    // blocks, block ta = ci / 4 of the item's J^T W [r 1], entry (ci mod 4, comp)
    std::vector<std::vector<int>> group_gitems(n_groups);
    for (int i = 0; i < (int)P->gitems.size(); ++i) group_gitems[P->pairs[P->gitems[i].pair].g].push_back(i);
    auto gram_src = [&](int gi, int ci, int comp) {
        const PairItem& it = P->gitems[gi];
        const int t = it.ta;
        return it.out_off + 16LL * (t * (t + 1) / 2 + ci / 4) + 4 * (ci % 4) + comp;
    };

    // A assembly: sources per upper entry (sub, a <= b) in a fixed order
    {
        std::vector<long long> ent_base(d->n_sub + 1, 0);
        for (int s = 0; s < d->n_sub; ++s) {
            const long long n = P->subs[s].n;
            ent_base[s + 1] = ent_base[s] + n * (n + 1) / 2;
        }
        const long long n_ent = ent_base[d->n_sub];
        auto ent_id = [&](int s, int a, int b) -> long long {
            // row-major upper triangle: row a holds entries (a, a..n-1)
            const long long n = P->subs[s].n;
            return ent_base[s] + (long long)a * n - (long long)a * (a - 1) / 2 + (b - a);
        };
        std::vector<std::pair<long long, long long>> contrib;   // (entry, src index)
        auto add = [&](int p, int q, long long src, int mult) {
            const int s = P->par_sub[p];
            const int p0 = P->subs[s].p0;
            const int a = std::min(p, q) - p0, b = std::max(p, q) - p0;
            const long long e = ent_id(s, a, b);
            for (int m = 0; m < mult; ++m) contrib.emplace_back(e, src);
        };
        auto add_items_tm = [&](const std::vector<PairItem>& items, int tm) {
            for (const PairItem& it : items) {
                const DPair& pr = P->pairs[it.pair];
                const DGroup& G = P->groups[pr.g];
                const DGroup& H = P->groups[pr.h];
                for (int i = 0; i < tm; ++i) {
                    const int ci = it.ta * tm + i;
                    if (ci >= G.ncols) break;
                    for (int j = 0; j < tm; ++j) {
                        const int cj = it.tb * tm + j;
                        if (cj >= H.ncols) break;
                        if (pr.g == pr.h && ci > cj) continue;
                        const int p = P->cols[G.col_begin + ci].par, q = P->cols[H.col_begin + cj].par;
                        const bool diag_same_col = (pr.g == pr.h && ci == cj);
                        add(p, q, it.out_off + (long long)i * tm + j, (p == q && !diag_same_col) ? 2 : 1);
                    }
                }
            }
        };
        // keep item order: 64-tiles, 16-tiles, then 4 x 4-block Gram items, each in item order
        add_items_tm(P->pitems64, 64);
        add_items_tm(P->pitems16, 16);
        for (const PairItem& it : P->gitems) {
            const DPair& pr = P->pairs[it.pair];
            const DGroup& G = P->groups[pr.g];
            int q = 0;
            for (int ta = 0; ta < it.ta; ++ta)
                for (int tb = ta; tb < it.ta; ++tb, ++q)
                    for (int i = 0; i < 4; ++i) {
                        const int ci = 4 * ta + i;
                        if (ci >= G.ncols) break;
                        for (int j = 0; j < 4; ++j) {
                            const int cj = 4 * tb + j;
                            if (cj >= G.ncols) break;
                            if (ci > cj) continue;
                            const int pp = P->cols[G.col_begin + ci].par, qq = P->cols[G.col_begin + cj].par;
                            add(pp, qq, it.out_off + (long long)q * 16 + i * 4 + j, (pp == qq && ci != cj) ? 2 : 1);
                        }
                    }
        }
        for (int k = 0; k < d->n_images; ++k) {
            const DImage& im = P->images[k];
            if (im.sky_par < 0) continue;
            for (int g = 0; g < n_groups; ++g) {
                const DGroup& gr = P->groups[g];
                if (gr.image != k || gr.oh <= 0 || gr.ow <= 0) continue;
                for (int ch = 0; ch < gr.ncols; ++ch) {
                    if (gram_part(g)) {
                        for (int gi : group_gitems[g]) add(im.sky_par, P->cols[gr.col_begin + ch].par, gram_src(gi, ch, 1), 1);
                    } else {
                        add(im.sky_par, P->cols[gr.col_begin + ch].par, P->asrc_col + 2LL * (gr.col_begin + ch) + 1, 1);
                    }
                }
            }
            add(im.sky_par, im.sky_par, P->asrc_img + 3LL * k + 2, 1);
        }
        std::stable_sort(contrib.begin(), contrib.end(),
                         [](const std::pair<long long, long long>& x, const std::pair<long long, long long>& y) {
                             return x.first < y.first;
                         });
        P->a_off_csr.assign(n_ent + 1, 0);
        P->a_src.resize(contrib.size());
        for (size_t i = 0; i < contrib.size(); ++i) {
            P->a_off_csr[contrib[i].first + 1]++;
            P->a_src[i] = contrib[i].second;
        }
        for (long long e = 0; e < n_ent; ++e) P->a_off_csr[e + 1] += P->a_off_csr[e];
        P->a_sub.resize(n_ent);
        P->a_row.resize(n_ent);
        P->a_col.resize(n_ent);
        for (int s = 0; s < d->n_sub; ++s) {
            const int n = P->subs[s].n;
            long long e = ent_base[s];
            for (int a = 0; a < n; ++a)
                for (int b = a; b < n; ++b, ++e) {
                    P->a_sub[e] = s;
                    P->a_row[e] = a;
                    P->a_col[e] = b;
                }
        }
    }

    // J^T W r and gradient per theta index; chi^2 per sub; dense-J scatter lists
    {
        std::vector<std::vector<int>> pc(d->n_par), ps(d->n_par);
        for (int c = 0; c < n_cols; ++c) pc[P->cols[c].par].push_back(c);
        for (int k = 0; k < d->n_images; ++k)
            if (P->images[k].sky_par >= 0) ps[P->images[k].sky_par].push_back(k);
        P->g_seg.assign(1, 0);
        P->gr_seg.assign(1, 0);
        P->par_off.assign(1, 0);
        P->par_sky_off.assign(1, 0);
        for (int p = 0; p < d->n_par; ++p) {
            for (int c : pc[p]) {
                const int g = P->cols[c].group;
                const DGroup& gr = P->groups[g];
                if (gram_part(g)) {
                    for (int gi : group_gitems[g]) {
                        P->g_idx.push_back((int)gram_src(gi, c - gr.col_begin, 0));
                        P->g_w.push_back(1.0);
                    }
                } else if (gr.oh > 0 && gr.ow > 0) {
                    P->g_idx.push_back((int)(P->asrc_col + 2LL * c));
                    P->g_w.push_back(1.0);
                }
                if (gr.type == GROUP_PSF) {
                    // d chi2 / d phi = -2 sum w r J_phi, from the column's JCOL partials
                    P->gr_idx.push_back((int)(P->asrc_col + 2LL * c));
                    P->gr_w.push_back(-2.0);
                } else {
                    P->gr_idx.push_back((int)(P->asrc_gcol + c));
                    P->gr_w.push_back(1.0);
                }
                P->par_cols.push_back(c);
            }
            for (int k : ps[p]) {
                P->g_idx.push_back((int)(P->asrc_img + 3LL * k + 1));
                P->g_w.push_back(1.0);
                P->gr_idx.push_back((int)(P->asrc_img + 3LL * k + 1));
                P->gr_w.push_back(-2.0);
                P->par_sky.push_back(k);
            }
            P->g_seg.push_back((int)P->g_idx.size());
            P->gr_seg.push_back((int)P->gr_idx.size());
            P->par_off.push_back((int)P->par_cols.size());
            P->par_sky_off.push_back((int)P->par_sky.size());
            P->g_sub.push_back(std::max(0, P->par_sub[p]));
        }
        P->chi_seg.assign(1, 0);
        for (int s = 0; s < d->n_sub; ++s) {
            for (int k = 0; k < d->n_images; ++k)
                if (P->images[k].sub == s) P->chi_idx.push_back((int)(P->asrc_img + 3LL * k));
            P->chi_seg.push_back((int)P->chi_idx.size());
        }
    }
    if ((long long)P->asrc_img + 3LL * d->n_images >= (1LL << 31))
        return fail(C, APX_E_UNSUPPORTED, "problem too large for 32-bit reduction indices");
    return APX_OK;
}

// ------------------------------------------------------------------ workspace
template <class T>
static size_t ws_take(apx_problem* P, const char* name, size_t count) {
    size_t o = P->L.take(count * sizeof(T) + 8);
    P->off[name] = o;
    return o;
}

static void layout(apx_problem* P) {
    P->L = Layout();
    P->off.clear();
    const int n_cols = (int)P->cols.size();
    ws_take<DImage>(P, "images", P->images.size());
    ws_take<DComp>(P, "comps", P->comps.size());
    ws_take<DGroup>(P, "groups", P->groups.size());
    ws_take<DCol>(P, "cols", P->cols.size());
    ws_take<DSub>(P, "subs", P->subs.size());
    ws_take<int>(P, "group_comps", P->group_comps.size());
    ws_take<RTile>(P, "rtiles", P->rtiles.size());
    ws_take<int>(P, "rtile_off", P->rtile_off.size());
    ws_take<int>(P, "rtile_comps", P->rtile_comps.size());
    ws_take<RTile>(P, "gtiles", P->gtiles.size());
    ws_take<ConvJob>(P, "fwd_jobs", P->fwd_jobs.size());
    ws_take<ConvItem>(P, "fwd_items", P->fwd_items.size());
    ws_take<ConvJob>(P, "jcol_jobs", P->jcol_jobs.size());
    ws_take<ConvItem>(P, "jcol_items", P->jcol_items.size());
    ws_take<ConvJob>(P, "psf_jobs", P->psf_jobs.size());
    ws_take<ConvItem>(P, "psf_items", P->psf_items.size());
    ws_take<ConvJob>(P, "adj_jobs", P->adj_jobs.size());
    ws_take<ConvItem>(P, "adj_items", P->adj_items.size());
    ws_take<DPair>(P, "pairs", P->pairs.size());
    ws_take<PairItem>(P, "pitems64", P->pitems64.size());
    ws_take<PairItem>(P, "pitems16", P->pitems16.size());
    ws_take<PairItem>(P, "gitems", P->gitems.size());
    ws_take<int>(P, "img_seg", P->img_seg.size());
    ws_take<int>(P, "img_idx", P->img_idx.size());
    ws_take<int>(P, "col_seg", P->col_seg.size());
    ws_take<int>(P, "col_idx", P->col_idx.size());
    ws_take<int>(P, "gcol_seg", P->gcol_seg.size());
    ws_take<int>(P, "chi_seg", P->chi_seg.size());
    ws_take<int>(P, "chi_idx", P->chi_idx.size());
    ws_take<int>(P, "g_seg", P->g_seg.size());
    ws_take<int>(P, "g_idx", P->g_idx.size());
    ws_take<double>(P, "g_w", P->g_w.size());
    ws_take<int>(P, "g_sub", P->g_sub.size());
    ws_take<int>(P, "gr_seg", P->gr_seg.size());
    ws_take<int>(P, "gr_idx", P->gr_idx.size());
    ws_take<double>(P, "gr_w", P->gr_w.size());
    ws_take<long long>(P, "a_off_csr", P->a_off_csr.size());
    ws_take<long long>(P, "a_src", P->a_src.size());
    ws_take<int>(P, "a_sub", P->a_sub.size());
    ws_take<int>(P, "a_row", P->a_row.size());
    ws_take<int>(P, "a_col", P->a_col.size());
    ws_take<int>(P, "par_sub", P->par_sub.size());
    ws_take<int>(P, "par_off", P->par_off.size());
    ws_take<int>(P, "par_cols", P->par_cols.size());
    ws_take<int>(P, "par_sky_off", P->par_sky_off.size());
    ws_take<int>(P, "par_sky", P->par_sky.size());
    ws_take<int>(P, "small_subs", P->small_subs.size());
    ws_take<double>(P, "bn_tab", P->bn_tab.size());
    ws_take<double>(P, "ptab", P->ptab.size());
    ws_take<float>(P, "psf_sep", P->psf_sep.size());
    ws_take<double>(P, "agl", P->agl.size());
    ws_take<AChunk>(P, "achunks", P->achunks.size());
    ws_take<int>(P, "acomp_chunk", P->acomp_chunk.size());
    ws_take<double>(P, "apart", P->achunks.size());
    ws_take<double>(P, "ae", P->agl.empty() ? 0 : P->comps.size());
    ws_take<double>(P, "av0", P->n_apix);
    ws_take<double>(P, "aval", P->n_apix);
    ws_take<int>(P, "aneed", P->n_apix);
    ws_take<int>(P, "acode", P->n_apix);
    ws_take<ARef>(P, "aref", P->n_apix);
    ws_take<float>(P, "adval", 7 * P->n_apix);
    ws_take<int>(P, "acount", 1);
    // buffers
    ws_take<CompConst>(P, "cc", P->comps.size());
    ws_take<double>(P, "stap", P->shift != APX_SHIFT_NONE ? STAP_STRIDE * P->comps.size() : 0);
    ws_take<float>(P, "S", P->n_ext);
    ws_take<double>(P, "S64", P->objective == APX_OBJECTIVE_FP64 ? P->n_ext : 0);
    ws_take<float>(P, "Abar", P->n_ext);
    ws_take<float>(P, "rbuf", P->n_pix);
    ws_take<float>(P, "D", P->n_d);
    ws_take<float>(P, "J", P->n_j);
    ws_take<float>(P, "psf_flip", P->n_psf);
    ws_take<double>(P, "fwd_part", 3 * P->fwd_items.size());
    ws_take<double>(P, "jcol_part", 2 * (P->jcol_items.size() + P->psf_items.size()));
    ws_take<float>(P, "psf_live", P->n_live);
    ws_take<double>(P, "psf64", P->n_psf);
    ws_take<float2>(P, "fft_spec", P->n_fft_spec);
    ws_take<float>(P, "fft_tw", P->fft_tw.size());
    ws_take<int4>(P, "fwd_pairs", P->fwd_pairs.size());
    ws_take<int4>(P, "jcol_pairs", P->jcol_pairs.size());
    ws_take<int4>(P, "adj_pairs", P->adj_pairs.size());
    ws_take<double>(P, "grad_part", P->n_gradpart);
    ws_take<double>(P, "asrc", P->asrc_img + 3LL * P->n_images);
    ws_take<double>(P, "A", P->a_total);
    ws_take<double>(P, "M", 2 * P->a_total);
    ws_take<double>(P, "gvec", P->n_par);
    ws_take<double>(P, "Ddiag", P->n_par);
    ws_take<double>(P, "hvec", 2 * P->n_par);
    ws_take<double>(P, "yvec", 2 * P->n_par);
    ws_take<double>(P, "theta_trial", P->n_par);
    ws_take<LMFlags>(P, "lmf", 2 * P->n_sub);
    ws_take<int>(P, "sflag", std::max(1, 2 * P->n_sflag));
    ws_take<double>(P, "chol_diag", 2 * (size_t)CHOL_NB * CHOL_NB * P->large_subs.size());
    ws_take<LMSpec>(P, "spec", P->n_sub);
    ws_take<int>(P, "sticky", 1);
    ws_take<double>(P, "sky_val", P->n_images);
    ws_take<double>(P, "seed_part", 64LL * P->n_images);
    ws_take<double>(P, "chi2_sub", P->n_sub);
    ws_take<double>(P, "chi2_trial", P->n_sub);
    ws_take<double>(P, "hmc_t0", P->n_par);
    ws_take<double>(P, "hmc_r", P->n_par);
    ws_take<double>(P, "hmc_g0", P->n_par);
    ws_take<double>(P, "hmc_g1", P->n_par);
    ws_take<double>(P, "hmc_c0", P->n_sub);
    ws_take<double>(P, "hmc_c1", P->n_sub);
    ws_take<double>(P, "hmc_h0", P->n_sub);
    // NUTS: per tree level an outer end, an inner end (theta, r, grad each) and a proposal;
    // the two trajectory edges; two velocities; reduction results
    ws_take<double>(P, "nuts_lvl", (size_t)(APX_NUTS_MAX_DEPTH + 1) * 7 * P->n_par);
    ws_take<double>(P, "nuts_edge", 6 * (size_t)P->n_par);
    ws_take<double>(P, "nuts_vel", 2 * (size_t)P->n_par);
    ws_take<double>(P, "nuts_dev", (sizeof(NutsDev) + sizeof(double) - 1) / sizeof(double));
    (void)n_cols;
}

template <class T>
static T* wsp(apx_problem* P, const char* name) {
    return reinterpret_cast<T*>(P->ws + P->off.at(name));
}

template <class T>
static hipError_t upload(apx_problem* P, const char* name, const std::vector<T>& v) {
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(wsp<T>(P, name), v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, P->ctx->stream);
}

// ------------------------------------------------------------------- C ABI
extern "C" {

const char* apx_version(void) { return "apx 0.1 (gfx950)"; }

const char* apx_status_string(apx_status s) {
    switch (s) {
        case APX_OK: return "ok";
        case APX_E_INVALID: return "invalid argument";
        case APX_E_HIP: return "HIP runtime error";
        case APX_E_NONFINITE: return "non-finite value";
        case APX_E_WORKSPACE: return "workspace missing or too small";
        case APX_E_UNSUPPORTED: return "unsupported configuration";
        case APX_E_DOMAIN: return "parameters outside the model domain";
        default: return "unknown status";
    }
}

apx_status apx_ctx_create(int device, void* hip_stream, apx_ctx** out) {
    if (!out) return APX_E_INVALID;
    *out = nullptr;
    if (device == -1) {                       // host-only: validate and plan, never launch
        apx_ctx* c = new apx_ctx();
        c->device = -1;
        *out = c;
        return APX_OK;
    }
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return APX_E_HIP;
    if (hipSetDevice(device) != hipSuccess) return APX_E_HIP;
    scratch_lookup(device);
    apx_ctx* c = new apx_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return APX_OK;
}

apx_status apx_ctx_set_stream(apx_ctx* ctx, void* hip_stream) {
    if (!ctx) return APX_E_INVALID;
    ctx->stream = (hipStream_t)hip_stream;
    return APX_OK;
}

apx_status apx_ctx_destroy(apx_ctx* ctx) {
    if (ctx && ctx->tune_mem) (void)hipFree(ctx->tune_mem);
    delete ctx;
    return APX_OK;
}

apx_status apx_ctx_set_tiles(apx_ctx* ctx, int32_t policy) {
    if (!ctx) return APX_E_INVALID;
    if (policy != APX_TILES_AUTOTUNE && policy != APX_TILES_MODEL &&
        !(policy >= APX_TILES_FIXED && policy < APX_TILES_FIXED + N_TILE_SHAPES))
        return fail(ctx, APX_E_INVALID, "unknown tile policy");
    ctx->tiles = policy;
    return APX_OK;
}

apx_status apx_ctx_tile_cost(const apx_ctx* ctx, int32_t kernel, int32_t P, double* us) {
    if (!ctx || !us || kernel < 0 || kernel > 3) return APX_E_INVALID;
    auto it = ctx->tile_us.find(kernel * 64 + P);
    if (it == ctx->tile_us.end()) return APX_E_INVALID;
    for (int s = 0; s < N_TILE_SHAPES; ++s) us[s] = it->second[s];
    return APX_OK;
}

apx_status apx_ctx_set_tile_cost(apx_ctx* ctx, int32_t kernel, int32_t P, const double* us) {
    if (!ctx || !us || kernel < 0 || kernel > 3 || P < 1 || P > APX_MAX_PSF || (P & 1) == 0)
        return APX_E_INVALID;
    std::array<double, 4> cost;
    for (int s = 0; s < N_TILE_SHAPES; ++s) {
        if (!(us[s] > 0.0) || !std::isfinite(us[s])) return APX_E_INVALID;
        cost[s] = us[s];
    }
    ctx->tile_us[kernel * 64 + P] = cost;
    return APX_OK;
}

const char* apx_last_error(const apx_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

apx_status apx_problem_create(apx_ctx* ctx, const apx_problem_desc* desc, apx_problem** out) {
    if (!ctx || !desc || !out) return APX_E_INVALID;
    *out = nullptr;
    apx_problem* P = new apx_problem();
    P->ctx = ctx;
    apx_status st;
    try {
        st = build_plan(P, desc);
    } catch (const std::exception& e) {
        st = fail(ctx, APX_E_INVALID, std::string("plan construction failed: ") + e.what());
    }
    if (st != APX_OK) {
        delete P;
        return st;
    }
    layout(P);
    *out = P;
    return APX_OK;
}

apx_status apx_problem_workspace_bytes(const apx_problem* P, uint64_t* bytes) {
    if (!P || !bytes) return APX_E_INVALID;
    *bytes = P->L.total;
    return APX_OK;
}

apx_status apx_problem_sizes(const apx_problem* P, int64_t* n_pix, int64_t* n_ext, int64_t* n_jac) {
    if (!P) return APX_E_INVALID;
    if (n_pix) *n_pix = P->n_pix;
    if (n_ext) *n_ext = P->n_ext;
    if (n_jac) *n_jac = P->n_j;
    return APX_OK;
}

apx_status apx_problem_bind_workspace(apx_problem* P, void* dev, uint64_t bytes) {
    if (!P) return APX_E_INVALID;
    if (P->ctx->device < 0) return fail(P->ctx, APX_E_INVALID, "host-only context cannot bind a workspace");
    if (!dev || bytes < P->L.total || ((uintptr_t)dev & 255) != 0)
        return fail(P->ctx, APX_E_WORKSPACE, "workspace null, misaligned or smaller than required");
    P->ws = (char*)dev;
    P->ws_bytes = bytes;
    P->on_scratch = false;
    HIPCHK(upload(P, "images", P->images));
    HIPCHK(upload(P, "comps", P->comps));
    HIPCHK(upload(P, "groups", P->groups));
    HIPCHK(upload(P, "cols", P->cols));
    HIPCHK(upload(P, "subs", P->subs));
    HIPCHK(upload(P, "group_comps", P->group_comps));
    HIPCHK(upload(P, "rtiles", P->rtiles));
    HIPCHK(upload(P, "rtile_off", P->rtile_off));
    HIPCHK(upload(P, "rtile_comps", P->rtile_comps));
    HIPCHK(upload(P, "gtiles", P->gtiles));
    HIPCHK(upload(P, "fwd_jobs", P->fwd_jobs));
    HIPCHK(upload(P, "fwd_items", P->fwd_items));
    HIPCHK(upload(P, "jcol_jobs", P->jcol_jobs));
    HIPCHK(upload(P, "jcol_items", P->jcol_items));
    HIPCHK(upload(P, "psf_jobs", P->psf_jobs));
    HIPCHK(upload(P, "psf_items", P->psf_items));
    HIPCHK(upload(P, "adj_jobs", P->adj_jobs));
    HIPCHK(upload(P, "adj_items", P->adj_items));
    HIPCHK(upload(P, "pairs", P->pairs));
    HIPCHK(upload(P, "pitems64", P->pitems64));
    HIPCHK(upload(P, "pitems16", P->pitems16));
    HIPCHK(upload(P, "gitems", P->gitems));
    HIPCHK(upload(P, "img_seg", P->img_seg));
    HIPCHK(upload(P, "img_idx", P->img_idx));
    HIPCHK(upload(P, "col_seg", P->col_seg));
    HIPCHK(upload(P, "col_idx", P->col_idx));
    HIPCHK(upload(P, "gcol_seg", P->gcol_seg));
    HIPCHK(upload(P, "chi_seg", P->chi_seg));
    HIPCHK(upload(P, "chi_idx", P->chi_idx));
    HIPCHK(upload(P, "g_seg", P->g_seg));
    HIPCHK(upload(P, "g_idx", P->g_idx));
    HIPCHK(upload(P, "g_w", P->g_w));
    HIPCHK(upload(P, "g_sub", P->g_sub));
    HIPCHK(upload(P, "gr_seg", P->gr_seg));
    HIPCHK(upload(P, "gr_idx", P->gr_idx));
    HIPCHK(upload(P, "gr_w", P->gr_w));
    HIPCHK(upload(P, "a_off_csr", P->a_off_csr));
    HIPCHK(upload(P, "a_src", P->a_src));
    HIPCHK(upload(P, "a_sub", P->a_sub));
    HIPCHK(upload(P, "a_row", P->a_row));
    HIPCHK(upload(P, "a_col", P->a_col));
    HIPCHK(upload(P, "par_sub", P->par_sub));
    HIPCHK(upload(P, "par_off", P->par_off));
    HIPCHK(upload(P, "par_cols", P->par_cols));
    HIPCHK(upload(P, "par_sky_off", P->par_sky_off));
    HIPCHK(upload(P, "par_sky", P->par_sky));
    HIPCHK(upload(P, "small_subs", P->small_subs));
    HIPCHK(upload(P, "bn_tab", P->bn_tab));
    HIPCHK(upload(P, "ptab", P->ptab));
    HIPCHK(upload(P, "psf_sep", P->psf_sep));
    HIPCHK(upload(P, "agl", P->agl));
    HIPCHK(upload(P, "fft_tw", P->fft_tw));
    HIPCHK(upload(P, "fwd_pairs", P->fwd_pairs));
    HIPCHK(upload(P, "jcol_pairs", P->jcol_pairs));
    HIPCHK(upload(P, "adj_pairs", P->adj_pairs));
    P->fft_fixed_ready = false;
    HIPCHK(upload(P, "achunks", P->achunks));
    HIPCHK(upload(P, "acomp_chunk", P->acomp_chunk));

    Plan& p = P->plan;
    p = Plan{};
    p.wait_spin_max = SUBST_SPIN_MAX;
    p.n_images = P->n_images;
    p.n_comps = P->n_comps;
    p.n_par = P->n_par;
    p.n_sub = P->n_sub;
    p.n_groups = (int)P->groups.size();
    p.n_cols = (int)P->cols.size();
    p.s = P->s;
    p.rule = P->rule;
    p.mode = P->mode;
    p.objective = P->objective;
    p.shift = P->shift;
    p.shift_a = P->shift_a;
    p.k_re = P->k_re;
    for (int k = 0; k < MAX_NODES_1D; ++k) {
        p.node_o[k] = k < (int)P->node_o.size() ? P->node_o[k] : 0.f;
        p.node_w[k] = k < (int)P->node_w.size() ? P->node_w[k] : 0.f;
        p.node_od[k] = k < (int)P->node_od.size() ? P->node_od[k] : 0.0;
        p.node_wd[k] = k < (int)P->node_wd.size() ? P->node_wd[k] : 0.0;
    }
    p.images = wsp<DImage>(P, "images");
    p.comps = wsp<DComp>(P, "comps");
    p.groups = wsp<DGroup>(P, "groups");
    p.cols = wsp<DCol>(P, "cols");
    p.subs = wsp<DSub>(P, "subs");
    p.group_comps = wsp<int>(P, "group_comps");
    p.psf = P->psf;
    p.psf_flip = wsp<float>(P, "psf_flip");
    p.rtiles = wsp<RTile>(P, "rtiles");
    p.n_rtiles = (int)P->rtiles.size();
    p.rtile_off = wsp<int>(P, "rtile_off");
    p.rtile_comps = wsp<int>(P, "rtile_comps");
    p.gtiles = wsp<RTile>(P, "gtiles");
    p.n_gtiles = (int)P->gtiles.size();
    p.cc = wsp<CompConst>(P, "cc");
    p.stap = wsp<double>(P, "stap");
    p.S = wsp<float>(P, "S");
    p.S64 = wsp<double>(P, "S64");
    p.Abar = wsp<float>(P, "Abar");
    p.rbuf = wsp<float>(P, "rbuf");
    p.D = wsp<float>(P, "D");
    p.J = wsp<float>(P, "J");
    p.fwd_part = wsp<double>(P, "fwd_part");
    p.jcol_part = wsp<double>(P, "jcol_part");
    p.psf_live = wsp<float>(P, "psf_live");
    p.psf64 = wsp<double>(P, "psf64");
    p.fft_spec = wsp<float2>(P, "fft_spec");
    p.fft_tw = reinterpret_cast<const float2*>(wsp<float>(P, "fft_tw"));
    p.grad_part = wsp<double>(P, "grad_part");
    P->asrc = wsp<double>(P, "asrc");
    p.pair_part = P->asrc;
    p.col_sum = P->asrc + P->asrc_col;
    p.grad_col = P->asrc + P->asrc_gcol;
    p.img_sum = P->asrc + P->asrc_img;
    p.A = wsp<double>(P, "A");
    p.M = wsp<double>(P, "M");
    p.gvec = wsp<double>(P, "gvec");
    p.Ddiag = wsp<double>(P, "Ddiag");
    p.hvec = wsp<double>(P, "hvec");
    p.yvec = wsp<double>(P, "yvec");
    p.theta_trial = wsp<double>(P, "theta_trial");
    p.lmf = wsp<LMFlags>(P, "lmf");
    p.sflag = wsp<int>(P, "sflag");
    p.chol_diag = wsp<double>(P, "chol_diag");
    p.spec = wsp<LMSpec>(P, "spec");
    p.a_total = P->a_total;
    p.n_sflag = P->n_sflag;
    p.n_large = (int)P->large_subs.size();
    p.sticky = wsp<int>(P, "sticky");
    p.sky_val = wsp<double>(P, "sky_val");
    p.par_sub = wsp<int>(P, "par_sub");
    p.bn_tab = wsp<double>(P, "bn_tab");
    p.ptab = wsp<double>(P, "ptab");
    p.psf_sep = wsp<float>(P, "psf_sep");
    p.agl = wsp<double>(P, "agl");
    p.achunks = wsp<AChunk>(P, "achunks");
    p.n_achunks = (int)P->achunks.size();
    p.acomp_chunk = wsp<int>(P, "acomp_chunk");
    p.apart = wsp<double>(P, "apart");
    p.ae = wsp<double>(P, "ae");
    p.av0 = wsp<double>(P, "av0");
    p.aval = wsp<double>(P, "aval");
    p.aneed = wsp<int>(P, "aneed");
    p.acode = wsp<int>(P, "acode");
    p.aref = wsp<ARef>(P, "aref");
    p.adval = wsp<float>(P, "adval");
    p.acount = wsp<int>(P, "acount");
    p.n_apix = P->n_apix;
    p.n_pix = P->n_pix;
    p.n_ext = P->n_ext;
    P->chi2_sub = wsp<double>(P, "chi2_sub");
    P->chi2_trial = wsp<double>(P, "chi2_trial");
    HIPCHK(hipMemsetAsync(p.sticky, 0, sizeof(int), P->ctx->stream));
    HIPCHK(hipMemsetAsync(p.lmf, 0, sizeof(LMFlags) * 2 * P->n_sub, P->ctx->stream));
    HIPCHK(hipMemsetAsync(p.spec, 0, sizeof(LMSpec) * P->n_sub, P->ctx->stream));
    P->bound = true;
    return APX_OK;
}

apx_status apx_problem_bind_scratch(apx_problem* P) {
    if (!P) return APX_E_INVALID;
    const int dev = P->ctx->device;
    if (dev < 0) return fail(P->ctx, APX_E_INVALID, "host-only context cannot bind the scratch");
    if (dev >= APX_SCRATCH_DEVICES) return fail(P->ctx, APX_E_UNSUPPORTED, "device index beyond the scratch table");
    if (P->L.total > APX_SCRATCH_BYTES)
        return fail(P->ctx, APX_E_WORKSPACE,
                    "the problem needs " + std::to_string(P->L.total) + " bytes of workspace; the library scratch holds " +
                        std::to_string(APX_SCRATCH_BYTES) + " (bind a caller workspace instead)");
    void* ptr = nullptr;
    uint64_t gen = 0;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        ScratchSlot& sl = g_scratch[dev];
        if (!sl.looked_up || sl.status != hipSuccess || !sl.ptr)
            return fail(P->ctx, APX_E_HIP, std::string("scratch address lookup failed: ") +
                                               (sl.looked_up ? hipGetErrorString(sl.status) : "not looked up"));
        ptr = sl.ptr;
        gen = ++sl.generation;
    }
    // the previous user of the scratch may still run on another stream of this device
    HIPCHK(hipDeviceSynchronize());
    const apx_status st = apx_problem_bind_workspace(P, ptr, APX_SCRATCH_BYTES);
    if (st != APX_OK) return st;
    P->on_scratch = true;
    P->scratch_gen = gen;
    return APX_OK;
}

apx_status apx_problem_tile_shapes(const apx_problem* P, int32_t kind, int32_t* counts) {
    if (!P || !counts || kind < 0 || kind > 2) return APX_E_INVALID;
    const std::vector<ConvJob>& jobs = kind == 0 ? P->fwd_jobs : kind == 1 ? P->jcol_jobs : P->adj_jobs;
    for (int s = 0; s <= SHAPE_SEP; ++s) counts[s] = 0;
    for (const ConvJob& jb : jobs)
        if (jb.out_h > 0 && jb.out_w > 0) counts[jb.shape] += 1;
    return APX_OK;
}

apx_status apx_problem_check(apx_problem* P) {
    if (!P || !P->bound) return APX_E_WORKSPACE;
    int flags = 0;
    HIPCHK(hipStreamSynchronize(P->ctx->stream));
    HIPCHK(hipMemcpy(&flags, P->plan.sticky, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemset(P->plan.sticky, 0, sizeof(int)));
    if (flags & FLAG_STALL)
        return fail(P->ctx, APX_E_HIP, "a substitution hand-off wait ran out (the step was dropped)");
    if (flags & FLAG_DOMAIN) return APX_E_DOMAIN;
    if (flags & FLAG_NONFINITE) return APX_E_NONFINITE;
    return APX_OK;
}

apx_status apx_problem_set_timing_classes(apx_problem* P, uint32_t mask) {
    if (!P) return APX_E_INVALID;
    if (P->capturing) return fail(P->ctx, APX_E_INVALID, "timing cannot change during capture");
    P->timing_mask = mask & ((1u << APX_TIME_CLASSES) - 1u);
    P->timing = P->timing_mask != 0;
    P->ev_used = 0;
    P->ev_recs.clear();
    return APX_OK;
}

apx_status apx_problem_set_timing(apx_problem* P, int32_t enabled) {
    return apx_problem_set_timing_classes(P, enabled ? (1u << APX_TIME_CLASSES) - 1u : 0u);
}

apx_status apx_problem_timing(apx_problem* P, int32_t klass, double* total_ms, int64_t* launches) {
    if (!P || !total_ms || !launches || klass < 0 || klass >= APX_TIME_CLASSES) return APX_E_INVALID;
    HIPCHK(hipStreamSynchronize(P->ctx->stream));
    double tot = 0.0;
    int64_t n = 0;
    for (const auto& r : P->ev_recs) {
        if (r.first != klass) continue;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, P->ev_pool[r.second], P->ev_pool[r.second + 1]));
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    return APX_OK;
}

apx_status apx_problem_set_wait_limit(apx_problem* P, int32_t polls) {
    if (!P || !P->bound) return APX_E_WORKSPACE;
    if (P->capturing) return fail(P->ctx, APX_E_INVALID, "the wait limit cannot change during capture");
    HIPCHK(hipStreamSynchronize(P->ctx->stream));
    P->plan.wait_spin_max = polls == 0 ? SUBST_SPIN_MAX : polls;
    drop_graph(P);                      // a captured iteration holds the old plan
    return APX_OK;
}

apx_status apx_problem_destroy(apx_problem* P) {
    if (!P) return APX_OK;
    if (P->ctx && P->ctx->stream) hipStreamSynchronize(P->ctx->stream);
    drop_graph(P);
    for (hipEvent_t e : P->ev_pool) hipEventDestroy(e);
    delete P;
    return APX_OK;
}

}  // extern "C"

// ------------------------------------------------------------ launch sequences
static apx_status run_conv(apx_problem* P, int kind, const ConvIO& io) {
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    const std::vector<PRange>* ranges;
    const char *jn, *inn;
    if (kind == CONV_FWD) { ranges = &P->fwd_ranges; jn = "fwd_jobs"; inn = "fwd_items"; }
    else if (kind == CONV_JCOL) { ranges = &P->jcol_ranges; jn = "jcol_jobs"; inn = "jcol_items"; }
    else if (kind == CONV_JCOL_PSF) { ranges = &P->psf_ranges; jn = "psf_jobs"; inn = "psf_items"; }
    else { ranges = &P->adj_ranges; jn = "adj_jobs"; inn = "adj_items"; }
    const int klass = kind == CONV_FWD ? APX_TIME_CONV_FWD
                    : (kind == CONV_JCOL || kind == CONV_JCOL_PSF) ? APX_TIME_CONV_JCOL : APX_TIME_CONV_ADJ;
    const char* pn = kind == CONV_FWD ? "fwd_pairs" : kind == CONV_JCOL ? "jcol_pairs" : "adj_pairs";
    for (const PRange& r : *ranges) {
        TimeScope ts(P, r.shape == SHAPE_SEP ? APX_TIME_CONV_SEP : r.shape == SHAPE_FFT ? APX_TIME_CONV_FFT : klass);
        ConvLaunch L{wsp<ConvJob>(P, jn), wsp<ConvItem>(P, inn), r.begin, r.count, r.P, r.shape, nullptr,
                     r.pair_begin, r.pair_count};
        if (r.shape == SHAPE_SEP) {
            hipError_t e = launch_conv_sep(p, L, io, st);
            if (e != hipSuccess) return fail(P->ctx, APX_E_HIP, std::string("separable conv launch: ") + hipGetErrorString(e));
            continue;
        }
        if (r.shape == SHAPE_FFT) {
            L.pairs = wsp<int4>(P, pn);
            hipError_t e = launch_conv_fft(p, kind, L, io, st);
            if (e != hipSuccess) return fail(P->ctx, APX_E_HIP, std::string("FFT conv launch: ") + hipGetErrorString(e));
            continue;
        }
        hipError_t e = kind == CONV_FWD ? (P->objective == APX_OBJECTIVE_FP64 ? launch_conv_fwd64(p, L, io, st)
                                                                               : launch_conv_fwd(p, L, io, st))
                     : (kind == CONV_JCOL || kind == CONV_JCOL_PSF) ? launch_conv_jcol(p, L, io, st)
                                         : launch_conv_adj(p, L, io, st);
        if (e != hipSuccess) return fail(P->ctx, APX_E_HIP, std::string("conv launch: ") + hipGetErrorString(e));
    }
    return APX_OK;
}

#define APXCHK(expr)                          \
    do {                                      \
        apx_status _s = (expr);               \
        if (_s != APX_OK) return _s;          \
    } while (0)

static SegSum segsum_base() {
    SegSum a{};
    a.stride = 1;
    a.ostride = 1;
    a.scale = 1.0;
    return a;
}

// Per-theta constants (component constants, stamps) and, in adaptive mode, the
// integration choices and values; want_grad: the refined pixels' derivatives too.
static apx_status prep(apx_problem* P, const double* theta, int lm_trial, int skip_mode,
                       const apx_lm_state* lm, int want_grad) {
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    {
        TimeScope ts(P, APX_TIME_PREP);
        HIPCHK(launch_prep(p, theta, lm_trial, st));
        if (P->fft_live < 0) {
            P->fft_live = 0;
            for (const DImage& im : P->images) P->fft_live += im.fft_off >= 0 && im.live ? 1 : 0;
        }
        // stamp spectra: live stamps per theta, fixed once (no launch once only fixed ones remain)
        if (P->n_fft_images > 0 && (!P->fft_fixed_ready || P->fft_live > 0)) {
            HIPCHK(launch_fft_stamps(p, P->fft_fixed_ready ? 1 : 0, st));
            P->fft_fixed_ready = true;
        }
    }
    if (P->mode == APX_MODE_ADAPTIVE) {
        TimeScope ts(P, APX_TIME_RENDER);
        HIPCHK(launch_adapt(p, skip_mode, lm, want_grad, st));
    }
    return APX_OK;
}

// Forward model + residual partials, reduced to img_sum (3 per image) and chi2[n_sub].
static apx_status fwd_chi2(apx_problem* P, const double* theta, const float* data, const float* weight,
                           float* model, double* chi2_out, int lm_trial, int skip_mode,
                           const apx_lm_state* lm, int want_grad) {
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    APXCHK(prep(P, theta, lm_trial, skip_mode, lm, want_grad));
    {
        TimeScope ts(P, APX_TIME_RENDER);
        if (P->objective == APX_OBJECTIVE_FP64) HIPCHK(launch_render64(p, skip_mode, lm, st));
        else HIPCHK(launch_render_mode(p, skip_mode, lm, st));
    }
    ConvIO io{};
    io.in = p.S;
    io.in64 = p.S64;
    io.out = model;
    io.data = data;
    io.weight = weight;
    io.part = p.fwd_part;
    io.skip_mode = skip_mode;
    io.lm = lm;
    APXCHK(run_conv(P, CONV_FWD, io));
    if (data) {
        TimeScope ts(P, APX_TIME_REDUCE);
        {
            SegSum a = segsum_base();               // sum w r^2, sum w r, sum w per image
            a.src = p.fwd_part;
            a.stride = 3;
            a.ncomp = 3;
            a.seg = wsp<int>(P, "img_seg");
            a.idx = wsp<int>(P, "img_idx");
            a.n_seg = P->n_images;
            a.out = p.img_sum;
            a.ostride = 3;
            HIPCHK(launch_segsum(a, st));
        }
        if (chi2_out) {
            SegSum a = segsum_base();
            a.src = P->asrc;
            a.seg = wsp<int>(P, "chi_seg");
            a.idx = wsp<int>(P, "chi_idx");
            a.n_seg = P->n_sub;
            a.out = chi2_out;
            HIPCHK(launch_segsum(a, st));
        }
    }
    return APX_OK;
}

// Derivative images and Jacobian blocks (with sum w r J, sum w J partials if weight).
// Live-PSF Jacobian columns (dK/dphi) * S: the FP32 pre-convolution model S at theta,
// then its convolutions with the derivative stamps, with Sigma w r J, Sigma w J partials
// after those of the main Jacobian list.
static apx_status psf_columns(apx_problem* P, const float* weight, int skip_mode, const apx_lm_state* lm) {
    if (!P->has_live_cols) return APX_OK;
    const Plan& p = P->plan;
    {
        TimeScope ts(P, APX_TIME_RENDER);
        HIPCHK(launch_render_mode(p, skip_mode, lm, P->ctx->stream));
    }
    ConvIO io{};
    io.in_s = p.S;
    io.out = p.J;
    io.weight = weight;
    io.part = p.jcol_part + 2 * P->jcol_items.size();
    io.skip_mode = skip_mode;
    io.lm = lm;
    return run_conv(P, CONV_JCOL_PSF, io);
}

static apx_status col_sums(apx_problem* P) {
    const Plan& p = P->plan;
    TimeScope ts(P, APX_TIME_REDUCE);
    SegSum a = segsum_base();                       // sum w r J, sum w J per column
    a.src = p.jcol_part;
    a.stride = 2;
    a.ncomp = 2;
    a.seg = wsp<int>(P, "col_seg");
    a.idx = wsp<int>(P, "col_idx");
    a.n_seg = (int)P->cols.size();
    a.out = p.col_sum;
    a.ostride = 2;
    HIPCHK(launch_segsum(a, P->ctx->stream));
    return APX_OK;
}

static apx_status jac_blocks(apx_problem* P, const float* weight, const apx_lm_state* lm) {
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    {
        TimeScope ts(P, APX_TIME_DERIV);
        HIPCHK(launch_deriv(p, lm, st));
    }
    ConvIO io{};
    io.in = p.D;
    io.out = p.J;
    io.weight = weight;
    io.part = p.jcol_part;
    io.skip_mode = lm ? 2 : 0;
    io.lm = lm;
    APXCHK(run_conv(P, CONV_JCOL, io));
    APXCHK(psf_columns(P, weight, lm ? 2 : 0, lm));
    if (weight) APXCHK(col_sums(P));
    return APX_OK;
}

// J^T W J and J^T W r into A_out / g_out from the stored blocks and partials.
static apx_status normal_eq(apx_problem* P, const float* weight, double* A_out, double* g_out,
                            const apx_lm_state* lm) {
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    PairLaunch L64{wsp<DPair>(P, "pairs"), wsp<PairItem>(P, "pitems64"), (int)P->pitems64.size(), 64};
    PairLaunch L16{wsp<DPair>(P, "pairs"), wsp<PairItem>(P, "pitems16"), (int)P->pitems16.size(), 16};
    {
        TimeScope ts(P, APX_TIME_PAIRS);
        HIPCHK(launch_pairs(p, L64, weight, lm, st));
        HIPCHK(launch_pairs(p, L16, weight, lm, st));
        for (int t = 1; t <= GRAM4_MAX_T; ++t) {
            const int b = P->gram_begin[t], n = P->gram_begin[t + 1] - b;
            if (n <= 0) continue;
            PairLaunch G4{wsp<DPair>(P, "pairs"), wsp<PairItem>(P, "gitems") + b, n, t};
            HIPCHK(launch_gram4(p, G4, weight, lm, st));
        }
    }
    TimeScope ts(P, APX_TIME_REDUCE);
    AsmA a{};
    a.ent_off = wsp<long long>(P, "a_off_csr");
    a.ent_sub = wsp<int>(P, "a_sub");
    a.ent_row = wsp<int>(P, "a_row");
    a.ent_col = wsp<int>(P, "a_col");
    a.ent_src = wsp<long long>(P, "a_src");
    a.n_ent = (long long)P->a_sub.size();
    a.src = P->asrc;
    a.subs = p.subs;
    a.out = A_out;
    a.lm = lm;
    HIPCHK(launch_assemble_A(a, st));
    SegSum g = segsum_base();
    g.src = P->asrc;
    g.seg = wsp<int>(P, "g_seg");
    g.idx = wsp<int>(P, "g_idx");
    g.wts = wsp<double>(P, "g_w");
    g.n_seg = P->n_par;
    g.out = g_out;
    g.seg_sub = wsp<int>(P, "g_sub");
    g.lm = lm;
    HIPCHK(launch_segsum(g, st));
    return APX_OK;
}

static apx_status ready(apx_problem* P) {
    if (!P) return APX_E_INVALID;
    if (!P->bound) return fail(P->ctx, APX_E_WORKSPACE, "no workspace bound");
    if (P->on_scratch) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (g_scratch[P->ctx->device].generation != P->scratch_gen)
            return fail(P->ctx, APX_E_WORKSPACE, "another problem has been bound to the library scratch since");
    }
    return APX_OK;
}

extern "C" {

// Buffers sized by n_par may be null when there are no free parameters.
static bool par_ok(const apx_problem* P, const void* ptr) { return ptr != nullptr || P->n_par == 0; }

apx_status apx_render(apx_problem* P, const double* theta, float* model) {
    APXCHK(ready(P));
    if (!par_ok(P, theta) || !model) return fail(P->ctx, APX_E_INVALID, "null pointer");
    return fwd_chi2(P, theta, nullptr, nullptr, model, nullptr, 0, 0, nullptr, 0);
}

apx_status apx_chi2(apx_problem* P, const double* theta, const float* data, const float* weight,
                    double* chi2) {
    APXCHK(ready(P));
    if (!par_ok(P, theta) || !data || !weight || !chi2) return fail(P->ctx, APX_E_INVALID, "null pointer");
    APXCHK(fwd_chi2(P, theta, data, weight, nullptr, chi2, 0, 0, nullptr, 0));
    HIPCHK(launch_chi2_check(chi2, P->n_sub, P->plan.sticky, P->ctx->stream));
    return APX_OK;
}

apx_status apx_jacobian(apx_problem* P, const double* theta, float* J, int64_t ldJ) {
    APXCHK(ready(P));
    if (!par_ok(P, theta) || !par_ok(P, J)) return fail(P->ctx, APX_E_INVALID, "null pointer");
    if (ldJ < P->n_pix) return fail(P->ctx, APX_E_INVALID, "ldJ < n_pix");
    hipStream_t st = P->ctx->stream;
    APXCHK(prep(P, theta, 0, 0, nullptr, 1));
    APXCHK(jac_blocks(P, nullptr, nullptr));
    HIPCHK(launch_jscatter(P->plan, wsp<int>(P, "par_off"), wsp<int>(P, "par_cols"), wsp<int>(P, "par_sky_off"),
                           wsp<int>(P, "par_sky"), J, ldJ, st));
    return APX_OK;
}

apx_status apx_jtwj(apx_problem* P, const double* theta, const float* data, const float* weight,
                    double* JtWJ, double* JtWr, double* chi2) {
    APXCHK(ready(P));
    if (!par_ok(P, theta) || !data || !weight || !par_ok(P, JtWJ) || !par_ok(P, JtWr) || !chi2)
        return fail(P->ctx, APX_E_INVALID, "null pointer");
    APXCHK(fwd_chi2(P, theta, data, weight, nullptr, chi2, 0, 0, nullptr, 1));
    APXCHK(jac_blocks(P, weight, nullptr));
    APXCHK(normal_eq(P, weight, JtWJ, JtWr, nullptr));
    HIPCHK(launch_chi2_check(chi2, P->n_sub, P->plan.sticky, P->ctx->stream));
    return APX_OK;
}

}  // extern "C"

// A^{-1} (factor = 0) or F = L^{-T} with A = L L^T (factor = 1) of every sub-problem's
// J^T W J at theta, into out (per-sub blocks at a_off).
static apx_status cov_core(apx_problem* P, const double* theta, const float* data, const float* weight,
                           double* out, double* chi2, int factor) {
    APXCHK(ready(P));
    if (!par_ok(P, theta) || !data || !weight || !par_ok(P, out) || !chi2)
        return fail(P->ctx, APX_E_INVALID, "null pointer");
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    APXCHK(fwd_chi2(P, theta, data, weight, nullptr, chi2, 0, 0, nullptr, 1));
    APXCHK(jac_blocks(P, weight, nullptr));
    APXCHK(normal_eq(P, weight, p.A, p.gvec, nullptr));
    {
        TimeScope ts(P, APX_TIME_SOLVE);
        HIPCHK(launch_cov_small(p, wsp<int>(P, "small_subs"), (int)P->small_subs.size(), P->nmax_small, out,
                                factor, st));
        for (int s : P->large_subs) {
            const int n = P->subs[s].n;
            HIPCHK(launch_chol_reset(p, s, st));
            HIPCHK(launch_cov_fill(p, s, n, st));
            HIPCHK(launch_chol_blocks(p, s, n, st));
            HIPCHK(launch_cov_cols(p, s, n, out, factor, st));
            if (factor) HIPCHK(launch_cov_transpose(p, s, n, out, st));
        }
    }
    HIPCHK(launch_chi2_check(chi2, P->n_sub, p.sticky, st));
    return APX_OK;
}

extern "C" {

apx_status apx_covariance(apx_problem* P, const double* theta, const float* data, const float* weight,
                          double* cov, double* chi2) {
    return cov_core(P, theta, data, weight, cov, chi2, 0);
}

apx_status apx_covariance_factor(apx_problem* P, const double* theta, const float* data, const float* weight,
                                 double* F, double* chi2) {
    return cov_core(P, theta, data, weight, F, chi2, 1);
}

}  // extern "C"

// chi2 and d chi2 / d theta at theta; lm_trial = 1 marks out-of-domain sub-problems in their
// trial flags instead of the sticky error flags (sampler trajectories).
static apx_status grad_core(apx_problem* P, const double* theta, const float* data, const float* weight,
                            double* grad, double* chi2, int lm_trial) {
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    APXCHK(fwd_chi2(P, theta, data, weight, nullptr, chi2, lm_trial, 0, nullptr, 1));
    HIPCHK(launch_flip_psf(p, st));
    ConvIO io{};
    io.out = p.Abar;
    io.weight = weight;
    APXCHK(run_conv(P, CONV_ADJ, io));
    {
        TimeScope ts(P, APX_TIME_GRAD);
        HIPCHK(launch_grad_tiles(p, st));
    }
    SegSum a = segsum_base();
    a.src = p.grad_part;
    a.seg = wsp<int>(P, "gcol_seg");
    a.n_seg = (int)P->cols.size();
    a.out = p.grad_col;
    HIPCHK(launch_segsum(a, st));
    if (P->has_live_cols) {                 // live-PSF columns: -2 sum w r J from their convolutions
        APXCHK(psf_columns(P, weight, 0, nullptr));
        APXCHK(col_sums(P));
    }
    SegSum g = segsum_base();
    g.src = P->asrc;
    g.seg = wsp<int>(P, "gr_seg");
    g.idx = wsp<int>(P, "gr_idx");
    g.wts = wsp<double>(P, "gr_w");
    g.n_seg = P->n_par;
    g.out = grad;
    HIPCHK(launch_segsum(g, st));
    return APX_OK;
}

extern "C" {

apx_status apx_chi2_grad(apx_problem* P, const double* theta, const float* data, const float* weight,
                         double* grad, double* chi2) {
    APXCHK(ready(P));
    if (!par_ok(P, theta) || !data || !weight || !par_ok(P, grad) || !chi2)
        return fail(P->ctx, APX_E_INVALID, "null pointer");
    APXCHK(grad_core(P, theta, data, weight, grad, chi2, 0));
    HIPCHK(launch_chi2_check(chi2, P->n_sub, P->plan.sticky, P->ctx->stream));
    return APX_OK;
}

}  // extern "C"

namespace {

// A point of a NUTS trajectory: theta, whitened momentum, d chi2 / d theta (device vectors).
struct NPoint { double *t, *r, *g; };

static NutsCopy copies(std::initializer_list<std::pair<double*, const double*>> l) {
    NutsCopy c{};
    for (const auto& e : l) {
        c.dst[c.n] = e.first;
        c.src[c.n] = e.second;
        ++c.n;
    }
    return c;
}
static NutsCopy copy3(const NPoint& d, const NPoint& s) { return copies({{d.t, s.t}, {d.r, s.r}, {d.g, s.g}}); }

// The slice-sampling NUTS of one chain.  The tree of a doubling is walked on the host in a
// fixed order (the recursion of Hoffman & Gelman: a subtree of depth j is its first half,
// then, unless that stopped, its second half, a draw between their proposals and a U-turn
// test of its ends); every step is a launch that acts only if the tree has not stopped
// (NutsDev), so the host waits once per doubling.  Leaves after a stop still run the
// gradient pass, on the last point computed, and change nothing.
struct Nuts {
    apx_problem* P;
    const float *data, *weight;
    const double *F, *Ft;
    double step;
    const double* u;          // this transition's uniforms (device)
    const double* uh;         // the same, host copy (the doubling directions)
    NPoint outer[APX_NUTS_MAX_DEPTH + 1], inner[APX_NUTS_MAX_DEPTH + 1];
    double* prop[APX_NUTS_MAX_DEPTH + 1];
    double *vel_m, *vel_p, *chi2;
    NutsDev* dev;
    NutsDev host;             // as read after the last doubling
    long long n;

    // one leapfrog step of size v * step from src into outer[0]
    apx_status leaf(const NPoint& src, double v) {
        const Plan& p = P->plan;
        hipStream_t st = P->ctx->stream;
        const NPoint& dst = outer[0];
        const int* stop = &dev->stop;
        HIPCHK(launch_nuts_copy(stop, 0, copy3(dst, src), n, st));
        HIPCHK(launch_hmc_matvec(p, F, dst.g, dst.r, -0.25 * v * step, st, stop));
        HIPCHK(launch_hmc_matvec(p, Ft, dst.r, dst.t, v * step, st, stop));
        APXCHK(grad_core(P, dst.t, data, weight, dst.g, chi2, 1));
        HIPCHK(launch_hmc_matvec(p, F, dst.g, dst.r, -0.25 * v * step, st, stop));
        HIPCHK(launch_nuts_leaf(p, dev, chi2, dst.r, st));
        return APX_OK;
    }
    // U-turn test of the trajectory (m, pp) when *flag == want
    apx_status uturn(const NPoint& m, const NPoint& pp, const int* flag, int want) {
        const Plan& p = P->plan;
        hipStream_t st = P->ctx->stream;
        HIPCHK(launch_fill(vel_m, n, 0.0, st));
        HIPCHK(launch_fill(vel_p, n, 0.0, st));
        HIPCHK(launch_hmc_matvec(p, Ft, m.r, vel_m, 1.0, st));
        HIPCHK(launch_hmc_matvec(p, Ft, pp.r, vel_p, 1.0, st));
        HIPCHK(launch_nuts_uturn(p, m.t, pp.t, vel_m, vel_p, dev, flag, want, st));
        return APX_OK;
    }
    // ends and proposal of the subtree of depth j (outer[0] for a leaf)
    NPoint outer_of(int j) const { return outer[j]; }
    NPoint inner_of(int j) const { return j == 0 ? outer[0] : inner[j]; }
    double* prop_of(int j) const { return j == 0 ? outer[0].t : prop[j]; }

    // Subtree of 2^j steps in direction v from src, entered when *entry != 0.
    apx_status build(const NPoint& src, double v, int j, const int* entry) {
        if (j == 0) return leaf(src, v);
        hipStream_t st = P->ctx->stream;
        APXCHK(build(src, v, j - 1, entry));
        const NPoint i1 = inner_of(j - 1), o1 = outer_of(j - 1);
        const NutsCopy keep = copies({{inner[j].t, i1.t}, {inner[j].r, i1.r}, {inner[j].g, i1.g},
                                      {outer[j].t, o1.t}, {outer[j].r, o1.r}, {outer[j].g, o1.g},
                                      {prop[j], prop_of(j - 1)}});
        HIPCHK(launch_nuts_level(dev, j, entry, keep, n, st));
        APXCHK(build(outer[j], v, j - 1, &dev->gate[j]));
        HIPCHK(launch_nuts_merge(dev, j, u, copies({{prop[j], prop_of(j - 1)}}), copy3(outer[j], outer_of(j - 1)), n, st));
        return v < 0 ? uturn(outer[j], inner[j], &dev->gate[j], 1) : uturn(inner[j], outer[j], &dev->gate[j], 1);
    }
};

}  // namespace

// Workspace views of the NUTS state; F^T goes to the LM's Cholesky scratch.
static apx_status nuts_setup(apx_problem* P, Nuts& N, const float* data, const float* weight, const double* F,
                             double step, NPoint& em, NPoint& ep) {
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    const long long n = P->n_par;
    N = Nuts{};
    N.P = P;
    N.data = data;
    N.weight = weight;
    N.F = F;
    N.Ft = p.M;
    N.step = step;
    N.n = n;
    double* lvl = wsp<double>(P, "nuts_lvl");
    for (int j = 0; j <= APX_NUTS_MAX_DEPTH; ++j) {
        double* b = lvl + (long long)j * 7 * n;
        N.outer[j] = NPoint{b, b + n, b + 2 * n};
        N.inner[j] = NPoint{b + 3 * n, b + 4 * n, b + 5 * n};
        N.prop[j] = b + 6 * n;
    }
    double* ed = wsp<double>(P, "nuts_edge");
    em = NPoint{ed, ed + n, ed + 2 * n};
    ep = NPoint{ed + 3 * n, ed + 4 * n, ed + 5 * n};
    N.vel_m = wsp<double>(P, "nuts_vel");
    N.vel_p = N.vel_m + n;
    N.dev = (NutsDev*)wsp<double>(P, "nuts_dev");
    N.chi2 = wsp<double>(P, "hmc_c1");
    HIPCHK(launch_hmc_transpose(p, F, p.M, st));
    HIPCHK(launch_clear_trial_flags(p, st));
    return APX_OK;
}

// One transition from theta (updated in place to the new sample) with momentum z and the
// uniforms u (device) / uh (host copy); first: the start's domain violations raise the
// sticky flag.  st = (depth, leapfrog steps, slice points, divergent, alpha, n_alpha).
static apx_status nuts_transition(Nuts& N, const NPoint& em, const NPoint& ep, double* theta, const double* z,
                                  const double* u, const double* uh, int max_depth, bool first, double st[6]) {
    apx_problem* P = N.P;
    const Plan& p = P->plan;
    hipStream_t s = P->ctx->stream;
    const long long n = N.n;
    N.u = u;
    N.uh = uh;
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(em.t, theta, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(em.r, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    APXCHK(grad_core(P, em.t, N.data, N.weight, em.g, N.chi2, first ? 0 : 1));
    HIPCHK(launch_nuts_start(p, N.dev, N.chi2, em.r, u, s));
    HIPCHK(launch_nuts_copy(nullptr, 0, copy3(ep, em), n, s));
    int k = 1, depth = 0;
    bool go = true;
    while (go && depth < max_depth) {
        const double v = uh[k] < 0.5 ? -1.0 : 1.0;
        HIPCHK(launch_nuts_doubling(N.dev, s));
        const NPoint& edge = v < 0 ? em : ep;
        APXCHK(N.build(edge, v, depth, &N.dev->one));
        HIPCHK(launch_nuts_top(N.dev, depth, u, copy3(edge, N.outer_of(depth)),
                               copies({{theta, N.prop_of(depth)}}), n, s));
        APXCHK(N.uturn(em, ep, &N.dev->stop, 0));
        HIPCHK(hipMemcpyAsync(&N.host, N.dev, sizeof(NutsDev), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        go = N.host.stop == 0;
        k = N.host.k;
        ++depth;
    }
    st[0] = depth;
    st[1] = N.host.steps;
    st[2] = (double)N.host.cnt;
    st[3] = N.host.divergent;
    st[4] = N.host.alpha;
    st[5] = N.host.n_alpha;
    return APX_OK;
}

static apx_status nuts_args(apx_problem* P, const float* data, const float* weight, const double* theta,
                            const double* F, double step, int32_t max_depth, int32_t n, const double* z,
                            const double* u) {
    APXCHK(ready(P));
    if (!data || !weight || !par_ok(P, theta) || !par_ok(P, F) || (n > 0 && (!par_ok(P, z) || !u)))
        return fail(P->ctx, APX_E_INVALID, "null pointer");
    if (max_depth < 1 || max_depth > APX_NUTS_MAX_DEPTH || n < 0 || !(step > 0.0) || !std::isfinite(step))
        return fail(P->ctx, APX_E_INVALID, "need 1 <= max_depth <= APX_NUTS_MAX_DEPTH, n >= 0, step > 0");
    return APX_OK;
}

static apx_status host_uniforms(apx_problem* P, const double* u, long long count, std::vector<double>& uh) {
    uh.resize((size_t)count);
    HIPCHK(hipMemcpyAsync(uh.data(), u, uh.size() * sizeof(double), hipMemcpyDeviceToHost, P->ctx->stream));
    HIPCHK(hipStreamSynchronize(P->ctx->stream));
    return APX_OK;
}

extern "C" {

apx_status apx_nuts_run(apx_problem* P, const float* data, const float* weight, double* theta, const double* F,
                        double step, int32_t max_depth, int32_t n_samples, const double* z, const double* u,
                        double* samples, double* stats) {
    APXCHK(nuts_args(P, data, weight, theta, F, step, max_depth, n_samples, z, u));
    if (n_samples > 0 && (!par_ok(P, samples) || !stats)) return fail(P->ctx, APX_E_INVALID, "null pointer");
    if (n_samples == 0) return APX_OK;
    hipStream_t st = P->ctx->stream;
    const long long n = P->n_par;
    const long long nd = 1 + max_depth + (1LL << (max_depth + 1));
    std::vector<double> uh;
    APXCHK(host_uniforms(P, u, nd * n_samples, uh));
    Nuts N;
    NPoint em, ep;
    APXCHK(nuts_setup(P, N, data, weight, F, step, em, ep));
    std::vector<double> sh((size_t)n_samples * 4);
    for (long long i = 0; i < n_samples; ++i) {
        double t6[6];
        APXCHK(nuts_transition(N, em, ep, theta, z + i * n, u + i * nd, uh.data() + i * nd, max_depth, i == 0, t6));
        if (n > 0)
            HIPCHK(hipMemcpyAsync(samples + i * n, theta, n * sizeof(double), hipMemcpyDeviceToDevice, st));
        for (int q = 0; q < 4; ++q) sh[i * 4 + q] = t6[q];
    }
    HIPCHK(hipMemcpyAsync(stats, sh.data(), sh.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return APX_OK;
}

apx_status apx_nuts_warmup(apx_problem* P, const float* data, const float* weight, double* theta, const double* F,
                           double* step, int32_t max_depth, int32_t n_warmup, double target_accept,
                           const double* z, const double* u) {
    if (!step) return fail(P ? P->ctx : nullptr, APX_E_INVALID, "null pointer");
    APXCHK(nuts_args(P, data, weight, theta, F, *step, max_depth, n_warmup, z, u));
    if (!(target_accept > 0.0 && target_accept < 1.0))
        return fail(P->ctx, APX_E_INVALID, "target acceptance must be in (0, 1)");
    if (n_warmup == 0) return APX_OK;
    const long long n = P->n_par;
    const long long nd = 1 + max_depth + (1LL << (max_depth + 1));
    std::vector<double> uh;
    APXCHK(host_uniforms(P, u, nd * n_warmup, uh));
    Nuts N;
    NPoint em, ep;
    APXCHK(nuts_setup(P, N, data, weight, F, *step, em, ep));
    // dual averaging of log step on the acceptance statistic
    const double mu = std::log(10.0 * *step);
    double hbar = 0.0, log_bar = 0.0;
    for (long long i = 0; i < n_warmup; ++i) {
        double t6[6];
        APXCHK(nuts_transition(N, em, ep, theta, z + i * n, u + i * nd, uh.data() + i * nd, max_depth, i == 0, t6));
        const double a = t6[5] > 0 ? t6[4] / t6[5] : 0.0;
        const double m = (double)(i + 1);
        hbar = (1.0 - 1.0 / (m + APX_NUTS_DA_T0)) * hbar + (target_accept - a) / (m + APX_NUTS_DA_T0);
        const double log_step = mu - std::sqrt(m) / APX_NUTS_DA_GAMMA * hbar;
        const double w = std::pow(m, -APX_NUTS_DA_KAPPA);
        log_bar = w * log_step + (1.0 - w) * log_bar;
        N.step = std::exp(log_step);
    }
    *step = std::exp(log_bar);
    return APX_OK;
}

apx_status apx_hmc_run(apx_problem* P, const float* data, const float* weight, double* theta, const double* F,
                       double step, int32_t n_leapfrog, int32_t n_samples, const double* z, const double* u,
                       double* samples, double* stats) {
    APXCHK(ready(P));
    if (!data || !weight || !par_ok(P, theta) || !par_ok(P, F) || (n_samples > 0 && (!par_ok(P, z) || !u)) ||
        (n_samples > 0 && (!par_ok(P, samples) || !stats)))
        return fail(P->ctx, APX_E_INVALID, "null pointer");
    if (n_leapfrog < 1 || n_samples < 0 || !(step > 0.0) || !std::isfinite(step))
        return fail(P->ctx, APX_E_INVALID, "need n_leapfrog >= 1, n_samples >= 0 and a finite step > 0");
    if (n_samples == 0) return APX_OK;
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    HmcIO h{};
    h.theta = theta;
    h.theta0 = wsp<double>(P, "hmc_t0");
    h.r = wsp<double>(P, "hmc_r");
    h.grad_cur = wsp<double>(P, "hmc_g0");
    h.grad_new = wsp<double>(P, "hmc_g1");
    h.chi2_cur = wsp<double>(P, "hmc_c0");
    h.chi2_new = wsp<double>(P, "hmc_c1");
    h.H0 = wsp<double>(P, "hmc_h0");
    h.z = z;
    h.u = u;
    h.samples = samples;
    h.stats = stats;
    double* Ft = p.M;                              // F^T (the Cholesky scratch is free here)
    HIPCHK(launch_hmc_transpose(p, F, Ft, st));
    // gradient at the start (an out-of-domain start raises the sticky flag)
    APXCHK(grad_core(P, theta, data, weight, h.grad_cur, h.chi2_cur, 0));
    for (long long i = 0; i < n_samples; ++i) {
        HIPCHK(launch_hmc_begin(p, h, i, st));
        for (int l = 0; l < n_leapfrog; ++l) {
            HIPCHK(launch_hmc_matvec(p, F, l == 0 ? h.grad_cur : h.grad_new, h.r, -0.25 * step, st));
            HIPCHK(launch_hmc_matvec(p, Ft, h.r, h.theta, step, st));
            APXCHK(grad_core(P, theta, data, weight, h.grad_new, h.chi2_new, 1));
            HIPCHK(launch_hmc_matvec(p, F, h.grad_new, h.r, -0.25 * step, st));
        }
        HIPCHK(launch_hmc_accept(p, h, i, st));
    }
    return APX_OK;
}

apx_status apx_render_vjp(apx_problem* P, const double* theta, const float* grad_model, double* grad_theta) {
    APXCHK(ready(P));
    if (!par_ok(P, theta) || !grad_model || !par_ok(P, grad_theta)) return fail(P->ctx, APX_E_INVALID, "null pointer");
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    APXCHK(prep(P, theta, 0, 0, nullptr, 1));
    HIPCHK(launch_flip_psf(p, st));
    ConvIO io{};
    io.out = p.Abar;
    io.seed = grad_model;
    APXCHK(run_conv(P, CONV_ADJ, io));
    {
        TimeScope ts(P, APX_TIME_GRAD);
        HIPCHK(launch_grad_tiles(p, st));
        HIPCHK(launch_seed_sums(p, grad_model, wsp<double>(P, "seed_part"), st));
    }
    SegSum a = segsum_base();
    a.src = p.grad_part;
    a.seg = wsp<int>(P, "gcol_seg");
    a.n_seg = (int)P->cols.size();
    a.out = p.grad_col;
    HIPCHK(launch_segsum(a, st));
    if (P->has_live_cols) {
        // live-PSF columns: sum seed J from their convolutions, with the residual buffer set
        // to -1/2 so that the gradient tables' weight -2 on sum w r J gives sum seed J
        HIPCHK(launch_fill_f(p.rbuf, P->n_pix, -0.5f, st));
        APXCHK(psf_columns(P, grad_model, 0, nullptr));
        APXCHK(col_sums(P));
    }
    SegSum g = segsum_base();
    g.src = P->asrc;
    g.seg = wsp<int>(P, "gr_seg");
    g.idx = wsp<int>(P, "gr_idx");
    g.wts = wsp<double>(P, "gr_w");
    g.n_seg = P->n_par;
    g.out = grad_theta;
    HIPCHK(launch_segsum(g, st));
    return APX_OK;
}

apx_status apx_lm_init(apx_problem* P, const double* theta, const float* data, const float* weight,
                       apx_lm_state* state) {
    APXCHK(ready(P));
    if (!par_ok(P, theta) || !data || !weight || !state) return fail(P->ctx, APX_E_INVALID, "null pointer");
    APXCHK(fwd_chi2(P, theta, data, weight, nullptr, P->chi2_sub, 0, 0, nullptr, 0));
    HIPCHK(launch_lm_init(P->plan, P->chi2_sub, state, P->ctx->stream));
    return APX_OK;
}

static apx_status lm_step_enqueue(apx_problem* P, const float* data, const float* weight, double* theta,
                                  apx_lm_state* state) {
    const Plan& p = P->plan;
    hipStream_t st = P->ctx->stream;
    {
        TimeScope ts(P, APX_TIME_LM);
        if (P->large_subs.empty()) HIPCHK(launch_lm_begin(p, state, st));
        else HIPCHK(launch_lm_begin_adopt(p, state, st));
    }
    // normal equations at theta for sub-problems whose last step was accepted
    APXCHK(prep(P, theta, 0, 2, state, 1));
    APXCHK(jac_blocks(P, weight, state));
    APXCHK(normal_eq(P, weight, p.A, p.gvec, state));
    // damped solves
    {
        TimeScope ts(P, APX_TIME_SOLVE);
        HIPCHK(launch_chol_small(p, wsp<int>(P, "small_subs"), (int)P->small_subs.size(), P->nmax_small, state, st));
        for (int s : P->large_subs) HIPCHK(launch_chol_large(p, s, P->subs[s].n, state, st));
    }
    // trial
    {
        TimeScope ts(P, APX_TIME_LM);
        HIPCHK(launch_lm_trial(p, theta, state, st));
    }
    APXCHK(fwd_chi2(P, p.theta_trial, data, weight, nullptr, P->chi2_trial, 1, 1, state, 0));
    {
        TimeScope ts(P, APX_TIME_LM);
        HIPCHK(launch_lm_accept(p, P->chi2_trial, theta, state, st));
    }
    return APX_OK;
}

apx_status apx_lm_step(apx_problem* P, const float* data, const float* weight, double* theta,
                       apx_lm_state* state) {
    APXCHK(ready(P));
    if (!par_ok(P, theta) || !data || !weight || !state) return fail(P->ctx, APX_E_INVALID, "null pointer");
    return lm_step_enqueue(P, data, weight, theta, state);
}

apx_status apx_lm_run(apx_problem* P, int32_t n_iter, const float* data, const float* weight,
                      double* theta, apx_lm_state* state, int32_t use_graph) {
    APXCHK(ready(P));
    if (!par_ok(P, theta) || !data || !weight || !state || n_iter < 0) return fail(P->ctx, APX_E_INVALID, "bad argument");
    if (!use_graph) {
        for (int i = 0; i < n_iter; ++i) APXCHK(lm_step_enqueue(P, data, weight, theta, state));
        return APX_OK;
    }
    hipStream_t st = P->ctx->stream;
    if (!st) return fail(P->ctx, APX_E_INVALID, "graph capture needs a non-default stream");
    const void* key[4] = {data, weight, theta, state};
    const uint32_t mask = P->timing ? P->timing_mask : 0u;
    if (!P->gexec || std::memcmp(key, P->gkey, sizeof(key)) != 0 || mask != P->gmask) {
        drop_graph(P);
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        P->capturing = true;
        apx_status s = lm_step_enqueue(P, data, weight, theta, state);
        P->capturing = false;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (s != APX_OK) {
            if (g) hipGraphDestroy(g);
            std::string m = P->cap_error;
            drop_graph(P);
            return m.empty() ? s : fail(P->ctx, APX_E_HIP, m + " (then: " + P->ctx->err + ")");
        }
        if (e != hipSuccess) { drop_graph(P); return fail(P->ctx, APX_E_HIP, std::string("capture: ") + hipGetErrorString(e)); }
        P->graph = g;
        if (!P->cap_error.empty()) {
            std::string m = P->cap_error;
            drop_graph(P);
            return fail(P->ctx, APX_E_HIP, m);
        }
        HIPCHK(hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0));
        std::memcpy(P->gkey, key, sizeof(key));
        P->gmask = mask;
    }
    for (int i = 0; i < n_iter; ++i) {
        if (mask) APXCHK(arm_mark_nodes(P));
        HIPCHK(hipGraphLaunch(P->gexec, st));
    }
    return APX_OK;
}

}  // extern "C"
