// Host side of the C ABI declared in include/vmcrnn.h: argument checks,
// workspace layout and the launch sequence of each call.
#include <string.h>

#include <cmath>

#include <array>
#include <map>
#include <mutex>

#include "kernels.h"

namespace vmc {

hipError_t launch_stage(const Dims &d, const float *prm, void *Bc, void *BcT, void *Bg, void *BgT,
                        float *E, float *Hd, float *hc, int4 *postab, hipStream_t st);
hipError_t launch_forward(const FwdArgs &a, int mode, int store_h, int store_lpc, int store_act,
                          int grid, hipStream_t st, const BatchInfo *bi = nullptr);
hipError_t launch_sched(int ham_kind, int Lx, int Ly, int64_t ns, const uint8_t *cfg, int *cnt,
                        int *list_off, int *list, int *tile_start, int *tile_counter, int MT,
                        hipStream_t st);
hipError_t launch_assemble(const vmc_ham &H, int cplx, int Lx, int Ly, int64_t ns, const uint8_t *cfg,
                           const float *lpc, const float *phc, const double2 *pre, const double2 *dsuf, int NC,
                           double *eloc, hipStream_t st);
int engine_kpx(const Dims &d);
size_t engine_lds(const Dims &d);
int forward_tile_rows(const Dims &d);
int chain_tile_rows(const Dims &d);
int row_tile_options(const Dims &d, int out[2]);
int chain_occupancy(const Dims &d);
int backward_tile_rows(int DH);
size_t backward_lds(const Dims &d);
hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t st);
hipError_t launch_grad(const GradBufs &b, hipStream_t st, const BatchInfo *bi = nullptr, bool chunk = false);
hipError_t launch_stats(int64_t ns, const double *eloc, const double *w, double *stats, hipStream_t st);
void grad_sizes(const Dims &d, int64_t ns, size_t *part_floats);
int64_t grad_nsp(int64_t ns);
hipError_t launch_grow(const vmc_model &from, const float *p0, int new_dh, uint64_t seed, double noise,
                       float *p1, const float *m0, const float *v0, float *m1, float *v1,
                       int64_t n_to, hipStream_t st);
hipError_t launch_bump(uint64_t *counter, hipStream_t st);
hipError_t launch_adam(int64_t n, float *p, const double *g, float *m, float *v, int64_t *t_dev,
                       const vmc_adam_cfg &c, hipStream_t st);
hipError_t launch_count_nonfinite(const float *x, int64_t n, unsigned long long *count, hipStream_t st);
hipError_t launch_batch_scan(const BatchInfo &bi, int MT, const int *cnt0, int4 *sched, int *counter,
                             hipStream_t st);

static const int kMaxN = 1024;
static const size_t kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950

static bool valid_model(const vmc_model *m) {
    if (!m) return false;
    if (m->dims != 1 && m->dims != 2) return false;
    if (m->Lx < 1 || m->Ly < 1 || (m->dims == 1 && m->Ly != 1)) return false;
    if ((int64_t)m->Lx * m->Ly < 2 || (int64_t)m->Lx * m->Ly > kMaxN) return false;
    if (m->d_h < 1) return false;
    if (m->precision != VMC_FP32 && m->precision != VMC_BF16) return false;
    if ((m->is_complex != 0 && m->is_complex != 1) || (m->glu != 0 && m->glu != 1)) return false;
    return true;
}

// The Hamiltonian descriptor against the model: known kind, finite
// couplings, the 1D-only kinds on a chain.
static vmc_status check_ham(const vmc_model *m, const vmc_ham *H) {
    if (!H) return VMC_EINVAL;
    if (H->kind != VMC_TFIM && H->kind != VMC_HEISENBERG && H->kind != VMC_LRTFIM && H->kind != VMC_CLUSTER)
        return VMC_EINVAL;
    if (!std::isfinite(H->J) || !std::isfinite(H->h)) return VMC_ENONFINITE;
    if (H->kind == VMC_LRTFIM) {
        if (!std::isfinite(H->alpha)) return VMC_ENONFINITE;
        if (H->alpha < 0.0) return VMC_EINVAL;
    }
    if ((H->kind == VMC_LRTFIM || H->kind == VMC_CLUSTER) && m->dims != 1) return VMC_EUNSUPPORTED;
    if (H->kind == VMC_CLUSTER && m->Lx < 3) return VMC_EINVAL;
    return VMC_OK;
}

// connection kind of the chain engine and the schedule: one flip per
// position (TFIM, LR-TFIM) or a connection list (Heisenberg, cluster)
static int engine_kind(const vmc_ham *H) { return H->kind == VMC_LRTFIM ? VMC_TFIM : H->kind; }
static bool list_kind(const vmc_ham *H) { return H && (H->kind == VMC_HEISENBERG || H->kind == VMC_CLUSTER); }

static int padded_dh(int d) {
    static const int sizes[] = {16, 32, 64, 128, 256};
    for (int s : sizes)
        if (d <= s) return s;
    return -1;
}

// ------------------------------------------------------------ tuning table
// Launch choices per model shape, process-wide.  Every choice gives the same
// result bits (rows are computed independently of their tile and of the
// work-group that runs them), so the table only changes speed.
static const int kChainWpcFallback = 2, kChainWpcMax = 4;
typedef std::array<int, 7> ShapeKey;
static std::mutex g_tune_mu;
static std::map<ShapeKey, vmc_tuning> g_tune;

static ShapeKey shape_key(const vmc_model *m) {
    return ShapeKey{m->dims, m->Lx, m->dims == 2 ? m->Ly : 1, m->d_h, m->precision, m->glu, m->is_complex};
}

// Built-in work-groups per CU of the chain launch: twice as many as fit one
// CU (measured 4 % faster than exactly the resident count at d_h = 128),
// queried once per shape, at most 4; 2 if the runtime cannot say.
static std::map<std::array<int, 4>, int> g_occ;
static int default_chain_wpc(const Dims &d) {
    const std::array<int, 4> k{d.prec, d.dims, d.DH, d.N};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_occ.find(k);
        if (it != g_occ.end()) return it->second;
    }
    int n = chain_occupancy(d);
    n = n < 1 ? kChainWpcFallback : 2 * n > kChainWpcMax ? kChainWpcMax : 2 * n;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_occ[k] = n;
    return n;
}

static vmc_tuning lookup_tuning(const vmc_model *m) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(shape_key(m));
    if (it == g_tune.end()) return vmc_tuning{0, 0};
    return it->second;
}

static Dims make_dims(const vmc_model *m) {
    Dims d;
    d.dims = m->dims;
    d.Lx = m->Lx;
    d.Ly = m->dims == 2 ? m->Ly : 1;
    d.N = d.Lx * d.Ly;
    d.dh = m->d_h;
    d.DH = padded_dh(m->d_h);
    d.K = d.dims == 1 ? d.DH : 2 * d.DH;
    int ks = m->precision == VMC_BF16 ? 32 : 16;
    d.KP = round_up(d.K, ks);
    d.cplx = m->is_complex;
    d.glu = m->glu;
    d.prec = m->precision;
    d.row_alt = 0;
    d.chain_wpc = 0;
    const vmc_tuning t = lookup_tuning(m);
    if (t.row_tile > 0) {
        int opt[2];
        const int n = row_tile_options(d, opt);
        d.row_alt = n > 1 && t.row_tile == opt[1];
    }
    d.chain_wpc = t.chain_wgs_per_cu > 0 ? t.chain_wgs_per_cu : default_chain_wpc(d);
    return d;
}

static int device_cus() {
    static int cached = 0;
    if (!cached) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            cached = n;
        else
            cached = 256;
    }
    return cached;
}

static size_t al(size_t x) { return (x + 255) / 256 * 256; }

// Workspace map; offsets in bytes from the workspace base.
struct WsMap {
    size_t Bc, BcT, Bg, BgT, E, Hd, hc;
    size_t hcache, hcs, postab, lpc, phc, pre, dsuf;
    size_t cnt, list_off, tile_start, tile_counter, list;
    size_t colbuf;
    size_t act, lgT, hT, gT, xT, dtc, dtg, dth, dcol, part, stats;
    size_t total;
    int chain_grid, fwd_grid, NC;
    int64_t nsp;
};

// part_floats_min: a batch sizes the weight-gradient partials of every
// region for the problem that needs the most
static WsMap ws_map(const Dims &d, const vmc_ham *H, int64_t ns, size_t part_floats_min = 0) {
    WsMap w;
    memset(&w, 0, sizeof(w));
    const size_t es = d.prec == VMC_BF16 ? 2 : 4;
    const int KGP = round_up(d.DH, d.prec == VMC_BF16 ? 32 : 16);
    const int MT = forward_tile_rows(d);
    size_t o = 0;
    auto put = [&](size_t bytes) {
        size_t at = o;
        o += al(bytes);
        return at;
    };
    w.Bc = put((size_t)3 * d.DH * engine_kpx(d) * es);
    w.BcT = put((size_t)round_up(3 * d.DH, d.prec == VMC_BF16 ? 32 : 16) * d.K * es);
    w.Bg = put((size_t)2 * d.DH * KGP * es);
    w.BgT = put((size_t)2 * d.DH * KGP * es);
    w.E = put((size_t)ESLOTS * d.DH * 4);
    w.Hd = put((size_t)4 * d.DH * 4);
    w.hc = put(16);
    // FP32 prefix states: not kept for 2D bfloat16 (only the operand copy is read)
    w.hcache = put(d.dims == 2 && d.prec == VMC_BF16 ? 16 : (size_t)d.N * ns * d.DH * 4);
    w.hcs = d.prec == VMC_BF16 ? put((size_t)d.N * ns * d.DH * 2) : w.hcache;
    w.postab = put((size_t)d.N * 16);
    w.lpc = put((size_t)ns * d.N * 2 * 4);
    w.phc = put((size_t)ns * d.N * 2 * 4);
    w.pre = put((size_t)ns * d.N * 16);
    const int nb = list_kind(H) ? conn_count(H->kind, d.Lx, d.Ly) : 0;
    w.NC = list_kind(H) ? nb : d.N;
    w.dsuf = put((size_t)ns * w.NC * 16);
    w.cnt = put((size_t)(d.N + 1) * 4);
    w.list_off = put((size_t)(d.N + 1) * 4);
    w.tile_start = put((size_t)(d.N + 1) * 4);
    w.tile_counter = put(4);
    w.list = put(list_kind(H) ? (size_t)ns * nb * 4 : 4);
    // the row launches cover every column of the transposed activation
    // arrays (nsp >= ns samples), so that the rows past ns hold zeros
    const int64_t nsp = grad_nsp(ns);
    w.fwd_grid = (int)((nsp + MT - 1) / MT);
    w.chain_grid = d.chain_wpc * device_cus();
    // the column buffer holds one tile-row block per work-group of the
    // largest launch any tuning can make, so a workspace sized once stays
    // valid when the tuning changes
    int opt[2];
    const int nopt = row_tile_options(d, opt);
    size_t rows = (size_t)kChainWpcMax * device_cus() * chain_tile_rows(d);
    for (int i = 0; i < nopt; i++) {
        const size_t f = (size_t)((nsp + opt[i] - 1) / opt[i]) * opt[i];
        rows = f > rows ? f : rows;
    }
    w.colbuf = put(d.dims == 2 ? rows * d.Lx * d.DH * es : 16);
    // backward
    const int nd_cell = d.dims == 1 ? 4 * d.DH : 3 * d.DH;
    w.nsp = nsp;
    w.act = put((size_t)d.N * act_feats(d.dims) * d.DH * w.nsp * es);
    w.lgT = put((size_t)d.N * 4 * w.nsp * 4);
    w.hT = put((size_t)d.N * d.DH * w.nsp * es);
    w.gT = put(d.glu ? (size_t)d.N * d.DH * w.nsp * es : 16);
    w.dtc = put((size_t)d.N * nd_cell * w.nsp * es);
    w.dtg = put(d.glu ? (size_t)d.N * 2 * d.DH * w.nsp * es : 16);
    w.dth = put((size_t)d.N * 4 * w.nsp * es);
    const int MTB = backward_tile_rows(d.DH);
    w.dcol = put(d.dims == 2 ? (size_t)((w.nsp + MTB - 1) / MTB) * d.Lx * MTB * d.DH * 4 : 16);
    w.xT = put((size_t)d.N * 5 * w.nsp * es);
    size_t part_floats = 0;
    grad_sizes(d, ns, &part_floats);
    w.part = put((part_floats > part_floats_min ? part_floats : part_floats_min) * 4);
    w.stats = put(8 * 8);
    w.total = o;
    return w;
}

template <class X>
static X *at(void *ws, size_t off) {
    return (X *)((char *)ws + off);
}

static vmc_status hip_status(hipError_t e) { return e == hipSuccess ? VMC_OK : VMC_EDEVICE; }

// every launch's LDS (static tiles plus the tile's configurations, rows x N
// bytes) must fit one compute unit, for every tile choice
static bool lds_fits(const Dims &d) { return engine_lds(d) <= kMaxLds && backward_lds(d) <= kMaxLds; }

static vmc_status check_common(const vmc_model *m, const float *params, int64_t n, void *ws, size_t ws_bytes,
                               const vmc_ham *H, size_t *need) {
    if (!valid_model(m)) return VMC_EINVAL;
    if (H) {
        const vmc_status hs = check_ham(m, H);
        if (hs != VMC_OK) return hs;
    }
    if (!params || n < 1 || !ws) return VMC_EINVAL;
    if (((uintptr_t)ws & 255) != 0) return VMC_EINVAL;
    if (padded_dh(m->d_h) < 0) return VMC_EUNSUPPORTED;
    if (n >= ((int64_t)1 << 31)) return VMC_EUNSUPPORTED;
    Dims d = make_dims(m);
    if (!lds_fits(d)) return VMC_EUNSUPPORTED;
    if (list_kind(H) && n * conn_count(H->kind, d.Lx, d.Ly) >= ((int64_t)1 << 31)) return VMC_EUNSUPPORTED;
    WsMap w = ws_map(d, H, n);
    if (need) *need = w.total;
    if (ws_bytes < w.total) return VMC_ENOSPACE;
    return VMC_OK;
}

static hipError_t stage(const Dims &d, const float *params, void *ws, const WsMap &w, hipStream_t st) {
    return launch_stage(d, params, at<void>(ws, w.Bc), at<void>(ws, w.BcT), at<void>(ws, w.Bg),
                        at<void>(ws, w.BgT), at<float>(ws, w.E), at<float>(ws, w.Hd), at<float>(ws, w.hc),
                        at<int4>(ws, w.postab), st);
}

static FwdArgs base_args(const Dims &d, void *ws, const WsMap &w, int64_t ns) {
    FwdArgs a;
    memset(&a, 0, sizeof(a));
    a.d = d;
    a.Bc = at<void>(ws, w.Bc);
    a.Bg = at<void>(ws, w.Bg);
    a.E = at<float>(ws, w.E);
    a.Hd = at<float>(ws, w.Hd);
    a.hc = at<float>(ws, w.hc);
    a.nrows = ns;
    a.ns_cache = ns;
    a.colbuf = at<void>(ws, w.colbuf);
    a.postab = at<int4>(ws, w.postab);
    a.hcs = at<void>(ws, w.hcs);
    return a;
}

// Event pairs around the suffix-chain launch (opt-in profiling).
struct ChainTiming {
    int enabled = 0, created = 0, n = 0;
    static const int kMax = 4096;
    hipEvent_t ev[2 * kMax];
};
static ChainTiming g_timing;

}  // namespace vmc

using namespace vmc;

extern "C" {

int64_t vmc_param_count(const vmc_model *m) {
    if (!valid_model(m)) return -1;
    return param_layout(m->dims, m->d_h, m->glu, m->is_complex).total;
}

vmc_status vmc_workspace_size(const vmc_model *m, const vmc_ham *H, int64_t ns, size_t *bytes) {
    if (!valid_model(m) || ns < 1 || !bytes) return VMC_EINVAL;
    if (H) {
        const vmc_status hs = check_ham(m, H);
        if (hs != VMC_OK) return hs;
    }
    if (padded_dh(m->d_h) < 0) return VMC_EUNSUPPORTED;
    Dims d = make_dims(m);
    if (!lds_fits(d)) return VMC_EUNSUPPORTED;
    *bytes = ws_map(d, H, ns).total;
    return VMC_OK;
}

vmc_status rnn_sample(const vmc_model *m, const float *params, int64_t ns, uint64_t seed, uint64_t counter,
                      const float *uniforms, uint8_t *configs, float *logp, float *phase, void *ws,
                      size_t ws_bytes, void *stream) {
    vmc_status s = check_common(m, params, ns, ws, ws_bytes, NULL, NULL);
    if (s != VMC_OK) return s;
    if (!configs || !logp) return VMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Dims d = make_dims(m);
    WsMap w = ws_map(d, NULL, ns);
    hipError_t e = stage(d, params, ws, w, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    FwdArgs a = base_args(d, ws, w, ns);
    a.uniforms = uniforms;
    a.seed = seed;
    a.counter = counter;
    a.cfg_out = configs;
    a.logp = logp;
    a.phase = d.cplx ? phase : NULL;
    if (phase && !d.cplx) {
        e = launch_fill(phase, ns, 0.0f, st);
        if (e != hipSuccess) return VMC_EDEVICE;
    }
    return hip_status(launch_forward(a, MODE_SAMPLE, 0, 0, 0, w.fwd_grid, st));
}

vmc_status rnn_logpsi(const vmc_model *m, const float *params, int64_t nc, const uint8_t *configs, float *logp,
                      float *phase, void *ws, size_t ws_bytes, void *stream) {
    vmc_status s = check_common(m, params, nc, ws, ws_bytes, NULL, NULL);
    if (s != VMC_OK) return s;
    if (!configs || !logp) return VMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Dims d = make_dims(m);
    WsMap w = ws_map(d, NULL, nc);
    hipError_t e = stage(d, params, ws, w, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    FwdArgs a = base_args(d, ws, w, nc);
    a.cfg_in = configs;
    a.logp = logp;
    a.phase = d.cplx ? phase : NULL;
    if (phase && !d.cplx) {
        e = launch_fill(phase, nc, 0.0f, st);
        if (e != hipSuccess) return VMC_EDEVICE;
    }
    return hip_status(launch_forward(a, MODE_LOGPSI, 0, 0, 0, w.fwd_grid, st));
}

// Local energy from a workspace whose prefix cache (hidden states,
// conditionals, prefix sums) holds the configurations.
static vmc_status eloc_from_cache(const Dims &d, const WsMap &w, void *ws, const vmc_ham *H, int64_t ns,
                                  const uint8_t *configs, double *eloc, hipStream_t st) {
    FwdArgs a = base_args(d, ws, w, ns);
    a.cfg_in = configs;
    a.hcache = at<float>(ws, w.hcache);
    a.lpc = at<float>(ws, w.lpc);
    a.phc = at<float>(ws, w.phc);
    a.pre = at<double2>(ws, w.pre);
    const int ek = engine_kind(H);
    hipError_t e = launch_sched(ek, d.Lx, d.Ly, ns, configs, at<int>(ws, w.cnt), at<int>(ws, w.list_off),
                                at<int>(ws, w.list), at<int>(ws, w.tile_start), at<int>(ws, w.tile_counter),
                                chain_tile_rows(d), st);
    if (e != hipSuccess) return VMC_EDEVICE;
    a.ham_kind = ek;
    a.nbond = ek == VMC_TFIM ? 0 : conn_count(ek, d.Lx, d.Ly);
    a.cnt = at<int>(ws, w.cnt);
    a.tile_start = at<int>(ws, w.tile_start);
    a.list_off = at<int>(ws, w.list_off);
    a.list = at<int>(ws, w.list);
    a.tile_counter = at<int>(ws, w.tile_counter);
    a.dsuf = at<double2>(ws, w.dsuf);
    a.NC = w.NC;
    const bool timed = g_timing.enabled && g_timing.n < ChainTiming::kMax;
    if (timed && hipEventRecord(g_timing.ev[2 * g_timing.n], st) != hipSuccess) return VMC_EDEVICE;
    e = launch_forward(a, MODE_CHAIN, 0, 0, 0, w.chain_grid, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    if (timed) {
        if (hipEventRecord(g_timing.ev[2 * g_timing.n + 1], st) != hipSuccess) return VMC_EDEVICE;
        g_timing.n++;
    }
    return hip_status(launch_assemble(*H, d.cplx, d.Lx, d.Ly, ns, configs, at<float>(ws, w.lpc), at<float>(ws, w.phc),
                                      at<double2>(ws, w.pre), at<double2>(ws, w.dsuf), w.NC, eloc, st));
}

// Gradient from a workspace whose hidden states and activations hold the
// configurations.
static vmc_status grad_from_cache(const Dims &d, const WsMap &w, void *ws, int64_t ns, const uint8_t *configs,
                                  const double *eloc, const double *weights, double *grad, double *stats,
                                  hipStream_t st, const float *coef_lp = NULL, const float *coef_ph = NULL,
                                  bool chunk = false) {
    GradBufs b;
    b.d = d;
    b.BcT = at<void>(ws, w.BcT);
    b.BgT = at<void>(ws, w.BgT);
    b.E = at<float>(ws, w.E);
    b.Hd = at<float>(ws, w.Hd);
    b.ns = ns;
    b.cfg = configs;
    b.hcache = at<float>(ws, w.hcache);
    b.act = at<void>(ws, w.act);
    b.lgT = at<float>(ws, w.lgT);
    b.eloc = eloc;
    b.weights = weights;
    b.coef_lp = coef_lp;
    b.coef_ph = coef_ph;
    b.stats = stats ? stats : at<double>(ws, w.stats);
    b.dtc = at<void>(ws, w.dtc);
    b.dtg = at<void>(ws, w.dtg);
    b.dth = at<void>(ws, w.dth);
    b.hT = at<void>(ws, w.hT);
    b.gT = at<void>(ws, w.gT);
    b.dcol = at<void>(ws, w.dcol);
    b.xT = at<void>(ws, w.xT);
    b.part = at<float>(ws, w.part);
    b.grad = grad;
    return hip_status(launch_grad(b, st, nullptr, chunk));
}

vmc_status local_energy(const vmc_model *m, const float *params, const vmc_ham *H, int64_t ns,
                        const uint8_t *configs, double *eloc, void *ws, size_t ws_bytes, void *stream) {
    if (!H) return VMC_EINVAL;
    vmc_status s = check_common(m, params, ns, ws, ws_bytes, H, NULL);
    if (s != VMC_OK) return s;
    if (!configs || !eloc) return VMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Dims d = make_dims(m);
    WsMap w = ws_map(d, H, ns);
    const int MT = forward_tile_rows(d);
    hipError_t e = stage(d, params, ws, w, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    // 1. teacher-forced pass: prefix hidden states and conditionals of every sample
    FwdArgs a = base_args(d, ws, w, ns);
    a.cfg_in = configs;
    a.hcache = at<float>(ws, w.hcache);
    a.lpc = at<float>(ws, w.lpc);
    a.phc = at<float>(ws, w.phc);
    a.pre = at<double2>(ws, w.pre);
    e = launch_forward(a, MODE_LOGPSI, 1, 1, 0, w.fwd_grid, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    // 2. all connected configurations of all samples: schedule, one persistent launch, assembly
    return eloc_from_cache(d, w, ws, H, ns, configs, eloc, st);
}

vmc_status vmc_grad(const vmc_model *m, const float *params, int64_t ns, const uint8_t *configs,
                    const double *eloc, const double *weights, double *grad, double *stats, void *ws,
                    size_t ws_bytes, void *stream) {
    vmc_status s = check_common(m, params, ns, ws, ws_bytes, NULL, NULL);
    if (s != VMC_OK) return s;
    if (!configs || !eloc || !grad) return VMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Dims d = make_dims(m);
    WsMap w = ws_map(d, NULL, ns);
    hipError_t e = stage(d, params, ws, w, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    FwdArgs a = base_args(d, ws, w, ns);
    a.cfg_in = configs;
    a.hcache = at<float>(ws, w.hcache);
    a.act = at<void>(ws, w.act);
    a.lgT = at<float>(ws, w.lgT);
    a.hT = at<void>(ws, w.hT);
    a.gT = at<void>(ws, w.gT);
    a.nsp = w.nsp;
    e = launch_forward(a, MODE_LOGPSI, 1, 0, 1, w.fwd_grid, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    return grad_from_cache(d, w, ws, ns, configs, eloc, weights, grad, stats, st);
}

vmc_status vmc_energy_stats(int64_t ns, const double *eloc, const double *weights, double *stats, void *stream) {
    if (ns <= 0) return VMC_EINVAL;
    if (!eloc || !stats) return VMC_EINVAL;
    return hip_status(launch_stats(ns, eloc, weights, stats, (hipStream_t)stream));
}

vmc_status vmc_grad_chunk(const vmc_model *m, const float *params, int64_t ns, const uint8_t *configs,
                          const double *eloc, const double *weights, const double *stats, double *grad, void *ws,
                          size_t ws_bytes, void *stream) {
    vmc_status s = check_common(m, params, ns, ws, ws_bytes, NULL, NULL);
    if (s != VMC_OK) return s;
    if (!configs || !eloc || !weights || !stats || !grad) return VMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Dims d = make_dims(m);
    WsMap w = ws_map(d, NULL, ns);
    hipError_t e = stage(d, params, ws, w, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    FwdArgs a = base_args(d, ws, w, ns);
    a.cfg_in = configs;
    a.hcache = at<float>(ws, w.hcache);
    a.act = at<void>(ws, w.act);
    a.lgT = at<float>(ws, w.lgT);
    a.hT = at<void>(ws, w.hT);
    a.gT = at<void>(ws, w.gT);
    a.nsp = w.nsp;
    e = launch_forward(a, MODE_LOGPSI, 1, 0, 1, w.fwd_grid, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    // (the statistics are read, never written: the cast only fits the buffer type)
    return grad_from_cache(d, w, ws, ns, configs, eloc, weights, grad, const_cast<double *>(stats), st, NULL, NULL,
                           true);
}

vmc_status rnn_logpsi_grad(const vmc_model *m, const float *params, int64_t nc, const uint8_t *configs,
                           const float *dlogp, const float *dphase, double *grad, void *ws, size_t ws_bytes,
                           void *stream) {
    vmc_status s = check_common(m, params, nc, ws, ws_bytes, NULL, NULL);
    if (s != VMC_OK) return s;
    if (!configs || !dlogp || !grad) return VMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Dims d = make_dims(m);
    WsMap w = ws_map(d, NULL, nc);
    hipError_t e = stage(d, params, ws, w, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    FwdArgs a = base_args(d, ws, w, nc);
    a.cfg_in = configs;
    a.hcache = at<float>(ws, w.hcache);
    a.act = at<void>(ws, w.act);
    a.lgT = at<float>(ws, w.lgT);
    a.hT = at<void>(ws, w.hT);
    a.gT = at<void>(ws, w.gT);
    a.nsp = w.nsp;
    e = launch_forward(a, MODE_LOGPSI, 1, 0, 1, w.fwd_grid, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    return grad_from_cache(d, w, ws, nc, configs, NULL, NULL, grad, NULL, st, dlogp, d.cplx ? dphase : NULL);
}

vmc_status vmc_step(const vmc_model *m, const float *params, const vmc_ham *H, int64_t ns, uint64_t seed,
                    uint64_t counter, uint64_t *counter_dev, const float *uniforms, uint8_t *configs, float *logp,
                    float *phase, double *eloc, double *grad, double *stats, void *ws, size_t ws_bytes,
                    void *stream) {
    if (!H) return VMC_EINVAL;
    vmc_status s = check_common(m, params, ns, ws, ws_bytes, H, NULL);
    if (s != VMC_OK) return s;
    if (!configs || !logp || !eloc || !grad) return VMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    Dims d = make_dims(m);
    WsMap w = ws_map(d, H, ns);
    hipError_t e = stage(d, params, ws, w, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    // sampling keeps everything the later phases read
    FwdArgs a = base_args(d, ws, w, ns);
    a.uniforms = uniforms;
    a.seed = seed;
    a.counter = counter;
    a.counter_dev = counter_dev;
    a.cfg_out = configs;
    a.cfg_in = configs;
    a.logp = logp;
    a.phase = d.cplx ? phase : NULL;
    a.hcache = at<float>(ws, w.hcache);
    a.lpc = at<float>(ws, w.lpc);
    a.phc = at<float>(ws, w.phc);
    a.pre = at<double2>(ws, w.pre);
    a.act = at<void>(ws, w.act);
    a.lgT = at<float>(ws, w.lgT);
    a.hT = at<void>(ws, w.hT);
    a.gT = at<void>(ws, w.gT);
    a.nsp = w.nsp;
    if (phase && !d.cplx) {
        e = launch_fill(phase, ns, 0.0f, st);
        if (e != hipSuccess) return VMC_EDEVICE;
    }
    e = launch_forward(a, MODE_SAMPLE, 1, 1, 1, w.fwd_grid, st);
    if (e != hipSuccess) return VMC_EDEVICE;
    s = eloc_from_cache(d, w, ws, H, ns, configs, eloc, st);
    if (s != VMC_OK) return s;
    s = grad_from_cache(d, w, ws, ns, configs, eloc, NULL, grad, stats, st);
    if (s != VMC_OK || !counter_dev) return s;
    return hip_status(launch_bump(counter_dev, st));
}

// ------------------------------------------------------- batched problems
// Layout of a batch workspace: one region per problem with the layout of
// the longest chain, at `pitch` bytes, then the chain-tile queue (int4
// entries) and its tile counter.
struct BatchMap {
    WsMap w;
    size_t pitch, sched, counter, total;
    int Nmax, E;
};

static vmc_status batch_check(int32_t nprob, const vmc_model *m, const int32_t *chain_len, const vmc_ham *H,
                              int64_t ns, BatchMap *bm) {
    if (nprob < 1 || nprob > kMaxBatch || !m || !chain_len || !H || ns < 1) return VMC_EINVAL;
    if (m->dims != 1) return VMC_EUNSUPPORTED;
    if (ns >= ((int64_t)1 << 31)) return VMC_EUNSUPPORTED;
    int Nmax = 0, E = 0;
    size_t part_max = 0;
    for (int k = 0; k < nprob; k++) {
        vmc_model mk = *m;
        mk.Lx = chain_len[k];
        mk.Ly = 1;
        if (!valid_model(&mk)) return VMC_EINVAL;
        if (H[k].kind != H[0].kind) return VMC_EINVAL;
        const vmc_status hs = check_ham(&mk, &H[k]);
        if (hs != VMC_OK) return hs;
        if (padded_dh(mk.d_h) < 0) return VMC_EUNSUPPORTED;
        const Dims dk = make_dims(&mk);
        if (!lds_fits(dk)) return VMC_EUNSUPPORTED;
        if (list_kind(&H[k]) && ns * conn_count(H[k].kind, dk.Lx, 1) >= ((int64_t)1 << 31)) return VMC_EUNSUPPORTED;
        size_t pf = 0;
        grad_sizes(dk, ns, &pf);
        part_max = pf > part_max ? pf : part_max;
        Nmax = chain_len[k] > Nmax ? chain_len[k] : Nmax;
        E += chain_len[k] - 1;
    }
    vmc_model mm = *m;
    mm.Lx = Nmax;
    mm.Ly = 1;
    const Dims dmax = make_dims(&mm);
    bm->w = ws_map(dmax, &H[0], ns, part_max);
    bm->pitch = al(bm->w.total);
    bm->sched = bm->pitch * nprob;
    bm->counter = bm->sched + al((size_t)(E + 1) * 16);
    bm->total = bm->counter + 256;
    bm->Nmax = Nmax;
    bm->E = E;
    return VMC_OK;
}

vmc_status vmc_batched_workspace_size(int32_t nprob, const vmc_model *m, const int32_t *chain_len, const vmc_ham *H,
                                      int64_t ns, size_t *bytes) {
    if (!bytes) return VMC_EINVAL;
    BatchMap bm;
    const vmc_status s = batch_check(nprob, m, chain_len, H, ns, &bm);
    if (s != VMC_OK) return s;
    *bytes = bm.total;
    return VMC_OK;
}

vmc_status vmc_step_batched(int32_t nprob, const vmc_model *m, const int32_t *chain_len, const vmc_ham *H,
                            const float *params, int64_t ns, uint64_t seed, uint64_t counter, uint64_t *counter_dev,
                            uint8_t *configs, float *logp, float *phase, double *eloc, double *grad, double *stats,
                            void *ws, size_t ws_bytes, void *stream) {
    BatchMap bm;
    vmc_status s = batch_check(nprob, m, chain_len, H, ns, &bm);
    if (s != VMC_OK) return s;
    if (!params || !configs || !logp || !eloc || !grad || !stats || !ws) return VMC_EINVAL;
    if (((uintptr_t)ws & 255) != 0) return VMC_EINVAL;
    if (ws_bytes < bm.total) return VMC_ENOSPACE;
    hipStream_t st = (hipStream_t)stream;
    const WsMap &w = bm.w;
    vmc_model mm = *m;
    mm.Lx = bm.Nmax;
    mm.Ly = 1;
    const Dims dmax = make_dims(&mm);
    const int64_t P = param_layout(1, m->d_h, m->glu, m->is_complex).total;
    BatchInfo bi;
    memset(&bi, 0, sizeof(bi));
    bi.n = nprob;
    bi.tiles = w.fwd_grid;
    bi.pitch_ws = (int64_t)bm.pitch;
    bi.pitch_cfg = ns * bm.Nmax;
    bi.pitch_p = P;
    bi.ns = ns;
    bi.sched = at<int4>(ws, bm.sched);
    bi.nsched = bm.E;
    for (int k = 0; k < nprob; k++) bi.N[k] = chain_len[k];
    // 1. staged weights and position table of every problem
    for (int k = 0; k < nprob; k++) {
        vmc_model mk = mm;
        mk.Lx = chain_len[k];
        const Dims dk = make_dims(&mk);
        if (stage(dk, params + (size_t)k * P, (char *)ws + (size_t)k * bm.pitch, w, st) != hipSuccess)
            return VMC_EDEVICE;
    }
    // 2. sampling of every problem in one launch (problem k: Philox key seed + k)
    FwdArgs a = base_args(dmax, ws, w, ns);
    a.seed = seed;
    a.counter = counter;
    a.counter_dev = counter_dev;
    a.cfg_out = configs;
    a.cfg_in = configs;
    a.logp = logp;
    a.phase = dmax.cplx ? phase : NULL;
    a.hcache = at<float>(ws, w.hcache);
    a.lpc = at<float>(ws, w.lpc);
    a.phc = at<float>(ws, w.phc);
    a.pre = at<double2>(ws, w.pre);
    a.act = at<void>(ws, w.act);
    a.lgT = at<float>(ws, w.lgT);
    a.hT = at<void>(ws, w.hT);
    a.gT = at<void>(ws, w.gT);
    a.nsp = w.nsp;
    if (phase && !dmax.cplx && launch_fill(phase, (int64_t)nprob * ns, 0.0f, st) != hipSuccess) return VMC_EDEVICE;
    if (launch_forward(a, MODE_SAMPLE, 1, 1, 1, nprob * w.fwd_grid, st, &bi) != hipSuccess) return VMC_EDEVICE;
    // 3. connection schedule of every problem, then one queue over all chain tiles
    const int ek = engine_kind(&H[0]);
    const int MTc = chain_tile_rows(dmax);
    for (int k = 0; k < nprob; k++) {
        char *r = (char *)ws + (size_t)k * bm.pitch;
        if (launch_sched(ek, chain_len[k], 1, ns, configs + (size_t)k * bi.pitch_cfg, at<int>(r, w.cnt),
                         at<int>(r, w.list_off), at<int>(r, w.list), at<int>(r, w.tile_start),
                         at<int>(r, w.tile_counter), MTc, st) != hipSuccess)
            return VMC_EDEVICE;
    }
    if (launch_batch_scan(bi, MTc, at<int>(ws, w.cnt), at<int4>(ws, bm.sched), at<int>(ws, bm.counter), st) !=
        hipSuccess)
        return VMC_EDEVICE;
    // 4. every connected configuration of every sample of every problem in one persistent launch
    FwdArgs c = base_args(dmax, ws, w, ns);
    c.cfg_in = configs;
    c.hcache = at<float>(ws, w.hcache);
    c.lpc = at<float>(ws, w.lpc);
    c.phc = at<float>(ws, w.phc);
    c.pre = at<double2>(ws, w.pre);
    c.ham_kind = ek;
    c.cnt = at<int>(ws, w.cnt);
    c.tile_start = at<int>(ws, w.tile_start);
    c.list_off = at<int>(ws, w.list_off);
    c.list = at<int>(ws, w.list);
    c.tile_counter = at<int>(ws, bm.counter);
    c.dsuf = at<double2>(ws, w.dsuf);
    const bool timed = g_timing.enabled && g_timing.n < ChainTiming::kMax;
    if (timed && hipEventRecord(g_timing.ev[2 * g_timing.n], st) != hipSuccess) return VMC_EDEVICE;
    if (launch_forward(c, MODE_CHAIN, 0, 0, 0, w.chain_grid, st, &bi) != hipSuccess) return VMC_EDEVICE;
    if (timed) {
        if (hipEventRecord(g_timing.ev[2 * g_timing.n + 1], st) != hipSuccess) return VMC_EDEVICE;
        g_timing.n++;
    }
    // 5. local energies of every problem
    for (int k = 0; k < nprob; k++) {
        char *r = (char *)ws + (size_t)k * bm.pitch;
        const int NCk = list_kind(&H[k]) ? conn_count(H[k].kind, chain_len[k], 1) : chain_len[k];
        if (launch_assemble(H[k], dmax.cplx, chain_len[k], 1, ns, configs + (size_t)k * bi.pitch_cfg,
                            at<float>(r, w.lpc), at<float>(r, w.phc), at<double2>(r, w.pre), at<double2>(r, w.dsuf),
                            NCk, eloc + (size_t)k * 2 * ns, st) != hipSuccess)
            return VMC_EDEVICE;
    }
    // 6. statistics and gradient of every problem (batched launches)
    GradBufs b;
    b.d = dmax;
    b.BcT = at<void>(ws, w.BcT);
    b.BgT = at<void>(ws, w.BgT);
    b.E = at<float>(ws, w.E);
    b.Hd = at<float>(ws, w.Hd);
    b.ns = ns;
    b.cfg = configs;
    b.hcache = at<float>(ws, w.hcache);
    b.act = at<void>(ws, w.act);
    b.lgT = at<float>(ws, w.lgT);
    b.eloc = eloc;
    b.weights = NULL;
    b.coef_lp = NULL;
    b.coef_ph = NULL;
    b.stats = stats;
    b.dtc = at<void>(ws, w.dtc);
    b.dtg = at<void>(ws, w.dtg);
    b.dth = at<void>(ws, w.dth);
    b.hT = at<void>(ws, w.hT);
    b.gT = at<void>(ws, w.gT);
    b.dcol = at<void>(ws, w.dcol);
    b.xT = at<void>(ws, w.xT);
    b.part = at<float>(ws, w.part);
    b.grad = grad;
    if (launch_grad(b, st, &bi) != hipSuccess) return VMC_EDEVICE;
    if (!counter_dev) return VMC_OK;
    return hip_status(launch_bump(counter_dev, st));
}

// ------------------------------------------------- step without allocation
// A fixed device array serves as the workspace of vmc_step_noalloc, for
// callers that cannot allocate.  In host code the name `scratch` is only a
// stand-in for the symbol: kernels get the device address that
// hipGetSymbolAddress returns, looked up once per device and kept.
static const size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_ptr;

static vmc_status scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return VMC_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = NULL;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VMC_EDEVICE;
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return VMC_OK;
}

vmc_status vmc_step_noalloc(const vmc_model *m, const float *params, const vmc_ham *H, int64_t ns, uint64_t seed,
                            uint64_t counter, uint64_t *counter_dev, const float *uniforms, uint8_t *configs,
                            float *logp, float *phase, double *eloc, double *grad, double *stats, void *stream) {
    size_t need = 0;
    const vmc_status s = vmc_workspace_size(m, H, ns, &need);
    if (s != VMC_OK) return s;
    if (!H) return VMC_EINVAL;
    if (need > kScratchBytes) return VMC_ENOSPACE;
    void *ws = NULL;
    const vmc_status a = scratch_address(&ws);
    if (a != VMC_OK) return a;
    return vmc_step(m, params, H, ns, seed, counter, counter_dev, uniforms, configs, logp, phase, eloc, grad, stats,
                    ws, kScratchBytes, stream);
}

size_t vmc_noalloc_scratch_bytes(void) { return kScratchBytes; }

vmc_status vmc_adam(int64_t n, float *params, const double *grad, float *m, float *v, int64_t *t_dev,
                    const vmc_adam_cfg *cfg, void *stream) {
    if (n < 1 || !params || !grad || !m || !v || !t_dev || !cfg) return VMC_EINVAL;
    const double vals[] = {cfg->lr0, cfg->lr1, cfg->tau, cfg->beta1, cfg->beta2, cfg->eps};
    for (double x : vals)
        if (!std::isfinite(x)) return VMC_ENONFINITE;
    if (cfg->lr0 < 0.0 || cfg->lr1 < 0.0 || cfg->tau < 0.0 || !(cfg->eps > 0.0)) return VMC_EINVAL;
    if (cfg->beta1 < 0.0 || cfg->beta1 >= 1.0 || cfg->beta2 < 0.0 || cfg->beta2 >= 1.0) return VMC_EINVAL;
    return hip_status(launch_adam(n, params, grad, m, v, t_dev, *cfg, (hipStream_t)stream));
}

vmc_status vmc_check_finite(const float *x, int64_t n, int64_t *count, void *ws, size_t ws_bytes, void *stream) {
    if (!x || n < 1 || !ws || ws_bytes < 256 || ((uintptr_t)ws & 255) != 0) return VMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    unsigned long long *dc = (unsigned long long *)ws, hc = 0;
    if (launch_count_nonfinite(x, n, dc, st) != hipSuccess) return VMC_EDEVICE;
    if (hipMemcpyAsync(&hc, dc, sizeof(hc), hipMemcpyDeviceToHost, st) != hipSuccess) return VMC_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return VMC_EDEVICE;
    if (count) *count = (int64_t)hc;
    return hc ? VMC_ENONFINITE : VMC_OK;
}

vmc_status grow_hidden(const vmc_model *from, const float *p_from, int32_t new_dh, uint64_t seed, double noise_std,
                       float *p_to, const float *m_from, const float *v_from, float *m_to, float *v_to,
                       void *stream) {
    if (!valid_model(from) || !p_from || !p_to) return VMC_EINVAL;
    if (new_dh < from->d_h) return VMC_EINVAL;
    if (!std::isfinite(noise_std)) return VMC_ENONFINITE;
    if (noise_std < 0.0) return VMC_EINVAL;
    int nmom = (m_from != NULL) + (v_from != NULL) + (m_to != NULL) + (v_to != NULL);
    if (nmom != 0 && nmom != 4) return VMC_EINVAL;
    vmc_model to = *from;
    to.d_h = new_dh;
    if (!valid_model(&to)) return VMC_EINVAL;
    int64_t n_to = param_layout(to.dims, new_dh, to.glu, to.is_complex).total;
    return hip_status(launch_grow(*from, p_from, new_dh, seed, noise_std, p_to, m_from, v_from, m_to, v_to, n_to,
                                  (hipStream_t)stream));
}

vmc_status vmc_chain_timing(int enable) {
    if (enable) {
        if (!g_timing.created) {
            for (int i = 0; i < 2 * ChainTiming::kMax; i++)
                if (hipEventCreate(&g_timing.ev[i]) != hipSuccess) return VMC_EDEVICE;
            g_timing.created = 1;
        }
        g_timing.n = 0;
        g_timing.enabled = 1;
    } else {
        g_timing.enabled = 0;
    }
    return VMC_OK;
}

vmc_status vmc_chain_time(double *ms_total, int64_t *launches) {
    if (!ms_total || !launches) return VMC_EINVAL;
    double tot = 0.0;
    for (int i = 0; i < g_timing.n; i++) {
        float ms = 0.f;
        if (hipEventSynchronize(g_timing.ev[2 * i + 1]) != hipSuccess) return VMC_EDEVICE;
        if (hipEventElapsedTime(&ms, g_timing.ev[2 * i], g_timing.ev[2 * i + 1]) != hipSuccess) return VMC_EDEVICE;
        tot += ms;
    }
    *ms_total = tot;
    *launches = g_timing.n;
    return VMC_OK;
}

vmc_status vmc_row_tile_options(const vmc_model *m, int32_t *opts, int32_t *count) {
    if (!valid_model(m) || !opts || !count) return VMC_EINVAL;
    if (padded_dh(m->d_h) < 0) return VMC_EUNSUPPORTED;
    Dims d = make_dims(m);
    int o[2];
    const int n = row_tile_options(d, o);
    for (int i = 0; i < n; i++) opts[i] = o[i];
    *count = n;
    return VMC_OK;
}

vmc_status vmc_set_tuning(const vmc_model *m, const vmc_tuning *t) {
    if (!valid_model(m)) return VMC_EINVAL;
    if (padded_dh(m->d_h) < 0) return VMC_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!t) {
        g_tune.erase(shape_key(m));
        return VMC_OK;
    }
    if (t->chain_wgs_per_cu < 0 || t->chain_wgs_per_cu > kChainWpcMax) return VMC_EINVAL;
    if (t->row_tile != 0) {
        Dims d = {};
        d.dims = m->dims;
        d.DH = padded_dh(m->d_h);
        d.prec = m->precision;
        int o[2];
        const int n = row_tile_options(d, o);
        if (t->row_tile != o[0] && (n < 2 || t->row_tile != o[1])) return VMC_EINVAL;
    }
    g_tune[shape_key(m)] = *t;
    return VMC_OK;
}

vmc_status vmc_get_tuning(const vmc_model *m, vmc_tuning *t) {
    if (!valid_model(m) || !t) return VMC_EINVAL;
    if (padded_dh(m->d_h) < 0) return VMC_EUNSUPPORTED;
    Dims d = make_dims(m);
    t->row_tile = forward_tile_rows(d);
    t->chain_wgs_per_cu = d.chain_wpc;
    return VMC_OK;
}

vmc_status vmc_autotune_step(const vmc_model *m, const float *params, const vmc_ham *H, int64_t ns, uint64_t seed,
                             uint64_t counter, const float *uniforms, uint8_t *configs, float *logp, float *phase,
                             double *eloc, double *grad, double *stats, void *ws, size_t ws_bytes, void *stream,
                             int32_t reps, vmc_tuning *best) {
    if (reps < 1 || reps > 100) return VMC_EINVAL;
    if (!H) return VMC_EINVAL;
    vmc_status s = check_common(m, params, ns, ws, ws_bytes, H, NULL);
    if (s != VMC_OK) return s;
    if (!configs || !logp || !eloc || !grad) return VMC_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess) return VMC_EDEVICE;
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        hipEventDestroy(ev[0]);
        return VMC_EDEVICE;
    }
    // fastest of `reps` steps under tuning t
    auto timed = [&](const vmc_tuning &t, float *ms) -> vmc_status {
        vmc_status r = vmc_set_tuning(m, &t);
        if (r != VMC_OK) return r;
        float bestms = 1e30f;
        for (int i = 0; i < reps; i++) {
            if (hipEventRecord(ev[0], st) != hipSuccess) return VMC_EDEVICE;
            r = vmc_step(m, params, H, ns, seed, counter, NULL, uniforms, configs, logp, phase, eloc, grad, stats,
                         ws, ws_bytes, stream);
            if (r != VMC_OK) return r;
            float t_ms = 0.f;
            if (hipEventRecord(ev[1], st) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                hipEventElapsedTime(&t_ms, ev[0], ev[1]) != hipSuccess)
                return VMC_EDEVICE;
            bestms = t_ms < bestms ? t_ms : bestms;
        }
        *ms = bestms;
        return VMC_OK;
    };
    // coordinate search from the tuning in effect: the row tile, then the
    // persistent work-groups per compute unit of the chain launch
    vmc_tuning cur;
    s = vmc_get_tuning(m, &cur);
    float cur_ms = 0.f;
    if (s == VMC_OK) s = timed(cur, &cur_ms);
    int32_t opts[2], nopt = 0;
    if (s == VMC_OK) s = vmc_row_tile_options(m, opts, &nopt);
    for (int i = 0; s == VMC_OK && i < nopt; i++) {
        if (opts[i] == cur.row_tile) continue;
        vmc_tuning t = cur;
        t.row_tile = opts[i];
        float ms = 0.f;
        s = timed(t, &ms);
        if (s == VMC_OK && ms < cur_ms) {
            cur = t;
            cur_ms = ms;
        }
    }
    for (int wpc = 1; s == VMC_OK && wpc <= kChainWpcMax; wpc++) {
        if (wpc == cur.chain_wgs_per_cu) continue;
        vmc_tuning t = cur;
        t.chain_wgs_per_cu = wpc;
        float ms = 0.f;
        s = timed(t, &ms);
        if (s == VMC_OK && ms < cur_ms) {
            cur = t;
            cur_ms = ms;
        }
    }
    // the outputs left behind are those of one step under the chosen tuning
    if (s == VMC_OK) s = timed(cur, &cur_ms);
    if (s == VMC_OK && best) *best = cur;
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    return s;
}

const char *vmc_status_str(vmc_status s) {
    switch (s) {
        case VMC_OK: return "ok";
        case VMC_EINVAL: return "invalid argument";
        case VMC_EUNSUPPORTED: return "unsupported configuration";
        case VMC_ENOSPACE: return "workspace too small";
        case VMC_EDEVICE: return "device error";
        case VMC_ENONFINITE: return "non-finite value";
    }
    return "unknown status";
}

}  // extern "C"
