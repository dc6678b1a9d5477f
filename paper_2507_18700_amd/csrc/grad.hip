// Energy gradient of VMC (Sec. III): FP64 statistics of the local energies,
// a reverse sweep (backpropagation through the autoregressive chain) that
// produces the per-(position, sample) deltas of every contraction, and the
// weight gradients as contractions of those deltas with the layer inputs over
// all (position, sample) pairs.  Deltas are stored transposed,
// [position][feature][sample], so the contraction over samples reads MFMA
// fragments straight from memory; the inputs (h, GLU output) in blocks of 16
// samples, [position][sample/16][feature][16], staged through LDS.  One
// partial per position (FP32 MFMA accumulation), summed over positions in FP64
// in a fixed order.
//
// With E held constant, the gradient is that of the surrogate
//   L = sum_s [a_s log P(sigma_s) + b_s phi(sigma_s)],
//   a_s = w_s Re(E_s - Ebar), b_s = 2 w_s Im(E_s - Ebar),
// i.e. 2 Re sum_s w_s conj(E_s - Ebar) d log psi(sigma_s) with
// d log psi = d log P / 2 + i d phi (Eq. 4).
#include "kernels.h"

namespace vmc {

constexpr int DW_TILE = 128;            // padding granule of the weight-gradient partials
constexpr int DW_NF = 9, DW_COLS = 144;  // input-column fragments / columns per contraction tile
// MFMA k-steps per pipeline step of the contraction: three for the 3-fragment
// tiles (one work-group per compute unit by registers, so the step size sets
// the bytes in flight); one for the smaller tiles, which keep two or more
// work-groups per compute unit that way
template <int MF>
constexpr int dw_sub() { return MF == 3 ? 3 : 1; }

// ------------------------------------------------------------- statistics

// One work-group: Ebar = sum w E, var = sum w |E - Ebar|^2, non-finite count.
// Fixed per-thread strides and a fixed tree: bitwise reproducible.  A batch
// runs one work-group per problem (blockIdx.y; no weights).
__global__ __launch_bounds__(1024) void stats_kernel(int64_t ns, const double *eloc, const double *w,
                                                     double *stats) {
    __shared__ double s0[1024], s1[1024], s2[1024];
    const int t = threadIdx.x;
    eloc += (int64_t)blockIdx.y * 2 * ns;
    stats += (int64_t)blockIdx.y * 4;
    double er = 0.0, ei = 0.0, bad = 0.0;
    for (int64_t s = t; s < ns; s += 1024) {
        double ws = w ? w[s] : 1.0 / (double)ns;
        double a = eloc[2 * s], b = eloc[2 * s + 1];
        if (!isfinite(a) || !isfinite(b)) bad += 1.0;
        er += ws * a;
        ei += ws * b;
    }
    s0[t] = er;
    s1[t] = ei;
    s2[t] = bad;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (t < h) {
            s0[t] += s0[t + h];
            s1[t] += s1[t + h];
            s2[t] += s2[t + h];
        }
        __syncthreads();
    }
    const double Er = s0[0], Ei = s1[0], nbad = s2[0];
    __syncthreads();
    double v = 0.0;
    for (int64_t s = t; s < ns; s += 1024) {
        double ws = w ? w[s] : 1.0 / (double)ns;
        double a = eloc[2 * s] - Er, b = eloc[2 * s + 1] - Ei;
        v += ws * (a * a + b * b);
    }
    s0[t] = v;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (t < h) s0[t] += s0[t + h];
        __syncthreads();
    }
    if (t == 0) {
        stats[0] = Er;
        stats[1] = Ei;
        stats[2] = s0[0];
        stats[3] = nbad;
    }
}

// ------------------------------------------------- weight-gradient contraction

// Per-problem shape of the weight-gradient contraction of a batch: regions
// of the workspace at pitch_ws, chain lengths and the sample chunking of each
// problem (the same as vmc_step chooses for it alone).
struct DwBatch {
    int n;
    int64_t pitch_ws, pitch_p;
    int N[kMaxBatch], nchunk[kMaxBatch];
    int64_t chunk[kMaxBatch];
};

struct DwArgs {
    Dims d;
    int seg;              // 0 cell, 1 GLU, 2 heads
    int64_t ns, nsp;      // samples, padded sample stride
    const void *A;        // transposed deltas [N][MD][nsp]
    int MD, K, Mp, Kp;    // delta rows, hidden input columns, padded output dims
    const void *hT, *gT;  // hidden states / GLU outputs [N][nsp/16][DH][16]
    const void *xT;       // transposed extra inputs [N][5][nsp]: 1, onehot_hz(2), onehot_vt(2)
    float *part;          // [N*nchunk][Mp][Kp]
    int nchunk;           // sample chunks per position (split of the contraction)
    int64_t chunk;        // samples per chunk (multiple of 32)
    int units;            // N * nchunk (position, chunk) pairs
    int tiles_m, tiles;   // output tiles along M, per unit
};

// Work-groups are handed to the XCDs round-robin by linear id; the output
// tiles of one (position, chunk) unit read the same delta rows and inputs, so
// they are given ids on one XCD (id = xcd + kXcds * slot) and share its L2.
constexpr int kXcds = 8;

// Source row of input column k of segment seg at position q: a hidden state
// (h or g) of some position, one of the extra rows (bias 1, one-hots), or
// none.  Returns the row pointer offset in elements or -1.
__device__ inline int64_t dw_source(const DwArgs &a, int q, int k, bool &extra) {
    const int DH = a.d.DH, Lx = a.d.Lx;
    const int64_t nsp = a.nsp;
    extra = false;
    if (k >= a.K) {
        const int c = k - a.K;
        if (c >= (a.seg == 0 ? (a.d.dims == 1 ? 3 : 5) : 1)) return -1;
        extra = true;
        return ((int64_t)q * 5 + c) * nsp;
    }
    // h and the GLU output: [position][16-sample block][DH][16]; the offset of
    // sample 0 of column k (sample s adds (s / 16) * 16 DH + s % 16)
    if (a.seg != 0) return (int64_t)q * DH * nsp + k * 16;
    if (k < DH) return (q % Lx) != 0 ? (int64_t)(q - 1) * DH * nsp + k * 16 : -1;
    if (q < Lx) return -1;
    return (int64_t)site_pos(order_site(q, Lx) - Lx, Lx) * DH * nsp + (k - DH) * 16;
}

// Extra input rows per position: 1, the one-hot of the horizontal
// predecessor's spin, the one-hot of the vertical predecessor's spin (zeros
// where the predecessor is absent), transposed [N][5][nsp].
template <class P>
__global__ void build_extras(Dims d, int64_t ns, int64_t nsp, const uint8_t *cfg, typename P::store_t *xT,
                             DwBatch gb, int64_t pitch_cfg) {
    if (gb.n > 0) {  // batch: problem blockIdx.y
        const int k = blockIdx.y;
        d.N = d.Lx = gb.N[k];
        cfg += (int64_t)k * pitch_cfg;
        xT = shift_bytes(xT, (int64_t)k * gb.pitch_ws);
    }
    const int N = d.N, Lx = d.Lx;
    const int64_t total = (int64_t)N * nsp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(e / nsp);
        const int64_t s = e % nsp;
        float v[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        if (s < ns) {
            v[0] = 1.f;
            if ((q % Lx) != 0) v[1 + cfg[s * N + order_site(q - 1, Lx)]] = 1.f;
            if (d.dims == 2 && q >= Lx) v[3 + cfg[s * N + order_site(q, Lx) - Lx]] = 1.f;
        }
#pragma unroll
        for (int c = 0; c < 5; c++) xT[((int64_t)q * 5 + c) * nsp + s] = P::from_float(v[c]);
    }
}

// dW[m][k] at one position q over one chunk of samples: the sum over samples
// of A[q][m][s] X[q][k][s] on MFMA.  A work-group of 8 waves covers 128*MF
// delta rows (MF 16-row fragments per wave, read straight from memory)
// against one tile of DW_COLS input columns that the whole work-group stages
// in LDS (double-buffered), so each input row is read from memory once per
// row tile instead of once per wave.  A pipeline step spans dw_sub<MF>()
// MFMA k-steps, and the next step's loads are in flight during the current
// step's MFMAs: the contraction is bound by memory latency, so the bytes in
// flight per compute unit set its rate.  Each accumulator takes its k-steps
// in sample order whatever the step size.
template <class P, int MF>
__global__ __launch_bounds__(512) void dw_mfma(DwArgs a, DwBatch gb) {
    typedef typename P::store_t T;
    if (gb.n > 0) {  // batch: problem blockIdx.y, its region and chunking
        const int k = blockIdx.y;
        const int64_t o = (int64_t)k * gb.pitch_ws;
        a.A = shift_bytes(a.A, o);
        a.hT = shift_bytes(a.hT, o);
        a.gT = shift_bytes(a.gT, o);
        a.xT = shift_bytes(a.xT, o);
        a.part = shift_bytes(a.part, o);
        a.d.N = a.d.Lx = gb.N[k];
        a.nchunk = gb.nchunk[k];
        a.chunk = gb.chunk[k];
        a.units = a.d.N * a.nchunk;
    }
    constexpr int DW_SUB = dw_sub<MF>();
    constexpr int VEC = P::VEC, KS = P::KSTEP, STEP = DW_SUB * KS;
    constexpr int LDB = STEP + 16 / (int)sizeof(T);  // padded row of the staged input tile
    constexpr int CPR = STEP / VEC;                  // 16-byte chunks per staged row
    constexpr int NCH = DW_COLS * CPR, CPT = (NCH + 511) / 512;
    __shared__ __align__(16) T sB[2][DW_COLS * LDB];
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6), l16 = lane & 15, lq = lane >> 4;
    const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
    const int u = xcd + kXcds * (slot / a.tiles);
    if (u >= a.units) return;  // padding slot: the whole work-group leaves before any barrier
    const int t = slot % a.tiles, mt = t % a.tiles_m, nt = t / a.tiles_m;
    const int q = u / a.nchunk, cidx = u - q * a.nchunk;
    const int64_t nsp = a.nsp;
    const int64_t sbeg = (int64_t)cidx * a.chunk, send = min(nsp, sbeg + a.chunk);
    const int m0 = (mt * 8 + w) * 16 * MF, k0 = nt * DW_COLS;
    const T *A = (const T *)a.A + (int64_t)q * a.MD * nsp;
    const T *X = (const T *)(a.seg == 2 && a.d.glu ? a.gT : a.hT);
    const T *XE = (const T *)a.xT;
    const T *ap[MF];
    bool mon[MF];
#pragma unroll
    for (int i = 0; i < MF; i++) {
        const int m = m0 + 16 * i + l16;
        mon[i] = (m0 + 16 * i) < a.MD;
        ap[i] = A + (int64_t)(m < a.MD ? m : 0) * nsp + VEC * lq;
    }
    // staging chunks of this thread: row j of the tile, 16-byte part c
    // (samples VEC*c .. VEC*c + VEC - 1 of the step); one step is STEP * DH
    // elements of the blocked h and GLU arrays (16 DH per 16 samples) and STEP
    // of the extra rows
    const T *bsrc[CPT];
    int bdst[CPT], boff[CPT], binc[CPT];
    const int DHa = a.d.DH;
    // (chunk order = address order of the blocked arrays: the parts of one
    // 16-sample block, then the tile's columns, then the blocks of the step)
    constexpr int PB = 16 / VEC;
#pragma unroll
    for (int i = 0; i < CPT; i++) {
        const int ch = tid + 512 * i, h = ch % PB, jb = ch / PB, j = jb % DW_COLS, c = (jb / DW_COLS) * PB + h;
        bsrc[i] = nullptr;
        bdst[i] = -1;
        boff[i] = VEC * c;
        binc[i] = 0;
        if (ch < NCH) {
            bool extra;
            const int64_t off = dw_source(a, q, k0 + j, extra);
            if (off >= 0) {
                // a running pointer: at the chunk's first step, advanced one step per load
                bsrc[i] = extra ? XE + off + VEC * c + sbeg
                                : X + off + ((VEC * c) >> 4) * (DHa * 16) + ((VEC * c) & 15) + sbeg * DHa;
                binc[i] = extra ? STEP : STEP * DHa;
            }
            bdst[i] = j * LDB + VEC * c;
        }
    }
    // input-column fragments with at least one source
    bool kon[DW_NF];
#pragma unroll
    for (int f = 0; f < DW_NF; f++) {
        bool live = false;
        for (int c = 0; c < 16; c++) {
            bool ex;
            live |= dw_source(a, q, k0 + 16 * f + c, ex) >= 0;
        }
        kon[f] = live;
    }
    f32x4_t acc[MF][DW_NF];
#pragma unroll
    for (int i = 0; i < MF; i++)
#pragma unroll
        for (int f = 0; f < DW_NF; f++) acc[i][f] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    // (send and every chunk start are multiples of 32 samples, so a 16-byte
    // part or a k-step lies wholly before or wholly after send; parts past
    // send are zeros)
    uint4 stg[CPT];
    // (called once per step, in order from sbeg)
    auto gload_b = [&](int64_t s0) {
#pragma unroll
        for (int i = 0; i < CPT; i++) {
            stg[i] = (bsrc[i] && s0 + boff[i] < send) ? *(const uint4 *)bsrc[i] : make_uint4(0, 0, 0, 0);
            bsrc[i] += binc[i];
        }
    };
    auto sstore_b = [&](int buf) {
#pragma unroll
        for (int i = 0; i < CPT; i++)
            if (bdst[i] >= 0) *(uint4 *)&sB[buf][bdst[i]] = stg[i];
    };
    auto load_a = [&](int64_t s0, uint4 (*fa)[MF]) {
#pragma unroll
        for (int j = 0; j < DW_SUB; j++)
#pragma unroll
            for (int i = 0; i < MF; i++)
                fa[j][i] = (mon[i] && s0 + j * KS < send) ? *(const uint4 *)(ap[i] + s0 + j * KS)
                                                          : make_uint4(0, 0, 0, 0);
    };
    // one step on buffer buf with fragments fa; the next step's loads (into
    // fn and the other buffer) are issued before the MFMAs
    auto body = [&](int64_t s0, int buf, uint4 (*fa)[MF], uint4 (*fn)[MF]) {
        const bool more = s0 + STEP < send;  // uniform over the work-group
        if (more) {
            gload_b(s0 + STEP);
            load_a(s0 + STEP, fn);
        }
#pragma unroll
        for (int j = 0; j < DW_SUB; j++)
#pragma unroll
            for (int f = 0; f < DW_NF; f++) {
                if (!kon[f]) continue;
                const uint4 bf = *(const uint4 *)&sB[buf][(16 * f + l16) * LDB + j * KS + VEC * lq];
#pragma unroll
                for (int i = 0; i < MF; i++)
                    if (mon[i]) P::mma(acc[i][f], fa[j][i], bf);
            }
        if (more) sstore_b(buf ^ 1);
        __syncthreads();
    };
    uint4 fa0[DW_SUB][MF], fa1[DW_SUB][MF];
    gload_b(sbeg);
    sstore_b(0);
    load_a(sbeg, fa0);
    __syncthreads();
    for (int64_t s0 = sbeg; s0 < send; s0 += 2 * STEP) {
        body(s0, 0, fa0, fa1);
        if (s0 + STEP < send) body(s0 + STEP, 1, fa1, fa0);
    }
    float *out = a.part + (int64_t)u * a.Mp * a.Kp;
#pragma unroll
    for (int i = 0; i < MF; i++)
#pragma unroll
        for (int f = 0; f < DW_NF; f++)
#pragma unroll
            for (int ii = 0; ii < 4; ii++) {
                const int m = m0 + 16 * i + 4 * lq + ii;
                const int k = k0 + 16 * f + l16;
                if (m < a.MD && k < a.Kp) out[(int64_t)m * a.Kp + k] = acc[i][f][ii];
            }
}

// Flat parameter index of the weight-gradient entry (seg, m, k), or -1 for
// padding and unused combinations.  k < K: hidden input columns; k = K: bias;
// k = K+1.. : one-hot columns.
__device__ inline int64_t dw_param(const Dims &d, int seg, int m, int k) {
    const int dh = d.dh, DH = d.DH;
    const ParamLayout L = param_layout(d.dims, dh, d.glu, d.cplx);
    if (seg == 2) {
        if (m >= 4 || (m >= 2 && !d.cplx)) return -1;
        if (k < DH) {
            if (k >= dh) return -1;
            return m < 2 ? L.Ua + (int64_t)m * dh + k : L.Up + (int64_t)(m - 2) * dh + k;
        }
        if (k == DH) return m < 2 ? L.ca + m : L.cp + (m - 2);
        return -1;
    }
    if (seg == 1) {
        if (!d.glu || m >= 2 * DH) return -1;
        const int half = m / DH, u = m % DH;
        if (u >= dh) return -1;
        if (k < DH) return k < dh ? (half ? L.W2 : L.W1) + (int64_t)u * dh + k : -1;
        if (k == DH) return (half ? L.b2 : L.b1) + u;
        return -1;
    }
    const int g = m / DH, u = m % DH;
    if (u >= dh) return -1;
    if (d.dims == 1) {
        if (g > 3) return -1;
        const int64_t rowg = L.Wg + (int64_t)u * (dh + 2), rowr = L.Wr + (int64_t)u * (dh + 2);
        if (k < DH) {
            if (k >= dh) return -1;
            if (g == 0) return rowg + k;
            if (g == 1) return rowr + k;
            if (g == 2) return L.Wh + (int64_t)u * dh + k;
            return -1;
        }
        if (k == DH) return g == 0 ? L.bg + u : g == 1 ? L.br + u : g == 2 ? L.bh + u : L.bin + u;
        if (k <= DH + 2) {
            const int c = k - DH - 1;
            if (g == 0) return rowg + dh + c;
            if (g == 1) return rowr + dh + c;
            if (g == 3) return L.Win + (int64_t)u * 2 + c;
            return -1;
        }
        return -1;
    }
    if (g > 2) return -1;
    const int64_t row = g == 0 ? L.W + (int64_t)u * (2 * dh + 4)
                      : g == 1 ? L.Wg + (int64_t)u * (2 * dh + 4)
                               : L.U + (int64_t)u * 2 * dh;
    if (k < DH) return k < dh ? row + k : -1;
    if (k < 2 * DH) return (k - DH) < dh ? row + dh + (k - DH) : -1;
    if (g == 2) return -1;
    if (k == 2 * DH) return g == 0 ? L.b + u : L.bg + u;
    if (k <= 2 * DH + 4) return row + 2 * dh + (k - 2 * DH - 1);
    return -1;
}

// FP64 sum of the per-position (and per-chunk) partials, scattered into the
// flat gradient.  A work-group reduces 32 consecutive columns of one output
// row: 8 groups of 32 threads take every 8th partial (4 loads in flight per
// thread), then the 8 group sums are added in a fixed order.
__global__ __launch_bounds__(256) void dw_reduce(Dims d, int seg, const float *part, int Q, int Mp, int Kp, int K,
                                                 int MD, double *grad, DwBatch gb, int accumulate) {
    __shared__ double sg[8][32];
    if (gb.n > 0) {  // batch: problem blockIdx.y
        const int kk = blockIdx.y;
        part = shift_bytes(part, (int64_t)kk * gb.pitch_ws);
        grad += (int64_t)kk * gb.pitch_p;
        Q = gb.N[kk] * gb.nchunk[kk];
    }
    const int W = K + 5, nkb = (W + 31) / 32;
    const int m = blockIdx.x / nkb, k = (blockIdx.x % nkb) * 32 + (threadIdx.x & 31), g = threadIdx.x >> 5;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (m < MD && k < W) {
        const float *src = part + (int64_t)m * Kp + k;
        const int64_t stride = (int64_t)Mp * Kp;
        int q = g;
        for (; q + 24 < Q; q += 32) {
#pragma unroll
            for (int u = 0; u < 4; u++) acc[u] += (double)src[(int64_t)(q + 8 * u) * stride];
        }
        for (int u = 0; q < Q; q += 8, u++) acc[u & 3] += (double)src[(int64_t)q * stride];
    }
    sg[g][threadIdx.x & 31] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (g == 0 && m < MD && k < W) {
        double t = 0.0;
        for (int i = 0; i < 8; i++) t += sg[i][threadIdx.x];
        const int64_t idx = dw_param(d, seg, m, k);
        if (idx >= 0) grad[idx] = accumulate ? grad[idx] + t : t;
    }
}

__global__ void fill_f64(double *p, int64_t n, double v) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

// ------------------------------------------------------------------ host

struct SegDims {
    int MD, K, Mp, Kp;
};

static SegDims seg_dims(const Dims &d, int seg) {
    SegDims s;
    if (seg == 0) {
        s.MD = d.dims == 1 ? 4 * d.DH : 3 * d.DH;
        s.K = d.dims == 1 ? d.DH : 2 * d.DH;
    } else if (seg == 1) {
        s.MD = 2 * d.DH;
        s.K = d.DH;
    } else {
        s.MD = 4;
        s.K = d.DH;
    }
    s.Kp = cround(s.K + 5, DW_TILE);
    s.Mp = cround(s.MD, DW_TILE);
    return s;
}

int64_t grad_nsp(int64_t ns) { return (ns + 31) / 32 * 32; }

// Delta-row fragments per wave (1..3) for MD delta rows: the fewest padded
// rows, then the larger fragment count; tiles along M and along the inputs.
static int dw_mf(int MD) {
    int best = 3, waste = 1 << 30;
    for (int mf = 3; mf >= 1; mf--) {
        const int rows = 128 * mf, wst = (MD + rows - 1) / rows * rows - MD;
        if (wst < waste) {
            waste = wst;
            best = mf;
        }
    }
    return best;
}
static int dw_tiles_m(const SegDims &s) { return (s.MD + 128 * dw_mf(s.MD) - 1) / (128 * dw_mf(s.MD)); }
static int dw_tiles_n(const SegDims &s) { return (s.K + 5 + DW_COLS - 1) / DW_COLS; }

// Resident work-groups per CU of dw_mfma<P, MF> on gfx950 (8 waves each; the
// register use of 1, 2 and 3 fragments per wave allows 6, 4 and 2 waves per
// SIMD), and the CUs of the chip.
static int dw_wg_per_cu(int mf) { return mf >= 3 ? 1 : mf == 2 ? 2 : 3; }
constexpr int kDwCUs = 256;

// Sample chunks per position of the weight-gradient contraction: chunks of
// >= 1024 samples, at most 16, and among those the count with the least
// time in rounds of the chip per sample, ceil(W / R) / c for W = tiles * c
// work-groups of which R are resident at once (the smallest such count).
static int dw_chunks(const Dims &d, const SegDims &s, int64_t nsp) {
    const int64_t tiles = (int64_t)dw_tiles_m(s) * dw_tiles_n(s) * d.N;
    const int64_t R = (int64_t)kDwCUs * dw_wg_per_cu(dw_mf(s.MD));
    int64_t cmax = nsp / 1024 > 1 ? nsp / 1024 : 1;
    if (cmax > 16) cmax = 16;
    int64_t best = 1, best_rounds = (tiles + R - 1) / R;
    for (int64_t c = 2; c <= cmax; c++) {
        const int64_t rounds = (tiles * c + R - 1) / R;
        if (rounds * best < best_rounds * c) {  // rounds / c < best_rounds / best
            best = c;
            best_rounds = rounds;
        }
    }
    return (int)best;
}

void grad_sizes(const Dims &d, int64_t ns, size_t *part_floats) {
    const int64_t nsp = grad_nsp(ns);
    size_t mx = 0;
    for (int seg = 0; seg < 3; seg++) {
        SegDims s = seg_dims(d, seg);
        const size_t n = (size_t)dw_chunks(d, s, nsp) * s.Mp * s.Kp;
        mx = n > mx ? n : mx;
    }
    *part_floats = (size_t)d.N * mx;
}

template <class P>
static void launch_dw_p(const DwArgs &a, const SegDims &sd, const DwBatch &gb, int units_max, hipStream_t st) {
    const dim3 grid(kXcds * ((units_max + kXcds - 1) / kXcds) * a.tiles, gb.n > 0 ? gb.n : 1);
    switch (dw_mf(sd.MD)) {
        case 1: hipLaunchKernelGGL((dw_mfma<P, 1>), grid, dim3(512), 0, st, a, gb); break;
        case 2: hipLaunchKernelGGL((dw_mfma<P, 2>), grid, dim3(512), 0, st, a, gb); break;
        default: hipLaunchKernelGGL((dw_mfma<P, 3>), grid, dim3(512), 0, st, a, gb); break;
    }
}

hipError_t launch_backward(const GradBufs &b, int64_t nsp, hipStream_t st, const BatchInfo *bi);

// Ebar, var and the non-finite count of ns local energies into stats[4].
hipError_t launch_stats(int64_t ns, const double *eloc, const double *w, double *stats, hipStream_t st) {
    hipLaunchKernelGGL(stats_kernel, dim3(1, 1), dim3(1024), 0, st, ns, eloc, w, stats);
    return hipGetLastError();
}

// bi: NULL, or the batch of vmc_step_batched; b then describes problem 0 with
// the longest chain's sizes (grad and stats of problem k at k * pitch_p and
// k * 4, local energies at k * 2 ns).
// chunk: the samples are one chunk of a larger set: b.stats holds that set's
// statistics (not computed here) and the chunk's gradient is added to b.grad.
hipError_t launch_grad(const GradBufs &b, hipStream_t st, const BatchInfo *bi, bool chunk) {
    const Dims &d = b.d;
    const int nb = bi ? bi->n : 0;
    if (nb > 0 && (b.coef_lp || b.weights || chunk)) return hipErrorInvalidValue;
    if (!b.coef_lp && !chunk)
        hipLaunchKernelGGL(stats_kernel, dim3(1, nb > 0 ? nb : 1), dim3(1024), 0, st, b.ns, b.eloc, b.weights,
                           b.stats);
    hipError_t e = launch_backward(b, grad_nsp(b.ns), st, bi);
    if (e != hipSuccess) return e;
    const int64_t nsp = grad_nsp(b.ns);
    // per-problem chunking of the weight-gradient contraction (as vmc_step alone)
    DwBatch gbs[3];
    for (int seg = 0; seg < 3; seg++) {
        gbs[seg].n = nb;
        if (nb == 0) continue;
        gbs[seg].pitch_ws = bi->pitch_ws;
        gbs[seg].pitch_p = bi->pitch_p;
        for (int k = 0; k < nb; k++) {
            Dims dk = d;
            dk.N = dk.Lx = bi->N[k];
            const SegDims sk = seg_dims(dk, seg);
            gbs[seg].N[k] = bi->N[k];
            gbs[seg].nchunk[k] = dw_chunks(dk, sk, nsp);
            gbs[seg].chunk[k] = ((nsp + gbs[seg].nchunk[k] - 1) / gbs[seg].nchunk[k] + 31) / 32 * 32;
        }
    }
    {
        const int64_t tot = (int64_t)d.N * nsp;
        const int g2 = (int)((tot + 255) / 256 < 8192 ? (tot + 255) / 256 : 8192);
        const dim3 grid(g2, nb > 0 ? nb : 1);
        const int64_t pcfg = nb > 0 ? bi->pitch_cfg : 0;
        if (d.prec == VMC_BF16)
            hipLaunchKernelGGL(build_extras<BF16>, grid, dim3(256), 0, st, d, b.ns, nsp, b.cfg, (uint16_t *)b.xT,
                               gbs[0], pcfg);
        else
            hipLaunchKernelGGL(build_extras<F32>, grid, dim3(256), 0, st, d, b.ns, nsp, b.cfg, (float *)b.xT, gbs[0],
                               pcfg);
    }
    const int64_t P = param_layout(d.dims, d.dh, d.glu, d.cplx).total;
    const int64_t Pall = nb > 0 ? (int64_t)(nb - 1) * bi->pitch_p + P : P;
    if (!chunk)
        hipLaunchKernelGGL(fill_f64, dim3((int)((Pall + 255) / 256 < 4096 ? (Pall + 255) / 256 : 4096)), dim3(256), 0,
                           st, b.grad, Pall, 0.0);
    for (int seg = 0; seg < 3; seg++) {
        if (seg == 1 && !d.glu) continue;
        SegDims sd = seg_dims(d, seg);
        DwArgs a;
        a.d = d;
        a.seg = seg;
        a.ns = b.ns;
        a.nsp = grad_nsp(b.ns);
        a.A = seg == 0 ? b.dtc : seg == 1 ? b.dtg : b.dth;
        a.MD = sd.MD;
        a.K = sd.K;
        a.Mp = sd.Mp;
        a.Kp = sd.Kp;
        a.hT = b.hT;
        a.gT = b.gT;
        a.xT = b.xT;
        a.part = b.part;
        a.nchunk = dw_chunks(d, sd, a.nsp);
        a.chunk = ((a.nsp + a.nchunk - 1) / a.nchunk + 31) / 32 * 32;
        a.units = d.N * a.nchunk;
        a.tiles_m = dw_tiles_m(sd);
        a.tiles = a.tiles_m * dw_tiles_n(sd);
        int units_max = a.units;
        for (int k = 0; k < nb; k++) {
            const int u = gbs[seg].N[k] * gbs[seg].nchunk[k];
            units_max = u > units_max ? u : units_max;
        }
        if (d.prec == VMC_BF16) launch_dw_p<BF16>(a, sd, gbs[seg], units_max, st);
        else launch_dw_p<F32>(a, sd, gbs[seg], units_max, st);
        const int rg = sd.MD * ((sd.K + 5 + 31) / 32);
        hipLaunchKernelGGL(dw_reduce, dim3(rg, nb > 0 ? nb : 1), dim3(256), 0, st, d, seg, b.part, d.N * a.nchunk,
                           sd.Mp, sd.Kp, sd.K, sd.MD, b.grad, gbs[seg], chunk ? 1 : 0);
    }
    return hipGetLastError();
}

}  // namespace vmc
