// Forward engine of the GRU RNN wave function on gfx950 (kernel template;
// instantiated per precision and dimension in engine_*.hip).
//
// One kernel runs the autoregressive chain (Eq. 1) for a tile of rows over a
// range of order positions.  A row is a sample (sampling, Sec. II A, or the
// teacher-forced log psi) or a connected configuration of the local energy
// (the chain after its first changed order position, Eqs. 6-7).  Per order
// position q a tile does:
//   1. operands in LDS: the hidden input(s) (1D: h_{n-1}; 2D: [h_hz | h_vt],
//      App. A) and an indicator block that carries the one-hot inputs and a
//      constant column, so the one-hot columns and the biases of the gate
//      matrices ride on the MFMA (bfloat16: hi/lo split of those weights,
//      i.e. ~16 significant bits);
//   2. the cell contraction on MFMA, each wave owning all gate columns of a
//      slice of hidden units, so the App. A gate algebra runs in registers on
//      the MFMA output;
//   3. the optional GLU contraction on MFMA;
//   4. the 2- or 4-logit heads (Eqs. 3, 5) in FP32 as lane partial dot
//      products, a sum over the lane groups and a cross-wave sum in LDS;
//   5. a per-row finalisation: log-softmax, the sampling decision or the
//      teacher-forced spin, FP64 accumulation of log P and the phase.
// The weights are the MFMA A operand, so a lane owns 4 consecutive hidden
// units of one row: the new h goes to LDS as one 8- or 16-byte store and a
// head sum needs only the four lane groups of a row.  With REGW the cell and
// GLU weights stay in registers for the whole persistent launch; otherwise
// both stream from L2.
//
// Teacher-forced rows (log psi, local energy) know every input in advance,
// so one workgroup barrier per position suffices: the phase of position q
// runs the GLU and heads of q, the cell of q+1, the operand staging of q+2
// and the finalisation of q-1, on double-buffered hidden, vertical and
// indicator tiles and triple-buffered head sums.  Sampling draws the spin of
// q before the cell of q+1 can start and keeps three barriers per position.
#pragma once
#include <algorithm>
#include <type_traits>

#include "kernels.h"

namespace vmc {

// Tile shape by tile class TC.  TC = 1: the suffix-chain launch (persistent).
// TC = 0: one tile per work-group over the samples (sampling, log psi); at
// bfloat16 d_h = 128 the 1D tile is made shorter (48 rows) so that 10^4
// samples occupy more compute units, while the 2D tile keeps 64 rows (its
// vertical-input prefetch makes the taller tile the faster one).  TC = 2: the
// alternative row tile that the tuning table can select (the other of 48 and
// 64 at bfloat16 d_h = 128, half the chain tile elsewhere); where it does not
// exist (HAS_ALT false) TC = 2 has the TC = 0 shape and is never launched.
// Every row of a tile is computed independently of the others, so the tile
// choice does not change any result bit.
template <class P, int DIMS, int DH, int NW, int TC = 0>
struct Eng {
    static constexpr int WU = (DH / 16 < NW) ? DH / 16 : NW;  // waves along hidden units
    static constexpr int WR = NW / WU;                        // waves along rows
    static constexpr int UW = DH / WU;
    static constexpr int UB = UW / 16;
    // rows per tile (FP32 tiles at d_h >= 128 are halved to fit the LDS;
    // bfloat16 d_h = 256 with 8 waves: 48, the most that fits)
    static constexpr int MT_CHAIN =
        (P::VEC == 4 && DH >= 128) ? 32 : DH >= 256 ? (P::VEC == 8 && NW == 8 ? 48 : 32) : 64;
    static constexpr bool BIG = P::VEC == 8 && DH == 128 && NW == 8;
    static constexpr int MT_ROW = BIG ? (DIMS == 2 ? 64 : 48) : MT_CHAIN;
    static constexpr int MT_ALT = BIG ? (DIMS == 2 ? 48 : 64) : MT_CHAIN / 2;
    static constexpr bool HAS_ALT = MT_ALT != MT_ROW && MT_ALT % (16 * WR) == 0;
    static constexpr int MT = TC == 1 ? MT_CHAIN : (TC == 2 && HAS_ALT) ? MT_ALT : MT_ROW;
    static constexpr int RW = MT / WR;
    static constexpr int RB = RW / 16;
    static constexpr int KS = P::KSTEP;
    static constexpr int KHB = cround(DH, KS);                 // one hidden block of the operand
    static constexpr int NKB = KHB / KS;                       // k-steps per hidden block
    static constexpr int NHB = DIMS == 1 ? 1 : 2;              // hidden blocks (hz, vt)
    static constexpr int NKS = NHB * NKB + 1;                  // + the indicator step
    static constexpr int KPX = NKS * KS;                       // staged row length of Bc
    static constexpr int PADE = 16 / (int)sizeof(typename P::store_t);
    static constexpr int H_LD = KHB + PADE;                    // row stride of sH / sV
    static constexpr int X_LD = KS + PADE;                     // row stride of the indicator tile
    static constexpr int NLOG = 3;                             // head-sum buffers
    // Register-resident weights (bfloat16, d_h <= 128): the one-hot inputs and
    // gate biases enter the cell as the accumulators' start values, read from an
    // FP32 table [gate][input class][unit] instead of an indicator k-step of
    // MFMAs.  Input class = (x_hz + 1) + 3 (x_vt + 1), x = -1 when absent.
    static constexpr bool XT = P::VEC == 8 && DH <= 128;
    static constexpr int NXC = DIMS == 1 ? 3 : 9;              // input classes
    static constexpr int NXG = DIMS == 1 ? 3 : 2;              // gates with inputs or a bias
    static constexpr int XT_LD = DH + 4;                       // class stride: classes on distinct banks
    // static LDS of the kernel (bytes), for the host-side capacity check
    static constexpr size_t LDS =
        sizeof(typename P::store_t) *
            ((size_t)2 * MT * H_LD + (DIMS == 2 ? 2 * MT * H_LD : 8) + (XT ? 16 : 2 * MT * X_LD)) +
        4 * ((size_t)NLOG * WU * MT * 4 + 6 * DH) + 8 * MT + 16 * MT + 16 +
        (XT ? 4 * ((size_t)NXG * NXC * XT_LD + 2 * MT) : 16);  // (+ the LDS constants of streamed weights)
};

constexpr int kXcdsE = 8;  // XCDs of the chip

// Read-only tables written by earlier launches (position table, tile
// schedule): through the constant address space, so that reads at uniform
// indices become scalar loads.
template <class T>
__device__ inline const __attribute__((address_space(4))) T *kconst(const T *p) {
    return (const __attribute__((address_space(4))) T *)p;
}

// Sums over the four 16-lane groups of two values at once: p ends up summed
// in lanes 0-31 and q in lanes 32-63 (same bits within each half).  One
// v_permlane32_swap exchanges the upper half of p with the lower half of q,
// one v_permlane16_swap then pairs the remaining rows.
__device__ inline float pair_sum4(float p, float q) {
    const auto x = __builtin_amdgcn_permlane32_swap(__float_as_uint(p), __float_as_uint(q), false, false);
    const float s = __uint_as_float(x[0]) + __uint_as_float(x[1]);
    const uint32_t c = __float_as_uint(s);
    const auto y = __builtin_amdgcn_permlane16_swap(c, c, false, false);
    return __uint_as_float(y[0]) + __uint_as_float(y[1]);
}

// Four consecutive units of one row (one 8- or 16-byte store).
template <class P>
__device__ inline void put4(typename P::store_t *dst, const float *v);
template <>
__device__ inline void put4<F32>(float *dst, const float *v) {
    *(float4 *)dst = make_float4(v[0], v[1], v[2], v[3]);
}
template <>
__device__ inline void put4<BF16>(uint16_t *dst, const float *v) {
    *(uint2 *)dst = make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
}

template <class P>
__device__ inline typename P::store_t cvt(float x);
template <>
__device__ inline float cvt<F32>(float x) { return x; }
template <>
__device__ inline uint16_t cvt<BF16>(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

// Facts of one order position (the position table, see build_postab).
struct PosInfo {
    int site, site_hz, site_vt, pos_vt, icol;
    int colw;  // h of this position is a later vertical input (kept in the column buffer);
               // an int, so that the struct has no padding bytes to copy through private memory
};

// CPX: the complex (phase) head fixed at compile time (0 or 1) or read at run
// time (-1).  The chain launch is instantiated for both values: without the
// run-time branches its epilogue basic blocks are larger and better scheduled.
// (waves per SIMD the compiler must allow: what the work-group size implies,
// except for the 1D d_h = 64 chain launch, which is latency-bound and runs
// faster with three 4-wave work-groups per compute unit at 168 registers, a
// few spilled, than with two at 184)
template <class P, int DIMS, int DH, int NW, int REGW, int STORE, int TF, int TC, int CPX = -1, int BATCH = 0>
__global__ __launch_bounds__(NW * 64)
__attribute__((amdgpu_waves_per_eu((DIMS == 1 && DH == 64 && TC == 1) ? 3 : (NW * 64 + 255) / 256)))
void rnn_engine(FwdArgs a0, BatchInfo bi, int mode, int store_h_, int store_lpc_, int store_act_) {
    // cache writes exist only in the STORE variant (the chain kernel has none)
    const int store_h = STORE && store_h_, store_lpc = STORE && store_lpc_, store_act = STORE && store_act_;
    // the launch mode is fixed by the instantiation: the chain tile class runs
    // MODE_CHAIN only, TF = 0 is sampling, TF = 1 otherwise (see launch_engine_t)
    constexpr bool CHAIN = TC == 1;
    typedef Eng<P, DIMS, DH, NW, TC> C;
    typedef typename P::store_t T;
    constexpr int MT = C::MT, RB = C::RB, UB = C::UB, KS = C::KS, VEC = P::VEC;
    constexpr int KHB = C::KHB, NKB = C::NKB, NKS = C::NKS, KPX = C::KPX;
    constexpr int H_LD = C::H_LD, X_LD = C::X_LD, NT = NW * 64;
    constexpr int NKG = KHB / KS;          // k-steps of the GLU contraction
    constexpr int NA = DIMS == 1 ? 4 : 3;  // gate features; the GLU pair follows
    constexpr int NCH = MT * (DH / VEC), PF = (NCH + NT - 1) / NT;  // 16-byte chunks of an h tile

    __shared__ __align__(16) T sH[2][MT * H_LD];
    __shared__ __align__(16) T sV[DIMS == 2 ? 2 : 1][DIMS == 2 ? MT * H_LD : 8];
    static_assert(C::XT == (bool)REGW, "input table goes with register-resident weights");
    constexpr bool XT = C::XT;
    __shared__ __align__(16) T sX[2][XT ? 8 : MT * X_LD];
    __shared__ __align__(16) float sXt[XT ? C::NXG : 1][XT ? C::NXC : 1][XT ? C::XT_LD : 4];
    __shared__ int sCmb[2][XT ? MT : 1];  // input class of each row, double-buffered like sX
    __shared__ __align__(16) float sLog[C::NLOG][C::WU][MT][4];
    __shared__ __align__(16) float sHw[2][DH];  // phase-head rows (complex amplitudes)
    // streamed weights (no REGW): the per-unit GLU biases and amplitude-head
    // rows live in LDS instead of registers
    constexpr bool CL = !REGW;
    __shared__ __align__(16) float sCst[CL ? 4 : 1][CL ? DH : 4];
    __shared__ int sRow[MT], sCid[MT];
    __shared__ double2 sAcc[MT];  // running (log P, phase) of each row, FP64
    __shared__ int sTile;
    extern __shared__ uint8_t sSig[];  // [MT][N]

    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = w / C::WU, wu = w % C::WU;
    // the arguments of this work-group's problem (a batched row launch: one
    // problem per group of `bi.tiles` work-groups; the batched chain launch
    // rebases per tile)
    FwdArgs a = a0;
    // row launches: work-groups go to the XCDs round-robin by id, and a tile
    // that is not a multiple of 32 rows shares 128-byte lines of the FP32
    // [logit][sample] arrays with its neighbours, so each XCD takes a
    // contiguous run of tiles (XCD x: G/8 tiles, plus one if x < G % 8)
    int row_tile = blockIdx.x;
    if (!CHAIN) {
        const int G = gridDim.x, b = blockIdx.x, x = b % kXcdsE;
        const int q = G / kXcdsE, rm = G - q * kXcdsE;
        row_tile = __builtin_amdgcn_readfirstlane(x * q + min(x, rm) + b / kXcdsE);
    }
    if (BATCH && !CHAIN) {
        const int k = row_tile / bi.tiles;
        row_tile -= k * bi.tiles;
        rebase_fwd(a, bi, k);
    }
    const int cplx = CPX >= 0 ? CPX : a.d.cplx, glu = a.d.glu;
    const int64_t ns_c = a.ns_cache;
    const int l16 = lane & 15, lq = lane >> 4;
    auto unit0 = [&](int ub) __attribute__((always_inline)) { return wu * C::UW + ub * 16 + 4 * lq; };

    // per-problem state, set by setup(): sizes, weight pointers, the per-lane
    // constants of this lane's units (GLU biases, amplitude head), the
    // register-resident weights and the LDS tables
    int N, Lx, Ly;
    const T *__restrict__ Bc;
    const T *__restrict__ Bg;
    const T *__restrict__ hcs;
    const int4 *__restrict__ postab;
    T *colbuf;
    float gb1[UB][4], gb2[UB][4], hw0[UB][4], hw1[UB][4];
    float bin_[DIMS == 1 ? UB : 1][4], win0[DIMS == 1 ? UB : 1][4], win1[DIMS == 1 ? UB : 1][4];
    float hc0, hc1, hc2, hc3;
    // REGW: cell and GLU weight fragments in registers for the whole launch
    // (the hidden k-steps; the indicator columns come from the input table)
    i32x4_t wreg[REGW ? 3 : 1][REGW ? NKS - 1 : 1][REGW ? UB : 1];
    uint4 wgl[REGW ? 2 : 1][REGW ? NKG : 1][REGW ? UB : 1];
    auto setup = [&]() __attribute__((always_inline)) {
        N = a.d.N;
        Lx = a.d.Lx;
        Ly = a.d.Ly;
        Bc = (const T *)a.Bc;
        Bg = (const T *)a.Bg;
        hcs = (const T *)a.hcs;
        postab = a.postab;
        colbuf = (T *)a.colbuf + (int64_t)blockIdx.x * Lx * MT * DH;
#pragma unroll
        for (int ub = 0; ub < UB; ub++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int u = unit0(ub) + i;
                if (!CL) {
                    gb1[ub][i] = a.E[E_B1 * DH + u];
                    gb2[ub][i] = a.E[E_B2 * DH + u];
                    hw0[ub][i] = a.Hd[u];
                    hw1[ub][i] = a.Hd[DH + u];
                }
                if (DIMS == 1) {
                    bin_[ub % (DIMS == 1 ? UB : 1)][i] = a.E[E1_BIN * DH + u];
                    win0[ub % (DIMS == 1 ? UB : 1)][i] = a.E[E1_XIN0 * DH + u];
                    win1[ub % (DIMS == 1 ? UB : 1)][i] = a.E[E1_XIN1 * DH + u];
                }
            }
        for (int e = tid; e < 2 * DH; e += NT) (&sHw[0][0])[e] = a.Hd[2 * DH + e];
        if (CL)
            for (int e = tid; e < 4 * DH; e += NT) {
                const int k = e / DH, u = e - k * DH;
                sCst[CL ? k : 0][CL ? u : 0] = k == 0 ? a.E[E_B1 * DH + u] : k == 1 ? a.E[E_B2 * DH + u] : a.Hd[(k - 2) * DH + u];
            }
        hc0 = a.hc[0];
        hc1 = a.hc[1];
        hc2 = a.hc[2];
        hc3 = a.hc[3];
        if (REGW) {
#pragma unroll
            for (int g = 0; g < 3; g++)
#pragma unroll
                for (int ks = 0; ks < NKS - 1; ks++)
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) {
                        const int n = g * DH + wu * C::UW + ub * 16 + l16;
                        wreg[g][ks][ub] = *(const i32x4_t *)&Bc[(int64_t)n * KPX + ks * KS + VEC * lq];
                    }
#pragma unroll
            for (int g = 0; g < 2; g++)
#pragma unroll
                for (int kq = 0; kq < NKG; kq++)
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) {
                        const int n = g * DH + wu * C::UW + ub * 16 + l16;
                        wgl[g][kq][ub] = *(const uint4 *)&Bg[(int64_t)n * KHB + kq * KS + VEC * lq];
                    }
        }
        if (XT)
            for (int e = tid; e < C::NXG * C::NXC * DH; e += NT) {
                const int g = e / (C::NXC * DH), r = e - g * (C::NXC * DH), cls = r / DH, u = r - cls * DH;
                const int xz = cls % 3 - 1, xv = cls / 3 - 1;
                float v;
                if (DIMS == 1) {
                    // gates u, r: bias + one-hot weight of x_{n-1}; gate m: its bias only
                    const float *e1 = a.E + (int64_t)(3 * g) * DH + u;
                    v = e1[0];
                    if (g < 2) v += xz == 0 ? e1[DH] : xz == 1 ? e1[2 * DH] : 0.f;
                } else {
                    // gates c, u: bias + one-hot weights of the horizontal and vertical inputs
                    const float *e2 = a.E + (int64_t)(5 * g) * DH + u;
                    v = e2[0];
                    v += xz == 0 ? e2[DH] : xz == 1 ? e2[2 * DH] : 0.f;
                    v += xv == 0 ? e2[3 * DH] : xv == 1 ? e2[4 * DH] : 0.f;
                }
                sXt[XT ? g : 0][XT ? cls : 0][XT ? u : 0] = v;
            }
    };
    if (!(BATCH && CHAIN)) setup();
    // constant k (0: GLU bias 1, 1: GLU bias 2, 2, 3: amplitude-head rows) of the lane's 4 units of block ub
    auto cst4 = [&](int k, int ub, float *v) __attribute__((always_inline)) {
        if (CL) {
            const float4 t = *(const float4 *)&sCst[CL ? k : 0][CL ? unit0(ub) : 0];
            v[0] = t.x;
            v[1] = t.y;
            v[2] = t.z;
            v[3] = t.w;
        } else {
#pragma unroll
            for (int i = 0; i < 4; i++) v[i] = k == 0 ? gb1[ub][i] : k == 1 ? gb2[ub][i] : k == 2 ? hw0[ub][i] : hw1[ub][i];
        }
    };
    for (int e = tid; e < C::NLOG * C::WU * MT * 4; e += NT) (&sLog[0][0][0][0])[e] = 0.f;
    // Philox counter of the sampling decisions: given, or read once from device memory
    const uint64_t ctr = (!TF && a.counter_dev) ? *kconst(a.counter_dev) : a.counter;
    // zero the operand tiles once (padding columns stay zero); the bias
    // class of the indicator block is always on
    for (int e = tid; e < 2 * MT * H_LD; e += NT) (&sH[0][0])[e] = cvt<P>(0.f);
    if (DIMS == 2)
        for (int e = tid; e < 2 * MT * H_LD; e += NT) (&sV[0][0])[e] = cvt<P>(0.f);
    if (!XT)
        for (int e = tid; e < 2 * MT * X_LD; e += NT) {
            const int c = e % X_LD;
            const bool bias_col = VEC == 8 ? (c == 8 || c == 9) : c == 4;
            (&sX[0][0])[e] = cvt<P>(bias_col ? 1.f : 0.f);
        }

    auto pos = [&](int qn) -> PosInfo __attribute__((always_inline)) {
        const auto *pt = kconst((const int *)postab) + 4 * qn;
        const int4 t = make_int4(pt[0], pt[1], pt[2], pt[3]);
        PosInfo r;
        r.site = t.x & 0xFFFF;
        r.colw = DIMS == 2 && ((t.x >> 16) & 1);
        r.site_hz = t.y;
        r.site_vt = DIMS == 2 ? t.z : -1;
        r.pos_vt = (t.w & 0xFFFF) - 1;
        r.icol = t.w >> 16;
        return r;
    };

    // Head outputs of one 16-row block: sum the lane partials over the four
    // lane groups of a row, then one lane group stores the wave's sums.
    // the wave's partial logits of row r: the amplitude pair from lanes 0-15
    // (logit 0) and 32-47 (logit 1), the phase pair likewise; the phase slots
    // of a positive RNN stay at the zeros written at the start
    auto head_out = [&](int lb, int r, float p0, float p1, float p2, float p3) __attribute__((always_inline)) {
        const float t01 = pair_sum4(p0, p1);
        const float t23 = cplx ? pair_sum4(p2, p3) : 0.f;
        if ((lq & 1) == 0) {
            float *d = &sLog[lb][wu][r][lq >> 1];
            d[0] = t01;
            if (cplx) d[2] = t23;
        }
    };
    // partial head sums of the lane's 4 units of one row
    auto head_part = [&](int ub, const float *g, float &p0, float &p1, float &p2, float &p3) __attribute__((always_inline)) {
        float w0[4], w1[4];
        cst4(2, ub, w0);
        cst4(3, ub, w1);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            p0 += w0[i] * g[i];
            p1 += w1[i] * g[i];
        }
        if (cplx) {
            const float4 z0 = *(const float4 *)&sHw[0][unit0(ub)];
            const float4 z1 = *(const float4 *)&sHw[1][unit0(ub)];
            p2 += z0.x * g[0] + z0.y * g[1] + z0.z * g[2] + z0.w * g[3];
            p3 += z1.x * g[0] + z1.y * g[1] + z1.z * g[2] + z1.w * g[3];
        }
    };

    bool first = true;
    int cur_prob = -1;  // batched chain launch: the problem whose state setup() loaded
    // chain launches: thread 0 claims the next tile from the queue while the
    // current one runs (a claimed tile is always run: the loop ends only on a
    // claim past the last tile)
    int claim = 0;
    for (;;) {
        // ---------------------------------------------------------- tile
        int p = -1, nrow;
        int64_t e0;
        if (CHAIN && BATCH) {
            __syncthreads();
            if (tid == 0) sTile = first ? atomicAdd(a0.tile_counter, 1) : claim;
            __syncthreads();
            // one queue over the tiles of every problem, longest chains first:
            // the entry (first tile, problem, position) that holds tile t
            const int t = __builtin_amdgcn_readfirstlane(sTile);
            const auto *sc = kconst((const int *)bi.sched);
            if (t >= sc[4 * bi.nsched]) break;
            if (tid == 0) claim = atomicAdd(a0.tile_counter, 1);
            int lo = 0, hi = bi.nsched - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (sc[4 * mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            const int k = sc[4 * lo + 1];
            p = sc[4 * lo + 2];
            e0 = (int64_t)(t - sc[4 * lo]) * MT;
            if (k != cur_prob) {
                a = a0;
                rebase_fwd(a, bi, k);
                setup();
                cur_prob = k;
            }
            nrow = (int)min((int64_t)MT, (int64_t)kconst(a.cnt)[p] - e0);
        } else if (CHAIN) {
            __syncthreads();
            if (tid == 0) sTile = first ? atomicAdd(a.tile_counter, 1) : claim;
            __syncthreads();
            // uniform across the work-group: the position loop, its table reads
            // and branches then run on the scalar unit
            const int t = __builtin_amdgcn_readfirstlane(sTile);
            const auto *ts = kconst(a.tile_start);
            if (t >= ts[N]) break;
            if (tid == 0) claim = atomicAdd(a.tile_counter, 1);
            int lo = 0, hi = N - 1;  // largest p with tile_start[p] <= t
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (ts[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            p = lo;
            e0 = (int64_t)(t - ts[p]) * MT;
            nrow = (int)min((int64_t)MT, (int64_t)kconst(a.cnt)[p] - e0);
        } else {
            if (!first) break;
            e0 = (int64_t)row_tile * MT;
            nrow = (int)min((int64_t)MT, a.nrows - e0);
        }
        first = false;

        // ------------------------------------------------------ row setup
        int my_s = -1, f1 = -1, f2 = -1, cidx = 0;  // of row tid (tid < MT)
        if (tid < MT) {
            if (tid < nrow) {
                const int64_t ent = e0 + tid;
                if (!CHAIN) {
                    my_s = (int)ent;
                } else if (a.ham_kind == 0) {
                    my_s = (int)ent;
                    f1 = order_site(p, Lx);
                    cidx = p;
                } else {
                    const int conn = a.list[a.list_off[p] + ent];
                    my_s = conn / a.nbond;
                    cidx = conn - my_s * a.nbond;
                    conn_sites(a.ham_kind, cidx, Lx, Ly, f1, f2);
                }
            }
            sRow[tid] = my_s;
            sCid[tid] = cidx;
            sAcc[tid] = make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (TF) {
            // eight loads per thread in flight together (an absent row reads row 0
            // and is zeroed), then the stores
            constexpr int BQ = 8;
            const int tot = MT * N;
            for (int eb = tid; eb < tot; eb += BQ * NT) {
                uint8_t v[BQ];
#pragma unroll
                for (int j = 0; j < BQ; j++) {
                    const int e = min(eb + j * NT, tot - 1), r = e / N, c = e - r * N;
                    const int s = sRow[r];
                    v[j] = a.cfg_in[(int64_t)(s >= 0 ? s : 0) * N + c];
                    v[j] = s >= 0 ? v[j] : (uint8_t)0;
                }
#pragma unroll
                for (int j = 0; j < BQ; j++)
                    if (eb + j * NT < tot) sSig[eb + j * NT] = v[j];
            }
        } else {
            for (int e = tid; e < MT * N; e += NT) sSig[e] = 0;
        }
        __syncthreads();
        if (tid < MT && my_s >= 0 && CHAIN) {
            sSig[tid * N + f1] ^= 1;
            if (f2 >= 0) sSig[tid * N + f2] ^= 1;
        }
        __syncthreads();
        // previous hidden state of the first step: h(p) from the prefix cache
        float hreg[DIMS == 1 ? RB : 1][DIMS == 1 ? UB : 1][4];
#pragma unroll
        for (int rb = 0; rb < (DIMS == 1 ? RB : 1); rb++)
#pragma unroll
            for (int ub = 0; ub < (DIMS == 1 ? UB : 1); ub++)
#pragma unroll
                for (int i = 0; i < 4; i++) hreg[rb][ub][i] = 0.f;
        if (p >= 0) {
            // every load first (an absent row reads row 0 and is zeroed), then
            // the LDS stores
            uint4 hv[PF];
#pragma unroll
            for (int i = 0; i < PF; i++) {
                const int e = min(tid + i * NT, NCH - 1);
                const int r = e / (DH / VEC), c = (e % (DH / VEC)) * VEC;
                const int s = sRow[r];
                hv[i] = *(const uint4 *)&hcs[((int64_t)p * ns_c + (s >= 0 ? s : 0)) * DH + c];
                if (s < 0) hv[i] = make_uint4(0, 0, 0, 0);
            }
            if (DIMS == 1) {
#pragma unroll
                for (int rb = 0; rb < RB; rb++) {
                    const int s = sRow[wr * C::RW + rb * 16 + l16];
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) {
                        float4 v = *(const float4 *)&a.hcache[((int64_t)p * ns_c + (s >= 0 ? s : 0)) * DH + unit0(ub)];
                        if (s < 0) v = make_float4(0.f, 0.f, 0.f, 0.f);
                        float *hr = hreg[rb % (DIMS == 1 ? RB : 1)][ub % (DIMS == 1 ? UB : 1)];
                        hr[0] = v.x;
                        hr[1] = v.y;
                        hr[2] = v.z;
                        hr[3] = v.w;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < PF; i++) {
                const int e = tid + i * NT;
                if (e < NCH) {
                    const int r = e / (DH / VEC), c = (e % (DH / VEC)) * VEC;
                    *(uint4 *)&sH[p & 1][r * H_LD + c] = hv[i];
                }
            }
        }

        // -------------------------------------------------- phase pieces
        // vertical input rows of a position (2D, not the row start): from the
        // prefix cache (positions <= p) or from the column buffer
        // (the prefetched chunks are a value passed from vt_issue to vt_store, so
        // that they live in registers for one phase, not in a private array)
        struct Pfv {
            uint4 v[PF];
        };
        auto vt_needed = [&](int qn, const PosInfo &pi) __attribute__((always_inline)) {
            return DIMS == 2 && pi.site_vt >= 0 && pi.pos_vt < qn - 1;
        };
        // (chunk e of a tile is row e / (DH / VEC), columns (e % (DH / VEC)) * VEC:
        // offset e * VEC in a row-major [MT][DH] block, so the column buffer is
        // addressed as a uniform base plus a 32-bit per-lane offset)
        auto vt_issue = [&](const PosInfo &pi) -> Pfv __attribute__((always_inline)) {
            const bool cache = CHAIN && pi.pos_vt <= p;
            const T *cb = colbuf + (int64_t)pi.icol * (MT * DH);
            Pfv f;
#pragma unroll
            for (int i = 0; i < PF; i++) {
                const int e = tid + i * NT;
                f.v[i] = make_uint4(0, 0, 0, 0);
                if (e < NCH) {
                    if (cache) {
                        const int r = e / (DH / VEC), c = (e % (DH / VEC)) * VEC;
                        const int s = sRow[r];
                        if (s >= 0) f.v[i] = *(const uint4 *)&hcs[((int64_t)pi.pos_vt * ns_c + s) * DH + c];
                    } else {
                        f.v[i] = *(const uint4 *)(cb + (uint32_t)(e * VEC));
                    }
                }
            }
            return f;
        };
        auto vt_store = [&](int buf, const Pfv &f) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < PF; i++) {
                const int e = tid + i * NT;
                if (e < NCH) {
                    const int r = e / (DH / VEC), c = (e % (DH / VEC)) * VEC;
                    *(uint4 *)&sV[DIMS == 2 ? buf : 0][r * H_LD + c] = f.v[i];
                }
            }
        };
        // h of position qn into the column buffer (its column's next vertical input)
        auto col_copy = [&](int qn, const PosInfo &pi) __attribute__((always_inline)) {
            T *cb = colbuf + (int64_t)pi.icol * (MT * DH);
            for (int e = tid; e < NCH; e += NT) {
                const int r = e / (DH / VEC), c = (e % (DH / VEC)) * VEC;
                *(uint4 *)(cb + (uint32_t)(e * VEC)) = *(const uint4 *)&sH[qn & 1][r * H_LD + c];
            }
        };
        // indicator columns of position qn, one row per lane of wave iw (one 16-byte store):
        // FP32 [x_hz0, x_hz1, x_vt0, x_vt1]; BF16 each twice (hi, lo)
        auto indicator = [&](const PosInfo &pi, int buf, int iw) __attribute__((always_inline)) {
            if (w != iw || lane >= MT) return;
            const int orow = lane;
            const int xz = pi.site_hz >= 0 ? sSig[orow * N + pi.site_hz] : -1;
            const int xv = pi.site_vt >= 0 ? sSig[orow * N + pi.site_vt] : -1;
            if (XT) {
                sCmb[buf][XT ? orow : 0] = (xz + 1) + 3 * (xv + 1);
            } else {
                const uint32_t one = VEC == 8 ? 0x3F803F80u : 0x3F800000u;
                *(uint4 *)&sX[buf][orow * X_LD] = make_uint4(xz == 0 ? one : 0u, xz == 1 ? one : 0u,
                                                             xv == 0 ? one : 0u, xv == 1 ? one : 0u);
            }
        };

        // cell of position qc: A fragment of row block rb, k-step ks
        auto a_frag = [&](int qc, bool vt_prev, int rb, int ks) -> uint4 __attribute__((always_inline)) {
            const int blk = ks / NKB;
            const bool is_x = ks == NKS - 1;
            const T *Aop = is_x ? sX[qc & 1] : (blk == 0 || vt_prev) ? sH[(qc - 1) & 1] : sV[DIMS == 2 ? (qc & 1) : 0];
            const int ald = is_x ? X_LD : H_LD;
            const int kc = is_x ? 0 : (ks % NKB) * KS;
            const int arow = wr * C::RW + rb * 16 + l16;
            return *(const uint4 *)&Aop[arow * ald + kc + VEC * lq];
        };
        // gate algebra (App. A) on the cell MFMA output of row block rb
        auto cell_epi = [&](int qc, const PosInfo &pi, int rb, const f32x4_t *acc) __attribute__((always_inline)) {
            const int r = wr * C::RW + rb * 16 + l16;
            const int s = sRow[r];
            int xz = 0;
            if (DIMS == 1) xz = pi.site_hz >= 0 ? sSig[r * N + pi.site_hz] : -1;
            float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
            for (int ub = 0; ub < UB; ub++) {
                const int u0 = unit0(ub);
                float hq[4], gv[STORE ? 4 : 1][4];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const float g0 = acc[ub][i], g1 = acc[UB + ub][i], g2 = acc[2 * UB + ub][i];
                    float h, s0, s1, s2, s3 = 0.f;
                    if (DIMS == 1) {
                        const int ud = ub % (DIMS == 1 ? UB : 1);
                        const float uu = sigmoidf_(g0);
                        const float rr = sigmoidf_(g1);
                        const float cin = bin_[ud][i] + (xz == 0 ? win0[ud][i] : (xz == 1 ? win1[ud][i] : 0.f));
                        const float c = tanhf_(rr * g2 + cin);
                        float &hp = hreg[rb % (DIMS == 1 ? RB : 1)][ud][i];
                        h = hp + uu * (c - hp);
                        hp = h;
                        s0 = uu; s1 = rr; s2 = g2; s3 = c;
                    } else {
                        const float c = tanhf_(g0);
                        const float uu = sigmoidf_(g1);
                        h = g2 + uu * (c - g2);
                        s0 = c; s1 = uu; s2 = g2;
                    }
                    hq[i] = (STORE && s < 0) ? 0.f : h;
                    if (STORE) {
                        const bool ok = s >= 0;
                        gv[0][i] = ok ? s0 : 0.f;
                        gv[STORE ? 1 : 0][i] = ok ? s1 : 0.f;
                        gv[STORE ? 2 : 0][i] = ok ? s2 : 0.f;
                        gv[STORE ? 3 : 0][i] = ok ? s3 : 0.f;
                    }
                }
                put4<P>(&sH[qc & 1][r * H_LD + u0], hq);
                if (!glu) head_part(ub, hq, p0, p1, p2, p3);
                if (STORE) {
                    if (s >= 0 && store_h) {
                        // FP32 states: read by the 1D chains and 1D backward, and the
                        // operand copy itself at FP32; 2D bfloat16 reads only the copy
                        if (DIMS == 1 || VEC == 4)
                            *(float4 *)&a.hcache[((int64_t)qc * ns_c + s) * DH + u0] =
                                make_float4(hq[0], hq[1], hq[2], hq[3]);
                        if (VEC == 8) put4<P>((T *)a.hcs + ((int64_t)qc * ns_c + s) * DH + u0, hq);
                    }
                    // [position][16-sample block][feature][16]: the 4 units of a
                    // lane are adjacent 16-sample rows, so the 4 stores of a wave
                    // fill whole 128-byte lines.  The row block starts at a
                    // multiple of 16 (e0, the wave's rows and rb * 16 are), so its
                    // block is uniform across the wave and the lane's sample
                    // within it is l16; nsp is a multiple of 16
                    const int64_t row0 = e0 + wr * C::RW + rb * 16;
                    if (store_act && row0 < a.nsp) {
                        T *hb = (T *)a.hT + ((int64_t)qc * a.nsp + row0) * DH;
                        T *ab = (T *)a.act + ((int64_t)qc * a.nsp + row0) * ((NA + 2) * DH);
                        const uint32_t lo = (uint32_t)(l16 + u0 * 16);
#pragma unroll
                        for (int i = 0; i < 4; i++) {
                            hb[lo + i * 16] = cvt<P>(hq[i]);
#pragma unroll
                            for (int f = 0; f < NA; f++) ab[lo + (f * DH + i) * 16] = cvt<P>(gv[STORE ? f : 0][i]);
                        }
                    }
                }
            }
            if (!glu) head_out(qc % C::NLOG, r, p0, p1, p2, p3);
        };
        // GLU of position qg on its MFMA output of row block rb, and the heads
        auto glu_epi = [&](int qg, int rb, const f32x4_t *acc2) __attribute__((always_inline)) {
            const int r = wr * C::RW + rb * 16 + l16;
            const int s = sRow[r];
            float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
            for (int ub = 0; ub < UB; ub++) {
                float g[4], a1[4], a2[4];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    a1[i] = acc2[ub][i];  // the biases entered as the accumulators' start
                    a2[i] = acc2[UB + ub][i];
                    g[i] = a1[i] * sigmoidf_(a2[i]);
                }
                head_part(ub, g, p0, p1, p2, p3);
                // (the same 16-sample blocked layout as the cell's arrays)
                const int64_t row0 = e0 + wr * C::RW + rb * 16;
                if (store_act && row0 < a.nsp) {
                    const bool ok = s >= 0;
                    T *gb = (T *)a.gT + ((int64_t)qg * a.nsp + row0) * DH;
                    T *ab = (T *)a.act + ((int64_t)qg * a.nsp + row0) * ((NA + 2) * DH);
                    const uint32_t lo = (uint32_t)(l16 + unit0(ub) * 16);
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        gb[lo + i * 16] = cvt<P>(ok ? g[i] : 0.f);
                        ab[lo + (NA * DH + i) * 16] = cvt<P>(ok ? a1[i] : 0.f);
                        ab[lo + ((NA + 1) * DH + i) * 16] = cvt<P>(ok ? a2[i] : 0.f);
                    }
                }
            }
            head_out(qg % C::NLOG, r, p0, p1, p2, p3);
        };
        auto glu_frag = [&](int qg, int rb, int kk) -> uint4 __attribute__((always_inline)) {
            const int arow = wr * C::RW + rb * 16 + l16;
            return *(const uint4 *)&sH[qg & 1][arow * H_LD + kk + VEC * lq];
        };

        // One phase: the GLU and heads of position qg (do_glu) and the cell of
        // position qc (do_cell, input pattern HZ/VT).  With register-resident
        // weights the MFMAs of the next row block are issued ahead of the
        // epilogue of the current one, across the GLU -> cell boundary too.
        // `mid` runs once the first MFMAs of the phase are issued (the one-wave
        // finalisation and indicator work then overlaps the matrix pipe)
        auto run_phase = [&](bool do_glu, int qg, bool do_cell, int qc, const PosInfo &pc, auto HZ, auto VT,
                             auto &&mid) __attribute__((always_inline)) {
            constexpr bool hz = decltype(HZ)::value, vt = decltype(VT)::value;
            const bool vt_prev = vt && pc.pos_vt == qc - 1;
            if (REGW) {
                auto gblock = [&](int rb, f32x4_t *acc2) __attribute__((always_inline)) {
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) {
                        float b1[4], b2[4];
                        cst4(0, ub, b1);
                        cst4(1, ub, b2);
                        acc2[ub] = f32x4_t{b1[0], b1[1], b1[2], b1[3]};
                        acc2[UB + ub] = f32x4_t{b2[0], b2[1], b2[2], b2[3]};
                    }
#pragma unroll
                    for (int kq = 0; kq < NKG; kq++) {
                        const uint4 af = glu_frag(qg, rb, kq * KS);
#pragma unroll
                        for (int g = 0; g < 2; g++)
#pragma unroll
                            for (int ub = 0; ub < UB; ub++)
                                P::mma(acc2[g * UB + ub], wgl[REGW ? g : 0][REGW ? kq : 0][REGW ? ub : 0], af);
                    }
                };
                auto cblock = [&](int rb, f32x4_t *acc) __attribute__((always_inline)) {
                    // scheduling hint: the strategy that interleaves exponentials
                    // with MFMAs (the gate algebra of the previous row block runs
                    // beside this block's MFMAs)
                    __builtin_amdgcn_iglp_opt(3);
                    // start values: bias and one-hot inputs of the row's input class
                    const int cls = sCmb[qc & 1][XT ? wr * C::RW + rb * 16 + l16 : 0];
#pragma unroll
                    for (int g = 0; g < 3; g++)
#pragma unroll
                        for (int ub = 0; ub < UB; ub++) {
                            if (g < C::NXG) {
                                const float4 t = *(const float4 *)&sXt[XT ? g : 0][XT ? cls : 0][XT ? unit0(ub) : 0];
                                acc[g * UB + ub] = f32x4_t{t.x, t.y, t.z, t.w};
                            } else {
                                acc[g * UB + ub] = f32x4_t{0.f, 0.f, 0.f, 0.f};
                            }
                        }
#pragma unroll
                    for (int ks = 0; ks < NKS - 1; ks++) {
                        const int blk = ks / NKB;
                        if (blk == 0 && !hz) continue;
                        if (blk == 1 && !vt) continue;
                        const uint4 af = a_frag(qc, vt_prev, rb, ks);
#pragma unroll
                        for (int g = 0; g < 3; g++)
#pragma unroll
                            for (int ub = 0; ub < UB; ub++)
                                P::mma(acc[g * UB + ub],
                                       __builtin_bit_cast(uint4, wreg[REGW ? g : 0][REGW ? ks : 0][REGW ? ub : 0]), af);
                    }
                };
                f32x4_t accg[2][2 * UB], accc[2][3 * UB];
                if (do_glu) {
                    gblock(0, accg[0]);
                    mid();
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) {
                        if (rb + 1 < RB) gblock(rb + 1, accg[(rb + 1) & 1]);
                        else if (do_cell) cblock(0, accc[0]);
                        glu_epi(qg, rb, accg[rb & 1]);
                    }
                } else if (do_cell) {
                    cblock(0, accc[0]);
                    mid();
                } else {
                    mid();
                }
                if (do_cell) {
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) {
                        if (rb + 1 < RB) cblock(rb + 1, accc[(rb + 1) & 1]);
                        cell_epi(qc, pc, rb, accc[rb & 1]);
                    }
                }
            } else {
                mid();
                if (do_glu) {
                    f32x4_t acc2[RB][2 * UB];
#pragma unroll
                    for (int rb = 0; rb < RB; rb++)
#pragma unroll
                        for (int ub = 0; ub < UB; ub++) {
                            float b1[4], b2[4];
                            cst4(0, ub, b1);
                            cst4(1, ub, b2);
                            acc2[rb][ub] = f32x4_t{b1[0], b1[1], b1[2], b1[3]};
                            acc2[rb][UB + ub] = f32x4_t{b2[0], b2[1], b2[2], b2[3]};
                        }
                    // weight fragments stream from L2, one k-step ahead
                    uint4 gw[2][2 * UB];
                    auto gwload = [&](int kk, uint4 *w) __attribute__((always_inline)) {
#pragma unroll
                        for (int g = 0; g < 2; g++)
#pragma unroll
                            for (int ub = 0; ub < UB; ub++) {
                                const int n = g * DH + wu * C::UW + ub * 16 + l16;
                                w[g * UB + ub] = *(const uint4 *)&Bg[(int64_t)n * KHB + kk + VEC * lq];
                            }
                    };
                    gwload(0, gw[0]);
#pragma unroll
                    for (int j = 0; j < NKG; j++) {
                        if (j + 1 < NKG) gwload((j + 1) * KS, gw[(j + 1) & 1]);
                        uint4 af[RB];
#pragma unroll
                        for (int rb = 0; rb < RB; rb++) af[rb] = glu_frag(qg, rb, j * KS);
#pragma unroll
                        for (int c = 0; c < 2 * UB; c++)
#pragma unroll
                            for (int rb = 0; rb < RB; rb++) P::mma(acc2[rb][c], gw[j & 1][c], af[rb]);
                    }
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) glu_epi(qg, rb, acc2[rb]);
                }
                if (do_cell) {
                    f32x4_t acc[RB][3 * UB];
#pragma unroll
                    for (int rb = 0; rb < RB; rb++)
#pragma unroll
                        for (int c = 0; c < 3 * UB; c++) acc[rb][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
                    // the k-steps with an input (hz block, vt block, indicator),
                    // weight fragments streaming from L2 one k-step ahead
                    constexpr int NH = hz ? NKB : 0, NV = (DIMS == 2 && vt) ? NKB : 0, NACT = NH + NV + 1;
                    auto ks_of = [&](int j) __attribute__((always_inline)) {
                        return j < NH ? j : j < NH + NV ? NKB + (j - NH) : NKS - 1;
                    };
                    uint4 cw[2][3 * UB];
                    auto cwload = [&](int ks, uint4 *w) __attribute__((always_inline)) {
#pragma unroll
                        for (int g = 0; g < 3; g++)
#pragma unroll
                            for (int ub = 0; ub < UB; ub++) {
                                const int n = g * DH + wu * C::UW + ub * 16 + l16;
                                w[g * UB + ub] = *(const uint4 *)&Bc[(int64_t)n * KPX + ks * KS + VEC * lq];
                            }
                    };
                    cwload(ks_of(0), cw[0]);
#pragma unroll
                    for (int j = 0; j < NACT; j++) {
                        if (j + 1 < NACT) cwload(ks_of(j + 1), cw[(j + 1) & 1]);
                        const int ks = ks_of(j);
                        uint4 af[RB];
#pragma unroll
                        for (int rb = 0; rb < RB; rb++) af[rb] = a_frag(qc, vt_prev, rb, ks);
#pragma unroll
                        for (int c = 0; c < 3 * UB; c++)
#pragma unroll
                            for (int rb = 0; rb < RB; rb++) P::mma(acc[rb][c], cw[j & 1][c], af[rb]);
                    }
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) cell_epi(qc, pc, rb, acc[rb]);
                }
            }
        };
        using T1 = std::integral_constant<bool, true>;
        using T0 = std::integral_constant<bool, false>;
        auto phase = [&](bool do_glu, int qg, bool do_cell, int qc, const PosInfo &pc, auto &&mid) __attribute__((always_inline)) {
            const bool hz = pc.site_hz >= 0, vt = DIMS == 2 && pc.site_vt >= 0;
            if (!do_cell || (!hz && !vt)) run_phase(do_glu, qg, do_cell, qc, pc, T0{}, T0{}, mid);
            else if (DIMS == 1 || !vt) run_phase(do_glu, qg, do_cell, qc, pc, T1{}, T0{}, mid);
            else if (hz) run_phase(do_glu, qg, do_cell, qc, pc, T1{}, T1{}, mid);
            else run_phase(do_glu, qg, do_cell, qc, pc, T0{}, T1{}, mid);
        };

        // per-row finalisation of position qf, one row per lane of wave fw:
        // log-softmax, the sampling decision or the given spin, FP64
        // accumulation
        auto finalize = [&](int qf, const PosInfo &pi, int fw) __attribute__((always_inline)) {
            if (w != fw || lane >= MT) return;
            const int r = lane, s = sRow[r], lb = qf % C::NLOG;
            if (s < 0) return;
            float l0 = hc0, l1 = hc1, z0 = hc2, z1 = hc3;
#pragma unroll
            for (int x = 0; x < C::WU; x++) {
                const float4 v = *(const float4 *)&sLog[lb][x][r][0];
                l0 += v.x;
                l1 += v.y;
                z0 += v.z;
                z1 += v.w;
            }
            const float mx = fmaxf(l0, l1);
            const float lse = mx + __logf(1.0f + __expf(-fabsf(l0 - l1)));
            const float ls0 = l0 - lse, ls1 = l1 - lse;
            const float ph0 = cplx ? PI_F * softsignf_(z0) : 0.f;
            const float ph1 = cplx ? PI_F * softsignf_(z1) : 0.f;
            int sg;
            if (!TF) {
                float uni;
                if (a.uniforms) {
                    uni = a.uniforms[(int64_t)s * N + qf];
                } else {
                    uint32_t c4[4] = {(uint32_t)(qf >> 2), (uint32_t)s, (uint32_t)ctr, (uint32_t)(ctr >> 32)};
                    philox4x32_10(c4, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
                    const uint32_t wsel =
                        (qf & 3) == 0 ? c4[0] : (qf & 3) == 1 ? c4[1] : (qf & 3) == 2 ? c4[2] : c4[3];
                    uni = (float)(wsel >> 8) * (1.0f / 16777216.0f);
                }
                sg = (uni < __expf(ls0)) ? 0 : 1;
                sSig[r * N + pi.site] = (uint8_t)sg;
            } else {
                sg = sSig[r * N + pi.site];
            }
            double2 acc = sAcc[r];
            acc.x += (double)(sg ? ls1 : ls0);
            acc.y += (double)(sg ? ph1 : ph0);
            sAcc[r] = acc;
            if (store_lpc) {
                *(float2 *)&a.lpc[((int64_t)s * N + qf) * 2] = make_float2(ls0, ls1);
                *(float2 *)&a.phc[((int64_t)s * N + qf) * 2] = make_float2(ph0, ph1);
                a.pre[(int64_t)s * N + qf] = acc;
            }
            if (store_act) {
                float *lg = a.lgT + (int64_t)qf * 4 * a.nsp + s;
                lg[0] = l0;
                lg[a.nsp] = l1;
                lg[2 * a.nsp] = z0;
                lg[3 * a.nsp] = z1;
            }
        };

        // ------------------------------------------------------ site loop
        if (TF) {
            const int q0 = p + 1;
            const PosInfo P0 = pos(q0);
            if (vt_needed(q0, P0)) vt_store(q0 & 1, vt_issue(P0));
            indicator(P0, q0 & 1, 0);
            if (q0 + 1 < N) {
                const PosInfo P1 = pos(q0 + 1);
                if (vt_needed(q0 + 1, P1)) vt_store((q0 + 1) & 1, vt_issue(P1));
                indicator(P1, (q0 + 1) & 1, NW / 2);
            }
            __syncthreads();
            auto nop = []() __attribute__((always_inline)) {};
            phase(false, q0, true, q0, P0, nop);
            __syncthreads();
            PosInfo Pc = P0, Pp = P0;
            for (int q = q0; q < N; q++) {
                const bool has_next = q + 1 < N, has_2 = q + 2 < N;
                const PosInfo Pn = has_next ? pos(q + 1) : Pc;
                const PosInfo P2 = has_2 ? pos(q + 2) : Pc;
                const bool vt2 = has_2 && vt_needed(q + 2, P2);
                Pfv f2;
                if (vt2) f2 = vt_issue(P2);
                if (Pc.colw) col_copy(q, Pc);
                // indicator of q+2 (its own buffer) and finalisation of q-1
                // (head sums complete since the last barrier), each by one wave
                auto mid = [&]() __attribute__((always_inline)) {
                    if (has_2) indicator(P2, q & 1, (q + 2 + NW / 2) % NW);
                    if (q > q0) finalize(q - 1, Pp, (q - 1) % NW);
                };
                phase(glu, q, has_next, q + 1, Pn, mid);
                if (vt2) vt_store(q & 1, f2);
                __syncthreads();
                Pp = Pc;
                Pc = Pn;
            }
            finalize(N - 1, Pp, (N - 1) % NW);
            __syncthreads();
        } else {
            PosInfo Pc = pos(0);
            indicator(Pc, 0, 0);
            __syncthreads();
            for (int q = 0; q < N; q++) {
                const bool has_next = q + 1 < N;
                const PosInfo Pn = has_next ? pos(q + 1) : Pc;
                const bool vtn = has_next && vt_needed(q + 1, Pn);
                Pfv fn;
                if (vtn) fn = vt_issue(Pn);
                auto nop = []() __attribute__((always_inline)) {};
                phase(false, q, true, q, Pc, nop);
                if (vtn) vt_store((q + 1) & 1, fn);
                __syncthreads();
                if (Pc.colw) col_copy(q, Pc);
                if (glu) phase(true, q, false, q, Pc, nop);
                __syncthreads();
                // the row's lane draws its spin and writes the next indicator
                finalize(q, Pc, q % NW);
                if (has_next) indicator(Pn, (q + 1) & 1, q % NW);
                __syncthreads();
                Pc = Pn;
            }
        }

        // ------------------------------------------------------ tile outputs
        if (tid < MT && sRow[tid] >= 0) {
            const int s = sRow[tid];
            const double2 acc = sAcc[tid];
            if (CHAIN) {
                a.dsuf[(int64_t)s * a.NC + sCid[tid]] = acc;
            } else {
                if (a.logp) a.logp[s] = (float)acc.x;
                if (a.phase) a.phase[s] = (float)acc.y;
            }
        }
        if (!TF) {
            for (int e = tid; e < MT * N; e += NT) {
                const int r = e / N, c = e - r * N;
                const int s = sRow[r];
                if (s >= 0) a.cfg_out[(int64_t)s * N + c] = sSig[e];
            }
        }
    }
}

// ------------------------------------------------------------ launchers

template <class P, int DIMS, int DH, int NW, int REGW, int STORE, int TF, int TC, int CPX = -1, int BATCH = 0>
static hipError_t launch_engine_s(const FwdArgs &a, const BatchInfo &bi, int mode, int sh, int sl, int sa, int grid,
                                  hipStream_t st) {
    typedef Eng<P, DIMS, DH, NW, TC> C;
    // (batched: a.d.N is the longest chain of the batch)
    size_t dyn = ((size_t)C::MT * a.d.N + 15) / 16 * 16;
    hipError_t e = hipFuncSetAttribute((const void *)rnn_engine<P, DIMS, DH, NW, REGW, STORE, TF, TC, CPX, BATCH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((rnn_engine<P, DIMS, DH, NW, REGW, STORE, TF, TC, CPX, BATCH>), dim3(grid), dim3(NW * 64), dyn,
                       st, a, bi, mode, sh, sl, sa);
    return hipGetLastError();
}

// row launches of tile class TC (0 or 2)
template <class P, int DIMS, int DH, int NW, int REGW, int TC>
static hipError_t launch_engine_r(const FwdArgs &a, const BatchInfo &bi, int mode, int sh, int sl, int sa, int grid,
                                  hipStream_t st) {
    const bool store = sh || sl || sa, tf = mode != MODE_SAMPLE;
    if constexpr (DIMS == 1) {
        // batched sampling (the only batched row launch: vmc_step_batched)
        if (bi.n > 0) {
            if (tf || !store) return hipErrorInvalidValue;
            return launch_engine_s<P, DIMS, DH, NW, REGW, 1, 0, TC, -1, 1>(a, bi, mode, sh, sl, sa, grid, st);
        }
    }
    if (store)
        return tf ? launch_engine_s<P, DIMS, DH, NW, REGW, 1, 1, TC>(a, bi, mode, sh, sl, sa, grid, st)
                  : launch_engine_s<P, DIMS, DH, NW, REGW, 1, 0, TC>(a, bi, mode, sh, sl, sa, grid, st);
    return tf ? launch_engine_s<P, DIMS, DH, NW, REGW, 0, 1, TC>(a, bi, mode, sh, sl, sa, grid, st)
              : launch_engine_s<P, DIMS, DH, NW, REGW, 0, 0, TC>(a, bi, mode, sh, sl, sa, grid, st);
}

template <class P, int DIMS, int DH, int NW, int REGW>
static hipError_t launch_engine_t(const FwdArgs &a, const BatchInfo &bi, int mode, int sh, int sl, int sa, int grid,
                                  hipStream_t st) {
    if (mode == MODE_CHAIN) {
        if constexpr (DIMS == 1) {
            if (bi.n > 0)
                return a.d.cplx
                           ? launch_engine_s<P, DIMS, DH, NW, REGW, 0, 1, 1, 1, 1>(a, bi, mode, sh, sl, sa, grid, st)
                           : launch_engine_s<P, DIMS, DH, NW, REGW, 0, 1, 1, 0, 1>(a, bi, mode, sh, sl, sa, grid, st);
        }
        return a.d.cplx ? launch_engine_s<P, DIMS, DH, NW, REGW, 0, 1, 1, 1>(a, bi, mode, sh, sl, sa, grid, st)
                        : launch_engine_s<P, DIMS, DH, NW, REGW, 0, 1, 1, 0>(a, bi, mode, sh, sl, sa, grid, st);
    }
    if constexpr (Eng<P, DIMS, DH, NW, 2>::HAS_ALT) {
        if (a.d.row_alt) return launch_engine_r<P, DIMS, DH, NW, REGW, 2>(a, bi, mode, sh, sl, sa, grid, st);
    }
    return launch_engine_r<P, DIMS, DH, NW, REGW, 0>(a, bi, mode, sh, sl, sa, grid, st);
}

// Variant per precision and width: bfloat16 up to d_h = 128 keeps the
// weights in registers (8 waves at 128, 4 below); the rest stream from L2.
template <class P, int DH>
struct Pick {
    static constexpr int REGW = (P::VEC == 8 && DH <= 128) ? 1 : 0;
    static constexpr int NW = (P::VEC == 8 && DH >= 128) ? 8 : 4;
};

template <class P, int DIMS>
static hipError_t launch_engine_d(const FwdArgs &a, const BatchInfo &bi, int mode, int sh, int sl, int sa, int grid,
                                  hipStream_t st) {
#define VMC_ENG(DHV) \
    launch_engine_t<P, DIMS, DHV, Pick<P, DHV>::NW, Pick<P, DHV>::REGW>(a, bi, mode, sh, sl, sa, grid, st)
    switch (a.d.DH) {
        case 16: return VMC_ENG(16);
        case 32: return VMC_ENG(32);
        case 64: return VMC_ENG(64);
        case 128: return VMC_ENG(128);
        case 256: return VMC_ENG(256);
    }
#undef VMC_ENG
    return hipErrorInvalidValue;
}

// Work-groups of the suffix-chain launch that fit one compute unit (its
// registers, LDS and waves), or 0 if the runtime cannot say.
template <class P, int DIMS>
static int chain_occupancy_d(int DH, int N) {
#define VMC_OCC(DHV)                                                                                         \
    {                                                                                                        \
        typedef Eng<P, DIMS, DHV, Pick<P, DHV>::NW, 1> C;                                                    \
        const size_t dyn = ((size_t)C::MT * N + 15) / 16 * 16;                                              \
        int nb = 0;                                                                                          \
        const void *f = (const void *)rnn_engine<P, DIMS, DHV, Pick<P, DHV>::NW, Pick<P, DHV>::REGW, 0, 1, 1, 0>; \
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) != hipSuccess ||    \
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, Pick<P, DHV>::NW * 64, dyn) != hipSuccess)  \
            return 0;                                                                                        \
        return nb;                                                                                           \
    }
    switch (DH) {
        case 16: VMC_OCC(16)
        case 32: VMC_OCC(32)
        case 64: VMC_OCC(64)
        case 128: VMC_OCC(128)
        case 256: VMC_OCC(256)
    }
#undef VMC_OCC
    return 0;
}

// rows per tile of tile class TC (2: 0 where no alternative exists)
template <class P, int DIMS, int TC>
static int tile_rows_d(int DH) {
#define VMC_TR(DHV) Eng<P, DIMS, DHV, Pick<P, DHV>::NW, TC>::MT
    switch (DH) {
        case 16: return VMC_TR(16);
        case 32: return VMC_TR(32);
        case 64: return VMC_TR(64);
        case 128: return VMC_TR(128);
        case 256: return VMC_TR(256);
    }
#undef VMC_TR
    return 64;
}

template <class P, int DIMS>
static size_t engine_lds_d(int DH, int N) {
#define VMC_LDS1(DHV, TC) (Eng<P, DIMS, DHV, Pick<P, DHV>::NW, TC>::LDS + (size_t)Eng<P, DIMS, DHV, Pick<P, DHV>::NW, TC>::MT * N)
#define VMC_LDS(DHV) std::max(std::max(VMC_LDS1(DHV, 0), VMC_LDS1(DHV, 1)), VMC_LDS1(DHV, 2))
    switch (DH) {
        case 16: return VMC_LDS(16);
        case 32: return VMC_LDS(32);
        case 64: return VMC_LDS(64);
        case 128: return VMC_LDS(128);
        case 256: return VMC_LDS(256);
    }
#undef VMC_LDS
#undef VMC_LDS1
    return (size_t)1 << 30;
}

}  // namespace vmc
