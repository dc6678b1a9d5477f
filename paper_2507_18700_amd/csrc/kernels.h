// Kernel-side declarations shared by the library's translation units.
#pragma once
#include "common.h"

namespace vmc {

// Everything a forward-engine launch needs (passed by value).
struct FwdArgs {
    Dims d;
    // staged weights (store_t arrays are passed as void*)
    const void *Bc, *Bg;
    const float *E, *Hd, *hc;
    // inputs
    int64_t nrows;           // samples (SAMPLE/LOGPSI)
    const uint8_t *cfg_in;   // [ns][N] lattice order (LOGPSI, CHAIN)
    const float *uniforms;   // [ns][N] order-indexed or NULL (SAMPLE)
    uint64_t seed, counter;  // Philox (SAMPLE without uniforms)
    const uint64_t *counter_dev;  // device-resident Philox counter (replaces `counter` when set)
    // outputs
    uint8_t *cfg_out;        // SAMPLE
    float *logp, *phase;     // SAMPLE/LOGPSI, may be NULL
    // caches (NULL = not written / not read)
    float *hcache;           // [N][ns][DH] fp32 hidden states
    void *hcs;               // [N][ns][DH] hidden states as MFMA operands (store_t; FP32: = hcache)
    const int4 *postab;      // [N] facts of each order position (build_postab)
    float *lpc, *phc;        // [ns][N][2] log-conditionals, phase conditionals
    double2 *pre;            // [ns][N] running (log P, phase) after each position, FP64
    void *act;               // [N][nsp/16][NF*DH][16] gate and GLU pre-activations for the backward (store_t)
    float *lgT;              // [N][4][nsp] logits (l0, l1, z0, z1) for the backward
    void *hT, *gT;           // with act: h and GLU output [N][nsp/16][DH][16] (store_t)
    int64_t nsp;             // sample stride of the transposed arrays
    int64_t ns_cache;        // row count of the cache arrays
    // per-workgroup scratch: column buffer of the 2D chain [grid][Lx][MT][DH]
    void *colbuf;
    // CHAIN mode
    int ham_kind;            // connection kind: 0 one flip per position (TFIM, LR-TFIM),
                             // 1 Heisenberg bond, 3 cluster term (see conn_sites)
    int nbond;
    const int *cnt, *tile_start, *list_off, *list;
    int *tile_counter;
    double2 *dsuf;           // [ns][NC] suffix sums of the connected chain (log P, phase)
    int NC;
};

enum { MODE_SAMPLE = 0, MODE_LOGPSI = 1, MODE_CHAIN = 2 };

// Buffers of the gradient (vmc_grad after its forward pass).
struct GradBufs {
    Dims d;
    const void *BcT, *BgT;
    const float *E, *Hd;
    int64_t ns;
    const uint8_t *cfg;
    const float *hcache, *lgT;
    const void *act;  // store_t
    const double *eloc, *weights;
    const float *coef_lp, *coef_ph;  // given per-sample coefficients (vector-Jacobian product), or NULL
    double *stats;
    void *dtc, *dtg, *dth;  // transposed deltas (cell, GLU, heads)
    const void *hT, *gT;    // hidden states and GLU outputs, [N][nsp/16][DH][16]
    void *xT;               // transposed extra inputs (bias, one-hots)
    void *dcol;
    float *part;
    double *grad;
};

// Four consecutive samples of one transposed feature row, as one store.
template <class P>
__device__ inline void store4(typename P::store_t *dst, float a0, float a1, float a2, float a3);
template <>
__device__ inline void store4<F32>(float *dst, float a0, float a1, float a2, float a3) {
    *(float4 *)dst = make_float4(a0, a1, a2, a3);
}
template <>
__device__ inline void store4<BF16>(uint16_t *dst, float a0, float a1, float a2, float a3) {
    *(uint2 *)dst = make_uint2(pack_bf16x2(a0, a1), pack_bf16x2(a2, a3));
}

__host__ __device__ constexpr int cround(int x, int m) { return (x + m - 1) / m * m; }

// number of activation floats per unit stored for the backward: 1D (u, r, m, c), 2D (c, u, v)
__host__ __device__ inline int nact_per_unit(int dims) { return dims == 1 ? 4 : 3; }

// Tile shape of the row-tile kernels (forward engine and backward sweep):
// 4 waves; waves split the hidden units (all three gate columns of a unit in
// one lane) and, for small widths, the rows.
template <class P, int DIMS, int DH>
struct FwdCfg {
    static constexpr int NW = 4;
    static constexpr int WU = (DH / 16 < NW) ? DH / 16 : NW;  // waves along hidden units
    static constexpr int WR = NW / WU;                        // waves along rows
    static constexpr int UW = DH / WU;                        // units per wave
    static constexpr int UB = UW / 16;                        // 16-unit blocks per wave
    static constexpr int MT = (DH >= 256) ? 32 : 64;          // rows per tile
    static constexpr int RW = MT / WR;                        // rows per wave
    static constexpr int RB = RW / 16;
    static constexpr int K = DIMS == 1 ? DH : 2 * DH;
    static constexpr int KP = cround(K, P::KSTEP);
    static constexpr int KGP = cround(DH, P::KSTEP);
    static constexpr int PADE = 16 / (int)sizeof(typename P::store_t);
    static constexpr int SA_LD = KP + PADE;
    static constexpr int SH_LD = KGP + PADE;
    static constexpr int NCP = cround(3 * DH, P::KSTEP);      // padded cell-delta width (backward)
};

// Transposed activation features per unit: the gate values (1D: u, r, m, c;
// 2D: c, u, v) followed by the GLU pre-activations a1, a2.
__host__ __device__ inline int act_feats(int dims) { return nact_per_unit(dims) + 2; }


// bonds of the open chain / square lattice in the order used everywhere:
// for each site a = j*Lx+i in lattice order, the bond to (i+1,j) then (i,j+1)
__host__ __device__ inline int bond_count(int Lx, int Ly) { return (Lx - 1) * Ly + Lx * (Ly - 1); }
__host__ __device__ inline void bond_sites(int b, int Lx, int Ly, int &a, int &c) {
    int per = 2 * Lx - 1;
    int j = b / per;
    if (j < Ly - 1) {
        int r = b - j * per;
        if (r == 2 * Lx - 2) {
            a = j * Lx + Lx - 1;
            c = a + Lx;
        } else {
            int i = r >> 1;
            a = j * Lx + i;
            c = (r & 1) ? a + Lx : a + 1;
        }
    } else {
        int i = b - (Ly - 1) * per;
        a = (Ly - 1) * Lx + i;
        c = a + 1;
    }
}

// Terms of the 1D cluster Hamiltonian (Eq. 9), 0-indexed sites, t < N:
//   t <= N-4: X_t Z_{t+1} X_{t+2}      (flips t, t+2; sign from site t+1)
//   t  = N-3: Z_0 X_1                   (flips 1;      sign from site 0)
//   t  = N-2: X_{N-2} X_{N-1}           (flips N-2, N-1)
//   t  = N-1: X_{N-3} Z_{N-2} Z_{N-1}   (flips N-3;    signs from N-2, N-1)
// f2, z1, z2 = -1 where absent.
__host__ __device__ inline void cluster_term(int t, int N, int &f1, int &f2, int &z1, int &z2) {
    if (t <= N - 4) {
        f1 = t; f2 = t + 2; z1 = t + 1; z2 = -1;
    } else if (t == N - 3) {
        f1 = 1; f2 = -1; z1 = 0; z2 = -1;
    } else if (t == N - 2) {
        f1 = N - 2; f2 = N - 1; z1 = -1; z2 = -1;
    } else {
        f1 = N - 3; f2 = -1; z1 = N - 2; z2 = N - 1;
    }
}

// Connections per sample of a list-scheduled connection kind (1 Heisenberg,
// 3 cluster) and the sites connection c flips (b = -1 for a single flip).
__host__ __device__ inline int conn_count(int kind, int Lx, int Ly) {
    return kind == VMC_CLUSTER ? Lx * Ly : bond_count(Lx, Ly);
}
__host__ __device__ inline void conn_sites(int kind, int c, int Lx, int Ly, int &a, int &b) {
    if (kind == VMC_CLUSTER) {
        int z1, z2;
        cluster_term(c, Lx * Ly, a, b, z1, z2);
    } else {
        bond_sites(c, Lx, Ly, a, b);
    }
}

// ------------------------------------------------------- batched problems
// vmc_step_batched runs several independent chains (same cell shape, own
// lengths, couplings and weights) through the same launches.  Problem k owns
// a workspace region at k * pitch_ws laid out for the longest chain, so every
// workspace pointer of problem k is the one of problem 0 shifted by that
// pitch; its configurations, log-probabilities, parameters and gradient sit
// in the caller's arrays at fixed pitches.  A kernel finds k from its tile
// (the chain launch's global schedule) or from its grid index and rebases
// its arguments.
constexpr int kMaxBatch = 64;
struct BatchInfo {
    int n;                 // problems (0: not batched)
    int tiles;             // row tiles per problem of the sampling / reverse-sweep launches
    int64_t pitch_ws;      // bytes between workspace regions
    int64_t pitch_cfg;     // bytes between configuration arrays (ns * longest chain)
    int64_t pitch_p;       // entries between parameter / gradient vectors
    int64_t ns;            // samples per problem
    const int4 *sched;     // chain tiles of all problems, longest chains first:
                           // {first tile, problem, first changed position, -}
    int nsched;            // entries; sched[nsched].x = total tile count
    int N[kMaxBatch];      // chain lengths
};

template <class T>
__host__ __device__ inline T *shift_bytes(T *p, int64_t bytes) {
    return p ? (T *)((char *)p + bytes) : p;
}

// Arguments of the forward engine for problem k of a batch.
__device__ inline void rebase_fwd(FwdArgs &a, const BatchInfo &b, int k) {
    const int64_t o = (int64_t)k * b.pitch_ws;
    a.Bc = shift_bytes(a.Bc, o);
    a.Bg = shift_bytes(a.Bg, o);
    a.E = shift_bytes(a.E, o);
    a.Hd = shift_bytes(a.Hd, o);
    a.hc = shift_bytes(a.hc, o);
    a.hcache = shift_bytes(a.hcache, o);
    a.hcs = shift_bytes(a.hcs, o);
    a.postab = shift_bytes(a.postab, o);
    a.lpc = shift_bytes(a.lpc, o);
    a.phc = shift_bytes(a.phc, o);
    a.pre = shift_bytes(a.pre, o);
    a.act = shift_bytes(a.act, o);
    a.lgT = shift_bytes(a.lgT, o);
    a.hT = shift_bytes(a.hT, o);
    a.gT = shift_bytes(a.gT, o);
    a.colbuf = shift_bytes(a.colbuf, o);
    a.cnt = shift_bytes(a.cnt, o);
    a.tile_start = shift_bytes(a.tile_start, o);
    a.list_off = shift_bytes(a.list_off, o);
    a.list = shift_bytes(a.list, o);
    a.dsuf = shift_bytes(a.dsuf, o);
    a.cfg_in = shift_bytes(a.cfg_in, (int64_t)k * b.pitch_cfg);
    a.cfg_out = shift_bytes(a.cfg_out, (int64_t)k * b.pitch_cfg);
    a.logp = shift_bytes(a.logp, (int64_t)k * b.ns * 4);
    a.phase = shift_bytes(a.phase, (int64_t)k * b.ns * 4);
    a.d.N = a.d.Lx = b.N[k];
    a.seed += (uint64_t)k;
    a.NC = a.ham_kind == 0 ? a.d.N : conn_count(a.ham_kind, a.d.N, 1);
    a.nbond = a.ham_kind == 0 ? 0 : a.NC;
}

}  // namespace vmc
