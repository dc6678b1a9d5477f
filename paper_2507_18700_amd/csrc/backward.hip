// Reverse sweep of the energy gradient (backpropagation through the
// autoregressive chain, Eq. 1 with the App. A cells) for a tile of samples.
//
// With E held constant the gradient is that of
//   L = sum_s [a_s log P(sigma_s) + b_s phi(sigma_s)],
//   a_s = w_s Re(E_s - Ebar), b_s = 2 w_s Im(E_s - Ebar),
// or, for the vector-Jacobian product of log psi, with a_s, b_s given.
// At each order position, last to first:
//   (a) head deltas: a_s (onehot(sigma) - softmax(l)) (Eq. 3) and
//       b_s pi softsign'(z_sigma) (Eq. 5);
//   (b) the gradient on the GLU output g, then the GLU deltas (App. A);
//   (c) their input gradient [d1 | d2] . [W_1 ; W_2] on MFMA;
//   (d) the gate deltas of the cell (App. A reversed);
//   (e) their input gradient delta . B_c on MFMA, routed to the one or two
//       predecessor positions: carried in registers (the previous position),
//       or parked per column for the vertical predecessor (2D).
// All deltas are written transposed [position][feature][sample] for the
// weight-gradient contraction.  Tiles, waves and weight residency follow the
// forward engine: bfloat16 up to d_h = 128 keeps the transposed weights in
// registers (8 waves at 128).
#include <type_traits>

#include "kernels.h"

namespace vmc {

struct BwdArgs {
    Dims d;
    const void *BcT, *BgT;  // [NHB*DH][NCP], [KHB][2*DH]
    const float *Hd;
    int64_t ns, nsp;
    const uint8_t *cfg;
    const void *act;        // [N][nsp/16][NF*DH][16] gate values and GLU pre-activations (store_t)
    const float *lgT;       // [N][4][nsp] logits
    const float *hcache;    // [N][ns][DH] FP32 hidden states (1D: h_{n-1} of the update-gate term)
    const double *eloc, *w, *stats;
    const float *coef_lp, *coef_ph;  // given coefficients a_s, b_s (then eloc, w, stats are unused)
    void *dtc, *dtg, *dth;  // transposed deltas: cell [N][NDC][nsp], GLU [N][2DH][nsp], heads [N][4][nsp]
    float *dcol;            // [grid][Lx][DH][MT]
};

// Arguments of the reverse sweep for problem k of a batch (see BatchInfo):
// workspace arrays of region k, the caller's configurations, local energies
// and statistics of problem k.
__device__ inline void rebase_bwd(BwdArgs &a, const BatchInfo &b, int k) {
    const int64_t o = (int64_t)k * b.pitch_ws;
    a.BcT = shift_bytes(a.BcT, o);
    a.BgT = shift_bytes(a.BgT, o);
    a.Hd = shift_bytes(a.Hd, o);
    a.act = shift_bytes(a.act, o);
    a.lgT = shift_bytes(a.lgT, o);
    a.hcache = shift_bytes(a.hcache, o);
    a.dtc = shift_bytes(a.dtc, o);
    a.dtg = shift_bytes(a.dtg, o);
    a.dth = shift_bytes(a.dth, o);
    a.dcol = shift_bytes(a.dcol, o);
    a.cfg = shift_bytes(a.cfg, (int64_t)k * b.pitch_cfg);
    a.eloc = shift_bytes(a.eloc, (int64_t)k * b.ns * 16);
    a.stats = shift_bytes(a.stats, (int64_t)k * 32);
    a.d.N = a.d.Lx = b.N[k];
}

// Rows per tile and waves per workgroup.  From d_h = 128 on, 8 waves (one or
// two 16-unit blocks per wave) hold the transposed weights; one such
// workgroup fills a compute unit, so the tile is sized to spread the usual
// sample counts over the chip in one round (48 rows at d_h = 128).
constexpr int kXcdsB = 8;  // XCDs of the chip (work-groups are dealt to them round-robin by id)

#define BWD_MT(DH) ((DH) == 128 ? 48 : (DH) >= 256 ? 32 : 64)
#define BWD_NW(DH) ((DH) >= 128 ? 8 : 4)

template <class P, int DIMS, int DH, int NW>
struct BwdCfg {
    static constexpr int WU = (DH / 16 < NW) ? DH / 16 : NW;
    static constexpr int WR = NW / WU;
    static constexpr int UW = DH / WU;
    static constexpr int UB = UW / 16;
    static constexpr int MT = BWD_MT(DH);
    static constexpr int RW = MT / WR;
    static constexpr int RB = RW / 16;
    static constexpr int KS = P::KSTEP;
    static constexpr int NCP = cround(3 * DH, KS);   // contraction of the cell dX
    static constexpr int NGK = 2 * DH / KS;         // k-steps of the GLU dX
    static constexpr int NCK = NCP / KS;            // k-steps of the cell dX
    static constexpr int NOB = DIMS == 1 ? UB : 2 * UB;  // output blocks of the cell dX (hz, vt)
    static constexpr int PADE = 16 / (int)sizeof(typename P::store_t);
    static constexpr int D_LD = NCP + PADE;         // shared row stride of the GLU and cell delta tiles
};

template <class P, int DIMS, int DH, int NW, int REGW, int BATCH = 0>
__global__ __launch_bounds__(NW * 64) void rnn_bwd(BwdArgs a0, BatchInfo bi) {
    typedef BwdCfg<P, DIMS, DH, NW> C;
    typedef typename P::store_t T;
    constexpr int MT = C::MT, RB = C::RB, UB = C::UB, VEC = P::VEC, KS = C::KS;
    constexpr int NCP = C::NCP, NGK = C::NGK, NCK = C::NCK, NOB = C::NOB, D_LD = C::D_LD, NT = NW * 64;
    constexpr int NA = DIMS == 1 ? 4 : 3;
    constexpr int NF = NA + 2;
    constexpr int NDC = DIMS == 1 ? 4 * DH : 3 * DH;

    __shared__ __align__(16) T sD[MT * D_LD];  // GLU deltas, then cell deltas
    __shared__ __align__(16) float sDL[MT][4];
    __shared__ float sCoef[MT][2];
    __shared__ int sRow[MT];
    // dynamic LDS: (REGW) the GLU weights BgT [DH][G_LD], then the tile's
    // configurations [MT][N]
    extern __shared__ __align__(16) uint8_t sDyn[];
    constexpr int G_LD = 2 * DH + C::PADE;
    T *const sBg = (T *)sDyn;
    uint8_t *const sSig = sDyn + (REGW ? (size_t)DH * G_LD * sizeof(T) : 0);

    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = w / C::WU, wu = w % C::WU;
    const int l16 = lane & 15, lq = lane >> 4;
    // batched: one problem per group of bi.tiles work-groups
    BwdArgs a = a0;
    // Work-groups go to the XCDs round-robin by id; neighbouring tiles share
    // the 128-byte lines of the transposed arrays (a tile is not a multiple
    // of 64 samples), so each XCD takes a contiguous run of tiles and a
    // shared line stays in one L2.
    int tile;
    {
        // XCD y takes G/8 tiles, plus one if y < G % 8
        const int G = gridDim.x, b = blockIdx.x, x = b % kXcdsB;
        const int q = G / kXcdsB, r = G - q * kXcdsB;
        tile = __builtin_amdgcn_readfirstlane(x * q + min(x, r) + b / kXcdsB);
    }
    if (BATCH) {
        const int k = tile / bi.tiles;
        tile -= k * bi.tiles;
        rebase_bwd(a, bi, k);
    }
    const int N = a.d.N, Lx = a.d.Lx, Ly = a.d.Ly;
    const int cplx = a.d.cplx, glu = a.d.glu;
    const int64_t ns = a.ns, nsp = a.nsp;
    const T *__restrict__ BcT = (const T *)a.BcT;
    const T *__restrict__ BgT = (const T *)a.BgT;
    float *dcol = a.dcol + (int64_t)tile * Lx * MT * DH;

    // head weights of this lane's units
    float hw[4][UB];
#pragma unroll
    for (int ub = 0; ub < UB; ub++)
#pragma unroll
        for (int o = 0; o < 4; o++) hw[o][ub] = a.Hd[o * DH + wu * C::UW + ub * 16 + l16];

    // REGW: transposed cell weights in registers, GLU weights in LDS
    uint4 wc[REGW ? NCK : 1][REGW ? NOB : 1];
    if (REGW) {
        for (int e = tid; e < DH * (2 * DH / VEC); e += NT) {
            const int k = e / (2 * DH / VEC), j = (e - k * (2 * DH / VEC)) * VEC;
            *(uint4 *)&sBg[k * G_LD + j] = *(const uint4 *)&BgT[(int64_t)k * 2 * DH + j];
        }
#pragma unroll
        for (int ks = 0; ks < NCK; ks++)
#pragma unroll
            for (int c = 0; c < NOB; c++) {
                const int k = (c / UB) * DH + wu * C::UW + (c % UB) * 16 + l16;
                wc[ks][c % NOB] = *(const uint4 *)&BcT[(int64_t)k * NCP + ks * KS + VEC * lq];
            }
    }

    const int64_t e0 = (int64_t)tile * MT;
    const int nrow = (int)min((int64_t)MT, ns - e0);
    if (tid < MT) {
        const int s = tid < nrow ? (int)(e0 + tid) : -1;
        sRow[tid] = s;
        float ca = 0.f, cb = 0.f;
        if (s >= 0) {
            if (a.coef_lp) {
                ca = a.coef_lp[s];
                cb = a.coef_ph ? a.coef_ph[s] : 0.f;
            } else {
                const double ws = a.w ? a.w[s] : 1.0 / (double)ns;
                ca = (float)(ws * (a.eloc[2 * s] - a.stats[0]));
                cb = (float)(2.0 * ws * (a.eloc[2 * s + 1] - a.stats[1]));
            }
        }
        sCoef[tid][0] = ca;
        sCoef[tid][1] = cb;
    }
    for (int e = tid; e < MT * D_LD; e += NT) sD[e] = P::from_float(0.f);
    __syncthreads();
    for (int e = tid; e < MT * N; e += NT) {
        const int r = e / N, c = e - r * N;
        const int s = sRow[r];
        sSig[e] = s >= 0 ? a.cfg[(int64_t)s * N + c] : (uint8_t)0;
    }

    float carry[RB][UB][4];
#pragma unroll
    for (int rb = 0; rb < RB; rb++)
#pragma unroll
        for (int ub = 0; ub < UB; ub++)
#pragma unroll
            for (int ii = 0; ii < 4; ii++) carry[rb][ub][ii] = 0.f;
    __syncthreads();

    // first sample of this lane's 4-row group in row block rb (transposed arrays)
    auto srow0 = [&](int rb) -> int64_t { return e0 + wr * C::RW + rb * 16 + 4 * lq; };
    // 4 samples of one activation feature as stored (FP32: float4; bfloat16:
    // 4 halves in a uint2, widened at use), so that every feature of a position
    // can be in flight from the start of the position at half the registers
    typedef typename std::conditional<VEC == 4, float4, uint2>::type RawF;
    auto feat = [&](int q, int f, int u, int rb) -> RawF {
        const int64_t s0 = srow0(rb);
        if (s0 >= nsp) {
            if constexpr (VEC == 4) return make_float4(0.f, 0.f, 0.f, 0.f);
            else return make_uint2(0u, 0u);
        }
        // [position][16-sample block][feature][16] (the forward's layout)
        return *(const RawF *)((const T *)a.act + (int64_t)q * NF * DH * nsp + (s0 >> 4) * (NF * DH * 16) +
                               (f * DH + u) * 16 + (s0 & 15));
    };
    auto widen = [](RawF v) -> float4 {
        if constexpr (VEC == 4) {
            return v;
        } else {
            return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xFFFF0000u),
                               __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xFFFF0000u));
        }
    };
    // logits of the next position (rows of lanes tid < MT), loaded one position ahead
    float lgn[4] = {0.f, 0.f, 0.f, 0.f};
    auto load_lg = [&](int q) {
        const int s = tid < MT ? sRow[tid] : -1;
        if (s >= 0) {
            const float *lg = a.lgT + (int64_t)q * 4 * nsp + s;
            lgn[0] = lg[0];
            lgn[1] = lg[nsp];
            if (cplx) {
                lgn[2] = lg[2 * nsp];
                lgn[3] = lg[3 * nsp];
            }
        }
    };
    load_lg(N - 1);

    for (int q = N - 1; q >= 0; q--) {
        const float lgc[4] = {lgn[0], lgn[1], lgn[2], lgn[3]};
        if (q > 0) load_lg(q - 1);
        const int site = order_site(q, Lx);
        const int jrow = q / Lx, icol = site - jrow * Lx;
        const bool row_start = (q % Lx) == 0;
        const bool last_in_row = ((q + 1) % Lx) == 0;
        const bool has_vt = DIMS == 2 && jrow > 0;
        const bool vt_succ_parked = DIMS == 2 && jrow + 1 < Ly && !last_in_row;

        // GLU pre-activations and gate values of this step, in flight during
        // the head and GLU phases
        RawF fa1[RB][UB], fa2[RB][UB];
        if (glu) {
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ub = 0; ub < UB; ub++) {
                    const int u = wu * C::UW + ub * 16 + l16;
                    fa1[rb][ub] = feat(q, NA, u, rb);
                    fa2[rb][ub] = feat(q, NA + 1, u, rb);
                }
        }


        // (a) head deltas
        if (tid < MT) {
            const int s = sRow[tid];
            float d0 = 0.f, d1 = 0.f, z0 = 0.f, z1 = 0.f;
            if (s >= 0) {
                const float l0 = lgc[0], l1 = lgc[1];
                const int sg = sSig[tid * N + site];
                const float p1 = rcpf_(1.0f + __expf(l0 - l1));  // softmax(l)[1]
                const float p0 = 1.0f - p1;
                const float ca = sCoef[tid][0];
                d0 = ca * ((sg == 0 ? 1.f : 0.f) - p0);
                d1 = ca * ((sg == 1 ? 1.f : 0.f) - p1);
                if (cplx) {
                    const float z = sg ? lgc[3] : lgc[2];
                    const float den = 1.0f + fabsf(z);
                    const float dz = sCoef[tid][1] * PI_F / (den * den);
                    if (sg) z1 = dz;
                    else z0 = dz;
                }
            }
            const int64_t sg_ = e0 + tid;
            if (sg_ < nsp) {
                T *dh = (T *)a.dth + (int64_t)q * 4 * nsp + sg_;
                dh[0] = P::from_float(d0);
                dh[nsp] = P::from_float(d1);
                dh[2 * nsp] = P::from_float(z0);
                dh[3 * nsp] = P::from_float(z1);
            }
            *(float4 *)&sDL[tid][0] = make_float4(d0, d1, z0, z1);
        }
        __syncthreads();

        // (b) gradient on g; GLU deltas into LDS and the transposed store
        float dgv[RB][UB][4];
#pragma unroll
        for (int rb = 0; rb < RB; rb++) {
#pragma unroll
            for (int ii = 0; ii < 4; ii++) {
                const int r = wr * C::RW + rb * 16 + 4 * lq + ii;
                const float4 dl = *(const float4 *)&sDL[r][0];
#pragma unroll
                for (int ub = 0; ub < UB; ub++)
                    dgv[rb][ub][ii] = hw[0][ub] * dl.x + hw[1][ub] * dl.y + hw[2][ub] * dl.z + hw[3][ub] * dl.w;
            }
        }
        // (the GLU test outside the row-block loop: inside it, the path that skips
        // the GLU part would leave the pre-activation loads pending, and every row
        // block would then wait for all earlier stores before reading them)
        if (glu) {
#pragma unroll
            for (int rb = 0; rb < RB; rb++) {
                const int64_t s0 = srow0(rb);
#pragma unroll
                for (int ub = 0; ub < UB; ub++) {
                    const int u = wu * C::UW + ub * 16 + l16;
                    float d1[4], d2[4];
                    const float4 w1 = widen(fa1[rb][ub]), w2 = widen(fa2[rb][ub]);
                    const float a1v[4] = {w1.x, w1.y, w1.z, w1.w};
                    const float a2v[4] = {w2.x, w2.y, w2.z, w2.w};
#pragma unroll
                    for (int ii = 0; ii < 4; ii++) {
                        const float sg2 = sigmoidf_(a2v[ii]);
                        d1[ii] = dgv[rb][ub][ii] * sg2;
                        d2[ii] = dgv[rb][ub][ii] * a1v[ii] * sg2 * (1.0f - sg2);
                        const int r = wr * C::RW + rb * 16 + 4 * lq + ii;
                        sD[r * D_LD + u] = P::from_float(d1[ii]);
                        sD[r * D_LD + DH + u] = P::from_float(d2[ii]);
                    }
                    if (s0 < nsp) {
                        T *dst = (T *)a.dtg + ((int64_t)q * 2 * DH + u) * nsp + s0;
                        store4<P>(dst, d1[0], d1[1], d1[2], d1[3]);
                        store4<P>(dst + (int64_t)DH * nsp, d2[0], d2[1], d2[2], d2[3]);
                    }
                }
            }
        }
        __syncthreads();

        // register-resident weights leave room to load the gate values before the
        // GLU input-gradient MFMAs (their latency then overlaps that phase)
        RawF fcr[NA][RB][UB];  // (streamed weights: loaded after the GLU input gradient)
        if (REGW) {
#pragma unroll
            for (int f = 0; f < NA; f++)
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) fcr[f][rb][ub] = feat(q, f, wu * C::UW + ub * 16 + l16, rb);
        }
        // (c) GLU input gradient: dh_glu = [d1 | d2] . [W_1 ; W_2] (MFMA)
        f32x4_t accg[RB][UB];
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ub = 0; ub < UB; ub++) accg[rb][ub] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        if (glu) {
            if constexpr (REGW) {
#pragma unroll
                for (int ks = 0; ks < NGK; ks++) {
                    uint4 af[RB];
#pragma unroll
                    for (int rb = 0; rb < RB; rb++)
                        af[rb] = *(const uint4 *)&sD[(wr * C::RW + rb * 16 + l16) * D_LD + ks * KS + VEC * lq];
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) {
                        const int k = wu * C::UW + ub * 16 + l16;
                        const uint4 bf = *(const uint4 *)&sBg[k * G_LD + ks * KS + VEC * lq];
#pragma unroll
                        for (int rb = 0; rb < RB; rb++) P::mma(accg[rb][ub], af[rb], bf);
                    }
                }
            } else {
                // streamed weights: the next k-step's fragments in flight (a
                // bounded prefetch; a full unroll hoists every load and spills)
                uint4 bw0[UB], bw1[UB];
                auto wload = [&](int ks, uint4 *bw) __attribute__((always_inline)) {
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) {
                        const int k = wu * C::UW + ub * 16 + l16;
                        bw[ub] = *(const uint4 *)&BgT[(int64_t)k * 2 * DH + ks * KS + VEC * lq];
                    }
                };
                auto kstep = [&](int ks, const uint4 *bw) __attribute__((always_inline)) {
                    uint4 af[RB];
#pragma unroll
                    for (int rb = 0; rb < RB; rb++)
                        af[rb] = *(const uint4 *)&sD[(wr * C::RW + rb * 16 + l16) * D_LD + ks * KS + VEC * lq];
#pragma unroll
                    for (int ub = 0; ub < UB; ub++)
#pragma unroll
                        for (int rb = 0; rb < RB; rb++) P::mma(accg[rb][ub], af[rb], bw[ub]);
                };
                wload(0, bw0);
#pragma unroll 1
                for (int ks = 0; ks < NGK; ks += 2) {
                    if (ks + 1 < NGK) wload(ks + 1, bw1);
                    kstep(ks, bw0);
                    if (ks + 1 < NGK) {
                        if (ks + 2 < NGK) wload(ks + 2, bw0);
                        kstep(ks + 1, bw1);
                    }
                }
            }
            __syncthreads();  // GLU deltas read before the cell deltas overwrite the tile
        }

        // gate values of this step, as stored (widened at use: half the registers)
        if (!REGW) {
#pragma unroll
            for (int f = 0; f < NA; f++)
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) fcr[f][rb][ub] = feat(q, f, wu * C::UW + ub * 16 + l16, rb);
        }
        float4 fhp[DIMS == 1 ? RB : 1][DIMS == 1 ? UB : 1];  // 1D: h_{n-1} (FP32)
        if (DIMS == 1) {
            // every load first (rows past ns read row ns - 1), then the rows past
            // ns zeroed: the loads are in flight together, with no per-lane branch
            float hv[DIMS == 1 ? RB : 1][DIMS == 1 ? UB : 1][4];
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ub = 0; ub < UB; ub++) {
                    const int64_t s0 = srow0(rb);
                    const float *hp = a.hcache + (int64_t)(q > 0 ? q - 1 : 0) * ns * DH + wu * C::UW + ub * 16 + l16;
#pragma unroll
                    for (int ii = 0; ii < 4; ii++)
                        hv[rb % (DIMS == 1 ? RB : 1)][ub % (DIMS == 1 ? UB : 1)][ii] =
                            hp[(s0 + ii < ns ? s0 + ii : ns - 1) * DH];
                }
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ub = 0; ub < UB; ub++) {
                    const int64_t s0 = srow0(rb);
                    float v[4];
#pragma unroll
                    for (int ii = 0; ii < 4; ii++)
                        v[ii] = (q > 0 && s0 + ii < ns) ? hv[rb % (DIMS == 1 ? RB : 1)][ub % (DIMS == 1 ? UB : 1)][ii] : 0.f;
                    fhp[rb % (DIMS == 1 ? RB : 1)][ub % (DIMS == 1 ? UB : 1)] = make_float4(v[0], v[1], v[2], v[3]);
                }
        }

        // (d) total dh and the gate deltas; the dh parked by the vertical
        // successor (2D) is read as one float4 per row block, every load issued
        // before the first use (positions without a parked value discard it)
        float4 dpk[DIMS == 2 ? RB : 1][DIMS == 2 ? UB : 1];
        if (DIMS == 2) {
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ub = 0; ub < UB; ub++) {
                    const int u = wu * C::UW + ub * 16 + l16, r0 = wr * C::RW + rb * 16 + 4 * lq;
                    dpk[rb % (DIMS == 2 ? RB : 1)][ub % (DIMS == 2 ? UB : 1)] =
                        *(const float4 *)&dcol[((int64_t)icol * DH + u) * MT + r0];
                }
        }
        float direct[RB][UB][4];
#pragma unroll
        for (int rb = 0; rb < RB; rb++) {
            const int64_t s0 = srow0(rb);
#pragma unroll
            for (int ub = 0; ub < UB; ub++) {
                const int u = wu * C::UW + ub * 16 + l16;
                float gd[4][4];
                const float4 f0 = widen(fcr[0][rb][ub]), f1 = widen(fcr[1][rb][ub]), f2 = widen(fcr[2][rb][ub]);
                const float v0[4] = {f0.x, f0.y, f0.z, f0.w}, v1[4] = {f1.x, f1.y, f1.z, f1.w};
                const float v2[4] = {f2.x, f2.y, f2.z, f2.w};
                float v3[4] = {0.f, 0.f, 0.f, 0.f}, hp[4] = {0.f, 0.f, 0.f, 0.f};
                if (DIMS == 1) {
                    const float4 f3 = widen(fcr[NA - 1][rb][ub]);
                    v3[0] = f3.x; v3[1] = f3.y; v3[2] = f3.z; v3[3] = f3.w;
                    const float4 h4 = fhp[rb % (DIMS == 1 ? RB : 1)][ub % (DIMS == 1 ? UB : 1)];
                    hp[0] = h4.x; hp[1] = h4.y; hp[2] = h4.z; hp[3] = h4.w;
                }
#pragma unroll
                for (int ii = 0; ii < 4; ii++) {
                    const int r = wr * C::RW + rb * 16 + 4 * lq + ii;
                    float dh = (glu ? accg[rb][ub][ii] : dgv[rb][ub][ii]) + carry[rb][ub][ii];
                    if (DIMS == 2) {
                        const float4 pk = dpk[rb % (DIMS == 2 ? RB : 1)][ub % (DIMS == 2 ? UB : 1)];
                        const float pv = ii == 0 ? pk.x : ii == 1 ? pk.y : ii == 2 ? pk.z : pk.w;
                        dh += vt_succ_parked ? pv : 0.f;
                    }
                    float g0, g1, g2, g3 = 0.f;
                    if (DIMS == 1) {
                        // h' = (1-u) h + u c, c = tanh(r m + x-term)
                        const float uu = v0[ii], rr = v1[ii], m = v2[ii], c = v3[ii];
                        const float du = dh * (c - hp[ii]), dc = dh * uu;
                        const float dac = dc * (1.0f - c * c);
                        g0 = du * uu * (1.0f - uu);
                        g1 = dac * m * rr * (1.0f - rr);
                        g2 = dac * rr;
                        g3 = dac;
                        direct[rb][ub][ii] = dh * (1.0f - uu);
                    } else {
                        // h = u c + (1-u) v
                        const float c = v0[ii], uu = v1[ii], v = v2[ii];
                        const float du = dh * (c - v), dc = dh * uu;
                        g0 = dc * (1.0f - c * c);
                        g1 = du * uu * (1.0f - uu);
                        g2 = dh * (1.0f - uu);
                        direct[rb][ub][ii] = 0.f;
                    }
                    gd[0][ii] = g0;
                    gd[1][ii] = g1;
                    gd[2][ii] = g2;
                    gd[3][ii] = g3;
                    sD[r * D_LD + u] = P::from_float(g0);
                    sD[r * D_LD + DH + u] = P::from_float(g1);
                    sD[r * D_LD + 2 * DH + u] = P::from_float(g2);
                }
                if (s0 < nsp) {
#pragma unroll
                    for (int g = 0; g < (DIMS == 1 ? 4 : 3); g++)
                        store4<P>((T *)a.dtc + ((int64_t)q * NDC + g * DH + u) * nsp + s0, gd[g][0], gd[g][1],
                                  gd[g][2], gd[g][3]);
                }
            }
        }
        __syncthreads();

        // (e) cell input gradient: dA = delta . B_c (MFMA); route to predecessors
        f32x4_t accx[RB][NOB];
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int c = 0; c < NOB; c++) accx[rb][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        if constexpr (REGW) {
#pragma unroll
            for (int ks = 0; ks < NCK; ks++) {
                uint4 af[RB];
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
                    af[rb] = *(const uint4 *)&sD[(wr * C::RW + rb * 16 + l16) * D_LD + ks * KS + VEC * lq];
#pragma unroll
                for (int c = 0; c < NOB; c++)
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) P::mma(accx[rb][c], af[rb], wc[REGW ? ks : 0][REGW ? c : 0]);
            }
        } else {
            // streamed weights: the next k-step's fragments in flight
            uint4 bw0[NOB], bw1[NOB];
            auto wload = [&](int ks, uint4 *bw) __attribute__((always_inline)) {
#pragma unroll
                for (int c = 0; c < NOB; c++) {
                    const int k = (c / UB) * DH + wu * C::UW + (c % UB) * 16 + l16;
                    bw[c] = *(const uint4 *)&BcT[(int64_t)k * NCP + ks * KS + VEC * lq];
                }
            };
            auto kstep = [&](int ks, const uint4 *bw) __attribute__((always_inline)) {
                uint4 af[RB];
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
                    af[rb] = *(const uint4 *)&sD[(wr * C::RW + rb * 16 + l16) * D_LD + ks * KS + VEC * lq];
#pragma unroll
                for (int c = 0; c < NOB; c++)
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) P::mma(accx[rb][c], af[rb], bw[c]);
            };
            wload(0, bw0);
#pragma unroll 1
            for (int ks = 0; ks < NCK; ks += 2) {
                if (ks + 1 < NCK) wload(ks + 1, bw1);
                kstep(ks, bw0);
                if (ks + 1 < NCK) {
                    if (ks + 2 < NCK) wload(ks + 2, bw0);
                    kstep(ks + 1, bw1);
                }
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ub = 0; ub < UB; ub++) {
                const int u = wu * C::UW + ub * 16 + l16, r0 = wr * C::RW + rb * 16 + 4 * lq;
                if (DIMS == 1) {
#pragma unroll
                    for (int ii = 0; ii < 4; ii++) carry[rb][ub][ii] = accx[rb][ub][ii] + direct[rb][ub][ii];
                } else {
#pragma unroll
                    for (int ii = 0; ii < 4; ii++)
                        carry[rb][ub][ii] = row_start ? (has_vt ? accx[rb][UB + ub][ii] : 0.f) : accx[rb][ub][ii];
                    if (!row_start && has_vt)
                        *(float4 *)&dcol[((int64_t)icol * DH + u) * MT + r0] =
                            make_float4(accx[rb][UB + ub][0], accx[rb][UB + ub][1], accx[rb][UB + ub][2],
                                        accx[rb][UB + ub][3]);
                }
            }
        __syncthreads();
    }
}

template <class P, int DH>
struct BwdPick {
    static constexpr int REGW = (P::VEC == 8 && DH <= 128) ? 1 : 0;
    static constexpr int NW = BWD_NW(DH);
};

template <class P, int DIMS, int DH, int BATCH>
static hipError_t launch_bwd_b(const BwdArgs &a, BatchInfo bi, hipStream_t st) {
    constexpr int NW = BwdPick<P, DH>::NW, REGW = BwdPick<P, DH>::REGW;
    typedef BwdCfg<P, DIMS, DH, NW> C;
    // every column below nsp gets written (zeros past ns); batched: that many
    // tiles per problem (a.d.N is then the longest chain)
    const int tiles = (int)((a.nsp + C::MT - 1) / C::MT);
    bi.tiles = tiles;
    const int grid = BATCH ? bi.n * tiles : tiles;
    size_t dyn = ((size_t)C::MT * a.d.N + 15) / 16 * 16;
    if (REGW) dyn += (size_t)DH * (2 * DH + C::PADE) * sizeof(typename P::store_t);
    hipError_t e = hipFuncSetAttribute((const void *)rnn_bwd<P, DIMS, DH, NW, REGW, BATCH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((rnn_bwd<P, DIMS, DH, NW, REGW, BATCH>), dim3(grid), dim3(NW * 64), dyn, st, a, bi);
    return hipGetLastError();
}

template <class P, int DIMS, int DH>
static hipError_t launch_bwd_t(const BwdArgs &a, const BatchInfo &bi, hipStream_t st) {
    if constexpr (DIMS == 1) {
        if (bi.n > 0) return launch_bwd_b<P, DIMS, DH, 1>(a, bi, st);
    }
    if (bi.n > 0) return hipErrorInvalidValue;
    return launch_bwd_b<P, DIMS, DH, 0>(a, bi, st);
}

template <class P, int DIMS>
static hipError_t launch_bwd_d(const BwdArgs &a, const BatchInfo &bi, hipStream_t st) {
    switch (a.d.DH) {
        case 16: return launch_bwd_t<P, DIMS, 16>(a, bi, st);
        case 32: return launch_bwd_t<P, DIMS, 32>(a, bi, st);
        case 64: return launch_bwd_t<P, DIMS, 64>(a, bi, st);
        case 128: return launch_bwd_t<P, DIMS, 128>(a, bi, st);
        case 256: return launch_bwd_t<P, DIMS, 256>(a, bi, st);
    }
    return hipErrorInvalidValue;
}

int backward_tile_rows(int DH) { return BWD_MT(DH); }

// LDS of one reverse-sweep work-group (static tiles, GLU weights, the tile's
// configurations), for the host-side capacity check
template <class P, int DIMS, int DH>
static size_t bwd_lds_t(int N) {
    constexpr int NW = BwdPick<P, DH>::NW, REGW = BwdPick<P, DH>::REGW;
    typedef BwdCfg<P, DIMS, DH, NW> C;
    const size_t es = sizeof(typename P::store_t);
    size_t n = (size_t)C::MT * C::D_LD * es + (size_t)C::MT * (16 + 8 + 4);
    n += ((size_t)C::MT * N + 15) / 16 * 16;
    if (REGW) n += (size_t)DH * (2 * DH + C::PADE) * es;
    return n;
}
template <class P, int DIMS>
static size_t bwd_lds_d(int DH, int N) {
    switch (DH) {
        case 16: return bwd_lds_t<P, DIMS, 16>(N);
        case 32: return bwd_lds_t<P, DIMS, 32>(N);
        case 64: return bwd_lds_t<P, DIMS, 64>(N);
        case 128: return bwd_lds_t<P, DIMS, 128>(N);
        case 256: return bwd_lds_t<P, DIMS, 256>(N);
    }
    return (size_t)1 << 30;
}
size_t backward_lds(const Dims &d) {
    if (d.prec == VMC_BF16) return d.dims == 1 ? bwd_lds_d<BF16, 1>(d.DH, d.N) : bwd_lds_d<BF16, 2>(d.DH, d.N);
    return d.dims == 1 ? bwd_lds_d<F32, 1>(d.DH, d.N) : bwd_lds_d<F32, 2>(d.DH, d.N);
}

// bi: NULL, or the batch of vmc_step_batched (b then describes problem 0
// with the longest chain's sizes)
hipError_t launch_backward(const GradBufs &b, int64_t nsp, hipStream_t st, const BatchInfo *bi) {
    BatchInfo none;
    none.n = 0;
    const BatchInfo &B = bi ? *bi : none;
    BwdArgs a;
    a.d = b.d;
    a.BcT = b.BcT;
    a.BgT = b.BgT;
    a.Hd = b.Hd;
    a.ns = b.ns;
    a.nsp = nsp;
    a.cfg = b.cfg;
    a.act = b.act;
    a.lgT = b.lgT;
    a.hcache = b.hcache;
    a.eloc = b.eloc;
    a.w = b.weights;
    a.stats = b.stats;
    a.coef_lp = b.coef_lp;
    a.coef_ph = b.coef_ph;
    a.dtc = b.dtc;
    a.dtg = b.dtg;
    a.dth = b.dth;
    a.dcol = (float *)b.dcol;
    if (b.d.prec == VMC_BF16) return b.d.dims == 1 ? launch_bwd_d<BF16, 1>(a, B, st) : launch_bwd_d<BF16, 2>(a, B, st);
    return b.d.dims == 1 ? launch_bwd_d<F32, 1>(a, B, st) : launch_bwd_d<F32, 2>(a, B, st);
}

}  // namespace vmc
