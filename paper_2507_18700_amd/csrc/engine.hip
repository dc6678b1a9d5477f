// Forward engine of the GRU RNN wave function on gfx950.
//
// One kernel runs the autoregressive chain (Eq. 1) for a tile of rows over a
// range of order positions.  A row is a sample (sampling, Sec. II A, or the
// teacher-forced log psi) or a connected configuration of the local energy
// (the chain after its first changed order position, Eqs. 6-7).  Per order
// position a tile does:
//   1. operands in LDS: the hidden input(s) (1D: h_{n-1}; 2D: [h_hz | h_vt],
//      App. A) and an indicator block that carries the one-hot inputs, so the
//      one-hot columns of the gate matrices ride on the MFMA (bfloat16: hi/lo
//      split of those weights, i.e. ~16 significant bits);
//   2. the cell contraction on MFMA, each wave owning all gate columns of a
//      slice of hidden units, so the App. A gate algebra runs in registers on
//      the MFMA output (biases as per-lane constants);
//   3. the optional GLU contraction on MFMA;
//   4. the 2- or 4-logit heads (Eqs. 3, 5) in FP32 as lane partial dot
//      products, a sum over the lane groups and a cross-wave sum in LDS;
//   5. a per-row finalisation: log-softmax, the sampling decision or the
//      teacher-forced spin, FP64 accumulation of log P and the phase.
// The hidden state is double-buffered in LDS (the previous h is the operand
// while the new h is written), so no operand copies are made.  With REGW the
// cell and GLU weights stay in registers for the whole persistent launch;
// otherwise both stream from L2.  The weights are the MFMA A operand, so each
// lane owns 4 consecutive units of one row: the new h goes to LDS as one
// 8-byte store and a head sum needs only the four lane groups of a row.
#include <type_traits>

#include "kernels.h"

namespace vmc {

template <class P, int DIMS, int DH, int NW>
struct Eng {
    static constexpr int WU = (DH / 16 < NW) ? DH / 16 : NW;  // waves along hidden units
    static constexpr int WR = NW / WU;                        // waves along rows
    static constexpr int UW = DH / WU;
    static constexpr int UB = UW / 16;
    static constexpr int MT = (DH >= 256) ? 32 : 64;
    static constexpr int RW = MT / WR;
    static constexpr int RB = RW / 16;
    static constexpr int KS = P::KSTEP;
    static constexpr int KHB = cround(DH, KS);                 // one hidden block of the operand
    static constexpr int NKB = KHB / KS;                       // k-steps per hidden block
    static constexpr int NHB = DIMS == 1 ? 1 : 2;              // hidden blocks (hz, vt)
    static constexpr int NKS = NHB * NKB + 1;                  // + the indicator step
    static constexpr int KPX = NKS * KS;                       // staged row length of Bc
    static constexpr int PADE = 16 / (int)sizeof(typename P::store_t);
    static constexpr int H_LD = KHB + PADE;                    // row stride of sH / sV / sG
    static constexpr int X_LD = KS + PADE;                     // row stride of the indicator tile
};

// Sum over the four 16-lane groups of a wave (lanes l, l^16, l^32, l^48);
// every lane gets the sum, with the same bits in all four lanes.  Two
// cross-row swaps (v_permlane16_swap, v_permlane32_swap) and two adds.
__device__ inline float group4_sum(float v) {
    const uint32_t b = __float_as_uint(v);
    const auto x = __builtin_amdgcn_permlane16_swap(b, b, false, false);
    const float s = __uint_as_float(x[0]) + __uint_as_float(x[1]);
    const uint32_t c = __float_as_uint(s);
    const auto y = __builtin_amdgcn_permlane32_swap(c, c, false, false);
    return __uint_as_float(y[0]) + __uint_as_float(y[1]);
}

template <class P>
__device__ inline typename P::store_t cvt(float x);
template <>
__device__ inline float cvt<F32>(float x) { return x; }
template <>
__device__ inline uint16_t cvt<BF16>(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

// Four consecutive units of one row into an operand tile (one 8- or 16-byte store).
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

template <class P, int DIMS, int DH, int NW, int REGW, int STORE>
__global__ __launch_bounds__(NW * 64) void rnn_engine(FwdArgs a, int mode, int store_h_, int store_lpc_,
                                                      int store_act_) {
    // cache writes exist only in the STORE variant (the chain kernel has none)
    const int store_h = STORE && store_h_, store_lpc = STORE && store_lpc_, store_act = STORE && store_act_;
    typedef Eng<P, DIMS, DH, NW> C;
    typedef typename P::store_t T;
    constexpr int MT = C::MT, RB = C::RB, UB = C::UB, KS = C::KS, VEC = P::VEC;
    constexpr int KHB = C::KHB, NKB = C::NKB, NKS = C::NKS, KPX = C::KPX;
    constexpr int H_LD = C::H_LD, X_LD = C::X_LD, NT = NW * 64;
    constexpr int NKG = KHB / KS;  // k-steps of the GLU contraction

    __shared__ __align__(16) T sH[2][MT * H_LD];
    __shared__ __align__(16) T sV[DIMS == 2 ? MT * H_LD : 8];
    __shared__ __align__(16) T sX[MT * X_LD];
    __shared__ __align__(16) float sLog[C::WU][MT][4];
    __shared__ __align__(16) float sHw[2][DH];  // phase-head rows (complex amplitudes)
    __shared__ int sRow[MT];
    __shared__ int sTile;
    extern __shared__ uint8_t sSig[];  // [MT][N]

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w / C::WU, wu = w % C::WU;
    const int N = a.d.N, Lx = a.d.Lx, Ly = a.d.Ly;
    const int cplx = a.d.cplx, glu = a.d.glu;
    const T *__restrict__ Bc = (const T *)a.Bc;
    const T *__restrict__ Bg = (const T *)a.Bg;
    const int64_t ns_c = a.ns_cache;
    constexpr int NA = DIMS == 1 ? 4 : 3;  // gate features; the GLU pair follows
    T *colbuf = (T *)a.colbuf + (int64_t)blockIdx.x * Lx * MT * DH;
    const int l16 = lane & 15, lq = lane >> 4;
    // The MFMAs run with the weights as the A operand, so a lane's outputs
    // are 4 consecutive hidden units (4*lq + i of a 16-unit block) of one
    // row (l16 of a 16-row block).
    auto unit0 = [&](int ub) { return wu * C::UW + ub * 16 + 4 * lq; };

    // per-lane constants of this lane's units: GLU biases, amplitude head
    float gb1[UB][4], gb2[UB][4], hw0[UB][4], hw1[UB][4];
    float bin_[DIMS == 1 ? UB : 1][4], win0[DIMS == 1 ? UB : 1][4], win1[DIMS == 1 ? UB : 1][4];
#pragma unroll
    for (int ub = 0; ub < UB; ub++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int u = unit0(ub) + i;
            gb1[ub][i] = a.E[E_B1 * DH + u];
            gb2[ub][i] = a.E[E_B2 * DH + u];
            hw0[ub][i] = a.Hd[u];
            hw1[ub][i] = a.Hd[DH + u];
            if (DIMS == 1) {
                bin_[ub % (DIMS == 1 ? UB : 1)][i] = a.E[E1_BIN * DH + u];
                win0[ub % (DIMS == 1 ? UB : 1)][i] = a.E[E1_XIN0 * DH + u];
                win1[ub % (DIMS == 1 ? UB : 1)][i] = a.E[E1_XIN1 * DH + u];
            }
        }
    for (int e = tid; e < 2 * DH; e += NT) (&sHw[0][0])[e] = a.Hd[2 * DH + e];
    const float hc0 = a.hc[0], hc1 = a.hc[1], hc2 = a.hc[2], hc3 = a.hc[3];

    // REGW: cell and GLU weight fragments in registers for the whole launch
    uint4 wreg[REGW ? 3 : 1][REGW ? NKS : 1][REGW ? UB : 1];
    uint4 wgl[REGW ? 2 : 1][REGW ? NKG : 1][REGW ? UB : 1];
    if (REGW) {
#pragma unroll
        for (int g = 0; g < 3; g++)
#pragma unroll
            for (int ks = 0; ks < NKS; ks++)
#pragma unroll
                for (int ub = 0; ub < UB; ub++) {
                    const int n = g * DH + wu * C::UW + ub * 16 + l16;
                    wreg[g][ks][ub] = *(const uint4 *)&Bc[(int64_t)n * KPX + ks * KS + VEC * lq];
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
    // zero the operand tiles once (padding columns stay zero); the bias
    // class of the indicator block is always on
    for (int e = tid; e < 2 * MT * H_LD; e += NT) (&sH[0][0])[e] = cvt<P>(0.f);
    if (DIMS == 2)
        for (int e = tid; e < MT * H_LD; e += NT) sV[e] = cvt<P>(0.f);
    for (int e = tid; e < MT * X_LD; e += NT) {
        const int c = e % X_LD;
        const bool bias_col = VEC == 8 ? (c == 8 || c == 9) : c == 4;
        sX[e] = cvt<P>(bias_col ? 1.f : 0.f);
    }

    // Head outputs of one 16-row block: sum the lane partials over the four
    // lane groups of a row, then one lane group stores the wave's sums.
    auto head_out = [&](int r, float p0, float p1, float p2, float p3) {
        p0 = group4_sum(p0);
        p1 = group4_sum(p1);
        if (cplx) {
            p2 = group4_sum(p2);
            p3 = group4_sum(p3);
        }
        if (lq == 0) *(float4 *)&sLog[wu][r][0] = make_float4(p0, p1, p2, p3);
    };
    // partial head sums of the lane's 4 units of row r for g (4 values per block)
    auto head_part = [&](int ub, const float *g, float &p0, float &p1, float &p2, float &p3) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            p0 += hw0[ub][i] * g[i];
            p1 += hw1[ub][i] * g[i];
        }
        if (cplx) {
            const float4 z0 = *(const float4 *)&sHw[0][unit0(ub)];
            const float4 z1 = *(const float4 *)&sHw[1][unit0(ub)];
            p2 += z0.x * g[0] + z0.y * g[1] + z0.z * g[2] + z0.w * g[3];
            p3 += z1.x * g[0] + z1.y * g[1] + z1.z * g[2] + z1.w * g[3];
        }
    };
    bool first = true;
    for (;;) {
        // ---------------------------------------------------------- tile
        int p = -1, nrow;
        int64_t e0;
        if (mode == MODE_CHAIN) {
            __syncthreads();
            if (tid == 0) sTile = atomicAdd(a.tile_counter, 1);
            __syncthreads();
            const int t = sTile;
            if (t >= a.tile_start[N]) break;
            int lo = 0, hi = N - 1;  // largest p with tile_start[p] <= t
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (a.tile_start[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            p = lo;
            e0 = (int64_t)(t - a.tile_start[p]) * MT;
            nrow = (int)min((int64_t)MT, (int64_t)a.cnt[p] - e0);
        } else {
            if (!first) break;
            e0 = (int64_t)blockIdx.x * MT;
            nrow = (int)min((int64_t)MT, a.nrows - e0);
        }
        first = false;

        // ------------------------------------------------------ row setup
        int my_s = -1, f1 = -1, f2 = -1, cidx = 0;
        if (tid < MT) {
            if (tid < nrow) {
                const int64_t ent = e0 + tid;
                if (mode != MODE_CHAIN) {
                    my_s = (int)ent;
                } else if (a.ham_kind == 0) {
                    my_s = (int)ent;
                    f1 = order_site(p, Lx);
                    cidx = p;
                } else {
                    const int conn = a.list[a.list_off[p] + ent];
                    my_s = conn / a.nbond;
                    cidx = conn - my_s * a.nbond;
                    bond_sites(cidx, Lx, Ly, f1, f2);
                }
            }
            sRow[tid] = my_s;
        }
        __syncthreads();
        for (int e = tid; e < MT * N; e += NT) {
            const int r = e / N, c = e - r * N;
            const int s = sRow[r];
            sSig[e] = (s >= 0 && mode != MODE_SAMPLE) ? a.cfg_in[(int64_t)s * N + c] : (uint8_t)0;
        }
        __syncthreads();
        if (tid < MT && my_s >= 0 && mode == MODE_CHAIN) {
            sSig[tid * N + f1] ^= 1;
            if (f2 >= 0) sSig[tid * N + f2] ^= 1;
        }
        // previous hidden state of the first step: h(p) from the prefix cache
        float hreg[DIMS == 1 ? RB : 1][DIMS == 1 ? UB : 1][4];
#pragma unroll
        for (int rb = 0; rb < (DIMS == 1 ? RB : 1); rb++)
#pragma unroll
            for (int ub = 0; ub < (DIMS == 1 ? UB : 1); ub++)
#pragma unroll
                for (int i = 0; i < 4; i++) hreg[rb][ub][i] = 0.f;
        if (p >= 0) {
            const int pb = ((p + 1) & 1) ^ 1;
            for (int e = tid; e < MT * (DH / 4); e += NT) {
                const int r = e / (DH / 4), c = (e % (DH / 4)) * 4;
                const int s = sRow[r];
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (s >= 0) v = *(const float4 *)&a.hcache[((int64_t)p * ns_c + s) * DH + c];
                const float vv[4] = {v.x, v.y, v.z, v.w};
                put4<P>(&sH[pb][r * H_LD + c], vv);
            }
            if (DIMS == 1) {
#pragma unroll
                for (int rb = 0; rb < RB; rb++) {
                    const int s = sRow[wr * C::RW + rb * 16 + l16];
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) {
                        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (s >= 0) v = *(const float4 *)&a.hcache[((int64_t)p * ns_c + s) * DH + unit0(ub)];
                        float *hr = hreg[rb % (DIMS == 1 ? RB : 1)][ub % (DIMS == 1 ? UB : 1)];
                        hr[0] = v.x;
                        hr[1] = v.y;
                        hr[2] = v.z;
                        hr[3] = v.w;
                    }
                }
            }
        }
        double acc_lp = 0.0, acc_ph = 0.0;
        __syncthreads();

        // ------------------------------------------------------ site loop
        // Vertical input of 2D position qn: from the prefix cache (first
        // steps of a chain), from the column buffer, or none (row 0, or the
        // row start, whose vertical input is h(qn-1) itself).
        auto vt_src = [&](int qn, int &icol_n, int &pos_n) -> int {  // 0 none, 1 cache, 2 column buffer
            if (DIMS != 2 || qn >= N) return 0;
            const int st = order_site(qn, Lx), jr = qn / Lx;
            icol_n = st - jr * Lx;
            if (jr == 0) return 0;
            pos_n = site_pos(st - Lx, Lx);
            if (pos_n == qn - 1) return 0;
            return pos_n <= p ? 1 : 2;
        };
        // REGW variants prefetch the next position's vertical rows into
        // registers while the current position's MFMAs run.
        constexpr int NCH = MT * (DH / VEC), PF = (NCH + NT - 1) / NT;
        float4 pfa[REGW ? PF : 1], pfb[REGW ? PF : 1];
        auto vt_issue = [&](int qn) {
            int ic = 0, pn = 0;
            const int src = vt_src(qn, ic, pn);
            if (!src) return;
#pragma unroll
            for (int i = 0; i < (REGW ? PF : 1); i++) {
                const int e = tid + i * NT;
                if (e >= NCH) break;
                const int r = e / (DH / VEC), c = (e % (DH / VEC)) * VEC;
                if (src == 1) {
                    const int s = sRow[r];
                    pfa[i] = pfb[i] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (s >= 0) {
                        const float *sp = &a.hcache[((int64_t)pn * ns_c + s) * DH + c];
                        pfa[i] = *(const float4 *)sp;
                        if (VEC == 8) pfb[i] = *(const float4 *)(sp + 4);
                    }
                } else {
                    pfa[i] = __builtin_bit_cast(float4, *(const uint4 *)&colbuf[((int64_t)ic * MT + r) * DH + c]);
                }
            }
        };
        auto vt_store = [&](int qn) {
            int ic = 0, pn = 0;
            const int src = vt_src(qn, ic, pn);
            if (!src) return;
#pragma unroll
            for (int i = 0; i < (REGW ? PF : 1); i++) {
                const int e = tid + i * NT;
                if (e >= NCH) break;
                const int r = e / (DH / VEC), c = (e % (DH / VEC)) * VEC;
                T *d = &sV[r * H_LD + c];
                if (src == 1) {
                    const float va[4] = {pfa[i].x, pfa[i].y, pfa[i].z, pfa[i].w};
                    put4<P>(d, va);
                    if (VEC == 8) {
                        const float vb[4] = {pfb[i].x, pfb[i].y, pfb[i].z, pfb[i].w};
                        put4<P>(d + 4, vb);
                    }
                } else {
                    *(uint4 *)d = __builtin_bit_cast(uint4, pfa[i]);
                }
            }
        };
        for (int q = p + 1; q < N; q++) {
            const int cb = q & 1, pb = cb ^ 1;
            const int site = order_site(q, Lx);
            const int jrow = q / Lx, icol = site - jrow * Lx;
            const bool has_hz = (q % Lx) != 0;
            const int site_hz = has_hz ? order_site(q - 1, Lx) : -1;
            const bool has_vt = DIMS == 2 && jrow > 0;
            const int site_vt = has_vt ? site - Lx : -1;
            const int pos_vt = has_vt ? site_pos(site_vt, Lx) : -1;
            const bool vt_prev = has_vt && pos_vt == q - 1;   // vertical input is h(q-1) (row start)
            const bool vt_load = has_vt && pos_vt < q - 1;    // vertical input from cache / column buffer

            // 1. operands: vertical hidden input (unless prefetched) and the indicator block
            if (DIMS == 2 && vt_load && (!REGW || q == p + 1)) {
                const bool from_cache = pos_vt <= p;
                for (int e = tid; e < MT * (DH / VEC); e += NT) {
                    const int r = e / (DH / VEC), c = (e % (DH / VEC)) * VEC;
                    const int s = sRow[r];
                    T *d = &sV[r * H_LD + c];
                    if (from_cache) {
                        if (s >= 0) {
                            const float *src = &a.hcache[((int64_t)pos_vt * ns_c + s) * DH + c];
#pragma unroll
                            for (int x = 0; x < VEC; x += 4) {
                                const float4 v = *(const float4 *)&src[x];
                                const float vv[4] = {v.x, v.y, v.z, v.w};
                                put4<P>(d + x, vv);
                            }
                        } else {
                            *(uint4 *)d = make_uint4(0, 0, 0, 0);
                        }
                    } else {
                        *(uint4 *)d = *(const uint4 *)&colbuf[((int64_t)icol * MT + r) * DH + c];
                    }
                }
            }
            if (tid < MT) {
                // indicator columns: FP32 [x_hz0, x_hz1, x_vt0, x_vt1]; BF16 each twice (hi, lo)
                const int r = tid;
                const int xz = has_hz ? sSig[r * N + site_hz] : -1;
                const int xv = has_vt ? sSig[r * N + site_vt] : -1;
                const int rep = VEC == 8 ? 2 : 1;
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    const bool on = (c < 2) ? (xz == c) : (xv == c - 2);
                    const T one = cvt<P>(on ? 1.f : 0.f);
                    sX[r * X_LD + c * rep] = one;
                    if (rep == 2) sX[r * X_LD + c * rep + 1] = one;
                }
            }
            __syncthreads();

            if (REGW) vt_issue(q + 1);

            // 2.+3. cell contraction on MFMA and the gate algebra (App. A); the
            // new h goes to sH[cb].  With register-resident weights one row
            // block at a time, so that the epilogue of one block runs under
            // the MFMAs of the next; with streamed weights all row blocks per
            // weight fragment (each fragment loaded once per step).
            auto a_frag = [&](int rb, int ks) -> uint4 {
                const int blk = ks / NKB;
                const bool is_x = ks == NKS - 1;
                const T *Aop = is_x ? sX : (blk == 0 || vt_prev) ? sH[pb] : sV;
                const int ald = is_x ? X_LD : H_LD;
                const int kc = is_x ? 0 : (ks % NKB) * KS;
                const int arow = wr * C::RW + rb * 16 + l16;
                return *(const uint4 *)&Aop[arow * ald + kc + VEC * lq];
            };
            auto ks_active = [&](int ks) -> bool {
                const int blk = ks / NKB;
                if (ks == NKS - 1) return true;
                if (blk == 0) return has_hz;
                return has_vt;
            };
            auto epilogue = [&](int rb, const f32x4_t *acc) {
                const int r = wr * C::RW + rb * 16 + l16;
                const int s = sRow[r];
                int xz = 0;
                if (DIMS == 1) xz = has_hz ? sSig[r * N + site_hz] : -1;
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
                            h = (1.0f - uu) * hp + uu * c;
                            hp = h;
                            s0 = uu; s1 = rr; s2 = g2; s3 = c;
                        } else {
                            const float c = tanhf_(g0);
                            const float uu = sigmoidf_(g1);
                            h = uu * c + (1.0f - uu) * g2;
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
                    put4<P>(&sH[cb][r * H_LD + u0], hq);
                    if (!glu) head_part(ub, hq, p0, p1, p2, p3);
                    if (STORE) {
                        if (s >= 0 && store_h)
                            *(float4 *)&a.hcache[((int64_t)q * ns_c + s) * DH + u0] =
                                make_float4(hq[0], hq[1], hq[2], hq[3]);
                        const int64_t sx = e0 + r;
                        if (store_act && sx < a.nsp) {
#pragma unroll
                            for (int i = 0; i < 4; i++) {
                                ((T *)a.hT)[((int64_t)q * DH + u0 + i) * a.nsp + sx] = cvt<P>(hq[i]);
#pragma unroll
                                for (int f = 0; f < NA; f++)
                                    a.act[((int64_t)q * (NA + 2) * DH + f * DH + u0 + i) * a.nsp + sx] =
                                        gv[STORE ? f : 0][i];
                            }
                        }
                    }
                }
                if (!glu) head_out(r, p0, p1, p2, p3);
            };
            if (REGW) {
                // branch-free variants per input pattern; the MFMAs of row
                // block rb+1 are issued ahead of the epilogue of block rb
                auto cell_phase = [&](auto HZ, auto VT) {
                    auto block = [&](int rb, f32x4_t *acc) {
#pragma unroll
                        for (int c = 0; c < 3 * UB; c++) acc[c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int ks = 0; ks < NKS; ks++) {
                            const int blk = ks / NKB;
                            const bool is_x = ks == NKS - 1;
                            if (!is_x && blk == 0 && !decltype(HZ)::value) continue;
                            if (!is_x && blk == 1 && !decltype(VT)::value) continue;
                            const uint4 af = a_frag(rb, ks);
#pragma unroll
                            for (int g = 0; g < 3; g++)
#pragma unroll
                                for (int ub = 0; ub < UB; ub++)
                                    P::mma(acc[g * UB + ub], wreg[REGW ? g : 0][REGW ? ks : 0][REGW ? ub : 0], af);
                        }
                    };
                    f32x4_t acc[2][3 * UB];
                    block(0, acc[0]);
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) {
                        if (rb + 1 < RB) block(rb + 1, acc[(rb + 1) & 1]);
                        epilogue(rb, acc[rb & 1]);
                    }
                };
                using T1 = std::integral_constant<bool, true>;
                using T0 = std::integral_constant<bool, false>;
                if (DIMS == 1) {
                    if (has_hz) cell_phase(T1{}, T0{});
                    else cell_phase(T0{}, T0{});
                } else {
                    if (has_hz && has_vt) cell_phase(T1{}, T1{});
                    else if (has_hz) cell_phase(T1{}, T0{});
                    else if (has_vt) cell_phase(T0{}, T1{});
                    else cell_phase(T0{}, T0{});
                }
            } else {
                f32x4_t acc[RB][3 * UB];
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int c = 0; c < 3 * UB; c++) acc[rb][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < NKS; ks++) {
                    if (!ks_active(ks)) continue;
                    uint4 af[RB];
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) af[rb] = a_frag(rb, ks);
#pragma unroll
                    for (int g = 0; g < 3; g++)
#pragma unroll
                        for (int ub = 0; ub < UB; ub++) {
                            const int n = g * DH + wu * C::UW + ub * 16 + l16;
                            const uint4 bf = *(const uint4 *)&Bc[(int64_t)n * KPX + ks * KS + VEC * lq];
#pragma unroll
                            for (int rb = 0; rb < RB; rb++) P::mma(acc[rb][g * UB + ub], bf, af[rb]);
                        }
                }
#pragma unroll
                for (int rb = 0; rb < RB; rb++) epilogue(rb, acc[rb]);
            }
            __syncthreads();

            if (REGW) vt_store(q + 1);

            // the column buffer keeps h for the vertical input of the next row
            if (DIMS == 2 && jrow + 1 < Ly && ((q + 1) % Lx) != 0) {
                for (int e = tid; e < MT * (DH / VEC); e += NT) {
                    const int r = e / (DH / VEC), c = (e % (DH / VEC)) * VEC;
                    *(uint4 *)&colbuf[((int64_t)icol * MT + r) * DH + c] = *(const uint4 *)&sH[cb][r * H_LD + c];
                }
            }

            // 4. GLU (MFMA) and heads (FP32)
            auto glu_epilogue = [&](int rb, const f32x4_t *acc2) {
                const int r = wr * C::RW + rb * 16 + l16;
                const int s = sRow[r];
                float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
                for (int ub = 0; ub < UB; ub++) {
                    float g[4], a1[4], a2[4];
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        a1[i] = acc2[ub][i] + gb1[ub][i];
                        a2[i] = acc2[UB + ub][i] + gb2[ub][i];
                        g[i] = a1[i] * sigmoidf_(a2[i]);
                    }
                    head_part(ub, g, p0, p1, p2, p3);
                    const int64_t sx = e0 + r;
                    if (store_act && sx < a.nsp) {
                        const bool ok = s >= 0;
                        const int u0 = unit0(ub);
#pragma unroll
                        for (int i = 0; i < 4; i++) {
                            ((T *)a.gT)[((int64_t)q * DH + u0 + i) * a.nsp + sx] = cvt<P>(ok ? g[i] : 0.f);
                            float *fa = &a.act[((int64_t)q * (NA + 2) * DH + NA * DH + u0 + i) * a.nsp + sx];
                            fa[0] = ok ? a1[i] : 0.f;
                            fa[(int64_t)DH * a.nsp] = ok ? a2[i] : 0.f;
                        }
                    }
                }
                head_out(r, p0, p1, p2, p3);
            };
            auto glu_frag = [&](int rb, int kk) -> uint4 {
                const int arow = wr * C::RW + rb * 16 + l16;
                return *(const uint4 *)&sH[cb][arow * H_LD + kk + VEC * lq];
            };
            if (glu && REGW) {
                auto gblock = [&](int rb, f32x4_t *acc2) {
#pragma unroll
                    for (int c = 0; c < 2 * UB; c++) acc2[c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kq = 0; kq < NKG; kq++) {
                        const uint4 af = glu_frag(rb, kq * KS);
#pragma unroll
                        for (int g = 0; g < 2; g++)
#pragma unroll
                            for (int ub = 0; ub < UB; ub++)
                                P::mma(acc2[g * UB + ub], wgl[REGW ? g : 0][REGW ? kq : 0][REGW ? ub : 0], af);
                    }
                };
                f32x4_t acc2[2][2 * UB];
                gblock(0, acc2[0]);
#pragma unroll
                for (int rb = 0; rb < RB; rb++) {
                    if (rb + 1 < RB) gblock(rb + 1, acc2[(rb + 1) & 1]);
                    glu_epilogue(rb, acc2[rb & 1]);
                }
            } else if (glu) {
                f32x4_t acc2[RB][2 * UB];
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int c = 0; c < 2 * UB; c++) acc2[rb][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < KHB; kk += KS) {
                    uint4 af[RB];
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) af[rb] = glu_frag(rb, kk);
#pragma unroll
                    for (int g = 0; g < 2; g++)
#pragma unroll
                        for (int ub = 0; ub < UB; ub++) {
                            const int n = g * DH + wu * C::UW + ub * 16 + l16;
                            const uint4 bf = *(const uint4 *)&Bg[(int64_t)n * KHB + kk + VEC * lq];
#pragma unroll
                            for (int rb = 0; rb < RB; rb++) P::mma(acc2[rb][g * UB + ub], bf, af[rb]);
                        }
                }
#pragma unroll
                for (int rb = 0; rb < RB; rb++) glu_epilogue(rb, acc2[rb]);
            }
            __syncthreads();

            // 5. per-row finalisation
            if (tid < MT && my_s >= 0) {
                const int r = tid, s = my_s;
                float l0 = hc0, l1 = hc1, z0 = hc2, z1 = hc3;
#pragma unroll
                for (int x = 0; x < C::WU; x++) {
                    l0 += sLog[x][r][0];
                    l1 += sLog[x][r][1];
                    z0 += sLog[x][r][2];
                    z1 += sLog[x][r][3];
                }
                const float mx = fmaxf(l0, l1);
                const float lse = mx + __logf(1.0f + __expf(-fabsf(l0 - l1)));
                const float ls0 = l0 - lse, ls1 = l1 - lse;
                const float ph0 = cplx ? PI_F * softsignf_(z0) : 0.f;
                const float ph1 = cplx ? PI_F * softsignf_(z1) : 0.f;
                int sg;
                if (mode == MODE_SAMPLE) {
                    float uni;
                    if (a.uniforms) {
                        uni = a.uniforms[(int64_t)s * N + q];
                    } else {
                        uint32_t c4[4] = {(uint32_t)(q >> 2), (uint32_t)s, (uint32_t)a.counter,
                                          (uint32_t)(a.counter >> 32)};
                        philox4x32_10(c4, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
                        const uint32_t wsel = (q & 3) == 0 ? c4[0] : (q & 3) == 1 ? c4[1] : (q & 3) == 2 ? c4[2] : c4[3];
                        uni = (float)(wsel >> 8) * (1.0f / 16777216.0f);
                    }
                    sg = (uni < __expf(ls0)) ? 0 : 1;
                    sSig[r * N + site] = (uint8_t)sg;
                } else {
                    sg = sSig[r * N + site];
                }
                acc_lp += (double)(sg ? ls1 : ls0);
                acc_ph += (double)(sg ? ph1 : ph0);
                if (store_lpc) {
                    *(float2 *)&a.lpc[((int64_t)s * N + q) * 2] = make_float2(ls0, ls1);
                    *(float2 *)&a.phc[((int64_t)s * N + q) * 2] = make_float2(ph0, ph1);
                    a.pre[(int64_t)s * N + q] = make_double2(acc_lp, acc_ph);
                }
                if (store_act) {
                    float *lg = a.lgT + (int64_t)q * 4 * a.nsp + s;
                    lg[0] = l0;
                    lg[a.nsp] = l1;
                    lg[2 * a.nsp] = z0;
                    lg[3 * a.nsp] = z1;
                }
            }
            __syncthreads();
        }

        // ------------------------------------------------------ tile outputs
        if (tid < MT && my_s >= 0) {
            if (mode == MODE_CHAIN) {
                a.dsuf[(int64_t)my_s * a.NC + cidx] = make_double2(acc_lp, acc_ph);
            } else {
                if (a.logp) a.logp[my_s] = (float)acc_lp;
                if (a.phase) a.phase[my_s] = (float)acc_ph;
            }
        }
        if (mode == MODE_SAMPLE) {
            for (int e = tid; e < MT * N; e += NT) {
                const int r = e / N, c = e - r * N;
                const int s = sRow[r];
                if (s >= 0) a.cfg_out[(int64_t)s * N + c] = sSig[e];
            }
        }
    }
}

// ------------------------------------------------------------ launchers

template <class P, int DIMS, int DH, int NW, int REGW, int STORE>
static hipError_t launch_engine_s(const FwdArgs &a, int mode, int sh, int sl, int sa, int grid, hipStream_t st) {
    typedef Eng<P, DIMS, DH, NW> C;
    size_t dyn = ((size_t)C::MT * a.d.N + 15) / 16 * 16;
    hipError_t e = hipFuncSetAttribute((const void *)rnn_engine<P, DIMS, DH, NW, REGW, STORE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((rnn_engine<P, DIMS, DH, NW, REGW, STORE>), dim3(grid), dim3(NW * 64), dyn, st, a, mode, sh,
                       sl, sa);
    return hipGetLastError();
}

template <class P, int DIMS, int DH, int NW, int REGW>
static hipError_t launch_engine_t(const FwdArgs &a, int mode, int sh, int sl, int sa, int grid, hipStream_t st) {
    if (sh || sl || sa) return launch_engine_s<P, DIMS, DH, NW, REGW, 1>(a, mode, sh, sl, sa, grid, st);
    return launch_engine_s<P, DIMS, DH, NW, REGW, 0>(a, mode, sh, sl, sa, grid, st);
}

// Variant per precision and width: bfloat16 up to d_h = 128 keeps the cell
// weights in registers (8 waves at 128, 4 below); the rest stream from L2.
template <class P, int DH>
struct Pick {
    static constexpr int REGW = (P::VEC == 8 && DH <= 128) ? 1 : 0;
    static constexpr int NW = (REGW && DH == 128) ? 8 : 4;
};

template <class P, int DIMS, int DH>
static hipError_t launch_engine_w(const FwdArgs &a, int mode, int sh, int sl, int sa, int grid, hipStream_t st) {
    return launch_engine_t<P, DIMS, DH, Pick<P, DH>::NW, Pick<P, DH>::REGW>(a, mode, sh, sl, sa, grid, st);
}

template <class P, int DIMS>
static hipError_t launch_engine_d(const FwdArgs &a, int mode, int sh, int sl, int sa, int grid, hipStream_t st) {
    switch (a.d.DH) {
        case 16: return launch_engine_w<P, DIMS, 16>(a, mode, sh, sl, sa, grid, st);
        case 32: return launch_engine_w<P, DIMS, 32>(a, mode, sh, sl, sa, grid, st);
        case 64: return launch_engine_w<P, DIMS, 64>(a, mode, sh, sl, sa, grid, st);
        case 128: return launch_engine_w<P, DIMS, 128>(a, mode, sh, sl, sa, grid, st);
        case 256: return launch_engine_w<P, DIMS, 256>(a, mode, sh, sl, sa, grid, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_forward(const FwdArgs &a, int mode, int store_h, int store_lpc, int store_act, int grid,
                          hipStream_t st) {
    if (a.d.prec == VMC_BF16)
        return a.d.dims == 1 ? launch_engine_d<BF16, 1>(a, mode, store_h, store_lpc, store_act, grid, st)
                             : launch_engine_d<BF16, 2>(a, mode, store_h, store_lpc, store_act, grid, st);
    return a.d.dims == 1 ? launch_engine_d<F32, 1>(a, mode, store_h, store_lpc, store_act, grid, st)
                         : launch_engine_d<F32, 2>(a, mode, store_h, store_lpc, store_act, grid, st);
}

int forward_tile_rows(int DH) { return DH >= 256 ? 32 : 64; }

// Row length of the staged forward cell weights [3*DH][kpx] for this model.
int engine_kpx(const Dims &d) {
    const int ks = d.prec == VMC_BF16 ? 32 : 16;
    const int khb = cround(d.DH, ks);
    return ((d.dims == 1 ? 1 : 2) * (khb / ks) + 1) * ks;
}

}  // namespace vmc
