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
//      products, DPP row sums and a cross-wave sum in LDS;
//   5. a per-row finalisation: log-softmax, the sampling decision or the
//      teacher-forced spin, FP64 accumulation of log P and the phase.
// The hidden state is double-buffered in LDS (the previous h is the operand
// while the new h is written), so no operand copies are made.  With REGW the
// cell weights stay in registers for the whole persistent launch and the GLU
// weights in LDS; otherwise both stream from L2.
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

// Sum over the 16 lanes of a DPP row; every lane of the row gets the sum.
// Each stage is one v_add_f32 with a DPP source (quad swaps, then the half-
// row and row mirrors).  A DPP read of a VGPR written by the previous VALU
// instruction needs two wait states, hence the s_nop before each stage.
__device__ inline float row16_sum(float v) {
    float t;
    asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf"
                 : "=&v"(t) : "v"(v));
    asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf"
                 : "=&v"(v) : "v"(t));
    asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 row_half_mirror row_mask:0xf bank_mask:0xf"
                 : "=&v"(t) : "v"(v));
    asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 row_mirror row_mask:0xf bank_mask:0xf"
                 : "=&v"(v) : "v"(t));
    return v;
}

template <class P>
__device__ inline typename P::store_t cvt(float x);
template <>
__device__ inline float cvt<F32>(float x) { return x; }
template <>
__device__ inline uint16_t cvt<BF16>(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

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
    constexpr int GLD = KHB + C::PADE;  // row stride of the GLU weights in LDS

    __shared__ __align__(16) T sH[2][MT * H_LD];
    __shared__ __align__(16) T sV[DIMS == 2 ? MT * H_LD : 8];
    __shared__ __align__(16) T sX[MT * X_LD];
    __shared__ __align__(16) T sG[REGW ? 2 * DH * GLD : 8];
    __shared__ float sLog[C::WU][MT][4];
    __shared__ int sRow[MT];
    __shared__ int sTile;
    extern __shared__ uint8_t sSig[];  // [MT][N]

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w / C::WU, wu = w % C::WU;
    const int N = a.d.N, Lx = a.d.Lx, Ly = a.d.Ly;
    const int cplx = a.d.cplx, glu = a.d.glu;
    const int NO = cplx ? 4 : 2;
    const T *__restrict__ Bc = (const T *)a.Bc;
    const T *__restrict__ Bg = (const T *)a.Bg;
    const int64_t ns_c = a.ns_cache;
    constexpr int NA = DIMS == 1 ? 4 : 3;  // gate features; the GLU pair follows
    T *colbuf = (T *)a.colbuf + (int64_t)blockIdx.x * Lx * MT * DH;
    const int l16 = lane & 15, lq = lane >> 4;

    // per-lane constants: biases, head weights (fixed unit per lane and block)
    float bias0[UB], bias1[UB], bias2[UB], bin_[UB], win0[UB], win1[UB], gb1[UB], gb2[UB], hw[4][UB];
#pragma unroll
    for (int ub = 0; ub < UB; ub++) {
        const int u = wu * C::UW + ub * 16 + l16;
        if (DIMS == 1) {
            bias0[ub] = a.E[E1_BG * DH + u];
            bias1[ub] = a.E[E1_BR * DH + u];
            bias2[ub] = a.E[E1_BH * DH + u];
            bin_[ub] = a.E[E1_BIN * DH + u];
            win0[ub] = a.E[E1_XIN0 * DH + u];
            win1[ub] = a.E[E1_XIN1 * DH + u];
        } else {
            bias0[ub] = a.E[E2_B * DH + u];
            bias1[ub] = a.E[E2_BG * DH + u];
            bias2[ub] = 0.f;
            bin_[ub] = win0[ub] = win1[ub] = 0.f;
        }
        gb1[ub] = a.E[E_B1 * DH + u];
        gb2[ub] = a.E[E_B2 * DH + u];
#pragma unroll
        for (int o = 0; o < 4; o++) hw[o][ub] = a.Hd[o * DH + u];
    }
    const float hc0 = a.hc[0], hc1 = a.hc[1], hc2 = a.hc[2], hc3 = a.hc[3];

    // cell weights in registers (REGW): fragment of gate g, k-step ks, unit block ub
    uint4 wreg[REGW ? 3 : 1][REGW ? NKS : 1][REGW ? UB : 1];
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
        // GLU weights into LDS
        for (int e = tid; e < 2 * DH * (KHB / VEC); e += NT) {
            const int n = e / (KHB / VEC), c = (e % (KHB / VEC)) * VEC;
            *(uint4 *)&sG[n * GLD + c] = *(const uint4 *)&Bg[(int64_t)n * KHB + c];
        }
    }
    // zero the operand tiles once (padding columns stay zero)
    for (int e = tid; e < 2 * MT * H_LD; e += NT) (&sH[0][0])[e] = cvt<P>(0.f);
    if (DIMS == 2)
        for (int e = tid; e < MT * H_LD; e += NT) sV[e] = cvt<P>(0.f);
    for (int e = tid; e < MT * X_LD; e += NT) sX[e] = cvt<P>(0.f);

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
                for (int ii = 0; ii < 4; ii++) hreg[rb][ub][ii] = 0.f;
        if (p >= 0) {
            const int pb = ((p + 1) & 1) ^ 1;
            for (int e = tid; e < MT * (DH / 4); e += NT) {
                const int r = e / (DH / 4), c = (e % (DH / 4)) * 4;
                const int s = sRow[r];
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (s >= 0) v = *(const float4 *)&a.hcache[((int64_t)p * ns_c + s) * DH + c];
                T *d = &sH[pb][r * H_LD + c];
                d[0] = cvt<P>(v.x);
                d[1] = cvt<P>(v.y);
                d[2] = cvt<P>(v.z);
                d[3] = cvt<P>(v.w);
            }
            if (DIMS == 1) {
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ub = 0; ub < UB; ub++)
#pragma unroll
                        for (int ii = 0; ii < 4; ii++) {
                            const int r = wr * C::RW + rb * 16 + 4 * lq + ii;
                            const int u = wu * C::UW + ub * 16 + l16;
                            const int s = sRow[r];
                            hreg[rb % (DIMS == 1 ? RB : 1)][ub % (DIMS == 1 ? UB : 1)][ii] =
                                s >= 0 ? a.hcache[((int64_t)p * ns_c + s) * DH + u] : 0.f;
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
                    d[0] = cvt<P>(pfa[i].x);
                    d[1] = cvt<P>(pfa[i].y);
                    d[2] = cvt<P>(pfa[i].z);
                    d[3] = cvt<P>(pfa[i].w);
                    if (VEC == 8) {
                        d[4] = cvt<P>(pfb[i].x);
                        d[5] = cvt<P>(pfb[i].y);
                        d[6] = cvt<P>(pfb[i].z);
                        d[7] = cvt<P>(pfb[i].w);
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
                                float4 v = *(const float4 *)&src[x];
                                d[x] = cvt<P>(v.x);
                                d[x + 1] = cvt<P>(v.y);
                                d[x + 2] = cvt<P>(v.z);
                                d[x + 3] = cvt<P>(v.w);
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
            float hv[RB][UB][4];
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
                float gvs[STORE ? 4 : 1][UB][4];  // gate values of this block, for the transposed store
#pragma unroll
                for (int ii = 0; ii < 4; ii++) {
                    const int r = wr * C::RW + rb * 16 + 4 * lq + ii;
                    const int s = sRow[r];
                    int xz = 0;
                    if (DIMS == 1) xz = has_hz ? sSig[r * N + site_hz] : -1;
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) {
                        const int u = wu * C::UW + ub * 16 + l16;
                        const float g0 = acc[ub][ii], g1 = acc[UB + ub][ii], g2 = acc[2 * UB + ub][ii];
                        float h, s0, s1, s2, s3 = 0.f;
                        if (DIMS == 1) {
                            const float uu = sigmoidf_(g0 + bias0[ub]);
                            const float rr = sigmoidf_(g1 + bias1[ub]);
                            const float m = g2 + bias2[ub];
                            const float cin = bin_[ub] + (xz == 0 ? win0[ub] : (xz == 1 ? win1[ub] : 0.f));
                            const float c = tanhf_(rr * m + cin);
                            const float hp = hreg[rb % (DIMS == 1 ? RB : 1)][ub % (DIMS == 1 ? UB : 1)][ii];
                            h = (1.0f - uu) * hp + uu * c;
                            hreg[rb % (DIMS == 1 ? RB : 1)][ub % (DIMS == 1 ? UB : 1)][ii] = h;
                            s0 = uu; s1 = rr; s2 = m; s3 = c;
                        } else {
                            const float c = tanhf_(g0 + bias0[ub]);
                            const float uu = sigmoidf_(g1 + bias1[ub]);
                            h = uu * c + (1.0f - uu) * g2;
                            s0 = c; s1 = uu; s2 = g2;
                        }
                        hv[rb][ub][ii] = (STORE && s < 0) ? 0.f : h;
                        if (DIMS == 2) sH[cb][r * H_LD + u] = cvt<P>(h);
                        if (s >= 0 && store_h) a.hcache[((int64_t)q * ns_c + s) * DH + u] = h;
                        if (STORE) {
                            const bool ok = s >= 0;
                            gvs[0][ub % UB][ii] = ok ? s0 : 0.f;
                            gvs[STORE ? 1 : 0][ub % UB][ii] = ok ? s1 : 0.f;
                            gvs[STORE ? 2 : 0][ub % UB][ii] = ok ? s2 : 0.f;
                            gvs[STORE ? 3 : 0][ub % UB][ii] = ok ? s3 : 0.f;
                        }
                    }
                }
                if (store_act) {
                    const int64_t s0 = e0 + wr * C::RW + rb * 16 + 4 * lq;
                    if (s0 < a.nsp) {
#pragma unroll
                        for (int ub = 0; ub < UB; ub++) {
                            const int u = wu * C::UW + ub * 16 + l16;
                            store4<P>((T *)a.hT + ((int64_t)q * DH + u) * a.nsp + s0, hv[rb][ub][0], hv[rb][ub][1],
                                      hv[rb][ub][2], hv[rb][ub][3]);
#pragma unroll
                            for (int f = 0; f < NA; f++)
                                *(float4 *)&a.act[((int64_t)q * (NA + 2) * DH + f * DH + u) * a.nsp + s0] =
                                    make_float4(gvs[STORE ? f : 0][ub][0], gvs[STORE ? f : 0][ub][1],
                                                gvs[STORE ? f : 0][ub][2], gvs[STORE ? f : 0][ub][3]);
                        }
                    }
                }
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
                                    P::mma(acc[g * UB + ub], af, wreg[REGW ? g : 0][REGW ? ks : 0][REGW ? ub : 0]);
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
                            for (int rb = 0; rb < RB; rb++) P::mma(acc[rb][g * UB + ub], af[rb], bf);
                        }
                }
#pragma unroll
                for (int rb = 0; rb < RB; rb++) epilogue(rb, acc[rb]);
            }
            if (DIMS == 1) {
                // in 1D the operand buffer of this step is sH[pb]; writing
                // sH[cb] could not race, but keep one writer pattern for both
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ii = 0; ii < 4; ii++)
#pragma unroll
                        for (int ub = 0; ub < UB; ub++)
                            sH[cb][(wr * C::RW + rb * 16 + 4 * lq + ii) * H_LD + wu * C::UW + ub * 16 + l16] =
                                cvt<P>(hv[rb][ub][ii]);
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
                float part[4][4], gk[UB][4], ga1[STORE ? UB : 1][4], ga2[STORE ? UB : 1][4];
#pragma unroll
                for (int ii = 0; ii < 4; ii++)
#pragma unroll
                    for (int o = 0; o < 4; o++) part[ii][o] = 0.f;
#pragma unroll
                for (int ii = 0; ii < 4; ii++) {
                    const int r = wr * C::RW + rb * 16 + 4 * lq + ii;
                    const int s = sRow[r];
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) {
                        const int u = wu * C::UW + ub * 16 + l16;
                        float g;
                        if (glu) {
                            const float a1 = acc2[ub][ii] + gb1[ub];
                            const float a2 = acc2[UB + ub][ii] + gb2[ub];
                            g = a1 * sigmoidf_(a2);
                            if (STORE) {
                                ga1[ub % UB][ii] = s >= 0 ? a1 : 0.f;
                                ga2[ub % UB][ii] = s >= 0 ? a2 : 0.f;
                            }
                        } else {
                            g = hv[rb][ub][ii];
                        }
                        part[ii][0] += hw[0][ub] * g;
                        part[ii][1] += hw[1][ub] * g;
                        if (cplx) {
                            part[ii][2] += hw[2][ub] * g;
                            part[ii][3] += hw[3][ub] * g;
                        }
                        if (STORE) gk[ub][ii] = s >= 0 ? g : 0.f;
                    }
                }
                if (store_act && glu) {
                    const int64_t s0 = e0 + wr * C::RW + rb * 16 + 4 * lq;
                    if (s0 < a.nsp) {
#pragma unroll
                        for (int ub = 0; ub < UB; ub++) {
                            const int u = wu * C::UW + ub * 16 + l16;
                            store4<P>((T *)a.gT + ((int64_t)q * DH + u) * a.nsp + s0, gk[ub][0], gk[ub][1], gk[ub][2],
                                      gk[ub][3]);
                            float *fa = &a.act[((int64_t)q * (NA + 2) * DH + NA * DH + u) * a.nsp + s0];
                            *(float4 *)fa = make_float4(ga1[ub % UB][0], ga1[ub % UB][1], ga1[ub % UB][2], ga1[ub % UB][3]);
                            *(float4 *)(fa + (int64_t)DH * a.nsp) =
                                make_float4(ga2[ub % UB][0], ga2[ub % UB][1], ga2[ub % UB][2], ga2[ub % UB][3]);
                        }
                    }
                }
#pragma unroll
                for (int ii = 0; ii < 4; ii++) {
                    const int r = wr * C::RW + rb * 16 + 4 * lq + ii;
                    const float v0 = row16_sum(part[ii][0]);
                    const float v1 = row16_sum(part[ii][1]);
                    float v2 = 0.f, v3 = 0.f;
                    if (cplx) {
                        v2 = row16_sum(part[ii][2]);
                        v3 = row16_sum(part[ii][3]);
                    }
                    if (l16 == 0) *(float4 *)&sLog[wu][r][0] = make_float4(v0, v1, v2, v3);
                }
            };
            auto glu_frag = [&](int rb, int kk) -> uint4 {
                const int arow = wr * C::RW + rb * 16 + l16;
                return *(const uint4 *)&sH[cb][arow * H_LD + kk + VEC * lq];
            };
            if (!glu) {
#pragma unroll
                for (int rb = 0; rb < RB; rb++) glu_epilogue(rb, nullptr);
            } else if (REGW) {
                auto gblock = [&](int rb, f32x4_t *acc2) {
#pragma unroll
                    for (int c = 0; c < 2 * UB; c++) acc2[c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kk = 0; kk < KHB; kk += KS) {
                        const uint4 af = glu_frag(rb, kk);
#pragma unroll
                        for (int g = 0; g < 2; g++)
#pragma unroll
                            for (int ub = 0; ub < UB; ub++) {
                                const int n = g * DH + wu * C::UW + ub * 16 + l16;
                                P::mma(acc2[g * UB + ub], af, *(const uint4 *)&sG[n * GLD + kk + VEC * lq]);
                            }
                    }
                };
                f32x4_t acc2[2][2 * UB];
                gblock(0, acc2[0]);
#pragma unroll
                for (int rb = 0; rb < RB; rb++) {
                    if (rb + 1 < RB) gblock(rb + 1, acc2[(rb + 1) & 1]);
                    glu_epilogue(rb, acc2[rb & 1]);
                }
            } else {
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
                            for (int rb = 0; rb < RB; rb++) P::mma(acc2[rb][g * UB + ub], af[rb], bf);
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
