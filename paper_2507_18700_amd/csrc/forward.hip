// Forward engine of the GRU RNN wave function on gfx950.
//
// One kernel runs the autoregressive chain (Eq. 1) for a tile of rows over a
// range of order positions; a row is a sample (sampling, Sec. II A, or
// teacher-forced log psi) or a connected configuration of the local energy
// (suffix chain after its first changed position, Eqs. 6-7).  Per order
// position the tile does:
//   1. gather the hidden inputs (1D: h_{n-1}; 2D: [h_hz | h_vt], App. A) into
//      an LDS operand tile;
//   2. the cell contraction [rows x K] . [K x 3*DH] on MFMA, each wave owning
//      all three gate columns of a slice of hidden units, so the gate algebra
//      of App. A runs in registers on the MFMA output;
//   3. the optional GLU contraction [rows x DH] . [DH x 2*DH] on MFMA;
//   4. the 2- or 4-logit heads (Eqs. 3, 5) as lane partial dot products,
//      16-lane shuffles and a cross-wave sum in LDS;
//   5. a per-row finalisation: log-softmax, the sampling decision or the
//      teacher-forced spin, log P and phase accumulation, cache writes.
#include "kernels.h"

namespace vmc {

// ------------------------------------------------------------------ staging

// Builds the MFMA-ready padded copies of the parameters (see common.h).
template <class P>
__global__ void stage_weights(Dims d, const float *__restrict__ prm, typename P::store_t *Bc,
                              typename P::store_t *BcT, typename P::store_t *Bg,
                              typename P::store_t *BgT, float *E, float *Hd, float *hc, int KP,
                              int KGP, int NCP) {
    typedef typename P::store_t T;
    const int dh = d.dh, DH = d.DH;
    ParamLayout L = param_layout(d.dims, dh, d.glu, d.cplx);
    const int64_t nBc = (int64_t)3 * DH * KP, nBg = (int64_t)2 * DH * KGP, nE = (int64_t)ESLOTS * DH;
    const int64_t nBcT = (int64_t)KP * NCP;
    const int64_t total = nBc + nBg + nE + 4 * DH + 4 + nBcT;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e;
        if (r < nBc) {
            int n = (int)(r / KP), k = (int)(r % KP);
            int g = n / DH, u = n % DH;
            float v = 0.0f;
            if (u < dh) {
                if (d.dims == 1) {
                    if (k < dh) {
                        if (g == 0) v = prm[L.Wg + (int64_t)u * (dh + 2) + k];
                        else if (g == 1) v = prm[L.Wr + (int64_t)u * (dh + 2) + k];
                        else v = prm[L.Wh + (int64_t)u * dh + k];
                    }
                } else {
                    int kb = k / DH, kk = k % DH;
                    if (kb < 2 && kk < dh) {
                        int src = kb * dh + kk;
                        if (g == 0) v = prm[L.W + (int64_t)u * (2 * dh + 4) + src];
                        else if (g == 1) v = prm[L.Wg + (int64_t)u * (2 * dh + 4) + src];
                        else v = prm[L.U + (int64_t)u * 2 * dh + src];
                    }
                }
            }
            Bc[(int64_t)n * KP + k] = P::from_float(v);
            continue;
        }
        r -= nBc;
        if (r < nBg) {
            int n = (int)(r / KGP), k = (int)(r % KGP);
            int half = n / DH, u = n % DH;
            float v = 0.0f;
            if (d.glu && u < dh && k < dh) v = prm[(half ? L.W2 : L.W1) + (int64_t)u * dh + k];
            T t = P::from_float(v);
            Bg[(int64_t)n * KGP + k] = t;
            BgT[(int64_t)k * 2 * DH + n] = t;
            continue;
        }
        r -= nBg;
        if (r < nE) {
            int slot = (int)(r / DH), u = (int)(r % DH);
            float v = 0.0f;
            if (u < dh) {
                if (slot == E_B1) v = d.glu ? prm[L.b1 + u] : 0.0f;
                else if (slot == E_B2) v = d.glu ? prm[L.b2 + u] : 0.0f;
                else if (d.dims == 1) {
                    const int64_t rg = L.Wg + (int64_t)u * (dh + 2), rr = L.Wr + (int64_t)u * (dh + 2);
                    switch (slot) {
                        case E1_BG: v = prm[L.bg + u]; break;
                        case E1_XG0: v = prm[rg + dh]; break;
                        case E1_XG1: v = prm[rg + dh + 1]; break;
                        case E1_BR: v = prm[L.br + u]; break;
                        case E1_XR0: v = prm[rr + dh]; break;
                        case E1_XR1: v = prm[rr + dh + 1]; break;
                        case E1_BH: v = prm[L.bh + u]; break;
                        case E1_BIN: v = prm[L.bin + u]; break;
                        case E1_XIN0: v = prm[L.Win + (int64_t)u * 2]; break;
                        case E1_XIN1: v = prm[L.Win + (int64_t)u * 2 + 1]; break;
                    }
                } else {
                    const int64_t rw = L.W + (int64_t)u * (2 * dh + 4), rg = L.Wg + (int64_t)u * (2 * dh + 4);
                    switch (slot) {
                        case E2_B: v = prm[L.b + u]; break;
                        case E2_XH0: v = prm[rw + 2 * dh]; break;
                        case E2_XH1: v = prm[rw + 2 * dh + 1]; break;
                        case E2_XV0: v = prm[rw + 2 * dh + 2]; break;
                        case E2_XV1: v = prm[rw + 2 * dh + 3]; break;
                        case E2_BG: v = prm[L.bg + u]; break;
                        case E2_XGH0: v = prm[rg + 2 * dh]; break;
                        case E2_XGH1: v = prm[rg + 2 * dh + 1]; break;
                        case E2_XGV0: v = prm[rg + 2 * dh + 2]; break;
                        case E2_XGV1: v = prm[rg + 2 * dh + 3]; break;
                    }
                }
            }
            E[(int64_t)slot * DH + u] = v;
            continue;
        }
        r -= nE;
        if (r >= 4 * DH + 4) {
            // transposed cell weights [KP][NCP], contraction over n = gate*DH + unit
            r -= 4 * DH + 4;
            int k = (int)(r / NCP), n = (int)(r % NCP);
            float v = 0.0f;
            int g = n / DH, u = n % DH;
            if (n < 3 * DH && u < dh) {
                if (d.dims == 1) {
                    if (k < dh) {
                        if (g == 0) v = prm[L.Wg + (int64_t)u * (dh + 2) + k];
                        else if (g == 1) v = prm[L.Wr + (int64_t)u * (dh + 2) + k];
                        else v = prm[L.Wh + (int64_t)u * dh + k];
                    }
                } else {
                    int kb = k / DH, kk = k % DH;
                    if (kb < 2 && kk < dh) {
                        int src = kb * dh + kk;
                        if (g == 0) v = prm[L.W + (int64_t)u * (2 * dh + 4) + src];
                        else if (g == 1) v = prm[L.Wg + (int64_t)u * (2 * dh + 4) + src];
                        else v = prm[L.U + (int64_t)u * 2 * dh + src];
                    }
                }
            }
            BcT[(int64_t)k * NCP + n] = P::from_float(v);
            continue;
        }
        if (r < 4 * DH) {
            int o = (int)(r / DH), u = (int)(r % DH);
            float v = 0.0f;
            if (u < dh) {
                if (o < 2) v = prm[L.Ua + (int64_t)o * dh + u];
                else if (d.cplx) v = prm[L.Up + (int64_t)(o - 2) * dh + u];
            }
            Hd[(int64_t)o * DH + u] = v;
        } else {
            int o = (int)(r - 4 * DH);
            float v = 0.0f;
            if (o < 2) v = prm[L.ca + o];
            else if (d.cplx) v = prm[L.cp + o - 2];
            hc[o] = v;
        }
    }
}

// ------------------------------------------------------------ engine kernel

template <class P, int DIMS, int DH>
__global__ __launch_bounds__(256) void rnn_forward(FwdArgs a, int mode, int store_h, int store_lpc,
                                                   int store_act) {
    typedef FwdCfg<P, DIMS, DH> C;
    typedef typename P::store_t T;
    constexpr int MT = C::MT, RB = C::RB, UB = C::UB, KP = C::KP, KGP = C::KGP;
    constexpr int SA_LD = C::SA_LD, SH_LD = C::SH_LD, VEC = P::VEC, KSTEP = P::KSTEP;

    __shared__ __align__(16) T sA[DIMS == 2 ? MT * SA_LD : 8];
    __shared__ __align__(16) T sH[MT * SH_LD];
    __shared__ float sLog[C::WU][MT][4];
    __shared__ int sRow[MT];
    __shared__ int sTile;
    extern __shared__ uint8_t sSig[];  // [MT][N]

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w / C::WU, wu = w % C::WU;
    const int N = a.d.N, Lx = a.d.Lx, Ly = a.d.Ly;
    const int cplx = a.d.cplx, glu = a.d.glu;
    const T *__restrict__ Bc = (const T *)a.Bc;
    const T *__restrict__ Bg = (const T *)a.Bg;
    const float *__restrict__ E = a.E;
    const float *__restrict__ Hd = a.Hd;
    const int64_t ns_c = a.ns_cache;
    const int NA = nact_per_unit(DIMS);
    const int AW = act_width(DIMS, DH);
    T *colbuf = (T *)a.colbuf + (int64_t)blockIdx.x * Lx * MT * DH;

    // zero both operand tiles once: padding columns stay zero for good
    for (int e = tid; e < MT * SH_LD; e += blockDim.x) sH[e] = P::from_float(0.0f);
    if (DIMS == 2)
        for (int e = tid; e < MT * SA_LD; e += blockDim.x) sA[e] = P::from_float(0.0f);

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
                int64_t ent = e0 + tid;
                if (mode != MODE_CHAIN) {
                    my_s = (int)ent;
                } else if (a.ham_kind == 0) {
                    my_s = (int)ent;
                    f1 = order_site(p, Lx);
                    cidx = p;
                } else {
                    int conn = a.list[a.list_off[p] + ent];
                    my_s = conn / a.nbond;
                    cidx = conn - my_s * a.nbond;
                    bond_sites(cidx, Lx, Ly, f1, f2);
                }
            }
            sRow[tid] = my_s;
        }
        __syncthreads();
        for (int e = tid; e < MT * N; e += blockDim.x) {
            int r = e / N, c = e - r * N;
            int s = sRow[r];
            sSig[e] = (s >= 0 && mode != MODE_SAMPLE) ? a.cfg_in[(int64_t)s * N + c] : (uint8_t)0;
        }
        __syncthreads();
        if (tid < MT && my_s >= 0 && mode == MODE_CHAIN) {
            sSig[tid * N + f1] ^= 1;
            if (f2 >= 0) sSig[tid * N + f2] ^= 1;
        }
        // initial hidden state of the operand tile
        float hreg[RB][UB][4];  // 1D: previous h of this lane's (row, unit) entries
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int ub = 0; ub < UB; ub++)
#pragma unroll
                for (int ii = 0; ii < 4; ii++) hreg[rb][ub][ii] = 0.0f;
        if (DIMS == 1) {
            for (int e = tid; e < MT * DH; e += blockDim.x) {
                int r = e / DH, u = e - r * DH;
                int s = sRow[r];
                float v = 0.0f;
                if (p >= 0 && s >= 0) v = a.hcache[((int64_t)p * ns_c + s) * DH + u];
                sH[r * SH_LD + u] = P::from_float(v);
            }
            if (p >= 0) {
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ub = 0; ub < UB; ub++)
#pragma unroll
                        for (int ii = 0; ii < 4; ii++) {
                            int r = wr * C::RW + rb * 16 + 4 * (lane >> 4) + ii;
                            int u = wu * C::UW + ub * 16 + (lane & 15);
                            int s = sRow[r];
                            hreg[rb][ub][ii] = s >= 0 ? a.hcache[((int64_t)p * ns_c + s) * DH + u] : 0.0f;
                        }
            }
        }
        float acc_lp = 0.0f, acc_ph = 0.0f;
        __syncthreads();

        // ------------------------------------------------------ site loop
        for (int q = p + 1; q < N; q++) {
            const int site = order_site(q, Lx);
            const int jrow = q / Lx, icol = site - jrow * Lx;
            const bool has_hz = (q % Lx) != 0;
            const int site_hz = has_hz ? order_site(q - 1, Lx) : -1;
            const bool has_vt = DIMS == 2 && jrow > 0;
            const int site_vt = has_vt ? site - Lx : -1;
            const int pos_vt = has_vt ? site_pos(site_vt, Lx) : -1;

            // 1. operand tile (2D): [h_hz | h_vt]
            if (DIMS == 2) {
                constexpr int C8 = 2 * DH / 8;
                for (int e = tid; e < MT * C8; e += blockDim.x) {
                    int r = e / C8, c8 = (e - r * C8) * 8;
                    int half = c8 >= DH, col = c8 - half * DH;
                    int s = sRow[r];
                    T *dst = &sA[r * SA_LD + c8];
                    int src;  // 0 zero, 1 cache at position ps, 2 own h (sH), 3 column buffer
                    int ps = -1;
                    if (!half) {
                        if (!has_hz) src = 0;
                        else if (q - 1 <= p) { src = 1; ps = q - 1; }
                        else src = 2;
                    } else {
                        if (!has_vt) src = 0;
                        else if (pos_vt <= p) { src = 1; ps = pos_vt; }
                        else if (pos_vt == q - 1) src = 2;
                        else src = 3;
                    }
                    if (src == 1 && s < 0) src = 0;
                    if (src == 0) {
#pragma unroll
                        for (int x = 0; x < 8; x++) dst[x] = P::from_float(0.0f);
                    } else if (src == 1) {
                        const float4 *sp = (const float4 *)&a.hcache[((int64_t)ps * ns_c + s) * DH + col];
                        float4 v0 = sp[0], v1 = sp[1];
                        dst[0] = P::from_float(v0.x); dst[1] = P::from_float(v0.y);
                        dst[2] = P::from_float(v0.z); dst[3] = P::from_float(v0.w);
                        dst[4] = P::from_float(v1.x); dst[5] = P::from_float(v1.y);
                        dst[6] = P::from_float(v1.z); dst[7] = P::from_float(v1.w);
                    } else if (src == 2) {
#pragma unroll
                        for (int x = 0; x < 8; x++) dst[x] = sH[r * SH_LD + col + x];
                    } else {
                        const T *cp = &colbuf[((int64_t)icol * MT + r) * DH + col];
#pragma unroll
                        for (int x = 0; x < 8; x++) dst[x] = cp[x];
                    }
                }
                __syncthreads();
            }

            // 2. cell contraction on MFMA
            f32x4_t acc[RB][3 * UB];
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int c = 0; c < 3 * UB; c++) acc[rb][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
            {
                const T *Aop = DIMS == 2 ? sA : sH;
                constexpr int ALD = DIMS == 2 ? SA_LD : SH_LD;
#pragma unroll 2
                for (int kk = 0; kk < KP; kk += KSTEP) {
                    uint4 af[RB];
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) {
                        int row = wr * C::RW + rb * 16 + (lane & 15);
                        af[rb] = *(const uint4 *)&Aop[row * ALD + kk + VEC * (lane >> 4)];
                    }
#pragma unroll
                    for (int g = 0; g < 3; g++)
#pragma unroll
                        for (int ub = 0; ub < UB; ub++) {
                            int n = g * DH + wu * C::UW + ub * 16 + (lane & 15);
                            uint4 bf = *(const uint4 *)&Bc[(int64_t)n * KP + kk + VEC * (lane >> 4)];
#pragma unroll
                            for (int rb = 0; rb < RB; rb++) P::mma(acc[rb][g * UB + ub], af[rb], bf);
                        }
                }
            }
            if (DIMS == 1) __syncthreads();  // sH is the operand: all waves done before overwrite

            // 3. gate algebra (App. A), h into sH / caches
            float hv[RB][UB][4];
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ii = 0; ii < 4; ii++) {
                    const int r = wr * C::RW + rb * 16 + 4 * (lane >> 4) + ii;
                    const int s = sRow[r];
                    const int xz = has_hz ? sSig[r * N + site_hz] : -1;
                    const int xv = has_vt ? sSig[r * N + site_vt] : -1;
#pragma unroll
                    for (int ub = 0; ub < UB; ub++) {
                        const int u = wu * C::UW + ub * 16 + (lane & 15);
                        float h, g0 = acc[rb][ub][ii], g1 = acc[rb][UB + ub][ii], g2 = acc[rb][2 * UB + ub][ii];
                        float s0, s1, s2, s3 = 0.f;
                        if (DIMS == 1) {
                            float pu = g0 + E[E1_BG * DH + u] + (xz >= 0 ? E[(E1_XG0 + xz) * DH + u] : 0.f);
                            float pr = g1 + E[E1_BR * DH + u] + (xz >= 0 ? E[(E1_XR0 + xz) * DH + u] : 0.f);
                            float m = g2 + E[E1_BH * DH + u];
                            float uu = sigmoidf_(pu), rr = sigmoidf_(pr);
                            float cin = E[E1_BIN * DH + u] + (xz >= 0 ? E[(E1_XIN0 + xz) * DH + u] : 0.f);
                            float c = tanhf_(rr * m + cin);
                            h = (1.0f - uu) * hreg[rb][ub][ii] + uu * c;
                            hreg[rb][ub][ii] = h;
                            s0 = uu; s1 = rr; s2 = m; s3 = c;
                        } else {
                            float pc = g0 + E[E2_B * DH + u] + (xz >= 0 ? E[(E2_XH0 + xz) * DH + u] : 0.f) +
                                       (xv >= 0 ? E[(E2_XV0 + xv) * DH + u] : 0.f);
                            float pu = g1 + E[E2_BG * DH + u] + (xz >= 0 ? E[(E2_XGH0 + xz) * DH + u] : 0.f) +
                                       (xv >= 0 ? E[(E2_XGV0 + xv) * DH + u] : 0.f);
                            float c = tanhf_(pc), uu = sigmoidf_(pu);
                            h = uu * c + (1.0f - uu) * g2;
                            s0 = c; s1 = uu; s2 = g2;
                        }
                        hv[rb][ub][ii] = h;
                        sH[r * SH_LD + u] = P::from_float(h);
                        if (s >= 0) {
                            if (store_h) a.hcache[((int64_t)q * ns_c + s) * DH + u] = h;
                            if (store_act) {
                                float *ar = a.act + ((int64_t)q * ns_c + s) * AW;
                                ar[0 * DH + u] = s0;
                                ar[1 * DH + u] = s1;
                                ar[2 * DH + u] = s2;
                                if (DIMS == 1) ar[3 * DH + u] = s3;
                            }
                        }
                        if (DIMS == 2 && Ly > 1) colbuf[((int64_t)icol * MT + r) * DH + u] = P::from_float(h);
                    }
                }
            __syncthreads();

            // 4. GLU and heads
            float part[RB][4][4];  // [rb][ii][out]
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ii = 0; ii < 4; ii++)
#pragma unroll
                    for (int o = 0; o < 4; o++) part[rb][ii][o] = 0.f;
            if (glu) {
                f32x4_t acc2[RB][2 * UB];
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int c = 0; c < 2 * UB; c++) acc2[rb][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < KGP; kk += KSTEP) {
                    uint4 af[RB];
#pragma unroll
                    for (int rb = 0; rb < RB; rb++) {
                        int row = wr * C::RW + rb * 16 + (lane & 15);
                        af[rb] = *(const uint4 *)&sH[row * SH_LD + kk + VEC * (lane >> 4)];
                    }
#pragma unroll
                    for (int g = 0; g < 2; g++)
#pragma unroll
                        for (int ub = 0; ub < UB; ub++) {
                            int n = g * DH + wu * C::UW + ub * 16 + (lane & 15);
                            uint4 bf = *(const uint4 *)&Bg[(int64_t)n * KGP + kk + VEC * (lane >> 4)];
#pragma unroll
                            for (int rb = 0; rb < RB; rb++) P::mma(acc2[rb][g * UB + ub], af[rb], bf);
                        }
                }
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ii = 0; ii < 4; ii++) {
                        const int r = wr * C::RW + rb * 16 + 4 * (lane >> 4) + ii;
                        const int s = sRow[r];
#pragma unroll
                        for (int ub = 0; ub < UB; ub++) {
                            const int u = wu * C::UW + ub * 16 + (lane & 15);
                            float a1 = acc2[rb][ub][ii] + E[E_B1 * DH + u];
                            float a2 = acc2[rb][UB + ub][ii] + E[E_B2 * DH + u];
                            float g = a1 * sigmoidf_(a2);
                            if (store_act && s >= 0) {
                                float *ar = a.act + ((int64_t)q * ns_c + s) * AW + NA * DH;
                                ar[u] = a1;
                                ar[DH + u] = a2;
                                ar[2 * DH + u] = g;
                            }
#pragma unroll
                            for (int o = 0; o < 4; o++) part[rb][ii][o] += Hd[o * DH + u] * g;
                        }
                    }
            } else {
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ii = 0; ii < 4; ii++) {
                        const int r = wr * C::RW + rb * 16 + 4 * (lane >> 4) + ii;
                        const int s = sRow[r];
#pragma unroll
                        for (int ub = 0; ub < UB; ub++) {
                            const int u = wu * C::UW + ub * 16 + (lane & 15);
                            float g = hv[rb][ub][ii];
                            if (store_act && s >= 0) a.act[((int64_t)q * ns_c + s) * AW + (NA + 2) * DH + u] = g;
#pragma unroll
                            for (int o = 0; o < 4; o++) part[rb][ii][o] += Hd[o * DH + u] * g;
                        }
                    }
            }
            // reduce the head partials over the 16 lanes that share rows
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int ii = 0; ii < 4; ii++)
#pragma unroll
                    for (int o = 0; o < 4; o++) {
                        float v = part[rb][ii][o];
                        v += __shfl_xor(v, 8, 16);
                        v += __shfl_xor(v, 4, 16);
                        v += __shfl_xor(v, 2, 16);
                        v += __shfl_xor(v, 1, 16);
                        part[rb][ii][o] = v;
                    }
            if ((lane & 15) == 0) {
#pragma unroll
                for (int rb = 0; rb < RB; rb++)
#pragma unroll
                    for (int ii = 0; ii < 4; ii++) {
                        const int r = wr * C::RW + rb * 16 + 4 * (lane >> 4) + ii;
#pragma unroll
                        for (int o = 0; o < 4; o++) sLog[wu][r][o] = part[rb][ii][o];
                    }
            }
            __syncthreads();

            // 5. per-row finalisation
            if (tid < MT && my_s >= 0) {
                const int r = tid, s = my_s;
                float l0 = a.hc[0], l1 = a.hc[1], z0 = a.hc[2], z1 = a.hc[3];
#pragma unroll
                for (int x = 0; x < C::WU; x++) {
                    l0 += sLog[x][r][0];
                    l1 += sLog[x][r][1];
                    z0 += sLog[x][r][2];
                    z1 += sLog[x][r][3];
                }
                const float mx = fmaxf(l0, l1);
                const float lse = mx + log1pf(expf(-fabsf(l0 - l1)));
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
                        uni = (float)(c4[q & 3] >> 8) * (1.0f / 16777216.0f);
                    }
                    sg = (uni < expf(ls0)) ? 0 : 1;
                    sSig[r * N + site] = (uint8_t)sg;
                } else {
                    sg = sSig[r * N + site];
                }
                const float lsel = sg ? ls1 : ls0, psel = sg ? ph1 : ph0;
                if (mode == MODE_CHAIN) {
                    const int so = a.cfg_in[(int64_t)s * N + site];
                    const float *lr = a.lpc + ((int64_t)s * N + q) * 2;
                    const float *pr = a.phc + ((int64_t)s * N + q) * 2;
                    acc_lp += lsel - lr[so];
                    acc_ph += psel - pr[so];
                } else {
                    acc_lp += lsel;
                    acc_ph += psel;
                }
                if (store_lpc) {
                    float *lr = a.lpc + ((int64_t)s * N + q) * 2;
                    float *pr = a.phc + ((int64_t)s * N + q) * 2;
                    lr[0] = ls0;
                    lr[1] = ls1;
                    pr[0] = ph0;
                    pr[1] = ph1;
                }
                if (store_act) {
                    float *ar = a.act + ((int64_t)q * ns_c + s) * AW + (NA + 3) * DH;
                    ar[0] = l0;
                    ar[1] = l1;
                    ar[2] = z0;
                    ar[3] = z1;
                }
            }
            __syncthreads();
        }

        // ------------------------------------------------------ tile outputs
        if (tid < MT && my_s >= 0) {
            if (mode == MODE_CHAIN) {
                a.dsuf[(int64_t)my_s * a.NC + cidx] = make_float2(acc_lp, acc_ph);
            } else {
                if (a.logp) a.logp[my_s] = acc_lp;
                if (a.phase) a.phase[my_s] = acc_ph;
            }
        }
        if (mode == MODE_SAMPLE) {
            for (int e = tid; e < MT * N; e += blockDim.x) {
                int r = e / N, c = e - r * N;
                int s = sRow[r];
                if (s >= 0) a.cfg_out[(int64_t)s * N + c] = sSig[e];
            }
        }
    }
}

// --------------------------------------------------------- chain schedule

// Per first-changed position p: capacity offsets of the connection list
// (Heisenberg) or the row counts (TFIM: every sample, p < N-1), the zeroed
// counters, and the tile counter.
__global__ void sched_prep(int ham_kind, int Lx, int Ly, int64_t ns, int *cnt, int *list_off,
                           int *tile_counter) {
    const int N = Lx * Ly;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *tile_counter = 0;
        if (ham_kind == 0) {
            for (int p = 0; p < N; p++) cnt[p] = (p < N - 1) ? (int)ns : 0;
        } else {
            const int nb = bond_count(Lx, Ly);
            int64_t off = 0;
            for (int p = 0; p < N; p++) {
                list_off[p] = (int)off;
                int k = 0;
                for (int b = 0; b < nb; b++) {
                    int sa, sc;
                    bond_sites(b, Lx, Ly, sa, sc);
                    int pa = site_pos(sa, Lx), pc = site_pos(sc, Lx);
                    if ((pa < pc ? pa : pc) == p) k++;
                }
                off += (int64_t)k * ns;
                cnt[p] = 0;
            }
            list_off[N] = (int)off;
        }
    }
}

// Heisenberg: every anti-aligned bond of every sample is one connection,
// filed under its first changed order position.
__global__ void heis_list(const uint8_t *cfg, int64_t ns, int Lx, int Ly, int *cnt,
                          const int *list_off, int *list) {
    const int nb = bond_count(Lx, Ly), N = Lx * Ly;
    const int64_t total = ns * nb;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int s = (int)(e / nb), b = (int)(e % nb);
        int sa, sc;
        bond_sites(b, Lx, Ly, sa, sc);
        if (cfg[(int64_t)s * N + sa] == cfg[(int64_t)s * N + sc]) continue;
        int pa = site_pos(sa, Lx), pc = site_pos(sc, Lx);
        int p = pa < pc ? pa : pc;
        int slot = atomicAdd(&cnt[p], 1);
        list[list_off[p] + slot] = s * nb + b;
    }
}

// Tiles per position, longest suffix (smallest p) first.
__global__ void tile_scan(int N, int MT, const int *cnt, int *tile_start) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int t = 0;
        for (int p = 0; p < N; p++) {
            tile_start[p] = t;
            t += (cnt[p] + MT - 1) / MT;
        }
        tile_start[N] = t;
    }
}

// E_loc assembly (Eqs. 6, 7): diagonal part from the bonds, off-diagonal
// part sum_k coupling * psi(sigma')/psi(sigma), where
//   log psi(sigma')/psi(sigma) = [head term at p] + [suffix sum after p] with
// the head term lpc[p][1-sigma_p] - lpc[p][sigma_p] (halved for |psi|).
// One thread per sample, FP64 sums in fixed connection order.
__global__ void eloc_assemble(int ham_kind, int marshall, double J, double hx, int Lx, int Ly,
                              int64_t ns, const uint8_t *cfg, const float *lpc, const float *phc,
                              const float2 *dsuf, int NC, double *eloc) {
    const int N = Lx * Ly, nb = bond_count(Lx, Ly);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < ns;
         s += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t *c = cfg + s * N;
        double diag = 0.0, ore = 0.0, oim = 0.0;
        for (int b = 0; b < nb; b++) {
            int sa, sc;
            bond_sites(b, Lx, Ly, sa, sc);
            diag += (c[sa] == c[sc]) ? 1.0 : -1.0;
        }
        const float *lr = lpc + s * N * 2, *pr = phc + s * N * 2;
        if (ham_kind == 0) {
            diag *= -J;
            for (int p = 0; p < N; p++) {
                int sg = c[order_site(p, Lx)];
                double dl = (double)lr[2 * p + (1 - sg)] - (double)lr[2 * p + sg];
                double dp = (double)pr[2 * p + (1 - sg)] - (double)pr[2 * p + sg];
                if (p < N - 1) {
                    float2 v = dsuf[s * NC + p];
                    dl += v.x;
                    dp += v.y;
                }
                double mag = exp(0.5 * dl);
                ore += -hx * mag * cos(dp);
                oim += -hx * mag * sin(dp);
            }
        } else {
            diag *= 0.25 * J;
            const double jx = (marshall ? -0.5 : 0.5) * J;
            for (int b = 0; b < nb; b++) {
                int sa, sc;
                bond_sites(b, Lx, Ly, sa, sc);
                if (c[sa] == c[sc]) continue;
                int pa = site_pos(sa, Lx), pc = site_pos(sc, Lx);
                int p = pa < pc ? pa : pc;
                int sg = c[order_site(p, Lx)];
                double dl = (double)lr[2 * p + (1 - sg)] - (double)lr[2 * p + sg];
                double dp = (double)pr[2 * p + (1 - sg)] - (double)pr[2 * p + sg];
                float2 v = dsuf[s * NC + b];
                dl += v.x;
                dp += v.y;
                double mag = exp(0.5 * dl);
                ore += jx * mag * cos(dp);
                oim += jx * mag * sin(dp);
            }
        }
        eloc[2 * s] = diag + ore;
        eloc[2 * s + 1] = oim;
    }
}

// ------------------------------------------------------------ launchers

template <class P, int DIMS, int DH>
hipError_t launch_forward_t(const FwdArgs &a, int mode, int store_h, int store_lpc, int store_act,
                            int grid, hipStream_t st) {
    typedef FwdCfg<P, DIMS, DH> C;
    size_t dyn = (size_t)C::MT * a.d.N;
    dyn = (dyn + 15) / 16 * 16;
    hipError_t e = hipFuncSetAttribute((const void *)rnn_forward<P, DIMS, DH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((rnn_forward<P, DIMS, DH>), dim3(grid), dim3(256), dyn, st, a, mode, store_h,
                       store_lpc, store_act);
    return hipGetLastError();
}

template <class P, int DIMS>
hipError_t launch_forward_d(const FwdArgs &a, int mode, int sh, int sl, int sa, int grid, hipStream_t st) {
    switch (a.d.DH) {
        case 16: return launch_forward_t<P, DIMS, 16>(a, mode, sh, sl, sa, grid, st);
        case 32: return launch_forward_t<P, DIMS, 32>(a, mode, sh, sl, sa, grid, st);
        case 64: return launch_forward_t<P, DIMS, 64>(a, mode, sh, sl, sa, grid, st);
        case 128: return launch_forward_t<P, DIMS, 128>(a, mode, sh, sl, sa, grid, st);
        case 256: return launch_forward_t<P, DIMS, 256>(a, mode, sh, sl, sa, grid, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_forward(const FwdArgs &a, int mode, int store_h, int store_lpc, int store_act,
                          int grid, hipStream_t st) {
    if (a.d.prec == VMC_BF16)
        return a.d.dims == 1 ? launch_forward_d<BF16, 1>(a, mode, store_h, store_lpc, store_act, grid, st)
                             : launch_forward_d<BF16, 2>(a, mode, store_h, store_lpc, store_act, grid, st);
    return a.d.dims == 1 ? launch_forward_d<F32, 1>(a, mode, store_h, store_lpc, store_act, grid, st)
                         : launch_forward_d<F32, 2>(a, mode, store_h, store_lpc, store_act, grid, st);
}

int forward_tile_rows(int DH) { return DH >= 256 ? 32 : 64; }

hipError_t launch_stage(const Dims &d, const float *prm, void *Bc, void *BcT, void *Bg, void *BgT,
                        float *E, float *Hd, float *hc, hipStream_t st) {
    int KGP = d.prec == VMC_BF16 ? cround(d.DH, 32) : cround(d.DH, 16);
    int NCP = d.prec == VMC_BF16 ? cround(3 * d.DH, 32) : cround(3 * d.DH, 16);
    int64_t n = (int64_t)3 * d.DH * d.KP + (int64_t)2 * d.DH * KGP + ESLOTS * d.DH + 4 * d.DH + 4 +
                (int64_t)d.KP * NCP;
    int grid = (int)((n + 255) / 256);
    if (grid > 4096) grid = 4096;
    if (d.prec == VMC_BF16)
        hipLaunchKernelGGL(stage_weights<BF16>, dim3(grid), dim3(256), 0, st, d, prm, (uint16_t *)Bc,
                           (uint16_t *)BcT, (uint16_t *)Bg, (uint16_t *)BgT, E, Hd, hc, d.KP, KGP, NCP);
    else
        hipLaunchKernelGGL(stage_weights<F32>, dim3(grid), dim3(256), 0, st, d, prm, (float *)Bc,
                           (float *)BcT, (float *)Bg, (float *)BgT, E, Hd, hc, d.KP, KGP, NCP);
    return hipGetLastError();
}

hipError_t launch_sched(int ham_kind, int Lx, int Ly, int64_t ns, const uint8_t *cfg, int *cnt,
                        int *list_off, int *list, int *tile_start, int *tile_counter, int MT,
                        hipStream_t st) {
    hipLaunchKernelGGL(sched_prep, dim3(1), dim3(64), 0, st, ham_kind, Lx, Ly, ns, cnt, list_off, tile_counter);
    if (ham_kind == 1) {
        int64_t total = ns * bond_count(Lx, Ly);
        int grid = (int)((total + 255) / 256);
        if (grid > 8192) grid = 8192;
        if (grid < 1) grid = 1;
        hipLaunchKernelGGL(heis_list, dim3(grid), dim3(256), 0, st, cfg, ns, Lx, Ly, cnt, list_off, list);
    }
    hipLaunchKernelGGL(tile_scan, dim3(1), dim3(64), 0, st, Lx * Ly, MT, cnt, tile_start);
    return hipGetLastError();
}

hipError_t launch_assemble(const vmc_ham &H, int Lx, int Ly, int64_t ns, const uint8_t *cfg,
                           const float *lpc, const float *phc, const float2 *dsuf, int NC, double *eloc,
                           hipStream_t st) {
    int grid = (int)((ns + 255) / 256);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(eloc_assemble, dim3(grid), dim3(256), 0, st, H.kind, H.marshall, H.J, H.h, Lx, Ly, ns,
                       cfg, lpc, phc, dsuf, NC, eloc);
    return hipGetLastError();
}

}  // namespace vmc
