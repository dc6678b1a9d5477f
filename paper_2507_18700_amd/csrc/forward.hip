// Parameter staging, the connection schedule of the local energy and its
// assembly (the forward engine itself is in engine.hip).
#include "kernels.h"

namespace vmc {

// ------------------------------------------------------------------ staging

// Builds the MFMA-ready padded copies of the parameters (see common.h).
//  Bc  [3*DH][KPX]: per gate row n = gate*DH + unit, the hidden block(s) of
//      width KHB (1D: h; 2D: h_hz then h_vt, zero-padded) followed by one
//      indicator block of width KS holding the one-hot columns of the gate
//      matrices (classes 0..3) and the gate biases (class 4), FP32: one
//      column per class; BF16: a hi and a lo bfloat16 column per class,
//      hi + lo = the FP32 weight to ~2^-16.
//  BcT [NHB*DH][NCP]: the hidden part transposed (backward), NCP >= 3*DH.
//  Bg  [2*DH][KHB], BgT [KHB][2*DH]: GLU (W_1 rows, then W_2 rows).
template <class P>
__global__ void stage_weights(Dims d, const float *__restrict__ prm, typename P::store_t *Bc,
                              typename P::store_t *BcT, typename P::store_t *Bg,
                              typename P::store_t *BgT, float *E, float *Hd, float *hc, int KPX,
                              int KHB, int NCP) {
    typedef typename P::store_t T;
    const int dh = d.dh, DH = d.DH, NHB = d.dims == 1 ? 1 : 2;
    const int KS = P::KSTEP;
    const int nx = d.dims == 1 ? 2 : 4;  // one-hot classes feeding the gate matrices
    ParamLayout L = param_layout(d.dims, dh, d.glu, d.cplx);
    const int64_t nBc = (int64_t)3 * DH * KPX, nBg = (int64_t)2 * DH * KHB, nE = (int64_t)ESLOTS * DH;
    const int64_t nBcT = (int64_t)NHB * DH * NCP;
    const int64_t total = nBc + nBg + nE + 4 * DH + 4 + nBcT;
    // weight of gate g, unit u at hidden-input column c (1D: c < dh; 2D: c < 2*dh)
    auto hid = [&](int g, int u, int c) -> float {
        if (d.dims == 1) {
            if (g == 0) return prm[L.Wg + (int64_t)u * (dh + 2) + c];
            if (g == 1) return prm[L.Wr + (int64_t)u * (dh + 2) + c];
            return prm[L.Wh + (int64_t)u * dh + c];
        }
        if (g == 0) return prm[L.W + (int64_t)u * (2 * dh + 4) + c];
        if (g == 1) return prm[L.Wg + (int64_t)u * (2 * dh + 4) + c];
        return prm[L.U + (int64_t)u * 2 * dh + c];
    };
    // one-hot weight of gate g (0, 1 only), unit u, class column c < nx
    auto onehot = [&](int g, int u, int c) -> float {
        if (d.dims == 1) return prm[(g == 0 ? L.Wg : L.Wr) + (int64_t)u * (dh + 2) + dh + c];
        return prm[(g == 0 ? L.W : L.Wg) + (int64_t)u * (2 * dh + 4) + 2 * dh + c];
    };
    // bias of gate g, unit u (2D: the U h' gate has none)
    auto gate_bias = [&](int g, int u) -> float {
        if (d.dims == 1) return prm[(g == 0 ? L.bg : g == 1 ? L.br : L.bh) + u];
        return g == 0 ? prm[L.b + u] : g == 1 ? prm[L.bg + u] : 0.0f;
    };
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e;
        if (r < nBc) {
            const int n = (int)(r / KPX), k = (int)(r % KPX);
            const int g = n / DH, u = n % DH;
            float v = 0.0f;
            if (u < dh) {
                if (k < NHB * KHB) {
                    const int blk = k / KHB, kk = k % KHB;
                    if (kk < dh) v = hid(g, u, blk * dh + kk);
                } else {
                    // indicator block: one-hot classes 0..nx-1, then the gate
                    // bias as class 4 (its indicator is always on)
                    const int xc = k - NHB * KHB;
                    const int c = KS == 32 ? xc >> 1 : xc;
                    float w = 0.0f;
                    if (c < nx && g < 2) w = onehot(g, u, c);
                    else if (c == 4) w = gate_bias(g, u);
                    if (KS == 32) {  // bfloat16: hi, lo per class
                        const float hi = bf2f(f2bf(w));
                        v = (xc & 1) ? w - hi : hi;
                    } else {
                        v = w;
                    }
                }
            }
            Bc[(int64_t)n * KPX + k] = P::from_float(v);
            continue;
        }
        r -= nBc;
        if (r < nBg) {
            const int n = (int)(r / KHB), k = (int)(r % KHB);
            const int half = n / DH, u = n % DH;
            float v = 0.0f;
            if (d.glu && u < dh && k < dh) v = prm[(half ? L.W2 : L.W1) + (int64_t)u * dh + k];
            const T t = P::from_float(v);
            Bg[(int64_t)n * KHB + k] = t;
            BgT[(int64_t)k * 2 * DH + n] = t;
            continue;
        }
        r -= nBg;
        if (r < nE) {
            const int slot = (int)(r / DH), u = (int)(r % DH);
            float v = 0.0f;
            if (u < dh) {
                if (slot == E_B1) v = d.glu ? prm[L.b1 + u] : 0.0f;
                else if (slot == E_B2) v = d.glu ? prm[L.b2 + u] : 0.0f;
                else if (d.dims == 1) {
                    switch (slot) {
                        case E1_BG: v = prm[L.bg + u]; break;
                        case E1_XG0: v = onehot(0, u, 0); break;
                        case E1_XG1: v = onehot(0, u, 1); break;
                        case E1_BR: v = prm[L.br + u]; break;
                        case E1_XR0: v = onehot(1, u, 0); break;
                        case E1_XR1: v = onehot(1, u, 1); break;
                        case E1_BH: v = prm[L.bh + u]; break;
                        case E1_BIN: v = prm[L.bin + u]; break;
                        case E1_XIN0: v = prm[L.Win + (int64_t)u * 2]; break;
                        case E1_XIN1: v = prm[L.Win + (int64_t)u * 2 + 1]; break;
                    }
                } else {
                    switch (slot) {
                        case E2_B: v = prm[L.b + u]; break;
                        case E2_XH0: v = onehot(0, u, 0); break;
                        case E2_XH1: v = onehot(0, u, 1); break;
                        case E2_XV0: v = onehot(0, u, 2); break;
                        case E2_XV1: v = onehot(0, u, 3); break;
                        case E2_BG: v = prm[L.bg + u]; break;
                        case E2_XGH0: v = onehot(1, u, 0); break;
                        case E2_XGH1: v = onehot(1, u, 1); break;
                        case E2_XGV0: v = onehot(1, u, 2); break;
                        case E2_XGV1: v = onehot(1, u, 3); break;
                    }
                }
            }
            E[(int64_t)slot * DH + u] = v;
            continue;
        }
        r -= nE;
        if (r >= 4 * DH + 4) {
            // transposed hidden part [NHB*DH][NCP], contraction over n = gate*DH + unit
            r -= 4 * DH + 4;
            const int k = (int)(r / NCP), n = (int)(r % NCP);
            const int g = n / DH, u = n % DH, blk = k / DH, kk = k % DH;
            float v = 0.0f;
            if (n < 3 * DH && u < dh && kk < dh) v = hid(g, u, blk * dh + kk);
            BcT[(int64_t)k * NCP + n] = P::from_float(v);
            continue;
        }
        if (r < 4 * DH) {
            const int o = (int)(r / DH), u = (int)(r % DH);
            float v = 0.0f;
            if (u < dh) {
                if (o < 2) v = prm[L.Ua + (int64_t)o * dh + u];
                else if (d.cplx) v = prm[L.Up + (int64_t)(o - 2) * dh + u];
            }
            Hd[(int64_t)o * DH + u] = v;
        } else {
            const int o = (int)(r - 4 * DH);
            float v = 0.0f;
            if (o < 2) v = prm[L.ca + o];
            else if (d.cplx) v = prm[L.cp + o - 2];
            hc[o] = v;
        }
    }
}

// Facts of each order position q of the chain, one int4:
//   x = site | colw << 16   (colw: h(q) is the vertical input of a later,
//                            non-row-start position of its column)
//   y = site of the horizontal predecessor q-1 (-1 at a row start)
//   z = site of the vertical predecessor (2D, -1 in the first row)
//   w = (position of the vertical predecessor + 1) | column << 16
__global__ void build_postab(Dims d, int4 *tab) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.N) return;
    const int Lx = d.Lx, Ly = d.Ly;
    int site, shz, svt = -1, pvt = -1, icol, colw = 0;
    if (d.dims == 1) {
        site = q;
        shz = q > 0 ? q - 1 : -1;
        icol = q;
    } else {
        const int j = q / Lx, k = q - j * Lx;
        site = order_site(q, Lx);
        icol = site - j * Lx;
        shz = k > 0 ? order_site(q - 1, Lx) : -1;
        if (j > 0) {
            svt = site - Lx;
            pvt = site_pos(svt, Lx);
        }
        colw = (j + 1 < Ly) && ((q + 1) % Lx != 0);
    }
    tab[q] = make_int4(site | (colw << 16), shz, svt, (pvt + 1) | (icol << 16));
}

// --------------------------------------------------------- chain schedule

// first changed order position of connection c (list kinds)
__device__ inline int conn_first_pos(int kind, int c, int Lx, int Ly) {
    int sa, sc;
    conn_sites(kind, c, Lx, Ly, sa, sc);
    const int pa = site_pos(sa, Lx);
    if (sc < 0) return pa;
    const int pc = site_pos(sc, Lx);
    return pa < pc ? pa : pc;
}

// Per first-changed position p: capacity offsets of the connection list
// (list kinds: Heisenberg bonds, cluster terms) or the row counts (one flip
// per position: every sample, p < N-1), the zeroed counters, and the tile
// counter.
__global__ __launch_bounds__(1024) void sched_prep(int ham_kind, int Lx, int Ly, int64_t ns, int *cnt,
                                                   int *list_off, int *tile_counter) {
    // one work-group: connections counted per first changed position in LDS,
    // then one thread lays out the list offsets (N <= 1024)
    __shared__ int kb[1025];
    const int N = Lx * Ly, tid = threadIdx.x;
    if (tid == 0) *tile_counter = 0;
    if (ham_kind == 0) {
        for (int p = tid; p < N; p += blockDim.x) cnt[p] = (p < N - 1) ? (int)ns : 0;
        return;
    }
    for (int p = tid; p < N; p += blockDim.x) kb[p] = 0;
    __syncthreads();
    const int nb = conn_count(ham_kind, Lx, Ly);
    for (int b = tid; b < nb; b += blockDim.x) atomicAdd(&kb[conn_first_pos(ham_kind, b, Lx, Ly)], 1);
    __syncthreads();
    if (tid == 0) {
        int64_t off = 0;
        for (int p = 0; p < N; p++) {
            list_off[p] = (int)off;
            off += (int64_t)kb[p] * ns;
        }
        list_off[N] = (int)off;
    }
    for (int p = tid; p < N; p += blockDim.x) cnt[p] = 0;
}

// List kinds: every nonzero connection of every sample, filed under its
// first changed order position.  Heisenberg: the anti-aligned bonds (an
// aligned pair has no off-diagonal element, Eq. 7); cluster: every term (its
// off-diagonal element is +-J, never zero, Eq. 9).
__global__ void conn_list(int ham_kind, const uint8_t *cfg, int64_t ns, int Lx, int Ly, int *cnt,
                          const int *list_off, int *list) {
    const int nb = conn_count(ham_kind, Lx, Ly), N = Lx * Ly;
    const int64_t total = ns * nb;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int s = (int)(e / nb), b = (int)(e % nb);
        if (ham_kind == VMC_HEISENBERG) {
            int sa, sc;
            bond_sites(b, Lx, Ly, sa, sc);
            if (cfg[(int64_t)s * N + sa] == cfg[(int64_t)s * N + sc]) continue;
        }
        const int p = conn_first_pos(ham_kind, b, Lx, Ly);
        int slot = atomicAdd(&cnt[p], 1);
        list[list_off[p] + slot] = s * nb + b;
    }
}

// Tiles per position, longest suffix (smallest p) first.
__global__ __launch_bounds__(256) void tile_scan(int N, int MT, const int *cnt, int *tile_start) {
    // each thread a contiguous run of positions, then an exclusive scan of the
    // per-thread tile counts in LDS (the loads of all threads in flight at once)
    __shared__ int part[256];
    const int tid = threadIdx.x, NT = blockDim.x;
    const int per = (N + NT - 1) / NT, p0 = min(N, tid * per), p1 = min(N, p0 + per);
    int sum = 0;
    for (int p = p0; p < p1; p++) sum += (cnt[p] + MT - 1) / MT;
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < NT; o <<= 1) {
        const int v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int t = part[tid] - sum;
    for (int p = p0; p < p1; p++) {
        tile_start[p] = t;
        t += (cnt[p] + MT - 1) / MT;
    }
    if (tid == NT - 1) tile_start[N] = part[NT - 1];
}

// One queue over the chain tiles of a batch, longest chains first.  The
// problems come sorted by decreasing length (Ns[j] = length of problem
// ord[j]), so the problems whose chains reach length L (first changed
// position p = N - 1 - L) are a prefix of that order: the entries, one per
// (L, problem), run L = Lmax..1 and within each L over that prefix.  Entry
// e = {first tile, problem, p}; sched[E] = {total tiles}; the tile counter
// of the launch is reset.  One work-group.
struct BatchSort {
    int n;
    int ord[kMaxBatch], Ns[kMaxBatch];
};

__global__ __launch_bounds__(1024) void batch_scan(BatchSort bs, int MT, int64_t pitch_ws, const int *cnt0,
                                                   int4 *sched, int *counter, int E) {
    __shared__ int off[1025];   // first entry of length index i = Lmax - L
    __shared__ int part[1024];
    const int tid = threadIdx.x, NT = blockDim.x;
    const int Lmax = bs.Ns[0] - 1;
    for (int i = tid; i < Lmax; i += NT) {
        const int L = Lmax - i;
        int c = 0;
        while (c < bs.n && bs.Ns[c] - 1 >= L) c++;
        off[i + 1] = c;  // entries of length L, prefix-summed below
    }
    __syncthreads();
    if (tid == 0) {
        off[0] = 0;
        for (int i = 1; i <= Lmax; i++) off[i] += off[i - 1];
    }
    __syncthreads();
    // tile counts of this thread's contiguous range of entries, then a scan
    const int per = (E + NT - 1) / NT, e0 = tid * per, e1 = min(E, e0 + per);
    int sum = 0;
    for (int e = e0; e < e1; e++) {
        int lo = 0, hi = Lmax - 1;  // largest i with off[i] <= e
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int L = Lmax - lo, j = e - off[lo], k = bs.ord[j], p = bs.Ns[j] - 1 - L;
        const int *cnt = (const int *)((const char *)cnt0 + (int64_t)k * pitch_ws);
        const int nt = (cnt[p] + MT - 1) / MT;
        sched[e] = make_int4(nt, k, p, 0);
        sum += nt;
    }
    part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        int t = 0;
        for (int i = 0; i < NT; i++) {
            const int v = part[i];
            part[i] = t;
            t += v;
        }
        sched[E] = make_int4(t, -1, -1, 0);
        *counter = 0;
    }
    __syncthreads();
    int t = part[tid];
    for (int e = e0; e < e1; e++) {
        const int nt = sched[e].x;
        sched[e].x = t;
        t += nt;
    }
}

// E_loc assembly (Eqs. 6-9): diagonal part (bonds; all pairs for the
// long-range TFIM; none for the cluster state), off-diagonal part
// sum_k coupling * psi(sigma')/psi(sigma), where
//   log psi(sigma') - log psi(sigma) =
//       [lpc[p][sigma'_p] - lpc[p][sigma_p]]              (head at p)
//     + [chain sum after p] - [original sum after p]     (suffix)
// halved for |psi|; the original suffix sum is pre[N-1] - pre[p] (FP64).
// FP64 sums in a fixed order (see below).
__global__ __launch_bounds__(256) void eloc_assemble(int ham_kind, int marshall, int cplx, double J, double hx,
                                                     double alpha, int Lx, int Ly, int64_t ns, const uint8_t *cfg,
                                                     const float *lpc,
                                                     const float *phc, const double2 *pre, const double2 *dsuf, int NC,
                                                     double *eloc) {
    // 16 lanes per sample, each over every 16th connection (and bond of the
    // diagonal), then a fixed butterfly over the 16 lanes: lane 0's sum has
    // a fixed order, so the result is bitwise reproducible
    const int N = Lx * Ly, nb = bond_count(Lx, Ly), sub = threadIdx.x & 15;
    const int64_t step = ((int64_t)gridDim.x * blockDim.x) >> 4;
    for (int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4; s < ns; s += step) {
        const uint8_t *c = cfg + s * N;
        double diag = 0.0, ore = 0.0, oim = 0.0;
        if (ham_kind == VMC_LRTFIM) {
            // sum_{i<j} s_i s_j / |i-j|^alpha, by distance d (Eq. 8)
            for (int dd = 1 + sub; dd < N; dd += 16) {
                int agree = 0;
                for (int i = 0; i + dd < N; i++) agree += (c[i] == c[i + dd]) ? 1 : -1;
                diag += (double)agree * pow((double)dd, -alpha);
            }
        } else if (ham_kind != VMC_CLUSTER) {
            for (int b = sub; b < nb; b += 16) {
                int sa, sc;
                bond_sites(b, Lx, Ly, sa, sc);
                diag += (c[sa] == c[sc]) ? 1.0 : -1.0;
            }
        }
        const float *lr = lpc + s * N * 2, *pr = phc + s * N * 2;
        const double2 *pp = pre + s * N;
        const double2 tot = pp[N - 1];
        // psi(sigma')/psi(sigma) of the connection whose first changed order
        // position is p: the flipped conditional at p, then the chain's suffix
        auto ratio = [&](int p, double2 chain, double coef) {
            const int sg = c[order_site(p, Lx)];
            double dl = (double)lr[2 * p + (1 - sg)] - (double)lr[2 * p + sg];
            double dp = (double)pr[2 * p + (1 - sg)] - (double)pr[2 * p + sg];
            if (p < N - 1) {
                dl += chain.x - (tot.x - pp[p].x);
                dp += chain.y - (tot.y - pp[p].y);
            }
            const double mag = exp(0.5 * dl);
            if (cplx) {
                ore += coef * mag * cos(dp);
                oim += coef * mag * sin(dp);
            } else {
                ore += coef * mag;  // a positive RNN has no phase
            }
        };
        if (ham_kind == VMC_TFIM || ham_kind == VMC_LRTFIM) {
            for (int p = sub; p < N; p += 16) ratio(p, p < N - 1 ? dsuf[s * NC + p] : make_double2(0.0, 0.0), -hx);
        } else if (ham_kind == VMC_CLUSTER) {
            // -J times the Z eigenvalues of the term (1D: position = site)
            for (int t = sub; t < N; t += 16) {
                int f1, f2, z1, z2;
                cluster_term(t, N, f1, f2, z1, z2);
                double coef = -J;
                if (z1 >= 0 && c[z1]) coef = -coef;
                if (z2 >= 0 && c[z2]) coef = -coef;
                ratio(f2 >= 0 && f2 < f1 ? f2 : f1, dsuf[s * NC + t], coef);
            }
        } else {
            const double jx = (marshall ? -0.5 : 0.5) * J;
            for (int b = sub; b < nb; b += 16) {
                int sa, sc;
                bond_sites(b, Lx, Ly, sa, sc);
                if (c[sa] == c[sc]) continue;
                const int pa = site_pos(sa, Lx), pc = site_pos(sc, Lx);
                ratio(pa < pc ? pa : pc, dsuf[s * NC + b], jx);
            }
        }
#pragma unroll
        for (int m = 8; m >= 1; m >>= 1) {
            diag += __shfl_xor(diag, m, 16);
            ore += __shfl_xor(ore, m, 16);
            oim += __shfl_xor(oim, m, 16);
        }
        if (sub == 0) {
            const double dscale = ham_kind == VMC_HEISENBERG ? 0.25 * J : -J;
            eloc[2 * s] = (ham_kind == VMC_CLUSTER ? 0.0 : diag * dscale) + ore;
            eloc[2 * s + 1] = oim;
        }
    }
}

// ------------------------------------------------------------ launchers


int engine_kpx(const Dims &d);

hipError_t launch_stage(const Dims &d, const float *prm, void *Bc, void *BcT, void *Bg, void *BgT,
                        float *E, float *Hd, float *hc, int4 *postab, hipStream_t st) {
    hipLaunchKernelGGL(build_postab, dim3((d.N + 255) / 256), dim3(256), 0, st, d, postab);
    const int ks = d.prec == VMC_BF16 ? 32 : 16;
    const int KHB = cround(d.DH, ks), NCP = cround(3 * d.DH, ks), KPX = engine_kpx(d);
    const int NHB = d.dims == 1 ? 1 : 2;
    int64_t n = (int64_t)3 * d.DH * KPX + (int64_t)2 * d.DH * KHB + ESLOTS * d.DH + 4 * d.DH + 4 +
                (int64_t)NHB * d.DH * NCP;
    int grid = (int)((n + 255) / 256);
    if (grid > 4096) grid = 4096;
    if (d.prec == VMC_BF16)
        hipLaunchKernelGGL(stage_weights<BF16>, dim3(grid), dim3(256), 0, st, d, prm, (uint16_t *)Bc,
                           (uint16_t *)BcT, (uint16_t *)Bg, (uint16_t *)BgT, E, Hd, hc, KPX, KHB, NCP);
    else
        hipLaunchKernelGGL(stage_weights<F32>, dim3(grid), dim3(256), 0, st, d, prm, (float *)Bc,
                           (float *)BcT, (float *)Bg, (float *)BgT, E, Hd, hc, KPX, KHB, NCP);
    return hipGetLastError();
}

hipError_t launch_sched(int ham_kind, int Lx, int Ly, int64_t ns, const uint8_t *cfg, int *cnt,
                        int *list_off, int *list, int *tile_start, int *tile_counter, int MT,
                        hipStream_t st) {
    hipLaunchKernelGGL(sched_prep, dim3(1), dim3(1024), 0, st, ham_kind, Lx, Ly, ns, cnt, list_off, tile_counter);
    if (ham_kind != 0) {
        int64_t total = ns * conn_count(ham_kind, Lx, Ly);
        int grid = (int)((total + 255) / 256);
        if (grid > 8192) grid = 8192;
        if (grid < 1) grid = 1;
        hipLaunchKernelGGL(conn_list, dim3(grid), dim3(256), 0, st, ham_kind, cfg, ns, Lx, Ly, cnt, list_off, list);
    }
    hipLaunchKernelGGL(tile_scan, dim3(1), dim3(256), 0, st, Lx * Ly, MT, cnt, tile_start);
    return hipGetLastError();
}

// Entries of the batch queue: one per (problem, first changed position)
// with a chain after it, i.e. sum_k (N_k - 1).
hipError_t launch_batch_scan(const BatchInfo &bi, int MT, const int *cnt0, int4 *sched, int *counter,
                             hipStream_t st) {
    BatchSort bs;
    bs.n = bi.n;
    int E = 0;
    for (int k = 0; k < bi.n; k++) {
        bs.ord[k] = k;
        E += bi.N[k] - 1;
    }
    for (int a = 1; a < bi.n; a++)  // stable sort by decreasing length
        for (int b = a; b > 0 && bi.N[bs.ord[b]] > bi.N[bs.ord[b - 1]]; b--) {
            const int t = bs.ord[b];
            bs.ord[b] = bs.ord[b - 1];
            bs.ord[b - 1] = t;
        }
    for (int j = 0; j < bi.n; j++) bs.Ns[j] = bi.N[bs.ord[j]];
    if (E != bi.nsched) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_scan, dim3(1), dim3(1024), 0, st, bs, MT, bi.pitch_ws, cnt0, sched, counter, E);
    return hipGetLastError();
}

hipError_t launch_assemble(const vmc_ham &H, int cplx, int Lx, int Ly, int64_t ns, const uint8_t *cfg,
                           const float *lpc, const float *phc, const double2 *pre, const double2 *dsuf, int NC,
                           double *eloc, hipStream_t st) {
    int64_t g = (ns * 16 + 255) / 256;
    const int grid = (int)(g < 1 ? 1 : g > 65536 ? 65536 : g);
    hipLaunchKernelGGL(eloc_assemble, dim3(grid), dim3(256), 0, st, H.kind, H.marshall, cplx, H.J, H.h, H.alpha, Lx,
                       Ly, ns, cfg, lpc, phc, pre, dsuf, NC, eloc);
    return hipGetLastError();
}

}  // namespace vmc
