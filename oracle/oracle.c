/*
 * FP64 CPU oracle for the variational-Monte-Carlo hot path of GRU RNN wave
 * functions (McNaughton & Hibat-Allah, "Adaptive Neural Quantum States: A
 * Recurrent Neural Network Perspective", arXiv 2507.18700).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file: only the tests, the smoke check and the CPU-baseline leg of the bench
 * use it.  It shares no code, header, table or helper with the HIP library.
 *
 * Plain loops in double precision, no BLAS, no blocking, no prefix reuse:
 * every connected configuration of the local energy is re-evaluated from the
 * first site.  Each function names the passage of the paper it follows.
 *
 * Conventions (readings where the paper is silent; listed in the design notes):
 *  - sigma_n in {0,1}; one-hot(0)=(1,0), one-hot(1)=(0,1); the spin value used
 *    by the Hamiltonians is s = 1 - 2*sigma (sigma=0 <-> s=+1).
 *  - h_0 = 0 and sigma_0 = (0,0) (Sec. II A, vanilla-RNN recursion, Eq. (2)).
 *  - 2D: site (i,j), column i in [0,Lx), row j in [0,Ly), lattice index j*Lx+i;
 *    zig-zag order: even rows left->right, odd rows right->left; horizontal
 *    predecessor (i-(-1)^j, j), vertical predecessor (i, j-1) (Sec. II A and
 *    App. A); a missing neighbour contributes h=0 and one-hot (0,0).
 *  - The phase head has its own weights (U_p, c_p), separate from the
 *    amplitude head (U_a, c_a) of Eq. (3); Eq. (5) reuses the symbols.
 *  - GLU (App. A) is optional in both 1D and 2D; d_model = d_h.
 *
 * Parameter layout (row-major [out][in], in this order):
 *  1D (App. A, GRU of Cho et al.):
 *     W_g [dh][dh+2], b_g[dh], W_r [dh][dh+2], b_r[dh],
 *     W_h [dh][dh],   b_h[dh], W_in[dh][2],    b_in[dh]
 *     input order of the gate matrices: [h_{n-1}; onehot(sigma_{n-1})]
 *  2D (App. A, 2D GRU):
 *     W [dh][2dh+4], b[dh], W_g[dh][2dh+4], b_g[dh], U[dh][2dh]
 *     input order: [h_hz; h_vt; onehot_hz; onehot_vt]
 *  GLU (App. A): W_1[dh][dh], b_1[dh], W_2[dh][dh], b_2[dh]
 *  amplitude head (Eq. (3)): U_a[2][dh], c_a[2]
 *  phase head (Eq. (5), complex RNN only): U_p[2][dh], c_p[2]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t dims;       /* 1 or 2 */
    int32_t Lx, Ly;     /* N = Lx*Ly; 1D uses Ly = 1 */
    int32_t d_h;        /* hidden width, d_model = d_h */
    int32_t is_complex; /* complex RNN: softsign phase head */
    int32_t glu;        /* GLU before the heads */
    int32_t bf16;       /* round GEMM operands to bfloat16 (emulation mode) */
} ora_model;

typedef struct {
    int32_t kind;       /* 0 = transverse-field Ising, 1 = Heisenberg,
                           2 = long-range transverse-field Ising, 3 = cluster */
    int32_t marshall;   /* Heisenberg: rotate by the Marshall sign */
    double J, h;        /* coupling, transverse field */
    double alpha;       /* long-range exponent (kind 2) */
} ora_ham;

typedef struct {
    int dh, N;
    long Wg, bg, Wr, br, Wh, bh, Win, bin; /* 1D */
    long W, b, U;                          /* 2D (W_g, b_g shared names) */
    long W1, b1, W2, b2;                   /* GLU */
    long Ua, ca, Up, cp;                   /* heads */
    long total;
} layout;

static void make_layout(const ora_model *m, layout *L)
{
    int d = m->d_h;
    long o = 0;
    memset(L, 0, sizeof(*L));
    L->dh = d;
    L->N = m->Lx * m->Ly;
    if (m->dims == 1) {
        L->Wg = o; o += (long)d * (d + 2);
        L->bg = o; o += d;
        L->Wr = o; o += (long)d * (d + 2);
        L->br = o; o += d;
        L->Wh = o; o += (long)d * d;
        L->bh = o; o += d;
        L->Win = o; o += (long)d * 2;
        L->bin = o; o += d;
    } else {
        L->W = o; o += (long)d * (2 * d + 4);
        L->b = o; o += d;
        L->Wg = o; o += (long)d * (2 * d + 4);
        L->bg = o; o += d;
        L->U = o; o += (long)d * 2 * d;
    }
    if (m->glu) {
        L->W1 = o; o += (long)d * d;
        L->b1 = o; o += d;
        L->W2 = o; o += (long)d * d;
        L->b2 = o; o += d;
    }
    L->Ua = o; o += 2L * d;
    L->ca = o; o += 2;
    if (m->is_complex) {
        L->Up = o; o += 2L * d;
        L->cp = o; o += 2;
    }
    L->total = o;
}

int64_t ora_param_count(const ora_model *m)
{
    layout L;
    make_layout(m, &L);
    return L.total;
}

/* ---------------------------------------------------------------- helpers */

static double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Round to the nearest bfloat16 (8 significant bits), ties to even, by way of
 * binary32 as a GPU does when it converts a float operand. */
static double to_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return x; /* inf / nan untouched */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double opnd(const ora_model *m, double x) { return m->bf16 ? to_bf16(x) : x; }

/* order position n -> lattice site, and the lattice coordinates */
static int order_site(const ora_model *m, int n, int *pi, int *pj)
{
    int j = n / m->Lx, k = n % m->Lx;
    int i = (j % 2 == 0) ? k : m->Lx - 1 - k;
    if (pi) *pi = i;
    if (pj) *pj = j;
    return j * m->Lx + i;
}

/* ---------------------------------------------------------- forward trace */

/* Everything the backward sweep needs, per order position. */
typedef struct {
    int N, dh, K;
    double *hz, *vt;   /* [N][dh] hidden inputs (1D: hz = h_{n-1}, vt unused) */
    int *xz, *xv;      /* [N] one-hot class of each input neighbour, -1 = absent */
    int *phz, *pvt;    /* [N] order position of the predecessors, -1 = absent */
    double *u, *r, *mm, *c, *v, *h;   /* [N][dh] gates, candidate, U h', h */
    double *a1, *a2, *g;              /* [N][dh] GLU */
    double *l, *z;                    /* [N][2] amplitude and phase logits */
} trace;

static void trace_alloc(trace *t, int N, int dh)
{
    size_t nd = (size_t)N * dh;
    t->N = N;
    t->dh = dh;
    t->hz = calloc(nd, sizeof(double));
    t->vt = calloc(nd, sizeof(double));
    t->u = calloc(nd, sizeof(double));
    t->r = calloc(nd, sizeof(double));
    t->mm = calloc(nd, sizeof(double));
    t->c = calloc(nd, sizeof(double));
    t->v = calloc(nd, sizeof(double));
    t->h = calloc(nd, sizeof(double));
    t->a1 = calloc(nd, sizeof(double));
    t->a2 = calloc(nd, sizeof(double));
    t->g = calloc(nd, sizeof(double));
    t->l = calloc((size_t)N * 2, sizeof(double));
    t->z = calloc((size_t)N * 2, sizeof(double));
    t->xz = calloc(N, sizeof(int));
    t->xv = calloc(N, sizeof(int));
    t->phz = calloc(N, sizeof(int));
    t->pvt = calloc(N, sizeof(int));
}

static void trace_free(trace *t)
{
    free(t->hz); free(t->vt); free(t->u); free(t->r); free(t->mm); free(t->c);
    free(t->v); free(t->h); free(t->a1); free(t->a2); free(t->g); free(t->l);
    free(t->z); free(t->xz); free(t->xv); free(t->phz); free(t->pvt);
}

/* One 1D GRU step (App. A, standard GRU of Cho et al.):
 *   u = sig(W_g [h;x] + b_g), r = sig(W_r [h;x] + b_r),
 *   c = tanh(r (.) (W_h h + b_h) + W_in x + b_in),  h' = (1-u) (.) h + u (.) c */
static void cell1d(const ora_model *m, const layout *L, const double *P, const double *hp,
                   int x, double *u, double *r, double *mm, double *c, double *hn)
{
    int d = L->dh, K = d + 2;
    for (int a = 0; a < d; a++) {
        double su = P[L->bg + a], sr = P[L->br + a], sm = P[L->bh + a], sx = P[L->bin + a];
        for (int k = 0; k < d; k++) {
            double hk = opnd(m, hp[k]);
            su += opnd(m, P[L->Wg + (long)a * K + k]) * hk;
            sr += opnd(m, P[L->Wr + (long)a * K + k]) * hk;
            sm += opnd(m, P[L->Wh + (long)a * d + k]) * hk;
        }
        if (x >= 0) {
            su += P[L->Wg + (long)a * K + d + x];
            sr += P[L->Wr + (long)a * K + d + x];
            sx += P[L->Win + (long)a * 2 + x];
        }
        u[a] = sigm(su);
        r[a] = sigm(sr);
        mm[a] = sm;
        c[a] = tanh(r[a] * sm + sx);
    }
    for (int a = 0; a < d; a++) hn[a] = (1.0 - u[a]) * hp[a] + u[a] * c[a];
}

/* One 2D GRU step (App. A, 2D GRU):
 *   c = tanh(W [h';s'] + b), u = sig(W_g [h';s'] + b_g),
 *   h = u (.) c + (1-u) (.) (U h'),  h' = [h_hz; h_vt], s' = [x_hz; x_vt] */
static void cell2d(const ora_model *m, const layout *L, const double *P, const double *hz,
                   const double *hv, int xz, int xv, double *u, double *c, double *v, double *hn)
{
    int d = L->dh, K = 2 * d + 4;
    for (int a = 0; a < d; a++) {
        double sc = P[L->b + a], su = P[L->bg + a], sv = 0.0;
        for (int k = 0; k < d; k++) {
            double z1 = opnd(m, hz[k]), z2 = opnd(m, hv[k]);
            sc += opnd(m, P[L->W + (long)a * K + k]) * z1 + opnd(m, P[L->W + (long)a * K + d + k]) * z2;
            su += opnd(m, P[L->Wg + (long)a * K + k]) * z1 + opnd(m, P[L->Wg + (long)a * K + d + k]) * z2;
            sv += opnd(m, P[L->U + (long)a * 2 * d + k]) * z1 + opnd(m, P[L->U + (long)a * 2 * d + d + k]) * z2;
        }
        if (xz >= 0) {
            sc += P[L->W + (long)a * K + 2 * d + xz];
            su += P[L->Wg + (long)a * K + 2 * d + xz];
        }
        if (xv >= 0) {
            sc += P[L->W + (long)a * K + 2 * d + 2 + xv];
            su += P[L->Wg + (long)a * K + 2 * d + 2 + xv];
        }
        c[a] = tanh(sc);
        u[a] = sigm(su);
        v[a] = sv;
    }
    for (int a = 0; a < d; a++) hn[a] = u[a] * c[a] + (1.0 - u[a]) * v[a];
}

/* GLU before the heads (App. A): g = (W_1 h + b_1) (.) sig(W_2 h + b_2);
 * the heads: amplitude logits l = U_a g + c_a (Eq. (3)), phase logits
 * z = U_p g + c_p (Eq. (5)).  Heads are evaluated in full precision. */
static void heads(const ora_model *m, const layout *L, const double *P, const double *h,
                  double *a1, double *a2, double *g, double *l, double *z)
{
    int d = L->dh;
    const double *src = h;
    if (m->glu) {
        for (int a = 0; a < d; a++) {
            double s1 = P[L->b1 + a], s2 = P[L->b2 + a];
            for (int k = 0; k < d; k++) {
                double hk = opnd(m, h[k]);
                s1 += opnd(m, P[L->W1 + (long)a * d + k]) * hk;
                s2 += opnd(m, P[L->W2 + (long)a * d + k]) * hk;
            }
            a1[a] = s1;
            a2[a] = s2;
            g[a] = s1 * sigm(s2);
        }
        src = g;
    } else {
        for (int a = 0; a < d; a++) g[a] = h[a];
    }
    for (int o = 0; o < 2; o++) {
        double s = P[L->ca + o];
        for (int k = 0; k < d; k++) s += P[L->Ua + (long)o * d + k] * src[k];
        l[o] = s;
    }
    if (m->is_complex) {
        for (int o = 0; o < 2; o++) {
            double s = P[L->cp + o];
            for (int k = 0; k < d; k++) s += P[L->Up + (long)o * d + k] * src[k];
            z[o] = s;
        }
    } else {
        z[0] = z[1] = 0.0;
    }
}

/* log-softmax of a 2-vector, both entries (Eq. (3)) */
static void logsoftmax2(const double *l, double *out)
{
    double mx = l[0] > l[1] ? l[0] : l[1];
    double lse = mx + log(exp(l[0] - mx) + exp(l[1] - mx));
    out[0] = l[0] - lse;
    out[1] = l[1] - lse;
}

static double softsign(double x) { return x / (1.0 + fabs(x)); }

/*
 * Autoregressive evaluation of one configuration along the sampling order
 * (chain rule, Eq. (1); conditionals, Eq. (3); phase, Eqs. (4)-(5)).
 * If `uni` is non-NULL the spins are drawn instead of read: at order position
 * n, sigma = 0 when uni[n] < P(sigma=0 | sigma_<n), else 1 (perfect
 * autoregressive sampling, Sec. II A).  Writes sigma back in lattice order.
 * lpc/phc (optional): per order position, log P(sigma_n = 0/1 | .) and
 * pi*softsign(z)[0/1].
 */
static void forward_one(const ora_model *m, const layout *L, const double *P, uint8_t *cfg,
                        const double *uni, double *logp, double *phase, double *lpc, double *phc,
                        trace *t)
{
    int N = L->N, d = L->dh;
    double *hbuf = calloc((size_t)N * d, sizeof(double)); /* h per order position */
    double *zero = calloc(d, sizeof(double));
    double *u = malloc(d * sizeof(double)), *r = malloc(d * sizeof(double));
    double *mm = malloc(d * sizeof(double)), *c = malloc(d * sizeof(double));
    double *v = malloc(d * sizeof(double));
    double *a1 = malloc(d * sizeof(double)), *a2 = malloc(d * sizeof(double));
    double *g = malloc(d * sizeof(double));
    int *pos_of = malloc(N * sizeof(int));
    double lp = 0.0, ph = 0.0;

    for (int n = 0; n < N; n++) pos_of[order_site(m, n, NULL, NULL)] = n;

    for (int n = 0; n < N; n++) {
        int i, j;
        int site = order_site(m, n, &i, &j);
        const double *hz, *hv = zero;
        int xz = -1, xv = -1, phz = -1, pvt = -1;
        double *hn = hbuf + (size_t)n * d;
        if (m->dims == 1) {
            if (n > 0) { phz = n - 1; xz = cfg[n - 1]; }
            hz = phz >= 0 ? hbuf + (size_t)phz * d : zero;
            cell1d(m, L, P, hz, xz, u, r, mm, c, hn);
        } else {
            int ih = (j % 2 == 0) ? i - 1 : i + 1; /* i - (-1)^j */
            if (ih >= 0 && ih < m->Lx) {
                int s2 = j * m->Lx + ih;
                phz = pos_of[s2];
                xz = cfg[s2];
            }
            if (j > 0) {
                int s2 = (j - 1) * m->Lx + i;
                pvt = pos_of[s2];
                xv = cfg[s2];
            }
            hz = phz >= 0 ? hbuf + (size_t)phz * d : zero;
            hv = pvt >= 0 ? hbuf + (size_t)pvt * d : zero;
            cell2d(m, L, P, hz, hv, xz, xv, u, c, v, hn);
        }
        double l[2], z[2], ls[2];
        heads(m, L, P, hn, a1, a2, g, l, z);
        logsoftmax2(l, ls);
        if (uni) cfg[site] = (uni[n] < exp(ls[0])) ? 0 : 1;
        int sg = cfg[site];
        lp += ls[sg];
        if (m->is_complex) ph += M_PI * softsign(z[sg]);
        if (lpc) { lpc[2 * n] = ls[0]; lpc[2 * n + 1] = ls[1]; }
        if (phc) {
            phc[2 * n] = m->is_complex ? M_PI * softsign(z[0]) : 0.0;
            phc[2 * n + 1] = m->is_complex ? M_PI * softsign(z[1]) : 0.0;
        }
        if (t) {
            memcpy(t->hz + (size_t)n * d, hz, d * sizeof(double));
            memcpy(t->vt + (size_t)n * d, hv, d * sizeof(double));
            t->xz[n] = xz; t->xv[n] = xv; t->phz[n] = phz; t->pvt[n] = pvt;
            memcpy(t->u + (size_t)n * d, u, d * sizeof(double));
            memcpy(t->c + (size_t)n * d, c, d * sizeof(double));
            memcpy(t->h + (size_t)n * d, hn, d * sizeof(double));
            if (m->dims == 1) {
                memcpy(t->r + (size_t)n * d, r, d * sizeof(double));
                memcpy(t->mm + (size_t)n * d, mm, d * sizeof(double));
            } else {
                memcpy(t->v + (size_t)n * d, v, d * sizeof(double));
            }
            memcpy(t->a1 + (size_t)n * d, a1, d * sizeof(double));
            memcpy(t->a2 + (size_t)n * d, a2, d * sizeof(double));
            memcpy(t->g + (size_t)n * d, g, d * sizeof(double));
            t->l[2 * n] = l[0]; t->l[2 * n + 1] = l[1];
            t->z[2 * n] = z[0]; t->z[2 * n + 1] = z[1];
        }
    }
    if (logp) *logp = lp;
    if (phase) *phase = ph;
    free(hbuf); free(zero); free(u); free(r); free(mm); free(c); free(v);
    free(a1); free(a2); free(g); free(pos_of);
}

/* --------------------------------------------------------------- log psi */

/* log P(sigma) and phi(sigma) of nc configurations (lattice order, [nc][N]).
 * log psi = logP/2 + i*phi (Eq. (4)).  lpc/phc: optional [nc][N][2]. */
void ora_logpsi(const ora_model *m, const double *P, int64_t nc, const uint8_t *cfg,
                double *logp, double *phase, double *lpc, double *phc)
{
    layout L;
    make_layout(m, &L);
    int N = L.N;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nc; s++) {
        uint8_t *c = malloc(N);
        memcpy(c, cfg + s * N, N);
        forward_one(m, &L, P, c, NULL, logp ? logp + s : NULL, phase ? phase + s : NULL,
                    lpc ? lpc + s * 2 * N : NULL, phc ? phc + s * 2 * N : NULL, NULL);
        free(c);
    }
}

/* Autoregressive sampling (Sec. II A) driven by the given uniforms
 * uni[ns][N], indexed by sample and order position. */
void ora_sample(const ora_model *m, const double *P, int64_t ns, const double *uni,
                uint8_t *cfg, double *logp, double *phase)
{
    layout L;
    make_layout(m, &L);
    int N = L.N;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < ns; s++) {
        memset(cfg + s * N, 0, N);
        forward_one(m, &L, P, cfg + s * N, uni + s * N, logp ? logp + s : NULL,
                    phase ? phase + s : NULL, NULL, NULL, NULL);
    }
}

/* ------------------------------------------------------------ Philox 4x32 */

/* Philox-4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11): per round, two 32x32->64 products
 * with the multipliers 0xD2511F53 and 0xCD9E8D57, an xor with the round key,
 * and a key bump by the Weyl constants 0x9E3779B9 and 0xBB67AE85. */
void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Sampling uniforms from Philox: u[s][n] = (word (n mod 4) of
 * Philox(key=seed, ctr={n/4, s, counter_lo, counter_hi}) >> 8) * 2^-24,
 * a 24-bit uniform in [0,1). */
void ora_philox_uniforms(uint64_t seed, uint64_t counter, int64_t ns, int32_t N, double *u)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t s = 0; s < ns; s++) {
        for (int n = 0; n < N; n++) {
            uint32_t ctr[4] = {(uint32_t)(n / 4), (uint32_t)s, (uint32_t)counter,
                               (uint32_t)(counter >> 32)};
            uint32_t o[4];
            ora_philox4x32_10(ctr, key, o);
            u[s * N + n] = (double)(o[n % 4] >> 8) * (1.0 / 16777216.0);
        }
    }
}

/* ---------------------------------------------------------- local energy */

/* Nearest-neighbour bonds with open boundaries, in a fixed order: for each
 * site j*Lx+i in lattice order, the bond to (i+1, j) then to (i, j+1). */
static int make_bonds(const ora_model *m, int *ba, int *bb)
{
    int nb = 0;
    for (int j = 0; j < m->Ly; j++)
        for (int i = 0; i < m->Lx; i++) {
            int a = j * m->Lx + i;
            if (i + 1 < m->Lx) { ba[nb] = a; bb[nb] = a + 1; nb++; }
            if (j + 1 < m->Ly) { ba[nb] = a; bb[nb] = a + m->Lx; nb++; }
        }
    return nb;
}

int32_t ora_bond_count(const ora_model *m)
{
    return (m->Lx - 1) * m->Ly + m->Lx * (m->Ly - 1);
}

/*
 * The 1D cluster Hamiltonian of Eq. (9), sites 1..n as the paper numbers them:
 *   H = -sum_{k=2}^{n-2} X_{k-1} Z_k X_{k+1} - Z_1 X_2 - X_{n-1} X_n
 *       - X_{n-2} Z_{n-1} Z_n,
 * stored as Pauli strings: for term t, the 0-indexed sites acted on by X
 * (xs, nx of them) and by Z (zs, nz).  Returns the number of terms.
 */
typedef struct {
    int nx, nz;
    int xs[2], zs[2];
} pauli_term;

static int cluster_terms(int n, pauli_term *T)
{
    int nt = 0;
    for (int k = 2; k <= n - 2; k++) { /* X_{k-1} Z_k X_{k+1} */
        pauli_term t = {2, 1, {k - 2, k}, {k - 1, 0}};
        T[nt++] = t;
    }
    pauli_term a = {1, 1, {1, 0}, {0, 0}};                 /* Z_1 X_2 */
    pauli_term b = {2, 0, {n - 2, n - 1}, {0, 0}};         /* X_{n-1} X_n */
    pauli_term c = {1, 2, {n - 3, 0}, {n - 2, n - 1}};     /* X_{n-2} Z_{n-1} Z_n */
    T[nt++] = a;
    T[nt++] = b;
    T[nt++] = c;
    return nt;
}

/*
 * Local energy E_loc(sigma) = sum_sigma' H_{sigma,sigma'} psi(sigma')/psi(sigma)
 * with every connected configuration sigma' re-evaluated in full.
 *  Transverse-field Ising (Eq. (6); on the square lattice for 2D):
 *    E_loc = -J sum_<ab> s_a s_b - h sum_k psi(sigma^(k))/psi(sigma)
 *  Heisenberg (Eq. (7)), H = J/4 sum_<ab> sigma.sigma:
 *    E_loc = J/4 sum_<ab> s_a s_b + sum_{<ab>: s_a != s_b} Jx psi(sigma^(ab))/psi(sigma)
 *    with Jx = +J/2, or -J/2 after the Marshall-sign rotation, which makes
 *    every off-diagonal element negative (Sec. III B).
 *  Long-range transverse-field Ising (Eq. (8), chain):
 *    E_loc = -J sum_{i<j} s_i s_j / |i-j|^alpha - h sum_k psi(sigma^(k))/psi(sigma)
 *  Cluster state (Eq. (9), chain; scaled by J): every term is a Pauli string
 *    of X and Z on distinct sites, so <sigma|term|sigma'> = prod_Z s_z with
 *    sigma' = sigma flipped on the X sites, and
 *    E_loc = -J sum_terms (prod_Z s_z) psi(sigma')/psi(sigma).
 * eloc[2s], eloc[2s+1] = real and imaginary part.
 */
void ora_local_energy(const ora_model *m, const double *P, const ora_ham *H, int64_t ns,
                      const uint8_t *cfg, double *eloc)
{
    layout L;
    make_layout(m, &L);
    int N = L.N;
    int nbmax = 2 * N + 2;
    int *ba = malloc(nbmax * sizeof(int)), *bb = malloc(nbmax * sizeof(int));
    int nb = make_bonds(m, ba, bb);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < ns; s++) {
        const uint8_t *c0 = cfg + s * N;
        uint8_t *c1 = malloc(N);
        double lp0, ph0, lp1, ph1;
        forward_one(m, &L, P, (uint8_t *)memcpy(c1, c0, N), NULL, &lp0, &ph0, NULL, NULL, NULL);
        double diag = 0.0, ore = 0.0, oim = 0.0;
        for (int b = 0; b < nb; b++) {
            double sa = 1.0 - 2.0 * c0[ba[b]], sb = 1.0 - 2.0 * c0[bb[b]];
            diag += sa * sb;
        }
        if (H->kind == 2) {
            diag = 0.0;
            for (int i = 0; i < N; i++)
                for (int j = i + 1; j < N; j++) {
                    double si = 1.0 - 2.0 * c0[i], sj = 1.0 - 2.0 * c0[j];
                    diag -= H->J * si * sj / pow((double)(j - i), H->alpha);
                }
            for (int k = 0; k < N; k++) {
                memcpy(c1, c0, N);
                c1[k] ^= 1;
                forward_one(m, &L, P, c1, NULL, &lp1, &ph1, NULL, NULL, NULL);
                double mag = exp(0.5 * (lp1 - lp0));
                ore += -H->h * mag * cos(ph1 - ph0);
                oim += -H->h * mag * sin(ph1 - ph0);
            }
        } else if (H->kind == 3) {
            pauli_term *T = malloc((size_t)(N + 3) * sizeof(pauli_term));
            int nt = cluster_terms(N, T);
            diag = 0.0;
            for (int t = 0; t < nt; t++) {
                double coef = -H->J;
                for (int z = 0; z < T[t].nz; z++) coef *= 1.0 - 2.0 * c0[T[t].zs[z]];
                memcpy(c1, c0, N);
                for (int x = 0; x < T[t].nx; x++) c1[T[t].xs[x]] ^= 1;
                forward_one(m, &L, P, c1, NULL, &lp1, &ph1, NULL, NULL, NULL);
                double mag = exp(0.5 * (lp1 - lp0));
                ore += coef * mag * cos(ph1 - ph0);
                oim += coef * mag * sin(ph1 - ph0);
            }
            free(T);
        } else if (H->kind == 0) {
            diag *= -H->J;
            for (int k = 0; k < N; k++) {
                memcpy(c1, c0, N);
                c1[k] ^= 1;
                forward_one(m, &L, P, c1, NULL, &lp1, &ph1, NULL, NULL, NULL);
                double mag = exp(0.5 * (lp1 - lp0));
                ore += -H->h * mag * cos(ph1 - ph0);
                oim += -H->h * mag * sin(ph1 - ph0);
            }
        } else {
            diag *= 0.25 * H->J;
            double jx = (H->marshall ? -0.5 : 0.5) * H->J;
            for (int b = 0; b < nb; b++) {
                if (c0[ba[b]] == c0[bb[b]]) continue;
                memcpy(c1, c0, N);
                c1[ba[b]] ^= 1;
                c1[bb[b]] ^= 1;
                forward_one(m, &L, P, c1, NULL, &lp1, &ph1, NULL, NULL, NULL);
                double mag = exp(0.5 * (lp1 - lp0));
                ore += jx * mag * cos(ph1 - ph0);
                oim += jx * mag * sin(ph1 - ph0);
            }
        }
        eloc[2 * s] = diag + ore;
        eloc[2 * s + 1] = oim;
        free(c1);
    }
    free(ba);
    free(bb);
}

/* ------------------------------------------------------------ statistics */

/* Energy statistics (Sec. III, Tables I-II): with weights w_s (NULL: 1/ns),
 * Ebar = sum_s w_s E_s (complex), var = sum_s w_s |E_s - Ebar|^2.
 * stats = {Re Ebar, Im Ebar, var, number of non-finite E_s}. */
void ora_stats(int64_t ns, const double *eloc, const double *w, double *stats)
{
    double er = 0.0, ei = 0.0, var = 0.0, bad = 0.0;
    for (int64_t s = 0; s < ns; s++) {
        double ws = w ? w[s] : 1.0 / (double)ns;
        if (!isfinite(eloc[2 * s]) || !isfinite(eloc[2 * s + 1])) bad += 1.0;
        er += ws * eloc[2 * s];
        ei += ws * eloc[2 * s + 1];
    }
    for (int64_t s = 0; s < ns; s++) {
        double ws = w ? w[s] : 1.0 / (double)ns;
        double dr = eloc[2 * s] - er, di = eloc[2 * s + 1] - ei;
        var += ws * (dr * dr + di * di);
    }
    stats[0] = er;
    stats[1] = ei;
    stats[2] = var;
    stats[3] = bad;
}

/* ------------------------------------------------------------- gradient */

/*
 * Reverse-mode derivative of one sample's L = a*logP(sigma) + b*phi(sigma)
 * through the autoregressive chain, added into grad.  A plain backward sweep
 * over the order positions, last to first: each position receives the
 * gradient of its hidden state from its own heads and from the one or two
 * cells that consumed it (horizontal and vertical successor in 2D).
 */
static void backward_one(const ora_model *m, const layout *L, const double *P, const uint8_t *cfg,
                         double a, double b, double *grad)
{
    int N = L->N, d = L->dh;
    trace t;
    trace_alloc(&t, N, d);
    uint8_t *c = malloc(N);
    memcpy(c, cfg, N);
    forward_one(m, L, P, c, NULL, NULL, NULL, NULL, NULL, &t);

    double *dh = calloc((size_t)N * d, sizeof(double)); /* dL/dh per order position */
    double *dg = malloc(d * sizeof(double)), *dhn = malloc(d * sizeof(double));
    double *dac = malloc(d * sizeof(double)), *dau = malloc(d * sizeof(double));
    double *dar = malloc(d * sizeof(double)), *dm = malloc(d * sizeof(double));
    double *dv = malloc(d * sizeof(double));

    for (int n = N - 1; n >= 0; n--) {
        int site = order_site(m, n, NULL, NULL);
        int sg = c[site];
        const double *g = t.g + (size_t)n * d, *h = t.h + (size_t)n * d;
        /* amplitude head: d logsoftmax(l)[sg] / dl = onehot(sg) - softmax(l) */
        double ls[2];
        logsoftmax2(t.l + 2 * n, ls);
        double dl[2] = {a * ((sg == 0) - exp(ls[0])), a * ((sg == 1) - exp(ls[1]))};
        double dz[2] = {0.0, 0.0};
        if (m->is_complex) {
            double zz = t.z[2 * n + sg];
            double den = 1.0 + fabs(zz);
            dz[sg] = b * M_PI / (den * den); /* d softsign(x)/dx = 1/(1+|x|)^2 */
        }
        for (int k = 0; k < d; k++) {
            double s = 0.0;
            for (int o = 0; o < 2; o++) {
                s += P[L->Ua + (long)o * d + k] * dl[o];
                grad[L->Ua + (long)o * d + k] += dl[o] * g[k];
                if (m->is_complex) {
                    s += P[L->Up + (long)o * d + k] * dz[o];
                    grad[L->Up + (long)o * d + k] += dz[o] * g[k];
                }
            }
            dg[k] = s;
        }
        for (int o = 0; o < 2; o++) {
            grad[L->ca + o] += dl[o];
            if (m->is_complex) grad[L->cp + o] += dz[o];
        }
        /* GLU */
        for (int k = 0; k < d; k++) dhn[k] = dh[(size_t)n * d + k];
        if (m->glu) {
            const double *a1 = t.a1 + (size_t)n * d, *a2 = t.a2 + (size_t)n * d;
            for (int q = 0; q < d; q++) {
                double sg2 = sigm(a2[q]);
                double d1 = dg[q] * sg2;
                double d2 = dg[q] * a1[q] * sg2 * (1.0 - sg2);
                grad[L->b1 + q] += d1;
                grad[L->b2 + q] += d2;
                for (int k = 0; k < d; k++) {
                    grad[L->W1 + (long)q * d + k] += d1 * h[k];
                    grad[L->W2 + (long)q * d + k] += d2 * h[k];
                    dhn[k] += P[L->W1 + (long)q * d + k] * d1 + P[L->W2 + (long)q * d + k] * d2;
                }
            }
        } else {
            for (int k = 0; k < d; k++) dhn[k] += dg[k];
        }
        const double *u = t.u + (size_t)n * d, *cc = t.c + (size_t)n * d;
        const double *hz = t.hz + (size_t)n * d, *hv = t.vt + (size_t)n * d;
        int xz = t.xz[n], xv = t.xv[n], phz = t.phz[n], pvt = t.pvt[n];
        if (m->dims == 1) {
            int K = d + 2;
            const double *r = t.r + (size_t)n * d, *mm = t.mm + (size_t)n * d;
            double *dprev = phz >= 0 ? dh + (size_t)phz * d : NULL;
            for (int q = 0; q < d; q++) {
                /* h' = (1-u) h + u c */
                double du = dhn[q] * (cc[q] - hz[q]);
                double dc = dhn[q] * u[q];
                dac[q] = dc * (1.0 - cc[q] * cc[q]);
                dar[q] = dac[q] * mm[q] * r[q] * (1.0 - r[q]);
                dm[q] = dac[q] * r[q];
                dau[q] = du * u[q] * (1.0 - u[q]);
                if (dprev) dprev[q] += dhn[q] * (1.0 - u[q]);
            }
            for (int q = 0; q < d; q++) {
                grad[L->bg + q] += dau[q];
                grad[L->br + q] += dar[q];
                grad[L->bh + q] += dm[q];
                grad[L->bin + q] += dac[q];
                for (int k = 0; k < d; k++) {
                    grad[L->Wg + (long)q * K + k] += dau[q] * hz[k];
                    grad[L->Wr + (long)q * K + k] += dar[q] * hz[k];
                    grad[L->Wh + (long)q * d + k] += dm[q] * hz[k];
                    if (dprev)
                        dprev[k] += P[L->Wg + (long)q * K + k] * dau[q] +
                                    P[L->Wr + (long)q * K + k] * dar[q] +
                                    P[L->Wh + (long)q * d + k] * dm[q];
                }
                if (xz >= 0) {
                    grad[L->Wg + (long)q * K + d + xz] += dau[q];
                    grad[L->Wr + (long)q * K + d + xz] += dar[q];
                    grad[L->Win + (long)q * 2 + xz] += dac[q];
                }
            }
        } else {
            int K = 2 * d + 4;
            const double *v = t.v + (size_t)n * d;
            double *dprev_hz = phz >= 0 ? dh + (size_t)phz * d : NULL;
            double *dprev_vt = pvt >= 0 ? dh + (size_t)pvt * d : NULL;
            for (int q = 0; q < d; q++) {
                /* h = u c + (1-u) v */
                double du = dhn[q] * (cc[q] - v[q]);
                double dc = dhn[q] * u[q];
                dv[q] = dhn[q] * (1.0 - u[q]);
                dac[q] = dc * (1.0 - cc[q] * cc[q]);
                dau[q] = du * u[q] * (1.0 - u[q]);
            }
            for (int q = 0; q < d; q++) {
                grad[L->b + q] += dac[q];
                grad[L->bg + q] += dau[q];
                for (int k = 0; k < d; k++) {
                    grad[L->W + (long)q * K + k] += dac[q] * hz[k];
                    grad[L->W + (long)q * K + d + k] += dac[q] * hv[k];
                    grad[L->Wg + (long)q * K + k] += dau[q] * hz[k];
                    grad[L->Wg + (long)q * K + d + k] += dau[q] * hv[k];
                    grad[L->U + (long)q * 2 * d + k] += dv[q] * hz[k];
                    grad[L->U + (long)q * 2 * d + d + k] += dv[q] * hv[k];
                    if (dprev_hz)
                        dprev_hz[k] += P[L->W + (long)q * K + k] * dac[q] +
                                  P[L->Wg + (long)q * K + k] * dau[q] +
                                  P[L->U + (long)q * 2 * d + k] * dv[q];
                    if (dprev_vt)
                        dprev_vt[k] += P[L->W + (long)q * K + d + k] * dac[q] +
                                  P[L->Wg + (long)q * K + d + k] * dau[q] +
                                  P[L->U + (long)q * 2 * d + d + k] * dv[q];
                }
                if (xz >= 0) {
                    grad[L->W + (long)q * K + 2 * d + xz] += dac[q];
                    grad[L->Wg + (long)q * K + 2 * d + xz] += dau[q];
                }
                if (xv >= 0) {
                    grad[L->W + (long)q * K + 2 * d + 2 + xv] += dac[q];
                    grad[L->Wg + (long)q * K + 2 * d + 2 + xv] += dau[q];
                }
            }
        }
    }
    free(dh); free(dg); free(dhn); free(dac); free(dau); free(dar); free(dm); free(dv);
    free(c);
    trace_free(&t);
}

/* The same gradient with, per parameter, the sum over samples of the
 * absolute per-sample contributions (absgrad), from which the cancellation
 * factor kappa = |sum |t_s|| / |sum t_s| of a block follows.  The sum itself is
 * formed per sample first, so its rounding may differ from
 * ora_surrogate_grad's in the last bits. */
void ora_surrogate_grad_abs(const ora_model *m, const double *P, int64_t ns, const uint8_t *cfg,
                            const double *a, const double *b, double *grad, double *absgrad)
{
    layout L;
    make_layout(m, &L);
    int N = L.N;
    long np = L.total;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *part = calloc((size_t)2 * nt * np, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gp = part + (size_t)2 * tid * np, *ap = gp + np;
        double *ts = malloc(np * sizeof(double));
#pragma omp for schedule(static)
        for (int64_t s = 0; s < ns; s++) {
            memset(ts, 0, np * sizeof(double));
            backward_one(m, &L, P, cfg + s * N, a[s], b ? b[s] : 0.0, ts);
            for (long k = 0; k < np; k++) {
                gp[k] += ts[k];
                ap[k] += fabs(ts[k]);
            }
        }
        free(ts);
    }
    memset(grad, 0, np * sizeof(double));
    memset(absgrad, 0, np * sizeof(double));
    for (int t2 = 0; t2 < nt; t2++)
        for (long k = 0; k < np; k++) {
            grad[k] += part[(size_t)2 * t2 * np + k];
            absgrad[k] += part[(size_t)(2 * t2 + 1) * np + k];
        }
    free(part);
}

/* Gradient of the surrogate L(theta) = sum_s [a_s logP(sigma_s) + b_s phi(sigma_s)]
 * with the configurations and the coefficients held fixed.  The per-thread
 * partial sums are added in thread order, so the result is reproducible for a
 * fixed thread count. */
void ora_surrogate_grad(const ora_model *m, const double *P, int64_t ns, const uint8_t *cfg,
                        const double *a, const double *b, double *grad)
{
    layout L;
    make_layout(m, &L);
    int N = L.N;
    long np = L.total;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *part = calloc((size_t)nt * np, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gp = part + (size_t)tid * np;
#pragma omp for schedule(static)
        for (int64_t s = 0; s < ns; s++)
            backward_one(m, &L, P, cfg + s * N, a[s], b ? b[s] : 0.0, gp);
    }
    memset(grad, 0, np * sizeof(double));
    for (int t2 = 0; t2 < nt; t2++)
        for (long k = 0; k < np; k++) grad[k] += part[(size_t)t2 * np + k];
    free(part);
}

/*
 * Energy gradient by the covariance estimator (VMC, Sec. III):
 *   g = 2 Re sum_s w_s conj(E_s - Ebar) d log psi(sigma_s)
 *     = sum_s w_s [Re(E_s - Ebar) d logP_s + 2 Im(E_s - Ebar) d phi_s],
 * using d log psi = d logP / 2 + i d phi (Eq. (4)); E is held constant.
 * w = NULL means 1/ns.  stats as in ora_stats.
 */
void ora_grad(const ora_model *m, const double *P, int64_t ns, const uint8_t *cfg,
              const double *eloc, const double *w, double *grad, double *stats)
{
    double st[4];
    ora_stats(ns, eloc, w, st);
    double *a = malloc(ns * sizeof(double)), *b = malloc(ns * sizeof(double));
    for (int64_t s = 0; s < ns; s++) {
        double ws = w ? w[s] : 1.0 / (double)ns;
        a[s] = ws * (eloc[2 * s] - st[0]);
        b[s] = 2.0 * ws * (eloc[2 * s + 1] - st[1]);
    }
    ora_surrogate_grad(m, P, ns, cfg, a, m->is_complex ? b : NULL, grad);
    if (stats) memcpy(stats, st, sizeof(st));
    free(a);
    free(b);
}

/* ------------------------------------------------------------ grow_hidden */

/* Standard normal deviate for the new parameter at destination index e:
 * Box-Muller on two 24-bit uniforms from Philox(key=seed, ctr={e_lo, e_hi, 0, 0}),
 * u1 = (w0>>8 + 1)/2^24 in (0,1], u2 = (w1>>8)/2^24 in [0,1). */
static double grow_normal(uint64_t seed, uint64_t e)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)e, (uint32_t)(e >> 32), 0u, 0u};
    uint32_t o[4];
    ora_philox4x32_10(ctr, key, o);
    double u1 = ((double)(o[0] >> 8) + 1.0) * (1.0 / 16777216.0);
    double u2 = (double)(o[1] >> 8) * (1.0 / 16777216.0);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* Map hidden-input column k of an old gate matrix to the new one (1D: [h;x];
 * 2D: [h_hz; h_vt; x_hz; x_vt]); new hidden units go to the end of each
 * h-block and the one-hot columns keep their order. */
static int map_col(int dims, int d0, int d1, int k)
{
    if (dims == 1) return k < d0 ? k : d1 + (k - d0);
    if (k < d0) return k;
    if (k < 2 * d0) return d1 + (k - d0);
    return 2 * d1 + (k - 2 * d0);
}

/*
 * Adaptive growth of the hidden width d_h -> new_dh (Sec. II B, Fig. 2(b)):
 * every old parameter keeps its value at its new position, every new entry is
 * an independent draw eps * N(0,1) with eps = noise_std, and the Adam moments
 * (App. B: carried over into the larger model) keep the old entries and start
 * the new ones at 0.  Moment pointers may be NULL.
 */
void ora_grow_hidden(const ora_model *from, const double *p0, int32_t new_dh, uint64_t seed,
                     double noise_std, double *p1, const double *m0, const double *v0,
                     double *m1, double *v1)
{
    ora_model to = *from;
    to.d_h = new_dh;
    layout A, B;
    make_layout(from, &A);
    make_layout(&to, &B);
    int d0 = A.dh, d1 = B.dh, dims = from->dims;
    /* every destination entry starts as new noise (moments: 0) */
    for (long e = 0; e < B.total; e++) {
        p1[e] = noise_std * grow_normal(seed, (uint64_t)e);
        if (m1) m1[e] = 0.0;
        if (v1) v1[e] = 0.0;
    }
#define COPY(dst, src)                  \
    do {                                \
        p1[dst] = p0[src];              \
        if (m1 && m0) m1[dst] = m0[src]; \
        if (v1 && v0) v1[dst] = v0[src]; \
    } while (0)
    if (dims == 1) {
        int K0 = d0 + 2, K1 = d1 + 2;
        long mats[2][2] = {{A.Wg, B.Wg}, {A.Wr, B.Wr}};
        for (int t2 = 0; t2 < 2; t2++)
            for (int q = 0; q < d0; q++)
                for (int k = 0; k < K0; k++)
                    COPY(mats[t2][1] + (long)q * K1 + map_col(1, d0, d1, k), mats[t2][0] + (long)q * K0 + k);
        for (int q = 0; q < d0; q++) {
            for (int k = 0; k < d0; k++) COPY(B.Wh + (long)q * d1 + k, A.Wh + (long)q * d0 + k);
            for (int k = 0; k < 2; k++) COPY(B.Win + (long)q * 2 + k, A.Win + (long)q * 2 + k);
            COPY(B.bg + q, A.bg + q);
            COPY(B.br + q, A.br + q);
            COPY(B.bh + q, A.bh + q);
            COPY(B.bin + q, A.bin + q);
        }
    } else {
        int K0 = 2 * d0 + 4, K1 = 2 * d1 + 4;
        long mats[2][2] = {{A.W, B.W}, {A.Wg, B.Wg}};
        for (int t2 = 0; t2 < 2; t2++)
            for (int q = 0; q < d0; q++)
                for (int k = 0; k < K0; k++)
                    COPY(mats[t2][1] + (long)q * K1 + map_col(2, d0, d1, k), mats[t2][0] + (long)q * K0 + k);
        for (int q = 0; q < d0; q++) {
            for (int k = 0; k < 2 * d0; k++)
                COPY(B.U + (long)q * 2 * d1 + map_col(2, d0, d1, k), A.U + (long)q * 2 * d0 + k);
            COPY(B.b + q, A.b + q);
            COPY(B.bg + q, A.bg + q);
        }
    }
    if (from->glu) {
        for (int q = 0; q < d0; q++) {
            for (int k = 0; k < d0; k++) {
                COPY(B.W1 + (long)q * d1 + k, A.W1 + (long)q * d0 + k);
                COPY(B.W2 + (long)q * d1 + k, A.W2 + (long)q * d0 + k);
            }
            COPY(B.b1 + q, A.b1 + q);
            COPY(B.b2 + q, A.b2 + q);
        }
    }
    for (int o = 0; o < 2; o++) {
        for (int k = 0; k < d0; k++) COPY(B.Ua + (long)o * d1 + k, A.Ua + (long)o * d0 + k);
        COPY(B.ca + o, A.ca + o);
        if (from->is_complex) {
            for (int k = 0; k < d0; k++) COPY(B.Up + (long)o * d1 + k, A.Up + (long)o * d0 + k);
            COPY(B.cp + o, A.cp + o);
        }
    }
#undef COPY
}

/* ------------------------------------------------------------------ Adam */

/* One Adam update (Kingma & Ba, ICLR 2015; the optimiser of App. B) at step
 * t >= 1 with learning rate lr:
 *   m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
 *   p = p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
void ora_adam(int64_t n, double *p, const double *g, double *m, double *v, int64_t t, double lr,
              double b1, double b2, double eps)
{
    for (int64_t i = 0; i < n; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / (1.0 - pow(b1, (double)t));
        double vh = v[i] / (1.0 - pow(b2, (double)t));
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Threads of the OpenMP loops (the CPU baseline's one-core rate). */
void ora_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* bfloat16 rounding used by the emulation mode, exported for its own test */
double ora_round_bf16(double x) { return to_bf16(x); }
