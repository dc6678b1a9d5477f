/*
 * vmcrnn.h -- C ABI of the MI355X (gfx950) variational-Monte-Carlo hot path
 * for GRU recurrent-neural-network wave functions (McNaughton & Hibat-Allah,
 * "Adaptive Neural Quantum States: A Recurrent Neural Network Perspective",
 * arXiv 2507.18700).
 *
 * General conventions
 *  - Every array argument is a DEVICE pointer owned by the caller, except the
 *    descriptors (vmc_model, vmc_ham), which are host structs read during the
 *    call.  No call allocates device memory: scratch space comes from the
 *    caller's workspace `ws` of at least vmc_workspace_size() bytes, aligned
 *    to 256 bytes.  The workspace holds no state between calls.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    All work is enqueued on it and the call returns without synchronising.
 *    Calls on one workspace must not overlap (same stream or ordered).
 *  - Argument errors are detected on the host before any launch and leave
 *    every output untouched.  A launch failure returns VMC_EDEVICE.
 *  - Spin configurations are uint8 in {0,1}, row-major [count][N], lattice
 *    order: site (i,j) (column i < Lx, row j < Ly) at index j*Lx + i.
 *    sigma = 0 is the +1 eigenvector of sigma^z.
 *  - Parameters are float32, one flat vector per model, in this order
 *    (row-major [out][in]; d = d_h):
 *      1D GRU (App. A): W_g[d][d+2], b_g[d], W_r[d][d+2], b_r[d],
 *                       W_h[d][d], b_h[d], W_in[d][2], b_in[d]
 *                       (gate input order [h_{n-1}; onehot(sigma_{n-1})])
 *      2D GRU (App. A): W[d][2d+4], b[d], W_g[d][2d+4], b_g[d], U[d][2d]
 *                       (input order [h_hz; h_vt; onehot_hz; onehot_vt])
 *      GLU (App. A, if glu):  W_1[d][d], b_1[d], W_2[d][d], b_2[d]
 *      amplitude head (Eq. 3): U_a[2][d], c_a[2]
 *      phase head (Eq. 5, if is_complex): U_p[2][d], c_p[2]
 *  - Order of the autoregressive chain (Sec. II A): 1D runs over the sites;
 *    2D runs in zig-zag order, even rows left to right, odd rows right to
 *    left, with the predecessors (i-(-1)^j, j) and (i, j-1).  h_0 = 0 and a
 *    missing neighbour contributes h = 0 and one-hot (0,0).
 */
#ifndef VMCRNN_H
#define VMCRNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VMC_OK = 0,
    VMC_EINVAL = -1,       /* bad argument (null pointer, size, descriptor) */
    VMC_EUNSUPPORTED = -2, /* valid but not supported: d_h not in {16,32,64,128,256},
                              or a kernel's LDS (its tile's configurations, tile rows
                              x N bytes, plus its static tiles) above 160 KiB */
    VMC_ENOSPACE = -3,     /* workspace smaller than vmc_workspace_size() */
    VMC_EDEVICE = -4,      /* a HIP call or kernel launch failed */
    VMC_ENONFINITE = -5    /* a non-finite value where a finite one is required: a
                              Hamiltonian coupling, field or exponent, the noise of
                              grow_hidden, an Adam setting, or (vmc_check_finite) an
                              entry of a device array */
} vmc_status;

enum { VMC_FP32 = 0, VMC_BF16 = 1 };      /* GEMM operand precision */
/* Hamiltonians: Eqs. (6), (7), (8), (9) */
enum { VMC_TFIM = 0, VMC_HEISENBERG = 1, VMC_LRTFIM = 2, VMC_CLUSTER = 3 };

/* Wave-function descriptor.  N = Lx*Ly sites (1D: Ly = 1).  d_h in [1,256];
 * d_model = d_h.  precision: VMC_FP32 = FP32 MFMA operands, VMC_BF16 =
 * bfloat16 operands of the cell and GLU contractions (weights and hidden
 * states rounded to nearest even), FP32 accumulation, FP32 activations and
 * heads in both. */
typedef struct {
    int32_t dims;       /* 1 or 2 */
    int32_t Lx, Ly;
    int32_t d_h;
    int32_t is_complex; /* complex RNN: softsign phase head (Eqs. 4-5) */
    int32_t glu;        /* gated linear unit before the heads (App. A) */
    int32_t precision;  /* VMC_FP32 or VMC_BF16 */
} vmc_model;

/* Hamiltonian with open boundaries on the chain (1D) or square lattice (2D):
 *  VMC_TFIM       H = -J sum_<ab> Z_a Z_b - h sum_k X_k                (Eq. 6)
 *  VMC_HEISENBERG H = J/4 sum_<ab> (X_a X_b + Y_a Y_b + Z_a Z_b)       (Eq. 7)
 *                 with marshall != 0, the Marshall-sign rotated form whose
 *                 off-diagonal elements are all negative (Sec. III B).
 *  VMC_LRTFIM     H = -J sum_{i<j} Z_i Z_j / |i-j|^alpha - h sum_k X_k
 *                 (Eq. 8, long-range TFIM; 1D only)
 *  VMC_CLUSTER    H = -J [ sum_{k=2}^{n-2} X_{k-1} Z_k X_{k+1}
 *                         + Z_1 X_2 + X_{n-1} X_n + X_{n-2} Z_{n-1} Z_n ]
 *                 (Eq. 9, 1D cluster state with the boundary terms as the
 *                 paper writes them, sites 1..n; n >= 3; 1D only).
 * Every coupling must be finite (VMC_ENONFINITE otherwise); alpha is read by
 * VMC_LRTFIM only and must be >= 0. */
typedef struct {
    int32_t kind;
    int32_t marshall;
    double J, h;
    double alpha;
} vmc_ham;

/* Number of float parameters of the flat vector described above; -1 if the
 * descriptor is invalid. */
int64_t vmc_param_count(const vmc_model *m);

/* Workspace bytes needed by any call below with this model, Hamiltonian
 * (may be NULL when local_energy is not used) and up to `ns` samples or
 * configurations per call.  Checks the Hamiltonian like the calls do
 * (VMC_ENONFINITE for a non-finite coupling, VMC_EUNSUPPORTED for a 1D-only
 * kind on a 2D lattice). */
vmc_status vmc_workspace_size(const vmc_model *m, const vmc_ham *H, int64_t ns, size_t *bytes);

/* Perfect autoregressive sampling (Sec. II A, Eq. 1): for each sample s and
 * order position n, sigma_n = 0 if u[s][n] < P(sigma_n = 0 | sigma_<n), else 1.
 *  uniforms: [ns][N] float in [0,1), indexed by ORDER position; or NULL, in
 *            which case u[s][n] = (word n%4 of Philox4x32-10(key = seed,
 *            ctr = {n/4, s, counter_lo, counter_hi}) >> 8) * 2^-24
 *            (Salmon et al., SC'11).  ns must be < 2^32.
 *  configs:  out [ns][N] uint8, lattice order.
 *  logp:     out [ns] log P(sigma) (log |psi|^2, Eq. 3 chained by Eq. 1).
 *  phase:    out [ns] phi(sigma) (Eq. 5), or NULL; ignored for positive RNNs. */
vmc_status rnn_sample(const vmc_model *m, const float *params, int64_t ns, uint64_t seed,
                      uint64_t counter, const float *uniforms, uint8_t *configs, float *logp,
                      float *phase, void *ws, size_t ws_bytes, void *stream);

/* Teacher-forced log P and phase of nc given configurations (Eqs. 1, 3, 5);
 * log psi = logp/2 + i*phase (Eq. 4).  phase may be NULL. */
vmc_status rnn_logpsi(const vmc_model *m, const float *params, int64_t nc,
                      const uint8_t *configs, float *logp, float *phase, void *ws,
                      size_t ws_bytes, void *stream);

/* Local energy E_loc(sigma) = sum_sigma' H(sigma,sigma') psi(sigma')/psi(sigma)
 * for ns configurations (Eqs. 6, 7).  Every connected configuration of every
 * sample is evaluated in the same call; only the part of the chain after the
 * first changed order position is recomputed.
 *  eloc: out [ns][2] double (real, imaginary). */
vmc_status local_energy(const vmc_model *m, const float *params, const vmc_ham *H, int64_t ns,
                        const uint8_t *configs, double *eloc, void *ws, size_t ws_bytes,
                        void *stream);

/* Energy statistics and the covariance estimate of the energy gradient
 * (VMC with the normalised autoregressive ansatz, Sec. III):
 *    Ebar = sum_s w_s E_s,  var = sum_s w_s |E_s - Ebar|^2,
 *    grad = 2 Re sum_s w_s conj(E_s - Ebar) d log psi(sigma_s)
 *         = sum_s w_s [Re(E_s-Ebar) d logP_s + 2 Im(E_s-Ebar) d phi_s],
 * with E held constant.  weights: [ns] double or NULL (w_s = 1/ns).
 *  eloc:  [ns][2] double.   grad: out [vmc_param_count] double.
 *  stats: out [4] double: Re Ebar, Im Ebar, var, count of non-finite E_s.
 * Cross-sample sums are FP64 in a fixed order (bitwise reproducible). */
vmc_status vmc_grad(const vmc_model *m, const float *params, int64_t ns, const uint8_t *configs,
                    const double *eloc, const double *weights, double *grad, double *stats,
                    void *ws, size_t ws_bytes, void *stream);

/* The gradient of vmc_grad over a sample set too large for one workspace
 * (Sec. III: the estimator is a weighted sum over independent samples once
 * Ebar is fixed, so it splits over sample chunks without recomputation):
 *  vmc_energy_stats: stats [4] double (out) of the whole set, as vmc_grad
 *    forms them: Re Ebar, Im Ebar, var, non-finite count; eloc [ns][2]
 *    double, weights [ns] double or NULL (w_s = 1/ns).  Needs no model and
 *    no workspace; ns >= 1.
 *  vmc_grad_chunk: the contribution of one chunk of ns samples of that set,
 *    sum over the chunk of w_s [Re(E_s-Ebar) d logP_s + 2 Im(E_s-Ebar) d phi_s],
 *    ADDED to grad [vmc_param_count] double (the caller zeroes grad before the
 *    first chunk).  weights [ns] double is required: the whole set's weights
 *    of these samples (1/ns_total for an unweighted set); stats [4] double is
 *    read only (Ebar of the whole set, from vmc_energy_stats).  configs,
 *    eloc, ws and stream as for vmc_grad with this chunk's ns (workspace of
 *    vmc_workspace_size(m, NULL, ns) bytes).  Over all chunks the sum equals
 *    vmc_grad on the whole set up to the FP32 rounding of the per-position
 *    partial sums (their sample ranges differ) and the FP64 order of the
 *    chunk additions.  Calls on one stream run in order; grad must not be
 *    written by another call in between.
 * Errors (before any launch): VMC_EINVAL for ns < 1 or a NULL eloc, stats,
 * weights (vmc_grad_chunk), configs or grad; the model, parameter and
 * workspace checks of vmc_grad (VMC_EUNSUPPORTED, VMC_ENOSPACE). */
vmc_status vmc_energy_stats(int64_t ns, const double *eloc, const double *weights, double *stats,
                            void *stream);
vmc_status vmc_grad_chunk(const vmc_model *m, const float *params, int64_t ns, const uint8_t *configs,
                          const double *eloc, const double *weights, const double *stats, double *grad,
                          void *ws, size_t ws_bytes, void *stream);

/* Vector-Jacobian product of rnn_logpsi (the backward of log psi as a
 * differentiable function of the parameters, Eq. 1 through App. A):
 *   grad[k] = sum_s ( dlogp[s] * d logP(sigma_s)/d theta_k
 *                   + dphase[s] * d phi(sigma_s)/d theta_k ),
 * logP = log |psi|^2 and phi the phase (Eqs. 3-5).  dlogp [nc] float32
 * (required), dphase [nc] float32 or NULL (= 0; ignored for a positive RNN),
 * grad [P] float64 (overwritten).  Same reverse sweep as vmc_grad, with the
 * per-sample coefficients given instead of formed from the local energies. */
vmc_status rnn_logpsi_grad(const vmc_model *m, const float *params, int64_t nc, const uint8_t *configs,
                           const float *dlogp, const float *dphase, double *grad, void *ws, size_t ws_bytes,
                           void *stream);

/* One VMC step in one call: rnn_sample, then local_energy of the samples,
 * then vmc_grad with w_s = 1/ns, sharing one forward pass (the sampler keeps
 * the hidden states, conditionals and activations that the local energy and
 * the backward sweep need).  Outputs equal those of the three separate calls
 * with the same arguments.  uniforms may be NULL (Philox as in rnn_sample);
 * phase may be NULL.
 *  counter_dev: NULL, or a device uint64 that replaces `counter`: the sampler
 *            reads the Philox counter from it when it runs, and the step's
 *            last kernel adds 1 to it, so that the replays of a captured HIP
 *            graph of this call draw fresh uniforms, step after step, equal
 *            to those of eager calls with counter = k, k+1, ...
 * Non-finite parameters are not detected here (that would need a host
 * synchronisation): they make the outputs non-finite, stats[3] = ns; see
 * vmc_check_finite. */
vmc_status vmc_step(const vmc_model *m, const float *params, const vmc_ham *H, int64_t ns,
                    uint64_t seed, uint64_t counter, uint64_t *counter_dev, const float *uniforms,
                    uint8_t *configs, float *logp, float *phase, double *eloc, double *grad,
                    double *stats, void *ws, size_t ws_bytes, void *stream);

/* Several independent 1D problems in one call (uneven chains or couplings;
 * the batched VMC step of Sec. III, one per problem): problem k is a chain of
 * chain_len[k] sites with the cell shape of m (d_h, precision, is_complex,
 * glu; m->dims must be 1, m->Lx is ignored), Hamiltonian H[k] (all of the
 * same kind, couplings free) and parameters params + k*P (P =
 * vmc_param_count of that shape), and its outputs equal, bit for bit, those
 * of vmc_step on that problem alone with Philox key seed + k and the same
 * counter.  The launches are shared: one sampling launch over the tiles of
 * every problem, one persistent suffix-chain launch over every connected
 * configuration of every sample of every problem (one queue, longest chains
 * first), one reverse sweep and one weight-gradient contraction per
 * segment.  At most 64 problems, all with ns samples.
 *  params:  [nprob][P] float.
 *  configs: [nprob][ns * Nmax] uint8; problem k's [ns][chain_len[k]]
 *           configurations start at k * ns * Nmax (Nmax = the longest chain).
 *  logp, phase: [nprob][ns] float (phase may be NULL).
 *  eloc: [nprob][ns][2] double; grad: [nprob][P] double; stats: [nprob][4].
 *  counter_dev: as in vmc_step (one counter for the batch).
 *  ws: at least vmc_batched_workspace_size() bytes. */
vmc_status vmc_step_batched(int32_t nprob, const vmc_model *m, const int32_t *chain_len, const vmc_ham *H,
                            const float *params, int64_t ns, uint64_t seed, uint64_t counter,
                            uint64_t *counter_dev, uint8_t *configs, float *logp, float *phase,
                            double *eloc, double *grad, double *stats, void *ws, size_t ws_bytes,
                            void *stream);

/* Workspace bytes of vmc_step_batched with these arguments (chain_len and H
 * are host arrays of nprob entries). */
vmc_status vmc_batched_workspace_size(int32_t nprob, const vmc_model *m, const int32_t *chain_len,
                                      const vmc_ham *H, int64_t ns, size_t *bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): vmc_step
 * with its workspace in a fixed device array of the library instead of a
 * caller-provided one.  The caller still passes every input and output.
 * The array holds vmc_noalloc_scratch_bytes() = 256 MiB on each GPU the
 * library runs on, from the first call on that GPU until the process ends;
 * a model, Hamiltonian and sample count whose vmc_workspace_size exceeds it
 * get VMC_ENOSPACE before any launch.  The call allocates nothing (no
 * hipMalloc or hipFree, no allocating library routine).  Every call on one
 * GPU uses the same array: calls that overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.  The array keeps
 * the last call's contents; the step needs no zeroed workspace.  Arguments
 * and results as for vmc_step. */
vmc_status vmc_step_noalloc(const vmc_model *m, const float *params, const vmc_ham *H, int64_t ns,
                            uint64_t seed, uint64_t counter, uint64_t *counter_dev, const float *uniforms,
                            uint8_t *configs, float *logp, float *phase, double *eloc, double *grad,
                            double *stats, void *stream);

/* Bytes of the fixed workspace of vmc_step_noalloc (per GPU). */
size_t vmc_noalloc_scratch_bytes(void);

/* Adam update (Kingma & Ba, ICLR 2015), the optimiser of every benchmark of
 * the paper (App. B), of n float32 parameters from an FP64 gradient:
 *    t = *t_dev + 1,  lr = lr(t - 1),
 *    m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * then *t_dev = t (a trailing one-thread kernel, so the update reads the old
 * value).  m and v are float32 [n], carried through grow_hidden when the
 * hidden width grows (App. B).  t_dev is a device int64 (updates done so
 * far), so a captured HIP graph keeps counting on replay.  The learning
 * rate at update index k = t - 1 follows the schedules of Table III:
 *    lr(k) = (k < t_switch ? lr0 : lr1) / (1 + max(0, k - t_decay) / tau)
 * with tau = 0 meaning no decay (constant, two-stage, inverse-time).
 * Every setting must be finite (VMC_ENONFINITE), lr >= 0, 0 <= b1, b2 < 1,
 * eps > 0, tau >= 0 (VMC_EINVAL). */
typedef struct {
    double lr0, lr1;
    int64_t t_switch;
    int64_t t_decay;
    double tau;
    double beta1, beta2, eps;
} vmc_adam_cfg;

vmc_status vmc_adam(int64_t n, float *params, const double *grad, float *m, float *v, int64_t *t_dev,
                    const vmc_adam_cfg *cfg, void *stream);

/* Synchronous check that the n float32 entries of the device array x are all
 * finite: counts the non-finite ones on `stream` (into the first 256 bytes of
 * the workspace, ws_bytes >= 256), waits for the stream, and returns
 * VMC_ENONFINITE if the count is not zero (*count, if not NULL, receives
 * it).  Meant before a run or after a failed step, not inside a captured
 * graph. */
vmc_status vmc_check_finite(const float *x, int64_t n, int64_t *count, void *ws, size_t ws_bytes,
                            void *stream);

/* Adaptive growth of the hidden width (Sec. II B, Fig. 2(b); App. B):
 * copies every parameter of `from` into the model with d_h = new_dh
 * (new hidden units at the end of each h-block of every matrix, one-hot
 * columns keep their order), fills every new entry with noise_std * z,
 * z standard normal from Box-Muller on Philox4x32-10(key = seed,
 * ctr = {e_lo, e_hi, 0, 0}) at destination index e (u1 = (w0>>8 + 1)/2^24,
 * u2 = (w1>>8)/2^24), and pads the Adam moments with zeros.
 *  p_from: [vmc_param_count(from)]; p_to: [count at new_dh].
 *  m_from/v_from/m_to/v_to: moments, all four NULL or all four non-NULL.
 *  new_dh must be >= from->d_h. */
vmc_status grow_hidden(const vmc_model *from, const float *p_from, int32_t new_dh, uint64_t seed,
                       double noise_std, float *p_to, const float *m_from, const float *v_from,
                       float *m_to, float *v_to, void *stream);

/* Launch tuning.  Two launch choices per model shape (dims, Lx, Ly, d_h,
 * precision, glu, is_complex) are kept in a process-wide table that every call
 * above reads:
 *  row_tile:          rows per work-group tile of the sampling and log psi
 *                     launches (rnn_sample, rnn_logpsi, and the forward pass
 *                     of local_energy, vmc_grad, rnn_logpsi_grad, vmc_step);
 *                     one of vmc_row_tile_options(); 0 = built-in choice;
 *  chain_wgs_per_cu:  persistent work-groups per compute unit of the
 *                     suffix-chain launch of local_energy, 1..4; 0 = built-in
 *                     (twice as many as fit one compute unit, from the
 *                     runtime's occupancy query, at most 4; 2 when it cannot
 *                     answer).
 * No choice changes any output bit: each row of a tile and each connected
 * configuration is computed independently of the tile and of the work-group
 * that runs it.  vmc_workspace_size() covers every choice, so a workspace
 * stays valid when the table changes.  The table is guarded by a mutex; a
 * change while another thread runs the same shape affects only its speed. */
typedef struct {
    int32_t row_tile;
    int32_t chain_wgs_per_cu;
} vmc_tuning;

/* The row-tile heights this model shape can run with (count 1 or 2; the
 * built-in one first).  opts must hold 2 entries. */
vmc_status vmc_row_tile_options(const vmc_model *m, int32_t *opts, int32_t *count);

/* Set the tuning of this model shape (t = NULL restores the built-in
 * choices).  EINVAL for a row_tile not among the options or a
 * chain_wgs_per_cu outside 0..4. */
vmc_status vmc_set_tuning(const vmc_model *m, const vmc_tuning *t);

/* The choices in effect for this model shape, resolved (no zeros). */
vmc_status vmc_get_tuning(const vmc_model *m, vmc_tuning *t);

/* Autotuner: times vmc_step (same arguments and outputs) under each
 * candidate, coordinate by coordinate from the tuning in effect (the row-tile
 * options, then chain_wgs_per_cu = 1..4), `reps` steps each, fastest step
 * kept (HIP events on `stream`), stores the winner in the table and returns
 * it in *best (may be NULL).  Blocks until done (it synchronises on its
 * events).  The outputs are those of a final step under the chosen tuning,
 * the same bits as one vmc_step.  reps in 1..100. */
vmc_status vmc_autotune_step(const vmc_model *m, const float *params, const vmc_ham *H, int64_t ns,
                             uint64_t seed, uint64_t counter, const float *uniforms, uint8_t *configs,
                             float *logp, float *phase, double *eloc, double *grad, double *stats,
                             void *ws, size_t ws_bytes, void *stream, int32_t reps, vmc_tuning *best);

/* Opt-in timing of the dominant launch, the batched suffix-chain kernel of
 * local_energy.  vmc_chain_timing(1) creates (once) a pool of HIP events,
 * resets the record and makes every following local_energy call record one
 * event pair around that launch on its stream (up to 4096 launches);
 * vmc_chain_timing(0) stops recording.  vmc_chain_time() waits for the
 * recorded events and returns the summed milliseconds and the number of
 * timed launches.  Process-wide; not meant for concurrent callers. */
vmc_status vmc_chain_timing(int enable);
vmc_status vmc_chain_time(double *ms_total, int64_t *launches);

/* Static description of a status code. */
const char *vmc_status_str(vmc_status s);

#ifdef __cplusplus
}
#endif

#endif /* VMCRNN_H */
