/*
 * chym.h -- C ABI of libchym, a gfx950 (MI355X) library that time-integrates
 * the coherent hyperspin machine (CHYM) of Calvanese Strinati & Conti,
 * "Hyperscaling in the coherent hyperspin machine", arXiv 2308.02329.
 *
 * The method (paper, Eq. (1)-(2) and the surrounding text): N hyperspins,
 * each a D-component vector of parametric-oscillator amplitudes, are
 * amplified by a pump, coupled through C = J_N (x) 1_D (the same N x N matrix
 * J_N acts on every component), limited by the nonlocal loss
 * W = beta 1_N (x) I_D (the squared norm of each hyperspin) and by the local
 * gain saturation of the chi(2) medium, while the coupling of component mu is
 * scaled by the annealing weights alpha_{mu,tau} that morph the
 * D-dimensional hypergraph back into the Ising model.  The library
 * integrates the continuous-time limit of the round-trip map of Eq. (2)
 * (small loss per round trip; time in photon lifetimes, pump in units of the
 * uncoupled threshold, amplitudes rescaled) by forward Euler:
 *
 *   x_{p,mu} <- x_{p,mu} + dt [ (r_i - 1) x_{p,mu}
 *                               + eps alpha_mu[k] sum_q J_pq x_{q,mu}
 *                               - btil x_{p,mu} sum_nu x_{p,nu}^2
 *                               - eta x_{p,mu}^3 ]
 *
 * (CHYM: btil = 1, eta = (kappa L)^2 / (2 beta b^2); conventional CIM with
 * D = 1: btil = 0, eta = 1), then reads the Ising spins from the sign of the
 * first component, and scores each run by its exact Ising energy and by the
 * hyperspin energy of Eq. (3).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers owned by the caller, unless a
 *     comment says "host".  The library never allocates or frees them.
 *   - Layouts are C-contiguous:
 *       J       [n][n]         row p, column q (symmetric, zero diagonal for
 *                              the Ising model; any matrix is accepted)
 *       x       [n][r][d]      float32 amplitudes: row p, replica i, component mu
 *       pump    [r]            float32 normalized pump r_i = h_i / h_th
 *       alpha   [T][d]         float32 annealing weights, row k for step k
 *       spins   [r][w]         uint64, w = ceil(n / 64); bit (p % 64) of word
 *                              p / 64 is 1 iff sigma_p = +1, i.e. x_{p,1} >= 0
 *                              (-0 reads +1, NaN reads -1); unused high bits 0
 *   - stream is a hipStream_t (NULL: the default stream).  Every call is
 *     asynchronous on that stream except where stated; the library never
 *     synchronizes the host unless documented.
 *   - Return value: CHYM_OK (0) or a negative CHYM_E* code.  Arguments are
 *     validated before any device work is queued; on error nothing is
 *     launched and chym_last_error() describes the failure.  No C++
 *     exception crosses this interface.
 */
#ifndef CHYM_H
#define CHYM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHYM_VERSION 1

/* return codes */
#define CHYM_OK 0
#define CHYM_EINVAL (-1)       /* invalid argument (null pointer, bad size, bad enum) */
#define CHYM_EUNSUPPORTED (-2) /* valid but not supported (size beyond the kernels' limits) */
#define CHYM_ENODEV (-3)       /* no gfx950 device visible */
#define CHYM_EHIP (-4)         /* a HIP runtime call failed; see chym_last_error() */
#define CHYM_ENOMEM (-5)       /* caller-provided workspace too small */

/* Storage type of the coupling matrix J_N of Eq. (1)-(2), row-major, row p
 * holding the couplings J_pq that feed hyperspin p. */
#define CHYM_J_I8 0  /* int8 [n][n] integer couplings (e.g. +-1 / 0): contraction and Ising energy exact */
#define CHYM_J_F32 1 /* float32 [n][n] couplings (e.g. Gaussian) */
#define CHYM_J_BF16 2 /* bfloat16 [n][n] (bit patterns as uint16) */
#define CHYM_J_FP8 3  /* OCP FP8 E4M3 (e4m3fn) [n][n] bytes followed by n OCP E8M0 row-exponent bytes:
                         J_pq = e4m3(q_pq) * 2^(E_p - 127), n * (n + 1) bytes in all.  Every such value
                         is exact in bf16 (and float32) as long as it is zero or at least 2^-126 in
                         magnitude, so the contraction sees the stored J exactly.  E4M3 0x7f / 0xff
                         and E8M0 0xff decode to NaN.  chym_quantize_fp8() writes this format. */
#define CHYM_J_ELL 4  /* sparse rows (ELL), int32 [n + 1][2 w]: row 0 = {n, w, 0, ...}; row p + 1 = w columns
                         q, then the w couplings J_pq as float32 bit patterns (pad unused entries with
                         coupling 0); columns outside [0, n) are ignored.  8 w (n + 1) bytes.  Integrated
                         by a gather kernel in float32 (both precision forms), n <= 4096; batches take
                         it (one group per d); not for plans, features or the map. */

/* arithmetic of the J x contraction (the state and every other step are float32) */
#define CHYM_PREC_F32 0  /* x fed to the matrix cores as an exact sum of three bf16 terms
                            (and J as three terms when it is not an integer matrix), float32
                            accumulation: float32-accurate products */
#define CHYM_PREC_BF16 1 /* x rounded to bf16 (round to nearest even) at the matrix-core
                            input, J rounded to bf16 (exact for integer |J| <= 256 and for
                            CHYM_J_BF16 / CHYM_J_FP8), float32 accumulation and float32 state */

typedef void *chym_stream_t; /* hipStream_t */

/* One coupled system.  Paper: J_N and D (text after Eq. (1)); eps, btil and
 * eta are the normalized coupling, nonlocal-loss and local-saturation
 * coefficients of the continuous-time limit of Eq. (2). */
typedef struct chym_problem {
    int32_t n;        /* hyperspins N >= 1 */
    int32_t d;        /* components per hyperspin, 1 <= D <= 4 */
    int32_t j_dtype;  /* CHYM_J_I8, CHYM_J_F32, CHYM_J_BF16 or CHYM_J_FP8 */
    int32_t reserved; /* must be 0 */
    const void *j;    /* device, layout by j_dtype (chym_j_bytes) */
    float eps;        /* coupling strength */
    float btil;       /* nonlocal loss coefficient (1 for the CHYM, 0 for the CIM) */
    float eta;        /* local cubic saturation coefficient */
    float reserved_f; /* must be 0 */
} chym_problem;

/* A block of independent runs (replicas) of one problem.  Paper: pump h
 * scanned as h = h_th (1 + delta h) and the annealing protocol alpha_{mu,tau}
 * (text after Fig. 2 and in the statistics paragraph). */
typedef struct chym_run {
    int32_t r;          /* replicas >= 1 */
    int32_t steps;      /* Euler steps taken by this call, >= 0 */
    int32_t start_step; /* global index of the first step (row of alpha), >= 0 */
    int32_t precision;  /* CHYM_PREC_F32 or CHYM_PREC_BF16 */
    float dt;           /* Euler step, > 0 */
    float reserved_f;   /* must be 0 */
    const float *pump;  /* device [r] */
    float *x;           /* device [n][r][d], read and overwritten in place */
    const float *alpha; /* device [start_step + steps][d] */
} chym_run;

/* Per-run results; every pointer may be NULL (that output is skipped). */
typedef struct chym_out {
    uint64_t *spins;     /* [r][ceil(n/64)] sign readout of the final state */
    int32_t *e_ising;    /* [r] exact Ising energy; CHYM_J_I8 only (else must be NULL) */
    double *e_ising_f64; /* [r] Ising energy in float64 (exact for integer J) */
    double *e_hs;        /* [r] hyperspin energy, Eq. (3), of the final state (float64) */
    double *extra_frac;  /* [r] max_p sum_{mu>=2} x^2 / |x_p|^2 of the final state */
    uint8_t *diverged;   /* [r] 1 if any final amplitude is non-finite or |x| > 1e3 */
} chym_out;

/* Library version (CHYM_VERSION). */
int chym_version(void);

/* Thread-local description of the last error returned on this thread. */
const char *chym_last_error(void);

/* Advance every replica by run->steps Euler steps of the equation above,
 * synchronous (Jacobi) update, using alpha rows start_step .. start_step +
 * steps - 1.  Splitting a run into calls with consecutive start_step gives
 * bit-identical results to one call.
 *
 * Two integrators, chosen by size, give identical results for the same
 * problem: a register-resident one (no workspace) up to n = 192 (d = 1),
 * 144/160 (d = 2, float32/bf16 form), 128 (d = 3), 112 (d = 4), or less
 * for float J in the float32 form; and a streamed-J one for larger n, up to
 * n = 1024 in both forms, which needs a caller workspace (chym_integrate_ws).
 * The streamed-J integrator keeps the bf16 operand of 16 replicas,
 * ceil(n/32) * d * terms KiB (terms = 1 in the bf16 form, 3 in the float32
 * form), in LDS; where that exceeds 159 KiB (the float32 form beyond n = 832,
 * 544, 416 for d = 2, 3, 4) it holds one component at a time and reads J d
 * times per step, with the same results.  chym_integrate returns
 * CHYM_EUNSUPPORTED where a workspace is needed. */
int chym_integrate(const chym_problem *prob, const chym_run *run, chym_stream_t stream);

/* Device workspace bytes chym_integrate_ws / chym_solve_ws need for this
 * problem (0 when the register-resident integrator applies). */
int chym_integrate_workspace_size(const chym_problem *prob, const chym_run *run, size_t *bytes);

/* chym_integrate with a caller workspace (256-byte aligned) for the staged
 * coupling matrix of the streamed-J integrator. */
int chym_integrate_ws(const chym_problem *prob, const chym_run *run, void *workspace, size_t ws_bytes,
                      chym_stream_t stream);

/* chym_integrate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * every size chym_integrate_ws takes, with no workspace argument.  The
 * streamed-J integrator's staged couplings go into a static device array of
 * the library (6.06 MiB, enough for n = 1024 with couplings in three bf16
 * terms; one copy per GPU, held until the process ends); sizes whose staging
 * would not fit are refused with CHYM_EUNSUPPORTED.  The call itself
 * allocates nothing.  All calls on one GPU share its array: calls that
 * overlap on one GPU (concurrent streams, or host threads) race and must be
 * serialized by the caller; consecutive calls on one stream are ordered and
 * safe.  Results are bit-identical to chym_integrate_ws. */
int chym_integrate_noalloc(const chym_problem *prob, const chym_run *run, chym_stream_t stream);

/* The round-trip map of Eq. (2) itself, one step per round trip (the
 * paper's own simulation model; chym_integrate integrates its continuous
 * limit).  For every parametric oscillator j = (p, mu):
 *   B_j  = K(A_j) A_j,  K(A) = P / (P cosh(kl P) - h sinh(kl P)),  P = sqrt(h^2 + A^2)
 *          (exact solution of the degenerate phase-matched coupled-mode
 *          equations over the medium, the NLM paragraph; h the pump),
 *   Y_j  = (1 - b) B_j + b jmag alpha_mu sum_q J_pq B_{q,mu} - beta_b2 B_j sum_nu B_{p,nu}^2,
 *   A'_j = (1 - loss) Y_j.
 * J holds the coupling pattern (e.g. +-1); jmag is the coupling magnitude J.
 * run->pump holds h per replica (absolute, not normalized), run->x the
 * amplitudes A [n][r][d] (in/out), run->dt must be 1 (one round trip per
 * step), run->alpha the annealing table as for chym_integrate.  N <= 112
 * (register-resident integrator); couplings must be exact in one bf16 term
 * (CHYM_J_I8, CHYM_J_BF16, CHYM_J_FP8); otherwise CHYM_EUNSUPPORTED. */
typedef struct chym_map_problem {
    int32_t n;        /* parametric-oscillator blocks (hyperspins) N >= 1 */
    int32_t d;        /* components per hyperspin, 1 <= D <= 4 */
    int32_t j_dtype;  /* CHYM_J_I8, CHYM_J_BF16 or CHYM_J_FP8 */
    int32_t reserved; /* must be 0 */
    const void *j;    /* device, layout by j_dtype */
    float b;          /* coupler fraction per round trip, 0 < b < 1 */
    float loss;       /* linear loss d per round trip, 0 <= d < 1 */
    float kl;         /* kappa L of the medium, > 0 */
    float beta_b2;    /* nonlocal-loss coefficient beta b^2, >= 0 */
    float jmag;       /* coupling magnitude J */
    float reserved_f; /* must be 0 */
} chym_map_problem;

int chym_map_integrate(const chym_map_problem *prob, const chym_run *run, chym_stream_t stream);

/* Many map problems, one persistent launch per kernel variant (row tiles,
 * d, precision).  Paper: the statistics are gathered over N_g graphs x N_s
 * pump values x N_r repetitions of the map, all independent (statistics
 * paragraph, Figs. 3-4).  Each problem t is chym_map_integrate(&probs[t],
 * &runs[t]); results are bit-identical to it.  The workspace (device, 256-byte
 * aligned, size from chym_map_batch_workspace_size) receives the task table,
 * the work list of (task, 16-replica group) items, longest run first, and
 * one work counter per variant.  The host tables are copied on `stream`,
 * which is synchronized once before the launches are queued; the launches
 * then run asynchronously.  Calls that share a workspace must not overlap.
 * Errors name the offending task; nothing is launched if any task is
 * invalid. */
int chym_map_batch_workspace_size(const chym_map_problem *probs, const chym_run *runs, int32_t n_tasks,
                                  size_t *bytes);
int chym_map_batch(const chym_map_problem *probs, const chym_run *runs, int32_t n_tasks, void *workspace,
                   size_t ws_bytes, chym_stream_t stream);

/* Sign readout of x (paper: the Ising spins are read at the end of a run).
 * spins [r][ceil(n/64)], extra_frac [r], diverged [r]; each may be NULL. */
int chym_readout(int32_t n, int32_t d, int32_t r, const float *x, uint64_t *spins,
                 double *extra_frac, uint8_t *diverged, chym_stream_t stream);

/* Ising energy E_i = -sum_{p,q} J_pq sigma_p sigma_q of each readout (paper:
 * the Ising Hamiltonian; Eq. (3) with D = 1).  e_i32 [r] is exact and allowed
 * for CHYM_J_I8 only (|E| must fit int32, n <= 2048); e_f64 [r] for any J.
 * Either may be NULL. */
int chym_ising_energy(int32_t n, int32_t r, const void *j, int32_t j_dtype,
                      const uint64_t *spins, int32_t *e_i32, double *e_f64,
                      chym_stream_t stream);

/* Hyperspin energy of Eq. (3), E_hs = -sum_{p,q} J_pq u_p . u_q with unit
 * vectors u_p = x_p / |x_p| (0 for a zero hyperspin), in float64.
 * n <= 2048, n * d <= 8192. */
int chym_hs_energy(int32_t n, int32_t d, int32_t r, const void *j, int32_t j_dtype,
                   const float *x, double *e_hs, chym_stream_t stream);

/* Whole run: integrate run->steps steps; if 0 < ss_step < steps and e_hs_ss
 * is not NULL, record the hyperspin energy after ss_step steps (the
 * hyperspin steady state before annealing); then fill every non-NULL output
 * of *out from the final state. */
int chym_solve(const chym_problem *prob, const chym_run *run, int32_t ss_step,
               double *e_hs_ss, const chym_out *out, chym_stream_t stream);

/* chym_solve with a caller workspace (see chym_integrate_ws). */
int chym_solve_ws(const chym_problem *prob, const chym_run *run, int32_t ss_step, double *e_hs_ss,
                  const chym_out *out, void *workspace, size_t ws_bytes, chym_stream_t stream);

/* ------------------------------------------------------------------------
 * Batched form: many problems (instances of different n, d, replica counts,
 * pumps, step counts) integrated by one launch.  Paper: the statistics are
 * gathered over N_g graphs x N_s pump values x N_r runs, all independent
 * (statistics paragraph and Fig. 4).
 *
 * Tasks are grouped by kernel variant (row tiles, d, precision, coupling
 * storage); each group runs as one persistent kernel whose wavefronts (or
 * blocks) pop (task, replica group) work items, longest first, from a
 * counter in the workspace.  Sparse-row couplings (CHYM_J_ELL) form one
 * group per d on the gather integrator; their Ising energies come out in
 * e_ising_f64 (e_ising is for CHYM_J_I8 only).  The groups run as parallel
 * branches of one HIP graph.  After integration every task's non-NULL
 * outputs are filled from its final state, as chym_solve does.
 */
typedef struct chym_task {
    chym_problem prob;
    chym_run run;
    chym_out out;
} chym_task;

typedef struct chym_batch chym_batch; /* opaque plan (host object owned by the library) */

/* Device workspace bytes a batch of these tasks (host array) needs. */
int chym_batch_workspace_size(const chym_task *tasks, int32_t n_tasks, size_t *bytes);

/* Validate every task (host array), write the task table and the work list
 * into the caller's device workspace (a synchronous host-to-device copy;
 * the workspace must stay allocated and untouched while the plan lives) and
 * record the launch sequence as a HIP graph.  The task arrays (J, pump, x,
 * alpha, outputs) are referenced, not copied: launches read and write them
 * as they are at launch time. */
int chym_batch_create(const chym_task *tasks, int32_t n_tasks, void *workspace, size_t ws_bytes,
                      chym_batch **plan);

/* Run the batch: one hipGraphLaunch on stream.  Launches of one plan must
 * not overlap (they share the work counters). */
int chym_batch_launch(const chym_batch *plan, chym_stream_t stream);

/* Same work as chym_batch_launch, issued as plain kernel launches on stream
 * (no graph). */
int chym_batch_launch_nograph(const chym_batch *plan, chym_stream_t stream);

/* Free the plan (host object, graph and its private streams); the caller's
 * workspace is not touched.  Waits for the plan's outstanding launches. */
int chym_batch_destroy(chym_batch *plan);

/* One-shot batched solve: the work of chym_batch_create + one
 * chym_batch_launch_nograph + chym_batch_destroy, without a HIP graph and
 * without keeping a plan.  The task table is copied into the caller's
 * workspace (size from chym_batch_workspace_size, 256-byte aligned) on
 * `stream`, which is synchronized once before the launches are queued; the
 * launches then run asynchronously on `stream`.  Results are those of the
 * plan's launches, bit for bit (and so those of one chym_solve per task).
 * Calls that share a workspace must not overlap.  Errors name the offending
 * task; nothing is launched if any task is invalid. */
int chym_solve_batched(const chym_task *tasks, int32_t n_tasks, void *workspace, size_t ws_bytes,
                       chym_stream_t stream);

/* ------------------------------------------------------------------------
 * Learned early restart.  A small network predicts, from features of the
 * first part of a run, whether the run will reach the Ising ground state;
 * runs predicted to fail are restarted from fresh initial states, and every
 * kept run is still integrated to the end and scored exactly.
 *
 * Features: CHYM_FEATURES = 8 checkpoints x 4 values per replica, stored
 * [r][CHYM_FEATURES] float32; checkpoint k fills columns 4k .. 4k+3 with
 *   R1            -(x_1^T J x_1) / (n x_1^T x_1): the Rayleigh quotient per
 *                 spin of the first components x_{p,1} (0 if they are all 0)
 *   E / n         Ising energy per spin of the current sign readout
 *   share1        sum_p x_{p,1}^2 / sum_{p,mu} x_{p,mu}^2, the first
 *                 component's share of the squared norm (0 for a zero state)
 *   flips / n     fraction of spins whose sign changed since the previous
 *                 checkpoint (sign words in prev_words, updated in place)
 * (float32 arithmetic).  All four concern the first component, the one the
 * anneal keeps and the readout reads: runs of one problem and pump reach the
 * same hyperspin configuration up to a rotation, and its orientation, not
 * rotation-invariant quantities such as E_hs, tells them apart.  Before the
 * network the features are standardized within each pump's batch of runs
 * (chym_feature_standardize), since the restart policy ranks runs within
 * such a batch.
 * Network: CHYM_FEATURES -> 128 -> 128 -> 1, ReLU, sigmoid output, binary
 * cross-entropy; parameters in one block of CHYM_MLP_PARAMS values in the
 * order W1 [128][32], b1 [128], W2 [128][128], b2 [128], w3 [128], b3, held
 * as a float32 master copy and a bf16 copy (bf16 bit patterns) that the
 * forward and backward passes read.  The hidden layers run on the matrix
 * cores: each one's input (the features, then the first layer's
 * activations) is rounded to bf16 (nearest even) and its products summed in
 * float32 with its float32 bias; the output layer is a float32 dot product.
 * The backward pass takes each rounding as the identity (straight-through):
 * a layer's weight gradient uses its rounded input.
 */
#define CHYM_FEATURES 32
#define CHYM_MLP_PARAMS 20865

/* Sign words [r][ceil(n/64)] of x (bit set iff x_{p,1} >= 0): the reference
 * of the first checkpoint. */
int chym_sign_words(int32_t n, int32_t d, int32_t r, const float *x, uint64_t *words, chym_stream_t stream);

/* Features of checkpoint `checkpoint` (0..7) of every replica of x; dense
 * couplings, n <= 8192. */
int chym_features(int32_t n, int32_t d, int32_t r, const void *j, int32_t j_dtype, const float *x,
                  uint64_t *prev_words, float *features, int32_t checkpoint, chym_stream_t stream);

/* Standardizes features [groups * group][CHYM_FEATURES] within each group of
 * `group` consecutive replicas (one pump's batch of runs): every column
 * becomes (f - mean) / sd with the group's mean and population standard
 * deviation (0 where sd = 0).  Deterministic; `out` may be `in`. */
int chym_feature_standardize(int32_t groups, int32_t group, const float *in, float *out, chym_stream_t stream);

/* For each group of `group` consecutive scores (one pump's batch of runs),
 * the indices of its `keep` highest scores (equal scores: the lower index
 * first; NaN ranks lowest), in ascending order, as global replica indices:
 * idx [groups][keep] int32.  1 <= keep <= group. */
int chym_select_top(int32_t groups, int32_t group, int32_t keep, const float *score, int32_t *idx,
                    chym_stream_t stream);

/* Copies the runs idx[0 .. m) of x_src [n][r_src][d] into x_dst [n][m][d]
 * (run j of x_dst is run idx[j] of x_src) and, if pump_dst is not NULL,
 * their pumps into pump_dst [m].  Every idx entry must lie in [0, r_src)
 * (device data, not checked: chym_select_top writes such indices). */
int chym_gather_replicas(int32_t n, int32_t d, int32_t r_src, const float *x_src, const float *pump_src, int32_t m,
                         const int32_t *idx, float *x_dst, float *pump_dst, chym_stream_t stream);

/* Float scratch the backward pass needs for a batch. */
int chym_mlp_scratch_floats(int32_t batch, size_t *floats);

/* Forward pass: logit [batch]; h1, h2 [batch][128] (post-ReLU activations,
 * h1 as rounded to bf16 for the second layer; may be NULL unless a backward
 * pass follows). */
int chym_mlp_forward(int32_t batch, const float *features, const uint16_t *w_bf16, float *logit, float *h1, float *h2,
                     chym_stream_t stream);

/* Gradient of the mean binary cross-entropy over the batch (labels 0/1 as
 * float) with respect to the parameters (grad [CHYM_MLP_PARAMS]), and each
 * sample's loss term (loss [batch]).  Deterministic.  scratch: see
 * chym_mlp_scratch_floats. */
int chym_mlp_backward(int32_t batch, const float *features, const float *labels, const uint16_t *w_bf16,
                      const float *logit, const float *h1, const float *h2, float *scratch, float *grad, float *loss,
                      chym_stream_t stream);

/* One Adam step (Kingma & Ba) on the float32 master weights (step count
 * t >= 1 for the bias corrections); refreshes the bf16 copy. */
int chym_mlp_adam(float *w_master, uint16_t *w_bf16, float *m, float *v, const float *grad, float lr, float beta1,
                  float beta2, float eps, int32_t t, chym_stream_t stream);

/* bf16 copy (round to nearest even) of n float32 values. */
int chym_to_bf16(const float *src, uint16_t *dst, int32_t n, chym_stream_t stream);

/* ------------------------------------------------------------------------
 * Launch plans and the autotuner.  A plan entry picks, for one kernel
 * variant (n rounded up to 16-row tiles, d, precision, J storage), how the
 * batched path runs it:
 *   CHYM_KERNEL_REGJ  each wavefront gathers J into its own registers and
 *                     takes work items of 16 replicas (one wavefront per
 *                     SIMD when the state is large);
 *   CHYM_KERNEL_LDSJ  a block of `waves` wavefronts stages J once in LDS and
 *                     takes work items of 16 * waves replicas, leaving
 *                     registers for two wavefronts per SIMD;
 *   CHYM_KERNEL_LDSJ1 the same with one wavefront per SIMD (the whole
 *                     register file for each wave);
 *   CHYM_KERNEL_PIPE  J in LDS as for LDSJ1, with the step loop software-
 *                     pipelined: the vector work of one step runs between
 *                     the matrix-core products of the next;
 *   CHYM_KERNEL_LDSJ3 as LDSJ, with registers for three wavefronts per SIMD
 *                     (built where the step loop fits in 168 registers:
 *                     up to 10 row tiles at d = 1, 7 at d = 2, 4 at d = 3,
 *                     3 at d = 4; 8, 5, 3, 3 with float couplings in the
 *                     float32 form);
 *   CHYM_KERNEL_SLAB  the streamed-J kernel, for the variants beyond the
 *                     register-resident ones (its only kind there): `waves`
 *                     is its block size, 8 (two wavefronts per SIMD) or 16
 *                     (four per SIMD, bf16 form, up to 32 row tiles, or
 *                     64 at d <= 2).
 * The table is process-wide and starts empty: CHYM_KERNEL_REGJ with 4 waves
 * per block for the register-resident variants, CHYM_KERNEL_SLAB with 16
 * waves up to 32 row tiles where built and 8 beyond for the streamed-J ones.
 * The single-problem calls (chym_integrate_ws, chym_solve_ws) use the
 * streamed-J entries too.  Plans change speed only, never results.
 */
#define CHYM_KERNEL_AUTO 0
#define CHYM_KERNEL_REGJ 1
#define CHYM_KERNEL_LDSJ 2
#define CHYM_KERNEL_LDSJ1 3
#define CHYM_KERNEL_PIPE 4  /* J in LDS, one wavefront per SIMD that interleaves the update of the previous
                               step and the operand split with the current step's products (two accumulator
                               sets); built for d = 2, 3 and 2 to 7 row tiles with couplings in one bf16
                               term (any storage in the bf16 form; int8, bf16 or FP8 in the float32 form) */
#define CHYM_KERNEL_SLAB 5  /* the streamed-J kernel (n beyond the register-resident variants) */
#define CHYM_KERNEL_LDSJ3 6 /* J in LDS, three wavefronts per SIMD (where built) */

typedef struct chym_plan_entry {
    int32_t n;         /* problem size the entry applies to (any n with the same 16-row tile count) */
    int32_t d;
    int32_t precision; /* CHYM_PREC_* */
    int32_t j_dtype;   /* CHYM_J_* */
    int32_t kernel;    /* CHYM_KERNEL_REGJ, _LDSJ, _LDSJ1, _LDSJ3 or _PIPE for register-resident variants,
                          CHYM_KERNEL_SLAB for streamed-J ones (CHYM_KERNEL_AUTO: remove the entry);
                          a kind not built for the shape is refused with CHYM_EUNSUPPORTED */
    int32_t waves;     /* wavefronts per block: 1..4, or 8 or 16 for CHYM_KERNEL_SLAB */
    float ms;          /* autotune: measured time of the probe run of this entry (informational) */
    float reserved;    /* must be 0 */
} chym_plan_entry;

/* Install (or, with CHYM_KERNEL_AUTO, remove) a plan entry. */
int chym_plan_set(const chym_plan_entry *entry);

/* The entry the batched path will use for this problem shape (the default
 * when none was set). */
int chym_plan_get(int32_t n, int32_t d, int32_t precision, int32_t j_dtype, chym_plan_entry *entry);

/* Device workspace bytes chym_plan_autotune needs for `replicas` replicas. */
int chym_plan_autotune_workspace_size(int32_t n, int32_t d, int32_t replicas, int32_t steps, size_t *bytes);

/* Times every candidate plan for this problem shape on a synthetic problem
 * (+-1 or Gaussian J, `replicas` replicas, `steps` Euler steps) built in the
 * caller's workspace, installs the fastest, and returns it in *best.  The
 * candidates and their times are written to cand[0 .. *n_cand-1] when cand
 * is not NULL (capacity max_cand).  Synchronizes the host with the device. */
int chym_plan_autotune(int32_t n, int32_t d, int32_t precision, int32_t j_dtype, int32_t replicas, int32_t steps,
                       void *workspace, size_t ws_bytes, chym_plan_entry *best, chym_plan_entry *cand,
                       int32_t max_cand, int32_t *n_cand, chym_stream_t stream);

/* Bytes of a coupling matrix of n hyperspins stored as j_dtype. */
int chym_j_bytes(int32_t n, int32_t j_dtype, size_t *bytes);

/* Quantizes a float32 coupling matrix J [n][n] (device) into the CHYM_J_FP8
 * format at out (device, n * (n + 1) bytes).  Row p gets the exponent
 * e_p = the least integer with max_q |J_pq| <= 448 * 2^e_p (E_p = e_p + 127;
 * e_p = 0 for an all-zero row), then q_pq = J_pq / 2^e_p rounded to the
 * nearest E4M3 value, ties to even (values below the smallest subnormal
 * round to a signed zero).  A row holding a non-finite value, or whose e_p
 * falls outside [-127, 127], gets E_p = 0xff (NaN), so runs on it end
 * flagged as diverged.  Deterministic; no host synchronization. */
int chym_quantize_fp8(int32_t n, const float *j, uint8_t *out, chym_stream_t stream);

/* The three-term bf16 split that the float32 form feeds to the matrix
 * cores, exposed for verification: for each of the n floats of x (device),
 * hi[i], mid[i], lo[i] (device, bf16 bit patterns) satisfy
 * hi = round-to-nearest-even bf16 of x and hi + mid + lo == x exactly when
 * |x| >= 2^-100 (the residual terms are then normal floats; below that they
 * may be flushed to zero, an error of at most 2^-8 |x|).  n must be a
 * multiple of 8; hi, mid and lo 16-byte aligned. */
int chym_split3_bf16(const float *x, int64_t n, uint16_t *hi, uint16_t *mid, uint16_t *lo, chym_stream_t stream);

/* Write the plan table to / merge it from a text file (one entry per line:
 * tiles d precision j_dtype kernel waves ms). */
int chym_plan_save(const char *path);
int chym_plan_load(const char *path);

#ifdef __cplusplus
}
#endif

#endif /* CHYM_H */
