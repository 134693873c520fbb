/*
 * lmag.h -- C ABI of the Lindblad-Magnus pulse propagator for AMD MI355X (gfx950).
 *
 * The library evaluates, for piecewise control pulses on a small open quantum
 * system, the superoperator propagator of the Lindblad master equation and the
 * process fidelity against a target unitary, together with the gradient of that
 * fidelity with respect to every pulse amplitude:
 *
 *   L(t)   = -i (I (x) H(t) - H(t)^T (x) I)
 *            + sum_k [ conj(L_k) (x) L_k - 1/2 I (x) L_k^dag L_k
 *                      - 1/2 (L_k^dag L_k)^T (x) I ]            (paper Eq. 8)
 *   H(t)   = sum_c eps_c u_c(t) H_ctrl[c] + sum_i b_i H_static[i]
 *   Omega_n = int_slice L dt                                     (Eq. 13)
 *             [+ (sqrt(3) h^2 / 12) [L(tau_2), L(tau_1)], second order]
 *             [order 6: a1 + a3/12 + [-20 a1 - a3 + C1, a2 + C2] / 240 with
 *              a1 = h B2, a2 = (sqrt(15) h/3)(B3 - B1), a3 = (10 h/3)(B3 - 2 B2 + B1),
 *              C1 = [a1, a2], C2 = -[a1, 2 a3 + C1] / 60, B_k = L at the three
 *              Gauss-Legendre nodes of the slice]
 *   S_n    = exp(Omega_n)                                        (Eq. 14)
 *   U      = S_N ... S_1                                         (Eq. 15)
 *   F      = Re Tr(S_T^dag U) / d^2,  S_T = conj(U_T) (x) U_T
 *
 * The problem statement follows the paper's Sec. III: a system (Hamiltonian
 * terms and jump operators built from T1/T2, Sec. II-B and Eq. 8), a
 * coefficient matrix of slices x controls (Sec. III-C) and a target unitary
 * (Sec. III-C); the outputs are the propagator (Eq. 15) and a score with its
 * gradient for the optimiser (Sec. III-C).
 *
 * Conventions
 *  - Complex numbers are interleaved (re, im). Hilbert-space operators are
 *    row-major d x d. Superoperators are row-major n x n, n = d^2, in the
 *    column-stacking convention vec(rho)[i + d j] = rho[i][j].
 *  - Units are the caller's (e.g. rad/us and us); hbar = 1.
 *  - Every call returns an lmag_status. Nothing aborts and no C++ exception
 *    crosses the ABI. On a non-OK status lmag_last_error() describes it and no
 *    output has been written (argument errors are detected on the host before
 *    any launch).
 *  - Compute calls are asynchronous on the caller's HIP stream (hipStream_t
 *    passed as void*, NULL = default stream), with one exception: on the
 *    block-tiled path (n > 64) the call blocks the host once per call, after
 *    the slice exponents, to read the largest scaling exponent and Neumann
 *    level count that size its squaring and inverse loops. Errors raised by
 *    the device surface on a later call or on lmag_sync().
 *  - A context may be used from several streams: every compute call shares
 *    the context's workspace, so a call on a stream other than the previous
 *    call's first waits, on the device (hipStreamWaitEvent, the host does not
 *    block), for the previous call to finish.
 *  - Reductions are deterministic (no floating-point atomics): repeated calls
 *    on the same inputs give bitwise-identical results.
 *  - The library owns only its workspace, which lmag_destroy() frees. The
 *    caller owns every pointer it passes in.
 *  - Supported superoperator sizes: n = d^2 <= 64 (d = 2, 4 or 8; smaller
 *    systems are embedded in 64 x 64 tiles with zero padding), FP32 or FP64;
 *    and n a multiple of 64 up to 4096 (d = 16, 32 or 64), FP32 only, on the
 *    block-tiled path.
 *  - Test and instrumentation entry points are declared in lmag_debug.h.
 */
#ifndef LMAG_H
#define LMAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LMAG_OK = 0,
  LMAG_E_INVALID = -1,     /* bad argument (dimension, pointer, count, NaN in host data) */
  LMAG_E_NOSYSTEM = -2,    /* compute call before lmag_set_system */
  LMAG_E_NOMEM = -3,       /* device allocation failed */
  LMAG_E_DEVICE = -4,      /* HIP runtime / kernel error */
  LMAG_E_UNSUPPORTED = -5  /* valid request outside what the library supports */
} lmag_status;

enum { LMAG_F32 = 32, LMAG_F64 = 64 };
enum { LMAG_ZOH = 0, LMAG_FOH = 1 };

typedef struct lmag_ctx lmag_ctx;  /* opaque; one per (device, host thread) */

/* Library version string (static storage). */
const char *lmag_version(void);

/* Create a context bound to HIP device hip_device. *out receives the context
 * (NULL on failure). LMAG_E_DEVICE if no such device exists. */
lmag_status lmag_create(lmag_ctx **out, int hip_device);

/* Destroy a context and free its workspace. NULL is ignored. Waits for work
 * the context queued on its last stream. */
void lmag_destroy(lmag_ctx *ctx);

/* Message for the last non-OK status of this context (static storage of the
 * context, valid until the next call on it). */
const char *lmag_last_error(const lmag_ctx *ctx);

/* System description (Sec. II-B, Eq. 6 and 8). All pointers are HOST pointers;
 * the arrays are copied before the call returns and the caller keeps them. */
typedef struct {
  int d;                        /* Hilbert dimension: d*d <= 64, or d*d a multiple of  */
                                /* 64 up to 4096 (FP32 only)                          */
  int n_static;                 /* number of static Hamiltonian terms               */
  const double *H_static;       /* [n_static][d][d] complex (e.g. sigma_z_i / 2)     */
  int n_ctrl;                   /* number of control terms, <= 8                     */
  const double *H_ctrl;         /* [n_ctrl][d][d] complex (e.g. S_c . S_{c+1})       */
  int n_jump;                   /* number of jump operators                          */
  const double *L_jump;         /* [n_jump][d][d] complex, rates folded in (op/sqrt T) */
  int precision;                /* LMAG_F32 or LMAG_F64: compute type of the slices  */
  int magnus_order;             /* 1 (Eq. 13), 2 (adds the two-node Gauss-Legendre    */
                                /* commutator) or 6 (three Gauss-Legendre nodes,     */
                                /* nested commutators; FP32, d*d a multiple of 64,   */
                                /* block-tiled path)                                 */
  int hold;                     /* LMAG_ZOH (u constant per slice) or LMAG_FOH        */
                                /* (u linear from u_n to u_{n+1}; u_N := u_{N-1})   */
  size_t workspace_bytes_max;   /* 0 = 85 % of free device memory. Gradient calls    */
                                /* over it split into waves and, where one item (or  */
                                /* group) alone exceeds it, re-run each chunk's      */
                                /* forward in the adjoint instead of storing the     */
                                /* per-slice tiles (the suffix side is recomputed)   */
  int chunk_slices;             /* slices per work unit; 0 = automatic: the autotuned */
                                /* length if one is cached for this call's size, else */
                                /* one chunk per compute unit up to 64 slices per unit,*/
                                /* above that about four chunks per workgroup within  */
                                /* 64..256 slices (64 when the adjoint recomputes)    */
  int basis;                    /* representation of the superoperators in single  */
                                /* precision: 0 = the real basis of Hermitian       */
                                /* operators (every matrix of the path is real      */
                                /* there: one real MFMA product per complex one),   */
                                /* 1 = column stacking (complex). Results agree up  */
                                /* to rounding; the slice degrees and squarings can */
                                /* differ (each is chosen from the 1-norm of the    */
                                /* slice exponent in its own basis). Double         */
                                /* precision always uses column stacking.           */
} lmag_system_desc;

/* Install (or replace) the system. Builds the superoperator basis on the
 * device in FP64 (and an FP32 copy). Blocks until the basis is built.
 * LMAG_E_INVALID for bad dimensions/counts/NULL arrays or non-finite entries. */
lmag_status lmag_set_system(lmag_ctx *ctx, const lmag_system_desc *desc);

/* A batch of items (pulse x quasi-static noise sample). Metadata arrays are
 * HOST pointers; data arrays are DEVICE pointers of the caller. */
typedef struct {
  int n_items;
  const int32_t *n_slices;      /* HOST [n_items], each >= 1                         */
  const int64_t *slice_offset;  /* HOST [n_items], first row of the item in amps     */
  const void *amps;             /* DEVICE [rows][n_ctrl] real, compute type          */
  const double *static_coef;    /* DEVICE [n_items][n_static] (b_i incl. offsets); NULL = 0 */
  const double *ctrl_scale;     /* DEVICE [n_items][n_ctrl] (eps_c); NULL = 1        */
  double dt;                    /* slice width h > 0                                 */
  int n_groups;                 /* 0 = none; else items are averaged per group        */
  const int32_t *group_of_item; /* HOST [n_items] in [0, n_groups); items of a group
                                   must share slice_offset and n_slices              */
} lmag_batch;

/* The propagator of every item (Eq. 13-15): per slice the Magnus exponent
 * Omega_n (Eq. 13, plus the Gauss-Legendre commutator term at second order),
 * S_n = exp(Omega_n) by scale-and-square Pade (Eq. 14), and the ordered product
 * U = S_N ... S_1, later slices on the left (Eq. 15).
 * S_out: DEVICE [n_items][n][n] complex of the compute type: U of every item,
 * row-major, in column stacking whatever the system's basis (a propagator
 * computed in the basis of Hermitian operators is transformed back).
 * Items may share amplitude rows. */
lmag_status lmag_propagate(lmag_ctx *ctx, const lmag_batch *batch, void *S_out,
                           void *hip_stream);

/* Score and gradient for the pulse optimiser (Sec. III-C: the coefficient
 * matrix of slices x controls and a target unitary in, a score and its
 * gradient out): the process fidelity F = Re Tr(S_T^dag U) / d^2 against
 * S_T = conj(U_T) (x) U_T, with U as in lmag_propagate, and dF/du from the
 * hand-written adjoint (Frechet derivative of every slice exponential with the
 * prefix and suffix products of Eq. 15).
 * U_target:       DEVICE [n_targets][d][d] complex128
 * target_of_item: HOST [n_items] in [0, n_targets) or NULL (= target 0)
 * F_out:          DEVICE double [n_items] (or [n_groups] when grouped)
 * grad_out:       DEVICE like amps (compute type) or NULL for F only. With
 *                 groups, the group mean of dF/du is written at the rows of the
 *                 group's shared amplitudes. Rows that belong to no item are
 *                 left unchanged. With grad_out, the row ranges of different
 *                 items (of different groups, when grouped) must not overlap
 *                 (LMAG_E_INVALID): items that share a pulse go into one group. */
lmag_status lmag_fidelity_and_grad(lmag_ctx *ctx, const lmag_batch *batch,
                                   const void *U_target, int n_targets,
                                   const int32_t *target_of_item, double *F_out,
                                   void *grad_out, void *hip_stream);

/* lmag_fidelity_and_grad without any allocation, for callers that cannot
 * allocate device memory during the call: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc. Same arguments, results and
 * kernels as lmag_fidelity_and_grad, for systems with n = d*d <= 64 (else
 * LMAG_E_UNSUPPORTED). The call makes no hipMalloc, hipFree, pinned-host or
 * other device allocation: its workspace is a fixed scratch array of 64 MiB
 * compiled into the library, one copy per GPU (held from the first context on
 * that GPU until the process ends); the plan metadata is staged through a
 * pageable host buffer of the context. A batch whose workspace exceeds the
 * scratch (about 160 KiB per slice and 192 KiB per chunk in FP32 with the
 * gradient; twice that in FP64) is rejected with LMAG_E_INVALID and nothing is
 * launched; it is never split into waves or recomputed. Every call on one GPU,
 * from any context, shares that GPU's scratch and leaves its contents behind
 * (the work counters are cleared by a kernel at the start of each call): calls
 * that overlap in time on one GPU race and must be ordered by the caller.
 * Calls on one context are ordered as for the other compute calls. */
lmag_status lmag_fidelity_and_grad_noalloc(lmag_ctx *ctx, const lmag_batch *batch,
                                           const void *U_target, int n_targets,
                                           const int32_t *target_of_item, double *F_out,
                                           void *grad_out, void *hip_stream);

/* Logical-subspace score of the propagator and (optionally) its gradient
 * (Sec. III-C, Eq. 16-17). With P the n x L matrix whose columns are the
 * vectorised (column-stacked) logical operators, every item's U is projected to
 * Pi = P^dag U P (Eq. 16) and scored:
 *   LMAG_SCORE_PROJECTED: s = ||Pi - T||_F^2 = Tr((Pi - T)^dag (Pi - T)), the
 *     Frobenius loss of Eq. 17 (read with the conjugate transpose);
 *   LMAG_SCORE_LINEAR:    s = Re Tr(T^dag Pi) / L (for the operator basis
 *     |a><b| of a logical qubit and T = conj(V) (x) V: the gate's process
 *     fidelity restricted to the logical subspace).
 * The gradient is that of s (with the fidelity's conventions for groups).
 * kind:            LMAG_SCORE_PROJECTED or LMAG_SCORE_LINEAR
 * L:               1..4 logical operators
 * P:               HOST double [L][n][2] (column k = vec of operator k, complex)
 * T:               DEVICE [n_targets][L][L] complex128, row-major
 * target_of_item:  HOST [n_items] in [0, n_targets) or NULL (= target 0)
 * score_out:       DEVICE double [n_items] (or [n_groups] when grouped)
 * grad_out:        DEVICE like amps, or NULL for the score only.
 * Systems with n = d * d <= 64 only (LMAG_E_UNSUPPORTED otherwise). */
enum { LMAG_SCORE_PROJECTED = 1, LMAG_SCORE_LINEAR = 2 };
lmag_status lmag_logical_score_and_grad(lmag_ctx *ctx, const lmag_batch *batch, int kind, int L,
                                        const double *P, const void *T, int n_targets,
                                        const int32_t *target_of_item, double *score_out,
                                        void *grad_out, void *hip_stream);

/* Autotuner: times lmag_fidelity_and_grad on this batch (reps timed calls
 * after one warm-up, HIP events on the stream) over a set of candidates.
 * Block-tiled systems (n > 64): the product kernel -- 0: one 64 x 64 output
 * tile per workgroup with the B tile in registers, 16x16x4 MFMA; 1: a 32 x 32
 * quadrant per wave with both operand tiles in LDS and the next k-step's tiles
 * loaded during the products, 16x16x4 MFMA; 2: as 1 with the 32x32x2 MFMA;
 * 3: as 1 with every FP32 operand split into three bfloat16 pieces and each
 * real product formed from the six leading cross terms on the 16x16x32 bf16
 * MFMA (FP32-level error); 4: as 0 with two output tiles (eight waves) per
 * workgroup sharing each staged A tile (n / 64 even); 5: as 0 with every
 * product's tiles on one XCD (n <= 1024); 6: as 0 without the operand pipeline,
 * three workgroups per CU; 7: as 6 with the grouping of 5; 8: as 0 with the A
 * tiles double-buffered in LDS by direct global-to-LDS loads (grouped as 5
 * where n <= 1024) -- at the automatic chunk length, half and twice it. In the
 * real basis of Hermitian operators (basis 0) the candidates are the real
 * product kernel (0) and, where n <= 1024, the same with the grouping of 5 (5).
 * 64 x 64 systems: the
 * persistent slice kernels, for every candidate chunk length (slices per work
 * unit) and the inverse variants
 * of the Pade step (0: per slice the cheapest whose error bound holds -- in
 * single precision r_2 itself by its power series truncated at degree 4
 * (Pade-2) or 1/q_3 by its truncated power series (Pade-3), else the MFMA
 * binary-Neumann product, else Gauss-Jordan; 1: Gauss-Jordan always; 2: Neumann
 * where its bound allows, else Gauss-Jordan; 1 and 2 always form
 * r_m = q_m^{-1} p_m). The fastest pair is kept
 * for calls with chunk_slices = 0 whose precision, representation, order, d
 * and total slice count (power-of-two bucket) match (key
 * "p<precision>[h]_o<order>_d<d>_s<log2 slices>", h for the real basis), and
 * appended as one JSON line {"key", "chunk", "variant", "ms"} to the file
 * named by the environment
 * variable LMAG_TUNE_CACHE if it is set. With LMAG_TUNE_VERBOSE set, each
 * candidate's time is written to stderr as it is measured.
 * best_out: HOST int32 [2] (chunk, variant: inverse variant or product kernel)
 * or NULL; best_ms_out: HOST or NULL.
 * Blocks. Outputs of the timed calls go to internal buffers. */
lmag_status lmag_autotune(lmag_ctx *ctx, const lmag_batch *batch, const void *U_target,
                          int n_targets, const int32_t *target_of_item, int reps,
                          int32_t *best_out, double *best_ms_out, void *hip_stream);
/* Load tuning lines written by lmag_autotune (path: HOST string). Lines that
 * do not parse are skipped. */
lmag_status lmag_load_tuning(lmag_ctx *ctx, const char *path);

/* Wait for the stream and report any pending device error. */
lmag_status lmag_sync(lmag_ctx *ctx, void *hip_stream);

/* Optimiser step on pulse amplitudes (the paper's Adam step, Sec. III-C,
 * Kingma & Ba 2015 Alg. 1) followed by projection onto [lo, hi]:
 *   g <- grad_scale * grad;  m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2
 *   amps <- clip(amps - lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps), lo, hi)
 * amps, grad, m_state, v_state: DEVICE [rows][n_ctrl] of the compute type of
 * `precision` (m, v zero before step 1); step >= 1. row_active: DEVICE
 * uint8 [rows] or NULL; rows with 0 are left unchanged (state included).
 * grad_scale = -1 ascends F (descends 1 - F). */
lmag_status lmag_adam_project(lmag_ctx *ctx, int precision, int64_t rows, int n_ctrl,
                              void *amps, const void *grad, void *m_state, void *v_state,
                              int step, double lr, double beta1, double beta2, double eps,
                              double grad_scale, double lo, double hi,
                              const uint8_t *row_active, void *hip_stream);

/* ---- Learned pulse proposal: multilayer perceptron kernels ----------------
 * bfloat16 operands (uint16_t storage, round to nearest even), FP32
 * accumulation on MFMA. All arrays are DEVICE, row-major. */
enum { LMAG_ACT_GELU = 1, LMAG_ACT_SIGMOID = 2 };

/* Forward of one Linear layer: pre = X W^T + b.
 * X: bf16 [rows][n_in]; W: bf16 [n_out][n_in]; b: fp32 [n_out].
 * pre_out: fp32 [rows][n_out] (needed by the backward) or NULL.
 * act = LMAG_ACT_GELU:    Y = bf16 [rows][n_out] = bf16(gelu(pre)), gelu exact (erf).
 * act = LMAG_ACT_SIGMOID: Y = fp32 [rows][n_out] = scale * sigmoid(pre). */
lmag_status lmag_mlp_forward(lmag_ctx *ctx, int rows, int n_in, int n_out, const uint16_t *X,
                             const uint16_t *W, const float *b, int act, float scale,
                             float *pre_out, void *Y, void *hip_stream);

/* Backward of one Linear layer given G = dL/dpre: bf16 G16 [rows][n_out] for
 * the products and fp32 G32 [rows][n_out] for the bias sum.
 * dW: fp32 [n_out][n_in] = G^T X;  db: fp32 [n_out] = column sums of G32.
 * If dprev16 != NULL: the gradient of the previous layer's pre-activation,
 * (G W) * gelu'(pre_prev), with pre_prev fp32 [rows][n_in], is written as
 * bf16 dprev16 and fp32 dprev32 [rows][n_in]. */
lmag_status lmag_mlp_backward(lmag_ctx *ctx, int rows, int n_in, int n_out, const uint16_t *X,
                              const uint16_t *W, const uint16_t *G16, const float *G32,
                              float *dW, float *db, const float *pre_prev, uint16_t *dprev16,
                              float *dprev32, void *hip_stream);

/* Mean squared error of sigmoid(z) against targets y in [0, 1] (z, y fp32 [n]):
 * loss (DEVICE double [1]) = mean((sigmoid(z) - y)^2); dz = dloss/dz as fp32
 * dz32 and bf16 dz16 [n] (either may be NULL). Deterministic. */
lmag_status lmag_mlp_mse(lmag_ctx *ctx, int64_t n, const float *z, const float *y, float *dz32,
                         uint16_t *dz16, double *loss, void *hip_stream);

/* out[i] = bf16(in[i]), round to nearest even; n elements. */
lmag_status lmag_cast_bf16(lmag_ctx *ctx, const float *in, uint16_t *out, int64_t n,
                           void *hip_stream);

/* Host-only queries (no device needed). */
/* Pade coefficients b_0..b_m of r_m = p_m / p_m(-x), m in {2, 3, 5, 7}. */
lmag_status lmag_pade_coefficients(int m, double *b_out);
/* theta_m used for degree and scaling selection: precision LMAG_F32 (m in
 * {2, 3}) or LMAG_F64 (m in {3, 5, 7}). */
lmag_status lmag_pade_theta(int precision, int m, double *theta_out);

/* Histogram of the (m, s) selections of the last forward pass of this context:
 * counts[m_index * 64 + s], m_index 0/1/2/3 for m = 2/3/5/7. Blocks (syncs the
 * stream of the last call). */
lmag_status lmag_last_selection_histogram(lmag_ctx *ctx, int64_t *counts_out /*[4*64]*/);

/* Per-stage kernel timers measured with HIP events recorded on the caller's
 * stream around every launch (the stream the kernels run on). Stages:
 * 0 Magnus coefficients, 1 slice exponents (Omega, FP64 norm, scaling),
 * 2 forward slices (Pade, chunk product), 3 chunk scan, 4 environments +
 * fidelity, 5 backward slices (adjoint), 6 basis traces, 7 chain rule.
 * enable = 0 turns recording off (default). */
enum { LMAG_STAGES = 8 };
lmag_status lmag_set_profiling(lmag_ctx *ctx, int enable);
/* Sum of stage durations (ms) and launch counts since the previous read; blocks
 * until the recorded work has finished, then clears the record. */
lmag_status lmag_read_profile(lmag_ctx *ctx, double *ms_out /*[LMAG_STAGES]*/,
                              int64_t *count_out /*[LMAG_STAGES]*/);
/* Plan of the last wave of the last compute call: total slices, total chunks,
 * slices per chunk, workgroups of the persistent slice kernels, workspace bytes
 * in use, recompute mode (1 = the backward re-ran each chunk's forward instead of
 * reading stored per-slice tiles), number of waves the call was split into to
 * fit workspace_bytes_max (or 85 % of free device memory), and the number of
 * support positions of the system's sparse basis tables (0: the basis is too
 * dense and the dense Omega and trace kernels are used; also 0 for systems
 * larger than one tile). */
lmag_status lmag_last_plan(lmag_ctx *ctx, int64_t *out /*[8]*/);

#ifdef __cplusplus
}
#endif

#endif /* LMAG_H */
