/*
 * opf.h -- C-ABI of the MI355X polar AC-OPF callback library (libopf.so).
 *
 * The library evaluates, on the GPU and in FP64, the callbacks an
 * interior-point solver calls every iteration (the NLPModels template of
 * the paper, Listing 1: obj, grad!, cons!, jac!, hess! with obj_weight) for
 * the polar AC optimal power flow model the paper builds in Listing 3, its
 * multi-period variant with generator ramp limits (Sec. III-C2) and a
 * security-constrained variant with N-1 branch-outage copies that share
 * generator set-points (the contingency structure of the GOC3 model,
 * Sec. III-C4).
 *
 * Conventions
 *  - Indices are 0-based int32; counts are int64; values are IEEE FP64.
 *  - Host structures (opf_case, opf_opts) are read during the call only.
 *  - Every per-call buffer (x, y, outputs, structure arrays) is a
 *    caller-owned DEVICE pointer on the model's device, contiguous.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Evaluation calls
 *    only enqueue kernels: results are valid once the stream has been
 *    synchronised.  No call synchronises the host or copies between host
 *    and device, except opf_model_create / opf_batch_create (one upload).
 *  - Every function returns 0 (OPF_OK) or a negative error code; the text of
 *    the last error on the calling thread is returned by opf_last_error().
 *    Faults inside a kernel surface at the next synchronisation.  NaN or Inf
 *    inside x or y propagate to the outputs and are not reported.
 *  - One model (or batch) must not be evaluated concurrently from two
 *    streams; different models are independent.
 *
 * Variable vector x (n entries), blocks in this order (Listing 3):
 *    va [N*P] | vm [N*P] | pg [G*Pg] | qg [G*P] | p [2L*P] | q [2L*P]
 *  P = replicas: n_periods (multi-period) or n_cont + 1 (contingency copies,
 *  copy 0 is the base case), else 1; Pg = 1 with contingency copies (pg is
 *  shared), else P.  Inside a block the entity index runs fastest, then the
 *  replica.  Arc a < L is the from-side arc of branch a (at f_bus), arc L+l
 *  the to-side arc of branch l (at t_bus).
 *
 * Constraint vector c (m entries), blocks in Listing 3 order, each
 * entity-fastest over the replicas:
 *    ref [R] | p_fr [L] | q_fr [L] | p_to [L] | q_to [L] | angle [L] |
 *    balance_p [N] | balance_q [N] | thermal_fr [L] | thermal_to [L]
 *  followed, for n_periods = T > 1, by ramp rows [G*(T-1)].
 *    ref          va_r                                     = 0
 *    flow         p_a - F_a(vm_f, vm_t, va_f - va_t)        = 0   (pi model)
 *    angle        va_f - va_t                   in [angmin, angmax]
 *    balance_p    pd + gs vm^2 + sum_arcs p_a - sum_gens pg = 0
 *    balance_q    qd - bs vm^2 + sum_arcs q_a - sum_gens qg = 0
 *    thermal      p_a^2 + q_a^2 - rate_a^2                 <= 0
 *    ramp         pg_{k,t} - pg_{k,t-1}     in +-ramp_ratio * pmax_k
 *  and then the storage rows soc | loss_p | loss_q | thermal | (comp) and
 *  the device rows ramp [D*(T-1)] | init [D] (opf_storage, opf_devices),
 *  each entity-fastest over the periods.  Storage units and devices add
 *  the variable blocks ps | qs | qsc | se | sc | sd | u after q, and their
 *  terms +ps, +cp u (+qs, +cq u) to the balance rows of their bus.
 *  In contingency copy s >= 1 the branch outaged_branch[s-1] carries no
 *  flow (its admittance terms are zero; its rows and pattern entries stay)
 *  and its angle row is unbounded.
 *
 * Objective f = sum over pg variables of c2 pg^2 + c1 pg + c0.
 *
 * Sparsity patterns are structural (independent of values), fixed at model
 * creation:
 *  - Jacobian: COO sorted by (row, col), unique.
 *  - Hessian of the Lagrangian obj_weight * hess f + sum_i y_i hess c_i:
 *    lower triangle (row >= col), sorted by (row, col), unique.
 */
#ifndef OPF_H
#define OPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
enum {
    OPF_OK = 0,
    OPF_E_ARG = -1,    /* NULL pointer, size or index out of range          */
    OPF_E_CASE = -2,   /* the network data fails validation                 */
    OPF_E_NOMEM = -3,  /* device or host allocation failed                  */
    OPF_E_HIP = -4,    /* HIP runtime or kernel launch error                */
    OPF_E_STATE = -5   /* destroyed or mismatched handle                    */
};

/* Text of the last error raised on the calling thread ("" if none). */
const char *opf_last_error(void);

/* ---------------------------------------------------------------- input */
typedef struct {
    int32_t n_bus, n_branch, n_gen, n_ref;
    const double *pd, *qd, *gs, *bs, *vmin, *vmax;        /* [n_bus]      */
    const int32_t *ref_bus;                               /* [n_ref]      */
    const int32_t *f_bus, *t_bus;                         /* [n_branch]   */
    const double *r, *x, *b, *tap, *shift, *rate_a;       /* [n_branch]   */
    const double *angmin, *angmax;                        /* [n_branch]   */
    const int32_t *gen_bus;                               /* [n_gen]      */
    const double *pmin, *pmax, *qmin, *qmax, *c2, *c1, *c0; /* [n_gen]    */
} opf_case;
/* Branch data is per unit with the pi model of the paper's formulation
 * (PowerModels): series impedance r + jx, total line charging b split b/2
 * per side, an ideal transformer of ratio tap and phase shift `shift`
 * (radians) on the from side. */

/* Storage units (Sec. III-C3: the multi-period model with storage; its
 * formulation is the storage model of Geth, Coffrin and Fobes 2020 that the
 * paper cites).  Per unit u at bus i and period t the variables are ps, qs
 * (the power the unit draws from the grid, a load in the balance rows),
 * qsc (the converter's reactive set-point), se (stored energy), sc, sd
 * (charging and discharging power), with bounds ps, qsc in +-rating,
 * qs in [qmin, qmax], se in [0, emax], sc in [0, chmax], sd in [0, dismax];
 * and the rows
 *   soc     se_t - se_{t-1} - dt (eta_c sc_t - sd_t / eta_d) = 0
 *           (se_{-1} = e0, the initial energy)
 *   loss_p  ps + sd - sc - ploss - r (ps^2 + qs^2) / vm_i^2   = 0
 *   loss_q  qs - qsc - qloss - x (ps^2 + qs^2) / vm_i^2       = 0
 *   thermal ps^2 + qs^2 - rating^2                           <= 0
 *   comp    sc sd <= 0 (with sc, sd >= 0: sc sd = 0)  only if comp != 0
 * Polar form only; not combined with contingency copies. */
typedef struct {
    int32_t n;                  /* units                                    */
    const int32_t *bus;         /* [n]                                      */
    const double *emax, *chmax, *dismax, *rating, *qmin, *qmax;    /* [n]   */
    const double *eta_c, *eta_d, *r, *x, *ploss, *qloss, *e0;      /* [n]   */
    double dt;                  /* duration of one period                   */
    int32_t comp;               /* 1: add the complementarity rows          */
} opf_storage;

/* User-extension devices (Sec. III-D: components a user adds to a built
 * model, the electrolyzer example of Listing 10), linear: per device d at
 * bus i and period t one variable u in [lo, hi]; the objective gains
 * cost u; the balance rows of bus i gain cp u (active) and cq u (reactive),
 * both entries structural; rows ramp u_t - u_{t-1} in +-ramp (t >= 1) and
 * init u_0 in [init_lo, init_hi].  Not combined with contingency copies. */
typedef struct {
    int32_t n;                  /* devices                                  */
    const int32_t *bus;         /* [n]                                      */
    const double *cp, *cq, *cost, *lo, *hi, *ramp, *init_lo, *init_hi; /* [n] */
} opf_devices;

typedef struct {
    int32_t n_periods;          /* >= 1; 1 = static model                   */
    const double *pd_t, *qd_t;  /* [n_periods*n_bus] bus fastest; NULL =    */
                                /* use the case loads in every period       */
    double ramp_ratio;          /* ramp bound = ramp_ratio * pmax (T > 1)   */
    int32_t n_cont;             /* contingency copies (0 = none); cannot be */
                                /* combined with n_periods > 1              */
    const int32_t *outaged_branch; /* [n_cont] branch out in copy s+1       */
    int32_t form;               /* OPF_FORM_POLAR (0) or OPF_FORM_RECT (1)  */
    const opf_storage *storage; /* NULL = none                              */
    const opf_devices *devices; /* NULL = none                              */
} opf_opts;
/* opts may be NULL: static polar model.
 *
 * form = OPF_FORM_RECT is the rectangular form (Sec. III-C1, form = :rect):
 * the two bus blocks hold vr, vi (V = vr + j vi) in place of va, vm, and
 * the rows are those of the ACR formulation of the cited PowerModels:
 *    ref          vi_r                                        = 0
 *    flow         p_a - F_a(V_f, V_t)                         = 0
 *                 F = alpha |V_f|^2 + beta |V_t|^2 + a CR + b SI with the
 *                 polar coefficients, CR = vr_f vr_t + vi_f vi_t,
 *                 SI = vi_f vr_t - vr_f vi_t (= vm_f vm_t cos / sin th)
 *    angle        SI - tan(angmax) CR   <= 0
 *    angle_lo     SI - tan(angmin) CR   >= 0     (a second row per branch)
 *    balance      as polar with vm^2 = vr^2 + vi^2
 *    thermal      as polar
 *    vmag         vr^2 + vi^2              in [vmin^2, vmax^2]  (per bus)
 *  Constraint blocks: ref | p_fr | q_fr | p_to | q_to | angle | angle_lo |
 *  balance_p | balance_q | thermal_fr | thermal_to | vmag | (ramp).
 *  Bounds: vr, vi in [-vmax, vmax]; start point vr = 1, all else 0. */
enum { OPF_FORM_POLAR = 0, OPF_FORM_RECT = 1 };

/* Maximum number of branches at one bus. */
#define OPF_MAX_DEGREE 1024

/* ------------------------------------------------ host-only helpers */
/* These run on the host only and need no GPU. */

/* Validate the case and options.  OPF_E_CASE with a message naming the
 * first offending item (bus, branch, generator, outage index, impedance,
 * tap, bound order, degree limit, size limits); OPF_E_ARG for NULL arrays. */
int opf_case_validate(const opf_case *cs, const opf_opts *opts);

/* Sizes of the model: variables n, constraints m, Jacobian and Hessian
 * nonzeros.  Any output pointer may be NULL. */
int opf_case_dims(const opf_case *cs, const opf_opts *opts,
                  int64_t *n, int64_t *m, int64_t *nnzj, int64_t *nnzh);

/* The Jacobian and Hessian patterns into HOST buffers of nnzj / nnzh
 * int32 entries (any may be NULL). */
int opf_case_structure(const opf_case *cs, const opf_opts *opts,
                       int32_t *jrows, int32_t *jcols, int32_t *hrows, int32_t *hcols);

/* Variable bounds, constraint bounds and the starting point (vm = 1, all
 * else 0; Listing 3) into HOST buffers of n, n, m, m, n doubles (any may be
 * NULL).  Infinite bounds are +-INFINITY. */
int opf_case_bounds(const opf_case *cs, const opf_opts *opts,
                    double *lvar, double *uvar, double *lcon, double *ucon, double *x0);

/* ---------------------------------------------------------------- model */
typedef struct opf_model_s *opf_model;

/* Device memory hook for model and batch storage (default hipMalloc /
 * hipFree).  alloc returns NULL on failure, which makes create fail with
 * OPF_E_NOMEM.  Applies to handles created afterwards; pass NULLs to
 * restore the default. */
void opf_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                       void (*release)(void *ptr, void *ctx), void *ctx);

/* Launch shape of opf_eval_set for models created afterwards.  A model
 * whose callback set is at most `waves` 64-lane work items (summed over
 * replicas) evaluates a set in ONE launch, its bus items recomputing the
 * branch terms they need (a small set is latency-bound); larger models use
 * two launches (branch items leave per-half-edge records that bus items
 * read).  A model keeps its shape for life.  Both shapes give bitwise the
 * same results (no floating-point contraction in the kernels), and so do
 * batches (opf_batch_eval) in either of their shapes.  J^T v always uses
 * two launches.  0 disables the single launch; the default is 4096.
 * OPF_E_ARG for a negative limit. */
int opf_set_single_launch_limit(int64_t waves);

/* Validate, derive branch admittance terms, adjacency and pattern on the
 * host, and upload everything to `device` in one copy.  The only call that
 * moves data from host to device.  *out receives the handle. */
int opf_model_create(const opf_case *cs, const opf_opts *opts, int device, opf_model *out);

/* Free the model's device memory (synchronises the device first).  NULL is
 * accepted.  The handle is invalid afterwards. */
int opf_model_destroy(opf_model model);

int opf_model_dims(opf_model model, int64_t *n, int64_t *m, int64_t *nnzj, int64_t *nnzh);

/* Launch shape of opf_eval_set for this model (see
 * opf_set_single_launch_limit): *launches = 1 or 2, *items = the 64-lane
 * work items of one set summed over replicas.  Either pointer may be NULL. */
int opf_model_launches(opf_model model, int32_t *launches, int64_t *items);

/* Offset and length of a variable or constraint block, the named handles
 * the paper's model builder returns (vars, cons; Sec. III-C1). */
enum {
    OPF_VAR_VA = 0, OPF_VAR_VM, OPF_VAR_PG, OPF_VAR_QG, OPF_VAR_P, OPF_VAR_Q,
    OPF_CON_REF = 16, OPF_CON_P_FR, OPF_CON_Q_FR, OPF_CON_P_TO, OPF_CON_Q_TO,
    OPF_CON_ANGLE, OPF_CON_BAL_P, OPF_CON_BAL_Q, OPF_CON_THERMAL_FR,
    OPF_CON_THERMAL_TO, OPF_CON_RAMP,
    OPF_CON_ANGLE_LO, OPF_CON_VMAG,         /* rectangular form (empty in polar) */
    OPF_VAR_VR = OPF_VAR_VA, OPF_VAR_VI = OPF_VAR_VM,  /* rectangular bus blocks */
    OPF_VAR_PS = 6, OPF_VAR_QS, OPF_VAR_QSC, OPF_VAR_SE, OPF_VAR_SC, OPF_VAR_SD, OPF_VAR_U,
    OPF_CON_SOC = 29, OPF_CON_STOR_LOSS_P, OPF_CON_STOR_LOSS_Q, OPF_CON_STOR_THERMAL, OPF_CON_STOR_COMP,
    OPF_CON_DEV_RAMP, OPF_CON_DEV_INIT
};
int opf_model_blocks(opf_model model, int32_t which, int64_t *offset, int64_t *len);

/* Bounds and starting point into device buffers (n, n, m, m, n doubles;
 * any may be NULL). */
int opf_bounds(opf_model model, double *lvar, double *uvar, double *lcon, double *ucon,
               double *x0, void *stream);

/* ------------------------------------------------------------ callbacks */
/* obj: *f (one device double) = f(x).                         (Listing 1) */
int opf_obj(opf_model model, const double *x, double *f, void *stream);
/* grad!: g[n] = grad f(x), dense.                                         */
int opf_grad(opf_model model, const double *x, double *g, void *stream);
/* cons!: c[m] = c(x).                                                     */
int opf_cons(opf_model model, const double *x, double *c, void *stream);
/* jac!: pattern rows/cols (int32[nnzj]) and values vals[nnzj] at x.       */
int opf_jac_structure(opf_model model, int32_t *rows, int32_t *cols, void *stream);
int opf_jac_coord(opf_model model, const double *x, double *vals, void *stream);
/* hess!: lower-triangle pattern and values of
 *   obj_weight * hess f(x) + sum_i y_i hess c_i(x),  y[m].                */
int opf_hess_structure(opf_model model, int32_t *rows, int32_t *cols, void *stream);
int opf_hess_coord(opf_model model, const double *x, const double *y, double obj_weight,
                   double *vals, void *stream);

/* All five callbacks in one or two kernel launches (the model's launch
 * shape, opf_model_launches); bitwise equal to the separate calls.  Any
 * output may be NULL (skipped); y may be NULL only when hvals is. */
int opf_eval_set(opf_model model, const double *x, const double *y, double obj_weight,
                 double *f, double *g, double *c, double *jvals, double *hvals, void *stream);

/* out[n] = J(x)^T v for v[m]: the vector-Jacobian product of the
 * constraints, each entry gathered in a fixed order (no atomics). */
int opf_jtprod(opf_model model, const double *x, const double *v, double *out, void *stream);

/* opf_eval_set for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same kernels and bitwise the same results, with their scratch (objective
 * partials, the one-launch arrival ticket, the half-edge records) taken
 * from one fixed device array of OPF_NOALLOC_SCRATCH_BYTES per GPU, held
 * from the first call on that GPU until the process ends, instead of the
 * model's own.  The call allocates nothing and enqueues at most one more
 * launch (it zeroes the ticket).  Every call on one GPU shares that array:
 * calls that overlap in time on one GPU (two streams, two threads) race and
 * give wrong results; calls ordered on one stream are safe.  OPF_E_ARG if
 * the model needs more scratch than the array holds (48 bytes per branch,
 * side and replica plus the partials: about 340k branch replicas), or for
 * a NULL x, or a NULL y with hvals. */
#define OPF_NOALLOC_SCRATCH_BYTES (32u << 20)
int opf_eval_set_noalloc(opf_model model, const double *x, const double *y, double obj_weight, double *f,
                         double *g, double *c, double *jvals, double *hvals, void *stream);

/* ---------------------------------------------------------------- batch */
/* Many instances of possibly different networks evaluated together: two
 * kernel launches (branch phase, bus phase) on the caller's stream, each
 * covering every instance's work items (batched AC-OPF is the paper's stated future
 * work, Sec. V).  Instance j uses model inst_model[j] (static,
 * multi-period or contingency) with its own loads: inst_pd / inst_qd hold
 * the concatenated per-instance load arrays, n_bus entries per instance
 * (n_periods * n_bus, bus fastest, for a multi-period model); NULL = every
 * instance uses its model's own loads.  The models must stay alive while
 * the batch exists. */
typedef struct opf_batch_s *opf_batch;

int opf_batch_create(const opf_model *models, int32_t n_models, const int32_t *inst_model,
                     const double *inst_pd, const double *inst_qd, int32_t n_inst,
                     opf_batch *out);
int opf_batch_destroy(opf_batch batch);

/* Per-instance offsets (n_inst+1 int64 each, host buffers; any may be NULL)
 * into the concatenated X (variables), C (constraints; also Y),
 * J and H value arrays.  Instance j's objective goes to F[j]. */
int opf_batch_offsets(opf_batch batch, int64_t *xoff, int64_t *coff, int64_t *joff,
                      int64_t *hoff);

/* Time the candidate schedules on this batch, each the best of three
 * rounds interleaved over the candidates, and keep the fastest in the
 * handle: the launch shape (one launch whose bus lanes recompute the branch
 * terms, or two launches passing records) and, for two launches, the grid
 * (flat, or persistent with 2 to 32 workgroups per compute unit).  Results
 * of opf_batch_eval do not depend on the schedule (bitwise).  Allocates
 * tuning buffers through the allocator; synchronises `stream`. */
int opf_batch_tune(opf_batch batch, void *stream);

/* The schedule in use: -1 for the one-launch shape, 0 for two flat
 * launches (one workgroup per work item), else two persistent launches of
 * wg_per_cu workgroups per compute unit.  J^T v (opf_batch_jtprod) always
 * takes two launches, flat when the schedule is -1 or 0. */
int opf_batch_schedule(opf_batch batch, int32_t *wg_per_cu);

/* Force a schedule: wg_per_cu in [-1, 64] (else OPF_E_ARG). */
int opf_batch_set_schedule(opf_batch batch, int32_t wg_per_cu);

/* All callbacks of every instance in one or two kernel launches (the
 * schedule), launched on `stream` with this call's buffers as kernel
 * arguments (no allocation; the launches can be captured into a HIP
 * graph).  sigma[n_inst] are the objective weights.  Any of F, G, C, J, H
 * may be NULL (skipped); Y and sigma may be NULL when H is.  Results are
 * bitwise equal to opf_eval_set on each instance's model, in either launch
 * shape. */
int opf_batch_eval(opf_batch batch, const double *X, const double *Y, const double *sigma,
                   double *F, double *G, double *C, double *J, double *H, void *stream);

/* OUT = J(X)^T V for every instance (concatenated like X and C). */
int opf_batch_jtprod(opf_batch batch, const double *X, const double *V, double *OUT,
                     void *stream);

/* Replace every instance's loads (device buffers laid out like inst_pd /
 * inst_qd of opf_batch_create) by an asynchronous copy on `stream`.
 * OPF_E_STATE if the batch was created without per-instance loads. */
int opf_batch_set_loads(opf_batch batch, const double *pd, const double *qd, void *stream);

/* Overwrite the arc variables p, q of every instance in X by the branch
 * flows F(vm, va) at X's voltages (so every flow-definition row of c(X) is
 * zero).  One launch. */
int opf_batch_flows(opf_batch batch, double *X, void *stream);

/* ------------------------------------------------ learned warm-start proxy */
/* Kernels of a multilayer perceptron that maps loads to (vm, va, pg, qg),
 * trained on the FP64 penalty the callbacks compute (ML proxies for OPF are
 * the paper's related work, Sec. I; feasibility is the open issue).  All
 * pointers are device pointers; all matrices row-major; FP32 unless noted.
 * Matrix dimensions and leading dimensions must be multiples of 4 and the
 * buffers 16-byte aligned (OPF_E_ARG otherwise). */

/* C[M,N] = A[M,K] B[K,N] on the BF16 matrix cores: FP32 operands rounded to
 * BF16 (nearest even), FP32 accumulation.  variant selects the storage of A
 * and B:  0  A(i,k) = A[i*lda+k],  B(k,j) = B[j*ldb+k]   (x W^T)
 *         1  A(i,k) = A[i*lda+k],  B(k,j) = B[k*ldb+j]   (dy W)
 *         2  A(i,k) = A[k*lda+i],  B(k,j) = B[k*ldb+j]   (dy^T x)
 *         3  A(i,k) = A[k*lda+i],  B(k,j) = B[j*ldb+k]
 * bias (may be NULL) is added per column; if act is non-NULL it receives
 * GELU(C) (exact erf form).  accumulate != 0 adds to the existing C. */
int prox_gemm_bf16(int variant, const float *A, int lda, const float *B, int ldb, float *C, int ldc, int M, int N,
                   int K, const float *bias, float *act, int accumulate, void *stream);

/* prox_gemm_bf16 with the K range cut into `splits` (1..64) parts of whole
 * 64-wide k tiles, computed by separate workgroups into work (splits * M * N
 * floats, 16-byte aligned, caller-owned, contents overwritten), then summed
 * part 0 first, with the bias / GELU / accumulate epilogue of prox_gemm_bf16.
 * For products whose M x N tiles alone cannot fill the device (weight
 * gradients, K = batch size).  splits = 1 is prox_gemm_bf16 (work unused). */
int prox_gemm_bf16_splitk(int variant, const float *A, int lda, const float *B, int ldb, float *C, int ldc, int M,
                          int N, int K, const float *bias, float *act, int accumulate, int splits, float *work,
                          void *stream);

/* prox_gemm_bf16_splitk with either operand stored as BF16 (a_bf16 /
 * b_bf16 != 0: A / B point to BF16 values, same layouts; no rounding is
 * then needed when staged, so the product equals the FP32-operand product of
 * the same values) and the GELU output act stored as BF16 (act_bf16 != 0,
 * rounded to nearest even; C stays FP32).  For the MLP's hidden activations
 * and the BF16 copy of its weights: half the operand bytes.  A k-contiguous
 * BF16 operand needs K and its leading dimension multiples of 8 (OPF_E_ARG
 * otherwise).  C may be NULL when act is given, accumulate is 0 and splits
 * is 1: act is then the only output (an MLP forward that no backward will
 * follow needs no pre-activations); OPF_E_ARG for a NULL C otherwise.  The
 * same rule holds for prox_gemm_bf16 and prox_gemm_bf16_splitk. */
int prox_gemm_bf16_mixed(int variant, const void *A, int a_bf16, int lda, const void *B, int b_bf16, int ldb, float *C,
                         int ldc, int M, int N, int K, const float *bias, void *act, int act_bf16, int accumulate,
                         int splits, float *work, void *stream);

/* y[i] = x[i] rounded to BF16 (nearest even), n values. */
int prox_to_bf16(const float *x, int64_t n, void *y, void *stream);

/* The proxy MLP's backward through a hidden layer in one product: out [M, N]
 * (BF16, leading dimension ldo) = (A B) * gelu'(pre) elementwise, for
 * row-major A [M, K] and B [K, N] (each FP32 or BF16 as a_bf16, b_bf16, as
 * prox_gemm_bf16_mixed's variant 1) and pre [M, N] (FP32, the layer's
 * pre-activation; gelu' of the exact GELU); part [ceil(M / 128), N] (FP32)
 * receives the column sums of each 128-row block of the FP32 product before
 * its rounding to BF16, in prox_colsum's first-pass order, so that
 * prox_colsum_parts gives the bias gradient.  The values equal the product,
 * prox_gelu_bwd and prox_colsum's first pass in sequence bit for bit.
 * Dimensions and leading dimensions are multiples of 4 (a BF16 A: K and lda
 * multiples of 8); A, B, pre 16-byte aligned, out 8-byte aligned.  Buffers
 * are device memory the caller owns; OPF_E_ARG for a violated rule. */
int prox_gemm_gelu_bwd(const void *A, int a_bf16, int lda, const void *B, int b_bf16, int ldb, const float *pre,
                       int ldp, void *out, int ldo, int M, int N, int K, float *part, void *stream);

/* out [N] = scale * column sums of part [chunks, N]: prox_colsum's second
 * pass over partial sums that prox_gemm_gelu_bwd left. */
int prox_colsum_parts(const float *part, int chunks, int N, float *out, float scale, void *stream);

/* A split count for prox_gemm_bf16_splitk: the smallest power of two (at
 * most 16) that gives 256 or more 128 x 128 workgroups while each part keeps
 * at least four k tiles.  Negative sizes: OPF_E_ARG. */
int prox_gemm_splits(int M, int N, int K);

/* dpre = dact * GELU'(pre), n elements. */
int prox_gelu_bwd(const float *pre, const float *dact, float *dpre, int64_t n, void *stream);

/* out[j] = scale * sum_i X[i, j] for X [M, N], summed in a fixed order;
 * work holds ((M + 127) / 128) * N floats. */
int prox_colsum(const float *X, int M, int N, float *work, float *out, float scale, void *stream);

/* One Adam step (Kingma and Ba 2015, bias-corrected) on n parameters;
 * step counts from 1. */
int prox_adam(float *p, const float *g, float *m1, float *m2, int64_t n, float lr, float beta1, float beta2,
              float eps, int step, void *stream);

/* prox_adam with the step count in device memory, for a training step
 * captured in a HIP graph: the update uses step = *step + 1 and a second
 * one-thread launch then stores it into *step (int32, device).  pb (may be
 * NULL) receives the updated parameters rounded to BF16 (nearest even, n
 * values, device): the copy the matrix-core products read. */
int prox_adam_dev(float *p, const float *g, float *m1, float *m2, int64_t n, float lr, float beta1, float beta2,
                  float eps, int32_t *step, void *pb, void *stream);

/* z [B, 2N+2G] (blocks vm, va, pg, qg) -> the va, vm, pg, qg entries of X
 * [B, n] (FP64): vm, pg, qg = lower + (upper - lower) sigmoid(z); va =
 * va_span tanh(z), 0 at reference buses; p, q set to 0.  Static models only
 * (OPF_E_ARG otherwise). */
int prox_squash_fwd(opf_model model, const float *z, int B, double va_span, double *X, void *stream);

/* prox_squash_fwd that leaves the arc variables p, q of X as they are (for
 * a caller that writes them next, as opf_batch_flows does): 2N + 2G entries
 * per instance written instead of n. */
int prox_squash_fwd_vars(opf_model model, const float *z, int B, double va_span, double *X, void *stream);

/* dz [B, 2N+2G] = scale * (d x / d z)^T g for the va, vm, pg, qg entries of
 * g = gX1 + gX2 + obj_scale * gObj ([B, n] FP64 each; gX2 and gObj may be
 * NULL). */
int prox_squash_bwd(opf_model model, const float *z, int B, double va_span, const double *gX1, const double *gX2,
                    const double *gObj, double obj_scale, float *dz, float scale, void *stream);

/* Per instance b of C [B, m], X [B, n]: pen[b] = rho * (sum of squared
 * constraint violations over the non-flow rows + squared bound violations of
 * p, q) + obj_scale * F[b] (the objective term is skipped when F is NULL);
 * cvio[b] = largest violation over every row and the p, q bounds (the
 * paper's Cvio, Sec. IV-A5); W [B, m] = d pen / d c on the non-flow rows;
 * gpq [B, 4L] = d pen / d (p, q).  The flow rows of W receive 0, or with
 * vjp != 0 the weights of prox_vjp_weights (computed in the same pass), so
 * that J^T W is the whole constraint part of the gradient.  With vjp != 0
 * and 4L <= 7680, gpq may be NULL: d pen / d (p, q), needed only by those
 * weights, then stays on chip (OPF_E_ARG for a NULL gpq otherwise). */
int prox_penalty(opf_model model, const double *C, const double *X, const double *F, double obj_scale, double rho,
                 int B, int vjp, double *pen, double *cvio, double *W, double *gpq, void *stream);

/* Wt [B, m] = W + W2 for the penalty's VJP through p, q = F(vm, va): W2 is
 * minus (G1 + gpq) of each arc variable placed on its flow row, G1 = J^T W
 * restricted to the arc variables, which has a closed form (2 p W on the
 * branch side's thermal row + W on the balance row of the arc's bus; W is 0
 * on the flow rows).  J^T Wt is then the whole constraint part of the
 * gradient (one product).  X [B, n] holds the arc flows; W, gpq as written
 * by prox_penalty.  Wt may be W: then only its flow rows are written. */
int prox_vjp_weights(opf_model model, const double *X, const double *W, const double *gpq, int B, double *Wt,
                     void *stream);

/* gX [B, n] = wb[b] * (gX1 + gX2 + obj_scale * grad f(X)) on the va, vm,
 * pg, qg entries, zero on the arc variables p, q (which the proxy sets to
 * the branch flows, so they are not free); grad f = 2 c2 pg + c1 on the pg
 * entries.  wb [B] is a device vector (the incoming gradient of each
 * instance's loss).  gX2 may be NULL; X may be NULL when obj_scale is 0. */
int prox_vjp_sum(opf_model model, const double *X, const double *gX1, const double *gX2, double obj_scale,
                 const double *wb, int B, double *gX, void *stream);

/* prox_vjp_sum followed by prox_squash_bwd in one pass: dz [B, 2N+2G] =
 * (d x / d z)^T g with g = wb[b] * (gX1 + obj_scale * grad f(X)) on the va,
 * vm, pg, qg entries (X may be NULL when obj_scale is 0).  The same values
 * as the two calls (no [B, n] intermediate). */
int prox_loss_bwd(opf_model model, const float *z, int B, double va_span, const double *X, const double *gX1,
                  double obj_scale, const double *wb, float *dz, void *stream);

/* The proxy's whole FP64 loss side in one launch, one workgroup per sample
 * with the sample's working set in LDS: squashing of z [B, 2N+2G] (FP32,
 * vm, va, pg, qg blocks) into the variable boxes, arc flows p, q := F(vm, va)
 * (Sec. III-C, the branch flow terms), the non-flow rows at loads [B, 2N]
 * (each sample's pd then qd, FP64), and
 *   loss[b] = rho * (squared violations of the non-flow rows and of the p, q
 *             bounds) + obj_scale * f(x_b),
 *   cvio[b] = largest violation over every row and the p, q bounds (Cvio,
 *             Sec. IV-A5),
 * the values of prox_squash_fwd_vars, opf_batch_flows, opf_batch_eval and
 * prox_penalty in sequence.  gz [B, 2N+2G] (FP64, z's layout) receives
 * d loss[b] / d z_b, the chain of prox_penalty (vjp), opf_batch_jtprod and
 * prox_loss_bwd at wb = 1 (NULL: not computed).  X [B, n] and C [B, m]
 * receive x (with the arc flows) and c(x) when non-NULL.  The arc values,
 * the thermal and angle rows and X equal those launches' bits; the balance
 * rows, loss and gz are summed in another fixed order (rounding-level
 * differences; the same bits on every run).  Takes a static polar model
 * without storage units or devices (prox_loss_fused_fits); OPF_E_ARG
 * otherwise.  Buffers are device memory the caller owns. */
int prox_loss_fused(opf_model model, const float *z, int B, double va_span, const double *loads, double rho,
                    double obj_scale, double *loss, double *cvio, double *gz, double *X, double *C, void *stream);

/* 1 when prox_loss_fused takes this model: static, polar, no storage units
 * or devices, and one sample's working set (4N + 2G + 4L doubles) within
 * 64 KiB of LDS; 0 when not; OPF_E_STATE for an invalid handle. */
int prox_loss_fused_fits(opf_model model);

/* dz [B, D] = (float)(wb[b] * gz[b, j]): the backward of prox_loss_fused's
 * loss under an incoming gradient wb [B] (device FP64). */
int prox_scale_rows(const double *gz, const double *wb, int B, int D, float *dz, void *stream);

/* The proxy's synthetic training samples (a uniform spread of every bus's
 * load around the base case): from uniform draws r [B, N] in [0, 1), bus i
 * of sample b has both pd and qd scaled by 1 + spread (2 r[b, i] - 1);
 * loads [B, 2N] (FP64, pd then qd) = base [2N] times that factor, feats
 * [B, 2N] (FP32) = (loads - base) * inv_scale [2N].  Each operation rounds
 * as written (no contraction).  Device buffers the caller owns. */
int prox_sample_loads(const double *r, const double *base, const double *inv_scale, double spread, int B, int N,
                      double *loads, float *feats, void *stream);

/* The proxy MLP's parameters and optimizer state, all device memory the
 * caller owns: n_layers layers of widths dims[0..n_layers] (host array,
 * multiples of 4), GELU after every layer but the last.  flat holds per
 * layer the weight [out, in] row-major then the bias (FP32); flat_bf16 is
 * its BF16 copy that the products read where the input width is a multiple
 * of 8 (NULL: FP32 operands and activations throughout); m1, m2 are Adam's
 * moments; step is Adam's step count (int32, on the device). */
typedef struct prox_mlp_desc {
    int32_t n_layers;
    const int32_t *dims;
    float *flat;
    void *flat_bf16;
    float *m1;
    float *m2;
    int32_t *step;
} prox_mlp_desc;

/* Bytes of the workspace prox_train_step needs for a batch of B samples. */
int prox_train_step_bytes(const prox_mlp_desc *mlp, int B, int64_t *bytes);

/* One training step of the warm-start proxy (the learned start of the
 * related-work proxies, Sec. I; Cvio of Sec. IV-A5), every launch issued
 * here: the MLP forward on feats [B, dims[0]] (FP32) with the hidden
 * activations stored BF16 where flat_bf16 is given and the width a multiple
 * of 8; prox_loss_fused on its output at loads [B, 2N]; the gradient of the
 * mean loss (weight 1/B); the MLP backward (split-K weight gradients, bias
 * column sums, the GELU backward in the dh product as prox_gemm_gelu_bwd);
 * and prox_adam_dev (lr, beta1, beta2, eps).  The same kernels in the same
 * order as those calls made one by one, so the parameters after a step are
 * theirs bit for bit.  loss, cvio [B] receive the per-sample loss and Cvio
 * before the update.  work: work_bytes of device memory (16-byte aligned,
 * at least prox_train_step_bytes) that the step uses as scratch; the model
 * is one prox_loss_fused takes and the MLP's output width is 2N + 2G;
 * OPF_E_ARG otherwise.  Calls on one stream run in order; concurrent calls
 * sharing a workspace race.  phase_ms: NULL, or a host array of 4 floats
 * that receives the GPU time of the forward, the loss (with its gradient
 * scaling), the backward and the Adam step, from events on the stream; the
 * call then waits for the step to finish. */
int prox_train_step(opf_model model, const prox_mlp_desc *mlp, const float *feats, const double *loads, int B,
                    double va_span, double rho, double obj_scale, float lr, float beta1, float beta2, float eps,
                    void *work, int64_t work_bytes, double *loss, double *cvio, float *phase_ms, void *stream);
#ifdef __cplusplus
}
#endif
#endif /* OPF_H */
