/*
 * tr.h — C ABI of the MI355X (gfx950) library for block-randomized
 * stochastic tensor-ring decomposition: TR-BRSGD and TR-ScaledBRSGD
 * (Yu, Li, Zhou, "Block-Randomized Stochastic Methods for Tensor Ring
 * Decomposition").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Indexing is 0-based (the paper is 1-based).
 *
 * Cores.  Core k (0 <= k < N) has shape R_k x I_k x R_{k+1}, R_N = R_0
 * (tensor-ring format, Section 1).  It is stored as its classical mode-2
 * unfolding G_{k(2)} (Definition "Classical Mode-n Unfolding"), an
 * I_k x (R_k R_{k+1}) row-major matrix with column c = r + R_k*s holding
 * G_k(r, i, s).  Lateral slice G_k(i) is then a contiguous column-major
 * R_k x R_{k+1} block.
 *
 * Tensor X.  Dense, addressed by explicit element strides x_stride[k]:
 * X(i_0..i_{N-1}) sits at sum_k i_k * x_stride[k].  Paper order
 * (Definition "Multi-index", first index fastest) has strides 1, I_0,
 * I_0*I_1, ...  A mode-major replica of mode n (tr_x_replicate) stores the
 * cyclic unfolding X_[n] column-major, i.e. strides with x_stride[n] = 1.
 *
 * Sampled rows.  For mode n, sample f draws one slice index i_k per core
 * k != n (Algorithm SSDTP).  idx is int32 [m][N] with idx[f][n] = -1.
 * S is [m][R_n R_{n+1}] row-major with S[f][r + R_n*s] = M_f(s, r),
 * M_f = G_{n+1}(i_{n+1}) ... G_{N-1}(i_{N-1}) G_0(i_0) ... G_{n-1}(i_{n-1})
 * (Definition "Subchain Tensor": S holds rows of G^{!=n}_[2]).
 *
 * Random draws.  Philox4x64-10 (Salmon et al., SC'11) with key (seed, 0)
 * and counter (step, sample, mode, stream); bounded integers by
 * floor(r * n / 2^64) (Lemire 2019).  The mode of step t is
 * floor(r * N / 2^64) with r from counter (t, 0, 0, TR_STREAM_MODE).
 * Non-uniform laws are sampled from inclusive prefix sums ("CDF") of
 * integer weights w_i = floor(p_i * 2^40) + 1: u = floor(r * W / 2^64),
 * pick the first i with C_i > u; that index has probability w_i / W.
 *
 * Ownership.  The caller allocates every buffer (device memory unless
 * marked host) and passes raw pointers and a HIP stream.  The library
 * never allocates or frees on the hot path: scratch space is a caller
 * workspace ``ws`` of at least the size returned by the matching
 * *_workspace_size query, aligned to 256 bytes.  Only a batch plan owns
 * memory; it is created and destroyed outside timed regions.
 *
 * Errors.  Host validation failures return a negative tr_status and
 * enqueue nothing.  Numerical conditions found on the device set sticky
 * bits (TR_DEV_*) in the caller's device word ``dev_status`` (OR-ed in,
 * never cleared by the library).  Calls are asynchronous on ``stream``;
 * results written to device scalars (loss, rse) are valid once the
 * stream reaches them.  The library keeps no mutable global state apart
 * from the per-GPU address of tr_run_noalloc's scratch, set once.
 */
#ifndef TR_H_
#define TR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* tr_stream_t;   /* a hipStream_t */

#define TR_ABI_VERSION 2
#define TR_MAX_ORDER 8
#define TR_MAX_RANK 16

typedef enum {
    TR_OK = 0,
    TR_E_ARG = -1,          /* null pointer or invalid scalar argument   */
    TR_E_SHAPE = -2,        /* N, I, R or m outside the supported range  */
    TR_E_DTYPE = -3,        /* unknown or unsupported dtype combination  */
    TR_E_ALIGN = -4,        /* pointer not aligned to its element size   */
    TR_E_WORKSPACE = -5,    /* workspace smaller than required           */
    TR_E_HIP = -6,          /* a HIP launch or runtime call failed       */
    TR_E_UNSUPPORTED = -7   /* valid request this library does not serve */
} tr_status;

/* Sticky device status bits. */
enum {
    TR_DEV_NONFINITE = 1,   /* NaN/Inf met in an update                  */
    TR_DEV_NOT_SPD = 2,     /* Gram not positive definite even damped    */
    TR_DEV_ZERO_DIST = 4,   /* law with zero total mass; uniform used    */
    TR_DEV_DAMPED = 8       /* Cholesky needed the damping fallback      */
};

typedef enum { TR_F64 = 0, TR_F32 = 1, TR_F16 = 2, TR_BF16 = 3 } tr_dtype;

/* Arithmetic of the contractions in tr_grad.
 *   TR_PREC_F64:  everything FP64 (FP64 cores and X).
 *   TR_PREC_F32:  FP32 products (matrix cores), FP32 accumulation.
 *   TR_PREC_BF16: mixed: the prediction G_{n(2)} S^T from hi/lo BF16
 *                 splits of both operands (three BF16 products), the
 *                 residual in BF16 times S split hi/lo, FP32 accumulation.
 *   TR_PREC_F16:  FP16 products, FP32 accumulation.
 * The Gram S^T D S is always accumulated in FP64. */
typedef enum { TR_PREC_F64 = 0, TR_PREC_F32 = 1, TR_PREC_BF16 = 2, TR_PREC_F16 = 3 } tr_prec;

/* Sampling laws of Section 3.2. */
typedef enum { TR_LAW_UNIFORM = 0, TR_LAW_LEVERAGE = 1, TR_LAW_EUCLID = 2, TR_LAW_OPTIMAL = 3 } tr_law;

/* Counter stream tags (fourth Philox counter word). */
enum { TR_STREAM_MODE = 0, TR_STREAM_IDX = 1, TR_STREAM_H = 2, TR_STREAM_ENTRY = 3 };

typedef struct {
    int32_t N;                          /* order, 2 <= N <= TR_MAX_ORDER       */
    int32_t I[TR_MAX_ORDER];            /* mode sizes I_k >= 1                  */
    int32_t R[TR_MAX_ORDER];            /* ring ranks: core k is R[k] x I[k] x R[(k+1)%N], 1 <= R <= TR_MAX_RANK */
    int64_t x_stride[TR_MAX_ORDER];     /* element strides of X                 */
    int32_t core_dtype;                 /* tr_dtype of the cores (F64 or F32)   */
    int32_t x_dtype;                    /* tr_dtype of X                        */
} tr_desc;

/* Step rule (equation eq:update_brsgd and the AdaGrad remark).
 *   kind 0: fixed alpha:       G += alpha * p
 *   kind 1: AdaGrad:           A += p*p;  G += eta * p / (b + A)^(1/2 + eps),
 *                              no change where b + A == 0
 *   kind 2: Robbins-Monro:     G += alpha / (1 + t/tau) * p                  */
typedef struct {
    int32_t kind;
    double alpha, tau, eta, b, eps;
} tr_step;

/* ------------------------------------------------------------------ */
/* Library metadata                                                    */
/* ------------------------------------------------------------------ */
int32_t tr_abi_version(void);
const char* tr_status_str(int32_t status);

/* Mode of step t (Algorithm TR-BRSGD: n uniform over the N modes).  Pure
 * host function; the same value the device computes inside tr_run. */
int32_t tr_mode(uint64_t seed, uint64_t step, int32_t N);

/* ------------------------------------------------------------------ */
/* a2: sampling laws                                                   */
/* ------------------------------------------------------------------ */

/* Integer-weight CDF of the leverage or Euclidean law of core k (Lemma
 * "lev_est": p(i) = l_i(G_{k(2)}) / rank; Lemma "euc_est":
 * p(i) = ||G_k(:,i,:)||_F^2 / ||G_k||_F^2).  core_k: G_{k(2)} in the core
 * dtype.  cdf_k: uint64 [I_k], inclusive prefix sums of the weights.
 * Leverage scores are l_i = g_i^T (G^T G)^{-1} g_i with the FP64 Gram
 * G^T G of G = G_{k(2)}, inverted by the blocked FP64 sweep for
 * R_k R_{k+1} <= 128 and through an FP64 Cholesky above.  The rank is
 * found on the Gram: when a pivot of that factorisation is at or below
 * 2^-43 of the largest diagonal entry, or when I_k <= R_k R_{k+1}, the
 * scores come from a Cholesky with diagonal pivoting of G^T G stopped at
 * pivots <= R_k R_{k+1} 2^-52 max diag: the rank r is the number of pivots
 * taken, l_i = g_i[P]^T (G_P^T G_P)^{-1} g_i[P] over the chosen columns P
 * (the diagonal of the projector onto the column space of G), and
 * p(i) = l_i / r (r = I_k, full row rank: the uniform law).  This agrees with an SVD rank at the usual tolerance unless a
 * singular value of G_{k(2)} lies between about 1e-13 and 1e-7 of the
 * largest.  A zero core (Euclidean total 0, or leverage rank 0) sets
 * TR_DEV_ZERO_DIST and writes the uniform CDF.  law must be
 * TR_LAW_LEVERAGE or TR_LAW_EUCLID.  ws: device workspace of at least
 * tr_dist_workspace_size bytes (row norms, or the Gram, its inverse and the
 * scores); the call fails with TR_E_WORKSPACE without it. */
tr_status tr_dist(const tr_desc* d, int32_t k, int32_t law, const void* core_k,
                  uint64_t* cdf_k, int32_t* dev_status,
                  void* ws, size_t ws_bytes, tr_stream_t stream);
size_t tr_dist_workspace_size(const tr_desc* d, int32_t k, int32_t law);

/* Integer-weight CDF over the J_n columns of X_[n] for the optimal law
 * (equation eq:optimal_prob, unsquared norms): q(j) proportional to
 * ||X_[n](:,j) - G_{n(2)} s_j||_2 * ||s_j||_2 with s_j the row j of
 * G^{!=n}_[2].  cores: host array of N device pointers.  X: device tensor
 * with the strides of d.  cdf_J: uint64 [J_n].  If every term is zero the
 * uniform CDF is written and TR_DEV_ZERO_DIST is set. */
tr_status tr_dist_optimal(const tr_desc* d, int32_t n, const void* const* cores,
                          const void* X, uint64_t* cdf_J, int32_t* dev_status,
                          void* ws, size_t ws_bytes, tr_stream_t stream);
size_t tr_dist_optimal_workspace_size(const tr_desc* d, int32_t n);

/* ------------------------------------------------------------------ */
/* a1/a3/a4: draws and sampled subchain rows (Algorithm SSDTP)         */
/* ------------------------------------------------------------------ */

/* Draw m samples for mode n at step ``step``: idx int32 [m][N]
 * (idx[f][n] = -1) and pF float64 [m] = prod_k p_k(i_k) multiplied in the
 * order n+1, ..., N-1, 0, ..., n-1.  cdf: host array of N device pointers
 * (entry k = CDF of mode k, or NULL for uniform, where p_k = 1/I_k); cdf
 * itself may be NULL (all uniform).  cdf_J: CDF over J_n for the optimal
 * law (then cdf is ignored and one index j is drawn per sample with
 * counter slot k = n, decoded by the cyclic order), else NULL.
 * stream_tag selects the counter stream (TR_STREAM_IDX for F_n,
 * TR_STREAM_H for an independent H_n). */
tr_status tr_sample(const tr_desc* d, uint64_t seed, uint64_t step, int32_t n, int32_t m,
                    const uint64_t* const* cdf, const uint64_t* cdf_J, int32_t stream_tag,
                    int32_t* idx, double* pF, tr_stream_t stream);

/* Sampled rows of G^{!=n}_[2] for the draws in idx: S [m][R_n R_{n+1}] in
 * the core dtype (slices-Hadamard products from identity slices). */
tr_status tr_subchain(const tr_desc* d, int32_t n, const void* const* cores,
                      const int32_t* idx, int32_t m, void* S, tr_stream_t stream);

/* ------------------------------------------------------------------ */
/* a5/a6: fiber gather and stochastic gradient (eq:S_gradient)         */
/* ------------------------------------------------------------------ */

/* g = (G_{n(2)} S^T D S - X_F D S) / (m J_n), D = diag(1/pF), computed as
 * E = X_F - G_{n(2)} S^T (fibers gathered from X by idx), g = -E D S/(m J_n).
 * g: [I_n][R_n R_{n+1}] in the core dtype.  loss (device float64 scalar,
 * may be NULL) = sum_f ||e_f||^2 / (2 m pF_f), an unbiased estimate of f.
 * gram (device float64 [RR][RR], may be NULL) = S^T D S / (m J_n), the
 * stochastic Hessian of eq:S_hessian with H_n = F_n.  Reductions over
 * samples run in a fixed order: results are bitwise reproducible. */
tr_status tr_grad(const tr_desc* d, int32_t n, const void* core_n, const void* X,
                  const int32_t* idx, const void* S, const double* pF, int32_t m,
                  int32_t prec, void* g, double* loss, double* gram,
                  void* ws, size_t ws_bytes, tr_stream_t stream);
size_t tr_grad_workspace_size(const tr_desc* d, int32_t m, int32_t prec);

/* Stochastic Hessian from an independent draw H_n (eq:S_hessian):
 * gram = S_H^T diag(1/pH) S_H / (m_H J_n), FP64 accumulation. */
tr_status tr_gram(const tr_desc* d, int32_t n, const void* S_H, const double* pH, int32_t m_H,
                  double* gram, void* ws, size_t ws_bytes, tr_stream_t stream);
size_t tr_gram_workspace_size(const tr_desc* d, int32_t m_H);

/* ------------------------------------------------------------------ */
/* a7/a8: direction and update                                         */
/* ------------------------------------------------------------------ */

/* Direction p = -g (gram == NULL) or p = -g (h + damping I)^{-1} with
 * h = gram (eq:scaledsg_direction and the amended preconditioner): for
 * RR <= 128 the FP64 blocked symmetric sweep forms -(h + damping I)^{-1}
 * and a row-parallel product applies it; for RR > 128 an FP64 Cholesky
 * and two triangular solves.  If h + damping I is not
 * positive definite the solve retries with damping + 10^(k-10) tr(h)/RR,
 * k = 0..6 (TR_DEV_DAMPED), else leaves the core unchanged
 * (TR_DEV_NOT_SPD).  Then core_n is updated in place by ``rule`` at step t;
 * accum_n ([I_n][RR], core dtype) is the AdaGrad accumulator (required for
 * kind 1, else may be NULL). */
tr_status tr_update(const tr_desc* d, int32_t n, void* core_n, const void* g,
                    const double* gram, double damping, const tr_step* rule, uint64_t t,
                    void* accum_n, int32_t* dev_status,
                    void* ws, size_t ws_bytes, tr_stream_t stream);
size_t tr_update_workspace_size(const tr_desc* d, int32_t n, int32_t scaled);

/* ------------------------------------------------------------------ */
/* a9: reconstruction and relative error (RSE of Section 4)            */
/* ------------------------------------------------------------------ */

/* rse = ||TR(cores) - X_true||_F / ||X_true||_F, FP64 reduction.
 * FP32 cores with R_1 R_2 <= 128 form TR(cores) on FP16 matrix cores from
 * a hi/lo split of both operands (three products per K step, FP32
 * accumulation, each operand tile scaled by a power of two), about 22
 * significant bits per operand; FP64 cores and larger ranks take FP64 or
 * FP32 dot products.
 * x_true_norm2 = ||X_true||_F^2 if known, else a negative value (then it
 * is computed in the same pass).  rse: device float64 scalar.  Also
 * writes ||TR(cores) - X_true||^2 and ||X_true||^2 into ws[0..1] (float64). */
tr_status tr_relerr(const tr_desc* d, const void* const* cores, const void* X_true,
                    double x_true_norm2, double* rse, void* ws, size_t ws_bytes,
                    tr_stream_t stream);
size_t tr_relerr_workspace_size(const tr_desc* d);

/* X = TR(cores) written with the strides of d in the x dtype. */
tr_status tr_reconstruct(const tr_desc* d, const void* const* cores, void* X, tr_stream_t stream);

/* Mode-major replica: Xn holds X_[n] column-major (fiber of mode n
 * contiguous, columns in the cyclic order n+1, ..., n-1), read from X with
 * the strides of d. */
tr_status tr_x_replicate(const tr_desc* d, const void* X, int32_t n, void* Xn, tr_stream_t stream);

/* ------------------------------------------------------------------ */
/* Whole iterations: Algorithm TR-BRSGD / TR-ScaledBRSGD on the device */
/* ------------------------------------------------------------------ */

typedef struct {
    tr_desc desc;                        /* X strides: paper order of X      */
    void* cores[TR_MAX_ORDER];           /* device G_{k(2)}, updated in place */
    void* accum[TR_MAX_ORDER];           /* AdaGrad accumulators or NULL     */
    const void* X;                       /* device tensor (fit target)       */
    const void* Xrep[TR_MAX_ORDER];      /* mode-major replicas or NULL (with
                                          * all N given, the fiber gathers and
                                          * the optimal law read them)        */
    uint64_t* cdf[TR_MAX_ORDER];         /* per-mode CDF buffers [I_k] (laws L, E) */
    uint64_t* cdf_J;                     /* CDF buffer [max_n J_n] (law O)   */
} tr_problem;

typedef struct {
    int32_t m;          /* |F_n|                                             */
    int32_t m_H;        /* |H_n| for an independent Hessian draw, 0: H_n = F_n */
    int32_t law;        /* tr_law                                            */
    int32_t scaled;     /* 0: TR-BRSGD, 1: TR-ScaledBRSGD                    */
    int32_t prec;       /* tr_prec                                           */
    double damping;     /* eta^0 of the amended preconditioner h + eta^t I   */
    tr_step rule;
    uint64_t seed;
    /* eta^t at step t (the remark after eq:scaledsg_direction asks only for
     * eta^t >= 0): 0 constant eta^0; 1 harmonic eta^0 / (1 + t/damping_tau),
     * damping_tau > 0; 2 geometric eta^0 damping_tau^t, 0 < damping_tau <= 1. */
    int32_t damping_schedule;
    double damping_tau;
} tr_config;

/* Enqueue ``steps`` iterations.  The step counter lives in device memory:
 * t_dev (uint64) is read by every kernel and incremented at the end of
 * each step, and the mode is computed on the device from (seed, t), so the
 * enqueued sequence can be captured once in a HIP graph and replayed.
 * loss_out (device float64 [steps] or NULL) receives each step's loss
 * estimate.  Grids are sized for the largest mode. */
tr_status tr_run(const tr_problem* p, const tr_config* c, uint64_t* t_dev, int32_t steps,
                 double* loss_out, int32_t* dev_status, void* ws, size_t ws_bytes,
                 tr_stream_t stream);
size_t tr_run_workspace_size(const tr_problem* p, const tr_config* c);

/* tr_run with HIP events (hipEvent_t handles created by the caller) as the
 * start and stop events of the dispatch of the dominant kernel of step i
 * (the fused fiber-gather / gradient contraction): ev_begin[i], ev_end[i]
 * for i < steps; NULL arrays or entries are skipped.  The dispatch records
 * them itself, so their elapsed time is that kernel's execution inside a
 * real run, without the queueing around it. */
tr_status tr_run_events(const tr_problem* p, const tr_config* c, uint64_t* t_dev, int32_t steps,
                        double* loss_out, int32_t* dev_status, void* ws, size_t ws_bytes,
                        void* const* ev_begin, void* const* ev_end, tr_stream_t stream);

/* Options of tr_run_ex (all fields may be NULL).
 *   aux, ev_fork, ev_gram, ev_join: a second stream and three hipEvent_t
 *     handles, created by the caller (default stream priority).  With them
 *     a scaled step (RR <= 128) runs the Gram, its reduction and the
 *     inverse (equation eq:scaledsg_direction) on ``aux`` and the gradient
 *     on ``stream``: ev_fork is recorded on ``stream`` after the draws and
 *     waited on by ``aux``; ev_gram is recorded on ``aux`` once the Gram's
 *     per-group sums are written and waited on by ``stream`` before the
 *     gradient (so the gradient runs beside the reduction and the one-
 *     workgroup inverse instead of competing with the Gram); ev_join is
 *     recorded on ``aux`` after the inverse and waited on by ``stream``
 *     before the update.  Work of one step never overlaps the next; the
 *     fork/join is graph-capturable; results are bitwise those of the
 *     one-stream run.  All four must be set together, or all NULL.
 *   ev_begin, ev_end: as in tr_run_events.
 *   ev_inv_begin, ev_inv_end: the same for the dispatch of the RR x RR
 *     inverse of step i (scaled steps with RR <= 128). */
typedef struct {
    tr_stream_t aux;
    void* ev_fork;
    void* ev_gram;
    void* ev_join;
    void* const* ev_begin;
    void* const* ev_end;
    void* const* ev_inv_begin;
    void* const* ev_inv_end;
} tr_run_opts;

/* tr_run with options; opts NULL is tr_run.  Same workspace. */
tr_status tr_run_ex(const tr_problem* p, const tr_config* c, uint64_t* t_dev, int32_t steps,
                    double* loss_out, int32_t* dev_status, void* ws, size_t ws_bytes,
                    tr_stream_t stream, const tr_run_opts* opts);

/* ------------------------------------------------------------------ */
/* The paper's comparison methods, one sweep over the cores at a time   */
/* ------------------------------------------------------------------ */

/*   TR_METHOD_GD:          TR-GD, the update rule after eq:gradient:
 *                          G_n -= alpha grad_n f for every n, all from the
 *                          iterate the sweep starts at.
 *   TR_METHOD_SCALED_GD:   TR-ScaledGD (eq:scaled_gd): G_n -= alpha grad_n f
 *                          ((G^{!=n}_[2])^T G^{!=n}_[2] + J_n damping I)^{-1},
 *                          all n from the sweep's starting iterate.
 *   TR_METHOD_ALS:         TR-ALS (Algorithm alg:tr_als): n = 1..N in turn,
 *                          G_n <- the least-squares solution with the other
 *                          cores at their latest values (= TR-ScaledGD's
 *                          block step at alpha = 1).
 *   TR_METHOD_ALS_SAMPLED: TR-ALS-Sampled (the sampled ALS subproblem after
 *                          Algorithm alg:tr_als): the same sweep on m fibers
 *                          drawn by Algorithm SSDTP under ``law`` (U, L or E)
 *                          with the rows weighted by 1/sqrt(m p_f), i.e. the
 *                          TR-ScaledBRSGD step at alpha = 1 with H_n = F_n.
 * The full-batch methods run the sampled-step kernels on every column of
 * X_[n] once (p = 1/J_n: the stochastic gradient of eq:S_gradient is then
 * grad f / J_n exactly); J_n must not exceed 2^24. */
typedef enum { TR_METHOD_GD = 0, TR_METHOD_SCALED_GD = 1, TR_METHOD_ALS = 2,
               TR_METHOD_ALS_SAMPLED = 3 } tr_method;

typedef struct {
    int32_t method;     /* tr_method                                           */
    int32_t m;          /* TR-ALS-Sampled: fibers per block; otherwise unused   */
    int32_t law;        /* TR-ALS-Sampled: TR_LAW_UNIFORM/LEVERAGE/EUCLID       */
    int32_t prec;       /* tr_prec of the contractions                         */
    double alpha;       /* TR-GD / TR-ScaledGD step size (> 0)                 */
    double damping;     /* eta added to the normalised Hessian factor          */
    uint64_t seed;      /* TR-ALS-Sampled draws                                */
} tr_sweep_config;

/* Enqueue ``sweeps`` sweeps; each is N block updates in the order
 * n = 0..N-1 and advances *t_dev by one per block (TR-ALS-Sampled draws block
 * n of a sweep at step t = *t_dev with mode n fixed).  Cores are updated in
 * place; dev_status collects TR_DEV_* bits.  Graph-capturable.  ws: device
 * workspace of tr_sweep_workspace_size bytes, 256-byte aligned.  Laws L and E
 * need the problem's per-mode CDF buffers. */
size_t tr_sweep_workspace_size(const tr_problem* p, const tr_sweep_config* c);
tr_status tr_sweep_run(const tr_problem* p, const tr_sweep_config* c, uint64_t* t_dev, int32_t sweeps,
                       int32_t* dev_status, void* ws, size_t ws_bytes, tr_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tr_run_ex
 * with the library's own device scratch instead of a caller workspace.  The
 * scratch is a static device array of TR_NOALLOC_SCRATCH_BYTES on every GPU
 * the library runs on (kept until the process ends); its address on the
 * current GPU is looked up on the first call there.  The call allocates
 * nothing and computes exactly what tr_run_ex computes with a workspace.
 * A problem/config whose tr_run_workspace_size exceeds
 * TR_NOALLOC_SCRATCH_BYTES is rejected with TR_E_WORKSPACE (nothing
 * enqueued).  Every call on one GPU shares that GPU's scratch and the
 * scratch keeps the last call's contents (each step rewrites what it reads;
 * the step counter scratch is cleared by a kernel at the start of every
 * call): calls that overlap on one GPU (other streams, other host threads)
 * race and must be serialised by the caller.  The current device must be
 * the device of ``stream``. */
#define TR_NOALLOC_SCRATCH_BYTES (16u << 20)
tr_status tr_run_noalloc(const tr_problem* p, const tr_config* c, uint64_t* t_dev, int32_t steps,
                         double* loss_out, int32_t* dev_status, tr_stream_t stream,
                         const tr_run_opts* opts);

/* ------------------------------------------------------------------ */
/* a10: sampled-entry loss, forward and backward for every core        */
/* ------------------------------------------------------------------ */

/* L = 1/(2B) sum_b (Trace(G_0(i_0^b) ... G_{N-1}(i_{N-1}^b)) - x_b)^2.
 * idx int32 [B][N]; x [B] in the x dtype; resid float32 [B] receives the
 * residuals (prediction - x); loss: device float64 scalar.  FP32 cores. */
tr_status tr_entry_fwd(const tr_desc* d, const void* const* cores, const int32_t* idx,
                       const void* x, int32_t B, float* resid, double* loss,
                       void* ws, size_t ws_bytes, tr_stream_t stream);
/* grads[k] (host array of N device pointers, G_{k(2)} layout, FP32) =
 * scale * (*scale_dev) * dL/dG_k = scale * (*scale_dev) * (1/B) *
 * sum_b resid_b * dTrace/dG_k at i^b, i.e. the block gradient of
 * eq:gradient restricted to the sampled entries
 * (dTrace/dG_k(i_k) is the transposed product of the other N-1 slices in
 * ring order, recomputed per entry from the cores, not stored).
 * scale_dev: device float64 multiplier (an upstream gradient) or NULL.
 * Overwrites grads; the sum over entries runs in a fixed order. */
tr_status tr_entry_bwd(const tr_desc* d, const void* const* cores, const int32_t* idx,
                       const float* resid, int32_t B, double scale, const double* scale_dev,
                       void* const* grads, void* ws, size_t ws_bytes, tr_stream_t stream);
size_t tr_entry_workspace_size(const tr_desc* d, int32_t B);

/* Tensor completion in the ring format with a ridge regulariser (uses of
 * the framework named in the concluding remarks): minimise over the cores
 *     1/(2|Omega|) sum_{i in Omega} (TR(G)(i) - x_i)^2 + lambda/2 sum_k ||G_k||^2
 * from the observed entries Omega alone.  Each step draws B observed
 * entries uniformly with replacement (position floor(r |Omega| / 2^64) of
 * Omega, r the Philox word of counter (t, b, 0, TR_STREAM_ENTRY)), evaluates
 * the batch loss L = 1/(2B) sum_b r_b^2 + lambda/2 sum_k ||G_k||^2 and its
 * gradient (tr_entry_fwd / tr_entry_bwd's kernels: the block gradient of
 * eq:gradient restricted to the drawn entries, plus lambda G_k), and applies
 * p_k = -dL/dG_k with ``rule`` to every core, or with block = 1 to core n
 * only, n the step's mode (the block choice of Algorithm TR-BRSGD).
 * obs_idx: int32 [n_obs][N]; obs_x: [n_obs] in the x dtype (F32 or F16);
 * cores FP32 in place; accum: per-core AdaGrad accumulators (rule kind 1),
 * else may be NULL; loss_out: device float64 [steps] (each step's L before
 * its update) or NULL.  An observed index outside the tensor, when drawn,
 * gives a NaN residual and loss for that step and no gradient contribution.
 * *t_dev advances by one per step.  Graph-capturable. */
typedef struct {
    int32_t B;          /* observed entries drawn per step                    */
    int32_t block;      /* 1: only the step's mode moves; 0: every core       */
    double lambda;      /* ridge weight (>= 0)                                */
    tr_step rule;
    uint64_t seed;
} tr_completion_config;
size_t tr_completion_workspace_size(const tr_desc* d, const tr_completion_config* c);
tr_status tr_completion_run(const tr_desc* d, void* const* cores, void* const* accum, const int32_t* obs_idx,
                            const void* obs_x, int64_t n_obs, const tr_completion_config* c, uint64_t* t_dev,
                            int32_t steps, double* loss_out, int32_t* dev_status, void* ws, size_t ws_bytes,
                            tr_stream_t stream);

/* ------------------------------------------------------------------ */
/* a11: many independent problems in one persistent launch             */
/* ------------------------------------------------------------------ */

/* One problem of a batch: TR-BRSGD (Algorithm alg:TR_BRSGD) with uniform
 * fiber sampling (Section "Four probability distributions", the uniform
 * case) and the step rule ``rule``.  Cores FP32 (updated in place), the
 * tensor as FP16 mode-major replicas (tr_x_replicate layout, all N
 * required).  Limits: N <= 5, I_n <= 128, R_n <= 12 (R_n R_{n+1} <= 144). */
typedef struct {
    tr_desc desc;                        /* core_dtype TR_F32, x_dtype TR_F16 */
    void* cores[TR_MAX_ORDER];
    void* accum[TR_MAX_ORDER];           /* AdaGrad accumulators, or NULL     */
    const void* Xrep[TR_MAX_ORDER];      /* mode-major replicas, FP16         */
    uint64_t* t_dev;                     /* the problem's step counter        */
    double* loss;                        /* device float64: last step's loss estimate, or NULL */
    int32_t* dev_status;                 /* sticky TR_DEV_* bits, or NULL     */
    int32_t m;                           /* |F_n| drawn per step              */
    int32_t reserved;                    /* 0                                 */
    tr_step rule;
    uint64_t seed;
} tr_batch_item;

/* Bytes of the device table that holds ``count`` items. */
size_t tr_batch_table_size(int32_t count);
/* Validate ``count`` host items and copy them to the device table (caller
 * allocated, 256-byte aligned).  Fails (nothing enqueued) on the first
 * invalid item. */
tr_status tr_batch_upload(const tr_batch_item* items, int32_t count, void* table, size_t table_bytes,
                          tr_stream_t stream);
/* Advance every problem of the table by ``steps`` steps in one launch:
 * workgroup p owns problem p for all its steps (no inter-problem
 * synchronisation).  Per step the gradient GEMMs run on FP16 matrix cores
 * with FP32 accumulation; the loss estimate is FP64.  chunk (samples per
 * round: 32 or 64) and waves (wavefronts per workgroup: 4 or 8) are the
 * tile choice (see the package's batch tuner); every choice computes the
 * same step.  Graph-capturable. */
tr_status tr_batch_run(const void* table, int32_t count, int32_t steps, int32_t chunk, int32_t waves,
                       tr_stream_t stream);

/* The same steps with every problem's samples split over ``splits``
 * workgroups (1..16): per step one launch computes the partial gradients
 * and loss sums of all (problem, share) pairs into ``ws`` and a second adds
 * the shares in share order and takes each problem's step, so a batch of
 * fewer problems than compute units still fills the device.  The draws,
 * hence the sampled fibers, are those of tr_batch_run; only the order in
 * which the gradient's FP32 partial sums are added differs.  ``ws``:
 * caller-allocated device workspace of tr_batch_split_workspace_size bytes,
 * 256-byte aligned, contents not preserved.  Graph-capturable. */
size_t tr_batch_split_workspace_size(int32_t count, int32_t splits);
tr_status tr_batch_run_split(const void* table, int32_t count, int32_t steps, int32_t chunk, int32_t waves,
                             int32_t splits, void* ws, size_t ws_bytes, tr_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TR_H_ */
