/*
 * kerdock.h -- C ABI of the MI355X (gfx950) Kerdock fast sparsifying
 * transform: Fuchs, Gross, Krahmer, Kueng, Mixon, "Sketching with Kerdock's
 * crayons: fast sparsifying transforms for arbitrary linear maps",
 * arXiv 2105.05879.
 *
 * The library solves Problem 1 of the paper with Algorithm 1: it preprocesses
 * an arbitrary A in R^{m x n} once into the sketch {A s_l : l in [L]} of a
 * Kerdock-set projective 2-design (Lemma 8), and then, for a stream of unit
 * vectors x, returns the epsilon-hard threshold h_eps(Ax) restricted to the
 * rows that a median-of-means estimate (Theorem 5) ranks highest.
 *
 * Conventions shared by every entry point:
 *   - Device pointers are HIP device allocations on the current device
 *     (torch tensors' data_ptr() qualify).  Host pointers are marked "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on it; outputs are valid once the
 *     stream has been synchronised.  Prepare synchronises before returning.
 *   - Matrices are row-major FP32.  X holds one vector per row.
 *   - Return value: KERDOCK_OK (0) or a negative kerdock_status; the last
 *     error message of the calling thread is kerdock_last_error().
 *   - A handle owns all the device memory it allocates (tables, a copy of A,
 *     sign bitmaps, a growable workspace); kerdock_destroy frees it.  The
 *     caller keeps ownership of every pointer it passes.  Calls on one
 *     handle must not overlap (they share its workspace).
 */
#ifndef KERDOCK_H
#define KERDOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kerdock_handle_s *kerdock_handle;

/* Element type of the stored sketch tables.  FP32 is the plain method;
 * BF16 (round to nearest even) and FP8 E4M3 (OCP format, max 448, saturating
 * round to nearest even, divided by a per-row FP32 scale) are the precision
 * forms.  Accumulation is FP32 in every case. */
typedef enum {
    KERDOCK_F32 = 0,
    KERDOCK_BF16 = 1,
    KERDOCK_FP8E4M3 = 2
} kerdock_dtype;

typedef enum {
    KERDOCK_OK = 0,
    KERDOCK_ERR_INVALID_ARG = -1,   /* bad size, pointer, eps, s_max, J, K ... */
    KERDOCK_ERR_UNSUPPORTED_N = -2, /* n outside [1, 4096] (d = 16384 beyond) */
    KERDOCK_ERR_OOM = -3,           /* a device allocation failed            */
    KERDOCK_ERR_HIP = -4,           /* a HIP runtime call or launch failed   */
    KERDOCK_ERR_NOT_PREPARED = -5   /* NULL or destroyed handle              */
} kerdock_status;

/* Geometry of a prepared handle (Algorithm 1, preprocessing step). */
typedef struct {
    int32_t m, n;          /* A is m x n                                      */
    int32_t k;             /* smallest even k with d = 2^k >= n (Lemma 8)     */
    int32_t d;             /* 2^k                                             */
    int64_t L;             /* design size d (d/2 + 1)                         */
    int32_t pitch;         /* elements between consecutive table columns     */
    uint32_t field_poly;   /* irreducible polynomial of F_{2^{k-1}} (bits)   */
    kerdock_dtype dtype;
    size_t table_bytes;    /* bytes of the sketch table in device memory      */
    float build_ms;        /* device time of the table construction kernels
                              in kerdock_prepare (HIP events around them)    */
} kerdock_info;

/* Streaming parameters (Algorithm 1 streaming step, Theorem 5).  A zeroed
 * struct is invalid (J = K = 0): set J and K. */
typedef struct {
    int32_t J;             /* samples per batch                               */
    int32_t K;             /* number of batches; N = J K draws per x          */
    uint64_t seed;         /* key of the Philox4x64-10 draws                  */
    int64_t t0;            /* stream position of X row 0: draw j of row t is a
                              pure function of (seed, t0 + t, j)              */
    float tau;             /* optional floor on |mu| inside S (0 = none)      */
    /* optional device outputs for parity checks (NULL = not written):       */
    uint32_t *dbg_samples; /* [batch][N] drawn design indices l_j (set together
                              with dbg_coef)                                  */
    float *dbg_coef;       /* [batch][N] s_{l_j}^T x                          */
    float *dbg_mu;         /* [batch][m] median-of-means estimate             */
    int32_t *dbg_survivors;/* [batch][s_max] S ascending, -1 padded           */
    float *dbg_values;     /* [batch][s_max] a_i.x for every i in S, 0 padded */
    /* optional host [4]: when set, the call records HIP events on `stream`
       around its kernels, waits for them and stores their durations in ms:
       [0] grouping of the draws by basis (0 when the call does not group
       them), [1] draws, coefficients and gather, [2] batch means, median
       and selection, [3] survivor dots and threshold. */
    float *kernel_ms;
    /* draws per FP32 partial sum of a batch mean: consecutive draws of
       the batch, in drawing order or, when the call groups its draws by
       basis (a cost rule of the handle: a few draws per basis on average
       and columns short against x, or the autotuned choice), in that
       order.  The exact rounding of mu depends on this and on nothing else
       about the launch (batch size, workgroup shape and unroll leave it
       unchanged): 0 = the value that
       kerdock_autotune stored in the handle, else min(C, max(16,
       ceil(J / 8))) with C = 768 for FP8 tables and 512 otherwise;
       1..1024 = that many (capped at J); other values are INVALID_ARG. */
    int32_t chunk;
} kerdock_apply_params;

/*
 * kerdock_prepare -- preprocessing step of Algorithm 1 via Lemma 8.
 *   A       device, m x n row-major FP32 (read; copied into the handle).
 *   m, n    1 <= m <= 16384, 1 <= n <= 4096.
 *   dtype   element type of the stored table.
 *   stream  HIP stream (void*); prepare synchronises it before returning.
 *   out     host; receives the new handle.
 * Builds, for k even with d = 2^k >= n and L = d(d/2+1), the table column
 * T[l] = A s_l for every l = b d + w: Kerdock blocks b < d/2 use the vectors
 * (-1)^{Q_b(x) + w.x} of equation (3) with the Kerdock matrices of
 * Proposition 7 (computed as a fast Walsh-Hadamard transform of A's signed
 * rows); block b = d/2 is the identity basis, T[l] = sqrt(d) A e_w (zero for
 * w >= n).  Errors: INVALID_ARG (NULL pointer, m < 1, m > 16384), UNSUPPORTED_N,
 * OOM (table larger than free device memory), HIP.
 */
int kerdock_prepare(const float *A, int m, int n, kerdock_dtype dtype, void *stream,
                    kerdock_handle *out);

/*
 * kerdock_sparse_apply -- streaming step of Algorithm 1 for `batch` vectors.
 *   X        device, batch x n row-major FP32, rows are unit vectors (the
 *            library does not normalise them: Problem 1 assumes unit x).
 *   batch    >= 0 (0 is a no-op).
 *   eps      > 0, the hard threshold of Problem 1 (|v| >= eps is kept).
 *   s_max    1 <= s_max <= m: size of S, the rows of largest |mu| (the
 *            numerical section uses 10 s).
 *   p        host; J >= 1, K >= 1 and the optional fields above.
 *   out_idx  device [batch][s_max] int32: kept row indices, ascending,
 *            padded with -1.
 *   out_val  device [batch][s_max] FP32: (Ax)_i for the kept rows, computed
 *            exactly from FP32 A and x (compensated dot product), 0 padded.
 *   out_cnt  device [batch] int32: number of kept rows, or -1 when some
 *            a_i.x with i in S is not finite (an inf or NaN in x or in a
 *            selected row of A); that vector's rows are then all padding.
 * For every row x: draws l_j (j < N) uniformly from [L]; forms
 * y_j = T[l_j] (s_{l_j}^T x); averages each batch of J draws; takes the
 * entrywise median of the K means (the mean of the two middle values for
 * even K); selects S = the s_max rows of largest |mu| (ties: smaller index),
 * optionally only those with |mu| >= tau; computes a_i.x for i in S and
 * keeps |a_i.x| >= eps.  May grow the handle's workspace (hipMalloc) unless
 * kerdock_reserve was called with sizes at least as large.  Calls on one
 * handle share its workspace: calls that overlap in time on one handle race
 * and must be serialised by the caller.
 * Errors: NOT_PREPARED, INVALID_ARG (NULL pointers with batch > 0, eps <= 0
 * or NaN, s_max out of range, J < 1, K < 1, K > 32, J K > 2^31), OOM, HIP.
 */
int kerdock_sparse_apply(kerdock_handle h, const float *X, int batch, float eps, int s_max,
                         const kerdock_apply_params *p, int32_t *out_idx, float *out_val,
                         int32_t *out_cnt, void *stream);

/*
 * kerdock_sparse_apply_static -- kerdock_sparse_apply for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels, draws and
 * results as kerdock_sparse_apply (bit for bit), but the workspace (chunk
 * partial sums, S, survivor values, row grouping) lives in a fixed device
 * array of KERDOCK_STATIC_SCRATCH_BYTES inside the library, one per device,
 * held until the process ends; the call allocates nothing.  A call whose
 * workspace would exceed it fails with INVALID_ARG (use fewer vectors per
 * call; the workspace grows with batch K ceil(J / chunk) 4 pitch bytes).
 * kernel_ms must be NULL.  Every call on a device shares that device's
 * array, so calls that overlap in time on one device (different streams,
 * host threads) race and must be serialised by the caller.
 * Errors: those of kerdock_sparse_apply, with OOM replaced by INVALID_ARG.
 */
#define KERDOCK_STATIC_SCRATCH_BYTES (64u << 20)
int kerdock_sparse_apply_static(kerdock_handle h, const float *X, int batch, float eps, int s_max,
                                const kerdock_apply_params *p, int32_t *out_idx, float *out_val,
                                int32_t *out_cnt, void *stream);

/*
 * kerdock_reserve -- allocate the workspace that kerdock_sparse_apply needs
 * for up to `batch` vectors with N = J K draws and the given s_max, so that
 * later calls within these sizes allocate nothing (needed before capturing
 * the calls in a HIP graph).  Errors: NOT_PREPARED, INVALID_ARG, OOM.
 */
int kerdock_reserve(kerdock_handle h, int batch, int J, int K, int s_max);

/*
 * kerdock_autotune -- pick the gather shape for this handle: draws per
 * workgroup (256, 512, 1024), draws in flight per thread and (when a batch
 * holds at least two draws per basis on average) whether the draws are
 * grouped by basis first, by timing the draws + gather kernels on X
 * (device, batch x n) with N = J K draws, three runs each (the first one
 * discarded).  The choice is kept in the handle for
 * later calls and, when the environment variable KERDOCK_TUNE_CACHE names a
 * file, appended to it and read back by later kerdock_prepare calls of the
 * same shape.  Outputs (host, optional): best_chunk, best_unroll, best_ms.
 * Synchronous.  Errors: NOT_PREPARED, INVALID_ARG, OOM, HIP.
 */
int kerdock_autotune(kerdock_handle h, const float *X, int batch, int J, int K, void *stream,
                     int *best_chunk, int *best_unroll, float *best_ms);

/* ----------------------------------------------------------------------- */
/* Batched form: several prepared matrices in one persistent launch.        */
/* ----------------------------------------------------------------------- */

#define KERDOCK_MAX_MULTI 8

typedef struct kerdock_multi_s *kerdock_multi;

/*
 * kerdock_multi_create -- a plan that runs the streaming step of Algorithm 1
 * for nh (1..8) prepared matrices at once.  Per handle q: X[q] device rows
 * [batch[q]][n_q] (batch[q] >= 1), params[q] (J, K, seed, t0 and tau; the
 * debug and timing fields are ignored), s_max[q] in [1, m_q] and device
 * outputs out_idx[q], out_val[q] [batch[q]][s_max[q]], out_cnt[q]
 * [batch[q]] with the meaning of kerdock_sparse_apply.  All handles must
 * share one table dtype and have columns of at most 16 KiB.  The pointers are
 * bound to the plan: every run reads the current contents of X[q] and
 * rewrites the outputs.  The plan owns a workspace (allocated here) and
 * must not outlive its handles.  Each handle's tuned draws-per-workgroup
 * (kerdock_autotune) is used.  Errors: INVALID_ARG, NOT_PREPARED, OOM, HIP.
 */
int kerdock_multi_create(const kerdock_handle *hs, int nh, const float *const *X, const int *batch,
                         const kerdock_apply_params *params, float eps, const int *s_max,
                         int32_t *const *out_idx, float *const *out_val, int32_t *const *out_cnt,
                         kerdock_multi *out);

/*
 * kerdock_multi_run -- enqueue one pass on `stream` (kernels only, no
 * allocation, no memset, no synchronisation, so it can be captured in a
 * graph): the draws + gather of every (handle, vector, chunk) work item in one
 * persistent launch whose workgroups take items longest-column first, then
 * selection and survivor dots for every vector, then every stream position
 * advances by its batch, so that consecutive runs draw for consecutive
 * stream positions (the results for handle q equal those of
 * kerdock_sparse_apply at the same stream position).
 */
int kerdock_multi_run(kerdock_multi plan, void *stream);

/* kerdock_multi_set_position -- set the stream positions (host t0[nh]) of the
 * next run.  Synchronises the device. */
int kerdock_multi_set_position(kerdock_multi plan, const int64_t *t0);

/* kerdock_multi_graph_launch -- on the first call capture one run into a HIP
 * graph owned by the plan; launch that graph on `stream`. */
int kerdock_multi_graph_launch(kerdock_multi plan, void *stream);

/* kerdock_multi_autotune -- time the persistent gather with each available
 * unroll depth (two runs each) and keep the fastest (host best_unroll,
 * optional).  Drops a previously captured graph.  Synchronous. */
int kerdock_multi_autotune(kerdock_multi plan, void *stream, int *best_unroll);

/* kerdock_multi_destroy -- free the plan (after synchronising the device). */
int kerdock_multi_destroy(kerdock_multi plan);

/* kerdock_sparse_apply_multi -- create a plan, run it once, synchronise
 * `stream`, destroy the plan. */
int kerdock_sparse_apply_multi(const kerdock_handle *hs, int nh, const float *const *X, const int *batch,
                               const kerdock_apply_params *params, float eps, const int *s_max,
                               int32_t *const *out_idx, float *const *out_val, int32_t *const *out_cnt,
                               void *stream);

/* ----------------------------------------------------------------------- */
/* Learned-proposal form.                                                   */
/* ----------------------------------------------------------------------- */

typedef struct kerdock_mlp_s *kerdock_mlp;

/*
 * kerdock_mlp_create -- an MLP z = W3 relu(W2 relu(W1 f + b1) + b2) + b3 with
 * d_in -> h1 -> h2 -> d_out units (each in [1, 16384]) that proposes the rows
 * of h_eps(Ax) from the basis coefficients f of x.  FP32 master parameters
 * (He-uniform weights from `seed`, zero biases), a BF16 copy for the GEMMs
 * (FP32 accumulation), Adam state.  Lives on the current device.
 * Parameter layout (kerdock_mlp_get_params): W1 [h1][d_in], b1 [h1],
 * W2 [h2][h1], b2 [h2], W3 [d_out][h2], b3 [d_out], FP32, concatenated.
 */
int kerdock_mlp_create(int d_in, int h1, int h2, int d_out, uint64_t seed, kerdock_mlp *out);
int kerdock_mlp_param_count(kerdock_mlp net, size_t *count);
/* host <-> device copies of the FP32 parameters; set also refreshes the BF16
 * copy and resets the Adam state.  Synchronous. */
int kerdock_mlp_get_params(kerdock_mlp net, float *host);
int kerdock_mlp_set_params(kerdock_mlp net, const float *host);

/* kerdock_mlp_forward -- logits Z [B][d_out] (device, FP32) from features
 * F [B][d_in] (device, FP32, rounded to BF16 as GEMM input). */
int kerdock_mlp_forward(kerdock_mlp net, const float *F, int B, float *Z, void *stream);

/*
 * kerdock_mlp_train_step -- one step of binary cross-entropy with logits
 * against labels Y [B][d_out] (device, uint8 0/1) with positive weight
 * pos_weight: loss = mean over all entries of
 * -[w+ y log s(z) + (1 - y) log(1 - s(z))], written to loss (device [1]).
 * Backward with BF16 GEMM inputs (activations and gradients rounded at the
 * GEMM boundaries) and FP32 accumulation; gradients in the parameter layout
 * are copied to grads (device, optional); if lr > 0 an Adam step
 * (beta1 0.9, beta2 0.999, eps 1e-8) updates the parameters.
 */
int kerdock_mlp_train_step(kerdock_mlp net, const float *F, const uint8_t *Y, int B, float lr,
                           float pos_weight, float *loss, float *grads, void *stream);
int kerdock_mlp_destroy(kerdock_mlp net);

/* kerdock_features -- F [B][d] = H_d x / sqrt(d) (x zero-padded to d): the
 * coefficients of x in the first Kerdock basis (M_0 = 0, Section 3), the
 * input of the proposal network.  X device [B][n], F device [B][d]. */
int kerdock_features(kerdock_handle h, const float *X, int B, float *F, void *stream);

/* kerdock_learned_attach -- use `net` (d_in = d, d_out = m) as the row
 * proposer of handle h; builds G = A^T A (FP32) once.  The network must
 * outlive the attachment.  Synchronous. */
int kerdock_learned_attach(kerdock_handle h, kerdock_mlp net);

/*
 * kerdock_learned_apply -- h_eps(Ax) with the learned proposal: features,
 * logits, C = the s_max rows of largest logit, exact a_i.x on C (compensated
 * dot product), threshold at eps; then the energy |Ax|^2 = x^T G x (G = A^T A
 * as a compensated pair, quadratic form with compensated sums) is compared
 * with the verified energy S = sum_{i in C} (a_i.x)^2, together with a
 * rigorous bound B on the FP32 rounding of both; a row is kept only when
 * |Ax|^2 - S <= eps^2 / 2 and B < eps^2 / 2, every other row is recomputed by
 * the plain streaming step of kerdock_sparse_apply with parameters p.  A row
 * of h_eps(Ax) outside C leaves at least eps^2 of energy outside C, so no
 * such row is ever accepted without the fallback, in floating point too.
 * (B grows like (m u)^2 |A|_F^2 |x|^2: when it reaches eps^2 / 2 every row
 * falls back.)  fallback (device [B] int32) receives 1 for the recomputed
 * rows.  Outputs as in kerdock_sparse_apply.  Debug: when p->dbg_survivors
 * is given it receives the candidate set C of every row ([B][s_max],
 * ascending, padded with -1); when p->dbg_mu is given (m >= 3), entries 0,
 * 1, 2 of its row t receive the computed |Ax|^2, S and B of vector t; the
 * other debug fields and kernel_ms are ignored.  Errors: NOT_PREPARED (no
 * attached network), INVALID_ARG, OOM, HIP.
 */
int kerdock_learned_apply(kerdock_handle h, const float *X, int B, float eps, int s_max,
                          const kerdock_apply_params *p, int32_t *out_idx, float *out_val,
                          int32_t *out_cnt, int32_t *fallback, void *stream);

/*
 * kerdock_sparse_apply_shared -- the streaming step with draws shared by
 * groups of KERDOCK_SHARED_TILE consecutive rows of X.  Rows t with the same
 * g = floor(t / KERDOCK_SHARED_TILE) use the N = J K indices drawn at stream
 * position t0 + g of a second Philox stream (counter (floor(j/4), t0 + g, 1,
 * 0), key (seed, 0)).  The draws never depend on x, so for every single x
 * they are N independent uniform draws as in Algorithm 1 and Theorem 5's
 * bound holds per x (the events of two vectors of one group are no longer
 * independent).  With one draw list per group the batch sums become the
 * matrix product of the gathered table columns and the coefficient block of
 * the group, which reads each drawn column once per group (FP32 tables on
 * the FP32 matrix cores; BF16 and FP8 tables on the BF16 matrix cores with
 * each FP32 coefficient split exactly into three BF16 parts, so that every
 * product is exact and only the FP32 accumulation rounds).  Arguments,
 * outputs, errors and the debug outputs are those of kerdock_sparse_apply
 * (dbg_samples row t holds its group's draws); params->chunk is ignored (the
 * batch sums are accumulated by the matrix cores), J K must stay below 2^26,
 * and kernel_ms receives [0] draws + coefficients, [1] matrix product,
 * [2] median and selection, [3] survivor dots and threshold.
 */
#define KERDOCK_SHARED_TILE 64
int kerdock_sparse_apply_shared(kerdock_handle h, const float *X, int batch, float eps, int s_max,
                                const kerdock_apply_params *p, int32_t *out_idx, float *out_val,
                                int32_t *out_cnt, void *stream);

/*
 * kerdock_theory_params -- the streaming parameters of Theorem 5 for a target
 * failure probability eta (0 < eta < 1) and x in Sigma(A, s, delta):
 * gamma = (eps - delta) / 2, J = ceil(4 e^2 |A|_{2->inf}^2 / gamma^2),
 * K = ceil(2 log(m / eta)), so that |mu - Ax|_inf < gamma with probability
 * at least 1 - eta; tau = (eps + delta) / 2 (the separation of Section 1)
 * and |A|_{2->inf}^2 (largest squared row norm, FP32) are returned too
 * (host outputs; tau and norm2inf optional).  Errors: NOT_PREPARED,
 * INVALID_ARG (eps <= delta, delta < 0, eta outside (0, 1), or J K beyond
 * the supported range).
 */
int kerdock_theory_params(kerdock_handle h, float eps, float delta, float eta, int32_t *J, int32_t *K,
                          float *tau, float *norm2inf);

/* kerdock_query -- geometry of a handle; `info` is host memory. */
int kerdock_query(kerdock_handle h, kerdock_info *info);

/*
 * kerdock_read_columns -- dequantised table columns, for parity checks.
 *   ells  device [count] uint32 design indices (< L).
 *   out   device [count][m] FP32: T[l] as stored (times the row scale for
 *         FP8 tables).
 */
int kerdock_read_columns(kerdock_handle h, const uint32_t *ells, int count, float *out,
                         void *stream);

/*
 * kerdock_debug_signs -- the sign pattern (-1)^{Q_b(x)} of Kerdock basis
 * b < d/2 (equation (3) with w = 0), as d/32 host words: bit x mod 32 of word
 * x / 32 is Q_b(x).  Synchronous.
 */
int kerdock_debug_signs(kerdock_handle h, int b, uint32_t *out_bits);

/*
 * kerdock_row_scales -- per-row FP32 scales of an FP8 table (1 for the other
 * dtypes): max(|a_i|_1, sqrt(d) |a_i|_inf) / 448, a bound on every |T[l]_i|.
 *   out  device [m].
 */
int kerdock_row_scales(kerdock_handle h, float *out, void *stream);

/* kerdock_destroy -- free every device allocation of the handle. */
int kerdock_destroy(kerdock_handle h);

/* kerdock_last_error -- message of the last failing call on this thread. */
const char *kerdock_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KERDOCK_H */
