/*
 * lp.h -- C ABI of the MI355X LocalPower library (liblp.so).
 *
 * LocalPower (Li, Wang, Chen, Zhang, "Communication-Efficient Distributed SVD
 * via Local Power Iterations", Algorithm 1) computes an orthonormal basis Z
 * (d x k) of the top-k right singular subspace of a row-partitioned matrix
 * A = [A_1; ...; A_m] (A_i is s_i x d).  Every communication round each of the
 * m partitions ("nodes") runs p local power iterations
 *     Y_i = M_i Z_i,  M_i = A_i^T A_i / s_i          (Eq. (power_yi))
 *     Z_i = orth(Y_i)                                   (between local steps)
 * then the inputs of the last local step are aligned against the base node
 * (sign-fixing, Eq. (opt:d), or orthogonal Procrustes, Eq. (opt:o)) and the
 * server aggregates Y = sum_i (s_i/n) Y_i D_i and orthonormalises it.
 * All m nodes run on one GPU; a "round" is one aggregation.
 *
 * Conventions for every entry point:
 *   - Every call returns lp_status; nothing throws or aborts across the ABI.
 *     lp_last_error() returns a thread-local description of the last failure.
 *   - "device" pointers are GPU memory of the current HIP device; "host"
 *     pointers are CPU memory.  Matrices are row-major with the stated leading
 *     dimension; d x k matrices are dense (leading dimension k).
 *   - Inputs are BORROWED (the caller keeps them alive while in use); outputs
 *     are caller-owned.  Problems allocate no device memory: their scratch
 *     lives in the workspace the caller passes to lp_create (and, for the
 *     local-Gram form and eta, in the buffer passed to lp_gram_enable);
 *     lp_sin_theta uses one of 64 result cells the library holds in static
 *     device memory.  The serving layer (lp_server_*) is the exception: it
 *     allocates one device arena of its budget at lp_server_create (freed by
 *     lp_server_destroy) and places each admitted job's footprint in a free
 *     range of it; plus pinned host cells.
 *   - All GPU work is enqueued on the stream given to lp_create (a hipStream_t;
 *     NULL means the legacy default stream); calls that return host results
 *     synchronise that stream before returning.
 *   - orth(Y) is the Q factor of the thin QR Y = QR with positive diagonal R
 *     (computed by CholeskyQR2 in FP64), the unique choice of the paper's
 *     "QR factorisation" orth.
 */
#ifndef LP_H
#define LP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LP_OK = 0,
  LP_EINVAL = -1,      /* invalid argument (see the entry point's contract) */
  LP_ENOMEM = -2,      /* workspace too small / admission refused for memory */
  LP_EDEVICE = -3,     /* a HIP call failed */
  LP_EBREAKDOWN = -4,  /* Cholesky of a Gram matrix broke down (rank-deficient iterate) */
  LP_ENOTCONV = -5,    /* a stop target was not reached within max_rounds */
  LP_EBUSY = -6        /* resource busy (no free serving slot) */
} lp_status;

typedef enum { LP_F64 = 0, LP_F32 = 1, LP_BF16 = 2 } lp_dtype;

/* Alignment of the local iterates before aggregation: the set F of the
 * unified update rule (Eq. (D0)): {I} (vanilla), D_k (sign-fixing, Eq.
 * (opt:d)), O_k (orthogonal Procrustes, Eq. (opt:o)). */
typedef enum { LP_AGG_VANILLA = 0, LP_AGG_SIGN = 1, LP_AGG_OPT = 2 } lp_agg;

typedef struct lp_problem lp_problem; /* opaque */

const char* lp_strerror(lp_status s);
const char* lp_last_error(void);

/* Bytes of device workspace lp_create needs for this problem.
 *   dtype, n, d : storage type and shape of A (n rows = samples, d columns);
 *   offsets     : host int64[m+1], offsets[0] = 0, offsets[m] = n, strictly
 *                 increasing: partition i is rows [offsets[i], offsets[i+1]);
 *   k_max       : the largest k any later lp_run will use (1 <= k_max <= d).
 * Writes the byte count to *bytes.  LP_EINVAL on inconsistent arguments. */
lp_status lp_workspace_size(lp_dtype dtype, int64_t n, int64_t d, const int64_t* offsets,
                            int32_t m, int32_t k_max, size_t* bytes);

/* Create a problem over a row-partitioned matrix (Section 2, data parallelism:
 * the rows of A are split into m contiguous partitions, one per node).
 *   A          : device, n x d row-major with leading dimension lda >= d,
 *                16-byte aligned, element type `dtype`; BORROWED until
 *                lp_destroy.  FP32/BF16 values are multiplied with FP32
 *                accumulation, FP64 values in FP64.
 *   offsets    : host int64[m+1] as for lp_workspace_size; COPIED.
 *   workspace  : device, >= lp_workspace_size(...) bytes, 256-byte aligned;
 *                BORROWED until lp_destroy.
 *   stream     : hipStream_t on which all work of this problem is enqueued.
 * The base node (the alignment target) is the partition with the most rows,
 * lowest index on ties.  LP_EINVAL for bad shapes/offsets/alignment, LP_ENOMEM
 * when ws_bytes is too small. */
lp_status lp_create(lp_problem** out, const void* A, lp_dtype dtype, int64_t n, int64_t d,
                    int64_t lda, const int64_t* offsets, int32_t m, int32_t k_max,
                    void* workspace, size_t ws_bytes, void* stream);

lp_status lp_destroy(lp_problem* P);

/* Tuning of the local-multiply kernel (what the autotuner varies).
 *   local_kernel: 0 automatic; 1 two-pass kernel (t = A Z, then A^T t; FP32 matrix cores
 *                 for FP32/BF16 A, FP64 arithmetic for FP64 A).  Fused matrix-core kernels
 *                 (A read once), one workgroup per CU:
 *                 FP32 A (k <= 16, d in {256, 512, 768, 1024}; a rank below 16 runs the
 *                 16-wide tiles with zero columns of Z): 2 four waves; 3 eight waves;
 *                 4 software-pipelined (two LDS tiles, product 2 of one tile interleaved with
 *                 product 1 of the next), eight waves; 5 pipelined, four waves; 6 eight
 *                 waves with the next two tiles in flight (deeper prefetch); 7 direct-to-LDS
 *                 tile loads (eight waves at d = 1024, else four); 8 direct-to-LDS, four
 *                 waves; 9 direct-to-LDS and software-pipelined (product 2 of one tile
 *                 overlapping the operand reads of the next; eight waves at d = 1024,
 *                 else four); 10 direct-to-LDS with two tiles in flight per wave (eight
 *                 waves at d = 1024, else four).  The eight-wave forms need d in {512, 1024} (else they run
 *                 with four waves).
 *                 BF16 A (k <= 32, d in {512, 1024, 1536, 2048}, the 16- or 32-wide tiles
 *                 padded likewise; Z and t rounded to BF16 as operands): 2 four waves;
 *                 3 eight waves (d in {1024, 2048});
 *                 4 and 5 the same with two tiles in flight per wave.
 *                 With local_kernel 0, ranks k <= 8 (FP32 or BF16 A, d a power of two in
 *                 [256, 4096]) run a fused vector-ALU kernel (A read once, FP32
 *                 arithmetic, no matrix cores), other ranks of the fused shapes the fused
 *                 matrix-core kernel in its default form (FP32: 9; BF16: 2); naming a
 *                 kernel (1..11) runs that one.  Other shapes and ranks use the two-pass
 *                 kernel.  (The serving layer, which does not autotune, runs ranks 5..8
 *                 of FP32 and 1..8 of BF16 A on the fused matrix-core kernel where one
 *                 takes the shape: measured faster there.)
 *                 11: the two-pass kernel on BF16 matrix cores: every FP32 operand (A,
 *                 Z_i, t) split exactly into three BF16 pieces and the six leading
 *                 partial products summed in FP32 (dropped terms below 2^-23 of each
 *                 product: FP32-class results); BF16 A needs three products.  With
 *                 local_kernel 0 the two-pass shapes run this form for BF16 A and for
 *                 k > 16, the FP32-matrix-core form (1) otherwise.
 *   chunk_rows  : rows of A per workgroup work item (a multiple of 16, at least the
 *                 default chosen at lp_create, which sized the workspace); 0 = default.
 *   cached_loads: 1 reads A with ordinary (cached) loads in the fused kernels; 0 (default)
 *                 with nontemporal loads, since A is streamed once per local iteration.
 *   split_operands: BF16 A only.  0 (default): the fused BF16 kernel rounds Z and
 *                 t = A Z once to BF16 (a sin theta floor near 1e-3 against FP64 on the
 *                 same values, within the BF16 tolerance of 2e-2).  1: each operand is a
 *                 pair hi = bf16(x), lo = bf16(x - hi) and every product is taken twice,
 *                 FP32-class results for twice the matrix-core work.  Where no fused
 *                 kernel takes the shape (and at k > 16, d = 2048, where the pairs do not
 *                 fit a CU's registers), local_kernel 0 runs the two-pass kernel on BF16
 *                 matrix cores with Z_i and t as the same pairs (two BF16 products per
 *                 FP32 product instead of three); a named two-pass kernel (1 or 11) keeps
 *                 its own operands.  The autotuner keeps this setting. */
typedef struct {
  int32_t struct_size;
  int32_t local_kernel;
  int64_t chunk_rows;
  int32_t cached_loads;
  int32_t split_operands;
} lp_tuning;

/* Apply a tuning to a problem (host-side; re-uploads the work list on the problem's
 * stream and drops captured graphs).  LP_EINVAL for values outside the ranges above. */
lp_status lp_set_tuning(lp_problem* P, const lp_tuning* t);

/* Read the tuning in effect (local_kernel reports the variant actually used for k = 16). */
lp_status lp_get_tuning(lp_problem* P, lp_tuning* t);

/* Pick the fastest local-multiply tuning for rank k on this problem and apply it.
 * Times every candidate (kernel variant x work-item size x load flavour) with HIP events
 * around a few launches on the problem's stream (A is only read; the workspace's working
 * copy of Z is overwritten with zeros).  cache_path: text file of earlier choices keyed by
 * device architecture, dtype, n, d, m, k and lda (read first, appended to); NULL uses the
 * environment variable LP_AUTOTUNE_CACHE, and no cache when that is unset.  Writes the
 * chosen tuning to *chosen (may be NULL).  Synchronous. */
lp_status lp_autotune(lp_problem* P, int32_t k, const char* cache_path, lp_tuning* chosen);

/* Options of lp_run; zero-initialise and set struct_size = sizeof(lp_run_opts). */
typedef struct {
  int32_t struct_size;
  const double* U_ref;  /* device d x k FP64 orthonormal reference or NULL */
  double* sin_hist;     /* host [T]: sin theta_k(Z_r, U_ref) after each round, or NULL */
  int8_t* signs_out;    /* host [T*m*k]: sign-fixing decisions (+1/-1) per round, 0 where
                           the round used none (p = 1 or another mode); or NULL */
  int32_t z0_orthonormal; /* 1: Y0 is already orthonormal and is used as Z_0 as is
                             (resume from a saved round); 0: Z_0 = orth(Y0) */
  int32_t use_graph;    /* 1 (default when struct_size covers it and it is 1): replay each
                           round shape as a captured hipGraph; 0: plain launches */
  int32_t time_local;   /* 1: bracket every local-multiply launch with a pair of HIP events
                           on the problem's stream (captured as event nodes when rounds are
                           replayed as graphs) and report their summed duration in
                           stats->ms_local; 2: the same for the first local-multiply launch
                           of every round only (each event pair costs a few microseconds of
                           stream time, so sampling keeps the rounds close to untimed
                           speed); 0: no events */
  int32_t split_rounds;  /* with m >= 2, run the partitions in two halves on two streams,
                            each half's orthonormalisations and alignment overlapping the
                            other half's local multiplies (bitwise the same results):
                            1 always, 2 never, 0 (default) when rank k's local multiply
                            runs on the two-pass kernels (many workgroups per work item,
                            so each half still fills the GPU; the fused kernels run one
                            workgroup per item, and half the items leave half the chip
                            idle) */
  int32_t k_ref;         /* columns of U_ref: 0 (default) means k; else 1 <= k_ref <= k, so
                            the run iterates at rank k (the iteration rank r of Algorithm 1,
                            r >= target rank) and sin_hist records sin theta_{k_ref}(Z_r,
                            U_ref) = ||(I - Z_r Z_r^T) U_ref|| with Z_r of k columns (the
                            distance of the appendix on the eigengap, Theorem there) */
  double* rho_out;       /* host [T] or NULL: the residual error of Definition 3 at each
                            round's last local step (its largest in the round), measured on
                            the inputs of that step against the first partition's:
                            max_i ||Z_i - Z_1||_2, or with OPT max_i min_O ||Z_i O - Z_1||_2
                            = 2 sin(theta_max(Z_i, Z_1) / 2); 0 for rounds with p = 1.
                            Rounds then run on one stream. */
  uint64_t seed;         /* with Y0 == NULL: the Gaussian start is drawn from this seed
                            (Philox4x32-10, element e = i k + j of the d x k start from
                            counter (e mod 2^32, e / 2^32, 0, 0x5a300001) under key (seed
                            mod 2^32, seed / 2^32); Box-Muller, cosine branch, of the
                            uniforms (w0 / 2^5 * 2^26 + w1 / 2^6 + 1) / 2^53 and likewise
                            from w2, w3) */
} lp_run_opts;

typedef struct {
  int32_t rounds;          /* communication rounds completed */
  int32_t local_iters;     /* local power iterations per node completed */
  int32_t breakdowns;      /* Cholesky breakdowns detected (0 on success) */
  int32_t near_singular;   /* OPT alignments whose Z_i^T Z_b was singular or too close to
                              singular for the polar iteration to converge (O not unique) */
  double ms_total;         /* duration of the rounds on the stream (HIP events) */
  double bytes_A;          /* algorithmic bytes of A streamed: local_iters * n * d * elem */
  double ms_local;         /* with opts->time_local: summed duration of the local-multiply
                              launches (HIP events), else 0 */
  int32_t local_launches;  /* local-multiply launches timed into ms_local */
  int32_t graph_rounds;    /* rounds replayed from captured hipGraphs */
  int32_t split_rounds;    /* 1 when the rounds ran in two halves on two streams */
} lp_run_stats;

/* Run LocalPower (Algorithm 1) for T communication rounds.
 *   k       : iteration rank r of Algorithm 1, 1 <= k <= k_max, k <= every s_i.  With a
 *             target rank below it (oversampling), pass the target as opts->k_ref and
 *             ritz_out: the first k_ref columns of Z_out (Ritz vectors, descending) and
 *             of ritz_out are the target-rank results.
 *   p_sched : host int32[T], p_sched[r] >= 1 local iterations in round r (fixed p,
 *             a decaying schedule, or p = T total for one-shot); COPIED.
 *   mode    : alignment used when p_sched[r] >= 2 (rounds with p = 1 use none).
 *   Y0      : device d x k FP64 start matrix (the Gaussian Y_0 of Algorithm 1);
 *             Z_0 = orth(Y0) unless opts->z0_orthonormal.  NULL: Y_0 is drawn on the
 *             device from opts->seed (seed 0 without opts) and Z_0 = orth(Y_0).
 *   Z_out   : device d x k FP64, receives Z_T = orth(aggregate of the last round).
 *   ritz_out: device [k] FP64 or NULL: when given, one extra p = 1 pass forms
 *             H = Z^T M Z, Z_out is rotated to its eigenvectors and ritz_out gets the
 *             Ritz values (eigenvalues of M = A^T A / n) in descending order.
 *   opts, stats : may be NULL.
 * Synchronises the stream before returning.  On LP_EBREAKDOWN Z_out holds the last
 * valid Z and stats->rounds how many rounds completed. */
lp_status lp_run(lp_problem* P, int32_t k, const int32_t* p_sched, int32_t T, lp_agg mode,
                 const double* Y0, double* Z_out, double* ritz_out, const lp_run_opts* opts,
                 lp_run_stats* stats);

/* Options of lp_solve; zero-initialise and set struct_size = sizeof(lp_solve_opts). */
typedef struct {
  int32_t struct_size;
  int32_t p0;              /* local steps of the first round, >= 1 */
  double target;           /* > 0: the run ends once the estimated distance of the p = 1
                              iterates to their limit is at most target / 2 */
  int32_t max_rounds;      /* >= 1 */
  int32_t z0_orthonormal;  /* as in lp_run_opts */
  int32_t* p_used;         /* host [max_rounds] or NULL: p of every round run */
  double* change_out;      /* host [max_rounds] or NULL: c_r of every round run */
  uint64_t seed;           /* with Y0 == NULL: seed of the Gaussian start, as in
                              lp_run_opts (a struct_size that stops before this field
                              means seed 0) */
} lp_solve_opts;

typedef struct {
  int32_t rounds, local_iters, breakdowns, near_singular;
  int32_t p_final;         /* p of the last round run */
  double change;           /* last c_r */
  double estimate;         /* last E */
  double ms_total;         /* duration of the rounds on the stream (HIP events) */
} lp_solve_stats;

/* LocalPower without a fixed schedule or a reference subspace: rounds start at
 * p = p0 local steps and p decays on the data's own signal (the paper's advice to
 * communicate rarely early and often late, Sections 3 and 5, turned into a rule;
 * the rule itself is this library's).  After round r the change
 * c_r = sin theta_k(Z_r, Z_{r-1}) (Definition 1) is measured on the device and read
 * back (one synchronisation per round); q_r = c_r / c_{r-1} over rounds at the same
 * p; with Q the larger of the last two such ratios, E = c_r Q / (1 - Q) estimates
 * the distance to the limit of the current p (the tail of a geometric series).
 * The iterates have settled when c_r == 0 or Q < 1 and E <= target / 2.  Settled at
 * p = 1: the run ends with LP_OK.  Settled at p > 1, or q_r > 0.5 (a stall): p
 * halves (the limit of a fixed p > 1 sits at an error floor, Corollary 1; p = 1
 * has none).  After max_rounds rounds: LP_ENOTCONV, with Z_out (and ritz_out) from
 * the last iterate and stats filled.  The serving layer applies the same rule to
 * every job.  k, Y0, Z_out, ritz_out and stats as in lp_run (k is the iteration
 * rank).  Synchronises the stream before returning. */
lp_status lp_solve(lp_problem* P, int32_t k, lp_agg mode, const double* Y0, double* Z_out,
                   double* ritz_out, const lp_solve_opts* opts, lp_solve_stats* stats);

/* ---------------------------------------------------------------------------
 * Local-Gram form of the local multiply.  Eq. (power_yi) costs O(d^2 k) per local
 * iteration with M_i formed and O(s_i d k) without it.  lp_gram_enable computes M_i' = A_i^T A_i
 * (d x d, FP32 accumulation of exact products, one launch on the FP32 matrix cores over
 * all partitions, on the problem's stream) into a caller-owned device buffer of
 * lp_gram_bytes bytes (which also holds the scratch of lp_eta); from then on
 * every local multiply of the problem (lp_run, lp_solve, lp_local_multiply, the
 * Ritz pass) computes Y_i = M_i' Z_i on the FP32 matrix cores, reading m d^2
 * FP32 values instead of n d values of A.  It pays when m d is well below n (the
 * HBM bytes per local multiply fall by n b / (4 m d) for b-byte A) and the run is
 * long enough to amortise the 2 n d^2 flops of the Gram products.  The products
 * round in FP32 (A^T A squares the condition of A; the top eigenvectors, not the
 * small ones, are what the method needs).
 *   requirements: FP32 or BF16 A, d % 4 == 0, m d <= n; buffer 256-byte aligned,
 *   BORROWED until lp_gram_disable or lp_destroy, holding M_i' and a small work list.
 *   Split rounds do not apply to this form; lp_autotune tunes the A form only.
 * lp_gram_disable returns the problem to the A form (the buffer may then be freed).
 * Both synchronise the problem's stream and drop its captured rounds. */
lp_status lp_gram_bytes(const lp_problem* P, size_t* bytes);
lp_status lp_gram_enable(lp_problem* P, void* buffer, size_t bytes);
lp_status lp_gram_disable(lp_problem* P);

/* eta = max_i ||M_i - M||_2 / ||M||_2 (Definition 2: how far the local matrices
 * M_i = A_i^T A_i / s_i are from M = A^T A / n; the analysis' error floor grows with
 * it).  Needs the local-Gram form (its FP32 M_i'); M is summed in FP64 and each
 * spectral norm is estimated by `iters` steps of power iteration from four fixed
 * pseudo-random start vectors (an estimate from below that converges at the rate
 * (lambda_2 / lambda_1)^2 per step).  eta_out: host double; per_part_out: host [m]
 * ||M_i - M||_2 / ||M||_2, or NULL.  Its scratch (about 8 d^2 + 64 (m + 1) d bytes) is
 * part of the buffer given to lp_gram_enable; allocates nothing; synchronises the
 * problem's stream. */
lp_status lp_eta(lp_problem* P, int32_t iters, double* eta_out, double* per_part_out);

/* One local power iteration on every partition with a shared Z (the worker step
 * of DPI, Eq. (power_yi), without the 1/s_i scale):
 *   Z     : device d x k FP64 (rounded to the working precision of A's dtype);
 *   Y_out : device m x d x k FP64, Y_out[i] = A_i^T (A_i Z).
 * Enqueued on the problem's stream; asynchronous. */
lp_status lp_local_multiply(lp_problem* P, int32_t k, const double* Z, double* Y_out);

/* One two-pass local multiply (as lp_local_multiply, without the reduction) with a
 * start and end stamp of every workgroup (the GPU's constant-rate wall clock), for
 * measuring how evenly uneven partitions spread over the GPU.  wg_out: host
 * [max_wg x 4] FP64 rows (pass 1 or 2, work-item index, start us, end us, times
 * relative to the earliest start); *n_wg receives the number of workgroups (also
 * when max_wg is too small, which returns LP_EINVAL; wg_out may then be NULL).  Only for problems whose
 * local multiply at rank k is the two-pass kernel, at the default work-item size.
 * Z: device d x k FP64.  Synchronous. */
lp_status lp_profile_local_multiply(lp_problem* P, int32_t k, const double* Z, double* wg_out,
                                    int32_t max_wg, int32_t* n_wg);

/* Batched orth: Q_b = orth(Y_b) for b < batch, each d x k FP64 (CholeskyQR2).
 *   Y, Q : device, batch * d * k FP64 (may alias);  flags: device int32[batch]
 *   or NULL, set to 1 where a Cholesky broke down.  Uses the problem's workspace and
 *   stream; requires d == the problem's d, k <= k_max, batch <= max(m, 1). */
lp_status lp_orth(lp_problem* P, int32_t k, int32_t batch, const double* Y, double* Q,
                  int32_t* flags);

/* lp_orth for callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same batched CholeskyQR2,
 * Q_b = orth(Y_b) for b < batch, each d x k FP64 (device; Q may alias Y), flags as
 * in lp_orth, enqueued on `stream`, with no problem and no allocation.  Its
 * scratch is a 16 MiB array in the library's static device memory, one per GPU,
 * held from the first call on that GPU until the process ends:
 * 8 (batch (d k + 2 ceil(d / 64) k^2 + 2 k^2)) bytes, each of the four parts
 * rounded up to 256, must fit (for example one 4096 x 64 matrix, or 64 matrices of
 * 1024 x 16); larger batches get LP_EINVAL.  All calls on one GPU share that
 * scratch: calls that overlap in time on one GPU (different streams or threads)
 * race and must be serialised by the caller.  1 <= k <= min(d, 64), batch >= 1.
 * Asynchronous. */
lp_status lp_orth_noalloc(int32_t k, int32_t batch, int64_t d, const double* Y, double* Q,
                          int32_t* flags, void* stream);

/* Alignment of batch iterates Zi (device, batch x d x k FP64) against Zb (device
 * d x k FP64):
 *   LP_AGG_SIGN: out is device int8[batch*k], sgn(<Zi[:,j], Zb[:,j]>) with sgn(0)=+1;
 *   LP_AGG_OPT : out is device FP64 [batch*k*k], O_i = W1 W2^T for the SVD
 *                W1 S W2^T = Zi^T Zb, computed as the orthogonal polar factor of
 *                Zi^T Zb by Newton-Schulz iteration in FP64 (the same matrix when
 *                Zi^T Zb is nonsingular).
 * Same workspace/stream rules as lp_orth. */
lp_status lp_align(lp_problem* P, int32_t k, int32_t batch, lp_agg mode, const double* Zi,
                   const double* Zb, void* out);

/* Measured HBM read bandwidth: reads `bytes` (a multiple of 16, >= 16) of the device
 * buffer `buf` once per launch, `iters` launches on `stream`, each bracketed by HIP
 * events; writes the best launch's GB/s to *gbs_out.  Synchronous. */
lp_status lp_bandwidth_probe(const void* buf, size_t bytes, int32_t iters, double* gbs_out,
                             void* stream);

/* Measured HBM copy bandwidth: copies `bytes` (a multiple of 16) from device `src` to
 * device `dst` (non-overlapping, 16-byte aligned) once per launch, `iters` launches on
 * `stream`; writes the best launch's GB/s, counting read plus written bytes (2 * bytes),
 * to *gbs_out.  Synchronous.  Also the known-traffic kernel for calibrating counters. */
lp_status lp_copy_probe(void* dst, const void* src, size_t bytes, int32_t iters, double* gbs_out,
                        void* stream);

/* Exact-truth test matrix (not part of the paper: a synthetic input whose top-k
 * subspace is known without an eigendecomposition, used by the serving layer to
 * generate jobs on the device).  A = W diag(sigma) V^T with
 *   W (n x d): n / d Sylvester-Hadamard blocks (entries +-1, W^T W = n I), rows
 *     permuted and sign-flipped, columns sign-flipped per block;
 *   V: a permutation matrix (a keyed permutation of the d columns);
 *   sigma_j = 1/(j+1) for j < k, sigma_{k-1}/gap at j = k, then times decay per
 *     index, each rounded to FP32 and then to BF16;
 * so A^T A = n V diag(sigma^2) V^T exactly, every entry +-sigma_j is exact in FP32
 * and BF16, and the top-k right singular vectors are V's columns for j < k.  All
 * random choices come from Philox4x32-10 under `seed` (Salmon et al., SC 2011).
 *   A     : device n x d, FP32 or BF16 (dtype), leading dimension lda (lda >= d,
 *           lda % 4 == 0, A aligned to 4 elements), or NULL;
 *   U_out : device d x k FP64 (U[c][j] = 1 where column c holds sigma_j), or NULL;
 *   shapes: d a power of two in [16, 8192], n a positive multiple of d, 1 <= k <= d,
 *           gap >= 1, 0 < decay <= 1.
 * Enqueued on `stream`; asynchronous.  LP_EINVAL for other shapes. */
lp_status lp_generate(void* A, lp_dtype dtype, int64_t n, int64_t d, int64_t lda, int32_t k,
                      double gap, double decay, uint64_t seed, double* U_out, void* stream);

/* sin theta_k(Z, U) = ||U - Z (Z^T U)||_2 (Definition 1), for device d x k FP64
 * matrices with orthonormal columns.  The result goes through one of 64 device
 * cells held by the library (taken under a lock for the duration of the call, so
 * calls from different threads on different streams do not share one); the call
 * synchronises `stream` and writes the result to *out_host.  LP_EBUSY when 64
 * calls are already in flight. */
lp_status lp_sin_theta(const double* Z, const double* U, int64_t d, int32_t k, double* out_host,
                       void* stream);

/* sin theta_k(Z, U) = ||(I - Z Z^T) U||_2 for a device d x r FP64 iterate Z with
 * orthonormal columns and a device d x k FP64 reference U, 1 <= k <= r <= min(d, 64)
 * (Definition 1 with the iteration rank above the target rank, as in the appendix on
 * the eigengap).  Same scratch, synchronisation and result as lp_sin_theta, which is
 * the case r = k. */
lp_status lp_sin_theta_r(const double* Z, int32_t r, const double* U, int32_t k, int64_t d,
                         double* out_host, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: many LocalPower jobs on one GPU.  (Runtime around the method, not
 * part of the paper.)  A server admits submitted jobs in order while their
 * device-memory footprint fits its budget and it has a free slot, runs one
 * communication round at a time for every admitted job, each job on its own
 * stream so that rounds of different jobs overlap on the GPU, admits waiting
 * jobs as soon as others finish (continuous batching), and ends every job by
 * its own stop rule.  A worker thread of the server does all GPU work.
 *
 * Per-job schedule and stop rule.  The job starts from Z_0 = orth(Y0) with
 * p = p0 local steps per round.  After round r the change
 * c_r = sin theta_k(Z_r, Z_{r-1}) (Definition 1) is measured, and the ratio
 * q_r = c_r / c_{r-1} over rounds run with the same p:
 *   - with Q the larger of the last two such ratios, E = c_r Q / (1 - Q) (the
 *     tail of a geometric series of changes, an estimate of the distance to
 *     the limit of the current p); the iterates have settled when Q < 1 and
 *     E <= target / 2 (a margin for the transient after p changes), or when
 *     c_r == 0;
 *   - settled at p = 1, the job ends with LP_OK;
 *   - settled at p > 1, or q_r > 0.5 (a stall), halves p: the limit of a fixed
 *     p > 1 sits at an error floor set by the heterogeneity of the partitions,
 *     and p = 1 has none (the decaying p of Sections 3 and 5);
 *   - after max_rounds rounds the job ends with LP_ENOTCONV.
 * Z_out then holds the last iterate.  Results of a job do not depend on what
 * else the server runs (bitwise): every job has its own workspace and stream.
 * --------------------------------------------------------------------------- */
typedef struct lp_server lp_server; /* opaque */

typedef struct {
  int32_t struct_size;     /* sizeof(lp_job); a size that stops before `stream` means
                              stream NULL and no generation (the fields below it) */
  const void* A;           /* device n x d row-major (leading dimension lda, 16-byte
                              aligned rows), BORROWED until the job's result is polled;
                              NULL: generated at admission (see gen_seed) */
  lp_dtype dtype;
  int64_t n, d, lda;
  const int64_t* offsets;  /* host, m + 1 entries as for lp_create; COPIED at submit */
  int32_t m;
  int32_t k;               /* 1 <= k <= min(d, 64), every partition has >= k rows */
  int32_t p0;              /* local steps of the first round, >= 1 */
  lp_agg mode;
  double target;           /* > 0 */
  int32_t max_rounds;      /* >= 1 */
  const double* Y0;        /* host d x k FP64 start, COPIED at submit; orthonormalised;
                              NULL: drawn on the device from gen_seed as lp_run draws it
                              from lp_run_opts.seed */
  double* Z_out;           /* device d x k FP64, caller-owned, written when the job ends */
  void* stream;            /* hipStream_t on which the caller writes A and uses Z_out
                              (NULL: the legacy default stream).  lp_server_submit records
                              an event on it; the job waits for that event before its
                              first GPU work, so work queued there before the submit (A
                              being written, Z_out's memory still being read) comes first.
                              Z_out is complete when the job's result is polled. */
  uint64_t gen_seed;       /* seed of the generated A and/or start */
  double gen_gap, gen_decay; /* A == NULL: the job's A is lp_generate(dtype, n, d, lda = d,
                              k, gen_gap, gen_decay, gen_seed) written at admission into
                              the job's own device memory (part of its footprint), so
                              only admitted jobs hold a matrix; needs the shapes
                              lp_generate takes */
  int32_t single_bf16;     /* BF16 A: 0 (default) the job's local multiplies use
                              FP32-class operands (split_operands of lp_tuning), since
                              its stop rule aims at a sin theta target; 1 one BF16
                              rounding of Z and t (faster; a floor near 1e-3) */
} lp_job;

typedef struct {
  uint64_t id;
  lp_status status;        /* LP_OK, LP_ENOTCONV, LP_EBREAKDOWN or LP_EDEVICE */
  int32_t rounds;          /* communication rounds run */
  int32_t local_iters;     /* local steps run (sum of p over the rounds) */
  int32_t p_final;         /* p of the last round */
  double change;           /* last c_r */
  double estimate;         /* last E (c_r while fewer than two ratios exist or Q >= 1) */
  double ms_queued;        /* submission -> admission, host clock */
  double ms_total;         /* submission -> result published */
} lp_job_result;

/* Device bytes the server allocates for `job` (its lp_workspace_size plus the
 * start, previous-iterate and change buffers, plus n d b bytes for A when the
 * job generates it); otherwise A and Z_out are the caller's. */
lp_status lp_server_footprint(const lp_job* job, size_t* bytes);

/* Create a server on the current HIP device with a device-memory budget and at
 * most max_active (1..64) jobs admitted at once; allocates the budget as one
 * device arena (LP_ENOMEM when it does not fit in free device memory) and starts
 * its worker thread.  Jobs are admitted in submission order when a contiguous
 * range of their footprint is free in the arena. */
lp_status lp_server_create(lp_server** out, size_t hbm_budget_bytes, int32_t max_active);

/* Queue a job (non-blocking).  LP_EINVAL for an invalid job, LP_ENOMEM when its
 * footprint alone exceeds the budget (it could never be admitted). */
lp_status lp_server_submit(lp_server* S, const lp_job* job, uint64_t* job_id);

/* Move up to `max` finished results into out[0 .. *n_done) (non-blocking). */
lp_status lp_server_poll(lp_server* S, lp_job_result* out, int32_t max, int32_t* n_done);

/* Block until at least min_done results are waiting to be polled, or
 * timeout_s seconds pass (then LP_EBUSY). */
lp_status lp_server_wait(lp_server* S, int32_t min_done, double timeout_s);

/* Finish every admitted job, drop the queued ones, stop the worker and free
 * the server.  Unpolled results are discarded. */
lp_status lp_server_destroy(lp_server* S);

#ifdef __cplusplus
}
#endif

#endif /* LP_H */
