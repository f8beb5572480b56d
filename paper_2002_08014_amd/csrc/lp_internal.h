// Internal declarations of the LocalPower HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/lp.h"
#include "stop_rule.h"

namespace lp {

constexpr int kMaxK = 64;        // largest iteration rank supported by the kernels
constexpr int kGramRows = 64;    // rows of a d x k matrix per Gram partial
constexpr int kBlock = 256;      // threads per workgroup for the small kernels

// A contiguous row range of one partition processed by one workgroup of the
// local-multiply kernel; `slot` indexes its FP32/FP64 partial d x k sum.
struct WorkItem {
  int32_t part;
  int32_t slot;
  int64_t row0;
  int64_t rows;
};

// Which local-multiply implementation a problem uses.
enum class LocalPath : int { TwoPass = 0, Mfma32 = 1, MfmaBf16 = 2 };

struct Layout {
  // byte offsets into the workspace
  size_t Zi, Zw, Yi, tmp, Z, Zw_shared, Y, Uref, part, tbuf, gram, gram2, rinv, omat, sgn, flags,
      items, slot_off, hist, ctr, scal, rho, rho_part, rho_ctr, sinw, stamps, total;
};

constexpr int kHistCap = 1024;  // rounds of sin-theta history buffered on the device

// Sizes that decide the workspace layout.
struct Plan {
  lp_dtype dtype;
  int64_t n, d;
  int32_t m, k_max;
  int64_t lda;               // leading dimension of A (set by lp_create; 0 before)
  int64_t chunk_rows;        // rows per work item (last one of a partition is shorter)
  std::vector<WorkItem> items;
  int32_t n_gram_chunks;     // ceil(d / kGramRows)
  size_t acc_bytes;          // 8 for FP64 A, 4 otherwise
  size_t zw_bytes;           // bytes per element of the working copy of Z
  LocalPath path;
  int32_t variant;           // fused kernel variant (see k_mfma.hip)
  bool nt_loads;             // nontemporal loads of A in the fused kernel
  bool split_operands;       // BF16 A: hi + lo BF16 operand pairs (FP32-class results)
  bool valu;                 // k <= 8: the fused vector-ALU kernel (off: two-pass kernel)
  bool split_products = false;   // two-pass kernel on BF16 matrix cores (split operands)
  bool two_pass_auto = true;      // no kernel named: the two-pass form is chosen per launch
  int64_t min_chunk_rows;    // the default chunking the workspace was sized for
  int64_t stamp_cap;         // workgroups of one two-pass local multiply the stamp area holds
  unsigned long long* stamps = nullptr;   // set while a profiled launch is enqueued
  Layout L;
};

// Rebuild the work list for `chunk_rows` rows per item (>= plan.min_chunk_rows).
void build_items(Plan* P, const int64_t* offsets, int64_t chunk_rows);

bool make_plan(lp_dtype dtype, int64_t n, int64_t d, const int64_t* offsets, int32_t m,
               int32_t k_max, Plan* plan, std::string* err);

struct GraphKey {
  int32_t k, p, mode, hist, slot;  // slot >= 0: timed instance with its own event pairs
  int32_t first_only;              // timed instance brackets only the round's first step
  int32_t split;                   // partitions in two halves on two streams
  int32_t rho = 0;                 // the round appends its residual error (Definition 3)
  bool operator<(const GraphKey& o) const {
    if (rho != o.rho) return rho < o.rho;
    if (k != o.k) return k < o.k;
    if (p != o.p) return p < o.p;
    if (mode != o.mode) return mode < o.mode;
    if (hist != o.hist) return hist < o.hist;
    if (slot != o.slot) return slot < o.slot;
    if (first_only != o.first_only) return first_only < o.first_only;
    return split < o.split;
  }
};

// One half of the partitions for split rounds: partitions [b0, b0 + nb) and
// their work items [it0, it0 + nit) (items are in partition order).
struct Half {
  int32_t b0, nb, it0, nit;
};

constexpr int kTimedSlots = 8;      // timed graph instances replayed before one harvest
constexpr int kPairsPerSlot = 32;   // local-multiply event pairs per timed instance

}  // namespace lp

struct lp_problem {
  int device;
  hipStream_t user_stream;
  hipStream_t stream;          // own non-blocking stream (capturable)
  hipEvent_t ev_join_in, ev_join_out, ev_t0, ev_t1;
  const void* A;
  lp_dtype dtype;
  int64_t n, d, lda;
  int32_t m, k_max, base;
  std::vector<int64_t> offsets;
  char* ws;
  size_t ws_bytes;
  lp::Plan plan;
  std::map<lp::GraphKey, hipGraphExec_t> graphs;
  // event pairs bracketing local-multiply launches when timing is requested
  std::vector<hipEvent_t> ev_pool;
  int ev_used = 0;
  bool timing = false;
  bool timing_first_only = false;  // time only the first local step of every round
  bool timing_now = false;         // the next local-multiply launch is bracketed
  int timing_slot = -1;   // >= 0 while capturing a timed graph instance
  int timing_pair = 0;
  bool timed_graphs_ok = true;
  double ms_local = 0.0;
  int local_launches = 0;
  // split rounds: half[0] holds the base partition and runs on `stream`, half[1]
  // on stream2; events order the two streams (fork/join, the chain of local
  // multiplies, the base iterate for the alignment)
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join2 = nullptr, ev_base = nullptr;
  hipEvent_t ev_k1[2] = {nullptr, nullptr};
  bool can_split = false;   // m >= 2
  bool split_now = false;   // the rounds being enqueued are split
  bool rho_now = false;     // the rounds being enqueued append their residual error
  lp::Half half[2];
  double* change_host = nullptr;   // pinned cell for lp_solve's per-round change
  // local-Gram form (lp_gram_enable): M_i = A_i^T A_i in a caller-owned buffer
  bool gram_on = false;
  float* gram_M = nullptr;
  lp::WorkItem* gram_items = nullptr;
  int32_t* gram_slot_off = nullptr;   // [0..m]: i (one slot each); [m+1..2m+1]: 2 i
  bool gram_split2 = false;           // tbuf holds two partial Y_i per partition
  char* gram_eta = nullptr;           // eta scratch inside the same buffer
};

namespace lp {

// Step-wise driving of a problem (the serving layer): begin sets Z = orth(Y0)
// (or copies Y0 when it is already orthonormal) and clears the flags; round
// enqueues one communication round with p local steps (graph-replayed); the
// current iterate is drive_z; drive_breakdowns synchronises and counts the
// breakdown flags.  Everything runs on drive_stream(P).
lp_status drive_begin(lp_problem* P, int k, const double* Y0, bool orthonormal);
lp_status drive_round(lp_problem* P, int k, int p, lp_agg mode);
const double* drive_z(lp_problem* P);
// out (device) = sin theta_k(drive_z, Zprev), enqueued on drive_stream(P) with the
// problem's own scratch (the change of a round).
hipError_t drive_change(lp_problem* P, int k, const double* Zprev, double* out);
hipStream_t drive_stream(lp_problem* P);
lp_status drive_breakdowns(lp_problem* P, int* breakdowns);
// BF16 operand pairs in the fused BF16 kernel (lp_tuning.split_operands) for a
// problem with no rounds yet, without lp_set_tuning's re-tuning; the work list
// is uploaded again (synchronising) only when the rank moves to the two-pass kernels.
lp_status drive_split_operands(lp_problem* P, bool split);
// Ranks up to 8 where the zero-padded fused matrix-core kernel measured faster than
// the vector-ALU kernel: BF16 A (0.88 of the HBM peak at k = 4 and 8, 1048576 x 2048,
// against about 0.5) and FP32 A at k >= 5 (180 against 204 us at k = 8, 262144 x
// 1024; k = 4 stays on the vector-ALU kernel, 166 us).  For a served job, which is
// not autotuned; call before its first round.
void drive_prefer_matrix_cores(lp_problem* P, int k);
// Record msg as the thread's last error (lp_last_error) and return s.
lp_status report(lp_status s, const std::string& msg);

// ---------------------------------------------------------------------------
// kernel launchers (all enqueue on `s`, return the launch status)
// ---------------------------------------------------------------------------

// Local multiply Y_i = A_i^T (A_i Z_i) for nitems work items starting at items_dev
// (all of them: plan.items.size()), partial sums per item.
//   Zw: working copy of the per-partition inputs, z_stride elements between
//   partitions (0 = one shared Z).  Writes part[slot] (d x k, acc type).
hipError_t launch_local_multiply(const Plan& P, const void* A, int64_t lda, int k,
                                 const void* Zw, int64_t z_stride, void* tbuf, void* part,
                                 const WorkItem* items_dev, int nitems,
                                 hipStream_t s);

// Fused single-pass matrix-core kernel: FP32 A, k = 16, d in {256, 512, 768, 1024}.
bool mfma32_eligible(lp_dtype dtype, int64_t d, int64_t lda, int k);
hipError_t launch_local_multiply_mfma32(const Plan& P, const void* A, int64_t lda, int k,
                                        const void* Zw, int64_t z_stride, void* part,
                                        const WorkItem* items, int nitems,
                                        hipStream_t s);

// Fused single-pass matrix-core kernel: BF16 A, k in {16, 32}, d in {512, 1024,
// 1536, 2048}, rows 16-byte aligned (BF16 operands, FP32 accumulation).
bool mfma16_eligible(lp_dtype dtype, int64_t d, int64_t lda, int k, const void* A, bool split);
hipError_t launch_local_multiply_mfma16(const Plan& P, const void* A, int64_t lda, int k,
                                        const void* Zw, int64_t z_stride, void* part,
                                        const WorkItem* items, int nitems,
                                        hipStream_t s);

// Fused single-pass vector-ALU kernel for small ranks: FP32 or BF16 A, k <= 8,
// d a power of two in [256, 4096], rows aligned to 16 bytes.
bool valu_eligible(lp_dtype dtype, int64_t d, int64_t lda, int k, const void* A);
hipError_t launch_local_multiply_valu(const Plan& P, const void* A, int64_t lda, int k,
                                      const void* Zw, int64_t z_stride, void* part,
                                      const WorkItem* items, int nitems, hipStream_t s);

// Two-pass form on FP32 matrix cores (t = A Z, then A^T t): FP32 or BF16 A,
// d % 4 == 0, any k <= 64.
bool gemm_eligible(lp_dtype dtype, int64_t d, int64_t lda, const void* A);
// Definition 2 diagnostics on the local-Gram form's matrices: scratch bytes, and
// est_host[(m + 1) x eta_start_vectors()] = power-iteration estimates of
// ||M_i'/s_i - M||_2 (rows 0..m-1) and ||M||_2 (row m) after `iters` steps.
size_t eta_scratch_bytes(int64_t d, int m);
hipError_t launch_eta(int64_t d, int m, int64_t n, const float* Mi, const double* inv_s_host,
                      int iters, char* scratch, double* est_host, hipStream_t s);
int eta_start_vectors();
// Local-Gram form: Y_i = M_i Z_i for the m stacked FP32 d x d matrices M_i = A_i^T A_i
// (row-major, M_i at M + i d d); items[i] = {i, i, i d, d}; writes Y_i (FP32) to
// tbuf + i d k, or with split == 2 (k <= 16 only) the two halves of the contraction
// to tbuf + (2 i + h) d k.
hipError_t launch_gram_multiply(const Plan& P, const float* M, int k, const void* Zw,
                                int64_t z_stride, void* tbuf, const WorkItem* items, int m,
                                int split, hipStream_t s);
// Local-Gram form setup: M_i = A_i^T A_i (FP32, d x d row-major at M + i d d) for the
// m partitions parts[i] = {i, i, first row, rows} (FP32 or BF16 A, d % 4 == 0).
hipError_t launch_gram_products(const Plan& P, const void* A, int64_t lda, const WorkItem* parts,
                                int m, float* M, hipStream_t s);
hipError_t launch_local_multiply_gemm(const Plan& P, const void* A, int64_t lda, int k,
                                      const void* Zw, int64_t z_stride, void* tbuf, void* part,
                                      const WorkItem* items, int nitems,
                                      hipStream_t s);

// The same two passes on BF16 matrix cores, every FP32 operand split exactly into three
// BF16 pieces and the six leading partial products kept (FP32-class results; the
// shapes and buffers of launch_local_multiply_gemm).
hipError_t launch_local_multiply_gemm3(const Plan& P, const void* A, int64_t lda, int k,
                                       const void* Zw, int64_t z_stride, void* tbuf, void* part,
                                       const WorkItem* items, int nitems, hipStream_t s);

// Rows per workgroup of pass 1 and columns per workgroup of pass 2 of the matrix-core
// two-pass local multiply the plan selects (the workgroup stamps follow this order).
void two_pass_geometry(const Plan& P, int64_t* rows_per_wg1, int64_t* cols_per_wg2);

hipError_t launch_local_multiply_twopass(const Plan& P, const void* A, int64_t lda, int k,
                                         const void* Zw, int64_t z_stride, void* tbuf, void* part,
                                         const WorkItem* items, int nitems,
                                         hipStream_t s);

// Y_i = sum of the partials of partition i in item order (FP64); slot_off is
// the device int32[m+1] prefix of partial slots per partition.
hipError_t launch_reduce_partials(const Plan& P, int k, const void* part, const int32_t* slot_off,
                                  double* Yi, hipStream_t s);

// Convert FP64 d x k matrices to the working copy (FP32 or FP64), batch of them,
// optionally scaling column j by sign[b*k+j] (int8, may be NULL).
hipError_t launch_to_working(const Plan& P, int batch, int64_t d, int k, const double* X,
                             void* Zw, hipStream_t s);

// G_b = X_b^T W_b (k x k) partials over row chunks of kGramRows rows:
//   X: batch x d x k; W: batch x d x k, or shared (w_stride = 0).
hipError_t launch_cross_gram(int batch, int64_t d, int k, const double* X, int64_t x_stride,
                             const double* W, int64_t w_stride, double* gram_part,
                             hipStream_t s);


// Q_b = X_b S_b (d x k times k x k); S upper triangular if `upper`.
//   S stride k*k between batches (s_stride = 0: shared).  Optionally also writes
//   the working copy of Q_b (zw != NULL, zw_bytes per element).
hipError_t launch_right_mult(int batch, int64_t d, int k, const double* X, const double* S,
                             int64_t s_stride, bool upper, double* Q, void* zw, size_t zw_bytes,
                             hipStream_t s);

// Sign decisions from the cross-Gram diagonals: sgn[b*k+j] = sign(sum of partials).
hipError_t launch_sign_from_gram(int batch, int nchunks, int k, const double* gram_part,
                                 int8_t* sgn, hipStream_t s);


// Procrustes factor O_b = W1 W2^T of C_b = sum of cross-gram partials (the orthogonal
// polar factor of C_b, by Newton-Schulz iteration in FP64); *flags (if not null)
// counts the C_b too close to singular for the iteration to converge.
hipError_t launch_procrustes(int batch, int nchunks, int k, const double* gram_part,
                             double* O, int32_t* flags, hipStream_t s);

// Y = scale * sum_i Yi (fixed order), d x k.
hipError_t launch_aggregate(int m, int64_t d, int k, const double* Yi, double scale, double* Y,
                            hipStream_t s);

// Symmetric k x k eigen-decomposition of H = sum of partials (cyclic Jacobi),
// eigenvalues descending into lam, eigenvectors into V (k x k, columns).
hipError_t launch_sym_eig(int nchunks, int k, const double* gram_part, double* lam, double* V,
                          hipStream_t s);

// sin theta_k(Z, U) of a d x r iterate Z against a d x k reference U (r >= k) in
// one workgroup (no scratch): writes out[0] (device) and, if hist != NULL,
// hist[*ctr] then increments *ctr.
hipError_t launch_sin_theta(int64_t d, int r, int k, const double* Z, const double* U,
                            double* out, double* hist, int32_t* ctr, hipStream_t s);
// The same distance with the O(d r k) work spread over ceil(d / 64) workgroups
// (five launches; the per-round form): scratch holds sin_theta_scratch_doubles
// FP64 values (the chunk partials of Z^T U and of the residual's Gram, and
// their sums).
size_t sin_theta_scratch_doubles(int64_t d, int r, int k);
hipError_t launch_sin_theta_chunked(int64_t d, int r, int k, const double* Z, const double* U,
                                    double* scratch, double* out, double* hist, int32_t* ctr,
                                    hipStream_t s);

hipError_t launch_fill_i32(int32_t* p, int count, int32_t v, hipStream_t s);

// The library's own random inputs (k_gen.hip): count standard normals of the
// start stream of `seed` (element e = i k + j of a d x k start); the exact-truth
// matrix (FP32 or BF16, n x d with leading dimension lda; truth_shape_ok) and
// its top-k right singular vectors U (d x k FP64).
hipError_t launch_gaussian(int64_t count, uint64_t seed, double* Y, hipStream_t s);
bool truth_shape_ok(int64_t n, int64_t d);
hipError_t launch_truth_matrix(void* A, lp_dtype dtype, int64_t n, int64_t d, int64_t lda, int k,
                               double gap, double decay, uint64_t seed, hipStream_t s);
hipError_t launch_truth_basis(int64_t d, int k, uint64_t seed, double* U, hipStream_t s);
// rho (Definition 3) of the m local iterates Zi (m x d x k, FP64) against the
// first partition's, appended to hist[*ctr]; part: m doubles of scratch.
hipError_t launch_rho(int m, int64_t d, int k, bool opt, const double* Zi, double* part,
                      double* hist, int32_t* ctr, hipStream_t s);

// Read `bytes` (a multiple of 16) of `buf` once with 128-bit loads.
hipError_t launch_stream_read(const void* buf, size_t bytes, hipStream_t s);
// Copy `bytes` (a multiple of 16) from src to dst with the same streaming pattern.
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// Address (on the current device) of the library's kSinSlots device result
// cells used by lp_sin_theta; a call owns one cell from take to give back.
constexpr int kSinSlots = 64;
hipError_t sin_slot_address(double** p);

// Y_i = sum of partials (item order, FP64) and the Gram partials of Y_i's row
// chunks (kGramRows rows) into gram, for the partitions [b0, b0 + nb); grid over
// (row chunks, partitions).
hipError_t launch_reduce_gram(const Plan& P, int k, const void* part, const int32_t* slot_off,
                              double* Yi, double* gram, int b0, int nb, hipStream_t s);

// Y = scale * sum_i Yi and the Gram partials of Y's row chunks into gram.
hipError_t launch_aggregate_gram(int m, int64_t d, int k, const double* Yi, double scale, double* Y,
                                 double* gram, hipStream_t s);




// One CholeskyQR pass: sum the nch_in Gram partials, factor them and invert the
// factor (k <= 16: in every 64-row-chunk workgroup, one launch; larger k: once
// per matrix into rfac = batch x 2 k^2 doubles, then the row chunks), multiply
// the rows by R^{-1} on FP64 matrix cores, optionally write the working copy
// and the Gram partials of Q (chol_solve_chunks(d, k) of them).
hipError_t launch_chol_solve(int batch, int64_t d, int k, int nch_in, const double* X,
                             const double* gram_in, double* rfac, double* Q, void* zw,
                             size_t zw_bytes, double* gram_out, int32_t* flags, hipStream_t s);
int chol_solve_chunks(int64_t d, int k);

// Sign-fixing in two launches: column dots <Zi[:,j], Zb[:,j]> partials per row
// chunk, then sum, sign (sgn(0) = +1), record sgn and flip Zi and its working copy.
hipError_t launch_diag_dot(int batch, int64_t d, int k, const double* Zi, const double* Zb,
                           double* part, hipStream_t s);
hipError_t launch_sign_apply(int batch, int64_t d, int k, const double* part, double* Zi, void* zw,
                             size_t zw_bytes, int8_t* sgn, hipStream_t s);

// The two CholeskyQR passes on explicit buffers: gram holds the Gram partials of
// the batch of Y's (ceil(d / 64) k x k partials per matrix); gram2 (the same
// size), tmp (batch d k) and rfac (batch 2 k^2) are scratch; Q may alias Y.
hipError_t cholqr2_passes(int batch, int64_t d, int k, const double* Y, const double* gram,
                          double* gram2, double* tmp, double* rfac, double* Q, void* zw,
                          size_t zw_bytes, int32_t* flags, hipStream_t s);

// CholeskyQR2 when the Gram partials of Y are already in the plan's gram buffer.
// b0: index of the first matrix of the batch among the plan's matrices (its
// partials and scratch are at that offset, so disjoint batches may run
// concurrently on different streams); Y, Q, zw and flags point at the batch.
hipError_t cholqr2_from_gram(const Plan& P, char* ws, int batch, int64_t d, int k, const double* Y,
                             double* Q, void* zw, int32_t* flags, hipStream_t s, int b0 = 0);

// CholeskyQR2: Q_b = orth(Y_b) for a batch of d x k FP64 matrices, using
// gram/rinv scratch from the plan; also writes the working copy when zw != NULL.
hipError_t cholqr2(const Plan& P, char* ws, int batch, int64_t d, int k, const double* Y,
                   double* Q, void* zw, int32_t* flags, hipStream_t s);

}  // namespace lp
