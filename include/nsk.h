/*
 * nsk.h -- C ABI of the sketch-and-solve null-space library for AMD MI355X (gfx950).
 *
 * The library computes the trailing k right singular vectors of a tall-skinny m x N
 * matrix A (the null space problem, Problem 2.1 of Park & Nakatsukasa, "A Fast
 * Randomized Algorithm for Computing an Approximate Null Space") by Algorithm 1:
 * draw a random sketching matrix S (s x m, N < s <= m), form SA reading A once, take the
 * SVD of the small s x N matrix SA and return V(:, N-k+1:N).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are row-major.  A matrix operand is a list of column blocks (nsk_operand),
 *   so [A | b] of Section 4 is passed as two blocks without a concatenated copy.
 * - Device pointers are HIP device memory owned by the caller.  The library allocates no
 *   device memory in the calls below: scratch comes from the caller's workspace, sized by the
 *   matching *_workspace_bytes query.  Host pointers are marked "host".  The host-built
 *   records that nsk_trailing_rsv_batched and nsk_sketch_rows copy to the device go through
 *   a few library-owned pinned host buffers (allocated on first use, grown when a larger
 *   batch arrives, kept until the process ends); a call reuses such a buffer only after the
 *   copy that last used it has completed.
 * - `stream` is a hipStream_t passed as void*.  Device entry points only enqueue work on
 *   it and return (nsk_aaa and the autotuner excepted, as documented there): every random
 *   draw, the SRFT row sample included, is made on the device; outputs (including nsk_info)
 *   are valid after the stream has drained.
 * - Every entry point returns an nsk_status; no exceptions cross the ABI.  Argument
 *   errors are detected on the host before anything is enqueued.  NaN and Inf inputs are
 *   not checked: they propagate to the outputs.
 * - The realisation of S is a pure function of (kind, m, s, zeta, seed): S is regenerated
 *   from Philox4x32-10 counters on every call and never kept between calls.  Within a
 *   sparse-sign sketch the draws are expanded once into a per-call table in the workspace
 *   (20 bytes per row of A for zeta <= 8, 68 for zeta <= 32) that its column tiles share;
 *   the DCT-II kind does the same with the signs of D (m_p / 8 bytes) and two rotations
 *   per sampled row (32 bytes each).
 */
#ifndef NSK_H
#define NSK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nsk_status {
  NSK_OK = 0,
  NSK_EINVAL = 1,        /* an argument violates the constraints stated below            */
  NSK_EWORKSPACE = 2,    /* workspace (or TLS state) smaller than the size query returns */
  NSK_ENOCONV = 3,       /* Jacobi did not converge in max_sweeps; outputs still written  */
  NSK_EDEVICE = 4,       /* a HIP runtime call failed (launch or copy)                   */
  NSK_EUNSUPPORTED = 5   /* valid arguments, but this kind/dtype combination is not built */
} nsk_status;

/* Sketch kinds (Section 2 of the paper). */
typedef enum nsk_kind {
  NSK_SRHT = 0,          /* subsampled randomized Hadamard transform: the SRFT of Section 2
                            with the Walsh-Hadamard transform as trig transform,
                            S = sqrt(m_p/s) R (H/sqrt(m_p)) D on A zero-padded to
                            m_p = 2^ceil(log2 m) rows; entries +-1/sqrt(s)                  */
  NSK_SPARSE_SIGN = 1,   /* zeta distinct nonzeros +-1/sqrt(zeta) per column of S
                            (the CountSketch family mentioned in Section 2)                 */
  NSK_GAUSSIAN = 2,      /* S = G_hat/sqrt(s), G i.i.d. N(0,1) (Section 2) rounded to the
                            operand format of A (bf16 or e4m3) and applied on MFMA          */
  NSK_SRDCT = 3,         /* subsampled randomized DCT-II: the SRFT of Section 2 with the
                            orthonormal DCT-II C of length m_p = max(1024, 2^ceil(log2 m)) as
                            trig transform (the real transform of Section 4's experiments),
                            S = sqrt(m_p/s) R C D on A zero-padded to m_p rows, with the
                            NSK_SRHT kind's D and row sample R (rows drawn from [0, m_p))   */
  NSK_HRHT = 4           /* hashed randomized Hadamard transform (Section 2's H-RHT): the row
                            sample replaced by a 1-hashing matrix Phi, S = Phi (H/sqrt(m_p)) D
                            on A zero-padded to m_p = 2^ceil(log2 m) <= 2^21 rows; Phi is the
                            sparse-sign draw with zeta = 1 over the m_p transformed rows.  FP64
                            arithmetic only; the workspace holds the m_p x N transform;
                            s + m_p / 1024 <= 10240                                          */
} nsk_kind;

typedef enum nsk_dtype {
  NSK_F64 = 0, NSK_F32 = 1, NSK_BF16 = 2, NSK_F8E4M3 = 3
} nsk_dtype;

#define NSK_FLAG_RESIDUAL 1   /* nsk_trailing_rsv also writes |A V_k|_F to info->residual */

/* Method parameters. Zero fields take the documented defaults. */
typedef struct nsk_desc {
  int32_t kind;        /* nsk_kind                                                         */
  int32_t zeta;        /* NSK_SPARSE_SIGN: nonzeros per column of S, 1 <= zeta <= min(s,32);
                          0 selects 8                                                       */
  int64_t s;           /* sketch size; N < s <= m (Algorithm 1 requires s > n; s <= m)      */
  uint64_t seed;       /* Philox key of the realisation                                     */
  int32_t acc;         /* NSK_SRHT / NSK_SRDCT / NSK_SPARSE_SIGN arithmetic: NSK_F64 (default,
                          FP32 or FP64 loads with FP64 accumulation) or NSK_F32 (plain FP32) */
  int32_t max_sweeps;  /* Jacobi sweep cap, 0 selects 30                                     */
  int32_t row_groups;  /* number of row partitions of the sketch (partial sums); 0 = tuned */
  int32_t flags;       /* NSK_FLAG_*                                                         */
} nsk_desc;

/* One column block of a row-major matrix operand. */
typedef struct nsk_operand {
  const void* ptr;        /* device pointer to element (0,0) of the block                   */
  int32_t dtype;          /* nsk_dtype of the elements                                       */
  int32_t reserved;       /* must be 0                                                       */
  int64_t cols;           /* number of columns, >= 1                                         */
  int64_t ld;             /* row stride in elements, >= cols                                 */
  const int8_t* col_exp;  /* NSK_F8E4M3 only, nullable: device array of per-column binary
                             exponents e_c; the logical entry is stored * 2^e_c             */
} nsk_operand;

/* Diagnostics written by the device (pass a device pointer, or NULL). */
typedef struct nsk_info {
  int32_t sweeps;      /* Jacobi sweeps performed                                            */
  int32_t converged;   /* 1 if every column pair met |x_p.x_q| <= N u |x_p||x_q|            */
  double off;          /* largest relative column cosine seen in the last sweep              */
  double residual;     /* |A V_k|_F (FP64 accumulation) when NSK_FLAG_RESIDUAL was set       */
  double sigma_max;    /* largest singular value of SA                                       */
} nsk_info;

const char* nsk_status_str(int status);
int nsk_version(void);

/*
 * Workspace bytes for nsk_sketch / nsk_trailing_rsv / nsk_residual / nsk_tls_solve on an
 * m x N operand with sketch size d->s and k trailing vectors. Returns 0 on invalid input.
 */
size_t nsk_workspace_bytes(int64_t m, int64_t N, int64_t k, const nsk_desc* d);

/*
 * Line 2 of Algorithm 1: SA = S A.
 * blocks/nblocks (host array, 1..4 blocks): the m x N operand, N = sum of block columns.
 *   SRHT, DCT-II and sparse sign take NSK_F32 or NSK_F64 blocks; Gaussian takes NSK_BF16
 *   or NSK_F8E4M3 blocks (all blocks of one dtype).
 * SA (device): s x N row-major FP64 output with row stride ldsa >= N.
 * Errors: NSK_EINVAL if m < N, s <= N, s > m, a block has cols < 1 or ld < cols, nblocks
 *   outside 1..4, zeta outside 1..min(s,32); NSK_EUNSUPPORTED for other dtype/kind pairs
 *   and for s > 2048 or m > 2^31 with NSK_SRHT or NSK_SRDCT, NSK_HRHT with acc = NSK_F32, m > 2^21 or
 *   s + m_p/1024 > 10240, and NSK_SPARSE_SIGN when its (s + 1)-row accumulator of 4 columns and
 *   two chunks of staged draws exceed 160 KB of LDS (zeta <= 8: s > 3839 with FP64 arithmetic,
 *   s > 7679 with NSK_F32; zeta > 8: s > 767 and s > 1535);
 *   NSK_EWORKSPACE if
 *   ws_bytes < nsk_workspace_bytes(m, N, 1, d).
 */
int nsk_sketch(const nsk_operand* blocks, int32_t nblocks, int64_t m, const nsk_desc* d,
               double* SA, int64_t ldsa, void* ws, size_t ws_bytes, void* stream);

/*
 * Algorithm 1: trailing k right singular vectors of A through the sketch.
 * SA is reduced by Householder QR (FP64) to R (N x N); R is diagonalised by one-sided
 * Jacobi (FP64) with cyclic round-robin pair order and tolerance N*u (past N = 320 or
 * s = 4096: one-sided Jacobi on SA itself across the GPU, no QR); singular values
 * are sorted non-increasing (Section 3 ordering) and W = V(:, N-k+1:N) is returned.
 * Vk (device): N x k row-major FP64; column j belongs to sigma_{N-k+1+j}; each column is
 *   sign-normalised so that its entry of largest magnitude (lowest index on ties) > 0.
 * sigma_k (device): k FP64 values sigma_{N-k+1..N}, non-increasing.
 * info (device, nullable): nsk_info.  With NSK_FLAG_RESIDUAL, info->residual = |A Vk|_F.
 * Errors: as nsk_sketch, plus NSK_EINVAL if k < 1 or k > N or N > 1024; NSK_ENOCONV is
 *   reported through info->converged (the call itself cannot wait for the device).
 */
int nsk_trailing_rsv(const nsk_operand* blocks, int32_t nblocks, int64_t m, int64_t k,
                     const nsk_desc* d, double* Vk, double* sigma_k, nsk_info* info,
                     void* ws, size_t ws_bytes, void* stream);

/*
 * nsk_trailing_rsv without a caller workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid allocation).  The
 * workspace is a fixed array of nsk_noalloc_scratch_bytes() bytes (96 MiB) that the library's
 * code object places in device memory, one copy per GPU, held until the process ends; its
 * device address is looked up once per GPU (first call with that GPU current).  The call
 * itself allocates nothing.  Arguments, outputs and errors as nsk_trailing_rsv, plus
 * NSK_EWORKSPACE when nsk_workspace_bytes(m, N, k, d) exceeds the array (the 1,000,000 x 201
 * TLS workload needs 57-63 MiB, the 2,000,000 x 257 one 80 MiB) and NSK_EDEVICE when the
 * array's address cannot be obtained.  `stream` must belong to the current GPU.  Every call on
 * one GPU uses that GPU's array: calls whose work overlaps on one GPU (several streams or host
 * threads) race; serialise them, e.g. on one stream.
 */
size_t nsk_noalloc_scratch_bytes(void);
int nsk_trailing_rsv_noalloc(const nsk_operand* blocks, int32_t nblocks, int64_t m, int64_t k,
                             const nsk_desc* d, double* Vk, double* sigma_k, nsk_info* info,
                             void* stream);

/*
 * Total least squares with k = nrhs right-hand sides (Section 4): the trailing nrhs right
 * singular vectors V_k of the sketched [A | B] (the operand's last nrhs columns are B, so
 * N = n + nrhs) give X = -V12 V22^{-1}, V12 = V_k(1:n, :), V22 = V_k(n+1:N, :).
 * X (device): n x nrhs row-major FP64.  Vk (device, N x nrhs) and sigma_k (device, nrhs, nullable)
 * receive the trailing vectors and singular values as in nsk_trailing_rsv.  Workspace as
 * nsk_workspace_bytes(m, N, nrhs, d).  Sizes past the register-blocked SVD (N > 320 or s > 4096)
 * run the multi-workgroup Jacobi on SA.  Errors: as nsk_trailing_rsv with k = nrhs, and
 * NSK_EINVAL for nrhs < 1, nrhs > 64 or nrhs >= N.  A singular V22 (no TLS solution) gives
 * non-finite entries of X.
 */
int nsk_tls_solve_multi(const nsk_operand* blocks, int32_t nblocks, int64_t m, int64_t nrhs,
                        const nsk_desc* d, double* X, double* Vk, double* sigma_k, nsk_info* info,
                        void* ws, size_t ws_bytes, void* stream);

/*
 * Epsilon-tolerance version of Algorithm 1 (Section 2): the right singular vectors of SA whose
 * singular values are below eps (relative = 0) or below eps * sigma_1(SA) (relative = 1); with
 * eps = O(u) and relative = 1, the numerical null space.  V (device, N x N row-major FP64)
 * receives all N right singular vectors with column j belonging to sigma (device, N FP64,
 * non-increasing), each sign-normalised as in nsk_trailing_rsv; count (device, one int32)
 * receives how many trailing columns of V lie below the threshold.  Workspace as
 * nsk_workspace_bytes(m, N, N, d).  Errors: as nsk_trailing_rsv with k = N, and NSK_EINVAL for
 * a negative or non-finite eps, relative outside {0, 1}, or a null count.
 */
int nsk_null_space(const nsk_operand* blocks, int32_t nblocks, int64_t m, double eps, int32_t relative,
                   const nsk_desc* d, double* V, double* sigma, int32_t* count, nsk_info* info,
                   void* ws, size_t ws_bytes, void* stream);

/*
 * AAA rational approximation with a reused sketch (Section 6), real sample points z (device,
 * m distinct FP64) and values f (device, m FP64).  Support points are taken greedily where
 * |f - r| is largest (the lowest index on ties; r is the mean of f before the first one), r the
 * barycentric approximant sum_j w_j f_j / (z - z_j) / sum_j w_j / (z - z_j); the weights w are
 * the trailing right singular vector of the s x k sketch of the Loewner matrix
 * L[i, j] = (f_i - f_j) / (z_i - z_j) (non-support rows i, support columns j), kept up to date
 * by one row downdate (Algorithm 3) and one column update per support point (Section 6.2).
 * The loop stops when the largest error is at most tol * max|f| or after n_max support points.
 * d: NSK_SRHT, NSK_SRDCT or NSK_SPARSE_SIGN (other kinds return NSK_EUNSUPPORTED), with
 * n_max < s <= m, n_max <= 320 and s <= 4096.
 * support (host, n_max): sample indices in the order taken; n_support (host): their number;
 * weights (device, n_max FP64): the first n_support entries are w, sign-normalised as in
 * nsk_trailing_rsv; err_hist (host, n_max + 1, nullable): the largest error before each
 * step, the last entry that of the returned approximant.  The call blocks: the host reads
 * each step's largest error to decide whether to go on.  ws: nsk_aaa_workspace_bytes.
 */
size_t nsk_aaa_workspace_bytes(int64_t m, int32_t n_max, const nsk_desc* d);
int nsk_aaa(const double* z, const double* f, int64_t m, int32_t n_max, double tol, const nsk_desc* d,
            int64_t* support, double* weights, int32_t* n_support, double* err_hist, void* ws,
            size_t ws_bytes, void* stream);

/*
 * Row updates and downdates of a sketch (Section 5, Algorithms 2 and 3), in place:
 *     SA += sum_t ops[t] S_r(:, rows[t]) a_t,
 * where a_t is row t of the r x N operand `blocks` (NSK_F32 / NSK_F64 rows, or the Gaussian
 * kind's NSK_BF16 / NSK_F8E4M3 with the same column exponents as the sketched matrix),
 * ops[t] = +1 adds the row (update) and -1 removes it (downdate), and S_r is the updated
 * sketching matrix of the sketch (d, m) that produced SA: its column j is column j of S for a
 * row j < m of the sketched matrix, and g_j / sqrt(s) for a row appended at index j >= m, with
 * g_j the j-th column of the Gaussian kind's G (Algorithm 2; Section 5.3 takes the same appended
 * column for the non-Gaussian kinds).  For NSK_GAUSSIAN every column is G_hat(:, j) / sqrt(s),
 * so an update equals sketching the changed matrix from scratch.  Keep m at the row count that
 * was sketched across a sequence of updates; a removed original row j is downdated with its
 * values A(j, :), an appended one with the values it was added with.
 * A column update is nsk_sketch of the new columns into the matching columns of SA (SA pointer
 * offset, same ldsa); a column downdate drops the column of SA.
 * rows, ops (host, r entries): row indices >= 0 and signs +-1, copied into a pinned staging
 * buffer before the call returns (the caller may reuse them at once).  SA (device): s x N
 * row-major FP64, row stride ldsa >= N.  ws (device): nsk_update_workspace_bytes(r, d) bytes.
 * NSK_HRHT returns NSK_EUNSUPPORTED (its columns are not regenerated one at a time).
 * Errors: as nsk_sketch for (m, N, d) and the operand; NSK_EINVAL for a negative row index, a
 * sign other than +-1, r < 0 or r > 2^30; NSK_EWORKSPACE for a short workspace.  r = 0 does
 * nothing.
 */
size_t nsk_update_workspace_bytes(int64_t r, const nsk_desc* d);
int nsk_sketch_rows(const nsk_operand* blocks, int32_t nblocks, int64_t r, const int64_t* rows,
                    const int8_t* ops, int64_t m, const nsk_desc* d, double* SA, int64_t ldsa,
                    void* ws, size_t ws_bytes, void* stream);

/*
 * Residual |A Vk|_F of Problem 2.1 with FP64 accumulation (one more read of A).
 * Vk (device): N x k row-major FP64.  out (device): one FP64 value.
 * NSK_EUNSUPPORTED if N * k > 16384 (V_k is staged in LDS); the same limit applies to
 * NSK_FLAG_RESIDUAL in nsk_trailing_rsv.
 */
int nsk_residual(const nsk_operand* blocks, int32_t nblocks, int64_t m, const double* Vk,
                 int64_t k, double* out, void* ws, size_t ws_bytes, void* stream);

/*
 * Batched Algorithm 1: `count` independent problems in one persistent launch.  Each
 * workgroup takes sketch tiles from a longest-first queue; the workgroup that completes
 * an instance's last tile reduces its partial sketches and runs its QR + Jacobi.
 * probs (host array): per-instance operand (single block), sizes, sketch size, seed, k
 *   and device output pointers; read before the call returns.  base: kind (NSK_SRHT; other
 *   kinds return NSK_EUNSUPPORTED), acc, max_sweeps; its s and seed are ignored.  Tile sizes
 *   come from the autotuner.  Each instance's row sample is drawn on the device.
 * Errors: NSK_EINVAL for an instance with n outside 1..256, s outside n+1..min(m, 1024),
 *   k outside 1..n, ld < n or a null pointer, or mixed dtypes; NSK_EUNSUPPORTED for m > 2^31.
 */
typedef struct nsk_problem {
  const void* A;        /* device, row-major m x n, NSK_F32 or NSK_F64                     */
  int32_t dtype;
  int32_t reserved;
  int64_t m, n, ld;
  int64_t k;            /* 1 <= k <= n                                                     */
  int64_t s;            /* n < s <= m                                                      */
  uint64_t seed;
  double* Vk;           /* device n x k                                                    */
  double* sigma_k;      /* device k                                                        */
  nsk_info* info;       /* device, nullable                                                */
} nsk_problem;

size_t nsk_batched_workspace_bytes(const nsk_problem* probs, int32_t count,
                                   const nsk_desc* base);
int nsk_trailing_rsv_batched(const nsk_problem* probs, int32_t count, const nsk_desc* base,
                             void* ws, size_t ws_bytes, void* stream);

/*
 * Autotuner of the batched launch: the tile height ("rows per tile", in 1024-row transform
 * blocks) is chosen per n-bucket (32 columns wide) by timing the candidates 2..64 on up to
 * `per_bucket` of the caller's instances with HIP events (host-blocking; overwrites those
 * instances' outputs; skips candidates whose workspace exceeds ws_bytes).  Results are kept
 * per process and, when the environment variable NSK_TUNE_CACHE names a file, persisted
 * there as text and reloaded by later processes.  nsk_tune_lookup returns the value in use
 * for an n (tuned, cached, or the default ~ n/16); nsk_tune_set overrides one entry;
 * nsk_tune_clear empties the table.
 */
int nsk_autotune_batched(const nsk_problem* probs, int32_t count, const nsk_desc* base, void* ws,
                         size_t ws_bytes, void* stream, int32_t per_bucket);
int nsk_tune_lookup(int n, int dtype, int acc);
int nsk_tune_set(int n, int dtype, int acc, int rows_per_tile);
int nsk_tune_clear(void);

/*
 * Total least squares with one right-hand side (Section 4, Golub-Van Loan): the trailing
 * right singular vector v of the sketched [A | b] (N = n + 1 columns) gives
 * x = -v(1:n) / v(N).  `state` (device, nsk_tls_state_bytes(n, s, d->max_sweeps) bytes)
 * receives what the backward pass needs: SA, the singular values, v, x and the Jacobi
 * rotation log (V is rebuilt from it only where the backward needs it).  Built for
 * N = n + 1 <= 320 and s <= 4096 (NSK_EUNSUPPORTED otherwise).
 * x (device): n FP64.  With NSK_FLAG_RESIDUAL, info->residual = |[A | b] v|_F.
 */
size_t nsk_tls_state_bytes(int64_t n, int64_t s, int32_t max_sweeps);
int nsk_tls_solve(const nsk_operand* blocks, int32_t nblocks, int64_t m, const nsk_desc* d,
                  double* x, void* state, size_t state_bytes, nsk_info* info, void* ws,
                  size_t ws_bytes, void* stream);

/*
 * Gradient of a loss L(x) with respect to [A | b] through the sketched TLS solution.
 * d, m, n: the same descriptor and sizes as the nsk_tls_solve call that filled `state`.
 * gx (device, n FP64): dL/dx.  With g_bar = dL/dv = -(1/v_N)[gx; gx.x],
 * w = sum_{j<N} v_j (v_j.g_bar) / (sigma_N^2 - sigma_j^2) (first-order perturbation of
 * the trailing right singular vector of SA), p = S^T (SA v), q = S^T (SA w) with S
 * regenerated from the seed, the gradient is the rank-2 matrix p w^T + q v^T:
 * dA (device, m x n, row stride ldda >= n) = its first n columns, db (device, m) the last.
 * out_dtype: NSK_F32 or NSK_F64 for dA and db.  Built for NSK_SPARSE_SIGN and NSK_SRHT;
 * NSK_GAUSSIAN, NSK_SRDCT and NSK_HRHT return NSK_EUNSUPPORTED.  A degenerate gap (sigma_N = sigma_j) gives
 * non-finite output: the TLS solution is then not differentiable.
 */
int nsk_tls_backward(const nsk_desc* d, int64_t m, int64_t n, const void* state, const double* gx,
                     void* dA, int64_t ldda, void* db, int32_t out_dtype, void* ws, size_t ws_bytes,
                     void* stream);

/*
 * Stage profiler (tracing aid).  nsk_profile_enable(max_calls) creates
 * NSK_PROF_STAGES+1 HIP events for each of up to max_calls subsequent calls of
 * nsk_trailing_rsv / nsk_tls_solve / nsk_sketch and records them on the call's stream at
 * the stage boundaries (0 host draws and uploads, 1 sketch kernel, 2 partial reduce,
 * 3 Householder QR of SA, 4 one-sided Jacobi, 5 ranking and vector rebuild from the
 * rotation log, 6 post-processing: residual or TLS extraction).  nsk_profile_read waits
 * for the recorded events and returns the summed milliseconds per stage and the number of
 * profiled calls; nsk_profile_enable(0) stops recording and frees the events.
 */
#define NSK_PROF_STAGES 7
int nsk_profile_enable(int32_t max_calls);
int nsk_profile_read(double* ms /* NSK_PROF_STAGES */, int32_t* calls);

/*
 * Draw hooks: the random objects behind S, bit-exact between host and device.
 * Philox4x32-10 block with counter (lo32(idx), hi32(idx), sub, stream) and key
 * (lo32(seed), hi32(seed)); streams: 1 signs, 2 SRHT rows, 3 sparse rows, 4 sparse
 * signs, 5 Gaussian entries.
 */
int nsk_philox(uint64_t seed, uint64_t idx, uint32_t sub, uint32_t stream,
               uint32_t out[4]);                                        /* host           */
int nsk_draw_signs(uint64_t seed, int64_t m, int8_t* d);                 /* host, +-1      */
int nsk_draw_srht_rows(uint64_t seed, int64_t m, int64_t s, int64_t* rows);  /* host, sorted */
int nsk_draw_sparse(uint64_t seed, int64_t m, int64_t s, int32_t zeta, int32_t* rows,
                    int8_t* signs);                                      /* host, m x zeta */
int nsk_draw_signs_device(uint64_t seed, int64_t m, int8_t* d, void* stream);
/* rows (device): the s sorted sampled rows of [0, 2^ceil(log2 m)) that nsk_draw_srht_rows
 * returns, drawn by the parallel resolution of Floyd's rule the sketches use (s <= 2048,
 * m <= 2^31). */
int nsk_draw_srht_rows_device(uint64_t seed, int64_t m, int64_t s, int32_t* rows, void* stream);
int nsk_draw_sparse_device(uint64_t seed, int64_t m, int64_t s, int32_t zeta, int32_t* rows,
                           int8_t* signs, void* stream);
/* G (device): s x (j1 - j0) row-major FP32, entries G_hat[i, j0 + c] rounded to dtype
 * (NSK_BF16 or NSK_F8E4M3; NSK_F32 leaves the FP32 Box-Muller value unrounded). */
int nsk_draw_gaussian_device(uint64_t seed, int64_t s, int64_t j0, int64_t j1, int32_t dtype,
                             float* G, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NSK_H */
