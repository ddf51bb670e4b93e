/*
 * tucker.h - C ABI of the MI355X (gfx950) library for fixed-rank Tucker
 * approximation by shifted randomized T-HOSVD and ST-HOSVD.
 *
 * The method is Algorithms 2 and 3 of Che, Wei, Wu, Yan, "Fixed-Rank
 * Approximations in Tucker Format with Adaptive Shifts based on Fast
 * Randomized Algorithms" (arXiv 2506.04840): for each mode k, a Gaussian
 * sketch Y = X_(k) Omega_k, then q shifted power steps
 * Y <- X_(k)(X_(k)^T Q) - alpha Q, each followed by an economy SVD and the
 * midpoint shift update, then U_k = Q(:, 1:r_k) and G <- G x_k U_k^T.
 * It solves the fixed-Tucker-rank problem of the paper's Problem 1.
 *
 * Conventions shared by every entry point:
 *  - Tensors are dense, row-major (C order, last index fastest), with
 *    order 1..TUCKER_MAX_ORDER. Modes are 0-based here; the paper counts from 1.
 *  - The mode-k unfolding is never materialised. A tensor is viewed as
 *    [P, n_k, S] with P = prod_{j<k} n_j and S = prod_{j>k} n_j, so that
 *    X_(k)[i, p*S + s] = X[p, i, s].
 *  - Matrices are row-major: Y, Q are n_k x l, U_k is n_k x r_k.
 *  - Every data pointer is a DEVICE pointer owned by the caller. The library
 *    allocates no caller-visible memory and frees nothing. Scratch comes from
 *    a caller workspace whose size the *_workspace_bytes queries give.
 *  - Every call is asynchronous on the given stream (NULL = default stream).
 *    A call either enqueues all of its work and returns TUCKER_OK, or
 *    enqueues nothing and returns a negative tucker_status for errors found
 *    on the host (bad arguments, small workspace). Numeric events found on
 *    the device are written to the device-resident tucker_info and are
 *    readable once the stream is synchronised.
 *  - Calls are reentrant given distinct workspaces. Two calls that share a
 *    workspace must be ordered on one stream.
 *  - Precision: TUCKER_FP64 keeps tensors, factors and products in FP64.
 *    TUCKER_FP32 stores tensors and factors in FP32 and forms the mode
 *    products to FP32 accuracy on the matrix cores: by default the large
 *    products split each FP32 operand into three BF16 pieces and sum six
 *    BF16 products per pair in FP32 accumulators (the pieces carry 24
 *    significant bits; the terms left out are below 3 * 2^-24 of each
 *    product), which gfx950 runs at its BF16 rate; the FP32 instructions
 *    throughout with tucker_options.fp32_products = TUCKER_FP32_NATIVE
 *    (the other products, and sizes the split kernels do not cover, always
 *    use them). TUCKER_BF16 stores tensors and
 *    factors in FP32, runs the sketch and power products with BF16 operands
 *    and FP32 accumulation, and runs the core contraction in FP32. In every
 *    precision the Gram matrices, Cholesky factors, small SVD and shift are
 *    FP64.
 */
#ifndef TUCKER_H
#define TUCKER_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TUCKER_MAX_ORDER 8
#define TUCKER_MAX_Q 16 /* largest power count q */
#define TUCKER_MAX_Q_PVE 1000 /* largest q_max of tucker_rsthosvd_pve / tucker_rthosvd_pve */
#define TUCKER_MAX_L 64 /* largest sketch width l_k = min(r_k + p, n_k, m_k) */

typedef enum {
  TUCKER_OK = 0,
  TUCKER_EINVAL = -1,      /* invalid argument (see each call) */
  TUCKER_EWORKSPACE = -2,  /* workspace pointer null or smaller than required */
  TUCKER_EDEVICE = -3,     /* a HIP call failed (launch error, no device) */
  TUCKER_EUNSUPPORTED = -4 /* valid request outside what the library handles */
} tucker_status;

typedef enum { TUCKER_FP64 = 0, TUCKER_FP32 = 1, TUCKER_BF16 = 2 } tucker_precision;

typedef enum {
  TUCKER_SHIFT_ADAPTIVE = 0, /* the paper's midpoint shift (Algorithms 2, 3) */
  TUCKER_SHIFT_NONE = 1      /* alpha = 0 throughout: appendix Algorithm A.1 */
} tucker_shift;

typedef struct {
  int32_t order; /* d, 1..TUCKER_MAX_ORDER */
  int32_t reserved;
  int64_t dims[TUCKER_MAX_ORDER]; /* n_1..n_d, each >= 1 */
} tucker_shape;

/* Status bits of tucker_info.flags. */
#define TUCKER_INFO_NONFINITE 1  /* a non-finite value reached an orthonormalisation */
#define TUCKER_INFO_DEFICIENT 2  /* an iterate was numerically rank deficient; the basis
                                    was completed with random orthonormal directions */
#define TUCKER_INFO_L_CLAMPED 4  /* some l_k < r_k + p because n_k or m_k is smaller */
#define TUCKER_INFO_INTERNAL 8   /* an internal consistency check failed (a one-pass power step
                                    found its chunk counter out of step); the results are invalid */

/* Device-resident report of one solve (caller allocates sizeof(tucker_info)
 * bytes of device memory). Written by the solve's kernels. */
typedef struct {
  int32_t flags;                                /* TUCKER_INFO_* bits */
  int32_t l[TUCKER_MAX_ORDER];                  /* sketch width l_k used at each mode */
  int32_t deficient[TUCKER_MAX_ORDER];          /* deficient columns seen at the last svd of mode k */
  int32_t jacobi_sweeps;                        /* most sweeps any small SVD of the solve took */
  double alpha[TUCKER_MAX_ORDER][TUCKER_MAX_Q + 1];   /* alpha_t^(k), t = 0..q */
  double sigma_1[TUCKER_MAX_ORDER][TUCKER_MAX_Q + 1]; /* Sigma_k(1,1) after svd t (t=0: sketch) */
  double sigma_l[TUCKER_MAX_ORDER][TUCKER_MAX_Q + 1]; /* Sigma_k(l,l) after svd t */
  double normG2;                                /* ||G||_F^2 of the returned core (FP64 sum) */
  double normA2;                                /* ||A||_F^2 of the input tensor (FP64 sum) */
  double rel_error;                             /* sqrt(max(normA2 - normG2, 0) / normA2), 0 for a zero A */
  int32_t deficient_steps[TUCKER_MAX_ORDER];    /* bit t: the factorisation of iterate t of mode k found
                                                   numerically dependent columns (TUCKER_INFO_DEFICIENT) */
  int32_t reserved[6];
} tucker_info;

/* Flags of tucker_shifted_power. */
#define TUCKER_POWER_RAW 1 /* write only Y = X_(k)(X_(k)^T Q) - alpha Q (n_k x l, FP64) */

/* Human-readable text for a tucker_status; also the last error's detail
 * (thread-local) when the code matches the last failing call on this thread. */
const char* tucker_status_string(int status);

/* Workspace bytes for a whole solve (tucker_rthosvd when sequential == 0,
 * tucker_rsthosvd when sequential != 0) with these arguments. Returns 0 when
 * the arguments are invalid for that solve. */
size_t tucker_workspace_bytes(const tucker_shape* shape, const int64_t* ranks, int32_t p, int32_t q,
                              tucker_precision prec, int32_t sequential);

/* Workspace bytes for one tucker_sketch / tucker_shifted_power / tucker_orth
 * call on the mode-`mode` unfolding of `shape` with sketch width l. */
size_t tucker_op_workspace_bytes(const tucker_shape* shape, int32_t mode, int64_t l,
                                 tucker_precision prec);

/* Omega_mode[row0 : row0 + rows, 0 : cols] of the Gaussian test matrix (the
 * standard Gaussian matrix the paper draws for each mode, section 2 and the
 * draw at the top of Algorithms 2 and 3), row-major into `out` (FP64 for
 * TUCKER_FP64, FP32 otherwise), exactly as the sketch kernels use it.
 * Generator: Philox4x32-10 with key = seed and counter = (row lo, row hi,
 * col / 4, mode), Box-Muller on (w0,w1) for (col/2) even and (w2,w3) for odd.
 * EINVAL: rows < 0, cols < 0, row0 < 0, mode outside 0..TUCKER_MAX_ORDER-1,
 * out null with rows*cols > 0. */
int tucker_fill_gaussian(uint64_t seed, int32_t mode, int64_t row0, int64_t rows, int64_t cols,
                         tucker_precision prec, void* out, hipStream_t stream);

/* Test-matrix kinds (section 5, comparison of random matrices). */
typedef enum {
  TUCKER_OMEGA_GAUSSIAN = 0,    /* standard Gaussian (the default of every solve) */
  TUCKER_OMEGA_UNIFORM = 1,     /* i.i.d. uniform on [-1, 1] */
  TUCKER_OMEGA_KR_GAUSSIAN = 2, /* Khatri-Rao product of Gaussian factors */
  TUCKER_OMEGA_KR_UNIFORM = 3   /* Khatri-Rao product of uniform factors */
} tucker_omega;

/* Omega_mode[row0 : row0 + rows, 0 : cols] of test-matrix kind `kind` for a
 * tensor of order d with current sizes dims[0..d-1] (the matrix has
 * prod_{i != mode} dims[i] rows, in the column order of the mode unfolding),
 * row-major into `out` (FP64 for TUCKER_FP64, FP32 otherwise). Streams of the
 * Philox4x32-10 generator of tucker_fill_gaussian: the fourth counter word is
 * `mode` for the dense kinds and 4096 + 16 mode + i for the Khatri-Rao factor
 * of mode i; uniform streams add 2^30 and map word (col mod 4) of the block to
 * (w + 1/2) 2^-31 - 1. Khatri-Rao: entry [c, j] is the product, in increasing
 * mode order, of the factors' entries [c_i, j], where (c_i) is c in row-major
 * order over the other modes. Gaussian kind: the same values as
 * tucker_fill_gaussian. EINVAL: bad kind, d outside 1..8, mode outside 0..d-1,
 * a size < 1, negative rows / cols / row0, out null with rows*cols > 0. */
int tucker_fill_test_matrix(int32_t kind, uint64_t seed, int32_t mode, int32_t d, const int64_t* dims, int64_t row0,
                            int64_t rows, int64_t cols, tucker_precision prec, void* out, hipStream_t stream);

/* Processing order of the modes (Section 2.2: ST-HOSVD may take the modes in
 * any order of the symmetric group; Section 3.2 takes n_{p_1} >= ... >= n_{p_d}
 * for its cost count). */
typedef enum {
  TUCKER_ORDER_NATURAL = 0,    /* 0, 1, ..., d-1 (the plain solves) */
  TUCKER_ORDER_GIVEN = 1,      /* opt->order[0..d-1], a permutation of 0..d-1 */
  TUCKER_ORDER_DECREASING = 2  /* by decreasing n_k; equal sizes in increasing mode */
} tucker_order;

/* How TUCKER_FP32 forms its mode products (the default first). */
typedef enum {
  TUCKER_FP32_SPLIT = 0,  /* three-piece BF16 split, six BF16 products, FP32 accumulation */
  TUCKER_FP32_NATIVE = 1  /* FP32 matrix-core instructions only */
} tucker_fp32_products;

/* Options of the _ex solves. A zeroed struct gives the plain solves. */
typedef struct {
  int32_t omega;                    /* tucker_omega */
  int32_t order_kind;               /* tucker_order */
  int32_t order[TUCKER_MAX_ORDER];  /* TUCKER_ORDER_GIVEN: processing order, first d entries */
  int32_t holistic;                 /* 0: Algorithms 2 / 3; 1: the holistic variants (below) */
  int32_t fp32_products;            /* tucker_fp32_products (TUCKER_FP32 only) */
  int32_t reserved[4];              /* zero */
} tucker_options;

/* Sketch Y = X_(mode) Omega_mode (Algorithms 2 and 3: the first product of
 * each mode). X has `shape` (FP64 for TUCKER_FP64, FP32 otherwise). Omega
 * is the m x l matrix of tucker_fill_gaussian(seed, mode, 0, m, l) with
 * m = numel(X) / n_mode. Y: n_mode x l row-major in the storage precision
 * (FP64 for TUCKER_FP64, FP32 otherwise: the split sums are added in FP64
 * in a fixed order, then rounded once), overwritten.
 * EINVAL: bad shape, mode, l < 1 or l > min(TUCKER_MAX_L, n_mode, m), null X/Y.
 * EWORKSPACE: ws_bytes < tucker_op_workspace_bytes(shape, mode, l, prec). */
int tucker_sketch(const tucker_shape* shape, int32_t mode, const void* X, int64_t l, uint64_t seed,
                  tucker_precision prec, void* Y, void* ws, size_t ws_bytes, hipStream_t stream);

/* One shifted power step (Algorithms 2 and 3, the inner loop):
 * M = X_(mode) (X_(mode)^T Q) - alpha Q with Q n_mode x l in the storage
 * precision and alpha a device double.
 * flags & TUCKER_POWER_RAW: write M (FP64, n_mode x l) to `out`; sigma and
 * alpha are left untouched.
 * otherwise: [Q', Sigma] = svd(M, econ); write Q' (storage precision,
 * n_mode x l, singular vectors in descending order of Sigma) to `out`,
 * Sigma (l doubles) to `sigma` and apply the midpoint rule to *alpha in
 * place: if Sigma(l,l) > alpha then alpha = (Sigma(l,l) + alpha) / 2.
 * `out` must not alias Q. EINVAL / EWORKSPACE as for tucker_sketch, plus
 * null Q, alpha or (non-raw) sigma.
 * Unfoldings viewed as P x n x S with n <= m form both products in one pass
 * over X (the same pass the solves use for their power steps) where a
 * one-pass kernel applies: on the BF16 matrix cores for S >= 32, S a multiple
 * of 4, l <= 64 and n <= 1024 (BF16 operands at any such n; FP32 products,
 * taken through the three-piece BF16 split, at n > 256); with FP32
 * instructions when the solve's options select native FP32 products (S >= 64,
 * S and n multiples of 4, n <= 512, l <= 48). The others run the two products
 * one after the other. */
int tucker_shifted_power(const tucker_shape* shape, int32_t mode, const void* X, int64_t l,
                         const void* Q, double* alpha, int32_t flags, tucker_precision prec,
                         void* out, double* sigma, void* ws, size_t ws_bytes, hipStream_t stream);

/* [Q, Sigma, ~] = svd(Y, 'econ') of an n x l FP64 matrix Y (the svd the
 * paper applies to every iterate), by CholeskyQR with a shifted first pass
 * and two re-orthogonalisation passes, then a one-sided Jacobi SVD of the
 * l x l triangular factor, all in FP64. Q: n x l in the storage precision,
 * columns ordered by descending Sigma; Sigma: l doubles. Numerically
 * deficient columns are completed with random orthonormal directions and
 * get Sigma = 0. Uses the workspace of tucker_op_workspace_bytes with a
 * shape whose mode-0 size is n. EINVAL: n < l, l < 1, l > TUCKER_MAX_L, nulls. */
int tucker_orth(int64_t n, int64_t l, const double* Y, tucker_precision prec, void* Q, double* sigma,
                void* ws, size_t ws_bytes, hipStream_t stream);

/* Core contraction step X_out = X x_mode U^T (Algorithms 2 and 3, the
 * update of G after each mode; the mode-k product of section 2).
 * U: n_mode x r in the storage precision. X_out has the dims of X with
 * dims[mode] replaced by r, same layout convention, storage precision (the
 * product runs in FP32 for TUCKER_BF16). No workspace.
 * EINVAL: bad shape or mode, r < 1, r > TUCKER_MAX_L, nulls. */
int tucker_core(const tucker_shape* shape, int32_t mode, const void* X, const void* U, int64_t r,
                tucker_precision prec, void* Xout, hipStream_t stream);

/* ||X||_F^2 of `numel` elements in the storage precision, FP64 accumulation
 * in a fixed order, written to *out (device double). ws: device scratch of
 * at least TUCKER_NORM2_WS_BYTES bytes. EINVAL: nulls, numel < 0. */
#define TUCKER_NORM2_WS_BYTES 8192
int tucker_norm2(const void* X, int64_t numel, tucker_precision prec, double* out, void* ws, size_t ws_bytes,
                 hipStream_t stream);

/* Shifted randomized T-HOSVD (Algorithm 2): every factor is computed from A;
 * then G = A x_1 U_1^T ... x_d U_d^T.
 * A: `shape`, storage precision. ranks: d host int64 values r_k with
 * 1 <= r_k <= n_k and r_k <= prod_{j != k} n_j. p >= 0 oversampling,
 * 0 <= q <= TUCKER_MAX_Q power steps. l_k = min(r_k + p, n_k, m_k) above
 * TUCKER_MAX_L returns TUCKER_EUNSUPPORTED. seed selects Omega_k = tucker_fill_gaussian(seed, k, ...).
 * G: r_1 x ... x r_d; U[k]: n_k x r_k (device pointers, storage precision;
 * columns ordered by descending singular value, each column's largest-
 * magnitude entry made positive). info: device tucker_info or NULL.
 * EINVAL on any violated bound, EWORKSPACE when ws_bytes is smaller than
 * tucker_workspace_bytes(shape, ranks, p, q, prec, 0). */
int tucker_rthosvd(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
                   tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U,
                   tucker_info* info, void* ws, size_t ws_bytes, hipStream_t stream);

/* Shifted randomized ST-HOSVD (Algorithm 3), processing order 1..d: mode k
 * works on X = A x_1 U_1^T ... x_{k-1} U_{k-1}^T, so m_k = r_1..r_{k-1}
 * n_{k+1}..n_d and the feasibility bound is r_k <= m_k. Arguments as for
 * tucker_rthosvd, with workspace tucker_workspace_bytes(..., 1). */
int tucker_rsthosvd(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
                    tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U,
                    tucker_info* info, void* ws, size_t ws_bytes, hipStream_t stream);

/* tucker_rsthosvd for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, with its scratch taken from a static device array of
 * TUCKER_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends, instead of a caller workspace. The caller still
 * passes A, G, U and info. Arguments, layouts, results and errors as
 * tucker_rsthosvd, plus EWORKSPACE when tucker_workspace_bytes(shape, ranks,
 * p, q, prec, 1) exceeds TUCKER_NOALLOC_SCRATCH_BYTES (checked on the host
 * before anything is enqueued). The call allocates nothing and creates no
 * stream or event: every launch goes to `stream`, so the small SVDs do not
 * overlap the products as they do in tucker_rsthosvd (same results).
 * The first call on a device resolves that device's copy of the array
 * (hipGetSymbolAddress, with the device current). Every call on one device
 * shares its array and finds the previous call's contents there (the solve
 * initialises what it reads): two calls on one device that may overlap in
 * time, on different streams or from different threads, race and give
 * undefined results. Order them on one stream. */
#define TUCKER_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int tucker_rsthosvd_noalloc(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
                            tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U,
                            tucker_info* info, hipStream_t stream);

/* tucker_rthosvd / tucker_rsthosvd with options (opt may be NULL: the plain
 * call). Mode k draws its test matrix of kind opt->omega as
 * tucker_fill_test_matrix(kind, seed, k, d, current sizes), the current sizes
 * being A's for T-HOSVD and, for ST-HOSVD, r_j for the modes j processed
 * before k and n_j for the others. ST-HOSVD processes the modes in the order
 * opt->order_kind selects: mode k works on A contracted with the U_j^T of the
 * modes before it, so m_k, l_k and the feasibility bound r_k <= m_k follow
 * the order, and the core is contracted in that order. T-HOSVD computes
 * every factor from A (the order does not change its result) and contracts
 * the core in mode order. Factors, info logs and test-matrix streams stay
 * indexed by mode. Workspace: tucker_workspace_bytes_ex with the same opt.
 *
 * opt->holistic = 1 selects the holistic variants of Appendices A and B
 * (Algorithm B.1 for tucker_rsthosvd_ex with the adaptive shift, its
 * unshifted model A.2 with TUCKER_SHIFT_NONE, and their T-HOSVD analogue for
 * tucker_rthosvd_ex). Phase 1 runs each mode's range finder as above but keeps
 * all l_k columns Q_k: ST-HOSVD contracts B = B x_k Q_k^T at once (later modes
 * see size l_k there, which sets their m and l), T-HOSVD forms B = A x_1
 * Q_1^T ... x_d Q_d^T after the loop. Phase 2 takes the deterministic
 * ST-HOSVD (T-HOSVD) of the small tensor B (l_1 x ... x l_d) in the same
 * order: V_k = leading r_k left singular vectors of the current unfolding
 * (CholeskyQR and one-sided Jacobi in FP64), U_k = Q_k V_k with the sign rule,
 * G = B x_k V_k^T with V_k's columns signed like U_k's. Info logs hold phase 1.
 * EINVAL also when some r_k exceeds the product of the other current sizes
 * in phase 2 (no unfolding of the small tensor has that rank); EUNSUPPORTED
 * for order d = 1.
 *
 * opt->fp32_products chooses how TUCKER_FP32 forms its products (see the
 * precision conventions at the top); other precisions ignore it.
 *
 * EINVAL for an unknown kind, an order that is not a permutation of 0..d-1,
 * holistic or fp32_products outside 0..1 or nonzero reserved fields;
 * otherwise as the plain calls. */
size_t tucker_workspace_bytes_ex(const tucker_shape* shape, const int64_t* ranks, int32_t p, int32_t q,
                                 tucker_precision prec, int32_t sequential, const tucker_options* opt);
int tucker_rthosvd_ex(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
                      tucker_shift shift, uint64_t seed, tucker_precision prec, const tucker_options* opt, void* G,
                      void* const* U, tucker_info* info, void* ws, size_t ws_bytes, hipStream_t stream);
int tucker_rsthosvd_ex(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q,
                       tucker_shift shift, uint64_t seed, tucker_precision prec, const tucker_options* opt, void* G,
                       void* const* U, tucker_info* info, void* ws, size_t ws_bytes, hipStream_t stream);

/* Algorithm 4: shifted randomized ST-HOSVD whose power count q_k is chosen per
 * mode by the per-vector-error test (Appendix, PVE accuracy control). Mode k
 * runs power steps t = 1, 2, ..., q_max and stops after the first step whose
 * estimates sigma_t(i) = Sigma_t(i,i) + alpha_{t-1} moved, for i <= r_k, by at
 * most tol * sigma_t(r_k + 1) since the previous step (sigma_t(l_k) when
 * l_k = r_k; the estimates of the step before the first are zero). The test
 * comes before that step's shift update, which is then skipped. With FP32
 * (and BF16) operands a change below 1e-6 sigma_t(1), the rounding level of
 * the iterate, counts as none (FP64: the test as printed). q_used[k]
 * receives q_k (host array, d entries). The remaining arguments are those of
 * tucker_rsthosvd (workspace tucker_workspace_bytes(..., min(q_max, 16),
 * prec, 1)); info logs the first TUCKER_MAX_Q steps.
 * Synchronisation: the next step's launch depends on this step's test, so the
 * call reads a 4-byte device flag after every power step and synchronises
 * `stream` that often; it returns with the solve complete.
 * BF16 operands: every power step runs on FP32 operands (any step may be the
 * last). EINVAL for q_max outside 1..TUCKER_MAX_Q_PVE, tol < 0 or NaN, or a
 * null q_used; otherwise as tucker_rsthosvd. */
int tucker_rsthosvd_pve(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q_max,
                        double tol, tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U,
                        tucker_info* info, int32_t* q_used, void* ws, size_t ws_bytes, hipStream_t stream);

/* The T-HOSVD form of Algorithm 4, which the paper names Algorithm 2-v3 (in
 * the remark after Algorithm 4; details omitted there): every mode from A, with
 * the power count of each mode chosen by the same test, and the core
 * A x_1 U_1^T ... x_d U_d^T at the end. The modes run one after the other on
 * `stream` (each reads its flag on the host). Arguments, synchronisation and
 * errors as tucker_rsthosvd_pve; workspace tucker_workspace_bytes(...,
 * min(q_max, 16), prec, 0). */
int tucker_rthosvd_pve(const tucker_shape* shape, const void* A, const int64_t* ranks, int32_t p, int32_t q_max,
                       double tol, tucker_shift shift, uint64_t seed, tucker_precision prec, void* G, void* const* U,
                       tucker_info* info, int32_t* q_used, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- Launch timing (measurement only) ---------------------------------------
 * When a kernel class is enabled, every launch of that class records a pair
 * of HIP events on its launch stream (up to `capacity` launches; later ones
 * are counted as dropped) and sums each launch's algorithmic HBM bytes and
 * flops (the unfolding read once, plus the skinny operand and result; flops
 * 2 * numel * width). One class at a time, process-wide. */
#define TUCKER_KC_COLREDUCE 0   /* X_(k) B: sketch and the second half of a power step */
#define TUCKER_KC_ROWCONTRACT 1 /* X_(k)^T W: first half of a power step and core step */
#define TUCKER_KC_ORTH 2        /* one whole svd(Y, econ) sequence */
#define TUCKER_KC_FILL 3        /* Gaussian test-matrix fill */
#define TUCKER_KC_REDUCE 4      /* split-partial reduction with the -alpha Q term */
#define TUCKER_KC_POWERSTEP 5   /* X_(k) (X_(k)^T Q) in one pass over X (the power steps that take a
                                   one-pass kernel, see tucker_shifted_power); bytes: X once plus Q;
                                   flops 4 * numel * l */
/* EINVAL: bad class or capacity outside 1..2^20. EDEVICE: event creation failed. */
int tucker_timing_enable(int32_t kernel_class, int32_t capacity);
/* Waits for the recorded events; total device milliseconds, launch count,
 * summed bytes and flops (bytes, flops may be NULL). EINVAL if the class is
 * not the enabled one; EUNSUPPORTED (values still written) if launches were
 * dropped for lack of capacity. */
int tucker_timing_read(int32_t kernel_class, double* total_ms, int64_t* launches, double* bytes, double* flops);
/* Forget recorded launches, keep the class enabled. */
int tucker_timing_reset(void);
/* Disable and free the events. */
int tucker_timing_disable(void);

/* ---- Batched solves: many small shifted randomized ST-HOSVDs at once ------
 * Algorithm 3 for a set of requests of one order d and one power count q,
 * FP32 storage (Section 3.1; the same arithmetic as tucker_rsthosvd with FP32
 * and the default TUCKER_FP32_SPLIT products, shift as given). Every phase of the method runs as one persistent launch
 * over all requests of the batch (a fixed grid looping over a table of work
 * items), so a batch costs the same number of launches as one request.
 *
 * The launch sequence of tucker_batch_step depends only on (capacity, d, q,
 * lclass) and on the plan buffer and workspace addresses: a step captured into
 * a graph replays correctly for any later plan made with the same
 * (capacity, d, q, lclass) into the same plan buffer and workspace.
 *
 * Limits: 1 <= d <= 8, every l_k <= lclass (16, 32, 48 or 64), nitems <=
 * capacity <= 4096. info->normG2 is not computed by the batch path (0).
 * Ownership: every pointer in an item is the caller's device memory; the plan
 * is caller host memory (pinned, e.g. hipHostMalloc, so the step's upload is
 * asynchronous and capturable); the workspace is caller device memory. */
typedef struct {
  tucker_shape shape;                 /* dims of A */
  int64_t ranks[TUCKER_MAX_ORDER];
  uint64_t seed;                      /* Omega_k as in tucker_fill_gaussian */
  const void* A;                      /* FP32 tensor, row-major */
  void* G;                            /* FP32 core r_1 x ... x r_d */
  void* U[TUCKER_MAX_ORDER];          /* FP32 n_k x r_k */
  tucker_info* info;                  /* device, or NULL */
} tucker_batch_item;

/* Host plan buffer bytes and the device table bytes (the start of the batch
 * workspace) for a capacity. 0 on bad arguments. */
size_t tucker_batch_plan_bytes(int32_t capacity, int32_t order, int32_t q);
size_t tucker_batch_table_bytes(int32_t capacity, int32_t order, int32_t q);
/* Device workspace one item needs (0 on bad arguments); a batch workspace is
 * tucker_batch_table_bytes + the sum over its items (each rounded up to 256). */
size_t tucker_batch_item_bytes(const tucker_batch_item* item, int32_t p, int32_t q);
/* Host-only: validates the items, carves ws and writes the plan (nitems may
 * be 0). EINVAL for a bad item (same checks as tucker_rsthosvd) or an item
 * whose order is not `order`, EUNSUPPORTED
 * when some l_k > lclass, EWORKSPACE when ws or the plan is too small. On
 * any error the plan is left invalid (tucker_batch_step rejects it). */
int tucker_batch_plan(int32_t capacity, int32_t order, int32_t lclass, int32_t nitems, const tucker_batch_item* items,
                      int32_t p, int32_t q, tucker_shift shift, void* ws, size_t ws_bytes, void* plan,
                      size_t plan_bytes);
/* Enqueues the batch on `stream`: one upload of the plan's tables into the
 * workspace, then the persistent launches. Results land in each item's G, U
 * and info when the stream reaches this point. With launch timing enabled,
 * the product phases are recorded under TUCKER_KC_COLREDUCE / ROWCONTRACT /
 * REDUCE / FILL with the batch's summed algorithmic bytes and flops (do not
 * capture a step into a graph while timing is enabled). */
int tucker_batch_step(const void* plan, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TUCKER_H */
