// Host-side launchers shared by the C-ABI front end and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stddef.h>
#include <stdint.h>

#include "tucker.h"

namespace tk {

struct View3 {
  int64_t P, n, S;  // X viewed as row-major [P, n, S]
};

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Kernel classes of the opt-in launch timing (values of TUCKER_KC_*).
enum KernelClass {
  KC_COLREDUCE = 0,
  KC_ROWCONTRACT = 1,
  KC_ORTH = 2,
  KC_FILL = 3,
  KC_REDUCE = 4,
  KC_POWERSTEP = 5,
  KC_COUNT = 6
};

// Records a HIP event pair around the launches in its scope when `cls` is the
// enabled class; bytes and flops are the launch's algorithmic traffic and work.
// A kernel launched through TK_LAUNCH inside an active scope carries the pair
// itself (hipExtLaunchKernelGGL: the dispatch records the kernel's own start
// and end), so the pair then measures that kernel alone, without the dispatch
// gaps of separately recorded events.
class TimingScope {
 public:
  // stamped: the scope's one kernel is launched through TK_LAUNCH, which
  // records both events (no event is recorded around it)
  TimingScope(int cls, hipStream_t st, double bytes, double flops, bool stamped = false);
  ~TimingScope();
  TimingScope(const TimingScope&) = delete;
  TimingScope& operator=(const TimingScope&) = delete;
  // The scope of this host thread that is timing a launch on `st` and has not
  // handed out its events yet (nullptr otherwise); the caller launches with
  // start() / stop().
  static TimingScope* claim(hipStream_t st);
  hipEvent_t start() const;
  hipEvent_t stop() const;

 private:
  int slot_;
  hipStream_t st_;
  bool stamped_;
  bool attached_;
  TimingScope* prev_;
};

// hipLaunchKernelGGL, or hipExtLaunchKernelGGL with the events of the
// thread's active timing scope on that stream.
#define TK_LAUNCH(kern, grid, block, shm, st, ...)                                                        \
  do {                                                                                                    \
    ::tk::TimingScope* tk_ts_ = ::tk::TimingScope::claim(st);                                             \
    if (tk_ts_ != nullptr)                                                                                \
      hipExtLaunchKernelGGL(kern, grid, block, shm, st, tk_ts_->start(), tk_ts_->stop(), 0, __VA_ARGS__); \
    else                                                                                                  \
      hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__);                                        \
  } while (0)
inline size_t elem_bytes(tucker_precision p) { return p == TUCKER_FP64 ? 8 : 4; }

// How the FP32 launches of the calling host thread form their products
// (tucker_fp32_products), for the duration of one entry-point call: the
// launch functions read it when they choose a kernel.
class ProductScope {
 public:
  explicit ProductScope(int fp32_products);
  ~ProductScope();
 private:
  int prev_;
};
bool fp32_split_products();

// ---- Gaussian test matrix -------------------------------------------------
// Writes Omega[row0 + c, j] for c < rows, j < cols: jmajor -> out[j * rows + c]
// (the [cols, rows] layout the column reduction reads), else out[c * cols + j].
hipError_t launch_fill_gaussian(tucker_precision prec, uint64_t seed, uint32_t mode, int64_t row0,
                                int64_t rows, int cols, bool jmajor, void* out, hipStream_t st);

// Test matrix of any kind (TUCKER_OMEGA_*) for mode `mode`: nfac other modes
// of sizes fdim[0..nfac-1] (increasing mode order, product = the matrix's row
// count) with Khatri-Rao stream tags ftag[]. Layout as launch_fill_gaussian.
struct OmegaSpec {
  int32_t kind;
  int32_t nfac;
  int64_t fdim[TUCKER_MAX_ORDER];
  uint32_t ftag[TUCKER_MAX_ORDER];
};
// The spec of mode k's test matrix for a tensor whose current sizes are cur[0..d-1].
OmegaSpec omega_spec(int kind, int d, const int64_t* cur, int k);
hipError_t launch_fill_omega(const OmegaSpec& sp, tucker_precision prec, uint64_t seed, uint32_t mode, int64_t row0,
                             int64_t rows, int cols, bool jmajor, void* out, hipStream_t st);

// ---- mode products ----------------------------------------------------------
// Column reduction: part[split][i][j] = sum over the split's columns c of
// X_(k)[i, c] * B[c, j], B stored j-major as Bt[j * m + c] (m = P S).
// Output type: double for FP64, float otherwise.
int colreduce_splits(const View3& v, int l);
int colreduce_splits_for(const View3& v, int l, tucker_precision prec);
size_t colreduce_part_bytes(const View3& v, int l, tucker_precision prec);
// npart (S > 1 only; ignored for S == 1): also ||X||_F^2 as colreduce_norm_slots
// FP64 partial sums, one per workgroup, each over the elements that workgroup
// staged; launch_norm2_final adds them in a fixed order.
hipError_t launch_colreduce(tucker_precision prec, const View3& v, const void* X, const void* B, int l,
                            void* part, int nsplit, hipStream_t st, double* npart = nullptr);
int colreduce_norm_slots(const View3& v, int nsplit);

// Both products of a power step, Y' = X_(k) (X_(k)^T Q) as split partials
// (part[split][i][j], FP32 or FP64 as the column reduction's), from Q given
// j-major in the storage precision (qt[j * n + i]). Steps that a one-pass
// kernel takes (power_fused_launch_splits > 0: on the BF16 matrix cores for
// BF16 operands at n <= 1024 and FP32 products through the split at
// 256 < n <= 1024, S >= 32, l <= 64; with FP32 instructions for native FP32
// products, S >= 64, n <= 512, l <= 48) run one pass over X (part needs
// power_fused_part_bytes, which also holds Q's pieces; ctr: a chunk counter,
// zeroed together with *fused_count = 0 before a series of launches on this
// (v, l); each one-pass launch counts itself in *fused_count; z may be null);
// the others run the row contraction into z (j-major, P S x l;
// hipErrorInvalidValue when z is null) and the column reduction with nsplit
// splits. *nsplit_used: the split count to reduce. err (may be null): a
// one-pass launch whose counter disagrees with the base ors
// TUCKER_INFO_INTERNAL into it.
// power_fused_splits: the chunk count of the FP32 one-pass kernel for the
// shape alone; power_fused_launch_splits: the chunk count of the pass the
// launch takes, or 0 for the two-kernel path.
int power_fused_splits(const View3& v, int l, tucker_precision prec);
int power_fused_launch_splits(const View3& v, int l, tucker_precision prec);
size_t power_fused_part_bytes(const View3& v, int l, tucker_precision prec);
hipError_t launch_power_products(tucker_precision prec, const View3& v, const void* X, const void* qt, int l,
                                 void* z, void* part, int nsplit, int* ctr, int* fused_count, int* nsplit_used,
                                 hipStream_t st, int* err = nullptr);
// Qt[j n + i] = Q[i l + j], FP32.
hipError_t launch_transpose_f32(const float* Q, int64_t n, int l, float* Qt, hipStream_t st);

// Y[e] = sum_s part[s][e] - (qsub ? alpha * qsub[e] : 0), FP64 out.
// qsub_prec gives qsub's element type (FP64 or FP32 storage).
hipError_t launch_reduce_splits(tucker_precision part_prec, const void* part, int nsplit, int64_t nl,
                                const void* qsub, tucker_precision qsub_prec, const double* alpha,
                                double* Y, hipStream_t st);

// Row contraction: out(p, j, s) = sum_i X[p, i, s] * W(i, j) with
// W(i, j) = W[i * wsi + j * wsj] (row-major n x lw: wsi = lw, wsj = 1;
// j-major: wsi = 1, wsj = n). out_jmajor: out[j * m + p * S + s] (the layout
// the column reduction reads), else the tensor layout [P, lw, S].
// mk selects the matrix-core type (TUCKER_BF16 runs BF16 operands with FP32
// accumulation on FP32 data).
hipError_t launch_rowcontract(tucker_precision mk, const View3& v, const void* X, const void* W, int64_t wsi,
                              int64_t wsj, int lw, void* out, bool out_jmajor, hipStream_t st);

// ||X||^2 with FP64 accumulation; part must hold norm2_blocks() doubles.
int norm2_blocks(int64_t numel);
hipError_t launch_norm2(tucker_precision prec, const void* X, int64_t numel, double* part, double* out,
                        hipStream_t st);
// *out = sum of part[0 .. nb) in a fixed order.
hipError_t launch_norm2_final(const double* part, int nb, double* out, hipStream_t st);
// info->rel_error = sqrt(max(normA2 - normG2, 0) / normA2) (0 when normA2 is 0).
hipError_t launch_info_rel_error(tucker_info* info, hipStream_t st);

// ---- orthonormalisation (FP64) --------------------------------------------
struct OrthWs {
  double* Qa;     // n x l: Q1, then Q2 and Q3 in place
  double* part;   // gram partials, ping-pong [2][nblk][l][l]
  double* R;      // 3 x kMaxL^2: R1, R2, R3 (each l x l row-major)
  double* Wm;     // l x l left singular vectors of R (columns, descending)
  int* defic;     // 3 x 64
  int* status;    // [0] flags, [1] deficient count, [2] 1 when pass 3 was skipped
  int* pf_ctr;    // chunk counter of the fused power step (not part of either set)
  // a second R / flags / status set, so that the factorisation of step t + 1
  // can run while the small SVD of step t still reads its own
  double* R_odd;
  int* defic_odd;
  int* status_odd;
  // the sketch's set when power steps follow: its small SVD only feeds the
  // info logs, so it reads and writes nothing the power steps use
  double* R_log;
  int* defic_log;
  int* status_log;
  double* Wm_log;
};
size_t orth_ws_bytes(int64_t n, int l);
OrthWs carve_orth(void* base, int64_t n, int l);
// The workspace of power step `step`: R, flags and status of its parity (odd
// steps use the second set), the rest shared.
OrthWs orth_step_set(const OrthWs& w, int step);
// The sketch's own set (R, flags, status and Wm), for a sketch whose small SVD
// only feeds the logs.
OrthWs orth_log_set(const OrthWs& w);

// CholeskyQR part of svd(Y): Y (FP64 n x l) = Q3 R with Q3 in ws.Qa and the R
// factors in ws.R. With Wrot != nullptr, Y is first replaced in place by
// Y Wrot (l x l). qt (when not nullptr) receives Q3 j-major (l x n) in the
// storage precision `prec`.
hipError_t launch_orth_qr(int64_t n, int l, double* Y, const double* Wrot, tucker_precision prec, void* qt,
                          const OrthWs& ws, uint64_t cseed, int step, hipStream_t st);
// Small SVD of R after launch_orth_qr: ws.Wm, sigma (l doubles, descending)
// and, when alpha != nullptr, the midpoint shift update of *alpha. When
// info != nullptr, Sigma(1,1), Sigma(l,l) and alpha are logged at
// [mode][step], and status bits are or-ed into info->flags.
// `prec` is the precision the iterate's products ran in (sets the rotation
// thresholds).
// Per-vector-error stopping test of Algorithm 4, evaluated by the small SVD of
// step `step` (nullptr: off). At step 0 it clears sig_hat and *stop. At step
// t >= 1 it forms sigma_t(i) = Sigma(i,i) + alpha_{t-1} (alpha_{t-1} read from
// alpha_prev), sets *stop when max_{i < r} |sigma_t(i) - sig_hat(i)| <= tol *
// sigma_t(min(r, l - 1)) (0-based), skips the shift update then, and else
// stores sigma_t into sig_hat.
// floor: changes below floor * sigma_t(1) count as none (the rounding level of
// an iterate formed from FP32 products; 0 for FP64, the test as printed).
struct SvdPve {
  int r;
  double tol;
  double floor;
  const double* alpha_prev;
  double* sig_hat;  // l doubles
  int* stop;
};
// vright (when not nullptr): the right singular vectors of R (l x l, columns,
// descending), unit columns of the rotated R^T (zero where Sigma is zero).
// last: this is the mode's last small SVD, whose deficient-column count goes
// to info->deficient[mode] (the others only set their step's bit).
hipError_t launch_orth_svd(int l, tucker_precision prec, const OrthWs& ws, double* sigma, double* alpha,
                           tucker_info* info, int mode, int step, hipStream_t st, const SvdPve* pve = nullptr,
                           double* vright = nullptr, bool last = true);
// Q = Q3 Wm to q_out (n x l, `prec` storage), qt (j-major l x n, `prec`
// storage) and q64 (n x l, FP64), each when not nullptr.
hipError_t launch_orth_rotate(int64_t n, int l, const OrthWs& ws, tucker_precision prec, void* q_out, void* qt,
                              double* q64, hipStream_t st);
// [Q, Sigma] = svd(Y, econ): launch_orth_qr + launch_orth_svd + launch_orth_rotate on one stream.
hipError_t launch_orth(int64_t n, int l, double* Y, tucker_precision prec, void* q_out, void* qt,
                       double* q64, double* sigma, double* alpha, tucker_info* info, int mode, int step,
                       const OrthWs& ws, uint64_t cseed, hipStream_t st);

// U[:, j] = sign_j * Q[:, j] for j < r (Q FP64 n x l): each column's
// largest-magnitude entry made positive (lowest row index on ties). U is
// n x r and Ut (when not nullptr) j-major r x n, both in `prec` storage.
hipError_t launch_signfix(tucker_precision prec, const double* Q, int64_t n, int l, int r, void* U, void* Ut,
                          hipStream_t st);

// Mode unfolding of X (view v, storage prec) in FP64: trans ? m x n : n x m
// (m = P S, columns in row-major order over the other modes).
hipError_t launch_unfold64(tucker_precision prec, const View3& v, const void* X, bool trans, double* Y,
                           hipStream_t st);
// The sign rule in place on every column of Q (FP64 n x l), and Qt = Q^T
// j-major (l x n) in `prec` storage.
hipError_t launch_signcols(tucker_precision prec, double* Q, int64_t n, int l, void* Qt, hipStream_t st);
// U = (Q V(:, 0:r)) S and Vt = (V(:, 0:r) S)^T j-major (r x l), S the sign
// rule of launch_signfix applied to Q V; Q FP64 n x l, V FP64 l x ldv.
hipError_t launch_assemble(tucker_precision prec, const double* Q, int64_t n, int l, const double* V, int ldv, int r,
                           void* U, void* Vt, hipStream_t st);

// Small helpers.
hipError_t launch_convert_to_f64(tucker_precision prec, const void* src, int64_t count, double* dst,
                                 hipStream_t st);
// dst (FP64, or FP32 for the other precisions) = src rounded to nearest.
hipError_t launch_convert_from_f64(tucker_precision prec, const double* src, int64_t count, void* dst,
                                   hipStream_t st);
hipError_t launch_info_init(tucker_info* info, const int32_t* l, int d, int32_t flags, hipStream_t st);
// *alpha = 0 (alpha may be null) and *ctr = 0: a mode's start, before its
// first fused power step.
hipError_t launch_mode_start(double* alpha, int* ctr, hipStream_t st);

// ---- batched persistent launches (many small solves at once) --------------
// A batched phase is one launch of a fixed grid whose workgroups loop over
// the phase's work items: hdr[0] = number of requests, hdr[1 + b] = first
// work item of request b (prefix sums, hdr[1 + nreq] = total), desc[b] = the
// arguments of request b. Work item w of request b runs the same workgroup
// body as a single-request launch with block index w - hdr[1 + b]. All FP32
// storage; lclass (16, 32, 48 or 64) fixes the tile templates for l <= lclass.
struct BInit {
  tucker_info* info;
  double* alpha;  // d shifts, set to 0
  int32_t l[TUCKER_MAX_ORDER];
  int32_t d, flags;
};
struct BFill {
  float* out;
  uint64_t seed;
  int64_t rows, ld;
  uint32_t mode;
  int32_t cols;
};
struct BCrSplit {
  const float* X;
  const float* Bt;
  float* part;
  int64_t n, S, m, spp, nsteps;
  int32_t l, nsplit, nrb;
};
struct BCrCols {
  const float* X;
  const float* Bt;
  float* part;
  int64_t P, n, nsteps;
  int32_t l, nsplit, nrb;
};
struct BReduce {
  const float* part;
  const double* qsub;
  const double* alpha;
  double* Y;
  int64_t nl;
  int32_t nsplit;
};
struct BRcSplit {
  const float* X;
  const float* W;
  float* out;
  int64_t n, S, wsi, wsj, tpp, ntiles, osp, osj;
  int32_t lw;
};
struct BRcCols {
  const float* X;
  const float* W;
  float* out;
  int64_t P, n, wsi, wsj, osp, osj;
  int32_t lw;
};
struct BGram {
  double* Y;
  const double* Wm;
  double* part;
  int* status;
  int64_t n;
  int32_t l;
};
struct BPass {
  const double* Qin;
  const double* part_in;
  double* Qout;
  void* qt;
  double* part_out;
  double* Rg;
  int* defic;
  int* status;
  uint64_t cseed;
  double tau, shift_scale, eps3;
  int64_t n;
  int32_t l, nblk, role;
  uint32_t ctag;
};
struct BSvd {
  const double* Rg;
  const int* status;
  double* Wm;
  double* sigma;
  double* alpha;
  tucker_info* info;
  double tol, negl;
  int32_t l, mode, step;
};
struct BRotate {
  const double* Q3;
  const double* Wm;
  double* q64;
  int64_t n;
  int32_t l;
};
struct BSignfix {
  const double* Q;
  float* U;
  float* Ut;
  int64_t n;
  int32_t l, r;
};
enum BatchKind {
  BK_INIT = 0, BK_FILL, BK_CR_SPLIT, BK_CR_COLS, BK_REDUCE, BK_RC_SPLIT, BK_RC_COLS,
  BK_GRAM, BK_PASS, BK_SVD, BK_ROTATE, BK_SIGNFIX, BK_COUNT
};
size_t batch_desc_bytes(BatchKind kind);
hipError_t launch_batch_ttm(BatchKind kind, int lclass, int* hdr, const void* desc, hipStream_t st);
hipError_t launch_batch_orth(BatchKind kind, int lclass, int* hdr, const void* desc, hipStream_t st);
// Work items (workgroups) of one request for the geometry-driven kinds.
int64_t cr_split_items(int64_t n, int nsplit);
int64_t cr_cols_items(int64_t n, int nsplit);
void cr_geometry(const View3& v, int64_t* nsteps, int64_t* spp, int* nrblocks);
void cr_split_geometry(const View3& v, int64_t* nsteps, int64_t* spp, int* nrblocks);
int64_t rc_split_tiles(const View3& v, int64_t* tpp);

}  // namespace tk
