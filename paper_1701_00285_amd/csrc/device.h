// Launchers of the device kernels (HIP, gfx950).  All launches go on the
// caller's stream; none allocates memory.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include <cstdint>
#include <functional>

#include "internal.h"

namespace mlb {

// hipError_t -> status with a message naming the call
int hip_check(hipError_t e, const char* what);
#define MLB_HIP(call)                                  \
  do {                                                 \
    int _st = ::mlb::hip_check((call), #call);         \
    if (_st != MLBLUP_OK) return _st;                  \
  } while (0)

// ---- pair kernel -------------------------------------------------------------
struct PairArgs {
  const double* rows;
  int64_t m;
  const double* cols;
  int64_t n;
  int32_t d;
  int32_t nu2;        // 2 nu: 1, 3 or 5
  double rho;
  double sigma2;
  int32_t precision;  // MLBLUP_FP64 ...
  int32_t outputs;    // MLBLUP_VALUE | MLBLUP_DLOGRHO
  const double* x;
  double* y;
  double* dy;
  double nu = 0.0;                // the smoothness itself (general nu)
  const double* gtab = nullptr;   // general-nu table on the device (set by pair_launch)
};

// nu2 code of a general smoothness (0 < nu <= 8, not a half-integer): the
// FP64 kernels evaluate it from a table (genu.h)
constexpr int kNuGeneral = -2;
// host copy of the general-nu table for nu (built once, kept for the process); NULL if nu is out of range
const double* genu_table_cached(double nu);

// Number of column splits (partial sums per row) used for an m x n product.
int32_t pair_splits(int64_t m, int64_t n, int32_t d, int32_t precision);
// Workspace bytes for the partial sums.
int64_t pair_workspace_bytes(int64_t m, int64_t n, int32_t d, int32_t precision, int32_t outputs);
// Symmetric square product (pair_sym.hip): each unordered pair once.
// tile launcher of a symmetric schedule: (T blocks, first round, rounds, diagonal?, partial buffers)
using SymTileLaunch = std::function<void(int, int, int, int, double*, double*, double*, double*)>;
// deterministic tournament schedule over blocks of blk_pts points (pair_sym.hip);
// rows_summed: the off-diagonal launches write one row partial for all their
// rounds (slot 0) instead of one per round; diag_splits: column ranges per
// diagonal tile (0: the default 4; at most 4)
int sym_schedule(const PairArgs& a, int blk_pts, void* work, hipStream_t s, const SymTileLaunch& fn,
                 bool rows_summed = false, int diag_splits = 0);
bool sym_supported(int d);
// the compiled dimension of the pair kernels that a point set of dimension d runs in: its coordinates
// are padded with zeros, which changes no distance or norm (0 past 32: no compiled kernel)
constexpr int padded_dim(int d) {
  return d <= 6 ? d : d <= 8 ? 8 : d <= 10 ? 10 : d <= 16 ? 16 : d <= 20 ? 20 : d <= 24 ? 24 : d <= 28 ? 28 : d <= 32 ? 32 : 0;
}
bool sym_worthwhile(int64_t n);
int64_t sym_workspace_bytes(int64_t n, int outputs);
int sym_launch(const PairArgs& a, double zs, void* work, hipStream_t s);
// Matrix-core distance Gram (pair_mfma.hip): MFMA precisions, value only, 8 <= d <= 32.
bool mfma_applies(const PairArgs& a);
// 2 nu of a covariance: 1, 3, 5 (half-integer Matern), 0 for nu = +inf, the
// Gaussian exp(-r^2 / (2 rho^2)) (the Matern limit in the sqrt(2 nu) r / rho
// parametrisation), kNuGeneral for any other 0 < nu <= 8; -1 otherwise
int nu2_of_nu(double nu);
// scale applied to the coordinates: sqrt(2 nu) / rho, or 1 / rho for the Gaussian
inline double kernel_scale(int nu2, double nu, double rho) {
  if (nu2 == 0) return 1.0 / rho;
  if (nu2 == kNuGeneral) return std::sqrt(2.0 * nu) / rho;
  return std::sqrt((double)nu2) / rho;
}
int32_t mfma_splits(int64_t m, int64_t n);
int mfma_launch(const PairArgs& a, double zs, double* part, hipStream_t s);
// square products (n >= 16,384): each unordered pair once, tournament schedule
int mfma_sym_launch(const PairArgs& a, double zs, void* work, hipStream_t s);
// Validates and launches (pair kernel + split reduction).
int pair_launch(const PairArgs& a, void* work, int64_t work_bytes, hipStream_t s);
// multilevel predictor with P C P^T and K P^T formed in double-double (small N;
// P = [W; L] dense, n x n row-major on the host).  info_host: iterations,
// breakdown flag, recurrence relres, true relres of the FP64 CG on C_W.
constexpr int64_t kDdMaxN = 4096;
int64_t dd_workspace_bytes(int64_t n, int64_t mt);
int dd_blup_predict(const Basis& B, const std::vector<double>& P_host, int nu2, double nu, double rho, double sigma2,
                    const double* z_dev, const double* tgt_dev, const double* tgt_host, int64_t mt, double rtol,
                    int32_t max_iter, double* zhat_dev, double* beta_host, double* cw_dev, double* info_host,
                    void* work, int64_t work_bytes, hipStream_t s);
// pair_launch on the library's static per-device scratch (no allocation)
int pair_launch_noalloc(const PairArgs& a, hipStream_t s);

// ---- multilevel transform ------------------------------------------------------
struct TransformDev {
  const NodeDesc* desc;
  const int32_t* level_nodes;
  const int32_t* lvl_begin_host;   // host array (levels + 1)
  int32_t levels;
  const double* V;     // dense m x m blocks (cells too large for the reflector form)
  const double* H;     // Householder reflectors and scales of every cell (NodeDesc::h_off)
  const int32_t* children = nullptr;  // left children (n_nodes), then right children; -1 for leaves
  int32_t n_nodes = 0;
};
// cells of up to kTransformMaxM candidates apply V as its reflectors (one 64-lane wave, up to 4
// entries per lane); larger ones read the dense m x m block
constexpr int32_t kTransformMaxM = 256;
// doubles one transform reads for a cell: the compact WY form (K reflectors of length m and the
// K x K triangle, stored full), or the m x m block
inline int64_t transform_node_doubles(const NodeDesc& D) {
  return D.m <= kTransformMaxM ? (int64_t)D.nref * D.m + (int64_t)D.nref * D.nref : (int64_t)D.m * D.m;
}
// vw = W v, vl = L v (vl may be null).  scal: scaling scratch.
int transform_analysis(const TransformDev& T, const double* v, double* vw, double* vl, double* scal,
                       hipStream_t s);
// v = W^T vw + L^T vl (vl may be null => 0).
int transform_synthesis(const TransformDev& T, const double* vw, const double* vl, double* v, double* scal,
                        hipStream_t s);

// ---- multilevel log-likelihood (loglik.hip) ----------------------------------------
// workspace layout (byte offsets) for the levels >= level
// device view of the multilevel transform of an uploaded basis
TransformDev transform_dev(const Basis& B);

struct LoglikLayout {
  int64_t phi = 0, a = 0, scal = 0, zw = 0, scalz = 0, out = 0, flag = 0, gtab = 0, linv = 0, total = 0;
  int64_t rowcell = 0, keep = 0;   // sparsity pattern of C~^n_W: cell of each row, cell-pair keep matrix
  int64_t rows = 0;    // N~: rows of [W_t; ...; W_level]
  int32_t cells = 0;   // cells with wavelets at levels >= level
  int64_t batch = 0;   // columns per batched-analysis pass
};
int64_t loglik_rows(const Basis& B, int32_t level);
LoglikLayout loglik_layout(const Basis& B, int32_t level);
// coarse block of C_W (rows [c0, c0 + nc) of W) for the preconditioner
struct CoarseLayout {
  int64_t phi = 0, a = 0, scal = 0, flag = 0, gtab = 0, linv = 0, total = 0, batch = 0;
};
CoarseLayout coarse_layout(const Basis& B, int64_t nc);
// Dense blocked Cholesky of the nt x nt lower triangle of C (row-major, ld nt) with row nt as a border
// row (C holds (nt + 1) x nt doubles): dout = {2 sum log G_ii, |G^-1 c|^2}, c the border row; linv:
// dense_cholesky_linv_doubles(nt) doubles; a pivot that is not positive sets flag[0] (loglik.hip)
int dense_cholesky_logdet(double* C, int64_t nt, double* linv, int* flag, double* dout, hipStream_t s);
int64_t dense_cholesky_linv_doubles(int64_t nt);
// sparse block Cholesky of C~^n_W (sparse_chol.hip): workspace layout (byte offsets) for a host analysis
struct SparseLayout {
  int64_t L = 0, linv = 0, psi = 0, zw = 0, scal = 0, zt = 0, y = 0, logd = 0, out = 0, flag = 0, gtab = 0;
  int64_t w = 0, row0 = 0, ypos = 0, inv_off = 0, sup_beg = 0, sup_cnt = 0, psi_off = 0, col_ptr = 0;
  int64_t blk_row = 0, blk_col = 0, blk_off = 0, row_ptr = 0, row_col = 0, row_blk = 0, lvl_blks = 0;
  int64_t lvl_cols = 0, kept = 0, total = 0, nkept = 0;
  int64_t dense = 0, dense_linv = 0, dense_out = 0, tail_blks = 0, tail_cols = 0;   // the dense tail
};
SparseLayout sparse_layout(const Basis& B, const SparseSymbolic& S);
// out = {l~, log det, quadratic form}; MLBLUP_EBREAKDOWN for a pivot that is not positive
int loglik_sparse_device(const Basis& B, const TransformDev& T, const PairArgs& k, const SparseSymbolic& S,
                         const double* z, void* work, const SparseLayout& Ly, double out[3], hipStream_t s);
// Y = G^-T (nc x nc row-major, host) with G G^T = (W C W^T)[c0:c0+nc, c0:c0+nc]
int coarse_inverse_factor(const Basis& B, const PairArgs& k, int64_t c0, int64_t nc, void* work, int64_t work_bytes,
                          std::vector<double>& Y, hipStream_t s);
// copies the pattern (built for the same level) into the workspace; synchronises s
int loglik_upload_pattern(const Pattern& P, void* work, const LoglikLayout& L, hipStream_t s);
// out = {l, log det C^n_W, (Z^n_W)^T (C^n_W)^-1 Z^n_W}; k supplies nu2, nu, rho, sigma2.
// masked: zero the blocks the uploaded pattern drops (C~^n_W in place of C^n_W)
int loglik_device(const Basis& B, const TransformDev& T, const PairArgs& k, int32_t level, const double* z,
                  void* work, const LoglikLayout& L, bool masked, double out[3], hipStream_t s);

// ---- vector kernels (deterministic FP64 reductions) -------------------------------
constexpr int kRedBlocks = 512;   // fixed partial count of every reduction

// scalars kept on the device by the Krylov loop
enum Scal { S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_RZNEW, S_FLAG, S_DOT, S_COUNT = 16 };

int vec_dot(const double* a, const double* b, int64_t n, double* part, double* out_dev, hipStream_t s);
int vec_copy(const double* a, double* b, int64_t n, hipStream_t s);
int vec_zero(double* a, int64_t n, hipStream_t s);
// b = a - b  (residual r = z - Cx when b holds Cx); partial |b|^2 into out_dev
int vec_sub_from(const double* a, double* b, int64_t n, hipStream_t s);
int vec_axpy(double alpha, const double* x, double* y, int64_t n, hipStream_t s);    // y += alpha x
// PCG pieces
int pcg_alpha(const double* p, const double* q, int64_t n, double* part, double* sc, hipStream_t s);
// x += alpha p, r -= alpha q, partial |r|^2 into part[0 .. kRedBlocks)
int pcg_update_xr(double* x, double* r, const double* p, const double* q, int64_t n, double* part, double* sc,
                  hipStream_t s);
// partial r.z into part[kRedBlocks .. 2 kRedBlocks)
int pcg_rz_partial(const double* r, const double* z, int64_t n, double* part, hipStream_t s);
// sc[S_RR] = |r|^2, beta = rz_new / rz (rz = |r|^2 without preconditioner)
int pcg_finish_beta(double* part, bool has_z, double* sc, hipStream_t s);
// part[0..) = partial sums of r.r (the layout pcg_update_xr leaves)
int pcg_rr_partial(const double* r, int64_t n, double* part, hipStream_t s);
// as pcg_finish_beta, with beta = r.z / rz_prev for a given previous r.z
int pcg_finish_beta_from(double* part, bool has_z, double rz_prev, double* sc, hipStream_t s);
int pcg_update_p(double* p, const double* z, int64_t n, const double* sc, hipStream_t s);
// flexible-CG direction: p = z - (z.q_prev / p_prev.q_prev) p  (sc[S_DOT] = z.q_prev, sc[S_PQ])
int fcg_update_p(double* p, const double* z, int64_t n, const double* sc, hipStream_t s);
// set sc[S_RZ] = r.z (start of an inner solve)
int pcg_start(const double* r, const double* z, int64_t n, double* part, double* sc, hipStream_t s);
// z = r / diag
int vec_div(const double* r, const double* diag, double* z, int64_t n, hipStream_t s);

// trend at targets: out[i] += sum_b beta[b] prod_k ((t_ik - c_k)/h)^e_bk
int trend_add(const double* tgt, int64_t m, int32_t d, const int32_t* exps, int32_t p, const double* c, double h,
              const double* beta, double* out, hipStream_t s);

// ---- instrumentation -------------------------------------------------------
void profile_note(hipEvent_t a, hipEvent_t b, double pairs, int bucket);
bool profile_on();
// While one lives on a thread, profile_on() is false there: the timing
// events (hipEventCreate) stay out of calls that must not allocate.
struct ProfileSuppress {
  ProfileSuppress();
  ~ProfileSuppress();
  ProfileSuppress(const ProfileSuppress&) = delete;
  ProfileSuppress& operator=(const ProfileSuppress&) = delete;
 private:
  bool prev_;
};

}  // namespace mlb
