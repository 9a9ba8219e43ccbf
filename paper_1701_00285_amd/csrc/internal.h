// Internal data structures of the multilevel BLUP library (host side).
#pragma once

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mlblup.h"

namespace mlb {

// Thread-local last error message; returns the status for `return fail(...)`.
int fail(int status, const std::string& msg);
void clear_error();

struct Tree {
  int64_t n = 0;
  int32_t d = 0;
  int32_t leaf_max = 0;
  std::vector<double> pts;        // input points, row-major n x d
  std::vector<int64_t> perm;      // tree position -> input index
  // nodes in preorder
  std::vector<int64_t> begin, end;
  std::vector<int32_t> depth, axis, left, right, parent;
  std::vector<double> threshold;
  int32_t max_depth = 0;
  int32_t n_nodes() const { return (int32_t)begin.size(); }
  bool leaf(int32_t v) const { return left[v] < 0; }
};

int build_tree(const double* pts, int64_t n, int32_t d, int32_t leaf_max, Tree& t);

// Per-node record of the device transform schedule.  `in_off` is the start
// of the node's candidate coefficients: for a leaf, its first tree position
// in the N-vector; for an internal node, the scaling slot of its left child
// (siblings' slots are contiguous).  `scal_off` is the node's own scaling
// slot (-1 at the root, whose scaling coefficients are L v).
struct NodeDesc {
  int64_t in_off;
  int64_t scal_off;
  int64_t w_off;     // first wavelet coefficient in W v
  int64_t v_off;     // offset (doubles) of the m x m block in the V array
  int32_t m;
  int32_t a;
  int32_t leaf;
  int32_t nref;      // Householder reflectors of V = H_0 ... H_{nref-1}: min(m, p)
  int64_t h_off;     // offset (doubles) in H: V = I - Y T Y^T, Y (nref rows of m), then T (nref x nref)
};

struct Basis {
  int64_t n = 0;
  int32_t d = 0;
  int32_t w = 0;
  int32_t p = 0;
  int32_t levels = 0;             // max depth + 1
  std::vector<std::vector<int32_t>> exps;   // p exponent tuples, graded lex
  // per node (preorder index)
  std::vector<NodeDesc> desc;
  std::vector<double> V;          // row-major m x m blocks, V[i*m + j] = column j (candidate i)
  // the same blocks as products of Householder reflectors V = H_0 H_1 ... H_{K-1}, H_k = I - tau_k h_k h_k^T,
  // in compact WY form V = I - Y T Y^T: per node the K reflectors h_k of length m (zero above k, 1 at
  // k) as the rows of Y, then the upper triangular K x K T (T_kk = tau_k), row-major
  std::vector<double> H;
  std::vector<int64_t> level_counts;   // wavelets per level q
  // device schedule: node ids grouped by level, level q in [lvl_begin[q], lvl_begin[q+1])
  std::vector<int32_t> level_nodes;
  std::vector<int32_t> lvl_begin;
  int64_t scal_total = 0;         // length of the scaling scratch
  // tree copy needed later
  std::vector<double> pts_tree;   // points in tree order, row-major
  std::vector<int64_t> begin, end;   // node point ranges (tree order)
  std::vector<int32_t> left, right;  // children (-1 for leaves)
  std::vector<int32_t> depth, axis;  // node depth; split axis (-1 for leaves)
  std::vector<double> threshold;     // split threshold: x_axis <= threshold goes left
  // trend: root frame (centre, scale) and L X_loc = Ms^T (p x p) for beta
  std::vector<double> root_c;
  double root_h = 1.0;
  std::vector<double> root_moments;   // Ms (p x p), row-major: Ms[beta][j]
  // device image
  void* dev_base = nullptr;
  int64_t dev_bytes = 0;
  // offsets inside the device image (bytes)
  int64_t off_desc = 0, off_V = 0, off_H = 0, off_pts = 0, off_levels = 0, off_exps = 0;
  int64_t off_rootc = 0;      // root-frame centre (d doubles, 256-byte aligned)
  int64_t off_children = 0;   // left, then right child of every node (-1 for leaves): 2 x nodes int32
  bool uploaded = false;
};

int build_basis(const Tree& t, int32_t w, double rank_rtol, Basis& b);

// Sparsity pattern of C~^n_W (Sec. 4.1): the cells with wavelets at levels
// >= level, each row's cell, and a symmetric cell-pair keep matrix.
struct Pattern {
  int32_t nc = 0;                  // cells
  std::vector<int32_t> rowcell;    // N~: cell of every row of C^n_W
  std::vector<uint8_t> keep;       // nc x nc, 1 = block kept
  int64_t nnz = 0;                 // kept entries of the N~ x N~ matrix
};
int32_t pattern_cells(const Basis& b, int32_t level);
void build_pattern(const Basis& b, int32_t level, double tau, Pattern& P);

// Block structure of the sparse Cholesky factor of C~^n_W (one block row and
// column per cell with wavelets at levels >= level), in elimination order
// (positions 0 .. nc-1), and the cells' wavelet vectors on their points.
constexpr int32_t kSparseMaxBlock = 64;   // wavelets per cell handled by the block kernels
struct SparseSymbolic {
  int32_t level = -1;
  double tau = 0.0;
  int32_t nc = 0;                  // block columns
  int64_t rows = 0;                // N~
  int64_t kept_entries = 0;        // entries of C~^n_W kept by the pattern
  int64_t factor_entries = 0;      // doubles of the block factor (full diagonal blocks)
  double flops = 0.0;              // factorization flops of the block structure
  std::vector<int32_t> order;      // position -> cell (the pattern's row order of cells)
  std::vector<int32_t> node;       // position -> basis node
  std::vector<int32_t> w;          // position -> wavelets (block size)
  std::vector<int64_t> row0;       // position -> first row of the cell in C^n_W
  std::vector<int64_t> ypos;       // position -> offset of its block in the position-ordered vectors
  // blocks, column by column: the diagonal block, then the blocks below in ascending row position;
  // block b is w[blk_row] x w[blk_col], row-major, at blk_off[b] doubles
  std::vector<int64_t> col_ptr;
  std::vector<int32_t> blk_row, blk_col;
  std::vector<int64_t> blk_off;
  std::vector<uint8_t> blk_kept;   // 1: a kept block of C~^n_W (assembled); 0: fill (starts at zero)
  // row structure: for column j, entries row_ptr[j] .. row_ptr[j+1]: earlier column k (ascending)
  // and the block (j, k)
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> row_col;
  std::vector<int64_t> row_blk;
  // dense tail: the columns [tail, nc) (tail_rows rows) are factored as one dense matrix after the
  // block columns before them have updated it (tail = nc: none)
  int32_t tail = 0;
  int64_t tail_rows = 0;
  double flops_tail = 0.0;         // tail_rows^3 / 3
  std::vector<int64_t> tail_blks;  // the blocks of the tail columns
  std::vector<int32_t> tail_cols;  // tail .. nc - 1
  // elimination-tree heights of the columns before the tail: the columns of height h and their blocks
  std::vector<int64_t> lvl_ptr;
  std::vector<int32_t> lvl_cols;
  std::vector<int64_t> lvl_blk_ptr;
  std::vector<int64_t> lvl_blks;
  // wavelet vectors of each position's cell on its points (tree order), |S| x w row-major
  std::vector<int64_t> psi_off;
  std::vector<double> psi;
};
// dense_tail: -1 chooses the tail start by the estimated time (block columns at kSparseBlockRate plus
// kSparseHeightTime per elimination-tree height, the dense tail at kSparseDenseRate) among the tails
// of at most max_tail rows, 0 .. nc forces it (nc: no dense tail).  The three constants are a least
// squares fit to timings of 12 tail positions at 65,536 and 262,144 points on one MI355X.
constexpr double kSparseBlockRate = 22e12;    // flop/s of the block kernels
constexpr double kSparseHeightTime = 0.77e-3; // s per height (its three launches, their serial depth)
constexpr double kSparseDenseRate = 38e12;    // flop/s of the dense blocked Cholesky
constexpr int64_t kSparseMaxTail = 49152;     // rows of the dense tail at most (18 GB)
int sparse_analyse(const Basis& b, int32_t level, double tau, SparseSymbolic& S, int32_t dense_tail = -1,
                   int64_t max_tail = kSparseMaxTail);
int64_t basis_device_bytes(const Basis& b);

// exponent tuples of the total-degree set, graded lexicographic
std::vector<std::vector<int32_t>> td_exponents(int32_t d, int32_t w);

}  // namespace mlb

struct mlblup_tree_s {
  mlb::Tree t;
};
struct mlblup_basis_s {
  mlb::Basis b;
  // the last sparse analysis (level, tau) of the estimator, reused by later evaluations
  std::mutex sparse_mu;
  std::shared_ptr<const mlb::SparseSymbolic> sparse;
  int sparse_req = -1;   // dense-tail request the cached analysis was built with
  int64_t sparse_cap = mlb::kSparseMaxTail;   // and its row limit
};
