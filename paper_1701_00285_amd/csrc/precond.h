// Preconditioner (diag(C_W) or its per-cell blocks): device-side helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.h"

namespace mlb {

struct PrecNode {
  int64_t begin, end;   // point range (tree order)
  int64_t v_off;        // V block offset
  int32_t m, a;
  int32_t left, right;  // children (-1 for leaves)
};

struct CrossTask {
  int64_t r0, r1, c0, c1;
};

int prec_leaf_blocks(const int64_t* lbegin, const int32_t* lsize, const int64_t* koff, int32_t nleaves,
                     const double* pts, int d, double zs, int nu2, const float* g32, double* K, hipStream_t s);
int prec_scal_values(const PrecNode* nodes, const int32_t* lvl, int32_t cnt, const double* V, const double* phi_in,
                     double* phi_out, int P, int64_t n, hipStream_t s);
int prec_zero(double* p, int64_t n, hipStream_t s);
int prec_cross(const CrossTask* tasks, int32_t ntasks, int NR, const double* pts, int d, double zs, int nu2,
               const float* g32, const double* phi, int P, double* part, hipStream_t s);
int prec_apply_blocks(const int64_t* w_off, const int32_t* mw, const int64_t* boff, int32_t cnt, const double* Binv,
                      const double* r, double* z, hipStream_t s);
int prec_apply_diag(const double* inv, const double* r, double* z, int64_t n, hipStream_t s);
// tri: 0 full, 1 lower triangular, 2 upper triangular (the other triangle holds exact zeros, not read)
int prec_gemv_rows(const float* M, int64_t n, int64_t ld, const double* x, double* out, hipStream_t s, int tri = 0);

// Host-side preconditioner object.
struct Precond {
  int32_t kind = 0;              // MLBLUP_PREC_JACOBI, MLBLUP_PREC_BLOCK or MLBLUP_PREC_COARSE
  int64_t nw = 0;
  // blocks B_v of C_W per cell (host, row-major mw x mw) and their inverses
  std::vector<int32_t> node;     // cells with mw > 0
  std::vector<int64_t> w_off;
  std::vector<int32_t> mw;
  std::vector<int64_t> boff;
  std::vector<double> blocks;    // B_v
  std::vector<double> inv;       // block inverses (block kind) or 1/diag (Jacobi, nw entries)
  // coarse kind: the rows [c0, c0 + nc) of the coarse levels form one block
  // C_c with C_c^-1 = Y X, Y = G^-T and X = G^-1 (nc x nc row-major each);
  // the cell blocks above cover only the rows < c0.  The device image holds
  // Y and X rounded to FP32 (X32 = Y32^T exactly, so Y32 X32 stays symmetric
  // positive definite: a fixed preconditioner of the same quality at half the
  // bytes of each apply)
  int64_t c0 = 0, nc = 0, ldc = 0;   // ldc: row stride of Y32 and X32 (nc rounded up to 4, zero padding)
  std::vector<double> ycoarse;
  std::vector<float> y32, x32;
  // device image (caller-owned)
  void* dev = nullptr;
  int64_t dev_bytes = 0;
  int64_t off_woff = 0, off_mw = 0, off_boff = 0, off_inv = 0, off_y = 0, off_x = 0;
  bool uploaded = false;
};

int precond_workspace_bytes(const Basis& B, int64_t* bytes);
// rows of the coarse block of the coarse kind: every level above the finest
void coarse_rows(const Basis& B, int64_t* c0, int64_t* nc);
// nu: the smoothness (+inf for the Gaussian; any 0 < nu <= 8)
int precond_build(const Basis& B, double nu, double rho, double sigma2, int kind, void* work, int64_t work_bytes,
                  hipStream_t s, Precond& P);
int precond_apply(const Precond& P, const double* r, double* z, hipStream_t s);

}  // namespace mlb

struct mlblup_precond_s {
  mlb::Precond p;
};
