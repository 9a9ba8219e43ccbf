// Host driver of the preconditioner build (see precond.hip for the method):
// task decomposition, level sweep on the device, bottom-up block assembly
// and inversion on the host, device image.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>

#include "device.h"
#include "genu.h"
#include "precond.h"


namespace mlb {
namespace {

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int nr_for(int p) {
  for (int c : {8, 16, 24, 32})
    if (p <= c) return c;
  return -1;
}

constexpr int64_t kRowsPerTask = 256;

std::vector<CrossTask> level_tasks(const Basis& B, int q) {
  std::vector<CrossTask> t;
  for (int32_t s = B.lvl_begin[q]; s < B.lvl_begin[q + 1]; ++s) {
    const int32_t v = B.level_nodes[s];
    if (B.left[v] < 0) continue;
    const int32_t L = B.left[v], R = B.right[v];
    const int64_t rl = B.end[L] - B.begin[L], cr = B.end[R] - B.begin[R];
    const int64_t rchunks = (rl + kRowsPerTask - 1) / kRowsPerTask;
    int64_t splits = (2048 + rchunks - 1) / rchunks;
    splits = std::max<int64_t>(1, std::min<int64_t>(splits, (cr + 2047) / 2048));
    const int64_t cchunk = (cr + splits - 1) / splits;
    for (int64_t r = 0; r < rchunks; ++r)
      for (int64_t c = 0; c < splits; ++c) {
        CrossTask T;
        T.r0 = B.begin[L] + r * kRowsPerTask;
        T.r1 = std::min(B.end[L], T.r0 + kRowsPerTask);
        T.c0 = B.begin[R] + c * cchunk;
        T.c1 = std::min(B.end[R], T.c0 + cchunk);
        if (T.c0 < T.c1) t.push_back(T);
      }
  }
  return t;
}

struct WsLayout {
  int64_t nodes, lbegin, lsize, koff, K, phi0, phi1, tasks, part, gtab, total;
  int64_t max_tasks, k_entries;
  int32_t nleaves;
  int NR;
};

WsLayout layout(const Basis& B) {
  WsLayout w{};
  w.NR = nr_for(B.p);
  const int64_t nn = (int64_t)B.desc.size();
  int64_t ke = 0, nl = 0;
  for (int64_t v = 0; v < nn; ++v)
    if (B.left[v] < 0) {
      ke += (int64_t)B.desc[v].m * B.desc[v].m;
      ++nl;
    }
  w.k_entries = ke;
  w.nleaves = (int32_t)nl;
  int64_t mt = 0;
  for (int q = 0; q < B.levels; ++q) mt = std::max<int64_t>(mt, (int64_t)level_tasks(B, q).size());
  w.max_tasks = mt;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off = align_up(off + std::max<int64_t>(bytes, 8));
    return o;
  };
  const int NR = std::max(w.NR, 8);
  w.nodes = take(nn * (int64_t)sizeof(PrecNode));
  w.lbegin = take(nl * 8);
  w.lsize = take(nl * 4);
  w.koff = take(nl * 8);
  w.K = take(ke * 8);
  w.phi0 = take(B.n * NR * 8);
  w.phi1 = take(B.n * NR * 8);
  w.tasks = take(mt * (int64_t)sizeof(CrossTask));
  w.part = take(mt * NR * NR * 8);
  w.gtab = take(kGenuBytes);
  w.total = off;
  return w;
}

// y = A x for small row-major matrices
void gemm_tn(int m, int a0, int a, const double* V, const double* G, int Gld, double* out) {
  // out (a x a) = V[:, a0:a0+a]^T G V[:, a0:a0+a], V is m x m row-major, G is m x m (ld Gld)
  std::vector<double> T((size_t)m * a, 0.0);  // T = G V_sub
  for (int i = 0; i < m; ++i)
    for (int k = 0; k < m; ++k) {
      const double g = G[(size_t)i * Gld + k];
      if (g == 0.0) continue;
      const double* vr = V + (size_t)k * m + a0;
      double* tr = &T[(size_t)i * a];
      for (int j = 0; j < a; ++j) tr[j] += g * vr[j];
    }
  for (int r = 0; r < a; ++r)
    for (int c = 0; c < a; ++c) out[(size_t)r * a + c] = 0.0;
  for (int i = 0; i < m; ++i) {
    const double* vr = V + (size_t)i * m + a0;
    const double* tr = &T[(size_t)i * a];
    for (int r = 0; r < a; ++r) {
      const double vv = vr[r];
      if (vv == 0.0) continue;
      double* orow = out + (size_t)r * a;
      for (int c = 0; c < a; ++c) orow[c] += vv * tr[c];
    }
  }
}

// inverse of an SPD matrix via Cholesky; false if not positive definite
bool spd_inverse(int n, const double* A, double* out) {
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0)) return false;
    const double ljj = std::sqrt(s);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / ljj;
    }
  }
  // inv(L) by forward substitution, then inv(A) = inv(L)^T inv(L)
  std::vector<double> Li((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    for (int i = c; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) t -= L[(size_t)i * n + k] * Li[(size_t)k * n + c];
      Li[(size_t)i * n + c] = t / L[(size_t)i * n + i];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      double t = 0.0;
      for (int k = std::max(r, c); k < n; ++k) t += Li[(size_t)k * n + r] * Li[(size_t)k * n + c];
      out[(size_t)r * n + c] = t;
    }
  return true;
}

}  // namespace

int precond_workspace_bytes(const Basis& B, int64_t* bytes) {
  if (nr_for(B.p) < 0) return fail(MLBLUP_EINVAL, "preconditioner: trend dimension p > 32 not supported");
  *bytes = layout(B).total;
  return MLBLUP_OK;
}

void coarse_rows(const Basis& B, int64_t* c0, int64_t* nc) {
  const int64_t f = B.levels > 0 ? B.level_counts[B.levels - 1] : 0;   // the finest level's rows come first
  *c0 = f;
  *nc = (B.n - B.p) - f;
}

int precond_build(const Basis& B, double nu, double rho, double sigma2, int kind, void* work, int64_t work_bytes,
                  hipStream_t s, Precond& P) {
  const WsLayout w = layout(B);
  if (w.NR < 0) return fail(MLBLUP_EINVAL, "preconditioner: trend dimension p > 32 not supported");
  if (!work || work_bytes < w.total)
    return fail(MLBLUP_EINVAL, "preconditioner workspace too small (need " + std::to_string(w.total) + ")");
  const int nu2 = nu2_of_nu(nu);
  if (nu2 == -1) return fail(MLBLUP_EINVAL, "preconditioner: nu must be in (0, 8] or +inf");
  const double zs = kernel_scale(nu2, nu, rho);
  const int32_t nn = (int32_t)B.desc.size();
  char* base = (char*)work;
  const char* img = (const char*)B.dev_base;
  const double* pts = (const double*)(img + B.off_pts);
  const double* Vd = (const double*)(img + B.off_V);
  const int32_t* lvl_dev = (const int32_t*)(img + B.off_levels);
  // node table and leaf lists
  std::vector<PrecNode> nodes(nn);
  std::vector<int64_t> lbegin, koff;
  std::vector<int32_t> lsize, leaf_id;
  int64_t ko = 0;
  for (int32_t v = 0; v < nn; ++v) {
    const NodeDesc& D = B.desc[v];
    nodes[v] = PrecNode{B.begin[v], B.end[v], D.v_off, D.m, D.a, B.left[v], B.right[v]};
    if (B.left[v] < 0) {
      leaf_id.push_back(v);
      lbegin.push_back(B.begin[v]);
      lsize.push_back(D.m);
      koff.push_back(ko);
      ko += (int64_t)D.m * D.m;
    }
  }
  // general nu: the FP32 value table (the pair values here are FP32)
  const float* g32 = nullptr;
  if (nu2 == kNuGeneral) {
    const double* host = genu_table_cached(nu);
    if (!host) return fail(MLBLUP_EINVAL, "preconditioner: nu out of range for the general-nu table");
    MLB_HIP(hipMemcpyAsync(base + w.gtab, host, kGenuBytes, hipMemcpyHostToDevice, s));
    g32 = reinterpret_cast<const float*>((const double*)(base + w.gtab) + kGenuOffF32);
  }
  MLB_HIP(hipMemcpyAsync(base + w.nodes, nodes.data(), nn * sizeof(PrecNode), hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + w.lbegin, lbegin.data(), lbegin.size() * 8, hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + w.lsize, lsize.data(), lsize.size() * 4, hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + w.koff, koff.data(), koff.size() * 8, hipMemcpyHostToDevice, s));
  int st = prec_leaf_blocks((const int64_t*)(base + w.lbegin), (const int32_t*)(base + w.lsize),
                            (const int64_t*)(base + w.koff), w.nleaves, pts, B.d, zs, nu2, g32, (double*)(base + w.K),
                            s);
  if (st) return st;
  std::vector<double> Kh(w.k_entries);
  MLB_HIP(hipMemcpyAsync(Kh.data(), base + w.K, w.k_entries * 8, hipMemcpyDeviceToHost, s));
  // level sweep: Phi^(q) for q = t..1, cross terms for parents at q-1
  const int NR = w.NR;
  double* phi_cur = (double*)(base + w.phi0);
  double* phi_nxt = (double*)(base + w.phi1);
  std::vector<std::vector<double>> Xnode(nn);  // a_L x a_R per internal node, row-major
  std::vector<CrossTask> tasks;
  std::vector<double> parth;
  for (int q = B.levels - 1; q >= 1; --q) {
    const int32_t lb = B.lvl_begin[q], cnt = B.lvl_begin[q + 1] - lb;
    if ((st = prec_scal_values((const PrecNode*)(base + w.nodes), lvl_dev + lb, cnt, Vd, phi_nxt, phi_cur, NR, B.n,
                               s)))
      return st;
    tasks = level_tasks(B, q - 1);
    if (!tasks.empty()) {
      MLB_HIP(hipMemcpyAsync(base + w.tasks, tasks.data(), tasks.size() * sizeof(CrossTask), hipMemcpyHostToDevice,
                             s));
      if ((st = prec_cross((const CrossTask*)(base + w.tasks), (int32_t)tasks.size(), NR, pts, B.d, zs, nu2, g32, phi_cur,
                           NR, (double*)(base + w.part), s)))
        return st;
      parth.assign(tasks.size() * NR * NR, 0.0);
      MLB_HIP(hipMemcpyAsync(parth.data(), base + w.part, parth.size() * 8, hipMemcpyDeviceToHost, s));
      MLB_HIP(hipStreamSynchronize(s));
      // tasks were generated per parent node in order; sum their partials in that order
      size_t ti = 0;
      for (int32_t sidx = B.lvl_begin[q - 1]; sidx < B.lvl_begin[q]; ++sidx) {
        const int32_t v = B.level_nodes[sidx];
        if (B.left[v] < 0) continue;
        const int32_t L = B.left[v], R = B.right[v];
        const int aL = B.desc[L].a, aR = B.desc[R].a;
        std::vector<double>& X = Xnode[v];
        X.assign((size_t)aL * aR, 0.0);
        while (ti < tasks.size() && tasks[ti].r0 >= B.begin[L] && tasks[ti].r1 <= B.end[L]) {
          const double* pp = &parth[ti * NR * NR];
          for (int i = 0; i < aL; ++i)
            for (int j = 0; j < aR; ++j) X[(size_t)i * aR + j] += pp[i * NR + j];
          ++ti;
        }
      }
    }
    std::swap(phi_cur, phi_nxt);
  }
  MLB_HIP(hipStreamSynchronize(s));
  // bottom-up assembly
  std::vector<std::vector<double>> G(nn);
  std::vector<std::vector<double>> Bblk(nn);
  std::vector<int64_t> kleaf(nn, -1);
  for (size_t l = 0; l < leaf_id.size(); ++l) kleaf[leaf_id[l]] = koff[l];
  for (int q = B.levels - 1; q >= 0; --q) {
    const int32_t lb = B.lvl_begin[q], le = B.lvl_begin[q + 1];
    auto work_fn = [&](int32_t s0, int32_t s1) {
      for (int32_t sidx = s0; sidx < s1; ++sidx) {
        const int32_t v = B.level_nodes[sidx];
        const NodeDesc& D = B.desc[v];
        const int m = D.m, a = D.a;
        std::vector<double> Gc((size_t)m * m, 0.0);
        if (B.left[v] < 0) {
          const double* K = &Kh[kleaf[v]];
          for (size_t e = 0; e < (size_t)m * m; ++e) Gc[e] = sigma2 * K[e];
        } else {
          const int32_t L = B.left[v], R = B.right[v];
          const int aL = B.desc[L].a, aR = B.desc[R].a;
          for (int i = 0; i < aL; ++i)
            for (int j = 0; j < aL; ++j) Gc[(size_t)i * m + j] = G[L][(size_t)i * aL + j];
          for (int i = 0; i < aR; ++i)
            for (int j = 0; j < aR; ++j) Gc[(size_t)(aL + i) * m + aL + j] = G[R][(size_t)i * aR + j];
          const std::vector<double>& X = Xnode[v];
          for (int i = 0; i < aL; ++i)
            for (int j = 0; j < aR; ++j) {
              const double x = sigma2 * X[(size_t)i * aR + j];
              Gc[(size_t)i * m + aL + j] = x;
              Gc[(size_t)(aL + j) * m + i] = x;
            }
        }
        const double* V = &B.V[D.v_off];
        if (a > 0) {
          G[v].assign((size_t)a * a, 0.0);
          gemm_tn(m, 0, a, V, Gc.data(), m, G[v].data());
        }
        if (m - a > 0) {
          Bblk[v].assign((size_t)(m - a) * (m - a), 0.0);
          gemm_tn(m, a, m - a, V, Gc.data(), m, Bblk[v].data());
        }
      }
    };
    const int32_t cnt = le - lb;
    const unsigned hw = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    const unsigned nt = (unsigned)std::min<int32_t>((int32_t)hw, std::max(1, cnt / 8));
    if (nt <= 1) {
      work_fn(lb, le);
    } else {
      std::vector<std::thread> th;
      for (unsigned i = 0; i < nt; ++i) th.emplace_back(work_fn, lb + cnt * i / nt, lb + cnt * (i + 1) / nt);
      for (auto& x : th) x.join();
    }
    for (int32_t sidx = lb; sidx < le; ++sidx) {
      const int32_t v = B.level_nodes[sidx];
      if (B.left[v] >= 0) {
        std::vector<double>().swap(G[B.left[v]]);
        std::vector<double>().swap(G[B.right[v]]);
      }
    }
  }
  // pack blocks in W-coefficient order (by w_off) and invert; the coarse
  // kind keeps the cells of the finest level (rows < c0) only
  P = Precond();
  P.kind = kind;
  P.nw = B.n - B.p;
  const bool coarse = kind == MLBLUP_PREC_COARSE;
  int64_t c0 = 0, nc = 0;
  if (coarse) coarse_rows(B, &c0, &nc);
  std::vector<int32_t> order;
  for (int32_t v = 0; v < nn; ++v)
    if (B.desc[v].m - B.desc[v].a > 0 && (!coarse || B.desc[v].w_off < c0)) order.push_back(v);
  std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return B.desc[x].w_off < B.desc[y].w_off; });
  int64_t bo = 0;
  for (int32_t v : order) {
    const int mw = B.desc[v].m - B.desc[v].a;
    P.node.push_back(v);
    P.w_off.push_back(B.desc[v].w_off);
    P.mw.push_back(mw);
    P.boff.push_back(bo);
    bo += (int64_t)mw * mw;
  }
  P.blocks.resize(bo);
  for (size_t k = 0; k < order.size(); ++k)
    std::copy(Bblk[order[k]].begin(), Bblk[order[k]].end(), P.blocks.begin() + P.boff[k]);
  if (kind == MLBLUP_PREC_JACOBI) {
    P.inv.assign(P.nw, 0.0);
    for (size_t k = 0; k < order.size(); ++k)
      for (int i = 0; i < P.mw[k]; ++i) {
        const double dgl = P.blocks[P.boff[k] + (size_t)i * P.mw[k] + i];
        if (!(dgl > 0)) return fail(MLBLUP_EBREAKDOWN, "preconditioner: non-positive diagonal of C_W");
        P.inv[P.w_off[k] + i] = 1.0 / dgl;
      }
  } else {
    P.inv.resize(bo);
    bool ok = true;
    for (size_t k = 0; k < order.size() && ok; ++k)
      ok = spd_inverse(P.mw[k], &P.blocks[P.boff[k]], &P.inv[P.boff[k]]);
    if (!ok) return fail(MLBLUP_EBREAKDOWN, "preconditioner: a diagonal block of C_W is not positive definite");
  }
  if (coarse) {
    PairArgs k{nullptr, 0, nullptr, B.n, B.d, nu2, rho, sigma2, MLBLUP_FP64, MLBLUP_VALUE, nullptr, nullptr, nullptr,
               nu, nullptr};
    if ((st = coarse_inverse_factor(B, k, c0, nc, work, work_bytes, P.ycoarse, s))) return st;
    const int64_t ldc = (nc + 3) / 4 * 4;
    P.y32.assign((size_t)nc * ldc, 0.0f);
    P.x32.assign((size_t)nc * ldc, 0.0f);
    for (int64_t i = 0; i < nc; ++i)
      for (int64_t j = 0; j < nc; ++j) {
        const float v = (float)P.ycoarse[(size_t)i * nc + j];
        P.y32[(size_t)i * ldc + j] = v;
        P.x32[(size_t)j * ldc + i] = v;
      }
    P.ldc = ldc;
    P.c0 = c0;
    P.nc = nc;
  }
  // device image layout
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off = align_up(off + std::max<int64_t>(bytes, 8));
    return o;
  };
  const int64_t nb = (int64_t)order.size();
  P.off_woff = take(nb * 8);
  P.off_mw = take(nb * 4);
  P.off_boff = take(nb * 8);
  P.off_inv = take((int64_t)P.inv.size() * 8);
  P.off_y = take(P.nc * P.ldc * 4);
  P.off_x = take(P.nc * P.ldc * 4);
  P.dev_bytes = off;
  return MLBLUP_OK;
}

int precond_apply(const Precond& P, const double* r, double* z, hipStream_t s) {
  const char* base = (const char*)P.dev;
  if (P.kind == MLBLUP_PREC_JACOBI) return prec_apply_diag((const double*)(base + P.off_inv), r, z, P.nw, s);
  if (P.kind == MLBLUP_PREC_COARSE) {
    // z[0:nc] = X r_c as scratch (c0 >= nc), then z_c = Y (X r_c); the cell
    // blocks then overwrite z[0:c0].  X = G^-1 is lower and Y = G^-T upper
    // triangular (the forward substitution of the identity leaves exact zeros
    // above G^-1's diagonal), so each product reads one triangle.
    int st = prec_gemv_rows((const float*)(base + P.off_x), P.nc, P.ldc, r + P.c0, z, s, 1);
    if (st) return st;
    if ((st = prec_gemv_rows((const float*)(base + P.off_y), P.nc, P.ldc, z, z + P.c0, s, 2))) return st;
  }
  return prec_apply_blocks((const int64_t*)(base + P.off_woff), (const int32_t*)(base + P.off_mw),
                           (const int64_t*)(base + P.off_boff), (int32_t)P.node.size(),
                           (const double*)(base + P.off_inv), r, z, s);
}

}  // namespace mlb

using namespace mlb;

extern "C" {

int mlblup_precond_workspace_bytes(mlblup_basis b, int64_t* bytes) {
  clear_error();
  if (!b || !bytes) return fail(MLBLUP_EINVAL, "NULL argument");
  return precond_workspace_bytes(b->b, bytes);
}

int mlblup_precond_build(mlblup_basis b, const mlblup_matern* k, int32_t kind, void* work_dev, int64_t work_bytes,
                         void* stream, mlblup_precond* out) {
  clear_error();
  if (!b || !k || !out) return fail(MLBLUP_EINVAL, "NULL argument");
  *out = nullptr;
  if (!b->b.uploaded) return fail(MLBLUP_ESTATE, "basis not uploaded");
  if (kind != MLBLUP_PREC_JACOBI && kind != MLBLUP_PREC_BLOCK && kind != MLBLUP_PREC_COARSE)
    return fail(MLBLUP_EINVAL, "unknown preconditioner kind");
  if (kind == MLBLUP_PREC_COARSE) {
    int64_t c0, nc;
    coarse_rows(b->b, &c0, &nc);
    if (b->b.levels < 3 || nc <= 0 || c0 < nc)
      return fail(MLBLUP_EINVAL, "coarse preconditioner: needs three or more levels, the finest holding most rows");
  }
  if (nu2_of_nu(k->nu) == -1) return fail(MLBLUP_EINVAL, "preconditioner: nu must be in (0, 8] or +inf (Gaussian)");
  if (!(k->rho > 0) || !(k->sigma2 > 0) || !std::isfinite(k->rho) || !std::isfinite(k->sigma2))
    return fail(MLBLUP_EINVAL, "rho and sigma2 must be finite and > 0");
  std::unique_ptr<mlblup_precond_s> pc(new (std::nothrow) mlblup_precond_s);
  if (!pc) return fail(MLBLUP_EINVAL, "out of host memory");
  const int st = precond_build(b->b, k->nu, k->rho, k->sigma2, kind, work_dev, work_bytes,
                               (hipStream_t)stream, pc->p);
  if (st) return st;
  *out = pc.release();
  return MLBLUP_OK;
}

int mlblup_precond_info(mlblup_precond pc, int64_t* device_bytes, int64_t* n_blocks, int64_t* block_entries) {
  clear_error();
  if (!pc) return fail(MLBLUP_EINVAL, "NULL preconditioner");
  if (device_bytes) *device_bytes = pc->p.dev_bytes;
  if (n_blocks) *n_blocks = (int64_t)pc->p.node.size();
  if (block_entries) *block_entries = (int64_t)pc->p.blocks.size();
  return MLBLUP_OK;
}

int mlblup_precond_upload(mlblup_precond pc, void* dev_buf, int64_t bytes, void* stream) {
  clear_error();
  if (!pc || !dev_buf) return fail(MLBLUP_EINVAL, "NULL argument");
  Precond& P = pc->p;
  if (bytes < P.dev_bytes) return fail(MLBLUP_EINVAL, "precond_upload: buffer too small");
  if (((uintptr_t)dev_buf) % 256) return fail(MLBLUP_EINVAL, "precond_upload: buffer must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)dev_buf;
  MLB_HIP(hipMemcpyAsync(base + P.off_woff, P.w_off.data(), P.w_off.size() * 8, hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + P.off_mw, P.mw.data(), P.mw.size() * 4, hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + P.off_boff, P.boff.data(), P.boff.size() * 8, hipMemcpyHostToDevice, s));
  MLB_HIP(hipMemcpyAsync(base + P.off_inv, P.inv.data(), P.inv.size() * 8, hipMemcpyHostToDevice, s));
  if (P.nc > 0) {
    MLB_HIP(hipMemcpyAsync(base + P.off_y, P.y32.data(), P.y32.size() * 4, hipMemcpyHostToDevice, s));
    MLB_HIP(hipMemcpyAsync(base + P.off_x, P.x32.data(), P.x32.size() * 4, hipMemcpyHostToDevice, s));
  }
  MLB_HIP(hipStreamSynchronize(s));
  P.dev = dev_buf;
  P.uploaded = true;
  return MLBLUP_OK;
}

int mlblup_precond_blocks(mlblup_precond pc, double* blocks_host, int64_t* w_off_host, int32_t* mw_host) {
  clear_error();
  if (!pc) return fail(MLBLUP_EINVAL, "NULL preconditioner");
  const Precond& P = pc->p;
  if (blocks_host) std::memcpy(blocks_host, P.blocks.data(), P.blocks.size() * 8);
  if (w_off_host) std::memcpy(w_off_host, P.w_off.data(), P.w_off.size() * 8);
  if (mw_host) std::memcpy(mw_host, P.mw.data(), P.mw.size() * 4);
  return MLBLUP_OK;
}

int mlblup_precond_workspace_bytes_kind(mlblup_basis b, int32_t kind, int64_t* bytes) {
  clear_error();
  if (!b || !bytes) return fail(MLBLUP_EINVAL, "NULL argument");
  int st = precond_workspace_bytes(b->b, bytes);
  if (st || kind != MLBLUP_PREC_COARSE) return st;
  int64_t c0, nc;
  coarse_rows(b->b, &c0, &nc);
  *bytes = std::max(*bytes, coarse_layout(b->b, std::max<int64_t>(nc, 1)).total);
  return MLBLUP_OK;
}

int mlblup_precond_coarse(mlblup_precond pc, int64_t* c0, int64_t* nc, double* y_host) {
  clear_error();
  if (!pc) return fail(MLBLUP_EINVAL, "NULL preconditioner");
  const Precond& P = pc->p;
  if (c0) *c0 = P.c0;
  if (nc) *nc = P.nc;
  if (y_host && P.nc > 0) std::memcpy(y_host, P.ycoarse.data(), P.ycoarse.size() * 8);
  return MLBLUP_OK;
}

void mlblup_precond_free(mlblup_precond pc) { delete pc; }

}  // extern "C"
