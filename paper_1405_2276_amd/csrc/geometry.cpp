// Host-side geometry: cluster tree, block partition, Chebyshev order selection
// and the straight-ray operator.  Plain C++ (no device code).
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <stdexcept>

#include "common.h"

namespace fkf {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

}  // namespace fkf

extern "C" const char *fkf_last_error(void) { return fkf::g_last_error.c_str(); }
extern "C" const char *fkf_version(void) { return "fkf-mi355x 0.1 (gfx950, fp64)"; }

namespace fkf {

// ------------------------------------------------------------ cluster tree ---
// Recursive bisection (Section 2.2.1 builds Gamma as an H-matrix over a cluster
// tree).  A cluster is split across the longest side of its bounding box; the
// left child receives leaf_size * ceil(ceil(m/leaf_size)/2) points so that all
// leaves are full except at most one, which keeps the near-field tiles dense
// on the GPU.
namespace {

struct Builder {
  const double *pts;
  int d;
  int leaf;
  Tree *t;

  void bbox(Node &nd) {
    for (int k = 0; k < d; ++k) {
      nd.lo[k] = INFINITY;
      nd.hi[k] = -INFINITY;
    }
    for (int64_t i = nd.begin; i < nd.end; ++i) {
      const double *x = pts + t->perm[i] * d;
      for (int k = 0; k < d; ++k) {
        nd.lo[k] = std::min(nd.lo[k], x[k]);
        nd.hi[k] = std::max(nd.hi[k], x[k]);
      }
    }
  }

  int make(int64_t b, int64_t e, int level, int parent) {
    int id = (int)t->nodes.size();
    t->nodes.emplace_back();
    {
      Node &nd = t->nodes[id];
      nd.begin = b;
      nd.end = e;
      nd.level = level;
      nd.parent = parent;
      bbox(nd);
    }
    t->depth = std::max(t->depth, level);
    int64_t m = e - b;
    if (m <= leaf) {
      t->nodes[id].leaf = (int)t->leaves.size();
      t->leaves.push_back(id);
      return id;
    }
    int axis = 0;
    double ext = -1;
    for (int k = 0; k < d; ++k) {
      double w = t->nodes[id].hi[k] - t->nodes[id].lo[k];
      if (w > ext) {
        ext = w;
        axis = k;
      }
    }
    auto first = t->perm.begin() + b, last = t->perm.begin() + e;
    const double *P = pts;
    const int dd = d;
    std::stable_sort(first, last, [P, dd, axis](int64_t a, int64_t c) {
      double xa = P[a * dd + axis], xc = P[c * dd + axis];
      if (xa != xc) return xa < xc;
      return a < c;
    });
    int64_t nleaf = (m + leaf - 1) / leaf;
    int64_t left = (int64_t)leaf * ((nleaf + 1) / 2);
    int c0 = make(b, b + left, level + 1, id);
    int c1 = make(b + left, e, level + 1, id);
    t->nodes[id].child[0] = c0;
    t->nodes[id].child[1] = c1;
    return id;
  }
};

}  // namespace

Tree build_tree(const double *pts, int64_t n, int d, int leaf_size) {
  Tree t;
  t.d = d;
  t.n = n;
  t.leaf_size = leaf_size;
  t.perm.resize(n);
  std::iota(t.perm.begin(), t.perm.end(), (int64_t)0);
  t.nodes.reserve(4 * (n / std::max(leaf_size, 1) + 1));
  Builder bld{pts, d, leaf_size, &t};
  bld.make(0, n, 0, -1);
  return t;
}

double node_diam(const Node &a, int d) {
  double s = 0;
  for (int k = 0; k < d; ++k) s += (a.hi[k] - a.lo[k]) * (a.hi[k] - a.lo[k]);
  return std::sqrt(s);
}

double node_dist(const Node &a, const Node &b, int d) {
  double s = 0;
  for (int k = 0; k < d; ++k) {
    double g = std::max(0.0, std::max(a.lo[k] - b.hi[k], b.lo[k] - a.hi[k]));
    s += g * g;
  }
  return std::sqrt(s);
}

// Block partition: (s, t) is admissible (a far, low-rank block) when
// max(diam s, diam t) <= eta * dist(s, t) and dist > 0; inadmissible leaf
// pairs form the dense near field; otherwise the larger side is split.
void partition(const Tree &t, double eta, std::vector<std::pair<int, int>> &near,
               std::vector<std::pair<int, int>> &far) {
  std::vector<std::pair<int, int>> stack{{0, 0}};
  while (!stack.empty()) {
    auto [s, q] = stack.back();
    stack.pop_back();
    const Node &a = t.nodes[s], &b = t.nodes[q];
    double dist = node_dist(a, b, t.d);
    if (dist > 0 && std::max(node_diam(a, t.d), node_diam(b, t.d)) <= eta * dist) {
      far.emplace_back(s, q);
      continue;
    }
    if (a.is_leaf() && b.is_leaf()) {
      near.emplace_back(s, q);
      continue;
    }
    // push in reverse so that pairs come out in tree order
    if (!a.is_leaf() && !b.is_leaf()) {
      for (int i = 1; i >= 0; --i)
        for (int j = 1; j >= 0; --j) stack.emplace_back(a.child[i], b.child[j]);
    } else if (!a.is_leaf()) {
      for (int i = 1; i >= 0; --i) stack.emplace_back(a.child[i], q);
    } else {
      for (int j = 1; j >= 0; --j) stack.emplace_back(s, b.child[j]);
    }
  }
}

// --------------------------------------------------------------- Chebyshev ---
void cheb_nodes(int p, double *u, double *w) {
  for (int a = 0; a < p; ++a) {
    double th = (2.0 * a + 1.0) * M_PI / (2.0 * p);
    u[a] = std::cos(th);
    w[a] = ((a & 1) ? -1.0 : 1.0) * std::sin(th);
  }
}

double matern_host(double r, int kind, double ell, double theta) {
  const int b = kind % 3;
  const double t = (b == 0 ? 1.0 : std::sqrt(b == 1 ? 3.0 : 5.0)) * r / ell;
  const double ex = std::exp(-t);
  switch (kind) {
    case FKF_MATERN_12: return theta * ex;
    case FKF_MATERN_32: return theta * (1.0 + t) * ex;
    case FKF_MATERN_52: return theta * (1.0 + t + t * t / 3.0) * ex;
    // d/d ell of theta C(t(ell)) = (theta / ell) (-t C'(t))
    case FKF_MATERN_12_DLENGTH: return theta / ell * t * ex;
    case FKF_MATERN_32_DLENGTH: return theta / ell * t * t * ex;
    default: return theta / ell * t * t * (1.0 + t) * ex / 3.0;
  }
}

namespace {

// Lagrange basis at normalised coordinate x (barycentric form, 1st-kind nodes).
void lagrange(int p, const double *u, const double *w, double x, double *L) {
  for (int a = 0; a < p; ++a)
    if (x == u[a]) {
      for (int b = 0; b < p; ++b) L[b] = (a == b) ? 1.0 : 0.0;
      return;
    }
  double s = 0;
  for (int a = 0; a < p; ++a) {
    L[a] = w[a] / (x - u[a]);
    s += L[a];
  }
  for (int a = 0; a < p; ++a) L[a] /= s;
}

// Tensor basis U (m x p^d) of a node box at the given points, plus its nodes.
void tensor_basis(const Node &nd, int d, int p, const std::vector<const double *> &xs,
                  std::vector<double> &U, std::vector<double> &xi) {
  double u[kMaxCheb], w[kMaxCheb];
  cheb_nodes(p, u, w);
  int pd = 1;
  for (int k = 0; k < d; ++k) pd *= p;
  size_t m = xs.size();
  U.assign(m * pd, 1.0);
  std::vector<double> L(p);
  for (size_t i = 0; i < m; ++i)
    for (int k = 0, stride = 1; k < d; ++k, stride *= p) {
      double mid = 0.5 * (nd.lo[k] + nd.hi[k]);
      double hw = 0.5 * (nd.hi[k] - nd.lo[k]);
      double x = hw > 0 ? (xs[i][k] - mid) / hw : 0.0;
      lagrange(p, u, w, x, L.data());
      for (int a = 0; a < pd; ++a) U[i * pd + a] *= L[(a / stride) % p];
    }
  xi.assign((size_t)pd * d, 0.0);
  for (int a = 0; a < pd; ++a)
    for (int k = 0, stride = 1; k < d; ++k, stride *= p) {
      double mid = 0.5 * (nd.lo[k] + nd.hi[k]);
      double hw = 0.5 * (nd.hi[k] - nd.lo[k]);
      xi[(size_t)a * d + k] = mid + hw * u[(a / stride) % p];
    }
}

}  // namespace

std::vector<int> choose_cheb_orders(const Tree &t, const double *pts,
                                    const std::vector<std::pair<int, int>> &far,
                                    int kind, double ell, double theta, int p_min,
                                    int p_max, double tol) {
  std::vector<int> p(t.depth + 1, p_min);
  if (tol <= 0) return p;
  const int d = t.d;
  // worst case per level: the admissible pair with the smallest dist/diam
  std::vector<int> worst(t.depth + 1, -1);
  std::vector<double> ratio(t.depth + 1, INFINITY);
  for (size_t i = 0; i < far.size(); ++i) {
    const Node &a = t.nodes[far[i].first], &b = t.nodes[far[i].second];
    double r = node_dist(a, b, d) / std::max(node_diam(a, d), node_diam(b, d));
    if (r < ratio[a.level]) {
      ratio[a.level] = r;
      worst[a.level] = (int)i;
    }
  }
  const size_t ns = 96;
  for (int lev = 0; lev <= t.depth; ++lev) {
    if (worst[lev] < 0) continue;
    const Node &a = t.nodes[far[worst[lev]].first], &b = t.nodes[far[worst[lev]].second];
    auto sample = [&](const Node &nd) {
      std::vector<const double *> xs;
      int64_t m = nd.size();
      size_t cnt = (size_t)std::min<int64_t>(m, ns);
      for (size_t i = 0; i < cnt; ++i) {
        int64_t pos = nd.begin + (int64_t)((double)i * m / cnt);
        xs.push_back(pts + t.perm[pos] * d);
      }
      return xs;
    };
    auto xa = sample(a), xb = sample(b);
    std::vector<double> E(xa.size() * xb.size());
    double en = 0;
    for (size_t i = 0; i < xa.size(); ++i)
      for (size_t j = 0; j < xb.size(); ++j) {
        double r2 = 0;
        for (int k = 0; k < d; ++k) r2 += (xa[i][k] - xb[j][k]) * (xa[i][k] - xb[j][k]);
        E[i * xb.size() + j] = matern_host(std::sqrt(r2), kind, ell, theta);
        en += E[i * xb.size() + j] * E[i * xb.size() + j];
      }
    int chosen = p_max;
    for (int q = p_min; q <= p_max; ++q) {
      std::vector<double> Ua, Ub, xia, xib;
      tensor_basis(a, d, q, xa, Ua, xia);
      tensor_basis(b, d, q, xb, Ub, xib);
      int pd = (int)(xia.size() / d);
      std::vector<double> K((size_t)pd * pd);
      for (int i = 0; i < pd; ++i)
        for (int j = 0; j < pd; ++j) {
          double r2 = 0;
          for (int k = 0; k < d; ++k) {
            double dx = xia[(size_t)i * d + k] - xib[(size_t)j * d + k];
            r2 += dx * dx;
          }
          K[(size_t)i * pd + j] = matern_host(std::sqrt(r2), kind, ell, theta);
        }
      // T = Ua K (ns x pd), approx = T Ub^T
      std::vector<double> T(xa.size() * pd, 0.0);
      for (size_t i = 0; i < xa.size(); ++i)
        for (int c = 0; c < pd; ++c) {
          double s = 0;
          for (int b2 = 0; b2 < pd; ++b2) s += Ua[i * pd + b2] * K[(size_t)b2 * pd + c];
          T[i * pd + c] = s;
        }
      double err = 0;
      for (size_t i = 0; i < xa.size(); ++i)
        for (size_t j = 0; j < xb.size(); ++j) {
          double s = 0;
          for (int c = 0; c < pd; ++c) s += T[i * pd + c] * Ub[j * pd + c];
          double e = s - E[i * xb.size() + j];
          err += e * e;
        }
      if (std::sqrt(err) <= tol * std::sqrt(en)) {
        chosen = q;
        break;
      }
    }
    p[lev] = chosen;
  }
  return p;
}

// ------------------------------------------------------------------- rays ---
// Straight-ray operator by a grid walk (cell-by-cell traversal): starting in
// the cell that contains the source, repeatedly step into the neighbour across
// the nearest grid line/plane, emitting the traversed length.  Equal crossing
// parameters (a grid corner) advance all tied axes at once.  An axis along
// which the ray is constant and sits exactly on an interior grid plane makes
// the piece shared equally by the two cells on either side.
void trace_rays(int d, const int *grid, int n_m, const double *src, const double *rcv,
                std::vector<int64_t> &rowptr, std::vector<int32_t> &col,
                std::vector<double> &val) {
  rowptr.assign(1, 0);
  col.clear();
  val.clear();
  for (int m = 0; m < n_m; ++m) {
    const double *a = src + (size_t)m * d;
    const double *b = rcv + (size_t)m * d;
    double dir[kMaxDim], len2 = 0;
    for (int k = 0; k < d; ++k) {
      dir[k] = b[k] - a[k];
      len2 += dir[k] * dir[k];
    }
    double len = std::sqrt(len2);
    std::map<int64_t, double> acc;
    if (len > 0) {
      int idx[kMaxDim];
      int shared[kMaxDim];   // 1 when the fixed coordinate lies on an interior plane
      int step[kMaxDim];
      for (int k = 0; k < d; ++k) {
        double g = a[k] * grid[k];
        double fl = std::floor(g);
        shared[k] = 0;
        if (dir[k] > 0) {
          idx[k] = (int)fl;
          step[k] = 1;
        } else if (dir[k] < 0) {
          idx[k] = (g == fl) ? (int)fl - 1 : (int)fl;
          step[k] = -1;
        } else {
          step[k] = 0;
          if (g == fl && fl > 0 && fl < grid[k]) {
            shared[k] = 1;
            idx[k] = (int)fl;   // cells idx-1 and idx
          } else {
            idx[k] = (int)fl;
          }
        }
        idx[k] = std::min(std::max(idx[k], 0), grid[k] - 1);
      }
      auto next_t = [&](int k) -> double {
        if (step[k] == 0) return INFINITY;
        double plane = (step[k] > 0 ? idx[k] + 1 : idx[k]) / (double)grid[k];
        return (plane - a[k]) / dir[k];
      };
      double t0 = 0.0;
      for (int guard = 0; guard < 4 * (grid[0] + grid[1] + (d > 2 ? grid[2] : 0)) + 8; ++guard) {
        double tn = 1.0;
        for (int k = 0; k < d; ++k) tn = std::min(tn, next_t(k));
        double seg = (tn - t0) * len;
        if (seg > 1e-14 * len) {
          int nshare = 0;
          for (int k = 0; k < d; ++k) nshare += shared[k];
          int combos = 1 << nshare;
          for (int c = 0; c < combos; ++c) {
            int64_t flat = 0, stride = 1;
            for (int k = 0, bit = 0; k < d; ++k) {
              int ik = idx[k];
              if (shared[k]) {
                if (!((c >> bit) & 1)) ik -= 1;
                ++bit;
              }
              flat += (int64_t)ik * stride;
              stride *= grid[k];
            }
            acc[flat] += seg / combos;
          }
        }
        if (tn >= 1.0) break;
        bool out = false;
        for (int k = 0; k < d; ++k)
          if (step[k] != 0 && std::fabs(next_t(k) - tn) <= 1e-13) {
            idx[k] += step[k];
            if (idx[k] < 0 || idx[k] >= grid[k]) out = true;
          }
        t0 = tn;
        if (out) break;
      }
    }
    for (auto &kv : acc) {
      col.push_back((int32_t)kv.first);
      val.push_back(kv.second);
    }
    rowptr.push_back((int64_t)col.size());
  }
}

}  // namespace fkf

extern "C" fkf_status fkf_rays_host(int32_t d, const int32_t *grid, int32_t n_m,
                                    const double *src, const double *rcv, int64_t *rowptr,
                                    int64_t *nnz, int32_t *col_host, double *val_host,
                                    int64_t capacity) {
  using namespace fkf;
  return guarded([&] {
    FKF_REQUIRE(grid && src && rcv && rowptr && nnz, "fkf_rays_host: NULL argument");
    FKF_REQUIRE(d == 2 || d == 3, "fkf_rays_host: d must be 2 or 3");
    FKF_REQUIRE(n_m >= 0, "fkf_rays_host: n_m < 0");
    for (int k = 0; k < d; ++k) FKF_REQUIRE(grid[k] >= 1, "fkf_rays_host: grid size < 1");
    for (int64_t i = 0; i < (int64_t)n_m * d; ++i)
      FKF_REQUIRE(src[i] >= 0 && src[i] <= 1 && rcv[i] >= 0 && rcv[i] <= 1,
                  "fkf_rays_host: ray endpoints must lie in the unit box");
    std::vector<int64_t> rp;
    std::vector<int32_t> c;
    std::vector<double> v;
    trace_rays(d, grid, n_m, src, rcv, rp, c, v);
    std::copy(rp.begin(), rp.end(), rowptr);
    *nnz = (int64_t)c.size();
    if (col_host || val_host) {
      FKF_REQUIRE(col_host && val_host, "fkf_rays_host: give both col and val");
      FKF_REQUIRE(capacity >= (int64_t)c.size(), "fkf_rays_host: capacity < nnz");
      std::copy(c.begin(), c.end(), col_host);
      std::copy(v.begin(), v.end(), val_host);
    }
  });
}
