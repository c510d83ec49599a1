// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fkf.h"

namespace fkf {

// ---------------------------------------------------------------- errors ---
void set_error(const std::string &msg);

struct Error {
  fkf_status code;
  std::string msg;
};

#define FKF_CHECK_HIP(expr)                                                        \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::fkf::Error{e_ == hipErrorOutOfMemory ? FKF_E_NOMEM : FKF_E_HIP,      \
                         std::string(#expr) + ": " + hipGetErrorString(e_)};       \
  } while (0)

#define FKF_REQUIRE(cond, msg)                                                     \
  do {                                                                             \
    if (!(cond)) throw ::fkf::Error{FKF_E_ARG, (msg)};                             \
  } while (0)

// Run `body`, translating exceptions into a status code.
template <class F>
fkf_status guarded(F &&body) {
  try {
    body();
    return FKF_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return FKF_E_NOMEM;
  } catch (const std::exception &e) {
    set_error(e.what());
    return FKF_E_ARG;
  }
}

// ------------------------------------------------------- device buffers ---
// Owning device allocation (hipMalloc/hipFree).
template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    FKF_CHECK_HIP(hipMalloc(&p, count * sizeof(T)));
    n = count;
  }
  // grow-only reallocation (contents not preserved)
  void reserve(size_t count) { if (count > n) alloc(count); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void upload(const T *host, size_t count, hipStream_t s) {
    if (count) FKF_CHECK_HIP(hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void upload(const std::vector<T> &v, hipStream_t s) {
    alloc(v.size());
    upload(v.data(), v.size(), s);
  }
  // device-to-device copy of count elements of src (stream-ordered)
  void copy_from(const T *src, size_t count, hipStream_t s) {
    alloc(count);
    if (count)
      FKF_CHECK_HIP(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyDeviceToDevice, s));
  }
  // the same into a buffer grown only when too small
  void copy_into(const T *src, size_t count, hipStream_t s) {
    reserve(count);
    if (count)
      FKF_CHECK_HIP(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyDeviceToDevice, s));
  }
};

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ----------------------------------------------------- host geometry -------
constexpr int kMaxDim = 3;
constexpr int kMaxCheb = 16;
constexpr int kTile = 64;   // padded leaf block edge (leaf_size <= 64)

struct Node {
  int64_t begin = 0, end = 0;   // range of tree positions
  int level = 0;
  int child[2] = {-1, -1};
  int parent = -1;
  int leaf = -1;                // leaf index, or -1
  double lo[kMaxDim] = {0, 0, 0}, hi[kMaxDim] = {0, 0, 0};
  bool is_leaf() const { return child[0] < 0; }
  int64_t size() const { return end - begin; }
};

struct Tree {
  int d = 2;
  int64_t n = 0;
  int leaf_size = 64;
  std::vector<int64_t> perm;    // tree position -> caller index
  std::vector<Node> nodes;      // nodes[0] = root
  std::vector<int> leaves;      // node id of leaf i, leaves in tree order
  int depth = 0;                // max level
};

Tree build_tree(const double *pts, int64_t n, int d, int leaf_size);
double node_diam(const Node &a, int d);
double node_dist(const Node &a, const Node &b, int d);
void partition(const Tree &t, double eta, std::vector<std::pair<int, int>> &near,
               std::vector<std::pair<int, int>> &far);

// Chebyshev nodes of the first kind on [-1, 1] and barycentric weights.
void cheb_nodes(int p, double *u, double *w);

// Matern kernel entry for the host (used for the order selection only).
double matern_host(double r, int kind, double ell, double theta);

// Chebyshev order per tree level from the sampled block error rule.
std::vector<int> choose_cheb_orders(const Tree &t, const double *pts,
                                    const std::vector<std::pair<int, int>> &far,
                                    int kind, double ell, double theta, int p_min,
                                    int p_max, double tol);

// Straight-ray operator on a regular grid of the unit box (CSR).
void trace_rays(int d, const int *grid, int n_m, const double *src, const double *rcv,
                std::vector<int64_t> &rowptr, std::vector<int32_t> &col,
                std::vector<double> &val);

}  // namespace fkf
