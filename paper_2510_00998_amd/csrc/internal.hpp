// Internal state of a libhpmg handle, shared by the single-problem and the
// batched drivers (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <type_traits>
#include <string>
#include <vector>

#include "hpmg.h"
#include "kernels.hpp"

namespace hpmg {
namespace detail {

void set_last_error(const std::string& m);

// Resolves the device address of the static scratch array of
// hpmg_smooth_noalloc for device `dev` (current), once per device.
void init_noalloc_scratch(int dev);



struct HpmgError : std::runtime_error {
  hpmg_status st;
  HpmgError(hpmg_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

#define HIPCHK(expr)                                                                                       \
  do {                                                                                                     \
    hipError_t e_ = (expr);                                                                                \
    if (e_ != hipSuccess)                                                                                  \
      throw HpmgError(e_ == hipErrorOutOfMemory ? HPMG_E_NOMEM : HPMG_E_DEVICE,                           \
                      std::string(#expr) + ": " + hipGetErrorString(e_));                                  \
  } while (0)

inline void require(bool c, const std::string& msg) {
  if (!c) throw HpmgError(HPMG_E_INVALID, msg);
}

// Device allocation owned by the handle: hipMalloc, or the caller's
// allocator (hpmg_options.alloc / free / alloc_ctx).
struct DevMem {
  std::vector<void*> ptrs;
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* ctx = nullptr;
  void* alloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) / 256 * 256;
    if (alloc_fn) {
      p = alloc_fn(bytes, ctx);
      if (!p) throw HpmgError(HPMG_E_NOMEM, "the caller's allocator returned NULL");
      if ((reinterpret_cast<size_t>(p) & 255) != 0) {
        free_fn(p, ctx);
        throw HpmgError(HPMG_E_INVALID, "the caller's allocator returned memory not aligned to 256 bytes");
      }
    } else {
      HIPCHK(hipMalloc(&p, bytes));
    }
    ptrs.push_back(p);
    return p;
  }
  template <typename T>
  T* upload(const std::vector<T>& v, hipStream_t s) {
    T* p = (T*)alloc(v.size() * sizeof(T));
    HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
  ~DevMem() {
    for (void* p : ptrs) {
      if (free_fn)
        free_fn(p, ctx);
      else
        (void)hipFree(p);
    }
  }
};

template <typename T>
std::vector<T> cast_vec(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

inline int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Per-precision device data of one DG level.
template <typename T>
struct DGData {
  T* ref = nullptr;
  T* eig = nullptr;
  T* rk = nullptr;       // block_recompute: [Khat | C^-1], Mhat = C C^T
  // block_recompute = 2: the two record buffers (eig is ebuf[ecur]) and the
  // [Khat | C^-1] table of the rebuild kernel
  T* ebuf[2] = {nullptr, nullptr};
  int ecur = 0;
  T* rkb = nullptr;
  T* kappa = nullptr;
  T* u = nullptr;        // coarse levels only
  T* b = nullptr;        // coarse levels only
  T* tr[2] = {nullptr, nullptr};
  T* contrib = nullptr;  // corner contributions (last DG level, restriction to Q1)
  T* mort = nullptr;     // adaptive meshes: hanging-facet remap tables [I_j | P_j], j < r
  T* rtmp = nullptr;     // adaptive meshes: residual of a level followed by a coarser spacetree level
};

// One leaf set of an adaptive mesh: the caller's leaves, or a coarser
// spacetree level (the deepest leaves of the previous set merged into
// their parents).  amask / nbslot / itab / hscale as the kernels read them;
// pmap / rmap: the transfer to the next coarser leaf set (pmap[cell] =
// 32 coarse cell + child position, 31 for the same cell; rmap[coarse cell]
// [r^d] = its cells in this set by child position, or [cell, -1, ...]).
struct AdaptMesh {
  int ncell = 0, nif = 0;
  std::vector<int> lev, X;  // host: level and 3 coordinates per cell
  unsigned short* amask = nullptr;
  unsigned char* bmask = nullptr;
  int* nbslot = nullptr;
  int* itab = nullptr;
  double* hs_d = nullptr;
  float* hs_f = nullptr;
  int* pmap = nullptr;
  int* rmap = nullptr;
};

struct DGLevel {
  int p = 0, N = 0, NC = 0;  // NC: nodes per direction of the next coarser level (2: Q1)
  bool next_cg = false;
  int am = 0;                // adaptive meshes: the leaf set of this level (index into hpmg_ctx::amesh)
  bool next_h = false;       // adaptive meshes: the next level has the same degree on the next coarser leaf set
  bool dyn_nc = false;       // next DG level not the halved degree: run-time NC transfer kernels
  double sigma_hat = 0.0;
  size_t ndof = 0, trsize = 0;  // per right-hand side
  DGData<double> d;
  DGData<float> f;
  // 16-bit storage (finest level only, allocated on first use): traces; the
  // operator tables and the coarse levels are those of f
  DGData<_Float16> h16;
  DGData<__bf16> b16;
};

template <typename T>
struct CGData {
  T* st = nullptr;
  T* dinv = nullptr;
  T* u[2] = {nullptr, nullptr};
  T* b = nullptr;
  T* r = nullptr;
  T* rw = nullptr;  // restriction weights to the next coarser level
  T* pw = nullptr;  // prolongation weights from it
};

struct CGLevel {
  int n = 0, nv = 0;
  size_t size = 0;
  int cur = 0;                // which of u[0], u[1] holds the iterate
  int rk = 3;                 // fine vertices per coarse vertex in the restriction (2 factor - 1)
  int* ridx = nullptr;        // [nvc][rk]
  int* pidx = nullptr;        // [nv][2]
  CGData<double> d;
  CGData<float> f;
};

}  // namespace detail
}  // namespace hpmg

struct hpmg_ctx {
  int dim = 0, n = 0, p = 0, ncell = 0;
  int dev = -1;  // HIP device the handle was set up on
  bool vark = false;
  double kappa_const = 1.0;
  std::vector<double> kappa;
  hpmg_options opt{};
  size_t ndof = 0;
  std::vector<hpmg::detail::DGLevel> dg;
  std::vector<hpmg::detail::CGLevel> cg;
  double* coarse_inv = nullptr;  // dense inverse of the coarsest Q1 operator
  unsigned char* bmask = nullptr;  // per cell boundary-facet mask (all DG levels)
  int coarse_m = 0;
  // Adaptive (spacetree) mesh, hpmg_setup_adaptive: n is the base mesh,
  // ncell the number of leaves.  rfac: subdivision factor r; mif = r^(d-1)
  // fine cells per hanging interface; amesh: the caller's leaf set, then the
  // coarser spacetree levels (options.spacetree_levels); CSR transfers
  // between the Q1 base vertices and the corners of the last leaf set's
  // cells (restriction: rows = vertices, prolongation: rows = cell
  // corners); leaf geometry of the caller's leaves for load vectors.
  bool adapt = false;
  int rfac = 0, mif = 0;
  std::vector<hpmg::detail::AdaptMesh> amesh;
  int q1r_rows = 0, q1p_rows = 0;
  int *q1r_ptr = nullptr, *q1r_col = nullptr, *q1p_ptr = nullptr, *q1p_col = nullptr;
  double *q1r_wd = nullptr, *q1p_wd = nullptr;
  float *q1r_wf = nullptr, *q1p_wf = nullptr;
  std::vector<double> leaf_h, leaf_org;  // per leaf: width, lower corner (dim values)
  // outer solver workspace (FP64) and the FP32 cycle vectors
  double *r = nullptr, *rold = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr;
  float *r32 = nullptr, *z32 = nullptr;
  _Float16 *r16 = nullptr, *z16 = nullptr;  // 16-bit cycle vectors (on first use)
  __bf16 *rb16 = nullptr, *zb16 = nullptr;
  double *partial = nullptr, *scal = nullptr;
  double* kpartial = nullptr;  // per-block shares of p.q (one per finest-level cell at most)
  double* host_scal = nullptr;  // pinned
  // which level-0 trace buffer holds the traces of the caller's u after
  // hpmg_project / hpmg_smooth / hpmg_sweep (-1: none), per dtype
  int trace_state[4] = {-1, -1, -1, -1};
  int trace_rhs[4] = {0, 0, 0, 0};
  hpmg::detail::DevMem mem;
  // hpmg_solve: one outer iteration captured as a HIP graph (index: restart
  // flag) for the cycle precision graph_prec, replayed on the internal
  // stream gs on the internal solution vector ug
  hipStream_t gs = nullptr;
  double* ug = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int graph_prec = -1;
  // block_recompute = 2: rebuild stream and, per precision (FP64, FP32) and
  // record buffer, the events "rebuild done" and "last sweep reading it done"
  hipStream_t bs = nullptr;
  hipEvent_t ev_built[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipEvent_t ev_used[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  ~hpmg_ctx() {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        if (ev_built[i][j]) (void)hipEventDestroy(ev_built[i][j]);
        if (ev_used[i][j]) (void)hipEventDestroy(ev_used[i][j]);
      }
    if (bs) (void)hipStreamDestroy(bs);
    for (int i = 0; i < 2; ++i) {
      if (gexec[i]) (void)hipGraphExecDestroy(gexec[i]);
      if (graph[i]) (void)hipGraphDestroy(graph[i]);
    }
    if (gs) (void)hipStreamDestroy(gs);
    if (host_scal) (void)hipHostFree(host_scal);
  }
};

namespace hpmg {
namespace detail {

template <typename T>
DGData<T>& data(DGLevel& l);
template <>
inline DGData<double>& data<double>(DGLevel& l) { return l.d; }
template <>
inline DGData<float>& data<float>(DGLevel& l) { return l.f; }
template <>
inline DGData<_Float16>& data<_Float16>(DGLevel& l) { return l.h16; }
template <>
inline DGData<__bf16>& data<__bf16>(DGLevel& l) { return l.b16; }
template <typename T>
CGData<T>& data(CGLevel& l);
template <>
inline CGData<double>& data<double>(CGLevel& l) { return l.d; }
template <>
inline CGData<float>& data<float>(CGLevel& l) { return l.f; }

// Kernel arguments of level L for storage type T (operator tables in the
// compute type CT<T>); vectors and traces are set by the caller.
template <typename T>
inline hpmg::DGArgs<T> dg_args(hpmg_ctx* h, DGLevel& L) {
  using C = hpmg::CT<T>;
  hpmg::DGArgs<T> a{};
  DGData<C>& d = data<C>(L);
  a.n = h->n;
  a.ncell = h->ncell;
  a.vark = h->vark ? 1 : 0;
  a.kappa_const = (C)h->kappa_const;
  a.ref = d.ref;
  a.eig = d.eig;
  a.rk = d.rk;
  a.kappa = d.kappa;
  a.bmask = h->bmask;
  const double hh = 1.0 / h->n;
  a.h_fwd = (C)std::pow(hh, 2 - h->dim);
  a.h_apply = (C)std::pow(hh, h->dim - 2);
  a.sigma_hat = (C)L.sigma_hat;
  a.omega = (C)h->opt.omega_dg;
  a.gl = h->opt.basis;
  a.ivar = h->opt.block_variant;
  a.mfma = h->opt.mfma;
  a.vstride = (long long)L.ndof;
  a.tstride = (long long)L.trsize;
  if (h->adapt) {
    const AdaptMesh& M = h->amesh[L.am];
    a.ncell = M.ncell;
    a.adapt = 1;
    a.amask = M.amask;
    a.bmask = M.bmask;
    a.nbslot = M.nbslot;
    if constexpr (std::is_same<C, double>::value)
      a.hscale = M.hs_d;
    else
      a.hscale = M.hs_f;
    a.sig_hang = (C)(L.sigma_hat * h->rfac);
    a.mort = d.mort;
    a.itab = M.itab;
    a.nif = M.nif;
    a.mif = h->mif;
    a.rfac = h->rfac;
  }
  return a;
}

template <typename T>
inline void dg_run(hpmg_ctx* h, int op, const hpmg::DGArgs<T>& a, int N, int nrhs, int flag, hipStream_t s) {
  if (!hpmg::dg_dispatch(h->dim, N, op, a, nrhs, flag, s))
    throw HpmgError(HPMG_E_UNSUPPORTED, "no kernel for this degree");
  HIPCHK(hipGetLastError());
  // adaptive meshes: every traversal that writes traces is followed by the
  // hanging-facet remap of the buffer it wrote
  if (h->adapt && (op == hpmg::OP_SWEEP || op == hpmg::OP_PROJECT || op == hpmg::OP_PROLONG ||
                   op == hpmg::OP_PROLONG_Q1 || op == hpmg::OP_PROLONG_DYN)) {
    if constexpr (sizeof(T) >= 4) {
      hpmg::remap_hanging<T>(h->dim, N, a.ncell, a.nif, a.mif, a.rfac, a.itab, a.mort, a.tr_out, a.tstride, nrhs,
                             s);
      HIPCHK(hipGetLastError());
    } else {
      throw HpmgError(HPMG_E_UNSUPPORTED, "adaptive meshes take FP64 or FP32 vectors");
    }
  }
}


}  // namespace detail
}  // namespace hpmg
