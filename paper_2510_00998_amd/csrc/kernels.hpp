// Host-callable launchers of every device kernel of libhpmg.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "dg_kernels.hpp"

namespace hpmg {

// Operations of the DG cell kernels (template dispatch by dimension, nodes
// per direction N = p+1 and the coarse partner's N).
enum DGOp {
  OP_SWEEP = 0,       // fused block-Jacobi sweep (flag: u == 0 on entry)
  OP_APPLY = 1,       // y = A u (flag: 1 -> r = b - A u)
  OP_RESTRICT = 2,    // r = b - A u restricted to the next coarser level
  OP_PROJECT = 3,     // traces of u
  OP_PROLONG = 4,     // u += P e, then traces of u
  OP_RESTRICT_Q1 = 5, // OP_RESTRICT to Q1 corner contributions from any degree (one-step p-coarsening)
  OP_PROLONG_Q1 = 6,  // OP_PROLONG from Q1 to any degree
  OP_RESTRICT_DYN = 7, // OP_RESTRICT to a DG level of a.ncd nodes per direction (explicit p schedules)
  OP_PROLONG_DYN = 8,  // OP_PROLONG from such a level
  OP_BUILD_EIG = 9     // per-cell fast-diagonalisation data of every cell (variable kappa) into a.out
};

// Next coarser level of a DG level with N nodes per direction: DG with
// NC = floor(p/2)+1 nodes while floor(p/2) >= 2, else Q1 (NC = 2).
constexpr int nc_next(int N) { return ((N - 1) / 2 >= 2) ? (N - 1) / 2 + 1 : 2; }

// Returns false if (dim, N) has no compiled kernel.  One definition per
// (dimension, storage type) in dg_inst_<dim>d_<type>.hip.
bool dg_dispatch2(int N, int op, const DGArgs<double>& a, int nrhs, int flag, hipStream_t s);
bool dg_dispatch2(int N, int op, const DGArgs<float>& a, int nrhs, int flag, hipStream_t s);
bool dg_dispatch2(int N, int op, const DGArgs<_Float16>& a, int nrhs, int flag, hipStream_t s);
bool dg_dispatch2(int N, int op, const DGArgs<__bf16>& a, int nrhs, int flag, hipStream_t s);
bool dg_dispatch3(int N, int op, const DGArgs<double>& a, int nrhs, int flag, hipStream_t s);
bool dg_dispatch3(int N, int op, const DGArgs<float>& a, int nrhs, int flag, hipStream_t s);
bool dg_dispatch3(int N, int op, const DGArgs<_Float16>& a, int nrhs, int flag, hipStream_t s);
bool dg_dispatch3(int N, int op, const DGArgs<__bf16>& a, int nrhs, int flag, hipStream_t s);
template <typename T>
inline bool dg_dispatch(int dim, int N, int op, const DGArgs<T>& a, int nrhs, int flag, hipStream_t s) {
  return dim == 2 ? dg_dispatch2(N, op, a, nrhs, flag, s) : dg_dispatch3(N, op, a, nrhs, flag, s);
}

template <typename T>
void cg_stencil(int D, int nv, const T* st, const T* dinv, const T* u, const T* b, T* out, T omega, int mode,
                int uzero, hipStream_t s);
template <typename T>
void cg_restrict(int D, int nvf, int nvc, int rk, const int* ridx, const T* rw, const T* rf, T* bc, hipStream_t s);
template <typename T>
void cg_prolong(int D, int nvf, int nvc, const int* pidx, const T* pw, const T* ec, T* uf, hipStream_t s);
template <typename T>
void gather_corners(int D, int n, const T* contrib, T* bcg, hipStream_t s);
template <typename T>
void dense_solve(int m, const double* Ainv, const T* b, T* x, hipStream_t s);
// Adaptive meshes: fill the hanging-facet slots of the trace buffer tr
// (nrhs columns tstride apart) from the cells' own traces; itab [nif][2 + m]
// = (coarse cell, its facet, the m = r^(d-1) fine cells), mort = [I_j | P_j]
// for j < r (N x N each, adapt_kernels.hip).
template <typename T>
void remap_hanging(int D, int N, int ncell, int nif, int m, int r, const int* itab, const CT<T>* mort, T* tr,
                   long long tstride, int nrhs, hipStream_t s);
// Transfers between two spacetree levels of one degree (adaptive meshes):
// restrict_ = true: dst (coarse, ncells cells) = P^T src (fine) with map =
// rmap [coarse][r^d]; false: dst (fine, ncells cells) += P src (coarse) with
// map = pmap [fine]; I = the level's interpolation tables I_j (j < r).
// fstride / cstride: per right-hand side strides of the fine / coarse vectors.
template <typename C>
void spacetree_transfer(bool restrict_, int D, int N, int ncells, const int* map, int r, const C* I, const C* src,
                        C* dst, long long fstride, long long cstride, int nrhs, hipStream_t s);
// y = W x for a CSR matrix W (the Q1 transfers of adaptive meshes)
template <typename T>
void csr_apply(int nrow, const int* ptr, const int* col, const T* w, const T* x, T* y, hipStream_t s);
template <typename T>
void fill(T* x, size_t n, T v, hipStream_t s);

// The Q1 V-cycle from level lv[0] (entered with a zero initial guess, its
// right-hand side in lv[0].b) down to the coarsest level lv[nlev - 1]
// (dense solve with Ainv, m unknowns), in one workgroup.
constexpr int CG_BLOCK_MAX_LEVELS = 8;
constexpr int CG_BLOCK_MAX_VERTICES = 512;  // largest level taken by the one-workgroup cycle
template <typename T>
struct CGBlockLevel {
  int nv;
  const T* st;
  const T* dinv;
  T* u[2];
  T* b;
  T* r;
  const int* ridx;  // restriction to the next level (RK slots per coarse vertex and axis)
  const T* rw;
  const int* pidx;  // prolongation from the next level (2 slots per vertex and axis)
  const T* pw;
};
template <typename T>
struct CGBlockArgs {
  int nlev, nu_pre, nu_post, m;
  T omega;
  const double* Ainv;
  CGBlockLevel<T> lv[CG_BLOCK_MAX_LEVELS];
};
template <typename T>
void cg_vcycle_block(int D, int rk, const CGBlockArgs<T>& a, hipStream_t s);

constexpr int KRYLOV_RED_BLOCKS = 1024;
void krylov_dot(size_t n, const double* x, const double* y, const double* z, double* partial, double* scal, int op,
                int a0, int first, hipStream_t s);
void krylov_update_p(size_t n, const double* z, double* p, const double* scal, hipStream_t s);
// scal[5] = scal[2] / (sum of partial[0..n)): alpha from per-block shares of p.q
void krylov_alpha(const double* partial, int n, double* scal, hipStream_t s);
void axpy(size_t n, double a, const double* x, double* y, hipStream_t s);
// r32 (nullable): also store (float) r for the next FP32 cycle
void krylov_update_ur(size_t n, double* u, double* r, double* rold, const double* p, const double* q, double* partial,
                      double* scal, float* r32, hipStream_t s);
// As krylov_dot (op 1) and krylov_update_p with z = zl * (scaled ? scal[8] / mul : 1),
// read from a reduced-precision cycle's output.
template <typename T>
void krylov_dot_lowz(size_t n, const T* zl, int scaled, double mul, const double* r, const double* rold,
                     double* partial, double* scal, int first, hipStream_t s);
template <typename T>
void krylov_update_p_lowz(size_t n, const T* zl, int scaled, double mul, double* p, const double* scal,
                          hipStream_t s);
// y = x * scal[7] * mul (scal null: y = x * mul)
template <typename T>
void cast_down(size_t n, const double* x, T* y, const double* scal, double mul, hipStream_t s);
template <typename T>
void cast_up(size_t n, const T* x, double* y, const double* scal, double mul, hipStream_t s);

}  // namespace hpmg
