// Batched execution of many independent problems (different meshes,
// degrees and right-hand sides) through persistent launches that walk a
// work list: one launch per multigrid phase for every problem at once.
#pragma once
#include <hip/hip_runtime.h>

#include "dg_kernels.hpp"

namespace hpmg {

// Operations of the batched DG kernel (3D, constant kappa, 2 <= N <= 6).
enum BatchDGOp {
  BOP_SWEEP = 0,     // fused sweep
  BOP_SWEEP0 = 1,    // fused sweep with u = 0 on entry
  BOP_RESTRICT = 2,  // r = b - A u restricted to the next coarser level
  BOP_PROLONG = 3,   // u += P e, then traces
  BOP_PROJECT = 4,   // traces of u
  BOP_RESID = 5,     // r = b - A u (no restriction)
  BOP_APPLY = 6      // y = A u
};
constexpr int BATCH_NMIN = 2, BATCH_NMAX = 6;

// Work item of a batched launch: x = index into the argument table,
// y = cell block (DG) or vertex block (Q1), z = right-hand side, w = N (DG).
using WorkItem = int4;

// Operations of the batched Q1 kernel.
enum BatchCGOp {
  CGOP_JACOBI = 0,    // out = u + omega Dinv (b - A u)
  CGOP_RESID = 1,     // out = b - A u
  CGOP_RESTRICT = 2,  // out = P^T in       (in: fine residual, out: coarse rhs)
  CGOP_PROLONG = 3,   // out += P in        (in: coarse solution, out: fine u)
  CGOP_GATHER = 4,    // out = sum of the per-cell corner contributions in
  CGOP_DENSE = 5      // out = Ainv in      (coarsest level)
};

template <typename T>
struct CGArgs {
  int op, nv, nvc, n, uzero, m;
  T omega;
  const T* st;
  const T* dinv;
  const T* u;
  const T* b;
  T* out;
  const T* in;
  const int* idx;
  const T* w;
  const double* Ainv;
  long long su, sb, sout, sin;  // per right-hand side strides
};

// Segments of the outer FP64 iteration: one per (problem, right-hand side).
struct SegTable {
  const long long* off;   // offset of the segment in the workspace vectors
  const int* len;         // its length
  double* const* u;       // caller's solution vector of the segment
  const double* const* b; // caller's right-hand side of the segment
  const int2* chunks;     // (segment, first element) of every chunk
  const int* cstart;      // first chunk of each segment
  const int* ccount;      // chunk count of each segment
  int nseg, nchunks;
};
constexpr int BATCH_CHUNK = 16384;
constexpr int BATCH_SCAL = 16;  // doubles of per-segment scalar state
constexpr double BATCH_MAX_RESTARTS = 3;  // restarts from the true residual per segment

template <typename T>
void batch_dg(int op, const DGArgs<T>* args, const WorkItem* items, int nitems, int grid, hipStream_t s);
// The same with one kernel per degree N (items must all have w = N) and the
// cells per block of tile variant 0 or 1 (DGShapeV; the items' cell blocks
// must be those of that variant).
template <typename T>
void batch_dg_n_t0(int op, int N, const DGArgs<T>* args, const WorkItem* items, int nitems, int grid, hipStream_t s);
template <typename T>
void batch_dg_n_t1(int op, int N, const DGArgs<T>* args, const WorkItem* items, int nitems, int grid, hipStream_t s);
template <typename T>
void batch_cg(const CGArgs<T>* args, const WorkItem* items, int nitems, int grid, hipStream_t s);

// Segmented FP64 vector operations of the flexible CG (see batch_kernels.hip).
void bk_dot(const SegTable& t, const double* x, const double* y, const double* z, double* partial, hipStream_t s);
void bk_dot_z(const SegTable& t, const float* z32, const double* r, const double* q, const double* scal,
              double* partial, hipStream_t s);
void bk_finalize(const SegTable& t, int op, const double* partial, double* scal, double rtol2, hipStream_t s);
void bk_update_p(const SegTable& t, const float* z32, double* p, const double* scal, hipStream_t s);
void bk_update_ur(const SegTable& t, double* r, float* r32, const double* p, const double* q, const double* scal,
                  double* partial, hipStream_t s);
void bk_cast_down(const SegTable& t, const double* x, float* y, const double* scal, hipStream_t s);
void bk_count(const SegTable& t, const double* scal, int* count, hipStream_t s);
void bk_select(const SegTable& t, const double* q, double* r, const double* scal, hipStream_t s);

}  // namespace hpmg
