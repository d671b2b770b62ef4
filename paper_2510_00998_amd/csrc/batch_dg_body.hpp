// Batched DG work items and the one-degree persistent kernels, compiled once
// per tile variant (HPMG_TILE, cells per block; see DGShapeV): included by
// batch_kernels.hip (variant 0) and batch_tile1.hip (variant 1).
#pragma once
#include "batch.hpp"
#include "dg_kernels_impl.hpp"
#include "kernels.hpp"

namespace hpmg {
namespace {

template <typename T, int N, int OP>
__device__ __forceinline__ void dg_item(const DGArgs<T>& a, int bx, int by, char* lds) {
  constexpr int NC = nc_next(N);
  if constexpr (OP == BOP_SWEEP)
    HPMG_DGK::sweep_body<T, 3, N, false, false>(a, bx, by, lds);
  else if constexpr (OP == BOP_SWEEP0)
    HPMG_DGK::sweep_body<T, 3, N, true, false>(a, bx, by, lds);
  else if constexpr (OP == BOP_RESTRICT)
    HPMG_DGK::apply_body<T, 3, N, NC, true, false>(a, bx, by, lds);
  else if constexpr (OP == BOP_PROLONG)
    HPMG_DGK::prolong_body<T, 3, N, NC>(a, bx, by, lds);
  else if constexpr (OP == BOP_PROJECT)
    HPMG_DGK::prolong_body<T, 3, N, 0>(a, bx, by, lds);
  else if constexpr (OP == BOP_RESID)
    HPMG_DGK::apply_body<T, 3, N, 0, true, false>(a, bx, by, lds);
  else
    HPMG_DGK::apply_body<T, 3, N, 0, false, false>(a, bx, by, lds);
}

template <typename T, int N, int OP>
constexpr int item_lds() {
  if constexpr (OP == BOP_PROLONG)
    return HPMG_DGK::prolong_lds_bytes<T, 3, N, nc_next(N)>();
  else if constexpr (OP == BOP_PROJECT)
    return HPMG_DGK::prolong_lds_bytes<T, 3, N, 0>();
  else
    return HPMG_DGK::cell_lds_bytes<T, 3, N, false>();
}

inline unsigned grid_for_n(int n, int cap) { return (unsigned)(n < cap ? (n > 0 ? n : 1) : cap); }

// One degree per launch: the kernel takes only that degree's registers and
// LDS (items of other degrees are not expected in its list).  ONE: the grid
// covers the list, one item per block and no item loop (the loop alone
// takes the FP64 items of degree 3 and 4 from 114 and 109 to 134 and 165
// VGPRs, three waves per SIMD instead of four).
template <typename T, int OP, int N, int V, bool ONE>
__global__ __launch_bounds__((HPMG_DGK::DGShape<3, N>::BLOCK)) void k_dg_batch_n(const DGArgs<T>* __restrict__ args,
                                                                          const WorkItem* __restrict__ items,
                                                                          int nitems) {
  __shared__ __attribute__((aligned(16))) char lds[item_lds<T, N, OP>()];
  if constexpr (ONE) {
    const WorkItem w = items[blockIdx.x];
    const DGArgs<T> a = args[w.x];
    dg_item<T, N, OP>(a, w.y, w.z, lds);
  } else {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
      const WorkItem w = items[it];
      const DGArgs<T> a = args[w.x];
      dg_item<T, N, OP>(a, w.y, w.z, lds);
      __syncthreads();  // the next item reuses the LDS
    }
  }
}

}  // namespace

namespace {
template <typename T, int OP, int N, bool ONE>
void launch_n1(const DGArgs<T>* args, const WorkItem* items, int nitems, dim3 g, hipStream_t s) {
  hipLaunchKernelGGL((k_dg_batch_n<T, OP, N, HPMG_TILE, ONE>), g, dim3(HPMG_DGK::DGShape<3, N>::BLOCK), 0, s, args,
                     items, nitems);
}

template <typename T, int OP, bool ONE>
void launch_nd(int N, const DGArgs<T>* args, const WorkItem* items, int nitems, dim3 g, hipStream_t s) {
  switch (N) {
    case 2: launch_n1<T, OP, 2, ONE>(args, items, nitems, g, s); break;
    case 3: launch_n1<T, OP, 3, ONE>(args, items, nitems, g, s); break;
    case 4: launch_n1<T, OP, 4, ONE>(args, items, nitems, g, s); break;
    case 5: launch_n1<T, OP, 5, ONE>(args, items, nitems, g, s); break;
    default: launch_n1<T, OP, 6, ONE>(args, items, nitems, g, s); break;
  }
}

// A grid of exactly one block per item takes the loop-free kernel.
template <typename T, int OP>
void launch_n(int N, const DGArgs<T>* args, const WorkItem* items, int nitems, dim3 g, hipStream_t s) {
  if (nitems > 0 && g.x == (unsigned)nitems)
    launch_nd<T, OP, true>(N, args, items, nitems, g, s);
  else
    launch_nd<T, OP, false>(N, args, items, nitems, g, s);
}

}  // namespace

#define HPMG_BATCH_CAT2(a, b) a##b
#define HPMG_BATCH_CAT(a, b) HPMG_BATCH_CAT2(a, b)
#define HPMG_BATCH_DG_N HPMG_BATCH_CAT(batch_dg_n_t, HPMG_TILE)

template <typename T>
void HPMG_BATCH_DG_N(int op, int N, const DGArgs<T>* args, const WorkItem* items, int nitems, int grid, hipStream_t s) {
  const dim3 g(grid_for_n(nitems, grid));
  switch (op) {
    case BOP_SWEEP: launch_n<T, BOP_SWEEP>(N, args, items, nitems, g, s); break;
    case BOP_SWEEP0: launch_n<T, BOP_SWEEP0>(N, args, items, nitems, g, s); break;
    case BOP_RESTRICT: launch_n<T, BOP_RESTRICT>(N, args, items, nitems, g, s); break;
    case BOP_PROLONG: launch_n<T, BOP_PROLONG>(N, args, items, nitems, g, s); break;
    case BOP_PROJECT: launch_n<T, BOP_PROJECT>(N, args, items, nitems, g, s); break;
    case BOP_RESID: launch_n<T, BOP_RESID>(N, args, items, nitems, g, s); break;
    default: launch_n<T, BOP_APPLY>(N, args, items, nitems, g, s); break;
  }
}
template void HPMG_BATCH_DG_N<float>(int, int, const DGArgs<float>*, const WorkItem*, int, int, hipStream_t);
template void HPMG_BATCH_DG_N<double>(int, int, const DGArgs<double>*, const WorkItem*, int, int, hipStream_t);

}  // namespace hpmg
