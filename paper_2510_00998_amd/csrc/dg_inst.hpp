// Shared body of the per-(type, dimension) instantiation files: dispatch of
// a DG operation to the kernel of degree N - 1.
#pragma once
#include "dg_kernels_impl.hpp"
#include "kernels.hpp"

namespace hpmg {
namespace inst {

template <typename T, int D, int N>
void run(int op, const DGArgs<T>& a, int nrhs, int flag, hipStream_t s) {
  constexpr int NC = nc_next(N);
  switch (op) {
    case OP_SWEEP: launch_sweep<T, D, N>(a, nrhs, flag != 0, s); break;
    case OP_APPLY: launch_apply<T, D, N, 0>(a, nrhs, flag != 0, s); break;
    case OP_RESTRICT: launch_apply<T, D, N, NC>(a, nrhs, true, s); break;
    case OP_PROJECT: launch_prolong<T, D, N, 0>(a, nrhs, s); break;
    case OP_PROLONG: launch_prolong<T, D, N, NC>(a, nrhs, s); break;
    case OP_RESTRICT_Q1: launch_apply<T, D, N, 2>(a, nrhs, true, s); break;
    case OP_PROLONG_Q1: launch_prolong<T, D, N, 2>(a, nrhs, s); break;
    case OP_RESTRICT_DYN:
      if constexpr (N >= 4) launch_apply<T, D, N, -1>(a, nrhs, true, s);
      break;
    case OP_PROLONG_DYN:
      if constexpr (N >= 4) launch_prolong<T, D, N, -1>(a, nrhs, s);
      break;
    case OP_BUILD_EIG:
      if constexpr (std::is_same<T, double>::value || std::is_same<T, float>::value) launch_build_eig<T, D, N>(a, s);
      break;
    default: break;
  }
}

template <typename T, int D>
bool dispatch(int N, int op, const DGArgs<T>& a, int nrhs, int flag, hipStream_t s) {
  switch (N) {
    case 2: run<T, D, 2>(op, a, nrhs, flag, s); return true;
    case 3: run<T, D, 3>(op, a, nrhs, flag, s); return true;
    case 4: run<T, D, 4>(op, a, nrhs, flag, s); return true;
    case 5: run<T, D, 5>(op, a, nrhs, flag, s); return true;
    case 6: run<T, D, 6>(op, a, nrhs, flag, s); return true;
    case 7: run<T, D, 7>(op, a, nrhs, flag, s); return true;
    case 8: run<T, D, 8>(op, a, nrhs, flag, s); return true;
    case 9: run<T, D, 9>(op, a, nrhs, flag, s); return true;
    default: return false;
  }
}

}  // namespace inst
}  // namespace hpmg
