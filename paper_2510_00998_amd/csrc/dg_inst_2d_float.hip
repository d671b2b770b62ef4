// Instantiation of the DG cell kernels for dim = 2, float.
#include "dg_kernels_impl.hpp"
#include "kernels.hpp"

namespace hpmg {
namespace {
template <int N>
void run(int op, const DGArgs<float>& a, int nrhs, int flag, hipStream_t s) {
  constexpr int NC = nc_next(N);
  switch (op) {
    case OP_SWEEP: launch_sweep<float, 2, N>(a, nrhs, flag != 0, s); break;
    case OP_APPLY: launch_apply<float, 2, N, 0>(a, nrhs, flag != 0, s); break;
    case OP_RESTRICT: launch_apply<float, 2, N, NC>(a, nrhs, true, s); break;
    case OP_PROJECT: launch_prolong<float, 2, N, 0>(a, nrhs, s); break;
    case OP_PROLONG: launch_prolong<float, 2, N, NC>(a, nrhs, s); break;
    default: break;
  }
}
}  // namespace

bool dg_dispatch2(int N, int op, const DGArgs<float>& a, int nrhs, int flag, hipStream_t s) {
  switch (N) {
    case 2: run<2>(op, a, nrhs, flag, s); return true;
    case 3: run<3>(op, a, nrhs, flag, s); return true;
    case 4: run<4>(op, a, nrhs, flag, s); return true;
    case 5: run<5>(op, a, nrhs, flag, s); return true;
    case 6: run<6>(op, a, nrhs, flag, s); return true;
    case 7: run<7>(op, a, nrhs, flag, s); return true;
    case 8: run<8>(op, a, nrhs, flag, s); return true;
    case 9: run<9>(op, a, nrhs, flag, s); return true;
    default: return false;
  }
}
}  // namespace hpmg
