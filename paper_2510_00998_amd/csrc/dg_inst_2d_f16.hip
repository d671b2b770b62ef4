// Instantiation of the DG cell kernels for dim = 2, storage type _Float16.
#include "dg_inst.hpp"

namespace hpmg {
bool dg_dispatch2(int N, int op, const DGArgs<_Float16>& a, int nrhs, int flag, hipStream_t s) {
  return inst::dispatch<_Float16, 2>(N, op, a, nrhs, flag, s);
}
}  // namespace hpmg
