// Instantiation of the DG cell kernels for dim = 2, storage type __bf16.
#include "dg_inst.hpp"

namespace hpmg {
bool dg_dispatch2(int N, int op, const DGArgs<__bf16>& a, int nrhs, int flag, hipStream_t s) {
  return inst::dispatch<__bf16, 2>(N, op, a, nrhs, flag, s);
}
}  // namespace hpmg
