// Instantiation of the DG cell kernels for dim = 3, storage type double.
#include "dg_inst.hpp"

namespace hpmg {
bool dg_dispatch3(int N, int op, const DGArgs<double>& a, int nrhs, int flag, hipStream_t s) {
  return inst::dispatch<double, 3>(N, op, a, nrhs, flag, s);
}
}  // namespace hpmg
