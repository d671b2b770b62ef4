// Adaptive (spacetree) meshes: the trace remap across hanging facets and
// the sparse transfers between the DG leaves and the Q1 base mesh.
//
// Hanging facet (paper Section 2.1: leaves of one spacetree level meet
// leaves one level finer): the facet f_B of the coarse cell B is covered by
// m = r^(d-1) facets of fine cells F_s, s = s_a + r s_b over the positions
// along the two tangential axes (increasing axis order).  Every cell writes
// its own traces (value g, reference-unit normal derivative q = h du/dn)
// into its own slot f ncell + c.  After each traversal that writes traces,
// k_remap fills the interface's m + 1 slots (base = 2 d ncell + i (m + 1)):
//   slot base + s (read by F_s): B's traces restricted to F_s's facet,
//     (I_{s_a} x I_{s_b}) g_B and (I x I) q_B / r, I_j[a][b] = l_b((xi_a + j)/r)
//     (B's facet polynomial evaluated at F_s's facet nodes; q into the fine
//     cell's units);
//   slot base + m (read by B): sum_s (P_{s_a} x P_{s_b}) g_{F_s} and the
//     same of r q_{F_s}, P_j = (1/r) Mhat^-1 I_j^T Mhat: the L2 projection
//     of the piecewise polynomial fine traces onto B's facet polynomials.
// Both are exact for the terms the cells form from them: a fine cell
// integrates over its own facet, where B's trace is a polynomial of its
// degree; B integrates over its whole facet against its own test functions
// (degree p on the facet), for which the projection changes no integral.
// So the sweep and apply kernels treat every facet as conforming.
#include <algorithm>

#include "kernels.hpp"

namespace hpmg {
namespace {

template <typename T>
__global__ void k_remap(T* tr, long long tstride, const int* itab, int nif, int m, int r, int ncell, int D, int N,
                        const CT<T>* mort) {
  using C = CT<T>;
  const int L = D == 2 ? N : N * N;
  const int TL = 2 * L;
  const long long items = (long long)nif * (m + 1) * L;
  T* t = tr + (size_t)blockIdx.y * tstride;
  const size_t base0 = (size_t)2 * D * ncell;
  const C* Ir = mort;                      // [r][N][N]
  const C* Pj = mort + (size_t)r * N * N;  // [r][N][N]
  const C qf = C(1) / C(r);
  for (long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x; it < items;
       it += (long long)gridDim.x * blockDim.x) {
    const int l = (int)(it % L);
    const int j = (int)((it / L) % (m + 1));
    const long long i = it / ((long long)L * (m + 1));
    const int* row = itab + (size_t)i * (2 + m);
    const int B = row[0], fB = row[1];
    const int a = l % N, b = l / N;  // b = 0 in 2D
    C g = 0, q = 0;
    if (j < m) {
      const int sa = j % r, sb = j / r;
      const T* src = t + ((size_t)fB * ncell + B) * TL;
      const C* Ia = Ir + ((size_t)sa * N + a) * N;
      if (D == 2) {
        for (int x = 0; x < N; ++x) {
          g += Ia[x] * (C)src[x];
          q += Ia[x] * (C)src[L + x];
        }
      } else {
        const C* Ib = Ir + ((size_t)sb * N + b) * N;
        for (int y = 0; y < N; ++y) {
          C gy = 0, qy = 0;
          for (int x = 0; x < N; ++x) {
            gy += Ia[x] * (C)src[x + N * y];
            qy += Ia[x] * (C)src[L + x + N * y];
          }
          g += Ib[y] * gy;
          q += Ib[y] * qy;
        }
      }
      q *= qf;
    } else {
      for (int s = 0; s < m; ++s) {
        const int sa = s % r, sb = s / r;
        const T* src = t + ((size_t)(fB ^ 1) * ncell + row[2 + s]) * TL;
        const C* Pa = Pj + ((size_t)sa * N + a) * N;
        if (D == 2) {
          for (int x = 0; x < N; ++x) {
            g += Pa[x] * (C)src[x];
            q += Pa[x] * (C)src[L + x];
          }
        } else {
          const C* Pb = Pj + ((size_t)sb * N + b) * N;
          for (int y = 0; y < N; ++y) {
            C gy = 0, qy = 0;
            for (int x = 0; x < N; ++x) {
              gy += Pa[x] * (C)src[x + N * y];
              qy += Pa[x] * (C)src[L + x + N * y];
            }
            g += Pb[y] * gy;
            q += Pb[y] * qy;
          }
        }
      }
      q *= C(r);
    }
    T* dst = t + (base0 + (size_t)i * (m + 1) + j) * TL;
    dst[l] = (T)g;
    dst[L + l] = (T)q;
  }
}

// y[i] = sum over e in [ptr[i], ptr[i+1]) of w[e] x[col[e]]
template <typename T>
__global__ void k_csr(int nrow, const int* ptr, const int* col, const T* w, const T* x, T* y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nrow; i += gridDim.x * blockDim.x) {
    T s = 0;
    for (int e = ptr[i]; e < ptr[i + 1]; ++e) s += w[e] * x[col[e]];
    y[i] = s;
  }
}

}  // namespace

template <typename T>
void remap_hanging(int D, int N, int ncell, int nif, int m, int r, const int* itab, const CT<T>* mort, T* tr,
                   long long tstride, int nrhs, hipStream_t s) {
  if (nif == 0) return;
  const int L = D == 2 ? N : N * N;
  const long long items = (long long)nif * (m + 1) * L;
  const int blocks = (int)std::min<long long>((items + 255) / 256, 4096);
  hipLaunchKernelGGL((k_remap<T>), dim3(blocks, nrhs), dim3(256), 0, s, tr, tstride, itab, nif, m, r, ncell, D,
                     N, mort);
}
template void remap_hanging<double>(int, int, int, int, int, int, const int*, const double*, double*, long long, int,
                                    hipStream_t);
template void remap_hanging<float>(int, int, int, int, int, int, const int*, const float*, float*, long long, int,
                                   hipStream_t);

template <typename T>
void csr_apply(int nrow, const int* ptr, const int* col, const T* w, const T* x, T* y, hipStream_t s) {
  if (nrow == 0) return;
  const int blocks = std::min((nrow + 255) / 256, 4096);
  hipLaunchKernelGGL((k_csr<T>), dim3(blocks), dim3(256), 0, s, nrow, ptr, col, w, x, y);
}
template void csr_apply<double>(int, const int*, const int*, const double*, const double*, double*, hipStream_t);
template void csr_apply<float>(int, const int*, const int*, const float*, const float*, float*, hipStream_t);

}  // namespace hpmg
