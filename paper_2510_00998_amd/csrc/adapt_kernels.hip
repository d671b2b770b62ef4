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
// So the sweep and apply kernels treat every facet as conforming.  The remap
// moves (m + 1) 2 (p+1)^(d-1) values in and out per interface, a few per cent
// of a sweep's bytes when hanging facets are a small part of the skeleton.
#include <algorithm>

#include "kernels.hpp"

namespace hpmg {
namespace {

// One workgroup per interface: the m + 1 source traces (the fine cells' own
// slots, then the coarse cell's) and the tables are staged in LDS with
// coalesced loads; the tensor-product maps run as two 1D contractions
// (3D: along the first tangential axis into LDS, then along the second).
constexpr int REMAP_THREADS = 256;
template <int D, int N>
constexpr int remap_lds_values(int r) {
  // sources (m+1) 2L, first-stage results (r + m) 2 N^2 (3D), tables 2 r N^2
  return (D == 2 ? (r + 1) * 2 * N : (r * r + 1) * 2 * N * N + (r + r * r) * 2 * N * N) + 2 * r * N * N;
}
template <typename T, int D, int N>
__global__ __launch_bounds__(REMAP_THREADS) void k_remap(T* tr, long long tstride, const int* itab, int m, int r,
                                                         int ncell, const CT<T>* mort) {
  using C = CT<T>;
  constexpr int L = D == 2 ? N : N * N;
  constexpr int TL = 2 * L;
  constexpr int NN = N * N;
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  C* sSrc = (C*)lds_raw;                   // [m + 1][2L]: fine cells 0..m-1, coarse cell m
  C* sMat = sSrc + (m + 1) * TL;           // [I_0 .. I_{r-1} | P_0 .. P_{r-1}]
  C* sTmp = sMat + 2 * r * NN;             // 3D: [r + m][2][N][N]
  T* t = tr + (size_t)blockIdx.y * tstride;
  const int i = blockIdx.x;
  const int* row = itab + (size_t)i * (2 + m);
  const int B = row[0], fB = row[1];
  const int tid = threadIdx.x;
  for (int e = tid; e < (m + 1) * TL; e += REMAP_THREADS) {
    const int j = e / TL, o = e % TL;
    const size_t slot = j < m ? (size_t)(fB ^ 1) * ncell + row[2 + j] : (size_t)fB * ncell + B;
    sSrc[e] = (C)t[slot * TL + o];
  }
  for (int e = tid; e < 2 * r * NN; e += REMAP_THREADS) sMat[e] = mort[e];
  __syncthreads();
  const C* sI = sMat;
  const C* sP = sMat + r * NN;
  const C qf = C(1) / C(r);
  const size_t base = (size_t)2 * D * ncell + (size_t)i * (m + 1);
  if constexpr (D == 2) {
    // fine slot j: I_j g_B; coarse slot: sum_j P_j g_j
    for (int e = tid; e < (m + 1) * TL; e += REMAP_THREADS) {
      const int j = e / TL, o = e % TL, f = o / L, a = o % L;
      C acc = 0;
      if (j < m) {
        const C* src = sSrc + m * TL + f * L;
#pragma unroll
        for (int x = 0; x < N; ++x) acc += sI[(j * N + a) * N + x] * src[x];
        if (f) acc *= qf;
      } else {
        for (int s = 0; s < m; ++s) {
          const C* src = sSrc + s * TL + f * L;
#pragma unroll
          for (int x = 0; x < N; ++x) acc += sP[(s * N + a) * N + x] * src[x];
        }
        if (f) acc *= C(r);
      }
      t[(base + j) * TL + o] = (T)acc;
    }
  } else {
    // first tangential axis: tmp[q][f][a][y] = sum_x M[a][x] src[f][x + N y]
    // with (q < r) M = I_q on the coarse trace, (q = r + s) M = P_{s mod r}
    // on fine trace s
    const int nq = r + m;
    for (int e = tid; e < nq * 2 * NN; e += REMAP_THREADS) {
      const int q = e / (2 * NN), rem = e % (2 * NN), f = rem / NN, ay = rem % NN, a = ay % N, y = ay / N;
      const C* M = q < r ? sI + (q * N + a) * N : sP + (((q - r) % r) * N + a) * N;
      const C* src = sSrc + (q < r ? m : q - r) * TL + f * L + N * y;
      C acc = 0;
#pragma unroll
      for (int x = 0; x < N; ++x) acc += M[x] * src[x];
      sTmp[e] = acc;
    }
    __syncthreads();
    // second axis: fine slot j = (sa, sb): sum_y I_sb[b][y] tmp[sa][f][a][y];
    // coarse slot: sum_s sum_y P_{sb(s)}[b][y] tmp[r + s][f][a][y]
    for (int e = tid; e < (m + 1) * TL; e += REMAP_THREADS) {
      const int j = e / TL, o = e % TL, f = o / L, l = o % L, a = l % N, b = l / N;
      C acc = 0;
      if (j < m) {
        const int sa = j % r, sb = j / r;
        const C* M = sI + (sb * N + b) * N;
        const C* tmp = sTmp + (sa * 2 + f) * NN + a;
#pragma unroll
        for (int y = 0; y < N; ++y) acc += M[y] * tmp[N * y];
        if (f) acc *= qf;
      } else {
        for (int s = 0; s < m; ++s) {
          const C* M = sP + ((s / r) * N + b) * N;
          const C* tmp = sTmp + ((r + s) * 2 + f) * NN + a;
#pragma unroll
          for (int y = 0; y < N; ++y) acc += M[y] * tmp[N * y];
        }
        if (f) acc *= C(r);
      }
      t[(base + j) * TL + o] = (T)acc;
    }
  }
}

// Transfers between two spacetree levels of the same degree (the coarser
// leaf set merges the deepest leaves into their parents).  A fine cell is
// either a coarse cell itself or the child at position (px, py, pz) of a
// coarse cell, whose polynomial restricted to the child is the tensor
// product of I_px, I_py, I_pz (I_j[a][b] = l_b((xi_a + j)/r), the first r
// tables of the level's remap data).  pmap[fine] = 32 coarse + child
// position (31: the same cell); rmap[coarse][r^d] = fine cells by child
// position (the same cell: [fine, -1, ...]).  One workgroup per cell, one
// thread per node, the 1D contractions through LDS.
template <typename C, int D, int N>
__device__ __forceinline__ void tensor_apply(const C* I, int r, int pos, bool transpose, C* s0, C* s1, int tid) {
  // s0 -> s0 (through s1): along x with I_px, along y with I_py (, z with I_pz),
  // I or I^T; s0 holds [c][b][a] with a fastest
  constexpr int NV = D == 2 ? N * N : N * N * N;
  const int pxyz[3] = {pos % r, (pos / r) % r, pos / (r * r)};
  C* src = s0;
  C* dst = s1;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const C* M = I + (size_t)pxyz[k] * N * N;
    const int st = k == 0 ? 1 : (k == 1 ? N : N * N);
    if (tid < NV) {
      const int j = (tid / st) % N, base = tid - j * st;
      C acc = 0;
#pragma unroll
      for (int x = 0; x < N; ++x) acc += (transpose ? M[x * N + j] : M[j * N + x]) * src[base + x * st];
      dst[tid] = acc;
    }
    __syncthreads();
    C* t = src;
    src = dst;
    dst = t;
  }
  if (src != s0) {  // D odd: the result is in s1
    if (tid < NV) s0[tid] = src[tid];
    __syncthreads();
  }
}

template <typename C, int D, int N>
__global__ void k_hprolong(C* uf, const C* ec, const int* pmap, int r, const C* I, long long fstride,
                           long long cstride) {
  constexpr int NV = D == 2 ? N * N : N * N * N;
  __shared__ C s0[NV], s1[NV];
  const int f = blockIdx.x, tid = threadIdx.x;
  uf += (size_t)blockIdx.y * fstride;
  ec += (size_t)blockIdx.y * cstride;
  const int pm = pmap[f], c = pm >> 5, pos = pm & 31;
  if (pos == 31) {
    if (tid < NV) uf[(size_t)f * NV + tid] += ec[(size_t)c * NV + tid];
    return;
  }
  if (tid < NV) s0[tid] = ec[(size_t)c * NV + tid];
  __syncthreads();
  tensor_apply<C, D, N>(I, r, pos, false, s0, s1, tid);
  if (tid < NV) uf[(size_t)f * NV + tid] += s0[tid];
}

template <typename C, int D, int N>
__global__ void k_hrestrict(const C* rf, C* bc, const int* rmap, int r, const C* I, long long fstride,
                            long long cstride) {
  constexpr int NV = D == 2 ? N * N : N * N * N;
  __shared__ C s0[NV], s1[NV];
  const int c = blockIdx.x, tid = threadIdx.x;
  rf += (size_t)blockIdx.y * fstride;
  bc += (size_t)blockIdx.y * cstride;
  const int rd = D == 2 ? r * r : r * r * r;
  const int* row = rmap + (size_t)c * rd;
  if (row[1] < 0) {
    if (tid < NV) bc[(size_t)c * NV + tid] = rf[(size_t)row[0] * NV + tid];
    return;
  }
  C acc = 0;
  for (int q = 0; q < rd; ++q) {
    if (tid < NV) s0[tid] = rf[(size_t)row[q] * NV + tid];
    __syncthreads();
    tensor_apply<C, D, N>(I, r, q, true, s0, s1, tid);
    if (tid < NV) acc += s0[tid];
    __syncthreads();
  }
  if (tid < NV) bc[(size_t)c * NV + tid] = acc;
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

template <typename T, int D, int N>
void remap_launch(int ncell, int nif, int m, int r, const int* itab, const CT<T>* mort, T* tr, long long tstride,
                  int nrhs, hipStream_t s) {
  const size_t lds = sizeof(CT<T>) * (size_t)remap_lds_values<D, N>(r);
  hipLaunchKernelGGL((k_remap<T, D, N>), dim3(nif, nrhs), dim3(REMAP_THREADS), lds, s, tr, tstride, itab, m, r,
                     ncell, mort);
}

template <typename T>
void remap_hanging(int D, int N, int ncell, int nif, int m, int r, const int* itab, const CT<T>* mort, T* tr,
                   long long tstride, int nrhs, hipStream_t s) {
  if (nif == 0) return;
  using F = void (*)(int, int, int, int, const int*, const CT<T>*, T*, long long, int, hipStream_t);
  static const F tab2[10] = {nullptr, nullptr, remap_launch<T, 2, 2>, remap_launch<T, 2, 3>, remap_launch<T, 2, 4>,
                             remap_launch<T, 2, 5>, remap_launch<T, 2, 6>, remap_launch<T, 2, 7>,
                             remap_launch<T, 2, 8>, remap_launch<T, 2, 9>};
  static const F tab3[10] = {nullptr, nullptr, remap_launch<T, 3, 2>, remap_launch<T, 3, 3>, remap_launch<T, 3, 4>,
                             remap_launch<T, 3, 5>, remap_launch<T, 3, 6>, remap_launch<T, 3, 7>,
                             remap_launch<T, 3, 8>, remap_launch<T, 3, 9>};
  if (N < 2 || N > 9) return;
  (D == 2 ? tab2 : tab3)[N](ncell, nif, m, r, itab, mort, tr, tstride, nrhs, s);
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

template <typename C, int D, int N>
void htransfer_launch(bool restrict_, int ncells, const int* map, int r, const C* I, const C* src, C* dst,
                      long long fstride, long long cstride, int nrhs, hipStream_t s) {
  constexpr int NV = D == 2 ? N * N : N * N * N;
  const dim3 grid(ncells, nrhs), blk((NV + 63) / 64 * 64);
  if (restrict_)
    hipLaunchKernelGGL((k_hrestrict<C, D, N>), grid, blk, 0, s, src, dst, map, r, I, fstride, cstride);
  else
    hipLaunchKernelGGL((k_hprolong<C, D, N>), grid, blk, 0, s, dst, src, map, r, I, fstride, cstride);
}

template <typename C>
void spacetree_transfer(bool restrict_, int D, int N, int ncells, const int* map, int r, const C* I, const C* src,
                        C* dst, long long fstride, long long cstride, int nrhs, hipStream_t s) {
  if (ncells == 0) return;
  using F = void (*)(bool, int, const int*, int, const C*, const C*, C*, long long, long long, int, hipStream_t);
  static const F tab2[10] = {nullptr, nullptr, htransfer_launch<C, 2, 2>, htransfer_launch<C, 2, 3>,
                             htransfer_launch<C, 2, 4>, htransfer_launch<C, 2, 5>, htransfer_launch<C, 2, 6>,
                             htransfer_launch<C, 2, 7>, htransfer_launch<C, 2, 8>, htransfer_launch<C, 2, 9>};
  static const F tab3[10] = {nullptr, nullptr, htransfer_launch<C, 3, 2>, htransfer_launch<C, 3, 3>,
                             htransfer_launch<C, 3, 4>, htransfer_launch<C, 3, 5>, htransfer_launch<C, 3, 6>,
                             htransfer_launch<C, 3, 7>, htransfer_launch<C, 3, 8>, htransfer_launch<C, 3, 9>};
  if (N < 2 || N > 9) return;
  (D == 2 ? tab2 : tab3)[N](restrict_, ncells, map, r, I, src, dst, fstride, cstride, nrhs, s);
}
template void spacetree_transfer<double>(bool, int, int, int, const int*, int, const double*, const double*, double*,
                                         long long, long long, int, hipStream_t);
template void spacetree_transfer<float>(bool, int, int, int, const int*, int, const float*, const float*, float*,
                                        long long, long long, int, hipStream_t);

}  // namespace hpmg
