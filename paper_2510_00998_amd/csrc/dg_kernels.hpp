// Matrix-free SIPG kernels on DG levels (gfx950).
//
// One thread per 1D line of a cell ("pencil"): a cell of N^d nodes owns
// N^(d-1) threads; a block holds CPB whole cells (about 256 threads).  The
// block stages the cell data of its cells, which are consecutive in memory,
// through LDS with coalesced loads, applies sum-factorised 1D contractions
// along x, y, z with the line in registers, and writes back coalesced.
//
// Operator (paper Section 2.3.1 eq. weak_form_IP with theta = -1 and the
// facet form eq. weak_form_IP_facet_spaces): in reference units the cell
// block is the Kronecker sum A_{K<-K} = h^(d-2) sum_k M x .. x L_k x .. x M,
// L_k = kappa_K Khat + facet terms of the two facets normal to axis k.  The
// neighbour coupling enters only through the traces (value g and outward
// normal derivative q = h du/dn) that each neighbour projected onto the
// shared facet (technique projection-variables); the flux variables
// w = kappa_F (q'/2 - sigma_hat g') and w' = kappa_F g'/2 (technique
// numerical-flux-outcome) are formed in registers and lifted back with the
// facet mass.  The block inverse uses the fast diagonalisation
// A_{K<-K}^{-1} = h^(2-d) (S x S x S) diag(1/(lx+ly+lz)) (S x S x S)^T with
// L_k S = M S diag(l), S^T M S = I.
//
// Sweep (technique shift-and-fuse, Algorithm BlockJacobi with loop fusion):
// each cell reads its own u, b and the neighbours' old traces, computes
//   u_new = (1-omega) u + omega A_{K<-K}^{-1} (b - A_{c<-f} w),
// which equals u + omega A_{K<-K}^{-1}(b - A u) (block-Jacobi, eq.
// block-Jacobi-IP) because A_{K<-K}^{-1} A_{K<-K} u = u, and writes u_new
// and its traces into the other trace buffer (ping-pong, so every cell of a
// sweep sees old traces: Jacobi semantics without a copy of u).
#pragma once
#include <hip/hip_runtime.h>

namespace hpmg {

// Cells per block: about 256 threads, unless a build overrides the 3D cell
// count per block for one degree (HPMG_CPB3D_N / HPMG_CPB3D, tile tuning).
#ifndef HPMG_CPB3D_N
#define HPMG_CPB3D_N 0
#define HPMG_CPB3D 0
#endif
__host__ __device__ constexpr int cells_per_block(int D, int N) {
  return (D == 3 && N == HPMG_CPB3D_N) ? HPMG_CPB3D
                                       : ((256 / (D == 2 ? N : N * N)) > 0 ? (256 / (D == 2 ? N : N * N)) : 1);
}
// Tile variants of a cell-block kernel (picked by the batched driver's
// autotuner): V = 0 the cells of about 256 threads, V = 1 half as many
// cells (about 128 threads, at least one cell).
constexpr int kTileVariants = 2;
__host__ __device__ constexpr int cells_per_block_v(int D, int N, int V) {
  return V == 0 ? cells_per_block(D, N) : (cells_per_block(D, N) / 2 > 0 ? cells_per_block(D, N) / 2 : 1);
}
template <int D, int N, int V>
struct DGShapeV {
  static constexpr int L = (D == 2) ? N : N * N;  // lines per cell = nodes per facet
  static constexpr int NV = L * N;                // nodes per cell
  static constexpr int NF = 2 * D;                // facets per cell
  static constexpr int CPB = cells_per_block_v(D, N, V);
  static constexpr int NT = CPB * L;
  static constexpr int BLOCK = (NT + 63) / 64 * 64;  // launch bound: whole waves
  static constexpr int EGS = 2 * N * N + N;       // S, Si, lambda of one direction
};
template <int D, int N>
using DGShape = DGShapeV<D, N, 0>;

// Per-level reference data (type T), in global memory:
//   [0, N^2)            Mhat (1D mass on [0,1], symmetric)
//   [N^2, N^2+N)        ep0: outward normal derivative functional at x=0
//   [N^2+N, N^2+2N)     ep1: same at x=1
//   [N^2+2N, N^2+3N)    ev0: value functional at x=0 (used with gl)
//   [N^2+3N, N^2+4N)    ev1: value functional at x=1
//   [N^2+4N, ...)       E: interpolation to the fine nodes from the next
//                       coarser nodes, E[a*NC + j] (only when NC > 0)
template <int N>
struct RefOff {
  static constexpr int M = 0, EP0 = N * N, EP1 = N * N + N, EV0 = N * N + 2 * N, EV1 = N * N + 3 * N,
                       E = N * N + 4 * N;
};

// Storage type T of the cell vectors and traces, compute type CT<T> of the
// arithmetic, LDS, operator tables and coarse-level vectors: half-precision
// storage (FP16 or BF16) computes in FP32.
template <typename T>
struct Compute {
  using type = T;
};
template <>
struct Compute<_Float16> {
  using type = float;
};
template <>
struct Compute<__bf16> {
  using type = float;
};
template <typename T>
using CT = typename Compute<T>::type;

template <typename T>
struct DGArgs {
  using C = CT<T>;
  int n, ncell;
  int vark;            // 0: class tables (constant kappa), 1: per-cell eigendata + kappa
  int gl;              // 0: Gauss-Lobatto nodes (facet values are the end nodes), 1: Gauss-Legendre
  C kappa_const;
  const C* ref;        // RefOff layout
  const C* eig;        // vark=0: [4 classes][S N^2 | Si N^2 | lam N]; vark=1: [cell][D][S N^2 | lam N]
  const C* kappa;      // vark=1: per cell
  const C* rk;         // vark=1 with the block recomputed in each traversal: [Khat | C^-1] (Mhat = C C^T),
                       // eig unused; nullptr: eig holds the precomputed per-cell data
  const unsigned char* bmask;  // per cell: bit 2k+side set if that facet is on the boundary
  C h_fwd;             // h^(2-d): scales b in the sweep
  C h_apply;           // h^(d-2): scales A u
  C sigma_hat;         // sigma * h = sigma0 (p_penalty+1)^2
  C omega;
  const T* u_in;       // cell vector
  T* u_out;            // cell vector (may alias u_in)
  const T* b;          // cell vector
  const T* tr_in;      // traces [2D][ncell][2][L] (adaptive meshes: then the hanging-facet slots)
  T* tr_out;
  C* out;              // apply: y; resid: r (NC=0) or coarse right-hand side (next level, compute type)
  const C* coarse;     // prolong: coarse cell vector (DG) or Q1 interior vertex vector (CG)
  int coarse_cg;       // prolong partner: 0 DG, 1 Q1 (vertex gather), 2 Q1 corner values per cell [c][2^d]
  long long vstride;   // per right-hand side stride of cell vectors
  long long tstride;   // per right-hand side stride of trace buffers
  long long cstride;   // per right-hand side stride of coarse vectors
  // Fusions of the outer FP64 Krylov iteration into the finest-level
  // kernels (one right-hand side, NC = 0, T = double):
  //   kry = 1 (projection): first p = z + beta p in place (u_in = u_out = p),
  //     z of type zkind (hpmg_dtype code) at zlow, read as
  //     z * (zscaled ? kscal[8] / kmul : 1), beta = kscal[3]
  //   kdot = 1 (apply, y = A p): kpartial[block] = the block's share of p.y
  int kry = 0, kdot = 0, zkind = 0, zscaled = 0;
  // Interior-block smoother (constant kappa; Section 4.1 technique
  // approximate boundary operators): ivar = 1 takes the block of an interior
  // cell (class 0 along every axis) as the block-Jacobi block D~ of every
  // cell.  The operator stays A: a boundary facet contributes the lift of
  // the cell's own traces with the sign reversed, i.e. (D~ - A_{K<-K}) u
  // (the difference of the two 1D operators is the boundary-facet term,
  // kappa/2 (e ep^T + ep e^T) - sigma_hat kappa e e^T), so that the sweep
  // computes u + omega D~^-1 (b - A u) and the apply A u.  Traces are then
  // stored on boundary facets too.
  int ivar = 0;
  int ncd = 0;         // nodes per direction of the coarse DG level (transfers with a run-time degree)
  // 16-bit storage sweeps (3D): 1 runs the six volume contractions of the
  // block solve on the matrix cores (16-bit operands, FP32 accumulation);
  // 0 keeps them on the vector units in FP32
  int mfma = 0;
  // Adaptive (spacetree) meshes with constant kappa (Section 2.1; the
  // kernels' AD instances): amask[c] holds bit f if facet f of cell c lies
  // on the boundary and bit 8 + f if facet f is the coarse side of a
  // hanging facet (r^(d-1) finer neighbours, penalty sig_hang = r
  // sigma_hat); nbslot[f ncell + c] is the trace slot (unit 2L values)
  // that holds the neighbour-side traces of facet f in the neighbour's
  // reference units: the neighbour's own slot (f^1) ncell + c' across a
  // conforming facet, else a slot filled by the hanging-facet remap;
  // hscale[c] = (h_base / h_c)^(d-2) (nullptr: 1); mort = the remap
  // tables of the level (host side only).
  int adapt = 0;
  C sig_hang = 0;
  const unsigned short* amask = nullptr;
  const int* nbslot = nullptr;
  const C* hscale = nullptr;
  const C* mort = nullptr;
  const int* itab = nullptr;   // hanging interfaces (host side: the remap launch)
  int nif = 0, mif = 0, rfac = 0;
  int* flag = nullptr;  // eigendata build: set to 1 if a block eigenvalue is not positive and finite
  const void* zlow = nullptr;
  const double* kscal = nullptr;
  double kmul = 1.0;
  double* kpartial = nullptr;
};

template <typename T, int D, int N> void launch_sweep(const DGArgs<T>& a, int nrhs, bool uzero, hipStream_t s);
template <typename C, int D, int N> void launch_build_eig(const DGArgs<C>& a, hipStream_t s);
template <typename T, int D, int N, int NC> void launch_apply(const DGArgs<T>& a, int nrhs, bool resid, hipStream_t s);
template <typename T, int D, int N, int NC> void launch_prolong(const DGArgs<T>& a, int nrhs, hipStream_t s);

}  // namespace hpmg
