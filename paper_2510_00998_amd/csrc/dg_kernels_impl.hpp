// Kernel bodies for dg_kernels.hpp (included by the per-instantiation .hip
// files).  See dg_kernels.hpp for the mathematics.
//
// Block structure of the fused sweep (3D, constant kappa):
//   P1  u, b lines -> registers; neighbour traces -> flux fields, first
//       tangential transform fused into the load -> LDS
//   P2  second tangential transform of the flux fields
//   P3..P5 forward transforms along x, y, z (lifts subtracted per axis),
//       diagonal scaling, first inverse transform
//   P6, P7 inverse transforms along y, x; update, store of u and of the
//       x-facet traces straight from registers
//   P8  y- and z-facet traces from the updated cell in LDS
// Seven barriers; the facet traces are written by each cell for its own
// interior facets and read once by the neighbour in the next sweep.
#pragma once
#include <type_traits>

#include "dg_kernels.hpp"

// A translation unit may compile the cell kernels for another tile variant
// (cells per block, see DGShapeV) by defining HPMG_TILE first: they then
// live in namespace dgk_t<HPMG_TILE>, the host launchers below are left
// out, and unqualified DGShape<D, N> names the variant's shape.
#ifndef HPMG_TILE
#define HPMG_TILE 0
#endif
#if HPMG_TILE == 0
#define HPMG_DGK dgk
#else
#define HPMG_DGK_CAT2(a, b) a##b
#define HPMG_DGK_CAT(a, b) HPMG_DGK_CAT2(a, b)
#define HPMG_DGK HPMG_DGK_CAT(dgk_t, HPMG_TILE)
#endif

namespace hpmg {
namespace HPMG_DGK {
template <int D, int N>
using DGShape = ::hpmg::DGShapeV<D, N, HPMG_TILE>;

// Offset of the first node of the line of thread `ln` along axis k, and the
// node stride along that axis (x fastest).  The facet node index of the line
// on the facets normal to k is `ln` itself for every axis.
template <int D, int N>
__device__ __forceinline__ int line_base(int k, int ln) {
  if constexpr (D == 2) {
    return k == 0 ? N * ln : ln;
  } else {
    const int i0 = ln % N, i1 = ln / N;
    if (k == 0) return N * i0 + N * N * i1;
    if (k == 1) return i0 + N * N * i1;
    return i0 + N * i1;
  }
}
template <int N>
__device__ __forceinline__ constexpr int line_stride(int k) {
  return k == 0 ? 1 : (k == 1 ? N : N * N);
}

// Read-only data addressed uniformly across a wave: the constant address
// space lets the compiler fetch it with scalar loads into SGPRs.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
}

// out = G in, G row-major N x N (TR: G^T)
template <int N, bool TR, typename T, typename P>
__device__ __forceinline__ void mv(P G, const T (&in)[N], T (&out)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) s += (TR ? G[j * N + i] : G[i * N + j]) * in[j];
    out[i] = s;
  }
}

// Even-odd forms of the products with the interior-class matrices, whose
// columns (S) or rows (Si = S^T Mhat) are mirror-even for the first
// (N+1)/2 and mirror-odd for the last N/2 indices: entry A(i, c) is G[i N + c]
// (S) or G[c N + i] (SI, i.e. Si accessed transposed), and
// A(N-1-i, c) = +-A(i, c).  Forward: out[c] = sum_i A(i, c) in[i], from the
// mirror sums and differences of in.  Inverse: out[i] = sum_c A(i, c) in[c],
// as even part +- odd part.  About half the multiply-adds of mv.
template <int N, bool SI, typename T, typename P>
__device__ __forceinline__ T eo_at(P G, int i, int c) {
  return SI ? G[c * N + i] : G[i * N + c];
}
template <int N, bool SI, typename T, typename P>
__device__ __forceinline__ void mv_fwd_eo(P G, const T (&in)[N], T (&out)[N]) {
  constexpr int H = N / 2, NE = (N + 1) / 2;
  T e[H], o[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    e[i] = in[i] + in[N - 1 - i];
    o[i] = in[i] - in[N - 1 - i];
  }
#pragma unroll
  for (int c = 0; c < NE; ++c) {
    T s = (N & 1) ? eo_at<N, SI, T>(G, H, c) * in[H] : T(0);
#pragma unroll
    for (int i = 0; i < H; ++i) s += eo_at<N, SI, T>(G, i, c) * e[i];
    out[c] = s;
  }
#pragma unroll
  for (int c = NE; c < N; ++c) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < H; ++i) s += eo_at<N, SI, T>(G, i, c) * o[i];
    out[c] = s;
  }
}
template <int N, bool SI, typename T, typename P>
__device__ __forceinline__ void mv_inv_eo(P G, const T (&in)[N], T (&out)[N]) {
  constexpr int H = N / 2, NE = (N + 1) / 2;
  T ev[NE], od[H > 0 ? H : 1];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    ev[i] = 0;
#pragma unroll
    for (int c = 0; c < NE; ++c) ev[i] += eo_at<N, SI, T>(G, i, c) * in[c];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    od[i] = 0;
#pragma unroll
    for (int c = NE; c < N; ++c) od[i] += eo_at<N, SI, T>(G, i, c) * in[c];
  }
  // out written in ascending order (as mv does), so that the stores of the
  // alternative paths of stage_mv coincide index by index
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = i < H ? ev[i] + od[i] : (i == H && (N & 1) ? ev[H] : ev[N - 1 - i] - od[N - 1 - i]);
}

template <int D>
__device__ __forceinline__ int ipow(int n, int k) {
  return k == 0 ? 1 : (k == 1 ? n : n * n);
}

// 1/d: hardware reciprocal refined by Newton steps (two for double, one for
// float) to full precision.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  return r;
}
__device__ __forceinline__ float recip(float d) {
  float r = __builtin_amdgcn_rcpf(d);
  return __builtin_fmaf(__builtin_fmaf(-d, r, 1.0f), r, r);
}

// Load scheme of the neighbour traces in the constant-kappa sweep: every
// load of a thread issued at once with the first tangential transform fused
// (facet_pass0_const), except for the 3D FP64 degree-1 and degree-4 sweeps,
// which measured faster with each (facet, cell) record first copied into LDS
// as whole 16-byte vectors (the apply kernels always use the fused loads).
template <typename T, int D, int N>
constexpr bool sweep_copies_traces() {
  return D == 3 && sizeof(T) == 8 && (N == 2 || N == 5);
}

// Thread index within the block's NT working threads; threads beyond NT
// (a batched launch uses one block size for every degree) get an index past
// every work range, so they only take part in the barriers.
template <int D, int N>
__device__ __forceinline__ int work_tid() {
  return threadIdx.x < DGShape<D, N>::NT ? (int)threadIdx.x : (1 << 28);
}

// Boundary mask of a cell (bit f = 2k + side set: facet f on the domain
// boundary); the class of the cell along axis k is (mask >> 2k) & 3.
__device__ __forceinline__ int axis_class(int mask, int k) { return (mask >> (2 * k)) & 3; }

// Adaptive meshes (AD): the mask also holds bit 8 + f for a facet f that is
// the coarse side of a hanging facet (its penalty is r times the conforming
// one), and the class of axis k adds those two bits: 16 class tables.
template <bool AD>
__device__ __forceinline__ int axis_cls(int mask, int k) {
  if constexpr (AD)
    return ((mask >> (2 * k)) & 3) | (((mask >> (8 + 2 * k)) & 3) << 2);
  else
    return (mask >> (2 * k)) & 3;
}
template <bool AD>
constexpr int n_classes() {
  return AD ? 16 : 4;
}
template <bool AD, typename T>
__device__ __forceinline__ int cell_mask(const DGArgs<T>& a, int c) {
  if constexpr (AD)
    return a.amask[c];
  else
    return a.bmask[c];
}

// LDS size of the staged eigendata: constant kappa shares the 4 (adaptive:
// 16) class tables, variable kappa stages one set per cell and axis.
template <int D, int N, bool VARK, bool AD = false>
struct EigLDS {
  static constexpr int SIZE =
      VARK ? DGShape<D, N>::CPB * D * DGShape<D, N>::EGS : n_classes<AD>() * DGShape<D, N>::EGS;
};

// LDS after the staged eigendata: kappa_F per (cell, facet) (variable
// kappa; one unused entry otherwise), kappa_K per cell (variable kappa),
// then the boundary masks of the block's cells (read by the facet passes
// that follow a barrier).
template <int D, int N, bool VARK>
constexpr int kappa_lds_entries() {
  return VARK ? DGShape<D, N>::CPB * (DGShape<D, N>::NF + 1) : 1;
}
template <int D, int N, bool VARK, typename C>
__device__ __forceinline__ int* mask_lds(C* sKF) {
  return (int*)(sKF + kappa_lds_entries<D, N, VARK>());
}
template <int D, int N, bool VARK, typename C>
__device__ __forceinline__ const int* mask_lds(const C* sKF) {
  return (const int*)(sKF + kappa_lds_entries<D, N, VARK>());
}

// Stage the eigendata (and, per cell, kappa_F of every facet; 0 on the
// boundary) of the block's cells.
template <typename T, int D, int N, bool VARK, bool AD = false>
__device__ __forceinline__ void load_eig(const DGArgs<T>& a, int c0, int nc, CT<T>* sE, CT<T>* sKF) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int NN = N * N;
  const int tid = work_tid<D, N>();
  if constexpr (!VARK) {
    for (int i = tid; i < n_classes<AD>() * Sh::EGS; i += Sh::NT) sE[i] = a.eig[i];
  } else {
    // every load of the thread is issued before the first LDS store (no
    // load waits on another): eigendata, then kappa of the cell and of its
    // neighbour across each facet (the neighbour index is clamped into the
    // mesh so that it needs no boundary test; boundary facets get 0)
    constexpr int NE = Sh::CPB * D * (NN + N);
    constexpr int IE = (NE + Sh::NT - 1) / Sh::NT;
    constexpr int NK = Sh::CPB * Sh::NF;
    constexpr int IK = (NK + Sh::NT - 1) / Sh::NT;
    const int ne = nc * D * (NN + N), nk = nc * Sh::NF;
    C ev[IE], k0[IK], k1[IK];
    int msk[IK];
    const bool stored = a.rk == nullptr;  // else rebuilt by recompute_eig
#pragma unroll
    for (int m = 0; m < IE; ++m) {
      const int i = tid + m * Sh::NT;
      ev[m] = (stored && i < ne) ? a.eig[(size_t)c0 * D * (NN + N) + i] : C(0);
    }
#pragma unroll
    for (int m = 0; m < IK; ++m) {
      const int i = tid + m * Sh::NT;
      const int cl = i / Sh::NF, f = i % Sh::NF;
      const int c = c0 + min(cl, nc - 1);
      const int st = ipow<D>(a.n, f >> 1);
      const int nb = min(max((f & 1) ? c + st : c - st, 0), a.ncell - 1);
      msk[m] = a.bmask[c];
      k0[m] = a.kappa[c];
      k1[m] = a.kappa[nb];
    }
#pragma unroll
    for (int m = 0; m < IE; ++m) {
      const int i = tid + m * Sh::NT;
      if (stored && i < ne) {
        const int e = i % (NN + N), ck = i / (NN + N);
        sE[ck * Sh::EGS + (e < NN ? e : NN + e)] = ev[m];
      }
    }
#pragma unroll
    for (int m = 0; m < IK; ++m) {
      const int i = tid + m * Sh::NT;
      if (i < nk) {
        const int f = i % Sh::NF;
        sKF[i] = ((msk[m] >> f) & 1) ? C(0) : C(2) * k0[m] * k1[m] / (k0[m] + k1[m]);
        if (f == 0) sKF[Sh::CPB * Sh::NF + i / Sh::NF] = k0[m];  // kappa_K
      }
    }
  }
}

// Round-robin slot moves of the parallel Jacobi sweep: the slots 0 .. M - 2
// form a circle (position c sits in slot M - 2 for c = 0, in slot 2 (c - 1)
// for 1 <= c < M / 2, in slot 2 (M - 2 - c) + 1 otherwise), paired so that
// circle positions c and M - 1 - c share a slot pair and position 0 pairs
// with the fixed slot M - 1; one step moves position c to c + 1.
template <int M>
__host__ __device__ constexpr int jac_circle_slot(int c) {
  return c == 0 ? M - 2 : (c < M / 2 ? 2 * (c - 1) : 2 * (M - 2 - c) + 1);
}
template <int M>
__host__ __device__ constexpr int jac_slot_circle(int s) {
  return s == M - 2 ? 0 : ((s & 1) == 0 ? s / 2 + 1 : M - 2 - (s - 1) / 2);
}
template <int M>
__host__ __device__ constexpr int jac_next(int s) {
  return s == M - 1 ? s : jac_circle_slot<M>((jac_slot_circle<M>(s) + 1) % (M - 1));
}
template <int M>
__host__ __device__ constexpr int jac_prev(int s) {
  return s == M - 1 ? s : jac_circle_slot<M>((jac_slot_circle<M>(s) + M - 2) % (M - 1));
}

// Fast-diagonalisation data of every staged (cell, axis), rebuilt from kappa
// (block_recompute; the paper's variant that forms the block inverse anew in
// each cell and traversal), in the cell's own S | Si | lambda record in LDS:
//   L   = kappa_K Khat + sum_s [c1_s (e_s ep_s^T + ep_s e_s^T) + c2_s e_s e_s^T]
//         (c1, c2) = (-kappa_F/2, sigma_hat kappa_F) interior, (-kappa_K,
//         2 sigma_hat kappa_K) on the boundary (a boundary facet has kappa_F 0)
//   A   = W L W^T with W = C^-1, Mhat = C C^T (symmetric), in the Si slot
//   parallel Jacobi rotations A <- J^T A J, V <- V J (V in the S slot) until A
//   is diagonal to working precision (at most 8 sweeps in FP64, 6 in FP32)
//   lambda = diag(A), S = W^T V, so that L S = Mhat S diag(lambda), S^T Mhat S = I.
// N lanes of one wave share a (cell, axis): lane r owns row r of every
// product; the products that form A and S go through the cell's LDS record,
// and the rotations run in registers with cross-lane shuffles.  The lanes of
// a problem are in one wave, whose LDS accesses complete in program order,
// so a wavefront-scope fence between the phases orders them.
template <typename T, int D, int N>
__device__ __forceinline__ void recompute_eig(const DGArgs<T>& a, int nc, CT<T>* sE, const CT<T>* sKF) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int NN = N * N;
  constexpr int SWEEPS = sizeof(C) == 8 ? 8 : 6;
  // the block has NT threads (not always whole waves): its last wave hosts
  // only the problems whose N lanes all exist
  constexpr int TPW = 64 / N;  // problems per full wave
  constexpr int NWT = (Sh::NT + 63) / 64;
  constexpr int CLAST = (Sh::NT - 64 * (NWT - 1)) / N < TPW ? (Sh::NT - 64 * (NWT - 1)) / N : TPW;
  constexpr int CAP = (NWT - 1) * TPW + CLAST;  // problems per round of the block
  static_assert(CAP > 0, "no wave can host a problem");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane % N, slot = lane / N;
  const int cap_w = wave == NWT - 1 ? CLAST : TPW;
  const C* sKK = sKF + Sh::CPB * Sh::NF;
  const cptr<C> Kh = as_const(a.rk);
  const cptr<C> Wi = as_const(a.rk) + NN;
  const cptr<C> ev0 = as_const(a.ref) + RefOff<N>::EV0;
  const cptr<C> ev1 = as_const(a.ref) + RefOff<N>::EV1;
  const cptr<C> ep0 = as_const(a.ref) + RefOff<N>::EP0;
  const cptr<C> ep1 = as_const(a.ref) + RefOff<N>::EP1;
  const auto wave_sync = []() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); };
  // rounds of CAP problems; every lane of the block runs the same rounds
  for (int R = 0; R * CAP < nc * D; ++R) {
    const int t = R * CAP + wave * TPW + slot;
    const bool act = slot < cap_w && t < nc * D;
    if (__all(!act)) continue;  // nothing for this wave in this round
    const int tt = act ? t : R * CAP;  // idle lanes shadow a valid problem, writing nothing
    const int cl = tt / D, k = tt % D;
    C* V = sE + tt * Sh::EGS;
    C* A = V + NN;
    C* lam = V + 2 * NN;
    const C kK = sKK[cl];
    const C kF0 = sKF[cl * Sh::NF + 2 * k], kF1 = sKF[cl * Sh::NF + 2 * k + 1];
    const bool b0 = kF0 == C(0), b1 = kF1 == C(0);
    const C c10 = b0 ? -kK : C(-0.5) * kF0, c20 = a.sigma_hat * (b0 ? C(2) * kK : kF0);
    const C c11 = b1 ? -kK : C(-0.5) * kF1, c21 = a.sigma_hat * (b1 ? C(2) * kK : kF1);
    // row r of L, of W L (into V), of A = (W L) W^T
    C row[N];
#pragma unroll
    for (int j = 0; j < N; ++j)
      row[j] = kK * Kh[r * N + j] + c10 * (ev0[r] * ep0[j] + ep0[r] * ev0[j]) + c20 * ev0[r] * ev0[j] +
               c11 * (ev1[r] * ep1[j] + ep1[r] * ev1[j]) + c21 * ev1[r] * ev1[j];
    if (act) {
#pragma unroll
      for (int j = 0; j < N; ++j) A[r * N + j] = row[j];
    }
    wave_sync();
#pragma unroll
    for (int j = 0; j < N; ++j) {
      C s = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) s += Wi[r * N + m] * A[m * N + j];  // W lower triangular: zeros above
      row[j] = s;
    }
    wave_sync();
    if (act) {
#pragma unroll
      for (int j = 0; j < N; ++j) V[r * N + j] = row[j];
    }
    wave_sync();
#pragma unroll
    for (int j = 0; j < N; ++j) {
      C s = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) s += V[r * N + m] * Wi[j * N + m];
      row[j] = s;
    }
    wave_sync();
    if (act) {
#pragma unroll
      for (int j = 0; j < N; ++j) A[r * N + j] = row[j];
#pragma unroll
      for (int j = 0; j < N; ++j) V[r * N + j] = j == r ? C(1) : C(0);
    }
    wave_sync();
    // symmetrise: A <- (A + A^T) / 2
#pragma unroll
    for (int j = 0; j < N; ++j) row[j] = C(0.5) * (A[r * N + j] + A[j * N + r]);
    wave_sync();
    if (act) {
#pragma unroll
      for (int j = 0; j < N; ++j) A[r * N + j] = row[j];
    }
    wave_sync();
    // Parallel Jacobi rotations in registers (round-robin ordering): the
    // rows and columns of A sit in M = N + (N & 1) slots; every round
    // rotates the disjoint slot pairs (2k, 2k+1) (for odd N slot N is an
    // empty placeholder, so slot N - 1 waits), then moves the indices one
    // step along a circle of the slots 0 .. M - 2 (slot M - 1 stays), so
    // that in M - 1 rounds every index pair meets once.  Lane r holds the
    // row of slot r of A and of V (V's rows stay in the original order, its
    // columns move with A's).  The order of the eigenpairs that results is
    // immaterial: lambda and the columns of S move together.
    constexpr int M = N + (N & 1);
    C arow[N], vrow[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      arow[j] = A[r * N + j];
      vrow[j] = j == r ? C(1) : C(0);
    }
    const int base = lane - r;  // lane of slot 0 of this problem
    const int pr = r ^ 1;       // partner slot
    const bool paired = pr < N;
    const bool lower = (r & 1) == 0;
    const int src_pair = base + (paired ? pr : r);
    const int src_move = base + jac_prev<M>(r);  // slot whose row moves into slot r
    bool done = !act;
#pragma unroll 1
    for (int sw = 0; sw < SWEEPS; ++sw) {
      // stop once the off-diagonal part is below working precision (every
      // lane of a problem forms the same sums)
      C offr = 0, dgr = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if (j == r)
          dgr = arow[j] * arow[j];
        else
          offr += arow[j] * arow[j];
      }
      C off = 0, dg = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        off += __shfl(offr, base + m, 64);
        dg += __shfl(dgr, base + m, 64);
      }
      done = done || C(0.5) * off <= (sizeof(C) == 8 ? C(1e-30) : C(1e-14)) * dg;
      if (__all(done)) break;  // every problem of the wave has converged
#pragma unroll 1
      for (int t = 0; t < M - 1; ++t) {
        C mydiag = 0, myoff = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          if (j == r) mydiag = arow[j];
          if (j == pr) myoff = arow[j];
        }
        const C pdiag = __shfl(mydiag, src_pair, 64);
        const C poff = __shfl(myoff, src_pair, 64);
        // both lanes of a pair form the angle from the lower slot's entry
        const C app = lower ? mydiag : pdiag, aqq = lower ? pdiag : mydiag, apq = lower ? myoff : poff;
        // an unpaired, converged or already zero pair rotates by the identity
        const bool rot = paired && !done && apq != C(0);
        const C tau = (aqq - app) / (C(2) * (rot ? apq : C(1)));
        const C at = __builtin_fabs(tau);
        // t = sign(tau) / (|tau| + sqrt(1 + tau^2)), without overflow
        const C ia = C(1) / (at > C(1) ? at : C(1));
        const C root = at > C(1) ? at * __builtin_sqrt(C(1) + ia * ia) : __builtin_sqrt(C(1) + at * at);
        const C tn = __builtin_copysign(C(1), tau) / (at + root);
        const C cs = rot ? C(1) / __builtin_sqrt(C(1) + tn * tn) : C(1);
        const C sn = rot ? tn * cs : C(0);
        // columns 2k, 2k+1 of the rows of A and V (the pair's angle is held
        // by the lane of slot 2k)
#pragma unroll
        for (int k = 0; 2 * k + 1 < N; ++k) {
          const C cj = __shfl(cs, base + 2 * k, 64), sj = __shfl(sn, base + 2 * k, 64);
          const C x = arow[2 * k], y = arow[2 * k + 1];
          arow[2 * k] = cj * x - sj * y;
          arow[2 * k + 1] = sj * x + cj * y;
          const C vx = vrow[2 * k], vy = vrow[2 * k + 1];
          vrow[2 * k] = cj * vx - sj * vy;
          vrow[2 * k + 1] = sj * vx + cj * vy;
        }
        // rows: p' = cs p - sn q, q' = sn p + cs q; the pair's entry is zero
        // afterwards
        const C so = lower ? -sn : sn;  // coefficient of the partner's row
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const C pj = __shfl(arow[j], src_pair, 64);
          const C nv = cs * arow[j] + so * pj;
          arow[j] = (rot && j == pr) ? C(0) : nv;
        }
        // move every index one step along the circle: row of slot prev(r)
        // into slot r, column j into column next(j)
        C na[N], nvr[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
          na[jac_next<M>(j)] = __shfl(arow[j], src_move, 64);
          nvr[jac_next<M>(j)] = vrow[j];
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
          arow[j] = na[j];
          vrow[j] = nvr[j];
        }
      }
    }
    wave_sync();
    if (act) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        A[r * N + j] = arow[j];
        V[r * N + j] = vrow[j];
      }
    }
    wave_sync();
    // lambda = diag(A); S = W^T V, row r: S[r][c] = sum_{m >= r} W[m][r] V[m][c]
    const C lr = A[r * N + r];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      C s = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) s += Wi[m * N + r] * V[m * N + c];
      row[c] = s;
    }
    wave_sync();
    if (act) {
      lam[r] = lr;
#pragma unroll
      for (int c = 0; c < N; ++c) V[r * N + c] = row[c];
    }
    wave_sync();
  }
}

// Si = S^T M for every staged (cell, axis) when the data came per cell.
template <typename T, int D, int N>
__device__ __forceinline__ void make_si(const DGArgs<T>& a, int nc, CT<T>* sE) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int NN = N * N;
  const cptr<C> Mh = as_const(a.ref) + RefOff<N>::M;
  for (int i = work_tid<D, N>(); i < nc * D * NN; i += Sh::NT) {
    const int e = i % NN, ck = i / NN;
    const int r = e / N, col = e % N;
    const C* S = sE + ck * Sh::EGS;
    C s = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) s += S[m * N + r] * Mh[m * N + col];
    sE[ck * Sh::EGS + NN + e] = s;
  }
}

// Matrix of (cell, axis k) at offset `off` within its S | Si | lambda record,
// applied to a line (TR: transposed).  Constant kappa: when every active
// lane of the wave needs the same boundary class the record is read from
// the global class table with scalar loads; otherwise from the LDS copy
// (LDS = true, after the block staged it) or per lane from global memory.
template <typename T, int D, int N, bool VARK, bool TR, bool SIM, bool LDS = true, bool AD = false>
__device__ __forceinline__ void stage_mv(const DGArgs<T>& a, const CT<T>* sE, int cl, int mask, int k,
                                         const CT<T> (&in)[N], CT<T> (&out)[N]) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int off = SIM ? N * N : 0;  // S or Si within the S | Si | lambda record
  // matrices that fit in about 72 SGPRs take the scalar path
  constexpr bool SCALAR_OK = N * N * (int)sizeof(C) / 4 <= 72;
  if constexpr (VARK) {
    mv<N, TR>(sE + (cl * D + k) * Sh::EGS + off, in, out);
  } else {
    const int cls = axis_cls<AD>(mask, k);
    bool uni = false;
    int c0 = cls;
    if constexpr (SCALAR_OK) {
      c0 = __builtin_amdgcn_readfirstlane(cls);
      uni = __all(cls == c0);
    }
    // interior class in FP32 arithmetic (bound by vector-ALU issue): even-odd
    // forms; FP64 (bound by memory latency) keeps the plain products
    if (uni && sizeof(C) == 4 && c0 == 0) {
      const cptr<C> G = as_const(a.eig) + off;
      if constexpr (TR != SIM)
        mv_fwd_eo<N, SIM>(G, in, out);
      else
        mv_inv_eo<N, SIM>(G, in, out);
    } else if (uni)
      mv<N, TR>(as_const(a.eig) + c0 * Sh::EGS + off, in, out);
    else if constexpr (LDS)
      mv<N, TR>(sE + cls * Sh::EGS + off, in, out);
    else
      mv<N, TR>(a.eig + cls * Sh::EGS + off, in, out);
  }
}

// Tangential axis of pass `pass` of the facet transform of facets normal to k.
template <int D>
__device__ __forceinline__ int tangential(int k, int pass) {
  if constexpr (D == 2)
    return 1 - k;
  else
    return pass == 0 ? ((k == 0) ? 1 : 0) : ((k == 2) ? 1 : 2);
}

// Facet flux fields.  From the neighbour's traces (g', q') across facet f
//   F1 = T_f (kappa_F (q'/2 - sigma_hat g')),  F2 = T_f (kappa_F g'/2),
// T_f = G_t1 x G_t2 over the tangential axes with G_t = Si_t for t < k
// (axes already transformed when facet k is processed) and Mhat otherwise.
// sNB[cl][f][F1|F2][L].  Pass 0 reads the neighbour traces (FROM_GLOBAL:
// straight from the trace buffer, item after item; else from the plain LDS
// copy) and transforms along t1; pass 1 transforms along t2 (3D).  Work items are
// ordered (facet, cell, line) so that a wave mostly sees one facet
// direction and therefore one matrix.
template <typename T, int D, int N, bool VARK, bool FROM_GLOBAL = false, bool IVAR = false, bool AD = false>
__device__ __forceinline__ void facet_pass(const DGArgs<T>& a, const T* tr, int c0, int nc, int pass, CT<T>* sNB,
                                           const CT<T>* sE, const CT<T>* sKF) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int NN = N * N;
  constexpr int L = Sh::L;
  constexpr int TL = 2 * L;
  constexpr int LINES = (D == 2) ? 1 : N;
  const cptr<C> Mh = as_const(a.ref) + RefOff<N>::M;
  for (int i = work_tid<D, N>(); i < Sh::CPB * Sh::NF * LINES; i += Sh::NT) {
    const int f = i / (Sh::CPB * LINES), rem = i % (Sh::CPB * LINES);
    const int cl = rem / LINES, li = rem % LINES;
    if (cl >= nc) continue;
    const int c = c0 + cl;
    const int k = f >> 1;
    const int t = tangential<D>(k, pass);
    const int st = pass == 0 ? 1 : N;  // node stride along t within the facet
    const int lo = pass == 0 ? N * li : li;
    C* g = sNB + (cl * Sh::NF + f) * TL + lo;
    const int mask = FROM_GLOBAL ? a.bmask[c] : mask_lds<D, N, VARK>(sKF)[cl];
    const int smask = IVAR ? 0 : mask;  // boundary classes of the block solve
    C x1[N], x2[N], o1[N], o2[N];
    if (pass == 0) {
      const bool bdy = (mask >> f) & 1;
      if (bdy && !(FROM_GLOBAL && IVAR)) {  // boundary facet: no neighbour, zero flux fields
#pragma unroll
        for (int j = 0; j < N; ++j) {
          g[j] = C(0);
          g[L + j] = C(0);
        }
        continue;
      }
      C gv[N], qv[N];
      if constexpr (FROM_GLOBAL) {
        const int s = f & 1;
        const int stc = ipow<D>(a.n, k);
        if constexpr (IVAR) {
          // interior-block smoother: a boundary facet reads the cell's own
          // traces, negated
          const T* src = bdy ? tr + ((size_t)f * a.ncell + c) * TL + lo
                             : tr + ((size_t)(f ^ 1) * a.ncell + (s ? c + stc : c - stc)) * TL + lo;
          const C sg = bdy ? C(-1) : C(1);
#pragma unroll
          for (int j = 0; j < N; ++j) {
            gv[j] = sg * (C)src[j];
            qv[j] = sg * (C)src[L + j];
          }
        } else {
          const T* src = tr + ((size_t)(f ^ 1) * a.ncell + (s ? c + stc : c - stc)) * TL + lo;
#pragma unroll
          for (int j = 0; j < N; ++j) {
            gv[j] = src[j];
            qv[j] = src[L + j];
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) {
          gv[j] = g[j];
          qv[j] = g[L + j];
        }
      }
      C kf;
      if constexpr (VARK)
        kf = sKF[cl * Sh::NF + f];
      else
        kf = a.kappa_const;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        x1[j] = kf * (C(0.5) * qv[j] - a.sigma_hat * gv[j]);
        x2[j] = C(0.5) * kf * gv[j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        x1[j] = g[st * j];
        x2[j] = g[L + st * j];
      }
    }
    if (t < k) {
      stage_mv<T, D, N, VARK, false, true, !FROM_GLOBAL, AD>(a, sE, cl, smask, t, x1, o1);
      stage_mv<T, D, N, VARK, false, true, !FROM_GLOBAL, AD>(a, sE, cl, smask, t, x2, o2);
    } else {
      mv<N, false>(Mh, x1, o1);
      mv<N, false>(Mh, x2, o2);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
      g[st * j] = o1[j];
      g[L + st * j] = o2[j];
    }
  }
}

// Pass 0 for constant kappa with every global load of the thread issued
// before the first use of any of them: the class tables, the boundary masks
// of its items' cells and the neighbour traces (neighbour index clamped into
// the mesh, boundary facets zeroed by a select afterwards), so that the
// block waits for memory once.  Stages the class tables in sE.  AD
// (adaptive meshes): the neighbour-side traces of (cell, facet) come from
// slot nbslot[f ncell + c], and the coarse side of a hanging facet takes
// the penalty sig_hang.
template <typename T, int D, int N, bool AD = false>
__device__ __forceinline__ void facet_pass0_const(const DGArgs<T>& a, const T* tr, int c0, int nc, CT<T>* sNB,
                                                  CT<T>* sE, int* sMask) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int NN = N * N;
  constexpr int L = Sh::L;
  constexpr int TL = 2 * L;
  constexpr int LINES = (D == 2) ? 1 : N;
  constexpr int ITEMS = Sh::CPB * Sh::NF * LINES;
  constexpr int IT = (ITEMS + Sh::NT - 1) / Sh::NT;
  constexpr int NE = n_classes<AD>() * Sh::EGS;
  constexpr int IE = (NE + Sh::NT - 1) / Sh::NT;
  const int tid = work_tid<D, N>();
  const cptr<C> Mh = as_const(a.ref) + RefOff<N>::M;
  C ev[IE];
#pragma unroll
  for (int m = 0; m < IE; ++m) {
    const int i = tid + m * Sh::NT;
    ev[m] = i < NE ? a.eig[i] : C(0);
  }
  // no branches around the loads: an item past the block's work reads the
  // first word of the trace buffer (one cache line for all such lanes)
  C gv[IT][N], qv[IT][N];
  int msk[IT];
#pragma unroll
  for (int m = 0; m < IT; ++m) {
    const int i = tid + m * Sh::NT;
    const int f = min(i / (Sh::CPB * LINES), Sh::NF - 1), rem = i % (Sh::CPB * LINES);
    const int cl = rem / LINES, li = rem % LINES;
    const bool valid = i < ITEMS && cl < nc;
    const int c = c0 + (valid ? cl : 0);
    size_t slot;
    if constexpr (AD) {
      slot = (size_t)a.nbslot[(size_t)f * a.ncell + c];
    } else {
      const int stc = ipow<D>(a.n, f >> 1);
      const int nb = min(max((f & 1) ? c + stc : c - stc, 0), a.ncell - 1);
      slot = (size_t)(f ^ 1) * a.ncell + nb;
    }
    const T* src = valid ? tr + slot * TL + N * li : tr;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      gv[m][j] = src[j];
      qv[m][j] = src[L + j];
    }
    msk[m] = cell_mask<AD>(a, c);
  }
  const int cmask = cell_mask<AD>(a, c0 + min(tid, nc - 1));
  // keep every use of the loaded values below this point, so that the
  // compiler does not wait for one item's data before issuing the next loads
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int m = 0; m < IE; ++m) {
    const int i = tid + m * Sh::NT;
    if (i < NE) sE[i] = ev[m];
  }
  if (tid < nc) sMask[tid] = cmask;
#pragma unroll
  for (int m = 0; m < IT; ++m) {
    const int i = tid + m * Sh::NT;
    const int f = i / (Sh::CPB * LINES), rem = i % (Sh::CPB * LINES);
    const int cl = rem / LINES, li = rem % LINES;
    if (!(i < ITEMS && cl < nc)) continue;
    const int k = f >> 1;
    const int t = tangential<D>(k, 0);
    const bool bdy = (msk[m] >> f) & 1;
    const C kf = a.kappa_const;
    C sh = a.sigma_hat;
    if constexpr (AD) sh = ((msk[m] >> (8 + f)) & 1) ? a.sig_hang : a.sigma_hat;
    C x1[N], x2[N], o1[N], o2[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const C g = bdy ? C(0) : gv[m][j];
      const C q = bdy ? C(0) : qv[m][j];
      x1[j] = kf * (C(0.5) * q - sh * g);
      x2[j] = C(0.5) * kf * g;
    }
    if (t < k) {
      stage_mv<T, D, N, false, false, true, false, AD>(a, sE, cl, msk[m], t, x1, o1);
      stage_mv<T, D, N, false, false, true, false, AD>(a, sE, cl, msk[m], t, x2, o2);
    } else {
      mv<N, false>(Mh, x1, o1);
      mv<N, false>(Mh, x2, o2);
    }
    C* g = sNB + (cl * Sh::NF + f) * TL + N * li;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      g[j] = o1[j];
      g[L + j] = o2[j];
    }
  }
}

// Plain copy of the neighbour traces into sNB (variable kappa path, whose
// facet transform needs the staged per-cell eigendata).  The 2L trace
// entries of a (facet, cell) record are contiguous in the trace buffer and
// in sNB, so the copy moves whole vectors of VB bytes (16 where the record
// size allows; trace buffers are 256-byte aligned and each right-hand side
// column starts at a multiple of the record size).  Item i of the block is
// (facet f, cell cl, vector v), i = (f CPB + cl) NVEC + v; all loads of a
// thread are issued before its LDS stores, from neighbour indices clamped
// into the mesh (boundary facets take zeros).
template <typename T, int D, int N>
__device__ __forceinline__ void copy_neighbour_traces(const DGArgs<T>& a, const T* tr, int c0, int nc, CT<T>* sNB) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int TL = 2 * Sh::L;
  constexpr int RB = TL * (int)sizeof(T);
  constexpr int VB = RB % 16 == 0 ? 16 : (RB % 8 == 0 ? 8 : (RB % 4 == 0 ? 4 : (int)sizeof(T)));
  constexpr int VE = VB / (int)sizeof(T);
  constexpr int NVEC = TL / VE;
  constexpr int NE = Sh::NF * Sh::CPB * NVEC;
  constexpr int IT = (NE + Sh::NT - 1) / Sh::NT;
  struct alignas(VB) Vec {
    T e[VE];
  };
  const int tid = work_tid<D, N>();
  Vec v[IT];
#pragma unroll
  for (int m = 0; m < IT; ++m) {
    const int i = min(tid + m * Sh::NT, NE - 1);
    const int r = i / NVEC, e = (i % NVEC) * VE;
    const int f = r / Sh::CPB, cl = min(r % Sh::CPB, nc - 1);
    const int c = c0 + cl;
    const int st = ipow<D>(a.n, f >> 1);
    const int nb = min(max((f & 1) ? c + st : c - st, 0), a.ncell - 1);
    const bool bdy = (a.bmask[c] >> f) & 1;
    v[m] = *reinterpret_cast<const Vec*>(tr + ((size_t)(f ^ 1) * a.ncell + nb) * TL + e);
    if (bdy) {
#pragma unroll
      for (int j = 0; j < VE; ++j) v[m].e[j] = T(0);
    }
  }
#pragma unroll
  for (int m = 0; m < IT; ++m) {
    const int i = tid + m * Sh::NT;
    const int r = i / NVEC, e = (i % NVEC) * VE;
    const int f = r / Sh::CPB, cl = r % Sh::CPB;
    if (i < NE && cl < nc) {
      C* dst = sNB + (cl * Sh::NF + f) * TL + e;
#pragma unroll
      for (int j = 0; j < VE; ++j) dst[j] = (C)v[m].e[j];
    }
  }
}

// All facet flux fields of the block in sNB, the eigendata in sE and the
// boundary masks of the block's cells in LDS; ends with a barrier.
template <typename T, int D, int N, bool VARK, bool COPY_FIRST = false, bool IVAR = false, bool AD = false>
__device__ __forceinline__ void flux_fields(const DGArgs<T>& a, const T* tr, int c0, int nc, CT<T>* sNB, CT<T>* sE, CT<T>* sKF) {
  static_assert(!AD || (!VARK && !COPY_FIRST && !IVAR), "adaptive meshes: constant kappa, exact blocks, fused loads");
  int* sMask = mask_lds<D, N, VARK>(sKF);
  const int tid = work_tid<D, N>();
  if constexpr (!VARK) {
    if constexpr (IVAR) {  // interior-block smoother: item after item (boundary facets read own traces)
      facet_pass<T, D, N, false, true, true>(a, tr, c0, nc, 0, sNB, sE, sKF);
      load_eig<T, D, N, false>(a, c0, nc, sE, sKF);
      if (tid < nc) sMask[tid] = a.bmask[c0 + tid];
    } else if constexpr (COPY_FIRST) {  // records copied, then the first transform from LDS
      copy_neighbour_traces<T, D, N>(a, tr, c0, nc, sNB);
      load_eig<T, D, N, false>(a, c0, nc, sE, sKF);
      if (tid < nc) sMask[tid] = a.bmask[c0 + tid];
      __syncthreads();
      facet_pass<T, D, N, false>(a, tr, c0, nc, 0, sNB, sE, sKF);
    } else {
      facet_pass0_const<T, D, N, AD>(a, tr, c0, nc, sNB, sE, sMask);
    }
    __syncthreads();
  } else {
    copy_neighbour_traces<T, D, N>(a, tr, c0, nc, sNB);
    load_eig<T, D, N, true>(a, c0, nc, sE, sKF);
    if (tid < nc) sMask[tid] = a.bmask[c0 + tid];
    __syncthreads();
    if (a.rk) {
      recompute_eig<T, D, N>(a, nc, sE, sKF);
      __syncthreads();
    }
    make_si<T, D, N>(a, nc, sE);
    __syncthreads();
    facet_pass<T, D, N, true>(a, tr, c0, nc, 0, sNB, sE, sKF);
    __syncthreads();
  }
  if constexpr (D == 3) {
    facet_pass<T, D, N, VARK, false, IVAR, AD>(a, tr, c0, nc, 1, sNB, sE, sKF);
    __syncthreads();
  }
}

// r -= lift of facets (k,0) and (k,1): value part at the facet node, normal
// derivative part along the line (sweep, SIGN = -1) or r += (apply, +1).
template <typename T, int D, int N, int SIGN>
__device__ __forceinline__ void add_lifts(const DGArgs<T>& a, int cl, int k, int ln, const CT<T>* sNB, CT<T> (&r)[N]) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int L = Sh::L;
  const cptr<C> ep0 = as_const(a.ref) + RefOff<N>::EP0;
  const cptr<C> ep1 = as_const(a.ref) + RefOff<N>::EP1;
  const C* f0 = sNB + (cl * Sh::NF + 2 * k) * 2 * L;
  const C* f1 = f0 + 2 * L;
  const C v0 = f0[ln], d0 = f0[L + ln], v1 = f1[ln], d1 = f1[L + ln];
  constexpr C sg = SIGN < 0 ? C(-1) : C(1);
  if (a.gl) {  // value functionals are dense (Gauss-Legendre nodes)
    const cptr<C> ev0 = as_const(a.ref) + RefOff<N>::EV0;
    const cptr<C> ev1 = as_const(a.ref) + RefOff<N>::EV1;
#pragma unroll
    for (int j = 0; j < N; ++j) r[j] += sg * (ev0[j] * v0 + ev1[j] * v1);
  } else {
    r[0] += sg * v0;
    r[N - 1] += sg * v1;
  }
#pragma unroll
  for (int j = 0; j < N; ++j) r[j] += sg * (ep0[j] * d0 + ep1[j] * d1);
}

// Traces (value, outward normal derivative) of a line along axis k, stored
// straight to the trace buffer for the facets that are not on the boundary.
template <typename T, int D, int N, bool IVAR = false>
__device__ __forceinline__ void store_line_traces(const DGArgs<T>& a, T* trout, int c, int mask, int k, int ln,
                                                  const CT<T> (&u)[N]) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int L = Sh::L;
  constexpr int TL = 2 * L;
  const cptr<C> ep0 = as_const(a.ref) + RefOff<N>::EP0;
  const cptr<C> ep1 = as_const(a.ref) + RefOff<N>::EP1;
  C d0 = 0, d1 = 0, g0 = u[0], g1 = u[N - 1];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    d0 += ep0[j] * u[j];
    d1 += ep1[j] * u[j];
  }
  if (a.gl) {  // value functionals are dense (Gauss-Legendre nodes)
    const cptr<C> ev0 = as_const(a.ref) + RefOff<N>::EV0;
    const cptr<C> ev1 = as_const(a.ref) + RefOff<N>::EV1;
    g0 = 0;
    g1 = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      g0 += ev0[j] * u[j];
      g1 += ev1[j] * u[j];
    }
  }
  if (IVAR || !((mask >> (2 * k)) & 1)) {
    T* t0 = trout + ((size_t)(2 * k) * a.ncell + c) * TL;
    t0[ln] = g0;
    t0[L + ln] = d0;
  }
  if (IVAR || !((mask >> (2 * k + 1)) & 1)) {
    T* t1 = trout + ((size_t)(2 * k + 1) * a.ncell + c) * TL;
    t1[ln] = g1;
    t1[L + ln] = d1;
  }
}

// Traces of the y (and z) lines of the cell vector staged in sU.
template <typename T, int D, int N, bool IVAR = false>
__device__ __forceinline__ void store_yz_traces(const DGArgs<T>& a, T* trout, const CT<T>* sU, int cl, int c, int mask,
                                                int ln) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
#pragma unroll
  for (int k = 1; k < D; ++k) {
    const int base = cl * Sh::NV + line_base<D, N>(k, ln);
    C u[N];
#pragma unroll
    for (int j = 0; j < N; ++j) u[j] = sU[base + j * line_stride<N>(k)];
    store_line_traces<T, D, N, IVAR>(a, trout, c, mask, k, ln, u);
  }
}

// z_j of the Krylov projection (see DGArgs::kry), read by its storage type.
__device__ __forceinline__ double krylov_z(const DGArgs<double>& a, size_t i, double sc) {
  switch (a.zkind) {
    case 1: return (double)((const float*)a.zlow)[i] * sc;
    case 2: return (double)(float)((const _Float16*)a.zlow)[i] * sc;
    case 3: return (double)(float)((const __bf16*)a.zlow)[i] * sc;
    default: return ((const double*)a.zlow)[i] * sc;
  }
}

// Sum of v over the block, written by thread 0 to out (sh: one double per wave).
__device__ __forceinline__ void block_partial(double v, double* sh, double* out) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)((blockDim.x + 63) >> 6); ++i) s += sh[i];
    *out = s;
  }
}

// ---------------------------------------------------------------------------
// Fused block-Jacobi sweep.  UZERO: u is identically zero on entry (first
// sweep of a coarse-level smoothing with zero initial guess): u and the
// neighbour traces are not read.  The x-line of u and b of each thread
// stay in registers from the load to the update.
// LDS bytes of the sweep / apply bodies.
template <typename T, int D, int N, bool VARK, bool AD = false>
constexpr int cell_lds_bytes() {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  return (int)sizeof(C) * (Sh::CPB * Sh::NV + Sh::CPB * Sh::NF * 2 * Sh::L + EigLDS<D, N, VARK, AD>::SIZE +
                           kappa_lds_entries<D, N, VARK>()) +
         (int)sizeof(int) * Sh::CPB;
}

// AD: adaptive mesh (neighbour traces by slot table, 16 class tables, per
// cell h scaling of b in 3D).
template <typename T, int D, int N, bool UZERO, bool VARK, bool IVAR = false, bool AD = false>
__device__ __forceinline__ void sweep_body(const DGArgs<T>& a, int bx, int by, char* lds) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int NN = N * N;
  constexpr int L = Sh::L;
  C* sW = (C*)lds;
  C* sNB = sW + Sh::CPB * Sh::NV;
  C* sE = sNB + Sh::CPB * Sh::NF * 2 * L;
  C* sKF = sE + EigLDS<D, N, VARK, AD>::SIZE;

  const int c0 = bx * Sh::CPB;
  const int nc = min(Sh::CPB, a.ncell - c0);
  const size_t rv = (size_t)by * a.vstride, rt = (size_t)by * a.tstride;
  const int tid = work_tid<D, N>();
  const int cl = tid / L, ln = tid % L;
  const bool act = tid < Sh::NT && cl < nc;
  const int c = c0 + (act ? cl : 0);
  const int base0 = cl * Sh::NV + line_base<D, N>(0, ln);
  const int mask = cell_mask<AD>(a, c);
  const int smask = IVAR ? 0 : mask;  // boundary classes of the block solve
  C hf = a.h_fwd;
  if constexpr (AD) {
    if (a.hscale) hf *= a.hscale[c];
  }

  C ul[N], bl[N];
  if (act) {
    const T* bs = a.b + rv + (size_t)c0 * Sh::NV + base0;
#pragma unroll
    for (int j = 0; j < N; ++j) bl[j] = bs[j];
    if (!UZERO) {
      const T* us = a.u_in + rv + (size_t)c0 * Sh::NV + base0;
#pragma unroll
      for (int j = 0; j < N; ++j) ul[j] = us[j];
    }
  }
  if (!UZERO) {
    flux_fields<T, D, N, VARK, !AD && sweep_copies_traces<T, D, N>(), IVAR, AD>(a, a.tr_in + rt, c0, nc, sNB, sE, sKF);
  } else {
    load_eig<T, D, N, VARK, AD>(a, c0, nc, sE, sKF);
    __syncthreads();
    if constexpr (VARK) {
      if (a.rk) {
        recompute_eig<T, D, N>(a, nc, sE, sKF);
        __syncthreads();
      }
      make_si<T, D, N>(a, nc, sE);
      __syncthreads();
    }
  }

  // forward transforms S^T along x, y(, z) with the facet lifts subtracted
  // just before each axis is transformed
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (act) {
      const int base = cl * Sh::NV + line_base<D, N>(k, ln);
      C r[N], t[N];
      if (k == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) r[j] = hf * bl[j];
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) r[j] = sW[base + j * line_stride<N>(k)];
      }
      if (!UZERO) add_lifts<T, D, N, -1>(a, cl, k, ln, sNB, r);
      stage_mv<T, D, N, VARK, true, false, true, AD>(a, sE, cl, smask, k, r, t);  // S^T
      if (k == D - 1) {
        // diagonal scaling and the first inverse transform along the last axis
        const C* E0 = VARK ? sE + (cl * D + 0) * Sh::EGS : sE + axis_cls<AD>(smask, 0) * Sh::EGS;
        const C* E1 = VARK ? sE + (cl * D + 1) * Sh::EGS : sE + axis_cls<AD>(smask, 1) * Sh::EGS;
        if constexpr (D == 2) {
          const C ls = E0[2 * NN + ln];
#pragma unroll
          for (int j = 0; j < N; ++j) t[j] *= recip(ls + E1[2 * NN + j]);
        } else {
          const C* E2 = VARK ? sE + (cl * D + 2) * Sh::EGS : sE + axis_cls<AD>(smask, 2) * Sh::EGS;
          const C ls = E0[2 * NN + ln % N] + E1[2 * NN + ln / N];
#pragma unroll
          for (int j = 0; j < N; ++j) t[j] *= recip(ls + E2[2 * NN + j]);
        }
        stage_mv<T, D, N, VARK, false, false, true, AD>(a, sE, cl, smask, k, t, r);  // S
#pragma unroll
        for (int j = 0; j < N; ++j) t[j] = r[j];
      }
#pragma unroll
      for (int j = 0; j < N; ++j) sW[base + j * line_stride<N>(k)] = t[j];
    }
    __syncthreads();
  }
  // inverse transforms S along the remaining axes; the last one is fused
  // with the update, the store of u and of the x-facet traces
  T* trout = a.tr_out + rt;
#pragma unroll
  for (int k = D - 2; k >= 0; --k) {
    if (act) {
      const int base = cl * Sh::NV + line_base<D, N>(k, ln);
      C r[N], t[N];
#pragma unroll
      for (int j = 0; j < N; ++j) r[j] = sW[base + j * line_stride<N>(k)];
      stage_mv<T, D, N, VARK, false, false, true, AD>(a, sE, cl, smask, k, r, t);
      if (k == 0) {
        T* uo = a.u_out + rv + (size_t)c0 * Sh::NV + base0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const C uo0 = UZERO ? C(0) : ul[j];
          t[j] = (C(1) - a.omega) * uo0 + a.omega * t[j];
          sW[base + j] = t[j];
          uo[j] = t[j];
        }
        store_line_traces<T, D, N, IVAR>(a, trout, c, mask, 0, ln, t);
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) sW[base + j * line_stride<N>(k)] = t[j];
      }
    }
    __syncthreads();
  }
  if (act) store_yz_traces<T, D, N, IVAR>(a, trout, sW, cl, c, mask, ln);
}

// ---------------------------------------------------------------------------
// Per-cell fast-diagonalisation data of a variable-coefficient level, built
// on the device at setup with the eigensolve of recompute_eig (FP64): for
// every cell and axis the record S (N^2) | lambda (N) of L_k S = Mhat S
// diag(lambda), S^T Mhat S = I, in the layout the stored-eigendata kernels
// read ([cell][axis][S | lambda]).  a.rk holds [Khat | C^-1], a.kappa the
// per-cell kappa; a.out receives the records, a.flag is set to 1 if an
// eigenvalue is not positive and finite (the cell block is not positive
// definite).
template <typename C, int D, int N>
constexpr int build_eig_lds_bytes() {
  return (int)sizeof(C) * (EigLDS<D, N, true>::SIZE + kappa_lds_entries<D, N, true>()) +
         (int)sizeof(int) * DGShape<D, N>::CPB;
}
template <typename C, int D, int N>
__global__ __launch_bounds__((DGShape<D, N>::BLOCK)) void k_build_eig(DGArgs<C> a) {
  using Sh = DGShape<D, N>;
  constexpr int NN = N * N;
  __shared__ __attribute__((aligned(16))) char lds[build_eig_lds_bytes<C, D, N>()];
  C* sE = (C*)lds;
  C* sKF = sE + EigLDS<D, N, true>::SIZE;
  const int c0 = blockIdx.x * Sh::CPB;
  const int nc = min(Sh::CPB, a.ncell - c0);
  load_eig<C, D, N, true>(a, c0, nc, sE, sKF);
  __syncthreads();
  recompute_eig<C, D, N>(a, nc, sE, sKF);
  __syncthreads();
  C* out = a.out + (size_t)c0 * D * (NN + N);
  bool bad = false;
  for (int i = work_tid<D, N>(); i < nc * D * (NN + N); i += Sh::NT) {
    const int ck = i / (NN + N), e = i % (NN + N);
    const C v = sE[ck * Sh::EGS + (e < NN ? e : NN + e)];
    out[i] = v;
    if (e >= NN && !(v > C(0) && v < C(1e30))) bad = true;
  }
  if (bad && a.flag) atomicOr(a.flag, 1);
}

// ---------------------------------------------------------------------------
// Volume contractions of the 16-bit storage sweep on the matrix cores.
//
// One contraction stage replaces every line along axis k of the block's
// cells (FP32, in sW) by G_cell x line, with G = S^T (TR) or S of the cell's
// axis-k record.  A 16x16x16 product D = A B holds NB = 16/N cells on the
// block diagonal of A = diag(G_c0, .., G_c(NB-1)) (zero padded) and 16 lines
// of each of those cells as the columns of B (row N kb + j of B: node j of
// the line in cell kb), so that D row N rb + i, column c is node i of line c
// of cell rb.  The operands are rounded to the storage format (FP16 or BF16)
// and the products accumulate in FP32.  Operand lane layout (16x16x16):
// lane l holds A[l%16][4(l/16)+j], B[4(l/16)+j][l%16] and D[4(l/16)+j][l%16],
// j = 0..3.  SCALE multiplies the result by 1 / (lambda sum) of the node
// (the diagonal of the fast-diagonalised block inverse, applied after S^T
// along the last axis).  Called by every thread of the block (whole waves);
// the products of a wave cover disjoint lines.
typedef _Float16 mf_half4 __attribute__((ext_vector_type(4)));
typedef short mf_short4 __attribute__((ext_vector_type(4)));
typedef float mf_float4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma16;
template <>
struct Mfma16<_Float16> {
  static __device__ __forceinline__ mf_float4 mul(const float (&a)[4], const float (&b)[4]) {
    mf_half4 x, y;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x[j] = (_Float16)a[j];
      y[j] = (_Float16)b[j];
    }
    const mf_float4 z = {0.f, 0.f, 0.f, 0.f};
    return __builtin_amdgcn_mfma_f32_16x16x16f16(x, y, z, 0, 0, 0);
  }
};
template <>
struct Mfma16<__bf16> {
  static __device__ __forceinline__ mf_float4 mul(const float (&a)[4], const float (&b)[4]) {
    mf_short4 x, y;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x[j] = __builtin_bit_cast(short, (__bf16)a[j]);
      y[j] = __builtin_bit_cast(short, (__bf16)b[j]);
    }
    const mf_float4 z = {0.f, 0.f, 0.f, 0.f};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, y, z, 0, 0, 0);
  }
};

template <typename T, int D, int N, bool VARK, bool IVAR, bool TR, bool SCALE>
__device__ __forceinline__ void mfma_stage(float* sW, const float* sE, const int* sMask, int nc, int k) {
  using Sh = DGShape<D, N>;
  constexpr int NN = N * N;
  constexpr int L = Sh::L;
  constexpr int NB = 16 / N;               // cells per product
  constexpr int CH = (L + 15) / 16;        // 16-line chunks per cell
  constexpr int TASKS = (Sh::CPB + NB - 1) / NB * CH;
  constexpr int NW = Sh::BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, kq = lane >> 4;
  const int stride = line_stride<N>(k);
  // cell record of block-diagonal block b (clamped to a staged cell)
  auto rec = [&](int cl) -> const float* {
    if constexpr (VARK)
      return sE + (cl * D + k) * Sh::EGS;
    else
      return sE + (IVAR ? 0 : axis_class(sMask[cl], k)) * Sh::EGS;
  };
  for (int t = wave; t < TASKS; t += NW) {  // uniform over the wave
    const int g = t / CH, q = t % CH;
    const int line = 16 * q + c;
    const int lc = min(line, L - 1);
    const int lb = line_base<D, N>(k, lc);
    float av[4], bv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = 4 * kq + j;
      const int kb = kk / N, jj = kk % N;
      const int cl = g * NB + kb;
      const bool okb = kb < NB && cl < nc && line < L;
      const int clc = min(cl, nc - 1);
      const float x = sW[clc * Sh::NV + lb + (jj < N ? jj : 0) * stride];
      bv[j] = okb ? x : 0.f;
      const int rb = c / N, ii = c % N;
      const int cla = g * NB + rb;
      const bool oka = rb == kb && rb < NB && cla < nc;
      const float* G = rec(min(cla, nc - 1));
      const float gv = TR ? G[jj * N + ii] : G[ii * N + jj];
      av[j] = oka ? gv : 0.f;
    }
    const mf_float4 d = Mfma16<T>::mul(av, bv);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * kq + j;
      const int rb = i / N, ii = i % N;
      const int cl = g * NB + rb;
      if (rb < NB && cl < nc && line < L) {
        float v = d[j];
        if constexpr (SCALE) {
          // lambda sum of node (line, ii) along the last axis k = D - 1
          const int clc = cl;
          float ls;
          if constexpr (D == 2) {
            const float* E0 = VARK ? sE + (clc * D + 0) * Sh::EGS : sE + (IVAR ? 0 : axis_class(sMask[clc], 0)) * Sh::EGS;
            const float* E1 = VARK ? sE + (clc * D + 1) * Sh::EGS : sE + (IVAR ? 0 : axis_class(sMask[clc], 1)) * Sh::EGS;
            ls = E0[2 * NN + line] + E1[2 * NN + ii];
          } else {
            const float* E0 = VARK ? sE + (clc * D + 0) * Sh::EGS : sE + (IVAR ? 0 : axis_class(sMask[clc], 0)) * Sh::EGS;
            const float* E1 = VARK ? sE + (clc * D + 1) * Sh::EGS : sE + (IVAR ? 0 : axis_class(sMask[clc], 1)) * Sh::EGS;
            const float* E2 = VARK ? sE + (clc * D + 2) * Sh::EGS : sE + (IVAR ? 0 : axis_class(sMask[clc], 2)) * Sh::EGS;
            ls = E0[2 * NN + line % N] + E1[2 * NN + line / N] + E2[2 * NN + ii];
          }
          v *= recip(ls);
        }
        sW[cl * Sh::NV + lb + ii * stride] = v;
      }
    }
  }
}

// Fused sweep of a 16-bit storage type with the volume contractions on the
// matrix cores (mfma_stage); facet flux fields, lifts, update and traces as
// in sweep_body.  Launched with whole waves (DGShape::BLOCK threads).
template <typename T, int D, int N, bool UZERO, bool VARK, bool IVAR>
__device__ __forceinline__ void sweep_body_mfma(const DGArgs<T>& a, int bx, int by, char* lds) {
  using C = CT<T>;
  static_assert(sizeof(C) == 4, "matrix-core sweep: 16-bit storage, FP32 compute");
  using Sh = DGShape<D, N>;
  constexpr int L = Sh::L;
  C* sW = (C*)lds;
  C* sNB = sW + Sh::CPB * Sh::NV;
  C* sE = sNB + Sh::CPB * Sh::NF * 2 * L;
  C* sKF = sE + EigLDS<D, N, VARK>::SIZE;
  int* sMask = mask_lds<D, N, VARK>(sKF);

  const int c0 = bx * Sh::CPB;
  const int nc = min(Sh::CPB, a.ncell - c0);
  const size_t rv = (size_t)by * a.vstride, rt = (size_t)by * a.tstride;
  const int tid = work_tid<D, N>();
  const int cl = tid / L, ln = tid % L;
  const bool act = tid < Sh::NT && cl < nc;
  const int c = c0 + (act ? cl : 0);
  const int base0 = cl * Sh::NV + line_base<D, N>(0, ln);
  const int mask = a.bmask[c];

  C ul[N], bl[N];
  if (act) {
    const T* bs = a.b + rv + (size_t)c0 * Sh::NV + base0;
#pragma unroll
    for (int j = 0; j < N; ++j) bl[j] = bs[j];
    if (!UZERO) {
      const T* us = a.u_in + rv + (size_t)c0 * Sh::NV + base0;
#pragma unroll
      for (int j = 0; j < N; ++j) ul[j] = us[j];
    }
  }
  if (!UZERO) {
    flux_fields<T, D, N, VARK, sweep_copies_traces<T, D, N>(), IVAR>(a, a.tr_in + rt, c0, nc, sNB, sE, sKF);
  } else {
    load_eig<T, D, N, VARK>(a, c0, nc, sE, sKF);
    if (tid < nc) sMask[tid] = a.bmask[c0 + tid];
    __syncthreads();
    if constexpr (VARK) {
      if (a.rk) {
        recompute_eig<T, D, N>(a, nc, sE, sKF);
        __syncthreads();
      }
      make_si<T, D, N>(a, nc, sE);
      __syncthreads();
    }
  }
  // forward: right-hand side minus the facet lifts along each axis (vector
  // units, one thread per line), then S^T along that axis on the matrix
  // cores; the last forward stage applies the diagonal scaling
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (act && (k == 0 || !UZERO)) {
      const int base = cl * Sh::NV + line_base<D, N>(k, ln);
      C r[N];
      if (k == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) r[j] = a.h_fwd * bl[j];
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) r[j] = sW[base + j * line_stride<N>(k)];
      }
      if (!UZERO) add_lifts<T, D, N, -1>(a, cl, k, ln, sNB, r);
#pragma unroll
      for (int j = 0; j < N; ++j) sW[base + j * line_stride<N>(k)] = r[j];
    }
    __syncthreads();
    if (k == D - 1)
      mfma_stage<T, D, N, VARK, IVAR, true, true>(sW, sE, sMask, nc, k);
    else
      mfma_stage<T, D, N, VARK, IVAR, true, false>(sW, sE, sMask, nc, k);
    __syncthreads();
  }
  // inverse: S along every axis, last axis first
#pragma unroll
  for (int k = D - 1; k >= 0; --k) {
    mfma_stage<T, D, N, VARK, IVAR, false, false>(sW, sE, sMask, nc, k);
    __syncthreads();
  }
  // update, store of u and of the traces
  T* trout = a.tr_out + rt;
  if (act) {
    T* uo = a.u_out + rv + (size_t)c0 * Sh::NV + base0;
    C t[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const C uo0 = UZERO ? C(0) : ul[j];
      t[j] = (C(1) - a.omega) * uo0 + a.omega * sW[base0 + j];
      sW[base0 + j] = t[j];
      uo[j] = t[j];
    }
    store_line_traces<T, D, N, IVAR>(a, trout, c, mask, 0, ln, t);
  }
  __syncthreads();
  if (act) store_yz_traces<T, D, N, IVAR>(a, trout, sW, cl, c, mask, ln);
}

// At least two waves per SIMD for the 3D FP64 degree 7 and 8 sweeps: left to
// itself the compiler keeps a whole 1D matrix (too large for scalar
// registers) in vector registers and reaches 256 VGPRs (one wave per SIMD).
template <typename T, int D, int N>
constexpr int sweep_waves_per_eu() {
  // the FP64 degree-4 sweep fits 128 VGPRs (four waves per SIMD) without
  // spills, which the compiler does not choose by itself
  return (D == 3 && sizeof(CT<T>) == 8 && N >= 8) ? 2 : ((D == 3 && sizeof(CT<T>) == 8 && N == 5) ? 4 : 1);
}
template <typename T, int D, int N, bool UZERO, bool VARK, bool IVAR, bool MF = false, bool AD = false>
__global__ __launch_bounds__((DGShape<D, N>::BLOCK))
__attribute__((amdgpu_waves_per_eu(sweep_waves_per_eu<T, D, N>()))) void k_sweep(DGArgs<T> a) {
  __shared__ __attribute__((aligned(16))) char lds[cell_lds_bytes<T, D, N, VARK, AD>()];
  if constexpr (MF)
    sweep_body_mfma<T, D, N, UZERO, VARK, IVAR>(a, blockIdx.x, blockIdx.y, lds);
  else
    sweep_body<T, D, N, UZERO, VARK, IVAR, AD>(a, blockIdx.x, blockIdx.y, lds);
}

// ---------------------------------------------------------------------------
// y = A u (RESID: r = b - A u), optionally restricted to the next coarser
// level: NC > 0 gives per cell (E^C x E^C x E^C) r with E the interpolation
// from the coarse nodes (DG_q: a coarse cell vector; Q1: the 2^d corner
// contributions of each cell, summed over cells by the gather kernel).
// Needs the traces of u in tr_in.
template <typename T, int D, int N, int NC, bool RESID, bool VARK, bool IVAR = false, bool AD = false>
__device__ __forceinline__ void apply_body(const DGArgs<T>& a, int bx, int by, char* lds) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int NN = N * N;
  constexpr int L = Sh::L;
  C* sW = (C*)lds;
  C* sNB = sW + Sh::CPB * Sh::NV;
  C* sE = sNB + Sh::CPB * Sh::NF * 2 * L;
  C* sKF = sE + EigLDS<D, N, VARK, AD>::SIZE;

  const int c0 = bx * Sh::CPB;
  const int nc = min(Sh::CPB, a.ncell - c0);
  const size_t rv = (size_t)by * a.vstride, rt = (size_t)by * a.tstride;
  const int tid = work_tid<D, N>();
  const int cl = tid / L, ln = tid % L;
  const bool act = tid < Sh::NT && cl < nc;
  const int c = c0 + (act ? cl : 0);
  const int base0 = cl * Sh::NV + line_base<D, N>(0, ln);
  const int mask = cell_mask<AD>(a, c);
  const int smask = IVAR ? 0 : mask;  // boundary classes of the block solve
  C ha = a.h_apply;
  if constexpr (AD) {
    if (a.hscale) ha /= a.hscale[c];
  }

  C ul[N], bl[N];
  if (act) {
    const T* us = a.u_in + rv + (size_t)c0 * Sh::NV + base0;
#pragma unroll
    for (int j = 0; j < N; ++j) ul[j] = us[j];
    if (RESID) {
      const T* bs = a.b + rv + (size_t)c0 * Sh::NV + base0;
#pragma unroll
      for (int j = 0; j < N; ++j) bl[j] = bs[j];
    }
  }
  flux_fields<T, D, N, VARK, false, IVAR, AD>(a, a.tr_in + rt, c0, nc, sNB, sE, sKF);
  double pdot = 0.0;  // share of p.(A p) (kdot)

  // Si along every axis, diagonal scaling, then Si^T (= M S) back with the
  // lifts added right after each axis is transformed back.
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (act) {
      const int base = cl * Sh::NV + line_base<D, N>(k, ln);
      C r[N], t[N];
      if (k == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) r[j] = ul[j];
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) r[j] = sW[base + j * line_stride<N>(k)];
      }
      stage_mv<T, D, N, VARK, false, true, true, AD>(a, sE, cl, smask, k, r, t);  // Si
      if (k == D - 1) {
        const C* E0 = VARK ? sE + (cl * D + 0) * Sh::EGS : sE + axis_cls<AD>(smask, 0) * Sh::EGS;
        const C* E1 = VARK ? sE + (cl * D + 1) * Sh::EGS : sE + axis_cls<AD>(smask, 1) * Sh::EGS;
        if constexpr (D == 2) {
          const C ls = E0[2 * NN + ln];
#pragma unroll
          for (int j = 0; j < N; ++j) t[j] *= (ls + E1[2 * NN + j]);
        } else {
          const C* E2 = VARK ? sE + (cl * D + 2) * Sh::EGS : sE + axis_cls<AD>(smask, 2) * Sh::EGS;
          const C ls = E0[2 * NN + ln % N] + E1[2 * NN + ln / N];
#pragma unroll
          for (int j = 0; j < N; ++j) t[j] *= (ls + E2[2 * NN + j]);
        }
        stage_mv<T, D, N, VARK, true, true, true, AD>(a, sE, cl, smask, k, t, r);  // Si^T
        add_lifts<T, D, N, +1>(a, cl, k, ln, sNB, r);
#pragma unroll
        for (int j = 0; j < N; ++j) t[j] = r[j];
      }
#pragma unroll
      for (int j = 0; j < N; ++j) sW[base + j * line_stride<N>(k)] = t[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = D - 2; k >= 0; --k) {
    if (act) {
      const int base = cl * Sh::NV + line_base<D, N>(k, ln);
      C r[N], t[N];
#pragma unroll
      for (int j = 0; j < N; ++j) r[j] = sW[base + j * line_stride<N>(k)];
      stage_mv<T, D, N, VARK, true, true, true, AD>(a, sE, cl, smask, k, r, t);
      add_lifts<T, D, N, +1>(a, cl, k, ln, sNB, t);
      if (k == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
          t[j] *= ha;
          if (RESID) t[j] = bl[j] - t[j];
        }
        if constexpr (NC == 0) {
          C* dst = a.out + rv + (size_t)c0 * Sh::NV + base0;
#pragma unroll
          for (int j = 0; j < N; ++j) dst[j] = t[j];
          if constexpr (std::is_same<T, double>::value && !RESID) {
#pragma unroll
            for (int j = 0; j < N; ++j) pdot += ul[j] * t[j];
          }
        } else {
#pragma unroll
          for (int j = 0; j < N; ++j) sW[base + j] = t[j];
        }
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) sW[base + j * line_stride<N>(k)] = t[j];
      }
    }
    if (k > 0 || NC != 0) __syncthreads();
  }
  if constexpr (std::is_same<T, double>::value && NC == 0 && !RESID) {
    if (a.kdot) {
      __shared__ double sh[16];
      block_partial(pdot, sh, a.kpartial + bx);
    }
  }
  if constexpr (NC != 0) {
    // restriction (E^T)^(x d) of the cell residual, one axis per pass; sNB
    // is free once every lift has been read (barrier above).  NC < 0: the
    // coarse node count ncr comes at run time (a.ncd <= N), loops run to N.
    constexpr int NCB = NC > 0 ? NC : N;
    const int ncr = NC > 0 ? NC : a.ncd;
    const cptr<C> E = as_const(a.ref) + RefOff<N>::E;
    const int NCD = (D == 2) ? ncr * ncr : ncr * ncr * ncr;
    constexpr int NBS = Sh::NF * 2 * L;  // per-cell stride of sNB
    C* dst = a.out + (size_t)by * a.cstride + (size_t)c0 * NCD;
    // x: sW[cl][..][a] -> sNB[cl][ln][a'] (a' + ncr*ln)
    for (int i = tid; i < nc * L; i += Sh::NT) {
      const int c2 = i / L, l2 = i % L;
      C x[N];
#pragma unroll
      for (int j = 0; j < N; ++j) x[j] = sW[c2 * Sh::NV + j + N * l2];
#pragma unroll
      for (int jc = 0; jc < NCB; ++jc) {
        if (jc < ncr) {
          C s = 0;
#pragma unroll
          for (int j = 0; j < N; ++j) s += E[j * ncr + jc] * x[j];
          sNB[c2 * NBS + jc + ncr * l2] = s;
        }
      }
    }
    __syncthreads();
    if constexpr (D == 2) {
      // y: sNB[cl][b][a'] -> dst[a' + ncr b']
      for (int i = tid; i < nc * ncr; i += Sh::NT) {
        const int c2 = i / ncr, ac = i % ncr;
        C x[N];
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = sNB[c2 * NBS + ac + ncr * j];
#pragma unroll
        for (int bc = 0; bc < NCB; ++bc) {
          if (bc < ncr) {
            C s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += E[j * ncr + bc] * x[j];
            dst[(size_t)c2 * NCD + ac + ncr * bc] = s;
          }
        }
      }
    } else {
      // y: sNB[cl][c][b][a'] (a' + ncr(b + N c)) -> sW[cl][c][b'][a'] (a' + ncr(b' + ncr c))
      for (int i = tid; i < nc * ncr * N; i += Sh::NT) {
        const int c2 = i / (ncr * N), rem = i % (ncr * N);
        const int ac = rem % ncr, cz = rem / ncr;
        C x[N];
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = sNB[c2 * NBS + ac + ncr * (j + N * cz)];
#pragma unroll
        for (int bc = 0; bc < NCB; ++bc) {
          if (bc < ncr) {
            C s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += E[j * ncr + bc] * x[j];
            sW[c2 * Sh::NV + ac + ncr * (bc + ncr * cz)] = s;
          }
        }
      }
      __syncthreads();
      // z: sW[cl][c][b'][a'] -> dst[a' + ncr b' + ncr^2 c']
      for (int i = tid; i < nc * ncr * ncr; i += Sh::NT) {
        const int c2 = i / (ncr * ncr), rem = i % (ncr * ncr);
        C x[N];
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = sW[c2 * Sh::NV + rem + ncr * ncr * j];
#pragma unroll
        for (int ccz = 0; ccz < NCB; ++ccz) {
          if (ccz < ncr) {
            C s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += E[j * ncr + ccz] * x[j];
            dst[(size_t)c2 * NCD + rem + ncr * ncr * ccz] = s;
          }
        }
      }
    }
  }
}

// Apply holds u, b and the neighbour traces in registers at once; for the
// FP64 degree-4 instances at most 128 VGPRs (four waves per SIMD, no spills).
template <typename T, int N>
constexpr int apply_waves_per_eu() {
  return (sizeof(T) == 8 && N <= 5) ? 4 : 1;
}
template <typename T, int D, int N, int NC, bool RESID, bool VARK, bool IVAR, bool AD = false>
__global__ __launch_bounds__((DGShape<D, N>::BLOCK))
__attribute__((amdgpu_waves_per_eu(apply_waves_per_eu<T, N>()))) void k_apply(DGArgs<T> a) {
  __shared__ __attribute__((aligned(16))) char lds[cell_lds_bytes<T, D, N, VARK, AD>()];
  apply_body<T, D, N, NC, RESID, VARK, IVAR, AD>(a, blockIdx.x, blockIdx.y, lds);
}

// ---------------------------------------------------------------------------
// u += P e (NC > 0; DG_q cell vector or Q1 vertex vector) and projection of
// u onto the facet traces (NC = 0: projection only, the warm-up traversal of
// Algorithm BlockJacobi; NC > 0: fused prolongation + projection,
// Section 5.1.1).
template <typename T, int D, int N, int NC>
constexpr int prolong_lds_bytes() {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  return (int)sizeof(C) * (Sh::CPB * Sh::NV + (NC != 0 ? Sh::CPB * Sh::NV + Sh::CPB * Sh::NF * 2 * Sh::L : 0));
}

template <typename T, int D, int N, int NC, bool IVAR = false, bool AD = false>
__device__ __forceinline__ void prolong_body(const DGArgs<T>& a, int bx, int by, char* lds) {
  using C = CT<T>;
  using Sh = DGShape<D, N>;
  constexpr int L = Sh::L;
  C* sU = (C*)lds;
  C* sW = sU + Sh::CPB * Sh::NV;
  C* sNB = sW + Sh::CPB * Sh::NV;

  const int c0 = bx * Sh::CPB;
  const int nc = min(Sh::CPB, a.ncell - c0);
  const size_t rv = (size_t)by * a.vstride, rt = (size_t)by * a.tstride;
  const int tid = work_tid<D, N>();
  const int cl = tid / L, ln = tid % L;
  const bool act = tid < Sh::NT && cl < nc;
  const int c = c0 + (act ? cl : 0);
  const int mask = cell_mask<AD>(a, c);
  // NC < 0: coarse node count ncr at run time (a.ncd <= N); loops run to
  // NCB = N with the entries past ncr skipped
  constexpr int NCB = NC > 0 ? NC : (NC < 0 ? N : 1);
  const int ncr = NC >= 0 ? NC : a.ncd;
  const int NCD = (NC == 0) ? 0 : ((D == 2) ? ncr * ncr : ncr * ncr * ncr);

  C u[N];
  if (act) {
    const size_t off = rv + (size_t)c0 * Sh::NV + cl * Sh::NV + line_base<D, N>(0, ln);
    const T* us = a.u_in + off;
#pragma unroll
    for (int j = 0; j < N; ++j) u[j] = us[j];
    if constexpr (std::is_same<T, double>::value && NC == 0) {
      if (a.kry) {  // p = z + beta p, in place
        const double beta = a.kscal[3];
        const double sc = a.zscaled ? a.kscal[8] / a.kmul : 1.0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const double zj = krylov_z(a, off + j, sc);
          u[j] = beta == 0.0 ? zj : zj + beta * u[j];
        }
        T* uo = a.u_out + off;
#pragma unroll
        for (int j = 0; j < N; ++j) uo[j] = u[j];
      }
    }
  }
  if constexpr (NC != 0) {
    const C* cs = a.coarse + (size_t)by * a.cstride;
    if (a.coarse_cg != 1) {
      // a coarse DG cell vector, or the Q1 corner values of every cell
      for (int i = tid; i < nc * NCD; i += Sh::NT) sW[(i / NCD) * Sh::NV + i % NCD] = cs[(size_t)c0 * NCD + i];
    } else {
      // Q1 corner values of each cell from the interior-vertex vector
      const int nv = a.n - 1;
      for (int i = tid; i < nc * NCD; i += Sh::NT) {
        const int c2 = i / NCD, corner = i % NCD;
        const int cc = c0 + c2;
        int x[3];
        x[0] = cc % a.n;
        const int rr = cc / a.n;
        x[1] = (D == 2) ? rr : rr % a.n;
        x[2] = (D == 2) ? 0 : rr / a.n;
        int vid = 0, mul = 1;
        bool inside = true;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const int v = x[k] + ((corner >> k) & 1);
          inside = inside && v > 0 && v < a.n;
          vid += (v - 1) * mul;
          mul *= nv;
        }
        sW[c2 * Sh::NV + corner] = inside ? cs[vid] : C(0);
      }
    }
    __syncthreads();
    const cptr<C> E = as_const(a.ref) + RefOff<N>::E;
    if constexpr (D == 3) {
      // z: [c'][b'][a'] -> sNB[cl][c][b'][a'] (a' + NC b' + NC^2 c)
      for (int i = tid; i < nc * ncr * ncr; i += Sh::NT) {
        const int c2 = i / (ncr * ncr), rem = i % (ncr * ncr);
        C x[NCB];
#pragma unroll
        for (int j = 0; j < NCB; ++j) x[j] = j >= ncr ? C(0) : sW[c2 * Sh::NV + rem + ncr * ncr * min(j, ncr - 1)];
#pragma unroll
        for (int cz = 0; cz < N; ++cz) {
          C s = 0;
#pragma unroll
          for (int j = 0; j < NCB; ++j) s += E[cz * ncr + min(j, ncr - 1)] * x[j];  // x[j] = 0 past ncr
          sNB[c2 * Sh::NF * 2 * L + rem + ncr * ncr * cz] = s;
        }
      }
      __syncthreads();
      // y: sNB[c][b'][a'] -> sW[cl][c][b][a'] (a' + NC b + NC N c)
      for (int i = tid; i < nc * ncr * N; i += Sh::NT) {
        const int c2 = i / (ncr * N), rem = i % (ncr * N);
        const int ac = rem % ncr, cz = rem / ncr;
        C x[NCB];
#pragma unroll
        for (int j = 0; j < NCB; ++j) x[j] = j >= ncr ? C(0) : sNB[c2 * Sh::NF * 2 * L + ac + ncr * min(j, ncr - 1) + ncr * ncr * cz];
#pragma unroll
        for (int by = 0; by < N; ++by) {
          C s = 0;
#pragma unroll
          for (int j = 0; j < NCB; ++j) s += E[by * ncr + min(j, ncr - 1)] * x[j];  // x[j] = 0 past ncr
          sW[c2 * Sh::NV + ac + ncr * (by + N * cz)] = s;
        }
      }
      __syncthreads();
    } else {
      // y: [b'][a'] -> sNB[cl][b][a'] -> copy back into sW layout (a' + NC b)
      for (int i = tid; i < nc * ncr; i += Sh::NT) {
        const int c2 = i / ncr, ac = i % ncr;
        C x[NCB];
#pragma unroll
        for (int j = 0; j < NCB; ++j) x[j] = j >= ncr ? C(0) : sW[c2 * Sh::NV + ac + ncr * min(j, ncr - 1)];
#pragma unroll
        for (int by = 0; by < N; ++by) {
          C s = 0;
#pragma unroll
          for (int j = 0; j < NCB; ++j) s += E[by * ncr + min(j, ncr - 1)] * x[j];  // x[j] = 0 past ncr
          sNB[c2 * Sh::NF * 2 * L + ac + ncr * by] = s;
        }
      }
      __syncthreads();
      for (int i = tid; i < nc * ncr * N; i += Sh::NT) {
        const int c2 = i / (ncr * N), rem = i % (ncr * N);
        sW[c2 * Sh::NV + rem] = sNB[c2 * Sh::NF * 2 * L + rem];
      }
      __syncthreads();
    }
  }
  // x: line of thread ln (facet index = (b[,c])): add the prolongated
  // correction, store u and the x-facet traces, stage u for the y/z traces
  T* trout = a.tr_out + rt;
  if (act) {
    const int base = cl * Sh::NV + line_base<D, N>(0, ln);
    if constexpr (NC != 0) {
      const cptr<C> E = as_const(a.ref) + RefOff<N>::E;
      C x[NCB];
#pragma unroll
      for (int j = 0; j < NCB; ++j) x[j] = j >= ncr ? C(0) : sW[cl * Sh::NV + min(j, ncr - 1) + ncr * ln];
#pragma unroll
      for (int ax = 0; ax < N; ++ax) {
        C s = 0;
#pragma unroll
        for (int j = 0; j < NCB; ++j) s += E[ax * ncr + min(j, ncr - 1)] * x[j];  // x[j] = 0 past ncr
        u[ax] += s;
      }
      T* uo = a.u_out + rv + (size_t)c0 * Sh::NV + base;
#pragma unroll
      for (int j = 0; j < N; ++j) uo[j] = u[j];
    }
#pragma unroll
    for (int j = 0; j < N; ++j) sU[base + j] = u[j];
    store_line_traces<T, D, N, IVAR>(a, trout, c, mask, 0, ln, u);
  }
  __syncthreads();
  if (act) store_yz_traces<T, D, N, IVAR>(a, trout, sU, cl, c, mask, ln);
}

template <typename T, int D, int N, int NC, bool IVAR, bool AD = false>
__global__ __launch_bounds__((DGShape<D, N>::BLOCK)) void k_prolong(DGArgs<T> a) {
  __shared__ __attribute__((aligned(16))) char lds[prolong_lds_bytes<T, D, N, NC>()];
  prolong_body<T, D, N, NC, IVAR, AD>(a, blockIdx.x, blockIdx.y, lds);
}

}  // namespace HPMG_DGK

#if HPMG_TILE == 0

template <typename C, int D, int N>
void launch_build_eig(const DGArgs<C>& a, hipStream_t s) {
  using Sh = DGShape<D, N>;
  hipLaunchKernelGGL((dgk::k_build_eig<C, D, N>), dim3((a.ncell + Sh::CPB - 1) / Sh::CPB), dim3(Sh::NT), 0, s, a);
}

// Matrix-core sweep (16-bit storage, 3D): whole waves per block.
template <typename T, int D, int N>
bool launch_sweep_mfma(const DGArgs<T>& a, dim3 grid, bool uzero, hipStream_t s) {
  if constexpr (sizeof(T) == 2 && D == 3) {
    using Sh = DGShape<D, N>;
    const dim3 blk(Sh::BLOCK);
    if (a.vark) {
      if (uzero)
        hipLaunchKernelGGL((dgk::k_sweep<T, D, N, true, true, false, true>), grid, blk, 0, s, a);
      else
        hipLaunchKernelGGL((dgk::k_sweep<T, D, N, false, true, false, true>), grid, blk, 0, s, a);
    } else if (a.ivar) {
      if (uzero)
        hipLaunchKernelGGL((dgk::k_sweep<T, D, N, true, false, true, true>), grid, blk, 0, s, a);
      else
        hipLaunchKernelGGL((dgk::k_sweep<T, D, N, false, false, true, true>), grid, blk, 0, s, a);
    } else {
      if (uzero)
        hipLaunchKernelGGL((dgk::k_sweep<T, D, N, true, false, false, true>), grid, blk, 0, s, a);
      else
        hipLaunchKernelGGL((dgk::k_sweep<T, D, N, false, false, false, true>), grid, blk, 0, s, a);
    }
    return true;
  } else {
    return false;
  }
}

template <typename T, int D, int N>
void launch_sweep(const DGArgs<T>& a, int nrhs, bool uzero, hipStream_t s) {
  using Sh = DGShape<D, N>;
  dim3 grid((a.ncell + Sh::CPB - 1) / Sh::CPB, nrhs);
  if (a.mfma && launch_sweep_mfma<T, D, N>(a, grid, uzero, s)) return;
  if (a.adapt) {  // adaptive meshes: FP64 and FP32 storage
    if constexpr (sizeof(T) >= 4) {
      if (uzero)
        hipLaunchKernelGGL((dgk::k_sweep<T, D, N, true, false, false, false, true>), grid, dim3(Sh::NT), 0, s, a);
      else
        hipLaunchKernelGGL((dgk::k_sweep<T, D, N, false, false, false, false, true>), grid, dim3(Sh::NT), 0, s, a);
    }
  } else if (a.vark) {
    if (uzero)
      hipLaunchKernelGGL((dgk::k_sweep<T, D, N, true, true, false>), grid, dim3(Sh::NT), 0, s, a);
    else
      hipLaunchKernelGGL((dgk::k_sweep<T, D, N, false, true, false>), grid, dim3(Sh::NT), 0, s, a);
  } else if (a.ivar) {
    if (uzero)
      hipLaunchKernelGGL((dgk::k_sweep<T, D, N, true, false, true>), grid, dim3(Sh::NT), 0, s, a);
    else
      hipLaunchKernelGGL((dgk::k_sweep<T, D, N, false, false, true>), grid, dim3(Sh::NT), 0, s, a);
  } else {
    if (uzero)
      hipLaunchKernelGGL((dgk::k_sweep<T, D, N, true, false, false>), grid, dim3(Sh::NT), 0, s, a);
    else
      hipLaunchKernelGGL((dgk::k_sweep<T, D, N, false, false, false>), grid, dim3(Sh::NT), 0, s, a);
  }
}

template <typename T, int D, int N, int NC>
void launch_apply(const DGArgs<T>& a, int nrhs, bool resid, hipStream_t s) {
  using Sh = DGShape<D, N>;
  dim3 grid((a.ncell + Sh::CPB - 1) / Sh::CPB, nrhs);
  if (a.adapt) {
    if constexpr (sizeof(T) >= 4) {
      if (resid)
        hipLaunchKernelGGL((dgk::k_apply<T, D, N, NC, true, false, false, true>), grid, dim3(Sh::NT), 0, s, a);
      else
        hipLaunchKernelGGL((dgk::k_apply<T, D, N, NC, false, false, false, true>), grid, dim3(Sh::NT), 0, s, a);
    }
  } else if (a.vark) {
    if (resid)
      hipLaunchKernelGGL((dgk::k_apply<T, D, N, NC, true, true, false>), grid, dim3(Sh::NT), 0, s, a);
    else
      hipLaunchKernelGGL((dgk::k_apply<T, D, N, NC, false, true, false>), grid, dim3(Sh::NT), 0, s, a);
  } else if (a.ivar) {
    if (resid)
      hipLaunchKernelGGL((dgk::k_apply<T, D, N, NC, true, false, true>), grid, dim3(Sh::NT), 0, s, a);
    else
      hipLaunchKernelGGL((dgk::k_apply<T, D, N, NC, false, false, true>), grid, dim3(Sh::NT), 0, s, a);
  } else {
    if (resid)
      hipLaunchKernelGGL((dgk::k_apply<T, D, N, NC, true, false, false>), grid, dim3(Sh::NT), 0, s, a);
    else
      hipLaunchKernelGGL((dgk::k_apply<T, D, N, NC, false, false, false>), grid, dim3(Sh::NT), 0, s, a);
  }
}

template <typename T, int D, int N, int NC>
void launch_prolong(const DGArgs<T>& a, int nrhs, hipStream_t s) {
  using Sh = DGShape<D, N>;
  dim3 grid((a.ncell + Sh::CPB - 1) / Sh::CPB, nrhs);
  if (a.adapt) {
    if constexpr (sizeof(T) >= 4) hipLaunchKernelGGL((dgk::k_prolong<T, D, N, NC, false, true>), grid, dim3(Sh::NT), 0, s, a);
  } else if (a.ivar)
    hipLaunchKernelGGL((dgk::k_prolong<T, D, N, NC, true>), grid, dim3(Sh::NT), 0, s, a);
  else
    hipLaunchKernelGGL((dgk::k_prolong<T, D, N, NC, false>), grid, dim3(Sh::NT), 0, s, a);
}

#endif  // HPMG_TILE == 0
}  // namespace hpmg
