// Persistent batched kernels: every launch walks a work list covering all
// problems of a batch, so one launch serves one multigrid phase of every
// problem regardless of its mesh size and polynomial degree.
#include "batch_dg_body.hpp"

namespace hpmg {
namespace {

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <typename T, int OP>
constexpr int batch_lds() {
  return cmax(cmax(cmax(item_lds<T, 2, OP>(), item_lds<T, 3, OP>()), cmax(item_lds<T, 4, OP>(), item_lds<T, 5, OP>())),
              item_lds<T, 6, OP>());
}

template <typename T, int OP>
__global__ __launch_bounds__(256) void k_dg_batch(const DGArgs<T>* __restrict__ args,
                                                  const WorkItem* __restrict__ items, int nitems) {
  __shared__ __attribute__((aligned(16))) char lds[batch_lds<T, OP>()];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem w = items[it];
    const DGArgs<T> a = args[w.x];
    switch (w.w) {
      case 2: dg_item<T, 2, OP>(a, w.y, w.z, lds); break;
      case 3: dg_item<T, 3, OP>(a, w.y, w.z, lds); break;
      case 4: dg_item<T, 4, OP>(a, w.y, w.z, lds); break;
      case 5: dg_item<T, 5, OP>(a, w.y, w.z, lds); break;
      case 6: dg_item<T, 6, OP>(a, w.y, w.z, lds); break;
      default: break;
    }
    __syncthreads();  // the next item reuses the LDS
  }
}

// ------------------------------------------------------------------ Q1
__device__ __forceinline__ void vc3(int v, int nv, int& x, int& y, int& z) {
  x = v % nv;
  y = (v / nv) % nv;
  z = v / (nv * nv);
}

template <typename T>
__device__ void cg_item(const CGArgs<T>& a, int blk, int rhs) {
  const int v = blk * 256 + (int)threadIdx.x;
  const T* u = a.u ? a.u + (size_t)rhs * a.su : nullptr;
  const T* b = a.b ? a.b + (size_t)rhs * a.sb : nullptr;
  const T* in = a.in ? a.in + (size_t)rhs * a.sin : nullptr;
  T* out = a.out + (size_t)rhs * a.sout;
  if (a.op == CGOP_JACOBI || a.op == CGOP_RESID) {
    const int nv = a.nv;
    if (v >= nv * nv * nv) return;
    T au = 0;
    if (!a.uzero) {
      // point-major stencil; clamped neighbour indices (an absent
      // neighbour has a zero stencil entry), independent loads
      const int total = nv * nv * nv;
      int x, y, z;
      vc3(v, nv, x, y, z);
      int cx[3], cy[3], cz[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        cx[d] = min(max(x + d - 1, 0), nv - 1);
        cy[d] = min(max(y + d - 1, 0), nv - 1) * nv;
        cz[d] = min(max(z + d - 1, 0), nv - 1) * nv * nv;
      }
      T sv[27], uv[27];
#pragma unroll
      for (int s = 0; s < 27; ++s) {
        sv[s] = a.st[(size_t)s * total + v];
        uv[s] = u[cx[s % 3] + cy[(s / 3) % 3] + cz[s / 9]];
      }
#pragma unroll
      for (int s = 0; s < 27; ++s) au += sv[s] * uv[s];
    }
    if (a.op == CGOP_JACOBI)
      out[v] = (a.uzero ? T(0) : u[v]) + a.omega * a.dinv[v] * (b[v] - au);
    else
      out[v] = b[v] - au;
  } else if (a.op == CGOP_RESTRICT) {
    const int nvc = a.nvc, nvf = a.nv;
    if (v >= nvc * nvc * nvc) return;
    int x, y, z;
    vc3(v, nvc, x, y, z);
    // empty parent slots (index < 0) take index 0 with weight 0
    int ix[3], iy[3], iz[3];
    T wx[3], wy[3], wz[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int jx = a.idx[3 * x + k], jy = a.idx[3 * y + k], jz = a.idx[3 * z + k];
      ix[k] = max(jx, 0);
      iy[k] = max(jy, 0);
      iz[k] = max(jz, 0);
      wx[k] = jx < 0 ? T(0) : a.w[3 * x + k];
      wy[k] = jy < 0 ? T(0) : a.w[3 * y + k];
      wz[k] = jz < 0 ? T(0) : a.w[3 * z + k];
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int bb = 0; bb < 3; ++bb)
#pragma unroll
        for (int aa = 0; aa < 3; ++aa) s += wz[c] * wy[bb] * wx[aa] * in[ix[aa] + nvf * (iy[bb] + nvf * iz[c])];
    out[v] = s;
  } else if (a.op == CGOP_PROLONG) {
    const int nvf = a.nv, nvc = a.nvc;
    if (v >= nvf * nvf * nvf) return;
    int x, y, z;
    vc3(v, nvf, x, y, z);
    int ix[2], iy[2], iz[2];
    T wx[2], wy[2], wz[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int jx = a.idx[2 * x + k], jy = a.idx[2 * y + k], jz = a.idx[2 * z + k];
      ix[k] = max(jx, 0);
      iy[k] = max(jy, 0);
      iz[k] = max(jz, 0);
      wx[k] = jx < 0 ? T(0) : a.w[2 * x + k];
      wy[k] = jy < 0 ? T(0) : a.w[2 * y + k];
      wz[k] = jz < 0 ? T(0) : a.w[2 * z + k];
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) s += wz[c] * wy[bb] * wx[aa] * in[ix[aa] + nvc * (iy[bb] + nvc * iz[c])];
    out[v] += s;
  } else if (a.op == CGOP_GATHER) {
    const int n = a.n, nv = n - 1;
    if (v >= nv * nv * nv) return;
    int x, y, z;
    vc3(v, nv, x, y, z);
    T s = 0;
    for (int c = 0; c < 8; ++c) {
      const int ix = c & 1, iy = (c >> 1) & 1, iz = (c >> 2) & 1;
      const int cell = (x + ix) + n * ((y + iy) + n * (z + iz));
      s += in[(size_t)cell * 8 + (1 - ix) + 2 * (1 - iy) + 4 * (1 - iz)];
    }
    out[v] = s;
  } else {  // dense coarsest solve
    if (v >= a.m) return;
    double s = 0.0;
    for (int j = 0; j < a.m; ++j) s += a.Ainv[(size_t)v * a.m + j] * (double)in[j];
    out[v] = (T)s;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cg_batch(const CGArgs<T>* __restrict__ args,
                                                  const WorkItem* __restrict__ items, int nitems) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem w = items[it];
    const CGArgs<T> a = args[w.x];
    cg_item<T>(a, w.y, w.z);
  }
}

// ----------------------------------------------------- segmented vectors
// One block of BV threads per 16,384-element chunk: 16 elements per thread,
// unrolled by 4, so that a single problem of a few million unknowns (a few
// hundred chunks) still keeps enough loads in flight to stream HBM.
constexpr int BV = 1024;

__device__ __forceinline__ double bsum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  __syncthreads();
  return s;
}

// partial[2*chunk + {0,1}] = x.y, x.z over the chunk (z may be NULL)
__global__ __launch_bounds__(BV) void k_bdot(SegTable t, const double* __restrict__ x, const double* __restrict__ y,
                                              const double* __restrict__ z, double* __restrict__ partial) {
  __shared__ double sh[BV / 64];
  for (int ci = blockIdx.x; ci < t.nchunks; ci += gridDim.x) {
    const int2 ch = t.chunks[ci];
    const long long o = t.off[ch.x] + ch.y;
    const int len = min(BATCH_CHUNK, t.len[ch.x] - ch.y);
    double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
      const double xi = x[o + i];
      s0 += xi * y[o + i];
      if (z) s1 += xi * z[o + i];
    }
    const double t0 = bsum(s0, sh);
    const double t1 = bsum(s1, sh);
    if (threadIdx.x == 0) {
      partial[2 * ci] = t0;
      partial[2 * ci + 1] = t1;
    }
  }
}

// Preconditioned residual straight from the FP32 cycle: z = z32 / s[14]
// (s[14]: scale the cycle's right-hand side was cast with).
// partial[2*chunk + {0,1}] = z.r, z.q over the chunk.
__global__ __launch_bounds__(BV) void k_bdot_z(SegTable t, const float* __restrict__ z32,
                                                const double* __restrict__ r, const double* __restrict__ q,
                                                const double* __restrict__ scal, double* __restrict__ partial) {
  __shared__ double sh[BV / 64];
  for (int ci = blockIdx.x; ci < t.nchunks; ci += gridDim.x) {
    const int2 ch = t.chunks[ci];
    const long long o = t.off[ch.x] + ch.y;
    const int len = min(BATCH_CHUNK, t.len[ch.x] - ch.y);
    const double sc = 1.0 / scal[(size_t)ch.x * BATCH_SCAL + 14];
    double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
      const double zi = (double)z32[o + i] * sc;
      s0 += zi * r[o + i];
      s1 += zi * q[o + i];
    }
    const double t0 = bsum(s0, sh);
    const double t1 = bsum(s1, sh);
    if (threadIdx.x == 0) {
      partial[2 * ci] = t0;
      partial[2 * ci + 1] = t1;
    }
  }
}

// Per-segment scalar state (BATCH_SCAL doubles): [0] rtol^2 of the current
// solve (written by op 4, which runs outside the captured iteration, so a
// replayed graph tests against the tolerance of the call that replays it),
// [2] rho, [3] beta,
// [5] alpha, [6] r.r, [7] 1/||r||, [8] ||r||, [9] ||r0||^2, [10] state
// (0 iterating, 1 recurrence converged, 2 done, 3 breakdown, 4 true residual
// stagnated above the tolerance), [11] restart, [12] last true residual^2,
// [13] iterations, [14] scale of the FP32 copy of r that the next cycle
// reads, [15] restarts so far.
__device__ __forceinline__ void set_rr(double* s, double t0) {
  s[6] = t0;
  s[7] = t0 > 0.0 ? 1.0 / sqrt(t0) : 1.0;
  s[8] = sqrt(t0);
}

__global__ __launch_bounds__(64) void k_bfinal(SegTable t, int op, const double* __restrict__ partial,
                                               double* __restrict__ scal, double rtol2) {
  __shared__ double sh[1];
  const int sg = blockIdx.x;
  double v0 = 0.0, v1 = 0.0;
  const int c0 = t.cstart[sg], cn = t.ccount[sg];
  for (int i = threadIdx.x; i < cn; i += blockDim.x) {
    v0 += partial[2 * (c0 + i)];
    v1 += partial[2 * (c0 + i) + 1];
  }
  const double t0 = bsum(v0, sh);
  const double t1 = bsum(v1, sh);
  if (threadIdx.x != 0) return;
  double* s = scal + (size_t)sg * BATCH_SCAL;
  const bool finite = t0 == t0 && t0 < 1e300;
  if (op == 1) {  // beta (flexible: z.(r - r_old) / rho_old, r - r_old = -alpha_old q)
    s[3] = (s[11] != 0.0 || s[10] != 0.0) ? 0.0 : -s[5] * t1 / s[2];
    s[2] = t0;
    s[11] = 0.0;
  } else if (op == 2) {  // alpha
    if (s[10] == 0.0 && !(finite && t0 != 0.0)) s[10] = 3.0;
    s[5] = s[10] != 0.0 ? 0.0 : s[2] / t0;
    if (s[10] == 0.0) s[13] += 1.0;
  } else if (op == 3) {  // recurrence residual; r32 was written with scale s[7]
    s[14] = s[7];
    if (s[10] == 0.0) {
      set_rr(s, t0);
      if (!finite)
        s[10] = 3.0;
      else if (t0 <= s[0] * s[9])
        s[10] = 1.0;
    }
  } else if (op == 4) {  // initial residual (cast to FP32 next, with scale s[7])
    s[0] = rtol2;
    set_rr(s, t0);
    s[14] = s[7];
    s[5] = 0.0;
    s[9] = t0;
    s[10] = !finite ? 3.0 : (t0 == 0.0 ? 2.0 : 0.0);
    s[11] = 1.0;
    s[12] = t0;
    s[13] = 0.0;
    s[15] = 0.0;
  } else {  // op 5: true residual of the segments whose recurrence converged
    if (s[10] == 1.0) {
      s[12] = t0;
      if (!finite) {
        s[10] = 3.0;
      } else if (t0 <= s[0] * s[9]) {
        s[10] = 2.0;
      } else if (s[15] >= BATCH_MAX_RESTARTS) {
        s[10] = 4.0;  // stagnated at the FP64 rounding floor of b - A u
      } else {  // restart from the true residual
        set_rr(s, t0);
        s[10] = 0.0;
        s[11] = 1.0;
        s[15] += 1.0;
      }
    }
    s[14] = s[7];  // every segment's r is cast to FP32 next with scale s[7]
  }
}

// p = z + beta p with z = z32 / s[14]
__global__ __launch_bounds__(BV) void k_bupdate_p(SegTable t, const float* __restrict__ z32, double* __restrict__ p,
                                                   const double* __restrict__ scal) {
  for (int ci = blockIdx.x; ci < t.nchunks; ci += gridDim.x) {
    const int2 ch = t.chunks[ci];
    const long long o = t.off[ch.x] + ch.y;
    const int len = min(BATCH_CHUNK, t.len[ch.x] - ch.y);
    const double* sg = scal + (size_t)ch.x * BATCH_SCAL;
    const double beta = sg[3], sc = 1.0 / sg[14];
#pragma unroll 4
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
      const double zi = (double)z32[o + i] * sc;
      p[o + i] = beta == 0.0 ? zi : zi + beta * p[o + i];
    }
  }
}

// u += alpha p, r -= alpha q, r32 = r s[7] (the next cycle's right-hand
// side), partial[2*chunk] = r.r
__global__ __launch_bounds__(BV) void k_bupdate_ur(SegTable t, double* __restrict__ r, float* __restrict__ r32,
                                                    const double* __restrict__ p, const double* __restrict__ q,
                                                    const double* __restrict__ scal, double* __restrict__ partial) {
  __shared__ double sh[BV / 64];
  for (int ci = blockIdx.x; ci < t.nchunks; ci += gridDim.x) {
    const int2 ch = t.chunks[ci];
    const long long o = t.off[ch.x] + ch.y;
    const int len = min(BATCH_CHUNK, t.len[ch.x] - ch.y);
    const double* sg = scal + (size_t)ch.x * BATCH_SCAL;
    const double alpha = sg[5], sc = sg[7];
    double* u = t.u[ch.x] + ch.y;
    double acc = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
      double rn = r[o + i];
      if (alpha != 0.0) {
        u[i] += alpha * p[o + i];
        rn -= alpha * q[o + i];
        r[o + i] = rn;
      }
      r32[o + i] = (float)(rn * sc);
      acc += rn * rn;
    }
    const double s0 = bsum(acc, sh);
    if (threadIdx.x == 0) {
      partial[2 * ci] = s0;
      partial[2 * ci + 1] = 0.0;
    }
  }
}

// Segments whose true residual missed the tolerance restart from it.
__global__ __launch_bounds__(BV) void k_bselect(SegTable t, const double* __restrict__ q, double* __restrict__ r,
                                                 const double* __restrict__ scal) {
  for (int ci = blockIdx.x; ci < t.nchunks; ci += gridDim.x) {
    const int2 ch = t.chunks[ci];
    const double* s = scal + (size_t)ch.x * BATCH_SCAL;
    if (!(s[10] == 0.0 && s[11] == 1.0)) continue;
    const long long o = t.off[ch.x] + ch.y;
    const int len = min(BATCH_CHUNK, t.len[ch.x] - ch.y);
#pragma unroll 4
    for (int i = threadIdx.x; i < len; i += blockDim.x) r[o + i] = q[o + i];
  }
}

__global__ __launch_bounds__(BV) void k_bcast_down(SegTable t, const double* __restrict__ x, float* __restrict__ y,
                                                    const double* __restrict__ scal) {
  for (int ci = blockIdx.x; ci < t.nchunks; ci += gridDim.x) {
    const int2 ch = t.chunks[ci];
    const long long o = t.off[ch.x] + ch.y;
    const int len = min(BATCH_CHUNK, t.len[ch.x] - ch.y);
    const double sc = scal[(size_t)ch.x * BATCH_SCAL + 7];
#pragma unroll 4
    for (int i = threadIdx.x; i < len; i += blockDim.x) y[o + i] = (float)(x[o + i] * sc);
  }
}

// count[0] = segments still iterating or waiting, count[1] = segments
// waiting for the true residual check, count[2] = segments that broke down,
// count[3] = segments whose true residual stagnated
__global__ __launch_bounds__(256) void k_bcount(SegTable t, const double* __restrict__ scal, int* __restrict__ count) {
  __shared__ int cs[4];
  if (threadIdx.x < 4) cs[threadIdx.x] = 0;
  __syncthreads();
  int a = 0, b = 0, c = 0, d = 0;
  for (int sg = threadIdx.x; sg < t.nseg; sg += blockDim.x) {
    const double st = scal[(size_t)sg * BATCH_SCAL + 10];
    a += st == 0.0 || st == 1.0;
    b += st == 1.0;
    c += st == 3.0;
    d += st == 4.0;
  }
  atomicAdd(&cs[0], a);
  atomicAdd(&cs[1], b);
  atomicAdd(&cs[2], c);
  atomicAdd(&cs[3], d);
  __syncthreads();
  if (threadIdx.x < 4) count[threadIdx.x] = cs[threadIdx.x];
}

inline unsigned grid_for(int n, int cap) { return (unsigned)(n < cap ? (n > 0 ? n : 1) : cap); }

}  // namespace

template <typename T>
void batch_dg(int op, const DGArgs<T>* args, const WorkItem* items, int nitems, int grid, hipStream_t s) {
  const dim3 g(grid_for(nitems, grid)), b(256);
  switch (op) {
    case BOP_SWEEP: hipLaunchKernelGGL((k_dg_batch<T, BOP_SWEEP>), g, b, 0, s, args, items, nitems); break;
    case BOP_SWEEP0: hipLaunchKernelGGL((k_dg_batch<T, BOP_SWEEP0>), g, b, 0, s, args, items, nitems); break;
    case BOP_RESTRICT: hipLaunchKernelGGL((k_dg_batch<T, BOP_RESTRICT>), g, b, 0, s, args, items, nitems); break;
    case BOP_PROLONG: hipLaunchKernelGGL((k_dg_batch<T, BOP_PROLONG>), g, b, 0, s, args, items, nitems); break;
    case BOP_PROJECT: hipLaunchKernelGGL((k_dg_batch<T, BOP_PROJECT>), g, b, 0, s, args, items, nitems); break;
    case BOP_RESID: hipLaunchKernelGGL((k_dg_batch<T, BOP_RESID>), g, b, 0, s, args, items, nitems); break;
    default: hipLaunchKernelGGL((k_dg_batch<T, BOP_APPLY>), g, b, 0, s, args, items, nitems); break;
  }
}

template <typename T>
void batch_cg(const CGArgs<T>* args, const WorkItem* items, int nitems, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_batch<T>), dim3(grid_for(nitems, grid)), dim3(256), 0, s, args, items, nitems);
}

template void batch_dg<float>(int, const DGArgs<float>*, const WorkItem*, int, int, hipStream_t);
template void batch_dg<double>(int, const DGArgs<double>*, const WorkItem*, int, int, hipStream_t);
template void batch_cg<float>(const CGArgs<float>*, const WorkItem*, int, int, hipStream_t);
template void batch_cg<double>(const CGArgs<double>*, const WorkItem*, int, int, hipStream_t);

void bk_dot(const SegTable& t, const double* x, const double* y, const double* z, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_bdot, dim3(grid_for(t.nchunks, 2048)), dim3(BV), 0, s, t, x, y, z, partial);
}
void bk_dot_z(const SegTable& t, const float* z32, const double* r, const double* q, const double* scal,
              double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_bdot_z, dim3(grid_for(t.nchunks, 2048)), dim3(BV), 0, s, t, z32, r, q, scal, partial);
}
void bk_finalize(const SegTable& t, int op, const double* partial, double* scal, double rtol2, hipStream_t s) {
  hipLaunchKernelGGL(k_bfinal, dim3(t.nseg), dim3(64), 0, s, t, op, partial, scal, rtol2);
}
void bk_update_p(const SegTable& t, const float* z32, double* p, const double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_bupdate_p, dim3(grid_for(t.nchunks, 2048)), dim3(BV), 0, s, t, z32, p, scal);
}
void bk_update_ur(const SegTable& t, double* r, float* r32, const double* p, const double* q, const double* scal,
                  double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_bupdate_ur, dim3(grid_for(t.nchunks, 2048)), dim3(BV), 0, s, t, r, r32, p, q, scal, partial);
}
void bk_cast_down(const SegTable& t, const double* x, float* y, const double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_bcast_down, dim3(grid_for(t.nchunks, 2048)), dim3(BV), 0, s, t, x, y, scal);
}
void bk_count(const SegTable& t, const double* scal, int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_bcount, dim3(1), dim3(256), 0, s, t, scal, count);
}
void bk_select(const SegTable& t, const double* q, double* r, const double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_bselect, dim3(grid_for(t.nchunks, 2048)), dim3(BV), 0, s, t, q, r, scal);
}

}  // namespace hpmg
