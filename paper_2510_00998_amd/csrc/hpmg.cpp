// libhpmg: level hierarchy, multigrid cycle, outer solver and the C ABI
// declared in include/hpmg.h.
#include "hpmg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "basis.hpp"
#include "kernels.hpp"

#include "internal.hpp"

using namespace hpmg::detail;

namespace {

thread_local std::string g_last_error;

}  // namespace

namespace hpmg {
namespace detail {
void set_last_error(const std::string& m) { g_last_error = m; }
}  // namespace detail
}  // namespace hpmg

namespace {

// ------------------------------------------------------------------ setup
// 1D operator of one axis of the cell block in reference units (Kronecker
// factor L_k of A_{K<-K}): kappa_K Khat plus, for each of the two facets,
// c1 (e ep^T + ep e^T) + c2 e e^T with (c1, c2) = (-kF/2, sigma_hat kF) on
// interior facets and (-kappa_K, 2 sigma_hat kappa_K) on boundary facets.
// pen0 / pen1 multiply the penalty of an interior facet (adaptive meshes:
// r on the coarse side of a hanging facet, whose penalty is that of the
// finer cells).
void axis_operator(const hpmg::Basis1D& B, double kK, double kF0, bool bdy0, double kF1, bool bdy1,
                   double sigma_hat, std::vector<double>& L, double pen0 = 1.0, double pen1 = 1.0) {
  const int N = B.N;
  L.assign((size_t)N * N, 0.0);
  for (int i = 0; i < N * N; ++i) L[i] = kK * B.K[i];
  for (int s = 0; s < 2; ++s) {
    const bool bdy = s ? bdy1 : bdy0;
    const double kF = s ? kF1 : kF0;
    const double c1 = bdy ? -kK : -0.5 * kF;
    const double c2 = bdy ? 2.0 * sigma_hat * kK : sigma_hat * kF * (s ? pen1 : pen0);
    const std::vector<double>& e = s ? B.e1 : B.e0;
    const std::vector<double>& ep = s ? B.ep1 : B.ep0;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j)
        L[(size_t)i * N + j] += c1 * (e[i] * ep[j] + ep[i] * e[j]) + c2 * e[i] * e[j];
  }
}

void eig_of(const hpmg::Basis1D& B, const std::vector<double>& L, double* S, double* lam) {
  if (!hpmg::gen_sym_eig(L.data(), B.M.data(), B.N, S, lam))
    throw HpmgError(HPMG_E_DEVICE, "mass matrix not positive definite");
  for (int i = 0; i < B.N; ++i)
    if (!(lam[i] > 0.0) || !std::isfinite(lam[i]))
      throw HpmgError(HPMG_E_INVALID, "cell block is not positive definite (penalty too small?)");
}

// Eigendata of a 1D operator that commutes with the node mirror i -> N-1-i
// (interior class with constant kappa: the Gauss-Lobatto and Gauss-Legendre
// nodes are symmetric about 1/2, so Mhat, Khat and the two-facet terms are
// centro-symmetric).  Its M-orthonormal eigenvectors split into mirror-even
// and mirror-odd ones; each group is solved in its own subspace, so that
// S = [even columns (N+1)/2 | odd columns N/2] holds the parity exactly:
// S[N-1-i][c] = S[i][c] for even c and -S[i][c] for odd c (bitwise, rows i
// and N-1-i are computed from identical data).  The kernels use this split
// to apply S, S^T, Si and Si^T with about half the multiply-adds.
void eig_even_odd(const hpmg::Basis1D& B, const std::vector<double>& L, double* S, double* lam) {
  const int N = B.N, H = N / 2, NE = (N + 1) / 2;
  const double r2 = std::sqrt(0.5);
  std::fill(S, S + (size_t)N * N, 0.0);
  for (int par = 0; par < 2; ++par) {
    const int m = par == 0 ? NE : H;  // subspace dimension
    if (m == 0) continue;
    // basis Q (N x m) of the even (par 0) or odd (par 1) vectors
    std::vector<double> Q((size_t)N * m, 0.0);
    for (int j = 0; j < H; ++j) {
      Q[(size_t)j * m + j] = r2;
      Q[(size_t)(N - 1 - j) * m + j] = par == 0 ? r2 : -r2;
    }
    if (par == 0 && (N & 1)) Q[(size_t)H * m + H] = 1.0;
    std::vector<double> Lr((size_t)m * m), Mr((size_t)m * m), Sr((size_t)m * m), lr(m);
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) {
        long double sl = 0.0L, sm = 0.0L;
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j) {
            const long double q = (long double)Q[(size_t)i * m + a] * Q[(size_t)j * m + b];
            sl += q * L[(size_t)i * N + j];
            sm += q * B.M[(size_t)i * N + j];
          }
        Lr[(size_t)a * m + b] = (double)sl;
        Mr[(size_t)a * m + b] = (double)sm;
      }
    if (!hpmg::gen_sym_eig(Lr.data(), Mr.data(), m, Sr.data(), lr.data()))
      throw HpmgError(HPMG_E_DEVICE, "mass matrix not positive definite");
    const int c0 = par == 0 ? 0 : NE;
    for (int c = 0; c < m; ++c) {
      lam[c0 + c] = lr[c];
      for (int i = 0; i < N; ++i) {
        long double acc = 0.0L;
        for (int a = 0; a < m; ++a) acc += (long double)Q[(size_t)i * m + a] * Sr[(size_t)a * m + c];
        S[(size_t)i * N + c0 + c] = (double)acc;
      }
    }
  }
  for (int i = 0; i < N; ++i)
    if (!(lam[i] > 0.0) || !std::isfinite(lam[i]))
      throw HpmgError(HPMG_E_INVALID, "cell block is not positive definite (penalty too small?)");
}

// [Khat | W] with W = C^-1 and Mhat = C C^T (Cholesky in long double).
std::vector<double> khat_and_inverse_cholesky(const hpmg::Basis1D& B) {
  const int N = B.N, NN = N * N;
  std::vector<double> tab((size_t)2 * NN, 0.0);
  std::copy(B.K.begin(), B.K.end(), tab.begin());
  std::vector<long double> Cm((size_t)NN, 0.0L), Wm((size_t)NN, 0.0L);
  for (int j = 0; j < N; ++j) {
    long double sd = B.M[(size_t)j * N + j];
    for (int k = 0; k < j; ++k) sd -= Cm[(size_t)j * N + k] * Cm[(size_t)j * N + k];
    if (!(sd > 0.0L)) throw HpmgError(HPMG_E_DEVICE, "mass matrix not positive definite");
    Cm[(size_t)j * N + j] = std::sqrt(sd);
    for (int i = j + 1; i < N; ++i) {
      long double t = B.M[(size_t)i * N + j];
      for (int k = 0; k < j; ++k) t -= Cm[(size_t)i * N + k] * Cm[(size_t)j * N + k];
      Cm[(size_t)i * N + j] = t / Cm[(size_t)j * N + j];
    }
  }
  for (int j = 0; j < N; ++j) {
    Wm[(size_t)j * N + j] = 1.0L / Cm[(size_t)j * N + j];
    for (int i = j + 1; i < N; ++i) {
      long double t = 0.0L;
      for (int k = j; k < i; ++k) t += Cm[(size_t)i * N + k] * Wm[(size_t)k * N + j];
      Wm[(size_t)i * N + j] = -t / Cm[(size_t)i * N + i];
    }
  }
  for (int i = 0; i < NN; ++i) tab[(size_t)NN + i] = (double)Wm[i];
  return tab;
}

// Solve Mhat X = Y for the N x N matrices of the hanging-facet projection
// (Gaussian elimination with partial pivoting in long double).
std::vector<double> mass_solve(const hpmg::Basis1D& B, const std::vector<double>& Y) {
  const int N = B.N;
  std::vector<long double> A(B.M.begin(), B.M.end()), X(Y.begin(), Y.end());
  for (int c = 0; c < N; ++c) {
    int piv = c;
    for (int r = c + 1; r < N; ++r)
      if (std::fabs((double)A[(size_t)r * N + c]) > std::fabs((double)A[(size_t)piv * N + c])) piv = r;
    for (int j = 0; j < N; ++j) {
      std::swap(A[(size_t)c * N + j], A[(size_t)piv * N + j]);
      std::swap(X[(size_t)c * N + j], X[(size_t)piv * N + j]);
    }
    for (int r = 0; r < N; ++r) {
      if (r == c) continue;
      const long double f = A[(size_t)r * N + c] / A[(size_t)c * N + c];
      for (int j = 0; j < N; ++j) {
        A[(size_t)r * N + j] -= f * A[(size_t)c * N + j];
        X[(size_t)r * N + j] -= f * X[(size_t)c * N + j];
      }
    }
  }
  std::vector<double> out((size_t)N * N);
  for (int r = 0; r < N; ++r)
    for (int j = 0; j < N; ++j) out[(size_t)r * N + j] = (double)(X[(size_t)r * N + j] / A[(size_t)r * N + r]);
  return out;
}

// Hanging-facet remap tables of a level (adaptive meshes): I_j[a][b] =
// l_b((xi_a + j) / r) (the coarse facet polynomial at the nodes of the j-th
// fine facet along one axis) for j < r, then P_j = (1/r) Mhat^-1 I_j^T Mhat
// (L2 projection of a polynomial on the j-th part onto the coarse facet).
std::vector<double> remap_tables(const hpmg::Basis1D& B, int r) {
  const int N = B.N, NN = N * N;
  std::vector<double> out((size_t)2 * r * NN);
  for (int j = 0; j < r; ++j) {
    std::vector<double> pts(N);
    for (int a = 0; a < N; ++a) pts[a] = (B.xi[a] + j) / r;
    const std::vector<double> I = hpmg::interp_matrix(pts, B.xi);
    std::copy(I.begin(), I.end(), out.begin() + (size_t)j * NN);
    std::vector<double> Y((size_t)NN, 0.0);  // (1/r) I^T Mhat
    for (int a = 0; a < N; ++a)
      for (int c = 0; c < N; ++c) {
        long double acc = 0.0L;
        for (int m = 0; m < N; ++m) acc += (long double)I[(size_t)m * N + a] * B.M[(size_t)m * N + c];
        Y[(size_t)a * N + c] = (double)(acc / r);
      }
    const std::vector<double> P = mass_solve(B, Y);
    std::copy(P.begin(), P.end(), out.begin() + (size_t)(r + j) * NN);
  }
  return out;
}

void build_dg_level(hpmg_ctx* h, DGLevel& L, const hpmg::Basis1D& B, const hpmg::Basis1D* Bnext,
                    hipStream_t s) {
  const int N = B.N, NN = N * N, D = h->dim;
  const size_t ncell = h->adapt ? (size_t)h->amesh[L.am].ncell : (size_t)h->ncell;
  const size_t nif = h->adapt ? (size_t)h->amesh[L.am].nif : 0;
  L.ndof = ncell * ipow(N, D);
  L.trsize = ((size_t)2 * D * ncell + nif * (h->mif + 1)) * 2 * ipow(N, D - 1);
  // reference data
  std::vector<double> ref;
  ref.insert(ref.end(), B.M.begin(), B.M.end());
  ref.insert(ref.end(), B.ep0.begin(), B.ep0.end());
  ref.insert(ref.end(), B.ep1.begin(), B.ep1.end());
  ref.insert(ref.end(), B.e0.begin(), B.e0.end());
  ref.insert(ref.end(), B.e1.begin(), B.e1.end());
  if (Bnext) {
    std::vector<double> E = hpmg::interp_matrix(B.xi, Bnext->xi);
    ref.insert(ref.end(), E.begin(), E.end());
  } else {
    for (int a = 0; a < N; ++a) {
      ref.push_back(1.0 - B.xi[a]);
      ref.push_back(B.xi[a]);
    }
  }
  L.d.ref = h->mem.upload(ref, s);
  L.f.ref = h->mem.upload(cast_vec<float>(ref), s);
  // eigendata of the cell blocks
  const int EGS = 2 * NN + N;
  std::vector<double> Lm;
  if (!h->vark) {
    // classes: bit 0 / 1 lower / upper facet on the boundary; adaptive
    // meshes add bit 2 / 3 for a lower / upper hanging facet (coarse side)
    const int ncls = h->adapt ? 16 : 4;
    std::vector<double> tab((size_t)ncls * EGS, 0.0);
    const double k = h->kappa_const;
    for (int cls = 0; cls < ncls; ++cls) {
      const bool b0 = cls & 1, b1 = (cls >> 1) & 1, g0 = (cls >> 2) & 1, g1 = (cls >> 3) & 1;
      if ((b0 && b1 && h->n > 1) || (b0 && g0) || (b1 && g1)) {
        // no cell has this class (both facets on the boundary only when
        // n == 1; a boundary facet does not hang)
        std::copy(tab.begin(), tab.begin() + EGS, tab.begin() + (size_t)cls * EGS);
        continue;
      }
      axis_operator(B, k, k, b0, k, b1, L.sigma_hat, Lm, g0 ? h->rfac : 1.0, g1 ? h->rfac : 1.0);
      double* S = &tab[(size_t)cls * EGS];
      double* Si = S + NN;
      double* lam = S + 2 * NN;
      if (cls == 0)
        eig_even_odd(B, Lm, S, lam);
      else
        eig_of(B, Lm, S, lam);
      for (int r = 0; r < N; ++r)
        for (int c = 0; c < N; ++c) {
          double acc = 0.0;
          for (int m = 0; m < N; ++m) acc += S[m * N + r] * B.M[m * N + c];
          Si[r * N + c] = acc;
        }
      if (cls == 0) {
        // Si = S^T Mhat inherits the parity of the columns of S along its
        // rows; make it exact (the two halves were summed in different order)
        for (int r = 0; r < N; ++r) {
          const double sg = r < (N + 1) / 2 ? 1.0 : -1.0;
          for (int c = 0; c < N / 2; ++c) Si[r * N + N - 1 - c] = sg * Si[r * N + c];
          if ((N & 1) && sg < 0) Si[r * N + N / 2] = 0.0;
        }
      }
    }
    L.d.eig = h->mem.upload(tab, s);
    L.f.eig = h->mem.upload(cast_vec<float>(tab), s);
    if (h->adapt) {
      const std::vector<double> mt = remap_tables(B, h->rfac);
      L.d.mort = h->mem.upload(mt, s);
      L.f.mort = h->mem.upload(cast_vec<float>(mt), s);
    }
  } else {
    // the kernels rebuild S, lambda per cell and axis from kappa
    // (block_recompute) or read them from per-cell records built here on the
    // device by the same eigensolve: both need Khat and W = C^-1 with
    // Mhat = C C^T (then W L W^T is symmetric and its eigenvectors V give
    // S = W^T V)
    const std::vector<double> tab = khat_and_inverse_cholesky(B);
    const double* rk = h->mem.upload(tab, s);
    L.d.kappa = h->mem.upload(h->kappa, s);
    L.f.kappa = h->mem.upload(cast_vec<float>(h->kappa), s);
    if (h->opt.block_recompute == 1) {
      L.d.rk = const_cast<double*>(rk);
      L.f.rk = h->mem.upload(cast_vec<float>(tab), s);
    } else {
      const size_t ne = (size_t)h->ncell * D * (NN + N);
      L.d.eig = (double*)h->mem.alloc(ne * sizeof(double));
      L.f.eig = (float*)h->mem.alloc(ne * sizeof(float));
      int* flag = (int*)h->mem.alloc(sizeof(int));
      HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), s));
      hpmg::DGArgs<double> a = dg_args<double>(h, L);
      a.rk = rk;
      a.out = L.d.eig;
      a.flag = flag;
      dg_run(h, hpmg::OP_BUILD_EIG, a, N, 1, 0, s);
      hpmg::cast_down<float>(ne, L.d.eig, L.f.eig, nullptr, 1.0, s);
      int hflag = 0;
      HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (hflag) throw HpmgError(HPMG_E_INVALID, "cell block is not positive definite (penalty too small?)");
      if (h->opt.block_recompute == 2) {
        // second record buffer of each precision (a copy: both valid), and
        // the rebuild tables
        L.d.ebuf[0] = L.d.eig;
        L.f.ebuf[0] = L.f.eig;
        L.d.ebuf[1] = (double*)h->mem.alloc(ne * sizeof(double));
        L.f.ebuf[1] = (float*)h->mem.alloc(ne * sizeof(float));
        HIPCHK(hipMemcpyAsync(L.d.ebuf[1], L.d.eig, ne * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(L.f.ebuf[1], L.f.eig, ne * sizeof(float), hipMemcpyDeviceToDevice, s));
        L.d.rkb = const_cast<double*>(rk);
        L.f.rkb = h->mem.upload(cast_vec<float>(tab), s);
      }
    }
  }
  const size_t R = (size_t)h->opt.max_rhs;
  for (int b = 0; b < 2; ++b) {
    L.d.tr[b] = (double*)h->mem.alloc(L.trsize * R * sizeof(double));
    L.f.tr[b] = (float*)h->mem.alloc(L.trsize * R * sizeof(float));
  }
}

// Q1 element stiffness on a cell of width h: h^(d-2) sum_k K1 (x) M1 ...
void q1_element(int D, double h, std::vector<double>& Ke) {
  const double M1[2][2] = {{1.0 / 3, 1.0 / 6}, {1.0 / 6, 1.0 / 3}};
  const double K1[2][2] = {{1.0, -1.0}, {-1.0, 1.0}};
  const int nc = 1 << D;
  Ke.assign((size_t)nc * nc, 0.0);
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) {
      double s = 0.0;
      for (int k = 0; k < D; ++k) {
        double t = 1.0;
        for (int m = 0; m < D; ++m) {
          const int a = (i >> m) & 1, b = (j >> m) & 1;
          t *= (m == k) ? K1[a][b] : M1[a][b];
        }
        s += t;
      }
      Ke[(size_t)i * nc + j] = s * std::pow(h, D - 2);
    }
}

int nstencil(int D) { return D == 2 ? 9 : 27; }

// Finest Q1 operator: Galerkin product of the DG operator with the Q1
// interpolation, i.e. sum_K kappa_K (grad phi_i, grad phi_j)_K on interior
// vertices, as a 3^d-point stencil per vertex.
std::vector<double> q1_stencil(int D, int n, const std::vector<double>& kap) {
  const int nv = n - 1, NS = nstencil(D), ncor = 1 << D;
  const size_t nvt = (size_t)ipow(nv, D);
  std::vector<double> st(nvt * NS, 0.0), Ke;
  q1_element(D, 1.0 / n, Ke);
  const int ncell = ipow(n, D);
  for (int c = 0; c < ncell; ++c) {
    int cc[3] = {c % n, (c / n) % n, D == 3 ? c / (n * n) : 0};
    for (int i = 0; i < ncor; ++i) {
      int vi[3] = {0, 0, 0};
      bool in = true;
      for (int k = 0; k < D; ++k) {
        vi[k] = cc[k] + ((i >> k) & 1);
        in = in && vi[k] > 0 && vi[k] < n;
      }
      if (!in) continue;
      const size_t row = (vi[0] - 1) + (size_t)nv * ((vi[1] - 1) + (size_t)nv * (D == 3 ? vi[2] - 1 : 0));
      for (int j = 0; j < ncor; ++j) {
        int off = 0, mul = 1;
        bool jin = true;
        for (int k = 0; k < D; ++k) {
          const int vj = cc[k] + ((j >> k) & 1);
          jin = jin && vj > 0 && vj < n;
          off += (vj - vi[k] + 1) * mul;
          mul *= 3;
        }
        if (!jin) continue;
        st[row * NS + off] += kap[c] * Ke[(size_t)i * ncor + j];
      }
    }
  }
  return st;
}

// 1D interpolation from the coarse vertex grid (every other fine vertex, the
// last fine vertex always kept) to the fine vertices 0..n.
// Fine vertices kept as coarse vertices: every f-th, plus the last one when
// f does not divide n.
std::vector<int> coarse_positions(int n, int f) {
  std::vector<int> pos;
  for (int i = 0; i <= n; i += f) pos.push_back(i);
  if (pos.back() != n) pos.push_back(n);
  return pos;
}

struct Transfer1D {
  std::vector<std::vector<std::pair<int, double>>> parents;  // fine vertex -> (coarse vertex, weight)
};

Transfer1D transfer_1d(int n, int f) {
  std::vector<int> pos = coarse_positions(n, f);
  Transfer1D T;
  T.parents.resize(n + 1);
  for (int i = 0; i <= n; ++i) {
    auto it = std::lower_bound(pos.begin(), pos.end(), i);
    const int J = (int)(it - pos.begin());
    if (pos[J] == i) {
      T.parents[i].push_back({J, 1.0});
    } else {
      const double t = double(i - pos[J - 1]) / double(pos[J] - pos[J - 1]);
      T.parents[i].push_back({J - 1, 1.0 - t});
      T.parents[i].push_back({J, t});
    }
  }
  return T;
}

// Galerkin coarse stencil P^T A P with the tensor-product 1D transfer.
std::vector<double> rap(int D, int n, const std::vector<double>& st, int nc, int f) {
  const int nv = n - 1, nvc = nc - 1, NS = nstencil(D);
  Transfer1D T1 = transfer_1d(n, f);
  std::vector<double> out((size_t)ipow(nvc, D) * NS, 0.0);
  const size_t nvt = (size_t)ipow(nv, D);
  for (size_t v = 0; v < nvt; ++v) {
    int x[3] = {(int)(v % nv), (int)((v / nv) % nv), D == 3 ? (int)(v / ((size_t)nv * nv)) : 0};
    for (int s = 0; s < NS; ++s) {
      const double a = st[v * NS + s];
      if (a == 0.0) continue;
      int y[3] = {x[0] + s % 3 - 1, x[1] + (s / 3) % 3 - 1, D == 3 ? x[2] + s / 9 - 1 : 0};
      // parents of fine interior vertex x+1 and y+1 (1-based vertex ids)
      auto& px = T1.parents[x[0] + 1];
      auto& py = T1.parents[x[1] + 1];
      auto& qx = T1.parents[y[0] + 1];
      auto& qy = T1.parents[y[1] + 1];
      static const std::vector<std::pair<int, double>> one = {{1, 1.0}};
      auto& pz = D == 3 ? T1.parents[x[2] + 1] : one;
      auto& qz = D == 3 ? T1.parents[y[2] + 1] : one;
      for (auto& Iz : pz)
        for (auto& Iy : py)
          for (auto& Ix : px) {
            if (Ix.first < 1 || Ix.first > nvc || Iy.first < 1 || Iy.first > nvc) continue;
            if (D == 3 && (Iz.first < 1 || Iz.first > nvc)) continue;
            const double wI = Ix.second * Iy.second * Iz.second;
            const size_t row = (Ix.first - 1) + (size_t)nvc * ((Iy.first - 1) + (size_t)nvc * (D == 3 ? Iz.first - 1 : 0));
            for (auto& Jz : qz)
              for (auto& Jy : qy)
                for (auto& Jx : qx) {
                  if (Jx.first < 1 || Jx.first > nvc || Jy.first < 1 || Jy.first > nvc) continue;
                  if (D == 3 && (Jz.first < 1 || Jz.first > nvc)) continue;
                  const int off = (Jx.first - Ix.first + 1) + 3 * (Jy.first - Iy.first + 1) +
                                  (D == 3 ? 9 * (Jz.first - Iz.first + 1) : 0);
                  out[row * NS + off] += wI * Jx.second * Jy.second * Jz.second * a;
                }
          }
    }
  }
  return out;
}

void build_cg_levels(hpmg_ctx* h, hipStream_t s) {
  const int D = h->dim;
  std::vector<double> kap = h->vark ? h->kappa : std::vector<double>((size_t)ipow(h->n, D), h->kappa_const);
  std::vector<double> st = q1_stencil(D, h->n, kap);
  int m = h->n;
  while (true) {
    CGLevel L;
    L.n = m;
    L.nv = m - 1;
    L.size = (size_t)ipow(L.nv, D);
    const int NS = nstencil(D);
    std::vector<double> dinv(L.size);
    for (size_t v = 0; v < L.size; ++v) dinv[v] = 1.0 / st[v * NS + NS / 2];
    // device copy point-major: st[s * size + v]
    std::vector<double> stp(st.size());
    for (size_t v = 0; v < L.size; ++v)
      for (int k = 0; k < NS; ++k) stp[(size_t)k * L.size + v] = st[v * NS + k];
    L.d.st = h->mem.upload(stp, s);
    L.f.st = h->mem.upload(cast_vec<float>(stp), s);
    L.d.dinv = h->mem.upload(dinv, s);
    L.f.dinv = h->mem.upload(cast_vec<float>(dinv), s);
    const size_t R = h->opt.max_rhs;
    for (int b = 0; b < 2; ++b) {
      L.d.u[b] = (double*)h->mem.alloc(L.size * R * sizeof(double));
      L.f.u[b] = (float*)h->mem.alloc(L.size * R * sizeof(float));
    }
    L.d.b = (double*)h->mem.alloc(L.size * R * sizeof(double));
    L.f.b = (float*)h->mem.alloc(L.size * R * sizeof(float));
    L.d.r = (double*)h->mem.alloc(L.size * R * sizeof(double));
    L.f.r = (float*)h->mem.alloc(L.size * R * sizeof(float));
    const bool last = m <= h->opt.coarsest_n;
    if (last) {
      // dense inverse of the coarsest operator by Cholesky (FP64)
      const int M = (int)L.size;
      std::vector<double> A((size_t)M * M, 0.0);
      for (int v = 0; v < M; ++v) {
        int x[3] = {v % L.nv, (v / L.nv) % L.nv, D == 3 ? v / (L.nv * L.nv) : 0};
        for (int k = 0; k < NS; ++k) {
          int y[3] = {x[0] + k % 3 - 1, x[1] + (k / 3) % 3 - 1, D == 3 ? x[2] + k / 9 - 1 : 0};
          if (y[0] < 0 || y[0] >= L.nv || y[1] < 0 || y[1] >= L.nv || y[2] < 0 || y[2] >= (D == 3 ? L.nv : 1)) continue;
          const int w = y[0] + L.nv * (y[1] + L.nv * y[2]);
          A[(size_t)v * M + w] = st[(size_t)v * NS + k];
        }
      }
      std::vector<double> C((size_t)M * M, 0.0);
      for (int j = 0; j < M; ++j) {
        double d = A[(size_t)j * M + j];
        for (int k = 0; k < j; ++k) d -= C[(size_t)j * M + k] * C[(size_t)j * M + k];
        require(d > 0.0, "coarsest operator not positive definite");
        C[(size_t)j * M + j] = std::sqrt(d);
        for (int i = j + 1; i < M; ++i) {
          double t = A[(size_t)i * M + j];
          for (int k = 0; k < j; ++k) t -= C[(size_t)i * M + k] * C[(size_t)j * M + k];
          C[(size_t)i * M + j] = t / C[(size_t)j * M + j];
        }
      }
      std::vector<double> inv((size_t)M * M, 0.0), e(M), y(M);
      for (int col = 0; col < M; ++col) {
        std::fill(e.begin(), e.end(), 0.0);
        e[col] = 1.0;
        for (int i = 0; i < M; ++i) {
          double t = e[i];
          for (int k = 0; k < i; ++k) t -= C[(size_t)i * M + k] * y[k];
          y[i] = t / C[(size_t)i * M + i];
        }
        for (int i = M - 1; i >= 0; --i) {
          double t = y[i];
          for (int k = i + 1; k < M; ++k) t -= C[(size_t)k * M + i] * e[k];
          e[i] = t / C[(size_t)i * M + i];
        }
        for (int i = 0; i < M; ++i) inv[(size_t)i * M + col] = e[i];
      }
      h->coarse_inv = h->mem.upload(inv, s);
      h->coarse_m = M;
      h->cg.push_back(L);
      break;
    }
    // transfer to the next coarser grid
    const int hf = h->opt.h_factor;
    std::vector<int> pos = coarse_positions(m, hf);
    const int mc = (int)pos.size() - 1;
    const int nvc = mc - 1;
    Transfer1D T1 = transfer_1d(m, hf);
    const int RK = 2 * hf - 1;  // fine vertices within reach of a coarse hat
    L.rk = RK;
    std::vector<int> ridx((size_t)nvc * RK, -1), pidx((size_t)L.nv * 2, -1);
    std::vector<double> rw((size_t)nvc * RK, 0.0), pw((size_t)L.nv * 2, 0.0);
    std::vector<int> cnt(nvc, 0);
    for (int i = 1; i < m; ++i) {  // fine interior vertex i
      int k = 0;
      for (auto& pr : T1.parents[i]) {
        if (pr.first >= 1 && pr.first <= nvc) {
          pidx[(size_t)(i - 1) * 2 + k] = pr.first - 1;
          pw[(size_t)(i - 1) * 2 + k] = pr.second;
          const int I = pr.first - 1;
          require(cnt[I] < RK, "internal: restriction stencil wider than 2 factor - 1");
          ridx[(size_t)I * RK + cnt[I]] = i - 1;
          rw[(size_t)I * RK + cnt[I]] = pr.second;
          ++cnt[I];
        }
        ++k;
      }
    }
    L.ridx = h->mem.upload(ridx, s);
    L.pidx = h->mem.upload(pidx, s);
    L.d.rw = h->mem.upload(rw, s);
    L.f.rw = h->mem.upload(cast_vec<float>(rw), s);
    L.d.pw = h->mem.upload(pw, s);
    L.f.pw = h->mem.upload(cast_vec<float>(pw), s);
    st = rap(D, m, st, mc, hf);
    h->cg.push_back(L);
    m = mc;
  }
}

// ------------------------------------------------------- adaptive meshes
// Leaves of a spacetree over the unit box (Section 2.1): n^dim base cells,
// a refined cell split into r^dim children.  Validated here: coordinates in
// range, no duplicate leaf, no leaf inside another, the leaves cover the
// box, facet neighbours at most one level apart.  Built: per cell the mask
// (boundary bits f, hanging-coarse-side bits 8 + f), the neighbour-side
// trace slot of every facet, the hanging interfaces, (h_base / h_c)^(d-2),
// the leaf geometry, and the Q1 transfers between the base mesh's interior
// vertices and the leaves' corners.
uint64_t leaf_key(int lvl, const int* x, int D) {
  uint64_t k = (uint64_t)lvl;
  for (int i = 0; i < D; ++i) k |= (uint64_t)x[i] << (4 + 20 * i);
  return k;
}

// Device tables of one leaf set (M.lev, M.X set, validated): per cell the
// facet mask and the neighbour-trace slot of every facet, the hanging
// interfaces, (h_base / h_c)^(d-2).  Facet neighbours more than one level
// apart are rejected.
void build_mesh_tables(hpmg_ctx* h, AdaptMesh& M, hipStream_t s) {
  const int D = h->dim, n = h->n, r = h->rfac, nl = M.ncell, m = h->mif;
  std::unordered_map<uint64_t, int> idx;
  idx.reserve((size_t)nl * 2);
  for (int c = 0; c < nl; ++c) idx.emplace(leaf_key(M.lev[c], &M.X[(size_t)c * 3], D), c);
  auto find = [&](int l, const int* y) -> int {
    auto it = idx.find(leaf_key(l, y, D));
    return it == idx.end() ? -1 : it->second;
  };
  std::vector<unsigned short> amask(nl, 0);
  std::vector<int> nbslot((size_t)2 * D * nl, 0);
  std::vector<int> itab;  // [nif][2 + m]
  std::unordered_map<long long, int> iface;  // (coarse cell, facet) -> interface
  auto get_iface = [&](int B, int fB) -> int {
    const long long key = (long long)B * 8 + fB;
    auto it = iface.find(key);
    if (it != iface.end()) return it->second;
    const int i = (int)iface.size();
    iface.emplace(key, i);
    itab.resize((size_t)(i + 1) * (2 + m), -1);
    itab[(size_t)i * (2 + m)] = B;
    itab[(size_t)i * (2 + m) + 1] = fB;
    return i;
  };
  std::vector<std::pair<int, int>> slot_fix;  // (index into nbslot, interface slot offset)
  std::vector<int> slot_if;
  for (int c = 0; c < nl; ++c) {
    const int l = M.lev[c];
    const int* x = &M.X[(size_t)c * 3];
    const long long ext = n * (long long)std::pow((double)r, l) + 0.5;
    for (int f = 0; f < 2 * D; ++f) {
      const int k = f >> 1, sd = f & 1;
      const size_t ns = (size_t)f * nl + c;
      int y[3] = {x[0], x[1], x[2]};
      y[k] += sd ? 1 : -1;
      if (y[k] < 0 || y[k] >= ext) {
        amask[c] |= (unsigned short)(1u << f);
        nbslot[ns] = (int)ns;  // read, then zeroed: any valid slot
        continue;
      }
      const int nb = find(l, y);
      if (nb >= 0) {
        nbslot[ns] = (int)((size_t)(f ^ 1) * nl + nb);
        continue;
      }
      int yc[3] = {y[0] / r, y[1] / r, y[2] / r};
      const int big = l > 0 ? find(l - 1, yc) : -1;
      if (big >= 0) {
        // c is a fine cell of the hanging facet (big, f ^ 1); its position
        // along the tangential axes, lower axis first
        const int i = get_iface(big, f ^ 1);
        int pos = 0, mul = 1;
        for (int t = 0; t < D; ++t) {
          if (t == k) continue;
          pos += (x[t] - r * yc[t]) * mul;
          mul *= r;
        }
        require(itab[(size_t)i * (2 + m) + 2 + pos] == -1, "two leaves on one part of a hanging facet");
        itab[(size_t)i * (2 + m) + 2 + pos] = c;
        slot_fix.push_back({(int)ns, pos});
        slot_if.push_back(i);
        continue;
      }
      // the neighbour region is refined: its r^(d-1) children on the facet
      // must be leaves
      const int i = get_iface(c, f);
      for (int q = 0; q < m; ++q) {
        int z[3] = {r * y[0], r * y[1], r * y[2]};
        z[k] = r * y[k] + (sd ? 0 : r - 1);
        int qq = q;
        for (int t = 0; t < D; ++t) {
          if (t == k) continue;
          z[t] += qq % r;
          qq /= r;
        }
        require(find(l + 1, z) >= 0, "facet neighbours more than one level apart (the mesh is not balanced)");
      }
      amask[c] |= (unsigned short)(1u << (8 + f));
      slot_fix.push_back({(int)ns, m});
      slot_if.push_back(i);
    }
  }
  M.nif = (int)iface.size();
  for (int i = 0; i < M.nif; ++i)
    for (int q = 0; q < m; ++q)
      require(itab[(size_t)i * (2 + m) + 2 + q] >= 0, "a hanging facet is not covered by finer leaves");
  const size_t base0 = (size_t)2 * D * nl;
  for (size_t j = 0; j < slot_fix.size(); ++j)
    nbslot[slot_fix[j].first] = (int)(base0 + (size_t)slot_if[j] * (m + 1) + slot_fix[j].second);
  require(base0 + (size_t)M.nif * (m + 1) < (size_t)1 << 31, "mesh too large");
  M.amask = h->mem.upload(amask, s);
  M.nbslot = h->mem.upload(nbslot, s);
  if (M.nif > 0) M.itab = h->mem.upload(itab, s);
  std::vector<unsigned char> bm(nl);
  for (int c = 0; c < nl; ++c) bm[c] = (unsigned char)(amask[c] & 0xff);
  M.bmask = h->mem.upload(bm, s);
  if (D == 3) {
    std::vector<double> hs(nl);
    for (int c = 0; c < nl; ++c) hs[c] = std::pow((double)r, M.lev[c]);
    M.hs_d = h->mem.upload(hs, s);
    M.hs_f = h->mem.upload(cast_vec<float>(hs), s);
  }
}

// The caller's leaves (validated: coordinates in range, no duplicate, no
// leaf inside another, the leaves cover the box), then, if the options ask
// for it, the coarser spacetree levels down to the base mesh with the
// transfers between consecutive sets, then the Q1 transfers of the last set.
void build_adaptive(hpmg_ctx* h, const hpmg_adaptive_mesh* am, hipStream_t s) {
  const int D = h->dim, n = h->n, r = h->rfac, nl = h->ncell;
  h->mif = ipow(r, D - 1);
  AdaptMesh M0;
  M0.ncell = nl;
  M0.lev.resize(nl);
  M0.X.assign((size_t)nl * 3, 0);
  int lmax = 0;
  for (int c = 0; c < nl; ++c) {
    const int* row = am->leaves + (size_t)c * (1 + D);
    M0.lev[c] = row[0];
    require(row[0] >= 0 && row[0] <= 12, "leaf level must be in [0, 12]");
    lmax = std::max(lmax, row[0]);
  }
  long long ext_max = n;
  for (int l = 0; l < lmax; ++l) ext_max *= r;
  require(ext_max <= (1 << 20), "leaves too fine: n r^level must not exceed 2^20");
  std::unordered_map<uint64_t, int> idx;
  idx.reserve((size_t)nl * 2);
  unsigned long long vol = 0, full = 1;
  for (int k = 0; k < D; ++k) full *= (unsigned long long)ext_max;
  for (int c = 0; c < nl; ++c) {
    const int* row = am->leaves + (size_t)c * (1 + D);
    const long long ext = n * (long long)std::pow((double)r, M0.lev[c]) + 0.5;
    for (int k = 0; k < D; ++k) {
      require(row[1 + k] >= 0 && row[1 + k] < ext, "leaf coordinate out of range for its level");
      M0.X[(size_t)c * 3 + k] = row[1 + k];
    }
    require(idx.emplace(leaf_key(M0.lev[c], &M0.X[(size_t)c * 3], D), c).second, "duplicate leaf");
    unsigned long long v = 1;
    for (int l = M0.lev[c]; l < lmax; ++l) v *= (unsigned long long)ipow(r, D);
    vol += v;
  }
  for (int c = 0; c < nl; ++c) {  // no leaf lies inside another leaf
    int y[3] = {M0.X[(size_t)c * 3], M0.X[(size_t)c * 3 + 1], M0.X[(size_t)c * 3 + 2]};
    for (int l = M0.lev[c] - 1; l >= 0; --l) {
      for (int k = 0; k < D; ++k) y[k] /= r;
      require(idx.find(leaf_key(l, y, D)) == idx.end(), "a leaf lies inside another leaf");
    }
  }
  require(vol == full, "the leaves do not cover the unit box");
  // leaf geometry of the caller's leaves (load vectors)
  h->leaf_h.resize(nl);
  h->leaf_org.resize((size_t)nl * D);
  for (int c = 0; c < nl; ++c) {
    h->leaf_h[c] = 1.0 / (n * std::pow((double)r, M0.lev[c]));
    for (int k = 0; k < D; ++k) h->leaf_org[(size_t)c * D + k] = M0.X[(size_t)c * 3 + k] * h->leaf_h[c];
  }
  build_mesh_tables(h, M0, s);
  h->amesh.clear();
  h->amesh.push_back(std::move(M0));
  // coarser spacetree levels: the deepest leaves merged into their parents
  // (each parent placed where its first child was), down to the base mesh
  const int rd = ipow(r, D);
  while (h->opt.spacetree_levels) {
    AdaptMesh& F = h->amesh.back();
    const int lm = *std::max_element(F.lev.begin(), F.lev.end());
    if (lm == 0) break;
    AdaptMesh C;
    std::unordered_map<uint64_t, int> where;
    std::vector<int> pmap(F.ncell);
    std::vector<std::vector<int>> kids;
    std::vector<char> merged;
    for (int c = 0; c < F.ncell; ++c) {
      int l = F.lev[c];
      int y[3] = {F.X[(size_t)c * 3], F.X[(size_t)c * 3 + 1], F.X[(size_t)c * 3 + 2]};
      int pos = 31;
      if (l == lm) {
        pos = 0;
        for (int k = D - 1; k >= 0; --k) pos = pos * r + y[k] % r;
        for (int k = 0; k < D; ++k) y[k] /= r;
        --l;
      }
      const uint64_t key = leaf_key(l, y, D);
      auto it = where.find(key);
      int ci;
      if (it == where.end()) {
        ci = C.ncell++;
        where.emplace(key, ci);
        C.lev.push_back(l);
        C.X.insert(C.X.end(), y, y + 3);
        kids.emplace_back(rd, -1);
        merged.push_back(pos != 31);
      } else {
        ci = it->second;
      }
      pmap[c] = ci * 32 + pos;
      kids[ci][pos == 31 ? 0 : pos] = c;
    }
    std::vector<int> rmap((size_t)C.ncell * rd);
    for (int ci = 0; ci < C.ncell; ++ci) {
      for (int q = 0; q < rd; ++q) {
        require(!merged[ci] || kids[ci][q] >= 0, "a refined cell without all its children");
        rmap[(size_t)ci * rd + q] = kids[ci][q];
      }
    }
    F.pmap = h->mem.upload(pmap, s);
    F.rmap = h->mem.upload(rmap, s);
    build_mesh_tables(h, C, s);
    h->amesh.push_back(std::move(C));
  }
  // Q1 transfers of the last leaf set: corner j of cell c lies at
  // t = (x - B r^l + bit(j)) / r^l inside its base cell B; the base vertex
  // B + w (w in {0,1}^d) has the weight prod_k (w_k ? t_k : 1 - t_k) there
  // (zero boundary vertices left out)
  const AdaptMesh& L = h->amesh.back();
  const int nv = n - 1, nc = 1 << D;
  std::vector<std::vector<std::pair<int, double>>> prow((size_t)L.ncell * nc);
  std::vector<std::vector<std::pair<int, double>>> rrow((size_t)ipow(nv, D));
  for (int c = 0; c < L.ncell; ++c) {
    const long long rl = (long long)(std::pow((double)r, L.lev[c]) + 0.5);
    for (int j = 0; j < nc; ++j) {
      double t[3];
      int Bc[3];
      for (int k = 0; k < D; ++k) {
        const long long xk = L.X[(size_t)c * 3 + k];
        Bc[k] = (int)(xk / rl);
        t[k] = (double)(xk - Bc[k] * rl + ((j >> k) & 1)) / (double)rl;
      }
      for (int w = 0; w < nc; ++w) {
        double wt = 1.0;
        int vid = 0, mul = 1;
        bool inside = true;
        for (int k = 0; k < D; ++k) {
          const int bit = (w >> k) & 1;
          wt *= bit ? t[k] : 1.0 - t[k];
          const int v = Bc[k] + bit;
          inside = inside && v > 0 && v < n;
          vid += (v - 1) * mul;
          mul *= nv;
        }
        if (!inside || wt == 0.0) continue;
        prow[(size_t)c * nc + j].push_back({vid, wt});
        rrow[vid].push_back({c * nc + j, wt});
      }
    }
  }
  auto upload_csr = [&](const std::vector<std::vector<std::pair<int, double>>>& rows, int** ptr, int** col,
                        double** wd, float** wf) {
    std::vector<int> pv(rows.size() + 1, 0), cv;
    std::vector<double> wv;
    for (size_t i = 0; i < rows.size(); ++i) {
      for (auto& e : rows[i]) {
        cv.push_back(e.first);
        wv.push_back(e.second);
      }
      pv[i + 1] = (int)cv.size();
    }
    if (cv.empty()) {
      cv.push_back(0);
      wv.push_back(0.0);
    }
    *ptr = h->mem.upload(pv, s);
    *col = h->mem.upload(cv, s);
    *wd = h->mem.upload(wv, s);
    *wf = h->mem.upload(cast_vec<float>(wv), s);
  };
  h->q1p_rows = (int)prow.size();
  h->q1r_rows = (int)rrow.size();
  upload_csr(prow, &h->q1p_ptr, &h->q1p_col, &h->q1p_wd, &h->q1p_wf);
  upload_csr(rrow, &h->q1r_ptr, &h->q1r_col, &h->q1r_wd, &h->q1r_wf);
}

// --------------------------------------------------------------- execution
template <typename T>
void project(hpmg_ctx* h, int l, const T* u, T* tr, int nrhs, hipStream_t s) {
  DGLevel& L = h->dg[l];
  hpmg::DGArgs<T> a = dg_args<T>(h, L);
  a.u_in = u;
  a.tr_out = tr;
  dg_run(h, hpmg::OP_PROJECT, a, L.N, nrhs, 0, s);
}

template <typename T>
void sweep(hpmg_ctx* h, int l, T* u, const T* b, const T* trin, T* trout, bool uzero, int nrhs, hipStream_t s) {
  DGLevel& L = h->dg[l];
  hpmg::DGArgs<T> a = dg_args<T>(h, L);
  a.u_in = u;
  a.u_out = u;
  a.b = b;
  a.tr_in = trin;
  a.tr_out = trout;
  dg_run(h, hpmg::OP_SWEEP, a, L.N, nrhs, uzero ? 1 : 0, s);
}

template <typename T>
void apply(hpmg_ctx* h, int l, const T* u, const T* tr, const T* b, T* out, int nrhs, hipStream_t s) {
  DGLevel& L = h->dg[l];
  hpmg::DGArgs<T> a = dg_args<T>(h, L);
  a.u_in = u;
  a.tr_in = tr;
  a.b = b;
  a.out = out;
  dg_run(h, hpmg::OP_APPLY, a, L.N, nrhs, b ? 1 : 0, s);
}

// Smoothing steps on the Q1 levels (their own counts, or the DG ones).
int cg_nu_pre(const hpmg_ctx* h) { return h->opt.nu_pre_cg >= 0 ? h->opt.nu_pre_cg : h->opt.nu_pre; }
int cg_nu_post(const hpmg_ctx* h) { return h->opt.nu_post_cg >= 0 ? h->opt.nu_post_cg : h->opt.nu_post; }

// The Q1 part of a V-cycle for right-hand side `col` (the level vectors
// hold max_rhs columns of L.size entries each).
template <typename T>
void vcycle_cg(hpmg_ctx* h, int m, bool uzero, int col, hipStream_t s) {
  CGLevel& L = h->cg[m];
  CGData<T>& d = data<T>(L);
  const int D = h->dim;
  const size_t o = (size_t)col * L.size;
  T* u[2] = {d.u[0] + o, d.u[1] + o};
  T* b = d.b + o;
  T* r = d.r + o;
  if (m + 1 == (int)h->cg.size()) {
    hpmg::dense_solve<T>(h->coarse_m, h->coarse_inv, b, u[0], s);
    L.cur = 0;
    HIPCHK(hipGetLastError());
    return;
  }
  const T w = (T)h->opt.omega_cg;
  const int npre = cg_nu_pre(h), npost = cg_nu_post(h);
  const int nlev = (int)h->cg.size() - m;
  if (uzero && L.size <= (size_t)hpmg::CG_BLOCK_MAX_VERTICES && nlev <= hpmg::CG_BLOCK_MAX_LEVELS) {
    // this level and all coarser ones are small: the rest of the cycle in
    // one workgroup
    hpmg::CGBlockArgs<T> a{};
    a.nlev = nlev;
    a.nu_pre = npre;
    a.nu_post = npost;
    a.m = h->coarse_m;
    a.omega = w;
    a.Ainv = h->coarse_inv;
    for (int k = 0; k < nlev; ++k) {
      CGLevel& Lk = h->cg[m + k];
      CGData<T>& dk = data<T>(Lk);
      const size_t ok = (size_t)col * Lk.size;
      a.lv[k] = {Lk.nv, dk.st, dk.dinv, {dk.u[0] + ok, dk.u[1] + ok}, dk.b + ok, dk.r + ok, Lk.ridx, dk.rw,
                 Lk.pidx, dk.pw};
      Lk.cur = k + 1 == nlev ? 0 : (npre + npost) & 1;
    }
    hpmg::cg_vcycle_block<T>(D, L.rk, a, s);
    HIPCHK(hipGetLastError());
    return;
  }
  int cur = 0;
  bool zero = uzero;
  for (int i = 0; i < npre; ++i) {
    hpmg::cg_stencil<T>(D, L.nv, d.st, d.dinv, u[cur], b, u[cur ^ 1], w, 0, zero ? 1 : 0, s);
    cur ^= 1;
    zero = false;
  }
  if (zero) {
    hpmg::fill<T>(u[cur], L.size, T(0), s);
    zero = false;
  }
  hpmg::cg_stencil<T>(D, L.nv, d.st, d.dinv, u[cur], b, r, w, 1, 0, s);
  CGLevel& C = h->cg[m + 1];
  CGData<T>& dc = data<T>(C);
  const size_t oc = (size_t)col * C.size;
  hpmg::cg_restrict<T>(D, L.nv, C.nv, L.rk, L.ridx, d.rw, r, dc.b + oc, s);
  vcycle_cg<T>(h, m + 1, true, col, s);
  hpmg::cg_prolong<T>(D, L.nv, C.nv, L.pidx, d.pw, dc.u[C.cur] + oc, u[cur], s);
  for (int i = 0; i < npost; ++i) {
    hpmg::cg_stencil<T>(D, L.nv, d.st, d.dinv, u[cur], b, u[cur ^ 1], w, 0, 0, s);
    cur ^= 1;
  }
  L.cur = cur;
  HIPCHK(hipGetLastError());
}

// Weights of the Q1 transfers of an adaptive mesh in the compute type
// (restriction: rows = base vertices; else prolongation: rows = corners).
template <typename C>
const C* q1_weights(const hpmg_ctx* h, bool restr) {
  if constexpr (std::is_same<C, double>::value)
    return restr ? h->q1r_wd : h->q1p_wd;
  else
    return restr ? h->q1r_wf : h->q1p_wf;
}

// One V-cycle on DG level l for nrhs stacked right-hand sides; u, b are the
// level's vectors (for l = 0 the caller's).  Traversals on the level:
// [projection], nu_pre sweeps, residual + restriction, prolongation +
// projection, nu_post sweeps (each one launch over all columns); the Q1
// levels run column after column.
template <typename T>
void vcycle_dg(hpmg_ctx* h, int l, T* u, const T* b, bool uzero, int nrhs, hipStream_t s) {
  // 16-bit storage applies to this level only: the coarser levels run in
  // the compute type C
  using C = hpmg::CT<T>;
  DGLevel& L = h->dg[l];
  DGData<T>& d = data<T>(L);
  int cur = 0;
  bool zero = uzero;
  if (zero && h->opt.nu_pre == 0) {
    hpmg::fill<T>(u, L.ndof * nrhs, T(0), s);
    zero = false;
  }
  if (!zero) project<T>(h, l, u, d.tr[0], nrhs, s);
  for (int i = 0; i < h->opt.nu_pre; ++i) {
    sweep<T>(h, l, u, b, d.tr[cur], d.tr[cur ^ 1], zero, nrhs, s);
    cur ^= 1;
    zero = false;
  }
  // residual and restriction
  hpmg::DGArgs<T> a = dg_args<T>(h, L);
  a.u_in = u;
  a.tr_in = d.tr[cur];
  a.b = b;
  if (L.next_h) {
    // the same degree on the next coarser spacetree level: r = b - A u,
    // restricted child by child; the correction prolongated by the parents'
    // polynomials, then the traces of the corrected u
    DGLevel& Cl = h->dg[l + 1];
    DGData<C>& dc = data<C>(Cl);
    DGData<C>& dl = data<C>(L);
    const AdaptMesh& Mf = h->amesh[L.am];
    const AdaptMesh& Mc = h->amesh[Cl.am];
    a.out = dl.rtmp;
    dg_run(h, hpmg::OP_APPLY, a, L.N, nrhs, 1, s);
    hpmg::spacetree_transfer<C>(true, h->dim, L.N, Mc.ncell, Mf.rmap, h->rfac, dl.mort, dl.rtmp, dc.b,
                                (long long)L.ndof, (long long)Cl.ndof, nrhs, s);
    HIPCHK(hipGetLastError());
    vcycle_dg<C>(h, l + 1, dc.u, dc.b, true, nrhs, s);
    if constexpr (std::is_same<T, C>::value) {
      hpmg::spacetree_transfer<C>(false, h->dim, L.N, Mf.ncell, Mf.pmap, h->rfac, dl.mort, dc.u, u,
                                  (long long)L.ndof, (long long)Cl.ndof, nrhs, s);
      HIPCHK(hipGetLastError());
    } else {
      throw HpmgError(HPMG_E_UNSUPPORTED, "adaptive meshes take FP64 or FP32 vectors");
    }
    project<T>(h, l, u, d.tr[cur], nrhs, s);
  } else if (!L.next_cg) {
    DGLevel& Cl = h->dg[l + 1];
    DGData<C>& dc = data<C>(Cl);
    a.out = dc.b;
    a.cstride = (long long)Cl.ndof;
    a.ncd = Cl.N;
    dg_run(h, L.dyn_nc ? hpmg::OP_RESTRICT_DYN : hpmg::OP_RESTRICT, a, L.N, nrhs, 1, s);
    vcycle_dg<C>(h, l + 1, dc.u, dc.b, true, nrhs, s);
    hpmg::DGArgs<T> pa = dg_args<T>(h, L);
    pa.u_in = u;
    pa.u_out = u;
    pa.tr_out = d.tr[cur];
    pa.coarse = dc.u;
    pa.coarse_cg = 0;
    pa.cstride = (long long)Cl.ndof;
    pa.ncd = Cl.N;
    dg_run(h, L.dyn_nc ? hpmg::OP_PROLONG_DYN : hpmg::OP_PROLONG, pa, L.N, nrhs, 0, s);
  } else {
    CGLevel& Cg = h->cg[0];
    CGData<C>& dc = data<C>(Cg);
    const size_t nct = (size_t)h->ncell << h->dim;
    C* contrib = data<C>(L).contrib;
    a.out = contrib;
    a.cstride = (long long)nct;
    dg_run(h, hpmg::OP_RESTRICT_Q1, a, L.N, nrhs, 1, s);
    for (int c = 0; c < nrhs; ++c) {
      if (h->adapt)  // base vertices <- corners of the leaves inside their cells
        hpmg::csr_apply<C>(h->q1r_rows, h->q1r_ptr, h->q1r_col, q1_weights<C>(h, true), contrib + c * nct,
                           dc.b + c * Cg.size, s);
      else
        hpmg::gather_corners<C>(h->dim, h->n, contrib + c * nct, dc.b + c * Cg.size, s);
      vcycle_cg<C>(h, 0, true, c, s);
    }
    hpmg::DGArgs<T> pa = dg_args<T>(h, L);
    pa.u_in = u;
    pa.u_out = u;
    pa.tr_out = d.tr[cur];
    if (h->adapt) {
      // corner values of every leaf from the base vertices (the Q1
      // function evaluated at the leaf's corners), then the per-cell
      // trilinear interpolation of the prolongation kernel
      for (int c = 0; c < nrhs; ++c)
        hpmg::csr_apply<C>(h->q1p_rows, h->q1p_ptr, h->q1p_col, q1_weights<C>(h, false),
                           dc.u[Cg.cur] + c * Cg.size, contrib + c * nct, s);
      pa.coarse = contrib;
      pa.coarse_cg = 2;
      pa.cstride = (long long)nct;
    } else {
      pa.coarse = dc.u[Cg.cur];
      pa.coarse_cg = 1;
      pa.cstride = (long long)Cg.size;
    }
    dg_run(h, hpmg::OP_PROLONG_Q1, pa, L.N, nrhs, 0, s);
  }
  for (int i = 0; i < h->opt.nu_post; ++i) {
    sweep<T>(h, l, u, b, d.tr[cur], d.tr[cur ^ 1], false, nrhs, s);
    cur ^= 1;
  }
}

// One finest-level sweep with block_recompute = 2 (split and postpone,
// Section 4.3): the sweep reads the current per-cell records while the
// records of the next traversal are rebuilt from kappa (the eigensolve of
// the recompute variant) on the handle's second stream into the other
// buffer; the next sweep waits for that rebuild, a rebuild waits for the
// last sweep that read its buffer.
template <typename T>
void sweep_split(hpmg_ctx* h, T* u, const T* b, const T* trin, T* trout, int nrhs, hipStream_t s) {
  using C = hpmg::CT<T>;
  DGLevel& L = h->dg[0];
  DGData<C>& dc = data<C>(L);
  const int pi = std::is_same<C, double>::value ? 0 : 1;
  const int cur = dc.ecur, nxt = cur ^ 1;
  HIPCHK(hipStreamWaitEvent(s, h->ev_built[pi][cur], 0));
  sweep<T>(h, 0, u, b, trin, trout, false, nrhs, s);
  HIPCHK(hipEventRecord(h->ev_used[pi][cur], s));
  HIPCHK(hipStreamWaitEvent(h->bs, h->ev_used[pi][nxt], 0));
  hpmg::DGArgs<C> a = dg_args<C>(h, L);
  a.rk = dc.rkb;
  a.out = dc.ebuf[nxt];
  a.flag = nullptr;
  dg_run(h, hpmg::OP_BUILD_EIG, a, L.N, 1, 0, h->bs);
  HIPCHK(hipEventRecord(h->ev_built[pi][nxt], h->bs));
  dc.ecur = nxt;
  dc.eig = dc.ebuf[nxt];
}

// After split sweeps: work queued next on s sees the current records.
template <typename T>
void split_join(hpmg_ctx* h, hipStream_t s) {
  using C = hpmg::CT<T>;
  const int pi = std::is_same<C, double>::value ? 0 : 1;
  HIPCHK(hipStreamWaitEvent(s, h->ev_built[pi][data<C>(h->dg[0]).ecur], 0));
}

// Finest-level traces of a 16-bit storage type, allocated on first use.
template <typename T>
void ensure_traces(hpmg_ctx* h) {
  DGLevel& L = h->dg[0];
  DGData<T>& d = data<T>(L);
  if (d.tr[0]) return;
  const size_t R = h->opt.max_rhs;
  for (int k = 0; k < 2; ++k) d.tr[k] = (T*)h->mem.alloc(L.trsize * R * sizeof(T));
}

// Calls f with a null T* for the storage type of dtype (16-bit traces
// allocated first).
template <class F>
void by_dtype(hpmg_ctx* h, int dtype, F f) {
  switch (dtype) {
    case HPMG_F64: f((double*)nullptr); break;
    case HPMG_F32: f((float*)nullptr); break;
    case HPMG_F16:
      if (h->adapt) throw HpmgError(HPMG_E_UNSUPPORTED, "adaptive meshes take FP64 or FP32 vectors");
      ensure_traces<_Float16>(h);
      f((_Float16*)nullptr);
      break;
    case HPMG_BF16:
      if (h->adapt) throw HpmgError(HPMG_E_UNSUPPORTED, "adaptive meshes take FP64 or FP32 vectors");
      ensure_traces<__bf16>(h);
      f((__bf16*)nullptr);
      break;
    default: throw HpmgError(HPMG_E_INVALID, "bad dtype");
  }
}

hpmg_status fail(const HpmgError& e) {
  g_last_error = e.what();
  return e.st;
}

}  // namespace

// ====================================================================== ABI
namespace {

// Restarts from the true residual allowed per right-hand side before a
// solve that cannot reach rtol in FP64 gives up.
constexpr int kMaxRestarts = 3;

// Workspace of the reduced-precision cycles (on first use) and the scale of
// the residual handed to a 16-bit cycle (see hpmg_solve).
double lowp_setup(hpmg_ctx* h) {
  const size_t nd = h->ndof;
  if (h->opt.precision == HPMG_PREC_F16) {
    ensure_traces<_Float16>(h);
    if (!h->r16) {
      h->r16 = (_Float16*)h->mem.alloc(nd * sizeof(_Float16));
      h->z16 = (_Float16*)h->mem.alloc(nd * sizeof(_Float16));
    }
  } else if (h->opt.precision == HPMG_PREC_BF16) {
    ensure_traces<__bf16>(h);
    if (!h->rb16) {
      h->rb16 = (__bf16*)h->mem.alloc(nd * sizeof(__bf16));
      h->zb16 = (__bf16*)h->mem.alloc(nd * sizeof(__bf16));
    }
  }
  // 16-bit cycles: the residual handed to the cycle gets mean square
  // lambda, lambda = d pi^2 kappa_min (h/N)^d (the smallest eigenvalue of
  // A for unit-scaled nodal vectors), so that its entries and those of the
  // correction (about r / lambda for smooth r) stay in FP16 range
  double kmin = h->kappa_const;
  if (h->vark) kmin = *std::min_element(h->kappa.begin(), h->kappa.end());
  const double lam = h->dim * M_PI * M_PI * kmin * std::pow(1.0 / (h->n * (h->p + 1.0)), h->dim);
  return std::sqrt((double)nd * lam);
}

// z = M r: one V-cycle from zero in the handle's cycle precision (r, z FP64;
// scal[7], scal[8] = 1/||r||, ||r|| must be current for the reduced ones).
void precondition(hpmg_ctx* h, double rms, hipStream_t stream) {
  const size_t nd = h->ndof;
  if (h->opt.precision == HPMG_PREC_F32) {
    hpmg::cast_down<float>(nd, h->r, h->r32, h->scal, 1.0, stream);
    vcycle_dg<float>(h, 0, h->z32, h->r32, true, 1, stream);
    hpmg::cast_up<float>(nd, h->z32, h->z, h->scal, 1.0, stream);
  } else if (h->opt.precision == HPMG_PREC_F16) {
    hpmg::cast_down<_Float16>(nd, h->r, h->r16, h->scal, rms, stream);
    vcycle_dg<_Float16>(h, 0, h->z16, h->r16, true, 1, stream);
    hpmg::cast_up<_Float16>(nd, h->z16, h->z, h->scal, rms, stream);
  } else if (h->opt.precision == HPMG_PREC_BF16) {
    hpmg::cast_down<__bf16>(nd, h->r, h->rb16, h->scal, rms, stream);
    vcycle_dg<__bf16>(h, 0, h->zb16, h->rb16, true, 1, stream);
    hpmg::cast_up<__bf16>(nd, h->zb16, h->z, h->scal, rms, stream);
  } else {
    vcycle_dg<double>(h, 0, h->z, h->r, true, 1, stream);
  }
}

// r = b - A u (FP64) and scal[6..8] = ||r||^2, 1/||r||, ||r||; returns ||r||.
double fp64_residual(hpmg_ctx* h, const double* u, const double* b, hipStream_t stream) {
  DGData<double>& d = h->dg[0].d;
  project<double>(h, 0, u, d.tr[0], 1, stream);
  apply<double>(h, 0, u, d.tr[0], b, h->r, 1, stream);
  hpmg::krylov_dot(h->ndof, h->r, h->r, nullptr, h->partial, h->scal, 3, 0, 0, stream);
  HIPCHK(hipMemcpyAsync(h->host_scal, h->scal, 16 * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  const double rn = std::sqrt(h->host_scal[6]);
  if (!std::isfinite(rn)) throw HpmgError(HPMG_E_BREAKDOWN, "non-finite residual");
  return rn;
}

// One outer FCG iteration on the internal vectors (ug, r, rold, pv, q and
// the cycle's z) enqueued on s, ending with the copy of the scalars to the
// pinned host buffer; restart = 1 takes beta = 0.  A reduced-precision
// cycle's z is read where it lies (the dots convert it, and the projection
// kernel forms p = z + beta p while it projects p onto its traces); the FP32
// cycle takes r unscaled, cast by the previous iteration's update (after a
// restart: by a cast here), the 16-bit cycles take r scaled to mean square
// lambda.  The apply q = A p leaves per-block shares of p.q for alpha.
void fcg_iteration(hpmg_ctx* h, double rms, int restart, hipStream_t s) {
  const size_t nd = h->ndof;
  DGLevel& L0 = h->dg[0];
  DGData<double>& d = L0.d;
  float* r32_next = nullptr;
  const void* zl = h->z;
  int zkind = HPMG_F64, scaled = 0;
  double mul = 1.0;
  switch (h->opt.precision) {
    case HPMG_PREC_F32:
      if (restart) hpmg::cast_down<float>(nd, h->r, h->r32, nullptr, 1.0, s);
      vcycle_dg<float>(h, 0, h->z32, h->r32, true, 1, s);
      hpmg::krylov_dot_lowz<float>(nd, h->z32, 0, 1.0, h->r, h->rold, h->partial, h->scal, restart, s);
      r32_next = h->r32;
      zl = h->z32;
      zkind = HPMG_F32;
      break;
    case HPMG_PREC_F16:
      hpmg::cast_down<_Float16>(nd, h->r, h->r16, h->scal, rms, s);
      vcycle_dg<_Float16>(h, 0, h->z16, h->r16, true, 1, s);
      hpmg::krylov_dot_lowz<_Float16>(nd, h->z16, 1, rms, h->r, h->rold, h->partial, h->scal, restart, s);
      zl = h->z16;
      zkind = HPMG_F16;
      scaled = 1;
      mul = rms;
      break;
    case HPMG_PREC_BF16:
      hpmg::cast_down<__bf16>(nd, h->r, h->rb16, h->scal, rms, s);
      vcycle_dg<__bf16>(h, 0, h->zb16, h->rb16, true, 1, s);
      hpmg::krylov_dot_lowz<__bf16>(nd, h->zb16, 1, rms, h->r, h->rold, h->partial, h->scal, restart, s);
      zl = h->zb16;
      zkind = HPMG_BF16;
      scaled = 1;
      mul = rms;
      break;
    default:
      vcycle_dg<double>(h, 0, h->z, h->r, true, 1, s);
      hpmg::krylov_dot(nd, h->z, h->r, h->rold, h->partial, h->scal, 1, 0, restart, s);
  }
  // p = z + beta p and its traces in one pass
  hpmg::DGArgs<double> pa = dg_args<double>(h, L0);
  pa.u_in = h->pv;
  pa.u_out = h->pv;
  pa.tr_out = d.tr[0];
  pa.kry = 1;
  pa.zkind = zkind;
  pa.zlow = zl;
  pa.zscaled = scaled;
  pa.kscal = h->scal;
  pa.kmul = mul;
  dg_run(h, hpmg::OP_PROJECT, pa, L0.N, 1, 0, s);
  // q = A p with the per-block shares of p.q, then alpha
  hpmg::DGArgs<double> aa = dg_args<double>(h, L0);
  aa.u_in = h->pv;
  aa.tr_in = d.tr[0];
  aa.out = h->q;
  aa.kdot = 1;
  aa.kpartial = h->kpartial;
  dg_run(h, hpmg::OP_APPLY, aa, L0.N, 1, 0, s);
  const int cpb = hpmg::cells_per_block(h->dim, L0.N);
  hpmg::krylov_alpha(h->kpartial, (h->ncell + cpb - 1) / cpb, h->scal, s);
  hpmg::krylov_update_ur(nd, h->ug, h->r, h->rold, h->pv, h->q, h->partial, h->scal, r32_next, s);
  HIPCHK(hipMemcpyAsync(h->host_scal, h->scal, 16 * sizeof(double), hipMemcpyDeviceToHost, s));
}

}  // namespace

extern "C" {

void hpmg_default_options(hpmg_options* o) {
  if (!o) return;
  o->sigma0 = 2.0;
  o->omega_dg = 0.7;
  o->omega_cg = 2.0 / 3.0;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->coarsest_n = 4;
  o->precision = HPMG_PREC_F32;
  o->max_rhs = 1;
  o->p_coarsening = 0;
  o->h_factor = 2;
  o->basis = 0;
  o->block_recompute = 0;
  o->nu_pre_cg = -1;
  o->nu_post_cg = -1;
  o->block_variant = 0;
  for (int i = 0; i < 8; ++i) o->p_schedule[i] = 0;
  o->alloc = nullptr;
  o->free = nullptr;
  o->alloc_ctx = nullptr;
  o->mfma = 0;
  o->spacetree_levels = 1;
}

const char* hpmg_status_string(hpmg_status s) {
  switch (s) {
    case HPMG_OK: return "ok";
    case HPMG_E_INVALID: return "invalid argument";
    case HPMG_E_NOMEM: return "out of memory";
    case HPMG_E_DEVICE: return "device error";
    case HPMG_E_NOT_CONVERGED: return "not converged";
    case HPMG_E_BREAKDOWN: return "breakdown";
    case HPMG_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* hpmg_last_error(void) { return g_last_error.c_str(); }

namespace {

// Common setup of hpmg_setup (am = NULL: the uniform n^dim mesh) and
// hpmg_setup_adaptive (the leaves of am over n^dim base cells).
hpmg_status setup_impl(int dim, int nbase, const hpmg_adaptive_mesh* am, int p, const hpmg_coeff* coeff,
                       const hpmg_options* opt, hipStream_t stream, hpmg_handle* out) {
  try {
    require(out != nullptr, "out is NULL");
    *out = nullptr;
    require(coeff != nullptr, "coeff is NULL");
    require(dim == 2 || dim == 3, "dim must be 2 or 3");
    require(nbase >= 2, "n must be >= 2");
    require(p >= 1 && p <= 8, "p must be in [1, 8]");
    const long long ncell_ll = am ? (long long)am->nleaf
                                  : (dim == 2 ? (long long)nbase * nbase : (long long)nbase * nbase * nbase);
    require(ncell_ll >= 1 && ncell_ll < (1LL << 31) / 2, "mesh too large");
    std::unique_ptr<hpmg_ctx> h(new hpmg_ctx());
    if (opt) {
      h->opt = *opt;
    } else {
      hpmg_default_options(&h->opt);
    }
    require(h->opt.sigma0 > 0.0 && std::isfinite(h->opt.sigma0), "sigma0 must be positive");
    require(h->opt.omega_dg > 0.0 && h->opt.omega_dg <= 1.0, "omega_dg must be in (0, 1]");
    require(h->opt.omega_cg > 0.0 && h->opt.omega_cg <= 1.0, "omega_cg must be in (0, 1]");
    require(h->opt.nu_pre >= 0 && h->opt.nu_post >= 0 && h->opt.nu_pre + h->opt.nu_post > 0, "bad nu");
    require(h->opt.coarsest_n >= 2, "coarsest_n must be >= 2");
    require(h->opt.max_rhs >= 1, "max_rhs must be >= 1");
    require(h->opt.precision >= HPMG_PREC_F64 && h->opt.precision <= HPMG_PREC_BF16, "bad precision");
    require(h->opt.p_coarsening == 0 || h->opt.p_coarsening == 1, "p_coarsening must be 0 or 1");
    require(h->opt.h_factor == 2 || h->opt.h_factor == 3, "h_factor must be 2 or 3");
    require(h->opt.basis == 0 || h->opt.basis == 1, "basis must be 0 (Gauss-Lobatto) or 1 (Gauss-Legendre)");
    require(h->opt.nu_pre_cg >= -1 && h->opt.nu_post_cg >= -1, "nu_pre_cg / nu_post_cg must be >= -1");
    require(h->opt.block_variant == 0 || h->opt.block_variant == 1, "block_variant must be 0 or 1");
    require(h->opt.mfma == 0 || (h->opt.mfma == 1 && dim == 3), "mfma must be 0, or 1 with dim 3");
    require(h->opt.spacetree_levels == 0 || h->opt.spacetree_levels == 1, "spacetree_levels must be 0 or 1");
    require((h->opt.alloc == nullptr) == (h->opt.free == nullptr), "alloc and free must be given together");
    h->mem.alloc_fn = h->opt.alloc;
    h->mem.free_fn = h->opt.free;
    h->mem.ctx = h->opt.alloc_ctx;
    h->dim = dim;
    h->n = nbase;
    h->p = p;
    h->ncell = (int)ncell_ll;
    if (am) {
      require(am->refine == 2 || am->refine == 3, "refine must be 2 or 3");
      require(!coeff->per_cell, "adaptive meshes take a constant kappa");
      require(h->opt.block_variant == 0 && h->opt.block_recompute == 0 && h->opt.mfma == 0,
              "adaptive meshes take the exact block, block_recompute 0 and mfma 0");
      require(h->opt.precision == HPMG_PREC_F64 || h->opt.precision == HPMG_PREC_F32,
              "adaptive meshes take an FP64 or FP32 cycle");
      h->adapt = true;
      h->rfac = am->refine;
    }
    if (coeff->per_cell) {
      require(coeff->kappa != nullptr, "kappa is NULL");
      h->vark = true;
      h->kappa.assign(coeff->kappa, coeff->kappa + h->ncell);
      for (double k : h->kappa) require(k > 0.0 && std::isfinite(k), "kappa must be positive and finite");
    } else {
      require(coeff->kappa_const > 0.0 && std::isfinite(coeff->kappa_const), "kappa_const must be positive");
      h->kappa_const = coeff->kappa_const;
    }
    require(h->opt.block_recompute == 0 || ((h->opt.block_recompute == 1 || h->opt.block_recompute == 2) && h->vark),
            "block_recompute must be 0, or 1 or 2 with a per-cell kappa");
    require(h->opt.block_variant == 0 || (!h->vark && h->n >= 3),
            "block_variant 1 (interior block) needs constant kappa and n >= 3");
    for (int i = 0, prev = p; i < 8 && h->opt.p_schedule[i] != 0; prev = h->opt.p_schedule[i], ++i)
      require(h->opt.p_schedule[i] >= 2 && h->opt.p_schedule[i] < prev,
              "p_schedule must be strictly decreasing, each entry in [2, p)");
    {
      const int npre = h->opt.nu_pre_cg >= 0 ? h->opt.nu_pre_cg : h->opt.nu_pre;
      const int npost = h->opt.nu_post_cg >= 0 ? h->opt.nu_post_cg : h->opt.nu_post;
      require(npre + npost > 0 || h->n <= h->opt.coarsest_n, "the Q1 levels need at least one smoothing step");
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    h->dev = dev;
    init_noalloc_scratch(dev);
    if (am) {
      build_adaptive(h.get(), am, stream);
    } else {
      std::vector<unsigned char> m(h->ncell);
      const int n = h->n;
      for (int c = 0; c < h->ncell; ++c) {
        int v = 0, r = c;
        for (int k = 0; k < h->dim; ++k) {
          const int x = r % n;
          r /= n;
          v |= (x == 0 ? 1 : 0) << (2 * k);
          v |= (x == n - 1 ? 1 : 0) << (2 * k + 1);
        }
        m[c] = (unsigned char)v;
      }
      h->bmask = h->mem.upload(m, stream);
    }
    // DG levels: p, then the explicit schedule, or floor(p/2), ... while
    // >= 2 (p_coarsening 0), or none (1); then Q1
    std::vector<int> degs = {p};
    if (h->opt.p_schedule[0] != 0) {
      for (int i = 0; i < 8 && h->opt.p_schedule[i] != 0; ++i) degs.push_back(h->opt.p_schedule[i]);
    } else if (h->opt.p_coarsening == 0) {
      for (int q = p / 2; q >= 2; q /= 2) degs.push_back(q);
    }
    const double sigma_hat = h->opt.sigma0 * (p + 1.0) * (p + 1.0);
    // adaptive meshes: after the p-levels (on the caller's leaves) the last
    // degree on every coarser spacetree level
    const int np = (int)degs.size();
    const int nh = h->adapt ? (int)h->amesh.size() - 1 : 0;
    for (int k = 0; k < nh; ++k) degs.push_back(degs[np - 1]);
    std::vector<hpmg::Basis1D> bases;
    for (int q : degs) bases.push_back(hpmg::make_basis(q, h->opt.basis == 1));
    h->dg.resize(degs.size());
    for (size_t l = 0; l < degs.size(); ++l) {
      DGLevel& L = h->dg[l];
      L.p = degs[l];
      L.N = degs[l] + 1;
      L.am = (int)l < np ? 0 : (int)l - np + 1;
      L.next_cg = (l + 1 == degs.size());
      L.next_h = !L.next_cg && (int)l + 1 >= np;
      L.NC = L.next_cg ? 2 : degs[l + 1] + 1;
      // transfers to a DG level other than the halved degree take the
      // kernels with a run-time coarse degree
      L.dyn_nc = !L.next_cg && !L.next_h && L.NC != hpmg::nc_next(L.N);
      L.sigma_hat = sigma_hat;
      build_dg_level(h.get(), L, bases[l], (L.next_cg || L.next_h) ? nullptr : &bases[l + 1], stream);
      const size_t R = h->opt.max_rhs;
      if (l > 0) {
        L.d.u = (double*)h->mem.alloc(L.ndof * R * sizeof(double));
        L.d.b = (double*)h->mem.alloc(L.ndof * R * sizeof(double));
        L.f.u = (float*)h->mem.alloc(L.ndof * R * sizeof(float));
        L.f.b = (float*)h->mem.alloc(L.ndof * R * sizeof(float));
      }
      if (L.next_h) {
        L.d.rtmp = (double*)h->mem.alloc(L.ndof * R * sizeof(double));
        L.f.rtmp = (float*)h->mem.alloc(L.ndof * R * sizeof(float));
      }
      if (L.next_cg) {
        const size_t ncl = h->adapt ? (size_t)h->amesh[L.am].ncell : (size_t)h->ncell;
        const size_t nct = ncl << h->dim;
        L.d.contrib = (double*)h->mem.alloc(nct * R * sizeof(double));
        L.f.contrib = (float*)h->mem.alloc(nct * R * sizeof(float));
      }
    }
    h->ndof = h->dg[0].ndof;
    if (h->opt.block_recompute == 2) {
      HIPCHK(hipStreamCreateWithFlags(&h->bs, hipStreamNonBlocking));
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          HIPCHK(hipEventCreateWithFlags(&h->ev_built[i][j], hipEventDisableTiming));
          HIPCHK(hipEventCreateWithFlags(&h->ev_used[i][j], hipEventDisableTiming));
        }
    }
    build_cg_levels(h.get(), stream);
    // outer solver workspace
    const size_t nd = h->ndof;
    h->r = (double*)h->mem.alloc(nd * sizeof(double));
    h->rold = (double*)h->mem.alloc(nd * sizeof(double));
    h->z = (double*)h->mem.alloc(nd * sizeof(double));
    h->pv = (double*)h->mem.alloc(nd * sizeof(double));
    h->q = (double*)h->mem.alloc(nd * sizeof(double));
    h->r32 = (float*)h->mem.alloc(nd * sizeof(float));
    h->z32 = (float*)h->mem.alloc(nd * sizeof(float));
    h->partial = (double*)h->mem.alloc(2 * hpmg::KRYLOV_RED_BLOCKS * sizeof(double));
    h->kpartial = (double*)h->mem.alloc((size_t)h->ncell * sizeof(double));
    h->scal = (double*)h->mem.alloc(16 * sizeof(double));
    HIPCHK(hipHostMalloc((void**)&h->host_scal, 16 * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipStreamSynchronize(stream));
    *out = h.release();
    return HPMG_OK;
  } catch (const HpmgError& e) {
    return fail(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HPMG_E_NOMEM;
  }
}

}  // namespace

hpmg_status hpmg_setup(const hpmg_mesh* mesh, int p, const hpmg_coeff* coeff, const hpmg_options* opt,
                       hipStream_t stream, hpmg_handle* out) {
  if (out) *out = nullptr;
  if (mesh == nullptr) {
    g_last_error = "mesh is NULL";
    return HPMG_E_INVALID;
  }
  if (mesh->n[1] != mesh->n[0] || (mesh->dim == 3 && mesh->n[2] != mesh->n[0])) {
    g_last_error = "only n x n (x n) meshes are supported";
    return HPMG_E_INVALID;
  }
  return setup_impl(mesh->dim, mesh->n[0], nullptr, p, coeff, opt, stream, out);
}

hpmg_status hpmg_setup_adaptive(const hpmg_adaptive_mesh* mesh, int p, const hpmg_coeff* coeff,
                                const hpmg_options* opt, hipStream_t stream, hpmg_handle* out) {
  if (out) *out = nullptr;
  if (mesh == nullptr || mesh->leaves == nullptr || mesh->nleaf < 1) {
    g_last_error = "mesh is NULL or has no leaves";
    return HPMG_E_INVALID;
  }
  return setup_impl(mesh->dim, mesh->n, mesh, p, coeff, opt, stream, out);
}

size_t hpmg_ndof(hpmg_handle h) { return h ? h->ndof : 0; }

void hpmg_destroy(hpmg_handle h) { delete h; }

hpmg_status hpmg_load_vector(hpmg_handle h, int kind, const double* params, double* b, hipStream_t stream) {
  try {
    require(h && b, "NULL argument");
    require(kind >= 0 && kind <= 2, "kind must be 0, 1 or 2");
    require(kind == 2 || params != nullptr, "params is NULL");
    require(kind != 2 || h->dim == 2, "kind 2 (two-peak) is two-dimensional");
    const int D = h->dim, n = h->n, N = h->p + 1;
    const double hh = 1.0 / n;
    hpmg::Basis1D B = hpmg::make_basis(h->p, h->opt.basis == 1);
    std::vector<double> xq, wq;
    hpmg::gauss_legendre(h->p + 3, xq, wq);
    std::vector<double> V = hpmg::interp_matrix(xq, B.xi);
    const int nq = (int)xq.size();
    // f = -Laplace u2, u2 = P G, P = x(1-x)y(1-y), G = 2 e1 - e2,
    // e = exp(-|x - x0|^2 / (2 s^2)):  Laplace u2 = G Laplace P
    // + 2 grad P . grad G + P Laplace G, grad e = -(x - x0) e / s^2,
    // Laplace e = (|x - x0|^2 / s^4 - 2 / s^2) e
    auto f2 = [](double x, double y) {
      const double cx[2] = {0.3, 0.8}, cy[2] = {0.4, 0.6}, sg[2] = {0.2, 0.1}, wt[2] = {2.0, -1.0};
      double G = 0.0, Gx = 0.0, Gy = 0.0, LG = 0.0;
      for (int i = 0; i < 2; ++i) {
        const double dx = x - cx[i], dy = y - cy[i], s2 = sg[i] * sg[i];
        const double r2 = dx * dx + dy * dy;
        const double e = std::exp(-r2 / (2.0 * s2));
        G += wt[i] * e;
        Gx += wt[i] * (-dx / s2) * e;
        Gy += wt[i] * (-dy / s2) * e;
        LG += wt[i] * (r2 / (s2 * s2) - 2.0 / s2) * e;
      }
      const double px = x * (1.0 - x), py = y * (1.0 - y);
      const double P = px * py, Px = (1.0 - 2.0 * x) * py, Py = px * (1.0 - 2.0 * y);
      const double LP = -2.0 * (py + px);
      return -(G * LP + 2.0 * (Px * Gx + Py * Gy) + P * LG);
    };
    if (h->adapt) {
      // per leaf: width hK, lower corner o; separable kinds per axis
      // G_k[a] = hK int g(o_k + hK xi) l_a(xi), the two-peak load by the
      // tensor rule on the leaf
      std::vector<double> out(h->ndof);
      const int nd = ipow(N, D);
      const double kf = kind == 1 ? params[0] : 0.0;
      const double coef = kind == 0 ? params[0] : D * kf * kf * M_PI * M_PI;
      std::vector<double> G((size_t)D * N);
      for (int c = 0; c < h->ncell; ++c) {
        const double hK = h->leaf_h[c];
        const double* o = &h->leaf_org[(size_t)c * D];
        if (kind == 2) {
          for (int i = 0; i < nd; ++i) {
            const int a = i % N, bb = i / N;
            double v = 0.0;
            for (int qy = 0; qy < nq; ++qy)
              for (int qx = 0; qx < nq; ++qx)
                v += wq[qx] * wq[qy] * f2(o[0] + hK * xq[qx], o[1] + hK * xq[qy]) * V[(size_t)qx * N + a] *
                     V[(size_t)qy * N + bb];
            out[(size_t)c * nd + i] = v * hK * hK;
          }
          continue;
        }
        for (int k = 0; k < D; ++k)
          for (int a = 0; a < N; ++a) {
            double sum = 0.0;
            for (int q = 0; q < nq; ++q) {
              const double g = kind == 0 ? 1.0 : std::sin(kf * M_PI * (o[k] + hK * xq[q]));
              sum += wq[q] * g * V[(size_t)q * N + a];
            }
            G[(size_t)k * N + a] = sum * hK;
          }
        for (int i = 0; i < nd; ++i) {
          double v = coef;
          for (int k = 0, ii = i; k < D; ++k, ii /= N) v *= G[(size_t)k * N + ii % N];
          out[(size_t)c * nd + i] = v;
        }
      }
      HIPCHK(hipMemcpyAsync(b, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice, stream));
      HIPCHK(hipStreamSynchronize(stream));
      return HPMG_OK;
    }
    if (kind == 2) {
      std::vector<double> out(h->ndof);
      const int nd2 = N * N;
      for (int c = 0; c < h->ncell; ++c) {
        const int cx = c % n, cy = c / n;
        for (int i = 0; i < nd2; ++i) {
          const int a = i % N, bb = i / N;
          double v = 0.0;
          for (int qy = 0; qy < nq; ++qy)
            for (int qx = 0; qx < nq; ++qx)
              v += wq[qx] * wq[qy] * f2((cx + xq[qx]) * hh, (cy + xq[qy]) * hh) * V[(size_t)qx * N + a] *
                   V[(size_t)qy * N + bb];
          out[(size_t)c * nd2 + i] = v * hh * hh;
        }
      }
      HIPCHK(hipMemcpyAsync(b, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice, stream));
      HIPCHK(hipStreamSynchronize(stream));
      return HPMG_OK;
    }
    // separable f: f = coef * prod_k g(x_k); per axis and cell coordinate,
    // G[x][a] = h int g l_a over the cell
    double coef;
    std::vector<double> G((size_t)n * N, 0.0);
    const double kf = kind == 1 ? params[0] : 0.0;
    coef = kind == 0 ? params[0] : D * kf * kf * M_PI * M_PI;
    for (int x = 0; x < n; ++x)
      for (int a = 0; a < N; ++a) {
        double s = 0.0;
        for (int q = 0; q < nq; ++q) {
          const double g = kind == 0 ? 1.0 : std::sin(kf * M_PI * (x + xq[q]) * hh);
          s += wq[q] * g * V[(size_t)q * N + a];
        }
        G[(size_t)x * N + a] = s * hh;
      }
    std::vector<double> out(h->ndof);
    const int nd = ipow(N, D);
    for (int c = 0; c < h->ncell; ++c) {
      const int cx = c % n, cy = (c / n) % n, cz = D == 3 ? c / (n * n) : 0;
      for (int i = 0; i < nd; ++i) {
        const int a = i % N, bb = (i / N) % N, cc = i / (N * N);
        double v = coef * G[(size_t)cx * N + a] * G[(size_t)cy * N + bb];
        if (D == 3) v *= G[(size_t)cz * N + cc];
        out[(size_t)c * nd + i] = v;
      }
    }
    HIPCHK(hipMemcpyAsync(b, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
    return HPMG_OK;
  } catch (const HpmgError& e) {
    return fail(e);
  }
}

hpmg_status hpmg_apply_A(hpmg_handle h, hpmg_dtype dtype, const void* u, void* y, int nrhs, hipStream_t stream) {
  try {
    require(h && u && y, "NULL argument");
    require(nrhs >= 1 && nrhs <= h->opt.max_rhs, "nrhs out of range");
    require(dtype == HPMG_F64 || dtype == HPMG_F32, "bad dtype");
    require(u != y, "u and y must not overlap");
    h->trace_state[dtype] = -1;
    if (dtype == HPMG_F64) {
      project<double>(h, 0, (const double*)u, h->dg[0].d.tr[0], nrhs, stream);
      apply<double>(h, 0, (const double*)u, h->dg[0].d.tr[0], nullptr, (double*)y, nrhs, stream);
    } else {
      project<float>(h, 0, (const float*)u, h->dg[0].f.tr[0], nrhs, stream);
      apply<float>(h, 0, (const float*)u, h->dg[0].f.tr[0], nullptr, (float*)y, nrhs, stream);
    }
    return HPMG_OK;
  } catch (const HpmgError& e) {
    return fail(e);
  }
}

hpmg_status hpmg_smooth(hpmg_handle h, hpmg_dtype dtype, void* u, const void* b, int nsweeps, int nrhs,
                        hipStream_t stream) {
  try {
    require(h && u && b, "NULL argument");
    require(nrhs >= 1 && nrhs <= h->opt.max_rhs, "nrhs out of range");
    require(nsweeps >= 0, "nsweeps must be >= 0");
    require(dtype >= HPMG_F64 && dtype <= HPMG_BF16, "bad dtype");
    if (nsweeps == 0) return HPMG_OK;
    h->trace_state[dtype] = -1;
    by_dtype(h, dtype, [&](auto tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      DGData<T>& d = data<T>(h->dg[0]);
      project<T>(h, 0, (const T*)u, d.tr[0], nrhs, stream);
      for (int k = 0; k < nsweeps; ++k) {
        if (h->opt.block_recompute == 2)
          sweep_split<T>(h, (T*)u, (const T*)b, d.tr[k & 1], d.tr[(k + 1) & 1], nrhs, stream);
        else
          sweep<T>(h, 0, (T*)u, (const T*)b, d.tr[k & 1], d.tr[(k + 1) & 1], false, nrhs, stream);
      }
      if (h->opt.block_recompute == 2) split_join<T>(h, stream);
    });
    h->trace_state[dtype] = nsweeps & 1;
    h->trace_rhs[dtype] = nrhs;
    return HPMG_OK;
  } catch (const HpmgError& e) {
    return fail(e);
  }
}

hpmg_status hpmg_project(hpmg_handle h, hpmg_dtype dtype, const void* u, int nrhs, hipStream_t stream) {
  try {
    require(h && u, "NULL argument");
    require(nrhs >= 1 && nrhs <= h->opt.max_rhs, "nrhs out of range");
    require(dtype >= HPMG_F64 && dtype <= HPMG_BF16, "bad dtype");
    h->trace_state[dtype] = -1;
    by_dtype(h, dtype, [&](auto tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      project<T>(h, 0, (const T*)u, data<T>(h->dg[0]).tr[0], nrhs, stream);
    });
    h->trace_state[dtype] = 0;
    h->trace_rhs[dtype] = nrhs;
    return HPMG_OK;
  } catch (const HpmgError& e) {
    return fail(e);
  }
}

hpmg_status hpmg_sweep(hpmg_handle h, hpmg_dtype dtype, void* u, const void* b, int nsweeps, int nrhs,
                       hipStream_t stream) {
  try {
    require(h && u && b, "NULL argument");
    require(dtype >= HPMG_F64 && dtype <= HPMG_BF16, "bad dtype");
    require(nsweeps >= 0, "nsweeps must be >= 0");
    require(h->trace_state[dtype] >= 0, "no current traces: call hpmg_project first");
    require(nrhs == h->trace_rhs[dtype], "nrhs differs from the call that produced the traces");
    int cur = h->trace_state[dtype];
    by_dtype(h, dtype, [&](auto tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      DGData<T>& d = data<T>(h->dg[0]);
      for (int k = 0; k < nsweeps; ++k) {
        if (h->opt.block_recompute == 2)
          sweep_split<T>(h, (T*)u, (const T*)b, d.tr[cur], d.tr[cur ^ 1], nrhs, stream);
        else
          sweep<T>(h, 0, (T*)u, (const T*)b, d.tr[cur], d.tr[cur ^ 1], false, nrhs, stream);
        cur ^= 1;
      }
      if (h->opt.block_recompute == 2) split_join<T>(h, stream);
    });
    h->trace_state[dtype] = cur;
    return HPMG_OK;
  } catch (const HpmgError& e) {
    return fail(e);
  }
}

hpmg_status hpmg_vcycle(hpmg_handle h, hpmg_dtype dtype, void* u, const void* b, int nrhs, hipStream_t stream) {
  try {
    require(h && u && b, "NULL argument");
    require(nrhs >= 1 && nrhs <= h->opt.max_rhs, "nrhs out of range");
    require(dtype >= HPMG_F64 && dtype <= HPMG_BF16, "bad dtype");
    h->trace_state[dtype] = -1;
    by_dtype(h, dtype, [&](auto tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      vcycle_dg<T>(h, 0, (T*)u, (const T*)b, false, nrhs, stream);
    });
    return HPMG_OK;
  } catch (const HpmgError& e) {
    return fail(e);
  }
}

hpmg_status hpmg_solve(hpmg_handle h, double* u, const double* b, int nrhs, double rtol, int maxit,
                       hpmg_solve_info* info, hipStream_t stream) {
  try {
    require(h && u && b, "NULL argument");
    require(nrhs >= 1, "nrhs must be >= 1");
    require(rtol > 0.0 && maxit >= 1, "bad rtol/maxit");
    const auto t0 = std::chrono::steady_clock::now();
    h->trace_state[0] = h->trace_state[1] = h->trace_state[2] = h->trace_state[3] = -1;
    const size_t nd = h->ndof;
    hpmg_status result = HPMG_OK;
    bool stagnated = false;
    const double rms = lowp_setup(h);
    // the iteration runs as a captured graph on an internal stream, on an
    // internal copy of u (so that one capture serves every call)
    if (!h->gs) HIPCHK(hipStreamCreateWithFlags(&h->gs, hipStreamNonBlocking));
    if (!h->ug) h->ug = (double*)h->mem.alloc(nd * sizeof(double));
    hipStream_t gs = h->gs;
    if (h->graph_prec != h->opt.precision) {
      for (int i = 0; i < 2; ++i) {
        if (h->gexec[i]) (void)hipGraphExecDestroy(h->gexec[i]);
        if (h->graph[i]) (void)hipGraphDestroy(h->graph[i]);
        h->gexec[i] = nullptr;
        h->graph[i] = nullptr;
      }
      for (int i = 0; i < 2; ++i) {
        HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        fcg_iteration(h, rms, i, gs);
        HIPCHK(hipStreamEndCapture(gs, &h->graph[i]));
        HIPCHK(hipGraphInstantiate(&h->gexec[i], h->graph[i], nullptr, nullptr, 0));
      }
      h->graph_prec = h->opt.precision;
    }
    HIPCHK(hipStreamSynchronize(stream));  // the caller's writes of u, b are done
    int its_total = 0;
    double r0_first = 0.0, rfin = 0.0;
    std::vector<double> hist;
    for (int rhs = 0; rhs < nrhs; ++rhs) {
      double* ur = u + (size_t)rhs * nd;
      const double* br = b + (size_t)rhs * nd;
      HIPCHK(hipMemcpyAsync(h->ug, ur, nd * sizeof(double), hipMemcpyDeviceToDevice, gs));
      const double r0 = fp64_residual(h, h->ug, br, gs);  // r = b - A u
      if (rhs == 0) r0_first = r0;
      double rn = r0;
      int it = 0;
      bool conv = r0 == 0.0;
      int restart = 1;
      int restarts = 0;
      while (!conv && it < maxit) {
        HIPCHK(hipGraphLaunch(h->gexec[restart], gs));
        HIPCHK(hipStreamSynchronize(gs));
        restart = 0;
        ++it;
        rn = std::sqrt(h->host_scal[6]);
        if (!std::isfinite(rn)) throw HpmgError(HPMG_E_BREAKDOWN, "non-finite residual");
        if (rhs == 0) hist.push_back(rn / r0);
        conv = rn <= rtol * r0;
        if (conv) {
          // the recurrence residual drifts from b - A u in finite precision:
          // accept only if the true residual meets the tolerance, else
          // restart the iteration from it
          rn = fp64_residual(h, h->ug, br, gs);
          conv = rn <= rtol * r0;
          restart = conv ? 0 : 1;
          // a true residual that stays above rtol after kMaxRestarts
          // restarts has reached the FP64 rounding floor of b - A u
          if (!conv && ++restarts > kMaxRestarts) {
            stagnated = true;
            break;
          }
        }
      }
      HIPCHK(hipMemcpyAsync(ur, h->ug, nd * sizeof(double), hipMemcpyDeviceToDevice, gs));
      HIPCHK(hipStreamSynchronize(gs));
      its_total = std::max(its_total, it);
      rfin = std::max(rfin, rn);
      if (!conv) result = HPMG_E_NOT_CONVERGED;
    }
    if (info) {
      info->iterations = its_total;
      info->initial_residual = r0_first;
      info->final_residual = rfin;
      for (int i = 0; i < 256; ++i) info->residual_history[i] = i < (int)hist.size() ? hist[i] : 0.0;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (result != HPMG_OK)
      g_last_error = stagnated ? "true residual stagnates above rtol (FP64 rounding floor of b - A u)"
                               : "maximum number of iterations reached";
    return result;
  } catch (const HpmgError& e) {
    return fail(e);
  }
}

hpmg_status hpmg_mgmult(hpmg_handle h, double* u, const double* b, double rtol, int maxit, int exit_kind,
                        hpmg_solve_info* info, hipStream_t stream) {
  try {
    require(h && u && b, "NULL argument");
    require(rtol > 0.0 && maxit >= 1, "bad rtol/maxit");
    require(exit_kind == 0 || exit_kind == 1, "exit_kind must be 0 or 1");
    const auto t0 = std::chrono::steady_clock::now();
    h->trace_state[0] = h->trace_state[1] = h->trace_state[2] = h->trace_state[3] = -1;
    const double rms = lowp_setup(h);
    // u_k = u_{k-1} + M (b - A u_{k-1}) equals the in-place cycle V(u_{k-1}, b)
    // for the linear V-cycle; z = M r is the preconditioned residual
    double rn = fp64_residual(h, u, b, stream);
    const double r0 = rn;
    double p1 = 0.0;
    std::vector<double> hist;
    int it = 0;
    bool conv = r0 == 0.0;
    while (!conv && it < maxit) {
      precondition(h, rms, stream);
      hpmg::krylov_dot(h->ndof, h->z, h->z, nullptr, h->partial, h->scal, 0, 10, 0, stream);
      hpmg::axpy(h->ndof, 1.0, h->z, u, stream);
      rn = fp64_residual(h, u, b, stream);  // synchronises; scal[10] = ||z||^2
      const double pz = std::sqrt(h->host_scal[10]);
      ++it;
      if (it == 1) p1 = pz;
      const double rel = exit_kind == 0 ? rn / r0 : (p1 > 0.0 ? pz / p1 : 0.0);
      hist.push_back(rel);
      conv = rel <= rtol;
    }
    if (info) {
      info->iterations = it;
      info->initial_residual = r0;
      info->final_residual = rn;
      for (int i = 0; i < 256; ++i) info->residual_history[i] = i < (int)hist.size() ? hist[i] : 0.0;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!conv) {
      g_last_error = "maximum number of cycles reached";
      return HPMG_E_NOT_CONVERGED;
    }
    return HPMG_OK;
  } catch (const HpmgError& e) {
    return fail(e);
  }
}

}  // extern "C"


