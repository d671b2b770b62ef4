// Host-side 1D reference data (see basis.hpp).
//
// Gauss-Lobatto nodes: interior nodes are the roots of P_p', found by Newton
// (Gauss-Legendre nodes: the roots of P_{p+1}, by the same recurrence)
// iteration in long double from Chebyshev-Lobatto guesses, using the
// Legendre recurrence and the Legendre differential equation for P_p''.
// Lagrange values use the barycentric formula, the nodal differentiation
// matrix its standard closed form (Berrut & Trefethen, SIAM Rev. 46, 2004).
// The stiffness matrix is Dn^T M Dn, exact because l_j' lies in the span of
// the degree-p basis.
#include "basis.hpp"

#include <cmath>
#include <cstring>

namespace hpmg {

namespace {

// P_n(x) and P_{n-1}(x) by the three-term recurrence.
void legendre_pair(int n, long double x, long double& pn, long double& pn1) {
  long double a = 1.0L, b = x;  // P_0, P_1
  if (n == 0) { pn = 1.0L; pn1 = 0.0L; return; }
  for (int k = 2; k <= n; ++k) {
    long double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
    a = b;
    b = c;
  }
  pn = b;
  pn1 = a;
}

}  // namespace

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double t = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double pn, pn1;
      legendre_pair(n, t, pn, pn1);
      dp = n * (t * pn - pn1) / (t * t - 1.0L);
      long double dt = pn / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-19L) break;
    }
    long double pn, pn1;
    legendre_pair(n, t, pn, pn1);
    dp = n * (t * pn - pn1) / (t * t - 1.0L);
    // map [-1,1] -> [0,1]; nodes come out descending in t
    x[n - 1 - i] = (double)(0.5L * (1.0L + t));
    w[n - 1 - i] = (double)(1.0L / ((1.0L - t * t) * dp * dp));
  }
}

std::vector<double> interp_matrix(const std::vector<double>& xf, const std::vector<double>& xc) {
  const int nf = (int)xf.size(), nc = (int)xc.size();
  std::vector<long double> bw(nc, 1.0L);
  for (int j = 0; j < nc; ++j)
    for (int k = 0; k < nc; ++k)
      if (k != j) bw[j] /= ((long double)xc[j] - xc[k]);
  std::vector<double> E((size_t)nf * nc, 0.0);
  for (int a = 0; a < nf; ++a) {
    int hit = -1;
    for (int j = 0; j < nc; ++j)
      if (xf[a] == xc[j]) hit = j;
    if (hit >= 0) {
      E[(size_t)a * nc + hit] = 1.0;
      continue;
    }
    long double den = 0.0L;
    for (int j = 0; j < nc; ++j) den += bw[j] / ((long double)xf[a] - xc[j]);
    for (int j = 0; j < nc; ++j)
      E[(size_t)a * nc + j] = (double)(bw[j] / ((long double)xf[a] - xc[j]) / den);
  }
  return E;
}

Basis1D make_basis(int p, bool gl) {
  Basis1D B;
  B.p = p;
  B.gl = gl;
  const int N = p + 1;
  B.N = N;
  if (gl) {
    std::vector<double> w;
    gauss_legendre(N, B.xi, w);
  }
  // Gauss-Lobatto nodes on [-1,1]
  std::vector<long double> t(N);
  const long double pi = 3.141592653589793238462643383279502884L;
  t[0] = -1.0L;
  t[p] = 1.0L;
  for (int j = 1; j < p; ++j) {
    long double x = -std::cos(pi * j / p);
    for (int it = 0; it < 100; ++it) {
      long double pn, pn1;
      legendre_pair(p, x, pn, pn1);
      long double d1 = p * (pn1 - x * pn) / (1.0L - x * x);               // P_p'
      long double d2 = (2.0L * x * d1 - p * (p + 1.0L) * pn) / (1.0L - x * x);  // P_p''
      long double dx = d1 / d2;
      x -= dx;
      if (std::fabs(dx) < 1e-19L) break;
    }
    t[j] = x;
  }
  if (!gl) {
    B.xi.resize(N);
    for (int j = 0; j < N; ++j) B.xi[j] = (double)(0.5L * (t[j] + 1.0L));
    B.xi[0] = 0.0;
    B.xi[p] = 1.0;
  }
  // barycentric weights and differentiation matrix at the nodes
  std::vector<long double> bw(N, 1.0L);
  for (int j = 0; j < N; ++j)
    for (int k = 0; k < N; ++k)
      if (k != j) bw[j] /= ((long double)B.xi[j] - B.xi[k]);
  B.Dn.assign((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i) {
    long double diag = 0.0L;
    for (int j = 0; j < N; ++j) {
      if (j == i) continue;
      long double v = (bw[j] / bw[i]) / ((long double)B.xi[i] - B.xi[j]);
      B.Dn[(size_t)i * N + j] = (double)v;
      diag -= v;
    }
    B.Dn[(size_t)i * N + i] = (double)diag;
  }
  // mass by (p+1)-point Gauss: exact for degree 2p
  std::vector<double> xq, wq;
  gauss_legendre(N, xq, wq);
  std::vector<double> V = interp_matrix(xq, B.xi);  // V[q*N+j] = l_j(xq)
  B.M.assign((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      long double s = 0.0L;
      for (int q = 0; q < N; ++q) s += (long double)wq[q] * V[q * N + i] * V[q * N + j];
      B.M[(size_t)i * N + j] = (double)s;
    }
  // stiffness K = Dn^T M Dn
  B.K.assign((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      long double s = 0.0L;
      for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b)
          s += (long double)B.Dn[a * N + i] * B.M[a * N + b] * B.Dn[b * N + j];
      B.K[(size_t)i * N + j] = (double)s;
    }
  // values at the end points, and the derivatives there: l_j' has degree
  // p-1, so l_j'(x) = sum_a l_a(x) l_j'(xi_a)
  B.e0 = interp_matrix({0.0}, B.xi);
  B.e1 = interp_matrix({1.0}, B.xi);
  B.ep0.assign(N, 0.0);
  B.ep1.assign(N, 0.0);
  for (int j = 0; j < N; ++j) {
    long double d0 = 0.0L, d1 = 0.0L;
    for (int a = 0; a < N; ++a) {
      d0 += (long double)B.e0[a] * B.Dn[(size_t)a * N + j];
      d1 += (long double)B.e1[a] * B.Dn[(size_t)a * N + j];
    }
    B.ep0[j] = (double)(-d0);
    B.ep1[j] = (double)d1;
  }
  return B;
}

bool gen_sym_eig(const double* L, const double* M, int N, double* S, double* lam) {
  // Cholesky M = C C^T (lower C)
  std::vector<long double> C((size_t)N * N, 0.0L);
  for (int j = 0; j < N; ++j) {
    long double s = M[j * N + j];
    for (int k = 0; k < j; ++k) s -= C[j * N + k] * C[j * N + k];
    if (!(s > 0.0L)) return false;
    C[j * N + j] = std::sqrt(s);
    for (int i = j + 1; i < N; ++i) {
      long double t = M[i * N + j];
      for (int k = 0; k < j; ++k) t -= C[i * N + k] * C[j * N + k];
      C[i * N + j] = t / C[j * N + j];
    }
  }
  // Ci = C^-1 (lower triangular)
  std::vector<long double> Ci((size_t)N * N, 0.0L);
  for (int j = 0; j < N; ++j) {
    Ci[j * N + j] = 1.0L / C[j * N + j];
    for (int i = j + 1; i < N; ++i) {
      long double s = 0.0L;
      for (int k = j; k < i; ++k) s += C[i * N + k] * Ci[k * N + j];
      Ci[i * N + j] = -s / C[i * N + i];
    }
  }
  // A = Ci L Ci^T
  std::vector<long double> T((size_t)N * N, 0.0L), A((size_t)N * N, 0.0L);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      long double s = 0.0L;
      for (int k = 0; k < N; ++k) s += Ci[i * N + k] * L[k * N + j];
      T[i * N + j] = s;
    }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      long double s = 0.0L;
      for (int k = 0; k < N; ++k) s += T[i * N + k] * Ci[j * N + k];
      A[i * N + j] = s;
    }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < i; ++j) {
      long double m = 0.5L * (A[i * N + j] + A[j * N + i]);
      A[i * N + j] = A[j * N + i] = m;
    }
  // cyclic Jacobi rotations: A = Q diag Q^T
  std::vector<long double> Q((size_t)N * N, 0.0L);
  for (int i = 0; i < N; ++i) Q[i * N + i] = 1.0L;
  for (int sweep = 0; sweep < 60; ++sweep) {
    long double off = 0.0L, tot = 0.0L;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        tot += A[i * N + j] * A[i * N + j];
        if (i != j) off += A[i * N + j] * A[i * N + j];
      }
    if (off <= 1e-36L * tot) break;
    for (int pI = 0; pI < N - 1; ++pI)
      for (int qI = pI + 1; qI < N; ++qI) {
        long double apq = A[pI * N + qI];
        if (apq == 0.0L) continue;
        long double app = A[pI * N + pI], aqq = A[qI * N + qI];
        long double theta = (aqq - app) / (2.0L * apq);
        long double tt = (theta >= 0 ? 1.0L : -1.0L) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0L));
        long double c = 1.0L / std::sqrt(tt * tt + 1.0L), s = tt * c;
        for (int k = 0; k < N; ++k) {  // columns p, q
          long double akp = A[k * N + pI], akq = A[k * N + qI];
          A[k * N + pI] = c * akp - s * akq;
          A[k * N + qI] = s * akp + c * akq;
        }
        for (int k = 0; k < N; ++k) {  // rows p, q
          long double apk = A[pI * N + k], aqk = A[qI * N + k];
          A[pI * N + k] = c * apk - s * aqk;
          A[qI * N + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < N; ++k) {
          long double qkp = Q[k * N + pI], qkq = Q[k * N + qI];
          Q[k * N + pI] = c * qkp - s * qkq;
          Q[k * N + qI] = s * qkp + c * qkq;
        }
      }
  }
  // S = C^-T Q, lam = diag(A)
  for (int i = 0; i < N; ++i) {
    lam[i] = (double)A[i * N + i];
    for (int j = 0; j < N; ++j) {
      long double s = 0.0L;
      for (int k = 0; k < N; ++k) s += Ci[k * N + i] * Q[k * N + j];
      S[i * N + j] = (double)s;
    }
  }
  return true;
}

}  // namespace hpmg
