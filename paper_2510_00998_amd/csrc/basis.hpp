// Host-side 1D reference data and small dense linear algebra used to set up
// the levels: Gauss-Lobatto nodes, Gauss quadrature, the nodal mass and
// stiffness matrices on [0,1], and the generalised symmetric eigenproblem
// behind the fast-diagonalised block inverse.
#pragma once
#include <vector>

namespace hpmg {

struct Basis1D {
  int p = 0, N = 0;
  std::vector<double> xi;   // nodes on [0,1], ascending
  std::vector<double> M;    // mass  M[i*N+j] = int_0^1 l_i l_j
  std::vector<double> K;    // stiffness K[i*N+j] = int_0^1 l_i' l_j'
  std::vector<double> Dn;   // nodal derivative Dn[a*N+j] = l_j'(xi_a)
  std::vector<double> ep0;  // outward normal derivative at x=0: -l_j'(0)
  std::vector<double> ep1;  // outward normal derivative at x=1: +l_j'(1)
  std::vector<double> e0;   // value at x=0: l_j(0) (unit vector for Gauss-Lobatto nodes)
  std::vector<double> e1;   // value at x=1: l_j(1)
  bool gl = false;          // nodes are the Gauss-Legendre points
};

// Lagrange basis of degree p (1 <= p <= 16) on the Gauss-Lobatto-Legendre
// nodes (gl = false) or on the p+1 Gauss-Legendre points (gl = true).
Basis1D make_basis(int p, bool gl = false);

// n-point Gauss-Legendre rule on [0,1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Lagrange interpolation matrix from nodes xc to points xf:
// E[a*nc + j] = l^c_j(xf[a]).
std::vector<double> interp_matrix(const std::vector<double>& xf, const std::vector<double>& xc);

// Generalised symmetric-definite eigenproblem L S = M S diag(lam) with
// S^T M S = I (Cholesky of M, cyclic Jacobi on C^-1 L C^-T).  N x N
// row-major.  Returns false if M is not positive definite.
bool gen_sym_eig(const double* L, const double* M, int N, double* S, double* lam);

}  // namespace hpmg
