// CPU oracle in plain C++ (TEST INFRASTRUCTURE ONLY): the SIPG operator of
// arXiv 2510.00998 (Section 2.3, eq. weak_form_IP with theta = -1) assembled
// explicitly as a sparse matrix on the uniform n^d mesh of the unit box, and
// the textbook solver components on it: block-Jacobi with the exact diagonal
// blocks (Section 2.3.2, eq. block-Jacobi-IP; dense Cholesky per block),
// point-Jacobi on the continuous Q1 levels (Section 2.4), Galerkin coarse
// operators P^T A P, the V-cycle of Algorithm CoarseGridCorrection /
// MGMult (Section 5) and flexible CG preconditioned by one V-cycle.
//
// The same definitions and readings as the NumPy oracle (oracle/sipg.py,
// oracle/mg.py): GLL nodes on [0,1], local node a + N b (+ N^2 c), cell
// cx + n cy (+ n^2 cz); harmonic kappa_F in flux and penalty, sigma =
// sigma0 (p+1)^2 / h on interior facets and 2 sigma on the boundary, the
// fine penalty on every p-coarse level; p halved while >= 2, then Q1 on the
// same mesh (interior vertices), Q1 h-coarsening by 2 keeping the last
// vertex for odd n, until n <= coarsest_n; dense Cholesky on the coarsest
// level.  All integrals by Gauss quadrature exact for the integrands.
//
// It shares no code with the HIP library (its own Legendre recurrences,
// quadrature, Lagrange products, sparse products).  Only tests/,
// __graft_entry__.smoke() and bench.py's CPU baseline load it, through
// oracle/coracle.py.  OpenMP parallelises the matrix-vector products and the
// block solves over rows and cells; nothing else.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <vector>

#include <omp.h>

namespace {

// ------------------------------------------------------------------ 1D
// Legendre P_n(x) and P_n'(x) by the three-term recurrence (|x| < 1).
void legendre(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

// m-point Gauss-Legendre rule mapped to [0,1] (Newton on P_m).
void gauss_rule(int m, std::vector<double>& x, std::vector<double>& w) {
  x.assign(m, 0.0);
  w.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (m + 0.5));
    double P, dP;
    for (int it = 0; it < 100; ++it) {
      legendre(m, t, P, dP);
      const double dt = P / dP;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    legendre(m, t, P, dP);
    x[m - 1 - i] = 0.5 * (t + 1.0);
    w[m - 1 - i] = 1.0 / ((1.0 - t * t) * dP * dP);  // 2/((1-t^2) P'^2), times 1/2 for [0,1]
  }
}

// Gauss-Lobatto nodes on [0,1]: the endpoints and the roots of P_p'
// (Newton on P_p' with its derivative from Legendre's equation).
std::vector<double> gll_nodes(int p) {
  std::vector<double> x(p + 1);
  x[0] = 0.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double t = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, t, P, dP);
      // (1 - t^2) P'' = 2 t P' - p (p + 1) P
      const double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
      const double dt = dP / d2P;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = 0.5 * (t + 1.0);
  }
  std::sort(x.begin(), x.end());
  return x;
}

// Values and derivatives at y of the Lagrange polynomials through `nodes`.
void lagrange(const std::vector<double>& nodes, double y, double* v, double* dv) {
  const int m = (int)nodes.size();
  for (int j = 0; j < m; ++j) {
    double val = 1.0, der = 0.0;
    for (int l = 0; l < m; ++l) {
      if (l == j) continue;
      val *= (y - nodes[l]) / (nodes[j] - nodes[l]);
    }
    for (int l = 0; l < m; ++l) {
      if (l == j) continue;
      double t = 1.0 / (nodes[j] - nodes[l]);
      for (int q = 0; q < m; ++q) {
        if (q == j || q == l) continue;
        t *= (y - nodes[q]) / (nodes[j] - nodes[q]);
      }
      der += t;
    }
    v[j] = val;
    dv[j] = der;
  }
}

// Dense row-major matrices (small).
struct Mat {
  int r = 0, c = 0;
  std::vector<double> a;
  Mat() = default;
  Mat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, 0.0) {}
  double& operator()(int i, int j) { return a[(size_t)i * c + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};
Mat kron(const Mat& A, const Mat& B) {  // A (x) B
  Mat K(A.r * B.r, A.c * B.c);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j)
      for (int k = 0; k < B.r; ++k)
        for (int l = 0; l < B.c; ++l) K(i * B.r + k, j * B.c + l) = A(i, j) * B(k, l);
  return K;
}
// Tensor product with x fastest: mats = [Mx, My(, Mz)] -> Mz (x) My (x) Mx.
Mat kron_dims(const std::vector<Mat>& mats) {
  Mat out = mats[0];
  for (size_t i = 1; i < mats.size(); ++i) out = kron(mats[i], out);
  return out;
}
Mat matmul(const Mat& A, const Mat& B) {
  Mat C(A.r, B.c);
  for (int i = 0; i < A.r; ++i)
    for (int k = 0; k < A.c; ++k) {
      const double a = A(i, k);
      if (a == 0.0) continue;
      for (int j = 0; j < B.c; ++j) C(i, j) += a * B(k, j);
    }
  return C;
}
Mat transpose(const Mat& A) {
  Mat T(A.c, A.r);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
  return T;
}
Mat diag(const std::vector<double>& w) {
  Mat D((int)w.size(), (int)w.size());
  for (size_t i = 0; i < w.size(); ++i) D((int)i, (int)i) = w[i];
  return D;
}

// --------------------------------------------------------------- sparse
struct Csr {
  int nr = 0, nc = 0;
  std::vector<long long> ptr;
  std::vector<int> col;
  std::vector<double> val;
  void matvec(const double* x, double* y) const {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; ++i) {
      double s = 0.0;
      for (long long e = ptr[i]; e < ptr[i + 1]; ++e) s += val[e] * x[col[e]];
      y[i] = s;
    }
  }
};

// Rows of (row, col, value) triplets summed into CSR.
Csr from_rows(int nr, int nc, std::vector<std::map<int, double>>& rows) {
  Csr A;
  A.nr = nr;
  A.nc = nc;
  A.ptr.assign(nr + 1, 0);
  for (int i = 0; i < nr; ++i) A.ptr[i + 1] = A.ptr[i] + (long long)rows[i].size();
  A.col.resize(A.ptr[nr]);
  A.val.resize(A.ptr[nr]);
  for (int i = 0; i < nr; ++i) {
    long long e = A.ptr[i];
    for (auto& kv : rows[i]) {
      A.col[e] = kv.first;
      A.val[e] = kv.second;
      ++e;
    }
  }
  return A;
}
Csr transpose(const Csr& A) {
  std::vector<std::map<int, double>> rows(A.nc);
  for (int i = 0; i < A.nr; ++i)
    for (long long e = A.ptr[i]; e < A.ptr[i + 1]; ++e) rows[A.col[e]][i] += A.val[e];
  return from_rows(A.nc, A.nr, rows);
}
Csr spmm(const Csr& A, const Csr& B) {
  std::vector<std::map<int, double>> rows(A.nr);
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < A.nr; ++i)
    for (long long e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      const int k = A.col[e];
      for (long long f = B.ptr[k]; f < B.ptr[k + 1]; ++f) rows[i][B.col[f]] += A.val[e] * B.val[f];
    }
  return from_rows(A.nr, B.nc, rows);
}
Csr galerkin(const Csr& A, const Csr& P) { return spmm(transpose(P), spmm(A, P)); }

// Dense Cholesky in place (lower), solve L L^T x = b.
bool cholesky(std::vector<double>& a, int n) {
  for (int j = 0; j < n; ++j) {
    double s = a[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    a[(size_t)j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = a[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
      a[(size_t)i * n + j] = t / a[(size_t)j * n + j];
    }
  }
  return true;
}
void cholesky_solve(const double* L, int n, const double* b, double* x) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * x[k];
    x[i] = s / L[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
    x[i] = s / L[(size_t)i * n + i];
  }
}

// ------------------------------------------------------------------ SIPG
// Assembled operator of eq. weak_form_IP on the n^d mesh, degree p, penalty
// factor of degree p_pen, kappa per cell.
Csr assemble(int d, int n, int p, int p_pen, const std::vector<double>& kappa, double sigma0) {
  const int N = p + 1;
  const double h = 1.0 / n;
  std::vector<double> nodes = gll_nodes(p), xq, wq;
  gauss_rule(N, xq, wq);
  Mat V(N, N), D(N, N), e0(1, N), d0(1, N), e1(1, N), d1(1, N);
  for (int q = 0; q < N; ++q) lagrange(nodes, xq[q], &V.a[(size_t)q * N], &D.a[(size_t)q * N]);
  lagrange(nodes, 0.0, e0.a.data(), d0.a.data());
  lagrange(nodes, 1.0, e1.a.data(), d1.a.data());
  // volume: h^(d-2) sum_k int grad_k phi_i grad_k phi_j on the unit cell
  std::vector<Mat> Wl(d, diag(wq));
  const Mat W = kron_dims(Wl);
  const int nd = (int)std::pow(N, d);
  Mat Kv(nd, nd);
  for (int k = 0; k < d; ++k) {
    std::vector<Mat> g;
    for (int j = 0; j < d; ++j) g.push_back(j == k ? D : V);
    const Mat G = kron_dims(g);
    const Mat T = matmul(transpose(G), matmul(W, G));
    for (size_t i = 0; i < T.a.size(); ++i) Kv.a[i] += T.a[i];
  }
  for (double& v : Kv.a) v *= std::pow(h, d - 2);
  // facets normal to axis k: "minus" cell sees xi_k = 1, "plus" xi_k = 0;
  // n_F = +e_k, physical d/dx = (1/h) d/dxi
  std::vector<Mat> Wfl(d - 1, diag(wq));
  Mat Wf = kron_dims(Wfl);
  for (double& v : Wf.a) v *= std::pow(h, d - 1);
  const double sigma = sigma0 * (p_pen + 1.0) * (p_pen + 1.0) / h;
  Mat d0h = d0, d1h = d1;
  for (double& v : d0h.a) v /= h;
  for (double& v : d1h.a) v /= h;
  // B[k][Y][X] (Y, X: 0 minus, 1 plus) without kappa_F; Bb[k][side] without kappa_K
  std::vector<Mat> Bint(d * 4), Bbdy(d * 2);
  for (int k = 0; k < d; ++k) {
    Mat val[2], dn[2];
    for (int side = 0; side < 2; ++side) {
      std::vector<Mat> gv, gd;
      for (int j = 0; j < d; ++j) {
        gv.push_back(j == k ? (side == 0 ? e1 : e0) : V);
        gd.push_back(j == k ? (side == 0 ? d1h : d0h) : V);
      }
      val[side] = kron_dims(gv);
      dn[side] = kron_dims(gd);
    }
    const double sg[2] = {1.0, -1.0};
    for (int Y = 0; Y < 2; ++Y)
      for (int X = 0; X < 2; ++X) {
        const Mat a = matmul(transpose(val[Y]), matmul(Wf, dn[X]));
        const Mat b = matmul(transpose(dn[Y]), matmul(Wf, val[X]));
        const Mat c = matmul(transpose(val[Y]), matmul(Wf, val[X]));
        Mat B(nd, nd);
        for (size_t i = 0; i < B.a.size(); ++i)
          B.a[i] = -0.5 * sg[Y] * a.a[i] - 0.5 * sg[X] * b.a[i] + sigma * sg[X] * sg[Y] * c.a[i];
        Bint[k * 4 + Y * 2 + X] = B;
      }
    for (int side = 0; side < 2; ++side) {
      // side 1 (x_k = 1): outward normal +e_k, the "minus" traces; side 0:
      // outward -e_k, the "plus" traces with the derivative negated
      const Mat& Vb = side == 1 ? val[0] : val[1];
      Mat Db = side == 1 ? dn[0] : dn[1];
      if (side == 0)
        for (double& v : Db.a) v = -v;
      const Mat a = matmul(transpose(Vb), matmul(Wf, Db));
      const Mat b = matmul(transpose(Db), matmul(Wf, Vb));
      const Mat c = matmul(transpose(Vb), matmul(Wf, Vb));
      Mat B(nd, nd);
      for (size_t i = 0; i < B.a.size(); ++i) B.a[i] = -a.a[i] - b.a[i] + 2.0 * sigma * c.a[i];
      Bbdy[k * 2 + side] = B;
    }
  }
  const int ncell = (int)std::pow(n, d);
  std::vector<std::map<int, double>> rows((size_t)ncell * nd);
  auto add = [&](int I, int J, const Mat& B, double s) {
    for (int i = 0; i < nd; ++i)
      for (int j = 0; j < nd; ++j) {
        const double v = s * B(i, j);
        if (v != 0.0) rows[(size_t)I * nd + i][J * nd + j] += v;
      }
  };
  for (int c = 0; c < ncell; ++c) {
    int cc[3] = {c % n, (c / n) % n, d == 3 ? c / (n * n) : 0};
    add(c, c, Kv, kappa[c]);
    for (int k = 0; k < d; ++k) {
      const int st = k == 0 ? 1 : (k == 1 ? n : n * n);
      for (int side = 0; side < 2; ++side) {
        const bool bdy = cc[k] == (side == 0 ? 0 : n - 1);
        if (bdy) {
          add(c, c, Bbdy[k * 2 + side], kappa[c]);
          continue;
        }
        const int nb = c + (side == 1 ? st : -st);
        const double kf = 2.0 * kappa[c] * kappa[nb] / (kappa[c] + kappa[nb]);
        const int own = side == 1 ? 0 : 1, oth = 1 - own;
        add(c, c, Bint[k * 4 + own * 2 + own], kf);
        add(c, nb, Bint[k * 4 + own * 2 + oth], kf);
      }
    }
  }
  return from_rows(ncell * nd, ncell * nd, rows);
}

// Nodal interpolation Q_q -> Q_p on every cell (block diagonal).
Csr dg_prolongation(int d, int ncell, int p, int q) {
  const std::vector<double> fine = gll_nodes(p), coarse = gll_nodes(q);
  const int N = p + 1, Nc = q + 1;
  Mat E(N, Nc);
  std::vector<double> dv(Nc);
  for (int a = 0; a < N; ++a) lagrange(coarse, fine[a], &E.a[(size_t)a * Nc], dv.data());
  const Mat Pc = kron_dims(std::vector<Mat>(d, E));
  std::vector<std::map<int, double>> rows((size_t)ncell * Pc.r);
  for (int c = 0; c < ncell; ++c)
    for (int i = 0; i < Pc.r; ++i)
      for (int j = 0; j < Pc.c; ++j)
        if (Pc(i, j) != 0.0) rows[(size_t)c * Pc.r + i][c * Pc.c + j] = Pc(i, j);
  return from_rows(ncell * Pc.r, ncell * Pc.c, rows);
}

// Q1 interior vertices -> DG nodal values: the trilinear hat of vertex V at
// the nodes of the cells around it.
Csr cg_to_dg(int d, int n, int p) {
  const std::vector<double> xi = gll_nodes(p);
  const int N = p + 1, nd = (int)std::pow(N, d), ncell = (int)std::pow(n, d), nv = n - 1;
  std::vector<std::map<int, double>> rows((size_t)ncell * nd);
  for (int c = 0; c < ncell; ++c) {
    int cc[3] = {c % n, (c / n) % n, d == 3 ? c / (n * n) : 0};
    for (int corner = 0; corner < (1 << d); ++corner) {
      int vid = 0, mul = 1;
      bool inside = true;
      for (int k = 0; k < d; ++k) {
        const int v = cc[k] + ((corner >> k) & 1);
        inside = inside && v > 0 && v < n;
        vid += (v - 1) * mul;
        mul *= nv;
      }
      if (!inside) continue;
      for (int i = 0; i < nd; ++i) {
        double w = 1.0;
        for (int k = 0, ii = i; k < d; ++k, ii /= N) w *= ((corner >> k) & 1) ? xi[ii % N] : 1.0 - xi[ii % N];
        if (w != 0.0) rows[(size_t)c * nd + i][vid] += w;
      }
    }
  }
  return from_rows(ncell * nd, (int)std::pow(nv, d), rows);
}

// Coarse vertex positions (every second fine vertex, the last kept).
std::vector<int> coarse_positions(int n) {
  std::vector<int> pos;
  for (int i = 0; i <= n; i += 2) pos.push_back(i);
  if (pos.back() != n) pos.push_back(n);
  return pos;
}

// Q1 h-prolongation from the coarse vertex grid (interior vertices).
Csr cg_prolongation(int d, int n) {
  const std::vector<int> pos = coarse_positions(n);
  const int m = (int)pos.size() - 1, nv = n - 1, nvc = m - 1;
  // 1D weights: fine vertex i (0..n) from coarse vertices
  std::vector<std::vector<std::pair<int, double>>> w1(n + 1);
  for (int i = 0; i <= n; ++i) {
    const int J = (int)(std::lower_bound(pos.begin(), pos.end(), i) - pos.begin());
    if (pos[J] == i) {
      w1[i].push_back({J, 1.0});
    } else {
      const double t = (double)(i - pos[J - 1]) / (pos[J] - pos[J - 1]);
      w1[i].push_back({J - 1, 1.0 - t});
      w1[i].push_back({J, t});
    }
  }
  const int nf = (int)std::pow(nv, d);
  std::vector<std::map<int, double>> rows(nf);
  for (int v = 0; v < nf; ++v) {
    int idx[3] = {v % nv + 1, (v / nv) % nv + 1, d == 3 ? v / (nv * nv) + 1 : 0};
    // tensor of the 1D weights over interior coarse vertices (1..m-1)
    std::vector<std::pair<int, double>> acc = {{0, 1.0}};
    int mul = 1;
    for (int k = 0; k < d; ++k) {
      std::vector<std::pair<int, double>> nxt;
      for (auto& a : acc)
        for (auto& b : w1[idx[k]]) {
          if (b.first == 0 || b.first == m) continue;  // boundary coarse vertex
          nxt.push_back({a.first + (b.first - 1) * mul, a.second * b.second});
        }
      acc = nxt;
      mul *= nvc;
    }
    for (auto& a : acc) rows[v][a.first] += a.second;
  }
  return from_rows(nf, (int)std::pow(nvc, d), rows);
}

struct Level {
  bool dg = false;
  int nd = 1;
  Csr A;
  std::vector<double> Lfac;  // DG: per-cell Cholesky factors of the diagonal blocks
  std::vector<double> dinv;  // Q1: 1 / diag(A)
};

}  // namespace

struct oc_hierarchy {
  int dim = 0, n = 0, p = 0;
  double omega_dg = 0.7, omega_cg = 2.0 / 3.0;
  int nu_pre = 2, nu_post = 2;
  std::vector<Level> lev;
  std::vector<Csr> P;  // P[l]: level l+1 -> level l
  std::vector<double> coarse;  // Cholesky factor of the coarsest operator
  int coarse_n = 0;

  void smooth(int l, double* u, const double* b, int nsweeps) const {
    const Level& L = lev[l];
    const int m = L.A.nr;
    std::vector<double> r(m);
    for (int s = 0; s < nsweeps; ++s) {
      L.A.matvec(u, r.data());
#pragma omp parallel for schedule(static)
      for (int i = 0; i < m; ++i) r[i] = b[i] - r[i];
      if (L.dg) {
        const int nc = m / L.nd, nd = L.nd;
#pragma omp parallel for schedule(static)
        for (int c = 0; c < nc; ++c) {
          std::vector<double> x(nd);
          cholesky_solve(&L.Lfac[(size_t)c * nd * nd], nd, &r[(size_t)c * nd], x.data());
          for (int i = 0; i < nd; ++i) u[(size_t)c * nd + i] += omega_dg * x[i];
        }
      } else {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < m; ++i) u[i] += omega_cg * r[i] * L.dinv[i];
      }
    }
  }

  void vcycle(int l, double* u, const double* b) const {
    if (l + 1 == (int)lev.size()) {
      cholesky_solve(coarse.data(), coarse_n, b, u);
      return;
    }
    const int m = lev[l].A.nr;
    smooth(l, u, b, nu_pre);
    std::vector<double> r(m);
    lev[l].A.matvec(u, r.data());
    for (int i = 0; i < m; ++i) r[i] = b[i] - r[i];
    const Csr& Pl = P[l];
    std::vector<double> bc(Pl.nc, 0.0), ec(Pl.nc, 0.0), e(m);
    for (int i = 0; i < Pl.nr; ++i)
      for (long long k = Pl.ptr[i]; k < Pl.ptr[i + 1]; ++k) bc[Pl.col[k]] += Pl.val[k] * r[i];
    vcycle(l + 1, ec.data(), bc.data());
    Pl.matvec(ec.data(), e.data());
    for (int i = 0; i < m; ++i) u[i] += e[i];
    smooth(l, u, b, nu_post);
  }
};

extern "C" {

// Build the hierarchy (kappa: n^d values, or NULL for the constant kc).
// Returns NULL if a diagonal block or the coarsest operator is not
// positive definite.
oc_hierarchy* oc_create(int dim, int n, int p, const double* kappa, double kc, double sigma0, double omega_dg,
                        double omega_cg, int nu_pre, int nu_post, int coarsest_n) {
  auto H = std::make_unique<oc_hierarchy>();
  H->dim = dim;
  H->n = n;
  H->p = p;
  H->omega_dg = omega_dg;
  H->omega_cg = omega_cg;
  H->nu_pre = nu_pre;
  H->nu_post = nu_post;
  const int ncell = (int)std::pow(n, dim);
  std::vector<double> kap(ncell, kc);
  if (kappa) kap.assign(kappa, kappa + ncell);
  std::vector<int> degs = {p};
  for (int q = p / 2; q >= 2; q /= 2) degs.push_back(q);
  Csr A = assemble(dim, n, p, p, kap, sigma0);
  // DG levels: exact diagonal blocks factored by Cholesky
  for (size_t li = 0; li < degs.size(); ++li) {
    const int q = degs[li], nd = (int)std::pow(q + 1, dim);
    Level L;
    L.dg = true;
    L.nd = nd;
    L.A = A;
    L.Lfac.assign((size_t)ncell * nd * nd, 0.0);
    bool ok = true;
#pragma omp parallel for schedule(static) reduction(&& : ok)
    for (int c = 0; c < ncell; ++c) {
      std::vector<double> B((size_t)nd * nd, 0.0);
      for (int i = 0; i < nd; ++i) {
        const int row = c * nd + i;
        for (long long e = A.ptr[row]; e < A.ptr[row + 1]; ++e) {
          const int j = A.col[e] - c * nd;
          if (j >= 0 && j < nd) B[(size_t)i * nd + j] = A.val[e];
        }
      }
      ok = cholesky(B, nd) && ok;
      std::copy(B.begin(), B.end(), L.Lfac.begin() + (size_t)c * nd * nd);
    }
    if (!ok) return nullptr;
    H->lev.push_back(std::move(L));
    Csr Pl = li + 1 < degs.size() ? dg_prolongation(dim, ncell, q, degs[li + 1]) : cg_to_dg(dim, n, q);
    A = galerkin(A, Pl);
    H->P.push_back(std::move(Pl));
  }
  // Q1 levels: point-Jacobi, h-coarsening by 2 while n > coarsest_n
  int m = n;
  while (true) {
    Level L;
    L.A = A;
    L.dinv.resize(A.nr);
    for (int i = 0; i < A.nr; ++i)
      for (long long e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
        if (A.col[e] == i) L.dinv[i] = 1.0 / A.val[e];
    H->lev.push_back(std::move(L));
    if (m <= coarsest_n) break;
    Csr Pl = cg_prolongation(dim, m);
    A = galerkin(A, Pl);
    H->P.push_back(std::move(Pl));
    m = (int)coarse_positions(m).size() - 1;
  }
  const Csr& C = H->lev.back().A;
  H->coarse_n = C.nr;
  H->coarse.assign((size_t)C.nr * C.nr, 0.0);
  for (int i = 0; i < C.nr; ++i)
    for (long long e = C.ptr[i]; e < C.ptr[i + 1]; ++e) H->coarse[(size_t)i * C.nr + C.col[e]] = C.val[e];
  if (!cholesky(H->coarse, C.nr)) return nullptr;
  return H.release();
}

void oc_destroy(oc_hierarchy* h) { delete h; }

long long oc_ndof(const oc_hierarchy* h) { return h->lev[0].A.nr; }

// Fine operator in CSR: nnz, then the arrays (ptr: ndof + 1 entries).
long long oc_nnz(const oc_hierarchy* h) { return h->lev[0].A.ptr.back(); }
void oc_csr(const oc_hierarchy* h, long long* ptr, int* col, double* val) {
  const Csr& A = h->lev[0].A;
  std::copy(A.ptr.begin(), A.ptr.end(), ptr);
  std::copy(A.col.begin(), A.col.end(), col);
  std::copy(A.val.begin(), A.val.end(), val);
}

void oc_apply(const oc_hierarchy* h, const double* u, double* y) { h->lev[0].A.matvec(u, y); }

void oc_smooth(const oc_hierarchy* h, double* u, const double* b, int nsweeps) { h->smooth(0, u, b, nsweeps); }

void oc_vcycle(const oc_hierarchy* h, double* u, const double* b) { h->vcycle(0, u, b); }

// Flexible CG preconditioned by one V-cycle from zero, from the initial guess
// in u, until ||b - A u|| <= rtol ||b - A u0|| (the recurrence residual, as
// the NumPy oracle); hist (maxit + 1 entries) receives the residual norms.
// Returns the number of iterations.
int oc_solve(const oc_hierarchy* h, double* u, const double* b, double rtol, int maxit, double* hist) {
  const Csr& A = h->lev[0].A;
  const int m = A.nr;
  std::vector<double> r(m), z(m, 0.0), p(m), q(m), rn(m), zn(m);
  auto dot = [&](const std::vector<double>& x, const std::vector<double>& y) {
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (int i = 0; i < m; ++i) s += x[i] * y[i];
    return s;
  };
  A.matvec(u, r.data());
  for (int i = 0; i < m; ++i) r[i] = b[i] - r[i];
  const double r0 = std::sqrt(dot(r, r));
  hist[0] = r0;
  if (r0 == 0.0) return 0;
  h->vcycle(0, z.data(), r.data());
  p = z;
  double rz = dot(r, z);
  int it = 0;
  while (it < maxit) {
    A.matvec(p.data(), q.data());
    const double alpha = rz / dot(p, q);
    for (int i = 0; i < m; ++i) {
      u[i] += alpha * p[i];
      rn[i] = r[i] - alpha * q[i];
    }
    ++it;
    hist[it] = std::sqrt(dot(rn, rn));
    if (hist[it] <= rtol * r0) break;
    std::fill(zn.begin(), zn.end(), 0.0);
    h->vcycle(0, zn.data(), rn.data());
    double beta = 0.0;
    for (int i = 0; i < m; ++i) beta += zn[i] * (rn[i] - r[i]);
    beta /= rz;
    rz = dot(zn, rn);
    for (int i = 0; i < m; ++i) p[i] = zn[i] + beta * p[i];
    r.swap(rn);
    z.swap(zn);
  }
  return it;
}

int oc_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
