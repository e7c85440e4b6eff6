// Oracle time step: block iteration of Newton solves with right-preconditioned
// restarted GMRES and (block) Jacobi.  TEST INFRASTRUCTURE ONLY (see orc.hpp).
//
// Sec. 3.5 (Newton with the analytic Jacobian, started from the previous
// iterate) and Fig. 1 of Sec. 3 (Navier-Stokes, then Cahn-Hilliard, repeated
// until the change of all fields between two sweeps is below block_tol).
// The paper uses PETSc's Krylov solvers; this restates plain GMRES(m) with
// classical Gram-Schmidt and one re-orthogonalisation pass.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "orc.hpp"

namespace orc {

namespace {

typedef std::vector<double> Vec;

double dot(const Vec& a, const Vec& b) {
  double s = 0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}
double norm2(const Vec& a) { return std::sqrt(dot(a, a)); }

// Solves the nf x nf system B x = y by Gaussian elimination with partial
// pivoting; returns false if B is singular.
bool solve_small(int nf, const double* B, const double* y, double* x) {
  double A[4][5];
  for (int r = 0; r < nf; ++r) {
    for (int c = 0; c < nf; ++c) A[r][c] = B[r * nf + c];
    A[r][nf] = y[r];
  }
  for (int c = 0; c < nf; ++c) {
    int piv = c;
    for (int r = c + 1; r < nf; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    if (A[piv][c] == 0.0) return false;
    for (int k = 0; k <= nf; ++k) std::swap(A[c][k], A[piv][k]);
    for (int r = c + 1; r < nf; ++r) {
      double f = A[r][c] / A[c][c];
      for (int k = c; k <= nf; ++k) A[r][k] -= f * A[c][k];
    }
  }
  for (int r = nf - 1; r >= 0; --r) {
    double s = A[r][nf];
    for (int k = r + 1; k < nf; ++k) s -= A[r][k] * x[k];
    x[r] = s / A[r][r];
  }
  return true;
}

struct BlockSystem {
  const Mesh& m;
  const Params& p;
  int block, f0, nf;
  const double* Unew;
  const double* Uold;
  std::vector<double> diag;  // n * nf * nf
  int precond;
  mutable std::vector<double> w6, o6;

  BlockSystem(const Mesh& m_, const Params& p_, int block_, const double* Unew_,
              const double* Uold_, int precond_)
      : m(m_), p(p_), block(block_), Unew(Unew_), Uold(Uold_), precond(precond_) {
    f0 = block == BLOCK_CH ? 0 : 2;
    nf = block == BLOCK_CH ? 2 : 4;
    w6.assign(m.nodes.size() * 6, 0.0);
    o6.assign(m.nodes.size() * 6, 0.0);
  }
  size_t size() const { return m.nodes.size() * nf; }
  std::string apply(const Vec& x, Vec& y) const {
    for (size_t i = 0; i < m.nodes.size(); ++i)
      for (int f = 0; f < nf; ++f) w6[i * 6 + f0 + f] = x[i * nf + f];
    std::string err = jvp(m, p, block, Unew, Uold, w6.data(), o6.data());
    if (!err.empty()) return err;
    y.resize(size());
    for (size_t i = 0; i < m.nodes.size(); ++i)
      for (int f = 0; f < nf; ++f) y[i * nf + f] = o6[i * 6 + f0 + f];
    return "";
  }
  std::string setup_precond() {
    diag.assign(m.nodes.size() * nf * nf, 0.0);
    return diag_blocks(m, p, block, Unew, Uold, diag.data());
  }
  // z = M^{-1} x
  bool precondition(const Vec& x, Vec& z) const {
    z.resize(size());
    for (size_t i = 0; i < m.nodes.size(); ++i) {
      const double* B = &diag[i * nf * nf];
      if (precond == 1) {
        if (!solve_small(nf, B, &x[i * nf], &z[i * nf])) return false;
      } else {
        for (int f = 0; f < nf; ++f) {
          double d = B[f * nf + f];
          if (d == 0.0) return false;
          z[i * nf + f] = x[i * nf + f] / d;
        }
      }
    }
    return true;
  }
};

// Restarted GMRES(m) for A x = b with right preconditioning, x0 = 0.
std::string gmres(const BlockSystem& S, const Vec& b, Vec& x, int restart, int max_it,
                  double rtol, int* its) {
  const size_t N = S.size();
  x.assign(N, 0.0);
  const double bn = norm2(b);
  *its = 0;
  if (bn == 0.0) return "";
  Vec r = b;
  double beta = bn;
  while (*its < max_it) {
    std::vector<Vec> V(restart + 1, Vec(N)), Z(restart);
    std::vector<std::vector<double>> H(restart + 1, std::vector<double>(restart, 0.0));
    std::vector<double> cs(restart), sn(restart), g(restart + 1, 0.0);
    for (size_t i = 0; i < N; ++i) V[0][i] = r[i] / beta;
    g[0] = beta;
    int k = 0;
    bool done = false;
    for (; k < restart && *its < max_it; ++k) {
      if (!S.precondition(V[k], Z[k])) return "singular diagonal block in the preconditioner";
      Vec w;
      std::string err = S.apply(Z[k], w);
      if (!err.empty()) return err;
      ++*its;
      // classical Gram-Schmidt, twice
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<double> h(k + 1);
        for (int j = 0; j <= k; ++j) h[j] = dot(V[j], w);
        for (int j = 0; j <= k; ++j)
          for (size_t i = 0; i < N; ++i) w[i] -= h[j] * V[j][i];
        for (int j = 0; j <= k; ++j) H[j][k] += h[j];
      }
      H[k + 1][k] = norm2(w);
      if (H[k + 1][k] > 0)
        for (size_t i = 0; i < N; ++i) V[k + 1][i] = w[i] / H[k + 1][k];
      // Givens rotations
      for (int j = 0; j < k; ++j) {
        double t = cs[j] * H[j][k] + sn[j] * H[j + 1][k];
        H[j + 1][k] = -sn[j] * H[j][k] + cs[j] * H[j + 1][k];
        H[j][k] = t;
      }
      double den = std::hypot(H[k][k], H[k + 1][k]);
      cs[k] = den > 0 ? H[k][k] / den : 1.0;
      sn[k] = den > 0 ? H[k + 1][k] / den : 0.0;
      H[k][k] = den;
      H[k + 1][k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      if (std::fabs(g[k + 1]) <= rtol * bn || den == 0.0) {
        ++k;
        done = true;
        break;
      }
    }
    // y = H^{-1} g, x += Z y
    std::vector<double> y(k, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int j = i + 1; j < k; ++j) s -= H[i][j] * y[j];
      y[i] = H[i][i] != 0 ? s / H[i][i] : 0.0;
    }
    for (int j = 0; j < k; ++j)
      for (size_t i = 0; i < N; ++i) x[i] += y[j] * Z[j][i];
    // true residual
    Vec Ax;
    std::string err = S.apply(x, Ax);
    if (!err.empty()) return err;
    for (size_t i = 0; i < N; ++i) r[i] = b[i] - Ax[i];
    beta = norm2(r);
    if (done || beta <= rtol * bn) break;
  }
  return "";
}

// Newton's method on one block (Sec. 3.5): U_{s+1} = U_s + dU with J dU = -F.
std::string newton(const Mesh& m, const Params& p, const SolverOpts& o, int block,
                   double* Unew, const double* Uold, const double* forcing, const double* bc,
                   int* newton_its,
                   int* gmres_its, double* rel_res, bool* converged) {
  const size_t n = m.nodes.size();
  const int f0 = block == BLOCK_CH ? 0 : 2, nf = block == BLOCK_CH ? 2 : 4;
  const int max_it = block == BLOCK_CH ? o.newton_max_it_ch : o.newton_max_it_ns;
  std::vector<double> R6(n * 6);
  Vec r(n * nf);
  auto eval = [&]() -> std::string {
    std::string err = residual(m, p, block, Unew, Uold, forcing, R6.data(), bc);
    if (!err.empty()) return err;
    for (size_t i = 0; i < n; ++i)
      for (int f = 0; f < nf; ++f) r[i * nf + f] = R6[i * 6 + f0 + f];
    return "";
  };
  std::string err = eval();
  if (!err.empty()) return err;
  const double r0 = norm2(r);
  *newton_its = 0;
  *gmres_its = 0;
  *converged = false;
  double rn = r0;
  for (;;) {
    if (!std::isfinite(rn)) return "non-finite residual";
    if (rn <= std::max(o.newton_rtol * r0, o.newton_atol)) {
      *converged = true;
      break;
    }
    if (*newton_its >= max_it) break;
    BlockSystem S(m, p, block, Unew, Uold, o.precond);
    err = S.setup_precond();
    if (!err.empty()) return err;
    Vec rhs(r.size()), dx;
    for (size_t i = 0; i < r.size(); ++i) rhs[i] = -r[i];
    int its = 0;
    err = gmres(S, rhs, dx, o.gmres_restart, o.gmres_max_it, o.gmres_rtol, &its);
    if (!err.empty()) return err;
    *gmres_its += its;
    for (size_t i = 0; i < n; ++i)
      for (int f = 0; f < nf; ++f) Unew[i * 6 + f0 + f] += dx[i * nf + f];
    ++*newton_its;
    err = eval();
    if (!err.empty()) return err;
    rn = norm2(r);
  }
  *rel_res = r0 > 0 ? rn / r0 : 0.0;
  return "";
}

}  // namespace

std::string step(const Mesh& m, const Params& p, const SolverOpts& o, double* U,
                 const double* forcing, const double* bc, StepStats* st) {
  const size_t n = m.nodes.size();
  std::vector<double> Uold(U, U + n * 6), Unew(U, U + n * 6), prev(n * 6);
  std::memset(st, 0, sizeof(StepStats));
  st->converged = 1;
  for (int l = 0; l < o.block_max_it; ++l) {
    prev = Unew;
    for (int b : {BLOCK_NS, BLOCK_CH}) {
      int nit = 0, git = 0;
      double rr = 0;
      bool conv = false;
      std::string err = newton(m, p, o, b, Unew.data(), Uold.data(), forcing, bc, &nit, &git, &rr,
                               &conv);
      if (!err.empty()) return err;
      st->newton_its[b] += nit;
      st->gmres_its[b] += git;
      st->rel_res[b] = rr;
      if (!conv) st->converged = 0;
    }
    st->block_its = l + 1;
    if (l >= o.block_min_it) {
      double change = 0;
      for (size_t i = 0; i < n * 6; ++i) change = std::max(change, std::fabs(Unew[i] - prev[i]));
      if (change <= o.block_tol) break;
    }
  }
  std::memcpy(U, Unew.data(), sizeof(double) * n * 6);
  diagnostics(m, p, U, &st->mass, &st->energy);
  return "";
}

}  // namespace orc
