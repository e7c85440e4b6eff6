// Oracle element machinery and the CH / NS block residuals.
// TEST INFRASTRUCTURE ONLY (see orc.hpp).
//
// Spatial discretisation: cG(1) trilinear hexahedra for every field (Sec. 3.4,
// opening paragraph).  Every integral is evaluated with the 2x2x2 Gauss rule
// on each leaf (the paper does not name a rule); hanging corners take their
// values through the constraint rows, and element vectors are returned to the
// independent nodes through the transpose of those rows (Sec. 4 "Handling
// hanging nodes").
//
// The Jacobian-vector product is the exact derivative of the same residual
// code, obtained with forward-mode dual numbers: the paper computes its
// Jacobian analytically from the variations of the operators (Sec. 3.5).
#include <cmath>
#include <cstring>
#include <vector>

#include "orc.hpp"

namespace orc {

// ---------------------------------------------------------- dual numbers --
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, Dual b) { return Dual(a / b.v, -a * b.d / (b.v * b.v)); }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
// x^(-1/2), derivative -1/2 x^(-3/2)
inline double inv_sqrt(double x) { return 1.0 / std::sqrt(x); }
inline Dual inv_sqrt(Dual x) {
  double r = 1.0 / std::sqrt(x.v);
  return Dual(r, -0.5 * r * r * r * x.d);
}
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }

// ------------------------------------------------------ Q1 on [-1,1]^3 ----
// Node a = i + 2j + 4k sits at (s_a0, s_a1, s_a2) with s = -1 for bit 0 and +1
// for bit 1.  N_a(xi) = prod_d (1 + s_ad xi_d) / 2.
static inline double sgn(int a, int d) { return ((a >> d) & 1) ? 1.0 : -1.0; }

struct QP {
  double N[8];
  double dN[8][3];      // physical gradient
  double d2N[8][3][3];  // physical second derivatives (pure ones are zero)
  double x[3];          // physical position
  double wdet;          // weight * det J
};

// Physical data at the 8 Gauss points (+-1/sqrt(3), weight 1) of a leaf with
// lower corner x0 and side h: grad = (2/h) grad_xi, det J = h^3/8.
static void element_qps(const double x0[3], double h, QP q[8]) {
  const double g = 1.0 / std::sqrt(3.0);
  for (int k = 0; k < 8; ++k) {
    double xi[3] = {sgn(k, 0) * g, sgn(k, 1) * g, sgn(k, 2) * g};
    for (int a = 0; a < 8; ++a) {
      double f[3];
      for (int d = 0; d < 3; ++d) f[d] = 0.5 * (1.0 + sgn(a, d) * xi[d]);
      q[k].N[a] = f[0] * f[1] * f[2];
      for (int d = 0; d < 3; ++d) {
        double p = 0.5 * sgn(a, d);
        for (int e = 0; e < 3; ++e)
          if (e != d) p *= f[e];
        q[k].dN[a][d] = (2.0 / h) * p;
      }
      for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) {
          if (d == e) {
            q[k].d2N[a][d][e] = 0.0;
            continue;
          }
          double p = 0.5 * sgn(a, d) * 0.5 * sgn(a, e);
          for (int c = 0; c < 3; ++c)
            if (c != d && c != e) p *= f[c];
          q[k].d2N[a][d][e] = (2.0 / h) * (2.0 / h) * p;
        }
    }
    for (int d = 0; d < 3; ++d) q[k].x[d] = x0[d] + 0.5 * h * (1.0 + xi[d]);
    q[k].wdet = 1.0 * h * h * h / 8.0;
  }
}

static void leaf_geometry(const Mesh& m, size_t e, double x0[3], double& h) {
  const Leaf& L = m.leaves[e];
  const double unit = std::ldexp(1.0, -m.D);
  x0[0] = L.x * unit;
  x0[1] = L.y * unit;
  x0[2] = L.z * unit;
  h = std::ldexp(1.0, -L.level);
}

// Value of field f of a node-major 6-field vector at corner c of element e
// (through the hanging constraint when the corner hangs).
static double corner_value(const Mesh& m, size_t e, int c, const double* U, int f) {
  int32_t r = m.elem[e][c];
  if (r >= 0) return U[(size_t)r * 6 + f];
  int32_t h = -1 - r;
  double s = 0;
  for (int64_t t = m.hang_off[h]; t < m.hang_off[h + 1]; ++t)
    s += m.hang_w[t] * U[(size_t)m.hang_ids[t] * 6 + f];
  return s;
}

// Adds an element vector (8 corners x 6 fields) into a global vector through
// the transpose of the constraint rows.
static void scatter(const Mesh& m, size_t e, const double r[8][6], double* R, int f0, int nf) {
  for (int c = 0; c < 8; ++c) {
    int32_t ref = m.elem[e][c];
    if (ref >= 0) {
      for (int f = f0; f < f0 + nf; ++f) R[(size_t)ref * 6 + f] += r[c][f];
    } else {
      int32_t h = -1 - ref;
      for (int64_t t = m.hang_off[h]; t < m.hang_off[h + 1]; ++t)
        for (int f = f0; f < f0 + nf; ++f)
          R[(size_t)m.hang_ids[t] * 6 + f] += m.hang_w[t] * r[c][f];
    }
  }
}

// Mixture properties (Sec. 2): rho = alpha phi + beta, eta = gamma phi + xi with
// the saturation pull-back phi* of the remark on excursions (eqn
// phi_for_density).  rho(+1) = 1, rho(-1) = rho_-/rho_+.
struct Mixture {
  double alpha, beta, gamma, xi;
  explicit Mixture(const Params& p) {
    alpha = 0.5 * (1.0 - p.rho_minus);
    beta = 0.5 * (1.0 + p.rho_minus);
    gamma = 0.5 * (1.0 - p.eta_minus);
    xi = 0.5 * (1.0 + p.eta_minus);
  }
};
static inline double phistar(double phi) {
  if (std::fabs(phi) <= 1.0) return phi;
  return phi > 0 ? 1.0 : -1.0;
}
static inline Dual phistar(Dual phi) {
  if (std::fabs(phi.v) <= 1.0) return phi;
  return Dual(phi.v > 0 ? 1.0 : -1.0);
}
// Mass flux coefficient: J = kappa grad(mu~) (thermo-consistency relation of
// Sec. 2).  With rho = alpha phi + beta, the continuity equation and the CH
// equation agree only for kappa = -alpha/Cn; the printed relation has -alpha.
static inline double kappa(const Params& p, const Mixture& mx) {
  return p.flux_mode == 1 ? -mx.alpha : -mx.alpha / p.Cn;
}

// ---------------------------------------------------------- CH element ----
// Residual of the phi and mu rows for test function q = N_a (Def. 1, eqns
// mu_eqn_var_semi_disc and phi_eqn_var_semi_disc, in their cG(1) form of
// Def. 2), with the Crank-Nicolson averages phi~ = (phi^k + phi^{k+1})/2,
// mu~ likewise, psi'~ = psi'(phi~) = phi~^3 - phi~, and the velocity
// v~ = (v^k + v^{k+1})/2 frozen from the Navier-Stokes block.
template <class S>
static void ch_element(const Mesh& m, const Params& p, size_t e, const S phi1[8],
                       const S mu1[8], const S v1[8][3], const double* Uold,
                       const double* forcing, S r[8][2]) {
  double x0[3], h;
  leaf_geometry(m, e, x0, h);
  QP q[8];
  element_qps(x0, h, q);
  double phi0[8], mu0[8];
  S vt[8][3];
  for (int c = 0; c < 8; ++c) {
    phi0[c] = corner_value(m, e, c, Uold, 0);
    mu0[c] = corner_value(m, e, c, Uold, 1);
    for (int d = 0; d < 3; ++d) vt[c][d] = 0.5 * (corner_value(m, e, c, Uold, 2 + d) + v1[c][d]);
  }
  for (int a = 0; a < 8; ++a) r[a][0] = r[a][1] = S(0.0);
  for (int k = 0; k < 8; ++k) {
    const QP& Q = q[k];
    S ph1 = 0.0, mt = 0.0;
    double ph0 = 0.0;
    S v[3] = {0.0, 0.0, 0.0};
    S gph[3] = {0.0, 0.0, 0.0}, gmu[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 8; ++c) {
      ph1 += Q.N[c] * phi1[c];
      ph0 += Q.N[c] * phi0[c];
      S phit_c = 0.5 * (phi1[c] + phi0[c]);
      S mut_c = 0.5 * (mu1[c] + mu0[c]);
      mt += Q.N[c] * mut_c;
      for (int d = 0; d < 3; ++d) {
        gph[d] += Q.dN[c][d] * phit_c;
        gmu[d] += Q.dN[c][d] * mut_c;
        v[d] += Q.N[c] * vt[c][d];
      }
    }
    S pt = 0.5 * (ph1 + ph0);                 // phi~ at the point
    S psi_prime = pt * pt * pt - pt;          // psi'(phi~)
    double f_phi = forcing ? forcing[(e * 8 + k) * 6 + 0] : 0.0;
    double f_mu = forcing ? forcing[(e * 8 + k) * 6 + 1] : 0.0;
    for (int a = 0; a < 8; ++a) {
      // (q, (phi^{k+1}-phi^k)/dt) - (dq/dx_i, v~_i phi~) + 1/(Pe Cn) (dq/dx_i, dmu~/dx_i)
      S rphi = Q.N[a] * (ph1 - ph0) / p.dt;
      for (int d = 0; d < 3; ++d) {
        rphi -= Q.dN[a][d] * v[d] * pt;
        rphi += (1.0 / (p.Pe * p.Cn)) * Q.dN[a][d] * gmu[d];
      }
      rphi -= Q.N[a] * f_phi;
      // -(q, mu~) + (q, psi'~) + Cn^2 (dq/dx_i, dphi~/dx_i)
      S rmu = -Q.N[a] * mt + Q.N[a] * psi_prime;
      for (int d = 0; d < 3; ++d) rmu += p.Cn * p.Cn * Q.dN[a][d] * gph[d];
      rmu -= Q.N[a] * f_mu;
      r[a][0] += Q.wdet * rphi;
      r[a][1] += Q.wdet * rmu;
    }
  }
}

// ---------------------------------------------------------- NS element ----
// Residual of the momentum and continuity rows of the fully discrete VMS form
// (Def. 2 of Sec. 3.4) for test functions w = N_a e_i and q = N_a, with
//  * rho, eta from phi^{k+1} (pulled back to [-1,1]) as in the time-discrete
//    momentum equation of Sec. 3; grad eta = gamma grad phi^{k+1} where
//    |phi^{k+1}| <= 1 and 0 where the pull-back is active;
//  * the coarse velocity and pressure in every VMS term and in tau_m taken at
//    the midpoint (v~, p~), the time derivative as (v^{k+1}-v^k)/dt;
//  * the capillary term with phi~;
//  * R_m the strong momentum residual; on trilinear elements the Laplacian of
//    a field vanishes but mixed second derivatives do not, so the capillary
//    divergence reduces to dphi~/dx_j d2phi~/dx_i dx_j and the viscous
//    divergence to deta/dx_k dv~_i/dx_k;
//  * tau_m, tau_c with G_ij = (4/h^2) delta_ij for the [-1,1]^3 reference
//    element and C_I from the parameters;
//  * the fine-scale convection term -(w_i, tau_m R_m,j dv~_i/dx_j) and the
//    continuity stabilisation +(dq/dx_i, tau_m R_m,i / rho), which is the
//    sign obtained by substituting v' = -tau_m R_m / rho into (q, dv'_i/dx_i).
template <class S>
static bool ns_element(const Mesh& m, const Params& p, size_t e, const S v1[8][3],
                       const S p1[8], const S phin[8], const S mun[8], const double* Uold,
                       const double* forcing, S r[8][4]) {
  const Mixture mx(p);
  const double kap = kappa(p, mx);
  double x0[3], h;
  leaf_geometry(m, e, x0, h);
  QP q[8];
  element_qps(x0, h, q);
  double v0[8][3], p0[8];
  S phi1[8], phit[8], mut[8];
  for (int c = 0; c < 8; ++c) {
    for (int d = 0; d < 3; ++d) v0[c][d] = corner_value(m, e, c, Uold, 2 + d);
    p0[c] = corner_value(m, e, c, Uold, 5);
    phi1[c] = phin[c];
    phit[c] = 0.5 * (phin[c] + corner_value(m, e, c, Uold, 0));
    mut[c] = 0.5 * (mun[c] + corner_value(m, e, c, Uold, 1));
  }
  const double G = 4.0 / (h * h);        // G_ij = G delta_ij
  const double trG = 3.0 * G;            // tr G
  const double GG = 3.0 * G * G;         // G_ij G_ij
  for (int a = 0; a < 8; ++a)
    for (int f = 0; f < 4; ++f) r[a][f] = S(0.0);
  bool ok = true;
  for (int k = 0; k < 8; ++k) {
    const QP& Q = q[k];
    // fields of the Cahn-Hilliard block (frozen in the block iteration)
    S ph1 = 0.0, gph1[3] = {0.0, 0.0, 0.0}, gpht[3] = {0.0, 0.0, 0.0}, Hpht[3][3], gmut[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d)
      for (int e2 = 0; e2 < 3; ++e2) Hpht[d][e2] = S(0.0);
    for (int c = 0; c < 8; ++c) {
      ph1 += Q.N[c] * phi1[c];
      for (int d = 0; d < 3; ++d) {
        gph1[d] += Q.dN[c][d] * phi1[c];
        gpht[d] += Q.dN[c][d] * phit[c];
        gmut[d] += Q.dN[c][d] * mut[c];
        for (int e2 = 0; e2 < 3; ++e2) Hpht[d][e2] += Q.d2N[c][d][e2] * phit[c];
      }
    }
    const S ps = phistar(ph1);
    const S rho = mx.alpha * ps + mx.beta;
    const S eta = mx.gamma * ps + mx.xi;
    S geta[3];
    for (int d = 0; d < 3; ++d) geta[d] = std::fabs(val(ph1)) <= 1.0 ? mx.gamma * gph1[d] : S(0.0);
    S J[3];
    for (int d = 0; d < 3; ++d) J[d] = kap * gmut[d];
    // unknown-dependent fields
    S vt[3] = {0.0, 0.0, 0.0}, dv[3] = {0.0, 0.0, 0.0}, gvt[3][3], pt = 0.0, gpt[3];
    for (int i = 0; i < 3; ++i) {
      gpt[i] = S(0.0);
      for (int j = 0; j < 3; ++j) gvt[i][j] = S(0.0);
    }
    for (int c = 0; c < 8; ++c) {
      S ptc = 0.5 * (p1[c] + p0[c]);
      pt += Q.N[c] * ptc;
      for (int i = 0; i < 3; ++i) {
        S vtc = 0.5 * (v1[c][i] + v0[c][i]);
        vt[i] += Q.N[c] * vtc;
        dv[i] += Q.N[c] * (v1[c][i] - v0[c][i]);
        gpt[i] += Q.dN[c][i] * ptc;
        for (int j = 0; j < 3; ++j) gvt[i][j] += Q.dN[c][j] * vtc;  // dv~_i/dx_j
      }
    }
    const double* fq = forcing ? forcing + (e * 8 + k) * 6 : nullptr;
    // strong residuals R_m, R_c
    S Rm[3];
    for (int i = 0; i < 3; ++i) {
      S t = rho * dv[i] / p.dt;
      for (int j = 0; j < 3; ++j) t += rho * vt[j] * gvt[i][j];
      for (int j = 0; j < 3; ++j) t += (1.0 / p.Pe) * J[j] * gvt[i][j];
      S cap = 0.0;
      for (int j = 0; j < 3; ++j) cap += gpht[j] * Hpht[i][j];
      t += (p.Cn / p.We) * cap;
      t += (1.0 / p.We) * gpt[i];
      for (int kk = 0; kk < 3; ++kk) t -= (1.0 / p.Re) * geta[kk] * gvt[i][kk];
      t -= rho * p.g[i] / p.Fr;
      if (fq) t -= fq[2 + i];
      Rm[i] = t;
    }
    S Rc = gvt[0][0] + gvt[1][1] + gvt[2][2];
    if (fq) Rc -= fq[5];
    // stabilisation parameters
    S vGv = G * (vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
    S vGJ = G * (vt[0] * J[0] + vt[1] * J[1] + vt[2] * J[2]);
    S visc = p.C_I * (eta / (rho * p.Re)) * (eta / (rho * p.Re)) * GG;
    S bracket = 4.0 / (p.dt * p.dt) + vGv + (1.0 / (rho * p.Pe)) * vGJ + visc;
    if (!(val(bracket) > 0.0)) {
      ok = false;
      continue;
    }
    S tau_m = inv_sqrt(bracket);
    S tau_c = 1.0 / (trG * tau_m);
    for (int a = 0; a < 8; ++a) {
      const double Na = Q.N[a];
      const double* dNa = Q.dN[a];
      for (int i = 0; i < 3; ++i) {
        S t = Na * rho * dv[i] / p.dt;                                    // (w_i, rho dv_i/dt)
        for (int j = 0; j < 3; ++j) t += Na * rho * vt[j] * gvt[i][j];    // (w_i, rho v_j dv_i/dx_j)
        for (int j = 0; j < 3; ++j) t -= Na * tau_m * Rm[j] * gvt[i][j];  // -(w_i, tau_m R_m,j dv_i/dx_j)
        for (int j = 0; j < 3; ++j) t += dNa[j] * vt[j] * tau_m * Rm[i];  // (dw_i/dx_j, v_j tau_m R_m,i)
        for (int j = 0; j < 3; ++j)
          t -= dNa[j] * (tau_m * tau_m / rho) * Rm[j] * Rm[i];            // -(dw_i/dx_j, tau^2/rho R_j R_i)
        for (int j = 0; j < 3; ++j) t += (1.0 / p.Pe) * Na * J[j] * gvt[i][j];
        for (int j = 0; j < 3; ++j)
          t += (1.0 / p.Pe) * dNa[j] * J[j] * (tau_m / rho) * Rm[i];
        for (int j = 0; j < 3; ++j) t -= (p.Cn / p.We) * dNa[j] * gpht[i] * gpht[j];
        t -= (1.0 / p.We) * dNa[i] * pt;                                  // -(1/We)(dw_i/dx_i, p)
        t += (1.0 / p.We) * dNa[i] * rho * tau_c * Rc;                    // +(1/We)(dw_i/dx_i, rho tau_c R_c)
        for (int kk = 0; kk < 3; ++kk) t += (1.0 / p.Re) * dNa[kk] * eta * gvt[i][kk];
        t -= Na * rho * p.g[i] / p.Fr;                                    // -(w_i, rho g_i / Fr)
        if (fq) t -= Na * fq[2 + i];
        r[a][i] += Q.wdet * t;
      }
      S tq = Na * (gvt[0][0] + gvt[1][1] + gvt[2][2]);                  // (q, dv_i/dx_i)
      for (int i = 0; i < 3; ++i) tq += dNa[i] * (tau_m / rho) * Rm[i];  // +(dq/dx_i, tau_m R_m,i / rho)
      if (fq) tq -= Na * fq[5];
      r[a][3] += Q.wdet * tq;
    }
  }
  return ok;
}

// --------------------------------------------------- assembled operators --
// Boundary rows (the paper's Dirichlet condition on the velocity and the
// pressure level, which the all-Dirichlet velocity leaves undetermined):
// velocity rows of boundary nodes read R = v^{k+1} - g with the wall data g
// (Bv, the velocity entries of Bv; Bv = U^k carries stationary walls); the
// pressure row of the pinned node reads R = p^{k+1} - p^k (Bp = U^k).
// Element contributions to those rows are dropped.  For the JVP both B are
// null and the rows are identity rows.
static void boundary_rows(const Mesh& m, int block, const double* A, const double* Bv,
                          const double* Bp, double* R) {
  if (block != BLOCK_NS) return;
  for (size_t n = 0; n < m.nodes.size(); ++n) {
    if (m.bflags[n] & 1)
      for (int d = 0; d < 3; ++d)
        R[n * 6 + 2 + d] = A[n * 6 + 2 + d] - (Bv ? Bv[n * 6 + 2 + d] : 0.0);
    if (m.bflags[n] & 2) R[n * 6 + 5] = A[n * 6 + 5] - (Bp ? Bp[n * 6 + 5] : 0.0);
  }
}

// Element vector of one element for the block, as duals whose derivative
// parts are seeded with the corner values dc[c][f] (all zero for a plain
// residual): out[c][f] (value) and dout[c][f] (derivative).
static bool element_eval_seeded(const Mesh& m, const Params& p, int block, size_t e,
                                const double* Unew, const double* Uold, const double dc[8][6],
                                const double* forcing, double out[8][6], double dout[8][6]) {
  for (int c = 0; c < 8; ++c)
    for (int f = 0; f < 6; ++f) out[c][f] = dout[c][f] = 0.0;
  Dual phi1[8], mu1[8], v1[8][3], p1[8];
  for (int c = 0; c < 8; ++c) {
    phi1[c] = Dual(corner_value(m, e, c, Unew, 0), dc[c][0]);
    mu1[c] = Dual(corner_value(m, e, c, Unew, 1), dc[c][1]);
    for (int d = 0; d < 3; ++d) v1[c][d] = Dual(corner_value(m, e, c, Unew, 2 + d), dc[c][2 + d]);
    p1[c] = Dual(corner_value(m, e, c, Unew, 5), dc[c][5]);
  }
  if (block == BLOCK_CH) {
    Dual r[8][2];
    ch_element<Dual>(m, p, e, phi1, mu1, v1, Uold, forcing, r);
    for (int c = 0; c < 8; ++c)
      for (int f = 0; f < 2; ++f) {
        out[c][f] = r[c][f].v;
        dout[c][f] = r[c][f].d;
      }
    return true;
  }
  Dual r[8][4];
  bool ok = ns_element<Dual>(m, p, e, v1, p1, phi1, mu1, Uold, forcing, r);
  for (int c = 0; c < 8; ++c)
    for (int f = 0; f < 4; ++f) {
      out[c][2 + f] = r[c][f].v;
      dout[c][2 + f] = r[c][f].d;
    }
  return ok;
}

// Seeds: the block's own unknowns (block Jacobian), or all six fields of
// U^{k+1} (full: the block's rows of the coupled Jacobian).
static bool element_eval(const Mesh& m, const Params& p, int block, size_t e,
                         const double* Unew, const double* Uold, const double* dU,
                         const double* forcing, double out[8][6], double dout[8][6], bool full = false) {
  const int f0 = block == BLOCK_CH ? 0 : 2, f1 = block == BLOCK_CH ? 2 : 6;
  double dc[8][6];
  for (int c = 0; c < 8; ++c)
    for (int f = 0; f < 6; ++f)
      dc[c][f] = (dU && (full || (f >= f0 && f < f1))) ? corner_value(m, e, c, dU, f) : 0.0;
  return element_eval_seeded(m, p, block, e, Unew, Uold, dc, forcing, out, dout);
}

static std::string assemble(const Mesh& m, const Params& p, int block, const double* Unew,
                            const double* Uold, const double* dU, const double* forcing,
                            double* out, bool want_derivative, bool full = false,
                            const double* bc = nullptr) {
  const size_t n = m.nodes.size(), E = m.leaves.size();
  std::memset(out, 0, sizeof(double) * n * 6);
  const int f0 = block == BLOCK_CH ? 0 : 2, nf = block == BLOCK_CH ? 2 : 4;
  // element vectors are computed independently (in parallel), then added in
  // element order so that the result does not depend on the thread count
  std::vector<double> ev(E * 48);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (long e = 0; e < (long)E; ++e) {
    double o[8][6], d[8][6];
    if (!element_eval(m, p, block, (size_t)e, Unew, Uold, dU, forcing, o, d, full)) bad += 1;
    std::memcpy(&ev[(size_t)e * 48], want_derivative ? &d[0][0] : &o[0][0], sizeof(double) * 48);
  }
  if (bad) return "tau_m bracket is not positive";
  for (size_t e = 0; e < E; ++e) {
    double r[8][6];
    std::memcpy(&r[0][0], &ev[e * 48], sizeof(double) * 48);
    scatter(m, e, r, out, f0, nf);
  }
  if (want_derivative)
    boundary_rows(m, block, dU, nullptr, nullptr, out);
  else
    boundary_rows(m, block, Unew, bc ? bc : Uold, Uold, out);
  return "";
}

std::string residual(const Mesh& m, const Params& p, int block, const double* Unew,
                     const double* Uold, const double* forcing, double* R, const double* bc) {
  return assemble(m, p, block, Unew, Uold, nullptr, forcing, R, false, false, bc);
}

std::string jvp(const Mesh& m, const Params& p, int block, const double* Unew,
                const double* Uold, const double* dU, double* JdU) {
  return assemble(m, p, block, Unew, Uold, dU, nullptr, JdU, true);
}

std::string jvp_full(const Mesh& m, const Params& p, int block, const double* Unew,
                     const double* Uold, const double* dU, double* JdU) {
  return assemble(m, p, block, Unew, Uold, dU, nullptr, JdU, true, true);
}

std::string residual_rows(const Mesh& m, const Params& p, int block, const double* Unew,
                          const double* Uold, const int32_t* rows, int64_t nrows,
                          const double* dU, double* out) {
  // elements touching any listed row (directly or through a constraint)
  const size_t n = m.nodes.size(), E = m.leaves.size();
  std::vector<char> want(n, 0);
  for (int64_t k = 0; k < nrows; ++k) {
    if (rows[k] < 0 || (size_t)rows[k] >= n) return "row out of range";
    want[rows[k]] = 1;
  }
  std::vector<double> full(n * 6, 0.0);
  const int f0 = block == BLOCK_CH ? 0 : 2, nf = block == BLOCK_CH ? 2 : 4;
  for (size_t e = 0; e < E; ++e) {
    bool touch = false;
    for (int c = 0; c < 8 && !touch; ++c) {
      int32_t r = m.elem[e][c];
      if (r >= 0) {
        touch = want[r];
      } else {
        int32_t h = -1 - r;
        for (int64_t t = m.hang_off[h]; t < m.hang_off[h + 1]; ++t)
          if (want[m.hang_ids[t]]) touch = true;
      }
    }
    if (!touch) continue;
    double o[8][6], d[8][6];
    if (!element_eval(m, p, block, e, Unew, Uold, dU, nullptr, o, d))
      return "tau_m bracket is not positive";
    scatter(m, e, dU ? d : o, full.data(), f0, nf);
  }
  if (dU)
    boundary_rows(m, block, dU, nullptr, nullptr, full.data());
  else
    boundary_rows(m, block, Unew, Uold, Uold, full.data());
  for (int64_t k = 0; k < nrows; ++k)
    for (int f = 0; f < 6; ++f) out[k * 6 + f] = full[(size_t)rows[k] * 6 + f];
  return "";
}

// Node-block diagonal of P^T J P: block n = d R_n / d U_n over the block's
// fields, from element Jacobian columns seeded at each independent node the
// element touches.  Boundary rows are identity rows.
std::string diag_blocks(const Mesh& m, const Params& p, int block, const double* Unew,
                        const double* Uold, double* out) {
  const size_t n = m.nodes.size(), E = m.leaves.size();
  const int f0 = block == BLOCK_CH ? 0 : 2, nf = block == BLOCK_CH ? 2 : 4;
  std::memset(out, 0, sizeof(double) * n * nf * nf);
  // per element: the independent nodes it touches and their nf x nf blocks;
  // computed in parallel, added in element order
  std::vector<std::vector<int32_t>> ids(E);
  std::vector<std::vector<double>> blk(E);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad)
  for (long e = 0; e < (long)E; ++e) {
    std::vector<int32_t> tid;
    std::vector<std::array<double, 8>> tw;
    auto add = [&](int32_t id, int c, double w) {
      for (size_t t = 0; t < tid.size(); ++t)
        if (tid[t] == id) {
          tw[t][c] += w;
          return;
        }
      std::array<double, 8> z{};
      z[c] = w;
      tid.push_back(id);
      tw.push_back(z);
    };
    for (int c = 0; c < 8; ++c) {
      int32_t r = m.elem[e][c];
      if (r >= 0) {
        add(r, c, 1.0);
      } else {
        int32_t h = -1 - r;
        for (int64_t t = m.hang_off[h]; t < m.hang_off[h + 1]; ++t) add(m.hang_ids[t], c, m.hang_w[t]);
      }
    }
    // unit seed at one independent node: corner c sees the weight P_{c,node}
    std::vector<double> b(tid.size() * nf * nf, 0.0);
    for (size_t t = 0; t < tid.size(); ++t) {
      for (int fc = 0; fc < nf; ++fc) {
        double dc[8][6] = {};
        for (int c = 0; c < 8; ++c) dc[c][f0 + fc] = tw[t][c];
        double o[8][6], d[8][6];
        if (!element_eval_seeded(m, p, block, (size_t)e, Unew, Uold, dc, nullptr, o, d)) bad += 1;
        for (int c = 0; c < 8; ++c) {
          double w = tw[t][c];
          if (w == 0.0) continue;
          for (int fr = 0; fr < nf; ++fr) b[t * nf * nf + fr * nf + fc] += w * d[c][f0 + fr];
        }
      }
    }
    ids[e].swap(tid);
    blk[e].swap(b);
  }
  if (bad) return "tau_m bracket is not positive";
  for (size_t e = 0; e < E; ++e)
    for (size_t t = 0; t < ids[e].size(); ++t)
      for (int k = 0; k < nf * nf; ++k) out[(size_t)ids[e][t] * nf * nf + k] += blk[e][t * nf * nf + k];
  if (block == BLOCK_NS) {
    for (size_t i = 0; i < n; ++i) {
      double* B = out + i * 16;
      if (m.bflags[i] & 1)
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 4; ++c) B[r * 4 + c] = (r == c) ? 1.0 : 0.0;
      if (m.bflags[i] & 2)
        for (int c = 0; c < 4; ++c) B[3 * 4 + c] = (c == 3) ? 1.0 : 0.0;
    }
  }
  return "";
}

// Total energy of Sec. 2 (eqn energy_functional) in the discrete form used by
// the stability proof: kinetic energy with rho(phi*), the free energy
// (1/(Cn We)) (psi(phi) + Cn^2/2 |grad phi|^2), and the gravitational
// potential (1/Fr) rho(phi*) (-g . x) outside the 1/(Cn We) factor, as the
// proof of Lemma 2 carries it.
void diagnostics(const Mesh& m, const Params& p, const double* U, double* mass,
                 double* energy) {
  const Mixture mx(p);
  double M = 0, En = 0;
  for (size_t e = 0; e < m.leaves.size(); ++e) {
    double x0[3], h;
    leaf_geometry(m, e, x0, h);
    QP q[8];
    element_qps(x0, h, q);
    double cv[8][6];
    for (int c = 0; c < 8; ++c)
      for (int f = 0; f < 6; ++f) cv[c][f] = corner_value(m, e, c, U, f);
    for (int k = 0; k < 8; ++k) {
      double phi = 0, v[3] = {0, 0, 0}, g[3] = {0, 0, 0};
      for (int c = 0; c < 8; ++c) {
        phi += q[k].N[c] * cv[c][0];
        for (int d = 0; d < 3; ++d) {
          v[d] += q[k].N[c] * cv[c][2 + d];
          g[d] += q[k].dN[c][d] * cv[c][0];
        }
      }
      double rho = mx.alpha * phistar(phi) + mx.beta;
      double psi = 0.25 * (phi * phi - 1.0) * (phi * phi - 1.0);
      double kin = 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      double grad2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
      double free_e = (1.0 / (p.Cn * p.We)) * (psi + 0.5 * p.Cn * p.Cn * grad2);
      double gx = p.g[0] * q[k].x[0] + p.g[1] * q[k].x[1] + p.g[2] * q[k].x[2];
      double pot = (1.0 / p.Fr) * rho * (-gx);
      M += q[k].wdet * phi;
      En += q[k].wdet * (kin + free_e + pot);
    }
  }
  *mass = M;
  *energy = En;
}

}  // namespace orc
