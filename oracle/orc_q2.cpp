// Oracle for the cG(2) variant of both blocks: triquadratic hexahedra with
// 27 nodes on the same balanced octree.  TEST INFRASTRUCTURE ONLY (see
// orc.hpp).
//
// The paper discretises every field with cG(1) (Sec. 3.4) and names
// higher-order cG spaces as future work (Sec. 7).  This file restates the CH
// block of Def. 2 (eqns mu_eqn_var_semi_disc and phi_eqn_var_semi_disc) and
// its VMS Navier-Stokes block, with the same Crank-Nicolson averages and
// readings as the cG(1) oracle, on the space of continuous piecewise
// triquadratic functions:
//  * nodes: the 3x3x3 lattice of every leaf (corners, edge midpoints, face
//    centres, cell centre);
//  * integrals: the 3x3x3 Gauss-Legendre rule on each leaf;
//  * hanging nodes (Sec. 4 "Handling hanging nodes", carried over to Q2): a
//    lattice point of a leaf that is not a lattice point of some other leaf
//    whose closure contains it takes the value of the coarsest such leaf's
//    triquadratic interpolant there; parents that hang themselves are
//    substituted recursively.
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <unordered_map>

#include "orc.hpp"

namespace orc {

namespace {

uint64_t leaf_key(int level, uint32_t x, uint32_t y, uint32_t z) {
  return ((uint64_t)level << 60) | ((uint64_t)x << 40) | ((uint64_t)y << 20) | (uint64_t)z;
}

// 1D Lagrange basis on [0, 2] with nodes 0, 1, 2 (the lattice coordinate of a
// point inside a leaf, in units of half the leaf side).
double lag(int i, double t) {
  if (i == 0) return 0.5 * (t - 1.0) * (t - 2.0);
  if (i == 1) return -t * (t - 2.0);
  return 0.5 * t * (t - 1.0);
}

}  // namespace

std::string build_q2(const Mesh& m, MeshQ2& out) {
  out = MeshQ2();
  out.D = m.D;
  const int64_t E = (int64_t)m.leaves.size();
  std::unordered_map<uint64_t, int32_t> leaf_of;
  for (int64_t e = 0; e < E; ++e) {
    const Leaf& L = m.leaves[e];
    leaf_of[leaf_key(L.level, L.x, L.y, L.z)] = (int32_t)e;
  }
  const int64_t ext[3] = {(int64_t)m.T[0] << m.D, (int64_t)m.T[1] << m.D, (int64_t)m.T[2] << m.D};
  // the leaf that holds the finest-level cell c, or -1 outside the brick
  auto locate = [&](const int64_t c[3]) -> int32_t {
    for (int d = 0; d < 3; ++d)
      if (c[d] < 0 || c[d] >= ext[d]) return -1;
    for (int l = m.D; l >= 0; --l) {
      const int64_t s = (int64_t)1 << (m.D - l);
      auto it = leaf_of.find(leaf_key(l, (uint32_t)(c[0] / s * s), (uint32_t)(c[1] / s * s),
                                      (uint32_t)(c[2] / s * s)));
      if (it != leaf_of.end()) return it->second;
    }
    return -1;
  };
  // lattice points in doubled units (2^-(D+1)): leaf anchor 2x, spacing s
  auto side = [&](int32_t e) -> int64_t { return (int64_t)1 << (m.D - m.leaves[e].level); };
  auto on_lattice = [&](int32_t e, const int64_t P[3]) {
    const Leaf& L = m.leaves[e];
    const int64_t a[3] = {2 * (int64_t)L.x, 2 * (int64_t)L.y, 2 * (int64_t)L.z};
    const int64_t s = side(e);
    for (int d = 0; d < 3; ++d) {
      const int64_t r = P[d] - a[d];
      if (r < 0 || r > 2 * s || r % s != 0) return false;
    }
    return true;
  };
  // every lattice point of every leaf, keyed by its Morton code
  std::map<uint64_t, std::array<int64_t, 3>> pts;
  for (int64_t e = 0; e < E; ++e) {
    const Leaf& L = m.leaves[e];
    const int64_t s = side((int32_t)e);
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i) {
          const std::array<int64_t, 3> P = {2 * (int64_t)L.x + i * s, 2 * (int64_t)L.y + j * s,
                                            2 * (int64_t)L.z + k * s};
          pts[morton3((uint32_t)P[0], (uint32_t)P[1], (uint32_t)P[2])] = P;
        }
  }
  // classification: the leaves around P (one per octant) and the coarsest of
  // them that does not have P on its lattice
  std::map<uint64_t, int32_t> constrainer;  // hanging point -> constraining leaf
  for (auto& kv : pts) {
    const auto& P = kv.second;
    int32_t best = -1;
    for (int o = 0; o < 8; ++o) {
      int64_t c[3];
      for (int d = 0; d < 3; ++d) {
        const int up = (o >> d) & 1;
        c[d] = (P[d] & 1) ? (P[d] - 1) / 2 : P[d] / 2 - (up ? 0 : 1);
      }
      const int32_t e = locate(c);
      if (e < 0) continue;
      if (on_lattice(e, P.data())) continue;
      if (best < 0 || side(e) > side(best) || (side(e) == side(best) && e < best)) best = e;
    }
    if (best >= 0) constrainer[kv.first] = best;
  }
  std::unordered_map<uint64_t, int32_t> id, hid;
  for (auto& kv : pts) {
    const auto& P = kv.second;
    if (constrainer.count(kv.first)) {
      hid[kv.first] = (int32_t)out.hang_xyz.size();
      out.hang_xyz.push_back({(uint32_t)P[0], (uint32_t)P[1], (uint32_t)P[2]});
    } else {
      id[kv.first] = (int32_t)out.nodes.size();
      out.nodes.push_back({(uint32_t)P[0], (uint32_t)P[1], (uint32_t)P[2]});
    }
  }
  // constraint rows: the constraining leaf's interpolant, parents expanded
  std::unordered_map<uint64_t, std::map<int32_t, double>> rows;
  std::unordered_map<uint64_t, int> state;  // 1 in progress, 2 done
  std::string err;
  std::function<const std::map<int32_t, double>&(uint64_t)> expand =
      [&](uint64_t key) -> const std::map<int32_t, double>& {
    auto& row = rows[key];
    if (state[key] == 2) return row;
    if (state[key] == 1) {
      err = "cyclic hanging-node constraints";
      return row;
    }
    state[key] = 1;
    const auto& P = pts[key];
    const int32_t e = constrainer[key];
    const Leaf& L = m.leaves[e];
    const int64_t s = side(e);
    const int64_t a[3] = {2 * (int64_t)L.x, 2 * (int64_t)L.y, 2 * (int64_t)L.z};
    double t[3];
    for (int d = 0; d < 3; ++d) t[d] = (double)(P[d] - a[d]) / (double)s;
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i) {
          const double w = lag(i, t[0]) * lag(j, t[1]) * lag(k, t[2]);
          if (w == 0.0) continue;
          const uint64_t q = morton3((uint32_t)(a[0] + i * s), (uint32_t)(a[1] + j * s),
                                     (uint32_t)(a[2] + k * s));
          if (q == key) {
            err = "hanging node constrained by itself";
            continue;
          }
          auto it = id.find(q);
          if (it != id.end()) {
            row[it->second] += w;
          } else {
            const auto& sub = expand(q);
            for (auto& tw : sub) row[tw.first] += w * tw.second;
          }
        }
    state[key] = 2;
    return row;
  };
  out.hang_off.push_back(0);
  for (auto& hx : out.hang_xyz) {
    const uint64_t key = morton3(hx[0], hx[1], hx[2]);
    const auto& row = expand(key);
    if (!err.empty()) return err;
    for (auto& tw : row) {
      if (tw.second == 0.0) continue;
      out.hang_ids.push_back(tw.first);
      out.hang_w.push_back(tw.second);
    }
    out.hang_off.push_back((int64_t)out.hang_ids.size());
  }
  // boundary flags of the independent nodes (bit 0 on the brick's boundary,
  // bit 1 the pressure pin on the Morton-first node, as in the cG(1) mesh)
  out.bflags.assign(out.nodes.size(), 0);
  for (size_t i = 0; i < out.nodes.size(); ++i)
    for (int d = 0; d < 3; ++d)
      if (out.nodes[i][d] == 0 || (int64_t)out.nodes[i][d] == 2 * ext[d]) out.bflags[i] = 1;
  if (!out.bflags.empty()) out.bflags[0] |= 2;
  // element connectivity, node a = i + 3j + 9k
  out.elem.resize(E);
  for (int64_t e = 0; e < E; ++e) {
    const Leaf& L = m.leaves[e];
    const int64_t s = side((int32_t)e);
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i) {
          const uint64_t q = morton3((uint32_t)(2 * (int64_t)L.x + i * s),
                                     (uint32_t)(2 * (int64_t)L.y + j * s),
                                     (uint32_t)(2 * (int64_t)L.z + k * s));
          auto it = id.find(q);
          out.elem[e][i + 3 * j + 9 * k] = it != id.end() ? it->second : -1 - hid.at(q);
        }
  }
  return "";
}

namespace {

// Dual numbers for the JVP (the CH rows' exact derivative in the direction of
// (phi^{k+1}, mu^{k+1}), as the cG(1) oracle obtains it).
struct D2 {
  double v, d;
  D2(double a = 0, double b = 0) : v(a), d(b) {}
};
inline D2 operator+(D2 a, D2 b) { return D2(a.v + b.v, a.d + b.d); }
inline D2 operator-(D2 a, D2 b) { return D2(a.v - b.v, a.d - b.d); }
inline D2 operator*(D2 a, D2 b) { return D2(a.v * b.v, a.d * b.v + a.v * b.d); }
inline D2 operator*(double a, D2 b) { return D2(a * b.v, a * b.d); }
inline D2 operator/(D2 a, double b) { return D2(a.v / b, a.d / b); }
inline D2 operator/(D2 a, D2 b) { return D2(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
inline D2 operator/(double a, D2 b) { return D2(a / b.v, -a * b.d / (b.v * b.v)); }
inline D2 operator-(D2 a) { return D2(-a.v, -a.d); }
inline D2& operator+=(D2& a, D2 b) { a = a + b; return a; }
inline D2& operator-=(D2& a, D2 b) { a = a - b; return a; }
inline double val2(double x) { return x; }
inline double val2(D2 x) { return x.v; }
inline double rsqrt2(double x) { return 1.0 / std::sqrt(x); }
inline D2 rsqrt2(D2 x) {
  const double r = 1.0 / std::sqrt(x.v);
  return D2(r, -0.5 * r * r * r * x.d);
}
// phi pulled back to [-1, 1] (the remark on excursions, eqn phi_for_density)
inline double pull2(double x) { return std::fabs(x) <= 1.0 ? x : (x > 0 ? 1.0 : -1.0); }
inline D2 pull2(D2 x) { return std::fabs(x.v) <= 1.0 ? x : D2(x.v > 0 ? 1.0 : -1.0); }

// 3-point Gauss-Legendre rule on [0, 1]
const double kGq[3] = {0.5 - 0.5 * 0.77459666924148337704, 0.5, 0.5 + 0.5 * 0.77459666924148337704};
const double kGw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

// basis on [0, 1] with nodes 0, 1/2, 1, and its derivative
double b1(int i, double u) { return lag(i, 2.0 * u); }
double db1(int i, double u) {
  const double t = 2.0 * u;
  if (i == 0) return 2.0 * (t - 1.5);
  if (i == 1) return 2.0 * (2.0 - 2.0 * t);
  return 2.0 * (t - 0.5);
}

// second derivative d2/du2 of the basis on [0, 1] with nodes 0, 1/2, 1
double d2b1(int i) { return i == 1 ? -8.0 : 4.0; }

// Values, physical gradients and Hessians of the 27 basis functions at a
// point (u in [0, 1]^3) of a leaf of side h.
struct Q2Pt {
  double N[27], dN[27][3], d2N[27][3][3];
};
void q2_point(const double u[3], double h, Q2Pt& P) {
  for (int a = 0; a < 27; ++a) {
    const int ia[3] = {a % 3, (a / 3) % 3, a / 9};
    double b[3], db[3], dd[3];
    for (int d = 0; d < 3; ++d) {
      b[d] = b1(ia[d], u[d]);
      db[d] = db1(ia[d], u[d]) / h;
      dd[d] = d2b1(ia[d]) / (h * h);
    }
    P.N[a] = b[0] * b[1] * b[2];
    for (int d = 0; d < 3; ++d) {
      double g = db[d];
      for (int e = 0; e < 3; ++e)
        if (e != d) g *= b[e];
      P.dN[a][d] = g;
      for (int e = 0; e < 3; ++e) {
        double H = 1.0;
        for (int c = 0; c < 3; ++c) {
          if (c == d && c == e) H *= dd[c];
          else if (c == d || c == e) H *= db[c];
          else H *= b[c];
        }
        P.d2N[a][d][e] = H;
      }
    }
  }
}

template <class S>
S node_value(const MeshQ2& q, int32_t ref, const S* U, int f) {
  if (ref >= 0) return U[(size_t)ref * 6 + f];
  const int32_t h = -1 - ref;
  S s = 0.0;
  for (int64_t t = q.hang_off[h]; t < q.hang_off[h + 1]; ++t)
    s = s + q.hang_w[t] * U[(size_t)q.hang_ids[t] * 6 + f];
  return s;
}

// CH rows of one leaf for test functions q = N_a, a = 0..26, with the
// Crank-Nicolson averages of the cG(1) oracle: phi~, mu~, v~ the midpoints,
// psi'(phi~) = phi~^3 - phi~.
template <class S>
void ch_element_q2(const Mesh& m, const MeshQ2& q, const Params& p, size_t e, const S* U1,
                   const double* U0, S r[27][2]) {
  const Leaf& L = m.leaves[e];
  const double h = std::ldexp(1.0, -L.level);
  S phi1[27], mu1[27], vt[27][3];
  double phi0[27], mu0[27];
  for (int a = 0; a < 27; ++a) {
    const int32_t ref = q.elem[e][a];
    phi1[a] = node_value<S>(q, ref, U1, 0);
    mu1[a] = node_value<S>(q, ref, U1, 1);
    phi0[a] = node_value<double>(q, ref, U0, 0);
    mu0[a] = node_value<double>(q, ref, U0, 1);
    for (int d = 0; d < 3; ++d)
      vt[a][d] = 0.5 * (node_value<S>(q, ref, U1, 2 + d) + S(node_value<double>(q, ref, U0, 2 + d)));
  }
  for (int a = 0; a < 27; ++a) r[a][0] = r[a][1] = S(0.0);
  const double kd = 1.0 / (p.Pe * p.Cn), cn2 = p.Cn * p.Cn;
  for (int gk = 0; gk < 3; ++gk)
    for (int gj = 0; gj < 3; ++gj)
      for (int gi = 0; gi < 3; ++gi) {
        const double u[3] = {kGq[gi], kGq[gj], kGq[gk]};
        const double wdet = kGw[gi] * kGw[gj] * kGw[gk] * h * h * h;
        double N[27], dN[27][3];
        for (int a = 0; a < 27; ++a) {
          const int ia[3] = {a % 3, (a / 3) % 3, a / 9};
          double b[3], db[3];
          for (int d = 0; d < 3; ++d) {
            b[d] = b1(ia[d], u[d]);
            db[d] = db1(ia[d], u[d]) / h;
          }
          N[a] = b[0] * b[1] * b[2];
          dN[a][0] = db[0] * b[1] * b[2];
          dN[a][1] = b[0] * db[1] * b[2];
          dN[a][2] = b[0] * b[1] * db[2];
        }
        S ph1 = 0.0, mt = 0.0, v[3] = {0.0, 0.0, 0.0}, gph[3] = {0.0, 0.0, 0.0},
          gmu[3] = {0.0, 0.0, 0.0};
        double ph0 = 0.0;
        for (int a = 0; a < 27; ++a) {
          ph1 = ph1 + N[a] * phi1[a];
          ph0 += N[a] * phi0[a];
          const S pta = 0.5 * (phi1[a] + S(phi0[a]));
          const S mta = 0.5 * (mu1[a] + S(mu0[a]));
          mt = mt + N[a] * mta;
          for (int d = 0; d < 3; ++d) {
            gph[d] = gph[d] + dN[a][d] * pta;
            gmu[d] = gmu[d] + dN[a][d] * mta;
            v[d] = v[d] + N[a] * vt[a][d];
          }
        }
        const S pt = 0.5 * (ph1 + S(ph0));
        const S psi_prime = pt * pt * pt - pt;
        for (int a = 0; a < 27; ++a) {
          // (q, (phi^{k+1}-phi^k)/dt) - (dq/dx_i, v~_i phi~) + 1/(Pe Cn) (dq/dx_i, dmu~/dx_i)
          S rphi = N[a] * (ph1 - S(ph0)) / p.dt;
          for (int d = 0; d < 3; ++d) rphi = rphi - dN[a][d] * (v[d] * pt) + kd * dN[a][d] * gmu[d];
          // -(q, mu~) + (q, psi'(phi~)) + Cn^2 (dq/dx_i, dphi~/dx_i)
          S rmu = N[a] * (psi_prime - mt);
          for (int d = 0; d < 3; ++d) rmu = rmu + cn2 * dN[a][d] * gph[d];
          r[a][0] = r[a][0] + wdet * rphi;
          r[a][1] = r[a][1] + wdet * rmu;
        }
      }
}

// NS rows of one leaf for test functions w = N_a e_i and q = N_a: the VMS form
// of the cG(1) oracle (Def. 2 of Sec. 3.4, with its readings: rho, eta from
// phi^{k+1} pulled back to [-1, 1]; grad eta = gamma grad phi^{k+1} inside
// [-1, 1]; the coarse velocity and pressure at the midpoint; J = kappa grad
// mu~; tau_m, tau_c with G = 4/h^2; the fine-scale convection term and the
// continuity stabilisation) on the triquadratic space.  The strong momentum
// residual R_m keeps every second-derivative term, which on trilinear leaves
// reduce to their mixed parts: the capillary divergence
// d/dx_j (dphi~/dx_i dphi~/dx_j) = d2phi~/dx_i dx_j dphi~/dx_j +
// dphi~/dx_i lap phi~, and the viscous divergence d/dx_j (eta dv~_i/dx_j) =
// deta/dx_j dv~_i/dx_j + eta lap v~_i.  Returns false where the tau_m bracket
// is not positive.
template <class S>
bool ns_element_q2(const Mesh& m, const MeshQ2& q, const Params& p, size_t e, const S* U1,
                   const double* U0, S r[27][4]) {
  const double alpha = 0.5 * (1.0 - p.rho_minus), beta = 0.5 * (1.0 + p.rho_minus);
  const double gamma = 0.5 * (1.0 - p.eta_minus), xi = 0.5 * (1.0 + p.eta_minus);
  const double kap = p.flux_mode == 1 ? -alpha : -alpha / p.Cn;
  const Leaf& L = m.leaves[e];
  const double h = std::ldexp(1.0, -L.level);
  S phi1[27], phit[27], mut[27], vt[27][3], dvn[27][3], ptn[27];
  for (int a = 0; a < 27; ++a) {
    const int32_t ref = q.elem[e][a];
    phi1[a] = node_value<S>(q, ref, U1, 0);
    phit[a] = 0.5 * (phi1[a] + S(node_value<double>(q, ref, U0, 0)));
    mut[a] = 0.5 * (node_value<S>(q, ref, U1, 1) + S(node_value<double>(q, ref, U0, 1)));
    for (int d = 0; d < 3; ++d) {
      const S v1 = node_value<S>(q, ref, U1, 2 + d);
      const double v0 = node_value<double>(q, ref, U0, 2 + d);
      vt[a][d] = 0.5 * (v1 + S(v0));
      dvn[a][d] = v1 - S(v0);
    }
    ptn[a] = 0.5 * (node_value<S>(q, ref, U1, 5) + S(node_value<double>(q, ref, U0, 5)));
  }
  const double G = 4.0 / (h * h), trG = 3.0 * G, GG = 3.0 * G * G;
  for (int a = 0; a < 27; ++a)
    for (int f = 0; f < 4; ++f) r[a][f] = S(0.0);
  bool ok = true;
  for (int gk = 0; gk < 3; ++gk)
    for (int gj = 0; gj < 3; ++gj)
      for (int gi = 0; gi < 3; ++gi) {
        const double u[3] = {kGq[gi], kGq[gj], kGq[gk]};
        const double wdet = kGw[gi] * kGw[gj] * kGw[gk] * h * h * h;
        Q2Pt Q;
        q2_point(u, h, Q);
        S ph1 = 0.0, gph1[3], gpht[3], Hpht[3][3], gmut[3], vv[3], dv[3], gvt[3][3], lvt[3], pt = 0.0, gpt[3];
        for (int i = 0; i < 3; ++i) {
          gph1[i] = gpht[i] = gmut[i] = vv[i] = dv[i] = lvt[i] = gpt[i] = S(0.0);
          for (int j = 0; j < 3; ++j) Hpht[i][j] = gvt[i][j] = S(0.0);
        }
        for (int a = 0; a < 27; ++a) {
          ph1 += Q.N[a] * phi1[a];
          pt += Q.N[a] * ptn[a];
          const double lap = Q.d2N[a][0][0] + Q.d2N[a][1][1] + Q.d2N[a][2][2];
          for (int i = 0; i < 3; ++i) {
            gph1[i] += Q.dN[a][i] * phi1[a];
            gpht[i] += Q.dN[a][i] * phit[a];
            gmut[i] += Q.dN[a][i] * mut[a];
            gpt[i] += Q.dN[a][i] * ptn[a];
            vv[i] += Q.N[a] * vt[a][i];
            dv[i] += Q.N[a] * dvn[a][i];
            lvt[i] += lap * vt[a][i];
            for (int j = 0; j < 3; ++j) {
              Hpht[i][j] += Q.d2N[a][i][j] * phit[a];
              gvt[i][j] += Q.dN[a][j] * vt[a][i];  // dv~_i/dx_j
            }
          }
        }
        const S ps = pull2(ph1);
        const S rho = alpha * ps + beta, eta = gamma * ps + xi;
        S geta[3], J[3];
        for (int d = 0; d < 3; ++d) {
          geta[d] = std::fabs(val2(ph1)) <= 1.0 ? gamma * gph1[d] : S(0.0);
          J[d] = kap * gmut[d];
        }
        const S lpht = Hpht[0][0] + Hpht[1][1] + Hpht[2][2];
        S Rm[3];
        for (int i = 0; i < 3; ++i) {
          S t = rho * dv[i] / p.dt;
          for (int j = 0; j < 3; ++j) t += rho * vv[j] * gvt[i][j];
          for (int j = 0; j < 3; ++j) t += (1.0 / p.Pe) * J[j] * gvt[i][j];
          S cap = gpht[i] * lpht;
          for (int j = 0; j < 3; ++j) cap += gpht[j] * Hpht[i][j];
          t += (p.Cn / p.We) * cap;
          t += (1.0 / p.We) * gpt[i];
          S visc = eta * lvt[i];
          for (int k = 0; k < 3; ++k) visc += geta[k] * gvt[i][k];
          t -= (1.0 / p.Re) * visc;
          t -= rho * p.g[i] / p.Fr;
          Rm[i] = t;
        }
        const S Rc = gvt[0][0] + gvt[1][1] + gvt[2][2];
        const S vGv = G * (vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
        const S vGJ = G * (vv[0] * J[0] + vv[1] * J[1] + vv[2] * J[2]);
        const S nu = eta / (rho * p.Re);
        const S bracket = 4.0 / (p.dt * p.dt) + vGv + (1.0 / (rho * p.Pe)) * vGJ + p.C_I * nu * nu * GG;
        if (!(val2(bracket) > 0.0)) {
          ok = false;
          continue;
        }
        const S tau_m = rsqrt2(bracket);
        const S tau_c = 1.0 / (trG * tau_m);
        for (int a = 0; a < 27; ++a) {
          const double Na = Q.N[a];
          const double* dNa = Q.dN[a];
          for (int i = 0; i < 3; ++i) {
            S t = Na * rho * dv[i] / p.dt;
            for (int j = 0; j < 3; ++j) t += Na * rho * vv[j] * gvt[i][j];
            for (int j = 0; j < 3; ++j) t -= Na * tau_m * Rm[j] * gvt[i][j];
            for (int j = 0; j < 3; ++j) t += dNa[j] * vv[j] * tau_m * Rm[i];
            for (int j = 0; j < 3; ++j) t -= dNa[j] * (tau_m * tau_m / rho) * Rm[j] * Rm[i];
            for (int j = 0; j < 3; ++j) t += (1.0 / p.Pe) * Na * J[j] * gvt[i][j];
            for (int j = 0; j < 3; ++j) t += (1.0 / p.Pe) * dNa[j] * J[j] * (tau_m / rho) * Rm[i];
            for (int j = 0; j < 3; ++j) t -= (p.Cn / p.We) * dNa[j] * gpht[i] * gpht[j];
            t -= (1.0 / p.We) * dNa[i] * pt;
            t += (1.0 / p.We) * dNa[i] * rho * tau_c * Rc;
            for (int k = 0; k < 3; ++k) t += (1.0 / p.Re) * dNa[k] * eta * gvt[i][k];
            t -= Na * rho * p.g[i] / p.Fr;
            r[a][i] += wdet * t;
          }
          S tq = Na * Rc;
          for (int i = 0; i < 3; ++i) tq += dNa[i] * (tau_m / rho) * Rm[i];
          r[a][3] += wdet * tq;
        }
      }
  return ok;
}

// Element vectors of the block assembled through the transpose of the
// constraint rows; NS boundary rows as in the cG(1) oracle (velocity rows of
// boundary nodes read v^{k+1} - v^k, the pinned node's pressure row p^{k+1} -
// p^k; for the JVP the identity on those rows).
template <class S>
bool assemble_q2(const Mesh& m, const MeshQ2& q, const Params& p, int block, const S* U1, const double* U0,
                 S* R) {
  const int f0 = block == BLOCK_CH ? 0 : 2, nf = block == BLOCK_CH ? 2 : 4;
  bool ok = true;
  for (size_t e = 0; e < m.leaves.size(); ++e) {
    S r[27][4];
    if (block == BLOCK_CH) {
      S rc[27][2];
      ch_element_q2<S>(m, q, p, e, U1, U0, rc);
      for (int a = 0; a < 27; ++a) r[a][0] = rc[a][0], r[a][1] = rc[a][1];
    } else if (!ns_element_q2<S>(m, q, p, e, U1, U0, r)) {
      ok = false;
    }
    for (int a = 0; a < 27; ++a) {
      const int32_t ref = q.elem[e][a];
      if (ref >= 0) {
        for (int f = 0; f < nf; ++f) R[(size_t)ref * 6 + f0 + f] += r[a][f];
      } else {
        const int32_t h = -1 - ref;
        for (int64_t t = q.hang_off[h]; t < q.hang_off[h + 1]; ++t)
          for (int f = 0; f < nf; ++f) R[(size_t)q.hang_ids[t] * 6 + f0 + f] += q.hang_w[t] * r[a][f];
      }
    }
  }
  return ok;
}

}  // namespace

std::string residual_q2(const Mesh& m, const MeshQ2& q, const Params& p, int block, const double* Unew,
                        const double* Uold, double* R) {
  if (q.elem.size() != m.leaves.size()) return "Q2 numbering does not belong to this mesh";
  if (block != BLOCK_CH && block != BLOCK_NS) return "unknown block";
  const size_t n = q.nodes.size();
  std::fill(R, R + n * 6, 0.0);
  if (!assemble_q2<double>(m, q, p, block, Unew, Uold, R)) return "tau_m bracket is not positive";
  if (block == BLOCK_NS)
    for (size_t i = 0; i < n; ++i) {
      if (q.bflags[i] & 1)
        for (int d = 0; d < 3; ++d) R[i * 6 + 2 + d] = Unew[i * 6 + 2 + d] - Uold[i * 6 + 2 + d];
      if (q.bflags[i] & 2) R[i * 6 + 5] = Unew[i * 6 + 5] - Uold[i * 6 + 5];
    }
  return "";
}

std::string jvp_q2(const Mesh& m, const MeshQ2& q, const Params& p, int block, const double* Unew,
                   const double* Uold, const double* dU, double* JdU) {
  if (q.elem.size() != m.leaves.size()) return "Q2 numbering does not belong to this mesh";
  if (block != BLOCK_CH && block != BLOCK_NS) return "unknown block";
  const int f0 = block == BLOCK_CH ? 0 : 2, f1 = block == BLOCK_CH ? 2 : 6;
  const size_t n = q.nodes.size();
  std::vector<D2> U1(n * 6), R(n * 6);
  for (size_t i = 0; i < n * 6; ++i) {
    const int f = (int)(i % 6);
    U1[i] = D2(Unew[i], (f >= f0 && f < f1) ? dU[i] : 0.0);  // the block's own unknowns
  }
  if (!assemble_q2<D2>(m, q, p, block, U1.data(), Uold, R.data())) return "tau_m bracket is not positive";
  for (size_t i = 0; i < n * 6; ++i) {
    const int f = (int)(i % 6);
    JdU[i] = (f >= f0 && f < f1) ? R[i].d : 0.0;
  }
  if (block == BLOCK_NS)
    for (size_t i = 0; i < n; ++i) {
      if (q.bflags[i] & 1)
        for (int d = 0; d < 3; ++d) JdU[i * 6 + 2 + d] = dU[i * 6 + 2 + d];
      if (q.bflags[i] & 2) JdU[i * 6 + 5] = dU[i * 6 + 5];
    }
  return "";
}

}  // namespace orc
