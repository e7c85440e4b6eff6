// Host side of the cG(2) (triquadratic, 27 nodes per leaf) Cahn-Hilliard
// block: node numbering, hanging-node constraints and the fixed-order gather
// plan of the element results.
//
// Lattice points are kept in doubled units 2^-(D+1): leaf (x, y, z, level) of
// side s = 2^(D-level) units has its 3x3x3 lattice at (2x + i s, 2y + j s,
// 2z + k s), local node a = i + 3j + 9k.  A lattice point P hangs when some
// leaf whose closure contains P does not have P on its own lattice (the
// hanging-node rule of Sec. 4, "Handling hanging nodes", applied to the Q2
// lattice).  Its value is the triquadratic interpolant of the coarsest such
// leaf at P; parents that hang are replaced by their own rows.  Independent
// and hanging points are numbered in Morton order of their doubled
// coordinates.
#include <algorithm>
#include <map>

#include "internal.hpp"

namespace chns {

namespace {

// 1D quadratic Lagrange basis with nodes 0, 1, 2 at r in [0, 2] (r in half
// sides); exact for the dyadic r that occur (0, 1/2, 1, 3/2, 2)
double q2_lagrange(int i, double r) {
  switch (i) {
    case 0: return (r - 1.0) * (r - 2.0) * 0.5;
    case 1: return r * (2.0 - r);
    default: return r * (r - 1.0) * 0.5;
  }
}

}  // namespace

std::string build_host_q2(const HostMesh& h, HostQ2& out) {
  out = HostQ2();
  const int64_t E = (int64_t)h.leaf_key.size();
  const int D = h.D;
  if (D + 1 > 20) return "level_max too large for the Q2 lattice";
  if (E * 27 > (int64_t)INT32_MAX) return "too many leaves for the Q2 gather plan";
  std::vector<uint32_t> ax(E), ay(E), az(E);
  std::vector<int64_t> side(E);
  for (int64_t e = 0; e < E; ++e) {
    unkey(h.leaf_key[e], ax[e], ay[e], az[e]);
    side[e] = (int64_t)1 << (D - h.leaf_level[e]);
  }
  // all lattice points, Morton order
  std::vector<uint64_t> pts;
  pts.reserve((size_t)E * 27);
  for (int64_t e = 0; e < E; ++e) {
    const int64_t s = side[e];
    for (int a = 0; a < 27; ++a)
      pts.push_back(mkey((uint32_t)(2 * ax[e] + (a % 3) * s), (uint32_t)(2 * ay[e] + (a / 3 % 3) * s),
                         (uint32_t)(2 * az[e] + (a / 9) * s)));
  }
  std::sort(pts.begin(), pts.end());
  pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
  const int64_t NP = (int64_t)pts.size();
  auto index_of = [&](uint64_t k) -> int64_t {
    auto it = std::lower_bound(pts.begin(), pts.end(), k);
    return (it != pts.end() && *it == k) ? (int64_t)(it - pts.begin()) : -1;
  };
  // the leaf holding unit cell (cx, cy, cz): the last leaf whose anchor key
  // does not exceed the cell's key (the leaves tile the brick in Morton
  // order), checked for containment
  const int64_t ext[3] = {(int64_t)h.T[0] << D, (int64_t)h.T[1] << D, (int64_t)h.T[2] << D};
  auto cell_leaf = [&](int64_t cx, int64_t cy, int64_t cz) -> int64_t {
    if (cx < 0 || cy < 0 || cz < 0 || cx >= ext[0] || cy >= ext[1] || cz >= ext[2]) return -1;
    const uint64_t k = mkey((uint32_t)cx, (uint32_t)cy, (uint32_t)cz);
    auto it = std::upper_bound(h.leaf_key.begin(), h.leaf_key.end(), k);
    if (it == h.leaf_key.begin()) return -1;
    const int64_t e = (int64_t)(it - h.leaf_key.begin()) - 1;
    const int64_t s = side[e];
    if (cx < ax[e] || cx >= ax[e] + s || cy < ay[e] || cy >= ay[e] + s || cz < az[e] || cz >= az[e] + s)
      return -1;
    return e;
  };
  auto on_lattice = [&](int64_t e, const int64_t P[3]) {
    const int64_t s = side[e];
    const int64_t r[3] = {P[0] - 2 * (int64_t)ax[e], P[1] - 2 * (int64_t)ay[e], P[2] - 2 * (int64_t)az[e]};
    for (int d = 0; d < 3; ++d)
      if (r[d] % s != 0) return false;
    return true;
  };
  // classification
  std::vector<int64_t> owner(NP, -1);  // constraining leaf of a hanging point
  for (int64_t i = 0; i < NP; ++i) {
    uint32_t px, py, pz;
    unkey(pts[i], px, py, pz);
    const int64_t P[3] = {px, py, pz};
    int64_t lo[3], hi[3];  // the unit cells on either side of P along each axis
    for (int d = 0; d < 3; ++d) {
      if (P[d] & 1) {
        lo[d] = hi[d] = (P[d] - 1) / 2;
      } else {
        lo[d] = P[d] / 2 - 1;
        hi[d] = P[d] / 2;
      }
    }
    int64_t best = -1;
    for (int o = 0; o < 8; ++o) {
      const int64_t e = cell_leaf((o & 1) ? hi[0] : lo[0], (o & 2) ? hi[1] : lo[1], (o & 4) ? hi[2] : lo[2]);
      if (e < 0 || on_lattice(e, P)) continue;
      if (best < 0 || side[e] > side[best] || (side[e] == side[best] && e < best)) best = e;
    }
    owner[i] = best;
  }
  std::vector<int32_t> num(NP);  // id for independent points, -1-h for hanging ones
  for (int64_t i = 0; i < NP; ++i) {
    if (owner[i] < 0) {
      num[i] = (int32_t)out.node_key.size();
      out.node_key.push_back(pts[i]);
    } else {
      num[i] = -1 - (int32_t)out.hang_key.size();
      out.hang_key.push_back(pts[i]);
    }
  }
  // constraint rows, parents expanded (memoised, depth-first)
  const int64_t NH = (int64_t)out.hang_key.size();
  std::vector<std::map<int32_t, double>> rows(NH);
  std::vector<char> done(NH, 0), busy(NH, 0);
  std::string err;
  std::vector<int64_t> stack;
  for (int64_t h0 = 0; h0 < NH && err.empty(); ++h0) {
    if (done[h0]) continue;
    stack.push_back(h0);
    while (!stack.empty() && err.empty()) {
      const int64_t hh = stack.back();
      const int64_t i = index_of(out.hang_key[hh]);
      const int64_t e = owner[i];
      uint32_t px, py, pz;
      unkey(pts[i], px, py, pz);
      const int64_t s = side[e];
      const double r[3] = {(double)((int64_t)px - 2 * (int64_t)ax[e]) / (double)s,
                           (double)((int64_t)py - 2 * (int64_t)ay[e]) / (double)s,
                           (double)((int64_t)pz - 2 * (int64_t)az[e]) / (double)s};
      // parents still to expand first
      bool ready = true;
      for (int a = 0; a < 27 && ready; ++a) {
        const double w = q2_lagrange(a % 3, r[0]) * q2_lagrange(a / 3 % 3, r[1]) * q2_lagrange(a / 9, r[2]);
        if (w == 0.0) continue;
        const int64_t j = index_of(mkey((uint32_t)(2 * ax[e] + (a % 3) * s), (uint32_t)(2 * ay[e] + (a / 3 % 3) * s),
                                        (uint32_t)(2 * az[e] + (a / 9) * s)));
        if (j < 0 || j == i) {
          err = "Q2 constraint parent is not a lattice point";
          break;
        }
        if (num[j] < 0 && !done[-1 - num[j]]) {
          const int64_t hp = -1 - num[j];
          if (busy[hp]) {
            err = "cyclic Q2 constraints";
            break;
          }
          busy[hh] = 1;
          stack.push_back(hp);
          ready = false;
        }
      }
      if (!err.empty() || !ready) continue;
      auto& row = rows[hh];
      for (int a = 0; a < 27; ++a) {
        const double w = q2_lagrange(a % 3, r[0]) * q2_lagrange(a / 3 % 3, r[1]) * q2_lagrange(a / 9, r[2]);
        if (w == 0.0) continue;
        const int64_t j = index_of(mkey((uint32_t)(2 * ax[e] + (a % 3) * s), (uint32_t)(2 * ay[e] + (a / 3 % 3) * s),
                                        (uint32_t)(2 * az[e] + (a / 9) * s)));
        if (num[j] >= 0) {
          row[num[j]] += w;
        } else {
          for (auto& pw : rows[-1 - num[j]]) row[pw.first] += w * pw.second;
        }
      }
      done[hh] = 1;
      busy[hh] = 0;
      stack.pop_back();
    }
  }
  if (!err.empty()) return err;
  out.hang_off.assign(1, 0);
  for (int64_t hh = 0; hh < NH; ++hh) {
    for (auto& pw : rows[hh]) {
      if (pw.second == 0.0) continue;
      out.hang_ids.push_back(pw.first);
      out.hang_w.push_back(pw.second);
    }
    out.hang_off.push_back((int32_t)out.hang_ids.size());
  }
  // wall and pressure-pin flags (the cG(1) mesh's rules: a node on the
  // brick's boundary; the Morton-first node)
  out.bflags.assign(out.node_key.size(), 0);
  for (size_t i = 0; i < out.node_key.size(); ++i) {
    uint32_t c[3];
    unkey(out.node_key[i], c[0], c[1], c[2]);
    for (int d = 0; d < 3; ++d)
      if (c[d] == 0 || (int64_t)c[d] == 2 * ext[d]) out.bflags[i] = 1;
  }
  if (!out.bflags.empty()) out.bflags[0] |= 2;
  // connectivity
  out.elem.resize((size_t)E * 27);
  for (int64_t e = 0; e < E; ++e) {
    const int64_t s = side[e];
    for (int a = 0; a < 27; ++a) {
      const int64_t j = index_of(mkey((uint32_t)(2 * ax[e] + (a % 3) * s), (uint32_t)(2 * ay[e] + (a / 3 % 3) * s),
                                      (uint32_t)(2 * az[e] + (a / 9) * s)));
      out.elem[(size_t)e * 27 + a] = num[j];
    }
  }
  // gather plan: per independent node, the element results it sums, in
  // increasing (leaf, local node) order, with their constraint weights
  const int64_t n = (int64_t)out.node_key.size();
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t t = 0; t < E * 27; ++t) {
    const int32_t ref = out.elem[t];
    if (ref >= 0) {
      ++cnt[ref + 1];
    } else {
      for (int32_t k = out.hang_off[-1 - ref]; k < out.hang_off[-ref]; ++k) ++cnt[out.hang_ids[k] + 1];
    }
  }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  out.g_off = cnt;
  out.g_slot.resize((size_t)cnt[n]);
  out.g_w.resize((size_t)cnt[n]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t t = 0; t < E * 27; ++t) {
    const int32_t ref = out.elem[t];
    if (ref >= 0) {
      out.g_slot[fill[ref]] = (int32_t)t;
      out.g_w[fill[ref]++] = 1.0;
    } else {
      for (int32_t k = out.hang_off[-1 - ref]; k < out.hang_off[-ref]; ++k) {
        const int32_t p = out.hang_ids[k];
        out.g_slot[fill[p]] = (int32_t)t;
        out.g_w[fill[p]++] = out.hang_w[k];
      }
    }
  }
  return "";
}

}  // namespace chns
