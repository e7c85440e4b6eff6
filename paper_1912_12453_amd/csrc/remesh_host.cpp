// Host side of remeshing and of the intergrid transfer between two octree
// meshes of the same brick (Sec. 4, "Remeshing" and "Intergrid transfers").
//
// Evaluation of a nodal field at a point x: find the leaf whose closed cube
// holds x (the leaf that holds the unit cell at floor(x * 2^D), clamped to
// the domain: leaves are a Morton-ordered partition, so it is the last leaf
// anchor at or below that cell's key), take the local coordinates
// xi = (x - anchor) / side in [0,1]^3, and sum the eight trilinear weights
// times the corner values, a hanging corner contributing through its
// constraint.  The field is continuous, so any leaf holding x gives the same
// value.  Points on a dyadic grid give dyadic weights, exact in FP64.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.hpp"

namespace chns {

namespace {

// Appends (node, weight) of mesh m at point x (physical coordinates) to acc.
bool weights_at(const HostMesh& m, const double x[3], std::vector<std::pair<int32_t, double>>& acc) {
  const double scale = std::ldexp(1.0, m.D);
  uint32_t q[3];
  uint32_t ext[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = (uint32_t)m.T[d] << m.D;
    double c = std::floor(x[d] * scale);
    if (c < 0) c = 0;
    if (c > (double)(ext[d] - 1)) c = (double)(ext[d] - 1);
    q[d] = (uint32_t)c;
  }
  const uint64_t kq = mkey(q[0], q[1], q[2]);
  auto it = std::upper_bound(m.leaf_key.begin(), m.leaf_key.end(), kq);
  if (it == m.leaf_key.begin()) return false;
  const size_t e = (size_t)(it - m.leaf_key.begin()) - 1;
  uint32_t a[3];
  unkey(m.leaf_key[e], a[0], a[1], a[2]);
  const uint32_t side = 1u << (m.D - m.leaf_level[e]);
  double xi[3];
  for (int d = 0; d < 3; ++d) {
    if (q[d] < a[d] || q[d] >= a[d] + side) return false;
    xi[d] = (x[d] * scale - (double)a[d]) / (double)side;
    if (xi[d] < 0) xi[d] = 0;
    if (xi[d] > 1) xi[d] = 1;
  }
  for (int k = 0; k < 8; ++k) {
    const double w = ((k & 1) ? xi[0] : 1 - xi[0]) * ((k & 2) ? xi[1] : 1 - xi[1]) * ((k & 4) ? xi[2] : 1 - xi[2]);
    if (w == 0.0) continue;
    const int32_t ref = m.elem[e * 8 + k];
    if (ref >= 0) {
      acc.push_back({ref, w});
    } else {
      const int h = -1 - ref;
      for (int j = m.hang_off[h]; j < m.hang_off[h + 1]; ++j) acc.push_back({m.hang_ids[j], w * m.hang_w[j]});
    }
  }
  return true;
}

void merge_sorted(std::vector<std::pair<int32_t, double>>& acc, std::vector<int32_t>& idx, std::vector<double>& w) {
  std::sort(acc.begin(), acc.end(),
            [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) { return a.first < b.first; });
  for (size_t j = 0; j < acc.size();) {
    double s = 0;
    size_t k = j;
    for (; k < acc.size() && acc[k].first == acc[j].first; ++k) s += acc[k].second;
    idx.push_back(acc[j].first);
    w.push_back(s);
    j = k;
  }
}

struct FieldOnMesh {
  const HostMesh* m;
  const double* U;  // n * 6, node-major
  int field;
  std::string err;
};

// phi0 callback of the remeshing build: the old trilinear field at the points
void eval_field(const double* xyz, int64_t n, double* out, void* user) {
  FieldOnMesh* F = (FieldOnMesh*)user;
  std::vector<std::pair<int32_t, double>> acc;
  for (int64_t i = 0; i < n; ++i) {
    acc.clear();
    if (!weights_at(*F->m, xyz + 3 * i, acc)) {
      F->err = "a sample point lies outside the old mesh";
      out[i] = 0;
      continue;
    }
    // weights merged per node (exact: they are dyadic), then summed in
    // ascending node order, as the transfer applies them
    std::vector<int32_t> ids;
    std::vector<double> ws;
    merge_sorted(acc, ids, ws);
    double s = 0;
    for (size_t k = 0; k < ids.size(); ++k) s += ws[k] * F->U[(int64_t)ids[k] * 6 + F->field];
    out[i] = s;
  }
}

}  // namespace

std::string build_interp(const HostMesh& from, const HostMesh& to, std::vector<int32_t>& off,
                         std::vector<int32_t>& idx, std::vector<double>& w) {
  for (int d = 0; d < 3; ++d)
    if (from.T[d] != to.T[d]) return "the meshes cover different domains";
  const size_t n = to.node_key.size();
  off.assign(n + 1, 0);
  idx.clear();
  w.clear();
  const double unit = std::ldexp(1.0, -to.D);
  std::vector<std::pair<int32_t, double>> acc;
  for (size_t i = 0; i < n; ++i) {
    uint32_t p[3];
    unkey(to.node_key[i], p[0], p[1], p[2]);
    const double x[3] = {p[0] * unit, p[1] * unit, p[2] * unit};
    acc.clear();
    if (!weights_at(from, x, acc)) return "a node lies outside the source mesh";
    merge_sorted(acc, idx, w);
    off[i + 1] = (int32_t)idx.size();
  }
  return "";
}

std::string remesh_host(const HostMesh& old, const double* U, int level_min, int level_max, double band,
                        HostMesh& out) {
  FieldOnMesh F{&old, U, 0, ""};
  chns_mesh_spec s{};
  for (int d = 0; d < 3; ++d) s.trees[d] = old.T[d];
  s.level_min = level_min;
  s.level_max = level_max;
  s.phi0 = eval_field;
  s.user = &F;
  s.band = band;
  std::string err = build_host_mesh(s, out);
  if (err.empty() && !F.err.empty()) err = F.err;
  return err;
}

}  // namespace chns
