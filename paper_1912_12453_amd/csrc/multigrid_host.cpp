// Host side of the octree multigrid hierarchy: coarsening of a balanced
// octree and the intergrid transfer between a mesh and its coarsening.
//
// Coarsening merges every sibling group of the finest level D into its
// parent.  Leaf levels only decrease and by at most one, so neighbour level
// differences cannot grow and the coarse tree is 2:1 balanced again; every
// coarse leaf is a leaf of the fine tree or the parent of eight of them, so
// every coarse node (a corner of a coarse leaf) is a fine node, and a coarse
// independent node is a fine independent node (a position hanging in the
// coarse tree stays hanging in the fine tree).
//
// Prolongation P maps coarse nodal values to fine independent nodes by
// evaluating the coarse trilinear field there: the fine node lies in a coarse
// leaf at local coordinates t/S (integers t, S in fine units), the weight of
// corner c is prod_d (c_d ? t_d : S - t_d) / S^3, and hanging corners expand
// through their constraints.  All weights are dyadic, so they are exact in
// binary floating point.  Restriction is P^T, stored as its own CSR so that
// both transfers are gathers.
#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "internal.hpp"

namespace chns {

std::string coarsen_host_mesh(const HostMesh& f, HostMesh& c) {
  if (f.D < 1) return "a mesh of level 0 cannot be coarsened";
  const size_t E = f.leaf_key.size();
  std::vector<int32_t> leaves;
  leaves.reserve(E * 4);
  for (size_t e = 0; e < E; ++e) {
    uint32_t x, y, z;
    unkey(f.leaf_key[e], x, y, z);
    int l = f.leaf_level[e];
    if (l == f.D) {
      if ((x | y | z) & 1) continue;  // the sibling at the parent's anchor stands for all 8
      l = f.D - 1;
    }
    leaves.push_back((int32_t)(x >> 1));
    leaves.push_back((int32_t)(y >> 1));
    leaves.push_back((int32_t)(z >> 1));
    leaves.push_back(l);
  }
  chns_mesh_spec s{};
  for (int d = 0; d < 3; ++d) s.trees[d] = f.T[d];
  s.level_min = 0;
  s.level_max = f.D - 1;
  s.leaves = leaves.data();
  s.n_leaves = (int64_t)(leaves.size() / 4);
  return build_host_mesh(s, c);
}

std::string build_transfer(const HostMesh& f, const HostMesh& c, Transfer& out) {
  if (c.D + 1 != f.D) return "the coarse mesh is not one level coarser";
  for (int d = 0; d < 3; ++d)
    if (c.T[d] != f.T[d]) return "the meshes cover different domains";
  out = Transfer();
  const size_t nf = f.node_key.size(), ncn = c.node_key.size();
  uint32_t ext[3];
  for (int d = 0; d < 3; ++d) ext[d] = (uint32_t)f.T[d] << f.D;
  out.p_off.assign(nf + 1, 0);
  std::vector<std::pair<int32_t, double>> acc;
  for (size_t i = 0; i < nf; ++i) {
    uint32_t p[3];
    unkey(f.node_key[i], p[0], p[1], p[2]);
    // a fine unit cube inside the domain with p as a corner, in coarse units
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) q[d] = (p[d] == ext[d] ? p[d] - 1 : p[d]) >> 1;
    const uint64_t kq = mkey(q[0], q[1], q[2]);
    auto it = std::upper_bound(c.leaf_key.begin(), c.leaf_key.end(), kq);
    if (it == c.leaf_key.begin()) return "fine node outside the coarse mesh";
    const size_t e = (size_t)(it - c.leaf_key.begin()) - 1;
    uint32_t a[3];
    unkey(c.leaf_key[e], a[0], a[1], a[2]);
    const uint32_t sc = 1u << (c.D - c.leaf_level[e]);  // side in coarse units
    int64_t t[3];
    const int64_t S = 2 * (int64_t)sc;                   // side in fine units
    for (int d = 0; d < 3; ++d) {
      if (q[d] < a[d] || q[d] >= a[d] + sc) return "coarse leaf search failed";
      t[d] = (int64_t)p[d] - 2 * (int64_t)a[d];
    }
    const double inv = 1.0 / (double)(S * S * S);
    acc.clear();
    for (int k = 0; k < 8; ++k) {
      const int64_t wx = (k & 1) ? t[0] : S - t[0];
      const int64_t wy = (k & 2) ? t[1] : S - t[1];
      const int64_t wz = (k & 4) ? t[2] : S - t[2];
      const int64_t wi = wx * wy * wz;
      if (wi == 0) continue;
      const double w = (double)wi * inv;
      const int32_t ref = c.elem[e * 8 + k];
      if (ref >= 0) {
        acc.push_back({ref, w});
      } else {
        const int h = -1 - ref;
        for (int j = c.hang_off[h]; j < c.hang_off[h + 1]; ++j) acc.push_back({c.hang_ids[j], w * c.hang_w[j]});
      }
    }
    std::sort(acc.begin(), acc.end(),
              [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) { return x.first < y.first; });
    for (size_t j = 0; j < acc.size();) {
      double w = 0;
      size_t k = j;
      for (; k < acc.size() && acc[k].first == acc[j].first; ++k) w += acc[k].second;
      out.p_idx.push_back(acc[j].first);
      out.p_w.push_back(w);
      j = k;
    }
    out.p_off[i + 1] = (int32_t)out.p_idx.size();
  }
  // restriction = P^T, fine ids ascending per coarse node
  out.r_off.assign(ncn + 1, 0);
  for (int32_t j : out.p_idx) out.r_off[j + 1] += 1;
  for (size_t j = 0; j < ncn; ++j) out.r_off[j + 1] += out.r_off[j];
  out.r_idx.resize(out.p_idx.size());
  out.r_w.resize(out.p_idx.size());
  std::vector<int32_t> fill(out.r_off.begin(), out.r_off.end() - 1);
  for (size_t i = 0; i < nf; ++i)
    for (int k = out.p_off[i]; k < out.p_off[i + 1]; ++k) {
      const int32_t j = out.p_idx[k];
      out.r_idx[fill[j]] = (int32_t)i;
      out.r_w[fill[j]] = out.p_w[k];
      fill[j] += 1;
    }
  // injection: the fine node at each coarse node
  out.inj.resize(ncn);
  for (size_t j = 0; j < ncn; ++j) {
    uint32_t x, y, z;
    unkey(c.node_key[j], x, y, z);
    const uint64_t k = mkey(2 * x, 2 * y, 2 * z);
    auto it = std::lower_bound(f.node_key.begin(), f.node_key.end(), k);
    if (it == f.node_key.end() || *it != k) return "a coarse node is not a fine independent node";
    out.inj[j] = (int32_t)(it - f.node_key.begin());
  }
  return "";
}

}  // namespace chns
