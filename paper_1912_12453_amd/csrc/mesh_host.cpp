// Host construction of the balanced octree mesh (Sec. 4): top-down
// refinement, 2:1 balance, node numbering and flattened hanging-node
// constraints.  Everything here is integer work over sorted Morton-key arrays.
//
// Balance works level by level from the finest level down: the set A_l of
// octants of level l present in the final tree (leaves and interior) forces,
// at level l-1, every parent of A_l and all 26 neighbours of those parents
// (a leaf of level l may only touch leaves of level >= l-1), closed under
// siblings.  Octants of A_l that are parents of A_{l+1} are interior; the
// rest are leaves.  This gives the coarsest 2:1-balanced refinement.
//
// Hanging nodes: a leaf corner P is a vertex of exactly one leaf in each
// in-domain octant around it unless it lies inside an edge or a face of a
// coarser leaf, so P hangs iff its corner multiplicity is below the number of
// in-domain octants around it.  Under 2:1 balance a hanging P sits at the
// midpoint of an edge or a face of side s = 2^(D - lambda(P) + 1), lambda(P)
// being the coarsest level whose grid contains P; its parents are P +- s/2
// along the axes where P is off that grid.
#include <algorithm>
#include <cmath>
#include <functional>
#include <thread>
#include <unordered_map>

#include "internal.hpp"

namespace chns {

namespace {

void psort(std::vector<uint64_t>& v) {
  const size_t n = v.size();
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < (1u << 20) || nt == 1) {
    std::sort(v.begin(), v.end());
    return;
  }
  std::vector<size_t> cut(nt + 1);
  for (unsigned t = 0; t <= nt; ++t) cut[t] = n * t / nt;
  {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
      th.emplace_back([&, t] { std::sort(v.begin() + cut[t], v.begin() + cut[t + 1]); });
    for (auto& x : th) x.join();
  }
  for (unsigned w = 1; w < nt; w *= 2) {
    std::vector<std::thread> th;
    for (unsigned t = 0; t + w < nt; t += 2 * w) {
      size_t a = cut[t], b = cut[t + w], c = cut[std::min(nt, t + 2 * w)];
      th.emplace_back([&v, a, b, c] {
        std::inplace_merge(v.begin() + a, v.begin() + b, v.begin() + c);
      });
    }
    for (auto& x : th) x.join();
  }
}

void sort_unique(std::vector<uint64_t>& v) {
  psort(v);
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

struct Geo {
  int D;
  uint32_t ext[3];
  uint32_t size(int level) const { return 1u << (D - level); }
  // Morton stride of one child digit at level l (children of a level-l octant)
  uint64_t child_stride(int l) const { return 1ULL << (3 * (D - l - 1)); }
  uint64_t parent_mask(int l) const {  // clears the digits finer than level l-1
    return ~((1ULL << (3 * (D - l + 1))) - 1);
  }
};

std::string refine(const chns_mesh_spec& s, const Geo& g, std::vector<std::vector<uint64_t>>& init) {
  std::vector<uint64_t> cur;
  for (int k = 0; k < s.trees[2]; ++k)
    for (int j = 0; j < s.trees[1]; ++j)
      for (int i = 0; i < s.trees[0]; ++i)
        cur.push_back(mkey((uint32_t)i << g.D, (uint32_t)j << g.D, (uint32_t)k << g.D));
  std::sort(cur.begin(), cur.end());
  const double unit = std::ldexp(1.0, -g.D);
  for (int l = 0; l < g.D && !cur.empty(); ++l) {
    std::vector<uint8_t> split(cur.size(), 0);
    if (l < s.level_min) {
      std::fill(split.begin(), split.end(), 1);
    } else if (s.phi0) {
      const uint32_t sz = g.size(l);
      std::vector<double> pts(cur.size() * 27), val(cur.size() * 9);
      for (size_t o = 0; o < cur.size(); ++o) {
        uint32_t x, y, z;
        unkey(cur[o], x, y, z);
        double* p = &pts[o * 27];
        for (int c = 0; c < 8; ++c) {
          p[3 * c + 0] = (double)(x + ((c & 1) ? sz : 0)) * unit;
          p[3 * c + 1] = (double)(y + ((c & 2) ? sz : 0)) * unit;
          p[3 * c + 2] = (double)(z + ((c & 4) ? sz : 0)) * unit;
        }
        p[24] = (double)(x + sz / 2) * unit;
        p[25] = (double)(y + sz / 2) * unit;
        p[26] = (double)(z + sz / 2) * unit;
      }
      s.phi0(pts.data(), (int64_t)cur.size() * 9, val.data(), s.user);
      for (size_t o = 0; o < cur.size(); ++o) {
        const double* v = &val[o * 9];
        double lo = v[0], hi = v[0], amin = std::fabs(v[0]);
        for (int c = 1; c < 9; ++c) {
          lo = std::min(lo, v[c]);
          hi = std::max(hi, v[c]);
          amin = std::min(amin, std::fabs(v[c]));
        }
        split[o] = (amin < s.band || (lo < 0.0 && hi > 0.0)) ? 1 : 0;
      }
    }
    std::vector<uint64_t> next;
    const uint64_t cs = g.child_stride(l);
    for (size_t o = 0; o < cur.size(); ++o) {
      if (!split[o]) {
        init[l].push_back(cur[o]);
        continue;
      }
      for (uint64_t c = 0; c < 8; ++c) next.push_back(cur[o] + c * cs);
    }
    cur.swap(next);
  }
  for (uint64_t k : cur) init[g.D].push_back(k);
  return "";
}

std::string load_leaves(const chns_mesh_spec& s, const Geo& g, std::vector<std::vector<uint64_t>>& init) {
  std::vector<std::pair<uint64_t, uint64_t>> ranges;  // [key, key + size^3)
  ranges.reserve((size_t)s.n_leaves);
  long double vol = 0;
  for (int64_t i = 0; i < s.n_leaves; ++i) {
    const int32_t* q = s.leaves + 4 * i;
    if (q[3] < 0 || q[3] > g.D) return "leaf level out of range";
    uint32_t sz = g.size(q[3]);
    if (q[0] < 0 || q[1] < 0 || q[2] < 0) return "negative leaf coordinate";
    uint32_t x = (uint32_t)q[0], y = (uint32_t)q[1], z = (uint32_t)q[2];
    if ((x | y | z) & (sz - 1)) return "leaf not aligned to its size";
    if (x + sz > g.ext[0] || y + sz > g.ext[1] || z + sz > g.ext[2]) return "leaf outside the domain";
    uint64_t k = mkey(x, y, z);
    ranges.push_back({k, k + (uint64_t)sz * sz * sz});
    init[q[3]].push_back(k);
    vol += (long double)sz * sz * sz;
  }
  if (vol != (long double)g.ext[0] * g.ext[1] * g.ext[2]) return "leaves do not tile the domain";
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second) return "leaves overlap";
  return "";
}

// 26 neighbours (in the domain) of every key of P at level l, plus P itself
void with_neighbours(const Geo& g, int l, const std::vector<uint64_t>& P, std::vector<uint64_t>& out) {
  const int64_t s = g.size(l);
  out.reserve(out.size() + P.size() * 27);
  for (uint64_t k : P) {
    uint32_t x, y, z;
    unkey(k, x, y, z);
    for (int dz = -1; dz <= 1; ++dz) {
      int64_t nz = (int64_t)z + dz * s;
      if (nz < 0 || nz >= (int64_t)g.ext[2]) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        int64_t ny = (int64_t)y + dy * s;
        if (ny < 0 || ny >= (int64_t)g.ext[1]) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          int64_t nx = (int64_t)x + dx * s;
          if (nx < 0 || nx >= (int64_t)g.ext[0]) continue;
          out.push_back(mkey((uint32_t)nx, (uint32_t)ny, (uint32_t)nz));
        }
      }
    }
  }
}

// Balanced leaves per level (keys sorted within each level).
void balance(const Geo& g, const std::vector<std::vector<uint64_t>>& init,
             std::vector<std::vector<uint64_t>>& leaves) {
  const int D = g.D;
  std::vector<std::vector<uint64_t>> A(D + 1), interior(D + 1);
  A[D] = init[D];
  sort_unique(A[D]);
  for (int l = D; l >= 1; --l) {
    std::vector<uint64_t> P;
    P.reserve(A[l].size() / 8 + 1);
    const uint64_t pm = g.parent_mask(l);
    for (uint64_t k : A[l]) P.push_back(k & pm);
    sort_unique(P);
    interior[l - 1] = P;
    std::vector<uint64_t> cand;
    with_neighbours(g, l - 1, P, cand);
    cand.insert(cand.end(), init[l - 1].begin(), init[l - 1].end());
    if (l - 1 == 0) {
      sort_unique(cand);
      A[0] = cand;
      continue;
    }
    // sibling closure: all 8 children of the parents (level l-2) of cand
    const uint64_t pm2 = g.parent_mask(l - 1);
    for (auto& k : cand) k &= pm2;
    sort_unique(cand);
    const uint64_t cs = g.child_stride(l - 2);
    std::vector<uint64_t> full;
    full.reserve(cand.size() * 8);
    for (uint64_t k : cand)
      for (uint64_t c = 0; c < 8; ++c) full.push_back(k + c * cs);
    A[l - 1].swap(full);  // already sorted and unique
  }
  leaves.assign(D + 1, {});
  for (int l = 0; l <= D; ++l) {
    const auto& in = interior[l];
    for (uint64_t k : A[l])
      if (!std::binary_search(in.begin(), in.end(), k)) leaves[l].push_back(k);
  }
}

}  // namespace

std::string build_host_mesh(const chns_mesh_spec& s, HostMesh& M) {
  for (int d = 0; d < 3; ++d)
    if (s.trees[d] < 1 || s.trees[d] > 64) return "tree counts must be in [1, 64]";
  if (s.level_max < 0 || s.level_max > 16) return "level_max must be in [0, 16]";
  if (!s.leaves && (s.level_min < 0 || s.level_min > s.level_max))
    return "need 0 <= level_min <= level_max";
  if (s.leaves && s.n_leaves <= 0) return "n_leaves must be positive";
  Geo g;
  g.D = s.level_max;
  for (int d = 0; d < 3; ++d) {
    g.ext[d] = (uint32_t)s.trees[d] << g.D;
    // node coordinates reach ext; keys carry a 5-bit level tag below 59 bits
    if (g.ext[d] >= (1u << 19)) return "trees * 2^level_max must stay below 2^19 per axis";
  }
  M = HostMesh();
  for (int d = 0; d < 3; ++d) M.T[d] = s.trees[d];
  M.D = g.D;

  std::vector<std::vector<uint64_t>> init(g.D + 1), lv;
  std::string err = s.leaves ? load_leaves(s, g, init) : refine(s, g, init);
  if (!err.empty()) return err;
  balance(g, init, lv);

  // leaves in Morton order (anchors are unique across levels)
  {
    std::vector<uint64_t> tagged;  // key * 32 + level keeps the level with the key
    size_t n = 0;
    for (auto& v : lv) n += v.size();
    tagged.reserve(n);
    for (int l = 0; l <= g.D; ++l)
      for (uint64_t k : lv[l]) tagged.push_back((k << 5) | (uint64_t)l);
    psort(tagged);
    M.leaf_key.resize(n);
    M.leaf_level.resize(n);
    for (size_t i = 0; i < n; ++i) {
      M.leaf_key[i] = tagged[i] >> 5;
      M.leaf_level[i] = (uint8_t)(tagged[i] & 31);
    }
  }
  const size_t E = M.leaf_key.size();

  // corner keys with multiplicity
  std::vector<uint64_t> corners(E * 8);
  for (size_t e = 0; e < E; ++e) {
    uint32_t x, y, z;
    unkey(M.leaf_key[e], x, y, z);
    uint32_t sz = g.size(M.leaf_level[e]);
    for (int c = 0; c < 8; ++c)
      corners[e * 8 + c] = mkey(x + ((c & 1) ? sz : 0), y + ((c & 2) ? sz : 0), z + ((c & 4) ? sz : 0));
  }
  std::vector<uint64_t> sorted = corners;
  psort(sorted);
  std::vector<uint64_t> all_keys;
  all_keys.reserve(sorted.size() / 4);
  for (size_t i = 0; i < sorted.size();) {
    size_t j = i;
    while (j < sorted.size() && sorted[j] == sorted[i]) ++j;
    uint64_t k = sorted[i];
    uint32_t P[3];
    unkey(k, P[0], P[1], P[2]);
    int expected = 1;
    for (int d = 0; d < 3; ++d) expected *= (P[d] == 0 || P[d] == g.ext[d]) ? 1 : 2;
    if ((int)(j - i) == expected)
      M.node_key.push_back(k);
    else
      M.hang_key.push_back(k);
    all_keys.push_back(k);
    i = j;
  }
  { std::vector<uint64_t>().swap(sorted); }

  auto node_id = [&](uint64_t k) -> int64_t {
    auto it = std::lower_bound(M.node_key.begin(), M.node_key.end(), k);
    return (it != M.node_key.end() && *it == k) ? (int64_t)(it - M.node_key.begin()) : -1;
  };
  auto hang_id = [&](uint64_t k) -> int64_t {
    auto it = std::lower_bound(M.hang_key.begin(), M.hang_key.end(), k);
    return (it != M.hang_key.end() && *it == k) ? (int64_t)(it - M.hang_key.begin()) : -1;
  };

  // constraints: direct parents, then recursive substitution (memoised)
  const size_t NH = M.hang_key.size();
  std::vector<std::vector<std::pair<int64_t, double>>> flat(NH);
  std::vector<uint8_t> state(NH, 0);  // 0 todo, 1 in progress, 2 done
  std::string cerr;
  std::function<void(size_t)> resolve = [&](size_t h) {
    if (state[h] == 2) return;
    if (state[h] == 1) {
      cerr = "cyclic hanging-node constraint";
      return;
    }
    state[h] = 1;
    uint32_t P[3];
    unkey(M.hang_key[h], P[0], P[1], P[2]);
    int lam = 0;  // coarsest level whose grid holds P
    for (; lam <= g.D; ++lam) {
      uint32_t sz = g.size(lam);
      if (P[0] % sz == 0 && P[1] % sz == 0 && P[2] % sz == 0) break;
    }
    if (lam == 0 || lam > g.D) {
      cerr = "hanging node on the coarsest grid";
      state[h] = 2;
      return;
    }
    const uint32_t half = g.size(lam);  // s/2 of the constraining edge/face
    int fr[3], nfr = 0;
    for (int d = 0; d < 3; ++d)
      if (P[d] % (2 * half) != 0) fr[nfr++] = d;
    if (nfr < 1 || nfr > 2) {
      cerr = "hanging node is neither an edge midpoint nor a face centre";
      state[h] = 2;
      return;
    }
    const double w = nfr == 1 ? 0.5 : 0.25;
    std::vector<std::pair<int64_t, double>> acc;
    for (int m = 0; m < (1 << nfr); ++m) {
      uint32_t Q[3] = {P[0], P[1], P[2]};
      for (int t = 0; t < nfr; ++t) Q[fr[t]] = ((m >> t) & 1) ? P[fr[t]] + half : P[fr[t]] - half;
      uint64_t qk = mkey(Q[0], Q[1], Q[2]);
      int64_t id = node_id(qk);
      if (id >= 0) {
        acc.push_back({id, w});
        continue;
      }
      int64_t hq = hang_id(qk);
      if (hq < 0) {
        cerr = "constraint parent is not a mesh node (tree not 2:1 balanced)";
        state[h] = 2;
        return;
      }
      resolve((size_t)hq);
      for (auto& t : flat[hq]) acc.push_back({t.first, w * t.second});
    }
    std::sort(acc.begin(), acc.end());
    std::vector<std::pair<int64_t, double>> merged;
    for (auto& t : acc) {
      if (!merged.empty() && merged.back().first == t.first)
        merged.back().second += t.second;
      else
        merged.push_back(t);
    }
    flat[h].swap(merged);
    state[h] = 2;
  };
  for (size_t h = 0; h < NH && cerr.empty(); ++h) resolve(h);
  if (!cerr.empty()) return cerr;
  M.hang_off.assign(NH + 1, 0);
  for (size_t h = 0; h < NH; ++h) {
    M.hang_off[h + 1] = M.hang_off[h] + (int32_t)flat[h].size();
    M.max_fanin = std::max(M.max_fanin, (int)flat[h].size());
    for (auto& t : flat[h]) {
      M.hang_ids.push_back((int32_t)t.first);
      M.hang_w.push_back(t.second);
    }
  }

  // element table
  M.elem.resize(E * 8);
  for (size_t i = 0; i < E * 8; ++i) {
    int64_t id = node_id(corners[i]);
    M.elem[i] = id >= 0 ? (int32_t)id : (int32_t)(-1 - hang_id(corners[i]));
  }

  // boundary flags: bit0 on the boundary, bit1 the pressure pin (first node)
  M.bflags.assign(M.node_key.size(), 0);
  for (size_t i = 0; i < M.node_key.size(); ++i) {
    uint32_t P[3];
    unkey(M.node_key[i], P[0], P[1], P[2]);
    for (int d = 0; d < 3; ++d)
      if (P[d] == 0 || P[d] == g.ext[d]) M.bflags[i] = 1;
  }
  if (!M.bflags.empty()) M.bflags[0] |= 2;
  if (M.node_key.size() > (size_t)INT32_MAX / 8) return "mesh too large for 32-bit node ids";
  return "";
}

}  // namespace chns

namespace chns {

std::string build_scatter_plan(const HostMesh& m, ScatterPlan& P) {
  const int64_t E = (int64_t)m.leaf_key.size(), n = (int64_t)m.node_key.size();
  const int64_t C = (E + kChunk - 1) / kChunk;
  P = ScatterPlan();
  P.tgt_off.assign(C + 1, 0);
  P.inc_off.push_back(0);
  std::vector<std::pair<int64_t, int64_t>> ent;  // (node, corner slot)
  std::vector<float> entw;
  std::vector<std::pair<std::pair<int64_t, int64_t>, float>> tmp;
  for (int64_t c = 0; c < C; ++c) {
    tmp.clear();
    const int64_t e0 = c * kChunk, e1 = std::min(E, e0 + kChunk);
    for (int64_t e = e0; e < e1; ++e)
      for (int k = 0; k < 8; ++k) {
        const int64_t slot = (e - e0) * 8 + k;
        const int32_t r = m.elem[e * 8 + k];
        if (r >= 0) {
          tmp.push_back({{r, slot}, 1.0f});
        } else {
          const int32_t h = -1 - r;
          for (int32_t t = m.hang_off[h]; t < m.hang_off[h + 1]; ++t)
            tmp.push_back({{m.hang_ids[t], slot}, (float)m.hang_w[t]});
        }
      }
    std::sort(tmp.begin(), tmp.end(),
              [](const auto& a, const auto& b) { return a.first < b.first; });
    int ntg = 0;
    for (size_t i = 0; i < tmp.size(); ++i) {
      if (i == 0 || tmp[i].first.first != tmp[i - 1].first.first) {
        if (i) P.inc_off.push_back((int32_t)P.inc_corner.size());
        P.tgt.push_back((int32_t)tmp[i].first.first);
        ++ntg;
      }
      P.inc_corner.push_back((uint8_t)tmp[i].first.second);
      P.inc_w.push_back(tmp[i].second);
    }
    if (!tmp.empty()) P.inc_off.push_back((int32_t)P.inc_corner.size());
    P.tgt_off[c + 1] = P.tgt_off[c] + ntg;
    // corner map: positions in this chunk's (sorted) target list
    const int32_t* tb = P.tgt.data() + P.tgt_off[c];
    auto pos = [&](int32_t node) {
      return (int32_t)(std::lower_bound(tb, tb + ntg, node) - tb);
    };
    for (int64_t e = e0; e < e1; ++e)
      for (int k = 0; k < 8; ++k) {
        const int32_t r = m.elem[e * 8 + k];
        if (r >= 0) {
          P.cmap.push_back(pos(r));
          continue;
        }
        const int32_t h = -1 - r, t0 = m.hang_off[h], np = m.hang_off[h + 1] - t0;
        if (np > 8) return "hanging-node fan-in above 8 is not supported";
        const int64_t j = (int64_t)P.hmap.size() / kHMap;
        if (j >= INT32_MAX) return "scatter plan too large";
        P.cmap.push_back((int32_t)(-1 - j));
        int32_t ent[kHMap] = {t0, np, -1, -1, -1, -1, 0, 0};
        for (int q = 0; q < np; ++q) {
          const uint32_t v = (uint32_t)(uint16_t)pos(m.hang_ids[t0 + q]);
          uint32_t& w = reinterpret_cast<uint32_t&>(ent[2 + q / 2]);
          w = (q & 1) ? ((w & 0xFFFFu) | (v << 16)) : ((w & 0xFFFF0000u) | v);
        }
        P.hmap.insert(P.hmap.end(), ent, ent + kHMap);
      }
    P.max_targets = std::max(P.max_targets, ntg);
    P.max_inc = std::max(P.max_inc, (int)tmp.size());
    if ((int64_t)P.inc_corner.size() > INT32_MAX) return "scatter plan too large";
  }
  P.chunk_inc.resize(C + 1);
  for (int64_t c = 0; c <= C; ++c) P.chunk_inc[c] = P.inc_off[P.tgt_off[c]];
  // node -> slots (counting sort keeps slots ascending)
  const int64_t S = (int64_t)P.tgt.size();
  P.node_off.assign(n + 1, 0);
  for (int64_t s = 0; s < S; ++s) ++P.node_off[P.tgt[s] + 1];
  for (int64_t i = 0; i < n; ++i) P.node_off[i + 1] += P.node_off[i];
  P.node_slot.resize(S);
  {
    std::vector<int32_t> fill(P.node_off.begin(), P.node_off.end() - 1);
    for (int64_t s = 0; s < S; ++s) P.node_slot[fill[P.tgt[s]]++] = (int32_t)s;
  }
  // touched nodes per element, in the order the diagonal kernel visits them
  P.touch_off.assign(E + 1, 0);
  std::vector<int32_t>& touch = P.touch_node;
  touch.reserve(E * 9);
  for (int64_t e = 0; e < E; ++e) {
    const size_t start = touch.size();
    for (int k = 0; k < 8; ++k)
      if (m.elem[e * 8 + k] >= 0) touch.push_back(m.elem[e * 8 + k]);
    for (int k = 0; k < 8; ++k) {
      const int32_t r = m.elem[e * 8 + k];
      if (r >= 0) continue;
      const int32_t h = -1 - r;
      for (int32_t t = m.hang_off[h]; t < m.hang_off[h + 1]; ++t) {
        const int32_t g = m.hang_ids[t];
        bool seen = false;
        for (size_t q = start; q < touch.size(); ++q) seen = seen || touch[q] == g;
        if (!seen) touch.push_back(g);
      }
    }
    P.touch_off[e + 1] = (int64_t)touch.size();
    P.max_touch = std::max(P.max_touch, (int)(touch.size() - start));
  }
  const int64_t T = (int64_t)touch.size();
  P.ntouch_off.assign(n + 1, 0);
  for (int64_t t = 0; t < T; ++t) ++P.ntouch_off[touch[t] + 1];
  for (int64_t i = 0; i < n; ++i) P.ntouch_off[i + 1] += P.ntouch_off[i];
  P.ntouch_slot.resize(T);
  {
    std::vector<int64_t> fill(P.ntouch_off.begin(), P.ntouch_off.end() - 1);
    for (int64_t t = 0; t < T; ++t) P.ntouch_slot[fill[touch[t]]++] = t;
  }
  return "";
}

}  // namespace chns
