// Oracle octree mesh: refinement, 2:1 balance, nodes, hanging-node
// constraints and boundary flags, each written from its definition.
// TEST INFRASTRUCTURE ONLY (see orc.hpp).
//
// Paper: Sec. 4 "Refinement", "2:1 Balancing", "Meshing" and "Handling
// hanging nodes".  Conventions the paper leaves open are fixed here:
//   * brick of unit trees, level l means side h = 2^-l;
//   * refinement splits an octant below level_max when it is below
//     level_min, or when any of its 9 samples (8 corners + centre) has
//     |phi0| < band, or the samples change sign;
//   * 2:1 balance over the full 26-neighbourhood (face, edge and corner);
//   * Morton order interleaves x in the lowest bit, then y, then z.
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <unordered_map>

#include "orc.hpp"

namespace orc {

uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t k = 0;
  for (int b = 0; b < 21; ++b) {
    k |= (uint64_t)((x >> b) & 1u) << (3 * b);
    k |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
    k |= (uint64_t)((z >> b) & 1u) << (3 * b + 2);
  }
  return k;
}

namespace {

struct Ctx {
  int T[3];
  int D;
  uint32_t ext[3];  // domain extent in integer units
  // leaf set: anchor Morton key -> level.  Leaves never overlap, so their
  // anchors are unique.
  std::unordered_map<uint64_t, int> leaf;

  uint32_t size_of(int level) const { return 1u << (D - level); }
  bool in_domain(int64_t x, int64_t y, int64_t z) const {
    return x >= 0 && y >= 0 && z >= 0 && x < (int64_t)ext[0] && y < (int64_t)ext[1] &&
           z < (int64_t)ext[2];
  }
  // The leaf that contains the finest cell with min corner (x,y,z): the
  // octant of some level l, aligned to its size, that is in the leaf set.
  bool locate(uint32_t x, uint32_t y, uint32_t z, Leaf& out) const {
    for (int l = 0; l <= D; ++l) {
      uint32_t s = size_of(l);
      uint32_t ax = x - x % s, ay = y - y % s, az = z - z % s;
      auto it = leaf.find(morton3(ax, ay, az));
      if (it != leaf.end() && it->second == l) {
        out = Leaf{ax, ay, az, l};
        return true;
      }
    }
    return false;
  }
  void split(const Leaf& L) {
    leaf.erase(morton3(L.x, L.y, L.z));
    uint32_t h = size_of(L.level + 1);
    for (int c = 0; c < 8; ++c) {
      uint32_t cx = L.x + ((c & 1) ? h : 0), cy = L.y + ((c & 2) ? h : 0),
               cz = L.z + ((c & 4) ? h : 0);
      leaf[morton3(cx, cy, cz)] = L.level + 1;
    }
  }
};

// Top-down refinement (Sec. 4 "Refinement"), level by level so that the
// indicator can be sampled in one batch per level.
std::string refine(Ctx& C, int lmin, int lmax, Phi0Fn phi0, void* user, double band) {
  std::vector<Leaf> cur;
  for (int k = 0; k < C.T[2]; ++k)
    for (int j = 0; j < C.T[1]; ++j)
      for (int i = 0; i < C.T[0]; ++i)
        cur.push_back(Leaf{(uint32_t)i << C.D, (uint32_t)j << C.D, (uint32_t)k << C.D, 0});
  const double unit = std::ldexp(1.0, -C.D);
  for (int l = 0;; ++l) {
    if (l == lmax) {
      for (auto& L : cur) C.leaf[morton3(L.x, L.y, L.z)] = L.level;
      break;
    }
    std::vector<char> split(cur.size(), 0);
    if (l < lmin) {
      std::fill(split.begin(), split.end(), 1);
    } else if (phi0) {
      std::vector<double> pts(cur.size() * 9 * 3), val(cur.size() * 9);
      uint32_t s = C.size_of(l);
      for (size_t o = 0; o < cur.size(); ++o) {
        for (int c = 0; c < 9; ++c) {
          double px, py, pz;
          if (c < 8) {
            px = (double)(cur[o].x + ((c & 1) ? s : 0)) * unit;
            py = (double)(cur[o].y + ((c & 2) ? s : 0)) * unit;
            pz = (double)(cur[o].z + ((c & 4) ? s : 0)) * unit;
          } else {
            px = (double)(cur[o].x + s / 2) * unit;
            py = (double)(cur[o].y + s / 2) * unit;
            pz = (double)(cur[o].z + s / 2) * unit;
          }
          pts[(o * 9 + c) * 3 + 0] = px;
          pts[(o * 9 + c) * 3 + 1] = py;
          pts[(o * 9 + c) * 3 + 2] = pz;
        }
      }
      phi0(pts.data(), (int64_t)cur.size() * 9, val.data(), user);
      for (size_t o = 0; o < cur.size(); ++o) {
        bool pos = false, neg = false, near = false;
        for (int c = 0; c < 9; ++c) {
          double v = val[o * 9 + c];
          if (std::fabs(v) < band) near = true;
          if (v > 0) pos = true;
          if (v < 0) neg = true;
        }
        split[o] = (near || (pos && neg)) ? 1 : 0;
      }
    }
    std::vector<Leaf> next;
    uint32_t h = C.size_of(l + 1);
    for (size_t o = 0; o < cur.size(); ++o) {
      const Leaf& L = cur[o];
      if (!split[o]) {
        C.leaf[morton3(L.x, L.y, L.z)] = L.level;
        continue;
      }
      for (int c = 0; c < 8; ++c)
        next.push_back(Leaf{L.x + ((c & 1) ? h : 0), L.y + ((c & 2) ? h : 0),
                            L.z + ((c & 4) ? h : 0), l + 1});
    }
    cur.swap(next);
    if (cur.empty()) break;
  }
  return "";
}

std::string load_leaves(Ctx& C, const int32_t* q, int64_t n) {
  // A valid input is a set of aligned octants that tile the domain.
  long double vol = 0;
  std::map<uint64_t, Leaf> sorted;
  for (int64_t i = 0; i < n; ++i) {
    int32_t x = q[4 * i], y = q[4 * i + 1], z = q[4 * i + 2], l = q[4 * i + 3];
    if (l < 0 || l > C.D) return "leaf level out of range";
    uint32_t s = C.size_of(l);
    if (x < 0 || y < 0 || z < 0 || x % s || y % s || z % s) return "leaf not aligned";
    if ((uint32_t)x + s > C.ext[0] || (uint32_t)y + s > C.ext[1] || (uint32_t)z + s > C.ext[2])
      return "leaf outside the domain";
    uint64_t k = morton3(x, y, z);
    if (sorted.count(k)) return "duplicate leaf anchor";
    sorted[k] = Leaf{(uint32_t)x, (uint32_t)y, (uint32_t)z, l};
    vol += (long double)s * s * s;
  }
  long double full = (long double)C.ext[0] * C.ext[1] * C.ext[2];
  if (vol != full) return "leaves do not tile the domain";
  // aligned octants occupy disjoint Morton ranges iff they do not overlap
  uint64_t end = 0;
  bool first = true;
  for (auto& kv : sorted) {
    uint64_t s = C.size_of(kv.second.level);
    if (!first && kv.first < end) return "leaves overlap";
    end = kv.first + s * s * s;
    first = false;
  }
  for (auto& kv : sorted) C.leaf[kv.first] = kv.second.level;
  return "";
}

// 2:1 balance (Sec. 4 "2:1 Balancing"): the coarsest refinement in which any
// two leaves that touch differ by at most one level.  Every split below is
// forced (a coarser neighbour of a leaf two levels finer must be split in any
// balanced refinement), so the result is that unique tree.  Leaves are
// visited from the finest level to the coarsest; leaves created while
// visiting level l are coarser than l and are visited later.
void balance(Ctx& C) {
  for (int l = C.D; l >= 2; --l) {
    std::vector<Leaf> lev;
    for (auto& kv : C.leaf)
      if (kv.second == l) {
        // decode anchor
        uint64_t k = kv.first;
        uint32_t x = 0, y = 0, z = 0;
        for (int b = 0; b < 21; ++b) {
          x |= (uint32_t)((k >> (3 * b)) & 1) << b;
          y |= (uint32_t)((k >> (3 * b + 1)) & 1) << b;
          z |= (uint32_t)((k >> (3 * b + 2)) & 1) << b;
        }
        lev.push_back(Leaf{x, y, z, l});
      }
    uint32_t s = C.size_of(l);
    for (auto& L : lev) {
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (!dx && !dy && !dz) continue;
            int64_t nx = (int64_t)L.x + dx * (int64_t)s, ny = (int64_t)L.y + dy * (int64_t)s,
                    nz = (int64_t)L.z + dz * (int64_t)s;
            if (!C.in_domain(nx, ny, nz)) continue;
            for (;;) {
              Leaf N{};
              C.locate((uint32_t)nx, (uint32_t)ny, (uint32_t)nz, N);
              if (N.level >= l - 1) break;
              C.split(N);
            }
          }
    }
  }
}

struct Constraint {
  std::vector<std::pair<int32_t, double>> terms;  // (independent id, weight)
};

}  // namespace

std::string build_mesh(const int T[3], int level_min, int level_max, Phi0Fn phi0,
                       void* user, double band, const int32_t* leaves, int64_t n_leaves,
                       Mesh& out) {
  Ctx C;
  for (int d = 0; d < 3; ++d) {
    if (T[d] < 1 || T[d] > 64) return "tree counts must be in [1,64]";
    C.T[d] = T[d];
  }
  if (level_max < 0 || level_max > 16) return "level_max must be in [0,16]";
  if (level_min < 0 || level_min > level_max) return "need 0 <= level_min <= level_max";
  C.D = level_max;
  for (int d = 0; d < 3; ++d) C.ext[d] = (uint32_t)T[d] << C.D;
  std::string err = leaves ? load_leaves(C, leaves, n_leaves)
                           : refine(C, level_min, level_max, phi0, user, band);
  if (!err.empty()) return err;
  balance(C);

  // leaves in Morton order
  std::vector<std::pair<uint64_t, int>> kl(C.leaf.begin(), C.leaf.end());
  std::sort(kl.begin(), kl.end());
  out = Mesh();
  for (int d = 0; d < 3; ++d) out.T[d] = T[d];
  out.D = C.D;
  for (auto& p : kl) {
    uint64_t k = p.first;
    uint32_t x = 0, y = 0, z = 0;
    for (int b = 0; b < 21; ++b) {
      x |= (uint32_t)((k >> (3 * b)) & 1) << b;
      y |= (uint32_t)((k >> (3 * b + 1)) & 1) << b;
      z |= (uint32_t)((k >> (3 * b + 2)) & 1) << b;
    }
    out.leaves.push_back(Leaf{x, y, z, p.second});
  }

  // corners of all leaves (node keys)
  std::vector<uint64_t> ck;
  ck.reserve(out.leaves.size() * 8);
  for (auto& L : out.leaves) {
    uint32_t s = C.size_of(L.level);
    for (int c = 0; c < 8; ++c)
      ck.push_back(morton3(L.x + ((c & 1) ? s : 0), L.y + ((c & 2) ? s : 0),
                           L.z + ((c & 4) ? s : 0)));
  }
  std::sort(ck.begin(), ck.end());
  ck.erase(std::unique(ck.begin(), ck.end()), ck.end());

  auto decode = [](uint64_t k, uint32_t& x, uint32_t& y, uint32_t& z) {
    x = y = z = 0;
    for (int b = 0; b < 21; ++b) {
      x |= (uint32_t)((k >> (3 * b)) & 1) << b;
      y |= (uint32_t)((k >> (3 * b + 1)) & 1) << b;
      z |= (uint32_t)((k >> (3 * b + 2)) & 1) << b;
    }
  };

  // Hanging classification (Sec. 4 "Handling hanging nodes"): a corner P
  // hangs iff some leaf whose closure contains P does not have P as a vertex.
  // The leaves whose closure contains P are those holding one of the 8 finest
  // cells around P.  For a hanging P the constraining leaf is the coarsest
  // such leaf (ties: smallest anchor key).
  std::vector<char> hanging(ck.size(), 0);
  std::vector<Leaf> owner(ck.size());
  for (size_t i = 0; i < ck.size(); ++i) {
    uint32_t px, py, pz;
    decode(ck[i], px, py, pz);
    bool have = false;
    Leaf best{};
    for (int o = 0; o < 8; ++o) {
      int64_t cx = (int64_t)px - ((o & 1) ? 0 : 1), cy = (int64_t)py - ((o & 2) ? 0 : 1),
              cz = (int64_t)pz - ((o & 4) ? 0 : 1);
      if (!C.in_domain(cx, cy, cz)) continue;
      Leaf L{};
      C.locate((uint32_t)cx, (uint32_t)cy, (uint32_t)cz, L);
      uint32_t s = C.size_of(L.level);
      bool vx = (px == L.x || px == L.x + s), vy = (py == L.y || py == L.y + s),
           vz = (pz == L.z || pz == L.z + s);
      if (vx && vy && vz) continue;
      if (!have || L.level < best.level ||
          (L.level == best.level && morton3(L.x, L.y, L.z) < morton3(best.x, best.y, best.z))) {
        best = L;
        have = true;
      }
    }
    if (have) {
      hanging[i] = 1;
      owner[i] = best;
    }
  }

  // independent nodes and hanging nodes, each in Morton order
  std::unordered_map<uint64_t, int32_t> nid, hid;
  for (size_t i = 0; i < ck.size(); ++i) {
    uint32_t x, y, z;
    decode(ck[i], x, y, z);
    if (hanging[i]) {
      hid[ck[i]] = (int32_t)out.hang_xyz.size();
      out.hang_xyz.push_back({x, y, z});
    } else {
      nid[ck[i]] = (int32_t)out.nodes.size();
      out.nodes.push_back({x, y, z});
    }
  }
  std::unordered_map<uint64_t, size_t> cidx;
  for (size_t i = 0; i < ck.size(); ++i) cidx[ck[i]] = i;

  // Constraints: an edge-interior hanging node takes 1/2 of the two edge
  // endpoints, a face-interior one 1/4 of the four face corners of the
  // constraining leaf; hanging endpoints are substituted recursively.
  std::map<uint64_t, Constraint> memo;
  std::string cerr;
  std::function<const Constraint&(uint64_t)> resolve;
  resolve = [&](uint64_t key) -> const Constraint& {
    auto mit = memo.find(key);
    if (mit != memo.end()) return mit->second;
    Constraint c;
    auto nit = nid.find(key);
    if (nit != nid.end()) {
      c.terms.push_back({nit->second, 1.0});
      return memo[key] = c;
    }
    auto ci = cidx.find(key);
    if (ci == cidx.end() || !hanging[ci->second]) {
      cerr = "constraint parent is not a mesh corner";
      return memo[key] = c;
    }
    uint32_t px, py, pz;
    decode(key, px, py, pz);
    const Leaf& L = owner[ci->second];
    uint32_t s = C.size_of(L.level);
    uint32_t P[3] = {px, py, pz}, A[3] = {L.x, L.y, L.z};
    int free_axes[3], nfree = 0;
    for (int d = 0; d < 3; ++d) {
      uint32_t o = P[d] - A[d];
      if (o == 0 || o == s) continue;
      if (o * 2 != s) {
        cerr = "hanging node not at an edge or face midpoint (tree not 2:1 balanced)";
        return memo[key] = c;
      }
      free_axes[nfree++] = d;
    }
    if (nfree < 1 || nfree > 2) {
      cerr = "hanging node is neither edge- nor face-interior";
      return memo[key] = c;
    }
    double w = nfree == 1 ? 0.5 : 0.25;
    std::map<int32_t, double> acc;
    for (int m = 0; m < (1 << nfree); ++m) {
      uint32_t Q[3] = {P[0], P[1], P[2]};
      for (int t = 0; t < nfree; ++t) {
        int d = free_axes[t];
        Q[d] = A[d] + (((m >> t) & 1) ? s : 0);
      }
      const Constraint& sub = resolve(morton3(Q[0], Q[1], Q[2]));
      for (auto& tw : sub.terms) acc[tw.first] += w * tw.second;
    }
    for (auto& kv : acc) c.terms.push_back({kv.first, kv.second});
    return memo[key] = c;
  };

  out.hang_off.push_back(0);
  for (auto& hx : out.hang_xyz) {
    const Constraint& c = resolve(morton3(hx[0], hx[1], hx[2]));
    if (!cerr.empty()) return cerr;
    for (auto& tw : c.terms) {
      out.hang_ids.push_back(tw.first);
      out.hang_w.push_back(tw.second);
    }
    out.hang_off.push_back((int64_t)out.hang_ids.size());
  }

  // element table
  out.elem.resize(out.leaves.size());
  for (size_t e = 0; e < out.leaves.size(); ++e) {
    const Leaf& L = out.leaves[e];
    uint32_t s = C.size_of(L.level);
    for (int c = 0; c < 8; ++c) {
      uint64_t k = morton3(L.x + ((c & 1) ? s : 0), L.y + ((c & 2) ? s : 0),
                           L.z + ((c & 4) ? s : 0));
      auto it = nid.find(k);
      out.elem[e][c] = it != nid.end() ? it->second : -1 - hid.at(k);
    }
  }

  // boundary flags (Sec. 4 "Meshing": two bits per node)
  out.bflags.assign(out.nodes.size(), 0);
  for (size_t i = 0; i < out.nodes.size(); ++i) {
    bool b = false;
    for (int d = 0; d < 3; ++d)
      if (out.nodes[i][d] == 0 || out.nodes[i][d] == C.ext[d]) b = true;
    out.bflags[i] = b ? 1 : 0;
  }
  if (!out.bflags.empty()) out.bflags[0] |= 2;  // pressure pin: Morton-first node
  return "";
}

}  // namespace orc
