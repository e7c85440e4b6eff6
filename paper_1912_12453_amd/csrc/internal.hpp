// Internal declarations of libchns (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/chns.h"

namespace chns {

// ------------------------------------------------------------ Morton ------
// 3 x 21-bit interleave, x in the lowest bit of each triple.
inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | (v << 32)) & 0x1f00000000ffffULL;
  v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}
inline uint32_t compact3(uint64_t v) {
  v &= 0x1249249249249249ULL;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ULL;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00fULL;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffULL;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffULL;
  v = (v ^ (v >> 32)) & 0x1fffffULL;
  return (uint32_t)v;
}
inline uint64_t mkey(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}
inline void unkey(uint64_t k, uint32_t& x, uint32_t& y, uint32_t& z) {
  x = compact3(k);
  y = compact3(k >> 1);
  z = compact3(k >> 2);
}

// --------------------------------------------------------- host mesh ------
struct HostMesh {
  int T[3] = {1, 1, 1};
  int D = 0;                         // level_max
  std::vector<uint64_t> leaf_key;    // anchor keys, Morton order
  std::vector<uint8_t> leaf_level;
  std::vector<uint64_t> node_key;    // independent nodes, Morton order
  std::vector<uint64_t> hang_key;    // hanging nodes, Morton order
  std::vector<int32_t> hang_off;     // CSR over hang_ids / hang_w
  std::vector<int32_t> hang_ids;
  std::vector<double> hang_w;
  std::vector<int32_t> elem;         // 8 per leaf
  std::vector<uint8_t> bflags;
  int max_fanin = 0;
};

// Returns "" or an error message.
std::string build_host_mesh(const chns_mesh_spec& spec, HostMesh& out);

// cG(2) numbering of a host mesh for the triquadratic CH block (q2_host.cpp):
// Morton keys of the doubled lattice coordinates of the independent and
// hanging points, the constraint rows (CSR), the 27 node refs per leaf (id,
// or -1 - h) and the gather plan: node n sums the element results g_slot[k]
// (leaf * 27 + local node) times g_w[k], g_off[n] <= k < g_off[n+1], in
// increasing slot order.
struct HostQ2 {
  std::vector<uint64_t> node_key, hang_key;
  std::vector<int32_t> hang_off, hang_ids;
  std::vector<double> hang_w;
  std::vector<int32_t> elem;
  std::vector<int64_t> g_off;
  std::vector<int32_t> g_slot;
  std::vector<double> g_w;
  std::vector<uint8_t> bflags;  // per node: bit 0 on the brick's boundary, bit 1 the pressure pin
};
std::string build_host_q2(const HostMesh& h, HostQ2& out);

// Scatter plan of the element loop (all integer, built once per mesh).
// Elements are cut into Morton chunks of kChunk consecutive leaves, one
// workgroup each.  The targets of chunk c are the independent nodes its
// corners touch (directly or as constraint parents), sorted:
// tgt[tgt_off[c] .. tgt_off[c+1]).  Target slot s sums, in this order, the
// corner results inc_corner[k] (local element * 8 + corner) times inc_w[k] for
// inc_off[s] <= k < inc_off[s+1].  Node n then sums the target slots
// node_slot[node_off[n] .. node_off[n+1]) in increasing slot order.
// For the node-block diagonal every element lists the nodes it touches (its
// direct corners in corner order, then the parents of its hanging corners in
// corner and constraint order, first occurrence only): touch_off[e] ..
// touch_off[e+1]; node n sums touch_slot[ntouch_off[n] .. ntouch_off[n+1]).
// Corner map (for kernels that read a corner's record from the staged chunk
// without searching the target list): cmap[e*8 + k] is the position of
// corner k's node in its chunk's target list, or -1 - j for a hanging corner
// whose entry j in hmap holds kHMap ints: the first index t0 of its
// constraint row, the parent count, then the parents' target-list positions
// (16 bits each, two per int, constraint-row order, -1 when unused).
constexpr int kChunk = 32;
constexpr int kHMap = 8;   // ints per hanging-corner entry (8 parents at most)
struct ScatterPlan {
  std::vector<int32_t> tgt_off, tgt, inc_off;
  std::vector<int32_t> chunk_inc;  // per chunk: inc_off at its first target
  std::vector<uint8_t> inc_corner;
  std::vector<float> inc_w;
  std::vector<int32_t> node_off, node_slot;
  std::vector<int64_t> touch_off;
  std::vector<int32_t> touch_node;  // per element touch: the node
  std::vector<int64_t> ntouch_off, ntouch_slot;
  std::vector<int32_t> cmap, hmap;
  int max_targets = 0;  // targets of the largest chunk
  int max_inc = 0;      // incidences of the largest chunk
  int max_touch = 0;
};
std::string build_scatter_plan(const HostMesh& m, ScatterPlan& out);

// Multigrid hierarchy (multigrid_host.cpp).  coarsen_host_mesh merges the
// finest level of f into its parents; build_transfer gives the prolongation
// P (fine independent node i <- sum_k p_w[k] * coarse node p_idx[k], k in
// [p_off[i], p_off[i+1])), its transpose R (coarse node j <- fine nodes,
// ascending), and the injection inj[j] = the fine node at coarse node j.
std::string coarsen_host_mesh(const HostMesh& f, HostMesh& c);
struct Transfer {
  std::vector<int32_t> p_off, p_idx, r_off, r_idx, inj;
  std::vector<double> p_w, r_w;
};
std::string build_transfer(const HostMesh& f, const HostMesh& c, Transfer& out);

// Remeshing and intergrid transfer between any two meshes of one brick
// (remesh_host.cpp).  build_interp: node i of `to` takes sum_k w[k] *
// (node idx[k] of `from`), k in [off[i], off[i+1]), the trilinear field of
// `from` at that node.  remesh_host: a new mesh refined as build_host_mesh
// does, with the trilinear field of U's phi on `old` as the indicator.
std::string build_interp(const HostMesh& from, const HostMesh& to, std::vector<int32_t>& off,
                         std::vector<int32_t>& idx, std::vector<double>& w);
std::string remesh_host(const HostMesh& old, const double* U, int level_min, int level_max, double band,
                        HostMesh& out);

}  // namespace chns
