// CPU FP64 oracle for the CHNS element loop -- TEST INFRASTRUCTURE ONLY.
//
// This tree is a plain, slow, deliberately unoptimised restatement of the
// method of Khanwale et al., "Simulating two-phase flows with
// thermodynamically consistent energy stable Cahn-Hilliard Navier-Stokes
// equations on parallel adaptive octree based meshes" (arXiv 1912.12453).
// Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
// load it.  It shares no code with the GPU library: it has its own octree
// builder, its own element machinery and its own solver.
//
// Every function cites the passage of the paper it restates.
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace orc {

// ---------------------------------------------------------------- mesh ----
// Octree over a brick of T[0] x T[1] x T[2] unit-cube trees (Sec. 4,
// "Refinement").  Integer coordinates: 2^D units per tree side, D = level_max.
struct Leaf {
  uint32_t x, y, z;
  int level;
};

typedef void (*Phi0Fn)(const double* xyz, int64_t n, double* out, void* user);

struct Mesh {
  int T[3];
  int D;  // level_max: finest level, integer unit = 2^-D
  std::vector<Leaf> leaves;                      // Morton order of anchors
  std::vector<std::array<uint32_t, 3>> nodes;    // independent nodes, Morton order
  std::vector<uint8_t> bflags;                   // bit0 on boundary, bit1 pressure pin
  std::vector<std::array<int32_t, 8>> elem;      // corner c=i+2j+4k -> id>=0 node, <0 hanging -1-h
  std::vector<std::array<uint32_t, 3>> hang_xyz; // hanging nodes, Morton order
  std::vector<int64_t> hang_off;                 // CSR offsets into hang_ids / hang_w
  std::vector<int32_t> hang_ids;                 // independent node ids (ascending per row)
  std::vector<double> hang_w;                    // dyadic weights
};

uint64_t morton3(uint32_t x, uint32_t y, uint32_t z);

// Builds the balanced octree and its node numbering.  Either explicit
// leaves (x,y,z,level quadruples) or top-down refinement driven by phi0.
// Returns "" on success, otherwise an error message.
std::string build_mesh(const int T[3], int level_min, int level_max, Phi0Fn phi0,
                       void* user, double band, const int32_t* leaves,
                       int64_t n_leaves, Mesh& out);

// ------------------------------------------------------------ physics ----
struct Params {
  double Cn, Pe, Re, We, Fr;
  double rho_minus;  // rho_- / rho_+
  double eta_minus;  // eta_- / eta_+
  double dt;
  double g[3];       // unit gravity direction
  double C_I;
  int flux_mode;     // 0: J = -(alpha/Cn) grad mu ; 1: J = -alpha grad mu
};

enum { BLOCK_CH = 0, BLOCK_NS = 1 };

// Optional manufactured-solution forcing at quadrature points:
// forcing[(e*8 + q)*6 + f], f in (phi-eq, mu-eq, momentum x,y,z, continuity).
// May be null.
//
// Optional Dirichlet data: bc is a node-major 6-field vector whose velocity
// entries at boundary nodes are the wall velocity at t^{k+1}; the velocity
// rows of boundary nodes then read v^{k+1} - bc.  When bc is null the wall
// data is carried by the state (rows v^{k+1} - v^k), which keeps stationary
// walls (no-slip) fixed.

// Element loop over all elements (or the listed subset), assembled through
// the hanging-node transpose, followed by the boundary rows.
std::string residual(const Mesh& m, const Params& p, int block, const double* Unew,
                     const double* Uold, const double* forcing, double* R,
                     const double* bc = nullptr);
std::string jvp(const Mesh& m, const Params& p, int block, const double* Unew,
                const double* Uold, const double* dU, double* JdU);
// The block's rows of the coupled Jacobian: the derivative with respect to all
// six fields of U^{k+1} (the block iteration freezes the other block's fields;
// a fully coupled Newton solve needs these cross terms).
std::string jvp_full(const Mesh& m, const Params& p, int block, const double* Unew,
                     const double* Uold, const double* dU, double* JdU);
// Rows of R (6-interleaved) restricted to the listed nodes; out[k*6+f].
std::string residual_rows(const Mesh& m, const Params& p, int block, const double* Unew,
                          const double* Uold, const int32_t* rows, int64_t nrows,
                          const double* dU, double* out);
// Node-block diagonal of the block Jacobian: nf x nf per node, row-major.
std::string diag_blocks(const Mesh& m, const Params& p, int block, const double* Unew,
                        const double* Uold, double* out);
// Diagnostics: integral of phi and total energy.
void diagnostics(const Mesh& m, const Params& p, const double* U, double* mass,
                 double* energy);

struct SolverOpts {
  double newton_rtol, newton_atol, block_tol, gmres_rtol;
  int newton_max_it_ch, newton_max_it_ns, gmres_restart, gmres_max_it, block_max_it;
  int block_min_it;
  int precond;  // 0 point Jacobi, 1 node-block Jacobi
};
struct StepStats {
  int block_its, newton_its[2], gmres_its[2], converged;
  double rel_res[2], mass, energy;
};
std::string step(const Mesh& m, const Params& p, const SolverOpts& o, double* U,
                 const double* forcing, const double* bc, StepStats* st);

// ------------------------------------------------------ cG(2), CH block ----
// Triquadratic (27-node) numbering on the leaves of a Mesh.  Coordinates are
// in doubled units 2^-(D+1), so every lattice point of every leaf is an
// integer point.  Node a = i + 3j + 9k of a leaf sits at its anchor plus
// (i, j, k) half sides.
struct MeshQ2 {
  int D = 0;
  std::vector<std::array<int32_t, 27>> elem;     // id >= 0 node, < 0 hanging -1-h
  std::vector<std::array<uint32_t, 3>> nodes;    // independent nodes, Morton order
  std::vector<std::array<uint32_t, 3>> hang_xyz; // hanging nodes, Morton order
  std::vector<int64_t> hang_off;
  std::vector<int32_t> hang_ids;
  std::vector<double> hang_w;
  std::vector<uint8_t> bflags;                   // bit0 on boundary, bit1 pressure pin
};
std::string build_q2(const Mesh& m, MeshQ2& out);
// Block rows over the Q2 nodes (node-major 6-field vectors): CH fields 0, 1
// (the velocities enter as the frozen v~ of the block iteration), or NS
// fields 2..5 with the boundary rows of the cG(1) oracle.
std::string residual_q2(const Mesh& m, const MeshQ2& q, const Params& p, int block, const double* Unew,
                        const double* Uold, double* R);
std::string jvp_q2(const Mesh& m, const MeshQ2& q, const Params& p, int block, const double* Unew,
                   const double* Uold, const double* dU, double* JdU);

}  // namespace orc
