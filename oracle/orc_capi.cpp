// C entry points of the oracle, loaded with ctypes by the test suite and by
// the CPU-baseline leg of the benchmark.  TEST INFRASTRUCTURE ONLY.
#include <cstring>
#include <string>

#include "orc.hpp"

namespace {
thread_local std::string g_err;
int fail(const std::string& e) {
  g_err = e;
  return -1;
}
}  // namespace

extern "C" {

const char* orc_last_error(void) { return g_err.c_str(); }

int orc_mesh_build(const int32_t* T, int level_min, int level_max, orc::Phi0Fn phi0, void* user,
                   double band, const int32_t* leaves, int64_t n_leaves, void** out) {
  orc::Mesh* m = new orc::Mesh();
  int t[3] = {T[0], T[1], T[2]};
  std::string err =
      orc::build_mesh(t, level_min, level_max, phi0, user, band, leaves, n_leaves, *m);
  if (!err.empty()) {
    delete m;
    return fail(err);
  }
  *out = m;
  return 0;
}

void orc_mesh_free(void* m) { delete (orc::Mesh*)m; }

// sizes: n_leaves, n_nodes, n_hanging, n_constraint_entries, level_max
void orc_mesh_sizes(void* mp, int64_t* s) {
  const orc::Mesh& m = *(orc::Mesh*)mp;
  s[0] = (int64_t)m.leaves.size();
  s[1] = (int64_t)m.nodes.size();
  s[2] = (int64_t)m.hang_xyz.size();
  s[3] = (int64_t)m.hang_ids.size();
  s[4] = m.D;
}

void orc_mesh_arrays(void* mp, int32_t* leaves4, int32_t* elem8, int32_t* nodes3, uint8_t* bflags,
                     int32_t* hang3, int64_t* hang_off, int32_t* hang_ids, double* hang_w) {
  const orc::Mesh& m = *(orc::Mesh*)mp;
  for (size_t e = 0; e < m.leaves.size(); ++e) {
    leaves4[4 * e] = (int32_t)m.leaves[e].x;
    leaves4[4 * e + 1] = (int32_t)m.leaves[e].y;
    leaves4[4 * e + 2] = (int32_t)m.leaves[e].z;
    leaves4[4 * e + 3] = m.leaves[e].level;
    for (int c = 0; c < 8; ++c) elem8[8 * e + c] = m.elem[e][c];
  }
  for (size_t i = 0; i < m.nodes.size(); ++i) {
    for (int d = 0; d < 3; ++d) nodes3[3 * i + d] = (int32_t)m.nodes[i][d];
    bflags[i] = m.bflags[i];
  }
  for (size_t i = 0; i < m.hang_xyz.size(); ++i)
    for (int d = 0; d < 3; ++d) hang3[3 * i + d] = (int32_t)m.hang_xyz[i][d];
  for (size_t i = 0; i < m.hang_off.size(); ++i) hang_off[i] = m.hang_off[i];
  for (size_t i = 0; i < m.hang_ids.size(); ++i) {
    hang_ids[i] = m.hang_ids[i];
    hang_w[i] = m.hang_w[i];
  }
}

int orc_residual(void* m, const orc::Params* p, int block, const double* Unew, const double* Uold,
                 const double* forcing, const double* bc, double* R) {
  std::string e = orc::residual(*(orc::Mesh*)m, *p, block, Unew, Uold, forcing, R, bc);
  return e.empty() ? 0 : fail(e);
}

int orc_jvp(void* m, const orc::Params* p, int block, const double* Unew, const double* Uold,
            const double* dU, double* JdU) {
  std::string e = orc::jvp(*(orc::Mesh*)m, *p, block, Unew, Uold, dU, JdU);
  return e.empty() ? 0 : fail(e);
}

int orc_jvp_full(void* m, const orc::Params* p, int block, const double* Unew, const double* Uold,
                 const double* dU, double* JdU) {
  std::string e = orc::jvp_full(*(orc::Mesh*)m, *p, block, Unew, Uold, dU, JdU);
  return e.empty() ? 0 : fail(e);
}

int orc_residual_rows(void* m, const orc::Params* p, int block, const double* Unew,
                      const double* Uold, const int32_t* rows, int64_t nrows, const double* dU,
                      double* out) {
  std::string e = orc::residual_rows(*(orc::Mesh*)m, *p, block, Unew, Uold, rows, nrows, dU, out);
  return e.empty() ? 0 : fail(e);
}

int orc_diag_blocks(void* m, const orc::Params* p, int block, const double* Unew,
                    const double* Uold, double* out) {
  std::string e = orc::diag_blocks(*(orc::Mesh*)m, *p, block, Unew, Uold, out);
  return e.empty() ? 0 : fail(e);
}

void orc_diagnostics(void* m, const orc::Params* p, const double* U, double* mass,
                     double* energy) {
  orc::diagnostics(*(orc::Mesh*)m, *p, U, mass, energy);
}

int orc_step(void* m, const orc::Params* p, const orc::SolverOpts* o, double* U,
             const double* forcing, const double* bc, orc::StepStats* st) {
  std::string e = orc::step(*(orc::Mesh*)m, *p, *o, U, forcing, bc, st);
  return e.empty() ? 0 : fail(e);
}

// cG(2) numbering of a mesh and the CH block on it
int orc_q2_build(void* m, void** out) {
  orc::MeshQ2* q = new orc::MeshQ2();
  std::string e = orc::build_q2(*(orc::Mesh*)m, *q);
  if (!e.empty()) {
    delete q;
    return fail(e);
  }
  *out = q;
  return 0;
}

void orc_q2_free(void* q) { delete (orc::MeshQ2*)q; }

// sizes: n_nodes, n_hanging, n_constraint_entries
void orc_q2_sizes(void* qp, int64_t* s) {
  const orc::MeshQ2& q = *(orc::MeshQ2*)qp;
  s[0] = (int64_t)q.nodes.size();
  s[1] = (int64_t)q.hang_xyz.size();
  s[2] = (int64_t)q.hang_ids.size();
}

void orc_q2_arrays(void* qp, int32_t* elem27, int32_t* nodes3, int32_t* hang3, int64_t* hang_off,
                   int32_t* hang_ids, double* hang_w, uint8_t* bflags) {
  const orc::MeshQ2& q = *(orc::MeshQ2*)qp;
  for (size_t i = 0; i < q.bflags.size(); ++i) bflags[i] = q.bflags[i];
  for (size_t e = 0; e < q.elem.size(); ++e)
    for (int a = 0; a < 27; ++a) elem27[27 * e + a] = q.elem[e][a];
  for (size_t i = 0; i < q.nodes.size(); ++i)
    for (int d = 0; d < 3; ++d) nodes3[3 * i + d] = (int32_t)q.nodes[i][d];
  for (size_t i = 0; i < q.hang_xyz.size(); ++i)
    for (int d = 0; d < 3; ++d) hang3[3 * i + d] = (int32_t)q.hang_xyz[i][d];
  for (size_t i = 0; i < q.hang_off.size(); ++i) hang_off[i] = q.hang_off[i];
  for (size_t i = 0; i < q.hang_ids.size(); ++i) {
    hang_ids[i] = q.hang_ids[i];
    hang_w[i] = q.hang_w[i];
  }
}

int orc_q2_residual(void* m, void* q, const orc::Params* p, int block, const double* Unew,
                    const double* Uold, double* R) {
  std::string e = orc::residual_q2(*(orc::Mesh*)m, *(orc::MeshQ2*)q, *p, block, Unew, Uold, R);
  return e.empty() ? 0 : fail(e);
}

int orc_q2_jvp(void* m, void* q, const orc::Params* p, int block, const double* Unew, const double* Uold,
               const double* dU, double* JdU) {
  std::string e = orc::jvp_q2(*(orc::Mesh*)m, *(orc::MeshQ2*)q, *p, block, Unew, Uold, dU, JdU);
  return e.empty() ? 0 : fail(e);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads of the following parallel loops (timing only; results do not depend
// on it, every reduction runs in a fixed order).
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
}
