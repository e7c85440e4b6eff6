// C ABI of libchns: mesh handles, device upload, element-loop launches and
// the Crank-Nicolson step driver (block iteration of Fig. 1, Newton per block
// as in Sec. 3.5, right-preconditioned GMRES with classical Gram-Schmidt).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hip"
#include "linalg.hpp"
#include "multigrid.hpp"

using namespace chns;

namespace {

thread_local std::string g_err;

// Allocation, release, stream creation and graph capture of every mesh and
// server go through this lock, so that a capture in progress on one host
// thread never overlaps an allocation or a free (with its implicit device
// synchronisation) made by another.  Kernel launches, copies and
// synchronisation of streams do not take it.
std::mutex g_struct_mu;
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(CHNS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int dalloc(T** p, size_t count, int64_t* bytes) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(CHNS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  if (bytes) *bytes += (int64_t)(count * sizeof(T));
  return CHNS_OK;
}

inline unsigned grid_for(int64_t threads, int block = 256) {
  int64_t g = (threads + block - 1) / block;
  return (unsigned)std::max<int64_t>(1, g);
}
inline unsigned grid_stride(int64_t n, int block = 256, int cap = 2048) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap, (n + block - 1) / block));
}

// A part of a GMRES restart cycle captured as a HIP graph, valid for one
// block, basis type, restart length and parameter set of the mesh it was
// captured on.
struct CycleGraph {
  int block = 0, tv = 0, mres = 0, seg = 0;
  int precond = 0, mg_levels = 0, mg_smooth = 0, mg_coarse = 0;
  double mg_omega = 0;
  dev::PhysView pv;
  hipGraphExec_t exec = nullptr;
};

struct Workspace {
  int64_t n = 0;
  int restart64 = 0, restart32 = 0;  // basis length allocated per precision
  double *U1 = nullptr;              // the step's iterate U^{k+1}
  double *Uk = nullptr, *Uprev = nullptr, *r = nullptr, *x = nullptr;
  double *D = nullptr, *Di = nullptr, *DiC = nullptr;  // Di: NS blocks, DiC: CH blocks
  float *Di32 = nullptr, *DiC32 = nullptr, *U1f = nullptr, *U0f = nullptr;
  double *pk64 = nullptr, *pz64 = nullptr;  // coupled solve: one block's part of a vector
  float *pk32 = nullptr, *pz32 = nullptr;
  int nfw = 4;                              // values per node of the Krylov vectors
  double *V64 = nullptr, *Z64 = nullptr, *w64 = nullptr, *b64 = nullptr;
  float *V32 = nullptr, *Z32 = nullptr, *w32 = nullptr, *b32 = nullptr;
  double *part = nullptr, *dots = nullptr;
  double* hdots = nullptr;  // pinned host
  int* flag = nullptr;
  int* hflag = nullptr;     // pinned host
  dev::GmresCtl* ctl = nullptr;
  int* hctl = nullptr;      // pinned host: the first ints of *ctl
  hipStream_t cap = nullptr;  // capture stream (graphs are launched on the caller's)
  std::vector<CycleGraph> graphs;
  int nb_part = 0;
  int64_t bytes = 0;
};

void drop_graphs(Workspace& w) {
  for (auto& g : w.graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  w.graphs.clear();
}

void free_basis(Workspace& w, int precision) {
  drop_graphs(w);
  const int64_t N = w.n * w.nfw;
  if (precision == 0) {
    if (w.V64) w.bytes -= (N * (2 * w.restart64 + 3)) * (int64_t)sizeof(double);
    void* ptrs[] = {w.V64, w.Z64, w.w64, w.b64};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    w.V64 = w.Z64 = w.w64 = w.b64 = nullptr;
    w.restart64 = 0;
  } else {
    if (w.V32) w.bytes -= (N * (2 * w.restart32 + 3) + w.n * 12) * (int64_t)sizeof(float);
    void* ptrs[] = {w.V32, w.Z32, w.w32, w.b32, w.U1f, w.U0f};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    w.V32 = w.Z32 = w.w32 = w.b32 = nullptr;
    w.U1f = w.U0f = nullptr;
    w.restart32 = 0;
  }
}

void free_workspace(Workspace& w) {
  free_basis(w, 0);
  free_basis(w, 1);
  void* ptrs[] = {w.U1, w.Uk, w.Uprev, w.r, w.x, w.D, w.Di, w.Di32, w.DiC, w.DiC32, w.pk64, w.pz64, w.pk32,
                  w.pz32, w.part, w.dots, w.flag, w.ctl};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (w.hdots) (void)hipHostFree(w.hdots);
  if (w.hflag) (void)hipHostFree(w.hflag);
  if (w.hctl) (void)hipHostFree(w.hctl);
  if (w.cap) (void)hipStreamDestroy(w.cap);
  w = Workspace();
}

// One mesh of the multigrid hierarchy.  Level 0 is the mesh itself; the
// transfer arrays of level l connect it with level l + 1.
struct MGLevel {
  chns_mesh* mesh = nullptr;  // owned for levels >= 1
  int64_t n = 0;
  int32_t *p_off = nullptr, *p_idx = nullptr, *r_off = nullptr, *inj = nullptr;
  double* p_w = nullptr;
  int32_t* r_eidx = nullptr;  // restriction lists, padded column-major (k_restrict)
  float* r_ew = nullptr;
  double *U1 = nullptr, *U0 = nullptr, *D = nullptr, *Di = nullptr, *DiC = nullptr;  // levels >= 1
  float *U1f = nullptr, *U0f = nullptr, *Di32 = nullptr, *DiC32 = nullptr;
  double *b64 = nullptr, *x64 = nullptr, *r64 = nullptr;
  float *b32 = nullptr, *x32 = nullptr, *r32 = nullptr;
};

}  // namespace

struct chns_mesh {
  HostMesh h;
  ScatterPlan plan;
  bool plan_ready = false;  // built ahead of upload (the serving builder does)
  int device = -1;
  bool uploaded = false;
  int32_t *d_elem = nullptr, *d_hoff = nullptr, *d_hids = nullptr, *d_anchor = nullptr;
  uint8_t* d_level = nullptr;
  // scatter plan
  int32_t *d_tgt_off = nullptr, *d_tgt = nullptr, *d_inc_off = nullptr, *d_node_off = nullptr, *d_node_slot = nullptr;
  int32_t* d_chunk_inc = nullptr;
  uint8_t *d_inc_corner = nullptr, *d_bflags = nullptr;
  float* d_inc_w = nullptr;
  int64_t *d_touch_off = nullptr, *d_ntouch_off = nullptr, *d_ntouch_slot = nullptr;
  int32_t* d_touch_node = nullptr;
  int32_t *d_cmap = nullptr, *d_hmap = nullptr;  // corner map of the plan
  double* d_partial = nullptr;  // target slots x 4 (FP64), or x 8 FP32 values
  double* d_tbuf = nullptr;     // element touches x 16, allocated on first diagonal
  int64_t n_chunks = 0;
  double* d_hw = nullptr;
  float* d_hw32 = nullptr;
  int* d_flag = nullptr;
  int* h_flag = nullptr;
  double* d_part = nullptr;  // diagnostics partials
  double* d_sum = nullptr;
  double* h_sum = nullptr;
  int64_t device_bytes = 0;
  Workspace ws;
  void* d_lin[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // cached linearisation points [block][FP64, FP32]
  void* d_mid[2] = {nullptr, nullptr};  // nodal midpoints of the NS linearisation point [FP64, FP32]
  std::vector<MGLevel> mg;  // multigrid hierarchy, built on first use
  int mg_key = -1;          // mg_levels it was built for
  int64_t mg_bytes = 0;     // level buffers and transfers of the hierarchy (coarse meshes count their own)
};

namespace {
void free_mesh_locked(chns_mesh* m);  // frees everything; caller holds g_struct_mu
void free_mg_locked(chns_mesh* m);    // frees the multigrid hierarchy; same
}  // namespace

namespace {

dev::MeshView view(const chns_mesh* m) {
  dev::MeshView v;
  v.elem = m->d_elem;
  v.level = m->d_level;
  v.hoff = m->d_hoff;
  v.hids = m->d_hids;
  v.hw = m->d_hw;
  v.hw32 = m->d_hw32;
  v.E = (int64_t)m->h.leaf_key.size();
  return v;
}

dev::ChunkCaps caps(const chns_mesh* m) {
  return dev::ChunkCaps{m->plan.max_targets, m->plan.max_inc};
}

dev::PlanView plan_view(const chns_mesh* m) {
  dev::PlanView v;
  v.tgt_off = m->d_tgt_off;
  v.tgt = m->d_tgt;
  v.inc_off = m->d_inc_off;
  v.chunk_inc = m->d_chunk_inc;
  v.inc_corner = m->d_inc_corner;
  v.inc_w = m->d_inc_w;
  v.node_off = m->d_node_off;
  v.node_slot = m->d_node_slot;
  v.touch_off = m->d_touch_off;
  v.touch_node = m->d_touch_node;
  v.ntouch_off = m->d_ntouch_off;
  v.ntouch_slot = m->d_ntouch_slot;
  v.bflags = m->d_bflags;
  v.cmap = m->d_cmap;
  v.hmap = m->d_hmap;
  return v;
}

template <class T>
int h2d(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return CHNS_OK;
  HIPCHK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return CHNS_OK;
}

int phys_view(const chns_params* p, dev::PhysView& v) {
  if (!p) return fail(CHNS_EINVAL, "params is NULL");
  const double vals[] = {p->Cn, p->Pe, p->Re, p->We, p->Fr, p->rho_minus, p->eta_minus, p->dt,
                         p->gravity[0], p->gravity[1], p->gravity[2], p->C_I};
  for (double x : vals)
    if (!std::isfinite(x)) return fail(CHNS_EINVAL, "non-finite parameter");
  if (p->Cn <= 0 || p->Pe <= 0 || p->Re <= 0 || p->We <= 0 || p->Fr <= 0 || p->dt <= 0)
    return fail(CHNS_EINVAL, "Cn, Pe, Re, We, Fr and dt must be positive");
  if (p->rho_minus <= 0 || p->eta_minus <= 0)
    return fail(CHNS_EINVAL, "density and viscosity ratios must be positive");
  if (p->flux_mode != 0 && p->flux_mode != 1) return fail(CHNS_EINVAL, "flux_mode must be 0 or 1");
  v.dt = p->dt;
  v.inv_dt = 1.0 / p->dt;
  v.Cn = p->Cn;
  v.inv_PeCn = 1.0 / (p->Pe * p->Cn);
  v.Cn2 = p->Cn * p->Cn;
  v.alpha = 0.5 * (1.0 - p->rho_minus);
  v.beta = 0.5 * (1.0 + p->rho_minus);
  v.gamma = 0.5 * (1.0 - p->eta_minus);
  v.xi = 0.5 * (1.0 + p->eta_minus);
  v.kappa = p->flux_mode == 1 ? -v.alpha : -v.alpha / p->Cn;
  v.inv_Pe = 1.0 / p->Pe;
  v.inv_Re = 1.0 / p->Re;
  v.inv_We = 1.0 / p->We;
  v.inv_Fr = 1.0 / p->Fr;
  v.CnWe = p->Cn / p->We;
  for (int d = 0; d < 3; ++d) v.g[d] = p->gravity[d];
  v.C_I = p->C_I;
  return CHNS_OK;
}

int upload(chns_mesh* m, hipStream_t s) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (m->uploaded) {
    if (dev != m->device) return fail(CHNS_EINVAL, "mesh was uploaded to another device");
    return CHNS_OK;
  }
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
    return fail(CHNS_ENODEV, std::string("libchns is built for gfx950, device is ") + prop.gcnArchName);
  const HostMesh& h = m->h;
  const size_t E = h.leaf_key.size(), NH = h.hang_key.size(), NC = h.hang_ids.size();
  if (h.max_fanin > 8) return fail(CHNS_EINVAL, "hanging-node fan-in above 8 is not supported");
  if (!m->plan_ready) {
    std::string perr;
    try {
      perr = build_scatter_plan(h, m->plan);
    } catch (const std::bad_alloc&) {
      perr = "out of host memory building the scatter plan";
    }
    if (!perr.empty()) return fail(CHNS_ENOMEM, perr);
    m->plan_ready = true;
  }
  const ScatterPlan& P = m->plan;
  std::vector<int32_t> anchor(E * 3);
  for (size_t e = 0; e < E; ++e) {
    uint32_t x, y, z;
    unkey(h.leaf_key[e], x, y, z);
    anchor[3 * e] = (int32_t)x;
    anchor[3 * e + 1] = (int32_t)y;
    anchor[3 * e + 2] = (int32_t)z;
  }
  std::vector<float> w32(h.hang_w.begin(), h.hang_w.end());
  std::lock_guard<std::mutex> lk(g_struct_mu);
  int64_t& B = m->device_bytes;
  B = 0;
  int rc;
  if ((rc = dalloc(&m->d_elem, E * 8, &B)) || (rc = dalloc(&m->d_level, E, &B)) ||
      (rc = dalloc(&m->d_anchor, E * 3, &B)) || (rc = dalloc(&m->d_hoff, NH + 1, &B)) ||
      (rc = dalloc(&m->d_hids, NC, &B)) || (rc = dalloc(&m->d_hw, NC, &B)) ||
      (rc = dalloc(&m->d_hw32, NC, &B)) || (rc = dalloc(&m->d_flag, 1, &B)) ||
      (rc = dalloc(&m->d_part, (int64_t)dev::diag_blocks(E) * 2, &B)) || (rc = dalloc(&m->d_sum, 2, &B)) ||
      (rc = dalloc(&m->d_tgt_off, P.tgt_off.size(), &B)) || (rc = dalloc(&m->d_tgt, P.tgt.size(), &B)) ||
      (rc = dalloc(&m->d_inc_off, P.inc_off.size(), &B)) ||
      (rc = dalloc(&m->d_chunk_inc, P.chunk_inc.size(), &B)) ||
      (rc = dalloc(&m->d_inc_corner, P.inc_corner.size(), &B)) ||
      (rc = dalloc(&m->d_inc_w, P.inc_w.size(), &B)) ||
      (rc = dalloc(&m->d_node_off, P.node_off.size(), &B)) ||
      (rc = dalloc(&m->d_node_slot, P.node_slot.size(), &B)) ||
      (rc = dalloc(&m->d_touch_off, P.touch_off.size(), &B)) ||
      (rc = dalloc(&m->d_touch_node, P.touch_node.size(), &B)) ||
      (rc = dalloc(&m->d_ntouch_off, P.ntouch_off.size(), &B)) ||
      (rc = dalloc(&m->d_ntouch_slot, P.ntouch_slot.size(), &B)) ||
      (rc = dalloc(&m->d_bflags, h.bflags.size(), &B)) ||
      (rc = dalloc(&m->d_cmap, P.cmap.size(), &B)) || (rc = dalloc(&m->d_hmap, P.hmap.size(), &B)) ||
      (rc = dalloc(&m->d_partial, P.tgt.size() * 4, &B)))
    return rc;
  HIPCHK(hipHostMalloc((void**)&m->h_flag, sizeof(int)));
  HIPCHK(hipHostMalloc((void**)&m->h_sum, 2 * sizeof(double)));
  if ((rc = h2d(m->d_elem, h.elem, s)) || (rc = h2d(m->d_level, h.leaf_level, s)) ||
      (rc = h2d(m->d_anchor, anchor, s)) || (rc = h2d(m->d_hoff, h.hang_off, s)) ||
      (rc = h2d(m->d_hids, h.hang_ids, s)) || (rc = h2d(m->d_hw, h.hang_w, s)) ||
      (rc = h2d(m->d_hw32, w32, s)) || (rc = h2d(m->d_tgt_off, P.tgt_off, s)) || (rc = h2d(m->d_tgt, P.tgt, s)) ||
      (rc = h2d(m->d_inc_off, P.inc_off, s)) || (rc = h2d(m->d_chunk_inc, P.chunk_inc, s)) ||
      (rc = h2d(m->d_inc_corner, P.inc_corner, s)) ||
      (rc = h2d(m->d_inc_w, P.inc_w, s)) || (rc = h2d(m->d_node_off, P.node_off, s)) ||
      (rc = h2d(m->d_node_slot, P.node_slot, s)) || (rc = h2d(m->d_touch_off, P.touch_off, s)) ||
      (rc = h2d(m->d_touch_node, P.touch_node, s)) ||
      (rc = h2d(m->d_ntouch_off, P.ntouch_off, s)) ||
      (rc = h2d(m->d_ntouch_slot, P.ntouch_slot, s)) || (rc = h2d(m->d_bflags, h.bflags, s)) ||
      (rc = h2d(m->d_cmap, P.cmap, s)) || (rc = h2d(m->d_hmap, P.hmap, s)))
    return rc;
  m->n_chunks = (int64_t)P.tgt_off.size() - 1;
  if (dev::ChunkLDS<double, 6, 4, 4>::bytes(caps(m)) > 65536)
    return fail(CHNS_EINVAL, "a chunk of the mesh needs more than 64 KiB of LDS");
  // the host vectors above must outlive the copies
  HIPCHK(hipStreamSynchronize(s));
  m->device = dev;
  m->uploaded = true;
  return CHNS_OK;
}

int ensure_tbuf(chns_mesh* m) {
  if (m->d_tbuf) return CHNS_OK;
  std::lock_guard<std::mutex> lk(g_struct_mu);
  return dalloc(&m->d_tbuf, (size_t)m->plan.ntouch_slot.size() * 16, &m->device_bytes);
}

int check_mesh(chns_mesh* m, hipStream_t s) {
  if (!m) return fail(CHNS_EINVAL, "mesh is NULL");
  return upload(m, s);
}

// ----------------------------------------------------------- launches ----
// Element kernel (one workgroup per chunk of 32 leaves) writing the chunk's
// target partials, then the node gather writing every row of the output.
int launch_residual(chns_mesh* m, const dev::PhysView& pv, int block, const double* U1,
                    const double* U0, double* R, int ld, int off, hipStream_t s, bool check_tau,
                    bool keep = false) {
  const int64_t n = (int64_t)m->h.node_key.size();
  const auto mv = view(m);
  const auto pl = plan_view(m);
  const dim3 g((unsigned)m->n_chunks), b(dev::kChunkThreads);
  const dev::ChunkCaps cc = caps(m);
  double* part = m->d_partial;
  if (block == CHNS_BLOCK_CH) {
    hipLaunchKernelGGL(dev::k_ch_residual<double>, g, b, (dev::ChunkLDS<double, 5, 0, 2>::bytes(cc)), s,
                       mv, pl, pv, cc, U1, U0, part);
    hipLaunchKernelGGL((dev::k_gather<2, double, double, 0>), dim3(grid_stride(n)), dim3(256), 0, s,
                       pl, n, part, R, ld, off, U1, U0, (const double*)nullptr, 0, 0, (const int*)nullptr);
    HIPCHK(hipGetLastError());
    return CHNS_OK;
  }
  hipLaunchKernelGGL(dev::k_fill<int>, dim3(1), dim3(64), 0, s, m->d_flag, (int64_t)1, 0);
  hipLaunchKernelGGL(dev::k_ns_residual<double>, g, b, (dev::ChunkLDS<double, 6, 0, 4>::bytes(cc)), s, mv,
                     pl, pv, cc, U1, U0, part, m->d_flag);
  if (keep)  // the CH entries of R are left as they are
    hipLaunchKernelGGL((dev::k_gather<4, double, double, 1, true>), dim3(grid_stride(n)), dim3(256), 0, s, pl,
                       n, part, R, ld, off, U1, U0, (const double*)nullptr, 0, 0, (const int*)nullptr);
  else
    hipLaunchKernelGGL((dev::k_gather<4, double, double, 1>), dim3(grid_stride(n)), dim3(256), 0, s, pl,
                       n, part, R, ld, off, U1, U0, (const double*)nullptr, 0, 0, (const int*)nullptr);
  HIPCHK(hipGetLastError());
  if (check_tau) {
    HIPCHK(hipMemcpyAsync(m->h_flag, m->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*m->h_flag & 1) return fail(CHNS_ETAU, "tau_m bracket is not positive at some Gauss point");
  }
  return CHNS_OK;
}

// T: arithmetic, TS: state storage, TD: direction and output storage (partials
// are kept in T)
// partials of the chunk targets: the mesh's own buffer unless `part` is given
// (chns_jvp_noalloc passes the library's static scratch).
template <class T, class TS, class TD>
int launch_jvp(chns_mesh* m, const dev::PhysView& pv, int block, const TS* U1, const TS* U0,
               const TD* dU, int ldD, int offD, TD* out, int ldO, int offO, hipStream_t s,
               const int* skip = nullptr, void* part_buf = nullptr) {
  const int64_t n = (int64_t)m->h.node_key.size();
  const auto mv = view(m);
  const auto pl = plan_view(m);
  const dim3 g((unsigned)m->n_chunks), b(dev::kChunkThreads);
  const dev::ChunkCaps cc = caps(m);
  T* part = (T*)(part_buf ? part_buf : (void*)m->d_partial);
  if (block == CHNS_BLOCK_CH) {
    hipLaunchKernelGGL((dev::k_ch_jvp<T, TS, TD>), g, b, (dev::ChunkLDS<T, 5, 2, 2>::bytes(cc)), s, mv, pl,
                       pv, cc, U1, U0, dU, ldD, offD, part, skip);
    hipLaunchKernelGGL((dev::k_gather<2, T, TD, 0>), dim3(grid_stride(n)), dim3(256), 0, s, pl, n, part,
                       out, ldO, offO, (const double*)nullptr, (const double*)nullptr, dU, ldD, offD, skip);
  } else {
    hipLaunchKernelGGL((dev::k_ns_jvp<T, TS, TD>), g, b, (dev::ChunkLDS<T, 6, 4, 4>::bytes(cc)), s, mv, pl,
                       pv, cc, U1, U0, dU, ldD, offD, part, skip);
    hipLaunchKernelGGL((dev::k_gather<4, T, TD, 2>), dim3(grid_stride(n)), dim3(256), 0, s, pl, n, part,
                       out, ldO, offO, (const double*)nullptr, (const double*)nullptr, dU, ldD, offD, skip);
  }
  HIPCHK(hipGetLastError());
  return CHNS_OK;
}

// Both blocks' rows of the coupled Jacobian applied to dU (node-major, 6 per
// node): CH rows, then NS rows (which keep the CH rows).
template <class T, class TS, class TD>
int launch_jvp_full(chns_mesh* m, const dev::PhysView& pv, const TS* U1, const TS* U0, const TD* dU, TD* out,
                    hipStream_t s, const int* skip = nullptr) {
  const int64_t n = (int64_t)m->h.node_key.size();
  const auto mv = view(m);
  const auto pl = plan_view(m);
  const dim3 g((unsigned)m->n_chunks), b(dev::kChunkThreads);
  const dev::ChunkCaps cc = caps(m);
  T* part = (T*)m->d_partial;
  hipLaunchKernelGGL((dev::k_ch_jvp_full<T, TS, TD>), g, b, (dev::ChunkLDS<T, 5, 5, 2>::bytes(cc)), s, mv, pl, pv,
                     cc, U1, U0, dU, part, skip);
  hipLaunchKernelGGL((dev::k_gather<2, T, TD, 0>), dim3(grid_stride(n)), dim3(256), 0, s, pl, n, part, out, 6, 0,
                     (const double*)nullptr, (const double*)nullptr, dU, 6, 0, skip);
  hipLaunchKernelGGL((dev::k_ns_jvp_full<T, TS, TD>), g, b, (dev::ChunkLDS<T, 6, 6, 4>::bytes(cc)), s, mv, pl, pv,
                     cc, U1, U0, dU, part, skip);
  hipLaunchKernelGGL((dev::k_gather<4, T, TD, 2, true>), dim3(grid_stride(n)), dim3(256), 0, s, pl, n, part, out,
                     6, 2, (const double*)nullptr, (const double*)nullptr, dU, 6, 2, skip);
  HIPCHK(hipGetLastError());
  return CHNS_OK;
}

// Cached linearisation points (k_ns_lin, k_ch_lin) and the JVPs that read
// them, per block and precision.
int lin_values(int block) { return block == CHNS_BLOCK_CH ? dev::kCHLin : dev::kNSLin; }

template <class T>
int ensure_lin(chns_mesh* m, int block) {
  const int k = std::is_same<T, double>::value ? 0 : 1;
  void*& slot = m->d_lin[block][k];
  if (slot) return CHNS_OK;
  std::lock_guard<std::mutex> lk(g_struct_mu);
  T *p = nullptr, *q = nullptr;
  int rc = dalloc(&p, (size_t)m->n_chunks * lin_values(block) * dev::kChunkThreads, &m->device_bytes);
  if (rc) return rc;
  if (block == CHNS_BLOCK_NS && !m->d_mid[k]) {
    if ((rc = dalloc(&q, m->h.node_key.size() * dev::kNSMid, &m->device_bytes))) {
      (void)hipFree(p);
      m->device_bytes -= (int64_t)((size_t)m->n_chunks * lin_values(block) * dev::kChunkThreads * sizeof(T));
      return rc;
    }
    m->d_mid[k] = q;
  }
  slot = p;
  return CHNS_OK;
}

template <class T, class TS>
int launch_lin(chns_mesh* m, const dev::PhysView& pv, int block, const TS* U1, const TS* U0, hipStream_t s) {
  int rc = ensure_lin<T>(m, block);
  if (rc) return rc;
  const dev::ChunkCaps cc = caps(m);
  T* lin = (T*)m->d_lin[block][std::is_same<T, double>::value ? 0 : 1];
  const dim3 g((unsigned)m->n_chunks), b(dev::kChunkThreads);
  if (block == CHNS_BLOCK_CH)
    hipLaunchKernelGGL((dev::k_ch_lin<T, TS>), g, b, (dev::ChunkLDS<T, 5, 0, 2>::bytes(cc)), s, view(m),
                       plan_view(m), pv, cc, U1, U0, lin);
  else {
    hipLaunchKernelGGL((dev::k_ns_lin<T, TS>), g, b, (dev::ChunkLDS<T, 6, 0, 4>::bytes(cc)), s, view(m),
                       plan_view(m), pv, cc, U1, U0, lin);
    const int64_t n = (int64_t)m->h.node_key.size();
    hipLaunchKernelGGL((dev::k_ns_mid<T, TS>), dim3(grid_stride(n * dev::kNSMid)), dim3(256), 0, s, n, U1, U0,
                       (T*)m->d_mid[std::is_same<T, double>::value ? 0 : 1]);
  }
  HIPCHK(hipGetLastError());
  return CHNS_OK;
}

template <class T>
const T* ns_mid(const chns_mesh* m) {
  return (const T*)m->d_mid[std::is_same<T, double>::value ? 0 : 1];
}

// The element pass of a cached JVP alone (partials; the caller gathers).
template <class T, class TD>
int launch_jvp_lin_elements(chns_mesh* m, const dev::PhysView& pv, int block, const TD* dU, int ldD, int offD,
                            hipStream_t s, const int* skip) {
  const T* lin = (const T*)m->d_lin[block][std::is_same<T, double>::value ? 0 : 1];
  if (!lin) return fail(CHNS_EINVAL, "no linearisation point: call chns_linearize first");
  const dev::ChunkCaps cc = caps(m);
  const dim3 g((unsigned)m->n_chunks), b(dev::kChunkThreads);
  T* part = (T*)m->d_partial;
  if (block == CHNS_BLOCK_CH)
    hipLaunchKernelGGL((dev::k_ch_jvp_lin<T, TD>), g, b, (dev::ChunkLDS<T, 0, 2, 2>::bytes(cc)), s, view(m),
                       plan_view(m), pv, cc, lin, dU, ldD, offD, part, skip);
  else
    hipLaunchKernelGGL((dev::k_ns_jvp_lin<T, TD>), g, b, (dev::ChunkLDS<T, 0, 4 + dev::kNSMid, 4>::bytes(cc)), s,
                       view(m), plan_view(m), pv, cc, lin, ns_mid<T>(m), dU, ldD, offD, part, skip);
  HIPCHK(hipGetLastError());
  return CHNS_OK;
}

template <class T, class TD>
int launch_jvp_lin(chns_mesh* m, const dev::PhysView& pv, int block, const TD* dU, int ldD, int offD, TD* out,
                   int ldO, int offO, hipStream_t s, const int* skip = nullptr) {
  const T* lin = (const T*)m->d_lin[block][std::is_same<T, double>::value ? 0 : 1];
  if (!lin) return fail(CHNS_EINVAL, "no linearisation point: call chns_linearize first");
  const int64_t n = (int64_t)m->h.node_key.size();
  const dev::ChunkCaps cc = caps(m);
  const auto pl = plan_view(m);
  T* part = (T*)m->d_partial;
  const dim3 g((unsigned)m->n_chunks), b(dev::kChunkThreads);
  if (block == CHNS_BLOCK_CH) {
    hipLaunchKernelGGL((dev::k_ch_jvp_lin<T, TD>), g, b, (dev::ChunkLDS<T, 0, 2, 2>::bytes(cc)), s, view(m), pl,
                       pv, cc, lin, dU, ldD, offD, part, skip);
    hipLaunchKernelGGL((dev::k_gather<2, T, TD, 0>), dim3(grid_stride(n)), dim3(256), 0, s, pl, n, part, out,
                       ldO, offO, (const double*)nullptr, (const double*)nullptr, dU, ldD, offD, skip);
  } else {
    hipLaunchKernelGGL((dev::k_ns_jvp_lin<T, TD>), g, b, (dev::ChunkLDS<T, 0, 4 + dev::kNSMid, 4>::bytes(cc)), s,
                       view(m), pl, pv, cc, lin, ns_mid<T>(m), dU, ldD, offD, part, skip);
    hipLaunchKernelGGL((dev::k_gather<4, T, TD, 2>), dim3(grid_stride(n)), dim3(256), 0, s, pl, n, part, out,
                       ldO, offO, (const double*)nullptr, (const double*)nullptr, dU, ldD, offD, skip);
  }
  HIPCHK(hipGetLastError());
  return CHNS_OK;
}

int launch_diag(chns_mesh* m, const dev::PhysView& pv, int block, const double* U1, const double* U0,
                double* D, hipStream_t s) {
  const int64_t n = (int64_t)m->h.node_key.size();
  int rc = ensure_tbuf(m);
  if (rc) return rc;
  const auto mv = view(m);
  const auto pl = plan_view(m);
  const dim3 g((unsigned)m->n_chunks), b(dev::kChunkThreads);
  if (block == CHNS_BLOCK_CH) {
    hipLaunchKernelGGL((dev::k_diag<double, 0>), g, b, 0, s, mv, pl, pv, U1, U0, m->d_tbuf);
    hipLaunchKernelGGL(dev::k_gather_diag<2>, dim3(grid_stride(n)), dim3(256), 0, s, pl, n, m->d_tbuf, D);
  } else {
    hipLaunchKernelGGL((dev::k_diag<double, 1>), g, b, 0, s, mv, pl, pv, U1, U0, m->d_tbuf);
    hipLaunchKernelGGL(dev::k_gather_diag<4>, dim3(grid_stride(n)), dim3(256), 0, s, pl, n, m->d_tbuf, D);
  }
  HIPCHK(hipGetLastError());
  return CHNS_OK;
}

int launch_diagnostics(chns_mesh* m, const dev::PhysView& pv, const double* U, double* mass,
                       double* energy, hipStream_t s) {
  const int64_t E = (int64_t)m->h.leaf_key.size();
  const auto mv = view(m);
  const int nb = dev::diag_blocks(E);
  hipLaunchKernelGGL(dev::k_diagnostics, dim3(nb), dim3(256), 0, s, mv, pv, m->d_anchor,
                     std::ldexp(1.0, -m->h.D), U, m->d_part);
  hipLaunchKernelGGL(dev::k_finish_sum, dim3(2), dim3(256), 0, s, m->d_part, nb, 2, m->d_sum,
                     (const int*)nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(m->h_sum, m->d_sum, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *mass = m->h_sum[0];
  *energy = m->h_sum[1];
  return CHNS_OK;
}

// ------------------------------------------------------ multigrid setup ----
constexpr int64_t kMGCoarsest = 4096;  // automatic depth stops at this many nodes

int mg_alloc_level(MGLevel& L, bool coarse, int64_t* bytes) {
  std::lock_guard<std::mutex> lk(g_struct_mu);
  const size_t n = (size_t)L.n;
  int64_t* B = bytes;
  int rc;
  if ((rc = dalloc(&L.r64, 4 * n, B)) || (rc = dalloc(&L.r32, 4 * n, B))) return rc;
  if (!coarse) return CHNS_OK;
  if ((rc = dalloc(&L.U1, 6 * n, B)) || (rc = dalloc(&L.U0, 6 * n, B)) ||
      (rc = dalloc(&L.U1f, 6 * n, B)) || (rc = dalloc(&L.U0f, 6 * n, B)) ||
      (rc = dalloc(&L.D, 16 * n, B)) || (rc = dalloc(&L.Di, 16 * n, B)) ||
      (rc = dalloc(&L.Di32, 16 * n, B)) || (rc = dalloc(&L.DiC, 4 * n, B)) ||
      (rc = dalloc(&L.DiC32, 4 * n, B)) || (rc = dalloc(&L.b64, 4 * n, B)) ||
      (rc = dalloc(&L.x64, 4 * n, B)) || (rc = dalloc(&L.b32, 4 * n, B)) ||
      (rc = dalloc(&L.x32, 4 * n, B)))
    return rc;
  return CHNS_OK;
}

int mg_upload_transfer(MGLevel& F, const Transfer& t, hipStream_t s, int64_t* bytes) {
  // the restriction lists padded column-major, weights in FP32 (dyadic, exact)
  const int64_t nc = (int64_t)t.r_off.size() - 1;
  int64_t K = 0;
  for (int64_t j = 0; j < nc; ++j) K = std::max<int64_t>(K, t.r_off[j + 1] - t.r_off[j]);
  std::vector<int32_t> eidx((size_t)std::max<int64_t>(K * nc, 1), 0);
  std::vector<float> ew(eidx.size(), 0.0f);
  for (int64_t j = 0; j < nc; ++j)
    for (int64_t k = 0; k < t.r_off[j + 1] - t.r_off[j]; ++k) {
      const double w = t.r_w[t.r_off[j] + k];
      if ((double)(float)w != w) return fail(CHNS_EINVAL, "a restriction weight is not exact in FP32");
      eidx[k * nc + j] = t.r_idx[t.r_off[j] + k];
      ew[k * nc + j] = (float)w;
    }
  {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    int rc;
    if ((rc = dalloc(&F.p_off, t.p_off.size(), bytes)) || (rc = dalloc(&F.p_idx, t.p_idx.size(), bytes)) ||
        (rc = dalloc(&F.p_w, t.p_w.size(), bytes)) || (rc = dalloc(&F.r_off, t.r_off.size(), bytes)) ||
        (rc = dalloc(&F.r_eidx, eidx.size(), bytes)) || (rc = dalloc(&F.r_ew, ew.size(), bytes)) ||
        (rc = dalloc(&F.inj, t.inj.size(), bytes)))
      return rc;
  }
  int rc;
  if ((rc = h2d(F.p_off, t.p_off, s)) || (rc = h2d(F.p_idx, t.p_idx, s)) || (rc = h2d(F.p_w, t.p_w, s)) ||
      (rc = h2d(F.r_off, t.r_off, s)) || (rc = h2d(F.r_eidx, eidx, s)) || (rc = h2d(F.r_ew, ew, s)) ||
      (rc = h2d(F.inj, t.inj, s)))
    return rc;
  HIPCHK(hipStreamSynchronize(s));  // t is released by the caller
  return CHNS_OK;
}

// Builds (once per requested depth) the coarse meshes, their device copies,
// the transfers and the per-level buffers of the V-cycle.
int build_mg(chns_mesh* m, int levels, hipStream_t s) {
  if (m->mg_key == levels && !m->mg.empty()) return CHNS_OK;
  {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    drop_graphs(m->ws);
    free_mg_locked(m);
  }
  auto bail = [&](int rc) {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    free_mg_locked(m);
    return rc;
  };
  m->mg.resize(1);
  m->mg[0].mesh = m;
  m->mg[0].n = (int64_t)m->h.node_key.size();
  int rc = mg_alloc_level(m->mg[0], false, &m->mg_bytes);
  if (rc) return bail(rc);
  const int maxl = levels > 0 ? levels : 64;
  while ((int)m->mg.size() < maxl) {
    const size_t f = m->mg.size() - 1;
    const HostMesh& hf = m->mg[f].mesh->h;
    if (hf.D < 1) break;
    if (levels == 0 && ((int64_t)hf.node_key.size() <= kMGCoarsest || hf.D <= 1)) break;
    chns_mesh* c = new (std::nothrow) chns_mesh();
    if (!c) return bail(fail(CHNS_ENOMEM, "out of host memory"));
    Transfer t;
    std::string err;
    try {
      err = coarsen_host_mesh(hf, c->h);
      if (err.empty()) err = build_transfer(hf, c->h, t);
    } catch (const std::bad_alloc&) {
      err = "out of host memory while building the multigrid hierarchy";
    }
    if (!err.empty()) {
      delete c;
      return bail(fail(CHNS_EINVAL, err));
    }
    if ((rc = upload(c, s)) || (rc = ensure_tbuf(c))) {
      {
        std::lock_guard<std::mutex> lk(g_struct_mu);
        free_mesh_locked(c);
      }
      return bail(rc);
    }
    MGLevel C;
    C.mesh = c;
    C.n = (int64_t)c->h.node_key.size();
    m->mg.push_back(C);
    if ((rc = mg_alloc_level(m->mg.back(), true, &m->mg_bytes)) ||
        (rc = mg_upload_transfer(m->mg[f], t, s, &m->mg_bytes)))
      return bail(rc);
  }
  m->mg_key = levels;
  return CHNS_OK;
}

// --------------------------------------------------------------- solver ----
// The whole 6-field system of the fully coupled Newton solve (an internal
// block id next to CHNS_BLOCK_CH and CHNS_BLOCK_NS).
constexpr int kCoupled = 2;
inline int nf_of(int block) { return block == CHNS_BLOCK_CH ? 2 : (block == CHNS_BLOCK_NS ? 4 : 6); }

struct Solver {
  const std::atomic<bool>* cancel = nullptr;  // set by a server that is shutting down
  chns_mesh* m;
  dev::PhysView pv;
  chns_solver_opts o;
  hipStream_t s;
  Workspace& w;
  int64_t n;
  Solver(chns_mesh* m_, const dev::PhysView& pv_, const chns_solver_opts& o_, hipStream_t s_)
      : m(m_), pv(pv_), o(o_), s(s_), w(m_->ws), n((int64_t)m_->h.node_key.size()) {}

  bool cancelled() const { return cancel && cancel->load(std::memory_order_relaxed); }
  int singular = 0;  // Newton iterations of this step with a singular diagonal block

  int ensure_workspace() {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    int rc;
    int64_t& B = w.bytes;
    const int nfw = o.coupled ? 6 : 4;
    const size_t N = (size_t)n * std::max(nfw, w.n == n ? w.nfw : 0);
    if (w.n != n || w.nfw < nfw) {
      free_workspace(w);
      w.nfw = nfw;
      w.nb_part = (int)grid_stride((int64_t)N, 256, 1024);
      if ((rc = dalloc(&w.U1, n * 6, &B)) || (rc = dalloc(&w.Uk, n * 6, &B)) ||
          (rc = dalloc(&w.Uprev, n * 6, &B)) || (rc = dalloc(&w.r, N, &B)) || (rc = dalloc(&w.x, N, &B)) ||
          (rc = dalloc(&w.D, n * 16, &B)) || (rc = dalloc(&w.Di, n * 16, &B)) ||
          (rc = dalloc(&w.Di32, n * 16, &B)) || (rc = dalloc(&w.DiC, n * 4, &B)) ||
          (rc = dalloc(&w.DiC32, n * 4, &B)) || (rc = dalloc(&w.pk64, n * 4, &B)) ||
          (rc = dalloc(&w.pz64, n * 4, &B)) || (rc = dalloc(&w.pk32, n * 4, &B)) ||
          (rc = dalloc(&w.pz32, n * 4, &B)) ||
          (rc = dalloc(&w.part, (size_t)w.nb_part * (2 * dev::kMaxBasis + 2), &B)) ||
          (rc = dalloc(&w.dots, dev::kMaxBasis + 1, &B)) || (rc = dalloc(&w.flag, 1, &B)) ||
          (rc = dalloc(&w.ctl, 1, &B))) {
        free_workspace(w);
        return rc;
      }
      HIPCHK(hipHostMalloc((void**)&w.hdots, sizeof(double) * (dev::kMaxBasis + 1)));
      HIPCHK(hipHostMalloc((void**)&w.hflag, sizeof(int)));
      HIPCHK(hipHostMalloc((void**)&w.hctl, sizeof(int) * 8));
      HIPCHK(hipStreamCreateWithFlags(&w.cap, hipStreamNonBlocking));
      w.n = n;
    }
    const int restart = o.gmres_restart;
    if (o.precision == 0 && w.restart64 < restart) {
      free_basis(w, 0);
      if ((rc = dalloc(&w.V64, N * (restart + 1), &B)) || (rc = dalloc(&w.Z64, N * restart, &B)) ||
          (rc = dalloc(&w.w64, N, &B)) || (rc = dalloc(&w.b64, N, &B))) {
        free_basis(w, 0);
        return rc;
      }
      w.restart64 = restart;
    }
    if (o.precision == 1 && w.restart32 < restart) {
      free_basis(w, 1);
      if ((rc = dalloc(&w.V32, N * (restart + 1), &B)) || (rc = dalloc(&w.Z32, N * restart, &B)) ||
          (rc = dalloc(&w.w32, N, &B)) || (rc = dalloc(&w.b32, N, &B)) ||
          (rc = dalloc(&w.U1f, n * 6, &B)) || (rc = dalloc(&w.U0f, n * 6, &B))) {
        free_basis(w, 1);
        return rc;
      }
      w.restart32 = restart;
    }
    return CHNS_OK;
  }

  // sums the k partial rows left in w.part by a reduction kernel and copies
  // them to the host
  int finish_sums(int k, double* out) {
    hipLaunchKernelGGL(dev::k_finish_sum, dim3(k), dim3(256), 0, s, w.part, w.nb_part, k, w.dots,
                       (const int*)nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(w.hdots, w.dots, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j) out[j] = w.hdots[j];
    return CHNS_OK;
  }

  template <class TV>
  int dots(const TV* V, int64_t stride, int k, const TV* x, int64_t N, double* out) {
    hipLaunchKernelGGL(dev::k_multidot<TV>, dim3(w.nb_part, (k + dev::kDotTile - 1) / dev::kDotTile),
                       dim3(256), 0, s, V, stride, k, x, N, w.part,
                       (const int*)nullptr);
    return finish_sums(k, out);
  }

  template <class TV>
  int apply(int block, const TV* x, TV* y, const double* U1, const double* U0, const int* skip) {
    const int nf = block == CHNS_BLOCK_CH ? 2 : 4;
    if (block == kCoupled) {
      if (std::is_same<TV, double>::value)
        return launch_jvp_full<double, double, TV>(m, pv, (const double*)U1, (const double*)U0, x, y, s, skip);
      return launch_jvp_full<float, float, TV>(m, pv, w.U1f, w.U0f, x, y, s, skip);
    }
    return launch_jvp_lin<TV, TV>(m, pv, block, x, nf, 0, y, nf, 0, s, skip);
  }

  template <class TV>
  int precondition(int block, const TV* v, TV* z, const int* skip, const double* U1, const double* U0) {
    if (block == kCoupled) return precondition_coupled<TV>(v, z, skip, U1, U0);
    if (o.precond == 2) {
      if (block == CHNS_BLOCK_CH) return vcycle<TV, 2>(block, 0, v, z, skip, U1, U0);
      return vcycle<TV, 4>(block, 0, v, z, skip, U1, U0);
    }
    const dim3 g(grid_stride(n)), b(256);
    if (block == CHNS_BLOCK_CH) {
      if (std::is_same<TV, double>::value)
        hipLaunchKernelGGL((dev::k_precond<2, TV, double>), g, b, 0, s, w.DiC, v, z, n, skip);
      else
        hipLaunchKernelGGL((dev::k_precond<2, TV, float>), g, b, 0, s, w.DiC32, v, z, n, skip);
    } else {
      if (std::is_same<TV, double>::value)
        hipLaunchKernelGGL((dev::k_precond<4, TV, double>), g, b, 0, s, w.Di, v, z, n, skip);
      else
        hipLaunchKernelGGL((dev::k_precond<4, TV, float>), g, b, 0, s, w.Di32, v, z, n, skip);
    }
    HIPCHK(hipGetLastError());
    return CHNS_OK;
  }

  // Coupled system: the two blocks' preconditioners side by side (the cross
  // blocks of the Jacobian are left out of the preconditioner).
  template <class TV>
  int precondition_coupled(const TV* v, TV* z, const int* skip, const double* U1, const double* U0) {
    const bool dbl = std::is_same<TV, double>::value;
    TV* pk = dbl ? (TV*)w.pk64 : (TV*)w.pk32;
    TV* pz = dbl ? (TV*)w.pz64 : (TV*)w.pz32;
    const dim3 g(grid_stride(n)), b(256);
    int rc;
    for (int blk : {CHNS_BLOCK_CH, CHNS_BLOCK_NS}) {
      const int nf = blk == CHNS_BLOCK_CH ? 2 : 4, off = blk == CHNS_BLOCK_CH ? 0 : 2;
      hipLaunchKernelGGL(dev::k_pack<TV>, g, b, 0, s, v, 6, off, nf, n, pk, skip);
      if ((rc = precondition<TV>(blk, pk, pz, skip, U1, U0))) return rc;
      hipLaunchKernelGGL(dev::k_unpack<TV>, g, b, 0, s, pz, nf, n, z, 6, off, skip);
    }
    HIPCHK(hipGetLastError());
    return CHNS_OK;
  }

  // One V-cycle x = M^-1 b on level l of the hierarchy (x overwritten).
  // Level 0 is the Krylov system itself: its operator is the Jacobian of
  // (U1, U0) and its block inverse the Newton iteration's w.Di.
  template <class TV, int NF>
  int vcycle(int block, size_t l, const TV* b, TV* x, const int* skip, const double* U1, const double* U0,
             bool x_ready = false) {
    using TM = TV;  // the block inverse is used at the basis precision
    MGLevel& L = m->mg[l];
    chns_mesh* mm = L.mesh;
    const int64_t nl = L.n;
    const bool dbl = std::is_same<TV, double>::value;
    TV* r = dbl ? (TV*)L.r64 : (TV*)L.r32;
    const bool ch = block == CHNS_BLOCK_CH;
    const TM* Di = l == 0 ? (dbl ? (const TM*)(ch ? w.DiC : w.Di) : (const TM*)(ch ? w.DiC32 : w.Di32))
                          : (dbl ? (const TM*)(ch ? L.DiC : L.Di) : (const TM*)(ch ? L.DiC32 : L.Di32));
    const dim3 g(grid_stride(nl)), bl(256);
    const TV* part = (const TV*)mm->d_partial;
    const auto pl = plan_view(mm);
    // one sweep: the element pass of A x, then the node gather fused with the
    // Jacobi update (EPI 1) or with the residual b - A x into r (EPI 2)
    auto sweep = [&](bool residual) -> int {
      int rc = launch_jvp_lin_elements<TV, TV>(mm, pv, block, x, NF, 0, s, skip);
      if (rc) return rc;
      if (residual)
        hipLaunchKernelGGL((dev::k_gather_vcycle<NF, TV, TM, 2>), g, bl, 0, s, pl, nl, part, block, x, b, Di,
                           o.mg_omega, r, skip);
      else
        hipLaunchKernelGGL((dev::k_gather_vcycle<NF, TV, TM, 1>), g, bl, 0, s, pl, nl, part, block, x, b, Di,
                           o.mg_omega, r, skip);
      return CHNS_OK;
    };
    const bool coarsest = l + 1 == m->mg.size();
    const int pre = coarsest ? o.mg_coarse_sweeps : o.mg_smooth;
    int rc;
    if (!x_ready)  // x = omega Di b (coarser levels get it from the restriction)
      hipLaunchKernelGGL((dev::k_jacobi<NF, TV, TM>), g, bl, 0, s, Di, b, (const TV*)nullptr, x, mm->d_bflags,
                         block, o.mg_omega, nl, skip);
    for (int i = 1; i < pre; ++i)
      if ((rc = sweep(false))) return rc;
    if (coarsest) {
      HIPCHK(hipGetLastError());
      return CHNS_OK;
    }
    if ((rc = sweep(true))) return rc;
    MGLevel& C = m->mg[l + 1];
    TV* bc = dbl ? (TV*)C.b64 : (TV*)C.b32;
    TV* xc = dbl ? (TV*)C.x64 : (TV*)C.x32;
    const TM* Dic = dbl ? (const TM*)(ch ? C.DiC : C.Di) : (const TM*)(ch ? C.DiC32 : C.Di32);
    hipLaunchKernelGGL((dev::k_restrict<NF, TV, TM>), dim3(grid_stride(C.n)), bl, 0, s, r, L.r_off, L.r_eidx,
                       L.r_ew, C.n, C.mesh->d_bflags, block, bc, Dic, o.mg_omega, xc, skip);
    if ((rc = vcycle<TV, NF>(block, l + 1, bc, xc, skip, U1, U0, true))) return rc;
    hipLaunchKernelGGL((dev::k_prolong_add<NF, TV>), g, bl, 0, s, x, mm->d_bflags, L.p_off, L.p_idx, L.p_w, nl,
                       xc, block, skip);
    for (int i = 0; i < o.mg_smooth; ++i)
      if ((rc = sweep(false))) return rc;
    HIPCHK(hipGetLastError());
    return CHNS_OK;
  }

  // Coarse-level states (injected from the level above) and node-block
  // diagonals, once per Newton iteration.
  int mg_setup(int block, const double* U1, const double* U0) {
    const int nf = block == CHNS_BLOCK_CH ? 2 : 4;
    for (size_t l = 1; l < m->mg.size(); ++l) {
      MGLevel& F = m->mg[l - 1];
      MGLevel& C = m->mg[l];
      const double* s1 = l == 1 ? U1 : F.U1;
      const double* s0 = l == 1 ? U0 : F.U0;
      const dim3 g(grid_stride(C.n * 6)), b(256);
      hipLaunchKernelGGL(dev::k_inject6, g, b, 0, s, s1, F.inj, C.n, C.U1, C.U1f);
      hipLaunchKernelGGL(dev::k_inject6, g, b, 0, s, s0, F.inj, C.n, C.U0, C.U0f);
      int rc = launch_diag(C.mesh, pv, block, C.U1, C.U0, C.D, s);
      if (rc) return rc;
      rc = o.precision == 0 ? launch_lin<double, double>(C.mesh, pv, block, C.U1, C.U0, s)
                            : launch_lin<float, float>(C.mesh, pv, block, C.U1f, C.U0f, s);
      if (rc) return rc;
      if (nf == 2)
        hipLaunchKernelGGL(dev::k_invert_blocks<2>, dim3(grid_for(C.n)), b, 0, s, C.D, C.DiC, C.DiC32, C.n, 0,
                           w.flag);
      else
        hipLaunchKernelGGL(dev::k_invert_blocks<4>, dim3(grid_for(C.n)), b, 0, s, C.D, C.Di, C.Di32, C.n, 0,
                           w.flag);
    }
    HIPCHK(hipGetLastError());
    return CHNS_OK;
  }

  // Right-preconditioned restarted GMRES(mres) with classical Gram-Schmidt
  // twice, the second pass delayed into the next step (k_dc_* in
  // linalg.hpp), all control on the device (GmresCtl).  A cycle is enqueued in
  // parts: Arnoldi steps [k0, k1), then the tail (the last provisional
  // vector's second pass, the least-squares update x += Z~ R^-1 y, the true
  // residual b - J x and the start of the next cycle).
  // Steps after the stop test has fired return at once; nothing is read back
  // here.
  static constexpr int kSegment = 16;  // Arnoldi steps between host checks

  template <class TV>
  int enqueue_steps(int block, TV* V, TV* Z, TV* wv, const double* U1, const double* U0, int k0,
                    int k1) {
    const int nf = nf_of(block);
    const int64_t N = n * nf;
    dev::GmresCtl* C = w.ctl;
    const int* idle = &C->idle;
    const dim3 b(256);
    int rc;
    for (int k = k0; k < k1; ++k) {
      TV* Vk = V + (int64_t)k * N;
      TV* Zk = Z + (int64_t)k * N;
      const dim3 gp(w.nb_part, std::max(1, (k + dev::kDcTile - 1) / dev::kDcTile));
      if ((rc = precondition<TV>(block, Vk, Zk, idle, U1, U0))) return rc;
      if ((rc = apply<TV>(block, Zk, wv, U1, U0, idle))) return rc;
      hipLaunchKernelGGL(dev::k_dc_dots<TV>, gp, b, 0, s, V, N, k, (const int*)nullptr, wv, N, w.part, idle);
      hipLaunchKernelGGL(dev::k_finish_sum, dim3(2 * k + 2), b, 0, s, w.part, w.nb_part, 2 * k + 2, C->dsum, idle);
      hipLaunchKernelGGL(dev::k_dc_coef, dim3(1), b, 0, s, C, k);
      hipLaunchKernelGGL(dev::k_dc_update<TV>, dim3(w.nb_part), b, 0, s, V, N, k, wv, N, C, w.part, idle);
      hipLaunchKernelGGL(dev::k_dc_norm, dim3(1), b, 0, s, C, k, w.part, w.nb_part);
    }
    HIPCHK(hipGetLastError());
    return CHNS_OK;
  }

  template <class TV>
  int enqueue_tail(int block, TV* V, TV* Z, TV* wv, const TV* bvec, const double* U1, const double* U0) {
    const int nf = nf_of(block);
    const int64_t N = n * nf;
    dev::GmresCtl* C = w.ctl;
    const int* fin = &C->finished;
    const dim3 gs(grid_stride(N)), b(256);
    int rc;
    // the second pass of the cycle's last provisional vector (k = C->kfin <= mres)
    const int mres = std::max(1, std::min(o.gmres_restart, dev::kMaxBasis - 1));
    const dim3 gp(w.nb_part, std::max(1, (mres + dev::kDcTile - 1) / dev::kDcTile));
    hipLaunchKernelGGL(dev::k_dc_dots<TV>, gp, b, 0, s, V, N, 0, &C->kfin, (const TV*)nullptr, N, w.part,
                       &C->noprov);
    hipLaunchKernelGGL(dev::k_finish_sum_n, dim3(2 * mres + 2), b, 0, s, w.part, w.nb_part, &C->nfin, C->dsum,
                       &C->noprov);
    hipLaunchKernelGGL(dev::k_dc_final, dim3(1), b, 0, s, C);
    hipLaunchKernelGGL(dev::k_gmres_solve, dim3(1), b, 0, s, C);
    hipLaunchKernelGGL(dev::k_multi_update<TV>, gs, b, 0, s, w.x, Z, N, &C->ncols, C->y, N);
    hipLaunchKernelGGL((dev::k_convert<double, TV>), gs, b, 0, s, w.x, Z, N, fin);
    if ((rc = apply<TV>(block, Z, wv, U1, U0, fin))) return rc;
    hipLaunchKernelGGL(dev::k_rsub<TV>, gs, b, 0, s, wv, bvec, N, fin);
    hipLaunchKernelGGL(dev::k_multidot<TV>, dim3(w.nb_part), b, 0, s, wv, 0, 1, wv, N, w.part, fin);
    hipLaunchKernelGGL(dev::k_gmres_restart, dim3(1), b, 0, s, C, w.part, w.nb_part);
    hipLaunchKernelGGL(dev::k_scale_dev<TV>, gs, b, 0, s, V, wv, &C->inv_scale, N, fin);
    HIPCHK(hipGetLastError());
    return CHNS_OK;
  }

  // Enqueues part `seg` of a cycle (seg < 0: the tail), directly or as a HIP
  // graph captured on the workspace's own stream the first time this (block,
  // basis type, restart length, parameters, part) is seen.  Every pointer in
  // a graph belongs to the mesh or its workspace, so it stays valid until
  // the workspace is reallocated (which drops the cache).
  template <class TV>
  int enqueue_part(int block, TV* V, TV* Z, TV* wv, const TV* bvec, const double* U1,
                   const double* U0, int mres, int seg) {
    auto direct = [&]() {
      if (seg < 0) return enqueue_tail<TV>(block, V, Z, wv, bvec, U1, U0);
      return enqueue_steps<TV>(block, V, Z, wv, U1, U0, seg * kSegment,
                               std::min(mres, (seg + 1) * kSegment));
    };
    if (!o.graphs) return direct();
    const int tv = std::is_same<TV, double>::value ? 0 : 1;
    hipGraphExec_t ex = nullptr;
    for (auto& g : w.graphs)
      if (g.block == block && g.tv == tv && g.mres == mres && g.seg == seg && g.precond == o.precond &&
          g.mg_levels == o.mg_levels && g.mg_smooth == o.mg_smooth && g.mg_coarse == o.mg_coarse_sweeps &&
          g.mg_omega == o.mg_omega && std::memcmp(&g.pv, &pv, sizeof(pv)) == 0) {
        ex = g.exec;
        break;
      }
    if (!ex) {
      std::lock_guard<std::mutex> lk(g_struct_mu);
      if (w.graphs.size() >= 64) drop_graphs(w);
      hipGraph_t graph = nullptr;
      hipStream_t caller = s;
      s = w.cap;
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      const int rc = direct();
      const hipError_t e = hipStreamEndCapture(s, &graph);
      s = caller;
      if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (e != hipSuccess) return fail(CHNS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      CycleGraph g;
      g.block = block;
      g.tv = tv;
      g.mres = mres;
      g.seg = seg;
      g.precond = o.precond;
      g.mg_levels = o.mg_levels;
      g.mg_smooth = o.mg_smooth;
      g.mg_coarse = o.mg_coarse_sweeps;
      g.mg_omega = o.mg_omega;
      g.pv = pv;
      const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return fail(CHNS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
      w.graphs.push_back(g);
      ex = g.exec;
    }
    HIPCHK(hipGraphLaunch(ex, s));
    return CHNS_OK;
  }

  int read_ctl() {
    HIPCHK(hipMemcpyAsync(w.hctl, w.ctl, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (w.hctl[3]) return fail(CHNS_ENONFINITE, "non-finite value in GMRES");
    return CHNS_OK;
  }

  // Solves J x = b (b in bvec) from x0 = 0; x returned in w.x (FP64).  The
  // host checks the device's stop flags after every kSegment Arnoldi steps
  // and after each cycle's tail.
  template <class TV>
  int gmres(int block, TV* V, TV* Z, TV* wv, TV* bvec, const double* U1, const double* U0,
            int* its) {
    const int nf = nf_of(block);
    const int64_t N = n * nf;
    const int mres = std::max(1, std::min(o.gmres_restart, dev::kMaxBasis - 1));
    const int nseg = (mres + kSegment - 1) / kSegment;
    const dim3 gs(grid_stride(N)), b(256);
    dev::GmresCtl* C = w.ctl;
    hipLaunchKernelGGL(dev::k_fill<double>, gs, b, 0, s, w.x, N, 0.0);
    hipLaunchKernelGGL(dev::k_multidot<TV>, dim3(w.nb_part), b, 0, s, bvec, 0, 1, bvec, N, w.part,
                       (const int*)nullptr);
    hipLaunchKernelGGL(dev::k_gmres_begin, dim3(1), b, 0, s, C, w.part, w.nb_part, o.gmres_max_it, mres,
                       o.gmres_rtol);
    hipLaunchKernelGGL(dev::k_scale_dev<TV>, gs, b, 0, s, V, bvec, &C->inv_scale, N, &C->finished);
    int rc;
    for (;;) {
      for (int seg = 0; seg < nseg; ++seg) {
        if ((rc = enqueue_part<TV>(block, V, Z, wv, bvec, U1, U0, mres, seg))) return rc;
        if (seg + 1 < nseg) {
          if ((rc = read_ctl())) return rc;
          if (w.hctl[0]) break;  // idle: the cycle ended early
        }
      }
      if ((rc = enqueue_part<TV>(block, V, Z, wv, bvec, U1, U0, mres, -1))) return rc;
      if ((rc = read_ctl())) return rc;
      if (w.hctl[1]) break;
      if (cancelled()) return fail(CHNS_ECANCELED, "step cancelled");
    }
    *its = w.hctl[2];
    return CHNS_OK;
  }

  int residual_norm(int block, double* U, double* rn) {
    const int nf = nf_of(block);
    int rc;
    if (block == kCoupled) {  // both blocks' rows, node-major 6 per node
      if ((rc = launch_residual(m, pv, CHNS_BLOCK_CH, U, w.Uk, w.r, 6, 0, s, false)) ||
          (rc = launch_residual(m, pv, CHNS_BLOCK_NS, U, w.Uk, w.r, 6, 2, s, true, true)))
        return rc;
    } else if ((rc = launch_residual(m, pv, block, U, w.Uk, w.r, nf, 0, s, block == CHNS_BLOCK_NS))) {
      return rc;
    }
    double d;
    if ((rc = dots<double>(w.r, 0, 1, w.r, n * nf, &d))) return rc;
    *rn = std::sqrt(d);
    return CHNS_OK;
  }

  int newton(int block, double* U, int* nits, int* gits, double* relres, bool* conv) {
    const int nf = block == CHNS_BLOCK_CH ? 2 : 4, f0 = block == CHNS_BLOCK_CH ? 0 : 2;
    const int max_it = block == CHNS_BLOCK_CH ? o.newton_max_it_ch : o.newton_max_it_ns;
    const int64_t N = n * nf;
    double r0, rn;
    int rc = residual_norm(block, U, &r0);
    if (rc) return rc;
    rn = r0;
    *conv = false;
    for (;;) {
      if (!std::isfinite(rn)) return fail(CHNS_ENONFINITE, "non-finite Newton residual");
      if (rn <= std::max(o.newton_rtol * r0, o.newton_atol)) {
        *conv = true;
        break;
      }
      if (*nits >= max_it) break;
      if (cancelled()) return fail(CHNS_ECANCELED, "step cancelled");
      if ((rc = launch_diag(m, pv, block, U, w.Uk, w.D, s))) return rc;
      hipLaunchKernelGGL(dev::k_fill<int>, dim3(1), dim3(64), 0, s, w.flag, (int64_t)1, 0);
      if (nf == 2)
        hipLaunchKernelGGL(dev::k_invert_blocks<2>, dim3(grid_for(n)), dim3(256), 0, s, w.D, w.DiC, w.DiC32,
                           n, o.precond == 0 ? 1 : 0, w.flag);
      else
        hipLaunchKernelGGL(dev::k_invert_blocks<4>, dim3(grid_for(n)), dim3(256), 0, s, w.D, w.Di, w.Di32,
                           n, o.precond == 0 ? 1 : 0, w.flag);
      HIPCHK(hipGetLastError());
      if (o.precond == 2 && (rc = mg_setup(block, U, w.Uk))) return rc;
      // the singular-block flag of these inversions, read after the next sync
      HIPCHK(hipMemcpyAsync(w.hflag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
      int its = 0;
      if (o.precision == 0) {
        hipLaunchKernelGGL((dev::k_scale<double, double>), dim3(grid_stride(N)), dim3(256), 0, s, w.b64,
                           w.r, -1.0, N);
        if ((rc = launch_lin<double, double>(m, pv, block, U, w.Uk, s))) return rc;
        rc = gmres<double>(block, w.V64, w.Z64, w.w64, w.b64, U, w.Uk, &its);
      } else {
        hipLaunchKernelGGL((dev::k_convert<double, float>), dim3(grid_stride(n * 6)), dim3(256), 0, s, U,
                           w.U1f, n * 6, (const int*)nullptr);
        hipLaunchKernelGGL((dev::k_convert<double, float>), dim3(grid_stride(n * 6)), dim3(256), 0, s,
                           w.Uk, w.U0f, n * 6, (const int*)nullptr);
        hipLaunchKernelGGL((dev::k_scale<double, float>), dim3(grid_stride(N)), dim3(256), 0, s, w.b32,
                           w.r, -1.0, N);
        if ((rc = launch_lin<float, float>(m, pv, block, w.U1f, w.U0f, s))) return rc;
        rc = gmres<float>(block, w.V32, w.Z32, w.w32, w.b32, U, w.Uk, &its);
      }
      if (rc) return rc;
      *gits += its;
      hipLaunchKernelGGL(dev::k_add_block<double>, dim3(grid_stride(N)), dim3(256), 0, s, U, w.x, n, f0, nf, 1.0);
      ++*nits;
      if ((rc = residual_norm(block, U, &rn))) return rc;  // synchronises the stream
      if (*w.hflag & 2) ++singular;
    }
    *relres = r0 > 0 ? rn / r0 : 0.0;
    return CHNS_OK;
  }

  // Newton on the whole 6-field system R(U^{k+1}) = [R_CH; R_NS] = 0 with the
  // coupled Jacobian (no block iteration); the preconditioner is the two
  // blocks' own (node-block Jacobi or the multigrid V-cycle), side by side.
  int newton_coupled(double* U, int* nits, int* gits, double* relres, bool* conv) {
    const int64_t N = n * 6;
    double r0, rn;
    int rc = residual_norm(kCoupled, U, &r0);
    if (rc) return rc;
    rn = r0;
    *conv = false;
    for (;;) {
      if (!std::isfinite(rn)) return fail(CHNS_ENONFINITE, "non-finite Newton residual");
      if (rn <= std::max(o.newton_rtol * r0, o.newton_atol)) {
        *conv = true;
        break;
      }
      if (*nits >= o.newton_max_it_ns) break;
      if (cancelled()) return fail(CHNS_ECANCELED, "step cancelled");
      hipLaunchKernelGGL(dev::k_fill<int>, dim3(1), dim3(64), 0, s, w.flag, (int64_t)1, 0);
      if ((rc = launch_diag(m, pv, CHNS_BLOCK_CH, U, w.Uk, w.D, s))) return rc;
      hipLaunchKernelGGL(dev::k_invert_blocks<2>, dim3(grid_for(n)), dim3(256), 0, s, w.D, w.DiC, w.DiC32, n,
                         o.precond == 0 ? 1 : 0, w.flag);
      if ((rc = launch_diag(m, pv, CHNS_BLOCK_NS, U, w.Uk, w.D, s))) return rc;
      hipLaunchKernelGGL(dev::k_invert_blocks<4>, dim3(grid_for(n)), dim3(256), 0, s, w.D, w.Di, w.Di32, n,
                         o.precond == 0 ? 1 : 0, w.flag);
      HIPCHK(hipGetLastError());
      if (o.precond == 2 && ((rc = mg_setup(CHNS_BLOCK_CH, U, w.Uk)) || (rc = mg_setup(CHNS_BLOCK_NS, U, w.Uk))))
        return rc;
      HIPCHK(hipMemcpyAsync(w.hflag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
      int its = 0;
      if (o.precision == 0) {
        hipLaunchKernelGGL((dev::k_scale<double, double>), dim3(grid_stride(N)), dim3(256), 0, s, w.b64, w.r,
                           -1.0, N);
        if (o.precond == 2 && ((rc = launch_lin<double, double>(m, pv, CHNS_BLOCK_CH, U, w.Uk, s)) ||
                               (rc = launch_lin<double, double>(m, pv, CHNS_BLOCK_NS, U, w.Uk, s))))
          return rc;
        rc = gmres<double>(kCoupled, w.V64, w.Z64, w.w64, w.b64, U, w.Uk, &its);
      } else {
        hipLaunchKernelGGL((dev::k_convert<double, float>), dim3(grid_stride(n * 6)), dim3(256), 0, s, U,
                           w.U1f, n * 6, (const int*)nullptr);
        hipLaunchKernelGGL((dev::k_convert<double, float>), dim3(grid_stride(n * 6)), dim3(256), 0, s, w.Uk,
                           w.U0f, n * 6, (const int*)nullptr);
        hipLaunchKernelGGL((dev::k_scale<double, float>), dim3(grid_stride(N)), dim3(256), 0, s, w.b32, w.r,
                           -1.0, N);
        if (o.precond == 2 && ((rc = launch_lin<float, float>(m, pv, CHNS_BLOCK_CH, w.U1f, w.U0f, s)) ||
                               (rc = launch_lin<float, float>(m, pv, CHNS_BLOCK_NS, w.U1f, w.U0f, s))))
          return rc;
        rc = gmres<float>(kCoupled, w.V32, w.Z32, w.w32, w.b32, U, w.Uk, &its);
      }
      if (rc) return rc;
      *gits += its;
      hipLaunchKernelGGL(dev::k_add_block<double>, dim3(grid_stride(N)), dim3(256), 0, s, U, w.x, n, 0, 6, 1.0);
      ++*nits;
      if ((rc = residual_norm(kCoupled, U, &rn))) return rc;  // synchronises the stream
      if (*w.hflag & 2) ++singular;
    }
    *relres = r0 > 0 ? rn / r0 : 0.0;
    return CHNS_OK;
  }

  int max_change(const double* a, const double* b, double* out) {
    const int64_t N = n * 6;
    hipLaunchKernelGGL(dev::k_maxabs_diff, dim3(w.nb_part), dim3(256), 0, s, a, b, N, w.part);
    hipLaunchKernelGGL(dev::k_finish_max, dim3(1), dim3(256), 0, s, w.part, w.nb_part, w.dots);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(w.hdots, w.dots, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = w.hdots[0];
    return CHNS_OK;
  }

  // The step works on the workspace copy w.U1 of the caller's U, so that the
  // captured GMRES cycles only ever see workspace pointers.
  int step(double* Uout, chns_step_stats* st) {
    int rc = ensure_workspace();
    if (rc) return rc;
    singular = 0;
    if (o.precond == 2 && (rc = build_mg(m, o.mg_levels, s))) return rc;
    double* U = w.U1;
    HIPCHK(hipMemcpyAsync(U, Uout, sizeof(double) * n * 6, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(w.Uk, Uout, sizeof(double) * n * 6, hipMemcpyDeviceToDevice, s));
    double r_init[2];
    for (int b : {CHNS_BLOCK_CH, CHNS_BLOCK_NS})
      if ((rc = residual_norm(b, U, &r_init[b]))) return rc;
    bool all_conv = true, block_conv = false;
    if (o.coupled) {  // one Newton solve of the whole system replaces the block iteration
      int nits = 0, gits = 0;
      double rr = 0;
      bool conv = false;
      if ((rc = newton_coupled(U, &nits, &gits, &rr, &conv))) return rc;
      st->block_its = 1;
      st->newton_its[CHNS_BLOCK_NS] = nits;
      st->gmres_its[CHNS_BLOCK_NS] = gits;
      all_conv = conv;
      block_conv = true;
    }
    for (int l = 0; !o.coupled && l < o.block_max_it; ++l) {
      HIPCHK(hipMemcpyAsync(w.Uprev, U, sizeof(double) * n * 6, hipMemcpyDeviceToDevice, s));
      for (int b : {CHNS_BLOCK_NS, CHNS_BLOCK_CH}) {
        int nits = 0, gits = 0;
        double rr = 0;
        bool conv = false;
        if ((rc = newton(b, U, &nits, &gits, &rr, &conv))) return rc;
        st->newton_its[b] += nits;
        st->gmres_its[b] += gits;
        all_conv = all_conv && conv;
      }
      st->block_its = l + 1;
      if (l >= o.block_min_it) {
        double ch;
        if ((rc = max_change(U, w.Uprev, &ch))) return rc;
        if (!std::isfinite(ch)) return fail(CHNS_ENONFINITE, "non-finite block change");
        if (ch <= o.block_tol) {
          block_conv = true;
          break;
        }
      }
    }
    for (int b : {CHNS_BLOCK_CH, CHNS_BLOCK_NS}) {
      double rf;
      if ((rc = residual_norm(b, U, &rf))) return rc;
      st->rel_res[b] = r_init[b] > 0 ? rf / r_init[b] : 0.0;
    }
    HIPCHK(hipMemcpyAsync(Uout, U, sizeof(double) * n * 6, hipMemcpyDeviceToDevice, s));
    if ((rc = launch_diagnostics(m, pv, U, &st->mass, &st->energy, s))) return rc;
    st->converged = (all_conv && block_conv) ? 1 : 0;
    st->singular_blocks = singular;
    return st->converged ? CHNS_OK : CHNS_NOT_CONVERGED;
  }
};

}  // namespace

int check_opts(const chns_solver_opts* opts) {
  if (opts->gmres_restart < 1 || opts->gmres_restart > dev::kMaxBasis - 1)
    return fail(CHNS_EINVAL, "gmres_restart must be in [1, " + std::to_string(dev::kMaxBasis - 1) + "]");
  if (opts->precision != 0 && opts->precision != 1) return fail(CHNS_EINVAL, "precision must be 0 or 1");
  if (opts->precond < 0 || opts->precond > 2) return fail(CHNS_EINVAL, "precond must be 0, 1 or 2");
  if (opts->coupled != 0 && opts->coupled != 1) return fail(CHNS_EINVAL, "coupled must be 0 or 1");
  if (opts->precond == 2) {
    if (!(opts->mg_omega > 0.0 && opts->mg_omega < 2.0)) return fail(CHNS_EINVAL, "mg_omega must be in (0, 2)");
    if (opts->mg_smooth < 1 || opts->mg_smooth > 16 || opts->mg_coarse_sweeps < 1 ||
        opts->mg_coarse_sweeps > 256 || opts->mg_levels < 0 || opts->mg_levels > 16)
      return fail(CHNS_EINVAL, "mg_smooth in [1, 16], mg_coarse_sweeps in [1, 256], mg_levels in [0, 16]");
  }
  if (opts->block_max_it < 1 || opts->gmres_max_it < 1)
    return fail(CHNS_EINVAL, "iteration limits must be positive");
  if (opts->newton_max_it_ch < 0 || opts->newton_max_it_ns < 0 || opts->block_min_it < 0)
    return fail(CHNS_EINVAL, "iteration limits must not be negative");
  return CHNS_OK;
}

// =================================================================== ABI ==
extern "C" {

const char* chns_last_error(void) { return g_err.c_str(); }

int chns_mesh_build(const chns_mesh_spec* spec, chns_mesh** out) {
  if (!spec || !out) return fail(CHNS_EINVAL, "spec and out must not be NULL");
  *out = nullptr;
  chns_mesh* m = new (std::nothrow) chns_mesh();
  if (!m) return fail(CHNS_ENOMEM, "out of host memory");
  std::string err;
  try {
    err = build_host_mesh(*spec, m->h);
  } catch (const std::bad_alloc&) {
    err = "out of host memory while building the mesh";
  }
  if (!err.empty()) {
    delete m;
    return fail(err.find("memory") != std::string::npos ? CHNS_ENOMEM : CHNS_EINVAL, err);
  }
  *out = m;
  return CHNS_OK;
}

int chns_mesh_info(const chns_mesh* m, chns_mesh_stats* out) {
  if (!m || !out) return fail(CHNS_EINVAL, "mesh and out must not be NULL");
  out->n_leaves = (int64_t)m->h.leaf_key.size();
  out->n_nodes = (int64_t)m->h.node_key.size();
  out->n_hanging = (int64_t)m->h.hang_key.size();
  out->n_constraint = (int64_t)m->h.hang_ids.size();
  out->level_max = m->h.D;
  out->max_fanin = m->h.max_fanin;
  int64_t b = m->device_bytes + m->ws.bytes + m->mg_bytes;
  for (size_t l = 1; l < m->mg.size(); ++l)
    if (m->mg[l].mesh) b += m->mg[l].mesh->device_bytes + m->mg[l].mesh->ws.bytes;
  out->device_bytes = b;
  return CHNS_OK;
}

int chns_mesh_arrays(const chns_mesh* m, int32_t* leaves, int32_t* elem, int32_t* nodes,
                     uint8_t* bflags, int32_t* hang_xyz, int64_t* hang_off, int32_t* hang_ids,
                     double* hang_w) {
  if (!m) return fail(CHNS_EINVAL, "mesh is NULL");
  const HostMesh& h = m->h;
  const size_t E = h.leaf_key.size();
  for (size_t e = 0; e < E; ++e) {
    uint32_t x, y, z;
    unkey(h.leaf_key[e], x, y, z);
    if (leaves) {
      leaves[4 * e] = (int32_t)x;
      leaves[4 * e + 1] = (int32_t)y;
      leaves[4 * e + 2] = (int32_t)z;
      leaves[4 * e + 3] = h.leaf_level[e];
    }
  }
  if (elem) std::memcpy(elem, h.elem.data(), h.elem.size() * sizeof(int32_t));
  for (size_t i = 0; i < h.node_key.size(); ++i) {
    uint32_t x, y, z;
    unkey(h.node_key[i], x, y, z);
    if (nodes) {
      nodes[3 * i] = (int32_t)x;
      nodes[3 * i + 1] = (int32_t)y;
      nodes[3 * i + 2] = (int32_t)z;
    }
    if (bflags) bflags[i] = h.bflags[i];
  }
  for (size_t i = 0; i < h.hang_key.size(); ++i) {
    uint32_t x, y, z;
    unkey(h.hang_key[i], x, y, z);
    if (hang_xyz) {
      hang_xyz[3 * i] = (int32_t)x;
      hang_xyz[3 * i + 1] = (int32_t)y;
      hang_xyz[3 * i + 2] = (int32_t)z;
    }
  }
  if (hang_off)
    for (size_t i = 0; i < h.hang_off.size(); ++i) hang_off[i] = h.hang_off[i];
  if (hang_ids) std::memcpy(hang_ids, h.hang_ids.data(), h.hang_ids.size() * sizeof(int32_t));
  if (hang_w) std::memcpy(hang_w, h.hang_w.data(), h.hang_w.size() * sizeof(double));
  return CHNS_OK;
}

int chns_mesh_nodes(const chns_mesh* m, double* xyz, uint8_t* bflags) {
  if (!m) return fail(CHNS_EINVAL, "mesh is NULL");
  const double unit = std::ldexp(1.0, -m->h.D);
  for (size_t i = 0; i < m->h.node_key.size(); ++i) {
    uint32_t x, y, z;
    unkey(m->h.node_key[i], x, y, z);
    if (xyz) {
      xyz[3 * i] = x * unit;
      xyz[3 * i + 1] = y * unit;
      xyz[3 * i + 2] = z * unit;
    }
    if (bflags) bflags[i] = m->h.bflags[i];
  }
  return CHNS_OK;
}

int chns_mesh_coarsen(const chns_mesh* m, chns_mesh** out) {
  if (!m || !out) return fail(CHNS_EINVAL, "mesh and out must not be NULL");
  *out = nullptr;
  chns_mesh* c = new (std::nothrow) chns_mesh();
  if (!c) return fail(CHNS_ENOMEM, "out of host memory");
  std::string err;
  try {
    err = coarsen_host_mesh(m->h, c->h);
  } catch (const std::bad_alloc&) {
    err = "out of host memory while coarsening the mesh";
  }
  if (!err.empty()) {
    delete c;
    return fail(CHNS_EINVAL, err);
  }
  *out = c;
  return CHNS_OK;
}

int chns_mesh_transfer(const chns_mesh* f, const chns_mesh* c, int64_t* nnz, int32_t* p_off,
                       int32_t* p_idx, double* p_w, int32_t* inj) {
  if (!f || !c) return fail(CHNS_EINVAL, "meshes must not be NULL");
  Transfer t;
  std::string err;
  try {
    err = build_transfer(f->h, c->h, t);
  } catch (const std::bad_alloc&) {
    err = "out of host memory while building the transfer";
  }
  if (!err.empty()) return fail(CHNS_EINVAL, err);
  if (nnz) *nnz = (int64_t)t.p_idx.size();
  if (p_off) std::memcpy(p_off, t.p_off.data(), t.p_off.size() * sizeof(int32_t));
  if (p_idx) std::memcpy(p_idx, t.p_idx.data(), t.p_idx.size() * sizeof(int32_t));
  if (p_w) std::memcpy(p_w, t.p_w.data(), t.p_w.size() * sizeof(double));
  if (inj) std::memcpy(inj, t.inj.data(), t.inj.size() * sizeof(int32_t));
  return CHNS_OK;
}

int chns_mesh_remesh(const chns_mesh* m, const double* U_host, int level_min, int level_max, double band,
                     chns_mesh** out) {
  if (!m || !U_host || !out) return fail(CHNS_EINVAL, "mesh, U_host and out must not be NULL");
  *out = nullptr;
  chns_mesh* c = new (std::nothrow) chns_mesh();
  if (!c) return fail(CHNS_ENOMEM, "out of host memory");
  std::string err;
  try {
    err = remesh_host(m->h, U_host, level_min, level_max, band, c->h);
  } catch (const std::bad_alloc&) {
    err = "out of host memory while remeshing";
  }
  if (!err.empty()) {
    delete c;
    return fail(err.find("memory") != std::string::npos ? CHNS_ENOMEM : CHNS_EINVAL, err);
  }
  *out = c;
  return CHNS_OK;
}

int chns_mesh_interp_weights(const chns_mesh* from, const chns_mesh* to, int64_t* nnz, int32_t* off,
                             int32_t* idx, double* w) {
  if (!from || !to) return fail(CHNS_EINVAL, "meshes must not be NULL");
  std::vector<int32_t> o, ix;
  std::vector<double> ww;
  std::string err;
  try {
    err = build_interp(from->h, to->h, o, ix, ww);
  } catch (const std::bad_alloc&) {
    err = "out of host memory while building the transfer";
  }
  if (!err.empty()) return fail(CHNS_EINVAL, err);
  if (nnz) *nnz = (int64_t)ix.size();
  if (off) std::memcpy(off, o.data(), o.size() * sizeof(int32_t));
  if (idx) std::memcpy(idx, ix.data(), ix.size() * sizeof(int32_t));
  if (w) std::memcpy(w, ww.data(), ww.size() * sizeof(double));
  return CHNS_OK;
}

int chns_mesh_interpolate(chns_mesh* from, chns_mesh* to, const double* U_from, double* U_to,
                          const chns_params* params, int conserve_mass, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (!from || !to || !U_from || !U_to) return fail(CHNS_EINVAL, "NULL argument");
  if (conserve_mass && !params) return fail(CHNS_EINVAL, "conserve_mass needs params");
  int rc;
  if ((rc = check_mesh(from, s)) || (rc = check_mesh(to, s))) return rc;
  std::vector<int32_t> o, ix;
  std::vector<double> ww;
  std::string err;
  try {
    err = build_interp(from->h, to->h, o, ix, ww);
  } catch (const std::bad_alloc&) {
    err = "out of host memory while building the transfer";
  }
  if (!err.empty()) return fail(CHNS_EINVAL, err);
  int32_t *d_off = nullptr, *d_idx = nullptr;
  double *d_w = nullptr, *d_c = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    if ((rc = dalloc(&d_off, o.size(), nullptr)) || (rc = dalloc(&d_idx, ix.size(), nullptr)) ||
        (rc = dalloc(&d_w, ww.size(), nullptr)) || (rc = dalloc(&d_c, 1, nullptr))) {
      void* ps[] = {d_off, d_idx, d_w, d_c};
      for (void* p : ps)
        if (p) (void)hipFree(p);
      return rc;
    }
  }
  auto cleanup = [&]() {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    void* ps[] = {d_off, d_idx, d_w, d_c};
    for (void* p : ps)
      if (p) (void)hipFree(p);
  };
  const int64_t nt = (int64_t)to->h.node_key.size();
  if ((rc = h2d(d_off, o, s)) || (rc = h2d(d_idx, ix, s)) || (rc = h2d(d_w, ww, s))) {
    cleanup();
    return rc;
  }
  hipLaunchKernelGGL(dev::k_interp6, dim3(grid_stride(nt)), dim3(256), 0, s, U_from, d_off, d_idx, d_w, nt,
                     U_to);
  if (hipGetLastError() != hipSuccess) {
    cleanup();
    return fail(CHNS_EHIP, "launching the transfer failed");
  }
  if (conserve_mass) {
    dev::PhysView pv;
    double m0, m1, e;
    if ((rc = phys_view(params, pv)) || (rc = launch_diagnostics(from, pv, U_from, &m0, &e, s)) ||
        (rc = launch_diagnostics(to, pv, U_to, &m1, &e, s))) {
      cleanup();
      return rc;
    }
    const double vol = (double)to->h.T[0] * to->h.T[1] * to->h.T[2];
    const double c = (m0 - m1) / vol;
    if (hipMemcpyAsync(d_c, &c, sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess) {
      cleanup();
      return fail(CHNS_EHIP, "copying the mass shift failed");
    }
    hipLaunchKernelGGL(dev::k_shift_phi, dim3(grid_stride(nt)), dim3(256), 0, s, U_to, nt, d_c);
  }
  const hipError_t e = hipStreamSynchronize(s);  // the host arrays above must outlive the copies
  cleanup();
  if (e != hipSuccess) return fail(CHNS_EHIP, std::string("transfer: ") + hipGetErrorString(e));
  return CHNS_OK;
}

int chns_mesh_upload(chns_mesh* m, void* stream) {
  if (!m) return fail(CHNS_EINVAL, "mesh is NULL");
  return upload(m, (hipStream_t)stream);
}

int chns_mesh_free(chns_mesh* m) {
  if (!m) return CHNS_OK;
  std::lock_guard<std::mutex> lk(g_struct_mu);
  free_mesh_locked(m);
  return CHNS_OK;
}

}  // extern "C"

// Scratch of chns_jvp_noalloc: the per-target partial rows of one JVP.  Each
// GPU holds its own copy of this array for the life of the process.  In host
// code `scratch` is only a stand-in for the symbol: the device address is
// looked up once per device (hipGetSymbolAddress) and kept in
// g_scratch_ptr, which is what the kernels receive.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, which must be current.
int noalloc_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(CHNS_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(CHNS_EHIP, "hipGetSymbolAddress returned a null address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CHNS_OK;
}

void free_mg_locked(chns_mesh* m) {
  for (size_t l = 0; l < m->mg.size(); ++l) {
    MGLevel& L = m->mg[l];
    void* ptrs[] = {L.p_off, L.p_idx, L.r_off, L.r_eidx, L.inj, L.p_w, L.r_ew, L.U1, L.U0, L.D, L.Di,
                    L.DiC, L.U1f, L.U0f, L.Di32, L.DiC32, L.b64, L.x64, L.r64, L.b32, L.x32, L.r32};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    if (l > 0 && L.mesh) free_mesh_locked(L.mesh);
  }
  m->mg.clear();
  m->mg_key = -1;
  m->mg_bytes = 0;
}

void free_mesh_locked(chns_mesh* m) {
  free_mg_locked(m);
  free_workspace(m->ws);
  void* ptrs[] = {m->d_elem, m->d_hoff, m->d_hids, m->d_anchor, m->d_level,
                  m->d_hw, m->d_hw32, m->d_flag, m->d_part, m->d_sum,
                  m->d_tgt_off, m->d_tgt, m->d_inc_off, m->d_chunk_inc, m->d_node_off, m->d_node_slot,
                  m->d_inc_corner,
                  m->d_bflags, m->d_inc_w, m->d_touch_off, m->d_touch_node, m->d_ntouch_off, m->d_ntouch_slot,
                  m->d_partial, m->d_tbuf, m->d_cmap, m->d_hmap, m->d_lin[0][0], m->d_lin[0][1], m->d_lin[1][0], m->d_lin[1][1],
                  m->d_mid[0], m->d_mid[1]};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (m->h_flag) (void)hipHostFree(m->h_flag);
  if (m->h_sum) (void)hipHostFree(m->h_sum);
  delete m;
}

}  // namespace

extern "C" {

int chns_residual(chns_mesh* m, const chns_params* params, int block, const double* U_new,
                  const double* U_old, double* R, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int rc = check_mesh(m, s);
  if (rc) return rc;
  dev::PhysView pv;
  if ((rc = phys_view(params, pv))) return rc;
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_NS) return fail(CHNS_EINVAL, "unknown block");
  if (!U_new || !U_old || !R) return fail(CHNS_EINVAL, "state and output pointers must not be NULL");
  return launch_residual(m, pv, block, U_new, U_old, R, 6, block == CHNS_BLOCK_CH ? 0 : 2, s, true);
}

int chns_jvp(chns_mesh* m, const chns_params* params, int block, const double* U_new,
             const double* U_old, const void* dU, void* JdU, int prec, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int rc = check_mesh(m, s);
  if (rc) return rc;
  dev::PhysView pv;
  if ((rc = phys_view(params, pv))) return rc;
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_NS) return fail(CHNS_EINVAL, "unknown block");
  if (!U_new || !U_old || !dU || !JdU) return fail(CHNS_EINVAL, "pointers must not be NULL");
  const int off = block == CHNS_BLOCK_CH ? 0 : 2;
  if (prec == CHNS_F64)
    return launch_jvp<double, double, double>(m, pv, block, U_new, U_old, (const double*)dU, 6, off,
                                              (double*)JdU, 6, off, s);
  if (prec == CHNS_F32)
    return launch_jvp<float, double, float>(m, pv, block, U_new, U_old, (const float*)dU, 6, off,
                                            (float*)JdU, 6, off, s);
  return fail(CHNS_EINVAL, "prec must be CHNS_F64 or CHNS_F32");
}

int chns_jvp_noalloc(chns_mesh* m, const chns_params* params, int block, const double* U_new,
                     const double* U_old, const void* dU, void* JdU, int prec, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (!m) return fail(CHNS_EINVAL, "mesh is NULL");
  if (!m->uploaded)
    return fail(CHNS_EINVAL, "chns_jvp_noalloc needs a mesh already on the device (chns_mesh_upload)");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != m->device) return fail(CHNS_EINVAL, "mesh was uploaded to another device");
  dev::PhysView pv;
  int rc;
  if ((rc = phys_view(params, pv))) return rc;
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_NS) return fail(CHNS_EINVAL, "unknown block");
  if (!U_new || !U_old || !dU || !JdU) return fail(CHNS_EINVAL, "pointers must not be NULL");
  if (prec != CHNS_F64 && prec != CHNS_F32) return fail(CHNS_EINVAL, "prec must be CHNS_F64 or CHNS_F32");
  const size_t need = m->plan.tgt.size() * 4 * sizeof(double);
  if (need > kNoAllocScratchBytes)
    return fail(CHNS_EINVAL, "mesh needs " + std::to_string(need) + " bytes of partial rows; chns_jvp_noalloc "
                "holds at most " + std::to_string(kNoAllocScratchBytes) + " (use chns_jvp)");
  void* part = nullptr;
  if ((rc = noalloc_scratch(dev, &part))) return rc;
  const int off = block == CHNS_BLOCK_CH ? 0 : 2;
  if (prec == CHNS_F64)
    return launch_jvp<double, double, double>(m, pv, block, U_new, U_old, (const double*)dU, 6, off,
                                              (double*)JdU, 6, off, s, nullptr, part);
  return launch_jvp<float, double, float>(m, pv, block, U_new, U_old, (const float*)dU, 6, off,
                                          (float*)JdU, 6, off, s, nullptr, part);
}

int chns_jvp_full(chns_mesh* m, const chns_params* params, const double* U_new, const double* U_old,
                  const void* dU, void* JdU, int prec, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int rc = check_mesh(m, s);
  if (rc) return rc;
  dev::PhysView pv;
  if ((rc = phys_view(params, pv))) return rc;
  if (!U_new || !U_old || !dU || !JdU) return fail(CHNS_EINVAL, "pointers must not be NULL");
  if (prec == CHNS_F64)
    return launch_jvp_full<double, double, double>(m, pv, U_new, U_old, (const double*)dU, (double*)JdU, s);
  if (prec == CHNS_F32)
    return launch_jvp_full<float, double, float>(m, pv, U_new, U_old, (const float*)dU, (float*)JdU, s);
  return fail(CHNS_EINVAL, "prec must be CHNS_F64 or CHNS_F32");
}

int chns_linearize(chns_mesh* m, const chns_params* params, int block, const double* U_new,
                   const double* U_old, int prec, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int rc = check_mesh(m, s);
  if (rc) return rc;
  dev::PhysView pv;
  if ((rc = phys_view(params, pv))) return rc;
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_NS) return fail(CHNS_EINVAL, "unknown block");
  if (!U_new || !U_old) return fail(CHNS_EINVAL, "pointers must not be NULL");
  if (prec == CHNS_F64) return launch_lin<double, double>(m, pv, block, U_new, U_old, s);
  if (prec == CHNS_F32) return launch_lin<float, double>(m, pv, block, U_new, U_old, s);
  return fail(CHNS_EINVAL, "prec must be CHNS_F64 or CHNS_F32");
}

int chns_jvp_lin(chns_mesh* m, const chns_params* params, int block, const void* dU, void* JdU, int prec,
                 void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int rc = check_mesh(m, s);
  if (rc) return rc;
  dev::PhysView pv;
  if ((rc = phys_view(params, pv))) return rc;
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_NS) return fail(CHNS_EINVAL, "unknown block");
  if (!dU || !JdU) return fail(CHNS_EINVAL, "pointers must not be NULL");
  const int off = block == CHNS_BLOCK_CH ? 0 : 2;
  if (prec == CHNS_F64)
    return launch_jvp_lin<double, double>(m, pv, block, (const double*)dU, 6, off, (double*)JdU, 6, off, s);
  if (prec == CHNS_F32)
    return launch_jvp_lin<float, float>(m, pv, block, (const float*)dU, 6, off, (float*)JdU, 6, off, s);
  return fail(CHNS_EINVAL, "prec must be CHNS_F64 or CHNS_F32");
}

int chns_diag_blocks(chns_mesh* m, const chns_params* params, int block, const double* U_new,
                     const double* U_old, double* D, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int rc = check_mesh(m, s);
  if (rc) return rc;
  dev::PhysView pv;
  if ((rc = phys_view(params, pv))) return rc;
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_NS) return fail(CHNS_EINVAL, "unknown block");
  if (!U_new || !U_old || !D) return fail(CHNS_EINVAL, "pointers must not be NULL");
  return launch_diag(m, pv, block, U_new, U_old, D, s);
}

int chns_diagnostics(chns_mesh* m, const chns_params* params, const double* U, double* mass,
                     double* energy, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int rc = check_mesh(m, s);
  if (rc) return rc;
  dev::PhysView pv;
  if ((rc = phys_view(params, pv))) return rc;
  if (!U || !mass || !energy) return fail(CHNS_EINVAL, "pointers must not be NULL");
  return launch_diagnostics(m, pv, U, mass, energy, s);
}

int chns_step(chns_mesh* m, const chns_params* params, const chns_solver_opts* opts, double* U,
              chns_step_stats* out, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int rc = check_mesh(m, s);
  if (rc) return rc;
  dev::PhysView pv;
  if ((rc = phys_view(params, pv))) return rc;
  if (!opts || !U || !out) return fail(CHNS_EINVAL, "opts, U and out must not be NULL");
  if ((rc = check_opts(opts))) return rc;
  std::memset(out, 0, sizeof(*out));
  const auto t0 = std::chrono::steady_clock::now();
  Solver S(m, pv, *opts, s);
  rc = S.step(U, out);
  out->t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

int chns_launch_element_loop(chns_mesh* m, const chns_params* params, int block, int op,
                             const double* U_new, const double* U_old, const void* dU, void* out,
                             int reps, void* stream, int64_t* grid) {
  hipStream_t s = (hipStream_t)stream;
  int rc = check_mesh(m, s);
  if (rc) return rc;
  dev::PhysView pv;
  if ((rc = phys_view(params, pv))) return rc;
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_NS) return fail(CHNS_EINVAL, "unknown block");
  if (!U_new || !U_old || (op != 0 && op != 3 && op != 5 && op != 7 && !dU)) return fail(CHNS_EINVAL, "NULL pointer");
  if (reps < 1) return fail(CHNS_EINVAL, "reps must be positive");
  if (op == 3 && (rc = ensure_tbuf(m))) return rc;
  (void)out;
  const auto mv = view(m);
  const auto pl = plan_view(m);
  const dim3 g((unsigned)m->n_chunks), b(dev::kChunkThreads);
  const int off = block == CHNS_BLOCK_CH ? 0 : 2;
  double* p64 = m->d_partial;
  float* p32 = (float*)m->d_partial;
  const dev::ChunkCaps cc = caps(m);
  for (int r = 0; r < reps; ++r) {
    if (op == 0) {
      if (block == CHNS_BLOCK_CH)
        hipLaunchKernelGGL(dev::k_ch_residual<double>, g, b, (dev::ChunkLDS<double, 5, 0, 2>::bytes(cc)), s,
                           mv, pl, pv, cc, U_new, U_old, p64);
      else
        hipLaunchKernelGGL(dev::k_ns_residual<double>, g, b, (dev::ChunkLDS<double, 6, 0, 4>::bytes(cc)), s,
                           mv, pl, pv, cc, U_new, U_old, p64, m->d_flag);
    } else if (op == 1) {
      if (block == CHNS_BLOCK_CH)
        hipLaunchKernelGGL((dev::k_ch_jvp<double, double, double>), g, b,
                           (dev::ChunkLDS<double, 5, 2, 2>::bytes(cc)), s, mv, pl, pv, cc, U_new, U_old,
                           (const double*)dU, 6, off, p64, (const int*)nullptr);
      else
        hipLaunchKernelGGL((dev::k_ns_jvp<double, double, double>), g, b,
                           (dev::ChunkLDS<double, 6, 4, 4>::bytes(cc)), s, mv, pl, pv, cc, U_new, U_old,
                           (const double*)dU, 6, off, p64, (const int*)nullptr);
    } else if (op == 2) {
      if (block == CHNS_BLOCK_CH)
        hipLaunchKernelGGL((dev::k_ch_jvp<float, double, float>), g, b,
                           (dev::ChunkLDS<float, 5, 2, 2>::bytes(cc)), s, mv, pl, pv, cc, U_new, U_old,
                           (const float*)dU, 6, off, p32, (const int*)nullptr);
      else
        hipLaunchKernelGGL((dev::k_ns_jvp<float, double, float>), g, b,
                           (dev::ChunkLDS<float, 6, 4, 4>::bytes(cc)), s, mv, pl, pv, cc, U_new, U_old,
                           (const float*)dU, 6, off, p32, (const int*)nullptr);
    } else if (op == 4 || op == 6) {  // JVP from the cached linearisation points (FP64 / FP32)
      const int k = op == 4 ? 0 : 1;
      if (!m->d_lin[block][k]) return fail(CHNS_EINVAL, "ops 4 and 6 need ops 5 and 7 first");
      if (block == CHNS_BLOCK_CH && k == 0)
        hipLaunchKernelGGL((dev::k_ch_jvp_lin<double, double>), g, b, (dev::ChunkLDS<double, 0, 2, 2>::bytes(cc)),
                           s, mv, pl, pv, cc, (const double*)m->d_lin[block][0], (const double*)dU, 6, off, p64,
                           (const int*)nullptr);
      else if (block == CHNS_BLOCK_CH)
        hipLaunchKernelGGL((dev::k_ch_jvp_lin<float, float>), g, b, (dev::ChunkLDS<float, 0, 2, 2>::bytes(cc)),
                           s, mv, pl, pv, cc, (const float*)m->d_lin[block][1], (const float*)dU, 6, off, p32,
                           (const int*)nullptr);
      else if (k == 0)
        hipLaunchKernelGGL((dev::k_ns_jvp_lin<double, double>), g, b,
                           (dev::ChunkLDS<double, 0, 4 + dev::kNSMid, 4>::bytes(cc)), s, mv, pl, pv, cc,
                           (const double*)m->d_lin[block][0], ns_mid<double>(m), (const double*)dU, 6, off, p64,
                           (const int*)nullptr);
      else
        hipLaunchKernelGGL((dev::k_ns_jvp_lin<float, float>), g, b,
                           (dev::ChunkLDS<float, 0, 4 + dev::kNSMid, 4>::bytes(cc)), s, mv, pl, pv, cc,
                           (const float*)m->d_lin[block][1], ns_mid<float>(m), (const float*)dU, 6, off, p32,
                           (const int*)nullptr);
    } else if (op == 5) {
      if ((rc = launch_lin<double, double>(m, pv, block, U_new, U_old, s))) return rc;
    } else if (op == 7) {
      if ((rc = launch_lin<float, double>(m, pv, block, U_new, U_old, s))) return rc;
    } else if (op == 3) {
      if (block == CHNS_BLOCK_CH)
        hipLaunchKernelGGL((dev::k_diag<double, 0>), g, b, 0, s, mv, pl, pv, U_new, U_old, m->d_tbuf);
      else
        hipLaunchKernelGGL((dev::k_diag<double, 1>), g, b, 0, s, mv, pl, pv, U_new, U_old, m->d_tbuf);
    } else {
      return fail(CHNS_EINVAL, "op must be 0..7");
    }
  }
  HIPCHK(hipGetLastError());
  if (grid) *grid = (int64_t)g.x;
  return CHNS_OK;
}

}  // extern "C"

#include "serve.inl"
#include "q2.inl"
