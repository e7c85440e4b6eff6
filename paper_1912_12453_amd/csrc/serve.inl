// Serving loop of libchns (chns_server_*): independent two-phase problems
// of different octree sizes share one device.  Included at the end of
// capi.hip (it drives the same Solver and upload code).
//
// Request life: QUEUED (spec copied) -> builder thread: host octree, scatter
// plan, U^0 and exact device footprint -> READY -> admitted by
// chns_server_run_round while the footprint fits the budget: upload on the
// request's own stream -> RESIDENT: a driver thread of its own runs its
// Crank-Nicolson steps back to back on that stream -> DONE after its last
// step (state copied to the host, device memory freed) or FAILED.  Steps of
// different residents overlap on the device; none waits for another.

#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

namespace {

using Clock = std::chrono::steady_clock;

// Device bytes that upload() and ensure_tbuf() allocate for a mesh whose
// scatter plan is built (counts of zero take one element, as dalloc does).
int64_t mesh_footprint(const chns_mesh* m) {
  const HostMesh& h = m->h;
  const ScatterPlan& P = m->plan;
  auto sz = [](size_t count, size_t elem) { return (int64_t)(std::max<size_t>(count, 1) * elem); };
  const size_t E = h.leaf_key.size(), NH = h.hang_key.size(), NC = h.hang_ids.size();
  return sz(E * 8, 4) + sz(E, 1) + sz(E * 3, 4) + sz(NH + 1, 4) + sz(NC, 4) + sz(NC, 8) + sz(NC, 4) +
         sz(1, 4) + sz((size_t)dev::diag_blocks((int64_t)E) * 2, 8) + sz(2, 8) + sz(P.tgt_off.size(), 4) + sz(P.tgt.size(), 4) +
         sz(P.inc_off.size(), 4) + sz(P.chunk_inc.size(), 4) + sz(P.inc_corner.size(), 1) +
         sz(P.inc_w.size(), 4) +
         sz(P.node_off.size(), 4) + sz(P.node_slot.size(), 4) + sz(P.touch_off.size(), 8) + sz(P.touch_node.size(), 4) +
         sz(P.ntouch_off.size(), 8) + sz(P.ntouch_slot.size(), 8) + sz(h.bflags.size(), 1) +
         sz(P.tgt.size() * 4, 8) + sz(P.ntouch_slot.size() * 16, 8) + sz(P.cmap.size(), 4) +
         sz(P.hmap.size(), 4);
}

// Device bytes of the cached linearisation points of a mesh, both blocks, and
// the NS nodal midpoints (ensure_lin), at the precision of the inner solve.  The coupled solve
// builds them only for its multigrid preconditioner.
int64_t lin_footprint(const chns_mesh* m, const chns_solver_opts& o) {
  if (o.coupled && o.precond != 2) return 0;
  const int64_t chunks = std::max<int64_t>((int64_t)m->plan.tgt_off.size() - 1, 1);
  const int64_t n = std::max<int64_t>((int64_t)m->h.node_key.size(), 1);
  return (chunks * (dev::kNSLin + dev::kCHLin) * dev::kChunkThreads + n * dev::kNSMid) *
         (o.precision == 0 ? 8 : 4);
}

// Device bytes of Solver::ensure_workspace() for n nodes under opts.
int64_t workspace_footprint(int64_t n, const chns_solver_opts& o) {
  const int64_t N = n * (o.coupled ? 6 : 4), m = o.gmres_restart;
  const int64_t nb = grid_stride(N, 256, 1024);
  int64_t b = (3 * 6 * n + 2 * N + 2 * 16 * n) * 8 + 16 * n * 4 + nb * (2 * dev::kMaxBasis + 2) * 8 +
              (dev::kMaxBasis + 1) * 8 + 4 + (int64_t)sizeof(dev::GmresCtl) +
              (4 + 8) * n * 8 + (4 + 8) * n * 4;  // CH block inverses and the coupled pack buffers
  if (o.precision == 0)
    b += (N * (2 * m + 3)) * 8;
  else
    b += (N * (2 * m + 3) + 12 * n) * 4;
  return b;
}

struct Request {
  int64_t ticket = 0;
  chns_mesh_spec spec{};
  std::vector<int32_t> leaves;  // owned copy of spec.leaves
  chns_params params{};
  dev::PhysView pv{};
  int n_steps = 0, steps_done = 0;
  int state = CHNS_REQ_QUEUED, status = CHNS_OK;
  std::string err;
  chns_mesh* mesh = nullptr;
  std::vector<double> U0;        // host U^0, then the final state
  int64_t footprint = 0;
  int64_t n_leaves = 0, n_nodes = 0;
  double* dU = nullptr;          // device state
  hipStream_t stream = nullptr;
  std::vector<chns_step_stats> stats;
  std::vector<double> latency_ms;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::thread driver;
  bool finished = false;  // the driver has left (joined by the next round)
};

}  // namespace

struct chns_server {
  int device = 0;
  int64_t budget = 0;
  int max_resident = 1;
  chns_solver_opts opts{};
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;        // builder work
  std::condition_variable progress;  // a step ended, a request left or became READY
  bool stop = false;
  std::atomic<bool> cancel{false};  // running steps stop at their next check
  std::deque<Request*> build_queue;
  std::vector<Request*> ready;     // arrival order
  std::vector<Request*> resident;
  std::map<int64_t, std::unique_ptr<Request>> all;
  int64_t next_ticket = 0, in_use = 0, rounds = 0, steps = 0;
  int wait_ms = 20;     // longest wait of a round for progress
  int64_t events = 0;   // steps ended, requests left or became READY
  std::thread builder;

  double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
};

namespace {

// Host part of a request: octree, scatter plan, U^0 (phi0 at the nodes,
// mu = phi^3 - phi, v = p = 0) and the footprint.
void build_request(chns_server* S, Request* r) {
  std::string err;
  chns_mesh* m = new (std::nothrow) chns_mesh();
  if (!m) err = "out of host memory";
  try {
    if (err.empty()) err = build_host_mesh(r->spec, m->h);
    if (err.empty()) err = build_scatter_plan(m->h, m->plan);
  } catch (const std::bad_alloc&) {
    err = "out of host memory while building the mesh";
  }
  if (err.empty()) {
    m->plan_ready = true;
    const size_t n = m->h.node_key.size();
    const double unit = std::ldexp(1.0, -m->h.D);
    std::vector<double> xyz(n * 3), phi(n, 1.0);
    for (size_t i = 0; i < n; ++i) {
      uint32_t x, y, z;
      unkey(m->h.node_key[i], x, y, z);
      xyz[3 * i] = x * unit;
      xyz[3 * i + 1] = y * unit;
      xyz[3 * i + 2] = z * unit;
    }
    if (r->spec.phi0) r->spec.phi0(xyz.data(), (int64_t)n, phi.data(), r->spec.user);
    r->U0.assign(n * 6, 0.0);
    for (size_t i = 0; i < n; ++i) {
      if (!std::isfinite(phi[i])) {
        err = "phi0 returned a non-finite value";
        break;
      }
      r->U0[6 * i] = phi[i];
      r->U0[6 * i + 1] = phi[i] * phi[i] * phi[i] - phi[i];
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  r->mesh = m;
  if (err.empty()) {
    r->n_leaves = (int64_t)m->h.leaf_key.size();
    r->n_nodes = (int64_t)m->h.node_key.size();
    r->footprint = mesh_footprint(m) + workspace_footprint((int64_t)m->h.node_key.size(), S->opts) +
                   lin_footprint(m, S->opts);
    if (S->opts.precond == 2)  // coarse levels: at most the fine level's size again, plus V-cycle buffers
      r->footprint += mesh_footprint(m) + lin_footprint(m, S->opts) + 656 * (int64_t)m->h.node_key.size();
    if (r->footprint > S->budget) err = "request needs " + std::to_string(r->footprint) +
                                        " device bytes, above the server budget";
  }
  if (!err.empty()) {
    r->state = CHNS_REQ_FAILED;
    r->status = CHNS_EINVAL;
    r->err = err;
    r->t_done = S->now_ms();
    if (m) chns_mesh_free(m);
    r->mesh = nullptr;
    S->events += 1;
    S->progress.notify_all();
    return;
  }
  r->state = CHNS_REQ_READY;
  S->ready.push_back(r);
  S->events += 1;
  S->progress.notify_all();
}

void builder_main(chns_server* S) {
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] { return S->stop || !S->build_queue.empty(); });
      if (S->stop) return;
      r = S->build_queue.front();
      S->build_queue.pop_front();
    }
    build_request(S, r);
  }
}

void free_request(Request* r) {
  if (r->mesh) chns_mesh_free(r->mesh);  // takes the structural lock itself
  r->mesh = nullptr;
  std::lock_guard<std::mutex> lk(g_struct_mu);
  if (r->dU) (void)hipFree(r->dU);
  r->dU = nullptr;
  if (r->stream) (void)hipStreamDestroy(r->stream);
  r->stream = nullptr;
}

int admit_upload(chns_server* S, Request* r, hipEvent_t after) {
  const size_t n = r->mesh->h.node_key.size();
  {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    HIPCHK(hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking));
    const int rc = dalloc(&r->dU, n * 6, nullptr);
    if (rc) return rc;
  }
  HIPCHK(hipStreamWaitEvent(r->stream, after, 0));
  int rc = upload(r->mesh, r->stream);
  if (rc) return rc;
  if ((rc = ensure_tbuf(r->mesh))) return rc;
  HIPCHK(hipMemcpyAsync(r->dU, r->U0.data(), n * 6 * sizeof(double), hipMemcpyHostToDevice, r->stream));
  HIPCHK(hipStreamSynchronize(r->stream));
  return CHNS_OK;
}

// Driver of one resident request: its steps back to back on its stream.
// Per-step latency runs from the moment the step became runnable (admission
// or the end of the previous step) to its end.
void drive(chns_server* S, Request* r) {
  int rc = CHNS_OK;
  std::string err;
  if (hipSetDevice(S->device) != hipSuccess) {
    rc = CHNS_EHIP;
    err = "hipSetDevice failed in a request driver";
  }
  auto t_ready = Clock::now();
  for (int k = 0; rc >= 0 && k < r->n_steps; ++k) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->stop) {
        rc = CHNS_EINVAL;
        err = "server destroyed while the request ran";
        break;
      }
    }
    chns_step_stats st;
    std::memset(&st, 0, sizeof(st));
    const auto ts = Clock::now();
    Solver sol(r->mesh, r->pv, S->opts, r->stream);
    sol.cancel = &S->cancel;
    const int src = sol.step(r->dU, &st);
    const auto te = Clock::now();
    if (src < 0) {
      rc = src;
      err = g_err;
      break;
    }
    st.t_ms = std::chrono::duration<double, std::milli>(te - ts).count();
    std::lock_guard<std::mutex> lk(S->mu);
    r->stats.push_back(st);
    r->latency_ms.push_back(std::chrono::duration<double, std::milli>(te - t_ready).count());
    r->steps_done += 1;
    r->status = src;
    S->steps += 1;
    t_ready = te;
    S->events += 1;
    S->progress.notify_all();
  }
  if (rc >= 0) {
    if (hipMemcpyAsync(r->U0.data(), r->dU, r->U0.size() * sizeof(double), hipMemcpyDeviceToHost,
                       r->stream) != hipSuccess ||
        hipStreamSynchronize(r->stream) != hipSuccess) {
      rc = CHNS_EHIP;
      err = "copying the final state to the host failed";
    }
  }
  free_request(r);
  std::lock_guard<std::mutex> lk(S->mu);
  S->in_use -= r->footprint;
  S->resident.erase(std::find(S->resident.begin(), S->resident.end(), r));
  r->t_done = S->now_ms();
  if (rc < 0) {
    r->state = CHNS_REQ_FAILED;
    r->status = rc;
    r->err = err;
  } else {
    r->state = CHNS_REQ_DONE;
  }
  r->finished = true;
  S->events += 1;
  S->progress.notify_all();
}

}  // namespace

extern "C" {

int chns_server_create(size_t hbm_budget_bytes, int max_resident, const chns_solver_opts* opts,
                       chns_server** out) {
  if (!opts || !out) return fail(CHNS_EINVAL, "opts and out must not be NULL");
  *out = nullptr;
  if (max_resident < 1 || max_resident > 64) return fail(CHNS_EINVAL, "max_resident must be in [1, 64]");
  if (hbm_budget_bytes == 0) return fail(CHNS_EINVAL, "the HBM budget must be positive");
  int rc = check_opts(opts);
  if (rc) return rc;
  std::unique_ptr<chns_server> S(new (std::nothrow) chns_server());
  if (!S) return fail(CHNS_ENOMEM, "out of host memory");
  HIPCHK(hipGetDevice(&S->device));
  S->budget = (int64_t)hbm_budget_bytes;
  S->max_resident = max_resident;
  S->opts = *opts;
  S->opts.graphs = 1;
  S->t0 = Clock::now();
  try {
    S->builder = std::thread(builder_main, S.get());
  } catch (...) {
    return fail(CHNS_ENOMEM, "cannot start the builder thread");
  }
  *out = S.release();
  return CHNS_OK;
}

int chns_server_submit(chns_server* S, const chns_mesh_spec* spec, const chns_params* params,
                       int n_steps, int64_t* ticket) {
  if (!S || !spec || !params || !ticket) return fail(CHNS_EINVAL, "NULL argument");
  if (n_steps < 1) return fail(CHNS_EINVAL, "n_steps must be positive");
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return fail(CHNS_ENOMEM, "out of host memory");
  int rc = phys_view(params, r->pv);
  if (rc) return rc;
  r->spec = *spec;
  if (spec->leaves && spec->n_leaves > 0) {
    r->leaves.assign(spec->leaves, spec->leaves + spec->n_leaves * 4);
    r->spec.leaves = r->leaves.data();
  }
  r->params = *params;
  r->n_steps = n_steps;
  std::lock_guard<std::mutex> lk(S->mu);
  r->ticket = S->next_ticket++;
  r->t_submit = S->now_ms();
  *ticket = r->ticket;
  S->build_queue.push_back(r.get());
  S->all[r->ticket] = std::move(r);
  S->cv.notify_one();
  return CHNS_OK;
}

int chns_server_poll(chns_server* S, int64_t ticket, chns_request_info* info, double* U_host_out,
                     chns_step_stats* per_step, double* step_latency_ms) {
  if (!S) return fail(CHNS_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(CHNS_EINVAL, "unknown ticket");
  const Request* r = it->second.get();
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->state = r->state;
    info->status = r->status;
    info->n_steps = r->n_steps;
    info->steps_done = r->steps_done;
    info->n_nodes = r->n_nodes;
    info->n_leaves = r->n_leaves;
    info->footprint_bytes = r->footprint;
    info->t_submit_ms = r->t_submit;
    info->t_admit_ms = r->t_admit;
    info->t_done_ms = r->t_done;
  }
  if (U_host_out && r->state == CHNS_REQ_DONE)
    std::memcpy(U_host_out, r->U0.data(), r->U0.size() * sizeof(double));
  for (size_t k = 0; k < r->stats.size(); ++k) {
    if (per_step) per_step[k] = r->stats[k];
    if (step_latency_ms) step_latency_ms[k] = r->latency_ms[k];
  }
  if (r->state == CHNS_REQ_FAILED && !r->err.empty()) g_err = r->err;
  return CHNS_OK;
}

int chns_server_run_round(chns_server* S, void* stream) {
  if (!S) return fail(CHNS_EINVAL, "server is NULL");
  HIPCHK(hipSetDevice(S->device));
  // join drivers that have left
  std::vector<Request*> gone;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (auto& kv : S->all)
      if (kv.second->finished && kv.second->driver.joinable()) gone.push_back(kv.second.get());
  }
  for (Request* r : gone) r->driver.join();
  // admission: arrival order, skipping requests that do not fit yet
  std::vector<Request*> admitted;
  int64_t s0, e0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    s0 = S->steps;
    e0 = S->events;
    for (auto it = S->ready.begin(); it != S->ready.end();) {
      Request* r = *it;
      if ((int)(S->resident.size() + admitted.size()) >= S->max_resident) break;
      if (S->in_use + r->footprint > S->budget) {
        ++it;
        continue;
      }
      S->in_use += r->footprint;
      r->state = CHNS_REQ_RESIDENT;
      r->t_admit = S->now_ms();
      admitted.push_back(r);
      it = S->ready.erase(it);
    }
  }
  if (!admitted.empty()) {
    // uploads start after the work already queued on the caller's stream
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, (hipStream_t)stream));
    for (Request* r : admitted) {
      const int rc = admit_upload(S, r, ev);
      if (rc) {
        const std::string msg = g_err;
        free_request(r);
        std::lock_guard<std::mutex> lk(S->mu);
        S->in_use -= r->footprint;
        r->state = CHNS_REQ_FAILED;
        r->status = rc;
        r->err = msg;
        r->t_done = S->now_ms();
        r->finished = true;
        continue;
      }
      std::lock_guard<std::mutex> lk(S->mu);
      S->resident.push_back(r);
      try {
        r->driver = std::thread(drive, S, r);
      } catch (...) {
        S->resident.pop_back();
        S->in_use -= r->footprint;
        r->state = CHNS_REQ_FAILED;
        r->status = CHNS_ENOMEM;
        r->err = "cannot start a request driver thread";
        r->t_done = S->now_ms();
        r->finished = true;
      }
    }
    (void)hipEventDestroy(ev);
  }
  // wait for progress: a step ends, a request leaves or becomes READY
  std::unique_lock<std::mutex> lk(S->mu);
  S->rounds += 1;
  if (S->resident.empty()) return 0;
  S->progress.wait_for(lk, std::chrono::milliseconds(S->wait_ms), [&] { return S->events > e0; });
  return (int)(S->steps - s0);
}

int chns_server_stats_get(chns_server* S, chns_server_stats* out) {
  if (!S || !out) return fail(CHNS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(out, 0, sizeof(*out));
  for (auto& kv : S->all) {
    switch (kv.second->state) {
      case CHNS_REQ_QUEUED: ++out->queued; break;
      case CHNS_REQ_READY: ++out->ready; break;
      case CHNS_REQ_RESIDENT: ++out->resident; break;
      case CHNS_REQ_DONE: ++out->done; break;
      default: ++out->failed; break;
    }
  }
  out->bytes_in_use = S->in_use;
  out->budget_bytes = S->budget;
  out->rounds = S->rounds;
  out->steps = S->steps;
  return CHNS_OK;
}

int chns_server_destroy(chns_server* S) {
  if (!S) return CHNS_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cancel.store(true);
  S->cv.notify_all();
  S->progress.notify_all();
  if (S->builder.joinable()) S->builder.join();
  // drivers stop at their next Newton iteration or GMRES cycle
  for (auto& kv : S->all)
    if (kv.second->driver.joinable()) kv.second->driver.join();
  for (auto& kv : S->all) free_request(kv.second.get());
  delete S;
  return CHNS_OK;
}

}  // extern "C"
