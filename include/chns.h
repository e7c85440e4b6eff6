/* chns.h -- C ABI of the MI355X (gfx950) matrix-free CHNS element loop.
 *
 * Implements the hot path of the Cahn-Hilliard Navier-Stokes method of
 * Khanwale et al., "Simulating two-phase flows with thermodynamically
 * consistent energy stable Cahn-Hilliard Navier-Stokes equations on parallel
 * adaptive octree based meshes" (arXiv 1912.12453):
 *   - the octree mesh of Sec. 4 (top-down refinement, 2:1 balance, hanging
 *     nodes as element temporaries), built on the host and uploaded once;
 *   - the residual and Jacobian-vector product of the two sub-problems of the
 *     block iteration of Sec. 3 (Fig. 1): the Cahn-Hilliard block (phi, mu;
 *     Def. 1 with the Crank-Nicolson averages) and the VMS-stabilised
 *     Navier-Stokes block (v, p; Def. 2 of Sec. 3.4), on trilinear hexahedra;
 *   - one Crank-Nicolson time step: the block iteration of Fig. 1 with a
 *     Newton solve per block (Sec. 3.5) and right-preconditioned GMRES.
 *
 * Conventions
 *   - All entry points return an int status (CHNS_OK = 0).  On a negative
 *     status nothing useful was written; chns_last_error() returns a message
 *     (thread-local, valid until the next call on the same thread).
 *   - "device" pointers are addresses in HBM of the current HIP device
 *     (hipMalloc'd or torch-allocated); the library never frees or keeps
 *     them.  "stream" is a hipStream_t (NULL = the null stream); every device
 *     operation of a call is enqueued on it and the call returns without
 *     synchronising unless stated otherwise.
 *   - State vectors are node-major with 6 doubles per independent node, in
 *     the mesh's Morton node order: [phi, mu, u, v, w, p].
 *   - Errors are never thrown across the ABI.
 */
#ifndef CHNS_H
#define CHNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CHNS_OK = 0,
  CHNS_NOT_CONVERGED = 1, /* chns_step: outputs and stats written (best iterate) */
  CHNS_EINVAL = -1,       /* bad argument (null pointer, size, unknown enum)      */
  CHNS_ENOMEM = -2,       /* device or host allocation failed                     */
  CHNS_EHIP = -3,         /* a HIP runtime call failed                            */
  CHNS_ENONFINITE = -4,   /* a NaN or Inf appeared in a residual norm             */
  CHNS_ETAU = -5,         /* the tau_m bracket of Sec. 3.4 was not positive       */
  CHNS_ENODEV = -6,       /* no usable gfx950 device                              */
  CHNS_ECANCELED = -7     /* a server step stopped because the server is destroyed */
};

/* The two sub-problems of the block iteration (Sec. 3, Fig. 1). */
enum { CHNS_BLOCK_CH = 0, CHNS_BLOCK_NS = 1 };
/* Arithmetic of a Jacobian-vector product. */
enum { CHNS_F64 = 0, CHNS_F32 = 1 };

/* Non-dimensional parameters (Sec. 2).  rho(+1) = 1 and rho(-1) = rho_minus,
 * i.e. rho = alpha phi + beta with alpha = (1 - rho_minus)/2,
 * beta = (1 + rho_minus)/2; eta likewise with eta_minus.  gravity is the
 * unit direction g^ of the momentum equation ((0,-1,0) in the paper).  C_I is
 * the constant of tau_m (6 in the paper).  flux_mode selects the mass flux of
 * the thermo-consistency relation: 0 -> J = -(alpha/Cn) grad mu (the value
 * that makes the continuity equation agree with the CH equation), 1 ->
 * J = -alpha grad mu (the relation as printed). */
typedef struct {
  double Cn, Pe, Re, We, Fr;
  double rho_minus, eta_minus;
  double dt;
  double gravity[3];
  double C_I;
  int32_t flux_mode;
} chns_params;

/* Refinement indicator phi0, evaluated on the host in batches: out[i] =
 * phi0(xyz[3i], xyz[3i+1], xyz[3i+2]) for i < n. */
typedef void (*chns_phi0_fn)(const double* xyz, int64_t n, double* out, void* user);

/* Mesh description (Sec. 4 "Refinement").  The domain is a brick of
 * trees[0] x trees[1] x trees[2] unit cubes; level l means leaf side 2^-l.
 * Either explicit leaves are given (n_leaves rows of (x, y, z, level) in
 * integer units of 2^-level_max, tiling the domain; level_min and phi0 are
 * then ignored), or the mesh is refined top-down from the tree roots: an
 * octant below level_max is split when it is below level_min, or when phi0
 * sampled at its 8 corners and centre has |phi0| < band somewhere or changes
 * sign.  The result is then 2:1 balanced over face, edge and corner
 * neighbours (Sec. 4 "2:1 Balancing").  level_max <= 16. */
typedef struct {
  int32_t trees[3];
  int32_t level_min, level_max;
  chns_phi0_fn phi0; /* may be NULL: uniform refinement to level_min */
  void* user;
  double band;
  const int32_t* leaves; /* host, optional */
  int64_t n_leaves;
} chns_mesh_spec;

typedef struct chns_mesh chns_mesh;

typedef struct {
  int64_t n_leaves;       /* elements                                      */
  int64_t n_nodes;        /* independent nodes (unknowns per field)        */
  int64_t n_hanging;      /* hanging nodes (not stored as unknowns)        */
  int64_t n_constraint;   /* entries of the flattened hanging constraints  */
  int32_t level_max;      /* integer unit = 2^-level_max                   */
  int32_t max_fanin;      /* largest number of parents of a hanging node   */
  int64_t device_bytes;   /* HBM held by the mesh now: its arrays, solver
                           * workspace, cached linearisations and any
                           * multigrid hierarchy built for it            */
} chns_mesh_stats;

/* Builds the balanced octree, numbers its nodes and flattens the hanging
 * constraints on the host (no GPU needed).  The device copy is made on first
 * use by a device entry point (or by chns_mesh_upload).  *out is owned by the
 * library; release it with chns_mesh_free. */
int chns_mesh_build(const chns_mesh_spec* spec, chns_mesh** out);
int chns_mesh_info(const chns_mesh* mesh, chns_mesh_stats* out);
/* Host copies of the mesh arrays, caller-allocated from chns_mesh_info:
 *   leaves [n_leaves*4]  (x, y, z, level), Morton order;
 *   elem   [n_leaves*8]  corner c = i + 2j + 4k: node id >= 0, or -1-h for
 *                        hanging node h;
 *   nodes  [n_nodes*3]   integer coordinates of the independent nodes;
 *   bflags [n_nodes]     bit0: on the domain boundary; bit1: pressure pin;
 *   hang_xyz [n_hanging*3], hang_off [n_hanging+1], hang_ids [n_constraint],
 *   hang_w [n_constraint]: hanging node h = sum_t hang_w[t] * node hang_ids[t]
 *                        for hang_off[h] <= t < hang_off[h+1].
 * Any pointer may be NULL to skip that array. */
int chns_mesh_arrays(const chns_mesh* mesh, int32_t* leaves, int32_t* elem, int32_t* nodes,
                     uint8_t* bflags, int32_t* hang_xyz, int64_t* hang_off, int32_t* hang_ids,
                     double* hang_w);
/* Node coordinates (physical, [n_nodes*3]) and boundary flags, host arrays. */
int chns_mesh_nodes(const chns_mesh* mesh, double* xyz, uint8_t* bflags);
/* Copies the mesh to the current device on `stream` (optional; the device
 * entry points upload on first use). */
int chns_mesh_upload(chns_mesh* mesh, void* stream);
int chns_mesh_free(chns_mesh* mesh);

/* Residual of one block (Sec. 3.4, Def. 2; CH rows from Def. 1) at the
 * iterate U_new given the previous step U_old (device, n_nodes*6 doubles
 * each).  R (device, n_nodes*6 doubles) receives the block's rows; the other
 * block's entries are set to 0.  NS boundary rows: velocity rows of boundary
 * nodes read v_new - v_old (the wall data travels with the state: no-slip
 * walls keep v = 0), the pressure row of the pinned node reads
 * p_new - p_old.  Returns CHNS_ETAU (after the launch completes) when a
 * tau_m bracket was not positive. */
int chns_residual(chns_mesh* mesh, const chns_params* params, int block, const double* U_new,
                  const double* U_old, double* R, void* stream);

/* Jacobian-vector product of the block residual with respect to the block's
 * unknowns at U_new (Sec. 3.5: the analytic Jacobian, here applied without
 * being assembled).  dU and JdU are device arrays of n_nodes*6 elements of
 * type double (prec = CHNS_F64) or float (prec = CHNS_F32, computed in FP32
 * with FP32 accumulation); only the block's entries of dU are read and the
 * other block's entries of JdU are set to 0.  Boundary rows are identity
 * rows. */
int chns_jvp(chns_mesh* mesh, const chns_params* params, int block, const double* U_new,
             const double* U_old, const void* dU, void* JdU, int prec, void* stream);

/* chns_jvp for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, kernels and results (bit for bit) as chns_jvp, but the
 * per-target partial rows live in a static 64 MiB device array of the
 * library (one per GPU, held until the process ends) instead of the mesh's
 * own buffer, and nothing is allocated: the mesh must already be on the
 * current device (chns_mesh_upload or any earlier device call), else
 * CHNS_EINVAL.  Meshes whose partial rows (4 doubles per chunk target, about
 * 2.5 targets per leaf) exceed 64 MiB are rejected with CHNS_EINVAL; use
 * chns_jvp for them.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (different streams or threads) race; serialise them. */
int chns_jvp_noalloc(chns_mesh* mesh, const chns_params* params, int block, const double* U_new,
                     const double* U_old, const void* dU, void* JdU, int prec, void* stream);

/* Rows of the coupled Jacobian (both blocks, derivatives with respect to all
 * six fields of U^{k+1}, the cross terms d R_NS / d(phi, mu) and
 * d R_CH / d v included) applied to dU (n_nodes*6 in the arithmetic of
 * prec); JdU gets all six rows per node, the NS boundary rows being identity
 * rows as in chns_jvp.  The block iteration of Fig. 1 uses the diagonal
 * blocks only; a fully coupled Newton solve (chns_solver_opts.coupled) uses
 * this operator.  Computed by forward-mode differentiation (dual numbers) of
 * the residual kernels. */
int chns_jvp_full(chns_mesh* mesh, const chns_params* params, const double* U_new, const double* U_old,
                  const void* dU, void* JdU, int prec, void* stream);

/* Cached linearisation points.  Within one Newton iteration the state is
 * fixed, so the quantities of the block's weak form (Def. 1 and 2) that the
 * JVP differentiates around can be evaluated once:
 *   NS: per Gauss point phi^{k+1} pulled back to [-1,1], the transport
 *       velocity of R_m and R_m (7 values), and per node the midpoints
 *       u~, v~, w~, mu~ (4 values), from which v~, its gradient, the mass
 *       flux J, rho, eta, R_c, tau_m and tau_c are rebuilt at the point;
 *   CH: per Gauss point psi''(phi~) = 3 phi~^2 - 1 and v~ (4 values).
 * chns_linearize does that for (U_new, U_old) and keeps the values with the
 * mesh (device memory, 7 or 4 times 8 values per element plus 4 per node
 * for NS, in the arithmetic of prec, allocated on first use, one cache per
 * block and precision);
 * chns_jvp_lin then applies the chns_jvp of that state, block and prec to dU
 * (same layout; same results up to rounding, since the compiler may contract
 * multiply-adds differently in the two kernels, and a hanging corner's
 * midpoint is interpolated after averaging the two time levels).
 * A cache holds the last chns_linearize, or the last Newton iteration of
 * chns_step, on this mesh. */
int chns_linearize(chns_mesh* mesh, const chns_params* params, int block, const double* U_new,
                   const double* U_old, int prec, void* stream);
int chns_jvp_lin(chns_mesh* mesh, const chns_params* params, int block, const void* dU, void* JdU,
                 int prec, void* stream);

/* Node-block diagonal of the block Jacobian at (U_new, U_old) (2x2 for CH,
 * 4x4 for NS per node, row-major, device, n_nodes*nf*nf doubles): the
 * diagonal blocks of P^T J P, hanging-node couplings included, the Jacobi
 * preconditioner of the Newton-Krylov solves of Sec. 3.5.  NS boundary rows
 * are identity rows.  Work memory (touch blocks) is allocated with the mesh
 * on first use. */
int chns_diag_blocks(chns_mesh* mesh, const chns_params* params, int block,
                     const double* U_new, const double* U_old, double* D, void* stream);

/* Integral of phi and total energy of U (device, n_nodes*6): kinetic
 * (1/2) rho |v|^2, free (1/(Cn We)) (psi(phi) + Cn^2/2 |grad phi|^2) and
 * gravitational (1/Fr) rho (-g^ . x) parts (Sec. 2, eqn energy_functional).
 * Synchronises the stream; results on the host. */
int chns_diagnostics(chns_mesh* mesh, const chns_params* params, const double* U,
                     double* mass, double* energy, void* stream);

typedef struct {
  double newton_rtol;  /* 1e-8: ||R|| <= max(rtol ||R_0||, atol) per block    */
  double newton_atol;  /* 1e-12                                              */
  double block_tol;    /* 1e-4: max change of all fields between two sweeps  */
  double gmres_rtol;   /* 1e-7 (FP64) / 1e-5 is typical for mixed precision  */
  int32_t newton_max_it_ch, newton_max_it_ns; /* 20, 40                      */
  int32_t gmres_restart;                      /* 1..127; 120: basis of (2m+3) block vectors */
  int32_t gmres_max_it;                       /* 1000 per linear solve       */
  int32_t block_max_it;                       /* 10                          */
  int32_t block_min_it;                       /* 1: sweeps 0 and 1 always run */
  int32_t precision;   /* 0: FP64 throughout; 1: FP32 inner Krylov (JVP,
                          preconditioner, basis) with FP64 dot products,
                          Hessenberg, update and Newton residual            */
  int32_t precond;     /* 0: point Jacobi; 1: node-block Jacobi; 2: octree
                          geometric multigrid V-cycle (below)             */
  int32_t graphs;      /* 1: each GMRES restart cycle is captured once as a
                          HIP graph (per mesh, block, precision, restart
                          length and parameters) and replayed; 0: the same
                          kernels are launched one by one.  Results are
                          identical.                                        */
  /* precond = 2: one V-cycle per preconditioner application.  The coarse
   * meshes merge the finest sibling groups level by level (chns_mesh_coarsen)
   * down to mg_levels meshes in all (0: until a mesh has at most 4096 nodes
   * or is level 1).  Coarse operators are the same element loop on the
   * coarse mesh with the state injected at its nodes; transfers are the
   * trilinear prolongation and its transpose; smoothing is damped node-block
   * Jacobi (mg_smooth sweeps before and after the coarse correction,
   * mg_coarse_sweeps on the coarsest mesh).  The V-cycle is a fixed linear
   * operator, as right preconditioning in GMRES requires. */
  double mg_omega;          /* damping of the Jacobi sweeps, 0.5            */
  int32_t mg_levels;        /* 0: automatic                                 */
  int32_t mg_smooth;        /* 2                                            */
  int32_t mg_coarse_sweeps; /* 8                                            */
  int32_t coupled;          /* 0: block iteration of Fig. 1 (a Newton solve
                               per block, sweeps until the fields settle);
                               1: one Newton solve of the whole 6-field
                               system with the coupled Jacobian
                               (chns_jvp_full) and the two blocks'
                               preconditioners side by side; newton_max_it_ns
                               bounds its iterations, and newton_its[1] /
                               gmres_its[1] of chns_step_stats count them  */
} chns_solver_opts;

typedef struct {
  int32_t block_its;
  int32_t newton_its[2]; /* indexed by CHNS_BLOCK_*, summed over sweeps      */
  int32_t gmres_its[2];
  int32_t converged;     /* every Newton solve and the block iteration met
                            their tolerances                               */
  double rel_res[2];     /* ||R_b(U^{k+1})|| / ||R_b(U^k)|| per block, both
                            evaluated at the end of the step               */
  double mass, energy;   /* diagnostics of U^{k+1}                          */
  double t_ms;           /* wall time of the step                           */
  int32_t singular_blocks; /* Newton iterations whose Jacobi or V-cycle
                            diagonal had a singular node block (replaced by
                            the identity in the preconditioner); 0 normally */
} chns_step_stats;

/* One Crank-Nicolson step (Fig. 1): U (device, n_nodes*6) holds U^k on entry
 * and U^{k+1} on return.  Synchronises the stream: Newton decisions are taken
 * on the host from device-computed FP64 norms; GMRES runs its Arnoldi
 * control (Hessenberg, Givens rotations, stopping test) on the device and
 * the host waits once per restart cycle.
 * Work buffers are allocated on first use and kept with the mesh.  Returns
 * CHNS_NOT_CONVERGED with U and stats written when a tolerance was missed. */
int chns_step(chns_mesh* mesh, const chns_params* params, const chns_solver_opts* opts,
              double* U, chns_step_stats* out, void* stream);

/* Measurement helper: enqueues `reps` back-to-back launches of one element
 * kernel alone (the per-chunk element loop, without the node gather) on
 * `stream` and returns without synchronising, so that the caller can bracket
 * them with its own HIP events on that stream.  The kernels write the mesh's
 * internal partial buffers; `out` is not used and may be NULL.  op: 0 residual
 * (FP64), 1 JVP FP64 (dU: n_nodes*6 doubles), 2 JVP FP32 (dU: n_nodes*6
 * floats), 3 node-block diagonal, 5 cached linearisation points of
 * (U_new, U_old) in FP64, 4 the JVP from them (FP64 dU), 7 and 6 the same in
 * FP32 (4 and 6 fail unless 5 or 7 ran before on the mesh and block).
 * *grid (may be NULL) receives the number of workgroups of one launch. */
int chns_launch_element_loop(chns_mesh* mesh, const chns_params* params, int block, int op,
                             const double* U_new, const double* U_old, const void* dU, void* out,
                             int reps, void* stream, int64_t* grid);

/* ------------------------------------------------ multigrid hierarchy ----
 * Host-only helpers of the octree multigrid preconditioner (precond = 2 in
 * chns_solver_opts); they also give the intergrid transfer between nested
 * octree meshes (Sec. 4 "Intergrid transfer").
 *
 * chns_mesh_coarsen: the mesh with every sibling group of its finest level
 * merged into the parent (level_max - 1).  The result is 2:1 balanced and
 * each of its nodes is a node of `mesh`.  *coarse is released with
 * chns_mesh_free. */
int chns_mesh_coarsen(const chns_mesh* mesh, chns_mesh** coarse);
/* Transfer between `fine` and `coarse` = chns_mesh_coarsen(fine).  Fine
 * independent node i takes sum_k p_w[k] * value(coarse node p_idx[k]),
 * k in [p_off[i], p_off[i+1]): the coarse trilinear field (through its
 * hanging-node constraints) evaluated at node i; weights are dyadic and
 * exact.  inj[j] is the fine node at coarse node j.  *nnz receives the
 * number of entries; any array may be NULL (sizes: p_off n_fine + 1, p_idx
 * and p_w nnz, inj n_coarse). */
int chns_mesh_transfer(const chns_mesh* fine, const chns_mesh* coarse, int64_t* nnz, int32_t* p_off,
                       int32_t* p_idx, double* p_w, int32_t* inj);

/* ------------------------------------------ remeshing and transfer ----
 * Sec. 4 "Remeshing": as the interface moves it leaves the finely refined
 * band, so the octree is rebuilt around the current phi and the fields are
 * carried over by the intergrid transfer.
 *
 * chns_mesh_remesh: a new mesh of the same brick, refined top-down and 2:1
 * balanced exactly as chns_mesh_build does, with phi0 replaced by the
 * trilinear field of phi = U_host[6i] on `mesh` (host array, n_nodes*6).
 * Host only; *out is released with chns_mesh_free. */
int chns_mesh_remesh(const chns_mesh* mesh, const double* U_host, int level_min, int level_max,
                     double band, chns_mesh** out);
/* Intergrid transfer between any two meshes of one brick: node i of `to`
 * takes sum_k w[k] * (node idx[k] of `from`), k in [off[i], off[i+1]), the
 * trilinear field of `from` (through its hanging constraints) at that node.
 * chns_mesh_interp_weights returns the lists (host only; arrays may be NULL,
 * sizes off n_to + 1, idx and w *nnz).  chns_mesh_interpolate applies them
 * to all 6 fields on the device (U_from: from's n_nodes*6, U_to: to's);
 * with conserve_mass != 0 it then shifts phi by the constant that restores
 * the integral of phi (params needed for that, else may be NULL).
 * Synchronises the stream. */
int chns_mesh_interp_weights(const chns_mesh* from, const chns_mesh* to, int64_t* nnz, int32_t* off,
                             int32_t* idx, double* w);
int chns_mesh_interpolate(chns_mesh* from, chns_mesh* to, const double* U_from, double* U_to,
                          const chns_params* params, int conserve_mass, void* stream);

/* ------------------------------------------------------------ serving ----
 * A request loop for many independent droplet / bubble problems of different
 * octree sizes.  Each request is (mesh spec, parameters, number of Crank-
 * Nicolson steps); its initial state is phi = phi0 at the nodes, mu = phi^3 -
 * phi, v = 0, p = 0.  A builder thread inside the server makes the host mesh,
 * the scatter plan and U^0 of queued requests while the GPU works.
 * chns_server_run_round admits built requests in arrival order while their
 * device footprint fits in the HBM budget (mesh arrays + solver workspace for
 * the server's options, exact; with precond = 2 plus a bound for the coarse
 * levels: the fine mesh's size again), a request that does not fit yet
 * letting later, smaller ones pass.  An admitted request is uploaded on a
 * stream of its own and a driver thread of its own runs its steps back to
 * back, so the element loops and Krylov kernels of all residents overlap on
 * the device and no request waits for another's step; GMRES cycles are
 * replayed as HIP graphs.  After its last step a request's final state is
 * copied to host memory the server owns and its device memory is freed,
 * which lets the next round admit more.  Requests never share data, so a
 * request's result does not depend on what else is resident.  One host
 * thread drives a server (submit, poll and run_round). */
typedef struct chns_server chns_server;

enum {
  CHNS_REQ_QUEUED = 0,   /* waiting for the builder                        */
  CHNS_REQ_READY = 1,    /* mesh and U^0 built, waiting for device memory  */
  CHNS_REQ_RESIDENT = 2, /* on the device, stepping                        */
  CHNS_REQ_DONE = 3,     /* all steps taken; final state on the host       */
  CHNS_REQ_FAILED = 4    /* build, upload or a step returned an error      */
};

typedef struct {
  int32_t state;            /* CHNS_REQ_*                                   */
  int32_t status;           /* last library status of the request           */
  int32_t n_steps, steps_done;
  int64_t n_leaves, n_nodes;
  int64_t footprint_bytes;  /* device bytes reserved while resident         */
  double t_submit_ms, t_admit_ms, t_done_ms; /* since server creation       */
} chns_request_info;

typedef struct {
  int64_t queued, ready, resident, done, failed;
  int64_t bytes_in_use, budget_bytes;
  int64_t rounds, steps;
} chns_server_stats;

/* Creates a server on the current device.  hbm_budget_bytes bounds the sum
 * of the footprints of resident requests; max_resident bounds their number
 * (1..64); opts apply to every step (graphs forced on).  Up to max_resident
 * driver threads run at once. */
int chns_server_create(size_t hbm_budget_bytes, int max_resident, const chns_solver_opts* opts,
                       chns_server** out);
/* Queues a request.  spec is copied (including explicit leaves); spec->phi0
 * and spec->user must stay valid until the request leaves CHNS_REQ_QUEUED
 * (the builder thread calls phi0).  params are validated here.  *ticket
 * identifies the request (increasing from 0). */
int chns_server_submit(chns_server* srv, const chns_mesh_spec* spec, const chns_params* params,
                       int n_steps, int64_t* ticket);
/* State of a request.  Any output may be NULL.  U_host_out (n_nodes*6
 * doubles, see info->n_nodes) is written once the request is DONE;
 * per_step (n_steps entries) and step_latency_ms (n_steps doubles: from the
 * moment the step became runnable, i.e. admission or the end of the
 * request's previous step, to its end) receive the steps taken so far. */
int chns_server_poll(chns_server* srv, int64_t ticket, chns_request_info* info,
                     double* U_host_out, chns_step_stats* per_step, double* step_latency_ms);
/* One scheduling round: joins the drivers of requests that have left,
 * admits what fits (uploads start after the work already queued on
 * `stream`), then waits up to 20 ms for progress (a step ending, a request
 * leaving or becoming READY).  Returns the number of steps that ended during
 * the call (>= 0), or a negative status for a failure of the server itself;
 * a failing request only moves to CHNS_REQ_FAILED. */
int chns_server_run_round(chns_server* srv, void* stream);
int chns_server_stats_get(chns_server* srv, chns_server_stats* out);
/* Stops the builder, frees every request's device and host memory. */
int chns_server_destroy(chns_server* srv);

/* ---------------------------------------------------------- cG(2) blocks ---
 * Triquadratic (27-node) elements on the leaves of a mesh: the paper
 * discretises with cG(1) (Sec. 3.4) and names higher-order cG spaces as the
 * next step (Sec. 7).  Nodes are the 3x3x3 lattice of every leaf; a lattice
 * point that is not on the lattice of some other leaf whose closure contains
 * it hangs, and takes the triquadratic interpolant of the coarsest such leaf
 * (Sec. 4 "Handling hanging nodes", carried over), with hanging parents
 * substituted.  Independent nodes are numbered in Morton order of their
 * coordinates in units of 2^-(level_max+1); wall and pressure-pin flags
 * follow the cG(1) mesh's rules.  Integrals use the 3x3x3 Gauss rule; the
 * rows are those of chns_residual for the same block on the cG(2) space,
 * except that the NS strong residual R_m keeps the Laplacian parts of the
 * capillary and viscous divergences (zero on trilinear leaves).  FP64 only. */
typedef struct chns_q2 chns_q2;
/* Builds the numbering and its gather plan on the host and copies them to
 * the current device (which must be the mesh's; the mesh is uploaded first if
 * needed).  The mesh must outlive the returned object. */
int chns_q2_build(chns_mesh* mesh, chns_q2** out, void* stream);
/* Sizes (any output may be NULL): independent nodes, hanging nodes,
 * constraint entries, device bytes held by the numbering. */
int chns_q2_info(const chns_q2* q, int64_t* n_nodes, int64_t* n_hanging, int64_t* n_constraint,
                 int64_t* device_bytes);
/* Physical coordinates of the independent nodes (host, n_nodes*3). */
int chns_q2_nodes(const chns_q2* q, double* xyz);
/* Residual rows of a block over the Q2 nodes.  U_new, U_old, R: device,
 * node-major n_nodes*6 FP64 (phi, mu, u, v, w, p); the state vectors must be
 * 16-byte aligned (node records are read as 16-byte loads), else
 * CHNS_EINVAL.  CH: R's fields 0, 1 (the
 * velocities enter as the frozen v~ of the block iteration); NS: fields 2..5,
 * velocity rows of wall nodes v^{k+1} - v^k and the pinned pressure row
 * p^{k+1} - p^k.  The other block's fields are set to 0.  A point whose
 * tau_m bracket is not positive gives non-finite rows.  Asynchronous on
 * `stream`. */
int chns_q2_residual(chns_q2* q, const chns_params* params, int block, const double* U_new,
                     const double* U_old, double* R, void* stream);
/* The block's Jacobian (derivative in its own unknowns) applied to dU
 * (device, n_nodes*6; the block's fields are read); JdU like R above, with
 * identity rows on the NS wall and pin rows. */
int chns_q2_jvp(chns_q2* q, const chns_params* params, int block, const double* U_new,
                const double* U_old, const double* dU, double* JdU, void* stream);
int chns_q2_free(chns_q2* q);
/* Host-only view of the same numbering (no device needed): sizes[0..2] =
 * independent nodes, hanging nodes, constraint entries; then, for non-NULL
 * outputs (caller-allocated from the sizes; a first call with NULL arrays
 * gives them): the 27 refs per leaf (id, or -1 - hanging index), node and
 * hanging-node coordinates (n*3), the constraint rows as CSR (hang_off of
 * n_hanging+1 entries into hang_ids / hang_w, ascending ids) and the nodes'
 * wall / pressure-pin flags.  Builds the numbering on every call. */
int chns_q2_host_arrays(const chns_mesh* mesh, int64_t* sizes, int32_t* elem27, double* node_xyz,
                        double* hang_xyz, int32_t* hang_off, int32_t* hang_ids, double* hang_w,
                        uint8_t* bflags);

const char* chns_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CHNS_H */
