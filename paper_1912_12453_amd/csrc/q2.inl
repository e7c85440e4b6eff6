// cG(2) Cahn-Hilliard block on the octree: triquadratic leaves (27 nodes),
// the 3x3x3 Gauss rule, the residual rows of Def. 2's chemical-potential and
// CH equations (eqns mu_eqn_var_semi_disc, phi_eqn_var_semi_disc) with the
// Crank-Nicolson midpoints of the cG(1) element loop, and their Jacobian in
// the direction of (phi^{k+1}, mu^{k+1}).  The paper discretises with cG(1)
// (Sec. 3.4) and names higher-order cG spaces as the next step (Sec. 7).
//
// Device layout: one 64-lane wave per two leaves, 32 lanes per leaf (27 in
// use).  Lane a gathers local node a's fields (through its constraint row
// when it hangs) into LDS; lane g evaluates the fields at Gauss point g from
// the 27 nodal values with the tensor-product basis and writes the point's
// coefficients (c, F) to LDS; lane a then contracts them against its test
// function.  Element results go to an E x 27 x 2 array; the gather kernel
// sums them per node through the host-built fixed-order plan (leaf, local
// node, constraint weight), so the result does not depend on scheduling.
// Included by capi.hip.

namespace chns {
namespace dev {

constexpr double kQ2Gauss = 0.77459666924148337704;  // sqrt(3/5)

// basis with nodes 0, 1/2, 1 on [0, 1] and its derivative d/du
__device__ __forceinline__ void q2_basis_1d(double u, double (&b)[3], double (&d)[3]) {
  b[0] = 2.0 * (u - 0.5) * (u - 1.0);
  b[1] = 4.0 * u * (1.0 - u);
  b[2] = 2.0 * u * (u - 0.5);
  d[0] = 4.0 * u - 3.0;
  d[1] = 4.0 - 8.0 * u;
  d[2] = 4.0 * u - 1.0;
}
__device__ __forceinline__ double q2_gauss_u(int g) {
  return g == 1 ? 0.5 : (g == 0 ? 0.5 - 0.5 * kQ2Gauss : 0.5 + 0.5 * kQ2Gauss);
}
__device__ __forceinline__ double q2_gauss_w(int g) { return g == 1 ? 8.0 / 18.0 : 5.0 / 18.0; }

struct Q2View {
  const int32_t* elem;   // E x 27: node id, or -1 - hanging entry
  const uint8_t* level;  // E
  const int32_t* hoff;   // NH + 1
  const int32_t* hids;
  const double* hw;
  int64_t E;
};

__device__ __forceinline__ double q2_node(const Q2View& q, int32_t ref, const double* __restrict__ U, int f) {
  if (ref >= 0) return U[(int64_t)ref * 6 + f];
  const int32_t hh = -1 - ref;
  double s = 0.0;
  for (int32_t t = q.hoff[hh]; t < q.hoff[hh + 1]; ++t) s += q.hw[t] * U[(int64_t)q.hids[t] * 6 + f];
  return s;
}

// MODE 0: residual rows; MODE 1: Jacobian rows applied to dU (phi, mu parts).
template <int MODE>
__global__ __launch_bounds__(64) void k_q2_ch(Q2View q, PhysView p, const double* __restrict__ U1,
                                              const double* __restrict__ U0, const double* __restrict__ dU,
                                              double* __restrict__ part) {
  __shared__ double sn[2][6][27];  // per leaf: three scalar fields and v~ at the nodes
  __shared__ double sq[2][8][27];  // per leaf: c and F of the two rows at the points
  const int half = threadIdx.x >> 5, lane = threadIdx.x & 31;
  const int64_t e0 = (int64_t)blockIdx.x * 2 + half;
  const bool live = e0 < q.E;
  const int64_t e = live ? e0 : q.E - 1;
  const int lev = q.level[e];
  const double h = ldexp(1.0, -lev), ih = ldexp(1.0, lev);
  if (lane < 27) {
    const int32_t ref = q.elem[e * 27 + lane];
    const double p1 = q2_node(q, ref, U1, 0), p0 = q2_node(q, ref, U0, 0);
    sn[half][0][lane] = 0.5 * (p1 + p0);  // phi~
    if (MODE == 0) {
      sn[half][1][lane] = 0.5 * (q2_node(q, ref, U1, 1) + q2_node(q, ref, U0, 1));  // mu~
      sn[half][2][lane] = p1 - p0;                                                  // phi^{k+1} - phi^k
    } else {
      sn[half][1][lane] = q2_node(q, ref, dU, 1);  // d mu^{k+1}
      sn[half][2][lane] = q2_node(q, ref, dU, 0);  // d phi^{k+1}
    }
    for (int d = 0; d < 3; ++d)
      sn[half][3 + d][lane] = 0.5 * (q2_node(q, ref, U1, 2 + d) + q2_node(q, ref, U0, 2 + d));
  }
  __syncthreads();
  if (lane < 27) {
    const int g0 = lane % 3, g1 = (lane / 3) % 3, g2 = lane / 9;
    double bx[3], dx[3], by[3], dy[3], bz[3], dz[3];
    q2_basis_1d(q2_gauss_u(g0), bx, dx);
    q2_basis_1d(q2_gauss_u(g1), by, dy);
    q2_basis_1d(q2_gauss_u(g2), bz, dz);
    double val[3] = {0.0, 0.0, 0.0}, grd[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    double v[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 27; ++a) {
      const int i = a % 3, j = (a / 3) % 3, k = a / 9;
      const double yz = by[j] * bz[k];
      const double N = bx[i] * yz, Nx = dx[i] * yz * ih, Ny = bx[i] * dy[j] * bz[k] * ih,
                   Nz = bx[i] * by[j] * dz[k] * ih;
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        const double u = sn[half][f][a];
        val[f] += N * u;
        grd[f][0] += Nx * u;
        grd[f][1] += Ny * u;
        grd[f][2] += Nz * u;
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) v[d] += N * sn[half][3 + d][a];
    }
    const double w = q2_gauss_w(g0) * q2_gauss_w(g1) * q2_gauss_w(g2) * h * h * h;
    const double kd = p.inv_PeCn, cn2 = p.Cn2, pt = val[0];
    double c0, c1, F0[3], F1[3];
    if (MODE == 0) {
      // (q, (phi^{k+1}-phi^k)/dt) - (grad q, v~ phi~) + 1/(Pe Cn) (grad q, grad mu~)
      // -(q, mu~) + (q, psi'(phi~)) + Cn^2 (grad q, grad phi~)
      c0 = val[2] * p.inv_dt;
      c1 = pt * pt * pt - pt - val[1];
      for (int d = 0; d < 3; ++d) {
        F0[d] = kd * grd[1][d] - v[d] * pt;
        F1[d] = cn2 * grd[0][d];
      }
    } else {
      // the same rows' derivative: phi~ and mu~ move by half the direction
      c0 = val[2] * p.inv_dt;
      c1 = (3.0 * pt * pt - 1.0) * 0.5 * val[2] - 0.5 * val[1];
      for (int d = 0; d < 3; ++d) {
        F0[d] = kd * 0.5 * grd[1][d] - v[d] * 0.5 * val[2];
        F1[d] = cn2 * 0.5 * grd[2][d];
      }
    }
    sq[half][0][lane] = w * c0;
    sq[half][4][lane] = w * c1;
    for (int d = 0; d < 3; ++d) {
      sq[half][1 + d][lane] = w * F0[d];
      sq[half][5 + d][lane] = w * F1[d];
    }
  }
  __syncthreads();
  if (lane < 27 && live) {
    const int ia = lane % 3, ja = (lane / 3) % 3, ka = lane / 9;
    double cx[3], cy[3], cz[3], ex[3], ey[3], ez[3];
    for (int g = 0; g < 3; ++g) {
      double b[3], d[3];
      q2_basis_1d(q2_gauss_u(g), b, d);
      cx[g] = b[ia];
      ex[g] = d[ia] * ih;
      cy[g] = b[ja];
      ey[g] = d[ja] * ih;
      cz[g] = b[ka];
      ez[g] = d[ka] * ih;
    }
    double r0 = 0.0, r1 = 0.0;
    for (int g = 0; g < 27; ++g) {
      const int g0 = g % 3, g1 = (g / 3) % 3, g2 = g / 9;
      const double N = cx[g0] * cy[g1] * cz[g2], Nx = ex[g0] * cy[g1] * cz[g2], Ny = cx[g0] * ey[g1] * cz[g2],
                   Nz = cx[g0] * cy[g1] * ez[g2];
      r0 += N * sq[half][0][g] + Nx * sq[half][1][g] + Ny * sq[half][2][g] + Nz * sq[half][3][g];
      r1 += N * sq[half][4][g] + Nx * sq[half][5][g] + Ny * sq[half][6][g] + Nz * sq[half][7][g];
    }
    part[(e * 27 + lane) * 2] = r0;
    part[(e * 27 + lane) * 2 + 1] = r1;
  }
}

// out[n][0..1] = sum over the node's plan entries of weight x element result;
// out[n][2..5] = 0 (the CH block's rows only)
__global__ __launch_bounds__(256) void k_q2_gather(int64_t n, const int64_t* __restrict__ goff,
                                                   const int32_t* __restrict__ gslot,
                                                   const double* __restrict__ gw,
                                                   const double* __restrict__ part, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s0 = 0.0, s1 = 0.0;
    for (int64_t k = goff[i]; k < goff[i + 1]; ++k) {
      const int64_t t = gslot[k];
      s0 += gw[k] * part[t * 2];
      s1 += gw[k] * part[t * 2 + 1];
    }
    double* o = out + i * 6;
    o[0] = s0;
    o[1] = s1;
    o[2] = o[3] = o[4] = o[5] = 0.0;
  }
}

}  // namespace dev
}  // namespace chns

struct chns_q2 {
  chns_mesh* m = nullptr;
  HostQ2 h;
  int device = -1;
  int32_t *d_elem = nullptr, *d_hoff = nullptr, *d_hids = nullptr, *d_gslot = nullptr;
  double *d_hw = nullptr, *d_gw = nullptr, *d_part = nullptr;
  int64_t* d_goff = nullptr;
  int64_t bytes = 0;
};

namespace {

void free_q2_locked(chns_q2* q) {
  (void)hipFree(q->d_elem);
  (void)hipFree(q->d_hoff);
  (void)hipFree(q->d_hids);
  (void)hipFree(q->d_gslot);
  (void)hipFree(q->d_hw);
  (void)hipFree(q->d_gw);
  (void)hipFree(q->d_part);
  (void)hipFree(q->d_goff);
}

int q2_launch(chns_q2* q, const chns_params* params, const double* U1, const double* U0, const double* dU,
              double* out, void* stream, int mode) {
  if (!q) return fail(CHNS_EINVAL, "Q2 numbering is NULL");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != q->device) return fail(CHNS_EINVAL, "Q2 numbering was built on another device");
  dev::PhysView pv;
  int rc = phys_view(params, pv);
  if (rc) return rc;
  if (!U1 || !U0 || !out || (mode == 1 && !dU)) return fail(CHNS_EINVAL, "pointers must not be NULL");
  const int64_t E = (int64_t)q->m->h.leaf_key.size(), n = (int64_t)q->h.node_key.size();
  dev::Q2View v{q->d_elem, q->m->d_level, q->d_hoff, q->d_hids, q->d_hw, E};
  const dim3 g((unsigned)((E + 1) / 2)), b(64);
  if (mode == 0)
    hipLaunchKernelGGL(dev::k_q2_ch<0>, g, b, 0, s, v, pv, U1, U0, (const double*)nullptr, q->d_part);
  else
    hipLaunchKernelGGL(dev::k_q2_ch<1>, g, b, 0, s, v, pv, U1, U0, dU, q->d_part);
  hipLaunchKernelGGL(dev::k_q2_gather, dim3(grid_stride(n)), dim3(256), 0, s, n, q->d_goff, q->d_gslot, q->d_gw,
                     q->d_part, out);
  HIPCHK(hipGetLastError());
  return CHNS_OK;
}

}  // namespace

extern "C" {

int chns_q2_build(chns_mesh* m, chns_q2** out, void* stream) {
  if (!out) return fail(CHNS_EINVAL, "out must not be NULL");
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  int rc = check_mesh(m, s);  // the leaf levels are read from the mesh's device copy
  if (rc) return rc;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != m->device) return fail(CHNS_EINVAL, "mesh was uploaded to another device");
  chns_q2* q = new (std::nothrow) chns_q2();
  if (!q) return fail(CHNS_ENOMEM, "out of host memory");
  q->m = m;
  q->device = dev;
  std::string err;
  try {
    err = build_host_q2(m->h, q->h);
  } catch (const std::bad_alloc&) {
    err = "out of host memory building the Q2 numbering";
  }
  if (!err.empty()) {
    delete q;
    return fail(CHNS_EINVAL, err);
  }
  const HostQ2& H = q->h;
  const size_t E = m->h.leaf_key.size();
  {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    int64_t* B = &q->bytes;
    if ((rc = dalloc(&q->d_elem, H.elem.size(), B)) || (rc = dalloc(&q->d_hoff, H.hang_off.size(), B)) ||
        (rc = dalloc(&q->d_hids, H.hang_ids.size(), B)) || (rc = dalloc(&q->d_hw, H.hang_w.size(), B)) ||
        (rc = dalloc(&q->d_goff, H.g_off.size(), B)) || (rc = dalloc(&q->d_gslot, H.g_slot.size(), B)) ||
        (rc = dalloc(&q->d_gw, H.g_w.size(), B)) || (rc = dalloc(&q->d_part, E * 27 * 2, B))) {
      free_q2_locked(q);
      delete q;
      return rc;
    }
  }
  if ((rc = h2d(q->d_elem, H.elem, s)) || (rc = h2d(q->d_hoff, H.hang_off, s)) ||
      (rc = h2d(q->d_hids, H.hang_ids, s)) || (rc = h2d(q->d_hw, H.hang_w, s)) ||
      (rc = h2d(q->d_goff, H.g_off, s)) || (rc = h2d(q->d_gslot, H.g_slot, s)) || (rc = h2d(q->d_gw, H.g_w, s))) {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    free_q2_locked(q);
    delete q;
    return rc;
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    free_q2_locked(q);
    delete q;
    return fail(CHNS_EHIP, "hipStreamSynchronize after the Q2 upload failed");
  }
  *out = q;
  return CHNS_OK;
}

int chns_q2_info(const chns_q2* q, int64_t* n_nodes, int64_t* n_hanging, int64_t* n_constraint,
                 int64_t* device_bytes) {
  if (!q) return fail(CHNS_EINVAL, "Q2 numbering is NULL");
  if (n_nodes) *n_nodes = (int64_t)q->h.node_key.size();
  if (n_hanging) *n_hanging = (int64_t)q->h.hang_key.size();
  if (n_constraint) *n_constraint = (int64_t)q->h.hang_ids.size();
  if (device_bytes) *device_bytes = q->bytes;
  return CHNS_OK;
}

int chns_q2_nodes(const chns_q2* q, double* xyz) {
  if (!q || !xyz) return fail(CHNS_EINVAL, "pointers must not be NULL");
  const double unit = std::ldexp(1.0, -(q->m->h.D + 1));
  for (size_t i = 0; i < q->h.node_key.size(); ++i) {
    uint32_t x, y, z;
    unkey(q->h.node_key[i], x, y, z);
    xyz[3 * i] = x * unit;
    xyz[3 * i + 1] = y * unit;
    xyz[3 * i + 2] = z * unit;
  }
  return CHNS_OK;
}

int chns_q2_residual(chns_q2* q, const chns_params* params, const double* U_new, const double* U_old, double* R,
                     void* stream) {
  return q2_launch(q, params, U_new, U_old, nullptr, R, stream, 0);
}

int chns_q2_jvp(chns_q2* q, const chns_params* params, const double* U_new, const double* U_old, const double* dU,
                double* JdU, void* stream) {
  return q2_launch(q, params, U_new, U_old, dU, JdU, stream, 1);
}

int chns_q2_host_arrays(const chns_mesh* m, int64_t* sizes, int32_t* elem27, double* node_xyz, double* hang_xyz,
                        int32_t* hang_off, int32_t* hang_ids, double* hang_w) {
  if (!m || !sizes) return fail(CHNS_EINVAL, "mesh and sizes must not be NULL");
  HostQ2 H;
  std::string err;
  try {
    err = build_host_q2(m->h, H);
  } catch (const std::bad_alloc&) {
    err = "out of host memory building the Q2 numbering";
  }
  if (!err.empty()) return fail(CHNS_EINVAL, err);
  sizes[0] = (int64_t)H.node_key.size();
  sizes[1] = (int64_t)H.hang_key.size();
  sizes[2] = (int64_t)H.hang_ids.size();
  const double unit = std::ldexp(1.0, -(m->h.D + 1));
  auto coords = [&](const std::vector<uint64_t>& keys, double* out) {
    for (size_t i = 0; i < keys.size(); ++i) {
      uint32_t x, y, z;
      unkey(keys[i], x, y, z);
      out[3 * i] = x * unit;
      out[3 * i + 1] = y * unit;
      out[3 * i + 2] = z * unit;
    }
  };
  if (elem27) std::copy(H.elem.begin(), H.elem.end(), elem27);
  if (node_xyz) coords(H.node_key, node_xyz);
  if (hang_xyz) coords(H.hang_key, hang_xyz);
  if (hang_off) std::copy(H.hang_off.begin(), H.hang_off.end(), hang_off);
  if (hang_ids) std::copy(H.hang_ids.begin(), H.hang_ids.end(), hang_ids);
  if (hang_w) std::copy(H.hang_w.begin(), H.hang_w.end(), hang_w);
  return CHNS_OK;
}

int chns_q2_free(chns_q2* q) {
  if (!q) return CHNS_OK;
  {
    std::lock_guard<std::mutex> lk(g_struct_mu);
    free_q2_locked(q);
  }
  delete q;
  return CHNS_OK;
}

}  // extern "C"
