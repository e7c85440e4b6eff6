// cG(2) blocks on the octree: triquadratic leaves (27 nodes), the 3x3x3
// Gauss rule, and the residual rows and block Jacobians of the cG(1) element
// loop on that space: the CH block (Def. 2's chemical-potential and CH
// equations, eqns mu_eqn_var_semi_disc, phi_eqn_var_semi_disc) and the VMS
// Navier-Stokes block, whose strong residual R_m keeps the Laplacian parts of
// the capillary and viscous divergences (they vanish on trilinear leaves).
// The paper discretises with cG(1) (Sec. 3.4) and names higher-order cG
// spaces as the next step (Sec. 7).
//
// Device layout: one 64-lane wave per two leaves, 32 lanes per leaf (27 in
// use).  Lane a gathers local node a's fields (through its constraint row
// when it hangs) into LDS; the fields are evaluated at the 27 Gauss points
// (CH: sum factorisation, three 3-term passes; NS: 27-term sums with the
// tensor-product basis, Hessians included), each point's coefficients (c, F)
// go to LDS, and lane a contracts them against its test function.  Element
// results go to an E x 27 x NF array; the gather kernel sums them per node
// through the host-built fixed-order plan (leaf, local node, constraint
// weight), so the result does not depend on scheduling.
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

// The six fields of a node (or, for a hanging node, its constraint row's
// combination) as three 16-byte loads per node record: the row's ids and
// weights are read once for all fields.  Node records are 48 bytes, so a
// 16-byte aligned vector keeps every record 16-byte aligned.
__device__ __forceinline__ void q2_load6(const double* __restrict__ U, int64_t id, double (&o)[6]) {
  const double2* r = reinterpret_cast<const double2*>(U + id * 6);
  const double2 x = r[0], y = r[1], z = r[2];
  o[0] = x.x;
  o[1] = x.y;
  o[2] = y.x;
  o[3] = y.y;
  o[4] = z.x;
  o[5] = z.y;
}
__device__ __forceinline__ void q2_node6(const Q2View& q, int32_t ref, const double* __restrict__ U,
                                         double (&o)[6]) {
  if (ref >= 0) {
    q2_load6(U, ref, o);
    return;
  }
  const int32_t hh = -1 - ref;
  for (int f = 0; f < 6; ++f) o[f] = 0.0;
  for (int32_t t = q.hoff[hh]; t < q.hoff[hh + 1]; ++t) {
    double v[6];
    q2_load6(U, q.hids[t], v);
    const double w = q.hw[t];
    for (int f = 0; f < 6; ++f) o[f] += w * v[f];
  }
}

// second derivative d2/du2 of the basis on [0, 1] with nodes 0, 1/2, 1
__device__ __forceinline__ double q2_basis_dd(int i) { return i == 1 ? -8.0 : 4.0; }


// MODE 0: residual rows; MODE 1: Jacobian rows applied to dU (phi, mu parts).
// Sum factorisation on the tensor-product lattice: the 27-point evaluation
// is three passes of 3-term sums, one axis at a time (x, then y, then z),
// and the contraction the same passes transposed (z, y, x).  Lane l of a
// leaf stands for the index triple (l % 3, l / 3 % 3, l / 9) of the pass;
// each pass reads the previous one's LDS array and writes the next, so one
// leaf needs two LDS buffers of 12 x 27 values.
template <int MODE>
__global__ __launch_bounds__(64) void k_q2_ch(Q2View q, PhysView p, const double* __restrict__ U1,
                                              const double* __restrict__ U0, const double* __restrict__ dU,
                                              double* __restrict__ part) {
  __shared__ double sa[2][12][27];
  __shared__ double sb[2][12][27];
  const int half = threadIdx.x >> 5, lane = threadIdx.x & 31;
  const int64_t e0 = (int64_t)blockIdx.x * 2 + half;
  const bool live = e0 < q.E;
  const int64_t e = live ? e0 : q.E - 1;
  const int lev = q.level[e];
  const double h = ldexp(1.0, -lev), ih = ldexp(1.0, lev);
  // B[g][i], Dh[g][i]: basis i and its physical derivative at Gauss coordinate g
  double B[3][3], Dh[3][3];
  for (int g = 0; g < 3; ++g) {
    double b[3], d[3];
    q2_basis_1d(q2_gauss_u(g), b, d);
    for (int i = 0; i < 3; ++i) {
      B[g][i] = b[i];
      Dh[g][i] = d[i] * ih;
    }
  }
  const bool act = lane < 27;
  const int p0 = lane % 3, p1 = (lane / 3) % 3, p2 = lane / 9;
  double (*A)[27] = sa[half];
  double (*C)[27] = sb[half];
  // nodal fields: 0 phi~, 1 mu~ (residual) or d mu^{k+1} (JVP), 2 phi^{k+1} - phi^k
  // (residual) or d phi^{k+1} (JVP), 3..5 v~
  if (act) {
    const int32_t ref = q.elem[e * 27 + lane];
    double a1[6], a0[6];
    q2_node6(q, ref, U1, a1);
    q2_node6(q, ref, U0, a0);
    A[0][lane] = 0.5 * (a1[0] + a0[0]);
    if (MODE == 0) {
      A[1][lane] = 0.5 * (a1[1] + a0[1]);
      A[2][lane] = a1[0] - a0[0];
    } else {
      double dd[6];
      q2_node6(q, ref, dU, dd);
      A[1][lane] = dd[1];
      A[2][lane] = dd[0];
    }
    for (int d = 0; d < 3; ++d) A[3 + d][lane] = 0.5 * (a1[2 + d] + a0[2 + d]);
  }
  __syncthreads();
  // x pass, lane (g0, j, k): values of all six fields, x-derivatives of the first three
  if (act) {
    for (int f = 0; f < 6; ++f) {
      const double* u = A[f] + 3 * p1 + 9 * p2;
      C[f][lane] = B[p0][0] * u[0] + B[p0][1] * u[1] + B[p0][2] * u[2];
      if (f < 3) C[6 + f][lane] = Dh[p0][0] * u[0] + Dh[p0][1] * u[1] + Dh[p0][2] * u[2];
    }
  }
  __syncthreads();
  // y pass, lane (g0, g1, k): values; y-derivatives of values; x-derivatives carried
  if (act) {
    for (int f = 0; f < 6; ++f) {
      const double* u = C[f] + p0 + 9 * p2;
      A[f][lane] = B[p1][0] * u[0] + B[p1][1] * u[3] + B[p1][2] * u[6];
      if (f < 3) {
        A[6 + f][lane] = Dh[p1][0] * u[0] + Dh[p1][1] * u[3] + Dh[p1][2] * u[6];
        const double* t = C[6 + f] + p0 + 9 * p2;
        A[9 + f][lane] = B[p1][0] * t[0] + B[p1][1] * t[3] + B[p1][2] * t[6];
      }
    }
  }
  __syncthreads();
  // z pass at Gauss point (g0, g1, g2), then the point's coefficients
  if (act) {
    double val[6], grd[3][3];
    for (int f = 0; f < 6; ++f) {
      const double* u = A[f] + p0 + 3 * p1;
      val[f] = B[p2][0] * u[0] + B[p2][1] * u[9] + B[p2][2] * u[18];
      if (f < 3) {
        const double* ty = A[6 + f] + p0 + 3 * p1;
        const double* tx = A[9 + f] + p0 + 3 * p1;
        grd[f][0] = B[p2][0] * tx[0] + B[p2][1] * tx[9] + B[p2][2] * tx[18];
        grd[f][1] = B[p2][0] * ty[0] + B[p2][1] * ty[9] + B[p2][2] * ty[18];
        grd[f][2] = Dh[p2][0] * u[0] + Dh[p2][1] * u[9] + Dh[p2][2] * u[18];
      }
    }
    const double w = q2_gauss_w(p0) * q2_gauss_w(p1) * q2_gauss_w(p2) * h * h * h;
    const double kd = p.inv_PeCn, cn2 = p.Cn2, pt = val[0];
    const double v[3] = {val[3], val[4], val[5]};
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
    C[0][lane] = w * c0;
    C[4][lane] = w * c1;
    for (int d = 0; d < 3; ++d) {
      C[1 + d][lane] = w * F0[d];
      C[5 + d][lane] = w * F1[d];
    }
  }
  __syncthreads();
  // transposed z pass, lane (g0, g1, k): per row r, the terms with factor
  // N_x N_y (c and F_z), N_x' N_y (F_x) and N_x N_y' (F_y)
  if (act) {
    for (int r = 0; r < 2; ++r) {
      const double* c = C[4 * r] + p0 + 3 * p1;
      const double* fx = C[4 * r + 1] + p0 + 3 * p1;
      const double* fy = C[4 * r + 2] + p0 + 3 * p1;
      const double* fz = C[4 * r + 3] + p0 + 3 * p1;
      double s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int g2 = 0; g2 < 3; ++g2) {
        s1 += B[g2][p2] * c[9 * g2] + Dh[g2][p2] * fz[9 * g2];
        s2 += B[g2][p2] * fx[9 * g2];
        s3 += B[g2][p2] * fy[9 * g2];
      }
      A[3 * r][lane] = s1;
      A[3 * r + 1][lane] = s2;
      A[3 * r + 2][lane] = s3;
    }
  }
  __syncthreads();
  // transposed y pass, lane (g0, j, k)
  if (act) {
    for (int r = 0; r < 2; ++r) {
      const double* t1 = A[3 * r] + p0 + 9 * p2;
      const double* t2 = A[3 * r + 1] + p0 + 9 * p2;
      const double* t3 = A[3 * r + 2] + p0 + 9 * p2;
      double s1 = 0.0, s2 = 0.0;
      for (int g1 = 0; g1 < 3; ++g1) {
        s1 += B[g1][p1] * t1[3 * g1] + Dh[g1][p1] * t3[3 * g1];
        s2 += B[g1][p1] * t2[3 * g1];
      }
      C[2 * r][lane] = s1;
      C[2 * r + 1][lane] = s2;
    }
  }
  __syncthreads();
  // transposed x pass, lane = node (i, j, k)
  if (act && live) {
    for (int r = 0; r < 2; ++r) {
      const double* t1 = C[2 * r] + 3 * p1 + 9 * p2;
      const double* t2 = C[2 * r + 1] + 3 * p1 + 9 * p2;
      double s = 0.0;
      for (int g0 = 0; g0 < 3; ++g0) s += B[g0][p0] * t1[g0] + Dh[g0][p0] * t2[g0];
      part[(e * 27 + lane) * 2 + r] = s;
    }
  }
}

// NS block on one leaf.  MODE 0: residual rows; MODE 1: the block Jacobian
// (derivative in v^{k+1}, p^{k+1}) applied to dU.  The point quantities are
// those of the cG(1) kernels (NSPoint, ns_material, ns_stab, ns_jvp_coef)
// with R_m completed by -(eta/Re) lap v~ and (Cn/We) grad phi~ lap phi~.
template <int MODE>
__global__ __launch_bounds__(64) void k_q2_ns(Q2View q, PhysView p, const double* __restrict__ U1,
                                              const double* __restrict__ U0, const double* __restrict__ dU,
                                              double* __restrict__ part) {
  constexpr int NS_ = MODE == 0 ? 10 : 14;  // nodal arrays per leaf
  __shared__ double sn[2][NS_][27];
  __shared__ double sq[2][16][27];
  const int half = threadIdx.x >> 5, lane = threadIdx.x & 31;
  const int64_t e0 = (int64_t)blockIdx.x * 2 + half;
  const bool live = e0 < q.E;
  const int64_t e = live ? e0 : q.E - 1;
  const int lev = q.level[e];
  const double h = ldexp(1.0, -lev), ih = ldexp(1.0, lev), ih2 = ih * ih;
  if (lane < 27) {
    const int32_t ref = q.elem[e * 27 + lane];
    double a1[6], a0[6];
    q2_node6(q, ref, U1, a1);
    q2_node6(q, ref, U0, a0);
    sn[half][0][lane] = a1[0];                       // phi^{k+1}
    sn[half][1][lane] = 0.5 * (a1[0] + a0[0]);       // phi~
    sn[half][2][lane] = 0.5 * (a1[1] + a0[1]);       // mu~
    for (int d = 0; d < 3; ++d) {
      sn[half][3 + d][lane] = 0.5 * (a1[2 + d] + a0[2 + d]);  // v~
      sn[half][6 + d][lane] = a1[2 + d] - a0[2 + d];          // v^{k+1} - v^k
    }
    sn[half][9][lane] = 0.5 * (a1[5] + a0[5]);  // p~
    if (MODE == 1) {
      double dd[6];
      q2_node6(q, ref, dU, dd);
      for (int d = 0; d < 4; ++d) sn[half][10 + d][lane] = dd[2 + d];  // dv, dp
    }
  }
  __syncthreads();
  if (lane < 27) {
    const int g0 = lane % 3, g1 = (lane / 3) % 3, g2 = lane / 9;
    double bx[3], dx[3], by[3], dy[3], bz[3], dz[3];
    q2_basis_1d(q2_gauss_u(g0), bx, dx);
    q2_basis_1d(q2_gauss_u(g1), by, dy);
    q2_basis_1d(q2_gauss_u(g2), bz, dz);
    double ph1 = 0.0, gph1[3] = {0.0, 0.0, 0.0}, gpt[3] = {0.0, 0.0, 0.0}, Hpt[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double gmu[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0}, gv[3][3] = {{0.0}}, lv[3] = {0.0, 0.0, 0.0};
    double dvv[3] = {0.0, 0.0, 0.0}, pp = 0.0, gp[3] = {0.0, 0.0, 0.0};
    double ev[3] = {0.0, 0.0, 0.0}, egv[3][3] = {{0.0}}, elv[3] = {0.0, 0.0, 0.0}, ep = 0.0, egp[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 27; ++a) {
      const int i = a % 3, j = (a / 3) % 3, k = a / 9;
      const double N = bx[i] * by[j] * bz[k];
      const double G[3] = {dx[i] * by[j] * bz[k] * ih, bx[i] * dy[j] * bz[k] * ih, bx[i] * by[j] * dz[k] * ih};
      // Hessian xx, yy, zz, xy, xz, yz
      const double H[6] = {q2_basis_dd(i) * by[j] * bz[k] * ih2, bx[i] * q2_basis_dd(j) * bz[k] * ih2,
                           bx[i] * by[j] * q2_basis_dd(k) * ih2, dx[i] * dy[j] * bz[k] * ih2,
                           dx[i] * by[j] * dz[k] * ih2, bx[i] * dy[j] * dz[k] * ih2};
      const double lap = H[0] + H[1] + H[2];
      const double u1 = sn[half][0][a], ut = sn[half][1][a], um = sn[half][2][a], up = sn[half][9][a];
      ph1 += N * u1;
      pp += N * up;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        gph1[d] += G[d] * u1;
        gpt[d] += G[d] * ut;
        gmu[d] += G[d] * um;
        gp[d] += G[d] * up;
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) Hpt[c] += H[c] * ut;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double uv = sn[half][3 + d][a];
        v[d] += N * uv;
        lv[d] += lap * uv;
        dvv[d] += N * sn[half][6 + d][a];
#pragma unroll
        for (int c = 0; c < 3; ++c) gv[d][c] += G[c] * uv;
      }
      if (MODE == 1) {
        const double ud = sn[half][13][a];
        ep += N * ud;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          egp[d] += G[d] * ud;
          const double uv = sn[half][10 + d][a];
          ev[d] += N * uv;
          elv[d] += lap * uv;
#pragma unroll
          for (int c = 0; c < 3; ++c) egv[d][c] += G[c] * uv;
        }
      }
    }
    // the linearisation point (as ns_point, with the second-derivative terms completed)
    NSPoint<double> P;
    ns_material<double>(p, clamp1(ph1), P);
    const bool inside = ph1 <= 1.0 && ph1 >= -1.0;
    const double gg = inside ? p.gamma : 0.0;
    const double iPe = p.inv_Pe, iRe = p.inv_Re, iWe = p.inv_We, cw = p.CnWe;
    for (int d = 0; d < 3; ++d) {
      P.vt[d] = v[d];
      P.J[d] = p.kappa * gmu[d];
      P.gpht[d] = gpt[d];
      for (int c = 0; c < 3; ++c) P.G[d][c] = gv[d][c];
    }
    for (int d = 0; d < 3; ++d) P.adv[d] = P.rho * P.vt[d] + iPe * P.J[d] - iRe * gg * gph1[d];
    P.pt = pp;
    const double Hm[3][3] = {{Hpt[0], Hpt[3], Hpt[4]}, {Hpt[3], Hpt[1], Hpt[5]}, {Hpt[4], Hpt[5], Hpt[2]}};
    const double lpt = Hpt[0] + Hpt[1] + Hpt[2];
    for (int i = 0; i < 3; ++i) {
      P.tg[i] = P.rho * (dvv[i] * p.inv_dt - p.g[i] * p.inv_Fr);
      const double cap = cw * (gpt[0] * Hm[i][0] + gpt[1] * Hm[i][1] + gpt[2] * Hm[i][2] + gpt[i] * lpt);
      P.Rm[i] = P.tg[i] + P.adv[0] * P.G[i][0] + P.adv[1] * P.G[i][1] + P.adv[2] * P.G[i][2] + cap +
                iWe * gp[i] - P.eta * iRe * lv[i];
    }
    Lane<double> L;
    L.Gh = 4.0 * ih2;
    ns_stab<double>(p, L, P);
    double c[4], F[4][3];
    if (MODE == 0) {
      // the cG(1) residual integrand (ns_residual_point) before the contraction
      const double tm = P.tau_m, er = P.eta * iRe;
      double W[3];
      for (int j = 0; j < 3; ++j) W[j] = P.vt[j] + (P.J[j] * iPe - tm * P.Rm[j]) * P.inv_rho;
      const double dgl = iWe * (P.rho * P.tau_c * P.Rc - P.pt);
      for (int i = 0; i < 3; ++i) {
        double ci = P.tg[i];
        for (int j = 0; j < 3; ++j) ci += (P.rho * P.vt[j] + iPe * P.J[j] - tm * P.Rm[j]) * P.G[i][j];
        c[i] = ci;
        for (int j = 0; j < 3; ++j) F[i][j] = P.Rm[i] * tm * W[j] - cw * P.gpht[i] * P.gpht[j] + er * P.G[i][j];
        F[i][i] += dgl;
      }
      c[3] = P.Rc;
      for (int j = 0; j < 3; ++j) F[3][j] = tm * P.inv_rho * P.Rm[j];
    } else {
      VG<double> dvt[3], dpt;
      double ddv[3], dlap[3];
      for (int d = 0; d < 3; ++d) {
        dvt[d].v = 0.5 * ev[d];
        dvt[d].dx = 0.5 * egv[d][0];
        dvt[d].dy = 0.5 * egv[d][1];
        dvt[d].dz = 0.5 * egv[d][2];
        ddv[d] = ev[d];
        dlap[d] = 0.5 * elv[d];
      }
      dpt.v = 0.5 * ep;
      dpt.dx = 0.5 * egp[0];
      dpt.dy = 0.5 * egp[1];
      dpt.dz = 0.5 * egp[2];
      ns_jvp_coef<double, true>(p, P, dvt, ddv, dpt, c, F, dlap);
    }
    const double w = q2_gauss_w(g0) * q2_gauss_w(g1) * q2_gauss_w(g2) * h * h * h;
    for (int f = 0; f < 4; ++f) {
      sq[half][4 * f][lane] = w * c[f];
      for (int d = 0; d < 3; ++d) sq[half][4 * f + 1 + d][lane] = w * F[f][d];
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
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = 0; g < 27; ++g) {
      const int g0 = g % 3, g1 = (g / 3) % 3, g2 = g / 9;
      const double N = cx[g0] * cy[g1] * cz[g2], Nx = ex[g0] * cy[g1] * cz[g2], Ny = cx[g0] * ey[g1] * cz[g2],
                   Nz = cx[g0] * cy[g1] * ez[g2];
#pragma unroll
      for (int f = 0; f < 4; ++f)
        r[f] += N * sq[half][4 * f][g] + Nx * sq[half][4 * f + 1][g] + Ny * sq[half][4 * f + 2][g] +
                Nz * sq[half][4 * f + 3][g];
    }
    for (int f = 0; f < 4; ++f) part[(e * 27 + lane) * 4 + f] = r[f];
  }
}

// Node rows of a block from the element results (NF per slot): out[n][OFF +
// f] = sum of weight x result over the node's plan entries, the other block's
// fields set to 0.  NS: velocity rows of wall nodes read v^{k+1} - v^k (A =
// U1, B = U0) or, for the JVP, dv (A = dU, B = null); the pinned node's
// pressure row likewise.
template <int NF, int OFF>
__global__ __launch_bounds__(256) void k_q2_gather(int64_t n, const int64_t* __restrict__ goff,
                                                   const int32_t* __restrict__ gslot,
                                                   const double* __restrict__ gw,
                                                   const double* __restrict__ part, const uint8_t* __restrict__ bflags,
                                                   const double* __restrict__ A, const double* __restrict__ B,
                                                   double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) s[f] = 0.0;
    for (int64_t k = goff[i]; k < goff[i + 1]; ++k) {
      const int64_t t = gslot[k];
#pragma unroll
      for (int f = 0; f < NF; ++f) s[f] += gw[k] * part[t * NF + f];
    }
    double* o = out + i * 6;
    for (int f = 0; f < 6; ++f) o[f] = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) o[OFF + f] = s[f];
    if (NF == 4) {
      const uint8_t b = bflags[i];
      for (int f = 2; f < 6; ++f) {
        const bool wall = f < 5 ? (b & 1) : (b & 2);
        if (wall) o[f] = A[i * 6 + f] - (B ? B[i * 6 + f] : 0.0);
      }
    }
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
  uint8_t* d_bflags = nullptr;
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
  (void)hipFree(q->d_bflags);
}

int q2_launch(chns_q2* q, const chns_params* params, int block, const double* U1, const double* U0,
              const double* dU, double* out, void* stream, int mode) {
  if (!q) return fail(CHNS_EINVAL, "Q2 numbering is NULL");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != q->device) return fail(CHNS_EINVAL, "Q2 numbering was built on another device");
  dev::PhysView pv;
  int rc = phys_view(params, pv);
  if (rc) return rc;
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_NS) return fail(CHNS_EINVAL, "unknown block");
  if (!U1 || !U0 || !out || (mode == 1 && !dU)) return fail(CHNS_EINVAL, "pointers must not be NULL");
  auto misaligned = [](const void* ptr) { return ((uintptr_t)ptr & 15) != 0; };
  if (misaligned(U1) || misaligned(U0) || (mode == 1 && misaligned(dU)))
    return fail(CHNS_EINVAL, "state vectors must be 16-byte aligned");
  const int64_t E = (int64_t)q->m->h.leaf_key.size(), n = (int64_t)q->h.node_key.size();
  dev::Q2View v{q->d_elem, q->m->d_level, q->d_hoff, q->d_hids, q->d_hw, E};
  const dim3 g((unsigned)((E + 1) / 2)), b(64), gg(grid_stride(n)), bg(256);
  const double* nd = nullptr;
  if (block == CHNS_BLOCK_CH) {
    if (mode == 0)
      hipLaunchKernelGGL(dev::k_q2_ch<0>, g, b, 0, s, v, pv, U1, U0, nd, q->d_part);
    else
      hipLaunchKernelGGL(dev::k_q2_ch<1>, g, b, 0, s, v, pv, U1, U0, dU, q->d_part);
    hipLaunchKernelGGL((dev::k_q2_gather<2, 0>), gg, bg, 0, s, n, q->d_goff, q->d_gslot, q->d_gw, q->d_part,
                       q->d_bflags, nd, nd, out);
  } else {
    if (mode == 0) {
      hipLaunchKernelGGL(dev::k_q2_ns<0>, g, b, 0, s, v, pv, U1, U0, nd, q->d_part);
      hipLaunchKernelGGL((dev::k_q2_gather<4, 2>), gg, bg, 0, s, n, q->d_goff, q->d_gslot, q->d_gw, q->d_part,
                         q->d_bflags, U1, U0, out);
    } else {
      hipLaunchKernelGGL(dev::k_q2_ns<1>, g, b, 0, s, v, pv, U1, U0, dU, q->d_part);
      hipLaunchKernelGGL((dev::k_q2_gather<4, 2>), gg, bg, 0, s, n, q->d_goff, q->d_gslot, q->d_gw, q->d_part,
                         q->d_bflags, dU, nd, out);
    }
  }
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
        (rc = dalloc(&q->d_gw, H.g_w.size(), B)) || (rc = dalloc(&q->d_part, E * 27 * 4, B)) ||
        (rc = dalloc(&q->d_bflags, H.bflags.size(), B))) {
      free_q2_locked(q);
      delete q;
      return rc;
    }
  }
  if ((rc = h2d(q->d_elem, H.elem, s)) || (rc = h2d(q->d_hoff, H.hang_off, s)) ||
      (rc = h2d(q->d_hids, H.hang_ids, s)) || (rc = h2d(q->d_hw, H.hang_w, s)) ||
      (rc = h2d(q->d_goff, H.g_off, s)) || (rc = h2d(q->d_gslot, H.g_slot, s)) || (rc = h2d(q->d_gw, H.g_w, s)) ||
      (rc = h2d(q->d_bflags, H.bflags, s))) {
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

int chns_q2_residual(chns_q2* q, const chns_params* params, int block, const double* U_new, const double* U_old,
                     double* R, void* stream) {
  return q2_launch(q, params, block, U_new, U_old, nullptr, R, stream, 0);
}

int chns_q2_jvp(chns_q2* q, const chns_params* params, int block, const double* U_new, const double* U_old,
                const double* dU, double* JdU, void* stream) {
  return q2_launch(q, params, block, U_new, U_old, dU, JdU, stream, 1);
}

int chns_q2_host_arrays(const chns_mesh* m, int64_t* sizes, int32_t* elem27, double* node_xyz, double* hang_xyz,
                        int32_t* hang_off, int32_t* hang_ids, double* hang_w, uint8_t* bflags) {
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
  if (bflags) std::copy(H.bflags.begin(), H.bflags.end(), bflags);
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
