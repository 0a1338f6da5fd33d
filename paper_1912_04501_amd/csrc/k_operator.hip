// Operator assembly and readouts.
//
// prep:     f = w sigma (FP64 and FP32 copies) and per-particle moments
//           F_q = sum w sigma, tau_q = sum w (x - c)^perp . sigma, stresslet_q (Sec. 5 operator L).
// assemble: y = sigma/2 + T + alpha n + L sigma,  alpha = -(T(x0) . n0)   (Sec. 5 eq. BIEPerturbed;
//           Sec. 6.2 pressure pin with x0 the first node of the first particle),
//           L_q sigma (x) = F_q + (x - c_q)^perp tau_q.
// readout:  v_q = u0(c_q) + u_near(c_q) + u_corr(c_q) - u_corr(c_U) (u_near by the FMM's tree when the
//           FMM near sum is on), then the constant that makes
//           the area-weighted mean of v_q - u0(c_q) over the cell zero is removed;
//           omega_q = (vort_near(c_q) + vort_corr(c_q))/2 - gamma/2   (Sec. 3 eq. RigidBodyMotion).
//           mu_eff = mu - sum_q stresslet_q / (2 gamma |U|)           (Sec. 3 eq. mueff via the
//           cell force balance: the traction on a particle is -sigma).
// contour:  mu_eff by contour deformation (Sec. 7, efficient evaluation of the effective
//           viscosity) for the 3x3 near set: the force through a curve C joining D's end points
//           around the particles is, by translation invariance of G^t and Gauss' law on the
//           strips between shifted copies of three cells of C,
//             sum_q [2 J_q(-1) + J_q(2) - W_q(p0 + 2e1 - e2) + W_q(p0 - e1 - e2)
//                                       + W_q(p0 + 2e1 + e2) - W_q(p0 - e1 + e2)] + int_D T_corr,
//           J_q(a): the single-layer traction of the unshifted curve q on the straight line from
//           p0 - e1 + a e2 to p0 + 2e1 + a e2 (normal (0, 1)); W_q(P): on the segment from P to
//           P + e2 (normal e2 turned clockwise); p0 = c_U - e1/2 - e2/2. Every such target is
//           about half a cell or more from its sources, so m Gauss-Legendre nodes per cell edge
//           and the trapezoid rule on the curves are accurate wherever the particles sit.
#include "spm_internal.h"

namespace spm {

__global__ __launch_bounds__(256) void k_prep(int64_t N, Geo g, const double* __restrict__ sigma,
                                              double* __restrict__ f1, double* __restrict__ f2,
                                              float* __restrict__ f1f, float* __restrict__ f2f,
                                              double* __restrict__ pF) {
  __shared__ double sc[32];
  const int q = blockIdx.x;
  const double cx = g.pcx[q], cy = g.pcy[q];
  dd F1 = {0, 0}, F2 = {0, 0};   // the net force is small against its terms and feeds the proxy solve
  double tq = 0, st = 0;
  for (int64_t i = g.poff[q] + threadIdx.x; i < g.poff[q + 1]; i += blockDim.x) {
    const double w = g.w[i], s1 = sigma[i], s2 = sigma[N + i];
    const double a = w * s1, b = w * s2;
    f1[i] = a;
    f2[i] = b;
    f1f[i] = (float)a;
    f2f[i] = (float)b;
    const double rx = g.x[i] - cx, ry = g.y[i] - cy;
    F1 = dd_add_d(F1, a);
    F2 = dd_add_d(F2, b);
    tq += -ry * a + rx * b;
    st += rx * b + ry * a;
  }
  F1 = dd_block_sum(F1, sc);
  F2 = dd_block_sum(F2, sc);
  tq = block_sum(tq, sc);
  st = block_sum(st, sc);
  if (threadIdx.x == 0) {
    pF[4 * q + 0] = F1.hi + F1.lo;
    pF[4 * q + 1] = F2.hi + F2.lo;
    pF[4 * q + 2] = tq;
    pF[4 * q + 3] = st;
  }
}

void launch_prep(spm_handle* h, const double* sigma) {
  k_prep<<<h->geo.No, 256, 0, h->stream>>>(h->geo.N, h->geo, sigma, h->wk.f1, h->wk.f2, h->wk.f1f, h->wk.f2f,
                                           h->wk.pF);
  SPM_HIP_CHECK(hipGetLastError());
}

__global__ void k_assemble(int64_t N, Geo g, const double* __restrict__ sigma, const double* __restrict__ T,
                           const double* __restrict__ pF, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t i0 = g.cnoff[g.ncell[i]];  // pin node: the first node of the cell
  const double alpha = -(T[i0] * g.nx[i0] + T[N + i0] * g.ny[i0]);
  const int q = g.pid[i];
  const double rx = g.x[i] - g.pcx[q], ry = g.y[i] - g.pcy[q];
  const double F1 = pF[4 * q + 0], F2 = pF[4 * q + 1], tq = pF[4 * q + 2];
  out[i] = 0.5 * sigma[i] + T[i] + alpha * g.nx[i] + F1 - ry * tq;
  out[N + i] = 0.5 * sigma[N + i] + T[N + i] + alpha * g.ny[i] + F2 + rx * tq;
}

void launch_assemble(spm_handle* h, const double* sigma, double* out) {
  const int64_t N = h->geo.N;
  k_assemble<<<(unsigned)((N + 255) / 256), 256, 0, h->stream>>>(N, h->geo, sigma, h->wk.T, h->wk.pF, out);
  SPM_HIP_CHECK(hipGetLastError());
}

// Velocity and vorticity at the particle centres: one block per particle, the nodes of
// its cell x 9 images (or, when near3 is given, the near-image part computed by the FMM).
__global__ __launch_bounds__(256) void k_velocities(Geo g, const double* __restrict__ f1, const double* __restrict__ f2,
                                                    int M, const double* __restrict__ px, const double* __restrict__ py,
                                                    const double* __restrict__ xi_all, double cUx, double cUy, double mu,
                                                    double gamma, const double* __restrict__ near3,
                                                    double* __restrict__ vel, double* __restrict__ omega) {
  __shared__ double sc[16];
  const int q = blockIdx.x;
  const int cell = g.pcell[q];
  const double skew = g.cskew[cell];
  const double cx = g.pcx[q], cy = g.pcy[q];
  const double k4 = 1.0 / (4.0 * kPi * mu), k2 = -1.0 / (2.0 * kPi * mu);
  double u1 = 0, u2 = 0, vo = 0;
  const int64_t j_end = near3 ? g.cnoff[cell] : g.cnoff[cell + 1];
  for (int64_t j = g.cnoff[cell] + threadIdx.x; j < j_end; j += blockDim.x) {
    // 3x3 set: the nodes with the nine shifts; dilated set: the wrapped nodes with their four
    // images {0, ms} x {0, ns} inside U~
    const double yx = g.dilated ? g.xw[j] : g.x[j], yy = g.dilated ? g.yw[j] : g.y[j], a = f1[j], b = f2[j];
    const int32_t w = g.dilated ? g.nwrap[j] : 0;
    for (int s = 0; s < kShifts; ++s) {
      int sm = s / 3 - 1, sn = s % 3 - 1;
      if (g.dilated) {
        if (s >= 4) break;
        sm = (s & 1) ? node_wrap_ms(w) : 0;
        sn = (s & 2) ? node_wrap_ns(w) : 0;
      }
      const double rx = cx - (yx + shift_xmn(sm, sn, skew)), ry = cy - (yy + (double)sn);
      const double r2 = rx * rx + ry * ry;
      const double ir2 = rcp64(r2);
      const double lg = -0.5 * log(r2);
      const double rf = (rx * a + ry * b) * ir2;
      u1 += k4 * (lg * a + rx * rf);
      u2 += k4 * (lg * b + ry * rf);
      vo += k2 * (rx * b - ry * a) * ir2;
    }
  }
  u1 = block_sum(u1, sc);
  u2 = block_sum(u2, sc);
  vo = block_sum(vo, sc);
  if (near3) {
    u1 = near3[3 * q];
    u2 = near3[3 * q + 1];
    vo = near3[3 * q + 2];
  }
  if (threadIdx.x == 0) {
    const double* xi = xi_all + (int64_t)cell * 2 * M;
    px += (int64_t)cell * M;
    py += (int64_t)cell * M;
    double c1 = 0, c2 = 0, z1 = 0, z2 = 0, cv = 0;
    for (int p = 0; p < M; ++p) {
      const double a = xi[p], b = xi[M + p];
      {
        const double rx = cx - px[p], ry = cy - py[p];
        const double r2 = rx * rx + ry * ry;
        const double lg = -0.5 * log(r2);
        const double rf = (rx * a + ry * b) / r2;
        c1 += k4 * (lg * a + rx * rf);
        c2 += k4 * (lg * b + ry * rf);
        cv += k2 * (rx * b - ry * a) / r2;
      }
      {
        const double rx = cUx - px[p], ry = cUy - py[p];
        const double r2 = rx * rx + ry * ry;
        const double lg = -0.5 * log(r2);
        const double rf = (rx * a + ry * b) / r2;
        z1 += k4 * (lg * a + rx * rf);
        z2 += k4 * (lg * b + ry * rf);
      }
    }
    if (vel) {
      vel[2 * q] = gamma * cy + u1 + (c1 - z1);
      vel[2 * q + 1] = u2 + (c2 - z2);
    }
    if (omega) omega[q] = 0.5 * (vo + cv) - 0.5 * gamma;
  }
}

// Velocity gauge, one block per cell: subtract the area-weighted mean disturbance
// sum_q |Omega_q| (v_q - u0(c_q)) / sum_q |Omega_q| from every velocity of the cell, so the
// reported velocities do not depend on where the particles sit relative to the cell
// centre (a uniform translation of all particles is a symmetry of the periodic problem).
__global__ __launch_bounds__(256) void k_velocity_gauge(const int32_t* __restrict__ cpoff,
                                                        const double* __restrict__ pcy,
                                                        const double* __restrict__ parea, double gamma,
                                                        double* __restrict__ vel, double* __restrict__ gauge) {
  __shared__ double sc[16];
  const int c = blockIdx.x;
  double a = 0, m1 = 0, m2 = 0;
  for (int q = cpoff[c] + threadIdx.x; q < cpoff[c + 1]; q += blockDim.x) {
    a += parea[q];
    m1 += parea[q] * (vel[2 * q] - gamma * pcy[q]);
    m2 += parea[q] * vel[2 * q + 1];
  }
  a = block_sum(a, sc);
  m1 = block_sum(m1, sc) / a;
  m2 = block_sum(m2, sc) / a;
  for (int q = cpoff[c] + threadIdx.x; q < cpoff[c + 1]; q += blockDim.x) {
    vel[2 * q] -= m1;
    vel[2 * q + 1] -= m2;
  }
  if (threadIdx.x == 0) {
    gauge[2 * c] = m1;
    gauge[2 * c + 1] = m2;
  }
}

__global__ void k_add_cell_velocity(int No, const int32_t* __restrict__ pcell, const double* __restrict__ du,
                                    double* __restrict__ vel) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < No) vel[2 * i] += du[pcell[i]];
}

void launch_add_cell_velocity(spm_handle* h, const double* du, double* vel) {
  const int n = h->geo.No;
  k_add_cell_velocity<<<(n + 255) / 256, 256, 0, h->stream>>>(n, h->geo.pcell, du, vel);
  SPM_HIP_CHECK(hipGetLastError());
}

void launch_velocities(spm_handle* h, double* vel, double* omega) {
  const double* near3 = nullptr;
  if (h->fmm.on) {                      // near-image part by the FMM's tree (w sigma is staged)
    launch_fmm_velocities(h, h->fmm.vnear);
    near3 = h->fmm.vnear;
  }
  k_velocities<<<h->geo.No, 256, 0, h->stream>>>(h->geo, h->wk.f1, h->wk.f2, h->per.M, h->per.px, h->per.py,
                                                 h->wk.xi, h->cU[0], h->cU[1], h->cfg.mu, h->cfg.gamma, near3, vel,
                                                 omega);
  SPM_HIP_CHECK(hipGetLastError());
  if (vel) {
    k_velocity_gauge<<<h->geo.C, 256, 0, h->stream>>>(h->geo.cpoff, h->geo.pcy, h->geo.parea, h->cfg.gamma, vel,
                                                      h->wk.gauge);
    SPM_HIP_CHECK(hipGetLastError());
  }
}

// mu_eff of every cell (|U| = |det(e1, e2)| = 1 for e1 = (1, 0), e2 = (s, 1)).
__global__ void k_mu_eff(const int32_t* __restrict__ cpoff, const double* __restrict__ pF, double mu, double gamma,
                         double* __restrict__ out) {
  __shared__ double sc[16];
  const int cell = blockIdx.x;
  double s = 0;
  for (int q = cpoff[cell] + threadIdx.x; q < cpoff[cell + 1]; q += blockDim.x) s += pF[4 * q + 3];
  s = block_sum(s, sc);
  if (threadIdx.x == 0) out[cell] = mu - s / (2.0 * gamma * 1.0);
}

void launch_mu_eff(spm_handle* h, double* mu_eff) {
  k_mu_eff<<<h->geo.C, 256, 0, h->stream>>>(h->geo.cpoff, h->wk.pF, h->cfg.mu, h->cfg.gamma, mu_eff);
  SPM_HIP_CHECK(hipGetLastError());
}

// One block per quadrature point (blockIdx.x < 11 m) of cell blockIdx.y: segments 0-2 carry
// J(-1) (weight 2), 3-5 J(2), 6-9 the four sides, 10 the correction on D. Writes the weighted
// shear component of the traction at the point.
__global__ __launch_bounds__(256) void k_contour_points(Geo g, const double* __restrict__ f1,
                                                        const double* __restrict__ f2, int M,
                                                        const double* __restrict__ px,
                                                        const double* __restrict__ py,
                                                        const double* __restrict__ xi_all, double cUx, double cUy,
                                                        int m, const double* __restrict__ gl,
                                                        double* __restrict__ part) {
  __shared__ double sc[16];
  const int cell = blockIdx.y;
  const int seg = blockIdx.x / m, k = blockIdx.x % m;
  const double skew = g.cskew[cell];
  const double l2 = sqrt(1.0 + skew * skew);
  const double t = 0.5 * gl[k], w = 0.5 * gl[m + k];
  const double p0x = cUx - 0.5 - 0.5 * skew, p0y = cUy - 0.5;
  double xq, yq, nxq, nyq, wq;
  if (seg < 6) {                               // lines D - e2 (twice) and D + 2 e2, three cells each
    const double a = seg < 3 ? -1.0 : 2.0;
    const double s = (double)(seg % 3 - 1) + 0.5 + t;
    xq = p0x + a * skew + s;
    yq = p0y + a;
    nxq = 0.0;
    nyq = 1.0;
    wq = (seg < 3 ? 2.0 : 1.0) * w;
  } else if (seg < 10) {                       // sides from corner P to P + e2
    const double cm[4] = {2.0, -1.0, 2.0, -1.0}, cn[4] = {-1.0, -1.0, 1.0, 1.0}, sg[4] = {-1.0, 1.0, 1.0, -1.0};
    const int i = seg - 6;
    const double s = 0.5 + t;
    xq = p0x + cm[i] + (cn[i] + s) * skew;
    yq = p0y + cn[i] + s;
    nxq = 1.0 / l2;
    nyq = -skew / l2;
    wq = sg[i] * w * l2;
  } else {                                     // D, correction field
    xq = p0x + 0.5 + t;
    yq = p0y;
    nxq = 0.0;
    nyq = 1.0;
    wq = w;
  }
  double T1 = 0.0;
  if (seg < 10) {
    for (int64_t j = g.cnoff[cell] + threadIdx.x; j < g.cnoff[cell + 1]; j += blockDim.x) {
      const double rx = xq - g.x[j], ry = yq - g.y[j];
      const double r2 = rx * rx + ry * ry;
      const double rn = rx * nxq + ry * nyq, rf = rx * f1[j] + ry * f2[j];
      T1 += rx * rn * rf / (r2 * r2);
    }
  } else {
    const double* xi = xi_all + (int64_t)cell * 2 * M;
    px += (int64_t)cell * M;
    py += (int64_t)cell * M;
    for (int p = threadIdx.x; p < M; p += blockDim.x) {
      const double rx = xq - px[p], ry = yq - py[p];
      const double r2 = rx * rx + ry * ry;
      const double rn = rx * nxq + ry * nyq, rf = rx * xi[p] + ry * xi[M + p];
      T1 += rx * rn * rf / (r2 * r2);
    }
  }
  T1 = block_sum(T1, sc);
  if (threadIdx.x == 0) part[(int64_t)cell * 11 * m + blockIdx.x] = -wq * T1 / kPi;
}

// mu_eff = mu + (force through C) . e1 / (gamma |e1|), |e1| = 1; fixed summation order.
__global__ void k_contour_sum(int m, const double* __restrict__ part, double mu, double gamma,
                              double* __restrict__ out) {
  __shared__ double sc[16];
  const int cell = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < 11 * m; i += blockDim.x) s += part[(int64_t)cell * 11 * m + i];
  s = block_sum(s, sc);
  if (threadIdx.x == 0) out[cell] = mu + s / gamma;
}

void launch_mu_eff_contour(spm_handle* h, int m, double* mu_eff) {
  const Geo& g = h->geo;
  k_contour_points<<<dim3(11 * m, g.C), 256, 0, h->stream>>>(g, h->wk.f1, h->wk.f2, h->per.M, h->per.px,
                                                             h->per.py, h->wk.xi, h->cU[0], h->cU[1], m,
                                                             h->wk.contour_gl, h->wk.contour);
  SPM_HIP_CHECK(hipGetLastError());
  k_contour_sum<<<g.C, 256, 0, h->stream>>>(m, h->wk.contour, h->cfg.mu, h->cfg.gamma, mu_eff);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace spm
