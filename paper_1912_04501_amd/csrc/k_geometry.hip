// Geometry (Sec. 2, Sec. 6 trapezoid rule), RHS (Sec. 3) and close-pair lists (Sec. 6.3).
#include "spm_internal.h"

namespace spm {

// One thread per node: x(t) = c + R(theta) x_body(t), t = 2 pi k / N_p (x_body: ellipse
// (a cos t, b sin t) or star r(t) (cos t, sin t)). w = (2 pi / N_p)|x'|, tau = x'/|x'|,
// n = (tau_2, -tau_1), kappa = (x' y'' - y' x'') / |x'|^3 (= a b / |x'|^3 for an ellipse).
// With the dilated near set every node is also wrapped into the cell on its own: lattice
// coordinates (alpha, beta) of x - c_U reduced to [-1/2, 1/2) as floor(. + 1/2) (Sec. 4.2, the
// sources of G_near are points of the cell); the FP32 shadows then hold the wrapped node.
__global__ void k_geometry(int64_t N, const int32_t* __restrict__ pid, const int32_t* __restrict__ poff,
                           const int32_t* __restrict__ pn, const double* __restrict__ pcx,
                           const double* __restrict__ pcy, const double* __restrict__ pth,
                           const int32_t* __restrict__ pkind, const double* __restrict__ pprm, double cUx,
                           double cUy, Geo g) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int p = pid[i];
  const int k = (int)(i - poff[p]);
  const int n = pn[p];
  const double t = 2.0 * kPi * (double)k / (double)n;
  double px, py, dx, dy, ddx, ddy;
  shape_point(pkind[p], pprm + 4 * (int64_t)p, t, px, py, dx, dy, ddx, ddy);
  double sth, cth;
  sincos(pth[p], &sth, &cth);
  const double x = pcx[p] + (cth * px - sth * py);
  const double y = pcy[p] + (sth * px + cth * py);
  const double xpx = cth * dx - sth * dy;
  const double xpy = sth * dx + cth * dy;
  const double sp = sqrt(xpx * xpx + xpy * xpy);
  const double tx = xpx / sp, ty = xpy / sp;
  g.x[i] = x;
  g.y[i] = y;
  g.xpx[i] = xpx;
  g.xpy[i] = xpy;
  g.tx[i] = tx;
  g.ty[i] = ty;
  g.nx[i] = ty;
  g.ny[i] = -tx;
  g.w[i] = 2.0 * kPi * sp / (double)n;
  g.kap[i] = (dx * ddy - dy * ddx) / (sp * sp * sp);
  // spectral derivative weight at index distance k (N_p even): (1/2) (-1)^k cot(k pi / N_p), 0 at k = 0
  g.dcot[i] = k > 0 ? ((k & 1) ? -0.5 : 0.5) * (cos(kPi * (double)k / (double)n) / sin(kPi * (double)k / (double)n))
                    : 0.0;
  g.nxf[i] = (float)ty;
  g.nyf[i] = (float)(-tx);
  if (g.dilated) {
    const double skew = g.cskew[g.ncell[i]];
    const double be = y - cUy, al = (x - cUx) - skew * be;
    const double ka = -floor(al + 0.5), kb = -floor(be + 0.5);
    const double xw = x + ka + kb * skew, yw = y + kb;
    g.xw[i] = xw;
    g.yw[i] = yw;
    g.nwrap[i] = node_wrap_pack((int)ka, (int)kb, (al + ka) < 0.0 ? 1 : -1, (be + kb) < 0.0 ? 1 : -1);
    g.xf[i] = (float)xw;
    g.yf[i] = (float)yw;
  } else {
    g.xf[i] = (float)x;
    g.yf[i] = (float)y;
  }
}

// Perimeter of every particle (sum of its trapezoid weights) and its area by the
// boundary quadrature (1/2) sum ((x - c) y' - (y - c) x') (2 pi / N_p), one block per particle.
__global__ void k_perimeter(const int32_t* __restrict__ poff, Geo g, double* per, double* area) {
  __shared__ double sc[16];
  const int p = blockIdx.x;
  const double cx = g.pcx[p], cy = g.pcy[p];
  double s = 0.0, a = 0.0;
  for (int k = poff[p] + threadIdx.x; k < poff[p + 1]; k += blockDim.x) {
    s += g.w[k];
    a += (g.x[k] - cx) * g.xpy[k] - (g.y[k] - cy) * g.xpx[k];
  }
  s = block_sum(s, sc);
  a = block_sum(a, sc);
  if (threadIdx.x == 0) {
    per[p] = s;
    area[p] = a * kPi / (double)(poff[p + 1] - poff[p]);
  }
}

void launch_geometry(spm_handle* h) {
  Geo& g = h->geo;
  const int bs = 256;
  k_geometry<<<(unsigned)((g.N + bs - 1) / bs), bs, 0, h->stream>>>(g.N, g.pid, g.poff, g.pn, g.pcx, g.pcy,
                                                                    g.pth, g.pkind, g.pprm, h->cU[0], h->cU[1], g);
  SPM_HIP_CHECK(hipGetLastError());
  k_perimeter<<<g.No, 256, 0, h->stream>>>(g.poff, g, g.pper, g.parea);
  SPM_HIP_CHECK(hipGetLastError());
}

// b = -mu gamma (n_2, n_1): minus the traction of the background shear u0 = (gamma x_2, 0), p0 = 0.
__global__ void k_rhs(int64_t N, const double* __restrict__ nx, const double* __restrict__ ny, double c,
                      double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  out[i] = c * ny[i];
  out[N + i] = c * nx[i];
}

void launch_rhs(spm_handle* h, double* out) {
  const int bs = 256;
  const int64_t N = h->geo.N;
  k_rhs<<<(unsigned)((N + bs - 1) / bs), bs, 0, h->stream>>>(N, h->geo.nx, h->geo.ny,
                                                             -h->cfg.mu * h->cfg.gamma, out);
  SPM_HIP_CHECK(hipGetLastError());
}

// ----------------------------------------------------------------------------
// Close pairs: target x_i on particle p, source image Gamma_q + s with (q, s) != (p, 0),
// close when min_k |x_i - (y_k + s)| < factor * h_q, h_q = perimeter_q / N_q.
// Pass 1 counts per target (and records the smallest node distance to any other
// particle image and whether the node lies inside one: the overlap check);
// a scan makes row pointers; pass 2 fills (q, s) in ascending (q, s) order.
// ----------------------------------------------------------------------------
template <bool FILL>
__global__ void k_close_pass(int64_t N, Geo g, double factor, const int32_t* __restrict__ row,
                             int32_t* __restrict__ count, int32_t* __restrict__ outq, int32_t* __restrict__ outs,
                             double* __restrict__ dmin, int32_t* __restrict__ inside) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double xi = g.x[i], yi = g.y[i];
  const int pi = g.pid[i];
  const int c = g.ncell[i];
  const double skew = g.cskew[c];
  int cnt = 0;
  int64_t pos = FILL ? row[i] : 0;
  double best = 1e300;
  int ins = 0;
  for (int q = g.cpoff[c]; q < g.cpoff[c + 1]; ++q) {
    const double lim = factor * g.pper[q] / (double)g.pn[q];
    const double reach = g.pa[q] + (lim > 0.0 ? lim : 0.0);
    for (int s = 0; s < kShifts; ++s) {
      if (q == pi && s == kZeroShift) continue;
      const double sx = shift_x(s, skew), sy = shift_y(s);
      const double cx = g.pcx[q] + sx, cy = g.pcy[q] + sy;
      const double ddx = xi - cx, ddy = yi - cy;
      if (ddx * ddx + ddy * ddy >= reach * reach) continue;
      // inside test against the curve (body frame)
      double sth, cth;
      sincos(g.pth[q], &sth, &cth);
      const double bu = cth * ddx + sth * ddy, bv = -sth * ddx + cth * ddy;
      const double* pp = g.pprm + 4 * (int64_t)q;
      if (g.pkind[q] == SPM_SHAPE_ELLIPSE) {
        const double u = bu / pp[0], v = bv / pp[1];
        if (u * u + v * v < 1.0) ins = 1;
      } else {   // star-shaped about the reference point: inside when closer than r(angle)
        const double r = pp[0] * (1.0 + pp[1] * cos(pp[2] * atan2(bv, bu) + pp[3]));
        if (bu * bu + bv * bv < r * r) ins = 1;
      }
      double m2 = 1e300;
      for (int k = g.poff[q]; k < g.poff[q + 1]; ++k) {
        const double rx = xi - (g.x[k] + sx);
        const double ry = yi - (g.y[k] + sy);
        const double d2 = rx * rx + ry * ry;
        m2 = d2 < m2 ? d2 : m2;
      }
      best = m2 < best ? m2 : best;
      if (lim > 0.0 && m2 < lim * lim) {
        if (FILL) {
          outq[pos] = q;
          outs[pos] = s;
          ++pos;
        }
        ++cnt;
      }
    }
  }
  if (!FILL) {
    count[i] = cnt;
    dmin[i] = sqrt(best);
    inside[i] = ins;
  }
}

// Exclusive scan of count[N] into row[N+1] by one block; also collects the
// targets with a nonempty row. scal[0] = total pairs, scal[1] = number of targets.
__global__ void k_scan(int64_t N, const int32_t* __restrict__ count, int32_t* __restrict__ row,
                       int32_t* __restrict__ tlist, int32_t* __restrict__ totals) {
  __shared__ int32_t part[1024];
  __shared__ int32_t tpart[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const int64_t per = (N + nt - 1) / nt;
  const int64_t lo = t * per, hi = (lo + per < N) ? lo + per : N;
  int32_t s = 0, c = 0;
  for (int64_t i = lo; i < hi; ++i) {
    s += count[i];
    c += count[i] > 0;
  }
  part[t] = s;
  tpart[t] = c;
  __syncthreads();
  if (t == 0) {
    int32_t acc = 0, acc2 = 0;
    for (int k = 0; k < nt; ++k) {
      const int32_t v = part[k], v2 = tpart[k];
      part[k] = acc;
      tpart[k] = acc2;
      acc += v;
      acc2 += v2;
    }
    totals[0] = acc;
    totals[1] = acc2;
    row[N] = acc;
  }
  __syncthreads();
  int32_t acc = part[t], acc2 = tpart[t];
  for (int64_t i = lo; i < hi; ++i) {
    row[i] = acc;
    acc += count[i];
    if (count[i] > 0) tlist[acc2++] = (int32_t)i;
  }
}

void launch_close_count(spm_handle* h) {
  const int bs = 128;
  const int64_t N = h->geo.N;
  k_close_pass<false><<<(unsigned)((N + bs - 1) / bs), bs, 0, h->stream>>>(
      N, h->geo, h->cfg.close_factor, nullptr, h->cl.count, nullptr, nullptr, h->cl.dmin, h->cl.inside);
  SPM_HIP_CHECK(hipGetLastError());
}

void launch_close_scan(spm_handle* h, int32_t* total_host, int32_t* ntargets_host) {
  int32_t* tot = reinterpret_cast<int32_t*>(h->wk.scal);
  k_scan<<<1, 1024, 0, h->stream>>>(h->geo.N, h->cl.count, h->cl.row, h->cl.tlist, tot);
  SPM_HIP_CHECK(hipGetLastError());
  int32_t hv[2];
  SPM_HIP_CHECK(hipMemcpyAsync(hv, tot, sizeof(hv), hipMemcpyDeviceToHost, h->stream));
  SPM_HIP_CHECK(hipStreamSynchronize(h->stream));
  *total_host = hv[0];
  *ntargets_host = hv[1];
}

void launch_close_fill(spm_handle* h) {
  const int bs = 128;
  const int64_t N = h->geo.N;
  k_close_pass<true><<<(unsigned)((N + bs - 1) / bs), bs, 0, h->stream>>>(
      N, h->geo, h->cfg.close_factor, h->cl.row, nullptr, h->cl.q, h->cl.s, nullptr, nullptr);
  SPM_HIP_CHECK(hipGetLastError());
}

// flags of the particles that are the source of at least one close pair
__global__ void k_close_sources(int32_t No, int64_t npairs, const int32_t* __restrict__ q, int32_t* __restrict__ flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < No) flag[i] = 0;
}
__global__ void k_close_sources_mark(int64_t npairs, const int32_t* __restrict__ q, int32_t* __restrict__ flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < npairs) flag[q[i]] = 1;   // every writer stores the same value
}

void launch_close_sources(spm_handle* h) {
  const int32_t No = h->geo.No;
  k_close_sources<<<(unsigned)((No + 255) / 256), 256, 0, h->stream>>>(No, h->cl.npairs, h->cl.q, h->cl.qsrc);
  SPM_HIP_CHECK(hipGetLastError());
  if (h->cl.npairs > 0) {
    k_close_sources_mark<<<(unsigned)((h->cl.npairs + 255) / 256), 256, 0, h->stream>>>(h->cl.npairs, h->cl.q,
                                                                                       h->cl.qsrc);
    SPM_HIP_CHECK(hipGetLastError());
  }
}

// min over nodes of dmin, max of inside, one block
__global__ void k_gap_reduce(int64_t N, const double* __restrict__ dmin, const int32_t* __restrict__ inside,
                             double* out) {
  __shared__ double sm[1024];
  __shared__ int si[1024];
  double b = 1e300;
  int in = 0;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    b = dmin[i] < b ? dmin[i] : b;
    in |= inside[i];
  }
  sm[threadIdx.x] = b;
  si[threadIdx.x] = in;
  __syncthreads();
  if (threadIdx.x == 0) {
    double bb = 1e300;
    int ii = 0;
    for (int k = 0; k < (int)blockDim.x; ++k) {
      bb = sm[k] < bb ? sm[k] : bb;
      ii |= si[k];
    }
    out[0] = bb;
    out[1] = (double)ii;
  }
}

void launch_gap(spm_handle* h, double* gap_host, int32_t* overlap_host) {
  double* o = h->wk.scal + 4;
  k_gap_reduce<<<1, 1024, 0, h->stream>>>(h->geo.N, h->cl.dmin, h->cl.inside, o);
  SPM_HIP_CHECK(hipGetLastError());
  double hv[2];
  SPM_HIP_CHECK(hipMemcpyAsync(hv, o, sizeof(hv), hipMemcpyDeviceToHost, h->stream));
  SPM_HIP_CHECK(hipStreamSynchronize(h->stream));
  *gap_host = hv[0];
  *overlap_host = hv[1] != 0.0;
}

}  // namespace spm
