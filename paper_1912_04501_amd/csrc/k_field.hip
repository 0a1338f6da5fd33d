// Flow velocity and pressure at points of the fluid (Sec. 3; Sec. 5 eqs. BIEurep, BIEprep;
// Sec. 7 lists u(x), p(x) among the quasi-static solver's outputs).
//
// A target x is evaluated at its periodic copy x_w in the cell U:
//   u(x) = u0(x) + sum_q sum_{s in S9} S_{Gamma_q + s}[sigma](x_w) + u_corr(x_w) - u_corr(c_U) - V,
//   p(x) =         sum_q sum_{s in S9} P_{Gamma_q + s}[sigma](x_w) + p_corr(x_w),
// S the Stokeslet single layer, P its pressure, V the readout's velocity gauge; p up to the
// constant of this representation. Inside a particle image the result is its rigid motion
// (and p = NaN).
//
// Close to a curve (minimum node distance below close_factor * h_q) the plain trapezoid
// terms of that image are replaced by the Laplace decomposition of Sec. 6.3,
//   S[sigma](x) = (1/mu) [ S_L[sigma]/2 + grad S_L[sigma~]/2 - X_1 grad S_L[sigma_1]/2 - X_2 grad S_L[sigma_2]/2 ],
//   p(x) = -(d1 S_L[sigma_1] + d2 S_L[sigma_2]),     X = x - c_q, sigma~ = (y - c_q).sigma,
// with S_L[f] = (1/2 pi) int log(1/|x - y|) f ds. The gradients come from the exterior
// barycentric Cauchy rule already used by the close traction (v of phi = f conj(tau),
// grad S_L = (-Im v, -Re v)). The values come from the complex log potential
//   int log(z - y) f ds = Q log(z - c) + H(z),   Q = int f ds,
// where H is analytic outside the curve and vanishes at infinity, so the same exterior rule
// evaluates it from its boundary values H+. Those follow from H' = -2 pi i v - Q/(z - c):
// H+ is the spectral antiderivative in t of y'(t) H'+(y(t)), plus the constant that makes
// the interior Cauchy integral of H+ vanish (H has no part analytic inside). Then
// S_L[f](z) = -(1/2 pi) (Q log|z - c| + Re H(z)).
#include "spm_internal.h"

namespace spm {
namespace {

struct zc {
  double re, im;
};
__device__ __forceinline__ zc zmul(zc a, zc b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ zc zinv(zc a) {
  const double d = rcp64(a.re * a.re + a.im * a.im);
  return {a.re * d, -a.im * d};
}

}  // namespace

// iw[o_q + l] = (2/n) sum_{m=1}^{n/2-1} sin(2 pi m l / n) / m: the antiderivative of the
// trigonometric interpolant (zero mean, Nyquist mode dropped) is sum_k iw[(j - k) mod n] g_k.
__global__ __launch_bounds__(256) void k_int_weights(Geo g, double* __restrict__ iw) {
  const int q = blockIdx.x;
  const int o = g.poff[q], n = g.pn[q];
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    double s = 0.0;
    for (int m = 1; m < n / 2; ++m) {
      const int r = (int)(((int64_t)m * l) % n);   // exact argument reduction
      s += sin(2.0 * kPi * (double)r / (double)n) / (double)m;
    }
    iw[o + l] = 2.0 * s / (double)n;
  }
}

// H+ of sigma_1 and sigma_2 on every curve; block (q, d), d the density. hp layout:
// [d][re|im][N].
__global__ __launch_bounds__(256) void k_hplus(int64_t N, Geo g, const double* __restrict__ vp,
                                               const double* __restrict__ pF, const double* __restrict__ iw,
                                               double* __restrict__ hp) {
  __shared__ double sc[16];
  const int q = blockIdx.x, d = blockIdx.y;
  const int o = g.poff[q], n = g.pn[q];
  const double cx = g.pcx[q], cy = g.pcy[q];
  const double Q = pF[4 * q + d];
  const double* vre = vp + (int64_t)(2 * d) * N;
  const double* vim = vp + (int64_t)(2 * d + 1) * N;
  double* hre = hp + (int64_t)(2 * d) * N;
  double* him = hp + (int64_t)(2 * d + 1) * N;
  // g_k = y'_k H'+_k, H'+ = -2 pi i v+ - Q / (y - c), staged in LDS; then its antiderivative
  __shared__ double gre[kMaxNodesPerParticle], gim[kMaxNodesPerParticle];
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int64_t i = o + k;
    const zc dv = {2.0 * kPi * vim[i], -2.0 * kPi * vre[i]};
    const zc qc = zinv({g.x[i] - cx, g.y[i] - cy});
    const zc gv = zmul({g.xpx[i], g.xpy[i]}, {dv.re - Q * qc.re, dv.im - Q * qc.im});
    gre[k] = gv.re;
    gim[k] = gv.im;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double ar = 0.0, ai = 0.0;
    for (int k = 0; k < n; ++k) {
      const int l = j - k >= 0 ? j - k : j - k + n;
      const double w = iw[o + l];
      ar += w * gre[k];
      ai += w * gim[k];
    }
    hre[o + j] = ar;
    him[o + j] = ai;
  }
  __syncthreads();
  // constant: the interior Cauchy integral at c vanishes, C = -sum H W/(y - c) / sum W/(y - c)
  double nr = 0, ni = 0, dr = 0, di = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int64_t i = o + k;
    const zc W = {g.xpy[i] / (double)n, -g.xpx[i] / (double)n};
    const zc u = zmul(W, zinv({g.x[i] - cx, g.y[i] - cy}));
    const zc t = zmul({hre[i], him[i]}, u);
    nr += t.re;
    ni += t.im;
    dr += u.re;
    di += u.im;
  }
  nr = block_sum(nr, sc);
  ni = block_sum(ni, sc);
  dr = block_sum(dr, sc);
  di = block_sum(di, sc);
  const zc Cn = zmul({nr, ni}, zinv({dr, di}));
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    hre[o + k] -= Cn.re;
    him[o + k] -= Cn.im;
  }
}

struct FieldArgs {
  int64_t N, nt;
  const double *xt, *yt;
  Geo g;
  const double *f1, *f2;      // w sigma
  const double* vp;           // v+ of sigma_1, sigma_2, sigma~ [6][N]
  const double* hp;           // H+ of sigma_1, sigma_2 [4][N]
  const double* pF;           // per particle: F1, F2 (= Q of sigma_1, sigma_2), ...
  const double *px, *py, *xi; // proxies and strengths (cell 0)
  int M;
  const double *vel, *om, *gauge;
  double mu, gamma, cUx, cUy, close_factor;
  int plain_given;            // u, p already hold the near-image plain sums (FMM tree walk)
  double *u, *p;
};

__device__ __forceinline__ void stokeslet_up(double rx, double ry, double f1, double f2, double k4, double& u1,
                                             double& u2, double& pp) {
  const double r2 = rx * rx + ry * ry;
  const double ir2 = rcp64(r2);
  const double lg = -0.5 * log(r2);
  const double rf = (rx * f1 + ry * f2) * ir2;
  u1 += k4 * (lg * f1 + rx * rf);
  u2 += k4 * (lg * f2 + ry * rf);
  pp += rf * (0.5 / kPi);
}

// One 64-lane wave per target.
__global__ __launch_bounds__(256) void k_field(FieldArgs A) {
  const int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (t >= A.nt) return;
  const Geo& g = A.g;
  const double skew = g.cskew[0];
  const double x = A.xt[t], y = A.yt[t];
  // periodic copy in U: lattice coordinates (alpha, beta) of x - c_U reduced to [-1/2, 1/2)
  const double be = y - A.cUy, al = (x - A.cUx) - skew * be;
  const double ka = floor(al + 0.5), kb = floor(be + 0.5);
  const double xw = x - ka - kb * skew, yw = y - kb;
  const double k4 = 1.0 / (4.0 * kPi * A.mu);
  // interior of a particle image: its rigid motion
  for (int q = 0; q < g.No; ++q) {
    for (int s = 0; s < kShifts; ++s) {
      const double sx = shift_x(s, skew), sy = shift_y(s);
      const double dx = xw - (g.pcx[q] + sx), dy = yw - (g.pcy[q] + sy);
      if (dx * dx + dy * dy >= g.pa[q] * g.pa[q]) continue;
      double sth, cth;
      sincos(g.pth[q], &sth, &cth);
      const double bu = cth * dx + sth * dy, bv = -sth * dx + cth * dy;
      const double* pp = g.pprm + 4 * (int64_t)q;
      bool ins;
      if (g.pkind[q] == SPM_SHAPE_ELLIPSE) {
        ins = (bu / pp[0]) * (bu / pp[0]) + (bv / pp[1]) * (bv / pp[1]) < 1.0;
      } else {
        const double r = pp[0] * (1.0 + pp[1] * cos(pp[2] * atan2(bv, bu) + pp[3]));
        ins = bu * bu + bv * bv < r * r;
      }
      if (ins) {
        if (lane == 0) {
          A.u[t] = A.vel[2 * q] + A.gamma * (sy + (y - yw)) - A.om[q] * dy;
          A.u[A.nt + t] = A.vel[2 * q + 1] + A.om[q] * dx;
          A.p[t] = __builtin_nan("");
        }
        return;
      }
    }
  }
  // near images (plain rule) and the proxy correction
  double u1 = 0, u2 = 0, pr = 0;
  if (A.plain_given && lane == 0) {
    u1 = A.u[t];
    u2 = A.u[A.nt + t];
    pr = A.p[t];
  }
  for (int64_t j = A.plain_given ? A.N : lane; j < A.N; j += 64) {
    const double yx = g.x[j], yy = g.y[j], a = A.f1[j], b = A.f2[j];
    for (int s = 0; s < kShifts; ++s)
      stokeslet_up(xw - (yx + shift_x(s, skew)), yw - (yy + shift_y(s)), a, b, k4, u1, u2, pr);
  }
  for (int m = lane; m < A.M; m += 64) {
    const double a = A.xi[m], b = A.xi[A.M + m];
    stokeslet_up(xw - A.px[m], yw - A.py[m], a, b, k4, u1, u2, pr);
    double z1 = 0, z2 = 0, zp = 0;
    stokeslet_up(A.cUx - A.px[m], A.cUy - A.py[m], a, b, k4, z1, z2, zp);
    u1 -= z1;
    u2 -= z2;
  }
  // close curve images: replace the plain terms by the Laplace decomposition
  for (int q = 0; q < g.No; ++q) {
    const int o = g.poff[q], n = g.pn[q];
    const double lim = A.close_factor * g.pper[q] / (double)n;
    if (!(lim > 0.0)) continue;
    const double cx = g.pcx[q], cy = g.pcy[q];
    for (int s = 0; s < kShifts; ++s) {
      const double sx = shift_x(s, skew), sy = shift_y(s);
      const double zr = xw - sx, zi = yw - sy;   // target shifted instead of the image
      const double rc = sqrt((zr - cx) * (zr - cx) + (zi - cy) * (zi - cy));
      if (rc >= g.pa[q] + lim) continue;
      double m2 = 1e300;
      for (int k = lane; k < n; k += 64) {
        const double rx = zr - g.x[o + k], ry = zi - g.y[o + k];
        const double d2 = rx * rx + ry * ry;
        m2 = d2 < m2 ? d2 : m2;
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double w = __shfl_xor(m2, off, 64);
        m2 = w < m2 ? w : m2;
      }
      if (m2 >= lim * lim) continue;
      // plain terms of this image, barycentric sums
      double q1 = 0, q2 = 0, qp = 0;
      zc den = {0, 0}, v[3] = {{0, 0}, {0, 0}, {0, 0}}, H[2] = {{0, 0}, {0, 0}};
      for (int k = lane; k < n; k += 64) {
        const int64_t i = o + k;
        stokeslet_up(zr - g.x[i], zi - g.y[i], A.f1[i], A.f2[i], k4, q1, q2, qp);
        const zc W = {g.xpy[i] / (double)n, -g.xpx[i] / (double)n};
        const zc uu = zmul(W, zinv({g.x[i] - zr, g.y[i] - zi}));
        den.re += uu.re;
        den.im += uu.im;
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
          const zc tv = zmul({A.vp[(2 * dd) * A.N + i], A.vp[(2 * dd + 1) * A.N + i]}, uu);
          v[dd].re += tv.re;
          v[dd].im += tv.im;
        }
#pragma unroll
        for (int dd = 0; dd < 2; ++dd) {
          const zc th = zmul({A.hp[(2 * dd) * A.N + i], A.hp[(2 * dd + 1) * A.N + i]}, uu);
          H[dd].re += th.re;
          H[dd].im += th.im;
        }
      }
      q1 = wave_sum(q1);
      q2 = wave_sum(q2);
      qp = wave_sum(qp);
      den.re = wave_sum(den.re) - 1.0;
      den.im = wave_sum(den.im);
      const zc idn = zinv(den);
      double gx[3], gy[3];
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) {
        const zc vv = zmul({wave_sum(v[dd].re), wave_sum(v[dd].im)}, idn);
        gx[dd] = -vv.im;   // grad S_L = (Re A, -Im A), A = i v
        gy[dd] = -vv.re;
      }
      const double X1 = zr - cx, X2 = zi - cy;
      const double lgc = 0.5 * log(X1 * X1 + X2 * X2);
      double SL[2];
#pragma unroll
      for (int dd = 0; dd < 2; ++dd) {
        const zc hh = zmul({wave_sum(H[dd].re), wave_sum(H[dd].im)}, idn);
        SL[dd] = -(0.5 / kPi) * (A.pF[4 * q + dd] * lgc + hh.re);
      }
      const double c1 = (0.5 * SL[0] + 0.5 * gx[2] - 0.5 * X1 * gx[0] - 0.5 * X2 * gx[1]) / A.mu;
      const double c2 = (0.5 * SL[1] + 0.5 * gy[2] - 0.5 * X1 * gy[0] - 0.5 * X2 * gy[1]) / A.mu;
      const double cp = -(gx[0] + gy[1]);
      // every lane holds the same sums; lane 0 carries the replacement into its partial sums
      if (lane == 0) {
        u1 += c1 - q1;
        u2 += c2 - q2;
        pr += cp - qp;
      }
    }
  }
  u1 = wave_sum(u1);
  u2 = wave_sum(u2);
  pr = wave_sum(pr);
  if (lane == 0) {
    A.u[t] = A.gamma * y + u1 - A.gauge[0];
    A.u[A.nt + t] = u2 - A.gauge[1];
    A.p[t] = pr;
  }
}

void launch_field(spm_handle* h, int64_t n_targets, const double* xt, const double* yt, double* u, double* p) {
  const Geo& g = h->geo;
  Field& F = h->fd;
  k_int_weights<<<g.No, 256, 0, h->stream>>>(g, F.iw);
  SPM_HIP_CHECK(hipGetLastError());
  k_hplus<<<dim3((unsigned)g.No, 2), 256, 0, h->stream>>>(g.N, g, h->cl.vp, h->wk.pF, F.iw, F.hp);
  SPM_HIP_CHECK(hipGetLastError());
  FieldArgs A;
  A.N = g.N;
  A.nt = n_targets;
  A.xt = xt;
  A.yt = yt;
  A.g = g;
  A.f1 = h->wk.f1;
  A.f2 = h->wk.f2;
  A.vp = h->cl.vp;
  A.hp = F.hp;
  A.pF = h->wk.pF;
  A.px = h->per.px;
  A.py = h->per.py;
  A.xi = h->wk.xi;
  A.M = h->per.M;
  A.vel = F.vel;
  A.om = F.om;
  A.gauge = h->wk.gauge;
  A.mu = h->cfg.mu;
  A.gamma = h->cfg.gamma;
  A.cUx = h->cU[0];
  A.cUy = h->cU[1];
  A.close_factor = h->cfg.close_factor;
  A.u = u;
  A.p = p;
  A.plain_given = 0;
  if (h->fmm.on) {           // near-image plain sums by the FMM's tree walk
    launch_fmm_points(h, n_targets, xt, yt, u, p);
    A.plain_given = 1;
  }
  const int64_t blocks = (n_targets * 64 + 255) / 256;
  k_field<<<(unsigned)blocks, 256, 0, h->stream>>>(A);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace spm
