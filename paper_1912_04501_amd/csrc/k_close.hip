// Close evaluation of the single-layer traction (Sec. 6.3), exterior barycentric rule.
//
// For source curve q with nodes y_k (complex), y'_k = dy/dt, tangent tau_k, and the three
// real densities f in {sigma_1, sigma_2, (y - c_q).sigma}: phi = f conj(tau),
//   v+_j = sum_{k != j} (phi_k - phi_j) W_k / (y_k - y_j) + phi'_j / (i N),  W_k = y'_k / (i N),
// phi' the spectral t-derivative (Nyquist mode zeroed) by the closed-form matrix
//   D_jk = (1/2) (-1)^(j-k) cot((j-k) pi / N), j != k  (N even).
// At an exterior target z:  den = -1 + sum W_k/(y_k - z),  v = sum v+_k W_k/(y_k - z) / den,
//   v' = sum (v+_k - v) W_k/(y_k - z)^2 / den.
// With A = i v, A' = i v':  grad S_L[f] = (Re A, -Im A), Hess S_L[f] = [[Re A', -Im A'], [-Im A', -Re A']],
// and the traction of the Stokes single layer (the Sec. 6.3 decomposition; sign as in eq. Gt)
//   T = H[f3] n - (x-c)_1 H[f1] n - (x-c)_2 H[f2] n + (d1 S_L[f1] + d2 S_L[f2]) n.
// The correction for a close (target, image) pair is T minus the plain near-sum terms of
// that image, recomputed with the near kernel's own per-pair arithmetic and precision.
#include "spm_internal.h"

namespace spm {

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cinv(cplx a) {
  const double d = rcp64(a.re * a.re + a.im * a.im);
  return {a.re * d, -a.im * d};
}

// v+ of the three densities, written to vp[6][N]. Block (q, by) takes the nodes
// j in [by R, by R + R) of particle q (R = blockDim / L rows, L lanes per node); the source
// nodes pass through LDS in tiles of kVplusTile. Lane `sub` of a node takes k = sub, sub + L,
// ... (tile sizes are multiples of L) and the lanes' sums are combined by a fixed butterfly.
__global__ __launch_bounds__(1024) void k_vplus(int64_t N, Geo g, const double* __restrict__ sigma, int L,
                                                const int32_t* __restrict__ need, const int32_t* __restrict__ active,
                                                double* __restrict__ vp) {
  __shared__ double s_yr[kVplusTile], s_yi[kVplusTile];
  __shared__ double s_wr[kVplusTile], s_wi[kVplusTile];
  __shared__ double s_ph[6][kVplusTile];
  const int q = blockIdx.x;
  if (need && need[q] == 0) return;   // no close pair takes this particle as its source
  if (active && active[g.pcell[q]] == 0) return;   // its cell is not iterating
  const int o = g.poff[q], n = g.pn[q];
  const int R = blockDim.x / L;
  const int j = blockIdx.y * R + threadIdx.x / L;
  if (blockIdx.y * R >= n) return;   // whole block: this particle has fewer nodes
  const double cx = g.pcx[q], cy = g.pcy[q];
  const bool own = j < n;
  const int sub = threadIdx.x % L;
  double yjr = 0, yji = 0, pj[6] = {0, 0, 0, 0, 0, 0};
  if (own) {   // phi = f conj(tau) at node j
    const int64_t i = o + j;
    yjr = g.x[i];
    yji = g.y[i];
    const double t1 = g.tx[i], t2 = g.ty[i], sg1 = sigma[i], sg2 = sigma[N + i];
    const double f[3] = {sg1, sg2, (yjr - cx) * sg1 + (yji - cy) * sg2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pj[2 * d] = f[d] * t1;
      pj[2 * d + 1] = -f[d] * t2;
    }
  }
  double acc[6] = {0, 0, 0, 0, 0, 0};
  double der[6] = {0, 0, 0, 0, 0, 0};
  for (int kb = 0; kb < n; kb += kVplusTile) {
    const int nt = min(kVplusTile, n - kb);
    __syncthreads();   // the previous tile has been consumed
    for (int k = threadIdx.x; k < nt; k += blockDim.x) {
      const int64_t i = o + kb + k;
      s_yr[k] = g.x[i];
      s_yi[k] = g.y[i];
      // W = y' / (i n) = (y'_im - i y'_re) / n
      s_wr[k] = g.xpy[i] / (double)n;
      s_wi[k] = -g.xpx[i] / (double)n;
      const double t1 = g.tx[i], t2 = g.ty[i], sg1 = sigma[i], sg2 = sigma[N + i];
      const double f[3] = {sg1, sg2, (g.x[i] - cx) * sg1 + (g.y[i] - cy) * sg2};
      for (int d = 0; d < 3; ++d) {
        s_ph[2 * d][k] = f[d] * t1;
        s_ph[2 * d + 1][k] = -f[d] * t2;
      }
    }
    __syncthreads();
    if (own) {
      for (int kk = sub; kk < nt; kk += L) {
        const int k = kb + kk;
        if (k == j) continue;
        const cplx u = cmul({s_wr[kk], s_wi[kk]}, cinv({s_yr[kk] - yjr, s_yi[kk] - yji}));
        const int dm = j - k >= 0 ? j - k : j - k + n;
        const double dw = g.dcot[o + dm];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const cplx dp = {s_ph[2 * d][kk] - pj[2 * d], s_ph[2 * d + 1][kk] - pj[2 * d + 1]};
          const cplx t = cmul(dp, u);
          acc[2 * d] += t.re;
          acc[2 * d + 1] += t.im;
          der[2 * d] += dw * s_ph[2 * d][kk];
          der[2 * d + 1] += dw * s_ph[2 * d + 1][kk];
        }
      }
    }
  }
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    acc[d] = group_sum(acc[d], L);
    der[d] = group_sum(der[d], L);
  }
  if (!own || sub != 0) return;
  const int64_t i = o + j;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // phi' / (i n) = (phi'_im - i phi'_re) / n
    vp[(2 * d) * N + i] = acc[2 * d] + der[2 * d + 1] / (double)n;
    vp[(2 * d + 1) * N + i] = acc[2 * d + 1] - der[2 * d] / (double)n;
  }
}

// Lanes per node of k_vplus: enough rows for the largest curve in one 1024-thread block
// while curves fit one block; above that, 16 lanes and more blocks per particle.
inline int vplus_lanes(int nmax) { return nmax <= kVplusTile ? lanes_per_row(nmax) : 16; }

// all_particles: every curve (field evaluation near any particle); otherwise only the sources of
// the close pairs, which is all the operator's close correction reads
void launch_vplus(spm_handle* h, const double* sigma, bool all_particles, bool with_active) {
  const int L = vplus_lanes(h->geo.nmax);
  const int R = 1024 / L;
  const dim3 grid((unsigned)h->geo.No, (unsigned)((h->geo.nmax + R - 1) / R));
  k_vplus<<<grid, 1024, 0, h->stream>>>(h->geo.N, h->geo, sigma, L, all_particles ? nullptr : h->cl.qsrc,
                                        with_active ? h->kr.active : nullptr, h->cl.vp);
  SPM_HIP_CHECK(hipGetLastError());
}

// One 64-lane wave per close target; lanes stride over the source nodes.
template <int PREC>
__global__ __launch_bounds__(256) void k_close_apply(int64_t N, int32_t ntargets, Geo g,
                                                     const int32_t* __restrict__ tlist, const int32_t* __restrict__ row,
                                                     const int32_t* __restrict__ cq, const int32_t* __restrict__ cs,
                                                     const double* __restrict__ vp, const double* __restrict__ f1,
                                                     const double* __restrict__ f2, const float* __restrict__ f1f,
                                                     const float* __restrict__ f2f, const int32_t* __restrict__ active,
                                                     double* __restrict__ T) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= ntargets) return;
  const int i = tlist[wave];
  const double skew = g.cskew[g.ncell[i]];
  if (active != nullptr && active[g.ncell[i]] == 0) return;
  const double xi = g.x[i], yi = g.y[i], nxi = g.nx[i], nyi = g.ny[i];
  double dT1 = 0, dT2 = 0;
  for (int e = row[i]; e < row[i + 1]; ++e) {
    const int q = cq[e], s = cs[e];
    const int o = g.poff[q], n = g.pn[q];
    const double shx = shift_x(s, skew), shy = shift_y(s);
    const float shxf = (float)shx, shyf = (float)shy;
    const double zr = xi - shx, zi = yi - shy;  // target shifted instead of the image
    // pass 1: den and v for the three densities; plain near-sum terms of this image
    double dr = 0, di = 0, v[6] = {0, 0, 0, 0, 0, 0};
    double p1 = 0, p2 = 0;
    for (int k = lane; k < n; k += 64) {
      const int64_t kk = o + k;
      const cplx W = {g.xpy[kk] / (double)n, -g.xpx[kk] / (double)n};
      const cplx u = cmul(W, cinv({g.x[kk] - zr, g.y[kk] - zi}));
      dr += u.re;
      di += u.im;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const cplx t = cmul({vp[(2 * d) * N + kk], vp[(2 * d + 1) * N + kk]}, u);
        v[2 * d] += t.re;
        v[2 * d + 1] += t.im;
      }
      if (PREC == SPM_FP64) {
        const double dx = xi - g.x[kk], dy = yi - g.y[kk];
        double a1 = 0.0, a2 = 0.0;
        gt_pair(dx - shx, row_terms(dy, shy, nyi, f2[kk]), nxi, f1[kk], a1, a2);
        p1 += a1;
        p2 += a2;
      } else if (!g.dilated) {
        const float dx = g.xf[i] - g.xf[kk], dy = g.yf[i] - g.yf[kk];
        float a1 = 0.f, a2 = 0.f;
        const PairTerms32 pt = pair_terms32(g.nxf[i], g.nyf[i], f1f[kk], f2f[kk]);
        gt_pair32(dx - shxf, row_terms32_any(dy, shyf, pt), pt, a1, a2);
        p1 += (double)a1;
        p2 += (double)a2;
      } else {
        // dilated set: the FP32 shadows are the wrapped nodes, and the near sum met node kk of
        // this curve image at the lattice shift t = s + (wrap of i) - (wrap of kk); the same
        // shift expression and per-pair arithmetic as the near kernel's
        const int32_t wi = g.nwrap[i], wk = g.nwrap[kk];
        const int tm = s / 3 - 1 + node_wrap_ka(wi) - node_wrap_ka(wk);
        const int tn = s % 3 - 1 + node_wrap_kb(wi) - node_wrap_kb(wk);
        const float dx = g.xf[i] - g.xf[kk], dy = g.yf[i] - g.yf[kk];
        float a1 = 0.f, a2 = 0.f;
        gt_pair(dx - (float)shift_xmn(tm, tn, skew), row_terms(dy, (float)tn, g.nyf[i], f2f[kk]), g.nxf[i], f1f[kk],
                a1, a2);
        p1 += (double)a1;
        p2 += (double)a2;
      }
    }
    dr = wave_sum(dr);
    di = wave_sum(di);
#pragma unroll
    for (int d = 0; d < 6; ++d) v[d] = wave_sum(v[d]);
    p1 = wave_sum(p1);
    p2 = wave_sum(p2);
    const cplx iden = cinv({dr - 1.0, di});
    cplx vv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) vv[d] = cmul({v[2 * d], v[2 * d + 1]}, iden);
    // pass 2: v' = sum (v+_k - v) W_k / (y_k - z)^2 / den
    double w[6] = {0, 0, 0, 0, 0, 0};
    for (int k = lane; k < n; k += 64) {
      const int64_t kk = o + k;
      const cplx W = {g.xpy[kk] / (double)n, -g.xpx[kk] / (double)n};
      const cplx id = cinv({g.x[kk] - zr, g.y[kk] - zi});
      const cplx u2 = cmul(cmul(W, id), id);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const cplx t = cmul({vp[(2 * d) * N + kk] - vv[d].re, vp[(2 * d + 1) * N + kk] - vv[d].im}, u2);
        w[2 * d] += t.re;
        w[2 * d + 1] += t.im;
      }
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) w[d] = wave_sum(w[d]);
    // A = i v, A' = i v'
    double g1[3], g2[3], h11[3], h12[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const cplx vd = cmul({w[2 * d], w[2 * d + 1]}, iden);
      const cplx A = {-vv[d].im, vv[d].re};
      const cplx Ap = {-vd.im, vd.re};
      g1[d] = A.re;
      g2[d] = -A.im;
      h11[d] = Ap.re;
      h12[d] = -Ap.im;
    }
    const double rx = zr - g.pcx[q], ry = zi - g.pcy[q];
    double Hn1[3], Hn2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      Hn1[d] = h11[d] * nxi + h12[d] * nyi;
      Hn2[d] = h12[d] * nxi - h11[d] * nyi;
    }
    const double dv = g1[0] + g2[1];
    const double Tb1 = Hn1[2] - rx * Hn1[0] - ry * Hn1[1] + dv * nxi;
    const double Tb2 = Hn2[2] - rx * Hn2[0] - ry * Hn2[1] + dv * nyi;
    dT1 += Tb1 - (-(1.0 / kPi)) * p1;
    dT2 += Tb2 - (-(1.0 / kPi)) * p2;
  }
  if (lane == 0) {
    T[i] += dT1;
    T[N + i] += dT2;
  }
}

void launch_close_apply_impl(spm_handle* h, double* T, int precision, bool with_active) {
  const int nt = h->cl.ntargets;
  if (nt == 0) return;
  const int waves_per_block = 4;
  const unsigned blocks = (unsigned)((nt + waves_per_block - 1) / waves_per_block);
  if (precision == SPM_FP64)
    k_close_apply<SPM_FP64><<<blocks, 256, 0, h->stream>>>(
        h->geo.N, nt, h->geo, h->cl.tlist, h->cl.row, h->cl.q, h->cl.s, h->cl.vp, h->wk.f1, h->wk.f2, h->wk.f1f,
        h->wk.f2f, with_active ? h->kr.active : nullptr, T);
  else
    k_close_apply<SPM_FP32><<<blocks, 256, 0, h->stream>>>(
        h->geo.N, nt, h->geo, h->cl.tlist, h->cl.row, h->cl.q, h->cl.s, h->cl.vp, h->wk.f1, h->wk.f2, h->wk.f1f,
        h->wk.f2f, with_active ? h->kr.active : nullptr, T);
  SPM_HIP_CHECK(hipGetLastError());
}

void launch_close_apply(spm_handle* h, const double* sigma, double* T, int precision) {
  (void)sigma;
  launch_close_apply_impl(h, T, precision, false);
}

// Own-curve terms of the FP32 near sum. For a target and the other nodes of its own
// curve (zero shift), r = x_i - y_k is a short chord nearly tangent to the curve: FP32
// node coordinates leave r with a relative error of about eps32 |x| / |r| and the
// cancellation in r.n magnifies it, so these few terms (sum of N_q^2 over particles,
// a tiny fraction of all pairs) are recomputed in FP64 and the FP32 ones, evaluated
// with the near kernel's own per-pair arithmetic, are removed:
//   T_i += -(1/pi) sum_{k on the curve of i} (a64(i, k) - a32(i, k)).
// Groups of kSelfFixLanes lanes per target (sources k = sub, sub + lanes, ...), 256-thread
// blocks over (particle, range of its targets).
constexpr int kSelfFixLanes = 16;
__global__ __launch_bounds__(256) void k_self_fix(int64_t N, Geo g, const double* __restrict__ f1,
                                                   const double* __restrict__ f2, const float* __restrict__ f1f,
                                                   const float* __restrict__ f2f, const int32_t* __restrict__ active,
                                                   int L, double* __restrict__ T) {
  const int q = blockIdx.x;
  if (active != nullptr && active[g.pcell[q]] == 0) return;
  const int o = g.poff[q], n = g.pn[q];
  const int sub = threadIdx.x % L, per = blockDim.x / L;
  for (int k0 = blockIdx.y * per + threadIdx.x / L; k0 < n; k0 += gridDim.y * per) {
    const int64_t i = o + k0;
    const double xi = g.x[i], yi = g.y[i], nxi = g.nx[i], nyi = g.ny[i];
    const float xif = g.xf[i], yif = g.yf[i], nxif = g.nxf[i], nyif = g.nyf[i];
    const int32_t wi = g.dilated ? g.nwrap[i] : 0;
    const double skew = g.cskew[g.pcell[q]];
    double d1 = 0.0, d2 = 0.0, e1 = 0.0, e2 = 0.0;
    for (int k = sub; k < n; k += L) {
      const int64_t kk = o + k;
      {
        const double dx = xi - g.x[kk], dy = yi - g.y[kk];
        double a1 = 0.0, a2 = 0.0;
        gt_pair(dx - 0.0, row_terms(dy, 0.0, nyi, f2[kk]), nxi, f1[kk], a1, a2);
        d1 += a1;
        d2 += a2;
      }
      if (!g.dilated) {
        const float dx = xif - g.xf[kk], dy = yif - g.yf[kk];
        float a1 = 0.f, a2 = 0.f;
        const PairTerms32 pt = pair_terms32(nxif, nyif, f1f[kk], f2f[kk]);
        gt_pair32(dx - 0.0f, row_terms32<true>(dy, 0.0f, pt), pt, a1, a2);
        e1 += (double)a1;
        e2 += (double)a2;
      } else {   // wrapped nodes: the own curve's node kk sits at shift (wrap of i) - (wrap of kk)
        const int tm = node_wrap_ka(wi) - node_wrap_ka(g.nwrap[kk]);
        const int tn = node_wrap_kb(wi) - node_wrap_kb(g.nwrap[kk]);
        const float dx = xif - g.xf[kk], dy = yif - g.yf[kk];
        float a1 = 0.f, a2 = 0.f;
        gt_pair(dx - (float)shift_xmn(tm, tn, skew), row_terms(dy, (float)tn, nyif, f2f[kk]), nxif, f1f[kk], a1, a2);
        e1 += (double)a1;
        e2 += (double)a2;
      }
    }
    const double c1 = group_sum(d1 - e1, L), c2 = group_sum(d2 - e2, L);
    if (sub == 0) {
      T[i] += -(1.0 / kPi) * c1;
      T[N + i] += -(1.0 / kPi) * c2;
    }
  }
}

void launch_self_fix(spm_handle* h, double* T, bool with_active) {
  const int per = 256 / kSelfFixLanes;
  const dim3 grid((unsigned)h->geo.No, (unsigned)((h->geo.nmax + per - 1) / per));
  k_self_fix<<<grid, 256, 0, h->stream>>>(h->geo.N, h->geo, h->wk.f1, h->wk.f2, h->wk.f1f, h->wk.f2f,
                                          with_active ? h->kr.active : nullptr, kSelfFixLanes, T);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace spm
