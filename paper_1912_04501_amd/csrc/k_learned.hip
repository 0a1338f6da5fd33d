// Learned warm start: per-particle neighbour features, body-frame Fourier targets of a
// density, decoding of predicted coefficients back to the nodes, and the cell-wide
// normal-offset updates.
//
// The completed operator maps the normal field n to n/2 (the single layer with density
// n is a pure pressure, so K n = n/2; the pin subtracts n/2; L n = 0). A density is
// therefore fixed by local geometry only up to a cell-wide multiple of n: the targets
// leave that multiple out, and the warm start fits it to its own residual.
#include "spm_internal.h"

namespace spm {

constexpr int kNeigh = 8;

// One thread per particle: the 8 nearest other particle images of its cell (3x3
// images, own images included), ordered by (squared distance, particle, shift).
__global__ void k_features(Geo g, float* __restrict__ feat) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.No) return;
  const int c = g.pcell[q];
  const double skew = g.cskew[c];
  const double cx = g.pcx[q], cy = g.pcy[q];
  double bd[kNeigh];
  int bj[kNeigh], bs[kNeigh];
#pragma unroll
  for (int k = 0; k < kNeigh; ++k) {
    bd[k] = 1e300;
    bj[k] = 0x7fffffff;
    bs[k] = 0;
  }
  for (int j = g.cpoff[c]; j < g.cpoff[c + 1]; ++j) {
    const double jx = g.pcx[j], jy = g.pcy[j];
    for (int s = 0; s < kShifts; ++s) {
      if (j == q && s == kZeroShift) continue;
      const double dx = (jx + shift_x(s, skew)) - cx;
      const double dy = (jy + shift_y(s)) - cy;
      const double d2 = dx * dx + dy * dy;
      // candidates arrive in increasing (j, s): the new one goes before the first entry
      // with a strictly larger d2 (ties keep the earlier entry first) and every entry
      // after it moves down one slot
      if (!(d2 < bd[kNeigh - 1])) continue;
      double vd = d2;
      int vj = j, vs = s;
      bool moved = false;
#pragma unroll
      for (int k = 0; k < kNeigh; ++k) {
        if (moved || vd < bd[k]) {
          moved = true;
          const double td = bd[k];
          const int tj = bj[k], ts = bs[k];
          bd[k] = vd;
          bj[k] = vj;
          bs[k] = vs;
          vd = td;
          vj = tj;
          vs = ts;
        }
      }
    }
  }
  double st, ct;
  sincos(g.pth[q], &st, &ct);
  const double ia = 1.0 / g.pa[q];
  float* f = feat + (int64_t)q * SPM_MLP_IN;
#pragma unroll
  for (int k = 0; k < kNeigh; ++k) {
    const int j = bj[k], s = bs[k];
    if (j >= g.No) {   // unreachable: every particle has 8 images of itself
      f[4 * k + 0] = f[4 * k + 1] = f[4 * k + 2] = f[4 * k + 3] = 0.f;
      continue;
    }
    const double dx = (g.pcx[j] + shift_x(s, skew)) - cx;
    const double dy = (g.pcy[j] + shift_y(s)) - cy;
    const double dth = 2.0 * (g.pth[j] - g.pth[q]);
    double sd, cd;
    sincos(dth, &sd, &cd);
    f[4 * k + 0] = (float)((ct * dx + st * dy) * ia);
    f[4 * k + 1] = (float)((-st * dx + ct * dy) * ia);
    f[4 * k + 2] = (float)cd;
    f[4 * k + 3] = (float)sd;
  }
  f[SPM_MLP_IN - 1] = (float)(g.pa[q] / g.pb[q]);
}

// Round FP32 to bfloat16, nearest even (the network's matrix-core operand format).
__global__ void k_to_bf16(int64_t n, const float* __restrict__ in, uint16_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned u = __float_as_uint(in[i]);
  u += 0x7fffu + ((u >> 16) & 1u);
  out[i] = (uint16_t)(u >> 16);
}

void launch_to_bf16(spm_handle* h, const float* in, int64_t n, uint16_t* out) {
  if (n <= 0) return;
  k_to_bf16<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>(n, in, out);
  SPM_HIP_CHECK(hipGetLastError());
}

void launch_features(spm_handle* h, float* feat) {
  const int n = h->geo.No;
  k_features<<<(n + 127) / 128, 128, 0, h->stream>>>(h->geo, feat);
  SPM_HIP_CHECK(hipGetLastError());
}

// angle 2 pi ((m k) mod n) / n of the twiddle exp(i m t_k), reduced exactly in integers
__device__ __forceinline__ void twiddle(int m, int k, int n, double& c, double& s) {
  int r = (m * k) % n;
  if (r < 0) r += n;
  sincos(2.0 * kPi * (double)r / (double)n, &s, &c);
}

// One block (128 threads) per particle: c_m = (1/N) sum_k s_k exp(-i m t_k), m = -32..31,
// of s = R(-theta) (sigma - beta n) / (mu gamma), beta = num[cell] / den[cell].
__global__ __launch_bounds__(128) void k_modes(Geo g, const double* __restrict__ sigma,
                                               const double* __restrict__ num, const double* __restrict__ den,
                                               double inv_mg, float* __restrict__ modes) {
  __shared__ double s1[kMaxNodesStaged], s2[kMaxNodesStaged];
  const int q = blockIdx.x;
  const int64_t i0 = g.poff[q];
  const int n = g.pn[q];
  const int cell = g.pcell[q];
  const double beta = num ? num[cell] / den[cell] : 0.0;
  double st, ct;
  sincos(g.pth[q], &st, &ct);
  const int64_t N = g.N;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int64_t i = i0 + k;
    const double a = sigma[i] - beta * g.nx[i], b = sigma[N + i] - beta * g.ny[i];
    s1[k] = (ct * a + st * b) * inv_mg;
    s2[k] = (-st * a + ct * b) * inv_mg;
  }
  __syncthreads();
  const int o = threadIdx.x;   // 0..63 real part of mode o - 32, 64..127 imaginary part
  const int m = (o & 63) - 32;
  double re = 0.0, im = 0.0;
  for (int k = 0; k < n; ++k) {
    double c, s;
    twiddle(m, k, n, c, s);
    // (s1 + i s2)(c - i s)
    re += s1[k] * c + s2[k] * s;
    im += s2[k] * c - s1[k] * s;
  }
  modes[(int64_t)q * SPM_MLP_OUT + o] = (float)((o < 64 ? re : im) / (double)n);
}

void launch_modes(spm_handle* h, const double* sigma, const double* num, const double* den, float* modes) {
  if (h->geo.nmax > kMaxNodesStaged)
    throw ApiError(SPM_EINVAL, "density modes need at most " + std::to_string(kMaxNodesStaged) + " nodes per particle");
  k_modes<<<h->geo.No, 128, 0, h->stream>>>(h->geo, sigma, num, den, 1.0 / (h->cfg.mu * h->cfg.gamma), modes);
  SPM_HIP_CHECK(hipGetLastError());
}

// One block per particle: sigma_k = mu gamma R(theta) sum_m c_m exp(i m t_k).
__global__ __launch_bounds__(128) void k_decode(Geo g, const float* __restrict__ modes, double mg,
                                                double* __restrict__ sigma) {
  __shared__ double cr[64], ci[64];
  const int q = blockIdx.x;
  const float* c = modes + (int64_t)q * SPM_MLP_OUT;
  if (threadIdx.x < 64) {
    cr[threadIdx.x] = c[threadIdx.x];
    ci[threadIdx.x] = c[64 + threadIdx.x];
  }
  __syncthreads();
  const int64_t i0 = g.poff[q];
  const int n = g.pn[q];
  double st, ct;
  sincos(g.pth[q], &st, &ct);
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    double a = 0.0, b = 0.0;
    for (int mi = 0; mi < 64; ++mi) {
      double cc, ss;
      twiddle(mi - 32, k, n, cc, ss);
      // (cr + i ci)(cc + i ss)
      a += cr[mi] * cc - ci[mi] * ss;
      b += cr[mi] * ss + ci[mi] * cc;
    }
    sigma[i0 + k] = mg * (ct * a - st * b);
    sigma[g.N + i0 + k] = mg * (st * a + ct * b);
  }
}

void launch_decode(spm_handle* h, const float* modes, double* sigma) {
  k_decode<<<h->geo.No, 128, 0, h->stream>>>(h->geo, modes, h->cfg.mu * h->cfg.gamma, sigma);
  SPM_HIP_CHECK(hipGetLastError());
}

// Per cell: (alpha, beta) minimising |b - alpha z - beta n/2| from the dots
// d = [<z,z>, <z,n>, <n,n>, <b,z>, <b,n>] (each [C]); coef = [alpha(C), beta(C)].
// A zero z (zero guess) gives alpha = 0.
__global__ void k_fit_guess(int C, const double* __restrict__ d, double* __restrict__ coef) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const double zz = d[c], zh = 0.5 * d[C + c], hh = 0.25 * d[2 * C + c];
  const double bz = d[3 * C + c], bh = 0.5 * d[4 * C + c];
  const double det = zz * hh - zh * zh;
  double alpha = 0.0, beta = hh > 0.0 ? bh / hh : 0.0;
  if (zz > 0.0 && det > 1e-14 * zz * hh) {
    alpha = (bz * hh - bh * zh) / det;
    beta = (zz * bh - zh * bz) / det;
  }
  coef[c] = alpha;
  coef[C + c] = beta;
}

void launch_fit_guess(spm_handle* h, const double* dots, double* coef) {
  const int C = h->geo.C;
  k_fit_guess<<<(C + 63) / 64, 64, 0, h->stream>>>(C, dots, coef);
  SPM_HIP_CHECK(hipGetLastError());
}

// x = alpha x + beta n;  r = b - alpha z - (beta / 2) n   (per cell coefficients)
__global__ void k_apply_fit(int64_t N, const int32_t* __restrict__ ncell, const double* __restrict__ nx,
                            const double* __restrict__ ny, const double* __restrict__ coef, int C,
                            const double* __restrict__ b, const double* __restrict__ z, double* __restrict__ x,
                            double* __restrict__ r) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int c = ncell[i];
  const double al = coef[c], be = coef[C + c];
  x[i] = al * x[i] + be * nx[i];
  x[N + i] = al * x[N + i] + be * ny[i];
  r[i] = b[i] - al * z[i] - 0.5 * be * nx[i];
  r[N + i] = b[N + i] - al * z[N + i] - 0.5 * be * ny[i];
}

void launch_apply_fit(spm_handle* h, const double* coef, const double* b, const double* z, double* x, double* r) {
  const int64_t N = h->geo.N;
  k_apply_fit<<<(unsigned)((N + 255) / 256), 256, 0, h->stream>>>(N, h->geo.ncell, h->geo.nx, h->geo.ny, coef,
                                                                  h->geo.C, b, z, x, r);
  SPM_HIP_CHECK(hipGetLastError());
}

// Cells whose fitted guess is rejected (mask[cell] != 0) start from zero: x = 0, r = b.
__global__ void k_reject_guess(int64_t N, const int32_t* __restrict__ ncell, const int32_t* __restrict__ mask,
                               const double* __restrict__ b, double* __restrict__ x, double* __restrict__ r) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N || mask[ncell[i]] == 0) return;
  x[i] = 0.0;
  x[N + i] = 0.0;
  r[i] = b[i];
  r[N + i] = b[N + i];
}

void launch_reject_guess(spm_handle* h, const int32_t* mask, const double* b, double* x, double* r) {
  const int64_t N = h->geo.N;
  k_reject_guess<<<(unsigned)((N + 255) / 256), 256, 0, h->stream>>>(N, h->geo.ncell, mask, b, x, r);
  SPM_HIP_CHECK(hipGetLastError());
}

// x += f * (num[cell] / den[cell]) n over all nodes (SoA [2N])
__global__ void k_add_normal(int64_t N, const int32_t* __restrict__ ncell, const double* __restrict__ nx,
                             const double* __restrict__ ny, const double* __restrict__ num,
                             const double* __restrict__ den, double f, double* __restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int c = ncell[i];
  const double beta = f * num[c] / den[c];
  x[i] += beta * nx[i];
  x[N + i] += beta * ny[i];
}

void launch_add_normal(spm_handle* h, const double* num, const double* den, double f, double* x) {
  const int64_t N = h->geo.N;
  k_add_normal<<<(unsigned)((N + 255) / 256), 256, 0, h->stream>>>(N, h->geo.ncell, h->geo.nx, h->geo.ny, num, den,
                                                                   f, x);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace spm
