// GMRES on the device (solver of Sec. 6.2 / Sec. 8: relative residual 1e-10).
//
// Arnoldi by classical Gram-Schmidt with one reorthogonalisation pass (CGS2: two
// block dot-product passes instead of j+1 sequential MGS steps, same stability in
// practice); Givens rotations and the residual estimate |g_{j+1}| are updated on the
// device by one thread; the host only reads that scalar to stop.
// All reductions are two-phase in fixed order (chunk partials, then a per-coefficient
// sum), so results do not depend on scheduling.
#include "spm_internal.h"

namespace spm {

// part[c * ldp + i] = sum_{r in chunk c} V[i * ld + r] * w[r],  i < cnt.  One wave per (chunk, i).
__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ V, int64_t ld, int cnt,
                                                     const double* __restrict__ w, int64_t n, int64_t chunk,
                                                     double* __restrict__ part, int ldp) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= cnt) return;
  const int64_t r0 = blockIdx.x * chunk;
  const int64_t r1 = (r0 + chunk < n) ? r0 + chunk : n;
  const double* vi = V + i * ld;
  double s = 0.0;
  for (int64_t r = r0 + lane; r < r1; r += 64) s += vi[r] * w[r];
  s = wave_sum(s);
  if (lane == 0) part[(int64_t)blockIdx.x * ldp + i] = s;
}

__global__ void k_dot_reduce(const double* __restrict__ part, int nchunk, int ldp, int cnt, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * ldp + i];
  out[i] = s;
}

void gm_dot_many(spm_handle* h, const double* V, int64_t ld, int cnt, const double* w, double* out) {
  Krylov& k = h->kr;
  const int64_t n = k.n2;
  const int nc = k.nchunk;
  const int64_t chunk = (n + nc - 1) / nc;
  dim3 grid((unsigned)nc, (unsigned)((cnt + 3) / 4));
  k_dot_partial<<<grid, 256, 0, h->stream>>>(V, ld, cnt, w, n, chunk, k.part, k.kmax + 1);
  SPM_HIP_CHECK(hipGetLastError());
  k_dot_reduce<<<(cnt + 255) / 256, 256, 0, h->stream>>>(k.part, nc, k.kmax + 1, cnt, out);
  SPM_HIP_CHECK(hipGetLastError());
}

// w[r] += sign * sum_{i < cnt} V[i * ld + r] * coef[i]
__global__ void k_update(const double* __restrict__ V, int64_t ld, int cnt, const double* __restrict__ coef,
                         double* __restrict__ w, int64_t n, double sign) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  double s = 0.0;
  for (int i = 0; i < cnt; ++i) s += V[i * ld + r] * coef[i];
  w[r] += sign * s;
}

void gm_update(spm_handle* h, const double* V, int64_t ld, int cnt, const double* coef, double* w, double sign) {
  const int64_t n = h->kr.n2;
  k_update<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>(V, ld, cnt, coef, w, n, sign);
  SPM_HIP_CHECK(hipGetLastError());
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  out[r] = a * x[r] + (y ? b * y[r] : 0.0);
}

void gm_axpby(spm_handle* h, int64_t n, double a, const double* x, double b, const double* y, double* out) {
  k_axpby<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>(n, a, x, b, y, out);
  SPM_HIP_CHECK(hipGetLastError());
}

__global__ void k_copy(int64_t n, double* __restrict__ d, const double* __restrict__ s) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r < n) d[r] = s ? s[r] : 0.0;
}

void gm_copy(spm_handle* h, double* dst, const double* src, int64_t n) {
  k_copy<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>(n, dst, src);
  SPM_HIP_CHECK(hipGetLastError());
}

void gm_zero(spm_handle* h, double* dst, int64_t n) { gm_copy(h, dst, nullptr, n); }

// v /= sqrt(nrm2[0]) (zero vector stays zero); norm_out[0] = sqrt(nrm2[0])
__global__ void k_scale(const double* __restrict__ nrm2, double* __restrict__ v, int64_t n, double* __restrict__ norm_out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double nr = sqrt(nrm2[0]);
  if (r == 0 && norm_out) norm_out[0] = nr;
  if (r >= n) return;
  v[r] = nr > 0.0 ? v[r] / nr : 0.0;
}

void gm_scale_by_norm(spm_handle* h, const double* nrm2, double* v, int64_t n, double* norm_out) {
  k_scale<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>(nrm2, v, n, norm_out);
  SPM_HIP_CHECK(hipGetLastError());
}

// g = [beta, 0, ...]
__global__ void k_init(const double* __restrict__ nrm2, double* __restrict__ g, int kmax) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > kmax) return;
  g[i] = (i == 0) ? sqrt(nrm2[0]) : 0.0;
}

void gm_init(spm_handle* h, const double* nrm2) {
  k_init<<<(h->kr.kmax + 256) / 256, 256, 0, h->stream>>>(nrm2, h->kr.g, h->kr.kmax);
  SPM_HIP_CHECK(hipGetLastError());
}

// Column j of H = h1 + h2 (CGS2 passes), subdiagonal sqrt(nrm2); apply the previous
// rotations, make rotation j, update g; res[0] = |g_{j+1}| / bnorm.
__global__ void k_givens(int j, int kmax, const double* __restrict__ h1, const double* __restrict__ h2,
                         const double* __restrict__ nrm2, double bnorm, double* __restrict__ H, double* __restrict__ cs,
                         double* __restrict__ sn, double* __restrict__ g, double* __restrict__ res) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* col = H + (int64_t)j * (kmax + 1);
  for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
  col[j + 1] = sqrt(nrm2[0]);
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double a = col[j], b = col[j + 1];
  const double r = hypot(a, b);
  const double c = r > 0.0 ? a / r : 1.0, s = r > 0.0 ? b / r : 0.0;
  cs[j] = c;
  sn[j] = s;
  col[j] = r;
  col[j + 1] = 0.0;
  g[j + 1] = -s * g[j];
  g[j] = c * g[j];
  res[0] = fabs(g[j + 1]) / bnorm;
  res[1] = r;
}

void gm_givens(spm_handle* h, int j, const double* h1, const double* h2, const double* nrm2, double bnorm,
               double* res_out) {
  Krylov& k = h->kr;
  k_givens<<<1, 64, 0, h->stream>>>(j, k.kmax, h1, h2, nrm2, bnorm, k.H, k.cs, k.sn, k.g, res_out);
  SPM_HIP_CHECK(hipGetLastError());
}

// y = R^{-1} g[0..k) by back substitution (R upper triangular in H).
__global__ void k_backsolve(int k, int kmax, const double* __restrict__ H, const double* __restrict__ g,
                            double* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int c = i + 1; c < k; ++c) s -= H[(int64_t)c * (kmax + 1) + i] * y[c];
    const double d = H[(int64_t)i * (kmax + 1) + i];
    y[i] = d != 0.0 ? s / d : 0.0;
  }
}

void gm_backsolve(spm_handle* h, int k) {
  k_backsolve<<<1, 64, 0, h->stream>>>(k, h->kr.kmax, h->kr.H, h->kr.g, h->kr.yv);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace spm
