// GMRES on the device for every cell of the ensemble (solver of Sec. 6.2 / Sec. 8:
// relative residual 1e-10).
//
// Cells iterate in lockstep on one iteration index j held in device memory, so the
// kernels of one iteration have fixed arguments and can be captured once and replayed.
// Each cell has its own Hessenberg matrix, Givens rotations, right-hand-side norm,
// tolerance and active flag; a cell that converges freezes (its rows are skipped) and
// records the device wall clock.
// Arnoldi: classical Gram-Schmidt with one reorthogonalisation pass (CGS2): two block
// dot-product passes per iteration instead of j + 1 sequential MGS steps.
// All reductions are two-phase in fixed order (segment partials, then per-cell sums),
// so results do not depend on scheduling.
#include "spm_internal.h"

namespace spm {

// part[s] = sum over the nodes of segment s of a.b (both components).
__global__ __launch_bounds__(256) void k_dot_seg(const double* __restrict__ a, const double* __restrict__ b, int64_t N,
                                                 const int64_t* __restrict__ n0, const int64_t* __restrict__ n1,
                                                 double* __restrict__ part) {
  __shared__ double sc[16];
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int64_t r = n0[s] + threadIdx.x; r < n1[s]; r += blockDim.x) acc += a[r] * b[r] + a[N + r] * b[N + r];
  acc = block_sum(acc, sc);
  if (threadIdx.x == 0) part[s] = acc;
}

// One wave per cell: lanes take the cell's segment partials k = lane, lane + 64, ..., then a
// fixed butterfly.
__global__ __launch_bounds__(256) void k_dot_cells(const double* __restrict__ part, const int32_t* __restrict__ seg_off,
                                                   int C, double* __restrict__ out) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= C) return;
  double s = 0.0;
  for (int k = seg_off[c] + lane; k < seg_off[c + 1]; k += 64) s += part[k];
  s = wave_sum(s);
  if (lane == 0) out[c] = s;
}

void gm_dot(spm_handle* h, const double* a, const double* b, double* out) {
  Krylov& K = h->kr;
  k_dot_seg<<<K.nseg, 256, 0, h->stream>>>(a, b, h->geo.N, K.seg_n0, K.seg_n1, K.part);
  SPM_HIP_CHECK(hipGetLastError());
  k_dot_cells<<<(h->geo.C + 3) / 4, 256, 0, h->stream>>>(K.part, K.seg_off, h->geo.C, out);
  SPM_HIP_CHECK(hipGetLastError());
}

// part[s][i] = sum over segment s of V_i . w, for i <= j; one wave per (segment, i).
__global__ __launch_bounds__(256) void k_cgs_partial(const double* __restrict__ V, int64_t n2, int64_t N,
                                                     const int32_t* __restrict__ jdev, const double* __restrict__ w,
                                                     const int64_t* __restrict__ n0, const int64_t* __restrict__ n1,
                                                     const int32_t* __restrict__ seg_cell,
                                                     const int32_t* __restrict__ active, int ldp,
                                                     double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int s = blockIdx.x;
  if (i > jdev[0] || active[seg_cell[s]] == 0) return;
  const double* vi = V + (int64_t)i * n2;
  double acc = 0.0;
  for (int64_t r = n0[s] + lane; r < n1[s]; r += 64) acc += vi[r] * w[r] + vi[N + r] * w[N + r];
  acc = wave_sum(acc);
  if (lane == 0) part[(int64_t)s * ldp + i] = acc;
}

// coef[c][i] = sum of the cell's segment partials part[k][i]: one wave per (cell, i), lanes over
// the segments k = lane, lane + 64, ..., then a fixed butterfly.
__global__ __launch_bounds__(256) void k_cgs_reduce(const double* __restrict__ part, const int32_t* __restrict__ seg_off,
                                                    const int32_t* __restrict__ jdev,
                                                    const int32_t* __restrict__ active, int ldp,
                                                    double* __restrict__ coef) {
  const int c = blockIdx.x;
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (active[c] == 0 || i > jdev[0]) return;
  double s = 0.0;
  for (int k = seg_off[c] + lane; k < seg_off[c + 1]; k += 64) s += part[(int64_t)k * ldp + i];
  s = wave_sum(s);
  if (lane == 0) coef[(int64_t)c * ldp + i] = s;
}

void gm_cgs_pass(spm_handle* h, const double* w, double* coef) {
  Krylov& K = h->kr;
  const int ldp = K.kmax + 1;
  dim3 grid((unsigned)K.nseg, (unsigned)((ldp + 3) / 4));
  k_cgs_partial<<<grid, 256, 0, h->stream>>>(K.V, K.n2, h->geo.N, K.jdev, w, K.seg_n0, K.seg_n1, K.seg_cell,
                                             K.active, ldp, K.part);
  SPM_HIP_CHECK(hipGetLastError());
  k_cgs_reduce<<<dim3((unsigned)h->geo.C, (unsigned)((ldp + 3) / 4)), 256, 0, h->stream>>>(K.part, K.seg_off, K.jdev,
                                                                                            K.active, ldp, coef);
  SPM_HIP_CHECK(hipGetLastError());
}

// w[r] -= sum_{i <= j} V_i[r] coef[cell(r)][i] (active cells only).
// A 256-thread block covers 64 entries r with 4 groups; group g sums the basis vectors
// i = g, g+4, ... (coalesced over r for every i), and the four partial sums are added in
// fixed order through LDS.
constexpr int kUpdGroups = 4;

__global__ __launch_bounds__(256) void k_update_j(const double* __restrict__ V, int64_t n2, int64_t N,
                                                  const int32_t* __restrict__ jdev, const double* __restrict__ coef,
                                                  int ldp, const int32_t* __restrict__ ncell,
                                                  const int32_t* __restrict__ active, double* __restrict__ w) {
  __shared__ double part[kUpdGroups][64];
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t r = blockIdx.x * (int64_t)64 + lane;
  const bool live = r < n2;
  const int c = live ? ncell[r < N ? r : r - N] : 0;
  const bool act = live && active[c] != 0;
  double s = 0.0;
  if (act) {
    const int cnt = jdev[0] + 1;
    const double* cf = coef + (int64_t)c * ldp;
    for (int i = grp; i < cnt; i += kUpdGroups) s += V[(int64_t)i * n2 + r] * cf[i];
  }
  part[grp][lane] = s;
  __syncthreads();
  if (grp == 0 && act) w[r] -= (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

void gm_update_j(spm_handle* h, const double* coef, double* w) {
  Krylov& K = h->kr;
  k_update_j<<<(unsigned)((K.n2 + 63) / 64), 256, 0, h->stream>>>(K.V, K.n2, h->geo.N, K.jdev, coef, K.kmax + 1,
                                                                  h->geo.ncell, K.active, w);
  SPM_HIP_CHECK(hipGetLastError());
}

// V_{j+1} = w / |w|_cell (active cells)
__global__ void k_store_next(double* __restrict__ V, int64_t n2, int64_t N, const int32_t* __restrict__ jdev,
                             const double* __restrict__ w, const double* __restrict__ nrm2,
                             const int32_t* __restrict__ ncell, const int32_t* __restrict__ active) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n2) return;
  const int c = ncell[r < N ? r : r - N];
  if (active[c] == 0) return;
  const double nr = sqrt(nrm2[c]);
  V[(int64_t)(jdev[0] + 1) * n2 + r] = nr > 0.0 ? w[r] / nr : 0.0;
}

void gm_store_next(spm_handle* h) {
  Krylov& K = h->kr;
  k_store_next<<<(unsigned)((K.n2 + 255) / 256), 256, 0, h->stream>>>(K.V, K.n2, h->geo.N, K.jdev, K.w, K.nrm2,
                                                                      h->geo.ncell, K.active);
  SPM_HIP_CHECK(hipGetLastError());
}

// One wavefront per cell: column j of H = h1 + h2 (CGS2), subdiagonal |w|; apply the previous
// rotations, make rotation j, update g; res = |g_{j+1}| / bnorm; a cell whose residual
// estimate reaches its tolerance freezes and records the wall clock. The lanes stage the
// column and the stored rotations in LDS in pieces of kGivensPiece and write the rotated
// column back; lane 0 applies the rotations in order (the same arithmetic, in the same order,
// as one thread working from device memory). The last wavefront to finish (a counter in device
// memory that it resets) counts the cells still active and advances j.
constexpr int kGivensPiece = 256;

__global__ __launch_bounds__(64) void k_givens(int C, int kmax, int32_t* __restrict__ jdev,
                                               const double* __restrict__ h1, const double* __restrict__ h2,
                                               const double* __restrict__ nrm2, const double* __restrict__ bnorm,
                                               const double* __restrict__ tolc, double* __restrict__ H,
                                               double* __restrict__ cs, double* __restrict__ sn,
                                               double* __restrict__ g, double* __restrict__ res,
                                               int32_t* __restrict__ active, int32_t* __restrict__ kdone,
                                               unsigned long long* __restrict__ stamp,
                                               int32_t* __restrict__ done_count) {
  __shared__ double hp[kGivensPiece], cp[kGivensPiece], sp[kGivensPiece];
  const int c = blockIdx.x, lane = threadIdx.x;
  const int j = jdev[0];
  const int ldp = kmax + 1;
  if (active[c] != 0) {
    double* col = H + ((int64_t)c * kmax + j) * ldp;
    const double* a1 = h1 + (int64_t)c * ldp;
    const double* a2 = h2 + (int64_t)c * ldp;
    double* csc = cs + (int64_t)c * kmax;
    double* snc = sn + (int64_t)c * kmax;
    double* gc = g + (int64_t)c * ldp;
    double x = a1[0] + a2[0];   // h_0, then h_i after rotations 0..i-1 (lane 0's copy is used)
    for (int i0 = 0; i0 < j; i0 += kGivensPiece) {
      const int i1 = min(i0 + kGivensPiece, j);
      for (int i = i0 + lane; i < i1; i += 64) {
        cp[i - i0] = csc[i];
        sp[i - i0] = snc[i];
        hp[i - i0] = a1[i + 1] + a2[i + 1];   // h_{i+1}
      }
      __syncthreads();
      if (lane == 0) {
        for (int i = i0; i < i1; ++i) {
          const double y = hp[i - i0], cc = cp[i - i0], ss = sp[i - i0];
          const double t = cc * x + ss * y;
          x = -ss * x + cc * y;
          hp[i - i0] = t;   // rotated h_i
        }
      }
      __syncthreads();
      for (int i = i0 + lane; i < i1; i += 64) col[i] = hp[i - i0];
      __syncthreads();
    }
    if (lane == 0) {
      const double b = sqrt(nrm2[c]);
      const double r = hypot(x, b);
      const double cc = r > 0.0 ? x / r : 1.0, ss = r > 0.0 ? b / r : 0.0;
      csc[j] = cc;
      snc[j] = ss;
      col[j] = r;
      col[j + 1] = 0.0;
      const double gj = gc[j];
      gc[j + 1] = -ss * gj;
      gc[j] = cc * gj;
      const double e = fabs(gc[j + 1]) / bnorm[c];
      res[c] = e;
      if (!(e > tolc[c]) || j + 1 >= kmax || r == 0.0) {   // converged, out of space, or exact (breakdown)
        active[c] = 0;
        kdone[c] = j + 1;
        stamp[c] = wall_clock64();
      }
    }
  }
  if (lane == 0) {
    __threadfence();
    if (atomicAdd(done_count, 1) == C - 1) {   // the last cell's wavefront
      __threadfence();
      int t = 0;
      for (int k = 0; k < C; ++k) t += active[k];
      jdev[1] = t;
      jdev[0] = j + 1;
      *done_count = 0;
    }
  }
}

void gm_givens(spm_handle* h) {
  Krylov& K = h->kr;
  k_givens<<<h->geo.C, 64, 0, h->stream>>>(h->geo.C, K.kmax, K.jdev, K.h1, K.h2, K.nrm2, K.bnorm, K.tolc, K.H, K.cs,
                                           K.sn, K.g, K.res, K.active, K.kdone, K.stamp, K.gcount);
  SPM_HIP_CHECK(hipGetLastError());
}

// vin = V_j
__global__ void k_copy_in(const double* __restrict__ V, int64_t n2, const int32_t* __restrict__ jdev,
                          double* __restrict__ vin) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n2) return;
  vin[r] = V[(int64_t)jdev[0] * n2 + r];
}

void gm_copy_in(spm_handle* h) {
  Krylov& K = h->kr;
  k_copy_in<<<(unsigned)((K.n2 + 255) / 256), 256, 0, h->stream>>>(K.V, K.n2, K.jdev, K.vin);
  SPM_HIP_CHECK(hipGetLastError());
}

// Start of a Krylov cycle for r = V_0 (unnormalised, already in V): nrm2 = |r|^2 per cell.
// Cells whose |r| is already within tolerance start inactive (kdone 0).
__global__ void k_start(int C, int kmax, const double* __restrict__ nrm2, const double* __restrict__ bnorm,
                        const double* __restrict__ tolc, double* __restrict__ g, int32_t* __restrict__ active,
                        int32_t* __restrict__ kdone, double* __restrict__ res, int32_t* __restrict__ jdev) {
  __shared__ int cnt[1024];
  int n = 0;
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    const double beta = sqrt(nrm2[c]);
    double* gc = g + (int64_t)c * (kmax + 1);
    for (int i = 0; i <= kmax; ++i) gc[i] = 0.0;
    gc[0] = beta;
    const int act = (active[c] != 0) && (beta > tolc[c] * bnorm[c]);
    active[c] = act;
    kdone[c] = 0;
    res[c] = beta / bnorm[c];
    n += act;
  }
  cnt[threadIdx.x] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < (int)blockDim.x; ++k) t += cnt[k];
    jdev[0] = 0;
    jdev[1] = t;
  }
}

__global__ void k_normalize0(double* __restrict__ V, int64_t n2, int64_t N, const double* __restrict__ nrm2,
                             const int32_t* __restrict__ ncell) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n2) return;
  const double nr = sqrt(nrm2[ncell[r < N ? r : r - N]]);
  V[r] = nr > 0.0 ? V[r] / nr : 0.0;
}

// V_0 holds r; active/bnorm/tolc are set by the caller.
void gm_start(spm_handle* h) {
  Krylov& K = h->kr;
  gm_dot(h, K.V, K.V, K.nrm2);
  const int bs = h->geo.C >= 1024 ? 1024 : ((h->geo.C + 63) / 64) * 64;
  k_start<<<1, bs, 0, h->stream>>>(h->geo.C, K.kmax, K.nrm2, K.bnorm, K.tolc, K.g, K.active, K.kdone, K.res, K.jdev);
  SPM_HIP_CHECK(hipGetLastError());
  k_normalize0<<<(unsigned)((K.n2 + 255) / 256), 256, 0, h->stream>>>(K.V, K.n2, h->geo.N, K.nrm2, h->geo.ncell);
  SPM_HIP_CHECK(hipGetLastError());
}

// y_c = R_c^{-1} g_c[0..k_c) (k_c = kdone, or j for cells still active), then
// x[r] += sum_{i < k_c} V_i[r] y_c[i] (k_update_x). One wavefront per cell, column by column:
// lane r % 64 holds the running right-hand side of rows r (up to kBackRegs per lane); y_i is
// formed on its lane and broadcast, and every row above takes its column-i term. Cycles longer
// than 64 kBackRegs iterations are solved row by row on one lane.
constexpr int kBackRegs = 8;

__global__ __launch_bounds__(64) void k_backsolve(int C, int kmax, const int32_t* __restrict__ jdev,
                                                  const double* __restrict__ H, const double* __restrict__ g,
                                                  const int32_t* __restrict__ active, int32_t* __restrict__ kdone,
                                                  double* __restrict__ y) {
  const int c = blockIdx.x, lane = threadIdx.x;
  if (c >= C) return;
  const int k = active[c] != 0 ? jdev[0] : kdone[c];
  if (lane == 0 && active[c] != 0) kdone[c] = k;
  const int ldp = kmax + 1;
  const double* gc = g + (int64_t)c * ldp;
  const double* Hc = H + (int64_t)c * kmax * ldp;   // column q of R at Hc + q ldp (rows 0..q)
  double* yc = y + (int64_t)c * kmax;
  if (k > 64 * kBackRegs) {
    if (lane == 0)
      for (int i = k - 1; i >= 0; --i) {
        double s = gc[i];
        for (int q = i + 1; q < k; ++q) s -= Hc[(int64_t)q * ldp + i] * yc[q];
        const double d = Hc[(int64_t)i * ldp + i];
        yc[i] = d != 0.0 ? s / d : 0.0;
      }
    return;
  }
  double v[kBackRegs];
#pragma unroll
  for (int t = 0; t < kBackRegs; ++t) {
    const int r = lane + 64 * t;
    v[t] = r < k ? gc[r] : 0.0;
  }
  for (int i = k - 1; i >= 0; --i) {
    const int owner = i & 63, slot = i >> 6;
    double vi = 0.0;
#pragma unroll
    for (int t = 0; t < kBackRegs; ++t)
      if (t == slot) vi = v[t];
    const double d = Hc[(int64_t)i * ldp + i];
    double yi = d != 0.0 ? vi / d : 0.0;
    yi = __shfl(yi, owner, 64);
    const double* Ri = Hc + (int64_t)i * ldp;
#pragma unroll
    for (int t = 0; t < kBackRegs; ++t) {
      const int r = lane + 64 * t;
      if (t == slot && lane == owner) v[t] = yi;
      else if (r < i) v[t] = fma(-Ri[r], yi, v[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < kBackRegs; ++t) {
    const int r = lane + 64 * t;
    if (r < k) yc[r] = v[t];
  }
}

__global__ void k_update_x(const double* __restrict__ V, int64_t n2, int64_t N, int kmax,
                           const int32_t* __restrict__ kdone, const double* __restrict__ y,
                           const int32_t* __restrict__ ncell, double* __restrict__ x) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n2) return;
  const int c = ncell[r < N ? r : r - N];
  const int k = kdone[c];
  const double* yc = y + (int64_t)c * kmax;
  double s = 0.0;
  for (int i = 0; i < k; ++i) s += V[(int64_t)i * n2 + r] * yc[i];
  x[r] += s;
}

void gm_backsolve(spm_handle* h) {
  Krylov& K = h->kr;
  k_backsolve<<<h->geo.C, 64, 0, h->stream>>>(h->geo.C, K.kmax, K.jdev, K.H, K.g, K.active, K.kdone, K.yv);
  SPM_HIP_CHECK(hipGetLastError());
}

void gm_update_only(spm_handle* h, double* x) {
  Krylov& K = h->kr;
  k_update_x<<<(unsigned)((K.n2 + 255) / 256), 256, 0, h->stream>>>(K.V, K.n2, h->geo.N, K.kmax, K.kdone, K.yv,
                                                                    h->geo.ncell, x);
  SPM_HIP_CHECK(hipGetLastError());
}

void gm_backsolve_update(spm_handle* h, double* x) {
  gm_backsolve(h);
  gm_update_only(h, x);
}

__global__ void k_zero_i32(int64_t n, int32_t* __restrict__ p) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r < n) p[r] = 0;
}

void gm_zero_i32(spm_handle* h, int32_t* p, int64_t n) {
  k_zero_i32<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>(n, p);
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

// out[r] = a deterministic pseudo-random value in [-1, 1) of index r (the splitmix64 finaliser
// of r + seed; a probe vector for measuring operator errors, not part of the method).
__global__ void k_probe_fill(int64_t n, uint64_t seed, double* __restrict__ out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  uint64_t z = (uint64_t)r + seed + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  out[r] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

void gm_probe_fill(spm_handle* h, int64_t n, uint64_t seed, double* out) {
  k_probe_fill<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>(n, seed, out);
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

__global__ void k_stamp_start(unsigned long long* stamp, int C) {
  if (threadIdx.x == 0 && blockIdx.x == 0) stamp[C] = wall_clock64();
}

void gm_stamp_start(spm_handle* h) {
  k_stamp_start<<<1, 64, 0, h->stream>>>(h->kr.stamp, h->geo.C);
  SPM_HIP_CHECK(hipGetLastError());
}

// stamp[C + 1] = wall clock at the start of a Krylov cycle
__global__ void k_stamp_cycle(unsigned long long* stamp, int C) {
  if (threadIdx.x == 0 && blockIdx.x == 0) stamp[C + 1] = wall_clock64();
}

void gm_stamp_cycle(spm_handle* h) {
  k_stamp_cycle<<<1, 64, 0, h->stream>>>(h->kr.stamp, h->geo.C);
  SPM_HIP_CHECK(hipGetLastError());
}

// For the cells flagged in mask (convergence confirmed by the host after a cycle): keep the
// stamp k_givens wrote when the cell's Krylov iteration stopped in this cycle; a cell that
// stopped without iterating in this cycle gets the current wall clock.
__global__ void k_stamp_mask(unsigned long long* stamp, const int32_t* __restrict__ mask, int C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < C && mask[c] != 0 && stamp[c] < stamp[C + 1]) stamp[c] = wall_clock64();
}

void gm_stamp_mask(spm_handle* h, const int32_t* mask_dev) {
  k_stamp_mask<<<(h->geo.C + 63) / 64, 64, 0, h->stream>>>(h->kr.stamp, mask_dev, h->geo.C);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace spm
