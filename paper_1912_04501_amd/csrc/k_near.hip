// Near-image traction sum (Sec. 4.2, G_near with the 3x3 images of every particle; Sec. 6 Nystrom):
//
//   T_near(x_i) = -(1/pi) sum_j sum_{s in S9} r (r.n_i)(r.f_j) / |r|^4,  r = x_i - (y_j + s),  f_j = w_j sigma_j
//
// Tiled direct N-body: one target per lane, source tiles staged in LDS (every lane of a
// wave reads the same source: LDS broadcast), the 9 image shifts applied to the source
// difference from scalar registers, sources split over blockIdx.y so that small
// problems still fill the 256 CUs; the split partials are summed in fixed order by
// the combine kernel (no atomics: deterministic).
#include "spm_internal.h"

namespace spm {

template <typename R>
struct Src {
  R y1, y2, f1, f2;
};

// TPT targets per lane (i, i + BLOCK, ...) share every LDS source read. Each LDS tile is
// summed in a fresh accumulator of the kernel's precision and then added to an FP64
// running sum, which keeps the FP32 summation error at the level of one tile.
template <typename R, int BLOCK, int TPT>
__global__ __launch_bounds__(BLOCK) void k_near(int64_t N, const R* __restrict__ x, const R* __restrict__ y,
                                                const R* __restrict__ nx, const R* __restrict__ ny,
                                                const R* __restrict__ f1, const R* __restrict__ f2,
                                                int64_t chunk, int tile, Shifts<R> sh, double* __restrict__ Tpart) {
  extern __shared__ unsigned char smem_raw[];
  Src<R>* src = reinterpret_cast<Src<R>*>(smem_raw);
  const int64_t i0 = blockIdx.x * (int64_t)(BLOCK * TPT) + threadIdx.x;
  const int64_t j0 = blockIdx.y * chunk;
  const int64_t j1 = (j0 + chunk < N) ? j0 + chunk : N;
  R xi[TPT], yi[TPT], nxi[TPT], nyi[TPT];
  double A1[TPT], A2[TPT];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const int64_t i = i0 + t * BLOCK;
    xi[t] = 0;
    yi[t] = 0;
    nxi[t] = 0;
    nyi[t] = 0;
    if (i < N) {
      xi[t] = x[i];
      yi[t] = y[i];
      nxi[t] = nx[i];
      nyi[t] = ny[i];
    }
    A1[t] = 0.0;
    A2[t] = 0.0;
  }
  for (int64_t jt = j0; jt < j1; jt += tile) {
    const int cnt = (int)((jt + tile < j1) ? tile : (j1 - jt));
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += BLOCK) {
      Src<R> s;
      s.y1 = x[jt + k];
      s.y2 = y[jt + k];
      s.f1 = f1[jt + k];
      s.f2 = f2[jt + k];
      src[k] = s;
    }
    __syncthreads();
    R a1[TPT], a2[TPT];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
      a1[t] = 0;
      a2[t] = 0;
    }
    for (int k = 0; k < cnt; ++k) {
      const Src<R> s = src[k];
#pragma unroll
      for (int t = 0; t < TPT; ++t) {
        const R dx = xi[t] - s.y1, dy = yi[t] - s.y2;
#pragma unroll
        for (int m = 0; m < kShifts; ++m)
          gt_pair(dx - sh.x[m], dy - sh.y[m], nxi[t], nyi[t], s.f1, s.f2, a1[t], a2[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
      A1[t] += (double)a1[t];
      A2[t] += (double)a2[t];
    }
  }
  double* out = Tpart + blockIdx.y * 2 * N;
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const int64_t i = i0 + t * BLOCK;
    if (i < N) {
      out[i] = -(1.0 / kPi) * A1[t];
      out[N + i] = -(1.0 / kPi) * A2[t];
    }
  }
}

template <typename R>
static Shifts<R> make_shifts(spm_handle* h) {
  Shifts<R> sh;
  for (int m = -1; m <= 1; ++m)
    for (int n = -1; n <= 1; ++n) {
      const int s = 3 * (m + 1) + (n + 1);
      sh.x[s] = (R)((double)m * h->e1[0] + (double)n * h->e2[0]);
      sh.y[s] = (R)((double)m * h->e1[1] + (double)n * h->e2[1]);
    }
  return sh;
}

template <typename R, int BLOCK, int TPT>
static void near_launch(spm_handle* h, const R* x, const R* y, const R* nx, const R* ny, const R* f1, const R* f2,
                        int splits, int tile) {
  const int64_t N = h->geo.N;
  const int64_t chunk = (N + splits - 1) / splits;
  const size_t lds = sizeof(Src<R>) * (size_t)tile;
  dim3 grid((unsigned)((N + BLOCK * TPT - 1) / (BLOCK * TPT)), (unsigned)splits);
  k_near<R, BLOCK, TPT><<<grid, BLOCK, lds, h->stream>>>(N, x, y, nx, ny, f1, f2, chunk, tile, make_shifts<R>(h),
                                                         h->wk.Tpart);
  SPM_HIP_CHECK(hipGetLastError());
}

template <typename R>
static void near_dispatch(spm_handle* h, const R* x, const R* y, const R* nx, const R* ny, const R* f1,
                          const R* f2, const NearConfig& c) {
  const int key = c.block * 10 + c.tpt;
  switch (key) {
    case 641: near_launch<R, 64, 1>(h, x, y, nx, ny, f1, f2, c.splits, c.tile); break;
    case 642: near_launch<R, 64, 2>(h, x, y, nx, ny, f1, f2, c.splits, c.tile); break;
    case 644: near_launch<R, 64, 4>(h, x, y, nx, ny, f1, f2, c.splits, c.tile); break;
    case 1281: near_launch<R, 128, 1>(h, x, y, nx, ny, f1, f2, c.splits, c.tile); break;
    case 1282: near_launch<R, 128, 2>(h, x, y, nx, ny, f1, f2, c.splits, c.tile); break;
    case 1284: near_launch<R, 128, 4>(h, x, y, nx, ny, f1, f2, c.splits, c.tile); break;
    case 2561: near_launch<R, 256, 1>(h, x, y, nx, ny, f1, f2, c.splits, c.tile); break;
    case 2562: near_launch<R, 256, 2>(h, x, y, nx, ny, f1, f2, c.splits, c.tile); break;
    case 2564: near_launch<R, 256, 4>(h, x, y, nx, ny, f1, f2, c.splits, c.tile); break;
    default: throw ApiError(SPM_EINVAL, "unsupported near-sum launch configuration");
  }
}

bool near_config_valid(const NearConfig& c) {
  const bool b = c.block == 64 || c.block == 128 || c.block == 256;
  const bool t = c.tpt == 1 || c.tpt == 2 || c.tpt == 4;
  return b && t && c.tile >= 16 && c.tile <= 1024 && c.splits >= 1;
}

void prof_flush(spm_handle* h) {
  if (h->ev_used == 0) return;
  SPM_HIP_CHECK(hipEventSynchronize(h->ev_pool[2 * h->ev_used - 1]));
  for (size_t k = 0; k < h->ev_used; ++k) {
    float ms = 0.f;
    SPM_HIP_CHECK(hipEventElapsedTime(&ms, h->ev_pool[2 * k], h->ev_pool[2 * k + 1]));
    h->prof_ms[h->ev_kind[k]] += ms;
  }
  h->ev_used = 0;
}

void launch_near(spm_handle* h, int precision) {
  const Geo& g = h->geo;
  const int kind = precision == SPM_FP64 ? 0 : 1;
  if (h->prof) {
    if (h->ev_used * 2 + 2 > h->ev_pool.size()) {
      if (h->ev_pool.size() >= 512) prof_flush(h);
      while (h->ev_used * 2 + 2 > h->ev_pool.size()) {
        hipEvent_t e;
        SPM_HIP_CHECK(hipEventCreate(&e));
        h->ev_pool.push_back(e);
      }
    }
    if (h->ev_kind.size() < h->ev_pool.size() / 2) h->ev_kind.resize(h->ev_pool.size() / 2);
    h->ev_kind[h->ev_used] = kind;
    SPM_HIP_CHECK(hipEventRecord(h->ev_pool[2 * h->ev_used], h->stream));
  }
  if (precision == SPM_FP64)
    near_dispatch<double>(h, g.x, g.y, g.nx, g.ny, h->wk.f1, h->wk.f2, h->wk.near[0]);
  else
    near_dispatch<float>(h, g.xf, g.yf, g.nxf, g.nyf, h->wk.f1f, h->wk.f2f, h->wk.near[1]);
  if (h->prof) {
    SPM_HIP_CHECK(hipEventRecord(h->ev_pool[2 * h->ev_used + 1], h->stream));
    ++h->ev_used;
    h->prof_launches[kind] += 1;
    h->prof_pairs[kind] += (double)kShifts * (double)g.N * (double)g.N;
  }
}

// Sum of the split partials only (stage entry point for checking the near sum).
__global__ void k_sum_splits(int64_t n2, int S, const double* __restrict__ Tpart, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n2) return;
  double s = 0.0;
  for (int k = 0; k < S; ++k) s += Tpart[k * n2 + i];
  out[i] = s;
}

void launch_near_sum_only(spm_handle* h, double* out, int precision) {
  const int64_t n2 = 2 * h->geo.N;
  const int S = h->wk.near[precision == SPM_FP64 ? 0 : 1].splits;
  k_sum_splits<<<(unsigned)((n2 + 255) / 256), 256, 0, h->stream>>>(n2, S, h->wk.Tpart, out);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace spm
