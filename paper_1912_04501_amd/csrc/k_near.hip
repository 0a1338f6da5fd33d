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

template <typename R, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_near(int64_t N, const R* __restrict__ x, const R* __restrict__ y,
                                                const R* __restrict__ nx, const R* __restrict__ ny,
                                                const R* __restrict__ f1, const R* __restrict__ f2,
                                                int64_t chunk, int tile, Shifts<R> sh, double* __restrict__ Tpart) {
  extern __shared__ unsigned char smem_raw[];
  Src<R>* src = reinterpret_cast<Src<R>*>(smem_raw);
  const int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
  const int64_t j0 = blockIdx.y * chunk;
  const int64_t j1 = (j0 + chunk < N) ? j0 + chunk : N;
  R xi = 0, yi = 0, nxi = 0, nyi = 0;
  if (i < N) {
    xi = x[i];
    yi = y[i];
    nxi = nx[i];
    nyi = ny[i];
  }
  R a1 = 0, a2 = 0;
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
    for (int k = 0; k < cnt; ++k) {
      const Src<R> s = src[k];
      const R dx = xi - s.y1, dy = yi - s.y2;
#pragma unroll
      for (int m = 0; m < kShifts; ++m) gt_pair(dx - sh.x[m], dy - sh.y[m], nxi, nyi, s.f1, s.f2, a1, a2);
    }
  }
  if (i < N) {
    double* out = Tpart + blockIdx.y * 2 * N;
    out[i] = -(1.0 / kPi) * (double)a1;
    out[N + i] = -(1.0 / kPi) * (double)a2;
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

template <typename R>
static void near_dispatch(spm_handle* h, const R* x, const R* y, const R* nx, const R* ny, const R* f1,
                          const R* f2) {
  const int64_t N = h->geo.N;
  const int S = h->wk.splits;
  const int64_t chunk = (N + S - 1) / S;
  const int tile = h->wk.tile;
  const size_t lds = sizeof(Src<R>) * (size_t)tile;
  const Shifts<R> sh = make_shifts<R>(h);
  switch (h->wk.block) {
    case 64: {
      dim3 grid((unsigned)((N + 63) / 64), (unsigned)S);
      k_near<R, 64><<<grid, 64, lds, h->stream>>>(N, x, y, nx, ny, f1, f2, chunk, tile, sh, h->wk.Tpart);
      break;
    }
    case 128: {
      dim3 grid((unsigned)((N + 127) / 128), (unsigned)S);
      k_near<R, 128><<<grid, 128, lds, h->stream>>>(N, x, y, nx, ny, f1, f2, chunk, tile, sh, h->wk.Tpart);
      break;
    }
    default: {
      dim3 grid((unsigned)((N + 255) / 256), (unsigned)S);
      k_near<R, 256><<<grid, 256, lds, h->stream>>>(N, x, y, nx, ny, f1, f2, chunk, tile, sh, h->wk.Tpart);
      break;
    }
  }
  SPM_HIP_CHECK(hipGetLastError());
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
    near_dispatch<double>(h, g.x, g.y, g.nx, g.ny, h->wk.f1, h->wk.f2);
  else
    near_dispatch<float>(h, g.xf, g.yf, g.nxf, g.nyf, h->wk.f1f, h->wk.f2f);
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

void launch_near_sum_only(spm_handle* h, double* out) {
  const int64_t n2 = 2 * h->geo.N;
  k_sum_splits<<<(unsigned)((n2 + 255) / 256), 256, 0, h->stream>>>(n2, h->wk.splits, h->wk.Tpart, out);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace spm
