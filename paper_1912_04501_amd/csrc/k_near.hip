// Near-image traction sum (Sec. 4.2, G_near with the 3x3 images of every particle; Sec. 6 Nystrom):
//
//   T_near(x_i) = -(1/pi) sum_j sum_{s in S9} r (r.n_i)(r.f_j) / |r|^4,  r = x_i - (y_j + s),  f_j = w_j sigma_j
//
// for every cell of the ensemble (targets and sources of one cell only). Tiled direct
// N-body in one persistent launch: the grid drains a cost-sorted queue of work items
// (cell, block of targets, chunk of sources) through an atomic head. One target per
// lane (or TPT targets), source tiles staged in LDS (every lane of a wave reads the same
// source: LDS broadcast), the 9 image shifts of the item's cell applied to the source
// difference. Each item writes its own partial slot; the combine kernel sums the
// slots of a node in fixed order (deterministic, no floating-point atomics).
#include <algorithm>

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
                                                const double* __restrict__ cskew, const NearItem* __restrict__ items,
                                                int nitems, int* __restrict__ counter,
                                                const int32_t* __restrict__ active, int tile,
                                                double* __restrict__ Tpart) {
  extern __shared__ unsigned char smem_raw[];
  Src<R>* src = reinterpret_cast<Src<R>*>(smem_raw);
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= nitems) break;
    const NearItem I = items[it];
    if (active != nullptr && active[I.c] == 0) continue;
    R sx[kShifts], sy[kShifts];
    {
      const double skew = cskew[I.c];
#pragma unroll
      for (int m = 0; m < kShifts; ++m) {
        sx[m] = (R)shift_x(m, skew);
        sy[m] = (R)shift_y(m);
      }
    }
    R xi[TPT], yi[TPT], nxi[TPT], nyi[TPT];
    double A1[TPT], A2[TPT];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
      const int64_t i = I.t0 + threadIdx.x + t * BLOCK;
      xi[t] = 0;
      yi[t] = 0;
      nxi[t] = 0;
      nyi[t] = 0;
      if (i < I.t1) {
        xi[t] = x[i];
        yi[t] = y[i];
        nxi[t] = nx[i];
        nyi[t] = ny[i];
      }
      A1[t] = 0.0;
      A2[t] = 0.0;
    }
    for (int64_t jt = I.s0; jt < I.s1; jt += tile) {
      const int cnt = (int)((jt + tile < I.s1) ? tile : (I.s1 - jt));
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
          RowTerms<R> row[3];
#pragma unroll
          for (int n = 0; n < 3; ++n) row[n] = row_terms(dy, sy[n], nyi[t], s.f2);
#pragma unroll
          for (int m = 0; m < kShifts; ++m) gt_pair(dx - sx[m], row[m % 3], nxi[t], s.f1, a1[t], a2[t]);
        }
      }
#pragma unroll
      for (int t = 0; t < TPT; ++t) {
        A1[t] += (double)a1[t];
        A2[t] += (double)a2[t];
      }
    }
    double* out = Tpart + (int64_t)I.split * 2 * N;
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
      const int64_t i = I.t0 + threadIdx.x + t * BLOCK;
      if (i < I.t1) {
        out[i] = -(1.0 / kPi) * A1[t];
        out[N + i] = -(1.0 / kPi) * A2[t];
      }
    }
  }
}

__global__ void k_reset_counter(int* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[0] = 0;
}

template <typename R, int BLOCK, int TPT>
static int near_grid(int tile) {
  int per_cu = 0;
  const size_t lds = sizeof(Src<R>) * (size_t)tile;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_near<R, BLOCK, TPT>, BLOCK, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  int dev = 0, ncu = 0;
  SPM_HIP_CHECK(hipGetDevice(&dev));
  SPM_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  return per_cu * ncu;
}

template <typename R, int BLOCK, int TPT>
static void near_launch(spm_handle* h, const R* x, const R* y, const R* nx, const R* ny, const R* f1, const R* f2,
                        NearPlan& P, bool with_active) {
  const size_t lds = sizeof(Src<R>) * (size_t)P.cfg.tile;
  if (P.grid <= 0) P.grid = near_grid<R, BLOCK, TPT>(P.cfg.tile);
  const int grid = std::max(1, std::min(P.grid, P.nitems));
  k_reset_counter<<<1, 64, 0, h->stream>>>(P.counter);
  SPM_HIP_CHECK(hipGetLastError());
  k_near<R, BLOCK, TPT><<<grid, BLOCK, lds, h->stream>>>(h->geo.N, x, y, nx, ny, f1, f2, h->geo.cskew, P.items,
                                                         P.nitems, P.counter, with_active ? h->kr.active : nullptr,
                                                         P.cfg.tile, h->wk.Tpart);
  SPM_HIP_CHECK(hipGetLastError());
}

template <typename R>
static void near_dispatch(spm_handle* h, const R* x, const R* y, const R* nx, const R* ny, const R* f1,
                          const R* f2, NearPlan& P, bool with_active) {
  const int key = P.cfg.block * 10 + P.cfg.tpt;
  switch (key) {
    case 641: near_launch<R, 64, 1>(h, x, y, nx, ny, f1, f2, P, with_active); break;
    case 642: near_launch<R, 64, 2>(h, x, y, nx, ny, f1, f2, P, with_active); break;
    case 644: near_launch<R, 64, 4>(h, x, y, nx, ny, f1, f2, P, with_active); break;
    case 1281: near_launch<R, 128, 1>(h, x, y, nx, ny, f1, f2, P, with_active); break;
    case 1282: near_launch<R, 128, 2>(h, x, y, nx, ny, f1, f2, P, with_active); break;
    case 1284: near_launch<R, 128, 4>(h, x, y, nx, ny, f1, f2, P, with_active); break;
    case 2561: near_launch<R, 256, 1>(h, x, y, nx, ny, f1, f2, P, with_active); break;
    case 2562: near_launch<R, 256, 2>(h, x, y, nx, ny, f1, f2, P, with_active); break;
    case 2564: near_launch<R, 256, 4>(h, x, y, nx, ny, f1, f2, P, with_active); break;
    default: throw ApiError(SPM_EINVAL, "unsupported near-sum launch configuration");
  }
}

bool near_config_valid(const NearConfig& c) {
  const bool b = c.block == 64 || c.block == 128 || c.block == 256;
  const bool t = c.tpt == 1 || c.tpt == 2 || c.tpt == 4;
  return b && t && c.tile >= 16 && c.tile <= 1024 && c.chunk >= 16;
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

void launch_near_impl(spm_handle* h, int precision, bool with_active) {
  const Geo& g = h->geo;
  const int kind = precision == SPM_FP64 ? 0 : 1;
  NearPlan& P = h->wk.near[kind];
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
    near_dispatch<double>(h, g.x, g.y, g.nx, g.ny, h->wk.f1, h->wk.f2, P, with_active);
  else
    near_dispatch<float>(h, g.xf, g.yf, g.nxf, g.nyf, h->wk.f1f, h->wk.f2f, P, with_active);
  if (h->prof) {
    SPM_HIP_CHECK(hipEventRecord(h->ev_pool[2 * h->ev_used + 1], h->stream));
    ++h->ev_used;
    h->prof_launches[kind] += 1;
    double pairs = 0;
    for (const auto& c : h->cells) pairs += (double)kShifts * (double)(c.n1 - c.n0) * (double)(c.n1 - c.n0);
    h->prof_pairs[kind] += pairs;
  }
}

void launch_near(spm_handle* h, int precision) { launch_near_impl(h, precision, false); }

// Sum of the split partials only (stage entry point for checking the near sum).
__global__ void k_sum_splits(int64_t N, const int32_t* __restrict__ ncell, const int32_t* __restrict__ nsplit,
                             const double* __restrict__ Tpart, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int S = nsplit[ncell[i]];
  double s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < S; ++k) {
    s1 += Tpart[(int64_t)k * 2 * N + i];
    s2 += Tpart[(int64_t)k * 2 * N + N + i];
  }
  out[i] = s1;
  out[N + i] = s2;
}

void launch_near_sum_only(spm_handle* h, double* out, int precision) {
  const int64_t N = h->geo.N;
  const NearPlan& P = h->wk.near[precision == SPM_FP64 ? 0 : 1];
  k_sum_splits<<<(unsigned)((N + 255) / 256), 256, 0, h->stream>>>(N, h->geo.ncell, P.nsplit, h->wk.Tpart, out);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace spm
