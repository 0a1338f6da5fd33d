// Near-image traction sum (Sec. 4.2, G_near with the 3x3 images of every particle; Sec. 6 Nystrom):
//
//   T_near(x_i) = -(1/pi) sum_j sum_{s in S9} r (r.n_i)(r.f_j) / |r|^4,  r = x_i - (y_j + s),  f_j = w_j sigma_j
//
// for every cell of the ensemble (targets and sources of one cell only). Tiled direct
// N-body in one persistent launch. The work of a cell is cut into units: a block of
// BLOCK * TPT targets against one tile of `tile` sources. The units of the active cells, in
// the order (cell, target block, source tile), are divided evenly over the persistent
// workgroups (workgroup g takes units [g U / G, (g + 1) U / G)). Each workgroup keeps the FP64
// sum of its consecutive tiles of one target block in registers and writes one partial per
// target block it touches: at most (target blocks + workgroups) partials in all, which the
// combine step sums per block in workgroup order (deterministic, no floating-point atomics).
//
// The wave scheduler issues from the oldest ready wave first, so in this issue-bound kernel
// equal shares would finish at very different times (1.6 to 7 ms for one launch measured with
// per-workgroup wall clocks). Each workgroup therefore sets its waves' issue priority from its
// own progress (s_setprio: 3 in the first quarter of its share, down to 0 in the last): a
// workgroup that has fallen behind issues ahead of those that are further along.
//
// Inside a unit: one target per lane (or TPT targets i, i + BLOCK, ...), the source tile
// staged in LDS (every lane of a wave reads the same source: LDS broadcast), the 9 image
// shifts of the cell applied to the source difference, the three images of a lattice row
// sharing their row terms. In FP32 the pair's (r.n)(r.f) is a quadratic in rx whose
// coefficients are formed once per source and row (two fused multiply-adds per image).
#include <algorithm>
#include <type_traits>
#include <mutex>

#include "spm_internal.h"

namespace spm {

template <typename R>
struct Src {
  R y1, y2, f1, f2;
};

// A source of the dilated near set: its wrapped position and force, and the x components of
// its three non-zero image shifts (ms, 0), (0, ns), (ms, ns) and the y component ns.
template <typename R>
struct SrcD {
  R y1, y2, f1, f2, sxA, sxB, sxC, syB;
};

template <typename R, bool DIL>
struct SrcOf {
  typedef Src<R> type;
};
template <typename R>
struct SrcOf<R, true> {
  typedef SrcD<R> type;
};

// Owner of position p of the unit sequence [0, U) divided over G workgroups (the largest g
// with floor(g U / G) <= p).
__host__ __device__ __forceinline__ int64_t unit_owner(int64_t p, int64_t U, int64_t G) {
  return ((p + 1) * G - 1) / U;
}

// One workgroup of 1024 threads (C <= 1024 cells): unit offsets of the active cells
// (inactive cells contribute none), the number of workgroups G = min(grid, U) that share
// them, and for every target block the range of partial slots its owners write.
__global__ __launch_bounds__(1024) void k_near_partition(int C, const int32_t* __restrict__ cell_nt,
                                                         const int32_t* __restrict__ cell_blk,
                                                         const int32_t* __restrict__ active, int grid,
                                                         int64_t* __restrict__ unit_off,
                                                         int32_t* __restrict__ slot_off) {
  __shared__ int64_t s_off[1025];
  __shared__ int32_t s_blk[1025];
  __shared__ int32_t s_nt[1024];
  __shared__ int32_t s_scan[1024];
  __shared__ int32_t s_carry;
  const int t = threadIdx.x;
  if (t < C) s_nt[t] = cell_nt[t];
  if (t < C) s_blk[t] = cell_blk[t];
  if (t == 0) {
    s_blk[C] = cell_blk[C];
    s_off[0] = 0;
    s_carry = 0;
  }
  __syncthreads();
  int64_t u = 0;
  if (t < C && (active == nullptr || active[t] != 0)) u = (int64_t)(s_blk[t + 1] - s_blk[t]) * s_nt[t];
  s_off[t + 1] = u;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {   // inclusive scan of s_off[1..1024]
    const int64_t v = t >= o ? s_off[t + 1 - o] : 0;
    __syncthreads();
    s_off[t + 1] += v;
    __syncthreads();
  }
  if (t < C) unit_off[t] = s_off[t];
  if (t == 0) unit_off[C] = s_off[C];
  const int64_t U = s_off[C];
  const int64_t G = U < grid ? U : grid;
  const int nblocks = s_blk[C];
  for (int base = 0; base < nblocks; base += 1024) {
    const int b = base + t;
    int32_t P = 0;
    if (b < nblocks && U > 0) {
      int lo = 0, hi = C;   // s_blk[lo] <= b < s_blk[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_blk[mid] <= b)
          lo = mid;
        else
          hi = mid;
      }
      const int64_t nt = s_nt[lo];
      if (s_off[lo + 1] > s_off[lo]) {
        const int64_t s = s_off[lo] + (int64_t)(b - s_blk[lo]) * nt;
        P = (int32_t)(unit_owner(s + nt - 1, U, G) - unit_owner(s, U, G) + 1);
      }
    }
    s_scan[t] = P;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive scan
      const int32_t v = t >= o ? s_scan[t - o] : 0;
      __syncthreads();
      s_scan[t] += v;
      __syncthreads();
    }
    if (b < nblocks) slot_off[b] = s_carry + s_scan[t] - P;
    __syncthreads();
    if (t == 1023) s_carry += s_scan[1023];
    __syncthreads();
  }
  if (t == 0) slot_off[nblocks] = s_carry;
}

// One run: targets t0 .. t0 + BLOCK * TPT (clipped at n1) against sources [s_begin, s_end) of
// the cell, in tiles staged through LDS; writes -(1/pi) x the FP64 sum to out[local] and
// out[BLOCK * TPT + local]. TPT targets per lane (i, i + BLOCK, ...) share every LDS source
// read. Each LDS tile is summed in a fresh accumulator of the kernel's precision and then added
// to an FP64 running sum, which keeps the FP32 summation error at the level of one tile. Every
// thread of the workgroup takes part (the tile loop synchronises).
// done0, share: units of the workgroup's share finished before this run and the share's size
// (the issue priority follows done / share). DIL: the dilated near set (Sec. 4.2): x, y are the
// wrapped nodes, and every source has the four images {0, ms} x {0, ns} given by nwrap (two
// lattice rows of two images each) instead of the nine of the 3x3 set.
template <typename R, int BLOCK, int TPT, bool DIL>
__device__ __forceinline__ void near_run(typename SrcOf<R, DIL>::type* src, const R* __restrict__ x,
                                         const R* __restrict__ y, const R* __restrict__ nx,
                                         const R* __restrict__ ny, const R* __restrict__ f1,
                                         const R* __restrict__ f2, const int32_t* __restrict__ nwrap, double skew,
                                         int64_t t0, int64_t n1, int64_t s_begin, int64_t s_end, int tile,
                                         int64_t done0, int64_t share, double* __restrict__ out) {
  constexpr int BT = BLOCK * TPT;
  R sx[kShifts], sy[kShifts];
#pragma unroll
  for (int m = 0; m < kShifts; ++m) {
    sx[m] = (R)shift_x(m, skew);
    sy[m] = (R)shift_y(m);
  }
  R xi[TPT], yi[TPT], nxi[TPT], nyi[TPT];
  double A1[TPT], A2[TPT];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const int64_t i = t0 + threadIdx.x + t * BLOCK;
    xi[t] = 0;
    yi[t] = 0;
    nxi[t] = 0;
    nyi[t] = 0;
    if (i < n1) {
      xi[t] = x[i];
      yi[t] = y[i];
      nxi[t] = nx[i];
      nyi[t] = ny[i];
    }
    A1[t] = 0.0;
    A2[t] = 0.0;
  }
  for (int64_t jt = s_begin; jt < s_end; jt += tile) {
    const int cnt = (int)((jt + tile < s_end) ? tile : (s_end - jt));
    {
      const int64_t level = (4 * (done0 + (jt - s_begin) / tile)) / share;
      if (level <= 0)
        __builtin_amdgcn_s_setprio(3);
      else if (level == 1)
        __builtin_amdgcn_s_setprio(2);
      else if (level == 2)
        __builtin_amdgcn_s_setprio(1);
      else
        __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += BLOCK) {
      typename SrcOf<R, DIL>::type s;
      s.y1 = x[jt + k];
      s.y2 = y[jt + k];
      s.f1 = f1[jt + k];
      s.f2 = f2[jt + k];
      if constexpr (DIL) {
        const int32_t w = nwrap[jt + k];
        const int ms = node_wrap_ms(w), ns = node_wrap_ns(w);
        s.sxA = (R)shift_xmn(ms, 0, skew);
        s.sxB = (R)shift_xmn(0, ns, skew);
        s.sxC = (R)shift_xmn(ms, ns, skew);
        s.syB = (R)ns;
      }
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
      const typename SrcOf<R, DIL>::type s = src[k];
#pragma unroll
      for (int t = 0; t < TPT; ++t) {
        const R dx = xi[t] - s.y1, dy = yi[t] - s.y2;
        // The unshifted image takes dx and dy as they are: its shift (R)shift_xmn(0, 0, skew) is
        // +0 for every skew and x - (+0) == x bit for bit, so the kernels that remove close and
        // own-curve terms with this arithmetic still match it exactly.
        if constexpr (DIL) {
          const RowTerms<R> r0 = row_terms(dy, (R)0, nyi[t], s.f2);
          const RowTerms<R> rB = row_terms(dy, s.syB, nyi[t], s.f2);
          gt_pair(dx, r0, nxi[t], s.f1, a1[t], a2[t]);
          gt_pair(dx - s.sxA, r0, nxi[t], s.f1, a1[t], a2[t]);
          gt_pair(dx - s.sxB, rB, nxi[t], s.f1, a1[t], a2[t]);
          gt_pair(dx - s.sxC, rB, nxi[t], s.f1, a1[t], a2[t]);
        } else if constexpr (std::is_same<R, float>::value) {
          const PairTerms32 pt = pair_terms32(nxi[t], nyi[t], s.f1, s.f2);
          RowTerms32 row[3];
          row[0] = row_terms32<false>(dy, sy[0], pt);
          row[1] = row_terms32<true>(dy, sy[1], pt);
          row[2] = row_terms32<false>(dy, sy[2], pt);
#pragma unroll
          for (int m = 0; m < kShifts; ++m)
            gt_pair32(m == kShifts / 2 ? dx : dx - sx[m], row[m % 3], pt, a1[t], a2[t]);
        } else {
          RowTerms<R> row[3];
#pragma unroll
          for (int n = 0; n < 3; ++n) row[n] = row_terms(dy, sy[n], nyi[t], s.f2);
#pragma unroll
          for (int m = 0; m < kShifts; ++m)
            gt_pair(m == kShifts / 2 ? dx : dx - sx[m], row[m % 3], nxi[t], s.f1, a1[t], a2[t]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
      A1[t] += (double)a1[t];
      A2[t] += (double)a2[t];
    }
  }
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const int local = threadIdx.x + t * BLOCK;
    if (t0 + local < n1) {
      out[local] = -(1.0 / kPi) * A1[t];
      out[BT + local] = -(1.0 / kPi) * A2[t];
    }
  }
}

template <typename R, int BLOCK, int TPT, bool DIL>
__global__ __launch_bounds__(BLOCK) void k_near(int C, const R* __restrict__ x, const R* __restrict__ y,
                                                       const R* __restrict__ nx, const R* __restrict__ ny,
                                                       const R* __restrict__ f1, const R* __restrict__ f2,
                                                       const int32_t* __restrict__ nwrap,
                                                       const double* __restrict__ cskew,
                                                       const int64_t* __restrict__ cnoff,
                                                       const int32_t* __restrict__ cell_nt,
                                                       const int32_t* __restrict__ cell_blk,
                                                       const int64_t* __restrict__ unit_off,
                                                       const int32_t* __restrict__ slot_off, int grid, int tile,
                                                       double* __restrict__ Tpart) {
  extern __shared__ unsigned char smem_raw[];
  typedef typename SrcOf<R, DIL>::type S;
  S* src = reinterpret_cast<S*>(smem_raw);
  constexpr int BT = BLOCK * TPT;
  const int64_t U = unit_off[C];
  const int64_t G = U < grid ? U : grid;
  const int64_t g = blockIdx.x;
  if (g >= G) return;
  const int64_t pbeg = g * U / G;
  const int64_t pend = (g + 1) * U / G;
  int64_t p = pbeg;
  while (p < pend) {
    int lo = 0, hi = C;   // unit_off[lo] <= p < unit_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (unit_off[mid] <= p)
        lo = mid;
      else
        hi = mid;
    }
    const int c = lo;
    const int64_t nt = cell_nt[c];
    const int64_t lu = p - unit_off[c];
    const int64_t bb = lu / nt, k0 = lu - bb * nt;
    const int64_t run = (nt - k0 < pend - p) ? nt - k0 : pend - p;
    const int64_t n0 = cnoff[c], n1 = cnoff[c + 1];
    const int64_t s_end = (n0 + (k0 + run) * tile < n1) ? n0 + (k0 + run) * tile : n1;
    // slot of this workgroup among the owners of target block (c, bb)
    const int64_t first = unit_owner(unit_off[c] + bb * nt, U, G);
    double* out = Tpart + ((int64_t)slot_off[cell_blk[c] + bb] + (g - first)) * 2 * BT;
    near_run<R, BLOCK, TPT, DIL>(src, x, y, nx, ny, f1, f2, nwrap, cskew[c], n0 + bb * BT, n1, n0 + k0 * tile, s_end,
                                 tile, p - pbeg, pend - pbeg, out);
    p += run;
  }
}

// LDS of one workgroup: the source tile, padded when wg_per_cu > 0 so that at most wg_per_cu
// workgroups fit on a compute unit (the grid is then exactly wg_per_cu x compute units).
template <typename R, bool DIL>
static size_t near_lds(int tile, int wg_per_cu) {
  size_t lds = sizeof(typename SrcOf<R, DIL>::type) * (size_t)tile;
  if (wg_per_cu > 0) {
    int dev = 0, per_cu = 0;
    SPM_HIP_CHECK(hipGetDevice(&dev));
    SPM_HIP_CHECK(hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
    const size_t over = (size_t)per_cu / (size_t)(wg_per_cu + 1) + 256;
    if (lds < over) lds = (over + 255) / 256 * 256;
  }
  return lds;
}

template <typename R, int BLOCK, int TPT, bool DIL>
static int near_grid(int tile, int wg_per_cu) {
  const size_t lds = near_lds<R, DIL>(tile, wg_per_cu);
  if (lds > 65536)
    SPM_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_near<R, BLOCK, TPT, DIL>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_near<R, BLOCK, TPT, DIL>, BLOCK, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (wg_per_cu > 0) per_cu = std::min(per_cu, wg_per_cu);
  int dev = 0, ncu = 0;
  SPM_HIP_CHECK(hipGetDevice(&dev));
  SPM_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  return per_cu * ncu;
}

template <typename R, int BLOCK, int TPT, bool DIL>
static void near_launch(spm_handle* h, const R* x, const R* y, const R* nx, const R* ny, const R* f1, const R* f2,
                        const NearPlan& P) {
  const size_t lds = near_lds<R, DIL>(P.cfg.tile, P.cfg.wg_per_cu);
  k_near<R, BLOCK, TPT, DIL><<<P.grid, BLOCK, lds, h->stream>>>(
      h->geo.C, x, y, nx, ny, f1, f2, h->geo.nwrap, h->geo.cskew, h->geo.cnoff, P.cell_nt, P.cell_blk, P.unit_off,
      P.slot_off, P.grid, P.cfg.tile, h->wk.Tpart);
  SPM_HIP_CHECK(hipGetLastError());
}

#define SPM_NEAR_SHAPES(X)                                                                                     \
  X(64, 1) X(64, 2) X(64, 4) X(128, 1) X(128, 2) X(128, 4) X(256, 1) X(256, 2) X(256, 4) X(512, 1) X(512, 2) \
      X(1024, 1) X(1024, 2)

template <typename R, bool DIL>
static void near_dispatch(spm_handle* h, const R* x, const R* y, const R* nx, const R* ny, const R* f1,
                          const R* f2, const NearPlan& P) {
  const int key = P.cfg.block * 10 + P.cfg.tpt;
  switch (key) {
#define SPM_CASE(B, T)                                          \
  case B * 10 + T:                                              \
    near_launch<R, B, T, DIL>(h, x, y, nx, ny, f1, f2, P);      \
    break;
    SPM_NEAR_SHAPES(SPM_CASE)
#undef SPM_CASE
    default: throw ApiError(SPM_EINVAL, "unsupported near-sum launch configuration");
  }
}

template <typename R, bool DIL>
static int near_grid_of(const NearConfig& c) {
  const int key = c.block * 10 + c.tpt;
  switch (key) {
#define SPM_CASE(B, T) \
  case B * 10 + T:     \
    return near_grid<R, B, T, DIL>(c.tile, c.wg_per_cu);
    SPM_NEAR_SHAPES(SPM_CASE)
#undef SPM_CASE
    default: throw ApiError(SPM_EINVAL, "unsupported near-sum launch configuration");
  }
}

int near_persistent_grid(const NearConfig& c, int precision, bool dilated) {
  if (precision == SPM_FP64) return dilated ? near_grid_of<double, true>(c) : near_grid_of<double, false>(c);
  return dilated ? near_grid_of<float, true>(c) : near_grid_of<float, false>(c);
}

bool near_config_valid(const NearConfig& c) {
  const bool b = c.block == 64 || c.block == 128 || c.block == 256 || c.block == 512 || c.block == 1024;
  const bool t = c.tpt == 1 || c.tpt == 2 || (c.tpt == 4 && c.block <= 256);
  return b && t && c.tile >= 16 && c.tile <= 4096 && c.wg_per_cu >= 0 && c.wg_per_cu <= 32;
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
  const NearPlan& P = h->wk.near[kind];
  if (g.C > 1024) throw ApiError(SPM_EINVAL, "at most 1024 cells");
  k_near_partition<<<1, 1024, 0, h->stream>>>(g.C, P.cell_nt, P.cell_blk, with_active ? h->kr.active : nullptr,
                                              P.grid, P.unit_off, P.slot_off);
  SPM_HIP_CHECK(hipGetLastError());
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
  if (precision == SPM_FP64) {
    if (g.dilated)
      near_dispatch<double, true>(h, g.xw, g.yw, g.nx, g.ny, h->wk.f1, h->wk.f2, P);
    else
      near_dispatch<double, false>(h, g.x, g.y, g.nx, g.ny, h->wk.f1, h->wk.f2, P);
  } else {   // the FP32 shadows hold the wrapped nodes with the dilated set
    if (g.dilated)
      near_dispatch<float, true>(h, g.xf, g.yf, g.nxf, g.nyf, h->wk.f1f, h->wk.f2f, P);
    else
      near_dispatch<float, false>(h, g.xf, g.yf, g.nxf, g.nyf, h->wk.f1f, h->wk.f2f, P);
  }
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

// ----------------------------------------------------------------------------
// Allocation-free near sum of one cell (spm_near_traction_noalloc). Its forces, FP32
// shadows, plan and partials live in one file-scope device array (`scratch`, kNoallocBytes)
// instead of handle memory; a fixed launch shape, the handle's default one (64 threads, one target
// per lane, 128-source tiles, so that both entry points round the FP32 tile sums alike), and at
// most kNoallocGrid workgroups bound the partials. Host code reaches the array
// through the per-device address hipGetSymbolAddress returns, never through its name.
// ----------------------------------------------------------------------------
namespace {
constexpr int64_t kNoallocMaxN = SPM_NOALLOC_MAX_N;
constexpr int kNoallocBlock = 64, kNoallocTile = 128, kNoallocGrid = 8192;
constexpr int64_t kNoallocBlocks = kNoallocMaxN / kNoallocBlock;
constexpr int64_t kNoallocSlots = kNoallocBlocks + kNoallocGrid;
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kOffF64 = 0;                                                   // f1, f2 [2 maxN] double
constexpr size_t kOffF32 = kOffF64 + align256(2 * kNoallocMaxN * sizeof(double));   // x y nx ny f1 f2 [6 maxN] float
constexpr size_t kOffPlan = kOffF32 + align256(6 * kNoallocMaxN * sizeof(float));
// plan: cskew [1] double, cnoff [2] int64, unit_off [2] int64, cell_nt [1], cell_blk [2], slot_off [blocks + 1] int32
constexpr size_t kOffSlot = kOffPlan + 64;
constexpr size_t kOffPart = kOffSlot + align256((kNoallocBlocks + 1) * sizeof(int32_t));
constexpr size_t kNoallocBytes = kOffPart + kNoallocSlots * 2 * kNoallocBlock * sizeof(double);
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// forces f = w sigma, the FP32 shadows (FP32 precision) and the one-cell plan
__global__ __launch_bounds__(256) void k_noalloc_prep(int64_t N, double skew, const double* __restrict__ x,
                                                      const double* __restrict__ y, const double* __restrict__ nx,
                                                      const double* __restrict__ ny, const double* __restrict__ w,
                                                      const double* __restrict__ sigma, int fp32,
                                                      unsigned char* __restrict__ base) {
  double* f1 = reinterpret_cast<double*>(base + kOffF64);
  double* f2 = f1 + kNoallocMaxN;
  float* xf = reinterpret_cast<float*>(base + kOffF32);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N) {
    const double a = w[i] * sigma[i], b = w[i] * sigma[N + i];
    f1[i] = a;
    f2[i] = b;
    if (fp32) {
      xf[i] = (float)x[i];
      xf[kNoallocMaxN + i] = (float)y[i];
      xf[2 * kNoallocMaxN + i] = (float)nx[i];
      xf[3 * kNoallocMaxN + i] = (float)ny[i];
      xf[4 * kNoallocMaxN + i] = (float)a;
      xf[5 * kNoallocMaxN + i] = (float)b;
    }
  }
  if (i == 0) {
    unsigned char* plan = base + kOffPlan;
    reinterpret_cast<double*>(plan)[0] = skew;
    int64_t* cnoff = reinterpret_cast<int64_t*>(plan + 8);
    cnoff[0] = 0;
    cnoff[1] = N;
    int32_t* ints = reinterpret_cast<int32_t*>(plan + 40);
    ints[0] = (int32_t)((N + kNoallocTile - 1) / kNoallocTile);      // cell_nt
    ints[1] = 0;                                                      // cell_blk
    ints[2] = (int32_t)((N + kNoallocBlock - 1) / kNoallocBlock);
  }
}

// out[i] = sum of the partial slots of target i's block (one cell)
__global__ __launch_bounds__(256) void k_noalloc_sum(int64_t N, const unsigned char* __restrict__ base,
                                                     double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int32_t* slot_off = reinterpret_cast<const int32_t*>(base + kOffSlot);
  const double* part = reinterpret_cast<const double*>(base + kOffPart);
  const int64_t b = i / kNoallocBlock, local = i % kNoallocBlock;
  double t1 = 0.0, t2 = 0.0;
  for (int k = slot_off[b]; k < slot_off[b + 1]; ++k) {
    t1 += part[(int64_t)k * 2 * kNoallocBlock + local];
    t2 += part[(int64_t)k * 2 * kNoallocBlock + kNoallocBlock + local];
  }
  out[i] = t1;
  out[N + i] = t2;
}

namespace {
struct NoallocDevice {
  unsigned char* ptr = nullptr;   // device address of `scratch` on this device
  int grid = 0;
};
std::mutex g_noalloc_mu;
NoallocDevice g_noalloc_dev[64];

template <typename R>
void noalloc_launch(hipStream_t st, int64_t N, const R* x, const R* y, const R* nx, const R* ny, const R* f1,
                    const R* f2, unsigned char* base, int grid) {
  unsigned char* plan = base + kOffPlan;
  const double* cskew = reinterpret_cast<const double*>(plan);
  const int64_t* cnoff = reinterpret_cast<const int64_t*>(plan + 8);
  int64_t* unit_off = reinterpret_cast<int64_t*>(plan + 24);
  const int32_t* cell_nt = reinterpret_cast<const int32_t*>(plan + 40);
  const int32_t* cell_blk = cell_nt + 1;
  int32_t* slot_off = reinterpret_cast<int32_t*>(base + kOffSlot);
  double* part = reinterpret_cast<double*>(base + kOffPart);
  k_near_partition<<<1, 1024, 0, st>>>(1, cell_nt, cell_blk, nullptr, grid, unit_off, slot_off);
  SPM_HIP_CHECK(hipGetLastError());
  k_near<R, kNoallocBlock, 1, false><<<grid, kNoallocBlock, sizeof(Src<R>) * kNoallocTile, st>>>(
      1, x, y, nx, ny, f1, f2, nullptr, cskew, cnoff, cell_nt, cell_blk, unit_off, slot_off, grid, kNoallocTile, part);
  SPM_HIP_CHECK(hipGetLastError());
}
}  // namespace

}  // namespace spm

using namespace spm;

extern "C" int spm_near_traction_noalloc(void* hip_stream, int64_t n, double skew, const double* x, const double* y,
                                         const double* nx, const double* ny, const double* w, const double* sigma,
                                         int32_t precision, double* out) {
  if (n < 1 || n > kNoallocMaxN) return SPM_EINVAL;
  if (!x || !y || !nx || !ny || !w || !sigma || !out || !std::isfinite(skew)) return SPM_EINVAL;
  if (precision != SPM_FP64 && precision != SPM_FP32) return SPM_EINVAL;
  try {
    int dev = 0;
    SPM_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return SPM_EINVAL;
    NoallocDevice D;
    {
      std::lock_guard<std::mutex> lock(g_noalloc_mu);
      NoallocDevice& d = g_noalloc_dev[dev];
      if (!d.ptr) {   // first call on this device (which is current): the array's device address
        void* p = nullptr;
        SPM_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return SPM_EHIP;
        NearConfig c;
        c.block = kNoallocBlock;
        c.tpt = 1;
        c.tile = kNoallocTile;
        c.wg_per_cu = 0;
        const int g64 = near_persistent_grid(c, SPM_FP64, false), g32 = near_persistent_grid(c, SPM_FP32, false);
        d.grid = std::max(1, std::min(kNoallocGrid, std::min(g64, g32)));
        d.ptr = static_cast<unsigned char*>(p);
      }
      D = d;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const double s = skew - std::floor(skew + 0.5);   // e2 = (s, 1) reduced to [-1/2, 1/2)
    const unsigned g = (unsigned)((n + 255) / 256);
    k_noalloc_prep<<<g, 256, 0, st>>>(n, s, x, y, nx, ny, w, sigma, precision == SPM_FP32 ? 1 : 0, D.ptr);
    SPM_HIP_CHECK(hipGetLastError());
    if (precision == SPM_FP64) {
      const double* f1 = reinterpret_cast<const double*>(D.ptr + kOffF64);
      noalloc_launch<double>(st, n, x, y, nx, ny, f1, f1 + kNoallocMaxN, D.ptr, D.grid);
    } else {
      const float* xf = reinterpret_cast<const float*>(D.ptr + kOffF32);
      noalloc_launch<float>(st, n, xf, xf + kNoallocMaxN, xf + 2 * kNoallocMaxN, xf + 3 * kNoallocMaxN,
                            xf + 4 * kNoallocMaxN, xf + 5 * kNoallocMaxN, D.ptr, D.grid);
    }
    k_noalloc_sum<<<g, 256, 0, st>>>(n, D.ptr, out);
    SPM_HIP_CHECK(hipGetLastError());
    SPM_HIP_CHECK(hipStreamSynchronize(st));
    return SPM_OK;
  } catch (const HipError&) {
    return SPM_EHIP;
  } catch (const ApiError& e) {
    return e.code;
  }
}
