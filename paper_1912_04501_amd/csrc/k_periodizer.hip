// Periodizing correction by proxy Stokeslets (Sec. 4.2; Sec. 6.1 MFS; Sec. 6.2 four steps).
//
// Walls: L(t) = c_U - e1/2 + t e2, D(t) = c_U - e2/2 + t e1 at m Gauss-Legendre points;
// R = L + e1, U = D + e2; normals n_L = (e2_2, -e2_1)/|e2|, n_D = (0, 1) on both walls of a pair.
// Discrepancy rows (length 8m): [u_R-u_L (2m); T_R-T_L (2m); u_U-u_D (2m); T_U-T_D (2m)],
// each block ordered first components then second components.
// Jump target: g0 = [0; -F/(2|e2|); 0; -F/(2|e1|)], F = sum_j f_j (net force balance of the cell).
// xi = Q^+ (g0 - g): [xi_1 (M); xi_2 (M)].
#include "spm_internal.h"

namespace spm {

// Stokeslet velocity G(r) f (eq. Gv) and traction G^t(r; n) f (eq. Gt), r = x - y.
__device__ __forceinline__ void stokeslet_uv(double rx, double ry, double f1, double f2, double inv4pimu,
                                             double& u1, double& u2) {
  const double r2 = rx * rx + ry * ry;
  const double ir2 = rcp64(r2);
  const double lg = -0.5 * log(r2);
  const double rf = (rx * f1 + ry * f2) * ir2;
  u1 += inv4pimu * (lg * f1 + rx * rf);
  u2 += inv4pimu * (lg * f2 + ry * rf);
}

// G(r_a) f - G(r_b) f with the two logarithms taken as one: -log|r_a| + log|r_b| = -(1/2) log(|r_a|^2 / |r_b|^2).
__device__ __forceinline__ void stokeslet_diff_uv(double ax, double ay, double bx, double by, double f1, double f2,
                                                  double inv4pimu, double& d1, double& d2) {
  const double a2 = ax * ax + ay * ay, b2 = bx * bx + by * by;
  const double ia2 = rcp64(a2), ib2 = rcp64(b2);
  const double lg = -0.5 * log(a2 * ib2);
  const double af = (ax * f1 + ay * f2) * ia2, bf = (bx * f1 + by * f2) * ib2;
  d1 = inv4pimu * (lg * f1 + (ax * af - bx * bf));
  d2 = inv4pimu * (lg * f2 + (ay * af - by * bf));
}

__device__ __forceinline__ void traction_uv(double rx, double ry, double nx, double ny, double f1, double f2,
                                            double& t1, double& t2) {
  const double r2 = rx * rx + ry * ry;
  const double ir2 = rcp64(r2);
  const double c = -(1.0 / kPi) * (rx * nx + ry * ny) * (rx * f1 + ry * f2) * ir2 * ir2;
  t1 += c * rx;
  t2 += c * ry;
}

struct Lat {
  double inv4pimu;
  int m, M;
};

static Lat lattice_args(spm_handle* h) {
  Lat L;
  L.inv4pimu = 1.0 / (4.0 * kPi * h->cfg.mu);
  L.m = h->per.m;
  L.M = h->per.M;
  return L;
}

// Lattice of a cell: e1 = (1, 0), e2 = (skew, 1); wall normals n_L = (e2_2, -e2_1)/|e2|, n_D = (0, 1).
struct CellLat {
  double e2x, nLx, nLy;
};
__device__ __forceinline__ CellLat cell_lat(double skew) {
  const double l2 = sqrt(skew * skew + 1.0);
  return {skew, 1.0 / l2, -skew / l2};
}

// Q[row][col], row in [0, 8m), col = comp * M + p: the wall jumps of the field of a unit
// force e_comp at proxy p.
__global__ void k_build_Q(Lat L, const double* __restrict__ cskew, const double* __restrict__ wx_all,
                          const double* __restrict__ wy_all, const double* __restrict__ px_all,
                          const double* __restrict__ py_all, double* __restrict__ Q_all) {
  const int m = L.m, M = L.M;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 8 * m * 2 * M) return;
  const int cell = blockIdx.y;
  const CellLat CL = cell_lat(cskew[cell]);
  const double* wx = wx_all + (int64_t)cell * 2 * m;
  const double* wy = wy_all + (int64_t)cell * 2 * m;
  const double* px = px_all + (int64_t)cell * M;
  const double* py = py_all + (int64_t)cell * M;
  double* Q = Q_all + (int64_t)cell * 8 * m * 2 * M;
  const int row = idx / (2 * M), col = idx % (2 * M);
  const int comp = col / M, p = col % M;
  const int blk = row / m, q = row % m;       // blk: 0,1 u on L; 2,3 T on L; 4,5 u on D; 6,7 T on D
  const bool onD = blk >= 4;
  const int kind = (blk % 4) / 2;              // 0 velocity, 1 traction
  const int outc = blk % 2;                    // output component
  const double x0 = wx[onD ? m + q : q], y0 = wy[onD ? m + q : q];
  const double sx = onD ? CL.e2x : 1.0, sy = onD ? 1.0 : 0.0;
  const double nx = onD ? 0.0 : CL.nLx, ny = onD ? 1.0 : CL.nLy;
  const double f1 = comp == 0 ? 1.0 : 0.0, f2 = comp == 1 ? 1.0 : 0.0;
  double a1 = 0, a2 = 0, b1 = 0, b2 = 0;
  if (kind == 0) {
    stokeslet_uv(x0 + sx - px[p], y0 + sy - py[p], f1, f2, L.inv4pimu, a1, a2);
    stokeslet_uv(x0 - px[p], y0 - py[p], f1, f2, L.inv4pimu, b1, b2);
  } else {
    traction_uv(x0 + sx - px[p], y0 + sy - py[p], nx, ny, f1, f2, a1, a2);
    traction_uv(x0 - px[p], y0 - py[p], nx, ny, f1, f2, b1, b2);
  }
  Q[idx] = outc == 0 ? (a1 - b1) : (a2 - b2);
}

void launch_build_Q(spm_handle* h) {
  const Lat L = lattice_args(h);
  const int n = 8 * L.m * 2 * L.M;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)h->geo.C);
  k_build_Q<<<grid, 256, 0, h->stream>>>(L, h->geo.cskew, h->per.wx, h->per.wy, h->per.px, h->per.py, h->per.Q);
  SPM_HIP_CHECK(hipGetLastError());
}

// ----------------------------------------------------------------------------
// Pseudo-inverse of Q by one-sided (Hestenes) Jacobi SVD in one workgroup.
// A = Q (rows x ncol, column-major copy) is orthogonalised column pair by column pair,
// A V = U S; round-robin pairing gives ncol/2 disjoint pairs per round, one group of
// G = blockDim/(ncol/2) lanes per pair. The three smallest singular triplets (the
// gauge modes of the empty-box problem: constant velocity and pressure) and any
// singular value below rcond * s_max are dropped:  Q^+ = sum_k v_k u_k^T / s_k.
// ----------------------------------------------------------------------------
// One-sided Jacobi SVD of Q (rows x ncol) per cell, one workgroup per cell: columns of
// A = Q V are rotated in pairs until mutually orthogonal; then s_k = |A_k|, u_k = A_k / s_k.
// Pairs follow the circle method (column 0 fixed, the others rotate by one position per
// round), so each round rotates ncol/2 disjoint pairs in parallel. A warm start begins from
// the previous V of the same cell (A = Q V_prev): any orthogonal start converges to the
// SVD, and for the slowly changing lattice of a time step it needs few sweeps.
// LDS_RES: A and V live in LDS for the whole iteration (rows*ncol + ncol^2 <= kJacobiLds).
constexpr int kJacobiLds = 16384;   // doubles (128 KiB)

__device__ __forceinline__ int circle_col(int k, int round, int n) {
  return k == 0 ? 0 : 1 + ((k - 1 - round) % (n - 1) + (n - 1)) % (n - 1);
}

template <bool LDS_RES>
__global__ __launch_bounds__(1024) void k_jacobi(int rows, int ncol, const double* __restrict__ Q_all,
                                                 double* __restrict__ A_all, double* __restrict__ V_all,
                                                 double* __restrict__ S_all, int max_sweeps, int warm) {
  __shared__ double lds[LDS_RES ? kJacobiLds : 1];
  __shared__ double offmax[1024];
  const int cell = blockIdx.x;
  const double* Q = Q_all + (int64_t)cell * rows * ncol;
  double* Ag = A_all + (int64_t)cell * rows * ncol;
  double* Vg = V_all + (int64_t)cell * ncol * ncol;
  double* S = S_all + (int64_t)cell * (ncol + 1);
  double* A = LDS_RES ? lds : Ag;
  double* V = LDS_RES ? lds + rows * ncol : Vg;
  const int tid = threadIdx.x, nt = blockDim.x;
  // V(:, c) is stored contiguously: V[c * ncol + i]
  if (warm) {
    if (LDS_RES)
      for (int k = tid; k < ncol * ncol; k += nt) V[k] = Vg[k];
    __syncthreads();
    for (int k = tid; k < rows * ncol; k += nt) {
      const int c = k / rows, r = k % rows;
      double a = 0.0;
      for (int i = 0; i < ncol; ++i) a += Q[r * ncol + i] * V[c * ncol + i];
      A[k] = a;
    }
  } else {
    for (int k = tid; k < rows * ncol; k += nt) {
      const int r = k / ncol, c = k % ncol;
      A[c * rows + r] = Q[k];
    }
    for (int k = tid; k < ncol * ncol; k += nt) V[k] = (k / ncol == k % ncol) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int npair = ncol / 2;
  const int G = nt / npair;  // lanes per pair (power of two, <= 64)
  const int pair = tid / G, gl = tid % G;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    double local_off = 0.0;
    for (int round = 0; round < ncol - 1; ++round) {
      if (pair < npair) {
        const int cp = circle_col(pair, round, ncol), cq = circle_col(ncol - 1 - pair, round, ncol);
        const int p = cp < cq ? cp : cq, q = cp < cq ? cq : cp;
        double al = 0, be = 0, ga = 0;
        for (int r = gl; r < rows; r += G) {
          const double ap = A[p * rows + r], aq = A[q * rows + r];
          al += ap * ap;
          be += aq * aq;
          ga += ap * aq;
        }
        for (int o = G / 2; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, G);
          be += __shfl_xor(be, o, G);
          ga += __shfl_xor(ga, o, G);
        }
        const double nrm = sqrt(al * be);
        if (nrm > 0.0 && fabs(ga) > 1e-15 * nrm) {
          const double rel = fabs(ga) / nrm;
          local_off = rel > local_off ? rel : local_off;
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          for (int r = gl; r < rows; r += G) {
            const double ap = A[p * rows + r], aq = A[q * rows + r];
            A[p * rows + r] = c * ap - s * aq;
            A[q * rows + r] = s * ap + c * aq;
          }
          for (int r = gl; r < ncol; r += G) {
            const double vp = V[p * ncol + r], vq = V[q * ncol + r];
            V[p * ncol + r] = c * vp - s * vq;
            V[q * ncol + r] = s * vp + c * vq;
          }
        }
      }
      __syncthreads();
    }
    offmax[tid] = local_off;
    __syncthreads();
    for (int o = nt / 2; o > 0; o >>= 1) {
      if (tid < o) offmax[tid] = offmax[tid + o] > offmax[tid] ? offmax[tid + o] : offmax[tid];
      __syncthreads();
    }
    const bool done = offmax[0] <= 1e-15;
    __syncthreads();
    if (done) break;
  }
  if (LDS_RES) {
    for (int k = tid; k < rows * ncol; k += nt) Ag[k] = A[k];
    for (int k = tid; k < ncol * ncol; k += nt) Vg[k] = V[k];
  }
  for (int c = tid; c < ncol; c += nt) {
    double s = 0;
    for (int r = 0; r < rows; ++r) s += A[c * rows + r] * A[c * rows + r];
    S[c] = sqrt(s);
  }
  if (tid == 0) S[ncol] = (double)sweep;
}

// Qp[i][r] = sum_{k kept} V[k][i] A[k][r] / s_k^2  (u_k = A_k / s_k)
__global__ void k_pinv_assemble(int rows, int ncol, const double* __restrict__ A_all,
                                const double* __restrict__ V_all, const double* __restrict__ S_all, double rcond,
                                int n_gauge, double* __restrict__ Qp_all) {
  const int cell = blockIdx.y;
  const double* A = A_all + (int64_t)cell * rows * ncol;
  const double* V = V_all + (int64_t)cell * ncol * ncol;
  const double* S = S_all + (int64_t)cell * (ncol + 1);
  double* Qp = Qp_all + (int64_t)cell * rows * ncol;
  __shared__ double w[1024];
  if (threadIdx.x == 0) {
    double smax = 0;
    for (int k = 0; k < ncol; ++k) smax = S[k] > smax ? S[k] : smax;
    // the n_gauge smallest are the gauge modes, dropped whether or not they fall below the
    // cutoff; then every other value at or below rcond * s_max
    for (int k = 0; k < ncol; ++k) w[k] = 1.0;
    for (int g = 0; g < n_gauge; ++g) {
      int arg = -1;
      double best = 1e300;
      for (int k = 0; k < ncol; ++k)
        if (w[k] != 0.0 && S[k] < best) {
          best = S[k];
          arg = k;
        }
      if (arg >= 0) w[arg] = 0.0;
    }
    for (int k = 0; k < ncol; ++k) w[k] = (w[k] != 0.0 && S[k] > rcond * smax) ? 1.0 / (S[k] * S[k]) : 0.0;
  }
  __syncthreads();
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncol * rows) return;
  const int i = idx / rows, r = idx % rows;
  double s = 0;
  for (int k = 0; k < ncol; ++k)
    if (w[k] != 0.0) s += V[k * ncol + i] * A[k * rows + r] * w[k];
  Qp[idx] = s;
}

void launch_pinv(spm_handle* h) {
  const int rows = 8 * h->per.m, ncol = 2 * h->per.M;
  const int npair = ncol / 2;
  int G = 1;
  while (G * 2 * npair <= 1024 && G < 64) G *= 2;
  const int nt = G * npair;
  const int warm = h->per.warm_ok ? 1 : 0;
  if ((int64_t)rows * ncol + (int64_t)ncol * ncol <= kJacobiLds)
    k_jacobi<true><<<h->geo.C, nt, 0, h->stream>>>(rows, ncol, h->per.Q, h->per.svd_a, h->per.svd_v, h->per.svd_s,
                                                    60, warm);
  else
    k_jacobi<false><<<h->geo.C, nt, 0, h->stream>>>(rows, ncol, h->per.Q, h->per.svd_a, h->per.svd_v,
                                                     h->per.svd_s, 60, warm);
  SPM_HIP_CHECK(hipGetLastError());
  h->per.warm_ok = true;
  const int n = rows * ncol;
  // every block recomputes the truncation weights of its cell (cheap, ncol <= 1024)
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)h->geo.C);
  k_pinv_assemble<<<grid, 256, 0, h->stream>>>(rows, ncol, h->per.svd_a, h->per.svd_v, h->per.svd_s, h->cfg.rcond, 3,
                                               h->per.Qp);
  SPM_HIP_CHECK(hipGetLastError());
}

// ----------------------------------------------------------------------------
// Wall discrepancy (step 2), telescoped: at a point x_L of L,
//   u_near(x_L+e1) - u_near(x_L) = sum_j sum_{n=-1..1} [G(x_L, y_j - 2e1 + n e2) - G(x_L, y_j + e1 + n e2)] f_j
// and on D with the roles of e1, e2 exchanged; the same with G^t(.; n_wall).
// Grid (chunks, 2m): block (c, w) sums its source chunk for wall point w in double-double
// (the result is small against the sum of the terms' sizes and Q+ amplifies its rounding);
// partials disc[c][w][8] = (du1, du2, dT1, dT2) hi parts then lo parts, summed in fixed
// order by k_xi.
// ----------------------------------------------------------------------------
//
// Dilated near set (nwrap given; x, y the wrapped nodes): a node's images are the shifts
// {0, ms} x {0, ns}. Across the wall pair with lattice vector a (e1 for L/R, e2 for D/U) the
// images are i a with i in I = {0, s_a}; shifting the target by a maps them to i - 1, so the
// jump is, for each image position j along the wall, G(x, y + (min I - 1) a + j b) -
// G(x, y + (max I) a + j b), j in {0, s_b}: two far-minus-near pairs per node, each image at
// least half a cell from the wall.
__global__ __launch_bounds__(256) void k_disc(int64_t N, Lat L, const double* __restrict__ cskew,
                                              const double* __restrict__ wx_all, const double* __restrict__ wy_all,
                                              const double* __restrict__ x, const double* __restrict__ y,
                                              const double* __restrict__ f1, const double* __restrict__ f2,
                                              const int32_t* __restrict__ nwrap,
                                              const int64_t* __restrict__ cs0, const int64_t* __restrict__ cs1,
                                              const int32_t* __restrict__ ccell, const int32_t* __restrict__ active,
                                              double* __restrict__ disc) {
  __shared__ double sc[32];
  const int chunk = blockIdx.x;
  const int wpt = blockIdx.y;
  const int cell = ccell[chunk];
  if (active != nullptr && active[cell] == 0) return;
  const CellLat CL = cell_lat(cskew[cell]);
  const bool onD = wpt >= L.m;
  const double x0 = wx_all[(int64_t)cell * 2 * L.m + wpt], y0 = wy_all[(int64_t)cell * 2 * L.m + wpt];
  const double nx = onD ? 0.0 : CL.nLx, ny = onD ? 1.0 : CL.nLy;
  // far column/row (-2 along the lattice vector across the wall pair) minus the near one (+1)
  const double ax_ = onD ? CL.e2x : 1.0, ay_ = onD ? 1.0 : 0.0;   // across the wall pair
  const double bx_ = onD ? 1.0 : CL.e2x, by_ = onD ? 0.0 : 1.0;   // along the wall
  const int64_t j0 = cs0[chunk], j1 = cs1[chunk];
  dd u1 = {0, 0}, u2 = {0, 0}, t1 = {0, 0}, t2 = {0, 0};
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const double yj = x[j], zj = y[j], g1 = f1[j], g2 = f2[j];
    // 3x3 set: far image -2 a, near image +a, rows n = -1, 0, 1 along the wall;
    // dilated set: far (min I - 1) a, near (max I) a, rows {0, s_b}
    int far = -2, near = 1, nlo = -1, nhi = 1, nstep = 1;
    if (nwrap != nullptr) {
      const int32_t w = nwrap[j];
      const int sa = onD ? node_wrap_ns(w) : node_wrap_ms(w), sb = onD ? node_wrap_ms(w) : node_wrap_ns(w);
      far = sa > 0 ? -1 : -2;
      near = sa > 0 ? 1 : 0;
      nlo = sb > 0 ? 0 : -1;
      nhi = sb > 0 ? 1 : 0;
    }
    // the rows of one source: their logarithms combine into one of the product of the squared-distance
    // ratios, and the source's far-minus-near differences (all rows) are rounded once into the
    // double-double sums
    double ratio = 1.0, s1 = 0.0, s2 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int n = nlo; n <= nhi; n += nstep) {
      const double ax = x0 - (yj + far * ax_ + n * bx_), ay = y0 - (zj + far * ay_ + n * by_);
      const double bxn = x0 - (yj + near * ax_ + n * bx_), byn = y0 - (zj + near * ay_ + n * by_);
      const double a2 = ax * ax + ay * ay, b2 = bxn * bxn + byn * byn;
      const double ia2 = rcp64(a2), ib2 = rcp64(b2);
      ratio *= a2 * ib2;
      const double af = (ax * g1 + ay * g2) * ia2, bf = (bxn * g1 + byn * g2) * ib2;
      s1 += ax * af - bxn * bf;
      s2 += ay * af - byn * bf;
      const double cf = (ax * nx + ay * ny) * af * ia2, cn = (bxn * nx + byn * ny) * bf * ib2;
      p1 += cf * ax - cn * bxn;
      p2 += cf * ay - cn * byn;
    }
    const double lg = -0.5 * log(ratio);
    u1 = dd_add_d(u1, L.inv4pimu * (lg * g1 + s1));
    u2 = dd_add_d(u2, L.inv4pimu * (lg * g2 + s2));
    t1 = dd_add_d(t1, -(1.0 / kPi) * p1);
    t2 = dd_add_d(t2, -(1.0 / kPi) * p2);
  }
  u1 = dd_block_sum(u1, sc);
  u2 = dd_block_sum(u2, sc);
  t1 = dd_block_sum(t1, sc);
  t2 = dd_block_sum(t2, sc);
  if (threadIdx.x == 0) {
    double* o = disc + ((int64_t)chunk * 2 * L.m + wpt) * 8;
    o[0] = u1.hi;
    o[1] = u2.hi;
    o[2] = t1.hi;
    o[3] = t2.hi;
    o[4] = u1.lo;
    o[5] = u2.lo;
    o[6] = t1.lo;
    o[7] = t2.lo;
  }
}

void launch_disc_impl(spm_handle* h, bool with_active) {
  const Lat L = lattice_args(h);
  dim3 grid((unsigned)h->wk.ndisc, (unsigned)(2 * L.m));
  const Geo& g = h->geo;
  k_disc<<<grid, 256, 0, h->stream>>>(g.N, L, g.cskew, h->per.wx, h->per.wy, g.dilated ? g.xw : g.x,
                                      g.dilated ? g.yw : g.y, h->wk.f1, h->wk.f2, g.dilated ? g.nwrap : nullptr,
                                      h->wk.disc_s0, h->wk.disc_s1, h->wk.disc_cell,
                                      with_active ? h->kr.active : nullptr, h->wk.disc);
  SPM_HIP_CHECK(hipGetLastError());
}

void launch_disc(spm_handle* h) { launch_disc_impl(h, false); }

// One block per cell: g = sum of the cell's chunk partials, F = sum of its particles'
// forces, xi = Q^+ (g0 - g). Every double-double sum runs along one thread (no cross-lane
// reductions, which cost far more issue slots than the sums themselves): one thread per
// (wall point, component) over the chunks in order, then one thread per segment of a row of
// Q^+, the segment partials of a row summed in order by one thread.
constexpr int kXiThreads = 1024, kXiBatch = 8;
__global__ __launch_bounds__(kXiThreads) void k_xi(Lat L, const double* __restrict__ cskew, const int32_t* __restrict__ disc_off,
                     const int32_t* __restrict__ cpoff, const double* __restrict__ disc, const double* __restrict__ pF,
                     const double* __restrict__ Qp_all, const int32_t* __restrict__ active, double* __restrict__ xi_all) {
  __shared__ double gt[8 * 256];
  __shared__ double part[2 * kXiThreads];   // segment partials (hi, lo) of the rows of Q+
  __shared__ double Fs[2];
  const int cell = blockIdx.x;
  if (active != nullptr && active[cell] == 0) return;
  const int m = L.m, M = L.M;
  const double* Qp = Qp_all + (int64_t)cell * 2 * M * 8 * m;
  double* xi = xi_all + (int64_t)cell * 2 * M;
  {
    __shared__ double sc[32];
    dd F1 = {0, 0}, F2 = {0, 0};
    for (int q = cpoff[cell] + threadIdx.x; q < cpoff[cell + 1]; q += blockDim.x) {
      F1 = dd_add_d(F1, pF[4 * q + 0]);
      F2 = dd_add_d(F2, pF[4 * q + 1]);
    }
    F1 = dd_block_sum(F1, sc);
    F2 = dd_block_sum(F2, sc);
    if (threadIdx.x == 0) {
      Fs[0] = F1.hi + F1.lo;
      Fs[1] = F2.hi + F2.lo;
    }
  }
  __syncthreads();
  const double skew = cskew[cell];
  const double l1 = 1.0, l2 = sqrt(skew * skew + 1.0);
  // g0 - g at wall point wpt, component k (thread t = 4 wpt + k: neighbouring threads read
  // neighbouring words of a chunk's partials)
  const int c0 = disc_off[cell], c1 = disc_off[cell + 1];
  for (int t = threadIdx.x; t < 8 * m; t += blockDim.x) {
    const int wpt = t >> 2, k = t & 3;
    dd sum = {0, 0};
    int c = c0;
    for (; c + kXiBatch <= c1; c += kXiBatch) {   // the batch's loads in flight together
      double hi[kXiBatch], lo[kXiBatch];
#pragma unroll
      for (int u = 0; u < kXiBatch; ++u) {
        const double* o = disc + ((int64_t)(c + u) * 2 * m + wpt) * 8;
        hi[u] = o[k];
        lo[u] = o[4 + k];
      }
#pragma unroll
      for (int u = 0; u < kXiBatch; ++u) sum = dd_add(sum, dd{hi[u], lo[u]});
    }
    for (; c < c1; ++c) {
      const double* o = disc + ((int64_t)c * 2 * m + wpt) * 8;
      sum = dd_add(sum, dd{o[k], o[4 + k]});
    }
    const bool onD = wpt >= m;
    const int q = onD ? wpt - m : wpt;
    const int base = onD ? 4 * m : 0;
    const double l = onD ? l1 : l2;
    const double g0 = k < 2 ? 0.0 : -Fs[k - 2] / (2.0 * l);
    const dd v = dd_add(dd{g0, 0.0}, dd{-sum.hi, -sum.lo});   // g0 - g, rounded once
    gt[base + k * m + q] = v.hi + v.lo;
  }
  __syncthreads();
  // rows of Q+: S segments per row (2M S <= threads), compensated dot products
  const int rows = 2 * M, n8 = 8 * m;
  const int S = rows >= kXiThreads ? 1 : kXiThreads / rows;
  const int seg = (n8 + S - 1) / S;
  for (int t = threadIdx.x; t < rows * S; t += blockDim.x) {
    const int i = t / S, j = t - i * S;
    const int r0 = j * seg, r1 = min(n8, r0 + seg);
    const double* qrow = Qp + (int64_t)i * n8;
    dd sum = {0, 0};
    int r = r0;
    for (; r + kXiBatch <= r1; r += kXiBatch) {
      double qv[kXiBatch];
#pragma unroll
      for (int u = 0; u < kXiBatch; ++u) qv[u] = qrow[r + u];
#pragma unroll
      for (int u = 0; u < kXiBatch; ++u) sum = dd_fma(sum, qv[u], gt[r + u]);
    }
    for (; r < r1; ++r) sum = dd_fma(sum, qrow[r], gt[r]);
    part[2 * t] = sum.hi;
    part[2 * t + 1] = sum.lo;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < rows; i += blockDim.x) {
    dd sum = {0, 0};
    for (int j = 0; j < S; ++j) sum = dd_add(sum, dd{part[2 * (i * S + j)], part[2 * (i * S + j) + 1]});
    xi[i] = sum.hi + sum.lo;
  }
}

void launch_xi_impl(spm_handle* h, bool with_active) {
  const Lat L = lattice_args(h);
  k_xi<<<h->geo.C, 1024, 0, h->stream>>>(L, h->geo.cskew, h->wk.disc_off, h->geo.cpoff, h->wk.disc, h->wk.pF,
                                        h->per.Qp, with_active ? h->kr.active : nullptr, h->wk.xi);
  SPM_HIP_CHECK(hipGetLastError());
}

void launch_xi(spm_handle* h) { launch_xi_impl(h, false); }

// ----------------------------------------------------------------------------
// Combine: T_i = sum of near-sum split partials + self term + proxy correction.
// Self term (limit of the smooth kernel on the curve): -(kappa/2pi) tau (tau . w sigma).
// Proxy correction (step 4): sum_p G^t(x_i, y_p; n_i) xi_p.
// ----------------------------------------------------------------------------
// Four lanes per target: lane l sums the partial slots k = l, l+4, ... of the target's block
// and the proxies p = l, l+4, ...; the four partial sums are combined by a fixed butterfly
// (deterministic). Slots: the near sum's partials of target block b are slots
// slot_off[b] .. slot_off[b+1]-1, each [2 x bt] (first components, then second components of
// the block's targets); block b of target i is cell_blk[cell] + (i - first node of the cell) / bt.
constexpr int kCombineLanes = 4;

__global__ __launch_bounds__(256) void k_combine(int64_t N, int64_t bt, const int32_t* __restrict__ cell_blk,
                                                 const int32_t* __restrict__ slot_off,
                                                 const double* __restrict__ Tpart, Geo g,
                                                 const double* __restrict__ sigma, int M,
                                                 const double* __restrict__ px, const double* __restrict__ py,
                                                 const double* __restrict__ xi_all, int with_extra,
                                                 const int32_t* __restrict__ active, double* __restrict__ T) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t i = gid / kCombineLanes;
  const int l = (int)(gid % kCombineLanes);
  const int64_t i0 = i < N ? i : N - 1;   // idle lanes shadow the last target so shuffles stay uniform
  const int cell = g.ncell[i0];
  // targets of cells that are not active (given a mask) are left as they are; the lanes of a
  // target share its cell, so a group skips together
  const bool live = i < N && (active == nullptr || active[cell] != 0);
  const int64_t ii = i0;
  const int64_t li = ii - g.cnoff[cell];
  const int64_t b = cell_blk[cell] + li / bt, local = li % bt;
  const int s1 = live ? slot_off[b + 1] : 0;
  double t1 = 0, t2 = 0;
  for (int k = slot_off[b] + l; k < s1; k += kCombineLanes) {
    t1 += Tpart[(int64_t)k * 2 * bt + local];
    t2 += Tpart[(int64_t)k * 2 * bt + bt + local];
  }
  if (with_extra && live) {   // the correction field at the target's position in the cell (wrapped node, dilated set)
    const double xx = g.dilated ? g.xw[ii] : g.x[ii], yy = g.dilated ? g.yw[ii] : g.y[ii];
    const double nx = g.nx[ii], ny = g.ny[ii];
    const double* xi = xi_all + (int64_t)cell * 2 * M;
    const double* pxc = px + (int64_t)cell * M;
    const double* pyc = py + (int64_t)cell * M;
    for (int p = l; p < M; p += kCombineLanes)
      traction_uv(xx - pxc[p], yy - pyc[p], nx, ny, xi[p], xi[M + p], t1, t2);
  }
#pragma unroll
  for (int o = kCombineLanes / 2; o > 0; o >>= 1) {
    t1 += __shfl_xor(t1, o, kCombineLanes);
    t2 += __shfl_xor(t2, o, kCombineLanes);
  }
  if (!live || l != 0) return;
  if (with_extra) {
    const double w = g.w[i], tx = g.tx[i], ty = g.ty[i];
    const double tf = tx * w * sigma[i] + ty * w * sigma[N + i];
    const double ks = -(g.kap[i] / (2.0 * kPi)) * tf;
    t1 += ks * tx;
    t2 += ks * ty;
  }
  T[i] = t1;
  T[N + i] = t2;
}

static void combine_into(spm_handle* h, const double* sigma, bool with_self_corr, int precision, double* out,
                         bool with_active = false) {
  const int64_t N = h->geo.N;
  const NearPlan& P = h->wk.near[precision == SPM_FP64 ? 0 : 1];
  const int64_t threads = N * kCombineLanes;
  // the FMM writes one block of all N nodes into one slot
  const int64_t bt = h->fmm.on ? N : P.bt;
  const int32_t* cell_blk = h->fmm.on ? h->fmm.one_block : P.cell_blk;
  const int32_t* slot_off = h->fmm.on ? h->fmm.one_block : P.slot_off;
  k_combine<<<(unsigned)((threads + 255) / 256), 256, 0, h->stream>>>(N, bt, cell_blk, slot_off, h->wk.Tpart,
                                                                     h->geo, sigma, h->per.M, h->per.px, h->per.py,
                                                                     h->wk.xi, with_self_corr ? 1 : 0,
                                                                     with_active ? h->kr.active : nullptr, out);
  SPM_HIP_CHECK(hipGetLastError());
}

void launch_combine(spm_handle* h, const double* sigma, bool with_self_corr, int precision, bool with_active) {
  combine_into(h, sigma, with_self_corr, precision, h->wk.T, with_active);
}

// The near-image sum alone (stage entry point for checking the near sum).
void launch_near_sum_only(spm_handle* h, double* out, int precision) {
  combine_into(h, nullptr, false, precision, out);
}

}  // namespace spm
