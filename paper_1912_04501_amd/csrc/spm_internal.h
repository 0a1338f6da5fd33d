// Internal declarations of the MI355X mobility solver (not part of the ABI).
//
// A handle holds C >= 1 independent unit cells (an ensemble); the single-cell calls
// of the ABI are the case C = 1. Nodes and particles of all cells are stored
// back to back (cell-major, then particle-major), so every kernel works on the
// whole ensemble at once and finds a node's cell through ncell[].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/spm.h"

namespace spm {

constexpr double kPi = 3.14159265358979323846;
constexpr int kShifts = 9;   // 3x3 images m e1 + n e2, index 3 (m + 1) + (n + 1)
constexpr int kZeroShift = 4;
constexpr int kMaxNodesPerParticle = 4096;  // nodes of one particle curve
constexpr int kMaxNodesStaged = 512;        // curves held whole in LDS: block preconditioner, density modes
constexpr int kVplusTile = 512;             // source nodes per LDS stage of the close-evaluation boundary values

// Body-frame point of a particle curve at parameter t (SPM_SHAPE_ELLIPSE: (a cos t, b sin t);
// SPM_SHAPE_STAR: r(t) (cos t, sin t), r = s (1 + A cos(omega t + phi))) with its first and
// second t-derivatives.
__host__ __device__ __forceinline__ void shape_point(int kind, const double* p, double t, double& X, double& Y,
                                                     double& Xp, double& Yp, double& Xpp, double& Ypp) {
  const double st = sin(t), ct = cos(t);
  if (kind == SPM_SHAPE_ELLIPSE) {
    X = p[0] * ct;
    Y = p[1] * st;
    Xp = -p[0] * st;
    Yp = p[1] * ct;
    Xpp = -X;
    Ypp = -Y;
  } else {
    const double su = sin(p[2] * t + p[3]), cu = cos(p[2] * t + p[3]);
    const double r = p[0] * (1.0 + p[1] * cu);
    const double rp = -p[0] * p[1] * p[2] * su;
    const double rpp = -p[0] * p[1] * p[2] * p[2] * cu;
    X = r * ct;
    Y = r * st;
    Xp = rp * ct - r * st;
    Yp = rp * st + r * ct;
    Xpp = rpp * ct - 2.0 * rp * st - r * ct;
    Ypp = rpp * st + 2.0 * rp * ct - r * st;
  }
}

// Image shift s = m e1 + n e2 of a cell with e1 = (1, 0), e2 = (skew, 1), computed the
// same way by every kernel (the FP32 close correction needs bit-identical shifts).
__host__ __device__ __forceinline__ double shift_x(int s, double skew) {
  return (double)(s / 3 - 1) + (double)(s % 3 - 1) * skew;
}
__host__ __device__ __forceinline__ double shift_y(int s) { return (double)(s % 3 - 1); }

// Lattice shift m e1 + n e2 (e1 = (1, 0), e2 = (skew, 1)) for integers m, n: x component.
// The near sum of the dilated set and the kernels that remove its close terms form the FP32
// shifts from this one expression, so those terms agree bit for bit.
__host__ __device__ __forceinline__ double shift_xmn(int m, int n, double skew) { return (double)m + (double)n * skew; }

// Packed per-node wrap of the dilated near set: the node was moved by ka e1 + kb e2 into the
// cell (|ka|, |kb| < 2^14), and its images inside U~ are the shifts {0, ms} x {0, ns} with
// ms = +1 when its first lattice coordinate (after the wrap) is negative, else -1; ns likewise.
__host__ __device__ __forceinline__ int32_t node_wrap_pack(int ka, int kb, int ms, int ns) {
  return ((ka + 16384) & 0x7fff) | (((kb + 16384) & 0x7fff) << 15) | ((ms > 0) << 30) | ((int32_t)(ns > 0) << 31);
}
__host__ __device__ __forceinline__ int node_wrap_ka(int32_t w) { return (w & 0x7fff) - 16384; }
__host__ __device__ __forceinline__ int node_wrap_kb(int32_t w) { return ((w >> 15) & 0x7fff) - 16384; }
__host__ __device__ __forceinline__ int node_wrap_ms(int32_t w) { return ((w >> 30) & 1) ? 1 : -1; }
__host__ __device__ __forceinline__ int node_wrap_ns(int32_t w) { return ((unsigned)w >> 31) ? 1 : -1; }

// ----------------------------------------------------------------------------
// Pairs of the single-layer traction sum (Sec. 4.1 eq. Gt without the -1/pi, which
// is applied once per target):  a += r (r.n)(r.f) / |r|^4,  r = (dx - sx, dy - sy).
//
// The three images of a lattice row share sy, so per source the row terms
//   ry = dy - sy,  ry2 = ry^2 + floor,  ryn = ry n_y,  ryf = ry f_y
// are formed once per row and every pair then costs 9 VALU operations + 1 reciprocal
// (FP64: + 3 for the reciprocal correction).
//
// The self pair (r == 0) is handled without a branch: |r|^2 gets a tiny floor
// (1e-300 in FP64, 1e-30 in FP32) far below any physical pair distance, so the
// reciprocal stays finite and (r.n)(r.f) == 0 makes the term exactly zero.
//
// FP64: v_rcp_f64 is accurate to ~2^-24 only, so one third-order correction
// step  inv = i0 (1 + e + e^2), e = 1 - r2 i0  restores full precision.
// FP32: v_rcp_f32 is within 1 ulp; no correction.
//
// Both the near-sum kernel and the close-correction kernel call these, so the
// FP32 plain terms the close correction removes are bit-identical to the ones
// the near sum added. Compile with -ffp-contract=off: only the fma() calls fuse.
// ----------------------------------------------------------------------------
template <typename R>
struct RowTerms {
  R ry, ry2, ryn, ryf;
};

__device__ __forceinline__ RowTerms<double> row_terms(double dy, double sy, double ny, double f2) {
  RowTerms<double> t;
  t.ry = dy - sy;
  t.ry2 = fma(t.ry, t.ry, 1e-300);
  t.ryn = t.ry * ny;
  t.ryf = t.ry * f2;
  return t;
}

__device__ __forceinline__ RowTerms<float> row_terms(float dy, float sy, float ny, float f2) {
  RowTerms<float> t;
  t.ry = dy - sy;
  t.ry2 = fmaf(t.ry, t.ry, 1e-30f);
  t.ryn = t.ry * ny;
  t.ryf = t.ry * f2;
  return t;
}

__device__ __forceinline__ void gt_pair(double rx, const RowTerms<double>& t, double nx, double f1, double& a1,
                                        double& a2) {
  const double r2 = fma(rx, rx, t.ry2);
  const double rn = fma(rx, nx, t.ryn);
  const double rf = fma(rx, f1, t.ryf);
  const double i0 = __builtin_amdgcn_rcp(r2);
  const double e = fma(-r2, i0, 1.0);
  const double ee = fma(e, e, e);
  const double inv = fma(i0, ee, i0);
  const double p = rn * rf;
  double c = p * inv;
  c = c * inv;
  a1 = fma(c, rx, a1);
  a2 = fma(c, t.ry, a2);
}

__device__ __forceinline__ void gt_pair(float rx, const RowTerms<float>& t, float nx, float f1, float& a1, float& a2) {
  const float r2 = fmaf(rx, rx, t.ry2);
  const float rn = fmaf(rx, nx, t.ryn);
  const float rf = fmaf(rx, f1, t.ryf);
  const float inv = __builtin_amdgcn_rcpf(r2);
  const float p = rn * rf;
  float c = p * inv;
  c = c * inv;
  a1 = fmaf(c, rx, a1);
  a2 = fmaf(c, t.ry, a2);
}

// FP32 terms of the 3x3 image set in Horner form. With A = n1 f1, D = n1 f2 + n2 f1 and
// E = n2 f2 (target normal n, source force f, once per target-source pair),
//   (r.n)(r.f) = (A rx + B) rx + C,   B = ry D,   C = ry^2 E   (once per lattice row),
// two fused multiply-adds per image where the product form takes three operations. The row of
// zero y shift, which holds the target's own node, takes C from the exact square (zero for
// ry = 0, so the self pair is exactly zero as above); the other rows take it from the floored
// square they already hold. Every kernel that removes FP32 plain terms of the 3x3 set calls
// these with the same row rule, so its terms are bit-identical to the near sum's.
struct PairTerms32 {
  float A, D, E;
};

__device__ __forceinline__ PairTerms32 pair_terms32(float nx, float ny, float f1, float f2) {
  PairTerms32 p;
  p.A = nx * f1;
  p.D = fmaf(nx, f2, ny * f1);
  p.E = ny * f2;
  return p;
}

struct RowTerms32 {
  float ry, ry2, B, C;
};

template <bool ZERO_ROW>
__device__ __forceinline__ RowTerms32 row_terms32(float dy, float sy, const PairTerms32& p) {
  RowTerms32 t;
  t.ry = dy - sy;
  t.ry2 = fmaf(t.ry, t.ry, 1e-30f);
  t.B = t.ry * p.D;
  t.C = ZERO_ROW ? (t.ry * t.ry) * p.E : t.ry2 * p.E;
  return t;
}

// Row terms for a shift known only at run time (the zero-shift row by value, as in the near sum).
__device__ __forceinline__ RowTerms32 row_terms32_any(float dy, float sy, const PairTerms32& p) {
  return sy == 0.0f ? row_terms32<true>(dy, sy, p) : row_terms32<false>(dy, sy, p);
}

__device__ __forceinline__ void gt_pair32(float rx, const RowTerms32& t, const PairTerms32& p, float& a1, float& a2) {
  const float r2 = fmaf(rx, rx, t.ry2);
  const float q = fmaf(p.A, rx, t.B);
  const float pr = fmaf(q, rx, t.C);
  const float inv = __builtin_amdgcn_rcpf(r2);
  float c = pr * inv;
  c = c * inv;
  a1 = fmaf(c, rx, a1);
  a2 = fmaf(c, t.ry, a2);
}

// Accurate FP64 reciprocal (correctly rounded division is not needed here).
__device__ __forceinline__ double rcp64(double v) {
  const double i0 = __builtin_amdgcn_rcp(v);
  const double e = fma(-v, i0, 1.0);
  return fma(i0, fma(e, e, e), i0);
}

// Wave (64-lane) sum with a fixed butterfly order: deterministic.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Lanes that share one row of a per-particle loop: the largest power of two <= 16 with
// n_max * lanes <= 1024 (a 1024-thread block covers a whole particle in one pass).
inline int lanes_per_row(int nmax) {
  int L = 1;
  while (L < 16 && 2 * L * nmax <= 1024) L *= 2;
  return L;
}

// Sum over the `width` lanes of a group (a power of two dividing 64), fixed butterfly order.
__device__ __forceinline__ double group_sum(double v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
  return v;
}

// Block sum for blockDim.x a multiple of 64 (<= 1024), deterministic; result valid in all threads.
__device__ __forceinline__ double block_sum(double v, double* scratch /* >= 16 doubles */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += scratch[k];
  return t;
}

// Double-double accumulation (error-free transformations, Knuth's two-sum and an FMA
// two-product): a sum carried as an unevaluated hi + lo pair keeps the rounding error of
// every addition. Used where a small result is the sum of many larger terms and an
// ill-conditioned step follows (the wall discrepancy, then the proxy least squares).
struct dd {
  double hi, lo;
};
__device__ __forceinline__ dd dd_add_d(dd a, double b) {
  const double s = a.hi + b, bb = s - a.hi;
  const double e = ((a.hi - (s - bb)) + (b - bb)) + a.lo;
  const double h = s + e;
  return {h, e - (h - s)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  const double s = a.hi + b.hi, bb = s - a.hi;
  const double e = ((a.hi - (s - bb)) + (b.hi - bb)) + (a.lo + b.lo);
  const double h = s + e;
  return {h, e - (h - s)};
}
__device__ __forceinline__ dd dd_fma(dd acc, double a, double b) {   // acc + a b
  const double p = a * b;
  const double pe = fma(a, b, -p);
  dd r = dd_add_d(acc, p);
  return dd_add_d(r, pe);
}
// Wave sum of pairs by a xor butterfly (dd_add is symmetric, so every lane ends equal).
__device__ __forceinline__ dd dd_wave_sum(dd v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = dd_add(v, dd{__shfl_xor(v.hi, o, 64), __shfl_xor(v.lo, o, 64)});
  return v;
}
// Block sum of pairs for blockDim.x a multiple of 64 (<= 1024); result valid in all threads.
__device__ __forceinline__ dd dd_block_sum(dd v, double* scratch /* >= 32 doubles */) {
  v = dd_wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
    scratch[2 * wid] = v.hi;
    scratch[2 * wid + 1] = v.lo;
  }
  __syncthreads();
  dd t = {0.0, 0.0};
  for (int k = 0; k < nw; ++k) t = dd_add(t, dd{scratch[2 * k], scratch[2 * k + 1]});
  return t;
}

// ----------------------------------------------------------------------------
// Device buffers of a handle (all SoA; N nodes, No particles, C cells).
// ----------------------------------------------------------------------------
struct Geo {
  int64_t N = 0;
  int32_t No = 0;
  int32_t C = 0;
  int32_t nmax = 0;           // largest node count of a particle
  // nodes, FP64
  double *x = nullptr, *y = nullptr, *nx = nullptr, *ny = nullptr, *w = nullptr, *kap = nullptr;
  double* dcot = nullptr;     // [N] spectral differentiation weights of the particle's own N_q, by distance
  double *tx = nullptr, *ty = nullptr, *xpx = nullptr, *xpy = nullptr;
  // nodes, FP32 shadows (targets and sources of the FP32 near sum; with the dilated near set the
  // node positions wrapped into the cell one by one)
  float *xf = nullptr, *yf = nullptr, *nxf = nullptr, *nyf = nullptr;
  // dilated near set only: node positions wrapped into the cell (FP64) and per node the lattice
  // vector added by the wrap and the side of the cell it lies on (node_wrap_* below)
  double *xw = nullptr, *yw = nullptr;
  int32_t* nwrap = nullptr;
  int32_t dilated = 0;
  int32_t* pid = nullptr;     // [N] particle of each node
  int32_t* ncell = nullptr;   // [N] cell of each node
  // particles
  // pa, pb: largest and smallest distance from the reference point to the curve
  double *pcx = nullptr, *pcy = nullptr, *pth = nullptr, *pa = nullptr, *pb = nullptr, *pper = nullptr;
  double* parea = nullptr;    // [No] particle areas (boundary quadrature of (1/2) x ^ dx)
  int32_t *poff = nullptr, *pn = nullptr;
  int32_t* pcell = nullptr;   // [No] cell of each particle
  int32_t* pkind = nullptr;   // [No] SPM_SHAPE_*
  double* pprm = nullptr;     // [No x 4] shape parameters (ellipse a, b; star s, A, omega, phi)
  // cells
  int64_t* cnoff = nullptr;   // [C + 1] node offsets
  int32_t* cpoff = nullptr;   // [C + 1] particle offsets
  double* cskew = nullptr;    // [C] reduced skew (e2 = (skew, 1))
};

struct Periodizer {
  int32_t m = 0, M = 0;
  double* wx = nullptr;     // [C x 2m] wall points: L then D
  double* wy = nullptr;
  double* px = nullptr;     // [M] proxies (the same circle about c_U for every cell)
  double* py = nullptr;
  double* Q = nullptr;      // [C x 8m x 2M] row-major
  double* Qp = nullptr;     // [C x 2M x 8m] row-major pseudo-inverse
  double* svd_a = nullptr;  // Jacobi workspace [C x 8m x 2M] column-major
  double* svd_v = nullptr;  // [C x 2M x 2M]
  double* svd_s = nullptr;  // [C x (2M + 1)]: singular values and the sweep count
  bool warm_ok = false;     // svd_v holds orthogonal V's of the current shape (C, m, M): warm start
  int32_t warm_C = -1, warm_m = -1, warm_M = -1;
};

struct CloseList {
  int64_t npairs = 0;
  int32_t ntargets = 0;
  int32_t* count = nullptr;   // [N]
  int32_t* row = nullptr;     // [N + 1] row pointers into q/s
  int32_t* q = nullptr;       // [npairs] source particle
  int32_t* s = nullptr;       // [npairs] shift index
  int32_t* tlist = nullptr;   // [ntargets] targets with at least one close pair
  double* dmin = nullptr;     // [N] min node distance to other particles (gap estimate)
  int32_t* inside = nullptr;  // [N] 1 if the node lies inside another particle
  double* vp = nullptr;       // [6 N] v+ of the three densities: re0 im0 re1 im1 re2 im2 (each N)
  int32_t* qsrc = nullptr;    // [No] 1 if the particle is the source of a close pair (the operator needs its v+)
};

// Launch shape of the near sum: block threads, targets per lane, sources per LDS
// tile, sources per split (each cell's sources are cut into ceil(N_c / chunk)
// splits). Picked by the heuristic or the autotuner.
struct NearConfig {
  int32_t block = 256;
  int32_t tpt = 1;
  int32_t tile = 256;
  int32_t wg_per_cu = 0;      // persistent workgroups per compute unit (0: the occupancy limit)
};

// Plan of the near-sum launch of one precision. The work is split into units (target block of
// block * tpt targets, source tile of `tile` sources of the same cell); the units of the active
// cells, taken in order (cell, target block, tile), are divided evenly over the persistent
// workgroups, and each workgroup writes one FP64 partial per target block it touches. The
// partition kernel fills unit_off and slot_off before every launch (the active cells change
// during an ensemble solve); the combine step sums the slots of a block in workgroup order.
struct NearPlan {
  NearConfig cfg;
  int32_t nblocks = 0;          // target blocks over all cells
  int32_t bt = 0;               // targets per block (block * tpt)
  int32_t* cell_nt = nullptr;   // [C] source tiles of the cell (= units per target block)
  int32_t* cell_blk = nullptr;  // [C + 1] first target block of each cell
  int64_t* unit_off = nullptr;  // [C + 1] offsets of the active cells' units
  int32_t* slot_off = nullptr;  // [nblocks + 1] partial slots of each target block
  int32_t grid = 0;             // persistent grid size (workgroups)
};

struct Work {
  NearPlan near[2];           // [0] FP64, [1] FP32
  bool tuned = false;         // near[].cfg came from the autotuner (for tuned_N nodes)
  int64_t tuned_N = -1;
  // wall discrepancy work items (source chunks of every cell)
  int32_t ndisc = 0;
  int64_t* disc_s0 = nullptr; // [ndisc] chunk source ranges
  int64_t* disc_s1 = nullptr;
  int32_t* disc_cell = nullptr;
  int32_t* disc_off = nullptr;  // [C + 1] chunks of each cell
  double *f1 = nullptr, *f2 = nullptr;   // w sigma
  float *f1f = nullptr, *f2f = nullptr;
  double* Tpart = nullptr;    // near-sum partials: [slots x 2 x targets per block]
  double* T = nullptr;        // [2N]
  double* batch_sigma = nullptr;  // [2N] density of the one-call ensemble solve
  double* cell_du = nullptr;  // [C] velocity added to the particles of each cell by that solve
  double* pF = nullptr;       // [No x 4]: F1, F2, torque, stresslet
  double* disc = nullptr;     // [ndisc x 2m x 8] (double-double partials)
  double* xi = nullptr;       // [C x 2M]
  double* scal = nullptr;     // [16] device scalars
  double* gauge = nullptr;    // [C x 2] velocity constant removed by the readout gauge
  double* contour = nullptr;  // [C x 11 m] point terms of the contour-deformation mu_eff
  double* contour_gl = nullptr;  // [2 m] Gauss-Legendre nodes and weights on [-1, 1]
};

// Fast multipole evaluation of the near-image sum (one cell, FP64): a uniform quadtree over
// the 9 N image sources, complex multipole and local expansions of p terms (k_fmm.hip).
struct FmmPlan {
  bool on = false;
  int32_t p = 0, L = 0;                   // expansion terms; leaf level (root box = level 0)
  double D0 = 0, c0x = 0, c0y = 0;        // root box side and centre
  int64_t nsrc = 0;                       // 9 N
  double *sx = nullptr, *sy = nullptr;    // [9N] image sources sorted by leaf
  int32_t* sj = nullptr;                  // [9N] node of each sorted source
  double *fs1 = nullptr, *fs2 = nullptr;  // [9N] w sigma in sorted order
  int32_t* leaf_s = nullptr;              // [4^L + 1] source offsets of the leaves
  int32_t* tperm = nullptr;               // [N] nodes sorted by leaf
  int32_t* leaf_t = nullptr;              // [4^L + 1] target offsets of the leaves
  int32_t* bsrc = nullptr;                // [boxes of all levels] sources in each box
  int32_t* lists = nullptr;               // box lists of the passes (global box ids)
  std::vector<int64_t> seg;               // list segments: P2M, M2M levels L-1..2, M2L, L2L levels 3..L,
                                          // target leaves
  double* fact = nullptr;                 // [2p] factorials
  double* m2l_tab = nullptr;              // [49 x 2 x p] complex M2L scalings per box displacement
  double *Mx = nullptr, *Lx = nullptr;    // [boxes x 3 x p] complex multipole / local expansions
  int32_t* one_block = nullptr;           // {0, 1}: the combine step reads one block of all N nodes, one slot
  double* vnear = nullptr;                // [3 No] near-image velocity and vorticity at the centres
  double p2p_pairs = 0, m2l = 0;          // work of one evaluation
};

// Flow-field evaluation at points of the fluid.
struct Field {
  double* iw = nullptr;       // [N] spectral antiderivative weights of each particle's own N_q, by distance
  double* hp = nullptr;       // [4N] H+ of sigma_1, sigma_2 (re, im): boundary values of the log potential part
  double* vel = nullptr;      // [2 No] readout velocities (gauged)
  double* om = nullptr;       // [No]
};

// Krylov state. Cells iterate in lockstep on one global iteration index j (kept in
// device memory so one captured iteration can be replayed); each cell has its own
// Hessenberg matrix, rotations, tolerance and active flag and stops on its own.
struct Krylov {
  int32_t kmax = 0;
  int64_t n2 = 0;
  double* V = nullptr;        // [(kmax+1) x n2]
  double* H = nullptr;        // [C x kmax x (kmax+1)], column j of cell c at H + (c*kmax + j)*(kmax+1)
  double* cs = nullptr;       // [C x kmax]
  double* sn = nullptr;
  double* g = nullptr;        // [C x (kmax+1)]
  double* yv = nullptr;       // [C x kmax]
  double* h1 = nullptr;       // [C x (kmax+1)] CGS pass 1 coefficients
  double* h2 = nullptr;       // [C x (kmax+1)] pass 2
  double* nrm2 = nullptr;     // [C]
  double* bnorm = nullptr;    // [C] norm of this solve's right-hand side
  double* tolc = nullptr;     // [C] stopping tolerance relative to bnorm
  double* res = nullptr;      // [C] residual estimate |g_{j+1}| / bnorm
  int32_t* active = nullptr;  // [C]
  int32_t* kdone = nullptr;   // [C] Krylov iterations of each cell
  unsigned long long* stamp = nullptr;  // [C + 2] device wall clock at convergence; [C] = solve start,
                                        // [C + 1] = start of the current Krylov cycle
  int32_t* jdev = nullptr;    // [2]: current j, number of active cells
  int32_t* gcount = nullptr;  // [1] k_givens wavefronts finished in the running launch (the last resets it)
  double* part = nullptr;     // [nseg x (kmax+1)] dot partials
  int32_t nseg = 0;
  int64_t* seg_n0 = nullptr;  // [nseg] node range of each dot segment
  int64_t* seg_n1 = nullptr;
  int32_t* seg_cell = nullptr;// [nseg] cell of each segment
  int32_t* seg_off = nullptr; // [C + 1] segments of each cell
  double* tmp = nullptr;      // [n2]
  double* tmp2 = nullptr;     // [n2]
  double* vin = nullptr;      // [n2] matvec input of the current iteration
  double* w = nullptr;        // [n2] matvec output of the current iteration
  double* b = nullptr;        // [n2] right-hand side of the current solve
  double* d = nullptr;        // [n2] refinement correction (FP32_IR)
  double* stepbuf = nullptr;  // state of spm_step
  double* dots = nullptr;     // [C] small per-cell reductions
  void* host = nullptr;       // pinned host scratch
  size_t host_bytes = 0;
  double* z = nullptr;        // [n2] preconditioned matvec input / correction
  double* z2 = nullptr;       // [n2]
  // captured iteration graphs: index precision (0: FP64, 1: FP32) + 2 * preconditioned
  hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraph_t graph_src[4] = {nullptr, nullptr, nullptr, nullptr};
  hipStream_t cap_stream = nullptr;   // private stream used only to capture graphs
  int32_t* mask = nullptr;            // [C] scratch mask uploaded from the host
};

// Learned warm start buffers.
struct Learned {
  double* nvec = nullptr;     // [2N] outward normals, SoA
  double* num = nullptr;      // [C] <r, n> (or <sigma, n>) per cell
  double* den = nullptr;      // [C] <n, n> per cell
  double* fit = nullptr;      // [5C] dots of the warm-start fit, then [2C] alpha, beta
  float* feat = nullptr;      // [No x 33]
  float* modes = nullptr;     // [No x 128]
};

// Shape of one self block being built: ellipse semi-axes, nodes, offsets of its
// [B | I] work matrix and of its FP32 inverse.
struct ShapeDesc {
  double p[4];      // shape parameters
  int32_t kind;     // SPM_SHAPE_*
  int32_t n;
  int64_t woff;
  int64_t ioff;
};

// Block preconditioner: one FP32 inverse per distinct shape (a, b, N) of the current
// particles (kept while the shapes stay the same).
struct Precond {
  bool valid = false;
  std::vector<std::vector<double>> keys;   // distinct shapes {kind, p0..p3, N}, in order of first appearance
  int32_t* pshape = nullptr;    // [No] shape of each particle
  size_t pshape_cap = 0;
  int64_t* ioff = nullptr;      // [shapes] offset of each inverse
  size_t ioff_cap = 0;
  float* inv = nullptr;         // inverses, (2n)^2 floats each, by row segment (k_precond.hip)
  size_t inv_cap = 0;
  int32_t segs = 1;             // row segments of every inverse (the apply's grid.y)
  double* work = nullptr;       // build workspace
  size_t work_cap = 0;
  ShapeDesc* desc = nullptr;
  size_t desc_cap = 0;
  int32_t* status = nullptr;
  size_t status_cap = 0;
};

struct CellHost {
  double skew_raw = 0.0, skew = 0.0;
  int32_t p0 = 0, p1 = 0;
  int64_t n0 = 0, n1 = 0;
};

}  // namespace spm

struct spm_handle {
  spm_config cfg{};
  hipStream_t stream = nullptr;
  spm_alloc_fn alloc = nullptr;
  spm_free_fn free_fn = nullptr;
  void* alloc_ctx = nullptr;
  std::string err;

  bool have_lattice = false, have_particles = false;
  double cU[2] = {0, 0};
  double pending_skew = 0.0;          // set by spm_set_lattice for the next spm_set_ellipses
  std::vector<spm::CellHost> cells;   // host view of the cells
  // host copy of the particle table (wrapped centres), all cells
  std::vector<double> cx, cy, th, a, b;   // a, b: largest and smallest radius
  std::vector<int32_t> nn, off, pcell, kind;
  std::vector<double> prm;                // [4 n] shape parameters

  spm::Geo geo;
  spm::Periodizer per;
  spm::CloseList cl;
  spm::Work wk;
  spm::Field fd;
  spm::FmmPlan fmm;
  spm::Krylov kr;
  spm::Learned ln;
  spm::Precond pc;
  spm_mlp* net = nullptr;             // borrowed warm-start network
  double min_gap_est = 0.0;
  double delta32 = -1.0;              // measured relative error of the FP32 operator (< 0: not measured for this geometry)
  std::vector<int32_t> guess_rejected;   // [C] per cell of the last solve: learned guess rejected
  double wallclock_hz = 1e8;

  // opt-in kernel timing: HIP events around near-sum launches (kernel 0 = FP64, 1 = FP32; FMM: 2 = evaluation, 3 = M2L)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;      // kernel id of each recorded start/stop pair
  size_t ev_used = 0;            // pairs recorded since the last flush
  double prof_ms[4] = {0, 0, 0, 0};
  int64_t prof_launches[4] = {0, 0, 0, 0};
  double prof_pairs[4] = {0, 0, 0, 0};
};

// The warm-start network (k_mlp.hip): FP32 master parameters, Adam moments and the
// activation buffers of the largest batch seen so far.
struct spm_mlp {
  hipStream_t stream = nullptr;
  spm_alloc_fn alloc = nullptr;
  spm_free_fn free_fn = nullptr;
  void* alloc_ctx = nullptr;
  std::string err;
  float *params = nullptr, *grads = nullptr, *m1 = nullptr, *m2 = nullptr;   // [SPM_MLP_NPARAMS]
  float* h[3] = {nullptr, nullptr, nullptr};   // hidden activations [cap x 256]
  float* y = nullptr;                          // output [cap x 128]
  float* dz[2] = {nullptr, nullptr};           // back-propagated gradients [cap x 256]
  double* part = nullptr;                      // loss partial sums
  double* loss = nullptr;                      // [1]
  int32_t* flag = nullptr;                     // [1] argument check
  int64_t cap = 0;                             // batch capacity of the buffers
  int64_t t = 0;                               // Adam step count
};

namespace spm {

void mlp_forward(spm_mlp* net, hipStream_t s, const float* x, const int32_t* xrow, int64_t B, float* y, int mode);

// --- launch wrappers (defined in the k_*.hip files) --------------------------
void launch_field(spm_handle* h, int64_t n_targets, const double* xt, const double* yt, double* u, double* p);
void launch_geometry(spm_handle* h);
void launch_rhs(spm_handle* h, double* out);
void launch_prep(spm_handle* h, const double* sigma);
void launch_near(spm_handle* h, int precision);
void prof_flush(spm_handle* h);
void launch_near_sum_only(spm_handle* h, double* out, int precision);
bool near_config_valid(const NearConfig& c);
int near_persistent_grid(const NearConfig& c, int precision, bool dilated);   // workgroups of the persistent near-sum grid
void build_near_plan(spm_handle* h, int precision);
void autotune(spm_handle* h, const char* cache_path, double* best_ms_out);
double time_near(spm_handle* h, int prec, const NearConfig& c, int reps);
NearConfig heuristic_near(spm_handle* h, int precision);
void launch_combine(spm_handle* h, const double* sigma, bool with_self_corr, int precision,
                    bool with_active = false);
void launch_disc(spm_handle* h);
void launch_xi(spm_handle* h);
void launch_build_Q(spm_handle* h);
void launch_pinv(spm_handle* h);
void launch_close_count(spm_handle* h);
void launch_close_scan(spm_handle* h, int32_t* total_host, int32_t* ntargets_host);
void launch_close_fill(spm_handle* h);
void launch_vplus(spm_handle* h, const double* sigma, bool all_particles, bool with_active = false);
void launch_close_sources(spm_handle* h);
void launch_close_apply(spm_handle* h, const double* sigma, double* T, int precision);
void launch_self_fix(spm_handle* h, double* T, bool with_active);
void launch_assemble(spm_handle* h, const double* sigma, double* out);
void launch_velocities(spm_handle* h, double* vel, double* omega);
void launch_mu_eff(spm_handle* h, double* mu_eff);
void launch_mu_eff_contour(spm_handle* h, int m, double* mu_eff);
// FMM near sum (k_fmm.hip): plan from the device node positions; evaluation into out [2N]
void build_fmm_plan(spm_handle* h);
void launch_fmm(spm_handle* h, double* out);
void launch_fmm_tables(spm_handle* h);   // per-displacement M2L scalings (once per plan)
void launch_fmm_velocities(spm_handle* h, double* near3);
void launch_fmm_points(spm_handle* h, int64_t nt, const double* xt, const double* yt, double* u, double* p);
void launch_gap(spm_handle* h, double* gap_host, int32_t* overlap_host);

// GMRES building blocks (k_gmres.hip); per cell, cells in lockstep
void gm_dot(spm_handle* h, const double* a, const double* b, double* out /*[C]*/);
void gm_cgs_pass(spm_handle* h, const double* w, double* coef);
void gm_update_j(spm_handle* h, const double* coef, double* w);
void gm_store_next(spm_handle* h);
void gm_givens(spm_handle* h);
void gm_zero_i32(spm_handle* h, int32_t* p, int64_t n);
void gm_copy_in(spm_handle* h);
void gm_start(spm_handle* h);
void gm_backsolve_update(spm_handle* h, double* x);
void gm_axpby(spm_handle* h, int64_t n, double a, const double* x, double b, const double* y, double* out);
void gm_copy(spm_handle* h, double* dst, const double* src, int64_t n);
void gm_zero(spm_handle* h, double* dst, int64_t n);
void gm_probe_fill(spm_handle* h, int64_t n, uint64_t seed, double* out);   // deterministic values in [-1, 1)
void gm_stamp_start(spm_handle* h);
void gm_stamp_mask(spm_handle* h, const int32_t* mask_dev);
void gm_stamp_cycle(spm_handle* h);
void launch_disc_impl(spm_handle* h, bool with_active);
void launch_xi_impl(spm_handle* h, bool with_active);
void launch_near_impl(spm_handle* h, int precision, bool with_active);
void launch_close_apply_impl(spm_handle* h, double* T, int precision, bool with_active);

// learned warm start (k_learned.hip) and block preconditioner (k_precond.hip)
void launch_features(spm_handle* h, float* feat);
void launch_to_bf16(spm_handle* h, const float* in, int64_t n, uint16_t* out);   // nearest even
void launch_reject_guess(spm_handle* h, const int32_t* mask, const double* b, double* x, double* r);
void launch_add_cell_velocity(spm_handle* h, const double* du, double* vel);   // vel[2i] += du[cell of i]
void launch_modes(spm_handle* h, const double* sigma, const double* num, const double* den, float* modes);
void launch_decode(spm_handle* h, const float* modes, double* sigma);
void launch_add_normal(spm_handle* h, const double* num, const double* den, double f, double* x);
void launch_fit_guess(spm_handle* h, const double* dots, double* coef);
void launch_apply_fit(spm_handle* h, const double* coef, const double* b, const double* z, double* x, double* r);
void build_precond(spm_handle* h);
void launch_precond_apply(spm_handle* h, const double* v, double* out, bool with_active);
void* precond_alloc(spm_handle* h, void* old, size_t bytes, size_t& cap);
void precond_release_work(spm_handle* h);
void gm_update_only(spm_handle* h, double* x);   // x += V y (after gm_backsolve)
void gm_backsolve(spm_handle* h);

}  // namespace spm

#define SPM_HIP_CHECK(expr)                                         \
  do {                                                              \
    hipError_t _e = (expr);                                         \
    if (_e != hipSuccess) throw spm::HipError(_e, #expr, __LINE__); \
  } while (0)

namespace spm {
struct HipError {
  hipError_t code;
  const char* what;
  int line;
  HipError(hipError_t c, const char* w, int l) : code(c), what(w), line(l) {}
};
struct ApiError {
  int code;
  std::string msg;
  ApiError(int c, std::string m) : code(c), msg(std::move(m)) {}
};
}  // namespace spm
