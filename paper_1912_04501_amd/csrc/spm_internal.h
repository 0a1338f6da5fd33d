// Internal declarations of the MI355X mobility solver (not part of the ABI).
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
constexpr int kMaxNodesPerParticle = 512;   // close-evaluation LDS staging (k_vplus) holds one curve

// Image shifts as kernel arguments (land in scalar registers).
template <typename R>
struct Shifts {
  R x[kShifts];
  R y[kShifts];
};

// ----------------------------------------------------------------------------
// One pair of the single-layer traction sum (Sec. 4.1 eq. Gt without the -1/pi,
// which is applied once per target):  a += r (r.n)(r.f) / |r|^4.
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
__device__ __forceinline__ void gt_pair(double rx, double ry, double nx, double ny, double f1,
                                        double f2, double& a1, double& a2) {
  double r2 = fma(rx, rx, 1e-300);
  r2 = fma(ry, ry, r2);
  double rn = rx * nx;
  rn = fma(ry, ny, rn);
  double rf = rx * f1;
  rf = fma(ry, f2, rf);
  const double i0 = __builtin_amdgcn_rcp(r2);
  const double e = fma(-r2, i0, 1.0);
  const double ee = fma(e, e, e);
  const double inv = fma(i0, ee, i0);
  const double p = rn * rf;
  double c = p * inv;
  c = c * inv;
  a1 = fma(c, rx, a1);
  a2 = fma(c, ry, a2);
}

__device__ __forceinline__ void gt_pair(float rx, float ry, float nx, float ny, float f1, float f2,
                                        float& a1, float& a2) {
  float r2 = fmaf(rx, rx, 1e-30f);
  r2 = fmaf(ry, ry, r2);
  float rn = rx * nx;
  rn = fmaf(ry, ny, rn);
  float rf = rx * f1;
  rf = fmaf(ry, f2, rf);
  const float inv = __builtin_amdgcn_rcpf(r2);
  const float p = rn * rf;
  float c = p * inv;
  c = c * inv;
  a1 = fmaf(c, rx, a1);
  a2 = fmaf(c, ry, a2);
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

// ----------------------------------------------------------------------------
// Device buffers of a handle (all SoA; N nodes, No particles).
// ----------------------------------------------------------------------------
struct Geo {
  int64_t N = 0;
  int32_t No = 0;
  // nodes, FP64
  double *x = nullptr, *y = nullptr, *nx = nullptr, *ny = nullptr, *w = nullptr, *kap = nullptr;
  double *tx = nullptr, *ty = nullptr, *xpx = nullptr, *xpy = nullptr;
  // nodes, FP32 shadows (targets and sources of the FP32 near sum)
  float *xf = nullptr, *yf = nullptr, *nxf = nullptr, *nyf = nullptr;
  int32_t* pid = nullptr;
  // particles
  double *pcx = nullptr, *pcy = nullptr, *pth = nullptr, *pa = nullptr, *pb = nullptr, *pper = nullptr;
  int32_t *poff = nullptr, *pn = nullptr;
};

struct Periodizer {
  int32_t m = 0, M = 0;
  double* wx = nullptr;   // [2m] wall points: L then D
  double* wy = nullptr;
  double* px = nullptr;   // [M] proxies
  double* py = nullptr;
  double* Q = nullptr;    // [8m x 2M] row-major
  double* Qp = nullptr;   // [2M x 8m] row-major pseudo-inverse
  double* svd_a = nullptr;  // Jacobi workspace [8m x 2M] column-major
  double* svd_v = nullptr;  // [2M x 2M]
  double* svd_s = nullptr;  // [2M]
  double nL[2] = {1, 0}, nD[2] = {0, 1};
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
};

// Launch shape of the near sum: block threads, targets per lane, sources per LDS
// tile, source splits (gridDim.y). Picked by the heuristic or the autotuner.
struct NearConfig {
  int32_t block = 256;
  int32_t tpt = 1;
  int32_t tile = 256;
  int32_t splits = 1;
};

struct Work {
  NearConfig near[2];         // [0] FP64, [1] FP32
  bool tuned = false;         // near[] came from the autotuner (for tuned_N nodes)
  int64_t tuned_N = -1;
  int32_t nchunk_disc = 1;    // source chunks of the wall discrepancy
  double *f1 = nullptr, *f2 = nullptr;   // w sigma
  float *f1f = nullptr, *f2f = nullptr;
  double* Tpart = nullptr;    // [splits x 2N]
  double* T = nullptr;        // [2N]
  double* pF = nullptr;       // [No x 4]: F1, F2, torque, stresslet
  double* disc = nullptr;     // [nchunk x 2m x 4]
  double* xi = nullptr;       // [2M]
  double* scal = nullptr;     // [16] device scalars
  size_t tpart_cap = 0;
};

struct Krylov {
  int32_t kmax = 0;
  int64_t n2 = 0;
  double* V = nullptr;        // [(kmax+1) x n2]
  double* H = nullptr;        // [(kmax+1) x kmax], column j at H + j*(kmax+1)
  double* cs = nullptr;       // [kmax]
  double* sn = nullptr;
  double* g = nullptr;        // [kmax+1]
  double* yv = nullptr;       // [kmax]
  double* h = nullptr;        // [kmax+1] CGS coefficients
  double* part = nullptr;     // [nchunk x (kmax+1)] dot partials
  double* tmp = nullptr;      // [n2]
  double* tmp2 = nullptr;     // [n2]
  double* res = nullptr;      // [4] device scalars: |g_{j+1}|, norm, ...
  double* host_res = nullptr; // pinned
  double* b = nullptr;        // [n2] right-hand side of the current solve
  double* d = nullptr;        // [n2] refinement correction (FP32_IR)
  double* stepbuf = nullptr;  // [n2 + 3 No + 2] state of spm_step
  int32_t nchunk = 0;
};

}  // namespace spm

struct spm_handle {
  spm_config cfg{};
  hipStream_t stream = nullptr;
  spm_alloc_fn alloc = nullptr;
  spm_free_fn free_fn = nullptr;
  void* alloc_ctx = nullptr;
  std::string err;
  std::vector<void*> owned;   // allocations to release

  bool have_lattice = false, have_particles = false;
  double e1[2] = {1, 0}, e2[2] = {0, 1}, cU[2] = {0, 0};
  double skew = 0.0, skew_raw = 0.0;
  // host copy of the particle table (wrapped centres)
  std::vector<double> cx, cy, th, a, b;
  std::vector<int32_t> nn, off;

  spm::Geo geo;
  spm::Periodizer per;
  spm::CloseList cl;
  spm::Work wk;
  spm::Krylov kr;
  double min_gap_est = 0.0;

  // opt-in kernel timing: HIP events around near-sum launches (kernel 0 = FP64, 1 = FP32)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;      // kernel id of each recorded start/stop pair
  size_t ev_used = 0;            // pairs recorded since the last flush
  double prof_ms[2] = {0, 0};
  int64_t prof_launches[2] = {0, 0};
  double prof_pairs[2] = {0, 0};
};

namespace spm {

// --- launch wrappers (defined in the k_*.hip files) --------------------------
void launch_geometry(spm_handle* h);
void launch_rhs(spm_handle* h, double* out);
void launch_prep(spm_handle* h, const double* sigma);
void launch_near(spm_handle* h, int precision);
void prof_flush(spm_handle* h);
void launch_near_sum_only(spm_handle* h, double* out, int precision);
bool near_config_valid(const NearConfig& c);
void autotune(spm_handle* h, const char* cache_path, double* best_ms_out);
double time_near(spm_handle* h, int prec, const NearConfig& c, int reps);
void launch_combine(spm_handle* h, const double* sigma, bool with_self_corr, int precision);
void launch_disc(spm_handle* h);
void launch_xi(spm_handle* h);
void launch_build_Q(spm_handle* h);
void launch_pinv(spm_handle* h);
void launch_close_count(spm_handle* h);
void launch_close_scan(spm_handle* h, int32_t* total_host, int32_t* ntargets_host);
void launch_close_fill(spm_handle* h);
void launch_vplus(spm_handle* h, const double* sigma);
void launch_close_apply(spm_handle* h, const double* sigma, double* T, int precision);
void launch_assemble(spm_handle* h, const double* sigma, double* out);
void launch_velocities(spm_handle* h, double* vel, double* omega);
void launch_mu_eff(spm_handle* h, double* mu_eff);
void launch_gap(spm_handle* h, double* gap_host, int32_t* overlap_host);

// GMRES building blocks (k_gmres.hip)
void gm_dot_many(spm_handle* h, const double* V, int64_t ld, int cnt, const double* w, double* out);
void gm_update(spm_handle* h, const double* V, int64_t ld, int cnt, const double* coef, double* w, double sign);
void gm_axpby(spm_handle* h, int64_t n, double a, const double* x, double b, const double* y, double* out);
void gm_scale_by_norm(spm_handle* h, const double* nrm2, double* v, int64_t n, double* norm_out);
void gm_givens(spm_handle* h, int j, const double* h1, const double* h2, const double* nrm2, double bnorm,
               double* res_out);
void gm_backsolve(spm_handle* h, int k);
void gm_init(spm_handle* h, const double* nrm2);
void gm_copy(spm_handle* h, double* dst, const double* src, int64_t n);
void gm_zero(spm_handle* h, double* dst, int64_t n);

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
