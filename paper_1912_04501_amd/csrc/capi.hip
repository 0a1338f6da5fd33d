// C ABI of the solver: handle, setup, matvec pipeline, GMRES driver, readouts, time stepping.
#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <utility>

#include "spm_internal.h"

using namespace spm;

namespace spm {
// Default near-sum launch shape: enough source splits for ~8 waves per SIMD, at
// least 128 sources per split.
NearConfig heuristic_near(int64_t N, int block, int tpt, int tile) {
  NearConfig c;
  c.block = block;
  c.tpt = tpt;
  c.tile = tile;
  const int64_t nblocks = (N + block * tpt - 1) / (block * tpt);
  const int64_t waves = nblocks * (block / 64);
  int64_t S = (8192 + waves - 1) / waves;
  S = std::max<int64_t>(1, std::min<int64_t>(S, std::max<int64_t>(1, N / 128)));
  c.splits = (int32_t)S;
  return c;
}
}  // namespace spm

namespace {

// ---------------------------------------------------------------------------
// allocation through the caller's callbacks (or hipMalloc), grow-only per slot
// ---------------------------------------------------------------------------
struct Slots {
  std::map<void**, size_t> cap;
};
std::map<const spm_handle*, Slots> g_slots;

void* raw_alloc(spm_handle* h, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 256;
  if (h->alloc) {
    p = h->alloc(bytes, (void*)h->stream, h->alloc_ctx);
    if (!p) throw ApiError(SPM_ENOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw ApiError(SPM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  return p;
}

void raw_free(spm_handle* h, void* p) {
  if (!p) return;
  if (h->free_fn)
    h->free_fn(p, (void*)h->stream, h->alloc_ctx);
  else
    (void)hipFree(p);
}

template <typename T>
void ensure(spm_handle* h, T*& p, size_t count) {
  auto& cap = g_slots[h].cap;
  void** key = reinterpret_cast<void**>(&p);
  const size_t bytes = count * sizeof(T);
  auto it = cap.find(key);
  if (it != cap.end() && it->second >= bytes && p) return;
  if (p) raw_free(h, p);
  p = static_cast<T*>(raw_alloc(h, bytes));
  cap[key] = bytes;
}

void free_all(spm_handle* h) {
  auto it = g_slots.find(h);
  if (it == g_slots.end()) return;
  for (auto& kv : it->second.cap) {
    void* p = *kv.first;
    raw_free(h, p);
    *kv.first = nullptr;
  }
  g_slots.erase(it);
}

// Setup-time upload from pageable host memory; waits so the source may be freed on return.
void upload(spm_handle* h, void* dst, const void* src, size_t bytes) {
  SPM_HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
  SPM_HIP_CHECK(hipStreamSynchronize(h->stream));
}

void sync(spm_handle* h) { SPM_HIP_CHECK(hipStreamSynchronize(h->stream)); }

bool verbose() {
  static const bool v = std::getenv("SPM_VERBOSE") != nullptr;
  return v;
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_m.
void gauss_legendre(int m, std::vector<double>& t, std::vector<double>& w) {
  t.assign(m, 0.0);
  w.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (m + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= m; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = m * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) {
        double q0 = 1.0, q1 = x;
        for (int k = 2; k <= m; ++k) {
          const double q2 = ((2.0 * k - 1.0) * x * q1 - (k - 1.0) * q0) / k;
          q0 = q1;
          q1 = q2;
        }
        const double dq = m * (x * q1 - q0) / (x * x - 1.0);
        w[i] = 2.0 / ((1.0 - x * x) * dq * dq);
        break;
      }
    }
    t[i] = x;
  }
  // ascending order (-1 -> 1)
  for (int i = 0, j = m - 1; i < j; ++i, --j) {
    std::swap(t[i], t[j]);
    std::swap(w[i], w[j]);
  }
}

int fail(spm_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

template <typename F>
int guarded(spm_handle* h, F&& f) {
  if (!h) return SPM_EINVAL;
  try {
    h->err.clear();
    return f();
  } catch (const HipError& e) {
    return fail(h, SPM_EHIP, std::string("HIP error ") + hipGetErrorString(e.code) + " in " + e.what + " (line " +
                                 std::to_string(e.line) + ")");
  } catch (const ApiError& e) {
    return fail(h, e.code, e.msg);
  } catch (const std::exception& e) {
    return fail(h, SPM_EINVAL, e.what());
  }
}

void need_particles(spm_handle* h) {
  if (!h->have_lattice || !h->have_particles) throw ApiError(SPM_ESTATE, "set the lattice and the particles first");
}

// ---------------------------------------------------------------------------
// lattice: walls, proxies, Q and its pseudo-inverse
// ---------------------------------------------------------------------------
void build_lattice(spm_handle* h) {
  Periodizer& P = h->per;
  P.m = h->cfg.m_wall;
  P.M = h->cfg.M;
  const int m = P.m, M = P.M;
  ensure(h, P.wx, 2 * m);
  ensure(h, P.wy, 2 * m);
  ensure(h, P.px, M);
  ensure(h, P.py, M);
  ensure(h, P.Q, (size_t)8 * m * 2 * M);
  ensure(h, P.Qp, (size_t)8 * m * 2 * M);
  ensure(h, P.svd_a, (size_t)8 * m * 2 * M);
  ensure(h, P.svd_v, (size_t)4 * M * M);
  ensure(h, P.svd_s, (size_t)2 * M + 1);
  std::vector<double> t, w;
  gauss_legendre(m, t, w);
  std::vector<double> wx(2 * m), wy(2 * m), px(M), py(M);
  for (int i = 0; i < m; ++i) {
    const double s = 0.5 * t[i];
    wx[i] = h->cU[0] - 0.5 * h->e1[0] + s * h->e2[0];
    wy[i] = h->cU[1] - 0.5 * h->e1[1] + s * h->e2[1];
    wx[m + i] = h->cU[0] - 0.5 * h->e2[0] + s * h->e1[0];
    wy[m + i] = h->cU[1] - 0.5 * h->e2[1] + s * h->e1[1];
  }
  for (int p = 0; p < M; ++p) {
    const double th = 2.0 * kPi * p / M;
    px[p] = h->cU[0] + h->cfg.R_proxy * std::cos(th);
    py[p] = h->cU[1] + h->cfg.R_proxy * std::sin(th);
  }
  const double l2 = std::hypot(h->e2[0], h->e2[1]);
  P.nL[0] = h->e2[1] / l2;
  P.nL[1] = -h->e2[0] / l2;
  P.nD[0] = 0.0;
  P.nD[1] = 1.0;
  upload(h, P.wx, wx.data(), 2 * m * sizeof(double));
  upload(h, P.wy, wy.data(), 2 * m * sizeof(double));
  upload(h, P.px, px.data(), M * sizeof(double));
  upload(h, P.py, py.data(), M * sizeof(double));
  launch_build_Q(h);
  launch_pinv(h);
  ensure(h, h->wk.xi, (size_t)2 * M);
  ensure(h, h->wk.scal, 16);
}

size_t max_splits(spm_handle* h) { return (size_t)std::max(h->wk.near[0].splits, h->wk.near[1].splits); }

void choose_launch(spm_handle* h) {
  const int64_t N = h->geo.N;
  Work& W = h->wk;
  if (W.tuned && W.tuned_N != N) W.tuned = false;
  if (!W.tuned) {
    W.near[0] = heuristic_near(N, 256, 1, 256);
    W.near[1] = heuristic_near(N, 256, 1, 256);
  }
  W.nchunk_disc = (int32_t)std::max<int64_t>(1, (N + 2047) / 2048);
}

void alloc_work(spm_handle* h) {
  const int64_t N = h->geo.N;
  Work& W = h->wk;
  ensure(h, W.f1, N);
  ensure(h, W.f2, N);
  ensure(h, W.f1f, N);
  ensure(h, W.f2f, N);
  ensure(h, W.T, 2 * N);
  ensure(h, W.Tpart, max_splits(h) * 2 * N);
  ensure(h, W.pF, (size_t)4 * h->geo.No);
  ensure(h, W.disc, (size_t)W.nchunk_disc * 2 * h->per.m * 4);
}

void alloc_krylov(spm_handle* h) {
  Krylov& K = h->kr;
  const int64_t n2 = 2 * h->geo.N;
  const int kmax = std::max(1, h->cfg.max_iter);
  K.kmax = kmax;
  K.n2 = n2;
  K.nchunk = (int32_t)std::min<int64_t>(256, std::max<int64_t>(1, n2 / 2048));
  ensure(h, K.V, (size_t)(kmax + 1) * n2);
  ensure(h, K.H, (size_t)(kmax + 1) * kmax);
  ensure(h, K.cs, kmax);
  ensure(h, K.sn, kmax);
  ensure(h, K.g, kmax + 1);
  ensure(h, K.yv, kmax);
  ensure(h, K.h, (size_t)2 * (kmax + 1) + 8);
  ensure(h, K.part, (size_t)K.nchunk * (kmax + 1));
  ensure(h, K.tmp, n2);
  ensure(h, K.tmp2, n2);
  ensure(h, K.res, 8);
  if (!K.host_res) SPM_HIP_CHECK(hipHostMalloc((void**)&K.host_res, 8 * sizeof(double), hipHostMallocDefault));
}

// ---------------------------------------------------------------------------
// operator
// ---------------------------------------------------------------------------
void stage_xi(spm_handle* h, const double* sigma) {
  launch_prep(h, sigma);
  launch_disc(h);
  launch_xi(h);
}

void matvec(spm_handle* h, const double* sigma, double* out, int precision) {
  stage_xi(h, sigma);
  launch_near(h, precision);
  launch_combine(h, sigma, true, precision);
  if (h->cl.ntargets > 0) {
    launch_vplus(h, sigma);
    launch_close_apply(h, sigma, h->wk.T, precision);
  }
  launch_assemble(h, sigma, out);
}

double host_dot(spm_handle* h, const double* a, const double* b) {
  double* out = h->kr.res + 4;
  gm_dot_many(h, a, 0, 1, b, out);
  SPM_HIP_CHECK(hipMemcpyAsync(h->kr.host_res + 4, out, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  sync(h);
  return h->kr.host_res[4];
}

struct KrylovResult {
  int iterations = 0;
  bool converged = false;
  double est = 0.0;
};

// GMRES for A x = b (A at `precision`), x holds the initial guess if x_nonzero.
// Stops when |g_{j+1}| <= tol * bnorm.
KrylovResult gmres(spm_handle* h, int precision, const double* b, double* x, bool x_nonzero, double tol, int maxit,
                   double bnorm, spm_solve_info* info) {
  Krylov& K = h->kr;
  const int64_t n2 = K.n2;
  double* V = K.V;
  double* h1 = K.h;
  double* h2 = K.h + K.kmax + 1;
  double* nrm2 = K.h + 2 * (K.kmax + 1);
  KrylovResult R;
  if (x_nonzero) {
    matvec(h, x, K.tmp, precision);
    if (precision == SPM_FP64) info->fp64_matvecs++; else info->fp32_matvecs++;
    gm_axpby(h, n2, 1.0, b, -1.0, K.tmp, V);
  } else {
    gm_copy(h, V, b, n2);
  }
  gm_dot_many(h, V, 0, 1, V, nrm2);
  gm_init(h, nrm2);
  gm_scale_by_norm(h, nrm2, V, n2, nullptr);
  SPM_HIP_CHECK(hipMemcpyAsync(K.host_res, nrm2, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  sync(h);
  const double beta = std::sqrt(K.host_res[0]);
  R.est = beta / bnorm;
  if (beta <= tol * bnorm) {
    R.converged = true;
    return R;
  }
  maxit = std::min(maxit, K.kmax);
  int k = 0;
  for (int j = 0; j < maxit; ++j) {
    double* w = V + (int64_t)(j + 1) * n2;
    matvec(h, V + (int64_t)j * n2, w, precision);
    if (precision == SPM_FP64) info->fp64_matvecs++; else info->fp32_matvecs++;
    gm_dot_many(h, V, n2, j + 1, w, h1);
    gm_update(h, V, n2, j + 1, h1, w, -1.0);
    gm_dot_many(h, V, n2, j + 1, w, h2);
    gm_update(h, V, n2, j + 1, h2, w, -1.0);
    gm_dot_many(h, w, 0, 1, w, nrm2);
    gm_scale_by_norm(h, nrm2, w, n2, nullptr);
    gm_givens(h, j, h1, h2, nrm2, bnorm, K.res);
    SPM_HIP_CHECK(hipMemcpyAsync(K.host_res, K.res, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    sync(h);
    k = j + 1;
    R.est = K.host_res[0];
    if (!std::isfinite(R.est)) throw ApiError(SPM_EHIP, "GMRES residual is not finite");
    if (R.est <= tol) {
      R.converged = true;
      break;
    }
  }
  R.iterations = k;
  if (k > 0) {
    gm_backsolve(h, k);
    gm_update(h, V, n2, k, K.yv, x, 1.0);
  }
  return R;
}

double true_residual(spm_handle* h, const double* b, const double* x, double bnorm, spm_solve_info* info) {
  Krylov& K = h->kr;
  matvec(h, x, K.tmp, SPM_FP64);
  info->fp64_matvecs++;
  gm_axpby(h, K.n2, 1.0, b, -1.0, K.tmp, K.tmp2);
  return std::sqrt(host_dot(h, K.tmp2, K.tmp2)) / bnorm;
}

int solve_impl(spm_handle* h, const double* sigma0, double* sigma, spm_solve_info* info) {
  Krylov& K = h->kr;
  const int64_t n2 = K.n2;
  ensure(h, K.b, n2);
  double* bb = K.b;
  launch_rhs(h, bb);
  const double bnorm = std::sqrt(host_dot(h, bb, bb));
  if (sigma0)
    gm_copy(h, sigma, sigma0, n2);
  else
    gm_zero(h, sigma, n2);
  bool nonzero = sigma0 != nullptr;
  const double tol = h->cfg.tol;
  int status = SPM_OK;
  if (h->cfg.precision == SPM_FP32_IR) {
    double rel = nonzero ? true_residual(h, bb, sigma, bnorm, info) : 1.0;
    if (!nonzero) gm_copy(h, K.tmp2, bb, n2);
    int outer = 0;
    // inner tolerance: cfg.inner_tol, raised to half the reduction the previous
    // refinement actually achieved (the FP32 operator error bounds what one
    // refinement can gain; solving the inner system deeper than that is wasted)
    double itol_next = h->cfg.inner_tol;
    while (rel > tol && outer < 40) {
      ensure(h, K.d, n2);
      double* d = K.d;
      double* r = K.tmp2;
      const double rnorm = rel * bnorm;
      double itol = itol_next;
      if (tol / rel > itol) itol = 0.5 * tol / rel;
      gm_zero(h, d, n2);
      KrylovResult kr = gmres(h, SPM_FP32, r, d, false, itol, h->cfg.max_iter, rnorm, info);
      info->iterations += kr.iterations;
      gm_axpby(h, n2, 1.0, sigma, 1.0, d, sigma);
      ++outer;
      const double rel_new = true_residual(h, bb, sigma, bnorm, info);
      const double rho = rel_new / rel;
      if (verbose())
        std::fprintf(stderr, "[spm] refinement %d: inner its %d (inner tol %.1e, est %.1e) FP64 residual %.3e -> %.3e\n",
                     outer, kr.iterations, itol, kr.est, rel, rel_new);
      itol_next = std::min(0.1, std::max(h->cfg.inner_tol, 0.5 * rho));
      rel = rel_new;
      if (kr.iterations >= h->cfg.max_iter && rel > tol) {
        status = SPM_ENOCONV;
        break;
      }
    }
    info->refinements = outer;
    info->rel_residual = rel;
    if (rel > tol) status = SPM_ENOCONV;
  } else {
    int used = 0;
    double rel = 1.0;
    for (int restart = 0; restart < 6; ++restart) {
      KrylovResult kr = gmres(h, SPM_FP64, bb, sigma, nonzero, tol, h->cfg.max_iter - used, bnorm, info);
      used += kr.iterations;
      info->iterations += kr.iterations;
      nonzero = true;
      rel = true_residual(h, bb, sigma, bnorm, info);
      if (rel <= tol || used >= h->cfg.max_iter) break;
    }
    info->rel_residual = rel;
    if (rel > tol) status = SPM_ENOCONV;
  }
  info->status = status;
  return status;
}

void readout(spm_handle* h, const double* sigma, double* vel, double* omega, double* mu_eff) {
  stage_xi(h, sigma);
  if (vel || omega) launch_velocities(h, vel, omega);
  if (mu_eff) launch_mu_eff(h, mu_eff);
}

}  // namespace

namespace spm {
void ensure_tpart(spm_handle* h, size_t splits) {
  const size_t need = std::max(splits, max_splits(h));
  ensure(h, h->wk.Tpart, need * 2 * h->geo.N);
}
void launch_prep_for_timing(spm_handle* h) {
  // fill the force arrays from the right-hand side so the timed kernels see finite data
  launch_rhs(h, h->kr.tmp);
  launch_prep(h, h->kr.tmp);
  sync(h);
}
}  // namespace spm

// ===========================================================================
extern "C" {

void spm_default_config(spm_config* c) {
  if (!c) return;
  c->mu = 1.0;
  c->gamma = 1.0;
  c->M = 32;
  c->R_proxy = 1.5;
  c->m_wall = 24;
  c->close_factor = 10.0;
  c->tol = 1e-10;
  c->max_iter = 500;
  c->precision = SPM_FP64;
  c->inner_tol = 1e-5;
  c->min_gap = 0.0;
  c->rcond = 1e-14;
}

int spm_create(spm_handle** out, const spm_config* cfg, void* stream, spm_alloc_fn alloc, spm_free_fn free_fn,
               void* ctx) {
  if (!out) return SPM_EINVAL;
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) return SPM_EINVAL;
  spm_handle* h = new spm_handle();
  if (cfg)
    h->cfg = *cfg;
  else
    spm_default_config(&h->cfg);
  const spm_config& c = h->cfg;
  if (!(c.mu > 0) || !(c.gamma > 0) || c.M < 4 || c.M > 512 || c.m_wall < 4 || c.m_wall > 256 || !(c.R_proxy > 0.75) ||
      !(c.tol > 0) || c.max_iter < 1 || c.max_iter > 5000 || c.close_factor < 0 ||
      (c.precision != SPM_FP64 && c.precision != SPM_FP32_IR) || !(c.inner_tol > 0 && c.inner_tol < 1)) {
    delete h;
    return SPM_EINVAL;
  }
  h->stream = (hipStream_t)stream;
  h->alloc = alloc;
  h->free_fn = free_fn;
  h->alloc_ctx = ctx;
  *out = h;
  return SPM_OK;
}

void spm_destroy(spm_handle* h) {
  if (!h) return;
  try {
    (void)hipStreamSynchronize(h->stream);
    free_all(h);
    if (h->kr.host_res) (void)hipHostFree(h->kr.host_res);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  } catch (...) {
  }
  delete h;
}

const char* spm_last_error(const spm_handle* h) { return h ? h->err.c_str() : "null handle"; }

int spm_set_lattice(spm_handle* h, const double e1[2], const double e2[2], const double center[2]) {
  return guarded(h, [&]() {
    if (!e1 || !e2) throw ApiError(SPM_EINVAL, "null lattice vector");
    if (e1[0] != 1.0 || e1[1] != 0.0 || e2[1] != 1.0 || !std::isfinite(e2[0]))
      throw ApiError(SPM_EINVAL, "lattice must be e1 = (1, 0), e2 = (s, 1)");
    h->skew_raw = e2[0];
    const double s = e2[0] - std::floor(e2[0] + 0.5);
    h->skew = s;
    h->e1[0] = 1.0;
    h->e1[1] = 0.0;
    h->e2[0] = s;
    h->e2[1] = 1.0;
    h->cU[0] = center ? center[0] : 0.0;
    h->cU[1] = center ? center[1] : 0.0;
    build_lattice(h);
    sync(h);
    h->have_lattice = true;
    h->have_particles = false;
    return SPM_OK;
  });
}

int spm_set_ellipses(spm_handle* h, int32_t n, const double* centers, const double* theta, const double* a,
                     const double* b, const int32_t* n_nodes) {
  return guarded(h, [&]() {
    if (!h->have_lattice) throw ApiError(SPM_ESTATE, "set the lattice first");
    if (n < 1 || !centers || !theta || !a || !b || !n_nodes) throw ApiError(SPM_EINVAL, "bad particle arrays");
    h->cx.resize(n);
    h->cy.resize(n);
    h->th.assign(theta, theta + n);
    h->a.assign(a, a + n);
    h->b.assign(b, b + n);
    h->nn.assign(n_nodes, n_nodes + n);
    h->off.assign(n + 1, 0);
    // wrap centres: (alpha, beta) = [e1 e2]^{-1} (c - c_U), reduced to [-1/2, 1/2)
    const double det = h->e1[0] * h->e2[1] - h->e1[1] * h->e2[0];
    for (int i = 0; i < n; ++i) {
      if (!(a[i] > 0) || !(b[i] > 0) || !std::isfinite(centers[2 * i]) || !std::isfinite(centers[2 * i + 1]) ||
          !std::isfinite(theta[i]))
        throw ApiError(SPM_EINVAL, "bad ellipse " + std::to_string(i));
      if (n_nodes[i] < 8 || n_nodes[i] > kMaxNodesPerParticle || (n_nodes[i] & 1))
        throw ApiError(SPM_EINVAL, "node count must be even and in [8, 512]");
      if (std::max(a[i], b[i]) >= 0.45) throw ApiError(SPM_EINVAL, "ellipse larger than the 3x3 image rule allows");
      const double dx = centers[2 * i] - h->cU[0], dy = centers[2 * i + 1] - h->cU[1];
      double al = (dx * h->e2[1] - dy * h->e2[0]) / det;
      double be = (h->e1[0] * dy - h->e1[1] * dx) / det;
      al -= std::floor(al + 0.5);
      be -= std::floor(be + 0.5);
      h->cx[i] = h->cU[0] + al * h->e1[0] + be * h->e2[0];
      h->cy[i] = h->cU[1] + al * h->e1[1] + be * h->e2[1];
      h->off[i + 1] = h->off[i] + n_nodes[i];
    }
    Geo& g = h->geo;
    g.No = n;
    g.N = h->off[n];
    const int64_t N = g.N;
    ensure(h, g.x, N);
    ensure(h, g.y, N);
    ensure(h, g.nx, N);
    ensure(h, g.ny, N);
    ensure(h, g.w, N);
    ensure(h, g.kap, N);
    ensure(h, g.tx, N);
    ensure(h, g.ty, N);
    ensure(h, g.xpx, N);
    ensure(h, g.xpy, N);
    ensure(h, g.xf, N);
    ensure(h, g.yf, N);
    ensure(h, g.nxf, N);
    ensure(h, g.nyf, N);
    ensure(h, g.pid, N);
    ensure(h, g.pcx, n);
    ensure(h, g.pcy, n);
    ensure(h, g.pth, n);
    ensure(h, g.pa, n);
    ensure(h, g.pb, n);
    ensure(h, g.pper, n);
    ensure(h, g.poff, n + 1);
    ensure(h, g.pn, n);
    std::vector<int32_t> pid(N);
    for (int i = 0; i < n; ++i)
      for (int k = h->off[i]; k < h->off[i + 1]; ++k) pid[k] = i;
    upload(h, g.pid, pid.data(), N * sizeof(int32_t));
    upload(h, g.pcx, h->cx.data(), n * sizeof(double));
    upload(h, g.pcy, h->cy.data(), n * sizeof(double));
    upload(h, g.pth, h->th.data(), n * sizeof(double));
    upload(h, g.pa, h->a.data(), n * sizeof(double));
    upload(h, g.pb, h->b.data(), n * sizeof(double));
    upload(h, g.poff, h->off.data(), (n + 1) * sizeof(int32_t));
    upload(h, g.pn, h->nn.data(), n * sizeof(int32_t));
    launch_geometry(h);
    // close pairs + overlap check
    CloseList& C = h->cl;
    ensure(h, C.count, N);
    ensure(h, C.row, N + 1);
    ensure(h, C.tlist, N);
    ensure(h, C.dmin, N);
    ensure(h, C.inside, N);
    ensure(h, C.vp, 6 * N);
    launch_close_count(h);
    double gap;
    int32_t overlap;
    launch_gap(h, &gap, &overlap);
    h->min_gap_est = gap;
    if (overlap || (h->cfg.min_gap > 0 && gap < h->cfg.min_gap)) {
      h->have_particles = false;
      throw ApiError(SPM_EOVERLAP, overlap ? "particles overlap" : "particles closer than min_gap");
    }
    int32_t total, nt;
    launch_close_scan(h, &total, &nt);
    C.npairs = total;
    C.ntargets = nt;
    ensure(h, C.q, std::max<int64_t>(1, total));
    ensure(h, C.s, std::max<int64_t>(1, total));
    if (total > 0) launch_close_fill(h);
    choose_launch(h);
    alloc_work(h);
    alloc_krylov(h);
    sync(h);
    h->have_particles = true;
    return SPM_OK;
  });
}

int spm_num_nodes(const spm_handle* h, int64_t* N) {
  if (!h || !N) return SPM_EINVAL;
  if (!h->have_particles) return SPM_ESTATE;
  *N = h->geo.N;
  return SPM_OK;
}

int spm_num_particles(const spm_handle* h, int32_t* n) {
  if (!h || !n) return SPM_EINVAL;
  if (!h->have_particles) return SPM_ESTATE;
  *n = h->geo.No;
  return SPM_OK;
}

int spm_get_nodes(spm_handle* h, double* x, double* y, double* nx, double* ny, double* w) {
  return guarded(h, [&]() {
    need_particles(h);
    const size_t bytes = h->geo.N * sizeof(double);
    if (x) SPM_HIP_CHECK(hipMemcpyAsync(x, h->geo.x, bytes, hipMemcpyDeviceToDevice, h->stream));
    if (y) SPM_HIP_CHECK(hipMemcpyAsync(y, h->geo.y, bytes, hipMemcpyDeviceToDevice, h->stream));
    if (nx) SPM_HIP_CHECK(hipMemcpyAsync(nx, h->geo.nx, bytes, hipMemcpyDeviceToDevice, h->stream));
    if (ny) SPM_HIP_CHECK(hipMemcpyAsync(ny, h->geo.ny, bytes, hipMemcpyDeviceToDevice, h->stream));
    if (w) SPM_HIP_CHECK(hipMemcpyAsync(w, h->geo.w, bytes, hipMemcpyDeviceToDevice, h->stream));
    sync(h);
    return SPM_OK;
  });
}

int spm_get_centers(spm_handle* h, double* c) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!c) throw ApiError(SPM_EINVAL, "null output");
    for (int i = 0; i < h->geo.No; ++i) {
      c[2 * i] = h->cx[i];
      c[2 * i + 1] = h->cy[i];
    }
    return SPM_OK;
  });
}

int spm_apply(spm_handle* h, const double* sigma, double* out, int32_t precision) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma || !out) throw ApiError(SPM_EINVAL, "null vector");
    if (precision != SPM_FP64 && precision != SPM_FP32) throw ApiError(SPM_EINVAL, "precision must be FP64 or FP32");
    matvec(h, sigma, out, precision);
    sync(h);
    return SPM_OK;
  });
}

int spm_rhs(spm_handle* h, double* out) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!out) throw ApiError(SPM_EINVAL, "null vector");
    launch_rhs(h, out);
    sync(h);
    return SPM_OK;
  });
}

int spm_solve(spm_handle* h, const double* sigma0, double* sigma, double* vel, double* omega, double* mu_eff,
              spm_solve_info* info_out) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma) throw ApiError(SPM_EINVAL, "null sigma");
    spm_solve_info info;
    std::memset(&info, 0, sizeof(info));
    info.n_close_pairs = (int32_t)h->cl.npairs;
    const double t0 = now();
    const int st = solve_impl(h, sigma0, sigma, &info);
    sync(h);
    const double t1 = now();
    readout(h, sigma, vel, omega, mu_eff);
    sync(h);
    info.seconds_solve = t1 - t0;
    info.seconds_readout = now() - t1;
    if (info_out) *info_out = info;
    if (st == SPM_ENOCONV) h->err = "GMRES did not reach the tolerance; outputs hold the last iterate";
    return st;
  });
}

int spm_velocities(spm_handle* h, const double* sigma, double* vel, double* omega) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma) throw ApiError(SPM_EINVAL, "null sigma");
    readout(h, sigma, vel, omega, nullptr);
    sync(h);
    return SPM_OK;
  });
}

int spm_effective_viscosity(spm_handle* h, const double* sigma, double* mu_eff) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma || !mu_eff) throw ApiError(SPM_EINVAL, "null pointer");
    launch_prep(h, sigma);
    launch_mu_eff(h, mu_eff);
    sync(h);
    return SPM_OK;
  });
}

int spm_near_traction(spm_handle* h, const double* sigma, double* out, int32_t precision) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma || !out) throw ApiError(SPM_EINVAL, "null vector");
    if (precision != SPM_FP64 && precision != SPM_FP32) throw ApiError(SPM_EINVAL, "precision must be FP64 or FP32");
    launch_prep(h, sigma);
    launch_near(h, precision);
    launch_near_sum_only(h, out, precision);
    sync(h);
    return SPM_OK;
  });
}

int spm_close_correction(spm_handle* h, const double* sigma, double* out, int32_t precision) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma || !out) throw ApiError(SPM_EINVAL, "null vector");
    if (precision != SPM_FP64 && precision != SPM_FP32) throw ApiError(SPM_EINVAL, "precision must be FP64 or FP32");
    launch_prep(h, sigma);
    gm_zero(h, out, 2 * h->geo.N);
    if (h->cl.ntargets > 0) {
      launch_vplus(h, sigma);
      launch_close_apply(h, sigma, out, precision);
    }
    sync(h);
    return SPM_OK;
  });
}

int spm_proxy_strengths(spm_handle* h, const double* sigma, double* xi) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma || !xi) throw ApiError(SPM_EINVAL, "null vector");
    stage_xi(h, sigma);
    SPM_HIP_CHECK(hipMemcpyAsync(xi, h->wk.xi, 2 * h->per.M * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    sync(h);
    return SPM_OK;
  });
}

int spm_close_pairs(spm_handle* h, int64_t* count, int32_t* target, int32_t* particle, int32_t* shift,
                    int64_t capacity) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!count) throw ApiError(SPM_EINVAL, "null count");
    *count = h->cl.npairs;
    if (!target && !particle && !shift) return SPM_OK;
    if (capacity < h->cl.npairs) throw ApiError(SPM_EINVAL, "capacity too small");
    const int64_t N = h->geo.N, P = h->cl.npairs;
    std::vector<int32_t> row(N + 1), q(std::max<int64_t>(P, 1)), s(std::max<int64_t>(P, 1));
    SPM_HIP_CHECK(hipMemcpyAsync(row.data(), h->cl.row, (N + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    if (P > 0) {
      SPM_HIP_CHECK(hipMemcpyAsync(q.data(), h->cl.q, P * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
      SPM_HIP_CHECK(hipMemcpyAsync(s.data(), h->cl.s, P * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    }
    sync(h);
    for (int64_t i = 0; i < N; ++i)
      for (int32_t e = row[i]; e < row[i + 1]; ++e) {
        if (target) target[e] = (int32_t)i;
        if (particle) particle[e] = q[e];
        if (shift) shift[e] = s[e];
      }
    return SPM_OK;
  });
}

int spm_proxy_pinv(spm_handle* h, double* out) {
  return guarded(h, [&]() {
    if (!h->have_lattice) throw ApiError(SPM_ESTATE, "set the lattice first");
    if (!out) throw ApiError(SPM_EINVAL, "null output");
    const size_t n = (size_t)8 * h->per.m * 2 * h->per.M;
    SPM_HIP_CHECK(hipMemcpyAsync(out, h->per.Qp, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    sync(h);
    return SPM_OK;
  });
}

int spm_step(spm_handle* h, double dt, int32_t n_steps, double* t_inout, double* centers, double* theta,
             double* mu_series, spm_solve_info* infos) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!t_inout || !centers || !theta || !mu_series || n_steps < 1 || !(dt > 0))
      throw ApiError(SPM_EINVAL, "bad step arguments");
    const int n = h->geo.No;
    std::vector<double> a(h->a), b(h->b);
    std::vector<int32_t> nn(h->nn);
    const double s0 = h->skew_raw;
    const double t0 = *t_inout;
    double *sig = nullptr, *vel = nullptr, *om = nullptr, *mu = nullptr;
    const int64_t n2 = 2 * h->geo.N;
    ensure(h, h->kr.stepbuf, n2 + 3 * n + 2);
    double* buf = h->kr.stepbuf;
    sig = buf;
    vel = buf + n2;
    om = vel + 2 * n;
    mu = om + n;
    std::vector<double> hv(3 * n + 1);
    bool have_prev = false;
    for (int k = 0; k < n_steps; ++k) {
      const double t = k * dt;  // elapsed since entry
      const double e1[2] = {1.0, 0.0};
      const double e2[2] = {s0 + h->cfg.gamma * t, 1.0};
      const double cU[2] = {h->cU[0], h->cU[1]};
      int rc = spm_set_lattice(h, e1, e2, cU);
      if (rc) return rc;
      h->skew_raw = s0;  // keep the reference skew of this call
      rc = spm_set_ellipses(h, n, centers, theta, a.data(), b.data(), nn.data());
      if (rc) return rc;
      spm_solve_info info;
      rc = spm_solve(h, have_prev ? sig : nullptr, sig, vel, om, mu, &info);
      if (rc && rc != SPM_ENOCONV) return rc;
      have_prev = true;
      SPM_HIP_CHECK(hipMemcpyAsync(hv.data(), vel, (3 * n + 1) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      sync(h);
      mu_series[k] = hv[3 * n];
      if (infos) infos[k] = info;
      for (int i = 0; i < n; ++i) {
        centers[2 * i] = h->cx[i] + dt * hv[2 * i];
        centers[2 * i + 1] = h->cy[i] + dt * hv[2 * i + 1];
        theta[i] += dt * hv[2 * n + i];
      }
      if (rc == SPM_ENOCONV) return rc;
    }
    *t_inout = t0 + n_steps * dt;
    h->skew_raw = s0 + h->cfg.gamma * n_steps * dt;
    return SPM_OK;
  });
}

int spm_proxy_svd(spm_handle* h, double* Q_host, double* s_host, int32_t* sweeps_host) {
  return guarded(h, [&]() {
    if (!h->have_lattice) throw ApiError(SPM_ESTATE, "set the lattice first");
    const size_t n = (size_t)8 * h->per.m * 2 * h->per.M;
    if (Q_host) SPM_HIP_CHECK(hipMemcpyAsync(Q_host, h->per.Q, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if (s_host)
      SPM_HIP_CHECK(hipMemcpyAsync(s_host, h->per.svd_s, 2 * h->per.M * sizeof(double), hipMemcpyDeviceToHost,
                                   h->stream));
    double sw = 0;
    SPM_HIP_CHECK(hipMemcpyAsync(&sw, h->per.svd_s + 2 * h->per.M, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    sync(h);
    if (sweeps_host) *sweeps_host = (int32_t)sw;
    return SPM_OK;
  });
}

int spm_autotune(spm_handle* h, const char* cache_path, double* best_ms_host) {
  return guarded(h, [&]() {
    need_particles(h);
    autotune(h, cache_path, best_ms_host);
    sync(h);
    return SPM_OK;
  });
}

int spm_get_launch(spm_handle* h, int32_t precision, int32_t* cfg_host) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!cfg_host || (precision != SPM_FP64 && precision != SPM_FP32)) throw ApiError(SPM_EINVAL, "bad arguments");
    const NearConfig& c = h->wk.near[precision == SPM_FP64 ? 0 : 1];
    cfg_host[0] = c.block;
    cfg_host[1] = c.tpt;
    cfg_host[2] = c.tile;
    cfg_host[3] = c.splits;
    return SPM_OK;
  });
}

int spm_set_launch(spm_handle* h, int32_t precision, const int32_t* cfg_host) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!cfg_host || (precision != SPM_FP64 && precision != SPM_FP32)) throw ApiError(SPM_EINVAL, "bad arguments");
    NearConfig c;
    c.block = cfg_host[0];
    c.tpt = cfg_host[1];
    c.tile = cfg_host[2];
    c.splits = cfg_host[3];
    if (!near_config_valid(c)) throw ApiError(SPM_EINVAL, "unsupported near-sum launch configuration");
    ensure_tpart(h, (size_t)c.splits);
    h->wk.near[precision == SPM_FP64 ? 0 : 1] = c;
    h->wk.tuned = true;
    h->wk.tuned_N = h->geo.N;
    return SPM_OK;
  });
}

int spm_profile(spm_handle* h, int32_t enable) {
  return guarded(h, [&]() {
    prof_flush(h);
    h->prof = enable != 0;
    for (int k = 0; k < 2; ++k) {
      h->prof_ms[k] = 0;
      h->prof_launches[k] = 0;
      h->prof_pairs[k] = 0;
    }
    return SPM_OK;
  });
}

int spm_profile_read(spm_handle* h, int32_t kernel, double* total_ms, int64_t* launches, double* pairs) {
  return guarded(h, [&]() {
    if (kernel < 0 || kernel > 1) throw ApiError(SPM_EINVAL, "kernel id must be 0 (FP64 near sum) or 1 (FP32)");
    prof_flush(h);
    if (total_ms) *total_ms = h->prof_ms[kernel];
    if (launches) *launches = h->prof_launches[kernel];
    if (pairs) *pairs = h->prof_pairs[kernel];
    return SPM_OK;
  });
}

}  // extern "C"
