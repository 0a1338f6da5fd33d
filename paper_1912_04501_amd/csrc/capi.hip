// C ABI of the solver: handle, setup of an ensemble of cells, matvec pipeline, GMRES
// driver (FP64 and FP32 + FP64 iterative refinement), readouts, time stepping.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <thread>
#include <tuple>
#include <utility>

#include "spm_internal.h"

using namespace spm;

namespace spm {
// Default near-sum launch shape: 256 threads, 256-source LDS tiles; FP64 with four targets
// per lane (the FP64 pair is ALU-heavier, so reusing each staged source for more targets
// pays), FP32 with one; as many persistent workgroups as fit on a compute unit.
// Launch shape of the near sum before (or without) autotuning: one target per lane in blocks of
// 64 against tiles of 128 sources in both precisions. Small blocks and tiles give many units
// (target block, source tile) for the persistent grid to share out even at a few thousand nodes,
// and at N = 51,200 this shape is within 1% of the autotuner's best in either precision.
NearConfig heuristic_near(spm_handle* h, int precision) {
  (void)h;
  (void)precision;
  NearConfig c;
  c.block = 64;
  c.tpt = 1;
  c.tile = 128;
  c.wg_per_cu = 0;
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
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
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

void sync(spm_handle* h) { SPM_HIP_CHECK(hipStreamSynchronize(h->stream)); }

// Setup-time upload from pageable host memory; waits so the source may be freed on return.
void upload(spm_handle* h, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  SPM_HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
  SPM_HIP_CHECK(hipStreamSynchronize(h->stream));
}

void download(spm_handle* h, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  SPM_HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream));
  SPM_HIP_CHECK(hipStreamSynchronize(h->stream));
}

bool verbose() {
  static const bool v = std::getenv("SPM_VERBOSE") != nullptr;
  return v;
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Gauss-Legendre nodes/weights on [-1, 1] (ascending) by Newton iteration on P_m.
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
  if (!h->have_particles) throw ApiError(SPM_ESTATE, "set the lattice and the particles (or the cells) first");
}

void drop_graphs(spm_handle* h) {
  for (int k = 0; k < 4; ++k) {
    if (h->kr.graph[k]) (void)hipGraphExecDestroy(h->kr.graph[k]);
    if (h->kr.graph_src[k]) (void)hipGraphDestroy(h->kr.graph_src[k]);
    h->kr.graph[k] = nullptr;
    h->kr.graph_src[k] = nullptr;
  }
}

template <typename T>
T* host_scratch(spm_handle* h, size_t count) {
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (h->kr.host_bytes < bytes) {
    if (h->kr.host) SPM_HIP_CHECK(hipHostFree(h->kr.host));
    h->kr.host = nullptr;
    SPM_HIP_CHECK(hipHostMalloc(&h->kr.host, bytes, hipHostMallocDefault));
    h->kr.host_bytes = bytes;
  }
  return static_cast<T*>(h->kr.host);
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
void build_periodizers(spm_handle* h) {
  Periodizer& P = h->per;
  const int C = h->geo.C;
  P.m = h->cfg.m_wall;
  P.M = h->cfg.M;
  const int m = P.m, M = P.M;
  ensure(h, P.wx, (size_t)C * 2 * m);
  ensure(h, P.wy, (size_t)C * 2 * m);
  ensure(h, P.px, (size_t)C * M);
  ensure(h, P.py, (size_t)C * M);
  ensure(h, P.Q, (size_t)C * 8 * m * 2 * M);
  ensure(h, P.Qp, (size_t)C * 8 * m * 2 * M);
  ensure(h, P.svd_a, (size_t)C * 8 * m * 2 * M);
  {
    // the previous V's warm-start the SVD only for the same number of cells and sizes
    double* before = P.svd_v;
    ensure(h, P.svd_v, (size_t)C * 4 * M * M);
    if (P.svd_v != before || C != P.warm_C || m != P.warm_m || M != P.warm_M) P.warm_ok = false;
    P.warm_C = C;
    P.warm_m = m;
    P.warm_M = M;
  }
  ensure(h, P.svd_s, (size_t)C * (2 * M + 1));
  std::vector<double> t, w;
  gauss_legendre(m, t, w);
  std::vector<double> wx((size_t)C * 2 * m), wy((size_t)C * 2 * m), px, py;
  for (int c = 0; c < C; ++c) {
    const double s = h->cells[c].skew;
    for (int i = 0; i < m; ++i) {
      const double u = 0.5 * t[i];
      // L(u) = c_U - e1/2 + u e2 ; D(u) = c_U - e2/2 + u e1
      wx[(size_t)c * 2 * m + i] = h->cU[0] - 0.5 + u * s;
      wy[(size_t)c * 2 * m + i] = h->cU[1] + u;
      wx[(size_t)c * 2 * m + m + i] = h->cU[0] - 0.5 * s + u;
      wy[(size_t)c * 2 * m + m + i] = h->cU[1] - 0.5;
    }
  }
  // proxies of every cell: M on a circle about c_U (3x3 near set) or M/4 on each wall of the
  // dilated cell U~ = c_U + [-1, 1) e1 + [-1, 1) e2, at the midpoints of equal parameter
  // intervals, counter-clockwise from the bottom side (dilated near set, Sec. 6.1 remark)
  px.assign((size_t)C * M, 0.0);
  py.assign((size_t)C * M, 0.0);
  for (int c = 0; c < C; ++c) {
    const double sk = h->cells[c].skew;
    for (int p = 0; p < M; ++p) {
      double X, Y;
      if (h->cfg.near_set == SPM_NEAR_SET_DILATED) {
        const int k = M / 4, side = p / k;
        const double t = -1.0 + (p % k + 0.5) * (2.0 / k);
        double a = 0, b = 0;   // lattice coordinates
        if (side == 0) { a = t; b = -1.0; }
        else if (side == 1) { a = 1.0; b = t; }
        else if (side == 2) { a = -t; b = 1.0; }
        else { a = -1.0; b = -t; }
        X = h->cU[0] + a + b * sk;
        Y = h->cU[1] + b;
      } else {
        const double th = 2.0 * kPi * p / M;
        X = h->cU[0] + h->cfg.R_proxy * std::cos(th);
        Y = h->cU[1] + h->cfg.R_proxy * std::sin(th);
      }
      px[(size_t)c * M + p] = X;
      py[(size_t)c * M + p] = Y;
    }
  }
  upload(h, P.wx, wx.data(), wx.size() * sizeof(double));
  upload(h, P.wy, wy.data(), wy.size() * sizeof(double));
  upload(h, P.px, px.data(), px.size() * sizeof(double));
  upload(h, P.py, py.data(), py.size() * sizeof(double));
  launch_build_Q(h);
  launch_pinv(h);
  ensure(h, h->wk.xi, (size_t)C * 2 * M);
}

// work items of the wall discrepancy (source chunks of each cell) and the dot segments
void build_chunks(spm_handle* h) {
  const int C = h->geo.C;
  std::vector<int64_t> s0, s1, n0, n1;
  std::vector<int32_t> cc, off(C + 1, 0), sc, soff(C + 1, 0);
  for (int c = 0; c < C; ++c) {
    const int64_t a = h->cells[c].n0, b = h->cells[c].n1;
    for (int64_t x = a; x < b; x += 2048) {   // wall-discrepancy chunks: 8 sources per thread
      s0.push_back(x);
      s1.push_back(std::min(b, x + 2048));
      cc.push_back(c);
    }
    off[c + 1] = (int32_t)s0.size();
    for (int64_t x = a; x < b; x += 1024) {
      n0.push_back(x);
      n1.push_back(std::min(b, x + 1024));
      sc.push_back(c);
    }
    soff[c + 1] = (int32_t)n0.size();
  }
  Work& W = h->wk;
  W.ndisc = (int32_t)s0.size();
  ensure(h, W.disc_s0, s0.size());
  ensure(h, W.disc_s1, s1.size());
  ensure(h, W.disc_cell, cc.size());
  ensure(h, W.disc_off, C + 1);
  upload(h, W.disc_s0, s0.data(), s0.size() * sizeof(int64_t));
  upload(h, W.disc_s1, s1.data(), s1.size() * sizeof(int64_t));
  upload(h, W.disc_cell, cc.data(), cc.size() * sizeof(int32_t));
  upload(h, W.disc_off, off.data(), off.size() * sizeof(int32_t));
  ensure(h, W.disc, (size_t)W.ndisc * 2 * h->per.m * 8);
  Krylov& K = h->kr;
  K.nseg = (int32_t)n0.size();
  ensure(h, K.seg_n0, n0.size());
  ensure(h, K.seg_n1, n1.size());
  ensure(h, K.seg_cell, sc.size());
  ensure(h, K.seg_off, C + 1);
  upload(h, K.seg_n0, n0.data(), n0.size() * sizeof(int64_t));
  upload(h, K.seg_n1, n1.data(), n1.size() * sizeof(int64_t));
  upload(h, K.seg_cell, sc.data(), sc.size() * sizeof(int32_t));
  upload(h, K.seg_off, soff.data(), soff.size() * sizeof(int32_t));
}

void alloc_work(spm_handle* h) {
  const int64_t N = h->geo.N;
  Work& W = h->wk;
  ensure(h, W.f1, N);
  ensure(h, W.f2, N);
  ensure(h, W.f1f, N);
  ensure(h, W.f2f, N);
  ensure(h, W.T, 2 * N);
  ensure(h, W.pF, (size_t)4 * h->geo.No);
  ensure(h, W.scal, 16);
  ensure(h, W.gauge, (size_t)2 * h->geo.C);
}

void alloc_krylov(spm_handle* h) {
  Krylov& K = h->kr;
  const int64_t n2 = 2 * h->geo.N;
  const int C = h->geo.C;
  const int kmax = std::max(2, h->cfg.max_iter);
  K.kmax = kmax;
  K.n2 = n2;
  ensure(h, K.V, (size_t)(kmax + 1) * n2);
  ensure(h, K.H, (size_t)C * kmax * (kmax + 1));
  ensure(h, K.cs, (size_t)C * kmax);
  ensure(h, K.sn, (size_t)C * kmax);
  ensure(h, K.g, (size_t)C * (kmax + 1));
  ensure(h, K.yv, (size_t)C * kmax);
  ensure(h, K.h1, (size_t)C * (kmax + 1));
  ensure(h, K.h2, (size_t)C * (kmax + 1));
  ensure(h, K.nrm2, C);
  ensure(h, K.bnorm, C);
  ensure(h, K.tolc, C);
  ensure(h, K.res, C);
  ensure(h, K.active, C);
  ensure(h, K.kdone, C);
  ensure(h, K.mask, C);
  ensure(h, K.stamp, C + 2);
  ensure(h, K.jdev, 2);
  ensure(h, K.gcount, 1);
  gm_zero_i32(h, K.gcount, 1);
  ensure(h, K.part, (size_t)std::max(1, K.nseg) * (kmax + 1));
  ensure(h, K.tmp, n2);
  ensure(h, K.tmp2, n2);
  ensure(h, K.vin, n2);
  ensure(h, K.w, n2);
  ensure(h, K.b, n2);
  ensure(h, K.d, n2);
  ensure(h, K.z, n2);
  ensure(h, K.z2, n2);
  ensure(h, K.dots, C);
}

// Learned warm start buffers and the normal field as one SoA vector.
void alloc_learned(spm_handle* h) {
  Learned& L = h->ln;
  const int64_t N = h->geo.N;
  const int C = h->geo.C, n = h->geo.No;
  ensure(h, L.nvec, 2 * N);
  ensure(h, L.num, C);
  ensure(h, L.den, C);
  ensure(h, L.fit, (size_t)7 * C);
  ensure(h, L.feat, (size_t)n * SPM_MLP_IN);
  ensure(h, L.modes, (size_t)n * SPM_MLP_OUT);
  SPM_HIP_CHECK(hipMemcpyAsync(L.nvec, h->geo.nx, N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  SPM_HIP_CHECK(hipMemcpyAsync(L.nvec + N, h->geo.ny, N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
}

// Distinct particle shapes (kind, parameters, N) in order of first appearance; the
// preconditioner is rebuilt (lazily) only when this list changes.
void update_shapes(spm_handle* h) {
  Precond& P = h->pc;
  const int n = h->geo.No;
  std::map<std::vector<double>, int32_t> id;
  std::vector<std::vector<double>> keys;
  std::vector<int32_t> ps(n);
  for (int i = 0; i < n; ++i) {
    std::vector<double> key = {(double)h->kind[i], h->prm[4 * i], h->prm[4 * i + 1], h->prm[4 * i + 2],
                               h->prm[4 * i + 3], (double)h->nn[i]};
    auto it = id.find(key);
    if (it == id.end()) {
      const int32_t sid = (int32_t)keys.size();
      id.emplace(key, sid);
      keys.push_back(key);
      ps[i] = sid;
    } else {
      ps[i] = it->second;
    }
  }
  if (keys != P.keys) {
    P.valid = false;
    P.keys = keys;
  }
  ensure(h, P.pshape, n);
  upload(h, P.pshape, ps.data(), n * sizeof(int32_t));
}

// Largest and smallest distance from a particle's reference point to its curve.
void shape_radii(int32_t kind, const double* p, double& rmax, double& rmin) {
  if (kind == SPM_SHAPE_ELLIPSE) {
    rmax = std::max(p[0], p[1]);
    rmin = std::min(p[0], p[1]);
  } else {
    rmax = p[0] * (1.0 + std::fabs(p[1]));
    rmin = p[0] * (1.0 - std::fabs(p[1]));
  }
}

// Node count of a particle curve by its perimeter P: clamp(8 ceil(P / (8 h)), 64, 256), h the
// configured node spacing. The ellipse perimeter comes from Ramanujan's second approximation
// (relative error below 1e-9 for aspect ratios up to 3), a star's from the trapezoid rule on
// |x'(t)| (spectrally accurate for these smooth periodic curves); the count only picks the
// discretisation.
int32_t perimeter_nodes(int32_t kind, const double* p, double h) {
  double P = 0.0;
  if (kind == SPM_SHAPE_ELLIPSE) {
    const double a = p[0], b = p[1];
    const double l = ((a - b) / (a + b)) * ((a - b) / (a + b));
    P = kPi * (a + b) * (1.0 + 3.0 * l / (10.0 + std::sqrt(4.0 - 3.0 * l)));
  } else {
    const int K = 1024;
    for (int k = 0; k < K; ++k) {
      double X, Y, Xp, Yp, Xpp, Ypp;
      shape_point(kind, p, 2.0 * kPi * k / K, X, Y, Xp, Yp, Xpp, Ypp);
      P += std::sqrt(Xp * Xp + Yp * Yp);
    }
    P *= 2.0 * kPi / K;
  }
  if (!std::isfinite(P) || !(P > 0) || !(h > 0)) return 64;
  const double n = 8.0 * std::ceil(P / (8.0 * h));
  return (int32_t)std::min(256.0, std::max(64.0, n));
}

void set_cells_impl(spm_handle* h, int C, const double* skews, const int32_t* part_off, const double* centers,
                    const double* theta, const int32_t* kind, const double* prm, const int32_t* n_nodes) {
  if (C < 1 || C > 1024) throw ApiError(SPM_EINVAL, "number of cells must be in [1, 1024]");
  const int n = part_off[C];
  if (part_off[0] != 0 || n < 1) throw ApiError(SPM_EINVAL, "bad particle offsets");
  std::vector<int32_t> rule_nodes;
  if (!n_nodes) {   // node counts by the perimeter rule
    rule_nodes.resize(n);
    for (int i = 0; i < n; ++i) rule_nodes[i] = perimeter_nodes(kind[i], prm + 4 * (size_t)i, h->cfg.node_spacing);
    n_nodes = rule_nodes.data();
  }
  h->have_particles = false;
  h->delta32 = -1.0;
  drop_graphs(h);
  double tmark = now();
  auto mark = [&](const char* what) {      // set-up phase times with SPM_VERBOSE
    if (!verbose()) return;
    sync(h);
    const double t = now();
    std::fprintf(stderr, "[spm] set-up %s %.1f ms\n", what, 1e3 * (t - tmark));
    tmark = t;
  };
  h->cells.assign(C, CellHost());
  h->cx.resize(n);
  h->cy.resize(n);
  h->th.assign(theta, theta + n);
  h->kind.assign(kind, kind + n);
  h->prm.assign(prm, prm + 4 * (size_t)n);
  h->a.assign(n, 0.0);
  h->b.assign(n, 0.0);
  h->nn.assign(n_nodes, n_nodes + n);
  h->off.assign(n + 1, 0);
  h->pcell.assign(n, 0);
  for (int c = 0; c < C; ++c) {
    CellHost& cl = h->cells[c];
    if (part_off[c + 1] <= part_off[c]) throw ApiError(SPM_EINVAL, "every cell needs at least one particle");
    if (!std::isfinite(skews[c])) throw ApiError(SPM_EINVAL, "bad skew");
    cl.skew_raw = skews[c];
    cl.skew = skews[c] - std::floor(skews[c] + 0.5);
    cl.p0 = part_off[c];
    cl.p1 = part_off[c + 1];
    const double s = cl.skew;  // e1 = (1, 0), e2 = (s, 1), det = 1
    for (int i = cl.p0; i < cl.p1; ++i) {
      const double* pp = prm + 4 * (size_t)i;
      bool ok = std::isfinite(centers[2 * i]) && std::isfinite(centers[2 * i + 1]) && std::isfinite(theta[i]);
      if (kind[i] == SPM_SHAPE_ELLIPSE) {
        ok = ok && pp[0] > 0 && pp[1] > 0;
      } else if (kind[i] == SPM_SHAPE_STAR) {
        // r(t) = s (1 + A cos(omega t + phi)) > 0, closed for integer omega
        ok = ok && pp[0] > 0 && std::fabs(pp[1]) < 1.0 && pp[2] >= 0 && pp[2] <= 64 &&
             pp[2] == std::floor(pp[2]) && std::isfinite(pp[3]);
      } else {
        ok = false;
      }
      if (!ok) throw ApiError(SPM_EINVAL, "bad particle " + std::to_string(i));
      if (n_nodes[i] < 8 || n_nodes[i] > kMaxNodesPerParticle || (n_nodes[i] & 1))
        throw ApiError(SPM_EINVAL, "node count must be even and in [8, 4096]");
      shape_radii(kind[i], pp, h->a[i], h->b[i]);
      if (h->a[i] >= 0.45) throw ApiError(SPM_EINVAL, "particle larger than the 3x3 image rule allows");
      // wrap: (alpha, beta) = [e1 e2]^{-1} (c - c_U), reduced to [-1/2, 1/2)
      const double dx = centers[2 * i] - h->cU[0], dy = centers[2 * i + 1] - h->cU[1];
      double be = dy;
      double al = dx - s * dy;
      al -= std::floor(al + 0.5);
      be -= std::floor(be + 0.5);
      h->cx[i] = h->cU[0] + al + be * s;
      h->cy[i] = h->cU[1] + be;
      h->off[i + 1] = h->off[i] + n_nodes[i];
      h->pcell[i] = c;
    }
    cl.n0 = h->off[cl.p0];
    cl.n1 = h->off[cl.p1];
  }
  Geo& g = h->geo;
  g.No = n;
  g.C = C;
  g.N = h->off[n];
  g.nmax = *std::max_element(h->nn.begin(), h->nn.end());
  const int64_t N = g.N;
  if (N > (int64_t)1 << 30) throw ApiError(SPM_EINVAL, "too many nodes");
  for (double** p : {&g.x, &g.y, &g.nx, &g.ny, &g.w, &g.kap, &g.tx, &g.ty, &g.xpx, &g.xpy, &g.dcot}) ensure(h, *p, N);
  for (float** p : {&g.xf, &g.yf, &g.nxf, &g.nyf}) ensure(h, *p, N);
  ensure(h, g.pid, N);
  ensure(h, g.ncell, N);
  for (double** p : {&g.pcx, &g.pcy, &g.pth, &g.pa, &g.pb, &g.pper, &g.parea}) ensure(h, *p, n);
  ensure(h, g.poff, n + 1);
  ensure(h, g.pn, n);
  ensure(h, g.pcell, n);
  ensure(h, g.cnoff, C + 1);
  ensure(h, g.cpoff, C + 1);
  ensure(h, g.cskew, C);
  std::vector<int32_t> pid(N), ncell(N);
  for (int i = 0; i < n; ++i)
    for (int k = h->off[i]; k < h->off[i + 1]; ++k) {
      pid[k] = i;
      ncell[k] = h->pcell[i];
    }
  std::vector<int64_t> cnoff(C + 1);
  std::vector<int32_t> cpoff(C + 1);
  std::vector<double> cskew(C);
  for (int c = 0; c < C; ++c) {
    cnoff[c] = h->cells[c].n0;
    cpoff[c] = h->cells[c].p0;
    cskew[c] = h->cells[c].skew;
  }
  cnoff[C] = N;
  cpoff[C] = n;
  upload(h, g.pid, pid.data(), N * sizeof(int32_t));
  upload(h, g.ncell, ncell.data(), N * sizeof(int32_t));
  upload(h, g.pcx, h->cx.data(), n * sizeof(double));
  upload(h, g.pcy, h->cy.data(), n * sizeof(double));
  upload(h, g.pth, h->th.data(), n * sizeof(double));
  upload(h, g.pa, h->a.data(), n * sizeof(double));
  upload(h, g.pb, h->b.data(), n * sizeof(double));
  ensure(h, g.pkind, n);
  ensure(h, g.pprm, 4 * (size_t)n);
  upload(h, g.pkind, h->kind.data(), n * sizeof(int32_t));
  upload(h, g.pprm, h->prm.data(), 4 * (size_t)n * sizeof(double));
  upload(h, g.poff, h->off.data(), (n + 1) * sizeof(int32_t));
  upload(h, g.pn, h->nn.data(), n * sizeof(int32_t));
  upload(h, g.pcell, h->pcell.data(), n * sizeof(int32_t));
  upload(h, g.cnoff, cnoff.data(), (C + 1) * sizeof(int64_t));
  upload(h, g.cpoff, cpoff.data(), (C + 1) * sizeof(int32_t));
  upload(h, g.cskew, cskew.data(), C * sizeof(double));
  g.dilated = h->cfg.near_set == SPM_NEAR_SET_DILATED ? 1 : 0;
  if (g.dilated) {
    ensure(h, g.xw, N);
    ensure(h, g.yw, N);
    ensure(h, g.nwrap, N);
  }
  launch_geometry(h);
  if (g.dilated) {
    // every particle and its close neighbourhood within lattice distance 1/2 of each of its
    // nodes, so that each close source curve lies whole inside the dilated cell seen from a
    // target in the cell: (1 + |s|)(2 r_max + close_factor h_q) < 1/2, h_q = perimeter / N_q
    std::vector<double> per(n);
    download(h, per.data(), g.pper, n * sizeof(double));
    for (int i = 0; i < n; ++i) {
      const double s = std::fabs(h->cells[h->pcell[i]].skew);
      if ((1.0 + s) * (2.0 * h->a[i] + h->cfg.close_factor * per[i] / h->nn[i]) >= 0.5)
        throw ApiError(SPM_EINVAL, "particle " + std::to_string(i) + " too large for the dilated near set");
    }
  }
  mark("geometry");
  build_periodizers(h);
  mark("periodizers");
  // close pairs + overlap check
  CloseList& CL = h->cl;
  ensure(h, CL.count, N);
  ensure(h, CL.row, N + 1);
  ensure(h, CL.tlist, N);
  ensure(h, CL.dmin, N);
  ensure(h, CL.inside, N);
  ensure(h, CL.vp, 6 * N);
  alloc_work(h);
  launch_close_count(h);
  double gap;
  int32_t overlap;
  launch_gap(h, &gap, &overlap);
  h->min_gap_est = gap;
  if (overlap || (h->cfg.min_gap > 0 && gap < h->cfg.min_gap))
    throw ApiError(SPM_EOVERLAP, overlap ? "particles overlap" : "particles closer than min_gap");
  int32_t total, nt;
  launch_close_scan(h, &total, &nt);
  CL.npairs = total;
  CL.ntargets = nt;
  ensure(h, CL.q, std::max<int64_t>(1, total));
  ensure(h, CL.s, std::max<int64_t>(1, total));
  if (total > 0) launch_close_fill(h);
  ensure(h, CL.qsrc, (size_t)h->geo.No);
  launch_close_sources(h);
  mark("close pairs");
  build_chunks(h);
  alloc_krylov(h);
  alloc_learned(h);
  update_shapes(h);
  mark("work arrays");
  if (h->wk.tuned && h->wk.tuned_N != N) h->wk.tuned = false;
  if (!h->wk.tuned) {
    h->wk.near[0].cfg = heuristic_near(h, SPM_FP64);
    h->wk.near[1].cfg = heuristic_near(h, SPM_FP32);
  }
  if (h->cfg.near_method == SPM_NEAR_FMM) {
    build_fmm_plan(h);    // the direct kernels are not planned (their work lists grow like N^2)
  } else {
    build_near_plan(h, SPM_FP64);
    build_near_plan(h, SPM_FP32);
  }
  mark("near-sum plans");
  sync(h);
  h->have_particles = true;
}

// ---------------------------------------------------------------------------
// operator
// ---------------------------------------------------------------------------
void stage_xi(spm_handle* h, const double* sigma, bool with_active) {
  launch_prep(h, sigma);
  launch_disc_impl(h, with_active);
  launch_xi_impl(h, with_active);
}

void matvec(spm_handle* h, const double* sigma, double* out, int precision, bool with_active) {
  if (h->fmm.on) precision = SPM_FP64;     // the FMM sum is FP64: FP64 close and self terms
  stage_xi(h, sigma, with_active);
  if (h->fmm.on)
    launch_fmm(h, h->wk.Tpart);
  else
    launch_near_impl(h, precision, with_active);
  launch_combine(h, sigma, true, precision, with_active);
  if (h->cl.ntargets > 0) {
    launch_vplus(h, sigma, false, with_active);
    launch_close_apply_impl(h, h->wk.T, precision, with_active);
  }
  if (precision == SPM_FP32) launch_self_fix(h, h->wk.T, with_active);
  launch_assemble(h, sigma, out);
}

// one GMRES iteration of every active cell (fixed arguments: capturable); with the block
// preconditioner the operator is A P^{-1} (right preconditioning)
void iteration(spm_handle* h, int precision, bool pc) {
  Krylov& K = h->kr;
  gm_copy_in(h);
  if (pc) {
    launch_precond_apply(h, K.vin, K.z, true);
    matvec(h, K.z, K.w, precision, true);
  } else {
    matvec(h, K.vin, K.w, precision, true);
  }
  gm_cgs_pass(h, K.w, K.h1);
  gm_update_j(h, K.h1, K.w);
  gm_cgs_pass(h, K.w, K.h2);
  gm_update_j(h, K.h2, K.w);
  gm_dot(h, K.w, K.w, K.nrm2);
  gm_store_next(h);
  gm_givens(h);
}

hipGraphExec_t iteration_graph(spm_handle* h, int precision, bool pc) {
  const int k = (precision == SPM_FP64 ? 0 : 1) + (pc ? 2 : 0);
  Krylov& K = h->kr;
  if (K.graph[k]) return K.graph[k];
  if (!K.cap_stream) SPM_HIP_CHECK(hipStreamCreateWithFlags(&K.cap_stream, hipStreamNonBlocking));
  hipStream_t saved = h->stream;
  h->stream = K.cap_stream;
  try {
    SPM_HIP_CHECK(hipStreamBeginCapture(K.cap_stream, hipStreamCaptureModeThreadLocal));
    iteration(h, precision, pc);
    SPM_HIP_CHECK(hipStreamEndCapture(K.cap_stream, &K.graph_src[k]));
  } catch (...) {
    hipGraph_t dummy = nullptr;
    (void)hipStreamEndCapture(K.cap_stream, &dummy);
    if (dummy) (void)hipGraphDestroy(dummy);
    h->stream = saved;
    throw;
  }
  h->stream = saved;
  SPM_HIP_CHECK(hipGraphInstantiate(&K.graph[k], K.graph_src[k], nullptr, nullptr, 0));
  return K.graph[k];
}

// per-cell (host) state of one solve
struct CellStats {
  std::vector<int32_t> its, m64, m32, refine;
  std::vector<double> bnorm, rel;
  explicit CellStats(int C) : its(C, 0), m64(C, 0), m32(C, 0), refine(C, 0), bnorm(C, 0), rel(C, 1) {}
};

void upload_cell_arrays(spm_handle* h, const std::vector<double>& bn, const std::vector<double>& tol,
                        const std::vector<int32_t>& act) {
  const int C = h->geo.C;
  double* hb = host_scratch<double>(h, 3 * (size_t)C);
  std::memcpy(hb, bn.data(), C * sizeof(double));
  std::memcpy(hb + C, tol.data(), C * sizeof(double));
  int32_t* ha = reinterpret_cast<int32_t*>(hb + 2 * C);
  std::memcpy(ha, act.data(), C * sizeof(int32_t));
  SPM_HIP_CHECK(hipMemcpyAsync(h->kr.bnorm, hb, C * sizeof(double), hipMemcpyHostToDevice, h->stream));
  SPM_HIP_CHECK(hipMemcpyAsync(h->kr.tolc, hb + C, C * sizeof(double), hipMemcpyHostToDevice, h->stream));
  SPM_HIP_CHECK(hipMemcpyAsync(h->kr.active, ha, C * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  sync(h);
}

// GMRES cycle on V_0 = r for the cells in `act` (others untouched); x += correction.
// Returns the Krylov iterations of every cell.
//
// relax_at > 0 (FP64 cycles only): once every active cell's residual estimate is at or
// below relax_at (relative to |b|), the remaining iterations apply the operator with the
// FP32 near sum. In GMRES with inexact products, the error allowed in the k-th product
// grows like tol / |r_k|, so the late iterations tolerate FP32 sums while the early
// ones, which set the leading digits, keep FP64. *switched_at (if given) receives the
// iteration index of the switch (-1 if none).
std::vector<int32_t> krylov_cycle(spm_handle* h, int precision, bool pc, double* x, const std::vector<double>& bn,
                                  const std::vector<double>& tol, const std::vector<int32_t>& act, int maxit,
                                  double relax_at = 0.0, int* switched_at = nullptr) {
  Krylov& K = h->kr;
  const int C = h->geo.C;
  upload_cell_arrays(h, bn, tol, act);
  gm_stamp_cycle(h);
  gm_start(h);
  // pinned host scratch: jdev [2], active [C], (padding to 8 bytes), res [C] doubles
  int32_t* hj = host_scratch<int32_t>(h, 4 + 3 * (size_t)C);
  int32_t* hact = hj + 2;
  double* hres = reinterpret_cast<double*>(hj + 2 + C + (C & 1));
  download(h, hj, K.jdev, 2 * sizeof(int32_t));
  maxit = std::max(0, std::min(maxit, K.kmax));
  const bool graph = h->cfg.use_graph != 0 && !h->prof;
  const int poll = std::max(1, h->cfg.poll_every);
  int cur = precision;
  bool relax = relax_at > 0.0 && precision == SPM_FP64;
  if (switched_at) *switched_at = -1;
  if (hj[1] > 0) {
    hipGraphExec_t ge = graph ? iteration_graph(h, cur, pc) : nullptr;
    for (int it = 0; it < maxit; ++it) {
      if (graph)
        SPM_HIP_CHECK(hipGraphLaunch(ge, h->stream));
      else
        iteration(h, cur, pc);
      if ((it + 1) % poll == 0 || it + 1 == maxit) {
        SPM_HIP_CHECK(hipMemcpyAsync(hj, K.jdev, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
        if (relax) {
          SPM_HIP_CHECK(hipMemcpyAsync(hact, K.active, C * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
          SPM_HIP_CHECK(hipMemcpyAsync(hres, K.res, C * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        }
        sync(h);
        if (hj[1] == 0) break;
        if (relax) {
          double worst = 0.0;
          for (int c = 0; c < C; ++c)
            if (hact[c]) worst = std::max(worst, hres[c]);
          if (worst <= relax_at) {
            relax = false;
            cur = SPM_FP32;
            if (switched_at) *switched_at = it + 1;
            if (graph) ge = iteration_graph(h, cur, pc);
          }
        }
      }
    }
  }
  if (pc) {   // x += P^{-1} (V y)
    gm_backsolve(h);
    gm_zero(h, K.z2, K.n2);
    gm_update_only(h, K.z2);
    launch_precond_apply(h, K.z2, K.z, false);
    gm_axpby(h, K.n2, 1.0, x, 1.0, K.z, x);
  } else {
    gm_backsolve_update(h, x);
  }
  std::vector<int32_t> kd(C, 0);
  int32_t* hk = host_scratch<int32_t>(h, C);
  download(h, hk, K.kdone, C * sizeof(int32_t));
  for (int c = 0; c < C; ++c) kd[c] = act[c] ? hk[c] : 0;
  return kd;
}

// r = b - A x per cell for the cells in act; rel_c = |r_c| / |b_c|. r goes to tmp2.
void residual(spm_handle* h, const double* x, const std::vector<int32_t>& act, CellStats& st) {
  Krylov& K = h->kr;
  const int C = h->geo.C;
  upload_cell_arrays(h, st.bnorm, std::vector<double>(C, 0.0), act);
  matvec(h, x, K.tmp, SPM_FP64, true);
  gm_axpby(h, K.n2, 1.0, K.b, -1.0, K.tmp, K.tmp2);
  gm_dot(h, K.tmp2, K.tmp2, K.dots);
  double* hd = host_scratch<double>(h, C);
  download(h, hd, K.dots, C * sizeof(double));
  for (int c = 0; c < C; ++c)
    if (act[c]) {
      st.rel[c] = std::sqrt(hd[c]) / st.bnorm[c];
      st.m64[c] += 1;
    }
}

void stamp_newly(spm_handle* h, const std::vector<int32_t>& newly) {
  const int C = h->geo.C;
  int32_t* hm = host_scratch<int32_t>(h, C);
  std::memcpy(hm, newly.data(), C * sizeof(int32_t));
  SPM_HIP_CHECK(hipMemcpyAsync(h->kr.mask, hm, C * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  gm_stamp_mask(h, h->kr.mask);
  sync(h);
}

// Warm-start fit (b in K.b): with z = A g for the decoded guess g in x, per cell
// x <- alpha g + beta n with (alpha, beta) minimising |b - alpha z - beta n/2|
// (A n = n/2), and the residual of the result into tmp2.
void offset_fit(spm_handle* h, double* x) {
  Krylov& K = h->kr;
  Learned& L = h->ln;
  const int C = h->geo.C;
  matvec(h, x, K.tmp, SPM_FP64, false);
  gm_dot(h, K.tmp, K.tmp, L.fit);
  gm_dot(h, K.tmp, L.nvec, L.fit + C);
  gm_dot(h, L.nvec, L.nvec, L.fit + 2 * C);
  gm_dot(h, K.b, K.tmp, L.fit + 3 * C);
  gm_dot(h, K.b, L.nvec, L.fit + 4 * C);
  launch_fit_guess(h, L.fit, L.fit + 5 * C);
  launch_apply_fit(h, L.fit + 5 * C, K.b, K.tmp, x, K.tmp2);
}

// features -> network (BF16) -> decoded density in x (no offset fit)
void network_decode(spm_handle* h, double* x) {
  if (!h->net) throw ApiError(SPM_ESTATE, "no network set (spm_set_network)");
  launch_features(h, h->ln.feat);
  mlp_forward(h->net, h->stream, h->ln.feat, nullptr, h->geo.No, h->ln.modes, SPM_MLP_BF16);
  launch_decode(h, h->ln.modes, x);
}

// Relative error of the FP32 operator on the current geometry: the largest over the cells of
// |A32 v - A64 v| / |A64 v| for a fixed pseudo-random density v (two operator products, once
// per geometry). It sets where the relaxed solve may switch to FP32 products.
double fp32_operator_error(spm_handle* h) {
  if (h->delta32 >= 0.0) return h->delta32;
  Krylov& K = h->kr;
  const int C = h->geo.C;
  gm_probe_fill(h, K.n2, 12345, K.z2);
  matvec(h, K.z2, K.tmp, SPM_FP64, false);
  matvec(h, K.z2, K.tmp2, SPM_FP32, false);
  gm_axpby(h, K.n2, 1.0, K.tmp2, -1.0, K.tmp, K.tmp2);
  gm_dot(h, K.tmp2, K.tmp2, K.dots);
  std::vector<double> e(C), a(C);
  download(h, e.data(), K.dots, C * sizeof(double));
  gm_dot(h, K.tmp, K.tmp, K.dots);
  download(h, a.data(), K.dots, C * sizeof(double));
  double d = 0.0;
  for (int c = 0; c < C; ++c) d = std::max(d, std::sqrt(e[c] / std::max(a[c], 1e-300)));
  h->delta32 = d;
  if (verbose()) std::fprintf(stderr, "[spm] FP32 operator relative error %.3e\n", d);
  return d;
}

// Adaptive switch point of the relaxed solve. In GMRES with inexact products the error of the
// k-th product may grow like tol |b| / |r_k| without moving the attained residual by more than
// about tol (the relaxation bound of inexact Krylov methods), so products may use the FP32 near
// sum once the residual estimate is below theta tol / delta32, delta32 the measured relative
// error of the FP32 operator and theta = cfg.relax_safety a margin for the conditioning of the
// small Hessenberg problem; kept within [10 tol, 1e-2]. theta = 0.01 by default: of 0.003 to 0.1
// it was the fastest on a 51,200-node cell and on forward-Euler steps of 9,000-node cells (a
// larger theta switches so early that the solve needs a second cycle).
double relax_switch_point(spm_handle* h, double tol) {
  const double d = fp32_operator_error(h);
  const double at = d > 0.0 ? h->cfg.relax_safety * tol / d : 1e-2;
  return std::min(1e-2, std::max(10.0 * tol, at));
}

// How one solve attempt starts and iterates.
struct Attempt {
  bool network = false;   // learned warm start (when no sigma0 is given)
  bool pc = false;        // block preconditioner
  int max_iter = 0;
};

int solve_impl(spm_handle* h, const double* sigma0, double* sigma, std::vector<spm_solve_info>& infos,
               const Attempt& at) {
  Krylov& K = h->kr;
  const int C = h->geo.C;
  const int64_t n2 = K.n2;
  const double tol = h->cfg.tol;
  const int max_iter = at.max_iter;
  const bool pc = at.pc;
  if (pc && !h->pc.valid) build_precond(h);
  CellStats st(C);
  launch_rhs(h, K.b);
  gm_dot(h, K.b, K.b, K.dots);
  {
    double* hd = host_scratch<double>(h, C);
    download(h, hd, K.dots, C * sizeof(double));
    for (int c = 0; c < C; ++c) st.bnorm[c] = std::sqrt(hd[c]);
  }
  gm_stamp_start(h);
  const bool net = !sigma0 && at.network;
  h->guess_rejected.assign(C, 0);
  if (sigma0)
    gm_copy(h, sigma, sigma0, n2);
  else if (net)
    network_decode(h, sigma);
  else
    gm_zero(h, sigma, n2);
  std::vector<int32_t> act(C, 1), conv(C, 0), newly(C, 0);
  if (sigma0) {
    residual(h, sigma, act, st);
  } else if (net) {
    offset_fit(h, sigma);
    gm_dot(h, K.tmp2, K.tmp2, K.dots);
    double* hd = host_scratch<double>(h, C);
    download(h, hd, K.dots, C * sizeof(double));
    // acceptance test of the guess: a cell whose fitted guess leaves more than learned_accept of
    // the zero start's residual starts from zero (a loose guess puts every slowly converging
    // error component into the starting residual and costs iterations)
    std::vector<int32_t> reject(C, 0);
    int nrej = 0;
    for (int c = 0; c < C; ++c) {
      st.rel[c] = std::sqrt(hd[c]) / st.bnorm[c];
      st.m64[c] += 1;
      if (st.rel[c] > h->cfg.learned_accept) {
        reject[c] = 1;
        st.rel[c] = 1.0;
        ++nrej;
      }
    }
    h->guess_rejected = reject;
    if (nrej > 0) {
      int32_t* hm = host_scratch<int32_t>(h, C);
      std::memcpy(hm, reject.data(), C * sizeof(int32_t));
      SPM_HIP_CHECK(hipMemcpyAsync(K.mask, hm, C * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
      launch_reject_guess(h, K.mask, K.b, sigma, K.tmp2);
      sync(h);
    }
  } else {
    gm_copy(h, K.tmp2, K.b, n2);
    std::fill(st.rel.begin(), st.rel.end(), 1.0);
  }
  auto mark = [&]() {
    bool any = false;
    for (int c = 0; c < C; ++c) {
      newly[c] = (!conv[c] && st.rel[c] <= tol) ? 1 : 0;
      if (newly[c]) conv[c] = 1;
      act[c] = (!conv[c] && st.its[c] < max_iter) ? 1 : 0;
      any = any || act[c];
    }
    stamp_newly(h, newly);
    return any;
  };
  bool any = mark();
  if (h->cfg.precision == SPM_FP32_IR) {
    // first inner tolerance: with the block preconditioner the inner solves are cheap and
    // loose ones pay (fewer FP32 products in all); measured on the 200-ellipse cell
    const double it0 = h->cfg.inner_tol > 0 ? h->cfg.inner_tol : (pc ? 3e-3 : 1e-4);
    std::vector<double> itol(C, it0), bn(C), tl(C);
    for (int outer = 0; outer < 40 && any; ++outer) {
      for (int c = 0; c < C; ++c) {
        bn[c] = st.rel[c] * st.bnorm[c];
        tl[c] = (tol / st.rel[c] > itol[c]) ? 0.5 * tol / st.rel[c] : itol[c];
      }
      gm_copy(h, K.V, K.tmp2, n2);   // V_0 = r
      gm_zero(h, K.d, n2);
      const std::vector<int32_t> kd = krylov_cycle(h, SPM_FP32, pc, K.d, bn, tl, act, max_iter);
      gm_axpby(h, n2, 1.0, sigma, 1.0, K.d, sigma);
      const std::vector<double> before = st.rel;
      std::vector<int32_t> was = act;
      for (int c = 0; c < C; ++c)
        if (was[c]) {
          st.its[c] += kd[c];
          st.m32[c] += kd[c];
          st.refine[c] += 1;
        }
      residual(h, sigma, was, st);
      for (int c = 0; c < C; ++c)
        if (was[c]) {
          const double rho = st.rel[c] / before[c];
          itol[c] = std::min(0.1, std::max(it0, 0.5 * rho));
          if (verbose())
            std::fprintf(stderr, "[spm] cell %d refinement %d: inner its %d (inner tol %.1e) residual %.3e -> %.3e\n",
                         c, st.refine[c], kd[c], tl[c], before[c], st.rel[c]);
          if (kd[c] == 0 && st.rel[c] > tol) st.its[c] = max_iter;  // no progress possible
        }
      any = mark();
    }
  } else {
    std::vector<double> tl(C, tol);
    for (int restart = 0; restart < 6 && any; ++restart) {
      gm_copy(h, K.V, K.tmp2, n2);   // V_0 = r
      int budget = max_iter;
      for (int c = 0; c < C; ++c)
        if (act[c]) budget = std::min(budget, max_iter - st.its[c]);
      const double relax_at = h->cfg.precision != SPM_FP32_RELAXED ? 0.0
                              : h->cfg.relax_tol > 0.0 ? h->cfg.relax_tol
                                                       : relax_switch_point(h, tol);
      int sw = -1;
      const std::vector<int32_t> kd =
          krylov_cycle(h, SPM_FP64, pc, sigma, st.bnorm, tl, act, std::max(1, budget), relax_at, &sw);
      std::vector<int32_t> was = act;
      for (int c = 0; c < C; ++c)
        if (was[c]) {
          const int k64 = sw < 0 ? kd[c] : std::min(kd[c], sw);
          st.its[c] += kd[c];
          st.m64[c] += k64;
          st.m32[c] += kd[c] - k64;
        }
      residual(h, sigma, was, st);
      if (verbose())
        for (int c = 0; c < C; ++c)
          if (was[c]) std::fprintf(stderr, "[spm] cell %d cycle %d: its %d residual %.3e\n", c, restart, kd[c], st.rel[c]);
      any = mark();
    }
  }
  int status = SPM_OK;
  infos.assign(C, spm_solve_info{});
  for (int c = 0; c < C; ++c) {
    spm_solve_info& in = infos[c];
    std::memset(&in, 0, sizeof(in));
    in.iterations = st.its[c];
    in.fp64_matvecs = st.m64[c];
    in.fp32_matvecs = st.m32[c];
    in.refinements = st.refine[c];
    in.rel_residual = st.rel[c];
    in.status = st.rel[c] <= tol ? SPM_OK : SPM_ENOCONV;
    if (in.status != SPM_OK) status = SPM_ENOCONV;
  }
  return status;
}

void readout(spm_handle* h, const double* sigma, double* vel, double* omega, double* mu_eff) {
  stage_xi(h, sigma, false);
  if (vel || omega) launch_velocities(h, vel, omega);
  if (mu_eff) launch_mu_eff(h, mu_eff);
}

int solve_api(spm_handle* h, const double* sigma0, double* sigma, double* vel, double* omega, double* mu_eff,
              spm_solve_info* info_out, double* latency_out) {
  need_particles(h);
  if (!sigma) throw ApiError(SPM_EINVAL, "null sigma");
  const int C = h->geo.C;
  std::vector<spm_solve_info> infos;
  const double t0 = now();
  Attempt first;
  first.network = !sigma0 && h->cfg.x0 == SPM_X0_NETWORK;
  first.pc = h->cfg.precond == SPM_PRECOND_BLOCK;
  const bool special = first.network || first.pc;
  first.max_iter = (special && h->cfg.learned_max_iter > 0) ? std::min(h->cfg.learned_max_iter, h->cfg.max_iter)
                                                             : h->cfg.max_iter;
  int st = solve_impl(h, sigma0, sigma, infos, first);
  if (st == SPM_ENOCONV && special) {
    // fallback: plain GMRES from zero without the preconditioner
    std::vector<int32_t> first_its(C);
    for (int c = 0; c < C; ++c) first_its[c] = infos[c].iterations;
    Attempt plain;
    plain.max_iter = h->cfg.max_iter;
    st = solve_impl(h, nullptr, sigma, infos, plain);
    for (int c = 0; c < C; ++c) {
      infos[c].fallback = 1;
      infos[c].first_iterations = first_its[c];
    }
  }
  sync(h);
  const double t1 = now();
  readout(h, sigma, vel, omega, mu_eff);
  sync(h);
  const double t2 = now();
  std::vector<unsigned long long> stamps(C + 1);
  download(h, stamps.data(), h->kr.stamp, (C + 1) * sizeof(unsigned long long));
  for (int c = 0; c < C; ++c) {
    infos[c].n_close_pairs = (int32_t)h->cl.npairs;
    infos[c].min_gap = h->min_gap_est;
    infos[c].seconds_solve = t1 - t0;
    infos[c].seconds_readout = t2 - t1;
    infos[c].guess_rejected = c < (int)h->guess_rejected.size() ? h->guess_rejected[c] : 0;
    if (latency_out) latency_out[c] = (double)(stamps[c] - stamps[C]) / h->wallclock_hz;
    if (info_out) info_out[c] = infos[c];
  }
  if (st == SPM_ENOCONV) h->err = "GMRES did not reach the tolerance; outputs hold the last iterate";
  return st;
}

}  // namespace

namespace spm {
namespace {
inline int64_t fmm_box_off(int l) { return (((int64_t)1 << (2 * l)) - 1) / 3; }

// Counts of a leaf grid summed into every level: out[box_off(l) + iy 2^l + ix], levels 0..L.
std::vector<int64_t> fmm_levels(const std::vector<int64_t>& leaf, int L) {
  std::vector<int64_t> out(fmm_box_off(L + 1), 0);
  std::copy(leaf.begin(), leaf.end(), out.begin() + fmm_box_off(L));
  for (int l = L - 1; l >= 0; --l) {
    const int n = 1 << l;
    for (int iy = 0; iy < n; ++iy)
      for (int ix = 0; ix < n; ++ix) {
        int64_t v = 0;
        for (int ch = 0; ch < 4; ++ch)
          v += out[fmm_box_off(l + 1) + (int64_t)(2 * iy + (ch >> 1)) * (2 * n) + (2 * ix + (ch & 1))];
        out[fmm_box_off(l) + (int64_t)iy * n + ix] = v;
      }
  }
  return out;
}

// Direct pairs of the leaves and multipole-to-local translations of one evaluation.
std::pair<double, double> fmm_work(const std::vector<int64_t>& bs, const std::vector<int64_t>& bt, int L) {
  double p2p = 0, m2l = 0;
  const int nL = 1 << L;
  for (int iy = 0; iy < nL; ++iy)
    for (int ix = 0; ix < nL; ++ix) {
      const int64_t t = bt[fmm_box_off(L) + (int64_t)iy * nL + ix];
      if (!t) continue;
      int64_t s = 0;
      for (int jy = std::max(iy - 1, 0); jy <= std::min(iy + 1, nL - 1); ++jy)
        for (int jx = std::max(ix - 1, 0); jx <= std::min(ix + 1, nL - 1); ++jx)
          s += bs[fmm_box_off(L) + (int64_t)jy * nL + jx];
      p2p += (double)t * (double)s;
    }
  for (int l = 2; l <= L; ++l) {
    const int n = 1 << l, np = n >> 1;
    for (int iy = 0; iy < n; ++iy)
      for (int ix = 0; ix < n; ++ix) {
        if (!bt[fmm_box_off(l) + (int64_t)iy * n + ix]) continue;
        for (int qy = std::max((iy >> 1) - 1, 0); qy <= std::min((iy >> 1) + 1, np - 1); ++qy)
          for (int qx = std::max((ix >> 1) - 1, 0); qx <= std::min((ix >> 1) + 1, np - 1); ++qx)
            for (int ch = 0; ch < 4; ++ch) {
              const int bx = 2 * qx + (ch & 1), by = 2 * qy + (ch >> 1);
              if (std::abs(bx - ix) <= 1 && std::abs(by - iy) <= 1) continue;
              if (bs[fmm_box_off(l) + (int64_t)by * n + bx]) m2l += 1;
            }
      }
  }
  return {p2p, m2l};
}
}  // namespace

// Quadtree of the FMM near sum for the current geometry (one cell): the root box holds the 9 N
// image sources (node + m e1 + n e2 with the shifts of the direct sum, so the target's own node is
// the source at zero distance); the leaf level minimises an operation count (direct pairs at
// ~25 flop against multipole-to-local translations at ~12 p^2 flop); sources and targets are
// sorted by leaf; box lists of every pass are uploaded with the expansion buffers.
// Host array left uninitialised: its pages are first touched by the threads that fill it (a
// std::vector would zero them all on one thread first).
template <class T>
struct HostArray {
  std::unique_ptr<T[]> p;
  explicit HostArray(size_t n) : p(new T[n]) {}
  T& operator[](size_t i) { return p[i]; }
  const T& operator[](size_t i) const { return p[i]; }
  T* data() { return p.get(); }
};

size_t fmm_table_doubles(int p);   // the FMM plan's table sizes (k_fmm.hip)

void build_fmm_plan(spm_handle* h) {
  FmmPlan& F = h->fmm;
  F.on = false;
  const Geo& g = h->geo;
  const int64_t N = g.N;
  if (g.C != 1) throw ApiError(SPM_EINVAL, "the FMM near sum runs on single-cell handles");
  if (9 * N >= ((int64_t)1 << 31)) throw ApiError(SPM_EINVAL, "too many nodes for the FMM");
  const int p = h->cfg.fmm_order > 0 ? h->cfg.fmm_order : 40;
  double tm = now();
  auto mark = [&](const char* what) {      // phase times with SPM_VERBOSE
    if (!verbose()) return;
    const double t = now();
    std::fprintf(stderr, "[spm]   quadtree %s %.1f ms\n", what, 1e3 * (t - tm));
    tm = t;
  };
  std::vector<double> x(N), y(N);
  download(h, x.data(), g.x, N * sizeof(double));
  download(h, y.data(), g.y, N * sizeof(double));
  const double skew = h->cells[0].skew;
  const int64_t ns = 9 * N;
  // host threads over contiguous index ranges (results do not depend on their number)
  const int T = (int)std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::max(1u, std::thread::hardware_concurrency()),
                                                             ns / 65536 + 1}));
  auto par = [&](int64_t n, const std::function<void(int64_t, int64_t, int)>& f) {
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) {
      const int64_t a = n * t / T, b = n * (t + 1) / T;
      th.emplace_back(f, a, b, t);
    }
    for (auto& x : th) x.join();
  };
  HostArray<double> sx(ns), sy(ns);       // every entry written below
  std::vector<double> mm(4 * T);
  par(ns, [&](int64_t a, int64_t b, int t) {
    double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
    int sh = (int)(a / N);                 // source k is image sh of node j = k - sh N
    int64_t j = a - sh * N;
    double ox = shift_x(sh, skew), oy = shift_y(sh);
    for (int64_t k = a; k < b; ++k) {
      const double u = x[j] + ox, v = y[j] + oy;
      sx[k] = u;
      sy[k] = v;
      x0 = std::min(x0, u);
      x1 = std::max(x1, u);
      y0 = std::min(y0, v);
      y1 = std::max(y1, v);
      if (++j == N && sh < 8) {
        j = 0;
        ++sh;
        ox = shift_x(sh, skew);
        oy = shift_y(sh);
      }
    }
    mm[4 * t] = x0;
    mm[4 * t + 1] = x1;
    mm[4 * t + 2] = y0;
    mm[4 * t + 3] = y1;
  });
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  for (int t = 0; t < T; ++t) {
    xmin = std::min(xmin, mm[4 * t]);
    xmax = std::max(xmax, mm[4 * t + 1]);
    ymin = std::min(ymin, mm[4 * t + 2]);
    ymax = std::max(ymax, mm[4 * t + 3]);
  }
  mark("images");
  const double D0 = std::max(xmax - xmin, ymax - ymin) * (1.0 + 1e-6) + 1e-12;
  const double c0x = 0.5 * (xmin + xmax), c0y = 0.5 * (ymin + ymax);
  const int64_t ctr = 4 * N;   // shift index 4 is m = n = 0: the targets themselves
  // leaf level: bin once at the finest candidate level; every coarser tree is an aggregate of it
  // (same root box, and a box index at level L is the finest index shifted right). Candidates
  // bracket about 60 image sources per leaf.
  const int Lg = (int)std::lround(std::log((double)ns / 60.0) / std::log(4.0));
  const int Llo = std::max(2, std::min(9, Lg - 1)), Lhi = std::min(10, std::max(Llo, Lg + 1));
  const int nh = 1 << Lhi;
  HostArray<int32_t> ixh(ns), iyh(ns);     // finest-level box coordinates of every source
  std::vector<int64_t> bs_all, bt_all;
  {
    const int64_t nlh = (int64_t)nh * nh;
    std::vector<int64_t> cs(nlh, 0), ct(nlh, 0);
    par(ns, [&](int64_t a, int64_t b, int) {
      for (int64_t k = a; k < b; ++k) {
        const int ix = std::min(std::max((int)std::floor((sx[k] - (c0x - 0.5 * D0)) / D0 * nh), 0), nh - 1);
        const int iy = std::min(std::max((int)std::floor((sy[k] - (c0y - 0.5 * D0)) / D0 * nh), 0), nh - 1);
        ixh[k] = ix;
        iyh[k] = iy;
        __atomic_fetch_add(&cs[(int64_t)iy * nh + ix], (int64_t)1, __ATOMIC_RELAXED);   // counts only
      }
    });
    for (int64_t j = ctr; j < ctr + N; ++j) ct[(int64_t)iyh[j] * nh + ixh[j]]++;
    bs_all = fmm_levels(cs, Lhi);
    bt_all = fmm_levels(ct, Lhi);
  }
  mark("binning");
  int bestL = Llo;
  double best = 1e300, best_p2p = 0, best_m2l = 0;
  for (int L = Llo; L <= Lhi; ++L) {
    const auto w = fmm_work(bs_all, bt_all, L);
    const double cost = 25.0 * w.first + 12.0 * p * p * w.second;
    if (cost < best) {
      best = cost;
      bestL = L;
      best_p2p = w.first;
      best_m2l = w.second;
    }
  }
  mark("level choice");
  const int L = bestL;
  const int64_t nl = (int64_t)1 << (2 * L);
  const int dsh = Lhi - L;
  auto leaf = [&](int64_t k) -> int64_t { return ((int64_t)(iyh[k] >> dsh) << L) + (ixh[k] >> dsh); };
  // stable counting sort of the sources by leaf: per-thread histograms over contiguous ranges, so
  // within a leaf the sources keep their index order whatever the number of threads
  std::vector<int64_t> cs(nl, 0), ct(nl, 0);
  std::vector<std::vector<int32_t>> hist(T, std::vector<int32_t>(nl, 0));
  par(ns, [&](int64_t a, int64_t b, int t) {
    for (int64_t k = a; k < b; ++k) hist[t][leaf(k)]++;
  });
  for (int t = 0; t < T; ++t)
    for (int64_t b = 0; b < nl; ++b) cs[b] += hist[t][b];
  for (int64_t j = ctr; j < ctr + N; ++j) ct[leaf(j)]++;
  std::vector<int32_t> leaf_s(nl + 1, 0), leaf_t(nl + 1, 0);
  for (int64_t b = 0; b < nl; ++b) {
    leaf_s[b + 1] = leaf_s[b] + (int32_t)cs[b];
    leaf_t[b + 1] = leaf_t[b] + (int32_t)ct[b];
  }
  for (int64_t b = 0; b < nl; ++b) {       // hist[t][b] becomes thread t's first slot in leaf b
    int32_t run = leaf_s[b];
    for (int t = 0; t < T; ++t) {
      const int32_t c = hist[t][b];
      hist[t][b] = run;
      run += c;
    }
  }
  HostArray<double> ssx(ns), ssy(ns);     // the scatter below writes every slot once
  HostArray<int32_t> ssj(ns);
  std::vector<int32_t> tperm(N);
  par(ns, [&](int64_t a, int64_t b, int t) {
    std::vector<int32_t>& fill = hist[t];
    int64_t j = a % N;                     // node of source k
    for (int64_t k = a; k < b; ++k) {
      const int32_t d = fill[leaf(k)]++;
      ssx[d] = sx[k];
      ssy[d] = sy[k];
      ssj[d] = (int32_t)j;
      if (++j == N) j = 0;
    }
  });
  {
    std::vector<int32_t> tf(leaf_t.begin(), leaf_t.end() - 1);
    for (int64_t j = 0; j < N; ++j) tperm[tf[leaf(ctr + j)]++] = (int32_t)j;
  }
  mark("sort");
  const std::vector<int64_t> bs = fmm_levels(cs, L), bt = fmm_levels(ct, L);
  const int64_t nbox = fmm_box_off(L + 1);
  std::vector<int32_t> bsrc(nbox);
  for (int64_t b = 0; b < nbox; ++b) bsrc[b] = (int32_t)std::min<int64_t>(bs[b], INT32_MAX);
  // box lists: P2M (leaves with sources), M2M levels L-1..2, M2L (target boxes of levels 2..L),
  // L2L levels 3..L, evaluation (leaves with targets)
  std::vector<int32_t> lists;
  F.seg.assign(1, 0);
  auto push_level = [&](int l, const std::vector<int64_t>& cnt) {
    for (int64_t b = fmm_box_off(l); b < fmm_box_off(l + 1); ++b)
      if (cnt[b]) lists.push_back((int32_t)b);
  };
  push_level(L, bs);
  F.seg.push_back((int64_t)lists.size());
  for (int l = L - 1; l >= 2; --l) {
    push_level(l, bs);
    F.seg.push_back((int64_t)lists.size());
  }
  for (int l = 2; l <= L; ++l) push_level(l, bt);
  F.seg.push_back((int64_t)lists.size());
  for (int l = 3; l <= L; ++l) {
    push_level(l, bt);
    F.seg.push_back((int64_t)lists.size());
  }
  push_level(L, bt);
  F.seg.push_back((int64_t)lists.size());
  mark("lists");
  std::vector<double> fact(2 * p);
  fact[0] = 1.0;
  for (int k = 1; k < 2 * p; ++k) fact[k] = fact[k - 1] * k;
  ensure(h, F.sx, ns);
  ensure(h, F.sy, ns);
  ensure(h, F.sj, ns);
  ensure(h, F.fs1, ns);
  ensure(h, F.fs2, ns);
  ensure(h, F.leaf_s, nl + 1);
  ensure(h, F.tperm, N);
  ensure(h, F.leaf_t, nl + 1);
  ensure(h, F.bsrc, nbox);
  ensure(h, F.lists, lists.size());
  ensure(h, F.fact, 2 * p);
  ensure(h, F.m2l_tab, fmm_table_doubles(p));
  ensure(h, F.Mx, (size_t)nbox * 3 * p * 2);
  ensure(h, F.Lx, (size_t)nbox * 3 * p * 2);
  ensure(h, F.one_block, 2);
  ensure(h, F.vnear, 3 * (size_t)g.No);
  ensure(h, h->wk.Tpart, 2 * (size_t)N);
  upload(h, F.sx, ssx.data(), ns * sizeof(double));
  upload(h, F.sy, ssy.data(), ns * sizeof(double));
  upload(h, F.sj, ssj.data(), ns * sizeof(int32_t));
  upload(h, F.leaf_s, leaf_s.data(), (nl + 1) * sizeof(int32_t));
  upload(h, F.tperm, tperm.data(), N * sizeof(int32_t));
  upload(h, F.leaf_t, leaf_t.data(), (nl + 1) * sizeof(int32_t));
  upload(h, F.bsrc, bsrc.data(), nbox * sizeof(int32_t));
  upload(h, F.lists, lists.data(), lists.size() * sizeof(int32_t));
  upload(h, F.fact, fact.data(), fact.size() * sizeof(double));
  F.p = p;
  launch_fmm_tables(h);
  const int32_t one_block[2] = {0, 1};
  upload(h, F.one_block, one_block, sizeof(one_block));
  mark("upload");
  F.L = L;
  F.D0 = D0;
  F.c0x = c0x;
  F.c0y = c0y;
  F.nsrc = ns;
  F.p2p_pairs = best_p2p;
  F.m2l = best_m2l;
  F.on = true;
  drop_graphs(h);
}

// Plan of the near-sum launch of one precision: target blocks of block * tpt targets and
// source tiles of every cell, the persistent grid, and room for the partials (at most one
// per target block and one more per workgroup boundary that falls inside a block).
void build_near_plan(spm_handle* h, int precision) {
  NearPlan& P = h->wk.near[precision == SPM_FP64 ? 0 : 1];
  if (!near_config_valid(P.cfg)) throw ApiError(SPM_EINVAL, "unsupported near-sum launch configuration");
  const int C = h->geo.C;
  const int64_t BT = (int64_t)P.cfg.block * P.cfg.tpt;
  std::vector<int32_t> nt(C), blk(C + 1, 0);
  for (int c = 0; c < C; ++c) {
    const int64_t Nc = h->cells[c].n1 - h->cells[c].n0;
    nt[c] = (int32_t)((Nc + P.cfg.tile - 1) / P.cfg.tile);
    blk[c + 1] = blk[c] + (int32_t)((Nc + BT - 1) / BT);
  }
  P.nblocks = blk[C];
  P.bt = (int32_t)BT;
  ensure(h, P.cell_nt, C);
  ensure(h, P.cell_blk, C + 1);
  ensure(h, P.unit_off, C + 1);
  ensure(h, P.slot_off, (size_t)P.nblocks + 1);
  upload(h, P.cell_nt, nt.data(), C * sizeof(int32_t));
  upload(h, P.cell_blk, blk.data(), (C + 1) * sizeof(int32_t));
  P.grid = near_persistent_grid(P.cfg, precision, h->geo.dilated != 0);
  size_t need = 2 * (size_t)h->geo.N;
  for (const NearPlan& Q : h->wk.near)
    if (Q.bt > 0) need = std::max(need, ((size_t)Q.nblocks + (size_t)Q.grid) * 2 * (size_t)Q.bt);
  ensure(h, h->wk.Tpart, need);
  drop_graphs(h);
}

void* precond_alloc(spm_handle* h, void* old, size_t bytes, size_t& cap) {
  if (old && cap >= bytes) return old;
  if (old) raw_free(h, old);
  void* p = raw_alloc(h, bytes);
  cap = bytes;
  return p;
}

void precond_release_work(spm_handle* h) {
  sync(h);
  raw_free(h, h->pc.work);
  h->pc.work = nullptr;
  h->pc.work_cap = 0;
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
  c->inner_tol = 0.0;
  c->relax_tol = 0.0;
  c->near_method = SPM_NEAR_DIRECT;
  c->fmm_order = 0;
  c->min_gap = 0.0;
  c->rcond = 1e-14;
  c->use_graph = 1;
  c->poll_every = 2;
  c->x0 = SPM_X0_ZERO;
  c->precond = SPM_PRECOND_NONE;
  c->learned_max_iter = 0;
  c->node_spacing = 2.170590708293102e-3;
  c->relax_safety = 0.01;
  c->learned_accept = 0.5;
  c->near_set = SPM_NEAR_SET_3X3;
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
      (c.precision != SPM_FP64 && c.precision != SPM_FP32_IR && c.precision != SPM_FP32_RELAXED) ||
      !(c.inner_tol >= 0 && c.inner_tol < 1) || !(c.relax_tol >= 0 && c.relax_tol < 1) ||
      !(c.relax_safety > 0 && c.relax_safety <= 1) || !(c.node_spacing > 0) || !(c.learned_accept > 0) ||
      c.poll_every < 1 || c.x0 < SPM_X0_ZERO || c.x0 > SPM_X0_NETWORK ||
      (c.precond != SPM_PRECOND_NONE && c.precond != SPM_PRECOND_BLOCK) || c.learned_max_iter < 0 ||
      (c.near_method != SPM_NEAR_DIRECT && c.near_method != SPM_NEAR_FMM) ||
      (c.near_method == SPM_NEAR_FMM && c.precision != SPM_FP64) ||
      (c.fmm_order != 0 && (c.fmm_order < 8 || c.fmm_order > 64)) ||
      (c.near_set != SPM_NEAR_SET_3X3 && c.near_set != SPM_NEAR_SET_DILATED) ||
      (c.near_set == SPM_NEAR_SET_DILATED && (c.near_method != SPM_NEAR_DIRECT || c.M % 4 != 0))) {
    delete h;
    return SPM_EINVAL;
  }
  h->stream = (hipStream_t)stream;
  h->alloc = alloc;
  h->free_fn = free_fn;
  h->alloc_ctx = ctx;
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess &&
      khz > 0)
    h->wallclock_hz = 1e3 * (double)khz;
  *out = h;
  return SPM_OK;
}

void spm_destroy(spm_handle* h) {
  if (!h) return;
  try {
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (h->kr.cap_stream) (void)hipStreamDestroy(h->kr.cap_stream);
    free_all(h);
    for (void* p : {(void*)h->pc.inv, (void*)h->pc.ioff, (void*)h->pc.work, (void*)h->pc.desc, (void*)h->pc.status})
      raw_free(h, p);
    if (h->kr.host) (void)hipHostFree(h->kr.host);
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
    h->pending_skew = e2[0];
    h->cU[0] = center ? center[0] : 0.0;
    h->cU[1] = center ? center[1] : 0.0;
    h->have_lattice = true;
    h->have_particles = false;
    return SPM_OK;
  });
}

int spm_set_ellipses(spm_handle* h, int32_t n, const double* centers, const double* theta, const double* a,
                     const double* b, const int32_t* n_nodes) {
  return guarded(h, [&]() {
    if (!h->have_lattice) throw ApiError(SPM_ESTATE, "set the lattice first");
    if (n < 1 || !centers || !theta || !a || !b) throw ApiError(SPM_EINVAL, "bad particle arrays");
    const int32_t off[2] = {0, n};
    const double sk = h->pending_skew;
    std::vector<int32_t> kind(n, SPM_SHAPE_ELLIPSE);
    std::vector<double> prm(4 * (size_t)n, 0.0);
    for (int i = 0; i < n; ++i) {
      prm[4 * i] = a[i];
      prm[4 * i + 1] = b[i];
    }
    set_cells_impl(h, 1, &sk, off, centers, theta, kind.data(), prm.data(), n_nodes);
    return SPM_OK;
  });
}

int spm_set_cells(spm_handle* h, int32_t n_cells, const double* skews, const int32_t* part_offsets,
                  const double* centers, const double* theta, const double* a, const double* b,
                  const int32_t* n_nodes) {
  return guarded(h, [&]() {
    if (!skews || !part_offsets || !centers || !theta || !a || !b) throw ApiError(SPM_EINVAL, "null array");
    h->cU[0] = 0.0;
    h->cU[1] = 0.0;
    h->have_lattice = true;
    if (n_cells < 1 || n_cells > 1024) throw ApiError(SPM_EINVAL, "number of cells must be in [1, 1024]");
    const int n = part_offsets[n_cells];
    if (n < 1) throw ApiError(SPM_EINVAL, "bad particle offsets");
    std::vector<int32_t> kind(n, SPM_SHAPE_ELLIPSE);
    std::vector<double> prm(4 * (size_t)n, 0.0);
    for (int i = 0; i < n; ++i) {
      prm[4 * i] = a[i];
      prm[4 * i + 1] = b[i];
    }
    set_cells_impl(h, n_cells, skews, part_offsets, centers, theta, kind.data(), prm.data(), n_nodes);
    return SPM_OK;
  });
}

int spm_set_cells_shapes(spm_handle* h, int32_t n_cells, const double* skews, const int32_t* part_offsets,
                         const double* centers, const double* theta, const int32_t* kind, const double* params,
                         const int32_t* n_nodes) {
  return guarded(h, [&]() {
    if (!skews || !part_offsets || !centers || !theta || !kind || !params) throw ApiError(SPM_EINVAL, "null array");
    h->cU[0] = 0.0;
    h->cU[1] = 0.0;
    h->have_lattice = true;
    set_cells_impl(h, n_cells, skews, part_offsets, centers, theta, kind, params, n_nodes);
    return SPM_OK;
  });
}

int spm_num_cells(const spm_handle* h, int32_t* C) {
  if (!h || !C) return SPM_EINVAL;
  if (!h->have_particles) return SPM_ESTATE;
  *C = h->geo.C;
  return SPM_OK;
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
    matvec(h, sigma, out, precision, false);
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
  return guarded(h, [&]() { return solve_api(h, sigma0, sigma, vel, omega, mu_eff, info_out, nullptr); });
}

int spm_solve_cells(spm_handle* h, const double* sigma0, double* sigma, double* vel, double* omega, double* mu_eff,
                    spm_solve_info* infos_host, double* cell_latency_s_host) {
  return guarded(h, [&]() {
    return solve_api(h, sigma0, sigma, vel, omega, mu_eff, infos_host, cell_latency_s_host);
  });
}

int spm_solve_batch(spm_handle* h, int32_t n_cells, const double* lattices, const int32_t* part_offsets,
                    const double* centers, const double* theta, const double* semi_a, const double* semi_b,
                    const int32_t* n_nodes, double* vel, double* omega, double* mu_eff, spm_solve_info* infos_host,
                    double* cell_latency_s_host) {
  return guarded(h, [&]() {
    if (!lattices || !part_offsets || !centers || !theta || !semi_a || !semi_b)
      throw ApiError(SPM_EINVAL, "null array");
    if (n_cells < 1 || n_cells > 1024) throw ApiError(SPM_EINVAL, "number of cells must be in [1, 1024]");
    const int n = part_offsets[n_cells];
    if (part_offsets[0] != 0 || n < 1) throw ApiError(SPM_EINVAL, "bad particle offsets");
    std::vector<double> skews(n_cells), du(n_cells), cen(2 * (size_t)n);
    std::vector<int32_t> kind(n, SPM_SHAPE_ELLIPSE);
    std::vector<double> prm(4 * (size_t)n, 0.0);
    for (int c = 0; c < n_cells; ++c) {
      const double* L = lattices + 6 * (size_t)c;
      if (L[0] != 1.0 || L[1] != 0.0 || L[3] != 1.0 || !std::isfinite(L[2]) || !std::isfinite(L[4]) ||
          !std::isfinite(L[5]))
        throw ApiError(SPM_EINVAL, "cell " + std::to_string(c) + ": the lattice must be e1 = (1, 0), e2 = (s, 1)");
      if (part_offsets[c + 1] < part_offsets[c] || part_offsets[c + 1] > n)
        throw ApiError(SPM_EINVAL, "bad particle offsets");
      skews[c] = L[2];
      // the cell is solved about the origin; u0 = (gamma y, 0) adds gamma c_y to the velocities
      du[c] = h->cfg.gamma * L[5];
      for (int i = part_offsets[c]; i < part_offsets[c + 1]; ++i) {
        cen[2 * i] = centers[2 * i] - L[4];
        cen[2 * i + 1] = centers[2 * i + 1] - L[5];
      }
    }
    for (int i = 0; i < n; ++i) {
      prm[4 * i] = semi_a[i];
      prm[4 * i + 1] = semi_b[i];
    }
    h->cU[0] = 0.0;
    h->cU[1] = 0.0;
    h->have_lattice = true;
    set_cells_impl(h, n_cells, skews.data(), part_offsets, cen.data(), theta, kind.data(), prm.data(), n_nodes);
    ensure(h, h->wk.batch_sigma, 2 * (size_t)h->geo.N);
    const int st = solve_api(h, nullptr, h->wk.batch_sigma, vel, omega, mu_eff, infos_host, cell_latency_s_host);
    if (vel) {
      ensure(h, h->wk.cell_du, (size_t)n_cells);
      upload(h, h->wk.cell_du, du.data(), n_cells * sizeof(double));
      launch_add_cell_velocity(h, h->wk.cell_du, vel);
      sync(h);
    }
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

int spm_eval_field(spm_handle* h, const double* sigma, int64_t n_targets, const double* xt, const double* yt,
                   double* u, double* p) {
  return guarded(h, [&]() {
    need_particles(h);
    if (h->geo.dilated) throw ApiError(SPM_EINVAL, "not available with the dilated near set");
    if (h->geo.C != 1) throw ApiError(SPM_EINVAL, "field evaluation runs on a single-cell handle");
    if (!sigma || n_targets < 0 || n_targets > ((int64_t)1 << 28) ||
        (n_targets > 0 && (!xt || !yt || !u || !p)))
      throw ApiError(SPM_EINVAL, "bad field arguments");
    if (n_targets == 0) return SPM_OK;
    Field& F = h->fd;
    ensure(h, F.iw, (size_t)h->geo.N);
    ensure(h, F.hp, 4 * (size_t)h->geo.N);
    ensure(h, F.vel, 2 * (size_t)h->geo.No);
    ensure(h, F.om, (size_t)h->geo.No);
    stage_xi(h, sigma, false);              // f = w sigma, net forces, proxy strengths
    launch_velocities(h, F.vel, F.om);      // rigid motions and the velocity gauge
    launch_vplus(h, sigma, true);           // boundary values of the Cauchy integrals
    launch_field(h, n_targets, xt, yt, u, p);
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

int spm_effective_viscosity_contour(spm_handle* h, const double* sigma, int32_t m, double* mu_eff) {
  return guarded(h, [&]() {
    need_particles(h);
    if (h->geo.dilated) throw ApiError(SPM_EINVAL, "not available with the dilated near set");
    if (!sigma || !mu_eff) throw ApiError(SPM_EINVAL, "null pointer");
    if (m == 0) m = 16;
    if (m < 4 || m > 128) throw ApiError(SPM_EINVAL, "contour quadrature order outside [4, 128]");
    std::vector<double> t, w;
    gauss_legendre(m, t, w);
    t.insert(t.end(), w.begin(), w.end());
    ensure(h, h->wk.contour_gl, (size_t)2 * m);
    ensure(h, h->wk.contour, (size_t)h->geo.C * 11 * m);
    SPM_HIP_CHECK(hipMemcpyAsync(h->wk.contour_gl, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice,
                                 h->stream));
    stage_xi(h, sigma, false);              // f = w sigma, proxy strengths of every cell
    launch_mu_eff_contour(h, m, mu_eff);
    sync(h);                                // also keeps t alive until its copy has run
    return SPM_OK;
  });
}

int spm_near_traction(spm_handle* h, const double* sigma, double* out, int32_t precision) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma || !out) throw ApiError(SPM_EINVAL, "null vector");
    if (precision != SPM_FP64 && precision != SPM_FP32) throw ApiError(SPM_EINVAL, "precision must be FP64 or FP32");
    launch_prep(h, sigma);
    if (h->fmm.on) {
      launch_fmm(h, out);
    } else {
      launch_near(h, precision);
      launch_near_sum_only(h, out, precision);
    }
    sync(h);
    return SPM_OK;
  });
}

int spm_fmm_stats(spm_handle* h, int32_t* levels, int32_t* order, double* p2p_pairs, double* m2l_translations) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!h->fmm.on) throw ApiError(SPM_ESTATE, "no FMM plan (near_method is not SPM_NEAR_FMM)");
    if (levels) *levels = h->fmm.L;
    if (order) *order = h->fmm.p;
    if (p2p_pairs) *p2p_pairs = h->fmm.p2p_pairs;
    if (m2l_translations) *m2l_translations = h->fmm.m2l;
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
      launch_vplus(h, sigma, false);
      launch_close_apply(h, sigma, out, precision);
    }
    if (precision == SPM_FP32) launch_self_fix(h, out, false);
    sync(h);
    return SPM_OK;
  });
}

int spm_proxy_strengths(spm_handle* h, const double* sigma, double* xi) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma || !xi) throw ApiError(SPM_EINVAL, "null vector");
    stage_xi(h, sigma, false);
    SPM_HIP_CHECK(hipMemcpyAsync(xi, h->wk.xi, (size_t)h->geo.C * 2 * h->per.M * sizeof(double),
                                 hipMemcpyDeviceToDevice, h->stream));
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
    download(h, row.data(), h->cl.row, (N + 1) * sizeof(int32_t));
    if (P > 0) {
      download(h, q.data(), h->cl.q, P * sizeof(int32_t));
      download(h, s.data(), h->cl.s, P * sizeof(int32_t));
    }
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
    need_particles(h);
    if (!out) throw ApiError(SPM_EINVAL, "null output");
    const size_t n = (size_t)h->geo.C * 8 * h->per.m * 2 * h->per.M;
    download(h, out, h->per.Qp, n * sizeof(double));
    return SPM_OK;
  });
}

int spm_proxy_svd(spm_handle* h, double* Q_host, double* s_host, int32_t* sweeps_host) {
  return guarded(h, [&]() {
    need_particles(h);
    const int C = h->geo.C, M = h->per.M;
    const size_t n = (size_t)C * 8 * h->per.m * 2 * M;
    if (Q_host) download(h, Q_host, h->per.Q, n * sizeof(double));
    std::vector<double> sv((size_t)C * (2 * M + 1));
    download(h, sv.data(), h->per.svd_s, sv.size() * sizeof(double));
    for (int c = 0; c < C; ++c) {
      if (s_host) std::memcpy(s_host + (size_t)c * 2 * M, sv.data() + (size_t)c * (2 * M + 1), 2 * M * sizeof(double));
      if (sweeps_host) sweeps_host[c] = (int32_t)sv[(size_t)c * (2 * M + 1) + 2 * M];
    }
    return SPM_OK;
  });
}

int spm_autotune(spm_handle* h, const char* cache_path, double* best_ms_host) {
  return guarded(h, [&]() {
    need_particles(h);
    if (h->fmm.on) throw ApiError(SPM_ESTATE, "the FMM near sum has no direct launch shapes to tune");
    autotune(h, cache_path, best_ms_host);
    sync(h);
    return SPM_OK;
  });
}

int spm_get_launch(spm_handle* h, int32_t precision, int32_t* cfg_host) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!cfg_host || (precision != SPM_FP64 && precision != SPM_FP32)) throw ApiError(SPM_EINVAL, "bad arguments");
    const NearConfig& c = h->wk.near[precision == SPM_FP64 ? 0 : 1].cfg;
    cfg_host[0] = c.block;
    cfg_host[1] = c.tpt;
    cfg_host[2] = c.tile;
    cfg_host[3] = c.wg_per_cu;
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
    c.wg_per_cu = cfg_host[3];
    if (!near_config_valid(c)) throw ApiError(SPM_EINVAL, "unsupported near-sum launch configuration");
    h->wk.near[precision == SPM_FP64 ? 0 : 1].cfg = c;
    if (!h->fmm.on) build_near_plan(h, precision);   // an FMM handle only keeps the shape
    h->wk.tuned = true;
    h->wk.tuned_N = h->geo.N;
    return SPM_OK;
  });
}

int spm_profile(spm_handle* h, int32_t enable) {
  return guarded(h, [&]() {
    prof_flush(h);
    h->prof = enable != 0;
    for (int k = 0; k < 4; ++k) {
      h->prof_ms[k] = 0;
      h->prof_launches[k] = 0;
      h->prof_pairs[k] = 0;
    }
    return SPM_OK;
  });
}

int spm_profile_read(spm_handle* h, int32_t kernel, double* total_ms, int64_t* launches, double* pairs) {
  return guarded(h, [&]() {
    if (kernel < 0 || kernel > 3) throw ApiError(SPM_EINVAL, "kernel id must be in [0, 3]");
    prof_flush(h);
    if (total_ms) *total_ms = h->prof_ms[kernel];
    if (launches) *launches = h->prof_launches[kernel];
    if (pairs) *pairs = h->prof_pairs[kernel];
    return SPM_OK;
  });
}

int spm_step_record(spm_handle* h, double dt, int32_t n_steps, double* t_inout, double* centers, double* theta,
                    double* mu_series, spm_solve_info* infos, float* features, float* targets) {
  return guarded(h, [&]() {
    need_particles(h);
    if (h->geo.C != 1) throw ApiError(SPM_EINVAL, "time stepping runs on a single cell");
    if (!t_inout || !centers || !theta || !mu_series || n_steps < 1 || !(dt > 0))
      throw ApiError(SPM_EINVAL, "bad step arguments");
    const int n = h->geo.No;
    std::vector<int32_t> kind(h->kind), nn(h->nn);
    std::vector<double> prm(h->prm);
    const double s0 = h->cells[0].skew_raw;
    const double t0 = *t_inout;
    const int64_t n2 = 2 * h->geo.N;
    ensure(h, h->kr.stepbuf, n2 + 3 * n + 2);
    double* sig = h->kr.stepbuf;
    double* vel = sig + n2;
    double* om = vel + 2 * n;
    double* mu = om + n;
    std::vector<double> hv(3 * n + 1);
    bool have_prev = false;
    for (int k = 0; k < n_steps; ++k) {
      const double sk = s0 + h->cfg.gamma * (k * dt);
      const int32_t off[2] = {0, n};
      *t_inout = t0 + k * dt;   // time of the state being solved (kept if this step fails)
      // a failure leaves the handle without particles (its lattice is the failing step's)
      h->have_particles = false;
      set_cells_impl(h, 1, &sk, off, centers, theta, kind.data(), prm.data(), nn.data());
      sig = h->kr.stepbuf;  // (buffers are stable: same sizes)
      spm_solve_info info;
      const double* guess = (h->cfg.x0 == SPM_X0_PREVIOUS && have_prev) ? sig : nullptr;
      const int rc = solve_api(h, guess, sig, vel, om, mu, &info, nullptr);
      if (infos) infos[k] = info;
      if (rc) {   // the state stays the one solved at *t_inout
        h->have_particles = false;
        return rc;
      }
      have_prev = true;
      if (features) launch_features(h, features + (int64_t)k * n * SPM_MLP_IN);
      if (targets) {
        gm_dot(h, sig, h->ln.nvec, h->ln.num);
        gm_dot(h, h->ln.nvec, h->ln.nvec, h->ln.den);
        launch_modes(h, sig, h->ln.num, h->ln.den, targets + (int64_t)k * n * SPM_MLP_OUT);
      }
      download(h, hv.data(), vel, (3 * n + 1) * sizeof(double));
      mu_series[k] = hv[3 * n];
      for (int i = 0; i < n; ++i) {
        centers[2 * i] = h->cx[i] + dt * hv[2 * i];
        centers[2 * i + 1] = h->cy[i] + dt * hv[2 * i + 1];
        theta[i] += dt * hv[2 * n + i];
      }
    }
    *t_inout = t0 + n_steps * dt;
    h->cells[0].skew_raw = s0 + h->cfg.gamma * n_steps * dt;
    h->pending_skew = h->cells[0].skew_raw;
    return SPM_OK;
  });
}

int spm_step(spm_handle* h, double dt, int32_t n_steps, double* t_inout, double* centers, double* theta,
             double* mu_series, spm_solve_info* infos) {
  return spm_step_record(h, dt, n_steps, t_inout, centers, theta, mu_series, infos, nullptr, nullptr);
}

int spm_precond_apply(spm_handle* h, const double* v, double* out) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!v || !out) throw ApiError(SPM_EINVAL, "null vector");
    if (!h->pc.valid) build_precond(h);
    launch_precond_apply(h, v, out, false);
    sync(h);
    return SPM_OK;
  });
}

int spm_features_f32(spm_handle* h, float* features) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!features) throw ApiError(SPM_EINVAL, "null features");
    launch_features(h, features);
    sync(h);
    return SPM_OK;
  });
}

int spm_features(spm_handle* h, uint16_t* feat_bf16) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!feat_bf16) throw ApiError(SPM_EINVAL, "null features");
    launch_features(h, h->ln.feat);
    launch_to_bf16(h, h->ln.feat, (int64_t)h->geo.No * SPM_MLP_IN, feat_bf16);
    sync(h);
    return SPM_OK;
  });
}

int spm_density_modes(spm_handle* h, const double* sigma, float* modes) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma || !modes) throw ApiError(SPM_EINVAL, "null argument");
    gm_dot(h, sigma, h->ln.nvec, h->ln.num);
    gm_dot(h, h->ln.nvec, h->ln.nvec, h->ln.den);
    launch_modes(h, sigma, h->ln.num, h->ln.den, modes);
    sync(h);
    return SPM_OK;
  });
}

int spm_warm_start(spm_handle* h, const float* modes, double* sigma0) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!modes || !sigma0) throw ApiError(SPM_EINVAL, "null argument");
    launch_rhs(h, h->kr.b);
    launch_decode(h, modes, sigma0);
    offset_fit(h, sigma0);
    sync(h);
    return SPM_OK;
  });
}

int spm_set_network(spm_handle* h, spm_mlp* net) {
  if (!h) return SPM_EINVAL;
  h->net = net;
  return SPM_OK;
}

int spm_learned_guess(spm_handle* h, double* sigma0) {
  return guarded(h, [&]() {
    need_particles(h);
    if (!sigma0) throw ApiError(SPM_EINVAL, "null sigma0");
    launch_rhs(h, h->kr.b);
    network_decode(h, sigma0);
    offset_fit(h, sigma0);
    sync(h);
    return SPM_OK;
  });
}

}  // extern "C"
