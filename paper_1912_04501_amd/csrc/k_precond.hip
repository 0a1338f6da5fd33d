// Block preconditioner: inverses of the isolated-body self blocks of the completed
// operator (Sec. 5 eq. BIEPerturbed for one body in free space, Sec. 6 Nystrom rule),
// one per particle shape (a, b, N), in the body frame.
//
//   B sigma = sigma/2 + sum_{j != i} G^t(x_i, y_j; n_i) w_j sigma_j
//             - (kappa_i / 2 pi) tau_i tau_i^T w_i sigma_i + F + x_i^perp tau,
//   F = sum_j w_j sigma_j,  tau = sum_j w_j x_j^perp . sigma_j  (x relative to the centre).
//
// Unknowns and rows are ordered [sigma_1(0..n-1), sigma_2(0..n-1)] (m = 2n). The blocks are
// assembled in FP64 (m x m, row-major), inverted in place by blocked Gauss-Jordan elimination
// with partial pivoting (one 1024-thread workgroup per shape), and stored in FP32 column-major,
// so that applying them reads coalesced columns.
#include "spm_internal.h"

namespace spm {

__device__ __forceinline__ void body_node(const ShapeDesc& d, int k, double& x, double& y, double& tx, double& ty,
                                          double& w, double& kap) {
  const double t = 2.0 * kPi * (double)k / (double)d.n;
  double dx, dy, ddx, ddy;
  shape_point(d.kind, d.p, t, x, y, dx, dy, ddx, ddy);
  const double sp = sqrt(dx * dx + dy * dy);
  tx = dx / sp;
  ty = dy / sp;
  w = 2.0 * kPi * sp / (double)d.n;
  kap = (dx * ddy - dy * ddx) / (sp * sp * sp);
}

// block (row i, shape): both rows (component 1 and 2) of node i of B
__global__ __launch_bounds__(256) void k_self_block(const ShapeDesc* __restrict__ sh, double* __restrict__ work) {
  const ShapeDesc d = sh[blockIdx.y];
  const int n = d.n, m = 2 * n, ld = m;
  const int i = blockIdx.x;
  if (i >= n) return;
  double xi, yi, txi, tyi, wi, ki;
  body_node(d, i, xi, yi, txi, tyi, wi, ki);
  const double nxi = tyi, nyi = -txi;
  double* r1 = work + d.woff + (int64_t)i * ld;         // row of component 1
  double* r2 = work + d.woff + (int64_t)(n + i) * ld;   // row of component 2
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double xj, yj, txj, tyj, wj, kj;
    body_node(d, j, xj, yj, txj, tyj, wj, kj);
    double m11, m12, m21, m22;
    if (j == i) {
      const double c = -(ki / (2.0 * kPi)) * wi;
      m11 = c * txi * txi;
      m12 = c * txi * tyi;
      m21 = m12;
      m22 = c * tyi * tyi;
    } else {
      const double rx = xi - xj, ry = yi - yj;
      const double r2 = rx * rx + ry * ry;
      const double c = -(rx * nxi + ry * nyi) / (kPi * r2 * r2) * wj;
      m11 = c * rx * rx;
      m12 = c * rx * ry;
      m21 = m12;
      m22 = c * ry * ry;
    }
    // completion: net force (w_j delta_cd) and torque (perp_c(i) w_j perp_d(j)), perp = (-y, x)
    const double pi1 = -yi, pi2 = xi, pj1 = -yj, pj2 = xj;
    m11 += wj + pi1 * wj * pj1;
    m12 += pi1 * wj * pj2;
    m21 += pi2 * wj * pj1;
    m22 += wj + pi2 * wj * pj2;
    if (j == i) {
      m11 += 0.5;
      m22 += 0.5;
    }
    r1[j] = m11;
    r1[n + j] = m12;
    r2[j] = m21;
    r2[n + j] = m22;
  }
}

// One workgroup per shape: B (m x m, row-major) -> X = (P B)^-1 in place, P the row
// permutation of partial pivoting (perm[i] = the row of B that ends at row i, stored after the
// matrix); B^-1 = X P, i.e. column i of X is column perm[i] of B^-1. status[shape] = 1 if a
// pivot is zero.
//
// Blocked Gauss-Jordan: the columns are taken in panels of kGJPanel. Within a panel each pivot
// column is eliminated from every row on the panel's columns only: rows swap whole (their pending
// updates travel with them), the pivot row is scaled, and the pivot column is replaced by its
// column of the inverse (1/piv at the pivot, -a_ik/piv elsewhere). The panel's composite
// elementary transform E is the identity with the pivot columns replaced by the panel P, so the
// other columns T are then updated in one pass: T_i += P_i T_R for the non-pivot rows i and
// T_R = P_R T_R for the pivot rows R (T_R read before it is overwritten). One pass over the
// matrix per panel instead of one per pivot.
constexpr int kGJPanel = 32;
constexpr int kGJRowChunk = 128;

__global__ __launch_bounds__(1024) void k_gauss_jordan(const ShapeDesc* __restrict__ sh, double* __restrict__ work,
                                                       int32_t* __restrict__ status) {
  constexpr int PB = kGJPanel, RC = kGJRowChunk;
  __shared__ double Pl[RC * PB];                   // panel rows of one row chunk
  __shared__ double fcol[2 * kMaxNodesStaged];     // pivot column, every row
  __shared__ double prow[PB];                      // scaled pivot row, panel columns
  __shared__ double rv[1024];
  __shared__ int ri[1024];
  const ShapeDesc d = sh[blockIdx.x];
  const int m = 2 * d.n;
  double* A = work + d.woff;
  int32_t* perm = reinterpret_cast<int32_t*>(A + (int64_t)m * m);
  const int t = threadIdx.x, T = blockDim.x;
  for (int i = t; i < m; i += T) perm[i] = i;
  int bad = 0;
  for (int kb = 0; kb < m; kb += PB) {
    const int ke = min(kb + PB, m), pw = ke - kb;
    // ---- panel ----
    for (int k = kb; k < ke; ++k) {
      double best = -1.0;
      int bi = k;
      for (int i = k + t; i < m; i += T) {
        const double v = fabs(A[(int64_t)i * m + k]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      rv[t] = best;
      ri[t] = bi;
      __syncthreads();
      for (int o = T / 2; o > 0; o >>= 1) {
        if (t < o) {
          const double v2 = rv[t + o];
          const int i2 = ri[t + o];
          if (v2 > rv[t] || (v2 == rv[t] && i2 < ri[t])) {
            rv[t] = v2;
            ri[t] = i2;
          }
        }
        __syncthreads();
      }
      const int p = ri[0];
      double piv = A[(int64_t)p * m + k];
      if (piv == 0.0) {
        bad = 1;
        piv = 1.0;
      }
      __syncthreads();   // every thread has read ri[0] and the pivot before the rows move
      if (p != k) {
        for (int j = t; j < m; j += T) {
          const double a = A[(int64_t)k * m + j];
          A[(int64_t)k * m + j] = A[(int64_t)p * m + j];
          A[(int64_t)p * m + j] = a;
        }
        if (t == 0) {
          const int32_t q = perm[k];
          perm[k] = perm[p];
          perm[p] = q;
        }
      }
      __syncthreads();
      for (int i = t; i < m; i += T) fcol[i] = A[(int64_t)i * m + k];
      if (t < pw) prow[t] = (kb + t == k) ? 1.0 / piv : A[(int64_t)k * m + kb + t] / piv;
      __syncthreads();
      for (int e = t; e < m * pw; e += T) {
        const int i = e / pw, jj = e - i * pw;
        double* a = A + (int64_t)i * m + kb + jj;
        if (i == k)
          *a = prow[jj];
        else if (kb + jj == k)
          *a = -fcol[i] / piv;
        else
          *a = fma(-fcol[i], prow[jj], *a);
      }
      __syncthreads();
    }
    // ---- the other columns: j in [0, kb) and [ke, m), at most one per thread (m <= 1024) ----
    const int nJ = m - pw;
    if (nJ > 0) {
      const int CT = min(T, (nJ + 63) / 64 * 64);   // column threads
      const int G = T / CT;                          // row groups
      const int cg = t % CT, g = t / CT;
      const bool col = g < G && cg < nJ;
      const int j = cg < kb ? cg : cg + pw;
      double tr[PB];
#pragma unroll
      for (int r = 0; r < PB; ++r) tr[r] = (col && r < pw) ? A[(int64_t)(kb + r) * m + j] : 0.0;
      // non-pivot rows, in chunks of RC rows whose panel entries pass through LDS
      for (int i0 = 0; i0 < m; i0 += RC) {
        const int ie = min(i0 + RC, m);
        __syncthreads();
        for (int e = t; e < (ie - i0) * PB; e += T) {
          const int ii = e / PB, r = e - ii * PB;
          Pl[e] = r < pw ? A[(int64_t)(i0 + ii) * m + kb + r] : 0.0;
        }
        __syncthreads();
        if (col) {
          for (int i = i0 + g; i < ie; i += G) {
            if (i >= kb && i < ke) continue;
            double acc = A[(int64_t)i * m + j];
            const double* pr = Pl + (i - i0) * PB;
#pragma unroll
            for (int r = 0; r < PB; ++r) acc = fma(pr[r], tr[r], acc);
            A[(int64_t)i * m + j] = acc;
          }
        }
      }
      // pivot rows: T_R = P_R T_R (the old T_R is in tr)
      __syncthreads();
      for (int e = t; e < PB * PB; e += T) {
        const int q = e / PB, r = e - q * PB;
        Pl[e] = (q < pw && r < pw) ? A[(int64_t)(kb + q) * m + kb + r] : 0.0;
      }
      __syncthreads();
      if (col) {
        for (int q = g; q < pw; q += G) {
          double acc = 0.0;
#pragma unroll
          for (int r = 0; r < PB; ++r) acc = fma(Pl[q * PB + r], tr[r], acc);
          A[(int64_t)(kb + q) * m + j] = acc;
        }
      }
    }
    __syncthreads();
  }
  if (t == 0) status[blockIdx.x] = bad;
}

// Row segments of a 2n x 2n inverse: segment y holds nodes [y nk, y nk + kn) (kn = min(nk, n - y nk),
// nk = ceil(n / R) rounded up to even), i.e. rows k and n + k of the inverse for those nodes. Storage is
// by segment, each segment column-major over its own 2 kn rows (first the kn rows k, then the kn rows
// n + k), so that the workgroup applying a segment streams one contiguous region:
//   element (r, c), r = k or n + k with k in segment y: ioff + y (2 nk) m + c (2 kn) + (r < n ? 0 : kn) + k - y nk.
__host__ __device__ __forceinline__ int precond_seg_nodes(int n, int R) { return 2 * ((n + 2 * R - 1) / (2 * R)); }

__device__ __forceinline__ int64_t precond_index(int n, int R, int r, int c) {
  const int m = 2 * n, nk = precond_seg_nodes(n, R);
  const int k = r < n ? r : r - n;
  const int y = k / nk, k0 = y * nk;
  const int kn = min(nk, n - k0);
  return (int64_t)y * 2 * nk * m + (int64_t)c * 2 * kn + (r < n ? 0 : kn) + (k - k0);
}

// element (r, perm[i]) of the inverse = (float) X[r][i]: column i of X is column perm[i] of B^-1
__global__ void k_store_inverse(const ShapeDesc* __restrict__ sh, const double* __restrict__ work, int R,
                                float* __restrict__ inv) {
  const ShapeDesc d = sh[blockIdx.y];
  const int m = 2 * d.n;
  const int i = blockIdx.x;
  if (i >= m) return;
  const double* X = work + d.woff;
  const int32_t* perm = reinterpret_cast<const int32_t*>(X + (int64_t)m * m);
  const int c = perm[i];
  for (int r = threadIdx.x; r < m; r += blockDim.x) inv[d.ioff + precond_index(d.n, R, r, c)] = (float)X[(int64_t)r * m + i];
}

// Non-temporal load of a pair of inverse entries: each entry is read once per product, and the
// inverses (about 2 GB for 1000 particles of 350 nodes) would only evict what the caches hold.
__device__ __forceinline__ float2 stream_load(const float2* p) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
  return make_float2(v.x, v.y);
}

// Blocks (particle, row segment): out = R (B^-1 (R^T v)) on the particle's nodes, segment y
// producing nodes [y nk, (y + 1) nk) (rows k and n + k of the 2n x 2n inverse, nk = ceil(n / R)
// rounded up to even), so that small particle counts still spread over the chip. Particles of
// inactive cells are skipped when active is given. The segment's 2 kn rows are contiguous in every
// column (kn and n even), read as pairs (8-byte loads); the columns are split into S = blockDim / nk
// groups whose lanes run over consecutive row pairs. The S partial rows are summed in a fixed order.
__global__ __launch_bounds__(1024) void k_precond_apply(Geo g, const int32_t* __restrict__ pshape,
                                                        const int64_t* __restrict__ ioff,
                                                        const float* __restrict__ inv,
                                                        const int32_t* __restrict__ active, int R,
                                                        const double* __restrict__ v, double* __restrict__ out) {
  __shared__ double vb[2 * kMaxNodesStaged];
  __shared__ double part[2048];
  const int q = blockIdx.x;
  if (active && active[g.pcell[q]] == 0) return;
  const int n = g.pn[q], m = 2 * n;
  const int nk = precond_seg_nodes(n, R);
  const int k0 = blockIdx.y * nk;
  if (k0 >= n) return;
  const int kn = min(nk, n - k0);            // even: n and k0 are
  const int64_t i0 = g.poff[q], N = g.N;
  double st, ct;
  sincos(g.pth[q], &st, &ct);
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double a = v[i0 + k], b = v[N + i0 + k];
    vb[k] = ct * a + st * b;
    vb[n + k] = -st * a + ct * b;
  }
  __syncthreads();
  const float2* M2 = reinterpret_cast<const float2*>(inv + ioff[pshape[q]] + (int64_t)blockIdx.y * 2 * nk * m);
  const int pairs = nk;                      // row pairs of the block: nk / 2 per range, two ranges
  const int S = max(1, (int)blockDim.x / pairs);
  const int grp = threadIdx.x / pairs, rp = threadIdx.x % pairs;
  const int half = nk / 2;
  const int lk = 2 * (rp < half ? rp : rp - half);   // first node of the pair within the segment
  if (grp < S && lk < kn) {
    const int rr = (rp < half ? 0 : kn) + lk;          // even row within the segment
    double a0 = 0.0, a1 = 0.0;
    int c = grp;
    for (; c + 3 * S < m; c += 4 * S) {   // four columns' loads in flight, summed in column order
      float2 w[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] = stream_load(M2 + (((int64_t)(c + u * S) * 2 * kn + rr) >> 1));
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a0 = fma((double)w[u].x, vb[c + u * S], a0);
        a1 = fma((double)w[u].y, vb[c + u * S], a1);
      }
    }
    for (; c < m; c += S) {
      const float2 w = stream_load(M2 + (((int64_t)c * 2 * kn + rr) >> 1));
      a0 = fma((double)w.x, vb[c], a0);
      a1 = fma((double)w.y, vb[c], a1);
    }
    part[grp * 2 * pairs + 2 * rp] = a0;
    part[grp * 2 * pairs + 2 * rp + 1] = a1;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kn; k += blockDim.x) {
    double a = 0.0, b = 0.0;
    for (int s = 0; s < S; ++s) {
      a += part[s * 2 * pairs + k];
      b += part[s * 2 * pairs + nk + k];
    }
    out[i0 + k0 + k] = ct * a - st * b;
    out[N + i0 + k0 + k] = st * a + ct * b;
  }
}

// Row segments per particle: about 1,024 apply workgroups in all, at most 8 per particle.
static int precond_segments(const spm_handle* h) {
  return std::max(1, std::min({8, (1024 + h->geo.No - 1) / h->geo.No, h->geo.nmax}));
}

// Builds the inverses of the shapes listed in h->pc (host keys), in batches whose
// [B | I] work arrays stay below ~1 GB.
void build_precond(spm_handle* h) {
  Precond& P = h->pc;
  if (h->geo.nmax > kMaxNodesStaged)
    throw ApiError(SPM_EINVAL, "the block preconditioner needs at most " + std::to_string(kMaxNodesStaged) +
                                   " nodes per particle");
  const int S = (int)P.keys.size();
  auto nodes = [&](int s) { return (int32_t)P.keys[s][5]; };
  P.segs = precond_segments(h);
  std::vector<int64_t> ioff(S);
  int64_t total = 0;
  for (int s = 0; s < S; ++s) {
    ioff[s] = total;
    total += 4LL * nodes(s) * nodes(s);
  }
  P.inv = static_cast<float*>(precond_alloc(h, P.inv, (size_t)total * sizeof(float), P.inv_cap));
  P.ioff = static_cast<int64_t*>(precond_alloc(h, P.ioff, (size_t)S * sizeof(int64_t), P.ioff_cap));
  SPM_HIP_CHECK(hipMemcpyAsync(P.ioff, ioff.data(), S * sizeof(int64_t), hipMemcpyHostToDevice, h->stream));
  const int64_t budget = (int64_t)1 << 27;   // doubles of work per batch (1 GiB)
  int s0 = 0;
  while (s0 < S) {
    std::vector<ShapeDesc> batch;
    int64_t w = 0;
    int maxn = 0;
    for (int s = s0; s < S; ++s) {
      const int64_t need = 4LL * nodes(s) * nodes(s) + nodes(s);   // m x m doubles, then m int32 (perm)
      if (!batch.empty() && w + need > budget) break;
      ShapeDesc d;
      d.kind = (int32_t)P.keys[s][0];
      for (int k = 0; k < 4; ++k) d.p[k] = P.keys[s][1 + k];
      d.n = nodes(s);
      d.woff = w;
      d.ioff = ioff[s];
      batch.push_back(d);
      w += need;
      maxn = std::max(maxn, nodes(s));
    }
    const int nb = (int)batch.size();
    P.work = static_cast<double*>(precond_alloc(h, P.work, (size_t)w * sizeof(double), P.work_cap));
    P.desc = static_cast<ShapeDesc*>(precond_alloc(h, P.desc, (size_t)nb * sizeof(ShapeDesc), P.desc_cap));
    P.status = static_cast<int32_t*>(precond_alloc(h, P.status, (size_t)nb * sizeof(int32_t), P.status_cap));
    SPM_HIP_CHECK(hipMemcpyAsync(P.desc, batch.data(), nb * sizeof(ShapeDesc), hipMemcpyHostToDevice, h->stream));
    k_self_block<<<dim3((unsigned)maxn, (unsigned)nb), 256, 0, h->stream>>>(P.desc, P.work);
    SPM_HIP_CHECK(hipGetLastError());
    k_gauss_jordan<<<nb, 1024, 0, h->stream>>>(P.desc, P.work, P.status);
    SPM_HIP_CHECK(hipGetLastError());
    k_store_inverse<<<dim3((unsigned)(2 * maxn), (unsigned)nb), 256, 0, h->stream>>>(P.desc, P.work, P.segs, P.inv);
    SPM_HIP_CHECK(hipGetLastError());
    std::vector<int32_t> st(nb);
    SPM_HIP_CHECK(hipMemcpyAsync(st.data(), P.status, nb * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    SPM_HIP_CHECK(hipStreamSynchronize(h->stream));
    for (int k = 0; k < nb; ++k)
      if (st[k]) throw ApiError(SPM_EINVAL, "singular self block");
    s0 += nb;
  }
  // the work array is only needed while building
  precond_release_work(h);
  P.valid = true;
}

void launch_precond_apply(spm_handle* h, const double* v, double* out, bool with_active) {
  Precond& P = h->pc;
  if (h->geo.nmax > kMaxNodesStaged)
    throw ApiError(SPM_EINVAL, "the block preconditioner needs at most " + std::to_string(kMaxNodesStaged) +
                                   " nodes per particle");
  // the row segments the inverses were stored with
  const int R = P.segs;
  k_precond_apply<<<dim3(h->geo.No, R), 1024, 0, h->stream>>>(h->geo, P.pshape, P.ioff, P.inv,
                                                              with_active ? h->kr.active : nullptr, R, v, out);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace spm
