// The warm-start network: a 33 -> 256 -> 256 -> 256 -> 128 ReLU MLP, trained and run
// on the device (forward, back-propagation, mean-squared loss, Adam).
//
// Every layer product is one tiled matrix-core GEMM: 64 x 64 output tiles per
// 256-thread workgroup, four waves of 2 x 2 16x16 MFMA blocks, 32-deep K slices
// staged through LDS. Operands are FP32 in memory (master weights, activations);
// in BF16 mode they are rounded to bfloat16 (nearest even) when fragments are
// built and multiplied with v_mfma_f32_16x16x32_bf16, the whole 32-deep slice in one
// instruction per 16x16 block (FP32 accumulation); in FP32
// mode v_mfma_f32_16x16x4_f32 multiplies them exactly (the gradient-check mode).
// Bias, ReLU and the ReLU derivative mask are fused into the GEMM epilogue.
//
// Parameter packing (FP32, one array): W0 [256 x 33], b0 [256], W1 [256 x 256], b1,
// W2 [256 x 256], b2, W3 [128 x 256], b3; W is row-major (out x in).
#include "spm_internal.h"

namespace spm {

namespace {

typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kIn = SPM_MLP_IN, kHid = SPM_MLP_HIDDEN, kOut = SPM_MLP_OUT;
constexpr int kLayers = 4;
constexpr int kFanIn[kLayers] = {kIn, kHid, kHid, kHid};
constexpr int kFanOut[kLayers] = {kHid, kHid, kHid, kOut};

constexpr int64_t w_off(int l) {
  int64_t o = 0;
  for (int k = 0; k < l; ++k) o += (int64_t)kFanOut[k] * kFanIn[k] + kFanOut[k];
  return o;
}
constexpr int64_t b_off(int l) { return w_off(l) + (int64_t)kFanOut[l] * kFanIn[l]; }
static_assert(w_off(kLayers) == SPM_MLP_NPARAMS, "parameter count");

// C(m, n) = epilogue(sum_k A(m, k) B(k, n))
//   A(m, k) = A[row_a(m) * sam + k * sak], row_a(m) = arow ? arow[m] : m
//   B(k, n) = B[row_b(k) * sbk + n * sbn], row_b(k) = bk ? bk[k] : k
//   epilogue: + bias[n], then ReLU, then * (mask(m, n) > 0); C[m * ldc + n] = value.
struct Gemm {
  const float* A;
  int64_t sam, sak;
  const int32_t* arow;
  const float* B;
  int64_t sbk, sbn;
  const int32_t* bk;
  float* C;
  int64_t ldc;
  int M, N, K;
  const float* bias;
  int relu;
  const float* mask;
  int64_t ldm;
};

__device__ __forceinline__ short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

constexpr int BM = 64, BN = 64, BK = 32, LDP = BK + 1;

template <int MODE>
__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
  __shared__ float As[BM * LDP];   // As[r][k]
  __shared__ float Bs[BN * LDP];   // Bs[n][k]
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
    for (int i = 0; i < (BM * BK) / 256; ++i) {
      const int e = t + 256 * i;
      int r, kk;
      if (g.sak == 1) {
        r = e / BK;
        kk = e % BK;
      } else {
        r = e % BM;
        kk = e / BM;
      }
      const int m = m0 + r, k = k0 + kk;
      float v = 0.f;
      if (m < g.M && k < g.K) {
        const int64_t row = g.arow ? (int64_t)g.arow[m] : (int64_t)m;
        v = g.A[row * g.sam + (int64_t)k * g.sak];
      }
      As[r * LDP + kk] = v;
    }
#pragma unroll
    for (int i = 0; i < (BN * BK) / 256; ++i) {
      const int e = t + 256 * i;
      int n, kk;
      if (g.sbn == 1) {
        n = e % BN;
        kk = e / BN;
      } else {
        n = e / BK;
        kk = e % BK;
      }
      const int nn = n0 + n, k = k0 + kk;
      float v = 0.f;
      if (nn < g.N && k < g.K) {
        const int64_t row = g.bk ? (int64_t)g.bk[k] : (int64_t)k;
        v = g.B[row * g.sbk + (int64_t)nn * g.sbn];
      }
      Bs[n * LDP + kk] = v;
    }
    __syncthreads();
    const int lr = lane & 15, lq = lane >> 4;
    if (MODE == SPM_MLP_BF16) {
      // Lane l holds row (or column) l % 16 and the eight k of group l / 16; A and B use the
      // same k assignment, so the product is the sum over the whole slice.
      static_assert(BK == 32, "one 16x16x32 product per slice");
      shortx8 fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float* pa = As + (32 * wm + 16 * i + lr) * LDP + 8 * lq;
        const float* pb = Bs + (32 * wn + 16 * i + lr) * LDP + 8 * lq;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          fa[i][q] = to_bf16(pa[q]);
          fb[i][q] = to_bf16(pb[q]);
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, fa[i]),
                                                              __builtin_bit_cast(bf16x8, fb[j]), acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        float fa[2], fb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          fa[i] = As[(32 * wm + 16 * i + lr) * LDP + ks + lq];
          fb[i] = Bs[(32 * wn + 16 * i + lr) * LDP + ks + lq];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // D layout of a 16x16 block: lane l, element q -> row 4 (l / 16) + q, column l % 16
  const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 32 * wm + 16 * i + 4 * lq + q;
        const int n = n0 + 32 * wn + 16 * j + lr;
        if (m < g.M && n < g.N) {
          float v = acc[i][j][q];
          if (g.bias) v += g.bias[n];
          if (g.relu) v = v > 0.f ? v : 0.f;
          if (g.mask && !(g.mask[(int64_t)m * g.ldm + n] > 0.f)) v = 0.f;
          g.C[(int64_t)m * g.ldc + n] = v;
        }
      }
}

void gemm(hipStream_t s, int mode, const Gemm& g) {
  if (g.M <= 0 || g.N <= 0) return;
  dim3 grid((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM));
  if (mode == SPM_MLP_BF16)
    k_gemm<SPM_MLP_BF16><<<grid, 256, 0, s>>>(g);
  else
    k_gemm<SPM_MLP_FP32><<<grid, 256, 0, s>>>(g);
  SPM_HIP_CHECK(hipGetLastError());
}

// dZ = (Y - T(row)) / B; part[block] = sum of (Y - T)^2 over the block's elements.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ Y, const float* __restrict__ T,
                                              const int32_t* __restrict__ trow, int64_t B, float invB,
                                              float* __restrict__ dZ, double* __restrict__ part) {
  __shared__ double sc[16];
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double s = 0.0;
  if (e < B * kOut) {
    const int64_t b = e / kOut, o = e % kOut;
    const int64_t row = trow ? (int64_t)trow[b] : b;
    const float d = Y[e] - T[row * kOut + o];
    dZ[e] = d * invB;
    s = (double)d * (double)d;
  }
  s = block_sum(s, sc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[0] = 0.5 sum(part) / B (one block, fixed order)
__global__ void k_loss_final(const double* __restrict__ part, int64_t nb, double invB, float* __restrict__ out,
                             double* __restrict__ out64) {
  __shared__ double sc[16];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < nb; k += blockDim.x) s += part[k];
  s = block_sum(s, sc);
  if (threadIdx.x == 0) {
    if (out) out[0] = (float)(0.5 * s * invB);
    if (out64) out64[0] = 0.5 * s * invB;
  }
}

// db[n] = sum_m dZ[m, n]
__global__ void k_colsum(const float* __restrict__ dZ, int64_t M, int N, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int64_t m = 0; m < M; ++m) s += dZ[m * N + n];
  db[n] = s;
}

__global__ void k_adam(int64_t P, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  p[i] -= lr * (a / bc1) / (sqrtf(v / bc2) + eps);
}

// flag[0] = 1 if any idx is outside [0, n) (the flag is cleared before the launch;
// every writer stores the same value).
__global__ void k_check_rows(const int32_t* __restrict__ idx, int64_t cnt, int64_t n, int32_t* __restrict__ flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    if (idx[i] < 0 || idx[i] >= n) flag[0] = 1;
}

__global__ void k_fill(int64_t n, float* __restrict__ a, float v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// master[i] = bf16 value widened to FP32 (exact).
__global__ void k_widen_bf16(int64_t n, const uint16_t* __restrict__ b, float* __restrict__ d) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) d[i] = __uint_as_float((unsigned)b[i] << 16);
}

// flag[0] = 1 if some b[i] is not the nearest-even bfloat16 rounding of master[i] (the flag
// is cleared before the launch; every writer stores the same value).
__global__ void k_check_bf16(int64_t n, const uint16_t* __restrict__ b, const float* __restrict__ master,
                             int32_t* __restrict__ flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && (uint16_t)to_bf16(master[i]) != b[i]) flag[0] = 1;
}

__global__ void k_copyf(int64_t n, float* __restrict__ d, const float* __restrict__ s) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

template <typename T>
void grow(spm_mlp* net, T*& p, size_t count) {
  if (p) {
    if (net->free_fn)
      net->free_fn(p, net->stream, net->alloc_ctx);
    else
      (void)hipFree(p);
    p = nullptr;
  }
  void* q = nullptr;
  const size_t bytes = count * sizeof(T);
  if (net->alloc) {
    q = net->alloc(bytes, net->stream, net->alloc_ctx);
  } else if (hipMalloc(&q, bytes) != hipSuccess) {
    q = nullptr;
  }
  if (!q) throw ApiError(SPM_ENOMEM, "allocation of " + std::to_string(bytes) + " bytes failed");
  p = static_cast<T*>(q);
}

void ensure_batch(spm_mlp* net, int64_t B) {
  if (B <= net->cap) return;
  const int64_t c = std::max<int64_t>(B, 256);
  grow(net, net->h[0], (size_t)c * kHid);
  grow(net, net->h[1], (size_t)c * kHid);
  grow(net, net->h[2], (size_t)c * kHid);
  grow(net, net->y, (size_t)c * kOut);
  grow(net, net->dz[0], (size_t)c * kHid);
  grow(net, net->dz[1], (size_t)c * kHid);
  grow(net, net->part, (size_t)((c * kOut + 255) / 256));
  net->cap = c;
}

void launch_fill(hipStream_t s, float* a, int64_t n, float v) {
  k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, a, v);
  SPM_HIP_CHECK(hipGetLastError());
}

}  // namespace

// Forward pass of B rows; x rows are x[xrow[b]] (xrow may be null). Activations stay
// in the network's buffers (h[0..2]); the output goes to y (may be net->y).
void mlp_forward(spm_mlp* net, hipStream_t s, const float* x, const int32_t* xrow, int64_t B, float* y, int mode) {
  ensure_batch(net, B);
  const float* in = x;
  const int32_t* rows = xrow;
  int64_t ld_in = kIn;
  for (int l = 0; l < kLayers; ++l) {
    Gemm g{};
    g.A = in;
    g.sam = ld_in;
    g.sak = 1;
    g.arow = rows;
    g.B = net->params + w_off(l);   // B(k, n) = W[n][k]
    g.sbk = 1;
    g.sbn = kFanIn[l];
    g.bk = nullptr;
    g.M = (int)B;
    g.N = kFanOut[l];
    g.K = kFanIn[l];
    g.bias = net->params + b_off(l);
    g.relu = l < kLayers - 1;
    g.mask = nullptr;
    g.C = l < kLayers - 1 ? net->h[l] : y;
    g.ldc = kFanOut[l];
    gemm(s, mode, g);
    in = g.C;
    rows = nullptr;
    ld_in = kFanOut[l];
  }
}

// Gradients of the packed parameters for the upstream gradient dY [B x 128] (dL/dy of the
// rows of the last forward pass, which left its activations in h[0..2]); x rows xrow[b]
// (xrow may be null). dY is only read.
void mlp_backprop(spm_mlp* net, hipStream_t s, const float* x, const int32_t* xrow, const float* dY, int64_t B,
                  int mode, float* grads) {
  const float* dZ = dY;
  for (int l = kLayers - 1; l >= 0; --l) {
    const float* hin = l > 0 ? net->h[l - 1] : x;
    const int32_t* hrow = l > 0 ? nullptr : xrow;
    // dW_l [out x in] = dZ^T [out x B] . H_in [B x in]
    Gemm gw{};
    gw.A = dZ;
    gw.sam = 1;
    gw.sak = kFanOut[l];
    gw.arow = nullptr;
    gw.B = hin;
    gw.sbk = kFanIn[l];
    gw.sbn = 1;
    gw.bk = hrow;
    gw.M = kFanOut[l];
    gw.N = kFanIn[l];
    gw.K = (int)B;
    gw.C = grads + w_off(l);
    gw.ldc = kFanIn[l];
    gemm(s, mode, gw);
    k_colsum<<<(kFanOut[l] + 255) / 256, 256, 0, s>>>(dZ, B, kFanOut[l], grads + b_off(l));
    SPM_HIP_CHECK(hipGetLastError());
    if (l == 0) break;
    // dZ_{l-1} [B x in] = (dZ [B x out] . W_l [out x in]) * (H_{l-1} > 0)
    float* dn = dZ == net->dz[0] ? net->dz[1] : net->dz[0];
    Gemm gd{};
    gd.A = dZ;
    gd.sam = kFanOut[l];
    gd.sak = 1;
    gd.B = net->params + w_off(l);
    gd.sbk = kFanIn[l];
    gd.sbn = 1;
    gd.M = (int)B;
    gd.N = kFanIn[l];
    gd.K = kFanOut[l];
    gd.mask = net->h[l - 1];
    gd.ldm = kFanIn[l];
    gd.C = dn;
    gd.ldc = kFanIn[l];
    gemm(s, mode, gd);
    dZ = dn;
  }
}

// Loss and gradients of B rows (x rows xrow[b], target rows trow[b]; either may be null).
void mlp_backward(spm_mlp* net, hipStream_t s, const float* x, const int32_t* xrow, const float* T,
                  const int32_t* trow, int64_t B, int mode, float* grads, float* loss_f, double* loss_d) {
  mlp_forward(net, s, x, xrow, B, net->y, mode);
  const int64_t nel = B * kOut;
  const int64_t nb = (nel + 255) / 256;
  float* dZ = net->dz[0];
  k_loss<<<(unsigned)nb, 256, 0, s>>>(net->y, T, trow, B, 1.0f / (float)B, dZ, net->part);
  SPM_HIP_CHECK(hipGetLastError());
  k_loss_final<<<1, 256, 0, s>>>(net->part, nb, 1.0 / (double)B, loss_f, loss_d);
  SPM_HIP_CHECK(hipGetLastError());
  mlp_backprop(net, s, x, xrow, dZ, B, mode, grads);
}

}  // namespace spm

using namespace spm;

namespace {
int mlp_fail(spm_mlp* n, int code, const std::string& msg) {
  if (n) n->err = msg;
  return code;
}

template <typename F>
int mlp_guarded(spm_mlp* n, F&& f) {
  if (!n) return SPM_EINVAL;
  try {
    return f();
  } catch (const HipError& e) {
    return mlp_fail(n, SPM_EHIP, std::string("HIP error ") + hipGetErrorString(e.code) + " in " + e.what);
  } catch (const ApiError& e) {
    return mlp_fail(n, e.code, e.msg);
  } catch (const std::exception& e) {
    return mlp_fail(n, SPM_EHIP, e.what());
  }
}
}  // namespace

extern "C" {

int spm_mlp_create(spm_mlp** out, void* stream, spm_alloc_fn alloc, spm_free_fn free_fn, void* ctx) {
  if (!out || ((alloc == nullptr) != (free_fn == nullptr))) return SPM_EINVAL;
  spm_mlp* n = new spm_mlp();
  n->stream = static_cast<hipStream_t>(stream);
  n->alloc = alloc;
  n->free_fn = free_fn;
  n->alloc_ctx = ctx;
  const int rc = mlp_guarded(n, [&]() {
    grow(n, n->params, SPM_MLP_NPARAMS);
    grow(n, n->grads, SPM_MLP_NPARAMS);
    grow(n, n->m1, SPM_MLP_NPARAMS);
    grow(n, n->m2, SPM_MLP_NPARAMS);
    grow(n, n->loss, 1);
    grow(n, n->flag, 1);
    launch_fill(n->stream, n->params, SPM_MLP_NPARAMS, 0.f);
    launch_fill(n->stream, n->m1, SPM_MLP_NPARAMS, 0.f);
    launch_fill(n->stream, n->m2, SPM_MLP_NPARAMS, 0.f);
    ensure_batch(n, 256);
    SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
    return SPM_OK;
  });
  if (rc != SPM_OK) {
    spm_mlp_destroy(n);
    return rc;
  }
  *out = n;
  return SPM_OK;
}

void spm_mlp_destroy(spm_mlp* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  float* bufs[] = {n->params, n->grads, n->m1, n->m2, n->h[0], n->h[1], n->h[2], n->y, n->dz[0], n->dz[1]};
  for (float* p : bufs)
    if (p) {
      if (n->free_fn)
        n->free_fn(p, n->stream, n->alloc_ctx);
      else
        (void)hipFree(p);
    }
  void* more[] = {n->part, n->loss, n->flag};
  for (void* p : more)
    if (p) {
      if (n->free_fn)
        n->free_fn(p, n->stream, n->alloc_ctx);
      else
        (void)hipFree(p);
    }
  delete n;
}

const char* spm_mlp_last_error(const spm_mlp* n) { return n ? n->err.c_str() : "null network"; }

int spm_mlp_set_params(spm_mlp* n, const float* params) {
  return mlp_guarded(n, [&]() {
    if (!params) throw ApiError(SPM_EINVAL, "null params");
    k_copyf<<<(SPM_MLP_NPARAMS + 255) / 256, 256, 0, n->stream>>>(SPM_MLP_NPARAMS, n->params, params);
    SPM_HIP_CHECK(hipGetLastError());
    launch_fill(n->stream, n->m1, SPM_MLP_NPARAMS, 0.f);
    launch_fill(n->stream, n->m2, SPM_MLP_NPARAMS, 0.f);
    n->t = 0;
    SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
    return SPM_OK;
  });
}

int spm_mlp_set_weights(spm_mlp* n, const uint16_t* params_bf16, const float* master_fp32, int64_t n_params) {
  return mlp_guarded(n, [&]() {
    if (n_params != SPM_MLP_NPARAMS) throw ApiError(SPM_EINVAL, "n_params must be SPM_MLP_NPARAMS");
    if (!params_bf16 && !master_fp32) throw ApiError(SPM_EINVAL, "no weights given");
    const unsigned grid = (SPM_MLP_NPARAMS + 255) / 256;
    if (master_fp32) {
      if (params_bf16) {
        SPM_HIP_CHECK(hipMemsetAsync(n->flag, 0, sizeof(int32_t), n->stream));
        k_check_bf16<<<grid, 256, 0, n->stream>>>(SPM_MLP_NPARAMS, params_bf16, master_fp32, n->flag);
        SPM_HIP_CHECK(hipGetLastError());
        int32_t bad = 0;
        SPM_HIP_CHECK(hipMemcpyAsync(&bad, n->flag, sizeof(int32_t), hipMemcpyDeviceToHost, n->stream));
        SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
        if (bad) throw ApiError(SPM_EINVAL, "params_bf16 is not the bfloat16 rounding of master_fp32");
      }
      k_copyf<<<grid, 256, 0, n->stream>>>(SPM_MLP_NPARAMS, n->params, master_fp32);
    } else {
      k_widen_bf16<<<grid, 256, 0, n->stream>>>(SPM_MLP_NPARAMS, params_bf16, n->params);
    }
    SPM_HIP_CHECK(hipGetLastError());
    launch_fill(n->stream, n->m1, SPM_MLP_NPARAMS, 0.f);
    launch_fill(n->stream, n->m2, SPM_MLP_NPARAMS, 0.f);
    n->t = 0;
    SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
    return SPM_OK;
  });
}

int spm_mlp_get_params(spm_mlp* n, float* params) {
  return mlp_guarded(n, [&]() {
    if (!params) throw ApiError(SPM_EINVAL, "null params");
    k_copyf<<<(SPM_MLP_NPARAMS + 255) / 256, 256, 0, n->stream>>>(SPM_MLP_NPARAMS, params, n->params);
    SPM_HIP_CHECK(hipGetLastError());
    SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
    return SPM_OK;
  });
}

int spm_mlp_forward(spm_mlp* n, const float* x, int64_t batch, float* y, int32_t mode) {
  return mlp_guarded(n, [&]() {
    if (!x || !y || batch < 1 || batch > (int64_t)1 << 24) throw ApiError(SPM_EINVAL, "bad forward arguments");
    if (mode != SPM_MLP_BF16 && mode != SPM_MLP_FP32) throw ApiError(SPM_EINVAL, "bad mode");
    mlp_forward(n, n->stream, x, nullptr, batch, y, mode);
    SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
    return SPM_OK;
  });
}

int spm_mlp_loss_grad(spm_mlp* n, const float* x, const float* t, int64_t batch, int32_t mode, float* grads,
                      double* loss_host) {
  return mlp_guarded(n, [&]() {
    if (!x || !t || batch < 1 || batch > (int64_t)1 << 24) throw ApiError(SPM_EINVAL, "bad gradient arguments");
    if (mode != SPM_MLP_BF16 && mode != SPM_MLP_FP32) throw ApiError(SPM_EINVAL, "bad mode");
    ensure_batch(n, batch);
    mlp_backward(n, n->stream, x, nullptr, t, nullptr, batch, mode, grads ? grads : n->grads, nullptr, n->loss);
    double l = 0.0;
    SPM_HIP_CHECK(hipMemcpyAsync(&l, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
    if (loss_host) *loss_host = l;
    return SPM_OK;
  });
}

int spm_mlp_backward(spm_mlp* n, const float* x, const float* dy, int64_t batch, float* grad, int32_t mode) {
  return mlp_guarded(n, [&]() {
    if (!x || !dy || !grad || batch < 1 || batch > (int64_t)1 << 24)
      throw ApiError(SPM_EINVAL, "bad backward arguments");
    if (mode != SPM_MLP_BF16 && mode != SPM_MLP_FP32) throw ApiError(SPM_EINVAL, "bad mode");
    mlp_forward(n, n->stream, x, nullptr, batch, n->y, mode);
    mlp_backprop(n, n->stream, x, nullptr, dy, batch, mode, grad);
    SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
    return SPM_OK;
  });
}

int spm_mlp_adam_step(spm_mlp* n, const float* grad, float lr, float beta1, float beta2, float eps, int32_t step) {
  return mlp_guarded(n, [&]() {
    if (!grad || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) ||
        step < 1)
      throw ApiError(SPM_EINVAL, "bad Adam arguments");
    const float bc1 = 1.f - std::pow(beta1, (float)step), bc2 = 1.f - std::pow(beta2, (float)step);
    k_adam<<<(SPM_MLP_NPARAMS + 255) / 256, 256, 0, n->stream>>>(SPM_MLP_NPARAMS, n->params, grad, n->m1, n->m2, lr,
                                                                 beta1, beta2, eps, bc1, bc2);
    SPM_HIP_CHECK(hipGetLastError());
    n->t = step;
    SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
    return SPM_OK;
  });
}

int spm_mlp_train(spm_mlp* n, const float* x, const float* t, int64_t n_samples, const int32_t* idx,
                  int32_t n_batches, int32_t batch, float lr, int32_t mode, float* losses) {
  return mlp_guarded(n, [&]() {
    if (!x || !t || !idx || n_samples < 1 || n_samples > INT32_MAX || n_batches < 1 || batch < 1 ||
        batch > (1 << 24) || !(lr > 0.f))
      throw ApiError(SPM_EINVAL, "bad train arguments");
    if (mode != SPM_MLP_BF16 && mode != SPM_MLP_FP32) throw ApiError(SPM_EINVAL, "bad mode");
    ensure_batch(n, batch);
    {   // every row index must address a sample
      const int64_t cnt = (int64_t)n_batches * batch;
      SPM_HIP_CHECK(hipMemsetAsync(n->flag, 0, sizeof(int32_t), n->stream));
      k_check_rows<<<(unsigned)std::min<int64_t>((cnt + 255) / 256, 65535), 256, 0, n->stream>>>(
          idx, cnt, n_samples, n->flag);
      SPM_HIP_CHECK(hipGetLastError());
      int32_t bad = 0;
      SPM_HIP_CHECK(hipMemcpyAsync(&bad, n->flag, sizeof(int32_t), hipMemcpyDeviceToHost, n->stream));
      SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
      if (bad) throw ApiError(SPM_EINVAL, "row index out of range");
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int32_t k = 0; k < n_batches; ++k) {
      const int32_t* rows = idx + (int64_t)k * batch;
      mlp_backward(n, n->stream, x, rows, t, rows, batch, mode, n->grads, losses ? losses + k : nullptr, nullptr);
      n->t += 1;
      const float bc1 = 1.f - std::pow(b1, (float)n->t), bc2 = 1.f - std::pow(b2, (float)n->t);
      k_adam<<<(SPM_MLP_NPARAMS + 255) / 256, 256, 0, n->stream>>>(SPM_MLP_NPARAMS, n->params, n->grads, n->m1, n->m2,
                                                                   lr, b1, b2, eps, bc1, bc2);
      SPM_HIP_CHECK(hipGetLastError());
    }
    SPM_HIP_CHECK(hipStreamSynchronize(n->stream));
    return SPM_OK;
  });
}

}  // extern "C"
