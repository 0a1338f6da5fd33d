// Fast multipole evaluation of the near-image traction sum (FP64, one cell).
//
// The paper evaluates the near sum from the image sources to the nodes with an FMM (Sec. 6.2,
// remark on the cost; Sec. 8 runs at tolerances 1e-9 to 1e-12). Here it is a complex-variable FMM
// on a uniform quadtree. With z the target, n its unit normal and r = z - z_j (complex), the
// traction kernel of eq. Gt applied to f_j = w_j sigma_j splits into Cauchy sums:
//
//   (r.n)(r.f) r / |r|^4 = n f / (4 r) + (conj(n) f + n conj(f)) / (4 conj(r)) + conj(n) conj(f) r / (4 conj(r)^2),
//   T(z) = -(1/4pi) [ 2 n Re A(z) + conj(n) conj(B(z) + C'(z) - conj(z) A'(z)) ],
//   A = sum_j f_j / (z - z_j),  B = sum_j conj(f_j) / (z - z_j),  C = sum_j f_j conj(z_j) / (z - z_j).
//
// C is carried about the centre c of every box, C_c = sum_j f_j conj(z_j - c) / (z - z_j) = C - conj(c) A,
// so that no expansion holds the large factor conj(z_j): moving an expansion from centre c to c'
// adds conj(c - c') times the moved A expansion, and at the target C' - conj(z) A' = C_c' - conj(z - c) A'.
//
// Expansions are scaled by the box side h: multipole a_k = sum_j q_j ((z_j - c)/h)^k, so that
// sum_j q_j / (z - z_j) = (1/h) sum_k a_k (h / (z - c))^(k+1); local L_l with
// sum_j q_j / (z - z_j) = sum_l L_l ((z - c)/h)^l. Translations (binomial sums) use factorial
// tables:
//   M2M (child c' to parent c, t = (c' - c)/h_P): a_k = k! sum_{m<=k} (a'_m 2^-m / m!) (t^(k-m) / (k-m)!)
//   M2L (source c_s to target c_t, rho = h / (c_t - c_s)):
//       L_l = (-1)^l rho^(l+1) / (h l!) sum_k (k + l)! (a_k rho^k / k!)
//   L2L (parent c to child c', t = (c' - c)/h_P): L'_m = (2^-m / m!) sum_{l>=m} (L_l l!) (t^(l-m) / (l-m)!)
// Interaction lists are the usual ones (children of the parent's neighbours that are not
// neighbours); leaves evaluate their 3x3 neighbourhood directly, where the pair at zero
// distance (the target's own node) adds nothing. Every pass is deterministic: one wavefront per box (three per
// leaf in the evaluation), lanes over expansion terms (in the multipole pass over runs of terms and source
// phases), fixed loop orders.
#include "spm_internal.h"

namespace spm {
namespace {

struct cx {
  double r, i;
};
__device__ __forceinline__ cx operator+(cx a, cx b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cx operator-(cx a, cx b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cx operator*(cx a, cx b) { return {fma(a.r, b.r, -a.i * b.i), fma(a.r, b.i, a.i * b.r)}; }
__device__ __forceinline__ cx operator*(cx a, double s) { return {a.r * s, a.i * s}; }
__device__ __forceinline__ cx conj(cx a) { return {a.r, -a.i}; }
// acc + a b and acc + a s with fused multiply-adds (the library builds without contraction)
__device__ __forceinline__ cx cmac(cx acc, cx a, cx b) {
  return {fma(a.r, b.r, fma(-a.i, b.i, acc.r)), fma(a.r, b.i, fma(a.i, b.r, acc.i))};
}
__device__ __forceinline__ cx cmac(cx acc, cx a, double s) { return {fma(a.r, s, acc.r), fma(a.i, s, acc.i)}; }
__device__ __forceinline__ cx cdiv(cx a, cx b) {
  const double d = b.r * b.r + b.i * b.i;
  return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}
__device__ __forceinline__ cx cpow(cx w, int k) {   // binary powering, k >= 0
  cx r = {1.0, 0.0};
  while (k) {
    if (k & 1) r = r * w;
    w = w * w;
    k >>= 1;
  }
  return r;
}

__host__ __device__ __forceinline__ int64_t box_off(int l) { return (((int64_t)1 << (2 * l)) - 1) / 3; }

struct FmmArgs {
  int p, L;
  double D0, c0x, c0y;
  const double *sx, *sy, *fs1, *fs2;
  const int32_t *leaf_s, *bsrc;
  const double* fact;
  const cx* m2l_tab;               // [49][2][p] M2L scalings per displacement
  const cx* m2m_tp;                // [4][p] (child offset / parent side)^k / k!
  const int32_t* m2m_asg;          // [16][5] M2M terms per lane of a child (-1: none)
  cx *Mx, *Lx;                     // [box][3][p]
};

__device__ __forceinline__ cx box_center(const FmmArgs& a, int l, int64_t loc) {
  const int n = 1 << l;
  const double h = a.D0 / n;
  const int ix = (int)(loc & (n - 1)), iy = (int)(loc >> l);
  return {a.c0x - 0.5 * a.D0 + (ix + 0.5) * h, a.c0y - 0.5 * a.D0 + (iy + 0.5) * h};
}

__global__ __launch_bounds__(256) void k_fmm_gather(int64_t ns, const int32_t* __restrict__ sj,
                                                    const double* __restrict__ f1, const double* __restrict__ f2,
                                                    double* __restrict__ fs1, double* __restrict__ fs2) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= ns) return;
  const int32_t j = sj[k];
  fs1[k] = f1[j];
  fs2[k] = f2[j];
}

// multipoles of the leaves with sources. The p terms are cut into eight runs of CS = ceil(p / 8)
// consecutive powers; the eight lanes of a run take every eighth source of the leaf, so that all
// 64 lanes work, each on CS terms of its sources. Sources go 64 at a time: lane t stages source
// t's w = (z_j - c)/h, q_j, q_j conj(z_j - c) and the run starts w^(CS r), r < 8, in LDS; a lane of
// run r starts from w^(CS r) and steps by w. The eight partial sums of a term are then added in
// lane order through LDS.
constexpr int kP2mRuns = 8, kP2mPhases = 8;   // runs of terms x source phases = 64 lanes
template <int CS>
__global__ __launch_bounds__(64) void k_fmm_p2m(FmmArgs a, const int32_t* __restrict__ list) {
  constexpr int kStage = 64 * (3 + kP2mRuns), kRed = 64 * 3 * CS;
  __shared__ cx sh[kStage > kRed ? kStage : kRed];
  cx* const sw = sh;              // w of source t
  cx* const sq = sh + 64;         // q
  cx* const sqd = sh + 128;       // q conj(d)
  cx* const sp = sh + 192;        // w^(CS r) at [t kP2mRuns + r]
  const int64_t gid = list[blockIdx.x];
  const int64_t loc = gid - box_off(a.L);
  const cx c = box_center(a, a.L, loc);
  const double ih = (double)(1 << a.L) / a.D0;
  const int lane = threadIdx.x, run = lane / kP2mPhases, ph = lane % kP2mPhases;
  cx A[CS], B[CS], C[CS];
#pragma unroll
  for (int i = 0; i < CS; ++i) A[i] = B[i] = C[i] = {0.0, 0.0};
  const int32_t s0 = a.leaf_s[loc], s1 = a.leaf_s[loc + 1];
  for (int32_t j0 = s0; j0 < s1; j0 += 64) {
    const int ng = min(64, (int)(s1 - j0));
    if (lane < ng) {
      const int32_t j = j0 + lane;
      const cx d = {a.sx[j] - c.r, a.sy[j] - c.i};
      const cx w = d * ih, q = {a.fs1[j], a.fs2[j]};
      sw[lane] = w;
      sq[lane] = q;
      sqd[lane] = q * conj(d);
      cx wc = w;
#pragma unroll
      for (int e = 1; e < CS; ++e) wc = wc * w;
      cx pw = {1.0, 0.0};
#pragma unroll
      for (int r = 0; r < kP2mRuns; ++r) {
        sp[lane * kP2mRuns + r] = pw;
        pw = pw * wc;
      }
    }
    __syncthreads();
    for (int t = ph; t < ng; t += kP2mPhases) {
      const cx w = sw[t], q = sq[t], qd = sqd[t];
      cx pw = sp[t * kP2mRuns + run];
#pragma unroll
      for (int i = 0; i < CS; ++i) {
        A[i] = cmac(A[i], q, pw);
        B[i] = cmac(B[i], conj(q), pw);
        C[i] = cmac(C[i], qd, pw);
        if (i + 1 < CS) pw = pw * w;
      }
    }
    __syncthreads();   // the stage is rewritten next (or reused below)
  }
  cx* const red = sh;             // lane's partials at [lane 3 CS + series CS + i]
#pragma unroll
  for (int i = 0; i < CS; ++i) {
    red[lane * 3 * CS + i] = A[i];
    red[lane * 3 * CS + CS + i] = B[i];
    red[lane * 3 * CS + 2 * CS + i] = C[i];
  }
  __syncthreads();
  for (int o = lane; o < 3 * a.p; o += 64) {
    const int sr = o / a.p, k = o - sr * a.p;
    const int r = k / CS, i = k - r * CS;
    cx acc = {0.0, 0.0};
    for (int f = 0; f < kP2mPhases; ++f) acc = acc + red[(r * kP2mPhases + f) * 3 * CS + sr * CS + i];
    a.Mx[gid * 3 * a.p + o] = acc;
  }
}

void launch_p2m(const FmmArgs& a, unsigned nb, const int32_t* list, hipStream_t st) {
  switch ((a.p + kP2mRuns - 1) / kP2mRuns) {
    case 1: k_fmm_p2m<1><<<nb, 64, 0, st>>>(a, list); break;
    case 2: k_fmm_p2m<2><<<nb, 64, 0, st>>>(a, list); break;
    case 3: k_fmm_p2m<3><<<nb, 64, 0, st>>>(a, list); break;
    case 4: k_fmm_p2m<4><<<nb, 64, 0, st>>>(a, list); break;
    case 5: k_fmm_p2m<5><<<nb, 64, 0, st>>>(a, list); break;
    case 6: k_fmm_p2m<6><<<nb, 64, 0, st>>>(a, list); break;
    case 7: k_fmm_p2m<7><<<nb, 64, 0, st>>>(a, list); break;
    case 8: k_fmm_p2m<8><<<nb, 64, 0, st>>>(a, list); break;
    default: throw ApiError(SPM_EINVAL, "FMM order must be between 1 and 64");
  }
}

constexpr int kM2lMaxP = 64;   // largest expansion order (LDS and table sizes)
constexpr int kM2mLanes = 16, kM2mSlots = 5;   // lanes per child, terms per lane (16 x 5 >= 64)

// multipoles of level l from their children at level l + 1; the four children are staged in LDS
// in one phase (their loads overlap). Term k of a child is a sum of k + 1 products, so each child
// takes sixteen lanes and its terms go to them by a table built once per plan (largest sums first,
// each to the least loaded lane), which evens out the triangular sums; the children's terms are
// then added in child order through LDS. A child's centre is (+-1 +-i) / 4 parent sides from the
// parent's at every level, so the powers of that offset come from a table too.
__global__ __launch_bounds__(64) void k_fmm_m2m(FmmArgs a, int l, const int32_t* __restrict__ list) {
  __shared__ cx ac[4][3][kM2lMaxP];     // child multipoles times 2^-m / m!, then the child sums
  __shared__ cx tp[4][kM2lMaxP];        // (child offset / parent side)^k / k!
  const int64_t gid = list[blockIdx.x];
  const int64_t loc = gid - box_off(l);
  const int n = 1 << l;
  const int ix = (int)(loc & (n - 1)), iy = (int)(loc >> l);
  const cx c = box_center(a, l, loc);
  const int k = threadIdx.x, p = a.p;
  bool has[4];
  cx dch[4];
  for (int ch = 0; ch < 4; ++ch) {
    const int64_t cloc = (int64_t)(2 * iy + (ch >> 1)) * (2 * n) + (2 * ix + (ch & 1));
    const int64_t cgid = box_off(l + 1) + cloc;
    has[ch] = a.bsrc[cgid] != 0;
    dch[ch] = box_center(a, l + 1, cloc) - c;
    if (has[ch] && k < p) {
      const cx* m = a.Mx + cgid * 3 * p;
      const double sc = ldexp(1.0, -k) / a.fact[k];
      ac[ch][0][k] = m[k] * sc;
      ac[ch][1][k] = m[p + k] * sc;
      ac[ch][2][k] = m[2 * p + k] * sc;
      tp[ch][k] = a.m2m_tp[ch * p + k];
    }
  }
  __syncthreads();
  const int ch = k >> 4, j = k & 15;
  int kks[kM2mSlots];
#pragma unroll
  for (int sl = 0; sl < kM2mSlots; ++sl) kks[sl] = a.m2m_asg[j * kM2mSlots + sl];
  cx sum[kM2mSlots][3];
  if (has[ch]) {
#pragma unroll
    for (int row = 0; row < kM2mSlots; ++row) {
      const int kk = kks[row];
      if (kk < 0) continue;
      cx sA = {0, 0}, sB = {0, 0}, sC = {0, 0};
      for (int m = 0; m <= kk; ++m) {
        const cx t = tp[ch][kk - m];
        sA = cmac(sA, ac[ch][0][m], t);
        sB = cmac(sB, ac[ch][1][m], t);
        sC = cmac(sC, ac[ch][2][m], t);
      }
      const double fk = a.fact[kk];
      sum[row][0] = sA * fk;
      sum[row][1] = sB * fk;
      sum[row][2] = sC * fk;
    }
  }
  __syncthreads();   // every lane is done reading the staged multipoles
  if (has[ch]) {
#pragma unroll
    for (int row = 0; row < kM2mSlots; ++row) {
      const int kk = kks[row];
      if (kk < 0) continue;
      ac[ch][0][kk] = sum[row][0];
      ac[ch][1][kk] = sum[row][1];
      ac[ch][2][kk] = sum[row][2];
    }
  }
  __syncthreads();
  if (k < p) {
    cx oA = {0, 0}, oB = {0, 0}, oC = {0, 0};
    for (int c4 = 0; c4 < 4; ++c4) {
      if (!has[c4]) continue;
      const cx sA = ac[c4][0][k];
      oA = oA + sA;
      oB = oB + ac[c4][1][k];
      oC = oC + ac[c4][2][k] + conj(dch[c4]) * sA;
    }
    cx* out = a.Mx + gid * 3 * p;
    out[k] = oA;
    out[p + k] = oB;
    out[2 * p + k] = oC;
  }
}

// local expansions from the interaction lists, every level in one launch (written, not added).
// The list (at most 27 source boxes with sources) is formed first; the next box's multipole is
// loaded into registers while the current one is summed.
// M2L: one wavefront per target box. The source boxes go nb = 64 / ceil(p / 2) at a time (three at
// 40 terms): their three multipoles, scaled by rho^k / k!, are staged in LDS, and lane (b, j) takes
// the Hankel sums over k with (k + l)! of box b for the two output terms l = j and j + ceil(p / 2)
// (each staged value feeds both), scaled by (-1)^l rho^(l+1) / (h l!). rho = h / (c_t - c_s)
// depends only on the integer displacement of the two boxes in box units (one of 7 x 7), so both
// scalings come from per-displacement tables built once per plan; the next round's multipoles and
// table entries are loaded while the current sums run, and the lanes' partial expansions are added
// over the boxes of a round in a fixed order at the end.

// M2M tables: tp[ch p + k] = t^k / k! for the child offset t = (+-1 +-i) / 4 (x by ch & 1, y by
// ch >> 1); asg[j kM2mSlots + s] = the terms of lane j, the largest sums first, each to the least
// loaded lane with a free slot (ties to the lowest lane), -1 after the last.
__global__ __launch_bounds__(64) void k_fmm_m2m_tables(int p, const double* __restrict__ fact, cx* __restrict__ tp,
                                                       int32_t* __restrict__ asg) {
  const int k = threadIdx.x;
  if (k < p)
    for (int ch = 0; ch < 4; ++ch) {
      const cx t = {(ch & 1) ? 0.25 : -0.25, (ch >> 1) ? 0.25 : -0.25};
      tp[ch * p + k] = cpow(t, k) * (1.0 / fact[k]);
    }
  if (k == 0) {
    int load[kM2mLanes], cnt[kM2mLanes];
    for (int l = 0; l < kM2mLanes; ++l) {
      load[l] = 0;
      cnt[l] = 0;
      for (int sl = 0; sl < kM2mSlots; ++sl) asg[l * kM2mSlots + sl] = -1;
    }
    for (int kk = p - 1; kk >= 0; --kk) {
      int best = -1;
      for (int l = 0; l < kM2mLanes; ++l)
        if (cnt[l] < kM2mSlots && (best < 0 || load[l] < load[best])) best = l;
      asg[best * kM2mSlots + cnt[best]] = kk;
      ++cnt[best];
      load[best] += kk + 1;
    }
  }
}

// tab[(2 d) p + k] = rho^k / k!, tab[(2 d + 1) p + k] = (-1)^k rho^(k+1) / k!, rho = 1 / D for the
// displacement D = (c_t - c_s) / h = (d % 7 - 3) + i (d / 7 - 3); zero for the 3 x 3 neighbours.
__global__ __launch_bounds__(64) void k_fmm_m2l_tables(int p, const double* __restrict__ fact, cx* __restrict__ tab) {
  const int d = blockIdx.x, k = threadIdx.x;
  if (k >= p) return;
  const int ex = d % 7 - 3, ey = d / 7 - 3;
  cx sk = {0.0, 0.0}, gk = {0.0, 0.0};
  if (abs(ex) > 1 || abs(ey) > 1) {
    const cx rho = cdiv({1.0, 0.0}, {(double)ex, (double)ey});
    const cx rk = cpow(rho, k);
    sk = rk * (1.0 / fact[k]);
    gk = rk * rho * (((k & 1) ? -1.0 : 1.0) / fact[k]);
  }
  tab[(2 * d) * p + k] = sk;
  tab[(2 * d + 1) * p + k] = gk;
}

__global__ __launch_bounds__(64) void k_fmm_m2l(FmmArgs a, const int32_t* __restrict__ list) {
  __shared__ cx bs[3][2 * kM2lMaxP];   // scaled multipoles of the boxes of a round, [series][box p + k]
  __shared__ cx red[3][64][2];         // per lane: its two terms' sums, then the reduction over boxes
  __shared__ double fs[2 * kM2lMaxP];
  __shared__ int64_t srcs[27];
  __shared__ int dsp[27];
  __shared__ int nsrc;
  const int64_t gid = list[blockIdx.x];
  int l = 2;
  while (l < a.L && gid >= box_off(l + 1)) ++l;
  const int64_t loc = gid - box_off(l);
  const int n = 1 << l;
  const int ix = (int)(loc & (n - 1)), iy = (int)(loc >> l);
  const cx c = box_center(a, l, loc);
  const double ih = n / a.D0;
  const int t = threadIdx.x, p = a.p;
  for (int i = t; i < 2 * p; i += 64) fs[i] = a.fact[i];
  if (t == 0) {
    const int px = ix >> 1, py = iy >> 1, np = n >> 1;
    int cnt = 0;
    for (int qy = max(py - 1, 0); qy <= min(py + 1, np - 1); ++qy)
      for (int qx = max(px - 1, 0); qx <= min(px + 1, np - 1); ++qx)
        for (int ch = 0; ch < 4; ++ch) {
          const int bx = 2 * qx + (ch & 1), by = 2 * qy + (ch >> 1);
          if (abs(bx - ix) <= 1 && abs(by - iy) <= 1) continue;
          const int64_t sloc = (int64_t)by * n + bx;
          if (a.bsrc[box_off(l) + sloc] != 0) {
            srcs[cnt] = sloc;
            dsp[cnt] = (iy - by + 3) * 7 + (ix - bx + 3);
            ++cnt;
          }
        }
    nsrc = cnt;
  }
  __syncthreads();
  const int ns = nsrc;
  const cx* Mb = a.Mx + box_off(l) * 3 * p;
  // lane (b, j): box b of the round, output terms j and j + hp
  const int hp = (p + 1) / 2, nb = 64 / hp;
  const int b = t / hp, j = t % hp;
  const int l1 = j, l2 = j + hp;
  const bool act = b < nb, has2 = act && l2 < p;
  // staging slots of a round: slot q < nb p is term q % p of box q / p; lane t fills slots t and t + 64
  cx pre[2][4];
  auto fetch = [&](int i0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = t + 64 * u, bq = q / p, mq = q - bq * p;
      if (q < nb * p && i0 + bq < ns) {
        const cx* m = Mb + srcs[i0 + bq] * 3 * p;
        pre[u][0] = m[mq];
        pre[u][1] = m[p + mq];
        pre[u][2] = m[2 * p + mq];
        pre[u][3] = a.m2l_tab[(2 * dsp[i0 + bq]) * p + mq];
      }
    }
  };
  fetch(0);
  cx oA1 = {0, 0}, oB1 = {0, 0}, oC1 = {0, 0}, oA2 = {0, 0}, oB2 = {0, 0}, oC2 = {0, 0};
  for (int i0 = 0; i0 < ns; i0 += nb) {
    __syncthreads();                       // the previous round's sums are done with bs
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = t + 64 * u, bq = q / p;
      if (q < nb * p && i0 + bq < ns) {
        bs[0][q] = pre[u][0] * pre[u][3];
        bs[1][q] = pre[u][1] * pre[u][3];
        bs[2][q] = pre[u][2] * pre[u][3];
      }
    }
    __syncthreads();
    if (i0 + nb < ns) fetch(i0 + nb);      // the next round's multipoles and scalings
    const int i = i0 + b;
    if (act && i < ns) {
      const cx* g2tab = a.m2l_tab + (2 * dsp[i] + 1) * p;
      const cx g1 = g2tab[l1] * ih, g2 = has2 ? g2tab[l2] * ih : cx{0, 0};
      const cx dc = conj(box_center(a, l, srcs[i]) - c);
      const cx* x0 = bs[0] + b * p;
      const cx* x1 = bs[1] + b * p;
      const cx* x2 = bs[2] + b * p;
      cx sA1 = {0, 0}, sB1 = {0, 0}, sC1 = {0, 0}, sA2 = {0, 0}, sB2 = {0, 0}, sC2 = {0, 0};
      const int e2 = has2 ? l2 : l1;     // a lane without a second term repeats its first
      for (int m = 0; m < p; ++m) {
        const double f1 = fs[m + l1], f2 = fs[m + e2];
        const cx A = x0[m], B = x1[m], C = x2[m];
        sA1 = cmac(sA1, A, f1);
        sB1 = cmac(sB1, B, f1);
        sC1 = cmac(sC1, C, f1);
        sA2 = cmac(sA2, A, f2);
        sB2 = cmac(sB2, B, f2);
        sC2 = cmac(sC2, C, f2);
      }
      sA1 = sA1 * g1;
      oA1 = oA1 + sA1;
      oB1 = oB1 + sB1 * g1;
      oC1 = oC1 + sC1 * g1 + dc * sA1;
      sA2 = sA2 * g2;
      oA2 = oA2 + sA2;
      oB2 = oB2 + sB2 * g2;
      oC2 = oC2 + sC2 * g2 + dc * sA2;
    }
  }
  __syncthreads();
  red[0][t][0] = oA1;
  red[1][t][0] = oB1;
  red[2][t][0] = oC1;
  red[0][t][1] = oA2;
  red[1][t][1] = oB2;
  red[2][t][1] = oC2;
  __syncthreads();
  if (t < p) {                             // term t: the lanes (b, t % hp) in box order
    const int jj = t < hp ? t : t - hp, w = t < hp ? 0 : 1;
    cx oA = {0, 0}, oB = {0, 0}, oC = {0, 0};
    for (int bb = 0; bb < nb; ++bb) {
      oA = oA + red[0][bb * hp + jj][w];
      oB = oB + red[1][bb * hp + jj][w];
      oC = oC + red[2][bb * hp + jj][w];
    }
    cx* out = a.Lx + gid * 3 * p;
    out[t] = oA;
    out[p + t] = oB;
    out[2 * p + t] = oC;
  }
}

// adds the parent's local expansion (level l - 1) to the boxes of level l
__global__ __launch_bounds__(64) void k_fmm_l2l(FmmArgs a, int l, const int32_t* __restrict__ list) {
  __shared__ cx al[3][64];
  __shared__ cx tp[64];
  const int64_t gid = list[blockIdx.x];
  const int64_t loc = gid - box_off(l);
  const int n = 1 << l;
  const int ix = (int)(loc & (n - 1)), iy = (int)(loc >> l);
  const cx c = box_center(a, l, loc);
  const int64_t ploc = (int64_t)(iy >> 1) * (n >> 1) + (ix >> 1);
  const int64_t pgid = box_off(l - 1) + ploc;
  const cx cp = box_center(a, l - 1, ploc);
  const double ihP = (double)(n >> 1) / a.D0;
  const int k = threadIdx.x, p = a.p;
  const cx d = c - cp;
  if (k < p) {
    const cx* m = a.Lx + pgid * 3 * p;
    const double f = a.fact[k];
    al[0][k] = m[k] * f;
    al[1][k] = m[p + k] * f;
    al[2][k] = m[2 * p + k] * f;
    tp[k] = cpow(d * ihP, k) * (1.0 / f);
  }
  __syncthreads();
  if (k < p) {
    cx sA = {0, 0}, sB = {0, 0}, sC = {0, 0};
    for (int j = k; j < p; ++j) {
      const cx t = tp[j - k];
      sA = cmac(sA, al[0][j], t);
      sB = cmac(sB, al[1][j], t);
      sC = cmac(sC, al[2][j], t);
    }
    const double s = ldexp(1.0, -k) / a.fact[k];
    sA = sA * s;
    cx* out = a.Lx + gid * 3 * p;
    out[k] = out[k] + sA;
    out[p + k] = out[p + k] + sB * s;
    out[2 * p + k] = out[2 * p + k] + sC * s + conj(cp - c) * sA;
  }
}

// three wavefronts per target leaf: the sources of the 3x3 neighbour leaves (three contiguous rows
// of the sorted order, taken as one list) are staged through LDS 192 at a time. The leaf's targets
// go 64 at a time and a batch of n_t takes the whole block: each target floor(192 / n_t) threads,
// which split every staged chunk of sources between them (about 95% of the threads work over the
// leaves of a dense cell, against 76% with a third of every chunk per wave and floor(64 / n_t)
// lanes per target). The threads' partial sums of a target are added in a fixed order, then wave 0
// adds the local expansion.
constexpr int kEvalWaves = 3;
__global__ __launch_bounds__(64 * kEvalWaves) void k_fmm_eval(FmmArgs a, int64_t N, const int32_t* __restrict__ list,
                                                              const int32_t* __restrict__ leaf_t,
                                                              const int32_t* __restrict__ tperm, Geo g,
                                                              double* __restrict__ out) {
  constexpr int B = 64 * kEvalWaves;
  __shared__ double shx[B], shy[B], sf1[B], sf2[B];
  __shared__ double red1[64 * kEvalWaves], red2[64 * kEvalWaves];
  const int64_t gid = list[blockIdx.x];
  const int64_t loc = gid - box_off(a.L);
  const int n = 1 << a.L;
  const int ix = (int)(loc & (n - 1)), iy = (int)(loc >> a.L);
  const cx c = box_center(a, a.L, loc);
  const double h = a.D0 / n;
  const cx* Le = a.Lx + gid * 3 * a.p;
  const int p = a.p;
  // the neighbour rows as one list of up to three ranges
  int32_t rb[3], rl[3];
  int nr = 0;
  int32_t total = 0;
  for (int jy = max(iy - 1, 0); jy <= min(iy + 1, n - 1); ++jy) {
    rb[nr] = a.leaf_s[(int64_t)jy * n + max(ix - 1, 0)];
    rl[nr] = a.leaf_s[(int64_t)jy * n + min(ix + 1, n - 1) + 1] - rb[nr];
    total += rl[nr];
    ++nr;
  }
  const int32_t t0 = leaf_t[loc], t1 = leaf_t[loc + 1];
  for (int32_t tb = t0; tb < t1; tb += 64) {
    const int nt = min(64, (int)(t1 - tb));
    const int S = B / nt;                  // threads per target
    const int tl = threadIdx.x % nt, r = threadIdx.x / nt;
    const bool act = r < S;
    const int64_t i = tperm[tb + tl];
    const double x = g.x[i], y = g.y[i], nx = g.nx[i], ny = g.ny[i];
    double d1 = 0.0, d2 = 0.0;
    for (int32_t cb = 0; cb < total; cb += B) {
      __syncthreads();
      const int32_t q = cb + (int32_t)threadIdx.x;
      if (q < total) {
        int32_t j = q, k = 0;
        while (j >= rl[k]) {
          j -= rl[k];
          ++k;
        }
        j += rb[k];
        shx[threadIdx.x] = a.sx[j];
        shy[threadIdx.x] = a.sy[j];
        sf1[threadIdx.x] = a.fs1[j];
        sf2[threadIdx.x] = a.fs2[j];
      }
      __syncthreads();
      const int m = min(B, (int)(total - cb));
      if (act) {
        for (int qq = r; qq < m; qq += S) {
          const double rx = x - shx[qq], ry = y - shy[qq];
          // the target's own node (r = 0): the added 1e-300 keeps 1/|r|^2 finite (and below the
          // rounding of every other pair's |r|^2) while (r.n)(r.f) = 0
          const double ir2 = rcp64(fma(rx, rx, fma(ry, ry, 1e-300)));
          const double cf = ((fma(rx, nx, ry * ny) * fma(rx, sf1[qq], ry * sf2[qq])) * ir2) * ir2;
          d1 = fma(cf, rx, d1);
          d2 = fma(cf, ry, d2);
        }
      }
    }
    __syncthreads();
    red1[threadIdx.x] = act ? d1 : 0.0;
    red2[threadIdx.x] = act ? d2 : 0.0;
    __syncthreads();
    if (threadIdx.x < nt) {
      double e1 = 0.0, e2 = 0.0;
      for (int sl = 0; sl < S; ++sl) {
        e1 += red1[sl * nt + threadIdx.x];
        e2 += red2[sl * nt + threadIdx.x];
      }
      const cx dz = {x - c.r, y - c.i};
      const cx u = dz * (1.0 / h);
      cx A = {0, 0}, Bv = {0, 0}, Ad = {0, 0}, Cd = {0, 0};
      for (int k = p - 1; k >= 1; --k) {
        A = cmac(Le[k], A, u);
        Bv = cmac(Le[p + k], Bv, u);
        Ad = cmac(Le[k] * (double)k, Ad, u);
        Cd = cmac(Le[2 * p + k] * (double)k, Cd, u);
      }
      A = cmac(Le[0], A, u);
      Bv = cmac(Le[p], Bv, u);
      const cx E = (Cd - conj(dz) * Ad) * (1.0 / h);
      const cx BE = Bv + E;
      const double k4 = -1.0 / (4.0 * kPi);
      out[i] = k4 * (2.0 * nx * A.r + (nx * BE.r - ny * BE.i)) - e1 / kPi;
      out[N + i] = k4 * (2.0 * ny * A.r - (nx * BE.i + ny * BE.r)) - e2 / kPi;
    }
  }
}

// Per-lane partial sums of the near-image velocity, vorticity and pressure (G^p of eq. Gp:
// (r.f) / (2 pi |r|^2) = Re(f / r) / (2 pi), so the boxes contribute Re A / (2 pi)) at the point z
// (inside the root box); the caller sums the lanes.
struct Pt4 {
  double u1, u2, vo, pr;
};
__device__ Pt4 fmm_point(const FmmArgs& a, double zx, double zy, double mu) {
  const int k = threadIdx.x & 63, p = a.p;
  const int nL = 1 << a.L;
  const int ixL = min(max((int)floor((zx - (a.c0x - 0.5 * a.D0)) / a.D0 * nL), 0), nL - 1);
  const int iyL = min(max((int)floor((zy - (a.c0y - 0.5 * a.D0)) / a.D0 * nL), 0), nL - 1);
  cx sA = {0, 0}, sE = {0, 0}, sLog = {0, 0}, sF = {0, 0};
  for (int l = 2; l <= a.L; ++l) {
    const int n = 1 << l, np = n >> 1;
    const int ix = ixL >> (a.L - l), iy = iyL >> (a.L - l);
    const double h = a.D0 / n;
    for (int qy = max((iy >> 1) - 1, 0); qy <= min((iy >> 1) + 1, np - 1); ++qy) {
      for (int qx = max((ix >> 1) - 1, 0); qx <= min((ix >> 1) + 1, np - 1); ++qx) {
        for (int ch = 0; ch < 4; ++ch) {
          const int bx = 2 * qx + (ch & 1), by = 2 * qy + (ch >> 1);
          if (abs(bx - ix) <= 1 && abs(by - iy) <= 1) continue;
          const int64_t sloc = (int64_t)by * n + bx;
          const int64_t sgid = box_off(l) + sloc;
          if (a.bsrc[sgid] == 0) continue;
          if (k >= p) continue;
          const cx cs = box_center(a, l, sloc);
          const cx d = {zx - cs.r, zy - cs.i};
          const cx iw = cdiv({h, 0.0}, d);           // h / (z - c_s)
          const cx pk = cpow(iw, k);                  // iw^k
          const cx pk1 = pk * iw;                     // iw^(k+1)
          const cx* m = a.Mx + sgid * 3 * p;
          const cx am = m[k], bm = m[p + k], cm = m[2 * p + k];
          const cx tA = am * pk1 * (1.0 / h);
          sA = sA + tA;
          sE = sE + conj(d) * tA - cm * pk1 * (1.0 / h);
          if (k == 0) {
            const cx lg = {0.5 * log(d.r * d.r + d.i * d.i), atan2(d.i, d.r)};
            sLog = sLog + (am * lg + conj(bm * lg)) * 0.5;
            sF = sF + am;
          } else {
            sLog = sLog - (am * pk + conj(bm * pk)) * (0.5 / k);
          }
        }
      }
    }
  }
  const double k4 = 1.0 / (4.0 * kPi * mu), k2 = -1.0 / (2.0 * kPi * mu);
  Pt4 o;
  o.u1 = k4 * (-sLog.r + 0.5 * sF.r + 0.5 * sE.r);
  o.u2 = k4 * (-sLog.i + 0.5 * sF.i - 0.5 * sE.i);
  o.vo = k2 * sA.i;
  o.pr = sA.r * (0.5 / kPi);
  for (int jy = max(iyL - 1, 0); jy <= min(iyL + 1, nL - 1); ++jy) {
    const int32_t r0 = a.leaf_s[(int64_t)jy * nL + max(ixL - 1, 0)];
    const int32_t r1 = a.leaf_s[(int64_t)jy * nL + min(ixL + 1, nL - 1) + 1];
    for (int32_t j = r0 + k; j < r1; j += 64) {
      const double rx = zx - a.sx[j], ry = zy - a.sy[j], fa = a.fs1[j], fb = a.fs2[j];
      const double r2 = rx * rx + ry * ry;
      const double ir2 = rcp64(r2);
      const double lg = -0.5 * log(r2);
      const double rf = (rx * fa + ry * fb) * ir2;
      o.u1 += k4 * (lg * fa + rx * rf);
      o.u2 += k4 * (lg * fb + ry * rf);
      o.vo += k2 * (rx * fb - ry * fa) * ir2;
      o.pr += rf * (0.5 / kPi);
    }
  }
  return o;
}

__global__ __launch_bounds__(64) void k_fmm_velocities(FmmArgs a, Geo g, double mu, double* __restrict__ near3) {
  const int q = blockIdx.x;
  Pt4 o = fmm_point(a, g.pcx[q], g.pcy[q], mu);
  o.u1 = wave_sum(o.u1);
  o.u2 = wave_sum(o.u2);
  o.vo = wave_sum(o.vo);
  if (threadIdx.x == 0) {
    near3[3 * q] = o.u1;
    near3[3 * q + 1] = o.u2;
    near3[3 * q + 2] = o.vo;
  }
}

// Near-image velocity and pressure at field points (one wavefront each), at the point's periodic
// copy in U computed exactly as the field kernel computes it: u [2 nt] and p [nt] receive them
// and the field kernel adds the rest.
__global__ __launch_bounds__(64) void k_fmm_points(FmmArgs a, Geo g, double mu, double cUx, double cUy, int64_t nt,
                                                   const double* __restrict__ xt, const double* __restrict__ yt,
                                                   double* __restrict__ u, double* __restrict__ p) {
  const int64_t t = blockIdx.x;
  const double skew = g.cskew[0];
  const double x = xt[t], y = yt[t];
  const double be = y - cUy, al = (x - cUx) - skew * be;
  const double ka = floor(al + 0.5), kb = floor(be + 0.5);
  const double xw = x - ka - kb * skew, yw = y - kb;
  Pt4 o = fmm_point(a, xw, yw, mu);
  o.u1 = wave_sum(o.u1);
  o.u2 = wave_sum(o.u2);
  o.pr = wave_sum(o.pr);
  if (threadIdx.x == 0) {
    u[t] = o.u1;
    u[nt + t] = o.u2;
    p[t] = o.pr;
  }
}

FmmArgs args(spm_handle* h) {
  const FmmPlan& F = h->fmm;
  FmmArgs a;
  a.p = F.p;
  a.L = F.L;
  a.D0 = F.D0;
  a.c0x = F.c0x;
  a.c0y = F.c0y;
  a.sx = F.sx;
  a.sy = F.sy;
  a.fs1 = F.fs1;
  a.fs2 = F.fs2;
  a.leaf_s = F.leaf_s;
  a.bsrc = F.bsrc;
  a.fact = F.fact;
  a.m2l_tab = reinterpret_cast<const cx*>(F.m2l_tab);
  a.m2m_tp = a.m2l_tab + (size_t)49 * 2 * F.p;
  a.m2m_asg = reinterpret_cast<const int32_t*>(a.m2m_tp + (size_t)4 * F.p);
  a.Mx = reinterpret_cast<cx*>(F.Mx);
  a.Lx = reinterpret_cast<cx*>(F.Lx);
  return a;
}

// HIP events around one kernel (kind 2: evaluation, 3: M2L) when timing is on
void prof_mark(spm_handle* h, int kind, bool start, double work) {
  if (!h->prof) return;
  if (start) {
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
  } else {
    SPM_HIP_CHECK(hipEventRecord(h->ev_pool[2 * h->ev_used + 1], h->stream));
    ++h->ev_used;
    h->prof_launches[kind] += 1;
    h->prof_pairs[kind] += work;
  }
}

// gather w sigma into the sorted order, multipoles of the leaves, then of every coarser level
// down to 2; returns the index of the next list segment (M2L)
int launch_fmm_upward(spm_handle* h) {
  const FmmPlan& F = h->fmm;
  const FmmArgs a = args(h);
  auto n_of = [&](int s) { return (unsigned)(F.seg[s + 1] - F.seg[s]); };
  auto list = [&](int s) { return F.lists + F.seg[s]; };
  k_fmm_gather<<<(unsigned)((F.nsrc + 255) / 256), 256, 0, h->stream>>>(F.nsrc, F.sj, h->wk.f1, h->wk.f2, F.fs1,
                                                                         F.fs2);
  SPM_HIP_CHECK(hipGetLastError());
  int s = 0;
  if (n_of(s)) launch_p2m(a, n_of(s), list(s), h->stream);
  SPM_HIP_CHECK(hipGetLastError());
  ++s;
  for (int l = F.L - 1; l >= 2; --l, ++s) {
    if (n_of(s)) k_fmm_m2m<<<n_of(s), 64, 0, h->stream>>>(a, l, list(s));
    SPM_HIP_CHECK(hipGetLastError());
  }
  return s;
}

}  // namespace

void launch_fmm_points(spm_handle* h, int64_t nt, const double* xt, const double* yt, double* u, double* p) {
  launch_fmm_upward(h);
  k_fmm_points<<<(unsigned)nt, 64, 0, h->stream>>>(args(h), h->geo, h->cfg.mu, h->cU[0], h->cU[1], nt, xt, yt, u, p);
  SPM_HIP_CHECK(hipGetLastError());
}

void launch_fmm_velocities(spm_handle* h, double* near3) {
  launch_fmm_upward(h);
  k_fmm_velocities<<<h->geo.No, 64, 0, h->stream>>>(args(h), h->geo, h->cfg.mu, near3);
  SPM_HIP_CHECK(hipGetLastError());
}

// doubles of the per-plan tables: M2L scalings [49][2][p] cx, M2M powers [4][p] cx, M2M lanes [16][5] int32
size_t fmm_table_doubles(int p) {
  return (size_t)49 * 2 * p * 2 + (size_t)4 * p * 2 + (kM2mLanes * kM2mSlots + 1) / 2;
}

void launch_fmm_tables(spm_handle* h) {
  const FmmPlan& F = h->fmm;
  if (F.p < 1 || F.p > kM2lMaxP) throw ApiError(SPM_EINVAL, "FMM order must be at most 64");
  k_fmm_m2l_tables<<<49, 64, 0, h->stream>>>(F.p, F.fact, reinterpret_cast<cx*>(F.m2l_tab));
  SPM_HIP_CHECK(hipGetLastError());
  cx* tp = reinterpret_cast<cx*>(F.m2l_tab) + (size_t)49 * 2 * F.p;
  k_fmm_m2m_tables<<<1, 64, 0, h->stream>>>(F.p, F.fact, tp, reinterpret_cast<int32_t*>(tp + (size_t)4 * F.p));
  SPM_HIP_CHECK(hipGetLastError());
}

void launch_fmm(spm_handle* h, double* out) {
  const FmmPlan& F = h->fmm;
  const FmmArgs a = args(h);
  const int L = F.L;
  auto n_of = [&](int s) { return (unsigned)(F.seg[s + 1] - F.seg[s]); };
  auto list = [&](int s) { return F.lists + F.seg[s]; };
  int s = launch_fmm_upward(h);
  prof_mark(h, 3, true, 0);
  if (n_of(s)) k_fmm_m2l<<<n_of(s), 64, 0, h->stream>>>(a, list(s));
  SPM_HIP_CHECK(hipGetLastError());
  prof_mark(h, 3, false, F.m2l);
  ++s;
  for (int l = 3; l <= L; ++l, ++s) {
    if (n_of(s)) k_fmm_l2l<<<n_of(s), 64, 0, h->stream>>>(a, l, list(s));
    SPM_HIP_CHECK(hipGetLastError());
  }
  const int64_t N = h->geo.N;
  prof_mark(h, 2, true, 0);
  if (n_of(s)) k_fmm_eval<<<n_of(s), 64 * kEvalWaves, 0, h->stream>>>(a, N, list(s), F.leaf_t, F.tperm, h->geo, out);
  SPM_HIP_CHECK(hipGetLastError());
  prof_mark(h, 2, false, F.p2p_pairs);
}

}  // namespace spm
