// Block (several vectors) two-pass matrix-free apply, templated; instantiated
// per precision by block_c128.hip and block_c64.hip.
#pragma once

#include <hip/hip_ext.h>

#include "coef_pack.h"
#include "kernels_common.h"

namespace hub {
namespace dev {

// H x for NV vectors interleaved per tile element, psi[(a dim_dn + b) NV + v]
// (the tensor-sum form H = D + T_up (x) 1 + 1 (x) T_dn of the spin-separated
// basis, Eq. (hubbardhamiltonian) with the phases of Eq. (peierls)):
//   row pass    z[a, b] = D[a, b] x[a, b] + sum over down hops b' -> b of coef x[a, b']
//   column pass y[a, b] = z[a, b] + sum over up hops a' -> a of coef x[a', b]
// The column pass either stores y (plain product) or finishes a Lanczos
// iteration: y = s_j (H u_j) - beta_{j-1} s_{j-1} u_{j-1}, alpha_j partials.
// Each pass stages its tile row (column) of all NV vectors once in LDS,
// followed by a zero element; a hop's table entry is src, src + dim + 1 for a
// negative fermion sign, or dim (the zero element) for padding.  The NV
// values of a tile element are L = NV / VPL 16-byte words (VPL = 2 complex64
// or 1 complex128 value per word), and L consecutive lanes own one element,
// a word each: global loads and stores of an element are contiguous across
// its lanes, a hop is one 16-byte LDS read per lane at consecutive words, and
// each lane keeps the coefficients of its VPL vectors in registers.  The
// table gives every class a slot range that is a multiple of four, so each
// group of four slots has one class: its signed staged values are summed
// first and the sum is multiplied by the class coefficient once.
struct BArgs {
  int dim_up, dim_dn, nc, j, m_max;
  double tol, norm_inf, U;
  const uint32_t* up_bits;
  const uint32_t* dn_bits;
  const double* eps_up;
  const double* eps_dn;
  const uint16_t* tab;   // this pass's grouped table [dim][MAXS]
  uint8_t grp_class[8];  // class of each group of four slots
  double coef[2 * kMaxNV * kMaxClasses];      // [v][c] complex hop coefficient
  double coef_obs[2 * kMaxNV * kMaxClasses];  // the same at the observation time
  const void* x;
  void* y;
  const void* xprev;
  VecState* st;
  StepCtl* ctl;
  double* partials;             // this kernel's partial sums
  const double* prev_partials;  // row pass, Lanczos: |u_j|^2 partials [prev_nblk][NV]
  int prev_nblk;
  // fused iterations (j >= 1): the row pass finishes the previous update
  const double* alpha_partials;  // the previous column pass's partials [alpha_nblk][alpha_stride][NV]
  int alpha_nblk, alpha_stride;
  const double* obs_row;         // j = 1 after the observables apply: its row-pass partials [dim_up][kObsQ][NV]
  double* norm;                  // |u_j|^2 per row [dim_up][NV]: written by the row pass, read by the column pass
};

// The VPL complex values of one 16-byte word.
template <typename V>
__device__ __forceinline__ void from_word(const uint4& u, V (&w)[16 / sizeof(V)]) {
  if constexpr (sizeof(V) == 16) {
    __builtin_memcpy(&w[0], &u, 16);
  } else {
    float4 f;
    __builtin_memcpy(&f, &u, 16);
    w[0] = V{f.x, f.y};
    w[1] = V{f.z, f.w};
  }
}

template <typename V>
__device__ __forceinline__ uint4 to_word(const V (&w)[16 / sizeof(V)]) {
  uint4 u;
  if constexpr (sizeof(V) == 16) {
    __builtin_memcpy(&u, &w[0], 16);
  } else {
    const float4 f = make_float4(w[0].x, w[0].y, w[1].x, w[1].y);
    __builtin_memcpy(&u, &f, 16);
  }
  return u;
}

// Sums over the workgroup of NQ per-lane values, separately for each word
// index k = lane % L (the lanes of one word index hold the same vectors):
// out[q * L + k] = sum over the threads with that k of vals[q], fixed order
// (shuffles in each wave, then the waves in order).  lds holds W * NQ * L
// doubles.
template <int W, int L, int NQ>
__device__ __forceinline__ void word_sums(const double (&vals)[NQ], double* lds, double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double v = vals[q];
#pragma unroll
    for (int off = 32; off >= L; off >>= 1) v += __shfl_xor(v, off);
    if (lane < L) lds[(w * NQ + q) * L + lane] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < NQ * L; t += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < W; ++k) s += lds[k * NQ * L + t];
    out[t] = s;
  }
}

// One group of four slots: the signed sum of the staged words they index
// (word k of each source element of L words), from the table word pair w.
template <typename R, int L>
__device__ __forceinline__ void group_sum(uint2 w, const uint4* xs, uint32_t dim, int k,
                                          typename CT<R>::T (&sum)[16 / sizeof(typename CT<R>::T)]) {
  using V = typename CT<R>::T;
  constexpr int VPL = 16 / sizeof(V);
#pragma unroll
  for (int i = 0; i < VPL; ++i) sum[i] = V{0, 0};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const uint32_t w2 = s < 2 ? w.x : w.y;
    const uint32_t idx = (s & 1) ? (w2 >> 16) : (w2 & 0xFFFFu);
    const bool neg = idx > dim;
    const uint32_t src = neg ? idx - dim - 1u : idx;
    const R sg = neg ? R(-1) : R(1);
    V t[VPL];
    from_word<V>(xs[static_cast<size_t>(src) * L + k], t);
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      sum[i].x = fma(sg, t[i].x, sum[i].x);
      sum[i].y = fma(sg, t[i].y, sum[i].y);
    }
  }
}

// The Krylov decision for m = j of every running vector (krylov_decide's
// rule: non-finite, breakdown, tolerance, m_max) from the estimate the fused
// row pass already recorded in S.eps and S.y; beta_new[v] = |u_j|.  Run by
// one workgroup.
template <int NV, int W>
__device__ void block_decide_pre(int j, const double* beta_new, VecState* st, StepCtl* ctl, int m_max, double tol,
                                 double norm_inf) {
  if (threadIdx.x < NV) {
    VecState& S = st[threadIdx.x];
    if (S.status == 0) {
      const double b = beta_new[threadIdx.x], eps = S.eps;
      S.beta[j - 1] = b;
      S.m = j;
      int status = 0;
      if (!isfinite(b) || !isfinite(eps)) status = 4;
      else if (b < norm_inf * tol) status = 2;
      else if (eps < tol) status = 1;
      else if (j >= m_max) status = 3;
      S.status = status;
      S.scale[j] = (status == 0 && b > 0.0) ? 1.0 / b : 0.0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int done = 1, maxed = 0;
    for (int v = 0; v < NV; ++v) {
      done &= (st[v].status != 0);
      maxed |= (st[v].status >= 3);
    }
    ctl->all_done = done;
    ctl->any_maxed = maxed;
    ctl->iter = j;
  }
}

// Row pass (one tile row a per workgroup).  Lanczos modes: an extra last
// workgroup takes the Krylov decision for m = j from the |u_j|^2 partials
// (the column pass reads what it recorded), so that no row waits for the
// estimate.  FUSE (iterations j >= 1): x holds w_{j-1} and the row pass first
// forms u_j = w_{j-1} - alpha_{j-1} s_{j-1} u_{j-1} of its row in place while
// staging it, with |u_j|^2 per row and vector for the column pass, which then
// takes the decision; the extra workgroup records alpha_{j-1}, at j = 1 the
// observables of the step's first apply, and the estimate for m = j of every
// running vector (it needs T_j only, not |u_j|; one wavefront per vector), and
// when every running vector's estimate is below tol the step ends at m = j
// and the column pass skips its apply.  M_LANCZOS_OBS (the step's first apply): per
// row, [diag, docc, |x|^2, down-hop part of Re <x|K(t_obs)|x>] for every
// vector into partials [dim_up][kObsQ][NV].
template <typename R, int NV, int MODE, int MAXS, int BLK, bool FUSE>
__global__ __launch_bounds__(BLK) void k_brow(BArgs p) {
  using V = typename CT<R>::T;
  constexpr int VPL = 16 / sizeof(V), L = NV / VPL, EPW = BLK / L, W = BLK / 64, kG = MAXS / 4;
  static_assert(L >= 1 && NV % VPL == 0 && BLK % L == 0, "whole words per element");
  constexpr bool kL = MODE == M_LANCZOS || MODE == M_LANCZOS_OBS;
  constexpr bool kO = MODE == M_LANCZOS_OBS;
  __shared__ double red[W * kObsQ * NV + W];
  __shared__ double sh_beta[NV];
  static_assert(!FUSE || MODE == M_LANCZOS, "fused row pass: Lanczos iterations j >= 1");
  const int tid = threadIdx.x;
  const int k = tid % L, e0 = tid / L;
  R cu[VPL];  // FUSE: alpha_{j-1} s_{j-1} of this lane's vectors
  if (FUSE) {
    if (p.ctl->all_done) return;
    for (int t = 0; t < NV; ++t) {
      const double s = reduce_column<W>(p.alpha_partials, p.alpha_nblk, p.alpha_stride * NV, t, red);
      if (tid == 0) sh_beta[t] = s;  // alpha_{j-1} of vector t
    }
    __syncthreads();
    if (blockIdx.x == gridDim.x - 1) {
      if (tid < NV && p.st[tid].status == 0) p.st[tid].alpha[p.j - 1] = sh_beta[tid];
      if (p.obs_row)  // [diag, docc, n2, down-hop part] of the rows, up-hop part in the columns' second column
        for (int t = 0; t < kObsQ * NV; ++t) {
          double s = reduce_column<W>(p.obs_row, p.dim_up, kObsQ * NV, t, red);
          if (t / NV == kObsQ - 1) s += reduce_column<W>(p.alpha_partials, p.alpha_nblk, p.alpha_stride * NV, NV + t % NV, red);
          if (tid == 0) p.st[t % NV].obs[t / NV] = s;
        }
      __shared__ int sh_end;  // every running vector's estimate for m = j is below tol
      if (tid == 0) sh_end = 1;
      __syncthreads();
      const int lane = tid & 63, wv = tid >> 6;
      for (int v = wv; v < NV; v += W) {
        VecState& S = p.st[v];
        if (S.status != 0) continue;
        const double aj = lane < p.j - 1 ? S.alpha[lane] : (lane == p.j - 1 ? sh_beta[v] : 0.0);
        double yr, yi;
        const double eps = wave_krylov_eps(p.j, aj, S.beta, S.tau, S.y, lane, yr, yi);
        if (lane < p.j) {  // every lane has read y^(j-1): its reductions fed eps
          S.y[2 * lane] = yr;
          S.y[2 * lane + 1] = yi;
        }
        if (lane == 0) {
          S.eps = eps;
          if (!(eps < p.tol)) sh_end = 0;
        }
      }
      __syncthreads();
      if (tid == 0) p.ctl->eps_stop = sh_end ? p.j : -1;
      return;
    }
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      const int v = k * VPL + i;
      cu[i] = static_cast<R>(sh_beta[v] * p.st[v].scale[p.j - 1]);
    }
  } else if (kL) {
    if (p.ctl->all_done) return;
    if (blockIdx.x == gridDim.x - 1) {
      for (int t = 0; t < NV; ++t) {
        const double s = reduce_column<W>(p.prev_partials, p.prev_nblk, NV, t, red);
        if (tid == 0) sh_beta[t] = sqrt(s);
      }
      __syncthreads();
      krylov_decide<NV, W>(p.j, sh_beta, p.st, p.ctl, p.m_max, p.tol, p.norm_inf);
      return;
    }
    if (p.j >= p.m_max) return;  // only the decision was needed
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint4* xs = reinterpret_cast<uint4*>(smem_raw);
  const int a = xcd_remap(blockIdx.x, kL ? gridDim.x - 1 : gridDim.x);
  const int dd = p.dim_dn;
  const size_t roww = static_cast<size_t>(a) * dd * L;  // first word of the row
  if (FUSE) {
    // u_j = w_{j-1} - alpha s u_{j-1} of the row, in place and staged; |u_j|^2
    // per vector (a thread's words all hold the vectors of word index k)
    uint4* w4 = static_cast<uint4*>(const_cast<void*>(p.x)) + roww;
    const uint4* u4 = static_cast<const uint4*>(p.xprev) + roww;
    double n2[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) n2[i] = 0.0;
    for (int t = tid; t < (dd + 1) * L; t += BLK) {
      uint4 o = make_uint4(0u, 0u, 0u, 0u);
      if (t < dd * L) {
        V wv[VPL], uv[VPL];
        from_word<V>(w4[t], wv);
        from_word<V>(u4[t], uv);
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
          wv[i].x -= cu[i] * uv[i].x;
          wv[i].y -= cu[i] * uv[i].y;
          n2[i] += static_cast<double>(wv[i].x) * wv[i].x + static_cast<double>(wv[i].y) * wv[i].y;
        }
        o = to_word<V>(wv);
        w4[t] = o;
      }
      xs[t] = o;
    }
    __shared__ double tn[NV];
    word_sums<W, L, VPL>(n2, red, tn);
    __syncthreads();
    for (int t = tid; t < NV; t += BLK) p.norm[static_cast<size_t>(a) * NV + t] = tn[(t % VPL) * L + t / VPL];
    if (!p.y) return;  // j = m_max: only the norm was needed
  } else {
    const uint4* x4 = static_cast<const uint4*>(p.x) + roww;
    for (int t = tid; t < (dd + 1) * L; t += BLK) xs[t] = t < dd * L ? x4[t] : make_uint4(0u, 0u, 0u, 0u);
  }
  // coefficients of this lane's vectors v = k VPL + i
  V cf[kG][VPL];
  double2 ocf[kO ? kG : 1][VPL];
#pragma unroll
  for (int g = 0; g < kG; ++g)
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      const int v = k * VPL + i, c = p.grp_class[g];
      cf[g][i] = V{static_cast<R>(p.coef[2 * (v * p.nc + c)]), static_cast<R>(p.coef[2 * (v * p.nc + c) + 1])};
      if constexpr (kO) ocf[g][i] = make_double2(p.coef_obs[2 * (v * p.nc + c)], p.coef_obs[2 * (v * p.nc + c) + 1]);
    }
  __syncthreads();

  const uint32_t ua = p.up_bits[a];
  const double ea = p.eps_up ? p.eps_up[a] : 0.0;
  const uint2* tab2 = reinterpret_cast<const uint2*>(p.tab);
  uint4* __restrict__ y4 = static_cast<uint4*>(p.y) + roww;
  double q[kO ? kObsQ * VPL : 1];
#pragma unroll
  for (int i = 0; i < (kO ? kObsQ * VPL : 1); ++i) q[i] = 0.0;
  for (int b = e0; b < dd; b += EPW) {
    uint2 ev[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) ev[g] = tab2[static_cast<size_t>(b) * kG + g];
    const double nd = static_cast<double>(__popc(ua & p.dn_bits[b]));
    const double dg = p.U * nd + ea + (p.eps_dn ? p.eps_dn[b] : 0.0);
    V xv[VPL], acc[VPL];
    from_word<V>(xs[static_cast<size_t>(b) * L + k], xv);
#pragma unroll
    for (int i = 0; i < VPL; ++i) acc[i] = V{static_cast<R>(dg) * xv[i].x, static_cast<R>(dg) * xv[i].y};
    double2 ko[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) ko[i] = make_double2(0.0, 0.0);
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      V sum[VPL];
      group_sum<R, L>(ev[g], xs, static_cast<uint32_t>(dd), k, sum);
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        acc[i] = cfma(cf[g][i], sum[i], acc[i]);
        if constexpr (kO) ko[i] = cfma(ocf[g][i], make_double2(sum[i].x, sum[i].y), ko[i]);
      }
    }
    y4[static_cast<size_t>(b) * L + k] = to_word<V>(acc);
    if constexpr (kO) {
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        const double m2 = static_cast<double>(xv[i].x) * xv[i].x + static_cast<double>(xv[i].y) * xv[i].y;
        q[0 * VPL + i] += dg * m2;
        q[1 * VPL + i] += nd * m2;
        q[2 * VPL + i] += m2;
        q[3 * VPL + i] += static_cast<double>(xv[i].x) * ko[i].x + static_cast<double>(xv[i].y) * ko[i].y;
      }
    }
  }
  // out[(qq VPL + i) L + k] -> partials [row][qq][v = k VPL + i]
  if constexpr (kO) {
    __shared__ double tot[kObsQ * NV];
    word_sums<W, L, kObsQ * VPL>(q, red, tot);
    __syncthreads();
    for (int t = tid; t < kObsQ * NV; t += BLK) {
      const int qq = t / NV, v = t % NV;
      p.partials[static_cast<size_t>(a) * kObsQ * NV + t] = tot[(qq * VPL + v % VPL) * L + v / VPL];
    }
  }
}

// Column pass (one tile column b per workgroup).  Lanczos modes read the
// decision the row pass recorded and write alpha partials [grid][NV]
// (M_LANCZOS_OBS: [grid][2][NV], alpha and the up-hop part of
// Re <x|K(t_obs)|x>).  A vector whose step ended at an earlier iteration
// gets a zero result.  FUSE: |u_j| comes from the row pass's per-row norms and
// an extra last workgroup takes the decision for m = j (a vector that has
// stopped gets a result no later step reads).
template <typename R, int NV, int MODE, int MAXS, int BLK, bool FUSE>
__global__ __launch_bounds__(BLK) void k_bcol(BArgs p) {
  using V = typename CT<R>::T;
  constexpr int VPL = 16 / sizeof(V), L = NV / VPL, EPW = BLK / L, W = BLK / 64, kG = MAXS / 4;
  static_assert(L >= 1 && NV % VPL == 0 && BLK % L == 0, "whole words per element");
  constexpr bool kL = MODE == M_LANCZOS || MODE == M_LANCZOS_OBS;
  constexpr bool kO = MODE == M_LANCZOS_OBS;
  constexpr int kNQ = kO ? 2 : 1;  // per vector: alpha [, up-hop obs part]
  __shared__ double red[W * kNQ * NV];
  const int tid = threadIdx.x;
  const int k = tid % L, e0 = tid / L;
  R sj[VPL], bp[VPL];
#pragma unroll
  for (int i = 0; i < VPL; ++i) {
    sj[i] = 1;
    bp[i] = 0;
  }
  static_assert(!FUSE || MODE == M_LANCZOS, "fused column pass: Lanczos iterations j >= 1");
  if (FUSE) {
    if (p.ctl->all_done) return;
    // the row pass found every running vector's estimate for m = j below tol:
    // the step ends here and only the decision is left
    const bool decide = blockIdx.x == gridDim.x - 1;
    if (p.ctl->eps_stop == p.j && !decide) return;
    __shared__ double sh_b[NV];
    for (int t = 0; t < NV; ++t) {
      const double s = reduce_column<W>(p.norm, p.dim_up, NV, t, red);
      if (tid == 0) sh_b[t] = sqrt(s);  // |u_j| = beta_{j-1} of vector t
    }
    __syncthreads();
    if (decide) {
      block_decide_pre<NV, W>(p.j, sh_b, p.st, p.ctl, p.m_max, p.tol, p.norm_inf);
      return;
    }
    if (p.j >= p.m_max) return;  // only the decision was needed
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      const int v = k * VPL + i;
      const double bv = sh_b[v];
      sj[i] = static_cast<R>(bv > 0.0 ? 1.0 / bv : 0.0);
      bp[i] = static_cast<R>(bv > 0.0 ? bv * p.st[v].scale[p.j - 1] : 0.0);
    }
  } else if (kL) {
    if (p.ctl->all_done) return;
    if (p.j >= p.m_max) return;
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      const VecState& S = p.st[k * VPL + i];
      const double bv = p.j == 0 ? S.beta0 : (S.m >= p.j ? S.beta[p.j - 1] : 0.0);
      sj[i] = static_cast<R>(bv > 0.0 ? 1.0 / bv : 0.0);
      bp[i] = static_cast<R>(p.j > 0 && bv > 0.0 ? bv * S.scale[p.j - 1] : 0.0);
    }
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint4* xs = reinterpret_cast<uint4*>(smem_raw);
  const int b = xcd_remap(blockIdx.x, FUSE ? gridDim.x - 1 : gridDim.x);
  const int du = p.dim_up, dd = p.dim_dn;
  {
    const uint4* x4 = static_cast<const uint4*>(p.x);
    for (int t = tid; t < (du + 1) * L; t += BLK) {
      const int a = t / L, kk = t % L;
      xs[t] = a < du ? x4[(static_cast<size_t>(a) * dd + b) * L + kk] : make_uint4(0u, 0u, 0u, 0u);
    }
  }
  V cf[kG][VPL];
  double2 ocf[kO ? kG : 1][VPL];
#pragma unroll
  for (int g = 0; g < kG; ++g)
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      const int v = k * VPL + i, c = p.grp_class[g];
      cf[g][i] = V{static_cast<R>(p.coef[2 * (v * p.nc + c)]), static_cast<R>(p.coef[2 * (v * p.nc + c) + 1])};
      if constexpr (kO) ocf[g][i] = make_double2(p.coef_obs[2 * (v * p.nc + c)], p.coef_obs[2 * (v * p.nc + c) + 1]);
    }
  __syncthreads();

  const uint2* tab2 = reinterpret_cast<const uint2*>(p.tab);
  uint4* __restrict__ y4 = static_cast<uint4*>(p.y);
  const uint4* __restrict__ xp4 = static_cast<const uint4*>(p.xprev);
  double q[kL ? kNQ * VPL : 1];
#pragma unroll
  for (int i = 0; i < (kL ? kNQ * VPL : 1); ++i) q[i] = 0.0;
  for (int a = e0; a < du; a += EPW) {
    uint2 ev[kG];
#pragma unroll
    for (int g = 0; g < kG; ++g) ev[g] = tab2[static_cast<size_t>(a) * kG + g];
    const size_t o = (static_cast<size_t>(a) * dd + b) * L + k;  // this lane's word of element (a, b)
    V acc[VPL], pv[VPL];
    from_word<V>(y4[o], acc);
    if (kL && p.j > 0) from_word<V>(xp4[o], pv);
    double2 ko[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) ko[i] = make_double2(0.0, 0.0);
#pragma unroll
    for (int g = 0; g < kG; ++g) {
      V sum[VPL];
      group_sum<R, L>(ev[g], xs, static_cast<uint32_t>(du), k, sum);
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        acc[i] = cfma(cf[g][i], sum[i], acc[i]);
        if constexpr (kO) ko[i] = cfma(ocf[g][i], make_double2(sum[i].x, sum[i].y), ko[i]);
      }
    }
    if constexpr (kL) {
      V xv[VPL];
      from_word<V>(xs[static_cast<size_t>(a) * L + k], xv);
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        const V pvv = p.j > 0 ? pv[i] : V{0, 0};
        acc[i].x = acc[i].x * sj[i] - bp[i] * pvv.x;
        acc[i].y = acc[i].y * sj[i] - bp[i] * pvv.y;
        q[i] += static_cast<double>(sj[i]) *
                (static_cast<double>(xv[i].x) * acc[i].x + static_cast<double>(xv[i].y) * acc[i].y);
        if constexpr (kO) q[VPL + i] += static_cast<double>(xv[i].x) * ko[i].x + static_cast<double>(xv[i].y) * ko[i].y;
      }
    }
    y4[o] = to_word<V>(acc);
  }
  if constexpr (kL) {
    __shared__ double tot[kNQ * NV];
    word_sums<W, L, kNQ * VPL>(q, red, tot);
    __syncthreads();
    for (int t = tid; t < kNQ * NV; t += BLK) {
      const int qq = t / NV, v = t % NV;
      p.partials[static_cast<size_t>(b) * kNQ * NV + t] = tot[(qq * VPL + v % VPL) * L + v / VPL];
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers.

inline BArgs block_args(const ApplyLaunch& L, bool row) {
  const DevBasis& db = *L.db;
  BArgs p{};
  p.dim_up = db.dim_up;
  p.dim_dn = db.dim_dn;
  p.nc = db.nc;
  p.j = L.j;
  p.m_max = L.m_max;
  p.tol = L.tol;
  p.norm_inf = L.norm_inf;
  p.U = db.U;
  p.up_bits = db.up_bits;
  p.dn_bits = db.dn_bits;
  p.eps_up = db.eps_up;
  p.eps_dn = db.eps_dn;
  p.tab = row ? db.dn_tabg : db.up_tabg;
  for (int g = 0; g < 8; ++g) p.grp_class[g] = row ? db.dn_gclass[g] : db.up_gclass[g];
  // the caller's coefficient arrays hold [nv][nc] complex pairs
  pack_block_coefs(L.coef, L.nv, db.nc, p.coef, 2 * kMaxNV * kMaxClasses);
  pack_block_coefs(L.coef_obs, L.nv, db.nc, p.coef_obs, 2 * kMaxNV * kMaxClasses);
  p.x = L.x;
  p.y = L.y;
  p.xprev = L.xprev;
  p.st = L.st;
  p.ctl = L.ctl;
  p.prev_partials = L.prev_partials;
  p.prev_nblk = L.prev_nblk;
  p.alpha_partials = L.alpha_partials;
  p.alpha_nblk = L.alpha_nblk;
  p.alpha_stride = L.alpha_stride;
  p.obs_row = L.obs_row;
  p.norm = L.norm_partials;
  return p;
}

// Threads per block-kernel workgroup.
constexpr int kBlkThreads = 512;

template <typename R, int NV, int MODE, int MAXS_R, int MAXS_C, bool FUSE>
hipError_t block_pair(const ApplyLaunch& L, int* pgrid) {
  const DevBasis& db = *L.db;
  constexpr bool kO = MODE == M_LANCZOS_OBS;
  const size_t es = sizeof(typename CT<R>::T);
  // row pass
  BArgs pr = block_args(L, true);
  pr.partials = kO ? L.row_obs : nullptr;
  auto fr = k_brow<R, NV, MODE, MAXS_R, kBlkThreads, FUSE>;
  static const int max_r = dyn_lds_opt_in(reinterpret_cast<const void*>(fr));
  const size_t lds_r = (static_cast<size_t>(db.dim_dn) + 1) * NV * es;
  if (lds_r > static_cast<size_t>(max_r)) return hipErrorInvalidValue;
  // Lanczos modes: one more workgroup for the Krylov decision (fused: for
  // alpha_{j-1} and the observables)
  constexpr bool kDecide = MODE == M_LANCZOS || MODE == M_LANCZOS_OBS;
  hipError_t e = launch_ev(fr, kDecide ? db.dim_up + 1 : db.dim_up, kBlkThreads, lds_r, L.stream, L.ev_start,
                           L.ev_stop, pr);
  if (e != hipSuccess) return e;
  // column pass
  BArgs pc = block_args(L, false);
  pc.partials = L.partials;
  auto fc = k_bcol<R, NV, MODE, MAXS_C, kBlkThreads, FUSE>;
  static const int max_c = dyn_lds_opt_in(reinterpret_cast<const void*>(fc));
  const size_t lds_c = (static_cast<size_t>(db.dim_up) + 1) * NV * es;
  if (lds_c > static_cast<size_t>(max_c)) return hipErrorInvalidValue;
  if (pgrid) *pgrid = db.dim_dn;
  // fused: one more workgroup for the Krylov decision
  return launch_ev(fc, FUSE ? db.dim_dn + 1 : db.dim_dn, kBlkThreads, lds_c, L.stream, L.ev2_start, L.ev2_stop, pc);
}

template <typename R, int NV, int MODE, int MAXS_R, bool FUSE>
hipError_t block_col_s(const ApplyLaunch& L, int* pgrid) {
  switch (L.db->up_gslots) {
    case 8: return block_pair<R, NV, MODE, MAXS_R, 8, FUSE>(L, pgrid);
    case 12: return block_pair<R, NV, MODE, MAXS_R, 12, FUSE>(L, pgrid);
    case 16: return block_pair<R, NV, MODE, MAXS_R, 16, FUSE>(L, pgrid);
    case 20: return block_pair<R, NV, MODE, MAXS_R, 20, FUSE>(L, pgrid);
    case 24: return block_pair<R, NV, MODE, MAXS_R, 24, FUSE>(L, pgrid);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, int NV, int MODE, bool FUSE = false>
hipError_t block_row_s(const ApplyLaunch& L, int* pgrid) {
  switch (L.db->dn_gslots) {
    case 8: return block_col_s<R, NV, MODE, 8, FUSE>(L, pgrid);
    case 12: return block_col_s<R, NV, MODE, 12, FUSE>(L, pgrid);
    case 16: return block_col_s<R, NV, MODE, 16, FUSE>(L, pgrid);
    case 20: return block_col_s<R, NV, MODE, 20, FUSE>(L, pgrid);
    case 24: return block_col_s<R, NV, MODE, 24, FUSE>(L, pgrid);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, int NV>
hipError_t block_mode(const ApplyLaunch& L, int* pgrid) {
  if (L.mode == kPlain) return block_row_s<R, NV, M_PLAIN>(L, pgrid);
  if (L.mode != kLanczos) return hipErrorInvalidValue;
  if (L.obs) return block_row_s<R, NV, M_LANCZOS_OBS>(L, pgrid);
  if (L.fuse) return block_row_s<R, NV, M_LANCZOS, true>(L, pgrid);
  return block_row_s<R, NV, M_LANCZOS>(L, pgrid);
}

template <typename R>
hipError_t block_nv(const ApplyLaunch& L, int* pgrid) {
  switch (L.nv) {
    case 2: return block_mode<R, 2>(L, pgrid);
    case 4: return block_mode<R, 4>(L, pgrid);
    case 8: return block_mode<R, 8>(L, pgrid);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dev
}  // namespace hub
