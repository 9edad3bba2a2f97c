// HIP kernels for gfx950 (CDNA4, wave64): matrix-free Peierls-Hubbard apply
// with fused Lanczos epilogue and Krylov decision, Lanczos update, Krylov
// combine, and BLAS-1 helpers.
//
// Cross-workgroup reductions never use in-kernel fences (an agent-scope
// release writes back the whole L2 of an XCD).  Every kernel writes
// per-workgroup partial sums; the NEXT kernel on the stream sums them in a
// fixed order (kernel boundaries make them visible), so results are
// deterministic and bitwise reproducible.
#include "kernels_common.h"

#include <algorithm>

namespace hub {
namespace dev {

// u_{j+1} = w - alpha_j s_j u_j in place (w holds s_j H u_j - beta s u_{j-1}),
// with alpha_j the fixed-order total of the apply's partials; |u_{j+1}|^2
// partials for the next apply.  Workgroup 0 records alpha_j and, after the
// step's first apply, the observables.
template <typename R, int NV>
__global__ __launch_bounds__(kBlock) void k_update(int64_t n, typename CT<R>::T* w,
                                                   const typename CT<R>::T* uj, VecState* st,
                                                   StepCtl* ctl, int j, const double* apply_partials,
                                                   int apply_nblk, int apply_nq, const double* row_obs,
                                                   int row_nblk, double* partials) {
  using V = typename CT<R>::T;
  __shared__ double red[kWaves * kMaxNV];
  __shared__ double sh_alpha[kMaxNV];
  if (ctl->all_done) return;
  const int tid = threadIdx.x;
  const int qn = apply_nq * NV;
  for (int t = 0; t < NV; ++t) {
    const double s = reduce_column(apply_partials, apply_nblk, qn, t, red);  // alpha is column 0 * NV + t
    if (tid == 0) sh_alpha[t] = s;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid < NV && st[tid].status == 0) st[tid].alpha[j] = sh_alpha[tid];
    if (!row_obs) {
      for (int t = NV; t < qn; ++t) {  // observables of the step's first vector
        const double s = reduce_column(apply_partials, apply_nblk, qn, t, red);
        if (tid == 0) st[t % NV].obs[t / NV - 1] = s;
      }
    } else {
      // two-pass apply: [diag, docc, n2, down-hop part] from the row pass,
      // the up-hop part of <x|K(t_obs)|x> in column 1 of the column pass
      for (int t = 0; t < kObsQ * NV; ++t) {
        double s = reduce_column(row_obs, row_nblk, kObsQ * NV, t, red);
        if (t / NV == kObsQ - 1) s += reduce_column(apply_partials, apply_nblk, qn, NV + t % NV, red);
        if (tid == 0) st[t % NV].obs[t / NV] = s;
      }
    }
  }
  const int v = tid % NV;
  const R c = static_cast<R>(sh_alpha[v] * st[v].scale[j]);
  double n2 = 0.0;
  const int64_t total = n * NV;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + tid; i < total; i += (int64_t)gridDim.x * kBlock) {
    const V u = uj[i];
    V t = w[i];
    t.x -= c * u.x;
    t.y -= c * u.y;
    w[i] = t;
    n2 += (double)t.x * t.x + (double)t.y * t.y;
  }
  block_partials<NV>(&n2, 1, red, partials + (size_t)blockIdx.x * NV);
}

// Records a finished step (workgroup 0 of its combine, or k_step_log):
// Krylov report into log, first-apply observables into obs_log, and a cleared
// control block; after a step where a vector hit m_max, the combines from
// sequence number seq + 1 on do nothing and the Lanczos kernels stay idle.
template <int NV>
__device__ void record_step(const VecState* st, StepCtl* ctl, CombineLog* log, double* obs_log, int nobs, int seq) {
  const int v = threadIdx.x;
  if (v < NV) {
    const VecState& S = st[v];
    if (log) {
      log[v].m = S.m;
      log[v].status = S.status;
      log[v].eps = S.eps;
      log[v].beta_last = S.m > 0 ? S.beta[S.m - 1] : 0.0;
    }
    if (obs_log)
      for (int k = 0; k < nobs; ++k) obs_log[v * nobs + k] = S.obs[k];
  }
  if (v == 0) {
    ctl->all_done = 0;
    ctl->any_maxed = 0;
    ctl->iter = 0;
    ctl->steps_done += 1;
    int maxed = 0;
    for (int w = 0; w < NV; ++w) maxed |= (st[w].status >= 3);
    if (maxed && log) {  // a vector hit m_max (or went non-finite): later enqueued steps do nothing
      ctl->halt_from = seq + 1;
      ctl->all_done = 1;
    }
  }
}

// v <- beta0 sum_{k<m_v} s_k y_k u_k into slot 0, and |v|^2 partials for the
// next step's first apply; workgroup 0 then records the step (its other
// workgroups read the control block only at their start, and the record's
// halt applies from the next sequence number on).
template <typename R, int NV>
__global__ __launch_bounds__(kBlock) void k_combine(int64_t n, void* const* slots, const VecState* st,
                                                    StepCtl* ctl, double* partials, int seq, CombineLog* log,
                                                    double* obs_log, int nobs, void* out2) {
  using V = typename CT<R>::T;
  __shared__ double red[kWaves * kMaxNV];
  __shared__ double cr[kMaxNV][kMMax], ci[kMaxNV][kMMax];
  __shared__ int mv[kMaxNV];
  const int tid = threadIdx.x;
  // A step whose launches ended before every vector was decided is abandoned
  // with slot 0 unchanged; the flag makes the rest of the enqueued work idle.
  if (ctl->abort || (ctl->halt_from > 0 && seq >= ctl->halt_from)) return;
  bool undecided = false;
  for (int v = 0; v < NV; ++v) undecided |= (st[v].status == 0);
  if (undecided) {
    if (blockIdx.x == 0 && tid == 0) {
      ctl->abort = 1;
      ctl->all_done = 1;
    }
    return;
  }
  for (int t = tid; t < NV * kMMax; t += kBlock) {
    const int vv = t / kMMax, k = t % kMMax;
    const VecState& S = st[vv];
    const double f = S.beta0 * S.scale[k];
    cr[vv][k] = (k < S.m) ? f * S.y[2 * k] : 0.0;
    ci[vv][k] = (k < S.m) ? f * S.y[2 * k + 1] : 0.0;
    if (k == 0) mv[vv] = S.m;
  }
  __syncthreads();
  const int v = tid % NV;
  const int m = mv[v];
  V* out = static_cast<V*>(slots[0]);
  double n2 = 0.0;
  const int64_t total = n * NV;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + tid; i < total; i += (int64_t)gridDim.x * kBlock) {
    double ar = 0.0, ai = 0.0;
    for (int k = 0; k < m; ++k) {
      const V u = static_cast<const V*>(slots[k])[i];
      ar += cr[v][k] * u.x - ci[v][k] * u.y;
      ai += cr[v][k] * u.y + ci[v][k] * u.x;
    }
    const V o = V{static_cast<R>(ar), static_cast<R>(ai)};
    out[i] = o;
    if (out2) static_cast<V*>(out2)[i] = o;
    n2 += (double)o.x * o.x + (double)o.y * o.y;
  }
  block_partials<NV>(&n2, 1, red, partials + (size_t)blockIdx.x * NV);
  if (blockIdx.x == 0) record_step<NV>(st, ctl, log, obs_log, nobs, seq);
}

// |v|^2 partials of the step's input (first step of a call), tau for every
// vector, and a cleared control block.
template <typename R, int NV>
__global__ __launch_bounds__(kBlock) void k_step_begin(int64_t n, const typename CT<R>::T* x, VecState* st,
                                                       StepCtl* ctl, double tau, int norm, double* partials) {
  using V = typename CT<R>::T;
  __shared__ double red[kWaves * kMaxNV];
  if (ctl->abort) return;
  const int tid = threadIdx.x;
  double n2 = 0.0;
  if (norm) {
    const int64_t total = n * NV;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + tid; i < total; i += (int64_t)gridDim.x * kBlock) {
      const V t = x[i];
      n2 += (double)t.x * t.x + (double)t.y * t.y;
    }
    block_partials<NV>(&n2, 1, red, partials + (size_t)blockIdx.x * NV);
  }
  if (blockIdx.x == 0 && tid < NV) st[tid].tau = tau;
  if (blockIdx.x == 0 && tid == 0) {
    ctl->all_done = 0;
    ctl->any_maxed = 0;
    ctl->iter = 0;
  }
}

// Records the observables of the last sample time (no log): a cleared
// control block and obs_log; nothing after an abandoned step.
template <int NV>
__global__ void k_step_log(const VecState* st, StepCtl* ctl, CombineLog* log, double* obs_log, int nobs) {
  if (ctl->abort) return;
  record_step<NV>(st, ctl, log, obs_log, nobs, 0);
}

// Column sums (op 0) or maxima (op 1) of a [nrows][ncols] partial array,
// one workgroup per column, fixed order.
__global__ __launch_bounds__(kBlock) void k_finalize(const double* partials, int nrows, int ncols, double* out,
                                                     int op) {
  __shared__ double red[kWaves];
  const int t = blockIdx.x;
  double s = 0.0;  // the maxima are of non-negative partials
  for (int b = threadIdx.x; b < nrows; b += blockDim.x) {
    const double x = partials[(size_t)b * ncols + t];
    s = op ? fmax(s, x) : s + x;
  }
  if (op) {
    s = wave_max(s);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = 0.0;
      for (int k = 0; k < kWaves; ++k) m = fmax(m, red[k]);
      out[t] = m;
    }
  } else {
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[t] = s;
  }
}

// Observables of an apply in kObsOnly mode: finalize its partials into st.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_finalize_obs(const double* partials, int nrows, int nq, VecState* st) {
  __shared__ double red[kWaves];
  const int qn = nq * NV;
  for (int t = 0; t < qn; ++t) {
    const double s = reduce_column(partials, nrows, qn, t, red);
    if (threadIdx.x == 0) st[t % NV].obs[t / NV] = s;
  }
}

template <typename R>
__global__ void k_interleave(int64_t n, int nv, const typename CT<R>::T* src, typename CT<R>::T* dst,
                             int to_block) {
  const int64_t total = n * nv;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = i / nv, v = i % nv;  // block layout i = k*nv + v ; ABI layout v*n + k
    if (to_block) dst[i] = src[v * n + k];
    else dst[v * n + k] = src[i];
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_site_docc(int dim_up, int dim_dn, int n_sites, const uint32_t* up,
                                                      const uint32_t* dn, const typename CT<R>::T* x,
                                                      double* partials) {
  __shared__ double red[kWaves * kMaxSites];
  double acc[kMaxSites];
#pragma unroll
  for (int i = 0; i < kMaxSites; ++i) acc[i] = 0.0;
  const int64_t n = (int64_t)dim_up * dim_dn;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock) {
    const auto t = x[k];
    const double m2 = (double)t.x * t.x + (double)t.y * t.y;
    const uint32_t d = up[k / dim_dn] & dn[k % dim_dn];
#pragma unroll
    for (int i = 0; i < kMaxSites; ++i)
      if ((d >> i) & 1u) acc[i] += m2;
  }
  block_partials<1>(acc, n_sites, red, partials + (size_t)blockIdx.x * n_sites);
}

// y = sign * x at the mapped source element: a creation or annihilation
// operator between two sectors.  For an up operator the map acts on tile rows
// (map[a'] = source row, -1 = no source), for a down operator on columns.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cop(int64_t n_t, int dim_dn_t, int dim_dn_s, int64_t n_s, int nvec,
                                                 int down, const int32_t* map, const int8_t* sgn,
                                                 const typename CT<R>::T* x, typename CT<R>::T* y) {
  using V = typename CT<R>::T;
  const int64_t total = n_t * nvec;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int64_t k = i / n_t, e = i % n_t;
    const int a = static_cast<int>(e / dim_dn_t), b = static_cast<int>(e % dim_dn_t);
    const int r = down ? b : a;
    const int src = map[r];
    V out = V{0, 0};
    if (src >= 0) {
      const int64_t se = down ? (int64_t)a * dim_dn_s + src : (int64_t)src * dim_dn_s + b;
      const V v = x[k * n_s + se];
      const R f = static_cast<R>(sgn[r]);
      out = V{f * v.x, f * v.y};
    }
    y[i] = out;
  }
}

// <x_k | y_k> partials for nvec vector pairs (ABI layout), [grid][2 * nvec].
template <typename R>
__global__ __launch_bounds__(kBlock) void k_dots(int64_t n, int nvec, const typename CT<R>::T* x,
                                                  const typename CT<R>::T* y, double* partials) {
  __shared__ double red[kWaves];
  for (int k = 0; k < nvec; ++k) {
    double re = 0.0, im = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
      const auto a = x[k * n + i];
      const auto b = y[k * n + i];
      re += (double)a.x * b.x + (double)a.y * b.y;
      im += (double)a.x * b.y - (double)a.y * b.x;
    }
    re = block_sum(re, red);
    im = block_sum(im, red);
    if (threadIdx.x == 0) {
      partials[(size_t)blockIdx.x * 2 * nvec + 2 * k] = re;
      partials[(size_t)blockIdx.x * 2 * nvec + 2 * k + 1] = im;
    }
  }
}

// Overlaps of NV members with the state they were made from (Sec. 2.5,
// Eq. (Glg)): member v, in the target sector, with operator map map_v (tile
// rows for an up operator, columns for a down one; -1 = no source) and signs
// sgn_v, and psi_v the source-sector state at its time,
//   o_v = <c_v psi_v | phi_v> = sum_y sgn_v(y) conj(psi_v[src_v(y)]) phi_v[y],
// gathered straight from psi_v (no copy of c_v psi_v).  phi is interleaved
// ([y][NV]) or in the ABI layout ([v][n_t]).  Partials [NV][grid][2]; the
// kernel does nothing after an abandoned step (ctl->abort).
template <typename R, int NV>
__global__ __launch_bounds__(kBlock) void k_overlaps(OverlapArgs p) {
  using V = typename CT<R>::T;
  __shared__ double red[kWaves];
  if (p.ctl && p.ctl->abort) return;
  const V* psi = static_cast<const V*>(p.traj);
  const V* phi = static_cast<const V*>(p.phi);
  double acc[2 * NV];
#pragma unroll
  for (int q = 0; q < 2 * NV; ++q) acc[q] = 0.0;
  for (int64_t y = (int64_t)blockIdx.x * kBlock + threadIdx.x; y < p.n_t; y += (int64_t)gridDim.x * kBlock) {
    const int a = static_cast<int>(y / p.dim_dn_t), b = static_cast<int>(y % p.dim_dn_t);
    const int r = p.down ? b : a;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int src = p.maps[v * p.map_len + r];
      if (src < 0) continue;
      const int64_t se = p.down ? (int64_t)a * p.dim_dn_s + src : (int64_t)src * p.dim_dn_s + b;
      const V x = psi[p.psi_off[v] + se];
      const V f = p.interleaved ? phi[y * NV + v] : phi[v * p.n_t + y];
      const double sg = static_cast<double>(p.sgns[v * p.map_len + r]);
      acc[2 * v] += sg * ((double)x.x * f.x + (double)x.y * f.y);
      acc[2 * v + 1] += sg * ((double)x.x * f.y - (double)x.y * f.x);
    }
  }
  // member v's pair goes to partials + (v grid + workgroup) 2
#pragma unroll
  for (int q = 0; q < 2 * NV; ++q) {
    const double t = block_sum(acc[q], red);
    if (threadIdx.x == 0) p.partials[((size_t)(q >> 1) * gridDim.x + blockIdx.x) * 2 + (q & 1)] = t;
  }
}

// Deterministic test vector: x[i] = (sin(0.618 i), cos(0.377 i + 1)).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_fill_probe(int64_t n, typename CT<R>::T* x) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    x[i] = typename CT<R>::T{static_cast<R>(sin(0.618 * (double)i)), static_cast<R>(cos(0.377 * (double)i + 1.0))};
}

// out[s * out_stride + q] = sum over r < rows of part[s * set_stride + r * cols + q]
// for q < cols, one workgroup per set s (fixed order).
__global__ __launch_bounds__(kBlock) void k_reduce_sets(const double* part, int64_t set_stride, int rows, int cols,
                                                        double* out, int64_t out_stride) {
  __shared__ double red[kWaves];
  const double* P = part + (int64_t)blockIdx.x * set_stride;
  for (int q = 0; q < cols; ++q) {
    const double s = reduce_column(P, rows, cols, q, red);
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * out_stride + q] = s;
  }
}

// --------------------- CGS2 re-orthogonalisation ---------------------------
// One classical Gram-Schmidt pass of w = u_{j+1} against the Krylov vectors
// v_k = s_k u_k, k = 0..j (FP64 coefficients):  w <- w - sum_k v_k <v_k, w>.
// Three kernels: partial inner products, their fixed-order reduction into
// coefficients s_k^2 <u_k, w>, and the subtraction with |w|^2 partials.
// All exit at once after the step's decision.
constexpr int kReorthK = 4;  // inner products accumulated per pass over w

template <typename R, int NV>
__global__ __launch_bounds__(kBlock) void k_reorth_dot(int64_t n, void* const* slots, int j, const StepCtl* ctl,
                                                       double* partials) {
  using V = typename CT<R>::T;
  __shared__ double red[kWaves * 2 * kReorthK * kMaxNV];
  if (ctl->all_done) return;
  const V* w = static_cast<const V*>(slots[j + 1]);
  const int64_t total = n * NV;
  const int tid = threadIdx.x;
  for (int kb = 0; kb <= j; kb += kReorthK) {
    const int kn = min(kReorthK, j + 1 - kb);
    double acc[2 * kReorthK];
#pragma unroll
    for (int q = 0; q < 2 * kReorthK; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + tid; i < total; i += (int64_t)gridDim.x * kBlock) {
      const V x = w[i];
#pragma unroll
      for (int q = 0; q < kReorthK; ++q) {
        if (q < kn) {
          const V u = static_cast<const V*>(slots[kb + q])[i];
          acc[2 * q] += (double)u.x * x.x + (double)u.y * x.y;      // conj(u) w
          acc[2 * q + 1] += (double)u.x * x.y - (double)u.y * x.x;
        }
      }
    }
    block_partials<NV>(acc, 2 * kn, red, partials + ((size_t)blockIdx.x * (j + 1) * 2 + 2 * kb) * NV);
  }
}

template <int NV>
__global__ __launch_bounds__(kBlock) void k_reorth_coef(const double* partials, int nrows, int j, const VecState* st,
                                                        const StepCtl* ctl, double* coef) {
  __shared__ double red[kWaves];
  if (ctl->all_done) return;
  const int ncols = (j + 1) * 2 * NV;  // column (k * 2 + c) * NV + v
  for (int t = 0; t < ncols; ++t) {
    const double s = reduce_column(partials, nrows, ncols, t, red);
    if (threadIdx.x == 0) {
      const int v = t % NV, c = (t / NV) % 2, k = t / (2 * NV);
      const double sc = st[v].scale[k];
      coef[(k * NV + v) * 2 + c] = s * sc * sc;
    }
  }
}

template <typename R, int NV>
__global__ __launch_bounds__(kBlock) void k_reorth_axpy(int64_t n, void* const* slots, int j, const double* coef,
                                                        const StepCtl* ctl, double* partials) {
  using V = typename CT<R>::T;
  __shared__ double red[kWaves * kMaxNV];
  __shared__ double cr[kMMax + 1][kMaxNV], ci[kMMax + 1][kMaxNV];
  if (ctl->all_done) return;
  const int tid = threadIdx.x;
  for (int t = tid; t < (j + 1) * NV; t += kBlock) {
    cr[t / NV][t % NV] = coef[2 * t];
    ci[t / NV][t % NV] = coef[2 * t + 1];
  }
  __syncthreads();
  V* w = static_cast<V*>(slots[j + 1]);
  const int v = tid % NV;
  const int64_t total = n * NV;
  double n2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + tid; i < total; i += (int64_t)gridDim.x * kBlock) {
    const V x = w[i];
    double ar = x.x, ai = x.y;
    for (int k = 0; k <= j; ++k) {
      const V u = static_cast<const V*>(slots[k])[i];
      ar -= cr[k][v] * u.x - ci[k][v] * u.y;
      ai -= cr[k][v] * u.y + ci[k][v] * u.x;
    }
    const V o = V{static_cast<R>(ar), static_cast<R>(ai)};
    w[i] = o;
    n2 += (double)o.x * o.x + (double)o.y * o.y;
  }
  block_partials<NV>(&n2, 1, red, partials + (size_t)blockIdx.x * NV);
}

// ------------------- broadened spectral functions ---------------------------
// A(nu) = (1/pi) Re sum_k w_k e^{-eps s_k} e^{i nu s_k} z_k on s_k = k dt with
// trapezoidal weights, z = conj(o) for removal (lesser) members and z = o for
// addition (greater) members; one thread per (member, frequency), FP64.
__global__ __launch_bounds__(kBlock) void k_spectral(int n_s, const double2* __restrict__ o,
                                                     unsigned long long lesser_mask, double dt, double eps,
                                                     int n_nu, const double* __restrict__ nu,
                                                     double* __restrict__ out) {
  const int f = blockIdx.x * kBlock + threadIdx.x;
  const int m = blockIdx.y;
  if (f >= n_nu) return;
  const double w = nu[f];
  const double cj = ((lesser_mask >> m) & 1ull) ? -1.0 : 1.0;
  const double2* om = o + (size_t)m * n_s;
  double acc = 0.0;
  for (int k = 0; k < n_s; ++k) {
    const double s = k * dt;
    const double wt = (k == 0 || k == n_s - 1) ? 0.5 * dt : dt;
    double sn, cs;
    sincos(w * s, &sn, &cs);
    const double2 z = om[k];
    acc += wt * exp(-eps * s) * (cs * z.x - sn * (cj * z.y));
  }
  out[(size_t)m * n_nu + f] = n_s > 1 ? acc / M_PI : 0.0;
}

// ------------------------------- BLAS-1 ------------------------------------
// <v_k, w> partials for k < kv: workgroup column blockIdx.y takes the chunk
// of (up to) 8 vectors k0 = 8 blockIdx.y.., each in registers; partials
// [gridDim.x][2 kv].
__global__ __launch_bounds__(kBlock) void k_multidot(int64_t n, const double2* const* vecs, int kv,
                                                     const double2* w, double* partials) {
  __shared__ double red[kWaves * 16];
  const int k0 = blockIdx.y * 8;
  const int K = min(8, kv - k0);
  const double2* vp[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) vp[k] = k < K ? vecs[k0 + k] : nullptr;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double2 b = w[i];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k < K) {
        const double2 a = vp[k][i];
        acc[2 * k] += a.x * b.x + a.y * b.y;  // conj(a) * b
        acc[2 * k + 1] += a.x * b.y - a.y * b.x;
      }
    }
  }
  // workgroup sums (fixed order), 2 K values for this chunk
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == 0) red[wv * 16 + q] = t;
  }
  __syncthreads();
  if (threadIdx.x < 2 * K) {
    double t = 0.0;
    for (int k = 0; k < kWaves; ++k) t += red[k * 16 + threadIdx.x];
    partials[(size_t)blockIdx.x * 2 * kv + 2 * k0 + threadIdx.x] = t;
  }
}

__global__ void k_multiaxpy(int64_t n, const double2* const* vecs, int kv, const double2* coef, double2* w) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double2 t = w[i];
    for (int k = 0; k < kv; ++k) {
      const double2 a = vecs[k][i];
      const double2 c = coef[k];
      t.x -= c.x * a.x - c.y * a.y;
      t.y -= c.x * a.y + c.y * a.x;
    }
    w[i] = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_norm2(int64_t n, const double2* w, double* partials) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double2 t = w[i];
    s += t.x * t.x + t.y * t.y;
  }
  block_partials<1>(&s, 1, red, partials + blockIdx.x);
}

__global__ void k_scale(int64_t n, double2* w, const double* inv_from, double2 f) {
  double2 c = f;
  if (inv_from) {
    const double nn = sqrt(*inv_from);
    c = double2{nn > 0.0 ? 1.0 / nn : 0.0, 0.0};
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 t = w[i];
    w[i] = double2{c.x * t.x - c.y * t.y, c.x * t.y + c.y * t.x};
  }
}

__global__ __launch_bounds__(kBlock) void k_absmax(int64_t n, const double2* w, double* partials) {
  __shared__ double red[kWaves];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double2 t = w[i];
    m = fmax(m, t.x * t.x + t.y * t.y);
  }
  m = wave_max(m);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int k = 0; k < kWaves; ++k) r = fmax(r, red[k]);
    partials[blockIdx.x] = r;
  }
}

__global__ __launch_bounds__(kBlock) void k_first_above(int64_t n, const double2* w, const double* thresh,
                                                        int64_t* partials) {
  __shared__ int64_t red[kBlock];
  const double th = *thresh;
  int64_t best = n;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double2 t = w[i];
    if (t.x * t.x + t.y * t.y >= th) {
      best = i;
      break;
    }
  }
  red[threadIdx.x] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t r = n;
    for (int k = 0; k < kBlock; ++k) r = red[k] < r ? red[k] : r;
    partials[blockIdx.x] = r;
  }
}

__global__ void k_first_final(const int64_t* partials, int nrows, int64_t n, int64_t* out) {
  if (threadIdx.x == 0) {
    int64_t r = n;
    for (int b = 0; b < nrows; ++b) r = partials[b] < r ? partials[b] : r;
    *out = r;
  }
}

}  // namespace dev
using namespace dev;

hipError_t launch_apply_c128(const ApplyLaunch& L, int grid, size_t lds, int* pgrid);
hipError_t launch_apply_c64(const ApplyLaunch& L, int grid, size_t lds, int* pgrid);
hipError_t launch_block_c128(const ApplyLaunch& L, int* pgrid);
hipError_t launch_block_c64(const ApplyLaunch& L, int* pgrid);

int elem_grid(int64_t n) {
  // four workgroups per CU at most (16 waves) for these memory-bound passes;
  // every Lanczos apply workgroup sums the partials they leave
  const int64_t g = (n + 4 * kBlock - 1) / (4 * kBlock);
  return static_cast<int>(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

int apply_chunks(const DevBasis& db, int prec, int nv) {
  // Several column chunks per row would keep more up-hop gathers in flight
  // (measured: at most ~15% faster for plain applies at 12 sites, and slower
  // inside the Lanczos loop, whose first phase sums the previous kernel's
  // partials in every workgroup) -- one chunk per row.  The fused Lanczos row
  // pass requires one chunk (it updates and sums whole rows); its launcher
  // refuses anything else.
  (void)db;
  (void)prec;
  (void)nv;
  return 1;
}

// Column block of the column pass: kColW columns, staged as +x and -x, or as
// +x alone (sign from the stage index) when two copies do not fit; 2 columns
// of one copy when 4 do not fit either.
static size_t colpass_copy_bytes(const DevBasis& db, int prec, int w) {
  return (static_cast<size_t>(db.dim_up) + 1) * w * (prec == 0 ? 16 : 8);
}
int colpass_width(const DevBasis& db, int prec) {
  return colpass_copy_bytes(db, prec, kColW) <= 150 * 1024 ? kColW : 2;
}
bool colpass_single(const DevBasis& db, int prec) {
  return 2 * colpass_copy_bytes(db, prec, colpass_width(db, prec)) > 150 * 1024;
}
int colpass_grid(const DevBasis& db, int prec) {
  const int w = colpass_width(db, prec);
  return (db.dim_dn + w - 1) / w;
}

size_t colpass_lds_bytes(const DevBasis& db, int prec) {
  const size_t copy = colpass_copy_bytes(db, prec, colpass_width(db, prec));
  return colpass_single(db, prec) ? copy : 2 * copy;
}

bool apply_global_rows(const DevBasis& db, int prec, int nv) {
  return nv == 1 && apply_lds_bytes(db, prec, 1, 1) > 150 * 1024;
}

bool apply_two_pass(const DevBasis& db, int prec, int nv, int mode, bool obs) {
  if (nv != 1 || !(mode == kPlain || mode == kLanczos) || db.two_pass == 0 || !db.up_tab) return false;
  if (obs && mode != kLanczos) return false;
  if (colpass_lds_bytes(db, prec) > 150 * 1024) return false;
  if (db.two_pass == 1) return true;
  if (db.tuned_single[prec] >= 0) return db.tuned_single[prec] == 1;
  // automatic: when a vector is larger than one XCD's L2 the up-hop row
  // gathers of the one-pass kernel stream from the Infinity Cache.  With 2
  // staged columns (complex128, 14 sites) only the Lanczos iterations gain
  // (fused updates); a plain apply stays faster in one pass (263 vs 306 us,
  // while complex64's 4 single-copy columns take 151 instead of 213 us).
  if (mode == kPlain && colpass_width(db, prec) < kColW) return false;
  return static_cast<double>(db.dim) * (prec == 0 ? 16 : 8) >= 4.0 * 1024 * 1024;
}

int apply_grid(const DevBasis& db, int prec, int nv) {
  return std::max({db.dim_up * apply_chunks(db, prec, nv), colpass_grid(db, prec), db.dim_dn});
}

static bool block_slots_ok(int g) { return g == 8 || g == 12 || g == 16 || g == 20 || g == 24; }

size_t block_lds_bytes(const DevBasis& db, int prec, int nv) {
  const size_t es = prec == 0 ? 16 : 8;
  return (static_cast<size_t>(std::max(db.dim_up, db.dim_dn)) + 1) * nv * es;
}

bool block_two_pass(const DevBasis& db, int prec, int nv) {
  if (!(nv == 2 || nv == 4 || nv == 8) || db.block_path == 0 || !db.dn_tabg || !db.up_tabg) return false;
  const int gi = nv == 2 ? 1 : (nv == 4 ? 2 : 3);
  if (db.block_path == -1 && db.tuned_block[prec][gi] == 0) return false;
  if (!block_slots_ok(db.dn_gslots) || !block_slots_ok(db.up_gslots)) return false;
  return block_lds_bytes(db, prec, nv) <= 150 * 1024;
}

int apply_nq_two_pass(bool obs) { return obs ? 2 : 1; }  // column pass: alpha [, up-hop obs part]

int apply_nq(int mode, bool obs, int nc) {
  const bool kL = mode == kLanczos;
  const bool kO = mode == kObsOnly || (kL && obs);
  (void)nc;
  return (kL ? 1 : 0) + (kO ? kObsQ : 0);
}

size_t apply_lds_bytes(const DevBasis& db, int prec, int nv, int rows) {
  (void)rows;
  const size_t elem = prec == 0 ? 16 : 8;
  return 2 * (static_cast<size_t>(db.dim_dn) + 1) * nv * elem;  // +x and -x copies with zero slots
}

bool apply_fits(const DevBasis& db, int prec, int nv) {
  return nv == 1 || apply_lds_bytes(db, prec, nv, 1) <= 150 * 1024;
}

hipError_t launch_apply(const ApplyLaunch& L, int* grid_out) {
  if (L.nv > 1 && L.mode != kObsOnly && block_two_pass(*L.db, L.prec, L.nv)) {
    int pgrid = 0;
    const hipError_t e = L.prec == 0 ? launch_block_c128(L, &pgrid) : launch_block_c64(L, &pgrid);
    if (grid_out) *grid_out = pgrid;
    return e;
  }
  const int grid = L.db->dim_up * apply_chunks(*L.db, L.prec, L.nv);
  int pgrid = grid;
  const size_t lds = apply_lds_bytes(*L.db, L.prec, L.nv, L.rows);
  const hipError_t e = L.prec == 0 ? launch_apply_c128(L, grid, lds, &pgrid) : launch_apply_c64(L, grid, lds, &pgrid);
  if (grid_out) *grid_out = pgrid;
  return e;
}

#define HUB_NV_SWITCH(nv, CALL)                         \
  switch (nv) {                                         \
    case 1: { constexpr int NVC = 1; CALL; } break;     \
    case 2: { constexpr int NVC = 2; CALL; } break;     \
    case 4: { constexpr int NVC = 4; CALL; } break;     \
    case 8: { constexpr int NVC = 8; CALL; } break;     \
    default: return hipErrorInvalidValue;               \
  }

hipError_t launch_reorth(int prec, int nv, int64_t n, void* const* slots_dev, int j, const VecState* st,
                         const StepCtl* ctl, double* dot_partials, double* coef, double* norm_partials,
                         hipStream_t s) {
  const int grid = elem_grid(n * nv);
  if (prec == 0) {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_reorth_dot<double, NVC>), dim3(grid), dim3(kBlock), 0, s, n, slots_dev,
                                         j, ctl, dot_partials));
  } else {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_reorth_dot<float, NVC>), dim3(grid), dim3(kBlock), 0, s, n, slots_dev,
                                         j, ctl, dot_partials));
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_reorth_coef<NVC>), dim3(1), dim3(kBlock), 0, s, dot_partials, grid, j, st,
                                       ctl, coef));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (prec == 0) {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_reorth_axpy<double, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         slots_dev, j, coef, ctl, norm_partials));
  } else {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_reorth_axpy<float, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         slots_dev, j, coef, ctl, norm_partials));
  }
  return hipGetLastError();
}

hipError_t launch_spectral(int n_members, int n_s, const void* overlaps, const int32_t* lesser, double dt, double eps,
                           int n_nu, const double* nu, double* out, hipStream_t s) {
  for (int m0 = 0; m0 < n_members; m0 += 64) {
    const int mc = std::min(64, n_members - m0);
    unsigned long long mask = 0;
    for (int k = 0; k < mc; ++k)
      if (lesser[m0 + k]) mask |= 1ull << k;
    const dim3 grid((n_nu + kBlock - 1) / kBlock, mc);
    hipLaunchKernelGGL(k_spectral, grid, dim3(kBlock), 0, s, n_s,
                       static_cast<const double2*>(overlaps) + static_cast<size_t>(m0) * n_s, mask, dt, eps, n_nu,
                       nu, out + static_cast<size_t>(m0) * n_nu);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_update(int prec, int nv, int64_t n, void* w, const void* uj, VecState* st, StepCtl* ctl, int j,
                         const double* apply_partials, int apply_nblk, int apply_nq, const double* row_obs,
                         int row_nblk, double* partials, hipStream_t s) {
  const int grid = elem_grid(n * nv);
  if (prec == 0) {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_update<double, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         static_cast<double2*>(w), static_cast<const double2*>(uj), st, ctl, j,
                                         apply_partials, apply_nblk, apply_nq, row_obs, row_nblk, partials));
  } else {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_update<float, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         static_cast<float2*>(w), static_cast<const float2*>(uj), st, ctl, j,
                                         apply_partials, apply_nblk, apply_nq, row_obs, row_nblk, partials));
  }
  return hipGetLastError();
}

hipError_t launch_combine(int prec, int nv, int64_t n, void* const* slots_dev, const VecState* st,
                          StepCtl* ctl, double* partials, int seq, CombineLog* log, double* obs_log, int nobs,
                          hipStream_t s, void* copy_to) {
  const int grid = elem_grid(n * nv);
  if (prec == 0) {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_combine<double, NVC>), dim3(grid), dim3(kBlock), 0, s, n, slots_dev,
                                         st, ctl, partials, seq, log, obs_log, nobs, copy_to));
  } else {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_combine<float, NVC>), dim3(grid), dim3(kBlock), 0, s, n, slots_dev,
                                         st, ctl, partials, seq, log, obs_log, nobs, copy_to));
  }
  return hipGetLastError();
}

hipError_t launch_overlaps(int prec, int nv, const OverlapArgs& a, hipStream_t s) {
  const int grid = overlap_grid(a.n_t);
  if (prec == 0) {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_overlaps<double, NVC>), dim3(grid), dim3(kBlock), 0, s, a));
  } else {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_overlaps<float, NVC>), dim3(grid), dim3(kBlock), 0, s, a));
  }
  return hipGetLastError();
}

hipError_t launch_reduce_sets(const double* part, int64_t set_stride, int n_sets, int rows, int cols, double* out,
                              int64_t out_stride, hipStream_t s) {
  if (n_sets < 1) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_sets, dim3(n_sets), dim3(kBlock), 0, s, part, set_stride, rows, cols, out, out_stride);
  return hipGetLastError();
}

hipError_t launch_fill_probe(int prec, int64_t n, void* x, hipStream_t s) {
  const int grid = elem_grid(n);
  if (prec == 0) hipLaunchKernelGGL(k_fill_probe<double>, dim3(grid), dim3(kBlock), 0, s, n, static_cast<double2*>(x));
  else hipLaunchKernelGGL(k_fill_probe<float>, dim3(grid), dim3(kBlock), 0, s, n, static_cast<float2*>(x));
  return hipGetLastError();
}

int overlap_grid(int64_t n_t) {
  const int64_t g = (n_t + 4 * kBlock - 1) / (4 * kBlock);
  return static_cast<int>(g < 1 ? 1 : (g > 256 ? 256 : g));
}

hipError_t launch_step_log(int nv, const VecState* st, StepCtl* ctl, void* log, double* obs_log, int nobs,
                           hipStream_t s) {
  HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_step_log<NVC>), dim3(1), dim3(64), 0, s, st, ctl,
                                       static_cast<CombineLog*>(log), obs_log, nobs));
  return hipGetLastError();
}

hipError_t launch_step_begin(int prec, int nv, int64_t n, const void* v, VecState* st, StepCtl* ctl, double tau,
                             bool norm, double* partials, hipStream_t s) {
  const int grid = elem_grid(n * nv);
  if (prec == 0) {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_step_begin<double, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         static_cast<const double2*>(v), st, ctl, tau, norm ? 1 : 0, partials));
  } else {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_step_begin<float, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         static_cast<const float2*>(v), st, ctl, tau, norm ? 1 : 0, partials));
  }
  return hipGetLastError();
}

hipError_t launch_finalize_obs(int nv, const double* partials, int nrows, int nq, VecState* st, hipStream_t s) {
  HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_finalize_obs<NVC>), dim3(1), dim3(kBlock), 0, s, partials, nrows, nq, st));
  return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int nrows, int ncols, double* out, int op, hipStream_t s) {
  if (ncols < 1) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(ncols), dim3(kBlock), 0, s, partials, nrows, ncols, out, op);
  return hipGetLastError();
}

hipError_t launch_interleave(int prec, int nv, int64_t n, const void* src, void* dst, bool to_block,
                             hipStream_t s) {
  const int grid = elem_grid(n * nv);
  if (prec == 0)
    hipLaunchKernelGGL(k_interleave<double>, dim3(grid), dim3(kBlock), 0, s, n, nv,
                       static_cast<const double2*>(src), static_cast<double2*>(dst), to_block ? 1 : 0);
  else
    hipLaunchKernelGGL(k_interleave<float>, dim3(grid), dim3(kBlock), 0, s, n, nv,
                       static_cast<const float2*>(src), static_cast<float2*>(dst), to_block ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_site_docc(int prec, const DevBasis& db, const void* x, double* out, double* partials,
                            hipStream_t s) {
  const int grid = elem_grid(db.dim);
  if (prec == 0)
    hipLaunchKernelGGL(k_site_docc<double>, dim3(grid), dim3(kBlock), 0, s, db.dim_up, db.dim_dn, db.n_sites,
                       db.up_bits, db.dn_bits, static_cast<const double2*>(x), partials);
  else
    hipLaunchKernelGGL(k_site_docc<float>, dim3(grid), dim3(kBlock), 0, s, db.dim_up, db.dim_dn, db.n_sites,
                       db.up_bits, db.dn_bits, static_cast<const float2*>(x), partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(partials, grid, db.n_sites, out, 0, s);
}

hipError_t launch_cop(int prec, int64_t n_t, int dim_dn_t, int dim_dn_s, int64_t n_s, int nvec, bool down,
                      const int32_t* map, const int8_t* sgn, const void* x, void* y, hipStream_t s) {
  const int grid = elem_grid(n_t * nvec) * 4;
  if (prec == 0)
    hipLaunchKernelGGL(k_cop<double>, dim3(grid), dim3(kBlock), 0, s, n_t, dim_dn_t, dim_dn_s, n_s, nvec,
                       down ? 1 : 0, map, sgn, static_cast<const double2*>(x), static_cast<double2*>(y));
  else
    hipLaunchKernelGGL(k_cop<float>, dim3(grid), dim3(kBlock), 0, s, n_t, dim_dn_t, dim_dn_s, n_s, nvec,
                       down ? 1 : 0, map, sgn, static_cast<const float2*>(x), static_cast<float2*>(y));
  return hipGetLastError();
}

hipError_t launch_dots(int prec, int64_t n, int nvec, const void* x, const void* y, double* out, double* partials,
                       hipStream_t s) {
  const int grid = elem_grid(n);
  if (prec == 0)
    hipLaunchKernelGGL(k_dots<double>, dim3(grid), dim3(kBlock), 0, s, n, nvec, static_cast<const double2*>(x),
                       static_cast<const double2*>(y), partials);
  else
    hipLaunchKernelGGL(k_dots<float>, dim3(grid), dim3(kBlock), 0, s, n, nvec, static_cast<const float2*>(x),
                       static_cast<const float2*>(y), partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(partials, grid, 2 * nvec, out, 0, s);
}

hipError_t launch_multidot(int64_t n, const double2* const* vecs, int k, const double2* w, double2* out,
                           double* partials, hipStream_t s) {
  if (k > 64) return hipErrorInvalidValue;
  const int grid = elem_grid(n);
  hipLaunchKernelGGL(k_multidot, dim3(grid, (k + 7) / 8), dim3(kBlock), 0, s, n, vecs, k, w, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(partials, grid, 2 * k, reinterpret_cast<double*>(out), 0, s);
}
hipError_t launch_multiaxpy(int64_t n, const double2* const* vecs, int k, const double2* coef, double2* w,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_multiaxpy, dim3(elem_grid(n)), dim3(kBlock), 0, s, n, vecs, k, coef, w);
  return hipGetLastError();
}
hipError_t launch_norm2(int64_t n, const double2* w, double* out, double* partials, hipStream_t s) {
  const int grid = elem_grid(n);
  hipLaunchKernelGGL(k_norm2, dim3(grid), dim3(kBlock), 0, s, n, w, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(partials, grid, 1, out, 0, s);
}
hipError_t launch_scale(int64_t n, double2* w, const double* inv_from, double2 factor, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(elem_grid(n)), dim3(kBlock), 0, s, n, w, inv_from, factor);
  return hipGetLastError();
}
hipError_t launch_absmax(int64_t n, const double2* w, double* out, double* partials, hipStream_t s) {
  const int grid = elem_grid(n);
  hipLaunchKernelGGL(k_absmax, dim3(grid), dim3(kBlock), 0, s, n, w, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(partials, grid, 1, out, 1, s);
}
hipError_t launch_first_above(int64_t n, const double2* w, const double* thresh, int64_t* out, int64_t* partials,
                              hipStream_t s) {
  const int grid = elem_grid(n);
  hipLaunchKernelGGL(k_first_above, dim3(grid), dim3(kBlock), 0, s, n, w, thresh, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_first_final, dim3(1), dim3(64), 0, s, partials, grid, n, out);
  return hipGetLastError();
}

}  // namespace hub
