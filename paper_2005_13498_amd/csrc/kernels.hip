// HIP kernels for gfx950 (CDNA4, wave64): matrix-free Peierls-Hubbard apply
// with fused Lanczos epilogue, Lanczos update + small exponential + stopping
// rule, Krylov combine, and BLAS-1 helpers.
//
// Reductions are deterministic: every workgroup writes its partial sums, and
// the last workgroup to finish (ticket counter) adds them in a fixed order.
#include "kernels.h"

#include <cmath>

namespace hub {
namespace {

template <typename R> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };

enum KMode : int { M_PLAIN = 0, M_LANCZOS = 1, M_LANCZOS_OBS = 2, M_OBS = 3 };

constexpr int kWaves = kBlock / 64;
constexpr int kRowsMax = 4;

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so that neighbouring rows of the tile
// share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  const int q = nblk >> 3, rem = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + min(x, rem) + k;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Sum of one value over the workgroup, identical on every thread, fixed order.
__device__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) r += lds[k];
  __syncthreads();
  return r;
}

// Reduce nq per-thread quantities, separately for each of the NV interleaved
// vectors (thread's vector = tid % NV), and store the workgroup's sums to
// out[q * NV + v].
template <int NV>
__device__ void block_partials(const double* vals, int nq, double* lds, double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int q = 0; q < nq; ++q) {
    double v = vals[q];
#pragma unroll
    for (int off = 32; off >= NV; off >>= 1) v += __shfl_xor(v, off);
    if (lane < NV) lds[(w * nq + q) * NV + lane] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nq * NV; t += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < kWaves; ++k) s += lds[k * nq * NV + t];
    out[t] = s;
  }
}

// Ticket: true on exactly one workgroup, the last to arrive.  The release
// fence before the ticket and the acquire fence after it make every other
// workgroup's partials visible to it.
__device__ bool last_block(uint32_t* ticket, unsigned nblk) {
  __shared__ bool is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = atomicAdd(ticket, 1u);
    is_last = (t == nblk - 1);
    if (is_last) atomicExch(ticket, 0u);
  }
  __syncthreads();
  if (is_last) __threadfence();
  return is_last;
}

// Fixed-order total of column t over nblk partial rows of width qn.
__device__ double reduce_column(const double* partials, int nblk, int qn, int t, double* lds) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += partials[(size_t)b * qn + t];
  return block_sum(s, lds);
}

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }

// ---------------------------------------------------------------------------
// Matrix-free H x on the [dim_up x dim_dn] tile (NV vectors interleaved per
// element): y[a,b] = (U popc(u_a & d_b) + e_a + e_b) x[a,b]
//   + sum_c coef_c ( sum_{up hops a'->a of class c} sgn x[a',b]
//                  + sum_{down hops b'->b of class c} sgn x[a,b'] ).
// A workgroup owns `rows` consecutive tile rows: it stages them in LDS (the
// down hops gather inside a row) and reads the up-hop source rows from
// global memory (a coalesced row read per hop; the hop list is uniform over
// the workgroup).
struct KArgs {
  int dim_up, dim_dn, nc, rows, j, nblk;
  double U;
  const uint32_t* up_bits;
  const uint32_t* dn_bits;
  const double* eps_up;
  const double* eps_dn;
  const int32_t* up_cls_ptr;
  const uint32_t* up_hops;
  const uint16_t* dn_tab;
  int slot_begin[kMaxClasses + 1];
  double coef[2 * kMaxNV * kMaxClasses];
  const void* x;
  void* y;
  const void* xprev;
  VecState* st;
  StepCtl* ctl;
  double* partials;
};

template <typename R, int NV, int MODE>
__global__ __launch_bounds__(kBlock) void k_apply(KArgs p) {
  using V = typename CT<R>::T;
  constexpr bool kL = (MODE == M_LANCZOS || MODE == M_LANCZOS_OBS);
  constexpr bool kO = (MODE == M_LANCZOS_OBS || MODE == M_OBS);
  constexpr bool kW = (MODE != M_OBS);
  __shared__ double red[kWaves * (1 + 3 + 2 * kMaxClasses) * kMaxNV];

  if (kL && p.ctl->all_done) return;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* xs = reinterpret_cast<V*>(smem_raw);
  const V* __restrict__ x = static_cast<const V*>(p.x);
  V* __restrict__ y = static_cast<V*>(p.y);

  const int nc = p.nc;
  const int rows = p.rows;
  const int rowlen = p.dim_dn * NV;          // complex elements of one tile row
  const int srow = rowlen + NV;              // staged row + zero slot
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int a0 = blk * rows;
  const int tid = threadIdx.x;
  const int v = tid % NV;

  // stage rows a0 .. a0+rows-1 (zero slot at index dim_dn)
  for (int r = 0; r < rows; ++r) {
    const int a = a0 + r;
    const V* src = x + (size_t)a * rowlen;
    for (int q = tid; q < srow; q += kBlock) {
      V val = V{0, 0};
      if (a < p.dim_up && q < rowlen) val = src[q];
      xs[r * srow + q] = val;
    }
  }
  uint32_t ua[kRowsMax];
  double ea[kRowsMax];
  bool rok[kRowsMax];
#pragma unroll
  for (int r = 0; r < kRowsMax; ++r) {
    const int a = a0 + r;
    rok[r] = (r < rows) && (a < p.dim_up);
    ua[r] = rok[r] ? p.up_bits[a] : 0u;
    ea[r] = (rok[r] && p.eps_up) ? p.eps_up[a] : 0.0;
  }
  // per-vector coefficients
  V cf[kMaxClasses];
#pragma unroll
  for (int c = 0; c < kMaxClasses; ++c) {
    if (c < nc) {
      cf[c].x = static_cast<R>(p.coef[2 * (v * nc + c)]);
      cf[c].y = static_cast<R>(p.coef[2 * (v * nc + c) + 1]);
    } else {
      cf[c] = V{0, 0};
    }
  }
  R sj = 1, bprev = 0;
  if (kL) {
    sj = static_cast<R>(p.st[v].scale[p.j]);
    if (p.j > 0) bprev = static_cast<R>(p.st[v].beta[p.j - 1] * p.st[v].scale[p.j - 1]);
  }
  __syncthreads();

  double q_alpha = 0.0;
  double q_diag = 0.0, q_docc = 0.0, q_n2 = 0.0;
  double q_pr[kMaxClasses], q_pi[kMaxClasses];
#pragma unroll
  for (int c = 0; c < kMaxClasses; ++c) { q_pr[c] = 0.0; q_pi[c] = 0.0; }

  for (int q = tid; q < rowlen; q += kBlock) {
    const int b = q / NV;
    const uint32_t db = p.dn_bits[b];
    const double eb = p.eps_dn ? p.eps_dn[b] : 0.0;
    V acc[kRowsMax], xv[kRowsMax];
#pragma unroll
    for (int r = 0; r < kRowsMax; ++r) {
      xv[r] = (r < rows) ? xs[r * srow + q] : V{0, 0};
      const double nd = static_cast<double>(__popc(ua[r] & db));
      const double dg = p.U * nd + ea[r] + eb;
      acc[r].x = static_cast<R>(dg) * xv[r].x;
      acc[r].y = static_cast<R>(dg) * xv[r].y;
      if (kO && rok[r]) {
        const double m2 = (double)xv[r].x * xv[r].x + (double)xv[r].y * xv[r].y;
        q_diag += dg * m2;
        q_docc += nd * m2;
        q_n2 += m2;
      }
    }
#pragma unroll
    for (int c = 0; c < kMaxClasses; ++c) {
      if (c < nc) {
        V S[kRowsMax];
#pragma unroll
        for (int r = 0; r < kRowsMax; ++r) S[r] = V{0, 0};
        // down hops: gather inside the staged rows
        for (int s = p.slot_begin[c]; s < p.slot_begin[c + 1]; ++s) {
          const uint32_t e = p.dn_tab[(size_t)s * p.dim_dn + b];
          const int off = static_cast<int>(e & 0x7FFFu) * NV + v;
          const bool neg = (e >> 15) != 0;
#pragma unroll
          for (int r = 0; r < kRowsMax; ++r) {
            if (r < rows) {
              const V t = xs[r * srow + off];
              S[r] = neg ? csub(S[r], t) : cadd(S[r], t);
            }
          }
        }
        // up hops: whole source rows from global memory
#pragma unroll
        for (int r = 0; r < kRowsMax; ++r) {
          if (rok[r]) {
            const int a = a0 + r;
            const int hb = p.up_cls_ptr[a * (nc + 1) + c];
            const int he = p.up_cls_ptr[a * (nc + 1) + c + 1];
            for (int h = hb; h < he; ++h) {
              const uint32_t e = p.up_hops[h];
              const V t = x[(size_t)(e & 0xFFFFu) * rowlen + q];
              S[r] = (e >> 31) ? csub(S[r], t) : cadd(S[r], t);
            }
          }
        }
#pragma unroll
        for (int r = 0; r < kRowsMax; ++r) {
          acc[r].x += cf[c].x * S[r].x - cf[c].y * S[r].y;
          acc[r].y += cf[c].x * S[r].y + cf[c].y * S[r].x;
          if (kO && rok[r]) {
            // <x | K_c x> contribution: conj(x) * S
            q_pr[c] += (double)xv[r].x * S[r].x + (double)xv[r].y * S[r].y;
            q_pi[c] += (double)xv[r].x * S[r].y - (double)xv[r].y * S[r].x;
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kRowsMax; ++r) {
      if (!rok[r]) continue;
      const size_t idx = (size_t)(a0 + r) * rowlen + q;
      V out = acc[r];
      if (kL) {
        out.x *= sj;
        out.y *= sj;
        if (p.j > 0) {
          const V pv = static_cast<const V*>(p.xprev)[idx];
          out.x -= bprev * pv.x;
          out.y -= bprev * pv.y;
        }
        // alpha_j = Re <s_j u_j, w>
        q_alpha += (double)sj * ((double)xv[r].x * out.x + (double)xv[r].y * out.y);
      }
      if (kW) y[idx] = out;
    }
  }

  // workgroup partials: [alpha] [diag, docc, n2, (Re, Im) P_c ...]
  const int nqL = kL ? 1 : 0;
  const int nqO = kO ? 3 + 2 * nc : 0;
  const int nq = nqL + nqO;
  if (nq == 0) return;
  double vals[1 + 3 + 2 * kMaxClasses];
  int k = 0;
  if (kL) vals[k++] = q_alpha;
  if (kO) {
    vals[k++] = q_diag;
    vals[k++] = q_docc;
    vals[k++] = q_n2;
#pragma unroll
    for (int c = 0; c < kMaxClasses; ++c) {
      if (c < nc) {
        vals[k++] = q_pr[c];
        vals[k++] = q_pi[c];
      }
    }
  }
  const int qn = nq * NV;
  block_partials<NV>(vals, nq, red, p.partials + (size_t)blk * qn);
  if (!last_block(&p.ctl->ticket[0], gridDim.x)) return;
  for (int t = 0; t < qn; ++t) {
    const double tot = reduce_column(p.partials, gridDim.x, qn, t, red);
    if (tid == 0) {
      const int qq = t / NV, vv = t % NV;
      if (kL && qq == 0) {
        if (p.st[vv].status == 0) p.st[vv].alpha[p.j] = tot;
      } else {
        p.st[vv].obs[qq - nqL] = tot;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// One wavefront: y = exp(-i tau T) e_1 for the j x j real symmetric
// tridiagonal T (diagonal alpha, off-diagonal beta).  Taylor series of the
// action on a vector with scaling, exp(-i tau T) = exp(-i (tau/s) T)^s,
// s chosen so that |tau/s| |T|_inf <= 1/2; the series of each factor is
// summed until a term is below 1e-18 of the partial sum.  Lane i holds
// component i (j <= 64).
__device__ void wave_small_expm(int j, const double* alpha, const double* beta, double tau,
                                int lane, double& yr, double& yi) {
  const double a = lane < j ? alpha[lane] : 0.0;
  const double bl = (lane >= 1 && lane < j) ? beta[lane - 1] : 0.0;
  const double bu = (lane + 1 < j) ? beta[lane] : 0.0;
  const double nrm = wave_max(fabs(a) + fabs(bl) + fabs(bu));
  const int s = max(1, static_cast<int>(ceil(fabs(tau) * nrm * 2.0)));
  const double h = tau / s;
  double zr = (lane == 0) ? 1.0 : 0.0, zi = 0.0;
  for (int sub = 0; sub < s; ++sub) {
    double tr = zr, ti = zi, sr = zr, si = zi;
    for (int k = 1; k <= 60; ++k) {
      const double tr_m = __shfl_up(tr, 1), ti_m = __shfl_up(ti, 1);
      const double tr_p = __shfl_down(tr, 1), ti_p = __shfl_down(ti, 1);
      const double ur = a * tr + bl * tr_m + bu * tr_p;
      const double ui = a * ti + bl * ti_m + bu * ti_p;
      const double f = h / k;
      tr = f * ui;   // (-i f) (ur + i ui) = f ui - i f ur
      ti = -f * ur;
      sr += tr;
      si += ti;
      const double tm = wave_max(fabs(tr) + fabs(ti));
      const double sm = wave_max(fabs(sr) + fabs(si));
      if (tm <= 1e-18 * sm) break;
    }
    zr = sr;
    zi = si;
  }
  yr = zr;
  yi = zi;
}

// u_{j+1} = w - alpha_j s_j u_j in place (w holds s_j H u_j - beta s u_{j-1});
// then in the last workgroup: beta_j = |u_{j+1}|, the small exponential of
// T_{j+1}, the a-posteriori estimate of Alg. 6 and the stopping decision.
template <typename R, int NV>
__global__ __launch_bounds__(kBlock) void k_update(int64_t n, typename CT<R>::T* w,
                                                   const typename CT<R>::T* uj, VecState* st,
                                                   StepCtl* ctl, int j, double* partials) {
  using V = typename CT<R>::T;
  __shared__ double red[kWaves * kMaxNV];
  if (ctl->all_done) return;
  const int tid = threadIdx.x;
  const int v = tid % NV;
  const R c = static_cast<R>(st[v].alpha[j] * st[v].scale[j]);
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
  if (!last_block(&ctl->ticket[1], gridDim.x)) return;
  __shared__ double tot[kMaxNV];
  for (int t = 0; t < NV; ++t) {
    const double s = reduce_column(partials, gridDim.x, NV, t, red);
    if (tid == 0) tot[t] = s;
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  const int m = j + 1;  // Krylov vectors u_0..u_j, T is m x m
  for (int vv = wv; vv < NV; vv += kWaves) {
    VecState& S = st[vv];
    if (S.status != 0) continue;
    const double beta = sqrt(tot[vv]);
    double yr, yi;
    wave_small_expm(m, S.alpha, S.beta, S.tau, lane, yr, yi);
    const double pr = (lane < m - 1) ? S.y[2 * lane] : 0.0;
    const double pi = (lane < m - 1) ? S.y[2 * lane + 1] : 0.0;
    const double d2 = wave_sum((yr - pr) * (yr - pr) + (yi - pi) * (yi - pi));
    const double y2 = wave_sum(yr * yr + yi * yi);
    const double ny = sqrt(y2);
    const double delta = sqrt(d2) / ny;
    const double eps = (delta < 1.0) ? fmin(1.0 + ny, delta / (1.0 - delta) * ny) : 1.0 + ny;
    if (lane < m) {
      S.y[2 * lane] = yr;
      S.y[2 * lane + 1] = yi;
    }
    if (lane == 0) {
      S.beta[j] = beta;
      S.eps = eps;
      S.m = m;
      int status = 0;
      if (beta < ctl->norm_inf * ctl->tol) status = 2;
      else if (eps < ctl->tol) status = 1;
      else if (m >= ctl->m_max) status = 3;
      S.status = status;
      S.scale[m] = (status == 0 && beta > 0.0) ? 1.0 / beta : 0.0;
    }
  }
  __syncthreads();
  if (tid == 0) {
    int done = 1, maxed = 0;
    for (int vv = 0; vv < NV; ++vv) {
      done &= (st[vv].status != 0);
      maxed |= (st[vv].status == 3);
    }
    ctl->all_done = done;
    ctl->any_maxed = maxed;
    ctl->iter = j + 1;
  }
}

// v <- beta0 sum_{k<m_v} s_k y_k u_k (into slot 0), |v|^2 for the next step;
// the last workgroup resets the per-step state and sets beta0 / scale[0].
template <typename R, int NV>
__global__ __launch_bounds__(kBlock) void k_combine(int64_t n, void* const* slots, VecState* st,
                                                    StepCtl* ctl, double* partials) {
  using V = typename CT<R>::T;
  __shared__ double red[kWaves * kMaxNV];
  __shared__ double cr[kMaxNV][kMMax], ci[kMaxNV][kMMax];
  __shared__ int mv[kMaxNV];
  const int tid = threadIdx.x;
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
    n2 += (double)o.x * o.x + (double)o.y * o.y;
  }
  block_partials<NV>(&n2, 1, red, partials + (size_t)blockIdx.x * NV);
  if (!last_block(&ctl->ticket[2], gridDim.x)) return;
  for (int t = 0; t < NV; ++t) {
    const double s = reduce_column(partials, gridDim.x, NV, t, red);
    if (tid == 0) {
      VecState& S = st[t];
      S.beta0 = sqrt(s);
      S.scale[0] = S.beta0 > 0.0 ? 1.0 / S.beta0 : 0.0;
    }
  }
}

// Records the finished step (into log) and resets the state for the next one.
template <int NV>
__global__ void k_step_log(VecState* st, StepCtl* ctl, CombineLog* log, double* obs_log, int nobs) {
  const int v = threadIdx.x;
  if (v < NV) {
    VecState& S = st[v];
    if (log) {
      log[v].m = S.m;
      log[v].status = S.status;
      log[v].eps = S.eps;
      log[v].beta_last = S.m > 0 ? S.beta[S.m - 1] : 0.0;
    }
    if (obs_log)
      for (int k = 0; k < nobs; ++k) obs_log[v * nobs + k] = S.obs[k];
    S.status = 0;
    S.m = 0;
    S.eps = 0.0;
  }
  if (v == 0) {
    ctl->all_done = 0;
    ctl->iter = 0;
  }
}

template <typename R, int NV>
__global__ __launch_bounds__(kBlock) void k_step_begin(int64_t n, const typename CT<R>::T* x,
                                                       VecState* st, StepCtl* ctl, double tau,
                                                       int norm_known, double* partials) {
  using V = typename CT<R>::T;
  __shared__ double red[kWaves * kMaxNV];
  const int tid = threadIdx.x;
  const int v = tid % NV;
  double n2 = 0.0;
  if (!norm_known) {
    const int64_t total = n * NV;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + tid; i < total; i += (int64_t)gridDim.x * kBlock) {
      const V t = x[i];
      n2 += (double)t.x * t.x + (double)t.y * t.y;
    }
  }
  block_partials<NV>(&n2, 1, red, partials + (size_t)blockIdx.x * NV);
  if (!last_block(&ctl->ticket[3], gridDim.x)) return;
  for (int t = 0; t < NV; ++t) {
    const double s = reduce_column(partials, gridDim.x, NV, t, red);
    if (tid == 0) {
      VecState& S = st[t];
      if (!norm_known) {
        S.beta0 = sqrt(s);
        S.scale[0] = S.beta0 > 0.0 ? 1.0 / S.beta0 : 0.0;
      }
      S.tau = tau;
      S.status = (S.beta0 > 0.0) ? 0 : 2;  // a zero vector stays zero
      S.m = (S.beta0 > 0.0) ? 0 : 1;
      S.eps = 0.0;
      S.y[0] = 1.0;
      S.y[1] = 0.0;
    }
  }
  __syncthreads();
  if (tid == 0) {
    int done = 1;
    for (int t = 0; t < NV; ++t) done &= (st[t].status != 0);
    ctl->all_done = done;
    ctl->any_maxed = 0;
    ctl->iter = 0;
  }
}

template <typename R>
__global__ void k_interleave(int64_t n, int nv, const typename CT<R>::T* src, typename CT<R>::T* dst,
                             int to_block) {
  const int64_t total = n * nv;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    // block layout index i = k*nv + v ; ABI layout index v*n + k
    const int64_t k = i / nv, v = i % nv;
    if (to_block) dst[i] = src[v * n + k];
    else dst[v * n + k] = src[i];
  }
}

// ------------------------------- BLAS-1 ------------------------------------
__global__ __launch_bounds__(kBlock) void k_multidot(int64_t n, const double2* const* vecs, int kv,
                                                     const double2* w, double2* out, double* partials,
                                                     uint32_t* ticket) {
  __shared__ double red[kWaves * 2 * 64];
  double acc[2 * 64];
  const int K = min(kv, 64);
  for (int k = 0; k < 2 * K; ++k) acc[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double2 b = w[i];
    for (int k = 0; k < K; ++k) {
      const double2 a = vecs[k][i];
      acc[2 * k] += a.x * b.x + a.y * b.y;      // conj(a) * b
      acc[2 * k + 1] += a.x * b.y - a.y * b.x;
    }
  }
  block_partials<1>(acc, 2 * K, red, partials + (size_t)blockIdx.x * 2 * K);
  if (!last_block(ticket, gridDim.x)) return;
  for (int t = 0; t < 2 * K; ++t) {
    const double s = reduce_column(partials, gridDim.x, 2 * K, t, red);
    if (threadIdx.x == 0) {
      if (t & 1) out[t / 2].y = s;
      else out[t / 2].x = s;
    }
  }
}

__global__ void k_multiaxpy(int64_t n, const double2* const* vecs, int kv, const double2* coef,
                            double2* w) {
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

__global__ __launch_bounds__(kBlock) void k_norm2(int64_t n, const double2* w, double* out,
                                                  double* partials, uint32_t* ticket) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double2 t = w[i];
    s += t.x * t.x + t.y * t.y;
  }
  block_partials<1>(&s, 1, red, partials + blockIdx.x);
  if (!last_block(ticket, gridDim.x)) return;
  const double tot = reduce_column(partials, gridDim.x, 1, 0, red);
  if (threadIdx.x == 0) *out = tot;
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

__global__ __launch_bounds__(kBlock) void k_absmax(int64_t n, const double2* w, double* out,
                                                   double* partials, uint32_t* ticket) {
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
  if (!last_block(ticket, gridDim.x)) return;
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b) r = fmax(r, partials[b]);
    *out = r;
  }
}

__global__ __launch_bounds__(kBlock) void k_first_above(int64_t n, const double2* w, const double* thresh,
                                                        int64_t* out, int64_t* partials, uint32_t* ticket) {
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
  if (!last_block(ticket, gridDim.x)) return;
  if (threadIdx.x == 0) {
    int64_t r = n;
    for (unsigned b = 0; b < gridDim.x; ++b) r = partials[b] < r ? partials[b] : r;
    *out = r;
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_site_docc(int dim_up, int dim_dn, int n_sites,
                                                      const uint32_t* up, const uint32_t* dn,
                                                      const typename CT<R>::T* x, double* out,
                                                      double* partials, uint32_t* ticket) {
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
  if (!last_block(ticket, gridDim.x)) return;
  for (int i = 0; i < n_sites; ++i) {
    const double s = reduce_column(partials, gridDim.x, n_sites, i, red);
    if (threadIdx.x == 0) out[i] = s;
  }
}

int grid_for(int64_t n) {
  const int64_t g = (n + kBlock - 1) / kBlock;
  return static_cast<int>(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

template <typename R, int NV, int MODE>
hipError_t apply_t(const ApplyLaunch& L, int grid, size_t lds) {
  const DevBasis& db = *L.db;
  KArgs p;
  p.dim_up = db.dim_up;
  p.dim_dn = db.dim_dn;
  p.nc = db.nc;
  p.rows = L.rows;
  p.j = L.j;
  p.nblk = grid;
  p.U = db.U;
  p.up_bits = db.up_bits;
  p.dn_bits = db.dn_bits;
  p.eps_up = db.eps_up;
  p.eps_dn = db.eps_dn;
  p.up_cls_ptr = db.up_cls_ptr;
  p.up_hops = db.up_hops;
  p.dn_tab = db.dn_tab;
  for (int c = 0; c <= kMaxClasses; ++c) p.slot_begin[c] = db.dn_slot_begin[c];
  for (int k = 0; k < 2 * kMaxNV * kMaxClasses; ++k) p.coef[k] = L.coef[k];
  p.x = L.x;
  p.y = L.y;
  p.xprev = L.xprev;
  p.st = L.st;
  p.ctl = L.ctl;
  p.partials = L.partials;
  auto fn = k_apply<R, NV, MODE>;
  // dynamic LDS above the 64 KB default must be opted into, up to the CU's
  // 160 KB minus the kernel's static LDS
  static int max_dyn = -1;
  if (max_dyn < 0) {
    hipFuncAttributes fa{};
    size_t stat = 0;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(fn)) == hipSuccess) stat = fa.sharedSizeBytes;
    const int want = 160 * 1024 - static_cast<int>(stat);
    max_dyn = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, want) == hipSuccess
                  ? want
                  : 64 * 1024 - static_cast<int>(stat);
    (void)hipGetLastError();  // do not report a refused opt-in as a launch error
  }
  if (lds > static_cast<size_t>(max_dyn)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), lds, L.stream, p);
  return hipGetLastError();
}

template <typename R, int NV>
hipError_t apply_mode(const ApplyLaunch& L, int grid, size_t lds) {
  if (L.mode == kPlain) return apply_t<R, NV, M_PLAIN>(L, grid, lds);
  if (L.mode == kObsOnly) return apply_t<R, NV, M_OBS>(L, grid, lds);
  if (L.obs) return apply_t<R, NV, M_LANCZOS_OBS>(L, grid, lds);
  return apply_t<R, NV, M_LANCZOS>(L, grid, lds);
}

template <typename R>
hipError_t apply_nv(const ApplyLaunch& L, int grid, size_t lds) {
  switch (L.nv) {
    case 1: return apply_mode<R, 1>(L, grid, lds);
    case 2: return apply_mode<R, 2>(L, grid, lds);
    case 4: return apply_mode<R, 4>(L, grid, lds);
    case 8: return apply_mode<R, 8>(L, grid, lds);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int apply_grid(const DevBasis& db, int rows) { return (db.dim_up + rows - 1) / rows; }

size_t apply_lds_bytes(const DevBasis& db, int prec, int nv, int rows) {
  const size_t elem = prec == 0 ? 16 : 8;
  return static_cast<size_t>(rows) * (static_cast<size_t>(db.dim_dn) + 1) * nv * elem;
}

hipError_t launch_apply(const ApplyLaunch& L, int* grid_out) {
  if (L.rows < 1 || L.rows > kRowsMax) return hipErrorInvalidValue;
  const int grid = apply_grid(*L.db, L.rows);
  if (grid_out) *grid_out = grid;
  const size_t lds = apply_lds_bytes(*L.db, L.prec, L.nv, L.rows);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  return L.prec == 0 ? apply_nv<double>(L, grid, lds) : apply_nv<float>(L, grid, lds);
}

#define HUB_NV_SWITCH(nv, CALL)                 \
  switch (nv) {                                 \
    case 1: { constexpr int NVC = 1; CALL; } break; \
    case 2: { constexpr int NVC = 2; CALL; } break; \
    case 4: { constexpr int NVC = 4; CALL; } break; \
    case 8: { constexpr int NVC = 8; CALL; } break; \
    default: return hipErrorInvalidValue;       \
  }

hipError_t launch_update(int prec, int nv, int64_t n, void* w, const void* uj, VecState* st,
                         StepCtl* ctl, int j, double* partials, hipStream_t s) {
  const int grid = grid_for(n * nv);
  if (prec == 0) {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_update<double, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         static_cast<double2*>(w), static_cast<const double2*>(uj), st,
                                         ctl, j, partials));
  } else {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_update<float, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         static_cast<float2*>(w), static_cast<const float2*>(uj), st,
                                         ctl, j, partials));
  }
  return hipGetLastError();
}

hipError_t launch_combine(int prec, int nv, int64_t n, void* const* slots_dev, VecState* st,
                          StepCtl* ctl, double* partials, hipStream_t s) {
  const int grid = grid_for(n * nv);
  if (prec == 0) {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_combine<double, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         slots_dev, st, ctl, partials));
  } else {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_combine<float, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         slots_dev, st, ctl, partials));
  }
  return hipGetLastError();
}

hipError_t launch_step_log(int nv, VecState* st, StepCtl* ctl, void* log, double* obs_log, int nobs,
                           hipStream_t s) {
  HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_step_log<NVC>), dim3(1), dim3(64), 0, s, st, ctl,
                                       static_cast<CombineLog*>(log), obs_log, nobs));
  return hipGetLastError();
}

hipError_t launch_step_begin(int prec, int nv, int64_t n, const void* v, VecState* st, StepCtl* ctl,
                             double tau, int m_max, double tol, double norm_inf, bool norm_known,
                             double* partials, hipStream_t s) {
  (void)m_max;
  (void)tol;
  (void)norm_inf;
  const int grid = norm_known ? 1 : grid_for(n * nv);
  if (prec == 0) {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_step_begin<double, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         static_cast<const double2*>(v), st, ctl, tau, norm_known ? 1 : 0,
                                         partials));
  } else {
    HUB_NV_SWITCH(nv, hipLaunchKernelGGL((k_step_begin<float, NVC>), dim3(grid), dim3(kBlock), 0, s, n,
                                         static_cast<const float2*>(v), st, ctl, tau, norm_known ? 1 : 0,
                                         partials));
  }
  return hipGetLastError();
}

hipError_t launch_interleave(int prec, int nv, int64_t n, const void* src, void* dst, bool to_block,
                             hipStream_t s) {
  const int grid = grid_for(n * nv);
  if (prec == 0)
    hipLaunchKernelGGL(k_interleave<double>, dim3(grid), dim3(kBlock), 0, s, n, nv,
                       static_cast<const double2*>(src), static_cast<double2*>(dst), to_block ? 1 : 0);
  else
    hipLaunchKernelGGL(k_interleave<float>, dim3(grid), dim3(kBlock), 0, s, n, nv,
                       static_cast<const float2*>(src), static_cast<float2*>(dst), to_block ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_site_docc(int prec, const DevBasis& db, const void* x, double* out, double* partials,
                            uint32_t* ticket, hipStream_t s) {
  const int grid = grid_for(db.dim);
  if (prec == 0)
    hipLaunchKernelGGL(k_site_docc<double>, dim3(grid), dim3(kBlock), 0, s, db.dim_up, db.dim_dn, db.n_sites,
                       db.up_bits, db.dn_bits, static_cast<const double2*>(x), out, partials, ticket);
  else
    hipLaunchKernelGGL(k_site_docc<float>, dim3(grid), dim3(kBlock), 0, s, db.dim_up, db.dim_dn, db.n_sites,
                       db.up_bits, db.dn_bits, static_cast<const float2*>(x), out, partials, ticket);
  return hipGetLastError();
}

hipError_t launch_multidot(int64_t n, const double2* const* vecs, int k, const double2* w, double2* out,
                           double* partials, uint32_t* ticket, hipStream_t s) {
  if (k > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_multidot, dim3(grid_for(n)), dim3(kBlock), 0, s, n, vecs, k, w, out, partials, ticket);
  return hipGetLastError();
}
hipError_t launch_multiaxpy(int64_t n, const double2* const* vecs, int k, const double2* coef, double2* w,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_multiaxpy, dim3(grid_for(n)), dim3(kBlock), 0, s, n, vecs, k, coef, w);
  return hipGetLastError();
}
hipError_t launch_norm2(int64_t n, const double2* w, double* out, double* partials, uint32_t* ticket,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_norm2, dim3(grid_for(n)), dim3(kBlock), 0, s, n, w, out, partials, ticket);
  return hipGetLastError();
}
hipError_t launch_scale(int64_t n, double2* w, const double* inv_from, double2 factor, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kBlock), 0, s, n, w, inv_from, factor);
  return hipGetLastError();
}
hipError_t launch_absmax(int64_t n, const double2* w, double* out, double* partials, uint32_t* ticket,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_absmax, dim3(grid_for(n)), dim3(kBlock), 0, s, n, w, out, partials, ticket);
  return hipGetLastError();
}
hipError_t launch_first_above(int64_t n, const double2* w, const double* thresh, int64_t* out,
                              int64_t* partials, uint32_t* ticket, hipStream_t s) {
  hipLaunchKernelGGL(k_first_above, dim3(grid_for(n)), dim3(kBlock), 0, s, n, w, thresh, out, partials, ticket);
  return hipGetLastError();
}

}  // namespace hub
