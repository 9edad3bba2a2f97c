// Device helpers shared by the HIP translation units of the library.
#pragma once

#include <cmath>

#include <hip/hip_ext.h>

#include "kernels.h"

namespace hub {
namespace dev {


template <typename R> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };

enum KMode : int { M_PLAIN = 0, M_LANCZOS = 1, M_LANCZOS_OBS = 2, M_OBS = 3 };

constexpr int kWaves = kBlock / 64;

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks (tile rows with the same high-site
// occupation, whose up hops mostly stay inside the range) so they share an L2.
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

// Sum over the workgroup (W waves), identical on every thread, fixed order.
template <int W = kWaves>
__device__ inline double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < W; ++k) r += lds[k];
  __syncthreads();
  return r;
}

// Reduce nq per-thread quantities separately for each of the NV interleaved
// vectors (thread's vector = tid % NV) and store the workgroup's sums at
// out[q * NV + v].
template <int NV, int W = kWaves>
__device__ void block_partials(const double* vals, int nq, double* lds, double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  for (int q = 0; q < nq; ++q) {
    double v = vals[q];
#pragma unroll
    for (int off = 32; off >= NV; off >>= 1) v += __shfl_xor(v, off);
    if (lane < NV) lds[(w * nq + q) * NV + lane] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nq * NV; t += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < W; ++k) s += lds[k * nq * NV + t];
    out[t] = s;
  }
}

// Fixed-order total of column t of a [nrows][ncols] partial-sum array,
// identical on every thread of the workgroup.
template <int W = kWaves>
__device__ inline double reduce_column(const double* partials, int nrows, int ncols, int t, double* lds) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nrows; b += blockDim.x) s += partials[(size_t)b * ncols + t];
  return block_sum<W>(s, lds);
}

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
// acc + c s with the fused multiply-adds written out, so that every kernel
// rounds a given sequence of terms the same way (the one- and two-pass
// applies give bit-identical products whatever the compiler's contraction).
template <typename V> __device__ __forceinline__ V cfma(V c, V s, V acc) {
  return V{fma(-c.y, s.y, fma(c.x, s.x, acc.x)), fma(c.y, s.x, fma(c.x, s.y, acc.y))};
}

// ---------------------------------------------------------------------------
// x of lane i - 1 (wave_up) and of lane i + 1 (wave_down), zero past the
// wavefront's ends (every lane active): whole-wavefront DPP shifts by one
// lane, wave_shr:1 and wave_shl:1 with out-of-range lanes reading zero, so
// the neighbour exchange of a tridiagonal product costs no LDS permute.
__device__ __forceinline__ double wave_up(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_down(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x130, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// One wavefront: y = exp(-i tau T) e_1 for the j x j real symmetric
// tridiagonal T.  Taylor series of the action on a vector with scaling,
// exp(-i tau T) = exp(-i (tau/s) T)^s, s chosen so that |tau/s| |T|_inf <=
// 1/2; each factor's series is summed until a term falls below 1e-18 of the
// partial sum, tested every fourth term (the test's two wave-wide maxima cost
// more than a term).  Lane i holds row i of T (diagonal a, off-diagonals bl
// left and bu right of it; zero past j) and returns component i of y
// (j <= 64).  Every lane of the wavefront must be active.
__device__ inline void wave_small_expm(int j, double a, double bl, double bu, double tau, int lane, double& yr,
                                       double& yi) {
  const double nrm = wave_max(fabs(a) + fabs(bl) + fabs(bu));
  const int s = max(1, static_cast<int>(ceil(fabs(tau) * nrm * 2.0)));
  const double h = tau / s;
  double zr = (lane == 0) ? 1.0 : 0.0, zi = 0.0;
  for (int sub = 0; sub < s; ++sub) {
    double tr = zr, ti = zi, sr = zr, si = zi;
    for (int k = 1; k <= 60; ++k) {
      const double tr_m = wave_up(tr), ti_m = wave_up(ti);
      const double tr_p = wave_down(tr), ti_p = wave_down(ti);
      const double ur = a * tr + bl * tr_m + bu * tr_p;
      const double ui = a * ti + bl * ti_m + bu * ti_p;
      const double f = h / k;
      tr = f * ui;  // (-i f) (ur + i ui) = f ui - i f ur
      ti = -f * ur;
      sr += tr;
      si += ti;
      if ((k & 3) == 0 && wave_max(fabs(tr) + fabs(ti)) <= 1e-18 * wave_max(fabs(sr) + fabs(si))) break;
    }
    zr = sr;
    zi = si;
  }
  yr = zr;
  yi = zi;
}

// y^(j) = exp(-i tau T_j) e_1 (lane i: component i) and the estimate of
// Alg. 6 for m = j: delta = |y^(j) - y^(j-1)| / |y^(j)|, eps = min(1 + |y|,
// delta/(1-delta) |y|) (or 1 + |y| if delta >= 1).  a: alpha_i of lane i (the
// diagonal of T_j); beta: the off-diagonals beta_0..beta_{j-2}; yprev: y^(j-1)
// (j - 1 complex components).
__device__ inline double wave_krylov_eps(int j, double a, const double* beta, double tau, const double* yprev,
                                         int lane, double& yr, double& yi) {
  const double bl = (lane >= 1 && lane < j) ? beta[lane - 1] : 0.0;
  const double bu = (lane + 1 < j) ? beta[lane] : 0.0;
  wave_small_expm(j, a, bl, bu, tau, lane, yr, yi);
  const double pr = (lane < j - 1) ? yprev[2 * lane] : 0.0;
  const double pi = (lane < j - 1) ? yprev[2 * lane + 1] : 0.0;
  const double d2 = wave_sum((yr - pr) * (yr - pr) + (yi - pi) * (yi - pi));
  const double y2 = wave_sum(yr * yr + yi * yi);
  const double ny = sqrt(y2);
  const double delta = sqrt(d2) / ny;
  return (delta < 1.0) ? fmin(1.0 + ny, delta / (1.0 - delta) * ny) : 1.0 + ny;
}

// Krylov decision for Krylov dimension m = j (T_j complete: alpha[0..j-1],
// beta[0..j-2]; the new off-diagonal beta_{j-1} = beta_new[v]); for j == 0
// it starts the step (beta0 = beta_new).  One wave per vector; run by one
// workgroup.  Alg. 6: y^(j) = exp(-i tau T_j) e_1, delta = |y^(j) - y^(j-1)|
// / |y^(j)|, eps = min(1 + |y|, delta/(1-delta) |y|) (or 1 + |y| if
// delta >= 1); stop when eps < tol or beta_{j-1} < |H| tol.
template <int NV, int W = kWaves>
__device__ void krylov_decide(int j, const double* beta_new, VecState* st, StepCtl* ctl, int m_max, double tol,
                              double norm_inf) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int v = wv; v < NV; v += W) {
    VecState& S = st[v];
    const double b = beta_new[v];
    if (j == 0) {
      if (lane == 0) {
        // a zero vector stays zero; a NaN or infinite norm stops the run (status 4)
        const bool fin = isfinite(b);
        S.beta0 = b;
        S.scale[0] = (fin && b > 0.0) ? 1.0 / b : 0.0;
        S.status = !fin ? 4 : (b > 0.0 ? 0 : 2);
        S.m = (fin && b > 0.0) ? 0 : 1;
        S.eps = 0.0;
        S.y[0] = 1.0;
        S.y[1] = 0.0;
      }
      continue;
    }
    if (S.status != 0) continue;
    double yr, yi;
    // beta[j-1] is not part of T_j; store it after the exponential
    const double eps = wave_krylov_eps(j, lane < j ? S.alpha[lane] : 0.0, S.beta, S.tau, S.y, lane, yr, yi);
    if (lane < j) {
      S.y[2 * lane] = yr;
      S.y[2 * lane + 1] = yi;
    }
    if (lane == 0) {
      S.beta[j - 1] = b;
      S.eps = eps;
      S.m = j;
      int status = 0;
      if (!isfinite(b) || !isfinite(eps)) status = 4;  // NaN or Inf in the recurrence
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
      maxed |= (st[v].status >= 3);  // m_max, or a non-finite vector: the run stops
    }
    ctl->all_done = done;
    ctl->any_maxed = maxed;
    ctl->iter = j;
  }
}

// The end of a single vector's step at m = j, decided before |u_j| was
// known: an earlier kernel found the estimate for m = j below tol and
// recorded y^(j) and eps.  Records beta_{j-1} = b and the status as
// krylov_decide would (breakdown if b < |H| tol, else converged).  One thread.
__device__ inline void krylov_end_at(int j, double b, VecState& S, StepCtl* ctl, double tol, double norm_inf) {
  S.beta[j - 1] = b;
  S.m = j;
  S.status = !isfinite(b) ? 4 : (b < norm_inf * tol ? 2 : 1);
  S.scale[j] = 0.0;
  ctl->all_done = 1;
  ctl->any_maxed = S.status == 4;
  ctl->iter = j;
}

// Launch with optional timing events attached to the dispatch.
template <typename K, typename A>
hipError_t launch_ev(K fn, int grid, int blk, size_t lds, hipStream_t st, hipEvent_t e0, hipEvent_t e1, A& args) {
  if (!e0 && !e1) {
    hipLaunchKernelGGL(fn, dim3(grid), dim3(blk), lds, st, args);
    return hipGetLastError();
  }
  void* kargs[] = {&args};
  return hipExtLaunchKernel(reinterpret_cast<const void*>(fn), dim3(grid), dim3(blk), kargs, lds, st, e0, e1, 0);
}

// Opts kernel fn into the largest dynamic LDS a CU allows (160 KB minus its
// static LDS); returns the dynamic LDS bytes a launch may then request.
inline int dyn_lds_opt_in(const void* fn) {
  hipFuncAttributes fa{};
  size_t stat = 0;
  if (hipFuncGetAttributes(&fa, fn) == hipSuccess) stat = fa.sharedSizeBytes;
  const int want = 160 * 1024 - static_cast<int>(stat);
  const int got = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, want) == hipSuccess
                      ? want
                      : 64 * 1024 - static_cast<int>(stat);
  (void)hipGetLastError();  // a refused opt-in is not a launch error
  return got;
}

// ---------------------------------------------------------------------------
}  // namespace dev
}  // namespace hub
