// Resident stepper of small sectors: one launch runs every midpoint step
// (Eq. (time-stepping)) of a propagation, one workgroup per vector, with the
// whole tile of the vector resident in LDS and the Lanczos recurrence of
// Alg. 6 in registers.  Meant for sectors whose applies are far too short to
// fill the GPU one launch at a time (8 sites: 4,900 states, a 157 KB apply).
//
// Each thread owns up to EPT tile elements (wavefront 0 fewer where the tile
// leaves room, since it also evaluates the Krylov estimate).  The tile is
// staged once per Lanczos iteration as (dim_up + 1) x (dim_dn + 1) elements,
// each row followed by a zero and a zero row last, so that a down hop of
// element (a, b) reads row a and an up hop reads column b of the same array,
// both at an index that carries the fermion sign (src, src + dim + 1 for a
// negative sign, dim for padding), four slots of one class summed before the
// class coefficient is applied.  Iteration j (v_j = s_j u_j):
//   w_j = s_j H u_j - beta_{j-1} s_{j-1} u_{j-1}      (registers)
//   alpha_j = s_j Re <u_j, w_j>
//   u_{j+1} = w_j - alpha_j s_j u_j                   (registers -> LDS)
//   beta_j = |u_{j+1}|, the estimate for m = j + 1 (one wavefront), and the
//   decision of Alg. 6 as the launch path takes it.
// Only u_1 .. u_{m-1} go to memory, for the combine psi <- beta_0 sum_k y_k
// s_k u_k.  The observables of each step's input (Eqs. (docc), (energy)) are
// summed in FP64 from the first iteration's group sums with the coefficients
// of the sample time.
#include "kernels_common.h"
#include "resident.h"

namespace hub {
namespace dev {

namespace {

constexpr int kRT = kResidentThreads;
constexpr int kRW = kRT / 64;

// Signed sum of the four staged values one table word pair indexes; staged
// element q is at xs[q * stride], dim is the zero element.
template <typename V>
__device__ __forceinline__ V slot_sum4(uint2 w, const V* xs, uint32_t dim, int stride) {
  V s = V{0, 0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t w2 = k < 2 ? w.x : w.y;
    const uint32_t idx = (k & 1) ? (w2 >> 16) : (w2 & 0xFFFFu);
    const bool neg = idx > dim;
    const uint32_t src = neg ? idx - dim - 1u : idx;
    const V t = xs[static_cast<int>(src) * stride];
    s.x += neg ? -t.x : t.x;
    s.y += neg ? -t.y : t.y;
  }
  return s;
}

// The same over staged columns, skipping padding entries (index dim): the
// lanes of a wavefront mostly share the up string and so its padding, and a
// padding read of the zero row would cost a full-width LDS access.
template <typename V>
__device__ __forceinline__ V slot_sum4_skip(uint2 w, const V* xs, uint32_t dim, int stride) {
  V s = V{0, 0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t w2 = k < 2 ? w.x : w.y;
    const uint32_t idx = (k & 1) ? (w2 >> 16) : (w2 & 0xFFFFu);
    if (idx == dim) continue;
    const bool neg = idx > dim;
    const uint32_t src = neg ? idx - dim - 1u : idx;
    const V t = xs[static_cast<int>(src) * stride];
    s.x += neg ? -t.x : t.x;
    s.y += neg ? -t.y : t.y;
  }
  return s;
}

// Sums over the workgroup of NQ per-thread values, identical on every
// thread, fixed order: each wave's butterfly sum, then the kRW wave sums
// butterflied across lanes (lane l reads wave l % kRW's sum).  lds holds
// kRW * NQ doubles; successive calls alternate between two such buffers (the
// caller's flip), so one barrier per call suffices: a buffer is written again
// only after every thread has passed the next call's barrier, which follows
// its reads of this one.
template <int NQ>
__device__ __forceinline__ void block_sums(double (&v)[NQ], double* lds2, int& flip) {
  static_assert(kRW == 16, "wave sums are combined by a 16-lane butterfly");
  double* lds = lds2 + flip * kRW * (1 + kObsQ);
  flip ^= 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[w * NQ + q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double r = lds[(lane & (kRW - 1)) * NQ + q];
#pragma unroll
    for (int off = 1; off < kRW; off <<= 1) r += __shfl_xor(r, off);
    v[q] = r;
  }
}

__device__ __forceinline__ double block_sum1(double v, double* lds2, int& flip) {
  double q[1] = {v};
  block_sums<1>(q, lds2, flip);
  return q[0];
}

// Hides x's value from the optimiser, so that what is derived from it (LDS
// and table addresses of a thread's elements) is computed where it is used
// instead of being kept live in registers across the whole propagation.
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

}  // namespace

template <typename R, int EPT>
__global__ __launch_bounds__(kRT) void k_resident(ResidentArgs P) {
  using V = typename CT<R>::T;
  __shared__ double red[2 * kRW * (1 + kObsQ)];  // two reduction buffers (block_sums)
  int flip = 0;
  __shared__ double sh_a[kMMax], sh_b[kMMax], sh_s[kMMax + 1], sh_y[2 * kMMax], sh_c[2 * kMMax];
  __shared__ double sh_eps;
  __shared__ V cf_dn[8], cf_up[8];
  __shared__ double2 of_dn[8], of_up[8];
  extern __shared__ __align__(16) unsigned char smem_raw[];

  const int vec = blockIdx.x, tid = threadIdx.x;
  const int du = P.dim_up, dd = P.dim_dn, ld = dd + 1;
  const int dim = du * dd;  // below kRT * EPT
  const int gdn = P.gs_dn / 4, gup = P.gs_up / 4;
  const bool want_obs = P.coef_obs != nullptr;
  V* const psi = static_cast<V*>(P.v) + static_cast<size_t>(vec) * dim;
  V* const sl = static_cast<V*>(P.slots) + static_cast<size_t>(vec) * P.m_max * dim;
  auto slot = [&](int k) { return k == 0 ? psi : sl + static_cast<size_t>(k - 1) * dim; };

  // LDS: tables, strings, on-site energies (as resident_lds_bytes), then the tile
  unsigned char* lp = smem_raw;
  auto carve = [&](size_t bytes) {
    unsigned char* q = lp;
    lp += (bytes + 15) & ~size_t(15);
    return q;
  };
  uint2* tdn = reinterpret_cast<uint2*>(carve(static_cast<size_t>(dd) * gdn * 8));
  uint2* tup = reinterpret_cast<uint2*>(carve(static_cast<size_t>(du) * gup * 8));
  uint32_t* upb = reinterpret_cast<uint32_t*>(carve(static_cast<size_t>(du) * 4));
  uint32_t* dnb = reinterpret_cast<uint32_t*>(carve(static_cast<size_t>(dd) * 4));
  const bool has_eps = P.eps_up != nullptr || P.eps_dn != nullptr;
  double* epu = has_eps ? reinterpret_cast<double*>(carve(static_cast<size_t>(du) * 8)) : nullptr;
  double* epd = has_eps ? reinterpret_cast<double*>(carve(static_cast<size_t>(dd) * 8)) : nullptr;
  V* xs = reinterpret_cast<V*>(lp);
  {
    const uint2* g1 = reinterpret_cast<const uint2*>(P.dn_tab);
    for (int i = tid; i < dd * gdn; i += kRT) tdn[i] = g1[i];
    const uint2* g2 = reinterpret_cast<const uint2*>(P.up_tab);
    for (int i = tid; i < du * gup; i += kRT) tup[i] = g2[i];
    for (int i = tid; i < du; i += kRT) {
      upb[i] = P.up_bits[i];
      if (has_eps) epu[i] = P.eps_up ? P.eps_up[i] : 0.0;
    }
    for (int i = tid; i < dd; i += kRT) {
      dnb[i] = P.dn_bits[i];
      if (has_eps) epd[i] = P.eps_dn ? P.eps_dn[i] : 0.0;
    }
    // the zero column and the zero row are never overwritten
    for (int a = tid; a < du; a += kRT) xs[a * ld + dd] = V{0, 0};
    for (int b = tid; b <= dd; b += kRT) xs[du * ld + b] = V{0, 0};
  }
  // This thread's elements as (a << 16 | b), -1 for none.  Slots s = e * kRT
  // + tid take consecutive elements in the order of s, except that wavefront
  // 0 keeps only its first w0 slots when the tile leaves room: it also
  // evaluates the Krylov estimate while the others run their applies.
  int ab[EPT];
  {
    const int spare = (EPT * kRT - dim) / 64;
    const int w0 = EPT - min(EPT, spare);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int i = e * kRT + tid - (e >= w0 ? 64 * (e - w0 + 1) : 0);
      const bool live = !(tid < 64 && e >= w0) && i < dim;
      ab[e] = live ? ((i / dd) << 16 | (i % dd)) : -1;
    }
  }
  auto lpos = [&](int q) { return (q >> 16) * ld + (q & 0xFFFF); };
  auto gidx = [&](int q) { return (q >> 16) * dd + (q & 0xFFFF); };
  __syncthreads();

  // H x at one element from the staged tile: the diagonal and the hop groups
  // with the midpoint coefficients (mid) and, in FP64, the hop part with the
  // sample-time coefficients (obs).
  auto hx = [&](int q, V x, bool mid, bool obs, V& acc, double2& ko, double& dg, double& nd) {
    const int a = q >> 16, b = q & 0xFFFF;
    nd = static_cast<double>(__popc(upb[a] & dnb[b]));
    dg = P.U * nd + (has_eps ? epu[a] : 0.0) + (has_eps ? epd[b] : 0.0);
    acc = V{static_cast<R>(dg) * x.x, static_cast<R>(dg) * x.y};
    ko = make_double2(0.0, 0.0);
    const V* row = xs + a * ld;
#pragma unroll 2
    for (int g = 0; g < gdn; ++g) {
      const V s = slot_sum4(tdn[b * gdn + g], row, static_cast<uint32_t>(dd), 1);
      if (mid) acc = cfma(cf_dn[g], s, acc);
      if (obs) ko = cfma(of_dn[g], make_double2(s.x, s.y), ko);
    }
    const V* col = xs + b;
#pragma unroll 2
    for (int g = 0; g < gup; ++g) {
      const V s = slot_sum4_skip(tup[a * gup + g], col, static_cast<uint32_t>(du), ld);
      if (mid) acc = cfma(cf_up[g], s, acc);
      if (obs) ko = cfma(of_up[g], make_double2(s.x, s.y), ko);
    }
  };
  auto load_coefs = [&](const double* c, bool obs) {
    if (tid < gdn) {
      const int k = P.dn_gclass[tid];
      if (obs) of_dn[tid] = make_double2(c[2 * k], c[2 * k + 1]);
      else cf_dn[tid] = V{static_cast<R>(c[2 * k]), static_cast<R>(c[2 * k + 1])};
    }
    if (tid >= 8 && tid < 8 + gup) {
      const int k = P.up_gclass[tid - 8];
      if (obs) of_up[tid - 8] = make_double2(c[2 * k], c[2 * k + 1]);
      else cf_up[tid - 8] = V{static_cast<R>(c[2 * k]), static_cast<R>(c[2 * k + 1])};
    }
  };
  auto obs_row = [&](int n) { return P.coef_obs + (static_cast<size_t>(vec) * (P.n_steps + 1) + n) * 2 * P.nc; };
  // observables [<D>, docc, |x|^2, Re <x|K(t)|x>] of the staged state into row n
  auto store_obs = [&](int n, double qd, double qo, double qn, double qh) {
    double q[kObsQ] = {qd, qo, qn, qh};
    block_sums<kObsQ>(q, red, flip);
    if (tid == 0) {
      double* o = P.obs + (static_cast<size_t>(n) * P.nvec + vec) * kObsQ;
#pragma unroll
      for (int k = 0; k < kObsQ; ++k) o[k] = q[k];
    }
  };
  // observables only, of the state in psi at sample row n
  auto obs_pass = [&](int n) {
    load_coefs(obs_row(n), true);
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (ab[e] >= 0) xs[lpos(opaque(ab[e]))] = psi[gidx(opaque(ab[e]))];
    __syncthreads();
    double qd = 0.0, qo = 0.0, qn = 0.0, qh = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      if (ab[e] < 0) continue;
      const int q = opaque(ab[e]);
      const V x = xs[lpos(q)];
      V acc;
      double2 ko;
      double dg, nd;
      hx(q, x, false, true, acc, ko, dg, nd);
      const double m2 = static_cast<double>(x.x) * x.x + static_cast<double>(x.y) * x.y;
      qd += dg * m2;
      qo += nd * m2;
      qn += m2;
      qh += static_cast<double>(x.x) * ko.x + static_cast<double>(x.y) * ko.y;
    }
    store_obs(n, qd, qo, qn, qh);
  };

  V w[EPT], up[EPT];  // w_j and u_{j-1} of this thread's elements
  int done = P.n_steps;
  const int S = P.n_exp * P.substeps;  // Krylov solves per step, each of length tau
  for (int n = 0; n < P.n_steps; ++n) {
    // the step's log: the largest m and eps of its solves, the last beta, the
    // worst status (non-finite, then m_max, then invariant subspace)
    int step_m = 0, step_status = 1;
    double step_eps = 0.0, step_beta = 0.0;
    for (int sub = 0; sub < S; ++sub) {
      const bool obs_now = want_obs && sub == 0;
      load_coefs(P.coef_mid + ((static_cast<size_t>(vec) * P.n_steps + n) * P.n_exp + sub / P.substeps) * 2 * P.nc,
                 false);
      if (obs_now) load_coefs(obs_row(n), true);
      // u_0 = psi, staged; beta_0 = |psi|
      double n2 = 0.0;
  #pragma unroll
      for (int e = 0; e < EPT; ++e) {
        if (ab[e] < 0) continue;
        const int q = opaque(ab[e]);
        const V x = psi[gidx(q)];
        xs[lpos(q)] = x;
        n2 += static_cast<double>(x.x) * x.x + static_cast<double>(x.y) * x.y;
      }
      const double beta0 = sqrt(block_sum1(n2, red, flip));
      const bool fin0 = isfinite(beta0), live = fin0 && beta0 > 0.0;
      const R s0 = static_cast<R>(live ? 1.0 / beta0 : 0.0);
      // iteration 0: w_0 = s_0 H u_0, alpha_0, and the observables of psi(t_n)
      {
        double qa = 0.0, qd = 0.0, qo = 0.0, qn = 0.0, qh = 0.0;
  #pragma unroll
        for (int e = 0; e < EPT; ++e) {
          if (ab[e] < 0) continue;
          const int q = opaque(ab[e]);
          const V x = xs[lpos(q)];
          V acc;
          double2 ko;
          double dg, nd;
          hx(q, x, true, obs_now, acc, ko, dg, nd);
          const V out = V{acc.x * s0, acc.y * s0};
          w[e] = out;
          qa += static_cast<double>(s0) * (static_cast<double>(x.x) * out.x + static_cast<double>(x.y) * out.y);
          if (obs_now) {
            const double m2 = static_cast<double>(x.x) * x.x + static_cast<double>(x.y) * x.y;
            qd += dg * m2;
            qo += nd * m2;
            qn += m2;
            qh += static_cast<double>(x.x) * ko.x + static_cast<double>(x.y) * ko.y;
          }
        }
        double q[1 + kObsQ] = {qa, qd, qo, qn, qh};
        block_sums<1 + kObsQ>(q, red, flip);
        const double a0 = q[0];
        if (obs_now && tid == 0) {
          double* o = P.obs + (static_cast<size_t>(n) * P.nvec + vec) * kObsQ;
  #pragma unroll
          for (int k = 0; k < kObsQ; ++k) o[k] = q[1 + k];
        }
        if (tid == 0) {
          sh_a[0] = a0;
          sh_s[0] = static_cast<double>(s0);
          sh_y[0] = 1.0;
          sh_y[1] = 0.0;
        }
        __syncthreads();
      }
      // a zero state stays zero (m = 1, invariant subspace); NaN or Inf stops the vector
      int m = 1, status = live ? 0 : (fin0 ? 2 : 4);
      double eps = 0.0, blast = 0.0;
      for (int j = 0; live; ++j) {
        const int J = j + 1;
        // u_J = w_j - alpha_j s_j u_j, staged in place of u_j
        const R c = static_cast<R>(sh_a[j] * sh_s[j]);
        double nn = 0.0;
  #pragma unroll
        for (int e = 0; e < EPT; ++e) {
          if (ab[e] < 0) continue;
          const int p = lpos(opaque(ab[e]));
          const V u = xs[p];
          V t = w[e];
          t.x -= c * u.x;
          t.y -= c * u.y;
          xs[p] = t;
          up[e] = u;
          nn += static_cast<double>(t.x) * t.x + static_cast<double>(t.y) * t.y;
        }
        const double bj = sqrt(block_sum1(nn, red, flip));
        // Iteration J's apply is needed unless beta_{J-1} = |u_J| or J = m_max
        // ends the step; it runs while wavefront 0 evaluates the estimate for
        // m = J (T_J: alpha_0..j, beta_0..j-1), and is discarded if that ends it.
        const bool work = isfinite(bj) && bj >= P.norm_inf * P.tol && J < P.m_max;
        if (tid < 64) {
          double yr, yi;
          const double e = wave_krylov_eps(J, tid < J ? sh_a[tid] : 0.0, sh_b, P.tau, sh_y, tid, yr, yi);
          if (tid < J) {
            sh_y[2 * tid] = yr;
            sh_y[2 * tid + 1] = yi;
          }
          if (tid == 0) {
            sh_eps = e;
            sh_b[j] = bj;
            sh_s[J] = work ? 1.0 / bj : 0.0;
          }
        }
        double qa = 0.0;
        if (work) {
          const R sJ = static_cast<R>(1.0 / bj), bp = static_cast<R>(bj * sh_s[j]);
  #pragma unroll
          for (int e = 0; e < EPT; ++e) {
            if (ab[e] < 0) continue;
            const int q = opaque(ab[e]);
            const V x = xs[lpos(q)];
            slot(J)[gidx(q)] = x;  // u_J for the combine
            V acc;
            double2 ko;
            double dg, nd;
            hx(q, x, true, false, acc, ko, dg, nd);
            V out = acc;
            out.x = out.x * sJ - bp * up[e].x;
            out.y = out.y * sJ - bp * up[e].y;
            w[e] = out;
            qa += static_cast<double>(sJ) * (static_cast<double>(x.x) * out.x + static_cast<double>(x.y) * out.y);
          }
        }
        const double aJ = block_sum1(qa, red, flip);  // also publishes the estimate
        const double ej = sh_eps;
        int st = 0;
        if (!isfinite(bj) || !isfinite(ej)) st = 4;
        else if (bj < P.norm_inf * P.tol) st = 2;
        else if (ej < P.tol) st = 1;
        else if (J >= P.m_max) st = 3;
        if (st != 0) {
          m = J;
          status = st;
          eps = ej;
          blast = bj;
          break;
        }
        if (tid == 0) sh_a[J] = aJ;
        __syncthreads();
      }
      // psi <- beta_0 sum_{k < m} y_k s_k u_k (u_0 = psi itself), the loads of
      // one Krylov vector for all of the thread's elements in flight together
      if (tid < m) {
        sh_c[2 * tid] = beta0 * sh_s[tid] * sh_y[2 * tid];
        sh_c[2 * tid + 1] = beta0 * sh_s[tid] * sh_y[2 * tid + 1];
      }
      __syncthreads();
      {
        double ar[EPT], ai[EPT];
  #pragma unroll
        for (int e = 0; e < EPT; ++e) ar[e] = ai[e] = 0.0;
        for (int k = 0; k < m; ++k) {
          const V* __restrict__ sk = slot(k);
          const double cr = sh_c[2 * k], ci = sh_c[2 * k + 1];
          V u[EPT];
  #pragma unroll
          for (int e = 0; e < EPT; ++e) u[e] = ab[e] >= 0 ? sk[gidx(opaque(ab[e]))] : V{0, 0};
  #pragma unroll
          for (int e = 0; e < EPT; ++e) {
            ar[e] += cr * u[e].x - ci * u[e].y;
            ai[e] += cr * u[e].y + ci * u[e].x;
          }
        }
  #pragma unroll
        for (int e = 0; e < EPT; ++e)
          if (ab[e] >= 0) psi[gidx(opaque(ab[e]))] = V{static_cast<R>(ar[e]), static_cast<R>(ai[e])};
      }
      step_m = max(step_m, m);
      step_eps = fmax(step_eps, eps);
      step_beta = blast;
      if (status == 4) step_status = 4;
      else if (status == 3 && step_status != 4) step_status = 3;
      else if (status == 2 && step_status < 3) step_status = 2;
      __syncthreads();  // the next solve restages the tile and reloads the coefficients
      if (status >= 3) break;  // m_max without the tolerance, or non-finite: this vector stops here
    }
    if (tid == 0) {
      CombineLog& L = P.log[static_cast<size_t>(n) * P.nvec + vec];
      L.m = step_m;
      L.status = step_status;
      L.eps = step_eps;
      L.beta_last = step_beta;
    }
    if (step_status >= 3) {
      done = n + 1;
      break;
    }
  }
  if (want_obs) obs_pass(done);
  if (tid == 0) P.done[vec] = done;
}

// Elements per thread of the instantiation a sector runs on: the smallest
// that covers it (five covers 8 sites at half filling; each larger one holds
// more of a thread's elements in registers and spills more).
int resident_ept(int prec, int64_t dim) {
  static constexpr int kEpts[] = {1, 2, 4, 5, 6, 8, 12, 16};
  for (int e : kEpts)
    if (e <= kResidentEpt[prec] && dim <= static_cast<int64_t>(e) * kRT) return e;
  return 0;
}

template <typename R, int EPT>
hipError_t launch_resident_t(const ResidentArgs& a, size_t lds, hipStream_t s) {
  auto fn = k_resident<R, EPT>;
  static const int max_dyn = dyn_lds_opt_in(reinterpret_cast<const void*>(fn));
  if (lds > static_cast<size_t>(max_dyn)) return hipErrorInvalidValue;
  ResidentArgs args = a;
  void* kargs[] = {&args};
  return hipLaunchKernel(reinterpret_cast<const void*>(fn), dim3(a.nvec), dim3(kRT), kargs, lds, s);
}

}  // namespace dev

int resident_lds_limit(int prec) {
  // every instantiation has the same static LDS; the largest one stands for all
  static const int lim_d = dev::dyn_lds_opt_in(reinterpret_cast<const void*>(dev::k_resident<double, 8>));
  static const int lim_f = dev::dyn_lds_opt_in(reinterpret_cast<const void*>(dev::k_resident<float, 16>));
  return prec == 0 ? lim_d : lim_f;
}

hipError_t launch_resident(int prec, const ResidentArgs& a, size_t lds, hipStream_t s) {
  if (a.nvec < 1) return hipSuccess;
  if (a.dim_up < 1 || a.dim_dn < 1 || a.dim_up >= 65535 || a.dim_dn >= 65535 || a.m_max < 1 || a.m_max > kMMax ||
      a.gs_dn / 4 > 8 || a.gs_up / 4 > 8)
    return hipErrorInvalidValue;
  const int64_t dim = static_cast<int64_t>(a.dim_up) * a.dim_dn;
  switch (dev::resident_ept(prec, dim) * (prec == 0 ? 1 : -1)) {
    case 1: return dev::launch_resident_t<double, 1>(a, lds, s);
    case 2: return dev::launch_resident_t<double, 2>(a, lds, s);
    case 4: return dev::launch_resident_t<double, 4>(a, lds, s);
    case 5: return dev::launch_resident_t<double, 5>(a, lds, s);
    case 6: return dev::launch_resident_t<double, 6>(a, lds, s);
    case 8: return dev::launch_resident_t<double, 8>(a, lds, s);
    case -1: return dev::launch_resident_t<float, 1>(a, lds, s);
    case -2: return dev::launch_resident_t<float, 2>(a, lds, s);
    case -4: return dev::launch_resident_t<float, 4>(a, lds, s);
    case -5: return dev::launch_resident_t<float, 5>(a, lds, s);
    case -6: return dev::launch_resident_t<float, 6>(a, lds, s);
    case -8: return dev::launch_resident_t<float, 8>(a, lds, s);
    case -12: return dev::launch_resident_t<float, 12>(a, lds, s);
    case -16: return dev::launch_resident_t<float, 16>(a, lds, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hub
