// Persistent stepper of the excited members of the Green's-function runs
// (Sec. 2.5, Eq. (Glg); Sec. 3.7): one launch propagates every member of a
// batch, each in its own workgroup, for all its midpoint steps (Eq.
// (time-stepping)) with no kernel boundary: the Lanczos iterations with the
// a-posteriori estimate of Alg. 6, the combine, and after every step the
// overlap <c psi(t' + s) | phi(t' + s)> with the recorded source-sector state.
// Members of several sectors (different hop tables) share the launch through
// per-member descriptors.  Meant for small sectors (10 sites), whose applies
// are far too short to fill the GPU one launch at a time.
#include "kernels_common.h"
#include "members.h"

namespace hub {
namespace dev {

namespace {

constexpr int kMT = 1024;          // threads per member workgroup
constexpr int kMW = kMT / 64;      // its wavefronts

// Sum over the workgroup, identical on every thread, fixed order.
__device__ inline double msum(double v, double* red) { return block_sum<kMW>(v, red); }

// Signed sum of the four staged values one table word pair indexes (src,
// src + dim + 1 for a negative sign, dim = the zero slot); staged element q
// is at xs[q * stride].
template <typename V>
__device__ __forceinline__ V group4(uint2 w, const V* xs, uint32_t dim, int stride) {
  V s = V{0, 0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t w2 = k < 2 ? w.x : w.y;
    const uint32_t idx = (k & 1) ? (w2 >> 16) : (w2 & 0xFFFFu);
    const bool neg = idx > dim;
    const uint32_t src = neg ? idx - dim - 1u : idx;
    const V t = xs[static_cast<size_t>(src) * stride];
    s.x += neg ? -t.x : t.x;
    s.y += neg ? -t.y : t.y;
  }
  return s;
}

}  // namespace

// One workgroup = one member.  Vectors of the member: slot k = u_k of the
// Krylov basis (v_k = s_k u_k, slot 0 = the member's state), z = row-pass
// product.  Per iteration j: w = s_j H u_j - beta_{j-1} s_{j-1} u_{j-1}
// (row pass over blocks of staged tile rows, then column pass over blocks of
// staged tile columns), alpha_j = s_j Re <u_j, w>, u_{j+1} = w - alpha_j s_j
// u_j, beta_j = |u_{j+1}|, and the decision for m = j + 1 by one wavefront.
template <typename R>
__global__ __launch_bounds__(kMT) void k_members(MembersArgs P) {
  using V = typename CT<R>::T;
  __shared__ double red[kMW];
  __shared__ double sh_a[kMMax], sh_b[kMMax], sh_s[kMMax + 1], sh_y[2 * kMMax];
  __shared__ V cf_dn[8], cf_up[8];
  __shared__ int sh_ctl[2];  // [0]: stop, [1]: status
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* xs = reinterpret_cast<V*>(smem_raw);

  const MemberDesc& M = P.members[blockIdx.x];
  const MemberSector& S = P.sectors[M.sector];
  const int tid = threadIdx.x;
  const int du = S.dim_up, dd = S.dim_dn;
  const int64_t dim = static_cast<int64_t>(du) * dd;
  V* const slots = static_cast<V*>(M.slots);
  V* const z = static_cast<V*>(M.z);
  const uint2* tdn = reinterpret_cast<const uint2*>(S.dn_tab);
  const uint2* tup = reinterpret_cast<const uint2*>(S.up_tab);
  const int gdn = S.gs_dn / 4, gup = S.gs_up / 4;
  const int rb = S.row_block, cb = S.col_block;

  // <c psi(step n) | slot 0>, gathered through the member's operator map
  auto overlap = [&](int n, int s_rel) {
    const V* psi = static_cast<const V*>(P.traj) + static_cast<int64_t>(n) * P.traj_stride;
    double re = 0.0, im = 0.0;
    for (int64_t y = tid; y < dim; y += kMT) {
      const int a = static_cast<int>(y / dd), b = static_cast<int>(y % dd);
      const int r = M.down ? b : a;
      const int src = M.map[r];
      if (src < 0) continue;
      const int64_t se = M.down ? static_cast<int64_t>(a) * P.dim_dn_s + src : static_cast<int64_t>(src) * P.dim_dn_s + b;
      const V x = psi[se];
      const V f = slots[y];
      const double sg = static_cast<double>(M.sgn[r]);
      re += sg * (static_cast<double>(x.x) * f.x + static_cast<double>(x.y) * f.y);
      im += sg * (static_cast<double>(x.x) * f.y - static_cast<double>(x.y) * f.x);
    }
    re = msum(re, red);
    im = msum(im, red);
    if (tid == 0) {
      M.out[2 * s_rel] = re;
      M.out[2 * s_rel + 1] = im;
    }
  };

  overlap(M.start, 0);
  for (int s_rel = 0; s_rel < P.n_rel; ++s_rel) {
    const int n = M.start + s_rel;  // global step: coefficients at its midpoint
    if (tid < gdn) {
      const int c = S.dn_gclass[tid];
      cf_dn[tid] = V{static_cast<R>(S.coef_tab[static_cast<size_t>(n) * 2 * S.nc + 2 * c]),
                     static_cast<R>(S.coef_tab[static_cast<size_t>(n) * 2 * S.nc + 2 * c + 1])};
    }
    if (tid < gup) {
      const int c = S.up_gclass[tid];
      cf_up[tid] = V{static_cast<R>(S.coef_tab[static_cast<size_t>(n) * 2 * S.nc + 2 * c]),
                     static_cast<R>(S.coef_tab[static_cast<size_t>(n) * 2 * S.nc + 2 * c + 1])};
    }
    // beta_0 = |u_0|
    double n2 = 0.0;
    for (int64_t i = tid; i < dim; i += kMT) {
      const V t = slots[i];
      n2 += static_cast<double>(t.x) * t.x + static_cast<double>(t.y) * t.y;
    }
    const double beta0 = sqrt(msum(n2, red));
    if (tid == 0) {
      sh_s[0] = beta0 > 0.0 ? 1.0 / beta0 : 0.0;
      sh_y[0] = 1.0;
      sh_y[1] = 0.0;
      sh_ctl[0] = beta0 > 0.0 ? 0 : 1;
      sh_ctl[1] = beta0 > 0.0 ? 0 : 2;  // a zero state stays zero
    }
    __syncthreads();
    int m = sh_ctl[0] ? 1 : 0;
    for (int j = 0; j < P.m_max && !sh_ctl[0]; ++j) {
      const V* u = slots + static_cast<int64_t>(j) * dim;
      V* w = slots + static_cast<int64_t>(j + 1) * dim;
      const V* up = j > 0 ? slots + static_cast<int64_t>(j - 1) * dim : nullptr;
      const R sj = static_cast<R>(sh_s[j]);
      const R bp = static_cast<R>(j > 0 ? sh_b[j - 1] * sh_s[j - 1] : 0.0);
      // row pass: z = D u + down hops of u, rb tile rows at a time
      for (int a0 = 0; a0 < du; a0 += rb) {
        const int nr = min(rb, du - a0);
        for (int t = tid; t < nr * (dd + 1); t += kMT) {
          const int r = t / (dd + 1), b = t % (dd + 1);
          xs[t] = b < dd ? u[static_cast<int64_t>(a0 + r) * dd + b] : V{0, 0};
        }
        __syncthreads();
        for (int t = tid; t < nr * dd; t += kMT) {
          const int r = t / dd, b = t % dd, a = a0 + r;
          const V* row = xs + r * (dd + 1);
          const double dg = S.U * __popc(S.up_bits[a] & S.dn_bits[b]) + (S.eps_up ? S.eps_up[a] : 0.0) +
                            (S.eps_dn ? S.eps_dn[b] : 0.0);
          const V xv = row[b];
          V acc = V{static_cast<R>(dg) * xv.x, static_cast<R>(dg) * xv.y};
          for (int g = 0; g < gdn; ++g) acc = cfma(cf_dn[g], group4(tdn[static_cast<size_t>(b) * gdn + g], row,
                                                                    static_cast<uint32_t>(dd), 1), acc);
          z[static_cast<int64_t>(a) * dd + b] = acc;
        }
        __syncthreads();
      }
      // column pass: w = s_j (z + up hops of u) - bp u_{j-1}, cb columns at a time
      double qa = 0.0;
      for (int b0 = 0; b0 < dd; b0 += cb) {
        const int nc = min(cb, dd - b0);
        for (int t = tid; t < (du + 1) * nc; t += kMT) {
          const int a = t / nc, c = t % nc;
          xs[a * cb + c] = a < du ? u[static_cast<int64_t>(a) * dd + b0 + c] : V{0, 0};
        }
        __syncthreads();
        for (int t = tid; t < du * nc; t += kMT) {
          const int a = t / nc, c = t % nc;
          const int64_t o = static_cast<int64_t>(a) * dd + b0 + c;
          V acc = z[o];
          for (int g = 0; g < gup; ++g) acc = cfma(cf_up[g], group4(tup[static_cast<size_t>(a) * gup + g], xs + c,
                                                                    static_cast<uint32_t>(du), cb), acc);
          const V pv = up ? up[o] : V{0, 0};
          const V out = V{acc.x * sj - bp * pv.x, acc.y * sj - bp * pv.y};
          const V xv = xs[a * cb + c];
          qa += static_cast<double>(sj) * (static_cast<double>(xv.x) * out.x + static_cast<double>(xv.y) * out.y);
          w[o] = out;
        }
        __syncthreads();
      }
      const double aj = msum(qa, red);
      // u_{j+1} = w - alpha_j s_j u_j and its norm
      const R cu = static_cast<R>(aj * sh_s[j]);
      double q2 = 0.0;
      for (int64_t i = tid; i < dim; i += kMT) {
        const V uu = u[i];
        V t = w[i];
        t.x -= cu * uu.x;
        t.y -= cu * uu.y;
        w[i] = t;
        q2 += static_cast<double>(t.x) * t.x + static_cast<double>(t.y) * t.y;
      }
      const double bj = sqrt(msum(q2, red));
      // decision for m = j + 1 (one wavefront): T_{j+1} = alpha_0..j, beta_0..j-1
      if (tid < 64) {
        if (tid == 0) sh_a[j] = aj;
        const double a_l = tid < j ? sh_a[tid] : (tid == j ? aj : 0.0);
        double yr, yi;
        const double eps = wave_krylov_eps(j + 1, a_l, sh_b, P.tau, sh_y, tid, yr, yi);
        if (tid <= j) {
          sh_y[2 * tid] = yr;
          sh_y[2 * tid + 1] = yi;
        }
        if (tid == 0) {
          sh_b[j] = bj;
          int status = 0;
          if (bj < S.norm_inf * P.tol) status = 2;
          else if (eps < P.tol) status = 1;
          else if (j + 1 >= P.m_max) status = 3;
          sh_s[j + 1] = (status == 0 && bj > 0.0) ? 1.0 / bj : 0.0;
          sh_ctl[0] = status != 0;
          sh_ctl[1] = status;
        }
      }
      __syncthreads();
      m = j + 1;
    }
    // state <- beta0 sum_{k < m} y_k s_k u_k (in place into slot 0)
    for (int64_t i = tid; i < dim; i += kMT) {
      double ar = 0.0, ai = 0.0;
      for (int k = 0; k < m; ++k) {
        const double cr = beta0 * sh_s[k] * sh_y[2 * k], ci = beta0 * sh_s[k] * sh_y[2 * k + 1];
        const V t = slots[static_cast<int64_t>(k) * dim + i];
        ar += cr * t.x - ci * t.y;
        ai += cr * t.y + ci * t.x;
      }
      slots[i] = V{static_cast<R>(ar), static_cast<R>(ai)};
    }
    __syncthreads();
    if (tid == 0) {
      M.status[s_rel] = sh_ctl[1];
      M.m_used[s_rel] = m;
    }
    overlap(n + 1, s_rel + 1);
    if (sh_ctl[1] == 3) {  // m_max without the tolerance: the member stops, later overlaps are NaN
      for (int r = s_rel + 2 + tid; r <= P.n_rel; r += kMT) {
        M.out[2 * r] = __builtin_nan("");
        M.out[2 * r + 1] = __builtin_nan("");
      }
      for (int r = s_rel + 1 + tid; r < P.n_rel; r += kMT) {
        M.status[r] = 0;
        M.m_used[r] = 0;
      }
      return;
    }
    __syncthreads();
  }
}

}  // namespace dev

hipError_t launch_members(int prec, int n_members, const MembersArgs& a, size_t lds, hipStream_t s) {
  if (n_members < 1) return hipSuccess;
  static const int max_d = dev::dyn_lds_opt_in(reinterpret_cast<const void*>(dev::k_members<double>));
  static const int max_f = dev::dyn_lds_opt_in(reinterpret_cast<const void*>(dev::k_members<float>));
  if (lds > static_cast<size_t>(prec == 0 ? max_d : max_f)) return hipErrorInvalidValue;
  const void* fn = prec == 0 ? reinterpret_cast<const void*>(dev::k_members<double>)
                             : reinterpret_cast<const void*>(dev::k_members<float>);
  MembersArgs args = a;
  void* kargs[] = {&args};
  return hipLaunchKernel(fn, dim3(n_members), dim3(dev::kMT), kargs, lds, s);
}

}  // namespace hub
