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

constexpr int kMT = 1024;      // threads per member workgroup
constexpr int kMW = kMT / 64;  // its wavefronts
constexpr int kB = 4;          // elements per thread whose memory loads are issued together

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
// Krylov basis (v_k = s_k u_k, slot 0 = the member's state), z = the row
// pass's product.  The sector's hop tables, strings and on-site energies and
// the member's operator map sit in LDS (MemberSector::tab_lds bytes), so the
// only memory traffic is the vectors', loaded kB elements per thread at a
// time.  Iteration j: the column pass finishes w = s_j H u_j - beta_{j-1}
// s_{j-1} u_{j-1} into slot j + 1 with alpha_j = s_j Re <u_j, w>; one
// wavefront evaluates the estimate for m = j + 1 (it needs T_{j+1} only, not
// beta_j); unless that ends the step, the next row pass forms u_{j+1} = w -
// alpha_j s_j u_j in place while staging it, and its norm beta_j decides
// breakdown before the next column pass.  The combine writes the new state
// into slot 0 and in the same pass sums its norm (the next step's beta_0) and
// its overlap with the recorded source-sector state.
template <typename R>
__global__ __launch_bounds__(kMT) void k_members(MembersArgs P) {
  using V = typename CT<R>::T;
  __shared__ double red[kMW];
  __shared__ double sh_a[kMMax], sh_b[kMMax], sh_s[kMMax + 1], sh_y[2 * kMMax];
  __shared__ double sh_c[2 * kMMax];  // combine coefficients beta_0 s_k y_k
  __shared__ V cf_dn[8], cf_up[8];
  __shared__ int sh_ctl[2];  // [0]: the step ends, [1]: its status
  extern __shared__ __align__(16) unsigned char smem_raw[];

  const MemberDesc& M = P.members[blockIdx.x];
  const MemberSector& S = P.sectors[M.sector];
  const int tid = threadIdx.x;
  const int du = S.dim_up, dd = S.dim_dn;
  const int dim = du * dd;  // the stepper takes sectors of fewer than 2^31 states
  const int gdn = S.gs_dn / 4, gup = S.gs_up / 4;
  const int mlen = M.down ? dd : du;
  const int rb = S.row_block, cb = S.col_block;
  V* const slots = static_cast<V*>(M.slots);
  V* const z = static_cast<V*>(M.z);
  auto slot = [&](int k) { return slots + static_cast<size_t>(k) * dim; };

  // LDS: the tables (layout as members_table_lds computes it), then staging
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
  const bool has_eps = S.eps_up != nullptr || S.eps_dn != nullptr;
  double* epu = has_eps ? reinterpret_cast<double*>(carve(static_cast<size_t>(du) * 8)) : nullptr;
  double* epd = has_eps ? reinterpret_cast<double*>(carve(static_cast<size_t>(dd) * 8)) : nullptr;
  int32_t* mp = reinterpret_cast<int32_t*>(carve(static_cast<size_t>(mlen) * 4));
  int8_t* sg = reinterpret_cast<int8_t*>(carve(static_cast<size_t>(mlen)));
  V* xs = reinterpret_cast<V*>(smem_raw + S.tab_lds);
  {
    const uint2* g1 = reinterpret_cast<const uint2*>(S.dn_tab);
    for (int i = tid; i < dd * gdn; i += kMT) tdn[i] = g1[i];
    const uint2* g2 = reinterpret_cast<const uint2*>(S.up_tab);
    for (int i = tid; i < du * gup; i += kMT) tup[i] = g2[i];
    for (int i = tid; i < du; i += kMT) {
      upb[i] = S.up_bits[i];
      if (has_eps) epu[i] = S.eps_up ? S.eps_up[i] : 0.0;
    }
    for (int i = tid; i < dd; i += kMT) {
      dnb[i] = S.dn_bits[i];
      if (has_eps) epd[i] = S.eps_dn ? S.eps_dn[i] : 0.0;
    }
    for (int i = tid; i < mlen; i += kMT) {
      mp[i] = M.map[i];
      sg[i] = M.sgn[i];
    }
  }
  __syncthreads();

  // Row pass over u in blocks of rb staged tile rows: z = D u + down hops of
  // u.  With `form`, u is first formed in place as u - c uprev and the
  // thread's part of |u|^2 is returned; without `want_z` only that is done.
  auto row_pass = [&](V* __restrict__ u, const V* __restrict__ uprev, R c, bool form, bool want_z) -> double {
    double n2 = 0.0;
    for (int a0 = 0; a0 < du; a0 += rb) {
      const int nr = min(rb, du - a0);
      const int ns = nr * (dd + 1);
      for (int t0 = tid; t0 < ns; t0 += kB * kMT) {
        V val[kB], q[kB];
        int off[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
          const int t = t0 + k * kMT;
          const int r = t / (dd + 1), b = t - r * (dd + 1);
          const bool ok = t < ns && b < dd;
          off[k] = ok ? (a0 + r) * dd + b : -1;
          val[k] = ok ? u[off[k]] : V{0, 0};
          q[k] = (ok && form) ? uprev[off[k]] : V{0, 0};
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
          const int t = t0 + k * kMT;
          if (t >= ns) continue;
          V v = val[k];
          if (form && off[k] >= 0) {
            v.x -= c * q[k].x;
            v.y -= c * q[k].y;
            u[off[k]] = v;
            n2 += static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y;
          }
          xs[t] = v;
        }
      }
      __syncthreads();
      if (want_z) {
        for (int t = tid; t < nr * dd; t += kMT) {
          const int r = t / dd, b = t - r * dd, a = a0 + r;
          const V* row = xs + r * (dd + 1);
          const double dg = S.U * __popc(upb[a] & dnb[b]) + (epu ? epu[a] : 0.0) + (epd ? epd[b] : 0.0);
          const V xv = row[b];
          V acc = V{static_cast<R>(dg) * xv.x, static_cast<R>(dg) * xv.y};
          for (int g = 0; g < gdn; ++g)
            acc = cfma(cf_dn[g], group4(tdn[b * gdn + g], row, static_cast<uint32_t>(dd), 1), acc);
          z[a * dd + b] = acc;
        }
      }
      __syncthreads();
    }
    return n2;
  };

  // Column pass in blocks of cb staged tile columns: w = sj (z + up hops of
  // u) - bp uprev; returns the thread's part of sj Re <u, w>.
  auto col_pass = [&](const V* __restrict__ u, const V* __restrict__ uprev, V* __restrict__ w, R sj,
                      R bp) -> double {
    double qa = 0.0;
    for (int b0 = 0; b0 < dd; b0 += cb) {
      const int nc = min(cb, dd - b0);
      const int ns = (du + 1) * nc;
      for (int t0 = tid; t0 < ns; t0 += kB * kMT) {
        V val[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
          const int t = t0 + k * kMT;
          const int a = t / nc, c = t - a * nc;
          val[k] = (t < ns && a < du) ? u[a * dd + b0 + c] : V{0, 0};
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
          const int t = t0 + k * kMT;
          if (t >= ns) continue;
          const int a = t / nc, c = t - a * nc;
          xs[a * cb + c] = val[k];
        }
      }
      __syncthreads();
      const int ne = du * nc;
      for (int t0 = tid; t0 < ne; t0 += kB * kMT) {
        V zv[kB], pv[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
          const int t = t0 + k * kMT;
          const int a = t / nc, c = t - a * nc;
          const bool ok = t < ne;
          const int o = a * dd + b0 + c;
          zv[k] = ok ? z[o] : V{0, 0};
          pv[k] = (ok && uprev) ? uprev[o] : V{0, 0};
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
          const int t = t0 + k * kMT;
          if (t >= ne) continue;
          const int a = t / nc, c = t - a * nc;
          V acc = zv[k];
          for (int g = 0; g < gup; ++g)
            acc = cfma(cf_up[g], group4(tup[a * gup + g], xs + c, static_cast<uint32_t>(du), cb), acc);
          const V out = V{acc.x * sj - bp * pv[k].x, acc.y * sj - bp * pv[k].y};
          const V xv = xs[a * cb + c];
          qa += static_cast<double>(sj) * (static_cast<double>(xv.x) * out.x + static_cast<double>(xv.y) * out.y);
          w[a * dd + b0 + c] = out;
        }
      }
      __syncthreads();
    }
    return qa;
  };

  // Sums over the state f (in slot 0 after `fill`, which computes element
  // i): |f|^2 and <c psi(recorded state n) | f>, the record gathered through
  // the member's operator map; kB elements per thread at a time.
  auto state_sums = [&](int n, auto fill, double& n2, double& re, double& im) {
    const V* __restrict__ psi = static_cast<const V*>(P.traj) + static_cast<int64_t>(n) * P.traj_stride;
    n2 = re = im = 0.0;
    for (int i0 = tid; i0 < dim; i0 += kB * kMT) {
      V f[kB], x[kB];
      double sgv[kB];
      fill(i0, f);
#pragma unroll
      for (int e = 0; e < kB; ++e) {
        const int i = i0 + e * kMT;
        x[e] = V{0, 0};
        sgv[e] = 0.0;
        if (i < dim) {
          const int a = i / dd, b = i - a * dd;
          const int r = M.down ? b : a;
          const int src = mp[r];
          if (src >= 0) {
            const int64_t se =
                M.down ? static_cast<int64_t>(a) * P.dim_dn_s + src : static_cast<int64_t>(src) * P.dim_dn_s + b;
            x[e] = psi[se];
            sgv[e] = static_cast<double>(sg[r]);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < kB; ++e) {
        n2 += static_cast<double>(f[e].x) * f[e].x + static_cast<double>(f[e].y) * f[e].y;
        re += sgv[e] * (static_cast<double>(x[e].x) * f[e].x + static_cast<double>(x[e].y) * f[e].y);
        im += sgv[e] * (static_cast<double>(x[e].x) * f[e].y - static_cast<double>(x[e].y) * f[e].x);
      }
    }
    n2 = msum(n2, red);
    re = msum(re, red);
    im = msum(im, red);
  };

  // overlap at s = 0 and |state|^2
  double n2s;
  {
    double re, im;
    state_sums(
        M.start,
        [&](int i0, V (&f)[kB]) {
#pragma unroll
          for (int e = 0; e < kB; ++e) f[e] = i0 + e * kMT < dim ? slot(0)[i0 + e * kMT] : V{0, 0};
        },
        n2s, re, im);
    if (tid == 0) {
      M.out[0] = re;
      M.out[1] = im;
    }
  }
  for (int s_rel = 0; s_rel < P.n_rel; ++s_rel) {
    const int n = M.start + s_rel;  // global step: coefficients at its midpoint
    const double* ct = S.coef_tab + static_cast<size_t>(n) * 2 * S.nc;
    if (tid < gdn) cf_dn[tid] = V{static_cast<R>(ct[2 * S.dn_gclass[tid]]), static_cast<R>(ct[2 * S.dn_gclass[tid] + 1])};
    if (tid < gup) cf_up[tid] = V{static_cast<R>(ct[2 * S.up_gclass[tid]]), static_cast<R>(ct[2 * S.up_gclass[tid] + 1])};
    const double beta0 = sqrt(n2s);
    const bool fin0 = isfinite(beta0);
    if (tid == 0) {
      sh_s[0] = (fin0 && beta0 > 0.0) ? 1.0 / beta0 : 0.0;
      sh_y[0] = 1.0;
      sh_y[1] = 0.0;
      sh_ctl[1] = !fin0 ? 4 : (beta0 > 0.0 ? 0 : 2);  // a zero state stays zero; NaN or Inf stops the member
    }
    __syncthreads();
    int m = 1;
    if (fin0 && beta0 > 0.0) {
      for (int j = 0;; ++j) {
        // row pass: u_j (for j > 0 formed in place as w - alpha_{j-1} s_{j-1}
        // u_{j-1}) and z = D u_j + down hops; at j = m_max only |u_j|
        const bool last = j >= P.m_max;
        const R c = static_cast<R>(j > 0 ? sh_a[j - 1] * sh_s[j - 1] : 0.0);
        const double nn = row_pass(slot(j), j > 0 ? slot(j - 1) : nullptr, c, j > 0, !last);
        if (j > 0) {  // beta_{j-1} = |u_j|: breakdown, or m_max without the tolerance
          const double bj = sqrt(msum(nn, red));
          if (tid == 0) {
            sh_b[j - 1] = bj;
            const int status = !isfinite(bj) ? 4 : (bj < S.norm_inf * P.tol ? 2 : (last ? 3 : 0));
            sh_s[j] = (status == 0 && bj > 0.0) ? 1.0 / bj : 0.0;
            sh_ctl[1] = status;
          }
          __syncthreads();
          if (sh_ctl[1] != 0) {
            m = j;
            break;
          }
        }
        // column pass: w = s_j H u_j - beta_{j-1} s_{j-1} u_{j-1} into slot j + 1
        const R sj = static_cast<R>(sh_s[j]);
        const R bp = static_cast<R>(j > 0 ? sh_b[j - 1] * sh_s[j - 1] : 0.0);
        const double aj = msum(col_pass(slot(j), j > 0 ? slot(j - 1) : nullptr, slot(j + 1), sj, bp), red);
        // estimate for m = j + 1: T_{j+1} = alpha_0..j, beta_0..j-1
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
            sh_ctl[0] = (eps < P.tol || !isfinite(eps)) ? 1 : 0;
            if (eps < P.tol) sh_ctl[1] = 1;
            else if (!isfinite(eps)) sh_ctl[1] = 4;
          }
        }
        __syncthreads();
        if (sh_ctl[0]) {
          m = j + 1;
          break;
        }
      }
    }
    // state <- beta_0 sum_{k < m} y_k s_k u_k in place into slot 0, with its
    // norm and its overlap with the recorded state after the step
    if (tid < m) {
      sh_c[2 * tid] = beta0 * sh_s[tid] * sh_y[2 * tid];
      sh_c[2 * tid + 1] = beta0 * sh_s[tid] * sh_y[2 * tid + 1];
    }
    __syncthreads();
    double re, im;
    state_sums(
        n + 1,
        [&](int i0, V (&f)[kB]) {
          double ar[kB], ai[kB];
#pragma unroll
          for (int e = 0; e < kB; ++e) ar[e] = ai[e] = 0.0;
          for (int k = 0; k < m; ++k) {
            const V* __restrict__ sk = slot(k);
            const double cr = sh_c[2 * k], ci = sh_c[2 * k + 1];
#pragma unroll
            for (int e = 0; e < kB; ++e) {
              const int i = i0 + e * kMT;
              const V t = i < dim ? sk[i] : V{0, 0};
              ar[e] += cr * t.x - ci * t.y;
              ai[e] += cr * t.y + ci * t.x;
            }
          }
#pragma unroll
          for (int e = 0; e < kB; ++e) {
            const int i = i0 + e * kMT;
            f[e] = V{static_cast<R>(ar[e]), static_cast<R>(ai[e])};
            if (i < dim) slot(0)[i] = f[e];
          }
        },
        n2s, re, im);
    const int status = sh_ctl[1];
    if (tid == 0) {
      M.out[2 * (s_rel + 1)] = re;
      M.out[2 * (s_rel + 1) + 1] = im;
      M.status[s_rel] = status;
      M.m_used[s_rel] = m;
    }
    if (status >= 3) {  // m_max without the tolerance, or non-finite: the member stops, later overlaps are NaN
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
