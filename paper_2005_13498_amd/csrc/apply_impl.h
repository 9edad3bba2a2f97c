// Matrix-free Hamiltonian apply (templated); instantiated per precision by
// apply_c128.hip and apply_c64.hip.
#pragma once

#include <hip/hip_ext.h>

#include "coef_pack.h"
#include "kernels_common.h"

namespace hub {
namespace dev {

// Matrix-free H x on the [dim_up x dim_dn] tile (NV vectors interleaved per
// element):
//   y[a,b] = (U popc(u_a & d_b) + e_a + e_b) x[a,b]
//          + sum over up hops a'->a:   sgn coef_c x[a',b]
//          + sum over down hops b'->b: sgn coef_c x[a,b'].
// The observables modes also accumulate, in FP64, the same hop sum with the
// coefficients of the observation time (K(t_obs) x), and per workgroup the
// diagonal energy, the double occupation, |x|^2 and Re <x|K(t_obs)|x>.
// A workgroup owns one tile row.  The row is staged in LDS twice, as +x and
// -x, followed by a zero slot, so a down hop is one LDS read at an index that
// already encodes its fermion sign (pad slots read the zero).  Each thread
// takes one column at a time: it loads the column's padded, class-sorted hop
// indices with 16-byte loads and runs a fully unrolled, branch-free slot loop
// (one LDS read, one complex FMA with the slot's class coefficient).  Up hops
// read whole source rows from global memory (coalesced; the hop list is
// uniform over the workgroup), in independent batches of eight, each with a
// uniform signed class coefficient.
struct KArgs {  // passed by value as kernel arguments (at most 4 KB)
  int dim_up, dim_dn, nc, j, nslots, m_max, chunks;
  double tol, norm_inf, U;
  const uint32_t* up_bits;
  const uint32_t* dn_bits;
  const double* eps_up;
  const double* eps_dn;
  const int32_t* up_ptr;      // [dim_up + 1]
  const uint32_t* up_hops;    // src | class << 16 | sign << 31
  const uint16_t* dn_tab;     // [dim_dn][MAXS] stage index (src + copy * (dim_dn + 1)), pad = dim_dn
  uint8_t slot_class[64];
  union {
    double coef[2 * kMaxNV * kMaxClasses];  // NV > 1: [v][c] complex
    double slot_coef_obs[2 * 64];           // NV = 1, observables: coefficient of every down slot at t_obs
  };
  double slot_coef[2 * 64];                // vector 0: coefficient of every down slot
  double up_coef[2 * 2 * kMaxClasses];     // vector 0: [c][sign] signed coefficient
  double coef_obs[2 * kMaxNV * kMaxClasses];  // [v][c] complex, observation time (obs modes)
  const void* x;
  void* y;
  const void* xprev;
  VecState* st;
  StepCtl* ctl;
  double* partials;
  const double* prev_partials;
  int prev_nblk;
  const double* alpha_partials;    // fused: the previous column pass's alpha partials
  int alpha_nblk, alpha_stride;
  const double* obs_row;           // fused j = 1: observables partials of the step's first apply
  int dim_up_rows;
  double* norm_out;                // fused: |u_j|^2 partial of every row
};

static_assert(kMaxNV * kMaxClasses == 64, "the single-vector observation coefficients share coef's storage");

// Threads per apply workgroup.  Long rows of single vectors use 1024 threads
// (fewer column passes per thread); short rows, interleaved blocks and the
// observables pass use 256 (more workgroups per CU, more registers per thread).
constexpr int kRowsLong = 2048;

// Per-quantity workgroup reduction (W waves, NV interleaved vectors):
// out[q * NV + v] = sum over the workgroup's threads of vector v, for q < nq.
// Each wave reduces every quantity with shuffles (static indices keep vals in
// registers), leaves its sums in lds[(w * nq + q) * NV + v] (lds holds at
// least W * nq * NV doubles), and after one
// barrier the first nq * NV threads add the W wave sums in a fixed order.
template <int NV, int W, int NQ>
__device__ __forceinline__ void block_partials_seq(const double (&vals)[NQ], int nq, double* lds, double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q < nq) {
      double v = vals[q];
#pragma unroll
      for (int off = 32; off >= NV; off >>= 1) v += __shfl_xor(v, off);
      if (lane < NV) lds[(w * nq + q) * NV + lane] = v;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < nq * NV) {
    const int q = t / NV, v = t % NV;
    double s = 0.0;
    for (int k = 0; k < W; ++k) s += lds[(k * nq + q) * NV + v];
    out[q * NV + v] = s;
  }
}

// UPH = false: row pass of the two-pass apply (diagonal and down hops only;
// in Lanczos mode the prologue still takes the Krylov decision, and the raw
// partial product is written for the column pass to finish).
// FUSE: row pass of a fused Lanczos iteration j >= 1 (forms u_j first; one
// extra workgroup for the recording and the early estimate, see below).
// GDN: rows too long for LDS (16 sites): the down hops read the row of x in
// global memory (it stays in L2) and decode sign and padding from the index.
template <typename R, int NV, int MODE, int MAXS, int BLK, bool UPH, bool FUSE, bool GDN>
__global__ __launch_bounds__(BLK) void k_apply(KArgs p) {
  using V = typename CT<R>::T;
  constexpr int kBlockA = BLK;
  constexpr int kWavesA = kBlockA / 64;
  constexpr bool kL = (MODE == M_LANCZOS || MODE == M_LANCZOS_OBS);
  constexpr bool kEpi = kL && UPH;  // Lanczos epilogue and alpha partials here
  constexpr bool kO = (MODE == M_LANCZOS_OBS || MODE == M_OBS);
  constexpr bool kW = (MODE != M_OBS);
  constexpr int kNQ = 1 + kObsQ;  // alpha, diag, docc, n2, Re <x|K(t_obs)|x>
  constexpr int kUB = 4;  // up hops gathered before the staging barrier (more costs registers)
  __shared__ double red[kWavesA * NV * (kO ? kNQ : 1) + kWavesA];
  __shared__ double sh_beta[kMaxNV];
  __shared__ V sh_slot[NV > 1 ? 64 * NV : 1];
  __shared__ V sh_up[NV > 1 ? 2 * kMaxClasses * NV : 1];
  __shared__ double2 sh_oslot[kO && NV > 1 ? 64 * NV : 1];    // observation-time coefficient per slot
  __shared__ double2 sh_oup[kO ? 2 * kMaxClasses * NV : 1];  // and per signed up-hop class

  const int tid = threadIdx.x;
  const int v = tid % NV;
  const int nc = p.nc;

  R sj = 1, bprev = 0;
  static_assert(!FUSE || (NV == 1 && MODE == M_LANCZOS && !UPH), "fused update: single-vector row pass");
  static_assert(!GDN || (NV == 1 && UPH && !FUSE), "global down-hop gathers: one-pass single vectors");
  R c_upd = 0;  // fused update: alpha_{j-1} s_{j-1}
  if (FUSE) {
    // Row pass of a fused iteration: finish u_j = w_{j-1} - alpha_{j-1} s_{j-1}
    // u_{j-1} while staging; its norm, and so the Krylov decision for m = j,
    // are taken by the column pass.
    if (p.ctl->all_done) return;
    const double al = reduce_column<kWavesA>(p.alpha_partials, p.alpha_nblk, p.alpha_stride, 0, red);
    if (blockIdx.x == gridDim.x - 1) {
      // The extra last workgroup records alpha_{j-1} and (j = 1) finalizes
      // the observables of the step's first vector: [diag, docc, n2,
      // down-hop part] from its row pass plus the up-hop part from its
      // column pass.  The estimate for m = j needs only T_j (alpha_{j-1} =
      // al, the rest recorded), not |u_j|.  When it is below tol the step
      // ends at m = j whatever |u_j| turns out to be: y^(j) and eps are
      // recorded here, and the column pass skips this iteration's apply and
      // only records |u_j| and the status.
      if (tid == 0 && p.st[0].status == 0) p.st[0].alpha[p.j - 1] = al;
      if (p.obs_row) {
        for (int t = 0; t < kObsQ; ++t) {
          double s2 = reduce_column<kWavesA>(p.obs_row, p.dim_up_rows, kObsQ, t, red);
          if (t == kObsQ - 1) s2 += reduce_column<kWavesA>(p.alpha_partials, p.alpha_nblk, p.alpha_stride, 1, red);
          if (tid == 0) p.st[0].obs[t] = s2;
        }
      }
      if (tid < 64) {
        VecState& S = p.st[0];
        bool stop = false;
        if (S.status == 0) {
          const double aj = tid < p.j - 1 ? S.alpha[tid] : (tid == p.j - 1 ? al : 0.0);
          double yr, yi;
          const double eps = wave_krylov_eps(p.j, aj, S.beta, S.tau, S.y, tid, yr, yi);
          stop = eps < p.tol;
          if (stop) {  // every lane has read y^(j-1): its reductions fed eps
            if (tid < p.j) {
              S.y[2 * tid] = yr;
              S.y[2 * tid + 1] = yi;
            }
            if (tid == 0) S.eps = eps;
          }
        }
        if (tid == 0) p.ctl->eps_stop = stop ? p.j : -1;
      }
      return;
    }
    c_upd = static_cast<R>(al * p.st[0].scale[p.j - 1]);
  } else if (kL) {
    if (p.ctl->all_done) return;
    // norm of the vector just completed (|u_j|, j >= 1) or of the step input;
    // a row pass needs it only in the workgroup that takes the decision (the
    // column pass reads the recorded value).  A one-pass apply takes the
    // decision in an extra last workgroup, so that no apply workgroup waits
    // for the estimate (a single round of workgroups would otherwise end with
    // the decider's estimate plus its apply).
    const bool decider = UPH ? blockIdx.x == gridDim.x - 1 : blockIdx.x == 0;
    if (UPH || decider) {
      for (int t = 0; t < NV; ++t) {
        const double s = reduce_column<kWavesA>(p.prev_partials, p.prev_nblk, NV, t, red);
        if (tid == 0) sh_beta[t] = sqrt(s);
      }
      __syncthreads();
      if (decider) krylov_decide<NV, kWavesA>(p.j, sh_beta, p.st, p.ctl, p.m_max, p.tol, p.norm_inf);
      if (UPH && decider) return;
    }
    if (p.j >= p.m_max) return;  // only the decision was needed
    if (UPH) {
      const double bv = sh_beta[v];
      sj = static_cast<R>(bv > 0.0 ? 1.0 / bv : 0.0);
      if (p.j > 0) bprev = static_cast<R>(bv * p.st[v].scale[p.j - 1]);
    }
  }

  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* xs = reinterpret_cast<V*>(smem_raw);
  const V* __restrict__ x = static_cast<const V*>(p.x);
  V* __restrict__ y = static_cast<V*>(p.y);
  const int rowlen = p.dim_dn * NV;       // complex elements of one tile row
  const int half = (p.dim_dn + 1) * NV;   // one staged copy incl. the zero slot
  // workgroup = (row a, column chunk); the chunks of one row are consecutive
  // logical blocks, so they run on one XCD and re-read the staged row from L2
  constexpr bool kExtra = FUSE || (kL && UPH);  // an extra last workgroup takes the decision
  const int lb = xcd_remap(blockIdx.x, kExtra ? gridDim.x - 1 : gridDim.x);
  const int a = lb / p.chunks;
  const int cw = (rowlen + p.chunks - 1) / p.chunks;
  const int qbeg = (lb % p.chunks) * cw;
  const int qend = min(rowlen, qbeg + cw);
  const int hb = p.up_ptr[a], hcnt = UPH ? p.up_ptr[a + 1] - hb : 0;
  const uint32_t ua = p.up_bits[a];
  const double ea = p.eps_up ? p.eps_up[a] : 0.0;
  const uint2* tab2 = reinterpret_cast<const uint2*>(p.dn_tab);
  constexpr int kQ2 = MAXS / 4;

  // Global loads of this thread's first column (table entries, the first
  // batch of up-hop sources, the previous Lanczos vector) are issued before
  // the row is staged, so their latency overlaps the staging.
  int q = qbeg + tid;
  uint2 ev[kQ2];
  uint32_t eu[kUB];
  V tu[kUB];
  V pv = V{0, 0};
  auto load_column = [&](int qq) {
    const int b = qq / NV;
#pragma unroll
    for (int k = 0; k < kQ2; ++k) ev[k] = tab2[(size_t)b * kQ2 + k];
#pragma unroll
    for (int k = 0; k < kUB; ++k) eu[k] = (k < hcnt) ? p.up_hops[hb + k] : 0u;
#pragma unroll
    for (int k = 0; k < kUB; ++k) tu[k] = (k < hcnt) ? x[(size_t)(eu[k] & 0xFFFFu) * rowlen + qq] : V{0, 0};
    if (kEpi && p.j > 0) pv = static_cast<const V*>(p.xprev)[(size_t)a * rowlen + qq];
  };
  if (q < qend) load_column(q);

  // stage +x, -x (zero slot at column dim_dn of each copy)
  if (FUSE) {
    // x holds w_{j-1}: form the row of u_j in place, stage it, sum |u_j|^2
    V* wr = static_cast<V*>(const_cast<void*>(p.x)) + (size_t)a * rowlen;
    const V* ur = static_cast<const V*>(p.xprev) + (size_t)a * rowlen;
    double n2 = 0.0;
    for (int t = tid; t < half; t += kBlockA) {
      V val = V{0, 0};
      if (t < rowlen) {
        const V u = ur[t];
        val = wr[t];
        val.x -= c_upd * u.x;
        val.y -= c_upd * u.y;
        wr[t] = val;
        n2 += (double)val.x * val.x + (double)val.y * val.y;
      }
      xs[t] = val;
      xs[half + t] = V{-val.x, -val.y};
    }
    const double rs = block_sum<kWavesA>(n2, red);
    if (tid == 0) p.norm_out[lb] = rs;
    if (!p.y) return;  // j = m_max: only the norm was needed
  } else if (!GDN) {
    const V* src = x + (size_t)a * rowlen;
    for (int t = tid; t < half; t += kBlockA) {
      const V val = (t < rowlen) ? src[t] : V{0, 0};
      xs[t] = val;
      xs[half + t] = V{-val.x, -val.y};
    }
  }
  const V* __restrict__ xrow = x + (size_t)a * rowlen;  // GDN: the row in global memory
  if (NV > 1) {
    for (int t = tid; t < 64 * NV; t += kBlockA) {
      const int s = t / NV, vv = t % NV;
      const int c = p.slot_class[s];
      sh_slot[t] = (s < p.nslots) ? V{static_cast<R>(p.coef[2 * (vv * nc + c)]),
                                       static_cast<R>(p.coef[2 * (vv * nc + c) + 1])}
                                  : V{0, 0};
    }
    for (int t = tid; t < 2 * nc * NV; t += kBlockA) {
      const int cs = t / NV, vv = t % NV, c = cs >> 1;
      const R sg = (cs & 1) ? R(-1) : R(1);
      sh_up[t] = V{sg * static_cast<R>(p.coef[2 * (vv * nc + c)]), sg * static_cast<R>(p.coef[2 * (vv * nc + c) + 1])};
    }
  }
  if (kO) {
    for (int t = tid; NV > 1 && t < 64 * NV; t += kBlockA) {
      const int s = t / NV, vv = t % NV;
      const int c = p.slot_class[s];
      sh_oslot[t] = (s < p.nslots) ? make_double2(p.coef_obs[2 * (vv * nc + c)], p.coef_obs[2 * (vv * nc + c) + 1])
                                   : make_double2(0.0, 0.0);
    }
    for (int t = tid; t < 2 * nc * NV; t += kBlockA) {
      const int cs = t / NV, vv = t % NV, c = cs >> 1;
      const double sg = (cs & 1) ? -1.0 : 1.0;
      sh_oup[t] = make_double2(sg * p.coef_obs[2 * (vv * nc + c)], sg * p.coef_obs[2 * (vv * nc + c) + 1]);
    }
  }
  __syncthreads();

  double q_alpha = 0.0, q_diag = 0.0, q_docc = 0.0, q_n2 = 0.0, q_hop = 0.0;

  while (q < qend) {
    const int b = q / NV;
    const uint32_t db = p.dn_bits[b];
    const double eb = p.eps_dn ? p.eps_dn[b] : 0.0;
    const V xv = GDN ? xrow[q] : xs[q];
    const double nd = static_cast<double>(__popc(ua & db));
    const double dg = p.U * nd + ea + eb;
    V acc = V{static_cast<R>(dg) * xv.x, static_cast<R>(dg) * xv.y};
    double2 ko = make_double2(0.0, 0.0);  // K(t_obs) x at this element (obs modes)
    if (kO) {
      const double m2 = (double)xv.x * xv.x + (double)xv.y * xv.y;
      q_diag += dg * m2;
      q_docc += nd * m2;
      q_n2 += m2;
    }
    // down hops: one LDS read and one complex FMA per slot, no branches
    // (slots past the string's hops read the zero slot with a zero coefficient)
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const uint32_t w2 = (s & 3) < 2 ? ev[s >> 2].x : ev[s >> 2].y;
      const uint32_t idx = (s & 1) ? (w2 >> 16) : (w2 & 0xFFFFu);
      V t;
      if (GDN) {  // index = src, src + dim_dn + 1 (negative hop), or dim_dn (pad)
        const uint32_t dd = static_cast<uint32_t>(p.dim_dn);
        const bool neg = idx > dd;
        const uint32_t src = neg ? idx - dd - 1 : idx;
        t = V{0, 0};
        if (src < dd) t = xrow[src];
        if (neg) t = V{-t.x, -t.y};
      } else {
        t = xs[idx * NV + v];
      }
      V cf;
      if (NV == 1) cf = V{static_cast<R>(p.slot_coef[2 * s]), static_cast<R>(p.slot_coef[2 * s + 1])};
      else cf = sh_slot[s * NV + v];
      acc = cfma(cf, t, acc);
      if (kO) {  // staged value carries the sign
        const double2 co = NV == 1 ? make_double2(p.slot_coef_obs[2 * s], p.slot_coef_obs[2 * s + 1])
                                   : sh_oslot[s * NV + v];
        ko = cfma(co, make_double2(t.x, t.y), ko);
      }
    }
    // up hops: whole source rows from global memory, uniform signed coefficients
    auto up_term = [&](uint32_t e, V t) {
      const int cs = static_cast<int>(((e >> 16) & 0xFFu) * 2u + (e >> 31));
      V cf;
      if (NV == 1) cf = V{static_cast<R>(p.up_coef[2 * cs]), static_cast<R>(p.up_coef[2 * cs + 1])};
      else cf = sh_up[cs * NV + v];
      acc = cfma(cf, t, acc);
      if (kO) ko = cfma(sh_oup[cs * NV + v], make_double2(t.x, t.y), ko);
    };
#pragma unroll
    for (int k = 0; k < kUB; ++k)
      if (k < hcnt) up_term(eu[k], tu[k]);
    for (int h0 = kUB; h0 < hcnt; h0 += 8) {
      uint32_t e[8];
      V t[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) e[k] = (h0 + k < hcnt) ? p.up_hops[hb + h0 + k] : 0u;
#pragma unroll
      for (int k = 0; k < 8; ++k) t[k] = (h0 + k < hcnt) ? x[(size_t)(e[k] & 0xFFFFu) * rowlen + q] : V{0, 0};
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (h0 + k < hcnt) up_term(e[k], t[k]);
    }
    if (kO) q_hop += (double)xv.x * ko.x + (double)xv.y * ko.y;  // Re conj(x) K x
    const size_t idx = (size_t)a * rowlen + q;
    V out = acc;
    if (kEpi) {
      out.x = out.x * sj - bprev * pv.x;
      out.y = out.y * sj - bprev * pv.y;
      // alpha_j = Re <s_j u_j, w>
      q_alpha += (double)sj * ((double)xv.x * out.x + (double)xv.y * out.y);
    }
    if (kW) y[idx] = out;
    q += kBlockA;
    if (q < qend) load_column(q);
  }

  // workgroup partials: [alpha] [diag, docc, n2, Re <x|K(t_obs)|x>]
  constexpr int nqL = kEpi ? 1 : 0;
  constexpr int nq = nqL + (kO ? kObsQ : 0);
  if (nq == 0) return;
  double vals[kNQ];
  if (kEpi) vals[0] = q_alpha;
  if (kO) {
    vals[nqL + 0] = q_diag;
    vals[nqL + 1] = q_docc;
    vals[nqL + 2] = q_n2;
    vals[nqL + 3] = q_hop;
  }
  block_partials_seq<NV, kWavesA>(vals, nq, red, p.partials + (size_t)lb * nq * NV);
}

template <typename R, int NV, int MODE, int MAXS, int BLK, bool UPH, bool FUSE, bool GDN = false>
hipError_t apply_t(const ApplyLaunch& L, int grid, size_t lds) {
  const DevBasis& db = *L.db;
  KArgs p;
  p.dim_up = db.dim_up;
  p.dim_dn = db.dim_dn;
  p.nc = db.nc;
  p.j = L.j;
  p.nslots = db.nslots;
  p.m_max = L.m_max;
  p.chunks = apply_chunks(db, L.prec, L.nv);
  // The fused row pass forms u_j in place over the whole row and writes one
  // norm partial per row: every row must belong to exactly one workgroup.
  if (FUSE && p.chunks != 1) return hipErrorInvalidValue;
  p.tol = L.tol;
  p.norm_inf = L.norm_inf;
  p.U = db.U;
  p.up_bits = db.up_bits;
  p.dn_bits = db.dn_bits;
  p.eps_up = db.eps_up;
  p.eps_dn = db.eps_dn;
  p.up_ptr = db.up_ptr;
  p.up_hops = db.up_hops;
  p.dn_tab = db.dn_tab;
  for (int s = 0; s < 64; ++s) p.slot_class[s] = db.slot_class[s];
  // the caller's coefficient arrays hold [nv][nc] complex pairs, no more
  if (NV > 1) pack_block_coefs(L.coef, L.nv, db.nc, p.coef, 2 * kMaxNV * kMaxClasses);
  else pack_slot_coefs(L.coef_obs, db.nc, db.slot_class, db.nslots, p.slot_coef_obs);
  pack_block_coefs(L.coef_obs, L.nv, db.nc, p.coef_obs, 2 * kMaxNV * kMaxClasses);
  pack_slot_coefs(L.coef, db.nc, db.slot_class, db.nslots, p.slot_coef);
  pack_signed_coefs(L.coef, db.nc, kMaxClasses, p.up_coef);
  p.x = L.x;
  p.y = L.y;
  p.xprev = L.xprev;
  p.st = L.st;
  p.ctl = L.ctl;
  // the row pass of a two-pass apply with observables has its own partials
  constexpr bool kObsMode = (MODE == M_LANCZOS_OBS || MODE == M_OBS);
  p.partials = (!UPH && kObsMode) ? L.row_obs : L.partials;
  p.prev_partials = L.prev_partials;
  p.prev_nblk = L.prev_nblk;
  p.alpha_partials = L.alpha_partials;
  p.alpha_nblk = L.alpha_nblk;
  p.alpha_stride = L.alpha_stride;
  p.obs_row = L.obs_row;
  p.dim_up_rows = db.dim_up;
  p.norm_out = L.norm_partials;
  auto fn = k_apply<R, NV, MODE, MAXS, BLK, UPH, FUSE, GDN>;
  // dynamic LDS above the 64 KB default must be opted into (CU total 160 KB);
  // once per kernel, also when host threads launch it concurrently
  static const int max_dyn = dyn_lds_opt_in(reinterpret_cast<const void*>(fn));
  if (lds > static_cast<size_t>(max_dyn)) return hipErrorInvalidValue;
  // fused row pass: one more workgroup for the early estimate; one-pass
  // Lanczos apply: one more for the Krylov decision
  constexpr bool kExtra = FUSE || ((MODE == M_LANCZOS || MODE == M_LANCZOS_OBS) && UPH);
  return launch_ev(fn, kExtra ? grid + 1 : grid, BLK, lds, L.stream, L.ev_start, L.ev_stop, p);
}

template <typename R, int NV, int MODE, int BLK, bool UPH = true, bool FUSE = false>
hipError_t apply_s(const ApplyLaunch& L, int grid, size_t lds) {
  switch (L.db->maxs_pad) {
    case 4: return apply_t<R, NV, MODE, 4, BLK, UPH, FUSE>(L, grid, lds);
    case 8: return apply_t<R, NV, MODE, 8, BLK, UPH, FUSE>(L, grid, lds);
    case 12: return apply_t<R, NV, MODE, 12, BLK, UPH, FUSE>(L, grid, lds);
    case 16: return apply_t<R, NV, MODE, 16, BLK, UPH, FUSE>(L, grid, lds);
    case 20: return apply_t<R, NV, MODE, 20, BLK, UPH, FUSE>(L, grid, lds);
    case 24: return apply_t<R, NV, MODE, 24, BLK, UPH, FUSE>(L, grid, lds);
    case 32: return apply_t<R, NV, MODE, 32, BLK, UPH, FUSE>(L, grid, lds);
    case 48: return apply_t<R, NV, MODE, 48, BLK, UPH, FUSE>(L, grid, lds);
    case 64: return apply_t<R, NV, MODE, 64, BLK, UPH, FUSE>(L, grid, lds);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Column pass of the two-pass apply (one vector).  A workgroup owns CW
// consecutive columns b0.. of the tile and stages them for every up string a
// in LDS as +x, -x and a zero row (layout [copy][a][CW]), so an up hop is
// one LDS read at an index that carries its fermion sign, exactly like the
// down hops of the row pass.  Each thread finishes elements (a, b): it adds
// the up hops (padded, class-sorted slots, coefficients in SGPRs) to the row
// pass's partial product in y and, in Lanczos mode, applies the epilogue and
// accumulates alpha partials.  Every x element is read from memory once per
// pass instead of once per up hop.
struct ColArgs {
  int dim_up, dim_dn, j, m_max;
  const double* norm_partials;  // fused: |u_j|^2 per row [dim_up]
  double tol, norm_inf;
  const uint16_t* up_tab;   // [dim_up][MAXS]
  double slot_coef[2 * 64]; // coefficient of every up slot (complex)
  double slot_coef_obs[2 * 64];  // the same at the observation time (observables mode)
  const void* x;
  void* y;                  // in: row-pass partial product, out: result
  const void* xprev;
  VecState* st;
  StepCtl* ctl;
  double* partials;         // Lanczos: [grid][alpha (, Re <x|K_up(t_obs)|x>)]
};

// FUSE: the row pass formed u_j; reduce its norm here and take the decision.
// ONE: a single staged copy (+x and the zero row; tiles whose two copies do
// not fit LDS): a negative hop's index src + dim_up + 1 reads +x and negates.
template <typename R, int MODE, int MAXS, int BLK, bool FUSE, bool ONE, int CW>
__global__ __launch_bounds__(BLK) void k_colpass(ColArgs p) {
  using V = typename CT<R>::T;
  constexpr bool kL = MODE == M_LANCZOS || MODE == M_LANCZOS_OBS;
  constexpr bool kO = MODE == M_LANCZOS_OBS;
  constexpr int kW = BLK / 64;
  __shared__ double red[2 * kW];
  __shared__ double sh_b[1];
  R sj = 1, bprev = 0;
  if (kL) {
    if (p.ctl->all_done) return;
    double bv;
    if (FUSE) {
      // |u_j| from the row pass's partials.  An extra last workgroup takes
      // the decision for m = j alongside the column blocks (a single round of
      // workgroups: the decision would otherwise add to the kernel's time).
      // When the row pass already found the estimate for m = j below tol,
      // the step ends here and the column blocks have nothing to do.
      const bool decide = blockIdx.x == gridDim.x - 1;
      const bool ends = p.ctl->eps_stop == p.j;
      if (ends && !decide) return;
      const double s2 = reduce_column<kW>(p.norm_partials, p.dim_up, 1, 0, red);
      bv = sqrt(s2);
      if (decide) {
        if (ends) {
          if (threadIdx.x == 0) krylov_end_at(p.j, bv, p.st[0], p.ctl, p.tol, p.norm_inf);
          return;
        }
        if (threadIdx.x == 0) sh_b[0] = bv;
        __syncthreads();
        krylov_decide<1, kW>(p.j, sh_b, p.st, p.ctl, p.m_max, p.tol, p.norm_inf);
        return;
      }
    } else {
      // |u_j| as recorded by the row pass's decision (beta0 at j = 0)
      const VecState& S = p.st[0];
      bv = p.j == 0 ? S.beta0 : S.beta[p.j - 1];
    }
    if (p.j >= p.m_max) return;
    sj = static_cast<R>(bv > 0.0 ? 1.0 / bv : 0.0);
    if (p.j > 0) bprev = static_cast<R>(bv * p.st[0].scale[p.j - 1]);
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V* xs = reinterpret_cast<V*>(smem_raw);
  const int nwork = FUSE ? gridDim.x - 1 : gridDim.x;  // column blocks
  const int lb = xcd_remap(blockIdx.x, nwork);
  const int b0 = lb * CW;
  const V* __restrict__ x = static_cast<const V*>(p.x);
  V* __restrict__ y = static_cast<V*>(p.y);
  const int half = (p.dim_up + 1) * CW;
  for (int t = threadIdx.x; t < half; t += BLK) {
    const int a = t / CW, c = t % CW;
    V v = V{0, 0};
    if (a < p.dim_up && b0 + c < p.dim_dn) v = x[(size_t)a * p.dim_dn + b0 + c];
    xs[t] = v;
    if (!ONE) xs[half + t] = V{-v.x, -v.y};
  }
  __syncthreads();
  const uint2* tab2 = reinterpret_cast<const uint2*>(p.up_tab);
  constexpr int kQ2 = MAXS / 4;
  double q_alpha = 0.0, q_hop = 0.0;
  for (int q = threadIdx.x; q < p.dim_up * CW; q += BLK) {
    const int a = q / CW, c = q % CW;
    if (b0 + c >= p.dim_dn) continue;
    uint2 ev[kQ2];
#pragma unroll
    for (int k = 0; k < kQ2; ++k) ev[k] = tab2[(size_t)a * kQ2 + k];
    const size_t o = (size_t)a * p.dim_dn + b0 + c;
    V acc = y[o];
    V pv = V{0, 0};
    if (kL && p.j > 0) pv = static_cast<const V*>(p.xprev)[o];
    double2 ko = make_double2(0.0, 0.0);  // up-hop part of K(t_obs) x (observables mode)
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const uint32_t w2 = (s & 3) < 2 ? ev[s >> 2].x : ev[s >> 2].y;
      const uint32_t idx = (s & 1) ? (w2 >> 16) : (w2 & 0xFFFFu);
      V t;
      if (ONE) {  // index = src, src + dim_up + 1 (negative hop), or dim_up (the zero row)
        const uint32_t du = static_cast<uint32_t>(p.dim_up);
        const bool neg = idx > du;
        t = xs[(neg ? idx - du - 1 : idx) * CW + c];
        if (neg) t = V{-t.x, -t.y};
      } else {
        t = xs[idx * CW + c];
      }
      const V cf = V{static_cast<R>(p.slot_coef[2 * s]), static_cast<R>(p.slot_coef[2 * s + 1])};
      acc = cfma(cf, t, acc);
      if (kO) ko = cfma(make_double2(p.slot_coef_obs[2 * s], p.slot_coef_obs[2 * s + 1]), make_double2(t.x, t.y), ko);
    }
    V out = acc;
    if (kL) {
      const V xv = xs[a * CW + c];
      if (kO) q_hop += (double)xv.x * ko.x + (double)xv.y * ko.y;
      out.x = out.x * sj - bprev * pv.x;
      out.y = out.y * sj - bprev * pv.y;
      q_alpha += (double)sj * ((double)xv.x * out.x + (double)xv.y * out.y);
    }
    y[o] = out;
  }
  if (kO) {
    const double vals[2] = {q_alpha, q_hop};
    block_partials_seq<1, kW>(vals, 2, red, p.partials + 2 * lb);
  } else if (kL) {
    const double vals[1] = {q_alpha};
    block_partials_seq<1, kW>(vals, 1, red, p.partials + lb);
  }
}

template <typename R, int MODE, int MAXS, bool FUSE, bool ONE, int CW>
hipError_t colpass_t(const ApplyLaunch& L, int* pgrid) {
  const DevBasis& db = *L.db;
  constexpr int BLK = 1024;
  ColArgs p;
  p.dim_up = db.dim_up;
  p.dim_dn = db.dim_dn;
  p.j = L.j;
  p.m_max = L.m_max;
  p.norm_partials = L.norm_partials;
  p.tol = L.tol;
  p.norm_inf = L.norm_inf;
  p.up_tab = db.up_tab;
  pack_slot_coefs(L.coef, db.nc, db.up_slot_class, db.up_nslots, p.slot_coef);
  pack_slot_coefs(L.coef_obs, db.nc, db.up_slot_class, db.up_nslots, p.slot_coef_obs);
  p.x = L.x;
  p.y = L.y;
  p.xprev = L.xprev;
  p.st = L.st;
  p.ctl = L.ctl;
  p.partials = L.partials;
  const int prec = sizeof(R) == 8 ? 0 : 1;
  if (colpass_width(db, prec) != CW || colpass_single(db, prec) != ONE) return hipErrorInvalidValue;
  const int grid = colpass_grid(db, prec);
  const size_t lds = colpass_lds_bytes(db, prec);
  auto fn = k_colpass<R, MODE, MAXS, BLK, FUSE, ONE, CW>;
  static const int max_dyn = dyn_lds_opt_in(reinterpret_cast<const void*>(fn));
  if (lds > static_cast<size_t>(max_dyn)) return hipErrorInvalidValue;
  if (pgrid) *pgrid = grid;
  // fused: one more workgroup for the Krylov decision
  return launch_ev(fn, FUSE ? grid + 1 : grid, BLK, lds, L.stream, L.ev2_start, L.ev2_stop, p);
}

template <typename R, int MODE, bool FUSE, bool ONE, int CW>
hipError_t colpass_w(const ApplyLaunch& L, int* pgrid) {
  switch (L.db->up_maxs_pad) {
    case 4: return colpass_t<R, MODE, 4, FUSE, ONE, CW>(L, pgrid);
    case 8: return colpass_t<R, MODE, 8, FUSE, ONE, CW>(L, pgrid);
    case 12: return colpass_t<R, MODE, 12, FUSE, ONE, CW>(L, pgrid);
    case 16: return colpass_t<R, MODE, 16, FUSE, ONE, CW>(L, pgrid);
    case 20: return colpass_t<R, MODE, 20, FUSE, ONE, CW>(L, pgrid);
    case 24: return colpass_t<R, MODE, 24, FUSE, ONE, CW>(L, pgrid);
    case 32: return colpass_t<R, MODE, 32, FUSE, ONE, CW>(L, pgrid);
    case 48: return colpass_t<R, MODE, 48, FUSE, ONE, CW>(L, pgrid);
    case 64: return colpass_t<R, MODE, 64, FUSE, ONE, CW>(L, pgrid);
    default: return hipErrorInvalidValue;
  }
}

// staging variants: kColW columns as +x and -x, kColW columns as +x alone,
// 2 columns as +x alone (the first that fits)
template <typename R, int MODE, bool FUSE = false>
hipError_t colpass_s(const ApplyLaunch& L, int* pgrid) {
  const int prec = sizeof(R) == 8 ? 0 : 1;
  if (colpass_width(*L.db, prec) == 2) return colpass_w<R, MODE, FUSE, true, 2>(L, pgrid);
  return colpass_single(*L.db, prec) ? colpass_w<R, MODE, FUSE, true, kColW>(L, pgrid)
                                     : colpass_w<R, MODE, FUSE, false, kColW>(L, pgrid);
}

template <typename R, int MODE, int BLK>
hipError_t apply_gdn_s(const ApplyLaunch& L, int grid) {
  switch (L.db->maxs_pad) {
    case 4: return apply_t<R, 1, MODE, 4, BLK, true, false, true>(L, grid, 0);
    case 8: return apply_t<R, 1, MODE, 8, BLK, true, false, true>(L, grid, 0);
    case 12: return apply_t<R, 1, MODE, 12, BLK, true, false, true>(L, grid, 0);
    case 16: return apply_t<R, 1, MODE, 16, BLK, true, false, true>(L, grid, 0);
    case 20: return apply_t<R, 1, MODE, 20, BLK, true, false, true>(L, grid, 0);
    case 24: return apply_t<R, 1, MODE, 24, BLK, true, false, true>(L, grid, 0);
    case 32: return apply_t<R, 1, MODE, 32, BLK, true, false, true>(L, grid, 0);
    case 48: return apply_t<R, 1, MODE, 48, BLK, true, false, true>(L, grid, 0);
    case 64: return apply_t<R, 1, MODE, 64, BLK, true, false, true>(L, grid, 0);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, int NV>
hipError_t apply_mode(const ApplyLaunch& L, int grid, size_t lds, int* pgrid) {
  if (pgrid) *pgrid = grid;
  if constexpr (NV == 1) {
    if (apply_global_rows(*L.db, L.prec, 1)) {  // a row does not fit LDS
      if (L.mode == kPlain) return apply_gdn_s<R, M_PLAIN, 1024>(L, grid);
      if (L.mode == kObsOnly) return apply_gdn_s<R, M_OBS, 256>(L, grid);
      if (L.obs) return apply_gdn_s<R, M_LANCZOS_OBS, 256>(L, grid);
      return apply_gdn_s<R, M_LANCZOS, 1024>(L, grid);
    }
    const bool longrow = L.db->dim_dn >= kRowsLong;
    if (apply_two_pass(*L.db, L.prec, 1, L.mode, L.obs)) {
      hipError_t e;
      if (L.mode == kPlain) {
        e = longrow ? apply_s<R, 1, M_PLAIN, 1024, false>(L, grid, lds)
                    : apply_s<R, 1, M_PLAIN, 256, false>(L, grid, lds);
        return e != hipSuccess ? e : colpass_s<R, M_PLAIN>(L, pgrid);
      }
      if (L.obs) {  // observables of the step's first vector
        e = apply_s<R, 1, M_LANCZOS_OBS, 256, false>(L, grid, lds);
        return e != hipSuccess ? e : colpass_s<R, M_LANCZOS_OBS>(L, pgrid);
      }
      if (L.fuse) {
        e = longrow ? apply_s<R, 1, M_LANCZOS, 1024, false, true>(L, grid, lds)
                    : apply_s<R, 1, M_LANCZOS, 256, false, true>(L, grid, lds);
        return e != hipSuccess ? e : colpass_s<R, M_LANCZOS, true>(L, pgrid);
      }
      e = longrow ? apply_s<R, 1, M_LANCZOS, 1024, false>(L, grid, lds)
                  : apply_s<R, 1, M_LANCZOS, 256, false>(L, grid, lds);
      return e != hipSuccess ? e : colpass_s<R, M_LANCZOS>(L, pgrid);
    }
    if (longrow) {
      if (L.mode == kPlain) return apply_s<R, 1, M_PLAIN, 1024>(L, grid, lds);
      if (L.mode != kObsOnly && !L.obs) return apply_s<R, 1, M_LANCZOS, 1024>(L, grid, lds);
    }
  }
  if (L.mode == kPlain) return apply_s<R, NV, M_PLAIN, 256>(L, grid, lds);
  if (L.mode == kObsOnly) return apply_s<R, NV, M_OBS, 256>(L, grid, lds);
  if (L.obs) return apply_s<R, NV, M_LANCZOS_OBS, 256>(L, grid, lds);
  return apply_s<R, NV, M_LANCZOS, 256>(L, grid, lds);
}

template <typename R>
hipError_t apply_nv(const ApplyLaunch& L, int grid, size_t lds, int* pgrid) {
  switch (L.nv) {
    case 1: return apply_mode<R, 1>(L, grid, lds, pgrid);
    case 2: return apply_mode<R, 2>(L, grid, lds, pgrid);
    case 4: return apply_mode<R, 4>(L, grid, lds, pgrid);
    case 8: return apply_mode<R, 8>(L, grid, lds, pgrid);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dev
}  // namespace hub
