// C ABI of the library (include/hub.h): argument validation, device tables,
// workspace, and the host orchestration of the Krylov midpoint steps.
#include "hub.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <array>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <utility>
#include <vector>

#include "basis.h"
#include "host_eig.h"
#include "kernels.h"
#include "members.h"
#include "mlp.h"
#include "resident.h"

using hub::CombineLog;
using hub::DevBasis;
using hub::kMaxClasses;
using hub::kMaxNV;
using hub::kMMax;
using hub::kObsQ;
using hub::StepCtl;
using hub::VecState;

namespace {

thread_local std::string g_err;

hub_status fail(hub_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HUB_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(e_ == hipErrorOutOfMemory ? HUB_E_NOMEM : HUB_E_DEVICE,               \
                  std::string(#call) + ": " + hipGetErrorString(e_));                    \
  } while (0)

size_t elem_bytes(hub_prec p) { return p == HUB_C128 ? 16 : 8; }

constexpr int kCtrlMaxChunk = 256;

// Static device scratch of hub_observables_noalloc (one copy per device, held
// until the process ends).  Host code never uses this name as an address: it
// passes the pointer that hipGetSymbolAddress returned for the device.
constexpr size_t kNoAllocScratchBytes = size_t(512) << 10;
// Event pool of the apply timing: created when timing is enabled, and read
// back (elapsed times) only when fewer than kProfLowWater events are left.
constexpr size_t kProfPool = 8192, kProfLowWater = 512;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// One timed apply: start/stop events of its kernel(s) until they are read
// (then returned to the pool), its kernel time, and whether it did work.
struct ProfSample {
  std::array<hipEvent_t, 4> ev{nullptr, nullptr, nullptr, nullptr};
  double ms = 0.0;
  int n = -1, sub = 0, j = 0;  // Lanczos launch: step, substep, iteration (n = -1: plain apply)
  bool fused = false;          // fused two-pass iteration
  int worked = 1;              // 0: launched past the Krylov decision (exits at once); -1: not yet known
};

// Device workspace of one propagation lane.  The handle's own lane (w)
// serves every entry point; a propagation of several vector groups runs the
// groups on up to kMaxLanes lanes at once, each extra lane with its own
// workspace and stream (HIP keeps the per-lane kernels independent, so
// latency-bound applies of different groups overlap on the GPU).
struct Work {
  void* slots = nullptr;
  size_t slots_bytes = 0;
  void* blockbuf = nullptr;
  size_t blockbuf_bytes = 0;
  void** slot_ptrs = nullptr;     // device [kMMax + 2]
  VecState* st = nullptr;         // device [kMaxNV]
  StepCtl* ctl = nullptr;         // device
  StepCtl* h_ctl = nullptr;       // pinned host
  double* partials = nullptr;
  size_t partials_bytes = 0;
  double* partials_e = nullptr;   // partial sums of the elementwise kernels
  size_t partials_e_bytes = 0;
  double* scal = nullptr;         // device scalars [kMMax*2 + 16]
  double* rcoef = nullptr;        // device re-orthogonalisation coefficients [kMMax + 1][kMaxNV] complex
  hipStream_t stream = nullptr;   // extra lanes: their own stream (lane 0 runs on the caller's)
  void** h_ptrs = nullptr;        // pinned host mirror of slot_ptrs (uploaded without a wait)
  void* dlog = nullptr;           // device step logs and observables of a propagation (grow only)
  size_t dlog_bytes = 0;
  double* dobs = nullptr;
  size_t dobs_bytes = 0;
  hub_controller_stats cstats{};  // schedule counters of this lane's runs (folded into the handle's)
};

constexpr int kMaxLanes = 4;
// Blocks on the two-pass block kernels take fused Lanczos iterations up to
// this many states (measured, member-steps/s fused vs with an update kernel:
// 8-site blocks of 8 122 k vs 114 k, 10-site Green's-function members per
// sector 67.6 k vs 66.2 k; 12-site c64 blocks of 4 8,569 vs 9,135 and
// 14-site 454 vs 485 lose).
constexpr int64_t kBlockFuseMaxDim = 65536;
// Extra lanes are used only while all lanes' Krylov workspaces together stay
// below this many bytes of device memory.
constexpr size_t kLaneWorkBudget = size_t(48) << 30;

struct hub_basis_s {
  hub::Basis B;
  DevBasis D;
  int device = 0;
  std::vector<void*> allocs;  // table allocations
  Work w;                     // lane 0
  std::vector<std::unique_ptr<Work>> lanes;  // extra lanes, created on demand
  int rows_c128 = 1, rows_c64 = 1;
  // learned Krylov controller
  bool ctrl_on = false, ctrl_loaded = false;
  int ctrl_chunk = 16, ctrl_margin = 1;
  float* ctrl_params = nullptr;  // device [HUB_MLP_NPARAM]
  float* ctrl_feat = nullptr;    // device [kCtrlMaxChunk * kMaxNV][HUB_MLP_IN]
  float* ctrl_out = nullptr;     // device [kCtrlMaxChunk * kMaxNV][HUB_MLP_OUT]
  float* ctrl_hfeat = nullptr;   // pinned host copies of the two
  float* ctrl_hout = nullptr;
  hub_controller_stats cstats{};
  int sched_chunk = 32, sched_margin = 1;  // default chunked schedule (chunk 0: synchronous)
  // tuned vectors per group per precision (-1: the built-in rule): hub_apply_H
  // and hub_propagate with several vectors; force_group (> 0) overrides both
  // while hub_tune measures
  int apply_group[2] = {-1, -1};
  int prop_group[2] = {-1, -1};
  int prop_group_large[2] = {-1, -1};  // hub_propagate with more than kMaxNV vectors
  int force_group = 0;
  // Green's functions: -1 automatic, 0 per-sector groups, 1 persistent members
  int greens_path = -1;
  // hub_propagate: -1 automatic, 0 launches per Lanczos iteration, 1 resident stepper
  int prop_path = -1;
  // profiling of the apply kernel
  bool prof = false;
  int prof_period = 1;
  int64_t prof_count = 0;
  std::vector<ProfSample> prof_samples;
  std::vector<hipEvent_t> ev_free;
  double prof_bytes = 0.0;
};

namespace {

hub_status dev_alloc(hub_basis h, void** p, size_t bytes) {
  HUB_HIP(hipMalloc(p, bytes == 0 ? 16 : bytes));
  return HUB_OK;
}

template <typename T>
hub_status upload(hub_basis h, T** dst, const std::vector<T>& src) {
  if (src.empty()) {
    *dst = nullptr;
    return HUB_OK;
  }
  void* p = nullptr;
  hub_status s = dev_alloc(h, &p, src.size() * sizeof(T));
  if (s != HUB_OK) return s;
  h->allocs.push_back(p);
  HUB_HIP(hipMemcpy(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  *dst = static_cast<T*>(p);
  return HUB_OK;
}

int pick_rows(const hub_basis, int) { return 1; }  // one tile row per apply workgroup

// Fixed-size part of a lane's workspace (the rest grows in ensure_workspace);
// an extra lane also gets its own stream (default priority).
hub_status work_init(Work& W, bool own_stream) {
  if (hipMalloc(reinterpret_cast<void**>(&W.slot_ptrs), (kMMax + 2) * sizeof(void*)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&W.st), kMaxNV * sizeof(VecState)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&W.ctl), sizeof(StepCtl)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&W.scal), (2 * kMMax + 64) * sizeof(double) * 2) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&W.rcoef), (kMMax + 1) * kMaxNV * 2 * sizeof(double)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&W.h_ctl), sizeof(StepCtl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&W.h_ptrs), (kMMax + 2) * sizeof(void*), hipHostMallocDefault) !=
          hipSuccess)
    return fail(HUB_E_NOMEM, "workspace allocation failed");
  if (hipMemset(W.ctl, 0, sizeof(StepCtl)) != hipSuccess || hipMemset(W.st, 0, kMaxNV * sizeof(VecState)) != hipSuccess)
    return fail(HUB_E_DEVICE, "workspace initialisation failed");
  if (own_stream && hipStreamCreateWithFlags(&W.stream, hipStreamNonBlocking) != hipSuccess)
    return fail(HUB_E_DEVICE, "stream creation failed");
  return HUB_OK;
}

void work_free(Work& W) {
  if (W.slots) (void)hipFree(W.slots);
  if (W.blockbuf) (void)hipFree(W.blockbuf);
  if (W.slot_ptrs) (void)hipFree(W.slot_ptrs);
  if (W.st) (void)hipFree(W.st);
  if (W.ctl) (void)hipFree(W.ctl);
  if (W.partials_e) (void)hipFree(W.partials_e);
  if (W.scal) (void)hipFree(W.scal);
  if (W.rcoef) (void)hipFree(W.rcoef);
  if (W.partials) (void)hipFree(W.partials);
  if (W.h_ctl) (void)hipHostFree(W.h_ctl);
  if (W.h_ptrs) (void)hipHostFree(W.h_ptrs);
  if (W.dlog) (void)hipFree(W.dlog);
  if (W.dobs) (void)hipFree(W.dobs);
  if (W.stream) (void)hipStreamDestroy(W.stream);
  W = Work{};
}

hub_status ensure_workspace(hub_basis h, Work& W, size_t slot_bytes, int nslots, size_t blockbuf_bytes) {
  const size_t need = slot_bytes * static_cast<size_t>(nslots);
  if (need > W.slots_bytes) {
    if (W.slots) HUB_HIP(hipFree(W.slots));
    W.slots = nullptr;
    W.slots_bytes = 0;
    HUB_HIP(hipMalloc(&W.slots, need));
    W.slots_bytes = need;
  }
  if (blockbuf_bytes > W.blockbuf_bytes) {
    if (W.blockbuf) HUB_HIP(hipFree(W.blockbuf));
    W.blockbuf = nullptr;
    W.blockbuf_bytes = 0;
    HUB_HIP(hipMalloc(&W.blockbuf, blockbuf_bytes));
    W.blockbuf_bytes = blockbuf_bytes;
  }
  // partial sums of an apply: grid * (1 + kObsQ) * nv doubles at most
  // (also the CGS inner-product partials: elem_grid * (kMMax + 1) * 2 * nv)
  size_t pb = static_cast<size_t>(1024) * (kMMax + 1) * 2 * kMaxNV * sizeof(double);
  for (int pr = 0; pr < 2; ++pr)
    for (int nv = 1; nv <= kMaxNV; nv *= 2)
      pb = std::max(pb, static_cast<size_t>(hub::apply_grid(h->D, pr, nv)) * (1 + kObsQ) * nv * sizeof(double));
  // two-pass regions: column-pass partials, row-pass obs partials, row norms
  const int cgmax = std::max(hub::colpass_grid(h->D, 0), hub::colpass_grid(h->D, 1));
  pb = std::max(pb, (2 * static_cast<size_t>(cgmax) +
                     static_cast<size_t>(h->D.dim_up) * (kObsQ + 1)) * sizeof(double));
  // block two-pass: column-pass partials [dim_dn][2][nv], row-pass obs partials [dim_up][kObsQ][nv],
  // fused row norms [dim_up][nv]
  pb = std::max(pb, (2 * static_cast<size_t>(h->D.dim_dn) + static_cast<size_t>(h->D.dim_up) * (kObsQ + 1)) *
                        kMaxNV * sizeof(double));
  if (pb > W.partials_bytes) {
    if (W.partials) HUB_HIP(hipFree(W.partials));
    W.partials = nullptr;
    W.partials_bytes = 0;
    HUB_HIP(hipMalloc(&W.partials, pb));
    W.partials_bytes = pb;
  }
  // elementwise partials: elem_grid (<= 1024) rows of up to 2 * 64 columns
  const size_t pe = static_cast<size_t>(1024) * 2 * 64 * sizeof(double);
  if (pe > W.partials_e_bytes) {
    if (W.partials_e) HUB_HIP(hipFree(W.partials_e));
    W.partials_e = nullptr;
    W.partials_e_bytes = 0;
    HUB_HIP(hipMalloc(&W.partials_e, pe));
    W.partials_e_bytes = pe;
  }
  return HUB_OK;
}

hub_status ensure_workspace(hub_basis h, size_t slot_bytes, int nslots, size_t blockbuf_bytes) {
  return ensure_workspace(h, h->w, slot_bytes, nslots, blockbuf_bytes);
}

void coef_for(const hub::Basis& B, double A, double* out /* 2*nc */) {
  for (size_t c = 0; c < B.classes.size(); ++c) {
    const double t = B.classes[c].t, d = B.classes[c].d;
    out[2 * c] = -t * std::cos(A * d);
    out[2 * c + 1] = -t * std::sin(A * d);
  }
}

double pulse_value(const hub_pulse& p, double t) {
  const double s = t - p.t0;
  const double env = std::exp(-s * s / (2.0 * p.sigma * p.sigma));
  if (p.kind == 0) return p.A0 * env * std::sin(p.omega * s);
  return p.A0 * (std::cos(p.omega * s) - p.b) * env;
}

// dA/dt of pulse_value.
double pulse_deriv(const hub_pulse& p, double t) {
  const double s = t - p.t0;
  const double is2 = 1.0 / (p.sigma * p.sigma);
  const double env = std::exp(-0.5 * s * s * is2);
  if (p.kind == 0) return p.A0 * env * (p.omega * std::cos(p.omega * s) - s * is2 * std::sin(p.omega * s));
  return p.A0 * env * (-p.omega * std::sin(p.omega * s) - s * is2 * (std::cos(p.omega * s) - p.b));
}

// Controller features of one (step, vector) row: pulse at the step's
// midpoint, tau |H|_inf, the a-posteriori estimates of the last four finished
// steps (newest first, NaN where there is none) and the last finished step's
// Krylov dimension (-1 if none).
void ctrl_features(double A, double dA, double tau_norm, const double* eps_hist, int m_last, double tol, int m_hint,
                   float* x) {
  x[0] = static_cast<float>(A);
  x[1] = static_cast<float>(dA / 10.0);
  x[2] = static_cast<float>(tau_norm);
  for (int k = 0; k < 4; ++k) {
    const double e = eps_hist[k];
    const double l = std::isnan(e) ? std::log10(tol) : std::log10(std::max(e, 1e-40));
    x[3 + k] = static_cast<float>(l / 10.0);
  }
  const int m = m_last >= 0 ? m_last : (m_hint > 0 ? m_hint : 8);
  x[7] = static_cast<float>(m / 10.0);
}

// Pulse values the controller needs, per (step, vector) of a group.
struct CtrlInputs {
  std::vector<double> A_mid, dA_mid;  // [n * nv + v]
};

hub_status check_pulse(const hub_pulse& p) {
  if (p.kind != 0 && p.kind != 1) return fail(HUB_E_INVALID, "pulse kind must be 0 or 1");
  if (!(p.sigma > 0.0) || !std::isfinite(p.A0) || !std::isfinite(p.omega) || !std::isfinite(p.t0) ||
      !std::isfinite(p.b))
    return fail(HUB_E_INVALID, "pulse parameters must be finite with sigma > 0");
  return HUB_OK;
}

hub_status check_opts(const hub_krylov_opts& o) {
  if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(HUB_E_INVALID, "opts.tol must be > 0");
  if (o.m_max < 1 || o.m_max > kMMax) return fail(HUB_E_INVALID, "opts.m_max must be in 1..60");
  if (o.substeps < 1) return fail(HUB_E_INVALID, "opts.substeps must be >= 1");
  if (o.reorth != 0 && o.reorth != 1) return fail(HUB_E_INVALID, "opts.reorth must be 0 or 1");
  if (o.m_hint < 0) return fail(HUB_E_INVALID, "opts.m_hint must be >= 0");
  if (o.scheme != 0 && o.scheme != 1) return fail(HUB_E_INVALID, "opts.scheme must be 0 or 1");
  return HUB_OK;
}

// Exponentials per step of the scheme, and the Krylov solves per step.
int scheme_exps(const hub_krylov_opts& o) { return o.scheme == 1 ? 2 : 1; }
int solves_per_step(const hub_krylov_opts& o) { return o.substeps * scheme_exps(o); }

// Fourth-order commutator-free exponential (two exponentials per step): Gauss
// nodes c_{1,2} = 1/2 -+ sqrt(3)/6 and weights a_{1,2} = (3 -+ 2 sqrt(3))/12;
// the step is exp(-i dt (a1 H1 + a2 H2)) exp(-i dt (a2 H1 + a1 H2)) (right
// factor first).  Since a1 + a2 = 1/2 each factor is exp(-i (dt/2) H_eff)
// with the same diagonal and hop coefficients 2 (a H1 + b H2) per class.
constexpr double kCf4C1 = 0.5 - 0.28867513459481287;  // sqrt(3)/6
constexpr double kCf4C2 = 0.5 + 0.28867513459481287;
constexpr double kCf4A1 = (3.0 - 3.4641016151377546) / 12.0;  // 2 sqrt(3)
constexpr double kCf4A2 = (3.0 + 3.4641016151377546) / 12.0;

hub_status check_common(hub_basis h, hub_prec prec, int32_t nvec) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (prec != HUB_C128 && prec != HUB_C64) return fail(HUB_E_INVALID, "unknown precision");
  if (nvec < 1) return fail(HUB_E_INVALID, "nvec must be >= 1");
  if (h->device < 0) return fail(HUB_E_DEVICE, "host-only handle (created with device -1)");
  HUB_HIP(hipSetDevice(h->device));
  return HUB_OK;
}

// Timing events ride on the dispatches of plain applies (hub_apply_H) and of
// Lanczos-mode applies that do not also accumulate observables (every
// prof_period-th such apply): one start/end pair per kernel, so a sampled
// apply's time is its kernel time (row plus column pass for two passes).
hub_status launch_apply_timed(hub_basis h, const hub::ApplyLaunch& L, int* grid = nullptr, bool fusing = false,
                              int step = -1, int sub = 0) {
  // with fused iterations in the loop, only those (the dominant kernels) are timed
  bool timed = h->prof && (L.mode == hub::kPlain || (L.mode == hub::kLanczos && !L.obs && (!fusing || L.fuse)));
  if (timed) timed = (h->prof_count++ % h->prof_period) == 0;
  if (!timed) {
    HUB_HIP(hub::launch_apply(L, grid));
    return HUB_OK;
  }
  const bool two = hub::apply_two_pass(h->D, L.prec, L.nv, L.mode, L.obs) ||
                   (L.nv > 1 && hub::block_two_pass(h->D, L.prec, L.nv));
  std::array<hipEvent_t, 4> ev{nullptr, nullptr, nullptr, nullptr};
  for (int k = 0; k < (two ? 4 : 2); ++k) {
    if (!h->ev_free.empty()) {
      ev[k] = h->ev_free.back();
      h->ev_free.pop_back();
    } else {
      HUB_HIP(hipEventCreate(&ev[k]));
    }
  }
  hub::ApplyLaunch T = L;
  T.ev_start = ev[0];
  T.ev_stop = ev[1];
  T.ev2_start = ev[2];
  T.ev2_stop = ev[3];
  HUB_HIP(hub::launch_apply(T, grid));
  ProfSample smp;
  smp.ev = ev;
  smp.n = step;
  smp.sub = sub;
  smp.j = L.j;
  smp.fused = L.fuse;
  smp.worked = step < 0 ? 1 : -1;
  h->prof_samples.push_back(smp);
  // algorithmic bytes: H*v reads x, writes y; a fused iteration also reads
  // w_{j-1} and u_{j-1} and writes u_j instead of reading x
  h->prof_bytes = (L.fuse ? 4.0 : 2.0) * L.nv * static_cast<double>(h->D.dim) * (L.prec == 0 ? 16.0 : 8.0);
  return HUB_OK;
}

// Kernel times of the samples [from, end) (their events must have completed:
// call after synchronising the stream they were recorded on); the events go
// back to the pool.  Returns the end.
hub_status prof_harvest(hub_basis h, size_t from, size_t* end) {
  for (size_t i = from; i < h->prof_samples.size(); ++i) {
    ProfSample& p = h->prof_samples[i];
    for (int k = 0; k < 4; k += 2) {
      if (!p.ev[k]) continue;
      float ms = 0.0f;
      HUB_HIP(hipEventElapsedTime(&ms, p.ev[k], p.ev[k + 1]));
      p.ms += ms;
    }
    for (hipEvent_t& x : p.ev)
      if (x) {
        h->ev_free.push_back(x);
        x = nullptr;
      }
  }
  *end = h->prof_samples.size();
  return HUB_OK;
}

// Group sizes for nvec vectors: powers of two up to 8 whose staged row keeps
// at least three apply workgroups per CU (<= 48 KB of the 160 KB LDS), or one
// vector per group; single vectors where the two-pass kernels apply.
std::vector<int> groups_for(hub_basis h, int nvec, int prec, bool propagate = true) {
  const int prop = nvec > kMaxNV && h->prop_group_large[prec] > 0 ? h->prop_group_large[prec] : h->prop_group[prec];
  const int tuned = h->force_group > 0 ? h->force_group : (propagate ? prop : h->apply_group[prec]);
  if (tuned > 0) {
    std::vector<int> g;
    // a tuned size smaller where neither the block kernels nor the one-pass
    // kernel can take a group of that size
    for (int left = nvec; left > 0;) {
      int s = tuned;
      while (s > left || (s > 1 && !hub::block_two_pass(h->D, prec, s) && !hub::apply_fits(h->D, prec, s))) s /= 2;
      g.push_back(s);
      left -= s;
    }
    return g;
  }
  int gmax = kMaxNV;
  while (gmax > 1 && hub::apply_lds_bytes(h->D, prec, gmax, 1) > 48 * 1024) gmax /= 2;
  // single vectors run the two-pass kernels with fused updates, which beat
  // interleaved one-pass blocks whenever they apply
  if (hub::apply_two_pass(h->D, prec, 1, hub::kLanczos, false)) gmax = 1;
  // except complex64 propagations of several vectors: there blocks of 4 on
  // the two-pass block kernels beat single vectors on concurrent lanes (per
  // vector-step, 8 vectors: 12 sites 139.5 vs 165.5 us, 14 sites 2,204 vs
  // 2,382 us; complex128 singles stay ahead at 12 sites, 251 vs 259 us)
  if (propagate && prec == 1 && nvec > 1 && gmax == 1 && hub::block_two_pass(h->D, prec, 4)) gmax = 4;
  // plain applies of blocks on the two-pass block kernels: the largest group
  // whose staged row keeps two workgroups per CU (else one).  Propagations
  // keep the rules above unless a tuned plan says otherwise: at 12 sites
  // complex128 single vectors on the fused two-pass iterations, several groups
  // on concurrent lanes, were measured faster than blocks.
  if (nvec > 1 && !propagate) {
    int gb = 0;
    for (int g = kMaxNV; g >= 2 && !gb; g /= 2)
      if (hub::block_two_pass(h->D, prec, g) && hub::block_lds_bytes(h->D, prec, g) <= 80 * 1024) gb = g;
    for (int g = kMaxNV; g >= 2 && !gb; g /= 2)
      if (hub::block_two_pass(h->D, prec, g)) gb = g;
    if (gb) gmax = gb;
  }
  std::vector<int> g;
  int left = nvec;
  while (left > 0) {
    int s = gmax;
    while (s > left) s /= 2;
    g.push_back(s);
    left -= s;
  }
  return g;
}

struct StepReport {
  int m = 0, status = 0;
  double eps = 0.0, beta_last = 0.0;
};

// Work enqueued after every finished step of a propagation, on the group's
// stream right after the step's combine (so it sees the new state, and like
// every kernel of the step it must do nothing when ctl->abort is set: the
// step is then re-run and the hook enqueued again).
struct StepHook {
  char* traj = nullptr;  // single vectors: the state after step n also goes to traj + (n + 1) * traj_stride
  size_t traj_stride = 0;
  // k0, nv: the group's first vector in the call and its size; n_done: steps
  // finished; state: the group's vectors, interleaved [dim][nv] when nv > 1
  std::function<hipError_t(int k0, int nv, int n_done, const void* state, const StepCtl* ctl, hipStream_t s)> after;
};

// Runs n_steps Krylov midpoint steps for one group of nv vectors stored in
// the ABI layout at `user` (vector k at user + k*dim).  coef_mid[n][v][2*nc].
hub_status run_group(hub_basis h, hub_prec prec, int nv, void* user, int n_steps,
                     const std::vector<double>& coef_mid, double dt, const hub_krylov_opts& o,
                     bool want_obs, const std::vector<double>* coef_obs, std::vector<double>* obs_out,
                     std::vector<StepReport>* reports, hipStream_t stream, bool* not_converged,
                     int* steps_done, const CtrlInputs* ctrl, Work& W, const StepHook* hook = nullptr,
                     int k0 = 0) {
  const size_t es = elem_bytes(prec);
  const int64_t dim = h->D.dim;
  const size_t vbytes = static_cast<size_t>(dim) * nv * es;
  const int nc = static_cast<int>(h->B.classes.size());
  const int pi = prec == HUB_C128 ? 0 : 1;
  hub_status s = ensure_workspace(h, W, vbytes, o.m_max, nv > 1 ? vbytes : 0);
  if (s != HUB_OK) return s;
  // timed applies of this call: when the event pool runs low, their kernel
  // times are read at the next synchronisation (so the events are reused);
  // at the end the launches past a step's Krylov decision are marked as such
  const size_t prof_s0 = h->prof_samples.size();
  size_t prof_hv = prof_s0;
  auto harvest = [&]() -> hub_status {
    if (!h->prof || h->ev_free.size() >= kProfLowWater) return HUB_OK;
    return prof_harvest(h, prof_hv, &prof_hv);
  };

  void* slot0 = user;
  if (nv > 1) {
    slot0 = W.blockbuf;
    HUB_HIP(hub::launch_interleave(pi, nv, dim, user, slot0, true, stream));
  }
  std::vector<void*> ptrs(kMMax + 2, nullptr);
  ptrs[0] = slot0;
  for (int k = 1; k <= o.m_max; ++k) ptrs[k] = static_cast<char*>(W.slots) + (k - 1) * vbytes;
  // from the pinned mirror (free again: the previous run on this lane ended with a wait on its stream)
  std::copy(ptrs.begin(), ptrs.end(), W.h_ptrs);
  HUB_HIP(hipMemcpyAsync(W.slot_ptrs, W.h_ptrs, ptrs.size() * sizeof(void*), hipMemcpyHostToDevice, stream));

  // device logs
  const int nobs_rows = want_obs ? n_steps + 1 : 0;
  const size_t log_bytes = static_cast<size_t>(std::max(1, n_steps)) * solves_per_step(o) * nv * sizeof(CombineLog);
  const size_t obs_bytes = static_cast<size_t>(std::max(1, nobs_rows)) * nv * kObsQ * sizeof(double);
  if (log_bytes > W.dlog_bytes) {
    if (W.dlog) HUB_HIP(hipFree(W.dlog));
    W.dlog = nullptr;
    W.dlog_bytes = 0;
    HUB_HIP(hipMalloc(&W.dlog, log_bytes));
    W.dlog_bytes = log_bytes;
  }
  if (want_obs && obs_bytes > W.dobs_bytes) {
    if (W.dobs) HUB_HIP(hipFree(W.dobs));
    W.dobs = nullptr;
    W.dobs_bytes = 0;
    HUB_HIP(hipMalloc(reinterpret_cast<void**>(&W.dobs), obs_bytes));
    W.dobs_bytes = obs_bytes;
  }
  void* dlog = W.dlog;
  double* dobs = want_obs ? W.dobs : nullptr;

  StepCtl ctl0{};
  HUB_HIP(hipMemcpyAsync(W.ctl, &ctl0, sizeof(StepCtl), hipMemcpyHostToDevice, stream));
  HUB_HIP(hipStreamSynchronize(stream));

  // each of the scheme's exponentials exp(-i (dt/E) H_e) is split into
  // `substeps` equal factors: S Krylov solves of length tau per step
  const int E = scheme_exps(o);
  const double tau = dt / solves_per_step(o);
  const int rows = pi == 0 ? h->rows_c128 : h->rows_c64;
  hub::ApplyLaunch L{};
  L.db = &h->D;
  L.prec = pi;
  L.nv = nv;
  L.rows = rows;
  L.st = W.st;
  L.ctl = W.ctl;
  L.m_max = o.m_max;
  L.tol = o.tol;
  L.norm_inf = h->B.norm_inf;
  L.partials = W.partials;
  L.prev_partials = W.partials_e;
  L.prev_nblk = hub::elem_grid(dim * nv);
  L.stream = stream;

  const int S = solves_per_step(o);
  CombineLog* dlog_c = static_cast<CombineLog*>(dlog);
  // one Lanczos iteration j of substep `sub` of step n (apply, then update)
  auto enqueue_iter = [&](int n, int sub, int jj) -> hub_status {
    hub::ApplyLaunch A = L;
    A.mode = hub::kLanczos;
    A.obs = want_obs && sub == 0 && jj == 0;
    A.coef_obs = A.obs ? coef_obs->data() + static_cast<size_t>(n) * nv * 2 * nc : nullptr;
    A.x = ptrs[jj];
    A.y = jj < o.m_max ? ptrs[jj + 1] : nullptr;
    A.xprev = jj > 0 ? ptrs[jj - 1] : nullptr;
    A.coef = coef_mid.data() + (static_cast<size_t>(n) * E + sub / o.substeps) * nv * 2 * nc;
    A.j = jj;
    // a two-pass apply with observables leaves the row pass's partials after
    // the column pass's
    const bool blk = nv > 1 && hub::block_two_pass(h->D, pi, nv);
    const bool two_obs = A.obs && (blk || hub::apply_two_pass(h->D, pi, nv, hub::kLanczos, true));
    const size_t cg2 = blk ? 2 * static_cast<size_t>(h->D.dim_dn) * nv
                           : 2 * static_cast<size_t>(hub::colpass_grid(h->D, pi));
    if (two_obs) A.row_obs = W.partials + cg2;
    // From the second iteration on, the two-pass row pass (single vectors, or
    // blocks on the block kernels in small sectors) also finishes the previous
    // update (u_j = w_{j-1} - alpha s u_{j-1}) and the column pass takes the
    // decision, so no separate update kernel runs in between (at j = 1 the row
    // pass also finalizes the first apply's observables).  Fused blocks pay a
    // full column pass in a step's last iteration (the decision comes one
    // kernel later) and per-workgroup reductions over per-row and per-column
    // partials; they gain only where the saved update launch dominates.
    const bool blk_fuse = blk && dim <= kBlockFuseMaxDim;
    const bool fusable = !o.reorth && (blk_fuse || hub::apply_two_pass(h->D, pi, nv, hub::kLanczos, false));
    A.fuse = fusable && jj >= 1;
    if (A.fuse) {
      const bool after_obs = jj == 1 && want_obs && sub == 0 &&
                             (blk_fuse || hub::apply_two_pass(h->D, pi, nv, hub::kLanczos, true));
      A.alpha_partials = W.partials;
      A.alpha_nblk = blk ? h->D.dim_dn : hub::colpass_grid(h->D, pi);
      A.alpha_stride = after_obs ? hub::apply_nq_two_pass(true) : 1;
      A.obs_row = after_obs ? W.partials + cg2 : nullptr;
      // per-row |u_j|^2 [dim_up][nv] after the row pass's observables partials [dim_up][kObsQ][nv]
      A.norm_partials = W.partials + cg2 + static_cast<size_t>(h->D.dim_up) * kObsQ * (blk ? nv : 1);
    }
    int agrid = 0;  // workgroups that wrote the apply's partial sums
    hub_status r = launch_apply_timed(h, A, &agrid, fusable, n, sub);
    if (r != HUB_OK) return r;
    const bool next_fused = fusable;  // every later iteration finishes this update itself
    if (jj < o.m_max && !next_fused) {
      HUB_HIP(hub::launch_update(pi, nv, dim, ptrs[jj + 1], ptrs[jj], W.st, W.ctl, jj, W.partials, agrid,
                                 two_obs ? hub::apply_nq_two_pass(true) : hub::apply_nq(hub::kLanczos, A.obs, nc),
                                 two_obs ? A.row_obs : nullptr, h->D.dim_up, W.partials_e, stream));
      if (o.reorth)  // CGS2: two Gram-Schmidt passes against u_0..u_j
        for (int pass = 0; pass < 2; ++pass)
          HUB_HIP(hub::launch_reorth(pi, nv, dim, W.slot_ptrs, jj, W.st, W.ctl, W.partials, W.rcoef,
                                     W.partials_e, stream));
    }
    return HUB_OK;
  };
  // the combine also records the (sub)step: log, observables, cleared control block
  auto finish_sub = [&](int n, int sub) -> hub_status {
    const bool last = sub == S - 1;
    void* copy_to = (hook && hook->traj && nv == 1 && last) ? hook->traj + (n + 1) * hook->traj_stride : nullptr;
    HUB_HIP(hub::launch_combine(pi, nv, dim, W.slot_ptrs, W.st, W.ctl, W.partials_e, n * S + sub + 1,
                                dlog_c + (static_cast<size_t>(n) * S + sub) * nv,
                                (want_obs && sub == 0) ? dobs + static_cast<size_t>(n) * nv * kObsQ : nullptr,
                                kObsQ, stream, copy_to));
    if (hook && hook->after && last) HUB_HIP(hook->after(k0, nv, n + 1, slot0, W.ctl, stream));
    return HUB_OK;
  };

  // Adaptive schedule.  The decision for Krylov dimension m is taken by the
  // first workgroup of the m-th apply; iterations are enqueued speculatively
  // up to the previous step's m (a step that needs more waits for one host
  // round trip per extra iteration; kernels past the decision exit at once).
  int m_pred = o.m_hint > 0 ? std::min(o.m_hint, o.m_max) : std::min(8, o.m_max);
  bool first = true;  // the next step_begin computes |v| itself
  int64_t sync_launches = 0;  // Lanczos launches of the synchronous steps (counted for the first step)
  *not_converged = false;
  *steps_done = 0;
  auto adaptive_step = [&](int n, int sub0, bool* maxed) -> hub_status {
    int m_step_max = 0;
    *maxed = false;
    for (int sub = sub0; sub < S; ++sub) {
      // later substeps need no step_begin: tau is set, k_combine left the
      // |v|^2 partials and cleared the control block
      if (first) HUB_HIP(hub::launch_step_begin(pi, nv, dim, slot0, W.st, W.ctl, tau, true, W.partials_e, stream));
      first = false;
      int j = 0;
      for (; j <= m_pred && j <= o.m_max; ++j) {
        hub_status r = enqueue_iter(n, sub, j);
        if (r != HUB_OK) return r;
        ++sync_launches;
      }
      while (true) {
        HUB_HIP(hipMemcpyAsync(W.h_ctl, W.ctl, sizeof(StepCtl), hipMemcpyDeviceToHost, stream));
        HUB_HIP(hipStreamSynchronize(stream));
        if (W.h_ctl->all_done) break;
        if (j > o.m_max) return fail(HUB_E_DEVICE, "Krylov loop ended without a decision");
        hub_status r = enqueue_iter(n, sub, j);
        if (r != HUB_OK) return r;
        ++sync_launches;
        ++j;
      }
      m_step_max = std::max(m_step_max, static_cast<int>(W.h_ctl->iter));
      *maxed = W.h_ctl->any_maxed != 0;
      hub_status r = harvest();
      if (r != HUB_OK) return r;
      r = finish_sub(n, sub);
      if (r != HUB_OK) return r;
      if (*maxed) break;
    }
    // next step's speculative depth: the deepest this step needed
    m_pred = std::max(1, std::min(o.m_max, m_step_max));
    return HUB_OK;
  };

  // Chunked schedule: with the learned controller, or (default) with the
  // previous chunk's largest m as the prediction; results are the same as
  // the synchronous loop below either way.
  const bool learned = h->ctrl_on && ctrl != nullptr;
  const bool controlled = n_steps > 0 && (learned || (h->sched_chunk > 0 && n_steps >= 2));
  const int chunk = learned ? h->ctrl_chunk : h->sched_chunk;
  const int margin = learned ? h->ctrl_margin : h->sched_margin;
  if (!controlled) {
    for (int n = 0; n < n_steps; ++n) {
      bool maxed = false;
      hub_status r = adaptive_step(n, 0, &maxed);
      if (r != HUB_OK) return r;
      *steps_done = n + 1;
      if (maxed) {  // stop at the first step where a vector hit m_max
        *not_converged = true;
        break;
      }
    }
  } else {
    // Chunked schedule: plan `chunk` steps (one MLP launch, or the largest m
    // of the previous chunk), enqueue them without host synchronisation, then
    // check on the device counters how many finished; an undecided step is
    // re-run adaptively.
    std::vector<CombineLog> hlog(static_cast<size_t>(n_steps) * S * nv);
    std::vector<int> L_of(chunk);
    auto step_hist = [&](int n, int v, double* eps, int* m) {  // step n's log of vector v
      double e = 0.0;
      int mm = 0;
      for (int sub = 0; sub < S; ++sub) {
        const CombineLog& c = hlog[(static_cast<size_t>(n) * S + sub) * nv + v];
        e = std::max(e, c.eps);
        mm = std::max(mm, static_cast<int>(c.m));
      }
      *eps = e;
      *m = mm;
    };
    auto fetch_logs = [&](int n_from, int n_to) -> hub_status {  // enqueue only
      if (n_to <= n_from) return HUB_OK;
      const size_t off = static_cast<size_t>(n_from) * S * nv;
      const size_t cnt = static_cast<size_t>(n_to - n_from) * S * nv;
      HUB_HIP(hipMemcpyAsync(hlog.data() + off, dlog_c + off, cnt * sizeof(CombineLog), hipMemcpyDeviceToHost,
                             stream));
      return HUB_OK;
    };
    int n = 0;
    // Without a prediction to start from (default schedule, no m_hint) the
    // first step runs synchronously and its Krylov dimension seeds the first
    // chunk, instead of a fixed guess whose surplus launches every step of
    // that chunk would pay.
    if (!learned && o.m_hint == 0) {
      bool mx = false;
      sync_launches = 0;
      hub_status r = adaptive_step(0, 0, &mx);
      if (r != HUB_OK) return r;
      r = fetch_logs(0, 1);
      if (r != HUB_OK) return r;
      HUB_HIP(hipStreamSynchronize(stream));
      *steps_done = 1;
      n = 1;
      W.cstats.steps += 1;
      W.cstats.lanczos_launches += sync_launches;
      for (int v = 0; v < nv; ++v) {
        double e;
        int mm;
        step_hist(0, v, &e, &mm);
        W.cstats.iterations += mm;
      }
      if (mx) {
        *not_converged = true;
        n = n_steps;  // stop after this step, as the chunks would
      }
    }
    while (n < n_steps) {
      const int K = std::min(chunk, n_steps - n);
      // plan: features of every (step, vector) row, history up to step n-1
      float* hf = h->ctrl_hfeat;
      for (int k = 0; learned && k < K; ++k)
        for (int v = 0; v < nv; ++v) {
          double eh[4];
          for (int q = 0; q < 4; ++q) {
            const int hs = n - 1 - q;
            int mm = 0;
            if (hs >= 0) step_hist(hs, v, &eh[q], &mm);
            else eh[q] = NAN;
          }
          double e0 = 0.0;
          int m_last = -1;
          if (n >= 1) step_hist(n - 1, v, &e0, &m_last);
          const size_t r = static_cast<size_t>(n + k) * nv + v;
          ctrl_features((*ctrl).A_mid[r], (*ctrl).dA_mid[r], tau * h->B.norm_inf, eh, m_last, o.tol, o.m_hint,
                        hf + (static_cast<size_t>(k) * nv + v) * HUB_MLP_IN);
        }
      const int rows = K * nv;
      if (learned) {
        HUB_HIP(hipMemcpyAsync(h->ctrl_feat, hf, static_cast<size_t>(rows) * HUB_MLP_IN * sizeof(float),
                               hipMemcpyHostToDevice, stream));
        HUB_HIP(hub::launch_mlp_forward(h->ctrl_params, rows, h->ctrl_feat, h->ctrl_out, stream));
        HUB_HIP(hipMemcpyAsync(h->ctrl_hout, h->ctrl_out, static_cast<size_t>(rows) * HUB_MLP_OUT * sizeof(float),
                               hipMemcpyDeviceToHost, stream));
      }
      StepCtl c0 = *W.h_ctl;
      c0.abort = 0;
      c0.halt_from = 0;
      c0.steps_done = 0;
      c0.all_done = 0;
      c0.any_maxed = 0;
      c0.iter = 0;
      *W.h_ctl = c0;
      HUB_HIP(hipMemcpyAsync(W.ctl, W.h_ctl, sizeof(StepCtl), hipMemcpyHostToDevice, stream));
      if (learned) {
        HUB_HIP(hipStreamSynchronize(stream));  // the predictions
        for (int k = 0; k < K; ++k) {
          double lg = 0.0;
          for (int v = 0; v < nv; ++v) {
            const double ov = h->ctrl_hout[(static_cast<size_t>(k) * nv + v) * HUB_MLP_OUT];
            lg = std::max(lg, std::isfinite(ov) ? ov : 64.0);
          }
          const double mpred = std::ceil(std::exp2(std::min(lg, 10.0)) - 1e-6);
          L_of[k] = std::min(o.m_max, static_cast<int>(mpred) + margin) + 1;  // launches j = 0..L-1
        }
      } else {
        // the largest m of the previous chunk's steps (the first chunk: the hint)
        int m_ref = 0;
        for (int q = std::max(0, n - chunk); q < n; ++q)
          for (int v = 0; v < nv; ++v) {
            double e;
            int mm;
            step_hist(q, v, &e, &mm);
            m_ref = std::max(m_ref, mm);
          }
        if (m_ref == 0) m_ref = m_pred;
        for (int k = 0; k < K; ++k) L_of[k] = std::min(o.m_max, m_ref + margin) + 1;
      }
      // enqueue the chunk
      const size_t chunk_s = h->prof_samples.size();
      for (int k = 0; k < K; ++k)
        for (int sub = 0; sub < S; ++sub) {
          if (first)
            HUB_HIP(hub::launch_step_begin(pi, nv, dim, slot0, W.st, W.ctl, tau, true, W.partials_e, stream));
          first = false;
          for (int j = 0; j < L_of[k] && j <= o.m_max; ++j) {
            hub_status r = enqueue_iter(n + k, sub, j);
            if (r != HUB_OK) return r;
          }
          hub_status r = finish_sub(n + k, sub);
          if (r != HUB_OK) return r;
          W.cstats.lanczos_launches += std::min(L_of[k], o.m_max + 1);
        }
      HUB_HIP(hipMemcpyAsync(W.h_ctl, W.ctl, sizeof(StepCtl), hipMemcpyDeviceToHost, stream));
      { hub_status r = fetch_logs(n, n + K); if (r != HUB_OK) return r; }
      HUB_HIP(hipStreamSynchronize(stream));
      { hub_status r = harvest(); if (r != HUB_OK) return r; }
      W.cstats.chunks += 1;
      const int done_sub = W.h_ctl->steps_done;
      const int complete = std::min(K, done_sub / S);
      bool maxed = false;
      for (int k = 0; k < complete && !maxed; ++k)
        for (int v = 0; v < nv; ++v) {
          double e;
          int mm;
          step_hist(n + k, v, &e, &mm);
          for (int sub = 0; sub < S; ++sub)
            maxed |= hlog[(static_cast<size_t>(n + k) * S + sub) * nv + v].status >= 3;
          W.cstats.iterations += mm;
        }
      W.cstats.steps += complete;
      *steps_done = n + complete;
      if (maxed) {  // a vector hit m_max: the device stopped after that step
        int k = 0;
        for (; k < complete; ++k) {
          bool mk = false;
          for (int sub = 0; sub < S; ++sub)
            for (int v = 0; v < nv; ++v) mk |= hlog[(static_cast<size_t>(n + k) * S + sub) * nv + v].status >= 3;
          if (mk) break;
        }
        *steps_done = n + k + 1;
        *not_converged = true;
        break;
      }
      if (W.h_ctl->abort == 0) {
        n += K;
        continue;
      }
      // fallback: the first unfinished step, from its first unfinished substep
      const int nb = n + complete;
      for (size_t i = chunk_s; i < h->prof_samples.size(); ++i) {  // launched after the stop
        ProfSample& p = h->prof_samples[i];
        if (p.n > nb || (p.n == nb && p.sub > done_sub % S)) p.worked = 0;
      }
      StepCtl c1 = *W.h_ctl;
      c1.abort = 0;
      c1.halt_from = 0;
      c1.all_done = 0;
      c1.any_maxed = 0;
      c1.iter = 0;
      c1.steps_done = 0;
      *W.h_ctl = c1;
      HUB_HIP(hipMemcpyAsync(W.ctl, W.h_ctl, sizeof(StepCtl), hipMemcpyHostToDevice, stream));
      first = true;  // the abandoned step overwrote the |v|^2 partials
      int mp = 0;
      for (int v = 0; v < nv; ++v) {
        double e;
        int mm;
        if (nb >= 1) step_hist(nb - 1, v, &e, &mm);
        else mm = 0;
        mp = std::max(mp, mm);
      }
      if (mp > 0) m_pred = std::min(o.m_max, mp);
      bool mx = false;
      hub_status r = adaptive_step(nb, done_sub % S, &mx);
      if (r != HUB_OK) return r;
      r = fetch_logs(nb, nb + 1);
      if (r != HUB_OK) return r;
      HUB_HIP(hipStreamSynchronize(stream));
      W.cstats.fallbacks += 1;
      *steps_done = nb + 1;
      if (mx) {
        *not_converged = true;
        break;
      }
      n = nb + 1;
    }
  }
  // observables at the last sample time reached (after n_steps steps, or
  // after the step that stopped at m_max)
  bool split_obs = false;
  if (want_obs) {
    StepCtl c2 = StepCtl{};  // clear a stop flag left by the last step
    *W.h_ctl = c2;
    HUB_HIP(hipMemcpyAsync(W.ctl, W.h_ctl, sizeof(StepCtl), hipMemcpyHostToDevice, stream));
    hub::ApplyLaunch A = L;
    A.mode = hub::kObsOnly;
    A.obs = true;
    A.x = slot0;
    A.y = nullptr;
    A.coef = coef_obs->data() + static_cast<size_t>(*steps_done) * nv * 2 * nc;
    A.coef_obs = A.coef;
    A.j = 0;
    int ogrid = 0;
    if (nv > 1 && !hub::apply_fits(h->D, pi, nv)) {
      // the group's row does not fit the one-pass kernel (blocks on the
      // two-pass block kernels): back to the caller's layout first, then the
      // observables of one vector at a time
      HUB_HIP(hub::launch_interleave(pi, nv, dim, slot0, user, false, stream));
      split_obs = true;
      for (int v = 0; v < nv; ++v) {
        hub::ApplyLaunch A1 = A;
        A1.nv = 1;
        A1.x = static_cast<const char*>(user) + static_cast<size_t>(v) * dim * es;
        A1.coef = A.coef + static_cast<size_t>(v) * 2 * nc;
        A1.coef_obs = A1.coef;
        HUB_HIP(hub::launch_apply(A1, &ogrid));
        HUB_HIP(hub::launch_finalize_obs(1, W.partials, ogrid, hub::apply_nq(hub::kObsOnly, true, nc), W.st + v,
                                         stream));
      }
    } else {
      HUB_HIP(hub::launch_apply(A, &ogrid));
      HUB_HIP(hub::launch_finalize_obs(nv, W.partials, ogrid, hub::apply_nq(hub::kObsOnly, true, nc), W.st, stream));
    }
    HUB_HIP(hub::launch_step_log(nv, W.st, W.ctl, nullptr, dobs + static_cast<size_t>(*steps_done) * nv * kObsQ,
                                 kObsQ, stream));
  }
  if (nv > 1 && !split_obs) HUB_HIP(hub::launch_interleave(pi, nv, dim, slot0, user, false, stream));

  // copy logs back
  const int nd = *steps_done;
  const bool classify = h->prof_samples.size() > prof_s0;
  std::vector<CombineLog> lg;
  if ((reports || classify) && nd > 0) {
    lg.resize(static_cast<size_t>(nd) * S * nv);
    HUB_HIP(hipMemcpyAsync(lg.data(), dlog, lg.size() * sizeof(CombineLog), hipMemcpyDeviceToHost, stream));
    HUB_HIP(hipStreamSynchronize(stream));
  }
  if (classify) {
    // launch j of a (sub)step with Krylov dimension m did work iff j <= m
    // (j = m builds u_m, whose norm the decision needs) and j < m_max
    // (launch m_max only takes the decision); a fused iteration j = m is left
    // out too: its column pass skips the apply when the row pass already
    // found the estimate below tol
    for (size_t i = prof_s0; i < h->prof_samples.size(); ++i) {
      ProfSample& p = h->prof_samples[i];
      if (p.worked != -1) continue;
      if (p.n < 0 || p.n >= nd) {
        p.worked = 0;
        continue;
      }
      int m = 0;
      for (int v = 0; v < nv; ++v)
        m = std::max(m, static_cast<int>(lg[(static_cast<size_t>(p.n) * S + p.sub) * nv + v].m));
      p.worked = (p.fused ? p.j < m : p.j <= m) && p.j < o.m_max ? 1 : 0;
    }
  }
  if (reports && nd > 0) {
    reports->assign(static_cast<size_t>(nd) * nv, StepReport{});
    for (int n = 0; n < nd; ++n)
      for (int v = 0; v < nv; ++v) {
        StepReport& R = (*reports)[static_cast<size_t>(n) * nv + v];
        R.status = 1;
        for (int sub = 0; sub < S; ++sub) {
          const CombineLog& c = lg[(static_cast<size_t>(n) * S + sub) * nv + v];
          R.m = std::max(R.m, static_cast<int>(c.m));
          R.eps = std::max(R.eps, c.eps);
          R.beta_last = c.beta_last;
          if (c.status == 4) R.status = 4;
          else if (c.status == 3 && R.status != 4) R.status = 3;
          else if (c.status == 2 && R.status < 3) R.status = 2;
        }
      }
  }
  if (want_obs && obs_out) {
    obs_out->assign(static_cast<size_t>(n_steps + 1) * nv * kObsQ, 0.0);
    HUB_HIP(hipMemcpyAsync(obs_out->data(), dobs, obs_out->size() * sizeof(double), hipMemcpyDeviceToHost,
                           stream));
  }
  HUB_HIP(hipStreamSynchronize(stream));
  return HUB_OK;
}

// o = [<D>, docc, |x|^2, Re <x|K(t)|x>] of one vector at sample time t.
void fill_obs(const hub::Basis& B, const double* o /* kObsQ */, double t, hub_obs* out) {
  const double e = o[0] + o[3];
  out->t = t;
  out->norm = std::sqrt(std::max(0.0, o[2]));
  out->energy_per_site = e / B.lat.n_sites;
  out->docc_per_site = o[1] / B.lat.n_sites;
}

// Observables of nvec vectors with the given device buffers: st (one
// VecState), partials (apply_grid rows of kObsQ doubles), site_out (n_sites
// doubles) and site_partials (elem_grid rows of n_sites doubles).  Every
// buffer is fully written before it is read, so none needs clearing.  No
// allocation on either side.
hub_status observables_into(hub_basis h, const double* A, hub_prec prec, int32_t nvec, const void* v, hub_obs* out,
                            double* site_docc, hipStream_t st, VecState* vst, double* partials, double* site_out,
                            double* site_partials) {
  const int pi = prec == HUB_C128 ? 0 : 1;
  const size_t es = elem_bytes(prec);
  const int64_t dim = h->D.dim;
  const int nc = h->D.nc;
  for (int k = 0; k < nvec; ++k) {
    double cf[2 * kMaxNV * kMaxClasses] = {};
    coef_for(h->B, A[k], cf);
    hub::ApplyLaunch L{};
    L.db = &h->D;
    L.prec = pi;
    L.nv = 1;
    L.rows = pi == 0 ? h->rows_c128 : h->rows_c64;
    L.mode = hub::kObsOnly;
    L.obs = true;
    L.x = static_cast<const char*>(v) + static_cast<size_t>(k) * dim * es;
    L.coef = cf;
    L.coef_obs = cf;
    L.st = vst;
    L.ctl = nullptr;  // observables-only applies take no Krylov decision
    L.partials = partials;
    L.stream = st;
    int grid = 0;
    HUB_HIP(hub::launch_apply(L, &grid));
    HUB_HIP(hub::launch_finalize_obs(1, partials, grid, hub::apply_nq(hub::kObsOnly, true, nc), vst, st));
    double o[kObsQ];
    HUB_HIP(hipMemcpyAsync(o, reinterpret_cast<char*>(vst) + offsetof(VecState, obs), sizeof(o),
                           hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));
    fill_obs(h->B, o, 0.0, &out[k]);
    out[k].t = 0.0;
    if (site_docc) {
      HUB_HIP(hub::launch_site_docc(pi, h->D, L.x, site_out, site_partials, st));
      HUB_HIP(hipMemcpyAsync(site_docc + static_cast<size_t>(k) * h->D.n_sites, site_out,
                             h->D.n_sites * sizeof(double), hipMemcpyDeviceToHost, st));
      HUB_HIP(hipStreamSynchronize(st));
    }
  }
  return HUB_OK;
}

// Byte offsets of the no-allocation variant's buffers in the static scratch
// array (each 256-byte aligned).
struct NoAllocLayout {
  size_t st, site, partials, site_partials, total;
};

NoAllocLayout noalloc_layout(const DevBasis& D) {
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  NoAllocLayout L{};
  L.st = 0;
  L.site = up(sizeof(VecState));
  L.partials = L.site + up(hub::kMaxSites * sizeof(double));
  const size_t rows = static_cast<size_t>(std::max(hub::apply_grid(D, 0, 1), hub::apply_grid(D, 1, 1)));
  L.site_partials = L.partials + up(rows * kObsQ * sizeof(double));
  L.total = L.site_partials + up(static_cast<size_t>(hub::elem_grid(D.dim)) * hub::kMaxSites * sizeof(double));
  return L;
}

// Device address of each device's copy of `scratch`, looked up once per
// device when the first handle is created on it.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hub_status scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(HUB_E_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return HUB_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the current device's copy
  if (e != hipSuccess || !p)
    return fail(HUB_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  return HUB_OK;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

const char* hub_last_error(void) { return g_err.c_str(); }

hub_status hub_pulse_A(const hub_pulse* pulse, double t, double* A) {
  if (!pulse || !A) return fail(HUB_E_INVALID, "null argument");
  hub_status s = check_pulse(*pulse);
  if (s != HUB_OK) return s;
  *A = pulse_value(*pulse, t);
  return HUB_OK;
}

hub_status hub_basis_create(const hub_lattice* lat, int32_t n_up, int32_t n_dn, int32_t device,
                            hub_basis* out) {
  if (!out) return fail(HUB_E_INVALID, "null output handle");
  *out = nullptr;
  if (!lat) return fail(HUB_E_INVALID, "null lattice");
  if (lat->n_bonds < 0) return fail(HUB_E_INVALID, "negative bond count");
  if (lat->n_bonds > 0 && (!lat->bond_i || !lat->bond_j || !lat->bond_t || !lat->bond_dx))
    return fail(HUB_E_INVALID, "null bond array");
  if (lat->n_sites < 1 || lat->n_sites > hub::kMaxSites) return fail(HUB_E_INVALID, "n_sites must be in 1..16");
  hub::Lattice L;
  L.n_sites = lat->n_sites;
  L.U = lat->U;
  for (int k = 0; k < lat->n_bonds; ++k) {
    L.bi.push_back(lat->bond_i[k]);
    L.bj.push_back(lat->bond_j[k]);
    L.bt.push_back(lat->bond_t[k]);
    L.bdx.push_back(lat->bond_dx[k]);
  }
  if (lat->onsite) L.onsite.assign(lat->onsite, lat->onsite + lat->n_sites);
  if (device != -1) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(HUB_E_DEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(HUB_E_INVALID, "device index out of range");
  }

  hub_basis h = new (std::nothrow) hub_basis_s();
  if (!h) return fail(HUB_E_NOMEM, "host allocation failed");
  bool sector_err = false;
  const std::string msg = hub::build_basis(L, n_up, n_dn, h->B, sector_err);
  if (!msg.empty()) {
    delete h;
    return fail(sector_err ? HUB_E_SECTOR : HUB_E_INVALID, msg);
  }
  h->device = device;
  if (device == -1) {  // host-only handle: tables, no device state
    *out = h;
    g_err.clear();
    return HUB_OK;
  }
  auto cleanup = [&](hub_status s) {
    hub_basis_destroy(h);
    return s;
  };
  if (hipSetDevice(device) != hipSuccess) return cleanup(fail(HUB_E_DEVICE, "hipSetDevice failed"));
  DevBasis& D = h->D;
  const hub::Basis& B = h->B;
  D.dim_up = B.up.dim;
  D.dim_dn = B.dn.dim;
  D.dim = B.dim;
  D.nc = static_cast<int>(B.classes.size());
  D.n_sites = B.lat.n_sites;
  D.U = B.lat.U;
  hub_status s = HUB_OK;
  if ((s = upload(h, &D.up_bits, B.up.states)) != HUB_OK) return cleanup(s);
  if ((s = upload(h, &D.dn_bits, B.dn.states)) != HUB_OK) return cleanup(s);
  if ((s = upload(h, &D.eps_up, B.up.onsite)) != HUB_OK) return cleanup(s);
  if ((s = upload(h, &D.eps_dn, B.dn.onsite)) != HUB_OK) return cleanup(s);
  std::vector<int32_t> uptr(static_cast<size_t>(B.up.dim) + 1);
  for (int r = 0; r < B.up.dim; ++r) uptr[r] = B.up.cls_ptr[static_cast<size_t>(r) * (D.nc + 1)];
  uptr[B.up.dim] = static_cast<int32_t>(B.up.hops.size());
  if ((s = upload(h, &D.up_ptr, uptr)) != HUB_OK) return cleanup(s);
  std::vector<uint32_t> uh = B.up.hops;
  uh.resize(uh.size() + 8, 0u);  // batches of eight may read past the last hop
  if ((s = upload(h, &D.up_hops, uh)) != HUB_OK) return cleanup(s);
  if ((s = upload(h, &D.dn_tab, B.dn.tabc)) != HUB_OK) return cleanup(s);
  D.nslots = B.dn.nslots;
  D.maxs_pad = B.dn.maxs_pad;
  for (int k = 0; k < 64; ++k) D.slot_class[k] = B.dn.slot_class[k];
  if ((s = upload(h, &D.up_tab, B.up.tabc)) != HUB_OK) return cleanup(s);
  D.up_nslots = B.up.nslots;
  D.up_maxs_pad = B.up.maxs_pad;
  for (int k = 0; k < 64; ++k) D.up_slot_class[k] = B.up.slot_class[k];
  if ((s = upload(h, &D.dn_tabg, B.dn.tabg)) != HUB_OK) return cleanup(s);
  if ((s = upload(h, &D.up_tabg, B.up.tabg)) != HUB_OK) return cleanup(s);
  D.dn_gslots = B.dn.gslots;
  D.up_gslots = B.up.gslots;
  for (int k = 0; k < 8; ++k) {
    D.dn_gclass[k] = B.dn.grp_class[k];
    D.up_gclass[k] = B.up.grp_class[k];
  }

  if ((s = work_init(h->w, false)) != HUB_OK) return cleanup(s);
  if ((s = scratch_init(device)) != HUB_OK) return cleanup(s);
  h->rows_c128 = pick_rows(h, 0);
  h->rows_c64 = pick_rows(h, 1);
  *out = h;
  g_err.clear();
  return HUB_OK;
}

void hub_basis_destroy(hub_basis h) {
  if (!h) return;
  if (h->device < 0) {
    delete h;
    return;
  }
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  for (void* p : h->allocs) (void)hipFree(p);
  work_free(h->w);
  for (auto& l : h->lanes) work_free(*l);
  if (h->ctrl_params) (void)hipFree(h->ctrl_params);
  if (h->ctrl_feat) (void)hipFree(h->ctrl_feat);
  if (h->ctrl_out) (void)hipFree(h->ctrl_out);
  if (h->ctrl_hfeat) (void)hipHostFree(h->ctrl_hfeat);
  if (h->ctrl_hout) (void)hipHostFree(h->ctrl_hout);
  for (auto& p : h->prof_samples)
    for (hipEvent_t x : p.ev)
      if (x) (void)hipEventDestroy(x);
  for (hipEvent_t x : h->ev_free) (void)hipEventDestroy(x);
  delete h;
}

hub_status hub_basis_info(hub_basis h, int64_t* dim, int32_t* dim_up, int32_t* dim_dn) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (dim) *dim = h->B.dim;
  if (dim_up) *dim_up = h->B.up.dim;
  if (dim_dn) *dim_dn = h->B.dn.dim;
  return HUB_OK;
}

hub_status hub_basis_states(hub_basis h, uint32_t* up_bits, uint32_t* dn_bits) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (up_bits) std::memcpy(up_bits, h->B.up.states.data(), h->B.up.states.size() * sizeof(uint32_t));
  if (dn_bits) std::memcpy(dn_bits, h->B.dn.states.data(), h->B.dn.states.size() * sizeof(uint32_t));
  return HUB_OK;
}

hub_status hub_basis_classes(hub_basis h, double* t, double* d, int32_t* n_classes, double* norm_inf) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  const int nc = static_cast<int>(h->B.classes.size());
  for (int c = 0; c < nc; ++c) {
    if (t) t[c] = h->B.classes[c].t;
    if (d) d[c] = h->B.classes[c].d;
  }
  if (n_classes) *n_classes = nc;
  if (norm_inf) *norm_inf = h->B.norm_inf;
  return HUB_OK;
}

hub_status hub_basis_hops(hub_basis h, int32_t spin, int32_t* ptr, int32_t* src, int32_t* sgn, int32_t* cls,
                          int64_t* n_hops) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (spin != 0 && spin != 1) return fail(HUB_E_INVALID, "spin must be 0 or 1");
  const hub::SpinTable& T = spin == 0 ? h->B.up : h->B.dn;
  const int nc = static_cast<int>(h->B.classes.size());
  if (n_hops) *n_hops = static_cast<int64_t>(T.hops.size());
  if (ptr) {
    for (int r = 0; r < T.dim; ++r) ptr[r] = T.cls_ptr[static_cast<size_t>(r) * (nc + 1)];
    ptr[T.dim] = static_cast<int32_t>(T.hops.size());
  }
  for (int r = 0; r < T.dim; ++r)
    for (int c = 0; c < nc; ++c) {
      const int b = T.cls_ptr[static_cast<size_t>(r) * (nc + 1) + c];
      const int e = T.cls_ptr[static_cast<size_t>(r) * (nc + 1) + c + 1];
      for (int k = b; k < e; ++k) {
        if (src) src[k] = static_cast<int32_t>(T.hops[k] & 0xFFFFu);
        if (sgn) sgn[k] = (T.hops[k] >> 31) ? -1 : 1;
        if (cls) cls[k] = c;
      }
    }
  return HUB_OK;
}

hub_status hub_apply_H(hub_basis h, const double* A, hub_prec prec, int32_t nvec, const void* x, void* y,
                       void* stream) {
  hub_status s = check_common(h, prec, nvec);
  if (s != HUB_OK) return s;
  if (!A || !x || !y) return fail(HUB_E_INVALID, "null argument");
  if (x == y) return fail(HUB_E_INVALID, "x and y must be distinct buffers");
  for (int k = 0; k < nvec; ++k)
    if (!std::isfinite(A[k])) return fail(HUB_E_INVALID, "non-finite A");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int pi = prec == HUB_C128 ? 0 : 1;
  const size_t es = elem_bytes(prec);
  const int64_t dim = h->D.dim;
  const int nc = h->D.nc;
  const std::vector<int> groups = groups_for(h, nvec, pi, false);
  int gmax = 1;
  for (int g : groups) gmax = std::max(gmax, g);
  s = ensure_workspace(h, static_cast<size_t>(dim) * gmax * es, 1, gmax > 1 ? static_cast<size_t>(dim) * gmax * es : 0);
  if (s != HUB_OK) return s;
  int k0 = 0;
  for (int nv : groups) {
    std::vector<double> cf(static_cast<size_t>(2) * kMaxNV * kMaxClasses, 0.0);
    for (int v = 0; v < nv; ++v) coef_for(h->B, A[k0 + v], cf.data() + static_cast<size_t>(2) * v * nc);
    const char* xin = static_cast<const char*>(x) + static_cast<size_t>(k0) * dim * es;
    char* yout = static_cast<char*>(y) + static_cast<size_t>(k0) * dim * es;
    hub::ApplyLaunch L{};
    L.db = &h->D;
    L.prec = pi;
    L.nv = nv;
    L.rows = pi == 0 ? h->rows_c128 : h->rows_c64;
    L.mode = hub::kPlain;
    L.coef = cf.data();
    L.stream = st;
    if (nv == 1) {
      L.x = xin;
      L.y = yout;
      s = launch_apply_timed(h, L);
      if (s != HUB_OK) return s;
    } else {
      HUB_HIP(hub::launch_interleave(pi, nv, dim, xin, h->w.blockbuf, true, st));
      L.x = h->w.blockbuf;
      L.y = h->w.slots;
      s = launch_apply_timed(h, L);
      if (s != HUB_OK) return s;
      HUB_HIP(hub::launch_interleave(pi, nv, dim, h->w.slots, yout, false, st));
    }
    k0 += nv;
  }
  return HUB_OK;
}

hub_status hub_observables(hub_basis h, const double* A, hub_prec prec, int32_t nvec, const void* v,
                           hub_obs* out, double* site_docc, void* stream) {
  hub_status s = check_common(h, prec, nvec);
  if (s != HUB_OK) return s;
  if (!A || !v || !out) return fail(HUB_E_INVALID, "null argument");
  s = ensure_workspace(h, 16, 1, 0);
  if (s != HUB_OK) return s;
  return observables_into(h, A, prec, nvec, v, out, site_docc, static_cast<hipStream_t>(stream), h->w.st,
                          h->w.partials, h->w.scal, h->w.partials_e);
}

hub_status hub_observables_noalloc(hub_basis h, const double* A, hub_prec prec, int32_t nvec, const void* v,
                                   hub_obs* out, double* site_docc, void* stream) {
  hub_status s = check_common(h, prec, nvec);
  if (s != HUB_OK) return s;
  if (!A || !v || !out) return fail(HUB_E_INVALID, "null argument");
  char* base = static_cast<char*>(scratch_of(h->device));
  if (!base) return fail(HUB_E_DEVICE, "static scratch of this device not initialised");
  const NoAllocLayout Lo = noalloc_layout(h->D);
  if (Lo.total > kNoAllocScratchBytes)
    return fail(HUB_E_INVALID, "hub_observables_noalloc: the sector needs " + std::to_string(Lo.total) +
                                   " bytes of scratch, the static buffer holds " +
                                   std::to_string(kNoAllocScratchBytes));
  return observables_into(h, A, prec, nvec, v, out, site_docc, static_cast<hipStream_t>(stream),
                          reinterpret_cast<VecState*>(base + Lo.st), reinterpret_cast<double*>(base + Lo.partials),
                          reinterpret_cast<double*>(base + Lo.site),
                          reinterpret_cast<double*>(base + Lo.site_partials));
}

namespace {

// Automatic choice of the resident stepper: nvec vectors of dim states run
// there when nvec * kResidentAutoElems >= dim.  One workgroup per vector runs
// at a compute unit's rate, so a single large vector is better spread over
// the GPU one launch at a time (measured, steps/s resident vs launches, one
// vector: 6-site 400 states 2.3x, 8-site 4,900 states 1.13-1.16x (c128) and
// 1.27x (c64), 9-site 7,056 states 0.76x (c128; 1.11x with 4 vectors) and
// 0.95x (c64); batches of 64 vectors 3-9x).
constexpr int64_t kResidentAutoElems = 6144;

// The resident stepper takes the sector: one workgroup's threads own every
// state and the tile with the tables fits its LDS.
bool resident_fits(hub_basis h, int pi) {
  const DevBasis& D = h->D;
  if (D.dim < 1 || D.dim > static_cast<int64_t>(hub::kResidentThreads) * hub::kResidentEpt[pi]) return false;
  if (D.dn_gslots > 32 || D.up_gslots > 32) return false;
  if ((D.dn_gslots > 0 && !D.dn_tabg) || (D.up_gslots > 0 && !D.up_tabg)) return false;
  const size_t lds = hub::resident_lds_bytes(D.dim_up, D.dim_dn, D.up_gslots, D.dn_gslots,
                                             D.eps_up != nullptr || D.eps_dn != nullptr, pi);
  return lds <= static_cast<size_t>(hub::resident_lds_limit(pi));
}

// Options the resident stepper runs as the launch path does: either scheme,
// any substeps, the three-term recurrence, and none of the launch-path
// instruments (apply timing, the learned controller's plan, per-step hooks).
bool resident_options(hub_basis h, const hub_krylov_opts& o, bool controlled, bool hooked) {
  return o.reorth == 0 && !h->prof && !controlled && !hooked;
}

// hub_propagate on the resident stepper: coefficient tables of every vector
// and step, one launch, logs and observables back to the host in the layout
// run_all gives them.
hub_status run_resident(hub_basis h, hub_prec prec, int32_t nvec, void* v_inout, int n_steps,
                        const std::vector<std::vector<double>>& A_mid,
                        const std::vector<std::vector<double>>* A_sample,
                        const std::vector<std::vector<double>>* A_gauss, double t_start, double dt,
                        const hub_krylov_opts& o, hub_obs* obs, hub_step_info* log, hipStream_t st) {
  const int pi = prec == HUB_C128 ? 0 : 1;
  const size_t es = elem_bytes(prec);
  const DevBasis& D = h->D;
  const int nc = D.nc;
  const bool want_obs = obs != nullptr && A_sample != nullptr;
  Work& W = h->w;
  hub_status s = ensure_workspace(h, W, static_cast<size_t>(D.dim) * nvec * es, o.m_max, 0);
  if (s != HUB_OK) return s;
  // host tables: [nvec][n_steps][E][2 nc] for the step's exponentials (the
  // midpoint, or the fourth-order scheme's two Gauss-node combinations as the
  // launch path forms them), [nvec][n_steps + 1][2 nc] at the sample times
  const int E = scheme_exps(o);
  std::vector<double> cm(std::max<size_t>(1, static_cast<size_t>(nvec) * n_steps * E * 2 * nc), 0.0);
  std::vector<double> co(want_obs ? static_cast<size_t>(nvec) * (n_steps + 1) * 2 * nc : 0);
  for (int v = 0; v < nvec; ++v) {
    for (int n = 0; n < n_steps; ++n) {
      double* c = cm.data() + (static_cast<size_t>(v) * n_steps + n) * E * 2 * nc;
      if (E == 1) {
        coef_for(h->B, A_mid[v][n], c);
        continue;
      }
      double c1[2 * kMaxClasses], c2[2 * kMaxClasses];
      coef_for(h->B, (*A_gauss)[v][2 * n], c1);
      coef_for(h->B, (*A_gauss)[v][2 * n + 1], c2);
      for (int k = 0; k < 2 * nc; ++k) {
        c[k] = 2.0 * (kCf4A2 * c1[k] + kCf4A1 * c2[k]);           // applied first
        c[2 * nc + k] = 2.0 * (kCf4A1 * c1[k] + kCf4A2 * c2[k]);
      }
    }
    if (want_obs)
      for (int n = 0; n <= n_steps; ++n)
        coef_for(h->B, (*A_sample)[v][n], co.data() + (static_cast<size_t>(v) * (n_steps + 1) + n) * 2 * nc);
  }
  // device: [log | done | coef_mid | coef_obs] in the lane's log buffer, observables in its obs buffer
  auto a256 = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t log_b = a256(static_cast<size_t>(std::max(1, n_steps)) * nvec * sizeof(CombineLog));
  const size_t done_b = a256(static_cast<size_t>(nvec) * sizeof(int32_t));
  const size_t cm_b = a256(cm.size() * sizeof(double));
  const size_t co_b = a256(co.size() * sizeof(double));
  const size_t need = log_b + done_b + cm_b + co_b;
  if (need > W.dlog_bytes) {
    if (W.dlog) HUB_HIP(hipFree(W.dlog));
    W.dlog = nullptr;
    W.dlog_bytes = 0;
    HUB_HIP(hipMalloc(&W.dlog, need));
    W.dlog_bytes = need;
  }
  const size_t obs_bytes = static_cast<size_t>(n_steps + 1) * nvec * kObsQ * sizeof(double);
  if (want_obs && obs_bytes > W.dobs_bytes) {
    if (W.dobs) HUB_HIP(hipFree(W.dobs));
    W.dobs = nullptr;
    W.dobs_bytes = 0;
    HUB_HIP(hipMalloc(reinterpret_cast<void**>(&W.dobs), obs_bytes));
    W.dobs_bytes = obs_bytes;
  }
  char* base = static_cast<char*>(W.dlog);
  auto* dlog = reinterpret_cast<CombineLog*>(base);
  auto* ddone = reinterpret_cast<int32_t*>(base + log_b);
  auto* dcm = reinterpret_cast<double*>(base + log_b + done_b);
  auto* dco = want_obs ? reinterpret_cast<double*>(base + log_b + done_b + cm_b) : nullptr;
  HUB_HIP(hipMemcpyAsync(dcm, cm.data(), cm.size() * sizeof(double), hipMemcpyHostToDevice, st));
  if (want_obs) HUB_HIP(hipMemcpyAsync(dco, co.data(), co.size() * sizeof(double), hipMemcpyHostToDevice, st));

  hub::ResidentArgs A{};
  A.dim_up = D.dim_up;
  A.dim_dn = D.dim_dn;
  A.gs_up = D.up_gslots;
  A.gs_dn = D.dn_gslots;
  A.nc = nc;
  std::memcpy(A.up_gclass, D.up_gclass, sizeof(A.up_gclass));
  std::memcpy(A.dn_gclass, D.dn_gclass, sizeof(A.dn_gclass));
  A.up_bits = D.up_bits;
  A.dn_bits = D.dn_bits;
  A.eps_up = D.eps_up;
  A.eps_dn = D.eps_dn;
  A.up_tab = D.up_tabg;
  A.dn_tab = D.dn_tabg;
  A.U = D.U;
  A.norm_inf = h->B.norm_inf;
  A.tol = o.tol;
  A.tau = dt / solves_per_step(o);
  A.m_max = o.m_max;
  A.n_steps = n_steps;
  A.nvec = nvec;
  A.n_exp = E;
  A.substeps = o.substeps;
  A.coef_mid = dcm;
  A.coef_obs = dco;
  A.v = v_inout;
  A.slots = W.slots;
  A.log = dlog;
  A.obs = want_obs ? W.dobs : nullptr;
  A.done = ddone;
  const size_t lds = hub::resident_lds_bytes(D.dim_up, D.dim_dn, D.up_gslots, D.dn_gslots,
                                             D.eps_up != nullptr || D.eps_dn != nullptr, pi);
  const hipError_t e = hub::launch_resident(pi, A, lds, st);
  if (e != hipSuccess) return fail(HUB_E_DEVICE, std::string("resident stepper: ") + hipGetErrorString(e));
  std::vector<CombineLog> lg(static_cast<size_t>(n_steps) * nvec);
  std::vector<int32_t> done(nvec);
  std::vector<double> raw(want_obs ? static_cast<size_t>(n_steps + 1) * nvec * kObsQ : 0);
  if (!lg.empty()) HUB_HIP(hipMemcpyAsync(lg.data(), dlog, lg.size() * sizeof(CombineLog), hipMemcpyDeviceToHost, st));
  HUB_HIP(hipMemcpyAsync(done.data(), ddone, done.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  if (want_obs) HUB_HIP(hipMemcpyAsync(raw.data(), W.dobs, raw.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HUB_HIP(hipStreamSynchronize(st));

  bool any_nc = false;
  int nonfinite_step = -1;
  for (int v = 0; v < nvec; ++v) {
    const int nd = std::min(std::max(done[v], 0), n_steps);
    for (int n = 0; n < nd; ++n) {
      const CombineLog& c = lg[static_cast<size_t>(n) * nvec + v];
      if (c.status == 4 && (nonfinite_step < 0 || n < nonfinite_step)) nonfinite_step = n;
      any_nc |= c.status == 3;
      if (log) {
        hub_step_info& I = log[static_cast<size_t>(n) * nvec + v];
        I.m_used = c.m;
        I.substeps = o.substeps;
        I.converged = c.status < 3;
        I.breakdown = c.status == 2;
        I.err_est = c.eps;
        I.beta_last = c.beta_last;
      }
    }
    if (want_obs)
      for (int n = 0; n <= n_steps; ++n) {
        hub_obs& O = obs[static_cast<size_t>(n) * nvec + v];
        if (n > nd) {  // past the step that stopped this vector
          O = hub_obs{t_start + n * dt, NAN, NAN, NAN};
          continue;
        }
        fill_obs(h->B, raw.data() + (static_cast<size_t>(n) * nvec + v) * kObsQ, t_start + n * dt, &O);
      }
  }
  if (nonfinite_step >= 0)
    return fail(HUB_E_INVALID, "non-finite (NaN or Inf) vector in step " + std::to_string(nonfinite_step) +
                                   ": the propagation stopped there");
  if (any_nc) return fail(HUB_E_NOT_CONVERGED, "a Krylov step reached m_max before the tolerance");
  return HUB_OK;
}

}  // namespace

static hub_status run_all(hub_basis h, hub_prec prec, int32_t nvec, void* v_inout, int n_steps,
                          const std::vector<std::vector<double>>& A_mid /* [nvec][n_steps] */,
                          const std::vector<std::vector<double>>* A_sample /* [nvec][n_steps+1] */,
                          double t_start, double dt, const hub_krylov_opts& o, hub_obs* obs,
                          hub_step_info* log, void* stream,
                          const std::vector<std::vector<double>>* dA_mid = nullptr /* [nvec][n_steps] */,
                          const std::vector<std::vector<double>>* A_gauss = nullptr /* [nvec][2 n_steps] */,
                          const StepHook* hook = nullptr) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int pi = prec == HUB_C128 ? 0 : 1;
  const size_t es = elem_bytes(prec);
  const int64_t dim = h->D.dim;
  const int nc = h->D.nc;
  if (h->prop_path != 0) {
    const bool opts_ok = resident_options(h, o, h->ctrl_on && dA_mid, hook != nullptr);
    const bool fits = resident_fits(h, pi);
    if (h->prop_path == 1 && !(opts_ok && fits))
      return fail(HUB_E_INVALID, fits ? "the resident stepper takes reorth 0, and no apply timing, learned "
                                        "controller or step hook"
                                      : "the sector does not fit the resident stepper");
    // automatic: not where the caller chose the apply kernels (hub_set_apply_path),
    // and only for enough vectors per state
    const bool kernels_auto = h->D.two_pass == -1 && h->D.block_path == -1;
    const bool worth = static_cast<int64_t>(nvec) * kResidentAutoElems >= dim;
    if (opts_ok && fits && (h->prop_path == 1 || (kernels_auto && worth)))
      return run_resident(h, prec, nvec, v_inout, n_steps, A_mid, A_sample, A_gauss, t_start, dt, o, obs, log, st);
  }
  const std::vector<int> groups = groups_for(h, nvec, pi);
  const bool want_obs = obs != nullptr && A_sample != nullptr;
  const int E = scheme_exps(o);

  // host inputs of every group: hop coefficients of every exponential of
  // every step [n][e][v][2 nc], at the sample times [n][v][2 nc], controller rows
  struct GroupRun {
    int nv = 0, k0 = 0;
    std::vector<double> cm, co;
    CtrlInputs ci;
    std::vector<double> obs_raw;
    std::vector<StepReport> reps;
    bool ncv = false, ran = false;
    int done = 0;
    hub_status s = HUB_OK;
    std::string err;
  };
  std::vector<GroupRun> runs(groups.size());
  for (size_t g = 0, k0 = 0; g < groups.size(); k0 += groups[g], ++g) {
    GroupRun& R = runs[g];
    const int nv = groups[g];
    R.nv = nv;
    R.k0 = static_cast<int>(k0);
    R.cm.assign(static_cast<size_t>(n_steps) * E * nv * 2 * nc, 0.0);
    for (int n = 0; n < n_steps; ++n)
      for (int v = 0; v < nv; ++v) {
        if (E == 1) {
          coef_for(h->B, A_mid[k0 + v][n], R.cm.data() + (static_cast<size_t>(n) * nv + v) * 2 * nc);
          continue;
        }
        double c1[2 * kMaxClasses], c2[2 * kMaxClasses];
        coef_for(h->B, (*A_gauss)[k0 + v][2 * n], c1);
        coef_for(h->B, (*A_gauss)[k0 + v][2 * n + 1], c2);
        double* e0 = R.cm.data() + ((static_cast<size_t>(n) * E + 0) * nv + v) * 2 * nc;  // applied first
        double* e1 = R.cm.data() + ((static_cast<size_t>(n) * E + 1) * nv + v) * 2 * nc;
        for (int k = 0; k < 2 * nc; ++k) {
          e0[k] = 2.0 * (kCf4A2 * c1[k] + kCf4A1 * c2[k]);
          e1[k] = 2.0 * (kCf4A1 * c1[k] + kCf4A2 * c2[k]);
        }
      }
    if (want_obs) {
      R.co.assign(static_cast<size_t>(n_steps + 1) * nv * 2 * nc, 0.0);
      for (int n = 0; n <= n_steps; ++n)
        for (int v = 0; v < nv; ++v)
          coef_for(h->B, (*A_sample)[k0 + v][n], R.co.data() + (static_cast<size_t>(n) * nv + v) * 2 * nc);
    }
    if (dA_mid) {
      R.ci.A_mid.resize(static_cast<size_t>(n_steps) * nv);
      R.ci.dA_mid.resize(static_cast<size_t>(n_steps) * nv);
      for (int n = 0; n < n_steps; ++n)
        for (int v = 0; v < nv; ++v) {
          R.ci.A_mid[static_cast<size_t>(n) * nv + v] = A_mid[k0 + v][n];
          R.ci.dA_mid[static_cast<size_t>(n) * nv + v] = (*dA_mid)[k0 + v][n];
        }
    }
  }
  auto run_one = [&](GroupRun& R, Work& W, hipStream_t s_lane) {
    char* user = static_cast<char*>(v_inout) + static_cast<size_t>(R.k0) * dim * es;
    R.s = run_group(h, prec, R.nv, user, n_steps, R.cm, dt, o, want_obs, &R.co, &R.obs_raw, &R.reps, s_lane, &R.ncv,
                    &R.done, dA_mid ? &R.ci : nullptr, W, hook, R.k0);
    if (R.s != HUB_OK) R.err = g_err;
    R.ran = true;
  };

  // Lanes: groups run concurrently when there are several, unless the apply
  // timing (shared event pool) or the learned controller (shared MLP buffers)
  // is on, or the lanes' Krylov workspaces would exceed the budget.
  int nlanes = 1;
  if (groups.size() > 1 && !h->prof && !(h->ctrl_on && dA_mid)) {
    const int gmax = *std::max_element(groups.begin(), groups.end());
    const size_t per_lane = static_cast<size_t>(o.m_max + 2) * dim * gmax * es;  // slots and block buffer
    nlanes = static_cast<int>(std::min<size_t>(kMaxLanes, groups.size()));
    while (nlanes > 1 && per_lane * nlanes > kLaneWorkBudget) --nlanes;
  }
  if (nlanes == 1) {
    for (GroupRun& R : runs) {
      run_one(R, h->w, st);
      if (R.s != HUB_OK || R.ncv) break;  // stop at the first group that hit m_max
    }
  } else {
    while (static_cast<int>(h->lanes.size()) < nlanes - 1) {
      auto l = std::make_unique<Work>();
      hub_status s = work_init(*l, true);
      if (s != HUB_OK) {
        work_free(*l);
        return s;
      }
      h->lanes.push_back(std::move(l));
    }
    // the lanes start after the work already on the caller's stream
    hipEvent_t ready = nullptr;
    HUB_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    HUB_HIP(hipEventRecord(ready, st));
    for (int l = 1; l < nlanes; ++l) HUB_HIP(hipStreamWaitEvent(h->lanes[l - 1]->stream, ready, 0));
    std::vector<std::thread> threads;
    for (int l = 0; l < nlanes; ++l)
      threads.emplace_back([&, l]() {
        Work& W = l == 0 ? h->w : *h->lanes[l - 1];
        const hipStream_t s_lane = l == 0 ? st : W.stream;
        if (hipSetDevice(h->device) != hipSuccess) {
          for (size_t g = l; g < runs.size(); g += nlanes) {
            runs[g].s = HUB_E_DEVICE;
            runs[g].err = "hipSetDevice failed in a propagation lane";
          }
          return;
        }
        for (size_t g = l; g < runs.size(); g += nlanes) {
          try {
            run_one(runs[g], W, s_lane);
          } catch (const std::bad_alloc&) {
            runs[g].s = HUB_E_NOMEM;
            runs[g].err = "host allocation failed";
          }
          if (runs[g].s != HUB_OK) break;
        }
      });
    for (auto& t : threads) t.join();
    (void)hipEventDestroy(ready);
  }
  for (Work* W : [&] {
         std::vector<Work*> ws{&h->w};
         for (auto& l : h->lanes) ws.push_back(l.get());
         return ws;
       }()) {
    h->cstats.steps += W->cstats.steps;
    h->cstats.chunks += W->cstats.chunks;
    h->cstats.fallbacks += W->cstats.fallbacks;
    h->cstats.lanczos_launches += W->cstats.lanczos_launches;
    h->cstats.iterations += W->cstats.iterations;
    W->cstats = hub_controller_stats{};
  }
  for (const GroupRun& R : runs)
    if (R.ran && R.s != HUB_OK) return fail(R.s, R.err);

  bool any_nc = false;
  int nonfinite_step = -1;
  for (const GroupRun& R : runs) {
    if (!R.ran) continue;
    const int nv = R.nv, k0 = R.k0, done = R.done;
    for (int n = 0; n < done && nonfinite_step < 0; ++n)
      for (int v = 0; v < nv; ++v)
        if (R.reps[static_cast<size_t>(n) * nv + v].status == 4) nonfinite_step = n;
    if (log)
      for (int n = 0; n < done; ++n)
        for (int v = 0; v < nv; ++v) {
          const StepReport& P = R.reps[static_cast<size_t>(n) * nv + v];
          hub_step_info& I = log[static_cast<size_t>(n) * nvec + k0 + v];
          I.m_used = P.m;
          I.substeps = o.substeps;
          I.converged = P.status < 3;
          I.breakdown = P.status == 2;
          I.err_est = P.eps;
          I.beta_last = P.beta_last;
        }
    if (want_obs) {
      for (int n = 0; n <= n_steps; ++n)
        for (int v = 0; v < nv; ++v) {
          hub_obs& O = obs[static_cast<size_t>(n) * nvec + k0 + v];
          if (n > done) {  // past the step that stopped at m_max
            O = hub_obs{t_start + n * dt, NAN, NAN, NAN};
            continue;
          }
          fill_obs(h->B, R.obs_raw.data() + (static_cast<size_t>(n) * nv + v) * kObsQ, t_start + n * dt, &O);
        }
    }
    any_nc |= R.ncv;
  }
  if (nonfinite_step >= 0)
    return fail(HUB_E_INVALID, "non-finite (NaN or Inf) vector in step " + std::to_string(nonfinite_step) +
                                   ": the propagation stopped there");
  if (any_nc) return fail(HUB_E_NOT_CONVERGED, "a Krylov step reached m_max before the tolerance");
  return HUB_OK;
}

hub_status hub_krylov_expm_step(hub_basis h, const double* A_mid, double dt, const hub_krylov_opts* opts,
                                hub_prec prec, int32_t nvec, void* v_inout, hub_step_info* info, void* stream) {
  hub_status s = check_common(h, prec, nvec);
  if (s != HUB_OK) return s;
  if (!A_mid || !opts || !v_inout) return fail(HUB_E_INVALID, "null argument");
  if ((s = check_opts(*opts)) != HUB_OK) return s;
  if (opts->scheme != 0) return fail(HUB_E_INVALID, "a single exponential takes opts.scheme = 0");
  if (!std::isfinite(dt)) return fail(HUB_E_INVALID, "non-finite dt");
  std::vector<std::vector<double>> am(nvec, std::vector<double>(1));
  for (int k = 0; k < nvec; ++k) {
    if (!std::isfinite(A_mid[k])) return fail(HUB_E_INVALID, "non-finite A_mid");
    am[k][0] = A_mid[k];
  }
  return run_all(h, prec, nvec, v_inout, 1, am, nullptr, 0.0, dt, *opts, nullptr, info, stream);
}

hub_status hub_propagate(hub_basis h, const hub_pulse* pulses, double t_start, double dt, int32_t n_steps,
                         const hub_krylov_opts* opts, hub_prec prec, int32_t nvec, void* v_inout, hub_obs* obs,
                         hub_step_info* log, void* stream) {
  hub_status s = check_common(h, prec, nvec);
  if (s != HUB_OK) return s;
  if (!pulses || !opts || !v_inout) return fail(HUB_E_INVALID, "null argument");
  if (n_steps < 0) return fail(HUB_E_INVALID, "n_steps must be >= 0");
  if (!std::isfinite(dt) || !std::isfinite(t_start)) return fail(HUB_E_INVALID, "non-finite time");
  if ((s = check_opts(*opts)) != HUB_OK) return s;
  for (int k = 0; k < nvec; ++k)
    if ((s = check_pulse(pulses[k])) != HUB_OK) return s;
  std::vector<std::vector<double>> am(nvec, std::vector<double>(n_steps)), as(nvec, std::vector<double>(n_steps + 1));
  std::vector<std::vector<double>> dam(nvec, std::vector<double>(n_steps));
  std::vector<std::vector<double>> ag;
  if (opts->scheme == 1) ag.assign(nvec, std::vector<double>(2 * static_cast<size_t>(n_steps)));
  for (int k = 0; k < nvec; ++k) {
    for (int n = 0; n < n_steps; ++n) am[k][n] = pulse_value(pulses[k], t_start + n * dt + 0.5 * dt);
    for (int n = 0; n < n_steps; ++n) dam[k][n] = pulse_deriv(pulses[k], t_start + n * dt + 0.5 * dt);
    for (int n = 0; n <= n_steps; ++n) as[k][n] = pulse_value(pulses[k], t_start + n * dt);
    if (opts->scheme == 1)
      for (int n = 0; n < n_steps; ++n) {
        ag[k][2 * n] = pulse_value(pulses[k], t_start + (n + kCf4C1) * dt);
        ag[k][2 * n + 1] = pulse_value(pulses[k], t_start + (n + kCf4C2) * dt);
      }
  }
  return run_all(h, prec, nvec, v_inout, n_steps, am, &as, t_start, dt, *opts, obs, log, stream, &dam,
                 opts->scheme == 1 ? &ag : nullptr);
}

// ---------------------------------------------------------------------------
// Creation / annihilation operators between sectors and overlaps (Sec. 2.5,
// Sec. 3.7).  Spin-separated order: an up operator on site i passes the up
// creators of sites < i; a down operator also passes all n_up up creators.
namespace {

struct OpMap {
  std::vector<int32_t> map;
  std::vector<int8_t> sgn;
  bool down = false;
};

hub_status build_op_map(hub_basis from, hub_basis to, int site, int spin, int dagger, OpMap& M) {
  if (!from || !to) return fail(HUB_E_INVALID, "null basis handle");
  if (spin != 0 && spin != 1) return fail(HUB_E_INVALID, "spin must be 0 or 1");
  const int ns = from->B.lat.n_sites;
  if (site < 0 || site >= ns) return fail(HUB_E_INVALID, "site out of range");
  if (to->B.lat.n_sites != ns) return fail(HUB_E_SECTOR, "bases belong to lattices of different size");
  const int d = dagger ? 1 : -1;
  const int nu = from->B.n_up + (spin == 0 ? d : 0), nd = from->B.n_dn + (spin == 1 ? d : 0);
  if (to->B.n_up != nu || to->B.n_dn != nd) return fail(HUB_E_SECTOR, "target basis is not the operator's sector");
  const hub::SpinTable& Tt = spin == 0 ? to->B.up : to->B.dn;
  M.down = spin == 1;
  M.map.assign(Tt.dim, -1);
  M.sgn.assign(Tt.dim, 0);
  const uint32_t bit = 1u << site;
  for (int r = 0; r < Tt.dim; ++r) {
    const uint32_t t = Tt.states[r];
    uint32_t src;
    if (dagger) {
      if (!(t & bit)) continue;
      src = t ^ bit;
    } else {
      if (t & bit) continue;
      src = t | bit;
    }
    int sign = (__builtin_popcount(src & (bit - 1u)) & 1) ? -1 : 1;
    if (spin == 1 && (from->B.n_up & 1)) sign = -sign;
    M.map[r] = static_cast<int32_t>(hub::rank_of(src, ns));
    M.sgn[r] = static_cast<int8_t>(sign);
  }
  return HUB_OK;
}

struct DevOpMap {
  int32_t* map = nullptr;
  int8_t* sgn = nullptr;
  bool down = false;
  void release() {
    if (map) (void)hipFree(map);
    if (sgn) (void)hipFree(sgn);
    map = nullptr;
    sgn = nullptr;
  }
};

hub_status upload_op(hub_basis h, const OpMap& M, DevOpMap& D) {
  D.down = M.down;
  HUB_HIP(hipMalloc(reinterpret_cast<void**>(&D.map), M.map.size() * sizeof(int32_t)));
  HUB_HIP(hipMalloc(reinterpret_cast<void**>(&D.sgn), M.sgn.size()));
  HUB_HIP(hipMemcpy(D.map, M.map.data(), M.map.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HUB_HIP(hipMemcpy(D.sgn, M.sgn.data(), M.sgn.size(), hipMemcpyHostToDevice));
  (void)h;
  return HUB_OK;
}

}  // namespace

hub_status hub_apply_cop(hub_basis from, hub_basis to, int32_t site, int32_t spin, int32_t dagger, hub_prec prec,
                         int32_t nvec, const void* x, void* y, void* stream) {
  hub_status s = check_common(from, prec, nvec);
  if (s != HUB_OK) return s;
  if (!to || to->device != from->device) return fail(HUB_E_INVALID, "target basis on another device");
  if (!x || !y || x == y) return fail(HUB_E_INVALID, "x and y must be distinct device buffers");
  OpMap M;
  if ((s = build_op_map(from, to, site, spin, dagger, M)) != HUB_OK) return s;
  DevOpMap D;
  if ((s = upload_op(from, M, D)) != HUB_OK) {
    D.release();
    return s;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e = hub::launch_cop(prec == HUB_C128 ? 0 : 1, to->D.dim, to->D.dim_dn, from->D.dim_dn,
                                       from->D.dim, nvec, D.down, D.map, D.sgn, x, y, st);
  const hipError_t e2 = hipStreamSynchronize(st);
  D.release();
  if (e != hipSuccess || e2 != hipSuccess) return fail(HUB_E_DEVICE, "operator kernel failed");
  return HUB_OK;
}

hub_status hub_dot(hub_basis h, hub_prec prec, int32_t nvec, const void* x, const void* y, double* out,
                   void* stream) {
  hub_status s = check_common(h, prec, nvec);
  if (s != HUB_OK) return s;
  if (!x || !y || !out) return fail(HUB_E_INVALID, "null argument");
  s = ensure_workspace(h, 16, 1, 0);
  if (s != HUB_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* dout = nullptr;
  HUB_HIP(hipMalloc(reinterpret_cast<void**>(&dout), 2 * nvec * sizeof(double)));
  hipError_t e = hub::launch_dots(prec == HUB_C128 ? 0 : 1, h->D.dim, nvec, x, y, dout, h->w.partials_e, st);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 2 * nvec * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dout);
  if (e != hipSuccess) return fail(HUB_E_DEVICE, std::string("dot: ") + hipGetErrorString(e));
  return HUB_OK;
}

namespace {

// LDS staging of the persistent member stepper; the largest target sector and
// the fewest members (per compute unit) for which it is the automatic choice:
// one workgroup per member runs well below a compute unit's share of the
// bandwidth, so it pays only once every unit has a member (10-site sectors:
// 64 members 0.6x, 256 members 1.45x the per-sector batches), and larger
// sectors fill the GPU one apply at a time.
constexpr size_t kMembersLds = 148 << 10;  // tables + staging per member workgroup
constexpr int64_t kMembersAutoDim = 1 << 18;
constexpr int kMembersAutoPerCU = 1;

// Members of one target sector in hub_greens_diag.
struct GreensSector {
  hub_basis T = nullptr;
  std::vector<int> mem;  // member indices, ordered by start step
  void* buf = nullptr;
  int32_t* maps = nullptr;  // [member][map_len]
  int8_t* sgns = nullptr;
  int map_len = 0, ogrid = 0;
  bool down = false;
  double* part = nullptr;
  double* tot = nullptr;
  hipStream_t stream = nullptr;
  hub_status s = HUB_OK;
  std::string err;
};

// Steps 2-4 of hub_greens_diag on the persistent member stepper: every
// member's Krylov slots and row-pass buffer, c_k psi(t'_k) into its slot 0,
// one launch for all members and steps, overlaps straight into the ABI
// layout [member][n_rel + 1][2].
hub_status greens_members(hub_basis h, const std::vector<GreensSector>& secs, const hub_greens_member* members,
                          int n_members, const void* traj, int n_total, int n_rel, double t_start, double dt,
                          const hub_pulse& pulse, const hub_krylov_opts& o, hub_prec prec, double* overlaps,
                          hipStream_t st) {
  const int pi = prec == HUB_C128 ? 0 : 1;
  const size_t es = elem_bytes(prec);
  const int m_max = o.m_max;
  std::vector<void*> bufs;
  auto done = [&](hub_status r) {
    for (void* p : bufs) (void)hipFree(p);
    return r;
  };
  // a failed HIP call frees the buffers before it returns
#define MEMBERS_HIP(call)                                                                                  \
  do {                                                                                                     \
    const hipError_t e_ = (call);                                                                          \
    if (e_ != hipSuccess)                                                                                  \
      return done(fail(e_ == hipErrorOutOfMemory ? HUB_E_NOMEM : HUB_E_DEVICE,                             \
                       std::string(#call) + ": " + hipGetErrorString(e_)));                                \
  } while (0)
  auto alloc = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes == 0 ? 16 : bytes) != hipSuccess) return nullptr;
    bufs.push_back(p);
    return p;
  };
  std::vector<hub::MemberSector> hs(secs.size());
  std::vector<hub::MemberDesc> hd(n_members);
  std::vector<std::vector<double>> ctabs;
  ctabs.reserve(secs.size());
  size_t lds = 0;
  double* out = static_cast<double*>(alloc(static_cast<size_t>(n_members) * (n_rel + 1) * 2 * sizeof(double)));
  int32_t* stat = static_cast<int32_t*>(alloc(static_cast<size_t>(n_members) * std::max(n_rel, 1) * 2 * sizeof(int32_t)));
  if (!out || !stat) return done(fail(HUB_E_NOMEM, "member outputs"));
  for (size_t g = 0; g < secs.size(); ++g) {
    const GreensSector& S = secs[g];
    const DevBasis& TD = S.T->D;
    hub::MemberSector& M = hs[g];
    M.dim_up = TD.dim_up;
    M.dim_dn = TD.dim_dn;
    M.gs_up = TD.up_gslots;
    M.gs_dn = TD.dn_gslots;
    M.up_bits = TD.up_bits;
    M.dn_bits = TD.dn_bits;
    M.eps_up = TD.eps_up;
    M.eps_dn = TD.eps_dn;
    M.up_tab = TD.up_tabg;
    M.dn_tab = TD.dn_tabg;
    std::memcpy(M.up_gclass, TD.up_gclass, sizeof(M.up_gclass));
    std::memcpy(M.dn_gclass, TD.dn_gclass, sizeof(M.dn_gclass));
    M.U = TD.U;
    M.norm_inf = S.T->B.norm_inf;
    M.nc = TD.nc;
    const size_t tab = hub::members_table_lds(TD.dim_up, TD.dim_dn, TD.up_gslots, TD.dn_gslots,
                                              TD.eps_up != nullptr || TD.eps_dn != nullptr, S.map_len);
    const size_t stage = kMembersLds - tab;  // the caller checked that a tile row and column fit
    M.tab_lds = static_cast<int>(tab);
    M.row_block = static_cast<int>(std::min<size_t>(TD.dim_up, stage / ((TD.dim_dn + 1) * es)));
    M.col_block = static_cast<int>(std::min<size_t>(TD.dim_dn, stage / ((TD.dim_up + 1) * es)));
    lds = std::max({lds, tab + static_cast<size_t>(M.row_block) * (TD.dim_dn + 1) * es,
                    tab + static_cast<size_t>(M.col_block) * (TD.dim_up + 1) * es});
    ctabs.emplace_back(static_cast<size_t>(std::max(n_total, 1)) * 2 * TD.nc, 0.0);  // alive until the sync
    std::vector<double>& ct = ctabs.back();
    for (int n = 0; n < n_total; ++n)
      coef_for(S.T->B, pulse_value(pulse, t_start + n * dt + 0.5 * dt), ct.data() + static_cast<size_t>(n) * 2 * TD.nc);
    double* dct = static_cast<double*>(alloc(ct.size() * sizeof(double)));
    if (!dct) return done(fail(HUB_E_NOMEM, "coefficient table"));
    MEMBERS_HIP(hipMemcpyAsync(dct, ct.data(), ct.size() * sizeof(double), hipMemcpyHostToDevice, st));
    M.coef_tab = dct;
    // Krylov slots (m_max + 1 vectors) and the row-pass buffer of each member
    const size_t vb = static_cast<size_t>(TD.dim) * es;
    const int nm = static_cast<int>(S.mem.size());
    char* mb = static_cast<char*>(alloc(static_cast<size_t>(nm) * (m_max + 2) * vb));
    if (!mb) return done(fail(HUB_E_NOMEM, "member Krylov slots"));
    for (int q = 0; q < nm; ++q) {
      const int k = S.mem[q];
      hub::MemberDesc& D = hd[k];
      D.sector = static_cast<int>(g);
      D.start = members[k].start_step;
      D.slots = mb + static_cast<size_t>(q) * (m_max + 2) * vb;
      D.z = static_cast<char*>(D.slots) + static_cast<size_t>(m_max + 1) * vb;
      D.map = S.maps + static_cast<size_t>(q) * S.map_len;
      D.sgn = S.sgns + static_cast<size_t>(q) * S.map_len;
      D.down = S.down ? 1 : 0;
      D.out = out + static_cast<size_t>(k) * (n_rel + 1) * 2;
      D.status = stat + static_cast<size_t>(k) * std::max(n_rel, 1) * 2;
      D.m_used = D.status + std::max(n_rel, 1);
      MEMBERS_HIP(hub::launch_cop(pi, TD.dim, TD.dim_dn, h->D.dim_dn, h->D.dim, 1, S.down, D.map, D.sgn,
                              static_cast<const char*>(traj) + static_cast<size_t>(D.start) * h->D.dim * es, D.slots,
                              st));
    }
  }
  auto* dsec = static_cast<hub::MemberSector*>(alloc(hs.size() * sizeof(hub::MemberSector)));
  auto* dmem = static_cast<hub::MemberDesc*>(alloc(hd.size() * sizeof(hub::MemberDesc)));
  if (!dsec || !dmem) return done(fail(HUB_E_NOMEM, "member descriptors"));
  MEMBERS_HIP(hipMemcpyAsync(dsec, hs.data(), hs.size() * sizeof(hub::MemberSector), hipMemcpyHostToDevice, st));
  MEMBERS_HIP(hipMemcpyAsync(dmem, hd.data(), hd.size() * sizeof(hub::MemberDesc), hipMemcpyHostToDevice, st));
  hub::MembersArgs A{};
  A.sectors = dsec;
  A.members = dmem;
  A.n_rel = n_rel;
  A.m_max = m_max;
  A.tol = o.tol;
  A.tau = dt;
  A.traj = traj;
  A.traj_stride = h->D.dim;
  A.dim_dn_s = h->D.dim_dn;
  const hipError_t e = hub::launch_members(pi, n_members, A, lds, st);
  if (e != hipSuccess) return done(fail(HUB_E_DEVICE, std::string("member stepper: ") + hipGetErrorString(e)));
  std::vector<int32_t> hstat(static_cast<size_t>(n_members) * std::max(n_rel, 1) * 2);
  MEMBERS_HIP(hipMemcpyAsync(overlaps, out, static_cast<size_t>(n_members) * (n_rel + 1) * 2 * sizeof(double),
                         hipMemcpyDeviceToHost, st));
  MEMBERS_HIP(hipMemcpyAsync(hstat.data(), stat, hstat.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  MEMBERS_HIP(hipStreamSynchronize(st));
  bool maxed = false, nonfinite = false;
  for (int k = 0; k < n_members; ++k)
    for (int r = 0; r < n_rel; ++r) {
      const int32_t sk = hstat[static_cast<size_t>(k) * std::max(n_rel, 1) * 2 + r];
      maxed |= sk == 3;
      nonfinite |= sk == 4;
    }
  if (nonfinite) return done(fail(HUB_E_INVALID, "a member's vector became non-finite (NaN or Inf)"));
  if (maxed) return done(fail(HUB_E_NOT_CONVERGED, "a member's Krylov step reached m_max before the tolerance"));
  return done(HUB_OK);
#undef MEMBERS_HIP
}

}  // namespace

hub_status hub_greens_diag(hub_basis h, int32_t n_targets, const hub_basis* targets, const hub_pulse* pulse,
                           double t_start, double dt, int32_t n_rel, const hub_krylov_opts* opts, hub_prec prec,
                           int32_t n_members, const hub_greens_member* members, void* psi_inout, double* overlaps,
                           void* stream) {
  hub_status s = check_common(h, prec, 1);
  if (s != HUB_OK) return s;
  if (!targets || !pulse || !opts || !members || !psi_inout || !overlaps || n_targets < 1 || n_members < 1 ||
      n_rel < 0)
    return fail(HUB_E_INVALID, "null or empty argument");
  if ((s = check_opts(*opts)) != HUB_OK) return s;
  if (opts->scheme != 0) return fail(HUB_E_INVALID, "Green's functions use the midpoint scheme (opts.scheme = 0)");
  if ((s = check_pulse(*pulse)) != HUB_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int pi = prec == HUB_C128 ? 0 : 1;
  const size_t es = elem_bytes(prec);
  // target basis of every member, members grouped by target and sorted by start
  std::vector<int> tb(n_members, -1);
  int max_start = 0;
  for (int k = 0; k < n_members; ++k) {
    const hub_greens_member& m = members[k];
    if (m.start_step < 0) return fail(HUB_E_INVALID, "negative start step");
    max_start = std::max(max_start, static_cast<int>(m.start_step));
    const int d = m.dagger ? 1 : -1;
    const int nu = h->B.n_up + (m.spin == 0 ? d : 0), nd = h->B.n_dn + (m.spin == 1 ? d : 0);
    for (int g = 0; g < n_targets; ++g)
      if (targets[g] && targets[g]->B.n_up == nu && targets[g]->B.n_dn == nd && targets[g]->device == h->device) {
        tb[k] = g;
        break;
      }
    if (tb[k] < 0) return fail(HUB_E_SECTOR, "no target basis for a member's sector");
  }
  std::vector<std::vector<int>> grp(n_targets);
  for (int k = 0; k < n_members; ++k) grp[tb[k]].push_back(k);
  for (auto& v : grp)
    std::stable_sort(v.begin(), v.end(), [&](int a, int b) { return members[a].start_step < members[b].start_step; });
  const int n_total = max_start + n_rel;
  const int64_t dim_s = h->D.dim;
  // The persistent member stepper (one launch, a workgroup per member) needs
  // the three-term recurrence with one solve per step and the grouped hop
  // tables of every target sector, with a tile row and a tile column in LDS.
  bool members_fit = opts->reorth == 0 && opts->substeps == 1;
  bool members_small = true;
  for (int k = 0; k < n_members && members_fit; ++k) {
    const hub::Basis& TB = targets[tb[k]]->B;
    const DevBasis& TD = targets[tb[k]]->D;
    const int map_len = members[k].spin == 0 ? TD.dim_up : TD.dim_dn;
    const size_t tab = hub::members_table_lds(TD.dim_up, TD.dim_dn, TD.up_gslots, TD.dn_gslots,
                                              TD.eps_up != nullptr || TD.eps_dn != nullptr, map_len);
    members_fit = (TD.dn_gslots > 0 || TB.dn.max_hops == 0) && (TD.up_gslots > 0 || TB.up.max_hops == 0) &&
                  tab + (TD.dim_dn + 1) * es <= kMembersLds && tab + (TD.dim_up + 1) * es <= kMembersLds;
    members_small &= TD.dim <= kMembersAutoDim;
  }
  if (h->greens_path == 1 && !members_fit)
    return fail(HUB_E_INVALID, "the persistent member stepper needs reorth 0, substeps 1 and grouped hop tables");
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || n_cu < 1)
    n_cu = 256;
  const bool members_many = n_members >= kMembersAutoPerCU * n_cu;
  const bool use_members =
      h->greens_path == 1 || (h->greens_path == -1 && members_fit && members_small && members_many);
  // Device buffers: psi at every step (the trajectory), the members of every
  // target sector in the ABI layout (ordered by start step), their operator
  // maps packed per sector [member][map_len], overlap partials per sector
  // [n_rel + 1][members][grid][2] and their totals [n_rel + 1][members][2].
  using Sector = GreensSector;
  std::vector<Sector> secs;
  void* traj = nullptr;
  auto cleanup = [&](hub_status r) {
    for (Sector& S : secs) {
      if (S.buf) (void)hipFree(S.buf);
      if (S.maps) (void)hipFree(S.maps);
      if (S.sgns) (void)hipFree(S.sgns);
      if (S.part) (void)hipFree(S.part);
      if (S.tot) (void)hipFree(S.tot);
      if (S.stream) (void)hipStreamDestroy(S.stream);
    }
    if (traj) (void)hipFree(traj);
    return r;
  };
  for (int g = 0; g < n_targets; ++g) {
    if (grp[g].empty()) continue;
    Sector S;
    S.T = targets[g];
    S.mem = grp[g];
    secs.push_back(S);
  }
  const size_t sbytes = static_cast<size_t>(dim_s) * es;
  if (hipMalloc(&traj, static_cast<size_t>(n_total + 1) * sbytes) != hipSuccess)
    return cleanup(fail(HUB_E_NOMEM, "trajectory buffer"));
  for (Sector& S : secs) {
    const int nm = static_cast<int>(S.mem.size());
    const int64_t dt_ = S.T->D.dim;
    S.ogrid = hub::overlap_grid(dt_);
    std::vector<int32_t> maps;
    std::vector<int8_t> sg;
    for (int q = 0; q < nm; ++q) {
      const hub_greens_member& m = members[S.mem[q]];
      OpMap M;
      if ((s = build_op_map(h, S.T, m.site, m.spin, m.dagger, M)) != HUB_OK) return cleanup(s);
      if (q == 0) {
        S.map_len = static_cast<int>(M.map.size());
        S.down = M.down;
      } else if (static_cast<int>(M.map.size()) != S.map_len || M.down != S.down) {
        return cleanup(fail(HUB_E_INVALID, "members of one sector need operators of one spin"));
      }
      maps.insert(maps.end(), M.map.begin(), M.map.end());
      sg.insert(sg.end(), M.sgn.begin(), M.sgn.end());
    }
    if ((!use_members && hipMalloc(&S.buf, static_cast<size_t>(nm) * dt_ * es) != hipSuccess) ||
        hipMalloc(reinterpret_cast<void**>(&S.maps), maps.size() * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&S.sgns), sg.size()) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&S.part),
                  static_cast<size_t>(n_rel + 1) * nm * S.ogrid * 2 * sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&S.tot), static_cast<size_t>(n_rel + 1) * nm * 2 * sizeof(double)) !=
            hipSuccess)
      return cleanup(fail(HUB_E_NOMEM, "member buffers"));
    HUB_HIP(hipMemcpy(S.maps, maps.data(), maps.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HUB_HIP(hipMemcpy(S.sgns, sg.data(), sg.size(), hipMemcpyHostToDevice));
    if (hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking) != hipSuccess)
      return cleanup(fail(HUB_E_DEVICE, "stream creation failed"));
  }
  hub_krylov_opts o1 = *opts;
  // 1. psi over the whole grid, its state after every step kept in traj
  HUB_HIP(hipMemcpyAsync(traj, psi_inout, sbytes, hipMemcpyDeviceToDevice, st));
  if (n_total > 0) {
    std::vector<std::vector<double>> am(1, std::vector<double>(n_total));
    for (int n = 0; n < n_total; ++n) am[0][n] = pulse_value(*pulse, t_start + n * dt + 0.5 * dt);
    StepHook hk;
    hk.traj = static_cast<char*>(traj);
    hk.traj_stride = sbytes;
    if ((s = run_all(h, prec, 1, psi_inout, n_total, am, nullptr, t_start, dt, o1, nullptr, nullptr, st, nullptr,
                     nullptr, &hk)) != HUB_OK)
      return cleanup(s);
  }
  if (use_members) {
    s = greens_members(h, secs, members, n_members, traj, n_total, n_rel, t_start, dt, *pulse, o1, prec, overlaps,
                       st);
    return cleanup(s);
  }
  // 2. every member from c_k psi(t'_k); overlaps after s = 0..n_rel steps,
  // gathered from the trajectory, partials at [s][member][grid][2]
  auto overlap_launch = [&](Sector& S, int k0, int nv, int n_done, const void* phi, bool interleaved,
                            const StepCtl* ctl, hipStream_t s_) -> hipError_t {
    const int nm = static_cast<int>(S.mem.size());
    hub::OverlapArgs a{};
    a.n_t = S.T->D.dim;
    a.dim_dn_t = S.T->D.dim_dn;
    a.dim_dn_s = h->D.dim_dn;
    a.down = S.down ? 1 : 0;
    a.map_len = S.map_len;
    a.interleaved = interleaved ? 1 : 0;
    for (int v = 0; v < nv; ++v) a.psi_off[v] = (members[S.mem[k0 + v]].start_step + n_done) * dim_s;
    a.maps = S.maps + static_cast<size_t>(k0) * S.map_len;
    a.sgns = S.sgns + static_cast<size_t>(k0) * S.map_len;
    a.traj = traj;
    a.phi = phi;
    a.ctl = ctl;
    a.partials = S.part + (static_cast<size_t>(n_done) * nm + k0) * S.ogrid * 2;
    return hub::launch_overlaps(pi, nv, a, s_);
  };
  for (Sector& S : secs) {
    const int nm = static_cast<int>(S.mem.size());
    hub_basis T = S.T;
    for (int q = 0; q < nm; ++q) {
      const int k = S.mem[q];
      const char* src = static_cast<const char*>(traj) + static_cast<size_t>(members[k].start_step) * sbytes;
      void* dst = static_cast<char*>(S.buf) + static_cast<size_t>(q) * T->D.dim * es;
      HUB_HIP(hub::launch_cop(pi, T->D.dim, T->D.dim_dn, h->D.dim_dn, h->D.dim, 1, S.down, S.maps + (size_t)q * S.map_len,
                              S.sgns + static_cast<size_t>(q) * S.map_len, src, dst, st));
    }
    for (int q = 0; q < nm;) {  // the kernel takes 1, 2, 4 or 8 consecutive members
      int w = kMaxNV;
      while (w > nm - q) w /= 2;
      HUB_HIP(overlap_launch(S, q, w, 0, static_cast<char*>(S.buf) + static_cast<size_t>(q) * T->D.dim * es, false,
                             nullptr, st));
      q += w;
    }
  }
  HUB_HIP(hipStreamSynchronize(st));
  // 3. the sectors side by side (own stream and host thread each; groups of
  // a sector run on its handle's lanes)
  if (n_rel > 0) {
    std::vector<std::thread> threads;
    for (Sector& S : secs)
      threads.emplace_back([&, pS = &S]() {
        Sector& S = *pS;
        if (hipSetDevice(h->device) != hipSuccess) {
          S.s = HUB_E_DEVICE;
          S.err = "hipSetDevice failed";
          return;
        }
        try {
          const int nm = static_cast<int>(S.mem.size());
          std::vector<std::vector<double>> am(nm, std::vector<double>(n_rel));
          for (int q = 0; q < nm; ++q)
            for (int n = 0; n < n_rel; ++n)
              am[q][n] = pulse_value(*pulse, t_start + (members[S.mem[q]].start_step + n) * dt + 0.5 * dt);
          StepHook hk;
          hk.after = [&](int k0, int nv, int n_done, const void* state, const StepCtl* ctl, hipStream_t s_) {
            return overlap_launch(S, k0, nv, n_done, state, nv > 1, ctl, s_);
          };
          S.s = run_all(S.T, prec, nm, S.buf, n_rel, am, nullptr, t_start, dt, o1, nullptr, nullptr, S.stream,
                        nullptr, nullptr, &hk);
        } catch (const std::bad_alloc&) {
          S.s = fail(HUB_E_NOMEM, "host allocation failed");
        }
        if (S.s != HUB_OK) S.err = g_err;
      });
    for (auto& t : threads) t.join();
    for (const Sector& S : secs)
      if (S.s != HUB_OK) return cleanup(fail(S.s, S.err));
  }
  // 4. totals and the host copy
  std::vector<double> host;
  for (Sector& S : secs) {
    const int nm = static_cast<int>(S.mem.size());
    HUB_HIP(hub::launch_reduce_sets(S.part, static_cast<int64_t>(S.ogrid) * 2, (n_rel + 1) * nm, S.ogrid, 2, S.tot, 2,
                                    S.stream));
    host.assign(static_cast<size_t>(n_rel + 1) * nm * 2, 0.0);
    HUB_HIP(hipMemcpyAsync(host.data(), S.tot, host.size() * sizeof(double), hipMemcpyDeviceToHost, S.stream));
    HUB_HIP(hipStreamSynchronize(S.stream));
    for (int q = 0; q < nm; ++q)
      for (int n = 0; n <= n_rel; ++n)
        for (int c = 0; c < 2; ++c)
          overlaps[(static_cast<size_t>(S.mem[q]) * (n_rel + 1) + n) * 2 + c] =
              host[(static_cast<size_t>(n) * nm + q) * 2 + c];
  }
  return cleanup(HUB_OK);
}

// ---------------------------------------------------------------------------
// Ground state: restarted Lanczos with full reorthogonalisation (classical
// Gram-Schmidt applied twice), complex double; Ritz pairs from the
// tridiagonal by Jacobi rotations on the host.
namespace {

struct GSBufs {
  std::vector<void*> V;  // device vectors
  void** Vdev = nullptr;
  double2* coef = nullptr;
  double2* coef2 = nullptr;
};

hub_status gs_lanczos(hub_basis h, double A, hipStream_t st, GSBufs& G, int kmax, const void* deflate,
                      double tol_res, std::vector<double>& ritz, std::vector<double>& svec, int& kused,
                      double& resid) {
  const int64_t dim = h->D.dim;
  std::vector<double> cf(static_cast<size_t>(2) * kMaxNV * kMaxClasses, 0.0);
  coef_for(h->B, A, cf.data());
  std::vector<double> alpha, beta;
  // vectors used for orthogonalisation: [deflate] + V[0..j]
  std::vector<void*> basis;
  if (deflate) basis.push_back(const_cast<void*>(deflate));
  int j = 0;
  resid = INFINITY;
  for (j = 0; j < kmax; ++j) {
    basis.push_back(G.V[j]);
    void* w = G.V[j + 1];
    hub::ApplyLaunch L{};
    L.db = &h->D;
    L.prec = 0;
    L.nv = 1;
    L.rows = h->rows_c128;
    L.mode = hub::kPlain;
    L.coef = cf.data();
    L.x = G.V[j];
    L.y = w;
    L.stream = st;
    HUB_HIP(hub::launch_apply(L));
    HUB_HIP(hipMemcpyAsync(G.Vdev, basis.data(), basis.size() * sizeof(void*), hipMemcpyHostToDevice, st));
    HUB_HIP(hipStreamSynchronize(st));
    double a_j = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      const int nb = static_cast<int>(basis.size());
      for (int k0 = 0; k0 < nb; k0 += 64) {
        const int kk = std::min(64, nb - k0);
        HUB_HIP(hub::launch_multidot(dim, reinterpret_cast<const double2* const*>(G.Vdev) + k0, kk,
                                     static_cast<const double2*>(w), G.coef + k0, h->w.partials_e, st));
      }
      for (int k0 = 0; k0 < nb; k0 += 64) {
        const int kk = std::min(64, nb - k0);
        HUB_HIP(hub::launch_multiaxpy(dim, reinterpret_cast<const double2* const*>(G.Vdev) + k0, kk, G.coef + k0,
                                      static_cast<double2*>(w), st));
      }
      double2 cj;
      HUB_HIP(hipMemcpyAsync(&cj, G.coef + nb - 1, sizeof(double2), hipMemcpyDeviceToHost, st));
      HUB_HIP(hipStreamSynchronize(st));
      a_j += cj.x;
    }
    HUB_HIP(hub::launch_norm2(dim, static_cast<const double2*>(w), h->w.scal, h->w.partials_e, st));
    double n2 = 0.0;
    HUB_HIP(hipMemcpyAsync(&n2, h->w.scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HUB_HIP(hipStreamSynchronize(st));
    const double b_j = std::sqrt(n2);
    alpha.push_back(a_j);
    beta.push_back(b_j);
    // Ritz values of T_{j+1}
    const int m = j + 1;
    std::vector<double> T(static_cast<size_t>(m) * m, 0.0), vals, vecs;
    for (int i = 0; i < m; ++i) {
      T[static_cast<size_t>(i) * m + i] = alpha[i];
      if (i + 1 < m) T[static_cast<size_t>(i) * m + i + 1] = T[static_cast<size_t>(i + 1) * m + i] = beta[i];
    }
    hub::sym_eig(m, T, vals, vecs);
    resid = b_j * std::fabs(vecs[static_cast<size_t>(m - 1) * m + 0]);
    ritz = vals;
    svec.assign(m, 0.0);
    for (int i = 0; i < m; ++i) svec[i] = vecs[static_cast<size_t>(i) * m + 0];
    kused = m;
    if (resid < tol_res || b_j < 1e-14 * h->B.norm_inf || m == dim - (deflate ? 1 : 0)) break;
    HUB_HIP(hub::launch_scale(dim, static_cast<double2*>(w), h->w.scal, double2{0, 0}, st));
  }
  return HUB_OK;
}

// x = sum_i s_i V[i] into `out`
hub_status gs_ritz_vector(hub_basis h, hipStream_t st, GSBufs& G, const std::vector<double>& s, void* out) {
  const int64_t dim = h->D.dim;
  const int m = static_cast<int>(s.size());
  HUB_HIP(hipMemsetAsync(out, 0, dim * 16, st));
  std::vector<double2> c(m);
  for (int i = 0; i < m; ++i) c[i] = double2{-s[i], 0.0};  // multiaxpy subtracts
  HUB_HIP(hipMemcpyAsync(G.coef, c.data(), m * sizeof(double2), hipMemcpyHostToDevice, st));
  HUB_HIP(hipMemcpyAsync(G.Vdev, G.V.data(), m * sizeof(void*), hipMemcpyHostToDevice, st));
  HUB_HIP(hipStreamSynchronize(st));
  for (int k0 = 0; k0 < m; k0 += 64) {
    const int kk = std::min(64, m - k0);
    HUB_HIP(hub::launch_multiaxpy(dim, reinterpret_cast<const double2* const*>(G.Vdev) + k0, kk, G.coef + k0,
                                  static_cast<double2*>(out), st));
  }
  // normalise
  HUB_HIP(hub::launch_norm2(dim, static_cast<const double2*>(out), h->w.scal, h->w.partials_e, st));
  HUB_HIP(hub::launch_scale(dim, static_cast<double2*>(out), h->w.scal, double2{0, 0}, st));
  HUB_HIP(hipStreamSynchronize(st));
  return HUB_OK;
}

}  // namespace

hub_status hub_ground_state(hub_basis h, double A, const hub_krylov_opts* opts, void* v_out, double* E0,
                            double* gap, void* stream) {
  hub_status s = check_common(h, HUB_C128, 1);
  if (s != HUB_OK) return s;
  if (!v_out || !E0) return fail(HUB_E_INVALID, "null argument");
  if (!std::isfinite(A)) return fail(HUB_E_INVALID, "non-finite A");
  const double tol = opts ? opts->tol : 1e-12;
  int kmax = opts ? opts->m_max : 60;
  if (!(tol > 0.0)) return fail(HUB_E_INVALID, "opts.tol must be > 0");
  if (kmax < 2) return fail(HUB_E_INVALID, "opts.m_max must be >= 2");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t dim = h->D.dim;
  kmax = static_cast<int>(std::min<int64_t>(kmax, dim));
  s = ensure_workspace(h, static_cast<size_t>(dim) * 16, kmax + 1, 0);
  if (s != HUB_OK) return s;
  GSBufs G;
  for (int k = 0; k <= kmax; ++k) G.V.push_back(static_cast<char*>(h->w.slots) + static_cast<size_t>(k) * dim * 16);
  void* extra = nullptr;
  HUB_HIP(hipMalloc(&extra, (kmax + 2) * (sizeof(void*) + 2 * sizeof(double2))));
  struct Fr {
    void* p;
    ~Fr() { (void)hipFree(p); }
  } fr{extra};
  G.Vdev = static_cast<void**>(extra);
  G.coef = reinterpret_cast<double2*>(static_cast<char*>(extra) + (kmax + 2) * sizeof(void*));
  G.coef2 = G.coef + (kmax + 2);

  // seeded random start (host), normalised on the device
  auto random_start = [&](void* dst, uint64_t seed) -> hub_status {
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<double2> x(static_cast<size_t>(dim));
    for (auto& e : x) e = double2{nd(rng), nd(rng)};
    HUB_HIP(hipMemcpy(dst, x.data(), x.size() * sizeof(double2), hipMemcpyHostToDevice));
    HUB_HIP(hub::launch_norm2(dim, static_cast<const double2*>(dst), h->w.scal, h->w.partials_e, st));
    HUB_HIP(hub::launch_scale(dim, static_cast<double2*>(dst), h->w.scal, double2{0, 0}, st));
    return HUB_OK;
  };
  const double tol_res = tol * h->B.norm_inf;
  s = random_start(G.V[0], 0x13498ULL);
  if (s != HUB_OK) return s;
  std::vector<double> ritz, svec;
  int kused = 0;
  double resid = INFINITY, e0 = 0.0;
  bool conv = false;
  for (int restart = 0; restart < 200; ++restart) {
    s = gs_lanczos(h, A, st, G, kmax, nullptr, tol_res, ritz, svec, kused, resid);
    if (s != HUB_OK) return s;
    e0 = ritz[0];
    s = gs_ritz_vector(h, st, G, svec, v_out);
    if (s != HUB_OK) return s;
    if (resid < tol_res) {
      conv = true;
      break;
    }
    HUB_HIP(hipMemcpyAsync(G.V[0], v_out, dim * 16, hipMemcpyDeviceToDevice, st));
  }
  if (!conv) return fail(HUB_E_NOT_CONVERGED, "ground-state Lanczos did not reach the tolerance");
  // phase: largest-modulus component (lowest index within 1e-12 of the max) real positive
  HUB_HIP(hub::launch_absmax(dim, static_cast<const double2*>(v_out), h->w.scal, h->w.partials_e, st));
  double mx2 = 0.0;
  HUB_HIP(hipMemcpyAsync(&mx2, h->w.scal, sizeof(double), hipMemcpyDeviceToHost, st));
  HUB_HIP(hipStreamSynchronize(st));
  const double th = mx2 * (1.0 - 1e-12) * (1.0 - 1e-12);
  HUB_HIP(hipMemcpy(h->w.scal + 1, &th, sizeof(double), hipMemcpyHostToDevice));
  HUB_HIP(hub::launch_first_above(dim, static_cast<const double2*>(v_out), h->w.scal + 1,
                                  reinterpret_cast<int64_t*>(h->w.scal + 2), reinterpret_cast<int64_t*>(h->w.partials_e),
                                  st));
  int64_t kmaxidx = 0;
  HUB_HIP(hipMemcpyAsync(&kmaxidx, h->w.scal + 2, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HUB_HIP(hipStreamSynchronize(st));
  double2 comp;
  HUB_HIP(hipMemcpy(&comp, static_cast<double2*>(v_out) + kmaxidx, sizeof(double2), hipMemcpyDeviceToHost));
  const double mag = std::hypot(comp.x, comp.y);
  HUB_HIP(hub::launch_scale(dim, static_cast<double2*>(v_out), nullptr, double2{comp.x / mag, -comp.y / mag}, st));
  *E0 = e0;
  // gap: lowest Ritz value of H restricted to the complement of the ground state
  double g = INFINITY;
  if (dim > 1) {
    s = random_start(G.V[0], 0x5eedULL);
    if (s != HUB_OK) return s;
    // remove the ground-state component of the start vector
    HUB_HIP(hipMemcpyAsync(G.Vdev, &v_out, sizeof(void*), hipMemcpyHostToDevice, st));
    HUB_HIP(hipStreamSynchronize(st));
    HUB_HIP(hub::launch_multidot(dim, reinterpret_cast<const double2* const*>(G.Vdev), 1,
                                 static_cast<const double2*>(G.V[0]), G.coef, h->w.partials_e, st));
    HUB_HIP(hub::launch_multiaxpy(dim, reinterpret_cast<const double2* const*>(G.Vdev), 1, G.coef,
                                  static_cast<double2*>(G.V[0]), st));
    HUB_HIP(hub::launch_norm2(dim, static_cast<const double2*>(G.V[0]), h->w.scal, h->w.partials_e, st));
    HUB_HIP(hub::launch_scale(dim, static_cast<double2*>(G.V[0]), h->w.scal, double2{0, 0}, st));
    double r1 = INFINITY;
    for (int restart = 0; restart < 20; ++restart) {
      s = gs_lanczos(h, A, st, G, kmax, v_out, 1e-6 * h->B.norm_inf, ritz, svec, kused, r1);
      if (s != HUB_OK) return s;
      if (r1 < 1e-6 * h->B.norm_inf) break;
      void* tmp = G.V[kmax];  // Ritz vector into the spare slot, then restart from it
      s = gs_ritz_vector(h, st, G, svec, tmp);
      if (s != HUB_OK) return s;
      HUB_HIP(hipMemcpyAsync(G.V[0], tmp, dim * 16, hipMemcpyDeviceToDevice, st));
    }
    g = ritz[0] - e0;
  }
  HUB_HIP(hipStreamSynchronize(st));
  if (gap) *gap = g;
  if (g < 1e-8 * h->B.norm_inf) return fail(HUB_E_DEGENERATE, "ground state is degenerate within 1e-8 |H|");
  return HUB_OK;
}

// ---------------------------------------------------------------------------
// Learned Krylov controller: MLP kernels and the controlled schedule.
hub_status hub_mlp_forward(int32_t device, const float* params, int32_t n_rows, const float* feats, float* out,
                           void* stream) {
  if (!params || !feats || !out) return fail(HUB_E_INVALID, "null argument");
  if (n_rows < 0) return fail(HUB_E_INVALID, "n_rows must be >= 0");
  HUB_HIP(hipSetDevice(device));
  HUB_HIP(hub::launch_mlp_forward(params, n_rows, feats, out, static_cast<hipStream_t>(stream)));
  return HUB_OK;
}

int64_t hub_mlp_workspace_bytes(int32_t n_rows) { return n_rows < 1 ? 0 : hub::mlp_workspace_bytes(n_rows); }

hub_status hub_mlp_train_step(int32_t device, float* params, float* adam_m, float* adam_v, int32_t t, float lr,
                              int32_t n_rows, const float* feats, const float* targets, float* loss, void* workspace,
                              void* stream) {
  if (!params || !adam_m || !adam_v || !feats || !targets || !loss || !workspace)
    return fail(HUB_E_INVALID, "null argument");
  if (n_rows < 1) return fail(HUB_E_INVALID, "n_rows must be >= 1");
  if (t < 1) return fail(HUB_E_INVALID, "Adam step count t must be >= 1");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(HUB_E_INVALID, "lr must be finite and > 0");
  HUB_HIP(hipSetDevice(device));
  HUB_HIP(hub::launch_mlp_train_step(params, adam_m, adam_v, t, lr, n_rows, feats, targets, loss, workspace,
                                     static_cast<hipStream_t>(stream)));
  return HUB_OK;
}

hub_status hub_controller_features(const hub_pulse* pulse, double t_start, double dt, int32_t n_steps,
                                   double norm_inf, const hub_krylov_opts* opts, const hub_step_info* log,
                                   int32_t chunk, float* feats, float* targets) {
  if (!pulse || !opts || !log || !feats || !targets) return fail(HUB_E_INVALID, "null argument");
  if (n_steps < 0 || chunk < 1) return fail(HUB_E_INVALID, "n_steps must be >= 0 and chunk >= 1");
  hub_status s = check_pulse(*pulse);
  if (s != HUB_OK) return s;
  if ((s = check_opts(*opts)) != HUB_OK) return s;
  if (!std::isfinite(dt) || !std::isfinite(t_start) || !std::isfinite(norm_inf))
    return fail(HUB_E_INVALID, "non-finite argument");
  const double tau = dt / solves_per_step(*opts);
  for (int n = 0; n < n_steps; ++n) {
    const int hs = n - 1 - (n % chunk);
    double eh[4];
    for (int q = 0; q < 4; ++q) eh[q] = (hs - q >= 0) ? log[hs - q].err_est : NAN;
    const int m_last = hs >= 0 ? log[hs].m_used : -1;
    const double tm = t_start + n * dt + 0.5 * dt;
    ctrl_features(pulse_value(*pulse, tm), pulse_deriv(*pulse, tm), tau * norm_inf, eh, m_last, opts->tol,
                  opts->m_hint, feats + static_cast<size_t>(n) * HUB_MLP_IN);
    targets[static_cast<size_t>(n) * HUB_MLP_OUT] = static_cast<float>(std::log2(std::max(1, log[n].m_used)));
  }
  return HUB_OK;
}

hub_status hub_controller_load(hub_basis h, const float* params, int32_t n_params) {
  if (!h || !params) return fail(HUB_E_INVALID, "null argument");
  if (n_params != HUB_MLP_NPARAM) return fail(HUB_E_INVALID, "n_params must be HUB_MLP_NPARAM");
  if (h->device < 0) return fail(HUB_E_DEVICE, "host-only handle (created with device -1)");
  for (int k = 0; k < n_params; ++k)
    if (!std::isfinite(params[k])) return fail(HUB_E_INVALID, "non-finite controller parameter");
  HUB_HIP(hipSetDevice(h->device));
  const size_t rows = static_cast<size_t>(kCtrlMaxChunk) * kMaxNV;
  if (!h->ctrl_params) {
    HUB_HIP(hipMalloc(reinterpret_cast<void**>(&h->ctrl_params), HUB_MLP_NPARAM * sizeof(float)));
    HUB_HIP(hipMalloc(reinterpret_cast<void**>(&h->ctrl_feat), rows * HUB_MLP_IN * sizeof(float)));
    HUB_HIP(hipMalloc(reinterpret_cast<void**>(&h->ctrl_out), rows * HUB_MLP_OUT * sizeof(float)));
    HUB_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->ctrl_hfeat), rows * HUB_MLP_IN * sizeof(float)));
    HUB_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->ctrl_hout), rows * HUB_MLP_OUT * sizeof(float)));
  }
  HUB_HIP(hipMemcpy(h->ctrl_params, params, HUB_MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
  h->ctrl_loaded = true;
  return HUB_OK;
}

hub_status hub_controller_enable(hub_basis h, int32_t on, int32_t chunk, int32_t margin) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (on && !h->ctrl_loaded) return fail(HUB_E_INVALID, "no controller parameters loaded");
  if (on && (chunk < 1 || chunk > kCtrlMaxChunk)) return fail(HUB_E_INVALID, "chunk must be in [1, 256]");
  if (on && (margin < 0 || margin > 16)) return fail(HUB_E_INVALID, "margin must be in [0, 16]");
  h->ctrl_on = on != 0;
  if (on) {
    h->ctrl_chunk = chunk;
    h->ctrl_margin = margin;
  }
  return HUB_OK;
}

hub_status hub_controller_read_stats(hub_basis h, hub_controller_stats* out) {
  if (!h || !out) return fail(HUB_E_INVALID, "null argument");
  *out = h->cstats;
  h->cstats = hub_controller_stats{};
  return HUB_OK;
}

hub_status hub_spectral(int32_t device, int32_t n_members, int32_t n_s, const double* overlaps, const int32_t* lesser,
                        double dt, double eps, int32_t n_nu, const double* nu, double* out, void* stream) {
  if (n_members < 0 || n_s < 0 || n_nu < 0) return fail(HUB_E_INVALID, "negative size");
  if (n_members == 0 || n_nu == 0) return HUB_OK;
  if (!overlaps || !lesser || !nu || !out) return fail(HUB_E_INVALID, "null argument");
  if (!std::isfinite(dt) || !(dt > 0.0) || !std::isfinite(eps) || eps < 0.0)
    return fail(HUB_E_INVALID, "dt must be > 0 and eps >= 0, both finite");
  HUB_HIP(hipSetDevice(device));
  HUB_HIP(hub::launch_spectral(n_members, n_s, overlaps, lesser, dt, eps, n_nu, nu, out,
                               static_cast<hipStream_t>(stream)));
  return HUB_OK;
}

// ---------------------------------------------------------------------------
// Kernel plan tuning.
namespace {

int gidx(int g) { return g == 1 ? 0 : (g == 2 ? 1 : (g == 4 ? 2 : 3)); }

// Can group size g run on path (0 one pass, 1 two pass) for precision pi?
bool path_feasible(const DevBasis& D, int pi, int g, int path) {
  DevBasis T = D;
  T.two_pass = path;
  T.block_path = path ? -1 : 0;
  T.tuned_single[pi] = -1;
  for (int k = 0; k < 4; ++k) T.tuned_block[pi][k] = -1;
  if (g == 1) return path ? hub::apply_two_pass(T, pi, 1, hub::kPlain, false) : true;
  if (path) return hub::block_two_pass(T, pi, g);
  return hub::apply_lds_bytes(T, pi, g, 1) <= 150 * 1024;
}

}  // namespace

hub_status hub_tune(hub_basis h, hub_prec prec, int32_t reps, hub_tuning* out, void* stream) {
  hub_status s = check_common(h, prec, 1);
  if (s != HUB_OK) return s;
  if (!out) return fail(HUB_E_INVALID, "null output");
  if (reps < 1) return fail(HUB_E_INVALID, "reps must be >= 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int pi = prec == HUB_C128 ? 0 : 1;
  const size_t es = elem_bytes(prec);
  const int64_t dim = h->D.dim;
  constexpr int kN = kMaxNV;  // vectors per measured call
  void* x = nullptr;
  void* y = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const DevBasis saved = h->D;
  const int saved_ag = h->apply_group[pi], saved_pg = h->prop_group[pi], saved_pgl = h->prop_group_large[pi];
  // the plans are the launch path's: its propagations are timed, not the resident stepper's
  const int saved_path = h->prop_path;
  h->prop_path = 0;
  auto done = [&](hub_status r) {
    h->D = saved;
    h->force_group = 0;
    h->prop_path = saved_path;
    if (r != HUB_OK) {
      h->apply_group[pi] = saved_ag;
      h->prop_group[pi] = saved_pg;
      h->prop_group_large[pi] = saved_pgl;
    }
    if (x) (void)hipFree(x);
    if (y) (void)hipFree(y);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return r;
  };
  // a failed HIP call restores the handle and frees the buffers before it returns
#define TUNE_HIP(call)                                                                                     \
  do {                                                                                                     \
    const hipError_t e_ = (call);                                                                          \
    if (e_ != hipSuccess) return done(fail(HUB_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_))); \
  } while (0)
  if (hipMalloc(&x, static_cast<size_t>(dim) * kN * es) != hipSuccess ||
      hipMalloc(&y, static_cast<size_t>(dim) * kN * es) != hipSuccess)
    return done(fail(HUB_E_NOMEM, "tuning buffers"));
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return done(fail(HUB_E_DEVICE, "event creation failed"));
  if (hub::launch_fill_probe(pi, dim * kN, x, st) != hipSuccess) return done(fail(HUB_E_DEVICE, "fill kernel"));
  hub_tuning T{};
  const double A[kN] = {0.5, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5};
  // 1. plain H*v of kN vectors in groups of g on either path
  for (int g : {1, 2, 4, 8})
    for (int path = 0; path < 2; ++path) {
      if (!path_feasible(saved, pi, g, path)) continue;
      h->D = saved;
      h->D.two_pass = path;
      h->D.block_path = path ? -1 : 0;
      h->force_group = g;
      for (int r = 0; r < 2; ++r)
        if ((s = hub_apply_H(h, A, prec, kN, x, y, stream)) != HUB_OK) return done(s);
      TUNE_HIP(hipEventRecord(e0, st));
      for (int r = 0; r < reps; ++r)
        if ((s = hub_apply_H(h, A, prec, kN, x, y, stream)) != HUB_OK) return done(s);
      TUNE_HIP(hipEventRecord(e1, st));
      TUNE_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      TUNE_HIP(hipEventElapsedTime(&ms, e0, e1));
      T.apply_us[gidx(g)][path] = 1e3 * ms / (static_cast<double>(reps) * kN);
    }
  auto best_path = [&](int g) {
    const double* u = T.apply_us[gidx(g)];
    if (u[0] > 0.0 && u[1] > 0.0) return u[1] < u[0] ? 1 : 0;
    return u[1] > 0.0 ? 1 : 0;
  };
  T.single_two_pass = best_path(1);
  for (int g : {2, 4, 8}) T.block_two_pass[gidx(g)] = best_path(g);
  // install the path choices
  h->D = saved;
  h->D.tuned_single[pi] = T.single_two_pass;
  for (int g : {2, 4, 8}) h->D.tuned_block[pi][gidx(g)] = T.block_two_pass[gidx(g)];
  const DevBasis chosen = h->D;
  double best = 0.0;
  for (int g : {1, 2, 4, 8}) {
    const int path = g == 1 ? T.single_two_pass : T.block_two_pass[gidx(g)];
    const double u = T.apply_us[gidx(g)][path];
    if (u > 0.0 && (best == 0.0 || u < best)) {
      best = u;
      T.apply_group = g;
    }
  }
  // 2. midpoint steps of nv vectors in groups of g (the chosen paths), dt
  // such that dt |H|_inf = 1/2, tol 1e-10: time per vector-step, for nv =
  // kN (a group of 8 then runs on one lane) and nv = kN * kMaxLanes (every
  // group size fills the concurrent lanes)
  hub_krylov_opts o{};
  o.tol = 1e-10;
  o.m_max = 30;
  o.substeps = 1;
  const double dtp = 0.5 / std::max(h->B.norm_inf, 1e-300);
  constexpr int kNL = kN * kMaxLanes;
  std::vector<std::vector<double>> am(kNL, std::vector<double>(3, 0.5));
  auto time_steps = [&](int nv, void* buf, int g, double* us_per_vector_step) -> hub_status {
    h->D = chosen;
    h->force_group = g;
    if (hub::launch_fill_probe(pi, dim * nv, buf, st) != hipSuccess) return fail(HUB_E_DEVICE, "fill kernel");
    hub_status r = run_all(h, prec, nv, buf, 1, am, nullptr, 0.0, dtp, o, nullptr, nullptr, stream);
    if (r != HUB_OK) return r;
    if (hipStreamSynchronize(st) != hipSuccess) return fail(HUB_E_DEVICE, "tuning: stream synchronisation");
    const auto t0 = std::chrono::steady_clock::now();
    if ((r = run_all(h, prec, nv, buf, 2, am, nullptr, 0.0, dtp, o, nullptr, nullptr, stream)) != HUB_OK) return r;
    if (hipStreamSynchronize(st) != hipSuccess) return fail(HUB_E_DEVICE, "tuning: stream synchronisation");
    *us_per_vector_step = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() /
                          (2.0 * nv);
    return HUB_OK;
  };
  auto group_ok = [&](int g) {
    return g == 1 || hub::block_two_pass(chosen, pi, g) || hub::apply_lds_bytes(chosen, pi, g, 1) <= 150 * 1024;
  };
  best = 0.0;
  for (int g : {1, 2, 4, 8}) {
    if (!group_ok(g)) continue;
    if ((s = time_steps(kN, x, g, &T.step_us[gidx(g)])) != HUB_OK) return done(s);
    if (best == 0.0 || T.step_us[gidx(g)] < best) {
      best = T.step_us[gidx(g)];
      T.prop_group = g;
    }
  }
  // the larger batch in its own buffer, each group size only where its
  // vectors and the lanes' Krylov workspaces fit the free device memory
  T.prop_group_large = T.prop_group;
  void* xl = nullptr;
  size_t mem_free = 0, mem_total = 0;
  const size_t vec_b = static_cast<size_t>(dim) * es;
  if (hipMemGetInfo(&mem_free, &mem_total) == hipSuccess && mem_free > kNL * vec_b &&
      hipMalloc(&xl, kNL * vec_b) == hipSuccess) {
    best = 0.0;
    for (int g : {1, 2, 4, 8}) {
      if (!group_ok(g)) continue;
      const size_t lanes = std::min<size_t>(kMaxLanes, kNL / g);
      const size_t need = lanes * static_cast<size_t>(o.m_max + 2) * g * vec_b;
      if (hipMemGetInfo(&mem_free, &mem_total) != hipSuccess || need + need / 8 > mem_free) continue;
      if ((s = time_steps(kNL, xl, g, &T.step_us_large[gidx(g)])) != HUB_OK) {
        (void)hipFree(xl);
        return done(s);
      }
      if (best == 0.0 || T.step_us_large[gidx(g)] < best) {
        best = T.step_us_large[gidx(g)];
        T.prop_group_large = g;
      }
    }
    TUNE_HIP(hipFree(xl));
  }
  h->D = chosen;
  h->force_group = 0;
  h->prop_path = saved_path;
  h->apply_group[pi] = T.apply_group;
  h->prop_group[pi] = T.prop_group;
  h->prop_group_large[pi] = T.prop_group_large;
  *out = T;
  if (x) (void)hipFree(x);
  if (y) (void)hipFree(y);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return HUB_OK;
#undef TUNE_HIP
}

hub_status hub_set_tuning(hub_basis h, hub_prec prec, const hub_tuning* t) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (prec != HUB_C128 && prec != HUB_C64) return fail(HUB_E_INVALID, "unknown precision");
  const int pi = prec == HUB_C128 ? 0 : 1;
  if (!t) {  // back to the built-in rules
    h->D.tuned_single[pi] = -1;
    for (int k = 0; k < 4; ++k) h->D.tuned_block[pi][k] = -1;
    h->apply_group[pi] = h->prop_group[pi] = h->prop_group_large[pi] = -1;
    return HUB_OK;
  }
  auto pow2 = [](int g) { return g == 1 || g == 2 || g == 4 || g == 8; };
  if (!pow2(t->apply_group) || !pow2(t->prop_group) || !pow2(t->prop_group_large) ||
      (t->single_two_pass != 0 && t->single_two_pass != 1))
    return fail(HUB_E_INVALID, "tuning: groups must be 1, 2, 4 or 8 and paths 0 or 1");
  for (int k = 1; k < 4; ++k)
    if (t->block_two_pass[k] != 0 && t->block_two_pass[k] != 1) return fail(HUB_E_INVALID, "tuning: block path");
  h->D.tuned_single[pi] = t->single_two_pass;
  for (int k = 1; k < 4; ++k) h->D.tuned_block[pi][k] = t->block_two_pass[k];
  h->apply_group[pi] = t->apply_group;
  h->prop_group[pi] = t->prop_group;
  h->prop_group_large[pi] = t->prop_group_large;
  return HUB_OK;
}

hub_status hub_get_plan(hub_basis h, hub_prec prec, int32_t nvec, int32_t propagate, int32_t* n_groups,
                        int32_t* sizes, int32_t* kernels) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (prec != HUB_C128 && prec != HUB_C64) return fail(HUB_E_INVALID, "unknown precision");
  if (nvec < 1 || !n_groups) return fail(HUB_E_INVALID, "nvec must be >= 1 and n_groups non-null");
  const int pi = prec == HUB_C128 ? 0 : 1;
  const std::vector<int> g = groups_for(h, nvec, pi, propagate != 0);
  *n_groups = static_cast<int32_t>(g.size());
  for (size_t k = 0; k < g.size(); ++k) {
    if (sizes) sizes[k] = g[k];
    if (kernels) {
      if (g[k] > 1) kernels[k] = hub::block_two_pass(h->D, pi, g[k]) ? 2 : 0;
      else kernels[k] = hub::apply_two_pass(h->D, pi, 1, propagate ? hub::kLanczos : hub::kPlain, false) ? 1 : 0;
    }
  }
  return HUB_OK;
}

hub_status hub_set_schedule(hub_basis h, int32_t chunk, int32_t margin) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (chunk < 0 || chunk > kCtrlMaxChunk) return fail(HUB_E_INVALID, "chunk must be in [0, 256]");
  if (margin < 0 || margin > 16) return fail(HUB_E_INVALID, "margin must be in [0, 16]");
  h->sched_chunk = chunk;
  h->sched_margin = margin;
  return HUB_OK;
}

hub_status hub_set_apply_path(hub_basis h, int32_t path) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (path < -1 || path > 1) return fail(HUB_E_INVALID, "path must be -1, 0 or 1");
  h->D.two_pass = path;
  h->D.block_path = path == 0 ? 0 : -1;
  return HUB_OK;
}

hub_status hub_set_propagate_path(hub_basis h, int32_t path) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (path < -1 || path > 1) return fail(HUB_E_INVALID, "path must be -1, 0 or 1");
  h->prop_path = path;
  return HUB_OK;
}

hub_status hub_set_greens_path(hub_basis h, int32_t path) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (path < -1 || path > 1) return fail(HUB_E_INVALID, "path must be -1, 0 or 1");
  h->greens_path = path;
  return HUB_OK;
}

// ---------------------------------------------------------------------------
hub_status hub_profile_enable(hub_basis h, int32_t on) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  if (on < 0) return fail(HUB_E_INVALID, "on must be >= 0");
  h->prof = on != 0;
  h->prof_period = on > 0 ? on : 1;
  h->prof_count = 0;
  if (on > 0) {  // events for a few thousand samples (recycled when they run low)
    HUB_HIP(hipSetDevice(h->device));
    while (h->ev_free.size() < kProfPool) {
      hipEvent_t e;
      HUB_HIP(hipEventCreate(&e));
      h->ev_free.push_back(e);
    }
  }
  return HUB_OK;
}

hub_status hub_profile_read(hub_basis h, int64_t* launches, double* total_ms, double* bytes_per_launch) {
  if (!h) return fail(HUB_E_INVALID, "null basis handle");
  HUB_HIP(hipSetDevice(h->device));
  HUB_HIP(hipDeviceSynchronize());
  size_t end = 0;
  hub_status r = prof_harvest(h, 0, &end);
  if (r != HUB_OK) return r;
  double tot = 0.0;
  int64_t cnt = 0;
  for (const ProfSample& p : h->prof_samples) {
    if (p.worked == 0) continue;
    tot += p.ms;
    ++cnt;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = tot;
  if (bytes_per_launch) *bytes_per_launch = h->prof_bytes;
  h->prof_samples.clear();
  return HUB_OK;
}

}  // extern "C"
