// Device data structures and launchers of the HIP kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "basis.h"

namespace hub {

constexpr int kMMax = 60;                       // largest Krylov dimension (one wavefront)
constexpr int kObsQ = 4;  // <D>, docc, |x|^2, Re <x|K(t_obs)|x> (all unnormalised)
constexpr int kMaxNV = 8;                       // vectors per interleaved block
constexpr int kBlock = 256;                     // threads per workgroup

// Krylov state of one vector during one step, device resident.
struct VecState {
  double alpha[kMMax];       // T_jj
  double beta[kMMax];        // T_{j+1,j}
  double scale[kMMax + 1];   // v_k = scale[k] * u_k (u_k stored unnormalised)
  double y[2 * kMMax];       // y^(j) = exp(-i tau T_j) e_1 of the last iteration
  double beta0;              // |v| at the step start
  double eps;                // a-posteriori estimate of the last iteration
  double tau;                // step length of the current Krylov step
  int32_t m;                 // Krylov vectors in use (iterations done)
  int32_t status;            // 0 running, 1 converged, 2 invariant subspace, 3 hit m_max
  double obs[kObsQ];         // observables of the step's first vector (unnormalised)
  double site[kMaxSites];    // site-resolved double occupation
};

struct StepCtl {
  int32_t all_done;          // every vector of the block has stopped
  int32_t iter;              // Lanczos iterations completed in this step
  int32_t m_max;
  int32_t any_maxed;         // some vector reached m_max in this step
  int32_t abort;             // a step ended undecided: later kernels do nothing
  int32_t steps_done;        // (sub)steps logged since the host last cleared it
  int32_t eps_stop;          // fused iteration j whose row pass found the estimate for m = j below tol, else -1
  int32_t halt_from;         // > 0: (sub)step sequence number from which combines do nothing (a vector hit m_max)
  double tol;
  double norm_inf;
};

// Device copy of a basis.
struct DevBasis {
  int dim_up = 0, dim_dn = 0, nc = 0, n_sites = 0;
  int64_t dim = 0;
  double U = 0.0;
  uint32_t* up_bits = nullptr;
  uint32_t* dn_bits = nullptr;
  double* eps_up = nullptr;      // null if no on-site energies
  double* eps_dn = nullptr;
  int32_t* up_ptr = nullptr;     // [dim_up + 1] hop ranges of each up string
  uint32_t* up_hops = nullptr;   // src | class << 16 | sign << 31
  uint16_t* dn_tab = nullptr;    // [dim_dn][maxs_pad] staged-row index src + sign * (dim_dn + 1), pad dim_dn
  uint8_t slot_class[64] = {0};  // class of every down slot (uniform over strings)
  int nslots = 0, maxs_pad = 8;
  // the same padded, class-sorted table for the up strings (column pass)
  uint16_t* up_tab = nullptr;    // [dim_up][up_maxs_pad] index src + sign * (dim_up + 1), pad dim_up
  uint8_t up_slot_class[64] = {0};
  int up_nslots = 0, up_maxs_pad = 8;
  // grouped tables of the block apply (class ranges rounded up to a multiple
  // of four slots): [dim][gslots] entries as above, class of every group
  uint16_t* dn_tabg = nullptr;
  uint16_t* up_tabg = nullptr;
  uint8_t dn_gclass[8] = {0};
  uint8_t up_gclass[8] = {0};
  int dn_gslots = 0, up_gslots = 0;
  int two_pass = -1;             // -1 automatic, 0 never, 1 whenever it fits
  int block_path = -1;           // blocks of vectors: -1 two-pass block kernels where they fit, 0 one pass
  // tuned choices per precision [c128, c64] (-1 = the built-in rule), used
  // while two_pass / block_path are automatic: single vectors two-pass (1) or
  // one pass (0); blocks of 2, 4, 8 ([1], [2], [3]) on the two-pass block
  // kernels (1) or the one-pass kernel (0)
  int tuned_single[2] = {-1, -1};
  int tuned_block[2][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}};
  int up_max_hops = 0, dn_max_hops = 0;
};

enum ApplyMode : int {
  kPlain = 0,     // y = H x
  kLanczos = 1,   // y = s_j H u_j - beta_{j-1} s_{j-1} u_{j-1}, alpha_j reduced
  kObsOnly = 2,   // observables of x, no y
};

struct ApplyLaunch {
  const DevBasis* db;
  int prec;              // 0 = c128, 1 = c64
  int nv;                // vectors interleaved per (a, b): 1, 2, 4, 8
  int rows;              // rows of the tile per workgroup
  int mode;
  bool obs;              // also accumulate observables of x (Lanczos/obs modes)
  const void* x;
  void* y;
  const void* xprev;     // Lanczos: u_{j-1} (null at j = 0)
  const double* coef;    // host [nv][nc] complex pairs (copied into the launch arguments)
  const double* coef_obs;  // host [nv][nc] hop coefficients at the observation time (obs modes)
  VecState* st;          // device [nv] (Lanczos/obs)
  StepCtl* ctl;
  int j;                 // Lanczos iteration (0-based); the Krylov decision for m = j is taken here
  int m_max;
  double tol, norm_inf;
  double* partials;      // device [grid][nq][nv] partial sums written by this launch
  const double* prev_partials;  // Lanczos: |u_j|^2 (or |v|^2) partials [prev_nblk][nv]
  int prev_nblk;
  hipStream_t stream;
  // optional timing events attached to the dispatches: start/end of the
  // (first) kernel, and of the column pass when the apply has two kernels
  hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev2_start = nullptr, ev2_stop = nullptr;
  // two-pass Lanczos apply with observables: the row pass's obs partials
  // [dim_up][kObsQ][nv] go here (the column pass writes alpha and the up-hop part)
  double* row_obs = nullptr;
  // two-pass Lanczos iteration j >= 2 with the update of u_j fused into the
  // row pass: alpha_{j-1} from the previous column pass's partials, |u_j|^2
  // partials [dim_up] to norm_partials, the Krylov decision in the column pass
  bool fuse = false;
  const double* alpha_partials = nullptr;
  int alpha_nblk = 0;
  int alpha_stride = 1;             // columns of alpha_partials (2 after an observables apply)
  const double* obs_row = nullptr;  // fused j = 1 after an observables apply: its row-pass obs partials
  double* norm_partials = nullptr;
};

// Each launcher returns the hipError_t of its launch.
// grid_out: workgroups of the kernel that wrote the launch's partial sums.
hipError_t launch_apply(const ApplyLaunch& L, int* grid_out = nullptr);
int apply_grid(const DevBasis& db, int prec, int nv);    // most workgroups any apply kernel writes partials for
// Two-pass apply of blocks of nv = 2, 4, 8 interleaved vectors (a row pass
// and a column pass, each staging its tile row or column of the whole block
// once in LDS): where the grouped tables and the staged row and column fit.
// The column pass writes its partial sums for dim_dn workgroups.
bool block_two_pass(const DevBasis& db, int prec, int nv);
size_t block_lds_bytes(const DevBasis& db, int prec, int nv);
// Two-pass apply (single vectors, plain and Lanczos modes): a row pass does
// the diagonal and the down hops, a column pass stages kColW columns of x
// for all up strings in LDS and adds the up hops (and the Lanczos epilogue).
constexpr int kColW = 4;
bool apply_two_pass(const DevBasis& db, int prec, int nv, int mode, bool obs);
// Rows whose staged copy (+x, -x) exceeds the LDS budget (16 sites): the
// one-pass kernel then gathers the down hops from the row in global memory.
bool apply_global_rows(const DevBasis& db, int prec, int nv);
int colpass_width(const DevBasis& db, int prec);    // columns per column-pass workgroup (kColW or 2)
bool colpass_single(const DevBasis& db, int prec);  // one staged copy of the columns (sign from the index)
int colpass_grid(const DevBasis& db, int prec);
size_t colpass_lds_bytes(const DevBasis& db, int prec);
int apply_chunks(const DevBasis& db, int prec, int nv);  // column chunks per tile row
int apply_nq(int mode, bool obs, int nc);
// Partial columns the column pass of a two-pass Lanczos apply writes; with
// observables the row pass writes its kObsQ columns to ApplyLaunch.row_obs.
int apply_nq_two_pass(bool obs);
size_t apply_lds_bytes(const DevBasis& db, int prec, int nv, int rows);
// Whether the one-pass kernel can stage a tile row of nv interleaved vectors
// (single vectors always have a path: two passes or rows read from memory).
bool apply_fits(const DevBasis& db, int prec, int nv);
int elem_grid(int64_t n);  // grid of the elementwise kernels (update, combine, norms)

// u_{j+1} = w - alpha_j s_j u_j in place; alpha_j from the apply's partials;
// |u_{j+1}|^2 partials [elem_grid][nv].
hipError_t launch_update(int prec, int nv, int64_t n, void* w, const void* uj, VecState* st, StepCtl* ctl, int j,
                         const double* apply_partials, int apply_nblk, int apply_nq, const double* row_obs,
                         int row_nblk, double* partials, hipStream_t s);

// One CGS pass of u_{j+1} (slot j+1) against v_k = s_k u_k, k <= j, with FP64
// coefficients: dot partials [elem_grid][j+1][2][nv] in dot_partials, the
// coefficients [j+1][nv] complex in coef, and |u_{j+1}|^2 partials
// [elem_grid][nv] for the next apply.  Idle after the step's decision.
hipError_t launch_reorth(int prec, int nv, int64_t n, void* const* slots_dev, int j, const VecState* st,
                         const StepCtl* ctl, double* dot_partials, double* coef, double* norm_partials,
                         hipStream_t s);
// Broadened spectral functions of n_members overlap series [n_members][n_s]
// (complex, device) on the frequencies nu [n_nu] (device) into out
// [n_members][n_nu] (device); lesser[m] (host) selects conj(o) for removal.
hipError_t launch_spectral(int n_members, int n_s, const void* overlaps, const int32_t* lesser, double dt, double eps,
                           int n_nu, const double* nu, double* out, hipStream_t s);
struct CombineLog {
  int32_t m, status;
  double eps, beta_last;
};

// v = beta0 sum_k y_k s_k u_k over the m_v vectors of each vector v (in place
// into slot 0), and |v|^2 partials [elem_grid][nv].  If some vector is still
// undecided the step is abandoned: ctl->abort is set and slot 0 is kept.
// Otherwise the first workgroup also records the step (as launch_step_log:
// log [nv] and, if obs_log, the first apply's observables [nv][nobs]) and
// clears the control block for the next step; seq >= 1 numbers the
// (sub)steps of a call, and after one where a vector hit m_max the later
// combines do nothing.
hipError_t launch_combine(int prec, int nv, int64_t n, void* const* slots_dev, const VecState* st,
                          StepCtl* ctl, double* partials, int seq, CombineLog* log, double* obs_log, int nobs,
                          hipStream_t s, void* copy_to = nullptr);  // copy_to: a second copy of the result (nv = 1)

// Overlaps o_v = <c_v psi_v | phi_v> of nv members (same target sector and
// spin of the operator) with source-sector states psi_v = traj + psi_off[v],
// gathered through the members' operator maps maps/sgns [nv][map_len] (tile
// rows for an up operator, columns for a down one).  phi: the members in the
// target sector, interleaved [n_t][nv] or in the ABI layout [nv][n_t].
// Partials [nv][overlap_grid(n_t)][2] (re, im); nothing after an abandoned step.
struct OverlapArgs {
  int64_t n_t;
  int dim_dn_t, dim_dn_s, down, map_len, interleaved;
  int64_t psi_off[kMaxNV];
  const int32_t* maps;
  const int8_t* sgns;
  const void* traj;
  const void* phi;
  const StepCtl* ctl;
  double* partials;
};
hipError_t launch_overlaps(int prec, int nv, const OverlapArgs& a, hipStream_t s);
// out[s * out_stride + q] = sum over r < rows of part[s * set_stride + r * cols + q], q < cols, s < n_sets.
hipError_t launch_reduce_sets(const double* part, int64_t set_stride, int n_sets, int rows, int cols, double* out,
                              int64_t out_stride, hipStream_t s);
int overlap_grid(int64_t n_t);
// x[i] = (sin(0.618 i), cos(0.377 i + 1)) for i < n (complex of precision prec): test vectors of the tuner.
hipError_t launch_fill_probe(int prec, int64_t n, void* x, hipStream_t s);

// |v|^2 partials of the step input (if norm), tau of every vector, cleared control block.
hipError_t launch_step_begin(int prec, int nv, int64_t n, const void* v, VecState* st, StepCtl* ctl, double tau,
                             bool norm, double* partials, hipStream_t s);

// Copies the finished step's Krylov report and first-apply observables.
hipError_t launch_step_log(int nv, const VecState* st, StepCtl* ctl, void* log, double* obs_log, int nobs,
                           hipStream_t s);

// One-workgroup reductions of partial sums.
hipError_t launch_finalize_obs(int nv, const double* partials, int nrows, int nq, VecState* st, hipStream_t s);
hipError_t launch_finalize(const double* partials, int nrows, int ncols, double* out, int op, hipStream_t s);

// Site-resolved double occupation sum_k n_{i up} n_{i down} |x_k|^2 of one vector.
hipError_t launch_site_docc(int prec, const DevBasis& db, const void* x, double* out, double* partials,
                            hipStream_t s);

// Layout changes between [v][k] (ABI) and [k][v] (interleaved block).
hipError_t launch_interleave(int prec, int nv, int64_t n, const void* src, void* dst, bool to_block,
                             hipStream_t s);

// Creation/annihilation operator between sectors: y_k = op x_k for nvec
// vectors (ABI layout).  map/sgn: per target row (up operator) or column
// (down operator): source index (-1: none) and sign.
hipError_t launch_cop(int prec, int64_t n_t, int dim_dn_t, int dim_dn_s, int64_t n_s, int nvec, bool down,
                      const int32_t* map, const int8_t* sgn, const void* x, void* y, hipStream_t s);

// out[2k], out[2k+1] = <x_k | y_k> for nvec pairs (device output, fixed order).
hipError_t launch_dots(int prec, int64_t n, int nvec, const void* x, const void* y, double* out, double* partials,
                       hipStream_t s);

// BLAS-1 helpers for the ground-state Lanczos (complex double, one vector).
hipError_t launch_multidot(int64_t n, const double2* const* vecs, int k, const double2* w, double2* out,
                           double* partials, hipStream_t s);
hipError_t launch_multiaxpy(int64_t n, const double2* const* vecs, int k, const double2* coef, double2* w,
                            hipStream_t s);
hipError_t launch_norm2(int64_t n, const double2* w, double* out, double* partials, hipStream_t s);
hipError_t launch_scale(int64_t n, double2* w, const double* inv_from, double2 factor, hipStream_t s);
hipError_t launch_absmax(int64_t n, const double2* w, double* out, double* partials, hipStream_t s);
hipError_t launch_first_above(int64_t n, const double2* w, const double* thresh, int64_t* out, int64_t* partials,
                              hipStream_t s);

}  // namespace hub
