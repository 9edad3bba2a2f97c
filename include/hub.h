/*
 * hub.h — C ABI of the MI355X exact-diagonalization time stepper for the
 * Peierls-driven Hubbard model (arXiv:2005.13498).
 *
 * The library evolves a state of one particle-number sector with the
 * exponential midpoint rule of Eq. (time-stepping),
 *     v(t + dt) = exp(-i dt H(t + dt/2)) v(t),
 * each exponential taken by the adaptive Lanczos/Krylov step of Alg. 6 with
 * the a-posteriori error estimate of Sec. 3.4.  H(t) is Eq. (hubbardhamiltonian)
 * with the Peierls phases of Eq. (peierls), applied matrix-free.
 *
 * Conventions shared by every call
 *  - Geometry (Sec. 2.1): undirected bonds (i, j) with amplitude t_ij > 0 and
 *    displacement dx_ij = (R_i - R_j) projected on the field.  Each bond adds
 *        -t_ij e^{+i A dx_ij} c^dag_{i s} c_{j s} - t_ij e^{-i A dx_ij} c^dag_{j s} c_{i s}
 *    for both spins s.  On a periodic wrap bond dx is the minimum image.
 *    Optional on-site energies eps_i add eps_i (n_{i up} + n_{i down})
 *    (eps_i = -v_ii in the paper's notation).
 *  - Basis and layout: a sector state is the pair (a, b) of an up string and
 *    a down string (bit i = site i); a (b) is the rank of the up (down)
 *    string among all strings with n_up (n_dn) bits in increasing integer
 *    order, which equals the combinatorial rank of Eq. (hashing).  The
 *    operator order is spin-separated: all up creators (site 0 leftmost),
 *    then all down creators.  (The paper's interleaved order of Eq. (statedef)
 *    differs from this by a sign per basis state only.)  A vector is
 *    psi[a * dim_dn + b], complex interleaved (re, im): double pairs for
 *    HUB_C128, float pairs for HUB_C64.  nvec vectors are stored one after the
 *    other: psi[v * dim + a * dim_dn + b].
 *  - Memory: every vector argument is a caller-owned DEVICE pointer on the
 *    handle's device; every struct or scalar array argument is a HOST pointer.
 *    Input and output vectors must not alias unless stated.
 *  - Streams: `stream` is a hipStream_t (NULL = default stream).  Calls that
 *    only write device memory are asynchronous; calls that fill host structs
 *    synchronise `stream` before returning.
 *  - Errors: every call returns a hub_status and never aborts; arguments are
 *    validated before any launch.  hub_last_error() gives a message for the
 *    last non-OK status on the calling thread.  A handle may not be used by
 *    two threads at once.
 */
#ifndef HUB_H
#define HUB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HUB_OK = 0,
  HUB_E_INVALID = -1,       /* bad argument (null, out of range, aliasing)      */
  HUB_E_SECTOR = -2,        /* particle numbers impossible for the lattice     */
  HUB_E_NOMEM = -3,         /* device allocation failed                        */
  HUB_E_DEVICE = -4,        /* HIP runtime error                               */
  HUB_E_NOT_CONVERGED = -5, /* Krylov step hit m_max before the tolerance      */
  HUB_E_DEGENERATE = -6     /* ground state not separated from the next level  */
} hub_status;

typedef enum { HUB_C128 = 0, HUB_C64 = 1 } hub_prec;

/* Geometry = the paper's hopping matrix v (Sec. 2.1, Fig. 1). Host arrays. */
typedef struct {
  int32_t n_sites;          /* 1 .. 16                                          */
  int32_t n_bonds;          /* >= 0                                             */
  const int32_t *bond_i;    /* [n_bonds], 0 <= i < n_sites                      */
  const int32_t *bond_j;    /* [n_bonds], j != i, no bond listed twice          */
  const double *bond_t;     /* [n_bonds], hopping amplitude t_ij                */
  const double *bond_dx;    /* [n_bonds], (R_i - R_j) along the field           */
  const double *onsite;     /* [n_sites] eps_i, or NULL                         */
  double U;                 /* on-site interaction                              */
} hub_lattice;

/* Pulse (Sec. 2.2).  kind 0: A(t) = A0 exp(-(t-t0)^2/(2 sigma^2)) sin(omega (t-t0)),
 * a Gaussian-windowed sine (the shape of Eq. (efield)) used as the vector
 * potential.  kind 1: the phase of Eq. (vt), A(t) = a [cos(omega (t-t_p)) - b]
 * exp(-(t-t_p)^2/(2 sigma^2)) with a = A0, t_p = t0, so bonds with dx = 1 carry f(t). */
typedef struct {
  int32_t kind;
  double A0, omega, t0, sigma, b;
} hub_pulse;

/* Krylov options (Alg. 6).  tol: stop when the a-posteriori estimate eps < tol
 * or the new off-diagonal element beta_j < |H|_inf * tol.  m_max: N_max of
 * Alg. 6 (1..60).  reorth: 0 = three-term recurrence only (as printed),
 * 1 = full reorthogonalisation (classical Gram-Schmidt, twice) against all
 * previous Krylov vectors with FP64 coefficients.  substeps: the step's
 * exponential exp(-i dt H(t_mid)) is split into this many equal factors of
 * the same H(t_mid) (>= 1).  m_hint: Lanczos iterations enqueued before the
 * first convergence check (0 = the library's own choice). */
typedef struct {
  double tol;
  int32_t m_max;
  int32_t reorth;
  int32_t substeps;
  int32_t m_hint;
  int32_t scheme;  /* hub_propagate only: 0 = exponential midpoint rule (Eq. (time-stepping));
                      1 = fourth-order commutator-free exponential: per step
                      exp(-i dt (a1 H1 + a2 H2)) exp(-i dt (a2 H1 + a1 H2)), H_k = H(t + c_k dt),
                      c = 1/2 -+ sqrt(3)/6, a = (3 -+ 2 sqrt(3))/12, each factor a Krylov
                      step of length dt/2 (and split into `substeps`) */
} hub_krylov_opts;

/* Per step (per vector) report. err_est = last a-posteriori estimate eps. */
typedef struct {
  int32_t m_used, substeps, converged, breakdown;
  double err_est, beta_last;
} hub_step_info;

/* Observables at one sample time (Eqs. (docc), (energy), Sec. 3.5), per vector:
 * norm |psi|, <psi|H(t)|psi>/n_sites, <psi|sum_i d_i|psi>/n_sites.  For a
 * vector that is not normalised the expectation values are NOT divided by
 * the norm. */
typedef struct {
  double t, norm, energy_per_site, docc_per_site;
} hub_obs;

typedef struct hub_basis_s *hub_basis;

/* ------------------------------------------------------------------------ */
/* Sector basis and hop tables (Sec. 3.1 "Discrete basis", Sec. 3.2 linear-
 * complexity structure via the ranking of Eq. (hashing)).  Builds, on the
 * host, the increasing list of up and down strings, and for every string the
 * list of one-electron hops along the bonds (target rank, fermionic sign of
 * Eq. (sign-explanation), amplitude class), then copies them to `device`.
 * device = -1 builds a host-only handle: tables can be inspected
 * (hub_basis_info/states/hops/classes) but every compute call returns
 * HUB_E_DEVICE.  Errors: HUB_E_INVALID (bad geometry, more than 8 distinct
 * (t, dx) hop classes), HUB_E_SECTOR (n_up or n_dn outside 0..n_sites),
 * HUB_E_NOMEM, HUB_E_DEVICE.  On error *out is NULL. */
hub_status hub_basis_create(const hub_lattice *lattice, int32_t n_up, int32_t n_dn,
                            int32_t device, hub_basis *out);

/* Frees the handle, its tables and its workspace.  NULL is ignored.
 * Synchronises the handle's device first. */
void hub_basis_destroy(hub_basis basis);

/* Sector dimension C(Ns,n_up) C(Ns,n_dn) (Eq. (statedim)) and its factors. */
hub_status hub_basis_info(hub_basis basis, int64_t *dim, int32_t *dim_up, int32_t *dim_dn);

/* Host copies of the up strings [dim_up] and down strings [dim_dn] (bit i =
 * site i), in rank order.  Either pointer may be NULL. */
hub_status hub_basis_states(hub_basis basis, uint32_t *up_bits, uint32_t *dn_bits);

/* Hop classes: class c contributes -t[c] exp(i A d[c]) per hop (d = R_dst -
 * R_src along the field).  t, d: host arrays of length >= 8 or NULL;
 * n_classes receives the count.  norm_inf (nullable) receives |H|_inf, the
 * largest absolute row sum of H, which the Peierls phases leave unchanged. */
hub_status hub_basis_classes(hub_basis basis, double *t, double *d, int32_t *n_classes,
                             double *norm_inf);

/* Gather-form hop table of one spin (0 = up, 1 = down): for target rank r
 * the hops are entries ptr[r] .. ptr[r+1]-1 with source rank src[k], sign
 * sgn[k] in {+1, -1} (Eq. (sign-explanation)) and class cls[k], so that the
 * one-spin hopping matrix is T[r][src] += sgn * coef_cls.  Call with NULL
 * arrays to get *n_hops first; ptr has dim_spin + 1 entries. */
hub_status hub_basis_hops(hub_basis basis, int32_t spin, int32_t *ptr, int32_t *src, int32_t *sgn,
                          int32_t *cls, int64_t *n_hops);

/* ------------------------------------------------------------------------ */
/* y = H(A_v) x_v for nvec vectors (Eq. (hubbardhamiltonian) with the Peierls
 * phases of Eq. (peierls) at vector potential A_v; matrix-free).  A: host
 * array [nvec].  x, y: device, nvec * dim complex of precision `prec`,
 * distinct buffers.  Asynchronous on `stream`. */
hub_status hub_apply_H(hub_basis basis, const double *A, hub_prec prec, int32_t nvec,
                       const void *x, void *y, void *stream);

/* Observables of Sec. 3.5 at vector potential A_v (host [nvec]) for the nvec
 * device vectors v.  out: host [nvec] (out[k].t is set to 0).  site_docc:
 * host [nvec * n_sites] <n_{i up} n_{i down}> per site, or NULL.
 * Synchronises `stream`. */
hub_status hub_observables(hub_basis basis, const double *A, hub_prec prec, int32_t nvec,
                           const void *v, hub_obs *out, double *site_docc, void *stream);

/* hub_observables without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as hub_observables
 * (bit for bit).  Its intermediate sums live in one static device array of
 * 512 KiB per device (allocated with the library's code object, looked up when
 * the first handle is created on that device, held until the process ends),
 * enough for every sector of up to 14 sites; a sector that needs more (16
 * sites) is rejected with HUB_E_INVALID before any launch.  Every buffer in it
 * is fully written before it is read, so nothing is cleared between calls.
 * All calls on one device share the array: calls that overlap in time on one
 * device (other host threads, or other streams still running one) race and
 * must be serialised by the caller.  Synchronises `stream`. */
hub_status hub_observables_noalloc(hub_basis basis, const double *A, hub_prec prec, int32_t nvec,
                                   const void *v, hub_obs *out, double *site_docc, void *stream);

/* One Krylov step (Alg. 6): v_k <- exp(-i dt H(A_mid_k)) v_k for nvec device
 * vectors (in place).  A_mid: host [nvec].  info: host [nvec] or NULL.
 * Returns HUB_E_NOT_CONVERGED if any vector hit m_max (its result is then
 * the m_max approximation, info.converged = 0), HUB_E_INVALID if a vector or
 * its recurrence is not finite (NaN or Inf).  Synchronises `stream`. */
hub_status hub_krylov_expm_step(hub_basis basis, const double *A_mid, double dt,
                                const hub_krylov_opts *opts, hub_prec prec, int32_t nvec,
                                void *v_inout, hub_step_info *info, void *stream);

/* n_steps midpoint steps (Eq. (time-stepping)) from t_start: step n uses
 * H(A_k(t_start + n dt + dt/2)) for vector k with pulse pulses[k] (host
 * [nvec]).  v_inout: device, nvec vectors, in place.  obs: host
 * [(n_steps + 1) * nvec] or NULL: observables at t_start + n dt (row n,
 * column k), with H(t) evaluated at the sample time.  log: host
 * [n_steps * nvec] or NULL.  Returns HUB_E_INVALID (and stops) at the first
 * step where a vector or its Krylov recurrence is not finite (NaN or Inf in
 * the input or produced on the way), and HUB_E_NOT_CONVERGED (and stops) at the
 * first step where a vector hits m_max; v_inout then holds that step's
 * m_max approximation, the obs row after that step holds its observables and
 * later rows are NaN.  The schedule (hub_set_schedule,
 * hub_controller_enable) changes how the launches overlap the host, never the
 * result.  In small sectors the whole call is one launch of the resident
 * stepper (hub_set_propagate_path), each vector stopping at its own first
 * m_max or non-finite step.  Otherwise the library propagates the vectors in
 * groups (interleaved blocks, or single vectors where the two-pass kernels
 * apply); several groups run concurrently on up to 4 lanes, each with its
 * own workspace, stream and host
 * thread, started after the work already on `stream` (not while apply timing
 * or the learned controller is enabled, and not beyond 48 GiB of Krylov
 * workspace).  Results do not depend on this; with concurrent groups each
 * group stops at its own first m_max step.  Synchronises `stream`. */
hub_status hub_propagate(hub_basis basis, const hub_pulse *pulses, double t_start, double dt,
                         int32_t n_steps, const hub_krylov_opts *opts, hub_prec prec,
                         int32_t nvec, void *v_inout, hub_obs *obs, hub_step_info *log,
                         void *stream);

/* Path of hub_propagate (and hub_krylov_expm_step) on this handle.  path 0:
 * launches per Lanczos iteration (the kernels above, groups, lanes and the
 * schedules of hub_set_schedule / hub_controller_enable).  path 1: the
 * resident stepper, one launch for the whole call and one workgroup per
 * vector that keeps the vector's tile (with a zero row and column) and the
 * sector's hop tables in LDS and runs every step: the Lanczos recurrence of
 * Alg. 6 with its a-posteriori estimate and the same stopping rules, the
 * combine, and the observables of each step's input at its sample time; only
 * the Krylov vectors u_1 .. u_{m-1} of a step go to device memory.  It takes
 * sectors of at most 8,192 states (c128) or 16,384 (c64) whose tile and
 * tables fit a workgroup's LDS (8 sites at half filling: 4,900 states),
 * opts.reorth = 0 (either scheme, any substeps: the step's Krylov solves run
 * one after another in the workgroup), and neither apply timing
 * (hub_profile_enable) nor the learned controller; else hub_propagate
 * returns HUB_E_INVALID.  Each vector stops at its own first step that hits
 * m_max or turns non-finite (its later observables are NaN), as concurrent
 * groups do on the launch path.  path -1 (default): 1 where it applies, the
 * apply kernels are automatic (hub_set_apply_path -1) and nvec * 6144 is at
 * least the sector's dimension (one workgroup per
 * vector runs at one compute unit's LDS rate: a single large vector is
 * better spread over the GPU), else 0.  Both paths give the same results up
 * to rounding.  Errors: HUB_E_INVALID. */
hub_status hub_set_propagate_path(hub_basis basis, int32_t path);

/* Ground state of H(A) (Sec. 3.4 "Ground state"): restarted Lanczos with
 * full reorthogonalisation in FP64 until the residual |H x - E0 x| falls
 * below opts->tol * |H|_inf (opts NULL: tol 1e-12, m_max 60).  v_out:
 * device, dim complex doubles, normalised, phase fixed so that the component
 * of largest modulus is real positive (lowest index among ties within 1e-12).
 * E0, gap (E1 - E0 of the Ritz values): host, gap may be NULL.  Returns
 * HUB_E_DEGENERATE when gap < 1e-8 * |H|_inf (v_out and E0 still written).
 * Synchronises `stream`. */
hub_status hub_ground_state(hub_basis basis, double A, const hub_krylov_opts *opts,
                            void *v_out, double *E0, double *gap, void *stream);

/* Creation (dagger = 1) or annihilation (dagger = 0) operator c_{site,spin}
 * (spin 0 = up, 1 = down) from the sector of `from` to the sector of `to`
 * (Eq. (creation-annihilation)): y_k = c x_k for nvec vectors (device, ABI
 * layout; x in from's sector, y in to's).  Signs follow the spin-separated
 * operator order of the basis (an up operator passes the up creators of lower
 * sites; a down operator also passes all up creators).  Errors: HUB_E_SECTOR
 * when `to` is not the operator's target sector, HUB_E_INVALID.  Synchronises
 * `stream`. */
hub_status hub_apply_cop(hub_basis from, hub_basis to, int32_t site, int32_t spin, int32_t dagger,
                         hub_prec prec, int32_t nvec, const void *x, void *y, void *stream);

/* out[2k] + i out[2k+1] = <x_k | y_k> (conjugate on x) for nvec pairs of
 * device vectors of the basis's sector.  out: host [2 * nvec].  Fixed-order
 * (reproducible) reduction.  Synchronises `stream`. */
hub_status hub_dot(hub_basis basis, hub_prec prec, int32_t nvec, const void *x, const void *y, double *out,
                   void *stream);

/* Diagonal two-time Green's functions (Eq. (Glg), Sec. 3.7).  Member k applies
 * op_k = c (dagger 0) or c^dag (dagger 1) on (site, spin) to psi(t'_k),
 * t'_k = t_start + start_step * dt, propagates the result in op_k's sector with
 * the midpoint Krylov stepper on the same time grid as psi, and records
 *     o_k(s) = < op_k psi(t'_k + s dt) | phi_k(t'_k + s dt) >,  s = 0..n_rel,
 * so that G^<(t', t'+s) = i o(s) for c and G^>(t'+s, t') = -i o(s) for c^dag.
 * targets: host array of n_targets basis handles covering the members'
 * sectors (matched by particle numbers).  psi is propagated first over the
 * whole grid, its state after every step kept on the device; the members then
 * run on one of two steppers (hub_set_greens_path): per sector, members
 * sharing a sector are propagated together as the vectors of hub_propagate
 * (the sectors side by side, own streams and host threads, after the work on
 * `stream`, so the handles must be distinct and not in use elsewhere during
 * the call); or the persistent member stepper, one launch in which every
 * member runs all its steps in a workgroup of its own.  psi_inout: device
 * vector of `basis` in precision `prec`, advanced in place to t_start + (max
 * start_step + n_rel) dt.  overlaps: host [n_members][n_rel + 1][2].
 * HUB_E_NOT_CONVERGED when a member's step hits m_max, HUB_E_INVALID when a
 * member's vector becomes non-finite (on the persistent stepper that member's
 * later overlaps are NaN).  Synchronises `stream`. */
typedef struct {
  int32_t site, spin, dagger, start_step;
} hub_greens_member;

hub_status hub_greens_diag(hub_basis basis, int32_t n_targets, const hub_basis *targets,
                           const hub_pulse *pulse, double t_start, double dt, int32_t n_rel,
                           const hub_krylov_opts *opts, hub_prec prec, int32_t n_members,
                           const hub_greens_member *members, void *psi_inout, double *overlaps,
                           void *stream);

/* Stepper of hub_greens_diag's members (set on the source basis, not in the
 * paper: how the library schedules the same steps).  path 0: per target
 * sector, the members as a batch of hub_propagate vectors (one launch per
 * Lanczos pass); path 1: the persistent member stepper, one launch for all
 * members, each member a workgroup that runs its Lanczos iterations
 * (three-term recurrence, Alg. 6's estimate), its combines and its overlaps
 * for every step, with the sector's hop tables and the member's operator map
 * in LDS beside staged tile rows and tile columns; it needs opts.reorth = 0,
 * opts.substeps = 1 and target sectors with at most 32 grouped hop slots per
 * string whose tables plus one tile row (and one tile column) fit 148 KiB,
 * else hub_greens_diag returns HUB_E_INVALID.  path -1 (default): 1 where it
 * applies, every target sector has at most 2^18 states and there are at
 * least as many members as compute units (one workgroup per member runs well
 * below a compute unit's share of the bandwidth), else 0.  Both give the same
 * overlaps up to rounding.  Errors: HUB_E_INVALID. */
hub_status hub_set_greens_path(hub_basis basis, int32_t path);

/* Broadened spectral functions, Eq. (A_noneq_broad), from the overlaps of
 * hub_greens_diag on the stepper grid s_k = k dt, k < n_s:
 *     A(nu) = (1/pi) Re sum_k w_k e^{-eps s_k} e^{i nu s_k} z_k,
 * w_k the trapezoidal weights of [0, (n_s - 1) dt], z = conj(o) for a removal
 * member (lesser[m] = 1, o from c: A<(nu, t'), the lesser function G<(t'+s,
 * t') = -conj G<(t', t'+s) transformed) and z = o for an addition member
 * (lesser[m] = 0, o from c^dag: A>(nu, t')).  In equilibrium this is the
 * Lorentzian Lehmann form of Eq. (spectralplot) divided by pi, removal peaks
 * at E0 - E_phi and addition peaks at E_phi - E0.  overlaps [n_members][n_s]
 * complex (double pairs), nu [n_nu] and out [n_members][n_nu] are device
 * pointers on `device`; lesser [n_members] is a host array.  Asynchronous. */
hub_status hub_spectral(int32_t device, int32_t n_members, int32_t n_s, const double *overlaps,
                        const int32_t *lesser, double dt, double eps, int32_t n_nu, const double *nu,
                        double *out, void *stream);

/* Value of the pulse's A(t) (host arithmetic, as used by hub_propagate). */
hub_status hub_pulse_A(const hub_pulse *pulse, double t, double *A);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *hub_last_error(void);

/* ------------------------------------------------------------------------ */
/* Learned Krylov controller.  Not in the paper: a schedule optimisation on
 * top of Alg. 6 that never changes results.  A small FP32 MLP
 *     x (8) -> 64 -> GELU -> 64 -> GELU -> 1,   GELU(z) = z (1 + erf(z/sqrt2)) / 2
 * predicts, for each step of a chunk of upcoming midpoint steps, o[0] =
 * log2 of the Krylov dimension m the adaptive step will use.  (Splitting a
 * step into substeps would change the results, not only the schedule, and
 * at the steps these workloads take, tau |H|_inf ~ 1/2, one Krylov solve is
 * always cheaper, so the network predicts no substep count.)  Features of the row
 * for step n, whose history ends at step h <= n - 1 (the last step finished
 * when the chunk was planned):
 *     x[0] = A(t_mid_n)            x[1] = A'(t_mid_n) / 10
 *     x[2] = tau |H|_inf           (tau = the length of one Krylov solve: dt / substeps,
 *                                   halved for scheme 1; |H|_inf as in Alg. 6)
 *     x[3..6] = log10(eps_{h-k}) / 10, k = 0..3   (a-posteriori estimate of
 *               step h-k, floored at 1e-40; log10(tol)/10 before step 0)
 *     x[7] = m_h / 10              (m_hint / 10, or 0.8, before step 0)
 * Parameters (HUB_MLP_NPARAM floats, row-major, output unit first):
 *     W1[64][8], b1[64], W2[64][64], b2[64], W3[1][64], b3[1].
 * When enabled on a handle, hub_propagate plans `chunk` steps at a time: one
 * MLP launch predicts m for each, each step gets ceil(2^o[0]) + margin + 1
 * Lanczos launches (capped by m_max + 1) without host synchronisation, and
 * the adaptive test of Alg. 6 still decides every step on the device.  A
 * step that is not decided within its launches is abandoned unchanged (the
 * rest of the chunk does nothing) and re-run with the adaptive schedule.
 * Results are therefore bit-identical to the adaptive schedule. */
#define HUB_MLP_IN 8
#define HUB_MLP_HID 64
#define HUB_MLP_OUT 1
#define HUB_MLP_NPARAM (HUB_MLP_HID * HUB_MLP_IN + HUB_MLP_HID + HUB_MLP_HID * HUB_MLP_HID + HUB_MLP_HID + \
                        HUB_MLP_OUT * HUB_MLP_HID + HUB_MLP_OUT)

/* out[r][0] = MLP(feats[r][8]) for r < n_rows.  params, feats, out: device
 * pointers on `device`.  Asynchronous on stream. */
hub_status hub_mlp_forward(int32_t device, const float *params, int32_t n_rows, const float *feats,
                           float *out, void *stream);

/* Device workspace bytes hub_mlp_train_step needs for n_rows rows. */
int64_t hub_mlp_workspace_bytes(int32_t n_rows);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with step
 * count t >= 1, learning rate lr) on the mean squared error
 *     L = (1/n_rows) sum_r sum_o (out[r][o] - targets[r][o])^2.
 * params, adam_m, adam_v (HUB_MLP_NPARAM floats each, updated in place),
 * feats [n_rows][8], targets [n_rows][1], loss (1 float: L before the
 * update) and workspace (hub_mlp_workspace_bytes) are device pointers.
 * Gradient partial sums are reduced in a fixed order (deterministic).
 * Asynchronous on stream. */
hub_status hub_mlp_train_step(int32_t device, float *params, float *adam_m, float *adam_v, int32_t t,
                              float lr, int32_t n_rows, const float *feats, const float *targets,
                              float *loss, void *workspace, void *stream);

/* Training rows from a finished run of one vector (host arrays): for each
 * step n in [0, n_steps), feats[n] as above with history end
 * h = n - 1 - (n mod chunk) (the planning point of n's chunk when chunks
 * start at multiples of `chunk`), and targets[n] = log2 m_n.  log is
 * that vector's hub_step_info of the run (n_steps entries, stride 1). */
hub_status hub_controller_features(const hub_pulse *pulse, double t_start, double dt, int32_t n_steps,
                                   double norm_inf, const hub_krylov_opts *opts, const hub_step_info *log,
                                   int32_t chunk, float *feats, float *targets);

/* Copy HUB_MLP_NPARAM host floats into the handle's controller. */
hub_status hub_controller_load(hub_basis basis, const float *params, int32_t n_params);

/* Enable (on = 1, after a load) or disable the controlled schedule of
 * hub_propagate; chunk in [1, 256] steps, margin in [0, 16] iterations. */
hub_status hub_controller_enable(hub_basis basis, int32_t on, int32_t chunk, int32_t margin);

typedef struct {
  int64_t steps;          /* steps finished under the controlled schedule     */
  int64_t chunks;         /* chunks planned (one MLP launch, one sync each)   */
  int64_t fallbacks;      /* steps re-run with the adaptive schedule          */
  int64_t lanczos_launches; /* H*v launches enqueued by controlled chunks     */
  int64_t iterations;     /* Krylov iterations those steps needed (sum of m over steps and vectors) */
} hub_controller_stats;

/* Counters since the last read (then reset).  They count the chunks of the
 * default schedule (hub_set_schedule) as well as the learned controller's. */
hub_status hub_controller_read_stats(hub_basis basis, hub_controller_stats *out);

/* Schedule of hub_propagate when the learned controller is off.
 *   chunk >= 1 (default 32, margin 1): chunks of `chunk` steps are enqueued
 *     without waiting for the host; every step of a chunk runs
 *     min(m_max, m_ref + margin) + 1 Lanczos launches, m_ref being the largest
 *     Krylov dimension of the previous chunk's steps (the first chunk:
 *     m_hint; without a hint the call's first step runs synchronously and its
 *     dimension is used).  A step that has not decided within its launches stops
 *     the chunk on the device and is re-run with the synchronous schedule.
 *   chunk = 0: synchronous schedule, one host round trip per (sub)step plus
 *     one per iteration beyond the previous step's m.
 * Both give bit-identical states, observables and logs (the decisions are
 * taken on the device either way); only the host/device overlap differs.
 * chunk in [0, 256], margin in [0, 16]; HUB_E_INVALID otherwise.  Runs of a
 * single step use the synchronous schedule. */
hub_status hub_set_schedule(hub_basis basis, int32_t chunk, int32_t margin);

/* ------------------------------------------------------------------------ */
/* Choice of the H*v kernels for single vectors (plain applies and the
 * Lanczos iterations that do not also accumulate observables) and for
 * interleaved blocks of vectors.
 *   path 0: one pass (rows staged in LDS; up hops gathered as whole rows of
 *           x from global memory), for single vectors and blocks alike;
 *   path 1: two passes whenever 4 (else 2) columns of x for all up
 *           strings fit in LDS (a row pass for the diagonal and the down
 *           hops, then a column pass that stages those columns, as +x and
 *           -x or, when two copies do not fit, as +x with the sign taken
 *           from the hop's index, and adds the up hops);
 *   path -1 (default): two passes when they fit and the vector is larger
 *           than 4 MiB, one pass otherwise.
 * Blocks of 2, 4 or 8 vectors (paths 1 and -1) run the two-pass block
 * kernels where a tile row and a tile column of the whole block fit LDS: a
 * row pass (diagonal and down hops) and a column pass (up hops, Lanczos
 * epilogue), each staging its row or column of all vectors once.
 * Plain applies give bit-identical results on both paths; in Lanczos mode
 * the alpha_j reduction is summed in another order (deterministic either
 * way). */
hub_status hub_set_apply_path(hub_basis basis, int32_t path);

/* ------------------------------------------------------------------------ */
/* Kernel plan of a basis (not in the paper: which kernels the library runs).
 * Per precision, the library chooses (a) the H*v kernels of single vectors,
 * one pass or two passes (hub_set_apply_path); (b) for interleaved blocks
 * of 2, 4 or 8 vectors, the two-pass block kernels or the one-pass kernel;
 * (c) the vectors per group when a call carries many vectors, separately for
 * hub_apply_H and hub_propagate.  Without tuning these follow built-in rules
 * (LDS fit and vector size); hub_tune measures them on this basis's sector:
 * plain H*v of 8 vectors in groups of 1, 2, 4, 8 on each feasible path
 * (`reps` timed calls each, HIP events), then two midpoint steps (after one
 * untimed) per group size on the chosen paths (dt |H|_inf = 1/2, tol 1e-10,
 * host clock), of 8 vectors and of 32, and installs the fastest choices in
 * the handle.  Groups run on up to 4 concurrent lanes, so the best group
 * size depends on how many groups a call has: 8 vectors in groups of 8 run
 * on one lane, 32 fill every lane at every group size.  A hub_propagate call
 * of at most 8 vectors takes prop_group, a larger one prop_group_large.
 * The 32-vector measurement skips a group size whose vectors and Krylov
 * workspace would not fit the device's free memory (step_us_large 0 there;
 * prop_group_large = prop_group when none fits).  Results never
 * depend on the plan (only how the work is split into kernels).  hub_tune
 * allocates its test vectors; hub_set_tuning installs a table from an
 * earlier hub_tune (e.g. cached per sector shape and device), or the
 * built-in rules again with t = NULL.  hub_apply_path 0 still forces the
 * one-pass kernels. */
typedef struct {
  int32_t single_two_pass;    /* single vectors: 1 = two-pass kernels, 0 = one pass       */
  int32_t block_two_pass[4];  /* [1], [2], [3]: groups of 2, 4, 8 on the two-pass block
                                 kernels (1) or the one-pass kernel (0); [0] unused         */
  int32_t apply_group;        /* vectors per group of hub_apply_H (1, 2, 4, 8)             */
  int32_t prop_group;         /* vectors per group of hub_propagate (1, 2, 4, 8)           */
  double apply_us[4][2];      /* measured H*v time per vector (us), groups of 1, 2, 4, 8 x
                                 (one pass, two passes); 0 = infeasible                     */
  double step_us[4];          /* measured midpoint step time per vector (us) per group size;
                                 0 = infeasible                                             */
  int32_t prop_group_large;   /* vectors per group of hub_propagate calls of more than 8
                                 vectors (1, 2, 4, 8)                                       */
  double step_us_large[4];    /* step_us measured with 32 vectors; 0 = infeasible or skipped */
} hub_tuning;

hub_status hub_tune(hub_basis basis, hub_prec prec, int32_t reps, hub_tuning *out, void *stream);
hub_status hub_set_tuning(hub_basis basis, hub_prec prec, const hub_tuning *t);

/* The plan for nvec vectors (propagate = 1: hub_propagate, 0: hub_apply_H):
 * n_groups, and per group (host arrays of >= nvec entries, either may be
 * NULL) its size and kernels: 0 one pass, 1 two-pass single vector, 2
 * two-pass block kernels. */
hub_status hub_get_plan(hub_basis basis, hub_prec prec, int32_t nvec, int32_t propagate, int32_t *n_groups,
                        int32_t *sizes, int32_t *kernels);

/* ------------------------------------------------------------------------ */
/* Kernel timing of the matrix-free apply (for roofline reporting).  on = 0
 * disables it; on = k >= 1 attaches HIP start/end events to the kernel
 * dispatches of every k-th eligible H*v: hub_apply_H launches and Lanczos
 * H*v launches of a propagation except the first of each step, which also
 * records observables (a different kernel).  When a propagation runs the
 * two-pass kernels without re-orthogonalisation, iterations j >= 1 fuse the
 * Lanczos update into the row pass, and only those fused iterations are
 * timed.  A two-pass apply is timed as the sum of its two kernels.
 * Launches enqueued past a step's Krylov decision (speculative iterations,
 * which exit at once) are left out once the step's m is known, and so is a
 * step's last fused iteration (j = m), whose column pass skips the apply
 * when the row pass has already found the error estimate below tol.  The events
 * come from a pool of 8192 created here (on >= 1); a propagation reads them
 * back and reuses them only when fewer than 512 are left, so a run of up to
 * about 2000 timed launches adds neither event creation nor read-back to it. 
 * hub_profile_read returns the number of timed launches, their summed kernel
 * time in ms, and the algorithmic bytes of one timed launch (H*v: 2 * nvec *
 * dim * complex size, read x once and write y once; fused iteration: 4 *
 * nvec * dim * complex size, read w_{j-1} and u_{j-1}, write u_j and y), then
 * resets the counters.  Synchronises the device. */
hub_status hub_profile_enable(hub_basis basis, int32_t on);
hub_status hub_profile_read(hub_basis basis, int64_t *launches, double *total_ms,
                            double *bytes_per_launch);

#ifdef __cplusplus
}
#endif
#endif /* HUB_H */
