// Resident stepper of small sectors (resident.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace hub {

// Threads of a resident workgroup, and the most tile elements one thread
// owns per precision (c128, c64): the largest sector the stepper takes has
// kResidentThreads * kResidentEpt[prec] states.
constexpr int kResidentThreads = 1024;
constexpr int kResidentEpt[2] = {8, 16};

// One launch propagates nvec vectors of one sector for all their steps (Eq.
// (time-stepping), or the fourth-order scheme's two exponentials, each split
// into equal substeps), one workgroup per vector.  Device pointers unless
// noted.
struct ResidentArgs {
  int dim_up, dim_dn, gs_up, gs_dn, nc;
  uint8_t up_gclass[8], dn_gclass[8];  // class of each group of four slots
  const uint32_t* up_bits;
  const uint32_t* dn_bits;
  const double* eps_up;  // null without on-site energies
  const double* eps_dn;
  const uint16_t* up_tab;  // grouped tables [dim_up][gs_up], [dim_dn][gs_dn]
  const uint16_t* dn_tab;
  double U, norm_inf, tol, tau;  // tau: the length of one Krylov solve, dt / (n_exp substeps)
  int m_max, n_steps, nvec;
  int n_exp;     // exponentials per step (1: midpoint rule, 2: the fourth-order commutator-free scheme)
  int substeps;  // equal Krylov solves per exponential
  const double* coef_mid;  // [nvec][n_steps][n_exp][2 nc]: class coefficients of each exponential of each step
  const double* coef_obs;  // [nvec][n_steps + 1][2 nc] at the sample times, or null (no observables)
  void* v;                 // [nvec][dim] states, advanced in place
  void* slots;             // [nvec][m_max][dim] Krylov vectors u_1 .. u_{m_max - 1}
  CombineLog* log;         // [n_steps][nvec]
  double* obs;             // [n_steps + 1][nvec][kObsQ]: <D>, docc, |x|^2, Re <x|K(t)|x>
  int32_t* done;           // [nvec] steps whose results are in (a vector stops at m_max or non-finite)
};

// LDS bytes of a resident workgroup: the tables, strings and on-site energies
// (16-byte aligned pieces in the kernel's order), then the tile with a zero
// column and a zero row, (dim_up + 1) (dim_dn + 1) elements.
inline size_t resident_lds_bytes(int dim_up, int dim_dn, int gs_up, int gs_dn, bool eps, int prec) {
  auto a16 = [](size_t b) { return (b + 15) & ~size_t(15); };
  size_t t = a16(size_t(dim_dn) * (gs_dn / 4) * 8) + a16(size_t(dim_up) * (gs_up / 4) * 8) + a16(size_t(dim_up) * 4) +
             a16(size_t(dim_dn) * 4);
  if (eps) t += a16(size_t(dim_up) * 8) + a16(size_t(dim_dn) * 8);
  return t + size_t(dim_up + 1) * (dim_dn + 1) * (prec == 0 ? 16 : 8);
}

// Dynamic LDS the resident kernel of `prec` may use on this device (0 if none).
int resident_lds_limit(int prec);

// Launches nvec workgroups; returns hipErrorInvalidValue when the sector does
// not fit (dimension or LDS).
hipError_t launch_resident(int prec, const ResidentArgs& a, size_t lds, hipStream_t s);

}  // namespace hub
