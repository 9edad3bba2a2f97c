// Persistent member stepper of the Green's-function runs (members.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace hub {

// Hop tables of one target sector (device pointers of its basis): the
// grouped tables (class ranges of whole groups of four slots) and the class
// of every group.
struct MemberSector {
  int dim_up, dim_dn, gs_up, gs_dn;  // grouped slots per up / down string (multiples of 4, <= 32)
  const uint32_t* up_bits;
  const uint32_t* dn_bits;
  const double* eps_up;  // null without on-site energies
  const double* eps_dn;
  const uint16_t* up_tab;  // [dim_up][gs_up]
  const uint16_t* dn_tab;  // [dim_dn][gs_dn]
  uint8_t up_gclass[8], dn_gclass[8];
  double U, norm_inf;
  int nc;                  // hop classes
  const double* coef_tab;  // [n_total][2 nc]: coefficient of every class at each global step's midpoint
  int row_block, col_block;  // tile rows / tile columns staged in LDS at a time
  int tab_lds;               // LDS bytes of the tables before the staging area (members_table_lds)
};

// One member: its sector, first global step, Krylov slots ((m_max + 1)
// vectors of the sector's dimension; slot 0 holds the member's state on entry
// and exit), one scratch vector, its operator map into the source sector and
// its outputs.
struct MemberDesc {
  int sector, start;
  void* slots;
  void* z;
  const int32_t* map;  // [dim of the operated spin] source rank or -1
  const int8_t* sgn;
  int down;
  double* out;     // [n_rel + 1][2] overlaps
  int32_t* status;  // [n_rel] 1 converged, 2 invariant subspace, 3 m_max, 4 non-finite (3 and 4 stop the member)
  int32_t* m_used;  // [n_rel]
};

struct MembersArgs {
  const MemberSector* sectors;  // device
  const MemberDesc* members;    // device [n_members]
  int n_rel, m_max;
  double tol, tau;
  const void* traj;     // device: the source-sector state before the first and after every step
  int64_t traj_stride;  // elements between two recorded states
  int dim_dn_s;         // source sector's dim_dn
};

// LDS bytes a member workgroup keeps its sector's tables, strings, on-site
// energies and its operator map in (16-byte aligned pieces, in the kernel's
// order): gs_dn / 4 words of 8 bytes per down string, gs_up / 4 per up string,
// the strings, the energies when present, the map and its signs.
inline size_t members_table_lds(int dim_up, int dim_dn, int gs_up, int gs_dn, bool eps, int map_len) {
  auto a16 = [](size_t b) { return (b + 15) & ~size_t(15); };
  size_t t = a16(size_t(dim_dn) * (gs_dn / 4) * 8) + a16(size_t(dim_up) * (gs_up / 4) * 8) + a16(size_t(dim_up) * 4) +
             a16(size_t(dim_dn) * 4);
  if (eps) t += a16(size_t(dim_up) * 8) + a16(size_t(dim_dn) * 8);
  return t + a16(size_t(map_len) * 4) + a16(size_t(map_len));
}

// One workgroup per member (1,024 threads, `lds` bytes: tables and staging).
hipError_t launch_members(int prec, int n_members, const MembersArgs& a, size_t lds, hipStream_t s);

}  // namespace hub
