// Host-side sector basis and hop tables for the matrix-free Hubbard apply.
//
// Per spin: the C(Ns, n) occupation strings in increasing integer order; the
// rank of a string is the combinatorial number of Eq. (hashing)
// (sum over electrons k of C(p_k, k+1), positions p_k ascending, 0-based),
// which equals its position in that order.  For every string r the table
// lists the one-electron hops along bonds that END in r (gather form):
// source rank, fermionic sign (-1)^{electrons strictly between the two
// sites} of Eq. (sign-explanation), and the amplitude class.  A class is a
// distinct (t, d) pair, d the displacement of the directed hop, so that the
// hop contributes coef_c(A) = -t e^{i A d} times the sign.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace hub {

constexpr int kMaxSites = 16;
constexpr int kMaxClasses = 8;

struct HopClass {
  double t;   // hopping amplitude
  double d;   // displacement (R_dst - R_src) along the field
};

struct SpinTable {
  int n_el = 0;
  int dim = 0;
  std::vector<uint32_t> states;       // [dim], increasing
  std::vector<double> onsite;         // [dim] sum of eps_i over occupied sites (empty if none)
  // gather hops, CSR by target with class sub-ranges:
  // hops of target r and class c are hops[cls_ptr[r*(nc+1)+c] .. cls_ptr[r*(nc+1)+c+1])
  std::vector<int32_t> cls_ptr;       // [dim*(nc+1)]
  std::vector<uint32_t> hops;         // packed: src (bits 0..15) | class (16..23) | sign (bit 31)
  int max_hops = 0;
  // padded copy used by the row-staged apply: class c occupies slots
  // [slot_begin[c], slot_begin[c+1]) of every string (slot_class[s] = c);
  // entry tabc[r*maxs_pad + s] = src for a positive hop, src + dim + 1 for a
  // negative one, dim (a zero slot) where the string has fewer hops of that
  // class.  maxs_pad is the slot count rounded up to 4, 8, 12, 16, 20, 24, 32,
  // 48 or 64.
  std::vector<int32_t> slot_begin;    // [nc+1]
  std::vector<uint16_t> tabc;         // [dim*maxs_pad]
  std::vector<uint8_t> slot_class;    // [64]
  int nslots = 0, maxs_pad = 8;
  // the same entries with every class's slot range rounded up to a multiple
  // of 4 (group g = slots 4g..4g+3 belongs to class grp_class[g]), so the
  // block apply sums each group of staged values first and multiplies the
  // sum by its class coefficient once; gslots = total slots (0 if > 32)
  std::vector<uint16_t> tabg;         // [dim*gslots]
  std::vector<uint8_t> grp_class;     // [8]
  int gslots = 0;
};

struct Lattice {
  int n_sites = 0;
  std::vector<int> bi, bj;
  std::vector<double> bt, bdx;
  std::vector<double> onsite;  // empty if none
  double U = 0.0;
};

struct Basis {
  Lattice lat;
  int n_up = 0, n_dn = 0;
  std::vector<HopClass> classes;
  SpinTable up, dn;
  int64_t dim = 0;
  double norm_inf = 0.0;   // max absolute row sum of H (A-independent)
};

uint64_t binom(int n, int k);
uint32_t rank_of(uint32_t s, int n_sites);

// Validates the lattice and builds everything; returns "" on success or an
// error message.  `sector_error` is set when the particle numbers are invalid.
std::string build_basis(const Lattice& lat, int n_up, int n_dn, Basis& out, bool& sector_error);

}  // namespace hub
