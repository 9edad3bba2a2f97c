// Host-side sector basis and hop tables (see basis.h).
#include "basis.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <utility>

namespace hub {

uint64_t binom(int n, int k) {
  if (k < 0 || n < 0 || k > n) return 0;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * static_cast<uint64_t>(n - k + i) / static_cast<uint64_t>(i);
  return r;
}

// Eq. (hashing): I = sum_k C(p_k, k+1) over the electrons, positions ascending.
uint32_t rank_of(uint32_t s, int n_sites) {
  uint64_t r = 0;
  int k = 0;
  for (int p = 0; p < n_sites; ++p) {
    if (s >> p & 1u) {
      ++k;
      r += binom(p, k);
    }
  }
  return static_cast<uint32_t>(r);
}

static int find_class(std::vector<HopClass>& cls, double t, double d) {
  for (size_t c = 0; c < cls.size(); ++c)
    if (cls[c].t == t && cls[c].d == d) return static_cast<int>(c);
  cls.push_back({t, d});
  return static_cast<int>(cls.size()) - 1;
}

static void build_spin(const Lattice& lat, int n_el, const std::vector<HopClass>& classes,
                       const std::vector<std::pair<std::pair<int, int>, int>>& directed,
                       SpinTable& T) {
  const int ns = lat.n_sites;
  const int nc = static_cast<int>(classes.size());
  T.n_el = n_el;
  T.dim = static_cast<int>(binom(ns, n_el));
  T.states.resize(T.dim);
  // increasing integers with n_el set bits below 2^ns (next-combination step)
  if (n_el == 0) {
    T.states[0] = 0;
  } else {
    uint32_t s = (1u << n_el) - 1u;
    for (int k = 0; k < T.dim; ++k) {
      T.states[k] = s;
      const uint32_t c = s & (0u - s);
      const uint32_t r = s + c;
      s = (((r ^ s) >> 2) / c) | r;
    }
  }
  if (!lat.onsite.empty()) {
    T.onsite.resize(T.dim);
    for (int k = 0; k < T.dim; ++k) {
      double e = 0.0;
      for (int i = 0; i < ns; ++i)
        if (T.states[k] >> i & 1u) e += lat.onsite[i];
      T.onsite[k] = e;
    }
  }
  // gather hops by class
  T.cls_ptr.assign(static_cast<size_t>(T.dim) * (nc + 1), 0);
  T.hops.clear();
  std::vector<std::vector<int>> count(nc, std::vector<int>(T.dim, 0));
  T.max_hops = 0;
  for (int r = 0; r < T.dim; ++r) {
    const uint32_t s = T.states[r];
    int nh = 0;
    for (int c = 0; c < nc; ++c) {
      T.cls_ptr[static_cast<size_t>(r) * (nc + 1) + c] = static_cast<int32_t>(T.hops.size());
      for (const auto& dh : directed) {
        if (dh.second != c) continue;
        const int dst = dh.first.first, src = dh.first.second;
        // the hop src -> dst ends in s: dst occupied, src empty in s
        if (!(s >> dst & 1u) || (s >> src & 1u)) continue;
        const uint32_t from = s ^ (1u << dst) ^ (1u << src);
        const int lo = std::min(dst, src), hi = std::max(dst, src);
        const uint32_t between = (hi - lo > 1) ? ((s >> (lo + 1)) & ((1u << (hi - lo - 1)) - 1u)) : 0u;
        const uint32_t sign = static_cast<uint32_t>(__builtin_popcount(between) & 1);
        T.hops.push_back(rank_of(from, ns) | (static_cast<uint32_t>(c) << 16) | (sign << 31));
        ++count[c][r];
        ++nh;
      }
    }
    T.cls_ptr[static_cast<size_t>(r) * (nc + 1) + nc] = static_cast<int32_t>(T.hops.size());
    T.max_hops = std::max(T.max_hops, nh);
  }
  // padded, class-sorted copy for the apply kernel
  T.slot_begin.assign(nc + 1, 0);
  for (int c = 0; c < nc; ++c) {
    int mx = 0;
    for (int r = 0; r < T.dim; ++r) mx = std::max(mx, count[c][r]);
    T.slot_begin[c + 1] = T.slot_begin[c] + mx;
  }
  const int slots = T.slot_begin[nc];
  T.nslots = slots;
  T.maxs_pad = 64;
  for (int cand : {4, 8, 12, 16, 20, 24, 32, 48, 64})
    if (slots <= cand) {
      T.maxs_pad = cand;
      break;
    }
  // entry = source rank, plus (dim + 1) when the hop's sign is negative: the
  // apply stages each row as +x, -x with a zero slot at index dim; pads read it
  T.tabc.assign(static_cast<size_t>(T.maxs_pad) * T.dim, static_cast<uint16_t>(T.dim));
  for (int r = 0; r < T.dim; ++r) {
    for (int c = 0; c < nc; ++c) {
      const int b = T.cls_ptr[static_cast<size_t>(r) * (nc + 1) + c];
      const int e = T.cls_ptr[static_cast<size_t>(r) * (nc + 1) + c + 1];
      for (int k = b; k < e; ++k) {
        const uint32_t h = T.hops[k];
        const uint32_t v = (h & 0xFFFFu) + ((h >> 31) ? static_cast<uint32_t>(T.dim + 1) : 0u);
        T.tabc[static_cast<size_t>(r) * T.maxs_pad + T.slot_begin[c] + (k - b)] = static_cast<uint16_t>(v);
      }
    }
  }
  T.slot_class.assign(64, 0);
  for (int c = 0; c < nc; ++c)
    for (int s = T.slot_begin[c]; s < T.slot_begin[c + 1] && s < 64; ++s) T.slot_class[s] = static_cast<uint8_t>(c);
  // grouped copy: class c gets round_up(max hops of c, 4) slots
  std::vector<int> gbeg(nc + 1, 0);
  for (int c = 0; c < nc; ++c) gbeg[c + 1] = gbeg[c] + ((T.slot_begin[c + 1] - T.slot_begin[c] + 3) / 4) * 4;
  T.grp_class.assign(8, 0);
  T.gslots = gbeg[nc] <= 32 ? gbeg[nc] : 0;
  T.tabg.clear();
  if (T.gslots > 0) {
    for (int c = 0; c < nc; ++c)
      for (int g = gbeg[c] / 4; g < gbeg[c + 1] / 4; ++g) T.grp_class[g] = static_cast<uint8_t>(c);
    T.tabg.assign(static_cast<size_t>(T.gslots) * T.dim, static_cast<uint16_t>(T.dim));
    for (int r = 0; r < T.dim; ++r)
      for (int c = 0; c < nc; ++c)
        for (int s = T.slot_begin[c]; s < T.slot_begin[c + 1]; ++s)
          T.tabg[static_cast<size_t>(r) * T.gslots + gbeg[c] + (s - T.slot_begin[c])] =
              T.tabc[static_cast<size_t>(r) * T.maxs_pad + s];
  }
}

std::string build_basis(const Lattice& lat, int n_up, int n_dn, Basis& B, bool& sector_error) {
  sector_error = false;
  const int ns = lat.n_sites;
  if (ns < 1 || ns > kMaxSites) return "n_sites must be in 1..16";
  if (n_up < 0 || n_up > ns || n_dn < 0 || n_dn > ns) {
    sector_error = true;
    return "particle numbers must lie in 0..n_sites";
  }
  const size_t nb = lat.bi.size();
  if (lat.bj.size() != nb || lat.bt.size() != nb || lat.bdx.size() != nb)
    return "bond arrays differ in length";
  std::set<std::pair<int, int>> seen;
  for (size_t k = 0; k < nb; ++k) {
    const int i = lat.bi[k], j = lat.bj[k];
    if (i < 0 || i >= ns || j < 0 || j >= ns) return "bond endpoint out of range";
    if (i == j) return "bond from a site to itself (use onsite)";
    if (!std::isfinite(lat.bt[k]) || !std::isfinite(lat.bdx[k])) return "non-finite bond data";
    const auto key = std::make_pair(std::min(i, j), std::max(i, j));
    if (seen.count(key)) return "bond listed twice";
    seen.insert(key);
  }
  if (!std::isfinite(lat.U)) return "non-finite U";
  for (double e : lat.onsite)
    if (!std::isfinite(e)) return "non-finite onsite energy";
  if (!lat.onsite.empty() && static_cast<int>(lat.onsite.size()) != ns) return "onsite size";

  B.lat = lat;
  B.n_up = n_up;
  B.n_dn = n_dn;
  B.classes.clear();
  // directed hops: bond (i, j, t, dx) gives j -> i with displacement dx and
  // i -> j with -dx.  Normalise -0.0 to 0.0 so equal displacements share a class.
  std::vector<std::pair<std::pair<int, int>, int>> directed;
  for (size_t k = 0; k < nb; ++k) {
    if (lat.bt[k] == 0.0) continue;  // a zero amplitude contributes nothing
    const double d = lat.bdx[k] + 0.0, md = -lat.bdx[k] + 0.0;
    directed.push_back({{lat.bi[k], lat.bj[k]}, find_class(B.classes, lat.bt[k], d)});
    directed.push_back({{lat.bj[k], lat.bi[k]}, find_class(B.classes, lat.bt[k], md)});
  }
  if (static_cast<int>(B.classes.size()) > kMaxClasses)
    return "more than 8 distinct (t, displacement) hop classes";
  build_spin(lat, n_up, B.classes, directed, B.up);
  build_spin(lat, n_dn, B.classes, directed, B.dn);
  if (B.dn.nslots > 64) return "more than 64 padded hop slots per string (too many bonds for the apply kernel)";
  B.dim = static_cast<int64_t>(B.up.dim) * B.dn.dim;

  // |H|_inf = max over (a, b) of |diag| + sum of |hop amplitudes|
  const int nc = static_cast<int>(B.classes.size());
  auto hop_abs = [&](const SpinTable& T, int r) {
    double s = 0.0;
    for (int c = 0; c < nc; ++c) {
      const int b = T.cls_ptr[static_cast<size_t>(r) * (nc + 1) + c];
      const int e = T.cls_ptr[static_cast<size_t>(r) * (nc + 1) + c + 1];
      s += std::fabs(B.classes[c].t) * (e - b);
    }
    return s;
  };
  std::vector<double> hu(B.up.dim), hd(B.dn.dim);
  for (int a = 0; a < B.up.dim; ++a) hu[a] = hop_abs(B.up, a);
  for (int b = 0; b < B.dn.dim; ++b) hd[b] = hop_abs(B.dn, b);
  double mx = 0.0;
  for (int a = 0; a < B.up.dim; ++a) {
    for (int b = 0; b < B.dn.dim; ++b) {
      double diag = lat.U * __builtin_popcount(B.up.states[a] & B.dn.states[b]);
      if (!lat.onsite.empty()) diag += B.up.onsite[a] + B.dn.onsite[b];
      mx = std::max(mx, std::fabs(diag) + hu[a] + hd[b]);
    }
  }
  B.norm_inf = mx;
  return "";
}

}  // namespace hub
