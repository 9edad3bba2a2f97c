// Packing of the caller's hop coefficients into the fixed-size arrays of the
// kernel arguments (host code, no HIP).  The caller's array holds nv vectors
// of nc complex coefficients, [v][c] as (re, im) pairs, 2 nv nc doubles: no
// function here reads past it, and every entry it does not fill is zero.
#pragma once

#include <cstdint>

namespace hub {

// out[k] = coef[k] for k < 2 nv nc, else 0 (k < out_len); coef may be null.
inline void pack_block_coefs(const double* coef, int nv, int nc, double* out, int out_len) {
  const int n = 2 * nv * nc;
  for (int k = 0; k < out_len; ++k) out[k] = (coef && k < n) ? coef[k] : 0.0;
}

// Coefficient of vector 0 for each of 64 padded slots: slot s < nslots has
// class slot_class[s] (< nc), later slots get zero.  out: 128 doubles.
inline void pack_slot_coefs(const double* coef, int nc, const uint8_t* slot_class, int nslots, double* out) {
  for (int s = 0; s < 64; ++s) {
    const int c = slot_class[s];
    const bool ok = coef && s < nslots && c < nc;
    out[2 * s] = ok ? coef[2 * c] : 0.0;
    out[2 * s + 1] = ok ? coef[2 * c + 1] : 0.0;
  }
}

// Signed coefficient of vector 0 per (class, sign): out[2 (2 c + sg)] =
// (sg ? -1 : +1) coef_c for c < nc, zero up to max_classes.  out: 4
// max_classes doubles.
inline void pack_signed_coefs(const double* coef, int nc, int max_classes, double* out) {
  for (int c = 0; c < max_classes; ++c)
    for (int sg = 0; sg < 2; ++sg) {
      const double f = sg ? -1.0 : 1.0;
      const bool ok = coef && c < nc;
      out[2 * (2 * c + sg)] = ok ? f * coef[2 * c] : 0.0;
      out[2 * (2 * c + sg) + 1] = ok ? f * coef[2 * c + 1] : 0.0;
    }
}

}  // namespace hub
