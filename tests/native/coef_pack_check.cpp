// Host check of the launch-argument coefficient packing (coef_pack.h) under
// AddressSanitizer/UBSan: for nv = 1..8 vectors and nc = 1..8 classes the
// caller's array is allocated with exactly 2 nv nc doubles, so any read past
// it aborts; the packed values are compared with their definition.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "coef_pack.h"

static int fails = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++fails;                                                        \
    }                                                                 \
  } while (0)

int main() {
  constexpr int kMaxNV = 8, kMaxClasses = 8;
  for (int nv = 1; nv <= kMaxNV; ++nv)
    for (int nc = 1; nc <= kMaxClasses; ++nc) {
      const int n = 2 * nv * nc;
      double* coef = static_cast<double*>(std::malloc(sizeof(double) * n));  // exactly the caller's size
      for (int k = 0; k < n; ++k) coef[k] = 1.0 + k;
      std::vector<double> blk(2 * kMaxNV * kMaxClasses, -7.0);
      hub::pack_block_coefs(coef, nv, nc, blk.data(), static_cast<int>(blk.size()));
      for (int k = 0; k < static_cast<int>(blk.size()); ++k) CHECK(blk[k] == (k < n ? 1.0 + k : 0.0));
      // slots: classes in ascending runs, nslots below, at and above 64 boundaries
      for (int nslots : {0, 1, 5, nc * 3, 63, 64}) {
        uint8_t cls[64];
        for (int s = 0; s < 64; ++s) cls[s] = static_cast<uint8_t>(s < nslots ? (s * nc) / (nslots ? nslots : 1) : 0);
        std::vector<double> sl(128, -7.0);
        hub::pack_slot_coefs(coef, nc, cls, nslots, sl.data());
        for (int s = 0; s < 64; ++s) {
          const bool on = s < nslots;
          CHECK(sl[2 * s] == (on ? coef[2 * cls[s]] : 0.0));
          CHECK(sl[2 * s + 1] == (on ? coef[2 * cls[s] + 1] : 0.0));
        }
      }
      std::vector<double> sg(4 * kMaxClasses, -7.0);
      hub::pack_signed_coefs(coef, nc, kMaxClasses, sg.data());
      for (int c = 0; c < kMaxClasses; ++c)
        for (int s = 0; s < 2; ++s) {
          const double f = s ? -1.0 : 1.0;
          CHECK(sg[2 * (2 * c + s)] == (c < nc ? f * coef[2 * c] : 0.0));
          CHECK(sg[2 * (2 * c + s) + 1] == (c < nc ? f * coef[2 * c + 1] : 0.0));
        }
      std::free(coef);
    }
  // a null caller array packs zeros
  std::vector<double> z(128, -7.0);
  hub::pack_block_coefs(nullptr, 8, 8, z.data(), 128);
  for (double v : z) CHECK(v == 0.0);
  std::printf("%s\n", fails ? "FAIL" : "coef_pack ok");
  return fails ? 1 : 0;
}
