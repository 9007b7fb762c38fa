// Checks of the factor-table index maps (test infrastructure): for several
// chunk counts G and chunk lengths M, both layouts place every (field,
// position) and every (field, chunk) at a distinct index inside the table,
// and in the paired layout each pair of fields of one position (or chunk)
// occupies one 16-byte-aligned slot, first field first.  Prints "ok" or the
// first failure and exits non-zero.
#include <cstdio>
#include <vector>

#include "hip/hip_runtime.h"
#include "device.hpp"

using namespace adi;

static int fail(const char* what, int G, int M, int f, long i) {
  std::printf("FAIL %s G=%d M=%d field=%d index=%ld\n", what, G, M, f, i);
  return 1;
}

int main() {
  const int Gs[] = {2, 64, 128, 256, 512, 1024};
  const int Ms[] = {3, 4, 5, 8, 10};
  const int pairs_pos[][2] = {{P_W, P_QA}, {P_CP, P_SP}, {P_OC, P_OK}};
  const int pairs_chk[][2] = {{C_CS, C_AE}, {C_W0, C_Q0}, {C_C0, C_W1}, {C_Q1, C_C1}};
  for (int G : Gs)
    for (int M : Ms) {
      const long GM = (long)G * M;
      for (int paired = 0; paired < 2; ++paired) {
        std::vector<int> seen(P_NFIELDS * GM, 0), cseen(C_NFIELDS * G, 0);
        for (int f = 0; f < P_NFIELDS; ++f)
          for (long ix = 0; ix < GM; ++ix) {
            const long a = pos_at(f, GM, ix, paired);
            if (a < 0 || a >= P_NFIELDS * GM) return fail("position index outside the table", G, M, f, ix);
            if (seen[a]++) return fail("two entries at one position index", G, M, f, ix);
            if (!paired && a != f * GM + ix) return fail("plain layout is not field-major", G, M, f, ix);
          }
        for (int f = 0; f < C_NFIELDS; ++f)
          for (long k = 0; k < G; ++k) {
            const long a = chk_at(f, G, k, paired);
            if (a < 0 || a >= C_NFIELDS * G) return fail("chunk index outside the table", G, M, f, k);
            if (cseen[a]++) return fail("two entries at one chunk index", G, M, f, k);
            if (!paired && a != f * G + k) return fail("plain chunk layout is not field-major", G, M, f, k);
          }
        if (!paired) continue;
        for (auto& p : pairs_pos)
          for (long ix = 0; ix < GM; ++ix) {
            const long a = pos_at(p[0], GM, ix, true), b = pos_at(p[1], GM, ix, true);
            if (b != a + 1 || a % 2) return fail("position pair not in one aligned slot", G, M, p[0], ix);
          }
        for (auto& p : pairs_chk)
          for (long k = 0; k < G; ++k) {
            const long a = chk_at(p[0], G, k, true), b = chk_at(p[1], G, k, true);
            if (b != a + 1 || a % 2) return fail("chunk pair not in one aligned slot", G, M, p[0], k);
          }
        // the class tables of a direction follow one another at multiples of
        // P_NFIELDS*GM and C_NFIELDS*G doubles: pair slots stay 16-byte aligned
        if ((P_NFIELDS * GM) % 2 || (C_NFIELDS * (long)G) % 2) return fail("class stride breaks pair alignment", G, M, -1, 0);
      }
    }
  std::printf("ok\n");
  return 0;
}
