// Host check of the core SVD's pair order (the schedule helpers of
// small_body.hpp, which the Jacobi kernel and the V replay share): for every
// width l <= 128, one sweep meets every pair (p < q) exactly once, the pairs
// of a step are disjoint, every pair sits in a slot below the log's stride,
// and the step count matches jac_sweep_steps. Prints "ok" or the first
// failure; exit status 0 on success.
#include <cstdio>
#include <vector>
#include "small_body.hpp"

using namespace sor;

int main() {
  for (int l = 1; l <= 128; ++l) {
    const int slots = jac_groups(l);
    const int groups = slots;  // lane groups of the workgroup (8 or 16 lanes each)
    std::vector<int> met((size_t)l * l, 0);
    int steps = 0;
    for (int d = 0; d < jac_levels(l); ++d) {
      const int H = jac_level_steps(l, d);
      if ((1 << d) * H > slots) {
        printf("l %d level %d: %d slots needed, %d available\n", l, d, (1 << d) * H, slots);
        return 1;
      }
      for (int j = 0; j < H; ++j, ++steps) {
        std::vector<int> used(l, 0);
        for (int s = 0; s < groups; ++s) {
          const JacSlot sl = jac_slot(l, d, H, s);
          if (!(sl.g < sl.a) || j >= sl.R) continue;
          int mi = sl.g + j;
          if (mi >= sl.R) mi -= sl.R;
          if (mi >= sl.m) continue;
          const int p = sl.p, q = sl.s1 + mi;
          if (!(0 <= p && p < q && q < l)) {
            printf("l %d level %d step %d slot %d: pair (%d, %d) out of order or range\n", l, d, j, s, p, q);
            return 1;
          }
          if (++used[p] > 1 || ++used[q] > 1) {
            printf("l %d level %d step %d: column met twice in one step\n", l, d, j);
            return 1;
          }
          ++met[(size_t)p * l + q];
        }
      }
    }
    if (steps != jac_sweep_steps(l) || steps > 127) {
      printf("l %d: %d steps, jac_sweep_steps %d\n", l, steps, jac_sweep_steps(l));
      return 1;
    }
    for (int p = 0; p < l; ++p)
      for (int q = p + 1; q < l; ++q)
        if (met[(size_t)p * l + q] != 1) {
          printf("l %d: pair (%d, %d) met %d times\n", l, p, q, met[(size_t)p * l + q]);
          return 1;
        }
  }
  printf("ok\n");
  return 0;
}
