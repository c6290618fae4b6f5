// Host check of the XCD-contiguous work-group numbering (compiled with the host compiler).
// For every grid size up to 20,000 work-groups: the map is a bijection of [0, total), and the ids
// that one XCD runs (b = x, x + 8, x + 16, ... under round-robin dispatch) form one contiguous
// range, the ranges of XCDs 0..7 following each other in order.
#include <cstdio>
#include <vector>

#include "xcd.h"

int main() {
  for (int64_t total = 1; total <= 20000; ++total) {
    std::vector<int> seen(total, 0);
    for (int64_t b = 0; b < total; ++b) {
      const int64_t id = sfm::xcd_contiguous_id(b, total);
      if (id < 0 || id >= total || seen[id]++) {
        std::printf("total %lld: id %lld of b %lld repeated or out of range\n", (long long)total, (long long)id,
                    (long long)b);
        return 1;
      }
    }
    int64_t next = 0;
    for (int64_t x = 0; x < 8; ++x)
      for (int64_t b = x; b < total; b += 8) {
        const int64_t id = sfm::xcd_contiguous_id(b, total);
        if (id != next) {
          std::printf("total %lld: XCD %lld, b %lld has id %lld, expected %lld\n", (long long)total, (long long)x,
                      (long long)b, (long long)id, (long long)next);
          return 1;
        }
        ++next;
      }
  }
  std::printf("xcd numbering checks passed\n");
  return 0;
}
