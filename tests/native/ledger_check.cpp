// Checks of the residency ledger's rule (tg_ledger.h) on the CPU: which
// in-flight persistent launches a new launch must follow in stream order.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tg_ledger.h"

using tg::Flight;

static int failures = 0;

static void expect(const char* what, const std::vector<size_t>& got, const std::vector<size_t>& want) {
  if (got != want) {
    std::printf("FAIL %s: got", what);
    for (size_t i : got) std::printf(" %zu", i);
    std::printf(", want");
    for (size_t i : want) std::printf(" %zu", i);
    std::printf("\n");
    ++failures;
  }
}

static Flight fl(const void* key, uint64_t variant, uint64_t workers, uint64_t cap, uintptr_t stream, int dev = 0) {
  Flight f;
  f.key = key;
  f.dev = dev;
  f.variant = variant;
  f.workers = workers;
  f.capacity = cap;
  f.stream = stream;
  return f;
}

int main() {
  const uint64_t wave = tg::flight_variant(1, 1, 1), wg4 = tg::flight_variant(2, 4, 1),
                 gang = tg::flight_variant(3, 4, 8);
  int k[8];
  const uint64_t cap = 8192;
  // nothing in flight
  expect("empty", tg::flights_to_follow({}, fl(&k[0], wave, cap, cap, 1)), {});
  // the same stream is ordered already, even when the two do not fit together
  expect("same stream", tg::flights_to_follow({fl(&k[1], wave, cap, cap, 1)}, fl(&k[0], wave, cap, cap, 1)), {});
  // two full launches on two streams must not overlap
  expect("full + full", tg::flights_to_follow({fl(&k[1], wave, cap, cap, 2)}, fl(&k[0], wave, cap, cap, 1)), {0});
  // halves of one variant fit together
  expect("half + half", tg::flights_to_follow({fl(&k[1], wave, cap / 2, cap, 2)}, fl(&k[0], wave, cap / 2, cap, 1)), {});
  // one worker over the capacity: wait
  expect("half + half + 1",
         tg::flights_to_follow({fl(&k[1], wave, cap / 2, cap, 2)}, fl(&k[0], wave, cap / 2 + 1, cap, 1)), {0});
  // four serving slots of capacity / 4 overlap; a fifth launch on a fifth
  // stream does not fit and follows all four
  std::vector<Flight> slots;
  for (int i = 0; i < 4; ++i) {
    expect("slot admitted", tg::flights_to_follow(slots, fl(&k[i], wave, cap / 4, cap, 10 + i)), {});
    slots.push_back(fl(&k[i], wave, cap / 4, cap, 10 + i));
  }
  expect("fifth slot", tg::flights_to_follow(slots, fl(&k[4], wave, cap / 4, cap, 20)), {0, 1, 2, 3});
  // ... but on one of the slots' own streams it only needs the other three
  // to fit with it, and they do (3 x cap/4 + cap/4)
  expect("slot stream reuse", tg::flights_to_follow(slots, fl(&k[4], wave, cap / 4, cap, 11)), {});
  // different variants never share the device, even if both are small
  expect("variants differ",
         tg::flights_to_follow({fl(&k[1], wg4, 16, 2048, 2), fl(&k[2], wave, 64, cap, 3)}, fl(&k[0], wave, 64, cap, 1)),
         {0, 1});
  expect("gang vs workgroup", tg::flights_to_follow({fl(&k[1], wg4, 16, 2048, 2)}, fl(&k[0], gang, 16, 2048, 1)), {0});
  // launches on another device are not counted
  expect("other device", tg::flights_to_follow({fl(&k[1], wave, cap, cap, 2, 1)}, fl(&k[0], wave, cap, cap, 1, 0)), {});
  // a mix: same-stream entries skipped, the others all followed when over
  expect("mixed", tg::flights_to_follow({fl(&k[1], wave, cap / 2, cap, 1), fl(&k[2], wave, cap / 2, cap, 2),
                                         fl(&k[3], wave, cap / 4, cap, 3)},
                                        fl(&k[0], wave, cap / 2, cap, 1)),
         {1, 2});
  if (failures) return 1;
  std::printf("ledger rule: all cases pass\n");
  return 0;
}
