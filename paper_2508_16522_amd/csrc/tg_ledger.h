// Residency ledger of persistent launches (plain C++, no HIP types, so the
// rule can be checked on a machine without a GPU).
//
// Every worker of a persistent launch waits on counters that other workers
// of the same launch decrement, so all of its workers must be resident on
// the device at the same time.  The library never launches more workers of
// a kernel variant than a probe launch has shown to be co-resident (the
// variant's capacity).  Two launches in flight on different streams share
// the device, however: if their workers together exceed what fits, some
// workers of one launch wait in the dispatcher behind workers of the other
// that spin on counters owned by them.  The ledger records every launch in
// flight and, before a new launch is issued, decides which earlier ones it
// must follow in stream order (the caller makes the new launch's stream wait
// on their completion events):
//   - launches on the same stream are ordered already and are not counted;
//   - the new launch may overlap the in-flight launches of other streams only
//     if all of them are of the same kernel variant (same per-worker
//     resources, so the calibrated capacity applies to their sum) and their
//     workers together with its own fit that capacity;
//   - otherwise it waits for all of them.
// The serving loop's launch slots are sized so that their launches always
// overlap (each takes capacity / slots workers of one variant).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace tg {

struct Flight {
  const void* key = nullptr;  // the layout launched (one entry per layout)
  int dev = 0;                // device ordinal
  uint64_t variant = 0;       // kernel variant: mapping, workgroup size, gang size
  uint64_t workers = 0;       // co-resident units this launch occupies (workgroups)
  uint64_t capacity = 0;      // calibrated co-resident units of the variant
  uintptr_t stream = 0;       // stream the launch was issued on
};

inline uint64_t flight_variant(uint32_t mapping, uint32_t wg_waves, uint32_t gang) {
  return ((uint64_t)mapping << 40) | ((uint64_t)wg_waves << 20) | (uint64_t)gang;
}

// Indices into `in_flight` (launches not yet finished) that the launch
// `next` must wait for.
inline std::vector<size_t> flights_to_follow(const std::vector<Flight>& in_flight, const Flight& next) {
  std::vector<size_t> others;
  uint64_t sum = next.workers;
  bool same_variant = true;
  for (size_t i = 0; i < in_flight.size(); ++i) {
    const Flight& f = in_flight[i];
    if (f.dev != next.dev || f.stream == next.stream) continue;
    others.push_back(i);
    sum += f.workers;
    if (f.variant != next.variant) same_variant = false;
  }
  if (others.empty() || (same_variant && sum <= next.capacity)) return {};
  return others;
}

}  // namespace tg
