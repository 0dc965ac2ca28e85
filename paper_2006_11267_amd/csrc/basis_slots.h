// Slot bookkeeping of the resident Krylov basis (host only, no HIP): slot k
// of a run lives in chunk k / per_chunk at byte offset (k % per_chunk) *
// stride, and the run's device table of slot pointers is extended in whole
// chunks by launches that each see the bases of at most per_launch chunks.
#pragma once

#include <algorithm>
#include <cstddef>

namespace ciq {

// Chunks holding slots [0, slots).
inline size_t basis_chunks_for(int slots, int per_chunk) {
    return ((size_t)slots + (size_t)per_chunk - 1) / (size_t)per_chunk;
}

// Extends a table that holds the first `first` slot pointers so that it
// holds at least min(slots, max_slots): whole chunks, so the new count is
// min(chunks * per_chunk, max_slots), which is returned. fn(lo, hi, k0) is
// called once per launch for the new entries [lo, hi), all of them in
// chunks k0 .. k0 + per_launch - 1; the launches cover [first, new count)
// once each, in order.
template <typename F>
int basis_table_ranges(int first, int slots, int per_chunk, int max_slots, int per_launch, F&& fn) {
    slots = std::min(slots, max_slots);
    if (slots <= first) return first;
    const size_t kend = basis_chunks_for(slots, per_chunk);
    const int cap = (int)std::min(kend * (size_t)per_chunk, (size_t)max_slots);
    for (size_t k0 = (size_t)first / per_chunk; k0 < kend; k0 += per_launch) {
        const int lo = std::max(first, (int)(k0 * per_chunk));
        const int hi = (int)std::min((k0 + per_launch) * (size_t)per_chunk, (size_t)cap);
        if (hi > lo) fn(lo, hi, (int)k0);
    }
    return cap;
}

}  // namespace ciq
