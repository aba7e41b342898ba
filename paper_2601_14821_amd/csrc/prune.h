// Pruning controller step and survivor compaction (paper Sec. 4.3).
#pragma once

#include "common.h"

namespace potr {

// State of the radix select, in the scratch buffer (device).
struct PruneState {
    uint64_t key;     // leading bits of the cut's key fixed so far (kbits of them)
    uint32_t id;      // leading bits of the cut's index fixed so far (ibits of them)
    int32_t kbits, ibits;
    int32_t done;     // nothing more to select (no candidate importance, or bad input)
    int32_t bad;      // an importance outside [0, 1] (or NaN) was seen
    int32_t pad;
    int64_t base;     // integer importance of the candidates ordered before the region
    int64_t total;    // integer importance of all candidates
    int64_t need;     // ceil(total / remaining): the budget in the same units
};

struct PruneArrays {
    const float* means;
    const float* scales;
    const float* quats;
    const float* opac;
    const float* sh;
    const int32_t* ids;
};

struct PruneOut {
    float* means;
    float* scales;
    float* quats;
    float* opac;
    float* sh;
    int32_t* ids;
};

size_t prune_select_scratch_bytes();
potr_status launch_prune_select(int64_t N, const float* dmse, const float* imp, double dmax, int32_t remaining,
                                double a, void* scratch, uint8_t* remove, int64_t* n_removed, hipStream_t s);
// The same with the scratch in the library's static device array (no allocation).
potr_status launch_prune_select_noalloc(int64_t N, const float* dmse, const float* imp, double dmax,
                                        int32_t remaining, double a, uint8_t* remove, int64_t* n_removed,
                                        hipStream_t s);
size_t prune_compact_scratch_bytes(int64_t N);
potr_status launch_prune_compact(int64_t N, const uint8_t* remove, const PruneArrays& in, const PruneOut& out,
                                 void* scratch, int64_t* n_kept, hipStream_t s);

}  // namespace potr
