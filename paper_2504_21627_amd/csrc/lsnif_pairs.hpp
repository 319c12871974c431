// Plan of one instanced pair query: inputs and the workspace regions it uses.
#pragma once
#include "lsnif_kernels.hpp"

namespace lsnif {

constexpr uint32_t kPairBins = 32768;  // per object: 8 octants x 16^3 cells (coarser grids use a subset)

struct PairPlan {
    const float4 *rays;
    uint32_t n_rays;
    const uint32_t *pair_ray, *pair_inst;
    uint32_t n_pairs;
    const lsnif_instance *inst;
    uint32_t n_inst;
    const ObjDev *objs;
    uint32_t n_objs;                 // entries of the object table (ids 0 .. n_objs-1)
    lsnif_hit *out;
    // workspace
    unsigned long long *minkey;      // [n_rays]
    PairRes *res;                    // [n_pairs]
    uint32_t *keys;                  // [n_pairs] bin of each pair, or 0xffffffff if dropped
    uint32_t *slot_pair;             // [n_slots]
    int32_t *tile_obj;               // [n_tiles]
    uint32_t *hist;                  // [n_objs * kPairBins]
    uint32_t *obj_total, *obj_off;   // [n_objs]
    uint32_t n_slots, n_tiles;       // n_tiles * 256 == n_slots
};

}  // namespace lsnif
