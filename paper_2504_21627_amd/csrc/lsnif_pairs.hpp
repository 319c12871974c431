// Plan of one instanced pair query: inputs and the workspace regions it uses.
#pragma once
#include "lsnif_kernels.hpp"

namespace lsnif {

// Counters per object of the pair grouping at 2^bits cells per axis: 8 octants x cells^3 up
// to 5 bits, cells^3 alone (no octant) at 6, at least 4096 (the per-object scan works in
// chunks of 2048).  A query uses the finest pair_bits of its objects (coarser objects use a
// subset of their bins).
constexpr uint32_t kMaxPairBits = 6;
__host__ __device__ inline uint32_t pair_bins(uint32_t bits)
{
    return bits >= 6u ? 1u << 18 : 8u << (3u * (bits < 3u ? 3u : bits));
}

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
    uint32_t *keys;                  // [n_pairs] key of each pair: object bins + bin, n_objs bins if dropped
    uint32_t *slot_pair;             // [n_slots]
    int32_t *tile_obj;               // [n_tiles]
    uint32_t *rk[2], *rv[2];         // [n_pairs] each: the radix passes' keys and pair indices
    uint32_t *hist;                  // radix_hist_words(n_pairs): digit counters, then their scan partials
    uint32_t bins, bits;             // pair_bins(bits) keys per object; bits = the finest pair_bits
    uint32_t *obj_start;             // [n_objs + 1] first sorted position of each object; [n_objs]: live pairs
    uint32_t *obj_off;               // [n_objs] first slot of each object's tiles
    uint32_t n_slots, n_tiles;       // n_tiles * 256 == n_slots
};

}  // namespace lsnif
