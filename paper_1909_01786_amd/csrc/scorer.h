// scorer.h -- launch interface of the learned Decision scorer (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

namespace asp {

// A tile is 64 consecutive rows (variables or static nogoods) of one instance.
struct ScorerTile {
    int32_t inst, row0;
};

struct ScorerArgs {
    const InstDesc* inst;
    const int32_t *ng_off, *ng_lits, *map_off, *rule_head;
    const MapEntry* map_ent;
    const uint8_t* w;            // device copy of asp_scorer_weights
    const int64_t* hv_off;       // per instance: byte offset of its (V+1) x 64 codes
    const int64_t* hc_off;       // per instance: byte offset of its n_static x 64 codes
    const ScorerTile* vtiles;
    const ScorerTile* ctiles;
    const int32_t* inst_list;    // instances whose rule scores are gathered,
    int32_t n_vtiles, n_ctiles, n_inst;
    int32_t single;              // or, with inst_list null, this one instance
    uint8_t* ws;
    int32_t* atom_score;
    int32_t* rule_score;
    int32_t* rule_ord_sc;              // (rule, head) pairs by rule score, descending
    unsigned long long* sort_tmp;      // one 8-byte word per rule (sort buffer)
};

// Readout training state (device pointers into the workspace).
struct TrainArgs {
    const int8_t* labels;   // per atom, laid out like the models output: 1, 0, or -1 (none)
    float* wb;              // [65] readout weights and bias (float)
    float* grad;            // [66] gradient sums and the loss
    float* m;               // [65] Adam first moments
    float* v;               // [65] Adam second moments
    float* loss;            // [steps] mean loss per step
    float inv_n;            // 1 / number of labelled atoms
    float lr;
};

hipError_t launch_readout_train(const ScorerArgs& a, const TrainArgs& t, int steps, int grid,
                                hipStream_t s);
hipError_t launch_scorer_embed(const ScorerArgs& a, int grid, hipStream_t s);
hipError_t launch_scorer_nogoods(const ScorerArgs& a, int layer, int grid, hipStream_t s);
hipError_t launch_scorer_vars(const ScorerArgs& a, int layer, int grid, hipStream_t s);
hipError_t launch_rule_scores(const ScorerArgs& a, hipStream_t s);

}  // namespace asp
