// layout.h -- device data layout of libasp (internal to the library).
//
// One arena (caller-owned device memory) holds, 256-byte aligned:
//   [static]  per-instance descriptors, the instance order, and every
//             instance's completion nogoods (CSR), literal->nogood map (CSR),
//             rule table and rule bodies, packed one instance after another;
//   [results] verdicts, per-instance counters, model bytes, queue counters;
//   [slots]   one dynamic search state per persistent workgroup, reused by
//             every instance that workgroup solves.
//
// Variables are 1..V (0 unused).  Literal index of literal l is 2*|l| + (l<0).
#pragma once
#include <stdint.h>

namespace asp {

constexpr int kMaxW = 64;           // Deps words per variable
constexpr int kAlign = 256;

// Static description of one instance (element offsets into the packed arrays).
struct InstDesc {
    int64_t ng_off;    // into ng_off[]: n_static+1 entries, values relative to ng_lits
    int64_t ng_lits;   // into ng_lits[]
    int64_t map_off;   // into map_off[]: 2(V+1)+1 entries, values relative to map_ids
    int64_t map_ids;   // into map_ids[]
    int64_t rules;     // into rule_head[] / rule_occ[] (Rh entries)
    int64_t rb_off;    // into rb_off[] (Rh+1 entries, values relative to rb_lits)
    int64_t rb_lits;   // into rb_lits[] (rule bodies, +a body+ / -a body-)
    int64_t model;     // byte offset of this instance's model in models[]
    int32_t A, Rh, V, n_static;
    int32_t u0, u1;    // ids of the unit nogoods: [u0, u1)
    int32_t has_empty; // an empty nogood (empty-body constraint) exists
    int32_t pad;
};

// Per-slot control block (the persistent state of the search between
// launches of the step kernels; the solve kernel keeps it in LDS).
struct SlotCtrl {
    int32_t inst, cdl, qh, qt;
    int32_t n_learned, pool_top, pending, pend_kind;  // pend_kind 0 none, 1 round, 2 gate
    int32_t status, init_done, last_step, pad0;
    int64_t learned_lits;
    int64_t rounds, visits, checks, props, decisions, conflicts, learned, learned_len,
            gate_fail, completes;
    uint64_t hash;
    uint64_t pend_B[kMaxW];           // gate conflict bitmap awaiting learning
};

// Element offsets of each array inside one slot (bytes for val8).
struct SlotLayout {
    int64_t ctrl;       // bytes
    int64_t val8;       // bytes, int8[Vmax+1]
    int64_t lvl;        // bytes, int32[Vmax+1]
    int64_t deps;       // bytes, uint64[(Vmax+1)*W]
    int64_t win;        // bytes, int32[Vmax+1]
    int64_t trail;      // bytes, int32[Vmax+1]
    int64_t tlim;       // bytes, int32[Rhmax+3]
    int64_t dec;        // bytes, int32[Rhmax+3]
    int64_t locc_ptr;   // bytes, int32[2(Vmax+1)]
    int64_t locc_n;     // bytes, int32[2(Vmax+1)]
    int64_t locc_cap;   // bytes, int32[2(Vmax+1)]
    int64_t l_off;      // bytes, int32[cap_ng+1]
    int64_t l_lits;     // bytes, int32[cap_lits]
    int64_t pool;       // bytes, int32[pool_cap]
    int64_t stride;     // bytes per slot
    int64_t pool_cap;   // entries
};

struct DevStats {
    int64_t rounds, visits, checks, props, decisions, conflicts, learned, learned_len,
            gate_fail, completes;
    uint64_t hash;
    int32_t status, last_step;
};

enum StepKind : int32_t {
    STEP_NONE = 0, STEP_INIT = 1, STEP_ROUND = 2, STEP_LEARN = 3, STEP_DECIDE = 4,
    STEP_COMPLETE = 5, STEP_GATE = 6, STEP_DONE = 7
};

enum Mode : int32_t {
    MODE_SOLVE = 0,      // persistent: pop instances, solve each to a verdict
    MODE_STEPS = 1,      // slot 0, instance 0: run up to max_steps steps
    MODE_RESET = 2,      // slot 0, instance 0: fresh search state
};

// Status values (match asp.h).
enum : int32_t {
    ST_RUNNING = 6, ST_SAT = 1, ST_UNSAT = 2, ST_UNKNOWN = 3,
    ST_E_CAPACITY = -2, ST_E_INTERNAL = -5, ST_E_TIMEOUT = -6
};

struct KArgs {
    const InstDesc* inst;
    const int32_t* order;        // instance ids, largest first
    int32_t n_inst;
    int32_t mode;
    const int32_t* ng_off;
    const int32_t* ng_lits;
    const int32_t* map_off;
    const int32_t* map_ids;
    const int32_t* rule_head;
    const int32_t* rule_occ;
    const int32_t* rb_off;
    const int32_t* rb_lits;
    uint8_t* slots;
    SlotLayout lay;
    int32_t* queue;              // [0] next order index, [1] finished count
    int32_t* verdicts;
    DevStats* stats;
    uint8_t* models;
    int32_t W, gate_mode;
    int32_t words;               // LDS words per 2-bit bitmap (Vmax+1 vars)
    int32_t step_mask;           // MODE_STEPS: kinds allowed to run (bit k)
    int64_t max_steps;           // MODE_STEPS: steps to run; MODE_SOLVE: guard
    int64_t max_conflicts;       // <0 unlimited
    int64_t cap_ng, cap_lits;
    uint64_t max_ticks;          // wall-clock guard in s_memrealtime ticks, 0 none
};

}  // namespace asp
