// layout.h -- device data layout of libasp (internal to the library).
//
// One arena (caller-owned device memory) holds, 256-byte aligned:
//   [static]  per-instance descriptors, the instance order, and every
//             instance's completion nogoods (CSR), literal->nogood map (CSR),
//             rule table and rule bodies, packed one instance after another;
//   [scores]  per-instance decision scores of atoms and of rules (the score
//             of each rule's head), written before a score-driven search;
//   [results] verdicts, per-instance counters, model bytes;
//   [slots]   one dynamic search state per instance, sized for it.
//
// Variables are 1..V (0 unused).  Literal index of literal l is 2*|l| + (l<0).
#pragma once
#include <stdint.h>

namespace asp {

constexpr int kMaxW = 64;           // Deps words per variable
constexpr int kAlign = 256;

// One entry of the literal -> nogood map: the nogood's id, the map's own
// literal, and the nogood's other literals when it has at most three (0
// pads the unused ones), each with the map segment (start, size) of its
// complement -- the literal a unit nogood makes true.  A longer nogood has
// o1 = kLongNogood, o2 = the start of its literals in the nogood CSR and
// a1 = their count, so that its literals are read right after the entry.
// A visit of a short nogood is one 32-byte load.
struct alignas(32) MapEntry {
    int32_t id, self, o1, o2;
    int32_t a1, n1, a2, n2;
};
constexpr int32_t kLongNogood = (int32_t)0x80000000;

// Static description of one instance (element offsets into the packed arrays).
struct InstDesc {
    int64_t ng_off;    // into ng_off[]: n_static+1 entries, values relative to ng_lits
    int64_t ng_lits;   // into ng_lits[]
    int64_t map_off;   // into map_off[]: 2(V+1)+1 entries, values relative to map_ids
    int64_t map_ids;   // into map_ent[]
    int64_t rules;     // into rule_head[] / rule_occ[] (Rh entries)
    int64_t rb_off;    // into rb_off[] (Rh+1 entries, values relative to rb_lits)
    int64_t rb_lits;   // into rb_lits[] (rule bodies, +a body+ / -a body-)
    int64_t model;     // byte offset of this instance's answer sets in models[]
                       // (model_store of them, A bytes each)
    int64_t ascore;    // into atom_score[] (A+1 entries, [0] unused)
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
    int32_t status, init_done, last_step, use_score;
    int32_t consec, dec_open;                // learned-Decision fallback state
    int32_t epoch, exhausted;                // resolution marks; no answer set left
    int32_t n_pend, pend_more[7];            // round conflicts selected for learning
    int64_t learned_lits;
    int64_t models, restarts, since_restart; // answer sets found, restarts
    int64_t rounds, visits, checks, props, decisions, conflicts, learned, learned_len,
            gate_fail, completes;
    uint64_t hash;
    uint64_t pend_B[kMaxW];           // gate conflict bitmap awaiting learning
};

// Byte offsets of each array inside one instance's state slot.
struct SlotLayout {
    int64_t ctrl;       // SlotCtrl
    int64_t val8;       // int8[V+1]
    int64_t pend;       // uint32[(V+1+15)/16] values implied in the current round for
                        // variables past the LDS winner table (2 bits each); zero at rest
    int64_t lvl;        // int32[V+1] (Res-learning only: the Fwd search derives
                        // a level from the trail position and tlim)
    int64_t deps;       // uint64[(V+1)*W]
    int64_t win;        // uint64[V+1] winner key: (id*2 + pol) << 32 | map entry
    int64_t trail;      // int32[V+1]
    int64_t tlim;       // int32[Rh+3]
    int64_t dec;        // int32[Rh+3]
    int64_t locc_ptr;   // int32[2(V+1)]
    int64_t locc_n;     // int32[2(V+1)]
    int64_t locc_cap;   // int32[2(V+1)]
    int64_t l_off;      // int32[cap_ng+1]
    int64_t l_lits;     // int32[cap_lits]
    int64_t pool;       // int32[pool_cap]
    int64_t gpos;       // int32[V+1] trail position where the assigning step begins
    int64_t reason;     // int32[V+1] nogood that implied the assignment, -1 none
    int64_t mark;       // int32[V+1] resolution membership (epoch)
    int64_t resd;       // int32[V+1] variables of the nogood being resolved
    int64_t act;        // int32[V+1] activity of each atom (activity Decision)
    int64_t stride;     // bytes of the slot
    int64_t pool_cap;   // entries
};

// Slot of an instance with V variables and Rh headed rules.  A doubling
// list of n entries has used at most 4n + 8 pool entries.  Fwd-learning
// learns decision literals T b_r only, so at most Rh occurrence lists exist;
// Res-learning may learn any literal (at most min(cap_lits, 2(V+1)) lists).
__host__ __device__ inline SlotLayout slot_layout(int64_t V, int64_t Rh, int32_t W,
                                                  int64_t cap_ng, int64_t cap_lits,
                                                  int32_t learning) {
    SlotLayout L;
    int64_t o = 0;
    const int64_t V1 = V + 1, R3 = Rh + 3;
#define ASP_TAKE(field, bytes) do { L.field = o; o = (o + (bytes) + kAlign - 1) / kAlign * kAlign; } while (0)
    ASP_TAKE(ctrl, (int64_t)sizeof(SlotCtrl));
    ASP_TAKE(val8, V1);
    ASP_TAKE(pend, 4 * ((V1 + 15) / 16));
    ASP_TAKE(lvl, 4 * V1);
    ASP_TAKE(deps, 8 * V1 * W);
    ASP_TAKE(win, 8 * V1);
    ASP_TAKE(trail, 4 * V1);
    ASP_TAKE(tlim, 4 * R3);
    ASP_TAKE(dec, 4 * R3);
    ASP_TAKE(locc_ptr, 8 * V1);
    ASP_TAKE(locc_n, 8 * V1);
    ASP_TAKE(locc_cap, 8 * V1);
    ASP_TAKE(l_off, 4 * (cap_ng + 1));
    ASP_TAKE(l_lits, 4 * cap_lits);
    const int64_t lists = learning ? (cap_lits < 2 * V1 ? cap_lits : 2 * V1) : Rh + 1;
    L.pool_cap = 4 * cap_lits + 8 * lists;
    ASP_TAKE(pool, 4 * L.pool_cap);
    ASP_TAKE(gpos, 4 * V1);
    ASP_TAKE(reason, 4 * V1);
    ASP_TAKE(mark, 4 * V1);
    ASP_TAKE(resd, 4 * V1);
    ASP_TAKE(act, 4 * V1);
#undef ASP_TAKE
    L.stride = o;
    return L;
}

struct DevStats {
    int64_t rounds, visits, checks, props, decisions, conflicts, learned, learned_len,
            gate_fail, completes;
    uint64_t hash;
    int32_t status, last_step;
    uint64_t t_total, t_round, t_learn, t_decide, t_gate;   // wall-clock ticks
    int64_t models, restarts;
    int32_t exhausted, pad;
};

enum StepKind : int32_t {
    STEP_NONE = 0, STEP_INIT = 1, STEP_ROUND = 2, STEP_LEARN = 3, STEP_DECIDE = 4,
    STEP_COMPLETE = 5, STEP_GATE = 6, STEP_DONE = 7
};

enum Decision : int32_t {
    DECISION_OCC = 0, DECISION_SCORE = 1, DECISION_JW = 2, DECISION_ACTIVITY = 3
};
enum Learning : int32_t { LEARN_FWD = 0, LEARN_RES = 1 };

enum Mode : int32_t {
    MODE_SOLVE = 0,      // workgroup b solves instance order[first + b] to a verdict
    MODE_STEPS = 1,      // instance 0: run up to max_steps steps
    MODE_RESET = 2,      // instance 0: fresh search state
};

// Status values (match asp.h).
enum : int32_t {
    ST_RUNNING = 6, ST_SAT = 1, ST_UNSAT = 2, ST_UNKNOWN = 3,
    ST_E_CAPACITY = -2, ST_E_INTERNAL = -5, ST_E_TIMEOUT = -6
};

struct KArgs {
    const InstDesc* inst;
    const int32_t* order;        // instance ids grouped by LDS class, largest first
    int32_t first, count;        // this launch: order[first .. first+count)
    int32_t mode;
    int32_t pad0;
    const int32_t* ng_off;
    const int32_t* ng_lits;
    const int32_t* map_off;
    const MapEntry* map_ent;
    const int32_t* rule_head;
    const int32_t* rule_occ;
    const int32_t* rule_score;   // score of each rule's head (score-driven Decision)
    const int32_t* rule_ord;     // (rule, head) pairs in the static score's Decision order
    const int32_t* rule_ord_sc;  // (rule, head) pairs in the supplied scores' Decision order
    const int32_t* rb_off;
    const int32_t* rb_lits;
    uint8_t* slots;              // base of the state slots
    const int64_t* slot_off;     // byte offset of each instance's slot
    int32_t* verdicts;
    DevStats* stats;
    uint8_t* models;
    int32_t W, gate_mode;
    int32_t decision;            // DECISION_OCC, _SCORE, _JW or _ACTIVITY
    int32_t fallback_after;      // conflicts in a row before scores give way; <0 never
    int32_t learning;            // LEARN_FWD or LEARN_RES
    int32_t learn_k;             // round conflicts learned per step, 1..8
    int32_t words;               // LDS words per 2-bit map (this launch's largest V)
    int32_t step_mask;           // MODE_STEPS: kinds allowed to run (bit k)
    int64_t max_steps;           // MODE_STEPS: steps to run; MODE_SOLVE: guard
    int64_t max_conflicts;       // <0 unlimited
    int64_t cap_ng, cap_lits;
    uint64_t max_ticks;          // wall-clock guard in s_memrealtime ticks, 0 none
    int64_t max_models;          // answer sets asked for; 0 all, 1 the plain search
    int64_t restart_every;       // conflicts between restarts; 0 never
    int64_t model_store;         // answer sets kept per instance (n_atoms bytes each)
    int32_t lookahead;           // Decision candidates tried by propagation (<= 1: off)
    int32_t awords;              // LDS words of the 1-bit atom map (this launch's largest A)
};

}  // namespace asp
