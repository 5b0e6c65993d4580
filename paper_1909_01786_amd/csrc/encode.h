// encode.h -- host-side program preparation of libasp (internal).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "layout.h"

namespace asp {

// A ground program turned into the data the device search reads.
struct HostProgram {
    int32_t A = 0, Rh = 0, Rc = 0, V = 0;
    int32_t has_empty = 0;
    int32_t u0 = 0, u1 = 0;              // unit nogood ids [u0, u1)
    std::vector<int32_t> ng_off;         // Delta_0 CSR offsets (n+1)
    std::vector<int32_t> ng_lits;
    std::vector<int32_t> map_off;        // 2(V+1)+1
    std::vector<MapEntry> map_ent;       // literal -> nogood entries, ids ascending
    std::vector<int32_t> rule_head;      // per headed rule
    std::vector<int32_t> rule_occ;       // occurrence count of the head in Delta_0
    std::vector<int32_t> rule_jw;        // Jeroslow-Wang score of the head (fixed point)
    // the rules by score, descending, then by rule, ascending, as (rule, head)
    // pairs: the order in which the Decision prefers them under either score
    std::vector<int32_t> rule_by_occ, rule_by_jw;
    std::vector<int32_t> rb_off;         // per headed rule body (deduplicated)
    std::vector<int32_t> rb_lits;
    int64_t n_nogoods() const { return (int64_t)ng_off.size() - 1; }
};

// Validates and encodes; returns 0 or a negative status with *err set.
int encode_program(int32_t n_atoms, int32_t n_rules, const int32_t* head,
                   const int64_t* body_off, const int32_t* body_lits, HostProgram* out,
                   std::string* err);

}  // namespace asp
