// solver.hip -- device search of libasp for gfx950 (CDNA4, wave64).
//
// One workgroup runs one instance's whole conflict-driven search (Alg. 1 of
// the paper): InitialPropagation, PropagateAndCheck rounds (Sect. 4.1),
// Fwd-learning from Deps bitmaps with Backjump (Sect. 4.2), the
// ASP-computation Decision and CompleteAssignment (Sect. 2), and a stability
// check of total assignments.  In the batched form each workgroup solves one
// instance; instances are launched by LDS size class, largest first.
//
// Data placement:
//  * LDS: the assignment as 2 bits per variable (1 = true, 2 = false); the
//    round's winner table (implied variable -> lowest implier, and the values
//    implied for it); scan buffers that spread a round's (literal, nogood)
//    visits over the lanes; a 1-bit atom map for the stability check.
//  * HBM (read-only, per instance): nogood CSR, literal->nogood map CSR,
//    rule table.  Visits read a map segment and then the nogood's literals.
//  * HBM (per instance slot): levels, Deps bitmaps (W x 64 bit per
//    variable), the trail (assigned variables in order, whose tail is the
//    round frontier), the lowest-id implier and the implied values of the
//    variables that do not fit the LDS table, the learned nogoods and their
//    literal occurrence lists.
//
// Control discipline: the search state (decision level, trail pointers, counters,
// status) is a struct that every lane of every wave holds and updates
// identically; it is derived only from values that all lanes see alike (LDS
// words read after a barrier, uniform global loads, block reductions), and
// is pinned to scalar registers with readfirstlane.  No branch of the
// control flow depends on the lane index, so the compiler cannot give lanes
// different paths through the search loop, and single-writer effects are
// identical stores from every lane.
//
// A round is a Jacobi step: every nogood reached from the previous round's
// assignments is classified against the same assignment; among the nogoods
// implying a variable the lowest id wins (its Deps come from it), and a
// unit nogood implying the other value is a conflict.  The conflict kept is
// the shortest (then lowest id) violated or losing nogood.  This makes the
// search deterministic, where the paper's atomicSet picks any thread.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

namespace asp {

#define DEV __device__ __forceinline__

constexpr uint32_t VT = 1u, VF = 2u;          // 2-bit value codes
constexpr unsigned long long WIN_NONE = ~0ull;   // no implier this round
constexpr uint32_t NO_ENTRY = 0xffffffffu;      // implier without a map entry (learned)
constexpr uint64_t FNV_BASIS = 1469598103934665603ull;
constexpr uint64_t FNV_PRIME = 1099511628211ull;
constexpr int kMaxWaves = 16;
constexpr int kFrontCap = 128;   // frontier records kept in LDS (at least; one per thread
                                 // for wider workgroups)
constexpr int kWinBits = 8;
constexpr int kWinCap = 1 << kWinBits;   // LDS winner table (variables implied in a round)
constexpr int kWinProbe = 32;
constexpr int kImplCap = 128;    // LDS implication slots (Deps candidate and record; at
                                 // least, one per thread for wider workgroups)
constexpr uint32_t SLOT_TAG = 0x80000000u;
constexpr int kLitBatch = 4;     // literals of a long nogood loaded together in a visit

// Uniform search state: identical in every lane.
struct Ctl {
    int32_t inst, A, Rh, V, nS, u0, u1, has_empty;
    int32_t cdl, qh, qt, n_learned, pend_kind, pending, status, init_done, last_step, pool_top;
    int32_t use_score, consec, dec_open;   // score-driven Decision and its fallback
    int32_t fr_ok;    // the LDS records describe the frontier trail[qh..qt)
    int32_t epoch;          // resolution-mark epoch (Res-learning)
    int32_t exhausted;      // the search showed no further answer set exists
    int32_t n_pend;         // round conflicts selected for learning (pending, then pend_more)
    int32_t pend_more[7];
    int64_t learned_lits, rounds, props, decisions, conflicts, learned, learned_len, gate_fail,
            completes, steps, visits, checks;
    int64_t models, restarts, since_restart;
    uint64_t hash;
    // device time per step kind (wall-clock ticks; read per wave, so the
    // copies of different waves may differ -- timing only, never control)
    uint64_t t_round, t_learn, t_decide, t_gate;
};

// LDS words through which lanes exchange per-phase results.
struct Scr {
    unsigned long long conf_key;
    unsigned long long conf_key2, conf_thr;   // conflict selection passes
    int32_t tail, clash, changed, pool_top, cap_err, nimpl;
    int32_t flag[kMaxWaves];
    int32_t wsum[kMaxWaves + 1];
    unsigned long long red[kMaxWaves];
};

struct Ctx {
    // per-instance static arrays
    const int32_t *NO, *NL, *MO, *RH, *RO, *RS, *RD, *RDS, *RBO, *RBL;
    const MapEntry* ME;
    // per-slot arrays
    SlotCtrl* ctrl;
    int8_t* val8;
    int32_t *lvl, *trail, *tlim, *dec, *lptr, *ln, *lcap, *loff, *llits, *pool;
    int32_t *gpos, *reason, *mark, *resd;
    int32_t* act;           // activity of each atom (activity Decision)
    unsigned long long* win;
    uint64_t* deps;
    int64_t pool_cap;
    uint32_t* pendb;        // 2-bit pending map past the LDS table (workgroup atomics)
    // LDS
    uint32_t *valb, *lm;
    int32_t* sOff;
    // frontier records: map segment (start, size) and learned occurrence
    // list (start, size) of each frontier variable's true literal, and the
    // variables the current round implies (in trail order)
    int32_t *fS0, *fCs, *fL0, *fCl, *fNew, *fSlot;
    // the round's winner table (variable -> lowest implier key) and the
    // implication slots (W = 1): the Deps of an implier's other variables
    // and the record of the literal it makes true, computed at visit time so
    // that applying the winner reads LDS only
    int32_t *tKey, *tCode;
    unsigned long long *tWin, *iDeps;
    // Deps word of each frontier variable (W = 1), per record; a T-entry
    // buffer (Res-learning's rank tiles)
    unsigned long long *fDeps, *sTile;
    int32_t *iS0, *iCs, *iL0, *iCl;
    unsigned long long* sB;
    Scr* scr;
    int32_t W, T, tid, lane, wid, nw;
    int32_t FC;             // frontier records in LDS: max(T, kFrontCap)
    int32_t IC;             // implication slots in LDS: max(T, kImplCap)
    int32_t decision, fallback_after, learning;
    int32_t ext;            // extended search: several answer sets, restarts, activity,
                            // several conflicts learned per step (compile-time in k_search)
    int32_t multi;          // several conflicts learned per step (compile-time in k_search)
    int32_t learn_k;        // round conflicts learned per step
    int32_t lookahead;      // Decision candidates tried by propagation (extended search)
    unsigned long long my_visits, my_checks;
};

// ------------------------------------------------------------ helpers
DEV void bar() { __syncthreads(); }
DEV int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
DEV int64_t uni64(int64_t x) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

DEV uint32_t vget(const uint32_t* b, int v) { return (b[v >> 4] >> ((v & 15) << 1)) & 3u; }
DEV void vset(uint32_t* b, int v, uint32_t code) { atomicOr(&b[v >> 4], code << ((v & 15) << 1)); }
DEV void vclr(uint32_t* b, int v) { atomicAnd(&b[v >> 4], ~(3u << ((v & 15) << 1))); }
// The pending map lives in the slot (global memory), shared inside the
// workgroup only: workgroup-scope atomics, ordered by the barriers.
DEV uint32_t pend_or(uint32_t* b, int v, uint32_t code) {
    const uint32_t sh = (uint32_t)(v & 15) << 1;
    const uint32_t old = __hip_atomic_fetch_or(&b[v >> 4], code << sh, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
    return (old >> sh) & 3u;
}
DEV uint32_t pend_get(uint32_t* b, int v) {
    return (__hip_atomic_load(&b[v >> 4], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >>
            ((v & 15) << 1)) & 3u;
}
DEV void pend_clr(uint32_t* b, int v) {
    __hip_atomic_fetch_and(&b[v >> 4], ~(3u << ((v & 15) << 1)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}
DEV void pend_zero(uint32_t* b, int i) {
    __hip_atomic_store(&b[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
DEV uint32_t lcode(int l) { return l > 0 ? VT : VF; }     // value making literal l true
DEV int lvar(int l) { return l < 0 ? -l : l; }
DEV int lidx(int l) { return 2 * lvar(l) + (l < 0 ? 1 : 0); }

// The lowest-id implier per variable is shared only inside the workgroup:
// workgroup-scope atomics, ordered by the barriers' workgroup fences.
DEV unsigned long long ld_wg(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
DEV void st_wg(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
DEV void min_wg(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

DEV uint64_t fnv(uint64_t h, int32_t w) {
    uint32_t u = (uint32_t)w;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h ^= (uint64_t)((u >> (8 * q)) & 0xffu);
        h *= FNV_PRIME;
    }
    return h;
}

// Inclusive prefix sum over the 64 lanes of a wave (every lane active), by
// data-parallel-primitive moves: shifts by 1, 2, 4 and 8 lanes inside each
// row of 16 (lanes shifted in from outside the row add 0), then lane 15 of
// rows 0 and 2 added to rows 1 and 3, then lane 31 added to rows 2 and 3.
// Each step is a VALU move, not an LDS round trip.
DEV int wave_incl_scan(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return x;
}
DEV int wave_last(int x) { return __builtin_amdgcn_readlane(x, 63); }

// Block-wide reductions; every lane must call them.
DEV unsigned long long block_max_u64(Ctx& c, unsigned long long x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        unsigned long long y = __shfl_xor(x, d, 64);
        x = x > y ? x : y;
    }
    bar();
    c.scr->red[c.wid] = x;
    bar();
    unsigned long long r = 0;
    for (int i = 0; i < c.nw; ++i) r = r > c.scr->red[i] ? r : c.scr->red[i];
    return (unsigned long long)uni64((int64_t)r);
}

DEV unsigned long long block_sum_u64(Ctx& c, unsigned long long x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    bar();
    c.scr->red[c.wid] = x;
    bar();
    unsigned long long r = 0;
    for (int i = 0; i < c.nw; ++i) r += c.scr->red[i];
    return (unsigned long long)uni64((int64_t)r);
}

DEV int block_min_i32(Ctx& c, int x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        int y = __shfl_xor(x, d, 64);
        x = x < y ? x : y;
    }
    bar();
    c.scr->red[c.wid] = (unsigned long long)(uint32_t)x;
    bar();
    int r = 0x7fffffff;
    for (int i = 0; i < c.nw; ++i) {
        int v = (int)(uint32_t)c.scr->red[i];
        r = r < v ? r : v;
    }
    return uni(r);
}

// Sum of `cnt` and minimum of `mn` over the block, with one pair of barriers.
DEV void block_sum_min(Ctx& c, int cnt, int mn, int* sum_out, int* min_out) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        cnt += __shfl_xor(cnt, d, 64);
        const int y = __shfl_xor(mn, d, 64);
        mn = mn < y ? mn : y;
    }
    bar();
    c.scr->red[c.wid] = ((unsigned long long)(uint32_t)cnt << 32) | (uint32_t)mn;
    bar();
    int sm = 0, m = 0x7fffffff;
    for (int i = 0; i < c.nw; ++i) {
        const unsigned long long r = c.scr->red[i];
        sm += (int)(r >> 32);
        const int v = (int)(uint32_t)r;
        m = m < v ? m : v;
    }
    *sum_out = uni(sm);
    *min_out = uni(m);
}

// OR of a per-wave flag over the block.
DEV int block_any(Ctx& c, int f) {
    bar();
    c.scr->flag[c.wid] = f;
    bar();
    int r = 0;
    for (int i = 0; i < c.nw; ++i) r |= c.scr->flag[i];
    return uni(r);
}

DEV void ng_span(const Ctx& c, const Ctl& k, int id, const int32_t*& p, int& len) {
    if (id < k.nS) {
        int b = c.NO[id];
        p = c.NL + b;
        len = c.NO[id + 1] - b;
    } else {
        int j = id - k.nS;
        int b = c.loff[j];
        p = c.llits + b;
        len = c.loff[j + 1] - b;
    }
}

// Deps bit of the decision at level l >= 2; the last bit stands for every
// level >= 64W.
DEV int level_bit(int l, int W) {
    int b = l - 1, top = 64 * W - 1;
    return b < top ? b : top;
}

// Bits of every decision level 2..cdl, word w.
DEV unsigned long long alldec_word(int w, int cdl, int W) {
    int hi = cdl - 1;
    int top = 64 * W - 1;
    if (hi > top) hi = top;
    if (hi < 1) return 0ull;
    int lo = 1;
    int b0 = 64 * w, b1 = 64 * w + 63;
    int a = lo > b0 ? lo : b0, z = hi < b1 ? hi : b1;
    if (a > z) return 0ull;
    int n = z - a + 1;
    unsigned long long m = n == 64 ? ~0ull : ((1ull << n) - 1ull);
    return m << (a - b0);
}

DEV int tab_hash(int x) { return (int)(((uint32_t)x * 0x9E3779B1u) >> (32 - kWinBits)); }

// Slot of variable x in the round's winner table (inserted if absent;
// `first` is set for the one lane that inserted it); -1 when the probe
// window is full (the global table is used instead).  For a given x every
// lane gets the same answer: entries are never removed during a round, so
// a lane probing for x passes the same occupied slots as the lane that
// inserted it, and a full window stays full.
DEV int tab_insert(Ctx& c, int x, int& first) {
    const int h = tab_hash(x);
    for (int p = 0; p < kWinProbe; ++p) {
        const int sl = (h + p) & (kWinCap - 1);
        const int old = atomicCAS(&c.tKey[sl], -1, x);
        if (old == -1) first = 1;
        if (old == -1 || old == x) return sl;
    }
    return -1;
}

// Slot of x once every insertion of the round is done; -1 if absent.
DEV int tab_find(const Ctx& c, int x) {
    const int h = tab_hash(x);
    for (int p = 0; p < kWinProbe; ++p) {
        const int sl = (h + p) & (kWinCap - 1);
        const int key = c.tKey[sl];
        if (key == x) return sl;
        if (key == -1) return -1;
    }
    return -1;
}

DEV void tab_clear_all(Ctx& c) {
    for (int i = c.tid; i < kWinCap; i += c.T) {
        c.tKey[i] = -1;
        c.tCode[i] = 0;
        c.tWin[i] = WIN_NONE;
    }
}

// --------------------------------------------------------- state moves
DEV void bind_instance(Ctx& c, Ctl& k, const KArgs& a, int inst) {
    const InstDesc& d = a.inst[inst];
    k.inst = inst;
    k.A = uni(d.A);
    k.Rh = uni(d.Rh);
    k.V = uni(d.V);
    k.nS = uni(d.n_static);
    k.u0 = uni(d.u0);
    k.u1 = uni(d.u1);
    k.has_empty = uni(d.has_empty);
    const SlotLayout lay = slot_layout(k.V, k.Rh, a.W, a.cap_ng, a.cap_lits, a.learning);
    uint8_t* slot = a.slots + a.slot_off[inst];
    c.NO = a.ng_off + d.ng_off;
    c.NL = a.ng_lits + d.ng_lits;
    c.MO = a.map_off + d.map_off;
    c.ME = a.map_ent + d.map_ids;
    c.RH = a.rule_head + d.rules;
    c.RO = a.rule_occ + d.rules;
    c.RS = a.rule_score + d.rules;
    c.RD = a.rule_ord + 2 * d.rules;
    c.RDS = a.rule_ord_sc + 2 * d.rules;
    c.RBO = a.rb_off + d.rb_off;
    c.RBL = a.rb_lits + d.rb_lits;
    c.ctrl = (SlotCtrl*)(slot + lay.ctrl);
    c.val8 = (int8_t*)(slot + lay.val8);
    c.pendb = (uint32_t*)(slot + lay.pend);
    c.lvl = (int32_t*)(slot + lay.lvl);
    c.deps = (uint64_t*)(slot + lay.deps);
    c.win = (unsigned long long*)(slot + lay.win);
    c.trail = (int32_t*)(slot + lay.trail);
    c.tlim = (int32_t*)(slot + lay.tlim);
    c.dec = (int32_t*)(slot + lay.dec);
    c.lptr = (int32_t*)(slot + lay.locc_ptr);
    c.ln = (int32_t*)(slot + lay.locc_n);
    c.lcap = (int32_t*)(slot + lay.locc_cap);
    c.loff = (int32_t*)(slot + lay.l_off);
    c.llits = (int32_t*)(slot + lay.l_lits);
    c.pool = (int32_t*)(slot + lay.pool);
    c.gpos = (int32_t*)(slot + lay.gpos);
    c.reason = (int32_t*)(slot + lay.reason);
    c.mark = (int32_t*)(slot + lay.mark);
    c.resd = (int32_t*)(slot + lay.resd);
    c.act = (int32_t*)(slot + lay.act);
    c.pool_cap = lay.pool_cap;
}

// Fresh search state: nothing assigned, no learned nogoods.
DEV void reset_search(Ctx& c, Ctl& k) {
    const int V = k.V, W = c.W, T = c.T, tid = c.tid;
    const int words = (V + 1 + 15) >> 4;
    for (int i = tid; i < words; i += T) {
        c.valb[i] = 0u;
        pend_zero(c.pendb, i);
    }
    for (int i = tid; i < ((k.A + 1 + 31) >> 5); i += T) c.lm[i] = 0u;
    for (int v = tid; v <= V; v += T) {
        c.lvl[v] = 0;
        c.val8[v] = 0;
        st_wg(&c.win[v], WIN_NONE);
        c.mark[v] = 0;
    }
    for (int q = tid; q < (V + 1) * W; q += T) c.deps[q] = 0ull;
    for (int q = tid; q < 2 * (V + 1); q += T) {
        c.ln[q] = 0;
        c.lcap[q] = 0;
        c.lptr[q] = 0;
    }
    for (int w = tid; w < W; w += T) c.sB[w] = 0ull;
    // activities start at the heads' occurrence counts (the static table)
    if (c.ext && c.decision == DECISION_ACTIVITY)
        for (int j = tid; j < k.Rh; j += T) c.act[c.RH[j]] = c.RO[j];
    c.loff[0] = 0;
    k.cdl = 1;
    k.qh = k.qt = 0;
    k.n_learned = 0;
    k.pool_top = 0;
    k.pending = -1;
    k.pend_kind = 0;
    k.status = ST_RUNNING;
    k.init_done = 0;
    k.last_step = STEP_NONE;
    k.learned_lits = 0;
    k.rounds = k.props = k.decisions = k.conflicts = 0;
    k.learned = k.learned_len = k.gate_fail = k.completes = 0;
    k.visits = k.checks = 0;
    k.hash = FNV_BASIS;
    k.steps = 0;
    k.use_score = c.decision == DECISION_SCORE ? 1 : 0;
    k.consec = 0;
    k.dec_open = 0;
    k.t_round = k.t_learn = k.t_decide = k.t_gate = 0;
    k.fr_ok = 0;
    k.epoch = 0;
    k.exhausted = 0;
    k.n_pend = 0;
    k.models = k.restarts = k.since_restart = 0;
    tab_clear_all(c);
    bar();
}

DEV void load_ctrl(Ctx& c, Ctl& k) {
    const int V = k.V, T = c.T, tid = c.tid;
    const int words = (V + 1 + 15) >> 4;
    for (int i = tid; i < words; i += T) pend_zero(c.pendb, i);
    for (int i = tid; i < ((k.A + 1 + 31) >> 5); i += T) c.lm[i] = 0u;
    for (int i = tid; i < words; i += T) {
        uint32_t wv = 0;
        for (int q = 0; q < 16; ++q) {
            int v = i * 16 + q;
            if (v > V) break;
            int8_t x = c.val8[v];
            uint32_t code = x > 0 ? VT : (x < 0 ? VF : 0u);
            wv |= code << (2 * q);
        }
        c.valb[i] = wv;
    }
    for (int w = tid; w < c.W; w += T) c.sB[w] = c.ctrl->pend_B[w];
    const SlotCtrl& g = *c.ctrl;
    k.cdl = uni(g.cdl);
    k.qh = uni(g.qh);
    k.qt = uni(g.qt);
    k.n_learned = uni(g.n_learned);
    k.pool_top = uni(g.pool_top);
    k.pending = uni(g.pending);
    k.pend_kind = uni(g.pend_kind);
    k.status = uni(g.status);
    k.init_done = uni(g.init_done);
    k.last_step = uni(g.last_step);
    k.learned_lits = uni64(g.learned_lits);
    k.rounds = uni64(g.rounds);
    k.visits = uni64(g.visits);
    k.checks = uni64(g.checks);
    k.props = uni64(g.props);
    k.decisions = uni64(g.decisions);
    k.conflicts = uni64(g.conflicts);
    k.learned = uni64(g.learned);
    k.learned_len = uni64(g.learned_len);
    k.gate_fail = uni64(g.gate_fail);
    k.completes = uni64(g.completes);
    k.hash = (uint64_t)uni64((int64_t)g.hash);
    k.use_score = uni(g.use_score);
    k.consec = uni(g.consec);
    k.dec_open = uni(g.dec_open);
    k.epoch = uni(g.epoch);
    k.exhausted = uni(g.exhausted);
    k.n_pend = uni(g.n_pend);
    for (int i = 0; i < 7; ++i) k.pend_more[i] = uni(g.pend_more[i]);
    k.models = uni64(g.models);
    k.restarts = uni64(g.restarts);
    k.since_restart = uni64(g.since_restart);
    k.steps = 0;
    k.t_round = k.t_learn = k.t_decide = k.t_gate = 0;
    k.fr_ok = 0;
    tab_clear_all(c);
    bar();
}

// Fold every lane's visit and check counts into the uniform state.
DEV void flush_counters(Ctx& c, Ctl& k) {
    k.visits += (int64_t)block_sum_u64(c, c.my_visits);
    k.checks += (int64_t)block_sum_u64(c, c.my_checks);
    c.my_visits = c.my_checks = 0ull;
    bar();
}

// Every lane stores the same control values (identical stores).
DEV void save_ctrl(Ctx& c, const Ctl& k) {
    const int V = k.V, T = c.T, tid = c.tid;
    for (int v = tid; v <= V; v += T) {
        uint32_t code = vget(c.valb, v);
        c.val8[v] = code == VT ? (int8_t)1 : (code == VF ? (int8_t)-1 : (int8_t)0);
    }
    for (int w = tid; w < c.W; w += T) c.ctrl->pend_B[w] = c.sB[w];
    SlotCtrl& g = *c.ctrl;
    g.inst = k.inst;
    g.cdl = k.cdl;
    g.qh = k.qh;
    g.qt = k.qt;
    g.n_learned = k.n_learned;
    g.pool_top = k.pool_top;
    g.pending = k.pending;
    g.pend_kind = k.pend_kind;
    g.status = k.status;
    g.init_done = k.init_done;
    g.last_step = k.last_step;
    g.learned_lits = k.learned_lits;
    g.rounds = k.rounds;
    g.visits = k.visits;
    g.checks = k.checks;
    g.props = k.props;
    g.decisions = k.decisions;
    g.conflicts = k.conflicts;
    g.learned = k.learned;
    g.learned_len = k.learned_len;
    g.gate_fail = k.gate_fail;
    g.completes = k.completes;
    g.hash = k.hash;
    g.use_score = k.use_score;
    g.consec = k.consec;
    g.dec_open = k.dec_open;
    g.epoch = k.epoch;
    g.exhausted = k.exhausted;
    g.n_pend = k.n_pend;
    for (int i = 0; i < 7; ++i) g.pend_more[i] = k.pend_more[i];
    g.models = k.models;
    g.restarts = k.restarts;
    g.since_restart = k.since_restart;
    bar();
}

// ------------------------------------------------------------- steps
// InitialPropagation (Alg. 1): each unit nogood {l} -- the static ones and,
// after a restart, the learned ones -- assigns the complement of l at level
// 1 with empty Deps; opposite units, or an empty learned nogood, mean no
// answer set.
DEV void step_init(Ctx& c, Ctl& k) {
    const int T = c.T, tid = c.tid;
    c.scr->clash = k.has_empty;
    c.scr->tail = k.qt;
    bar();
    if (!k.has_empty) {
        const int nu = k.u1 - k.u0;
        for (int q = tid; q < nu + k.n_learned; q += T) {
            int l;
            if (q < nu) {
                l = c.NL[c.NO[k.u0 + q]];
            } else {
                const int o = c.loff[q - nu], len = c.loff[q - nu + 1] - o;
                if (len == 0) c.scr->clash = 1;
                if (len != 1) continue;
                l = c.llits[o];
            }
            int x = lvar(l);
            uint32_t code = l > 0 ? VF : VT;
            const uint32_t ob = pend_or(c.pendb, x, code);
            if (ob == 0u) {
                int pos = atomicAdd(&c.scr->tail, 1);
                c.trail[pos] = x;
            } else if ((ob | code) == 3u) {
                c.scr->clash = 1;
            }
        }
    }
    bar();
    const int q0 = k.qt;
    const int q1 = uni(c.scr->tail);
    const int clash = uni(c.scr->clash);
    if (!clash) {
        for (int i = q0 + tid; i < q1; i += T) {
            int x = c.trail[i];
            uint32_t code = pend_get(c.pendb, x);
            vset(c.valb, x, code);
            if (c.learning == LEARN_RES) {
                c.lvl[x] = 1;
                c.gpos[x] = q0;
                c.reason[x] = -1;    // never resolved: conflicts at level 1 mean UNSAT
            }
        }
    }
    bar();
    for (int i = q0 + tid; i < q1; i += T) pend_clr(c.pendb, c.trail[i]);
    bar();
    k.init_done = 1;
    if (clash) {
        k.status = ST_UNSAT;
    } else {
        k.qh = q0;
        k.qt = q1;
    }
    k.fr_ok = 0;
}

// Frontier record i for variable x taking value `code` with Deps word d0:
// where the visits of its now-true literal are (static map segment,
// learned occurrence list).
DEV void put_record(Ctx& c, int i, int x, uint32_t code, unsigned long long d0) {
    const int li = 2 * x + (code == VF ? 1 : 0);
    const int s0 = c.MO[li];
    c.fS0[i] = s0;
    c.fCs[i] = c.MO[li + 1] - s0;
    c.fL0[i] = c.lptr[li];
    c.fCl[i] = c.ln[li];
    c.fDeps[i] = d0;
}

// Classification of one visited nogood against the round's snapshot.  A
// short static nogood comes with its map entry, whose other literals are
// all that must be read (the map's own literal is true in the snapshot);
// any other nogood is read through the nogood arrays.
// pass 0: record violations and unit implications (winner key: id and
// implied value, then the map entry the Deps will be read from); pass 1:
// conflicts of unit nogoods that lost their variable to a lower-id implier
// of the other value.
DEV void visit_one(Ctx& c, const Ctl& k, int id, const MapEntry& e, uint32_t eidx,
                   unsigned long long selfd, int pass) {
    int len, open = 0, u = 0;
    const bool inl = e.o1 != kLongNogood;
    const int32_t* lits = nullptr;
    if (inl) {
        const int o1 = e.o1, o2 = e.o2;
        len = 1 + (o1 != 0 ? 1 : 0) + (o2 != 0 ? 1 : 0);
        if (pass == 0) {
            c.my_visits += 1ull;
            c.my_checks += (unsigned long long)len;
        }
        if (o1 != 0) {
            const uint32_t s = vget(c.valb, lvar(o1));
            if (s == 0u) { open = 1; u = o1; }
            else if (s != lcode(o1)) return;   // satisfied
        }
        if (o2 != 0) {
            const uint32_t s = vget(c.valb, lvar(o2));
            if (s == 0u) { if (++open > 1) return; u = o2; }
            else if (s != lcode(o2)) return;
        }
    } else {
        eidx = NO_ENTRY;
        if (id < k.nS) {
            // a long static nogood: its map entry locates its literals
            lits = c.NL + e.o2;
            len = e.a1;
        } else {
            ng_span(c, k, id, lits, len);
        }
        if (pass == 0) {
            c.my_visits += 1ull;
            c.my_checks += (unsigned long long)len;
        }
        // from the last literal back, kLitBatch loads in flight: a learned
        // nogood holds its newest literal last, the one most likely to be
        // open or false after a backjump (the outcome -- violated, unit on
        // one literal, or neither -- does not depend on the order)
        for (int q = len; q > 0; q -= kLitBatch) {
            int l[kLitBatch];
#pragma unroll
            for (int j = 0; j < kLitBatch; ++j) l[j] = j < q ? lits[q - 1 - j] : 0;
#pragma unroll
            for (int j = 0; j < kLitBatch; ++j) {
                if (j >= q) break;
                const uint32_t s = vget(c.valb, lvar(l[j]));
                if (s == 0u) {
                    if (++open > 1) return;
                    u = l[j];
                } else if (s != lcode(l[j])) {
                    return;  // satisfied
                }
            }
        }
    }
    // a conflict's key: pass 0 and 1 keep the smallest; a selection pass
    // (2) the smallest above the keys already selected
    auto note = [&](unsigned long long key) {
        if (pass != 2) atomicMin(&c.scr->conf_key, key);
        else if (key > c.scr->conf_thr) atomicMin(&c.scr->conf_key2, key);
    };
    if (open == 0) {
        if (pass != 1) note(((unsigned long long)(uint32_t)len << 32) | (uint32_t)id);
        return;
    }
    const int x = lvar(u);
    const uint32_t code = u > 0 ? VF : VT;   // implied value of x
    if (pass == 0) {
        const uint32_t hi = (uint32_t)(id * 2 + (code == VF ? 1 : 0));
        uint32_t lo = eidx;
        // W = 1: the Deps this implication would give x (the snapshot's Deps
        // of the nogood's other variables) and the record of the literal it
        // makes true, kept in a slot in case this implier wins (the map
        // literal's variable is the frontier variable: its Deps come with
        // the frontier; a short nogood's entry holds the map segment of each
        // literal it can make true; under Fwd-learning learned occurrence
        // lists exist only for decision literals T b_r -- and, when answer
        // sets are blocked, atoms T p -- under Res-learning for literals of
        // either sign).  Their global reads are issued first; the LDS
        // atomics that follow (x's winner-table entry, the slot) overlap them.
        unsigned long long dA = 0ull, dB = 0ull;
        int s0 = 0, s1 = 0, l0 = 0, cl = 0;
        const bool dec_lit = c.learning == LEARN_RES || (c.ext && code == VT) ||
                             (code == VT && x > k.A && (x - k.A - 1) % 3 == 0);
        if (c.W == 1) {
            if (inl) {
                if (e.o1 != 0 && lvar(e.o1) != x) dA = c.deps[lvar(e.o1)];
                if (e.o2 != 0 && lvar(e.o2) != x) dB = c.deps[lvar(e.o2)];
            } else {
                for (int q = 0; q < len; ++q) {
                    const int y = lvar(lits[q]);
                    if (y != x) dA |= c.deps[y];
                }
                const int li = 2 * x + (code == VF ? 1 : 0);
                s0 = c.MO[li];
                s1 = c.MO[li + 1];
            }
            if (dec_lit) {
                const int lli = 2 * x + (code == VF ? 1 : 0);
                l0 = c.lptr[lli];
                cl = c.ln[lli];
            }
        }
        int first = 0;
        const int t = tab_insert(c, x, first);
        const int sl = c.W == 1 ? atomicAdd(&c.scr->nimpl, 1) : c.IC;
        if (sl < c.IC) {
            if (inl) {
                s0 = u == e.o1 ? e.a1 : e.a2;
                s1 = s0 + (u == e.o1 ? e.n1 : e.n2);
            }
            c.iDeps[sl] = (inl ? selfd : 0ull) | dA | dB;
            c.iS0[sl] = s0;
            c.iCs[sl] = s1 - s0;
            c.iL0[sl] = l0;
            c.iCl[sl] = cl;
            lo = SLOT_TAG | (uint32_t)sl;
        }
        const unsigned long long key = ((unsigned long long)hi << 32) | lo;
        // x joins the round's implied variables (the trail) with its first
        // implier; both values implied for x in one round is a clash.  In
        // the LDS table the first implier is the lane that inserted x, and
        // the values seen are OR-ed into the entry's code; past the table,
        // the pending map plays both parts.
        int append = 0;
        if (t >= 0) {
            atomicMin(&c.tWin[t], key);
            const uint32_t oc = (uint32_t)atomicOr(&c.tCode[t], (int)code);
            if ((oc | code) == 3u) c.scr->clash = 1;
            append = first;
        } else {
            min_wg(&c.win[x], key);
            const uint32_t ob = pend_or(c.pendb, x, code);
            if (ob == 0u) append = 1;
            else if ((ob | code) == 3u) c.scr->clash = 1;
        }
        if (append) {
            const int pos = atomicAdd(&c.scr->tail, 1);
            c.trail[pos] = x;
            if (pos - k.qt < c.FC) {
                c.fNew[pos - k.qt] = x;
                c.fSlot[pos - k.qt] = t;
            }
        }
    } else {
        const int t = tab_find(c, x);
        const unsigned long long key = t >= 0 ? c.tWin[t] : ld_wg(&c.win[x]);
        const uint32_t wcode = ((key >> 32) & 1ull) ? VF : VT;
        if (wcode != code) note(((unsigned long long)(uint32_t)len << 32) | (uint32_t)id);
    }
}

// Spread the visits of frontier trail[qh..qt) over the block: each frontier
// variable contributes its static map segment and its learned occurrence
// list; a scan of the segment sizes gives each lane its visits.  The
// frontier is taken in chunks of T variables, whose records
// (map segment, learned list, Deps word) the visits read from the LDS
// frontier records: left there by whoever made the frontier, or, when
// they were not (fr_ok clear), computed into them for the chunk.
DEV void visit_pass(Ctx& c, const Ctl& k, int qh, int qt, int pass) {
    const int T = c.T, tid = c.tid;
    const int C = T;   // <= c.FC
    for (int base = qh; base < qt; base += C) {
        const int f = base + tid;
        const int rb = k.fr_ok ? base - qh : 0;   // the chunk's first record
        int cs = 0, cl = 0;
        if (tid < C && f < qt) {
            if (k.fr_ok) {
                cs = c.fCs[rb + tid];
                cl = c.fCl[rb + tid];
            } else {
                const int v = c.trail[f];
                const int L = vget(c.valb, v) == VT ? v : -v;
                const int li = lidx(L);
                const int s0 = c.MO[li];
                cs = c.MO[li + 1] - s0;
                cl = c.ln[li];
                c.fS0[tid] = s0;
                c.fCs[tid] = cs;
                c.fL0[tid] = c.lptr[li];
                c.fDeps[tid] = c.deps[(size_t)v * c.W];
            }
        }
        // wave-local exclusive offsets of the visit counts, and the wave
        // totals: one barrier makes every visit's position known
        const int cnt_all = cs + cl;
        const int inc = wave_incl_scan(cnt_all);
        c.sOff[tid] = inc - cnt_all;
        c.scr->wsum[c.wid] = wave_last(inc);   // identical from the wave's lanes
        bar();
        const int nf = (qt - base) < C ? (qt - base) : C;
        const int nwv = (nf + 63) >> 6;
        int total = 0;
        for (int w = 0; w < nwv; ++w) total += c.scr->wsum[w];
        total = uni(total);
        for (int q = tid; q < total; q += T) {
            // the wave whose lanes hold visit q, then the lane within it
            int w = 0, wb = 0;
            while (w + 1 < nwv && wb + c.scr->wsum[w] <= q) {
                wb += c.scr->wsum[w];
                ++w;
            }
            // the last of the wave's 64 start offsets that is <= qq (they
            // ascend; lanes past the frontier hold the wave total, > qq):
            // count the offsets <= qq among every eighth, then among the
            // eight of that group -- two rounds of independent LDS reads
            const int qq = q - wb;
            const int32_t* so = c.sOff + w * 64;
            int g = 0;
#pragma unroll
            for (int m = 1; m < 8; ++m) g += so[8 * m] <= qq ? 1 : 0;
            int r = 0;
#pragma unroll
            for (int m = 1; m < 8; ++m) r += so[8 * g + m] <= qq ? 1 : 0;
            const int lo = w * 64 + 8 * g + r;
            const int j = qq - c.sOff[lo];
            const int ri = rb + lo;
            const int cnt = c.fCs[ri];
            if (j < cnt) {
                const uint32_t eidx = (uint32_t)(c.fS0[ri] + j);
                const MapEntry e = c.ME[eidx];
                visit_one(c, k, e.id, e, eidx, c.fDeps[ri], pass);
            } else {
                const MapEntry none{0, 0, kLongNogood, 0, 0, 0, 0, 0};
                visit_one(c, k, c.pool[c.fL0[ri] + (j - cnt)], none, NO_ENTRY, c.fDeps[ri], pass);
            }
        }
        bar();
    }
}

// One PropagateAndCheck round (Sect. 4.1, Alg. 2) in Jacobi form.
DEV void step_round(Ctx& c, Ctl& k) {
    const int T = c.T, tid = c.tid, W = c.W;
    const int qh = k.qh, qt = k.qt, cdl = k.cdl;
    c.scr->conf_key = ~0ull;
    c.scr->clash = 0;
    c.scr->tail = qt;
    c.scr->nimpl = 0;
    bar();
    visit_pass(c, k, qh, qt, 0);
    bar();
    if (uni(c.scr->clash)) {
        visit_pass(c, k, qh, qt, 1);
        bar();
    }
    // several conflicts learned per step: the next smallest keys, one
    // selection pass each, on the same snapshot and winners
    int nsel = 1;
    if (c.multi && c.learn_k > 1) {
        unsigned long long thr = (unsigned long long)uni64((int64_t)c.scr->conf_key);
        for (int r = 1; r < c.learn_k && thr != ~0ull; ++r) {
            c.scr->conf_key2 = ~0ull;       // identical from every lane
            c.scr->conf_thr = thr;
            bar();
            visit_pass(c, k, qh, qt, 2);    // ends with a barrier
            thr = (unsigned long long)uni64((int64_t)c.scr->conf_key2);
            bar();                          // every lane has read it
            if (thr == ~0ull) break;
            k.pend_more[r - 1] = (int32_t)(uint32_t)(thr & 0xffffffffull);
            nsel += 1;
        }
    }
    const int nt = uni(c.scr->tail);
    // apply every implication, its Deps being the OR of the Deps of the
    // other variables of the winning nogood (mk_dl_bitmap).  The implied
    // variables come from LDS when they fit (with their winner-table
    // entries, recorded by the lanes that appended them), and so does the
    // winner: its key from the LDS table, its Deps and frontier record from
    // its slot; the apply also writes the next round's frontier records.
    // When the implied variables fit, no lane searches the table here, so
    // each lane empties the entries it has read.
    const bool rec = nt - qt <= c.FC;
    for (int i = qt + tid; i < nt; i += T) {
        const int x = rec ? c.fNew[i - qt] : c.trail[i];
        const int t = rec ? c.fSlot[i - qt] : tab_find(c, x);
        unsigned long long key;
        if (t >= 0) {
            key = c.tWin[t];
            if (rec) {
                c.tKey[t] = -1;
                c.tCode[t] = 0;
                c.tWin[t] = WIN_NONE;
            }
        } else {
            key = ld_wg(&c.win[x]);
            st_wg(&c.win[x], WIN_NONE);
        }
        const int id = (int)(key >> 33);
        const uint32_t code = ((key >> 32) & 1ull) ? VF : VT;
        const uint32_t lo = (uint32_t)key;
        uint64_t* dx = c.deps + (size_t)x * W;
        if (lo != NO_ENTRY && (lo & SLOT_TAG)) {
            const int sl = (int)(lo & ~SLOT_TAG);
            const unsigned long long d0 = c.iDeps[sl];
            dx[0] = d0;
            if (rec) {
                c.fS0[i - qt] = c.iS0[sl];
                c.fCs[i - qt] = c.iCs[sl];
                c.fL0[i - qt] = c.iL0[sl];
                c.fCl[i - qt] = c.iCl[sl];
                c.fDeps[i - qt] = d0;
            }
        } else {
            // OR of the Deps of the winner's other variables; a short static
            // nogood's literals are in its map entry (0 marks an absent one)
            auto each_other = [&](auto&& add) {
                if (lo != NO_ENTRY) {
                    const MapEntry e = c.ME[lo];
                    add(lvar(e.self));
                    add(lvar(e.o1));
                    add(lvar(e.o2));
                } else {
                    const int32_t* lits;
                    int len;
                    ng_span(c, k, id, lits, len);
                    for (int q = 0; q < len; ++q) add(lvar(lits[q]));
                }
            };
            if (W == 1) {
                unsigned long long acc = 0ull;
                each_other([&](int y) {
                    if (y != 0 && y != x) acc |= c.deps[y];
                });
                dx[0] = acc;
            } else {
                for (int w = 0; w < W; ++w) dx[w] = 0ull;
                each_other([&](int y) {
                    if (y == 0 || y == x) return;
                    const uint64_t* dy = c.deps + (size_t)y * W;
                    for (int w = 0; w < W; ++w) dx[w] |= dy[w];
                });
            }
            if (rec) put_record(c, i - qt, x, code, dx[0]);
        }
        if (c.learning == LEARN_RES) {
            c.lvl[x] = cdl;
            c.gpos[x] = qt;
            c.reason[x] = id;
        }
        vset(c.valb, x, code);
        if (t < 0) pend_clr(c.pendb, x);   // only variables past the table use the pending map
    }
    bar();
    const unsigned long long ck = (unsigned long long)uni64((int64_t)c.scr->conf_key);
    // the winner table is empty again for the next round
    if (!rec) tab_clear_all(c);
    // (the step loop's barrier orders the table clearing before the next use)
    k.qh = qt;
    k.qt = nt;
    k.fr_ok = rec ? 1 : 0;
    k.rounds += 1;
    k.props += nt - qt;
    if (ck != ~0ull) {
        k.pending = (int32_t)(uint32_t)(ck & 0xffffffffull);
        k.pend_kind = 1;
        k.n_pend = nsel;
    }
}

// Res-learning (Alg. 3) of round conflict `conf` at level `top`,
// resolution to the first UIP.  The trail is walked back one assigning step
// at a time (a round, a decision, an assertion, a CompleteAssignment; gpos
// gives the trail position where a variable's step begins, so (gpos,
// variable) orders the assigned variables as they were assigned, and an
// implying nogood's other variables come from earlier steps).  The marked
// variables of one step all sit at the top level: every one but the lowest
// numbered is resolved away with the nogood that implied it (none of them
// can be the last marked variable at the top level), and the lowest
// numbered is the UIP when it is the only marked variable left there, else
// it is resolved too.  Writes the nogood's literals (true now) ordered by
// (gpos, variable), the UIP last, to the learned store at `base`.  Returns
// 1; 0 when a variable to resolve has no implying nogood (a
// CompleteAssignment literal: the caller learns by Fwd-learning); -1 when
// the learned store is full; -2 on a broken invariant.
DEV int res_learn(Ctx& c, Ctl& k, const KArgs& a, int conf, int base, int top, int* nN_out,
                  int* bj_out) {
    const int T = c.T, tid = c.tid;
    const int ep = k.epoch + 1;
    k.epoch = ep;
    const int32_t* lits;
    int len;
    ng_span(c, k, conf, lits, len);
    c.scr->tail = len;                         // identical from every lane
    unsigned long long at_top = 0ull;
    for (int q = tid; q < len; q += T) {
        const int v = lvar(lits[q]);
        c.mark[v] = ep;
        c.resd[q] = v;
        at_top += c.lvl[v] == top ? 1ull : 0ull;
    }
    int ntop = (int)block_sum_u64(c, at_top);  // (its barriers order the marks)
    int p = k.qt - 1, uip = -1;
    while (uip < 0) {
        if (p < 0) return -2;
        // the latest marked variable at or below p, T trail positions at a time
        {
            const int i = p - tid;
            const int hm = (int)block_max_u64(
                c, (i >= 0 && c.mark[c.trail[i]] == ep) ? (unsigned long long)(i + 1) : 0ull);
            if (hm == 0) {
                p -= T;
                continue;
            }
            p = hm - 1;
        }
        const int g0 = uni(c.gpos[uni(c.trail[p])]);
        // the marked variables of the step trail[g0..p]: how many, the lowest
        int cnt = 0, mn = 0x7fffffff;
        for (int i = g0 + tid; i <= p; i += T) {
            const int v = c.trail[i];
            if (c.mark[v] == ep) {
                cnt += 1;
                mn = v < mn ? v : mn;
            }
        }
        int m;
        block_sum_min(c, cnt, mn, &m, &mn);
        c.scr->clash = 0;                      // set: a variable without implying nogood
        c.scr->nimpl = 0;                      // newly marked variables at the top level
        bar();
        if (m > 1) {
            for (int i = g0 + tid; i <= p; i += T) {
                const int v = c.trail[i];
                if (v == mn || c.mark[v] != ep) continue;
                const int e = c.reason[v];
                if (e < 0) {
                    c.scr->clash = 1;
                    continue;
                }
                c.mark[v] = 0;
                const int32_t* E;
                int elen;
                ng_span(c, k, e, E, elen);
                for (int q = 0; q < elen; ++q) {
                    const int w = lvar(E[q]);
                    if (w == v || atomicExch(&c.mark[w], ep) == ep) continue;
                    c.resd[atomicAdd(&c.scr->tail, 1)] = w;
                    if (c.lvl[w] == top) atomicAdd(&c.scr->nimpl, 1);
                }
            }
            bar();
            if (uni(c.scr->clash)) return 0;
            ntop += uni(c.scr->nimpl) - (m - 1);
        }
        if (ntop == 1) {
            uip = mn;
            break;
        }
        // the lowest numbered is resolved too, the block over its nogood
        const int e = uni(c.reason[mn]);
        if (e < 0) return 0;
        bar();
        c.scr->nimpl = 0;
        c.mark[mn] = 0;                        // identical from every lane
        bar();
        const int32_t* E;
        int elen;
        ng_span(c, k, e, E, elen);
        for (int q = tid; q < elen; q += T) {
            const int w = lvar(E[q]);
            if (w == mn || atomicExch(&c.mark[w], ep) == ep) continue;
            c.resd[atomicAdd(&c.scr->tail, 1)] = w;
            if (c.lvl[w] == top) atomicAdd(&c.scr->nimpl, 1);
        }
        bar();
        ntop += uni(c.scr->nimpl) - 1;
        if (ntop < 1) return -2;
        p = g0 - 1;
    }
    // the live (still marked) variables, compacted in place chunk by chunk
    // (a chunk is read before any of it is overwritten; writes stay below
    // the next chunk), and the highest level among them but the UIP's
    const int n = uni(c.scr->tail);
    bar();
    c.scr->nimpl = 0;
    bar();
    unsigned long long mk = 0ull;
    for (int b = 0; b < n; b += T) {
        const int i = b + tid;
        const int v = i < n ? c.resd[i] : 0;
        const bool live = i < n && c.mark[v] == ep;
        bar();
        if (live) {
            c.resd[atomicAdd(&c.scr->nimpl, 1)] = v;
            if (v != uip) {
                const unsigned long long l = (unsigned long long)c.lvl[v];
                mk = l > mk ? l : mk;
            }
        }
    }
    const int kk = (int)block_max_u64(c, mk);
    const int nN = uni(c.scr->nimpl);
    if (k.n_learned + 1 > a.cap_ng || k.learned_lits + nN > a.cap_lits) return -1;
    // each live variable's rank by (gpos, variable), counted against tiles
    // of the keys staged in LDS
    unsigned long long* tile = c.sTile;
    for (int r = 0; r < nN; r += T) {
        const int i = r + tid;
        const int v = i < nN ? c.resd[i] : 0;
        const unsigned long long kv =
            i < nN ? (((unsigned long long)(uint32_t)c.gpos[v] << 32) | (uint32_t)v) : ~0ull;
        int rank = 0;
        for (int t0 = 0; t0 < nN; t0 += T) {
            bar();
            const int j = t0 + tid;
            if (j < nN) {
                const int w = c.resd[j];
                tile[tid] = ((unsigned long long)(uint32_t)c.gpos[w] << 32) | (uint32_t)w;
            } else {
                tile[tid] = ~0ull;
            }
            bar();
            const int nt = nN - t0 < T ? nN - t0 : T;
            for (int jj = 0; jj < nt; ++jj) rank += tile[jj] < kv ? 1 : 0;
        }
        if (i < nN) c.llits[base + rank] = vget(c.valb, v) == VT ? v : -v;
    }
    bar();
    *nN_out = nN;
    *bj_out = kk > 1 ? kk : 1;
    return 1;
}

// Literal occurrence lists of a new learned nogood llits[base..base+nN)
// (one lane per literal; the literals are distinct): doubling arrays in the
// slot's pool, claimed from scr->pool_top; an overflow sets scr->cap_err.
DEV void add_occurrences(Ctx& c, int base, int nN, int newid) {
    for (int i = c.tid; i < nN; i += c.T) {
        int li = lidx(c.llits[base + i]);
        int n = c.ln[li], cap = c.lcap[li], p = c.lptr[li];
        if (n == cap) {
            int ncap = cap ? 2 * cap : 4;
            int np = atomicAdd(&c.scr->pool_top, ncap);
            if ((int64_t)np + ncap > c.pool_cap) {
                c.scr->cap_err = 1;
                continue;
            }
            for (int q = 0; q < n; ++q) c.pool[np + q] = c.pool[p + q];
            c.lptr[li] = np;
            c.lcap[li] = ncap;
            p = np;
        }
        c.pool[p + n] = newid;
        c.ln[li] = n + 1;
    }
}

// Restart: every assigned variable (the trail) is unassigned, the learned
// nogoods stay, and InitialPropagation runs next.
DEV void restart(Ctx& c, Ctl& k) {
    const int W = c.W, T = c.T, tid = c.tid;
    const int words = (k.V + 1 + 15) >> 4;
    for (int i = tid; i < words; i += T) c.valb[i] = 0u;
    for (int i = tid; i < k.qt; i += T) {
        const int v = c.trail[i];
        if (c.learning == LEARN_RES) c.lvl[v] = 0;
        for (int w = 0; w < W; ++w) c.deps[(size_t)v * W + w] = 0ull;
    }
    for (int w = tid; w < W; w += T) c.sB[w] = 0ull;
    k.cdl = 1;
    k.qh = k.qt = 0;
    k.pending = -1;
    k.pend_kind = 0;
    k.n_pend = 0;
    k.init_done = 0;
    k.fr_ok = 0;
    k.since_restart = 0;
    k.restarts += 1;
    k.hash = fnv(k.hash, 9);
    bar();
}

// B of a round conflict -- the OR of the Deps of its variables -- into sB.
DEV void conflict_B(Ctx& c, Ctl& k, int conf) {
    const int T = c.T, tid = c.tid, W = c.W;
    for (int w = tid; w < W; w += T) c.sB[w] = 0ull;
    bar();
    const int32_t* lits;
    int len;
    ng_span(c, k, conf, lits, len);
    for (int q = tid; q < len * W; q += T) {
        int i = q / W, w = q - i * W;
        unsigned long long d = c.deps[(size_t)lvar(lits[i]) * W + w];
        if (d) atomicOr(&c.sB[w], d);
    }
    bar();
}

// The reading of B (W words in sB), identical in every lane: empty, the
// saturated bit, the two highest level bits below it, the bit count.
struct BRead {
    bool zero, sat;
    int hi1, hi2, npop;
};
DEV BRead read_B(Ctx& c) {
    const int W = c.W;
    bool zero = true, sat = false;
    int hi1 = -1, hi2 = -1, npop = 0;
    for (int w = W - 1; w >= 0; --w) {
        unsigned long long x = c.sB[w];
        zero = zero && x == 0ull;
        if (w == W - 1) {
            sat = (x >> 63) & 1ull;
            x &= ~(1ull << 63);
        }
        if (w == 0) x &= ~1ull;
        npop += __popcll(x);
        while (x && hi2 < 0) {
            int b = 63 - __clzll((long long)x);
            int idx = w * 64 + b;
            if (hi1 < 0) hi1 = idx; else hi2 = idx;
            x &= ~(1ull << b);
        }
    }
    BRead r;
    r.zero = uni(zero ? 1 : 0) != 0;
    r.sat = uni(sat ? 1 : 0) != 0;
    r.hi1 = uni(hi1);
    r.hi2 = uni(hi2);
    r.npop = uni(npop);
    return r;
}

// The highest level among a round conflict's literals.
DEV int conflict_top(Ctx& c, Ctl& k, int conf) {
    const int32_t* lits;
    int len;
    ng_span(c, k, conf, lits, len);
    unsigned long long mx = 0ull;
    for (int q = c.tid; q < len; q += c.T) {
        const unsigned long long l = (unsigned long long)c.lvl[lvar(lits[q])];
        mx = l > mx ? l : mx;
    }
    return (int)block_max_u64(c, mx);
}

// The nogood learned from one conflict -- conf >= 0 a round conflict, -1
// the gate's (its B in sB) -- written to the learned store at `base`:
// Res-learning (Alg. 3) when selected, else (and when resolution reaches a
// literal without implying nogood) Fwd-learning (Sect. 4.2, Alg. 4), the
// decision literal of every level in levels(B) by increasing level.
// have_B: sB already holds conf's B; ctop: the conflict's highest level,
// or -1 to compute it.  Returns 0, or the status that ends the search.
DEV int learn_one(Ctx& c, Ctl& k, const KArgs& a, int conf, bool have_B, int ctop, int base,
                  int* nN_out, int* bj_out) {
    const int T = c.T, tid = c.tid, W = c.W;
    const int cdl = k.cdl;
    if (conf >= 0 && c.learning == LEARN_RES) {
        if (ctop < 0) ctop = conflict_top(c, k, conf);
        const int got = res_learn(c, k, a, conf, base, ctop, nN_out, bj_out);
        if (got < 0) return got == -1 ? ST_UNKNOWN : ST_E_INTERNAL;
        if (got) return 0;
        have_B = false;
    }
    if (conf >= 0 && !have_B) conflict_B(c, k, conf);
    const BRead b = read_B(c);
    int topl, bj, nN;
    if (b.sat) {
        topl = cdl;
        bj = (cdl - 1 >= 64 * W) ? cdl - 1 : (b.hi1 >= 0 ? b.hi1 + 1 : 1);
        nN = b.npop + (cdl - 64 * W + 1);
    } else {
        topl = b.hi1 + 1;
        bj = b.hi2 >= 0 ? b.hi2 + 1 : 1;
        nN = b.npop;
    }
    // Deps naming a level above cdl would be a broken invariant
    if (b.hi1 + 1 > cdl || (b.sat && cdl < 64 * W) || topl < 2) return ST_E_INTERNAL;
    if (k.n_learned + 1 > a.cap_ng || k.learned_lits + nN > a.cap_lits) return ST_UNKNOWN;
    bar();
    for (int w = tid; w < W; w += T) {
        int pos = 0;
        for (int w2 = 0; w2 < w; ++w2) {
            unsigned long long y = c.sB[w2];
            if (w2 == W - 1) y &= ~(1ull << 63);
            if (w2 == 0) y &= ~1ull;
            pos += __popcll(y);
        }
        unsigned long long x = c.sB[w];
        if (w == W - 1) x &= ~(1ull << 63);
        if (w == 0) x &= ~1ull;
        while (x) {
            int bt = __ffsll((long long)x) - 1;
            x &= x - 1ull;
            c.llits[base + pos] = c.dec[w * 64 + bt + 1];
            ++pos;
        }
    }
    if (b.sat)
        for (int l = 64 * W + tid; l <= cdl; l += T) c.llits[base + b.npop + (l - 64 * W)] = c.dec[l];
    *nN_out = nN;
    *bj_out = bj;
    return 0;
}

// Learning of the pending conflict -- or, with several conflicts learned
// per step, of each selected round conflict in rank order (Sect. 4.2: the
// lowest backjump level among the learned nogoods is taken) -- then
// Backjump and assertion of the latest literal of the first nogood that
// reaches that level.
DEV void step_learn(Ctx& c, Ctl& k, const KArgs& a) {
    const int T = c.T, tid = c.tid, W = c.W;
    c.scr->pool_top = k.pool_top;
    c.scr->cap_err = 0;
    const int nsel = (c.multi && k.pend_kind == 1) ? k.n_pend : 1;
    auto conf_of = [&](int i) {
        return k.pend_kind != 1 ? -1 : (i == 0 ? k.pending : k.pend_more[i - 1]);
    };
    // every selected conflict first: one that follows from level-1 facts
    // alone (B = 0; under Res-learning no literal above level 1) is UNSAT
    bool zero = false;
    int ctop0 = -1;
    for (int i = 0; i < nsel && !zero; ++i) {
        const int conf = conf_of(i);
        if (conf >= 0 && c.learning == LEARN_RES) {
            const int t = conflict_top(c, k, conf);
            if (i == 0) ctop0 = t;
            zero = t <= 1;
        } else {
            if (conf >= 0) conflict_B(c, k, conf);
            else bar();
            zero = read_B(c).zero;
            if (nsel > 1) bar();   // every lane has read B before another conflict's clears it
        }
    }
    if (zero) {
        k.conflicts += 1;
        k.status = ST_UNSAT;
        bar();
        return;
    }
    if (a.max_conflicts >= 0 && k.conflicts >= a.max_conflicts) {
        k.status = ST_UNKNOWN;
        bar();
        return;
    }
    k.conflicts += 1;
    // learned Decision: a run of fallback_after conflicts with no decision
    // reaching a conflict-free fixpoint hands Decision back to occurrences
    k.dec_open = 0;
    if (k.use_score) {
        k.consec += 1;
        if (c.fallback_after >= 0 && k.consec >= c.fallback_after) {
            k.use_score = 0;
            k.hash = fnv(k.hash, 7);
        }
    }
    int bj = 0, base = 0, nN = 0, newid = -1;   // the nogood that asserts
    for (int i = 0; i < nsel; ++i) {
        const int conf = conf_of(i);
        const int ibase = uni(c.loff[k.n_learned]);
        const int iid = k.nS + k.n_learned;
        int inN = 0, ibj = 1;
        const int st = learn_one(c, k, a, conf, nsel == 1, i == 0 ? ctop0 : -1, ibase, &inN, &ibj);
        if (st) {
            k.status = st;
            bar();
            return;
        }
        k.hash = fnv(k.hash, 2);
        k.hash = fnv(k.hash, conf);
        k.hash = fnv(k.hash, inN);
        k.hash = fnv(k.hash, ibj);
        c.loff[k.n_learned + 1] = ibase + inN;
        bar();
        add_occurrences(c, ibase, inN, iid);
        k.n_learned += 1;
        k.learned_lits += inN;
        k.learned += 1;
        k.learned_len += inN;
        if (c.ext && c.decision == DECISION_ACTIVITY) {
            // every literal bumps its atom (an auxiliary variable of rule r
            // stands for the head of r); all are halved after every 64th nogood
            for (int q = tid; q < inN; q += T) {
                const int v = lvar(c.llits[ibase + q]);
                atomicAdd(&c.act[v <= k.A ? v : c.RH[(v - k.A - 1) / 3]], 8);
            }
            if (k.learned % 64 == 0) {
                bar();
                for (int p = 1 + tid; p <= k.A; p += T) c.act[p] >>= 1;
            }
        }
        if (newid < 0 || ibj < bj) {
            bj = ibj;
            base = ibase;
            nN = inN;
            newid = iid;
        }
        bar();
    }
    k.since_restart += 1;
    if (c.ext && a.restart_every > 0 && k.since_restart >= a.restart_every) {
        k.pool_top = uni(c.scr->pool_top);
        if (uni(c.scr->cap_err)) {
            k.status = ST_E_CAPACITY;
            bar();
            return;
        }
        restart(c, k);
        return;
    }
    // Backjump: unassign every variable above level bj (the trail holds
    // levels in non-decreasing order, level l starting at tlim[l])
    const int start = uni(c.tlim[bj + 1]);
    for (int i = start + tid; i < k.qt; i += T) {
        int v = c.trail[i];
        vclr(c.valb, v);
        if (c.learning == LEARN_RES) {
            c.lvl[v] = 0;
            for (int w = 0; w < W; ++w) c.deps[(size_t)v * W + w] = 0ull;
        }
    }
    bar();
    k.pool_top = uni(c.scr->pool_top);
    if (uni(c.scr->cap_err)) {
        k.status = ST_E_CAPACITY;
        bar();
        return;
    }
    // assert the complement of the latest decision at level bj, its Deps
    // being those of the other decisions of the learned nogood
    for (int w = tid; w < W; w += T) c.sB[w] = 0ull;
    bar();
    for (int q = tid; q < (nN - 1) * W; q += T) {
        int i = q / W, w = q - i * W;
        unsigned long long d = c.deps[(size_t)lvar(c.llits[base + i]) * W + w];
        if (d) atomicOr(&c.sB[w], d);
    }
    bar();
    const int top = uni(c.llits[base + nN - 1]);
    const int x = lvar(top);
    for (int w = tid; w < W; w += T) c.deps[(size_t)x * W + w] = c.sB[w];
    vset(c.valb, x, top > 0 ? VF : VT);   // identical from every lane
    if (c.learning == LEARN_RES) {
        c.lvl[x] = bj;
        c.gpos[x] = start;
        c.reason[x] = newid;
    }
    c.trail[start] = x;
    bar();
    for (int w = tid; w < W; w += T) c.sB[w] = 0ull;
    put_record(c, 0, x, top > 0 ? VF : VT, c.deps[(size_t)x * W]);   // identical from every lane
    bar();
    k.cdl = bj;
    k.qh = start;
    k.qt = start + 1;
    k.fr_ok = 1;
    k.pending = -1;
    k.pend_kind = 0;
    k.n_pend = 0;
}

// Decision (Sect. 2): among rules with unassigned head, T t_r and not F n_r,
// the highest occurrence count of the head wins, ties to the lowest rule;
// T b_r is assigned at a new level.  Without a candidate,
// CompleteAssignment falsifies every unassigned atom.
// The search stands at a conflict-free fixpoint: if a decision led here,
// the run of consecutive conflicts is over.
DEV void at_fixpoint(Ctl& k) {
    if (k.dec_open) k.consec = 0;
}

// This lane's best applicable rule: key (score of the head, biased to keep
// its order as unsigned) << 32 | (~rule), 0 if none.  BY_ACT reads the
// head's activity, else score[j]; four rules per lane at a time, so their
// loads are issued together.
template <bool BY_ACT, bool BELOW = false>
DEV unsigned long long best_rule(Ctx& c, const Ctl& k, const int32_t* score,
                                 unsigned long long below = 0ull) {
    const int T = c.T, A = k.A, Rh = k.Rh;
    unsigned long long best = 0ull;
    constexpr int U = 4;
    for (int j0 = c.tid; j0 < Rh; j0 += U * T) {
        int hp[U], sc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u * T;
            hp[u] = j < Rh ? c.RH[j] : 0;
            if (!BY_ACT) sc[u] = j < Rh ? score[j] : 0;
        }
        if (BY_ACT) {
#pragma unroll
            for (int u = 0; u < U; ++u) sc[u] = j0 + u * T < Rh ? c.act[hp[u]] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u * T;
            if (j >= Rh || vget(c.valb, hp[u]) != 0u) continue;
            const int t = A + 3 * j + 2;
            if (vget(c.valb, t) != VT || vget(c.valb, t + 1) == VF) continue;
            const unsigned long long key =
                ((unsigned long long)((uint32_t)sc[u] ^ 0x80000000u) << 32) |
                (unsigned long long)(0xffffffffu - (uint32_t)j);
            if (BELOW && key >= below) continue;
            best = key > best ? key : best;
        }
    }
    return best;
}

// The Decision under a per-rule score that stays fixed during the search
// (the static table, or supplied scores): the first candidate in the
// order `ord` of the rules (score descending, then rule ascending; sorted
// by the host for the static table, on the device for supplied scores) is
// the candidate of greatest (score, -rule) key, the one best_rule finds.  Each
// wave scans its own 64-position chunks of that order (wave w: chunks w,
// w + nw, ...), four in flight, and stops at its first chunk that holds a
// candidate; the block keeps the lowest position.  Returns
// (2^32-1 - position) << 32 | rule for the caller's block maximum, 0 when no
// rule is a candidate.
DEV unsigned long long first_rule(Ctx& c, const Ctl& k, const int32_t* ord) {
    const int Rh = k.Rh, A = k.A, nw = c.nw, lane = c.lane;
    constexpr int U = 4;
    for (int p0 = c.wid * 64; p0 < Rh; p0 += U * nw * 64) {
        int jj[U], hh[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = p0 + u * nw * 64 + lane;
            jj[u] = p < Rh ? ord[2 * p] : 0;
            hh[u] = p < Rh ? ord[2 * p + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = p0 + u * nw * 64 + lane;
            bool cand = false;
            if (p < Rh && vget(c.valb, hh[u]) == 0u) {
                const int t = A + 3 * jj[u] + 2;
                cand = vget(c.valb, t) == VT && vget(c.valb, t + 1) != VF;
            }
            const unsigned long long m = __ballot(cand);
            if (m != 0ull) {
                const int l = __ffsll((long long)m) - 1;
                const uint32_t pos = (uint32_t)(p0 + u * nw * 64 + l);
                const int j = __builtin_amdgcn_readlane(jj[u], l);
                return ((unsigned long long)(0xffffffffu - pos) << 32) | (uint32_t)j;
            }
        }
    }
    return 0ull;
}

// Assign T b_j at the next level (the decided literal; its Deps is the
// level's bit) and make it the frontier.  Counters and trace untouched.
DEV void decide_rule(Ctx& c, Ctl& k, int j) {
    const int T = c.T, tid = c.tid, W = c.W;
    const int b = k.A + 3 * j + 1;
    const int ncdl = k.cdl + 1;
    const int bit = level_bit(ncdl, W);
    for (int w = tid; w < W; w += T)
        c.deps[(size_t)b * W + w] = (w == (bit >> 6)) ? (1ull << (bit & 63)) : 0ull;
    c.tlim[ncdl] = k.qt;                 // identical stores from every lane
    c.dec[ncdl] = b;
    if (c.learning == LEARN_RES) {
        c.lvl[b] = ncdl;
        c.gpos[b] = k.qt;
        c.reason[b] = -1;
    }
    c.trail[k.qt] = b;
    vset(c.valb, b, VT);
    put_record(c, 0, b, VT, bit < 64 ? (1ull << bit) : 0ull);   // identical from every lane
    bar();
    k.cdl = ncdl;
    k.qh = k.qt;
    k.qt = k.qt + 1;
    k.fr_ok = 1;
}

DEV int rule_of(unsigned long long key) { return (int)(0xffffffffu - (uint32_t)(key & 0xffffffffull)); }

// Lookahead Decision (extended search, Fwd-learning): the candidates with
// the `lookahead` best keys -- best first, `best` the first -- are tried in
// order; a trial decides the rule and runs rounds until a fixpoint or a
// conflict.  A trial ending in a conflict or with every variable assigned
// stands as the Decision.  Otherwise the variables it assigned are counted
// (trace event 10, rule, count) and it is undone: the trail is cut back and
// the values cleared (Deps of unassigned variables are never read).  With
// no trial standing, the candidate with the most assignments (earliest on
// ties) is decided.
DEV void lookahead_decide(Ctx& c, Ctl& k, unsigned long long best, const int32_t* score) {
    const int T = c.T, tid = c.tid;
    unsigned long long keys[8];
    int n = 1;
    keys[0] = best;
    const bool by_act = c.decision == DECISION_ACTIVITY;
    for (int i = 1; i < c.lookahead && i < 8; ++i) {
        const unsigned long long mine = by_act ? best_rule<true, true>(c, k, c.RO, keys[i - 1])
                                               : best_rule<false, true>(c, k, score, keys[i - 1]);
        const unsigned long long nxt = block_max_u64(c, mine);
        bar();
        if (nxt == 0ull) break;
        keys[n++] = nxt;
    }
    int pick = rule_of(best);
    if (n > 1) {
        const int consec0 = k.consec, open0 = k.dec_open, cdl0 = k.cdl, qt0 = k.qt;
        int best_p = -1;
        for (int i = 0; i < n; ++i) {
            const int j = rule_of(keys[i]);
            decide_rule(c, k, j);
            k.dec_open = 1;
            while (k.qt > k.qh && !k.pend_kind && k.status == ST_RUNNING) {
                step_round(c, k);
                bar();
            }
            if (k.pend_kind || k.qt == k.V || k.status != ST_RUNNING) {
                k.decisions += 1;
                k.hash = fnv(k.hash, 1);
                k.hash = fnv(k.hash, j);
                return;
            }
            const int p = k.qt - qt0;
            k.hash = fnv(k.hash, 10);
            k.hash = fnv(k.hash, j);
            k.hash = fnv(k.hash, p);
            for (int q = qt0 + tid; q < k.qt; q += T) vclr(c.valb, c.trail[q]);
            bar();
            k.qt = k.qh = qt0;
            k.cdl = cdl0;
            k.fr_ok = 0;
            k.consec = consec0;
            k.dec_open = open0;
            if (p > best_p) {
                best_p = p;
                pick = j;
            }
        }
    }
    decide_rule(c, k, pick);
    k.decisions += 1;
    k.dec_open = 1;
    k.hash = fnv(k.hash, 1);
    k.hash = fnv(k.hash, pick);
}

DEV int step_decide_or_complete(Ctx& c, Ctl& k) {
    const int T = c.T, tid = c.tid, W = c.W, A = k.A;
    at_fixpoint(k);
    // key: head score (signed, biased to keep its order) then lowest rule;
    // the score is the static per-rule table (occurrences or Jeroslow-Wang),
    // the supplied scores, or the head's activity
    const int32_t* score = k.use_score ? c.RS : c.RO;
    unsigned long long best;
    int j;
    if (!c.ext) {
        best = block_max_u64(c, first_rule(c, k, k.use_score ? c.RDS : c.RD));
        j = (int)(uint32_t)(best & 0xffffffffull);
    } else {
        const unsigned long long mine = c.ext && c.decision == DECISION_ACTIVITY
                                            ? best_rule<true>(c, k, c.RO)
                                            : best_rule<false>(c, k, score);
        best = block_max_u64(c, mine);
        j = rule_of(best);
    }
    bar();
    if (best != 0ull) {
        if (c.ext && c.lookahead > 1) {
            lookahead_decide(c, k, best, score);
            return STEP_DECIDE;
        }
        decide_rule(c, k, j);
        k.decisions += 1;
        k.dec_open = 1;
        k.hash = fnv(k.hash, 1);
        k.hash = fnv(k.hash, j);
        return STEP_DECIDE;
    }
    // CompleteAssignment
    const int cdl = k.cdl;
    c.scr->tail = k.qt;
    bar();
    for (int p = 1 + tid; p <= A; p += T) {
        if (vget(c.valb, p) != 0u) continue;
        for (int w = 0; w < W; ++w) c.deps[(size_t)p * W + w] = alldec_word(w, cdl, W);
        if (c.learning == LEARN_RES) {
            c.lvl[p] = cdl;
            c.gpos[p] = k.qt;
            c.reason[p] = -1;
        }
        int pos = atomicAdd(&c.scr->tail, 1);
        c.trail[pos] = p;
    }
    bar();
    const int nt = uni(c.scr->tail);
    for (int i = k.qt + tid; i < nt; i += T) vset(c.valb, c.trail[i], VF);
    bar();
    const int n = nt - k.qt;
    k.completes += 1;
    k.hash = fnv(k.hash, 3);
    k.hash = fnv(k.hash, n);
    k.qh = k.qt;
    k.qt = nt;
    k.fr_ok = 0;
    if (n == 0) k.status = ST_E_INTERNAL;
    return STEP_COMPLETE;
}

// Stability check of a total assignment: M = true atoms must equal the
// least model of the reduct (rules whose body- misses M, body- dropped).
// Otherwise the unfounded set U = M \ LM gives the conflict: its least atom
// u with every external support (head in U, body+ disjoint from U), whose
// b_r is false in M.
// An answer set M was found (and stored).  Asking for one answer set, or
// having all asked for, ends the search; otherwise M is blocked by the
// learned nogood {T p : p in M} (answer sets are incomparable under set
// inclusion, so it excludes M alone) and the search restarts.
DEV void answer_set(Ctx& c, Ctl& k, const KArgs& a) {
    const int T = c.T, tid = c.tid, A = k.A;
    k.models += 1;
    if (!c.ext || a.max_models == 1) {
        k.status = ST_SAT;
        return;
    }
    k.hash = fnv(k.hash, 8);
    k.hash = fnv(k.hash, (int32_t)k.models);
    if (a.max_models > 0 && k.models >= a.max_models) {
        k.status = ST_SAT;
        return;
    }
    unsigned long long cnt = 0ull;
    for (int p = 1 + tid; p <= A; p += T) cnt += vget(c.valb, p) == VT ? 1ull : 0ull;
    const int nN = (int)block_sum_u64(c, cnt);
    if (k.n_learned + 1 > a.cap_ng || k.learned_lits + nN > a.cap_lits) {
        k.status = ST_UNKNOWN;
        bar();
        return;
    }
    // the true atoms, ascending: a block scan per chunk of T atoms
    const int base = uni(c.loff[k.n_learned]);
    int done = 0;
    for (int b0 = 1; b0 <= A; b0 += T) {
        const int p = b0 + tid;
        const int f = (p <= A && vget(c.valb, p) == VT) ? 1 : 0;
        const int inc = wave_incl_scan(f);
        c.scr->wsum[c.wid] = wave_last(inc);   // identical from the wave's lanes
        bar();
        int off = 0, tot = 0;
        for (int w = 0; w < c.nw; ++w) {
            const int x = c.scr->wsum[w];
            off += w < c.wid ? x : 0;
            tot += x;
        }
        if (f) c.llits[base + done + off + inc - 1] = p;
        done += uni(tot);
        bar();
    }
    const int newid = k.nS + k.n_learned;
    c.loff[k.n_learned + 1] = base + nN;
    c.scr->pool_top = k.pool_top;
    c.scr->cap_err = 0;
    bar();
    add_occurrences(c, base, nN, newid);
    bar();
    k.pool_top = uni(c.scr->pool_top);
    if (uni(c.scr->cap_err)) {
        k.status = ST_E_CAPACITY;
        bar();
        return;
    }
    k.n_learned += 1;
    k.learned_lits += nN;
    restart(c, k);
}

DEV void step_gate(Ctx& c, Ctl& k, const KArgs& a, uint8_t* model) {
    const int T = c.T, tid = c.tid, W = c.W, A = k.A, Rh = k.Rh;
    at_fixpoint(k);
    uint32_t* lm = c.lm;   // 1 bit per atom, zero between checks
    for (;;) {
        c.scr->changed = 0;
        bar();
        for (int j = tid; j < Rh; j += T) {
            int h = c.RH[j];
            if ((lm[h >> 5] >> (h & 31)) & 1u) continue;
            bool ok = true;
            for (int q = c.RBO[j]; ok && q < c.RBO[j + 1]; ++q) {
                int l = c.RBL[q];
                if (l < 0) ok = vget(c.valb, -l) != VT;
                else ok = (lm[l >> 5] >> (l & 31)) & 1u;
            }
            if (ok) {
                atomicOr(&lm[h >> 5], 1u << (h & 31));
                c.scr->changed = 1;
            }
        }
        bar();
        const int ch = uni(c.scr->changed);
        bar();
        if (!ch) break;
    }
    int u = 0x7fffffff;
    for (int p = 1 + tid; p <= A; p += T) {
        bool inM = vget(c.valb, p) == VT, inLM = (lm[p >> 5] >> (p & 31)) & 1u;
        if (inM && !inLM) {
            u = p;
            break;
        }
    }
    u = block_min_i32(c, u);
    if (u == 0x7fffffff) {
        if (k.models < a.model_store) {
            uint8_t* out = model + (size_t)k.models * (size_t)A;
            for (int p = 1 + tid; p <= A; p += T)
                out[p - 1] = vget(c.valb, p) == VT ? (uint8_t)1 : (uint8_t)0;
        }
    } else {
        for (int w = tid; w < W; w += T)
            c.sB[w] = a.gate_mode == 1 ? alldec_word(w, k.cdl, W) : c.deps[(size_t)u * W + w];
        bar();
        if (a.gate_mode == 0) {
            for (int j = tid; j < Rh; j += T) {
                int h = c.RH[j];
                bool hU = vget(c.valb, h) == VT && !((lm[h >> 5] >> (h & 31)) & 1u);
                if (!hU) continue;
                bool ext = true;
                for (int q = c.RBO[j]; ext && q < c.RBO[j + 1]; ++q) {
                    int l = c.RBL[q];
                    if (l > 0) ext = !(vget(c.valb, l) == VT && !((lm[l >> 5] >> (l & 31)) & 1u));
                }
                if (!ext) continue;
                int b = A + 3 * j + 1;
                for (int w = 0; w < W; ++w) {
                    unsigned long long d = c.deps[(size_t)b * W + w];
                    if (d) atomicOr(&c.sB[w], d);
                }
            }
        }
    }
    bar();
    for (int i = tid; i < ((A + 1 + 31) >> 5); i += T) lm[i] = 0u;
    bar();
    if (u == 0x7fffffff) {
        answer_set(c, k, a);
    } else {
        k.gate_fail += 1;
        k.pend_kind = 2;
        k.pending = -1;
    }
}

// Run the state machine until the search ends, the step budget is used, or
// the next step is not allowed (step kernels).
DEV void run_search(Ctx& c, Ctl& k, const KArgs& a, uint8_t* model, uint64_t t0) {
    for (;;) {
        {
            // The thread index passes through an empty asm statement at each
            // step, so the compiler derives the lanes' LDS addresses inside
            // the step instead of keeping dozens of them live across the
            // whole search loop (the registers that buy a fourth wave per
            // SIMD).
            int t = c.tid;
            asm volatile("" : "+v"(t));
            c.tid = t;
            c.lane = t & 63;
            c.wid = t >> 6;
        }
        int halt = 0;
        if (k.status == ST_RUNNING) {
            if (a.mode == MODE_STEPS) {
                if (k.steps >= a.max_steps) halt = 1;
            } else if (a.max_steps >= 0 && k.steps >= a.max_steps) {
                k.status = ST_E_INTERNAL;
            }
            // the clock is read per wave, every 64 steps; the workgroup
            // acts on the OR
            if ((k.steps & 63) == 0) {
                int late = (a.max_ticks && (uint64_t)(wall_clock64() - t0) > a.max_ticks) ? 1 : 0;
                if (block_any(c, late)) k.status = ST_E_TIMEOUT;
            }
        }
        int kind = STEP_DONE;
        if (!halt && k.status == ST_RUNNING) {
            if (!k.init_done) kind = STEP_INIT;
            else if (k.pend_kind) kind = STEP_LEARN;
            else if (k.qt > k.qh) kind = STEP_ROUND;
            else if (k.qt == k.V) kind = STEP_GATE;
            else kind = STEP_DECIDE;
            if (a.mode == MODE_STEPS) {
                int allowed = a.step_mask;
                bool ok = (allowed >> kind) & 1;
                if (kind == STEP_DECIDE) ok = ok || ((allowed >> STEP_COMPLETE) & 1);
                if (!ok) kind = STEP_DONE;
            }
        }
        kind = uni(kind);
        if (kind == STEP_DONE) break;
        const uint64_t ts = wall_clock64();
        switch (kind) {
        case STEP_INIT: step_init(c, k); break;
        case STEP_ROUND: step_round(c, k); break;
        case STEP_LEARN: step_learn(c, k, a); break;
        case STEP_GATE: step_gate(c, k, a, model); break;
        default: kind = step_decide_or_complete(c, k); break;
        }
        const uint64_t dt = wall_clock64() - ts;
        if (kind == STEP_ROUND || kind == STEP_INIT) k.t_round += dt;
        else if (kind == STEP_LEARN) k.t_learn += dt;
        else if (kind == STEP_GATE) k.t_gate += dt;
        else k.t_decide += dt;
        k.steps += 1;
        k.last_step = kind;
        if ((k.status == ST_UNSAT || k.status == ST_UNKNOWN) && k.models > 0) {
            // the search ended after answer sets were found
            k.exhausted = k.status == ST_UNSAT ? 1 : 0;
            k.status = ST_SAT;
        }
        if (k.status == ST_SAT) k.hash = fnv(k.hash, 4);
        else if (k.status == ST_UNSAT) k.hash = fnv(k.hash, 5);
        else if (k.status == ST_UNKNOWN) k.hash = fnv(k.hash, 6);
        bar();
    }
}

// Every lane stores the same result values (identical stores).
DEV void write_result(Ctx& c, const Ctl& k, const KArgs& a, uint64_t t0) {
    DevStats& d = a.stats[k.inst];
    d.t_total = wall_clock64() - t0;
    d.t_round = k.t_round;
    d.t_learn = k.t_learn;
    d.t_decide = k.t_decide;
    d.t_gate = k.t_gate;
    d.rounds = k.rounds;
    d.visits = k.visits;
    d.checks = k.checks;
    d.props = k.props;
    d.decisions = k.decisions;
    d.conflicts = k.conflicts;
    d.learned = k.learned;
    d.learned_len = k.learned_len;
    d.gate_fail = k.gate_fail;
    d.completes = k.completes;
    d.hash = k.hash;
    d.status = k.status;
    d.last_step = k.last_step;
    d.models = k.models;
    d.restarts = k.restarts;
    d.exhausted = k.exhausted;
    a.verdicts[k.inst] = k.status;
    bar();
}

// Four waves per SIMD for the plain search with Fwd-learning: the register
// budget (128 VGPRs) at which it keeps eight 128-thread workgroups resident
// per CU (LDS allowing); Res-learning and the extended search, with more
// live state, keep three (168 VGPRs) rather than spill.  The Learning
// step and the search mode are compile-time parameters -- EN 0 plain, 1
// extended (several answer sets, restarts, the activity Decision), 2 the
// extended search learning several conflicts per step -- so each search
// carries only its own code and registers.
template <int MAXT, int LR, int EN>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu((EN == 0 && LR == 0) ? 4 : 3))) void k_search(KArgs a) {
    HIP_DYNAMIC_SHARED(unsigned long long, smem64);  // 8-byte aligned base
    __shared__ Scr scr;
    Ctx c;
    Ctl k;
    c.W = a.W;
    c.decision = a.decision;
    c.fallback_after = a.fallback_after;
    c.learning = LR;
    c.ext = EN >= 1;
    c.multi = EN == 2;
    c.learn_k = a.learn_k;
    c.lookahead = a.lookahead;
    c.T = MAXT;
    c.tid = threadIdx.x;
    c.lane = threadIdx.x & 63;
    c.wid = threadIdx.x >> 6;
    c.nw = MAXT / 64;
    c.FC = MAXT > kFrontCap ? MAXT : kFrontCap;
    c.IC = MAXT > kImplCap ? MAXT : kImplCap;
    c.scr = &scr;
    c.my_visits = c.my_checks = 0ull;
    {
        // 8-byte arrays first (the base is 8-byte aligned), then 4-byte ones
        unsigned char* p = (unsigned char*)smem64;
        c.sB = (unsigned long long*)p; p += sizeof(unsigned long long) * kMaxW;
        c.tWin = (unsigned long long*)p; p += sizeof(unsigned long long) * kWinCap;
        c.iDeps = (unsigned long long*)p; p += sizeof(unsigned long long) * c.IC;
        c.fDeps = (unsigned long long*)p; p += sizeof(unsigned long long) * c.FC;
        c.sTile = nullptr;   // Res-learning only
        if (LR == LEARN_RES) {
            c.sTile = (unsigned long long*)p;
            p += sizeof(unsigned long long) * MAXT;
        }
        c.valb = (uint32_t*)p; p += sizeof(uint32_t) * a.words;
        c.lm = (uint32_t*)p; p += sizeof(uint32_t) * a.awords;
        c.tKey = (int32_t*)p; p += sizeof(int32_t) * kWinCap;
        c.tCode = (int32_t*)p; p += sizeof(int32_t) * kWinCap;
        c.iS0 = (int32_t*)p; p += sizeof(int32_t) * c.IC;
        c.iCs = (int32_t*)p; p += sizeof(int32_t) * c.IC;
        c.iL0 = (int32_t*)p; p += sizeof(int32_t) * c.IC;
        c.iCl = (int32_t*)p; p += sizeof(int32_t) * c.IC;
        c.sOff = (int32_t*)p; p += sizeof(int32_t) * MAXT;
        c.fS0 = (int32_t*)p; p += sizeof(int32_t) * c.FC;
        c.fCs = (int32_t*)p; p += sizeof(int32_t) * c.FC;
        c.fL0 = (int32_t*)p; p += sizeof(int32_t) * c.FC;
        c.fCl = (int32_t*)p; p += sizeof(int32_t) * c.FC;
        c.fNew = (int32_t*)p; p += sizeof(int32_t) * c.FC;
        c.fSlot = (int32_t*)p; p += sizeof(int32_t) * c.FC;
    }
    const uint64_t t0 = wall_clock64();
    if (a.mode == MODE_SOLVE) {
        // one workgroup per instance; the hardware dispatcher keeps as many
        // resident as LDS and wave slots allow
        if ((int)blockIdx.x >= a.count) return;
        const int inst = uni(a.order[a.first + (int)blockIdx.x]);
        bind_instance(c, k, a, inst);
        reset_search(c, k);
        run_search(c, k, a, a.models + a.inst[inst].model, t0);
        flush_counters(c, k);
        write_result(c, k, a, t0);
        save_ctrl(c, k);
    } else {
        bind_instance(c, k, a, 0);
        if (a.mode == MODE_STEPS) {
            load_ctrl(c, k);
            run_search(c, k, a, a.models + a.inst[0].model, t0);
        } else {
            reset_search(c, k);
        }
        flush_counters(c, k);
        save_ctrl(c, k);
    }
}

// ------------------------------------------------------------ launchers
size_t lds_bytes(int threads, int words, int awords, int learning) {
    const size_t fc = threads > kFrontCap ? (size_t)threads : (size_t)kFrontCap;
    const size_t ic = threads > kImplCap ? (size_t)threads : (size_t)kImplCap;
    return sizeof(uint32_t) * ((size_t)words + (size_t)awords) + sizeof(unsigned long long) * kMaxW +
           sizeof(int32_t) * (size_t)threads + sizeof(int32_t) * 6 * fc +
           (sizeof(unsigned long long) + 2 * sizeof(int32_t)) * (size_t)kWinCap +
           (sizeof(unsigned long long) + 4 * sizeof(int32_t)) * ic +
           sizeof(unsigned long long) * (fc + (learning == LEARN_RES ? (size_t)threads : 0));
}

template <int LR, int EN>
static hipError_t launch_v(const KArgs& a, int threads, int grid, size_t lds, hipStream_t s) {
    switch (threads) {
    case 64: hipLaunchKernelGGL((k_search<64, LR, EN>), dim3(grid), dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL((k_search<128, LR, EN>), dim3(grid), dim3(128), lds, s, a); break;
    case 256: hipLaunchKernelGGL((k_search<256, LR, EN>), dim3(grid), dim3(256), lds, s, a); break;
    case 512: hipLaunchKernelGGL((k_search<512, LR, EN>), dim3(grid), dim3(512), lds, s, a); break;
    case 1024: hipLaunchKernelGGL((k_search<1024, LR, EN>), dim3(grid), dim3(1024), lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static int search_mode(const KArgs& a) {
    if (a.learn_k > 1) return 2;
    return (a.max_models != 1 || a.restart_every != 0 || a.decision == DECISION_ACTIVITY ||
            a.lookahead > 1) ? 1 : 0;
}

template <int LR>
static hipError_t launch_lr(const KArgs& a, int threads, int grid, size_t lds, hipStream_t s) {
    switch (search_mode(a)) {
    case 0: return launch_v<LR, 0>(a, threads, grid, lds, s);
    case 1: return launch_v<LR, 1>(a, threads, grid, lds, s);
    default: return launch_v<LR, 2>(a, threads, grid, lds, s);
    }
}

hipError_t launch_search(const KArgs& a, int threads, int grid, size_t lds, hipStream_t s) {
    if (a.learning == LEARN_FWD) return launch_lr<LEARN_FWD>(a, threads, grid, lds, s);
    if (a.learning == LEARN_RES) return launch_lr<LEARN_RES>(a, threads, grid, lds, s);
    return hipErrorInvalidValue;
}

template <int LR, int EN>
static const void* search_fn_v(int threads) {
    switch (threads) {
    case 64: return (const void*)k_search<64, LR, EN>;
    case 128: return (const void*)k_search<128, LR, EN>;
    case 256: return (const void*)k_search<256, LR, EN>;
    case 512: return (const void*)k_search<512, LR, EN>;
    case 1024: return (const void*)k_search<1024, LR, EN>;
    default: return nullptr;
    }
}

template <int LR>
static const void* search_fn_lr(int threads, int en) {
    switch (en) {
    case 0: return search_fn_v<LR, 0>(threads);
    case 1: return search_fn_v<LR, 1>(threads);
    default: return search_fn_v<LR, 2>(threads);
    }
}

static const void* search_fn(int threads, int learning, int en) {
    if (learning == LEARN_FWD) return search_fn_lr<LEARN_FWD>(threads, en);
    if (learning == LEARN_RES) return search_fn_lr<LEARN_RES>(threads, en);
    return nullptr;
}

hipError_t set_max_lds(int threads, size_t lds) {
    for (int lr : {(int)LEARN_FWD, (int)LEARN_RES})
        for (int en = 0; en < 3; ++en) {
            const void* f = search_fn(threads, lr, en);
            if (!f) return hipErrorInvalidValue;
            const hipError_t e =
                hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace asp
