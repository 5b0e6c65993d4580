// api.cpp -- C ABI of libasp (declared in include/asp.h).
//
// Host side: validates and encodes programs (encode.cpp), plans the device
// arena, uploads the static tables, launches the search kernels
// (solver.hip) and moves states and results.  Device memory is always the
// caller's; nothing here allocates on the device.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/asp.h"
#include "encode.h"
#include "layout.h"
#include "scorer.h"
#include "train.h"

namespace asp {
size_t lds_bytes(int threads, int words, int awords, int learning);
hipError_t launch_search(const KArgs& a, int threads, int grid, size_t lds, hipStream_t s);
hipError_t set_max_lds(int threads, size_t lds);
}  // namespace asp

using namespace asp;

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(ASP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int g_clock_khz = 0;   // device wall-clock rate (kHz), set by device_info()

struct DeviceInfo {
    int ok = 0;
    int cus = 0;
    size_t max_lds = 0;
    int clock_khz = 0;  // wall clock rate
};

DeviceInfo device_info() {
    DeviceInfo d;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return d;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return d;
    d.cus = p.multiProcessorCount;
    d.max_lds = p.sharedMemPerBlock;
    int rate = 0;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev) == hipSuccess)
        d.clock_khz = rate;
    g_clock_khz = d.clock_khz;
    d.ok = d.cus > 0;
    return d;
}

bool valid_threads(int t) { return t == 64 || t == 128 || t == 256 || t == 512 || t == 1024; }

}  // namespace

// ---------------------------------------------------------------- handles
// One launch of the search kernel: instances order[first .. first+count),
// LDS sized for the largest of them.
struct LaunchClass {
    int32_t first = 0, count = 0, words = 1, awords = 1, threads = 128;
    size_t lds = 0;
};

struct Plan {
    int32_t n = 0, threads = 256, W = 1, gate = 0, decision = 0, fallback_after = 10, learning = 0;
    int64_t Vmax = 0, Rhmax = 0, cap_ng = 0, cap_lits = 0;
    int64_t max_models = 1, restart_every = 0, model_store = 1;
    int32_t learn_k = 1;
    int32_t lookahead = 0;
    std::vector<LaunchClass> classes;
    std::vector<InstDesc> desc;
    std::vector<int32_t> order;
    std::vector<int64_t> slot_off;      // per instance, bytes from off_slots
    uint64_t off_desc = 0, off_order = 0, off_slotoff = 0, off_ngo = 0, off_ngl = 0, off_mo = 0,
             off_mi = 0, off_rh = 0, off_ro = 0, off_rbo = 0, off_rbl = 0, off_asc = 0,
             off_rs = 0, off_rord = 0, off_rords = 0, off_rsort = 0, off_verd = 0, off_stats = 0, off_models = 0, off_slots = 0, total = 0;
    int64_t tot_ngo = 0, tot_ngl = 0, tot_mo = 0, tot_mi = 0, tot_rules = 0, tot_rbo = 0,
            tot_rbl = 0, tot_model = 0, tot_asc = 0, slots_bytes = 0;
    size_t max_lds() const {
        size_t m = 0;
        for (auto& c : classes) m = std::max(m, c.lds);
        return m;
    }
};

// Scorer workspace: weights, per-instance row offsets, tile lists, and the
// activation codes (64 bytes per variable and per static nogood).
struct ScorerPlan {
    std::vector<int64_t> hv_off, hc_off;
    std::vector<ScorerTile> vt, ct;
    std::vector<int32_t> list;
    uint64_t off_w = 0, off_hvo = 0, off_hco = 0, off_vt = 0, off_ct = 0, off_list = 0,
             off_lab = 0, off_train = 0, total = 0;
    bool planned = false;
    uint8_t* uploaded_to = nullptr;   // workspace holding the tables
    asp_scorer_weights w{};           // host copy kept alive for async copies
};

struct asp_program {
    HostProgram hp;
    asp_options opt{};
    // single-instance binding
    bool bound = false;
    bool scores_ready = false;
    uint8_t* arena = nullptr;
    uint64_t bytes = 0;
    Plan plan;
    Plan load_plan;   // 256 threads, one class: fixed at load (allocation-free solve)
    int32_t threads = 256;
    ScorerPlan scorer;
};

struct asp_batch {
    std::vector<const HostProgram*> progs;
    asp_options opt{};
    Plan plan;
    bool bound = false;
    std::vector<uint8_t> ready;       // decision scores set, per instance
    int32_t n_ready = 0;
    ScorerPlan scorer;
    uint8_t* arena = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_fork = nullptr;
    std::vector<hipStream_t> streams;    // four, one per launch class (default priority)
    std::vector<hipEvent_t> ev_start, ev_join;  // per launch class (timed)
    bool timed = false;
    bool class_timed = false;                    // ev_start/ev_join hold the last launches
    // graph form of the batched solve (stream capture of the fork/join)
    hipGraphExec_t gexec = nullptr;
    hipStream_t gstream = nullptr;
    asp_limits glim{};
    std::vector<hipEvent_t> ev_cjoin;           // capture-time joins (untimed)
};

namespace {

// Wall-clock guard applied when the caller gives none: every launch ends.
constexpr int64_t kDefaultMaxMs = 600000;
// Readout training steps per call.
constexpr int32_t kMaxTrainSteps = 4096;

asp_options default_options() {
    asp_options o;
    o.W = 1;
    o.gate = ASP_GATE_UNFOUNDED;
    o.learned_cap_ng = 1 << 20;
    o.learned_cap_lits = 1 << 22;
    o.decision = ASP_DECISION_OCC;
    o.fallback_after = 10;
    o.learning = ASP_LEARN_FWD;
    o.learn_conflicts = 1;
    o.max_models = 1;
    o.restart_every = 0;
    o.lookahead = 0;
    o.reserved = 0;
    return o;
}

// LDS size classes by variable count (the 2-bit maps take V/4 bytes each).
std::vector<int64_t> class_bounds(int32_t classes) {
    switch (classes) {
    case 1: return {};
    case 2: return {16383};
    case 3: return {8191, 32767};
    default: return {4095, 16383, 32767};
    }
}

int32_t make_plan(const std::vector<const HostProgram*>& progs, const asp_options& opt,
                  int32_t threads, int32_t n_classes, Plan& P,
                  const int32_t* class_threads = nullptr) {
    P = Plan();
    P.n = (int32_t)progs.size();
    P.threads = threads;
    P.W = opt.W;
    P.gate = opt.gate;
    P.decision = opt.decision;
    P.fallback_after = opt.fallback_after;
    P.learning = opt.learning;
    P.cap_ng = opt.learned_cap_ng;
    P.cap_lits = opt.learned_cap_lits;
    P.max_models = opt.max_models;
    P.learn_k = opt.learn_conflicts > 1 ? opt.learn_conflicts : 1;
    P.restart_every = opt.restart_every;
    P.lookahead = opt.lookahead > 1 ? opt.lookahead : 0;
    P.model_store = opt.max_models > 0 ? opt.max_models : 1;
    P.desc.resize(P.n);
    P.slot_off.resize(P.n);
    for (int32_t i = 0; i < P.n; ++i) {
        const HostProgram& h = *progs[i];
        InstDesc& d = P.desc[i];
        d.ng_off = P.tot_ngo;
        d.ng_lits = P.tot_ngl;
        d.map_off = P.tot_mo;
        d.map_ids = P.tot_mi;
        d.rules = P.tot_rules;
        d.rb_off = P.tot_rbo;
        d.rb_lits = P.tot_rbl;
        d.model = P.tot_model;
        d.ascore = P.tot_asc;
        d.A = h.A;
        d.Rh = h.Rh;
        d.V = h.V;
        d.n_static = (int32_t)h.n_nogoods();
        d.u0 = h.u0;
        d.u1 = h.u1;
        d.has_empty = h.has_empty;
        d.pad = 0;
        if ((int64_t)h.n_nogoods() + P.cap_ng >= ((int64_t)1 << 30))
            return fail(ASP_E_CAPACITY, "nogood ids beyond 2^30");
        P.tot_ngo += (int64_t)h.ng_off.size();
        P.tot_ngl += (int64_t)h.ng_lits.size();
        P.tot_mo += (int64_t)h.map_off.size();
        P.tot_mi += (int64_t)h.map_ent.size();
        P.tot_rules += (int64_t)h.rule_head.size();
        P.tot_rbo += (int64_t)h.rb_off.size();
        P.tot_rbl += (int64_t)h.rb_lits.size();
        P.tot_model += (int64_t)h.A * P.model_store;
        P.tot_asc += (int64_t)h.A + 1;
        P.Vmax = std::max<int64_t>(P.Vmax, h.V);
        P.Rhmax = std::max<int64_t>(P.Rhmax, h.Rh);
        P.slot_off[i] = P.slots_bytes;
        P.slots_bytes += slot_layout(h.V, h.Rh, P.W, P.cap_ng, P.cap_lits, P.learning).stride;
    }
    // launch classes by variable count; largest first inside a class
    const std::vector<int64_t> bounds = class_bounds(std::max(1, n_classes));
    auto cls = [&](int32_t i) {
        int c = 0;
        while (c < (int)bounds.size() && progs[i]->V > bounds[c]) ++c;
        return c;
    };
    P.order.resize(P.n);
    std::iota(P.order.begin(), P.order.end(), 0);
    auto work = [&](int32_t i) { return progs[i]->ng_lits.size() + (size_t)progs[i]->V; };
    std::stable_sort(P.order.begin(), P.order.end(), [&](int32_t a, int32_t b) {
        int ca = cls(a), cb = cls(b);
        if (ca != cb) return ca > cb;
        return work(a) > work(b);
    });
    for (int32_t k = 0; k < P.n;) {
        LaunchClass lc;
        lc.first = k;
        const int c = cls(P.order[k]);
        int64_t vmax = 0, amax = 0;
        while (k < P.n && cls(P.order[k]) == c) {
            vmax = std::max<int64_t>(vmax, progs[P.order[k]]->V);
            amax = std::max<int64_t>(amax, progs[P.order[k]]->A);
            ++k;
        }
        lc.count = k - lc.first;
        lc.words = (int32_t)((vmax + 1 + 15) / 16);
        lc.awords = (int32_t)((amax + 1 + 31) / 32);
        const int ci = (int)P.classes.size();
        lc.threads = (class_threads && ci < 4 && class_threads[ci] > 0) ? class_threads[ci] : threads;
        lc.lds = lds_bytes(lc.threads, lc.words, lc.awords, P.learning);
        P.classes.push_back(lc);
    }
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    P.off_desc = take(sizeof(InstDesc) * (uint64_t)P.n);
    P.off_order = take(4 * (uint64_t)P.n);
    P.off_slotoff = take(8 * (uint64_t)P.n);
    P.off_ngo = take(4 * (uint64_t)P.tot_ngo);
    P.off_ngl = take(4 * (uint64_t)P.tot_ngl);
    P.off_mo = take(4 * (uint64_t)P.tot_mo);
    P.off_mi = take(sizeof(MapEntry) * (uint64_t)P.tot_mi);
    P.off_rh = take(4 * (uint64_t)P.tot_rules);
    P.off_ro = take(4 * (uint64_t)P.tot_rules);
    P.off_rbo = take(4 * (uint64_t)P.tot_rbo);
    P.off_rbl = take(4 * (uint64_t)P.tot_rbl);
    P.off_asc = take(4 * (uint64_t)P.tot_asc);
    P.off_rs = take(4 * (uint64_t)P.tot_rules);
    P.off_rord = take(8 * (uint64_t)P.tot_rules);
    P.off_rords = take(8 * (uint64_t)P.tot_rules);
    P.off_rsort = take(8 * (uint64_t)P.tot_rules);
    P.off_verd = take(4 * (uint64_t)P.n);
    P.off_stats = take(sizeof(DevStats) * (uint64_t)P.n);
    P.off_models = take((uint64_t)P.tot_model + 1);
    P.off_slots = take((uint64_t)P.slots_bytes);
    P.total = o;
    return ASP_OK;
}

template <class T>
std::vector<T> concat(const std::vector<const HostProgram*>& progs,
                      const std::vector<T> HostProgram::*field) {
    size_t n = 0;
    for (auto* p : progs) n += (p->*field).size();
    std::vector<T> out;
    out.reserve(n);
    for (auto* p : progs) out.insert(out.end(), (p->*field).begin(), (p->*field).end());
    return out;
}

int32_t upload_static(const std::vector<const HostProgram*>& progs, const Plan& P,
                      uint8_t* arena, hipStream_t s) {
    auto put = [&](uint64_t off, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(arena + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    std::vector<int32_t> ngo = concat(progs, &HostProgram::ng_off);
    std::vector<int32_t> ngl = concat(progs, &HostProgram::ng_lits);
    std::vector<int32_t> mo = concat(progs, &HostProgram::map_off);
    std::vector<MapEntry> mi = concat(progs, &HostProgram::map_ent);
    std::vector<int32_t> rh = concat(progs, &HostProgram::rule_head);
    // the static per-rule score: the head's Jeroslow-Wang score, or its
    // occurrence count (also the start of the activity and the learned
    // Decision's fallback)
    std::vector<int32_t> ro = concat(progs, P.decision == ASP_DECISION_JW ? &HostProgram::rule_jw
                                                                           : &HostProgram::rule_occ);
    std::vector<int32_t> rord = concat(progs, P.decision == ASP_DECISION_JW
                                                  ? &HostProgram::rule_by_jw
                                                  : &HostProgram::rule_by_occ);
    std::vector<int32_t> rbo = concat(progs, &HostProgram::rb_off);
    std::vector<int32_t> rbl = concat(progs, &HostProgram::rb_lits);
    HIPCHK(put(P.off_desc, P.desc.data(), sizeof(InstDesc) * P.desc.size()));
    HIPCHK(put(P.off_order, P.order.data(), 4 * P.order.size()));
    HIPCHK(put(P.off_slotoff, P.slot_off.data(), 8 * P.slot_off.size()));
    HIPCHK(put(P.off_ngo, ngo.data(), 4 * ngo.size()));
    HIPCHK(put(P.off_ngl, ngl.data(), 4 * ngl.size()));
    HIPCHK(put(P.off_mo, mo.data(), 4 * mo.size()));
    HIPCHK(put(P.off_mi, mi.data(), sizeof(MapEntry) * mi.size()));
    HIPCHK(put(P.off_rh, rh.data(), 4 * rh.size()));
    HIPCHK(put(P.off_ro, ro.data(), 4 * ro.size()));
    HIPCHK(put(P.off_rord, rord.data(), 4 * rord.size()));
    HIPCHK(put(P.off_rbo, rbo.data(), 4 * rbo.size()));
    HIPCHK(put(P.off_rbl, rbl.data(), 4 * rbl.size()));
    HIPCHK(hipStreamSynchronize(s));  // host staging vectors die here
    return ASP_OK;
}

KArgs make_args(const Plan& P, uint8_t* arena, int32_t mode, const LaunchClass& lc) {
    KArgs a{};
    a.inst = (const InstDesc*)(arena + P.off_desc);
    a.order = (const int32_t*)(arena + P.off_order);
    a.first = lc.first;
    a.count = lc.count;
    a.mode = mode;
    a.ng_off = (const int32_t*)(arena + P.off_ngo);
    a.ng_lits = (const int32_t*)(arena + P.off_ngl);
    a.map_off = (const int32_t*)(arena + P.off_mo);
    a.map_ent = (const MapEntry*)(arena + P.off_mi);
    a.rule_head = (const int32_t*)(arena + P.off_rh);
    a.rule_occ = (const int32_t*)(arena + P.off_ro);
    a.rule_score = (const int32_t*)(arena + P.off_rs);
    a.rule_ord = (const int32_t*)(arena + P.off_rord);
    a.rule_ord_sc = (const int32_t*)(arena + P.off_rords);
    a.rb_off = (const int32_t*)(arena + P.off_rbo);
    a.rb_lits = (const int32_t*)(arena + P.off_rbl);
    a.slots = arena + P.off_slots;
    a.slot_off = (const int64_t*)(arena + P.off_slotoff);
    a.verdicts = (int32_t*)(arena + P.off_verd);
    a.stats = (DevStats*)(arena + P.off_stats);
    a.models = arena + P.off_models;
    a.W = P.W;
    a.gate_mode = P.gate;
    a.decision = P.decision;
    a.fallback_after = P.fallback_after;
    a.learning = P.learning;
    a.max_models = P.max_models;
    a.learn_k = P.learn_k;
    a.restart_every = P.restart_every;
    a.model_store = P.model_store;
    a.lookahead = P.lookahead;
    a.words = lc.words;
    a.awords = lc.awords;
    a.step_mask = 0;
    a.max_steps = -1;
    a.max_conflicts = -1;
    a.cap_ng = P.cap_ng;
    a.cap_lits = P.cap_lits;
    a.max_ticks = 0;
    return a;
}

void apply_limits(KArgs& a, const Plan& P, const asp_limits* lim, const DeviceInfo& di) {
    a.max_conflicts = lim ? lim->max_conflicts : -1;
    int64_t ms = (lim && lim->max_ms > 0) ? lim->max_ms : kDefaultMaxMs;
    a.max_ticks = di.clock_khz > 0 ? (uint64_t)ms * (uint64_t)di.clock_khz : 0;
    // step guard: between two conflicts, or two answer sets, a search runs at
    // most 3V + 4 steps (no guard when every answer set is asked for)
    if (a.max_conflicts >= 0 && P.max_models > 0)
        a.max_steps = (a.max_conflicts + P.max_models + 2) * (3 * P.Vmax + P.Rhmax + 16) + 16;
    else
        a.max_steps = -1;
}


int64_t ticks_ns(uint64_t t) {
    return g_clock_khz > 0 ? (int64_t)((double)t * 1e6 / (double)g_clock_khz) : 0;
}

void to_stats(const DevStats& d, asp_stats* s) {
    s->rounds = d.rounds;
    s->visits = d.visits;
    s->literal_checks = d.checks;
    s->propagations = d.props;
    s->decisions = d.decisions;
    s->conflicts = d.conflicts;
    s->learned = d.learned;
    s->learned_len = d.learned_len;
    s->gate_failures = d.gate_fail;
    s->completes = d.completes;
    s->trace_hash = d.hash;
    s->status = d.status;
    s->last_step = d.last_step;
    s->models = d.models;
    s->restarts = d.restarts;
    s->exhausted = d.exhausted;
    s->reserved = 0;
    s->ns_total = ticks_ns(d.t_total);
    s->ns_round = ticks_ns(d.t_round);
    s->ns_learn = ticks_ns(d.t_learn);
    s->ns_decide = ticks_ns(d.t_decide);
    s->ns_gate = ticks_ns(d.t_gate);
}

void ctrl_stats(const SlotCtrl& k, asp_stats* s) {
    s->rounds = k.rounds;
    s->visits = k.visits;
    s->literal_checks = k.checks;
    s->propagations = k.props;
    s->decisions = k.decisions;
    s->conflicts = k.conflicts;
    s->learned = k.learned;
    s->learned_len = k.learned_len;
    s->gate_failures = k.gate_fail;
    s->completes = k.completes;
    s->trace_hash = k.hash;
    s->status = k.status;
    s->last_step = k.last_step;
    s->ns_total = s->ns_round = s->ns_learn = s->ns_decide = s->ns_gate = 0;
    s->models = k.models;
    s->restarts = k.restarts;
    s->exhausted = k.exhausted;
    s->reserved = 0;
}

int32_t check_launch(const Plan& P, const DeviceInfo& di) {
    if (!di.ok) return fail(ASP_E_DEVICE, "no HIP device");
    if (P.max_lds() > di.max_lds)
        return fail(ASP_E_CAPACITY, "largest instance needs " + std::to_string(P.max_lds()) +
                                        " bytes of LDS, device allows " +
                                        std::to_string(di.max_lds));
    for (const LaunchClass& c : P.classes)
        (void)set_max_lds(c.threads, c.lds);  // best effort: older runtimes ignore it
    return ASP_OK;
}

// single program: run the step kernel on slot 0
int32_t run_single(asp_program* p, hipStream_t s, int32_t mode, int32_t mask, int64_t steps,
                   const asp_limits* lim) {
    DeviceInfo di = device_info();
    int32_t rc = check_launch(p->plan, di);
    if (rc) return rc;
    const LaunchClass& lc = p->plan.classes[0];
    KArgs a = make_args(p->plan, p->arena, mode, lc);
    apply_limits(a, p->plan, lim, di);
    a.step_mask = mask;
    a.max_steps = steps;
    HIPCHK(launch_search(a, lc.threads, 1, lc.lds, s));
    HIPCHK(hipStreamSynchronize(s));
    return ASP_OK;
}

// the single program's slot (instance 0)
SlotLayout slot0(const asp_program* p) {
    return slot_layout(p->hp.V, p->hp.Rh, p->opt.W, p->opt.learned_cap_ng, p->opt.learned_cap_lits,
                       p->opt.learning);
}

SlotCtrl* ctrl_ptr(asp_program* p) { return (SlotCtrl*)(p->arena + p->plan.off_slots + slot0(p).ctrl); }

int32_t read_ctrl(asp_program* p, hipStream_t s, SlotCtrl* out) {
    HIPCHK(hipMemcpyAsync(out, ctrl_ptr(p), sizeof(SlotCtrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ASP_OK;
}

template <class T>
T* slot_arr(asp_program* p, int64_t off) {
    return (T*)(p->arena + p->plan.off_slots + off);
}

// ------------------------------------------------------ decision scores
// Upload atom scores of instance i and gather its rule scores on the device.
int32_t put_scores(const Plan& P, uint8_t* arena, int32_t i, const int32_t* scores, hipStream_t s) {
    const InstDesc& d = P.desc[i];
    std::vector<int32_t> sc(scores, scores + d.A + 1);
    sc[0] = 0;
    HIPCHK(hipMemcpyAsync(arena + P.off_asc + 4 * (uint64_t)d.ascore, sc.data(), 4 * sc.size(),
                          hipMemcpyHostToDevice, s));
    ScorerArgs a{};
    a.inst = (const InstDesc*)(arena + P.off_desc);
    a.rule_head = (const int32_t*)(arena + P.off_rh);
    a.atom_score = (int32_t*)(arena + P.off_asc);
    a.rule_score = (int32_t*)(arena + P.off_rs);
    a.rule_ord_sc = (int32_t*)(arena + P.off_rords);
    a.sort_tmp = (unsigned long long*)(arena + P.off_rsort);
    a.inst_list = nullptr;   // gather instance i only
    a.single = i;
    HIPCHK(launch_rule_scores(a, s));
    HIPCHK(hipStreamSynchronize(s));
    return ASP_OK;
}

int32_t get_scores(const Plan& P, uint8_t* arena, int32_t i, int32_t* out, hipStream_t s) {
    const InstDesc& d = P.desc[i];
    HIPCHK(hipMemcpyAsync(out, arena + P.off_asc + 4 * (uint64_t)d.ascore, 4 * ((size_t)d.A + 1),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ASP_OK;
}

// ------------------------------------------------------------- scorer
bool bf16_code(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f == (float)(int)f && f >= -127.f && f <= 127.f;
}

int32_t check_weights(const asp_scorer_weights* w) {
    if (!w) return fail(ASP_E_INVALID, "null scorer weights");
    auto mats = [&](const uint16_t* m, size_t n) {
        for (size_t i = 0; i < n; ++i)
            if (!bf16_code(m[i])) return false;
        return true;
    };
    const size_t HH = (size_t)ASP_SCORER_L * ASP_SCORER_H * ASP_SCORER_H;
    const size_t FH = (size_t)ASP_SCORER_F * ASP_SCORER_H;
    if (!mats(w->Ev, FH) || !mats(w->Ec, FH) || !mats(w->P, HH) || !mats(w->N, HH) ||
        !mats(w->S, HH) || !mats(w->Q, HH) || !mats(w->R, HH) || !mats(w->T, HH))
        return fail(ASP_E_INVALID, "scorer matrices must hold integers in [-127, 127]");
    const int32_t lim = 1 << 24;
    auto vecs = [&](const int32_t* v, size_t n, int32_t m) {
        for (size_t i = 0; i < n; ++i)
            if (v[i] < -m || v[i] > m) return false;
        return true;
    };
    const size_t LH = (size_t)ASP_SCORER_L * ASP_SCORER_H;
    if (!vecs(w->ev, ASP_SCORER_H, lim) || !vecs(w->ec, ASP_SCORER_H, lim) ||
        !vecs(w->bc, LH, lim) || !vecs(w->bv, LH, lim) || !vecs(&w->bo, 1, lim))
        return fail(ASP_E_INVALID, "scorer biases must be within +-2^24");
    if (!vecs(w->wo, ASP_SCORER_H, 127)) return fail(ASP_E_INVALID, "scorer readout must be in [-127, 127]");
    return ASP_OK;
}

void scorer_plan(const std::vector<const HostProgram*>& progs, ScorerPlan& S) {
    if (S.planned) return;
    const size_t n = progs.size();
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    S.hv_off.assign(n, 0);
    S.hc_off.assign(n, 0);
    S.vt.clear();
    S.ct.clear();
    S.list.resize(n);
    for (size_t i = 0; i < n; ++i) {
        const HostProgram& h = *progs[i];
        for (int32_t r = 0; r <= h.V; r += 64) S.vt.push_back({(int32_t)i, r});
        for (int32_t r = 0; r < (int32_t)h.n_nogoods(); r += 64) S.ct.push_back({(int32_t)i, r});
        S.list[i] = (int32_t)i;
    }
    S.off_w = take(sizeof(asp_scorer_weights));
    S.off_hvo = take(8 * n);
    S.off_hco = take(8 * n);
    S.off_vt = take(sizeof(ScorerTile) * S.vt.size());
    S.off_ct = take(sizeof(ScorerTile) * S.ct.size());
    S.off_list = take(4 * n);
    uint64_t atoms = 0;
    for (auto* p : progs) atoms += (uint64_t)p->A;
    S.off_lab = take(atoms + 1);
    S.off_train = take(4 * (uint64_t)(3 * 65 + 66 + kMaxTrainSteps));
    for (size_t i = 0; i < n; ++i) {
        S.hv_off[i] = (int64_t)take(64 * ((uint64_t)progs[i]->V + 1));
        S.hc_off[i] = (int64_t)take(64 * std::max<uint64_t>(1, progs[i]->n_nogoods()));
    }
    S.total = o;
    S.planned = true;
}

ScorerArgs scorer_args(const std::vector<const HostProgram*>& progs, const Plan& P, uint8_t* arena,
                       const ScorerPlan& S, uint8_t* ws);

// Enqueue the scorer over every instance of the plan on stream s.
int32_t run_scorer(const std::vector<const HostProgram*>& progs, const Plan& P, uint8_t* arena,
                   ScorerPlan& S, const asp_scorer_weights* w, uint8_t* ws, uint64_t ws_bytes,
                   hipStream_t s) {
    int32_t rc = check_weights(w);
    if (rc) return rc;
    if (!ws || (uintptr_t)ws % kAlign) return fail(ASP_E_INVALID, "workspace must be 256-byte aligned");
    scorer_plan(progs, S);
    if (ws_bytes < S.total)
        return fail(ASP_E_CAPACITY, "scorer workspace of " + std::to_string(ws_bytes) +
                                        " bytes, need " + std::to_string(S.total));
    DeviceInfo di = device_info();
    if (!di.ok) return fail(ASP_E_DEVICE, "no HIP device");
    S.w = *w;
    HIPCHK(hipMemcpyAsync(ws + S.off_w, &S.w, sizeof(S.w), hipMemcpyHostToDevice, s));
    if (S.uploaded_to != ws) {
        HIPCHK(hipMemcpyAsync(ws + S.off_hvo, S.hv_off.data(), 8 * S.hv_off.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(ws + S.off_hco, S.hc_off.data(), 8 * S.hc_off.size(), hipMemcpyHostToDevice, s));
        if (!S.vt.empty())
            HIPCHK(hipMemcpyAsync(ws + S.off_vt, S.vt.data(), sizeof(ScorerTile) * S.vt.size(),
                                  hipMemcpyHostToDevice, s));
        if (!S.ct.empty())
            HIPCHK(hipMemcpyAsync(ws + S.off_ct, S.ct.data(), sizeof(ScorerTile) * S.ct.size(),
                                  hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(ws + S.off_list, S.list.data(), 4 * S.list.size(), hipMemcpyHostToDevice, s));
        S.uploaded_to = ws;
    }
    ScorerArgs a = scorer_args(progs, P, arena, S, ws);
    auto grid = [&](size_t tiles) { return (int)std::max<size_t>(1, std::min<size_t>(tiles, (size_t)di.cus * 8)); };
    HIPCHK(launch_scorer_embed(a, grid(S.vt.size() + S.ct.size()), s));
    for (int l = 0; l < ASP_SCORER_L; ++l) {
        HIPCHK(launch_scorer_nogoods(a, l, grid(S.ct.size()), s));
        HIPCHK(launch_scorer_vars(a, l, grid(S.vt.size()), s));
    }
    HIPCHK(launch_rule_scores(a, s));
    return ASP_OK;
}

ScorerArgs scorer_args(const std::vector<const HostProgram*>& progs, const Plan& P, uint8_t* arena,
                       const ScorerPlan& S, uint8_t* ws) {
    ScorerArgs a{};
    a.inst = (const InstDesc*)(arena + P.off_desc);
    a.ng_off = (const int32_t*)(arena + P.off_ngo);
    a.ng_lits = (const int32_t*)(arena + P.off_ngl);
    a.map_off = (const int32_t*)(arena + P.off_mo);
    a.map_ent = (const MapEntry*)(arena + P.off_mi);
    a.rule_head = (const int32_t*)(arena + P.off_rh);
    a.w = ws + S.off_w;
    a.hv_off = (const int64_t*)(ws + S.off_hvo);
    a.hc_off = (const int64_t*)(ws + S.off_hco);
    a.vtiles = (const ScorerTile*)(ws + S.off_vt);
    a.ctiles = (const ScorerTile*)(ws + S.off_ct);
    a.inst_list = (const int32_t*)(ws + S.off_list);
    a.n_vtiles = (int32_t)S.vt.size();
    a.n_ctiles = (int32_t)S.ct.size();
    a.n_inst = (int32_t)progs.size();
    a.ws = ws;
    a.atom_score = (int32_t*)(arena + P.off_asc);
    a.rule_score = (int32_t*)(arena + P.off_rs);
    a.rule_ord_sc = (int32_t*)(arena + P.off_rords);
    a.sort_tmp = (unsigned long long*)(arena + P.off_rsort);
    return a;
}

}  // namespace

// ------------------------------------------------- allocation-free solve
// Device memory of asp_solve_noalloc: the program's tables, its search slot
// and the results, laid out as a bound arena.  Each GPU the library runs on
// holds its own copy until the process ends.  In host code `scratch` is only
// a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) uint8_t scratch[ASP_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per
// device, with that device current).
int32_t scratch_base(uint8_t** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ASP_E_DEVICE, "device index beyond 64");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(ASP_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
        g_scratch[dev] = (uint8_t*)ptr;
    }
    *out = g_scratch[dev];
    return ASP_OK;
}

// Copy one program's static tables into an arena laid out by P, straight
// from the program's own arrays (no staging buffers).
int32_t upload_one(const HostProgram& h, const Plan& P, int32_t decision, uint8_t* arena,
                   hipStream_t s) {
    auto put = [&](uint64_t off, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(arena + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    const std::vector<int32_t>& ro = decision == ASP_DECISION_JW ? h.rule_jw : h.rule_occ;
    const std::vector<int32_t>& rord = decision == ASP_DECISION_JW ? h.rule_by_jw : h.rule_by_occ;
    HIPCHK(put(P.off_desc, P.desc.data(), sizeof(InstDesc) * P.desc.size()));
    HIPCHK(put(P.off_order, P.order.data(), 4 * P.order.size()));
    HIPCHK(put(P.off_slotoff, P.slot_off.data(), 8 * P.slot_off.size()));
    HIPCHK(put(P.off_ngo, h.ng_off.data(), 4 * h.ng_off.size()));
    HIPCHK(put(P.off_ngl, h.ng_lits.data(), 4 * h.ng_lits.size()));
    HIPCHK(put(P.off_mo, h.map_off.data(), 4 * h.map_off.size()));
    HIPCHK(put(P.off_mi, h.map_ent.data(), sizeof(MapEntry) * h.map_ent.size()));
    HIPCHK(put(P.off_rh, h.rule_head.data(), 4 * h.rule_head.size()));
    HIPCHK(put(P.off_ro, ro.data(), 4 * ro.size()));
    HIPCHK(put(P.off_rord, rord.data(), 4 * rord.size()));
    HIPCHK(put(P.off_rbo, h.rb_off.data(), 4 * h.rb_off.size()));
    HIPCHK(put(P.off_rbl, h.rb_lits.data(), 4 * h.rb_lits.size()));
    return ASP_OK;
}

}  // namespace

// ============================================================== C ABI
extern "C" {

const char* asp_status_str(int32_t st) {
    switch (st) {
    case ASP_OK: return "ok";
    case ASP_SAT: return "sat";
    case ASP_UNSAT: return "unsat";
    case ASP_UNKNOWN: return "unknown";
    case ASP_FIXPOINT: return "fixpoint";
    case ASP_CONFLICT: return "conflict";
    case ASP_RUNNING: return "running";
    case ASP_E_INVALID: return "invalid input";
    case ASP_E_CAPACITY: return "capacity exceeded";
    case ASP_E_DEVICE: return "device error";
    case ASP_E_STATE: return "wrong call order";
    case ASP_E_INTERNAL: return "internal error";
    case ASP_E_TIMEOUT: return "device time limit";
    default: return "unknown status";
    }
}

int32_t asp_last_error(char* buf, uint64_t len) {
    if (!buf || len == 0) return ASP_E_INVALID;
    size_t n = std::min<size_t>(g_err.size(), (size_t)len - 1);
    memcpy(buf, g_err.data(), n);
    buf[n] = 0;
    return ASP_OK;
}

int32_t asp_load_program(int32_t n_atoms, int32_t n_rules, const int32_t* head,
                         const int64_t* body_off, const int32_t* body_lits,
                         const asp_options* opt, asp_program** out, asp_sizes* sizes) {
    if (!out) return fail(ASP_E_INVALID, "null output handle");
    *out = nullptr;
    asp_options o = opt ? *opt : default_options();
    if (o.W < 1 || o.W > kMaxW) return fail(ASP_E_INVALID, "W must be in 1..64");
    if (o.gate != ASP_GATE_UNFOUNDED && o.gate != ASP_GATE_ALLDEC)
        return fail(ASP_E_INVALID, "unknown gate option");
    if (o.learned_cap_ng < 1 || o.learned_cap_lits < 1 || o.learned_cap_ng > (1 << 29) ||
        o.learned_cap_lits > ((int64_t)1 << 29))
        return fail(ASP_E_INVALID, "learned capacities must be in 1..2^29");
    if (o.decision != ASP_DECISION_OCC && o.decision != ASP_DECISION_SCORE &&
        o.decision != ASP_DECISION_JW && o.decision != ASP_DECISION_ACTIVITY)
        return fail(ASP_E_INVALID, "unknown decision heuristic");
    if (o.learning != ASP_LEARN_FWD && o.learning != ASP_LEARN_RES)
        return fail(ASP_E_INVALID, "unknown learning step");
    if (o.learn_conflicts < 0 || o.learn_conflicts > 8)
        return fail(ASP_E_INVALID, "learn_conflicts must be in 0..8");
    if (o.lookahead < 0 || o.lookahead > 8)
        return fail(ASP_E_INVALID, "lookahead must be in 0..8");
    if (o.lookahead > 1 && o.learning != ASP_LEARN_FWD)
        return fail(ASP_E_INVALID, "the lookahead Decision needs Fwd-learning");
    if (o.max_models < 0 || o.max_models > ((int64_t)1 << 30) || o.restart_every < 0)
        return fail(ASP_E_INVALID, "max_models must be in 0..2^30, restart_every >= 0");
    if ((int64_t)n_atoms * (o.max_models > 0 ? o.max_models : 1) > ((int64_t)1 << 34))
        return fail(ASP_E_INVALID, "answer-set store beyond 2^34 bytes");
    std::unique_ptr<asp_program> p(new asp_program());
    std::string err;
    int rc = encode_program(n_atoms, n_rules, head, body_off, body_lits, &p->hp, &err);
    if (rc) return fail(ASP_E_INVALID, err);
    p->opt = o;
    std::vector<const HostProgram*> one{&p->hp};
    rc = make_plan(one, o, 256, 1, p->plan);
    if (rc) return rc;
    p->load_plan = p->plan;
    if (sizes) {
        sizes->n_atoms = p->hp.A;
        sizes->n_rules_headed = p->hp.Rh;
        sizes->n_constraints = p->hp.Rc;
        sizes->n_vars = p->hp.V;
        sizes->n_nogoods = p->hp.n_nogoods();
        sizes->n_lits = (int64_t)p->hp.ng_lits.size();
        sizes->n_units = p->hp.u1 - p->hp.u0;
        sizes->device_bytes = p->plan.total;
    }
    *out = p.release();
    return ASP_OK;
}

int32_t asp_free_program(asp_program* prog) {
    delete prog;
    return ASP_OK;
}

int32_t asp_program_nogoods(const asp_program* p, int32_t* off, int32_t* lits) {
    if (!p) return fail(ASP_E_INVALID, "null program");
    if (off) memcpy(off, p->hp.ng_off.data(), 4 * p->hp.ng_off.size());
    if (lits && !p->hp.ng_lits.empty()) memcpy(lits, p->hp.ng_lits.data(), 4 * p->hp.ng_lits.size());
    return ASP_OK;
}

int32_t asp_bind_device(asp_program* p, void* dev_arena, uint64_t bytes, void* stream,
                        const asp_schedule* sched) {
    if (!p || !dev_arena) return fail(ASP_E_INVALID, "null program or arena");
    if ((uintptr_t)dev_arena % kAlign) return fail(ASP_E_INVALID, "arena must be 256-byte aligned");
    int32_t threads = sched ? sched->threads : 256;
    if (!valid_threads(threads)) return fail(ASP_E_INVALID, "threads must be 64..1024, power of 2");
    std::vector<const HostProgram*> one{&p->hp};
    Plan P;
    int32_t rc = make_plan(one, p->opt, threads, 1, P);
    if (rc) return rc;
    if (bytes < P.total)
        return fail(ASP_E_CAPACITY, "arena of " + std::to_string(bytes) + " bytes, need " +
                                        std::to_string(P.total));
    hipStream_t s = (hipStream_t)stream;
    p->bound = false;
    p->plan = P;
    p->arena = (uint8_t*)dev_arena;
    p->bytes = bytes;
    p->threads = threads;
    rc = upload_static(one, P, p->arena, s);
    if (rc) return rc;
    rc = run_single(p, s, MODE_RESET, 0, 0, nullptr);
    if (rc) return rc;
    p->bound = true;
    p->scores_ready = false;
    return ASP_OK;
}

int32_t asp_set_scores(asp_program* p, const int32_t* scores, void* stream) {
    if (!p || !p->bound) return fail(ASP_E_STATE, "program not bound to a device arena");
    if (!scores) return fail(ASP_E_INVALID, "null scores");
    int32_t rc = put_scores(p->plan, p->arena, 0, scores, (hipStream_t)stream);
    if (rc) return rc;
    p->scores_ready = true;
    return ASP_OK;
}

int32_t asp_get_scores(asp_program* p, int32_t* scores, void* stream) {
    if (!p || !p->bound) return fail(ASP_E_STATE, "program not bound to a device arena");
    if (!scores) return fail(ASP_E_INVALID, "null scores");
    return get_scores(p->plan, p->arena, 0, scores, (hipStream_t)stream);
}

int32_t asp_scorer_workspace(const asp_program* p, uint64_t* bytes) {
    if (!p || !bytes) return fail(ASP_E_INVALID, "null program or output");
    ScorerPlan S;
    scorer_plan({&p->hp}, S);
    *bytes = S.total;
    return ASP_OK;
}

int32_t asp_score_program(asp_program* p, const asp_scorer_weights* w, void* ws, uint64_t ws_bytes,
                          void* stream) {
    if (!p || !p->bound) return fail(ASP_E_STATE, "program not bound to a device arena");
    hipStream_t s = (hipStream_t)stream;
    int32_t rc = run_scorer({&p->hp}, p->plan, p->arena, p->scorer, w, (uint8_t*)ws, ws_bytes, s);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(s));
    p->scores_ready = true;
    return ASP_OK;
}

int32_t asp_propagate(asp_program* p, void* stream, int32_t max_rounds, asp_prop_result* out) {
    if (!p || !p->bound) return fail(ASP_E_STATE, "program not bound to a device arena");
    hipStream_t s = (hipStream_t)stream;
    SlotCtrl b, e;
    int32_t rc = read_ctrl(p, s, &b);
    if (rc) return rc;
    if (b.status != ASP_RUNNING) return b.status;
    int64_t steps = max_rounds > 0 ? (int64_t)max_rounds + (b.init_done ? 0 : 1) : INT64_MAX;
    rc = run_single(p, s, MODE_STEPS, (1 << STEP_INIT) | (1 << STEP_ROUND), steps, nullptr);
    if (rc) return rc;
    rc = read_ctrl(p, s, &e);
    if (rc) return rc;
    int32_t st;
    if (e.status != ASP_RUNNING) st = e.status;
    else if (e.pend_kind == 1) st = ASP_CONFLICT;
    else if (e.qt == e.qh) st = ASP_FIXPOINT;
    else st = ASP_RUNNING;
    if (out) {
        out->status = st;
        out->conflict_id = e.pend_kind == 1 ? e.pending : -1;
        out->rounds = e.rounds - b.rounds;
        out->implied = e.props - b.props;
        out->visits = e.visits - b.visits;
        out->literal_checks = e.checks - b.checks;
    }
    return st;
}

int32_t asp_analyze_conflict(asp_program* p, void* stream, const asp_limits* lim,
                             int32_t* learned_lits, int32_t cap, int32_t* learned_len,
                             int32_t* backjump_level) {
    if (!p || !p->bound) return fail(ASP_E_STATE, "program not bound to a device arena");
    hipStream_t s = (hipStream_t)stream;
    SlotCtrl b, e;
    int32_t rc = read_ctrl(p, s, &b);
    if (rc) return rc;
    if (b.status != ASP_RUNNING || b.pend_kind != 1)
        return fail(ASP_E_STATE, "no pending propagation conflict");
    rc = run_single(p, s, MODE_STEPS, 1 << STEP_LEARN, 1, lim);
    if (rc) return rc;
    rc = read_ctrl(p, s, &e);
    if (rc) return rc;
    if (e.status != ASP_RUNNING) return e.status;
    if (e.status == ASP_RUNNING && e.pend_kind != 0) return fail(ASP_E_INTERNAL, "learning did not run");
    int32_t off[2];
    const SlotLayout L0 = slot0(p);
    HIPCHK(hipMemcpyAsync(off, slot_arr<int32_t>(p, L0.l_off) + (e.n_learned - 1), 8,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int32_t len = off[1] - off[0];
    if (learned_len) *learned_len = len;
    if (backjump_level) *backjump_level = e.cdl;
    if (learned_lits) {
        if (cap < len) return fail(ASP_E_CAPACITY, "learned nogood longer than cap");
        HIPCHK(hipMemcpyAsync(learned_lits, slot_arr<int32_t>(p, L0.l_lits) + off[0],
                              4 * (size_t)len, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    return ASP_OK;
}

int32_t asp_run_steps(asp_program* p, void* stream, const asp_limits* lim, int64_t n_steps,
                      asp_stats* stats) {
    if (!p || !p->bound) return fail(ASP_E_STATE, "program not bound to a device arena");
    if (p->opt.decision == ASP_DECISION_SCORE && !p->scores_ready)
        return fail(ASP_E_STATE, "decision scores not set");
    hipStream_t s = (hipStream_t)stream;
    int32_t rc = run_single(p, s, MODE_STEPS, 0xff, n_steps < 0 ? INT64_MAX : n_steps, lim);
    if (rc) return rc;
    SlotCtrl e;
    rc = read_ctrl(p, s, &e);
    if (rc) return rc;
    if (stats) ctrl_stats(e, stats);
    return e.status;
}

int32_t asp_solve(asp_program* p, void* stream, const asp_limits* lim, uint8_t* model,
                  asp_stats* stats) {
    if (!p || !p->bound) return fail(ASP_E_STATE, "program not bound to a device arena");
    if (p->opt.decision == ASP_DECISION_SCORE && !p->scores_ready)
        return fail(ASP_E_STATE, "decision scores not set");
    hipStream_t s = (hipStream_t)stream;
    DeviceInfo di = device_info();
    int32_t rc = check_launch(p->plan, di);
    if (rc) return rc;
    const LaunchClass& lc = p->plan.classes[0];
    KArgs a = make_args(p->plan, p->arena, MODE_SOLVE, lc);
    apply_limits(a, p->plan, lim, di);
    HIPCHK(launch_search(a, lc.threads, 1, lc.lds, s));
    DevStats d;
    int32_t verdict = 0;
    HIPCHK(hipMemcpyAsync(&d, a.stats, sizeof(DevStats), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&verdict, a.verdicts, 4, hipMemcpyDeviceToHost, s));
    if (model && p->hp.A > 0)
        HIPCHK(hipMemcpyAsync(model, a.models, (size_t)p->hp.A, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (stats) to_stats(d, stats);
    return verdict;
}

int32_t asp_solve_noalloc(const asp_program* p, void* stream, const asp_limits* lim,
                          uint8_t* model, asp_stats* stats) {
    if (!p) return fail(ASP_E_INVALID, "null program");
    if (p->opt.decision == ASP_DECISION_SCORE)
        return fail(ASP_E_INVALID, "score-driven Decision needs a bound arena (asp_set_scores)");
    const Plan& P = p->load_plan;
    if (P.total > (uint64_t)ASP_NOALLOC_MAX_BYTES)
        return fail(ASP_E_CAPACITY, "program needs " + std::to_string(P.total) +
                                        " bytes of device memory, the allocation-free solve has " +
                                        std::to_string((uint64_t)ASP_NOALLOC_MAX_BYTES) +
                                        " (lower learned_cap_lits / learned_cap_ng)");
    uint8_t* base = nullptr;
    int32_t rc = scratch_base(&base);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    DeviceInfo di = device_info();
    rc = check_launch(P, di);
    if (rc) return rc;
    rc = upload_one(p->hp, P, p->opt.decision, base, s);
    if (rc) return rc;
    // the solve kernel resets every part of the slot it reads (MODE_SOLVE),
    // and writes the verdict, the counters and the answer set it reports,
    // so nothing left by an earlier call is read
    const LaunchClass& lc = P.classes[0];
    KArgs a = make_args(P, base, MODE_SOLVE, lc);
    apply_limits(a, P, lim, di);
    HIPCHK(launch_search(a, lc.threads, 1, lc.lds, s));
    DevStats d;
    int32_t verdict = 0;
    HIPCHK(hipMemcpyAsync(&d, a.stats, sizeof(DevStats), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&verdict, a.verdicts, 4, hipMemcpyDeviceToHost, s));
    if (model && p->hp.A > 0)
        HIPCHK(hipMemcpyAsync(model, a.models, (size_t)p->hp.A, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (stats) to_stats(d, stats);
    return verdict;
}

int32_t asp_get_models(asp_program* p, void* stream, uint8_t* models, int64_t max_out,
                       int64_t* found) {
    if (!p || !p->bound) return fail(ASP_E_STATE, "program not bound to a device arena");
    if (max_out < 0 || (max_out > 0 && !models)) return fail(ASP_E_INVALID, "bad output buffer");
    hipStream_t s = (hipStream_t)stream;
    SlotCtrl k;
    int32_t rc = read_ctrl(p, s, &k);
    if (rc) return rc;
    const int64_t n = std::min(std::min(k.models, p->plan.model_store), max_out);
    if (n > 0 && p->hp.A > 0)
        HIPCHK(hipMemcpyAsync(models, p->arena + p->plan.off_models, (size_t)(n * p->hp.A),
                              hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (found) *found = k.models;
    return ASP_OK;
}

int32_t asp_state_export(asp_program* p, void* stream, asp_state* st) {
    if (!p || !p->bound || !st) return fail(ASP_E_STATE, "program not bound or null state");
    hipStream_t s = (hipStream_t)stream;
    SlotCtrl k;
    int32_t rc = read_ctrl(p, s, &k);
    if (rc) return rc;
    const int32_t V = p->hp.V, W = p->opt.W;
    st->n_vars = V;
    st->W = W;
    st->cdl = k.cdl;
    st->frontier_len = k.qt - k.qh;
    st->n_learned = k.n_learned;
    st->pending = k.pend_kind == 1 ? k.pending : -1;
    st->learned_lits = k.learned_lits;
    st->initialised = k.init_done;
    st->status = k.status;
    st->score_mode = k.use_score;
    st->consec = k.consec;
    st->dec_open = k.dec_open;
    ctrl_stats(k, &st->stats);
    if (!st->val) return ASP_OK;
    const SlotLayout L = slot0(p);
    auto get = [&](void* dst, int64_t off, size_t bytes) -> hipError_t {
        if (!dst || bytes == 0) return hipSuccess;
        return hipMemcpyAsync(dst, p->arena + p->plan.off_slots + off, bytes,
                              hipMemcpyDeviceToHost, s);
    };
    HIPCHK(get(st->val, L.val8, (size_t)V + 1));
    HIPCHK(get(st->lvl, L.lvl, 4 * ((size_t)V + 1)));
    HIPCHK(get(st->deps, L.deps, 8 * ((size_t)V + 1) * W));
    HIPCHK(get(st->dec, L.dec, 4 * ((size_t)k.cdl + 1)));
    HIPCHK(get(st->frontier, L.trail + 4 * (int64_t)k.qh, 4 * (size_t)(k.qt - k.qh)));
    HIPCHK(get(st->learned_off, L.l_off, 4 * ((size_t)k.n_learned + 1)));
    HIPCHK(get(st->learned, L.l_lits, 4 * (size_t)k.learned_lits));
    HIPCHK(hipStreamSynchronize(s));
    if (st->dec) {
        st->dec[0] = 0;
        if (k.cdl >= 1) st->dec[1] = 0;
    }
    if (st->frontier) std::sort(st->frontier, st->frontier + (k.qt - k.qh));
    if (p->opt.learning == ASP_LEARN_FWD && (st->lvl || st->deps)) {
        // The Fwd-learning search keeps no per-variable levels and leaves the
        // Deps of unassigned variables stale: the trail is in assignment
        // order and level l (2..cdl) begins at tlim[l], so a variable's level
        // is the highest l <= cdl whose segment starts at or before its trail
        // position (1 below tlim[2]); unassigned variables get level 0 and
        // empty Deps.
        std::vector<int32_t> trail((size_t)std::max(k.qt, 0)), tlim((size_t)k.cdl + 2, 0);
        HIPCHK(get(trail.data(), L.trail, 4 * trail.size()));
        HIPCHK(get(tlim.data(), L.tlim, 4 * tlim.size()));
        std::vector<int8_t> val((size_t)V + 1);
        HIPCHK(get(val.data(), L.val8, (size_t)V + 1));
        HIPCHK(hipStreamSynchronize(s));
        if (st->lvl) {
            std::fill(st->lvl, st->lvl + V + 1, 0);
            int32_t l = 1;
            for (int32_t q = 0; q < k.qt; ++q) {
                while (l < k.cdl && tlim[l + 1] <= q) ++l;
                st->lvl[trail[q]] = l;
            }
        }
        if (st->deps)
            for (int32_t v = 0; v <= V; ++v)
                if (val[v] == 0) std::fill(st->deps + (size_t)v * W, st->deps + (size_t)(v + 1) * W, 0ull);
    }
    return ASP_OK;
}

int32_t asp_state_import(asp_program* p, void* stream, const asp_state* st) {
    if (!p || !p->bound || !st) return fail(ASP_E_STATE, "program not bound or null state");
    if (p->opt.learning != ASP_LEARN_FWD)
        return fail(ASP_E_INVALID, "state import needs assignment stamps and reasons that "
                                   "Res-learning programs keep on the device only");
    if (p->opt.max_models != 1 || p->opt.restart_every != 0 || p->opt.learn_conflicts > 1 ||
        p->opt.lookahead > 1)
        return fail(ASP_E_INVALID, "state import is for the plain search (one answer set, "
                                   "no restarts)");
    const int32_t V = p->hp.V, W = p->opt.W, A = p->hp.A, Rh = p->hp.Rh;
    const int32_t nS = (int32_t)p->hp.n_nogoods();
    if (st->n_vars != V || st->W != W) return fail(ASP_E_INVALID, "state shape mismatch");
    if (!st->val || !st->lvl || !st->deps || !st->dec) return fail(ASP_E_INVALID, "null state arrays");
    const int32_t cdl = st->cdl;
    if (cdl < 1 || cdl > Rh + 1) return fail(ASP_E_INVALID, "cdl out of range");
    if (st->n_learned < 0 || st->n_learned > p->opt.learned_cap_ng ||
        st->learned_lits < 0 || st->learned_lits > p->opt.learned_cap_lits)
        return fail(ASP_E_CAPACITY, "learned store beyond capacity");
    if (st->n_learned > 0 && (!st->learned_off || !st->learned))
        return fail(ASP_E_INVALID, "null learned arrays");
    std::vector<uint8_t> infront(V + 1, 0);
    for (int32_t i = 0; i < st->frontier_len; ++i) {
        int32_t v = st->frontier[i];
        if (v < 1 || v > V || st->val[v] == 0 || st->lvl[v] != cdl)
            return fail(ASP_E_INVALID, "frontier variable not assigned at level cdl");
        infront[v] = 1;
    }
    std::vector<int32_t> trail;
    for (int32_t v = 1; v <= V; ++v) {
        int8_t x = st->val[v];
        if (x < -1 || x > 1) return fail(ASP_E_INVALID, "value out of range");
        if (x == 0 && st->lvl[v] != 0) return fail(ASP_E_INVALID, "level of unassigned variable");
        if (x != 0 && (st->lvl[v] < 1 || st->lvl[v] > cdl)) return fail(ASP_E_INVALID, "level out of range");
        if (x != 0) trail.push_back(v);
    }
    std::stable_sort(trail.begin(), trail.end(), [&](int32_t a, int32_t b) {
        if (st->lvl[a] != st->lvl[b]) return st->lvl[a] < st->lvl[b];
        return infront[a] < infront[b];
    });
    std::vector<int32_t> tlim(Rh + 3, 0);
    {
        size_t k = 0;
        for (int32_t l = 1; l <= cdl + 1 && l < Rh + 3; ++l) {
            while (k < trail.size() && st->lvl[trail[k]] < l) ++k;
            tlim[l] = (int32_t)k;
        }
    }
    for (int32_t l = 2; l <= cdl; ++l) {
        int32_t d = st->dec[l];
        if (d <= A || d > V || (d - A - 1) % 3 != 0 || st->val[d] != 1 || st->lvl[d] != l)
            return fail(ASP_E_INVALID, "decision literal of a level is not an assigned b variable");
    }
    // learned nogoods and their occurrence lists (exact-size arrays)
    const int32_t nL = st->n_learned;
    std::vector<int32_t> loff(nL + 1, 0), llits(st->learned_lits);
    for (int32_t j = 0; j <= nL; ++j) loff[j] = nL ? st->learned_off[j] : 0;
    if (loff[0] != 0 || loff[nL] != st->learned_lits) return fail(ASP_E_INVALID, "learned offsets");
    for (int64_t q = 0; q < st->learned_lits; ++q) {
        int32_t l = st->learned[q];
        // learned nogoods hold decision literals T b_r only
        if (l <= A || l > V || (l - A - 1) % 3 != 0)
            return fail(ASP_E_INVALID, "learned literal is not a decision literal T b_r");
        llits[q] = l;
    }
    const size_t NL = 2 * ((size_t)V + 1);
    std::vector<int32_t> lptr(NL, 0), ln(NL, 0), lcap(NL, 0), pool;
    for (int32_t j = 0; j < nL; ++j)
        for (int32_t q = loff[j]; q < loff[j + 1]; ++q) {
            int32_t l = llits[q];
            ln[2 * (l < 0 ? -l : l) + (l < 0)] += 1;
        }
    {
        int32_t run = 0;
        for (size_t i = 0; i < NL; ++i) {
            lptr[i] = run;
            lcap[i] = ln[i];
            run += ln[i];
        }
        pool.assign(run, 0);
        std::vector<int32_t> fill(lptr);
        for (int32_t j = 0; j < nL; ++j)
            for (int32_t q = loff[j]; q < loff[j + 1]; ++q) {
                int32_t l = llits[q];
                pool[fill[2 * (l < 0 ? -l : l) + (l < 0)]++] = nS + j;
            }
        if ((int64_t)pool.size() > slot0(p).pool_cap) return fail(ASP_E_CAPACITY, "pool");
    }
    SlotCtrl k;
    memset(&k, 0, sizeof(k));
    k.inst = 0;
    k.cdl = cdl;
    k.qt = (int32_t)trail.size();
    k.qh = k.qt - st->frontier_len;
    k.n_learned = nL;
    k.pool_top = (int32_t)pool.size();
    k.pending = st->pending;
    k.pend_kind = st->pending >= 0 ? 1 : 0;
    if (st->pending >= nS + nL) return fail(ASP_E_INVALID, "pending conflict id");
    k.status = ASP_RUNNING;
    k.init_done = st->initialised ? 1 : 0;
    if (st->score_mode && p->opt.decision != ASP_DECISION_SCORE)
        return fail(ASP_E_INVALID, "score mode on a program loaded for occurrence decisions");
    k.use_score = st->score_mode ? 1 : 0;
    k.consec = st->consec;
    k.dec_open = st->dec_open ? 1 : 0;
    k.last_step = st->stats.last_step;
    k.learned_lits = st->learned_lits;
    k.rounds = st->stats.rounds;
    k.visits = st->stats.visits;
    k.checks = st->stats.literal_checks;
    k.props = st->stats.propagations;
    k.decisions = st->stats.decisions;
    k.conflicts = st->stats.conflicts;
    k.learned = st->stats.learned;
    k.learned_len = st->stats.learned_len;
    k.gate_fail = st->stats.gate_failures;
    k.completes = st->stats.completes;
    k.hash = st->stats.trace_hash;
    std::vector<int32_t> dec(Rh + 3, 0);
    for (int32_t l = 2; l <= cdl; ++l) dec[l] = st->dec[l];
    std::vector<uint64_t> win(V + 1, ~0ull);
    std::vector<int32_t> lvl(st->lvl, st->lvl + V + 1);
    hipStream_t s = (hipStream_t)stream;
    const SlotLayout L = slot0(p);
    auto put = [&](int64_t off, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(p->arena + p->plan.off_slots + off, src, bytes,
                              hipMemcpyHostToDevice, s);
    };
    HIPCHK(put(L.ctrl, &k, sizeof(k)));
    HIPCHK(put(L.val8, st->val, (size_t)V + 1));
    HIPCHK(put(L.lvl, lvl.data(), 4 * lvl.size()));
    HIPCHK(put(L.deps, st->deps, 8 * ((size_t)V + 1) * W));
    HIPCHK(put(L.win, win.data(), 8 * win.size()));
    HIPCHK(put(L.trail, trail.data(), 4 * trail.size()));
    HIPCHK(put(L.tlim, tlim.data(), 4 * tlim.size()));
    HIPCHK(put(L.dec, dec.data(), 4 * dec.size()));
    HIPCHK(put(L.locc_ptr, lptr.data(), 4 * lptr.size()));
    HIPCHK(put(L.locc_n, ln.data(), 4 * ln.size()));
    HIPCHK(put(L.locc_cap, lcap.data(), 4 * lcap.size()));
    HIPCHK(put(L.l_off, loff.data(), 4 * loff.size()));
    HIPCHK(put(L.l_lits, llits.data(), 4 * llits.size()));
    HIPCHK(put(L.pool, pool.data(), 4 * pool.size()));
    HIPCHK(hipStreamSynchronize(s));
    return ASP_OK;
}

// ---------------------------------------------------------------- batches
int32_t asp_batch_create(int32_t n, asp_program* const* progs, const asp_schedule* sched,
                         asp_batch** out, uint64_t* device_bytes, uint64_t* model_bytes) {
    if (!out || n < 1 || !progs) return fail(ASP_E_INVALID, "empty batch or null output");
    *out = nullptr;
    int32_t threads = sched ? sched->threads : 128;
    int32_t classes = sched ? sched->classes : 4;
    if (!valid_threads(threads) || classes < 1 || classes > 4)
        return fail(ASP_E_INVALID, "bad schedule");
    int32_t cth[4] = {0, 0, 0, 0};
    for (int c = 0; sched && c < 4; ++c) {
        cth[c] = sched->class_threads[c];
        if (cth[c] != 0 && !valid_threads(cth[c])) return fail(ASP_E_INVALID, "bad class threads");
    }
    std::unique_ptr<asp_batch> b(new asp_batch());
    b->opt = progs[0] ? progs[0]->opt : default_options();
    for (int32_t i = 0; i < n; ++i) {
        if (!progs[i]) return fail(ASP_E_INVALID, "null program in batch");
        const asp_options& o = progs[i]->opt;
        if (o.W != b->opt.W || o.gate != b->opt.gate || o.learned_cap_ng != b->opt.learned_cap_ng ||
            o.learned_cap_lits != b->opt.learned_cap_lits || o.decision != b->opt.decision ||
            o.fallback_after != b->opt.fallback_after || o.learning != b->opt.learning ||
            o.max_models != b->opt.max_models || o.restart_every != b->opt.restart_every ||
            std::max(o.learn_conflicts, 1) != std::max(b->opt.learn_conflicts, 1) ||
            (o.lookahead > 1 ? o.lookahead : 0) != (b->opt.lookahead > 1 ? b->opt.lookahead : 0))
            return fail(ASP_E_INVALID, "batch programs must share their options");
        b->progs.push_back(&progs[i]->hp);
    }
    int32_t rc = make_plan(b->progs, b->opt, threads, classes, b->plan, cth);
    if (rc) return rc;
    if (device_bytes) *device_bytes = b->plan.total;
    if (model_bytes) *model_bytes = (uint64_t)b->plan.tot_model;
    *out = b.release();
    return ASP_OK;
}

int32_t asp_batch_bind(asp_batch* b, void* dev_arena, uint64_t bytes, void* stream) {
    if (!b || !dev_arena) return fail(ASP_E_INVALID, "null batch or arena");
    if ((uintptr_t)dev_arena % kAlign) return fail(ASP_E_INVALID, "arena must be 256-byte aligned");
    if (bytes < b->plan.total) return fail(ASP_E_CAPACITY, "arena too small");
    b->arena = (uint8_t*)dev_arena;
    int32_t rc = upload_static(b->progs, b->plan, b->arena, (hipStream_t)stream);
    if (rc) return rc;
    b->bound = true;
    b->ready.assign(b->plan.n, 0);
    b->n_ready = 0;
    return ASP_OK;
}

int32_t asp_batch_set_scores(asp_batch* b, int32_t i, const int32_t* scores, void* stream) {
    if (!b || !b->bound) return fail(ASP_E_STATE, "batch not bound");
    if (i < 0 || i >= b->plan.n || !scores) return fail(ASP_E_INVALID, "bad instance or null scores");
    int32_t rc = put_scores(b->plan, b->arena, i, scores, (hipStream_t)stream);
    if (rc) return rc;
    if (!b->ready[i]) {
        b->ready[i] = 1;
        b->n_ready += 1;
    }
    return ASP_OK;
}

int32_t asp_batch_get_scores(asp_batch* b, int32_t i, int32_t* scores, void* stream) {
    if (!b || !b->bound) return fail(ASP_E_STATE, "batch not bound");
    if (i < 0 || i >= b->plan.n || !scores) return fail(ASP_E_INVALID, "bad instance or null scores");
    return get_scores(b->plan, b->arena, i, scores, (hipStream_t)stream);
}

int32_t asp_batch_scorer_workspace(const asp_batch* b, uint64_t* bytes) {
    if (!b || !bytes) return fail(ASP_E_INVALID, "null batch or output");
    ScorerPlan S;
    scorer_plan(b->progs, S);
    *bytes = S.total;
    return ASP_OK;
}

int32_t asp_score_batch(asp_batch* b, const asp_scorer_weights* w, void* ws, uint64_t ws_bytes,
                        void* stream) {
    if (!b || !b->bound) return fail(ASP_E_STATE, "batch not bound");
    int32_t rc = run_scorer(b->progs, b->plan, b->arena, b->scorer, w, (uint8_t*)ws, ws_bytes,
                            (hipStream_t)stream);
    if (rc) return rc;
    b->ready.assign(b->plan.n, 1);
    b->n_ready = b->plan.n;
    return ASP_OK;
}

int32_t asp_batch_train_readout(asp_batch* b, const asp_scorer_weights* w, void* ws,
                                uint64_t ws_bytes, const int8_t* labels, int32_t steps, float lr,
                                float* wb_out, float* loss_out, void* stream) {
    if (!b || !b->bound) return fail(ASP_E_STATE, "batch not bound");
    if (!labels || !wb_out) return fail(ASP_E_INVALID, "null labels or output");
    if (steps < 1 || steps > kMaxTrainSteps) return fail(ASP_E_INVALID, "steps must be in 1..4096");
    if (!(lr > 0.f)) return fail(ASP_E_INVALID, "learning rate must be positive");
    hipStream_t s = (hipStream_t)stream;
    // forward pass: the last layer's codes stay in the workspace
    int32_t rc = run_scorer(b->progs, b->plan, b->arena, b->scorer, w, (uint8_t*)ws, ws_bytes, s);
    if (rc) return rc;
    const ScorerPlan& S = b->scorer;
    uint8_t* W8 = (uint8_t*)ws;
    const uint64_t atoms = (uint64_t)b->plan.tot_model;
    int64_t n_lab = 0;
    for (uint64_t i = 0; i < atoms; ++i) n_lab += labels[i] >= 0 ? 1 : 0;
    if (n_lab == 0) return fail(ASP_E_INVALID, "no labelled atom");
    std::vector<float> init(3 * 65 + 66, 0.f);
    for (int j = 0; j < 64; ++j) init[j] = wb_out[j];   // caller's starting point
    init[64] = wb_out[64];
    float* T = (float*)(W8 + S.off_train);
    if (atoms) HIPCHK(hipMemcpyAsync(W8 + S.off_lab, labels, atoms, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(T, init.data(), 4 * init.size(), hipMemcpyHostToDevice, s));
    TrainArgs t{};
    t.labels = (const int8_t*)(W8 + S.off_lab);
    t.wb = T;
    t.m = T + 65;
    t.v = T + 130;
    t.grad = T + 195;
    t.loss = T + 261;
    t.inv_n = 1.f / (float)n_lab;
    t.lr = lr;
    DeviceInfo di = device_info();
    ScorerArgs a = scorer_args(b->progs, b->plan, b->arena, S, W8);
    const int grid = (int)std::max<size_t>(1, std::min<size_t>(S.vt.size(), (size_t)di.cus * 4));
    HIPCHK(launch_readout_train(a, t, steps, grid, s));
    HIPCHK(hipMemcpyAsync(wb_out, T, 4 * 65, hipMemcpyDeviceToHost, s));
    if (loss_out) HIPCHK(hipMemcpyAsync(loss_out, t.loss, 4 * (size_t)steps, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ASP_OK;
}

// The launch classes of a batch run on streams of its own, all four of them
// created together the first time, every class on one of them, so that the
// classes can run at once.  Which hardware queue a stream takes is the
// runtime's choice (four queues per process by default): two classes that
// land on one queue run one after the other, with the same results.  The
// graph replay (asp_solve_batch_graph) overlaps them.
static hipError_t class_streams(asp_batch* b) {
    while (b->streams.size() < 4) {
        hipStream_t t;
        hipError_t e = hipStreamCreateWithFlags(&t, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        b->streams.push_back(t);
    }
    return hipSuccess;
}

int32_t asp_solve_batch(asp_batch* b, void* stream, const asp_limits* lim) {
    if (!b || !b->bound) return fail(ASP_E_STATE, "batch not bound");
    if (b->opt.decision == ASP_DECISION_SCORE && b->n_ready < b->plan.n)
        return fail(ASP_E_STATE, "decision scores not set for every instance");
    hipStream_t s = (hipStream_t)stream;
    DeviceInfo di = device_info();
    int32_t rc = check_launch(b->plan, di);
    if (rc) return rc;
    const size_t nc = b->plan.classes.size();
    if (!b->ev0) {
        HIPCHK(hipEventCreate(&b->ev0));
        HIPCHK(hipEventCreate(&b->ev1));
        HIPCHK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    }
    while (b->ev_join.size() < nc) {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        b->ev_start.push_back(e0);
        b->ev_join.push_back(e1);
    }
    if (nc > 1) HIPCHK(class_streams(b));
    HIPCHK(hipEventRecord(b->ev0, s));
    if (nc == 1) {
        const LaunchClass& lc = b->plan.classes[0];
        KArgs a = make_args(b->plan, b->arena, MODE_SOLVE, lc);
        apply_limits(a, b->plan, lim, di);
        HIPCHK(hipEventRecord(b->ev_start[0], s));
        HIPCHK(launch_search(a, lc.threads, lc.count, lc.lds, s));
        HIPCHK(hipEventRecord(b->ev_join[0], s));
    } else {
        // fork: every class launches on its own stream once the caller's
        // stream has reached this point; join back before ev1
        HIPCHK(hipEventRecord(b->ev_fork, s));
        for (size_t c = 0; c < nc; ++c) {
            const LaunchClass& lc = b->plan.classes[c];
            KArgs a = make_args(b->plan, b->arena, MODE_SOLVE, lc);
            apply_limits(a, b->plan, lim, di);
            hipStream_t cs = b->streams[c];
            HIPCHK(hipStreamWaitEvent(cs, b->ev_fork, 0));
            HIPCHK(hipEventRecord(b->ev_start[c], cs));
            HIPCHK(launch_search(a, lc.threads, lc.count, lc.lds, cs));
            HIPCHK(hipEventRecord(b->ev_join[c], cs));
        }
        for (size_t c = 0; c < nc; ++c) HIPCHK(hipStreamWaitEvent(s, b->ev_join[c], 0));
    }
    HIPCHK(hipEventRecord(b->ev1, s));
    b->timed = true;
    b->class_timed = true;
    return ASP_OK;
}

int32_t asp_solve_batch_graph(asp_batch* b, void* stream, const asp_limits* lim) {
    if (!b || !b->bound) return fail(ASP_E_STATE, "batch not bound");
    if (!stream) return fail(ASP_E_INVALID, "graph launches need a non-default stream");
    if (b->opt.decision == ASP_DECISION_SCORE && b->n_ready < b->plan.n)
        return fail(ASP_E_STATE, "decision scores not set for every instance");
    hipStream_t s = (hipStream_t)stream;
    DeviceInfo di = device_info();
    int32_t rc = check_launch(b->plan, di);
    if (rc) return rc;
    const asp_limits L = lim ? *lim : asp_limits{-1, 0};
    const size_t nc = b->plan.classes.size();
    if (!b->ev0) {
        HIPCHK(hipEventCreate(&b->ev0));
        HIPCHK(hipEventCreate(&b->ev1));
        HIPCHK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    }
    while (b->ev_cjoin.size() < nc) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->ev_cjoin.push_back(e);
    }
    if (nc > 1) HIPCHK(class_streams(b));
    if (!b->gexec || b->gstream != s || b->glim.max_conflicts != L.max_conflicts ||
        b->glim.max_ms != L.max_ms) {
        if (b->gexec) {
            HIPCHK(hipGraphExecDestroy(b->gexec));
            b->gexec = nullptr;
        }
        // capture the same fork/join as the eager launch, without timing
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipEventRecord(b->ev_fork, s);
        for (size_t c = 0; c < nc && e == hipSuccess; ++c) {
            const LaunchClass& lc = b->plan.classes[c];
            KArgs a = make_args(b->plan, b->arena, MODE_SOLVE, lc);
            apply_limits(a, b->plan, &L, di);
            hipStream_t cs = nc > 1 ? b->streams[c] : s;
            if (nc > 1) e = hipStreamWaitEvent(cs, b->ev_fork, 0);
            if (e == hipSuccess) e = launch_search(a, lc.threads, lc.count, lc.lds, cs);
            if (e == hipSuccess && nc > 1) e = hipEventRecord(b->ev_cjoin[c], cs);
        }
        for (size_t c = 0; c < nc && nc > 1 && e == hipSuccess; ++c) e = hipStreamWaitEvent(s, b->ev_cjoin[c], 0);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (e != hipSuccess) return fail(ASP_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        if (e2 != hipSuccess) return fail(ASP_E_DEVICE, std::string("end capture: ") + hipGetErrorString(e2));
        e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(ASP_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        b->gstream = s;
        b->glim = L;
    }
    HIPCHK(hipEventRecord(b->ev0, s));
    HIPCHK(hipGraphLaunch(b->gexec, s));
    HIPCHK(hipEventRecord(b->ev1, s));
    b->timed = true;
    b->class_timed = false;
    return ASP_OK;
}

int32_t asp_batch_results(asp_batch* b, void* stream, int32_t* verdicts, uint8_t* models,
                          asp_stats* stats) {
    if (!b || !b->bound) return fail(ASP_E_STATE, "batch not bound");
    hipStream_t s = (hipStream_t)stream;
    const Plan& P = b->plan;
    if (verdicts)
        HIPCHK(hipMemcpyAsync(verdicts, b->arena + P.off_verd, 4 * (size_t)P.n,
                              hipMemcpyDeviceToHost, s));
    if (models && P.tot_model > 0)
        HIPCHK(hipMemcpyAsync(models, b->arena + P.off_models, (size_t)P.tot_model,
                              hipMemcpyDeviceToHost, s));
    std::vector<DevStats> ds;
    if (stats) {
        ds.resize(P.n);
        HIPCHK(hipMemcpyAsync(ds.data(), b->arena + P.off_stats, sizeof(DevStats) * ds.size(),
                              hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (stats)
        for (int32_t i = 0; i < P.n; ++i) to_stats(ds[i], &stats[i]);
    return ASP_OK;
}

int32_t asp_batch_learned(asp_batch* b, int32_t i, int32_t* off, int64_t cap_ng, int32_t* lits,
                          int64_t cap_lits, int32_t* n_learned, int64_t* n_lits, void* stream) {
    if (!b || !b->bound) return fail(ASP_E_STATE, "batch not bound");
    if (i < 0 || i >= b->plan.n) return fail(ASP_E_INVALID, "instance index out of range");
    hipStream_t s = (hipStream_t)stream;
    const HostProgram& h = *b->progs[i];
    const SlotLayout L = slot_layout(h.V, h.Rh, b->plan.W, b->plan.cap_ng, b->plan.cap_lits,
                                     b->plan.learning);
    uint8_t* slot = b->arena + b->plan.off_slots + b->plan.slot_off[i];
    SlotCtrl k;
    HIPCHK(hipMemcpyAsync(&k, slot + L.ctrl, sizeof(k), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (n_learned) *n_learned = k.n_learned;
    if (n_lits) *n_lits = k.learned_lits;
    if (off && k.n_learned + 1 <= cap_ng)
        HIPCHK(hipMemcpyAsync(off, slot + L.l_off, 4 * ((size_t)k.n_learned + 1),
                              hipMemcpyDeviceToHost, s));
    if (lits && k.learned_lits > 0 && k.learned_lits <= cap_lits)
        HIPCHK(hipMemcpyAsync(lits, slot + L.l_lits, 4 * (size_t)k.learned_lits,
                              hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ASP_OK;
}

int32_t asp_scorer_train_workspace(int32_t n, asp_program* const* progs, uint64_t* bytes) {
    if (n < 1 || !progs || !bytes) return fail(ASP_E_INVALID, "empty program list or null output");
    std::vector<const HostProgram*> hp;
    for (int32_t i = 0; i < n; ++i) {
        if (!progs[i]) return fail(ASP_E_INVALID, "null program");
        hp.push_back(&progs[i]->hp);
    }
    return train_workspace(hp, bytes);
}

int32_t asp_scorer_train(int32_t n, asp_program* const* progs, const float* labels, float* params,
                         int32_t steps, float lr, void* ws, uint64_t ws_bytes, float* loss_out,
                         float* grad_out, void* stream) {
    if (n < 1 || !progs || !labels || !params || !ws)
        return fail(ASP_E_INVALID, "null argument or empty program list");
    if ((uintptr_t)ws % kAlign) return fail(ASP_E_INVALID, "workspace must be 256-byte aligned");
    if (steps < 0 || steps > 100000 || !(lr >= 0.f) || lr > 1.f)
        return fail(ASP_E_INVALID, "steps must be in 0..100000 and lr in [0, 1]");
    if (steps == 0 && !loss_out) return fail(ASP_E_INVALID, "a gradient pass needs loss_out");
    if (train_nparam() != ASP_SCORER_NPARAM) return fail(ASP_E_INTERNAL, "parameter layout");
    std::vector<const HostProgram*> hp;
    for (int32_t i = 0; i < n; ++i) {
        if (!progs[i]) return fail(ASP_E_INVALID, "null program");
        hp.push_back(&progs[i]->hp);
    }
    for (int64_t i = 0; i < ASP_SCORER_NPARAM; ++i)
        if (!std::isfinite(params[i])) return fail(ASP_E_INVALID, "non-finite parameter");
    std::string err;
    int32_t rc = train_run(hp, labels, params, steps, lr, (uint8_t*)ws, ws_bytes, loss_out,
                           grad_out, (hipStream_t)stream, &err);
    if (rc) return fail(rc, err);
    return ASP_OK;
}

int32_t asp_scorer_quantize(const float* params, asp_scorer_weights* w) {
    if (!params || !w) return fail(ASP_E_INVALID, "null argument");
    for (int64_t i = 0; i < ASP_SCORER_NPARAM; ++i)
        if (!std::isfinite(params[i])) return fail(ASP_E_INVALID, "non-finite parameter");
    train_quantize(params, w);
    return ASP_OK;
}

int32_t asp_scorer_dequantize(const asp_scorer_weights* w, float* params) {
    if (!params || !w) return fail(ASP_E_INVALID, "null argument");
    train_dequantize(w, params);
    return ASP_OK;
}

int32_t asp_batch_last_ms(asp_batch* b, double* ms) {
    if (!b || !b->timed || !ms) return fail(ASP_E_STATE, "no timed launch");
    HIPCHK(hipEventSynchronize(b->ev1));
    float f = 0.f;
    HIPCHK(hipEventElapsedTime(&f, b->ev0, b->ev1));
    *ms = (double)f;
    return ASP_OK;
}

int32_t asp_batch_launch_info(asp_batch* b, int32_t* n_classes, int32_t* first, int32_t* count,
                              int32_t* threads, double* ms, int32_t* order) {
    if (!b) return fail(ASP_E_INVALID, "null batch");
    const Plan& P = b->plan;
    const int nc = (int)P.classes.size();
    if (n_classes) *n_classes = nc;
    for (int c = 0; c < nc; ++c) {
        if (first) first[c] = P.classes[c].first;
        if (count) count[c] = P.classes[c].count;
        if (threads) threads[c] = P.classes[c].threads;
        if (ms) {
            ms[c] = 0.0;
            if (b->class_timed && c < (int)b->ev_join.size()) {
                HIPCHK(hipEventSynchronize(b->ev_join[c]));
                float f = 0.f;
                HIPCHK(hipEventElapsedTime(&f, b->ev_start[c], b->ev_join[c]));
                ms[c] = (double)f;
            }
        }
    }
    if (order) memcpy(order, P.order.data(), 4 * P.order.size());
    return ASP_OK;
}

int32_t asp_batch_free(asp_batch* b) {
    if (b) {
        if (b->ev0) (void)hipEventDestroy(b->ev0);
        if (b->ev1) (void)hipEventDestroy(b->ev1);
        if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
        for (hipEvent_t e : b->ev_join) (void)hipEventDestroy(e);
        for (hipEvent_t e : b->ev_start) (void)hipEventDestroy(e);
        for (hipEvent_t e : b->ev_cjoin) (void)hipEventDestroy(e);
        if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
        for (hipStream_t t : b->streams) (void)hipStreamDestroy(t);
        delete b;
    }
    return ASP_OK;
}

}  // extern "C"
