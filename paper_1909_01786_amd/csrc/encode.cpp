// encode.cpp -- completion nogoods of a ground normal program (Sect. 2).
//
// For a headed rule r with auxiliary atoms b_r, t_r, n_r, the completion
// b_r <-> t_r & n_r, t_r <-> body+(r), n_r <-> not body-(r), and for an atom
// p, p <-> OR_{r in rules(p)} b_r, give the nogoods
//   {F b_r, T t_r, T n_r}, {T b_r, F t_r}, {T b_r, F n_r},
//   {T t_r, F p} (p in body+), {T n_r, T q} (q in body-),
//   {F t_r} u {T p : body+}, {F n_r} u {F q : body-},
//   {F p, T b_r} (r in rules(p)), {T p} u {F b_r : r in rules(p)},
// and a constraint gives {T p : body+} u {F q : body-}.  They are produced
// rule by rule, then atom by atom, then constraint by constraint, and kept
// sorted by length (Sect. 4: nogoods are stored by increasing length), the
// position in that order being the nogood's id.
#include "encode.h"

#include <algorithm>
#include <numeric>

namespace asp {

namespace {

inline int32_t lit_index(int32_t l) { return 2 * (l < 0 ? -l : l) + (l < 0 ? 1 : 0); }

// Builder of nogoods in generation order.
struct Emitter {
    std::vector<int64_t> start;   // start of each nogood in `lits`
    std::vector<int32_t> lits;
    void open() { start.push_back((int64_t)lits.size()); }
    void put(int32_t l) { lits.push_back(l); }
};

}  // namespace

int encode_program(int32_t n_atoms, int32_t n_rules, const int32_t* head,
                   const int64_t* body_off, const int32_t* body_lits, HostProgram* P,
                   std::string* err) {
    if (n_atoms < 0 || n_rules < 0) {
        *err = "negative atom or rule count";
        return -1;
    }
    if (n_rules > 0 && (!head || !body_off)) {
        *err = "null rule arrays";
        return -1;
    }
    if (n_rules > 0 && body_off[0] != 0) {
        *err = "body_off[0] must be 0";
        return -1;
    }
    for (int32_t r = 0; r < n_rules; ++r) {
        if (body_off[r + 1] < body_off[r]) {
            *err = "body offsets decrease at rule " + std::to_string(r);
            return -1;
        }
        if (head[r] < 0 || head[r] > n_atoms) {
            *err = "head atom out of range at rule " + std::to_string(r);
            return -1;
        }
    }
    const int64_t total = n_rules > 0 ? body_off[n_rules] : 0;
    if (total > 0 && !body_lits) {
        *err = "null body literals";
        return -1;
    }
    for (int64_t k = 0; k < total; ++k) {
        int32_t l = body_lits[k];
        if (l == 0 || l == INT32_MIN || (l < 0 ? -l : l) > n_atoms) {
            *err = "body literal out of range at position " + std::to_string(k);
            return -1;
        }
    }

    // Rules with repeated body literals removed (first occurrence kept);
    // a constraint with both a and not a can never be violated: dropped.
    struct Body { std::vector<int32_t> pos, neg; };
    std::vector<Body> hb;       // headed rules
    std::vector<int32_t> hh;
    std::vector<Body> cb;       // constraints
    for (int32_t r = 0; r < n_rules; ++r) {
        Body b;
        std::vector<int32_t> seen;
        for (int64_t k = body_off[r]; k < body_off[r + 1]; ++k) {
            int32_t l = body_lits[k];
            if (std::find(seen.begin(), seen.end(), l) != seen.end()) continue;
            seen.push_back(l);
            (l > 0 ? b.pos : b.neg).push_back(l > 0 ? l : -l);
        }
        if (head[r] != 0) {
            hb.push_back(std::move(b));
            hh.push_back(head[r]);
        } else {
            bool taut = false;
            for (int32_t p : b.pos)
                if (std::find(b.neg.begin(), b.neg.end(), p) != b.neg.end()) taut = true;
            if (!taut) cb.push_back(std::move(b));
        }
    }
    const int64_t A = n_atoms, Rh = (int64_t)hb.size();
    if (A + 3 * Rh > (int64_t)0x3fffffff) {
        *err = "too many variables";
        return -1;
    }
    P->A = n_atoms;
    P->Rh = (int32_t)Rh;
    P->Rc = (int32_t)cb.size();
    P->V = (int32_t)(A + 3 * Rh);
    auto bvar = [&](int64_t j) { return (int32_t)(A + 3 * j + 1); };

    Emitter e;
    for (int64_t j = 0; j < Rh; ++j) {
        const int32_t b = bvar(j), t = b + 1, n = b + 2;
        const Body& bd = hb[j];
        e.open(); e.put(-b); e.put(t); e.put(n);
        e.open(); e.put(b); e.put(-t);
        e.open(); e.put(b); e.put(-n);
        for (int32_t p : bd.pos) { e.open(); e.put(t); e.put(-p); }
        for (int32_t q : bd.neg) { e.open(); e.put(n); e.put(q); }
        e.open(); e.put(-t);
        for (int32_t p : bd.pos) e.put(p);
        e.open(); e.put(-n);
        for (int32_t q : bd.neg) e.put(-q);
    }
    std::vector<std::vector<int32_t>> rules_of(A + 1);
    for (int64_t j = 0; j < Rh; ++j) rules_of[hh[j]].push_back((int32_t)j);
    for (int64_t p = 1; p <= A; ++p) {
        for (int32_t j : rules_of[p]) { e.open(); e.put((int32_t)-p); e.put(bvar(j)); }
        e.open(); e.put((int32_t)p);
        for (int32_t j : rules_of[p]) e.put(-bvar(j));
    }
    for (const Body& bd : cb) {
        e.open();
        for (int32_t p : bd.pos) e.put(p);
        for (int32_t q : bd.neg) e.put(-q);
    }
    const int64_t G = (int64_t)e.start.size();
    e.start.push_back((int64_t)e.lits.size());
    if ((int64_t)e.lits.size() > (int64_t)0x7fffffff || G > (int64_t)0x3fffffff) {
        *err = "program too large for 32-bit nogood offsets";
        return -1;
    }

    // ids: stable order by length
    std::vector<int32_t> ord(G);
    std::iota(ord.begin(), ord.end(), 0);
    auto len = [&](int32_t g) { return e.start[g + 1] - e.start[g]; };
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return len(x) < len(y); });

    P->ng_off.assign(G + 1, 0);
    P->ng_lits.resize(e.lits.size());
    int64_t pos = 0;
    P->has_empty = 0;
    P->u0 = P->u1 = 0;
    for (int64_t i = 0; i < G; ++i) {
        int32_t g = ord[i];
        int64_t L = len(g);
        if (L == 0) { P->has_empty = 1; P->u0 = P->u1 = (int32_t)(i + 1); }
        if (L == 1) P->u1 = (int32_t)(i + 1);
        std::copy(e.lits.begin() + e.start[g], e.lits.begin() + e.start[g + 1],
                  P->ng_lits.begin() + pos);
        pos += L;
        P->ng_off[i + 1] = (int32_t)pos;
    }
    if (P->u1 < P->u0) P->u1 = P->u0;

    // literal -> nogood ids, ascending (filled in id order)
    const int64_t NL = 2 * ((int64_t)P->V + 1);
    P->map_off.assign(NL + 1, 0);
    for (int32_t l : P->ng_lits) P->map_off[lit_index(l) + 1] += 1;
    for (int64_t i = 0; i < NL; ++i) P->map_off[i + 1] += P->map_off[i];
    P->map_ent.resize(P->ng_lits.size());
    {
        std::vector<int32_t> fill(P->map_off.begin(), P->map_off.end() - 1);
        for (int64_t id = 0; id < G; ++id) {
            const int32_t b = P->ng_off[id], e = P->ng_off[id + 1];
            for (int32_t k = b; k < e; ++k) {
                MapEntry m{(int32_t)id, P->ng_lits[k], 0, 0, 0, 0, 0, 0};
                if (e - b > 3) {
                    m.o1 = kLongNogood;   // the nogood's literals: ng_lits[o2 .. o2 + a1)
                    m.o2 = b;
                    m.a1 = e - b;
                } else {
                    int32_t* o = &m.o1;
                    int32_t* seg = &m.a1;
                    for (int32_t q = b; q < e; ++q) {
                        if (q == k) continue;
                        const int32_t l = P->ng_lits[q];
                        const int64_t ci = lit_index(-l);   // the complement's segment
                        *o++ = l;
                        seg[0] = P->map_off[ci];
                        seg[1] = P->map_off[ci + 1] - P->map_off[ci];
                        seg += 2;
                    }
                }
                P->map_ent[fill[lit_index(P->ng_lits[k])]++] = m;
            }
        }
    }

    // occurrence count and Jeroslow-Wang score (sum of 2^(16-|delta|), none
    // beyond 16 literals) of each atom over Delta_0 (an atom occurs at most
    // once per nogood), read per headed rule through its head
    std::vector<int32_t> occ(A + 1, 0), jw(A + 1, 0);
    for (size_t g = 0; g + 1 < P->ng_off.size(); ++g) {
        const int32_t len = P->ng_off[g + 1] - P->ng_off[g];
        for (int32_t q = P->ng_off[g]; q < P->ng_off[g + 1]; ++q) {
            int32_t v = P->ng_lits[q] < 0 ? -P->ng_lits[q] : P->ng_lits[q];
            if (v > A) continue;
            occ[v] += 1;
            if (len <= 16) jw[v] += 1 << (16 - len);
        }
    }
    P->rule_head.assign(hh.begin(), hh.end());
    P->rule_occ.resize(Rh);
    P->rule_jw.resize(Rh);
    P->rb_off.assign(Rh + 1, 0);
    P->rb_lits.clear();
    for (int64_t j = 0; j < Rh; ++j) {
        P->rule_occ[j] = occ[hh[j]];
        P->rule_jw[j] = jw[hh[j]];
        for (int32_t p : hb[j].pos) P->rb_lits.push_back(p);
        for (int32_t q : hb[j].neg) P->rb_lits.push_back(-q);
        P->rb_off[j + 1] = (int32_t)P->rb_lits.size();
    }
    auto by_score = [&](const std::vector<int32_t>& sc, std::vector<int32_t>& out) {
        std::vector<int32_t> ord(Rh);
        for (int64_t j = 0; j < Rh; ++j) ord[j] = (int32_t)j;
        std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
            return sc[a] != sc[b] ? sc[a] > sc[b] : a < b;
        });
        out.resize(2 * Rh);
        for (int64_t p = 0; p < Rh; ++p) {
            out[2 * p] = ord[p];
            out[2 * p + 1] = hh[ord[p]];
        }
    };
    by_score(P->rule_occ, P->rule_by_occ);
    by_score(P->rule_jw, P->rule_by_jw);
    return 0;
}

}  // namespace asp
