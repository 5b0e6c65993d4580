/*
 * oracle.c -- plain sequential CPU oracle of the conflict-driven ASP solver
 * (Dovier, Formisano, Vella: "GPU-based parallelism for ASP-solving").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link
 * or call this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the HIP library.
 *
 * It is written to be read against the paper, not to be fast: every step is
 * the plain definition, with no blocking, fusion or reordering.  Where the
 * paper leaves a choice open, the reading taken is stated at that step.
 *
 * Steps (one call of or_step runs exactly one):
 *   INIT     -- InitialPropagation of the unit nogoods (Alg. 1, first kernel).
 *   ROUND    -- one PropagateAndCheck round (Sect. 4.1, Alg. 2) in the
 *               deterministic Jacobi reading: all nogoods reached from the
 *               previous round's assignments are classified against one
 *               snapshot, the lowest-id implier wins a variable, clashing
 *               implications become conflicts.
 *   LEARN    -- Fwd-learning (Sect. 4.2, Alg. 4) from the Deps bitmaps, or
 *               (option) Res-learning (Alg. 3): resolution from the conflict
 *               back to the first UIP; then Backjump (Alg. 1) and assertion
 *               of the complement of the learned nogood's latest literal.
 *   DECIDE   -- the ASP-computation Decision (Sect. 2): among rules r whose
 *               head is unassigned with T t_r in A and F n_r not in A, pick the
 *               highest score of the head (ties: lowest rule) and assign T b_r
 *               at a new level.  The score is the occurrence count of the
 *               head in the static nogoods (the paper's occurrence heuristic)
 *               or, when a per-atom integer score is supplied (the learned
 *               Decision), that score until the fallback below fires.
 *   COMPLETE -- CompleteAssignment (Sect. 2): no applicable rule is left, so
 *               every unassigned original atom becomes false.
 *   GATE     -- on a total assignment, check M = least model of the reduct
 *               (the answer-set definition of the Preliminaries); a failure
 *               becomes a conflict over the unfounded set's loop nogood.
 *
 * Several answer sets and restarts (the paper restarts the solver when more
 * than one answer set is asked for, or by a restart strategy, and its
 * InitialPropagation then also takes the learned unit nogoods):
 *   - an answer set M found while more are asked for is recorded and blocked
 *     by the learned nogood {T p : p in M}: answer sets are pairwise
 *     incomparable under set inclusion, so this excludes M and no other
 *     answer set (an empty M leaves none); then the search restarts;
 *   - a restart unassigns every variable, keeps every learned nogood, and
 *     runs InitialPropagation again over the static and the learned unit
 *     nogoods (an empty learned nogood means no answer set is left);
 *   - with restart_every > 0, a conflict that makes restart_every conflicts
 *     since the last restart learns its nogood and restarts in place of the
 *     backjump;
 *   - when the search ends UNSAT (or UNKNOWN) after at least one answer set,
 *     the verdict is SAT; after UNSAT the enumeration is exhausted.
 *
 * Several conflicts per Learning step (the paper lets the solver select one
 * or more of a round's conflicts, and take the lowest backjump level among
 * the learned nogoods): with learn_conflicts = K > 1 the K shortest (then
 * lowest-id) distinct conflicts of a round are each learned on the same
 * assignment, in that order, with consecutive ids; the backjump goes to
 * the lowest of their levels and the first nogood reaching it asserts its
 * latest literal.  One of them holding at the root means no answer set.
 *
 * Readings of the paper taken here:
 *   - levels start at 1 (root); the decision at level l >= 2 sets Deps bit
 *     min(l-1, 64W-1), so bit 64W-1 stands for every level >= 64W;
 *   - the learned nogood holds the decision literals of every level whose
 *     bit is set in B = OR of the Deps of the conflict's variables; the
 *     backjump level is the second-highest such level (1 if only one);
 *   - T_Pi's second condition is read as body-(r) disjoint from I, the reduct
 *     as Gelfond-Lifschitz, and the decided literal as T b_r (T n_r, not
 *     F n_r, then follows by propagation);
 *   - CompleteAssignment's falsifications take level cdl and the Deps of all
 *     decisions;
 *   - Res-learning orders assignments by an event clock (one tick per round,
 *     decision, assertion, completion; the implications of a round share a
 *     tick) and breaks ties by variable id; a literal's reason is the nogood
 *     that implied it.  A round conflict whose resolution reaches a literal
 *     with no reason at the conflict level (a CompleteAssignment literal), and
 *     every stability-gate conflict, is learned by Fwd-learning instead; a
 *     round conflict with no literal above level 1 means UNSAT;
 *   - the Decision's score may also be the Jeroslow-Wang score of the head
 *     over the static nogoods, J(p) = sum over nogoods holding a literal of
 *     p of 2^-|delta|, in fixed point: sum of 2^(16-|delta|), nothing for
 *     |delta| > 16; or the activity of the head: it starts at the occurrence
 *     count, every literal of a nogood learned from a conflict adds 8 to its
 *     atom (an auxiliary variable of rule r counts for the head of r), and
 *     after every 64th such nogood all activities are halved;
 *   - supplied scores fall back to the occurrence heuristic, for the rest of
 *     the search, once `fallback_after` conflicts come in a row: the count
 *     grows at every conflict and restarts from zero whenever a decision's
 *     propagation ends at a conflict-free fixpoint.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_RUNNING = 0, OR_SAT = 1, OR_UNSAT = 2, OR_UNKNOWN = 3 };
enum { OR_E_INVALID = -1, OR_E_INTERNAL = -5 };
enum { ST_NONE = 0, ST_INIT = 1, ST_ROUND = 2, ST_LEARN = 3, ST_DECIDE = 4,
       ST_COMPLETE = 5, ST_GATE = 6, ST_DONE = 7 };
enum { GATE_UNFOUNDED = 0, GATE_ALLDEC = 1 };
enum { LEARN_FWD = 0, LEARN_RES = 1 };
enum { DEC_OCC = 0, DEC_SCORE = 1, DEC_JW = 2, DEC_ACTIVITY = 3 };

typedef struct {
    int64_t rounds, visits, literal_checks, propagations, decisions, conflicts,
            learned, learned_len, gate_failures, completes, models, restarts;
    uint64_t trace_hash;
    int64_t deps_reads;   /* measurement only: Deps words read to give the
                             implied variables theirs, sum over propagations
                             of (|winner| - 1) * W */
} or_stats;

typedef struct {
    int64_t max_conflicts;     /* <0: unlimited */
    int64_t learned_cap_ng;    /* <0: unlimited */
    int64_t learned_cap_lits;  /* <0: unlimited */
} or_limits;

typedef struct { int32_t *a; int64_t n, cap; } ivec;

static void iv_push(ivec *v, int32_t x) {
    if (v->n == v->cap) {
        v->cap = v->cap ? 2 * v->cap : 8;
        v->a = (int32_t *)realloc(v->a, (size_t)v->cap * sizeof(int32_t));
    }
    v->a[v->n++] = x;
}

typedef struct {
    /* program after normalisation */
    int32_t A, Rh, Rc, V, W, gate_mode;
    int32_t *rhead;            /* [Rh] head atom of headed rule j */
    int32_t *pos_off, *pos;    /* body+ of headed rule j */
    int32_t *neg_off, *neg;    /* body- of headed rule j */
    int32_t has_empty_nogood;

    /* nogoods: static ones first (ids 0..n0-1), learned ones appended */
    int64_t n0, lits0;
    ivec ng_off;               /* offsets, ng_off.a[i]..ng_off.a[i+1] */
    ivec ng_lits;
    ivec *map;                 /* [2(V+1)] literal -> nogood ids ascending */
    int32_t *occ;              /* [A+1] static occurrence count */
    int32_t *jw;               /* [A+1] static Jeroslow-Wang score (fixed point) */
    int32_t *act;              /* [A+1] activity */
    int32_t decision;          /* DEC_OCC, DEC_JW or DEC_ACTIVITY when no scores drive it */
    int32_t *score;            /* [A+1] supplied decision scores, or NULL */
    int32_t use_score;         /* 1 while the supplied scores drive Decision */
    int32_t fallback_after;    /* <0: never fall back */
    int32_t consec;            /* conflicts since a decision reached a fixpoint */
    int32_t dec_since_conf;    /* a decision was taken since the last conflict */
    int32_t learning;          /* LEARN_FWD or LEARN_RES */
    int32_t clock;             /* assignment event clock (Res-learning order) */
    int32_t *stamp;            /* [V+1] clock tick of each assignment */
    int32_t *reason;           /* [V+1] nogood that implied it, -1 if none */
    int32_t *mark;             /* [V+1] resolution membership (epoch) */
    int32_t epoch;
    int64_t max_models;        /* answer sets asked for; 0: all */
    int64_t restart_every;     /* conflicts between restarts; 0: never */
    int64_t since_restart;     /* conflicts since the last restart */
    int32_t need_init;         /* InitialPropagation comes next */
    int32_t exhausted;         /* no answer set is left */
    uint8_t *models;           /* [models found * A] answer sets found */
    int64_t models_cap;

    /* assignment */
    int8_t *val;
    int32_t *lvl;
    uint64_t *deps;            /* [(V+1)*W] */
    int32_t cdl;
    int32_t *dec;              /* [Rh+2] decision literal of each level */
    ivec frontier;

    /* pending conflict: kind 0 none, 1 round (ids), 2 gate (bits) */
    int32_t pend_kind;
    int32_t pend_id;           /* the first (shortest, then lowest id) round conflict */
    int32_t pend_ids[8];       /* the round conflicts selected for learning, ranked */
    int32_t n_pend;
    int32_t learn_conflicts;   /* round conflicts learned per Learning step, 1..8 */
    int32_t lookahead;         /* Decision candidates tried by propagation, 0..8 (<= 1: off) */
    uint64_t *pend_B;

    int32_t status, last_step;
    int64_t n_learned, learned_lits;
    or_stats st;

    /* scratch */
    int32_t *win;              /* [V+1] min implier id, -1 none */
    int8_t *winsign;           /* [V+1] value the winner implies */
    int64_t nass;              /* number of assigned variables */
    int32_t *touched;          /* [V+1] */
    uint64_t *tmpdeps;         /* [(V+1)*W] */
    int8_t *inM, *inLM;        /* [A+1] */
} or_solver;

/* ---------------------------------------------------------------- helpers */
static inline int32_t var_of(int32_t lit) { return lit > 0 ? lit : -lit; }
static inline int lit_index(int32_t lit) { return 2 * var_of(lit) + (lit < 0); }
/* the value a literal asserts: +1 for T v, -1 for F v */
static inline int8_t lit_sign(int32_t lit) { return lit > 0 ? 1 : -1; }

static void fnv(or_solver *s, int32_t w) {
    /* FNV-1a, 64 bit, over the 4 little-endian bytes of w */
    uint32_t u = (uint32_t)w;
    for (int k = 0; k < 4; ++k) {
        s->st.trace_hash ^= (uint64_t)((u >> (8 * k)) & 0xffu);
        s->st.trace_hash *= 1099511628211ull;
    }
}

static int32_t ng_len(const or_solver *s, int64_t id) {
    return s->ng_off.a[id + 1] - s->ng_off.a[id];
}
static const int32_t *ng_ptr(const or_solver *s, int64_t id) {
    return s->ng_lits.a + s->ng_off.a[id];
}

static void add_nogood(or_solver *s, const int32_t *lits, int32_t n) {
    int32_t id = (int32_t)(s->ng_off.n - 1);
    for (int32_t k = 0; k < n; ++k) {
        iv_push(&s->ng_lits, lits[k]);
        iv_push(&s->map[lit_index(lits[k])], id);
    }
    iv_push(&s->ng_off, (int32_t)s->ng_lits.n);
}

/* bit of the decision at level l (l >= 2) */
static inline int32_t level_bit(const or_solver *s, int32_t l) {
    int32_t b = l - 1, top = 64 * s->W - 1;
    return b < top ? b : top;
}

/* --------------------------------------------------------- S0/S1 encoding */
/* Completion nogoods of the program (Sect. 2): for headed rule r with aux
 * atoms b, t, n: {F b, T t, T n}, {T b, F t}, {T b, F n}, {T t, F p} per
 * p in body+, {T n, T q} per q in body-, {F t} u {T p : body+},
 * {F n} u {F q : body-}; per atom p: {F p, T b_r} per r in rules(p) and
 * {T p} u {F b_r : r in rules(p)}; per constraint {T p : body+} u
 * {F q : body-}.  Generated in that order, then stably sorted by length. */
static int encode(or_solver *s, int32_t n_atoms, int32_t n_rules,
                  const int32_t *head, const int64_t *body_off,
                  const int32_t *body_lits) {
    const int32_t A = n_atoms;
    if (A < 0 || n_rules < 0) return OR_E_INVALID;
    if (n_rules > 0 && body_off[0] != 0) return OR_E_INVALID;
    for (int32_t r = 0; r < n_rules; ++r) {
        if (body_off[r + 1] < body_off[r]) return OR_E_INVALID;
        if (head[r] < 0 || head[r] > A) return OR_E_INVALID;
        for (int64_t k = body_off[r]; k < body_off[r + 1]; ++k)
            if (body_lits[k] == 0 || var_of(body_lits[k]) > A) return OR_E_INVALID;
    }
    int32_t Rh = 0;
    for (int32_t r = 0; r < n_rules; ++r) Rh += head[r] != 0;
    if ((int64_t)A + 3 * (int64_t)Rh > 0x3fffffff) return OR_E_INVALID;
    s->A = A;
    s->Rh = Rh;
    s->V = A + 3 * Rh;

    /* per headed rule: body+ and body- with repeated literals removed
     * (first occurrence kept); constraints likewise, a constraint holding
     * both p and not p is dropped (it can never be violated). */
    int64_t tot = n_rules > 0 ? body_off[n_rules] : 0;
    s->rhead = (int32_t *)calloc((size_t)Rh + 1, sizeof(int32_t));
    s->pos_off = (int32_t *)calloc((size_t)Rh + 1, sizeof(int32_t));
    s->neg_off = (int32_t *)calloc((size_t)Rh + 1, sizeof(int32_t));
    s->pos = (int32_t *)calloc((size_t)tot + 1, sizeof(int32_t));
    s->neg = (int32_t *)calloc((size_t)tot + 1, sizeof(int32_t));
    int32_t *cpos_off = (int32_t *)calloc((size_t)n_rules + 1, sizeof(int32_t));
    int32_t *cneg_off = (int32_t *)calloc((size_t)n_rules + 1, sizeof(int32_t));
    int32_t *cpos = (int32_t *)calloc((size_t)tot + 1, sizeof(int32_t));
    int32_t *cneg = (int32_t *)calloc((size_t)tot + 1, sizeof(int32_t));
    int32_t np = 0, nn = 0, j = 0, ncp = 0, ncn = 0, c = 0;
    for (int32_t r = 0; r < n_rules; ++r) {
        int32_t p0 = head[r] ? np : ncp, n0 = head[r] ? nn : ncn;
        int32_t *P = head[r] ? s->pos : cpos, *N = head[r] ? s->neg : cneg;
        int32_t *pp = head[r] ? &np : &ncp, *pn = head[r] ? &nn : &ncn;
        for (int64_t k = body_off[r]; k < body_off[r + 1]; ++k) {
            int32_t l = body_lits[k], dup = 0;
            for (int64_t k2 = body_off[r]; k2 < k; ++k2) dup |= body_lits[k2] == l;
            if (dup) continue;
            if (l > 0) P[(*pp)++] = l; else N[(*pn)++] = -l;
        }
        if (head[r]) {
            s->rhead[j] = head[r];
            s->pos_off[j + 1] = np;
            s->neg_off[j + 1] = nn;
            ++j;
        } else {
            int taut = 0;
            for (int32_t a = p0; a < ncp; ++a)
                for (int32_t b = n0; b < ncn; ++b) taut |= cpos[a] == cneg[b];
            if (taut) { ncp = p0; ncn = n0; continue; }
            cpos_off[c + 1] = ncp;
            cneg_off[c + 1] = ncn;
            ++c;
        }
    }
    s->Rc = c;

    /* generation order into a temporary CSR */
    ivec goff = {0}, glits = {0}, tmp = {0};
    iv_push(&goff, 0);
#define FLUSH() do { for (int64_t q = 0; q < tmp.n; ++q) iv_push(&glits, tmp.a[q]); \
                     iv_push(&goff, (int32_t)glits.n); tmp.n = 0; } while (0)
    for (j = 0; j < Rh; ++j) {
        int32_t b = A + 3 * j + 1, t = A + 3 * j + 2, n = A + 3 * j + 3;
        iv_push(&tmp, -b); iv_push(&tmp, t); iv_push(&tmp, n); FLUSH();
        iv_push(&tmp, b); iv_push(&tmp, -t); FLUSH();
        iv_push(&tmp, b); iv_push(&tmp, -n); FLUSH();
        for (int32_t k = s->pos_off[j]; k < s->pos_off[j + 1]; ++k) {
            iv_push(&tmp, t); iv_push(&tmp, -s->pos[k]); FLUSH();
        }
        for (int32_t k = s->neg_off[j]; k < s->neg_off[j + 1]; ++k) {
            iv_push(&tmp, n); iv_push(&tmp, s->neg[k]); FLUSH();
        }
        iv_push(&tmp, -t);
        for (int32_t k = s->pos_off[j]; k < s->pos_off[j + 1]; ++k) iv_push(&tmp, s->pos[k]);
        FLUSH();
        iv_push(&tmp, -n);
        for (int32_t k = s->neg_off[j]; k < s->neg_off[j + 1]; ++k) iv_push(&tmp, -s->neg[k]);
        FLUSH();
    }
    /* rules(p) in input order, as a CSR over atoms */
    int32_t *by_off = (int32_t *)calloc((size_t)A + 2, sizeof(int32_t));
    int32_t *by = (int32_t *)calloc((size_t)Rh + 1, sizeof(int32_t));
    for (j = 0; j < Rh; ++j) by_off[s->rhead[j] + 1] += 1;
    for (int32_t p = 1; p <= A; ++p) by_off[p + 1] += by_off[p];
    for (j = 0; j < Rh; ++j) by[by_off[s->rhead[j]]++] = j;
    for (int32_t p = A; p >= 1; --p) by_off[p] = by_off[p - 1];
    by_off[0] = 0;
    for (int32_t p = 1; p <= A; ++p) {
        for (int32_t k = by_off[p]; k < by_off[p + 1]; ++k) {
            iv_push(&tmp, -p); iv_push(&tmp, A + 3 * by[k] + 1); FLUSH();
        }
        iv_push(&tmp, p);
        for (int32_t k = by_off[p]; k < by_off[p + 1]; ++k) iv_push(&tmp, -(A + 3 * by[k] + 1));
        FLUSH();
    }
    free(by_off);
    free(by);
    for (int32_t k = 0; k < c; ++k) {
        for (int32_t q = cpos_off[k]; q < cpos_off[k + 1]; ++q) iv_push(&tmp, cpos[q]);
        for (int32_t q = cneg_off[k]; q < cneg_off[k + 1]; ++q) iv_push(&tmp, -cneg[q]);
        FLUSH();
    }
#undef FLUSH
    int64_t G = goff.n - 1;

    /* stable sort by length (Sect. 4: nogoods are stored by increasing
     * length): a counting sort, which keeps generation order within a length */
    int32_t maxlen = 0;
    for (int64_t g = 0; g < G; ++g) {
        int32_t L = goff.a[g + 1] - goff.a[g];
        if (L > maxlen) maxlen = L;
    }
    int64_t *start = (int64_t *)calloc((size_t)maxlen + 2, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(G > 0 ? G : 1));
    for (int64_t g = 0; g < G; ++g) start[goff.a[g + 1] - goff.a[g] + 1] += 1;
    for (int32_t L = 0; L <= maxlen; ++L) start[L + 1] += start[L];
    for (int64_t g = 0; g < G; ++g) order[start[goff.a[g + 1] - goff.a[g]]++] = g;
    s->map = (ivec *)calloc(2 * ((size_t)s->V + 1), sizeof(ivec));
    iv_push(&s->ng_off, 0);
    for (int64_t i = 0; i < G; ++i) {
        int64_t g = order[i];
        int32_t L = goff.a[g + 1] - goff.a[g];
        if (L == 0) s->has_empty_nogood = 1;
        add_nogood(s, glits.a + goff.a[g], L);
    }
    free(start);
    free(order);
    s->n0 = G;
    s->lits0 = s->ng_lits.n;

    s->occ = (int32_t *)calloc((size_t)A + 1, sizeof(int32_t));
    s->jw = (int32_t *)calloc((size_t)A + 1, sizeof(int32_t));
    s->act = (int32_t *)calloc((size_t)A + 1, sizeof(int32_t));
    for (int64_t g = 0; g < G; ++g) {
        /* the atoms of a nogood are distinct, so each counts once per nogood */
        int32_t len = s->ng_off.a[g + 1] - s->ng_off.a[g];
        for (int32_t k = s->ng_off.a[g]; k < s->ng_off.a[g + 1]; ++k) {
            int32_t v = var_of(s->ng_lits.a[k]);
            if (v <= A) {
                s->occ[v] += 1;
                if (len <= 16) s->jw[v] += 1 << (16 - len);
            }
        }
    }
    for (int32_t p = 0; p <= A; ++p) s->act[p] = s->occ[p];
    free(goff.a); free(glits.a); free(tmp.a);
    free(cpos_off); free(cneg_off); free(cpos); free(cneg);
    return 0;
}

/* ------------------------------------------------------------- lifecycle */
void or_free(void *h);

void *or_create(int32_t n_atoms, int32_t n_rules, const int32_t *head,
                const int64_t *body_off, const int32_t *body_lits,
                int32_t W, int32_t gate_mode, int32_t *err) {
    if (W < 1 || W > 1024 || (gate_mode != GATE_UNFOUNDED && gate_mode != GATE_ALLDEC)) {
        if (err) *err = OR_E_INVALID;
        return NULL;
    }
    or_solver *s = (or_solver *)calloc(1, sizeof(or_solver));
    s->W = W;
    s->gate_mode = gate_mode;
    int rc = encode(s, n_atoms, n_rules, head, body_off, body_lits);
    if (rc) {
        or_free(s);
        if (err) *err = rc;
        return NULL;
    }
    size_t V1 = (size_t)s->V + 1;
    s->val = (int8_t *)calloc(V1, 1);
    s->lvl = (int32_t *)calloc(V1, sizeof(int32_t));
    s->deps = (uint64_t *)calloc(V1 * W, sizeof(uint64_t));
    s->tmpdeps = (uint64_t *)calloc(V1 * W, sizeof(uint64_t));
    s->pend_B = (uint64_t *)calloc((size_t)W, sizeof(uint64_t));
    s->dec = (int32_t *)calloc((size_t)s->Rh + 2, sizeof(int32_t));
    s->win = (int32_t *)malloc(V1 * sizeof(int32_t));
    for (size_t v = 0; v < V1; ++v) s->win[v] = -1;
    s->touched = (int32_t *)calloc(V1, sizeof(int32_t));
    s->winsign = (int8_t *)calloc(V1, 1);
    s->inM = (int8_t *)calloc((size_t)s->A + 1, 1);
    s->inLM = (int8_t *)calloc((size_t)s->A + 1, 1);
    s->stamp = (int32_t *)calloc(V1, sizeof(int32_t));
    s->reason = (int32_t *)malloc(V1 * sizeof(int32_t));
    for (size_t v = 0; v < V1; ++v) s->reason[v] = -1;
    s->mark = (int32_t *)calloc(V1, sizeof(int32_t));
    s->cdl = 1;
    s->max_models = 1;
    s->learn_conflicts = 1;
    s->need_init = 1;
    s->st.trace_hash = 1469598103934665603ull;
    s->status = OR_RUNNING;
    s->last_step = ST_NONE;
    if (err) *err = 0;
    return s;
}

void or_free(void *h) {
    or_solver *s = (or_solver *)h;
    if (!s) return;
    free(s->rhead); free(s->pos_off); free(s->pos); free(s->neg_off); free(s->neg);
    free(s->ng_off.a); free(s->ng_lits.a);
    if (s->map)
        for (size_t i = 0; i < 2 * ((size_t)s->V + 1); ++i) free(s->map[i].a);
    free(s->map); free(s->occ); free(s->jw); free(s->act); free(s->score);
    free(s->val); free(s->lvl); free(s->deps); free(s->tmpdeps); free(s->pend_B);
    free(s->dec); free(s->frontier.a); free(s->win); free(s->winsign); free(s->touched);
    free(s->inM); free(s->inLM);
    free(s->stamp); free(s->reason); free(s->mark); free(s->models);
    free(s);
}

/* ------------------------------------------------------------------ steps */
static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* S3: every unit nogood {l} -- the static ones, then (after a restart) the
 * learned ones, in id order -- assigns the complement of l at level 1 with
 * empty Deps; two opposite units, or an empty nogood, mean no answer set. */
static int init_unit(or_solver *s, int64_t id) {
    int32_t l = ng_ptr(s, id)[0], x = var_of(l);
    int8_t want = (int8_t)-lit_sign(l);
    if (s->val[x] == 0) {
        s->val[x] = want;
        s->lvl[x] = 1;
        s->stamp[x] = s->clock;
        s->reason[x] = (int32_t)id;
        s->nass += 1;
        iv_push(&s->frontier, x);
    } else if (s->val[x] != want) {
        return 0;
    }
    return 1;
}

static void step_init(or_solver *s) {
    s->need_init = 0;
    if (s->has_empty_nogood) { s->status = OR_UNSAT; return; }
    s->frontier.n = 0;
    /* static nogoods are sorted by length: the units come first */
    for (int64_t id = 0; id < s->n0 && ng_len(s, id) <= 1; ++id)
        if (ng_len(s, id) == 1 && !init_unit(s, id)) { s->status = OR_UNSAT; return; }
    for (int64_t id = s->n0; id < s->n0 + s->n_learned; ++id) {
        if (ng_len(s, id) == 0) { s->status = OR_UNSAT; return; }
        if (ng_len(s, id) == 1 && !init_unit(s, id)) { s->status = OR_UNSAT; return; }
    }
    qsort(s->frontier.a, (size_t)s->frontier.n, sizeof(int32_t), cmp_i32);
    s->clock += 1;
}

/* Classification of nogood id against the current assignment:
 * 0 = other (satisfied or more than one open literal), 1 = violated,
 * 2 = unit; for unit, *u is the open literal. */
static int classify(const or_solver *s, int64_t id, int32_t *u) {
    const int32_t *L = ng_ptr(s, id);
    int32_t n = ng_len(s, id), open = 0, in = 0;
    for (int32_t k = 0; k < n; ++k) {
        int8_t v = s->val[var_of(L[k])];
        if (v == 0) { ++open; *u = L[k]; }
        else if (v == lit_sign(L[k])) ++in;
    }
    if (in == n) return 1;
    if (open == 1 && in == n - 1) return 2;
    return 0;
}

/* S4: one PropagateAndCheck round (Sect. 4.1) in Jacobi form.
 * S5: among the round's conflicts, keep the shortest, ties by lowest id. */
/* keep the K = learn_conflicts smallest distinct (length, id) conflicts */
static void note_conflict(or_solver *s, int32_t id) {
    const int32_t K = s->learn_conflicts;
    int32_t n = s->n_pend;
    for (int32_t i = 0; i < n; ++i)
        if (s->pend_ids[i] == id) return;
    int32_t pos = n;
    while (pos > 0) {
        int32_t o = s->pend_ids[pos - 1];
        if (ng_len(s, o) < ng_len(s, id) || (ng_len(s, o) == ng_len(s, id) && o < id)) break;
        --pos;
    }
    if (pos >= K) return;
    for (int32_t i = (n < K ? n : K - 1); i > pos; --i) s->pend_ids[i] = s->pend_ids[i - 1];
    s->pend_ids[pos] = id;
    if (n < K) s->n_pend = n + 1;
}

static void step_round(or_solver *s) {
    const int32_t W = s->W;
    int32_t nt = 0;
    s->n_pend = 0;
    /* phase 1: classify every visit against the snapshot, find winners */
    for (int64_t f = 0; f < s->frontier.n; ++f) {
        int32_t v = s->frontier.a[f];
        int32_t L = s->val[v] > 0 ? v : -v;
        const ivec *m = &s->map[lit_index(L)];
        for (int64_t q = 0; q < m->n; ++q) {
            int32_t id = m->a[q], u = 0;
            s->st.visits += 1;
            s->st.literal_checks += ng_len(s, id);
            int c = classify(s, id, &u);
            if (c == 1) {
                note_conflict(s, (int32_t)id);
            } else if (c == 2) {
                int32_t x = var_of(u);
                if (s->win[x] < 0) s->touched[nt++] = x;
                if (s->win[x] < 0 || id < s->win[x]) {
                    s->win[x] = id;
                    s->winsign[x] = (int8_t)-lit_sign(u);
                }
            }
        }
    }
    /* phase 2: a unit nogood implying the other value than its variable's
     * winner is a conflict (the clash of Alg. 2, made deterministic) */
    for (int64_t f = 0; f < s->frontier.n; ++f) {
        int32_t v = s->frontier.a[f];
        int32_t L = s->val[v] > 0 ? v : -v;
        const ivec *m = &s->map[lit_index(L)];
        for (int64_t q = 0; q < m->n; ++q) {
            int32_t id = m->a[q], u = 0;
            if (classify(s, id, &u) != 2) continue;
            int32_t x = var_of(u);
            if (s->winsign[x] != -lit_sign(u)) note_conflict(s, (int32_t)id);
        }
    }
    /* phase 3: Deps of each implied variable = OR of the Deps of the other
     * variables of its winning nogood (mk_dl_bitmap), all read before any
     * write so that they come from the snapshot */
    qsort(s->touched, (size_t)nt, sizeof(int32_t), cmp_i32);
    for (int32_t i = 0; i < nt; ++i) {
        int32_t x = s->touched[i], w = s->win[x];
        uint64_t *d = s->tmpdeps + (size_t)i * W;
        memset(d, 0, sizeof(uint64_t) * W);
        const int32_t *L = ng_ptr(s, w);
        for (int32_t k = 0; k < ng_len(s, w); ++k) {
            int32_t y = var_of(L[k]);
            if (y == x) continue;
            for (int32_t q = 0; q < W; ++q) d[q] |= s->deps[(size_t)y * W + q];
        }
        s->st.deps_reads += (int64_t)(ng_len(s, w) - 1) * W;
    }
    /* phase 4: apply every implication, even when a conflict was found */
    for (int32_t i = 0; i < nt; ++i) {
        int32_t x = s->touched[i];
        s->val[x] = s->winsign[x];
        s->lvl[x] = s->cdl;
        s->stamp[x] = s->clock;
        s->reason[x] = s->win[x];
        memcpy(s->deps + (size_t)x * W, s->tmpdeps + (size_t)i * W, sizeof(uint64_t) * W);
    }
    for (int32_t i = 0; i < nt; ++i) s->win[s->touched[i]] = -1;
    s->frontier.n = 0;
    for (int32_t i = 0; i < nt; ++i) iv_push(&s->frontier, s->touched[i]);
    s->clock += 1;
    s->nass += nt;
    s->st.rounds += 1;
    s->st.propagations += nt;
    if (s->n_pend > 0) {
        s->pend_kind = 1;
        s->pend_id = s->pend_ids[0];
    }
}

static const or_solver *g_sort_s;   /* comparator context (single-threaded use) */
static int cmp_assigned(const void *a, const void *b) {
    const or_solver *s = g_sort_s;
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (s->stamp[x] != s->stamp[y]) return s->stamp[x] < s->stamp[y] ? -1 : 1;
    return (x > y) - (x < y);
}

/* Res-learning (Alg. 3): starting from the conflict nogood (all its
 * literals true), while the latest-assigned literal sigma shares its level
 * with another literal, replace sigma by the other literals of the nogood
 * that implied it.  On return the nogood has a single literal at its top
 * level (the first UIP); *N holds its true literals by assignment order
 * (sigma last) and *bj the highest level of the others (at least 1).
 * Returns 0, leaving nothing allocated, when sigma has no implying nogood
 * (a CompleteAssignment literal): the caller learns by Fwd-learning. */
static int res_learn(or_solver *s, int32_t conf, int32_t **outN, int64_t *outn, int32_t *outbj) {
    s->epoch += 1;
    const int32_t ep = s->epoch;
    ivec d = {0};
    const int32_t *L = ng_ptr(s, conf);
    for (int32_t q = 0; q < ng_len(s, conf); ++q) {
        int32_t v = var_of(L[q]);
        if (s->mark[v] != ep) { s->mark[v] = ep; iv_push(&d, v); }
    }
    int32_t sig = -1, k = 0;
    for (;;) {
        sig = -1;
        for (int64_t i = 0; i < d.n; ++i) {
            int32_t v = d.a[i];
            if (s->mark[v] != ep) continue;
            if (sig < 0 || s->stamp[v] > s->stamp[sig] ||
                (s->stamp[v] == s->stamp[sig] && v > sig)) sig = v;
        }
        k = 0;
        for (int64_t i = 0; i < d.n; ++i) {
            int32_t v = d.a[i];
            if (s->mark[v] == ep && v != sig && s->lvl[v] > k) k = s->lvl[v];
        }
        if (s->lvl[sig] != k) break;
        int32_t e = s->reason[sig];
        if (e < 0) { free(d.a); return 0; }
        s->mark[sig] = 0;                      /* resolve sigma away ... */
        const int32_t *E = ng_ptr(s, e);
        for (int32_t q = 0; q < ng_len(s, e); ++q) {   /* ... with its reason */
            int32_t v = var_of(E[q]);
            if (v == sig || s->mark[v] == ep) continue;
            s->mark[v] = ep;
            iv_push(&d, v);
        }
    }
    int64_t n = 0;
    for (int64_t i = 0; i < d.n; ++i)
        if (s->mark[d.a[i]] == ep) d.a[n++] = d.a[i];
    g_sort_s = s;
    qsort(d.a, (size_t)n, sizeof(int32_t), cmp_assigned);
    int32_t *N = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) N[i] = s->val[d.a[i]] > 0 ? d.a[i] : -d.a[i];
    free(d.a);
    *outN = N;
    *outn = n;
    *outbj = k > 1 ? k : 1;
    return 1;
}

/* Restart: every variable is unassigned, the learned nogoods stay, and
 * InitialPropagation runs next. */
static void restart(or_solver *s) {
    const int32_t W = s->W;
    for (int32_t v = 1; v <= s->V; ++v) {
        s->val[v] = 0;
        s->lvl[v] = 0;
        memset(s->deps + (size_t)v * W, 0, sizeof(uint64_t) * W);
    }
    s->nass = 0;
    s->cdl = 1;
    s->frontier.n = 0;
    s->pend_kind = 0;
    s->pend_id = -1;
    s->n_pend = 0;
    s->need_init = 1;
    s->since_restart = 0;
    s->st.restarts += 1;
    fnv(s, 9);
}

/* B of a round conflict: the OR of the Deps of its variables */
static void conflict_B(or_solver *s, int32_t conf, uint64_t *B) {
    const int32_t W = s->W;
    memset(B, 0, sizeof(uint64_t) * W);
    const int32_t *L = ng_ptr(s, conf);
    for (int32_t k = 0; k < ng_len(s, conf); ++k) {
        int32_t y = var_of(L[k]);
        for (int32_t q = 0; q < W; ++q) B[q] |= s->deps[(size_t)y * W + q];
    }
}

/* A conflict that follows from level-1 facts alone (no answer set): under
 * Fwd-learning B = 0; under Res-learning a round conflict with no literal
 * above level 1.  conf >= 0 is a round conflict, -1 the pending gate
 * conflict (its B is in pend_B). */
static int at_root(or_solver *s, int32_t conf) {
    if (conf >= 0 && s->learning == LEARN_RES) {
        const int32_t *L = ng_ptr(s, conf);
        for (int32_t k = 0; k < ng_len(s, conf); ++k)
            if (s->lvl[var_of(L[k])] > 1) return 0;
        return 1;
    }
    if (conf >= 0) conflict_B(s, conf, s->pend_B);
    for (int32_t q = 0; q < s->W; ++q)
        if (s->pend_B[q]) return 0;
    return 1;
}

/* S6: the nogood learned from one conflict and its backjump level --
 * Res-learning (Alg. 3) for a round conflict when selected, else (and when
 * resolution reaches a literal without reason) Fwd-learning (Alg. 4): the
 * decision literals of levels(B), ascending, and the second-highest level */
static void learn_one(or_solver *s, int32_t conf, int32_t **outN, int64_t *outn,
                      int32_t *outbj) {
    if (conf >= 0 && s->learning == LEARN_RES && res_learn(s, conf, outN, outn, outbj)) return;
    uint64_t *B = s->pend_B;
    if (conf >= 0) conflict_B(s, conf, B);
    /* levels(B), ascending: level l in 2..64W-1 for bit l-1, plus every
     * level 64W..cdl when the saturated bit 64W-1 is set */
    ivec lev = {0};
    for (int32_t l = 2; l <= s->cdl; ++l) {
        int32_t b = level_bit(s, l);
        if ((B[b / 64] >> (b % 64)) & 1u) iv_push(&lev, l);
    }
    int64_t nN = lev.n;
    int32_t *N = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nN > 0 ? nN : 1));
    for (int64_t i = 0; i < nN; ++i) N[i] = s->dec[lev.a[i]];
    *outbj = nN >= 2 ? lev.a[nN - 2] : 1;
    free(lev.a);
    *outN = N;
    *outn = nN;
}

/* S6 + S7: Learning of the pending conflict -- or, with learn_conflicts > 1,
 * of each selected round conflict in rank order -- then Backjump to the
 * lowest backjump level among the learned nogoods and assertion of the
 * latest literal of the first nogood that reaches it. */
static void step_learn(or_solver *s, const or_limits *lim) {
    const int32_t W = s->W;
    const int32_t n_sel = s->pend_kind == 1 ? s->n_pend : 1;
    int32_t conf[8];
    for (int32_t i = 0; i < n_sel; ++i) conf[i] = s->pend_kind == 1 ? s->pend_ids[i] : -1;
    for (int32_t i = 0; i < n_sel; ++i)
        if (at_root(s, conf[i])) {
            s->st.conflicts += 1;
            s->status = OR_UNSAT;
            return;
        }
    if (lim && lim->max_conflicts >= 0 && s->st.conflicts >= lim->max_conflicts) {
        s->status = OR_UNKNOWN;
        return;
    }
    s->st.conflicts += 1;
    s->dec_since_conf = 0;
    if (s->use_score) {
        s->consec += 1;
        if (s->fallback_after >= 0 && s->consec >= s->fallback_after) {
            s->use_score = 0;
            fnv(s, 7);
        }
    }
    int32_t *Nb = NULL, bjb = 0, idb = -1;
    int64_t nb = 0;
    for (int32_t i = 0; i < n_sel; ++i) {
        int32_t *N = NULL, bj = 1;
        int64_t nN = 0;
        learn_one(s, conf[i], &N, &nN, &bj);
        if ((lim && lim->learned_cap_ng >= 0 && s->n_learned + 1 > lim->learned_cap_ng) ||
            (lim && lim->learned_cap_lits >= 0 && s->learned_lits + nN > lim->learned_cap_lits)) {
            free(N);
            free(Nb);
            s->status = OR_UNKNOWN;
            return;
        }
        const int32_t newid = (int32_t)(s->n0 + s->n_learned);
        add_nogood(s, N, (int32_t)nN);
        s->n_learned += 1;
        s->learned_lits += nN;
        s->st.learned += 1;
        s->st.learned_len += nN;
        if (s->decision == DEC_ACTIVITY) {
            /* activity: every literal bumps its atom (an auxiliary variable
             * of rule r stands for the head of r); halve all every 64 nogoods */
            for (int64_t q = 0; q < nN; ++q) {
                int32_t v = var_of(N[q]);
                int32_t p = v <= s->A ? v : s->rhead[(v - s->A - 1) / 3];
                s->act[p] += 8;
            }
            if (s->st.learned % 64 == 0)
                for (int32_t p = 0; p <= s->A; ++p) s->act[p] >>= 1;
        }
        fnv(s, 2); fnv(s, conf[i]); fnv(s, (int32_t)nN); fnv(s, bj);
        if (idb < 0 || bj < bjb) {
            free(Nb);
            Nb = N; nb = nN; bjb = bj; idb = newid;
        } else {
            free(N);
        }
    }
    s->since_restart += 1;
    if (s->restart_every > 0 && s->since_restart >= s->restart_every) {
        free(Nb);
        restart(s);
        return;
    }
    /* Backjump: unassign everything above bj */
    for (int32_t v = 1; v <= s->V; ++v)
        if (s->lvl[v] > bjb) {
            s->nass -= s->val[v] != 0;
            s->val[v] = 0;
            s->lvl[v] = 0;
            memset(s->deps + (size_t)v * W, 0, sizeof(uint64_t) * W);
        }
    s->cdl = bjb;
    /* assert the complement of the chosen nogood's latest literal at bj, its
     * Deps those of the nogood's other variables */
    int32_t toplit = Nb[nb - 1], x = var_of(toplit);
    s->nass += 1;
    s->val[x] = (int8_t)-lit_sign(toplit);
    s->lvl[x] = bjb;
    s->stamp[x] = s->clock++;
    s->reason[x] = idb;
    uint64_t *d = s->deps + (size_t)x * W;
    memset(d, 0, sizeof(uint64_t) * W);
    for (int64_t i = 0; i + 1 < nb; ++i) {
        int32_t y = var_of(Nb[i]);
        for (int32_t q = 0; q < W; ++q) d[q] |= s->deps[(size_t)y * W + q];
    }
    s->frontier.n = 0;
    iv_push(&s->frontier, x);
    s->pend_kind = 0;
    s->pend_id = -1;
    s->n_pend = 0;
    free(Nb);
}

/* S8: pick an applicable rule (T t_r in A, F n_r not in A, head unassigned)
 * by the highest score of its head, ties to the lowest rule. */
static int32_t find_decision(const or_solver *s) {
    const int32_t *sc = s->use_score ? s->score
                      : s->decision == DEC_JW ? s->jw
                      : s->decision == DEC_ACTIVITY ? s->act : s->occ;
    int32_t best = -1;
    int64_t bestkey = INT64_MIN;
    for (int32_t j = 0; j < s->Rh; ++j) {
        int32_t p = s->rhead[j], t = s->A + 3 * j + 2, n = s->A + 3 * j + 3;
        if (s->val[p] != 0 || s->val[t] != 1 || s->val[n] == -1) continue;
        if ((int64_t)sc[p] > bestkey) { bestkey = sc[p]; best = j; }
    }
    return best;
}

/* the search stands at a conflict-free fixpoint: if a decision led here,
 * the run of consecutive conflicts is over */
static void at_fixpoint(or_solver *s) {
    if (s->dec_since_conf) s->consec = 0;
}

static void step_decide(or_solver *s, int32_t j) {
    const int32_t W = s->W;
    at_fixpoint(s);
    s->dec_since_conf = 1;
    int32_t b = s->A + 3 * j + 1;
    s->cdl += 1;
    s->dec[s->cdl] = b;
    s->nass += 1;
    s->val[b] = 1;
    s->lvl[b] = s->cdl;
    s->stamp[b] = s->clock++;
    s->reason[b] = -1;
    uint64_t *d = s->deps + (size_t)b * W;
    memset(d, 0, sizeof(uint64_t) * W);
    int32_t bit = level_bit(s, s->cdl);
    d[bit / 64] |= 1ull << (bit % 64);
    s->frontier.n = 0;
    iv_push(&s->frontier, b);
    s->st.decisions += 1;
    fnv(s, 1); fnv(s, j);
}

/* Lookahead Decision (parallel lookahead, named in the Conclusions as a
 * refinement to consider; this reading is the builder's): the K applicable
 * rules with the highest (score of the head, -r) are tried in that order.  A
 * trial decides T b_r at the next level and runs rounds until a fixpoint or
 * a conflict.  A trial that ends in a conflict, or leaves every variable
 * assigned, stands as the Decision (the search goes on from there: Learning,
 * or the stability gate).  Otherwise the variables it assigned are counted
 * and it is undone (everything above the current level unassigned).  When no
 * trial stands, the candidate whose trial assigned the most variables (the
 * earliest on ties) is decided.  Trial rounds count as rounds; an undone trial
 * adds the events (10, rule, count) to the trace hash, and the Decision that
 * stands or is taken adds (1, rule) and one decision. */
static int32_t top_candidates(const or_solver *s, int32_t K, int32_t *out) {
    const int32_t *sc = s->use_score ? s->score
                      : s->decision == DEC_JW ? s->jw
                      : s->decision == DEC_ACTIVITY ? s->act : s->occ;
    int32_t n = 0;
    int64_t keyv[8];
    for (int32_t j = 0; j < s->Rh; ++j) {
        int32_t p = s->rhead[j], t = s->A + 3 * j + 2, nn = s->A + 3 * j + 3;
        if (s->val[p] != 0 || s->val[t] != 1 || s->val[nn] == -1) continue;
        /* key (score, -j): insert into the sorted list of the best K */
        int64_t key = (int64_t)sc[p] * ((int64_t)1 << 32) - j;
        int32_t at = n;
        while (at > 0 && keyv[at - 1] < key) --at;
        if (at >= K) continue;
        int32_t last = n < K ? n : K - 1;
        for (int32_t q = last; q > at; --q) { keyv[q] = keyv[q - 1]; out[q] = out[q - 1]; }
        keyv[at] = key;
        out[at] = j;
        if (n < K) ++n;
    }
    return n;
}

static void decide_raw(or_solver *s, int32_t j) {
    const int32_t W = s->W;
    int32_t b = s->A + 3 * j + 1;
    s->cdl += 1;
    s->dec[s->cdl] = b;
    s->nass += 1;
    s->val[b] = 1;
    s->lvl[b] = s->cdl;
    s->stamp[b] = s->clock++;
    s->reason[b] = -1;
    uint64_t *d = s->deps + (size_t)b * W;
    memset(d, 0, sizeof(uint64_t) * W);
    int32_t bit = level_bit(s, s->cdl);
    d[bit / 64] |= 1ull << (bit % 64);
    s->frontier.n = 0;
    iv_push(&s->frontier, b);
}

static void step_lookahead(or_solver *s, int32_t j0) {
    int32_t cand[8];
    int32_t n = top_candidates(s, s->lookahead, cand);
    if (n <= 1) { step_decide(s, j0); return; }
    at_fixpoint(s);
    const int32_t consec0 = s->consec, since0 = s->dec_since_conf, cdl0 = s->cdl;
    const int64_t nass0 = s->nass;
    int32_t best = -1;
    int64_t best_p = -1;
    for (int32_t i = 0; i < n; ++i) {
        decide_raw(s, cand[i]);
        s->dec_since_conf = 1;
        while (s->frontier.n > 0 && s->pend_kind == 0) step_round(s);
        if (s->pend_kind != 0 || s->nass == s->V) {
            s->st.decisions += 1;
            fnv(s, 1); fnv(s, cand[i]);
            return;
        }
        const int64_t p = s->nass - nass0;
        fnv(s, 10); fnv(s, cand[i]); fnv(s, (int32_t)p);
        for (int32_t v = 1; v <= s->V; ++v) {
            if (s->lvl[v] <= cdl0) continue;
            s->val[v] = 0;
            s->lvl[v] = 0;
            memset(s->deps + (size_t)v * s->W, 0, sizeof(uint64_t) * s->W);
        }
        s->nass = nass0;
        s->cdl = cdl0;
        s->frontier.n = 0;
        s->consec = consec0;
        s->dec_since_conf = since0;
        if (p > best_p) { best_p = p; best = cand[i]; }
    }
    step_decide(s, best);
}

/* S9: CompleteAssignment -- every unassigned original atom becomes false at
 * level cdl, depending on every decision made so far. */
static void step_complete(or_solver *s) {
    const int32_t W = s->W;
    at_fixpoint(s);
    s->frontier.n = 0;
    for (int32_t p = 1; p <= s->A; ++p) {
        if (s->val[p] != 0) continue;
        s->val[p] = -1;
        s->nass += 1;
        s->lvl[p] = s->cdl;
        s->stamp[p] = s->clock;
        s->reason[p] = -1;
        uint64_t *d = s->deps + (size_t)p * W;
        memset(d, 0, sizeof(uint64_t) * W);
        for (int32_t l = 2; l <= s->cdl; ++l) {
            int32_t bit = level_bit(s, l);
            d[bit / 64] |= 1ull << (bit % 64);
        }
        iv_push(&s->frontier, p);
    }
    s->clock += 1;
    s->st.completes += 1;
    fnv(s, 3); fnv(s, (int32_t)s->frontier.n);
    if (s->frontier.n == 0) s->status = OR_E_INTERNAL;
}

/* S10: M = true original atoms; M is an answer set iff M equals the least
 * model of the reduct (rules whose body- misses M, with body- deleted). */
static void step_gate(or_solver *s, const or_limits *lim) {
    const int32_t A = s->A, W = s->W;
    at_fixpoint(s);
    for (int32_t p = 1; p <= A; ++p) { s->inM[p] = s->val[p] == 1; s->inLM[p] = 0; }
    for (int changed = 1; changed;) {
        changed = 0;
        for (int32_t j = 0; j < s->Rh; ++j) {
            int32_t h = s->rhead[j], ok = !s->inLM[h];
            for (int32_t k = s->neg_off[j]; ok && k < s->neg_off[j + 1]; ++k) ok = !s->inM[s->neg[k]];
            for (int32_t k = s->pos_off[j]; ok && k < s->pos_off[j + 1]; ++k) ok = s->inLM[s->pos[k]];
            if (ok) { s->inLM[h] = 1; changed = 1; }
        }
    }
    int32_t u = 0;
    for (int32_t p = 1; p <= A && !u; ++p)
        if (s->inM[p] && !s->inLM[p]) u = p;
    if (!u) {
        /* M is an answer set */
        if (s->st.models == s->models_cap) {
            s->models_cap = s->models_cap ? 2 * s->models_cap : 4;
            s->models = (uint8_t *)realloc(s->models, (size_t)(s->models_cap * (A > 0 ? A : 1)));
        }
        for (int32_t p = 1; p <= A; ++p) s->models[s->st.models * A + p - 1] = (uint8_t)s->inM[p];
        s->st.models += 1;
        if (s->max_models == 1) { s->status = OR_SAT; return; }
        fnv(s, 8); fnv(s, (int32_t)s->st.models);
        if (s->max_models > 0 && s->st.models >= s->max_models) { s->status = OR_SAT; return; }
        /* block M by {T p : p in M}, then restart */
        int32_t n = 0;
        for (int32_t p = 1; p <= A; ++p) n += s->inM[p];
        if ((lim && lim->learned_cap_ng >= 0 && s->n_learned + 1 > lim->learned_cap_ng) ||
            (lim && lim->learned_cap_lits >= 0 && s->learned_lits + n > lim->learned_cap_lits)) {
            s->status = OR_UNKNOWN;
            return;
        }
        int32_t *N = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        n = 0;
        for (int32_t p = 1; p <= A; ++p)
            if (s->inM[p]) N[n++] = p;
        add_nogood(s, N, n);
        free(N);
        s->n_learned += 1;
        s->learned_lits += n;
        restart(s);
        return;
    }
    s->st.gate_failures += 1;
    uint64_t *B = s->pend_B;
    memset(B, 0, sizeof(uint64_t) * W);
    if (s->gate_mode == GATE_ALLDEC) {
        for (int32_t l = 2; l <= s->cdl; ++l) {
            int32_t bit = level_bit(s, l);
            B[bit / 64] |= 1ull << (bit % 64);
        }
    } else {
        /* loop nogood of U = M \ LM: T u together with F b_r for every
         * external support r (head in U, body+ disjoint from U) */
        for (int32_t q = 0; q < W; ++q) B[q] |= s->deps[(size_t)u * W + q];
        for (int32_t j = 0; j < s->Rh; ++j) {
            int32_t h = s->rhead[j];
            if (!(s->inM[h] && !s->inLM[h])) continue;
            int ext = 1;
            for (int32_t k = s->pos_off[j]; ext && k < s->pos_off[j + 1]; ++k) {
                int32_t p = s->pos[k];
                ext = !(s->inM[p] && !s->inLM[p]);
            }
            if (!ext) continue;
            int32_t b = A + 3 * j + 1;
            for (int32_t q = 0; q < W; ++q) B[q] |= s->deps[(size_t)b * W + q];
        }
    }
    s->pend_kind = 2;
    s->pend_id = -1;
}

/* ----------------------------------------------------------- public API */
/* which step comes next; *j gets the chosen rule for a decision */
static int32_t next_step(or_solver *s, int32_t *j) {
    *j = -1;
    if (s->status != OR_RUNNING) return ST_DONE;
    if (s->need_init) return ST_INIT;
    if (s->pend_kind) return ST_LEARN;
    if (s->frontier.n > 0) return ST_ROUND;
    if (s->nass == s->V) return ST_GATE;
    *j = find_decision(s);
    return *j >= 0 ? ST_DECIDE : ST_COMPLETE;
}

int32_t or_next_step(void *h) {
    int32_t j;
    return next_step((or_solver *)h, &j);
}

int32_t or_step(void *h, const or_limits *lim) {
    or_solver *s = (or_solver *)h;
    int32_t j, k = next_step(s, &j);
    switch (k) {
    case ST_INIT: step_init(s); break;
    case ST_ROUND: step_round(s); break;
    case ST_LEARN: step_learn(s, lim); break;
    case ST_DECIDE:
        if (s->lookahead > 1) step_lookahead(s, j);
        else step_decide(s, j);
        break;
    case ST_COMPLETE: step_complete(s); break;
    case ST_GATE: step_gate(s, lim); break;
    default: return s->status;
    }
    s->last_step = k;
    if ((s->status == OR_UNSAT || s->status == OR_UNKNOWN) && s->st.models > 0) {
        /* the search ended after answer sets were found */
        s->exhausted = s->status == OR_UNSAT;
        s->status = OR_SAT;
    }
    if (s->status == OR_SAT) fnv(s, 4);
    else if (s->status == OR_UNSAT) fnv(s, 5);
    else if (s->status == OR_UNKNOWN) fnv(s, 6);
    return s->status;
}

/* runs up to max_steps steps (all when max_steps < 0) */
int32_t or_run(void *h, const or_limits *lim, int64_t max_steps) {
    or_solver *s = (or_solver *)h;
    for (int64_t i = 0; (max_steps < 0 || i < max_steps) && s->status == OR_RUNNING; ++i)
        or_step(s, lim);
    return s->status;
}

/* dims: [V, A, Rh, n_static_nogoods, static_lits, W, cdl, frontier size,
 *        n_learned, learned_lits, pending kind, pending id, status, last step,
 *        constraints kept, answer sets exhausted] */
void or_dims(void *h, int64_t *d) {
    or_solver *s = (or_solver *)h;
    d[0] = s->V; d[1] = s->A; d[2] = s->Rh; d[3] = s->n0; d[4] = s->lits0;
    d[5] = s->W; d[6] = s->cdl; d[7] = s->frontier.n; d[8] = s->n_learned;
    d[9] = s->learned_lits; d[10] = s->pend_kind; d[11] = s->pend_id;
    d[12] = s->status; d[13] = s->last_step; d[14] = s->Rc; d[15] = s->exhausted;
}

/* all nogoods (static then learned) as CSR */
void or_nogoods(void *h, int32_t *off, int32_t *lits) {
    or_solver *s = (or_solver *)h;
    memcpy(off, s->ng_off.a, sizeof(int32_t) * (size_t)s->ng_off.n);
    memcpy(lits, s->ng_lits.a, sizeof(int32_t) * (size_t)s->ng_lits.n);
}

/* Supply per-atom decision scores (score[p] for atom p = 1..A; score[0] is
 * ignored) before the first step.  Returns 0, or OR_E_INVALID after the
 * search has started. */
int32_t or_set_scores(void *h, const int32_t *score, int32_t fallback_after) {
    or_solver *s = (or_solver *)h;
    if (s->last_step != ST_NONE || !score) return OR_E_INVALID;
    if (!s->score) s->score = (int32_t *)calloc((size_t)s->A + 1, sizeof(int32_t));
    memcpy(s->score, score, sizeof(int32_t) * ((size_t)s->A + 1));
    s->score[0] = 0;
    s->use_score = 1;
    s->fallback_after = fallback_after;
    s->consec = 0;
    s->dec_since_conf = 0;
    return 0;
}

/* Choose the Decision score when no per-atom scores are supplied (DEC_OCC,
 * DEC_JW, DEC_ACTIVITY) before the first step.  Returns 0, or OR_E_INVALID. */
int32_t or_set_decision(void *h, int32_t mode) {
    or_solver *s = (or_solver *)h;
    if (s->last_step != ST_NONE || (mode != DEC_OCC && mode != DEC_JW && mode != DEC_ACTIVITY))
        return OR_E_INVALID;
    s->decision = mode;
    return 0;
}

/* static scores of atoms 0..A: kind 0 occurrences, 1 Jeroslow-Wang,
 * 2 current activity */
void or_atom_scores(void *h, int32_t kind, int32_t *out) {
    or_solver *s = (or_solver *)h;
    const int32_t *src = kind == 1 ? s->jw : kind == 2 ? s->act : s->occ;
    memcpy(out, src, sizeof(int32_t) * ((size_t)s->A + 1));
}

/* Choose the Learning step (LEARN_FWD, LEARN_RES) before the first step.
 * Returns 0, or OR_E_INVALID. */
int32_t or_set_learning(void *h, int32_t mode) {
    or_solver *s = (or_solver *)h;
    if (s->last_step != ST_NONE || (mode != LEARN_FWD && mode != LEARN_RES)) return OR_E_INVALID;
    if (mode == LEARN_RES && s->lookahead > 1) return OR_E_INVALID;
    s->learning = mode;
    return 0;
}

/* Ask for up to max_models answer sets (0: all; 1, the default, is the plain
 * search) and restart every restart_every conflicts (0: never), before the
 * first step.  Returns 0, or OR_E_INVALID. */
int32_t or_set_enum(void *h, int64_t max_models, int64_t restart_every) {
    or_solver *s = (or_solver *)h;
    if (s->last_step != ST_NONE || max_models < 0 || restart_every < 0) return OR_E_INVALID;
    s->max_models = max_models;
    s->restart_every = restart_every;
    return 0;
}

/* Learn up to k (1..8) round conflicts per Learning step (ranked by length,
 * then id), before the first step.  Returns 0, or OR_E_INVALID. */
int32_t or_set_learn_conflicts(void *h, int32_t k) {
    or_solver *s = (or_solver *)h;
    if (s->last_step != ST_NONE || k < 1 || k > 8) return OR_E_INVALID;
    s->learn_conflicts = k;
    return 0;
}

int32_t or_set_lookahead(void *h, int32_t k) {
    or_solver *s = (or_solver *)h;
    if (s->last_step != ST_NONE || k < 0 || k > 8) return OR_E_INVALID;
    if (k > 1 && s->learning != LEARN_FWD) return OR_E_INVALID;
    s->lookahead = k;
    return 0;
}

/* the answer sets found so far: out[k*A + p-1] = 1 iff atom p is true in
 * the k-th (at most max_out of them); returns how many were found */
int64_t or_models(void *h, uint8_t *out, int64_t max_out) {
    or_solver *s = (or_solver *)h;
    int64_t n = s->st.models < max_out ? s->st.models : max_out;
    if (n > 0) memcpy(out, s->models, (size_t)(n * s->A));
    return s->st.models;
}

/* 1 while the supplied scores drive Decision, 0 after the fallback (or when
 * none were supplied); *consec gets the current run of conflicts */
int32_t or_score_mode(void *h, int32_t *consec) {
    or_solver *s = (or_solver *)h;
    if (consec) *consec = s->consec;
    return s->use_score;
}

void or_occ(void *h, int32_t *occ) {
    or_solver *s = (or_solver *)h;
    memcpy(occ, s->occ, sizeof(int32_t) * ((size_t)s->A + 1));
}

/* state: val[V+1], lvl[V+1], deps[(V+1)W], dec[cdl+1], frontier[n] */
void or_state(void *h, int8_t *val, int32_t *lvl, uint64_t *deps, int32_t *dec,
              int32_t *frontier) {
    or_solver *s = (or_solver *)h;
    size_t V1 = (size_t)s->V + 1;
    memcpy(val, s->val, V1);
    memcpy(lvl, s->lvl, V1 * sizeof(int32_t));
    memcpy(deps, s->deps, V1 * s->W * sizeof(uint64_t));
    memset(dec, 0, sizeof(int32_t) * ((size_t)s->cdl + 1));
    for (int32_t l = 2; l <= s->cdl; ++l) dec[l] = s->dec[l];
    memcpy(frontier, s->frontier.a, sizeof(int32_t) * (size_t)s->frontier.n);
}

void or_get_stats(void *h, or_stats *out) { *out = ((or_solver *)h)->st; }

/* model over original atoms: model[p-1] = 1 iff p is true in the first
 * answer set found (before one is found: in the current assignment) */
void or_model(void *h, uint8_t *model) {
    or_solver *s = (or_solver *)h;
    if (s->st.models > 0) {
        memcpy(model, s->models, (size_t)s->A);
        return;
    }
    for (int32_t p = 1; p <= s->A; ++p) model[p - 1] = s->val[p] == 1;
}

/* one-call solve for timing: encode, run to a verdict, copy the model */
int32_t or_solve(int32_t n_atoms, int32_t n_rules, const int32_t *head,
                 const int64_t *body_off, const int32_t *body_lits, int32_t W,
                 int32_t gate_mode, const or_limits *lim, uint8_t *model,
                 or_stats *st, const int32_t *score, int32_t fallback_after,
                 int32_t learning, int64_t max_models, int64_t restart_every,
                 int32_t decision, int32_t learn_conflicts, int32_t lookahead) {
    int32_t err = 0;
    void *h = or_create(n_atoms, n_rules, head, body_off, body_lits, W, gate_mode, &err);
    if (!h) return err;
    if (score) or_set_scores(h, score, fallback_after);
    if (or_set_learning(h, learning) != 0 || or_set_enum(h, max_models, restart_every) != 0 ||
        (!score && or_set_decision(h, decision) != 0) ||
        or_set_learn_conflicts(h, learn_conflicts) != 0 || or_set_lookahead(h, lookahead) != 0) {
        or_free(h);
        return OR_E_INVALID;
    }
    int32_t rc = or_run(h, lim, -1);
    if (model && rc == OR_SAT) or_model(h, model);
    if (st) or_get_stats(h, st);
    or_free(h);
    return rc;
}
