/*
 * asp.h -- C ABI of libasp, a GPU (gfx950) implementation of the
 * conflict-driven ASP solver of Dovier, Formisano and Vella,
 * "GPU-based parallelism for ASP-solving".
 *
 * Problem (Sect. 2 and Alg. 1): given a ground normal program P, compute its
 * completion nogoods Delta on the host, then search on the device for the
 * first answer set (A^T restricted to atoms(P)) or report that none exists.
 * The device search alternates PropagateAndCheck (Sect. 4.1, Alg. 2), the
 * parallel Fwd-learning (Sect. 4.2, Alg. 4) with Backjump, and a Decision
 * step that follows ASP computations (Sect. 2; Preliminaries), closing with
 * CompleteAssignment.  A stability check of total assignments (M = least
 * model of the Gelfond-Lifschitz reduct, the answer-set definition of the
 * Preliminaries) turns unfounded models into conflicts.
 *
 * Conventions for every function below:
 *  - all functions are extern "C", never throw, and return an int32 status;
 *    negative values are errors, and asp_last_error() gives a message for the
 *    calling thread;
 *  - host arrays are owned by the caller and copied during the call;
 *  - device memory is never allocated by the library: the caller passes a
 *    device arena (e.g. a torch uint8 tensor) of the size the library asks
 *    for, and must keep it alive while the handle uses it;
 *  - "stream" is a hipStream_t passed as void* (NULL = default stream);
 *  - one handle may be used by one thread at a time.
 *
 * Literals are signed int32: +v is "v true" (T v), -v is "v false" (F v).
 * Variables 1..n_atoms are the program's atoms; headed rule j (0-based, in
 * input order among headed rules) owns the auxiliary variables
 * b_j = n_atoms+3j+1, t_j = n_atoms+3j+2, n_j = n_atoms+3j+3 of the
 * completion (Sect. 2: b_r <-> t_r and n_r, t_r <-> body+, n_r <-> not body-).
 */
#ifndef ASP_H
#define ASP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ statuses */
#define ASP_OK           0
#define ASP_SAT          1   /* an answer set was found */
#define ASP_UNSAT        2   /* the program has no answer set */
#define ASP_UNKNOWN      3   /* a budget or capacity limit stopped the search */
#define ASP_FIXPOINT     4   /* propagation reached a fixpoint without conflict */
#define ASP_CONFLICT     5   /* propagation found a conflict (pending analysis) */
#define ASP_RUNNING      6   /* a step budget ended while the search is open */
#define ASP_E_INVALID   -1   /* malformed input or argument */
#define ASP_E_CAPACITY  -2   /* arena too small, or a size beyond the layout */
#define ASP_E_DEVICE    -3   /* a HIP runtime call failed */
#define ASP_E_STATE     -4   /* wrong call order for this handle */
#define ASP_E_INTERNAL  -5   /* an internal consistency check failed */
#define ASP_E_TIMEOUT   -6   /* the device-side wall-clock guard fired */

/* Search step kinds, as reported by asp_run_steps. */
#define ASP_STEP_NONE      0
#define ASP_STEP_INIT      1  /* InitialPropagation (Alg. 1) */
#define ASP_STEP_ROUND     2  /* one PropagateAndCheck round (Sect. 4.1) */
#define ASP_STEP_LEARN     3  /* Fwd-learning + Backjump (Sect. 4.2, Alg. 1) */
#define ASP_STEP_DECIDE    4  /* ASP-computation Decision (Sect. 2) */
#define ASP_STEP_COMPLETE  5  /* CompleteAssignment (Sect. 2) */
#define ASP_STEP_GATE      6  /* stability check of a total assignment */
#define ASP_STEP_DONE      7

#define ASP_GATE_UNFOUNDED 0  /* learn from the unfounded set's loop nogood */
#define ASP_GATE_ALLDEC    1  /* learn the nogood of all current decisions */

/* Decision heuristics (Sect. 2, the ASP-computation Decision: an applicable
 * rule is chosen by a score of its head, ties to the lowest rule). */
#define ASP_LEARN_FWD      0  /* Fwd-learning from Deps bitmaps (Sect. 4.2, Alg. 4) */
#define ASP_LEARN_RES      1  /* Res-learning: resolution to the first UIP (Alg. 3);
                                 stability-gate conflicts, and resolutions that
                                 reach a CompleteAssignment literal, use
                                 Fwd-learning */

#define ASP_DECISION_OCC   0  /* occurrences of the head in Delta_0 */
#define ASP_DECISION_SCORE 1  /* per-atom integer scores set on the device
                                 (asp_set_scores, or the learned scorer of
                                 asp_score_program / asp_score_batch) */
#define ASP_DECISION_JW    2  /* Jeroslow-Wang score of the head over Delta_0,
                                 sum of 2^(16-|delta|) over the nogoods
                                 holding a literal of it (none beyond 16
                                 literals) */
#define ASP_DECISION_ACTIVITY 3  /* activity of the head: starts at its
                                 occurrence count; every literal of a nogood
                                 learned from a conflict adds 8 to its atom
                                 (an auxiliary variable of rule r counts for
                                 the head of r); all halved after every 64th
                                 such nogood */

typedef struct asp_program asp_program;
typedef struct asp_batch asp_batch;

/* Structural options; they are part of the search semantics (the CPU
 * reference must use the same values to reproduce a run). */
typedef struct {
    int32_t W;                 /* 64-bit words of the Deps bitmap per variable,
                                  1..64; the decision at level l >= 2 sets bit
                                  min(l-1, 64W-1) (Sect. 4.2) */
    int32_t gate;              /* ASP_GATE_UNFOUNDED or ASP_GATE_ALLDEC */
    int64_t learned_cap_ng;    /* learned nogoods kept per instance; exceeding
                                  it ends the search with ASP_UNKNOWN */
    int64_t learned_cap_lits;  /* learned literals kept per instance; idem */
    int32_t decision;          /* ASP_DECISION_OCC, _SCORE, _JW or _ACTIVITY */
    int32_t fallback_after;    /* ASP_DECISION_SCORE: after this many
                                  conflicts in a row (the count restarts when a
                                  decision's propagation ends at a
                                  conflict-free fixpoint) the occurrence
                                  heuristic takes over for the rest of the
                                  search; < 0 never.  Default 10 */
    int32_t learning;          /* ASP_LEARN_FWD (default) or ASP_LEARN_RES */
    int32_t learn_conflicts;   /* round conflicts learned per Learning step,
                                  1..8 (0 means 1): the shortest, then
                                  lowest-id, distinct conflicts of a round are
                                  each learned on the same assignment, the
                                  backjump goes to the lowest of their levels
                                  and the first nogood reaching it asserts
                                  (Sect. 4.2: the solver may select one or
                                  more conflicts and takes the lowest target
                                  level) */
    int64_t max_models;        /* answer sets asked for (the paper restarts the
                                  solver when more than one solution is
                                  requested, Sect. 3): 1 (default) is the
                                  plain search; k > 1 finds up to k; 0 finds
                                  all.  After an answer set M the search
                                  learns {T p : p in M} (answer sets are
                                  incomparable under inclusion, so this
                                  excludes M alone) and restarts: everything
                                  is unassigned, learned nogoods stay, and
                                  InitialPropagation also takes the learned
                                  unit nogoods.  The first max(1, max_models)
                                  answer sets are kept (n_atoms bytes each) */
    int64_t restart_every;     /* > 0: a conflict that makes this many
                                  conflicts since the last restart learns its
                                  nogood and restarts instead of backjumping
                                  (the paper's restart option, Sect. 3);
                                  0 (default) never */
    int32_t lookahead;         /* Fwd-learning only: 2..8 turns on the
                                  lookahead Decision (parallel lookahead, a
                                  refinement the Conclusions name): the
                                  `lookahead` best applicable rules are each
                                  tried -- decided and propagated to a
                                  fixpoint or a conflict; a trial ending in a
                                  conflict or a total assignment stands as
                                  the Decision, the others are undone and
                                  the one that assigned the most variables
                                  (the best-scored on ties) is decided.
                                  Trial rounds count as rounds; an undone
                                  trial enters the trace hash as (10, rule,
                                  count).  0 or 1 (default): off */
    int32_t reserved;          /* 0 */
} asp_options;

/* Run limits. */
typedef struct {
    int64_t max_conflicts;     /* <0 = unlimited; reaching it -> ASP_UNKNOWN */
    int64_t max_ms;            /* device wall-clock guard per launch; <=0 takes
                                  the default of 600000 ms (every launch is
                                  bounded); firing gives ASP_E_TIMEOUT for the
                                  instances still open */
} asp_limits;

/* Launch schedule (no effect on results). */
typedef struct {
    int32_t threads;           /* threads per workgroup: 64, 128, 256, 512 or 1024 */
    int32_t classes;           /* batches: LDS size classes by variable count,
                                  1..4; each class is one launch on its own
                                  stream, with LDS sized for its largest
                                  instance (more classes: more resident
                                  workgroups) */
    int32_t class_threads[4];  /* batches: threads per workgroup of class c
                                  (c = 0 holds the largest instances); 0 takes
                                  `threads` */
} asp_schedule;

/* Search counters (the paper's Fig. 1/2 metrics plus literal checks).
 * literal_checks = sum over every (propagated literal L, nogood containing L)
 * visit of the nogood's length. */
typedef struct {
    int64_t rounds, visits, literal_checks, propagations, decisions, conflicts,
            learned, learned_len, gate_failures, completes;
    uint64_t trace_hash;       /* FNV-1a 64 over the decision/learning events */
    int32_t status;            /* final status of the instance */
    int32_t last_step;         /* ASP_STEP_* of the last step run */
    int64_t ns_total;          /* device time of the solve (solve calls only) */
    int64_t ns_round, ns_learn, ns_decide, ns_gate;  /* split by step kind;
                                  ns_decide includes CompleteAssignment */
    int64_t models;            /* answer sets found */
    int64_t restarts;          /* restarts (after answer sets and by
                                  restart_every) */
    int32_t exhausted;         /* 1: the search showed no further answer set
                                  exists (the status is then ASP_SAT if one
                                  was found) */
    int32_t reserved;
} asp_stats;

typedef struct {
    int32_t n_atoms;
    int32_t n_rules_headed;
    int32_t n_constraints;     /* constraints kept (tautologies dropped) */
    int32_t n_vars;            /* n_atoms + 3 * n_rules_headed */
    int64_t n_nogoods;         /* |Delta_0| */
    int64_t n_lits;            /* literals over all nogoods of Delta_0 */
    int64_t n_units;           /* nogoods of length 1 */
    uint64_t device_bytes;     /* arena bytes asp_bind_device needs */
} asp_sizes;

/* Result of asp_propagate. */
typedef struct {
    int32_t status;            /* ASP_FIXPOINT or ASP_CONFLICT */
    int32_t conflict_id;       /* selected conflict nogood (shortest, then
                                  lowest id), -1 if none */
    int64_t rounds;            /* rounds run by this call */
    int64_t implied;           /* variables assigned by this call */
    int64_t visits;            /* (literal, nogood) visits by this call */
    int64_t literal_checks;    /* literal checks by this call */
} asp_prop_result;

/* Full solver state of a bound single program (test and checkpoint use). */
typedef struct {
    int32_t n_vars, W, cdl, frontier_len;
    int32_t n_learned, pending;   /* pending: nogood id of a round conflict
                                     awaiting asp_analyze_conflict, else -1 */
    int64_t learned_lits;
    int32_t initialised;          /* InitialPropagation has run */
    int32_t status;               /* ASP_RUNNING while the search is open */
    int32_t score_mode;           /* 1 while per-atom scores drive Decision */
    int32_t consec;               /* current run of conflicts (fallback count) */
    int32_t dec_open;             /* a decision was taken since the last conflict */
    int32_t reserved;
    int8_t *val;                  /* [n_vars+1] -1 / 0 / +1 */
    int32_t *lvl;                 /* [n_vars+1] decision level, 0 unassigned */
    uint64_t *deps;               /* [(n_vars+1)*W] Deps bitmaps */
    int32_t *dec;                 /* [cdl+1] decision literal of level l >= 2 */
    int32_t *frontier;            /* [frontier_len] variables assigned by the
                                     last step, ascending on export */
    int32_t *learned_off;         /* [n_learned+1] */
    int32_t *learned;             /* [learned_lits] */
    asp_stats stats;
} asp_state;

/* --------------------------------------------------------- programs */

/* Validate a ground program and compute its completion nogoods (Sect. 2).
 *  head[r]    : head atom of rule r in 1..n_atoms, or 0 for a constraint
 *  body_off   : n_rules+1 offsets, non-decreasing, body_off[0] = 0
 *  body_lits  : +a (atom a) or -a (not a), 1 <= a <= n_atoms
 *  opt        : NULL = {W=1, gate=UNFOUNDED, learned_cap_ng=1<<20,
 *               learned_cap_lits=1<<22, decision=OCC, fallback_after=10,
 *               learning=FWD, learn_conflicts=1, max_models=1,
 *               restart_every=0, lookahead=0}
 * Repeated body literals are removed (first kept); a constraint holding both
 * a and not a is dropped.  Nogoods are generated per headed rule, then per
 * atom, then per constraint, and stably sorted by length (Sect. 4); their
 * position is their id.  On success *out owns a host-side handle (free it
 * with asp_free_program) and *sizes (optional) is filled.
 * Errors: ASP_E_INVALID before anything is allocated. */
int32_t asp_load_program(int32_t n_atoms, int32_t n_rules, const int32_t *head,
                         const int64_t *body_off, const int32_t *body_lits,
                         const asp_options *opt, asp_program **out,
                         asp_sizes *sizes);

int32_t asp_free_program(asp_program *prog);

/* Copy Delta_0 as CSR: off[n_nogoods+1], lits[n_lits] (host arrays). */
int32_t asp_program_nogoods(const asp_program *prog, int32_t *off, int32_t *lits);

/* Bind a device arena of at least sizes.device_bytes bytes (256-byte
 * aligned) to the program, upload Delta_0, the literal-to-nogood map and the
 * rule tables on `stream`, and reset the search state (nothing assigned).
 * sched: NULL = 256 threads.  The arena must stay alive until the program is
 * freed or bound again.  Errors: ASP_E_CAPACITY if bytes is too small,
 * ASP_E_DEVICE on a HIP error. */
int32_t asp_bind_device(asp_program *prog, void *dev_arena, uint64_t bytes,
                        void *stream, const asp_schedule *sched);

/* Run PropagateAndCheck rounds (Sect. 4.1) from the current state until a
 * fixpoint, a conflict, or max_rounds rounds (max_rounds <= 0: no cap).
 * Runs InitialPropagation first if it has not run.  Synchronous.
 * Returns ASP_FIXPOINT, ASP_CONFLICT, ASP_RUNNING (round cap hit), ASP_UNSAT
 * (clashing unit nogoods), or an error; *out (optional) gets the details. */
int32_t asp_propagate(asp_program *prog, void *stream, int32_t max_rounds,
                      asp_prop_result *out);

/* Fwd-learning (Sect. 4.2) of the pending round conflict, then Backjump and
 * assertion.  learned_lits (optional, cap entries) receives the learned
 * nogood, *learned_len its length, *backjump_level the new level.
 * Returns ASP_OK, ASP_UNSAT (the conflict depends on no decision),
 * ASP_UNKNOWN (conflict budget or learned-store capacity), ASP_E_STATE (no
 * pending conflict), ASP_E_CAPACITY (cap too small; the state is still
 * updated).  Synchronous. */
int32_t asp_analyze_conflict(asp_program *prog, void *stream,
                             const asp_limits *lim, int32_t *learned_lits,
                             int32_t cap, int32_t *learned_len,
                             int32_t *backjump_level);

/* Set the decision scores of a bound program: scores[p] for atom p =
 * 1..n_atoms (scores[0] ignored), any int32 values, copied from the host on
 * `stream`; the score of each rule's head is then gathered on the device.
 * Programs loaded with ASP_DECISION_SCORE must have scores set (here or by
 * asp_score_program) after every asp_bind_device and before searching, or
 * the search calls return ASP_E_STATE.  Synchronous. */
int32_t asp_set_scores(asp_program *prog, const int32_t *scores, void *stream);

/* Copy the program's current device scores (n_atoms+1 int32) to the host. */
int32_t asp_get_scores(asp_program *prog, int32_t *scores, void *stream);

/* Run the next n_steps search steps of any kind (n_steps < 0: to the end).
 * Returns the search status (ASP_RUNNING if still open); *stats optional. */
int32_t asp_run_steps(asp_program *prog, void *stream, const asp_limits *lim,
                      int64_t n_steps, asp_stats *stats);

/* Solve from scratch (to the first answer set, or to max_models of them).
 * model (optional, n_atoms bytes, host) gets 1 for the true atoms of the
 * first answer set when the result is ASP_SAT.  A search that ends UNSAT or
 * UNKNOWN after finding answer sets reports ASP_SAT (stats.exhausted tells
 * whether no further one exists).  Returns ASP_SAT, ASP_UNSAT, ASP_UNKNOWN
 * or an error.  Synchronous. */
int32_t asp_solve(asp_program *prog, void *stream, const asp_limits *lim,
                  uint8_t *model, asp_stats *stats);

/* Allocation-free form of asp_solve, for callers that cannot allocate
 * device memory or bind an arena (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  The program's tables,
 * its search state and the results live in a library-owned device array of
 * ASP_NOALLOC_MAX_BYTES bytes, one per GPU, held from the first use until
 * the process ends; the call uploads the program into it, solves on the
 * current device with 256 threads, and copies the verdict, model (optional,
 * n_atoms bytes, host) and stats (optional) back, like asp_solve.  It calls
 * no device allocation or free.  Every call on one GPU uses that GPU's
 * array, which keeps the last call's contents (nothing of it is read before
 * the call writes it): calls that overlap on one GPU, from any stream or
 * thread, race and must be serialised by the caller.  The program need not
 * be bound, and a bound arena is left untouched.  Errors: ASP_E_CAPACITY
 * when the program needs more than ASP_NOALLOC_MAX_BYTES (the learned-store
 * capacities dominate: load with smaller learned_cap_lits / learned_cap_ng),
 * ASP_E_INVALID for ASP_DECISION_SCORE programs (their scores need a bound
 * arena), ASP_E_DEVICE on a HIP error.  Synchronous. */
#define ASP_NOALLOC_MAX_BYTES (64u << 20)
int32_t asp_solve_noalloc(const asp_program *prog, void *stream, const asp_limits *lim,
                          uint8_t *model, asp_stats *stats);

/* The answer sets found by the last search of a bound program, in the order
 * found: models (host, max_out * n_atoms bytes) gets the first
 * min(found, max(1, max_models), max_out), answer set k at k * n_atoms;
 * *found (optional) the number found.  Errors: ASP_E_STATE if unbound,
 * ASP_E_INVALID for max_out < 0 or a NULL buffer with max_out > 0.
 * Synchronous. */
int32_t asp_get_models(asp_program *prog, void *stream, uint8_t *models, int64_t max_out,
                       int64_t *found);

/* State export: with st->val == NULL only the scalars are filled (to size
 * the arrays); otherwise every non-NULL array is filled as well. */
int32_t asp_state_export(asp_program *prog, void *stream, asp_state *st);

/* State import (the frontier must hold variables of level cdl; the pending
 * field may name a round conflict; learned nogoods must hold decision
 * literals T b_r only).  Fwd-learning programs with max_models = 1, no
 * restarts and one conflict learned per step only.  Errors: ASP_E_INVALID
 * on inconsistent input, ASP_E_CAPACITY beyond the learned-store capacity. */
int32_t asp_state_import(asp_program *prog, void *stream, const asp_state *st);

/* ------------------------------------------------------------ batches */

/* Plan the batched solve of n programs (all loaded with the same options):
 * one workgroup per instance, instances grouped by LDS size class, largest
 * first inside a class, and one search-state slot per instance.  The
 * programs must stay alive until asp_batch_bind returns.
 * sched: NULL = {128 threads, 4 classes}.  *device_bytes gets the arena
 * size; *model_bytes (optional) the size of the model output, which holds
 * instance i's max(1, max_models) answer sets of n_atoms bytes each after
 * those of instances 0..i-1. */
int32_t asp_batch_create(int32_t n, asp_program *const *progs,
                         const asp_schedule *sched, asp_batch **out,
                         uint64_t *device_bytes, uint64_t *model_bytes);

/* Upload every program's static data into the arena (on stream). */
int32_t asp_batch_bind(asp_batch *batch, void *dev_arena, uint64_t bytes,
                       void *stream);

/* Enqueue the batched solve on stream (asynchronous): one launch per LDS
 * class, each forked onto one of four streams the batch creates together
 * at its first multi-class solve (so that each takes its own hardware
 * queue and the classes run at once), after the work already on `stream`,
 * and joined back into it; a single class launches on `stream` itself.
 * Each workgroup solves one instance to a verdict.  Results stay in the
 * arena. */
int32_t asp_solve_batch(asp_batch *batch, void *stream, const asp_limits *lim);

/* The same batched solve as one HIP graph launch: the first call (and any
 * call with other limits or another stream) captures the fork/join of the
 * class launches into a graph; every call replays it with hipGraphLaunch on
 * `stream` (a non-default stream).  Each launch resets the instances' search
 * state itself, so replays need no clearing; asp_batch_last_ms times the
 * replay, asp_batch_launch_info reports no per-class times for it. */
int32_t asp_solve_batch_graph(asp_batch *batch, void *stream, const asp_limits *lim);

/* Copy verdicts[n] (ASP_SAT/UNSAT/UNKNOWN or a negative error),
 * models[model_bytes] and stats[n] back (any may be NULL); synchronous. */
int32_t asp_batch_results(asp_batch *batch, void *stream, int32_t *verdicts,
                          uint8_t *models, asp_stats *stats);

/* Device time of the last asp_solve_batch, in milliseconds, between HIP
 * events recorded on the caller's stream around the forked launches. */
int32_t asp_batch_last_ms(asp_batch *batch, double *ms);

/* The launches of the batch: *n_classes launches; launch c solves instances
 * order[first[c] .. first[c]+count[c]) with threads[c] threads per
 * workgroup, and took ms[c] milliseconds in the last asp_solve_batch (HIP
 * events on its stream; 0 before any solve and after a graph replay).
 * Arrays of 4 entries (order:
 * n entries); any pointer may be NULL. */
int32_t asp_batch_launch_info(asp_batch *batch, int32_t *n_classes, int32_t *first,
                              int32_t *count, int32_t *threads, double *ms, int32_t *order);

int32_t asp_batch_free(asp_batch *batch);

/* Scores of a batch instance i (see asp_set_scores / asp_get_scores). */
int32_t asp_batch_set_scores(asp_batch *batch, int32_t i, const int32_t *scores,
                             void *stream);
int32_t asp_batch_get_scores(asp_batch *batch, int32_t i, int32_t *scores,
                             void *stream);

/* ------------------------------------------------- learned Decision scorer
 * A message-passing network over the bipartite graph of variables and the
 * static nogoods Delta_0 (edges: the nogood literals, with their sign) gives
 * each atom an integer score for the score-driven Decision.  It is
 * quantisation-aware: matrices hold integer codes in [-127, 127] stored as
 * bfloat16 and activations are integer codes in [0, 255], so every 64-term
 * product on the matrix cores (bfloat16 operands, float32 accumulation) is
 * an exact integer below 2^21 and the scores do not depend on the order of
 * any sum.  With act(z) = 0 for z <= 0, else min(255, (z + 256) >> 9), and
 * norm(s, n) = s >> k rounded half up, k = ceil(log2 n) (k = 0 for n <= 1):
 *   embed   hv = act(x Ev + ev),  hc = act(y Ec + ec)
 *   layer l hc = act(hc S_l + norm(sum_{Tv in c} hv P_l + sum_{Fv in c} hv N_l, |c|) + bc_l)
 *           hv = act(hv T_l + norm(sum_{c with Tv} hc Q_l + sum_{c with Fv} hc R_l, deg v) + bv_l)
 *   score   s_v = hv wo + bo    (atoms v = 1..n_atoms)
 * Features, 32 standing for 1, r(a, b) = (a + b/2) / b in integers (0 for
 * b = 0) and L(d) = min(255, 16 * bit length of d) a saturating log code:
 *   x_v = [32, 32*atom, 32*is_b, 32*is_t, 32*is_n, L(#c with Tv),
 *          L(#c with Fv), L(#c with Tv or Fv)]
 *   y_c = [32, r(32, |c|), 32*(|c|=1), 32*(|c|=2), 32*(|c|=3), 32*(|c|>=4),
 *          r(32 * #positive literals, |c|), 0]
 * Matrices are [in][out], row-major, bfloat16 bit patterns. */
#define ASP_SCORER_F 8
#define ASP_SCORER_H 64
#define ASP_SCORER_L 3

typedef struct {
    uint16_t Ev[ASP_SCORER_F * ASP_SCORER_H], Ec[ASP_SCORER_F * ASP_SCORER_H];
    uint16_t P[ASP_SCORER_L * ASP_SCORER_H * ASP_SCORER_H];
    uint16_t N[ASP_SCORER_L * ASP_SCORER_H * ASP_SCORER_H];
    uint16_t S[ASP_SCORER_L * ASP_SCORER_H * ASP_SCORER_H];
    uint16_t Q[ASP_SCORER_L * ASP_SCORER_H * ASP_SCORER_H];
    uint16_t R[ASP_SCORER_L * ASP_SCORER_H * ASP_SCORER_H];
    uint16_t T[ASP_SCORER_L * ASP_SCORER_H * ASP_SCORER_H];
    int32_t ev[ASP_SCORER_H], ec[ASP_SCORER_H];
    int32_t bc[ASP_SCORER_L * ASP_SCORER_H], bv[ASP_SCORER_L * ASP_SCORER_H];
    int32_t wo[ASP_SCORER_H];   /* in [-127, 127] */
    int32_t bo;
    int32_t reserved[63];
} asp_scorer_weights;

/* Device workspace (bytes) the scorer needs for the bound program / batch. */
int32_t asp_scorer_workspace(const asp_program *prog, uint64_t *bytes);
int32_t asp_batch_scorer_workspace(const asp_batch *batch, uint64_t *bytes);

/* Score every atom with the network (weights: host copy, validated: matrix
 * entries must be integers in [-127, 127], biases within +-2^24) into the
 * device scores used by ASP_DECISION_SCORE.  ws: device memory of at least
 * the workspace size, 256-byte aligned.  asp_score_program is synchronous;
 * asp_score_batch enqueues on `stream` (all instances in one set of
 * launches).  Errors: ASP_E_INVALID (weights), ASP_E_CAPACITY (workspace). */
int32_t asp_score_program(asp_program *prog, const asp_scorer_weights *w, void *ws,
                          uint64_t ws_bytes, void *stream);
int32_t asp_score_batch(asp_batch *batch, const asp_scorer_weights *w, void *ws,
                        uint64_t ws_bytes, void *stream);

/* Train the scorer's readout on the device (the learned Decision's
 * training): with the matrices of w fixed, the scorer runs once over the
 * batch, then `steps` full-batch Adam steps (learning rate lr) minimise the
 * mean binary cross-entropy of sigmoid(sum_j (hv_j / 256) wb[j] + wb[64])
 * against labels, where hv is an atom's code vector after the last layer.
 * labels: host int8, laid out like the models output (n_atoms per instance,
 * in batch order): 1 = true in the answer set found by the plain search,
 * 0 = false, -1 = no label.  wb_out[65] (host) holds the starting weights on
 * entry and the trained ones on return; loss_out[steps] (optional) the mean
 * loss before each step.  steps in 1..4096.  Synchronous. */
int32_t asp_batch_train_readout(asp_batch *batch, const asp_scorer_weights *w, void *ws,
                                uint64_t ws_bytes, const int8_t *labels, int32_t steps,
                                float lr, float *wb_out, float *loss_out, void *stream);

/* ------------------------------------------- learned Decision training
 * The scorer above is trained in its float form: activation a = code / 256
 * in [0, 1], matrix and readout entries w = code / 128 in [-127/128,
 * 127/128], layer and embedding biases b = code / 2^17, readout bias
 * bo = code / 2^15, so that each layer is
 *   a' = clamp(u / 4 + b, 0, 1),  u = (self term) + (edge sum) / 2^k
 * -- the integer layer divided by 256, up to its roundings -- and the
 * readout logit is a . wo + bo.  The float parameters are one vector of
 * ASP_SCORER_NPARAM floats, in this order: Ev[8][64], Ec[8][64], ev[64],
 * ec[64], P[3][64][64], N, S, Q, R, T (same shape), bc[3][64], bv[3][64],
 * wo[64], bo.  Training minimises the mean binary cross-entropy of
 * sigmoid(logit) against per-atom labels in [0, 1] over every layer, on the
 * device: forward and backward passes with bfloat16 operands and float32
 * accumulation on the matrix cores, full-batch Adam (beta 0.9 / 0.999,
 * eps 1e-8), and after every step each parameter is clipped to the range its
 * integer code can hold. */
#define ASP_SCORER_NPARAM 75329

/* Device workspace (bytes) for training on these programs: the graph (one
 * row per variable and per static nogood, the literals as edges in both
 * orders), features, labels, parameters and Adam state, and the
 * activations of every layer (about 2.3 KB per row). */
int32_t asp_scorer_train_workspace(int32_t n, asp_program *const *progs, uint64_t *bytes);

/* Train on programs progs[0..n) with labels (host float, n_atoms per
 * program in order; < 0 = no label).  params (host, ASP_SCORER_NPARAM):
 * starting values in, trained values out.  steps = 0 runs one forward and
 * backward pass only: loss_out[0] gets the loss and grad_out (optional,
 * ASP_SCORER_NPARAM) the gradient, params unchanged.  steps > 0 runs that
 * many Adam steps at learning rate lr: loss_out[t] (optional, steps floats)
 * gets the loss before step t, grad_out (optional) the last gradient.
 * ws: device memory of the workspace size, 256-byte aligned.  Errors:
 * ASP_E_INVALID (no labelled atom, bad arguments), ASP_E_CAPACITY
 * (workspace).  Synchronous. */
int32_t asp_scorer_train(int32_t n, asp_program *const *progs, const float *labels,
                         float *params, int32_t steps, float lr, void *ws, uint64_t ws_bytes,
                         float *loss_out, float *grad_out, void *stream);

/* Float parameters <-> integer weight codes (host only): codes are the
 * parameters times their scale, rounded to nearest and clipped to the code
 * ranges of asp_scorer_weights. */
int32_t asp_scorer_quantize(const float *params, asp_scorer_weights *w);
int32_t asp_scorer_dequantize(const asp_scorer_weights *w, float *params);

/* The nogoods learned by instance i of the last batched solve (decision
 * literals T b_r under Fwd-learning; any literals under Res-learning;
 * answer-set blocking nogoods included), as CSR: *n_learned and *n_lits get
 * the sizes; off (n_learned+1 entries) and lits (n_lits entries) are
 * filled when not NULL and cap_ng / cap_lits hold them.  The conflict traces
 * the learned Decision is trained on.  Synchronous. */
int32_t asp_batch_learned(asp_batch *batch, int32_t i, int32_t *off, int64_t cap_ng,
                          int32_t *lits, int64_t cap_lits, int32_t *n_learned,
                          int64_t *n_lits, void *stream);

/* ------------------------------------------------------------- misc */
const char *asp_status_str(int32_t status);
/* Copy the calling thread's last error message into buf (NUL-terminated). */
int32_t asp_last_error(char *buf, uint64_t len);

#ifdef __cplusplus
}
#endif
#endif /* ASP_H */
