/*
 * mctune.h -- C ABI of the MI355X explicit-state auto-tuning checker.
 *
 * The method (Garanina, Staroletov, Gorlatch, "Auto-Tuning High-Performance Programs
 * Using Model Checking in Promela"): a timed model of an OpenCL kernel on an abstract
 * platform picks its tuning parameters nondeterministically (Sec. 4, Step 1, the
 * `main` process of Listing 3); the over-time property G(FIN -> time > T) (Sec. 4,
 * Step 2) fails exactly when some run terminates with time <= T; the least such T
 * (Sec. 2, Fig. 1 and Step 3) and the parameter values on a counterexample path
 * (Step 4) are the tuning result.  This library answers those queries by exhaustive
 * explicit-state exploration on the GPU.
 *
 * Model (one descriptor = one kernel, one platform, a list of configurations):
 *   state       (cfg, clock, pending, rem[0..m-1]); rem_i = cycles left in the
 *               workgroup on compute unit i, 0 = idle; a distinguished root.
 *   SELECT(c)   root -> (c, 0, n_c, 0,..,0) for every configuration c.
 *   DISPATCH(i) pending > 0 and rem_i = 0: rem_i := d_c, pending -= 1; no time passes
 *               (host/device/unit hand-off of Listings 4-6).  One successor per free
 *               unit.
 *   ADVANCE     only when no DISPATCH is enabled and a unit is busy: the clock moves
 *               to the next operation end of any busy unit (the clock process of
 *               Listing 9 ticks when every active PE has reported its unit of work,
 *               Listing 8).
 *   terminal    pending = 0 and all units idle (FIN, Listing 4); its clock is the
 *               model time of the run.
 *   Operation lists per workgroup (global loads at Lg, local steps at Ll, barriers
 *   at Lb -- free by default, as the barrier process of Listing 7 never advances
 *   time -- compute at Lc):
 *     MC_KIND_REDUCTION (WG, TS):        n = G/WG; ceil(G/(WG*TS)) x Lg,
 *                                        log2(WG) x Ll, 1 x Lb, TS x Lc.
 *     MC_KIND_MATMUL (WGx, WGy, TS, VW): n = (M/WGx)(N/(WGy*VW)); 2K x Lg,
 *                                        K(1+VW) x Ll, 2K/TS x Lb, K*VW x Lc.
 *   Two kinds follow the paper's own Promela models of a unit with NP processing
 *   elements (size = {S, NP, 0}; GMT = Lg, the local step = Ll, the paper's 1; Lc and
 *   Lb unused).  A workgroup of WG > NP work items runs in WG/NP waves of NP elements
 *   (the unit relaunches finished elements, Listings 6 and 14); n = S/(WG*TS)
 *   workgroups, at least one (Table 1 times one workgroup where WG*TS > S):
 *     MC_KIND_ABSTRACT (WG, TS):  every wave is one run of the abstract pex of Sec. 4
 *       (Listing 8) over s = S/TS tiles.  Its long_work(gt, tz) returns on the first
 *       tick at which time exceeds start_time + gt*tz, and start_time is set at the
 *       start, before each local step and before the final write, so the operations
 *       last Lg*TS+1 (first tile's global load), then per tile Ll*TS+1 (local step)
 *       and, from the second tile on, max(0, (Lg-Ll)*TS) (global load), and finally
 *       Lg+1 (result write); a wave lasts S*Lg + S/TS + TS + Lg + 2 for Ll = 1 <= Lg.
 *     MC_KIND_MINIMUM (WG, TS):   the Minimum kernel of Sec. 7 (Listings 10 and 15):
 *       WG/NP waves x TS global accesses at Lg (MAP), then min(WG, NP) - 1 local
 *       steps at Ll and one global write at Lg by element 0 (REDUCE local), per
 *       workgroup as in the kernel.
 *   d_c is the workgroup duration; E_c the distinct cumulative operation end times.
 *
 * Units of unequal speed (the assumption of Sec. 4 that every unit works alike,
 * dropped): unit i takes s_i cycles per cycle of work, so a workgroup on it ends its
 * operations at s_i*E_c and lasts s_i*d_c; DISPATCH(i) sets rem_i := s_i*d_c and ADVANCE
 * moves to the next end on any unit's own grid.  Which free units take the last
 * workgroups now changes the makespan.  Dispatch stays eager, so while at least as many
 * workgroups are pending as units are idle the run is determined; the first instant with
 * fewer splits it into one tail per choice of units.  There is no closed-form count:
 * sizes come from walking that determined part and every tail (a tail's states are
 * counted even where tails meet, so the count is an upper bound, exact on the
 * determined part).  Round blocks are not cut for such models, and the graph is no
 * longer graded (tails meet at different depths): `levels` of the super-step engine is
 * then the depth of each state's first claim, not its BFS depth.
 *
 * Conventions.  Every call returns an int: MC_OK (0) or a negative MC_E_* code; no
 * call aborts and no C++ exception crosses the ABI.  Device pointers are plain
 * hipMalloc'd (or torch-allocated) device addresses; host pointers are ordinary host
 * memory.  A model handle is not thread-safe; separate handles on separate streams
 * may run concurrently.  Query calls are synchronous with respect to the host: they
 * enqueue on the handle's stream and wait for it.
 */
#ifndef MCTUNE_H
#define MCTUNE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes --------------------------------------------------------------- */
#define MC_OK 0
#define MC_E_INVAL (-1)      /* invalid descriptor, option or argument */
#define MC_E_NOMEM (-2)      /* workspace smaller than mc_workspace_bytes() */
#define MC_E_DEVICE (-3)     /* a HIP runtime call failed */
#define MC_E_TABLE_FULL (-4) /* visited-set capacity exceeded (reload with more slots) */
#define MC_E_BUFFER (-5)     /* output buffer too small; the needed size is returned */
#define MC_E_STATE (-6)      /* no query has produced what was asked for */
#define MC_E_OVERFLOW (-7)   /* a frontier or a packed field exceeded its bound */
#define MC_E_ADMIT (-8)      /* a query can never fit the engine's memory budget */
#define MC_E_NOTFOUND (-9)   /* no such ticket / state */
#define MC_E_INTERNAL (-10)  /* an internal consistency check failed (a round block of a
                                configuration did not end on its predicted state) */
#define MC_E_ABORTED (-11)   /* the query was stopped by mc_abort / mc_batch_abort before
                                it finished; it has no result */

/* ---- model descriptor ---------------------------------------------------------- */
#define MC_KIND_REDUCTION 0u
#define MC_KIND_MATMUL 1u
#define MC_KIND_ABSTRACT 2u  /* abstract kernel with NP elements per unit (Sec. 4) */
#define MC_KIND_MINIMUM 3u   /* Minimum problem model (Sec. 7.2) */

#define MC_MAX_CU 8u         /* compute units per model */

typedef struct mc_desc {
    uint32_t kind;           /* MC_KIND_* */
    uint32_t n_cu;           /* m, 1..MC_MAX_CU */
    uint32_t size[3];        /* reduction: {G, 0, 0}; matmul: {M, N, K};
                                abstract and minimum: {S, NP, 0} */
    uint32_t lat_global;     /* Lg >= 1 */
    uint32_t lat_local;      /* Ll >= 1 */
    uint32_t lat_compute;    /* Lc >= 1 */
    uint32_t lat_barrier;    /* Lb >= 0 */
    uint32_t n_cfg;          /* number of configurations, >= 1 */
    const uint32_t *params;  /* host pointer, n_cfg rows of 4: reduction, abstract and
                                minimum (WG, TS, 0, 0), matmul (WGx, WGy, TS, VW); VW = 0
                                means 1.  Powers of two; sizes must divide as the
                                operation lists require. */
    const uint32_t *unit_speed; /* host pointer, n_cu entries in 1..MC_MAX_SPEED, or NULL
                                (all 1): unit i runs every operation unit_speed[i] times
                                as long (see "Units of unequal speed" above) */
} mc_desc;

#define MC_MAX_SPEED 64u

/* ---- options ------------------------------------------------------------------- */
#define MC_ENGINE_SUPERSTEP 0u /* persistent kernel, one configuration's subgraph per
                                  workgroup, zero-time closures and lock-step runs
                                  expanded in one super-step */
#define MC_ENGINE_LEVEL 1u     /* plain level-synchronous BFS, one launch per level */

typedef struct mc_opts {
    uint32_t engine;         /* MC_ENGINE_* */
    uint32_t block;          /* threads per workgroup: 256, 512 or 1024 (0 = automatic:
                                512 when the query has fewer than 256 partitions, whose
                                critical chains of inserts then decide the launch time,
                                or when the units have unequal speeds; else 256) */
    uint32_t log2_slots;     /* visited-set capacity 2^log2_slots (0 = from load_factor) */
    float load_factor;       /* target states/slots when sizing (0 = automatic: at most
                                0.375 after rounding the slots up to a power of two, or
                                0.5 where that passes 2^31 slots) */
    uint32_t grid;           /* persistent workgroups (0 = automatic) */
    uint32_t batch_items;    /* super-step engine: states generated from one frontier state
                                before waiting for the visited set (0 = 2 x lanes) */
    uint32_t lane_items;     /* keys each thread inserts per round trip: 1 or 2
                                (else automatic: 2 for keys of up to 128 bits,
                                1 for wider keys) */
    uint32_t part_states;    /* super-step engine: target states per partition when a
                                configuration's subgraph is cut into blocks of whole
                                rounds and its long lock-step runs into run slices (a
                                round's states j0..j1-1 of every run; 1024..8192 states per
                                slice) (0 = automatic, UINT32_MAX = never cut) */
    uint32_t test_hash_bits; /* testing only: 0 = the full key hash; k in 1..24 keeps k
                                bits of it, so that keys crowd into 2^k probe sequences
                                (long probe chains, and keys of several words that share
                                word 0 meeting in one slot); results are unchanged */
} mc_opts;

/* ---- statistics of the last query ---------------------------------------------- */
typedef struct mc_stats {
    uint64_t states;         /* unique states (root included); count_T for mc_check */
    uint64_t levels;         /* BFS levels = deepest state's depth + 1 */
    uint64_t terminals;      /* unique terminal states */
    uint64_t edges;          /* successor generations performed (engine-specific) */
    uint64_t dups;           /* inserts that found the state present (engine-specific) */
    uint64_t probes;         /* hash-slot probes (engine-specific) */
    uint64_t launches;       /* kernel launches of the exploration */
    uint64_t explore_ns;     /* GPU time of the exploration kernels (HIP events) */
    uint64_t total_ns;       /* host wall time of the query call */
    uint64_t clear_ns;       /* GPU time clearing the visited set */
    uint64_t engine_ns;      /* GPU time of the exploration engine's own launch(es),
                                without the seed and result copies (HIP events) */
    uint64_t supersteps;     /* super-steps of the persistent engine */
    uint64_t batches;        /* insert batches of the persistent engine */
    uint64_t max_probe;      /* longest probe sequence of one insert */
    uint64_t critical_ns;    /* longest single-partition exploration (device clock) */
    uint64_t critical_cfg;   /* the configuration of that partition */
    uint64_t parts;          /* partitions of the persistent launch (configurations, or
                                blocks of whole rounds of them) */
    uint64_t cas_fail;       /* probes whose compare-and-swap met a slot holding another
                                state: every insert ends on one deciding probe (its claim,
                                or its own key found), so this is probes - new states -
                                dups of the query's exploration (0 if it explored nothing) */
} mc_stats;

typedef struct mc_model_info {
    uint32_t n_cu, n_cfg;
    uint32_t key_words;      /* packed key width in 64-bit words: 1, 2 or 4 */
    uint32_t key_bits;       /* bits actually used */
    uint64_t slots;          /* visited-set capacity */
    uint64_t slot_bytes;     /* bytes per visited-set slot */
    uint64_t bound_states;   /* reachable-state count the workspace was sized for */
    uint64_t max_depth;      /* longest path length (sizes the trace buffer) */
} mc_model_info;

typedef struct mc_model mc_model;

/* Bytes of device workspace a model needs (visited set, frontiers, tables, counters).
 * The visited set is sized from the exact reachable-state count of the lock-step
 * round structure and the load factor.  Pure host computation.
 * MC_E_INVAL: invalid descriptor (sizes not powers of two or not divisible, empty
 * domain, latencies out of range, packed state wider than 256 bits, clock above 2^32). */
int mc_workspace_bytes(const mc_desc *d, const mc_opts *o, size_t *bytes);

/* Reachable-state count of the model (root included), its longest path, and the packed
 * key width, without touching the GPU. */
int mc_describe(const mc_desc *d, uint64_t *states, uint64_t *max_depth, uint32_t *key_words);

/* The operation end times E_c of configuration `cfg` (the per-workgroup operation lists
 * of the model description above), without touching the GPU: *n = workgroups, *b =
 * |E_c|, *dur = d_c, ends[0..b-1] = E_c ascending (host memory, may be NULL when cap is
 * 0).  MC_E_BUFFER with *n, *b and *dur set if cap < b; MC_E_INVAL for a bad
 * descriptor or cfg >= n_cfg. */
int mc_config_ends(const mc_desc *d, uint32_t cfg, uint32_t *n, uint32_t *b, uint32_t *dur,
                   uint32_t *ends, uint64_t cap);

/* Load a model: validates, derives per-configuration tables, uploads them into
 * the caller's workspace and binds the stream.  dev_ws: device memory of ws_bytes
 * bytes owned by the caller, kept alive and left alone until mc_model_free.  stream:
 * hipStream_t (NULL = default stream).  The library owns *out.
 * Every call on the handle is ordered on that stream.  Besides it the handle holds a side
 * stream of its own: a query that needs less of the visited set than earlier queries
 * wrote clears the bytes past its own there, once its results are queued (while the host
 * reads them and loads the next query), so that a later larger query finds them cleared;
 * the handle's stream waits for that clear before it next touches the bytes, and
 * mc_model_free waits for it too.
 * MC_E_NOMEM if ws_bytes < mc_workspace_bytes(); MC_E_DEVICE wraps a HIP error. */
int mc_model_load(const mc_desc *d, const mc_opts *o, void *dev_ws, size_t ws_bytes,
                  void *stream, mc_model **out);

/* Replace the handle's model with d (the next tuning query, Sec. 4 step 1), with the
 * options, workspace and stream given at load: validates, derives the tables, uploads
 * them and starts the handle's query state over (no trace, nothing resident).  The bytes
 * of the visited set known to be cleared stay known, so a query after the reload clears only
 * what earlier queries wrote of what it needs.
 * MC_E_INVAL (bad descriptor) and MC_E_NOMEM (the workspace is too small for d): the
 * handle keeps its model.  MC_E_DEVICE wraps a HIP error; the handle can then only be
 * freed. */
int mc_model_reload(mc_model *h, const mc_desc *d);

/* Frees the handle after waiting for its side stream; the workspace is the caller's
 * again. */
int mc_model_free(mc_model *h);
int mc_model_info_get(const mc_model *h, mc_model_info *info);

/* min_time (Sec. 2 steps 3-4 in one pass; the single-run optimum of Sec. 8): explore
 * every reachable state, reduce the terminal clocks per configuration, return
 * T_min and the configurations attaining it in ascending order.  argmin may be NULL
 * with cap 0 to query *n_argmin; MC_E_BUFFER if cap < *n_argmin (the rest is valid).
 * st may be NULL. */
int mc_min_time(mc_model *h, uint32_t *t_min, uint32_t *argmin, size_t cap,
                size_t *n_argmin, mc_stats *st);

/* Branch-and-bound min_time: the single run that replaces the bisection of Sec. 4
 * Step 3 (finding optimal values without repeated verifier runs is the paper's future
 * work, Sec. 8).  The search prunes every state whose clock exceeds the incumbent, the
 * least terminal clock found so far, which starts at T_init (0 = no initial bound, for
 * instance the time of a simulated run, mc_simulate).  Clocks never decrease along a
 * path and the incumbent never falls below T_min, so no state on a path to an optimal
 * terminal is pruned: T_min and the configurations attaining it are exact, as from
 * mc_min_time, and mc_trace gives a counterexample at T_min.  The statistics count the
 * states this search claimed (between the count of clock <= T_min and that of clock
 * <= T_init; the order of the concurrent search decides where), not the reachable
 * set.  mc_terminal_clocks afterwards is exact for the argmin configurations only:
 * others carry a clock found before the incumbent fell below it, or none.
 * MC_E_STATE if no terminal has a clock <= T_init.  With the level engine the bound
 * stays at T_init (a check(T_init) search that also reduces the terminal clocks). */
int mc_min_time_bb(mc_model *h, uint32_t T_init, uint32_t *t_min, uint32_t *argmin, size_t cap,
                   size_t *n_argmin, mc_stats *st);

/* check(T): exhaustive exploration of the states with clock <= T (the clock never
 * decreases along a transition, so pruning at T is exact).  *violated = 1 iff some
 * terminal has clock <= T, i.e. G(FIN -> time > T) fails (Sec. 4, Step 2).
 * st->states = count of states with clock <= T. */
int mc_check(mc_model *h, uint32_t T, int *violated, mc_stats *st);

/* Per-configuration least terminal clock of the last query (UINT32_MAX = none reached
 * under its threshold).  tc: host array of cap >= n_cfg entries. */
int mc_terminal_clocks(const mc_model *h, uint32_t *tc, size_t cap);

/* Counterexample of the last query (Sec. 4, Step 4): the path root -> ... -> terminal
 * of the smallest configuration attaining T_min (after mc_min_time) or of the smallest
 * configuration with a terminal clock <= T (after a violated mc_check).  Rows of
 * (3 + n_cu) uint32 values: cfg (UINT32_MAX for the root), clock, pending,
 * rem_0..rem_{m-1}; root first.  rows may be NULL with cap 0 to query *len.
 * MC_E_STATE if no query ran or the last check held; MC_E_BUFFER if cap < *len. */
int mc_trace(mc_model *h, uint32_t *rows, size_t cap, size_t *len);

/* One seeded random run to termination (simulation mode, Sec. 2 and Step 3): uniform
 * choice among the successors at every step, choices drawn from splitmix64 of
 * (seed, step).  Returns the terminal clock and the configuration selected. */
int mc_simulate(mc_model *h, uint64_t seed, uint32_t *t_end, uint32_t *cfg);

/* The search of Sec. 2 (Fig. 1) and Step 3: T_ini from mc_simulate(seed), then integer
 * bisection keeping check(lo) holding and check(hi) failing, lo = 0.  Returns T_min,
 * the number of check calls, and leaves the trace of the last failing check.  With the
 * super-step engine on units that all work alike the checks share one visited set
 * (sized for T_ini): a check at or below the largest threshold explored so far is
 * answered from the per-configuration least clocks, a check above it continues that
 * exploration instead of starting over (the repeated verifier runs that Sec. 8 names);
 * st->states is then the number of states explored in all, once each.  Otherwise every
 * check is a fresh mc_check and st->states sums their counts. */
int mc_tune_bisect(mc_model *h, uint64_t seed, uint32_t *t_min, uint32_t *n_checks,
                   mc_stats *st);

/* Select the exploration engine used by later queries (MC_ENGINE_*); both engines
 * compute identical results. */
int mc_set_engine(mc_model *h, uint32_t engine);

/* Asks the query running on h (or, when none runs, the next one started) to stop.  It
 * is the one call that may come from another host thread while a query runs on h: it
 * stores to a pinned host word that the exploration kernels read when a workgroup takes
 * its next partition (super-step engine) or a launch starts (level engine).  Partitions
 * already being explored finish, the rest are skipped, and every kernel exits
 * normally; the query then returns MC_E_ABORTED with no result, which consumes the
 * request.  A request made after the exploration kernel has finished stays pending
 * for the next query.  Not a paper operation: it serves callers (servers, test
 * harnesses) that must bound a query's time. */
int mc_abort(mc_model *h);

/* ---- min_time without allocation ------------------------------------------------- */
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): mc_min_time of the descriptor d
 * with its whole workspace in a static device array of MC_STATIC_SCRATCH_BYTES (one
 * array per device, held from the first call on that device until the process ends).
 * The call allocates no device or pinned memory and creates no event or stream: it
 * loads d into the scratch, runs the query on `stream` (a hipStream_t, NULL = null
 * stream), waits for it and returns the results as mc_min_time does (argmin, cap,
 * n_argmin and st likewise; st's timings are host wall-clock only).  MC_E_NOMEM if
 * mc_workspace_bytes(d, o) exceeds MC_STATIC_SCRATCH_BYTES, with nothing run.  Calls
 * on one device share its array: calls that overlap on one device (from several host
 * threads or streams) race and must not be made; successive calls are independent
 * (each clears what it reads). */
#define MC_STATIC_SCRATCH_BYTES (128u << 20)
int mc_min_time_static(const mc_desc *d, const mc_opts *o, void *stream, uint32_t *t_min,
                       uint32_t *argmin, size_t cap, size_t *n_argmin, mc_stats *st);

/* Parameters of configuration cfg (4 values, as in the descriptor). */
int mc_config(const mc_model *h, uint32_t cfg, uint32_t *params4);

const char *mc_strerror(int code);

/* ---- swarm search (Sec. 5) ------------------------------------------------------ */
/* Swarm model checking: many independent, incomplete searches at once, each keeping a
 * bit array of its own (bitstate hashing) instead of storing states and reporting the
 * counterexamples (trails) it meets within a bounded number of model steps.  Against
 * the non-termination property G(!FIN) every run reaching a terminal is a trail whose
 * clock is a model time; against the over-time property with threshold T (prune = 1)
 * only terminals with clock <= T are.  Member i (one GPU lane) uses seed
 * splitmix64(seed + i) and makes random walks from the root: at its step t (counted
 * over all its walks) it takes successor number splitmix64(seed_i ^ splitmix64(t)) mod
 * k of the k successors (configurations in order at the root, free units in index
 * order for DISPATCH); with a threshold a walk ends at the first state with clock > T;
 * at every state it reaches (not the root) with other than exactly one successor it
 * hashes (cfg, clock, pending, rem_0..rem_{m-1}) by a splitmix64 chain to two bit
 * positions h mod 2^bits_log2 and (h >> 32) mod 2^bits_log2: both set, the walk ends;
 * else both are set; a new terminal ends the walk as a trail; a new walk starts only
 * while t < budget.  The swarm uses the model's visited-set memory (its bit arrays,
 * member records and a replay buffer); it invalidates the last query's trace. */
typedef struct mc_swarm_opts {
    uint32_t members;        /* searchers, >= 1 */
    uint32_t bits_log2;      /* bits per member = 2^bits_log2, 10..30 */
    uint64_t budget;         /* member steps after which no new walk starts */
    uint64_t seed;           /* base seed */
    uint32_t prune;          /* 1: over-time property with threshold T; 0: G(!FIN) */
    uint32_t T;
} mc_swarm_opts;

typedef struct mc_swarm_result {
    uint32_t best_clock;     /* least trail clock (UINT32_MAX: no trail) */
    uint32_t best_cfg;       /* its configuration */
    uint32_t best_member;    /* smallest member index that found it */
    uint32_t first_clock;    /* the trail found first on the device clock */
    uint32_t first_cfg;
    uint32_t pad;
    uint64_t trails, walks, steps;   /* totals over members */
    uint64_t first_trail_ns; /* device time from the swarm's start to its first trail */
    uint64_t swarm_ns;       /* GPU time of the swarm launch (HIP events) */
} mc_swarm_result;

/* Per-member record of the last swarm (80 bytes, as returned by mc_swarm_members). */
typedef struct mc_swarm_member {
    uint64_t walks, trails, steps;
    uint64_t best_walk_start;    /* member step at which the best trail's walk began */
    uint64_t first_step;         /* member step at which its first trail ended (~0: none) */
    uint64_t start_ticks, first_ticks;   /* device clock, 100 MHz */
    uint32_t best_clock, best_cfg;       /* UINT32_MAX without trails */
    uint32_t first_clock, first_cfg;
    uint32_t pad[2];
} mc_swarm_member;

/* One swarm.  MC_E_NOMEM if the model's visited set is smaller than the swarm needs:
 * members x (80 B + 2^bits_log2 / 8 B) plus one trail of the longest path. */
int mc_swarm(mc_model *h, const mc_swarm_opts *o, mc_swarm_result *r);
/* The last swarm's member records; out: host array of cap >= members records. */
int mc_swarm_members(const mc_model *h, mc_swarm_member *out, size_t cap);
/* The swarm search of Sec. 5: a swarm against G(!FIN) gives a time T; then swarms
 * against the over-time property with threshold T - 1 (new seeds, the same budget)
 * while one finds a trail, whose least clock becomes T.  Returns the last T found,
 * the number of swarms run, and that swarm's result.  MC_E_STATE if the first swarm
 * finds no trail. */
int mc_swarm_tune(mc_model *h, const mc_swarm_opts *o, uint32_t *t_found, uint32_t *rounds,
                  mc_swarm_result *best);
/* The trail of the best trail of the last mc_swarm or mc_swarm_tune (the walk replayed
 * from its seed), rows as mc_trace, root first.  MC_E_STATE if there is none. */
int mc_swarm_trace(mc_model *h, uint32_t *rows, size_t cap, size_t *len);

/* ---- batched exploration: many models in one persistent launch ----------------- */
/* The models of a batch are disjoint state graphs, and so are the configurations of a
 * model after SELECT: every (model, configuration) subgraph becomes one partition of a
 * single queue, largest first, consumed by one persistent launch.  Each model keeps its
 * own visited set, carved from one arena in the caller's workspace. */
typedef struct mc_batch mc_batch;

typedef struct mc_batch_opts {
    uint32_t block;          /* threads per workgroup: 256, 512, 1024 (0 = 512) */
    uint32_t grid;           /* persistent workgroups (0 = automatic) */
    float load_factor;       /* visited-set load factor (0 = 0.5) */
    uint32_t chunk;          /* states generated per super-step before waiting for the
                                visited set (0 = 2 x block x lane_items) */
    uint32_t use_graph;      /* 1: capture the query's launch sequence once in a hipGraph
                                and replay it (needs a non-null stream: MC_E_INVAL) */
    uint32_t lane_items;     /* keys each thread inserts per round trip: 1 or 2
                                (else automatic: 2 for keys of up to 128 bits,
                                1 for wider keys) */
    uint32_t part_states;    /* target states per partition when a configuration's
                                subgraph is cut into blocks of whole rounds
                                (0 = automatic, UINT32_MAX = never cut) */
    uint32_t reserved[1];
} mc_batch_opts;

/* Workspace bytes of a batch of n models (host array of n descriptors). */
int mc_batch_workspace_bytes(const mc_desc *models, uint32_t n, const mc_batch_opts *o,
                             size_t *bytes);
/* Create a batch in the caller's device workspace on the given stream.  The library
 * owns *out.  MC_E_NOMEM if ws_bytes is too small; MC_E_INVAL for any invalid model. */
int mc_batch_create(const mc_desc *models, uint32_t n, const mc_batch_opts *o, void *dev_ws,
                    size_t ws_bytes, void *stream, mc_batch **out);
/* min_time of every model: t_min[i] and the reachable count states[i] (host arrays of
 * n, either may be NULL); st aggregates the counters (explore_ns = the whole query on
 * the GPU).  Per-model argmin sets come from mc_batch_terminal_clocks. */
int mc_batch_min_time(mc_batch *b, uint32_t *t_min, uint64_t *states, mc_stats *st);
/* Per-configuration least terminal clocks of one model of the last mc_batch_min_time. */
int mc_batch_terminal_clocks(const mc_batch *b, uint32_t model, uint32_t *tc, size_t cap);
int mc_batch_free(mc_batch *b);
/* Autotuner: tries block in {256,512,1024} x load factor in {0.25,0.5,0.7} x lane_items
 * in {1,2} x chunk in {1,2} x block x lane_items on the batch itself, in the caller's
 * workspace (candidates that do not fit are skipped), and returns the fastest options and their GPU time (-1 when served
 * from the per-process cache, keyed by the batch and the device architecture). */
int mc_batch_autotune(const mc_desc *models, uint32_t n, void *dev_ws, size_t ws_bytes,
                      void *stream, mc_batch_opts *best, float *best_ms);

/* ---- serving: continuous batching of queries ------------------------------------ */
/* A query server over the persistent engine (Sec. 4 Steps 2-4 for each query).
 * Queries (min_time or check(T) of a model) are submitted at any time.  Each model
 * keeps its explored state on the device between queries: its visited set (sized for
 * all its states), per-configuration least clocks and the threshold T_done up to which
 * every state is in the set (min_time: all of them).  Each mc_engine_step:
 *   1. admits waiting queries in arrival order.  A query on a model whose state is
 *      resident and covers it (min_time after a min_time; check(T) with T <= T_done) is
 *      answered from that state: its count by a scan of the set, no exploration.  A
 *      check above T_done continues the exploration from the rounds that hold T_done
 *      (units that all work alike; otherwise it starts over in the same memory).  A
 *      model seen for the first time needs an arena region and a model slot: idle
 *      models are evicted, least recently used first, to make room; a query that still
 *      does not fit waits, and so do later queries needing new memory.  A query on a
 *      model whose previous query still explores is answered at once if the set
 *      already covers it (that exploration only adds states past T_done), else it
 *      waits for it without blocking others;
 *   2. runs one persistent launch over the unfinished partitions of every active
 *      query; while queries wait for memory, a partition explores at most `slice`
 *      super-step levels, then saves its frontier and yields;
 *   3. retires the queries whose partitions are all explored.
 * Queries admitted later therefore share the device with queries already running.
 * Each model has its own visited set and every count is that of the query's threshold,
 * so a result is the same alone, in the mix, resumed or answered from resident state
 * (`levels` excepted: 0 when answered from resident state without exploring). */
#define MC_QUERY_MIN_TIME 0u
#define MC_QUERY_CHECK 1u

typedef struct mc_engine mc_engine;

typedef struct mc_engine_opts {
    uint32_t max_active;     /* model slots: queries on the device at once (>= 1) */
    uint32_t max_cfg;        /* largest configuration count a query may have (>= 1) */
    uint32_t block;          /* threads per workgroup: 256, 512, 1024 (0 = 512) */
    uint32_t slice;          /* super-step levels per partition per step while queries
                                wait for memory (0 = no limit); with none waiting a
                                step runs its partitions to the end */
    uint32_t chunk;          /* states per super-step batch (0 = 2 x block x lane_items) */
    uint32_t grid;           /* persistent workgroups per step (0 = up to 1024) */
    float load_factor;       /* visited-set load factor (0 = 0.5) */
    uint32_t lane_items;     /* keys each thread inserts per round trip: 1 or 2
                                (else automatic: 2 for keys of up to 128 bits,
                                1 for wider keys) */
    uint32_t part_states;    /* target states per partition when a query's configurations
                                are cut into blocks of whole rounds (0 = automatic: about
                                states/256, at most 256 more partitions than
                                configurations; UINT32_MAX = never cut) */
    uint32_t no_reuse;       /* 1: free a model's state when its query retires (every
                                query explores from scratch, in a visited set sized for
                                its own threshold); 0: keep it (the default) */
    uint32_t reserved[2];
} mc_engine_opts;

typedef struct mc_query_result {
    uint32_t kind, T;
    int status;              /* MC_OK, MC_E_ADMIT (can never fit), or a query error */
    int done;                /* 1 once the result is final */
    int violated;            /* check(T): some terminal with clock <= T */
    uint32_t t_min;          /* least terminal clock reached (under T for check) */
    uint32_t n_argmin;       /* configurations attaining it */
    uint32_t argmin_first;   /* the smallest of them */
    uint64_t states;         /* states explored (count_T for check) */
    uint64_t levels;         /* BFS levels */
    uint64_t submit_ns, admit_ns, done_ns;  /* host monotonic clock */
    uint32_t steps;          /* engine steps the query was active */
    uint32_t reuse;          /* MC_REUSE_*: how the model's resident state served it */
} mc_query_result;

#define MC_REUSE_NONE 0u     /* explored from scratch */
#define MC_REUSE_RESUMED 1u  /* continued the model's resident exploration */
#define MC_REUSE_ANSWERED 2u /* answered from the resident state without exploring */

/* Device bytes for an engine whose query arena holds arena_bytes. */
int mc_engine_bytes(const mc_engine_opts *o, size_t arena_bytes, size_t *bytes);
/* Create an engine in the caller's device buffer on the given stream (library owns
 * *out; the buffer must outlive it).  MC_E_NOMEM if the buffer leaves no arena. */
int mc_engine_create(const mc_engine_opts *o, void *dev_buf, size_t buf_bytes, void *stream,
                     mc_engine **out);
/* Queue a query (kind MC_QUERY_*; T is used by check).  A query that can never fit the
 * arena or max_cfg completes at once with status MC_E_ADMIT.  MC_E_INVAL for an invalid
 * model. */
int mc_engine_submit(mc_engine *e, const mc_desc *model, uint32_t kind, uint32_t T,
                     uint64_t *ticket);
/* One engine iteration (admit, launch, retire); synchronous.  Returns the number of
 * active and waiting queries afterwards. */
int mc_engine_step(mc_engine *e, uint32_t *n_active, uint32_t *n_waiting);
/* Result of a ticket: MC_OK when done, MC_E_STATE while pending, MC_E_NOTFOUND. */
int mc_engine_poll(mc_engine *e, uint64_t ticket, mc_query_result *out);
/* The configurations attaining a finished query's t_min, ascending (Sec. 4 Step 4; as
 * mc_min_time's argmin): argmin may be NULL with cap 0 to query *n; MC_E_BUFFER if
 * cap < *n (the first cap are written).  MC_E_STATE while pending, MC_E_NOTFOUND. */
int mc_engine_argmin(mc_engine *e, uint64_t ticket, uint32_t *argmin, size_t cap, size_t *n);
/* Counterexample of a finished query whose t_min exists: a path from the root to a
 * terminal of its smallest argmin configuration at clock t_min, rows as mc_trace.  It is
 * read from the model's visited set, so the model's state must still be resident and
 * idle: MC_E_STATE otherwise (evicted, freed with no_reuse, or a later query on the
 * model running), or when the query has no terminal; MC_E_BUFFER if cap < *len;
 * MC_E_NOMEM if the arena has no room for the path's staging. */
int mc_engine_trace(mc_engine *e, uint64_t ticket, uint32_t *rows, size_t cap, size_t *len);
/* Forget a finished ticket. */
int mc_engine_release(mc_engine *e, uint64_t ticket);
int mc_engine_destroy(mc_engine *e);

#ifdef __cplusplus
}
#endif
#endif /* MCTUNE_H */
