/*
 * mc_oracle.c -- CPU oracle of the explicit-state auto-tuning checker.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load or run this code.  It shares nothing with the GPU
 * library: its own model derivation, its own state layout, its own hash set, its own
 * successor function.
 *
 * What it computes.  Garanina, Staroletov and Gorlatch, "Auto-Tuning High-Performance
 * Programs Using Model Checking in Promela", turn tuning into a model-checking query
 * (Sec. 2): a model of an OpenCL kernel on an abstract platform picks its tuning
 * parameters nondeterministically; the over-time property G(FIN -> time > T)
 * (Sec. 4, Step 2) is violated exactly when some run terminates with time <= T, and
 * the least such T with the configuration of its counterexample is the tuning result
 * (Sec. 2 steps 3-4; Sec. 4, Steps 3-4).  This file answers those queries by plain
 * sequential breadth-first search over explicit states with an exact hash set.
 *
 * The transition system.  It is the timed system of the Promela processes of Sec. 4
 * (main / host / device / unit / pex / clock, Listings 3-9) with these readings:
 *   state        (cfg, clock, pending, rem[0..m-1]); rem_i = cycles left in the
 *                workgroup on compute unit i, 0 = idle.  The root carries cfg = ROOT.
 *   SELECT(c)    root -> (c, 0, n_c, 0,...,0) for every configuration c: the
 *                nondeterministic choice of WG and TS made by `main` (Listing 3).
 *   DISPATCH(i)  enabled when pending > 0 and rem_i = 0; rem_i := d_c, pending -= 1,
 *                no time passes (host and device hand workgroups to free units,
 *                Listings 4-6).  Every free unit gives its own successor.
 *   ADVANCE      enabled only when no DISPATCH is enabled and some unit is busy; the
 *                clock moves to the next operation end on any busy unit: the clock
 *                process (Listing 9) ticks only when every active processing element
 *                has reported, and a processing element reports each unit of work
 *                (Listing 8), so no time passes while a free unit could take work.
 *   terminal     pending = 0 and all units idle: FIN of the host (Listing 4); the
 *                terminal clock is the model time of the run.
 * Operation lists per workgroup (global loads at Lg, local steps at Ll, barriers at
 * Lb, compute at Lc; a barrier costs no time by default since the barrier process of
 * Listing 7 never advances time):
 *   reduction (WG, TS):   n = G/WG workgroups; ceil(G/(WG*TS)) x Lg, log2(WG) x Ll,
 *                         1 x Lb, TS x Lc.
 *   matmul (WGx,WGy,TS,VW): n = (M/WGx)*(N/(WGy*VW)); 2K x Lg, K(1+VW) x Ll,
 *                         2K/TS x Lb, K*VW x Lc.
 * Two kinds follow the paper's own Promela models of a unit with NP processing elements
 * (data size S, GMT = Lg, the local step Ll; n = S/(WG*TS) workgroups, at least one;
 * a workgroup of WG > NP items runs as WG/NP waves of NP elements, Listings 6 and 14):
 *   abstract (WG, TS):    every wave is one run of the abstract pex (Listing 8) over
 *                         S/TS tiles, timed by its long_work (see abstract_wave below).
 *   minimum (WG, TS):     the Minimum kernel (Listings 10 and 15): TS global accesses
 *                         at Lg per item and wave, then min(WG,NP)-1 local steps at Ll
 *                         and one global write at Lg.
 * E_c lists the distinct cumulative operation end times of one workgroup, in order;
 * d_c = last(E_c) is the workgroup duration.
 *
 * Nothing here is blocked, fused or reordered: one state at a time, in BFS order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define OR_MAX_CU 16
#define OR_ROOT 0xFFFFFFFFu
#define OR_NONE 0xFFFFFFFFu

#define OR_OK 0
#define OR_E_INVAL (-1)
#define OR_E_NOMEM (-2)
#define OR_E_BUFFER (-3)

/* self-check flags */
#define OR_CHK_MEASURE 1u   /* an edge that neither lowers pending nor raises the clock */
#define OR_CHK_DEADLOCK 2u  /* a non-terminal state without successors */
#define OR_CHK_GRADED 4u    /* a state reached at two different depths */
#define OR_CHK_PERMUTE 8u   /* a state whose unit-permuted twin is unreachable */

enum { OR_REDUCTION = 0, OR_MATMUL = 1, OR_ABSTRACT = 2, OR_MINIMUM = 3 };

typedef struct {
    int32_t kind;
    uint32_t m;
    uint32_t G, M, N, K;
    uint32_t S, NP;         /* abstract and minimum kinds: data size, elements per unit */
    uint32_t Lg, Ll, Lc, Lb;
    uint32_t n_cfg;
    const uint32_t *params; /* n_cfg rows of 4 values */
    int32_t tick;           /* 1: the clock advances one cycle per step (test variant) */
    uint32_t speed[OR_MAX_CU]; /* cycles a unit takes per cycle of work (0 or 1: full speed) */
} or_model;

typedef struct {
    uint64_t reachable;
    uint64_t edges;
    uint64_t levels;
    uint64_t terminals;
    int32_t violated;
    uint32_t t_min;
    uint32_t self_check;
    uint32_t trace_cfg;
    double seconds;
} or_result;

typedef struct {
    uint32_t n;  /* workgroups */
    uint32_t b;  /* |E| */
    uint32_t d;  /* workgroup duration */
    uint32_t *E; /* distinct cumulative operation end times, increasing */
} or_cfg;

static int is_pow2(uint32_t x) { return x != 0 && (x & (x - 1)) == 0; }

static uint32_t ilog2(uint32_t x) {
    uint32_t r = 0;
    while (x > 1) { x >>= 1; r++; }
    return r;
}

/* Growing list of operation latencies of one workgroup. */
typedef struct {
    uint64_t *lat;
    uint64_t len, cap;
} or_ops;

static int ops_push(or_ops *o, uint64_t lat) {
    if (o->len == o->cap) {
        uint64_t nc = o->cap ? 2 * o->cap : 64;
        if (nc > (1ull << 27)) return OR_E_INVAL;
        uint64_t *p = (uint64_t *)realloc(o->lat, sizeof(uint64_t) * nc);
        if (!p) return OR_E_NOMEM;
        o->lat = p;
        o->cap = nc;
    }
    o->lat[o->len++] = lat;
    return OR_OK;
}

/* One wave of the abstract pex (Listing 8), from the time bookkeeping of the process.
 * long_work(gt, tz) keeps reporting a unit of work, each report letting the clock tick
 * once, until time exceeds start_time + gt*tz: it returns at start_time + gt*tz + 1, or
 * at once if time is already past that.  The pex sets start_time when it starts, before
 * the local step of every tile and before its final write; not before a tile's global
 * load.  Each long_work call is one operation (its length may be zero).  Barriers cost
 * no time (Listing 7). */
static int abstract_wave(uint64_t S, uint64_t TS, uint64_t GMT, uint64_t LOC, or_ops *o) {
    uint64_t time = 0, start_time = 0;
    int rc;
    for (uint64_t i = 0; i < S / TS; i++) {
        uint64_t until = start_time + GMT * TS + 1;     /* global load of tile i */
        uint64_t t1 = until > time ? until : time;
        if ((rc = ops_push(o, t1 - time)) != OR_OK) return rc;
        time = t1;
        start_time = time;                              /* local step of tile i */
        if ((rc = ops_push(o, LOC * TS + 1)) != OR_OK) return rc;
        time = start_time + LOC * TS + 1;
    }
    start_time = time;                                  /* result to global memory */
    return ops_push(o, GMT * 1 + 1);
}

/* Workgroup count and operation list of the abstract and minimum kinds. */
static int derive_unit_model(const or_model *mo, const uint32_t *p, uint64_t *n, or_ops *o) {
    uint64_t S = mo->S, NP = mo->NP, WG = p[0], TS = p[1];
    if (!is_pow2(mo->S) || !is_pow2(mo->NP) || !is_pow2(p[0]) || !is_pow2(p[1])) return OR_E_INVAL;
    if (WG > S || TS > S) return OR_E_INVAL;
    *n = S / (WG * TS);
    if (*n == 0) *n = 1;
    uint64_t waves = WG > NP ? WG / NP : 1;
    uint64_t nwe = WG < NP ? WG : NP;
    int rc;
    if (mo->kind == OR_ABSTRACT) {
        for (uint64_t w = 0; w < waves; w++)
            if ((rc = abstract_wave(S, TS, mo->Lg, mo->Ll, o)) != OR_OK) return rc;
        return OR_OK;
    }
    for (uint64_t w = 0; w < waves; w++)            /* MAP, wave by wave */
        for (uint64_t i = 0; i < TS; i++)
            if ((rc = ops_push(o, mo->Lg)) != OR_OK) return rc;
    for (uint64_t i = 1; i < nwe; i++)              /* REDUCE local by element 0 */
        if ((rc = ops_push(o, mo->Ll)) != OR_OK) return rc;
    return ops_push(o, mo->Lg);                     /* the minimum to global memory */
}

/* Per-configuration derivation: workgroup count and operation end times. */
static int derive(const or_model *mo, uint32_t c, or_cfg *out) {
    const uint32_t *p = mo->params + 4u * c;
    uint64_t cnt[4], lat[4];
    uint64_t n;
    if (mo->kind == OR_ABSTRACT || mo->kind == OR_MINIMUM) {
        or_ops o = {NULL, 0, 0};
        int rc = derive_unit_model(mo, p, &n, &o);
        uint64_t b = 0, t = 0;
        for (uint64_t i = 0; rc == OR_OK && i < o.len; i++) b += o.lat[i] ? 1 : 0;
        if (rc == OR_OK && (n > 0xFFFFFFFFull || b == 0 || b > (1u << 26))) rc = OR_E_INVAL;
        if (rc == OR_OK && !(out->E = (uint32_t *)malloc(sizeof(uint32_t) * b))) rc = OR_E_NOMEM;
        for (uint64_t i = 0, k = 0; rc == OR_OK && i < o.len; i++) {
            t += o.lat[i];
            if (t > 0xFFFFFFFFull) { free(out->E); out->E = NULL; rc = OR_E_INVAL; break; }
            if (o.lat[i]) out->E[k++] = (uint32_t)t;
        }
        free(o.lat);
        if (rc != OR_OK) return rc;
        out->n = (uint32_t)n;
        out->b = (uint32_t)b;
        out->d = (uint32_t)t;
        return OR_OK;
    }
    if (mo->kind == OR_REDUCTION) {
        uint32_t WG = p[0], TS = p[1];
        if (!is_pow2(WG) || !is_pow2(TS) || !is_pow2(mo->G) || WG > mo->G) return OR_E_INVAL;
        n = mo->G / WG;
        uint64_t per = (uint64_t)WG * TS;
        cnt[0] = (mo->G + per - 1) / per; lat[0] = mo->Lg;
        cnt[1] = ilog2(WG);               lat[1] = mo->Ll;
        cnt[2] = 1;                       lat[2] = mo->Lb;
        cnt[3] = TS;                      lat[3] = mo->Lc;
    } else if (mo->kind == OR_MATMUL) {
        uint32_t X = p[0], Y = p[1], TS = p[2], VW = p[3] ? p[3] : 1;
        if (!X || !Y || !TS) return OR_E_INVAL;
        if (mo->M % X || mo->N % ((uint64_t)Y * VW) || mo->K % TS) return OR_E_INVAL;
        n = (uint64_t)(mo->M / X) * (mo->N / ((uint64_t)Y * VW));
        cnt[0] = 2ull * mo->K;               lat[0] = mo->Lg;
        cnt[1] = (uint64_t)mo->K * (1 + VW); lat[1] = mo->Ll;
        cnt[2] = 2ull * (mo->K / TS);        lat[2] = mo->Lb;
        cnt[3] = (uint64_t)mo->K * VW;       lat[3] = mo->Lc;
    } else {
        return OR_E_INVAL;
    }
    if (n == 0 || n > 0xFFFFFFFFull) return OR_E_INVAL;
    uint64_t b = 0;
    for (int j = 0; j < 4; j++) if (lat[j]) b += cnt[j];
    if (b == 0 || b > (1u << 26)) return OR_E_INVAL;
    out->E = (uint32_t *)malloc(sizeof(uint32_t) * b);
    if (!out->E) return OR_E_NOMEM;
    uint64_t t = 0, k = 0;
    for (int j = 0; j < 4; j++) {
        for (uint64_t r = 0; r < cnt[j]; r++) {
            t += lat[j];
            if (t > 0xFFFFFFFFull) { free(out->E); out->E = NULL; return OR_E_INVAL; }
            if (lat[j]) out->E[k++] = (uint32_t)t;
        }
    }
    out->n = (uint32_t)n;
    out->b = (uint32_t)b;
    out->d = (uint32_t)t;
    return OR_OK;
}

/* ---- explicit state set ---------------------------------------------------------- */

typedef struct {
    uint32_t S;          /* words per state: 3 + m */
    uint32_t *st;        /* states, BFS order */
    uint32_t *parent;
    uint32_t *depth;
    uint64_t count, cap;
    uint32_t *slot;      /* open addressing: state index + 1, 0 = empty */
    uint64_t slots;
} or_set;

static uint64_t fnv1a(const uint32_t *w, uint32_t S) {
    uint64_t h = 1469598103934665603ull;
    for (uint32_t i = 0; i < S; i++) {
        for (int k = 0; k < 4; k++) {
            h ^= (w[i] >> (8 * k)) & 0xFFu;
            h *= 1099511628211ull;
        }
    }
    return h;
}

static int set_init(or_set *s, uint32_t S) {
    memset(s, 0, sizeof(*s));
    s->S = S;
    s->cap = 1024;
    s->slots = 4096;
    s->st = (uint32_t *)malloc(sizeof(uint32_t) * S * s->cap);
    s->parent = (uint32_t *)malloc(sizeof(uint32_t) * s->cap);
    s->depth = (uint32_t *)malloc(sizeof(uint32_t) * s->cap);
    s->slot = (uint32_t *)calloc(s->slots, sizeof(uint32_t));
    return (s->st && s->parent && s->depth && s->slot) ? OR_OK : OR_E_NOMEM;
}

static void set_free(or_set *s) {
    free(s->st); free(s->parent); free(s->depth); free(s->slot);
    memset(s, 0, sizeof(*s));
}

/* index of state w, or -1 */
static int64_t set_find(const or_set *s, const uint32_t *w) {
    uint64_t mask = s->slots - 1, i = fnv1a(w, s->S) & mask;
    for (;;) {
        uint32_t v = s->slot[i];
        if (v == 0) return -1;
        if (memcmp(s->st + (uint64_t)(v - 1) * s->S, w, sizeof(uint32_t) * s->S) == 0)
            return (int64_t)(v - 1);
        i = (i + 1) & mask;
    }
}

static int set_grow(or_set *s) {
    uint64_t ns = s->slots * 2;
    uint32_t *nsl = (uint32_t *)calloc(ns, sizeof(uint32_t));
    if (!nsl) return OR_E_NOMEM;
    for (uint64_t k = 0; k < s->count; k++) {
        uint64_t i = fnv1a(s->st + k * s->S, s->S) & (ns - 1);
        while (nsl[i]) i = (i + 1) & (ns - 1);
        nsl[i] = (uint32_t)(k + 1);
    }
    free(s->slot);
    s->slot = nsl;
    s->slots = ns;
    return OR_OK;
}

/* insert w; returns its index, sets *fresh */
static int64_t set_insert(or_set *s, const uint32_t *w, uint32_t parent, uint32_t depth,
                          int *fresh) {
    int64_t f = set_find(s, w);
    if (f >= 0) { *fresh = 0; return f; }
    if ((s->count + 1) * 2 > s->slots && set_grow(s) != OR_OK) return OR_E_NOMEM;
    if (s->count == s->cap) {
        uint64_t nc = s->cap * 2;
        uint32_t *a = (uint32_t *)realloc(s->st, sizeof(uint32_t) * s->S * nc);
        if (!a) return OR_E_NOMEM;
        s->st = a;
        uint32_t *b = (uint32_t *)realloc(s->parent, sizeof(uint32_t) * nc);
        if (!b) return OR_E_NOMEM;
        s->parent = b;
        uint32_t *c = (uint32_t *)realloc(s->depth, sizeof(uint32_t) * nc);
        if (!c) return OR_E_NOMEM;
        s->depth = c;
        s->cap = nc;
    }
    if (s->count >= 0xFFFFFFFEull) return OR_E_NOMEM;
    uint64_t k = s->count++;
    memcpy(s->st + k * s->S, w, sizeof(uint32_t) * s->S);
    s->parent[k] = parent;
    s->depth[k] = depth;
    uint64_t mask = s->slots - 1, i = fnv1a(w, s->S) & mask;
    while (s->slot[i]) i = (i + 1) & mask;
    s->slot[i] = (uint32_t)(k + 1);
    *fresh = 1;
    return (int64_t)k;
}

/* ---- successor function -------------------------------------------------------- */

static uint32_t unit_speed(const or_model *mo, uint32_t i) {
    return mo->speed[i] ? mo->speed[i] : 1u;
}

/* A unit of speed s runs every operation s times as long: its operation ends within a
 * workgroup are s*E and the workgroup lasts s*d.  Smallest s*x, x in E, with s*x > e,
 * for 0 <= e < s*d. */
static uint32_t next_end(const or_cfg *cf, uint32_t s, uint32_t e) {
    for (uint32_t k = 0; k < cf->b; k++)
        if ((uint64_t)s * cf->E[k] > e) return s * cf->E[k];
    return s * cf->d; /* unreachable for a busy unit */
}

/*
 * Writes the successors of state x (S words each) into out; returns their number.
 * out must hold at least max(n_cfg, m) states.
 */
static uint32_t successors(const or_model *mo, const or_cfg *cfs, const uint32_t *x,
                           uint32_t *out) {
    const uint32_t m = mo->m, S = 3 + m;
    uint32_t k = 0;
    if (x[0] == OR_ROOT) {                       /* SELECT */
        for (uint32_t c = 0; c < mo->n_cfg; c++) {
            uint32_t *y = out + (uint64_t)k++ * S;
            memset(y, 0, sizeof(uint32_t) * S);
            y[0] = c;
            y[1] = 0;
            y[2] = cfs[c].n;
        }
        return k;
    }
    const or_cfg *cf = &cfs[x[0]];
    const uint32_t *rem = x + 3;
    if (x[2] > 0) {                               /* DISPATCH */
        for (uint32_t i = 0; i < m; i++) {
            if (rem[i] != 0) continue;
            uint32_t *y = out + (uint64_t)k++ * S;
            memcpy(y, x, sizeof(uint32_t) * S);
            y[2] = x[2] - 1;
            y[3 + i] = unit_speed(mo, i) * cf->d;
        }
        if (k) return k;
    }
    int busy = 0;
    for (uint32_t i = 0; i < m; i++) busy |= rem[i] != 0;
    if (!busy) return 0;                          /* terminal */
    uint32_t delta = 0xFFFFFFFFu;                 /* ADVANCE */
    if (mo->tick) {
        delta = 1;
    } else {
        for (uint32_t i = 0; i < m; i++) {
            if (!rem[i]) continue;
            uint32_t s = unit_speed(mo, i);
            uint32_t e = s * cf->d - rem[i];
            uint32_t di = next_end(cf, s, e) - e;
            if (di < delta) delta = di;
        }
    }
    uint32_t *y = out;
    memcpy(y, x, sizeof(uint32_t) * S);
    y[1] = x[1] + delta;
    for (uint32_t i = 0; i < m; i++)
        if (rem[i]) y[3 + i] = rem[i] - delta;
    return 1;
}

static int is_terminal(const uint32_t *x, uint32_t m) {
    if (x[0] == OR_ROOT || x[2] != 0) return 0;
    for (uint32_t i = 0; i < m; i++)
        if (x[3 + i]) return 0;
    return 1;
}

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

static void free_cfgs(or_cfg *cfs, uint32_t n) {
    if (!cfs) return;
    for (uint32_t c = 0; c < n; c++) free(cfs[c].E);
    free(cfs);
}

static int load_cfgs(const or_model *mo, or_cfg **out) {
    if (mo->m == 0 || mo->m > OR_MAX_CU || mo->n_cfg == 0) return OR_E_INVAL;
    if (mo->Lg == 0 || mo->Ll == 0 || mo->Lc == 0) return OR_E_INVAL;
    or_cfg *cfs = (or_cfg *)calloc(mo->n_cfg, sizeof(or_cfg));
    if (!cfs) return OR_E_NOMEM;
    for (uint32_t c = 0; c < mo->n_cfg; c++) {
        int rc = derive(mo, c, &cfs[c]);
        if (rc != OR_OK) { free_cfgs(cfs, mo->n_cfg); return rc; }
    }
    *out = cfs;
    return OR_OK;
}

/* ---- exported entry points ------------------------------------------------------- */

/* Derivation of configuration c: workgroups, |E|, duration, and E itself (cap entries). */
int or_derive(const or_model *mo, uint32_t c, uint32_t *n, uint32_t *b, uint32_t *d,
              uint32_t *E, uint64_t cap) {
    if (c >= mo->n_cfg) return OR_E_INVAL;
    or_cfg cf;
    int rc = derive(mo, c, &cf);
    if (rc != OR_OK) return rc;
    *n = cf.n; *b = cf.b; *d = cf.d;
    if (E) {
        if (cap < cf.b) { free(cf.E); return OR_E_BUFFER; }
        memcpy(E, cf.E, sizeof(uint32_t) * cf.b);
    }
    free(cf.E);
    return OR_OK;
}

/* Successors of one state (rows of 3+m words); returns the count or a negative code. */
int or_successors(const or_model *mo, const uint32_t *x, uint32_t *out, uint64_t cap) {
    or_cfg *cfs;
    int rc = load_cfgs(mo, &cfs);
    if (rc != OR_OK) return rc;
    uint32_t need = mo->n_cfg > mo->m ? mo->n_cfg : mo->m;
    if (x[0] != OR_ROOT && x[0] >= mo->n_cfg) { free_cfgs(cfs, mo->n_cfg); return OR_E_INVAL; }
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (3 + mo->m) * need);
    if (!tmp) { free_cfgs(cfs, mo->n_cfg); return OR_E_NOMEM; }
    uint32_t k = successors(mo, cfs, x, tmp);
    if (k > cap) { free(tmp); free_cfgs(cfs, mo->n_cfg); return OR_E_BUFFER; }
    memcpy(out, tmp, sizeof(uint32_t) * (3 + mo->m) * k);
    free(tmp);
    free_cfgs(cfs, mo->n_cfg);
    return (int)k;
}

/*
 * Full exploration.  prune != 0 drops every successor with clock > T (the clock never
 * decreases along an edge, so this is exactly the set of states with clock <= T).
 * tc[c] receives the least terminal clock of configuration c (OR_NONE if none).
 * The trace (rows of 3+m words, root first) goes to the terminal of the smallest
 * configuration attaining T_min (no pruning) or of the smallest configuration with a
 * terminal clock <= T (pruning); trace may be NULL.
 * dump (may be NULL) receives every reached state in BFS order, dump_cap rows.
 */
int or_explore(const or_model *mo, int prune, uint32_t T, int self_check, or_result *res,
               uint32_t *tc, uint32_t *trace, uint64_t trace_cap, uint64_t *trace_len,
               uint32_t *dump, uint64_t dump_cap) {
    or_cfg *cfs;
    int rc = load_cfgs(mo, &cfs);
    if (rc != OR_OK) return rc;
    const uint32_t m = mo->m, S = 3 + m;
    uint32_t need = mo->n_cfg > m ? mo->n_cfg : m;
    uint32_t *succ = (uint32_t *)malloc(sizeof(uint32_t) * S * need);
    uint32_t *best = (uint32_t *)malloc(sizeof(uint32_t) * mo->n_cfg); /* terminal index */
    or_set set;
    if (!succ || !best || set_init(&set, S) != OR_OK) {
        free(succ); free(best); set_free(&set); free_cfgs(cfs, mo->n_cfg);
        return OR_E_NOMEM;
    }
    memset(res, 0, sizeof(*res));
    for (uint32_t c = 0; c < mo->n_cfg; c++) { tc[c] = OR_NONE; best[c] = OR_NONE; }

    double t0 = now_s();
    uint32_t *root = succ; /* scratch */
    memset(root, 0, sizeof(uint32_t) * S);
    root[0] = OR_ROOT;
    int fresh;
    uint32_t *rootcopy = (uint32_t *)malloc(sizeof(uint32_t) * S);
    if (!rootcopy) { rc = OR_E_NOMEM; goto done; }
    memcpy(rootcopy, root, sizeof(uint32_t) * S);
    if (set_insert(&set, rootcopy, OR_NONE, 0, &fresh) < 0) { free(rootcopy); rc = OR_E_NOMEM; goto done; }
    free(rootcopy);

    uint32_t flags = 0;
    uint64_t maxdepth = 0;
    uint32_t *x = (uint32_t *)malloc(sizeof(uint32_t) * S);
    if (!x) { rc = OR_E_NOMEM; goto done; }
    for (uint64_t head = 0; head < set.count; head++) {
        memcpy(x, set.st + head * S, sizeof(uint32_t) * S);
        uint32_t dx = set.depth[head];
        if (dx > maxdepth) maxdepth = dx;
        uint32_t k = successors(mo, cfs, x, succ);
        if (k == 0 && !is_terminal(x, m)) flags |= OR_CHK_DEADLOCK;
        for (uint32_t j = 0; j < k; j++) {
            uint32_t *y = succ + (uint64_t)j * S;
            if (x[0] != OR_ROOT && !(y[2] < x[2] || y[1] > x[1])) flags |= OR_CHK_MEASURE;
            if (prune && y[1] > T) continue;
            res->edges++;
            int64_t idx = set_insert(&set, y, (uint32_t)head, dx + 1, &fresh);
            if (idx < 0) { free(x); rc = OR_E_NOMEM; goto done; }
            if (!fresh) {
                if (set.depth[idx] != dx + 1) flags |= OR_CHK_GRADED;
                continue;
            }
            if (is_terminal(y, m)) {
                res->terminals++;
                uint32_t c = y[0];
                if (y[1] < tc[c]) { tc[c] = y[1]; best[c] = (uint32_t)idx; }
            }
        }
    }
    free(x);
    res->seconds = now_s() - t0;
    res->reachable = set.count;
    res->levels = maxdepth + 1;

    if (self_check && !prune) {
        /* swapping two units of equal speed maps a reachable state to a reachable one:
           test the transpositions of each unit with the first unit of its speed */
        uint32_t *y = (uint32_t *)malloc(sizeof(uint32_t) * S);
        if (!y) { rc = OR_E_NOMEM; goto done; }
        for (uint64_t k = 0; k < set.count && !(flags & OR_CHK_PERMUTE); k++) {
            const uint32_t *z = set.st + k * S;
            if (z[0] == OR_ROOT) continue;
            for (uint32_t i = 1; i < m; i++) {
                uint32_t f = 0;
                while (unit_speed(mo, f) != unit_speed(mo, i)) f++;
                if (f == i) continue;
                memcpy(y, z, sizeof(uint32_t) * S);
                y[3 + f] = z[3 + i];
                y[3 + i] = z[3 + f];
                if (set_find(&set, y) < 0) { flags |= OR_CHK_PERMUTE; break; }
            }
        }
        free(y);
    }
    if (!self_check) flags = 0;
    if (prune) flags &= ~(uint32_t)OR_CHK_DEADLOCK; /* pruned states lose successors */
    res->self_check = flags;

    res->t_min = OR_NONE;
    for (uint32_t c = 0; c < mo->n_cfg; c++)
        if (tc[c] < res->t_min) res->t_min = tc[c];
    res->violated = prune ? (res->terminals > 0) : 0;

    if (dump) {
        if (dump_cap < set.count) { rc = OR_E_BUFFER; goto done; }
        memcpy(dump, set.st, sizeof(uint32_t) * S * set.count);
    }

    /* trace target */
    uint32_t target = OR_NONE;
    res->trace_cfg = OR_NONE;
    for (uint32_t c = 0; c < mo->n_cfg; c++) {
        if (best[c] == OR_NONE) continue;
        if (!prune && tc[c] != res->t_min) continue;
        target = best[c];
        res->trace_cfg = c;
        break;
    }
    if (trace_len) *trace_len = 0;
    if (target != OR_NONE && trace_len) {
        uint64_t len = 0;
        for (uint32_t v = target; v != OR_NONE; v = set.parent[v]) len++;
        *trace_len = len;
        if (trace) {
            if (trace_cap < len) { rc = OR_E_BUFFER; goto done; }
            uint64_t pos = len;
            for (uint32_t v = target; v != OR_NONE; v = set.parent[v]) {
                pos--;
                memcpy(trace + pos * S, set.st + (uint64_t)v * S, sizeof(uint32_t) * S);
            }
        }
    }
    rc = OR_OK;
done:
    free(succ);
    free(best);
    set_free(&set);
    free_cfgs(cfs, mo->n_cfg);
    return rc;
}

/* Terminal clock of one seeded random walk (uniform choice among successors, drawn
 * from splitmix64 over (seed, step)).  *cfg gets the configuration it selected. */
static uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int or_simulate(const or_model *mo, uint64_t seed, uint32_t *t_end, uint32_t *cfg) {
    or_cfg *cfs;
    int rc = load_cfgs(mo, &cfs);
    if (rc != OR_OK) return rc;
    const uint32_t m = mo->m, S = 3 + m;
    uint32_t need = mo->n_cfg > m ? mo->n_cfg : m;
    uint32_t *succ = (uint32_t *)malloc(sizeof(uint32_t) * S * need);
    uint32_t *x = (uint32_t *)calloc(S, sizeof(uint32_t));
    if (!succ || !x) { free(succ); free(x); free_cfgs(cfs, mo->n_cfg); return OR_E_NOMEM; }
    x[0] = OR_ROOT;
    for (uint64_t step = 0;; step++) {
        uint32_t k = successors(mo, cfs, x, succ);
        if (k == 0) break;
        uint64_t r = splitmix64(seed ^ splitmix64(step));
        memcpy(x, succ + (r % k) * S, sizeof(uint32_t) * S);
    }
    *t_end = x[1];
    *cfg = x[0];
    free(succ);
    free(x);
    free_cfgs(cfs, mo->n_cfg);
    return OR_OK;
}

/*
 * Swarm search (Sec. 5).  Swarm model checking runs many independent, incomplete
 * searches at once: each member hashes states into a bit array of its own (bitstate
 * hashing) instead of storing them, and reports the counterexamples it meets within a
 * bounded number of model steps.  Against the non-termination property G(!FIN) every
 * run reaching a terminal is a counterexample whose terminal clock is a model time;
 * against the over-time property with threshold T only terminals with clock <= T are.
 *
 * One member, read as follows:
 *   seed_i   = splitmix64(base_seed + i)
 *   a walk   starts at the root and, at member step t (counted over all its walks),
 *            takes successor number splitmix64(seed_i ^ splitmix64(t)) mod k of the k
 *            successors (configurations in order at the root, free units in index
 *            order for DISPATCH), t += 1;
 *   pruning  with a threshold, a walk ends at the first state with clock > T;
 *   bitstate at every state it reaches (not the root) with other than exactly one
 *            successor, the walk computes h = a splitmix64 chain over (cfg, clock,
 *            pending, rem_0..rem_{m-1}) and bit positions h mod B and (h >> 32) mod B
 *            of its B = 2^bits_log2 bits; both set: the state was visited and the walk
 *            ends; else both are set;
 *   trail    a new terminal state ends the walk as a counterexample;
 *   budget   a new walk starts only while t < budget (a walk in progress finishes).
 */
typedef struct {
    uint64_t walks, trails, steps;
    uint64_t best_walk_start;  /* member step at which the walk of the best trail began */
    uint64_t first_step;       /* member step at which its first trail ended (or ~0) */
    uint32_t best_clock, best_cfg;   /* OR_NONE without trails */
    uint32_t first_clock, first_cfg; /* the first trail */
} or_swarm_member;

static uint64_t state_hash(const uint32_t *x, uint32_t m) {
    uint64_t h = splitmix64((uint64_t)x[0]);
    h = splitmix64(h ^ x[1]);
    h = splitmix64(h ^ x[2]);
    for (uint32_t i = 0; i < m; i++) h = splitmix64(h ^ x[3 + i]);
    return h;
}

int or_swarm(const or_model *mo, uint64_t base_seed, uint32_t members, uint64_t budget,
             uint32_t bits_log2, int prune, uint32_t T, or_swarm_member *out) {
    if (bits_log2 < 6 || bits_log2 > 34) return OR_E_INVAL;
    or_cfg *cfs;
    int rc = load_cfgs(mo, &cfs);
    if (rc != OR_OK) return rc;
    const uint32_t m = mo->m, S = 3 + m;
    const uint32_t need = mo->n_cfg > m ? mo->n_cfg : m;
    const uint64_t B = 1ull << bits_log2;
    uint32_t *succ = (uint32_t *)malloc(sizeof(uint32_t) * S * need);
    uint32_t *next = (uint32_t *)malloc(sizeof(uint32_t) * S * need);
    uint32_t *x = (uint32_t *)calloc(S, sizeof(uint32_t));
    uint8_t *bits = (uint8_t *)malloc(B / 8);
    if (!succ || !next || !x || !bits) {
        free(succ); free(next); free(x); free(bits);
        free_cfgs(cfs, mo->n_cfg);
        return OR_E_NOMEM;
    }
    for (uint32_t i = 0; i < members; i++) {
        or_swarm_member *r = &out[i];
        memset(r, 0, sizeof(*r));
        r->first_step = ~0ull;
        r->best_clock = r->best_cfg = r->first_clock = r->first_cfg = OR_NONE;
        memset(bits, 0, B / 8);
        const uint64_t seed = splitmix64(base_seed + i);
        uint64_t t = 0;
        while (t < budget) {
            r->walks++;
            const uint64_t start = t;
            memset(x, 0, sizeof(uint32_t) * S);
            x[0] = OR_ROOT;
            uint32_t k = successors(mo, cfs, x, succ);
            for (;;) {
                const uint64_t pick = splitmix64(seed ^ splitmix64(t)) % k;
                memcpy(x, succ + pick * S, sizeof(uint32_t) * S);
                t++;
                if (prune && x[1] > T) break;
                k = successors(mo, cfs, x, next);
                if (k != 1) {
                    const uint64_t h = state_hash(x, m);
                    const uint64_t p0 = h & (B - 1), p1 = (h >> 32) & (B - 1);
                    const int b0 = (bits[p0 >> 3] >> (p0 & 7)) & 1, b1 = (bits[p1 >> 3] >> (p1 & 7)) & 1;
                    if (b0 && b1) break;
                    bits[p0 >> 3] |= (uint8_t)(1u << (p0 & 7));
                    bits[p1 >> 3] |= (uint8_t)(1u << (p1 & 7));
                }
                if (k == 0) {
                    r->trails++;
                    if (r->first_step == ~0ull) {
                        r->first_step = t;
                        r->first_clock = x[1];
                        r->first_cfg = x[0];
                    }
                    if (r->best_clock == OR_NONE || x[1] < r->best_clock) {
                        r->best_clock = x[1];
                        r->best_cfg = x[0];
                        r->best_walk_start = start;
                    }
                    break;
                }
                uint32_t *tmp = succ; succ = next; next = tmp;
            }
        }
        r->steps = t;
    }
    free(succ); free(next); free(x); free(bits);
    free_cfgs(cfs, mo->n_cfg);
    return OR_OK;
}
