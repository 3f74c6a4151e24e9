/* Sanitizer driver of the CPU oracle: runs every oracle entry point on a spread of models
 * (every kind, partial rounds, one to eight units, units of unequal speed, the tick clock,
 * pruned and exhaustive searches with traces and state dumps, walks and swarms) so that an
 * AddressSanitizer / UndefinedBehaviorSanitizer build of oracle/mc_oracle.c reports any
 * invalid access.  Test infrastructure only; built and run by tests/test_sanitizers.py. */
#include "../../oracle/mc_oracle.c"

#include <stdio.h>

static int failures = 0;

static void expect(int ok, const char *what) {
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        failures++;
    }
}

static void run(or_model *mo, const char *name) {
    or_result r, q;
    uint32_t tc[256];
    uint64_t cap = 1u << 20, len = 0, dump_cap = 1u << 16;
    uint32_t *trace = (uint32_t *)malloc(sizeof(uint32_t) * cap * (3 + mo->m));
    uint32_t *dump = (uint32_t *)malloc(sizeof(uint32_t) * dump_cap * (3 + mo->m));
    int rc = or_explore(mo, 0, 0, 1, &r, tc, trace, cap, &len, dump, dump_cap);
    expect(rc == OR_OK, name);
    if (rc == OR_OK) {
        expect(r.terminals > 0 && len > 1, name);
        rc = or_explore(mo, 1, r.t_min - 1, 0, &q, tc, trace, cap, &len, NULL, 0);
        expect(rc == OR_OK && !q.violated && q.reachable < r.reachable, name);
        rc = or_explore(mo, 1, r.t_min, 0, &q, tc, trace, cap, &len, NULL, 0);
        expect(rc == OR_OK && q.violated, name);
        uint32_t t = 0, c = 0;
        for (uint64_t seed = 0; seed < 4; seed++) {
            expect(or_simulate(mo, seed, &t, &c) == OR_OK && t >= r.t_min, name);
        }
        or_swarm_member mem[8];
        expect(or_swarm(mo, 3, 8, 2000, 6, 0, 0, mem) == OR_OK, name);
        expect(or_swarm(mo, 5, 8, 2000, 10, 1, r.t_min, mem) == OR_OK, name);
        uint32_t n, b, d, E[4096];
        for (uint32_t k = 0; k < mo->n_cfg; k++) {
            int rr = or_derive(mo, k, &n, &b, &d, E, 4096);
            expect(rr == OR_OK || rr == OR_E_BUFFER, name);
        }
    }
    free(trace);
    free(dump);
}

int main(void) {
    static uint32_t red[] = {1, 1, 0, 0, 1, 2, 0, 0, 2, 1, 0, 0, 2, 4, 0, 0, 4, 1, 0, 0, 8, 2, 0, 0};
    static uint32_t mat[] = {1, 1, 1, 1, 1, 2, 2, 1, 2, 1, 1, 2, 2, 2, 2, 2};
    static uint32_t unit[] = {2, 1, 0, 0, 2, 4, 0, 0, 4, 2, 0, 0, 8, 1, 0, 0};
    for (uint32_t m = 1; m <= 8; m++) {
        or_model mo;
        memset(&mo, 0, sizeof(mo));
        mo.kind = OR_REDUCTION;
        mo.m = m;
        mo.G = 32;
        mo.Lg = 5 + m;
        mo.Ll = 2;
        mo.Lc = 1;
        mo.Lb = m & 1;
        mo.n_cfg = 6;
        mo.params = red;
        run(&mo, "reduction");
        mo.tick = 1;
        run(&mo, "reduction, tick clock");
        mo.tick = 0;
        for (uint32_t u = 0; u < m; u++) mo.speed[u] = 1 + (u % 3);
        run(&mo, "reduction, unequal units");
    }
    for (uint32_t m = 2; m <= 5; m++) {
        or_model mo;
        memset(&mo, 0, sizeof(mo));
        mo.kind = OR_MATMUL;
        mo.m = m;
        mo.M = mo.N = mo.K = 4;
        mo.Lg = 7;
        mo.Ll = 3;
        mo.Lc = 1;
        mo.n_cfg = 4;
        mo.params = mat;
        run(&mo, "matmul");
    }
    for (int kind = OR_ABSTRACT; kind <= OR_MINIMUM; kind++) {
        for (uint32_t np = 1; np <= 4; np *= 2) {
            or_model mo;
            memset(&mo, 0, sizeof(mo));
            mo.kind = kind;
            mo.m = 2;
            mo.S = 16;
            mo.NP = np;
            mo.Lg = 4;
            mo.Ll = 1;
            mo.Lc = 1;
            mo.n_cfg = 4;
            mo.params = unit;
            run(&mo, kind == OR_ABSTRACT ? "abstract" : "minimum");
        }
    }
    /* invalid descriptors are rejected, not read past */
    or_model bad;
    memset(&bad, 0, sizeof(bad));
    bad.kind = OR_REDUCTION;
    bad.m = 2;
    bad.G = 48;
    bad.Lg = bad.Ll = bad.Lc = 1;
    bad.n_cfg = 6;
    bad.params = red;
    or_result r;
    expect(or_explore(&bad, 0, 0, 0, &r, NULL, NULL, 0, NULL, NULL, 0) != OR_OK, "invalid G");
    printf("oracle driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
