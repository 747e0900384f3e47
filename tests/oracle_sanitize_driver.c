/* Exercises every entry point of the oracle on small and degenerate inputs, for a
 * build under AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure:
 * it checks memory safety and defined behaviour of the oracle, not its values).
 * Exit status 0 when every call succeeds and every output is finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/bh_oracle.h"

static uint64_t rng_state = 0x243f6a8885a308d3ull;
static double uniform(void) {   /* xorshift64*, inputs only */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 0x2545f4914f6cdd1dull) >> 11) * 0x1.0p-53;
}

static int finite_all(const double *a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int fail(const char *what, int64_t n, int kind) {
    fprintf(stderr, "oracle check failed: %s (n=%lld, kind=%d)\n", what, (long long)n, kind);
    return 1;
}

/* kind 0: spread points; 1: all coincident; 2: coordinates on a coarse grid with
 * a quarter of them on one point (duplicate keys at the depth limit); 3: two
 * distant clusters */
static void make(int64_t n, int kind, double *pos, double *vel, double *mass) {
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            double x = 2.0 * uniform() - 1.0;
            if (kind == 1) x = 0.25 * (d + 1);
            if (kind == 2) x = (i < n / 4) ? 0.5 : floor(x * 4.0) / 4.0;
            if (kind == 3) x = 1e-3 * x + (i % 2 ? 10.0 : -10.0);
            pos[3 * i + d] = x;
            vel[3 * i + d] = 0.1 * (uniform() - 0.5);
        }
        mass[i] = (0.5 + uniform()) / (double)n;
    }
}

static int run_case(int64_t n, int kind, int32_t leaf_cap) {
    double *pos = malloc(sizeof(double) * 3 * n), *vel = malloc(sizeof(double) * 3 * n);
    double *mass = malloc(sizeof(double) * n), *acc = malloc(sizeof(double) * 3 * n);
    double *pot = malloc(sizeof(double) * n);
    int64_t *nm = malloc(sizeof(int64_t) * n), *np = malloc(sizeof(int64_t) * n);
    uint64_t *hash = malloc(sizeof(uint64_t) * n);
    int bad = 0;
    make(n, kind, pos, vel, mass);

    double lo[3];
    int32_t k;
    or_root_cube(n, pos, lo, &k);
    uint64_t *keys = malloc(sizeof(uint64_t) * n);
    uint32_t *perm = malloc(sizeof(uint32_t) * n);
    or_keys(n, pos, lo, k, keys);
    or_order(n, keys, perm);

    or_tree *t = or_tree_create(n, pos, mass, leaf_cap);
    if (!t) return fail("or_tree_create", n, kind);
    const int64_t nn = or_tree_nn(t);
    {
        double lo2[3], *M = malloc(sizeof(double) * nn), *com = malloc(sizeof(double) * 3 * nn);
        int32_t k2, *level = malloc(sizeof(int32_t) * nn), *parent = malloc(sizeof(int32_t) * nn);
        int32_t *nchild = malloc(sizeof(int32_t) * nn);
        uint32_t *first = malloc(sizeof(uint32_t) * nn), *count = malloc(sizeof(uint32_t) * nn);
        double *S6 = malloc(sizeof(double) * 6 * nn);
        or_tree_export(t, lo2, &k2, keys, perm, level, first, count, parent, nchild, M, com);
        or_tree_moments(t, S6);
        if (!finite_all(M, nn) || !finite_all(com, 3 * nn) || !finite_all(S6, 6 * nn))
            bad |= fail("export/moments", n, kind);
        free(M), free(com), free(level), free(parent), free(nchild), free(first), free(count), free(S6);
    }
    const double thetas[3] = {0.0, 0.6, 1e6};
    const double epss[2] = {0.01, 0.0};
    for (int a = 0; a < 3; ++a) {
        if (a == 0 && n > 100) continue;   /* theta = 0 is the O(n^2) direct sum: small n only */
        for (int b = 0; b < 2; ++b)
            for (int open = OR_OPEN_SIDE; open <= OR_OPEN_OFFSET; ++open)
                for (int quad = 0; quad <= 1; ++quad) {
                    or_params p = {thetas[a], epss[b], 1.0, leaf_cap, quad, open};
                    for (int64_t id = 0; id < nn; ++id) {
                        const double r2 = or_open_r2(t, &p, (int32_t)id);
                        if (!(r2 >= 0.0) || !isfinite(r2)) bad |= fail("or_open_r2", n, kind);
                    }
                    if (or_tree_walk(t, pos, &p, n, NULL, acc, pot, nm, np, hash, 1) != 0)
                        bad |= fail("or_tree_walk", n, kind);
                    /* unsoftened walks of coincident bodies are singular by definition */
                    if (b == 0 && !finite_all(acc, 3 * n)) bad |= fail("walk output", n, kind);
                    if (open == OR_OPEN_SIDE && !quad) {
                        for (int32_t g = 1; g <= 64; g *= 8) {
                            if (or_tree_walk_group(t, &p, g, n, NULL, acc, pot, nm, np, hash, 1) != 0)
                                bad |= fail("or_tree_walk_group", n, kind);
                            /* the cube groups of at most g bodies */
                            const int64_t ng = or_tree_group_cubes(t, g, NULL);
                            int64_t *starts = malloc(sizeof(int64_t) * (ng > 0 ? ng + 1 : 1));
                            if (ng < 1 || or_tree_group_cubes(t, g, starts) != ng ||
                                or_tree_walk_group_ranges(t, &p, ng, starts, n, NULL, acc, pot, nm, np, hash, 1) != 0)
                                bad |= fail("or_tree_group_cubes / walk_group_ranges", n, kind);
                            free(starts);
                        }
                    }
                }
    }
    {   /* a subset of targets, in a scrambled order */
        const int64_t nt = n < 7 ? n : 7;
        int64_t targets[7];
        for (int64_t i = 0; i < nt; ++i) targets[i] = (i * 5 + 3) % n;
        or_params p = {0.5, 0.01, 1.0, leaf_cap, 0, OR_OPEN_SIDE};
        if (or_tree_walk(t, pos, &p, nt, targets, acc, NULL, NULL, NULL, NULL, 1) != 0)
            bad |= fail("or_tree_walk targets", n, kind);
        if (or_direct(n, pos, mass, 0.01, 1.0, nt, targets, acc, pot, 1) != 0)
            bad |= fail("or_direct", n, kind);
    }
    or_tree_destroy(t);

    or_params p = {0.5, 0.01, 1.0, leaf_cap, 0, OR_OPEN_SIDE};
    if (or_forces(n, pos, mass, &p, n, NULL, acc, pot, nm, np, hash, 1) != 0) bad |= fail("or_forces", n, kind);
    if (or_kdk(n, pos, vel, mass, &p, 1e-3, 2, acc, 0, pot, 1) != 0) bad |= fail("or_kdk", n, kind);
    double KW[2];
    or_energy(n, vel, mass, pot, KW);
    if (!finite_all(KW, 2) || !finite_all(pos, 3 * n)) bad |= fail("or_kdk/or_energy", n, kind);
    (void)or_mix64((uint64_t)n);

    free(pos), free(vel), free(mass), free(acc), free(pot), free(nm), free(np), free(hash), free(keys), free(perm);
    return bad;
}

int main(void) {
    const int64_t ns[6] = {1, 2, 3, 65, 300, 1500};
    const int32_t caps[3] = {1, 8, 64};
    int bad = 0;
    for (int a = 0; a < 6; ++a)
        for (int kind = 0; kind < 4; ++kind)
            for (int c = 0; c < 3; ++c) {
                if (ns[a] == 1500 && c > 0) continue;
                bad |= run_case(ns[a], kind, caps[c]);
            }
    if (!bad) printf("oracle sanitizer driver: all cases ok\n");
    return bad;
}
