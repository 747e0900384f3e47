/*
 * Barnes-Hut reference oracle (FP64, plain C).  TEST INFRASTRUCTURE ONLY:
 * used by the tests, the smoke check and the benchmark's CPU baseline, never
 * by the product library.  See bh_oracle.h for the overview.
 *
 * Readings of the paper taken here (the paper does not fix them):
 *  - root cube: anchored at the per-axis minimum corner `lo`, side the
 *    smallest power of two L = 2^k strictly above the largest extent
 *    (L = 1 when all particles coincide), so that quantisation is exact;
 *  - depth limit 21 (63-bit keys): coincident particles never separate, so a
 *    level-21 cube is a leaf whatever its count;
 *  - single-child cubes are removed from the tree (their child takes their
 *    place); this changes no interaction, as the walk test below is monotone
 *    in the side length and such a chain holds one particle set;
 *  - "r" of the opening test is the cube side, "D" the distance from the body
 *    to the cube's centre of mass; the test is strict: accept iff
 *    s*s < theta^2 * D^2, evaluated exactly as written below;
 *  - Newtonian force with Plummer softening eps for monopoles and pairs;
 *    the body itself is skipped in leaf pairs; a pair at zero distance with
 *    eps = 0 contributes nothing (it is still counted as evaluated).
 */
#include "bh_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

uint64_t or_mix64(uint64_t x)
{
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* ---- root cube: lo = per-axis minimum, ext = largest fl(hi - lo),
 *      L = 2^k with ext < L <= 2 ext (frexp), L = 1 when ext == 0 ---- */
void or_root_cube(int64_t n, const double *pos, double lo[3], int32_t *k)
{
    double hi[3];
    for (int d = 0; d < 3; d++) { lo[d] = pos[d]; hi[d] = pos[d]; }
    for (int64_t i = 1; i < n; i++)
        for (int d = 0; d < 3; d++) {
            double v = pos[3 * i + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    double ext = 0.0;
    for (int d = 0; d < 3; d++) {
        double e = hi[d] - lo[d];
        if (e > ext) ext = e;
    }
    if (ext == 0.0) { *k = 0; return; }
    int e2;
    frexp(ext, &e2);   /* ext = f 2^e2, f in [1/2, 1) */
    *k = e2;
}

/* ---- Morton key: bit b of qx at 3b+2, of qy at 3b+1, of qz at 3b ---- */
uint64_t or_interleave(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint64_t key = 0;
    for (int b = 0; b < OR_MAX_LEVEL; b++) {
        key |= (uint64_t)((qx >> b) & 1u) << (3 * b + 2);
        key |= (uint64_t)((qy >> b) & 1u) << (3 * b + 1);
        key |= (uint64_t)((qz >> b) & 1u) << (3 * b);
    }
    return key;
}

/* q_d = floor(fl(x_d - lo_d) * 2^(21-k)), in [0, 2^21) */
void or_keys(int64_t n, const double *pos, const double lo[3], int32_t k, uint64_t *keys)
{
    double scale = ldexp(1.0, OR_MAX_LEVEL - k);
    for (int64_t i = 0; i < n; i++) {
        uint32_t q[3];
        for (int d = 0; d < 3; d++) {
            double off = pos[3 * i + d] - lo[d];
            double c = floor(off * scale);
            if (c < 0.0) c = 0.0;                     /* cannot happen: off >= 0 */
            if (c > 2097151.0) c = 2097151.0;         /* cannot happen: off < L */
            q[d] = (uint32_t)c;
        }
        keys[i] = or_interleave(q[0], q[1], q[2]);
    }
}

/* ---- order by (key, original index) ---- */
static const uint64_t *g_sort_keys;
static int cmp_rank(const void *a, const void *b)
{
    uint32_t i = *(const uint32_t *)a, j = *(const uint32_t *)b;
    uint64_t ki = g_sort_keys[i], kj = g_sort_keys[j];
    if (ki != kj) return ki < kj ? -1 : 1;
    return (i > j) - (i < j);
}

void or_order(int64_t n, const uint64_t *keys, uint32_t *perm)
{
    for (int64_t i = 0; i < n; i++) perm[i] = (uint32_t)i;
    g_sort_keys = keys;   /* the oracle is not re-entrant here; tests call it from one thread */
    qsort(perm, (size_t)n, sizeof(uint32_t), cmp_rank);
}

/* ---- compressed octree, depth-first preorder ---- */
typedef struct {
    or_tree *t;
    int64_t cap;
    int32_t leaf_cap;
    int failed;
} builder;

static int32_t new_node(builder *b, int32_t level, uint32_t first, uint32_t count, int32_t parent)
{
    or_tree *t = b->t;
    if (t->nn >= b->cap) { b->failed = 1; return -1; }
    int32_t id = (int32_t)t->nn++;
    t->level[id] = level;
    t->first[id] = first;
    t->count[id] = count;
    t->parent[id] = parent;
    t->nchild[id] = 0;
    for (int c = 0; c < 8; c++) t->child[8 * id + c] = -1;
    if (parent >= 0) t->child[8 * parent + t->nchild[parent]++] = id;
    return id;
}

/* The cube at `level` holding sorted ranks [first, first+count):
 * a leaf if it holds at most leaf_cap particles or sits at the depth limit;
 * otherwise its particles are split over the 8 sub-cubes of level+1 (the
 * octant digit of a key at level+1 is (key >> (60 - 3 level)) & 7);
 * a cube whose particles all fall in one sub-cube is not kept: the sub-cube
 * takes its place under the same parent. */
static void build_rec(builder *b, int32_t level, uint32_t first, uint32_t count, int32_t parent)
{
    if (b->failed) return;
    const uint64_t *keys = b->t->keys;
    if ((int64_t)count <= b->leaf_cap || level == OR_MAX_LEVEL) {
        new_node(b, level, first, count, parent);
        return;
    }
    uint32_t cfirst[8], ccount[8];
    int nonempty = 0;
    int shift = 60 - 3 * level;
    for (int o = 0; o < 8; o++) { cfirst[o] = 0; ccount[o] = 0; }
    for (uint32_t r = first; r < first + count; r++) {
        int o = (int)((keys[r] >> shift) & 7u);
        if (ccount[o] == 0) { cfirst[o] = r; nonempty++; }
        ccount[o]++;
    }
    if (nonempty == 1) {
        build_rec(b, level + 1, first, count, parent);
        return;
    }
    int32_t id = new_node(b, level, first, count, parent);
    for (int o = 0; o < 8; o++)
        if (ccount[o]) build_rec(b, level + 1, cfirst[o], ccount[o], id);
}

/* ---- upward pass: leaves sum their particles in rank order, internal cubes
 *      sum their children in octant order; com = S / M ---- */
static void upward(or_tree *t)
{
    for (int64_t id = t->nn - 1; id >= 0; id--) {
        double M = 0.0, S[3] = {0.0, 0.0, 0.0};
        if (t->nchild[id] == 0) {
            for (uint32_t r = t->first[id]; r < t->first[id] + t->count[id]; r++) {
                double m = t->smass[r];
                M = M + m;
                for (int d = 0; d < 3; d++) S[d] = S[d] + m * t->spos[3 * r + d];
            }
        } else {
            for (int c = 0; c < t->nchild[id]; c++) {
                int32_t ch = t->child[8 * id + c];
                double Mc = t->M[ch];
                M = M + Mc;
                /* children store S in com until the parent has read it */
                for (int d = 0; d < 3; d++) S[d] = S[d] + t->com[3 * ch + d];
            }
        }
        t->M[id] = M;
        for (int d = 0; d < 3; d++) t->com[3 * id + d] = S[d];   /* S for now */
    }
    for (int64_t id = 0; id < t->nn; id++)
        for (int d = 0; d < 3; d++) t->com[3 * id + d] = t->com[3 * id + d] / t->M[id];
}

/* ---- second moments about the centre of mass, from the particles of each node ---- */
static void second_moments(or_tree *t)
{
    t->S2 = (double *)malloc(sizeof(double) * 6 * (t->nn > 0 ? t->nn : 1));
    for (int64_t id = 0; id < t->nn; id++) {
        const double *c = &t->com[3 * id];
        double S[6] = {0, 0, 0, 0, 0, 0};
        for (uint32_t r = t->first[id]; r < t->first[id] + t->count[id]; r++) {
            double m = t->smass[r];
            double x = t->spos[3 * r] - c[0], y = t->spos[3 * r + 1] - c[1], z = t->spos[3 * r + 2] - c[2];
            S[0] = S[0] + m * x * x;
            S[1] = S[1] + m * y * y;
            S[2] = S[2] + m * z * z;
            S[3] = S[3] + m * x * y;
            S[4] = S[4] + m * x * z;
            S[5] = S[5] + m * y * z;
        }
        memcpy(&t->S2[6 * id], S, sizeof(S));
    }
}

void or_tree_destroy(or_tree *t)
{
    if (!t) return;
    free(t->keys); free(t->perm); free(t->spos); free(t->smass);
    free(t->level); free(t->parent); free(t->nchild); free(t->child);
    free(t->first); free(t->count); free(t->M); free(t->com); free(t->S2);
    free(t);
}

or_tree *or_tree_create(int64_t n, const double *pos, const double *mass, int32_t leaf_cap)
{
    if (n < 1 || leaf_cap < 1) return NULL;
    or_tree *t = (or_tree *)calloc(1, sizeof(or_tree));
    int64_t cap = 2 * n + 1;
    t->n = n;
    uint64_t *ukeys = (uint64_t *)malloc(sizeof(uint64_t) * n);
    t->keys = (uint64_t *)malloc(sizeof(uint64_t) * n);
    t->perm = (uint32_t *)malloc(sizeof(uint32_t) * n);
    t->spos = (double *)malloc(sizeof(double) * 3 * n);
    t->smass = (double *)malloc(sizeof(double) * n);
    t->level = (int32_t *)malloc(sizeof(int32_t) * cap);
    t->parent = (int32_t *)malloc(sizeof(int32_t) * cap);
    t->nchild = (int32_t *)malloc(sizeof(int32_t) * cap);
    t->child = (int32_t *)malloc(sizeof(int32_t) * 8 * cap);
    t->first = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    t->count = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    t->M = (double *)malloc(sizeof(double) * cap);
    t->com = (double *)malloc(sizeof(double) * 3 * cap);

    or_root_cube(n, pos, t->lo, &t->k);
    or_keys(n, pos, t->lo, t->k, ukeys);
    or_order(n, ukeys, t->perm);
    for (int64_t r = 0; r < n; r++) {
        uint32_t i = t->perm[r];
        t->keys[r] = ukeys[i];
        t->smass[r] = mass[i];
        for (int d = 0; d < 3; d++) t->spos[3 * r + d] = pos[3 * i + d];
    }
    free(ukeys);

    builder b = {t, cap, leaf_cap, 0};
    t->nn = 0;
    build_rec(&b, 0, 0, (uint32_t)n, -1);
    if (b.failed) { or_tree_destroy(t); return NULL; }
    upward(t);
    second_moments(t);
    return t;
}

void or_tree_moments(const or_tree *t, double *S6)
{
    memcpy(S6, t->S2, sizeof(double) * 6 * t->nn);
}

int64_t or_tree_nn(const or_tree *t) { return t->nn; }

void or_tree_export(const or_tree *t, double lo[3], int32_t *k, uint64_t *keys, uint32_t *perm,
                    int32_t *level, uint32_t *first, uint32_t *count, int32_t *parent,
                    int32_t *nchild, double *M, double *com)
{
    if (lo) memcpy(lo, t->lo, sizeof(double) * 3);
    if (k) *k = t->k;
    if (keys) memcpy(keys, t->keys, sizeof(uint64_t) * t->n);
    if (perm) memcpy(perm, t->perm, sizeof(uint32_t) * t->n);
    if (level) memcpy(level, t->level, sizeof(int32_t) * t->nn);
    if (first) memcpy(first, t->first, sizeof(uint32_t) * t->nn);
    if (count) memcpy(count, t->count, sizeof(uint32_t) * t->nn);
    if (parent) memcpy(parent, t->parent, sizeof(int32_t) * t->nn);
    if (nchild) memcpy(nchild, t->nchild, sizeof(int32_t) * t->nn);
    if (M) memcpy(M, t->M, sizeof(double) * t->nn);
    if (com) memcpy(com, t->com, sizeof(double) * 3 * t->nn);
}

/* ---- softened Newtonian interaction of body x with a point mass m at y ---- */
static void interact(const double x[3], const double y[3], double m, double eps2, double G,
                     double a[3], double *phi)
{
    double d[3];
    for (int c = 0; c < 3; c++) d[c] = y[c] - x[c];
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    r2 = r2 + eps2;
    if (r2 == 0.0) return;   /* coincident pair without softening: no contribution */
    double rinv = 1.0 / sqrt(r2);
    double w = G * m * rinv * rinv * rinv;
    for (int c = 0; c < 3; c++) a[c] = a[c] + w * d[c];
    *phi = *phi - G * m * rinv;
}

/* ---- quadrupole term of a cube (mass distribution with second moments S about its
 *      centre c) on body x, from the second-order expansion of the same softened
 *      potential:  phi = -G [M / s + A / (2 s^5)],  with d = c - x,  s^2 = |d|^2 + eps^2,
 *      A = 3 d.S.d - s^2 tr S; the acceleration is minus its gradient in x,
 *      a = G [M d / s^3 + 5 A d / (2 s^7) - (3 S.d - tr S d) / s^5].
 *      This adds the second-order part only (the monopole is interact()). ---- */
static void interact_quad(const double x[3], const double c[3], const double S[6], double eps2, double G,
                          double a[3], double *phi)
{
    double d[3];
    for (int k = 0; k < 3; k++) d[k] = c[k] - x[k];
    double s2 = ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) + eps2;
    if (s2 == 0.0) return;
    double Sd[3];
    Sd[0] = (S[0] * d[0] + S[3] * d[1]) + S[4] * d[2];
    Sd[1] = (S[3] * d[0] + S[1] * d[1]) + S[5] * d[2];
    Sd[2] = (S[4] * d[0] + S[5] * d[1]) + S[2] * d[2];
    double dSd = (d[0] * Sd[0] + d[1] * Sd[1]) + d[2] * Sd[2];
    double tr = (S[0] + S[1]) + S[2];
    double A = 3.0 * dSd - s2 * tr;
    double s = sqrt(s2);
    double inv5 = 1.0 / (s2 * s2 * s);
    double inv7 = inv5 / s2;
    for (int k = 0; k < 3; k++) a[k] = a[k] + G * (2.5 * A * inv7 * d[k] - inv5 * (3.0 * Sd[k] - tr * d[k]));
    *phi = *phi - G * 0.5 * A * inv5;
}

#define WALK_STACK 256

/* quantised coordinate of axis a (0 = x, the most significant bit of each triple) */
static uint32_t key_coord(uint64_t key, int a)
{
    uint32_t q = 0;
    for (int b = 0; b < OR_MAX_LEVEL; b++) q |= (uint32_t)((key >> (3 * b + 2 - a)) & 1u) << b;
    return q;
}

double or_open_r2(const or_tree *t, const or_params *p, int32_t id)
{
    const double L = ldexp(1.0, t->k), h = ldexp(1.0, t->k - OR_MAX_LEVEL);
    const int l = t->level[id];
    const double s = ldexp(L, -l);
    if (p->open == OR_OPEN_SIDE) return s * s;
    const uint64_t key = t->keys[t->first[id]];
    const uint32_t w = 1u << (OR_MAX_LEVEL - l);
    const double *c = &t->com[3 * id];
    double e[3];
    for (int a = 0; a < 3; a++) {
        const uint32_t Q = key_coord(key, a) & ~(w - 1u);
        if (p->open == OR_OPEN_BMAX) {
            const double lo = t->lo[a] + (double)Q * h;
            const double hi = t->lo[a] + (double)(Q + w) * h;
            const double u = c[a] - lo, v = hi - c[a];
            e[a] = u > v ? u : v;
        } else {
            const double ctr = t->lo[a] + (double)(2u * Q + w) * (0.5 * h);
            e[a] = c[a] - ctr;
        }
    }
    const double e2 = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
    if (p->open == OR_OPEN_BMAX) return e2;
    const double r = s + p->theta * sqrt(e2);
    return r * r;
}

/* ---- the walk for one body (original index i, position x) ---- */
static void walk_one(const or_tree *t, int64_t i, const double x[3], const or_params *p,
                     double a[3], double *phi, int64_t *nm, int64_t *np, uint64_t *h)
{
    double theta2 = p->theta * p->theta;
    double eps2 = p->eps * p->eps;
    double L = ldexp(1.0, t->k);
    int32_t stack[WALK_STACK];
    int sp = 0;
    a[0] = a[1] = a[2] = 0.0;
    *phi = 0.0;
    *nm = 0; *np = 0; *h = 0;
    stack[sp++] = 0;   /* root */
    while (sp > 0) {
        int32_t id = stack[--sp];
        const double *c = &t->com[3 * id];
        double dx = c[0] - x[0], dy = c[1] - x[1], dz = c[2] - x[2];
        double D2 = (dx * dx + dy * dy) + dz * dz;
        double s = ldexp(L, -t->level[id]);
        double r2 = p->open == OR_OPEN_SIDE ? s * s : or_open_r2(t, p, id);
        if (r2 < theta2 * D2) {
            interact(x, c, t->M[id], eps2, p->G, a, phi);
            if (p->quad) interact_quad(x, c, &t->S2[6 * id], eps2, p->G, a, phi);
            (*nm)++;
            *h += or_mix64((uint64_t)id);
        } else if (t->nchild[id] == 0) {
            for (uint32_t r = t->first[id]; r < t->first[id] + t->count[id]; r++) {
                uint32_t j = t->perm[r];
                if ((int64_t)j == i) continue;
                interact(x, &t->spos[3 * r], t->smass[r], eps2, p->G, a, phi);
                (*np)++;
                *h += or_mix64((uint64_t)t->nn + j);
            }
        } else {
            /* push in descending octant order so they pop ascending */
            for (int cc = t->nchild[id] - 1; cc >= 0; cc--) stack[sp++] = t->child[8 * id + cc];
        }
    }
}

int or_tree_walk(const or_tree *t, const double *pos, const or_params *p, int64_t ntarget,
                 const int64_t *targets, double *acc, double *pot, int64_t *n_mono,
                 int64_t *n_p2p, uint64_t *hash, int nthreads)
{
    if (!t || !p || !(p->theta >= 0.0) || !(p->eps >= 0.0)) return 1;
    if (p->open < OR_OPEN_SIDE || p->open > OR_OPEN_OFFSET) return 1;
    if (!targets) ntarget = t->n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < ntarget; s++) {
        int64_t i = targets ? targets[s] : s;
        double a[3], phi;
        int64_t nm, np;
        uint64_t h;
        walk_one(t, i, &pos[3 * i], p, a, &phi, &nm, &np, &h);
        if (acc) { acc[3 * s] = a[0]; acc[3 * s + 1] = a[1]; acc[3 * s + 2] = a[2]; }
        if (pot) pot[s] = phi;
        if (n_mono) n_mono[s] = nm;
        if (n_p2p) n_p2p[s] = np;
        if (hash) hash[s] = h;
    }
    return 0;
}

/* ---- group-criterion walk: one interaction list per group of key-consecutive bodies ---- */
int or_tree_walk_group_ranges(const or_tree *t, const or_params *p, int64_t ngroups, const int64_t *starts,
                              int64_t ntarget, const int64_t *targets, double *acc, double *pot,
                              int64_t *n_mono, int64_t *n_p2p, uint64_t *hash, int nthreads);
typedef struct { int32_t *id; int64_t n, cap; } id_list;

static void list_push(id_list *l, int32_t v)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 256;
        l->id = (int32_t *)realloc(l->id, sizeof(int32_t) * l->cap);
    }
    l->id[l->n++] = v;
}

/* ---- the groups of the group criterion: largest cubes holding at most cap bodies ----
 * In depth-first preorder the cubes whose parent holds more than cap bodies (or the
 * root) and which hold at most cap bodies partition the key order into consecutive
 * runs; a leaf of more than cap bodies (coincident bodies at the depth limit) is cut
 * into runs of cap. */
int64_t or_tree_group_cubes(const or_tree *t, int32_t cap, int64_t *starts)
{
    if (!t || cap < 1) return -1;
    int64_t ng = 0;
    for (int64_t id = 0; id < t->nn; id++) {
        const uint32_t c = t->count[id];
        const int32_t par = t->parent[id];
        const int top = par < 0 || t->count[par] > (uint32_t)cap;
        if (!top) continue;
        if (c <= (uint32_t)cap) {
            if (starts) starts[ng] = t->first[id];
            ng++;
        } else if (t->nchild[id] == 0) {
            for (uint32_t r = 0; r < c; r += (uint32_t)cap) {
                if (starts) starts[ng] = (int64_t)t->first[id] + r;
                ng++;
            }
        }
    }
    if (starts) starts[ng] = t->n;
    return ng;
}

int or_tree_walk_group(const or_tree *t, const or_params *p, int32_t group, int64_t ntarget,
                       const int64_t *targets, double *acc, double *pot, int64_t *n_mono,
                       int64_t *n_p2p, uint64_t *hash, int nthreads)
{
    if (!t || group < 1) return 1;
    const int64_t ng = (t->n + group - 1) / group;
    int64_t *starts = (int64_t *)malloc(sizeof(int64_t) * (ng + 1));
    for (int64_t g = 0; g < ng; g++) starts[g] = g * group;
    starts[ng] = t->n;
    int rc = or_tree_walk_group_ranges(t, p, ng, starts, ntarget, targets, acc, pot, n_mono, n_p2p, hash,
                                       nthreads);
    free(starts);
    return rc;
}

int or_tree_walk_group_ranges(const or_tree *t, const or_params *p, int64_t ngroups, const int64_t *starts,
                              int64_t ntarget, const int64_t *targets, double *acc, double *pot,
                              int64_t *n_mono, int64_t *n_p2p, uint64_t *hash, int nthreads)
{
    if (!t || !p || ngroups < 1 || !starts || !(p->theta >= 0.0) || !(p->eps >= 0.0)) return 1;
    if (p->open != OR_OPEN_SIDE) return 1;   /* the group test is defined with the side only */
    if (starts[0] != 0 || starts[ngroups] != t->n) return 1;
    for (int64_t g = 0; g < ngroups; g++)
        if (starts[g + 1] <= starts[g]) return 1;
    const int64_t n = t->n;
    double *A = (double *)malloc(sizeof(double) * 3 * n), *P = (double *)malloc(sizeof(double) * n);
    int64_t *NM = (int64_t *)malloc(sizeof(int64_t) * n), *NP = (int64_t *)malloc(sizeof(int64_t) * n);
    uint64_t *H = (uint64_t *)malloc(sizeof(uint64_t) * n);
    const double theta2 = p->theta * p->theta, eps2 = p->eps * p->eps, L = ldexp(1.0, t->k);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < ngroups; g++) {
        const int64_t r0 = starts[g], r1 = starts[g + 1];
        double lo[3], hi[3];
        for (int k = 0; k < 3; k++) lo[k] = hi[k] = t->spos[3 * r0 + k];
        for (int64_t r = r0 + 1; r < r1; r++)
            for (int k = 0; k < 3; k++) {
                double v = t->spos[3 * r + k];
                if (v < lo[k]) lo[k] = v;
                if (v > hi[k]) hi[k] = v;
            }
        /* the group's list, in depth-first order */
        id_list mono = {0, 0, 0}, leaves = {0, 0, 0};
        int32_t stack[WALK_STACK];
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            int32_t id = stack[--sp];
            const double *c = &t->com[3 * id];
            double dd[3];
            for (int k = 0; k < 3; k++) {
                double u = lo[k] - c[k], v = c[k] - hi[k];
                double w = u > v ? u : v;
                dd[k] = w > 0.0 ? w : 0.0;
            }
            double D2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
            double s = ldexp(L, -t->level[id]);
            if (s * s < theta2 * D2) list_push(&mono, id);
            else if (t->nchild[id] == 0) list_push(&leaves, id);
            else for (int cc = t->nchild[id] - 1; cc >= 0; cc--) stack[sp++] = t->child[8 * id + cc];
        }
        for (int64_t r = r0; r < r1; r++) {
            const int64_t i = t->perm[r];
            const double *x = &t->spos[3 * r];
            double a[3] = {0.0, 0.0, 0.0}, phi = 0.0;
            int64_t nm = 0, np = 0;
            uint64_t h = 0;
            for (int64_t q = 0; q < mono.n; q++) {
                int32_t id = mono.id[q];
                interact(x, &t->com[3 * id], t->M[id], eps2, p->G, a, &phi);
                nm++;
                h += or_mix64((uint64_t)id);
            }
            for (int64_t q = 0; q < leaves.n; q++) {
                int32_t id = leaves.id[q];
                for (uint32_t rr = t->first[id]; rr < t->first[id] + t->count[id]; rr++) {
                    uint32_t j = t->perm[rr];
                    if ((int64_t)j == i) continue;
                    interact(x, &t->spos[3 * rr], t->smass[rr], eps2, p->G, a, &phi);
                    np++;
                    h += or_mix64((uint64_t)t->nn + j);
                }
            }
            for (int k = 0; k < 3; k++) A[3 * i + k] = a[k];
            P[i] = phi;
            NM[i] = nm;
            NP[i] = np;
            H[i] = h;
        }
        free(mono.id);
        free(leaves.id);
    }
    if (!targets) ntarget = n;
    for (int64_t s = 0; s < ntarget; s++) {
        int64_t i = targets ? targets[s] : s;
        if (acc) for (int k = 0; k < 3; k++) acc[3 * s + k] = A[3 * i + k];
        if (pot) pot[s] = P[i];
        if (n_mono) n_mono[s] = NM[i];
        if (n_p2p) n_p2p[s] = NP[i];
        if (hash) hash[s] = H[i];
    }
    free(A); free(P); free(NM); free(NP); free(H);
    return 0;
}

int or_forces(int64_t n, const double *pos, const double *mass, const or_params *p,
              int64_t ntarget, const int64_t *targets, double *acc, double *pot,
              int64_t *n_mono, int64_t *n_p2p, uint64_t *hash, int nthreads)
{
    or_tree *t = or_tree_create(n, pos, mass, p->leaf_cap);
    if (!t) return 1;
    int rc = or_tree_walk(t, pos, p, ntarget, targets, acc, pot, n_mono, n_p2p, hash, nthreads);
    or_tree_destroy(t);
    return rc;
}

/* ---- direct summation with Neumaier's compensated sum ---- */
static void neumaier_add(double *sum, double *comp, double v)
{
    double s = *sum + v;
    if (fabs(*sum) >= fabs(v)) *comp += (*sum - s) + v;
    else *comp += (v - s) + *sum;
    *sum = s;
}

int or_direct(int64_t n, const double *pos, const double *mass, double eps, double G,
              int64_t ntarget, const int64_t *targets, double *acc, double *pot, int nthreads)
{
    double eps2 = eps * eps;
    if (!targets) ntarget = n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < ntarget; s++) {
        int64_t i = targets ? targets[s] : s;
        const double *x = &pos[3 * i];
        double sa[3] = {0, 0, 0}, ca[3] = {0, 0, 0}, sp = 0.0, cp = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double d[3];
            for (int c = 0; c < 3; c++) d[c] = pos[3 * j + c] - x[c];
            double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            r2 = r2 + eps2;
            if (r2 == 0.0) continue;
            double rinv = 1.0 / sqrt(r2);
            double w = G * mass[j] * rinv * rinv * rinv;
            for (int c = 0; c < 3; c++) neumaier_add(&sa[c], &ca[c], w * d[c]);
            neumaier_add(&sp, &cp, -G * mass[j] * rinv);
        }
        if (acc) for (int c = 0; c < 3; c++) acc[3 * s + c] = sa[c] + ca[c];
        if (pot) pot[s] = sp + cp;
    }
    return 0;
}

/* ---- kick-drift-kick leapfrog: v += (dt/2) a; x += dt v; a = F(x); v += (dt/2) a ---- */
int or_kdk(int64_t n, double *pos, double *vel, const double *mass, const or_params *p,
           double dt, int32_t nsteps, double *acc, int32_t have_acc, double *pot, int nthreads)
{
    double h = 0.5 * dt;
    if (!have_acc && or_forces(n, pos, mass, p, n, NULL, acc, pot, NULL, NULL, NULL, nthreads))
        return 1;
    for (int32_t s = 0; s < nsteps; s++) {
        for (int64_t i = 0; i < 3 * n; i++) vel[i] = vel[i] + h * acc[i];
        for (int64_t i = 0; i < 3 * n; i++) pos[i] = pos[i] + dt * vel[i];
        if (or_forces(n, pos, mass, p, n, NULL, acc, pot, NULL, NULL, NULL, nthreads)) return 1;
        for (int64_t i = 0; i < 3 * n; i++) vel[i] = vel[i] + h * acc[i];
    }
    return 0;
}

void or_energy(int64_t n, const double *vel, const double *mass, const double *pot, double out_KW[2])
{
    double K = 0.0, W = 0.0;
    for (int64_t i = 0; i < n; i++) {
        const double *v = &vel[3 * i];
        K = K + mass[i] * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
        if (pot) W = W + mass[i] * pot[i];
    }
    out_KW[0] = 0.5 * K;
    out_KW[1] = 0.5 * W;
}
