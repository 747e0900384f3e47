/*
 * Barnes-Hut reference oracle: plain, slow, FP64, single-source C.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links
 * or loads this code; only the tests, the package smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the GPU
 * path.
 *
 * What it computes (paper: "Improving the scalability of parallel N-body
 * applications with an event driven constraint based execution model"):
 *  - the cube hierarchy built by recursive subdivision until a cube holds
 *    at most `leaf_cap` particles (section 1, introduction; Fig. 2 caption),
 *    with the root cube, Morton keys and depth limit as stated in each
 *    function below;
 *  - the centre of mass of every cube (section 1);
 *  - the force on every body, treating a cube as one body only when its
 *    distance D from the body exceeds r/theta (section 3, first paragraph,
 *    Fig. 1), with r the cube side and D measured to the centre of mass;
 *  - plain O(N^2) direct summation, which the walk reduces to at theta = 0;
 *  - kick-drift-kick leapfrog iterations and energy diagnostics.
 * Readings of points the paper leaves open are listed beside each function.
 *
 * Arithmetic: IEEE double, round to nearest, built with -ffp-contract=off
 * so that no multiply-add is fused.
 */
#ifndef BH_ORACLE_H
#define BH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_LEVEL 21   /* 3 x 21 = 63-bit keys */

typedef struct {
    double theta, eps, G;
    int32_t leaf_cap;
    int32_t quad;           /* 1: accepted cubes add their quadrupole term (see or_tree_moments) */
    int32_t open;           /* opening radius r of the test r^2 < theta^2 D^2: OR_OPEN_* */
} or_params;

/* Alternative ways of computing the opening criterion (section 6 lists them as
 * future work).  The test stays r*r < (theta*theta) * D2 with D2 as in the walk:
 *   OR_OPEN_SIDE   r = the cube side s (the paper's reading, the default);
 *   OR_OPEN_BMAX   r = the largest distance from the centre of mass to a corner
 *                  of the cube (Salmon and Warren's b_max);
 *   OR_OPEN_OFFSET accept iff D > s/theta + delta, delta the distance from the
 *                  centre of mass to the cube's geometric centre (Barnes 1994),
 *                  i.e. r = s + theta delta. */
#define OR_OPEN_SIDE 0
#define OR_OPEN_BMAX 1
#define OR_OPEN_OFFSET 2

typedef struct {
    int64_t n, nn;          /* particles, tree nodes */
    double lo[3];           /* root cube minimum corner */
    int32_t k;              /* root cube side L = 2^k */
    uint64_t *keys;         /* n, sorted ascending */
    uint32_t *perm;         /* n, perm[r] = original index of rank r */
    double *spos, *smass;   /* sorted copies of positions (n x 3) and masses */
    /* nodes in depth-first preorder, children in ascending octant order */
    int32_t *level, *parent, *nchild, *child; /* child: nn x 8, -1 padded */
    uint32_t *first, *count;
    double *M, *com;        /* node mass and centre of mass (nn x 3) */
    double *S2;             /* second moment about the centre of mass (nn x 6: xx yy zz xy xz yz) */
} or_tree;

/* root cube (c-1) and keys (c-2) */
void or_root_cube(int64_t n, const double *pos, double lo[3], int32_t *k);
uint64_t or_interleave(uint32_t qx, uint32_t qy, uint32_t qz);
void or_keys(int64_t n, const double *pos, const double lo[3], int32_t k, uint64_t *keys);
/* stable order by (key, original index) */
void or_order(int64_t n, const uint64_t *keys, uint32_t *perm);

/* full tree: keys, order, compressed octree, upward pass.  NULL on error. */
or_tree *or_tree_create(int64_t n, const double *pos, const double *mass, int32_t leaf_cap);
void or_tree_destroy(or_tree *t);
int64_t or_tree_nn(const or_tree *t);
void or_tree_export(const or_tree *t, double lo[3], int32_t *k, uint64_t *keys, uint32_t *perm,
                    int32_t *level, uint32_t *first, uint32_t *count, int32_t *parent,
                    int32_t *nchild, double *M, double *com);

/* Second moments about each node's centre of mass, by their definition
 * S_ab = sum over the node's particles of m (x_a - c_a)(x_b - c_b), summed in rank
 * order (nn x 6: xx yy zz xy xz yz).  They carry the quadrupole of the cube's mass
 * distribution: the paper names multipole moments as future work (section 6). */
void or_tree_moments(const or_tree *t, double *S6);

/* r^2 of node id under p->open, in FP64.  Cube geometry of a level-l node: with
 * (qx, qy, qz) the quantised coordinates of its first key, low 21 - l bits
 * cleared (Q), h = L 2^-21 and w = 2^(21-l): corner lo = fl(root_lo + Q h),
 * far corner hi = fl(root_lo + (Q + w) h), centre fl(root_lo + (2Q + w) h/2),
 * each a single rounding of an exact product.  b_max: e = max(c - lo, hi - c)
 * per axis, r^2 = (ex*ex + ey*ey) + ez*ez.  Offset: d = c - centre per axis,
 * delta = sqrt((dx*dx + dy*dy) + dz*dz), r = s + theta*delta, r^2 = r*r.
 * Side: r^2 = s*s. */
double or_open_r2(const or_tree *t, const or_params *p, int32_t id);

/* walk for the given targets (original indices; NULL = all n in index order).
 * Outputs are indexed by target slot.  Any output may be NULL. */
int or_tree_walk(const or_tree *t, const double *pos, const or_params *p, int64_t ntarget,
                 const int64_t *targets, double *acc, double *pot, int64_t *n_mono,
                 int64_t *n_p2p, uint64_t *hash, int nthreads);

/* Group-criterion walk (a variant, not the paper's per-body test) over fixed-size
 * groups: the bodies in key order are split into consecutive groups of `group` (the
 * last one shorter); the library's groups are the cube groups of or_tree_group_cubes,
 * walked by or_tree_walk_group_ranges;
 * a cube is accepted for a whole group iff side^2 < theta^2 D^2 with D the distance
 * from the cube's centre of mass to the group's bounding box (0 inside it), in
 * FP64 as ((dx*dx + dy*dy) + dz*dz) with dk = max(0, lo_k - c_k, c_k - hi_k).
 * Every member then takes the same cubes; opened leaves give pairs with every
 * particle but itself.  With group = 1 this is the per-body walk. */
int or_tree_walk_group(const or_tree *t, const or_params *p, int32_t group, int64_t ntarget,
                       const int64_t *targets, double *acc, double *pot, int64_t *n_mono,
                       int64_t *n_p2p, uint64_t *hash, int nthreads);

/* The same walk over explicit groups: group g holds the bodies of sorted ranks
 * [starts[g], starts[g + 1]), starts[0] = 0, starts[ngroups] = n, increasing. */
int or_tree_walk_group_ranges(const or_tree *t, const or_params *p, int64_t ngroups, const int64_t *starts,
                              int64_t ntarget, const int64_t *targets, double *acc, double *pot,
                              int64_t *n_mono, int64_t *n_p2p, uint64_t *hash, int nthreads);

/* Groups of the cube-based group criterion: the largest cubes holding at most cap
 * bodies, in key order (a leaf of more than cap bodies is cut into runs of cap).
 * Writes starts[0..ng] (nullable: count only) and returns ng (-1 on bad input). */
int64_t or_tree_group_cubes(const or_tree *t, int32_t cap, int64_t *starts);

/* build + walk in one call */
int or_forces(int64_t n, const double *pos, const double *mass, const or_params *p,
              int64_t ntarget, const int64_t *targets, double *acc, double *pot,
              int64_t *n_mono, int64_t *n_p2p, uint64_t *hash, int nthreads);

/* O(N^2) direct sum for the given targets, Neumaier-compensated */
int or_direct(int64_t n, const double *pos, const double *mass, double eps, double G,
              int64_t ntarget, const int64_t *targets, double *acc, double *pot, int nthreads);

/* kick-drift-kick leapfrog: `acc` holds a(x) on entry if have_acc != 0, else it is
 * computed first; pot (nullable) receives the potential at the final positions. */
int or_kdk(int64_t n, double *pos, double *vel, const double *mass, const or_params *p,
           double dt, int32_t nsteps, double *acc, int32_t have_acc, double *pot, int nthreads);

/* K = 1/2 sum m v^2, W = 1/2 sum m phi */
void or_energy(int64_t n, const double *vel, const double *mass, const double *pot, double out_KW[2]);

/* interaction-set checksum mixer (SplitMix64 finalizer of x + 0x9e3779b97f4a7c15) */
uint64_t or_mix64(uint64_t x);

#ifdef __cplusplus
}
#endif
#endif
