/*
 * bh.h -- C ABI of the MI355X Barnes-Hut library (libbh.so).
 *
 * The library computes, on one AMD Instinct MI355X (gfx950), the hot path of
 * the Barnes-Hut N-body method as described in "Improving the scalability of
 * parallel N-body applications with an event driven constraint based
 * execution model" (Dekate et al.):
 *   - the cube hierarchy: recursive subdivision of a root cube until a cube
 *     holds at most `leaf_cap` particles (section 1, introduction; Fig. 2);
 *   - the centre of mass of every cube (section 1);
 *   - the force on every body, where a cube is treated as one body only when
 *     its distance D from the body exceeds r/theta (section 3, first
 *     paragraph and Fig. 1), with r the cube side and D the distance to the
 *     cube's centre of mass; the test is strict and evaluated per body;
 *   - iterations: a new tree every step (section 1, load-balancing item;
 *     section 3, global barrier at tree construction), advanced with
 *     kick-drift-kick leapfrog.
 * Readings of points the paper leaves open (root cube, depth limit 21,
 * removal of single-child cubes, Plummer softening, self-exclusion) are the
 * same as in the oracle and are listed in the repository's design notes.
 *
 * Conventions for every entry point:
 *  - Return value: bh_status.  No exception or abort crosses the ABI.  On an
 *    error, bh_last_error() returns a thread-local message, valid until the
 *    next call on the same thread.
 *  - Memory: the CALLER owns all device memory: inputs, outputs, workspaces
 *    and the server arena.  The library sub-allocates inside the workspace it
 *    is given and never frees caller memory.  Handles (bh_ctx, bh_tree,
 *    bh_sim, bh_forest, bh_server) are small host objects.  A tree,
 *    simulation or forest belongs to the context it was created on: calls
 *    that pass another context are refused (BH_E_INVAL), and so are calls on
 *    a handle whose context was destroyed (only its free/destroy is allowed).
 *  - Ordering: calls are asynchronous on the context's HIP stream; a call
 *    returns once its work is enqueued.  Outputs are valid after the stream
 *    is synchronised (bh_ctx_sync).  Calls marked SYNC synchronise the stream
 *    themselves.
 *  - Device faults: kernels record faults (walk stack overflow, an
 *    inconsistent tree, a non-finite position or mass) in a fault word of the
 *    tree, simulation or forest they run for.  The next SYNC call on that
 *    object, or bh_ctx_sync, reports them (BH_E_OVERFLOW or BH_E_DEVICE) and
 *    clears them, so later calls start clean.  A tree found inconsistent is
 *    not walked (its outputs keep their contents) until it is rebuilt.
 *  - Layouts: positions, velocities and accelerations are row-major (n, 3)
 *    FP64 arrays in device memory in the caller's particle order; masses are
 *    (n,) FP64.  Results come back in the caller's order.
 *  - Sizes: 1 <= n <= 2^30 - 1 per call (per forest: the sum).
 */
#ifndef BH_H
#define BH_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BH_OK = 0,
    BH_E_INVAL = 1,      /* bad argument (null pointer, n < 1, theta < 0, eps < 0, leaf_cap not in [1,64], non-finite) */
    BH_E_NOMEM = 2,      /* workspace / arena too small, or a request that can never fit */
    BH_E_DEVICE = 3,     /* HIP error, or a device-side fault flag (non-finite position or mass) */
    BH_E_BUSY = 4,       /* request not finished yet */
    BH_E_NOTFOUND = 5,   /* unknown request id */
    BH_E_OVERFLOW = 6,   /* walk stack overflow (cannot happen for depth <= 21; reported if it does) */
    BH_E_CANCELLED = 7,  /* request was cancelled */
    BH_E_IO = 8          /* a tuning-cache file could not be read, parsed or written */
} bh_status;

typedef enum { BH_FP64 = 0, BH_FP32 = 1 } bh_precision;

/* Method parameters.
 *  theta     opening parameter (>= 0); theta = 0 reduces the walk to direct summation.
 *  eps       Plummer softening length (>= 0): pair kernel G m d / (|d|^2 + eps^2)^(3/2).
 *  G         gravitational constant.
 *  leaf_cap  a cube holding at most leaf_cap particles is a leaf (the paper uses 1); 1..64.
 *  precision BH_FP64: all walk arithmetic in FP64.
 *            BH_FP32: pair/monopole arithmetic in FP32 with compensated accumulation;
 *            opening decisions are certified against the FP64 test (re-evaluated in
 *            FP64 when the FP32 value is within its rounding bound of the threshold),
 *            so the interaction sets are those of the FP64 method.
 *  flags     bit set of
 *            BH_QUADRUPOLE: an accepted cube adds its quadrupole term, the second-order
 *              term of the same softened potential about its centre of mass (second
 *              moments S about the centre; with d = com - x, s^2 = |d|^2 + eps^2,
 *              A = 3 d.S.d - s^2 tr S: phi += -G A / (2 s^5), a += G [5 A d / (2 s^7)
 *              - (3 S.d - tr S d) / s^5]).  The paper names multipole moments as future
 *              work (section 6).  Interaction sets are unchanged.
 *            BH_GROUP_CRITERION: a variant of the opening test (not the paper's): the
 *              bodies of a group share one decision per cube, accepted iff
 *              side^2 < theta^2 D^2 with D the distance from the cube's centre of mass
 *              to the group's bounding box (FP64, as the per-body test); opened leaves
 *              give pairs with every particle but the body itself.  A body's group is
 *              the largest cube of the tree holding at most 64 bodies (a leaf of more
 *              than 64 coincident bodies is cut into runs of 64 in key order), so a
 *              group never spans cubes that a larger cube separates.  More
 *              conservative (and more accurate) than the per-body test.  Not combined
 *              with BH_QUADRUPOLE.
 *            BH_OPEN_BMAX: alternative opening radius (section 6 names other ways of
 *              computing the criterion as future work): accept iff r^2 < theta^2 D^2
 *              with r = b_max, the largest distance from the cube's centre of mass to
 *              a corner of the cube, in FP64 as ((ex*ex + ey*ey) + ez*ez) with
 *              e = max(c - lo, hi - c) per axis.  For theta < 1 no cube holding the
 *              body is ever accepted.
 *            BH_OPEN_OFFSET: accept iff D > side/theta + delta, delta the distance
 *              from the centre of mass to the cube's centre, i.e. r = side + theta
 *              delta in the same test.  Cube corners and centres are
 *              root_lo + (integer) * 2^(k-21) from the node's key, one rounding each.
 *              BH_OPEN_BMAX and BH_OPEN_OFFSET exclude each other and
 *              BH_GROUP_CRITERION.
 *            BH_REQ_RELEASE (server requests only): free the request's state when it
 *              completes (its energies stay available; bh_server_fetch is then refused).
 *            Other bits are rejected (BH_E_INVAL). */
#define BH_REQ_RELEASE 1u
#define BH_QUADRUPOLE 2u
#define BH_GROUP_CRITERION 4u
#define BH_OPEN_BMAX 8u
#define BH_OPEN_OFFSET 16u
typedef struct {
    double theta, eps, G;
    int32_t leaf_cap;
    int32_t precision;
    uint32_t flags;
    uint32_t reserved;
} bh_params;

/* Interaction totals of one force evaluation (filled by the *_stats calls, SYNC). */
typedef struct {
    uint64_t n_mono;      /* accepted cubes (monopole interactions) summed over bodies */
    uint64_t n_p2p;       /* body-body interactions in opened leaves, self excluded */
    uint64_t n_visits;    /* (cube, body) opening tests */
    uint64_t n_fallback;  /* FP32 opening tests re-evaluated in FP64 */
    /* wavefront-level diagnostics (FP32 mode; 0 in FP64 mode): cube visits, popped
     * stack entries, visits where at least one lane accepted, opened leaves */
    uint64_t wave_visits, wave_entries, wave_accepts, wave_leaves;
    double t_ms;          /* the walk's duration on the stream (HIP events around its launch) */
} bh_stats;

typedef struct bh_ctx bh_ctx;
typedef struct bh_tree bh_tree;
typedef struct bh_sim bh_sim;
typedef struct bh_forest bh_forest;
typedef struct bh_server bh_server;

/* ---------------------------------------------------------------- context --- */

/* Context bound to HIP device `device` and stream `hip_stream` (a hipStream_t,
 * NULL = the null stream).  The stream is not owned. */
bh_status bh_ctx_create(int device, void *hip_stream, bh_ctx **out);
bh_status bh_ctx_destroy(bh_ctx *ctx);
/* SYNC: waits for the stream, then reports (and clears) the fault flags of
 * the context's live trees, simulations and forests, the first found. */
bh_status bh_ctx_sync(bh_ctx *ctx);
const char *bh_last_error(void);
/* Library version string, e.g. "bh-mi355x 0.1". */
const char *bh_version(void);

/* ------------------------------------------------------------ single tree --- */

/* Bytes of device workspace needed by bh_build for n particles. */
size_t bh_workspace_bytes(int64_t n, const bh_params *p);

/* Octree construction (paper section 1; Fig. 2): root cube, 63-bit Morton
 * keys, stable radix sort, canonical compressed octree.  pos (n x 3) and
 * mass (n) are device pointers that must stay valid and unchanged until the
 * tree is freed.  ws: device workspace of ws_bytes >= bh_workspace_bytes.
 * *out receives a host handle. */
bh_status bh_build(bh_ctx *ctx, int64_t n, const double *pos, const double *mass,
                   const bh_params *p, void *ws, size_t ws_bytes, bh_tree **out);

/* Octree construction again, in the tree's own workspace, from new positions
 * and masses of the same n particles (same parameters): what bh_build does
 * after its one-time set-up (parameter upload and workspace layout), for a
 * caller that rebuilds every iteration (section 1: the tree is rebuilt each
 * time step).  pos and mass replace the tree's inputs under bh_build's
 * conditions; bh_upward must run again before bh_forces.  Asynchronous. */
bh_status bh_rebuild(bh_ctx *ctx, bh_tree *tree, const double *pos, const double *mass);

/* Upward pass (section 1: centre of mass of each cube): FP64 mass and centre
 * of mass of every node, summed in a fixed order (particles in key order at
 * leaves, children in octant order above), and the walk records. */
bh_status bh_upward(bh_ctx *ctx, bh_tree *tree);

/* Force walk (section 3: opening criterion; force stage): acc (n x 3 FP64,
 * device, caller's order) receives G * sum m d / (|d|^2+eps^2)^(3/2) over the
 * accepted cubes and the leaf pairs; pot (nullable, n FP64 device) the
 * potential -G sum m / sqrt(|d|^2+eps^2) over the same set. */
bh_status bh_forces(bh_ctx *ctx, bh_tree *tree, double *acc, double *pot);

/* As bh_forces, plus per-body interaction counts and set checksum (device
 * arrays of n, caller's order; each nullable) and the totals (SYNC).  The
 * checksum of body i is the sum mod 2^64 of mix64(node) over accepted cubes
 * and mix64(n_nodes + j) over pair partners j, with node the preorder index
 * and mix64 the SplitMix64 finalizer of x + 0x9e3779b97f4a7c15. */
bh_status bh_forces_stats(bh_ctx *ctx, bh_tree *tree, double *acc, double *pot, int64_t *n_mono,
                          int64_t *n_p2p, uint64_t *hash, bh_stats *totals);

/* ------------------------------------------------- one GPU's target share --- */

/* bh_forces for the bodies of sorted (Morton) ranks [first, first + count)
 * only: one GPU's share when the targets of one simulation are split across
 * GPUs that each hold the whole tree.  The rows of those bodies in acc (and
 * pot, n_mono, n_p2p, work when given; caller's order, as bh_forces and
 * bh_forces_stats write them) receive bh_forces's values bit for bit; every
 * other row is left as it was.  n_mono, n_p2p, work (device, n int64 each)
 * and group_work (device, ceil(n / 64) int64), each nullable, request the
 * counting walk: interaction counts as bh_forces_stats gives them; group_work,
 * the wavefront work W of each 64-body walk group (group g: sorted ranks
 * [64 g, min(64 g + 64, n))), the children tested plus the pair iterations of
 * the group's shared traversal, written for every group that meets the range;
 * work, that W spread evenly over the group's bodies (body k of c gets
 * floor(W (k+1) / c) - floor(W k / c), so a group's rows sum to its W).  They
 * feed bh_shard_bounds and bh_shard_bounds_groups.  The walk runs the 64-body
 * groups that meet the range (section 3: force stage), so a range costs its
 * share of the walk plus at most two partial groups.  Sorted rank r is body
 * perm[r] of bh_tree_export.  0 <= first, 0 <= count, first + count <= n,
 * else BH_E_INVAL; count == 0 does nothing.  Asynchronous. */
bh_status bh_forces_range(bh_ctx *ctx, bh_tree *tree, int64_t first, int64_t count, double *acc, double *pot,
                          int64_t *n_mono, int64_t *n_p2p, int64_t *work, int64_t *group_work);

/* Split of the tree's n bodies into G Morton-contiguous target ranges of equal
 * cost (section 1 names the per-particle work, which varies and changes with
 * every rebuilt tree, as what defeats static splits; this is the cost-zone
 * method of Singh et al., 1995).  Body i costs 1 + cost_a[i] + cost_b[i]
 * (device, n int64 each, caller's order, from a counting walk of a previous
 * step: n_mono and n_p2p, or work and NULL; a null array contributes 0, both
 * null give equal counts).  With P(r) the summed cost of the bodies of sorted
 * ranks below r and T = P(n), bounds (device, G + 1 int64) receives, for
 * j = 0..G, the smallest r with G P(r) >= j T: range j is
 * [bounds[j], bounds[j + 1]), bounds[0] = 0, bounds[G] = n.  Uses the tree's
 * build scratch (the tree stays valid); 1 <= G <= 65536, else BH_E_INVAL.
 * Asynchronous. */
bh_status bh_shard_bounds(bh_ctx *ctx, bh_tree *tree, const int64_t *cost_a, const int64_t *cost_b, int32_t G,
                          int64_t *bounds);

/* The same split over the 64-body walk groups, so that every range starts on a
 * group boundary and no group is walked by two ranges.  Group g costs its body
 * count plus group_work[g] (device, ceil(n / 64) int64, rank order, from a
 * counting walk); with P(m) the summed cost of groups below m and T the
 * total, bounds[j] (device, G + 1 int64) = min(64 x, n) for the smallest x
 * with G P(x) >= j T.  The costs are read contiguously (1/64 of the data of
 * bh_shard_bounds, none of it gathered).  Same scratch, limits and errors as
 * bh_shard_bounds.  Asynchronous. */
bh_status bh_shard_bounds_groups(bh_ctx *ctx, bh_tree *tree, const int64_t *group_work, int32_t G, int64_t *bounds);

/* ------------------------------------------------------ interaction lists --- */

/* Two-phase force stage, the paper's own structure (section 3: each body's
 * interaction list of cubes and bodies is formed, flattened, then evaluated).
 * Phase one, bh_lists_build, walks the tree with bh_forces's decisions and
 * writes the lists into a caller buffer; phase two, bh_lists_forces, evaluates
 * them and gives bh_forces's acc and pot bit for bit.  Trees with the
 * per-body test (any opening radius, either precision, with or without the
 * quadrupole) only; BH_GROUP_CRITERION trees give BH_E_INVAL.
 *
 * Lists are kept per walk group: group g holds the bodies of sorted ranks
 * [64 g, min(64 g + 64, n)); bit k of a mask is the group's k-th body.
 * Entry (a, b, mask), in walk order:
 *   a == 0xffffffff        start of a stack entry with b children (it times
 *                          the compensated-sum folds; FP32 lists only);
 *   b & 0x80000000         an opened leaf: particles of sorted ranks
 *                          [a, a + (b & 0x7fffffff)), paired with the bodies
 *                          in mask (not with themselves);
 *   otherwise              an accepted cube: walk slot a, node b (global
 *                          preorder id), for the bodies in mask.
 * Buffer layout (device memory, 256-byte aligned, `bytes` long; G groups and
 * C chunks of 64 entries, C the largest count that fits):
 *   byte 256 k (k < 256):   uint64, chunks the last build reserved from
 *                           partition k (chunk ids k, k + 256, k + 512, ...:
 *                           group g takes its chunks from partition g mod 256,
 *                           4 at a time; reserved chunks may stay unused);
 *   byte 65536:             uint32 head[G], first chunk of each group;
 *   next 256-byte boundary: uint32 count[G], entries of each group;
 *   next 256-byte boundary: uint32 next[C], the group's next chunk
 *                           (0xffffffff: last);
 *   next 256-byte boundary: bh_list_entry entries[64 C].
 * The lists stay owned by the caller and valid until the tree is rebuilt or
 * its upward pass runs again. */
typedef struct {
    uint32_t a, b;
    uint64_t mask;
} bh_list_entry;

/* Phase one.  SYNC.  *bytes_needed (nullable) receives the buffer size these
 * lists need; when it exceeds `bytes` the call returns BH_E_NOMEM and the
 * buffer holds no usable lists (call again with a buffer of that size).  If
 * `bytes` cannot even hold the counters and group tables, nothing runs and
 * *bytes_needed is only a lower bound. */
bh_status bh_lists_build(bh_ctx *ctx, bh_tree *tree, void *buf, size_t bytes, size_t *bytes_needed);

/* Phase two over the lists the last successful bh_lists_build of this tree
 * wrote into buf: acc (n x 3) and pot (nullable) as bh_forces.  Asynchronous. */
bh_status bh_lists_forces(bh_ctx *ctx, bh_tree *tree, const void *buf, double *acc, double *pot);

/* SYNC.  Number of tree nodes and the root cube (lo[3] host, k: side 2^k). */
bh_status bh_tree_info(bh_ctx *ctx, bh_tree *tree, int64_t *n_nodes, double lo[3], int32_t *k);

/* Canonical export (device pointers, each nullable): sorted keys (n), order
 * perm (n, perm[r] = original index of rank r), and per node in depth-first
 * preorder with children in ascending octant order: level, first rank, count,
 * parent (-1 for the root), mass M and centre of mass com (n_nodes x 3).
 * Node arrays must hold bh_tree_info's n_nodes entries.
 * n_nodes (host, nullable) receives the node count.  isect_hash (device, n,
 * caller's order, nullable) receives each body's interaction-set checksum as
 * bh_forces_stats defines it (section 3: each body's list of accepted cubes
 * and partner bodies), from a counting walk that writes nothing else.
 * SYNC when n_nodes or isect_hash is given, else asynchronous.  M, com and
 * isect_hash need bh_upward first (BH_E_INVAL otherwise). */
bh_status bh_tree_export(bh_ctx *ctx, bh_tree *tree, uint64_t *keys, uint32_t *perm, int32_t *level,
                         uint32_t *first, uint32_t *count, int32_t *parent, double *M, double *com,
                         int64_t *n_nodes, uint64_t *isect_hash);

bh_status bh_tree_free(bh_ctx *ctx, bh_tree *tree);

/* -------------------------------------------------------------- simulation --- */

/* A simulation views caller memory: pos, vel, acc (n x 3) are updated in place,
 * mass (n) is read.  acc is computed by the first bh_step. */
size_t bh_sim_workspace_bytes(int64_t n, const bh_params *p);
bh_status bh_sim_create(bh_ctx *ctx, int64_t n, double *pos, double *vel, const double *mass, double *acc,
                        const bh_params *p, void *ws, size_t ws_bytes, bh_sim **out);
/* nsteps kick-drift-kick steps with a full tree rebuild each step:
 * v += (dt/2) a; x += dt v; rebuild, upward, walk; v += (dt/2) a. */
bh_status bh_step(bh_ctx *ctx, bh_sim *sim, int32_t nsteps, double dt);
/* SYNC.  out_KW = {K, W}: K = 1/2 sum m |v|^2, W = 1/2 sum m phi, phi from a
 * walk at the current positions (FP64 reductions). */
bh_status bh_energy(bh_ctx *ctx, bh_sim *sim, double out_KW[2]);
bh_status bh_sim_destroy(bh_ctx *ctx, bh_sim *sim);

/* ------------------------------------------------------------------ forest --- */

/* Many independent simulations advanced together: their particles are
 * concatenated (simulation s owns rows [off_s, off_s + n[s]) of pos, vel,
 * acc and mass, off_s = n[0] + ... + n[s-1]); every kernel of a step covers
 * all of them in one launch. */
size_t bh_forest_workspace_bytes(int32_t n_sims, const int64_t *n, const bh_params *per_sim);
bh_status bh_forest_create(bh_ctx *ctx, int32_t n_sims, const int64_t *n, const bh_params *per_sim,
                           double *pos, double *vel, const double *mass, double *acc, void *ws,
                           size_t ws_bytes, bh_forest **out);
/* dt: host array of n_sims time steps. */
bh_status bh_forest_step(bh_ctx *ctx, bh_forest *f, int32_t nsteps, const double *dt);
/* Forces at the current positions into acc (and pot, nullable, concatenated). */
bh_status bh_forest_forces(bh_ctx *ctx, bh_forest *f, double *pot);
/* Record one step of the forest as a HIP graph (on first call) and replay it
 * nsteps times. */
bh_status bh_forest_step_graph(bh_ctx *ctx, bh_forest *f, int32_t nsteps, const double *dt);
/* Walk launch shapes (the load-balancing analogue of the paper's work queues and
 * grain size, sections 3 and 5).  A shape is the number of wavefronts per
 * workgroup, 1, 2, 4 or 8 (each wavefront walks one 64-body group at a time),
 * optionally or'ed with BH_WALK_PERSISTENT: then the launch has only as many
 * workgroups as the device holds at once and each wavefront takes the next group
 * from a counter in the workspace until none is left.  The shape changes no
 * result; it decides how the uneven per-group work meets the compute units.
 * Trees, simulations and forests start with shape 4. */
#define BH_WALK_PERSISTENT 0x100
#define BH_TUNE_SHAPES 8   /* 1, 2, 4, 8, then 1, 2, 4, 8 | BH_WALK_PERSISTENT */
bh_status bh_tree_set_walk_shape(bh_ctx *ctx, bh_tree *tree, int32_t shape);
bh_status bh_sim_set_walk_shape(bh_ctx *ctx, bh_sim *sim, int32_t shape);
/* A recorded step graph is re-recorded at its next replay when the shape changes. */
bh_status bh_forest_set_walk_shape(bh_ctx *ctx, bh_forest *f, int32_t shape);
/* SYNC.  Autotuner of the forest's walk launch shape: builds the tree at the
 * current positions and times the force walk (two launches after a warm-up, HIP
 * events on the context's stream) in each of the BH_TUNE_SHAPES shapes, keeps the
 * fastest for this forest's later evaluations (a recorded step graph is
 * re-recorded) and stores it in the process's tuning cache under the forest's key:
 * device (architecture and compute units), floor(log2 total bodies),
 * floor(log2 simulations), theta (body-weighted mean, to 0.01) and precision mix.
 * flags: BH_TUNE_CACHED takes the cached shape for that key without timing when
 * there is one.  shape_out (nullable): the chosen shape; ms_out (nullable, host
 * array of BH_TUNE_SHAPES): measured walk times in ms in the order above, all -1
 * when the shape came from the cache.  acc is refreshed as a side effect (forces
 * at the current positions).  With the environment variable BH_TUNE_CACHE naming
 * a file, the first autotuner call of the process merges that file into the cache
 * (a missing file is an empty cache) and every timed call writes the cache back. */
#define BH_TUNE_CACHED 1u
bh_status bh_forest_autotune(bh_ctx *ctx, bh_forest *f, uint32_t flags, int32_t *shape_out, double *ms_out);
/* The process's tuning cache as JSON text:
 *   {"format": "bh-tune-cache", "version": 1, "entries": [{"device": "gfx950:256",
 *    "n_log2": 20, "sims_log2": 0, "theta": 0.5, "precision": "fp32", "shape": 4,
 *    "ms": 2.77}, ...]}
 * load merges a file's entries (equal keys replaced; all or nothing: BH_E_IO with
 * the reason in bh_last_error on a missing file or any syntax or schema error);
 * save writes every entry (BH_E_IO when the file cannot be written); clear empties
 * the cache.  Thread-safe; the cache is shared by all contexts of the process. */
bh_status bh_tune_cache_load(const char *path);
bh_status bh_tune_cache_save(const char *path);
bh_status bh_tune_cache_clear(void);
/* Number of entries in the tuning cache. */
int64_t bh_tune_cache_size(void);
/* SYNC.  Per-simulation energies at the current positions: out_KW[2 s] = K_s,
 * out_KW[2 s + 1] = W_s (host array of 2 n_sims); also refreshes acc. */
bh_status bh_forest_energy(bh_ctx *ctx, bh_forest *f, double *out_KW);
bh_status bh_forest_destroy(bh_ctx *ctx, bh_forest *f);

/* ----------------------------------------------------- initial conditions --- */

/* Bytes of device workspace bh_ic_generate needs (independent of n: the
 * generator's per-block partial sums and its fault word). */
size_t bh_ic_workspace_bytes(void);

/* Device-side generation of the same inputs as the host generator: Philox4x32-10
 * keyed by seed, counter (i_lo, i_hi, call, tag).  kind 0: Plummer sphere by
 * Aarseth-Henon-Wielen with scale radius a, total mass M, mass-fraction cut
 * 0.999, shifted to its centre-of-mass frame; kind 1: uniform cube [-a, a]^3,
 * masses uniform in [0.5, 1.5] M / n, at rest.  pos, vel (n x 3), mass (n):
 * device outputs.  ws: caller-owned device workspace, 256-byte aligned, of
 * ws_bytes >= bh_ic_workspace_bytes() (BH_E_NOMEM otherwise).  SYNC: returns
 * BH_E_DEVICE if a velocity draw found no acceptance (the Plummer sampler
 * gives up after 401 rejection rounds and leaves the velocities non-finite;
 * never seen in practice). */
bh_status bh_ic_generate(bh_ctx *ctx, int32_t kind, int64_t n, uint64_t seed, double a, double M,
                         double *pos, double *vel, double *mass, void *ws, size_t ws_bytes);

/* bh_ic_generate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and results bit for bit, with the generator's partial sums
 * and fault word in a static array of the library (16 KiB per GPU, held until
 * the process ends; the generator needs bh_ic_workspace_bytes() of it whatever
 * n is, and the call returns BH_E_NOMEM should that ever exceed the array).
 * Allocates nothing and does not synchronise: asynchronous on the context's
 * stream.  A failed velocity draw is not reported; it leaves the velocities
 * non-finite.  Every call on one GPU uses that GPU's one array: calls that
 * overlap on one GPU (other streams or threads) race and must be ordered by
 * the caller.  Same argument checks as bh_ic_generate (1 <= n <= 2^30 - 1). */
bh_status bh_ic_generate_static(bh_ctx *ctx, int32_t kind, int64_t n, uint64_t seed, double a, double M,
                                double *pos, double *vel, double *mass);

/* ---------------------------------------------------------------- serving --- */

typedef struct {
    int64_t n;          /* particles */
    int32_t steps;      /* KDK steps */
    int32_t ic_kind;    /* 0 Plummer, 1 uniform cube */
    uint64_t seed;
    bh_params p;
    double dt;
} bh_request;

typedef struct {
    int32_t state;       /* 0 queued, 1 running, 2 done, 3 failed, 4 cancelled */
    int32_t steps_done;
    double t_submit, t_admit, t_done;   /* seconds on the server's monotonic clock */
    double K, W;         /* energies at completion */
} bh_result;

/* A continuous-batching server: its own host thread and HIP stream on ctx's
 * device; requests are admitted first-come first-served while their device
 * footprint fits the caller's arena (device memory, arena_bytes) and the slot
 * and resident-particle caps; every iteration advances all resident
 * simulations by one step in one forest launch sequence; finished ones retire
 * and free their arena space for the next. */
bh_status bh_server_create(bh_ctx *ctx, void *arena, size_t arena_bytes, int32_t max_slots,
                           int64_t max_resident_particles, bh_server **out);
/* BH_E_NOMEM if the request can never fit the arena or the caps. */
bh_status bh_server_submit(bh_server *s, const bh_request *req, uint64_t *id);
/* Thread-safe.  BH_E_BUSY while queued or running (res is still filled). */
bh_status bh_server_poll(bh_server *s, uint64_t id, bh_result *res);
/* Copy a finished request's final state into caller memory (n x 3 each,
 * nullable; device or host) and release it.  SYNC on the server's copy stream
 * only: it does not wait for the iteration in flight.  Thread-safe; must not
 * overlap bh_server_destroy. */
bh_status bh_server_fetch(bh_server *s, uint64_t id, double *pos, double *vel);
bh_status bh_server_cancel(bh_server *s, uint64_t id);
/* Seconds on the server clock (same clock as bh_result times). */
double bh_server_now(bh_server *s);
/* Drains running requests, stops the thread. */
bh_status bh_server_destroy(bh_server *s);

#ifdef __cplusplus
}
#endif
#endif /* BH_H */
