// Host-side objects behind the opaque C handles.
#pragma once
#include <string>
#include <vector>

#include "bh.h"
#include "bh_common.h"

struct ForestHost;

struct bh_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<ForestHost *> live;   // trees, simulations and forests of this context (fault words)
};

struct ForestCaps {
    uint32_t nseg = 0, ntot = 0, ntiles = 0, ngroups = 0;
    bool fp32 = false, fp64 = false;
    bool quad = false;   // second-moment buffers for quadrupole simulations
    bool group = false;  // group boxes for group-criterion simulations
};

struct ForestHost {
    bh::ForestDev dev{};
    std::vector<bh::SegDesc> seg;
    std::vector<bh::TileDesc> tiles;
    std::vector<bh::GroupDesc> groups;
    ForestCaps caps;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bh_ctx *ctx = nullptr;
    int walk_shape = 4;   // walk launch shape: wavefronts per workgroup, kWalkPersistent (bh_forest_autotune)
};

struct bh_tree {
    ForestHost F;
    const double *pos = nullptr;
    const double *mass = nullptr;
    bool upward_done = false;
    const void *lists_buf = nullptr;   // interaction lists of the current tree (bh_lists_build)
    uint32_t lists_chunks = 0;
};

struct bh_sim {
    ForestHost F;
    double *pos = nullptr, *vel = nullptr, *acc = nullptr;
    const double *mass = nullptr;
    bool have_acc = false;
};

struct bh_forest {
    ForestHost F;
    double *pos = nullptr, *vel = nullptr, *acc = nullptr;
    const double *mass = nullptr;
    bool have_acc = false;
    hipGraphExec_t graph = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream the step graph is recorded on
};

bh_status bh_fail(bh_status st, const std::string &msg);
bh_status bh_check_params(const bh_params *p);
size_t bh_plan_forest(ForestHost &F, int32_t nseg, const int64_t *n, const bh_params *p, char *ws);
void bh_forest_tables(ForestHost &F, int32_t nseg, const int64_t *n, const bh_params *p);
ForestCaps bh_caps_of(const ForestHost &F);
size_t bh_forest_carve(ForestHost &F, const ForestCaps &cap, char *ws);
bh_status bh_forest_upload_tables(ForestHost &F);
bh_status bh_forest_init(bh_ctx *ctx, ForestHost &F, int32_t nseg, const int64_t *n, const bh_params *p, void *ws,
                         size_t ws_bytes);
bh_status bh_forest_upload_seg(ForestHost &F);
// s == NULL: the context's stream
bh_status bh_forest_eval(ForestHost &F, const double *pos, const double *mass, double *acc, double *pot,
                         bool want_pot, hipStream_t s);
bh_status bh_forest_kdk(ForestHost &F, double *pos, double *vel, const double *mass, double *acc, hipStream_t s);
bh_status bh_forest_kdk_steps(ForestHost &F, double *pos, double *vel, const double *mass, double *acc,
                              int32_t nsteps, hipStream_t s);
bh_status bh_forest_check_err(ForestHost &F);
// Membership of a tree, simulation or forest in its context's list (bh_ctx_sync reports their faults).
void bh_ctx_attach(bh_ctx *ctx, ForestHost *F);
void bh_ctx_detach(bh_ctx *ctx, ForestHost *F);
