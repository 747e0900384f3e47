// Force walk on gfx950 (paper section 3: a remote cube is treated as one body
// only if its distance D from the body exceeds r/theta; the force stage is the
// computationally dominant part).
//
// One wavefront walks the tree for a group of 64 key-consecutive bodies, one
// body per lane.  The LDS stack holds (first child slot, number of children,
// lane mask) entries: a lane takes part in a cube only if it opened every
// ancestor, so each lane meets exactly the cubes of its own per-body walk and
// its interaction set is the per-body set of the method.
//
// Per popped entry, lane c loads child c's record (children are contiguous)
// and stages it in LDS; every lane then reads each child by broadcast.
// Per-lane predicates are formed as wave masks (one compare each, written to
// scalar registers) and combined with scalar logic, so a cube visit costs the
// distance, one fused opening test, two compares and, for accepting lanes,
// the softened monopole.  Opened leaves are queued (rank, lane mask) and their
// particles are loaded and converted 64 at a time.  No matrix cores: this is
// not a contraction.
//
// FP64 mode: the opening test s^2 < theta^2 D^2 is evaluated exactly as the
// oracle writes it; pair terms in FP64 with a Newton-refined rsqrt.
// FP32 mode: see k_walk32.
#include <map>
#include <mutex>
#include <utility>

#include "bh_walk_common.h"

namespace bh {

// Walk launches: one kernel per precision and walk variant present, in the
// grid form (W wavefronts per workgroup, one 64-body group each) or the persistent
// form (resident workgroups whose wavefronts take groups from a counter).  The
// shape does not change any result (each group's arithmetic is its own); forests
// pick it by measurement (bh_forest_autotune).
hipError_t launch_walk(const ForestDev &f, bool stats, bool want_pot, double *acc, double *pot, int64_t *n_mono,
                       int64_t *n_p2p, uint64_t *hash, hipStream_t s, int shape, uint32_t wlo, uint32_t whi,
                       int64_t *work, int64_t *gwork) {
    WalkOut o{acc, pot, n_mono, n_p2p, hash, wlo, whi, work, gwork};
    if (f.ngroups == 0) return hipSuccess;
    if (!stats && (shape & kWalkPersistent)) {
        hipError_t e = launch_fill_u32(f.wq, 0, kWalkQueues, s);   // every counter at the first group
        if (e != hipSuccess) return e;
    }
    launch_walk32_family(f, o, stats, want_pot, shape, s);
    launch_walk64_family(f, o, stats, want_pot, shape, s);
    return hipGetLastError();
}

// Resident workgroups per compute unit, by kernel (an occupancy query on first use
// per device), times the compute units.
uint32_t persistent_blocks(const void *kernel, uint32_t nb, int block) {
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, uint32_t> per_kernel;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nb;
    uint32_t resident = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = per_kernel.find({dev, kernel});
        if (it != per_kernel.end()) {
            resident = it->second;
        } else {
            int per_cu = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                return nb;   // the grid form's count: correct, only not resident at once
            resident = (uint32_t)(per_cu > 0 ? per_cu : 1) * (uint32_t)(cus > 0 ? cus : 1);
            per_kernel[{dev, kernel}] = resident;
        }
    }
    return resident < nb ? resident : nb;
}

}  // namespace bh
