// Host-side internals of libibops shared by the plan and batch entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ib.h"
#include "ib_internal.h"

struct ib_plan_s {
    ib_grid_desc grid;     // the grid the kernels run on (padded if the caller's has walls)
    ib_grid_desc user;     // the caller's grid
    int32_t dtype;
    int64_t npts;
    ibk::SortArgs sa;      // geometry, device pointers, radix configuration
    int32_t* sorted_keys;  // final sort output (kB of staggering 0)
    int32_t* perm;         // (vB of staggering 0)
    const void* X;         // positions of the last update
    int updated;
    int xn_valid;          // Xn holds the positions of the last ib_interpolate_advect
    int cleared;           // the per-update region was cleared once (later updates clear it
                           // through the bucket pass)
};

namespace ibk {

constexpr size_t ALIGN = 256;  // alignment of every workspace region

size_t align_up(size_t v);

// Byte layout of one plan's workspace.
struct Layout {
    int nstag, rb, cb, rows;
    int64_t ntiles, nseg_tiles, G;
    int sp_tile, sp_tiles, split;  // tile shape, tiles (x components), blocks per tile
    size_t kin, kA, vA, kB, vB, bhist, cstart, seg_off, q, Xs, Xb, Xn, Us, partial, tile_shift, fmax,
        zero_begin, seg_status, counters, flag, bad, cellmax, crowd, zero_end, total;
};

// Validate a descriptor; find the distinct staggerings (count, component -> stagger index,
// their offsets).  Returns an ib_status.
int32_t check_grid(const ib_grid_desc* g, int32_t dtype, int64_t npts, int* nstag,
                   int comp_stag[3], double stag_xi[3][3]);

// Workspace layout of a plan on the caller's descriptor g (sized for kernel_grid(*g), plus
// one padded grid field when g has walls).
void make_layout(const ib_grid_desc* g, int32_t dtype, int nstag, int64_t n, Layout* L,
                 const ib_tuning* tuning = nullptr);
// The periodic grid a plan runs on: the caller's grid with IB_WALL_GHOSTS ghost indices
// added along every walled dimension (same spacing), walls cleared.
ib_grid_desc kernel_grid(const ib_grid_desc& g);
// IB_OK if every field of a (possibly null) tuning is in range.
int32_t check_tuning(const ib_tuning* t, int32_t dtype);

// Fill a plan object for a validated (caller's) descriptor over a workspace of layout L.
// The kernels run on kernel_grid(*grid); keys and weights use the caller's spacing.
void plan_setup(ib_plan_s* p, const ib_grid_desc* grid, int32_t dtype, int64_t npts, int nstag,
                const int cs[3], const double sx[3][3], const Layout& L, void* workspace);

int32_t hip_status(hipError_t e);

// Batches (ib_batch.cpp).  Workspace of a batch: header (table and job array), then one
// plan region per job of batch_job_bytes bytes, each 256-byte aligned.
size_t batch_header_bytes(int32_t njobs);
size_t batch_job_bytes(const ib_job* job, int32_t dtype);  // 0 for an invalid job
size_t batch_flags_offset();                               // of the per-job flags in the header
size_t batch_jobs_offset();                                // of the job array in the header
int32_t batch_launch(const ib_job* jobs, int32_t njobs, int32_t dtype, const ib_tuning* tuning,
                     void* workspace, size_t workspace_bytes, void* host_staging, hipStream_t stream);
// Build a batch whose header lives at header_dev (batch_header_bytes(njobs)) and whose plan
// regions start at plans_dev: writes the header's host copy (to be uploaded) and the launch
// description with exact grids.  Launches nothing.
int32_t batch_prepare(const ib_job* jobs, int32_t njobs, int32_t dtype, void* header_dev,
                      void* plans_dev, size_t plans_bytes, void* host_header, BatchLaunch* bl);

}  // namespace ibk
