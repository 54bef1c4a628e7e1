// Batches of independent spread/interpolate jobs: one plan per job, carved from one
// workspace, and one launch per stage covering every job (keys, count scan, bucket
// scatter, bucket sort, force maxima, spreading, interpolation).
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstring>
#include <mutex>
#include <vector>

#include "ib.h"
#include "ib_host.h"
#include "ib_internal.h"

using namespace ibk;

namespace {

struct JobGeom {
    int nstag;
    int cs[3];
    double sx[3][3];
    Layout L;
    size_t off;  // byte offset of the job's plan region from the start of the plan regions
};

struct BatchLayout {
    size_t header;  // table and job array
    size_t plans;   // all plan regions
    std::vector<JobGeom> jobs;
};

// Validate the jobs and lay out their plan regions, one after another from offset 0, each
// with the batch's tuning (NULL: the built-in choices).
int32_t batch_layout(const ib_job* jobs, int32_t njobs, int32_t dtype, const ib_tuning* tuning,
                     BatchLayout* B)
{
    if (!jobs || njobs < 1) return IB_ERR_ARG;
    if (njobs > BATCH_MAX_JOBS) return IB_ERR_UNSUPPORTED;
    if (dtype != IB_F64 && dtype != IB_F32) return IB_ERR_UNSUPPORTED;
    if (check_tuning(tuning, dtype) != IB_OK) return IB_ERR_ARG;
    B->jobs.resize(njobs);
    B->header = batch_header_bytes(njobs);
    size_t off = 0;
    for (int j = 0; j < njobs; ++j) {
        const ib_job& J = jobs[j];
        JobGeom& G = B->jobs[j];
        std::memset(G.sx, 0, sizeof G.sx);
        int32_t st = check_grid(&J.grid, dtype, J.npts, &G.nstag, G.cs, G.sx);
        if (st != IB_OK) return st;
        if (J.grid.walls) return IB_ERR_UNSUPPORTED;  // batches run periodic jobs only
        if (J.grid.dim != jobs[0].grid.dim || J.grid.kernel != jobs[0].grid.kernel)
            return IB_ERR_UNSUPPORTED;
        if (J.npts > 0 && !J.X) return IB_ERR_ARG;
        if (J.f && J.npts > 0 && !J.F) return IB_ERR_ARG;
        if (J.u && J.npts > 0 && !J.U) return IB_ERR_ARG;
        make_layout(&J.grid, dtype, G.nstag, J.npts, &G.L, tuning);
        G.off = off;
        off += G.L.total;
    }
    B->plans = off;
    return IB_OK;
}

// Fill the host copy of the header (table, then job array, as batch_header_bytes lays them
// out) for jobs whose header will live at `header_dev` and whose plan regions start at
// `plans_dev`; and the launch description with exact grids.
void batch_build(const ib_job* jobs, int32_t njobs, int32_t dtype, const BatchLayout& B,
                 char* header_dev, char* plans_dev, char* host_header, BatchLaunch* bl)
{
    BatchTable* ht = (BatchTable*)host_header;
    BatchJob* hj = (BatchJob*)(host_header + batch_jobs_offset());
    std::memset(ht, 0, sizeof *ht);
    std::memset(host_header + batch_flags_offset(), 0, BATCH_MAX_JOBS * sizeof(uint32_t));
    ht->njobs = njobs;
    int counts[BS_COUNT];
    uint32_t* flags_dev = (uint32_t*)(header_dev + batch_flags_offset());
    for (int j = 0; j < njobs; ++j) {
        const ib_job& J = jobs[j];
        const JobGeom& G = B.jobs[j];
        ib_plan_s p;
        plan_setup(&p, &J.grid, dtype, J.npts, G.nstag, G.cs, G.sx, G.L, plans_dev + G.off);
        BatchJob& b = hj[j];
        std::memset(&b, 0, sizeof b);
        b.sa = p.sa;
        // All error flags of the batch sit in the table, so one copy reads them back.
        b.sa.d.flag = flags_dev + j;
        OpArgs& a = b.op;
        a.g = p.sa.g;
        a.sorted_keys = p.sorted_keys;
        a.perm = p.perm;
        a.cstart = p.sa.d.cstart;
        a.X = J.X;
        a.Xs = p.sa.d.Xs;
        a.F = J.F;
        a.Us = p.sa.d.Us;

        a.partial = p.sa.d.partial;
        a.tile_shift = p.sa.d.tile_shift;
        a.fmax = p.sa.d.fmax;
        a.cellmax = p.sa.d.cellmax;
        a.crowd = nullptr;  // batches keep one order of adds
        a.direct = 0;       // and run periodic jobs only
        a.f = J.f;
        a.u = J.u;
        a.U = J.U;
        a.out_scale = 1.0;
        a.accumulate = 0;
        spread_tiles(a.g.dim, a.g.sp_tile, a.g.n, a.tiles, &a.tile_slow);

        const SortArgs& sa = b.sa;
        const int64_t n = J.npts;
        counts[BS_RESET] = reset_blocks(sa);
        counts[BS_FMAX] = J.f ? FMAX_PARTS : 0;
        counts[BS_KEYS] = keys_blocks(sa);
        counts[BS_SCATTER] = n > 0 ? (int)sa.ntiles : 0;
        counts[BS_BUCKET] = bucket_blocks(sa);
        counts[BS_SPREAD] = J.f ? a.tiles[0] * a.tiles[1] * a.tiles[2] * a.g.ncomp * a.g.split : 0;
        counts[BS_SPLITSUM] =
            (J.f && a.g.split > 1)
                ? (int)((a.tiles[0] * a.tiles[1] * a.tiles[2] * a.g.ncomp *
                             (int64_t)spread_tile_cells(a.g.dim, a.g.sp_tile) + 255) / 256)
                : 0;
        const int itiles = J.u ? interp_tiles(a.g.dim, a.g.n, n) : 0;
        a.interp_tiled = itiles > 0;
        counts[BS_INTERP] = J.u ? (itiles > 0 ? itiles : interp_blocks(n)) : 0;
        for (int s = 0; s < BS_COUNT; ++s) ht->starts[s][j + 1] = ht->starts[s][j] + counts[s];
    }
    bl->jobs = (const BatchJob*)(header_dev + batch_jobs_offset());
    bl->table = (const BatchTable*)header_dev;
    bl->dtype = dtype;
    bl->dim = jobs[0].grid.dim;
    bl->kernel = jobs[0].grid.kernel;
    bl->sp_tile = B.jobs[0].L.sp_tile;  // one tuning for all jobs: one spreading tile shape
    for (int s = 0; s < BS_COUNT; ++s) bl->grid[s] = ht->starts[s][njobs];
}

}  // namespace

namespace ibk {

size_t batch_flags_offset() { return align_up(sizeof(BatchTable)); }

size_t batch_jobs_offset() { return batch_flags_offset() + align_up(BATCH_MAX_JOBS * sizeof(uint32_t)); }

size_t batch_header_bytes(int32_t njobs)
{
    return batch_jobs_offset() + align_up((size_t)njobs * sizeof(BatchJob));
}

size_t batch_job_bytes(const ib_job* job, int32_t dtype)
{
    int nstag, cs[3];
    double sx[3][3];
    if (!job || check_grid(&job->grid, dtype, job->npts, &nstag, cs, sx) != IB_OK) return 0;
    if (job->grid.walls) return 0;
    Layout L;
    make_layout(&job->grid, dtype, nstag, job->npts, &L, nullptr);
    return L.total;
}

int32_t batch_prepare(const ib_job* jobs, int32_t njobs, int32_t dtype, void* header_dev,
                      void* plans_dev, size_t plans_bytes, void* host_header, BatchLaunch* bl)
{
    BatchLayout B;
    int32_t st = batch_layout(jobs, njobs, dtype, nullptr, &B);
    if (st != IB_OK) return st;
    if (!header_dev || !plans_dev || !host_header) return IB_ERR_ARG;
    if (((uintptr_t)header_dev % ALIGN) != 0 || ((uintptr_t)plans_dev % ALIGN) != 0) return IB_ERR_ARG;
    if (plans_bytes < B.plans) return IB_ERR_OOM;
    batch_build(jobs, njobs, dtype, B, (char*)header_dev, (char*)plans_dev, (char*)host_header, bl);
    return IB_OK;
}

int32_t batch_launch(const ib_job* jobs, int32_t njobs, int32_t dtype, const ib_tuning* tuning,
                     void* workspace, size_t workspace_bytes, void* host_staging, hipStream_t hs)
{
    BatchLayout B;
    int32_t st = batch_layout(jobs, njobs, dtype, tuning, &B);
    if (st != IB_OK) return st;
    if (!workspace || ((uintptr_t)workspace % ALIGN) != 0) return IB_ERR_ARG;
    if (workspace_bytes < B.header + B.plans) return IB_ERR_OOM;
    char* base = (char*)workspace;
    // The header goes up in one copy from host memory laid out like its device copy.
    const size_t nbytes = batch_jobs_offset() + (size_t)njobs * sizeof(BatchJob);
    std::vector<char> pageable;
    char* stage = (char*)host_staging;
    if (!stage) {
        pageable.resize(nbytes);
        stage = pageable.data();
    }
    BatchLaunch bl;
    batch_build(jobs, njobs, dtype, B, base, base + B.header, stage, &bl);
    if (hipMemcpyAsync(base, stage, nbytes, hipMemcpyHostToDevice, hs) != hipSuccess)
        return IB_ERR_HIP;
    hipError_t e = launch_batch_plan(bl, hs);
    if (e == hipSuccess) e = launch_batch_ops(bl, hs);
    return hip_status(e);
}

}  // namespace ibk

// ---- the batch workspace of ib_batch_run_static -------------------------------------------
//
// A fixed array in device memory: each GPU the library runs on holds its own copy, at its own
// address, until the process ends.  In host code the array's name is only a host-side
// stand-in: the kernels and copies receive the device address taken once per device with
// hipGetSymbolAddress (static_scratch), never the name.
static __device__ __align__(256) unsigned char scratch[IB_STATIC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[SCRATCH_DEVICES];  // device address of scratch per device (null: not yet taken)

// The current device's copy of scratch (taken on the first call on that device).
int32_t static_scratch(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_DEVICES) return IB_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return IB_ERR_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return IB_OK;
}

}  // namespace

extern "C" {

size_t ib_batch_workspace_bytes(const ib_job* jobs, int32_t njobs, int32_t dtype)
{
    return ib_batch_workspace_bytes_tuned(jobs, njobs, dtype, nullptr);
}

size_t ib_batch_workspace_bytes_tuned(const ib_job* jobs, int32_t njobs, int32_t dtype,
                                      const ib_tuning* tuning)
{
    BatchLayout B;
    if (batch_layout(jobs, njobs, dtype, tuning, &B) != IB_OK) return 0;
    return B.header + B.plans;
}

size_t ib_batch_staging_bytes(int32_t njobs)
{
    if (njobs < 1 || njobs > BATCH_MAX_JOBS) return 0;
    return batch_jobs_offset() + (size_t)njobs * sizeof(BatchJob);
}


int32_t ib_batch_run(const ib_job* jobs, int32_t njobs, int32_t dtype, void* workspace,
                     size_t workspace_bytes, void* host_staging, void* stream)
{
    return ibk::batch_launch(jobs, njobs, dtype, nullptr, workspace, workspace_bytes, host_staging,
                             (hipStream_t)stream);
}

int32_t ib_batch_run_tuned(const ib_job* jobs, int32_t njobs, int32_t dtype, const ib_tuning* tuning,
                           void* workspace, size_t workspace_bytes, void* host_staging, void* stream)
{
    return ibk::batch_launch(jobs, njobs, dtype, tuning, workspace, workspace_bytes, host_staging,
                             (hipStream_t)stream);
}

int32_t ib_batch_run_static(const ib_job* jobs, int32_t njobs, int32_t dtype, void* host_staging,
                            uint32_t* job_flags, void* stream)
{
    BatchLayout B;
    int32_t st = batch_layout(jobs, njobs, dtype, nullptr, &B);
    if (st != IB_OK) return st;
    if (B.header + B.plans > (size_t)IB_STATIC_SCRATCH_BYTES) return IB_ERR_OOM;
    void* ws = nullptr;
    st = static_scratch(&ws);
    if (st != IB_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    st = batch_launch(jobs, njobs, dtype, nullptr, ws, IB_STATIC_SCRATCH_BYTES, host_staging, hs);
    if (st == IB_OK && job_flags &&
        hipMemcpyAsync(job_flags, (const char*)ws + batch_flags_offset(), njobs * sizeof(uint32_t),
                       hipMemcpyDeviceToDevice, hs) != hipSuccess)
        st = IB_ERR_HIP;
    return st;
}

int32_t ib_batch_status(const ib_job* jobs, int32_t njobs, int32_t dtype, const void* workspace,
                        int32_t* job_status, void* stream)
{
    BatchLayout B;
    int32_t st = batch_layout(jobs, njobs, dtype, nullptr, &B);  // validation only
    if (st != IB_OK) return st;
    if (!workspace) return IB_ERR_ARG;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return IB_ERR_HIP;
    std::vector<uint32_t> flags(njobs);
    const char* fp = (const char*)workspace + batch_flags_offset();
    if (hipMemcpy(flags.data(), fp, njobs * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return IB_ERR_HIP;
    int32_t worst = IB_OK;
    for (int j = 0; j < njobs; ++j) {
        const int32_t s = flags[j] ? IB_ERR_DEVICE_FLAG : IB_OK;
        if (job_status) job_status[j] = s;
        if (s != IB_OK) worst = s;
    }
    return worst;
}

}  // extern "C"
