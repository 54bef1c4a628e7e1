// Batches of independent spread/interpolate jobs: one plan per job, carved from one
// workspace, and one launch per stage covering every job (keys, radix passes, segments,
// force gather, spreading, interpolation).
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstring>
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
    size_t off;  // byte offset of the job's plan region in the workspace
};

struct BatchLayout {
    size_t table_off, jobs_off, total;
    std::vector<JobGeom> jobs;
};

// Validate the jobs and lay out the workspace: the table, the job array, then one plan
// region per job (radix digits of BATCH_RBITS bits for all).
int32_t batch_layout(const ib_job* jobs, int32_t njobs, int32_t dtype, BatchLayout* B)
{
    if (!jobs || njobs < 1) return IB_ERR_ARG;
    if (njobs > BATCH_MAX_JOBS) return IB_ERR_UNSUPPORTED;
    if (dtype != IB_F64 && dtype != IB_F32) return IB_ERR_UNSUPPORTED;
    B->jobs.resize(njobs);
    size_t off = 0;
    B->table_off = off;
    off += align_up(sizeof(BatchTable));
    B->jobs_off = off;
    off += align_up((size_t)njobs * sizeof(BatchJob));
    for (int j = 0; j < njobs; ++j) {
        const ib_job& J = jobs[j];
        JobGeom& G = B->jobs[j];
        std::memset(G.sx, 0, sizeof G.sx);
        int32_t st = check_grid(&J.grid, dtype, J.npts, &G.nstag, G.cs, G.sx);
        if (st != IB_OK) return st;
        if (J.grid.dim != jobs[0].grid.dim || J.grid.kernel != jobs[0].grid.kernel)
            return IB_ERR_UNSUPPORTED;
        if (J.npts > 0 && !J.X) return IB_ERR_ARG;
        if (J.f && J.npts > 0 && !J.F) return IB_ERR_ARG;
        if (J.u && J.npts > 0 && !J.U) return IB_ERR_ARG;
        make_layout(&J.grid, dtype, G.nstag, J.npts, &G.L, BATCH_RBITS);
        G.off = off;
        off += G.L.total;
    }
    B->total = off;
    return IB_OK;
}

// Host copies of the job array and the table for jobs laid out by B over `workspace`.
void batch_build(const ib_job* jobs, int32_t njobs, int32_t dtype, const BatchLayout& B,
                 char* workspace, BatchJob* hj, BatchTable* ht, BatchLaunch* bl)
{
    std::memset(ht, 0, sizeof *ht);
    ht->njobs = njobs;
    int counts[BS_COUNT];
    size_t keys_lds = 0;
    for (int j = 0; j < njobs; ++j) {
        const ib_job& J = jobs[j];
        const JobGeom& G = B.jobs[j];
        ib_plan_s p;
        plan_setup(&p, &J.grid, dtype, J.npts, G.nstag, G.cs, G.sx, G.L, workspace + G.off);
        BatchJob& b = hj[j];
        std::memset(&b, 0, sizeof b);
        b.sa = p.sa;
        // All error flags of the batch sit in the table, so one copy reads them back.
        b.sa.d.flag = (uint32_t*)(workspace + B.table_off + offsetof(BatchTable, flags)) + j;
        OpArgs& a = b.op;
        a.g = p.sa.g;
        a.sorted_keys = p.sorted_keys;
        a.perm = p.perm;
        a.cblk = p.sa.d.cblk;
        a.X = J.X;
        a.Xs = p.sa.d.Xs;
        a.F = J.F;
        a.Fs = p.sa.d.Fs;
        a.partial = p.sa.d.partial;
        a.tile_count = p.sa.d.tile_count;
        a.f = J.f;
        a.u = J.u;
        a.U = J.U;
        a.accumulate = 0;
        spread_tiles(a.g.dim, a.g.n, a.tiles);

        const SortArgs& sa = b.sa;
        const int64_t n = J.npts;
        counts[BS_RESET] = reset_blocks(sa);
        counts[BS_KEYS] = keys_blocks(sa);
        for (int q = 0; q < BATCH_MAX_PASSES; ++q)
            counts[BS_SORT0 + q] = (n > 0 && q < sa.npass) ? (int)sa.ntiles : 0;
        counts[BS_SEG] = (int)sa.nseg_tiles;
        counts[BS_GATHER] = J.f ? gather_blocks(n, a.g.ncomp) : 0;
        counts[BS_SPREAD] = J.f ? a.tiles[0] * a.tiles[1] * a.tiles[2] * a.g.ncomp * a.g.split : 0;
        counts[BS_INTERP] = J.u ? interp_blocks(n) : 0;
        for (int s = 0; s < BS_COUNT; ++s) ht->starts[s][j + 1] = ht->starts[s][j] + counts[s];
        if (counts[BS_KEYS] > 0 && keys_lds_bytes(sa) > keys_lds) keys_lds = keys_lds_bytes(sa);
    }
    bl->jobs = (const BatchJob*)(workspace + B.jobs_off);
    bl->table = (const BatchTable*)(workspace + B.table_off);
    bl->dtype = dtype;
    bl->dim = jobs[0].grid.dim;
    bl->kernel = jobs[0].grid.kernel;
    for (int s = 0; s < BS_COUNT; ++s) bl->grid[s] = ht->starts[s][njobs];
    bl->keys_lds = keys_lds;
}

}  // namespace

namespace ibk {

size_t batch_header_bytes(int32_t njobs)
{
    return align_up(sizeof(BatchTable)) + align_up((size_t)njobs * sizeof(BatchJob));
}

size_t batch_flags_offset() { return offsetof(BatchTable, flags); }

size_t batch_job_bytes(const ib_job* job, int32_t dtype)
{
    int nstag, cs[3];
    double sx[3][3];
    if (!job || check_grid(&job->grid, dtype, job->npts, &nstag, cs, sx) != IB_OK) return 0;
    Layout L;
    make_layout(&job->grid, dtype, nstag, job->npts, &L, BATCH_RBITS);
    return L.total;
}

int32_t batch_launch(const ib_job* jobs, int32_t njobs, int32_t dtype, void* workspace,
                     size_t workspace_bytes, void* host_staging, hipStream_t hs)
{
    BatchLayout B;
    int32_t st = batch_layout(jobs, njobs, dtype, &B);
    if (st != IB_OK) return st;
    if (!workspace || ((uintptr_t)workspace % ALIGN) != 0) return IB_ERR_ARG;
    if (workspace_bytes < B.total) return IB_ERR_OOM;
    char* base = (char*)workspace;

    // The table and the job array go up in one copy: [table | pad | jobs], the same
    // arrangement as at the head of the workspace.
    const size_t nbytes = align_up(sizeof(BatchTable)) + (size_t)njobs * sizeof(BatchJob);
    std::vector<char> pageable;
    char* stage = (char*)host_staging;
    if (!stage) {
        pageable.resize(nbytes);
        stage = pageable.data();
    }
    BatchTable* ht = (BatchTable*)stage;
    BatchJob* hj = (BatchJob*)(stage + B.jobs_off);
    BatchLaunch bl;
    batch_build(jobs, njobs, dtype, B, base, hj, ht, &bl);
    if (hipMemcpyAsync(base, stage, nbytes, hipMemcpyHostToDevice, hs) != hipSuccess)
        return IB_ERR_HIP;
    hipError_t e = launch_batch_plan(bl, hs);
    if (e == hipSuccess) e = launch_batch_ops(bl, hs);
    return hip_status(e);
}

}  // namespace ibk

extern "C" {

size_t ib_batch_workspace_bytes(const ib_job* jobs, int32_t njobs, int32_t dtype)
{
    BatchLayout B;
    if (batch_layout(jobs, njobs, dtype, &B) != IB_OK) return 0;
    return B.total;
}

size_t ib_batch_staging_bytes(int32_t njobs)
{
    if (njobs < 1 || njobs > BATCH_MAX_JOBS) return 0;
    return align_up(sizeof(BatchTable)) + (size_t)njobs * sizeof(BatchJob);
}


int32_t ib_batch_run(const ib_job* jobs, int32_t njobs, int32_t dtype, void* workspace,
                     size_t workspace_bytes, void* host_staging, void* stream)
{
    return ibk::batch_launch(jobs, njobs, dtype, workspace, workspace_bytes, host_staging,
                             (hipStream_t)stream);
}

int32_t ib_batch_status(const ib_job* jobs, int32_t njobs, int32_t dtype, const void* workspace,
                        int32_t* job_status, void* stream)
{
    BatchLayout B;
    int32_t st = batch_layout(jobs, njobs, dtype, &B);
    if (st != IB_OK) return st;
    if (!workspace) return IB_ERR_ARG;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return IB_ERR_HIP;
    std::vector<uint32_t> flags(njobs);
    const char* fp = (const char*)workspace + B.table_off + offsetof(BatchTable, flags);
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
