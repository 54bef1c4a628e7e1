// Internal declarations shared by the host runtime and the HIP kernels of libibops.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ib.h"

namespace ibk {

// Sort configuration: tiles of SORT_TILE points, SORT_BLOCK threads with SORT_IPT keys
// each (1024 threads measured 6 us faster per plan update at 10^6 points than 256 threads
// with eight keys).
constexpr int SORT_BLOCK = 1024;
constexpr int SORT_IPT = 2;
constexpr int SORT_TILE = SORT_BLOCK * SORT_IPT;
// Bucket pass: the top rb key bits (rb <= MAX_BUCKET_BITS) choose the bucket of 2^cb cells.
// A bucket block counts BKT_CELLS cells at a time in LDS and stages up to BKT_CAP points
// there (more go through global memory).
// FP32 sorts may use 2^11 buckets: at 256^3 cells a bucket of 2^10 would span more cells
// than a block counts in LDS at once.  FP64 keeps 2^10, so that the scatter's LDS (which
// carries the positions) still lets two blocks share a CU.
constexpr int MAX_BUCKET_BITS = 11;
constexpr int max_bucket_bits(int dtype) { return dtype == IB_F64 ? 10 : 11; }
constexpr int BKT_CELLS = 8192;
constexpr int BKT_CAP = 4096;
constexpr int BKT_SHARDS = 16;   // shards of the bucket histogram and fill cursors
constexpr int PLAN_COUNTERS = 2;  // tickets per staggering (the second: runs kernel)

// Look-back status words: 2 flag bits over a 30-bit count.
constexpr uint32_t LB_AGG = 1u << 30;
constexpr uint32_t LB_INC = 2u << 30;
constexpr uint32_t LB_MASK = (1u << 30) - 1u;
constexpr int64_t MAX_POINTS = (int64_t)LB_MASK;  // counts must fit in 30 bits

// A cell of at least CROWD_CELL points puts two of its points into one 16-lane group of a
// spreading chunk (consecutive sorted points go to different groups, four per round), so
// their adds meet at one LDS address.  When at least 1/CROWD_DIV of the points lie in such
// cells, spreading rotates each lane's order of adds (spread_kernel).
constexpr uint32_t CROWD_CELL = 5;
constexpr uint32_t CROWD_DIV = 12;

// Device error flag bits.
constexpr uint32_t FLAG_BAD_POINT = 1u;
constexpr uint32_t FLAG_LOOKBACK_STALL = 2u;

struct PlanDev {
    int32_t* kin;          // [nstag][n] keys in the source order of the last sort
    int32_t* kA;           // [nstag][n] keys and indices in bucket order (input order per bucket)
    int32_t* vA;
    int32_t* kB;           // [nstag][n] sorted keys
    int32_t* vB;           // [nstag][n] permutation: sorted position -> point index
    uint32_t* bhist;       // [nstag][3][BKT_SHARDS][R] bucket histogram, fill cursors, bucket starts
    uint32_t* counters;    // [nstag][PLAN_COUNTERS] tile tickets
    uint32_t* flag;        // device error flag
    uint32_t* bad;         // keys pass: a point was bad (moved into flag by the scatter pass)
    int32_t* cstart;       // [G + 1] first sorted position of each cell (staggering 0)
    int32_t* seg_off;      // [nstag][n + 1]
    int32_t* q;            // [nstag]
    uint32_t* seg_status;  // [nstag][nseg_tiles] look-back words of the runs kernel
    void* Xs;              // [dim][n] positions in the sorted order of staggering 0 (columns)
    void* Xb;              // [dim][n] positions in bucket order (carried by the sort)
    void* Xn;              // [dim][n] positions advanced by interpolation, in sorted order
    void* Us;              // [n][2] interpolation: the first components in that order
    long long* partial;    // [tiles][split][tile cells] partial fixed-point tile sums (split > 1 only)
    int32_t* tile_shift;   // [tiles] fixed-point scale exponent of each split tile
    unsigned long long* fmax;  // [3][FMAX_PARTS] partial maxima of |F| per component
    uint32_t* cellmax;     // most points in any staggering-0 cell (bucket pass; zero region)
    uint32_t* crowd;       // points in staggering-0 cells of at least CROWD_CELL points (likewise)
    uint32_t* zero_begin;  // per-update region: cleared before the first update, then by the sorts
    size_t zero_words;
};

// Geometry and per-call arguments passed by value to every kernel.
//
// Cell-start table: entry c (0 <= c <= G) is the first sorted position whose key is at
// least c, so the points of cells [ca, cb) of one x-row are the sorted range
// [cstart[ca], cstart[cb]).
//
// Staggering 0 (that of component 0) orders the points for spreading and interpolation.
// For component c, cell_c - cell_0 lies in [dlo, dhi] per dimension (each in {-1, 0, 1}).
struct GeomArgs {
    int dim;
    int ncomp;
    int nstag;
    int n[3];
    int rows;              // n1 * n2 (3-D) or n1 (2-D): number of x-rows
    double inv_n[3];       // 1 / n_k (periodic wrap of cell indices)
    int64_t npts;
    int comp_stag[3];      // component -> distinct-stagger index
    int dlo[3][3];         // per component and dimension
    int dhi[3][3];
    double inv_h_d[3];     // fl64(n_k / L_k) and its residual (n_k / L_k - inv_h_d)
    double inv_lo_d[3];
    float inv_h_f[3];      // fl32(n_k / L_k) and its residual
    float inv_lo_f[3];
    double stag_xi[3][3];  // per distinct stagger
    double comp_xi[3][3];  // per component
    double scale;          // (prod_k h_k)^-1 for spreading
    int split;             // blocks per spreading tile (see spread_split)
    int sp_tile;           // spreading tile shape (ib_tuning.spread_tile)
    int odd;               // odd-support kernel: a point's cell is its nearest node (Fig. 1(b))
};

struct SortArgs {
    GeomArgs g;
    PlanDev d;
    int rb;                // bucket digit bits (bucket = key >> cb)
    int cb;                // cell bits per bucket
    int64_t ntiles;        // sort tiles (SORT_TILE points) per stagger
    int64_t nseg_tiles;    // tiles of the runs kernel
};

struct OpArgs {
    GeomArgs g;
    const int32_t* sorted_keys;  // staggering 0: [n]
    const int32_t* perm;         // staggering 0: [n]
    const int32_t* cstart;       // staggering 0: [G + 1] cell-start table
    const void* X;               // input order
    const void* Xs;              // staggering-0 order, columns [dim][n]
    const void* F;
    void* Us;
    void* f;
    const void* u;
    void* U;
    int accumulate;
    int tiles[3];                // tiles per dimension (tiles[2] = 1 in 2-D)
    int tile_slow;               // dimension whose tile index varies slowest (spread_tiles)
    long long* partial;          // split spreading: partial fixed-point tile sums
    int32_t* tile_shift;         //   and each split tile's scale exponent
    const unsigned long long* fmax;  // partial maxima of |F| per component (fmax_kernel)
    const uint32_t* cellmax;     // most points in any staggering-0 cell
    const uint32_t* crowd;       // points in cells of at least CROWD_CELL points (or null)
    int interp_tiled;            // batches: interpolate through LDS tiles (see interp_tiles)
    // Walled plans run on a periodic grid with ghost cells added at the top of each walled
    // axis (a point's stencil may reach them; they are no grid points).  direct = 1: f
    // (spreading) or u (interpolation, the position gradient) is the caller's field of
    // user_n[0] x user_n[1] x user_n[2] cells per component, whose cells are the kernel
    // grid's first user_n[k] along each axis: ghost values are dropped when spreading and
    // read as zero when interpolating, with no padded copy.
    int direct;
    int user_n[3];
    double out_scale;            // interpolation and its gradient: results times this (1: none)
    void* Xadv;                  // interpolation: also advance these positions (or null)
    void* Xnext;                 //   and write them in sorted order here, columns (or null)
    double adv_dt;               //   X <- wrap(X + dt U) with box edges adv_len
    double adv_len[3];
};

// ---- batches: many independent jobs, one launch per stage ------------------------------
//
// Every stage kernel of a batch runs the virtual blocks of all jobs: virtual block vb of a
// stage belongs to job j when starts[stage][j] <= vb < starts[stage][j + 1], as block
// vb - starts[stage][j] of that job's own launch.  A launch's blocks stride over the
// virtual blocks, so a launch of any size (e.g. a fixed grid replayed in a graph) covers a
// batch of any shape.
constexpr int BATCH_MAX_JOBS = 128;
enum BatchStage {
    BS_RESET = 0,
    BS_FMAX,     // force maxima of every spreading job
    BS_KEYS,     // keys and the bucket histogram
    BS_SCATTER,  // bucket starts, and points into their buckets
    BS_BUCKET,   // per bucket: counting sort, cell-start table, positions in sorted order
    BS_SPREAD,
    BS_SPLITSUM,  // partial tiles of split spreading tiles added
    BS_INTERP,
    BS_COUNT
};

struct BatchJob {
    SortArgs sa;  // the job's plan (staggering 0 is sorted)
    OpArgs op;    // its operators (F/f and u/U null when not requested)
};

// Read-only during a batch.  The header of a batch in device memory is the table, then
// the jobs' error flags (uint32_t[BATCH_MAX_JOBS], cleared by the upload), then the jobs.
struct BatchTable {
    int32_t njobs;
    int32_t starts[BS_COUNT][BATCH_MAX_JOBS + 1];
};

// Host-side view of a batch resident in device memory.
struct BatchLaunch {
    const BatchJob* jobs;      // device
    const BatchTable* table;   // device
    int dtype, dim, kernel;
    int sp_tile;               // spreading tile shape of every job (3-D)
    int grid[BS_COUNT];        // blocks to launch per stage (0: skip the stage)
};

// Virtual-block counts of one job (host side).
int reset_blocks(const SortArgs& a);
int keys_blocks(const SortArgs& a);
int bucket_blocks(const SortArgs& a);
int interp_blocks(int64_t npts);
// Tiles of the LDS-staged interpolation of a 3-D plan, or 0 when its points should gather
// directly: staging pays off with at least 256 tiles (one block each) and 200 points per tile
// on average (measured crossover on 32^3..192^3 grids with 10^4..10^6 points).  Both paths
// give bitwise-equal results.
int interp_tiles(int dim, const int n[3], int64_t npts);
// 3-D spreading tile shapes (index into the shape table of the spreading kernels):
// 0 = 32x16x13, 1 = 32x8x13, 2 = 64x8x8.  Plans and batches of both precisions use 64x8x8
// by default: its long rows fill the 64-point chunks of a source slice best (fewer partial
// chunks and table builds per point) and its small LDS tile lets three blocks share a CU,
// which outweighs its larger halo (measured fastest of several shapes at 128^3 with 10^6
// points, both precisions; the sums are 64-bit integers in either).
constexpr int SPREAD_TILE_SHAPES = 3;
constexpr int builtin_spread_shape(int32_t) { return 2; }
void spread_tiles(int dim, int shape, const int n[3], int tiles[3], int* slow);
// Cells of one spreading tile, and the number of blocks that share a tile (1 .. SPLIT_MAX)
// for npts points over ntiles (tiles x components) tiles: a dense point set on a small grid
// would otherwise leave most of the GPU idle.  split_points as in ib_tuning.  The partial
// tiles of shared tiles are added by a second kernel, one thread per tile cell.
constexpr int SPLIT_MAX = 256;
constexpr int SPLIT_BLOCKS = 512;      // built-in target of blocks per spreading launch
constexpr int SPLIT_MIN_POINTS = 128;  // built-in floor of points per block
size_t spread_tile_cells(int dim, int shape);
int spread_split(int64_t npts, int ntiles, int split_points);

hipError_t launch_batch_plan(const BatchLaunch& b, hipStream_t st);
hipError_t launch_batch_ops(const BatchLaunch& b, hipStream_t st);

// Host launchers (stream-ordered; return hipError_t).
hipError_t launch_plan_reset(const SortArgs& a, hipStream_t st);
// Keys and sort of staggering s (sorted keys kB, permutation vB) of the points whose
// positions X are read in a source order: row i of the caller's (n x dim) array is point i
// (psrc null), or column entry i of a plan array ([dim][n]) is point psrc[i].  With outputs0, also the cell-start table and the positions in sorted
// order (staggering 0).
hipError_t launch_sort_stagger(const SortArgs& a, int s, int dtype, const void* X, const int32_t* psrc,
                               bool outputs0, hipStream_t st);
// keys[i] = the staggering-s key of point i (from the sorted keys and the permutation).
hipError_t launch_keys_out(const SortArgs& a, int s, int32_t* keys, hipStream_t st);
// Run heads, q and segment offsets of staggering s from its sorted keys.
hipError_t launch_runs(const SortArgs& a, int s, hipStream_t st);
// Spreading, preceded by the pass that finds the force maxima (fmax_kernel).
hipError_t launch_spread(const OpArgs& a, int dtype, int kernel, hipStream_t st);
constexpr int FMAX_PARTS = 1024;  // partial maxima per component (blocks of fmax_kernel)
hipError_t launch_interp(const OpArgs& a, int dtype, int kernel, hipStream_t st);
hipError_t launch_interp_grad(const OpArgs& a, int dtype, int kernel, const void* W, void* dX,
                              int accumulate, hipStream_t st);
hipError_t launch_advect(int dim, int ncomp, int64_t npts, const double length[3], int walls, int dtype,
                         void* X, const void* U, double dt, hipStream_t st);
hipError_t launch_tether(int dim, int walls, int64_t npts, const double length[3], int dtype,
                         const void* X0, const void* X, double k, void* F, hipStream_t st);

}  // namespace ibk
