// Internal declarations shared by the host runtime and the HIP kernels of libibops.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ib.h"

namespace ibk {

// Sort configuration: 256-thread blocks, SORT_IPT keys per thread.
constexpr int SORT_BLOCK = 256;
#ifndef IBK_SORT_IPT
#define IBK_SORT_IPT 8
#endif
constexpr int SORT_IPT = IBK_SORT_IPT;
constexpr int SORT_TILE = SORT_BLOCK * SORT_IPT;
// Sorted positions per thread of the segments kernel: 8, or 2 for plans below
// SEG_SMALL_POINTS points (four times the blocks, where few tiles would leave most CUs idle).
constexpr int SEG_IPT = 8;
constexpr int SEG_IPT_SMALL = 2;
constexpr int64_t SEG_SMALL_POINTS = int64_t(1) << 18;
#ifndef IBK_SCANNED_MIN_POINTS
#define IBK_SCANNED_MIN_POINTS (1 << 18)
#endif
constexpr int64_t SCANNED_MIN_POINTS = IBK_SCANNED_MIN_POINTS;  // plans: scanned passes from here
constexpr int SCAN_VPT = 16;                      // counts per thread of the count scan
constexpr int SCAN_TILE = SORT_BLOCK * SCAN_VPT;  // counts per scan block
constexpr int MAX_RADIX_BITS = 8;

// Look-back status words: 2 flag bits over a 30-bit count.
constexpr uint32_t LB_AGG = 1u << 30;
constexpr uint32_t LB_INC = 2u << 30;
constexpr uint32_t LB_MASK = (1u << 30) - 1u;
constexpr int64_t MAX_POINTS = (int64_t)LB_MASK;  // counts must fit in 30 bits

// Device error flag bits.
constexpr uint32_t FLAG_BAD_POINT = 1u;
constexpr uint32_t FLAG_LOOKBACK_STALL = 2u;

struct PlanDev {
    int32_t* keys0;        // [nstag][n] keys in input order
    int32_t* kA;           // ping-pong key/value buffers [nstag][n]
    int32_t* vA;
    int32_t* kB;
    int32_t* vB;
    uint32_t* hist;        // [nstag][npass][R] global digit counts
    uint32_t* sort_status; // [nstag][npass][ntiles][R] look-back words
    uint32_t* counters;    // [nstag][npass + 1] tile tickets (last: segments kernel)
    uint32_t* flag;        // device error flag
    int32_t* cblk;         // [nstag][rows * (nbx + 1)] cell-block start table (see GeomArgs)
    int32_t* seg_off;      // [nstag][n + 1]
    int32_t* q;            // [nstag]
    uint32_t* seg_status;  // [nstag][nseg_tiles] look-back words
    uint32_t* scan_status; // [nstag][npass][nscan_tiles] look-back words of the count scans
    void* Xs;              // [n][dim] positions in the sorted order of staggering 0
    void* Us;              // [n][2] interpolation: the first components in that order
    long long* partial;    // [tiles][split][tile cells] partial fixed-point tile sums (split > 1 only)
    int32_t* tile_shift;   // [tiles] fixed-point scale exponent of each split tile
    unsigned long long* fmax;  // [3][FMAX_BLOCKS] partial maxima of |F| per component
    uint32_t* zero_begin;  // region cleared at each update
    size_t zero_words;
};

// Exact division of non-negative 31-bit integers by a fixed divisor d >= 1:
// q = (n * m) >> s with s = 31 + ceil(log2 d) and m = ceil(2^s / d) (m < 2^32).
struct FastDiv {
    uint32_t d, m, s;
};

// Geometry and per-call arguments passed by value to every kernel.
//
// Cell-block start table: each x-row of cells is cut into blocks of 4 cells; entry
// (row r, block b), at flat index r * (nbx + 1) + b, holds the first sorted position whose
// cell lies in row r at x >= 4 b (b = nbx: the start of the next row).  A sorted range of
// cells [xa, xb) of one row is then bracketed in O(1) by entries xa / 4 and ceil(xb / 4).
//
// Staggering 0 (that of component 0) orders the points for spreading and interpolation.
// For component c, cell_c - cell_0 lies in [dlo, dhi] per dimension (each in {-1, 0, 1}).
constexpr int CBLK_SHIFT = 2;
struct GeomArgs {
    int dim;
    int ncomp;
    int nstag;
    int n[3];
    int rows;              // n1 * n2 (3-D) or n1 (2-D): number of x-rows
    int nbx;               // ceil(n0 / 4): cell blocks per x-row
    FastDiv div_n0;        // division by n0 (key -> row)
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
};

struct SortArgs {
    GeomArgs g;
    PlanDev d;
    int npass;
    int rbits;
    int64_t ntiles;        // sort tiles per stagger
    int64_t nseg_tiles;    // segment tiles per stagger
    int64_t nscan_tiles;   // scan tiles of one pass's digit-major tile counts
    int scanned;           // radix passes: count, scan, scatter (else one-sweep look-back)
    int seg_ipt;           // sorted positions per thread of the segments kernel
};

struct OpArgs {
    GeomArgs g;
    const int32_t* sorted_keys;  // staggering 0: [n]
    const int32_t* perm;         // staggering 0: [n]
    const int32_t* cblk;         // staggering 0: [rows * (nbx + 1)]
    const void* X;               // input order
    const void* Xs;              // staggering-0 order
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
    int interp_tiled;            // batches: interpolate through LDS tiles (see interp_tiles)
    void* Xadv;                  // interpolation: also advance these positions (or null)
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
constexpr int BATCH_RBITS = 8;       // one radix digit width for every job of a batch
constexpr int BATCH_MAX_PASSES = 4;  // ceil(31 / 8)
enum BatchStage {
    BS_RESET = 0,
    BS_FMAX,   // force maxima of every spreading job
    BS_KEYS,
    BS_SORT0,  // BS_SORT0 + p: radix pass p
    BS_SEG = BS_SORT0 + BATCH_MAX_PASSES,
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
    int grid[BS_COUNT];        // blocks to launch per stage (0: skip the stage)
    size_t keys_lds;           // dynamic LDS of the keys stage (largest job)
};

// Virtual-block counts of one job (host side).
int reset_blocks(const SortArgs& a);
int keys_blocks(const SortArgs& a);
size_t keys_lds_bytes(const SortArgs& a);
int interp_blocks(int64_t npts);
// Tiles of the LDS-staged interpolation of a 3-D plan, or 0 when its points should gather
// directly: staging pays off with at least 256 tiles (one block each) and 200 points per tile
// on average (measured crossover on 32^3..192^3 grids with 10^4..10^6 points).  Both paths
// give bitwise-equal results.
int interp_tiles(int dim, const int n[3], int64_t npts);
// 3-D spreading tile shapes (index into the shape table of the spreading kernels):
// 0 = 32x16x13, 1 = 32x8x13, 2 = 64x8x8.  FP32 plans and batches use 32x8x13 by default:
// its kernel fits four waves per SIMD (FP32 sums need half the registers), and its LDS tile
// lets four blocks share a CU.  FP64 plans use 32x16x13 (two waves per SIMD either way).
constexpr int SPREAD_TILE_SHAPES = 3;
constexpr int builtin_spread_shape(int32_t dtype) { return dtype == IB_F32 ? 1 : 0; }
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
// Keys of staggering s and its digit histograms.
hipError_t launch_keys(const SortArgs& a, int dtype, const void* X, int s, hipStream_t st);
// Sort staggering s, build its segments and cell-block table; with gather_x, also write
// the positions in that order (used for staggering 0 only).
hipError_t launch_sort_stagger(const SortArgs& a, int s, int dtype, const void* X, bool gather_x,
                               hipStream_t st);
// Spreading, preceded by the pass that finds the force maxima (fmax_kernel).
hipError_t launch_spread(const OpArgs& a, int dtype, int kernel, hipStream_t st);
constexpr int FMAX_PARTS = 1024;  // partial maxima per component (blocks of fmax_kernel)
hipError_t launch_interp(const OpArgs& a, int dtype, int kernel, hipStream_t st);
hipError_t launch_interp_grad(const OpArgs& a, int dtype, int kernel, const void* W, void* dX,
                              int accumulate, hipStream_t st);
hipError_t launch_advect(int dim, int ncomp, int64_t npts, const double length[3], int walls, int dtype,
                         void* X, const void* U, double dt, hipStream_t st);
// Walled plans: the caller's grid field (user grid) to the kernels' padded grid (zero ghost
// values), and back (ghost values dropped; accumulate adds into dst).
hipError_t launch_pad(const ib_grid_desc& user, const ib_grid_desc& kg, int dtype, const void* src,
                      void* dst, hipStream_t st);
hipError_t launch_unpad(const ib_grid_desc& user, const ib_grid_desc& kg, int dtype,
                        const void* src, void* dst, bool accumulate, hipStream_t st);
hipError_t launch_tether(int dim, int walls, int64_t npts, const double length[3], int dtype,
                         const void* X0, const void* X, double k, void* F, hipStream_t st);

}  // namespace ibk
