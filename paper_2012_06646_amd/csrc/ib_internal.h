// Internal declarations shared by the host runtime and the HIP kernels of libibops.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ib.h"

namespace ibk {

// Sort configuration: 256-thread blocks, 16 keys per thread (one tile = 4096 keys).
constexpr int SORT_BLOCK = 256;
constexpr int SORT_IPT = 16;
constexpr int SORT_TILE = SORT_BLOCK * SORT_IPT;
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
    uint32_t* sort_status; // [npass][nstag * ntiles][R] look-back words
    uint32_t* counters;    // [npass + 1] tile tickets (last one: segments kernel)
    uint32_t* flag;        // device error flag
    int32_t* row_start;    // [nstag][rows + 1]
    int32_t* seg_off;      // [nstag][n + 1]
    int32_t* q;            // [nstag]
    uint32_t* seg_status;  // [nstag * nseg_tiles] look-back words
    uint32_t* zero_begin;  // region cleared at each update
    size_t zero_words;
};

// Geometry and per-call arguments passed by value to every kernel.
struct GeomArgs {
    int dim;
    int ncomp;
    int nstag;
    int n[3];
    int rows;              // n1 * n2 (3-D) or n1 (2-D): number of x-rows
    int64_t npts;
    int comp_stag[3];      // component -> distinct-stagger index
    double inv_h_d[3];     // fl64(n_k / L_k) and its residual (n_k / L_k - inv_h_d)
    double inv_lo_d[3];
    float inv_h_f[3];      // fl32(n_k / L_k) and its residual
    float inv_lo_f[3];
    double stag_xi[3][3];  // per distinct stagger
    double comp_xi[3][3];  // per component
    double scale;          // (prod_k h_k)^-1 for spreading
};

struct SortArgs {
    GeomArgs g;
    PlanDev d;
    int npass;
    int rbits;
    int64_t ntiles;        // sort tiles per stagger
    int64_t nseg_tiles;    // segment tiles per stagger
};

struct OpArgs {
    GeomArgs g;
    const int32_t* sorted_keys;  // [nstag][n]
    const int32_t* perm;         // [nstag][n]
    const int32_t* row_start;    // [nstag][rows + 1]
    const void* X;
    const void* F;
    void* f;
    const void* u;
    void* U;
    int accumulate;
    int tiles[3];                // tiles per dimension (tiles[2] = 1 in 2-D)
};

// Host launchers (stream-ordered; return hipError_t).
hipError_t launch_plan_update(const SortArgs& a, int dtype, const void* X, hipStream_t st);
hipError_t launch_spread(const OpArgs& a, int dtype, int kernel, hipStream_t st);
hipError_t launch_interp(const OpArgs& a, int dtype, int kernel, hipStream_t st);

}  // namespace ibk
