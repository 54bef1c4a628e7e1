// Plan kernels: cell keys, a stable sort of the point indices by key, and the table of
// where each cell's points start in that order.
//
// These are the preparatory steps of the parallel spreading algorithm (Alg. 4, Sec. 3.4):
// one key per IB point from the cell it occupies, a key-value sort of the point indices
// that groups equal keys, and (Fig. 2) the count of distinct keys and where each run
// starts.  The sort is stable, so the permutation is unique: ties keep input order.
//
// gfx950 design.  Keys are cell indices below G, so the sort needs no comparison passes
// over all key bits.  It runs as one bucket pass on the top key bits followed by a
// counting sort of each bucket inside one block's LDS:
//   keys_kernel      the key of every point, and the count of each bucket (key >> cb, the
//                    top rb bits): per block in LDS, then added to a shard of the global
//                    histogram;
//   radix_scatter_kernel  where each bucket (and each shard of it) starts, found by every
//                    block from the whole histogram; then each tile's (key, index) pairs,
//                    grouped by bucket in LDS, written to a range of their bucket that the
//                    tile reserves with one atomic per bucket (so the order inside a bucket
//                    depends on timing);
//   bucket_kernel    per bucket of 2^cb cells: a histogram of its cells in LDS, its scan
//                    (the cell-start table of the bucket, written coalesced), placement of
//                    every point at a slot of its cell, then each point's final place from
//                    its rank among the cell's points by index.  Within a cell the order is
//                    therefore ascending index whatever came before: the stable sort.  The
//                    sorted keys, the permutation and the positions in sorted order are
//                    written from there.
// The run heads, q and segment offsets of Fig. 2 follow from the sorted keys
// (runs_kernel), computed when a plan is exported: the operators use the cell-start table.
#include "device_common.h"

namespace ibk {

// ---- reset: clear the per-update region (before a plan's first update) -----------------
__device__ __forceinline__ void plan_reset_body(uint32_t* __restrict__ p, size_t nwords, int bid, int nblk)
{
    for (size_t i = (size_t)bid * blockDim.x + threadIdx.x; i < nwords; i += (size_t)nblk * blockDim.x)
        p[i] = 0u;
}

__global__ void plan_reset_kernel(uint32_t* __restrict__ p, size_t nwords)
{
    plan_reset_body(p, nwords, blockIdx.x, gridDim.x);
}

// Bucket bookkeeping of staggering s, in three arrays of [BKT_SHARDS][R] words: the
// histogram, the fill cursors, and the bucket starts (the first R words of the third).
// Tile t counts and fills shard t mod BKT_SHARDS, so that no counter takes more than a
// BKT_SHARDS-th of the tiles' atomic additions; a bucket's range is its shards' ranges in
// shard order.
__device__ __forceinline__ uint32_t* stag_hist(const SortArgs& a, int s)
{
    return a.d.bhist + (int64_t)s * 3 * BKT_SHARDS * ((int64_t)1 << a.rb);
}

// The keys pass marks bad points in d.bad, which moves into the error flag once the pass
// is complete; an update (fresh) starts the flag and the bucket pass's cell statistics
// afresh, an export adds to them.  One thread.
__device__ __forceinline__ void absorb_bad_points(const SortArgs& a, bool fresh)
{
    const uint32_t bad = *a.d.bad ? FLAG_BAD_POINT : 0u;
    *a.d.bad = 0u;
    if (fresh) {
        *a.d.flag = bad;
        *a.d.cellmax = 0u;
        *a.d.crowd = 0u;
    } else if (bad) {
        *a.d.flag |= bad;
    }
}

// ---- keys: one per point, and the bucket histogram ----------------------------------
// The pass reads the points in a source order: the caller's (rows of X, point i is i) or
// a sorted order of the plan (columns of X, point i is psrc[i]).  Block `tile` keys source
// positions [tile * SORT_TILE, ...) of staggering s into kin.
template <typename T>
__device__ __forceinline__ void keys_body(const SortArgs& a, const T* __restrict__ X, bool soa, int s,
                                          int tile)
{
    __shared__ uint32_t lh[1 << max_bucket_bits(sizeof(T) == 8 ? IB_F64 : IB_F32)];
    const GeomArgs& g = a.g;
    const int R = 1 << a.rb;
    for (int i = threadIdx.x; i < R; i += blockDim.x) lh[i] = 0u;
    __syncthreads();

    const int64_t n = g.npts;
    const int64_t base = (int64_t)tile * SORT_TILE;
    bool any_bad = false;
    // All positions of this thread first, so their loads are in flight together: every
    // load is unconditional at a clamped in-range index (values past the point count or the
    // dimension are never used), so none waits behind a branch.
    // Rows (n x dim, the caller's layout) or columns ([dim][n], the plan's own arrays).
    const int64_t last = n * g.dim - 1;
    const int64_t sr = soa ? 1 : g.dim, sc = soa ? n : 1;
    T xs[SORT_IPT][3];
#pragma unroll
    for (int u = 0; u < SORT_IPT; ++u) {
        const int64_t j = base + u * SORT_BLOCK + threadIdx.x;
#pragma unroll
        for (int k = 0; k < 3; ++k) xs[u][k] = X[min(j * sr + k * sc, last)];
    }
#pragma unroll
    for (int u = 0; u < SORT_IPT; ++u) {
        const int64_t j = base + u * SORT_BLOCK + threadIdx.x;
        bool bad = false;
        int key = 0, stride = 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {  // static indices: the coordinates stay in registers
            if (k < g.dim) {
                const T y = shifted_scaled<T>(xs[u][k], Prec<T>::inv_h(g, k), (T)g.stag_xi[s][k]);
                int c = 0;
                T r;
                if (fabs(y) < T(1073741824.0)) c = floor_mod(axis_cell<T>(y, g.odd != 0, &r), g.n[k], g.inv_n[k]);
                else bad = true;
                key += c * stride;
                stride *= g.n[k];
            }
        }
        if (j < n) {
            a.d.kin[(int64_t)s * n + j] = key;
            atomicAdd(&lh[(uint32_t)key >> a.cb], 1u);
            any_bad |= bad;
        }
    }
    if (any_bad) atomicOr(a.d.bad, 1u);
    __syncthreads();
    uint32_t* hist = stag_hist(a, s) + (tile % BKT_SHARDS) * R;
    for (int d = threadIdx.x; d < R; d += blockDim.x)
        if (lh[d]) atomicAdd(&hist[d], lh[d]);
}

template <typename T>
__global__ __launch_bounds__(SORT_BLOCK) void keys_kernel(SortArgs a, const T* __restrict__ X, int soa, int s)
{
    keys_body<T>(a, X, soa != 0, s, blockIdx.x);
}

// ---- decoupled look-back over one counter per tile ------------------------------------
// A chain of stride 1, walked by a whole wave: tile t publishes its own count (flag AGG;
// tile 0 publishes INC), then each round reads the words of up to 64 earlier tiles at once
// and stops at the nearest one that holds an inclusive prefix.  Every earlier tile already
// holds a ticket, so it is running or done and publishes without waiting: the walk always
// ends.  A bounded spin guards against the impossible case.  Called by all 64 lanes of one
// wave; returns the exclusive prefix in every lane.
__device__ __forceinline__ uint32_t lookback_wave(uint32_t* chain, int64_t t, uint32_t mine,
                                                  uint32_t* flag)
{
    const int lane = lane_id();
    if (t == 0) {
        if (lane == 0)
            __hip_atomic_store(&chain[0], LB_INC | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0u;
    }
    if (lane == 0)
        __hip_atomic_store(&chain[t], LB_AGG | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t excl = 0;
    int64_t j = t - 1;  // newest tile of the window; lane l reads tile j - l
    uint32_t spins = 0;
    while (true) {
        const int64_t idx = j - lane;
        // before tile 0: an inclusive prefix of 0, which ends the walk
        const uint32_t v = idx >= 0 ? __hip_atomic_load(&chain[idx], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)
                                    : LB_INC;
        const uint32_t f = v & ~LB_MASK;
        const unsigned long long inc = __ballot(f == LB_INC);
        const unsigned long long pending = __ballot(f == 0u);
        const int stop = inc ? __ffsll((long long)inc) - 1 : 63;  // nearest inclusive prefix
        const unsigned long long upto = stop == 63 ? ~0ull : ((2ull << stop) - 1ull);
        if (pending & upto) {  // a tile in the window has not published yet
            if (++spins > (1u << 22)) {  // never expected; keep the kernel finite
                if (lane == 0) atomicOr(flag, FLAG_LOOKBACK_STALL);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += wave_last_u32(wave_incl_scan_u32(lane <= stop ? (v & LB_MASK) : 0u));
        if (inc) break;
        j -= 64;
    }
    if (lane == 0)
        __hip_atomic_store(&chain[t], LB_INC | (excl + mine), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// ---- a tile's (key, index, position) triples into their buckets -----------------------
// The tile's points are counted per bucket and given slots in LDS, grouped by bucket in
// LDS with their positions (when the pass produces positions in sorted order), and written
// as one contiguous run per bucket into a range that the tile reserves
// with one atomic addition on its shard's cursor of the bucket.  Points of a bucket
// therefore arrive in an order that depends on timing; the bucket kernel restores the
// stable order.
//
// The block finds its shard's start of every bucket from the complete histogram itself (16
// words per bucket, a scan of the bucket totals), so no pass between the keys and the
// scatter is needed; tile 0 also publishes the bucket starts for the bucket pass and
// absorbs the keys pass's bad-point mark (fresh: an update).
template <typename T>
__device__ __forceinline__ void scatter_body(const SortArgs& a, int s, int64_t t, const T* __restrict__ X,
                                             bool soa, const int32_t* __restrict__ psrc, T* __restrict__ Xb,
                                             bool fresh)
{
    constexpr int R_MAX = 1 << max_bucket_bits(sizeof(T) == 8 ? IB_F64 : IB_F32);
    __shared__ int32_t s_key[SORT_TILE];
    __shared__ int32_t s_val[SORT_TILE];
    __shared__ T s_row[SORT_TILE * 3];
    __shared__ uint32_t s_cnt[R_MAX];   // tile count per bucket
    __shared__ uint32_t s_tstart[R_MAX];
    __shared__ uint32_t s_gbase[R_MAX];
    __shared__ uint32_t s_red[SORT_BLOCK / 64 + 1];

    const int tid = threadIdx.x;
    const int rb = a.rb, R = 1 << rb, cb = a.cb;
    const int dim = a.g.dim;
    for (int i = tid; i < R; i += SORT_BLOCK) s_cnt[i] = 0u;
    const int64_t n = a.g.npts;
    const int64_t base = t * SORT_TILE;
    const int nvalid = (int)min((int64_t)SORT_TILE, n - base);
    const int32_t* srck = a.d.kin + (int64_t)s * n;
    int32_t* dstk = a.d.kA + (int64_t)s * n;
    int32_t* dstv = a.d.vA + (int64_t)s * n;
    const int shard = (int)(t % BKT_SHARDS);
    const uint32_t* hist = stag_hist(a, s);
    uint32_t* cur = stag_hist(a, s) + (BKT_SHARDS + shard) * R;
    uint32_t* base_tab = stag_hist(a, s) + 2 * BKT_SHARDS * R;  // [BKT_SHARDS][R]: shard 0 used
    if (t == 0 && tid == 0) absorb_bad_points(a, fresh);

    int32_t key[SORT_IPT], val[SORT_IPT];
    uint32_t slot[SORT_IPT];
    T row[SORT_IPT][3];
    // all loads first, unconditional at clamped in-range indices, so that they overlap
    const int64_t lastp = n - 1, lastx = n * dim - 1;
#pragma unroll
    for (int k = 0; k < SORT_IPT; ++k) {
        const int64_t i = min(base + k * SORT_BLOCK + tid, lastp);
        key[k] = srck[i];
        val[k] = psrc != nullptr ? psrc[i] : (int32_t)i;
    }
    if (Xb != nullptr) {
        const int64_t sr = soa ? 1 : dim, sc = soa ? n : 1;
#pragma unroll
        for (int k = 0; k < SORT_IPT; ++k) {
            const int64_t i = base + k * SORT_BLOCK + tid;
#pragma unroll
            for (int d = 0; d < 3; ++d) row[k][d] = X[min(i * sr + d * sc, lastx)];
        }
    }
    {
        // this shard's start of bucket d (into s_gbase): the points of the buckets below d,
        // and of bucket d in the shards below this tile's; the histogram's loads are in
        // flight with the tile's own
        uint32_t bcarry = 0;
        for (int d0 = 0; d0 < R; d0 += SORT_BLOCK) {
            const int d = d0 + tid;
            uint32_t h[BKT_SHARDS];
#pragma unroll
            for (int x = 0; x < BKT_SHARDS; ++x) h[x] = hist[x * R + min(d, R - 1)];
            uint32_t btot = 0, below = 0;
#pragma unroll
            for (int x = 0; x < BKT_SHARDS; ++x) {
                btot += h[x];
                below += x < shard ? h[x] : 0u;
            }
            if (d >= R) btot = 0;
            uint32_t ball;
            const uint32_t bstart = bcarry + block_excl_scan_u32<SORT_BLOCK>(btot, s_red, &ball);
            bcarry += ball;
            if (d < R) {
                s_gbase[d] = bstart + below;
                if (t == 0) base_tab[d] = bstart;  // the bucket starts (shard 0)
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SORT_IPT; ++k)
        if (k * SORT_BLOCK + tid < nvalid) slot[k] = atomicAdd(&s_cnt[(uint32_t)key[k] >> cb], 1u);
    __syncthreads();
    // the tile's start of each bucket in LDS (scan of the counts) and its reserved range, in
    // rounds of SORT_BLOCK buckets (bucket d0 + t by thread t)
    uint32_t carry = 0;
    for (int d0 = 0; d0 < R; d0 += SORT_BLOCK) {
        const int d = d0 + tid;
        const uint32_t c = d < R ? s_cnt[d] : 0u;
        uint32_t tot;
        const uint32_t run = carry + block_excl_scan_u32<SORT_BLOCK>(c, s_red, &tot);
        if (d < R) {
            s_tstart[d] = run;
            s_gbase[d] = (c ? atomicAdd(&cur[d], c) : 0u) + s_gbase[d];
        }
        carry += tot;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SORT_IPT; ++k) {
        const int li = k * SORT_BLOCK + tid;
        if (li < nvalid) {
            const uint32_t pos = s_tstart[(uint32_t)key[k] >> cb] + slot[k];
            s_key[pos] = key[k];
            s_val[pos] = val[k];
            if (Xb != nullptr) {
#pragma unroll
                for (int d = 0; d < 3; ++d) s_row[pos * 3 + d] = row[k][d];
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < nvalid; i += SORT_BLOCK) {
        const int32_t kk = s_key[i];
        const uint32_t d = (uint32_t)kk >> cb;
        const int64_t dst = (int64_t)s_gbase[d] + (i - (int64_t)s_tstart[d]);
        if (dst >= 0 && dst < n) {  // always true when the counts agree
            dstk[dst] = kk;
            dstv[dst] = s_val[i];
            if (Xb != nullptr) {
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    if (e < dim) Xb[e * n + dst] = s_row[i * 3 + e];  // columns
            }
        }
    }
}

// Built for eight waves per SIMD (at most 64 VGPRs), so that two blocks share a CU.
template <typename T>
__global__ __launch_bounds__(SORT_BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void
radix_scatter_kernel(SortArgs a, int s, const T* __restrict__ X,
                                                                   int soa, const int32_t* __restrict__ psrc,
                                                                   T* __restrict__ Xb, int fresh)
{
    scatter_body<T>(a, s, blockIdx.x, X, soa != 0, psrc, Xb, fresh != 0);
}

// ---- per bucket: counting sort in LDS, cell-start table, positions in sorted order ------
// Bucket b holds the cells [b << cb, (b + 1) << cb) (up to G) and, after the scatter, its
// points at positions [start, start + m) of kA / vA (and Xb).  The block counts its cells'
// points in LDS, scans the counts into the cells' first sorted positions (the cell-start
// table, written for staggering 0), places each point at a slot of its cell taken with an
// LDS atomic, and then moves it to the cell's start plus its rank by index among the cell's
// points.  The result is the stable sort whatever the order of arrival and of the atomics.
constexpr int BKT_THREADS = 1024;

// Common case: at most BKT_CELLS cells and BKT_CAP points, all in LDS, four points per
// thread held in registers throughout.
// The largest of the threads' cell counts into s_cstat[0] and the sum of their counts of
// points in cells of at least CROWD_CELL points into s_cstat[1] (LDS, cleared before the
// block's first barrier): one LDS atomic each per wave.
__device__ __forceinline__ void note_cell_stats(uint32_t vmax, uint32_t crowd, uint32_t* s_cstat)
{
    const int m = wave_max_i32((int)vmax);  // counts are below 2^30
    const uint32_t c = wave_last_u32(wave_incl_scan_u32(crowd));  // below n < 2^31
    if (lane_id() == 0) {
        if (m > 0) atomicMax(&s_cstat[0], (uint32_t)m);
        if (c > 0) atomicAdd(&s_cstat[1], c);
    }
}

// The block's statistics into the plan's (staggering 0 only; after a barrier).
__device__ __forceinline__ void publish_cell_stats(const SortArgs& a, const uint32_t* s_cstat)
{
    if (threadIdx.x == 0) {
        if (s_cstat[0] > 0) atomicMax(a.d.cellmax, s_cstat[0]);
        if (s_cstat[1] > 0) atomicAdd(a.d.crowd, s_cstat[1]);
    }
}

template <typename T>
__device__ __forceinline__ void bucket_fast(const SortArgs& a, int s, int64_t start, int m, int64_t c0,
                                            int nc, bool last, const T* __restrict__ Xb, T* __restrict__ Xs,
                                            int32_t* __restrict__ cstart, uint32_t* hist, int32_t* sidx,
                                            uint16_t* skey, uint32_t* s_red, uint32_t* s_cstat)
{
    constexpr int EPT = BKT_CAP / BKT_THREADS;
    constexpr int CPT = BKT_CELLS / BKT_THREADS;
    const GeomArgs& g = a.g;
    const int dim = g.dim;
    const int64_t n = g.npts;
    const int tid = threadIdx.x;
    const int32_t* __restrict__ ka = a.d.kA + (int64_t)s * n + start;
    const int32_t* __restrict__ va = a.d.vA + (int64_t)s * n + start;
    for (int i = tid; i <= nc; i += BKT_THREADS) hist[i] = 0u;
    if (tid == 0) s_cstat[0] = s_cstat[1] = 0u;
    int32_t key[EPT], idx[EPT];
    int cell[EPT];
    uint32_t slot[EPT];
    T row[EPT][3];
    // loads unconditional at clamped in-range indices (so they overlap); m >= 1 here
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = k * BKT_THREADS + tid;
        const int ec = min(e, m - 1);
        key[k] = ka[ec];
        idx[k] = va[ec];
        // a key outside the bucket never comes from a consistent scatter; keep it in range
        cell[k] = e < m ? (int)min(max((int64_t)key[k] - c0, (int64_t)0), (int64_t)nc - 1) : -1;
        if (Xs != nullptr) {  // columns of the bucket-order positions
#pragma unroll
            for (int d = 0; d < 3; ++d) row[k][d] = Xb[min(d, dim - 1) * n + start + ec];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < EPT; ++k)
        if (cell[k] >= 0) slot[k] = atomicAdd(&hist[cell[k]], 1u);
    __syncthreads();
    uint32_t loc[CPT], sum = 0, lmax = 0, crowd = 0;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int i = tid * CPT + q;
        loc[q] = i < nc ? hist[i] : 0u;
        sum += loc[q];
        lmax = max(lmax, loc[q]);
        crowd += loc[q] >= CROWD_CELL ? loc[q] : 0u;
    }
    if (cstart != nullptr) note_cell_stats(lmax, crowd, s_cstat);
    uint32_t tot;
    uint32_t run = block_excl_scan_u32<BKT_THREADS>(sum, s_red, &tot);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int i = tid * CPT + q;
        if (i < nc) {
            hist[i] = run;
            if (cstart != nullptr) cstart[c0 + i] = (int32_t)(start + run);
        }
        run += loc[q];
    }
    if (tid == 0) {
        hist[nc] = (uint32_t)m;
        if (cstart != nullptr && last) cstart[c0 + nc] = (int32_t)n;
    }
    __syncthreads();
    if (cstart != nullptr) publish_cell_stats(a, s_cstat);
#pragma unroll
    for (int k = 0; k < EPT; ++k)
        if (cell[k] >= 0) {
            const uint32_t pos = hist[cell[k]] + slot[k];
            if (pos < (uint32_t)m) sidx[pos] = idx[k];
        }
    __syncthreads();
    // final place: the cell's start plus the point's rank by index among the cell's points
    int fin[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        fin[k] = -1;
        if (cell[k] >= 0) {
            const uint32_t lo = hist[cell[k]], hi = min(hist[cell[k] + 1], (uint32_t)m);
            uint32_t rank = 0;
            for (uint32_t p = lo; p < hi; ++p) rank += sidx[p] < idx[k] ? 1u : 0u;
            fin[k] = (int)(lo + rank);
        }
    }
    __syncthreads();  // every rank read from sidx before it is overwritten
#pragma unroll
    for (int k = 0; k < EPT; ++k)
        if (fin[k] >= 0 && fin[k] < m) {
            sidx[fin[k]] = idx[k];
            skey[fin[k]] = (uint16_t)cell[k];
            if (Xs != nullptr) {  // within the bucket's range of the output
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    if (d < dim) Xs[d * n + start + fin[k]] = row[k][d];
            }
        }
    __syncthreads();
    // keys and permutation from LDS in sorted order: coalesced writes
    int32_t* ok = a.d.kB + (int64_t)s * n + start;
    int32_t* ov = a.d.vB + (int64_t)s * n + start;
    for (int e = tid; e < m; e += BKT_THREADS) {
        ok[e] = (int32_t)(c0 + skey[e]);
        ov[e] = sidx[e];
    }
}

// General case: a bucket of more cells (BKT_CELLS at a time) or more points, staged in
// place in the output arrays: the key array holds each slot's position in the bucket
// order while each cell's slots are sorted by point index (one thread per cell).
template <typename T>
__device__ __forceinline__ void bucket_general(const SortArgs& a, int s, int64_t start, int64_t m,
                                               int64_t cbeg, int64_t cend, bool last, const T* __restrict__ Xb,
                                               T* __restrict__ Xs, int32_t* __restrict__ cstart,
                                               uint32_t* hist, uint32_t* s_red, uint32_t* s_cstat)
{
    constexpr int CPT = BKT_CELLS / BKT_THREADS;
    const GeomArgs& g = a.g;
    const int dim = g.dim;
    const int64_t n = g.npts;
    const int32_t* __restrict__ ka = a.d.kA + (int64_t)s * n + start;
    const int32_t* __restrict__ va = a.d.vA + (int64_t)s * n + start;
    int32_t* sorg = a.d.kB + (int64_t)s * n + start;  // bucket position of each sorted slot
    int64_t sub_base = 0;
    uint32_t lmax = 0, crowd = 0;
    if (threadIdx.x == 0) s_cstat[0] = s_cstat[1] = 0u;
    for (int64_t c0 = cbeg; c0 < cend; c0 += BKT_CELLS) {
        const int nc = (int)min((int64_t)BKT_CELLS, cend - c0);
        for (int i = threadIdx.x; i < nc; i += BKT_THREADS) hist[i] = 0u;
        __syncthreads();
        for (int64_t e = threadIdx.x; e < m; e += BKT_THREADS) {
            const int64_t c = (int64_t)ka[e] - c0;
            if (c >= 0 && c < nc) atomicAdd(&hist[c], 1u);
        }
        __syncthreads();
        uint32_t loc[CPT];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int i = threadIdx.x * CPT + k;
            loc[k] = i < nc ? hist[i] : 0u;
            sum += loc[k];
            lmax = max(lmax, loc[k]);
            crowd += loc[k] >= CROWD_CELL ? loc[k] : 0u;
        }
        uint32_t tot;
        uint32_t run = block_excl_scan_u32<BKT_THREADS>(sum, s_red, &tot);
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int i = threadIdx.x * CPT + k;
            if (i < nc) {
                hist[i] = (uint32_t)sub_base + run;  // next free slot of the cell
                if (cstart != nullptr) cstart[c0 + i] = (int32_t)(start + sub_base + run);
            }
            run += loc[k];
        }
        __syncthreads();
        for (int64_t e = threadIdx.x; e < m; e += BKT_THREADS) {
            const int64_t c = (int64_t)ka[e] - c0;
            if (c >= 0 && c < nc) {
                const uint32_t pos = atomicAdd(&hist[c], 1u);
                if (pos < (uint64_t)m) sorg[pos] = (int32_t)e;  // always in range when the counts agree
            }
        }
        __syncthreads();
        // hist[i] is now the end of cell i's slots, and hist[i - 1] its start.
        for (int i = threadIdx.x; i < nc; i += BKT_THREADS) {
            const int64_t hi = min((int64_t)hist[i], m);
            const int64_t lo = i > 0 ? (int64_t)hist[i - 1] : sub_base;
            for (int64_t p = lo + 1; p < hi; ++p) {  // insertion sort by point index
                const int32_t v = sorg[p];
                const int32_t vi = va[v];
                int64_t q = p - 1;
                while (q >= lo && va[sorg[q]] > vi) {
                    sorg[q + 1] = sorg[q];
                    --q;
                }
                sorg[q + 1] = v;
            }
        }
        sub_base += tot;
        __syncthreads();
    }
    if (cstart != nullptr && last && threadIdx.x == 0) cstart[cend] = (int32_t)n;
    if (cstart != nullptr) {
        note_cell_stats(lmax, crowd, s_cstat);
        __syncthreads();
        publish_cell_stats(a, s_cstat);
    }
    int32_t* ok = a.d.kB + (int64_t)s * n + start;
    int32_t* ov = a.d.vB + (int64_t)s * n + start;
    for (int64_t p = threadIdx.x; p < m; p += BKT_THREADS) {
        const int64_t e = min((int64_t)(uint32_t)sorg[p], m - 1);  // this thread's own slot
        const int32_t key = ka[e];
        ov[p] = va[e];
        if (Xs != nullptr)
            for (int d = 0; d < dim; ++d) Xs[d * n + start + p] = Xb[d * n + start + e];
        ok[p] = key;  // after the slot's bucket position was read
    }
}

// Bucket b of staggering s (every bucket of the grid's cells has a block).
template <typename T>
__device__ __forceinline__ void bucket_entry(const SortArgs& a, int s, int b, const T* __restrict__ Xb,
                                             T* __restrict__ Xs, int32_t* __restrict__ cstart)
{
    __shared__ uint32_t hist[BKT_CELLS + 1];
    __shared__ int32_t sidx[BKT_CAP];
    __shared__ uint16_t skey[BKT_CAP];  // cell within the bucket
    __shared__ uint32_t s_red[BKT_THREADS / 64 + 1];
    __shared__ uint32_t s_cstat[2];
    static_assert(BKT_CELLS <= 65536, "cells of a bucket fit 16 bits");
    const GeomArgs& g = a.g;
    const int64_t G = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int R = 1 << a.rb;
    const uint32_t* base0 = stag_hist(a, s) + 2 * BKT_SHARDS * R;  // shard 0 = bucket start
    const int64_t n = g.npts;
    const int64_t start = n > 0 ? (int64_t)base0[b] : 0;
    const int64_t m = n > 0 ? (b + 1 < R ? (int64_t)base0[b + 1] : n) - start : 0;
    const int64_t cbeg = (int64_t)b << a.cb;
    const int64_t cend = min(G, (int64_t)(b + 1) << a.cb);
    const bool last = cend == G;
    // Nothing reads this bucket's histogram words and fill cursors (every shard) after the
    // scatter pass: clear them for the staggering's next sort, so that a plan needs the reset
    // kernel only before its first update.  Buckets without a block hold no points, so their
    // words stay zero.
    if ((int)threadIdx.x < 2 * BKT_SHARDS) const_cast<uint32_t*>(stag_hist(a, s))[(int64_t)threadIdx.x * R + b] = 0u;
    if (m >= 1 && m <= BKT_CAP && cend - cbeg <= BKT_CELLS)
        bucket_fast<T>(a, s, start, (int)m, cbeg, (int)(cend - cbeg), last, Xb, Xs, cstart, hist, sidx, skey, s_red,
                       s_cstat);
    else
        bucket_general<T>(a, s, start, m, cbeg, cend, last, Xb, Xs, cstart, hist, s_red, s_cstat);
}

template <typename T>
__global__ __launch_bounds__(BKT_THREADS) void bucket_kernel(SortArgs a, int s, const T* __restrict__ Xb,
                                                             T* __restrict__ Xs, int32_t* __restrict__ cstart)
{
    bucket_entry<T>(a, s, blockIdx.x, Xb, Xs, cstart);
}

// Keys of staggering s in the order of the points (export): keys[perm[i]] = sorted_keys[i].
__global__ __launch_bounds__(256) void keys_out_kernel(SortArgs a, int s, int32_t* __restrict__ keys)
{
    const int64_t n = a.g.npts;
    const int32_t* sk = a.d.kB + (int64_t)s * n;
    const int32_t* pm = a.d.vB + (int64_t)s * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        keys[clamp_index(pm[i], n)] = sk[i];
}

// The look-back words and the tile tickets of staggering s's runs, cleared before every
// runs pass (grid-stride).
__global__ __launch_bounds__(256) void runs_clear_kernel(SortArgs a, int s)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nseg_tiles;
         i += (int64_t)gridDim.x * blockDim.x)
        a.d.seg_status[(int64_t)s * a.nseg_tiles + i] = 0u;
    if (blockIdx.x == 0 && (int)threadIdx.x < PLAN_COUNTERS) a.d.counters[s * PLAN_COUNTERS + threadIdx.x] = 0u;
}

// ---- runs: heads, q and seg_off from the sorted keys (export) --------------------------
__device__ __forceinline__ void runs_body(const SortArgs& a, int s)
{
    constexpr int NW = SORT_BLOCK / 64;
    constexpr int IPT = SORT_IPT;
    __shared__ uint32_t s_wtot[NW];
    __shared__ uint32_t s_ticket;
    __shared__ uint32_t s_excl;
    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    if (tid == 0) s_ticket = atomicAdd(&a.d.counters[s * PLAN_COUNTERS + 1], 1u);
    __syncthreads();
    const int64_t n = a.g.npts;
    const int64_t t = s_ticket;
    const int64_t base = t * SORT_TILE;
    const int32_t* sk = a.d.kB + (int64_t)s * n;
    int32_t* seg = a.d.seg_off + (int64_t)s * (n + 1);
    uint32_t rank[IPT];
    bool head[IPT];
    uint32_t wrun = 0;
    const unsigned long long below = (1ull << lane) - 1ull;
    int32_t kc[IPT], kp[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int64_t i = base + w * (64 * IPT) + k * 64 + lane;
        kc[k] = i < n ? sk[i] : 0;
        kp[k] = (i < n && i > 0) ? sk[i - 1] : -1;
    }
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int64_t i = base + w * (64 * IPT) + k * 64 + lane;
        const bool hd = i < n && (i == 0 || kc[k] != kp[k]);
        const unsigned long long msk = __ballot(hd);
        head[k] = hd;
        rank[k] = wrun + (uint32_t)__popcll(msk & below);
        wrun += (uint32_t)__popcll(msk);
    }
    if (lane == 0) s_wtot[w] = wrun;
    __syncthreads();
    if (w == 0) {  // the whole first wave walks the look-back chain
        uint32_t wt[NW], run = 0;
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            wt[v] = s_wtot[v];
            run += wt[v];
        }
        uint32_t* chain = a.d.seg_status + (int64_t)s * a.nseg_tiles;
        const uint32_t excl = lookback_wave(chain, t, run, a.d.flag);
        if (lane == 0) {
            uint32_t r = 0;
            for (int v = 0; v < NW; ++v) {
                s_wtot[v] = r;
                r += wt[v];
            }
            s_excl = excl;
            if (t == a.nseg_tiles - 1) {
                const uint32_t q = excl + run;
                a.d.q[s] = (int32_t)q;
                seg[q] = (int32_t)n;
            }
        }
    }
    __syncthreads();
    const uint32_t off = s_excl + s_wtot[w];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int64_t i = base + w * (64 * IPT) + k * 64 + lane;
        if (head[k]) seg[off + rank[k]] = (int32_t)i;
    }
}

__global__ __launch_bounds__(SORT_BLOCK) void runs_kernel(SortArgs a, int s)
{
    runs_body(a, s);
}

// ---- batched plan stages ----------------------------------------------------------------

// Job of virtual block vb: the last j with starts[j] <= vb (jobs without blocks in a stage
// have starts[j] == starts[j + 1] and are passed over).
__device__ __forceinline__ int batch_job(const int32_t* starts, int njobs, int vb)
{
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (starts[mid] <= vb) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void batch_reset_kernel(const BatchJob* __restrict__ jobs,
                                                          const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_RESET];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job(st, nj, vb);
        const PlanDev& d = jobs[j].sa.d;
        plan_reset_body(d.zero_begin, d.zero_words, vb - st[j], st[j + 1] - st[j]);
    }
}

template <typename T>
__global__ __launch_bounds__(SORT_BLOCK) void batch_keys_kernel(const BatchJob* __restrict__ jobs,
                                                                const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_KEYS];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job(st, nj, vb);
        keys_body<T>(jobs[j].sa, (const T*)jobs[j].op.X, false, 0, vb - st[j]);
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(SORT_BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void batch_scatter_kernel(const BatchJob* __restrict__ jobs,
                                                                   const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_SCATTER];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job(st, nj, vb);
        const BatchJob& J = jobs[j];
        scatter_body<T>(J.sa, 0, vb - st[j], (const T*)J.op.X, false, nullptr, (T*)J.sa.d.Xb, true);
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(BKT_THREADS) void batch_bucket_kernel(const BatchJob* __restrict__ jobs,
                                                                  const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_BUCKET];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job(st, nj, vb);
        const BatchJob& J = jobs[j];
        bucket_entry<T>(J.sa, 0, vb - st[j], (const T*)J.sa.d.Xb, (T*)J.sa.d.Xs, J.sa.d.cstart);
        __syncthreads();
    }
}

hipError_t launch_batch_plan(const BatchLaunch& b, hipStream_t st)
{
    if (b.grid[BS_RESET] > 0)
        hipLaunchKernelGGL(batch_reset_kernel, dim3(b.grid[BS_RESET]), dim3(256), 0, st, b.jobs, b.table);
    if (b.grid[BS_KEYS] > 0) {
        if (b.dtype == IB_F64)
            hipLaunchKernelGGL(batch_keys_kernel<double>, dim3(b.grid[BS_KEYS]), dim3(SORT_BLOCK), 0, st,
                               b.jobs, b.table);
        else
            hipLaunchKernelGGL(batch_keys_kernel<float>, dim3(b.grid[BS_KEYS]), dim3(SORT_BLOCK), 0, st,
                               b.jobs, b.table);
    }
    if (b.grid[BS_SCATTER] > 0) {
        if (b.dtype == IB_F64)
            hipLaunchKernelGGL(batch_scatter_kernel<double>, dim3(b.grid[BS_SCATTER]), dim3(SORT_BLOCK), 0,
                               st, b.jobs, b.table);
        else
            hipLaunchKernelGGL(batch_scatter_kernel<float>, dim3(b.grid[BS_SCATTER]), dim3(SORT_BLOCK), 0,
                               st, b.jobs, b.table);
    }
    if (b.grid[BS_BUCKET] > 0) {
        if (b.dtype == IB_F64)
            hipLaunchKernelGGL(batch_bucket_kernel<double>, dim3(b.grid[BS_BUCKET]), dim3(BKT_THREADS), 0,
                               st, b.jobs, b.table);
        else
            hipLaunchKernelGGL(batch_bucket_kernel<float>, dim3(b.grid[BS_BUCKET]), dim3(BKT_THREADS), 0,
                               st, b.jobs, b.table);
    }
    return hipGetLastError();
}

// ---- host side ---------------------------------------------------------------------------

int reset_blocks(const SortArgs& a)
{
    return (int)min((size_t)1024, (a.d.zero_words + 255) / 256);
}

int keys_blocks(const SortArgs& a) { return a.g.npts > 0 ? (int)a.ntiles : 0; }

int bucket_blocks(const SortArgs& a)
{
    const int64_t G = (int64_t)a.g.n[0] * a.g.n[1] * a.g.n[2];
    return (int)((G + ((int64_t)1 << a.cb) - 1) >> a.cb);
}

hipError_t launch_plan_reset(const SortArgs& a, hipStream_t st)
{
    const int blocks = reset_blocks(a);
    if (blocks > 0)
        hipLaunchKernelGGL(plan_reset_kernel, dim3(blocks), dim3(256), 0, st, a.d.zero_begin,
                           a.d.zero_words);
    return hipGetLastError();
}

hipError_t launch_sort_stagger(const SortArgs& a, int s, int dtype, const void* X, const int32_t* psrc,
                               bool outputs0, hipStream_t st)
{
    const int64_t n = a.g.npts;
    void* Xb = outputs0 ? a.d.Xb : nullptr;  // positions carried into sorted order
    const int soa = psrc != nullptr ? 1 : 0;  // the plan's own arrays are columns
    if (n > 0) {
        if (dtype == IB_F64) {
            hipLaunchKernelGGL(keys_kernel<double>, dim3((unsigned)a.ntiles), dim3(SORT_BLOCK), 0, st, a,
                               (const double*)X, soa, s);
            hipLaunchKernelGGL(radix_scatter_kernel<double>, dim3((unsigned)a.ntiles), dim3(SORT_BLOCK), 0, st,
                               a, s, (const double*)X, soa, psrc, (double*)Xb, outputs0 ? 1 : 0);
        } else {
            hipLaunchKernelGGL(keys_kernel<float>, dim3((unsigned)a.ntiles), dim3(SORT_BLOCK), 0, st, a,
                               (const float*)X, soa, s);
            hipLaunchKernelGGL(radix_scatter_kernel<float>, dim3((unsigned)a.ntiles), dim3(SORT_BLOCK), 0, st,
                               a, s, (const float*)X, soa, psrc, (float*)Xb, outputs0 ? 1 : 0);
        }
    }
    // The buckets write the cell-start table even without points (every cell starts at 0).
    int32_t* cs = outputs0 ? a.d.cstart : nullptr;
    const dim3 grid((unsigned)bucket_blocks(a));
    if (dtype == IB_F64)
        hipLaunchKernelGGL(bucket_kernel<double>, grid, dim3(BKT_THREADS), 0, st, a, s, (const double*)Xb,
                           outputs0 ? (double*)a.d.Xs : nullptr, cs);
    else
        hipLaunchKernelGGL(bucket_kernel<float>, grid, dim3(BKT_THREADS), 0, st, a, s, (const float*)Xb,
                           outputs0 ? (float*)a.d.Xs : nullptr, cs);
    return hipGetLastError();
}

hipError_t launch_keys_out(const SortArgs& a, int s, int32_t* keys, hipStream_t st)
{
    if (a.g.npts == 0) return hipSuccess;
    const unsigned nb = (unsigned)min((int64_t)4096, (a.g.npts + 255) / 256);
    hipLaunchKernelGGL(keys_out_kernel, dim3(nb), dim3(256), 0, st, a, s, keys);
    return hipGetLastError();
}

hipError_t launch_runs(const SortArgs& a, int s, hipStream_t st)
{
    const int64_t nc64 = (a.nseg_tiles + 255) / 256;
    const unsigned nc = (unsigned)(nc64 < 64 ? (nc64 > 0 ? nc64 : 1) : 64);
    hipLaunchKernelGGL(runs_clear_kernel, dim3(nc), dim3(256), 0, st, a, s);
    hipLaunchKernelGGL(runs_kernel, dim3((unsigned)a.nseg_tiles), dim3(SORT_BLOCK), 0, st, a, s);
    return hipGetLastError();
}

}  // namespace ibk
