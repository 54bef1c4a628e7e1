// Plan kernels: cell keys, stable LSD radix sort of (key, index) pairs, and segments.
//
// These are the preparatory steps of the parallel spreading algorithm (Alg. 4, Sec. 3.3):
// one key per IB point from the cell it occupies, a key-value sort of the point indices
// that groups equal keys, the count of distinct keys and where each run starts (Fig. 2).
// The sort is stable, so the permutation is unique: ties keep input order.
//
// gfx950 design.  Only ceil(log2(#cells)) key bits are sorted, in passes of at most 8 bits,
// over tiles of SORT_TILE (2048) keys.  Within a tile, keys are ranked stably with wave64
// ballots and staged in LDS in digit order, so the global writes are contiguous runs per
// digit.  Where a tile's run of a digit goes comes from one of two schemes:
//   plans    three launches per pass: per-tile digit counts stored digit-major, one
//            exclusive scan over them (its blocks chained by a wave-parallel look-back),
//            and the ranked scatter;
//   batches  one launch per pass ("one-sweep"): digit histograms of every pass from the
//            keys kernel, and per digit a decoupled look-back over the earlier tiles.
// Both give the same permutation.
#include "device_common.h"

namespace ibk {

// ---- reset: clear histograms, look-back words, tickets and the error flag -------------
__device__ __forceinline__ void plan_reset_body(uint32_t* __restrict__ p, size_t nwords, int bid, int nblk)
{
    for (size_t i = (size_t)bid * blockDim.x + threadIdx.x; i < nwords; i += (size_t)nblk * blockDim.x)
        p[i] = 0u;
}

__global__ void plan_reset_kernel(uint32_t* __restrict__ p, size_t nwords)
{
    plan_reset_body(p, nwords, blockIdx.x, gridDim.x);
}

// ---- keys: one per point and distinct staggering, plus all pass histograms ----------
// Keys of staggerings [s0, s1) and their digit histograms for every pass.
template <typename T>
__device__ __forceinline__ void keys_body(const SortArgs& a, const T* __restrict__ X, int bid, int nblk, int s0,
                          int s1)
{
    extern __shared__ uint32_t lhist[];  // [s1 - s0][npass][R]
    const GeomArgs& g = a.g;
    const int R = 1 << a.rbits;
    const int nh = (s1 - s0) * a.npass * R;
    for (int i = threadIdx.x; i < nh; i += blockDim.x) lhist[i] = 0u;
    __syncthreads();

    const int64_t n = g.npts;
    bool any_bad = false;
    // Each thread takes KU points per round, all positions loaded before any is keyed, so
    // the loads of a round are in flight together.
    constexpr int KU = 4;
    const int64_t step = (int64_t)nblk * blockDim.x;
    for (int64_t j0 = (int64_t)bid * blockDim.x + threadIdx.x; j0 < n; j0 += KU * step) {
        T xs[KU][3];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int64_t j = j0 + u * step;
#pragma unroll
            for (int k = 0; k < 3; ++k) xs[u][k] = (j < n && k < g.dim) ? X[j * g.dim + k] : T(0);
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int64_t j = j0 + u * step;
            if (j >= n) break;
            const T* x = xs[u];
            bool bad = false;
            for (int s = s0; s < s1; ++s) {
                int key = 0, stride = 1;
                for (int k = 0; k < g.dim; ++k) {
                    const T y = shifted_scaled<T>(x[k], Prec<T>::inv_h(g, k), (T)g.stag_xi[s][k]);
                    int c = 0;
                    if (fabs(y) < T(1073741824.0)) c = floor_mod((double)floor(y), g.n[k], g.inv_n[k]);
                    else bad = true;
                    key += c * stride;
                    stride *= g.n[k];
                }
                a.d.keys0[(int64_t)s * n + j] = key;
                if (!a.scanned)  // one-sweep passes take digit histograms from here
                    for (int p = 0; p < a.npass; ++p)
                    atomicAdd(&lhist[((s - s0) * a.npass + p) * R + ((key >> (p * a.rbits)) & (R - 1))], 1u);
            }
            any_bad |= bad;
        }
    }
    if (any_bad) atomicOr(a.d.flag, FLAG_BAD_POINT);
    __syncthreads();
    uint32_t* gh = a.d.hist + (size_t)s0 * a.npass * R;
    if (!a.scanned)
        for (int i = threadIdx.x; i < nh; i += blockDim.x)
            if (lhist[i]) atomicAdd(&gh[i], lhist[i]);
}

template <typename T>
__global__ __launch_bounds__(256) void keys_kernel(SortArgs a, const T* __restrict__ X, int s0, int s1)
{
    keys_body<T>(a, X, blockIdx.x, gridDim.x, s0, s1);
}

// ---- decoupled look-back over one counter per tile ------------------------------------
// Tile `t` of a chain publishes its own count first (flag AGG; tile 0 publishes INC), then
// walks back over earlier tiles, summing AGG counts until it meets an INC prefix.  Every
// earlier tile already holds a ticket, so it is running or done and publishes without
// waiting: the walk always ends.  A bounded spin guards against the impossible case.
__device__ __forceinline__ uint32_t lookback_strided(uint32_t* chain, int64_t stride, int64_t t,
                                                     uint32_t mine, uint32_t* flag)
{
    if (t == 0) {
        __hip_atomic_store(&chain[0], LB_INC | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0u;
    }
    __hip_atomic_store(&chain[t * stride], LB_AGG | mine, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    uint32_t excl = 0;
    int64_t j = t - 1;
    uint32_t spins = 0;
    while (true) {
        uint32_t v = __hip_atomic_load(&chain[j * stride], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        uint32_t f = v & ~LB_MASK;
        if (f == 0u) {
            if (++spins > (1u << 22)) {  // never expected; keep the kernel finite
                atomicOr(flag, FLAG_LOOKBACK_STALL);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += v & LB_MASK;
        if (f == LB_INC || j == 0) break;
        --j;
    }
    __hip_atomic_store(&chain[t * stride], LB_INC | (excl + mine), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// The same over a chain of stride 1, walked by a whole wave: each round reads the words of
// up to 64 earlier tiles at once and stops at the nearest one that holds an inclusive
// prefix, so a chain of k tiles takes about k / 64 rounds instead of k reads one after
// another.  Called by all 64 lanes of one wave; returns the exclusive prefix in every lane.
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

// ---- one LSD radix pass over RBITS bits of every staggering's keys --------------------
// SCANNED: tile = block, and each digit's destination base for this tile comes from the
// scanned digit-major tile counts (radix_count_kernel + radix_scan_kernel) instead of the
// digit histogram plus a look-back over earlier tiles.  Both give the same stable order.
template <int RBITS, bool SCANNED = false>
__device__ __forceinline__ void radix_pass_body(const SortArgs& a, int s, int pass)
{
    constexpr int R = 1 << RBITS;
    constexpr int NW = SORT_BLOCK / 64;
    __shared__ int32_t s_key[SORT_TILE];
    __shared__ int32_t s_val[SORT_TILE];
    __shared__ uint32_t s_wcnt[NW][R];
    __shared__ uint32_t s_tstart[R];
    __shared__ uint32_t s_gbase[R];
    __shared__ uint32_t s_excl[R];
    __shared__ uint32_t s_scan[NW + 1];
    __shared__ uint32_t s_ticket;

    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    if (!SCANNED && tid == 0) s_ticket = atomicAdd(&a.d.counters[s * (a.npass + 1) + pass], 1u);
    for (int i = tid; i < NW * R; i += SORT_BLOCK) (&s_wcnt[0][0])[i] = 0u;
    __syncthreads();

    const int64_t n = a.g.npts;
    const int64_t t = SCANNED ? (int64_t)blockIdx.x : (int64_t)s_ticket;
    const int64_t base = t * SORT_TILE;
    const int nvalid = (int)min((int64_t)SORT_TILE, n - base);
    // The digit's global count (one-sweep) or this tile's destination base for the digit
    // (scanned), loaded now so its latency overlaps the ranking.
    const uint32_t* counts = a.d.sort_status + (((int64_t)s * a.npass + pass) * a.ntiles) * R;
    const uint32_t gcount = tid >= R ? 0u
                            : SCANNED ? counts[(int64_t)tid * a.ntiles + t]
                                      : a.d.hist[((int64_t)s * a.npass + pass) * R + tid];

    // Source and destination: pass 0 reads the unsorted keys and generates the indices.
    const int32_t* srck = (pass == 0) ? a.d.keys0 : ((pass & 1) ? a.d.kA : a.d.kB);
    const int32_t* srcv = (pass & 1) ? a.d.vA : a.d.vB;
    int32_t* dstk = (pass & 1) ? a.d.kB : a.d.kA;
    int32_t* dstv = (pass & 1) ? a.d.vB : a.d.vA;
    srck += (int64_t)s * n;
    srcv += (int64_t)s * n;
    dstk += (int64_t)s * n;
    dstv += (int64_t)s * n;
    const int shift = pass * RBITS;

    // Stable in-tile ranking: wave w owns items [w*64*IPT, (w+1)*64*IPT) of the tile, in
    // IPT steps of 64 consecutive items; the rank of an item among equal digits is the
    // count in earlier steps of its wave plus the count of lower lanes in its step.
    int32_t key[SORT_IPT], val[SORT_IPT];
    uint32_t rank[SORT_IPT];
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int k = 0; k < SORT_IPT; ++k) {  // all loads first, so that they overlap
        const int li = w * (64 * SORT_IPT) + k * 64 + lane;
        const bool valid = li < nvalid;
        key[k] = valid ? srck[base + li] : 0;
        val[k] = valid ? (pass == 0 ? (int32_t)(base + li) : srcv[base + li]) : 0;
    }
#pragma unroll
    for (int k = 0; k < SORT_IPT; ++k) {
        const int li = w * (64 * SORT_IPT) + k * 64 + lane;
        const bool valid = li < nvalid;
        const uint32_t digit = ((uint32_t)key[k] >> shift) & (R - 1);
        unsigned long long m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RBITS; ++b) {
            const bool bit = (digit >> b) & 1u;
            const unsigned long long bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t prior = 0;
        if (valid) prior = s_wcnt[w][digit];
        rank[k] = prior + (uint32_t)__popcll(m & below);
        if (valid && lane == 63 - __clzll(m)) s_wcnt[w][digit] = prior + (uint32_t)__popcll(m);
    }
    __syncthreads();

    // Per digit: wave offsets within the tile, the tile count, its exclusive prefix over
    // earlier tiles (look-back), the digit's global base and its start inside the tile.
    uint32_t cnt = 0;
    if (tid < R) {
        for (int v = 0; v < NW; ++v) {
            const uint32_t c = s_wcnt[v][tid];
            s_wcnt[v][tid] = cnt;
            cnt += c;
        }
    }
    uint32_t tot;
    const uint32_t tstart = block_excl_scan_u32<SORT_BLOCK>(tid < R ? cnt : 0u, s_scan, &tot);
    if (SCANNED) {
        if (tid < R) {
            s_tstart[tid] = tstart;
            s_gbase[tid] = gcount;
            s_excl[tid] = 0u;
        }
    } else {
        const uint32_t gbase = block_excl_scan_u32<SORT_BLOCK>(tid < R ? gcount : 0u, s_scan, &tot);
        if (tid < R) {
            s_tstart[tid] = tstart;
            s_gbase[tid] = gbase;
            // Look-back column of this digit: tile-major, digit-minor words.
            uint32_t* col = a.d.sort_status +
                            (((int64_t)s * a.npass + pass) * a.ntiles) * R + tid;
            const uint32_t excl = lookback_strided(col, R, t, cnt, a.d.flag);
            s_excl[tid] = excl;
        }
    }
    __syncthreads();

    // Stage the tile in digit order, then write contiguous runs per digit.
#pragma unroll
    for (int k = 0; k < SORT_IPT; ++k) {
        const int li = w * (64 * SORT_IPT) + k * 64 + lane;
        if (li < nvalid) {
            const uint32_t digit = ((uint32_t)key[k] >> shift) & (R - 1);
            const uint32_t pos = s_tstart[digit] + s_wcnt[w][digit] + rank[k];
            s_key[pos] = key[k];
            s_val[pos] = val[k];
        }
    }
    __syncthreads();
    for (int i = tid; i < nvalid; i += SORT_BLOCK) {
        const int32_t kk = s_key[i];
        const uint32_t digit = ((uint32_t)kk >> shift) & (R - 1);
        const int64_t dst = (int64_t)s_gbase[digit] + s_excl[digit] + (i - (int64_t)s_tstart[digit]);
        if (dst < n) {  // always true when the histograms and tile counts agree
            dstk[dst] = kk;
            dstv[dst] = s_val[i];
        }
    }
}

template <int RBITS>
__global__ __launch_bounds__(SORT_BLOCK) void radix_scatter_kernel(SortArgs a, int s, int pass)
{
    radix_pass_body<RBITS, true>(a, s, pass);
}

// A whole pass in one launch (plans with few points): digit bases from the keys kernel's
// histograms and a decoupled look-back over earlier tiles.
template <int RBITS>
__global__ __launch_bounds__(SORT_BLOCK) void radix_onesweep_kernel(SortArgs a, int s, int pass)
{
    radix_pass_body<RBITS, false>(a, s, pass);
}

// ---- scanned passes: per-tile digit counts, then one exclusive scan over them ---------
// Counts are stored digit-major, counts[digit][tile], so the exclusive scan of the whole
// array is, for each (digit, tile), the position of the tile's first key of that digit in
// the pass's output: all keys of smaller digits, then those of the digit in earlier tiles.
template <int RBITS>
__global__ __launch_bounds__(SORT_BLOCK) void radix_count_kernel(SortArgs a, int s, int pass)
{
    constexpr int R = 1 << RBITS;
    __shared__ uint32_t s_cnt[R];
    const int tid = threadIdx.x;
    for (int i = tid; i < R; i += SORT_BLOCK) s_cnt[i] = 0u;
    __syncthreads();
    const int64_t n = a.g.npts;
    const int64_t t = blockIdx.x;
    const int64_t base = t * SORT_TILE;
    const int nvalid = (int)min((int64_t)SORT_TILE, n - base);
    const int32_t* srck = (pass == 0) ? a.d.keys0 : ((pass & 1) ? a.d.kA : a.d.kB);
    srck += (int64_t)s * n;
    const int shift = pass * RBITS;
    int32_t key[SORT_IPT];
#pragma unroll
    for (int k = 0; k < SORT_IPT; ++k) {
        const int li = k * SORT_BLOCK + tid;
        key[k] = li < nvalid ? srck[base + li] : 0;
    }
#pragma unroll
    for (int k = 0; k < SORT_IPT; ++k)
        if (k * SORT_BLOCK + tid < nvalid) atomicAdd(&s_cnt[((uint32_t)key[k] >> shift) & (R - 1)], 1u);
    __syncthreads();
    uint32_t* counts = a.d.sort_status + (((int64_t)s * a.npass + pass) * a.ntiles) * R;
    for (int d = tid; d < R; d += SORT_BLOCK) counts[(int64_t)d * a.ntiles + t] = s_cnt[d];
}

// In-place exclusive scan of the R * ntiles counts of one pass: SCAN_TILE counts per block,
// blocks in ticket order, the prefix over earlier blocks by look-back.
__global__ __launch_bounds__(SORT_BLOCK) void radix_scan_kernel(SortArgs a, int s, int pass)
{
    __shared__ uint32_t s_scan[SORT_BLOCK / 64 + 1];
    __shared__ uint32_t s_ticket;
    __shared__ uint32_t s_excl;
    const int tid = threadIdx.x;
    if (tid == 0) s_ticket = atomicAdd(&a.d.counters[s * (a.npass + 1) + pass], 1u);
    __syncthreads();
    const int64_t t = s_ticket;
    const int64_t R = int64_t(1) << a.rbits;
    const int64_t V = R * a.ntiles;
    uint32_t* counts = a.d.sort_status + (((int64_t)s * a.npass + pass) * a.ntiles) * R;
    const int64_t first = t * SCAN_TILE + (int64_t)tid * SCAN_VPT;
    uint32_t v[SCAN_VPT];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_VPT; ++k) {
        v[k] = first + k < V ? counts[first + k] : 0u;
        sum += v[k];
    }
    uint32_t btot;
    const uint32_t excl = block_excl_scan_u32<SORT_BLOCK>(sum, s_scan, &btot);
    if (wave_id() == 0) {
        uint32_t* chain = a.d.scan_status + ((int64_t)s * a.npass + pass) * a.nscan_tiles;
        const uint32_t e = lookback_wave(chain, t, btot, a.d.flag);
        if (lane_id() == 0) s_excl = e;
    }
    __syncthreads();
    uint32_t run = s_excl + excl;
#pragma unroll
    for (int k = 0; k < SCAN_VPT; ++k) {
        if (first + k < V) counts[first + k] = run;
        run += v[k];
    }
}

// ---- segments: run heads, q, seg_off and the cell-block start table -------------------
// Rows base + t + k * SORT_BLOCK (k < SEG_IPT) of a tile: dst[i] = src[perm[i]] for rows
// of D values, all permutation entries first, then all rows.
template <typename T, int D, int SEG_IPT>
__device__ __forceinline__ void gather_tile_rows(const int32_t* __restrict__ perm,
                                                 const T* __restrict__ src, T* __restrict__ dst,
                                                 int64_t base, int64_t n)
{
    // Rows past n are neither read nor written (with n == 0, src may be null).
    int64_t p[SEG_IPT];
#pragma unroll
    for (int k = 0; k < SEG_IPT; ++k) {
        const int64_t i = base + threadIdx.x + k * SORT_BLOCK;
        const int32_t v = i < n ? perm[i] : 0;
        p[k] = (uint32_t)v < (uint64_t)n ? v : 0;
    }
    T row[SEG_IPT][D];
#pragma unroll
    for (int k = 0; k < SEG_IPT; ++k) {
        const int64_t i = base + threadIdx.x + k * SORT_BLOCK;
        if (i < n) {
#pragma unroll
            for (int d = 0; d < D; ++d) row[k][d] = src[p[k] * D + d];
        }
    }
#pragma unroll
    for (int k = 0; k < SEG_IPT; ++k) {
        const int64_t i = base + threadIdx.x + k * SORT_BLOCK;
        if (i < n) {
#pragma unroll
            for (int d = 0; d < D; ++d) dst[i * D + d] = row[k][d];
        }
    }
}

constexpr int CB_LANE_RUN = 16;  // table runs up to this long are written by their own lane

template <typename T, int SEG_IPT>
__device__ __forceinline__ void segments_body(const SortArgs& a, int s, const T* __restrict__ X, T* __restrict__ Xs)
{
    // Sorted keys live in the buffer the last pass wrote (A after an odd pass count).
    const bool in_a = (a.g.npts == 0) || (a.npass & 1);
    const int32_t* sk_all = in_a ? a.d.kA : a.d.kB;
    const int32_t* perm_all = in_a ? a.d.vA : a.d.vB;
    constexpr int NW = SORT_BLOCK / 64;
    __shared__ uint32_t s_wtot[NW];
    __shared__ uint32_t s_ticket;
    __shared__ uint32_t s_excl;
    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    if (tid == 0) s_ticket = atomicAdd(&a.d.counters[s * (a.npass + 1) + a.npass], 1u);
    __syncthreads();

    const GeomArgs& g = a.g;
    const int64_t n = g.npts;
    const int64_t t = s_ticket;
    constexpr int SEG_TILE = SORT_BLOCK * SEG_IPT;
    const int64_t base = t * SEG_TILE;
    const int32_t* sk = sk_all + (int64_t)s * n;
    int32_t* seg = a.d.seg_off + (int64_t)s * (n + 1);
    const int64_t nent = (int64_t)g.rows * (g.nbx + 1);
    int32_t* cb = a.d.cblk + (int64_t)s * nent;

    uint32_t rank[SEG_IPT];
    bool head[SEG_IPT];
    uint32_t wrun = 0;
    const unsigned long long below = (1ull << lane) - 1ull;
    // All keys of this thread (and their predecessors) first, so their loads overlap rather
    // than wait behind the table stores below.
    int32_t kcs[SEG_IPT], kps[SEG_IPT];
#pragma unroll
    for (int k = 0; k < SEG_IPT; ++k) {
        const int64_t i = base + w * (64 * SEG_IPT) + k * 64 + lane;
        kcs[k] = i < n ? sk[i] : 0;
        kps[k] = (i < n && i > 0) ? sk[i - 1] : -1;
    }
#pragma unroll
    for (int k = 0; k < SEG_IPT; ++k) {
        const int64_t i = base + w * (64 * SEG_IPT) + k * 64 + lane;
        bool hd = false;
        // Table entries (block(i-1), block(i)] start at sorted position i.  A lane writes a
        // short run itself; longer runs (empty stretches of the grid, e.g. ghost planes or
        // the space between clustered points) are written by the whole wave, one at a time.
        int32_t bp = 0, bc = 0;
        if (i < n) {
            const int32_t kc = kcs[k];
            const int32_t kp = kps[k];
            hd = (i == 0) || (kc != kp);
            bp = i > 0 ? (int32_t)min(cblk_index(kp, g), nent - 1) : -1;
            bc = (int32_t)min(cblk_index(kc, g), nent - 1);
            if (bc - bp <= CB_LANE_RUN)
                for (int32_t e = bp + 1; e <= bc; ++e) cb[e] = (int32_t)i;
        }
        unsigned long long longs = __ballot(bc - bp > CB_LANE_RUN);
        while (longs) {
            const int src = __ffsll((long long)longs) - 1;
            longs &= longs - 1ull;
            const int32_t b0 = __shfl(bp, src, 64) + 1, b1 = __shfl(bc, src, 64);
            const int32_t v = (int32_t)(base + w * (64 * SEG_IPT) + k * 64 + src);
            for (int32_t e = b0 + lane; e <= b1; e += 64) cb[e] = v;
        }
        const unsigned long long m = __ballot(hd);
        head[k] = hd;
        rank[k] = wrun + (uint32_t)__popcll(m & below);
        wrun += (uint32_t)__popcll(m);
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
    // The last tile fills the table entries after the last key with n.
    if (t == a.nseg_tiles - 1) {
        const int64_t blast = n > 0 ? min(cblk_index(sk[n - 1], g), nent - 1) : -1;
        for (int64_t e = blast + 1 + tid; e < nent; e += SORT_BLOCK) cb[e] = (int32_t)n;
    }
    __syncthreads();
    const uint32_t off = s_excl + s_wtot[w];
#pragma unroll
    for (int k = 0; k < SEG_IPT; ++k) {
        const int64_t i = base + w * (64 * SEG_IPT) + k * 64 + lane;
        if (head[k]) seg[off + rank[k]] = (int32_t)i;
    }
    // Positions in this sorted order (staggering 0 only): one row per sorted position, the
    // tile's SEG_IPT rows of a thread loaded together so their random reads overlap.
    if (Xs != nullptr) {
        const int32_t* perm = perm_all + (int64_t)s * n;
        if (g.dim == 3) gather_tile_rows<T, 3, SEG_IPT>(perm, X, Xs, base, n);
        else gather_tile_rows<T, 2, SEG_IPT>(perm, X, Xs, base, n);
    }
}

template <typename T, int SEG_IPT>
__global__ __launch_bounds__(SORT_BLOCK) void segments_kernel(SortArgs a, int s, const T* __restrict__ X,
                                                              T* __restrict__ Xs)
{
    segments_body<T, SEG_IPT>(a, s, X, Xs);
}

// ---- host launchers ---------------------------------------------------------------------
// ---- batched plan stages --------------------------------------------------------------

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
__global__ __launch_bounds__(256) void batch_keys_kernel(const BatchJob* __restrict__ jobs,
                                                                const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_KEYS];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job(st, nj, vb);
        keys_body<T>(jobs[j].sa, (const T*)jobs[j].op.X, vb - st[j], st[j + 1] - st[j], 0, 1);
        __syncthreads();
    }
}

// Radix pass p of every job with more than p passes.  Blocks take tiles by ticket inside
// the body, so only the number of virtual blocks per job (its tile count) matters.
__global__ __launch_bounds__(SORT_BLOCK) void batch_sort_kernel(const BatchJob* __restrict__ jobs,
                                                                const BatchTable* __restrict__ bt,
                                                                int pass)
{
    const int32_t* st = bt->starts[BS_SORT0 + pass];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job(st, nj, vb);
        radix_pass_body<BATCH_RBITS>(jobs[j].sa, 0, pass);
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(SORT_BLOCK) void batch_segments_kernel(
    const BatchJob* __restrict__ jobs, const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_SEG];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job(st, nj, vb);
        const BatchJob& J = jobs[j];
        segments_body<T, SEG_IPT>(J.sa, 0, (const T*)J.op.X, (T*)J.sa.d.Xs);
        __syncthreads();
    }
}

hipError_t launch_batch_plan(const BatchLaunch& b, hipStream_t st)
{
    if (b.grid[BS_RESET] > 0)
        hipLaunchKernelGGL(batch_reset_kernel, dim3(b.grid[BS_RESET]), dim3(256), 0, st, b.jobs, b.table);
    if (b.grid[BS_KEYS] > 0) {
        if (b.dtype == IB_F64)
            hipLaunchKernelGGL(batch_keys_kernel<double>, dim3(b.grid[BS_KEYS]), dim3(256), b.keys_lds,
                               st, b.jobs, b.table);
        else
            hipLaunchKernelGGL(batch_keys_kernel<float>, dim3(b.grid[BS_KEYS]), dim3(256), b.keys_lds,
                               st, b.jobs, b.table);
    }
    for (int p = 0; p < BATCH_MAX_PASSES; ++p)
        if (b.grid[BS_SORT0 + p] > 0)
            hipLaunchKernelGGL(batch_sort_kernel, dim3(b.grid[BS_SORT0 + p]), dim3(SORT_BLOCK), 0, st,
                               b.jobs, b.table, p);
    if (b.grid[BS_SEG] > 0) {
        if (b.dtype == IB_F64)
            hipLaunchKernelGGL(batch_segments_kernel<double>, dim3(b.grid[BS_SEG]), dim3(SORT_BLOCK), 0,
                               st, b.jobs, b.table);
        else
            hipLaunchKernelGGL(batch_segments_kernel<float>, dim3(b.grid[BS_SEG]), dim3(SORT_BLOCK), 0,
                               st, b.jobs, b.table);
    }
    return hipGetLastError();
}

int reset_blocks(const SortArgs& a)
{
    return (int)min((size_t)1024, (a.d.zero_words + 255) / 256);
}

// Few blocks: each adds its LDS histograms to the global ones with atomics.
int keys_blocks(const SortArgs& a)
{
    return a.g.npts > 0 ? (int)min((int64_t)1024, (a.g.npts + 255) / 256) : 0;
}

size_t keys_lds_bytes(const SortArgs& a)  // one staggering at a time
{
    return (size_t)a.npass * ((size_t)1 << a.rbits) * sizeof(uint32_t);
}

hipError_t launch_plan_reset(const SortArgs& a, hipStream_t st)
{
    const int blocks = reset_blocks(a);
    if (blocks > 0)
        hipLaunchKernelGGL(plan_reset_kernel, dim3(blocks), dim3(256), 0, st, a.d.zero_begin,
                           a.d.zero_words);
    return hipGetLastError();
}

hipError_t launch_keys(const SortArgs& a, int dtype, const void* X, int s, hipStream_t st)
{
    const int blocks = keys_blocks(a);
    if (blocks == 0) return hipSuccess;
    const size_t lds = keys_lds_bytes(a);
    if (dtype == IB_F64)
        hipLaunchKernelGGL(keys_kernel<double>, dim3(blocks), dim3(256), lds, st, a, (const double*)X,
                           s, s + 1);
    else
        hipLaunchKernelGGL(keys_kernel<float>, dim3(blocks), dim3(256), lds, st, a, (const float*)X,
                           s, s + 1);
    return hipGetLastError();
}

hipError_t launch_sort_stagger(const SortArgs& a, int s, int dtype, const void* X, bool gather_x,
                               hipStream_t st)
{
    const GeomArgs& g = a.g;
    if (g.npts > 0) {  // scanned passes (three launches each) or one-sweep passes
        const unsigned tiles = (unsigned)a.ntiles, sblocks = (unsigned)a.nscan_tiles;
        for (int p = 0; p < a.npass; ++p) {
            switch (a.rbits) {
#define IBK_SCANNED_PASS(B)                                                                        \
    case B:                                                                                        \
        if (!a.scanned) {                                                                          \
            hipLaunchKernelGGL(radix_onesweep_kernel<B>, dim3(tiles), dim3(SORT_BLOCK), 0, st, a, s, \
                               p);                                                                 \
            break;                                                                                 \
        }                                                                                          \
        hipLaunchKernelGGL(radix_count_kernel<B>, dim3(tiles), dim3(SORT_BLOCK), 0, st, a, s, p);   \
        hipLaunchKernelGGL(radix_scan_kernel, dim3(sblocks), dim3(SORT_BLOCK), 0, st, a, s, p);     \
        hipLaunchKernelGGL(radix_scatter_kernel<B>, dim3(tiles), dim3(SORT_BLOCK), 0, st, a, s, p); \
        break;
            IBK_SCANNED_PASS(4)
            IBK_SCANNED_PASS(5)
            IBK_SCANNED_PASS(6)
            IBK_SCANNED_PASS(7)
            IBK_SCANNED_PASS(8)
#undef IBK_SCANNED_PASS
            default: return hipErrorInvalidValue;
            }
        }
    }
    const dim3 grid((unsigned)a.nseg_tiles);
    const bool small = a.seg_ipt == SEG_IPT_SMALL;
    if (dtype == IB_F64) {
        double* Xs = gather_x ? (double*)a.d.Xs : nullptr;
        if (small)
            hipLaunchKernelGGL((segments_kernel<double, SEG_IPT_SMALL>), grid, dim3(SORT_BLOCK), 0, st,
                               a, s, (const double*)X, Xs);
        else
            hipLaunchKernelGGL((segments_kernel<double, SEG_IPT>), grid, dim3(SORT_BLOCK), 0, st, a,
                               s, (const double*)X, Xs);
    } else {
        float* Xs = gather_x ? (float*)a.d.Xs : nullptr;
        if (small)
            hipLaunchKernelGGL((segments_kernel<float, SEG_IPT_SMALL>), grid, dim3(SORT_BLOCK), 0, st,
                               a, s, (const float*)X, Xs);
        else
            hipLaunchKernelGGL((segments_kernel<float, SEG_IPT>), grid, dim3(SORT_BLOCK), 0, st, a, s,
                               (const float*)X, Xs);
    }
    return hipGetLastError();
}

}  // namespace ibk
