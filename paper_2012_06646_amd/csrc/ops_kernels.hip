// Spreading and interpolation kernels.
//
// Both operators visit the points in the sorted order of staggering 0 (the staggering of
// component 0): the plan stores the positions in that order, spreading reads each point's
// force through the permutation as it loads the point, and interpolation writes each
// point's values once.  So the only scattered memory accesses per call are the force reads
// (spreading) and one scatter of U (interpolation); everything else streams.  A point's cell for component c differs
// from its staggering-0 cell by at most one per dimension, so the tiles below widen their
// halos by that offset.
//
// Spreading (eq. disc-spread, Sec. 2; parallel algorithm Alg. 4, Sec. 3.4).  Each block
// owns a tile of one component's grid and produces every value of it exactly once.  It
// reads the sorted points whose cells can reach the tile (contiguous sorted ranges per
// x-row, since keys are x-fastest), one source plane at a time; a wave takes 64 of them,
// one per lane, computes their separable weights and adds the s^d products (s = 4, or 3
// for the odd-support kernel) into the tile held in LDS.  The sums are exact integer (fixed-point) sums, so their value does not
// depend on the order of the additions: waves and blocks need no ordering among
// themselves, no floating-point atomics are used, and the result is bitwise reproducible.
//
// Interpolation (eq. disc-interp; Alg. 3, Sec. 3.3).  One thread per point in the sorted
// order of staggering 0, gathering the s^d grid values of each component directly
// (neighbouring lanes hold neighbouring cells, so a wave's gathers share cache lines);
// the point's components are accumulated in registers in tensor-product order and
// written together.
#include <algorithm>
#include <type_traits>

#include "device_common.h"

namespace ibk {

// Calls f with the kernel id as a compile-time constant (std::integral_constant), so each
// launch site instantiates its kernels once per supported one-dimensional kernel.
template <typename F>
hipError_t with_kernel(int kernel, F&& f)
{
    switch (kernel) {
    case IB_KERNEL_COSINE4: return f(std::integral_constant<int, IB_KERNEL_COSINE4>{});
    case IB_KERNEL_ROMA3: return f(std::integral_constant<int, IB_KERNEL_ROMA3>{});
    default: return f(std::integral_constant<int, IB_KERNEL_PESKIN4>{});
    }
}

// Tiles of a 3-D grid are numbered with the tile dimensions varying in the cyclic order
// that ends with the slowest one: x, y, z (slowest z), z, x, y (slowest y) or y, z, x
// (slowest x).  Each XCD runs one contiguous range of tiles, so a nearly empty last row of
// tiles along the slowest dimension lands on one XCD and leaves that XCD a further round of
// full tiles after the others have drained (measured: +50 us of spreading on a
// 128 x 128 x 132 grid, whose last z row holds 2 of 13 planes).  z stays slowest, which
// reads the least from HBM (measured on 128^3: 445 MB per spreading launch against 588 MB
// with y slowest), unless its last row is at most half full; then the best-filled dimension
// (cells / tile capacity along it; ties go to z, then y) varies slowest.
__host__ __device__ __forceinline__ int slowest_tile_dim(const int n[3], const int tiles[3],
                                                         const int size[3])
{
    if (2 * (n[2] - (tiles[2] - 1) * size[2]) > size[2]) return 2;
    int s = 2;
    for (int k = 1; k >= 0; --k)  // fill_k > fill_s, cross-multiplied
        if ((int64_t)n[k] * tiles[s] * size[s] > (int64_t)n[s] * tiles[k] * size[k]) s = k;
    return s;
}

__device__ __forceinline__ void tile_coords(int b, const int tiles[3], int s, int& ix, int& iy,
                                            int& iz)
{
    const int t0 = s == 2 ? tiles[0] : s == 1 ? tiles[2] : tiles[1];
    const int t1 = s == 2 ? tiles[1] : s == 1 ? tiles[0] : tiles[2];
    const int i0 = b % t0, r = b / t0;
    const int i1 = r % t1, i2 = r / t1;
    ix = s == 2 ? i0 : s == 1 ? i1 : i2;
    iy = s == 2 ? i1 : s == 1 ? i2 : i0;
    iz = s == 2 ? i2 : s == 1 ? i0 : i1;
}

// Position update of the IB step for one coordinate: x + dt u wrapped into [0, L).
template <typename T>
__device__ __forceinline__ T advect_coord(T x, T u, T dt, T L)
{
    T y = fma(dt, u, x);
    y -= L * floor(y / L);
    if (y >= L || y < T(0)) y = T(0);
    return y;
}

// Weights of a point at coordinates x for component c, times 2^weight_shift<KERN>() each
// (weights_scaled), and the offset of its component-c cell from its staggering-0 cell per
// dimension.  The cells follow the key rule exactly
// (t = x * inv_h rounded once, minus the staggering; then axis_cell).
template <typename T, int DIM, int KERN>
__device__ __forceinline__ void comp_weights(const GeomArgs& g, int c, const T x[DIM],
                                             T w[DIM][4], int delta[DIM])
{
    constexpr bool odd = support_width<KERN>() == 3;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const T ih = Prec<T>::inv_h(g, k);
        const T yc = shifted_scaled<T>(x[k], ih, (T)g.comp_xi[c][k]);
        T r;
        const double fc = axis_cell<T>(yc, odd, &r);
        if (g.dlo[c][k] == g.dhi[c][k]) {
            delta[k] = g.dlo[c][k];  // the same staggering as staggering 0 along this axis
        } else {
            const T y0 = shifted_scaled<T>(x[k], ih, (T)g.stag_xi[0][k]);
            T r0;
            delta[k] = min(max((int)(fc - axis_cell<T>(y0, odd, &r0)), g.dlo[c][k]), g.dhi[c][k]);
        }
        r += product_residual<T>(x[k], ih, Prec<T>::inv_lo(g, k));
        weights_scaled<T, KERN>(r, w[k]);
    }
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------------------
// Spreading
// ---------------------------------------------------------------------------------------
//
// Exact fixed-point accumulation.  Every contribution F_j W to a grid value of a tile is
// rounded once to an integer multiple of 2^-S (S chosen per tile, below) and added to a
// 64-bit integer in LDS.  Integer addition is exact and associative, so the tile's sums do
// not depend on the order in which its points arrive: no wave waits for another, any number
// of blocks may share a tile, and the result is the same bits on every run.  The rounding
// of a contribution is the only error beyond those of the weights.
//
// The scale.  With vmax = max_j |F_{j,c}| < 2^e (all points) and M an upper bound on the
// contributions any one grid value receives (the points of the staggering-0 cells that can
// reach it, at most the largest cell count of the plan times the cells of that window, see
// spread_body), S = min(51 - e, 62 - ceil(log2 M) - e).  Then every
// contribution, scaled by 2^S, has magnitude below 2^51 (so one fused multiply-add with
// 1.5 * 2^52 rounds it to an integer held in the low bits of its result), and no partial
// sum reaches 2^62.  The rounding error of one contribution is at most
// 2^-(S+1) <= M vmax 2^-62 (or vmax 2^-52 when M is small).  Weights are at most 1 for
// every kernel, so |F W| <= vmax.

constexpr double FX_MAGIC = 6755399441055744.0;          // 1.5 * 2^52
constexpr long long FX_MAGIC_BITS = 0x4338000000000000LL; // its bit pattern
constexpr unsigned long long FX_NONFINITE = 0x7FF0000000000000ull;

// Nearest integer to a * b + 0 (|a b| < 2^51), as a two's-complement 64-bit word.
__device__ __forceinline__ unsigned long long fx_round(double a, double b)
{
    const double t = fma(a, b, FX_MAGIC);
    return (unsigned long long)(__double_as_longlong(t) - FX_MAGIC_BITS);
}

// Scale exponent of a tile from the bit pattern of vmax (non-negative, finite, not zero)
// and its bound on contributions per grid value.
__device__ __forceinline__ int fx_shift(unsigned long long vmax_bits, uint32_t nt)
{
    const int E = (int)((vmax_bits >> 52) & 0x7FFu);
    const int e = (E == 0 ? 1 : E) - 1022;  // vmax < 2^e
    const int m = nt <= 1u ? 0 : 32 - __clz((int)(nt - 1u));
    return min(51 - e, 62 - m - e);
}

// Largest |F_{j,c}| per component, as non-negative bit patterns (a NaN or infinity compares
// above every finite value): FMAX_PARTS blocks each write the maxima of their share of the
// rows, and a spreading block takes the maximum of those partial maxima.  The rows are read
// in input order as one flat array of n * NC elements (coalesced); element le of a pass
// belongs to component le mod NC.
constexpr int SPREAD_THREADS = 512;
constexpr int FMAX_THREADS = 256;
constexpr int FMAX_BATCH = 2;  // rows per thread per pass (measured 1.5 us faster than 4 at 10^6 rows)

template <typename T, int NC>
__device__ __forceinline__ void fmax_rows(const T* __restrict__ F, int64_t n, int bid,
                                          unsigned long long m[3])
{
    constexpr int E = NC * FMAX_BATCH;
    constexpr int64_t ROWS = (int64_t)FMAX_THREADS * FMAX_BATCH;
    const int tid = threadIdx.x;
    for (int64_t base = (int64_t)bid * ROWS; base < n; base += (int64_t)FMAX_PARTS * ROWS) {
        const int64_t lim = (n - base) * NC;  // elements left from the pass's first one
        const T* __restrict__ src = F + base * NC;
        T v[E];
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = src[min((int64_t)(k * FMAX_THREADS + tid), lim - 1)];
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int le = k * FMAX_THREADS + tid;
            const int c = le % NC;
            const unsigned long long b =
                le < lim ? (unsigned long long)__double_as_longlong(fabs((double)v[k])) : 0ull;  // exact for FP32
            m[0] = (c == 0 && b > m[0]) ? b : m[0];
            m[1] = (c == 1 && b > m[1]) ? b : m[1];
            m[2] = (c == 2 && b > m[2]) ? b : m[2];
        }
    }
}

template <typename T>
__device__ __forceinline__ void fmax_body(const OpArgs& a, int bid)
{
    __shared__ unsigned long long s_m[3][FMAX_THREADS / 64];
    unsigned long long m[3] = {0ull, 0ull, 0ull};
    const T* F = (const T*)a.F;
    if (a.g.ncomp == 3) fmax_rows<T, 3>(F, a.g.npts, bid, m);
    else if (a.g.ncomp == 2) fmax_rows<T, 2>(F, a.g.npts, bid, m);
    else fmax_rows<T, 1>(F, a.g.npts, bid, m);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int sh = 32; sh >= 1; sh >>= 1) {
            const unsigned long long o = __shfl_xor(m[c], sh, 64);
            m[c] = o > m[c] ? o : m[c];
        }
        if (lane_id() == 0) s_m[c][wave_id()] = m[c];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long r = 0ull;
        for (int w = 0; w < FMAX_THREADS / 64; ++w) r = s_m[threadIdx.x][w] > r ? s_m[threadIdx.x][w] : r;
        ((unsigned long long*)a.fmax)[threadIdx.x * FMAX_PARTS + bid] = r;
    }
}

template <typename T>
__global__ __launch_bounds__(FMAX_THREADS) void fmax_kernel(OpArgs a)
{
    fmax_body<T>(a, blockIdx.x);
}

// Maximum of the FMAX_PARTS partial maxima of component c, uniform over the block: the
// first wave reads them all at once (FMAX_PARTS / 64 per lane) and reduces across its
// lanes; one barrier publishes the result (and whatever the block wrote to LDS before it).
__device__ __forceinline__ unsigned long long fmax_of(const unsigned long long* __restrict__ part,
                                                      int c, unsigned long long* s_red)
{
    static_assert(FMAX_PARTS % 64 == 0, "whole partial maxima per lane");
    if (wave_id() == 0) {
        constexpr int PER = FMAX_PARTS / 64;
        unsigned long long v[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) v[i] = part[c * FMAX_PARTS + i * 64 + lane_id()];
        unsigned long long m = 0ull;
#pragma unroll
        for (int i = 0; i < PER; ++i) m = v[i] > m ? v[i] : m;
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            const unsigned long long o = __shfl_xor(m, s, 64);
            m = o > m ? o : m;
        }
        if (lane_id() == 0) s_red[0] = m;
    }
    __syncthreads();
    return s_red[0];
}

// A source slice (an x-y plane of staggering-0 cells in 3-D, one x-row in 2-D) as a list
// of sorted ranges, one per x-row piece (at most 3 pieces per row, since a tile is never
// wider than the grid), read exactly from the cell-start table.
template <int MAXR>
struct SliceTable {
    int32_t lo[MAXR];
    int32_t hi[MAXR];
    int32_t base[MAXR];   // sorted index of slice position v in range r: base[r] + v
    int32_t xo[MAXR];     // source-frame x of a key: key + xo
    int32_t uy[MAXR];     // source-frame y of the row
    int32_t pref[MAXR + 1];
};

template <typename T, int DIM, int KERN, int TX, int TY, int TZ>
struct SpreadTile {
    static constexpr int PXS = TX + 6;  // padded row pitch of the LDS tile (x from -3 to TX + 2)
    static constexpr int SW = support_width<KERN>();         // stencil nodes per dimension
    static constexpr int NZ = (DIM == 3) ? SW : 1;           // stencil extent in z
    static constexpr int MAXROWS = (DIM == 3) ? TY + 5 : 1;   // x-rows per slice
    static constexpr int MAXR = 3 * MAXROWS;
    static constexpr int CELLS = PXS * TY * TZ;               // LDS tile words
    static_assert(MAXR <= 64, "one lane per range of a slice");
    static_assert(3 * ((DIM == 3 ? TY * PXS * 8 : 0) + PXS * 8) + 24 < 65536,
                  "stencil offsets fit the LDS instruction offset field");
    using Table = SliceTable<MAXR>;

    // Range table of source slice q (frame origin ox, oy, oz; lenx cells per row, nrows
    // rows); returns the slice's point count.  Afterwards lane r < 3 * nrows holds range r's
    // first slice position (*rp) and whether the range is non-empty (*rn).
    __device__ static int build(const GeomArgs& g, const int32_t* __restrict__ cs, int q, int ox,
                                int oy, int oz, int lenx, int nrows, Table& tb, int* rp, bool* rn)
    {
        const int lane = lane_id();
        const int n0 = g.n[0];
        int count = 0;
        if (lane < nrows) {
            int r, uy;
            if (DIM == 3) {
                const int cz = wrap_small(oz + q, g.n[2]);
                uy = lane;
                r = cz * g.n[1] + wrap_small(oy + lane, g.n[1]);
            } else {
                uy = q;
                r = wrap_small(oy + q, g.n[1]);
            }
            const int32_t rowbase = r * n0;
            int done = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                int32_t lo = 0, hi = 0, xo = 0;
                if (done < lenx) {
                    const int xa = wrap_small(ox + done, n0);
                    const int len = min(lenx - done, n0 - xa);
                    lo = cs[rowbase + xa];
                    hi = cs[rowbase + xa + len];
                    xo = done - xa - rowbase;
                    done += len;
                }
                tb.lo[lane * 3 + k] = lo;
                tb.hi[lane * 3 + k] = hi;
                tb.xo[lane * 3 + k] = xo;
                tb.uy[lane * 3 + k] = uy;
                count += hi - lo;
            }
        }
        const uint32_t incl = wave_incl_scan_u32((uint32_t)count);
        if (lane < nrows) {
            int run = (int)incl - count;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                tb.pref[lane * 3 + k] = run;
                tb.base[lane * 3 + k] = tb.lo[lane * 3 + k] - run;
                run += tb.hi[lane * 3 + k] - tb.lo[lane * 3 + k];
            }
        }
        const int total_pts = (int)wave_last_u32(incl);
        if (lane == 0) tb.pref[nrows * 3] = total_pts;
        wave_sync();
        const int nranges = 3 * nrows;
        *rp = lane < nranges ? tb.pref[lane] : total_pts;
        *rn = lane < nranges && tb.hi[lane] > tb.lo[lane];
        wave_sync();
        return total_pts;
    }

    // Range of slice position v0 + lane, for v0 < total.  The range holding v0 is the last
    // one whose first position is <= v0 (it is non-empty); the non-empty ranges starting
    // inside the chunk are marked at their offsets, and a prefix maximum over the lanes
    // carries each mark up to the next one.  Called by the whole wave.
    __device__ static int locate(int32_t* mark, int rp, bool rn, int nranges, int v0)
    {
        const int lane = lane_id();
        const int carry = (int)__popcll(__ballot(lane < nranges && rp <= v0)) - 1;
        mark[lane] = 0;
        wave_sync();
        const int s = rp - v0;
        if (rn && s > 0 && s < 64) mark[s] = lane + 1;  // distinct offsets: non-empty ranges
        wave_sync();
        const int m = (int)wave_incl_max_u32((uint32_t)mark[lane]);
        wave_sync();
        return max(m - 1, carry);
    }

    // Slice positions v0 + lane: range, key, coordinates and force (zeros past the end).
    // The sorted index is kept inside [0, n) whatever the tables hold.  Called by the whole
    // wave.
    __device__ static void load(const OpArgs& a, int c, const int32_t* __restrict__ sk,
                                const Table& tb, int32_t* mark, int rp, bool rn, int nranges,
                                int total, int v0, int& rr, int32_t& key, T x[DIM], T& F)
    {
        // Lane l takes chunk position 4 (l mod 16) + l / 16: the LDS unit serves a wave's
        // 64-bit additions 16 lanes at a time, and consecutive sorted points (which often
        // share a cell, i.e. all 4^d target addresses) then fall into different groups.
        const int pos = chunk_pos(lane_id());
        rr = __shfl(locate(mark, rp, rn, nranges, v0), pos, 64);
        key = 0;
        F = T(0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) x[k] = T(0);
        const int v = v0 + pos;
        if (v < total) {
            const int64_t j = clamp_index(tb.base[rr] + v, a.g.npts);
            const T* __restrict__ Xs = (const T*)a.Xs;
            key = sk[j];
#pragma unroll
            for (int k = 0; k < DIM; ++k) x[k] = Xs[k * a.g.npts + j];  // columns
            // the force of the point, read through the permutation (its input-order row)
            F = ((const T*)a.F)[clamp_index(a.perm[j], a.g.npts) * a.g.ncomp + c];
        }
    }

    __device__ static int chunk_pos(int lane) { return ((lane & 15) << 2) | (lane >> 4); }

    // Add the SW^d contributions of every lane's point (lanes with has) into the tile, as
    // fixed-point integers.  Tile rows are padded in x (PXS = TX + 6, target x from -3 to
    // TX + 2), so only whole rows can fall outside the tile; those are skipped.
    // ROT: lane l adds its x-nodes of a row starting at (l mod 4) mod SW, so up to four lanes
    // of one 16-lane group that hold points of one cell (crowded cells) add to different
    // addresses at each instruction; the set of adds, and so every sum, is the same.
    template <bool ROT>
    __device__ static void add_point(const T w[DIM][4], double Fs, bool has, int cx, int cy, int cz,
                                     int ey, int ez, unsigned long long* tile)
    {
        const int zb = (DIM == 3) ? cz - 1 : 0, yb = cy - 1;
        const int base = (zb * TY + yb) * PXS + (cx + 2);
        double wz[4];
#pragma unroll
        for (int i = 0; i < SW; ++i) wz[i] = (DIM == 3) ? (double)w[DIM - 1][i] * Fs : 0.0;
        bool oka[4], okb[4];
#pragma unroll
        for (int i = 0; i < SW; ++i) {
            oka[i] = has && ((DIM == 3) ? (unsigned)(zb + i) < (unsigned)ez
                                        : (unsigned)(yb + i) < (unsigned)ey);
            okb[i] = (DIM == 3) ? (unsigned)(yb + i) < (unsigned)ey : i == 0;
        }
        double wx[4];
        int xo[4];
        const int rot = ROT ? (lane_id() & 3) % SW : 0;
#pragma unroll
        for (int ix = 0; ix < SW; ++ix) {
            double v = (double)w[0][ix];
            if (ROT) {
#pragma unroll
                for (int r = 1; r < SW; ++r) v = rot == r ? (double)w[0][(ix + r) % SW] : v;
            }
            wx[ix] = v;
            xo[ix] = ROT ? (ix + rot) % SW : ix;
        }
#pragma unroll
        for (int ia = 0; ia < SW; ++ia)
#pragma unroll
            for (int ib = 0; ib < ((DIM == 3) ? SW : 1); ++ib) {
                if (oka[ia] && okb[ib]) {
                    const double cyz = (DIM == 3) ? (double)w[1][ib] * wz[ia] : (double)w[1][ia] * Fs;
                    unsigned long long* row =
                        tile + base + ((DIM == 3) ? (ia * TY + ib) * PXS : ia * PXS);
#pragma unroll
                    for (int ix = 0; ix < SW; ++ix)
                        __hip_atomic_fetch_add(row + xo[ix], fx_round(wx[ix], cyz),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
    }

    // Add the slice's points, in chunks of 64 (one point per lane), into the tile.
    // off[k] = SW - 2 + dhi[k]: a point's tile-relative component-c cell is its source-frame
    // staggering-0 cell + delta - off.
    template <bool ROT>
    __device__ static void spread_slice(const OpArgs& a, int c, const Table& tb, int32_t* mark,
                                        int rp, bool rn, int nranges, int total, int q,
                                        const int off[3], int ex, int ey, int ez, int fshift,
                                        unsigned long long* tile, int k0, int kstride)
    {
        const GeomArgs& g = a.g;
        const int lane = lane_id();
        const int32_t* __restrict__ sk = a.sorted_keys;
        // Chunk data is loaded one chunk ahead, so its latency overlaps the current chunk.
        int nrr = 0;
        int32_t nkey = 0;
        T nx[DIM], nF = T(0);
        const int step = 64 * kstride;
        if (64 * k0 < total) load(a, c, sk, tb, mark, rp, rn, nranges, total, 64 * k0, nrr, nkey, nx, nF);
        for (int v0 = 64 * k0; v0 < total; v0 += step) {
            const bool valid = v0 + chunk_pos(lane) < total;
            const int rr = nrr;
            const int32_t key = nkey;
            T x[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) x[k] = nx[k];
            const T Fc = nF;
            if (v0 + step < total)
                load(a, c, sk, tb, mark, rp, rn, nranges, total, v0 + step, nrr, nkey, nx, nF);
            T w[DIM][4];
            int delta[DIM];
            comp_weights<T, DIM, KERN>(g, c, x, w, delta);
            const int cx = key + tb.xo[rr] + delta[0] - off[0];
            const int cy = tb.uy[rr] + delta[1] - off[1];
            const int cz = (DIM == 3) ? q + delta[DIM - 1] - off[2] : 0;
            const bool has = valid && cx >= 2 - SW && cx <= ex && cy >= 2 - SW && cy <= ey &&
                             (DIM == 2 || (cz >= 2 - SW && cz <= ez));
            add_point<ROT>(w, ldexp((double)Fc, fshift - DIM * weight_shift<KERN>()), has, cx, cy,
                           cz, ey, ez, tile);
        }
    }
};

// Component and first cell of spreading tile `tile_id`: tiles are numbered with the
// component fastest, then x, y, z.
template <int TX, int TY, int TZ>
__device__ __forceinline__ void spread_tile_at(const OpArgs& a, int tile_id, int& c, int& x0,
                                               int& y0, int& z0)
{
    int b = tile_id;
    c = b % a.g.ncomp;
    b /= a.g.ncomp;
    int ix, iy, iz;
    tile_coords(b, a.tiles, a.tile_slow, ix, iy, iz);
    x0 = ix * TX;
    y0 = iy * TY;
    z0 = iz * TZ;
}

// The grid value of one tile cell from its fixed-point sum: sum 2^-S h^-d, or NaN when a
// force was not finite.
template <typename T>
__device__ __forceinline__ T fx_value(unsigned long long acc, int fshift, bool finite, double scale)
{
    if (!finite) return T(__builtin_nan(""));
    return (T)(ldexp((double)(long long)acc, -fshift) * scale);
}

// LDS of a spreading block, declared once per kernel whichever order of adds it runs.
template <typename ST>
struct SpreadShared {
    static constexpr int NW = SPREAD_THREADS / 64;  // waves per block
    unsigned long long tile[ST::CELLS];
    typename ST::Table tables[NW];
    int32_t marks[NW][64];
    unsigned long long s_red[NW];
};

template <typename T, int DIM, int KERN, int TX, int TY, int TZ, bool ROT>
__device__ __forceinline__ void spread_body(const OpArgs& a, int bid,
                                            SpreadShared<SpreadTile<T, DIM, KERN, TX, TY, TZ>>& sm)
{
    using ST = SpreadTile<T, DIM, KERN, TX, TY, TZ>;
    constexpr int NW = SPREAD_THREADS / 64;  // waves per block
    unsigned long long* tile = sm.tile;
    auto& tables = sm.tables;
    auto& marks = sm.marks;
    unsigned long long* s_red = sm.s_red;
    const GeomArgs& g = a.g;
    // Blocks bid = tile * split + k: the split blocks of a tile each take every split-th
    // chunk of its points and publish their partial integer sums.  Tiles are numbered with
    // the component fastest, then the three dimensions (spread_tile_at): the components of
    // one region, and neighbouring regions, run close together and (through xcd_block) on
    // one XCD, so the points and forces that their source frames share are read from HBM
    // once and then from that L2.
    const int split = g.split;
    const int tile_id = bid / split, ksub = bid - tile_id * split;
    int c, x0, y0, z0;
    spread_tile_at<TX, TY, TZ>(a, tile_id, c, x0, y0, z0);
    const int ex = min(TX, g.n[0] - x0), ey = min(TY, g.n[1] - y0);
    const int ez = (DIM == 3) ? min(TZ, g.n[2] - z0) : 1;

    for (int i = threadIdx.x; i < ST::CELLS; i += blockDim.x) tile[i] = 0ull;

    // Source frame: staggering-0 cells that can reach the tile for this component.  The
    // nodes of a point with component-c cell i are i - 1 .. i + SW - 2, so a tile node m
    // receives from cells m - SW + 2 .. m + 1, and staggering-0 cells lie delta below.
    constexpr int SW = ST::SW;
    const int hx = g.dhi[c][0] - g.dlo[c][0], hy = g.dhi[c][1] - g.dlo[c][1];
    const int hz = (DIM == 3) ? g.dhi[c][2] - g.dlo[c][2] : 0;
    const int off[3] = {SW - 2 + g.dhi[c][0], SW - 2 + g.dhi[c][1], (DIM == 3) ? SW - 2 + g.dhi[c][2] : 0};
    const int ox = x0 - off[0], oy = y0 - off[1], oz = (DIM == 3) ? z0 - off[2] : 0;
    const int lenx = ex + SW - 1 + hx;
    const int nrows = (DIM == 3) ? ey + SW - 1 + hy : 1;
    const int nslices = (DIM == 3) ? ez + SW - 1 + hz : ey + SW - 1 + hy;
    const int nranges = 3 * nrows;
    const int w = wave_id();

    // The most contributions any grid value can receive: its stencil window holds
    // (SW + hx)(SW + hy)(SW + hz) staggering-0 cells (3-D), each with at most cellmax points.
    // With the maximum force of component c it sets the tile's scale (every split block of
    // the tile finds the same).
    const unsigned long long vmax = fmax_of(a.fmax, c, s_red);  // has a barrier
    const uint64_t win = (uint64_t)(SW + hx) * (SW + hy) * ((DIM == 3) ? SW + hz : 1);
    const uint32_t mbound = (uint32_t)min(win * (uint64_t)*a.cellmax, (uint64_t)0xFFFFFFFFu);
    const bool finite = vmax < FX_NONFINITE;
    const int fshift = (vmax == 0ull || !finite) ? 0 : fx_shift(vmax, mbound);

    typename ST::Table& tb = tables[w];
    if (finite) {
        // Slices in any order: the integer sums do not depend on it.
        for (int q = w; q < nslices; q += NW) {
            int rp;
            bool rn;
            const int total = ST::build(g, a.cstart, q, ox, oy, oz, lenx, nrows, tb, &rp, &rn);
            if (total > 0)
                ST::template spread_slice<ROT>(a, c, tb, marks[w], rp, rn, nranges, total, q, off, ex, ey, ez,
                                 fshift, tile, ksub, split);
            wave_sync();
        }
    }
    __syncthreads();

    constexpr int CELLS = TX * TY * TZ;
    if (split > 1) {
        // Publish this block's partial sums; split_sum_kernel adds a tile's partials (exact
        // integer sums, in any order) and writes the grid values.
        long long* part = a.partial + ((int64_t)tile_id * split + ksub) * CELLS;
        for (int i = threadIdx.x; i < CELLS; i += blockDim.x) {
            const int xr = i % TX, yr = (i / TX) % TY, zr = i / (TX * TY);
            part[i] = (long long)tile[(zr * TY + yr) * ST::PXS + xr + 3];
        }
        if (ksub == 0 && threadIdx.x == 0) a.tile_shift[tile_id] = finite ? fshift : INT32_MIN;
        return;
    }
    T* f = (T*)a.f;
    // the output grid: the plan's own, or the caller's unpadded one (ghost cells dropped)
    const int on0 = a.direct ? a.user_n[0] : g.n[0], on1 = a.direct ? a.user_n[1] : g.n[1];
    const int on2 = (DIM == 3) ? (a.direct ? a.user_n[2] : g.n[2]) : 1;
    const int64_t G = (int64_t)on0 * on1 * on2;
    for (int i = threadIdx.x; i < CELLS; i += blockDim.x) {
        const int xr = i % TX, yr = (i / TX) % TY, zr = i / (TX * TY);
        if (xr >= ex || yr >= ey || zr >= ez) continue;
        if (x0 + xr >= on0 || y0 + yr >= on1 || z0 + zr >= on2) continue;
        const int64_t gi = ((int64_t)(z0 + zr) * on1 + (y0 + yr)) * on0 + (x0 + xr);
        const T v = fx_value<T>(tile[(zr * TY + yr) * ST::PXS + xr + 3], fshift, finite, g.scale);
        T* dst = f + (int64_t)c * G + gi;
        *dst = a.accumulate ? *dst + v : v;
    }
}

// Grid values of split tiles, after the spreading kernel has published every block's
// partial sums: one thread per tile cell (i < ncells, the tiles' cells) adds the partials
// and writes the cell's value.
template <typename T, int DIM, int TX, int TY, int TZ>
__device__ __forceinline__ void split_sum_body(const OpArgs& a, int64_t i, int64_t ncells)
{
    constexpr int CELLS = TX * TY * TZ;
    if (i >= ncells) return;
    const GeomArgs& g = a.g;
    const int tile_id = (int)(i / CELLS), cell = (int)(i - (int64_t)tile_id * CELLS);
    int c, x0, y0, z0;
    spread_tile_at<TX, TY, TZ>(a, tile_id, c, x0, y0, z0);
    const int xr = cell % TX, yr = (cell / TX) % TY, zr = cell / (TX * TY);
    const int ex = min(TX, g.n[0] - x0), ey = min(TY, g.n[1] - y0);
    const int ez = (DIM == 3) ? min(TZ, g.n[2] - z0) : 1;
    if (xr >= ex || yr >= ey || zr >= ez) return;
    const int split = g.split;
    const long long* part = a.partial + (int64_t)tile_id * split * CELLS + cell;
    unsigned long long sum = 0ull;
    for (int kk = 0; kk < split; ++kk) sum += (unsigned long long)part[(int64_t)kk * CELLS];
    const int fshift = a.tile_shift[tile_id];
    const int on0 = a.direct ? a.user_n[0] : g.n[0], on1 = a.direct ? a.user_n[1] : g.n[1];
    const int on2 = (DIM == 3) ? (a.direct ? a.user_n[2] : g.n[2]) : 1;
    if (x0 + xr >= on0 || y0 + yr >= on1 || z0 + zr >= on2) return;  // a ghost cell
    const int64_t G = (int64_t)on0 * on1 * on2;
    const int64_t gi = ((int64_t)(z0 + zr) * on1 + (y0 + yr)) * on0 + (x0 + xr);
    const T v = fx_value<T>(sum, fshift == INT32_MIN ? 0 : fshift, fshift != INT32_MIN, g.scale);
    T* dst = (T*)a.f + (int64_t)c * G + gi;
    *dst = a.accumulate ? *dst + v : v;
}

template <typename T, int DIM, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void split_sum_kernel(OpArgs a, int64_t ncells)
{
    split_sum_body<T, DIM, TX, TY, TZ>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, ncells);
}

// The plan's count of points in crowded cells (bucket pass) picks the order of adds for
// the whole launch: rotated when at least 1/CROWD_DIV of the points lie in cells of at least
// CROWD_CELL points, where it removes most LDS bank conflicts between points of one cell;
// plain otherwise, where the rotation's extra selects cost more than it saves.
template <typename T, int DIM, int KERN, int TX, int TY, int TZ>
__global__ __launch_bounds__(SPREAD_THREADS) __attribute__((amdgpu_waves_per_eu(6))) void
spread_kernel(OpArgs a)
{
    __shared__ SpreadShared<SpreadTile<T, DIM, KERN, TX, TY, TZ>> sm;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    const bool rot = a.crowd != nullptr && (uint64_t)*a.crowd * CROWD_DIV >= (uint64_t)a.g.npts;
    if (rot) spread_body<T, DIM, KERN, TX, TY, TZ, true>(a, bid, sm);
    else spread_body<T, DIM, KERN, TX, TY, TZ, false>(a, bid, sm);
}

// ---------------------------------------------------------------------------------------
// Interpolation
// ---------------------------------------------------------------------------------------
// One thread per point, in the sorted order of staggering 0: neighbouring lanes hold
// neighbouring cells, so the SW^d gathers of a wave share cache lines.  All components of a
// point are accumulated in registers and written together.
// Interpolated value of component c at point coordinates x: weights per axis, then the
// SW^d gathers (SW = support_width<KERN>()) in tensor-product order.  DIRECT: u is the
// caller's unpadded field of un[0] x un[1] x un[2] cells per component (walled plans); the
// stencil's ghost nodes read as zero.
template <typename T, int DIM, int KERN, bool DIRECT>
__device__ __forceinline__ T interp_component(const GeomArgs& g, const T* __restrict__ u, int c,
                                              const T x[DIM], const int un[3])
{
    constexpr int SW = support_width<KERN>();
    const int n0 = g.n[0], n1 = g.n[1], n2 = (DIM == 3) ? g.n[2] : 1;
    const int f0 = DIRECT ? un[0] : n0, f1 = DIRECT ? un[1] : n1;  // the field read
    const int f2 = (DIM == 3) ? (DIRECT ? un[2] : n2) : 1;
    const int64_t G = (int64_t)f0 * f1 * f2;
    T w[DIM][4];
    int cell[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const T ih = Prec<T>::inv_h(g, k);
        const T y = shifted_scaled<T>(x[k], ih, (T)g.comp_xi[c][k]);
        T r;
        const double fyd = axis_cell<T>(y, SW == 3, &r);
        r += product_residual<T>(x[k], ih, Prec<T>::inv_lo(g, k));
        weights_of<T, KERN>(r, w[k]);
        cell[k] = fabs(fyd) < 1073741824.0 ? floor_mod(fyd, g.n[k], g.inv_n[k]) : 0;
    }
    int xi[4];
    bool xok[4];
#pragma unroll
    for (int ix = 0; ix < SW; ++ix) {
        xi[ix] = wrap_small(cell[0] - 1 + ix, n0);
        xok[ix] = !DIRECT || xi[ix] < f0;
        if (!xok[ix]) xi[ix] = 0;  // a ghost node: read an in-range value, use zero
    }
    const T* __restrict__ uc = u + (int64_t)c * G;
    T sum = T(0);
#pragma unroll
    for (int iz = 0; iz < ((DIM == 3) ? SW : 1); ++iz) {
        int zz = (DIM == 3) ? wrap_small(cell[DIM - 1] - 1 + iz, n2) : 0;
        T sy = T(0);
#pragma unroll
        for (int iy = 0; iy < SW; ++iy) {
            int yy = wrap_small(cell[1] - 1 + iy, n1);
            const bool rok = !DIRECT || (yy < f1 && zz < f2);
            const T* __restrict__ line = uc + (rok ? ((int64_t)zz * f1 + yy) * f0 : 0);
            T sx = T(0);
#pragma unroll
            for (int ix = 0; ix < SW; ++ix) {
                const T v = line[xi[ix]];
                sx = fma(w[0][ix], (rok && xok[ix]) ? v : T(0), sx);
            }
            sy = fma(w[1][iy], sx, sy);
        }
        sum = (DIM == 3) ? fma(w[DIM - 1][iz], sy, sum) : sy;
    }
    return sum;
}

// One thread per sorted point.  FP32 with a full set of components unrolls the component
// loop, so all 3 x 4^d gathers of a point can be in flight together (measured faster, at
// ~250 VGPRs); FP64 keeps one component at a time, since unrolling it would need ~360
// VGPRs and leave one wave per SIMD.
template <typename T, int DIM, int KERN, bool DIRECT>
__device__ __forceinline__ void interp_body(const OpArgs& a, int bid, int nblk)
{
    const GeomArgs& g = a.g;
    const int ncomp = g.ncomp;
    const int64_t n = g.npts;
    const T* __restrict__ Xs = (const T*)a.Xs;
    const T* __restrict__ u = (const T*)a.u;
    T* __restrict__ U = (T*)a.U;
    const T os = (T)a.out_scale;
    const bool unrolled = sizeof(T) == 4 && ncomp == DIM;
    for (int64_t j = (int64_t)bid * blockDim.x + threadIdx.x; j < n; j += (int64_t)nblk * blockDim.x) {
        T x[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) x[k] = Xs[k * n + j];  // columns
        const int64_t p = clamp_index(a.perm[j], n);
        T res[3] = {T(0), T(0), T(0)};
        if (sizeof(T) == 4 && unrolled) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) res[c] = interp_component<T, DIM, KERN, DIRECT>(g, u, c, x, a.user_n);
#pragma unroll
            for (int c = 0; c < DIM; ++c) U[p * DIM + c] = res[c] * os;
        } else {
#pragma unroll 1
            for (int c = 0; c < ncomp; ++c) res[c] = interp_component<T, DIM, KERN, DIRECT>(g, u, c, x, a.user_n);
            for (int c = 0; c < ncomp; ++c) U[p * ncomp + c] = res[c] * os;
        }
        if (a.Xadv) {  // fused position update (ncomp == DIM): the same arithmetic as advect
            T* __restrict__ Xa = (T*)a.Xadv;
            T* __restrict__ Xn = (T*)a.Xnext;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const T y = advect_coord(x[k], res[k], (T)a.adv_dt, (T)a.adv_len[k]);
                Xa[p * DIM + k] = y;
                if (Xn) Xn[k * n + j] = y;
            }
        }
    }
}

template <typename T, int DIM, int KERN, bool DIRECT>
__global__ __launch_bounds__(256) void interp_kernel(OpArgs a)
{
    interp_body<T, DIM, KERN, DIRECT>(a, xcd_block(blockIdx.x, gridDim.x), gridDim.x);
}

// Interpolation through LDS (3-D plans).  A block owns a TX x TY x TZ tile of staggering-0
// cells, i.e. the sorted points whose cells lie in it (one contiguous sorted range per
// x-row of the tile).  For each component in turn it stages the grid values that the
// stencils of those points can touch -- the tile widened by the stencil and by the offset
// between the component's cells and staggering-0 cells -- in LDS with coalesced loads, and
// every point then reads its s^3 values from LDS instead of gathering them from L2.  The
// weights and the order of the multiply-adds are those of interp_component, so the values
// are bitwise equal to the gather kernel's.  A point is handled by the same thread in every
// pass: the first components wait in a sorted-order scratch (written and read coalesced),
// and the last pass writes the point's row of U, and the position update if fused, once.
constexpr int IT_TX = 16, IT_TY = 16, IT_TZ = 8;  // interpolation tile (3-D plans)

// Tile `bid` of the plan (blocks of 256 threads).
template <typename T, int KERN, int TX, int TY, int TZ>
__device__ __forceinline__ void interp_tile_body(const OpArgs& a, int bid)
{
    constexpr int KP = 4;
    constexpr int SW = support_width<KERN>();
    constexpr int RX = TX + 4, RY = TY + 4, RZ = TZ + 4;  // largest staged region (SW <= 4)
    constexpr int ROWS = TY * TZ;
    __shared__ T su[RX * RY * RZ];
    __shared__ int32_t s_rowoff[RY * RZ];  // grid offset of each staged row (wrapped y, z)
    static_assert(RY * RZ <= 256, "one thread per staged row");
    __shared__ int32_t s_lo[ROWS];
    __shared__ int32_t s_pref[ROWS + 1];
    __shared__ uint32_t s_scan[256 / 64 + 1];
    const GeomArgs& g = a.g;
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const int64_t n = g.npts;
    const int tid = threadIdx.x;
    const int nt[3] = {(n0 + TX - 1) / TX, (n1 + TY - 1) / TY, (n2 + TZ - 1) / TZ};
    constexpr int size[3] = {TX, TY, TZ};
    int bx, by, bz;
    tile_coords(bid, nt, slowest_tile_dim(g.n, nt, size), bx, by, bz);
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int ex = min(TX, n0 - x0), ey = min(TY, n1 - y0), ez = min(TZ, n2 - z0);
    const int nrt = ey * ez;

    // Sorted range of each x-row of the tile (from the cell-start table), and their prefix
    // counts.
    uint32_t cnt = 0;
    int32_t lo = 0;
    if (tid < nrt) {
        const int64_t rowbase = ((int64_t)(z0 + tid / ey) * n1 + (y0 + tid % ey)) * n0;
        lo = a.cstart[rowbase + x0];
        const int32_t hi = a.cstart[rowbase + x0 + ex];
        cnt = hi > lo ? (uint32_t)(hi - lo) : 0u;
    }
    uint32_t total_u;
    const uint32_t pref = block_excl_scan_u32<256>(cnt, s_scan, &total_u);
    if (tid < nrt) {
        s_lo[tid] = lo;
        s_pref[tid] = (int32_t)pref;
    }
    if (tid == 0) s_pref[nrt] = (int32_t)total_u;
    const int total = (int)total_u;
    if (total == 0) return;  // no points in the tile: nothing to stage (uniform per block)

    const T* __restrict__ Xs = (const T*)a.Xs;
    const T* __restrict__ u = (const T*)a.u;
    T* __restrict__ U = (T*)a.U;
    T* __restrict__ Us = (T*)a.Us;
    // the grid read: the plan's own, or the caller's unpadded field (direct)
    const int un0 = a.direct ? a.user_n[0] : n0, un1 = a.direct ? a.user_n[1] : n1;
    const int un2 = a.direct ? a.user_n[2] : n2;
    const int64_t Gu = (int64_t)un0 * un1 * un2;
    // The sums use weights_scaled, 2^(3 ws) times the weights' product; the output scale and
    // the time step of the position update take the inverse power, so U and the positions
    // have the bits of the unscaled sums.
    constexpr int WS3 = 3 * weight_shift<KERN>();
    const T os = (T)ldexp(a.out_scale, -WS3);
    const T adt = (T)ldexp(a.adv_dt, -WS3);
    const int ncomp = g.ncomp;
    for (int c = 0; c < ncomp; ++c) {
        // Staged region: cells [x0 + dlo - 1, x0 + ex + dhi + SW - 2) per axis, wrapped.
        const int hx = g.dhi[c][0] - g.dlo[c][0], hy = g.dhi[c][1] - g.dlo[c][1];
        const int hz = g.dhi[c][2] - g.dlo[c][2];
        const int lx = ex + SW - 1 + hx, ly = ey + SW - 1 + hy, lz = ez + SW - 1 + hz;
        const int rx = x0 + g.dlo[c][0] - 1, ry = y0 + g.dlo[c][1] - 1, rz = z0 + g.dlo[c][2] - 1;
        const int nr = ly * lz;
        if (tid < nr) {  // one thread per staged row (nr <= RY * RZ <= 256)
            const int iz = tid / ly, iy = tid - iz * ly;
            const int wz = wrap_small(rz + iz, n2), wy = wrap_small(ry + iy, n1);
            // the caller's unpadded field: ghost rows (-1) read as zero
            s_rowoff[tid] = !a.direct ? (wz * n1 + wy) * n0
                          : (wz < un2 && wy < un1) ? (wz * un1 + wy) * un0 : -1;
        }
        __syncthreads();  // the previous component's points are done with su
        {
            // Thread tid stages x-column tid % lx of rows tid / lx, tid / lx + rstep, ...; SU
            // rows per round are loaded before any is stored, so their loads overlap.
            constexpr int SU = 12;
            const int rstep = 256 / lx;
            const int xi = tid % lx;
            const int r = tid / lx;
            if (r < rstep) {
                const int gx = wrap_small(rx + xi, n0);
                const bool xin = gx < un0;  // not a ghost column of the caller's field
                const T* __restrict__ uc = u + (int64_t)c * Gu;
                for (int r0 = r; r0 < nr; r0 += SU * rstep) {
                    T val[SU];
#pragma unroll
                    for (int q = 0; q < SU; ++q) {
                        const int rr = r0 + q * rstep;
                        val[q] = T(0);
                        const int ro = rr < nr ? s_rowoff[rr] : -1;
                        if (ro >= 0 && xin) val[q] = uc[(int64_t)ro + gx];
                    }
#pragma unroll
                    for (int q = 0; q < SU; ++q) {
                        const int rr = r0 + q * rstep;
                        if (rr < nr) su[rr * lx + xi] = val[q];
                    }
                }
            }
        }
        __syncthreads();
        // The first components of a point wait in sorted order (coalesced) until the last
        // pass writes its whole row of U, and the fused position update (ncomp == 3).
        const bool last = c == ncomp - 1;
        const bool adv = last && a.Xadv != nullptr;
        // KP points per thread and round: their lookups and loads are issued together, so a
        // round waits for one memory latency rather than one per point.
        for (int v0 = tid; v0 < total; v0 += 256 * KP) {
            int64_t pj[KP], jj[KP];
            int s0[KP][3];
            T x[KP][3], done[KP][2];
#pragma unroll
            for (int q = 0; q < KP; ++q) {
                const int v = v0 + 256 * q;
                int lo_r = 0, hi_r = nrt;  // row of position v: last row whose prefix is <= v
                while (hi_r - lo_r > 1) {
                    const int mid = (lo_r + hi_r) >> 1;
                    if (s_pref[mid] <= v) lo_r = mid;
                    else hi_r = mid;
                }
                const int ry_t = lo_r % ey, rz_t = lo_r / ey;
                const int64_t j = clamp_index(v < total ? s_lo[lo_r] + (v - s_pref[lo_r]) : 0, n);
                const int rowkey = ((z0 + rz_t) * n1 + (y0 + ry_t)) * n0;
                s0[q][0] = min(max(a.sorted_keys[j] - rowkey, x0), x0 + ex - 1) - x0;
                s0[q][1] = ry_t;
                s0[q][2] = rz_t;
#pragma unroll
                for (int k = 0; k < 3; ++k) x[q][k] = Xs[k * n + j];  // columns
                pj[q] = clamp_index(a.perm[j], n);
                jj[q] = j;
#pragma unroll
                for (int k = 0; k < 2; ++k) done[q][k] = (last && k < c) ? Us[j * 2 + k] : T(0);
            }
#pragma unroll
            for (int q = 0; q < KP; ++q) {
                if (v0 + 256 * q >= total) break;
                // weights as in interp_component; the component's cell from the
                // staggering-0 cell
                T w[3][4];
                int base[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const T ih = Prec<T>::inv_h(g, k);
                    const T y = shifted_scaled<T>(x[q][k], ih, (T)g.comp_xi[c][k]);
                    T r;
                    const double fy = axis_cell<T>(y, SW == 3, &r);
                    r += product_residual<T>(x[q][k], ih, Prec<T>::inv_lo(g, k));
                    weights_scaled<T, KERN>(r, w[k]);
                    int d = g.dlo[c][k];
                    if (g.dhi[c][k] != d) {
                        const T y0s = shifted_scaled<T>(x[q][k], ih, (T)g.stag_xi[0][k]);
                        T r0;
                        d = min(max((int)(fy - axis_cell<T>(y0s, SW == 3, &r0)), g.dlo[c][k]), g.dhi[c][k]);
                    }
                    base[k] = s0[q][k] + d - g.dlo[c][k];  // first stencil cell, region-relative
                }
                T sum = T(0);
#pragma unroll
                for (int iz = 0; iz < SW; ++iz) {
                    T sy = T(0);
#pragma unroll
                    for (int iy = 0; iy < SW; ++iy) {
                        const T* line = su + ((base[2] + iz) * ly + (base[1] + iy)) * lx + base[0];
                        T sx_ = T(0);
#pragma unroll
                        for (int ix = 0; ix < SW; ++ix) sx_ = fma(w[0][ix], line[ix], sx_);
                        sy = fma(w[1][iy], sx_, sy);
                    }
                    sum = fma(w[2][iz], sy, sum);
                }
                if (!last) {
                    Us[jj[q] * 2 + c] = sum;
                    continue;
                }
                const int64_t p = pj[q];
                const T res[3] = {c == 0 ? sum : done[q][0], c == 1 ? sum : done[q][1], sum};
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (k < ncomp) U[p * ncomp + k] = res[k] * os;
                if (adv) {
                    T* __restrict__ Xa = (T*)a.Xadv;
                    T* __restrict__ Xn = (T*)a.Xnext;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const T y = advect_coord(x[q][k], res[k], adt, (T)a.adv_len[k]);
                        Xa[p * 3 + k] = y;
                        if (Xn) Xn[k * n + jj[q]] = y;
                    }
                }
            }
        }
    }
}

// Built for four waves per SIMD (at most 128 VGPRs), which the FP64 body fits without
// spilling; left to itself the compiler takes more registers and runs three.  FP32 measured
// 1.5 us faster per call at four waves than at five (96 VGPRs).
template <typename T>
constexpr int interp_tile_waves() { return 4; }

template <typename T, int KERN, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(interp_tile_waves<T>()))) void
interp_tile_kernel(OpArgs a)
{
    interp_tile_body<T, KERN, TX, TY, TZ>(a, xcd_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------------------
// Position gradient of interpolation: dX_j += sum_c W_{j,c} dU_{j,c} / dX_j, U = J(X) u.
// dW/dX_k = (1/h_k) dw_k(r_k) prod_{l != k} w_l(r_l); one thread per sorted point.
// ---------------------------------------------------------------------------------------
template <typename T, int DIM, int KERN, bool DIRECT>
__global__ __launch_bounds__(256) void interp_grad_kernel(OpArgs a, const T* __restrict__ W,
                                                          T* __restrict__ dX, int accumulate)
{
    constexpr int SW = support_width<KERN>();
    const GeomArgs& g = a.g;
    const int64_t n = g.npts;
    const int n0 = g.n[0], n1 = g.n[1], n2 = (DIM == 3) ? g.n[2] : 1;
    // the field read: the plan's grid, or (DIRECT, walled plans) the caller's unpadded field,
    // whose ghost nodes read as zero
    const int f0 = DIRECT ? a.user_n[0] : n0, f1 = DIRECT ? a.user_n[1] : n1;
    const int f2 = (DIM == 3) ? (DIRECT ? a.user_n[2] : n2) : 1;
    const int64_t G = (int64_t)f0 * f1 * f2;
    const T* __restrict__ Xs = (const T*)a.Xs;
    const T* __restrict__ u = (const T*)a.u;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    for (int64_t j = (int64_t)bid * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        T x[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) x[k] = Xs[k * n + j];  // columns
        const int64_t p = clamp_index(a.perm[j], n);
        T grad[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) grad[k] = T(0);
        for (int c = 0; c < g.ncomp; ++c) {
            const T wc = W[p * g.ncomp + c];
            T w[DIM][4], dw[DIM][4];
            int cell[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const T ih = Prec<T>::inv_h(g, k);
                const T y = shifted_scaled<T>(x[k], ih, (T)g.comp_xi[c][k]);
                T r;
                const double fyd = axis_cell<T>(y, SW == 3, &r);
                r += product_residual<T>(x[k], ih, Prec<T>::inv_lo(g, k));
                weights_of<T, KERN>(r, w[k]);
                dweights_of<T, KERN>(r, dw[k]);
                cell[k] = fabs(fyd) < 1073741824.0 ? floor_mod(fyd, g.n[k], g.inv_n[k]) : 0;
            }
            int xi[4];
            bool xok[4];
#pragma unroll
            for (int ix = 0; ix < SW; ++ix) {
                xi[ix] = wrap_small(cell[0] - 1 + ix, n0);
                xok[ix] = !DIRECT || xi[ix] < f0;
                if (!xok[ix]) xi[ix] = 0;  // a ghost node: read an in-range value, use zero
            }
            const T* __restrict__ uc = a.u ? u + (int64_t)c * G : u;
            // s_* : sums with w in every axis except the one differentiated
            T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
            for (int iz = 0; iz < ((DIM == 3) ? SW : 1); ++iz) {
                const int zz = (DIM == 3) ? wrap_small(cell[DIM - 1] - 1 + iz, n2) : 0;
                T ay = T(0), by = T(0), cy = T(0);
#pragma unroll
                for (int iy = 0; iy < SW; ++iy) {
                    const int yy = wrap_small(cell[1] - 1 + iy, n1);
                    const bool rok = !DIRECT || (yy < f1 && zz < f2);
                    const T* __restrict__ line = uc + (rok ? ((int64_t)zz * f1 + yy) * f0 : 0);
                    T sx = T(0), dsx = T(0);
#pragma unroll
                    for (int ix = 0; ix < SW; ++ix) {
                        const T v = (rok && xok[ix]) ? line[xi[ix]] : T(0);
                        sx = fma(w[0][ix], v, sx);
                        dsx = fma(dw[0][ix], v, dsx);
                    }
                    ay = fma(w[1][iy], dsx, ay);   // d/dx
                    by = fma(dw[1][iy], sx, by);   // d/dy
                    cy = fma(w[1][iy], sx, cy);    // for d/dz
                }
                if (DIM == 3) {
                    gx = fma(w[2][iz], ay, gx);
                    gy = fma(w[2][iz], by, gy);
                    gz = fma(dw[2][iz], cy, gz);
                } else {
                    gx = ay;
                    gy = by;
                }
            }
            grad[0] = fma(wc, gx * Prec<T>::inv_h(g, 0), grad[0]);
            grad[1] = fma(wc, gy * Prec<T>::inv_h(g, 1), grad[1]);
            if (DIM == 3) grad[2] = fma(wc, gz * Prec<T>::inv_h(g, 2), grad[2]);
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            T* d = dX + p * DIM + k;
            const T v = grad[k] * (T)a.out_scale;
            *d = accumulate ? *d + v : v;
        }
    }
}

template <typename T, int D, int K>
void grad_launch(const OpArgs& a, const void* W, void* dX, int accumulate, unsigned nb,
                 hipStream_t st)
{
    if (a.direct)
        hipLaunchKernelGGL((interp_grad_kernel<T, D, K, true>), dim3(nb), dim3(256), 0, st, a,
                           (const T*)W, (T*)dX, accumulate);
    else
        hipLaunchKernelGGL((interp_grad_kernel<T, D, K, false>), dim3(nb), dim3(256), 0, st, a,
                           (const T*)W, (T*)dX, accumulate);
}

hipError_t launch_interp_grad(const OpArgs& a, int dtype, int kernel, const void* W, void* dX,
                              int accumulate, hipStream_t st)
{
    if (a.g.npts == 0) return hipSuccess;
    const unsigned nb = (unsigned)min((int64_t)65536, (a.g.npts + 255) / 256);
    return with_kernel(kernel, [&](auto K) {
        constexpr int KN = decltype(K)::value;
        if (dtype == IB_F64) {
            if (a.g.dim == 3) grad_launch<double, 3, KN>(a, W, dX, accumulate, nb, st);
            else grad_launch<double, 2, KN>(a, W, dX, accumulate, nb, st);
        } else {
            if (a.g.dim == 3) grad_launch<float, 3, KN>(a, W, dX, accumulate, nb, st);
            else grad_launch<float, 2, KN>(a, W, dX, accumulate, nb, st);
        }
        return hipGetLastError();
    });
}

// ---------------------------------------------------------------------------------------
// Position update: X <- wrap(X + dt U) into [0, L) per coordinate; along walled dimensions
// (bit k of walls) X + dt U without wrap.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void advect_kernel(int dim, int ncomp, int walls, int64_t npts,
                                                     T L0, T L1, T L2, T* __restrict__ X,
                                                     const T* __restrict__ U, T dt)
{
    const int64_t total = npts * dim;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i / dim;
        const int k = (int)(i - j * dim);
        const T L = k == 0 ? L0 : (k == 1 ? L1 : L2);
        const T u = U[j * ncomp + k];
        X[i] = ((walls >> k) & 1) ? fma(dt, u, X[i]) : advect_coord(X[i], u, dt, L);
    }
}

hipError_t launch_advect(int dim, int ncomp, int64_t npts, const double length[3], int walls,
                         int dtype, void* X, const void* U, double dt, hipStream_t st)
{
    if (npts == 0) return hipSuccess;
    const int64_t total = npts * dim;
    const unsigned blocks = (unsigned)min((int64_t)4096, (total + 255) / 256);
    if (dtype == IB_F64)
        hipLaunchKernelGGL(advect_kernel<double>, dim3(blocks), dim3(256), 0, st, dim, ncomp, walls,
                           npts, length[0], length[1], length[2], (double*)X, (const double*)U, dt);
    else
        hipLaunchKernelGGL(advect_kernel<float>, dim3(blocks), dim3(256), 0, st, dim, ncomp, walls,
                           npts, (float)length[0], (float)length[1], (float)length[2], (float*)X,
                           (const float*)U, (float)dt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Tether force of the unstructured-point test (Sec. 4.1): every point hangs on a Hookean
// spring from its initial position, F = k (X0 - X), with the difference taken to the
// nearest periodic image of X0 (the displacement is far below half a box); along walled
// dimensions the plain difference.
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T tether_coord(T x0, T x, T k, T L)
{
    T d = x0 - x;
    if (d >= T(0.5) * L) d -= L;
    else if (d < T(-0.5) * L) d += L;
    return k * d;
}

template <typename T>
__global__ __launch_bounds__(256) void tether_kernel(int dim, int walls, int64_t npts, T L0, T L1,
                                                     T L2, const T* __restrict__ X0,
                                                     const T* __restrict__ X, T k,
                                                     T* __restrict__ F)
{
    const int64_t total = npts * dim;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % dim);
        const T L = c == 0 ? L0 : (c == 1 ? L1 : L2);
        F[i] = ((walls >> c) & 1) ? k * (X0[i] - X[i]) : tether_coord(X0[i], X[i], k, L);
    }
}

hipError_t launch_tether(int dim, int walls, int64_t npts, const double length[3], int dtype,
                         const void* X0, const void* X, double k, void* F, hipStream_t st)
{
    if (npts == 0) return hipSuccess;
    const int64_t total = npts * dim;
    const unsigned blocks = (unsigned)min((int64_t)4096, (total + 255) / 256);
    if (dtype == IB_F64)
        hipLaunchKernelGGL(tether_kernel<double>, dim3(blocks), dim3(256), 0, st, dim, walls, npts,
                           length[0], length[1], length[2], (const double*)X0, (const double*)X,
                           k, (double*)F);
    else
        hipLaunchKernelGGL(tether_kernel<float>, dim3(blocks), dim3(256), 0, st, dim, walls, npts,
                           (float)length[0], (float)length[1], (float)length[2],
                           (const float*)X0, (const float*)X, (float)k, (float*)F);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
namespace {
// Spreading tiles (3-D) selectable per plan (960 blocks of 32x16x13 at 128^3).
constexpr int SP_SHAPE[SPREAD_TILE_SHAPES][3] = {{32, 16, 13}, {32, 8, 13}, {64, 8, 8}};
constexpr int SP2_TX = 64, SP2_TY = 32;             // spreading tile (2-D)

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

template <typename T, int DIM, int TX, int TY, int TZ>
void launch_split_sum(const OpArgs& a, hipStream_t st)
{
    const int64_t ncells =
        (int64_t)a.tiles[0] * a.tiles[1] * a.tiles[2] * a.g.ncomp * (TX * TY * TZ);
    hipLaunchKernelGGL((split_sum_kernel<T, DIM, TX, TY, TZ>), dim3((unsigned)((ncells + 255) / 256)),
                       dim3(256), 0, st, a, ncells);
}

template <typename T, int KERN>
hipError_t spread_dispatch(OpArgs a, hipStream_t st)
{
    // the force maxima that set each tile's fixed-point scale
    hipLaunchKernelGGL(fmax_kernel<T>, dim3(FMAX_PARTS), dim3(FMAX_THREADS), 0, st, a);
    spread_tiles(a.g.dim, a.g.sp_tile, a.g.n, a.tiles, &a.tile_slow);
    const unsigned nb = (unsigned)(a.tiles[0] * a.tiles[1] * a.tiles[2] * a.g.ncomp * a.g.split);
    if (a.g.dim == 3) {
        switch (a.g.sp_tile) {
#define IBK_SPREAD_SHAPE(i)                                                                       \
    case i:                                                                                       \
        hipLaunchKernelGGL((spread_kernel<T, 3, KERN, SP_SHAPE[i][0], SP_SHAPE[i][1], SP_SHAPE[i][2]>), \
                           dim3(nb), dim3(SPREAD_THREADS), 0, st, a);                             \
        if (a.g.split > 1)                                                                        \
            launch_split_sum<T, 3, SP_SHAPE[i][0], SP_SHAPE[i][1], SP_SHAPE[i][2]>(a, st);         \
        break;
            IBK_SPREAD_SHAPE(0)
            IBK_SPREAD_SHAPE(1)
            IBK_SPREAD_SHAPE(2)
#undef IBK_SPREAD_SHAPE
        default: return hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL((spread_kernel<T, 2, KERN, SP2_TX, SP2_TY, 1>), dim3(nb),
                           dim3(SPREAD_THREADS), 0, st, a);
        if (a.g.split > 1) launch_split_sum<T, 2, SP2_TX, SP2_TY, 1>(a, st);
    }
    return hipGetLastError();
}

template <typename T, int KERN>
hipError_t interp_dispatch(OpArgs a, hipStream_t st)
{
    const unsigned nb = (unsigned)interp_blocks(a.g.npts);
    const int nt = interp_tiles(a.g.dim, a.g.n, a.g.npts);
    if (nt > 0) {
        hipLaunchKernelGGL((interp_tile_kernel<T, KERN, IT_TX, IT_TY, IT_TZ>), dim3((unsigned)nt),
                           dim3(256), 0, st, a);
    } else if (a.g.dim == 3) {
        if (a.direct) hipLaunchKernelGGL((interp_kernel<T, 3, KERN, true>), dim3(nb), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((interp_kernel<T, 3, KERN, false>), dim3(nb), dim3(256), 0, st, a);
    } else {
        if (a.direct) hipLaunchKernelGGL((interp_kernel<T, 2, KERN, true>), dim3(nb), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((interp_kernel<T, 2, KERN, false>), dim3(nb), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

// ---- batched operator stages ----------------------------------------------------------

__device__ __forceinline__ int batch_job_of(const int32_t* starts, int njobs, int vb)
{
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (starts[mid] <= vb) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename T>
__global__ __launch_bounds__(FMAX_THREADS) void batch_fmax_kernel(const BatchJob* __restrict__ jobs,
                                                                const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_FMAX];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job_of(st, nj, vb);
        fmax_body<T>(jobs[j].op, vb - st[j]);
        __syncthreads();
    }
}

template <typename T, int DIM, int KERN, int TX, int TY, int TZ>
__global__ __launch_bounds__(SPREAD_THREADS) void batch_spread_kernel(const BatchJob* __restrict__ jobs,
                                                           const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_SPREAD];
    const int nj = bt->njobs, total = st[nj];
    __shared__ SpreadShared<SpreadTile<T, DIM, KERN, TX, TY, TZ>> sm;
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job_of(st, nj, vb);
        spread_body<T, DIM, KERN, TX, TY, TZ, false>(jobs[j].op, vb - st[j], sm);
        __syncthreads();
    }
}

template <typename T, int DIM, int KERN>
__global__ __launch_bounds__(256) void batch_interp_kernel(const BatchJob* __restrict__ jobs,
                                                                const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_INTERP];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job_of(st, nj, vb);
        const OpArgs& a = jobs[j].op;
        const int nb = st[j + 1] - st[j];
        if constexpr (DIM == 3) {
            if (a.interp_tiled) {  // a block per tile, as for a single plan (uniform per block)
                interp_tile_body<T, KERN, IT_TX, IT_TY, IT_TZ>(a, xcd_block(vb - st[j], nb));
                __syncthreads();  // the next virtual block reuses the LDS
                continue;
            }
        }
        interp_body<T, DIM, KERN, false>(a, vb - st[j], nb);
    }
}

// Split-tile sums of the jobs of a batch: virtual block vb of job j covers that job's tile
// cells 256 (vb - start) .. 256 (vb - start) + 255.
template <typename T, int DIM, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void batch_split_sum_kernel(const BatchJob* __restrict__ jobs,
                                                              const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_SPLITSUM];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job_of(st, nj, vb);
        const OpArgs& a = jobs[j].op;
        const int64_t ncells =
            (int64_t)a.tiles[0] * a.tiles[1] * a.tiles[2] * a.g.ncomp * (TX * TY * TZ);
        split_sum_body<T, DIM, TX, TY, TZ>(a, (int64_t)(vb - st[j]) * 256 + threadIdx.x, ncells);
    }
}

// The stages of the operators for a batch whose jobs share spreading tile shape S.
template <typename T, int DIM, int KERN, int S>
void batch_ops_shape(const BatchLaunch& b, hipStream_t st)
{
    constexpr int TX = DIM == 3 ? SP_SHAPE[S][0] : SP2_TX, TY = DIM == 3 ? SP_SHAPE[S][1] : SP2_TY;
    constexpr int TZ = DIM == 3 ? SP_SHAPE[S][2] : 1;
    if (b.grid[BS_FMAX] > 0)
        hipLaunchKernelGGL((batch_fmax_kernel<T>), dim3(b.grid[BS_FMAX]), dim3(FMAX_THREADS), 0, st,
                           b.jobs, b.table);
    if (b.grid[BS_SPREAD] > 0)
        hipLaunchKernelGGL((batch_spread_kernel<T, DIM, KERN, TX, TY, TZ>), dim3(b.grid[BS_SPREAD]),
                           dim3(SPREAD_THREADS), 0, st, b.jobs, b.table);
    if (b.grid[BS_SPLITSUM] > 0)
        hipLaunchKernelGGL((batch_split_sum_kernel<T, DIM, TX, TY, TZ>), dim3(b.grid[BS_SPLITSUM]),
                           dim3(256), 0, st, b.jobs, b.table);
    if (b.grid[BS_INTERP] > 0)
        hipLaunchKernelGGL((batch_interp_kernel<T, DIM, KERN>), dim3(b.grid[BS_INTERP]), dim3(256), 0,
                           st, b.jobs, b.table);
}

template <typename T>
void batch_ops_by_shape(const BatchLaunch& b, hipStream_t st)
{
    (void)with_kernel(b.kernel, [&](auto K) {
        constexpr int KV = decltype(K)::value;
        if (b.dim != 3) {
            batch_ops_shape<T, 2, KV, 0>(b, st);  // one 2-D tile shape
        } else {
            static_assert(SPREAD_TILE_SHAPES == 3, "a case per spreading tile shape");
            switch (b.sp_tile) {
            case 0: batch_ops_shape<T, 3, KV, 0>(b, st); break;
            case 1: batch_ops_shape<T, 3, KV, 1>(b, st); break;
            default: batch_ops_shape<T, 3, KV, 2>(b, st); break;
            }
        }
        return hipSuccess;
    });
}
}  // namespace

int interp_blocks(int64_t npts)
{
    return npts > 0 ? (int)min((int64_t)65536, (npts + 255) / 256) : 0;
}

int interp_tiles(int dim, const int n[3], int64_t npts)
{
    if (dim != 3) return 0;
    const int64_t nt = (int64_t)cdiv(n[0], IT_TX) * cdiv(n[1], IT_TY) * cdiv(n[2], IT_TZ);
    return (nt >= 256 && nt <= (1 << 30) && npts >= 200 * nt) ? (int)nt : 0;
}

// Tiles per dimension of a spreading launch, and its slowest tile dimension (tile_coords).
void spread_tiles(int dim, int shape, const int n[3], int tiles[3], int* slow)
{
    *slow = 2;
    if (dim == 3) {
        const int* t = SP_SHAPE[(shape >= 0 && shape < SPREAD_TILE_SHAPES) ? shape : 0];
        tiles[0] = cdiv(n[0], t[0]);
        tiles[1] = cdiv(n[1], t[1]);
        tiles[2] = cdiv(n[2], t[2]);
        *slow = slowest_tile_dim(n, tiles, t);
    } else {
        tiles[0] = cdiv(n[0], SP2_TX);
        tiles[1] = cdiv(n[1], SP2_TY);
        tiles[2] = 1;
    }
}

size_t spread_tile_cells(int dim, int shape)
{
    if (dim != 3) return (size_t)SP2_TX * SP2_TY;
    const int* t = SP_SHAPE[(shape >= 0 && shape < SPREAD_TILE_SHAPES) ? shape : 0];
    return (size_t)t[0] * t[1] * t[2];
}

// With split_points > 0, at least that many points per block.  Built in: about
// SPLIT_BLOCKS blocks in all, the most that run at once at two blocks per CU (measured best
// from 16^3 to 64^3 grids with 2^16 to 2^19 points), but no fewer than SPLIT_MIN_POINTS
// points per block.  The 128^3 grid keeps one block per tile up to about 10^8 points.
int spread_split(int64_t npts, int ntiles, int split_points)
{
    if (ntiles <= 0 || split_points < 0) return 1;
    int64_t s;
    if (split_points > 0) {
        s = npts / ((int64_t)ntiles * split_points);
    } else {
        s = (SPLIT_BLOCKS + ntiles - 1) / ntiles;
        s = std::min(s, npts / ((int64_t)ntiles * SPLIT_MIN_POINTS));
    }
    return (int)(s < 1 ? 1 : (s > SPLIT_MAX ? SPLIT_MAX : s));
}

hipError_t launch_batch_ops(const BatchLaunch& b, hipStream_t st)
{
    if (b.dtype == IB_F64) batch_ops_by_shape<double>(b, st);
    else batch_ops_by_shape<float>(b, st);
    return hipGetLastError();
}

hipError_t launch_spread(const OpArgs& a, int dtype, int kernel, hipStream_t st)
{
    return with_kernel(kernel, [&](auto K) {
        return dtype == IB_F64 ? spread_dispatch<double, decltype(K)::value>(a, st)
                               : spread_dispatch<float, decltype(K)::value>(a, st);
    });
}

hipError_t launch_interp(const OpArgs& a, int dtype, int kernel, hipStream_t st)
{
    return with_kernel(kernel, [&](auto K) {
        return dtype == IB_F64 ? interp_dispatch<double, decltype(K)::value>(a, st)
                               : interp_dispatch<float, decltype(K)::value>(a, st);
    });
}

}  // namespace ibk
