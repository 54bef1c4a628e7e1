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
// Spreading (eq. disc-spread, Sec. 2; parallel algorithm Alg. 4, Sec. 3.3).  Each block
// owns a tile of one component's grid and produces every value of it exactly once.  It
// reads the sorted points whose cells can reach the tile (contiguous sorted ranges per
// x-row, since keys are x-fastest), one source plane at a time.  A wave takes 64
// consecutive points of a plane and computes their weights; lanes holding the same
// component-c cell form a group (adjacent lanes for staggering 0, found by matching cell
// codes with ballots otherwise).  The group's sum over its points of the 4^d weight
// products -- the segmented reduce of Alg. 4, for all shifts at once -- is formed in
// registers (by one lane, or for a crowded cell by a few sub-leader lanes that add in
// separate rounds), and added into an FP64 LDS copy of the tile with LDS atomic adds.  The
// lanes adding in one round hold distinct cells, so for one shift the active lanes of an
// instruction hit distinct addresses; waves of a block work at the same time only on source
// planes far enough apart that their targets are disjoint, and overlapping planes follow one
// fixed order.  The order in which every grid
// value receives its contributions is therefore fixed by the data alone, and the result is
// bitwise reproducible; no global atomics are used.
//
// Interpolation (eq. disc-interp; Alg. 3, Sec. 3.2).  One thread per point in the sorted
// order of staggering 0, gathering the 4^d grid values of each component directly
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

// Point index from a permutation entry, kept inside [0, n) so that no data can steer a
// load or store out of bounds (a valid permutation is never changed by this).
__device__ __forceinline__ int64_t clamp_index(int32_t p, int64_t n)
{
    return (uint32_t)p < (uint64_t)n ? (int64_t)p : 0;
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

// Weights of a point at coordinates x for component c, and the offset of its component-c
// cell from its staggering-0 cell per dimension.  The cells follow the key rule exactly
// (t = x * inv_h rounded once, minus the staggering, floored).
template <typename T, int DIM, int KERN>
__device__ __forceinline__ void comp_weights(const GeomArgs& g, int c, const T x[DIM],
                                             T w[DIM][4], int delta[DIM])
{
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const T ih = Prec<T>::inv_h(g, k);
        const T yc = shifted_scaled<T>(x[k], ih, (T)g.comp_xi[c][k]);
        const T fc = floor(yc);
        if (g.dlo[c][k] == g.dhi[c][k]) {
            delta[k] = g.dlo[c][k];  // the same staggering as staggering 0 along this axis
        } else {
            const T y0 = shifted_scaled<T>(x[k], ih, (T)g.stag_xi[0][k]);
            delta[k] = min(max((int)(fc - floor(y0)), g.dlo[c][k]), g.dhi[c][k]);
        }
        T r = yc - fc;
        r += product_residual<T>(x[k], ih, Prec<T>::inv_lo(g, k));
        weights4<T, KERN>(r, w[k]);
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

// A source slice (an x-y plane of staggering-0 cells in 3-D, one x-row in 2-D) as a list
// of sorted ranges, one per x-row piece (at most 3 pieces per row, since a tile is never
// wider than the grid).  A range may include a few points of neighbouring cells (the
// cell-block table brackets ranges in blocks of 4 cells); such points map outside the
// tile and are dropped.
template <int MAXR>
struct SliceTable {
    int32_t lo[MAXR];
    int32_t hi[MAXR];
    int32_t base[MAXR];   // sorted index of slice position v in range r: base[r] + v
    int32_t xo[MAXR];     // source-frame x of a key: key + xo
    int32_t uy[MAXR];     // source-frame y of the row
    int32_t pref[MAXR + 1];
};

constexpr uint32_t NO_CELL = 0xFFFFFFu;

template <typename T, int DIM, int KERN, int TX, int TY, int TZ>
struct SpreadTile {
    static constexpr int PXS = TX + 6;  // padded row pitch of the LDS tile (x from -3 to TX + 2)
    static constexpr int NZ = (DIM == 3) ? 4 : 1;            // stencil extent in z
    static constexpr int MAXROWS = (DIM == 3) ? TY + 5 : 1;   // x-rows per slice
    static constexpr int MAXR = 3 * MAXROWS;
    static_assert(MAXR <= 64, "one lane per range of a slice");
    using Table = SliceTable<MAXR>;

    // Per-wave LDS scratch of the chunk loop.
    struct WaveScratch {
        int32_t ltab[64];  // lanes of each group in rank order (cells matched by code)
        int32_t mark[64];  // range starts inside a chunk
    };

    // Range table of source slice q (frame origin ox, oy, oz; lenx cells per row, nrows
    // rows); returns the slice's point count.  Afterwards lane r < 3 * nrows holds range r's
    // first slice position (*rp) and whether the range is non-empty (*rn).
    __device__ static int build(const GeomArgs& g, const int32_t* __restrict__ cb, int q, int ox,
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
            const int64_t rb = (int64_t)r * (g.nbx + 1);
            const int32_t rowbase = r * n0;
            int done = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                int32_t lo = 0, hi = 0, xo = 0;
                if (done < lenx) {
                    const int xa = wrap_small(ox + done, n0);
                    const int len = min(lenx - done, n0 - xa);
                    lo = cb[rb + (xa >> CBLK_SHIFT)];
                    hi = cb[rb + ((xa + len + (1 << CBLK_SHIFT) - 1) >> CBLK_SHIFT)];
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

    __device__ static void accumulate(T acc[NZ][4][4], const T w[DIM][4])
    {
#pragma unroll
        for (int iz = 0; iz < NZ; ++iz)
#pragma unroll
            for (int iy = 0; iy < 4; ++iy) {
                const T cyz = (DIM == 3) ? w[1][iy] * w[2][iz] : w[1][iy];
#pragma unroll
                for (int ix = 0; ix < 4; ++ix) acc[iz][iy][ix] = fma(w[0][ix], cyz, acc[iz][iy][ix]);
            }
    }

    // acc = the 4^d weight products of one point (a first term needs no addition).
    __device__ static void products(T acc[NZ][4][4], const T w[DIM][4])
    {
#pragma unroll
        for (int iz = 0; iz < NZ; ++iz)
#pragma unroll
            for (int iy = 0; iy < 4; ++iy) {
                const T cyz = (DIM == 3) ? w[1][iy] * w[2][iz] : w[1][iy];
#pragma unroll
                for (int ix = 0; ix < 4; ++ix) acc[iz][iy][ix] = w[0][ix] * cyz;
            }
    }

    static constexpr int bits_for(int v) { return v <= 1 ? 1 : 1 + bits_for((v + 1) / 2); }
    static constexpr int XB = bits_for(TX + 6);
    static constexpr int YB = bits_for(TY + 6);
    static constexpr int ZB = (DIM == 3) ? bits_for(TZ + 6) : 0;
    static constexpr int CB = XB + YB + ZB;
    static_assert(CB <= 24, "cell code too wide");

    // Lanes holding the same (tile-relative) cell as this lane, by matching the cell code
    // bit by bit with ballots; lanes without a cell match nothing.
    __device__ static unsigned long long match_code(uint32_t code, bool has)
    {
        unsigned long long m = __ballot(has);
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const bool bit = (code >> b) & 1u;
            const unsigned long long bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        return has ? m : 0ull;
    }

    // Add a leader's 4^d sums into the tile with LDS atomic adds (ds_add), which apply the
    // read-add-write inside the LDS unit, so no lane waits for a value.  The order of the
    // additions into any tile value is still fixed: the leaders of one wave hold distinct
    // cells, so for one shift the active lanes of an instruction hit distinct addresses;
    // a wave's LDS instructions execute in program order; and waves working at the same
    // time own disjoint target regions.  Tile rows are padded in x (PXS = TX + 6, target
    // x from -3 to TX + 2), so only whole rows can fall outside the tile; those are skipped.
    __device__ static void add_to_tile(const T acc[NZ][4][4], bool leader, int cx, int cy,
                                       int cz, int ey, int ez, double* tile)
    {
        // Rows of the stencil: slice-axis offset ia (z in 3-D, y in 2-D), in-plane offset ib
        // (y in 3-D); row (ia, ib) starts `base + (ia * TY + ib) * PXS` (3-D) or
        // `base + ia * PXS` (2-D) elements into the tile.
        const int zb = (DIM == 3) ? cz - 1 : 0, yb = cy - 1;
        const int base = (zb * TY + yb) * PXS + (cx + 2);
        bool oka[4], okb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            oka[i] = leader && ((DIM == 3) ? (unsigned)(zb + i) < (unsigned)ez
                                           : (unsigned)(yb + i) < (unsigned)ey);
            okb[i] = (DIM == 3) ? (unsigned)(yb + i) < (unsigned)ey : i == 0;
        }
#pragma unroll
        for (int ia = 0; ia < 4; ++ia)
#pragma unroll
            for (int ib = 0; ib < ((DIM == 3) ? 4 : 1); ++ib) {
                if (oka[ia] && okb[ib]) {
                    double* row = tile + base + ((DIM == 3) ? (ia * TY + ib) * PXS : ia * PXS);
#pragma unroll
                    for (int ix = 0; ix < 4; ++ix) {
                        const double v = (DIM == 3) ? acc[ia][ib][ix] : acc[0][ia][ix];
                        __hip_atomic_fetch_add(row + ix, v, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            }
    }

    // Slice positions v0 + lane: range, key, coordinates and force (zeros past the end).
    // The sorted index is kept inside [0, n) whatever the tables hold.  Called by the whole
    // wave.
    __device__ static void load(const OpArgs& a, int c, const int32_t* __restrict__ sk,
                                const Table& tb, int32_t* mark, int rp, bool rn, int nranges,
                                int total, int v0, int& rr, int32_t& key, T x[DIM], T& F)
    {
        rr = locate(mark, rp, rn, nranges, v0);
        key = 0;
        F = T(0);
#pragma unroll
        for (int k = 0; k < DIM; ++k) x[k] = T(0);
        const int v = v0 + lane_id();
        if (v < total) {
            const int64_t j = clamp_index(tb.base[rr] + v, a.g.npts);
            const T* __restrict__ Xs = (const T*)a.Xs;
            key = sk[j];
#pragma unroll
            for (int k = 0; k < DIM; ++k) x[k] = Xs[j * DIM + k];
            // the force of the point, read through the permutation (its input-order row)
            F = ((const T*)a.F)[clamp_index(a.perm[j], a.g.npts) * a.g.ncomp + c];
        }
    }

    // Reduce the slice in chunks of 64 points and add the sums into the tile.
    // off[k] = 2 + dhi[k]: a point's tile-relative component-c cell is its source-frame
    // staggering-0 cell + delta - off.  Within a chunk, the points of one cell form a
    // group; its lowest lanes (sub-leaders) sum the group's contributions to all 4^d shifts
    // in registers, pulling the other members' weights from their lanes.
    __device__ static void reduce(const OpArgs& a, int c, const int32_t* __restrict__ sk,
                                  const Table& tb, int rp, bool rn, int nranges, int total, int q,
                                  const int off[3], int ex, int ey, int ez, bool same0,
                                  double* tile, WaveScratch& ws, int k0, int kstride)
    {
        const GeomArgs& g = a.g;
        const int lane = lane_id();
        const unsigned long long below = (1ull << lane) - 1ull;
        // Chunk data is loaded one chunk ahead, so its latency overlaps the current chunk.
        int nrr = 0;
        int32_t nkey = 0;
        T nx[DIM], nF = T(0);
        // This block's chunks of the slice: k0, k0 + kstride, ... (all of them unless the
        // tile is split over several blocks).
        const int step = 64 * kstride;
        if (64 * k0 < total)
            load(a, c, sk, tb, ws.mark, rp, rn, nranges, total, 64 * k0, nrr, nkey, nx, nF);
        for (int v0 = 64 * k0; v0 < total; v0 += step) {
            const int v = v0 + lane;
            const bool valid = v < total;
            const int rr = nrr;
            const int32_t key = nkey;
            T x[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) x[k] = nx[k];
            const T Fc = nF;
            if (v0 + step < total)
                load(a, c, sk, tb, ws.mark, rp, rn, nranges, total, v0 + step, nrr, nkey, nx, nF);
            T w[DIM][4];
            int cx = 0, cy = 0, cz = 0;
            bool has = false;
            {
                int delta[DIM];
                comp_weights<T, DIM, KERN>(g, c, x, w, delta);
#pragma unroll
                for (int i = 0; i < 4; ++i) w[DIM - 1][i] *= Fc;
                cx = key + tb.xo[rr] + delta[0] - off[0];
                cy = tb.uy[rr] + delta[1] - off[1];
                cz = (DIM == 3) ? q + delta[DIM - 1] - off[2] : 0;
                has = valid && cx >= -2 && cx <= ex && cy >= -2 && cy <= ey &&
                      (DIM == 2 || (cz >= -2 && cz <= ez));
            }
            // Tile-relative cell code: x + 4, y + 4 and z + 4 in fields of XB, YB, ZB bits.
            const uint32_t code = (uint32_t)(cx + 4) | ((uint32_t)(cy + 4) << XB) |
                                  ((uint32_t)(cz + 4) << (XB + YB));
            unsigned long long grp;
            bool leader;
            int head = lane;
            if (same0) {
                // Cells of staggering 0 itself: a cell's points are adjacent in sorted order,
                // so a group runs from its first lane to the next change of cell.
                const uint32_t prev = wave_shr1_u32(code);
                const uint32_t hprev = wave_shr1_u32((uint32_t)has);
                leader = has && (lane == 0 || !hprev || prev != code);
                const unsigned long long heads = __ballot(leader);
                const unsigned long long holes = ~__ballot(has);
                // This lane's run starts at the highest head at or below it and ends at the
                // next head or hole above that.
                const unsigned long long hb = heads & ((2ull << lane) - 1ull);
                head = hb ? 63 - __clzll((long long)hb) : lane;
                const unsigned long long stop = (heads | holes) & ~((2ull << head) - 1ull);
                const int end = stop ? __ffsll((long long)stop) - 1 : 64;
                const unsigned long long upto = (end == 64) ? ~0ull : ((1ull << end) - 1ull);
                grp = has ? (upto & ~((1ull << head) - 1ull)) : 0ull;
            } else {
                grp = match_code(code, has);
                leader = has && (grp & below) == 0ull;
            }
            // The rank of a lane is the number of group lanes below it.  Adjacent groups hold
            // their members in lanes head + rank; matched groups list them in the wave's lane
            // table, one contiguous piece per group in rank order.
            const int rank = __popcll(grp & below);
            const int gk = __popcll(grp);
            const int maxk = wave_max_i32(gk);
            int gbase = 0;
            if (!same0 && maxk > 1) {
                const uint32_t kl = leader ? (uint32_t)gk : 0u;
                const int goff_l = (int)(wave_incl_scan_u32(kl) - kl);
                const int lead_lane = has ? __ffsll((long long)grp) - 1 : lane;
                gbase = __shfl(goff_l, lead_lane, 64);
                if (has) ws.ltab[(gbase + rank) & 63] = lane;
                wave_sync();
            }
            // The first P members of a group (sub-leaders) each sum every P-th member, then
            // add their sums into the tile in P rounds, one rank per round, so the active
            // lanes of each round still hold distinct cells.  P ~ sqrt(largest group * m / a)
            // balances the member rounds (cost m each) against the add rounds (cost a each,
            // measured ~1.3 m in FP64 and ~2 m in FP32, where member rounds move half the
            // bytes); it is uniform across the wave and depends only on the data, so the
            // order in which every tile value receives its contributions is fixed.
            constexpr int K1 = sizeof(T) == 8 ? 3 : 4, K2 = sizeof(T) == 8 ? 8 : 10;
            constexpr int K3 = sizeof(T) == 8 ? 15 : 20, K4 = sizeof(T) == 8 ? 24 : 32;
            constexpr int K5 = sizeof(T) == 8 ? 35 : 46, K6 = sizeof(T) == 8 ? 48 : 62;
            const int P = maxk <= K1 ? 1 : maxk <= K2 ? 2 : maxk <= K3 ? 3 : maxk <= K4 ? 4
                        : maxk <= K5 ? 5 : maxk <= K6 ? 6 : 7;
            const bool sub = has && rank < P;
            // Lanes other than sub-leaders compute sums that are never added.
            T acc[NZ][4][4];
            products(acc, w);
            const int iters = (maxk + P - 1) / P - 1;
            for (int j = 1; j <= iters; ++j) {
                const int mr = rank + j * P;
                const bool ok = sub && mr < gk;
                const int src = !ok ? lane : same0 ? head + mr : ws.ltab[(gbase + mr) & 63];
                T wk[DIM][4];
#pragma unroll
                for (int d = 0; d < DIM; ++d)
#pragma unroll
                    for (int i = 0; i < 4; ++i) wk[d][i] = __shfl(w[d][i], src, 64);
                const T on = ok ? T(1) : T(0);
#pragma unroll
                for (int i = 0; i < 4; ++i) wk[DIM - 1][i] *= on;
                accumulate(acc, wk);
            }
            wave_sync();
            if (P == 1) {
                add_to_tile(acc, sub, cx, cy, cz, ey, ez, tile);
            } else {
                for (int rr = 0; rr < P; ++rr)
                    add_to_tile(acc, sub && rank == rr, cx, cy, cz, ey, ez, tile);
            }
            wave_sync();
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

template <typename T, int DIM, int KERN, int TX, int TY, int TZ>
__device__ __forceinline__ void spread_body(const OpArgs& a, int bid)
{
    using ST = SpreadTile<T, DIM, KERN, TX, TY, TZ>;
    // Tile rows padded in x (3 before, 3 after).  The tile accumulates in FP64 for both
    // precisions: FP64 LDS atomic adds run at full LDS rate on gfx950, FP32 ones do not.
    __shared__ double tile[ST::PXS * TY * TZ];
    __shared__ typename ST::Table tables[4];
    __shared__ typename ST::WaveScratch scratch[4];
    const GeomArgs& g = a.g;
    // Blocks bid = tile * split + k: the split blocks of a tile each take every split-th
    // chunk of its points and add their partial tiles at the end.  Tiles are numbered with
    // the component fastest, then the three dimensions (spread_tile_at): the components of
    // one region, and neighbouring regions, run close together and (through xcd_block) on one XCD, so the points and
    // forces that their source frames share are read from HBM once and then from that L2.
    const int split = g.split;
    const int tile_id = bid / split, ksub = bid - tile_id * split;
    int c, x0, y0, z0;
    spread_tile_at<TX, TY, TZ>(a, tile_id, c, x0, y0, z0);
    const int ex = min(TX, g.n[0] - x0), ey = min(TY, g.n[1] - y0);
    const int ez = (DIM == 3) ? min(TZ, g.n[2] - z0) : 1;

    constexpr int MAXSLICES = ((DIM == 3) ? TZ : TY) + 4;
    __shared__ int s_done[MAXSLICES];
    for (int i = threadIdx.x; i < ST::PXS * TY * TZ; i += blockDim.x) tile[i] = 0.0;
    if (threadIdx.x < MAXSLICES) s_done[threadIdx.x] = 0;
    __syncthreads();

    // Source frame: staggering-0 cells that can reach the tile for this component.
    const int hx = g.dhi[c][0] - g.dlo[c][0], hy = g.dhi[c][1] - g.dlo[c][1];
    const int hz = (DIM == 3) ? g.dhi[c][2] - g.dlo[c][2] : 0;
    const int off[3] = {2 + g.dhi[c][0], 2 + g.dhi[c][1], (DIM == 3) ? 2 + g.dhi[c][2] : 0};
    const int ox = x0 - off[0], oy = y0 - off[1], oz = (DIM == 3) ? z0 - off[2] : 0;
    const int lenx = ex + 3 + hx;
    const int nrows = (DIM == 3) ? ey + 3 + hy : 1;
    const int nslices = (DIM == 3) ? ez + 3 + hz : ey + 3 + hy;
    const int nphase = 4 + ((DIM == 3) ? hz : hy);
    const int nranges = 3 * nrows;
    const bool same0 = hx == 0 && hy == 0 && hz == 0;
    const int w = wave_id();
    typename ST::Table& tb = tables[w];

    // Slices less than nphase apart have overlapping targets; slices nphase apart do not.
    // The slices are worked in one fixed order: by phase (q mod nphase), then by q; wave w
    // takes positions w, w + 4, ... of that order.  A slice starts once the overlapping
    // slices before it in the order are done (those after it wait for it in turn).  So slices
    // that run at the same time have disjoint targets, and every tile value receives its
    // contributions in an order fixed by the data alone.  Unlike barriers between phases,
    // this lets a wave go on as soon as its own dependences are met.  No wave waits forever:
    // the first unfinished position of the order has all its dependences done, and its wave
    // has finished everything before it.
    const int lane = lane_id();
    for (int t = __builtin_amdgcn_readfirstlane(w); t < nslices; t += 4) {
        int p = 0, first = 0;  // phase of position t and the first position of that phase
        for (;;) {
            const int cnt = (nslices - p + nphase - 1) / nphase;
            if (t < first + cnt) break;
            first += cnt;
            ++p;
        }
        const int q = p + nphase * (t - first);
        // Overlapping slices of earlier phases: q - p .. q - 1 and q + nphase - p .. q + nphase - 1.
        const int dep = lane < p ? q - p + lane : q + nphase - 2 * p + lane;
        const bool need = lane < 2 * p && dep >= 0 && dep < nslices;
        for (;;) {
            const bool ok = !need || __hip_atomic_load(&s_done[need ? dep : 0], __ATOMIC_ACQUIRE,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
            if (__ballot(!ok) == 0ull) break;
            __builtin_amdgcn_s_sleep(1);
        }
        int rp;
        bool rn;
        const int total = ST::build(g, a.cblk, q, ox, oy, oz, lenx, nrows, tb, &rp, &rn);
        if (total > 0)
            ST::reduce(a, c, a.sorted_keys, tb, rp, rn, nranges, total, q, off, ex, ey, ez,
                       same0, tile, scratch[w], ksub, split);
        wave_sync();
        // Every lane writes the same flag (no lane-dependent branch around the loop's back
        // edge); the release orders it after all of this wave's additions into the tile.
        __hip_atomic_store(&s_done[q], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();

    T* f = (T*)a.f;
    const int64_t G = (int64_t)g.n[0] * g.n[1] * (DIM == 3 ? g.n[2] : 1);
    constexpr int CELLS = TX * TY * TZ;
    if (split > 1) {
        // Publish this block's partial tile; split_sum_kernel adds a tile's partials in
        // block order (a fixed order) and writes the grid values.  (A last block to arrive
        // could add them here, but its agent-scope release and acquire write back and
        // invalidate the XCD's L2 for every block, which cost far more on this GPU.)
        double* part = a.partial + ((int64_t)tile_id * split + ksub) * CELLS;
        for (int i = threadIdx.x; i < CELLS; i += blockDim.x) {
            const int xr = i % TX, yr = (i / TX) % TY, zr = i / (TX * TY);
            part[i] = tile[(zr * TY + yr) * ST::PXS + xr + 3];
        }
        return;
    }
    for (int i = threadIdx.x; i < CELLS; i += blockDim.x) {
        const int xr = i % TX, yr = (i / TX) % TY, zr = i / (TX * TY);
        if (xr >= ex || yr >= ey || zr >= ez) continue;
        const int64_t gi = ((int64_t)(z0 + zr) * g.n[1] + (y0 + yr)) * g.n[0] + (x0 + xr);
        const T v = (T)(tile[(zr * TY + yr) * ST::PXS + xr + 3] * g.scale);
        T* dst = f + (int64_t)c * G + gi;
        *dst = a.accumulate ? *dst + v : v;
    }
}

// Grid values of split tiles, after the spreading kernel has published every block's
// partial tile: one thread per tile cell (i < ncells, the tiles' cells) adds the partials
// in block order and writes the cell's value.
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
    const double* part = a.partial + (int64_t)tile_id * split * CELLS + cell;
    double sum = 0.0;
    for (int kk = 0; kk < split; ++kk) sum += part[(int64_t)kk * CELLS];
    const int64_t G = (int64_t)g.n[0] * g.n[1] * (DIM == 3 ? g.n[2] : 1);
    const int64_t gi = ((int64_t)(z0 + zr) * g.n[1] + (y0 + yr)) * g.n[0] + (x0 + xr);
    const T v = (T)(sum * g.scale);
    T* dst = (T*)a.f + (int64_t)c * G + gi;
    *dst = a.accumulate ? *dst + v : v;
}

template <typename T, int DIM, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void split_sum_kernel(OpArgs a, int64_t ncells)
{
    split_sum_body<T, DIM, TX, TY, TZ>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, ncells);
}

// Waves per SIMD a spreading kernel is compiled for.  FP32 with the 32x8x13 tile fits four
// (its sums take half the registers of FP64, and four of its LDS tiles fit in a CU); the
// others keep two, with the registers they need.
template <typename T, int TX, int TY, int TZ>
constexpr int spread_waves_per_eu()
{
    return (sizeof(T) == 4 && TX == 32 && TY == 8 && TZ == 13) ? 4 : 1;
}

template <typename T, int DIM, int KERN, int TX, int TY, int TZ>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(spread_waves_per_eu<T, TX, TY, TZ>()))) void spread_kernel(OpArgs a)
{
    spread_body<T, DIM, KERN, TX, TY, TZ>(a, xcd_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------------------
// Interpolation
// ---------------------------------------------------------------------------------------
// One thread per point, in the sorted order of staggering 0: neighbouring lanes hold
// neighbouring cells, so the 4^d gathers of a wave share cache lines.  All components of a
// point are accumulated in registers and written together.
// Interpolated value of component c at point coordinates x: weights per axis, then the
// 4^d gathers in tensor-product order.
template <typename T, int DIM, int KERN>
__device__ __forceinline__ T interp_component(const GeomArgs& g, const T* __restrict__ u, int c,
                                              const T x[DIM])
{
    const int n0 = g.n[0], n1 = g.n[1], n2 = (DIM == 3) ? g.n[2] : 1;
    const int64_t G = (int64_t)n0 * n1 * n2;
    T w[DIM][4];
    int cell[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const T ih = Prec<T>::inv_h(g, k);
        const T y = shifted_scaled<T>(x[k], ih, (T)g.comp_xi[c][k]);
        const T fy = floor(y);
        T r = y - fy;
        r += product_residual<T>(x[k], ih, Prec<T>::inv_lo(g, k));
        weights4<T, KERN>(r, w[k]);
        const double fyd = (double)fy;
        cell[k] = fabs(fyd) < 1073741824.0 ? floor_mod(fyd, g.n[k], g.inv_n[k]) : 0;
    }
    int xi[4];
#pragma unroll
    for (int ix = 0; ix < 4; ++ix) xi[ix] = wrap_small(cell[0] - 1 + ix, n0);
    const T* __restrict__ uc = u + (int64_t)c * G;
    T sum = T(0);
#pragma unroll
    for (int iz = 0; iz < ((DIM == 3) ? 4 : 1); ++iz) {
        const int zz = (DIM == 3) ? wrap_small(cell[DIM - 1] - 1 + iz, n2) : 0;
        T sy = T(0);
#pragma unroll
        for (int iy = 0; iy < 4; ++iy) {
            const int yy = wrap_small(cell[1] - 1 + iy, n1);
            const T* __restrict__ line = uc + ((int64_t)zz * n1 + yy) * n0;
            T sx = T(0);
#pragma unroll
            for (int ix = 0; ix < 4; ++ix) sx = fma(w[0][ix], line[xi[ix]], sx);
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
template <typename T, int DIM, int KERN>
__device__ __forceinline__ void interp_body(const OpArgs& a, int bid, int nblk)
{
    const GeomArgs& g = a.g;
    const int ncomp = g.ncomp;
    const int64_t n = g.npts;
    const T* __restrict__ Xs = (const T*)a.Xs;
    const T* __restrict__ u = (const T*)a.u;
    T* __restrict__ U = (T*)a.U;
    const bool unrolled = sizeof(T) == 4 && ncomp == DIM;
    for (int64_t j = (int64_t)bid * blockDim.x + threadIdx.x; j < n; j += (int64_t)nblk * blockDim.x) {
        T x[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) x[k] = Xs[j * DIM + k];
        const int64_t p = clamp_index(a.perm[j], n);
        T res[3] = {T(0), T(0), T(0)};
        if (sizeof(T) == 4 && unrolled) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) res[c] = interp_component<T, DIM, KERN>(g, u, c, x);
#pragma unroll
            for (int c = 0; c < DIM; ++c) U[p * DIM + c] = res[c];
        } else {
#pragma unroll 1
            for (int c = 0; c < ncomp; ++c) res[c] = interp_component<T, DIM, KERN>(g, u, c, x);
            for (int c = 0; c < ncomp; ++c) U[p * ncomp + c] = res[c];
        }
        if (a.Xadv) {  // fused position update (ncomp == DIM): the same arithmetic as advect
            T* __restrict__ Xa = (T*)a.Xadv;
#pragma unroll
            for (int k = 0; k < DIM; ++k)
                Xa[p * DIM + k] = advect_coord(x[k], res[k], (T)a.adv_dt, (T)a.adv_len[k]);
        }
    }
}

template <typename T, int DIM, int KERN>
__global__ __launch_bounds__(256) void interp_kernel(OpArgs a)
{
    interp_body<T, DIM, KERN>(a, xcd_block(blockIdx.x, gridDim.x), gridDim.x);
}

// Interpolation through LDS (3-D plans).  A block owns a TX x TY x TZ tile of staggering-0
// cells, i.e. the sorted points whose cells lie in it (one contiguous sorted range per
// x-row of the tile).  For each component in turn it stages the grid values that the
// stencils of those points can touch -- the tile widened by the stencil and by the offset
// between the component's cells and staggering-0 cells -- in LDS with coalesced loads, and
// every point then reads its 4^3 values from LDS instead of gathering them from L2.  The
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
    constexpr int RX = TX + 4, RY = TY + 4, RZ = TZ + 4;  // largest staged region
    constexpr int ROWS = TY * TZ;
    __shared__ T su[RX * RY * RZ];
    __shared__ int32_t s_rowoff[RY * RZ];  // grid offset of each staged row (wrapped y, z)
    static_assert(RY * RZ <= 256, "one thread per staged row");
    __shared__ int32_t s_lo[ROWS];
    __shared__ int32_t s_pref[ROWS + 1];
    __shared__ uint32_t s_scan[256 / 64 + 1];
    const GeomArgs& g = a.g;
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const int64_t G = (int64_t)n0 * n1 * n2;
    const int64_t n = g.npts;
    const int tid = threadIdx.x;
    const int nt[3] = {(n0 + TX - 1) / TX, (n1 + TY - 1) / TY, (n2 + TZ - 1) / TZ};
    constexpr int size[3] = {TX, TY, TZ};
    int bx, by, bz;
    tile_coords(bid, nt, slowest_tile_dim(g.n, nt, size), bx, by, bz);
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int ex = min(TX, n0 - x0), ey = min(TY, n1 - y0), ez = min(TZ, n2 - z0);
    const int nrt = ey * ez;

    // Sorted range of each x-row of the tile (exact: tiles start at multiples of the
    // 4-cell blocks of the cell-block table), and their prefix counts.
    uint32_t cnt = 0;
    int32_t lo = 0;
    if (tid < nrt) {
        const int row = (z0 + tid / ey) * n1 + (y0 + tid % ey);
        const int64_t rb = (int64_t)row * (g.nbx + 1);
        lo = a.cblk[rb + (x0 >> CBLK_SHIFT)];
        const int32_t hi = a.cblk[rb + ((x0 + ex + (1 << CBLK_SHIFT) - 1) >> CBLK_SHIFT)];
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
    const int ncomp = g.ncomp;
    for (int c = 0; c < ncomp; ++c) {
        // Staged region: cells [x0 + dlo - 1, x0 + ex + dhi + 2) per axis, wrapped.
        const int hx = g.dhi[c][0] - g.dlo[c][0], hy = g.dhi[c][1] - g.dlo[c][1];
        const int hz = g.dhi[c][2] - g.dlo[c][2];
        const int lx = ex + 3 + hx, ly = ey + 3 + hy, lz = ez + 3 + hz;
        const int rx = x0 + g.dlo[c][0] - 1, ry = y0 + g.dlo[c][1] - 1, rz = z0 + g.dlo[c][2] - 1;
        const int nr = ly * lz;
        if (tid < nr) {  // one thread per staged row (nr <= RY * RZ <= 256)
            const int iz = tid / ly, iy = tid - iz * ly;
            s_rowoff[tid] = (wrap_small(rz + iz, n2) * n1 + wrap_small(ry + iy, n1)) * n0;
        }
        __syncthreads();  // the previous component's points are done with su
        {
            // Thread tid stages x-column tid % lx of rows tid / lx, tid / lx + rstep, ...; SU
            // rows per round are loaded before any is stored, so their loads overlap.
            constexpr int SU = 8;
            const int rstep = 256 / lx;
            const int xi = tid % lx;
            const int r = tid / lx;
            if (r < rstep) {
                const int gx = wrap_small(rx + xi, n0);
                const T* __restrict__ uc = u + (int64_t)c * G;
                for (int r0 = r; r0 < nr; r0 += SU * rstep) {
                    T val[SU];
#pragma unroll
                    for (int q = 0; q < SU; ++q) {
                        const int rr = r0 + q * rstep;
                        val[q] = T(0);
                        if (rr < nr) val[q] = uc[(int64_t)s_rowoff[rr] + gx];
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
                for (int k = 0; k < 3; ++k) x[q][k] = Xs[j * 3 + k];
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
                    const T fy = floor(y);
                    T r = y - fy;
                    r += product_residual<T>(x[q][k], ih, Prec<T>::inv_lo(g, k));
                    weights4<T, KERN>(r, w[k]);
                    int d = g.dlo[c][k];
                    if (g.dhi[c][k] != d) {
                        const T y0s = shifted_scaled<T>(x[q][k], ih, (T)g.stag_xi[0][k]);
                        d = min(max((int)(fy - floor(y0s)), g.dlo[c][k]), g.dhi[c][k]);
                    }
                    base[k] = s0[q][k] + d - g.dlo[c][k];  // first stencil cell, region-relative
                }
                T sum = T(0);
#pragma unroll
                for (int iz = 0; iz < 4; ++iz) {
                    T sy = T(0);
#pragma unroll
                    for (int iy = 0; iy < 4; ++iy) {
                        const T* line = su + ((base[2] + iz) * ly + (base[1] + iy)) * lx + base[0];
                        T sx_ = T(0);
#pragma unroll
                        for (int ix = 0; ix < 4; ++ix) sx_ = fma(w[0][ix], line[ix], sx_);
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
                for (int k = 0; k < ncomp; ++k) U[p * ncomp + k] = res[k];
                if (adv) {
                    T* __restrict__ Xa = (T*)a.Xadv;
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        Xa[p * 3 + k] = advect_coord(x[q][k], res[k], (T)a.adv_dt, (T)a.adv_len[k]);
                }
            }
        }
    }
}

template <typename T, int KERN, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void interp_tile_kernel(OpArgs a)
{
    interp_tile_body<T, KERN, TX, TY, TZ>(a, xcd_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------------------
// Position gradient of interpolation: dX_j += sum_c W_{j,c} dU_{j,c} / dX_j, U = J(X) u.
// dW/dX_k = (1/h_k) dw_k(r_k) prod_{l != k} w_l(r_l); one thread per sorted point.
// ---------------------------------------------------------------------------------------
template <typename T, int DIM, int KERN>
__global__ __launch_bounds__(256) void interp_grad_kernel(OpArgs a, const T* __restrict__ W,
                                                          T* __restrict__ dX, int accumulate)
{
    const GeomArgs& g = a.g;
    const int64_t n = g.npts;
    const int n0 = g.n[0], n1 = g.n[1], n2 = (DIM == 3) ? g.n[2] : 1;
    const int64_t G = (int64_t)n0 * n1 * n2;
    const T* __restrict__ Xs = (const T*)a.Xs;
    const T* __restrict__ u = (const T*)a.u;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    for (int64_t j = (int64_t)bid * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        T x[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) x[k] = Xs[j * DIM + k];
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
                const T fy = floor(y);
                T r = y - fy;
                r += product_residual<T>(x[k], ih, Prec<T>::inv_lo(g, k));
                weights4<T, KERN>(r, w[k]);
                dweights4<T, KERN>(r, dw[k]);
                const double fyd = (double)fy;
                cell[k] = fabs(fyd) < 1073741824.0 ? floor_mod(fyd, g.n[k], g.inv_n[k]) : 0;
            }
            int xi[4];
#pragma unroll
            for (int ix = 0; ix < 4; ++ix) xi[ix] = wrap_small(cell[0] - 1 + ix, n0);
            const T* __restrict__ uc = a.u ? u + (int64_t)c * G : u;
            // s_* : sums with w in every axis except the one differentiated
            T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
            for (int iz = 0; iz < ((DIM == 3) ? 4 : 1); ++iz) {
                const int zz = (DIM == 3) ? wrap_small(cell[DIM - 1] - 1 + iz, n2) : 0;
                T ay = T(0), by = T(0), cy = T(0);
#pragma unroll
                for (int iy = 0; iy < 4; ++iy) {
                    const int yy = wrap_small(cell[1] - 1 + iy, n1);
                    const T* __restrict__ line = uc + ((int64_t)zz * n1 + yy) * n0;
                    T sx = T(0), dsx = T(0);
#pragma unroll
                    for (int ix = 0; ix < 4; ++ix) {
                        const T v = line[xi[ix]];
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
            *d = accumulate ? *d + grad[k] : grad[k];
        }
    }
}

template <typename T, int D, int K>
void grad_launch(const OpArgs& a, const void* W, void* dX, int accumulate, unsigned nb,
                 hipStream_t st)
{
    hipLaunchKernelGGL((interp_grad_kernel<T, D, K>), dim3(nb), dim3(256), 0, st, a,
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
// Walled plans run on a periodic grid with ghost indices n_k .. m_k - 1 added along walled
// dimensions (m_k = n_k elsewhere).  The caller's field (n) sits at the same indices of the
// padded field (m): pad copies it in with zero ghost values (ghost points are no grid
// points, so interpolation reads nothing there), unpad copies the interior back out and
// drops the ghost values that spreading wrote.
// ---------------------------------------------------------------------------------------
// One wave per grid row (component, z, y), four rows per block, lanes along x with two
// values in flight per lane: the row's indices are worked out once, not per value.
constexpr int PAD_ROWS_PER_BLOCK = 4;

template <typename T>
__global__ __launch_bounds__(256) void pad_kernel(int64_t rows, int n0, int n1, int n2, int m0,
                                                  int m1, int m2, const T* __restrict__ src,
                                                  T* __restrict__ dst)
{
    const int lane = lane_id();
    for (int64_t r = (int64_t)blockIdx.x * PAD_ROWS_PER_BLOCK + wave_id(); r < rows;
         r += (int64_t)gridDim.x * PAD_ROWS_PER_BLOCK) {  // rows of the padded field
        const int y = (int)(r % m1);
        const int64_t cz = r / m1;
        const int z = (int)(cz % m2);
        const int64_t c = cz / m2;
        const bool inside = y < n1 && z < n2;
        const int64_t srow = inside ? ((c * n2 + z) * n1 + y) * n0 : 0;
        T* __restrict__ d = dst + r * m0;
        for (int x = lane; x < m0; x += 128) {
            const int x2 = x + 64;
            const T v0 = (inside && x < n0) ? src[srow + x] : T(0);
            const T v1 = (inside && x2 < n0) ? src[srow + x2] : T(0);
            d[x] = v0;
            if (x2 < m0) d[x2] = v1;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void unpad_kernel(int64_t rows, int n0, int n1, int n2, int m0,
                                                    int m1, int m2, const T* __restrict__ src,
                                                    T* __restrict__ dst, int accumulate)
{
    const int lane = lane_id();
    for (int64_t r = (int64_t)blockIdx.x * PAD_ROWS_PER_BLOCK + wave_id(); r < rows;
         r += (int64_t)gridDim.x * PAD_ROWS_PER_BLOCK) {  // rows of the caller's field
        const int y = (int)(r % n1);
        const int64_t cz = r / n1;
        const int z = (int)(cz % n2);
        const int64_t c = cz / n2;
        const T* __restrict__ s = src + ((c * m2 + z) * m1 + y) * m0;
        T* __restrict__ d = dst + r * n0;
        for (int x = lane; x < n0; x += 128) {
            const int x2 = x + 64;
            const bool two = x2 < n0;
            T v0 = s[x], v1 = two ? s[x2] : T(0);
            if (accumulate) {
                v0 += d[x];
                if (two) v1 += d[x2];
            }
            d[x] = v0;
            if (two) d[x2] = v1;
        }
    }
}

namespace {
struct PadDims {
    int n[3], m[3];
    int64_t user_rows, kernel_rows;  // x-rows of the caller's and the padded field (x ncomp)
};

PadDims pad_dims(const ib_grid_desc& user, const ib_grid_desc& kg)
{
    PadDims d;
    for (int k = 0; k < 3; ++k) {
        d.n[k] = k < user.dim ? user.n[k] : 1;
        d.m[k] = k < kg.dim ? kg.n[k] : 1;
    }
    d.user_rows = (int64_t)user.ncomp * d.n[1] * d.n[2];
    d.kernel_rows = (int64_t)user.ncomp * d.m[1] * d.m[2];
    return d;
}
}  // namespace

hipError_t launch_pad(const ib_grid_desc& user, const ib_grid_desc& kg, int dtype, const void* src,
                      void* dst, hipStream_t st)
{
    const PadDims d = pad_dims(user, kg);
    const unsigned blocks = (unsigned)min((int64_t)65536,
                                          (d.kernel_rows + PAD_ROWS_PER_BLOCK - 1) / PAD_ROWS_PER_BLOCK);
    if (dtype == IB_F64)
        hipLaunchKernelGGL(pad_kernel<double>, dim3(blocks), dim3(256), 0, st, d.kernel_rows,
                           d.n[0], d.n[1], d.n[2], d.m[0], d.m[1], d.m[2], (const double*)src,
                           (double*)dst);
    else
        hipLaunchKernelGGL(pad_kernel<float>, dim3(blocks), dim3(256), 0, st, d.kernel_rows,
                           d.n[0], d.n[1], d.n[2], d.m[0], d.m[1], d.m[2], (const float*)src,
                           (float*)dst);
    return hipGetLastError();
}

hipError_t launch_unpad(const ib_grid_desc& user, const ib_grid_desc& kg, int dtype,
                        const void* src, void* dst, bool accumulate, hipStream_t st)
{
    const PadDims d = pad_dims(user, kg);
    const unsigned blocks = (unsigned)min((int64_t)65536,
                                          (d.user_rows + PAD_ROWS_PER_BLOCK - 1) / PAD_ROWS_PER_BLOCK);
    if (dtype == IB_F64)
        hipLaunchKernelGGL(unpad_kernel<double>, dim3(blocks), dim3(256), 0, st, d.user_rows,
                           d.n[0], d.n[1], d.n[2], d.m[0], d.m[1], d.m[2], (const double*)src,
                           (double*)dst, (int)accumulate);
    else
        hipLaunchKernelGGL(unpad_kernel<float>, dim3(blocks), dim3(256), 0, st, d.user_rows,
                           d.n[0], d.n[1], d.n[2], d.m[0], d.m[1], d.m[2], (const float*)src,
                           (float*)dst, (int)accumulate);
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
    spread_tiles(a.g.dim, a.g.sp_tile, a.g.n, a.tiles, &a.tile_slow);
    const unsigned nb = (unsigned)(a.tiles[0] * a.tiles[1] * a.tiles[2] * a.g.ncomp * a.g.split);
    if (a.g.dim == 3) {
        switch (a.g.sp_tile) {
#define IBK_SPREAD_SHAPE(i)                                                                       \
    case i:                                                                                       \
        hipLaunchKernelGGL((spread_kernel<T, 3, KERN, SP_SHAPE[i][0], SP_SHAPE[i][1], SP_SHAPE[i][2]>), \
                           dim3(nb), dim3(256), 0, st, a);                                        \
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
        hipLaunchKernelGGL((spread_kernel<T, 2, KERN, SP2_TX, SP2_TY, 1>), dim3(nb), dim3(256),
                           0, st, a);
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
    } else if (a.g.dim == 3)
        hipLaunchKernelGGL((interp_kernel<T, 3, KERN>), dim3(nb), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((interp_kernel<T, 2, KERN>), dim3(nb), dim3(256), 0, st, a);
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

template <typename T, int DIM, int KERN, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    spread_waves_per_eu<T, TX, TY, TZ>()))) void batch_spread_kernel(const BatchJob* __restrict__ jobs,
                                                                     const BatchTable* __restrict__ bt)
{
    const int32_t* st = bt->starts[BS_SPREAD];
    const int nj = bt->njobs, total = st[nj];
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        const int j = batch_job_of(st, nj, vb);
        spread_body<T, DIM, KERN, TX, TY, TZ>(jobs[j].op, vb - st[j]);
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
        interp_body<T, DIM, KERN>(a, vb - st[j], nb);
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

template <typename T, int DIM, int KERN>
void batch_ops_dispatch(const BatchLaunch& b, hipStream_t st)
{
    // the built-in tile of the precision (batches are never tuned)
    constexpr int S = builtin_spread_shape(sizeof(T) == 4 ? IB_F32 : IB_F64);
    constexpr int TX = DIM == 3 ? SP_SHAPE[S][0] : SP2_TX, TY = DIM == 3 ? SP_SHAPE[S][1] : SP2_TY;
    constexpr int TZ = DIM == 3 ? SP_SHAPE[S][2] : 1;
    if (b.grid[BS_SPREAD] > 0)
        hipLaunchKernelGGL((batch_spread_kernel<T, DIM, KERN, TX, TY, TZ>), dim3(b.grid[BS_SPREAD]),
                           dim3(256), 0, st, b.jobs, b.table);
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
    with_kernel(b.kernel, [&](auto K) {
        if (b.dim == 3) batch_ops_dispatch<T, 3, decltype(K)::value>(b, st);
        else batch_ops_dispatch<T, 2, decltype(K)::value>(b, st);
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
