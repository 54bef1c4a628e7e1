// Spreading and interpolation kernels.
//
// Spreading (eq. disc-spread, Sec. 2; parallel algorithm Alg. 4, Sec. 3.3).  Each block
// owns a tile of one component's grid and produces every value of it exactly once.  It
// reads the sorted points whose cells lie in the tile grown by the stencil reach (cells
// x0-2 .. x0+ext+1 per dimension; contiguous sorted ranges per x-row because keys are
// x-fastest).  Within a wave, each lane takes one run of equal keys -- one occupied cell --
// and reduces the contributions of all its points to the 4^d shifts in registers (the
// segmented reduce of Alg. 4 for all shifts at once).  Lanes of one wave hold distinct
// cells, so for any shift their targets differ and the 4^d read-add-writes into the LDS
// tile never collide.  The four waves of a block work on source slices (planes in 3-D,
// rows in 2-D) whose indices differ by multiples of 4, so their targets are disjoint; the
// slices are visited in 4 phases separated by barriers.  The order in which every grid
// value receives its contributions is therefore fixed by the data alone: no atomics, and
// the result is bitwise reproducible.
//
// Interpolation (eq. disc-interp; Alg. 3, Sec. 3.2).  Each block owns a tile of cells of
// one component, stages the grid values of the tile plus its stencil halo in LDS with
// coalesced loads, and gives one thread to each sorted point in those cells; the thread
// accumulates the 4^d products in registers in tensor-product order and writes its value.
#include "device_common.h"

namespace ibk {

template <typename T>
__device__ __forceinline__ T ld(const void* p, int64_t i) { return ((const T*)p)[i]; }

// Point index from a permutation entry, kept inside [0, n) so that no data can steer a
// load or store out of bounds (a valid permutation is never changed by this).
__device__ __forceinline__ int64_t clamp_index(int32_t p, int64_t n)
{
    return (uint32_t)p < (uint64_t)n ? (int64_t)p : 0;
}

// First position in sk[lo, hi) whose key is >= v (keys ascending).
__device__ __forceinline__ int64_t lower_bound_key(const int32_t* __restrict__ sk, int64_t lo,
                                                   int64_t hi, int32_t v)
{
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (sk[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Fractional offsets of point p for component c and the 1-D weights per dimension.
template <typename T, int DIM, int KERN>
__device__ __forceinline__ void point_weights(const GeomArgs& g, int c, const T* __restrict__ X,
                                              int64_t p, T w[DIM][4])
{
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const T x = X[p * DIM + k];
        const T ih = Prec<T>::inv_h(g, k);
        const T y = shifted_scaled<T>(x, ih, (T)g.comp_xi[c][k]);
        T r = y - floor(y);
        r += product_residual<T>(x, ih, Prec<T>::inv_lo(g, k));
        weights4<T, KERN>(r, w[k]);
    }
}

// ---------------------------------------------------------------------------------------
// Spreading
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// A source slice (an x-y plane of cells in 3-D, one x-row in 2-D) as a list of sorted
// ranges: one per x-row piece (at most 3 pieces per row, since a tile is never wider than
// the grid).  Each range carries the unwrapped tile offsets of its cells.
template <int MAXR>
struct SliceTable {
    int32_t lo[MAXR];
    int32_t hi[MAXR];
    int32_t xoff[MAXR];   // unwrapped x position (relative to x0 - 2) = key % n0 + xoff
    int32_t uy[MAXR];     // unwrapped y position relative to y0 - 2
    int32_t pref[MAXR + 1];
};

template <typename T, int DIM, int KERN, int TX, int TY, int TZ>
struct SpreadTile {
    static constexpr int NZ = (DIM == 3) ? 4 : 1;          // stencil extent in z
    static constexpr int MAXROWS = (DIM == 3) ? TY + 3 : 1; // x-rows per slice
    static constexpr int MAXR = 3 * MAXROWS;
    using Table = SliceTable<MAXR>;

    // Build the range table of slice (cz or cy) for this wave; returns the point count.
    __device__ static int build(const OpArgs& a, const int32_t* __restrict__ sk,
                                const int32_t* __restrict__ rs, int qslice, int x0, int y0,
                                int z0, int ex, int ey, Table& tb)
    {
        const GeomArgs& g = a.g;
        const int lane = lane_id();
        const int n0 = g.n[0];
        const int nrows = (DIM == 3) ? ey + 3 : 1;
        int count = 0;
        if (lane < nrows) {
            int cy, r, uy;
            if (DIM == 3) {
                const int cz = emod(z0 - 2 + qslice, g.n[2]);
                uy = lane;
                cy = emod(y0 - 2 + lane, g.n[1]);
                r = cz * g.n[1] + cy;
            } else {
                uy = qslice;
                cy = emod(y0 - 2 + qslice, g.n[1]);
                r = cy;
            }
            const int32_t rlo = rs[r], rhi = rs[r + 1];
            const int32_t rowbase = r * n0;
            const int total = ex + 3;
            int done = 0;
            for (int k = 0; k < 3; ++k) {
                int32_t lo = 0, hi = 0, xoff = 0;
                if (done < total && rlo < rhi) {
                    const int xa = emod(x0 - 2 + done, n0);
                    const int len = min(total - done, n0 - xa);
                    lo = (int32_t)lower_bound_key(sk, rlo, rhi, rowbase + xa);
                    hi = (int32_t)lower_bound_key(sk, lo, rhi, rowbase + xa + len);
                    xoff = done - xa;
                    done += len;
                }
                tb.lo[lane * 3 + k] = lo;
                tb.hi[lane * 3 + k] = hi;
                tb.xoff[lane * 3 + k] = xoff;
                tb.uy[lane * 3 + k] = uy;
                count += hi - lo;
            }
        }
        const uint32_t incl = wave_incl_scan_u32((uint32_t)count);
        if (lane < nrows) {
            int run = (int)incl - count;
            for (int k = 0; k < 3; ++k) {
                tb.pref[lane * 3 + k] = run;
                run += tb.hi[lane * 3 + k] - tb.lo[lane * 3 + k];
            }
        }
        const int total_pts = __shfl((int)incl, 63, 64);
        if (lane == 0) tb.pref[nrows * 3] = total_pts;
        wave_sync();
        return total_pts;
    }

    // Reduce every run of equal keys of the slice in registers (one lane per run) and add
    // the 4^d sums into the tile.  uz: the slice's unwrapped z offset (3-D).
    __device__ static void reduce(const OpArgs& a, int c, const int32_t* __restrict__ sk,
                                  const int32_t* __restrict__ perm, const Table& tb,
                                  int nranges, int total, int uz, int ex, int ey, int ez,
                                  T* tile)
    {
        const GeomArgs& g = a.g;
        const T* __restrict__ X = (const T*)a.X;
        const T* __restrict__ F = (const T*)a.F;
        const int lane = lane_id();
        const int n0 = g.n[0];
        int v0 = 0;
        while (v0 < total) {
            const int v = v0 + lane;
            const bool valid = v < total;
            int rr = 0;
            if (valid) {  // last range whose prefix is <= v (it is non-empty)
                int lo = 0, hi = nranges;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (tb.pref[mid] <= v) lo = mid;
                    else hi = mid;
                }
                rr = lo;
            }
            const int32_t rlo = tb.lo[rr], rhi = tb.hi[rr], rpref = tb.pref[rr];
            const int64_t j = (int64_t)rlo + (v - rpref);
            const int32_t key = valid ? sk[j] : -1;
            const bool head = valid && (v == rpref || sk[j - 1] != key);
            int seg_end = valid ? v : v0;
            T acc[NZ][4][4];
#pragma unroll
            for (int iz = 0; iz < NZ; ++iz)
#pragma unroll
                for (int iy = 0; iy < 4; ++iy)
#pragma unroll
                    for (int ix = 0; ix < 4; ++ix) acc[iz][iy][ix] = T(0);
            if (head) {
                int64_t jj = j;
                do {
                    const int64_t p = clamp_index(perm[jj], g.npts);
                    T w[DIM][4];
                    point_weights<T, DIM, KERN>(g, c, X, p, w);
                    const T Fc = F[p * g.ncomp + c];
#pragma unroll
                    for (int iz = 0; iz < NZ; ++iz) {
                        const T wzF = (DIM == 3) ? w[DIM - 1][iz] * Fc : Fc;
#pragma unroll
                        for (int iy = 0; iy < 4; ++iy) {
                            const T cyz = w[1][iy] * wzF;
#pragma unroll
                            for (int ix = 0; ix < 4; ++ix)
                                acc[iz][iy][ix] = fma(w[0][ix], cyz, acc[iz][iy][ix]);
                        }
                    }
                    ++jj;
                } while (jj < rhi && sk[jj] == key);
                seg_end = rpref + (int)(jj - rlo);
            }
            const int next = wave_max_i32(seg_end);
            if (head) {
                const int ux = tb.xoff[rr] + (key % n0);
                const int uy = tb.uy[rr];
#pragma unroll
                for (int iz = 0; iz < NZ; ++iz) {
                    const int tz = (DIM == 3) ? uz - 3 + iz : 0;
                    if (tz < 0 || tz >= ez) continue;
#pragma unroll
                    for (int iy = 0; iy < 4; ++iy) {
                        const int ty = uy - 3 + iy;
                        if (ty < 0 || ty >= ey) continue;
                        T* row = tile + (tz * TY + ty) * TX;
#pragma unroll
                        for (int ix = 0; ix < 4; ++ix) {
                            const int tx = ux - 3 + ix;
                            if (tx >= 0 && tx < ex) row[tx] += acc[iz][iy][ix];
                        }
                    }
                }
            }
            v0 = next;
        }
    }
};

template <typename T, int DIM, int KERN, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void spread_kernel(OpArgs a)
{
    using ST = SpreadTile<T, DIM, KERN, TX, TY, TZ>;
    __shared__ T tile[TX * TY * TZ];
    __shared__ typename ST::Table tables[4];
    const GeomArgs& g = a.g;
    int b = blockIdx.x;
    const int bx = b % a.tiles[0]; b /= a.tiles[0];
    const int by = b % a.tiles[1]; b /= a.tiles[1];
    const int bz = b % a.tiles[2]; b /= a.tiles[2];
    const int c = b;
    const int s = g.comp_stag[c];
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int ex = min(TX, g.n[0] - x0), ey = min(TY, g.n[1] - y0);
    const int ez = (DIM == 3) ? min(TZ, g.n[2] - z0) : 1;

    for (int i = threadIdx.x; i < TX * TY * TZ; i += blockDim.x) tile[i] = T(0);
    __syncthreads();

    const int32_t* sk = a.sorted_keys + (int64_t)s * g.npts;
    const int32_t* perm = a.perm + (int64_t)s * g.npts;
    const int32_t* rs = a.row_start + (int64_t)s * (g.rows + 1);
    const int w = wave_id();
    const int nslices = (DIM == 3) ? ez + 3 : ey + 3;
    const int nranges = 3 * ((DIM == 3) ? ey + 3 : 1);
    typename ST::Table& tb = tables[w];

    // Slices q and q + 4 feed disjoint target slices, so the four waves take slices
    // q = phase + 4m concurrently and the phases are separated by barriers.
    for (int phase = 0; phase < 4; ++phase) {
        for (int m = w;; m += 4) {
            const int q = phase + 4 * m;
            if (q >= nslices) break;
            const int total = ST::build(a, sk, rs, q, x0, y0, z0, ex, ey, tb);
            if (total > 0) ST::reduce(a, c, sk, perm, tb, nranges, total, q, ex, ey, ez, tile);
            wave_sync();
        }
        __syncthreads();
    }

    T* f = (T*)a.f;
    const int64_t G = (int64_t)g.n[0] * g.n[1] * (DIM == 3 ? g.n[2] : 1);
    const T scale = (T)g.scale;
    const int cnt = ex * ey * ez;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const int xr = i % ex, yr = (i / ex) % ey, zr = i / (ex * ey);
        const int64_t gi = ((int64_t)(z0 + zr) * g.n[1] + (y0 + yr)) * g.n[0] + (x0 + xr);
        const T v = tile[(zr * TY + yr) * TX + xr] * scale;
        T* dst = f + (int64_t)c * G + gi;
        *dst = a.accumulate ? *dst + v : v;
    }
}

// ---------------------------------------------------------------------------------------
// Interpolation
// ---------------------------------------------------------------------------------------
template <typename T, int DIM, int KERN, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void interp_kernel(OpArgs a)
{
    constexpr int PX = TX + 3, PY = TY + 3, PZ = (DIM == 3) ? TZ + 3 : 1;
    constexpr int NROWS = TY * TZ;
    static_assert(NROWS <= 256, "row table sized for one block");
    __shared__ T ut[PX * PY * PZ];
    __shared__ int64_t s_lo[NROWS];
    __shared__ uint32_t s_pref[NROWS + 1];
    __shared__ uint32_t s_scan[5];

    const GeomArgs& g = a.g;
    int b = blockIdx.x;
    const int bx = b % a.tiles[0]; b /= a.tiles[0];
    const int by = b % a.tiles[1]; b /= a.tiles[1];
    const int bz = b % a.tiles[2]; b /= a.tiles[2];
    const int c = b;
    const int s = g.comp_stag[c];
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int ex = min(TX, g.n[0] - x0), ey = min(TY, g.n[1] - y0);
    const int ez = (DIM == 3) ? min(TZ, g.n[2] - z0) : 1;
    const int n0 = g.n[0], n1 = g.n[1], n2 = (DIM == 3) ? g.n[2] : 1;
    const int64_t G = (int64_t)n0 * n1 * n2;
    const T* __restrict__ u = (const T*)a.u + (int64_t)c * G;

    // Grid values of cells x0-1 .. x0+ex+1 (and likewise in y, z), periodic.
    const int lx = ex + 3, ly = ey + 3, lz = (DIM == 3) ? ez + 3 : 1;
    for (int i = threadIdx.x; i < lx * ly * lz; i += blockDim.x) {
        const int xr = i % lx, yr = (i / lx) % ly, zr = i / (lx * ly);
        const int gx = emod(x0 - 1 + xr, n0), gy = emod(y0 - 1 + yr, n1);
        const int gz = (DIM == 3) ? emod(z0 - 1 + zr, n2) : 0;
        ut[(zr * PY + yr) * PX + xr] = u[((int64_t)gz * n1 + gy) * n0 + gx];
    }

    // Sorted ranges of the tile's x-rows.
    const int32_t* sk = a.sorted_keys + (int64_t)s * g.npts;
    const int32_t* perm = a.perm + (int64_t)s * g.npts;
    const int32_t* rs = a.row_start + (int64_t)s * (g.rows + 1);
    const int nrows = ey * ez;
    uint32_t cnt = 0;
    if ((int)threadIdx.x < nrows) {
        const int yr = threadIdx.x % ey, zr = threadIdx.x / ey;
        const int r = (DIM == 3) ? (z0 + zr) * n1 + (y0 + yr) : (y0 + yr);
        const int32_t rowbase = r * n0;
        const int64_t lo = lower_bound_key(sk, rs[r], rs[r + 1], rowbase + x0);
        const int64_t hi = lower_bound_key(sk, lo, rs[r + 1], rowbase + x0 + ex);
        s_lo[threadIdx.x] = lo;
        cnt = (uint32_t)(hi - lo);
    }
    uint32_t total;
    const uint32_t pre = block_excl_scan_u32<256>(cnt, s_scan, &total);
    if ((int)threadIdx.x < nrows) s_pref[threadIdx.x] = pre;
    if (threadIdx.x == 0) s_pref[nrows] = total;
    __syncthreads();

    const T* __restrict__ X = (const T*)a.X;
    T* U = (T*)a.U;
    for (uint32_t i = threadIdx.x; i < total; i += blockDim.x) {
        int lo = 0, hi = nrows;  // find the row: s_pref[row] <= i < s_pref[row+1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_pref[mid] <= i) lo = mid;
            else hi = mid;
        }
        const int row = lo;
        const int64_t j = s_lo[row] + (i - s_pref[row]);
        const int yr = row % ey, zr = row / ey;
        const int xr = min(max(sk[j] % n0 - x0, 0), ex - 1);
        const int64_t p = clamp_index(perm[j], g.npts);
        T w[DIM][4];
        point_weights<T, DIM, KERN>(g, c, X, p, w);
        T sum = T(0);
#pragma unroll
        for (int iz = 0; iz < ((DIM == 3) ? 4 : 1); ++iz) {
            T sy = T(0);
#pragma unroll
            for (int iy = 0; iy < 4; ++iy) {
                const T* line = ut + ((zr + iz) * PY + (yr + iy)) * PX + xr;
                T sx = T(0);
#pragma unroll
                for (int ix = 0; ix < 4; ++ix) sx = fma(w[0][ix], line[ix], sx);
                sy = fma(w[1][iy], sx, sy);
            }
            sum = (DIM == 3) ? fma(w[DIM - 1][iz], sy, sum) : sy;
        }
        U[p * g.ncomp + c] = sum;
    }
}

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
namespace {
constexpr int SP_TX = 32, SP_TY = 16, SP_TZ = 13;   // spreading tile (3-D)
constexpr int SP2_TX = 64, SP2_TY = 32;             // spreading tile (2-D)
constexpr int IN_TX = 64, IN_TY = 8, IN_TZ = 2;     // interpolation tile (3-D)
constexpr int IN2_TX = 64, IN2_TY = 16;             // interpolation tile (2-D)

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

template <typename T, int KERN>
hipError_t spread_dispatch(OpArgs a, hipStream_t st)
{
    if (a.g.dim == 3) {
        a.tiles[0] = cdiv(a.g.n[0], SP_TX);
        a.tiles[1] = cdiv(a.g.n[1], SP_TY);
        a.tiles[2] = cdiv(a.g.n[2], SP_TZ);
        const unsigned nb = (unsigned)(a.tiles[0] * a.tiles[1] * a.tiles[2] * a.g.ncomp);
        hipLaunchKernelGGL((spread_kernel<T, 3, KERN, SP_TX, SP_TY, SP_TZ>), dim3(nb), dim3(256),
                           0, st, a);
    } else {
        a.tiles[0] = cdiv(a.g.n[0], SP2_TX);
        a.tiles[1] = cdiv(a.g.n[1], SP2_TY);
        a.tiles[2] = 1;
        const unsigned nb = (unsigned)(a.tiles[0] * a.tiles[1] * a.g.ncomp);
        hipLaunchKernelGGL((spread_kernel<T, 2, KERN, SP2_TX, SP2_TY, 1>), dim3(nb), dim3(256),
                           0, st, a);
    }
    return hipGetLastError();
}

template <typename T, int KERN>
hipError_t interp_dispatch(OpArgs a, hipStream_t st)
{
    if (a.g.dim == 3) {
        a.tiles[0] = cdiv(a.g.n[0], IN_TX);
        a.tiles[1] = cdiv(a.g.n[1], IN_TY);
        a.tiles[2] = cdiv(a.g.n[2], IN_TZ);
        const unsigned nb = (unsigned)(a.tiles[0] * a.tiles[1] * a.tiles[2] * a.g.ncomp);
        hipLaunchKernelGGL((interp_kernel<T, 3, KERN, IN_TX, IN_TY, IN_TZ>), dim3(nb), dim3(256),
                           0, st, a);
    } else {
        a.tiles[0] = cdiv(a.g.n[0], IN2_TX);
        a.tiles[1] = cdiv(a.g.n[1], IN2_TY);
        a.tiles[2] = 1;
        const unsigned nb = (unsigned)(a.tiles[0] * a.tiles[1] * a.g.ncomp);
        hipLaunchKernelGGL((interp_kernel<T, 2, KERN, IN2_TX, IN2_TY, 1>), dim3(nb), dim3(256),
                           0, st, a);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_spread(const OpArgs& a, int dtype, int kernel, hipStream_t st)
{
    if (dtype == IB_F64)
        return kernel == IB_KERNEL_COSINE4 ? spread_dispatch<double, IB_KERNEL_COSINE4>(a, st)
                                           : spread_dispatch<double, IB_KERNEL_PESKIN4>(a, st);
    return kernel == IB_KERNEL_COSINE4 ? spread_dispatch<float, IB_KERNEL_COSINE4>(a, st)
                                       : spread_dispatch<float, IB_KERNEL_PESKIN4>(a, st);
}

hipError_t launch_interp(const OpArgs& a, int dtype, int kernel, hipStream_t st)
{
    if (dtype == IB_F64)
        return kernel == IB_KERNEL_COSINE4 ? interp_dispatch<double, IB_KERNEL_COSINE4>(a, st)
                                           : interp_dispatch<double, IB_KERNEL_PESKIN4>(a, st);
    return kernel == IB_KERNEL_COSINE4 ? interp_dispatch<float, IB_KERNEL_COSINE4>(a, st)
                                       : interp_dispatch<float, IB_KERNEL_PESKIN4>(a, st);
}

}  // namespace ibk
