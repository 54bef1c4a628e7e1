// Device helpers shared by the HIP kernels: wave64 primitives, block scans, the cell /
// fractional-offset computation and the 4-point kernel weights.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ib_internal.h"

namespace ibk {

// Workgroups of a launch are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8), and each XCD has its own L2.  xcd_block renumbers the workgroups so that each
// XCD runs one contiguous range of logical blocks: neighbouring work then shares an L2.
// A bijection of [0, nblk) for every nblk.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_block(int b, int nblk)
{
    const int x = b % NUM_XCD, i = b / NUM_XCD;
    const int q = nblk / NUM_XCD, r = nblk % NUM_XCD;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }

// ---- cross-lane steps on DPP lane moves ------------------------------------------------
// A wave64 is four rows of 16 lanes.  DPP (data-parallel primitives) moves a VGPR between
// lanes inside the VALU instruction, with no LDS round trip.  Encodings (GFX9 DPP_CTRL):
// row_shr:n = 0x110 + n (lane l reads l - n within its row), row_bcast:15 = 0x142 (lane 15 of a row to every lane of the
// next row) and row_bcast:31 = 0x143 (lane 31 to rows 2 and 3).  ROWS masks the rows that
// are written; lanes that are not written, or whose source lane does not exist, get 0.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint32_t dpp_move(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}

// Inclusive prefix sum over the lanes of a wave (a Hillis-Steele scan within rows, then
// the row totals carried across rows).
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v)
{
    v += dpp_move<0x111>(v);
    v += dpp_move<0x112>(v);
    v += dpp_move<0x114>(v);
    v += dpp_move<0x118>(v);
    v += dpp_move<0x142, 0xa>(v);
    v += dpp_move<0x143, 0xc>(v);
    return v;
}

// Inclusive prefix maximum of non-negative values over the lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_max_u32(uint32_t v)
{
    v = max(v, dpp_move<0x111>(v));
    v = max(v, dpp_move<0x112>(v));
    v = max(v, dpp_move<0x114>(v));
    v = max(v, dpp_move<0x118>(v));
    v = max(v, dpp_move<0x142, 0xa>(v));
    v = max(v, dpp_move<0x143, 0xc>(v));
    return v;
}

// Value of lane 63, uniform across the wave.
__device__ __forceinline__ uint32_t wave_last_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Maximum of non-negative values over the wave, uniform across the wave.
__device__ __forceinline__ int wave_max_i32(int v)
{
    return (int)wave_last_u32(wave_incl_max_u32((uint32_t)v));
}

// Exclusive scan of one value per thread over a block of NT threads (NT a multiple of
// 64, at most 1024).  `scratch` holds NT/64 + 1 words of LDS.  Returns the exclusive
// prefix; *total receives the block sum.  Must be called by all threads.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t* scratch,
                                                        uint32_t* total)
{
    constexpr int NW = NT / 64;
    const int lane = lane_id(), w = wave_id();
    uint32_t incl = wave_incl_scan_u32(v);
    if (lane == 63) scratch[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < NW; ++i) {
            uint32_t t = scratch[i];
            scratch[i] = run;
            run += t;
        }
        scratch[NW] = run;
    }
    __syncthreads();
    uint32_t r = scratch[w] + incl - v;
    *total = scratch[NW];
    __syncthreads();
    return r;
}

// ---- scaled coordinates, cells and fractional offsets ----------------------------------
//
// The cell of coordinate X on staggering xi is floor(t - xi) with t = X * inv_h rounded
// once in the working precision and never fused with the subtraction, so that cell keys
// are reproducible bit for bit.  The fractional offset r = (t - xi) - floor(t - xi) is then
// corrected by the exact rounding residual of the product and by the residual of inv_h
// itself, so the weights see X / h to working precision.

template <typename T> struct Prec;
template <> struct Prec<double> {
    __device__ static double inv_h(const GeomArgs& g, int k) { return g.inv_h_d[k]; }
    __device__ static double inv_lo(const GeomArgs& g, int k) { return g.inv_lo_d[k]; }
};
template <> struct Prec<float> {
    __device__ static float inv_h(const GeomArgs& g, int k) { return g.inv_h_f[k]; }
    __device__ static float inv_lo(const GeomArgs& g, int k) { return g.inv_lo_f[k]; }
};

template <typename T>
__device__ __forceinline__ T shifted_scaled(T x, T inv_h, T xi)
{
#pragma clang fp contract(off)
    T t = x * inv_h;
    return t - xi;
}

template <typename T>
__device__ __forceinline__ T product_residual(T x, T inv_h, T inv_lo)
{
#pragma clang fp contract(off)
    T t = x * inv_h;
    return fma(x, inv_h, -t) + x * inv_lo;
}

// Square root of x in [1/4, 2] (the arguments of the 4-point and 3-point weights): the
// hardware reciprocal square root refined by one Goldschmidt step and one Newton
// correction, accurate to one ulp on that interval without the range handling of the
// general routine.  FP32 uses the
// hardware square root (one ulp).
__device__ __forceinline__ double weight_sqrt(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}

__device__ __forceinline__ float weight_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ---- support of the one-dimensional kernels -------------------------------------------
// A point's cell along one axis, from y = fl(x inv_h) - xi, and the nodes its weights fall
// on.  Even support (the 4-point kernels, s = 4): the cell is floor(y) and the nodes are
// cell - 1 .. cell + 2.  Odd support (the 3-point kernel, s = 3): the de facto cell of
// Fig. 1(b) is centred on a grid node -- the node nearest the point, floor(y + 1/2), ties
// going up -- and the nodes are cell - 1 .. cell + 1 (shifts -1, 0, 1).
template <int KERN>
constexpr int support_width() { return KERN == IB_KERNEL_ROMA3 ? 3 : 4; }

// Cell of y (as a double, not yet wrapped) and the point's offset from it: r = y - cell in
// [0, 1) for even support, in [-1/2, 1/2) for odd support (odd = the kernel's support is
// odd).  Both are exact: y - floor(y) is, and so is subtracting 1 from it.
template <typename T>
__device__ __forceinline__ double axis_cell(T y, bool odd, T* r)
{
    const T fy = floor(y);
    T rr = y - fy;
    const bool up = odd && rr >= T(0.5);
    *r = up ? rr - T(1) : rr;
    return (double)fy + (up ? 1.0 : 0.0);
}

// ---- one-dimensional kernel weights --------------------------------------------------
// Even support: w[k] = phi(k - 1 - r) for the four nodes cell - 1 + k, r in [0, 1).
template <typename T, int KERN>
__device__ __forceinline__ void weights4(T r, T w[4])
{
    static_assert(support_width<KERN>() == 4, "even-support kernels only");
    if constexpr (KERN == IB_KERNEL_COSINE4) {
        T s, c;
        if constexpr (sizeof(T) == 8) sincospi(0.5 * r, &s, &c);
        else sincospif(0.5f * r, &s, &c);
        const T q = T(0.25);
        w[0] = q - q * s;
        w[1] = q + q * c;
        w[2] = q + q * s;
        w[3] = q - q * c;
    } else {
        // Peskin 4-point, with s = sqrt(1 + 4r - 4r^2): phi(-1-r) = (3 - 2r - s)/8,
        // phi(r) = (3 - 2r + s)/8, phi(1-r) = (1 + 2r + s)/8, phi(2-r) = (1 + 2r - s)/8.
        // The two differences lose relative (not absolute) accuracy when a weight is
        // tiny, which leaves every weighted sum accurate to working precision.
        const T s = weight_sqrt(T(1) + T(4) * r * (T(1) - r));
        const T a = T(3) - T(2) * r;
        const T b = T(1) + T(2) * r;
        w[0] = (a - s) * T(0.125);
        w[1] = (a + s) * T(0.125);
        w[2] = (b + s) * T(0.125);
        w[3] = (b - s) * T(0.125);
    }
}

// Odd support (3-point kernel): the three nodes cell - 1, cell, cell + 1 for the point at
// signed offset m in [-1/2, 1/2] from its cell's node.  With s = sqrt(1 - 3 m^2): the node
// weighs (1 + s)/3, its lower neighbour (2 - 3m - s)/6, its upper neighbour (2 + 3m - s)/6.
template <typename T>
__device__ __forceinline__ void weights3(T m, T w[3])
{
    const T s = weight_sqrt(T(1) - T(3) * m * m);
    w[0] = (T(2) - s - T(3) * m) * T(1.0 / 6.0);
    w[1] = (T(1) + s) * T(1.0 / 3.0);
    w[2] = (T(2) - s + T(3) * m) * T(1.0 / 6.0);
}

// The weights of the SW = support_width<KERN>() nodes from the offset r of axis_cell.
template <typename T, int KERN>
__device__ __forceinline__ void weights_of(T r, T w[4])
{
    if constexpr (support_width<KERN>() == 3) weights3<T>(r, w);
    else weights4<T, KERN>(r, w);
}

// The weights times 2^weight_shift<KERN>(): the Peskin kernel's four weights without their
// common factor 1/8.  Scaling by a power of two is exact, so a product of scaled weights and
// a value scaled by the inverse power has the same bits as the product of the weights.
template <int KERN>
constexpr int weight_shift() { return KERN == IB_KERNEL_PESKIN4 ? 3 : 0; }

template <typename T, int KERN>
__device__ __forceinline__ void weights_scaled(T r, T w[4])
{
    if constexpr (KERN == IB_KERNEL_PESKIN4) {
        const T s = weight_sqrt(T(1) + T(4) * r * (T(1) - r));
        const T a = T(3) - T(2) * r;
        const T b = T(1) + T(2) * r;
        w[0] = a - s;
        w[1] = a + s;
        w[2] = b + s;
        w[3] = b - s;
    } else {
        weights_of<T, KERN>(r, w);
    }
}

// Derivatives d w[k] / d r of the weights of weights_of (r increases with X).
template <typename T, int KERN>
__device__ __forceinline__ void dweights_of(T r, T dw[4])
{
    if constexpr (KERN == IB_KERNEL_COSINE4) {
        T s, c;
        if constexpr (sizeof(T) == 8) sincospi(0.5 * r, &s, &c);
        else sincospif(0.5f * r, &s, &c);
        const T q = T(3.14159265358979323846 / 8.0);
        dw[0] = -q * c;
        dw[1] = -q * s;
        dw[2] = q * c;
        dw[3] = q * s;
    } else if constexpr (KERN == IB_KERNEL_PESKIN4) {
        // with s = sqrt(1 + 4r - 4r^2), ds/dr = (2 - 4r) / s
        const T s = sqrt(T(1) + T(4) * r * (T(1) - r));
        const T ds = (T(2) - T(4) * r) / s;
        dw[0] = (T(-2) - ds) * T(0.125);
        dw[1] = (T(-2) + ds) * T(0.125);
        dw[2] = (T(2) + ds) * T(0.125);
        dw[3] = (T(2) - ds) * T(0.125);
    } else {
        // 3-point kernel (see weights3), m = r: ds/dm = -3m / s.
        const T ds = T(-3) * r / sqrt(T(1) - T(3) * r * r);
        dw[0] = (T(-3) - ds) * T(1.0 / 6.0);
        dw[1] = ds * T(1.0 / 3.0);
        dw[2] = (T(3) - ds) * T(1.0 / 6.0);
        dw[3] = T(0);
    }
}

// a mod n for a in [-n, 2n) (unwrapped tile and halo coordinates), without division.
__device__ __forceinline__ int wrap_small(int a, int n)
{
    a = a < 0 ? a + n : a;
    return a >= n ? a - n : a;
}

// Euclidean floor(y) mod n for |y| < 2^30: double arithmetic on exact integers, with a
// one-step correction of the quotient.
__device__ __forceinline__ int floor_mod(double fy, int n, double inv_n)
{
    const double q = floor(fy * inv_n);
    double c = fy - q * (double)n;
    c = c < 0.0 ? c + (double)n : c;
    c = c >= (double)n ? c - (double)n : c;
    return (int)c;
}

// Point index from a permutation entry, kept inside [0, n) so that no data can steer a
// load or store out of bounds (a valid permutation is never changed by this).
__device__ __forceinline__ int64_t clamp_index(int32_t p, int64_t n)
{
    return (uint32_t)p < (uint64_t)n ? (int64_t)p : 0;
}

}  // namespace ibk
