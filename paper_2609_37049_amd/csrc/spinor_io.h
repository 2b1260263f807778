// Native (structure-of-arrays) spinor, link and clover storage for gfx950.
//
// A block of n spinor fields is stored plane by plane, and within a plane
// site-major with the right-hand side fastest: element (plane, site s, rhs r)
// at (plane*V + s)*n + r.  A wavefront whose lanes run over (site, rhs) with
// the rhs fastest therefore reads each plane with one fully coalesced access
// of 16 bytes per lane, and all lanes of one site share the link and clover
// loads of that site:
//   IO64  : [12][V][n] double2   plane k = spin*3 + colour
//   IO32  : [6][V][n]  float4    components (2p, 2p+1)
//   IOBF  : [3][V][n]  uint4     components 4q..4q+3, each 32-bit word = bf16 re (low), bf16 im (high)
// Links [mu][9][V] complex (double2 for IO64, float2 otherwise); clover
// [2][36 reals][V] (double2 pairs for IO64, float4 quads otherwise).
#pragma once
#include "common.h"

// float -> bf16 bits, round to nearest even (NaN kept quiet)
__host__ __device__ __forceinline__ uint32_t f2bf_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__host__ __device__ __forceinline__ float bf2f(uint32_t b) { return __uint_as_float(b << 16); }

// double -> float rounded to odd, so that a following float -> bf16 RNE step
// gives the correctly rounded double -> bf16 result
__device__ __forceinline__ float d2f_odd(double d) {
    float f = __double2float_rz(d);
    if ((double)f != d) f = __uint_as_float(__float_as_uint(f) | 1u);
    return f;
}

struct IO64 {
    typedef double T;
    typedef double2 LinkT;
    typedef double2 CloverT;
    static constexpr int planes = 12;
    static constexpr int spinor_bytes = 192;
    static constexpr int real_bytes_link = 8;
    __device__ __forceinline__ static void load(const void* b, long V, int n, long r, long s, cx<T> p[12]) {
        const double2* q = (const double2*)b + s * n + r;
        const long ps = V * n;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double2 v = q[k * ps];
            p[k] = mk(v.x, v.y);
        }
    }
    __device__ __forceinline__ static void store(void* b, long V, int n, long r, long s, const cx<T> p[12]) {
        double2* q = (double2*)b + s * n + r;
        const long ps = V * n;
#pragma unroll
        for (int k = 0; k < 12; k++) q[k * ps] = make_double2(p[k].re, p[k].im);
    }
    __device__ __forceinline__ static void load_link(const LinkT* U, long V, int mu, long s, cx<T> u[9]) {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            double2 v = U[((long)mu * 9 + k) * V + s];
            u[k] = mk(v.x, v.y);
        }
    }
    __device__ __forceinline__ static void load_clover(const CloverT* A, long V, int blk, long s, T f[36]) {
#pragma unroll
        for (int q = 0; q < 18; q++) {
            double2 v = A[((long)blk * 18 + q) * V + s];
            f[2 * q] = v.x;
            f[2 * q + 1] = v.y;
        }
    }
};

struct IO32 {
    typedef float T;
    typedef float2 LinkT;
    typedef float4 CloverT;
    static constexpr int planes = 6;
    static constexpr int spinor_bytes = 96;
    static constexpr int real_bytes_link = 4;
    __device__ __forceinline__ static void load(const void* b, long V, int n, long r, long s, cx<T> p[12]) {
        const float4* q = (const float4*)b + s * n + r;
        const long ps = V * n;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            float4 v = q[k * ps];
            p[2 * k] = mk(v.x, v.y);
            p[2 * k + 1] = mk(v.z, v.w);
        }
    }
    __device__ __forceinline__ static void store(void* b, long V, int n, long r, long s, const cx<T> p[12]) {
        float4* q = (float4*)b + s * n + r;
        const long ps = V * n;
#pragma unroll
        for (int k = 0; k < 6; k++) q[k * ps] = make_float4(p[2 * k].re, p[2 * k].im, p[2 * k + 1].re, p[2 * k + 1].im);
    }
    __device__ __forceinline__ static void load_link(const LinkT* U, long V, int mu, long s, cx<T> u[9]) {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            float2 v = U[((long)mu * 9 + k) * V + s];
            u[k] = mk(v.x, v.y);
        }
    }
    __device__ __forceinline__ static void load_clover(const CloverT* A, long V, int blk, long s, T f[36]) {
#pragma unroll
        for (int q = 0; q < 9; q++) {
            float4 v = A[((long)blk * 9 + q) * V + s];
            f[4 * q] = v.x;
            f[4 * q + 1] = v.y;
            f[4 * q + 2] = v.z;
            f[4 * q + 3] = v.w;
        }
    }
};

struct IOBF {
    typedef float T;
    typedef float2 LinkT;
    typedef float4 CloverT;
    static constexpr int planes = 3;
    static constexpr int spinor_bytes = 48;
    static constexpr int real_bytes_link = 4;
    __device__ __forceinline__ static void load(const void* b, long V, int n, long r, long s, cx<T> p[12]) {
        const uint4* q = (const uint4*)b + s * n + r;
        const long ps = V * n;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            uint4 v = q[k * ps];
            p[4 * k + 0] = mk(bf2f(v.x & 0xffffu), bf2f(v.x >> 16));
            p[4 * k + 1] = mk(bf2f(v.y & 0xffffu), bf2f(v.y >> 16));
            p[4 * k + 2] = mk(bf2f(v.z & 0xffffu), bf2f(v.z >> 16));
            p[4 * k + 3] = mk(bf2f(v.w & 0xffffu), bf2f(v.w >> 16));
        }
    }
    __device__ __forceinline__ static uint32_t pack(cx<T> c) { return f2bf_rne(c.re) | (f2bf_rne(c.im) << 16); }
    __device__ __forceinline__ static void store(void* b, long V, int n, long r, long s, const cx<T> p[12]) {
        uint4* q = (uint4*)b + s * n + r;
        const long ps = V * n;
#pragma unroll
        for (int k = 0; k < 3; k++)
            q[k * ps] = make_uint4(pack(p[4 * k]), pack(p[4 * k + 1]), pack(p[4 * k + 2]), pack(p[4 * k + 3]));
    }
    __device__ __forceinline__ static void load_link(const LinkT* U, long V, int mu, long s, cx<T> u[9]) {
        IO32::load_link(U, V, mu, s, u);
    }
    __device__ __forceinline__ static void load_clover(const CloverT* A, long V, int blk, long s, T f[36]) {
        IO32::load_clover(A, V, blk, s, f);
    }
};
