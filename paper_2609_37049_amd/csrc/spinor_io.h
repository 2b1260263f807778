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

// Element at byte offset `off` (32-bit, per lane) past the wave-uniform base
// b + plane_bytes: lets the compiler address every plane with one scalar base
// and the same vector offset instead of a 64-bit address per load.  All
// blocks handed to the stencil are below 4 GiB per plane.
template <typename E>
__device__ __forceinline__ E ld_at(const void* b, size_t plane_bytes, unsigned off) {
    const char* base = (const char*)b + plane_bytes;
    return *(const E*)(base + off);
}
// NT: a streaming (non-temporal) store, for outputs that the same launch
// never reads again, so that they do not displace reused inputs from L2.
template <bool NT = false, typename E>
__device__ __forceinline__ void st_at(void* b, size_t plane_bytes, unsigned off, E v) {
    char* base = (char*)b + plane_bytes;
    if constexpr (NT) {
        typedef unsigned wv __attribute__((ext_vector_type(sizeof(E) / 4)));
        __builtin_nontemporal_store(__builtin_bit_cast(wv, v), (wv*)(base + off));
    } else {
        *(E*)(base + off) = v;
    }
}

// Buffer-resource loads: one descriptor (wave-uniform, scalar registers) for a
// whole array, a 32-bit per-lane byte offset and a scalar per-plane offset.
// The hardware checks every access against num_records and returns zero
// beyond it.  Arrays passed this way stay below 4 GiB.
typedef __amdgpu_buffer_rsrc_t brsrc;
__device__ __forceinline__ brsrc make_rsrc(const void* p, unsigned nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}
typedef unsigned u4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u4v bld16(brsrc r, unsigned voff, unsigned soff) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
}
__device__ __forceinline__ u2v bld8(brsrc r, unsigned voff, unsigned soff) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
}

// Read-only views handed to the stencil: base pointer, bytes a descriptor
// covers (the whole block; one plane for FP64), and whether the buffer path
// applies (those bytes below 4 GiB).
struct RoView {
    const void* p;
    unsigned nbytes;
    int buf;
};

struct IO64 {
    typedef double T;
    typedef double2 LinkT;
    typedef double2 CloverT;
    static constexpr int planes = 12;
    static constexpr int spinor_bytes = 192;
    static constexpr int real_bytes_link = 8;
    __device__ __forceinline__ static void load(const void* b, long V, int n, int r, int s, cx<T> p[12]) {
        const unsigned off = ((unsigned)s * (unsigned)n + (unsigned)r) * 16u;
        const size_t ps = (size_t)V * n * 16;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double2 v = ld_at<double2>(b, k * ps, off);
            p[k] = mk(v.x, v.y);
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ static void store(void* b, long V, int n, int r, int s, const cx<T> p[12]) {
        const unsigned off = ((unsigned)s * (unsigned)n + (unsigned)r) * 16u;
        const size_t ps = (size_t)V * n * 16;
#pragma unroll
        for (int k = 0; k < 12; k++) st_at<NT>(b, k * ps, off, make_double2(p[k].re, p[k].im));
    }
    // FP64 blocks reach 4 GiB long before one plane does (12 planes of
    // V n 16 bytes): one descriptor per plane, b.nbytes = the plane's bytes
    template <bool BUF>
    __device__ __forceinline__ static void loadv(const RoView& b, long V, int n, int r, int s, cx<T> p[12]) {
        if constexpr (BUF) {
            const unsigned off = ((unsigned)s * (unsigned)n + (unsigned)r) * 16u;
            const size_t ps = (size_t)V * n * 16;
#pragma unroll
            for (int k = 0; k < 12; k++) {
                const brsrc rs = make_rsrc((const char*)b.p + k * ps, b.nbytes);
                u4v v = bld16(rs, off, 0u);
                p[k] = mk(__hiloint2double(v[1], v[0]), __hiloint2double(v[3], v[2]));
            }
        } else {
            load(b.p, V, n, r, s, p);
        }
    }
    __device__ __forceinline__ static void load_link(const LinkT* U, long V, int mu, int s, cx<T> u[9]) {
        const brsrc rs = make_rsrc(U, (unsigned)(V * 36 * 16));
        const unsigned off = (unsigned)s * 16u;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            u4v v = bld16(rs, off, (unsigned)((mu * 9 + k) * V * 16));
            u[k] = mk(__hiloint2double(v[1], v[0]), __hiloint2double(v[3], v[2]));
        }
    }
    __device__ __forceinline__ static void load_clover(const CloverT* A, long V, int blk, int s, T f[36]) {
        const brsrc rs = make_rsrc(A, (unsigned)(V * 36 * 16));
        const unsigned off = (unsigned)s * 16u;
#pragma unroll
        for (int q = 0; q < 18; q++) {
            u4v v = bld16(rs, off, (unsigned)((blk * 18 + q) * V * 16));
            f[2 * q] = __hiloint2double(v[1], v[0]);
            f[2 * q + 1] = __hiloint2double(v[3], v[2]);
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
    __device__ __forceinline__ static void load(const void* b, long V, int n, int r, int s, cx<T> p[12]) {
        const unsigned off = ((unsigned)s * (unsigned)n + (unsigned)r) * 16u;
        const size_t ps = (size_t)V * n * 16;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            float4 v = ld_at<float4>(b, k * ps, off);
            p[2 * k] = mk(v.x, v.y);
            p[2 * k + 1] = mk(v.z, v.w);
        }
    }
    template <bool NT = false>
    __device__ __forceinline__ static void store(void* b, long V, int n, int r, int s, const cx<T> p[12]) {
        const unsigned off = ((unsigned)s * (unsigned)n + (unsigned)r) * 16u;
        const size_t ps = (size_t)V * n * 16;
#pragma unroll
        for (int k = 0; k < 6; k++)
            st_at<NT>(b, k * ps, off, make_float4(p[2 * k].re, p[2 * k].im, p[2 * k + 1].re, p[2 * k + 1].im));
    }
    template <bool BUF>
    __device__ __forceinline__ static void loadv(const RoView& b, long V, int n, int r, int s, cx<T> p[12]) {
        if constexpr (BUF) {
            const brsrc rs = make_rsrc(b.p, b.nbytes);
            const unsigned off = ((unsigned)s * (unsigned)n + (unsigned)r) * 16u;
            const unsigned ps = (unsigned)V * (unsigned)n * 16u;
#pragma unroll
            for (int k = 0; k < 6; k++) {
                u4v v = bld16(rs, off, k * ps);
                p[2 * k] = mk(__uint_as_float(v[0]), __uint_as_float(v[1]));
                p[2 * k + 1] = mk(__uint_as_float(v[2]), __uint_as_float(v[3]));
            }
        } else {
            load(b.p, V, n, r, s, p);
        }
    }
    __device__ __forceinline__ static void load_link(const LinkT* U, long V, int mu, int s, cx<T> u[9]) {
        const brsrc rs = make_rsrc(U, (unsigned)(V * 36 * 8));
        const unsigned off = (unsigned)s * 8u;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            u2v v = bld8(rs, off, (unsigned)((mu * 9 + k) * V * 8));
            u[k] = mk(__uint_as_float(v[0]), __uint_as_float(v[1]));
        }
    }
    __device__ __forceinline__ static void load_clover(const CloverT* A, long V, int blk, int s, T f[36]) {
        const brsrc rs = make_rsrc(A, (unsigned)(V * 18 * 16));
        const unsigned off = (unsigned)s * 16u;
#pragma unroll
        for (int q = 0; q < 9; q++) {
            u4v v = bld16(rs, off, (unsigned)((blk * 9 + q) * V * 16));
            f[4 * q] = __uint_as_float(v[0]);
            f[4 * q + 1] = __uint_as_float(v[1]);
            f[4 * q + 2] = __uint_as_float(v[2]);
            f[4 * q + 3] = __uint_as_float(v[3]);
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
    __device__ __forceinline__ static void load(const void* b, long V, int n, int r, int s, cx<T> p[12]) {
        const unsigned off = ((unsigned)s * (unsigned)n + (unsigned)r) * 16u;
        const size_t ps = (size_t)V * n * 16;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            uint4 v = ld_at<uint4>(b, k * ps, off);
            p[4 * k + 0] = mk(bf2f(v.x & 0xffffu), bf2f(v.x >> 16));
            p[4 * k + 1] = mk(bf2f(v.y & 0xffffu), bf2f(v.y >> 16));
            p[4 * k + 2] = mk(bf2f(v.z & 0xffffu), bf2f(v.z >> 16));
            p[4 * k + 3] = mk(bf2f(v.w & 0xffffu), bf2f(v.w >> 16));
        }
    }
    __device__ __forceinline__ static void unpack(uint32_t w, cx<T>& c) { c = mk(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u)); }
    template <bool BUF>
    __device__ __forceinline__ static void loadv(const RoView& b, long V, int n, int r, int s, cx<T> p[12]) {
        if constexpr (BUF) {
            const brsrc rs = make_rsrc(b.p, b.nbytes);
            const unsigned off = ((unsigned)s * (unsigned)n + (unsigned)r) * 16u;
            const unsigned ps = (unsigned)V * (unsigned)n * 16u;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                u4v v = bld16(rs, off, k * ps);
                unpack(v[0], p[4 * k + 0]);
                unpack(v[1], p[4 * k + 1]);
                unpack(v[2], p[4 * k + 2]);
                unpack(v[3], p[4 * k + 3]);
            }
        } else {
            load(b.p, V, n, r, s, p);
        }
    }
    // (re, im) -> two bf16 in one word, round to nearest even (one v_cvt_pk_bf16_f32)
    __device__ __forceinline__ static uint32_t pack(cx<T> c) {
        typedef float f2v __attribute__((ext_vector_type(2)));
        typedef __bf16 b2v __attribute__((ext_vector_type(2)));
        f2v f = {c.re, c.im};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, b2v));
    }
    template <bool NT = false>
    __device__ __forceinline__ static void store(void* b, long V, int n, int r, int s, const cx<T> p[12]) {
        const unsigned off = ((unsigned)s * (unsigned)n + (unsigned)r) * 16u;
        const size_t ps = (size_t)V * n * 16;
#pragma unroll
        for (int k = 0; k < 3; k++)
            st_at<NT>(b, k * ps, off, make_uint4(pack(p[4 * k]), pack(p[4 * k + 1]), pack(p[4 * k + 2]), pack(p[4 * k + 3])));
    }
    __device__ __forceinline__ static void load_link(const LinkT* U, long V, int mu, int s, cx<T> u[9]) {
        IO32::load_link(U, V, mu, s, u);
    }
    __device__ __forceinline__ static void load_clover(const CloverT* A, long V, int blk, int s, T f[36]) {
        IO32::load_clover(A, V, blk, s, f);
    }
};
