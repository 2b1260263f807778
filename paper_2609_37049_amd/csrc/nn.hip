// Gauge-covariant convolutional network used as the learned preconditioner of
// the Dirac solves (the solver's own addition; the paper only needs D^-1).
//
// A layer maps C_in spinor channels to C_out:
//   out_o(x) = sum_i sum_{d in {-1,0,1}^4} W[d][o][i] . T_d(x) psi_i(x + d)
// with W[d][o][i] a complex 4x4 spin matrix and T_d(x) the colour transporter
// along the axis-ordered path from x to x + d (x hops first, then y, z, t;
// boundary phase bc[mu] on a hop across the wrap).  The network is three
// layers 1 -> C -> C -> 1 without nonlinearity, hence linear and gauge
// covariant.  Offsets are numbered k = (dx+1) + 3(dy+1) + 9(dz+1) + 27(dt+1).
//
// GPU design (gfx950):
//  * transporters of all 81 offsets are tabulated once per gauge field as
//    BF16 pairs ([81][V][9] x {(Re, -Im), (Im, Re)}, 5.8 KB per site), so a
//    complex multiply-add on packed BF16 activations is two v_dot2_f32_bf16;
//  * activations are BF16 complex, [rhs][V][C][12] (site-major, so one
//    neighbour gather reads 48 contiguous bytes per channel);
//  * one layer is one kernel per tile of 64 sites (a 4x4x2x2 block): for each
//    offset (or batch of offsets when C_in = 1) the workgroup transports the
//    neighbour spinors with vector FMAs into an LDS tile of BF16 values, then
//    contracts it with the spin x channel weights written as a real 2x2 block
//    matrix on v_mfma_f32_16x16x32_bf16 (FP32 accumulation).  Weights are
//    pre-arranged in MFMA fragment order, so each lane loads 16 bytes per
//    fragment;
//  * the adjoint layer (backward pass for inputs) is the same kernel with the
//    gather reversed (x - d), the transporter T_d(x - d)^+ and weights W^H;
//  * weight gradients G = sum_x g_out phi^H are MFMA contractions over the
//    sites, split over chunks of tiles with fixed-order reduction.
#include <algorithm>
#include <cmath>
#include <random>

#include "spinor_io.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kOff = 81;
constexpr int kTile = 64;           // sites per tile: 4 x 4 x 2 x 2
constexpr int kCols = kTile * 3;    // MFMA columns per tile: (site, colour)
constexpr int kLdk = 136;           // bf16 per LDS column of the layer kernel (128 + pad)
constexpr int kLdw = kCols + 8;     // bf16 per LDS row of the weight-gradient kernel

__device__ __forceinline__ uint32_t pk2(float a, float b) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef __bf16 b2v __attribute__((ext_vector_type(2)));
    f2v f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, b2v));
}
__device__ __forceinline__ cx<float> unpk(uint32_t w) {
    return mk(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}

typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf2v, a), __builtin_bit_cast(bf2v, b), c, false);
}
// o[s*3+a] = sum_b M[a][b] psi[s*3+b] on packed BF16 (re low, im high), M = T or
// T^+ (ADJ); T[k] = {(Tr, -Ti), (Ti, Tr)} of entry k = row*3 + col.  Conjugating
// flips the sign of Ti: (Tr, Ti) and (-Ti, Tr) by one XOR of a sign bit each.
template <bool ADJ>
__device__ __forceinline__ void transport_bf(const uint2 (&T)[9], const uint32_t (&psi)[12], uint32_t (&o)[12]) {
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int b = 0; b < 3; b++) {
                const uint2 t = T[ADJ ? b * 3 + a : a * 3 + b];
                const uint32_t wa = ADJ ? (t.x ^ 0x80000000u) : t.x;
                const uint32_t wb = ADJ ? (t.y ^ 0x00008000u) : t.y;
                re = dot2(wa, psi[s * 3 + b], re);
                im = dot2(wb, psi[s * 3 + b], im);
            }
            o[s * 3 + a] = pk2(re, im);
        }
}

struct TileGeo {
    int L[4];    // lattice extents
    int T[4];    // tiles per dimension (L/4, L/4, L/2, L/2)
    int ntile;
    int bc[4];
};

__device__ __forceinline__ void tile_origin(const TileGeo& g, int tile, int o[4]) {
    o[0] = (tile % g.T[0]) * 4;
    tile /= g.T[0];
    o[1] = (tile % g.T[1]) * 4;
    tile /= g.T[1];
    o[2] = (tile % g.T[2]) * 2;
    o[3] = (tile / g.T[2]) * 2;
}
__device__ __forceinline__ void local_coords(int sl, const int o[4], int c[4]) {
    c[0] = o[0] + (sl & 3);
    c[1] = o[1] + ((sl >> 2) & 3);
    c[2] = o[2] + ((sl >> 4) & 1);
    c[3] = o[3] + (sl >> 5);
}
__device__ __forceinline__ int site_of(const TileGeo& g, const int c[4]) {
    return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}
__device__ __forceinline__ int shifted_site(const TileGeo& g, const int c[4], int d, int sgn) {
    const int dd[4] = {d % 3 - 1, (d / 3) % 3 - 1, (d / 9) % 3 - 1, d / 27 - 1};
    int y[4];
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        int v = c[mu] + sgn * dd[mu];
        v += v < 0 ? g.L[mu] : 0;
        v -= v >= g.L[mu] ? g.L[mu] : 0;
        y[mu] = v;
    }
    return site_of(g, y);
}

// ------------------------------------------------------------------ transporters
// T[d][x]: product of the links along the axis-ordered path from x to x + d,
// computed in FP64 from the links, stored as BF16 pairs (round to nearest even).
// One thread per (site, offset).
__global__ void k_nn_ttab(const double2* __restrict__ U, long V, TileGeo g, uint2* __restrict__ ttab) {
    const long tot = V * kOff;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const int d = (int)(j / V);
        const long s = j - (long)d * V;
        int c[4];
        long r = s;
        c[0] = (int)(r % g.L[0]);
        r /= g.L[0];
        c[1] = (int)(r % g.L[1]);
        r /= g.L[1];
        c[2] = (int)(r % g.L[2]);
        c[3] = (int)(r / g.L[2]);
        const int dd[4] = {d % 3 - 1, (d / 3) % 3 - 1, (d / 9) % 3 - 1, d / 27 - 1};
        cd M[9];
        for (int k = 0; k < 9; k++) M[k] = mk(k % 4 == 0 ? 1.0 : 0.0, 0.0);
        for (int mu = 0; mu < 4; mu++) {
            if (!dd[mu]) continue;
            cd L[9];
            double ph = 1.0;
            if (dd[mu] > 0) {
                const long ls = c[0] + (long)g.L[0] * (c[1] + (long)g.L[1] * (c[2] + (long)g.L[2] * c[3]));
                for (int k = 0; k < 9; k++) {
                    double2 u = U[((long)mu * 9 + k) * V + ls];
                    L[k] = mk(u.x, u.y);
                }
                if (c[mu] == g.L[mu] - 1) ph = g.bc[mu];
                c[mu] = c[mu] + 1 == g.L[mu] ? 0 : c[mu] + 1;
            } else {
                if (c[mu] == 0) ph = g.bc[mu];
                c[mu] = c[mu] == 0 ? g.L[mu] - 1 : c[mu] - 1;
                const long ls = c[0] + (long)g.L[0] * (c[1] + (long)g.L[1] * (c[2] + (long)g.L[2] * c[3]));
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) {
                        double2 u = U[((long)mu * 9 + b * 3 + a) * V + ls];
                        L[a * 3 + b] = mk(u.x, -u.y);
                    }
            }
            cd P[9];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) {
                    cd acc = mk(0.0, 0.0);
                    for (int k = 0; k < 3; k++) acc = acc + M[a * 3 + k] * L[k * 3 + b];
                    P[a * 3 + b] = ph * acc;
                }
            for (int k = 0; k < 9; k++) M[k] = P[k];
        }
        for (int k = 0; k < 9; k++) {
            const float tr = (float)M[k].re, ti = (float)M[k].im;
            ttab[((long)d * V + s) * 9 + k] = make_uint2(pk2(tr, -ti), pk2(ti, tr));
        }
    }
}

// ------------------------------------------------------------------ weight fragments
// Fragments of the real 2x2-block matrix of a layer (adj = 0) or of its adjoint
// (adj = 1), in the order the layer kernel reads them:
//   frag[batch][kstep 4][rowtile][lane 64][8]  (bf16, round to nearest even)
// Row = (o, s, re/im) of the output, K = (d_local, i, t, re/im) of the input.
// w holds the layer in forward orientation: [81][co][ci][4][4] complex.
__global__ void k_nn_frag(const float* __restrict__ w, int ci, int co, int adj, uint16_t* __restrict__ frag, long total) {
    const int CIe = adj ? co : ci, COe = adj ? ci : co;
    const int RT = COe * 8 / 16 > 1 ? COe * 8 / 16 : 1;
    const int NB = 128 / (CIe * 8);
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int j = (int)(idx & 7), lane = (int)((idx >> 3) & 63);
        long rest = idx >> 9;
        const int rt = (int)(rest % RT);
        rest /= RT;
        const int ks = (int)(rest & 3);
        const int batch = (int)(rest >> 2);
        const int row = rt * 16 + (lane & 15);
        const int kk = ks * 32 + 8 * (lane >> 4) + j;
        const int dl = kk / (CIe * 8), rem = kk % (CIe * 8);
        const int ie = rem >> 3, te = (rem & 7) >> 1, b = rem & 1;
        const int d = batch * NB + dl;
        const int oe = row >> 3, se = (row & 7) >> 1, a = row & 1;
        float val = 0.f;
        if (row < COe * 8 && d < kOff) {
            if (!adj) {
                const long e = ((((long)d * co + oe) * ci + ie) * 4 + se) * 4 + te;
                const float wr = w[2 * e], wi = w[2 * e + 1];
                val = a == 0 ? (b == 0 ? wr : -wi) : (b == 0 ? wi : wr);
            } else {
                // (W^H)[(i,t),(o,s)] = conj(W[(o,s),(i,t)]): rows (i = oe, t = se), K (o = ie, s = te)
                const long e = ((((long)d * co + ie) * ci + oe) * 4 + te) * 4 + se;
                const float wr = w[2 * e], wi = w[2 * e + 1];
                val = a == 0 ? (b == 0 ? wr : wi) : (b == 0 ? -wi : wr);
            }
        }
        frag[idx] = (uint16_t)f2bf_rne(val);
    }
}

static inline int nb_of(int ci) { return 128 / (ci * 8); }
static inline int nbatch_of(int ci) { return (kOff + nb_of(ci) - 1) / nb_of(ci); }
static inline int rt_of(int co) { return std::max(1, co * 8 / 16); }
static inline long frag_elems(int ci, int co) { return (long)nbatch_of(ci) * 4 * rt_of(co) * 64 * 8; }

// ------------------------------------------------------------------ layer kernel
struct LayerArgs {
    const uint32_t* in;   // [n][V][CI][12] bf16 (re, im) pairs
    void* out;            // [n][V][CO][12] bf16 pairs (uint32) or float2
    const uint2* ttab;    // [81][V][9] BF16 pairs
    const uint4* frag;
    long V;
    int nlogical;
    TileGeo g;
};

template <int CI, int CO, bool ADJ, bool OUT32>
__global__ __launch_bounds__(256) void k_nn_layer(const LayerArgs a) {
    constexpr int NB = 128 / (CI * 8);
    constexpr int NBATCH = (kOff + NB - 1) / NB;
    constexpr int RT = CO * 8 / 16 > 0 ? CO * 8 / 16 : 1;
    constexpr int NR = RT >= 4 ? RT / 4 : 1;   // row tiles per wave
    constexpr int NC = RT >= 4 ? 12 : 3;       // column tiles per wave
    __shared__ __attribute__((aligned(16))) uint16_t lds[kCols * kLdk];

    const int lb = xcd_block(a.nlogical);
    if (lb < 0) return;
    const int tile = lb % a.g.ntile, rhs = lb / a.g.ntile;
    int org[4];
    tile_origin(a.g, tile, org);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rt0 = RT >= 4 ? wv * NR : 0;
    const int ct0 = RT >= 4 ? 0 : wv * NC;
    // transport work of this thread: site sl, pairs (d_local, i) q*4 .. q*4+3
    const int sl = tid >> 2, q = tid & 3;
    int cs[4];
    local_coords(sl, org, cs);
    const int site = site_of(a.g, cs);
    const uint32_t* inr = a.in + (size_t)rhs * a.V * CI * 12;

    f32x4 acc[NR][NC];
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int c = 0; c < NC; c++) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};

    // CI = 16: the four channels of a thread share the offset; the next offset's
    // transporter and neighbour spinors are fetched while the matrix cores work
    uint2 Tn[CI == 16 ? 9 : 1];
    uint32_t rn[CI == 16 ? 4 : 1][12];
    auto fetch16 = [&](int d) {
        const int ys = shifted_site(a.g, cs, d, ADJ ? -1 : 1);
        const uint2* tp = a.ttab + ((size_t)d * a.V + (ADJ ? ys : site)) * 9;
#pragma unroll
        for (int k = 0; k < 9; k++) Tn[k] = tp[k];
#pragma unroll
        for (int pp = 0; pp < 4; pp++) {
            const uint4* ip = (const uint4*)(inr + ((size_t)ys * CI + q * 4 + pp) * 12);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const uint4 v = ip[k];
                rn[pp][4 * k] = v.x;
                rn[pp][4 * k + 1] = v.y;
                rn[pp][4 * k + 2] = v.z;
                rn[pp][4 * k + 3] = v.w;
            }
        }
    };
    if constexpr (CI == 16) fetch16(0);

    for (int batch = 0; batch < NBATCH; batch++) {
        if constexpr (CI == 16) {
#pragma unroll
            for (int pp = 0; pp < 4; pp++) {
                uint32_t o[12];
                transport_bf<ADJ>(Tn, rn[pp], o);
                const int kk = (q * 4 + pp) * 8;
#pragma unroll
                for (int c = 0; c < 3; c++)
                    *(uint4*)&lds[(sl * 3 + c) * kLdk + kk] = make_uint4(o[c], o[3 + c], o[6 + c], o[9 + c]);
            }
        } else {
#pragma unroll
            for (int pp = 0; pp < 4; pp++) {
                const int p = q * 4 + pp;
                const int dl = p / CI, i = p % CI;
                const int d = batch * NB + dl;
                uint32_t o[12];
                if (d < kOff) {
                    const int ys = shifted_site(a.g, cs, d, ADJ ? -1 : 1);
                    const uint2* tp = a.ttab + ((size_t)d * a.V + (ADJ ? ys : site)) * 9;
                    uint2 T[9];
#pragma unroll
                    for (int k = 0; k < 9; k++) T[k] = tp[k];
                    const uint4* ip = (const uint4*)(inr + ((size_t)ys * CI + i) * 12);
                    uint32_t raw[12];
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        const uint4 v = ip[k];
                        raw[4 * k] = v.x;
                        raw[4 * k + 1] = v.y;
                        raw[4 * k + 2] = v.z;
                        raw[4 * k + 3] = v.w;
                    }
                    transport_bf<ADJ>(T, raw, o);
                } else {
#pragma unroll
                    for (int k = 0; k < 12; k++) o[k] = 0u;
                }
                const int kk = (dl * CI + i) * 8;
#pragma unroll
                for (int c = 0; c < 3; c++)
                    *(uint4*)&lds[(sl * 3 + c) * kLdk + kk] = make_uint4(o[c], o[3 + c], o[6 + c], o[9 + c]);
            }
        }
        __syncthreads();
        if constexpr (CI == 16) {
            if (batch + 1 < NBATCH) fetch16(batch + 1);
        }
        const uint4* fb = a.frag + (size_t)batch * 4 * RT * 64;
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
            bf16x8 af[NR];
#pragma unroll
            for (int r = 0; r < NR; r++) af[r] = __builtin_bit_cast(bf16x8, fb[((size_t)ks * RT + rt0 + r) * 64 + lane]);
            const int kb = ks * 32 + 8 * (lane >> 4);
#pragma unroll
            for (int c = 0; c < NC; c++) {
                const int col = (ct0 + c) * 16 + (lane & 15);
                const bf16x8 bfr = __builtin_bit_cast(bf16x8, *(const uint4*)&lds[col * kLdk + kb]);
#pragma unroll
                for (int r = 0; r < NR; r++)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[r], bfr, acc[r][c], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // epilogue: lane holds rows 4*(lane/16)+e (e = 0..3) of each tile = (o, spins s0 and s0+1, re/im)
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int row0 = (rt0 + r) * 16 + 4 * (lane >> 4);
        if (row0 >= CO * 8) continue;
        const int o = row0 >> 3, s0 = (row0 & 7) >> 1;
#pragma unroll
        for (int c = 0; c < NC; c++) {
            const int col = (ct0 + c) * 16 + (lane & 15);
            const int sl2 = col / 3, cc = col - 3 * (col / 3);
            int c2[4];
            local_coords(sl2, org, c2);
            const size_t base = (((size_t)rhs * a.V + site_of(a.g, c2)) * CO + o) * 12;
            const f32x4 v = acc[r][c];
            if (OUT32) {
                float2* op = (float2*)a.out + base;
                op[s0 * 3 + cc] = make_float2(v[0], v[1]);
                op[(s0 + 1) * 3 + cc] = make_float2(v[2], v[3]);
            } else {
                uint32_t* op = (uint32_t*)a.out + base;
                op[s0 * 3 + cc] = pk2(v[0], v[1]);
                op[(s0 + 1) * 3 + cc] = pk2(v[2], v[3]);
            }
        }
    }
}

// ------------------------------------------------------------------ weights-first form
// For a layer with one output channel (the last layer), and for the adjoint of
// a layer with one input channel (the first layer's input gradient), contract
// first and transport afterwards, so that only one channel is transported per
// offset:
//   Y_d(z) = sum_i R_d[i] psi_i(z)             (matrix cores, all 81 offsets)
//   out(x) = sum_d M_d(x) Y_d(x + sgn d)       (one-channel colour transport)
// forward: R_d[i] = W[d][0][i], M_d(x) = T_d(x), sgn = +1;
// adjoint: R_d[o] = W[d][o][0]^+, M_d(x) = T_d(x - d)^+, sgn = -1.
constexpr int kWfRows = 81 * 8;                 // (d, s, re/im)
constexpr int kWfRowTiles = (kWfRows + 15) / 16;  // 41

// fragments [rowtile 41][kstep 4][lane 64][8] of the (81*8) x 128 real block matrix
__global__ void k_nn_wf_frag(const float* __restrict__ w, int ci, int co, int adj, uint16_t* __restrict__ frag) {
    const long total = (long)kWfRowTiles * 4 * 64 * 8;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int j = (int)(idx & 7), lane = (int)((idx >> 3) & 63);
        const int ks = (int)((idx >> 9) & 3);
        const int rt = (int)(idx >> 11);
        const int row = rt * 16 + (lane & 15);
        const int kk = ks * 32 + 8 * (lane >> 4) + j;
        const int d = row >> 3, se = (row & 7) >> 1, a = row & 1;
        const int ch = kk >> 3, te = (kk & 7) >> 1, b = kk & 1;
        float val = 0.f;
        if (d < kOff) {
            if (!adj) {  // W[d][0][ch][se][te], layer with co = 1
                const long e = ((((long)d * co + 0) * ci + ch) * 4 + se) * 4 + te;
                const float wr = w[2 * e], wi = w[2 * e + 1];
                val = a == 0 ? (b == 0 ? wr : -wi) : (b == 0 ? wi : wr);
            } else {     // conj(W[d][ch][0][te][se]), layer with ci = 1: rows (t = se), K (o = ch, s = te)
                const long e = ((((long)d * co + ch) * ci + 0) * 4 + te) * 4 + se;
                const float wr = w[2 * e], wi = w[2 * e + 1];
                val = a == 0 ? (b == 0 ? wr : wi) : (b == 0 ? -wi : wr);
            }
        }
        frag[idx] = (uint16_t)f2bf_rne(val);
    }
}

struct WfArgs {
    const uint32_t* in;   // [n][V][16][12]
    uint32_t* Y;          // [n][81][V][12] BF16 pairs
    const uint4* frag;
    long V;
    int nlogical;
    TileGeo g;
};

__global__ __launch_bounds__(256) void k_nn_wf_gemm(const WfArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t lds[kCols * kLdk];
    const int lb = xcd_block(a.nlogical);
    if (lb < 0) return;
    const int tile = lb % a.g.ntile, rhs = lb / a.g.ntile;
    int org[4];
    tile_origin(a.g, tile, org);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    {
        const int sl = tid >> 2, q = tid & 3;
        int cs[4];
        local_coords(sl, org, cs);
        const int site = site_of(a.g, cs);
#pragma unroll
        for (int pp = 0; pp < 4; pp++) {
            const int i = q * 4 + pp;
            const uint4* ip = (const uint4*)(a.in + (((size_t)rhs * a.V + site) * 16 + i) * 12);
            uint32_t w[12];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const uint4 v = ip[k];
                w[4 * k] = v.x;
                w[4 * k + 1] = v.y;
                w[4 * k + 2] = v.z;
                w[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int c = 0; c < 3; c++)
                *(uint4*)&lds[(sl * 3 + c) * kLdk + i * 8] = make_uint4(w[c], w[3 + c], w[6 + c], w[9 + c]);
        }
    }
    __syncthreads();
    uint32_t* Yr = a.Y + (size_t)rhs * kOff * a.V * 12;
    for (int pass = 0; pass * 8 < kWfRowTiles; pass++) {
        f32x4 acc[2][12];
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
            for (int c = 0; c < 12; c++) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int rt0 = pass * 8 + wv * 2;
#pragma unroll
        for (int ks = 0; ks < 4; ks++) {
            bf16x8 af[2];
#pragma unroll
            for (int r = 0; r < 2; r++) {
                const int rt = rt0 + r;
                af[r] = rt < kWfRowTiles ? __builtin_bit_cast(bf16x8, a.frag[((size_t)rt * 4 + ks) * 64 + lane])
                                         : __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
            }
            const int kb = ks * 32 + 8 * (lane >> 4);
#pragma unroll
            for (int c = 0; c < 12; c++) {
                const int col = c * 16 + (lane & 15);
                const bf16x8 bfr = __builtin_bit_cast(bf16x8, *(const uint4*)&lds[col * kLdk + kb]);
#pragma unroll
                for (int r = 0; r < 2; r++) acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[r], bfr, acc[r][c], 0, 0, 0);
            }
        }
#pragma unroll
        for (int r = 0; r < 2; r++) {
            const int row0 = (rt0 + r) * 16 + 4 * (lane >> 4);
            if (row0 >= kWfRows) continue;
            const int d = row0 >> 3, s0 = (row0 & 7) >> 1;
#pragma unroll
            for (int c = 0; c < 12; c++) {
                const int col = c * 16 + (lane & 15);
                const int sl2 = col / 3, cc = col - 3 * (col / 3);
                int c2[4];
                local_coords(sl2, org, c2);
                uint32_t* yp = Yr + ((size_t)d * a.V + site_of(a.g, c2)) * 12;
                const f32x4 v = acc[r][c];
                yp[s0 * 3 + cc] = pk2(v[0], v[1]);
                yp[(s0 + 1) * 3 + cc] = pk2(v[2], v[3]);
            }
        }
    }
}

// out(x) = sum_d M_d(x) Y_d(x + sgn d): one thread per (site, rhs), FP32 output [n][V][12]
template <bool ADJ>
__global__ __launch_bounds__(256) void k_nn_wf_gather(const uint32_t* __restrict__ Y, const uint2* __restrict__ ttab,
                                                      float2* __restrict__ out, long V, int n, TileGeo g) {
    const long tot = V * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const int rhs = (int)(j / V);
        const int x = (int)(j - (long)rhs * V);
        int c[4];
        {
            int r = x;
            c[0] = r % g.L[0];
            r /= g.L[0];
            c[1] = r % g.L[1];
            r /= g.L[1];
            c[2] = r % g.L[2];
            c[3] = r / g.L[2];
        }
        float re[12], im[12];
#pragma unroll
        for (int k = 0; k < 12; k++) re[k] = im[k] = 0.f;
        const uint32_t* Yr = Y + (size_t)rhs * kOff * V * 12;
        for (int d = 0; d < kOff; d++) {
            const int z = shifted_site(g, c, d, ADJ ? -1 : 1);
            const uint2* tp = ttab + ((size_t)d * V + (ADJ ? z : x)) * 9;
            uint2 T[9];
#pragma unroll
            for (int k = 0; k < 9; k++) T[k] = tp[k];
            const uint4* yp = (const uint4*)(Yr + ((size_t)d * V + z) * 12);
            uint32_t y[12];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const uint4 v = yp[k];
                y[4 * k] = v.x;
                y[4 * k + 1] = v.y;
                y[4 * k + 2] = v.z;
                y[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int sp = 0; sp < 4; sp++)
#pragma unroll
                for (int aa = 0; aa < 3; aa++)
#pragma unroll
                    for (int b = 0; b < 3; b++) {
                        const uint2 t = T[ADJ ? b * 3 + aa : aa * 3 + b];
                        const uint32_t wa = ADJ ? (t.x ^ 0x80000000u) : t.x;
                        const uint32_t wb = ADJ ? (t.y ^ 0x00008000u) : t.y;
                        re[sp * 3 + aa] = dot2(wa, y[sp * 3 + b], re[sp * 3 + aa]);
                        im[sp * 3 + aa] = dot2(wb, y[sp * 3 + b], im[sp * 3 + aa]);
                    }
        }
        float2* op = out + ((size_t)rhs * V + x) * 12;
#pragma unroll
        for (int k = 0; k < 12; k++) op[k] = make_float2(re[k], im[k]);
    }
}

// ------------------------------------------------------------------ weight gradients
struct DwArgs {
    const uint32_t* act;  // layer input [n][V][CI][12]
    const uint32_t* g;    // gradient at the layer output [n][V][CO][12]
    const uint2* ttab;
    float* part;          // [nbatch][nchunk][MOP][128]
    long V;
    int n, nchunk, nlogical;
    TileGeo g_;
};

// C[(o,s,a)][(d_local,i,t,b)] += sum over (site, colour) of g[(o,s,a)] phi[(d,i,t,b)],
// K ordered colour-major (k = colour*64 + site) so that a thread's four sites
// land in one 8-byte LDS store.
// GBACK (one output channel, sixteen inputs): the gradient is carried back
// along the path instead of the inputs forward, sum_x g(x) conj(T_d(x) phi(x+d))
// = sum_y (T_d(y-d)^+ g(y-d)) conj(phi(y)): one channel transported per site
// and offset instead of sixteen, and phi read in place.
template <int CI, int CO, bool GBACK = false>
__global__ __launch_bounds__(256) void k_nn_dw(const DwArgs a) {
    constexpr int NB = 128 / (CI * 8);
    constexpr int MOP = CO * 8 < 16 ? 16 : CO * 8;
    constexpr int RT = MOP / 16;
    constexpr int NR = RT >= 4 ? RT / 4 : 1;
    constexpr int NCt = RT >= 4 ? 8 : 2;
    __shared__ __attribute__((aligned(16))) uint16_t sA[MOP * kLdw];
    __shared__ __attribute__((aligned(16))) uint16_t sB[128 * kLdw];
    const int lb = xcd_block(a.nlogical);
    if (lb < 0) return;
    const int batch = lb / a.nchunk, chunk = lb % a.nchunk;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rt0 = RT >= 4 ? wv * NR : 0;
    const int ct0 = RT >= 4 ? 0 : wv * NCt;
    for (int k = tid; k < MOP * kLdw; k += 256) sA[k] = 0;

    f32x4 acc[NR][NCt];
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int c = 0; c < NCt; c++) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};

    static_assert(!GBACK || (CO == 1 && CI == 16), "the gradient goes back along the path for 16 -> 1 only");
    const int p = tid & 15, sg = tid >> 4;  // B fill: (d_local, i) pair and group of 4 sites
    const int dl = p / CI, ich = p % CI, d = batch * NB + dl;
    const long total = (long)a.g_.ntile * a.n;
    for (long gidx = chunk; gidx < total; gidx += a.nchunk) {
        const int rhs = (int)(gidx / a.g_.ntile), tile = (int)(gidx % a.g_.ntile);
        int org[4];
        tile_origin(a.g_, tile, org);
        __syncthreads();
        // B: transported inputs phi, rows (d_local, i, t, b), K (colour, site)
        {
            uint32_t ph[4][12];  // [site u][spin*3 + colour], packed BF16
#pragma unroll
            for (int u = 0; u < 4; u++) {
                int cs[4];
                local_coords(sg * 4 + u, org, cs);
                if (GBACK && d < kOff) {
                    // phi(y) at the tile's own sites, untransported
                    const uint4* ip = (const uint4*)(a.act + (((size_t)rhs * a.V + site_of(a.g_, cs)) * CI + ich) * 12);
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        const uint4 v = ip[k];
                        ph[u][4 * k] = v.x;
                        ph[u][4 * k + 1] = v.y;
                        ph[u][4 * k + 2] = v.z;
                        ph[u][4 * k + 3] = v.w;
                    }
                } else if (d < kOff) {
                    const int s0 = site_of(a.g_, cs);
                    const int ys = shifted_site(a.g_, cs, d, 1);
                    const uint2* tp = a.ttab + ((size_t)d * a.V + s0) * 9;
                    uint2 T[9];
#pragma unroll
                    for (int k = 0; k < 9; k++) T[k] = tp[k];
                    const uint4* ip = (const uint4*)(a.act + (((size_t)rhs * a.V + ys) * CI + ich) * 12);
                    uint32_t raw[12];
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        const uint4 v = ip[k];
                        raw[4 * k] = v.x;
                        raw[4 * k + 1] = v.y;
                        raw[4 * k + 2] = v.z;
                        raw[4 * k + 3] = v.w;
                    }
                    transport_bf<false>(T, raw, ph[u]);
                } else {
#pragma unroll
                    for (int k = 0; k < 12; k++) ph[u][k] = 0u;
                }
            }
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const int k = c * 64 + sg * 4;
                    const int e = s * 3 + c;
                    *(uint2*)&sB[(p * 8 + s * 2) * kLdw + k] =
                        make_uint2((ph[0][e] & 0xffffu) | (ph[1][e] << 16), (ph[2][e] & 0xffffu) | (ph[3][e] << 16));
                    *(uint2*)&sB[(p * 8 + s * 2 + 1) * kLdw + k] =
                        make_uint2((ph[0][e] >> 16) | (ph[1][e] & 0xffff0000u),
                                   (ph[2][e] >> 16) | (ph[3][e] & 0xffff0000u));
                }
        }
        // A: gradient rows (o, s, a), K (colour, site)
        if constexpr (GBACK) {
            // one (site, spin) per thread: T_d(y-d)^+ g(y-d), three colours
            const int sl = tid >> 2, sp = tid & 3;
            int cs[4];
            local_coords(sl, org, cs);
            uint32_t o3[3] = {0u, 0u, 0u};
            if (d < kOff) {
                const int z = shifted_site(a.g_, cs, d, -1);
                const uint2* tp = a.ttab + ((size_t)d * a.V + z) * 9;
                uint2 T[9];
#pragma unroll
                for (int k = 0; k < 9; k++) T[k] = tp[k];
                const uint32_t* gp = a.g + ((size_t)rhs * a.V + z) * 12 + sp * 3;
                const uint32_t g3[3] = {gp[0], gp[1], gp[2]};
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    // row c of T^+: entries T[b][c] conjugated (sign bit of Ti flipped)
                    float re = 0.f, im = 0.f;
#pragma unroll
                    for (int b = 0; b < 3; b++) {
                        const uint2 t = T[b * 3 + c];
                        re = dot2(t.x ^ 0x80000000u, g3[b], re);
                        im = dot2(t.y ^ 0x00008000u, g3[b], im);
                    }
                    o3[c] = pk2(re, im);
                }
            }
#pragma unroll
            for (int c = 0; c < 3; c++) {
                sA[(sp * 2) * kLdw + c * 64 + sl] = (uint16_t)(o3[c] & 0xffffu);
                sA[(sp * 2 + 1) * kLdw + c * 64 + sl] = (uint16_t)(o3[c] >> 16);
            }
        } else if (CO == 16 || tid < 16) {
            const int o = CO == 16 ? (tid & 15) : 0;
            const int sgA = CO == 16 ? (tid >> 4) : tid;
            uint32_t raw[4][12];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                int cs[4];
                local_coords(sgA * 4 + u, org, cs);
                const uint4* gp = (const uint4*)(a.g + (((size_t)rhs * a.V + site_of(a.g_, cs)) * CO + o) * 12);
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    uint4 v = gp[k];
                    raw[u][4 * k] = v.x;
                    raw[u][4 * k + 1] = v.y;
                    raw[u][4 * k + 2] = v.z;
                    raw[u][4 * k + 3] = v.w;
                }
            }
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const int k = c * 64 + sgA * 4;
                    const int e = s * 3 + c;
                    // low halves are re, high halves im
                    *(uint2*)&sA[(o * 8 + s * 2) * kLdw + k] =
                        make_uint2((raw[0][e] & 0xffffu) | (raw[1][e] << 16), (raw[2][e] & 0xffffu) | (raw[3][e] << 16));
                    *(uint2*)&sA[(o * 8 + s * 2 + 1) * kLdw + k] =
                        make_uint2((raw[0][e] >> 16) | (raw[1][e] & 0xffff0000u),
                                   (raw[2][e] >> 16) | (raw[3][e] & 0xffff0000u));
                }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kCols / 32; ks++) {
            const int kb = ks * 32 + 8 * (lane >> 4);
            bf16x8 af[NR];
#pragma unroll
            for (int r = 0; r < NR; r++)
                af[r] = __builtin_bit_cast(bf16x8, *(const uint4*)&sA[((rt0 + r) * 16 + (lane & 15)) * kLdw + kb]);
#pragma unroll
            for (int c = 0; c < NCt; c++) {
                const bf16x8 bfr =
                    __builtin_bit_cast(bf16x8, *(const uint4*)&sB[((ct0 + c) * 16 + (lane & 15)) * kLdw + kb]);
#pragma unroll
                for (int r = 0; r < NR; r++)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[r], bfr, acc[r][c], 0, 0, 0);
            }
        }
    }
    float* pp = a.part + ((size_t)batch * a.nchunk + chunk) * MOP * 128;
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int c = 0; c < NCt; c++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = (rt0 + r) * 16 + 4 * (lane >> 4) + e;
                const int col = (ct0 + c) * 16 + (lane & 15);
                pp[(size_t)row * 128 + col] = acc[r][c][e];
            }
}

// Fixed-order sum of the chunk partials and assembly of the complex gradient
// G[d][o][i][s][t] = (C_rr + C_ii) + i (C_ir - C_ri) into gw (forward layout).
__global__ void k_nn_dw_reduce(const float* __restrict__ part, int nchunk, int ci, int co, float* __restrict__ gw) {
    const int NB = 128 / (ci * 8);
    const int MOP = co * 8 < 16 ? 16 : co * 8;
    const long tot = (long)kOff * co * ci * 16;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        long r = e;
        const int t = (int)(r & 3);
        r >>= 2;
        const int s = (int)(r & 3);
        r >>= 2;
        const int i = (int)(r % ci);
        r /= ci;
        const int o = (int)(r % co);
        const int d = (int)(r / co);
        const int batch = d / NB, dl = d % NB;
        const int nre = (dl * ci + i) * 8 + t * 2, rre = o * 8 + s * 2;
        double crr = 0, cii = 0, cir = 0, cri = 0;
        for (int c = 0; c < nchunk; c++) {
            const float* P = part + ((size_t)batch * nchunk + c) * MOP * 128;
            crr += P[(size_t)rre * 128 + nre];
            cii += P[(size_t)(rre + 1) * 128 + nre + 1];
            cir += P[(size_t)(rre + 1) * 128 + nre];
            cri += P[(size_t)rre * 128 + nre + 1];
        }
        gw[2 * e] = (float)(crr + cii);
        gw[2 * e + 1] = (float)(cir - cri);
    }
}

// ------------------------------------------------------------------ conversions
// canonical complex128 [n][V][4][3] <-> activations [n][V][1][12] (same order)
__global__ void k_nn_c128_to_act(const double2* __restrict__ in, uint32_t* __restrict__ out, long tot) {
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        double2 v = in[j];
        out[j] = pk2((float)v.x, (float)v.y);
    }
}
__global__ void k_nn_act32_to_c128(const float2* __restrict__ in, double2* __restrict__ out, long tot) {
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        float2 v = in[j];
        out[j] = make_double2(v.x, v.y);
    }
}
// native FP32 block [6][V][n] float4 <-> activation layouts
__global__ void k_nn_native32_to_act(const void* __restrict__ in, uint32_t* __restrict__ out, long V, int n) {
    const long tot = V * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const long s = j / n;
        const int r = (int)(j - s * n);
        cx<float> p[12];
        IO32::load(in, V, n, r, (int)s, p);
        uint32_t* o = out + ((size_t)r * V + s) * 12;
#pragma unroll
        for (int k = 0; k < 12; k++) o[k] = pk2(p[k].re, p[k].im);
    }
}
__global__ void k_nn_act32_to_native32(const float2* __restrict__ in, void* __restrict__ out, long V, int n) {
    const long tot = V * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const long s = j / n;
        const int r = (int)(j - s * n);
        const float2* ip = in + ((size_t)r * V + s) * 12;
        cx<float> p[12];
#pragma unroll
        for (int k = 0; k < 12; k++) p[k] = mk(ip[k].x, ip[k].y);
        IO32::store(out, V, n, r, (int)s, p);
    }
}

// ------------------------------------------------------------------ training helpers
// per-pair partial sums of |out - e|^2: part[p][blk]
__global__ void k_nn_loss_part(const float2* __restrict__ out, const float2* __restrict__ e, long per, double* part,
                               int nblk) {
    const int p = blockIdx.y;
    double acc[1] = {0.0};
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < per; j += (long)nblk * blockDim.x) {
        const float2 a = out[(size_t)p * per + j], b = e[(size_t)p * per + j];
        const double dr = (double)a.x - b.x, di = (double)a.y - b.y;
        acc[0] += dr * dr + di * di;
    }
    block_sum(acc);
    if (threadIdx.x == 0) part[(size_t)p * nblk + blockIdx.x] = acc[0];
}
// g = scale * (out - e) as bf16 activation
__global__ void k_nn_loss_grad(const float2* __restrict__ out, const float2* __restrict__ e, float scale,
                               uint32_t* __restrict__ g, long tot) {
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const float2 a = out[j], b = e[j];
        g[j] = pk2(scale * (a.x - b.x), scale * (a.y - b.y));
    }
}
__global__ void k_nn_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
        const float gj = g[j];
        const float mj = b1 * m[j] + (1.f - b1) * gj;
        const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
        m[j] = mj;
        v[j] = vj;
        w[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
    }
}
// counter-based Gaussian sources (splitmix64 + Box-Muller) in native FP64 layout
__global__ void k_nn_gauss(double2* __restrict__ b, long n, unsigned long long seed) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        unsigned long long z = seed + 0x9e3779b97f4a7c15ULL * (unsigned long long)(i + 1);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z ^= z >> 31;
        const double u1 = ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        unsigned long long y = z + 0x9e3779b97f4a7c15ULL;
        y = (y ^ (y >> 30)) * 0xbf58476d1ce4e5b9ULL;
        y = (y ^ (y >> 27)) * 0x94d049bb133111ebULL;
        y ^= y >> 31;
        const double u2 = (double)(y >> 11) * (1.0 / 9007199254740992.0);
        const double rr = sqrt(-2.0 * log(u1));
        b[i] = make_double2(rr * cos(6.283185307179586 * u2), rr * sin(6.283185307179586 * u2));
    }
}
// per-rhs partial sums of |a|^2 of a native FP64 block (flat index i -> rhs i % n)
__global__ void k_nn_norm64(const double2* __restrict__ a, long tot, int n, double* part) {
    __shared__ double sh[256];
    double acc = 0;
    const int bd = (256 / n) * n;
    if (threadIdx.x < bd)
        for (long j = (long)blockIdx.x * bd + threadIdx.x; j < tot; j += (long)gridDim.x * bd) {
            double2 v = a[j];
            acc += v.x * v.x + v.y * v.y;
        }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < n) {
        double s = 0;
        for (int t = threadIdx.x; t < bd; t += n) s += sh[t];
        part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}
// pair slot p: r_act = bf16(f_r * r), e32 = f_e * e, from native FP64 blocks
__global__ void k_nn_store_pairs(const double2* __restrict__ r64, const double2* __restrict__ e64, long V, int n,
                                 const double* __restrict__ scale, uint32_t* __restrict__ ract, float2* __restrict__ e32) {
    const long tot = V * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const long s = j / n;
        const int r = (int)(j - s * n);
        cd pr[12], pe[12];
        IO64::load(r64, V, n, r, (int)s, pr);
        IO64::load(e64, V, n, r, (int)s, pe);
        const double f = scale[r];
        uint32_t* ro = ract + ((size_t)r * V + s) * 12;
        float2* eo = e32 + ((size_t)r * V + s) * 12;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            ro[k] = pk2((float)(f * pr[k].re), (float)(f * pr[k].im));
            eo[k] = make_float2((float)(f * pe[k].re), (float)(f * pe[k].im));
        }
    }
}
__global__ void k_nn_sub64(const double2* __restrict__ a, const double2* __restrict__ b, double2* __restrict__ c,
                           long tot) {
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x)
        c[j] = make_double2(a[j].x - b[j].x, a[j].y - b[j].y);
}

static int gridfor(long tot, int cap = 8192) { return (int)std::max(1L, std::min((tot + 255) / 256, (long)cap)); }

}  // namespace

// ------------------------------------------------------------------ network object
struct disco_net {
    disco_ctx* ctx = nullptr;
    int C = 16;
    size_t nw = 0;                 // floats of the packed weights
    size_t loff[3] = {0, 0, 0};    // float offset of each layer
    int lci[3] = {1, 16, 16}, lco[3] = {16, 16, 1};
    float* w = nullptr;            // device master weights
    float* gw = nullptr;           // device gradient
    float* am = nullptr;           // Adam moments
    float* av = nullptr;
    int adam_t = 0;
    uint2* ttab = nullptr;
    uint16_t* ffwd[3] = {nullptr, nullptr, nullptr};
    uint16_t* fadj[3] = {nullptr, nullptr, nullptr};
    uint16_t* fwf_out = nullptr;   // weights-first fragments: last layer (forward)
    uint16_t* fwf_in = nullptr;    // and the first layer's adjoint
    bool frags_ok = false;
    TileGeo geo;
    // activation workspaces (grow-only)
    std::map<std::string, std::pair<void*, size_t>> ws;
};

namespace {

void* net_ws(disco_net* net, const std::string& name, size_t bytes) {
    auto it = net->ws.find(name);
    if (it != net->ws.end() && it->second.second >= bytes) return it->second.first;
    if (it != net->ws.end()) {
        HIPCHK(hipStreamSynchronize(net->ctx->stream));
        HIPCHK(hipFree(it->second.first));
        net->ws.erase(it);
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) disco_throw(DISCO_ENOMEM, "network workspace %s (%zu bytes): %s", name.c_str(), bytes,
                                     hipGetErrorString(e));
    net->ws[name] = {p, bytes};
    return p;
}

void net_frags(disco_net* net) {
    if (net->frags_ok) return;
    hipStream_t st = net->ctx->stream;
    for (int l = 0; l < 3; l++) {
        const long nf = frag_elems(net->lci[l], net->lco[l]);
        const long na = frag_elems(net->lco[l], net->lci[l]);
        hipLaunchKernelGGL(k_nn_frag, dim3(gridfor(nf)), dim3(256), 0, st, net->w + net->loff[l], net->lci[l],
                           net->lco[l], 0, net->ffwd[l], nf);
        hipLaunchKernelGGL(k_nn_frag, dim3(gridfor(na)), dim3(256), 0, st, net->w + net->loff[l], net->lci[l],
                           net->lco[l], 1, net->fadj[l], na);
    }
    const long nwf = (long)kWfRowTiles * 4 * 64 * 8;
    hipLaunchKernelGGL(k_nn_wf_frag, dim3(gridfor(nwf)), dim3(256), 0, st, net->w + net->loff[2], net->lci[2],
                       net->lco[2], 0, net->fwf_out);
    hipLaunchKernelGGL(k_nn_wf_frag, dim3(gridfor(nwf)), dim3(256), 0, st, net->w + net->loff[0], net->lci[0],
                       net->lco[0], 1, net->fwf_in);
    HIPCHK(hipGetLastError());
    net->frags_ok = true;
}

// weights-first one-channel layer: forward last layer (ADJ false) or adjoint of
// the first layer (ADJ true); in [n][V][16][12] BF16, out FP32 [n][V][12]
template <bool ADJ>
void wf_launch(disco_net* net, int n, const uint32_t* in, float2* out) {
    disco_ctx* ctx = net->ctx;
    const long V = ctx->V;
    uint32_t* Y = (uint32_t*)net_ws(net, "wf_Y", sizeof(uint32_t) * (size_t)n * kOff * V * 12);
    WfArgs a;
    a.in = in;
    a.Y = Y;
    a.frag = (const uint4*)(ADJ ? net->fwf_in : net->fwf_out);
    a.V = V;
    a.g = net->geo;
    a.nlogical = net->geo.ntile * n;
    const int prof = prof_begin(ctx, 20);
    hipLaunchKernelGGL(k_nn_wf_gemm, dim3(xcd_grid(a.nlogical)), dim3(256), 0, ctx->stream, a);
    hipLaunchKernelGGL((k_nn_wf_gather<ADJ>), dim3(gridfor(V * n)), dim3(256), 0, ctx->stream, Y, net->ttab, out, V, n,
                       net->geo);
    if (prof >= 0) prof_end(ctx, prof, DISCO_KERNEL_NN, 2.0 * 8 * 128 * kOff * 3.0 * (double)V * n);
}

template <int CI, int CO, bool ADJ, bool OUT32>
void layer_launch(disco_net* net, int n, const uint32_t* in, void* out, const uint16_t* frag) {
    LayerArgs a;
    a.in = in;
    a.out = out;
    a.ttab = net->ttab;
    a.frag = (const uint4*)frag;
    a.V = net->ctx->V;
    a.g = net->geo;
    a.nlogical = net->geo.ntile * n;
    const int prof = prof_begin(net->ctx, 20);
    hipLaunchKernelGGL((k_nn_layer<CI, CO, ADJ, OUT32>), dim3(xcd_grid(a.nlogical)), dim3(256), 0, net->ctx->stream, a);
    if (prof >= 0) {
        // MFMA work of the launch: real 2x2-block GEMM over all offsets
        const double flops = 2.0 * (CO * 8) * (CI * 8) * kOff * 3.0 * (double)a.V * n;
        prof_end(net->ctx, prof, DISCO_KERNEL_NN, flops);
    }
}

// forward pass on n activations (layer-0 input act0): activations kept for backward
void net_forward(disco_net* net, int n, const uint32_t* act0, uint32_t* act1, uint32_t* act2, float2* out) {
    net_frags(net);
    layer_launch<1, 16, false, false>(net, n, act0, act1, net->ffwd[0]);
    layer_launch<16, 16, false, false>(net, n, act1, act2, net->ffwd[1]);
    wf_launch<false>(net, n, act2, out);
    HIPCHK(hipGetLastError());
}

template <int CI, int CO>
void dw_launch(disco_net* net, int n, const uint32_t* act, const uint32_t* g, float* gw) {
    DwArgs a;
    a.act = act;
    a.g = g;
    a.ttab = net->ttab;
    a.V = net->ctx->V;
    a.n = n;
    a.g_ = net->geo;
    const int nbatch = nbatch_of(CI);
    const long units = (long)net->geo.ntile * n;
    a.nchunk = (int)std::max(1L, std::min(units, (long)(2048 / nbatch)));
    a.nlogical = nbatch * a.nchunk;
    constexpr int MOP = CO * 8 < 16 ? 16 : CO * 8;
    a.part = (float*)net_ws(net, "dw_part", sizeof(float) * (size_t)nbatch * a.nchunk * MOP * 128);
    hipLaunchKernelGGL((k_nn_dw<CI, CO, CO == 1 && CI == 16>), dim3(xcd_grid(a.nlogical)), dim3(256), 0,
                       net->ctx->stream, a);
    hipLaunchKernelGGL(k_nn_dw_reduce, dim3(gridfor((long)kOff * CO * CI * 16)), dim3(256), 0, net->ctx->stream,
                       a.part, a.nchunk, CI, CO, gw);
}

// backward pass: g3 = dL/d(out) (bf16), activations of the forward pass;
// writes the weight gradient into net->gw and, if g0 is given, dL/d(input)
void net_backward(disco_net* net, int n, const uint32_t* act0, const uint32_t* act1, const uint32_t* act2,
                  const uint32_t* g3, float2* g0) {
    net_frags(net);
    const size_t per16 = (size_t)n * net->ctx->V * 16 * 12 * sizeof(uint32_t);
    uint32_t* g2 = (uint32_t*)net_ws(net, "bw_g2", per16);
    uint32_t* g1 = (uint32_t*)net_ws(net, "bw_g1", per16);
    dw_launch<16, 1>(net, n, act2, g3, net->gw + net->loff[2]);
    layer_launch<1, 16, true, false>(net, n, g3, g2, net->fadj[2]);
    dw_launch<16, 16>(net, n, act1, g2, net->gw + net->loff[1]);
    layer_launch<16, 16, true, false>(net, n, g2, g1, net->fadj[1]);
    dw_launch<1, 16>(net, n, act0, g1, net->gw + net->loff[0]);
    if (g0) wf_launch<true>(net, n, g1, g0);
    HIPCHK(hipGetLastError());
}

void net_build_ttab(disco_net* net) {
    disco_ctx* ctx = net->ctx;
    const long tot = ctx->V * kOff;
    hipLaunchKernelGGL(k_nn_ttab, dim3(gridfor(tot)), dim3(256), 0, ctx->stream, ctx->U64, ctx->V, net->geo, net->ttab);
    HIPCHK(hipGetLastError());
}

}  // namespace

namespace disco {
// z = N(v) on native FP32 blocks of n right-hand sides (used by FGMRES)
void net_apply_native32(disco_net* net, int n, const void* in32, void* out32) {
    disco_ctx* ctx = net->ctx;
    const long V = ctx->V;
    uint32_t* a0 = (uint32_t*)net_ws(net, "ap_a0", sizeof(uint32_t) * 12 * V * n);
    uint32_t* a1 = (uint32_t*)net_ws(net, "ap_a1", sizeof(uint32_t) * 12 * 16 * V * n);
    uint32_t* a2 = (uint32_t*)net_ws(net, "ap_a2", sizeof(uint32_t) * 12 * 16 * V * n);
    float2* o = (float2*)net_ws(net, "ap_out", sizeof(float2) * 12 * V * n);
    hipLaunchKernelGGL(k_nn_native32_to_act, dim3(gridfor(V * n)), dim3(256), 0, ctx->stream, in32, a0, V, n);
    net_forward(net, n, a0, a1, a2, o);
    hipLaunchKernelGGL(k_nn_act32_to_native32, dim3(gridfor(V * n)), dim3(256), 0, ctx->stream, o, out32, V, n);
    HIPCHK(hipGetLastError());
}
disco_ctx* net_ctx(const disco_net* net) { return net->ctx; }
}  // namespace disco

// ------------------------------------------------------------------ C ABI
extern "C" int disco_net_create(disco_ctx* ctx, int channels, unsigned long long seed, disco_net** out) {
    if (!ctx || !out) return DISCO_EINVAL;
    *out = nullptr;
    disco_net* net = new disco_net();
    int rc = guarded(ctx, [&] {
        REQUIRE(channels == 16, DISCO_EINVAL, "the network has 16 hidden channels (got %d)", channels);
        REQUIRE(ctx->have_gauge, DISCO_ESTATE, "net_create before gauge_set");
        REQUIRE(ctx->dims[0] % 4 == 0 && ctx->dims[1] % 4 == 0 && ctx->dims[2] % 2 == 0 && ctx->dims[3] % 2 == 0,
                DISCO_EINVAL, "network tiles need Lx, Ly divisible by 4 and Lz, Lt by 2");
        activate(ctx);
        net->ctx = ctx;
        net->C = channels;
        size_t off = 0;
        for (int l = 0; l < 3; l++) {
            net->loff[l] = off;
            off += (size_t)kOff * net->lci[l] * net->lco[l] * 16 * 2;
        }
        net->nw = off;
        for (int mu = 0; mu < 4; mu++) {
            net->geo.L[mu] = ctx->dims[mu];
            net->geo.bc[mu] = ctx->bc[mu];
        }
        net->geo.T[0] = ctx->dims[0] / 4;
        net->geo.T[1] = ctx->dims[1] / 4;
        net->geo.T[2] = ctx->dims[2] / 2;
        net->geo.T[3] = ctx->dims[3] / 2;
        net->geo.ntile = net->geo.T[0] * net->geo.T[1] * net->geo.T[2] * net->geo.T[3];
        HIPCHK(hipMalloc(&net->w, sizeof(float) * net->nw));
        HIPCHK(hipMalloc(&net->gw, sizeof(float) * net->nw));
        HIPCHK(hipMalloc(&net->am, sizeof(float) * net->nw));
        HIPCHK(hipMalloc(&net->av, sizeof(float) * net->nw));
        HIPCHK(hipMalloc(&net->ttab, sizeof(uint2) * 9 * (size_t)kOff * ctx->V));
        for (int l = 0; l < 3; l++) {
            HIPCHK(hipMalloc(&net->ffwd[l], sizeof(uint16_t) * frag_elems(net->lci[l], net->lco[l])));
            HIPCHK(hipMalloc(&net->fadj[l], sizeof(uint16_t) * frag_elems(net->lco[l], net->lci[l])));
        }
        HIPCHK(hipMalloc(&net->fwf_out, sizeof(uint16_t) * (size_t)kWfRowTiles * 4 * 64 * 8));
        HIPCHK(hipMalloc(&net->fwf_in, sizeof(uint16_t) * (size_t)kWfRowTiles * 4 * 64 * 8));
        // start: identity through channel 0 of every layer plus small Gaussian noise
        std::vector<float> h(net->nw);
        std::mt19937_64 rng(seed);
        std::uniform_real_distribution<double> uni(1e-12, 1.0);
        const double sig = 0.01;
        for (size_t k = 0; k < net->nw; k += 2) {
            const double r = std::sqrt(-2.0 * std::log(uni(rng))), th = 6.283185307179586 * uni(rng);
            h[k] = (float)(sig * r * std::cos(th));
            h[k + 1] = (float)(sig * r * std::sin(th));
        }
        for (int l = 0; l < 3; l++)
            for (int s = 0; s < 4; s++) {
                const size_t e = ((((size_t)40 * net->lco[l] + 0) * net->lci[l] + 0) * 4 + s) * 4 + s;
                h[net->loff[l] + 2 * e] += 1.0f;
            }
        HIPCHK(hipMemcpyAsync(net->w, h.data(), sizeof(float) * net->nw, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemsetAsync(net->am, 0, sizeof(float) * net->nw, ctx->stream));
        HIPCHK(hipMemsetAsync(net->av, 0, sizeof(float) * net->nw, ctx->stream));
        net_build_ttab(net);
        HIPCHK(hipStreamSynchronize(ctx->stream));
    });
    if (rc != DISCO_OK) {
        disco_net_destroy(net);
        return rc;
    }
    *out = net;
    return DISCO_OK;
}

extern "C" int disco_net_destroy(disco_net* net) {
    if (!net) return DISCO_OK;
    if (net->ctx) {
        (void)hipSetDevice(net->ctx->device);
        (void)hipStreamSynchronize(net->ctx->stream);
    }
    for (auto& kv : net->ws) (void)hipFree(kv.second.first);
    for (int l = 0; l < 3; l++) {
        if (net->ffwd[l]) (void)hipFree(net->ffwd[l]);
        if (net->fadj[l]) (void)hipFree(net->fadj[l]);
    }
    for (void* p : {(void*)net->w, (void*)net->gw, (void*)net->am, (void*)net->av, (void*)net->ttab,
                    (void*)net->fwf_out, (void*)net->fwf_in})
        if (p) (void)hipFree(p);
    delete net;
    return DISCO_OK;
}

extern "C" long long disco_net_weights_count(const disco_net* net) { return net ? (long long)net->nw : -1; }

extern "C" int disco_net_refresh(disco_net* net) {
    if (!net) return DISCO_EINVAL;
    return guarded(net->ctx, [&] {
        REQUIRE(net->ctx->have_gauge, DISCO_ESTATE, "no gauge field");
        activate(net->ctx);
        net_build_ttab(net);
        HIPCHK(hipStreamSynchronize(net->ctx->stream));
    });
}

extern "C" int disco_net_set_weights(disco_net* net, const float* w, int where) {
    if (!net || !w) return DISCO_EINVAL;
    return guarded(net->ctx, [&] {
        activate(net->ctx);
        HIPCHK(hipMemcpyAsync(net->w, w, sizeof(float) * net->nw,
                              where == DISCO_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, net->ctx->stream));
        HIPCHK(hipMemsetAsync(net->am, 0, sizeof(float) * net->nw, net->ctx->stream));
        HIPCHK(hipMemsetAsync(net->av, 0, sizeof(float) * net->nw, net->ctx->stream));
        net->adam_t = 0;
        net->frags_ok = false;
        HIPCHK(hipStreamSynchronize(net->ctx->stream));
    });
}

extern "C" int disco_net_get_weights(disco_net* net, float* w, int where) {
    if (!net || !w) return DISCO_EINVAL;
    return guarded(net->ctx, [&] {
        activate(net->ctx);
        HIPCHK(hipMemcpyAsync(w, net->w, sizeof(float) * net->nw,
                              where == DISCO_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, net->ctx->stream));
        HIPCHK(hipStreamSynchronize(net->ctx->stream));
    });
}

extern "C" int disco_net_apply(disco_net* net, int nrhs, const void* in, void* out) {
    if (!net) return DISCO_EINVAL;
    return guarded(net->ctx, [&] {
        REQUIRE(nrhs >= 0 && (nrhs == 0 || (in && out)), DISCO_EINVAL, "bad arguments");
        disco_ctx* ctx = net->ctx;
        activate(ctx);
        if (nrhs == 0) return;
        const long V = ctx->V;
        const int blk = 8;
        for (int r0 = 0; r0 < nrhs; r0 += blk) {
            const int n = std::min(blk, nrhs - r0);
            uint32_t* a0 = (uint32_t*)net_ws(net, "ap_a0", sizeof(uint32_t) * 12 * V * n);
            uint32_t* a1 = (uint32_t*)net_ws(net, "ap_a1", sizeof(uint32_t) * 12 * 16 * V * n);
            uint32_t* a2 = (uint32_t*)net_ws(net, "ap_a2", sizeof(uint32_t) * 12 * 16 * V * n);
            float2* o = (float2*)net_ws(net, "ap_out", sizeof(float2) * 12 * V * n);
            const long tot = 12 * V * n;
            hipLaunchKernelGGL(k_nn_c128_to_act, dim3(gridfor(tot)), dim3(256), 0, ctx->stream,
                               (const double2*)in + 12 * V * r0, a0, tot);
            net_forward(net, n, a0, a1, a2, o);
            hipLaunchKernelGGL(k_nn_act32_to_c128, dim3(gridfor(tot)), dim3(256), 0, ctx->stream, o,
                               (double2*)out + 12 * V * r0, tot);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(ctx->stream));
    });
}

extern "C" int disco_net_backward(disco_net* net, int nrhs, const void* in, const void* grad_out, float* grad_w,
                                  void* grad_in) {
    if (!net) return DISCO_EINVAL;
    return guarded(net->ctx, [&] {
        REQUIRE(nrhs > 0 && nrhs <= 64 && in && grad_out && grad_w, DISCO_EINVAL, "bad arguments");
        disco_ctx* ctx = net->ctx;
        activate(ctx);
        const long V = ctx->V;
        const int n = nrhs;
        const long tot = 12 * V * n;
        uint32_t* a0 = (uint32_t*)net_ws(net, "bw_a0", sizeof(uint32_t) * tot);
        uint32_t* a1 = (uint32_t*)net_ws(net, "bw_a1", sizeof(uint32_t) * 16 * tot);
        uint32_t* a2 = (uint32_t*)net_ws(net, "bw_a2", sizeof(uint32_t) * 16 * tot);
        float2* o = (float2*)net_ws(net, "bw_out", sizeof(float2) * tot);
        uint32_t* g3 = (uint32_t*)net_ws(net, "bw_g3", sizeof(uint32_t) * tot);
        float2* g0 = grad_in ? (float2*)net_ws(net, "bw_g0", sizeof(float2) * tot) : nullptr;
        hipLaunchKernelGGL(k_nn_c128_to_act, dim3(gridfor(tot)), dim3(256), 0, ctx->stream, (const double2*)in, a0, tot);
        hipLaunchKernelGGL(k_nn_c128_to_act, dim3(gridfor(tot)), dim3(256), 0, ctx->stream, (const double2*)grad_out,
                           g3, tot);
        net_forward(net, n, a0, a1, a2, o);
        net_backward(net, n, a0, a1, a2, g3, g0);
        HIPCHK(hipMemcpyAsync(grad_w, net->gw, sizeof(float) * net->nw, hipMemcpyDeviceToDevice, ctx->stream));
        if (grad_in)
            hipLaunchKernelGGL(k_nn_act32_to_c128, dim3(gridfor(tot)), dim3(256), 0, ctx->stream, g0,
                               (double2*)grad_in, tot);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(ctx->stream));
    });
}

extern "C" int disco_net_train(disco_net* net, const disco_train_params* tp, disco_train_stats* ts) {
    if (!net || !tp) return DISCO_EINVAL;
    return guarded(net->ctx, [&] {
        disco_ctx* ctx = net->ctx;
        REQUIRE(ctx->have_clover, DISCO_ESTATE, "net_train before clover_setup");
        REQUIRE(tp->npairs > 0 && tp->batch > 0 && tp->batch <= 16 && tp->npairs % tp->batch == 0, DISCO_EINVAL,
                "npairs must be a positive multiple of batch (batch <= 16)");
        REQUIRE(tp->nsnap > 0 && tp->nsnap <= 8 && tp->npairs % tp->nsnap == 0, DISCO_EINVAL,
                "npairs must be a multiple of nsnap (1..8)");
        REQUIRE(tp->steps >= 0 && tp->lr > 0, DISCO_EINVAL, "bad steps or learning rate");
        activate(ctx);
        const long V = ctx->V;
        const size_t per = 12 * (size_t)V;
        const int P = tp->npairs;
        uint32_t* R = (uint32_t*)net_ws(net, "tr_r", sizeof(uint32_t) * per * P);
        float2* E = (float2*)net_ws(net, "tr_e", sizeof(float2) * per * P);
        // ---- pairs generated by the solver: sources b, converged x*, truncated solves x_k,
        //      e = x* - x_k and r = D e (FP64), scaled to |e| = 1
        const int nsrc = P / tp->nsnap;
        const int gb = 8;
        disco_solver_params sp{};
        sp.method = DISCO_BICGSTAB_DC;
        sp.inner_prec = DISCO_F32;
        sp.fallback = 1;
        sp.check_every = 4;
        double gen_s = 0;
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, ctx->stream));
        long long pair = 0;
        for (int s0 = 0; s0 < nsrc; s0 += gb) {
            const int n = std::min(gb, nsrc - s0);
            const size_t nb64 = disco::native_bytes(ctx, DISCO_F64, n);
            double2* b = (double2*)ws_get(ctx, "tr_b", nb64);
            double2* xs = (double2*)ws_get(ctx, "tr_xs", nb64);
            double2* xk = (double2*)ws_get(ctx, "tr_xk", nb64);
            double2* e = (double2*)ws_get(ctx, "tr_ee", nb64);
            double2* r = (double2*)ws_get(ctx, "tr_rr", nb64);
            const long tot = 12 * V * n;
            hipLaunchKernelGGL(k_nn_gauss, dim3(gridfor(tot)), dim3(256), 0, ctx->stream, b, tot,
                               tp->seed * 0x100000001b3ULL + (unsigned long long)s0);
            std::vector<disco_solver_stats> st(n);
            sp.tol = 1e-9;
            sp.max_iter = 0;
            disco::solve_native(ctx, nullptr, sp, n, b, xs, st.data());
            for (int k = 0; k < tp->nsnap; k++) {
                const int it = tp->snap_iters[k];
                if (it <= 0) {
                    HIPCHK(hipMemsetAsync(xk, 0, nb64, ctx->stream));
                } else {
                    disco_solver_params q = sp;
                    q.max_iter = it;
                    q.fallback = 0;
                    q.tol = 1e-14;
                    disco::solve_native(ctx, nullptr, q, n, b, xk, st.data());
                }
                hipLaunchKernelGGL(k_nn_sub64, dim3(gridfor(tot)), dim3(256), 0, ctx->stream, xs, xk, e, tot);
                disco::StencilCall c{DISCO_F64, 0, n, e, r, nullptr, nullptr, nullptr, nullptr, disco::EPI_NONE};
                disco::stencil_launch(ctx, c);
                // per-rhs |e|
                const int nblk = 256;
                double* part = (double*)ws_get(ctx, "tr_part", sizeof(double) * nblk * n);
                hipLaunchKernelGGL(k_nn_norm64, dim3(nblk), dim3(256), 0, ctx->stream, e, tot, n, part);
                std::vector<double> hp((size_t)nblk * n), sc(n);
                HIPCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * nblk * n, hipMemcpyDeviceToHost, ctx->stream));
                HIPCHK(hipStreamSynchronize(ctx->stream));
                for (int j = 0; j < n; j++) {
                    double s = 0;
                    for (int q2 = 0; q2 < nblk; q2++) s += hp[(size_t)j * nblk + q2];
                    sc[j] = s > 0 ? 1.0 / std::sqrt(s) : 0.0;
                }
                double* dsc = (double*)ws_get(ctx, "tr_sc", sizeof(double) * n);
                HIPCHK(hipMemcpyAsync(dsc, sc.data(), sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
                // pairs of this snapshot are stored at slots k*nsrc + s0 + j
                const long slot = (long)k * nsrc + s0;
                hipLaunchKernelGGL(k_nn_store_pairs, dim3(gridfor(V * n)), dim3(256), 0, ctx->stream, r, e, V, n, dsc,
                                   R + slot * per, E + slot * per);
                pair += n;
            }
        }
        HIPCHK(hipEventRecord(e1, ctx->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        gen_s = ms / 1e3;
        // ---- training: Adam on mini-batches of consecutive pairs, batches visited in a
        //      seeded random order each epoch
        const int B = tp->batch;
        const int nbatches = P / B;
        uint32_t* a1 = (uint32_t*)net_ws(net, "tr_a1", sizeof(uint32_t) * per * 16 * B);
        uint32_t* a2 = (uint32_t*)net_ws(net, "tr_a2", sizeof(uint32_t) * per * 16 * B);
        float2* o = (float2*)net_ws(net, "tr_out", sizeof(float2) * per * B);
        uint32_t* g3 = (uint32_t*)net_ws(net, "tr_g3", sizeof(uint32_t) * per * B);
        const int nblk = 128;
        double* lpart = (double*)net_ws(net, "tr_lpart", sizeof(double) * nblk * B);
        std::vector<int> order(nbatches);
        for (int k = 0; k < nbatches; k++) order[k] = k;
        std::mt19937_64 rng(tp->seed ^ 0x5bd1e995ULL);
        std::vector<double> hp((size_t)nblk * B);
        double first = -1, last_sum = 0;
        int last_cnt = 0;
        HIPCHK(hipEventRecord(e0, ctx->stream));
        for (int step = 0; step < tp->steps; step++) {
            if (step % nbatches == 0) std::shuffle(order.begin(), order.end(), rng);
            const long b0 = (long)order[step % nbatches] * B;
            const uint32_t* a0 = R + b0 * per;
            const float2* eb = E + b0 * per;
            net_forward(net, B, a0, a1, a2, o);
            hipLaunchKernelGGL(k_nn_loss_part, dim3(nblk, B), dim3(256), 0, ctx->stream, o, eb, (long)per, lpart, nblk);
            HIPCHK(hipMemcpyAsync(hp.data(), lpart, sizeof(double) * nblk * B, hipMemcpyDeviceToHost, ctx->stream));
            // loss = (1/B) sum_p |N(r_p) - e_p|^2 with |e_p| = 1;  dL/d(out) = (2/B)(out - e)
            hipLaunchKernelGGL(k_nn_loss_grad, dim3(gridfor((long)per * B)), dim3(256), 0, ctx->stream, o, eb,
                               2.0f / B, g3, (long)per * B);
            net_backward(net, B, a0, a1, a2, g3, nullptr);
            net->adam_t++;
            const float b1 = 0.9f, b2 = 0.999f;
            const float c1 = 1.f - std::pow(b1, (float)net->adam_t), c2 = 1.f - std::pow(b2, (float)net->adam_t);
            hipLaunchKernelGGL(k_nn_adam, dim3(gridfor((long)net->nw)), dim3(256), 0, ctx->stream, net->w, net->gw,
                               net->am, net->av, (long)net->nw, (float)tp->lr, b1, b2, 1e-8f, c1, c2);
            net->frags_ok = false;
            HIPCHK(hipStreamSynchronize(ctx->stream));
            double l = 0;
            for (double v : hp) l += v;
            l /= B;
            if (first < 0) first = l;
            if (step >= tp->steps - std::max(1, std::min(nbatches, tp->steps / 4))) {
                last_sum += l;
                last_cnt++;
            }
        }
        HIPCHK(hipEventRecord(e1, ctx->stream));
        HIPCHK(hipEventSynchronize(e1));
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        net_frags(net);
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (ts) {
            ts->pairs = (int)pair;
            ts->steps = tp->steps;
            ts->first_loss = first;
            ts->final_loss = last_cnt ? last_sum / last_cnt : first;
            ts->gen_seconds = gen_s;
            ts->train_seconds = ms / 1e3;
        }
    });
}
