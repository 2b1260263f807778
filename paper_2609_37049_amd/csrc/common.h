// Internal definitions shared by the libdisco translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <functional>
#include <vector>

#include "../../include/disco.h"

// ----------------------------------------------------------------- complex
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cj(cx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cjmul(cx<T> a, cx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a
template <typename T>
__host__ __device__ __forceinline__ cx<T> ti(cx<T> a) { return {-a.im, a.re}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> neg(cx<T> a) { return {-a.re, -a.im}; }
template <typename T>
__host__ __device__ __forceinline__ T nrm(cx<T> a) { return a.re * a.re + a.im * a.im; }

typedef cx<double> cd;

// ----------------------------------------------------------------- storage tags
struct StoreF64 {};
struct StoreF32 {};
struct StoreBF16 {};

// ----------------------------------------------------------------- domains
struct disco_domains {
    disco_ctx* ctx;
    uint8_t* d_mask;               // per-site allowed-hop bits (bit 2*mu: forward, 2*mu+1: backward)
    std::vector<uint8_t> cut;      // [4][lmax]
    int lmax;
};

// ----------------------------------------------------------------- context
struct ProfRec {
    hipEvent_t a, b;
    double bytes;
    int kernel;
};

struct disco_ctx {
    int dims[4];
    int bc[4];
    long V, Vs;
    int device;
    hipStream_t stream = nullptr;
    std::string err;

    // gauge: [mu][9][V] complex
    double2* U64 = nullptr;
    float2* U32 = nullptr;
    bool have_gauge = false;
    // smeared spatial links for the Laplacian: [3][9][V] complex double
    double2* Usm = nullptr;
    bool have_smeared = false;
    // clover: FP64 [2][18][V] double2, FP32 [2][9][V] float4
    double2* A64 = nullptr;
    float4* A32 = nullptr;
    // A^-1 in the same packed format (even-odd preconditioning)
    double2* Ai64 = nullptr;
    float4* Ai32 = nullptr;
    bool have_clover = false;
    double kappa = 0, csw = 0;

    // stencil traversal: trav[g] = {site, x | y<<8 | z<<16 | t<<24} in the order the
    // stencil visits sites (each XCD takes one contiguous range of g)
    int2* d_trav = nullptr;
    int trav_kind = 0;
    // the same order restricted to the sites of one parity (x+y+z+t even / odd);
    // a site s of either parity has index s/2 in a half-lattice vector
    int2* d_trav_eo[2] = {nullptr, nullptr};
    // tile of the site order: y rows and timeslices (0 = the default rule), and
    // the tile the tables were last built with
    int tile_y = 0, tile_t = 0;
    int tile_used[2] = {0, 0};

    // named, grow-only device workspaces
    std::map<std::string, std::pair<void*, size_t>> ws;

    // options
    int opt_graphs = 1;   // capture inner Krylov iteration chunks as HIP graphs
    int opt_stage = -1;   // LDS staging of links/clover in the stencil: -1 auto, 0 off, 1 on
    int opt_eo = 1;       // even-odd (Schur) preconditioned inner solves when every extent is even
    int opt_narrow = 1;   // reliable updates: narrow the block for the queue's tail
    // graph cache: key -> executable graph; private capture stream
    std::map<std::string, hipGraphExec_t> graphs;
    hipStream_t cap_stream = nullptr;
    // autotuned right-hand-side block per inner precision (0 = not tuned)
    int tuned_block[3] = {0, 0, 0};

    // right-hand sides solved by the last distillation driver call (packed count)
    long long last_solves = 0;

    // profiling
    bool prof_on = false;
    int prof_stride = 1;
    std::map<int, long long> prof_seen;  // launches seen per family (for the stride)
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
};

// ----------------------------------------------------------------- errors
struct DiscoError {
    int code;
    std::string msg;
};

[[noreturn]] void disco_throw(int code, const char* fmt, ...);

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            disco_throw(DISCO_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                \
    } while (0)

#define REQUIRE(cond, code, ...)                         \
    do {                                                 \
        if (!(cond)) disco_throw((code), __VA_ARGS__);   \
    } while (0)

// Runs body, converting thrown errors into return codes and ctx->err.
template <typename F>
int guarded(disco_ctx* ctx, F&& body) {
    try {
        body();
        if (ctx) ctx->err.clear();
        return DISCO_OK;
    } catch (const DiscoError& e) {
        if (ctx) ctx->err = e.msg;
        return e.code;
    } catch (const std::exception& e) {
        if (ctx) ctx->err = e.what();
        return DISCO_EINVAL;
    }
}

// device workspace owned by the context (grow-only, reused across calls)
void* ws_get(disco_ctx* ctx, const std::string& name, size_t bytes);
// release a workspace (no-op when absent): set-up buffers and buffers a large
// solve no longer needs go back to the device allocator
void ws_free(disco_ctx* ctx, const std::string& name);
void activate(disco_ctx* ctx);

// launch helpers for profiling
int prof_begin(disco_ctx* ctx, int family);    // returns record index or -1 (not sampled)
void prof_end(disco_ctx* ctx, int rec, int kernel, double bytes);

// ----------------------------------------------------------------- launch geometry
// Workgroups are dispatched round-robin over the 8 XCDs.  Padding the grid to
// a multiple of 8 and remapping lets each XCD own one contiguous range of
// logical blocks (neighbouring sites share that XCD's L2).
static constexpr int kXCD = 8;
__device__ __forceinline__ int xcd_block(int nlogical) {
    int per = gridDim.x / kXCD;
    int b = blockIdx.x;
    int l = (b % kXCD) * per + b / kXCD;
    return l < nlogical ? l : -1;
}
static inline int xcd_grid(int nlogical) { return ((nlogical + kXCD - 1) / kXCD) * kXCD; }

// ----------------------------------------------------------------- reductions
// Deterministic block sum of N doubles per thread; thread 0 receives the totals.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
    __shared__ double sh[N > 0 ? N : 1][16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < N; k++) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; k++) sh[k][wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; k++) {
            double s = 0;
            for (int w = 0; w < nw; w++) s += sh[k][w];
            v[k] = s;
        }
    }
}

// Per-right-hand-side block partial sums.  Lane t of the block holds NQ
// complex values of right-hand side t % n (the block size is a multiple of
// n).  Every lane parks its values in LDS, then lane r < n adds the entries
// of its right-hand side in lane order (fixed order: bitwise reproducible)
// and writes part[(r*NQ + q)*nslot + slot].
static constexpr int kMaxBlock = 256;
template <int NQ>
__device__ __forceinline__ void rhs_partials(const double (&v)[2 * NQ], int n, int nact, double2* part, int nslot,
                                             int slot) {
    __shared__ double sh[2 * NQ][kMaxBlock];
#pragma unroll
    for (int k = 0; k < 2 * NQ; k++) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    const int r = threadIdx.x;
    if (r < n) {
        double acc[2 * NQ];
#pragma unroll
        for (int k = 0; k < 2 * NQ; k++) acc[k] = 0;
        for (int t = r; t < nact; t += n) {
#pragma unroll
            for (int k = 0; k < 2 * NQ; k++) acc[k] += sh[k][t];
        }
#pragma unroll
        for (int q = 0; q < NQ; q++) part[((long)r * NQ + q) * nslot + slot] = make_double2(acc[2 * q], acc[2 * q + 1]);
    }
}

// host-side declarations of internal entry points used across units
namespace disco {
// stencil on native blocks; epilogue flags below; part may be null when no reduction is asked
// reductions, in this order of their partial-sum slots: DOTAUX <aux2, out>,
// NORM ||out||^2, DOTIN <out, in>, DOTAUXIN <aux2, in> (in = the operand the
// site-local term acts on: the input, or aux in even-odd mode)
enum Epi { EPI_NONE = 0, EPI_RESID = 1, EPI_DOTAUX = 2, EPI_NORM = 4, EPI_DOTIN = 8, EPI_DOTAUXIN = 16 };
struct StencilCall {
    int prec;             // DISCO_F64/F32/BF16
    int dagger;
    int nrhs;
    const void* in;
    void* out;
    const void* aux;      // b for EPI_RESID
    const void* aux2;     // w for EPI_DOTAUX / EPI_DOTAUXIN
    const uint8_t* mask;  // null = full operator
    double2* part;        // partial sums [r][nq][nsb]
    int epi;
    // even-odd mode: parity of the sites written (0 even, 1 odd), -1 = full operator;
    // out = ca*aux + A^-1 (cg*aux + cb*H in), in and aux/aux2/out half-lattice vectors
    int eo_target = -1;
    double ca = 0, cg = 0, cb = 0;
};
int nq_of(int epi);
int stencil_nsb(disco_ctx* ctx, int n, bool eo = false);
// right-hand sides a stencil launch can address (32-bit offsets within a spinor plane)
int plane_rhs_limit(const disco_ctx* ctx);
// largest block of a batched solve: 64 and the plane limit
int max_rhs_block(const disco_ctx* ctx);
// A queue of right-hand sides that feeds the lanes of a native FP64 block of
// `width` lanes: load writes right-hand side j into lane `lane` of b64; store
// takes the solutions of finished lanes (with their right-hand sides' indices)
// from x64 before the lanes are reused.
struct LaneFeeder {
    int total = 0;
    std::function<void(int lane, int j, int width)> load;
    std::function<void(const std::vector<int>& lanes, const std::vector<int>& js, int width)> store;
};
long long solve_fed(disco_ctx* ctx, const disco_domains* dom, const disco_solver_params& P, int n, LaneFeeder& f,
                    double2* b64, double2* x64, disco_solver_stats* st);   // partial-sum slots per (rhs, quantity)
bool eo_supported(const disco_ctx* ctx);
int stencil_spb(int n);                    // sites per stencil block
void build_traversal(disco_ctx* ctx);
// resolve the device address of the no-allocation scratch array on `device`
// (the current device), once per device
void scratch_bind(int device);
void stencil_launch(disco_ctx* ctx, const StencilCall& c);
size_t native_bytes(const disco_ctx* ctx, int prec, int nrhs);
void to_native(disco_ctx* ctx, int prec, int nrhs, const void* in, void* out);
void from_native(disco_ctx* ctx, int prec, int nrhs, const void* in, void* out);
void solve_native(disco_ctx* ctx, const disco_domains* dom, const disco_solver_params& P, int n, const double2* b64,
                  double2* x64, disco_solver_stats* st);
// learned preconditioner: z = N(v) on native FP32 blocks of n right-hand sides
void net_apply_native32(disco_net* net, int n, const void* in32, void* out32);
disco_ctx* net_ctx(const disco_net* net);
}  // namespace disco
