// Krylov solvers for D x = b and D_Lambda x = b on batches of right-hand sides.
//
//   CGNR (all FP64): conjugate gradients on D^+ D x = D^+ b.  The plain
//     reference solver; its residual r = b - D x is the true residual.
//   BiCGStab-DC: BiCGStab in FP32 or BF16 storage (FP32 arithmetic) on the
//     normalised defect, inside an FP64 defect-correction loop that keeps x,
//     recomputes r = b - D x with the FP64 operator, and decides convergence
//     on that true residual.  Optional FP64 CGNR fallback.
//   FGMRES-NN: flexible GMRES(m) with an FP32 Krylov basis, right-
//     preconditioned by the trained network (z_j = N(v_j)), inside the same
//     FP64 defect correction and fallback.  Classical Gram-Schmidt with one
//     re-orthogonalisation on the device; the small Hessenberg least-squares
//     problem of each right-hand side (complex Givens rotations) on the host.
//
// Every Krylov scalar lives on the device: reductions produce deterministic
// per-block partial sums that one small kernel per right-hand side folds in a
// fixed order and turns into the next step's scalars, so an iteration never
// waits for the host.  The host reads the per-RHS state every few iterations
// to stop; right-hand sides that have converged are frozen by zero scalars.
//
// Vectors are native blocks ([plane][V][n], right-hand side fastest): the
// flat unit index i of a block belongs to right-hand side i % n.  Vector
// kernels use blocks whose size is a multiple of n, so every lane keeps one
// right-hand side across its grid-stride loop.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <functional>

#include "spinor_io.h"

namespace {

// Per right-hand-side solver state.  rr/bb belong to the outer (FP64, true
// residual) level; irr/ibb to the inner Krylov iteration.
struct RhsScal {
    cd rho, alpha, omega, beta;
    double rr, bb, irr, ibb, gam, scale;
    int active, breakdown, outer_done;
    int reached;  // reliable updates: the inner residual has fallen by inner_tol since the last update
    double best;  // smallest inner ||r||^2 since it last halved (reliable updates)
    int since;    // inner iterations since then
    int reject;   // reliable updates: 1 = the last correction left the true residual far above the one
                  // before (it is taken back), 2 = the lane then restarts with a perturbed shadow residual
};

// inner iterations without a halving of a lane's inner residual before it
// stops (its Krylov process then restarts)
constexpr int kRuStall = 100;
// iterations the FP64 CGNR fallback of the reliable-update solver may take
constexpr int kFallbackIters = 100000;
// the narrowest block the tail of a reliable-update queue moves into
constexpr int kNarrowMin = 16;
// reliable updates: a lane whose true ||r||^2 after the fold-in exceeds this
// multiple of its value at the previous update (4x in norm) gets the
// correction taken back, and its Krylov process restarts from the old iterate
constexpr double kRejectGrowth = 16.0;
// threads of a per-RHS scalar step (one block per right-hand side folds its
// partial sums; more threads keep more loads in flight)
constexpr int kScalarBlock = 1024;

// --------------------------------------------------------------- vector units
// One "unit" is the widest natural load of a storage format: 1 complex
// (FP64 double2), 2 complex (FP32 float4) or 4 complex (BF16 uint4).
template <class IO>
struct Unit;
template <>
struct Unit<IO64> {
    static constexpr int C = 1;
    __device__ __forceinline__ static void ld(const void* p, long i, cx<double> c[1]) {
        double2 v = ((const double2*)p)[i];
        c[0] = mk(v.x, v.y);
    }
    __device__ __forceinline__ static void st(void* p, long i, const cx<double> c[1]) {
        ((double2*)p)[i] = make_double2(c[0].re, c[0].im);
    }
    // the values as st then ld would return them
    __device__ __forceinline__ static void rnd(cx<double>*) {}
};
template <>
struct Unit<IO32> {
    static constexpr int C = 2;
    __device__ __forceinline__ static void ld(const void* p, long i, cx<float> c[2]) {
        float4 v = ((const float4*)p)[i];
        c[0] = mk(v.x, v.y);
        c[1] = mk(v.z, v.w);
    }
    __device__ __forceinline__ static void st(void* p, long i, const cx<float> c[2]) {
        ((float4*)p)[i] = make_float4(c[0].re, c[0].im, c[1].re, c[1].im);
    }
    __device__ __forceinline__ static void rnd(cx<float>*) {}
};
template <>
struct Unit<IOBF> {
    static constexpr int C = 4;
    __device__ __forceinline__ static void ld(const void* p, long i, cx<float> c[4]) {
        uint4 v = ((const uint4*)p)[i];
        c[0] = mk(bf2f(v.x & 0xffffu), bf2f(v.x >> 16));
        c[1] = mk(bf2f(v.y & 0xffffu), bf2f(v.y >> 16));
        c[2] = mk(bf2f(v.z & 0xffffu), bf2f(v.z >> 16));
        c[3] = mk(bf2f(v.w & 0xffffu), bf2f(v.w >> 16));
    }
    __device__ __forceinline__ static void st(void* p, long i, const cx<float> c[4]) {
        ((uint4*)p)[i] = make_uint4(IOBF::pack(c[0]), IOBF::pack(c[1]), IOBF::pack(c[2]), IOBF::pack(c[3]));
    }
    // streaming store, for vectors not read again before other traffic evicts them
    __device__ __forceinline__ static void stnt(void* p, long i, const cx<float> c[4]) {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        const u4 v = {IOBF::pack(c[0]), IOBF::pack(c[1]), IOBF::pack(c[2]), IOBF::pack(c[3])};
        __builtin_nontemporal_store(v, (u4*)p + i);
    }
    // round to BF16 (nearest even) in registers
    __device__ __forceinline__ static void rnd(cx<float> c[4]) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const uint32_t w = IOBF::pack(c[k]);
            c[k] = mk(bf2f(w & 0xffffu), bf2f(w >> 16));
        }
    }
};

template <typename T>
__device__ __forceinline__ cx<T> cast(cd a) {
    return mk((T)a.re, (T)a.im);
}

struct VecGeo {
    long total;  // units in the whole block (all right-hand sides)
    int n;       // right-hand sides
    int bd;      // threads per block (multiple of n)
    int nb;      // blocks (= partial-sum slots per rhs and quantity)
};

#define VEC_LOOP(g) for (long i = (long)blockIdx.x * (g).bd + threadIdx.x; i < (g).total; i += (long)(g).nb * (g).bd)

// partial ||v||^2 per right-hand side
template <class IO>
__global__ void k_norm2(const void* v, VecGeo g, double2* part) {
    typedef Unit<IO> U;
    typedef typename IO::T T;
    double acc[2] = {0, 0};
    VEC_LOOP(g) {
        cx<T> a[U::C];
        U::ld(v, i, a);
#pragma unroll
        for (int c = 0; c < U::C; c++) acc[0] += (double)nrm(a[c]);
    }
    rhs_partials<1>(acc, g.n, g.bd, part, g.nb, blockIdx.x);
}

// dst (IOD) = scale[r] * src (IOS), site by site through the layout accessors
// (the native layouts of different precisions order components differently)
template <class IOS, class IOD>
__global__ void k_copy_scale(const void* src, void* dst, long V, int n, const RhsScal* sc, int use_scale) {
    const long tot = V * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const long s = j / n, r = j - s * n;
        const double f = use_scale ? sc[r].scale : 1.0;
        cx<typename IOS::T> a[12];
        cx<typename IOD::T> b[12];
        IOS::load(src, V, n, r, s, a);
#pragma unroll
        for (int k = 0; k < 12; k++)
            b[k] = mk((typename IOD::T)(f * (double)a[k].re), (typename IOD::T)(f * (double)a[k].im));
        IOD::store(dst, V, n, r, s, b);
    }
}

// x64 += (1/scale[r]) * e (inner precision) for right-hand sides that ran
// (not for finished ones, nor for inner solves that diverged).  UNDO: x64 -=
// the same, for the lanes whose correction is rejected.
template <class IO, bool UNDO = false>
__global__ void k_dc_update(double2* x64, const void* e, long V, int n, const RhsScal* sc) {
    const long tot = V * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const long s = j / n, r = j - s * n;
        if (UNDO ? sc[r].reject != 1 : (sc[r].outer_done || sc[r].breakdown == 2)) continue;
        const double f = (sc[r].scale > 0 ? 1.0 / sc[r].scale : 0.0) * (UNDO ? -1.0 : 1.0);
        cx<typename IO::T> a[12];
        cx<double> x[12];
        IO::load(e, V, n, r, s, a);
        IO64::load(x64, V, n, r, s, x);
#pragma unroll
        for (int k = 0; k < 12; k++) x[k] = mk(x[k].re + f * (double)a[k].re, x[k].im + f * (double)a[k].im);
        IO64::store(x64, V, n, r, s, x);
    }
}

template <class IO>
__global__ void k_zero(void* v, long nunits_total) {
    typedef typename IO::T T;
    cx<T> z[Unit<IO>::C];
#pragma unroll
    for (int c = 0; c < Unit<IO>::C; c++) z[c] = mk((T)0, (T)0);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nunits_total; i += (long)gridDim.x * blockDim.x)
        Unit<IO>::st(v, i, z);
}

// ---- BiCGStab vector steps
// s = r - alpha v
template <class IO>
__global__ void k_bicg_s(const void* r_, const void* v_, void* s_, VecGeo g, const RhsScal* sc) {
    typedef Unit<IO> U;
    typedef typename IO::T T;
    const cx<T> al = cast<T>(sc[threadIdx.x % g.n].alpha);
    VEC_LOOP(g) {
        cx<T> a[U::C], b[U::C], o[U::C];
        U::ld(r_, i, a);
        U::ld(v_, i, b);
#pragma unroll
        for (int c = 0; c < U::C; c++) o[c] = a[c] - al * b[c];
        U::st(s_, i, o);
    }
}

// Fused end of a BiCGStab iteration, once omega and beta are known:
//   x += alpha p + omega s ; r = s - omega t ; p = r + beta (p - omega v) ;
//   partial ||r||^2 of the stored (rounded) residual.
// In BF16, x and r are written with streaming stores: the next reads of x
// (this kernel, next iteration) and r (the s step, after two stencil launches)
// come after other traffic has evicted them, while p is read at once.
template <class IO>
__global__ void k_bicg_xrp(void* x_, void* p_, const void* s_, const void* t_, const void* v_, void* r_, VecGeo g,
                           const RhsScal* sc, double2* part) {
    typedef Unit<IO> U;
    typedef typename IO::T T;
    const int rr = threadIdx.x % g.n;
    const cx<T> al = cast<T>(sc[rr].alpha), om = cast<T>(sc[rr].omega), be = cast<T>(sc[rr].beta);
    double acc[2] = {0, 0};
    VEC_LOOP(g) {
        cx<T> x[U::C], p[U::C], s[U::C], t[U::C], v[U::C], rn[U::C];
        U::ld(x_, i, x);
        U::ld(p_, i, p);
        U::ld(s_, i, s);
        U::ld(t_, i, t);
        U::ld(v_, i, v);
#pragma unroll
        for (int c = 0; c < U::C; c++) {
            x[c] = x[c] + al * p[c] + om * s[c];
            rn[c] = s[c] - om * t[c];
        }
        if constexpr (IO::planes == 3) U::stnt(x_, i, x); else U::st(x_, i, x);
        U::rnd(rn);  // the stored (rounded) residual feeds p and the norm
        if constexpr (IO::planes == 3) U::stnt(r_, i, rn); else U::st(r_, i, rn);
#pragma unroll
        for (int c = 0; c < U::C; c++) {
            p[c] = rn[c] + be * (p[c] - om * v[c]);
            acc[0] += (double)nrm(rn[c]);
        }
        U::st(p_, i, p);
    }
    rhs_partials<1>(acc, g.n, g.bd, part, g.nb, blockIdx.x);
}

// uniform in [-1, 1) from a 32-bit integer hash of (k, salt) (the "lowbias32"
// mixing function: xor-shifts and two odd multipliers)
__device__ __forceinline__ double unit_hash(unsigned k, unsigned salt) {
    unsigned x = k ^ (salt * 0x9e3779b9u);
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return (double)(x >> 8) * (1.0 / 8388608.0) - 1.0;
}

// Reliable update of the inner BiCGStab (continued, not restarted): the
// recursive residual r is replaced by rn, the residual of the inner system
// recomputed from the FP64 true residual; p, built from the old r, takes the
// same change (p += rn - r); the inner correction e restarts at 0.  Lanes
// that broke down or stalled (and finished lanes) restart the Krylov process
// instead: p = rhat = rn.  Partials <rhat, rn>, ||rn||^2.
template <class IO>
__global__ void k_ru_refresh(void* r_, const void* rn_, void* p_, void* rh_, void* e_, VecGeo g, const RhsScal* sc,
                             double2* part, unsigned salt) {
    typedef Unit<IO> U;
    typedef typename IO::T T;
    const int rr = threadIdx.x % g.n;
    const bool restart = sc[rr].breakdown || sc[rr].outer_done;
    // a lane whose last correction was taken back: r^ = r (1 + xi / 2) component
    // by component, xi uniform in [-1, 1) from a hash of (unit, component,
    // update), so that <r^, r> stays a positive multiple of ||r||^2
    const bool perturb = restart && sc[rr].reject == 2;
    double acc[4] = {0, 0, 0, 0};
    cx<T> z[U::C];
#pragma unroll
    for (int c = 0; c < U::C; c++) z[c] = mk((T)0, (T)0);
    VEC_LOOP(g) {
        cx<T> rn[U::C], r[U::C], p[U::C], rh[U::C];
        U::ld(rn_, i, rn);
        if (restart) {
#pragma unroll
            for (int c = 0; c < U::C; c++) {
                p[c] = rn[c];
                rh[c] = rn[c];
                if (perturb) {
                    const T f = (T)(1.0 + 0.5 * unit_hash((unsigned)i * (unsigned)U::C + (unsigned)c, salt));
                    rh[c] = mk(f * rn[c].re, f * rn[c].im);
                }
            }
            U::st(rh_, i, rh);
        } else {
            U::ld(r_, i, r);
            U::ld(p_, i, p);
            U::ld(rh_, i, rh);
#pragma unroll
            for (int c = 0; c < U::C; c++) p[c] = p[c] + (rn[c] - r[c]);
        }
        U::st(r_, i, rn);
        U::st(p_, i, p);
        U::st(e_, i, z);
#pragma unroll
        for (int c = 0; c < U::C; c++) {
            cx<T> d = cjmul(rh[c], rn[c]);
            acc[0] += (double)d.re;
            acc[1] += (double)d.im;
            acc[2] += (double)nrm(rn[c]);
        }
    }
    rhs_partials<2>(acc, g.n, g.bd, part, g.nb, blockIdx.x);
}

// ---- CGNR vector steps (FP64)
// x += alpha p ; r -= alpha w ; partial ||r||^2
__global__ void k_cgnr_xr(double2* x, const double2* p, const double2* w, double2* rv, VecGeo g, const RhsScal* sc,
                          double2* part) {
    const double al = sc[threadIdx.x % g.n].alpha.re;
    double acc[2] = {0, 0};
    VEC_LOOP(g) {
        double2 xv = x[i], pv = p[i], wv = w[i], r = rv[i];
        xv.x += al * pv.x;
        xv.y += al * pv.y;
        r.x -= al * wv.x;
        r.y -= al * wv.y;
        x[i] = xv;
        rv[i] = r;
        acc[0] += r.x * r.x + r.y * r.y;
    }
    rhs_partials<1>(acc, g.n, g.bd, part, g.nb, blockIdx.x);
}

// p = z + beta p
__global__ void k_cgnr_p(double2* p, const double2* z, VecGeo g, const RhsScal* sc) {
    const double be = sc[threadIdx.x % g.n].beta.re;
    VEC_LOOP(g) {
        double2 pv = p[i], zv = z[i];
        p[i] = make_double2(zv.x + be * pv.x, zv.y + be * pv.y);
    }
}

// --------------------------------------------------------------- scalar steps
// Each block folds the partial sums of one right-hand side in a fixed order.
// Each thread issues the loads of U slots before adding them (in slot order,
// so the sums are the same as one slot at a time): the fold is bound by load
// latency, and one block per right-hand side has few waves to hide it.
template <int NQ>
__device__ __forceinline__ void fold(const double2* part, long r, int nparts, cd out[NQ]) {
    constexpr int U = NQ >= 4 ? 4 : 8;
    double acc[2 * NQ];
#pragma unroll
    for (int k = 0; k < 2 * NQ; k++) acc[k] = 0;
    const int bd = blockDim.x;
    int i = threadIdx.x;
    for (; i + (U - 1) * bd < nparts; i += U * bd) {
        double2 v[U][NQ];
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int q = 0; q < NQ; q++) v[u][q] = part[(r * NQ + q) * nparts + i + u * bd];
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                acc[2 * q] += v[u][q].x;
                acc[2 * q + 1] += v[u][q].y;
            }
    }
    for (; i < nparts; i += bd) {
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            double2 v = part[(r * NQ + q) * nparts + i];
            acc[2 * q] += v.x;
            acc[2 * q + 1] += v.y;
        }
    }
    block_sum(acc);
#pragma unroll
    for (int q = 0; q < NQ; q++) out[q] = mk(acc[2 * q], acc[2 * q + 1]);
}

__device__ __forceinline__ cd cdiv(cd a, cd b) {
    double d = b.re * b.re + b.im * b.im;
    return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}

// mode 0: bb = rr = ||b||^2 (outer start); mode 1: rr = ||r||^2.  Then decide
// outer convergence and set scale = 1/||r|| for the next defect.
// mode 2 (reliable updates): rr = ||r||^2 with the scale of the start kept;
// a lane whose inner residual reached its reduction while the true residual
// fell by less than a factor 2 (in the squared norm) is marked for a Krylov
// restart; gam keeps the previous update's ||r||^2.
__global__ void k_sc_outer(const double2* part, int nparts, RhsScal* sc, int mode, double tol2) {
    cd q[1];
    fold<1>(part, blockIdx.x, nparts, q);
    if (threadIdx.x) return;
    RhsScal& s = sc[blockIdx.x];
    if (mode == 0) {
        s.bb = q[0].re;
        s.rr = q[0].re;
        s.gam = q[0].re;
        s.outer_done = 0;
        s.reject = 0;
    } else {
        s.rr = q[0].re;
    }
    if (mode == 2 && !s.outer_done && s.gam > 0 && !(s.rr <= kRejectGrowth * s.gam)) {
        // the correction made things worse (or is not a number): it is taken
        // back and the true residual recomputed before the rest (mode 3)
        s.reject = 1;
        return;
    }
    if (mode == 3 && s.reject == 1) {
        // the restored iterate: its Krylov process restarts, with another
        // shadow residual (from the same state, r^ = r would retrace the same
        // iterations)
        s.reject = 2;
        s.breakdown = 1;
        s.gam = s.rr;
        if (s.rr <= tol2 * s.bb) s.outer_done = 1;
        if (s.outer_done) s.scale = 0.0;
        return;
    }
    if (mode == 3) return;
    if (mode == 4) {
        // a lane carried into a narrower block: the residual of its current
        // iterate starts the new process and sets the inner scale
        s.gam = s.rr;
        s.reject = 0;
        if (s.rr <= tol2 * s.bb) s.outer_done = 1;
        s.scale = (s.rr > 0 && !s.outer_done) ? 1.0 / sqrt(s.rr) : 0.0;
        return;
    }
    if (mode == 2) {
        if (!s.outer_done && (s.reached || !s.active) && !s.breakdown && s.rr > 0.5 * s.gam) s.breakdown = 1;
        s.gam = s.rr;
        if (s.rr <= tol2 * s.bb) s.outer_done = 1;
        if (s.outer_done) s.scale = 0.0;
        return;
    }
    if (s.rr <= tol2 * s.bb) s.outer_done = 1;
    s.scale = (s.rr > 0 && !s.outer_done) ? 1.0 / sqrt(s.rr) : 0.0;
}

// Lanes that take new right-hand sides (lanes[0..m)): x = 0 and r = b there.
__global__ void k_lane_restart(double2* __restrict__ x64, double2* __restrict__ r64, const double2* __restrict__ b64,
                               long V, int n, const int* __restrict__ lanes, int m) {
    const long tot = 12 * V * m;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
        const long row = i / m;
        const long j = row * n + lanes[i - row * m];
        x64[j] = make_double2(0.0, 0.0);
        r64[j] = b64[j];
    }
}

// dst (width n2) lane q = src (width n) lane lanes[q] for q < m, 0 for the
// other lanes: the open lanes of a block moved into a narrower one
__global__ void k_lanes_compact(const double2* __restrict__ src, double2* __restrict__ dst, long V, int n, int n2,
                                const int* __restrict__ lanes, int m) {
    const long tot = 12 * V * n2;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
        const long row = i / n2;
        const int q = (int)(i - row * n2);
        dst[i] = q < m ? src[row * n + lanes[q]] : make_double2(0.0, 0.0);
    }
}

// b = 0 in lanes[0..m) (idle lanes of a block whose queue has run dry)
__global__ void k_lane_clear(double2* __restrict__ b64, long V, int n, const int* __restrict__ lanes, int m) {
    const long tot = 12 * V * m;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
        const long row = i / m;
        b64[row * n + lanes[i - row * m]] = make_double2(0.0, 0.0);
    }
}

// partial ||b||^2 -> the outer state of the flagged lanes, as at the start of a
// solve; their Krylov process restarts at the next refresh (marked broken down)
__global__ void k_sc_lane_start(const double2* part, int nparts, RhsScal* sc, const int* flag, double tol2) {
    cd q[1];
    fold<1>(part, blockIdx.x, nparts, q);
    if (threadIdx.x || !flag[blockIdx.x]) return;
    RhsScal& s = sc[blockIdx.x];
    s.bb = q[0].re;
    s.rr = q[0].re;
    s.gam = q[0].re;
    s.outer_done = s.rr <= tol2 * s.bb ? 1 : 0;
    s.scale = (s.rr > 0 && !s.outer_done) ? 1.0 / sqrt(s.rr) : 0.0;
    s.breakdown = 1;
    s.reached = 0;
    s.active = 0;
    s.reject = 0;
}

// one right-hand side in the canonical layout [V][12] <-> lane r of a native FP64 block
__global__ void k_lane_in(const double2* __restrict__ src, double2* __restrict__ b64, long V, int n, int r) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < 12 * V; i += (long)gridDim.x * blockDim.x) {
        const long s = i / 12;
        const int k = (int)(i - s * 12);
        b64[((long)k * V + s) * n + r] = src[i];
    }
}
__global__ void k_lane_out(const double2* __restrict__ x64, double2* __restrict__ dst, long V, int n, int r) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < 12 * V; i += (long)gridDim.x * blockDim.x) {
        const long s = i / 12;
        const int k = (int)(i - s * 12);
        dst[i] = x64[((long)k * V + s) * n + r];
    }
}

// after a reliable update: rho = <rhat, r>, the reference ||r||^2 for the next
// update, and every unfinished lane active again
__global__ void k_sc_ru_refresh(const double2* part, int nparts, RhsScal* sc) {
    cd q[2];
    fold<2>(part, blockIdx.x, nparts, q);
    if (threadIdx.x) return;
    RhsScal& s = sc[blockIdx.x];
    s.rho = q[0];
    s.irr = q[1].re;
    s.ibb = q[1].re;
    s.best = q[1].re;
    s.since = 0;
    s.breakdown = 0;
    s.reached = 0;
    s.reject = 0;
    s.active = (!s.outer_done && s.irr > 0) ? 1 : 0;
    s.alpha = s.omega = s.beta = mk(0.0, 0.0);
}

// inner BiCGStab start: rho = <rhat, r> = ||r||^2 (rhat = r)
__global__ void k_sc_bicg_init(const double2* part, int nparts, RhsScal* sc) {
    cd q[1];
    fold<1>(part, blockIdx.x, nparts, q);
    if (threadIdx.x) return;
    RhsScal& s = sc[blockIdx.x];
    s.rho = q[0];
    s.irr = q[0].re;
    s.ibb = q[0].re;
    s.best = q[0].re;
    s.since = 0;
    s.reached = 0;
    s.active = (!s.outer_done && s.irr > 0) ? 1 : 0;
    s.breakdown = 0;
    s.alpha = s.omega = s.beta = mk(0.0, 0.0);
}

// partial <rhat, v> -> alpha = rho / <rhat, v>
__global__ void k_sc_bicg_alpha(const double2* part, int nparts, RhsScal* sc) {
    cd q[1];
    fold<1>(part, blockIdx.x, nparts, q);
    if (threadIdx.x) return;
    RhsScal& s = sc[blockIdx.x];
    double den = q[0].re * q[0].re + q[0].im * q[0].im;
    if (s.active && !(den > 1e-300)) {
        s.active = 0;
        s.breakdown = 1;
    }
    s.alpha = s.active ? cdiv(s.rho, q[0]) : mk(0.0, 0.0);
}

// partials <rhat, t>, ||t||^2, <t, s>, <rhat, s> of the second operator
// application -> omega, and with it the next rho = <rhat, s - omega t> and beta
// (the fused iteration: no separate pass over r for <rhat, r>)
__global__ void k_sc_bicg_omega_beta(const double2* part, int nparts, RhsScal* sc) {
    cd q[4];
    fold<4>(part, blockIdx.x, nparts, q);
    if (threadIdx.x) return;
    RhsScal& s = sc[blockIdx.x];
    if (s.active && !(q[1].re > 0)) {
        s.active = 0;
        s.breakdown = 1;
    }
    s.omega = s.active ? mk(q[2].re / q[1].re, q[2].im / q[1].re) : mk(0.0, 0.0);
    if (s.active && (nrm(s.omega) == 0.0 || nrm(s.rho) == 0.0)) {
        s.active = 0;
        s.breakdown = 1;
        s.omega = mk(0.0, 0.0);
    }
    if (!s.active) {
        s.beta = mk(0.0, 0.0);
        return;
    }
    const cd rho_new = q[3] - s.omega * q[0];
    s.beta = cdiv(rho_new, s.rho) * cdiv(s.alpha, s.omega);
    s.rho = rho_new;
}

// partial ||r||^2 -> inner convergence relative to the inner start.  With
// stall > 0, a lane whose ||r|| has not halved within stall iterations stops
// and is marked as broken down (reliable updates then restart its Krylov
// process; defect correction starts its next cycle).
__global__ void k_sc_bicg_conv(const double2* part, int nparts, RhsScal* sc, double tol2, int stall, double hard2) {
    cd q[1];
    fold<1>(part, blockIdx.x, nparts, q);
    if (threadIdx.x) return;
    RhsScal& s = sc[blockIdx.x];
    if (!s.active) return;
    s.irr = q[0].re;
    if (s.irr <= tol2 * s.ibb) {
        // with hard2 > 0 (reliable updates) the lane is marked and iterates on
        // until the next update, or until it has fallen by hard2 as well
        s.reached = 1;
        if (hard2 <= 0 || s.irr <= hard2 * s.ibb) s.active = 0;
        return;
    }
    if (!(s.irr <= 1e12 * s.best)) {
        // blown up (||r|| a million times its best, or not a number): stop,
        // and the correction is discarded rather than folded into the
        // solution (transient BiCGStab spikes stay far below this)
        s.active = 0;
        s.breakdown = 2;
        return;
    }
    if (stall > 0) {
        if (s.irr < 0.25 * s.best) {
            s.best = s.irr;
            s.since = 0;
        } else if (++s.since >= stall) {
            s.active = 0;
            s.breakdown = 1;
        }
    }
}

// CGNR: mode 0 init gam = ||z||^2 ; mode 1 alpha = gam / ||w||^2 ; mode 2 rr = ||r||^2 ;
//       mode 3 beta = ||z||^2 / gam
__global__ void k_sc_cgnr(const double2* part, int nparts, RhsScal* sc, int mode, double tol2) {
    cd q[1];
    fold<1>(part, blockIdx.x, nparts, q);
    if (threadIdx.x) return;
    RhsScal& s = sc[blockIdx.x];
    double v = q[0].re;
    if (mode == 0) {
        s.gam = v;
        s.active = (!s.outer_done && v > 0) ? 1 : 0;
        s.breakdown = 0;
    } else if (mode == 1) {
        if (s.active && !(v > 0)) {
            s.active = 0;
            s.breakdown = 1;
        }
        s.alpha = mk(s.active ? s.gam / v : 0.0, 0.0);
    } else if (mode == 2) {
        s.rr = v;
        if (s.rr <= tol2 * s.bb) s.active = 0;
    } else {
        s.beta = mk(s.active ? v / s.gam : 0.0, 0.0);
        s.gam = v;
    }
}

// --------------------------------------------------------------- host side
struct Work {
    disco_ctx* ctx;
    int n;            // rhs in this block
    long V;
    RhsScal* sc;      // device [n]
    double2* part;    // device partials
    int nsb;          // stencil partial slots
    std::vector<RhsScal> h;
};

static VecGeo vgeo(long V, int prec, int n) {
    int C = prec == DISCO_F64 ? 1 : prec == DISCO_F32 ? 2 : 4;
    VecGeo g;
    g.n = n;
    g.total = 12 * V / C * n;
    g.bd = (kMaxBlock / n) * n;
    long want = (g.total + g.bd - 1) / g.bd;
    g.nb = (int)std::max(1L, std::min(want, 2048L));
    return g;
}

static int site_grid(long V, int n) { return (int)std::min<long>((V * n + 255) / 256, 4096); }

template <class IO>
static void norm2(Work& w, const void* v, VecGeo g) {
    hipLaunchKernelGGL(k_norm2<IO>, dim3(g.nb), dim3(g.bd), 0, w.ctx->stream, v, g, w.part);
}

template <class IOS, class IOD>
static void copy_scale(Work& w, const void* src, void* dst, int use_scale) {
    hipLaunchKernelGGL((k_copy_scale<IOS, IOD>), dim3(site_grid(w.V, w.n)), dim3(256), 0, w.ctx->stream, src, dst,
                       w.V, w.n, w.sc, use_scale);
}

template <class IO>
static void dc_update(Work& w, double2* x64, const void* e) {
    hipLaunchKernelGGL((k_dc_update<IO>), dim3(site_grid(w.V, w.n)), dim3(256), 0, w.ctx->stream, x64, e, w.V, w.n,
                       w.sc);
}

static void pull(Work& w) {
    w.h.resize(w.n);
    HIPCHK(hipMemcpyAsync(w.h.data(), w.sc, sizeof(RhsScal) * w.n, hipMemcpyDeviceToHost, w.ctx->stream));
    HIPCHK(hipStreamSynchronize(w.ctx->stream));
}

static void push(Work& w, const std::vector<RhsScal>& h) {
    HIPCHK(hipMemcpyAsync(w.sc, h.data(), sizeof(RhsScal) * w.n, hipMemcpyHostToDevice, w.ctx->stream));
    HIPCHK(hipStreamSynchronize(w.ctx->stream));
}

static void stencil(Work& w, int prec, int dag, const void* in, void* out, const void* aux, const void* aux2,
                    const uint8_t* mask, int epi) {
    disco::StencilCall c{prec, dag, w.n, in, out, aux, aux2, mask, w.part, epi};
    disco::stencil_launch(w.ctx, c);
}

// r64 = b64 - D x64 with the FP64 operator and ||r||^2 -> outer scalars (mode 1)
static void outer_residual(Work& w, const double2* b64, const double2* x64, double2* r64, const uint8_t* mask,
                           double tol2) {
    stencil(w, DISCO_F64, 0, x64, r64, b64, nullptr, mask, disco::EPI_RESID | disco::EPI_NORM);
    k_sc_outer<<<w.n, kScalarBlock, 0, w.ctx->stream>>>(w.part, w.nsb, w.sc, 1, tol2);
}

// FP64 CGNR on D e = rhs (e starts at 0) to relative residual tol.  Uses and
// overwrites the device state (bb/rr/outer_done of the rhs system).
static void cgnr_run(Work& w, const double2* rhs, double2* e, const uint8_t* mask, double tol, int max_iter,
                     int check_every, int* iters) {
    disco_ctx* ctx = w.ctx;
    VecGeo g = vgeo(w.V, DISCO_F64, w.n);
    size_t nb = disco::native_bytes(ctx, DISCO_F64, w.n);
    double2* r = (double2*)ws_get(ctx, "cg_r", nb);
    double2* z = (double2*)ws_get(ctx, "cg_z", nb);
    double2* p = (double2*)ws_get(ctx, "cg_p", nb);
    double2* q = (double2*)ws_get(ctx, "cg_w", nb);
    const double tol2 = tol * tol;
    k_zero<IO64><<<1024, 256, 0, ctx->stream>>>(e, g.total);
    copy_scale<IO64, IO64>(w, rhs, r, 0);
    norm2<IO64>(w, r, g);
    k_sc_outer<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, g.nb, w.sc, 0, tol2);
    stencil(w, DISCO_F64, 1, r, z, nullptr, nullptr, mask, disco::EPI_NORM);
    k_sc_cgnr<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, w.nsb, w.sc, 0, tol2);
    copy_scale<IO64, IO64>(w, z, p, 0);
    int it = 0;
    while (it < max_iter) {
        for (int k = 0; k < check_every && it < max_iter; k++, it++) {
            stencil(w, DISCO_F64, 0, p, q, nullptr, nullptr, mask, disco::EPI_NORM);
            k_sc_cgnr<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, w.nsb, w.sc, 1, tol2);
            hipLaunchKernelGGL(k_cgnr_xr, dim3(g.nb), dim3(g.bd), 0, ctx->stream, e, p, q, r, g, w.sc, w.part);
            k_sc_cgnr<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, g.nb, w.sc, 2, tol2);
            stencil(w, DISCO_F64, 1, r, z, nullptr, nullptr, mask, disco::EPI_NORM);
            k_sc_cgnr<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, w.nsb, w.sc, 3, tol2);
            hipLaunchKernelGGL(k_cgnr_p, dim3(g.nb), dim3(g.bd), 0, ctx->stream, p, z, g, w.sc);
        }
        HIPCHK(hipGetLastError());
        pull(w);
        bool any = false;
        for (auto& s : w.h) any |= s.active != 0;
        if (!any) break;
    }
    *iters += it;
}

// Operator of an inner Krylov solve: the full (or domain-restricted) D on
// whole-lattice vectors, or the even-odd Schur complement
//   M = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe
// on even half-lattice vectors (two even-odd stencil launches, the second
// carrying the reduction epilogue).
struct InnerOp {
    bool eo = false;
    long Vv = 0;   // sites of the vectors
    int nsb = 0;   // partial-sum slots of the launch with the epilogue
};

static void op_apply(Work& w, const InnerOp& op, int prec, const void* in, void* out, const void* aux2,
                     const uint8_t* mask, int epi, void* tmp) {
    if (!op.eo) {
        stencil(w, prec, 0, in, out, nullptr, aux2, mask, epi);
        return;
    }
    const double k = w.ctx->kappa;
    disco::StencilCall c1{prec, 0, w.n, in, tmp, nullptr, nullptr, mask, nullptr, disco::EPI_NONE, 1, 0.0, 0.0, 1.0};
    disco::stencil_launch(w.ctx, c1);
    disco::StencilCall c2{prec, 0, w.n, tmp, out, in, aux2, mask, w.part, epi, 0, 1.0, 0.0, -k * k};
    disco::stencil_launch(w.ctx, c2);
}

// inner BiCGStab on op e = rin (normalised defect) in storage IO
// hint: iterations the previous inner solve of this system took; that many
// chunks (less one) run back to back before the host first reads the state.
// refresh (reliable updates): called, with w.V at the full lattice and the
// iterations so far, whenever an unfinished lane's inner residual has fallen
// by inner_tol (or broken down); it refreshes the inner state and returns
// false once every lane is finished (or it gives up).
template <class IO>
static int bicg_run(Work& w, const InnerOp& op, int prec, const void* rin, void* e, const uint8_t* mask,
                    double inner_tol, int max_iter, int check_every, int hint = 0,
                    const std::function<bool(int)>* refresh = nullptr, int stall = 0, double hard2 = 0.0) {
    disco_ctx* ctx = w.ctx;
    const long Vfull = w.V;
    w.V = op.Vv;  // vector helpers below work on the operator's vectors
    VecGeo g = vgeo(w.V, prec, w.n);
    size_t nb = disco::native_bytes(ctx, prec, w.n);
    void* r = ws_get(ctx, "bi_r", nb);
    void* rh = ws_get(ctx, "bi_rh", nb);
    void* p = ws_get(ctx, "bi_p", nb);
    void* v = ws_get(ctx, "bi_v", nb);
    void* s = ws_get(ctx, "bi_s", nb);
    void* t = ws_get(ctx, "bi_t", nb);
    void* tmp = op.eo ? ws_get(ctx, "bi_eotmp", nb / 2) : nullptr;
    k_zero<IO><<<1024, 256, 0, ctx->stream>>>(e, g.total);
    copy_scale<IO, IO>(w, rin, r, 0);
    copy_scale<IO, IO>(w, rin, rh, 0);
    copy_scale<IO, IO>(w, rin, p, 0);
    norm2<IO>(w, r, g);
    k_sc_bicg_init<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, g.nb, w.sc);
    const double tol2 = inner_tol * inner_tol;
    // one BiCGStab iteration: 2 operator applications with fused reductions
    // (the second one's four sums give omega and beta), 2 vector passes
    // (s, then x, r and p together), 3 scalar steps
    auto iteration = [&]() {
        op_apply(w, op, prec, p, v, rh, mask, disco::EPI_DOTAUX, tmp);
        k_sc_bicg_alpha<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, op.nsb, w.sc);
        hipLaunchKernelGGL(k_bicg_s<IO>, dim3(g.nb), dim3(g.bd), 0, ctx->stream, r, v, s, g, w.sc);
        op_apply(w, op, prec, s, t, rh, mask,
                 disco::EPI_DOTAUX | disco::EPI_NORM | disco::EPI_DOTIN | disco::EPI_DOTAUXIN, tmp);
        k_sc_bicg_omega_beta<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, op.nsb, w.sc);
        hipLaunchKernelGGL(k_bicg_xrp<IO>, dim3(g.nb), dim3(g.bd), 0, ctx->stream, e, p, s, t, v, r, g, w.sc, w.part);
        k_sc_bicg_conv<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, g.nb, w.sc, tol2, stall, hard2);
    };
    // A chunk of check_every iterations is captured once as a graph and replayed
    // between the host's convergence reads (eager when profiling or disabled).
    hipGraphExec_t exec = nullptr;
    if (ctx->opt_graphs && !ctx->prof_on && check_every > 1) {
        char key[512];
        snprintf(key, sizeof(key), "bicg/%d/%d/%d/%d/%p/%p/%p/%p/%p/%p/%p/%p/%p/%p/%p/%g/%d/%g", prec, w.n,
                 check_every, op.eo ? 1 : 0, (void*)mask, r, rh, p, v, s, t, e, tmp, (void*)w.sc, (void*)w.part, tol2,
                 stall, hard2);
        auto itg = ctx->graphs.find(key);
        if (itg != ctx->graphs.end()) {
            exec = itg->second;
        } else {
            if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
            // work already queued on the caller's stream must not be reordered around the capture
            HIPCHK(hipStreamSynchronize(ctx->stream));
            hipStream_t user = ctx->stream;
            ctx->stream = ctx->cap_stream;
            hipGraph_t graph = nullptr;
            HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            try {
                for (int k = 0; k < check_every; k++) iteration();
            } catch (...) {
                hipGraph_t dead = nullptr;
                (void)hipStreamEndCapture(ctx->cap_stream, &dead);
                if (dead) (void)hipGraphDestroy(dead);
                ctx->stream = user;
                w.V = Vfull;
                throw;
            }
            hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &graph);
            ctx->stream = user;
            HIPCHK(ec);
            hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIPCHK(ei);
            ctx->graphs[key] = exec;
        }
    }
    int it = 0;
    int blind = std::max(0, hint - check_every) / check_every;
    int last_update = 0;
    while (it < max_iter) {
        if (exec && max_iter - it >= check_every) {
            HIPCHK(hipGraphLaunch(exec, ctx->stream));
            it += check_every;
        } else {
            for (int k = 0; k < check_every && it < max_iter; k++, it++) iteration();
        }
        HIPCHK(hipGetLastError());
        if (blind > 0) {
            blind--;
            continue;
        }
        pull(w);
        if (refresh) {
            // an update when a lane has stopped (breakdown, stall, its hard
            // limit), or when a quarter of the open lanes have fallen by inner_tol
            bool need = false;
            int nopen = 0, nreached = 0;
            for (auto& sc : w.h) {
                if (sc.outer_done) continue;
                nopen++;
                nreached += sc.reached != 0;
                need |= sc.active == 0;
            }
            if (!nopen) break;
            need |= nreached >= std::max(1, nopen / 4);
            if (need) {
                w.V = Vfull;
                const bool more = (*refresh)(it);
                w.V = op.Vv;
                if (!more) break;
                // the next update is likely about as far away as this one was:
                // run half that many iterations without host reads
                blind = std::max(0, (it - last_update) / 2 - check_every) / check_every;
                last_update = it;
            }
            continue;
        }
        bool any = false;
        for (auto& sc : w.h) any |= sc.active != 0;
        if (!any) break;
    }
    w.V = Vfull;
    return it;
}

// ---- even-odd helpers on native blocks (site s of parity p <-> index s/2 of half vector p)
__device__ __forceinline__ int parity_of(long s, int Lx, int Ly, int Lz) {
    const long x = s % Lx, r1 = s / Lx;
    const long y = r1 % Ly, r2 = r1 / Ly;
    const long z = r2 % Lz, t = r2 / Lz;
    return (int)((x + y + z + t) & 1);
}
template <class IO>
__global__ void k_eo_split(const void* __restrict__ full, void* __restrict__ he, void* __restrict__ ho, long V, int n,
                           int Lx, int Ly, int Lz) {
    const long tot = V * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const long st = j / n;
        const int r = (int)(j - st * n);
        cx<typename IO::T> p[12];
        IO::load(full, V, n, r, (int)st, p);
        IO::store(parity_of(st, Lx, Ly, Lz) ? ho : he, V / 2, n, r, (int)(st >> 1), p);
    }
}
template <class IO>
__global__ void k_eo_merge(const void* __restrict__ he, const void* __restrict__ ho, void* __restrict__ full, long V,
                           int n, int Lx, int Ly, int Lz) {
    const long tot = V * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const long st = j / n;
        const int r = (int)(j - st * n);
        cx<typename IO::T> p[12];
        IO::load(parity_of(st, Lx, Ly, Lz) ? ho : he, V / 2, n, r, (int)(st >> 1), p);
        IO::store(full, V, n, r, (int)st, p);
    }
}
// k_copy_scale (FP64 -> inner precision, times scale[r]) and k_eo_split in
// one pass: the scaled residual goes straight to its even and odd halves.
template <class IO>
__global__ void k_scale_split(const double2* __restrict__ full, void* __restrict__ he, void* __restrict__ ho, long V,
                              int n, const RhsScal* __restrict__ sc, int Lx, int Ly, int Lz) {
    typedef typename IO::T T;
    const long tot = V * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const long st = j / n;
        const int r = (int)(j - st * n);
        const double f = sc[r].scale;
        cx<double> a[12];
        cx<T> b[12];
        IO64::load(full, V, n, r, (int)st, a);
#pragma unroll
        for (int k = 0; k < 12; k++) b[k] = mk((T)(f * a[k].re), (T)(f * a[k].im));
        IO::store(parity_of(st, Lx, Ly, Lz) ? ho : he, V / 2, n, r, (int)(st >> 1), b);
    }
}
// k_eo_merge and k_dc_update in one pass: x64 += (1/scale[r]) e with e read
// from its even and odd halves (same lanes skipped, and the same UNDO, as
// k_dc_update).
template <class IO, bool UNDO = false>
__global__ void k_dc_update_eo(double2* __restrict__ x64, const void* __restrict__ he, const void* __restrict__ ho,
                               long V, int n, const RhsScal* __restrict__ sc, int Lx, int Ly, int Lz) {
    const long tot = V * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const long st = j / n;
        const int r = (int)(j - st * n);
        if (UNDO ? sc[r].reject != 1 : (sc[r].outer_done || sc[r].breakdown == 2)) continue;
        const double f = (sc[r].scale > 0 ? 1.0 / sc[r].scale : 0.0) * (UNDO ? -1.0 : 1.0);
        cx<typename IO::T> a[12];
        cx<double> x[12];
        IO::load(parity_of(st, Lx, Ly, Lz) ? ho : he, V / 2, n, r, (int)(st >> 1), a);
        IO64::load(x64, V, n, r, (int)st, x);
#pragma unroll
        for (int k = 0; k < 12; k++) x[k] = mk(x[k].re + f * (double)a[k].re, x[k].im + f * (double)a[k].im);
        IO64::store(x64, V, n, r, (int)st, x);
    }
}

// out = A^-1 in on the half vector of parity par (site-local)
template <class IO>
__global__ void k_eo_clover_inv(const void* __restrict__ in, void* __restrict__ out, const void* __restrict__ Ai,
                                long V, int n, int par, int Lx, int Ly, int Lz) {
    typedef typename IO::T T;
    const long Vh = V / 2;
    const long tot = Vh * n;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < tot; j += (long)gridDim.x * blockDim.x) {
        const long h = j / n;
        const int r = (int)(j - h * n);
        const long st = parity_of(2 * h, Lx, Ly, Lz) == par ? 2 * h : 2 * h + 1;
        cx<T> p[12], o[12];
        IO::load(in, Vh, n, r, (int)h, p);
        T f[36];
#pragma unroll
        for (int b = 0; b < 2; b++) {
            IO::load_clover((const typename IO::CloverT*)Ai, V, b, (int)st, f);
#pragma unroll
            for (int i = 0; i < 6; i++) o[6 * b + i] = f[i] * p[6 * b + i];
            int m = 0;
#pragma unroll
            for (int i = 0; i < 6; i++)
#pragma unroll
                for (int k = i + 1; k < 6; k++, m++) {
                    const cx<T> a = mk(f[6 + 2 * m], f[7 + 2 * m]);
                    o[6 * b + i] = o[6 * b + i] + a * p[6 * b + k];
                    o[6 * b + k] = o[6 * b + k] + cj(a) * p[6 * b + i];
                }
        }
        IO::store(out, Vh, n, r, (int)h, o);
    }
}

// Inner solve D e = rin through the even-odd Schur complement:
//   rhat = A_ee^-1 (r_e + kappa H_eo A_oo^-1 r_o),  M e_e = rhat (BiCGStab),
//   e_o = A_oo^-1 (r_o + kappa H_oe e_e).
// With r64 and x64 given (defect correction), rin = scale[r] r64 is split into
// its halves straight from the FP64 residual, and the correction is folded
// into x64 from its halves (x64 += e / scale[r]) instead of being merged into e.
template <class IO>
static int bicg_run_eo(Work& w, int prec, const void* rin, void* e, const uint8_t* mask, double inner_tol,
                       int max_iter, int check_every, int hint = 0, int stall = 0, const double2* r64 = nullptr,
                       double2* x64 = nullptr) {
    disco_ctx* ctx = w.ctx;
    const long V = w.V;
    const int n = w.n;
    const size_t hb = disco::native_bytes(ctx, prec, n) / 2;
    void* re = ws_get(ctx, "eo_re", hb);
    void* ro = ws_get(ctx, "eo_ro", hb);
    void* uo = ws_get(ctx, "eo_uo", hb);
    void* rhat = ws_get(ctx, "eo_rhat", hb);
    void* ee = ws_get(ctx, "eo_ee", hb);
    void* eo = ws_get(ctx, "eo_eo", hb);
    const int Lx = ctx->dims[0], Ly = ctx->dims[1], Lz = ctx->dims[2];
    const void* Ai = prec == DISCO_F64 ? (const void*)ctx->Ai64 : (const void*)ctx->Ai32;
    const int grid = site_grid(V, n);
    const double k = ctx->kappa;
    if (r64)
        hipLaunchKernelGGL(k_scale_split<IO>, dim3(grid), dim3(256), 0, ctx->stream, r64, re, ro, V, n, w.sc, Lx, Ly,
                           Lz);
    else
        hipLaunchKernelGGL(k_eo_split<IO>, dim3(grid), dim3(256), 0, ctx->stream, rin, re, ro, V, n, Lx, Ly, Lz);
    hipLaunchKernelGGL(k_eo_clover_inv<IO>, dim3(site_grid(V / 2, n)), dim3(256), 0, ctx->stream, ro, uo, Ai, V, n, 1,
                       Lx, Ly, Lz);
    disco::StencilCall cp{prec, 0, n, uo, rhat, re, nullptr, mask, nullptr, disco::EPI_NONE, 0, 0.0, 1.0, k};
    disco::stencil_launch(ctx, cp);
    InnerOp op;
    op.eo = true;
    op.Vv = V / 2;
    op.nsb = disco::stencil_nsb(ctx, n, true);
    const int it = bicg_run<IO>(w, op, prec, rhat, ee, mask, inner_tol, max_iter, check_every, hint, nullptr, stall);
    disco::StencilCall cr{prec, 0, n, ee, eo, ro, nullptr, mask, nullptr, disco::EPI_NONE, 1, 0.0, 1.0, k};
    disco::stencil_launch(ctx, cr);
    if (x64)
        hipLaunchKernelGGL((k_dc_update_eo<IO>), dim3(grid), dim3(256), 0, ctx->stream, x64, ee, eo, V, n, w.sc, Lx, Ly,
                           Lz);
    else
        hipLaunchKernelGGL(k_eo_merge<IO>, dim3(grid), dim3(256), 0, ctx->stream, ee, eo, e, V, n, Lx, Ly, Lz);
    HIPCHK(hipGetLastError());
    return it;
}

static void fill_stats(Work& w, const disco_solver_params& P, int iters, int outer, int fb, disco_solver_stats* st) {
    for (int i = 0; i < w.n; i++) {
        st[i].iters = iters;
        st[i].outer_iters = outer;
        st[i].fallback_used = fb;
        st[i].true_rel_residual = w.h[i].bb > 0 ? std::sqrt(w.h[i].rr / w.h[i].bb) : 0.0;
        st[i].converged = st[i].true_rel_residual <= P.tol;
    }
}

// FP64 CGNR correction of x64 on the current defect r64 (the fallback, and the
// restart loop of the plain solver).  Restores the outer state afterwards and
// recomputes the true residual.
static void cgnr_correct(Work& w, const double2* b64, double2* x64, double2* r64, const uint8_t* mask, double tol,
                         int max_iter, int check, int* iters) {
    disco_ctx* ctx = w.ctx;
    double2* e = (double2*)ws_get(ctx, "dc_ecg", disco::native_bytes(ctx, DISCO_F64, w.n));
    pull(w);
    const std::vector<RhsScal> outer_state = w.h;
    double worst = 1e-300;
    for (auto& s : outer_state)
        if (!s.outer_done && s.bb > 0) worst = std::max(worst, std::sqrt(s.rr / s.bb));
    // relative target on the defect system: tol * ||b|| / ||r|| (with margin)
    const double rtol = std::max(1e-16, 0.5 * tol / worst);
    cgnr_run(w, r64, e, mask, rtol, max_iter, check, iters);
    std::vector<RhsScal> h = outer_state;
    for (auto& s : h) {
        s.scale = 1.0;  // x += e for the right-hand sides still running
        s.breakdown = 0;
    }
    push(w, h);
    dc_update<IO64>(w, x64, e);
    push(w, outer_state);
    outer_residual(w, b64, x64, r64, mask, tol * tol);
    pull(w);
}

template <class IO>
static void dc_solve(Work& w, const disco_solver_params& P, int prec, const double2* b64, double2* x64,
                     const uint8_t* mask, disco_solver_stats* st) {
    disco_ctx* ctx = w.ctx;
    size_t nb64 = disco::native_bytes(ctx, DISCO_F64, w.n);
    size_t nbp = disco::native_bytes(ctx, prec, w.n);
    double2* r64 = (double2*)ws_get(ctx, "dc_r64", nb64);
    void* rin = ws_get(ctx, "dc_rin", nbp);
    void* e = ws_get(ctx, "dc_e", nbp);
    VecGeo g64 = vgeo(w.V, DISCO_F64, w.n);
    const double tol2 = P.tol * P.tol;
    k_zero<IO64><<<1024, 256, 0, ctx->stream>>>(x64, g64.total);
    norm2<IO64>(w, b64, g64);
    k_sc_outer<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, g64.nb, w.sc, 0, tol2);
    copy_scale<IO64, IO64>(w, b64, r64, 0);
    int iters = 0, outer = 0;
    const int max_iter = P.max_iter > 0 ? P.max_iter : 100000;
    const int check = P.check_every > 0 ? P.check_every : 2;
    const double itol = P.inner_tol > 0 ? P.inner_tol : (prec == DISCO_BF16 ? 3e-2 : 1e-5);
    const int inner_cap = 2000;
    const bool trace = getenv("DISCO_TRACE") != nullptr;
    const bool use_eo = ctx->opt_eo && disco::eo_supported(ctx);
    double last_worst = 1e300;
    int stall = 0, it_best = 0;
    int hint = 0;
    while (true) {
        pull(w);
        bool done = true;
        double worst = 0;
        int nd = 0;
        for (auto& s : w.h) {
            done &= s.outer_done != 0;
            nd += s.outer_done;
            if (s.bb > 0) worst = std::max(worst, std::sqrt(s.rr / s.bb));
        }
        if (trace)
            fprintf(stderr, "[disco] outer %d: worst true rel residual %.3e, %d/%d done, %d inner iterations\n",
                    outer, worst, nd, w.n, iters);
        if (done || iters >= max_iter) break;
        // no halving of the worst true residual over 5 cycles and 800 inner
        // iterations: leave it to the fallback
        if (worst > 0.5 * last_worst) {
            stall++;
        } else {
            stall = 0;
            it_best = iters;
        }
        last_worst = std::min(last_worst, worst);
        if (stall >= 5 && iters - it_best >= 800) break;
        outer++;
        int ran;
        if (use_eo) {
            // scaled residual split and correction folded in by the inner solve
            ran = bicg_run_eo<IO>(w, prec, nullptr, nullptr, mask, itol, std::min(inner_cap, max_iter - iters), check,
                                  hint, kRuStall, r64, x64);
        } else {
            copy_scale<IO64, IO>(w, r64, rin, 1);
            InnerOp op;
            op.Vv = w.V;
            op.nsb = w.nsb;
            ran = bicg_run<IO>(w, op, prec, rin, e, mask, itol, std::min(inner_cap, max_iter - iters), check, hint,
                               nullptr, kRuStall);
            dc_update<IO>(w, x64, e);
        }
        iters += ran;
        hint = ran;
        outer_residual(w, b64, x64, r64, mask, tol2);
    }
    int fb = 0;
    pull(w);
    bool done = true;
    for (auto& s : w.h) done &= s.outer_done != 0;
    if (!done && P.fallback) {
        fb = 1;
        int before = iters;
        cgnr_correct(w, b64, x64, r64, mask, P.tol, std::max(1, max_iter - iters), check, &iters);
        if (trace) fprintf(stderr, "[disco] fallback CGNR %d iterations\n", iters - before);
    }
    fill_stats(w, P, iters, outer, fb, st);
}

// BiCGStab in inner precision with reliable updates (BICGSTAB_RU).  One
// Krylov process runs for the whole solve instead of one per defect-
// correction cycle.  Whenever the recursive residual of an unfinished lane
// has fallen by inner_tol since the last update, every lane's correction is
// folded into the FP64 solution, the FP64 true residual is recomputed, and
// the inner system's residual is replaced by the one it gives (its source in
// even-odd form), with the search direction adjusted to match; the shadow
// residual and the scalars carry on.  Lanes that break down, or whose true
// residual does not follow the recursive one, restart their Krylov process.
// The inner vectors keep the scale 1/||b|| of the start.
//
// With a feeder (continuous batching), a lane whose right-hand side has
// converged hands its solution over at that update and takes the next one
// from the queue, with a Krylov process of its own; st then has one entry per
// right-hand side of the queue.  When the block stops early (the worst true
// residual stalls, or the iteration cap of the lanes in flight is reached),
// the lanes in flight get the FP64 fallback (when allowed) and are handed
// over, and the rest of the queue runs on in a fresh Krylov process: one hard
// right-hand side does not cost the ones behind it.
static Work make_work(disco_ctx* ctx, int n) {
    Work w;
    w.ctx = ctx;
    w.n = n;
    w.V = ctx->V;
    w.nsb = disco::stencil_nsb(ctx, n);
    w.sc = (RhsScal*)ws_get(ctx, "sv_scal", sizeof(RhsScal) * n);
    VecGeo g = vgeo(ctx->V, DISCO_F64, n);
    size_t slots = (size_t)std::max(std::max(w.nsb, disco::stencil_nsb(ctx, n, true)), g.nb);
    w.part = (double2*)ws_get(ctx, "sv_part", sizeof(double2) * slots * 4 * n);
    HIPCHK(hipMemsetAsync(w.sc, 0, sizeof(RhsScal) * n, ctx->stream));
    return w;
}

template <class IO>
static void ru_solve(Work& w, const disco_solver_params& P, int prec, double2* b64, double2* x64,
                     const uint8_t* mask, disco_solver_stats* st, disco::LaneFeeder* feed = nullptr,
                     long long* block_iters = nullptr) {
    disco_ctx* ctx = w.ctx;
    int n = w.n;  // the block's width (narrower for the tail of a queue)
    const long V = w.V;
    const size_t nb64 = disco::native_bytes(ctx, DISCO_F64, n);
    const size_t nbp = disco::native_bytes(ctx, prec, n);
    double2* r64 = (double2*)ws_get(ctx, "dc_r64", nb64);
    void* rin = ws_get(ctx, "dc_rin", nbp);
    void* efull = ws_get(ctx, "dc_e", nbp);
    VecGeo g64 = vgeo(V, DISCO_F64, n);
    const double tol2 = P.tol * P.tol;
    const int check = P.check_every > 0 ? P.check_every : 2;
    const double delta = P.inner_tol > 0 ? P.inner_tol : (prec == DISCO_BF16 ? 3e-2 : 1e-3);
    const bool eo = ctx->opt_eo && disco::eo_supported(ctx);
    const long Vv = eo ? V / 2 : V;
    const size_t hb = eo ? nbp / 2 : nbp;
    const int Lx = ctx->dims[0], Ly = ctx->dims[1], Lz = ctx->dims[2];
    const double k = ctx->kappa;
    void* re = eo ? ws_get(ctx, "eo_re", hb) : nullptr;
    void* ro = eo ? ws_get(ctx, "eo_ro", hb) : nullptr;
    void* uo = eo ? ws_get(ctx, "eo_uo", hb) : nullptr;
    void* rhat = eo ? ws_get(ctx, "eo_rhat", hb) : rin;
    void* ee = eo ? ws_get(ctx, "eo_ee", hb) : efull;
    void* eodd = eo ? ws_get(ctx, "eo_eo", hb) : nullptr;
    const void* Ai = prec == DISCO_F64 ? (const void*)ctx->Ai64 : (const void*)ctx->Ai32;
    const bool trace = getenv("DISCO_TRACE") != nullptr;
    // queue state: lane -> right-hand side (-1 idle), and where each started
    std::vector<int> lane_src(n, -1), lane_it0(n, 0), lane_up0(n, 0);
    int next = 0;
    int* dflag = feed ? (int*)ws_get(ctx, "ru_flag", sizeof(int) * n) : nullptr;
    int* dlane = feed ? (int*)ws_get(ctx, "ru_lane", sizeof(int) * n) : nullptr;
    std::vector<int> hflag(n, 0), hlane(n, 0);
    // scale[r] r64 -> rhat, the inner system's source (in even-odd form the
    // scaled residual is split into re, ro on the way, without a full-lattice copy)
    auto prepare = [&]() {
        if (!eo) {
            copy_scale<IO64, IO>(w, r64, rin, 1);
            return;
        }
        hipLaunchKernelGGL(k_scale_split<IO>, dim3(site_grid(V, n)), dim3(256), 0, ctx->stream, r64, re, ro, V, n,
                           w.sc, Lx, Ly, Lz);
        hipLaunchKernelGGL(k_eo_clover_inv<IO>, dim3(site_grid(V / 2, n)), dim3(256), 0, ctx->stream, ro, uo, Ai, V,
                           n, 1, Lx, Ly, Lz);
        disco::StencilCall cp{prec, 0, n, uo, rhat, re, nullptr, mask, nullptr, disco::EPI_NONE, 0, 0.0, 1.0, k};
        disco::stencil_launch(ctx, cp);
    };
    // fold the correction into x64 (in even-odd form its odd half is first
    // reconstructed from the source it belongs to, and both halves are read
    // in place) and recompute the FP64 true residual
    auto fold_in = [&]() {
        if (eo) {
            disco::StencilCall cr{prec, 0, n, ee, eodd, ro, nullptr, mask, nullptr, disco::EPI_NONE, 1, 0.0, 1.0, k};
            disco::stencil_launch(ctx, cr);
            hipLaunchKernelGGL((k_dc_update_eo<IO>), dim3(site_grid(V, n)), dim3(256), 0, ctx->stream, x64, ee,
                               eodd, V, n, w.sc, Lx, Ly, Lz);
        } else {
            dc_update<IO>(w, x64, efull);
        }
        stencil(w, DISCO_F64, 0, x64, r64, b64, nullptr, mask, disco::EPI_RESID | disco::EPI_NORM);
        k_sc_outer<<<n, kScalarBlock, 0, ctx->stream>>>(w.part, w.nsb, w.sc, 2, tol2);
        pull(w);
        // a correction that raised its lane's true residual far above the last
        // update's is taken back (the inner process went astray; folding it in
        // would leave the lane further from the solution than before)
        int nrej = 0;
        for (const auto& h : w.h) nrej += h.reject == 1;
        if (nrej) {
            if (trace)
                for (int i = 0; i < n; i++)
                    if (w.h[i].reject == 1)
                        fprintf(stderr, "[disco] lane %d: correction taken back (true residual %.3e, before %.3e)\n",
                                i, std::sqrt(w.h[i].rr / w.h[i].bb), std::sqrt(w.h[i].gam / w.h[i].bb));
            if (eo)
                hipLaunchKernelGGL((k_dc_update_eo<IO, true>), dim3(site_grid(V, n)), dim3(256), 0, ctx->stream, x64,
                                   ee, eodd, V, n, w.sc, Lx, Ly, Lz);
            else
                hipLaunchKernelGGL((k_dc_update<IO, true>), dim3(site_grid(V, n)), dim3(256), 0, ctx->stream, x64,
                                   efull, V, n, w.sc);
            stencil(w, DISCO_F64, 0, x64, r64, b64, nullptr, mask, disco::EPI_RESID | disco::EPI_NORM);
            k_sc_outer<<<n, kScalarBlock, 0, ctx->stream>>>(w.part, w.nsb, w.sc, 3, tol2);
            pull(w);
        }
    };
    InnerOp op;
    op.eo = eo;
    op.Vv = Vv;
    op.nsb = disco::stencil_nsb(ctx, n, eo);
    long long iters_all = 0;
    // carry: the episode continues the open lanes of a wider block (their x64
    // and b64 already moved into lanes 0..held-1), instead of loading the queue
    bool carry = false;
    int carried = 0;
    // one episode per Krylov process of the block (a single one unless the
    // block stops before the queue is empty, or narrows for its tail)
    for (;;) {
        int outer = 0, stall = 0, it_best = 0;
        double last_worst = 1e300;
        bool gave_up = false, narrowing = false;
        int held = 0;
        if (feed && carry) {
            held = carried;
        } else if (feed) {
            // fill every lane from the queue; lanes left idle get b = 0 (they
            // may still hold a right-hand side of the previous episode), which
            // marks them finished at the start
            int m = 0;
            for (int r = 0; r < n; r++) {
                lane_it0[r] = 0;
                lane_up0[r] = 0;
                if (next < feed->total) {
                    feed->load(r, next, n);
                    lane_src[r] = next++;
                    held++;
                } else {
                    lane_src[r] = -1;
                    hlane[m++] = r;
                }
            }
            if (m) {
                HIPCHK(hipMemcpyAsync(dlane, hlane.data(), sizeof(int) * m, hipMemcpyHostToDevice, ctx->stream));
                hipLaunchKernelGGL(k_lane_clear, dim3(1024), dim3(256), 0, ctx->stream, b64, V, n, dlane, m);
            }
        }
        if (carry) {
            norm2<IO64>(w, b64, g64);
            k_sc_outer<<<n, kScalarBlock, 0, ctx->stream>>>(w.part, g64.nb, w.sc, 0, tol2);
            stencil(w, DISCO_F64, 0, x64, r64, b64, nullptr, mask, disco::EPI_RESID | disco::EPI_NORM);
            k_sc_outer<<<n, kScalarBlock, 0, ctx->stream>>>(w.part, w.nsb, w.sc, 4, tol2);
            carry = false;
        } else {
            k_zero<IO64><<<1024, 256, 0, ctx->stream>>>(x64, g64.total);
            norm2<IO64>(w, b64, g64);
            k_sc_outer<<<n, kScalarBlock, 0, ctx->stream>>>(w.part, g64.nb, w.sc, 0, tol2);
            copy_scale<IO64, IO64>(w, b64, r64, 0);
        }
        // with a queue the cap applies per wave of the right-hand sides this
        // episode starts with or still has to take
        const int waves = feed ? std::max(1, (held + (feed->total - next) + n - 1) / n) : 1;
        const int max_iter =
            (int)std::min<long long>(2000000000LL, (long long)(P.max_iter > 0 ? P.max_iter : 100000) * waves);
        prepare();
        std::vector<int> done_at(w.n, 0);
        // hand over the lanes whose right-hand side is finished (all lanes still
        // holding one when final), with their statistics
        auto hand_over = [&](int it, bool final, int fb) {
            std::vector<int> lanes, js;
            for (int r = 0; r < n; r++) {
                if (lane_src[r] < 0 || (!final && !w.h[r].outer_done)) continue;
                const int j = lane_src[r];
                disco_solver_stats& q = st[j];
                q.iters = it - lane_it0[r];
                q.outer_iters = std::max(1, outer - lane_up0[r]);
                q.fallback_used = fb;
                q.true_rel_residual = w.h[r].bb > 0 ? std::sqrt(w.h[r].rr / w.h[r].bb) : 0.0;
                q.converged = q.true_rel_residual <= P.tol;
                lanes.push_back(r);
                js.push_back(j);
                lane_src[r] = -1;
            }
            if (!lanes.empty()) feed->store(lanes, js, n);
            return lanes;
        };
        std::function<bool(int)> refresh = [&](int it) -> bool {
            fold_in();
            outer++;
            // finished lanes hand over and take the next right-hand sides; again
            // while a new one is finished at once (a zero right-hand side)
            for (bool again = feed != nullptr; again;) {
                again = false;
                const std::vector<int> freed = hand_over(it, false, 0);
                bool refill = false;
                std::fill(hflag.begin(), hflag.end(), 0);
                for (int r : freed) {
                    if (next >= feed->total) continue;
                    feed->load(r, next, n);
                    lane_src[r] = next++;
                    lane_it0[r] = it;
                    lane_up0[r] = outer;
                    hflag[r] = 1;
                    refill = true;
                }
                if (refill) {
                    int m = 0;
                    for (int r = 0; r < n; r++)
                        if (hflag[r]) hlane[m++] = r;
                    HIPCHK(hipMemcpyAsync(dflag, hflag.data(), sizeof(int) * n, hipMemcpyHostToDevice, ctx->stream));
                    HIPCHK(hipMemcpyAsync(dlane, hlane.data(), sizeof(int) * m, hipMemcpyHostToDevice, ctx->stream));
                    hipLaunchKernelGGL(k_lane_restart, dim3(1024), dim3(256), 0, ctx->stream, x64, r64, b64, V, n,
                                       dlane, m);
                    norm2<IO64>(w, b64, g64);
                    k_sc_lane_start<<<n, kScalarBlock, 0, ctx->stream>>>(w.part, g64.nb, w.sc, dflag, tol2);
                    pull(w);
                    // a new right-hand side starts the progress measure afresh
                    last_worst = 1e300;
                    stall = 0;
                    for (int r = 0; r < n; r++) again |= hflag[r] && w.h[r].outer_done;
                }
            }
            bool open = false;
            double worst = 0;
            for (auto& s : w.h) {
                open |= !s.outer_done;
                if (s.bb > 0 && !s.outer_done) worst = std::max(worst, std::sqrt(s.rr / s.bb));
            }
            if (trace) {
                fprintf(stderr, "[disco] reliable update %d at iteration %d: worst true rel residual %.3e\n", outer, it,
                        worst);
                // the three lanes furthest from their tolerance, with the state their inner process left
                std::vector<int> ord;
                for (int i = 0; i < w.n; i++)
                    if (!w.h[i].outer_done && w.h[i].bb > 0) ord.push_back(i);
                std::sort(ord.begin(), ord.end(),
                          [&](int a, int b) { return w.h[a].rr / w.h[a].bb > w.h[b].rr / w.h[b].bb; });
                for (size_t q = 0; q < ord.size() && q < 3; q++) {
                    const RhsScal& h = w.h[ord[q]];
                    fprintf(stderr, "[disco]   lane %d: true %.3e inner %.3e of %.3e, active %d reached %d breakdown %d\n",
                            ord[q], std::sqrt(h.rr / h.bb), std::sqrt(h.irr), std::sqrt(h.ibb), h.active, h.reached,
                            h.breakdown);
                }
                for (int i = 0; i < w.n; i++)
                    if (w.h[i].outer_done && !done_at[i])
                        fprintf(stderr, "[disco] lane %d done at iteration %d\n", i, it);
            }
            for (int i = 0; i < w.n; i++)
                if (w.h[i].outer_done && !done_at[i]) done_at[i] = it;
            if (!open) return false;
            if (worst > 0.5 * last_worst) {
                stall++;
            } else {
                stall = 0;
                it_best = it;
            }
            last_worst = std::min(last_worst, worst);
            // no halving of the worst true residual over 8 updates and 800
            // iterations (lanes restart on their own after 100): leave it to
            // the fallback.  The correction is already folded in, and the
            // inner state is not refreshed, so nothing is pending.
            if (stall >= 8 && it - it_best >= 800) {
                gave_up = true;
                return false;
            }
            // the queue is empty and at most half of the lanes are open: they
            // move into a block of half the width (where each launch costs
            // about half), their Krylov processes restarting from the current
            // iterates
            if (feed && next >= feed->total && ctx->opt_narrow && n / 2 >= kNarrowMin) {
                int nopen = 0;
                for (int r = 0; r < n; r++) nopen += lane_src[r] >= 0 && !w.h[r].outer_done;
                if (nopen > 0 && 2 * nopen <= n) {
                    narrowing = true;
                    return false;
                }
            }
            prepare();
            const VecGeo gh = vgeo(Vv, prec, n);
            void* r = ws_get(ctx, "bi_r", nbp);
            void* rh = ws_get(ctx, "bi_rh", nbp);
            void* p = ws_get(ctx, "bi_p", nbp);
            hipLaunchKernelGGL(k_ru_refresh<IO>, dim3(gh.nb), dim3(gh.bd), 0, ctx->stream, r, rhat, p, rh, ee, gh,
                               w.sc, w.part, (unsigned)outer);
            k_sc_ru_refresh<<<n, kScalarBlock, 0, ctx->stream>>>(w.part, gh.nb, w.sc);
            HIPCHK(hipGetLastError());
            return true;
        };
        // a marked lane iterates on until the update, but no further than delta^2
        const int iters = bicg_run<IO>(w, op, prec, rhat, ee, mask, delta, max_iter, check, 0, &refresh, kRuStall,
                                       delta * delta * delta * delta);
        pull(w);
        bool done = true;
        for (auto& s : w.h) done &= s.outer_done != 0;
        if (!done && !gave_up && !narrowing) {
            fold_in();  // the correction since the last update (zero right after one)
            done = true;
            for (auto& s : w.h) done &= s.outer_done != 0;
        }
        if (narrowing && !done) {
            // the open lanes (the correction is folded in, the finished ones are
            // handed over) move into lanes 0..m-1 of a block of half the width
            std::vector<int> keep;
            for (int r = 0; r < n; r++)
                if (lane_src[r] >= 0 && !w.h[r].outer_done) keep.push_back(r);
            const int n2 = n / 2, m = (int)keep.size();
            for (int q = 0; q < m; q++) hlane[q] = keep[q];
            HIPCHK(hipMemcpyAsync(dlane, hlane.data(), sizeof(int) * m, hipMemcpyHostToDevice, ctx->stream));
            const size_t nb2 = disco::native_bytes(ctx, DISCO_F64, n2);
            double2* tmp = (double2*)ws_get(ctx, "ru_narrow", nb2);
            for (double2* v : {x64, b64}) {
                hipLaunchKernelGGL(k_lanes_compact, dim3(1024), dim3(256), 0, ctx->stream, v, tmp, V, n, n2, dlane, m);
                HIPCHK(hipMemcpyAsync(v, tmp, nb2, hipMemcpyDeviceToDevice, ctx->stream));
            }
            HIPCHK(hipStreamSynchronize(ctx->stream));
            ws_free(ctx, "ru_narrow");
            std::vector<int> src2(n2, -1), it2(n2, 0), up2(n2, 0);
            for (int q = 0; q < m; q++) {
                // the iterations and updates so far carry over into the lane's statistics
                src2[q] = lane_src[keep[q]];
                it2[q] = lane_it0[keep[q]] - iters;
                up2[q] = lane_up0[keep[q]] - outer;
            }
            if (trace)
                fprintf(stderr, "[disco] %d open lanes move into a block of %d at iteration %d\n", m, n2, iters);
            n = n2;
            w = make_work(ctx, n);
            g64 = vgeo(V, DISCO_F64, n);
            op.nsb = disco::stencil_nsb(ctx, n, eo);
            lane_src = src2;
            lane_it0 = it2;
            lane_up0 = up2;
            iters_all += iters;
            carry = true;
            carried = m;
            continue;
        }
        int fb = 0;
        int total = iters;
        if (!done && P.fallback) {
            // the FP64 judge has a budget of its own: max_iter caps the inner iterations.
            // Its five FP64 blocks take the place of the inner Krylov vectors, which the
            // next episode allocates again (at 64 lanes of 32^3 x 64 both do not fit).
            fb = 1;
            for (const char* wn : {"bi_r", "bi_rh", "bi_p", "bi_v", "bi_s", "bi_t", "bi_eotmp", "eo_re", "eo_ro",
                                   "eo_uo", "eo_rhat", "eo_ee", "eo_eo", "dc_rin", "dc_e"})
                ws_free(ctx, wn);
            cgnr_correct(w, b64, x64, r64, mask, P.tol, kFallbackIters, check, &total);
            for (const char* wn : {"dc_ecg", "cg_r", "cg_z", "cg_p", "cg_w"}) ws_free(ctx, wn);
            if (feed && next < feed->total) {
                // the inner vectors of the next episode, re-allocated (the pointers may differ)
                rin = ws_get(ctx, "dc_rin", nbp);
                efull = ws_get(ctx, "dc_e", nbp);
                if (eo) {
                    re = ws_get(ctx, "eo_re", hb);
                    ro = ws_get(ctx, "eo_ro", hb);
                    uo = ws_get(ctx, "eo_uo", hb);
                    rhat = ws_get(ctx, "eo_rhat", hb);
                    ee = ws_get(ctx, "eo_ee", hb);
                    eodd = ws_get(ctx, "eo_eo", hb);
                } else {
                    rhat = rin;
                    ee = efull;
                }
            }
        }
        iters_all += total;
        if (feed) {
            hand_over(total, true, fb);
            if (trace && next < feed->total)
                fprintf(stderr, "[disco] block stopped early; %d right-hand sides left start a new process\n",
                        feed->total - next);
            if (next < feed->total) continue;
            break;
        }
        fill_stats(w, P, total, std::max(1, outer), fb, st);
        break;
    }
    if (block_iters) *block_iters = iters_all;
}

// --------------------------------------------------------------- FGMRES
// partial sums of <v_k, w> (k = k0 .. k0+NQ-1 < kn) per right-hand side, FP32 native blocks
template <int NQ>
__global__ void k_mdot32(const float4* __restrict__ basis, long vst, int k0, int kn, const float4* __restrict__ w,
                         VecGeo g, double2* part) {
    double acc[2 * NQ];
#pragma unroll
    for (int q = 0; q < 2 * NQ; q++) acc[q] = 0;
    VEC_LOOP(g) {
        const float4 b = w[i];
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            if (k0 + q < kn) {
                const float4 a = basis[(size_t)(k0 + q) * vst + i];
                acc[2 * q] += (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z + (double)a.w * b.w;
                acc[2 * q + 1] += (double)a.x * b.y - (double)a.y * b.x + (double)a.z * b.w - (double)a.w * b.z;
            }
        }
    }
    rhs_partials<NQ>(acc, g.n, g.bd, part, g.nb, blockIdx.x);
}
template <int NQ>
__global__ void k_fold_dots(const double2* part, int nparts, int k0, int kn, int n, double2* hd) {
    cd q[NQ];
    fold<NQ>(part, blockIdx.x, nparts, q);
    if (threadIdx.x) return;
#pragma unroll
    for (int k = 0; k < NQ; k++)
        if (k0 + k < kn) hd[(size_t)(k0 + k) * n + blockIdx.x] = make_double2(q[k].re, q[k].im);
}
__global__ void k_fold_norm(const double2* part, int nparts, double* nd) {
    cd q[1];
    fold<1>(part, blockIdx.x, nparts, q);
    if (threadIdx.x == 0) nd[blockIdx.x] = q[0].re;
}
// w += sign * sum_{k < kn} c[k][r] basis_k
__global__ void k_maxpy32(const float4* __restrict__ basis, long vst, int kn, const double2* __restrict__ c,
                          float4* __restrict__ w, VecGeo g, float sign) {
    const int r = threadIdx.x % g.n;
    VEC_LOOP(g) {
        float4 acc = w[i];
        for (int k = 0; k < kn; k++) {
            const double2 h = c[(size_t)k * g.n + r];
            const float hr = sign * (float)h.x, hi = sign * (float)h.y;
            const float4 a = basis[(size_t)k * vst + i];
            acc.x = fmaf(hr, a.x, fmaf(-hi, a.y, acc.x));
            acc.y = fmaf(hr, a.y, fmaf(hi, a.x, acc.y));
            acc.z = fmaf(hr, a.z, fmaf(-hi, a.w, acc.z));
            acc.w = fmaf(hr, a.w, fmaf(hi, a.z, acc.w));
        }
        w[i] = acc;
    }
}
// v = w / sqrt(nd[r]) (0 when the norm vanishes)
__global__ void k_scale32(const float4* __restrict__ w, float4* __restrict__ v, VecGeo g, const double* nd) {
    const int r = threadIdx.x % g.n;
    const double q = nd[r];
    const float f = q > 1e-60 ? (float)(1.0 / sqrt(q)) : 0.f;
    VEC_LOOP(g) {
        const float4 a = w[i];
        v[i] = make_float4(f * a.x, f * a.y, f * a.z, f * a.w);
    }
}

// One FGMRES(m) cycle on D e = rin (FP32 native, normalised defect), e = sum_j y_j z_j.
// Returns the number of Arnoldi steps.
static int fgmres_cycle(Work& w, const disco_solver_params& P, const void* rin, void* e, const uint8_t* mask,
                        double inner_tol) {
    disco_ctx* ctx = w.ctx;
    disco_net* net = const_cast<disco_net*>(P.net);
    const int m = P.restart > 0 ? P.restart : 16;
    const int n = w.n;
    VecGeo g = vgeo(w.V, DISCO_F32, n);
    const size_t vb = disco::native_bytes(ctx, DISCO_F32, n);
    const long vst = g.total;  // float4 units per vector
    float4* Vb = (float4*)ws_get(ctx, "fg_V", vb * (m + 1));
    float4* Zb = (float4*)ws_get(ctx, "fg_Z", vb * m);
    float4* wv = (float4*)ws_get(ctx, "fg_w", vb);
    double2* h1 = (double2*)ws_get(ctx, "fg_h1", sizeof(double2) * (m + 1) * n);
    double2* h2 = (double2*)ws_get(ctx, "fg_h2", sizeof(double2) * (m + 1) * n);
    double* nd = (double*)ws_get(ctx, "fg_nd", sizeof(double) * n);
    double2* yd = (double2*)ws_get(ctx, "fg_y", sizeof(double2) * m * n);
    typedef std::complex<double> C;
    // v_0 = rin / |rin|, beta = |rin|
    norm2<IO32>(w, rin, g);
    k_fold_norm<<<n, 256, 0, ctx->stream>>>(w.part, g.nb, nd);
    hipLaunchKernelGGL(k_scale32, dim3(g.nb), dim3(g.bd), 0, ctx->stream, (const float4*)rin, Vb, g, nd);
    std::vector<double> hn(n);
    HIPCHK(hipMemcpyAsync(hn.data(), nd, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::vector<std::vector<C>> R(n, std::vector<C>((size_t)m * m)), gv(n, std::vector<C>(m + 1));
    std::vector<std::vector<double>> cs(n, std::vector<double>(m));
    std::vector<std::vector<C>> sn(n, std::vector<C>(m));
    for (int r = 0; r < n; r++) gv[r][0] = std::sqrt(std::max(hn[r], 0.0));
    std::vector<double2> hh1((size_t)(m + 1) * n), hh2((size_t)(m + 1) * n);
    int steps = 0;
    for (int j = 0; j < m; j++) {
        float4* vj = Vb + (size_t)j * vst;
        float4* zj = Zb + (size_t)j * vst;
        disco::net_apply_native32(net, n, vj, zj);
        stencil(w, DISCO_F32, 0, zj, wv, nullptr, nullptr, mask, disco::EPI_NONE);
        double2* hp[2] = {h1, h2};
        for (int pass = 0; pass < 2; pass++) {
            for (int k0 = 0; k0 <= j; k0 += 4) {
                hipLaunchKernelGGL(k_mdot32<4>, dim3(g.nb), dim3(g.bd), 0, ctx->stream, Vb, vst, k0, j + 1, wv, g,
                                   w.part);
                k_fold_dots<4><<<n, 256, 0, ctx->stream>>>(w.part, g.nb, k0, j + 1, n, hp[pass]);
            }
            hipLaunchKernelGGL(k_maxpy32, dim3(g.nb), dim3(g.bd), 0, ctx->stream, Vb, vst, j + 1, hp[pass], wv, g,
                               -1.0f);
        }
        norm2<IO32>(w, wv, g);
        k_fold_norm<<<n, 256, 0, ctx->stream>>>(w.part, g.nb, nd);
        hipLaunchKernelGGL(k_scale32, dim3(g.nb), dim3(g.bd), 0, ctx->stream, wv, Vb + (size_t)(j + 1) * vst, g, nd);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hh1.data(), h1, sizeof(double2) * (j + 1) * n, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipMemcpyAsync(hh2.data(), h2, sizeof(double2) * (j + 1) * n, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipMemcpyAsync(hn.data(), nd, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        steps++;
        bool all = true;
        for (int r = 0; r < n; r++) {
            std::vector<C> col(j + 2);
            for (int k = 0; k <= j; k++) {
                const double2 a = hh1[(size_t)k * n + r], b = hh2[(size_t)k * n + r];
                col[k] = C(a.x + b.x, a.y + b.y);
            }
            col[j + 1] = std::sqrt(std::max(hn[r], 0.0));
            for (int k = 0; k < j; k++) {  // earlier rotations
                const C t = cs[r][k] * col[k] + sn[r][k] * col[k + 1];
                col[k + 1] = -std::conj(sn[r][k]) * col[k] + cs[r][k] * col[k + 1];
                col[k] = t;
            }
            const C a = col[j], b = col[j + 1];
            const double rr = std::sqrt(std::norm(a) + std::norm(b));
            double c = 1.0;
            C s = 0.0;
            if (rr > 0) {
                const double aa = std::abs(a);
                c = aa / rr;
                s = (aa > 0 ? a / aa : C(1.0)) * std::conj(b) / rr;
            }
            cs[r][j] = c;
            sn[r][j] = s;
            col[j] = c * a + s * b;
            for (int k = 0; k <= j; k++) R[r][(size_t)k * m + j] = col[k];
            gv[r][j + 1] = -std::conj(s) * gv[r][j];
            gv[r][j] = c * gv[r][j];
            const double beta = std::abs(gv[r][0]);
            all &= beta == 0.0 || std::abs(gv[r][j + 1]) <= inner_tol * beta;
        }
        if (all) break;
    }
    // y = R^-1 g (back substitution), e = sum_j y_j z_j
    const int kk = steps;
    std::vector<double2> hy((size_t)m * n);
    for (int r = 0; r < n; r++) {
        std::vector<C> y(kk);
        for (int i = kk - 1; i >= 0; i--) {
            C acc = gv[r][i];
            for (int k = i + 1; k < kk; k++) acc -= R[r][(size_t)i * m + k] * y[k];
            const C d = R[r][(size_t)i * m + i];
            y[i] = std::abs(d) > 0 ? acc / d : C(0.0);
        }
        for (int i = 0; i < kk; i++) hy[(size_t)i * n + r] = make_double2(y[i].real(), y[i].imag());
    }
    HIPCHK(hipMemcpyAsync(yd, hy.data(), sizeof(double2) * kk * n, hipMemcpyHostToDevice, ctx->stream));
    k_zero<IO32><<<1024, 256, 0, ctx->stream>>>(e, g.total);
    hipLaunchKernelGGL(k_maxpy32, dim3(g.nb), dim3(g.bd), 0, ctx->stream, Zb, vst, kk, yd, (float4*)e, g, 1.0f);
    HIPCHK(hipGetLastError());
    return steps;
}

static void fgmres_solve(Work& w, const disco_solver_params& P, const double2* b64, double2* x64, const uint8_t* mask,
                         disco_solver_stats* st) {
    disco_ctx* ctx = w.ctx;
    REQUIRE(P.net != nullptr, DISCO_EINVAL, "FGMRES_NN needs params.net");
    REQUIRE(disco::net_ctx(P.net) == ctx, DISCO_EINVAL, "the network belongs to another context");
    REQUIRE(P.restart >= 0 && P.restart <= 32, DISCO_EINVAL, "restart must be 0..32");
    size_t nb64 = disco::native_bytes(ctx, DISCO_F64, w.n);
    size_t nbp = disco::native_bytes(ctx, DISCO_F32, w.n);
    double2* r64 = (double2*)ws_get(ctx, "dc_r64", nb64);
    void* rin = ws_get(ctx, "dc_rin", nbp);
    void* e = ws_get(ctx, "dc_e", nbp);
    VecGeo g64 = vgeo(w.V, DISCO_F64, w.n);
    const double tol2 = P.tol * P.tol;
    k_zero<IO64><<<1024, 256, 0, ctx->stream>>>(x64, g64.total);
    norm2<IO64>(w, b64, g64);
    k_sc_outer<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, g64.nb, w.sc, 0, tol2);
    copy_scale<IO64, IO64>(w, b64, r64, 0);
    int iters = 0, outer = 0;
    const int max_iter = P.max_iter > 0 ? P.max_iter : 100000;
    const int check = P.check_every > 0 ? P.check_every : 10;
    const double itol = P.inner_tol > 0 ? P.inner_tol : 1e-4;
    const bool trace = getenv("DISCO_TRACE") != nullptr;
    double last_worst = 1e300;
    int stall = 0;
    while (true) {
        pull(w);
        bool done = true;
        double worst = 0;
        for (auto& s : w.h) {
            done &= s.outer_done != 0;
            if (s.bb > 0) worst = std::max(worst, std::sqrt(s.rr / s.bb));
        }
        if (trace)
            fprintf(stderr, "[disco] fgmres outer %d: worst true rel residual %.3e, %d Arnoldi steps\n", outer, worst,
                    iters);
        if (done || iters >= max_iter) break;
        stall = worst > 0.5 * last_worst ? stall + 1 : 0;
        last_worst = worst;
        if (stall >= 3) break;
        outer++;
        copy_scale<IO64, IO32>(w, r64, rin, 1);
        iters += fgmres_cycle(w, P, rin, e, mask, itol);
        dc_update<IO32>(w, x64, e);
        outer_residual(w, b64, x64, r64, mask, tol2);
    }
    int fb = 0;
    pull(w);
    bool done = true;
    for (auto& s : w.h) done &= s.outer_done != 0;
    if (!done && P.fallback) {
        fb = 1;
        cgnr_correct(w, b64, x64, r64, mask, P.tol, std::max(1, max_iter - iters), check, &iters);
    }
    fill_stats(w, P, iters, outer, fb, st);
}

static void cgnr_solve(Work& w, const disco_solver_params& P, const double2* b64, double2* x64, const uint8_t* mask,
                       disco_solver_stats* st) {
    disco_ctx* ctx = w.ctx;
    double2* r64 = (double2*)ws_get(ctx, "dc_r64", disco::native_bytes(ctx, DISCO_F64, w.n));
    VecGeo g64 = vgeo(w.V, DISCO_F64, w.n);
    const double tol2 = P.tol * P.tol;
    const int max_iter = P.max_iter > 0 ? P.max_iter : 100000;
    const int check = P.check_every > 0 ? P.check_every : 10;
    k_zero<IO64><<<1024, 256, 0, ctx->stream>>>(x64, g64.total);
    norm2<IO64>(w, b64, g64);
    k_sc_outer<<<w.n, kScalarBlock, 0, ctx->stream>>>(w.part, g64.nb, w.sc, 0, tol2);
    copy_scale<IO64, IO64>(w, b64, r64, 0);
    int iters = 0, outer = 0;
    // restarted from the true residual until it meets tol (a restart costs one
    // extra FP64 stencil and guards against drift of the recursive residual)
    while (true) {
        pull(w);
        bool done = true;
        for (auto& s : w.h) done &= s.outer_done != 0;
        if (done || iters >= max_iter || outer >= 8) break;
        outer++;
        cgnr_correct(w, b64, x64, r64, mask, P.tol, max_iter - iters, check, &iters);
    }
    fill_stats(w, P, iters, outer, 0, st);
}

}  // namespace

namespace disco {

// Per-block solver state: scalars, partial sums (up to 4 quantities per
// right-hand side: the stencil's four-sum epilogue, FGMRES dots), cleared.

// Every right-hand side of the queue f through a block of (at most) n lanes.
// BICGSTAB_RU keeps the lanes busy: a converged lane takes the next right-hand
// side at the update that finds it converged.  The other methods solve the
// queue block by block.  st (host) receives f.total entries; returns the
// inner iterations the block ran.
long long solve_fed(disco_ctx* ctx, const disco_domains* dom, const disco_solver_params& P, int n, LaneFeeder& f,
                    double2* b64, double2* x64, disco_solver_stats* st) {
    if (f.total <= 0) return 0;
    n = std::min(n, f.total);
    const uint8_t* mask = dom ? dom->d_mask : nullptr;
    if (P.method == DISCO_BICGSTAB_RU && (P.inner_prec == DISCO_F32 || P.inner_prec == DISCO_BF16)) {
        Work w = make_work(ctx, n);
        long long it = 0;
        if (P.inner_prec == DISCO_F32)
            ru_solve<IO32>(w, P, DISCO_F32, b64, x64, mask, st, &f, &it);
        else
            ru_solve<IOBF>(w, P, DISCO_BF16, b64, x64, mask, st, &f, &it);
        return it;
    }
    long long it = 0;
    std::vector<disco_solver_stats> bst(n);
    for (int j0 = 0; j0 < f.total; j0 += n) {
        const int m = std::min(n, f.total - j0);
        std::vector<int> lanes(m), js(m);
        for (int r = 0; r < m; r++) {
            f.load(r, j0 + r, m);
            lanes[r] = r;
            js[r] = j0 + r;
        }
        solve_native(ctx, dom, P, m, b64, x64, bst.data());
        for (int r = 0; r < m; r++) st[j0 + r] = bst[r];
        it += bst[0].iters;
        f.store(lanes, js, m);
    }
    return it;
}

// Solve on native FP64 blocks b64 -> x64 (n right-hand sides).
void solve_native(disco_ctx* ctx, const disco_domains* dom, const disco_solver_params& P, int n, const double2* b64,
                  double2* x64, disco_solver_stats* st) {
    Work w = make_work(ctx, n);
    const uint8_t* mask = dom ? dom->d_mask : nullptr;
    if (P.method == DISCO_CGNR_F64) {
        cgnr_solve(w, P, b64, x64, mask, st);
    } else if (P.method == DISCO_BICGSTAB_DC) {
        if (P.inner_prec == DISCO_F32)
            dc_solve<IO32>(w, P, DISCO_F32, b64, x64, mask, st);
        else if (P.inner_prec == DISCO_BF16)
            dc_solve<IOBF>(w, P, DISCO_BF16, b64, x64, mask, st);
        else if (P.inner_prec == DISCO_F64)
            dc_solve<IO64>(w, P, DISCO_F64, b64, x64, mask, st);
        else
            disco_throw(DISCO_EINVAL, "bad inner precision %d", P.inner_prec);
    } else if (P.method == DISCO_FGMRES_NN) {
        fgmres_solve(w, P, b64, x64, mask, st);
    } else if (P.method == DISCO_BICGSTAB_RU) {
        if (P.inner_prec == DISCO_F32)
            ru_solve<IO32>(w, P, DISCO_F32, const_cast<double2*>(b64), x64, mask, st);
        else if (P.inner_prec == DISCO_BF16)
            ru_solve<IOBF>(w, P, DISCO_BF16, const_cast<double2*>(b64), x64, mask, st);
        else
            disco_throw(DISCO_EINVAL, "reliable updates need FP32 or BF16 inner precision, not %d", P.inner_prec);
    } else {
        disco_throw(DISCO_EINVAL, "unknown solver method %d", P.method);
    }
}

int default_rhs_block(const disco_solver_params& P, int nrhs, const disco_ctx* ctx) {
    int b = P.rhs_block;
    if (b <= 0 && ctx && (P.method == DISCO_BICGSTAB_DC || P.method == DISCO_BICGSTAB_RU) && P.inner_prec >= 0 &&
        P.inner_prec <= 2) {
        b = ctx->tuned_block[P.inner_prec];
        // fixed blocks (defect correction) run until their slowest member is
        // done; beyond 32 lanes that idle time outweighs the cheaper iterations
        if (P.method == DISCO_BICGSTAB_DC) b = std::min(b, 32);
    }
    if (b <= 0) b = 16;
    return std::max(1, std::min({b, nrhs, 64, max_rhs_block(ctx)}));
}

// Largest solver block: 64, and no more than the stencil's plane limit.
int max_rhs_block(const disco_ctx* ctx) { return ctx ? std::min(64, plane_rhs_limit(ctx)) : 64; }

}  // namespace disco

namespace {
__global__ void k_rand_spinor(double2* b, long n, unsigned long long seed) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        unsigned long long z = seed + 0x9e3779b97f4a7c15ULL * (unsigned long long)(i + 1);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z ^= z >> 31;
        b[i] = make_double2((double)(z >> 40) / 16777216.0 - 0.5, (double)(z & 0xffffff) / 16777216.0 - 0.5);
    }
}
}  // namespace

extern "C" int disco_autotune(disco_ctx* ctx, const disco_domains* dom, int inner_prec, int* best, double* cost_us) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(inner_prec == DISCO_F32 || inner_prec == DISCO_BF16, DISCO_EINVAL, "tune FP32 or BF16 storage");
        REQUIRE(ctx->have_clover, DISCO_ESTATE, "autotune before clover_setup");
        REQUIRE(!dom || dom->ctx == ctx, DISCO_EINVAL, "domains belong to another context");
        activate(ctx);
        const int cand[4] = {8, 16, 32, 64};
        const int iters = 20;
        double cost[4] = {0, 0, 0, 0};
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        const uint8_t* mask = dom ? dom->d_mask : nullptr;
        // microseconds per right-hand side and inner iteration of a block of n
        // (one untimed pass for graph capture and caches, then the best of reps)
        auto time_block = [&](int n, int reps) {
            Work w;
            w.ctx = ctx;
            w.n = n;
            w.V = ctx->V;
            w.nsb = disco::stencil_nsb(ctx, n);
            w.sc = (RhsScal*)ws_get(ctx, "sv_scal", sizeof(RhsScal) * n);
            VecGeo g = vgeo(ctx->V, DISCO_F64, n);
            w.part = (double2*)ws_get(ctx, "sv_part", sizeof(double2) * (size_t)std::max(w.nsb, g.nb) * 4 * n);
            HIPCHK(hipMemsetAsync(w.sc, 0, sizeof(RhsScal) * n, ctx->stream));
            double2* b64 = (double2*)ws_get(ctx, "tune_b", disco::native_bytes(ctx, DISCO_F64, n));
            void* rin = ws_get(ctx, "dc_rin", disco::native_bytes(ctx, inner_prec, n));
            void* e = ws_get(ctx, "dc_e", disco::native_bytes(ctx, inner_prec, n));
            k_rand_spinor<<<2048, 256, 0, ctx->stream>>>(b64, ctx->V * 12L * n, 0x7157ULL + n);
            if (inner_prec == DISCO_F32) copy_scale<IO64, IO32>(w, b64, rin, 0);
            else copy_scale<IO64, IOBF>(w, b64, rin, 0);
            double best_ms = 1e300;
            for (int rep = 0; rep <= reps; rep++) {
                HIPCHK(hipEventRecord(e0, ctx->stream));
                const bool eo = ctx->opt_eo && disco::eo_supported(ctx);
                if (inner_prec == DISCO_F32) {
                    if (eo) bicg_run_eo<IO32>(w, DISCO_F32, rin, e, mask, 0.0, iters, 10);
                    else bicg_run<IO32>(w, InnerOp{false, w.V, w.nsb}, DISCO_F32, rin, e, mask, 0.0, iters, 10);
                } else {
                    if (eo) bicg_run_eo<IOBF>(w, DISCO_BF16, rin, e, mask, 0.0, iters, 10);
                    else bicg_run<IOBF>(w, InnerOp{false, w.V, w.nsb}, DISCO_BF16, rin, e, mask, 0.0, iters, 10);
                }
                HIPCHK(hipEventRecord(e1, ctx->stream));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0) best_ms = std::min(best_ms, (double)ms);
            }
            return 1e3 * best_ms / (double)(n * iters);
        };
        for (int c = 0; c < 4; c++)
            if (cand[c] <= disco::max_rhs_block(ctx)) cost[c] = time_block(cand[c], 1);
        int bi = 0;
        for (int c = 1; c < 4; c++)
            if (cost[c] > 0 && cost[c] < cost[bi]) bi = c;
        ctx->tuned_block[inner_prec] = cand[bi];
        // then the tile of the site order at that block: a few y-row and
        // timeslice extents around the default, kept when faster
        if (ctx->trav_kind == 1) {
            const int Lx = ctx->dims[0], Ly = ctx->dims[1], Lt = ctx->dims[3];
            const int tc = Lt % 8 == 0 ? Lt / 8 : Lt;
            const int ty0 = ctx->tile_y, tt0 = ctx->tile_t;
            double best_cost = time_block(cand[bi], 2);
            int by = ty0, bt = tt0;
            const int ys[6] = {1, 2, 3, 4, 6, 8};
            const int ts[2] = {tc, tc / 2};
            for (int yt : ys) {
                if (Ly % yt) continue;
                for (int k = 0; k < 2; k++) {
                    const int tt = ts[k];
                    if (tt < 1 || tc % tt || (k == 1 && tt == tc) || (long)Lx * yt * tt > 1024) continue;
                    ctx->tile_y = yt;
                    ctx->tile_t = tt;
                    disco::build_traversal(ctx);
                    const double c = time_block(cand[bi], 2);
                    // a tile replaces the best so far only when clearly faster
                    // (repeated timings of one tile spread by about 1%)
                    if (c < 0.99 * best_cost) {
                        best_cost = c;
                        by = yt;
                        bt = tt;
                    }
                }
            }
            ctx->tile_y = by;
            ctx->tile_t = bt;
            disco::build_traversal(ctx);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (best) *best = cand[bi];
        if (cost_us)
            for (int c = 0; c < 4; c++) cost_us[c] = cost[c];
    });
}

extern "C" int disco_solve_multi_rhs(disco_ctx* ctx, const disco_domains* dom, const disco_solver_params* p, int nrhs,
                                     const void* b, void* x, disco_solver_stats* stats) {
    if (!ctx) return DISCO_EINVAL;
    bool all_ok = true;
    int rc = guarded(ctx, [&] {
        REQUIRE(p && (nrhs == 0 || (b && x)), DISCO_EINVAL, "NULL argument");
        REQUIRE(nrhs >= 0, DISCO_EINVAL, "nrhs < 0");
        REQUIRE(p->tol > 0, DISCO_EINVAL, "tol must be > 0");
        REQUIRE(!dom || dom->ctx == ctx, DISCO_EINVAL, "domains belong to another context");
        REQUIRE(ctx->have_clover, DISCO_ESTATE, "solve before clover_setup");
        activate(ctx);
        if (nrhs == 0) return;
        const int blk = disco::default_rhs_block(*p, nrhs, ctx);
        const long V = ctx->V;
        const size_t nb64 = disco::native_bytes(ctx, DISCO_F64, blk);
        double2* b64 = (double2*)ws_get(ctx, "solve_b64", nb64);
        double2* x64 = (double2*)ws_get(ctx, "solve_x64", nb64);
        const double2* bc = (const double2*)b;
        double2* xc = (double2*)x;
        disco::LaneFeeder f;
        f.total = nrhs;
        f.load = [&](int lane, int j, int width) {
            hipLaunchKernelGGL(k_lane_in, dim3(site_grid(V, 12)), dim3(256), 0, ctx->stream, bc + (size_t)j * 12 * V,
                               b64, V, width, lane);
        };
        f.store = [&](const std::vector<int>& lanes, const std::vector<int>& js, int width) {
            for (size_t q = 0; q < lanes.size(); q++)
                hipLaunchKernelGGL(k_lane_out, dim3(site_grid(V, 12)), dim3(256), 0, ctx->stream, x64,
                                   xc + (size_t)js[q] * 12 * V, V, width, lanes[q]);
        };
        std::vector<disco_solver_stats> st(nrhs);
        disco::solve_fed(ctx, dom, *p, blk, f, b64, x64, st.data());
        for (int i = 0; i < nrhs; i++) {
            if (stats) stats[i] = st[i];
            all_ok &= st[i].converged != 0;
        }
        HIPCHK(hipStreamSynchronize(ctx->stream));
    });
    if (rc == DISCO_OK && !all_ok) {
        ctx->err = "solver did not reach the tolerance for every right-hand side";
        return DISCO_ENOCONV;
    }
    return rc;
}

// ----------------------------------------------------------------- even-odd pieces at the boundary
namespace {
// the NQ fused sums of right-hand side blockIdx.x into out[r][4] at slots s0..s3
template <int NQ>
__global__ void k_fold_epi(const double2* part, int nparts, int s0, int s1, int s2, int s3, double2* out) {
    cd q[NQ];
    fold<NQ>(part, blockIdx.x, nparts, q);
    if (threadIdx.x) return;
    const int slot[4] = {s0, s1, s2, s3};
#pragma unroll
    for (int k = 0; k < NQ; k++) out[(long)blockIdx.x * 4 + slot[k]] = make_double2(q[k].re, q[k].im);
}

template <class IO>
void eo_boundary(disco_ctx* ctx, const disco_domains* dom, int prec, int p, int n, double ca, double cg, double cb,
                 int epi, const void* in, const void* aux, const void* aux2, void* out, double* sums) {
    const long V = ctx->V;
    const int Lx = ctx->dims[0], Ly = ctx->dims[1], Lz = ctx->dims[2];
    const size_t full = disco::native_bytes(ctx, prec, n), half = full / 2;
    void* tmp = ws_get(ctx, "eoa_full", full);
    void* hin[2] = {ws_get(ctx, "eoa_in0", half), ws_get(ctx, "eoa_in1", half)};
    void* haux[2] = {ws_get(ctx, "eoa_aux0", half), ws_get(ctx, "eoa_aux1", half)};
    void* haux2[2] = {ws_get(ctx, "eoa_aux20", half), ws_get(ctx, "eoa_aux21", half)};
    void* hout = ws_get(ctx, "eoa_out", half);
    void* hzero = ws_get(ctx, "eoa_zero", half);
    const int grid = site_grid(V, n);
    auto split = [&](const void* src, void* h[2]) {
        disco::to_native(ctx, prec, n, src, tmp);
        hipLaunchKernelGGL(k_eo_split<IO>, dim3(grid), dim3(256), 0, ctx->stream, tmp, h[0], h[1], V, n, Lx, Ly, Lz);
    };
    split(in, hin);
    if (aux) split(aux, haux);
    if (aux2) split(aux2, haux2);
    const int nq = disco::nq_of(epi);
    const int nsb = disco::stencil_nsb(ctx, n, true);
    double2* part = nq ? (double2*)ws_get(ctx, "eoa_part", sizeof(double2) * (size_t)nsb * nq * n) : nullptr;
    disco::StencilCall c{prec, 0, n, hin[1 - p], hout, aux ? haux[p] : nullptr, aux2 ? haux2[p] : nullptr,
                         dom ? dom->d_mask : nullptr, part, epi, p, ca, cg, cb};
    disco::stencil_launch(ctx, c);
    const VecGeo gh = vgeo(V / 2, prec, n);
    k_zero<IO><<<1024, 256, 0, ctx->stream>>>(hzero, gh.total);
    hipLaunchKernelGGL(k_eo_merge<IO>, dim3(grid), dim3(256), 0, ctx->stream, p == 0 ? hout : hzero,
                       p == 1 ? hout : hzero, tmp, V, n, Lx, Ly, Lz);
    disco::from_native(ctx, prec, n, tmp, out);
    if (nq) {
        double2* d = (double2*)ws_get(ctx, "eoa_sums", sizeof(double2) * 4 * n);
        HIPCHK(hipMemsetAsync(d, 0, sizeof(double2) * 4 * n, ctx->stream));
        int slot[4] = {0, 0, 0, 0}, k = 0;
        const int bits[4] = {disco::EPI_DOTAUX, disco::EPI_NORM, disco::EPI_DOTIN, disco::EPI_DOTAUXIN};
        for (int b = 0; b < 4; b++)
            if (epi & bits[b]) slot[k++] = b;
        if (nq == 1) k_fold_epi<1><<<n, kScalarBlock, 0, ctx->stream>>>(part, nsb, slot[0], 0, 0, 0, d);
        else if (nq == 2) k_fold_epi<2><<<n, kScalarBlock, 0, ctx->stream>>>(part, nsb, slot[0], slot[1], 0, 0, d);
        else k_fold_epi<4><<<n, kScalarBlock, 0, ctx->stream>>>(part, nsb, slot[0], slot[1], slot[2], slot[3], d);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(sums, d, sizeof(double2) * 4 * n, hipMemcpyDeviceToHost, ctx->stream));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
}
}  // namespace

extern "C" int disco_dirac_eo_apply(disco_ctx* ctx, const disco_domains* dom, int prec, int parity, int nrhs,
                                    double ca, double cg, double cb, int epi, const void* in, const void* aux,
                                    const void* aux2, void* out, double* sums) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        using namespace disco;
        REQUIRE(in && out, DISCO_EINVAL, "NULL spinor");
        REQUIRE(prec >= 0 && prec <= 2, DISCO_EINVAL, "bad precision %d", prec);
        REQUIRE(parity == 0 || parity == 1, DISCO_EINVAL, "parity is 0 or 1");
        REQUIRE(!dom || dom->ctx == ctx, DISCO_EINVAL, "domains belong to another context");
        REQUIRE(ctx->have_clover, DISCO_ESTATE, "operator applied before clover_setup");
        REQUIRE(eo_supported(ctx), DISCO_EINVAL, "even-odd pieces need even extents");
        REQUIRE(nrhs >= 1 && nrhs <= max_rhs_block(ctx), DISCO_EINVAL, "nrhs must be in 1..%d", max_rhs_block(ctx));
        const int all4 = EPI_DOTAUX | EPI_NORM | EPI_DOTIN | EPI_DOTAUXIN;
        REQUIRE(epi == 0 || epi == EPI_DOTAUX || epi == (EPI_NORM | EPI_DOTIN) || epi == all4, DISCO_EINVAL,
                "epilogue %d is not one the solver launches", epi);
        const bool need_aux = ca != 0.0 || cg != 0.0 || (epi & (EPI_DOTIN | EPI_DOTAUXIN));
        REQUIRE(!need_aux || aux, DISCO_EINVAL, "aux is needed for ca, cg or the sums with it");
        REQUIRE(!(epi & (EPI_DOTAUX | EPI_DOTAUXIN)) || aux2, DISCO_EINVAL, "aux2 is needed for its sums");
        REQUIRE(!epi || sums, DISCO_EINVAL, "sums is NULL");
        REQUIRE(out != in && out != aux && out != aux2, DISCO_EINVAL, "out must not alias an input");
        activate(ctx);
        const void* a1 = need_aux ? aux : nullptr;
        const void* a2 = (epi & (EPI_DOTAUX | EPI_DOTAUXIN)) ? aux2 : nullptr;
        if (prec == DISCO_F64)
            eo_boundary<IO64>(ctx, dom, prec, parity, nrhs, ca, cg, cb, epi, in, a1, a2, out, sums);
        else if (prec == DISCO_F32)
            eo_boundary<IO32>(ctx, dom, prec, parity, nrhs, ca, cg, cb, epi, in, a1, a2, out, sums);
        else
            eo_boundary<IOBF>(ctx, dom, prec, parity, nrhs, ca, cg, cb, epi, in, a1, a2, out, sums);
    });
}
