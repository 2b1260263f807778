// Wilson-clover stencil D and its domain-restricted form D_Lambda on native
// multi-RHS spinor blocks, plus the canonical <-> native layout kernels.
//
// One lane owns one (site, right-hand side) pair, right-hand side fastest, so
// the n lanes of a site sit side by side in a wavefront: spinor planes are
// read with fully coalesced 16-byte-per-lane accesses and each link and
// clover entry is fetched once per site and broadcast to its n lanes.  The
// eight hops use the half-spinor form: (1 -/+ gamma_mu) has rank 2, so the
// neighbour spinor is projected to two spin components, multiplied by the
// link, and expanded again.  With a domain mask, a hop across a cut face is
// skipped and the clover term is kept (D_Lambda is D restricted to the fields
// inside each domain).  The optional epilogue fuses the Krylov reductions
// (deterministic per-block partial sums in FP64).
//
// Even-odd mode (EO): the launch visits the sites of one parity only, reads
// the other parity's half-lattice vector (site s at index s/2), and forms
//   out = ca * aux + A(x)^-1 (cg * aux + cb * H in)
// with H the hopping sum (D = A - kappa H).  With the right coefficients this
// is every piece of the Schur complement on the even sites,
//   M = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe,
// its source A_ee^-1 (r_e + kappa H_eo A_oo^-1 r_o) and the reconstruction
// x_o = A_oo^-1 (r_o + kappa H_oe x_e).
#include <algorithm>
#include <cstdlib>
#include <string>
#include <vector>

#include "spinor_io.h"

namespace {

constexpr int kStencilBlock = kMaxBlock;

struct StencilArgs {
    RoView in;
    void* out;
    RoView aux;   // b of out = b - D in
    RoView aux2;  // w of <w, out>
    const void* U;
    const void* A;
    const uint8_t* mask;
    const int2* trav;
    double2* part;
    long V;        // lattice sites (stride of the link and clover planes)
    long Vv;       // sites of the spinor vectors (V, or V/2 in even-odd mode)
    int nsites;    // sites visited by the launch (entries of trav)
    int eo_aux;    // even-odd mode: read aux at the site (ca, cg, DOTIN or DOTAUXIN need it)
    double ca, cg, cb;
    int L[4];
    long st[4];
    double ph[4];
    double kappa;
    int nsb;   // site blocks (= partial-sum slots per rhs and quantity)
    int spb;   // sites per block
    int n;     // right-hand sides in the block
    int dagger;
    int stage; // LDS staging requested (applies to FP32 links with at most kStageSites sites per block)
    unsigned allhops;  // 0xff: the hop word of the unmasked instance (an argument, not a constant, so
                       // that the hops stay separate blocks and the compiler does not hoist all loads)
};

// ---- spin projection (1 - gamma_mu) [FWD] or (1 + gamma_mu) [BWD], chiral basis
template <int MU, bool FWD, typename T>
__device__ __forceinline__ void project(const cx<T> p[12], cx<T> h[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cx<T> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        if (MU == 0) {
            h[c] = FWD ? p0 + ti(p3) : p0 - ti(p3);
            h[3 + c] = FWD ? p1 + ti(p2) : p1 - ti(p2);
        } else if (MU == 1) {
            h[c] = FWD ? p0 + p3 : p0 - p3;
            h[3 + c] = FWD ? p1 - p2 : p1 + p2;
        } else if (MU == 2) {
            h[c] = FWD ? p0 + ti(p2) : p0 - ti(p2);
            h[3 + c] = FWD ? p1 - ti(p3) : p1 + ti(p3);
        } else {
            h[c] = FWD ? p0 - p2 : p0 + p2;
            h[3 + c] = FWD ? p1 - p3 : p1 + p3;
        }
    }
}

// acc += expansion of the projected, link-multiplied half spinor u
template <int MU, bool FWD, typename T>
__device__ __forceinline__ void expand(cx<T> acc[12], const cx<T> u[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        cx<T> u0 = u[c], u1 = u[3 + c];
        acc[c] = acc[c] + u0;
        acc[3 + c] = acc[3 + c] + u1;
        if (MU == 0) {
            acc[6 + c] = FWD ? acc[6 + c] - ti(u1) : acc[6 + c] + ti(u1);
            acc[9 + c] = FWD ? acc[9 + c] - ti(u0) : acc[9 + c] + ti(u0);
        } else if (MU == 1) {
            acc[6 + c] = FWD ? acc[6 + c] - u1 : acc[6 + c] + u1;
            acc[9 + c] = FWD ? acc[9 + c] + u0 : acc[9 + c] - u0;
        } else if (MU == 2) {
            acc[6 + c] = FWD ? acc[6 + c] - ti(u0) : acc[6 + c] + ti(u0);
            acc[9 + c] = FWD ? acc[9 + c] + ti(u1) : acc[9 + c] - ti(u1);
        } else {
            acc[6 + c] = FWD ? acc[6 + c] - u0 : acc[6 + c] + u0;
            acc[9 + c] = FWD ? acc[9 + c] - u1 : acc[9 + c] + u1;
        }
    }
}

// acc += a * b and acc += conj(a) * b as explicit fused multiply-add chains
// (four FMAs per complex product; the compiler may not reassociate)
template <typename T>
__device__ __forceinline__ void cmac(cx<T>& acc, cx<T> a, cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
template <typename T>
__device__ __forceinline__ void cjmac(cx<T>& acc, cx<T> a, cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}

template <typename T>
__device__ __forceinline__ void su3_mul(const cx<T> u[9], const cx<T> h[6], cx<T> o[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; sp++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<T> acc = mk((T)0, (T)0);
            cmac(acc, u[a * 3 + 0], h[sp * 3 + 0]);
            cmac(acc, u[a * 3 + 1], h[sp * 3 + 1]);
            cmac(acc, u[a * 3 + 2], h[sp * 3 + 2]);
            o[sp * 3 + a] = acc;
        }
}

template <typename T>
__device__ __forceinline__ void su3_dag_mul(const cx<T> u[9], const cx<T> h[6], cx<T> o[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; sp++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<T> acc = mk((T)0, (T)0);
            cjmac(acc, u[0 * 3 + a], h[sp * 3 + 0]);
            cjmac(acc, u[1 * 3 + a], h[sp * 3 + 1]);
            cjmac(acc, u[2 * 3 + a], h[sp * 3 + 2]);
            o[sp * 3 + a] = acc;
        }
}

template <typename T>
__device__ __forceinline__ void g5(cx<T> p[12]) {
#pragma unroll
    for (int k = 6; k < 12; k++) p[k] = neg(p[k]);
}

template <typename T>
__device__ __forceinline__ void clover6(const T f[36], const cx<T>* x, cx<T>* y) {
#pragma unroll
    for (int i = 0; i < 6; i++) y[i] = f[i] * x[i];
    int m = 0;
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = i + 1; j < 6; j++, m++) {
            const cx<T> a = mk(f[6 + 2 * m], f[7 + 2 * m]);
            cmac(y[i], a, x[j]);
            cjmac(y[j], a, x[i]);
        }
}

// both hops in direction MU for right-hand side r at site s
template <class IO, bool BUF, bool STAGE, bool EO, int MU>
__device__ __forceinline__ void hops(const StencilArgs& a, int s, const int* x, uint32_t m, int n, int r,
                                     const float2* sl, cx<typename IO::T> acc[12]) {
    typedef typename IO::T T;
    const typename IO::LinkT* U = (const typename IO::LinkT*)a.U;
    const long V = a.V;
    const long Vv = a.Vv;
    const int L = a.L[MU];
    const int st = (int)a.st[MU];
    if (m & (1u << (2 * MU))) {
        // forward: (1 - gamma_mu) U_mu(x) psi(x+mu), boundary phase at the wrap
        const bool wrap = x[MU] == L - 1;
        const int nb = wrap ? s - (L - 1) * st : s + st;
        cx<T> u[9], p[12], h[6], o[6];
        IO::template loadv<BUF>(a.in, Vv, n, r, EO ? (nb >> 1) : nb, p);
        if constexpr (STAGE) {
#pragma unroll
            for (int k = 0; k < 9; k++) u[k] = mk((T)sl[(2 * MU) * 9 + k].x, (T)sl[(2 * MU) * 9 + k].y);
        } else {
            IO::load_link(U, V, MU, s, u);
        }
        if (a.dagger) g5(p);
        project<MU, true>(p, h);
        if (wrap) {
            const T ph = (T)a.ph[MU];
#pragma unroll
            for (int k = 0; k < 6; k++) h[k] = ph * h[k];
        }
        su3_mul(u, h, o);
        expand<MU, true>(acc, o);
    }
    if (m & (2u << (2 * MU))) {
        // backward: (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu)
        const bool wrap = x[MU] == 0;
        const int nb = wrap ? s + (L - 1) * st : s - st;
        cx<T> u[9], p[12], h[6], o[6];
        IO::template loadv<BUF>(a.in, Vv, n, r, EO ? (nb >> 1) : nb, p);
        if constexpr (STAGE) {
#pragma unroll
            for (int k = 0; k < 9; k++) u[k] = mk((T)sl[(2 * MU + 1) * 9 + k].x, (T)sl[(2 * MU + 1) * 9 + k].y);
        } else {
            IO::load_link(U, V, MU, nb, u);
        }
        if (a.dagger) g5(p);
        project<MU, false>(p, h);
        if (wrap) {
            const T ph = (T)a.ph[MU];
#pragma unroll
            for (int k = 0; k < 6; k++) h[k] = ph * h[k];
        }
        su3_dag_mul(u, h, o);
        expand<MU, false>(acc, o);
    }
}

template <int EPI>
struct EpiCount {
    static constexpr int nq = ((EPI & disco::EPI_DOTAUX) ? 1 : 0) + ((EPI & disco::EPI_NORM) ? 1 : 0) +
                              ((EPI & disco::EPI_DOTIN) ? 1 : 0) + ((EPI & disco::EPI_DOTAUXIN) ? 1 : 0);
};

// With STAGE (FP32 links and clover, at most kStageSites sites per block) the
// block first copies the eight links of each of its sites (U_mu(x) and
// U_mu(x-mu)) and their clover blocks into LDS with all lanes cooperating;
// the n lanes of a site then read them from LDS instead of each issuing the
// same global loads.
constexpr int kStageSites = 32;
constexpr int kStageLinkBytes = 8 * 9 * 8;   // 8 links x 9 complex float
constexpr int kStageCloverBytes = 18 * 16;   // 2 blocks x 9 float4

// MASK = false: the full operator (every hop present, no mask load; the hop
// tests are uniform).  MASK = true: hops removed where the domain mask says so.
// Blocks per CU the compiler must fit: six (six waves per SIMD, at most 80
// VGPRs) for the hot BF16 even-odd instances with buffer loads and staged
// links, which fit without spilling; no constraint for the others.
template <class IO, bool BUF, bool STAGE, bool EO>
struct MinBlocks {
    static constexpr int v = (EO && BUF && STAGE && sizeof(typename IO::T) == 4 && IO::planes == 3) ? 6 : 1;
};
template <class IO, int EPI, bool BUF, bool STAGE, bool EO, bool MASK>
__global__ __launch_bounds__(kStencilBlock, (MinBlocks<IO, BUF, STAGE, EO>::v)) void k_dslash(const StencilArgs a) {
    typedef typename IO::T T;
    constexpr int NQ = EpiCount<EPI>::nq;
    const int n = a.n;
    const long Vv = a.Vv;
    const int spb = a.spb;  // sites per block; the block has spb*n active lanes
    const int sb = xcd_block(a.nsb);
    if (sb < 0) return;
    const int t = threadIdx.x;
    const int nact = spb * n;
    const int g = sb * spb + t / n;
    const int r = t % n;
    const long V = a.V;
    double red[NQ > 0 ? 2 * NQ : 1];
#pragma unroll
    for (int k = 0; k < (NQ > 0 ? 2 * NQ : 1); k++) red[k] = 0;
    extern __shared__ __align__(16) unsigned char stage_mem[];
    const float2* sl = nullptr;
    const float4* sa = nullptr;
    if constexpr (STAGE) {
        float2* sU = (float2*)stage_mem;
        float4* sA = (float4*)(stage_mem + spb * kStageLinkBytes);
        const float2* U = (const float2*)a.U;
        const float4* A = (const float4*)a.A;
        const int g0 = sb * spb;
        for (int e = t; e < spb * 72; e += kStencilBlock) {
            const int i = e / 72, rem = e - i * 72, d = rem / 9, k = rem - d * 9;
            const int gi = g0 + i;
            float2 v = make_float2(0.f, 0.f);
            if (gi < a.nsites) {
                const int2 tr = a.trav[gi];
                const int mu = d >> 1;
                int site = tr.x;
                if (d & 1) {
                    const int xm = (tr.y >> (8 * mu)) & 0xff;
                    site = xm == 0 ? site + (a.L[mu] - 1) * (int)a.st[mu] : site - (int)a.st[mu];
                }
                v = U[((long)mu * 9 + k) * V + site];
            }
            sU[i * 72 + d * 9 + k] = v;
        }
        for (int e = t; e < spb * 18; e += kStencilBlock) {
            const int i = e / 18, q = e - i * 18;
            const int gi = g0 + i;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gi < a.nsites) v = A[((long)(q / 9) * 9 + (q % 9)) * V + a.trav[gi].x];
            sA[i * 18 + q] = v;
        }
        __syncthreads();
        sl = sU + (t / n) * 72;
        sa = sA + (t / n) * 18;
    }

    if (t < nact && g < a.nsites) {
        const int2 tr = a.trav[g];
        const int s = tr.x;
        const int x[4] = {tr.y & 0xff, (tr.y >> 8) & 0xff, (tr.y >> 16) & 0xff, (tr.y >> 24) & 0xff};
        const uint32_t m = (MASK && a.mask) ? (uint32_t)a.mask[s] : a.allhops;
        cx<T> acc[12];
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = mk((T)0, (T)0);
        hops<IO, BUF, STAGE, EO, 0>(a, s, x, m, n, r, sl, acc);
        hops<IO, BUF, STAGE, EO, 1>(a, s, x, m, n, r, sl, acc);
        hops<IO, BUF, STAGE, EO, 2>(a, s, x, m, n, r, sl, acc);
        hops<IO, BUF, STAGE, EO, 3>(a, s, x, m, n, r, sl, acc);

        // site-local part: A(x) psi(x) - kappa * hops, or in even-odd mode
        // ca * aux + A(x)^-1 (cg * aux + cb * hops)
        const int sv = EO ? (s >> 1) : s;
        cx<T> p[12], o[12];
        cx<T> pin[12];
        if constexpr (EO) {
            if (a.eo_aux) {
                IO::template loadv<BUF>(a.aux, Vv, n, r, sv, pin);
            } else {
#pragma unroll
                for (int k = 0; k < 12; k++) pin[k] = mk((T)0, (T)0);
            }
            const T cg = (T)a.cg, cb = (T)a.cb;
#pragma unroll
            for (int k = 0; k < 12; k++) p[k] = mk(fma(cb, acc[k].re, cg * pin[k].re), fma(cb, acc[k].im, cg * pin[k].im));
        } else {
            IO::template loadv<BUF>(a.in, Vv, n, r, sv, p);
            if (EPI & (disco::EPI_DOTIN | disco::EPI_DOTAUXIN)) {
#pragma unroll
                for (int k = 0; k < 12; k++) pin[k] = p[k];
            }
            if (a.dagger) g5(p);
        }
        {
            T f[36];
            if constexpr (STAGE) {
#pragma unroll
                for (int b = 0; b < 2; b++) {
#pragma unroll
                    for (int q = 0; q < 9; q++) {
                        const float4 v = sa[b * 9 + q];
                        f[4 * q] = v.x;
                        f[4 * q + 1] = v.y;
                        f[4 * q + 2] = v.z;
                        f[4 * q + 3] = v.w;
                    }
                    clover6(f, p + 6 * b, o + 6 * b);
                }
            } else {
                IO::load_clover((const typename IO::CloverT*)a.A, V, 0, s, f);
                clover6(f, p, o);
                IO::load_clover((const typename IO::CloverT*)a.A, V, 1, s, f);
                clover6(f, p + 6, o + 6);
            }
        }
        if constexpr (EO) {
            const T ca = (T)a.ca;
#pragma unroll
            for (int k = 0; k < 12; k++) o[k] = mk(fma(ca, pin[k].re, o[k].re), fma(ca, pin[k].im, o[k].im));
        } else {
            const T kap = (T)a.kappa;
#pragma unroll
            for (int k = 0; k < 12; k++) o[k] = mk(fma(-kap, acc[k].re, o[k].re), fma(-kap, acc[k].im, o[k].im));
            if (a.dagger) g5(o);
            if (EPI & disco::EPI_RESID) {
                cx<T> b[12];
                IO::template loadv<BUF>(a.aux, Vv, n, r, sv, b);
#pragma unroll
                for (int k = 0; k < 12; k++) o[k] = b[k] - o[k];
            }
        }
        IO::template store<true>(a.out, Vv, n, r, sv, o);
        int q = 0;
        cx<T> w[12];
        if (EPI & (disco::EPI_DOTAUX | disco::EPI_DOTAUXIN)) IO::template loadv<BUF>(a.aux2, Vv, n, r, sv, w);
        // each lane's twelve-term sums in the arithmetic precision (FMA
        // chains); the sums over lanes and blocks are FP64
        if (EPI & disco::EPI_DOTAUX) {
            cx<T> acc = mk((T)0, (T)0);
#pragma unroll
            for (int k = 0; k < 12; k++) cjmac(acc, w[k], o[k]);
            red[2 * q] = (double)acc.re;
            red[2 * q + 1] = (double)acc.im;
            q++;
        }
        if (EPI & disco::EPI_NORM) {
            T nn = 0;
#pragma unroll
            for (int k = 0; k < 12; k++) {
                nn = fma(o[k].re, o[k].re, nn);
                nn = fma(o[k].im, o[k].im, nn);
            }
            red[2 * q] = (double)nn;
            q++;
        }
        if (EPI & disco::EPI_DOTIN) {
            cx<T> acc = mk((T)0, (T)0);
#pragma unroll
            for (int k = 0; k < 12; k++) cjmac(acc, o[k], pin[k]);
            red[2 * q] = (double)acc.re;
            red[2 * q + 1] = (double)acc.im;
            q++;
        }
        if (EPI & disco::EPI_DOTAUXIN) {
            cx<T> acc = mk((T)0, (T)0);
#pragma unroll
            for (int k = 0; k < 12; k++) cjmac(acc, w[k], pin[k]);
            red[2 * q] = (double)acc.re;
            red[2 * q + 1] = (double)acc.im;
            q++;
        }
    }
    if constexpr (NQ > 0) rhs_partials<NQ>(red, n, nact, a.part, a.nsb, sb);
}

// ---- layout conversion: canonical complex128 [r][s][12] <-> native [plane][s][r]
template <class IO>
__global__ void k_to_native(const double2* __restrict__ in, void* __restrict__ out, long V, int nr, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long r = i / V, s = i - r * V;
    const double2* q = in + i * 12;
    cx<typename IO::T> p[12];
    if constexpr (sizeof(typename IO::T) == 8) {
#pragma unroll
        for (int k = 0; k < 12; k++) p[k] = mk(q[k].x, q[k].y);
    } else if constexpr (IO::planes == 3) {
#pragma unroll
        for (int k = 0; k < 12; k++) p[k] = mk(d2f_odd(q[k].x), d2f_odd(q[k].y));
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) p[k] = mk((float)q[k].x, (float)q[k].y);
    }
    IO::template store<true>(out, V, nr, r, s, p);
}

template <class IO>
__global__ void k_from_native(const void* __restrict__ in, double2* __restrict__ out, long V, int nr, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long r = i / V, s = i - r * V;
    cx<typename IO::T> p[12];
    IO::load(in, V, nr, r, s, p);
    double2* q = out + i * 12;
#pragma unroll
    for (int k = 0; k < 12; k++) q[k] = make_double2((double)p[k].re, (double)p[k].im);
}

// (the large-volume path without buffer descriptors keeps one generic
// instance that reads the mask when there is one)
template <class IO, int EPI, bool EO>
void launch_one(disco_ctx* ctx, const StencilArgs& a) {
    const dim3 grid(xcd_grid(a.nsb)), block(kStencilBlock);
    const bool stage = sizeof(typename IO::T) == 4 && a.spb <= kStageSites && a.stage;
    const bool masked = a.mask != nullptr;
    if (stage) {
        const size_t shm = (size_t)a.spb * (kStageLinkBytes + kStageCloverBytes);
        if (a.in.buf && masked)
            hipLaunchKernelGGL((k_dslash<IO, EPI, true, true, EO, true>), grid, block, shm, ctx->stream, a);
        else if (a.in.buf)
            hipLaunchKernelGGL((k_dslash<IO, EPI, true, true, EO, false>), grid, block, shm, ctx->stream, a);
        else
            hipLaunchKernelGGL((k_dslash<IO, EPI, false, true, EO, true>), grid, block, shm, ctx->stream, a);
    } else {
        if (a.in.buf && masked)
            hipLaunchKernelGGL((k_dslash<IO, EPI, true, false, EO, true>), grid, block, 0, ctx->stream, a);
        else if (a.in.buf)
            hipLaunchKernelGGL((k_dslash<IO, EPI, true, false, EO, false>), grid, block, 0, ctx->stream, a);
        else
            hipLaunchKernelGGL((k_dslash<IO, EPI, false, false, EO, true>), grid, block, 0, ctx->stream, a);
    }
}

template <class IO>
void launch_epi(disco_ctx* ctx, const StencilArgs& a, int epi, bool eo) {
    using namespace disco;
    if (eo) {
        switch (epi) {
            case EPI_NONE: launch_one<IO, EPI_NONE, true>(ctx, a); break;
            case EPI_DOTAUX: launch_one<IO, EPI_DOTAUX, true>(ctx, a); break;
            case EPI_NORM | EPI_DOTIN: launch_one<IO, EPI_NORM | EPI_DOTIN, true>(ctx, a); break;
            case EPI_DOTAUX | EPI_NORM | EPI_DOTIN | EPI_DOTAUXIN:
                launch_one<IO, EPI_DOTAUX | EPI_NORM | EPI_DOTIN | EPI_DOTAUXIN, true>(ctx, a);
                break;
            default: disco_throw(DISCO_EINVAL, "even-odd stencil epilogue %d not built", epi);
        }
        return;
    }
    switch (epi) {
        case EPI_NONE: launch_one<IO, EPI_NONE, false>(ctx, a); break;
        case EPI_DOTAUX: launch_one<IO, EPI_DOTAUX, false>(ctx, a); break;
        case EPI_NORM: launch_one<IO, EPI_NORM, false>(ctx, a); break;
        case EPI_NORM | EPI_DOTIN: launch_one<IO, EPI_NORM | EPI_DOTIN, false>(ctx, a); break;
        case EPI_DOTAUX | EPI_NORM | EPI_DOTIN | EPI_DOTAUXIN:
            launch_one<IO, EPI_DOTAUX | EPI_NORM | EPI_DOTIN | EPI_DOTAUXIN, false>(ctx, a);
            break;
        case EPI_RESID | EPI_NORM: launch_one<IO, EPI_RESID | EPI_NORM, false>(ctx, a); break;
        case EPI_RESID: launch_one<IO, EPI_RESID, false>(ctx, a); break;
        default: disco_throw(DISCO_EINVAL, "stencil epilogue %d not built", epi);
    }
}

}  // namespace

namespace disco {

int nq_of(int epi) {
    return ((epi & EPI_DOTAUX) ? 1 : 0) + ((epi & EPI_NORM) ? 1 : 0) + ((epi & EPI_DOTIN) ? 1 : 0) +
           ((epi & EPI_DOTAUXIN) ? 1 : 0);
}

int stencil_spb(int n) { return n >= kStencilBlock ? 1 : kStencilBlock / n; }

// Right-hand sides whose spinor planes (V n 16 bytes each, at every precision)
// stay below 4 GiB: the stencil addresses a plane with 32-bit offsets.
int plane_rhs_limit(const disco_ctx* ctx) {
    return (int)std::max(1LL, std::min((long long)kStencilBlock, ((1LL << 32) - 1) / (16LL * ctx->V)));
}

// Site order of the stencil.  Each XCD (8 contiguous ranges of the order)
// takes one slab of Lt/8 timeslices when Lt is a multiple of 8.  Inside a slab
// the order is x fastest, then y within a tile of yt rows, then t within a
// tile of tt timeslices, then z, then the y tiles, then the t tiles: hops in t
// and z then land a few hundred sites away in the visiting order (instead of a
// whole timeslice), so the neighbours of the sites in flight are still in that
// XCD's L2.  By default tt is the whole slab and yt the largest divisor of Ly
// with Lx * yt * (Lt/8) <= 320 sites per z step, but at least 2 when Ly is
// even: single-row tiles send every y hop across a tile (4, 2 and 2 rows at
// 16^3x32, 24^3x48 and 32^3x64).  ctx->tile_y and ctx->tile_t (divisors of Ly
// and of the slab; 0 = the default) override the tile; the autotuner sets
// them.  DISCO_TRAVERSAL = natural restores lexicographic order.  The tables
// are rewritten in place, so graphs captured with them stay valid.
void build_traversal(disco_ctx* ctx) {
    const int Lx = ctx->dims[0], Ly = ctx->dims[1], Lz = ctx->dims[2], Lt = ctx->dims[3];
    const long V = ctx->V;
    std::vector<int2> tr(V);
    const char* env = getenv("DISCO_TRAVERSAL");
    const bool natural = env && std::string(env) == "natural";
    auto put = [&](long g, int x, int y, int z, int t) {
        tr[g].x = (int)(x + (long)Lx * (y + (long)Ly * (z + (long)Lz * t)));
        tr[g].y = x | (y << 8) | (z << 16) | (t << 24);
    };
    long g = 0;
    if (natural) {
        for (int t = 0; t < Lt; t++)
            for (int z = 0; z < Lz; z++)
                for (int y = 0; y < Ly; y++)
                    for (int x = 0; x < Lx; x++) put(g++, x, y, z, t);
    } else {
        const int nch = (Lt % 8 == 0) ? 8 : 1;
        const int tc = Lt / nch;
        int yt = 1;
        for (int c = 1; c <= Ly; c++)
            if (Ly % c == 0 && (long)Lx * c * tc <= 320) yt = c;
        if (yt == 1 && Ly % 2 == 0) yt = 2;
        if (ctx->tile_y > 0) yt = ctx->tile_y;
        const int tt = ctx->tile_t > 0 ? ctx->tile_t : tc;
        REQUIRE(Ly % yt == 0 && tc % tt == 0, DISCO_EINVAL, "tile %d x %d does not divide Ly = %d and the slab of %d",
                yt, tt, Ly, tc);
        for (int ch = 0; ch < nch; ch++)
            for (int tb = 0; tb < tc / tt; tb++)
                for (int yb = 0; yb < Ly / yt; yb++)
                    for (int z = 0; z < Lz; z++)
                        for (int tl = 0; tl < tt; tl++)
                            for (int yi = 0; yi < yt; yi++)
                                for (int x = 0; x < Lx; x++) put(g++, x, yb * yt + yi, z, ch * tc + tb * tt + tl);
        ctx->tile_used[0] = yt;
        ctx->tile_used[1] = tt;
    }
    ctx->trav_kind = natural ? 0 : 1;
    // tables in flight on the stream must not change under a kernel
    if (ctx->d_trav) HIPCHK(hipStreamSynchronize(ctx->stream));
    if (!ctx->d_trav) HIPCHK(hipMalloc(&ctx->d_trav, sizeof(int2) * V));
    HIPCHK(hipMemcpy(ctx->d_trav, tr.data(), sizeof(int2) * V, hipMemcpyHostToDevice));
    if (V % 2 == 0) {
        std::vector<int2> par[2];
        for (long k = 0; k < V; k++) {
            const int c = tr[k].y;
            par[((c & 0xff) + ((c >> 8) & 0xff) + ((c >> 16) & 0xff) + ((c >> 24) & 0xff)) & 1].push_back(tr[k]);
        }
        for (int p = 0; p < 2; p++) {
            if (!ctx->d_trav_eo[p])
                HIPCHK(hipMalloc(&ctx->d_trav_eo[p], sizeof(int2) * std::max<size_t>(1, par[p].size())));
            HIPCHK(hipMemcpy(ctx->d_trav_eo[p], par[p].data(), sizeof(int2) * par[p].size(), hipMemcpyHostToDevice));
        }
    }
}

bool eo_supported(const disco_ctx* ctx) {
    return ctx->dims[0] % 2 == 0 && ctx->dims[1] % 2 == 0 && ctx->dims[2] % 2 == 0 && ctx->dims[3] % 2 == 0 &&
           ctx->d_trav_eo[0] != nullptr;
}

int stencil_nsb(disco_ctx* ctx, int n, bool eo) {
    int spb = stencil_spb(n);
    const long sites = eo ? ctx->V / 2 : ctx->V;
    return (int)((sites + spb - 1) / spb);
}

void stencil_launch(disco_ctx* ctx, const StencilCall& c) {
    REQUIRE(ctx->have_clover, DISCO_ESTATE, "operator applied before clover_setup");
    REQUIRE(c.nrhs >= 1 && c.nrhs <= kStencilBlock, DISCO_EINVAL, "nrhs per launch must be in 1..%d", kStencilBlock);
    REQUIRE(c.nrhs <= plane_rhs_limit(ctx), DISCO_EINVAL,
            "%d right-hand sides per launch exceed the %d that 32-bit plane offsets address at this volume", c.nrhs,
            plane_rhs_limit(ctx));
    REQUIRE(!(c.dagger && (c.epi & EPI_DOTIN)), DISCO_EINVAL, "DOTIN epilogue with dagger");
    const bool eo = c.eo_target >= 0;
    REQUIRE(!eo || (eo_supported(ctx) && c.eo_target <= 1 && !c.dagger && !(c.epi & EPI_RESID)), DISCO_EINVAL,
            "even-odd stencil needs even extents, no dagger and no residual epilogue");
    StencilArgs a;
    // bytes one buffer descriptor covers: the whole block, or one plane for
    // FP64 (whose twelve planes pass 4 GiB first)
    const size_t blk = native_bytes(ctx, c.prec, c.nrhs) / (eo ? 2 : 1) / (c.prec == DISCO_F64 ? 12 : 1);
    const int buf = blk < (1ULL << 32) ? 1 : 0;
    a.in = RoView{c.in, (unsigned)blk, buf};
    a.out = c.out;
    a.aux = RoView{c.aux, (unsigned)blk, buf};
    a.aux2 = RoView{c.aux2, (unsigned)blk, buf};
    a.mask = c.mask;
    a.allhops = 0xffu;
    a.trav = eo ? ctx->d_trav_eo[c.eo_target] : ctx->d_trav;
    a.part = c.part;
    a.V = ctx->V;
    a.Vv = eo ? ctx->V / 2 : ctx->V;
    a.nsites = (int)a.Vv;
    a.eo_aux = eo && (c.ca != 0.0 || c.cg != 0.0 || (c.epi & (EPI_DOTIN | EPI_DOTAUXIN))) ? 1 : 0;
    a.ca = c.ca;
    a.cg = c.cg;
    a.cb = c.cb;
    long st = 1;
    for (int m = 0; m < 4; m++) {
        a.L[m] = ctx->dims[m];
        a.st[m] = st;
        st *= ctx->dims[m];
        a.ph[m] = (double)ctx->bc[m];
    }
    a.kappa = ctx->kappa;
    a.n = c.nrhs;
    a.spb = stencil_spb(c.nrhs);
    a.nsb = stencil_nsb(ctx, c.nrhs, eo);
    a.dagger = c.dagger;
    // staging pays once a site has 16 or more lanes sharing its links
    a.stage = ctx->opt_stage == 1 || (ctx->opt_stage == -1 && c.nrhs >= 16);
    double sp = c.prec == DISCO_F64 ? 8 : c.prec == DISCO_F32 ? 4 : 2;  // bytes per spinor real
    double sg = c.prec == DISCO_F64 ? 8 : 4;                             // bytes per link/clover real
    int nvec = 2 + ((c.epi & EPI_RESID) ? 1 : 0) + ((c.epi & (EPI_DOTAUX | EPI_DOTAUXIN)) ? 1 : 0) + (a.eo_aux ? 1 : 0);
    // each spinor once, every link of the sites visited (all 4V links in even-odd
    // mode, where the backward links belong to the other parity), clover once
    double bytes = eo ? (double)a.Vv * (c.nrhs * nvec * 24 * sp + 144 * sg + 72 * sg + (c.mask ? 1 : 0))
                      : (double)ctx->V * (c.nrhs * nvec * 24 * sp + 72 * sg + 72 * sg + (c.mask ? 1 : 0));
    const int fam = (eo ? 13 : 10) + c.prec;
    int rec = prof_begin(ctx, fam);
    const bool f64 = c.prec == DISCO_F64;
    a.U = f64 ? (const void*)ctx->U64 : (const void*)ctx->U32;
    a.A = eo ? (f64 ? (const void*)ctx->Ai64 : (const void*)ctx->Ai32) : (f64 ? (const void*)ctx->A64 : (const void*)ctx->A32);
    if (c.prec == DISCO_F64)
        launch_epi<IO64>(ctx, a, c.epi, eo);
    else if (c.prec == DISCO_F32)
        launch_epi<IO32>(ctx, a, c.epi, eo);
    else if (c.prec == DISCO_BF16)
        launch_epi<IOBF>(ctx, a, c.epi, eo);
    else
        disco_throw(DISCO_EINVAL, "bad precision %d", c.prec);
    HIPCHK(hipGetLastError());
    prof_end(ctx, rec, fam, bytes);
}

size_t native_bytes(const disco_ctx* ctx, int prec, int nrhs) {
    size_t per = prec == DISCO_F64 ? 192 : prec == DISCO_F32 ? 96 : 48;
    return per * (size_t)ctx->V * (size_t)nrhs;
}

void to_native(disco_ctx* ctx, int prec, int nrhs, const void* in, void* out) {
    long n = ctx->V * (long)nrhs;
    int nb = (int)((n + 255) / 256);
    if (prec == DISCO_F64)
        k_to_native<IO64><<<nb, 256, 0, ctx->stream>>>((const double2*)in, out, ctx->V, nrhs, n);
    else if (prec == DISCO_F32)
        k_to_native<IO32><<<nb, 256, 0, ctx->stream>>>((const double2*)in, out, ctx->V, nrhs, n);
    else if (prec == DISCO_BF16)
        k_to_native<IOBF><<<nb, 256, 0, ctx->stream>>>((const double2*)in, out, ctx->V, nrhs, n);
    else
        disco_throw(DISCO_EINVAL, "bad precision %d", prec);
    HIPCHK(hipGetLastError());
}

void from_native(disco_ctx* ctx, int prec, int nrhs, const void* in, void* out) {
    long n = ctx->V * (long)nrhs;
    int nb = (int)((n + 255) / 256);
    if (prec == DISCO_F64)
        k_from_native<IO64><<<nb, 256, 0, ctx->stream>>>(in, (double2*)out, ctx->V, nrhs, n);
    else if (prec == DISCO_F32)
        k_from_native<IO32><<<nb, 256, 0, ctx->stream>>>(in, (double2*)out, ctx->V, nrhs, n);
    else if (prec == DISCO_BF16)
        k_from_native<IOBF><<<nb, 256, 0, ctx->stream>>>(in, (double2*)out, ctx->V, nrhs, n);
    else
        disco_throw(DISCO_EINVAL, "bad precision %d", prec);
    HIPCHK(hipGetLastError());
}

}  // namespace disco

// ----------------------------------------------------------------- C ABI
extern "C" {

long long disco_native_bytes(const disco_ctx* ctx, int prec, int nrhs) {
    if (!ctx || nrhs < 0 || prec < 0 || prec > 2) return -1;
    return (long long)disco::native_bytes(ctx, prec, nrhs);
}

int disco_to_native(disco_ctx* ctx, int prec, int nrhs, const void* in, void* out) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(in && out && nrhs >= 0, DISCO_EINVAL, "bad argument");
        activate(ctx);
        if (nrhs) disco::to_native(ctx, prec, nrhs, in, out);
    });
}

int disco_from_native(disco_ctx* ctx, int prec, int nrhs, const void* in, void* out) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(in && out && nrhs >= 0, DISCO_EINVAL, "bad argument");
        activate(ctx);
        if (nrhs) disco::from_native(ctx, prec, nrhs, in, out);
    });
}

int disco_dirac_apply_native(disco_ctx* ctx, const disco_domains* dom, int prec, int dagger, int nrhs,
                             const void* in, void* out) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(in && out, DISCO_EINVAL, "NULL spinor");
        REQUIRE(in != out, DISCO_EINVAL, "in and out must differ");
        REQUIRE(!dom || dom->ctx == ctx, DISCO_EINVAL, "domains belong to another context");
        activate(ctx);
        if (nrhs == 0) return;
        disco::StencilCall c{prec, dagger ? 1 : 0, nrhs, in, out, nullptr, nullptr, dom ? dom->d_mask : nullptr,
                             nullptr, disco::EPI_NONE};
        disco::stencil_launch(ctx, c);
    });
}

static int apply_canonical(disco_ctx* ctx, const disco_domains* dom, int prec, int dagger, int nrhs, const void* in,
                           void* out) {
    return guarded(ctx, [&] {
        REQUIRE(in && out, DISCO_EINVAL, "NULL spinor");
        REQUIRE(in != out, DISCO_EINVAL, "in and out must differ");
        REQUIRE(prec >= 0 && prec <= 2, DISCO_EINVAL, "bad precision %d", prec);
        REQUIRE(!dom || dom->ctx == ctx, DISCO_EINVAL, "domains belong to another context");
        REQUIRE(ctx->have_clover, DISCO_ESTATE, "operator applied before clover_setup");
        activate(ctx);
        if (nrhs == 0) return;
        const size_t field = (size_t)ctx->V * 12 * sizeof(double2);
        const int cap = std::min(64, disco::plane_rhs_limit(ctx));
        for (int r0 = 0; r0 < nrhs; r0 += cap) {
            const int n = std::min(cap, nrhs - r0);
            size_t nb = disco::native_bytes(ctx, prec, n);
            void* a = ws_get(ctx, "apply_in", nb);
            void* b = ws_get(ctx, "apply_out", nb);
            disco::to_native(ctx, prec, n, (const char*)in + r0 * field, a);
            disco::StencilCall c{prec, dagger ? 1 : 0, n, a, b, nullptr, nullptr, dom ? dom->d_mask : nullptr,
                                 nullptr, disco::EPI_NONE};
            disco::stencil_launch(ctx, c);
            disco::from_native(ctx, prec, n, b, (char*)out + r0 * field);
        }
    });
}

int disco_dirac_apply(disco_ctx* ctx, int prec, int dagger, int nrhs, const void* in, void* out) {
    if (!ctx) return DISCO_EINVAL;
    return apply_canonical(ctx, nullptr, prec, dagger, nrhs, in, out);
}

int disco_dirac_block_apply(disco_ctx* ctx, const disco_domains* dom, int prec, int dagger, int nrhs, const void* in,
                            void* out) {
    if (!ctx) return DISCO_EINVAL;
    if (!dom) {
        ctx->err = "dirac_block_apply needs domains";
        return DISCO_EINVAL;
    }
    return apply_canonical(ctx, dom, prec, dagger, nrhs, in, out);
}

}  // extern "C"
