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
#include <algorithm>

#include "spinor_io.h"

namespace {

constexpr int kStencilBlock = kMaxBlock;

struct StencilArgs {
    const void* in;
    void* out;
    const void* aux;   // b of out = b - D in
    const void* aux2;  // w of <w, out>
    const void* U;
    const void* A;
    const uint8_t* mask;
    double2* part;
    long V;
    int L[4];
    long st[4];
    double ph[4];
    double kappa;
    int nsb;   // site blocks (= partial-sum slots per rhs and quantity)
    int spb;   // sites per block
    int n;     // right-hand sides in the block
    int dagger;
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

template <typename T>
__device__ __forceinline__ void su3_mul(const cx<T> u[9], const cx<T> h[6], cx<T> o[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; sp++)
#pragma unroll
        for (int a = 0; a < 3; a++)
            o[sp * 3 + a] = u[a * 3 + 0] * h[sp * 3 + 0] + u[a * 3 + 1] * h[sp * 3 + 1] + u[a * 3 + 2] * h[sp * 3 + 2];
}

template <typename T>
__device__ __forceinline__ void su3_dag_mul(const cx<T> u[9], const cx<T> h[6], cx<T> o[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; sp++)
#pragma unroll
        for (int a = 0; a < 3; a++)
            o[sp * 3 + a] =
                cjmul(u[0 * 3 + a], h[sp * 3 + 0]) + cjmul(u[1 * 3 + a], h[sp * 3 + 1]) + cjmul(u[2 * 3 + a], h[sp * 3 + 2]);
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
            cx<T> a = mk(f[6 + 2 * m], f[7 + 2 * m]);
            y[i] = y[i] + a * x[j];
            y[j] = y[j] + cjmul(a, x[i]);
        }
}

// both hops in direction MU for right-hand side r at site s
template <class IO, int MU>
__device__ __forceinline__ void hops(const StencilArgs& a, long s, const int* x, uint32_t m, int n, long r,
                                     cx<typename IO::T> acc[12]) {
    typedef typename IO::T T;
    const typename IO::LinkT* U = (const typename IO::LinkT*)a.U;
    const long V = a.V;
    const int L = a.L[MU];
    const long st = a.st[MU];
    if (m & (1u << (2 * MU))) {
        // forward: (1 - gamma_mu) U_mu(x) psi(x+mu), boundary phase at the wrap
        const bool wrap = x[MU] == L - 1;
        const long nb = wrap ? s - (long)(L - 1) * st : s + st;
        cx<T> u[9], p[12], h[6], o[6];
        IO::load(a.in, V, n, r, nb, p);
        IO::load_link(U, V, MU, s, u);
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
        const long nb = wrap ? s + (long)(L - 1) * st : s - st;
        cx<T> u[9], p[12], h[6], o[6];
        IO::load(a.in, V, n, r, nb, p);
        IO::load_link(U, V, MU, nb, u);
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
                              ((EPI & disco::EPI_DOTIN) ? 1 : 0);
};

template <class IO, int EPI>
__global__ __launch_bounds__(kStencilBlock) void k_dslash(const StencilArgs a) {
    typedef typename IO::T T;
    constexpr int NQ = EpiCount<EPI>::nq;
    const int n = a.n;
    const int spb = a.spb;  // sites per block; the block has spb*n active lanes
    const int sb = xcd_block(a.nsb);
    if (sb < 0) return;
    const int t = threadIdx.x;
    const int nact = spb * n;
    const long s = (long)sb * spb + t / n;
    const long r = t % n;
    const long V = a.V;
    double red[NQ > 0 ? 2 * NQ : 1];
#pragma unroll
    for (int k = 0; k < (NQ > 0 ? 2 * NQ : 1); k++) red[k] = 0;

    if (t < nact && s < V) {
        int x[4];
        {
            long q = s;
            x[0] = (int)(q % a.L[0]); q /= a.L[0];
            x[1] = (int)(q % a.L[1]); q /= a.L[1];
            x[2] = (int)(q % a.L[2]); q /= a.L[2];
            x[3] = (int)q;
        }
        const uint32_t m = a.mask ? (uint32_t)a.mask[s] : 0xffu;
        cx<T> acc[12];
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = mk((T)0, (T)0);
        hops<IO, 0>(a, s, x, m, n, r, acc);
        hops<IO, 1>(a, s, x, m, n, r, acc);
        hops<IO, 2>(a, s, x, m, n, r, acc);
        hops<IO, 3>(a, s, x, m, n, r, acc);

        // site-local part: A(x) psi(x) - kappa * hops
        cx<T> p[12], o[12];
        IO::load(a.in, V, n, r, s, p);
        cx<T> pin[12];
        if (EPI & disco::EPI_DOTIN) {
#pragma unroll
            for (int k = 0; k < 12; k++) pin[k] = p[k];
        }
        if (a.dagger) g5(p);
        {
            T f[36];
            IO::load_clover((const typename IO::CloverT*)a.A, V, 0, s, f);
            clover6(f, p, o);
            IO::load_clover((const typename IO::CloverT*)a.A, V, 1, s, f);
            clover6(f, p + 6, o + 6);
        }
        const T kap = (T)a.kappa;
#pragma unroll
        for (int k = 0; k < 12; k++) o[k] = o[k] - kap * acc[k];
        if (a.dagger) g5(o);
        if (EPI & disco::EPI_RESID) {
            cx<T> b[12];
            IO::load(a.aux, V, n, r, s, b);
#pragma unroll
            for (int k = 0; k < 12; k++) o[k] = b[k] - o[k];
        }
        IO::store(a.out, V, n, r, s, o);
        int q = 0;
        if (EPI & disco::EPI_DOTAUX) {
            cx<T> w[12];
            IO::load(a.aux2, V, n, r, s, w);
            double re = 0, im = 0;
#pragma unroll
            for (int k = 0; k < 12; k++) {
                cx<T> d = cjmul(w[k], o[k]);
                re += (double)d.re;
                im += (double)d.im;
            }
            red[2 * q] = re;
            red[2 * q + 1] = im;
            q++;
        }
        if (EPI & disco::EPI_NORM) {
            double nn = 0;
#pragma unroll
            for (int k = 0; k < 12; k++) nn += (double)nrm(o[k]);
            red[2 * q] = nn;
            q++;
        }
        if (EPI & disco::EPI_DOTIN) {
            double re = 0, im = 0;
#pragma unroll
            for (int k = 0; k < 12; k++) {
                cx<T> d = cjmul(o[k], pin[k]);
                re += (double)d.re;
                im += (double)d.im;
            }
            red[2 * q] = re;
            red[2 * q + 1] = im;
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
    IO::store(out, V, nr, r, s, p);
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

template <class IO, int EPI>
void launch_one(disco_ctx* ctx, const StencilArgs& a) {
    hipLaunchKernelGGL((k_dslash<IO, EPI>), dim3(xcd_grid(a.nsb)), dim3(kStencilBlock), 0, ctx->stream, a);
}

template <class IO>
void launch_epi(disco_ctx* ctx, const StencilArgs& a, int epi) {
    using namespace disco;
    switch (epi) {
        case EPI_NONE: launch_one<IO, EPI_NONE>(ctx, a); break;
        case EPI_DOTAUX: launch_one<IO, EPI_DOTAUX>(ctx, a); break;
        case EPI_NORM: launch_one<IO, EPI_NORM>(ctx, a); break;
        case EPI_NORM | EPI_DOTIN: launch_one<IO, EPI_NORM | EPI_DOTIN>(ctx, a); break;
        case EPI_RESID | EPI_NORM: launch_one<IO, EPI_RESID | EPI_NORM>(ctx, a); break;
        case EPI_RESID: launch_one<IO, EPI_RESID>(ctx, a); break;
        default: disco_throw(DISCO_EINVAL, "stencil epilogue %d not built", epi);
    }
}

}  // namespace

namespace disco {

int nq_of(int epi) {
    return ((epi & EPI_DOTAUX) ? 1 : 0) + ((epi & EPI_NORM) ? 1 : 0) + ((epi & EPI_DOTIN) ? 1 : 0);
}

int stencil_spb(int n) { return n >= kStencilBlock ? 1 : kStencilBlock / n; }

int stencil_nsb(disco_ctx* ctx, int n) {
    int spb = stencil_spb(n);
    return (int)((ctx->V + spb - 1) / spb);
}

void stencil_launch(disco_ctx* ctx, const StencilCall& c) {
    REQUIRE(ctx->have_clover, DISCO_ESTATE, "operator applied before clover_setup");
    REQUIRE(c.nrhs >= 1 && c.nrhs <= kStencilBlock, DISCO_EINVAL, "nrhs per launch must be in 1..%d", kStencilBlock);
    REQUIRE(!(c.dagger && (c.epi & EPI_DOTIN)), DISCO_EINVAL, "DOTIN epilogue with dagger");
    StencilArgs a;
    a.in = c.in;
    a.out = c.out;
    a.aux = c.aux;
    a.aux2 = c.aux2;
    a.mask = c.mask;
    a.part = c.part;
    a.V = ctx->V;
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
    a.nsb = stencil_nsb(ctx, c.nrhs);
    a.dagger = c.dagger;
    double sp = c.prec == DISCO_F64 ? 8 : c.prec == DISCO_F32 ? 4 : 2;  // bytes per spinor real
    double sg = c.prec == DISCO_F64 ? 8 : 4;                             // bytes per link/clover real
    int nvec = 2 + ((c.epi & EPI_RESID) ? 1 : 0) + ((c.epi & EPI_DOTAUX) ? 1 : 0);
    double bytes = (double)ctx->V * (c.nrhs * nvec * 24 * sp + 72 * sg + 72 * sg + (c.mask ? 1 : 0));
    int rec = prof_begin(ctx);
    if (c.prec == DISCO_F64) {
        a.U = ctx->U64;
        a.A = ctx->A64;
        launch_epi<IO64>(ctx, a, c.epi);
    } else if (c.prec == DISCO_F32) {
        a.U = ctx->U32;
        a.A = ctx->A32;
        launch_epi<IO32>(ctx, a, c.epi);
    } else if (c.prec == DISCO_BF16) {
        a.U = ctx->U32;
        a.A = ctx->A32;
        launch_epi<IOBF>(ctx, a, c.epi);
    } else {
        disco_throw(DISCO_EINVAL, "bad precision %d", c.prec);
    }
    HIPCHK(hipGetLastError());
    prof_end(ctx, rec, 0, bytes);
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
        for (int r0 = 0; r0 < nrhs; r0 += 64) {
            const int n = std::min(64, nrhs - r0);
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
