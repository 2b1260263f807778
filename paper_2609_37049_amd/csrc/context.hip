// Context, error plumbing, gauge field loading, clover term, domains, profiling.
#include <cmath>
#include <cstdarg>

#include "common.h"

[[noreturn]] void disco_throw(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    throw DiscoError{code, std::string(buf)};
}

void activate(disco_ctx* ctx) { HIPCHK(hipSetDevice(ctx->device)); }

void* ws_get(disco_ctx* ctx, const std::string& name, size_t bytes) {
    auto it = ctx->ws.find(name);
    if (it != ctx->ws.end() && it->second.second >= bytes) return it->second.first;
    if (it != ctx->ws.end()) {
        // the old buffer may still be read by queued work
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipFree(it->second.first));
        ctx->ws.erase(it);
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess)
        disco_throw(DISCO_ENOMEM, "workspace '%s': cannot allocate %zu bytes", name.c_str(), bytes);
    ctx->ws[name] = {p, bytes};
    return p;
}

void ws_free(disco_ctx* ctx, const std::string& name) {
    auto it = ctx->ws.find(name);
    if (it == ctx->ws.end()) return;
    // queued work may still read it
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipFree(it->second.first));
    ctx->ws.erase(it);
}

static hipEvent_t ev_get(disco_ctx* ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

int prof_begin(disco_ctx* ctx, int family) {
    if (!ctx->prof_on) return -1;
    if ((ctx->prof_seen[family]++) % ctx->prof_stride) return -1;
    ProfRec r;
    r.a = ev_get(ctx);
    r.b = ev_get(ctx);
    r.bytes = 0;
    r.kernel = -1;
    HIPCHK(hipEventRecord(r.a, ctx->stream));
    ctx->prof.push_back(r);
    return (int)ctx->prof.size() - 1;
}

void prof_end(disco_ctx* ctx, int rec, int kernel, double bytes) {
    if (rec < 0) return;
    ProfRec& r = ctx->prof[rec];
    HIPCHK(hipEventRecord(r.b, ctx->stream));
    r.kernel = kernel;
    r.bytes = bytes;
}

// ----------------------------------------------------------------- gauge loading
// canonical U[s][mu][a][b] -> U64[mu][ab][s], U32 likewise; per-block SU(3) defect maximum
__global__ void k_gauge_import(const double2* __restrict__ Uc, double2* __restrict__ U64,
                               float2* __restrict__ U32, long V, double* __restrict__ defect) {
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double worst = 0;
    if (s < V) {
        for (int mu = 0; mu < 4; mu++) {
            cd m[9];
            for (int k = 0; k < 9; k++) {
                double2 v = Uc[(s * 4 + mu) * 9 + k];
                m[k] = mk(v.x, v.y);
                U64[((long)mu * 9 + k) * V + s] = v;
                U32[((long)mu * 9 + k) * V + s] = make_float2((float)v.x, (float)v.y);
            }
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) {
                    cd acc = mk(0.0, 0.0);
                    for (int c = 0; c < 3; c++) acc = acc + m[a * 3 + c] * cj(m[b * 3 + c]);
                    if (a == b) acc.re -= 1.0;
                    worst = fmax(worst, sqrt(nrm(acc)));
                }
            cd det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                     m[2] * (m[3] * m[7] - m[4] * m[6]);
            det.re -= 1.0;
            worst = fmax(worst, sqrt(nrm(det)));
        }
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = worst;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) defect[blockIdx.x] = sh[0];
}

// ----------------------------------------------------------------- clover term
struct Geo {
    int L[4];
    long st[4];
};

__device__ __forceinline__ long hop(const Geo& g, long s, const int* x, int mu, int d) {
    int xm = x[mu] + d;
    if (xm < 0) return s + (long)(g.L[mu] - 1) * g.st[mu];
    if (xm >= g.L[mu]) return s - (long)(g.L[mu] - 1) * g.st[mu];
    return s + d * g.st[mu];
}

__device__ __forceinline__ void ld_link(const double2* __restrict__ U, long V, int mu, long s, cd m[9]) {
#pragma unroll
    for (int k = 0; k < 9; k++) {
        double2 v = U[((long)mu * 9 + k) * V + s];
        m[k] = mk(v.x, v.y);
    }
}

__device__ __forceinline__ void mm3(const cd a[9], const cd b[9], bool da, bool db, cd c[9]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cd acc = mk(0.0, 0.0);
            for (int k = 0; k < 3; k++) {
                cd x = da ? cj(a[k * 3 + i]) : a[i * 3 + k];
                cd y = db ? cj(b[j * 3 + k]) : b[k * 3 + j];
                acc = acc + x * y;
            }
            c[i * 3 + j] = acc;
        }
}

// anti-hermitian part of the clover leaf sum in the (mu,nu) plane: (Q - Q^+)/8
__device__ void fhat(const double2* __restrict__ U, long V, const Geo& g, long s, const int* x, int mu, int nu,
                     cd F[9]) {
    cd Q[9];
    for (int k = 0; k < 9; k++) Q[k] = mk(0.0, 0.0);
    cd a[9], b[9], c[9], d[9], t1[9], t2[9], l[9];
    long smu = hop(g, s, x, mu, +1), snu = hop(g, s, x, nu, +1);
    long smm = hop(g, s, x, mu, -1), snm = hop(g, s, x, nu, -1);
    int xm[4] = {x[0], x[1], x[2], x[3]};
    xm[mu] = (x[mu] - 1 + g.L[mu]) % g.L[mu];
    long smm_nu = hop(g, smm, xm, nu, +1), smm_nm = hop(g, smm, xm, nu, -1);
    int xn[4] = {x[0], x[1], x[2], x[3]};
    xn[nu] = (x[nu] - 1 + g.L[nu]) % g.L[nu];
    long snm_mu = hop(g, snm, xn, mu, +1);
    // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    ld_link(U, V, mu, s, a); ld_link(U, V, nu, smu, b); ld_link(U, V, mu, snu, c); ld_link(U, V, nu, s, d);
    mm3(a, b, false, false, t1); mm3(t1, c, false, true, t2); mm3(t2, d, false, true, l);
    for (int k = 0; k < 9; k++) Q[k] = Q[k] + l[k];
    // leaf 2: U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    ld_link(U, V, nu, s, a); ld_link(U, V, mu, smm_nu, b); ld_link(U, V, nu, smm, c); ld_link(U, V, mu, smm, d);
    mm3(a, b, false, true, t1); mm3(t1, c, false, true, t2); mm3(t2, d, false, false, l);
    for (int k = 0; k < 9; k++) Q[k] = Q[k] + l[k];
    // leaf 3: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    ld_link(U, V, mu, smm, a); ld_link(U, V, nu, smm_nm, b); ld_link(U, V, mu, smm_nm, c); ld_link(U, V, nu, snm, d);
    mm3(a, b, true, true, t1); mm3(t1, c, false, false, t2); mm3(t2, d, false, false, l);
    for (int k = 0; k < 9; k++) Q[k] = Q[k] + l[k];
    // leaf 4: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+
    ld_link(U, V, nu, snm, a); ld_link(U, V, mu, snm, b); ld_link(U, V, nu, snm_mu, c); ld_link(U, V, mu, s, d);
    mm3(a, b, true, false, t1); mm3(t1, c, false, false, t2); mm3(t2, d, false, true, l);
    for (int k = 0; k < 9; k++) Q[k] = Q[k] + l[k];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cd q = Q[i * 3 + j], qt = cj(Q[j * 3 + i]);
            F[i * 3 + j] = 0.125 * (q - qt);
        }
}

// Flat order of one hermitian 6x6 block: 6 real diagonals, then the 15 upper
// off-diagonals (i<j, row-major) as (re, im).
__global__ void k_clover(const double2* __restrict__ U, Geo g, long V, double ck /* csw*kappa */,
                         double2* __restrict__ A64, float4* __restrict__ A32) {
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    int x[4];
    {
        long r = s;
        x[0] = r % g.L[0]; r /= g.L[0];
        x[1] = r % g.L[1]; r /= g.L[1];
        x[2] = r % g.L[2]; r /= g.L[2];
        x[3] = (int)r;
    }
    cd F[6][9];  // planes 01,02,03,12,13,23
    const int pm[6] = {0, 0, 0, 1, 1, 2}, pn[6] = {1, 2, 3, 2, 3, 3};
    for (int p = 0; p < 6; p++) fhat(U, V, g, s, x, pm[p], pn[p], F[p]);
    // chiral blocks: 1 + i ck [s1 (x) P1 + s2 (x) P2 + s3 (x) P3]
    //   upper: P1 = F03 - F12, P2 = F02 + F13, P3 = F23 - F01
    //   lower: P1 = -F03 - F12, P2 = F02 - F13, P3 = -F23 - F01
    for (int blk = 0; blk < 2; blk++) {
        double sg = blk == 0 ? 1.0 : -1.0;
        cd P1[9], P2[9], P3[9];
        for (int k = 0; k < 9; k++) {
            P1[k] = sg * F[2][k] - F[3][k];
            P2[k] = F[1][k] + sg * F[4][k];
            P3[k] = sg * F[5][k] - F[0][k];
        }
        cd B[6][6];
        for (int sa = 0; sa < 2; sa++)
            for (int sb = 0; sb < 2; sb++)
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        // sigma_1 = [[0,1],[1,0]], sigma_2 = [[0,-i],[i,0]], sigma_3 = diag(1,-1)
                        cd m = mk(0.0, 0.0);
                        if (sa != sb) {
                            m = m + P1[i * 3 + j];
                            cd t = P2[i * 3 + j];
                            m = m + (sa == 0 ? neg(ti(t)) : ti(t));
                        } else {
                            m = m + (sa == 0 ? P3[i * 3 + j] : neg(P3[i * 3 + j]));
                        }
                        cd v = ck * ti(m);
                        if (sa == sb && i == j) v.re += 1.0;
                        B[sa * 3 + i][sb * 3 + j] = v;
                    }
        double f[36];
        for (int i = 0; i < 6; i++) f[i] = B[i][i].re;
        int m = 0;
        for (int i = 0; i < 6; i++)
            for (int j = i + 1; j < 6; j++, m++) {
                f[6 + 2 * m] = B[i][j].re;
                f[7 + 2 * m] = B[i][j].im;
            }
        for (int q = 0; q < 18; q++) A64[((long)blk * 18 + q) * V + s] = make_double2(f[2 * q], f[2 * q + 1]);
        for (int q = 0; q < 9; q++)
            A32[((long)blk * 9 + q) * V + s] =
                make_float4((float)f[4 * q], (float)f[4 * q + 1], (float)f[4 * q + 2], (float)f[4 * q + 3]);
    }
}

// A(x)^-1 per site and chiral block (Gauss-Jordan with partial pivoting in
// FP64), stored in the packed format of A (the inverse of a hermitian matrix is
// hermitian: the upper triangle is the mean of (i,j) and conj(j,i)).
__global__ void k_clover_inv(const double2* __restrict__ A64, long V, double2* __restrict__ Ai64,
                             float4* __restrict__ Ai32) {
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    for (int blk = 0; blk < 2; blk++) {
        double f[36];
        for (int q = 0; q < 18; q++) {
            double2 v = A64[((long)blk * 18 + q) * V + s];
            f[2 * q] = v.x;
            f[2 * q + 1] = v.y;
        }
        cd M[6][12];
        for (int i = 0; i < 6; i++)
            for (int j = 0; j < 12; j++) M[i][j] = mk(j == i + 6 ? 1.0 : 0.0, 0.0);
        for (int i = 0; i < 6; i++) M[i][i] = mk(f[i], 0.0);
        int m = 0;
        for (int i = 0; i < 6; i++)
            for (int j = i + 1; j < 6; j++, m++) {
                M[i][j] = mk(f[6 + 2 * m], f[7 + 2 * m]);
                M[j][i] = mk(f[6 + 2 * m], -f[7 + 2 * m]);
            }
        for (int c = 0; c < 6; c++) {
            int pr = c;
            double best = nrm(M[c][c]);
            for (int r = c + 1; r < 6; r++)
                if (nrm(M[r][c]) > best) {
                    best = nrm(M[r][c]);
                    pr = r;
                }
            if (pr != c)
                for (int j = 0; j < 12; j++) {
                    cd t = M[c][j];
                    M[c][j] = M[pr][j];
                    M[pr][j] = t;
                }
            const cd piv = M[c][c];
            const double dn = nrm(piv);
            const cd inv = mk(piv.re / dn, -piv.im / dn);
            for (int j = 0; j < 12; j++) M[c][j] = inv * M[c][j];
            for (int r = 0; r < 6; r++) {
                if (r == c) continue;
                const cd fac = M[r][c];
                for (int j = 0; j < 12; j++) M[r][j] = M[r][j] - fac * M[c][j];
            }
        }
        double g[36];
        for (int i = 0; i < 6; i++) g[i] = M[i][i + 6].re;
        m = 0;
        for (int i = 0; i < 6; i++)
            for (int j = i + 1; j < 6; j++, m++) {
                const cd a = M[i][j + 6], b = M[j][i + 6];
                g[6 + 2 * m] = 0.5 * (a.re + b.re);
                g[7 + 2 * m] = 0.5 * (a.im - b.im);
            }
        for (int q = 0; q < 18; q++) Ai64[((long)blk * 18 + q) * V + s] = make_double2(g[2 * q], g[2 * q + 1]);
        for (int q = 0; q < 9; q++)
            Ai32[((long)blk * 9 + q) * V + s] =
                make_float4((float)g[4 * q], (float)g[4 * q + 1], (float)g[4 * q + 2], (float)g[4 * q + 3]);
    }
}

__global__ void k_clover_expand(const double2* __restrict__ A64, long V, double2* __restrict__ out) {
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    double2* o = out + s * 144;
    for (int k = 0; k < 144; k++) o[k] = make_double2(0, 0);
    for (int blk = 0; blk < 2; blk++) {
        double f[36];
        for (int q = 0; q < 18; q++) {
            double2 v = A64[((long)blk * 18 + q) * V + s];
            f[2 * q] = v.x;
            f[2 * q + 1] = v.y;
        }
        int base = blk * 6;  // spins 0,1 (upper) or 2,3 (lower): index spin*3 + colour
        for (int i = 0; i < 6; i++) o[(base + i) * 12 + base + i] = make_double2(f[i], 0);
        int m = 0;
        for (int i = 0; i < 6; i++)
            for (int j = i + 1; j < 6; j++, m++) {
                o[(base + i) * 12 + base + j] = make_double2(f[6 + 2 * m], f[7 + 2 * m]);
                o[(base + j) * 12 + base + i] = make_double2(f[6 + 2 * m], -f[7 + 2 * m]);
            }
    }
}

// ----------------------------------------------------------------- C ABI
extern "C" {

// Message of the last failed disco_create on this thread (its context is gone).
static thread_local std::string create_err;

int disco_create(const int dims[4], const int bc[4], int device, disco_ctx** out) {
    if (!out || !dims || !bc) return DISCO_EINVAL;
    *out = nullptr;
    disco_ctx* ctx = new disco_ctx();
    int rc = guarded(ctx, [&] {
        long V = 1;
        for (int m = 0; m < 4; m++) {
            REQUIRE(dims[m] >= 1, DISCO_EINVAL, "dims[%d] = %d must be >= 1", m, dims[m]);
            REQUIRE(bc[m] == 1 || bc[m] == -1, DISCO_EINVAL, "bc[%d] must be +1 or -1", m);
            ctx->dims[m] = dims[m];
            ctx->bc[m] = bc[m];
            V *= dims[m];
        }
        REQUIRE(V * 36 * 16 < (1L << 32), DISCO_EINVAL, "volume too large (links must stay below 4 GiB)");
        ctx->V = V;
        ctx->Vs = V / dims[3];
        ctx->device = device;
        activate(ctx);
        REQUIRE(dims[0] <= 255 && dims[1] <= 255 && dims[2] <= 255 && dims[3] <= 255, DISCO_EINVAL,
                "extents above 255 are not supported");
        disco::build_traversal(ctx);
        disco::scratch_bind(device);
    });
    if (rc != DISCO_OK) {
        create_err = ctx->err;
        delete ctx;
        return rc;
    }
    *out = ctx;
    return DISCO_OK;
}

int disco_destroy(disco_ctx* ctx) {
    if (!ctx) return DISCO_OK;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->ws) hipFree(kv.second.first);
    hipFree(ctx->U64);
    hipFree(ctx->U32);
    hipFree(ctx->Usm);
    hipFree(ctx->A64);
    hipFree(ctx->Ai64);
    hipFree(ctx->Ai32);
    hipFree(ctx->A32);
    hipFree(ctx->d_trav);
    hipFree(ctx->d_trav_eo[0]);
    hipFree(ctx->d_trav_eo[1]);
    for (auto& kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
    for (auto& r : ctx->prof) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : ctx->ev_pool) hipEventDestroy(e);
    delete ctx;
    return DISCO_OK;
}

int disco_set_stream(disco_ctx* ctx, void* s) {
    if (!ctx) return DISCO_EINVAL;
    ctx->stream = (hipStream_t)s;
    return DISCO_OK;
}

const char* disco_last_error(const disco_ctx* ctx) {
    if (ctx) return ctx->err.c_str();
    return create_err.empty() ? "null context" : create_err.c_str();
}

int disco_gauge_set(disco_ctx* ctx, const void* U, int where) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(U, DISCO_EINVAL, "U is NULL");
        REQUIRE(where == DISCO_HOST || where == DISCO_DEVICE, DISCO_EINVAL, "bad 'where'");
        activate(ctx);
        long V = ctx->V;
        size_t nbytes = (size_t)V * 36 * sizeof(double2);
        const double2* src = (const double2*)U;
        if (where == DISCO_HOST) {
            double2* st = (double2*)ws_get(ctx, "gauge_stage", nbytes);
            HIPCHK(hipMemcpyAsync(st, U, nbytes, hipMemcpyHostToDevice, ctx->stream));
            src = st;
        }
        if (!ctx->U64) {
            HIPCHK(hipMalloc(&ctx->U64, (size_t)V * 36 * sizeof(double2)));
            HIPCHK(hipMalloc(&ctx->U32, (size_t)V * 36 * sizeof(float2)));
        }
        int nb = (int)((V + 255) / 256);
        double* defect = (double*)ws_get(ctx, "gauge_defect", nb * sizeof(double));
        k_gauge_import<<<nb, 256, 0, ctx->stream>>>(src, ctx->U64, ctx->U32, V, defect);
        HIPCHK(hipGetLastError());
        std::vector<double> h(nb);
        HIPCHK(hipMemcpyAsync(h.data(), defect, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        double worst = 0;
        for (double v : h) worst = std::fmax(worst, v);
        ctx->have_gauge = false;
        ctx->have_clover = false;
        ctx->have_smeared = false;
        REQUIRE(worst <= 1e-12, DISCO_EINVAL, "links are not SU(3): defect %.3e > 1e-12", worst);
        ctx->have_gauge = true;
    });
}

int disco_clover_setup(disco_ctx* ctx, double kappa, double csw) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(ctx->have_gauge, DISCO_ESTATE, "clover_setup before gauge_set");
        activate(ctx);
        long V = ctx->V;
        if (!ctx->A64) {
            HIPCHK(hipMalloc(&ctx->A64, (size_t)V * 36 * sizeof(double2) / 1));
            HIPCHK(hipMalloc(&ctx->A32, (size_t)V * 18 * sizeof(float4)));
            HIPCHK(hipMalloc(&ctx->Ai64, (size_t)V * 36 * sizeof(double2)));
            HIPCHK(hipMalloc(&ctx->Ai32, (size_t)V * 18 * sizeof(float4)));
        }
        Geo g;
        long st = 1;
        for (int m = 0; m < 4; m++) {
            g.L[m] = ctx->dims[m];
            g.st[m] = st;
            st *= ctx->dims[m];
        }
        k_clover<<<(int)((V + 127) / 128), 128, 0, ctx->stream>>>(ctx->U64, g, V, csw * kappa, ctx->A64, ctx->A32);
        k_clover_inv<<<(int)((V + 127) / 128), 128, 0, ctx->stream>>>(ctx->A64, V, ctx->Ai64, ctx->Ai32);
        HIPCHK(hipGetLastError());
        ctx->kappa = kappa;
        ctx->csw = csw;
        ctx->have_clover = true;
    });
}

int disco_clover_get(disco_ctx* ctx, void* A_out) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(ctx->have_clover, DISCO_ESTATE, "no clover term");
        REQUIRE(A_out, DISCO_EINVAL, "A_out is NULL");
        activate(ctx);
        k_clover_expand<<<(int)((ctx->V + 255) / 256), 256, 0, ctx->stream>>>(ctx->A64, ctx->V, (double2*)A_out);
        HIPCHK(hipGetLastError());
    });
}

int disco_domains_create(disco_ctx* ctx, const uint8_t* cut, int lmax, disco_domains** out) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(cut && out, DISCO_EINVAL, "NULL argument");
        int Lm = 0;
        for (int m = 0; m < 4; m++) Lm = std::max(Lm, ctx->dims[m]);
        REQUIRE(lmax >= Lm, DISCO_EINVAL, "lmax %d < max extent %d", lmax, Lm);
        activate(ctx);
        long V = ctx->V;
        std::vector<uint8_t> mask(V);
        const int* L = ctx->dims;
        for (long s = 0; s < V; s++) {
            long r = s;
            int x[4];
            for (int m = 0; m < 4; m++) {
                x[m] = (int)(r % L[m]);
                r /= L[m];
            }
            uint8_t b = 0;
            for (int m = 0; m < 4; m++) {
                if (!cut[m * lmax + x[m]]) b |= (uint8_t)(1u << (2 * m));
                if (!cut[m * lmax + (x[m] - 1 + L[m]) % L[m]]) b |= (uint8_t)(1u << (2 * m + 1));
            }
            mask[s] = b;
        }
        disco_domains* d = new disco_domains();
        d->ctx = ctx;
        d->lmax = lmax;
        d->cut.assign(cut, cut + 4 * lmax);
        if (hipMalloc(&d->d_mask, V) != hipSuccess) {
            delete d;
            disco_throw(DISCO_ENOMEM, "domain mask allocation");
        }
        HIPCHK(hipMemcpy(d->d_mask, mask.data(), V, hipMemcpyHostToDevice));
        *out = d;
    });
}

int disco_domains_destroy(disco_domains* d) {
    if (!d) return DISCO_OK;
    hipFree(d->d_mask);
    delete d;
    return DISCO_OK;
}

long long disco_last_solves(const disco_ctx* ctx) { return ctx ? ctx->last_solves : -1; }

int disco_set_option(disco_ctx* ctx, int option, int value) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        if (option == DISCO_OPT_GRAPHS) {
            REQUIRE(value == 0 || value == 1, DISCO_EINVAL, "graphs option is 0 or 1");
            ctx->opt_graphs = value;
        } else if (option == DISCO_OPT_STAGE) {
            REQUIRE(value >= -1 && value <= 1, DISCO_EINVAL, "stage option is -1, 0 or 1");
            ctx->opt_stage = value;
        } else if (option == DISCO_OPT_EO) {
            REQUIRE(value == 0 || value == 1, DISCO_EINVAL, "even-odd option is 0 or 1");
            ctx->opt_eo = value;
        } else if (option == DISCO_OPT_NARROW) {
            REQUIRE(value == 0 || value == 1, DISCO_EINVAL, "narrow option is 0 or 1");
            ctx->opt_narrow = value;
        } else if (option == DISCO_OPT_TILE_Y || option == DISCO_OPT_TILE_T) {
            REQUIRE(value >= 0 && value <= 255, DISCO_EINVAL, "tile extent %d", value);
            activate(ctx);
            int& f = option == DISCO_OPT_TILE_Y ? ctx->tile_y : ctx->tile_t;
            const int old = f;
            f = value;
            try {
                disco::build_traversal(ctx);
            } catch (...) {
                f = old;
                throw;
            }
        } else {
            disco_throw(DISCO_EINVAL, "unknown option %d", option);
        }
    });
}

int disco_get_option(const disco_ctx* ctx, int option, int* value) {
    if (!ctx || !value) return DISCO_EINVAL;
    switch (option) {
        case DISCO_OPT_GRAPHS: *value = ctx->opt_graphs; break;
        case DISCO_OPT_STAGE: *value = ctx->opt_stage; break;
        case DISCO_OPT_EO: *value = ctx->opt_eo; break;
        case DISCO_OPT_NARROW: *value = ctx->opt_narrow; break;
        case DISCO_OPT_TILE_Y: *value = ctx->tile_used[0]; break;
        case DISCO_OPT_TILE_T: *value = ctx->tile_used[1]; break;
        default: return DISCO_EINVAL;
    }
    return DISCO_OK;
}

int disco_profile_enable(disco_ctx* ctx, int on) {
    if (!ctx) return DISCO_EINVAL;
    ctx->prof_on = on != 0;
    return DISCO_OK;
}

int disco_profile_stride(disco_ctx* ctx, int stride) {
    if (!ctx || stride < 1) return DISCO_EINVAL;
    ctx->prof_stride = stride;
    return DISCO_OK;
}

int disco_profile_reset(disco_ctx* ctx) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        for (auto& r : ctx->prof) {
            ctx->ev_pool.push_back(r.a);
            ctx->ev_pool.push_back(r.b);
        }
        ctx->prof.clear();
        ctx->prof_seen.clear();
    });
}

int disco_profile_get(disco_ctx* ctx, int kernel, long long* launches, double* total_ms, double* bytes) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        long long n = 0;
        double ms = 0, by = 0;
        for (auto& r : ctx->prof) {
            const bool match = r.kernel == kernel || (kernel == 0 && r.kernel >= 10 && r.kernel <= 12);
            if (!match) continue;
            float t = 0;
            HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
            ms += t;
            by += r.bytes;
            n++;
        }
        if (launches) *launches = n;
        if (total_ms) *total_ms = ms;
        if (bytes) *bytes = by;
    });
}

}  // extern "C"
