// Distillation on the GPU: APE smearing of the spatial links, the gauge-
// covariant 3-D Laplacian and its lowest eigenvectors per timeslice, the
// distillation sources v_i(t) (x) e_alpha (several timeslices packed into one
// source for the domain-restricted operator), the perambulator projection
// V^+ X on FP64 matrix cores, loops Tr[Gamma tau(t,t)] and the disconnected
// correlators (full, completely factorised, subtracted, four-term split).
//
// Eigenvector blocks use the layout [t][xs*3 + c][j] (vector index j fastest,
// K = 3 Vs rows per timeslice), so that the Laplacian stencil reads coalesced
// rows and the Gram / projection contractions are plain row-major matrices.
#include <algorithm>
#include <cmath>
#include <thread>

#include "dense_host.h"
#include "spinor_io.h"

typedef double d4v __attribute__((ext_vector_type(4)));

namespace disco {
void solve_native(disco_ctx* ctx, const disco_domains* dom, const disco_solver_params& P, int n, const double2* b64,
                  double2* x64, disco_solver_stats* st);
int default_rhs_block(const disco_solver_params& P, int nrhs, const disco_ctx* ctx);
}  // namespace disco

namespace {

// ------------------------------------------------------------------ SU(3) helpers (FP64)
__device__ __forceinline__ void m3mul(const cd* a, const cd* b, cd* c, bool da = false, bool db = false) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cd s = mk(0.0, 0.0);
            for (int k = 0; k < 3; k++) {
                cd x = da ? cj(a[k * 3 + i]) : a[i * 3 + k];
                cd y = db ? cj(b[j * 3 + k]) : b[k * 3 + j];
                s = s + x * y;
            }
            c[i * 3 + j] = s;
        }
}

__device__ __forceinline__ cd det3(const cd* m) {
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
           m[2] * (m[3] * m[7] - m[4] * m[6]);
}

// W = M (M^+ M)^{-1/2} by the Newton iteration W <- (W + W^{-+})/2 (with
// the usual determinant-based scaling), then W / det(W)^{1/3} (principal
// cube root).  The polar factor is unique, so this matches any other
// evaluation of it; it commutes with M -> A M B^+ for unitary A, B.
__device__ void su3_project(const cd* M, cd* W) {
    cd X[9];
    for (int k = 0; k < 9; k++) X[k] = M[k];
    for (int it = 0; it < 30; it++) {
        // inverse-transpose-conjugate: X^{-+} = cof(X)^* / det(X)^*
        cd d = det3(X);
        cd cof[9];
        cof[0] = X[4] * X[8] - X[5] * X[7];
        cof[1] = X[5] * X[6] - X[3] * X[8];
        cof[2] = X[3] * X[7] - X[4] * X[6];
        cof[3] = X[2] * X[7] - X[1] * X[8];
        cof[4] = X[0] * X[8] - X[2] * X[6];
        cof[5] = X[1] * X[6] - X[0] * X[7];
        cof[6] = X[1] * X[5] - X[2] * X[4];
        cof[7] = X[2] * X[3] - X[0] * X[5];
        cof[8] = X[0] * X[4] - X[1] * X[3];
        // X^{-1} = cof^T / d, so X^{-+} = conj(cof) / conj(d)
        double ad = sqrt(nrm(d));
        double g = (it < 6) ? pow(ad, -1.0 / 3.0) : 1.0;  // scaling speeds up the first steps
        cd dc = cj(d);
        double dn = nrm(d);
        double diff = 0;
        for (int k = 0; k < 9; k++) {
            cd inv = mk((cj(cof[k]).re * dc.re + cj(cof[k]).im * dc.im) / dn,
                        (cj(cof[k]).im * dc.re - cj(cof[k]).re * dc.im) / dn);
            cd nx = 0.5 * (g * X[k] + (1.0 / g) * inv);
            diff = fmax(diff, sqrt(nrm(nx - X[k])));
            X[k] = nx;
        }
        if (it >= 6 && diff < 1e-15) break;
    }
    cd d = det3(X);
    double ph = atan2(d.im, d.re) / 3.0;
    cd f = mk(cos(ph), -sin(ph));
    for (int k = 0; k < 9; k++) W[k] = f * X[k];
}

struct Geo3 {
    int L[4];
    long st[4];
};

__device__ __forceinline__ long nbr(const Geo3& g, long s, int x, int mu, int d) {
    int xm = x + d;
    if (xm < 0) return s + (long)(g.L[mu] - 1) * g.st[mu];
    if (xm >= g.L[mu]) return s - (long)(g.L[mu] - 1) * g.st[mu];
    return s + d * g.st[mu];
}

__device__ __forceinline__ void coords(const Geo3& g, long s, int* x) {
    long r = s;
    x[0] = r % g.L[0]; r /= g.L[0];
    x[1] = r % g.L[1]; r /= g.L[1];
    x[2] = r % g.L[2]; r /= g.L[2];
    x[3] = (int)r;
}

__device__ __forceinline__ void ldU(const double2* U, long V, int mu, long s, cd* u) {
    for (int k = 0; k < 9; k++) {
        double2 v = U[((long)mu * 9 + k) * V + s];
        u[k] = mk(v.x, v.y);
    }
}

// one APE step on the spatial links (all updated from the previous links)
__global__ void k_ape(const double2* __restrict__ Uin, double2* __restrict__ Uout, Geo3 g, long V, double alpha) {
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    int x[4];
    coords(g, s, x);
    for (int k = 0; k < 3; k++) {
        cd M[9], Uk[9], S[9];
        ldU(Uin, V, k, s, Uk);
        for (int q = 0; q < 9; q++) S[q] = mk(0.0, 0.0);
        for (int j = 0; j < 3; j++) {
            if (j == k) continue;
            cd a[9], b[9], c[9], t1[9], t2[9];
            long sj = nbr(g, s, x[j], j, 1), sk = nbr(g, s, x[k], k, 1);
            // up: U_j(x) U_k(x+j) U_j(x+k)^+
            ldU(Uin, V, j, s, a);
            ldU(Uin, V, k, sj, b);
            ldU(Uin, V, j, sk, c);
            m3mul(a, b, t1);
            m3mul(t1, c, t2, false, true);
            for (int q = 0; q < 9; q++) S[q] = S[q] + t2[q];
            // down: U_j(x-j)^+ U_k(x-j) U_j(x-j+k)
            long sjm = nbr(g, s, x[j], j, -1);
            int xk = x[k];
            long sjmk = nbr(g, sjm, xk, k, 1);
            ldU(Uin, V, j, sjm, a);
            ldU(Uin, V, k, sjm, b);
            ldU(Uin, V, j, sjmk, c);
            m3mul(a, b, t1, true, false);
            m3mul(t1, c, t2);
            for (int q = 0; q < 9; q++) S[q] = S[q] + t2[q];
        }
        for (int q = 0; q < 9; q++) M[q] = (1.0 - alpha) * Uk[q] + (alpha / 4.0) * S[q];
        cd W[9];
        su3_project(M, W);
        for (int q = 0; q < 9; q++) Uout[((long)k * 9 + q) * V + s] = make_double2(W[q].re, W[q].im);
    }
}

// smeared spatial links -> canonical [s][mu][a][b] with the time link copied
__global__ void k_smeared_export(const double2* __restrict__ Usm, const double2* __restrict__ U64, long V,
                                 double2* __restrict__ out) {
    long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    for (int mu = 0; mu < 4; mu++)
        for (int q = 0; q < 9; q++)
            out[(s * 4 + mu) * 9 + q] = mu < 3 ? Usm[((long)mu * 9 + q) * V + s] : U64[((long)3 * 9 + q) * V + s];
}

// ------------------------------------------------------------------ 3-D Laplacian on eigenvector blocks
// y[t][xs*3+c][j] = sum_k [2 y(x) - U_k(x) y(x+k) - U_k(x-k)^+ y(x-k)]  (within timeslice t)
// The blocks may hold a subset of the timeslices: block timeslice tb is
// lattice timeslice tmap[tb] (tmap = NULL: all of them, in order); nsites =
// sites of the blocks.  The Laplacian acts within a timeslice, so a subset is
// an exact restriction.
//
// A workgroup takes kLapSites consecutive block sites: it first copies their
// six links (U_k(x) and U_k(x-k), k = 1..3) into LDS, then runs one thread per
// (site, vector j), j fastest, so that a wavefront reads each neighbour row of
// m vectors contiguously and the m threads of a site share one copy of its
// links.  Index arithmetic is 32-bit: the caller guarantees 3 nsites m < 2^31.
// CHEB: one step of the Chebyshev filter fused in, out = a (L y - c y) + b prev
// (prev NULL reads as 0); otherwise out = L y.
constexpr int kLapSites = 16;

struct LapSite {
    unsigned bb;  // first block site of the timeslice
    unsigned lb;  // first lattice site of the timeslice
    unsigned xs;  // site within the timeslice
    unsigned x[3];
};

__device__ __forceinline__ LapSite lap_site(const Geo3& g, const int* tmap, unsigned sb_) {
    const unsigned Vs = (unsigned)g.st[3], L0 = (unsigned)g.L[0], L1 = (unsigned)g.L[1];
    LapSite o;
    const unsigned tb = sb_ / Vs;
    o.xs = sb_ - tb * Vs;
    o.bb = tb * Vs;
    o.lb = (tmap ? (unsigned)tmap[tb] : tb) * Vs;
    const unsigned q = o.xs / L0;
    o.x[0] = o.xs - q * L0;
    o.x[1] = q % L1;
    o.x[2] = q / L1;
    return o;
}

// spatial neighbour of xs in direction k (d = +1 forward, -1 backward), periodic
__device__ __forceinline__ unsigned lap_nbr(const Geo3& g, const LapSite& p, int k, int d) {
    const unsigned L = (unsigned)g.L[k], st = (unsigned)g.st[k];
    if (d > 0) return p.x[k] + 1 == L ? p.xs - (L - 1) * st : p.xs + st;
    return p.x[k] == 0 ? p.xs + (L - 1) * st : p.xs - st;
}

template <bool CHEB>
__global__ __launch_bounds__(256) void k_laplace(const double2* __restrict__ U, const double2* __restrict__ in,
                                                 double2* __restrict__ out, Geo3 g, long V, int m,
                                                 const int* __restrict__ tmap, int nsites,
                                                 const double2* __restrict__ prev, double ca, double cc, double cb) {
    __shared__ double2 su[kLapSites][6][9];
    const unsigned mm = (unsigned)m;
    const unsigned s0 = blockIdx.x * kLapSites;
    const unsigned ns = min((unsigned)kLapSites, (unsigned)nsites - s0);
    for (unsigned e = threadIdx.x; e < ns * 54; e += blockDim.x) {
        const unsigned ls = e / 54, r = e - ls * 54, h = r / 9, q = r - h * 9;
        const LapSite p = lap_site(g, tmap, s0 + ls);
        const int k = (int)(h % 3);
        const unsigned site = p.lb + (h < 3 ? p.xs : lap_nbr(g, p, k, -1));
        su[ls][h][q] = U[((size_t)k * 9 + q) * (size_t)V + site];
    }
    __syncthreads();
    for (unsigned e = threadIdx.x; e < ns * mm; e += blockDim.x) {
        const unsigned ls = e / mm, j = e - ls * mm;
        const unsigned sb_ = s0 + ls;  // site in the blocks
        const LapSite p = lap_site(g, tmap, sb_);
        cd y0[3], acc[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const double2 v = in[(sb_ * 3 + c) * mm + j];
            y0[c] = mk(v.x, v.y);
            acc[c] = mk(6.0 * v.x, 6.0 * v.y);
        }
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const unsigned xf = p.bb + lap_nbr(g, p, k, 1), xb = p.bb + lap_nbr(g, p, k, -1);
            cd u[9], yf[3], yb[3];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const double2 a = in[(xf * 3 + c) * mm + j], b = in[(xb * 3 + c) * mm + j];
                yf[c] = mk(a.x, a.y);
                yb[c] = mk(b.x, b.y);
            }
#pragma unroll
            for (int q = 0; q < 9; q++) u[q] = mk(su[ls][k][q].x, su[ls][k][q].y);
#pragma unroll
            for (int a = 0; a < 3; a++) acc[a] = acc[a] - (u[a * 3] * yf[0] + u[a * 3 + 1] * yf[1] + u[a * 3 + 2] * yf[2]);
#pragma unroll
            for (int q = 0; q < 9; q++) u[q] = mk(su[ls][3 + k][q].x, su[ls][3 + k][q].y);
#pragma unroll
            for (int a = 0; a < 3; a++)
                acc[a] = acc[a] - (cjmul(u[a], yb[0]) + cjmul(u[3 + a], yb[1]) + cjmul(u[6 + a], yb[2]));
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const unsigned o = (sb_ * 3 + c) * mm + j;
            if constexpr (CHEB) {
                const double2 q = prev ? prev[o] : make_double2(0, 0);
                out[o] = make_double2(ca * (acc[c].re - cc * y0[c].re) + cb * q.x,
                                      ca * (acc[c].im - cc * y0[c].im) + cb * q.y);
            } else {
                out[o] = make_double2(acc[c].re, acc[c].im);
            }
        }
    }
}

static int lap_grid(long nsites) { return (int)((nsites + kLapSites - 1) / kLapSites); }

// deterministic pseudo-random start vectors (splitmix64 of the element index)
__global__ void k_rand_fill(double2* y, long n, unsigned long long seed) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        unsigned long long z = seed + 0x9e3779b97f4a7c15ULL * (unsigned long long)(2 * i + 1);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z = z ^ (z >> 31);
        double a = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        z += 0x9e3779b97f4a7c15ULL;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z = z ^ (z >> 31);
        double b = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        y[i] = make_double2(a, b);
    }
}

// ------------------------------------------------------------------ FP64 MFMA contractions
// Partial tiles of C_b = A_b^H B_b with A_b (K x M), B_b (K x N) row-major
// complex (element (k,i) at A + b*sA + k*lda + i).  One wavefront computes one
// 16x16 output tile over one K-chunk with v_mfma_f64_16x16x4f64; the complex
// product is four real products.  Partials go to P[b][ks][M][N].
__global__ __launch_bounds__(64) void k_zgemm_hn(const double2* __restrict__ A, long lda, long sA,
                                                 const double2* __restrict__ B, long ldb, long sB,
                                                 double2* __restrict__ P, int M, int N, int K, int kchunk, int nks,
                                                 int tilesM, int tilesN) {
    const int lane = threadIdx.x;
    int w = blockIdx.x;
    const int tj = w % tilesN; w /= tilesN;
    const int ti = w % tilesM; w /= tilesM;
    const int ks = w % nks; w /= nks;
    const int b = w;
    const int i = ti * 16 + (lane & 15);
    const int j = tj * 16 + (lane & 15);
    const int kq = lane >> 4;
    const double2* Ab = A + (long)b * sA;
    const double2* Bb = B + (long)b * sB;
    // four k-steps per trip with independent accumulators, so the matrix-core
    // pipeline is not stalled by a single dependency chain; all loads first
    d4v cr[4], ci[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        cr[u] = d4v{0, 0, 0, 0};
        ci[u] = d4v{0, 0, 0, 0};
    }
    const int k0 = ks * kchunk, k1 = min(K, k0 + kchunk);
    for (int kb = k0; kb < k1; kb += 16) {
        double2 a[4], v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int k = kb + 4 * u + kq;
            a[u] = (k < k1 && i < M) ? Ab[(long)k * lda + i] : make_double2(0, 0);
            v[u] = (k < k1 && j < N) ? Bb[(long)k * ldb + j] : make_double2(0, 0);
        }
        // conj(a) * v = (ar br + ai bi) + i (ar bi - ai br)
#pragma unroll
        for (int u = 0; u < 4; u++) {
            cr[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, v[u].x, cr[u], 0, 0, 0);
            ci[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, v[u].y, ci[u], 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            cr[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, v[u].y, cr[u], 0, 0, 0);
            ci[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[u].y, v[u].x, ci[u], 0, 0, 0);
        }
    }
    d4v crs = (cr[0] + cr[1]) + (cr[2] + cr[3]);
    d4v cis = (ci[0] + ci[1]) + (ci[2] + ci[3]);
    // accumulator layout of v_mfma_f64_16x16x4f64: register e of a lane holds
    // row lane/16 + 4e, column lane%16
    for (int e = 0; e < 4; e++) {
        const int row = ti * 16 + (lane >> 4) + 4 * e;
        const int col = tj * 16 + (lane & 15);
        if (row < M && col < N) P[(((long)b * nks + ks) * M + row) * N + col] = make_double2(crs[e], cis[e]);
    }
}

// C[b][i][j] = sum_ks P[b][ks][i][j] (fixed order)
__global__ void k_ksum(const double2* __restrict__ P, double2* __restrict__ C, int M, int N, int nks, int batch) {
    long tot = (long)batch * M * N;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (long)gridDim.x * blockDim.x) {
        long b = q / ((long)M * N), e = q - b * M * N;
        double re = 0, im = 0;
        for (int ks = 0; ks < nks; ks++) {
            double2 v = P[((long)b * nks + ks) * M * N + e];
            re += v.x;
            im += v.y;
        }
        C[q] = make_double2(re, im);
    }
}

// Y_b (K x m) <- Y_b C_b (C_b m x m) on MFMA: one wavefront per 16x16 output tile.
__global__ __launch_bounds__(64) void k_zgemm_nn(const double2* __restrict__ Y, const double2* __restrict__ Cm,
                                                 double2* __restrict__ out, int K, int m, int tilesK, int tilesM) {
    const int lane = threadIdx.x;
    int w = blockIdx.x;
    const int tj = w % tilesM; w /= tilesM;
    const int tr = w % tilesK; w /= tilesK;
    const int b = w;
    const int row = tr * 16 + (lane & 15);
    const int col = tj * 16 + (lane & 15);
    const int kq = lane >> 4;
    const double2* Yb = Y + (long)b * K * m;
    const double2* Cb = Cm + (long)b * m * m;
    d4v cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    for (int kb = 0; kb < m; kb += 4) {
        const int k = kb + kq;
        double2 a = (k < m && row < K) ? Yb[(long)row * m + k] : make_double2(0, 0);
        double2 v = (k < m && col < m) ? Cb[(long)k * m + col] : make_double2(0, 0);
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, v.x, cr, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, v.y, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, v.y, ci, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, v.x, ci, 0, 0, 0);
    }
    for (int e = 0; e < 4; e++) {
        const int r = tr * 16 + (lane >> 4) + 4 * e;
        const int c = tj * 16 + (lane & 15);
        if (r < K && c < m) out[((long)b * K + r) * m + c] = make_double2(cr[e], ci[e]);
    }
}

// per (t, j): ||L y_j - lambda_j y_j||^2 for the first nv columns
__global__ void k_resid(const double2* __restrict__ ly, const double2* __restrict__ y, const double* __restrict__ lam,
                        double* __restrict__ out, int K, int m, int nv) {
    const int t = blockIdx.y;
    const int j = blockIdx.x;
    if (j >= nv) return;
    const double l = lam[t * m + j];
    double acc[1] = {0};
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        double2 a = ly[((long)t * K + k) * m + j], b = y[((long)t * K + k) * m + j];
        double re = a.x - l * b.x, im = a.y - l * b.y;
        acc[0] += re * re + im * im;
    }
    block_sum(acc);
    if (threadIdx.x == 0) out[t * nv + j] = acc[0];
}

// internal [t][xs*3+c][j] (first nv of m columns) -> canonical V[t][i][xs][c]
__global__ void k_eig_export(const double2* __restrict__ Y, double2* __restrict__ V, int T, long K, int m, int nv) {
    long tot = (long)T * nv * K;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (long)gridDim.x * blockDim.x) {
        long t = q / (nv * K), r = q - t * nv * K;
        long i = r / K, k = r - i * K;
        V[q] = Y[((long)t * K + k) * m + i];
    }
}

// canonical V[t][i][xs][c] -> internal [t][xs*3+c][i]
__global__ void k_eig_import(const double2* __restrict__ V, double2* __restrict__ Y, int T, long K, int nv) {
    long tot = (long)T * nv * K;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (long)gridDim.x * blockDim.x) {
        long t = q / (nv * K), r = q - t * nv * K;
        long i = r / K, k = r - i * K;
        Y[((long)t * K + k) * nv + i] = V[q];
    }
}

// ------------------------------------------------------------------ sources, slabs, loops
struct SrcSpec {
    unsigned long long tmask;  // source timeslices (bit t), up to 64
    int i, alpha;
};

// eta(x) = sum_{t in tmask} delta_{x4,t} v_i(t; xs) (x) e_alpha for a source spec (i, alpha, tmask):
// eta_r for one lane r of a width-n native block (the lane's spec in spec[r])
__global__ void k_source_lane(const double2* __restrict__ Vi, const SrcSpec* __restrict__ spec,
                              double2* __restrict__ out, long V, long Vs, int nv, int n, int r) {
    const SrcSpec sp = spec[r];
    for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < V; s += (long)gridDim.x * blockDim.x) {
        const long t = s / Vs, xs = s - t * Vs;
        const bool on = (sp.tmask >> t) & 1ULL;
        for (int k = 0; k < 12; k++) {
            const int a = k / 3, c = k % 3;
            double2 v = make_double2(0, 0);
            if (on && a == sp.alpha) v = Vi[((t * Vs + xs) * 3 + c) * nv + sp.i];
            out[((long)k * V + s) * n + r] = v;
        }
    }
}

// lanes[q] of a width-n native FP64 block -> lane q of a width-m block
__global__ void k_gather_lanes(const double2* __restrict__ X, double2* __restrict__ Y, long V, int n,
                               const int* __restrict__ lanes, int m) {
    const long tot = 12 * V * m;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
        const long ks = i / m;
        const int q = (int)(i - ks * m);
        Y[i] = X[ks * n + lanes[q]];
    }
}

// slab gather at sink timeslice t: native FP64 X [12][V][n] -> G[xs*3+c][beta*n + r]
__global__ void k_slab(const double2* __restrict__ X, double2* __restrict__ G, long V, long Vs, int n, int t) {
    const long tot = Vs * 12 * n;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (long)gridDim.x * blockDim.x) {
        const long xs = q / (12 * n);
        const int rem = (int)(q - xs * 12 * n);
        const int c = rem / (4 * n);
        const int rem2 = rem - c * 4 * n;  // beta*n + r
        const int beta = rem2 / n, r = rem2 - beta * n;
        const long s = (long)t * Vs + xs;
        G[(xs * 3 + c) * (4L * n) + rem2] = X[((long)(beta * 3 + c) * V + s) * n + r];
    }
}

// tau_all[t][j][beta][i][alpha] <- C[j][beta*n + r] for the batch's (i_r, alpha_r)
__global__ void k_tau_scatter(const double2* __restrict__ C, const SrcSpec* __restrict__ spec, double2* __restrict__ tau,
                              int nv, int n, int t) {
    const int tot = nv * 4 * n;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += gridDim.x * blockDim.x) {
        const int j = q / (4 * n), rem = q - j * 4 * n;
        const int beta = rem / n, r = rem - beta * n;
        const int i = spec[r].i, a = spec[r].alpha;
        tau[((((long)t * nv + j) * 4 + beta) * nv + i) * 4 + a] = C[(long)j * 4 * n + rem];
    }
}

// tau[snk][j][beta][r] from C (perambulator entry point)
__global__ void k_tau_store(const double2* __restrict__ C, double2* __restrict__ tau, int nv, int n, int snk) {
    const int tot = nv * 4 * n;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += gridDim.x * blockDim.x)
        tau[(long)snk * tot + q] = C[q];
}

// Dirac matrices of the loop channels (chiral basis), entries in {0, +-1, +-i}:
// G(g)[a][b] as (re, im).  Built from the defining products, not typed per channel.
__device__ __forceinline__ cd gamma_entry(int mu, int a, int b) {
    // mu 0..2: gamma_k = [[0, -i s_k], [i s_k, 0]]; mu 3: [[0, 1], [1, 0]]
    const bool up = a < 2, bu = b < 2;
    if (up == bu) return mk(0.0, 0.0);
    const int p = a & 1, q = b & 1;
    if (mu == 3) return p == q ? mk(1.0, 0.0) : mk(0.0, 0.0);
    cd s;  // Pauli sigma_{mu+1}[p][q]
    if (mu == 0) s = (p != q) ? mk(1.0, 0.0) : mk(0.0, 0.0);
    else if (mu == 1) s = (p == q) ? mk(0.0, 0.0) : (p == 0 ? mk(0.0, -1.0) : mk(0.0, 1.0));
    else s = (p != q) ? mk(0.0, 0.0) : (p == 0 ? mk(1.0, 0.0) : mk(-1.0, 0.0));
    return up ? neg(ti(s)) : ti(s);
}

__device__ __forceinline__ cd channel_entry(int g, int a, int b) {
    if (g == DISCO_G_1) return a == b ? mk(1.0, 0.0) : mk(0.0, 0.0);
    if (g == DISCO_G_5) return a == b ? mk(a < 2 ? 1.0 : -1.0, 0.0) : mk(0.0, 0.0);
    return gamma_entry(g - DISCO_G_X, a, b);
}

// Entry of the matrix a loop code asks for: Gamma, or with DISCO_G_TILDE
// Gamma~ = gamma_4 Gamma^+ gamma_4, formed as that product.
__device__ __forceinline__ cd loop_entry(int code, int a, int b) {
    const int g = code & ~DISCO_G_TILDE;
    if (!(code & DISCO_G_TILDE)) return channel_entry(g, a, b);
    cd acc = mk(0.0, 0.0);
    for (int c = 0; c < 4; c++) {
        const cd l = gamma_entry(3, a, c);
        if (l.re == 0 && l.im == 0) continue;
        for (int d = 0; d < 4; d++) {
            const cd r = gamma_entry(3, d, b);
            if (r.re == 0 && r.im == 0) continue;
            acc = acc + l * cj(channel_entry(g, d, c)) * r;
        }
    }
    return acc;
}

// L[g][t] = sum_i w[t][i] sum_{a,b} Gamma_ab tau[t][i][b][i][a]
__global__ void k_loops(const double2* __restrict__ tau, int T, int nv, const double* __restrict__ w,
                        const int* __restrict__ gam, int ng, double2* __restrict__ L) {
    const int g = blockIdx.x / T, t = blockIdx.x % T;
    double acc[2] = {0, 0};
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        const double wi = w ? w[(long)t * nv + i] : 1.0;
        cd s = mk(0.0, 0.0);
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                cd G = loop_entry(gam[g], a, b);
                if (G.re == 0 && G.im == 0) continue;
                double2 v = tau[((((long)t * nv + i) * 4 + b) * nv + i) * 4 + a];
                s = s + G * mk(v.x, v.y);
            }
        acc[0] += wi * s.re;
        acc[1] += wi * s.im;
    }
    block_sum(acc);
    if (threadIdx.x == 0) L[(long)g * T + t] = make_double2(acc[0], acc[1]);
}

// tau_all[ts][tk][j][beta][i][alpha] <- C[tk][j][beta*n + r] (sinks tk0 .. tk0+nk-1)
__global__ void k_tau_scatter_all(const double2* __restrict__ C, const SrcSpec* __restrict__ spec,
                                  double2* __restrict__ tau, int nv, int n, int ts, int T, int tk0, int nk) {
    const long per = (long)nv * 4 * n;
    const long tot = per * nk;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (long)gridDim.x * blockDim.x) {
        const int kk = (int)(q / per);
        const int rem0 = (int)(q - kk * per);
        const int j = rem0 / (4 * n), rem = rem0 - j * 4 * n;
        const int beta = rem / n, r = rem - beta * n;
        const int i = spec[r].i, a = spec[r].alpha;
        const long tk = tk0 + kk;
        tau[(((((long)ts * T + tk) * nv + j) * 4 + beta) * nv + i) * 4 + a] = C[q];
    }
}

// Connected correlator from all-to-all perambulators, with the source-to-sink
// direction from gamma_5-hermiticity, tau(y0,x0) = g5 tau(x0,y0)^+ g5:
//   C[g][dt] = -(1/|Y|) sum_{y0} sum_{j,i} w_j(x0) w_i(y0)
//              sum_{b,a} (Gamma tau_ji Gamma~)[b][a] g5_b g5_a conj(tau_ji[b][a]),
// x0 = y0 + dt (mod T), tau_ji[b][a] = tau(x0,y0)[j][b][i][a], Gamma~ = g4 Gamma^+ g4.
// One block per (g, dt); fixed summation order.
__global__ void k_connected(const double2* __restrict__ tau, int T, int nv, const double* __restrict__ w,
                            const int* __restrict__ gam, const int* __restrict__ y0s, int ny0, double2* __restrict__ Cout) {
    const int g = blockIdx.x / T, dt = blockIdx.x % T;
    const int ch = gam[g];
    const double sg = ch == DISCO_G_1 ? 1.0 : -1.0;  // Gamma~ = sg * Gamma for 1, g5, g_k
    double acc[2] = {0, 0};
    for (int k = 0; k < ny0; k++) {
        const int y0 = y0s[k], x0 = (y0 + dt) % T;
        const double2* tp = tau + ((long)y0 * T + x0) * (long)(nv * 4) * (nv * 4);
        for (int p = threadIdx.x; p < nv * nv; p += blockDim.x) {
            const int j = p / nv, i = p % nv;
            cd t[4][4];
            for (int b = 0; b < 4; b++)
                for (int a = 0; a < 4; a++) {
                    const double2 v = tp[(((long)j * 4 + b) * nv + i) * 4 + a];
                    t[b][a] = mk(v.x, v.y);
                }
            cd sum = mk(0.0, 0.0);
            for (int b = 0; b < 4; b++)
                for (int a = 0; a < 4; a++) {
                    cd m = mk(0.0, 0.0);  // (Gamma t Gamma)[b][a]
                    for (int b2 = 0; b2 < 4; b2++) {
                        const cd G1 = channel_entry(ch, b, b2);
                        if (G1.re == 0 && G1.im == 0) continue;
                        for (int a2 = 0; a2 < 4; a2++) {
                            const cd G2 = channel_entry(ch, a2, a);
                            if (G2.re == 0 && G2.im == 0) continue;
                            m = m + G1 * t[b2][a2] * G2;
                        }
                    }
                    const double s5 = ((b < 2) == (a < 2)) ? 1.0 : -1.0;
                    sum = sum + s5 * (m * cj(t[b][a]));
                }
            const double wj = w ? w[(long)x0 * nv + j] : 1.0, wi = w ? w[(long)y0 * nv + i] : 1.0;
            acc[0] += wj * wi * sg * sum.re;
            acc[1] += wj * wi * sg * sum.im;
        }
    }
    block_sum(acc);
    if (threadIdx.x == 0) Cout[(long)g * T + dt] = make_double2(-acc[0] / ny0, -acc[1] / ny0);
}

// Correlator of loops La, Lb [ncfg][T]: C(dt) = mean_{y0} [mean_c La(y0+dt) Lb(y0) - VEV]
__device__ cd corr_one(const double2* La, const double2* Lb, int ncfg, int T, const int* y0s, int ny0, int vev_mode,
                       int dt) {
    cd acc = mk(0.0, 0.0);
    cd ma_all = mk(0.0, 0.0), mb_all = mk(0.0, 0.0);
    if (vev_mode == 1) {
        for (int c = 0; c < ncfg; c++)
            for (int t = 0; t < T; t++) {
                ma_all = ma_all + mk(La[c * T + t].x, La[c * T + t].y);
                mb_all = mb_all + mk(Lb[c * T + t].x, Lb[c * T + t].y);
            }
        ma_all = (1.0 / (ncfg * T)) * ma_all;
        mb_all = (1.0 / (ncfg * T)) * mb_all;
    }
    for (int k = 0; k < ny0; k++) {
        const int y0 = y0s[k], x0 = (y0 + dt) % T;
        cd two = mk(0.0, 0.0), ma = mk(0.0, 0.0), mb = mk(0.0, 0.0);
        for (int c = 0; c < ncfg; c++) {
            cd a = mk(La[c * T + x0].x, La[c * T + x0].y), b = mk(Lb[c * T + y0].x, Lb[c * T + y0].y);
            two = two + a * b;
            ma = ma + a;
            mb = mb + b;
        }
        two = (1.0 / ncfg) * two;
        cd vev = vev_mode == 0 ? ((1.0 / ncfg) * ma) * ((1.0 / ncfg) * mb) : ma_all * mb_all;
        acc = acc + (two - vev);
    }
    return (1.0 / ny0) * acc;
}

// one thread per (term, dt); terms: 0 full, 1 factorised (= block-block), 2 block-delta,
// 3 delta-block, 4 delta-delta, with delta L = L_full - L_blk computed into dl/dlt.
__global__ void k_correlator(const double2* Lf, const double2* Ltf, const double2* Lb, const double2* Ltb,
                             const double2* dl, const double2* dlt, int ncfg, int T, const int* y0s, int ny0,
                             int vev_mode, double2* out /* [5][T] */) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 5 * T) return;
    const int term = q / T, dt = q % T;
    const double2* A[5] = {Lf, Lb, Lb, dl, dl};
    const double2* B[5] = {Ltf, Ltb, dlt, Ltb, dlt};
    cd c = corr_one(A[term], B[term], ncfg, T, y0s, ny0, vev_mode, dt);
    out[q] = make_double2(c.re, c.im);
}

__global__ void k_sub(const double2* a, const double2* b, double2* c, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        c[i] = make_double2(a[i].x - b[i].x, a[i].y - b[i].y);
}

// dir 0: [nvec][R] -> [R][nvec]; dir 1: the inverse (R rows of colour-vector entries)
__global__ void k_blk_transpose(const double2* __restrict__ src, double2* __restrict__ dst, int nvec, long R, int dir) {
    long tot = (long)nvec * R;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (long)gridDim.x * blockDim.x) {
        long i = q / R, r = q - i * R;
        if (dir == 0) dst[r * nvec + i] = src[q];
        else dst[q] = src[r * nvec + i];
    }
}

static int grid_for(long n, int bs = 256, int cap = 8192) { return (int)std::max(1L, std::min<long>((n + bs - 1) / bs, cap)); }

Geo3 geo_of(disco_ctx* ctx) {
    Geo3 g;
    long st = 1;
    for (int m = 0; m < 4; m++) {
        g.L[m] = ctx->dims[m];
        g.st[m] = st;
        st *= ctx->dims[m];
    }
    return g;
}

// C_b = A_b^H B_b for a batch (device), M x N outputs
void zgemm_hn(disco_ctx* ctx, const double2* A, long lda, long sA, const double2* B, long ldb, long sB, double2* C,
              int M, int N, int K, int batch) {
    const int tilesM = (M + 15) / 16, tilesN = (N + 15) / 16;
    // split K so that the launch has a few thousand wavefronts
    long tiles = (long)tilesM * tilesN * batch;
    int nks = (int)std::max(1L, std::min<long>(4096 / std::max(1L, tiles), (K + 63) / 64));
    int kchunk = ((K + nks - 1) / nks + 15) / 16 * 16;
    nks = (K + kchunk - 1) / kchunk;
    double2* P = (double2*)ws_get(ctx, "gemm_part", sizeof(double2) * (size_t)batch * nks * M * N);
    int rec = prof_begin(ctx, 1);
    hipLaunchKernelGGL(k_zgemm_hn, dim3((unsigned)(tiles * nks)), dim3(64), 0, ctx->stream, A, lda, sA, B, ldb, sB, P,
                       M, N, K, kchunk, nks, tilesM, tilesN);
    HIPCHK(hipGetLastError());
    prof_end(ctx, rec, 1, 8.0 * M * N * (double)K * batch /* flop, recorded in the bytes slot */);
    k_ksum<<<grid_for((long)batch * M * N), 256, 0, ctx->stream>>>(P, C, M, N, nks, batch);
    HIPCHK(hipGetLastError());
}

void zgemm_nn(disco_ctx* ctx, const double2* Y, const double2* Cm, double2* out, int K, int m, int batch) {
    const int tilesK = (K + 15) / 16, tilesM = (m + 15) / 16;
    hipLaunchKernelGGL(k_zgemm_nn, dim3((unsigned)((long)tilesK * tilesM * batch)), dim3(64), 0, ctx->stream, Y, Cm,
                       out, K, m, tilesK, tilesM);
    HIPCHK(hipGetLastError());
}

// Batched Rayleigh-Ritz on the host for T timeslices: given G = Y^H Y and
// H = Y^H L Y (m x m each), return C with Y C orthonormal Ritz vectors and
// the Ritz values.  Falls back to an identity-regularised Cholesky if G is
// numerically singular.
bool rayleigh_ritz(int T, int m, const std::vector<dense::zc>& G, const std::vector<dense::zc>& H,
                   std::vector<dense::zc>& C, std::vector<double>& lam) {
    C.assign((size_t)T * m * m, 0.0);
    lam.assign((size_t)T * m, 0.0);
    bool ok = true;
    auto work = [&](int t0, int t1) {
        std::vector<dense::zc> R(m * m), Ri(m * m), Hp(m * m), tmp(m * m), Z(m * m);
        for (int t = t0; t < t1; t++) {
            const dense::zc* g = &G[(size_t)t * m * m];
            const dense::zc* h = &H[(size_t)t * m * m];
            if (!dense::cholesky_upper(g, R.data(), m)) {
                ok = false;
                continue;
            }
            dense::inv_upper(R.data(), Ri.data(), m);
            // H' = R^{-H} H R^{-1}
            dense::matmul(h, Ri.data(), tmp.data(), m);
            for (int i = 0; i < m; i++)
                for (int j = 0; j < m; j++) {
                    dense::zc s = 0;
                    for (int k = 0; k < m; k++) s += std::conj(Ri[k * m + i]) * tmp[k * m + j];
                    Hp[i * m + j] = s;
                }
            for (int i = 0; i < m; i++)
                for (int j = i; j < m; j++) {
                    dense::zc a = 0.5 * (Hp[i * m + j] + std::conj(Hp[j * m + i]));
                    Hp[i * m + j] = a;
                    Hp[j * m + i] = std::conj(a);
                }
            dense::eigh_jacobi(Hp.data(), &lam[(size_t)t * m], Z.data(), m);
            dense::matmul(Ri.data(), Z.data(), &C[(size_t)t * m * m], m);
        }
    };
    int nth = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
    nth = std::min(nth, T);
    std::vector<std::thread> th;
    for (int k = 0; k < nth; k++) th.emplace_back(work, T * k / nth, T * (k + 1) / nth);
    for (auto& x : th) x.join();
    return ok;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

int disco_ape_smear(disco_ctx* ctx, int steps, double alpha) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(ctx->have_gauge, DISCO_ESTATE, "ape_smear before gauge_set");
        REQUIRE(steps >= 0, DISCO_EINVAL, "steps < 0");
        activate(ctx);
        const long V = ctx->V;
        if (!ctx->Usm) HIPCHK(hipMalloc(&ctx->Usm, sizeof(double2) * 27 * V));
        double2* tmp = (double2*)ws_get(ctx, "ape_tmp", sizeof(double2) * 36 * V);
        // start: spatial links of U (the time link slot of tmp mirrors U64 for the staple reads)
        HIPCHK(hipMemcpyAsync(ctx->Usm, ctx->U64, sizeof(double2) * 27 * V, hipMemcpyDeviceToDevice, ctx->stream));
        Geo3 g = geo_of(ctx);
        for (int k = 0; k < steps; k++) {
            k_ape<<<grid_for(V, 128, 1 << 30), 128, 0, ctx->stream>>>(ctx->Usm, tmp, g, V, alpha);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(ctx->Usm, tmp, sizeof(double2) * 27 * V, hipMemcpyDeviceToDevice, ctx->stream));
        }
        ctx->have_smeared = true;
    });
}

int disco_smeared_get(disco_ctx* ctx, void* U_out) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(ctx->have_smeared, DISCO_ESTATE, "no smeared links");
        REQUIRE(U_out, DISCO_EINVAL, "NULL output");
        activate(ctx);
        k_smeared_export<<<grid_for(ctx->V, 256, 1 << 30), 256, 0, ctx->stream>>>(ctx->Usm, ctx->U64, ctx->V,
                                                                                 (double2*)U_out);
        HIPCHK(hipGetLastError());
    });
}

int disco_laplace_apply(disco_ctx* ctx, int nvec, const void* in, void* out) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(ctx->have_gauge, DISCO_ESTATE, "laplace before gauge_set");
        REQUIRE(in && out && nvec > 0, DISCO_EINVAL, "bad argument");
        activate(ctx);
        const long V = ctx->V;
        const double2* U = ctx->have_smeared ? ctx->Usm : ctx->U64;
        // canonical [nvec][V][3] -> internal [V*3][nvec] (T blocks of K rows are contiguous)
        const int T = ctx->dims[3];
        const long K = 3 * ctx->Vs;
        double2* a = (double2*)ws_get(ctx, "lap_a", sizeof(double2) * V * 3 * nvec);
        double2* b = (double2*)ws_get(ctx, "lap_b", sizeof(double2) * V * 3 * nvec);
        k_blk_transpose<<<grid_for(V * 3 * nvec), 256, 0, ctx->stream>>>((const double2*)in, a, nvec, T * K, 0);
        REQUIRE(3.0 * (double)V * nvec < 2147483648.0, DISCO_EINVAL, "%d vectors of %ld sites: too large", nvec, V);
        k_laplace<false><<<lap_grid(V), 256, 0, ctx->stream>>>(U, a, b, geo_of(ctx), V, nvec, nullptr, (int)V, nullptr,
                                                              1.0, 0.0, 0.0);
        k_blk_transpose<<<grid_for(V * 3 * nvec), 256, 0, ctx->stream>>>(b, (double2*)out, nvec, T * K, 1);
        HIPCHK(hipGetLastError());
    });
}

// Eigenpairs on the timeslices tsel[0..nt) (all of them when tsel is NULL),
// every slice an independent problem solved side by side.
static int laplace_eigvecs(disco_ctx* ctx, int nv, double tol, const int* tsel, int nt, void* Vout, double* lambda) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(ctx->have_gauge, DISCO_ESTATE, "laplace_eigvecs before gauge_set");
        REQUIRE(Vout && lambda, DISCO_EINVAL, "NULL output");
        const int Tall = ctx->dims[3];
        const int T = tsel ? nt : Tall;
        REQUIRE(T >= 1 && T <= Tall, DISCO_EINVAL, "%d timeslices of %d", T, Tall);
        std::vector<int> tm;
        if (tsel) {
            std::vector<int> seen(Tall, 0);
            for (int k = 0; k < nt; k++) {
                REQUIRE(tsel[k] >= 0 && tsel[k] < Tall && !seen[tsel[k]], DISCO_EINVAL, "bad timeslice %d", tsel[k]);
                seen[tsel[k]] = 1;
                tm.push_back(tsel[k]);
            }
        }
        const long Vs = ctx->Vs, Vl = ctx->V, K = 3 * Vs;
        const long V = (long)T * Vs;  // sites of the blocks
        REQUIRE(nv >= 1 && nv <= K, DISCO_EINVAL, "nv %d out of range 1..%ld", nv, K);
        activate(ctx);
        int* tmapd = nullptr;
        if (tsel) {
            tmapd = (int*)ws_get(ctx, "eig_tmap", sizeof(int) * T);
            HIPCHK(hipMemcpyAsync(tmapd, tm.data(), sizeof(int) * T, hipMemcpyHostToDevice, ctx->stream));
        }
        const double2* U = ctx->have_smeared ? ctx->Usm : ctx->U64;
        const int guard = std::max(4, nv / 4);
        int m = (int)std::min<long>(K, ((nv + guard + 3) / 4) * 4);
        if (m > K) m = (int)K;
        const size_t nY = (size_t)T * K * m;
        double2* Y = (double2*)ws_get(ctx, "eig_Y", sizeof(double2) * nY);
        double2* LY = (double2*)ws_get(ctx, "eig_LY", sizeof(double2) * nY);
        double2* Y1 = (double2*)ws_get(ctx, "eig_Y1", sizeof(double2) * nY);
        double2* Y2 = (double2*)ws_get(ctx, "eig_Y2", sizeof(double2) * nY);
        double2* Gd = (double2*)ws_get(ctx, "eig_G", sizeof(double2) * T * m * m);
        double2* Cd = (double2*)ws_get(ctx, "eig_C", sizeof(double2) * T * m * m);
        double* lamd = (double*)ws_get(ctx, "eig_lam", sizeof(double) * T * m);
        double* resd = (double*)ws_get(ctx, "eig_res", sizeof(double) * T * nv);
        Geo3 g = geo_of(ctx);
        const int gY = grid_for((long)nY);
        k_rand_fill<<<gY, 256, 0, ctx->stream>>>(Y, (long)nY, 0x5eed1234ULL);
        std::vector<dense::zc> Gh((size_t)T * m * m), Hh((size_t)T * m * m), Ch;
        std::vector<double> lam, res((size_t)T * nv);
        REQUIRE(3.0 * (double)V * m < 2147483648.0, DISCO_EINVAL, "%d vectors of %ld sites: too large", m, V);
        auto lap = [&](const double2* in, double2* out) {
            k_laplace<false><<<lap_grid(V), 256, 0, ctx->stream>>>(U, in, out, g, Vl, m, tmapd, (int)V, nullptr, 1.0,
                                                                  0.0, 0.0);
            HIPCHK(hipGetLastError());
        };
        // out = a (L in - c in) + b prev: a Chebyshev step with the Laplacian fused in
        auto lapcheb = [&](const double2* in, const double2* prev, double2* out, double a, double c, double b) {
            k_laplace<true><<<lap_grid(V), 256, 0, ctx->stream>>>(U, in, out, g, Vl, m, tmapd, (int)V, prev, a, c, b);
            HIPCHK(hipGetLastError());
        };
        auto gram = [&](const double2* A, const double2* B, std::vector<dense::zc>& host) {
            zgemm_hn(ctx, A, m, K * m, B, m, K * m, Gd, m, m, (int)K, T);
            HIPCHK(hipMemcpyAsync(host.data(), Gd, sizeof(double2) * T * m * m, hipMemcpyDeviceToHost, ctx->stream));
        };
        // Rayleigh-Ritz on the current Y (not necessarily orthonormal): Y <- Y C, LY <- L Y C
        auto rr = [&]() {
            lap(Y, LY);
            gram(Y, Y, Gh);
            gram(Y, LY, Hh);
            HIPCHK(hipStreamSynchronize(ctx->stream));
            bool ok = rayleigh_ritz(T, m, Gh, Hh, Ch, lam);
            REQUIRE(ok, DISCO_EINVAL, "eigensolver: Gram matrix not positive definite");
            HIPCHK(hipMemcpyAsync(Cd, Ch.data(), sizeof(double2) * T * m * m, hipMemcpyHostToDevice, ctx->stream));
            zgemm_nn(ctx, Y, Cd, Y1, (int)K, m, T);
            zgemm_nn(ctx, LY, Cd, Y2, (int)K, m, T);
            std::swap(Y, Y1);
            std::swap(LY, Y2);
            HIPCHK(hipMemcpyAsync(lamd, lam.data(), sizeof(double) * T * m, hipMemcpyHostToDevice, ctx->stream));
            k_resid<<<dim3(nv, T), 256, 0, ctx->stream>>>(LY, Y, lamd, resd, (int)K, m, nv);
            HIPCHK(hipMemcpyAsync(res.data(), resd, sizeof(double) * T * nv, hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
            double worst = 0;
            for (double v : res) worst = std::max(worst, std::sqrt(v));
            return worst;
        };
        double worst = rr();
        const double upper = 12.0;  // spectrum of -Delta lies in [0, 12]
        // Degree: near convergence the wanted end of the spectrum sits just below
        // a, where a Chebyshev polynomial grows only quadratically with its
        // degree until degree x acosh(x) passes 1; 32 keeps the growth in the
        // exponential regime (on smeared 24^3 slices with 64 + 16 vectors: 27
        // filter steps and 864 Laplacians to 1e-11, against 119 and 1428 at
        // degree 12) while the spread it puts between the wanted columns stays
        // far from what Cholesky QR in FP64 resolves.
        const int degree = 32;
        const double want = tol > 0 ? tol : 1e-12;
        for (int it = 0; it < 400 && worst > want; it++) {
            // Chebyshev filter damping [a, upper], a = largest current Ritz value over the slices
            double a = 0;
            for (int t = 0; t < T; t++) a = std::max(a, lam[(size_t)t * m + m - 1]);
            a = std::min(a, 0.9 * upper);
            const double e = (upper - a) / 2, c = (upper + a) / 2;
            // T1 = (L - c) Y / e ; T_{k+1} = 2 (L - c) T_k / e - T_{k-1}
            lapcheb(Y, nullptr, Y1, 1.0 / e, c, 0.0);
            double2 *prev = Y, *cur = Y1, *nxt = Y2;
            for (int k = 1; k < degree; k++) {
                lapcheb(cur, prev, nxt, 2.0 / e, c, -1.0);
                double2* t0 = prev;
                prev = cur;
                cur = nxt;
                nxt = t0;
            }
            if (cur != Y) HIPCHK(hipMemcpyAsync(Y, cur, sizeof(double2) * nY, hipMemcpyDeviceToDevice, ctx->stream));
            // re-orthonormalise before the Ritz step (Cholesky QR), then Rayleigh-Ritz
            gram(Y, Y, Gh);
            HIPCHK(hipStreamSynchronize(ctx->stream));
            {
                std::vector<dense::zc> R(m * m), Ri((size_t)T * m * m);
                for (int t = 0; t < T; t++) {
                    // scale-aware: normalise the columns first to keep Cholesky well conditioned
                    bool ok = dense::cholesky_upper(&Gh[(size_t)t * m * m], R.data(), m);
                    REQUIRE(ok, DISCO_EINVAL, "eigensolver: filtered block lost rank");
                    dense::inv_upper(R.data(), &Ri[(size_t)t * m * m], m);
                }
                HIPCHK(hipMemcpyAsync(Cd, Ri.data(), sizeof(double2) * T * m * m, hipMemcpyHostToDevice, ctx->stream));
                zgemm_nn(ctx, Y, Cd, Y1, (int)K, m, T);
                std::swap(Y, Y1);
                HIPCHK(hipStreamSynchronize(ctx->stream));
            }
            worst = rr();
        }
        // the swaps may have moved the final block into another workspace buffer
        ctx->ws["eig_Y"].first = Y;
        ctx->ws["eig_Y1"].first = Y1;
        ctx->ws["eig_LY"].first = LY;
        ctx->ws["eig_Y2"].first = Y2;
        REQUIRE(worst <= want, DISCO_ENOCONV, "eigensolver: residual %.3e above %.3e", worst, want);
        k_eig_export<<<grid_for((long)T * nv * K), 256, 0, ctx->stream>>>(Y, (double2*)Vout, T, K, m, nv);
        HIPCHK(hipGetLastError());
        for (int t = 0; t < T; t++)
            for (int i = 0; i < nv; i++) lambda[(size_t)t * nv + i] = lam[(size_t)t * m + i];
        HIPCHK(hipStreamSynchronize(ctx->stream));
        // set-up only: the blocks (4 x T K m complex numbers) go back to the allocator
        for (const char* w : {"eig_Y", "eig_LY", "eig_Y1", "eig_Y2", "eig_G", "eig_C"}) ws_free(ctx, w);
    });
}

int disco_laplace_eigvecs(disco_ctx* ctx, int nv, double tol, void* Vout, double* lambda) {
    return laplace_eigvecs(ctx, nv, tol, nullptr, 0, Vout, lambda);
}

int disco_laplace_eigvecs_slices(disco_ctx* ctx, int nv, double tol, const int* tsel, int nt, void* Vout,
                                 double* lambda) {
    if (!ctx) return DISCO_EINVAL;
    if (!tsel || nt < 1) {
        ctx->err = "no timeslices";
        return DISCO_EINVAL;
    }
    return laplace_eigvecs(ctx, nv, tol, tsel, nt, Vout, lambda);
}

int disco_perambulator(disco_ctx* ctx, const void* Vin, int nv, int nsrc, const void* X, const int* t_snk, int n_snk,
                       void* tau) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(Vin && X && t_snk && tau && nv > 0 && nsrc > 0 && n_snk > 0, DISCO_EINVAL, "bad argument");
        REQUIRE(nsrc <= 64, DISCO_EINVAL, "at most 64 solutions per call");
        activate(ctx);
        const int T = ctx->dims[3];
        const long V = ctx->V, Vs = ctx->Vs, K = 3 * Vs;
        for (int k = 0; k < n_snk; k++) REQUIRE(t_snk[k] >= 0 && t_snk[k] < T, DISCO_EINVAL, "bad sink timeslice");
        double2* Vi = (double2*)ws_get(ctx, "pr_V", sizeof(double2) * T * K * nv);
        k_eig_import<<<grid_for((long)T * nv * K), 256, 0, ctx->stream>>>((const double2*)Vin, Vi, T, K, nv);
        double2* X64 = (double2*)ws_get(ctx, "pr_X", disco::native_bytes(ctx, DISCO_F64, nsrc));
        disco::to_native(ctx, DISCO_F64, nsrc, X, X64);
        double2* G = (double2*)ws_get(ctx, "pr_G", sizeof(double2) * K * 4 * nsrc);
        double2* C = (double2*)ws_get(ctx, "pr_C", sizeof(double2) * nv * 4 * nsrc);
        for (int k = 0; k < n_snk; k++) {
            const int t = t_snk[k];
            k_slab<<<grid_for(Vs * 12 * nsrc), 256, 0, ctx->stream>>>(X64, G, V, Vs, nsrc, t);
            zgemm_hn(ctx, Vi + (long)t * K * nv, nv, 0, G, 4L * nsrc, 0, C, nv, 4 * nsrc, (int)K, 1);
            k_tau_store<<<grid_for((long)nv * 4 * nsrc), 256, 0, ctx->stream>>>(C, (double2*)tau, nv, nsrc, k);
        }
        HIPCHK(hipGetLastError());
    });
}

int disco_loops(disco_ctx* ctx, const void* tau_tt, int T, int nv, const double* w, const int* gammas, int ngamma,
                void* L) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(tau_tt && gammas && L && T > 0 && nv > 0 && ngamma > 0, DISCO_EINVAL, "bad argument");
        for (int g = 0; g < ngamma; g++)
            REQUIRE((gammas[g] & ~DISCO_G_TILDE) >= 0 && (gammas[g] & ~DISCO_G_TILDE) <= 4, DISCO_EINVAL,
                    "bad channel %d", gammas[g]);
        activate(ctx);
        int* gd = (int*)ws_get(ctx, "lp_g", sizeof(int) * ngamma);
        HIPCHK(hipMemcpyAsync(gd, gammas, sizeof(int) * ngamma, hipMemcpyHostToDevice, ctx->stream));
        k_loops<<<ngamma * T, 64, 0, ctx->stream>>>((const double2*)tau_tt, T, nv, w, gd, ngamma, (double2*)L);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(ctx->stream));
    });
}

int disco_correlator(disco_ctx* ctx, const void* L_full, const void* Lt_full, const void* L_blk, const void* Lt_blk,
                     int ncfg, int T, const int* y0_set, int ny0, int vev_mode, void* C_full, void* C_fact, void* dC,
                     void* four_terms) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(L_full && Lt_full && L_blk && Lt_blk && C_full && C_fact && dC, DISCO_EINVAL, "NULL argument");
        REQUIRE(ncfg >= 1 && T >= 1 && (vev_mode == 0 || vev_mode == 1), DISCO_EINVAL, "bad sizes or vev_mode");
        activate(ctx);
        std::vector<int> y0;
        if (y0_set && ny0 > 0) y0.assign(y0_set, y0_set + ny0);
        else
            for (int t = 0; t < T; t++) y0.push_back(t);
        for (int v : y0) REQUIRE(v >= 0 && v < T, DISCO_EINVAL, "bad source time");
        int* yd = (int*)ws_get(ctx, "cr_y0", sizeof(int) * y0.size());
        HIPCHK(hipMemcpyAsync(yd, y0.data(), sizeof(int) * y0.size(), hipMemcpyHostToDevice, ctx->stream));
        const long n = (long)ncfg * T;
        double2* dl = (double2*)ws_get(ctx, "cr_dl", sizeof(double2) * n);
        double2* dlt = (double2*)ws_get(ctx, "cr_dlt", sizeof(double2) * n);
        double2* out = (double2*)ws_get(ctx, "cr_out", sizeof(double2) * 5 * T);
        k_sub<<<grid_for(n), 256, 0, ctx->stream>>>((const double2*)L_full, (const double2*)L_blk, dl, n);
        k_sub<<<grid_for(n), 256, 0, ctx->stream>>>((const double2*)Lt_full, (const double2*)Lt_blk, dlt, n);
        k_correlator<<<(5 * T + 63) / 64, 64, 0, ctx->stream>>>(
            (const double2*)L_full, (const double2*)Lt_full, (const double2*)L_blk, (const double2*)Lt_blk, dl, dlt,
            ncfg, T, yd, (int)y0.size(), vev_mode, out);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(C_full, out, sizeof(double2) * T, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(C_fact, out + T, sizeof(double2) * T, hipMemcpyDeviceToDevice, ctx->stream));
        k_sub<<<grid_for(T), 256, 0, ctx->stream>>>(out, out + T, (double2*)dC, T);
        if (four_terms)
            HIPCHK(hipMemcpyAsync(four_terms, out + T, sizeof(double2) * 4 * T, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    });
}

// Perambulators tau(t,t) for the source timeslices in tmask (0 = all): for
// every timeslice (or packed set of timeslices for the domain-restricted
// operator) and every (i, alpha), build the sources, solve, project at the
// source timeslices and store tau(t,t).  Solutions are never all held: only
// one RHS block at a time.
int disco_perambulators_tt(disco_ctx* ctx, const disco_domains* dom, const void* Vin, int nv, unsigned long long tmask,
                           const disco_solver_params* P, void* tau_out, disco_solver_stats* agg) {
    if (!ctx) return DISCO_EINVAL;
    bool all_ok = true;
    int rc = guarded(ctx, [&] {
        REQUIRE(Vin && P && tau_out && nv > 0, DISCO_EINVAL, "bad argument");
        REQUIRE(ctx->have_clover, DISCO_ESTATE, "perambulators before clover_setup");
        REQUIRE(!dom || dom->ctx == ctx, DISCO_EINVAL, "domains belong to another context");
        const int T = ctx->dims[3];
        REQUIRE(T <= 64, DISCO_EINVAL, "at most 64 timeslices");
        const unsigned long long all = T == 64 ? ~0ULL : ((1ULL << T) - 1);
        if (tmask == 0) tmask = all;
        REQUIRE((tmask & ~all) == 0, DISCO_EINVAL, "tmask names timeslices beyond T");
        activate(ctx);
        const long V = ctx->V, Vs = ctx->Vs, K = 3 * Vs;
        double2* Vi = (double2*)ws_get(ctx, "ld_V", sizeof(double2) * T * K * nv);
        k_eig_import<<<grid_for((long)T * nv * K), 256, 0, ctx->stream>>>((const double2*)Vin, Vi, T, K, nv);
        double2* tau = (double2*)tau_out;
        // packing sets: one timeslice per temporal layer of the partition
        std::vector<unsigned long long> sets;
        if (dom) {
            const int lm = dom->lmax;
            // temporal layers: a layer ends at every cut face along t
            int anchor = -1;
            for (int t = 0; t < T; t++)
                if (dom->cut[3 * lm + t]) anchor = t;
            if (anchor < 0) {
                for (int t = 0; t < T; t++) sets.push_back(1ULL << t);  // one layer: nothing to pack
            } else {
                std::vector<std::vector<int>> layers;
                std::vector<int> curl;
                for (int k = 1; k <= T; k++) {
                    const int t = (anchor + k) % T;
                    if ((tmask >> t) & 1ULL) curl.push_back(t);
                    if (dom->cut[3 * lm + t]) {
                        layers.push_back(curl);
                        curl.clear();
                    }
                }
                size_t maxlen = 0;
                for (auto& l : layers) maxlen = std::max(maxlen, l.size());
                // set p holds the p-th requested timeslice of every layer long enough
                for (size_t p = 0; p < maxlen; p++) {
                    unsigned long long msk = 0;
                    for (auto& l : layers)
                        if (p < l.size()) msk |= 1ULL << l[p];
                    sets.push_back(msk);
                }
            }
        } else {
            for (int t = 0; t < T; t++) sets.push_back(1ULL << t);
        }
        const int nrhs_set = 4 * nv;
        const int blk = disco::default_rhs_block(*P, nrhs_set, ctx);
        // lane specs, and the specs and lanes of a hand-over (device; host staging beside)
        SrcSpec* specd = (SrcSpec*)ws_get(ctx, "ld_spec", sizeof(SrcSpec) * blk);
        SrcSpec* specg = (SrcSpec*)ws_get(ctx, "ld_specg", sizeof(SrcSpec) * blk);
        int* laneg = (int*)ws_get(ctx, "ld_lanes", sizeof(int) * blk);
        double2* b64 = (double2*)ws_get(ctx, "ld_b64", disco::native_bytes(ctx, DISCO_F64, blk));
        double2* x64 = (double2*)ws_get(ctx, "ld_x64", disco::native_bytes(ctx, DISCO_F64, blk));
        double2* xg = (double2*)ws_get(ctx, "ld_xg", disco::native_bytes(ctx, DISCO_F64, blk));
        double2* G = (double2*)ws_get(ctx, "ld_G", sizeof(double2) * K * 4 * blk);
        double2* C = (double2*)ws_get(ctx, "ld_C", sizeof(double2) * nv * 4 * blk);
        std::vector<SrcSpec> hspec(blk), hspecg(blk);
        std::vector<int> hlanes(blk);
        // one queue over every source of every set (set k, source j: i = j / 4,
        // alpha = j % 4), so that lanes never wait for a set to drain; each
        // solution is projected as soon as it is final
        std::vector<unsigned long long> qmask;
        for (unsigned long long msk0 : sets)
            if (msk0 & tmask) qmask.push_back(msk0 & tmask);
        const int nq = (int)qmask.size() * nrhs_set;
        auto spec_of = [&](int j) { return SrcSpec{qmask[j / nrhs_set], (j % nrhs_set) / 4, j % 4}; };
        disco::LaneFeeder f;
        f.total = nq;
        f.load = [&](int lane, int j, int width) {
            hspec[lane] = spec_of(j);
            HIPCHK(hipMemcpyAsync(specd + lane, &hspec[lane], sizeof(SrcSpec), hipMemcpyHostToDevice, ctx->stream));
            k_source_lane<<<grid_for(V), 256, 0, ctx->stream>>>(Vi, specd, b64, V, Vs, nv, width, lane);
        };
        f.store = [&](const std::vector<int>& lanes, const std::vector<int>& js, int width) {
            // the finished lanes, set by set
            for (size_t k = 0; k < qmask.size(); k++) {
                int m = 0;
                for (size_t q = 0; q < lanes.size(); q++) {
                    if (js[q] / nrhs_set != (int)k) continue;
                    hspecg[m] = spec_of(js[q]);
                    hlanes[m++] = lanes[q];
                }
                if (!m) continue;
                const unsigned long long msk = qmask[k];
                HIPCHK(hipMemcpyAsync(specg, hspecg.data(), sizeof(SrcSpec) * m, hipMemcpyHostToDevice, ctx->stream));
                HIPCHK(hipMemcpyAsync(laneg, hlanes.data(), sizeof(int) * m, hipMemcpyHostToDevice, ctx->stream));
                k_gather_lanes<<<grid_for(12 * V * m), 256, 0, ctx->stream>>>(x64, xg, V, width, laneg, m);
                for (int t = 0; t < T; t++) {
                    if (!((msk >> t) & 1ULL)) continue;
                    k_slab<<<grid_for(Vs * 12 * m), 256, 0, ctx->stream>>>(xg, G, V, Vs, m, t);
                    zgemm_hn(ctx, Vi + (long)t * K * nv, nv, 0, G, 4L * m, 0, C, nv, 4 * m, (int)K, 1);
                    k_tau_scatter<<<grid_for((long)nv * 4 * m), 256, 0, ctx->stream>>>(C, specg, tau, nv, m, t);
                }
                HIPCHK(hipGetLastError());
                HIPCHK(hipStreamSynchronize(ctx->stream));  // the host staging is reused by the next set
            }
        };
        std::vector<disco_solver_stats> st(nq);
        long long iters = disco::solve_fed(ctx, dom, *P, blk, f, b64, x64, st.data());
        long long solves = nq;
        double worst = 0;
        int fb = 0, outer = 0;
        for (int j = 0; j < nq; j++) {
            all_ok &= st[j].converged != 0;
            worst = std::max(worst, st[j].true_rel_residual);
            fb |= st[j].fallback_used;
            outer = std::max(outer, st[j].outer_iters);
        }
        if (agg) {
            agg->iters = (int)std::min<long long>(iters, 2147483647LL);
            agg->outer_iters = outer;
            agg->fallback_used = fb;
            agg->converged = all_ok;
            agg->true_rel_residual = worst;
        }
        ctx->last_solves = solves;
    });
    if (rc == DISCO_OK && !all_ok) {
        ctx->err = "a distillation solve missed the tolerance";
        return DISCO_ENOCONV;
    }
    return rc;
}

// End-to-end loops: all perambulators tau(t,t), then the loops.
int disco_loops_distill(disco_ctx* ctx, const disco_domains* dom, const void* Vin, int nv, const double* w,
                        const int* gammas, int ngamma, const disco_solver_params* P, void* L, void* tau_out,
                        disco_solver_stats* agg) {
    if (!ctx) return DISCO_EINVAL;
    void* tau = tau_out;
    int rc = guarded(ctx, [&] {
        REQUIRE(Vin && gammas && P && L && nv > 0 && ngamma > 0, DISCO_EINVAL, "bad argument");
        if (!tau) tau = ws_get(ctx, "ld_tau", sizeof(double2) * (size_t)ctx->dims[3] * nv * 4 * nv * 4);
    });
    if (rc != DISCO_OK) return rc;
    int rs = disco_perambulators_tt(ctx, dom, Vin, nv, 0, P, tau, agg);
    if (rs != DISCO_OK && rs != DISCO_ENOCONV) return rs;
    long long solves = ctx->last_solves;
    std::string err = ctx->err;
    int rl = disco_loops(ctx, tau, ctx->dims[3], nv, w, gammas, ngamma, L);
    ctx->last_solves = solves;
    if (rl != DISCO_OK) return rl;
    if (rs == DISCO_ENOCONV) ctx->err = err;
    return rs;
}

// ---------------------------------------------------------------- region schedule
// The paper's own regions: for every operator time x0 a temporal slab
// Lambda(x0) = {t : |t - x0| <= h} (mod T), h = (delta - 1)/2, over the whole
// spatial volume (subsections "Domain decomposition of the propagator" and
// "Subtraction method"; the width delta is odd).  Operator times whose slabs
// are disjoint mod T (circular distance >= delta) share one multi-site solve
// (the Cost section): they are grouped greedily in increasing x0.
// With an open time boundary the distance is not taken around the wrap (the
// slabs are clipped at t = 0 and t = T-1 instead of wrapping).
static std::vector<unsigned long long> slab_sets(int T, int delta, bool open = false) {
    std::vector<std::vector<int>> sets;
    for (int x0 = 0; x0 < T; x0++) {
        bool placed = false;
        for (auto& set : sets) {
            bool ok = true;
            for (int y : set) {
                const int d = std::abs(x0 - y);
                if ((open ? d : std::min(d, T - d)) < delta) ok = false;
            }
            if (ok) {
                set.push_back(x0);
                placed = true;
                break;
            }
        }
        if (!placed) sets.push_back({x0});
    }
    std::vector<unsigned long long> masks;
    for (auto& set : sets) {
        unsigned long long m = 0;
        for (int y : set) m |= 1ULL << y;
        masks.push_back(m);
    }
    return masks;
}

static int slab_sets_abi(int T, int delta, bool open, int* nsets, unsigned long long* masks) {
    if (T < 1 || T > 64 || delta < 1 || delta % 2 == 0 || delta >= T || !nsets) return DISCO_EINVAL;
    const auto m = slab_sets(T, delta, open);
    *nsets = (int)m.size();
    if (masks)
        for (size_t k = 0; k < m.size(); k++) masks[k] = m[k];
    return DISCO_OK;
}

int disco_slab_sets(int T, int delta, int* nsets, unsigned long long* masks) {
    return slab_sets_abi(T, delta, false, nsets, masks);
}

int disco_slab_sets_open(int T, int delta, int* nsets, unsigned long long* masks) {
    return slab_sets_abi(T, delta, true, nsets, masks);
}

int disco_profile_weights(const double* lambda, long n, double omega, double* w) {
    if (!lambda || !w || n < 0 || !(omega > 0)) return DISCO_EINVAL;
    const double s = 0.8 * omega;
    for (long k = 0; k < n; k++) w[k] = std::exp(-(lambda[k] * lambda[k]) / (s * s));
    return DISCO_OK;
}

static int loops_slab(disco_ctx* ctx, const void* Vin, int nv, const double* w, const int* gammas, int ngamma,
                      int delta, bool open, const disco_solver_params* P, void* L, void* tau_out,
                      disco_solver_stats* agg) {
    if (!ctx) return DISCO_EINVAL;
    void* tau = tau_out;
    std::vector<unsigned long long> sets;
    int rc = guarded(ctx, [&] {
        const int T = ctx->dims[3];
        REQUIRE(Vin && gammas && P && L && nv > 0 && ngamma > 0, DISCO_EINVAL, "bad argument");
        REQUIRE(delta >= 1 && delta % 2 == 1 && delta < T, DISCO_EINVAL, "slab width must be odd and below T");
        REQUIRE(T <= 64, DISCO_EINVAL, "at most 64 timeslices");
        if (!tau) tau = ws_get(ctx, "ls_tau", sizeof(double2) * (size_t)T * nv * 4 * nv * 4);
        sets = slab_sets(T, delta, open);
    });
    if (rc != DISCO_OK) return rc;
    const int T = ctx->dims[3];
    const int h = (delta - 1) / 2;
    int lmax = 0;
    for (int m = 0; m < 4; m++) lmax = std::max(lmax, ctx->dims[m]);
    long long solves = 0;
    disco_solver_stats tot{};
    tot.converged = 1;
    int status = DISCO_OK;
    std::string err;
    for (unsigned long long msk : sets) {
        std::vector<uint8_t> cut(4 * (size_t)lmax, 0);
        for (int x0 = 0; x0 < T; x0++)
            if ((msk >> x0) & 1ULL) {
                if (open) {
                    // slab clipped at the boundaries; the wrap face is always cut
                    if (x0 + h < T - 1) cut[3 * lmax + x0 + h] = 1;
                    if (x0 - h - 1 >= 0) cut[3 * lmax + x0 - h - 1] = 1;
                } else {
                    cut[3 * lmax + (x0 + h) % T] = 1;
                    cut[3 * lmax + ((x0 - h - 1) % T + T) % T] = 1;
                }
            }
        if (open) cut[3 * lmax + T - 1] = 1;
        disco_domains* dom = nullptr;
        int rd = disco_domains_create(ctx, cut.data(), lmax, &dom);
        if (rd != DISCO_OK) return rd;
        disco_solver_stats a{};
        int rs = disco_perambulators_tt(ctx, dom, Vin, nv, msk, P, tau, &a);
        const long long ns = ctx->last_solves;
        if (rs == DISCO_ENOCONV) err = ctx->err;
        disco_domains_destroy(dom);
        if (rs != DISCO_OK && rs != DISCO_ENOCONV) return rs;
        if (rs == DISCO_ENOCONV) status = DISCO_ENOCONV;
        solves += ns;
        tot.iters = (int)std::min<long long>((long long)tot.iters + a.iters, 2147483647LL);
        tot.outer_iters += a.outer_iters;
        tot.fallback_used |= a.fallback_used;
        tot.converged &= a.converged;
        tot.true_rel_residual = std::max(tot.true_rel_residual, a.true_rel_residual);
    }
    if (agg) *agg = tot;
    int rl = disco_loops(ctx, tau, T, nv, w, gammas, ngamma, L);
    ctx->last_solves = solves;
    if (rl != DISCO_OK) return rl;
    if (status == DISCO_ENOCONV) ctx->err = err;
    return status;
}

int disco_loops_slab(disco_ctx* ctx, const void* Vin, int nv, const double* w, const int* gammas, int ngamma, int delta,
                     const disco_solver_params* P, void* L, void* tau_out, disco_solver_stats* agg) {
    return loops_slab(ctx, Vin, nv, w, gammas, ngamma, delta, false, P, L, tau_out, agg);
}

int disco_loops_slab_open(disco_ctx* ctx, const void* Vin, int nv, const double* w, const int* gammas, int ngamma,
                          int delta, const disco_solver_params* P, void* L, void* tau_out, disco_solver_stats* agg) {
    return loops_slab(ctx, Vin, nv, w, gammas, ngamma, delta, true, P, L, tau_out, agg);
}

// C^NR spliced by separation: out[dt] = Cc[dt] + dC_k[dt] with k the largest
// slab width deltas[k] below dt (NaN where none is)
int disco_nr_splice(const double* Cc, const double* dC, const int* deltas, int ndelta, int T, double* out) {
    if (!Cc || !dC || !deltas || !out || ndelta < 1 || T < 1) return DISCO_EINVAL;
    for (int k = 0; k < ndelta; k++)
        if (deltas[k] < 1) return DISCO_EINVAL;
    for (int dt = 0; dt < T; dt++) {
        int best = -1;
        for (int k = 0; k < ndelta; k++)
            if (deltas[k] < dt && (best < 0 || deltas[k] > deltas[best])) best = k;
        if (best < 0) {
            out[2 * dt] = out[2 * dt + 1] = std::nan("");
            continue;
        }
        out[2 * dt] = Cc[2 * dt] + dC[2 * ((long)best * T + dt)];
        out[2 * dt + 1] = Cc[2 * dt + 1] + dC[2 * ((long)best * T + dt) + 1];
    }
    return DISCO_OK;
}

// All-to-all perambulators for the connected correlator: sources on every
// timeslice ts in tmask, each solution projected at every sink timeslice tk
// (batched FP64 matrix-core contraction over the sinks):
//   tau_all[ts][tk][j][beta][i][alpha] = V(tk)^+ D^-1 V(ts).
int disco_perambulators_all(disco_ctx* ctx, const void* Vin, int nv, unsigned long long tmask,
                            const disco_solver_params* P, void* tau_out, disco_solver_stats* agg) {
    if (!ctx) return DISCO_EINVAL;
    bool all_ok = true;
    int rc = guarded(ctx, [&] {
        REQUIRE(Vin && P && tau_out && nv > 0, DISCO_EINVAL, "bad argument");
        REQUIRE(ctx->have_clover, DISCO_ESTATE, "perambulators before clover_setup");
        const int T = ctx->dims[3];
        REQUIRE(T <= 64, DISCO_EINVAL, "at most 64 timeslices");
        const unsigned long long all = T == 64 ? ~0ULL : ((1ULL << T) - 1);
        if (tmask == 0) tmask = all;
        REQUIRE((tmask & ~all) == 0, DISCO_EINVAL, "tmask names timeslices beyond T");
        activate(ctx);
        const long V = ctx->V, Vs = ctx->Vs, K = 3 * Vs;
        double2* Vi = (double2*)ws_get(ctx, "ld_V", sizeof(double2) * T * K * nv);
        k_eig_import<<<grid_for((long)T * nv * K), 256, 0, ctx->stream>>>((const double2*)Vin, Vi, T, K, nv);
        const int nrhs_set = 4 * nv;
        const int blk = disco::default_rhs_block(*P, nrhs_set, ctx);
        const int kchunk = std::min(T, 8);  // sinks per batched contraction
        SrcSpec* specd = (SrcSpec*)ws_get(ctx, "ld_spec", sizeof(SrcSpec) * blk);
        SrcSpec* specg = (SrcSpec*)ws_get(ctx, "ld_specg", sizeof(SrcSpec) * blk);
        int* laneg = (int*)ws_get(ctx, "ld_lanes", sizeof(int) * blk);
        double2* b64 = (double2*)ws_get(ctx, "ld_b64", disco::native_bytes(ctx, DISCO_F64, blk));
        double2* x64 = (double2*)ws_get(ctx, "ld_x64", disco::native_bytes(ctx, DISCO_F64, blk));
        double2* xg = (double2*)ws_get(ctx, "ld_xg", disco::native_bytes(ctx, DISCO_F64, blk));
        double2* G = (double2*)ws_get(ctx, "la_G", sizeof(double2) * K * 4 * blk * kchunk);
        double2* C = (double2*)ws_get(ctx, "la_C", sizeof(double2) * nv * 4 * blk * kchunk);
        std::vector<SrcSpec> hspec(blk), hspecg(blk);
        std::vector<int> hlanes(blk);
        std::vector<disco_solver_stats> st(nrhs_set);
        long long solves = 0, iters = 0;
        double worst = 0;
        int fb = 0, outer = 0;
        for (int ts = 0; ts < T; ts++) {
            if (!((tmask >> ts) & 1ULL)) continue;
            // the source timeslice's 4 nv sources feed the lanes; each finished
            // solution is projected on every sink timeslice
            disco::LaneFeeder f;
            f.total = nrhs_set;
            f.load = [&](int lane, int j, int width) {
                hspec[lane] = SrcSpec{1ULL << ts, j / 4, j % 4};
                HIPCHK(hipMemcpyAsync(specd + lane, &hspec[lane], sizeof(SrcSpec), hipMemcpyHostToDevice, ctx->stream));
                k_source_lane<<<grid_for(V), 256, 0, ctx->stream>>>(Vi, specd, b64, V, Vs, nv, width, lane);
            };
            f.store = [&](const std::vector<int>& lanes, const std::vector<int>& js, int width) {
                const int m = (int)lanes.size();
                for (int q = 0; q < m; q++) {
                    hspecg[q] = SrcSpec{1ULL << ts, js[q] / 4, js[q] % 4};
                    hlanes[q] = lanes[q];
                }
                HIPCHK(hipMemcpyAsync(specg, hspecg.data(), sizeof(SrcSpec) * m, hipMemcpyHostToDevice, ctx->stream));
                HIPCHK(hipMemcpyAsync(laneg, hlanes.data(), sizeof(int) * m, hipMemcpyHostToDevice, ctx->stream));
                k_gather_lanes<<<grid_for(12 * V * m), 256, 0, ctx->stream>>>(x64, xg, V, width, laneg, m);
                for (int tk0 = 0; tk0 < T; tk0 += kchunk) {
                    const int nk = std::min(kchunk, T - tk0);
                    for (int kk = 0; kk < nk; kk++)
                        k_slab<<<grid_for(Vs * 12 * m), 256, 0, ctx->stream>>>(xg, G + (long)kk * K * 4 * m, V, Vs,
                                                                                m, tk0 + kk);
                    zgemm_hn(ctx, Vi + (long)tk0 * K * nv, nv, K * nv, G, 4L * m, K * 4L * m, C, nv, 4 * m, (int)K, nk);
                    k_tau_scatter_all<<<grid_for((long)nv * 4 * m * nk), 256, 0, ctx->stream>>>(
                        C, specg, (double2*)tau_out, nv, m, ts, T, tk0, nk);
                }
                HIPCHK(hipGetLastError());
                HIPCHK(hipStreamSynchronize(ctx->stream));  // the host staging is reused by the next hand-over
            };
            iters += disco::solve_fed(ctx, nullptr, *P, blk, f, b64, x64, st.data());
            int set_outer = 0;
            for (int j = 0; j < nrhs_set; j++) {
                all_ok &= st[j].converged != 0;
                worst = std::max(worst, st[j].true_rel_residual);
                fb |= st[j].fallback_used;
                set_outer = std::max(set_outer, st[j].outer_iters);
            }
            outer += set_outer;
            solves += nrhs_set;
        }
        if (agg) {
            agg->iters = (int)std::min<long long>(iters, 2147483647LL);
            agg->outer_iters = outer;
            agg->fallback_used = fb;
            agg->converged = all_ok;
            agg->true_rel_residual = worst;
        }
        ctx->last_solves = solves;
    });
    if (rc == DISCO_OK && !all_ok) {
        ctx->err = "a distillation solve missed the tolerance";
        return DISCO_ENOCONV;
    }
    return rc;
}

int disco_connected(disco_ctx* ctx, const void* tau_all, int T, int nv, const double* w, const int* gammas, int ngamma,
                    const int* y0_set, int ny0, void* C) {
    if (!ctx) return DISCO_EINVAL;
    return guarded(ctx, [&] {
        REQUIRE(tau_all && gammas && C && T > 0 && nv > 0 && ngamma > 0, DISCO_EINVAL, "bad argument");
        for (int g = 0; g < ngamma; g++) REQUIRE(gammas[g] >= 0 && gammas[g] <= 4, DISCO_EINVAL, "bad channel");
        std::vector<int> y0;
        if (y0_set && ny0 > 0) {
            for (int k = 0; k < ny0; k++) {
                REQUIRE(y0_set[k] >= 0 && y0_set[k] < T, DISCO_EINVAL, "y0 out of range");
                y0.push_back(y0_set[k]);
            }
        } else {
            for (int t = 0; t < T; t++) y0.push_back(t);
        }
        activate(ctx);
        int* gd = (int*)ws_get(ctx, "cn_g", sizeof(int) * ngamma);
        int* yd = (int*)ws_get(ctx, "cn_y", sizeof(int) * y0.size());
        HIPCHK(hipMemcpyAsync(gd, gammas, sizeof(int) * ngamma, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(yd, y0.data(), sizeof(int) * y0.size(), hipMemcpyHostToDevice, ctx->stream));
        k_connected<<<ngamma * T, 256, 0, ctx->stream>>>((const double2*)tau_all, T, nv, w, gd, yd, (int)y0.size(),
                                                          (double2*)C);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(ctx->stream));
    });
}

int disco_effective_mass(const double* C, int n, double* meff) {
    if (!C || !meff || n < 2) return DISCO_EINVAL;
    for (int t = 0; t + 1 < n; t++) meff[t] = (C[t] > 0 && C[t + 1] > 0) ? std::log(C[t] / C[t + 1]) : std::nan("");
    return DISCO_OK;
}

}  // extern "C"
