/*
 * Plain FP64 CPU reference ("the oracle") for the Wilson-clover operator used
 * by the subtraction method for disconnected diagrams.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this code.  The GPU library never
 * links, calls or includes it, and it shares no code with the GPU library.
 *
 * Every routine here is the plain definition, written as loops over sites in
 * array-of-structures layout, with no blocking or reordering:
 *
 *   - the operator D of the Methodology section (Wilson-clover, the action
 *     named at the start of the Results section), in hopping normalisation
 *       D psi(x) = A(x) psi(x)
 *                - kappa sum_mu [ b (1 - g_mu) U_mu(x) psi(x+mu)
 *                               + b (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *     with A(x) = 1 + i csw kappa sum_{mu<nu} sigma_mu_nu Fhat_mu_nu(x),
 *     Fhat = (Q - Q^+)/8, Q the sum of the four plaquette leaves at x,
 *     sigma_mu_nu = (i/2)[g_mu, g_nu];  b = boundary phase of a hop that
 *     crosses the lattice wrap in direction mu (+1 periodic, -1 antiperiodic);
 *   - the domain-restricted operator D_Lambda of the "Domain decomposition of
 *     the propagator" subsection: D restricted to the quark fields inside each
 *     domain, i.e. the same operator with every hop that crosses a domain face
 *     removed (Dirichlet boundaries) and A(x) unchanged;
 *   - D^+ = g5 D g5;
 *   - CGNR (conjugate gradients on D^+ D) for D x = b.
 *
 * Layouts: site s = x + Lx(y + Ly(z + Lz t)); links U[s][mu][a][b];
 * spinors psi[s][spin][colour]; clover A[s][12][12] with index spin*3+colour;
 * cut masks cut[mu*Lmax + x] = 1 when the face between x and x+1 (mod L_mu)
 * is a domain boundary.
 */
#include <omp.h>
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

/* gamma_1..gamma_4 in slots 0..3 (directions x,y,z,t), gamma_5 in slot 4 */
static cplx GM[5][4][4];
static int gm_ready = 0;

static void mat4_mul(cplx a[4][4], cplx b[4][4], cplx c[4][4])
{
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx s = 0;
            for (int k = 0; k < 4; k++) s += a[i][k] * b[k][j];
            c[i][j] = s;
        }
}

/* Euclidean hermitian gamma matrices in the chiral basis:
 *   g_k = [[0, -i s_k], [i s_k, 0]] (k = 1,2,3),  g_4 = [[0, 1], [1, 0]],
 *   g_5 = g_1 g_2 g_3 g_4 (computed, not typed in). */
static void init_gamma(void)
{
    if (gm_ready) return;
    cplx pauli[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GM, 0, sizeof(GM));
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                GM[k][a][2 + b] = -I * pauli[k][a][b];
                GM[k][2 + a][b] = I * pauli[k][a][b];
            }
    for (int a = 0; a < 2; a++) {
        GM[3][a][2 + a] = 1;
        GM[3][2 + a][a] = 1;
    }
    cplx t1[4][4], t2[4][4];
    mat4_mul(GM[0], GM[1], t1);
    mat4_mul(t1, GM[2], t2);
    mat4_mul(t2, GM[3], GM[4]);
    gm_ready = 1;
}

void orc_gamma(int mu, double* out /* 4x4 complex as 32 doubles */)
{
    init_gamma();
    memcpy(out, GM[mu], sizeof(cplx) * 16);
}

static long vol(const int d[4]) { return (long)d[0] * d[1] * d[2] * d[3]; }

static void coords(const int d[4], long s, int x[4])
{
    x[0] = (int)(s % d[0]); s /= d[0];
    x[1] = (int)(s % d[1]); s /= d[1];
    x[2] = (int)(s % d[2]); s /= d[2];
    x[3] = (int)s;
}

static long index_of(const int d[4], const int x[4])
{
    return x[0] + (long)d[0] * (x[1] + (long)d[1] * (x[2] + (long)d[2] * x[3]));
}

/* site reached from x by steps[mu] hops in each direction (periodic wrap) */
static long moved(const int d[4], const int x[4], int s0, int s1, int s2, int s3)
{
    int y[4] = {x[0] + s0, x[1] + s1, x[2] + s2, x[3] + s3};
    for (int m = 0; m < 4; m++) y[m] = ((y[m] % d[m]) + d[m]) % d[m];
    return index_of(d, y);
}

static const cplx* link(const cplx* U, long s, int mu) { return U + (s * 4 + mu) * 9; }

static void m3_mul(const cplx* a, const cplx* b, cplx* c)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += a[i * 3 + k] * b[k * 3 + j];
            c[i * 3 + j] = s;
        }
}

static void m3_dag(const cplx* a, cplx* c)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) c[i * 3 + j] = conj(a[j * 3 + i]);
}

/* product of four 3x3 matrices, each optionally daggered */
static void m3_chain4(const cplx* m[4], const int dag[4], cplx* out)
{
    cplx a[9], b[9], t[9];
    if (dag[0]) m3_dag(m[0], a); else memcpy(a, m[0], sizeof(a));
    for (int k = 1; k < 4; k++) {
        if (dag[k]) m3_dag(m[k], b); else memcpy(b, m[k], sizeof(b));
        m3_mul(a, b, t);
        memcpy(a, t, sizeof(a));
    }
    memcpy(out, a, sizeof(a));
}

/* Clover term A(x) (12x12 per site, index spin*3+colour). */
void orc_clover(const int d[4], const cplx* U, double kappa, double csw, cplx* A)
{
    init_gamma();
    long V = vol(d);
    cplx sig[4][4][4][4];
    for (int mu = 0; mu < 4; mu++)
        for (int nu = 0; nu < 4; nu++) {
            cplx p[4][4], q[4][4];
            mat4_mul(GM[mu], GM[nu], p);
            mat4_mul(GM[nu], GM[mu], q);
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) sig[mu][nu][a][b] = 0.5 * I * (p[a][b] - q[a][b]);
        }
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        int x[4];
        coords(d, s, x);
        cplx* As = A + s * 144;
        for (int i = 0; i < 144; i++) As[i] = 0;
        for (int i = 0; i < 12; i++) As[i * 12 + i] = 1;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                int e[4] = {0, 0, 0, 0}, f[4] = {0, 0, 0, 0};
                e[mu] = 1;
                f[nu] = 1;
#define AT(a, b) moved(d, x, (a) * e[0] + (b) * f[0], (a) * e[1] + (b) * f[1], \
                       (a) * e[2] + (b) * f[2], (a) * e[3] + (b) * f[3])
                cplx Q[9] = {0}, leaf[9];
                /* x -> x+mu -> x+mu+nu -> x+nu -> x */
                {
                    const cplx* m[4] = {link(U, s, mu), link(U, AT(1, 0), nu),
                                        link(U, AT(0, 1), mu), link(U, s, nu)};
                    int dg[4] = {0, 0, 1, 1};
                    m3_chain4(m, dg, leaf);
                    for (int i = 0; i < 9; i++) Q[i] += leaf[i];
                }
                /* x -> x+nu -> x+nu-mu -> x-mu -> x */
                {
                    const cplx* m[4] = {link(U, s, nu), link(U, AT(-1, 1), mu),
                                        link(U, AT(-1, 0), nu), link(U, AT(-1, 0), mu)};
                    int dg[4] = {0, 1, 1, 0};
                    m3_chain4(m, dg, leaf);
                    for (int i = 0; i < 9; i++) Q[i] += leaf[i];
                }
                /* x -> x-mu -> x-mu-nu -> x-nu -> x */
                {
                    const cplx* m[4] = {link(U, AT(-1, 0), mu), link(U, AT(-1, -1), nu),
                                        link(U, AT(-1, -1), mu), link(U, AT(0, -1), nu)};
                    int dg[4] = {1, 1, 0, 0};
                    m3_chain4(m, dg, leaf);
                    for (int i = 0; i < 9; i++) Q[i] += leaf[i];
                }
                /* x -> x-nu -> x-nu+mu -> x+mu -> x */
                {
                    const cplx* m[4] = {link(U, AT(0, -1), nu), link(U, AT(0, -1), mu),
                                        link(U, AT(1, -1), nu), link(U, s, mu)};
                    int dg[4] = {1, 0, 0, 1};
                    m3_chain4(m, dg, leaf);
                    for (int i = 0; i < 9; i++) Q[i] += leaf[i];
                }
#undef AT
                cplx F[9];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) F[i * 3 + j] = (Q[i * 3 + j] - conj(Q[j * 3 + i])) / 8.0;
                cplx c = I * csw * kappa;
                for (int a = 0; a < 4; a++)
                    for (int b = 0; b < 4; b++) {
                        cplx sab = sig[mu][nu][a][b];
                        if (sab == 0) continue;
                        for (int i = 0; i < 3; i++)
                            for (int j = 0; j < 3; j++)
                                As[(a * 3 + i) * 12 + (b * 3 + j)] += c * sab * F[i * 3 + j];
                    }
            }
    }
}

/* out = D in (dagger = 0) or D^+ in (dagger = 1); cut == NULL means the
 * full operator, otherwise the domain-restricted one. */
void orc_dirac(const int d[4], const int bc[4], const cplx* U, const cplx* A, double kappa,
               const unsigned char* cut, int Lmax, int dagger, const cplx* in, cplx* out)
{
    init_gamma();
    long V = vol(d);
    const cplx* src = in;
    cplx* tmp = NULL;
    if (dagger) {
        tmp = (cplx*)malloc(sizeof(cplx) * V * 12);
#pragma omp parallel for schedule(static)
        for (long s = 0; s < V; s++)
            for (int a = 0; a < 4; a++)
                for (int c = 0; c < 3; c++) {
                    cplx v = 0;
                    for (int b = 0; b < 4; b++) v += GM[4][a][b] * in[s * 12 + b * 3 + c];
                    tmp[s * 12 + a * 3 + c] = v;
                }
        src = tmp;
    }
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        int x[4];
        coords(d, s, x);
        cplx o[12];
        const cplx* As = A + s * 144;
        for (int i = 0; i < 12; i++) {
            cplx v = 0;
            for (int j = 0; j < 12; j++) v += As[i * 12 + j] * src[s * 12 + j];
            o[i] = v;
        }
        for (int mu = 0; mu < 4; mu++) {
            int L = d[mu];
            for (int dir = 0; dir < 2; dir++) {
                /* dir 0: forward hop to x+mu;  dir 1: backward hop to x-mu */
                int face = dir == 0 ? x[mu] : (x[mu] - 1 + L) % L;
                if (cut && cut[mu * Lmax + face]) continue;
                int crosses = dir == 0 ? (x[mu] == L - 1) : (x[mu] == 0);
                double ph = crosses ? (double)bc[mu] : 1.0;
                int st[4] = {0, 0, 0, 0};
                st[mu] = dir == 0 ? 1 : -1;
                long n = moved(d, x, st[0], st[1], st[2], st[3]);
                cplx M[9];
                if (dir == 0) memcpy(M, link(U, s, mu), sizeof(M));
                else m3_dag(link(U, n, mu), M);
                cplx v[12]; /* colour-rotated neighbour spinor */
                for (int a = 0; a < 4; a++)
                    for (int i = 0; i < 3; i++) {
                        cplx t = 0;
                        for (int j = 0; j < 3; j++) t += M[i * 3 + j] * src[n * 12 + a * 3 + j];
                        v[a * 3 + i] = t;
                    }
                double sg = dir == 0 ? -1.0 : 1.0; /* (1 - g) forward, (1 + g) backward */
                for (int a = 0; a < 4; a++)
                    for (int i = 0; i < 3; i++) {
                        cplx t = v[a * 3 + i];
                        for (int b = 0; b < 4; b++) t += sg * GM[mu][a][b] * v[b * 3 + i];
                        o[a * 3 + i] -= kappa * ph * t;
                    }
            }
        }
        for (int i = 0; i < 12; i++) out[s * 12 + i] = o[i];
    }
    if (dagger) {
#pragma omp parallel for schedule(static)
        for (long s = 0; s < V; s++) {
            cplx w[12];
            for (int a = 0; a < 4; a++)
                for (int c = 0; c < 3; c++) {
                    cplx v = 0;
                    for (int b = 0; b < 4; b++) v += GM[4][a][b] * out[s * 12 + b * 3 + c];
                    w[a * 3 + c] = v;
                }
            memcpy(out + s * 12, w, sizeof(w));
        }
        free(tmp);
    }
}

static double norm2(const cplx* a, long n)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long i = 0; i < n; i++) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/* CGNR for D x = b: CG on D^+ D x = D^+ b, iterated until the true residual
 * ||b - D x|| / ||b|| is at most tol.  Returns 0 on success, 1 when maxit is
 * reached first.  x is overwritten (start from zero). */
int orc_cgnr(const int d[4], const int bc[4], const cplx* U, const cplx* A, double kappa,
             const unsigned char* cut, int Lmax, const cplx* b, cplx* x, double tol, int maxit,
             int* iters_out, double* relres_out)
{
    long n = vol(d) * 12;
    cplx* r = (cplx*)malloc(sizeof(cplx) * n);
    cplx* z = (cplx*)malloc(sizeof(cplx) * n);
    cplx* p = (cplx*)malloc(sizeof(cplx) * n);
    cplx* w = (cplx*)malloc(sizeof(cplx) * n);
    double bb = norm2(b, n);
    int it = 0, status = 1;
    for (long i = 0; i < n; i++) x[i] = 0;
    double rel = 0;
    while (it < maxit) {
        /* (re)start from the true residual */
        orc_dirac(d, bc, U, A, kappa, cut, Lmax, 0, x, w);
        for (long i = 0; i < n; i++) r[i] = b[i] - w[i];
        rel = sqrt(norm2(r, n) / bb);
        if (rel <= tol) { status = 0; break; }
        orc_dirac(d, bc, U, A, kappa, cut, Lmax, 1, r, z);
        memcpy(p, z, sizeof(cplx) * n);
        double zz = norm2(z, n);
        while (it < maxit) {
            orc_dirac(d, bc, U, A, kappa, cut, Lmax, 0, p, w);
            double a = zz / norm2(w, n);
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; i++) {
                x[i] += a * p[i];
                r[i] -= a * w[i];
            }
            it++;
            /* leave the inner loop a little below tol and confirm with the true residual */
            if (norm2(r, n) <= 0.25 * tol * tol * bb) break;
            orc_dirac(d, bc, U, A, kappa, cut, Lmax, 1, r, z);
            double zn = norm2(z, n);
            double beta = zn / zz;
            zz = zn;
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        }
    }
    if (status) {
        orc_dirac(d, bc, U, A, kappa, cut, Lmax, 0, x, w);
        for (long i = 0; i < n; i++) r[i] = b[i] - w[i];
        rel = sqrt(norm2(r, n) / bb);
        if (rel <= tol) status = 0;
    }
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = rel;
    free(r); free(z); free(p); free(w);
    return status;
}

/* Timing helper (no arithmetic): set the OpenMP thread count of later calls
 * when n > 0 and return the previous maximum. */
int orc_set_threads(int n) {
    const int old = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return old;
}
