/*
 * libdisco: C ABI of the MI355X (gfx950) implementation of the hot path of the
 * subtraction method for disconnected diagrams ("Subtraction method for
 * disconnected diagrams in full QCD", Barca, Crawford, Finkenrath, Schaefer,
 * Urrea-Nino).
 *
 * The path: the Wilson-clover operator D and its domain-restricted form
 * D_Lambda (hops across domain faces removed) are inverted on distillation
 * sources; the solutions are projected as V^+ D^-1 V (perambulators); the
 * Gamma-traced quark loops per timeslice give the full, completely factorised
 * and subtracted disconnected correlators.
 *
 * General rules
 *   - Every function returns an int: DISCO_OK (0) or a negative DISCO_E* code.
 *     disco_last_error(ctx) returns a message for the last failure on ctx.
 *     No C++ exception or abort crosses this interface.
 *   - The caller owns every buffer it passes.  "device" pointers must point to
 *     memory on the context's GPU (hipMalloc or a torch tensor); "host"
 *     pointers to ordinary host memory.  Each argument says which.
 *   - The context owns its internal copies (links, clover term, smeared links,
 *     workspaces) and frees them in disco_destroy.
 *   - All GPU work is issued on the context's stream (disco_set_stream; the
 *     default is the null stream).  Functions that return host results
 *     synchronise that stream before returning; the others are asynchronous
 *     with respect to the host unless stated.
 *   - One context per host thread at a time.
 *
 * Boundary layouts (all complex numbers are (re, im) pairs of doubles)
 *   site index   s = x + Lx*(y + Ly*(z + Lz*t)); mu = 0,1,2,3 is x,y,z,t
 *   links        U[s][mu][a][b]                       complex128, SU(3)
 *   spinor field psi[s][spin][colour]                 complex128, 12 per site
 *   spinor block psi[r][s][spin][colour]              r = 0..nrhs-1
 *   eigenvectors Vev[t][i][xs][c], xs = x + Lx*(y + Ly*z)
 *   perambulator tau[t][j][beta][i][alpha]            sink (j,beta), source (i,alpha)
 *   loops        L[g][t]                              g over the requested channels
 *
 * Conventions: Euclidean hermitian gamma matrices in the chiral basis,
 *   gamma_k = [[0, -i s_k], [i s_k, 0]] (k = 1,2,3 for x,y,z),
 *   gamma_4 = [[0, 1], [1, 0]] (time), gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4
 *   = diag(1,1,-1,-1).
 */
#ifndef DISCO_H
#define DISCO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct disco_ctx disco_ctx;
typedef struct disco_domains disco_domains;
typedef struct disco_net disco_net;

enum {
    DISCO_OK = 0,
    DISCO_EINVAL = -1,     /* bad argument (sizes, pointers, non-SU(3) links, ...) */
    DISCO_ENOMEM = -2,     /* device or host allocation failed */
    DISCO_EHIP = -3,       /* a HIP runtime call failed */
    DISCO_ENOCONV = -4,    /* solver did not reach the tolerance (stats still filled) */
    DISCO_EBREAKDOWN = -5, /* Krylov breakdown and no fallback allowed */
    DISCO_ESTATE = -6      /* call made before the state it needs (gauge, clover) */
};

/* arithmetic / storage precisions */
enum { DISCO_F64 = 0, DISCO_F32 = 1, DISCO_BF16 = 2 };
/* where a pointer lives */
enum { DISCO_HOST = 0, DISCO_DEVICE = 1 };
/* loop channels Gamma; a loop code may add DISCO_G_TILDE to ask for the loop of
 * Gamma~ = gamma_4 Gamma^+ gamma_4, the matrix of the conjugate operator at the
 * source time of the disconnected correlator (Methodology, the definition under
 * equation Cdisc): +1, -gamma_5 and -gamma_k for 1, gamma_5 and gamma_k */
enum { DISCO_G_1 = 0, DISCO_G_5 = 1, DISCO_G_X = 2, DISCO_G_Y = 3, DISCO_G_Z = 4, DISCO_G_TILDE = 8 };
/* solver methods */
enum {
    DISCO_CGNR_F64 = 0,    /* conjugate gradients on D^+ D, all FP64 (plain judge) */
    DISCO_BICGSTAB_DC = 1, /* BiCGStab in inner_prec inside FP64 defect correction */
    DISCO_FGMRES_NN = 2,   /* flexible GMRES(restart), FP32 Krylov basis, preconditioned by a
                            * trained network (params.net), inside FP64 defect correction */
    DISCO_BICGSTAB_RU = 3  /* BiCGStab in inner_prec with reliable updates: one Krylov process
                            * for the whole solve; whenever a recursive residual has fallen by
                            * inner_tol (default 3e-2 for BF16, 1e-3 for FP32) the corrections
                            * are folded into the FP64 solution, the FP64 true residual replaces
                            * the recursive one and the process continues (lanes that break
                            * down or stall restart it; a correction that leaves a lane's true
                            * residual more than 4x above the previous update's is taken back
                            * and that lane restarts with a perturbed shadow residual);
                            * even-odd as for BICGSTAB_DC.  The
                            * right-hand sides of a call form one queue: a lane whose right-hand
                            * side has converged takes the next one at that update, so no lane
                            * waits for the slowest of its block */
};

/* ---------------------------------------------------------------- context */

/* Create a context for a dims[0..3] = (Lx,Ly,Lz,Lt) lattice on HIP device
 * `device`.  bc[mu] = +1 (periodic) or -1 (antiperiodic) is the phase of a
 * fermion hop that crosses the lattice wrap in direction mu.  Extents must be
 * >= 1 and the volume < 2^31.  *out receives the context (caller frees it with
 * disco_destroy). */
int disco_create(const int dims[4], const int bc[4], int device, disco_ctx** out);
int disco_destroy(disco_ctx* ctx);
/* Issue all later work on `hip_stream` (a hipStream_t; NULL = null stream). */
int disco_set_stream(disco_ctx* ctx, void* hip_stream);
/* Message for the last error on ctx (never NULL; "" when none).  With
 * ctx = NULL: the message of the last failed disco_create on the calling
 * thread, or "null context" when there was none. */
const char* disco_last_error(const disco_ctx* ctx);

/* ---------------------------------------------------------------- gauge / clover setup
 * Wilson-clover operator in hopping normalisation (the action named at the
 * start of the paper's Results section):
 *   D psi(x) = A(x) psi(x) - kappa sum_mu [ b (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                         + b (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *   A(x) = 1 + i csw kappa sum_{mu<nu} sigma_mu_nu Fhat_mu_nu(x),
 *   Fhat = (Q - Q^+)/8 with Q the sum of the four plaquette leaves at x,
 *   sigma_mu_nu = (i/2)[gamma_mu, gamma_nu], b the boundary phase of the hop. */

/* Load links U (boundary layout, complex128, V*4*9 entries) from host
 * (where = DISCO_HOST) or device memory.  Returns DISCO_EINVAL when a link is
 * not SU(3) to 1e-12 (max |U U^+ - 1|, |det U - 1|).  Invalidates the clover
 * term and the smeared links. */
int disco_gauge_set(disco_ctx* ctx, const void* U, int where);
/* Build A(x) from the current links (FP64 arithmetic; FP64 and FP32 copies
 * kept).  ESTATE before disco_gauge_set. */
int disco_clover_setup(disco_ctx* ctx, double kappa, double csw);
/* Copy the FP64 clover term out as [V][12][12] complex128 (index spin*3+colour)
 * into device memory `A_out` (for checks). */
int disco_clover_get(disco_ctx* ctx, void* A_out);

/* ---------------------------------------------------------------- domains
 * A separable partition of the lattice into domains Lambda_i (Domain
 * decomposition subsection).  cut[mu*lmax + x] = 1 (host, uint8) marks the
 * face between x and x+1 (mod L_mu) in direction mu as a domain boundary;
 * lmax >= max(dims).  All cuts zero gives a single domain. */
int disco_domains_create(disco_ctx* ctx, const uint8_t* cut, int lmax, disco_domains** out);
int disco_domains_destroy(disco_domains* dom);

/* ---------------------------------------------------------------- operators
 * out = D in (dagger = 0) or D^+ in = gamma_5 D gamma_5 in (dagger = 1) for nrhs
 * spinor fields in the boundary layout (device, complex128, nrhs*V*12
 * entries).  prec selects the arithmetic: DISCO_F64, DISCO_F32 (inputs
 * rounded to FP32, FP32 accumulation) or DISCO_BF16 (inputs rounded to BF16
 * storage, FP32 links and accumulation).  in and out must not overlap. */
int disco_dirac_apply(disco_ctx* ctx, int prec, int dagger, int nrhs, const void* in, void* out);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): disco_dirac_apply
 * without any allocation.  The two native-layout staging blocks live in a
 * fixed 256 MiB device array of the library, one per GPU, held until the
 * process ends; right-hand sides are processed in chunks that fit (at most 64
 * per launch).  EINVAL when a single right-hand side does not fit: its native
 * block, 192 V bytes in FP64, 96 V in FP32, 48 V in BF16, must not exceed
 * 128 MiB less 256 bytes (so 24^3 x 48 fits in every precision, 32^3 x 64 in
 * FP32 and BF16).
 * Every call on one GPU shares that array: calls that overlap on one GPU (two
 * contexts or streams on the same device) race and must be serialised by the
 * caller.  Launches of this call are not profiled.  Otherwise as
 * disco_dirac_apply, with the same kernels and results. */
int disco_dirac_apply_noalloc(disco_ctx* ctx, int prec, int dagger, int nrhs, const void* in, void* out);
/* Same with the domain-restricted operator D_Lambda of the Domain
 * decomposition subsection: D restricted to the fields inside each domain of
 * `dom` (Dirichlet faces): every hop across a cut face is dropped, A(x) is
 * unchanged. */
int disco_dirac_block_apply(disco_ctx* ctx, const disco_domains* dom, int prec, int dagger, int nrhs,
                            const void* in, void* out);

/* Internal ("native") layout of an nrhs block, for callers that keep fields
 * resident; element (plane, site s, rhs r) at (plane*V + s)*nrhs + r:
 *   F64  : [12][V][nrhs] complex double, plane k = spin*3 + colour
 *   F32  : [6][V][nrhs]  float4 = components (2p, 2p+1) as (re, im, re, im)
 *   BF16 : [3][V][nrhs]  16 bytes = components 4q..4q+3 as bf16 (re, im) pairs
 * disco_native_bytes gives the size of an nrhs block (nrhs <= 256 per call).
 * disco_dirac_apply_native takes at most min(256, (2^32 - 1) / (16 V)) right-
 * hand sides per call (one plane, V * nrhs * 16 bytes, must stay below 4 GiB),
 * else it fails with DISCO_EINVAL. */
long long disco_native_bytes(const disco_ctx* ctx, int prec, int nrhs);
int disco_to_native(disco_ctx* ctx, int prec, int nrhs, const void* in_canonical, void* out_native);
int disco_from_native(disco_ctx* ctx, int prec, int nrhs, const void* in_native, void* out_canonical);
/* out_native = D in_native on native blocks (dom = NULL for the full operator). */
int disco_dirac_apply_native(disco_ctx* ctx, const disco_domains* dom, int prec, int dagger, int nrhs,
                             const void* in_native, void* out_native);

/* Even-odd pieces of D (dom = NULL) or D_Lambda, exactly as the production
 * solver launches them.  The solvers work on the Schur complement of the even
 * sites, M = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe with D = A - kappa H (a
 * factorisation of D, not in the paper: it leaves D^-1 and so the loop under
 * equation Cdisc unchanged).  With p = parity (0 even, 1 odd sites, parity of
 * x+y+z+t):
 *   out(x) = ca aux(x) + A(x)^-1 [cg aux(x) + cb (H in)(x)]   at every x of parity p,
 * where H reads `in` at the sites of parity 1-p.  ca = 0, cg = 0, cb = 1 is the
 * first half of M (A_oo^-1 H_oe); ca = 1, cg = 0, cb = -kappa^2 its second
 * half; ca = 0, cg = 1, cb = kappa the even-odd source and the odd
 * reconstruction.  in, aux, aux2 (device, boundary layout complex128
 * [nrhs][V][4][3]; aux NULL unless ca, cg or a sum with it is asked for, aux2
 * NULL unless a sum with it is) are read only at the sites of the parity the
 * piece uses; each is first rounded to prec storage as the solver stores it
 * (FP32 links and A^-1 for FP32 and BF16).  out (device, same layout) is
 * written everywhere: the piece at parity p, zero at the other sites.  epi
 * selects the fused reductions of the launch: 0, DISCO_EPI_DOTAUX,
 * DISCO_EPI_NORM | DISCO_EPI_DOTIN, or all four; sums (host, [nrhs][4]
 * complex128, needed when epi != 0) receives per right-hand side
 * <aux2, out>, ||out||^2, <out, aux>, <aux2, aux> (<a, b> = sum conj(a) b over
 * the sites of parity p; out before its rounding to storage) at slots 0..3,
 * zero for the sums not asked for.  One launch of nrhs (1..64, and the plane
 * limit of disco_dirac_apply_native) right-hand sides: the solver's launch
 * shape for a block of that width.  EINVAL for odd extents. */
enum { DISCO_EPI_DOTAUX = 2, DISCO_EPI_NORM = 4, DISCO_EPI_DOTIN = 8, DISCO_EPI_DOTAUXIN = 16 };
int disco_dirac_eo_apply(disco_ctx* ctx, const disco_domains* dom, int prec, int parity, int nrhs, double ca,
                         double cg, double cb, int epi, const void* in, const void* aux, const void* aux2, void* out,
                         double* sums);

/* ---------------------------------------------------------------- options */
enum {
    DISCO_OPT_GRAPHS = 1, /* 1 (default): inner Krylov iterations run as captured HIP graphs
                           * (captured on a private stream, launched on the context stream;
                           * skipped while profiling is enabled); 0: eager launches */
    DISCO_OPT_STAGE = 2   /* LDS staging of links/clover in FP32/BF16 stencils: -1 auto
                           * (16 or more right-hand sides per launch), 0 off, 1 on */,
    DISCO_OPT_EO = 3      /* 1 (default): inner BiCGStab solves of BICGSTAB_DC run on the
                           * even-odd Schur complement M = 1 - kappa^2 A_ee^-1 H_eo A_oo^-1 H_oe
                           * (D = A - kappa H; half-lattice vectors) when every extent is even,
                           * with the source A_ee^-1 (r_e + kappa H_eo A_oo^-1 r_o) and the odd
                           * sites reconstructed as A_oo^-1 (r_o + kappa H_oe e_e); the FP64
                           * outer residual stays that of the full operator.  0: full operator */,
    DISCO_OPT_TILE_Y = 4, /* the stencil's site order: y rows per tile (a divisor of Ly; 0 = the
                           * default rule); each XCD of the chip takes a slab of Lt/8
                           * timeslices (when 8 divides Lt) and visits it x fastest, then the
                           * y rows of a tile, the timeslices of a tile, z, the y tiles, the t
                           * tiles, so that neighbours stay in its L2.  Setting it rewrites the
                           * order: each site's arithmetic is unchanged, so operator outputs
                           * are the same bit for bit; the solvers' fused sums group sites by
                           * this order and change by rounding */
    DISCO_OPT_TILE_T = 5, /* timeslices per tile inside the slab (a divisor of it; 0 = the whole
                           * slab).  disco_autotune sets both */
    DISCO_OPT_NARROW = 6  /* 1 (default): once the queue of a BICGSTAB_RU call is empty and at
                           * most half of the block's lanes are still open, those lanes move
                           * into a block of half the width (down to 16) and restart their
                           * Krylov processes from their current iterates; 0: the block keeps
                           * its width to the end */
};
int disco_set_option(disco_ctx* ctx, int option, int value);
/* The current value of an option; for the tile options, the extents the site
 * order was built with. */
int disco_get_option(const disco_ctx* ctx, int option, int* value);

/* ---------------------------------------------------------------- solver */
typedef struct {
    int method;        /* DISCO_CGNR_F64, DISCO_BICGSTAB_DC, DISCO_FGMRES_NN, DISCO_BICGSTAB_RU */
    double tol;        /* target true ||b - D x|| / ||b|| per right-hand side, FP64 */
    int max_iter;      /* cap on inner iterations summed over outer cycles (0 = 100000);
                        * BICGSTAB_RU: per wave of rhs_block right-hand sides of the queue,
                        * and its FP64 fallback runs up to 100000 iterations of its own */
    int inner_prec;    /* DISCO_F32 or DISCO_BF16 (BICGSTAB_DC) */
    double inner_tol;  /* relative reduction asked of each inner solve (e.g. 1e-5) */
    int rhs_block;     /* right-hand sides per batched launch; 0 = the autotuned block for
                        * inner_prec if disco_autotune ran (at most 32 for BICGSTAB_DC), else
                        * 16; clamped to 64 and to the plane limit given under disco_autotune */
    int fallback;      /* 1: on inner breakdown/stagnation continue with FP64 CGNR */
    int check_every;   /* iterations between host convergence checks (0 = default: 2 for
                        * BICGSTAB_DC, whose inner solves first run, without checks, as many
                        * iterations as the previous inner solve of the same system took; 10
                        * for CGNR_F64) */
    int restart;       /* FGMRES_NN: Krylov vectors per cycle (1..32, 0 = 16) */
    const disco_net* net; /* FGMRES_NN: the preconditioner (required) */
} disco_solver_params;

typedef struct {
    int iters;              /* inner Krylov iterations (BICGSTAB_RU: those of this right-hand
                             * side's lane while it held it; otherwise its block's) */
    int outer_iters;        /* defect-correction cycles (1 for CGNR) */
    int fallback_used;      /* 1 when the FP64 fallback ran */
    int converged;          /* 1 when true_rel_residual <= tol */
    double true_rel_residual; /* ||b - D x|| / ||b||, FP64, recomputed at the end */
} disco_solver_stats;

/* Solve D x = b (dom = NULL) or D_Lambda x = b for nrhs right-hand sides b
 * (device, boundary layout complex128): the propagator D^-1 on sources, which
 * the quark loop under equation Cdisc of the Methodology section traces, and
 * D_Lambda^-1 of the Domain decomposition subsection.  x (device, same layout)
 * receives the solutions; stats (host, nrhs entries, may be NULL) per
 * right-hand side.  Returns DISCO_ENOCONV if any right-hand side misses tol
 * (every right-hand side is still solved and reported: with BICGSTAB_RU, a
 * block that stops early hands its lanes in flight to the fallback and runs
 * the rest of the queue on). */
int disco_solve_multi_rhs(disco_ctx* ctx, const disco_domains* dom, const disco_solver_params* p,
                          int nrhs, const void* b, void* x, disco_solver_stats* stats);

/* ---------------------------------------------------------------- distillation
 * Sources are built from the lowest eigenvectors v_i(t) of the gauge-covariant
 * 3-D Laplacian on APE-smeared links (standard distillation, the "Analysis with
 * standard distillation" subsection; eigenpairs per timeslice as in the
 * Gaussian-profiled subsection). */

/* APE smearing of the spatial links: `steps` sweeps of
 *   U_k <- P_SU(3)[(1 - alpha) U_k + (alpha/4) * (sum of the 4 spatial staples)]
 * with all links of a sweep updated from the previous sweep, P_SU(3) the polar
 * factor M (M^+ M)^{-1/2} divided by the principal cube root of its
 * determinant.  The smeared links are kept in the context and used only by the
 * Laplacian; D keeps the unsmeared links.  steps = 0 makes the Laplacian use
 * the unsmeared links.  ESTATE before disco_gauge_set. */
int disco_ape_smear(disco_ctx* ctx, int steps, double alpha);
/* Smeared links as [V][4][3][3] complex128 (device; time links unsmeared). */
int disco_smeared_get(disco_ctx* ctx, void* U_out);
/* out = -Delta in for nvec colour fields [nvec][V][3] complex128 (device):
 *   -Delta psi(x) = sum_{k=1..3} [2 psi(x) - U_k(x) psi(x+k) - U_k(x-k)^+ psi(x-k)],
 * smeared links if disco_ape_smear ran, else the gauge links. */
int disco_laplace_apply(disco_ctx* ctx, int nvec, const void* in, void* out);
/* Lowest nv eigenpairs of -Delta on every timeslice, eigenvalues ascending.
 * Vev (device, [T][nv][Vs][3] complex128) receives orthonormal eigenvectors
 * (arbitrary phases), lambda (host, [T][nv]) the eigenvalues.  tol bounds the
 * eigenvector residual ||-Delta v - lambda v|| (<= 0: 1e-12).  ENOCONV when
 * the eigensolver stops above tol. */
int disco_laplace_eigvecs(disco_ctx* ctx, int nv, double tol, void* Vev, double* lambda);
/* The same on the timeslices tsel[0..nt) only (host ints, distinct): the
 * Laplacian and the APE smearing act within a timeslice, so each timeslice's
 * eigenpairs do not depend on the others.  Vev (device, [nt][nv][Vs][3]) and
 * lambda (host, [nt][nv]) in the order of tsel.  For callers that need the
 * sources of a few timeslices only (one packing set of a large lattice). */
int disco_laplace_eigvecs_slices(disco_ctx* ctx, int nv, double tol, const int* tsel, int nt, void* Vev,
                                 double* lambda);
/* Perambulator projection tau[k][j][beta][r] = sum_{xs,c} conj(v_j(t_k; xs)_c)
 * X_r(t_k, xs)_{beta,c} for solutions X (device, [nsrc][V][4][3] complex128,
 * nsrc <= 64) at the sink timeslices t_snk[0..n_snk-1] (host ints): the sink
 * side of V^+ D^-1 V.  Vev as above (device); tau (device) [n_snk][nv][4][nsrc]. */
int disco_perambulator(disco_ctx* ctx, const void* Vev, int nv, int nsrc, const void* X, const int* t_snk, int n_snk,
                       void* tau);
/* Quark loops from diagonal elementals (Gamma (x) diag(w), the elementals
 * equation of the Gaussian-profiled subsection; w = 1 is standard
 * distillation): L[g][t] = sum_i w[t][i] sum_{a,b} Gamma_ab tau[t][i][b][i][a]
 * with tau_tt (device, [T][nv][4][nv][4]) = tau(t,t), w (device [T][nv], or
 * NULL for 1), gammas (host, DISCO_G_* codes, each optionally with
 * DISCO_G_TILDE: then Gamma~ = gamma_4 Gamma^+ gamma_4 replaces Gamma), L
 * (device, [ngamma][T]).  This
 * is the zero-momentum loop sum_x Tr[Gamma D^-1(x,x)] of the Methodology
 * section in its distillation form (no 1/Vs, no sign). */
int disco_loops(disco_ctx* ctx, const void* tau_tt, int T, int nv, const double* w, const int* gammas, int ngamma,
                void* L);
/* End-to-end loops: for every timeslice t and every (i, alpha) solve
 * D x = v_i(t) (x) e_alpha (dom = NULL) or D_Lambda x = ... (dom given),
 * project at t, and form the loops as in disco_loops.  With domains, sources
 * of timeslices in different temporal layers of the partition are added into
 * one multi-site source and solved together (exact, because D_Lambda does not
 * couple different layers: the multi-site sources of the Cost section).
 * Vev device [T][nv][Vs][3]; w device or NULL; L device [ngamma][T]; tau_out
 * device [T][nv][4][nv][4] or NULL; agg (host, may be NULL) gets the inner
 * iterations the solver's block ran in all, the most outer cycles (or
 * reliable updates) one right-hand side took, and the worst true residual.
 * T <= 64.  ENOCONV if any solve misses p->tol. */
int disco_loops_distill(disco_ctx* ctx, const disco_domains* dom, const void* Vev, int nv, const double* w,
                        const int* gammas, int ngamma, const disco_solver_params* p, void* L, void* tau_out,
                        disco_solver_stats* agg);
/* The perambulators tau(t,t) of disco_loops_distill alone, for the source
 * timeslices whose bit is set in tmask (0 = all); tau_out (device,
 * [T][nv][4][nv][4]) is written only at those t.  Lets a caller process a
 * configuration in batches of timeslices (for D_Lambda, one batch per
 * packing set) and form the loops afterwards with disco_loops. */
int disco_perambulators_tt(disco_ctx* ctx, const disco_domains* dom, const void* Vev, int nv, unsigned long long tmask,
                           const disco_solver_params* p, void* tau_out, disco_solver_stats* agg);
/* Right-hand sides solved by the last disco_loops_distill or
 * disco_perambulators_tt call (packed count). */
long long disco_last_solves(const disco_ctx* ctx);
/* Disconnected correlators (Methodology equations Cdisc, correlator_factorised,
 * subtracted_correlator, and corr1-corr4 of the Gaussian-profiled subsection),
 * averaged over source times y0 (Results):
 *   C(dt) = (1/|Y|) sum_{y0 in Y} [ <La(y0+dt mod T) Lb(y0)> - VEV ],
 *   VEV = <La(x0)><Lb(y0)> (vev_mode 0) or (mean over cfg and t of La) times
 *   the same of Lb (vev_mode 1), <.> the mean over configurations.
 * Inputs (device, [ncfg][T] complex128): loops L of Gamma and Lt of
 * Gamma-tilde = gamma_4 Gamma^+ gamma_4 for the full operator and for the
 * domain-restricted one.  Outputs (device, [T] complex128): C_full = C^(d),
 * C_fact = C^(d)_{L0,L1} from the restricted loops, dC = C_full - C_fact;
 * four_terms (device [4][T] or NULL): block-block, block-delta, delta-block,
 * delta-delta with delta L = L - L_Lambda.  y0_set (host) NULL = all T. */
int disco_correlator(disco_ctx* ctx, const void* L_full, const void* Lt_full, const void* L_blk, const void* Lt_blk,
                     int ncfg, int T, const int* y0_set, int ny0, int vev_mode, void* C_full, void* C_fact, void* dC,
                     void* four_terms);

/* The paper's region schedule (subsections "Domain decomposition of the
 * propagator" and "Subtraction method"; multi-site sources of the Cost
 * section).  For every operator time x0 the region is the temporal slab
 * Lambda(x0) = {t : |t - x0| <= (delta-1)/2} (mod T) over all space, delta odd
 * and below T.  disco_slab_sets groups the operator times 0..T-1 greedily (in
 * increasing x0) into sets whose slabs are pairwise disjoint mod T (circular
 * distance >= delta): masks[k] (host, room for T entries) gets the bits of
 * set k, *nsets the number of sets.  Host only. */
int disco_slab_sets(int T, int delta, int* nsets, unsigned long long* masks);
/* L[g][x0] = the loop of D_{Lambda(x0)}^-1 at x0 (as disco_loops) for every
 * x0, each set of disco_slab_sets solved as one multi-site source per (i,
 * alpha) on the partition cut at the faces of its slabs (slabs of one set are
 * disjoint; the rest of the time axis forms source-free domains).  Vev, w,
 * gammas, L, tau_out, agg as in disco_loops_distill (tau_out receives
 * tau_{Lambda(x0)}(x0, x0)).  These are the factorised loops of the
 * subtracted correlator: pass them as L_blk / Lt_blk to disco_correlator. */
int disco_loops_slab(disco_ctx* ctx, const void* Vev, int nv, const double* w, const int* gammas, int ngamma,
                     int delta, const disco_solver_params* p, void* L, void* tau_out, disco_solver_stats* agg);
/* The same schedule with the paper's open time boundary (Results: the ensemble
 * has open boundary conditions in time), read as one more cut: no hop crosses
 * the face between t = T-1 and t = 0, in the full operator as in every region
 * (no boundary improvement terms).  The slab of x0 is then clipped at the
 * boundaries, Lambda(x0) = {t : |t - x0| <= (delta-1)/2, 0 <= t < T}, and the
 * sets of disco_slab_sets_open group operator times whose slabs are disjoint
 * on the open line (distance |x0 - y0| >= delta, not taken around the wrap).
 * The loops of the full operator with the same boundary come from
 * disco_loops_distill with domains whose only cut is cut[3][T-1].  The paper
 * measures in a bulk window away from the boundaries (Cost section); pass
 * such a window as y0_set to disco_correlator.  Arguments as above. */
int disco_slab_sets_open(int T, int delta, int* nsets, unsigned long long* masks);
int disco_loops_slab_open(disco_ctx* ctx, const void* Vev, int nv, const double* w, const int* gammas, int ngamma,
                          int delta, const disco_solver_params* p, void* L, void* tau_out, disco_solver_stats* agg);
/* The noise-reduced estimator spliced by separation (Results, analysis with
 * standard distillation): C^NR(dt) = C^(c)(dt) + dC_Delta(dt) with, at each
 * separation dt, the widest slab width Delta of deltas[0..ndelta-1] below dt
 * (with widths 7, 9, 11, 13 this is the paper's choice: 7 for dt = 8, 9;
 * 9 for 10, 11; 11 for 12, 13; 13 from 14 on).  Cc (host, [T] complex128, the
 * connected correlator of disco_connected), dC (host, [ndelta][T] complex128,
 * the subtracted correlators of disco_correlator with the slab loops of each
 * width), out (host, [T] complex128): NaN at separations no width is below.
 * Host only. */
int disco_nr_splice(const double* Cc, const double* dC, const int* deltas, int ndelta, int T, double* out);
/* Gaussian distillation profiles (the Gaussian-profiled subsection): the
 * diagonal elemental weight |g_k(lambda)|^2 with g_k(lambda) =
 * exp(-lambda^2 / (2 (0.8 omega_k)^2)), i.e. w = exp(-lambda^2 / (0.8 omega)^2),
 * for n eigenvalues (host arrays; omega > 0).  Use as w of the loop calls. */
int disco_profile_weights(const double* lambda, long n, double omega, double* w);

/* Connected contraction (equation Cfull: C = C^(c) + C^(d)) in distillation.
 * disco_perambulators_all: for every source timeslice ts in tmask (0 = all) and
 * every (i, alpha), solve D x = v_i(ts) (x) e_alpha and project the solution at
 * every sink timeslice: tau_all (device, [T][T][nv][4][nv][4] complex128) =
 * tau_all[ts][tk][j][beta][i][alpha] = (V(tk)^+ D^-1 V(ts)).  agg as in
 * disco_loops_distill.  T <= 64. */
int disco_perambulators_all(disco_ctx* ctx, const void* Vev, int nv, unsigned long long tmask,
                            const disco_solver_params* p, void* tau_all, disco_solver_stats* agg);
/* C[g][dt] (device, [ngamma][T] complex128), averaged over the source times
 * y0 (host list; NULL = all T), x0 = y0 + dt mod T:
 *   C = -Tr[Phi_Gamma(x0) tau(x0,y0) Phi_Gammatilde(y0) tau(y0,x0)]
 * with Phi_Gamma(t) = Gamma (x) diag(w(t)) (w device [T][nv] or NULL = 1),
 * Gamma~ = gamma_4 Gamma^+ gamma_4, and tau(y0,x0) = g5 tau(x0,y0)^+ g5
 * (gamma_5-hermiticity), so only the sources at y0 are needed.  The minus
 * sign is the fermion loop of the connected Wick contraction; the loops
 * carry no sign, so C_full = C + C^(d) and the paper's noise-reduced
 * estimator is C^NR = C + dC (dC from disco_correlator). */
int disco_connected(disco_ctx* ctx, const void* tau_all, int T, int nv, const double* w, const int* gammas,
                    int ngamma, const int* y0_set, int ny0, void* C);
/* a m_eff(t) = ln(C(t) / C(t+1)) for t = 0 .. n-2 (host; NaN where the ratio is
 * not positive), the effective mass of the Gaussian-profiled subsection. */
int disco_effective_mass(const double* C, int n, double* meff);

/* Autotuner: time a fixed number of inner BiCGStab iterations (FP32 or BF16
 * storage, the full operator when dom is NULL) for right-hand-side blocks of
 * 8, 16, 32 and 64 on device-generated random sources, and keep the block with
 * the lowest cost per right-hand side and iteration for later solves with
 * rhs_block = 0 (BICGSTAB_DC uses at most 32 of it: its fixed blocks wait for
 * their slowest member, while BICGSTAB_RU refills finished lanes).  best (host) receives it; cost_us (host, 4 entries, may be
 * NULL) the measured microseconds per right-hand side and iteration, 0 for a
 * block not tried.  Then, at the chosen block, it times the tile of the
 * stencil's site order (DISCO_OPT_TILE_Y, DISCO_OPT_TILE_T: y rows 1, 2, 3, 4,
 * 6, 8 that divide Ly, and the whole XCD slab of timeslices or half of it, up
 * to 1024 sites per z step) and keeps the fastest, the current tile included;
 * disco_get_option reads the result.  A block is tried only if one spinor plane of it
 * (V * block * 16 bytes at every precision) stays below 4 GiB, the limit of
 * the stencil's 32-bit offsets; solves clamp rhs_block to the same limit. */
int disco_autotune(disco_ctx* ctx, const disco_domains* dom, int inner_prec, int* best, double* cost_us);

/* ---------------------------------------------------------------- learned preconditioner
 * Not part of the paper, which only needs D^-1: the production solver's own
 * approximation of D^-1, judged only through the FP64 true residual of the
 * solves it preconditions.  A gauge-covariant convolutional network of three
 * layers with channels 1 -> 16 -> 16 -> 1, no nonlinearity:
 *   out_o(x) = sum_i sum_{d in {-1,0,1}^4} W[d][o][i] . T_d(x) psi_i(x + d)
 * W[d][o][i] is a complex 4x4 matrix on the spin index; T_d(x) is the colour
 * transporter along the axis-ordered path from x to x + d (|d_x| hops in x,
 * then y, z, t; a forward hop from y takes U_mu(y), a backward hop
 * U_mu(y - mu)^+, and a hop across the wrap the boundary phase bc[mu]).
 * Offsets are numbered k = (dx+1) + 3(dy+1) + 9(dz+1) + 27(dt+1).
 * Weights: FP32, layers in order, each [81][C_out][C_in][4][4] complex stored
 * as (re, im) pairs: 2 * 81 * 16 * (16 + 256 + 16) floats = 746496.
 * Activations are BF16 with FP32 accumulation (matrix cores).
 * The lattice needs Lx, Ly divisible by 4 and Lz, Lt by 2. */
/* Create a network on the context's gauge field (tabulates the 81
 * transporters per site, 5.8 KB per site).  Initial weights: identity through
 * channel 0 of each layer plus Gaussian noise of standard deviation 0.01 from
 * `seed`.  channels must be 16.  ESTATE before disco_gauge_set.  The network
 * keeps the transporters of the gauge field current at creation. */
int disco_net_create(disco_ctx* ctx, int channels, unsigned long long seed, disco_net** out);
int disco_net_destroy(disco_net* net);
/* Re-tabulate the transporters from the context's current gauge field (after
 * disco_gauge_set with another configuration; the weights and the optimiser
 * state are kept, so training can continue over several ensembles). */
int disco_net_refresh(disco_net* net);
/* number of floats of the packed weights */
long long disco_net_weights_count(const disco_net* net);
int disco_net_set_weights(disco_net* net, const float* w, int where);
int disco_net_get_weights(disco_net* net, float* w, int where);
/* out = N(in) for nrhs fields [nrhs][V][4][3] complex128 (device). */
int disco_net_apply(disco_net* net, int nrhs, const void* in, void* out);
/* Gradients of the real function L with dL/dRe(out) + i dL/dIm(out) = grad_out
 * (device [nrhs][V][4][3] complex128) at inputs in (same layout, nrhs <= 64):
 * grad_w (device, weights layout) = dL/dRe(W) + i dL/dIm(W) summed over the
 * right-hand sides; grad_in (device, may be NULL) = dL/dRe(in) + i dL/dIm(in). */
int disco_net_backward(disco_net* net, int nrhs, const void* in, const void* grad_out, float* grad_w, void* grad_in);

typedef struct {
    int npairs;          /* (residual, error) pairs to generate (multiple of nsnap and batch) */
    int nsnap;           /* pairs per source: one per truncated solve (1..8) */
    int snap_iters[8];   /* inner iterations of each truncated solve (0: x_k = 0, i.e. e = x*) */
    int batch;           /* pairs per Adam step (1..16) */
    int steps;           /* Adam steps */
    double lr;           /* Adam learning rate */
    unsigned long long seed;
} disco_train_params;
typedef struct {
    int pairs, steps;
    double first_loss;   /* mean |N(r) - e|^2 of the first mini-batch (|e| = 1) */
    double final_loss;   /* mean over the last quarter of the steps (at most one epoch) */
    double gen_seconds, train_seconds;
} disco_train_stats;
/* Train on pairs the solver generates on this context's gauge field: Gaussian
 * sources b, converged x* (BiCGStab-DC to 1e-9), truncated solves x_k, error
 * e = x* - x_k, residual r = D e (FP64), each pair scaled to |e| = 1.  Loss
 * (1/B) sum_p |N(r_p) - e_p|^2, Adam (beta 0.9, 0.999, eps 1e-8) with this
 * library's own forward and backward kernels. */
int disco_net_train(disco_net* net, const disco_train_params* p, disco_train_stats* stats);

/* ---------------------------------------------------------------- profiling
 * Per-kernel-family timing of launches made while profiling is on, measured
 * with HIP events recorded on the context's stream around each launch.
 * kernel: 0 = Wilson-clover stencil (any precision): bytes = algorithmic
 * bytes of those launches (each input/output spinor, the links and the clover
 * term counted once per site); 10, 11, 12 = the same split by storage
 * precision (FP64, FP32, BF16); 1 = FP64 matrix-core contraction
 * (perambulator, eigensolver Gram matrices): bytes holds the flop count;
 * 2 = network layers (BF16 matrix cores): bytes holds the flop count;
 * 13, 14, 15 = even-odd (half-lattice) stencil launches by storage precision:
 * bytes = algorithmic bytes (spinors once, all links of the visited sites, A^-1). */
enum { DISCO_KERNEL_STENCIL = 0, DISCO_KERNEL_MFMA64 = 1, DISCO_KERNEL_NN = 2 };
int disco_profile_enable(disco_ctx* ctx, int on);
/* Time only every `stride`-th profiled launch of each family (default 1). */
int disco_profile_stride(disco_ctx* ctx, int stride);
int disco_profile_reset(disco_ctx* ctx);
int disco_profile_get(disco_ctx* ctx, int kernel, long long* launches, double* total_ms, double* bytes);

#ifdef __cplusplus
}
#endif
#endif
