/*
 * ndq -- the Neuberger-Dirac hot path on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libndq.so.  Operators follow Walk, Wittig, Dranischnikow, Schoemer,
 * "Implementation of the Neuberger-Dirac operator on GPUs" (Lattice 2010):
 *
 *   D_W phi(x) = (4+m) phi(x) - 1/2 sum_{mu=+-0..+-3} U_mu(x)(1-gamma_mu) phi(x+mu)   (Sec. 2.1, Eq. 1)
 *   U_{-mu}(x) = U_mu(x-mu)^{-1},  gamma_{-mu} = -gamma_mu                            (Eq. 2)
 *   Q = gamma5 D_W                                                                     (Eq. 1)
 *   D_N = (1 + gamma5 sign(Q)) / abar                                                  (Sec. 2.2, Eq. 4)
 *   sign(Q) ~ X P_n(X^2), X = Q/|Q|, P_n = sum_k c_k T_k                               (Eq. 5, Eq. 6)
 *   sign(Q) ~ P_+ - P_- + (1 - P_+ - P_-) X P_n(X^2)                                   (Sec. 2.3, Eq. 11)
 *
 * Conventions used everywhere (the paper leaves them open):
 *   - periodic boundaries; dims = {N0, N1, N2, N3}, N0 the time extent, every
 *     extent even and >= 2; lexicographic site index
 *     lex = ((x0*N1 + x1)*N2 + x2)*N3 + x3;
 *   - parity (x0+x1+x2+x3) & 1 (even = 0); within a parity, the site with
 *     lexicographic index lex has even/odd index lex >> 1;
 *   - chiral Dirac matrices, gamma5 = diag(1, 1, -1, -1); lattice spacing a = 1;
 *   - D_N with s = -1 - m (m the Wilson mass of Eq. 1), abar = 1/(1+s), and the
 *     massive operator D_N^m = (1 - abar mq/2) D_N + mq (the form bounded by Eq. 12).
 *
 * Memory and ownership:
 *   - every device buffer is allocated and owned by the caller; *_bytes()
 *     queries give the sizes (workspaces included).  The library allocates
 *     no memory of its own, except the objects of the graph replay of
 *     ndq_overlap_params.graph (a capture stream per device and up to four
 *     instantiated graphs per host thread) and the static scratch of
 *     ndq_apply_DN_noalloc;
 *   - "canonical" buffers are complex128 (interleaved re, im doubles) in device
 *     memory: gauge [V][4 mu][3 row][3 col] in lexicographic order; spinor
 *     [nrhs][nsites][4 spin][3 colour] with nsites = V (lexicographic order)
 *     for NDQ_FULL fields and V/2 (even/odd index order) for parity fields;
 *   - packed fields (ndq_gauge, ndq_spinor) use the library's internal
 *     structure-of-arrays layout and are opaque to the caller;
 *   - opaque host handles (ndq_geom, ndq_approx) are created and destroyed by
 *     the library;
 *   - `stream` is a hipStream_t (NULL = the null stream).  Apply calls are
 *     asynchronous on that stream; calls that return scalars to the host
 *     synchronise it.
 *
 * Errors: every call returns NDQ_OK (0) or a negative status.  Argument
 * checks run on the host before anything is launched.  ndq_last_error()
 * returns a thread-local message for the last failure.  No C++ exception
 * crosses this boundary.  A failed HIP call returns NDQ_EHIP.
 */
#ifndef NDQ_H
#define NDQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
enum {
    NDQ_OK = 0,
    NDQ_EINVAL = -1,     /* bad argument (NULL pointer, out-of-range value)      */
    NDQ_EDIMS = -2,      /* lattice extent odd, < 2, or volume too large          */
    NDQ_EPREC = -3,      /* unsupported precision / reconstruction combination    */
    NDQ_ENOMEM = -4,     /* caller-provided workspace too small                   */
    NDQ_ESINGULAR = -5,  /* 8-real link with |a2|^2+|a3|^2 < 1e-12, or nu_k = 0   */
    NDQ_ENOCONV = -6,    /* iterative method hit its iteration limit              */
    NDQ_ENAN = -7,       /* NaN or Inf in a norm                                   */
    NDQ_EHIP = -8        /* a HIP runtime call failed                              */
};

/* ---- enumerations ------------------------------------------------------- */
enum { NDQ_F64 = 0, NDQ_F32 = 1, NDQ_F16 = 2 };          /* storage precision  */
enum { NDQ_EVEN = 0, NDQ_ODD = 1, NDQ_FULL = 2 };        /* spinor site subset */
enum { NDQ_ZOLOTAREV = 0, NDQ_MINMAX_POLY = 1 };         /* sign approximant   */
enum { NDQ_LITERAL = 0, NDQ_SANDWICH = 1 };              /* Eq. 11 placement   */

/* ---- geometry ----------------------------------------------------------- */
typedef struct ndq_geom ndq_geom;

/* Create a host-side geometry for a periodic N0 x N1 x N2 x N3 lattice.
 * dims: host array of 4 extents, each even and >= 2, volume < 2^30.
 * On success *out receives a handle the caller releases with ndq_geom_destroy.
 * Errors: NDQ_EINVAL (NULL), NDQ_EDIMS. */
int ndq_geom_create(const int32_t dims[4], ndq_geom** out);
void ndq_geom_destroy(ndq_geom* g);
int64_t ndq_geom_volume(const ndq_geom* g);

/* Index tables produced on the device by the same index arithmetic the
 * stencil kernels use (Sec. 2.1: one site per lane, neighbours x +- mu).
 *   d_nb       int32 [V][8]      lexicographic neighbours: +0,+1,+2,+3,-0,-1,-2,-3
 *   d_lex_of_eo int32 [2][V/2]   lexicographic index of (parity, eo index)
 *   d_nb_eo    int32 [2][V/2][8] eo index (in the opposite parity) of each neighbour
 * Any pointer may be NULL to skip that table.  Asynchronous on `stream`. */
int ndq_geom_tables(const ndq_geom* g, int32_t* d_nb, int32_t* d_lex_of_eo, int32_t* d_nb_eo,
                    void* stream);

/* ---- fields ------------------------------------------------------------- */
/* A packed gauge field: data (device) holds all 4V links in `prec` with
 * `recon` reals per link: 18 (full matrix), 12 (two columns a, b; the third is
 * c = (a x b)^*, Sec. 2.1 Eq. 3) or 8 (a2, a3, b1, arg a1, arg c1; the rest
 * from unitarity, the 8-parameter idea of Sec. 2.1).  F64 links need F64
 * spinors; F16 links support recon 18 and 12. */
typedef struct {
    void* data;
    int32_t prec;
    int32_t recon;
} ndq_gauge;

/* A packed spinor field of nrhs right-hand sides on a site subset
 * (NDQ_EVEN, NDQ_ODD: V/2 sites; NDQ_FULL: V sites).  F16 fields carry one
 * F32 scale per site and right-hand side inside `data`. */
typedef struct {
    void* data;
    int32_t prec;
    int32_t parity;
    int32_t nrhs;
} ndq_spinor;

/* Bytes of a packed gauge field: 4V links of link_bytes(prec, recon), and for
 * 8-real links a 256-byte status area after them (the singularity flag that
 * ndq_gauge_pack reads back). */
size_t ndq_gauge_bytes(const ndq_geom* g, int prec, int recon);
size_t ndq_spinor_bytes(const ndq_geom* g, int prec, int parity, int nrhs);

/* Convert a canonical complex128 gauge field (device) to the packed format.
 * Errors: NDQ_EPREC; NDQ_ESINGULAR (recon 8 and some link has
 * |a2|^2 + |a3|^2 < 1e-12, e.g. the unit field).  Synchronises `stream` for
 * recon 8 (to read back the singularity flag from the field's status area);
 * otherwise asynchronous. */
int ndq_gauge_pack(const ndq_geom* g, const void* d_canon, const ndq_gauge* dst, void* stream);

/* Reconstruct a packed gauge field into canonical complex128 (device). */
int ndq_gauge_unpack(const ndq_geom* g, const ndq_gauge* src, void* d_canon, void* stream);

/* Canonical complex128 spinor (device) <-> packed spinor.  Asynchronous. */
int ndq_spinor_pack(const ndq_geom* g, const void* d_canon, const ndq_spinor* dst, void* stream);
int ndq_spinor_unpack(const ndq_geom* g, const ndq_spinor* src, void* d_canon, void* stream);

/* ---- operators ---------------------------------------------------------- */
/* out = Q in = gamma5 D_W in (Eq. 1) on NDQ_FULL fields; in != out.
 * Arithmetic in FP64 for F64 fields, FP32 otherwise.  Asynchronous. */
int ndq_apply_Q(const ndq_geom* g, const ndq_gauge* U, double m, const ndq_spinor* in,
                const ndq_spinor* out, void* stream);

/* Q on several lattices in one persistent launch (batching of the stencil:
 * uneven lattice sizes, each with its own links, mass and right-hand sides).
 * Each job computes out = Q in exactly as ndq_apply_Q with nrhs > 1 does
 * (links staged once per 64-site tile, every right-hand side of that tile
 * computed from them), so its results equal that call's bit for bit (and, for
 * nrhs = 1, those of the one-lane-per-site launch shape, block 64/128/256).
 * All jobs share the spinor precision and the link format; 1 <= njobs <= 8;
 * in, out: NDQ_FULL, same precision and nrhs, not aliased.  A fixed grid (a
 * multiple, ndq_set_multi_grid, of the workgroups the device holds at once)
 * walks the joint tile list in contiguous chunks.  Asynchronous. */
typedef struct {
    const ndq_geom* g;
    const ndq_gauge* U;
    double m;
    const ndq_spinor* in;
    const ndq_spinor* out;
} ndq_q_job;
int ndq_apply_Q_multi(const ndq_q_job* jobs, int32_t njobs, void* stream);

/* Even/odd hopping block: out_p = H_{p,1-p} in, where D_W = (4+m) - H/2 and
 * H psi(x) = sum_{mu=+-0..+-3} U_mu(x)(1-gamma_mu) psi(x+mu) (Eq. 1, Eq. 2).
 * `in` has parity 1-p, `out` parity p (both NDQ_EVEN/NDQ_ODD); 1320 flop per
 * output site by the usual convention.  Asynchronous. */
int ndq_apply_dslash(const ndq_geom* g, const ndq_gauge* U, const ndq_spinor* in,
                     const ndq_spinor* out, void* stream);

/* Even-site gamma5-Hermitian Schur complement
 *   Qhat_ee = gamma5 [ (4+m) - H_eo H_oe / (4 (4+m)) ],
 * using tmp (an NDQ_ODD field of the same precision) as scratch. */
int ndq_apply_Qhat_ee(const ndq_geom* g, const ndq_gauge* U, double m, const ndq_spinor* in,
                      const ndq_spinor* out, const ndq_spinor* tmp, void* stream);

/* ---- sign-function approximants (host) ----------------------------------- */
typedef struct ndq_approx ndq_approx;

/* Build an approximant of sign(x), x = lambda/|Q|:
 *   NDQ_MINMAX_POLY: x P(x^2), P = sum_{k=0}^{degree} c_k T_k(z), z = (2y-1-lo)/(1-lo),
 *     minimising max_{lo<=y<=1} |1 - sqrt(y) P(y)| (Sec. 2.2, Eq. 5 and Eq. 6; lo = eps);
 *     Remez exchange, degree in [0, 2000];
 *   NDQ_ZOLOTAREV: x sum_{l=1}^{degree} beta_l / (x^2 + sigma_l), the optimal rational
 *     approximation on lo <= |x| <= 1 (lo = k), degree (poles) in [1, 32].
 * Host only (no GPU needed).  Errors: NDQ_EINVAL, NDQ_ENOCONV. */
int ndq_approx_create(int kind, double lo, int degree, ndq_approx** out);
/* Wrap caller-supplied coefficients: a = sigma[n] and b = beta[n] (Zolotarev) or
 * a = c[n+1] (polynomial); `delta` is recorded as given. */
int ndq_approx_from_coeffs(int kind, int n, const double* a, const double* b, double lo, double delta,
                           ndq_approx** out);
/* kind, n (poles or degree), lo, and delta = max approximation error on the interval. */
int ndq_approx_info(const ndq_approx* ap, int* kind, int* n, double* lo, double* delta);
/* Copy coefficients to host arrays: a gets sigma[n] or c[n+1]; b gets beta[n] (may be NULL). */
int ndq_approx_coeffs(const ndq_approx* ap, double* a, double* b);
void ndq_approx_destroy(ndq_approx* ap);

/* ---- sign(Q) and D_N ------------------------------------------------------ */
typedef struct {
    double m;                 /* Wilson mass of Eq. 1; s = -1 - m, abar = 1/(1+s)            */
    double mq;                /* quark mass of D_N^m                                          */
    double lam_max;           /* |Q| (or an upper bound) used in X = Q / lam_max              */
    const ndq_approx* approx; /* approximant of sign on the complement of the low modes      */
    const void* modes;        /* device: nev packed F64 NDQ_FULL spinors, back to back,
                                 orthonormal Rayleigh-Ritz vectors u_k (may be NULL if nev=0) */
    const double* nu;         /* host: the nev eigenvalues nu_k (P Q u_k = nu_k u_k), nonzero */
    int32_t nev;              /* number of low modes treated exactly, 0..64                   */
    int32_t form;             /* NDQ_LITERAL (Eq. 11 as printed) or NDQ_SANDWICH              */
    double tol;               /* rational approximant: multi-shift CG relative residual       */
    int32_t max_iter;         /* rational approximant: CG iteration limit                     */
    int32_t check_every;      /* rational approximant: convergence read-back interval (>= 1)  */
    int32_t graph;            /* rational approximant: nonzero launches each block of
                                 check_every multi-shift iterations as one captured HIP graph
                                 (same kernels and arguments as the eager launches)           */
} ndq_overlap_params;

typedef struct {
    int64_t q_applies;        /* stencil applications                                         */
    int32_t iterations;       /* CG iterations (rational) or Clenshaw steps (polynomial)      */
    int32_t outer;            /* outer defect-correction steps (solve)                        */
    int64_t inner;            /* inner CG iterations summed over outer steps (solve)          */
    double residual;          /* final relative residual (CG, or true residual for a solve)   */
    double seconds;           /* host wall time of the call                                   */
} ndq_stats;

enum { NDQ_OP_SIGN = 0, NDQ_OP_DN = 1, NDQ_OP_SOLVE = 2 };

/* Workspace (device bytes) that ndq_apply_sign / ndq_apply_DN need for fields
 * of precision `prec` with one right-hand side (ndq_workspace_bytes) or nrhs
 * right-hand sides (ndq_workspace_bytes_nrhs, 1 <= nrhs <= 32).  0 on invalid
 * arguments. */
size_t ndq_workspace_bytes(const ndq_geom* g, const ndq_overlap_params* p, int prec, int op);
size_t ndq_workspace_bytes_nrhs(const ndq_geom* g, const ndq_overlap_params* p, int prec, int op, int nrhs);

/* out = sign(Q) in by Eq. 11: with c = U^H in and t = X r(X^2) in (the approximant
 * evaluated by Clenshaw's recurrence for the polynomial, by multi-shift CG for the
 * rational form), out = t + U (sign(nu) * c - U^H t); NDQ_SANDWICH applies the
 * approximant to (1 - P) in instead.  in, out: NDQ_FULL, same precision, the
 * same number nrhs (1..32) of right-hand sides (arithmetic FP64 for F64 fields,
 * FP32 otherwise; projections always FP64).  With nrhs > 1 and the polynomial
 * approximant every stencil application of the recurrence serves all nrhs
 * fields with one load of the links per tile, and the projections are block
 * products with the modes on the matrix cores (results equal the one-field call
 * up to the rounding of those sums); the rational approximant runs the fields
 * one after the other.  Workspace: ndq_workspace_bytes_nrhs.
 * Synchronises `stream` for the rational approximant (convergence checks).
 * Errors: NDQ_ENOMEM (workspace), NDQ_ENOCONV (CG limit), NDQ_ENAN, NDQ_ESINGULAR (nu_k = 0). */
int ndq_apply_sign(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p,
                   const ndq_spinor* in, const ndq_spinor* out, void* ws, size_t ws_bytes,
                   ndq_stats* stats, void* stream);

/* out = D_N^m in = (1/abar - mq/2)(in + gamma5 sign(Q) in) + mq in  (Eq. 4, Eq. 12),
 * for every right-hand side of in (as ndq_apply_sign). */
int ndq_apply_DN(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p,
                 const ndq_spinor* in, const ndq_spinor* out, void* ws, size_t ws_bytes,
                 ndq_stats* stats, void* stream);

/* ndq_apply_DN for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operation, kernels and results as ndq_apply_DN, with the workspace
 * taken from a static device array of ndq_noalloc_scratch_bytes() (32 MiB)
 * that each GPU holds from the first call on it until the process ends.  No
 * allocating call is made.  The caller still owns in and out.  Every call on
 * one GPU shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 * p->graph must be 0.  Errors: those of ndq_apply_DN; NDQ_ENOMEM when
 * ndq_workspace_bytes(g, p, in->prec, NDQ_OP_DN) exceeds the static size. */
size_t ndq_noalloc_scratch_bytes(void);
int ndq_apply_DN_noalloc(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p,
                         const ndq_spinor* in, const ndq_spinor* out, ndq_stats* stats, void* stream);

/* ---- solving D_N^m x = b --------------------------------------------------- */
typedef struct {
    double tol;           /* target true residual |b - D x| / |b|, D the FP64 operator of p64 */
    int32_t max_outer;    /* defect-correction steps (<= 0: 20)                             */
    int32_t max_inner;    /* CG iterations per inner solve (<= 0: no limit)                 */
    double inner_tol;     /* inner relative residual (<= 0: tol/2 plain FP64, 1e-5 for F32
                             storage, 8 * 2^-11 = 3.9e-3 for F16 storage: eight units of its
                             rounding)                                                        */
    int32_t inner_prec;   /* NDQ_F64: plain FP64 solve; NDQ_F32 / NDQ_F16: mixed precision  */
    int32_t sectors;      /* inner solver: 0 = CGNE on D^H D (two sign applies per iteration);
                             1 = CG on each chirality sector of D^H D, which commutes with
                             gamma5 (one sign apply per iteration; a chiral source, e.g. a
                             point source, needs one sector)                                 */
} ndq_solve_params;

size_t ndq_solve_workspace_bytes(const ndq_geom* g, const ndq_overlap_params* p64, const ndq_overlap_params* plo,
                                 const ndq_solve_params* sp);
/* The same for a block of nrhs right-hand sides (1 <= nrhs <= 32). */
size_t ndq_solve_workspace_bytes_nrhs(const ndq_geom* g, const ndq_overlap_params* p64, const ndq_overlap_params* plo,
                                      const ndq_solve_params* sp, int nrhs);

/* x = (D_N^m)^{-1} b (Eq. 4 with the massive form of Eq. 12).  FP64 defect
 * correction: r = b - D x with the FP64 operator (U64, p64); while |r| > tol |b|,
 * solve D e = r/|r| by CG on the normal equations (D^H = gamma5 D gamma5), or by
 * CG on their chirality sectors (sp->sectors), in the inner precision (U_lo and p_lo: F32 arithmetic on F32 or F16 storage, with their
 * own approximant; or FP64 with U64, p64 for the plain solve) and set x += |r| e.
 * Both operators apply Eq. 11 in its sandwich form whatever p64->form and
 * p_lo->form say: CG on the normal equations needs D^H = gamma5 D gamma5, i.e. a
 * Hermitian sign(Q), which the literal form is only up to O(rho_k).
 * b, x: F64 NDQ_FULL with the same nrhs (1..32); x holds the initial guess on
 * entry.  With nrhs > 1 (CGNE) every field has its own defect correction and
 * CGNE scalars, and all fields share each application of D: one call of the
 * stencil per step serves the whole block (links loaded once per tile), which
 * is the batched solve of many sources on one gauge field (e.g. the 12
 * spin-colour point sources); a field that has converged keeps its solution
 * while the others continue.  With sectors = 1 the fields are solved one after
 * the other.  Workspace: ndq_solve_workspace_bytes_nrhs.  Synchronises
 * `stream`.  stats: outer steps, inner CG iterations (block iterations for
 * nrhs > 1), Q applications, final true relative residual (the largest over the
 * fields).  Errors: NDQ_ENOCONV, NDQ_ENOMEM, NDQ_ENAN, NDQ_EPREC. */
int ndq_solve_DN(const ndq_geom* g, const ndq_gauge* U64, const ndq_gauge* U_lo, const ndq_overlap_params* p64,
                 const ndq_overlap_params* p_lo, const ndq_solve_params* sp, const ndq_spinor* b,
                 const ndq_spinor* x, void* ws, size_t ws_bytes, ndq_stats* stats, void* stream);

/* ---- low modes of Q (FP64) ----------------------------------------------- */
typedef struct {
    int32_t nev;          /* number l of low modes of Q to return (>= 1)                      */
    int32_t nextra;       /* extra Ritz vectors carried as a guard band (>= 1)                */
    int32_t basis;        /* Lanczos basis size m, nev + nextra + 2 <= m <= 63 (Lanczos only)  */
    int32_t cheb_degree;  /* degree d of the Chebyshev filter (even); <= 0: automatic        */
    double cheb_lo;       /* filter cutoff a on Q^2; <= 0: from a plain Lanczos run           */
    double tol;           /* stop when every rho_k <= tol * lam_max                          */
    int32_t max_restarts; /* iterations / restart cycles (<= 0: 200 subspace, 100 Lanczos)     */
    int32_t method;       /* NDQ_LM_SUBSPACE (block Chebyshev-filtered subspace iteration,
                             adaptive filter), NDQ_LM_LANCZOS (thick-restart Lanczos) or
                             NDQ_LM_RITZ (the paper's Ritz-functional minimisation of Q^2:
                             conjugate-gradient sweeps over the nev + 1 vectors, each kept
                             orthogonal to the ones before, alternating with Rayleigh-Ritz of
                             Q; max_restarts caps the CG steps per vector, default 5000)      */
    int32_t nev_min;      /* 0: use all nev modes.  1 <= nev_min <= nev: choose the number l of
                             modes to project in [nev_min, nev] where the relative gap
                             |nu_(l+1)| / |nu_l| to the next mode is largest (Sec. 2.3: the gap
                             should not be accidentally small); reported as nev_used          */
    const ndq_gauge* U_lo; /* NULL, or F32 links of the same gauge field (subspace method
                             only): the filter of the early restarts runs on F32 copies of the
                             block with these links, the orthonormalisation, Rayleigh-Ritz and
                             residues stay FP64; after the first restart whose largest rho_k is
                             <= lo_until * lam_max, or three F32 restarts that did not halve the
                             smallest such value so far, the filter is FP64.  Convergence is
                             decided in FP64 as without U_lo.                                */
    double lo_until;      /* switch point of U_lo (<= 0: 1e-5)                                */
} ndq_lowmode_params;

enum { NDQ_LM_SUBSPACE = 0, NDQ_LM_LANCZOS = 1, NDQ_LM_RITZ = 2 };

typedef struct {
    double lam_next;      /* |Q u| of the guard vector u (the next Ritz vector after the
                             nev returned, in the order of |Q u|^2)                          */
    double kappa_plus;    /* Eq. 9, with d_k = min(lam_next - rho_next - |nu_k|, |nu_k| + min|nu_j|
                             over the returned nu_j of opposite sign): lam_next - rho_next is
                             the certified lower end of the rest of the spectrum of |Q|      */
    double kappa_minus;
    double bound_plus;    /* Eq. 10: |P_+ - (P_+)_exact| <= kappa(1+2kappa)/(1-2kappa(1+2kappa)) */
    double bound_minus;
    double cheb_lo;       /* filter cutoff used                                               */
    int32_t cheb_degree;  /* filter degree used                                               */
    int32_t restarts;
    int64_t q_applies;
    double max_rho;       /* largest rho_k of the returned modes                             */
    double rho_next;      /* from the guard residue r = |Q^2 u - lam_next^2 u|: Q has an
                             eigenvalue with |lambda| >= lam_next - rho_next = sqrt(lam_next^2 - r);
                             with nev_used < nev: lam_next = |nu_(l+1)|, rho_next = rho_(l+1) */
    double seconds;
    int32_t nev_used;     /* number l of modes to project (nev unless nev_min chose fewer);
                             kappa and bounds refer to the first l modes                      */
    int32_t restarts_lo;  /* restarts whose filter ran on U_lo (F32)                          */
} ndq_lowmode_info;

size_t ndq_lowmodes_workspace_bytes(const ndq_geom* g, const ndq_lowmode_params* p);

/* The nev eigenmodes of Q closest to zero (Sec. 2.3): a Chebyshev filter of Q^2
 * inside block subspace iteration or thick-restart Lanczos (FP64, CGS2
 * orthogonalisation), Rayleigh-Ritz of Q in the space found (P Q u_k = nu_k u_k,
 * nev + nextra <= 64), residues rho_k = |(Q - nu_k) u_k|
 * (Eq. 8) and kappa_+- (Eq. 9), bound (Eq. 10).  Ritz pairs are ordered by
 * |Q u|^2, the Rayleigh quotient of Q^2 (equal to nu^2 once converged), which
 * keeps spurious near-zero Ritz values of the indefinite Q out of the result.
 * With p->U_lo (subspace method) the filter of the early iterations runs in
 * FP32 on F32 copies of the block (see ndq_lowmode_params); the returned modes
 * and residues are FP64 as without it.
 *   U: F64 links;  start: F64 NDQ_FULL spinor (nonzero);  d_modes: out, nev packed F64
 *   NDQ_FULL spinors back to back (orthonormal);  nu, rho: host arrays of nev, in
 *   that order (|nu| ascending once converged).  Converged means every rho_k <=
 *   tol * lam_max and the guard (the next Ritz vector) has a residue of Q^2 of at
 *   most max(tol, 1e-6) * lam_max^2.
 *   Synchronises `stream`.  Errors: NDQ_ENOCONV (tol not reached; the
 *   best modes found are still written), NDQ_ENOMEM, NDQ_EPREC, NDQ_ENAN. */
int ndq_lowmodes_compute(const ndq_geom* g, const ndq_gauge* U, double m, double lam_max,
                         const ndq_lowmode_params* p, const ndq_spinor* start, void* d_modes, double* nu,
                         double* rho, ndq_lowmode_info* info, void* ws, size_t ws_bytes, void* stream);

/* Host utility: eigen-decomposition of a dense Hermitian n x n matrix (row-major,
 * interleaved complex `a`, destroyed); w ascending, z columns = eigenvectors
 * (row-major, interleaved complex).  The library's own small-matrix solver. */
int ndq_host_eigh(int n, double* a, double* w, double* z);

/* ---- index of the massless D_N (the workload of the outlook, Sec. 4) -------- */
/* Zero-mode counting on D = (1 + gamma5 eps) / abar (Eq. 4 with m_q = 0), eps the
 * approximate sign of the overlap parameters (low modes exact, Eq. 11).  On the
 * chirality-s subspace (gamma5 psi = s psi) D^H D = (2 / abar^2) A_s with
 * A_s = 1 + s P_s eps P_s, P_s = (1 + s gamma5) / 2, spectrum in [0, 2]; its
 * lowest eigenpairs are found per sector by block Chebyshev-filtered subspace
 * iteration (one sign apply per application of A_s), and the Ritz values below
 * zero_cut are counted: n_+ and n_-, index = n_+ - n_-.  Nonzero eigenvalues of
 * A_+ and A_- coincide, so accidental near-zero pairs cancel in the index. */
#define NDQ_INDEX_REPORT 16
typedef struct {
    int32_t block;        /* vectors per sector, 2..64; must exceed the number of zero
                             modes of either chirality (0: 8)                           */
    int32_t degree;       /* Chebyshev filter degree per sweep (0: adaptive, the degree that
                             amplifies the null space ~1e4-fold over [a, 2] per sweep, <= 200) */
    int32_t max_sweeps;   /* filter sweeps per sector (0: 200)                          */
    int32_t reserved;
    double tol;           /* residue |A_s u - theta u| required of the Ritz pairs below the
                             cut (0: 1e-7); the first pair above the cut must satisfy
                             theta - residue > zero_cut, and the null space must have been
                             amplified 1e12-fold by the filter sweeps                    */
    double zero_cut;      /* Ritz values theta < zero_cut count as zero modes (0: 1e-7);
                             must exceed the approximant's error delta                   */
} ndq_index_params;

typedef struct {
    int32_t n_plus, n_minus;   /* zero modes of chirality +1 and -1                      */
    int32_t index;             /* n_plus - n_minus                                        */
    int32_t block;             /* block size used                                         */
    int32_t sweeps[2];         /* filter sweeps, sector + then -                          */
    int32_t converged[2];
    int32_t degree[2];         /* filter degree of the last sweep                         */
    double theta[2][NDQ_INDEX_REPORT];   /* lowest Ritz values of A_+ and A_-, ascending */
    double resid[2][NDQ_INDEX_REPORT];   /* their residues                               */
    int64_t sign_applies;
    double seconds;
} ndq_index_info;

size_t ndq_index_workspace_bytes(const ndq_geom* g, const ndq_overlap_params* p, const ndq_index_params* params);

/*   U: FP64 links;  p: overlap parameters (approximant, lam_max, Wilson mass m, optional
 *   exact low modes of Q; mq is not used; the projection of Eq. 11 is applied in its
 *   sandwich form, so that A_s is Hermitian);  params: NULL for the defaults;
 *   start: one nonzero FP64 NDQ_FULL field (the block start vectors are phase-
 *   randomised, chirally projected copies);  info: out (filled also on error).
 *   Synchronises `stream`.  Errors: NDQ_EINVAL, NDQ_EPREC, NDQ_ENOMEM (workspace),
 *   NDQ_ENOCONV (sweep limit, or every converged Ritz value of a sector below the
 *   cut: the block is too small), NDQ_ENAN (the block lost rank). */
int ndq_index_DN(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p, const ndq_index_params* params,
                 const ndq_spinor* start, ndq_index_info* info, void* ws, size_t ws_bytes, void* stream);

/* ---- derivatives (not in the paper; follow from Eq. 1) --------------------- */
/* For y = Q[U] psi and a cotangent g (dL = Re<g, dy>): the su(3) link force
 *   F^a_mu(x) = dL/dw for U_mu(x) -> exp(i w T_a) U_mu(x),  T_a = lambda_a / 2,
 * into d_force (device, double [V][4][8], lexicographic sites) and/or the
 * tangent-space gradient 2 i sum_a F^a T_a U_mu(x) into d_grad (device, complex128
 * [V][4][3][3]), i.e. the gradient with respect to the complex link tensor in the
 * convention dL = Re<grad, dU>.  (The spinor gradient is Q g: Q is Hermitian.)
 * FP64 links and spinors, NDQ_FULL, nrhs 1; either output may be NULL, not both.
 * Asynchronous. */
int ndq_gauge_force(const ndq_geom* g, const ndq_gauge* U, const ndq_spinor* psi, const ndq_spinor* gy,
                    double* d_force, void* d_grad, void* stream);

/* ---- launch tuning ------------------------------------------------------ */
/* Launch shape of the stencil kernels: `block` = 64, 128 or 256 lanes with one
 * lane per output site, or 0 for the direction-split form (4 wavefronts per 64
 * sites, one per direction mu, combined in LDS; more wavefronts in flight on
 * small lattices); `xcd_remap` remaps workgroups so that each of the 8 XCDs
 * works on one contiguous range of sites (neighbour re-reads then stay in that
 * XCD's L2).  Process-wide; not thread-safe against concurrent launches.
 * Errors: NDQ_EINVAL. */
int ndq_set_launch(int block, int xcd_remap);

/* The same for one storage format only (spinor precision, link precision,
 * recon); the autotuner records its choice per format this way. */
int ndq_set_launch_for(int sprec, int lprec, int recon, int block, int xcd_remap);

/* Work order of the multi-right-hand-side stencil (nrhs > 1: ndq_apply_Q,
 * ndq_apply_dslash and the block forms of sign, D_N and solve) for one lattice
 * g, storage format (spinor precision, link precision, recon), nrhs and number
 * ny of output parities per launch (1: dslash, 2: Q): rg right-hand sides per
 * workgroup of 64 sites (0: all nrhs; the links of a tile are staged in LDS
 * once per workgroup), group_major = 1 runs every tile for one group of rg
 * fields before the next group (the neighbour spinors re-read by nearby tiles
 * then stay in the caches), 0 runs the groups of a tile next to each other,
 * 2 gives each XCD one group and one part of the tiles (the number of groups
 * must divide 8, else group-major is used): the XCDs walk the same tiles
 * together, sharing the links through the last-level cache;
 * chunk: -1 automatic, 0 tiles in index order, c > 0 c consecutive tiles of
 * every time slice in turn (c must divide the 64-site tiles of a slice);
 * xcd_remap as in ndq_set_launch; link_nt: links loaded with the non-temporal
 * hint (1), without (0), or automatic (-1: when each link is read once).
 * Results do not depend on the work order.  Process-wide.  Errors: NDQ_EINVAL. */
int ndq_set_mrhs_launch(const ndq_geom* g, int sprec, int lprec, int recon, int nrhs, int ny, int rg,
                        int group_major, int chunk, int xcd_remap, int link_nt);
int ndq_get_mrhs_launch(const ndq_geom* g, int sprec, int lprec, int recon, int nrhs, int ny, int* rg,
                        int* group_major, int* chunk, int* xcd_remap, int* link_nt);

/* The launch shape currently used for one storage format (host outputs). */
int ndq_get_launch_for(int sprec, int lprec, int recon, int* block, int* xcd_remap);

/* Autotuner of the launch shape: times `reps` even/odd dslash applies on
 * lattice g with links U and spinors of precision sprec for each launch shape
 * (block 0/64/128/256, XCD remap off/on, tiles in index order or in the
 * slice-chunked order that keeps neighbouring time slices of a tile close in
 * time), on ceil(rotate_bytes / set size)
 * rotating copies of (links, even spinor, odd spinor) so that consecutive
 * applies stream from HBM as in a solver (rotate_bytes <= 0: one set), and
 * records the fastest shape for dslash launches of that storage format on
 * this lattice (other lattices keep the format's shape of ndq_set_launch_for,
 * and a later ndq_set_launch_for of the format replaces the tuned shapes);
 * the shape already in use is kept if it is within 3% of the fastest.  The
 * copies live in the caller's workspace ws of at least
 * ndq_autotune_workspace_bytes(g, U, sprec, rotate_bytes) bytes (the first set
 * uses U itself).  ndq_autotune_q does the same for the full Q launches (both
 * output parities in one launch, as in ndq_apply_Q and the sign iterations)
 * with full-field sets (ndq_autotune_q_workspace_bytes).  Synchronises
 * `stream`.  Errors: NDQ_EINVAL, NDQ_EPREC, NDQ_ENOMEM, NDQ_EHIP (the previous
 * shape is kept). */
typedef struct {
    int32_t block;        /* chosen shape                                            */
    int32_t xcd_remap;
    double us_best;       /* its average time per dslash, microseconds               */
    double us[8];         /* every shape: index 2 * b + xcd_remap, b over 0/64/128/256 */
    int32_t nsets;        /* rotating sets used                                      */
    int32_t order;        /* chosen tile order: 0 index order, 1 slice-chunked order  */
    double us_order[8];   /* every shape with the slice-chunked tile order           */
} ndq_tune_result;
size_t ndq_autotune_workspace_bytes(const ndq_geom* g, const ndq_gauge* U, int sprec, int64_t rotate_bytes);
int ndq_autotune(const ndq_geom* g, const ndq_gauge* U, int sprec, int reps, int64_t rotate_bytes, void* ws,
                 size_t ws_bytes, ndq_tune_result* out, void* stream);
size_t ndq_autotune_q_workspace_bytes(const ndq_geom* g, const ndq_gauge* U, int sprec, int64_t rotate_bytes);
int ndq_autotune_q(const ndq_geom* g, const ndq_gauge* U, int sprec, int reps, int64_t rotate_bytes, void* ws,
                   size_t ws_bytes, ndq_tune_result* out, void* stream);

/* The launch shape used on lattice g for one storage format and launch kind
 * (ny = 1: dslash, 2: Q): the autotuner's choice for this lattice, else the
 * format's (host outputs). */
int ndq_get_launch_lattice(const ndq_geom* g, int sprec, int lprec, int recon, int ny, int* block, int* xcd_remap);

/* Autotuner of the multi-right-hand-side work order (see ndq_set_mrhs_launch)
 * for lattice g, links U, spinor precision sprec, nrhs >= 2 fields and ny
 * output parities (2: Q, 1: the even/odd hopping block): times `reps` applies
 * of the order in use and of each candidate (fields per workgroup nrhs,
 * nrhs/2, nrhs/3, 6, 4, 2; group- and tile-major; automatic, index-order and
 * two-x1-row tile chunks) on a block of fields in ws (at least
 * ndq_autotune_mrhs_workspace_bytes(g, sprec, nrhs, ny) bytes), and records the
 * fastest, keeping the order in use unless another is more than 3% faster.
 * If the environment variable NDQ_TUNE_CACHE names a file, an entry for this
 * key found there is applied without timing (cached = 1) and a new result is
 * appended to it (one text line per key).  Synchronises `stream`.
 * Errors: NDQ_EINVAL, NDQ_EPREC, NDQ_ENOMEM, NDQ_EHIP. */
typedef struct {
    int32_t rg, group_major, chunk, xcd_remap, link_nt;   /* chosen order             */
    int32_t nshapes;      /* candidates timed                                           */
    int32_t cached;       /* 1: taken from NDQ_TUNE_CACHE                                */
    double us_best;       /* time per apply of the chosen order, microseconds            */
    double us_previous;   /* of the order in use before the call                         */
} ndq_mrhs_tune_result;
size_t ndq_autotune_mrhs_workspace_bytes(const ndq_geom* g, int sprec, int nrhs, int ny);
int ndq_autotune_mrhs(const ndq_geom* g, const ndq_gauge* U, int sprec, int nrhs, int ny, int reps, void* ws,
                      size_t ws_bytes, ndq_mrhs_tune_result* out, void* stream);

/* Grid of the persistent multi-lattice launch (ndq_apply_Q_multi): `factor`
 * times the workgroups the device holds at once, 1 <= factor <= 16 (default 4).
 * Process-wide; results do not depend on it (each tile is computed the same
 * way whichever workgroup takes it).  Errors: NDQ_EINVAL. */
int ndq_set_multi_grid(int factor);
int ndq_get_multi_grid(void);

/* Autotuner of that grid for one set of jobs (as ndq_apply_Q_multi): times
 * `reps` launches at each factor of 1, 2, 3, 4, 6, 8 and 12 on the jobs' own
 * fields (every launch writes out = Q in, so the outputs end as one
 * ndq_apply_Q_multi would leave them), and sets the fastest, keeping the
 * factor in use unless another is more than 3% faster.  No workspace.
 * Synchronises `stream`.  Errors: those of ndq_apply_Q_multi, NDQ_EHIP. */
typedef struct {
    int32_t factor;       /* chosen factor                                             */
    int32_t nfactors;     /* factors timed (us[0 .. nfactors-1], in the order above)   */
    double us[8];         /* time per launch at each factor, microseconds              */
    double us_best;       /* of the chosen factor                                      */
    double us_previous;   /* of the factor in use before the call                      */
} ndq_multi_tune_result;
int ndq_autotune_multi(const ndq_q_job* jobs, int32_t njobs, int reps, ndq_multi_tune_result* out, void* stream);

/* Gram matrix of two blocks of fields, G[i][j] = <A_i, B_j> = sum over sites and
 * spin-colour components of conj(A_i) B_j (the inner products of the
 * Rayleigh-Ritz step of Sec. 2.3), computed on the FP64 matrix cores.
 *   A, B: F64 NDQ_FULL spinors with nrhs = na, nb in [1, 64] (a block is nrhs
 *   consecutive fields);  d_G: device, na x nb complex doubles (re, im), row-major;
 *   ws: device workspace of ndq_gram_workspace_bytes(g, na, nb) bytes.
 * Asynchronous.  Errors: NDQ_EINVAL, NDQ_EPREC, NDQ_ENOMEM. */
size_t ndq_gram_workspace_bytes(const ndq_geom* g, int na, int nb);
int ndq_spinor_gram(const ndq_geom* g, const ndq_spinor* A, const ndq_spinor* B, void* d_G, void* ws,
                    size_t ws_bytes, void* stream);

/* ---- diagnostics -------------------------------------------------------- */
const char* ndq_last_error(void);
const char* ndq_status_string(int status);
/* Library version string, e.g. "ndq 0.1 gfx950". */
const char* ndq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NDQ_H */
