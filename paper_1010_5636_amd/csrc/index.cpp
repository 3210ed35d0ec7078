// Index of the massless Neuberger-Dirac operator by zero-mode counting, the
// workload the outlook of Sec. 4 names next, on the operator of Eq. 4 with
// m_q = 0: D = (1 + gamma5 eps) / abar, eps the approximate sign of Q with
// exact low modes (Eq. 11).
//
// D^H D commutes with gamma5.  On the chirality-s subspace (gamma5 psi = s psi,
// s = +-1) it equals (2 / abar^2) A_s with
//     A_s = 1 + s P_s eps P_s,   P_s = (1 + s gamma5) / 2,
// (using eps^2 = 1), so the zero modes of D of chirality s are the kernel of
// A_s, whose spectrum lies in [0, 2].  The lowest eigenpairs of A_s are found
// in each sector by block Chebyshev-filtered subspace iteration (Zhou & Saad):
// a block of nb chiral vectors is filtered by T_d of A_s mapped from
// [a, 2 + margin] onto [-1, 1] (a = the block's largest Ritz value; d chosen
// so that one sweep amplifies the null space about 1e4-fold over [a, 2]),
// orthonormalised (Gram matrix on the matrix cores, applied twice) and rotated
// onto the Ritz vectors of A_s.  Once the null space has been amplified
// 1e12-fold in total, the Ritz pairs below the cut have residues <= tol and
// the first pair above the cut lies clearly above it, the pairs below the
// cut are counted: n_s.  The index is n_+ - n_-.  One application of A_s is one sign
// apply; everything else is BLAS on FP64 fields.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <complex>
#include <vector>

#include "ndq_eig.h"
#include "ndq_solver.h"

namespace ndq {
namespace {

using cd = std::complex<double>;

constexpr double kUpperMargin = 0.05;   // |eps| <= 1 + delta: A_s <= 2 + delta
// Lowest filter cutoff.  When the block lies inside a degenerate null space
// larger than the block, its largest Ritz value tends to zero, and a cutoff
// following it would stop damping the rest of the spectrum; below this floor
// the interval [floor, 2] stays damped and the block still converges into
// the null space (and is then reported as too small).
constexpr double kCutoffFloor = 1e-2;
// Fields per block sign application (the block sign takes at most NDQ_MAX_BATCH).
constexpr int kSignBlock = NDQ_MAX_BATCH;

struct IxCtx {
    const ndq_geom* g;
    const ndq_gauge* U;
    const ndq_overlap_params* p;
    hipStream_t st;
    int64_t vb;                 // bytes per FP64 full spinor
    char* sign_ws;
    size_t sign_bytes;
    ndq_spinor S, R;            // sign output, residual scratch
    double *gpart, *G, *Y, *partials, *scal;
    int64_t signs = 0;

    ndq_spinor vec(char* base, int i) const { return ndq_spinor{base + (int64_t)i * vb, NDQ_F64, NDQ_FULL, 1}; }
    // fields i .. i+n-1 of a block, as one descriptor
    ndq_spinor vecs(char* base, int i, int n) const {
        return ndq_spinor{base + (int64_t)i * vb, NDQ_F64, NDQ_FULL, n};
    }

    // out = sign(Q) in for every field of the block `in` (one block sign: the
    // stencil applications of the recurrence serve all its fields)
    int sign(const ndq_spinor* in, const ndq_spinor* out) {
        Arena ar{sign_ws, sign_bytes};
        signs += in->nrhs;
        return apply_sign(g, U, p, in, out, ar, nullptr, st);
    }
    int norm2(const ndq_spinor* x, double* out) {
        int rc = dot(g, x, nullptr, partials, scal, st);
        if (rc) return rc;
        NDQ_HIP(hipMemcpyAsync(out, scal, sizeof(double), hipMemcpyDeviceToHost, st));
        NDQ_HIP(hipStreamSynchronize(st));
        return NDQ_OK;
    }
    // host h = A^H B (na x nb, row-major)
    int gram_host(char* A, int na, char* B, int nb, std::vector<cd>& h) {
        int rc = gram(g, A, na, B, nb, gpart, G, st);
        if (rc) return rc;
        h.resize((size_t)na * nb);
        NDQ_HIP(hipMemcpyAsync(h.data(), G, sizeof(cd) * h.size(), hipMemcpyDeviceToHost, st));
        NDQ_HIP(hipStreamSynchronize(st));
        return NDQ_OK;
    }
    // dst = src Z for a host matrix Z (nsrc x k, row-major)
    int rotate_host(char* src, int nsrc, const std::vector<cd>& Z, int k, char* dst) {
        NDQ_HIP(hipMemcpyAsync(Y, Z.data(), sizeof(cd) * (size_t)nsrc * k, hipMemcpyHostToDevice, st));
        NDQ_HIP(hipStreamSynchronize(st));   // Z is the caller's host memory
        return rotate(g, src, nsrc, Y, k, dst, st);
    }
};

// out = ax x + bA (A_s x) + cw w   (w optional; out may alias x or w):
// A_s x = x + (s/2) eps x + (1/2) gamma5 eps x for a chirality-s vector x.
// x, out and w may be blocks of up to kSignBlock fields.
int as_combo(IxCtx& c, int s, const ndq_spinor* x, const ndq_spinor* out, double ax, double bA,
             const ndq_spinor* w = nullptr, double cw = 0.0) {
    ndq_spinor S = c.S;
    S.nrhs = x->nrhs;
    int rc = c.sign(x, &S);
    if (rc) return rc;
    const ndq_spinor* v[4] = {x, &S, &S, w};
    const Coef cf[4] = {Coef{ax + bA, nullptr}, Coef{0.5 * s * bA, nullptr}, Coef{0.5 * bA, nullptr},
                        Coef{cw, nullptr}};
    const int g5[4] = {0, 0, 1, 0};
    return lincomb(c.g, NDQ_F64, out, w ? 4 : 3, v, cf, g5, nullptr, c.st);
}

// x <- P_s x = (x + s gamma5 x) / 2
int project(IxCtx& c, int s, const ndq_spinor* x) {
    const ndq_spinor* v[2] = {x, x};
    const Coef cf[2] = {Coef{0.5, nullptr}, Coef{0.5 * s, nullptr}};
    const int g5[2] = {0, 1};
    return lincomb(c.g, NDQ_F64, x, 2, v, cf, g5, nullptr, c.st);
}

int copy(IxCtx& c, const ndq_spinor* dst, const ndq_spinor* src) {
    const ndq_spinor* v[1] = {src};
    const Coef cf[1] = {Coef{1.0, nullptr}};
    return lincomb(c.g, NDQ_F64, dst, 1, v, cf, nullptr, nullptr, c.st);
}

// F_j = T_d(A~) X_j for every vector of the block, A~ = (2 A_s - (a + b)) / (b - a).
// T_{k+1} = 2 A~ T_k - T_{k-1} overwrites T_{k-1}; X is destroyed.
// The vectors go through in sub-blocks of up to kSignBlock fields.
int filter(IxCtx& c, int s, char* X, char* F, int nb, double a, double b, int d) {
    const double c1 = 2.0 / (b - a), c2 = -(a + b) / (b - a);
    int rc;
    for (int j = 0; j < nb; j += kSignBlock) {
        const int n = std::min(kSignBlock, nb - j);
        ndq_spinor tp = c.vecs(X, j, n), tc = c.vecs(F, j, n);
        if ((rc = as_combo(c, s, &tp, &tc, c2, c1))) return rc;   // T_1
        for (int k = 2; k <= d; ++k) {
            if ((rc = as_combo(c, s, &tc, &tp, 2.0 * c2, 2.0 * c1, &tp, -1.0))) return rc;
            std::swap(tp, tc);
        }
        if (tc.data != F + (int64_t)j * c.vb) {
            const ndq_spinor fj = c.vecs(F, j, n);
            if ((rc = copy(c, &fj, &tc))) return rc;
        }
    }
    return NDQ_OK;
}

// dst = src G^{-1/2} (G = src^H src), so that dst is orthonormal.
int orthonormalise(IxCtx& c, char* src, char* dst, int nb) {
    std::vector<cd> G, Z;
    std::vector<double> w;
    int rc = c.gram_host(src, nb, src, nb, G);
    if (rc) return rc;
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < i; ++j) G[(size_t)i * nb + j] = std::conj(G[(size_t)j * nb + i]);
    for (int i = 0; i < nb; ++i) G[(size_t)i * nb + i] = G[(size_t)i * nb + i].real();
    if ((rc = hermitian_eig(nb, G, w, Z))) return rc;
    if (!(w[0] > 1e-28 * w[nb - 1]) || !isfinite(w[nb - 1]))
        return fail(NDQ_ENAN, "index: the block lost rank (Gram eigenvalues %g .. %g)", w[0], w[nb - 1]);
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) Z[(size_t)i * nb + j] /= sqrt(w[j]);
    return c.rotate_host(src, nb, Z, nb, dst);
}

struct Sector {
    std::vector<double> theta, resid;
    int sweeps = 0;
    int count = 0;
    int degree = 0;          // filter degree of the last sweep
    double log_amp = 0.0;    // log of the null space's total amplification over [a, 2]
    bool converged = false;
};

// Filter degree that amplifies the null space by about kAmplify over the
// damped interval [a, b] in one sweep: |T_d(A~(0))| = cosh(d acosh((a + b) / (b - a))).
constexpr double kAmplify = 1e4;
constexpr int kMaxDegree = 200;
// Total amplification of the null space before a count is accepted: a null
// vector's weight in a random start vector is about dim^{-1/2} (>= 1e-4 for
// the lattices here), so after 1e12 it dominates every other direction by
// about 1e8 and cannot be missing from a block that still has room.
constexpr double kMinAmplification = 1e12;
double log_amplification(double a, double b, int d) {
    const double t = d * acosh((a + b) / (b - a));
    return t + log1p(exp(-2.0 * t)) - log(2.0);   // log cosh t
}
int adaptive_degree(double a, double b) {
    const double x = (a + b) / (b - a);
    const double d = ceil(acosh(kAmplify) / acosh(x));
    return (int)std::min<double>(std::max(d, 4.0), kMaxDegree);
}

// Rayleigh-Ritz of A_s in span(X) (orthonormal, nb vectors): W = A_s X into
// free1, M = X^H W, the Ritz vectors X Z into free2 and A_s X Z into X's
// block, residues |A_s u_j - theta_j u_j|.  On return X names the Ritz
// vectors and free1, free2 the two blocks no longer needed.
int rayleigh_ritz(IxCtx& c, int s, char*& X, char*& free1, char*& free2, int nb, Sector& sec) {
    int rc;
    for (int j = 0; j < nb; j += kSignBlock) {
        const int n = std::min(kSignBlock, nb - j);
        const ndq_spinor xj = c.vecs(X, j, n), wj = c.vecs(free1, j, n);
        if ((rc = as_combo(c, s, &xj, &wj, 0.0, 1.0))) return rc;
    }
    std::vector<cd> M, Z;
    if ((rc = c.gram_host(X, nb, free1, nb, M))) return rc;
    std::vector<cd> H((size_t)nb * nb);
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) H[(size_t)i * nb + j] = 0.5 * (M[(size_t)i * nb + j] + std::conj(M[(size_t)j * nb + i]));
    if ((rc = hermitian_eig(nb, H, sec.theta, Z))) return rc;
    if ((rc = c.rotate_host(X, nb, Z, nb, free2))) return rc;      // Ritz vectors
    if ((rc = c.rotate_host(free1, nb, Z, nb, X))) return rc;      // A_s times them
    sec.resid.assign(nb, 0.0);
    for (int j = 0; j < nb; ++j) {
        const ndq_spinor uj = c.vec(free2, j), wj = c.vec(X, j);
        const ndq_spinor* v[2] = {&wj, &uj};
        const Coef cf[2] = {Coef{1.0, nullptr}, Coef{-sec.theta[j], nullptr}};
        if ((rc = lincomb(c.g, NDQ_F64, &c.R, 2, v, cf, nullptr, nullptr, c.st))) return rc;
        double r2;
        if ((rc = c.norm2(&c.R, &r2))) return rc;
        sec.resid[j] = sqrt(std::max(r2, 0.0));
    }
    // new X = free2; the old X block (A_s U) and free1 are free
    std::swap(X, free2);
    return NDQ_OK;
}

int run_sector(IxCtx& c, int s, const ndq_spinor* start, char* B0, char* B1, char* B2, const ndq_index_params& ip,
               Sector& sec) {
    const int nb = ip.block;
    int rc;
    for (int j = 0; j < nb; ++j) {
        const ndq_spinor xj = c.vec(B1, j);
        if ((rc = phase_copy(c.g, start, &xj, 1 + j + (s > 0 ? 0 : 64), c.st))) return rc;
        if ((rc = project(c, s, &xj))) return rc;
    }
    char *X = B0, *F1 = B1, *F2 = B2;
    if ((rc = orthonormalise(c, F1, X, nb))) return rc;
    if ((rc = rayleigh_ritz(c, s, X, F1, F2, nb, sec))) return rc;
    const double up = 2.0 + kUpperMargin;
    for (sec.sweeps = 0;; ++sec.sweeps) {
        // Accept the count once the null space has been amplified enough that
        // no zero mode can be missing from the block, the pairs below the cut
        // have converged, and the first pair above it lies clearly above the
        // cut (an eigenvalue within its residue of theta).
        int below = 0;
        while (below < nb - 1 && sec.theta[below] < ip.zero_cut) ++below;
        bool ok = sec.log_amp >= log(kMinAmplification);
        for (int j = 0; j < below; ++j) ok = ok && sec.resid[j] <= ip.tol;
        if (below < nb - 1) ok = ok && sec.theta[below] - sec.resid[below] > ip.zero_cut;
        sec.count = below;
        if (ok) {
            if (below >= nb - 1)
                return fail(NDQ_ENOCONV, "index: every converged Ritz value of chirality %+d is below the cut; "
                                         "a block of %d vectors is too small", s, nb);
            sec.converged = true;
            return NDQ_OK;
        }
        if (sec.sweeps >= ip.max_sweeps)
            return fail(NDQ_ENOCONV, "index: chirality %+d not converged after %d sweeps (largest residue below "
                        "the cut %g, tol %g)", s, sec.sweeps,
                        below ? *std::max_element(sec.resid.begin(), sec.resid.begin() + below) : 0.0, ip.tol);
        const double a = std::min(std::max(sec.theta[nb - 1], kCutoffFloor), 1.9);
        sec.degree = ip.degree > 0 ? ip.degree : adaptive_degree(a, up);
        if ((rc = filter(c, s, X, F1, nb, a, up, sec.degree))) return rc;
        sec.log_amp += log_amplification(a, up, sec.degree);
        // two passes: the filtered block can be ill-conditioned
        if ((rc = orthonormalise(c, F1, X, nb))) return rc;
        if ((rc = orthonormalise(c, X, F1, nb))) return rc;
        std::swap(X, F1);
        if ((rc = rayleigh_ritz(c, s, X, F1, F2, nb, sec))) return rc;
    }
}

void with_defaults(const ndq_index_params* in, ndq_index_params& ip) {
    memset(&ip, 0, sizeof(ip));
    if (in) ip = *in;
    if (ip.block == 0) ip.block = 8;
    if (ip.max_sweeps == 0) ip.max_sweeps = 200;
    if (ip.tol == 0.0) ip.tol = 1e-7;
    if (ip.zero_cut == 0.0) ip.zero_cut = 1e-7;
}

size_t index_workspace(const ndq_geom* g, const ndq_overlap_params* p, const ndq_index_params& ip) {
    const int nsb = std::min(kSignBlock, ip.block);
    Arena ar{nullptr, 0};
    ar.take(sign_workspace(g, p, NDQ_F64, nsb));
    const size_t vb = (size_t)spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL);
    for (int k = 0; k < 3; ++k) ar.take(vb * ip.block);
    ar.take(vb * nsb);
    ar.take(vb);
    ar.take(gram_partials_bytes(g, ip.block, ip.block));
    ar.take(sizeof(cd) * 64 * 64);
    ar.take(sizeof(cd) * 64 * 64);
    ar.take(partials_capacity(g, 1));
    ar.take(256);
    return ar.used + 256;
}

}  // namespace
}  // namespace ndq

using namespace ndq;

extern "C" {

size_t ndq_index_workspace_bytes(const ndq_geom* g, const ndq_overlap_params* p, const ndq_index_params* params) {
    if (!g || !p || !p->approx || p->nev < 0 || p->nev > NDQ_MAX_MODES) return 0;
    ndq_index_params ip;
    with_defaults(params, ip);
    if (ip.block < 2 || ip.block > 64) return 0;
    const ndq_overlap_params ph = hermitian_form(p);
    return index_workspace(g, &ph, ip);
}

int ndq_index_DN(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p, const ndq_index_params* params,
                 const ndq_spinor* start, ndq_index_info* info, void* ws, size_t ws_bytes, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
    if (info) memset(info, 0, sizeof(*info));
    if (!g || !U || !p || !start || !info) return fail(NDQ_EINVAL, "index: NULL argument");
    ndq_index_params ip;
    with_defaults(params, ip);
    if (ip.block < 2 || ip.block > 64) return fail(NDQ_EINVAL, "index: block must be in [2, 64]");
    if (ip.degree < 0 || ip.degree > 1000) return fail(NDQ_EINVAL, "index: degree must be in [0, 1000]");
    if (ip.max_sweeps < 1) return fail(NDQ_EINVAL, "index: max_sweeps must be positive");
    if (!(ip.tol > 0) || !(ip.zero_cut > 0)) return fail(NDQ_EINVAL, "index: tol and zero_cut must be positive");
    int rc = check_gauge(U);
    if (!rc) rc = check_spinor(g, start, NDQ_FULL, "index start");
    if (rc) return rc;
    if (start->prec != NDQ_F64 || start->nrhs != 1 || U->prec != NDQ_F64)
        return fail(NDQ_EPREC, "index: FP64 links and one FP64 start field required");
    if (!p->approx) return fail(NDQ_EINVAL, "index: no approximant");
    // A_s must be Hermitian for its Rayleigh-Ritz step: sandwich projection
    const ndq_overlap_params ph = hermitian_form(p);
    p = &ph;
    const size_t need = index_workspace(g, p, ip);
    if (!ws || ws_bytes < need) return fail(NDQ_ENOMEM, "index: workspace too small (need %zu bytes)", need);

    hipStream_t st = as_stream(stream);
    Arena ar{static_cast<char*>(ws), ws_bytes};
    IxCtx c;
    c.g = g;
    c.U = U;
    c.p = p;
    c.st = st;
    c.vb = spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL);
    const int nsb = std::min(kSignBlock, ip.block);
    c.sign_bytes = sign_workspace(g, p, NDQ_F64, nsb);
    c.sign_ws = static_cast<char*>(ar.take(c.sign_bytes));
    char* B[3];
    for (int k = 0; k < 3; ++k) B[k] = static_cast<char*>(ar.take((size_t)c.vb * ip.block));
    c.S = ws_block(ar, g, NDQ_F64, nsb);
    c.R = ws_spinor(ar, g, NDQ_F64);
    c.gpart = static_cast<double*>(ar.take(gram_partials_bytes(g, ip.block, ip.block)));
    c.G = static_cast<double*>(ar.take(sizeof(cd) * 64 * 64));
    c.Y = static_cast<double*>(ar.take(sizeof(cd) * 64 * 64));
    c.partials = static_cast<double*>(ar.take(partials_capacity(g, 1)));
    c.scal = static_cast<double*>(ar.take(256));
    if (ar.overflow) return fail(NDQ_ENOMEM, "index: workspace too small (need %zu bytes)", ar.used);

    Sector sec[2];
    int status = NDQ_OK;
    for (int k = 0; k < 2 && status == NDQ_OK; ++k) status = run_sector(c, k == 0 ? 1 : -1, start, B[0], B[1], B[2], ip, sec[k]);
    info->block = ip.block;
    for (int k = 0; k < 2; ++k) {
        const int n = std::min<int>((int)sec[k].theta.size(), NDQ_INDEX_REPORT);
        for (int j = 0; j < n; ++j) {
            info->theta[k][j] = sec[k].theta[j];
            info->resid[k][j] = sec[k].resid[j];
        }
        info->sweeps[k] = sec[k].sweeps;
        info->degree[k] = sec[k].degree;
        info->converged[k] = sec[k].converged ? 1 : 0;
    }
    info->n_plus = sec[0].count;
    info->n_minus = sec[1].count;
    info->index = info->n_plus - info->n_minus;
    info->sign_applies = c.signs;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

}  // extern "C"
