// Low modes of Q in FP64 on the GPU (Sec. 2.3): the space V of the l lowest
// modes, the Rayleigh-Ritz vectors u_k in V with P Q u_k = nu_k u_k, their
// residues rho_k = |(Q - nu_k) u_k| (Eq. 8), kappa_+- (Eq. 9) and the projector
// bound of Eq. 10.
//
// Two methods find V, both built on the Chebyshev filter B = T_d(A~):
//  * block Chebyshev-filtered subspace iteration (default; Zhou & Saad): a block
//    of nev + nextra vectors is filtered, orthonormalised and rotated onto the
//    Ritz vectors of Q each iteration; the cutoff a follows the block's largest
//    Ritz value of Q^2 and the degree d the gap to the guard pair, so the filter
//    sharpens as the block converges; degenerate eigenspaces are no obstacle.
//    Optionally the filter of the early iterations runs on F32 copies of the
//    block with F32 links (half the bytes per stencil application): FP32
//    rounding limits the residues such a filtered block can reach to about
//    1e-5 relative, far below those of the first iterations; once the residues
//    fall below a switch point, or three F32 iterations pass without halving
//    the best of them, the filter is FP64, and the
//    orthonormalisation, Rayleigh-Ritz step and convergence test are FP64
//    throughout;
//  * thick-restart Lanczos (Wu & Simon) on B = T_d(A~), a Chebyshev
// polynomial of A = Q^2 mapped from [a, lam_max^2] onto [-1, 1]: the low end of
// the spectrum (below the cutoff a) becomes the dominant part of B's spectrum.
// Every Lanczos vector is orthogonalised twice against the whole basis
// (classical Gram-Schmidt, FP64).  The cutoff a comes from a short plain
// Lanczos run on A (its Ritz values bound the eigenvalues from above).  After
// each restart cycle the kept B-Ritz vectors are checked by Rayleigh-Ritz with
// Q itself; the cycle stops once every returned rho_k <= tol * lam_max and the
// next Ritz pair (whose |nu| is reported as lam_next) has rho <= max(tol, 1e-6) * lam_max.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <complex>
#include <numeric>
#include <vector>

#include "ndq_eig.h"
#include "ndq_solver.h"

namespace ndq {
namespace {

using cd = std::complex<double>;

struct LmCtx {
    const ndq_geom* g;
    const ndq_gauge* U;
    double m;
    hipStream_t st;
    int64_t vb;              // bytes per FP64 full spinor
    char *VA, *VB, *W, *QU, *UU;
    char* SB = nullptr;      // block of nkeep vectors: Q T_k of the block filter
    const ndq_gauge* Ulo = nullptr;   // F32 links for the early filter restarts (or null)
    char *XL = nullptr, *YL = nullptr, *SL = nullptr;   // F32 blocks of nkeep vectors
    int64_t vbl = 0;         // bytes per F32 full spinor
    double* gpart = nullptr; // Gram partial tiles (matrix-core kernel)
    double* gout = nullptr;  // Gram matrix, device, up to 64 x 64 complex
    ndq_spinor X0, X1, S;
    double *partials, *dots, *Ydev, *coef, *scal;
    int64_t qcount = 0;

    ndq_spinor vec(char* base, int i) const { return ndq_spinor{base + (int64_t)i * vb, NDQ_F64, NDQ_FULL, 1}; }

    int qapply(const ndq_spinor* in, const ndq_spinor* out, double c0, int nv = 0, const ndq_spinor* const* v = nullptr,
               const Coef* cv = nullptr) {
        qcount += 1;
        return q_combo(g, U, m, in, out, Coef{c0, nullptr}, nv, v, cv, nullptr, st);
    }
    ndq_spinor block(char* base, int nb, int prec = NDQ_F64) const { return ndq_spinor{base, prec, NDQ_FULL, nb}; }
    // the same as qapply for the nb vectors of a block, in one multi-RHS launch
    // (on the F32 links for F32 blocks)
    int qapply_block(const ndq_spinor* in, const ndq_spinor* out, double c0, int nv = 0,
                     const ndq_spinor* const* v = nullptr, const Coef* cv = nullptr) {
        qcount += in->nrhs;
        return q_combo_block(g, in->prec == NDQ_F64 ? U : Ulo, m, in, out, Coef{c0, nullptr}, nv, v, cv, st);
    }
    int copy(const ndq_spinor* dst, const ndq_spinor* src, double c = 1.0) {
        const ndq_spinor* v[1] = {src};
        const Coef cc[1] = {Coef{c, nullptr}};
        return lincomb(g, NDQ_F64, dst, 1, v, cc, nullptr, nullptr, st);
    }
    int norm2(const ndq_spinor* x, double* out) {
        int rc = dot(g, x, nullptr, partials, scal, st);
        if (rc) return rc;
        NDQ_HIP(hipMemcpyAsync(out, scal, sizeof(double), hipMemcpyDeviceToHost, st));
        NDQ_HIP(hipStreamSynchronize(st));
        return NDQ_OK;
    }
    // host h[k] = <V_k, x>, k < n
    int dots_to_host(char* base, int n, const ndq_spinor* x, std::vector<cd>& h) {
        int rc = mode_dots(g, base, n, x, partials, dots, st);
        if (rc) return rc;
        h.resize(n);
        NDQ_HIP(hipMemcpyAsync(h.data(), dots, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, st));
        NDQ_HIP(hipStreamSynchronize(st));
        return NDQ_OK;
    }
    // x -= sum_k h[k] V_k
    int subtract(char* base, int n, const std::vector<cd>& h, const ndq_spinor* x) {
        std::vector<cd> neg(n);
        for (int k = 0; k < n; ++k) neg[k] = -h[k];
        NDQ_HIP(hipMemcpyAsync(coef, neg.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice, st));
        return mode_update(g, base, n, coef, x, x, st);
    }
};

// out = A v = Q Q v
int apply_A(LmCtx& c, const ndq_spinor* v, const ndq_spinor* out) {
    int rc = c.qapply(v, &c.S, 1.0);
    if (!rc) rc = c.qapply(&c.S, out, 1.0);
    return rc;
}

// out = T_d(A~) v, A~ = (2A - (a+b))/(b-a); three-term recurrence, two Q per degree
int apply_filter(LmCtx& c, const ndq_spinor* v, const ndq_spinor* out, double a, double b, int d) {
    const double c1 = 2.0 / (b - a), c2 = -(a + b) / (b - a);
    int rc;
    ndq_spinor* tp = &c.X0;   // T_{k-1}
    ndq_spinor* tc = &c.X1;   // T_k
    if ((rc = c.copy(tp, v))) return rc;
    if ((rc = c.qapply(v, &c.S, 1.0))) return rc;
    {
        const ndq_spinor* vv[1] = {v};
        const Coef cv[1] = {Coef{c2, nullptr}};
        if ((rc = c.qapply(&c.S, tc, c1, 1, vv, cv))) return rc;
    }
    for (int k = 2; k <= d; ++k) {
        if ((rc = c.qapply(tc, &c.S, 1.0))) return rc;
        const ndq_spinor* vv[2] = {tc, tp};
        const Coef cv[2] = {Coef{2.0 * c2, nullptr}, Coef{-1.0, nullptr}};
        if ((rc = c.qapply(&c.S, tp, 2.0 * c1, 2, vv, cv))) return rc;   // T_{k+1} into T_{k-1}'s buffer
        std::swap(tp, tc);
    }
    return c.copy(out, tc);
}

// Y = T_d(A~) X for all nb vectors of the block X at once (the recurrence of
// apply_filter with multi-RHS stencil launches: the links are read once per
// step for the whole block).  T_{k+1} overwrites T_{k-1}, so the iterates
// alternate between X and Y; X is overwritten.  S: a block of nb vectors
// (c.SB for FP64).  prec: of X, Y and S (F32: on c.Ulo, arithmetic in FP32).
int apply_filter_block(LmCtx& c, char* X, char* Y, char* S, int prec, int nb, double a, double b, int d) {
    const double c1 = 2.0 / (b - a), c2 = -(a + b) / (b - a);
    int rc;
    const ndq_spinor s = c.block(S, nb, prec);
    ndq_spinor tp = c.block(X, nb, prec);   // T_{k-1}
    ndq_spinor tc = c.block(Y, nb, prec);   // T_k
    if ((rc = c.qapply_block(&tp, &s, 1.0))) return rc;
    {
        const ndq_spinor* vv[1] = {&tp};
        const Coef cv[1] = {Coef{c2, nullptr}};
        if ((rc = c.qapply_block(&s, &tc, c1, 1, vv, cv))) return rc;
    }
    for (int k = 2; k <= d; ++k) {
        if ((rc = c.qapply_block(&tc, &s, 1.0))) return rc;
        const ndq_spinor* vv[2] = {&tc, &tp};
        const Coef cv[2] = {Coef{2.0 * c2, nullptr}, Coef{-1.0, nullptr}};
        if ((rc = c.qapply_block(&s, &tp, 2.0 * c1, 2, vv, cv))) return rc;   // T_{k+1} into T_{k-1}'s buffer
        std::swap(tp, tc);
    }
    const size_t bytes = (size_t)(prec == NDQ_F64 ? c.vb : c.vbl) * nb;
    if (tc.data != Y) NDQ_HIP(hipMemcpyAsync(Y, tc.data, bytes, hipMemcpyDeviceToDevice, c.st));
    return NDQ_OK;
}

// The block filter of the early restarts: X (FP64) rounded to F32, filtered with
// the F32 links in FP32 arithmetic, the result widened into Y (FP64).
int apply_filter_block_lo(LmCtx& c, char* X, char* Y, int nb, double a, double b, int d) {
    int rc;
    const ndq_spinor x64 = c.block(X, nb), y64 = c.block(Y, nb);
    const ndq_spinor xl = c.block(c.XL, nb, NDQ_F32), yl = c.block(c.YL, nb, NDQ_F32);
    if ((rc = convert(c.g, &xl, &x64, c.st))) return rc;
    if ((rc = apply_filter_block(c, c.XL, c.YL, c.SL, NDQ_F32, nb, a, b, d))) return rc;
    return convert(c.g, &y64, &yl, c.st);
}

// Lanczos steps j = j0 .. m-1 on the basis block `base` (m+1 vectors), recording
// the projected matrix T (column j: <V_i, B V_j> for i <= j+1).  op: 0 = A, 1 = filter.
int lanczos_steps(LmCtx& c, char* base, int j0, int m, std::vector<cd>& T, int op, double a, double b, int d) {
    int rc;
    std::vector<cd> h, h2;
    for (int j = j0; j < m; ++j) {
        const ndq_spinor vj = c.vec(base, j), w = c.vec(base, j + 1);
        rc = op == 0 ? apply_A(c, &vj, &w) : apply_filter(c, &vj, &w, a, b, d);
        if (rc) return rc;
        if ((rc = c.dots_to_host(base, j + 1, &w, h))) return rc;
        if ((rc = c.subtract(base, j + 1, h, &w))) return rc;
        if ((rc = c.dots_to_host(base, j + 1, &w, h2))) return rc;
        if ((rc = c.subtract(base, j + 1, h2, &w))) return rc;
        double b2;
        if ((rc = c.norm2(&w, &b2))) return rc;
        const double beta = sqrt(b2);
        if (!isfinite(beta)) return fail(NDQ_ENAN, "low modes: NaN in the Lanczos recurrence");
        for (int i = 0; i <= j; ++i) T[(size_t)i * m + j] = h[i] + h2[i];
        if (j + 1 < m) T[(size_t)(j + 1) * m + j] = beta;
        if (beta == 0.0) return fail(NDQ_ENOCONV, "low modes: invariant subspace reached (beta = 0)");
        if ((rc = c.copy(&w, &w, 1.0 / beta))) return rc;
    }
    return NDQ_OK;
}

// Hermitian completion of T from its upper triangle, eigen-decomposition.
void eig_T(const std::vector<cd>& T, int m, std::vector<double>& w, std::vector<cd>& z) {
    std::vector<cd> a((size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) a[(size_t)i * m + j] = i <= j ? T[(size_t)i * m + j] : std::conj(T[(size_t)j * m + i]);
    for (int i = 0; i < m; ++i) a[(size_t)i * m + i] = a[(size_t)i * m + i].real();
    hermitian_eig(m, a, w, z);
}

// Rayleigh-Ritz of Q in span(X[0..nb-1]) (orthonormal): W = Q X, M = X^H W.
// The Ritz pairs (nu_j, u_j) are ordered by theta_j = |Q u_j|^2 = z_j^H (W^H W) z_j,
// the Rayleigh quotient of A = Q^2, not by |nu_j|: Q is indefinite, and a
// block vector still mixing eigenvectors of opposite sign has a Ritz value
// near zero while theta stays large, so ordering by theta keeps such spurious
// pairs out of the wanted set.  X and W are rotated in place onto the ordered
// Ritz vectors (via the scratch blocks XS, WS) when `rotate_block`, and the
// first nsel pairs are written to UU / QU with their residues |Q u - nu u|.
// For the guard pair (index nsel - 1) also the residue of A,
// r = |A u - theta u|, so that an eigenvalue of A lies in [theta - r, theta + r].
struct RRResult {
    std::vector<double> nu;      // all nb Ritz values of Q, in theta order
    std::vector<double> theta;   // all nb Rayleigh quotients of A
    std::vector<double> rho;     // residues of Q for the first nsel
    double guard_res = 0.0;      // |A u - theta u| of pair nsel - 1
};

int rayleigh_ritz_q(LmCtx& c, char*& X, char*& W, char*& XS, char*& WS, int nb, int nsel, bool rotate_block,
                    RRResult& out) {
    const ndq_geom* g = c.g;
    int rc;
    {
        const ndq_spinor xb = c.block(X, nb), wb = c.block(W, nb);
        if ((rc = c.qapply_block(&xb, &wb, 1.0))) return rc;
    }
    // M = X^H W and G = W^H W, one pass over the blocks each (matrix cores)
    std::vector<cd> M((size_t)nb * nb), G((size_t)nb * nb);
    if ((rc = gram(g, X, nb, W, nb, c.gpart, c.gout, c.st))) return rc;
    NDQ_HIP(hipMemcpyAsync(M.data(), c.gout, sizeof(cd) * M.size(), hipMemcpyDeviceToHost, c.st));
    NDQ_HIP(hipStreamSynchronize(c.st));
    if ((rc = gram(g, W, nb, W, nb, c.gpart, c.gout, c.st))) return rc;
    NDQ_HIP(hipMemcpyAsync(G.data(), c.gout, sizeof(cd) * G.size(), hipMemcpyDeviceToHost, c.st));
    NDQ_HIP(hipStreamSynchronize(c.st));
    for (int i = 0; i < nb; ++i) {
        M[(size_t)i * nb + i] = M[(size_t)i * nb + i].real();
        for (int k = i + 1; k < nb; ++k) {
            const cd avg = 0.5 * (M[(size_t)i * nb + k] + std::conj(M[(size_t)k * nb + i]));
            M[(size_t)i * nb + k] = avg;
            M[(size_t)k * nb + i] = std::conj(avg);
        }
    }
    std::vector<double> nuv;
    std::vector<cd> zq;
    hermitian_eig(nb, M, nuv, zq);
    std::vector<double> th(nb);
    for (int j = 0; j < nb; ++j) {
        double t = 0.0;
        for (int i = 0; i < nb; ++i) {
            cd gz = 0.0;
            for (int k = 0; k < nb; ++k) gz += G[(size_t)i * nb + k] * zq[(size_t)k * nb + j];
            t += (std::conj(zq[(size_t)i * nb + j]) * gz).real();
        }
        th[j] = t;
    }
    std::vector<int> idx(nb);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int i, int j) { return th[i] < th[j]; });
    const int ncol = rotate_block ? nb : nsel;
    std::vector<cd> Z((size_t)nb * ncol);
    out.nu.resize(nb);
    out.theta.resize(nb);
    for (int j = 0; j < nb; ++j) {
        out.nu[j] = nuv[idx[j]];
        out.theta[j] = th[idx[j]];
    }
    for (int j = 0; j < ncol; ++j)
        for (int i = 0; i < nb; ++i) Z[(size_t)i * ncol + j] = zq[(size_t)i * nb + idx[j]];
    NDQ_HIP(hipMemcpyAsync(c.Ydev, Z.data(), sizeof(cd) * Z.size(), hipMemcpyHostToDevice, c.st));
    char* Xr = c.UU;
    char* Wr = c.QU;
    if (rotate_block) {
        if ((rc = rotate(g, X, nb, c.Ydev, nb, XS, c.st))) return rc;
        if ((rc = rotate(g, W, nb, c.Ydev, nb, WS, c.st))) return rc;
        std::swap(X, XS);
        std::swap(W, WS);
        Xr = X;
        Wr = W;
    } else {
        if ((rc = rotate(g, X, nb, c.Ydev, nsel, c.UU, c.st))) return rc;
        if ((rc = rotate(g, W, nb, c.Ydev, nsel, c.QU, c.st))) return rc;
    }
    out.rho.assign(nsel, 0.0);
    for (int k = 0; k < nsel; ++k) {
        const ndq_spinor qu = c.vec(Wr, k);
        const ndq_spinor uk = c.vec(Xr, k);
        const ndq_spinor* v[2] = {&qu, &uk};
        const Coef cf[2] = {Coef{1.0, nullptr}, Coef{-out.nu[k], nullptr}};
        if ((rc = lincomb(g, NDQ_F64, &c.X0, 2, v, cf, nullptr, nullptr, c.st))) return rc;
        double r2;
        if ((rc = c.norm2(&c.X0, &r2))) return rc;
        out.rho[k] = sqrt(r2);
    }
    {
        const ndq_spinor qu = c.vec(Wr, nsel - 1);
        const ndq_spinor uk = c.vec(Xr, nsel - 1);
        if ((rc = c.qapply(&qu, &c.X1, 1.0))) return rc;
        const ndq_spinor* v[2] = {&c.X1, &uk};
        const Coef cf[2] = {Coef{1.0, nullptr}, Coef{-out.theta[nsel - 1], nullptr}};
        if ((rc = lincomb(g, NDQ_F64, &c.X0, 2, v, cf, nullptr, nullptr, c.st))) return rc;
        double r2;
        if ((rc = c.norm2(&c.X0, &r2))) return rc;
        out.guard_res = sqrt(r2);
    }
    if (rotate_block && Xr != c.UU) {
        NDQ_HIP(hipMemcpyAsync(c.UU, Xr, (size_t)c.vb * nsel, hipMemcpyDeviceToDevice, c.st));
    }
    return NDQ_OK;
}

// Orthonormalise the block X[0..nb-1] in place (classical Gram-Schmidt, twice).
int orthonormalise(LmCtx& c, char* X, int nb) {
    int rc;
    std::vector<cd> h;
    for (int j = 0; j < nb; ++j) {
        const ndq_spinor xj = c.vec(X, j);
        for (int pass = 0; pass < 2 && j > 0; ++pass) {
            if ((rc = c.dots_to_host(X, j, &xj, h))) return rc;
            if ((rc = c.subtract(X, j, h, &xj))) return rc;
        }
        double n2;
        if ((rc = c.norm2(&xj, &n2))) return rc;
        if (!(n2 > 0) || !isfinite(n2)) return fail(NDQ_ENAN, "low modes: block lost rank or overflowed");
        if ((rc = c.copy(&xj, &xj, 1.0 / sqrt(n2)))) return rc;
    }
    return NDQ_OK;
}

// Minimise the Ritz functional mu(x) = <x, A x> / |x|^2, A = Q^2, over x
// orthogonal to the k orthonormal vectors at `base` (Sec. 2.3): conjugate
// gradients on the unit sphere, each step minimising mu exactly in the plane
// of x and the search direction; g = (A x - mu x) with the lower vectors
// removed, next direction g + (|g_new|^2 / |g|^2) p.  Stops when |g| <= tol
// (times sqrt(mu) if tol_times_sqrt_mu).  x is vector k of `base` (start on
// entry, minimiser on exit); scratch: 5 vectors at `scr`.
int ritz_minimise(LmCtx& c, char* base, int k, char* scr, double tol, bool tol_times_sqrt_mu, int max_iter, int* iters,
                  double* mu_out, double* gnorm_out) {
    int rc;
    const ndq_geom* g = c.g;
    const ndq_spinor x = c.vec(base, k);
    const ndq_spinor y = c.vec(scr, 0), gr = c.vec(scr, 1), p = c.vec(scr, 2), pp = c.vec(scr, 3), z = c.vec(scr, 4);
    std::vector<cd> h;
    auto proj = [&](const ndq_spinor* v) -> int {
        if (k == 0) return NDQ_OK;
        int e = c.dots_to_host(base, k, v, h);
        if (!e) e = c.subtract(base, k, h, v);
        return e;
    };
    auto dot1 = [&](const ndq_spinor* a, const ndq_spinor* b, cd* out) -> int {
        std::vector<cd> d1;
        int e = c.dots_to_host(static_cast<char*>(a->data), 1, b, d1);
        if (!e) *out = d1[0];
        return e;
    };
    auto comb = [&](const ndq_spinor* dst, double ca, const ndq_spinor* a, double cb, const ndq_spinor* b) -> int {
        const ndq_spinor* v[2] = {a, b};
        const Coef cf[2] = {Coef{ca, nullptr}, Coef{cb, nullptr}};
        return lincomb(g, NDQ_F64, dst, b ? 2 : 1, v, cf, nullptr, nullptr, c.st);
    };
    if ((rc = proj(&x))) return rc;
    double n2;
    if ((rc = c.norm2(&x, &n2))) return rc;
    if (!(n2 > 0) || !isfinite(n2)) return fail(NDQ_ENAN, "low modes (Ritz): start vector lost");
    if ((rc = c.copy(&x, &x, 1.0 / sqrt(n2)))) return rc;
    if ((rc = apply_A(c, &x, &y))) return rc;
    cd t;
    if ((rc = dot1(&x, &y, &t))) return rc;
    double mu = t.real();
    if ((rc = comb(&gr, 1.0, &y, -mu, &x))) return rc;
    if ((rc = proj(&gr))) return rc;
    double g2;
    if ((rc = c.norm2(&gr, &g2))) return rc;
    if ((rc = c.copy(&p, &gr))) return rc;
    int it = 0;
    auto limit = [&]() { return tol_times_sqrt_mu ? tol * sqrt(std::max(mu, 0.0)) : tol; };
    while (sqrt(g2) > limit() && it < max_iter) {
        // pp = p - <x, p> x, ph = pp / |pp|
        if ((rc = dot1(&x, &p, &t))) return rc;
        {
            // complex coefficient: pp = p - t x as a rank-1 update
            const std::vector<cd> hh(1, t);
            if ((rc = c.copy(&pp, &p))) return rc;
            if ((rc = c.subtract(static_cast<char*>(x.data), 1, hh, &pp))) return rc;
        }
        double pn2;
        if ((rc = c.norm2(&pp, &pn2))) return rc;
        if (!(pn2 > 0)) break;   // direction parallel to x: converged as far as it goes
        const double pinv = 1.0 / sqrt(pn2);
        if ((rc = c.copy(&z, &pp, pinv))) return rc;       // z <- ph (temporarily)
        if ((rc = apply_A(c, &z, &c.X1))) return rc;       // X1 <- A ph
        cd bz, cz;
        if ((rc = dot1(&x, &c.X1, &bz))) return rc;
        if ((rc = dot1(&z, &c.X1, &cz))) return rc;
        const double a = mu, b = bz.real(), cc = cz.real();
        const double th = 0.5 * atan2(-b, 0.5 * (cc - a));
        const double cs = cos(th), sn = sin(th);
        if ((rc = comb(&x, cs, &x, sn, &z))) return rc;      // x <- cs x + sn ph
        if ((rc = comb(&y, cs, &y, sn, &c.X1))) return rc;   // y <- cs y + sn A ph
        if ((rc = proj(&x))) return rc;
        if ((rc = c.norm2(&x, &n2))) return rc;
        const double ninv = 1.0 / sqrt(n2);
        if ((rc = c.copy(&x, &x, ninv))) return rc;
        if ((rc = c.copy(&y, &y, ninv))) return rc;
        if ((rc = dot1(&x, &y, &t))) return rc;
        mu = t.real();
        if ((rc = comb(&gr, 1.0, &y, -mu, &x))) return rc;
        if ((rc = proj(&gr))) return rc;
        double g2n;
        if ((rc = c.norm2(&gr, &g2n))) return rc;
        if (!isfinite(g2n)) return fail(NDQ_ENAN, "low modes (Ritz): NaN in the minimisation");
        if ((rc = comb(&p, 1.0, &gr, g2n / g2, &pp))) return rc;
        g2 = g2n;
        ++it;
        // every 50 steps recompute A x (the update of y accumulates rounding)
        if (it % 50 == 0) {
            if ((rc = apply_A(c, &x, &y))) return rc;
            if ((rc = dot1(&x, &y, &t))) return rc;
            mu = t.real();
        }
    }
    *iters = it;
    *mu_out = mu;
    *gnorm_out = sqrt(g2);
    return NDQ_OK;
}

// Degree of the filter T_d on [a, b]: large enough to gain a factor ~2e3 at the
// guard eigenvalue per application, but with T_d(x(0)) <= 1e10 (A = Q^2 >= 0, so
// no eigenvalue is amplified more): a larger contrast than ~1/eps would leave the
// weakly amplified block vectors as rounding noise after orthogonalisation.
int filter_degree(double a, double b, double lam_guard) {
    const double x = 1.0 + 2.0 * (a - lam_guard) / (b - a);
    const double grow = x > 1.0 ? acosh(x) : 0.0;
    int d = grow > 0 ? (int)ceil(log(2e3) / grow) : 400;
    const double x0 = 1.0 + 2.0 * a / (b - a);
    const int dmax = (int)floor(log(2e10) / acosh(x0));
    d = std::min(d, dmax);
    d = std::min(400, std::max(4, d));
    return d + (d & 1);
}

}  // namespace
}  // namespace ndq

using namespace ndq;

extern "C" {

size_t ndq_lowmodes_workspace_bytes(const ndq_geom* g, const ndq_lowmode_params* p) {
    if (!g || !p || p->nev < 1) return 0;
    const size_t vb = (size_t)spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL);
    const int nkeep = p->nev + std::max(p->nextra, 1);
    const int m = p->method == NDQ_LM_LANCZOS ? p->basis : nkeep;
    if (m < 2) return 0;
    Arena ar{nullptr, 0};
    ar.take(vb * std::max(m + 1, 5));       // VA
    ar.take(vb * std::max(m + 1, 5));       // VB (Ritz: 5 work vectors)
    ar.take(vb * nkeep);            // W
    ar.take(vb * nkeep);            // WS
    ar.take(vb * (p->nev + 1));     // QU
    ar.take(vb * (p->nev + 1));     // UU
    if (p->method == NDQ_LM_SUBSPACE) ar.take(vb * nkeep);   // SB
    if (p->method == NDQ_LM_SUBSPACE && p->U_lo) {
        const size_t vbl = (size_t)spinor_rhs_bytes(g, NDQ_F32, NDQ_FULL);
        for (int i = 0; i < 3; ++i) ar.take(vbl * nkeep);    // XL, YL, SL
    }
    for (int i = 0; i < 3; ++i) ar.take(vb);
    ar.take(partials_capacity(g, 2 * NDQ_MAX_MODES));
    ar.take(2 * NDQ_MAX_MODES * sizeof(double));
    ar.take((size_t)2 * (m + 1) * (m + 1) * sizeof(double));
    ar.take(2 * NDQ_MAX_MODES * sizeof(double));
    ar.take(64 * sizeof(double));
    ar.take(gram_partials_bytes(g, nkeep, nkeep));
    ar.take(2 * 64 * 64 * sizeof(double));
    return ar.used + 256;
}

int ndq_lowmodes_compute(const ndq_geom* g, const ndq_gauge* U, double m, double lam_max, const ndq_lowmode_params* p,
                         const ndq_spinor* start, void* d_modes, double* nu, double* rho, ndq_lowmode_info* info,
                         void* ws, size_t ws_bytes, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!g || !p || !d_modes || !nu || !rho) return fail(NDQ_EINVAL, "ndq_lowmodes_compute: NULL argument");
    int rc = check_gauge(U);
    if (!rc) rc = check_spinor(g, start, NDQ_FULL, "ndq_lowmodes_compute start");
    if (rc) return rc;
    if (U->prec != NDQ_F64 || start->prec != NDQ_F64) return fail(NDQ_EPREC, "low modes: FP64 links and start vector");
    const bool lanczos = p->method == NDQ_LM_LANCZOS;
    const bool ritz = p->method == NDQ_LM_RITZ;
    if (p->method != NDQ_LM_SUBSPACE && !lanczos && !ritz)
        return fail(NDQ_EINVAL, "low modes: unknown method %d", p->method);
    if (p->nev_min < 0 || p->nev_min > p->nev) return fail(NDQ_EINVAL, "low modes: nev_min must be in [0, nev]");
    if (p->U_lo) {
        if (p->method != NDQ_LM_SUBSPACE) return fail(NDQ_EINVAL, "low modes: U_lo needs the subspace method");
        if ((rc = check_gauge(p->U_lo))) return rc;
        if (p->U_lo->prec != NDQ_F32) return fail(NDQ_EPREC, "low modes: U_lo must hold F32 links");
    }
    const int nev = p->nev, nkeep = nev + std::max(p->nextra, 1);
    const int mb = lanczos ? p->basis : nkeep;
    if (nev < 1 || nkeep > NDQ_MAX_MODES || (lanczos && (mb > NDQ_MAX_MODES - 1 || mb < nkeep + 2)))
        return fail(NDQ_EINVAL, "low modes: need 1 <= nev, nev + nextra <= %d (Lanczos: nev + nextra + 2 <= basis <= %d)",
                    NDQ_MAX_MODES, NDQ_MAX_MODES - 1);
    if (!(lam_max > 0)) return fail(NDQ_EINVAL, "low modes: lam_max must be positive");
    LmCtx c;
    c.g = g;
    c.U = U;
    c.m = m;
    c.st = as_stream(stream);
    c.vb = spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL);
    Arena ar{static_cast<char*>(ws), ws_bytes};
    c.VA = static_cast<char*>(ar.take(c.vb * std::max(mb + 1, 5)));
    c.VB = static_cast<char*>(ar.take(c.vb * std::max(mb + 1, 5)));
    c.W = static_cast<char*>(ar.take(c.vb * nkeep));
    char* WS = static_cast<char*>(ar.take(c.vb * nkeep));
    c.QU = static_cast<char*>(ar.take(c.vb * (nev + 1)));
    c.UU = static_cast<char*>(ar.take(c.vb * (nev + 1)));
    if (p->method == NDQ_LM_SUBSPACE) c.SB = static_cast<char*>(ar.take(c.vb * nkeep));
    if (p->method == NDQ_LM_SUBSPACE && p->U_lo) {
        c.Ulo = p->U_lo;
        c.vbl = spinor_rhs_bytes(g, NDQ_F32, NDQ_FULL);
        c.XL = static_cast<char*>(ar.take(c.vbl * nkeep));
        c.YL = static_cast<char*>(ar.take(c.vbl * nkeep));
        c.SL = static_cast<char*>(ar.take(c.vbl * nkeep));
    }
    c.X0 = ws_spinor(ar, g, NDQ_F64);
    c.X1 = ws_spinor(ar, g, NDQ_F64);
    c.S = ws_spinor(ar, g, NDQ_F64);
    c.partials = static_cast<double*>(ar.take(partials_capacity(g, 2 * NDQ_MAX_MODES)));
    c.dots = static_cast<double*>(ar.take(2 * NDQ_MAX_MODES * sizeof(double)));
    c.Ydev = static_cast<double*>(ar.take((size_t)2 * (mb + 1) * (mb + 1) * sizeof(double)));
    c.coef = static_cast<double*>(ar.take(2 * NDQ_MAX_MODES * sizeof(double)));
    c.scal = static_cast<double*>(ar.take(64 * sizeof(double)));
    c.gpart = static_cast<double*>(ar.take(gram_partials_bytes(g, nkeep, nkeep)));
    c.gout = static_cast<double*>(ar.take(2 * 64 * 64 * sizeof(double)));
    if (ar.overflow) return fail(NDQ_ENOMEM, "low modes: workspace too small (need %zu bytes)", ar.used);
    const double b = lam_max * lam_max;
    const double tol = p->tol > 0 ? p->tol : 1e-10;
    const double guard_tol = std::max(tol, 1e-6);
    const int max_restarts = p->max_restarts > 0 ? p->max_restarts : (lanczos ? 100 : ritz ? 5000 : 200);
    const int nsel = nev + 1;

    double s2;
    if ((rc = c.norm2(start, &s2))) return rc;
    if (!(s2 > 0) || !isfinite(s2)) return fail(NDQ_EINVAL, "low modes: zero or non-finite start vector");

    double a = p->cheb_lo;
    int d = p->cheb_degree;
    int restarts = 0, restarts_lo = 0;
    bool converged = false;
    RRResult rr;
    char* X = c.VA;
    char* XS = c.VB;
    char* W = c.W;

    if (ritz) {
        // ---- Ritz functional of Q^2 (the paper's method) with the acceleration
        // of Kalkreuter and Simma: sweeps of conjugate-gradient minimisation over
        // a block of nev + nextra vectors (vector i kept orthogonal to vectors
        // 0..i-1, at most `inner` steps each), then the Rayleigh-Ritz step of Q in
        // their span, which rotates the block onto Ritz vectors and decouples close
        // modes.  The wanted nev and the guard must converge; the rest only help.
        for (int i = 0; i < nkeep; ++i) {
            const ndq_spinor xi = c.vec(X, i);
            if ((rc = phase_copy(g, start, &xi, i, c.st))) return rc;
        }
        if ((rc = orthonormalise(c, X, nkeep))) return rc;
        const int inner = 40;
        const int max_sweeps = std::max(1, max_restarts / inner);
        for (int sweep = 0; sweep < max_sweeps; ++sweep) {
            for (int i = 0; i < nkeep; ++i) {
                // |(A - mu) x| ~ |lambda_j + nu| |(Q - nu) x| near an eigenvector: aim below the
                // target; the Rayleigh-Ritz residues decide convergence
                int iters = 0;
                double mu = 0.0, gn = 0.0;
                if (i < nev) rc = ritz_minimise(c, X, i, XS, 0.1 * tol * lam_max, true, inner, &iters, &mu, &gn);
                else rc = ritz_minimise(c, X, i, XS, 0.5 * guard_tol * b, false, inner, &iters, &mu, &gn);
                if (rc) return rc;
                restarts += iters;
            }
            if ((rc = rayleigh_ritz_q(c, X, W, XS, WS, nkeep, nsel, true, rr))) return rc;
            double max_rho = 0.0;
            for (int k = 0; k < nev; ++k) max_rho = std::max(max_rho, rr.rho[k]);
            if (max_rho <= tol * lam_max && rr.guard_res <= guard_tol * b) {
                converged = true;
                break;
            }
        }
        a = 0.0;
        d = 0;
    } else if (!lanczos) {
        // ---- Chebyshev-filtered subspace iteration on a block of nkeep vectors
        for (int i = 0; i < nkeep; ++i) {
            const ndq_spinor xi = c.vec(X, i);
            if ((rc = phase_copy(g, start, &xi, i, c.st))) return rc;
        }
        if ((rc = orthonormalise(c, X, nkeep))) return rc;
        // initial cutoff: the largest Rayleigh quotient |Q x|^2 of the start block
        if (!(a > 0)) {
            a = 0.0;
            for (int i = 0; i < nkeep; ++i) {
                const ndq_spinor xi = c.vec(X, i), wi = c.vec(W, i);
                if ((rc = c.qapply(&xi, &wi, 1.0))) return rc;
                double q2;
                if ((rc = c.norm2(&wi, &q2))) return rc;
                a = std::max(a, q2);
            }
            a = std::min(a, 0.5 * b);
        }
        const bool fixed_d = d > 0;
        if (!fixed_d) d = filter_degree(a, b, 0.5 * a);
        // F32 filter while the residues are far above what FP32 resolves
        bool lo = c.Ulo != nullptr;
        const double lo_until = (p->lo_until > 0 ? p->lo_until : 1e-5) * lam_max;
        double best_lo = HUGE_VAL;
        int stall = 0;
        for (;;) {
            if (lo) rc = apply_filter_block_lo(c, X, XS, nkeep, a, b, d);
            else rc = apply_filter_block(c, X, XS, c.SB, NDQ_F64, nkeep, a, b, d);
            if (rc) return rc;
            restarts_lo += lo ? 1 : 0;
            std::swap(X, XS);
            if ((rc = orthonormalise(c, X, nkeep))) return rc;
            if ((rc = rayleigh_ritz_q(c, X, W, XS, WS, nkeep, nsel, true, rr))) return rc;
            ++restarts;
            double max_rho = 0.0;
            for (int k = 0; k < nev; ++k) max_rho = std::max(max_rho, rr.rho[k]);
            if (max_rho <= tol * lam_max && rr.guard_res <= guard_tol * b) {
                converged = true;
                break;
            }
            if (lo) {
                // FP64 from here once the residues are small, or after three F32
                // restarts without halving the best residue so far
                if (max_rho < 0.5 * best_lo) {
                    best_lo = max_rho;
                    stall = 0;
                } else {
                    ++stall;
                }
                if (max_rho <= lo_until || stall >= 3) lo = false;
            }
            if (restarts >= max_restarts) break;
            // sharpen the filter: cutoff at the block's largest Rayleigh quotient of A
            a = std::min(std::max(rr.theta[nkeep - 1], 1e-12), 0.9 * b);
            if (!fixed_d) d = filter_degree(a, b, rr.theta[nev]);
        }
    } else {
        // ---- thick-restart Lanczos on the filter
        {
            const ndq_spinor v0 = c.vec(c.VA, 0);
            if ((rc = c.copy(&v0, start, 1.0 / sqrt(s2)))) return rc;
        }
        if (!(a > 0) || d <= 0) {
            const int m0 = mb;
            std::vector<cd> T((size_t)m0 * m0, 0.0);
            if ((rc = lanczos_steps(c, c.VA, 0, m0, T, 0, 0, 0, 0))) return rc;
            std::vector<double> th;
            std::vector<cd> z;
            eig_T(T, m0, th, z);
            if (!(a > 0)) a = th[std::min(nkeep, m0 - 1)];
            if (d <= 0) d = filter_degree(a, b, th[nev - 1]);
            const ndq_spinor v0 = c.vec(c.VA, 0);
            if ((rc = c.copy(&v0, start, 1.0 / sqrt(s2)))) return rc;
        }
        if (!(a > 0 && a < b)) return fail(NDQ_EINVAL, "low modes: filter cutoff %g outside (0, lam_max^2)", a);
        std::vector<cd> T((size_t)mb * mb, 0.0);
        int j0 = 0;
        for (;;) {
            if ((rc = lanczos_steps(c, c.VA, j0, mb, T, 1, a, b, d))) return rc;
            std::vector<double> th;
            std::vector<cd> z;
            eig_T(T, mb, th, z);
            std::vector<cd> Y((size_t)mb * nkeep);
            std::vector<double> thk(nkeep);
            for (int j = 0; j < nkeep; ++j) {
                const int col = mb - 1 - j;
                thk[j] = th[col];
                for (int i = 0; i < mb; ++i) Y[(size_t)i * nkeep + j] = z[(size_t)i * mb + col];
            }
            NDQ_HIP(hipMemcpyAsync(c.Ydev, Y.data(), sizeof(cd) * Y.size(), hipMemcpyHostToDevice, c.st));
            if ((rc = rotate(g, c.VA, mb, c.Ydev, nkeep, c.VB, c.st))) return rc;
            {
                const ndq_spinor r = c.vec(c.VA, mb), dst = c.vec(c.VB, nkeep);
                if ((rc = c.copy(&dst, &r))) return rc;
            }
            std::swap(c.VA, c.VB);
            ++restarts;
            char* Xl = c.VA;
            char* Wl = c.W;
            char* dummy1 = nullptr;
            char* dummy2 = nullptr;
            if ((rc = rayleigh_ritz_q(c, Xl, Wl, dummy1, dummy2, nkeep, nsel, false, rr))) return rc;
            double max_rho = 0.0;
            for (int k = 0; k < nev; ++k) max_rho = std::max(max_rho, rr.rho[k]);
            if (max_rho <= tol * lam_max && rr.guard_res <= guard_tol * b) {
                converged = true;
                break;
            }
            if (restarts >= max_restarts) break;
            std::fill(T.begin(), T.end(), cd(0.0, 0.0));
            for (int j = 0; j < nkeep; ++j) T[(size_t)j * mb + j] = thk[j];
            j0 = nkeep;
        }
    }
    // results: the first nev Ritz pairs (in theta order), guard pair -> lam_next
    NDQ_HIP(hipMemcpyAsync(d_modes, c.UU, (size_t)c.vb * nev, hipMemcpyDeviceToDevice, c.st));
    NDQ_HIP(hipStreamSynchronize(c.st));
    double max_rho = 0.0;
    for (int k = 0; k < nev; ++k) {
        nu[k] = rr.nu[k];
        rho[k] = rr.rho[k];
        max_rho = std::max(max_rho, rr.rho[k]);
    }
    // guard: A has an eigenvalue in [theta - r, theta + r] (r = |A u - theta u|),
    // so |Q| has one at or above sqrt(theta - r) = lam_next - rho_next
    double lam_next = sqrt(std::max(rr.theta[nev], 0.0));
    double rho_next = lam_next - sqrt(std::max(rr.theta[nev] - rr.guard_res, 0.0));
    // dynamic number of projected modes: the largest relative gap
    // |nu_(l+1)| / |nu_l| for l in [nev_min, nev] (|nu_(nev+1)| = lam_next)
    int l_used = nev;
    if (p->nev_min >= 1 && p->nev_min < nev) {
        double best = -1.0;
        for (int l = p->nev_min; l <= nev; ++l) {
            const double next = l < nev ? fabs(nu[l]) : lam_next;
            const double ratio = next / std::max(fabs(nu[l - 1]), 1e-300);
            if (ratio > best) {
                best = ratio;
                l_used = l;
            }
        }
        if (l_used < nev) {
            lam_next = fabs(nu[l_used]);
            rho_next = rho[l_used];
        }
    }
    if (info) {
        memset(info, 0, sizeof(*info));
        info->lam_next = lam_next;
        info->nev_used = l_used;
        // Eq. 9 with d_k = min(lam_lo - |nu_k|, |nu_k| + min over opposite-sign |nu_j|),
        // lam_lo = lam_next - rho_next the certified lower end of the rest of |spectrum|,
        // so that kappa and the Eq. 10 bounds err on the safe side
        const double lam_lo = lam_next - rho_next;
        double kp2 = 0.0, km2 = 0.0;
        for (int k = 0; k < l_used; ++k) {
            double dk = lam_lo - fabs(nu[k]);
            for (int j = 0; j < l_used; ++j)
                if ((nu[j] > 0) != (nu[k] > 0)) dk = std::min(dk, fabs(nu[k]) + fabs(nu[j]));
            const double q = dk > 0 ? rho[k] / dk : INFINITY;
            (nu[k] > 0 ? kp2 : km2) += q * q;
        }
        info->kappa_plus = sqrt(kp2);
        info->kappa_minus = sqrt(km2);
        auto bound = [](double k) {
            const double q = k * (1.0 + 2.0 * k);
            const double den = 1.0 - 2.0 * q;
            return den > 0 ? q / den : INFINITY;
        };
        info->bound_plus = bound(info->kappa_plus);
        info->bound_minus = bound(info->kappa_minus);
        info->cheb_lo = a;
        info->cheb_degree = d;
        info->restarts = restarts;
        info->restarts_lo = restarts_lo;
        info->q_applies = c.qcount;
        info->max_rho = max_rho;
        info->rho_next = rho_next;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!converged)
        return fail(NDQ_ENOCONV, "low modes: max rho %.3e (guard residue of Q^2 %.3e) > %.3e after %d iterations",
                    max_rho, rr.guard_res, tol * lam_max, restarts);
    return NDQ_OK;
}

}  // extern "C"
