// Solution of D_N^m x = b (Eq. 4 with the massive form of Eq. 12).
//
// Outer loop (FP64 defect correction): r = b - D x with the FP64 operator;
// stop once |r| <= tol |b|; otherwise solve D e = r / |r| approximately in the
// inner precision and update x += |r| e.  Inner solver: CG on the normal
// equations D^H D e = D^H r (CGNE) with D^H = gamma5 D gamma5, which holds
// because sign(Q) is Hermitian (the solve applies the projection of Eq. 11 in
// its sandwich form, Hermitian also for inexact low modes).  With inner precision F64 and an inner
// tolerance at the target this is the plain FP64 solve (normally one outer
// step plus the final true-residual check); with F32 (or F16 storage) the
// inner solves run in FP32 arithmetic on cheaper fields and approximant, and
// the FP64 outer steps restore the full accuracy.
//
// Alternative inner solver (sectors = 1): D = alpha + beta gamma5 eps, so D^H D
// commutes with gamma5 and on the chirality-s subspace equals
//     H_s = (alpha - beta)^2 + 2 alpha beta (1 + s P_s eps P_s)
// (with eps^2 = 1).  Then e = D^{-1} r = D^H (D^H D)^{-1} r =
// D^H (H_+^{-1} P_+ r + H_-^{-1} P_- r): one CG per chirality sector with one
// sign apply per iteration in the inner precision, and D^H applied with the
// FP64 operator.  A chiral source (a spin-colour point source in the chiral
// basis) needs only its own sector: half the sign applies of CGNE per
// iteration.  The normal equations square the condition number, so the inner
// operator's error reaches y amplified by ~1/mq^2 (CGNE: ~1/mq); mixed-precision
// sector solves therefore gain less per outer step than CGNE.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>

#include "ndq_solver.h"

namespace ndq {
namespace {

struct DOp {
    const ndq_geom* g;
    const ndq_gauge* U;
    const ndq_overlap_params* p;
    int prec;
    hipStream_t st;
    Arena* ar;            // rewound to `mark` before every application
    size_t mark;
    ndq_stats* stats;
    ndq_spinor S;         // sign(Q) in
};

// d.S = sign(Q) in (the approximant of d.p, low modes exact)
int sign_apply(DOp& d, const ndq_spinor* in) {
    d.ar->used = d.mark;
    d.ar->overflow = false;
    ndq_stats s;
    memset(&s, 0, sizeof(s));
    d.S.nrhs = in->nrhs;   // S has room for the largest block
    int rc = apply_sign(d.g, d.U, d.p, in, &d.S, *d.ar, &s, d.st);
    d.stats->q_applies += s.q_applies;
    return rc;
}

// out = D_N^m in
int d_apply(DOp& d, const ndq_spinor* in, const ndq_spinor* out) {
    int rc = sign_apply(d, in);
    if (rc) return rc;
    const double inv_abar = -d.p->m;
    const ndq_spinor* v[2] = {in, &d.S};
    const Coef c[2] = {Coef{inv_abar + 0.5 * d.p->mq, nullptr}, Coef{inv_abar - 0.5 * d.p->mq, nullptr}};
    const int g5[2] = {0, 1};
    return lincomb(d.g, d.prec, out, 2, v, c, g5, nullptr, d.st);
}

struct Vecs {
    ndq_spinor e, s, z, p, q, t;
};

int host_norm2(const ndq_geom* g, const ndq_spinor* x, double* partials, double* dscal, double* out, hipStream_t st) {
    int rc = dot(g, x, nullptr, partials, dscal, st);
    if (rc) return rc;
    NDQ_HIP(hipMemcpyAsync(out, dscal, sizeof(double), hipMemcpyDeviceToHost, st));
    NDQ_HIP(hipStreamSynchronize(st));
    if (!isfinite(*out)) return fail(NDQ_ENAN, "solve: NaN or Inf in a norm");
    return NDQ_OK;
}

Coef hc(double v) { return Coef{v, nullptr}; }

// Coefficients of D = alpha + beta gamma5 eps: alpha = 1/abar + mq/2, beta = 1/abar - mq/2.
double d_alpha(const DOp& d) { return -d.p->m + 0.5 * d.p->mq; }
double d_beta(const DOp& d) { return -d.p->m - 0.5 * d.p->mq; }

// out = D^H y = alpha y + beta eps (gamma5 y) with the operator of d; tmp: work field.
int dh_apply(DOp& d, const ndq_spinor* y, const ndq_spinor* tmp, const ndq_spinor* out) {
    const ndq_spinor* src[2] = {y, nullptr};
    Coef cf[2] = {hc(1.0), hc(0.0)};
    const int g5[2] = {1, 0};
    int rc = lincomb(d.g, d.prec, tmp, 1, src, cf, g5, nullptr, d.st);
    if (!rc) rc = sign_apply(d, tmp);
    if (rc) return rc;
    src[1] = &d.S;
    cf[0] = hc(d_alpha(d));
    cf[1] = hc(d_beta(d));
    return lincomb(d.g, d.prec, out, 2, src, cf, nullptr, nullptr, d.st);
}

// CGNE for D e = rhs (all in d.prec); e starts at zero.  Returns iterations.
int cgne(DOp& d, const ndq_spinor* rhs, Vecs& v, double tol, int max_iter, double* partials, double* dscal,
         int* iters) {
    const ndq_geom* g = d.g;
    hipStream_t st = d.st;
    int rc;
    const ndq_spinor* src[2];
    Coef cf[2];
    int g5[2] = {1, 0};
    // e = 0, s = rhs
    if ((rc = lincomb(g, d.prec, &v.e, 0, nullptr, nullptr, nullptr, nullptr, st))) return rc;
    src[0] = rhs;
    cf[0] = hc(1.0);
    if ((rc = lincomb(g, d.prec, &v.s, 1, src, cf, nullptr, nullptr, st))) return rc;
    double r0;
    if ((rc = host_norm2(g, &v.s, partials, dscal, &r0, st))) return rc;
    // z = D^H s = alpha s + beta eps (gamma5 s): one gamma5 pass before the sign
    // and the combination after it (gamma5 D gamma5 would take one more pass)
    auto dh = [&](const ndq_spinor* in, const ndq_spinor* out) { return dh_apply(d, in, &v.t, out); };
    if ((rc = dh(&v.s, &v.z))) return rc;
    src[0] = &v.z;
    if ((rc = lincomb(g, d.prec, &v.p, 1, src, cf, nullptr, nullptr, st))) return rc;
    double zz;
    if ((rc = host_norm2(g, &v.z, partials, dscal, &zz, st))) return rc;
    int it = 0;
    double ss = r0;
    while (it < max_iter && ss > tol * tol * r0) {
        if ((rc = d_apply(d, &v.p, &v.q))) return rc;
        double qq;
        if ((rc = host_norm2(g, &v.q, partials, dscal, &qq, st))) return rc;
        if (qq == 0.0) break;
        const double alpha = zz / qq;
        // e += alpha p ; s -= alpha q
        src[0] = &v.e;
        src[1] = &v.p;
        cf[0] = hc(1.0);
        cf[1] = hc(alpha);
        g5[0] = g5[1] = 0;
        if ((rc = lincomb(g, d.prec, &v.e, 2, src, cf, g5, nullptr, st))) return rc;
        src[0] = &v.s;
        src[1] = &v.q;
        cf[1] = hc(-alpha);
        if ((rc = lincomb(g, d.prec, &v.s, 2, src, cf, g5, nullptr, st))) return rc;
        if ((rc = host_norm2(g, &v.s, partials, dscal, &ss, st))) return rc;
        ++it;
        if (ss <= tol * tol * r0) break;
        if ((rc = dh(&v.s, &v.z))) return rc;
        double zz_new;
        if ((rc = host_norm2(g, &v.z, partials, dscal, &zz_new, st))) return rc;
        const double beta = zz_new / zz;
        zz = zz_new;
        src[0] = &v.z;
        src[1] = &v.p;
        cf[0] = hc(1.0);
        cf[1] = hc(beta);
        if ((rc = lincomb(g, d.prec, &v.p, 2, src, cf, g5, nullptr, st))) return rc;
    }
    *iters = it;
    return NDQ_OK;
}

// out = H_s in = (alpha^2 + beta^2) in + 2 s alpha beta P_s eps in, for a chirality-s `in`
// (2 s alpha beta P_s S = s alpha beta S + alpha beta gamma5 S).
int h_apply(DOp& d, int s, const ndq_spinor* in, const ndq_spinor* out) {
    int rc = sign_apply(d, in);
    if (rc) return rc;
    const double a = d_alpha(d), b = d_beta(d);
    const ndq_spinor* v[3] = {in, &d.S, &d.S};
    const Coef c[3] = {hc(a * a + b * b), hc(s * a * b), hc(a * b)};
    const int g5[3] = {0, 0, 1};
    return lincomb(d.g, d.prec, out, 3, v, c, g5, nullptr, d.st);
}

int host_dot_re(const ndq_geom* g, const ndq_spinor* x, const ndq_spinor* y, double* partials, double* dscal,
                double* out, hipStream_t st) {
    int rc = dot(g, x, y, partials, dscal, st);
    if (rc) return rc;
    double z[2];
    NDQ_HIP(hipMemcpyAsync(z, dscal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    NDQ_HIP(hipStreamSynchronize(st));
    if (!isfinite(z[0])) return fail(NDQ_ENAN, "solve: NaN or Inf in a dot product");
    *out = z[0];
    return NDQ_OK;
}

// y = H_s^{-1} rhs by CG (rhs of chirality s; y starts at zero); r, p, w work vectors.
int sector_cg(DOp& d, int s, const ndq_spinor* rhs, const ndq_spinor* y, const ndq_spinor* r, const ndq_spinor* p,
              const ndq_spinor* w, double tol, int max_iter, double* partials, double* dscal, int* iters) {
    const ndq_geom* g = d.g;
    hipStream_t st = d.st;
    int rc;
    if ((rc = lincomb(g, d.prec, y, 0, nullptr, nullptr, nullptr, nullptr, st))) return rc;
    const ndq_spinor* src[2] = {rhs, nullptr};
    Coef cf[2] = {hc(1.0), hc(0.0)};
    if ((rc = lincomb(g, d.prec, r, 1, src, cf, nullptr, nullptr, st))) return rc;
    if ((rc = lincomb(g, d.prec, p, 1, src, cf, nullptr, nullptr, st))) return rc;
    double rr;
    if ((rc = host_norm2(g, r, partials, dscal, &rr, st))) return rc;
    const double r0 = rr;
    int it = 0;
    while (it < max_iter && rr > tol * tol * r0) {
        if ((rc = h_apply(d, s, p, w))) return rc;
        double pw;
        if ((rc = host_dot_re(g, p, w, partials, dscal, &pw, st))) return rc;
        if (!(pw > 0)) return fail(NDQ_ENAN, "solve: sector operator not positive (p^H H p = %g)", pw);
        const double alpha = rr / pw;
        src[0] = y;
        src[1] = p;
        cf[0] = hc(1.0);
        cf[1] = hc(alpha);
        if ((rc = lincomb(g, d.prec, y, 2, src, cf, nullptr, nullptr, st))) return rc;
        src[0] = r;
        src[1] = w;
        cf[1] = hc(-alpha);
        if ((rc = lincomb(g, d.prec, r, 2, src, cf, nullptr, nullptr, st))) return rc;
        double rr_new;
        if ((rc = host_norm2(g, r, partials, dscal, &rr_new, st))) return rc;
        ++it;
        if (rr_new <= tol * tol * r0) break;
        const double beta = rr_new / rr;
        rr = rr_new;
        src[0] = r;
        src[1] = p;
        cf[0] = hc(1.0);
        cf[1] = hc(beta);
        if ((rc = lincomb(g, d.prec, p, 2, src, cf, nullptr, nullptr, st))) return rc;
    }
    *iters = it;
    return NDQ_OK;
}

// y = (D^H D)^{-1} rhs = H_+^{-1} P_+ rhs + H_-^{-1} P_- rhs into v.t, by the
// two chirality sectors (|rhs| = 1 on entry); the caller forms e = D^H y.
// Each sector is solved to the absolute residual tol / sqrt(2), so that the
// two together meet tol; a sector whose part of rhs is already below that is
// skipped (a chiral source stays chiral: the residual b - D D^H y is chiral
// when y is, because D D^H = D^H D commutes with gamma5).
int sectors_solve(DOp& d, const ndq_spinor* rhs, Vecs& v, double tol, int max_iter, double* partials, double* dscal,
                  int* iters) {
    const ndq_geom* g = d.g;
    hipStream_t st = d.st;
    int rc;
    *iters = 0;
    if ((rc = lincomb(g, d.prec, &v.t, 0, nullptr, nullptr, nullptr, nullptr, st))) return rc;
    for (int s = 1; s >= -1; s -= 2) {
        const ndq_spinor* src[2] = {rhs, rhs};
        const Coef cf[2] = {hc(0.5), hc(0.5 * s)};
        const int g5[2] = {0, 1};
        if ((rc = lincomb(g, d.prec, &v.e, 2, src, cf, g5, nullptr, st))) return rc;   // P_s rhs
        double n2;
        if ((rc = host_norm2(g, &v.e, partials, dscal, &n2, st))) return rc;
        const double tol_abs = tol / sqrt(2.0);
        if (sqrt(n2) <= tol_abs) continue;
        int its = 0;
        if ((rc = sector_cg(d, s, &v.e, &v.z, &v.s, &v.p, &v.q, tol_abs / sqrt(n2), max_iter, partials, dscal, &its)))
            return rc;
        *iters += its;
        const ndq_spinor* acc[2] = {&v.t, &v.z};
        const Coef ca[2] = {hc(1.0), hc(1.0)};
        if ((rc = lincomb(g, d.prec, &v.t, 2, acc, ca, nullptr, nullptr, st))) return rc;
    }
    return NDQ_OK;
}

// Inner relative residual when the caller leaves it open: half the target in
// plain FP64; 1e-5 for F32 storage; for F16 storage (11-bit significands with
// a per-site scale) eight units of its rounding, 8 * 2^-11, about where the
// rounding of the stored vectors stops the inner CG from converging further.
double default_inner_tol(int lo, double tol) {
    if (lo == NDQ_F64) return 0.5 * tol;
    if (lo == NDQ_F16) return 8.0 * 0x1p-11;
    return 1e-5;
}

// |x_r|^2 of every field of a block, to the host (nr values).
int host_norms(const ndq_geom* g, const ndq_spinor* x, double* partials, double* dscal, double* out, hipStream_t st) {
    int rc = dot(g, x, nullptr, partials, dscal, st);
    if (rc) return rc;
    NDQ_HIP(hipMemcpyAsync(out, dscal, sizeof(double) * x->nrhs, hipMemcpyDeviceToHost, st));
    NDQ_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < x->nrhs; ++r)
        if (!isfinite(out[r])) return fail(NDQ_ENAN, "solve: NaN or Inf in the norm of right-hand side %d", r);
    return NDQ_OK;
}

// Field views of a block: the first n fields, and field k alone.
ndq_spinor first(const ndq_spinor& b, int n) {
    ndq_spinor o = b;
    o.nrhs = n;
    return o;
}

// dst field kd = c * src field ks (one field; c = 0 clears it).
int copy_field(const ndq_geom* g, int prec, const ndq_spinor* dst, int kd, const ndq_spinor* src, int ks, double c,
               hipStream_t st) {
    const ndq_spinor d1 = rhs_slice(g, dst, kd), s1 = rhs_slice(g, src, ks);
    const ndq_spinor* v[1] = {&s1};
    const Coef cf[1] = {hc(c)};
    return lincomb(g, prec, &d1, c == 0.0 ? 0 : 1, v, cf, nullptr, nullptr, st);
}

// CGNE for D e_r = rhs_r on every field r of a block at once: one D (or D^H)
// application of the block per step, so that each sign application is shared
// (links loaded once per stencil tile for all fields), and scalars per field.
// A field leaves the block once its residual is below tol |rhs_r|: its e is
// written to eout (at its index in rhs), and the fields still running are
// moved to the front, so every application of D works on those only.  Returns
// the number of block iterations.
int cgne_block(DOp& d, const ndq_spinor* rhs, Vecs& v, const ndq_spinor* eout, double tol, int max_iter,
               double* partials, double* dscal, int* iters) {
    const ndq_geom* g = d.g;
    hipStream_t st = d.st;
    const int prec = d.prec;
    int nb = rhs->nrhs;
    int rc;
    double r0[NDQ_MAX_BATCH], ss[NDQ_MAX_BATCH], zz[NDQ_MAX_BATCH], qq[NDQ_MAX_BATCH], zn[NDQ_MAX_BATCH];
    double cf[2 * NDQ_MAX_BATCH];
    int orig[NDQ_MAX_BATCH], done[NDQ_MAX_BATCH];
    for (int k = 0; k < nb; ++k) orig[k] = k;
    *iters = 0;
    // Write finished fields out and move the others to the front (vectors of
    // the listed kinds and the per-field scalars).
    auto compact = [&](bool move_p) -> int {
        int w = 0;
        for (int k = 0; k < nb; ++k) {
            if (done[k]) {
                int e2;
                if ((e2 = copy_field(g, prec, eout, orig[k], &v.e, k, 1.0, st))) return e2;
                continue;
            }
            if (w != k) {
                int e2;
                if ((e2 = copy_field(g, prec, &v.e, w, &v.e, k, 1.0, st))) return e2;
                if ((e2 = copy_field(g, prec, &v.s, w, &v.s, k, 1.0, st))) return e2;
                if (move_p && (e2 = copy_field(g, prec, &v.p, w, &v.p, k, 1.0, st))) return e2;
                orig[w] = orig[k];
                r0[w] = r0[k];
                zz[w] = zz[k];
                ss[w] = ss[k];
            }
            ++w;
        }
        nb = w;
        return NDQ_OK;
    };
    ndq_spinor e = first(v.e, nb), s = first(v.s, nb);
    if ((rc = lincomb(g, prec, &e, 0, nullptr, nullptr, nullptr, nullptr, st))) return rc;
    {
        const ndq_spinor* src[1] = {rhs};
        const Coef c1[1] = {hc(1.0)};
        if ((rc = lincomb(g, prec, &s, 1, src, c1, nullptr, nullptr, st))) return rc;
    }
    if ((rc = host_norms(g, &s, partials, dscal, r0, st))) return rc;
    for (int k = 0; k < nb; ++k) {
        done[k] = !(r0[k] > 0.0);
        zz[k] = ss[k] = 0.0;
    }
    if ((rc = compact(false))) return rc;
    if (nb == 0) return NDQ_OK;
    // z = D^H s, p = z
    {
        const ndq_spinor sb = first(v.s, nb), zb = first(v.z, nb), tb = first(v.t, nb), pb = first(v.p, nb);
        if ((rc = dh_apply(d, &sb, &tb, &zb))) return rc;
        const ndq_spinor* src[1] = {&zb};
        const Coef c1[1] = {hc(1.0)};
        if ((rc = lincomb(g, prec, &pb, 1, src, c1, nullptr, nullptr, st))) return rc;
        if ((rc = host_norms(g, &zb, partials, dscal, zz, st))) return rc;
    }
    int it = 0;
    while (it < max_iter && nb > 0) {
        const ndq_spinor eb = first(v.e, nb), sb = first(v.s, nb), pb = first(v.p, nb), qb = first(v.q, nb);
        if ((rc = d_apply(d, &pb, &qb))) return rc;
        if ((rc = host_norms(g, &qb, partials, dscal, qq, st))) return rc;
        // e += alpha p, s -= alpha q
        for (int k = 0; k < nb; ++k) {
            cf[k] = 1.0;
            cf[nb + k] = qq[k] > 0.0 ? zz[k] / qq[k] : 0.0;
        }
        {
            const ndq_spinor* src[2] = {&eb, &pb};
            if ((rc = lincomb_rhs(g, prec, &eb, 2, src, cf, nullptr, nullptr, st))) return rc;
            for (int k = 0; k < nb; ++k) cf[nb + k] = -cf[nb + k];
            const ndq_spinor* src2[2] = {&sb, &qb};
            if ((rc = lincomb_rhs(g, prec, &sb, 2, src2, cf, nullptr, nullptr, st))) return rc;
        }
        if ((rc = host_norms(g, &sb, partials, dscal, ss, st))) return rc;
        ++it;
        bool any = false;
        for (int k = 0; k < nb; ++k) {
            done[k] = ss[k] <= tol * tol * r0[k] || !(qq[k] > 0.0);
            any |= done[k] != 0;
        }
        if (any && (rc = compact(true))) return rc;
        if (nb == 0) break;
        // z = D^H s, p = z + beta p
        const ndq_spinor sc = first(v.s, nb), zc = first(v.z, nb), tc = first(v.t, nb), pc = first(v.p, nb);
        if ((rc = dh_apply(d, &sc, &tc, &zc))) return rc;
        if ((rc = host_norms(g, &zc, partials, dscal, zn, st))) return rc;
        for (int k = 0; k < nb; ++k) {
            cf[k] = 1.0;
            cf[nb + k] = zn[k] / zz[k];
            zz[k] = zn[k];
        }
        const ndq_spinor* src[2] = {&zc, &pc};
        if ((rc = lincomb_rhs(g, prec, &pc, 2, src, cf, nullptr, nullptr, st))) return rc;
    }
    // fields stopped by the iteration limit
    for (int k = 0; k < nb; ++k)
        if ((rc = copy_field(g, prec, eout, orig[k], &v.e, k, 1.0, st))) return rc;
    *iters = it;
    return NDQ_OK;
}

int check_solve(const ndq_geom* g, const ndq_gauge* U64, const ndq_gauge* Ulo, const ndq_overlap_params* p64,
                const ndq_overlap_params* plo, const ndq_solve_params* sp, const ndq_spinor* b, const ndq_spinor* x) {
    if (!g || !p64 || !sp) return fail(NDQ_EINVAL, "solve: NULL argument");
    int rc = check_gauge(U64);
    if (!rc) rc = check_spinor(g, b, NDQ_FULL, "solve b");
    if (!rc) rc = check_spinor(g, x, NDQ_FULL, "solve x");
    if (rc) return rc;
    if (U64->prec != NDQ_F64 || b->prec != NDQ_F64 || x->prec != NDQ_F64)
        return fail(NDQ_EPREC, "solve: b, x and the outer links are F64");
    if (b->nrhs != x->nrhs) return fail(NDQ_EINVAL, "solve: b and x must hold the same number of fields");
    if (b->nrhs > NDQ_MAX_BATCH) return fail(NDQ_EINVAL, "solve: at most %d right-hand sides per call", NDQ_MAX_BATCH);
    if (sp->inner_prec != NDQ_F64) {
        if (!Ulo || !plo) return fail(NDQ_EINVAL, "solve: mixed precision needs inner links and parameters");
        if ((rc = check_gauge(Ulo))) return rc;
        if (Ulo->prec == NDQ_F64) return fail(NDQ_EPREC, "solve: inner links must be F32 or F16");
    }
    if (!(sp->tol > 0)) return fail(NDQ_EINVAL, "solve: tol must be positive");
    if (sp->sectors != 0 && sp->sectors != 1) return fail(NDQ_EINVAL, "solve: sectors must be 0 or 1");
    return NDQ_OK;
}



int solve_single(const ndq_geom* g, const ndq_gauge* U64, const ndq_gauge* Ulo, const ndq_overlap_params* p64_in,
                 const ndq_overlap_params* plo_in, const ndq_solve_params* sp, const ndq_spinor* b, const ndq_spinor* x,
                 void* ws, size_t ws_bytes, ndq_stats* stats, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
    ndq_stats local;
    ndq_stats* stt = stats ? stats : &local;
    memset(stt, 0, sizeof(*stt));
    int rc;
    // CGNE takes D^H = gamma5 D gamma5, which needs a Hermitian sign(Q): the
    // operators of the solve use the sandwich form of Eq. 11
    const ndq_overlap_params h64 = hermitian_form(p64_in);
    const ndq_overlap_params hlo = plo_in ? hermitian_form(plo_in) : h64;
    const ndq_overlap_params* p64 = &h64;
    const ndq_overlap_params* plo = plo_in ? &hlo : nullptr;
    hipStream_t st = as_stream(stream);
    const int lo = sp->inner_prec;
    const ndq_gauge* Ui = lo == NDQ_F64 ? U64 : Ulo;
    const ndq_overlap_params* pi = lo == NDQ_F64 ? p64 : plo;
    Arena ar{static_cast<char*>(ws), ws_bytes};
    ndq_spinor r = ws_spinor(ar, g, NDQ_F64), t64 = ws_spinor(ar, g, NDQ_F64), S64 = ws_spinor(ar, g, NDQ_F64);
    ndq_spinor rlo = ws_spinor(ar, g, lo), Slo = ws_spinor(ar, g, lo);
    Vecs v{ws_spinor(ar, g, lo), ws_spinor(ar, g, lo), ws_spinor(ar, g, lo), ws_spinor(ar, g, lo),
           ws_spinor(ar, g, lo), ws_spinor(ar, g, lo)};
    double* partials = static_cast<double*>(ar.take(partials_capacity(g, 2)));
    double* dscal = static_cast<double*>(ar.take(64 * sizeof(double)));
    if (ar.overflow) return fail(NDQ_ENOMEM, "solve: workspace too small (need %zu bytes)", ar.used);
    const size_t mark = ar.used;
    DOp d64{g, U64, p64, NDQ_F64, st, &ar, mark, stt, S64};
    DOp dlo{g, Ui, pi, lo, st, &ar, mark, stt, Slo};

    double bb;
    if ((rc = host_norm2(g, b, partials, dscal, &bb, st))) return rc;
    if (bb == 0.0) {
        rc = lincomb(g, NDQ_F64, x, 0, nullptr, nullptr, nullptr, nullptr, st);
        stt->residual = 0.0;
        return rc;
    }
    const int max_outer = sp->max_outer > 0 ? sp->max_outer : 20;
    const int max_inner = sp->max_inner > 0 ? sp->max_inner : 100000;
    const double inner_tol = sp->inner_tol > 0 ? sp->inner_tol : default_inner_tol(lo, sp->tol);
    double rr = 0.0;
    for (int outer = 0;; ++outer) {
        // r = b - D x (FP64)
        if ((rc = d_apply(d64, x, &t64))) return rc;
        const ndq_spinor* src[2] = {b, &t64};
        const Coef cf[2] = {Coef{1.0, nullptr}, Coef{-1.0, nullptr}};
        if ((rc = lincomb(g, NDQ_F64, &r, 2, src, cf, nullptr, nullptr, st))) return rc;
        if ((rc = host_norm2(g, &r, partials, dscal, &rr, st))) return rc;
        stt->residual = sqrt(rr / bb);
        stt->outer = outer;
        if (stt->residual <= sp->tol) break;
        if (outer >= max_outer) {
            stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            return fail(NDQ_ENOCONV, "solve: residual %.3e after %d outer steps", stt->residual, outer);
        }
        // r_lo = r / |r|
        const double rn = sqrt(rr);
        const ndq_spinor* s1[1] = {&r};
        const Coef c1[1] = {Coef{1.0 / rn, nullptr}};
        if (lo == NDQ_F64) {
            if ((rc = lincomb(g, NDQ_F64, &rlo, 1, s1, c1, nullptr, nullptr, st))) return rc;
        } else {
            if ((rc = lincomb(g, NDQ_F64, &t64, 1, s1, c1, nullptr, nullptr, st))) return rc;
            if ((rc = convert(g, &rlo, &t64, st))) return rc;
        }
        int its = 0;
        const ndq_spinor* ex = &v.e;
        if (sp->sectors) {
            // y in the inner precision; e = D^H y with the FP64 operator, so that
            // the next residual stays in the sectors of y (the inner operator's
            // error would otherwise reach e amplified by |y| ~ |r| / mq^2)
            if ((rc = sectors_solve(dlo, &rlo, v, inner_tol, max_inner, partials, dscal, &its))) return rc;
            const ndq_spinor* y64 = &v.t;
            if (lo != NDQ_F64) {
                if ((rc = convert(g, &t64, &v.t, st))) return rc;
                y64 = &t64;
            }
            if ((rc = dh_apply(d64, y64, &r, &r))) return rc;
            ex = &r;
        } else {
            if ((rc = cgne(dlo, &rlo, v, inner_tol, max_inner, partials, dscal, &its))) return rc;
            if (lo != NDQ_F64) {
                if ((rc = convert(g, &t64, &v.e, st))) return rc;
                ex = &t64;
            }
        }
        stt->inner += its;
        // x += |r| e
        const ndq_spinor* s2[2] = {x, ex};
        const Coef c2[2] = {Coef{1.0, nullptr}, Coef{rn, nullptr}};
        if ((rc = lincomb(g, NDQ_F64, x, 2, s2, c2, nullptr, nullptr, st))) return rc;
    }
    stt->iterations = (int32_t)stt->inner;
    stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return NDQ_OK;
}


// Block solve: FP64 defect correction with one CGNE per field in the inner
// precision, all fields of the block sharing every D application.  The
// residual reported is the largest over the fields; `inner` counts block
// iterations.
int solve_block(const ndq_geom* g, const ndq_gauge* U64, const ndq_gauge* Ulo, const ndq_overlap_params* p64_in,
                const ndq_overlap_params* plo_in, const ndq_solve_params* sp, const ndq_spinor* b, const ndq_spinor* x,
                void* ws, size_t ws_bytes, ndq_stats* stt, hipStream_t st) {
    const ndq_overlap_params h64 = hermitian_form(p64_in);
    const ndq_overlap_params hlo = plo_in ? hermitian_form(plo_in) : h64;
    const ndq_overlap_params* p64 = &h64;
    const ndq_overlap_params* plo = plo_in ? &hlo : nullptr;
    const int lo = sp->inner_prec;
    const int nr = b->nrhs;
    const ndq_gauge* Ui = lo == NDQ_F64 ? U64 : Ulo;
    const ndq_overlap_params* pi = lo == NDQ_F64 ? p64 : plo;
    Arena ar{static_cast<char*>(ws), ws_bytes};
    ndq_spinor r = ws_block(ar, g, NDQ_F64, nr), t64 = ws_block(ar, g, NDQ_F64, nr), S64 = ws_block(ar, g, NDQ_F64, nr);
    ndq_spinor rlo = ws_block(ar, g, lo, nr), Slo = ws_block(ar, g, lo, nr), Eo = ws_block(ar, g, lo, nr);
    Vecs v{ws_block(ar, g, lo, nr), ws_block(ar, g, lo, nr), ws_block(ar, g, lo, nr), ws_block(ar, g, lo, nr),
           ws_block(ar, g, lo, nr), ws_block(ar, g, lo, nr)};
    double* partials = static_cast<double*>(ar.take(partials_capacity(g, 2 * nr)));
    double* dscal = static_cast<double*>(ar.take((64 + 2 * nr) * sizeof(double)));
    if (ar.overflow) return fail(NDQ_ENOMEM, "solve: workspace too small (need %zu bytes)", ar.used);
    const size_t mark = ar.used;
    DOp d64{g, U64, p64, NDQ_F64, st, &ar, mark, stt, S64};
    DOp dlo{g, Ui, pi, lo, st, &ar, mark, stt, Slo};
    int rc;
    double bb[NDQ_MAX_BATCH], rr[NDQ_MAX_BATCH], rn[NDQ_MAX_BATCH], cf[2 * NDQ_MAX_BATCH];
    int act[NDQ_MAX_BATCH];
    if ((rc = host_norms(g, b, partials, dscal, bb, st))) return rc;
    // a zero right-hand side has the solution zero
    bool any_zero = false;
    for (int j = 0; j < nr; ++j) {
        cf[j] = bb[j] == 0.0 ? 0.0 : 1.0;
        any_zero |= bb[j] == 0.0;
    }
    if (any_zero) {
        const ndq_spinor* s1[1] = {x};
        if ((rc = lincomb_rhs(g, NDQ_F64, x, 1, s1, cf, nullptr, nullptr, st))) return rc;
    }
    const int max_outer = sp->max_outer > 0 ? sp->max_outer : 20;
    const int max_inner = sp->max_inner > 0 ? sp->max_inner : 100000;
    const double inner_tol = sp->inner_tol > 0 ? sp->inner_tol : default_inner_tol(lo, sp->tol);
    for (int outer = 0;; ++outer) {
        // r = b - D x (FP64)
        if ((rc = d_apply(d64, x, &t64))) return rc;
        const ndq_spinor* src[2] = {b, &t64};
        const Coef c2[2] = {Coef{1.0, nullptr}, Coef{-1.0, nullptr}};
        if ((rc = lincomb(g, NDQ_F64, &r, 2, src, c2, nullptr, nullptr, st))) return rc;
        if ((rc = host_norms(g, &r, partials, dscal, rr, st))) return rc;
        int nact = 0;
        double worst = 0.0;
        for (int j = 0; j < nr; ++j) {
            const double res = bb[j] > 0.0 ? sqrt(rr[j] / bb[j]) : 0.0;
            worst = std::max(worst, res);
            act[j] = res > sp->tol;
            nact += act[j];
            rn[j] = sqrt(rr[j]);
        }
        stt->residual = worst;
        stt->outer = outer;
        if (!nact) break;
        if (outer >= max_outer)
            return fail(NDQ_ENOCONV, "solve: largest residual %.3e after %d outer steps", worst, outer);
        // the fields still above the target, r_lo = r / |r|, moved to the front
        int idx[NDQ_MAX_BATCH];
        int na = 0;
        for (int j = 0; j < nr; ++j)
            if (act[j]) idx[na++] = j;
        for (int k = 0; k < na; ++k)
            if ((rc = copy_field(g, NDQ_F64, &t64, k, &r, idx[k], 1.0 / rn[idx[k]], st))) return rc;
        const ndq_spinor rl = first(rlo, na), tl = first(t64, na), el = first(Eo, na);
        if (lo == NDQ_F64) {
            const ndq_spinor* s1[1] = {&tl};
            const Coef c1[1] = {Coef{1.0, nullptr}};
            if ((rc = lincomb(g, NDQ_F64, &rl, 1, s1, c1, nullptr, nullptr, st))) return rc;
        } else if ((rc = convert(g, &rl, &tl, st))) {
            return rc;
        }
        int its = 0;
        if ((rc = cgne_block(dlo, &rl, v, &el, inner_tol, max_inner, partials, dscal, &its))) return rc;
        stt->inner += its;
        const ndq_spinor* ex = &el;
        if (lo != NDQ_F64) {
            if ((rc = convert(g, &tl, &el, st))) return rc;
            ex = &tl;
        }
        // x += |r| e
        for (int k = 0; k < na; ++k) {
            const ndq_spinor xk = rhs_slice(g, x, idx[k]), ek = rhs_slice(g, ex, k);
            const ndq_spinor* s2[2] = {&xk, &ek};
            const Coef c2[2] = {Coef{1.0, nullptr}, Coef{rn[idx[k]], nullptr}};
            if ((rc = lincomb(g, NDQ_F64, &xk, 2, s2, c2, nullptr, nullptr, st))) return rc;
        }
    }
    return NDQ_OK;
}

}  // namespace
}  // namespace ndq

using namespace ndq;

extern "C" {

size_t ndq_solve_workspace_bytes_nrhs(const ndq_geom* g, const ndq_overlap_params* p64_in,
                                      const ndq_overlap_params* plo_in, const ndq_solve_params* sp, int nrhs) {
    if (!g || !p64_in || !p64_in->approx || !sp || nrhs < 1 || nrhs > NDQ_MAX_BATCH) return 0;
    const ndq_overlap_params h64 = hermitian_form(p64_in);
    const ndq_overlap_params hlo = plo_in ? hermitian_form(plo_in) : h64;
    const ndq_overlap_params* p64 = &h64;
    const ndq_overlap_params* plo = plo_in ? &hlo : nullptr;
    const int lo = sp->inner_prec;
    const ndq_overlap_params* pi = lo == NDQ_F64 ? p64 : plo;
    if (!pi || !pi->approx) return 0;
    // the chirality-sector solver runs the fields one after the other
    const int nr = sp->sectors ? 1 : nrhs;
    size_t b = 0;
    b += 3 * ((size_t)spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL) * nr + 256);   // r, t64, S64
    b += 9 * ((size_t)spinor_rhs_bytes(g, lo, NDQ_FULL) * nr + 256);        // r_lo, S_lo, e_out, e s z p q t
    b += partials_capacity(g, 2 * nr) + (64 + 2 * nr) * sizeof(double) + 1024;
    const size_t s64 = sign_workspace(g, p64, NDQ_F64, nr);
    const size_t slo = sign_workspace(g, pi, lo, nr);
    return b + std::max(s64, slo) + 4096;
}

size_t ndq_solve_workspace_bytes(const ndq_geom* g, const ndq_overlap_params* p64_in, const ndq_overlap_params* plo_in,
                                 const ndq_solve_params* sp) {
    return ndq_solve_workspace_bytes_nrhs(g, p64_in, plo_in, sp, 1);
}

int ndq_solve_DN(const ndq_geom* g, const ndq_gauge* U64, const ndq_gauge* Ulo, const ndq_overlap_params* p64_in,
                 const ndq_overlap_params* plo_in, const ndq_solve_params* sp, const ndq_spinor* b, const ndq_spinor* x,
                 void* ws, size_t ws_bytes, ndq_stats* stats, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
    ndq_stats local;
    ndq_stats* stt = stats ? stats : &local;
    memset(stt, 0, sizeof(*stt));
    int rc = check_solve(g, U64, Ulo, p64_in, plo_in, sp, b, x);
    if (rc) return rc;
    if (b->nrhs == 1) return solve_single(g, U64, Ulo, p64_in, plo_in, sp, b, x, ws, ws_bytes, stt, stream);
    if (sp->sectors) {
        // one field after the other, each with the whole workspace
        for (int r = 0; r < b->nrhs; ++r) {
            const ndq_spinor b1 = rhs_slice(g, b, r), x1 = rhs_slice(g, x, r);
            ndq_stats s1;
            rc = solve_single(g, U64, Ulo, p64_in, plo_in, sp, &b1, &x1, ws, ws_bytes, &s1, stream);
            stt->q_applies += s1.q_applies;
            stt->inner += s1.inner;
            stt->outer = std::max(stt->outer, s1.outer);
            stt->residual = std::max(stt->residual, s1.residual);
            if (rc) break;
        }
        stt->iterations = (int32_t)stt->inner;
        stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return rc;
    }
    rc = solve_block(g, U64, Ulo, p64_in, plo_in, sp, b, x, ws, ws_bytes, stt, as_stream(stream));
    stt->iterations = (int32_t)stt->inner;
    stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

}  // extern "C"
