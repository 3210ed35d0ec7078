// Solution of D_N^m x = b (Eq. 4 with the massive form of Eq. 12).
//
// Outer loop (FP64 defect correction): r = b - D x with the FP64 operator;
// stop once |r| <= tol |b|; otherwise solve D e = r / |r| approximately in the
// inner precision and update x += |r| e.  Inner solver: CG on the normal
// equations D^H D e = D^H r (CGNE) with D^H = gamma5 D gamma5, which holds
// because sign(Q) is Hermitian.  With inner precision F64 and an inner
// tolerance at the target this is the plain FP64 solve (normally one outer
// step plus the final true-residual check); with F32 (or F16 storage) the
// inner solves run in FP32 arithmetic on cheaper fields and approximant, and
// the FP64 outer steps restore the full accuracy.
#include <math.h>
#include <string.h>

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

// out = D_N^m in (gamma5 on the input and/or output when herm)
int d_apply(DOp& d, const ndq_spinor* in, const ndq_spinor* out) {
    d.ar->used = d.mark;
    d.ar->overflow = false;
    ndq_stats s;
    memset(&s, 0, sizeof(s));
    int rc = apply_sign(d.g, d.U, d.p, in, &d.S, *d.ar, &s, d.st);
    d.stats->q_applies += s.q_applies;
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
    // z = D^H s = g5 D g5 s
    auto dh = [&](const ndq_spinor* in, const ndq_spinor* out) {
        const ndq_spinor* s1[1] = {in};
        const Coef c1[1] = {hc(1.0)};
        const int g1[1] = {1};
        int r = lincomb(g, d.prec, &v.t, 1, s1, c1, g1, nullptr, st);
        if (!r) r = d_apply(d, &v.t, out);
        if (!r) r = lincomb(g, d.prec, out, 1, &out, c1, g1, nullptr, st);
        return r;
    };
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

int check_solve(const ndq_geom* g, const ndq_gauge* U64, const ndq_gauge* Ulo, const ndq_overlap_params* p64,
                const ndq_overlap_params* plo, const ndq_solve_params* sp, const ndq_spinor* b, const ndq_spinor* x) {
    if (!g || !p64 || !sp) return fail(NDQ_EINVAL, "solve: NULL argument");
    int rc = check_gauge(U64);
    if (!rc) rc = check_spinor(g, b, NDQ_FULL, "solve b");
    if (!rc) rc = check_spinor(g, x, NDQ_FULL, "solve x");
    if (rc) return rc;
    if (U64->prec != NDQ_F64 || b->prec != NDQ_F64 || x->prec != NDQ_F64)
        return fail(NDQ_EPREC, "solve: b, x and the outer links are F64");
    if (b->nrhs != 1 || x->nrhs != 1) return fail(NDQ_EINVAL, "solve: one right-hand side per call");
    if (sp->inner_prec != NDQ_F64) {
        if (!Ulo || !plo) return fail(NDQ_EINVAL, "solve: mixed precision needs inner links and parameters");
        if ((rc = check_gauge(Ulo))) return rc;
        if (Ulo->prec == NDQ_F64) return fail(NDQ_EPREC, "solve: inner links must be F32 or F16");
    }
    if (!(sp->tol > 0)) return fail(NDQ_EINVAL, "solve: tol must be positive");
    return NDQ_OK;
}

}  // namespace
}  // namespace ndq

using namespace ndq;

extern "C" {

size_t ndq_solve_workspace_bytes(const ndq_geom* g, const ndq_overlap_params* p64, const ndq_overlap_params* plo,
                                 const ndq_solve_params* sp) {
    if (!g || !p64 || !p64->approx || !sp) return 0;
    const int lo = sp->inner_prec;
    const ndq_overlap_params* pi = lo == NDQ_F64 ? p64 : plo;
    if (!pi || !pi->approx) return 0;
    size_t b = 0;
    b += 3 * ((size_t)spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL) + 256);        // r, t64, S64
    b += 8 * ((size_t)spinor_rhs_bytes(g, lo, NDQ_FULL) + 256);             // r_lo, S_lo, e s z p q t
    b += partials_capacity(g, 2) + 1024;
    const size_t s64 = sign_workspace(g, p64, NDQ_F64);
    const size_t slo = sign_workspace(g, pi, lo);
    return b + std::max(s64, slo) + 4096;
}

int ndq_solve_DN(const ndq_geom* g, const ndq_gauge* U64, const ndq_gauge* Ulo, const ndq_overlap_params* p64,
                 const ndq_overlap_params* plo, const ndq_solve_params* sp, const ndq_spinor* b, const ndq_spinor* x,
                 void* ws, size_t ws_bytes, ndq_stats* stats, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
    ndq_stats local;
    ndq_stats* stt = stats ? stats : &local;
    memset(stt, 0, sizeof(*stt));
    int rc = check_solve(g, U64, Ulo, p64, plo, sp, b, x);
    if (rc) return rc;
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
    const double inner_tol = sp->inner_tol > 0 ? sp->inner_tol : (lo == NDQ_F64 ? 0.5 * sp->tol : 1e-5);
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
        if ((rc = cgne(dlo, &rlo, v, inner_tol, max_inner, partials, dscal, &its))) return rc;
        stt->inner += its;
        // x += |r| e
        const ndq_spinor* ex = &v.e;
        if (lo != NDQ_F64) {
            if ((rc = convert(g, &t64, &v.e, st))) return rc;
            ex = &t64;
        }
        const ndq_spinor* s2[2] = {x, ex};
        const Coef c2[2] = {Coef{1.0, nullptr}, Coef{rn, nullptr}};
        if ((rc = lincomb(g, NDQ_F64, x, 2, s2, c2, nullptr, nullptr, st))) return rc;
    }
    stt->iterations = (int32_t)stt->inner;
    stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return NDQ_OK;
}

}  // extern "C"
