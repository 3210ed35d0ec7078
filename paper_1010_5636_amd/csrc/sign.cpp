// sign(Q) with exact low modes (Sec. 2.3, Eq. 11) and the Neuberger-Dirac
// operator (Sec. 2.2, Eq. 4; massive form of Eq. 12): host orchestration of
// the stencil and vector kernels.
//
// Approximants act on X = Q / lam_max:
//  * polynomial, sign ~ X P(X^2), P = sum_k c_k T_k(Z), Z = (2 X^2 - 1 - eps)/(1 - eps),
//    evaluated by Clenshaw's recurrence b_j = c_j psi + 2 Z b_{j+1} - b_{j+2},
//    P psi = c_0 psi + Z b_1 - b_2, with every step fused into two stencil
//    launches (the second one's epilogue adds c_j psi, b_{j+1} and b_{j+2});
//    2n + 1 applications of Q, no reductions, no host synchronisation;
//  * rational, sign ~ X sum_l beta_l (X^2 + sigma_l)^{-1}, by multi-shift CG
//    with all scalars on the device; the host only reads the state every
//    `check_every` iterations.  Optionally each block of `check_every`
//    iterations is launched as one captured HIP graph.
#include <math.h>
#include <string.h>

#include <chrono>

#include "ndq_solver.h"

namespace ndq {

int q_combo_block(const ndq_geom* g, const ndq_gauge* U, double m, const ndq_spinor* in, const ndq_spinor* out,
                  Coef c0, int nv, const ndq_spinor* const* v, const Coef* cv, hipStream_t st) {
    WilsonArgs a = wilson_args(g, U, in->prec);
    a.p0 = 0;
    for (int p = 0; p < 2; ++p) {
        a.in[p] = view_of(g, in, 1 - p, 0);
        a.self[p] = view_of(g, in, p, 0);
        a.out[p] = view_of(g, out, p, 0);
        for (int j = 0; j < nv; ++j) a.v[j][p] = view_of(g, v[j], p, 0);
    }
    a.has_self = 1;
    a.a_self = 4.0 + m;
    a.b_hop = -0.5;
    a.gamma5 = 1;
    a.c0 = c0;
    a.nv = nv;
    for (int j = 0; j < nv; ++j) a.cv[j] = cv[j];
    NDQ_HIP(launch_wilson_mrhs(in->prec, U->prec, U->recon, a, 2, in->nrhs, st));
    return NDQ_OK;
}

int q_blocks(const ndq_geom* g, const ndq_gauge* U, int sprec) {
    return wilson_blocks(g, launch_tuning(g->k, sprec, U->prec, U->recon, 2).block, 2);
}

int q_combo(const ndq_geom* g, const ndq_gauge* U, double m, const ndq_spinor* in, const ndq_spinor* out, Coef c0,
            int nv, const ndq_spinor* const* v, const Coef* cv, double* partials, hipStream_t st) {
    WilsonArgs a = wilson_args(g, U, in->prec);
    a.p0 = 0;
    for (int p = 0; p < 2; ++p) {
        a.in[p] = view_of(g, in, 1 - p, 0);
        a.self[p] = view_of(g, in, p, 0);
        a.out[p] = view_of(g, out, p, 0);
        for (int j = 0; j < nv; ++j) a.v[j][p] = view_of(g, v[j], p, 0);
    }
    a.has_self = 1;
    a.a_self = 4.0 + m;
    a.b_hop = -0.5;
    a.gamma5 = 1;
    a.c0 = c0;
    a.nv = nv;
    for (int j = 0; j < nv; ++j) a.cv[j] = cv[j];
    a.partials = partials;
    NDQ_HIP(launch_wilson(in->prec, U->prec, U->recon, a, 2, -1, st));
    return NDQ_OK;
}

namespace {

struct Scratch {
    double* partials;      // generic partial sums
    double* part_tt;
    double* part_rr;
    double* part_pp;
    double* dots_c;        // <u_k, in>
    double* dots_d;        // <u_k, t>
    double* coef;
    MsState* ms;
};

Scratch take_scratch(Arena& ar, const ndq_geom* g, int nev, int nr = 1) {
    Scratch s;
    size_t pc = partials_capacity(g, std::max(2 * nev, 2));
    if (nr > 1 && nev > 0) pc = std::max(pc, gram_partials_bytes(g, nev, nr));
    s.partials = static_cast<double*>(ar.take(pc));
    s.part_tt = static_cast<double*>(ar.take(partials_capacity(g, 1)));
    s.part_rr = static_cast<double*>(ar.take(partials_capacity(g, 1)));
    s.part_pp = static_cast<double*>(ar.take(partials_capacity(g, 1)));
    s.dots_c = static_cast<double*>(ar.take(2 * NDQ_MAX_MODES * nr * sizeof(double)));
    s.dots_d = static_cast<double*>(ar.take(2 * NDQ_MAX_MODES * nr * sizeof(double)));
    s.coef = static_cast<double*>(ar.take(2 * NDQ_MAX_MODES * nr * sizeof(double)));
    s.ms = static_cast<MsState*>(ar.take(sizeof(MsState)));
    return s;
}

Coef host(double v) { return Coef{v, nullptr}; }

// out = c0 Q in + sum_k cv_k v_k: the one-lane-per-site stencil for one field,
// the multi-right-hand-side stencil (links loaded once per tile) for a block.
int q_any(const ndq_geom* g, const ndq_gauge* U, double m, const ndq_spinor* in, const ndq_spinor* out, Coef c0,
          int nv, const ndq_spinor* const* v, const Coef* cv, hipStream_t st) {
    if (in->nrhs == 1) return q_combo(g, U, m, in, out, c0, nv, v, cv, nullptr, st);
    return q_combo_block(g, U, m, in, out, c0, nv, v, cv, st);
}

// out = X P(X^2) src, Clenshaw's recurrence, for every field of the block src.
// Work blocks: B0, B1, T.
int poly_apply(const ndq_geom* g, const ndq_gauge* U, double m, const Approx& ap, double lam,
               const ndq_spinor* src, const ndq_spinor* out, Arena& ar, int64_t* qcount, hipStream_t st) {
    const int prec = src->prec;
    const int nr = src->nrhs;
    const int n = ap.n;
    const double eps = ap.lo;
    const double za = 4.0 / ((1.0 - eps) * lam * lam);     // coefficient of Q Q b in 2 Z b
    const double zb = -2.0 * (1.0 + eps) / (1.0 - eps);    // coefficient of b in 2 Z b
    if (n == 0) {
        *qcount += nr;
        return q_any(g, U, m, src, out, host(ap.a[0] / lam), 0, nullptr, nullptr, st);
    }
    ndq_spinor B[2] = {ws_block(ar, g, prec, nr), ws_block(ar, g, prec, nr)};
    ndq_spinor T = ws_block(ar, g, prec, nr);
    if (ar.overflow) return fail(NDQ_ENOMEM, "sign (polynomial): workspace too small (need %zu bytes)", ar.used);
    int rc;
    // b_n = c_n src
    {
        const ndq_spinor* v[1] = {src};
        const Coef c[1] = {host(ap.a[n])};
        if ((rc = lincomb(g, prec, &B[0], 1, v, c, nullptr, nullptr, st))) return rc;
    }
    const ndq_spinor* b1 = &B[0];      // b_{j+1}
    const ndq_spinor* b2 = nullptr;    // b_{j+2} (zero at the start)
    for (int j = n - 1; j >= 1; --j) {
        if ((rc = q_any(g, U, m, b1, &T, host(1.0), 0, nullptr, nullptr, st))) return rc;
        const ndq_spinor* target = b2 ? b2 : &B[1];
        const ndq_spinor* v[3] = {src, b1, b2};
        const Coef c[3] = {host(ap.a[j]), host(zb), host(-1.0)};
        if ((rc = q_any(g, U, m, &T, target, host(za), b2 ? 3 : 2, v, c, st))) return rc;
        b2 = b1;
        b1 = target;
        *qcount += 2 * nr;
    }
    // P src = c_0 src + Z b_1 - b_2
    if ((rc = q_any(g, U, m, b1, &T, host(1.0), 0, nullptr, nullptr, st))) return rc;
    const ndq_spinor* target = b2 ? b2 : &B[1];
    {
        const ndq_spinor* v[3] = {src, b1, b2};
        const Coef c[3] = {host(ap.a[0]), host(0.5 * zb), host(-1.0)};
        if ((rc = q_any(g, U, m, &T, target, host(0.5 * za), b2 ? 3 : 2, v, c, st))) return rc;
    }
    *qcount += 2 * nr;
    // out = Q (P src) / lam
    *qcount += nr;
    return q_any(g, U, m, target, out, host(1.0 / lam), 0, nullptr, nullptr, st);
}

// out = X sum_l beta_l (X^2 + sigma_l)^{-1} src by multi-shift CG.
int rational_apply(const ndq_geom* g, const ndq_gauge* U, double m, const Approx& ap, double lam,
                   const ndq_overlap_params* p, const ndq_spinor* src, const ndq_spinor* out, Arena& ar,
                   const Scratch& sc, int64_t* qcount, int* iters, double* resid, hipStream_t st) {
    const int prec = src->prec;
    const int n = ap.n;
    ndq_spinor r = ws_spinor(ar, g, prec), t = ws_spinor(ar, g, prec), y = ws_spinor(ar, g, prec);
    const size_t vb = (size_t)spinor_rhs_bytes(g, prec, NDQ_FULL);
    ndq_spinor P;
    P.data = ar.take(vb * n);
    P.prec = prec;
    P.parity = NDQ_FULL;
    P.nrhs = 1;
    if (ar.overflow) return fail(NDQ_ENOMEM, "sign (rational): workspace too small (need %zu bytes)", ar.used);
    MsConst k;
    memset(&k, 0, sizeof(k));
    k.n = n;
    k.inv_lam2 = 1.0 / (lam * lam);
    const double tol = p->tol > 0 ? p->tol : 1e-10;
    k.tol2 = tol * tol;
    for (int l = 0; l < n; ++l) {
        k.sigma[l] = ap.a[l];
        k.w[l] = ap.b[l];
    }
    int rc;
    // r = src (with |src|^2), y = 0, p_l = src
    {
        const ndq_spinor* v[1] = {src};
        const Coef c[1] = {host(1.0)};
        if ((rc = lincomb(g, prec, &r, 1, v, c, nullptr, sc.partials, st))) return rc;
        if ((rc = lincomb(g, prec, &y, 0, nullptr, nullptr, nullptr, nullptr, st))) return rc;
        for (int l = 0; l < n; ++l) {
            ndq_spinor pl = P;
            pl.data = static_cast<char*>(P.data) + vb * l;
            if ((rc = lincomb(g, prec, &pl, 1, v, c, nullptr, nullptr, st))) return rc;
        }
    }
    if ((rc = ms_init(sc.ms, k, sc.partials, lincomb_blocks(g), st))) return rc;
    const int nq = q_blocks(g, U, prec);
    const int nl = lincomb_blocks(g);
    const int max_iter = p->max_iter > 0 ? p->max_iter : 100000;
    const int every = p->check_every > 0 ? p->check_every : 8;
    ndq_spinor p0 = P;   // base shift sigma_0 (smallest)
    // one CG iteration for all shifts: two stencil launches, the scalar
    // recurrences on the device and the fused vector update
    auto iteration = [&](bool first, hipStream_t s) -> int {
        int e;
        if ((e = q_combo(g, U, m, &p0, &t, host(1.0), 0, nullptr, nullptr, sc.part_tt, s))) return e;
        if ((e = ms_alpha(sc.ms, k, sc.part_tt, nq, first ? nullptr : sc.part_pp, nl, s))) return e;
        // r <- r - alpha (X^2 + sigma_0) p_0 = (-alpha/lam^2) Q t + r - alpha sigma_0 p_0
        const ndq_spinor* v[2] = {&r, &p0};
        const Coef cv[2] = {host(1.0), Coef{1.0, &sc.ms->cp}};
        if ((e = q_combo(g, U, m, &t, &r, Coef{1.0, &sc.ms->c0}, 2, v, cv, sc.part_rr, s))) return e;
        if ((e = ms_beta(sc.ms, k, sc.part_rr, nq, s))) return e;
        return ms_update(g, prec, sc.ms, k, &r, &y, &P, sc.part_pp, s);
    };
    MsState hs;
    int it = 0;
    bool done = false;
    if (p->graph) {
        // the first iteration differs (no previous search direction); the
        // following blocks of `every` iterations are one captured graph each
        if ((rc = iteration(true, st))) return rc;
        *qcount += 2;
        ++it;
    }
    // everything the captured iterations depend on: lattice, links, mass,
    // launch shape, the workspace (all vectors and device scalars live in it)
    // and the shift constants
    std::string key;
    if (p->graph) {
        struct {
            const void* g;
            int32_t dims[4];      // a freed and re-created geometry may reuse the address
            const void* links;
            int32_t prec, lprec, recon, every, block, xcd;
            double m;
            const void* r;
            const void* ws;
        } head;
        memset(&head, 0, sizeof(head));
        const Tuning tu = launch_tuning(g->k, prec, U->prec, U->recon, 2);
        head.g = g;
        for (int d = 0; d < 4; ++d) head.dims[d] = g->dims[d];
        head.links = U->data;
        head.prec = prec;
        head.lprec = U->prec;
        head.recon = U->recon;
        head.every = every;
        head.block = tu.block;
        head.xcd = tu.xcd_remap;
        head.m = m;
        head.r = r.data;
        head.ws = sc.ms;
        key.assign(reinterpret_cast<const char*>(&head), sizeof(head));
        key.append(reinterpret_cast<const char*>(&k), sizeof(k));
    }
    while (!done) {
        if (p->graph) {
            rc = launch_captured([&](hipStream_t s) -> int {
                for (int c = 0; c < every; ++c) {
                    const int e = iteration(false, s);
                    if (e) return e;
                }
                return NDQ_OK;
            }, st, key);
            if (rc) return rc;
            *qcount += 2 * every;
            it += every;
        } else {
            for (int c = 0; c < every; ++c) {
                if ((rc = iteration(it == 0, st))) return rc;
                *qcount += 2;
                ++it;
            }
        }
        NDQ_HIP(hipMemcpyAsync(&hs, sc.ms, sizeof(MsState), hipMemcpyDeviceToHost, st));
        NDQ_HIP(hipStreamSynchronize(st));
        if (hs.bad) return fail(NDQ_ENAN, "sign (rational): NaN or Inf in the multi-shift CG");
        // iterations past convergence are no-ops for frozen shifts; count the real ones
        if (hs.done) {
            done = true;
            it = hs.iter;
        } else if (it >= max_iter) {
            *iters = hs.iter;
            *resid = hs.b2 > 0 ? sqrt(hs.rr / hs.b2) : 0.0;
            return fail(NDQ_ENOCONV, "sign (rational): no convergence in %d iterations (residual %.3e)", it, *resid);
        }
    }
    *iters = it;
    *resid = hs.b2 > 0 ? sqrt(hs.rr / hs.b2) : 0.0;
    *qcount += 1;
    return q_combo(g, U, m, &y, out, host(1.0 / lam), 0, nullptr, nullptr, nullptr, st);
}

int check_params(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p, const ndq_spinor* in,
                 const ndq_spinor* out) {
    if (!g || !p) return fail(NDQ_EINVAL, "sign: NULL geometry or parameters");
    int rc = check_gauge(U);
    if (!rc) rc = check_spinor(g, in, NDQ_FULL, "sign in");
    if (!rc) rc = check_spinor(g, out, NDQ_FULL, "sign out");
    if (!rc) rc = check_pair(U, in);
    if (rc) return rc;
    if (in->nrhs != out->nrhs) return fail(NDQ_EINVAL, "sign: in and out must hold the same number of fields");
    if (in->nrhs > NDQ_MAX_BATCH) return fail(NDQ_EINVAL, "sign: at most %d right-hand sides per call", NDQ_MAX_BATCH);
    if (in->prec != out->prec) return fail(NDQ_EINVAL, "sign: in and out must share precision");
    if (in->data == out->data) return fail(NDQ_EINVAL, "sign: in and out must not alias");
    if (!p->approx) return fail(NDQ_EINVAL, "sign: no approximant");
    if (!(p->lam_max > 0)) return fail(NDQ_EINVAL, "sign: lam_max must be positive");
    if (p->nev < 0 || p->nev > NDQ_MAX_MODES) return fail(NDQ_EINVAL, "sign: nev must be in [0, %d]", NDQ_MAX_MODES);
    if (p->nev > 0) {
        if (!p->modes || !p->nu) return fail(NDQ_EINVAL, "sign: nev > 0 needs modes and nu");
        for (int k = 0; k < p->nev; ++k)
            if (p->nu[k] == 0.0 || !isfinite(p->nu[k]))
                return fail(NDQ_ESINGULAR, "sign: low mode %d has nu = %g (no sign)", k, p->nu[k]);
    }
    if (p->form != NDQ_LITERAL && p->form != NDQ_SANDWICH) return fail(NDQ_EINVAL, "sign: bad projection form");
    return NDQ_OK;
}

}  // namespace

size_t sign_workspace(const ndq_geom* g, const ndq_overlap_params* p, int prec, int nr) {
    const Approx* ap = reinterpret_cast<const Approx*>(p->approx);
    // the rational approximant runs one field at a time
    const int nb = ap->kind == NDQ_MINMAX_POLY ? nr : 1;
    Arena ar{nullptr, 0};
    take_scratch(ar, g, p->nev, nb);
    if (p->nev > 0 && p->form == NDQ_SANDWICH) ws_block(ar, g, prec, nb);
    if (p->nev > 0 && nb > 1 && prec == NDQ_F16) ws_block(ar, g, NDQ_F32, nb);
    const size_t vb = (size_t)spinor_rhs_bytes(g, prec, NDQ_FULL);
    for (int i = 0; i < 3; ++i) ws_block(ar, g, prec, nb);
    if (ap->kind != NDQ_MINMAX_POLY) ar.take(vb * ap->n);
    return ar.used + 256;
}

namespace {

// Eq. 11 for a block of fields: out_r = in_r + sum_k coef[k][r] u_k with the
// coefficients in sc.coef; F16 fields pass through the F32 block t32.
int project_block(const ndq_geom* g, const ndq_overlap_params* p, const Scratch& sc, const ndq_spinor* in,
                  const ndq_spinor* out, const ndq_spinor* t32, hipStream_t st) {
    if (out->prec != NDQ_F16) return mode_update_block(g, p->modes, p->nev, sc.coef, in, out, st);
    int rc = mode_update_block(g, p->modes, p->nev, sc.coef, in, t32, st);
    if (!rc) rc = convert(g, out, t32, st);
    return rc;
}

// sign(Q) on a block of fields with the polynomial approximant: every stencil
// application of the recurrence serves the whole block (links loaded once per
// tile), and the projections of Eq. 11 run as block products with the modes.
int apply_sign_block(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p, const ndq_spinor* in,
                     const ndq_spinor* out, Arena& ar, ndq_stats* stats, hipStream_t st) {
    const Approx& ap = *reinterpret_cast<const Approx*>(p->approx);
    const int nev = p->nev;
    const int nr = in->nrhs;
    Scratch sc = take_scratch(ar, g, nev, nr);
    ndq_spinor t32;
    memset(&t32, 0, sizeof(t32));
    if (nev > 0 && in->prec == NDQ_F16) t32 = ws_block(ar, g, NDQ_F32, nr);
    if (ar.overflow) return fail(NDQ_ENOMEM, "sign: workspace too small");
    ModeSigns sg;
    for (int k = 0; k < NDQ_MAX_MODES; ++k) sg.s[k] = k < nev ? (p->nu[k] > 0 ? 1.0f : -1.0f) : 0.0f;
    const ndq_spinor* src = in;
    ndq_spinor defl;
    int rc;
    if (nev > 0) {
        // c[k][r] = <u_k, in_r>
        if ((rc = gram_block(g, p->modes, nev, in, sc.partials, sc.dots_c, st))) return rc;
        if (p->form == NDQ_SANDWICH) {
            defl = ws_block(ar, g, in->prec, nr);
            if (ar.overflow) return fail(NDQ_ENOMEM, "sign: workspace too small");
            if ((rc = mode_coef_block(sc.dots_c, nullptr, sg, 0, nev, nr, -1.0, 0.0, sc.coef, st))) return rc;
            if ((rc = project_block(g, p, sc, in, &defl, &t32, st))) return rc;
            src = &defl;
        }
    }
    int64_t q = 0;
    rc = poly_apply(g, U, p->m, ap, p->lam_max, src, out, ar, &q, st);
    if (stats) {
        stats->q_applies += q;
        stats->iterations += ap.n;
        stats->residual = 0.0;
    }
    if (rc) return rc;
    if (nev > 0) {
        // out_r <- t_r + sum_k (sign(nu_k) c[k][r] - <u_k, t_r>) u_k   (Eq. 11)
        if ((rc = gram_block(g, p->modes, nev, out, sc.partials, sc.dots_d, st))) return rc;
        if ((rc = mode_coef_block(sc.dots_c, sc.dots_d, sg, 1, nev, nr, 1.0, -1.0, sc.coef, st))) return rc;
        if ((rc = project_block(g, p, sc, out, out, &t32, st))) return rc;
    }
    return NDQ_OK;
}

}  // namespace

int apply_sign(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p, const ndq_spinor* in,
               const ndq_spinor* out, Arena& ar, ndq_stats* stats, hipStream_t st) {
    int rc = check_params(g, U, p, in, out);
    if (rc) return rc;
    const Approx& ap = *reinterpret_cast<const Approx*>(p->approx);
    if (in->nrhs > 1) {
        if (ap.kind == NDQ_MINMAX_POLY) return apply_sign_block(g, U, p, in, out, ar, stats, st);
        // the rational approximant: one field at a time (multi-shift CG keeps
        // scalars per field); every field reuses the same workspace
        const size_t mark = ar.used;
        for (int r = 0; r < in->nrhs; ++r) {
            ar.used = mark;
            ar.overflow = false;
            const ndq_spinor i1 = rhs_slice(g, in, r), o1 = rhs_slice(g, out, r);
            ndq_stats s1;
            memset(&s1, 0, sizeof(s1));
            if ((rc = apply_sign(g, U, p, &i1, &o1, ar, &s1, st))) return rc;
            if (stats) {
                stats->q_applies += s1.q_applies;
                stats->iterations += s1.iterations;
                stats->residual = std::max(stats->residual, s1.residual);
            }
        }
        return NDQ_OK;
    }
    const int nev = p->nev;
    Scratch sc = take_scratch(ar, g, nev);

    if (ar.overflow) return fail(NDQ_ENOMEM, "sign: workspace too small");
    ModeSigns sg;
    for (int k = 0; k < NDQ_MAX_MODES; ++k) sg.s[k] = k < nev ? (p->nu[k] > 0 ? 1.0f : -1.0f) : 0.0f;
    const ndq_spinor* src = in;
    ndq_spinor defl;
    if (nev > 0) {
        if ((rc = mode_dots(g, p->modes, nev, in, sc.partials, sc.dots_c, st))) return rc;
        if (p->form == NDQ_SANDWICH) {
            defl = ws_spinor(ar, g, in->prec);
            if (ar.overflow) return fail(NDQ_ENOMEM, "sign: workspace too small");
            if ((rc = mode_coef(sc.dots_c, nullptr, sg, 0, nev, -1.0, 0.0, sc.coef, st))) return rc;
            if ((rc = mode_update(g, p->modes, nev, sc.coef, in, &defl, st))) return rc;
            src = &defl;
        }
    }
    int64_t q = 0;
    int iters = 0;
    double resid = 0.0;
    if (ap.kind == NDQ_MINMAX_POLY) {
        rc = poly_apply(g, U, p->m, ap, p->lam_max, src, out, ar, &q, st);
        iters = ap.n;
    } else {
        rc = rational_apply(g, U, p->m, ap, p->lam_max, p, src, out, ar, sc, &q, &iters, &resid, st);
    }
    if (stats) {
        stats->q_applies += q;
        stats->iterations += iters;
        stats->residual = resid;
    }
    if (rc) return rc;
    if (nev > 0) {
        // out <- t + sum_k (sign(nu_k) c_k - <u_k, t>) u_k   (Eq. 11)
        if ((rc = mode_dots(g, p->modes, nev, out, sc.partials, sc.dots_d, st))) return rc;
        if ((rc = mode_coef(sc.dots_c, sc.dots_d, sg, 1, nev, 1.0, -1.0, sc.coef, st))) return rc;
        if ((rc = mode_update(g, p->modes, nev, sc.coef, out, out, st))) return rc;
    }
    return NDQ_OK;
}

}  // namespace ndq

using namespace ndq;

extern "C" {

size_t ndq_workspace_bytes_nrhs(const ndq_geom* g, const ndq_overlap_params* p, int prec, int op, int nrhs) {
    if (!g || !p || !p->approx || prec < NDQ_F64 || prec > NDQ_F16 || p->nev < 0 || p->nev > NDQ_MAX_MODES ||
        nrhs < 1 || nrhs > NDQ_MAX_BATCH)
        return 0;
    size_t b = sign_workspace(g, p, prec, nrhs);
    if (op == NDQ_OP_DN) b += (size_t)spinor_rhs_bytes(g, prec, NDQ_FULL) * nrhs + 256;
    return b;
}

size_t ndq_workspace_bytes(const ndq_geom* g, const ndq_overlap_params* p, int prec, int op) {
    return ndq_workspace_bytes_nrhs(g, p, prec, op, 1);
}

int ndq_apply_sign(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p, const ndq_spinor* in,
                   const ndq_spinor* out, void* ws, size_t ws_bytes, ndq_stats* stats, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
    Arena ar{static_cast<char*>(ws), ws_bytes};
    if (stats) memset(stats, 0, sizeof(*stats));
    const int rc = apply_sign(g, U, p, in, out, ar, stats, as_stream(stream));
    if (stats) stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int ndq_apply_DN(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p, const ndq_spinor* in,
                 const ndq_spinor* out, void* ws, size_t ws_bytes, ndq_stats* stats, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
    if (stats) memset(stats, 0, sizeof(*stats));
    int rc = check_params(g, U, p, in, out);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    Arena ar{static_cast<char*>(ws), ws_bytes};
    ndq_spinor S = ws_block(ar, g, in->prec, in->nrhs);
    if (ar.overflow) return fail(NDQ_ENOMEM, "D_N: workspace too small");
    if ((rc = apply_sign(g, U, p, in, &S, ar, stats, st))) return rc;
    // D_N^m in = (1/abar - mq/2)(in + gamma5 S in) + mq in, 1/abar = 1 + s = -m
    const double inv_abar = -p->m;
    const ndq_spinor* v[2] = {in, &S};
    const Coef c[2] = {Coef{inv_abar + 0.5 * p->mq, nullptr}, Coef{inv_abar - 0.5 * p->mq, nullptr}};
    const int g5[2] = {0, 1};
    rc = lincomb(g, in->prec, out, 2, v, c, g5, nullptr, st);
    if (stats) stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

}  // extern "C"
