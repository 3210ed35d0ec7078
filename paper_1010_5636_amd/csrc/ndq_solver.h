// Internal interfaces of the sign-function, D_N and solver layers.
#pragma once

#include <functional>
#include <string>
#include <vector>

#include "ndq_internal.h"
#include "wilson.h"

#define NDQ_MAX_SHIFTS 32
#define NDQ_MAX_MODES 64
#define NDQ_MAX_BATCH 32   // right-hand sides of one batched sign, D_N or solve call

namespace ndq {

struct Approx {
    int kind;                 // NDQ_ZOLOTAREV or NDQ_MINMAX_POLY
    int n;                    // poles, or polynomial degree
    double lo;                // k (Zolotarev, on |x|) or eps (polynomial, on y = x^2)
    double delta;             // max approximation error on the interval
    std::vector<double> a;    // sigma_l (ascending) or c_0..c_n
    std::vector<double> b;    // beta_l (Zolotarev only)
};

// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct Arena {
    char* base;
    size_t size;
    size_t used = 0;
    bool overflow = false;
    void* take(size_t bytes) {
        const size_t off = (used + 255) & ~size_t(255);
        if (off + bytes > size || base == nullptr) {
            overflow = true;
            used = off + bytes;
            return nullptr;
        }
        used = off + bytes;
        return base + off;
    }
};

// A full (both parities), single right-hand-side spinor in workspace memory.
inline ndq_spinor ws_spinor(Arena& ar, const ndq_geom* g, int prec) {
    ndq_spinor s;
    s.data = ar.take((size_t)spinor_rhs_bytes(g, prec, NDQ_FULL));
    s.prec = prec;
    s.parity = NDQ_FULL;
    s.nrhs = 1;
    return s;
}

// A block of nr full spinors of one precision in workspace memory.
inline ndq_spinor ws_block(Arena& ar, const ndq_geom* g, int prec, int nr) {
    ndq_spinor s;
    s.data = ar.take((size_t)spinor_rhs_bytes(g, prec, NDQ_FULL) * nr);
    s.prec = prec;
    s.parity = NDQ_FULL;
    s.nrhs = nr;
    return s;
}

// Field r of a block, as a one-field descriptor.
inline ndq_spinor rhs_slice(const ndq_geom* g, const ndq_spinor* s, int r) {
    ndq_spinor o = *s;
    o.data = static_cast<char*>(s->data) + spinor_rhs_bytes(g, s->prec, s->parity) * r;
    o.nrhs = 1;
    return o;
}

// View of a whole full spinor as V consecutive sites (for site-local kernels).
inline SpinorView flat_view(const ndq_geom* g, const ndq_spinor* s, int rhs = 0) {
    SpinorView v = view_of(g, s, 0, rhs);
    v.stride = (int32_t)g->volume;
    v.site0 = 0;
    return v;
}

// ---- BLAS-1 and reductions (blas.hip) --------------------------------------
// Upper bound on the per-block partial sums any kernel below writes.
size_t partials_capacity(const ndq_geom* g, int nvals);

// out = sum_k c_k G5^{g5_k} v_k (k < nv <= 4), optional |out|^2 partials.
// All vectors full fields of precision `prec`; out may alias a v_k.  Every
// operand holds out->nrhs fields; field r of out combines fields r of the v_k
// (partials: per field and block, field-major, one value each).
int lincomb(const ndq_geom* g, int prec, const ndq_spinor* out, int nv, const ndq_spinor* const* v,
            const Coef* c, const int* g5, double* partials, hipStream_t st);
// The same with coefficients per field: cr[k * out->nrhs + r] for vector k and
// field r (host array; out->nrhs <= NDQ_MAX_BATCH).
int lincomb_rhs(const ndq_geom* g, int prec, const ndq_spinor* out, int nv, const ndq_spinor* const* v,
                const double* cr, const int* g5, double* partials, hipStream_t st);
// Sum per-block partials into dst: nvals values interleaved per block
// (reduce_partials) or one row of nblocks partials per value (reduce_rows).
int reduce_partials(const double* partials, int nblocks, int nvals, double* dst, hipStream_t st);
int reduce_rows(const double* partials, int nblocks, int nvals, double* dst, hipStream_t st);
int lincomb_blocks(const ndq_geom* g);
// <x_r, y_r> (complex, FP64 accumulation) into dst[2r..2r+1] for every field r
// of the blocks x and y; |x_r|^2 into dst[r] if y == nullptr.  partials needs
// partials_capacity(g, 2 * x->nrhs).
int dot(const ndq_geom* g, const ndq_spinor* x, const ndq_spinor* y, double* partials, double* dst, hipStream_t st);
// Precision conversion between blocks of full fields (same site layout and count).
int convert(const ndq_geom* g, const ndq_spinor* dst, const ndq_spinor* src, hipStream_t st);

// Low modes: dots[k] = <u_k, v> for the nev packed F64 full spinors at `modes`.
// G (device, na x nb complex, row-major) = A^H B for blocks of na and nb FP64
// full spinor fields (contiguous, na, nb <= 64), on the matrix cores; partials
// needs gram_partials_bytes(g, na, nb).
size_t gram_partials_bytes(const ndq_geom* g, int na, int nb);
int gram(const ndq_geom* g, const void* A, int na, const void* B, int nb, double* partials, double* G,
         hipStream_t st);
int mode_dots(const ndq_geom* g, const void* modes, int nev, const ndq_spinor* v, double* partials,
              double* dots, hipStream_t st);
// coef_k = sc * (use_sign ? sign_k : 1) * c_k + sd * d_k (complex, device arrays of 2*nev doubles).
struct ModeSigns {
    float s[NDQ_MAX_MODES];
};
// Block forms for a block B of nr fields (any precision): G[k][r] = <u_k, B_r>
// (nev x nr complex, row-major) on the matrix cores (partials:
// gram_partials_bytes(g, nev, nr)); coef[k][r] as mode_coef; out_r = in_r +
// sum_k coef[k][r] u_k (out F64 or F32; in F64, F32 or F16).
int gram_block(const ndq_geom* g, const void* modes, int nev, const ndq_spinor* B, double* partials, double* G,
               hipStream_t st);
int mode_coef_block(const double* c, const double* d, const ModeSigns& sg, int use_sign, int nev, int nr, double sc,
                    double sd, double* coef, hipStream_t st);
int mode_update_block(const ndq_geom* g, const void* modes, int nev, const double* coef, const ndq_spinor* in,
                      const ndq_spinor* out, hipStream_t st);
int mode_coef(const double* c, const double* d, const ModeSigns& sg, int use_sign, int nev, double sc, double sd,
              double* coef, hipStream_t st);
// out = in + sum_k coef_k u_k (coef complex, device array of 2*nev doubles).
int mode_update(const ndq_geom* g, const void* modes, int nev, const double* coef, const ndq_spinor* in,
                const ndq_spinor* out, hipStream_t st);

// dst_j = sum_i src_i Y[i][j] (j < k) over contiguous blocks of FP64 full spinors;
// Y complex row-major [nsrc][k] in device memory; dst must not overlap src.
int rotate(const ndq_geom* g, const void* src, int nsrc, const double* Y, int k, void* dst, hipStream_t st);

// dst = src * exp(i theta(idx, site, component)), a hashed unit phase per
// component (idx = 0: plain copy); FP64 full fields.
int phase_copy(const ndq_geom* g, const ndq_spinor* src, const ndq_spinor* dst, int idx, hipStream_t st);

// ---- multi-shift CG device state (blas.hip) ---------------------------------
struct MsState {
    double b2;                        // |b|^2
    double rr;                        // |r|^2
    double tt;                        // |Q p_s|^2
    double pp;                        // |p_s|^2
    double alpha, alpha_prev, beta_prev;
    double c0, cp;                    // epilogue coefficients of the residual update
    double zeta[NDQ_MAX_SHIFTS], zeta_prev[NDQ_MAX_SHIFTS], zeta_new[NDQ_MAX_SHIFTS];
    double ycoef[NDQ_MAX_SHIFTS], pcoef[NDQ_MAX_SHIFTS], bl[NDQ_MAX_SHIFTS];
    int upd_y[NDQ_MAX_SHIFTS], upd_p[NDQ_MAX_SHIFTS];
    int iter, done, bad;
};

struct MsConst {
    int n;
    double inv_lam2;                  // 1 / lam_max^2
    double tol2;                      // tol^2
    double sigma[NDQ_MAX_SHIFTS];
    double w[NDQ_MAX_SHIFTS];         // residues
};

int ms_init(MsState* st_dev, const MsConst& k, const double* b2_partials, int nblk, hipStream_t st);
int ms_alpha(MsState* st_dev, const MsConst& k, const double* tt_partials, int nblk_tt, const double* pp_partials,
             int nblk_pp, hipStream_t st);
int ms_beta(MsState* st_dev, const MsConst& k, const double* rr_partials, int nblk, hipStream_t st);
int ms_update(const ndq_geom* g, int prec, MsState* st_dev, const MsConst& k, const ndq_spinor* r,
              const ndq_spinor* y, const ndq_spinor* p, double* partials, hipStream_t st);

// ---- sign and D_N (sign.cpp) --------------------------------------------------
// The overlap parameters with the projection of Eq. 11 in the sandwich form
// (1 - P) r(X) (1 - P) + P_+ - P_-, which keeps sign(Q) exactly Hermitian for
// inexact modes (the literal form differs by the commutator [r(X), P] = O(rho)).
// Used where an algorithm relies on that symmetry: CG on the normal equations
// (D^H = gamma5 D gamma5) and the Hermitian sector operators of the index.
inline ndq_overlap_params hermitian_form(const ndq_overlap_params* p) {
    ndq_overlap_params q = *p;
    q.form = NDQ_SANDWICH;
    return q;
}

size_t sign_workspace(const ndq_geom* g, const ndq_overlap_params* p, int prec, int nr = 1);
int apply_sign(const ndq_geom* g, const ndq_gauge* U, const ndq_overlap_params* p, const ndq_spinor* in,
               const ndq_spinor* out, Arena& ar, ndq_stats* stats, hipStream_t st);

// Stencil helper: out = c0 * Q in + sum_k cv_k v_k (full fields), optional partials.
int q_combo(const ndq_geom* g, const ndq_gauge* U, double m, const ndq_spinor* in, const ndq_spinor* out,
            Coef c0, int nv, const ndq_spinor* const* v, const Coef* cv, double* partials, hipStream_t st);
int q_blocks(const ndq_geom* g, const ndq_gauge* U, int sprec);
// The same for in->nrhs right-hand sides in one multi-RHS launch (links staged
// once per tile); in, out and v share nrhs; no partial sums.
int q_combo_block(const ndq_geom* g, const ndq_gauge* U, double m, const ndq_spinor* in, const ndq_spinor* out,
                  Coef c0, int nv, const ndq_spinor* const* v, const Coef* cv, hipStream_t st);

// Records the kernel launches `body` makes on the stream it is given into a HIP
// graph and launches the graph on `st` (kept instantiated graphs are refreshed
// with hipGraphExecUpdate).  `body` must launch kernels only.
// `key` (may be empty): bytes that determine every argument of the sequence;
// an equal key replays the kept graph without capturing.
int launch_captured(const std::function<int(hipStream_t)>& body, hipStream_t st, const std::string& key);

}  // namespace ndq
