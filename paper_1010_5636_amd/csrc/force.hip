// Derivatives of y = Q[U] psi (Q of Sec. 2.1, Eq. 1) for a cotangent g.
//
// For a real function L of y with dL = Re<g, dy>, and links perturbed along su(3)
// as U_mu(x) -> exp(i w T_a) U_mu(x) (T_a = lambda_a / 2):
//
//   dL/dw^a_mu(x) = 1/2 Im tr(T_a G),
//   G = U_mu(x) H - K U_mu(x)^H,
//   H_ba = sum_s [(1 - gamma_mu) psi(x + mu)]_{s b} conj(chi(x)_{s a}),
//   K_ba = sum_s [(1 + gamma_mu) psi(x)]_{s b} conj(chi(x + mu)_{s a}),   chi = gamma5 g,
//
// because U_mu(x) enters D_W through the forward hop at x and the backward hop
// at x + mu, each with weight -1/2.  The gradient with respect to the complex
// link tensor in the tangent space is then 2 i sum_a F^a T_a U_mu(x), which
// satisfies Re<grad, i w T_a U> = w F^a.  One lane per (site, mu); FP64.
#include "ndq_internal.h"

using namespace ndq;

namespace {

// (1 -+ gamma_mu) psi with the chiral gamma matrices: upper two spins h, lower
// two from the fixed spin map (the same maps as the stencil's hop functions).
template <bool MINUS>
__device__ __forceinline__ void spin_project_full(int mu, const C<double> s[12], C<double> out[12]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const C<double> s0 = s[c], s1 = s[3 + c], s2 = s[6 + c], s3 = s[9 + c];
        C<double> h0, h1, l2, l3;
        if (mu == 0) {
            h0 = MINUS ? cadd(s0, s2) : csub(s0, s2);
            h1 = MINUS ? cadd(s1, s3) : csub(s1, s3);
            l2 = MINUS ? h0 : cneg(h0);
            l3 = MINUS ? h1 : cneg(h1);
        } else if (mu == 1) {
            h0 = MINUS ? cadd(s0, cmuli(s3)) : csub(s0, cmuli(s3));
            h1 = MINUS ? cadd(s1, cmuli(s2)) : csub(s1, cmuli(s2));
            l2 = MINUS ? cmulmi(h1) : cmuli(h1);
            l3 = MINUS ? cmulmi(h0) : cmuli(h0);
        } else if (mu == 2) {
            h0 = MINUS ? cadd(s0, s3) : csub(s0, s3);
            h1 = MINUS ? csub(s1, s2) : cadd(s1, s2);
            l2 = MINUS ? cneg(h1) : h1;
            l3 = MINUS ? h0 : cneg(h0);
        } else {
            h0 = MINUS ? cadd(s0, cmuli(s2)) : csub(s0, cmuli(s2));
            h1 = MINUS ? csub(s1, cmuli(s3)) : cadd(s1, cmuli(s3));
            l2 = MINUS ? cmulmi(h0) : cmuli(h0);
            l3 = MINUS ? cmuli(h1) : cmulmi(h1);
        }
        out[c] = h0;
        out[3 + c] = h1;
        out[6 + c] = l2;
        out[9 + c] = l3;
    }
}

// O_ba = sum_s p_{s b} conj(q_{s a})
__device__ __forceinline__ void outer(const C<double> p[12], const C<double> q[12], C<double> o[3][3]) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            C<double> acc = {0.0, 0.0};
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) acc = cfmac(acc, q[3 * sp + a], p[3 * sp + b]);
            o[b][a] = acc;
        }
}

struct ForceArgs {
    GeomK g;
    const char* links;
    SpinorView psi[2];   // parity views of psi
    SpinorView gv[2];    // parity views of g
    double* force;       // [V][4][8] (lexicographic) or nullptr
    double2* grad;       // [V][4][3][3] complex (lexicographic) or nullptr
};

// One workgroup per 64 sites of one parity; wavefront w takes direction mu = w,
// so the four directions of a site read psi(x) and g(x) from the same cache
// lines at about the same time.
template <int RECON>
__global__ void __launch_bounds__(256) k_force(ForceArgs a) {
    const int p = blockIdx.y;
    const int mu = threadIdx.x >> 6;
    const int32_t i = blockIdx.x * 64 + (threadIdx.x & 63);
    if (i >= a.g.vh) return;
    const SiteCoord x = eo_coords(a.g, p, i);
    int32_t nb[8];
    eo_neighbours(a.g, i, x, nb);
    C<double> u[3][3];
    link_load<P64, RECON>(a.links, a.g.vh, p * 4 + mu, i, u);
    C<double> sx[12], sf[12], gx[12], gf[12];
    SpinorIO<P64>::load(a.psi[p], (int64_t)a.psi[p].site0 + i, sx);
    SpinorIO<P64>::load(a.psi[1 - p], (int64_t)a.psi[1 - p].site0 + nb[mu], sf);
    SpinorIO<P64>::load(a.gv[p], (int64_t)a.gv[p].site0 + i, gx);
    SpinorIO<P64>::load(a.gv[1 - p], (int64_t)a.gv[1 - p].site0 + nb[mu], gf);
#pragma unroll
    for (int k = 6; k < 12; ++k) {   // chi = gamma5 g
        gx[k] = cneg(gx[k]);
        gf[k] = cneg(gf[k]);
    }
    C<double> hm[12], kp[12];
    spin_project_full<true>(mu, sf, hm);    // (1 - gamma_mu) psi(x + mu)
    spin_project_full<false>(mu, sx, kp);   // (1 + gamma_mu) psi(x)
    C<double> H[3][3], K[3][3], G[3][3];
    outer(hm, gx, H);
    outer(kp, gf, K);
    // G = U H - K U^H
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            C<double> acc = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                acc = cfma(acc, u[r][k], H[k][c]);
                acc = csub(acc, cmul(K[r][k], cconj(u[c][k])));
            }
            G[r][c] = acc;
        }
    // F^a = 1/2 Im tr(T_a G), T_a = lambda_a / 2 (Gell-Mann)
    double f[8];
    const double is3 = 0.57735026918962576451;   // 1/sqrt(3)
    f[0] = 0.25 * (G[1][0].i + G[0][1].i);                       // lambda_1: (0,1),(1,0) = 1
    f[1] = 0.25 * (G[0][1].r - G[1][0].r);                       // lambda_2: (0,1) = -i, (1,0) = i
    f[2] = 0.25 * (G[0][0].i - G[1][1].i);                       // lambda_3
    f[3] = 0.25 * (G[2][0].i + G[0][2].i);                       // lambda_4
    f[4] = 0.25 * (G[0][2].r - G[2][0].r);                       // lambda_5
    f[5] = 0.25 * (G[2][1].i + G[1][2].i);                       // lambda_6
    f[6] = 0.25 * (G[1][2].r - G[2][1].r);                       // lambda_7
    f[7] = 0.25 * is3 * (G[0][0].i + G[1][1].i - 2.0 * G[2][2].i);  // lambda_8
    const int64_t lex = 2 * (int64_t)i + (x.x3 & 1);
    if (a.force) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a.force[(lex * 4 + mu) * 8 + k] = f[k];
    }
    if (a.grad) {
        // 2 i sum_a f_a T_a U = i (sum_a f_a lambda_a) U
        C<double> Lm[3][3];
        Lm[0][0] = {f[2] + is3 * f[7], 0.0};
        Lm[1][1] = {-f[2] + is3 * f[7], 0.0};
        Lm[2][2] = {-2.0 * is3 * f[7], 0.0};
        Lm[0][1] = {f[0], -f[1]};
        Lm[1][0] = {f[0], f[1]};
        Lm[0][2] = {f[3], -f[4]};
        Lm[2][0] = {f[3], f[4]};
        Lm[1][2] = {f[5], -f[6]};
        Lm[2][1] = {f[5], f[6]};
        double2* dst = a.grad + (lex * 4 + mu) * 9;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                C<double> acc = {0.0, 0.0};
#pragma unroll
                for (int k = 0; k < 3; ++k) acc = cfma(acc, Lm[r][k], u[k][c]);
                const C<double> v = cmuli(acc);
                dst[3 * r + c] = make_double2(v.r, v.i);
            }
    }
}

}  // namespace

extern "C" int ndq_gauge_force(const ndq_geom* g, const ndq_gauge* U, const ndq_spinor* psi, const ndq_spinor* gy,
                               double* d_force, void* d_grad, void* stream) {
    if (!g) return fail(NDQ_EINVAL, "ndq_gauge_force: NULL geometry");
    int rc = check_gauge(U);
    if (!rc) rc = check_spinor(g, psi, NDQ_FULL, "ndq_gauge_force psi");
    if (!rc) rc = check_spinor(g, gy, NDQ_FULL, "ndq_gauge_force g");
    if (rc) return rc;
    if (U->prec != NDQ_F64 || psi->prec != NDQ_F64 || gy->prec != NDQ_F64)
        return fail(NDQ_EPREC, "ndq_gauge_force: FP64 links and spinors");
    if (psi->nrhs != 1 || gy->nrhs != 1) return fail(NDQ_EINVAL, "ndq_gauge_force: one right-hand side");
    if (!d_force && !d_grad) return fail(NDQ_EINVAL, "ndq_gauge_force: no output requested");
    ForceArgs a;
    a.g = g->k;
    a.links = static_cast<const char*>(U->data);
    for (int p = 0; p < 2; ++p) {
        a.psi[p] = view_of(g, psi, p, 0);
        a.gv[p] = view_of(g, gy, p, 0);
    }
    a.force = d_force;
    a.grad = static_cast<double2*>(d_grad);
    const dim3 grid((g->vh + 63) / 64, 2);
    hipStream_t st = as_stream(stream);
    switch (U->recon) {
        case 18: hipLaunchKernelGGL(k_force<18>, grid, dim3(256), 0, st, a); break;
        case 12: hipLaunchKernelGGL(k_force<12>, grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL(k_force<8>, grid, dim3(256), 0, st, a); break;
    }
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}
