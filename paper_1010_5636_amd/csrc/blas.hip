// Site-local vector kernels of the sign-function and solver layers: linear
// combinations (with optional gamma5), FP64 reductions in a fixed order,
// precision conversion, the fused multi-shift CG update with its device-side
// scalar recurrences, and the low-mode projection (multi-dot and rank-nev
// update against FP64 eigenvectors).
//
// One lane per site; fields are full spinors viewed as V consecutive sites.
// Reductions: each block writes its partial sums; a single-block kernel adds
// them in index order, so results do not depend on scheduling.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "ndq_solver.h"

using namespace ndq;

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ double coefv(const Coef& c) { return c.d ? c.f * (*c.d) : c.f; }

struct LinArgs {
    SpinorView out;            // right-hand side r at base + r * rhs_bytes (every view)
    SpinorView v[4];
    Coef c[4];
    int g5[4];
    int nv;
    int32_t nsites;
    double* partials;          // per (right-hand side, block): partials[r * gridDim.x + block]
};

// Coefficients that differ between right-hand sides: c[j][r] for vector j.
struct LinRhs {
    double c[4][NDQ_MAX_BATCH];
};

// One site of out_r = sum_j c_j G5^{g5_j} v_j,r (grid row y = right-hand side r).
template <int P>
__device__ __forceinline__ void lincomb_site(const LinArgs& a, const double* cr) {
    using R = typename SpinorIO<P>::R;
    __shared__ double lds[kBlock / 64];
    const int r = blockIdx.y;
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    double red = 0.0;
    if (s < a.nsites) {
        C<R> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
        for (int j = 0; j < a.nv; ++j) {
            C<R> x[12];
            SpinorView vj = a.v[j];
            vj.base += (int64_t)r * vj.rhs_bytes;
            SpinorIO<P>::load(vj, s, x);
            const R c = (R)(cr ? cr[j * NDQ_MAX_BATCH + r] : coefv(a.c[j]));
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                const R ck = (a.g5[j] && k >= 6) ? -c : c;
                acc[k] = {acc[k].r + ck * x[k].r, acc[k].i + ck * x[k].i};
            }
        }
        SpinorView vo = a.out;
        vo.base += (int64_t)r * vo.rhs_bytes;
        SpinorIO<P>::store(vo, s, acc);
        if (a.partials) {
            if constexpr (P == P16) SpinorIO<P>::load(vo, s, acc);
#pragma unroll
            for (int k = 0; k < 12; ++k) red += (double)acc[k].r * acc[k].r + (double)acc[k].i * acc[k].i;
        }
    }
    if (a.partials) {
        const double t = block_sum(red, lds);
        if (threadIdx.x == 0) a.partials[(int64_t)r * gridDim.x + blockIdx.x] = t;
    }
}

template <int P>
__global__ void __launch_bounds__(kBlock) k_lincomb(LinArgs a) {
    lincomb_site<P>(a, nullptr);
}

template <int P>
__global__ void __launch_bounds__(kBlock) k_lincomb_rhs(LinArgs a, LinRhs b) {
    lincomb_site<P>(a, &b.c[0][0]);
}

// dst[j] = sum_b partials[j * jstride + b * bstride] for j < gridDim.x, one
// workgroup per value; every value adds its blocks in the same fixed order.
__global__ void __launch_bounds__(kBlock) k_reduce(const double* __restrict__ partials, int nblocks, int64_t jstride,
                                                   int bstride, double* __restrict__ dst) {
    __shared__ double lds[kBlock / 64];
    const int j = blockIdx.x;
    const double* p = partials + (int64_t)j * jstride;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) s += p[(int64_t)b * bstride];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) dst[j] = s;
}

// Per right-hand side r (grid row y): <x_r, y_r> (complex) or |x_r|^2 into
// partials[(nv * r + c) * gridDim.x + block], nv = 2 or 1 values per field.
template <int P>
__global__ void __launch_bounds__(kBlock) k_dot(SpinorView x, SpinorView y, int has_y, int32_t n,
                                                double* __restrict__ partials) {
    using R = typename SpinorIO<P>::R;
    __shared__ double lds[kBlock / 64];
    const int r = blockIdx.y;
    x.base += (int64_t)r * x.rhs_bytes;
    y.base += (int64_t)r * y.rhs_bytes;
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (s < n) {
        C<R> a[12];
        SpinorIO<P>::load(x, s, a);
        if (has_y) {
            C<R> b[12];
            SpinorIO<P>::load(y, s, b);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                re += (double)a[k].r * b[k].r + (double)a[k].i * b[k].i;
                im += (double)a[k].r * b[k].i - (double)a[k].i * b[k].r;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) re += (double)a[k].r * a[k].r + (double)a[k].i * a[k].i;
        }
    }
    const int64_t nb = gridDim.x;
    const double sr = block_sum(re, lds);
    __syncthreads();
    if (has_y) {
        const double si = block_sum(im, lds);
        if (threadIdx.x == 0) {
            partials[(2 * r) * nb + blockIdx.x] = sr;
            partials[(2 * r + 1) * nb + blockIdx.x] = si;
        }
    } else if (threadIdx.x == 0) {
        partials[r * nb + blockIdx.x] = sr;
    }
}

template <int PD, int PS>
__global__ void __launch_bounds__(kBlock) k_convert(SpinorView dst, SpinorView src, int32_t n) {
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    dst.base += (int64_t)blockIdx.y * dst.rhs_bytes;
    src.base += (int64_t)blockIdx.y * src.rhs_bytes;
    using RS = typename SpinorIO<PS>::R;
    using RD = typename SpinorIO<PD>::R;
    C<RS> a[12];
    SpinorIO<PS>::load(src, s, a);
    C<RD> b[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) b[k] = {(RD)a[k].r, (RD)a[k].i};
    SpinorIO<PD>::store(dst, s, b);
}

// ---- low-mode projection ----------------------------------------------------

// partials[block][2k + {0,1}] = sum over the block's sites of <u_k, v>.
template <int P>
__global__ void __launch_bounds__(kBlock) k_mode_dots(const char* __restrict__ modes, int64_t mode_bytes, int nev,
                                                      SpinorView v, SpinorView um, int32_t n,
                                                      double* __restrict__ partials) {
    using R = typename SpinorIO<P>::R;
    __shared__ double lds[kBlock / 64][2 * NDQ_MAX_MODES];
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    C<double> x[12];
    if (s < n) {
        C<R> t[12];
        SpinorIO<P>::load(v, s, t);
#pragma unroll
        for (int k = 0; k < 12; ++k) x[k] = {(double)t[k].r, (double)t[k].i};
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) x[k] = {0.0, 0.0};
    }
    for (int m = 0; m < nev; ++m) {
        double re = 0.0, im = 0.0;
        if (s < n) {
            SpinorView u = um;
            u.base = const_cast<char*>(modes) + (int64_t)m * mode_bytes;
            C<double> w[12];
            SpinorIO<P64>::load(u, s, w);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                re += w[k].r * x[k].r + w[k].i * x[k].i;
                im += w[k].r * x[k].i - w[k].i * x[k].r;
            }
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) {
            lds[wave][2 * m] = re;
            lds[wave][2 * m + 1] = im;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < 2 * nev; j += kBlock) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += lds[w][j];
        partials[(int64_t)blockIdx.x * 2 * nev + j] = t;
    }
}

// out = in + sum_k coef_k u_k
template <int P>
__global__ void __launch_bounds__(kBlock) k_mode_update(const char* __restrict__ modes, int64_t mode_bytes, int nev,
                                                        const double* __restrict__ coef, SpinorView in,
                                                        SpinorView out, SpinorView um, int32_t n) {
    using R = typename SpinorIO<P>::R;
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    C<R> t[12];
    SpinorIO<P>::load(in, s, t);
    C<double> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = {(double)t[k].r, (double)t[k].i};
    for (int m = 0; m < nev; ++m) {
        const C<double> c = {coef[2 * m], coef[2 * m + 1]};
        SpinorView u = um;
        u.base = const_cast<char*>(modes) + (int64_t)m * mode_bytes;
        C<double> w[12];
        SpinorIO<P64>::load(u, s, w);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = cfma(acc[k], c, w[k]);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = {(R)acc[k].r, (R)acc[k].i};
    SpinorIO<P>::store(out, s, t);
}

// ---- multi-shift CG ------------------------------------------------------------
// Shifted systems (A + sigma_l) x_l = b, A = X^2, solved on the Krylov space of
// the smallest shift sigma_0: the shifted residuals stay collinear,
// r_l = zeta_l r, with
//   zeta_l' = zeta_l zeta_l^- a^- / (a b^- (zeta_l^- - zeta_l) + zeta_l^- a^- (1 + (sigma_l - sigma_0) a)),
//   a_l = a zeta_l'/zeta_l,  b_l = b (zeta_l'/zeta_l)^2,
//   x_l += a_l p_l,  p_l = zeta_l' r + b_l p_l
// (Jegerlehner, hep-lat/9612014).  Only y = sum_l w_l x_l is accumulated.  A
// shift is frozen once |zeta_l| |r| <= tol |b|.

__device__ double block_reduce_partials(const double* partials, int nblocks, double* lds) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partials[b];
    return block_sum(s, lds);
}

__global__ void __launch_bounds__(kBlock) k_ms_init(MsState* st, MsConst k, const double* b2p, int nblk) {
    __shared__ double lds[kBlock / 64];
    const double b2 = block_reduce_partials(b2p, nblk, lds);
    if (threadIdx.x == 0) {
        st->b2 = b2;
        st->rr = b2;
        st->pp = b2;
        st->alpha_prev = 1.0;
        st->beta_prev = 0.0;
        st->iter = 0;
        st->done = (b2 == 0.0);
        st->bad = !isfinite(b2);
        for (int l = 0; l < NDQ_MAX_SHIFTS; ++l) {
            st->zeta[l] = st->zeta_prev[l] = 1.0;
            st->upd_p[l] = l < k.n;
            st->upd_y[l] = 0;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_ms_alpha(MsState* st, MsConst k, const double* ttp, int nblk_tt,
                                                     const double* ppp, int nblk_pp) {
    __shared__ double lds[kBlock / 64];
    const double tt = block_reduce_partials(ttp, nblk_tt, lds);
    __syncthreads();
    double pp = 0.0;
    if (ppp) pp = block_reduce_partials(ppp, nblk_pp, lds);
    if (threadIdx.x != 0) return;
    if (st->done) {
        // converged: leave every vector unchanged until the host notices
        st->c0 = 0.0;
        st->cp = 0.0;
        for (int l = 0; l < k.n; ++l) {
            st->upd_y[l] = 0;
            st->upd_p[l] = 0;
        }
        return;
    }
    if (ppp) st->pp = pp;
    st->tt = tt;
    const double denom = tt * k.inv_lam2 + k.sigma[0] * st->pp;
    const double a = st->rr / denom;
    if (!isfinite(a)) st->bad = 1;
    st->alpha = a;
    for (int l = 0; l < k.n; ++l) {
        if (!st->upd_p[l]) {
            st->upd_y[l] = 0;
            st->ycoef[l] = 0.0;
            continue;
        }
        double zn = 1.0;
        if (l > 0) {
            const double d = k.sigma[l] - k.sigma[0];
            const double den = a * st->beta_prev * (st->zeta_prev[l] - st->zeta[l]) +
                               st->zeta_prev[l] * st->alpha_prev * (1.0 + d * a);
            zn = st->zeta[l] * st->zeta_prev[l] * st->alpha_prev / den;
        }
        st->zeta_new[l] = zn;
        st->ycoef[l] = k.w[l] * a * zn / st->zeta[l];
        st->upd_y[l] = 1;
    }
    st->c0 = -a * k.inv_lam2;
    st->cp = -a * k.sigma[0];
}

__global__ void __launch_bounds__(kBlock) k_ms_beta(MsState* st, MsConst k, const double* rrp, int nblk) {
    __shared__ double lds[kBlock / 64];
    const double rr = block_reduce_partials(rrp, nblk, lds);
    if (threadIdx.x != 0 || st->done) return;
    const double b = rr / st->rr;
    if (!isfinite(b)) st->bad = 1;
    for (int l = 0; l < k.n; ++l) {
        if (!st->upd_y[l]) {
            st->upd_p[l] = 0;
            continue;
        }
        const double q = st->zeta_new[l] / st->zeta[l];
        st->bl[l] = b * q * q;
        st->pcoef[l] = st->zeta_new[l];
        st->zeta_prev[l] = st->zeta[l];
        st->zeta[l] = st->zeta_new[l];
        st->upd_p[l] = st->zeta[l] * st->zeta[l] * rr > k.tol2 * st->b2;
    }
    st->alpha_prev = st->alpha;
    st->beta_prev = b;
    st->rr = rr;
    st->iter += 1;
    st->done = rr <= k.tol2 * st->b2;
}

struct MsUpdArgs {
    SpinorView r, y;
    SpinorView p0;
    int64_t p_bytes;
    int n;
    int32_t nsites;
    const MsState* st;
    double* partials;
};

template <int P>
__global__ void __launch_bounds__(kBlock) k_ms_update(MsUpdArgs a) {
    using R = typename SpinorIO<P>::R;
    __shared__ double lds[kBlock / 64];
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    double red = 0.0;
    if (s < a.nsites) {
        C<R> r[12], y[12];
        SpinorIO<P>::load(a.r, s, r);
        SpinorIO<P>::load(a.y, s, y);
        for (int l = 0; l < a.n; ++l) {
            const int uy = a.st->upd_y[l], up = a.st->upd_p[l];
            if (!uy && !up) continue;
            SpinorView pv = a.p0;
            pv.base += (int64_t)l * a.p_bytes;
            C<R> p[12];
            SpinorIO<P>::load(pv, s, p);
            if (uy) {
                const R c = (R)a.st->ycoef[l];
#pragma unroll
                for (int k = 0; k < 12; ++k) y[k] = {y[k].r + c * p[k].r, y[k].i + c * p[k].i};
            }
            if (up) {
                const R zc = (R)a.st->pcoef[l], bc = (R)a.st->bl[l];
#pragma unroll
                for (int k = 0; k < 12; ++k) p[k] = {zc * r[k].r + bc * p[k].r, zc * r[k].i + bc * p[k].i};
                SpinorIO<P>::store(pv, s, p);
                if (l == 0) {
                    if constexpr (P == P16) SpinorIO<P>::load(pv, s, p);
#pragma unroll
                    for (int k = 0; k < 12; ++k) red += (double)p[k].r * p[k].r + (double)p[k].i * p[k].i;
                }
            }
        }
        SpinorIO<P>::store(a.y, s, y);
    }
    if (a.partials) {
        const double t = block_sum(red, lds);
        if (threadIdx.x == 0) a.partials[blockIdx.x] = t;
    }
}

__global__ void k_mode_coef(const double* c, const double* d, ModeSigns sg, int use_sign, int nev, double sc,
                            double sd, double* coef) {
    const int k = threadIdx.x;
    if (k >= nev) return;
    const double f = sc * (use_sign ? (double)sg.s[k] : 1.0);
    coef[2 * k] = f * c[2 * k] + (d ? sd * d[2 * k] : 0.0);
    coef[2 * k + 1] = f * c[2 * k + 1] + (d ? sd * d[2 * k + 1] : 0.0);
}

// Basis rotation dst_j = sum_i src_i Y[i][j] for the FP64 full spinors of a
// contiguous block (Y complex, row-major nsrc x k, on the device).  One lane
// per (complex component c, site s), sites fastest so that every load is a
// contiguous run of one plane; the outputs come in groups of kRotJ, and the
// groups of one run of lanes are the wavefronts of one workgroup (rot_shape),
// so the source planes they all read leave HBM once.  The sum over i runs in
// index order for every output, as a plain loop would.
constexpr int kRotJ = 16;

// Workgroup shape for ngroups output groups: wpg wavefronts of distinct lanes
// per group (4 wavefronts in all for 1, 2 or 4 groups).
__host__ __device__ inline int rot_wpg(int ngroups) { return ngroups == 1 ? 4 : ngroups == 2 ? 2 : 1; }

__global__ void __launch_bounds__(256) k_rotate(const char* __restrict__ src, int nsrc, const double* __restrict__ Y,
                                                int k, char* __restrict__ dst, int64_t vbytes, SpinorView lay,
                                                int32_t n) {
    const int ng = (k + kRotJ - 1) / kRotJ;
    const int wpg = rot_wpg(ng);
    // wavefront index, wave-uniform: the group's coefficients are then scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t = ((int64_t)blockIdx.x * wpg + wave % wpg) * 64 + (threadIdx.x & 63);
    if (t >= 12 * (int64_t)n) return;
    const int c = (int)(t / n);
    const int32_t s = (int32_t)(t - (int64_t)c * n);
    const int j0 = kRotJ * (wave / wpg);
    const int cnt = min(kRotJ, k - j0);
    C<double> acc[kRotJ];
#pragma unroll
    for (int j = 0; j < kRotJ; ++j) acc[j] = {0.0, 0.0};
    for (int i = 0; i < nsrc; ++i) {
        SpinorView v = lay;
        v.base = const_cast<char*>(src) + (int64_t)i * vbytes;
        const C<double> x = SpinorIO<P64>::load_comp(v, s, c);
        const double* yi = Y + 2 * ((int64_t)i * k + j0);
#pragma unroll
        for (int j = 0; j < kRotJ; ++j)
            if (j < cnt) acc[j] = cfma(acc[j], C<double>{yi[2 * j], yi[2 * j + 1]}, x);
    }
#pragma unroll
    for (int j = 0; j < kRotJ; ++j) {
        if (j < cnt) {
            SpinorView o = lay;
            o.base = dst + (int64_t)(j0 + j) * vbytes;
            SpinorIO<P64>::store_comp(o, s, c, acc[j]);
        }
    }
}

// out = start * exp(i theta) per component, theta = 2 pi u with u from the
// splitmix64 hash of (index, site, component): a deterministic family of
// independent start vectors derived from one (index 0 returns start itself).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(kBlock) k_phase_copy(SpinorView src, SpinorView dst, int idx, int32_t n) {
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    C<double> x[12];
    SpinorIO<P64>::load(src, s, x);
    if (idx > 0) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const uint64_t h = splitmix64(((uint64_t)idx << 40) ^ ((uint64_t)s * 12u + (uint64_t)c));
            const double u = (double)(h >> 11) * 0x1.0p-53;
            double sn, cs;
            sincos(6.283185307179586 * u, &sn, &cs);
            x[c] = cmul(x[c], C<double>{cs, sn});
        }
    }
    SpinorIO<P64>::store(dst, s, x);
}

// ---------------------------------------------------------------------------
// Gram matrix of two blocks of FP64 full spinor fields on the matrix cores:
//   G[i][j] = <A_i, B_j> = sum over sites and the 12 components of conj(A_i) B_j,
// a tall-skinny product (K = 12 V, at most 64 x 64 outputs).  One wavefront
// accumulates a 16-row tile of G against up to four 16-column tiles over a
// contiguous range of sites with v_mfma_f64_16x16x4f64: lane l supplies
// A_{16 ti + l%16} and B_{16 tj + l%16} at site s + l/16, so each instruction
// adds four sites' products; real and imaginary parts take four real products
// (ar br + ai bi, ar bi - ai br).  The accumulator lane l, element r holds
// row 4r + l/16, column l%16.  Per-wavefront partial tiles are summed in a
// fixed order by k_gram_reduce.
typedef double v4d __attribute__((ext_vector_type(4)));

// Component c of field `base` (precision PB, full-field layout with plane stride V) in FP64.
template <int PB>
__device__ __forceinline__ double2 field_comp(const char* base, int32_t V, int c, int32_t site) {
    SpinorView v;
    v.base = const_cast<char*>(base);
    v.stride = V;
    v.site0 = 0;
    v.rhs_bytes = 0;
    const auto x = SpinorIO<PB>::load_comp(v, site, c);
    return make_double2((double)x.r, (double)x.i);
}

// B may be F64, F32 or F16 (PB; converted to FP64 on load); A is FP64.
// A workgroup takes one chunk of sites with one wavefront per 16-row tile of
// G, so the B fields of the chunk are loaded by all its wavefronts at about the
// same time and leave HBM once.
template <int PB>
__global__ void __launch_bounds__(256) k_gram(const char* __restrict__ A, int na, const char* __restrict__ B, int nb,
                                              int64_t vb, int64_t vbB, int32_t V, int32_t sites_per_wave, int nchunks,
                                              double* __restrict__ partials) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x;   // the chunk
    if (wave >= nchunks) return;
    const int ti = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform row tile
    const int t = lane & 15, kk = lane >> 4;
    const int ntj = (nb + 15) / 16;
    const int NI = 16 * ((na + 15) / 16), NJ = 16 * ntj;
    const int32_t s0 = (int32_t)((int64_t)wave * sites_per_wave);
    const int32_t s1 = (int32_t)min((int64_t)V, (int64_t)s0 + sites_per_wave);
    const int ia = ti * 16 + t;
    const bool va = ia < na;
    const char* pa = A + (int64_t)(va ? ia : 0) * vb;
    v4d re[4], im[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        re[q] = v4d{0.0, 0.0, 0.0, 0.0};
        im[q] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    for (int c = 0; c < 12; ++c) {
        const int64_t plane = (int64_t)c * V;
        // several steps' loads in flight at once (each step only adds into
        // the accumulators)
#pragma unroll 4
        for (int32_t s = s0; s < s1; s += 4) {
            const int32_t site = s + kk;
            const bool vs = site < s1;
            double2 a = make_double2(0.0, 0.0);
            if (va && vs) a = reinterpret_cast<const double2*>(pa)[plane + site];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < ntj) {
                    const int jb = q * 16 + t;
                    double2 b = make_double2(0.0, 0.0);
                    if (jb < nb && vs) b = field_comp<PB>(B + (int64_t)jb * vbB, V, c, site);
                    re[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, re[q], 0, 0, 0);
                    re[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, re[q], 0, 0, 0);
                    im[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, im[q], 0, 0, 0);
                    im[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.x, im[q], 0, 0, 0);
                }
            }
        }
    }
    double2* out = reinterpret_cast<double2*>(partials) + (int64_t)wave * NI * NJ;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < ntj) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = ti * 16 + 4 * r + kk;
                const int j = q * 16 + t;
                out[(int64_t)i * NJ + j] = make_double2(re[q][r], im[q][r]);
            }
        }
    }
}

// G[i][j] = sum over the chunks (in a fixed order) of the partial tiles, one
// workgroup per element.
__global__ void __launch_bounds__(kBlock) k_gram_reduce(const double* __restrict__ partials, int na, int nb,
                                                        int nchunks, double* __restrict__ G) {
    __shared__ double lds[kBlock / 64];
    const int e = blockIdx.x;
    const int i = e / nb, j = e - (e / nb) * nb;
    const int NI = 16 * ((na + 15) / 16), NJ = 16 * ((nb + 15) / 16);
    const double2* p = reinterpret_cast<const double2*>(partials);
    double sr = 0.0, si = 0.0;
    for (int w = threadIdx.x; w < nchunks; w += kBlock) {
        const double2 v = p[((int64_t)w * NI + i) * NJ + j];
        sr += v.x;
        si += v.y;
    }
    sr = block_sum(sr, lds);
    __syncthreads();
    si = block_sum(si, lds);
    if (threadIdx.x == 0) {
        G[2 * e] = sr;
        G[2 * e + 1] = si;
    }
}

// Projection coefficients of a block of R fields: coef[k][r] = sc * (use_sign ?
// sign_k : 1) * c[k][r] + sd * d[k][r] (complex, row-major nev x R; d may be null).
__global__ void k_mode_coef_block(const double* c, const double* d, ModeSigns sg, int use_sign, int nev, int nr,
                                  double sc, double sd, double* coef) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nev * nr) return;
    const int k = e / nr;
    const double f = sc * (use_sign ? (double)sg.s[k] : 1.0);
    coef[2 * e] = f * c[2 * e] + (d ? sd * d[2 * e] : 0.0);
    coef[2 * e + 1] = f * c[2 * e + 1] + (d ? sd * d[2 * e + 1] : 0.0);
}

// out_r = in_r + sum_k coef[k][r] u_k for a block of fields (r < nr), one lane
// per (complex component c, site s) with sites fastest, so that every load is
// a contiguous run of one plane (measured faster than pairing the two
// components of an F32 word in one lane or in adjacent lanes, although the
// halves of a word are then stored by different wavefronts).  The fields come
// in groups of kRotJ laid out over the wavefronts of a workgroup as
// in k_rotate, so the mode planes leave HBM once.  The sum runs in the order
// of k_mode_update (start from in, add the modes in index order, FP64).  PI:
// precision of `in` (F64, F32 or F16); PO: precision of `out` (F64 or F32; an
// F16 result goes through an F32 block and k_convert, which rounds exactly as
// k_mode_update<P16> does).
template <int PI, int PO>
__global__ void __launch_bounds__(256) k_mode_update_block(const char* __restrict__ modes, int64_t mode_bytes,
                                                           int nev, const double* __restrict__ coef, int nr,
                                                           SpinorView in, SpinorView out, int32_t n) {
    const int ng = (nr + kRotJ - 1) / kRotJ;
    const int wpg = rot_wpg(ng);
    // wavefront index, wave-uniform: the group's coefficients are then scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t = ((int64_t)blockIdx.x * wpg + wave % wpg) * 64 + (threadIdx.x & 63);
    if (t >= 12 * (int64_t)n) return;
    const int c = (int)(t / n);
    const int32_t s = (int32_t)(t - (int64_t)c * n);
    const int r0 = kRotJ * (wave / wpg);
    const int cnt = min(kRotJ, nr - r0);
    C<double> acc[kRotJ];
#pragma unroll
    for (int j = 0; j < kRotJ; ++j) {
        if (j < cnt) {
            SpinorView v = in;
            v.base += (int64_t)(r0 + j) * in.rhs_bytes;
            const auto x = SpinorIO<PI>::load_comp(v, s, c);
            acc[j] = {(double)x.r, (double)x.i};
        } else {
            acc[j] = {0.0, 0.0};
        }
    }
    for (int k = 0; k < nev; ++k) {
        const double2 w = reinterpret_cast<const double2*>(modes + (int64_t)k * mode_bytes)[(int64_t)c * n + s];
        const double* ck = coef + 2 * ((int64_t)k * nr + r0);
#pragma unroll
        for (int j = 0; j < kRotJ; ++j)
            if (j < cnt) acc[j] = cfma(acc[j], C<double>{ck[2 * j], ck[2 * j + 1]}, C<double>{w.x, w.y});
    }
    using RO = typename SpinorIO<PO>::R;
#pragma unroll
    for (int j = 0; j < kRotJ; ++j) {
        if (j < cnt) {
            SpinorView o = out;
            o.base += (int64_t)(r0 + j) * out.rhs_bytes;
            SpinorIO<PO>::store_comp(o, s, c, C<RO>{(RO)acc[j].r, (RO)acc[j].i});
        }
    }
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

namespace ndq {

int lincomb_blocks(const ndq_geom* g) { return (int)nblocks(g->volume); }

size_t partials_capacity(const ndq_geom* g, int nvals) {
    const int64_t blocks = std::max<int64_t>(nblocks(g->volume), 2 * ((g->vh + 63) / 64));
    return (size_t)blocks * (size_t)std::max(nvals, 1) * sizeof(double);
}

namespace {
int lin_setup(const ndq_geom* g, const ndq_spinor* out, int nv, const ndq_spinor* const* v, const Coef* c,
              const int* g5, double* partials, LinArgs& a) {
    memset(&a, 0, sizeof(a));
    const int nr = out->nrhs;
    a.out = flat_view(g, out);
    a.nv = nv;
    for (int j = 0; j < nv; ++j) {
        if (v[j]->nrhs != nr) return fail(NDQ_EINVAL, "lincomb: operand %d has %d fields, the output %d", j, v[j]->nrhs, nr);
        a.v[j] = flat_view(g, v[j]);
        if (c) a.c[j] = c[j];
        a.g5[j] = g5 ? g5[j] : 0;
    }
    a.nsites = (int32_t)g->volume;
    a.partials = partials;
    return NDQ_OK;
}
}  // namespace

int lincomb(const ndq_geom* g, int prec, const ndq_spinor* out, int nv, const ndq_spinor* const* v, const Coef* c,
            const int* g5, double* partials, hipStream_t st) {
    LinArgs a;
    int rc = lin_setup(g, out, nv, v, c, g5, partials, a);
    if (rc) return rc;
    const dim3 grid(nblocks(g->volume), out->nrhs);
    switch (prec) {
        case NDQ_F64: hipLaunchKernelGGL(k_lincomb<P64>, grid, dim3(kBlock), 0, st, a); break;
        case NDQ_F32: hipLaunchKernelGGL(k_lincomb<P32>, grid, dim3(kBlock), 0, st, a); break;
        default: hipLaunchKernelGGL(k_lincomb<P16>, grid, dim3(kBlock), 0, st, a); break;
    }
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int lincomb_rhs(const ndq_geom* g, int prec, const ndq_spinor* out, int nv, const ndq_spinor* const* v,
                const double* cr, const int* g5, double* partials, hipStream_t st) {
    if (out->nrhs > NDQ_MAX_BATCH) return fail(NDQ_EINVAL, "lincomb: at most %d fields per block", NDQ_MAX_BATCH);
    LinArgs a;
    int rc = lin_setup(g, out, nv, v, nullptr, g5, partials, a);
    if (rc) return rc;
    LinRhs b;
    memset(&b, 0, sizeof(b));
    for (int j = 0; j < nv; ++j)
        for (int r = 0; r < out->nrhs; ++r) b.c[j][r] = cr[j * out->nrhs + r];
    const dim3 grid(nblocks(g->volume), out->nrhs);
    switch (prec) {
        case NDQ_F64: hipLaunchKernelGGL(k_lincomb_rhs<P64>, grid, dim3(kBlock), 0, st, a, b); break;
        case NDQ_F32: hipLaunchKernelGGL(k_lincomb_rhs<P32>, grid, dim3(kBlock), 0, st, a, b); break;
        default: hipLaunchKernelGGL(k_lincomb_rhs<P16>, grid, dim3(kBlock), 0, st, a, b); break;
    }
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int reduce_partials(const double* partials, int nb, int nvals, double* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(nvals), dim3(kBlock), 0, st, partials, nb, (int64_t)1, nvals, dst);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int reduce_rows(const double* partials, int nb, int nvals, double* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(nvals), dim3(kBlock), 0, st, partials, nb, (int64_t)nb, 1, dst);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int dot(const ndq_geom* g, const ndq_spinor* x, const ndq_spinor* y, double* partials, double* dst, hipStream_t st) {
    if (y && y->nrhs != x->nrhs) return fail(NDQ_EINVAL, "dot: operands with %d and %d fields", x->nrhs, y->nrhs);
    const SpinorView xv = flat_view(g, x);
    const SpinorView yv = y ? flat_view(g, y) : xv;
    const int32_t n = (int32_t)g->volume;
    const dim3 grid(nblocks(n), x->nrhs);
    const int hy = y != nullptr;
    switch (x->prec) {
        case NDQ_F64: hipLaunchKernelGGL(k_dot<P64>, grid, dim3(kBlock), 0, st, xv, yv, hy, n, partials); break;
        case NDQ_F32: hipLaunchKernelGGL(k_dot<P32>, grid, dim3(kBlock), 0, st, xv, yv, hy, n, partials); break;
        default: hipLaunchKernelGGL(k_dot<P16>, grid, dim3(kBlock), 0, st, xv, yv, hy, n, partials); break;
    }
    NDQ_HIP(hipGetLastError());
    return reduce_rows(partials, (int)grid.x, (hy ? 2 : 1) * x->nrhs, dst, st);
}

int convert(const ndq_geom* g, const ndq_spinor* dst, const ndq_spinor* src, hipStream_t st) {
    if (dst->nrhs != src->nrhs) return fail(NDQ_EINVAL, "convert: %d fields into %d", src->nrhs, dst->nrhs);
    const SpinorView d = flat_view(g, dst), s = flat_view(g, src);
    const int32_t n = (int32_t)g->volume;
    const dim3 grid(nblocks(n), dst->nrhs);
    const int key = dst->prec * 3 + src->prec;
    switch (key) {
        case NDQ_F64 * 3 + NDQ_F64: hipLaunchKernelGGL((k_convert<P64, P64>), grid, dim3(kBlock), 0, st, d, s, n); break;
        case NDQ_F64 * 3 + NDQ_F32: hipLaunchKernelGGL((k_convert<P64, P32>), grid, dim3(kBlock), 0, st, d, s, n); break;
        case NDQ_F64 * 3 + NDQ_F16: hipLaunchKernelGGL((k_convert<P64, P16>), grid, dim3(kBlock), 0, st, d, s, n); break;
        case NDQ_F32 * 3 + NDQ_F64: hipLaunchKernelGGL((k_convert<P32, P64>), grid, dim3(kBlock), 0, st, d, s, n); break;
        case NDQ_F32 * 3 + NDQ_F32: hipLaunchKernelGGL((k_convert<P32, P32>), grid, dim3(kBlock), 0, st, d, s, n); break;
        case NDQ_F32 * 3 + NDQ_F16: hipLaunchKernelGGL((k_convert<P32, P16>), grid, dim3(kBlock), 0, st, d, s, n); break;
        case NDQ_F16 * 3 + NDQ_F64: hipLaunchKernelGGL((k_convert<P16, P64>), grid, dim3(kBlock), 0, st, d, s, n); break;
        case NDQ_F16 * 3 + NDQ_F32: hipLaunchKernelGGL((k_convert<P16, P32>), grid, dim3(kBlock), 0, st, d, s, n); break;
        default: hipLaunchKernelGGL((k_convert<P16, P16>), grid, dim3(kBlock), 0, st, d, s, n); break;
    }
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

namespace {
// Site chunks of the Gram kernel: enough workgroups to fill the device, at
// least 64 sites each, and at most 32 MiB of partial tiles.
int gram_chunks(const ndq_geom* g, int na, int nb) {
    const int64_t tile = (int64_t)16 * ((na + 15) / 16) * 16 * ((nb + 15) / 16) * 2 * sizeof(double);
    const int64_t cap = std::max<int64_t>(1, (int64_t(32) << 20) / tile);
    return (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(4096, cap), (g->volume + 63) / 64));
}
}  // namespace

size_t gram_partials_bytes(const ndq_geom* g, int na, int nb) {
    const int NI = 16 * ((na + 15) / 16), NJ = 16 * ((nb + 15) / 16);
    return (size_t)gram_chunks(g, na, nb) * NI * NJ * 2 * sizeof(double);
}

int gram(const ndq_geom* g, const void* A, int na, const void* B, int nb, double* partials, double* G,
         hipStream_t st) {
    if (na < 1 || nb < 1 || na > 64 || nb > 64) return fail(NDQ_EINVAL, "gram: block sizes must be in [1, 64]");
    const int nw = gram_chunks(g, na, nb);
    const int64_t V = g->volume;
    int32_t spw = (int32_t)((V + nw - 1) / nw);
    spw = (spw + 3) & ~3;
    const int64_t vb = spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL);
    const dim3 block(64 * ((na + 15) / 16));
    hipLaunchKernelGGL(k_gram<P64>, dim3(nw), block, 0, st, static_cast<const char*>(A), na, static_cast<const char*>(B),
                       nb, vb, vb, (int32_t)V, spw, nw, partials);
    NDQ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gram_reduce, dim3(na * nb), dim3(kBlock), 0, st, partials, na, nb, nw, G);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int mode_dots(const ndq_geom* g, const void* modes, int nev, const ndq_spinor* v, double* partials, double* dots,
              hipStream_t st) {
    if (nev <= 0) return NDQ_OK;
    const int32_t n = (int32_t)g->volume;
    const dim3 grid(nblocks(n));
    const SpinorView vv = flat_view(g, v);
    ndq_spinor um_desc = {const_cast<void*>(modes), NDQ_F64, NDQ_FULL, 1};
    const SpinorView um = flat_view(g, &um_desc);
    const int64_t mb = spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL);
    const char* mp = static_cast<const char*>(modes);
    switch (v->prec) {
        case NDQ_F64: hipLaunchKernelGGL(k_mode_dots<P64>, grid, dim3(kBlock), 0, st, mp, mb, nev, vv, um, n, partials); break;
        case NDQ_F32: hipLaunchKernelGGL(k_mode_dots<P32>, grid, dim3(kBlock), 0, st, mp, mb, nev, vv, um, n, partials); break;
        default: hipLaunchKernelGGL(k_mode_dots<P16>, grid, dim3(kBlock), 0, st, mp, mb, nev, vv, um, n, partials); break;
    }
    NDQ_HIP(hipGetLastError());
    return reduce_partials(partials, (int)grid.x, 2 * nev, dots, st);
}

int mode_update(const ndq_geom* g, const void* modes, int nev, const double* coef, const ndq_spinor* in,
                const ndq_spinor* out, hipStream_t st) {
    const int32_t n = (int32_t)g->volume;
    const dim3 grid(nblocks(n));
    const SpinorView iv = flat_view(g, in), ov = flat_view(g, out);
    ndq_spinor um_desc = {const_cast<void*>(modes), NDQ_F64, NDQ_FULL, 1};
    const SpinorView um = flat_view(g, &um_desc);
    const int64_t mb = spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL);
    const char* mp = static_cast<const char*>(modes);
    switch (in->prec) {
        case NDQ_F64: hipLaunchKernelGGL(k_mode_update<P64>, grid, dim3(kBlock), 0, st, mp, mb, nev, coef, iv, ov, um, n); break;
        case NDQ_F32: hipLaunchKernelGGL(k_mode_update<P32>, grid, dim3(kBlock), 0, st, mp, mb, nev, coef, iv, ov, um, n); break;
        default: hipLaunchKernelGGL(k_mode_update<P16>, grid, dim3(kBlock), 0, st, mp, mb, nev, coef, iv, ov, um, n); break;
    }
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int mode_coef(const double* c, const double* d, const ModeSigns& sg, int use_sign, int nev, double sc, double sd,
              double* coef, hipStream_t st) {
    hipLaunchKernelGGL(k_mode_coef, dim3(1), dim3(NDQ_MAX_MODES), 0, st, c, d, sg, use_sign, nev, sc, sd, coef);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int gram_block(const ndq_geom* g, const void* A, int na, const ndq_spinor* B, double* partials, double* G,
               hipStream_t st) {
    const int nb = B->nrhs;
    if (na < 1 || nb < 1 || na > 64 || nb > 64) return fail(NDQ_EINVAL, "gram: block sizes must be in [1, 64]");
    const int nw = gram_chunks(g, na, nb);
    const int64_t V = g->volume;
    int32_t spw = (int32_t)((V + nw - 1) / nw);
    spw = (spw + 3) & ~3;
    const int64_t vb = spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL);
    const int64_t vbB = spinor_rhs_bytes(g, B->prec, NDQ_FULL);
    const dim3 grid(nw), blk(64 * ((na + 15) / 16));
    const char* a = static_cast<const char*>(A);
    const char* b = static_cast<const char*>(B->data);
    switch (B->prec) {
        case NDQ_F64: hipLaunchKernelGGL(k_gram<P64>, grid, blk, 0, st, a, na, b, nb, vb, vbB, (int32_t)V, spw, nw, partials); break;
        case NDQ_F32: hipLaunchKernelGGL(k_gram<P32>, grid, blk, 0, st, a, na, b, nb, vb, vbB, (int32_t)V, spw, nw, partials); break;
        default: hipLaunchKernelGGL(k_gram<P16>, grid, blk, 0, st, a, na, b, nb, vb, vbB, (int32_t)V, spw, nw, partials); break;
    }
    NDQ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gram_reduce, dim3(na * nb), dim3(kBlock), 0, st, partials, na, nb, nw, G);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int mode_coef_block(const double* c, const double* d, const ModeSigns& sg, int use_sign, int nev, int nr, double sc,
                    double sd, double* coef, hipStream_t st) {
    hipLaunchKernelGGL(k_mode_coef_block, dim3(nblocks((int64_t)nev * nr)), dim3(kBlock), 0, st, c, d, sg, use_sign,
                       nev, nr, sc, sd, coef);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int mode_update_block(const ndq_geom* g, const void* modes, int nev, const double* coef, const ndq_spinor* in,
                      const ndq_spinor* out, hipStream_t st) {
    const int nr = in->nrhs;
    if (out->nrhs != nr) return fail(NDQ_EINVAL, "mode update: %d fields into %d", nr, out->nrhs);
    if (out->prec == NDQ_F16) return fail(NDQ_EPREC, "mode update: the block form writes F64 or F32 fields");
    const SpinorView iv = flat_view(g, in), ov = flat_view(g, out);
    const int64_t mb = spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL);
    const char* mp = static_cast<const char*>(modes);
    const int ng = (nr + kRotJ - 1) / kRotJ;
    const int wpg = rot_wpg(ng);
    const int64_t lanes = 12 * (int64_t)g->volume;
    const dim3 grid((unsigned)((lanes + 64 * wpg - 1) / (64 * wpg)));
    const dim3 blk(64 * wpg * ng);
    const int32_t n = (int32_t)g->volume;
    if (ng * wpg > 4) return fail(NDQ_EINVAL, "mode update: at most 64 fields per block");
    const int key = in->prec * 3 + out->prec;
    switch (key) {
        case NDQ_F64 * 3 + NDQ_F64: hipLaunchKernelGGL((k_mode_update_block<P64, P64>), grid, blk, 0, st, mp, mb, nev, coef, nr, iv, ov, n); break;
        case NDQ_F32 * 3 + NDQ_F32: hipLaunchKernelGGL((k_mode_update_block<P32, P32>), grid, blk, 0, st, mp, mb, nev, coef, nr, iv, ov, n); break;
        case NDQ_F16 * 3 + NDQ_F32: hipLaunchKernelGGL((k_mode_update_block<P16, P32>), grid, blk, 0, st, mp, mb, nev, coef, nr, iv, ov, n); break;
        default: return fail(NDQ_EPREC, "mode update: unsupported precision pair (%d -> %d)", in->prec, out->prec);
    }
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int phase_copy(const ndq_geom* g, const ndq_spinor* src, const ndq_spinor* dst, int idx, hipStream_t st) {
    hipLaunchKernelGGL(k_phase_copy, dim3(nblocks(g->volume)), dim3(kBlock), 0, st, flat_view(g, src),
                       flat_view(g, dst), idx, (int32_t)g->volume);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int rotate(const ndq_geom* g, const void* src, int nsrc, const double* Y, int k, void* dst, hipStream_t st) {
    ndq_spinor d = {const_cast<void*>(src), NDQ_F64, NDQ_FULL, 1};
    const SpinorView lay = flat_view(g, &d);
    const int64_t vb = spinor_rhs_bytes(g, NDQ_F64, NDQ_FULL);
    const int ng = (k + kRotJ - 1) / kRotJ;
    if (ng > 4) return fail(NDQ_EINVAL, "rotate: at most 64 outputs");
    const int wpg = rot_wpg(ng);
    const int64_t lanes = 12 * (int64_t)g->volume;
    const dim3 grid((unsigned)((lanes + 64 * wpg - 1) / (64 * wpg)));
    hipLaunchKernelGGL(k_rotate, grid, dim3(64 * wpg * ng), 0, st, static_cast<const char*>(src), nsrc, Y, k,
                       static_cast<char*>(dst), vb, lay, (int32_t)g->volume);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int ms_init(MsState* s, const MsConst& k, const double* b2p, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_ms_init, dim3(1), dim3(kBlock), 0, st, s, k, b2p, nblk);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int ms_alpha(MsState* s, const MsConst& k, const double* ttp, int nblk_tt, const double* ppp, int nblk_pp,
             hipStream_t st) {
    hipLaunchKernelGGL(k_ms_alpha, dim3(1), dim3(kBlock), 0, st, s, k, ttp, nblk_tt, ppp, nblk_pp);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int ms_beta(MsState* s, const MsConst& k, const double* rrp, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_ms_beta, dim3(1), dim3(kBlock), 0, st, s, k, rrp, nblk);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int ms_update(const ndq_geom* g, int prec, MsState* s, const MsConst& k, const ndq_spinor* r, const ndq_spinor* y,
              const ndq_spinor* p, double* partials, hipStream_t st) {
    MsUpdArgs a;
    a.r = flat_view(g, r);
    a.y = flat_view(g, y);
    a.p0 = flat_view(g, p);
    a.p_bytes = spinor_rhs_bytes(g, prec, NDQ_FULL);
    a.n = k.n;
    a.nsites = (int32_t)g->volume;
    a.st = s;
    a.partials = partials;
    const dim3 grid(nblocks(g->volume));
    switch (prec) {
        case NDQ_F64: hipLaunchKernelGGL(k_ms_update<P64>, grid, dim3(kBlock), 0, st, a); break;
        case NDQ_F32: hipLaunchKernelGGL(k_ms_update<P32>, grid, dim3(kBlock), 0, st, a); break;
        default: hipLaunchKernelGGL(k_ms_update<P16>, grid, dim3(kBlock), 0, st, a); break;
    }
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

}  // namespace ndq

extern "C" size_t ndq_gram_workspace_bytes(const ndq_geom* g, int na, int nb) {
    if (!g || na < 1 || nb < 1 || na > 64 || nb > 64) return 0;
    return ndq::gram_partials_bytes(g, na, nb);
}

extern "C" int ndq_spinor_gram(const ndq_geom* g, const ndq_spinor* A, const ndq_spinor* B, void* d_G, void* ws,
                               size_t ws_bytes, void* stream) {
    using namespace ndq;
    if (!g || !d_G) return fail(NDQ_EINVAL, "ndq_spinor_gram: NULL argument");
    int rc = check_spinor(g, A, NDQ_FULL, "ndq_spinor_gram A");
    if (!rc) rc = check_spinor(g, B, NDQ_FULL, "ndq_spinor_gram B");
    if (rc) return rc;
    if (A->prec != NDQ_F64 || B->prec != NDQ_F64) return fail(NDQ_EPREC, "ndq_spinor_gram: F64 fields");
    if (A->nrhs > 64 || B->nrhs > 64) return fail(NDQ_EINVAL, "ndq_spinor_gram: at most 64 fields per block");
    const size_t need = gram_partials_bytes(g, A->nrhs, B->nrhs);
    if (!ws || ws_bytes < need) return fail(NDQ_ENOMEM, "ndq_spinor_gram: workspace too small (need %zu bytes)", need);
    return gram(g, A->data, A->nrhs, B->data, B->nrhs, static_cast<double*>(ws), static_cast<double*>(d_G),
                as_stream(stream));
}
