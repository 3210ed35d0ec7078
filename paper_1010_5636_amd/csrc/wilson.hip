// The Wilson-Dirac stencil (Sec. 2.1, Eq. 1 and Eq. 2) for gfx950.
//
// One lane per output site (the paper's one-thread-per-site gather, no
// inter-lane communication).  Per direction the neighbour spinor is projected
// onto the two-spin half spinor of (1 -+ gamma_mu), the link (decoded from
// 18/12/8 stored reals in registers) multiplies the two colour vectors, and
// the lower spin components are rebuilt by the fixed spin map of the chiral
// representation.  Accumulation is in registers; the epilogue forms
//
//   t   = G5? [ a * self + b * (H in) ]
//   out = c0 * t + c1 * v1 + c2 * v2 + c3 * v3        (c_k may be device scalars)
//
// and optionally adds |out|^2 (FP64) into per-block partial sums.
// Chiral basis: gamma_mu = [[0, A_mu], [A_mu^H, 0]], A_0 = -1, A_k = -i sigma_k,
// so (1 - gamma_mu) psi = (h, -A^H h) with h = psi_up - A psi_dn, and
// (1 + gamma_mu) psi = (g, A^H g) with g = psi_up + A psi_dn.
#include <string.h>

#include <algorithm>
#include <atomic>

#include "wilson.h"

using namespace ndq;

namespace {

// spin s, colour c -> component index 3*s + c
template <int MU, typename R>
__device__ __forceinline__ void hop_fwd(const C<R> s[12], const C<R> u[3][3], C<R> acc[12]) {
    C<R> h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if constexpr (MU == 0) {
            h0[c] = cadd(s[c], s[6 + c]);
            h1[c] = cadd(s[3 + c], s[9 + c]);
        } else if constexpr (MU == 1) {
            h0[c] = cadd(s[c], cmuli(s[9 + c]));
            h1[c] = cadd(s[3 + c], cmuli(s[6 + c]));
        } else if constexpr (MU == 2) {
            h0[c] = cadd(s[c], s[9 + c]);
            h1[c] = csub(s[3 + c], s[6 + c]);
        } else {
            h0[c] = cadd(s[c], cmuli(s[6 + c]));
            h1[c] = csub(s[3 + c], cmuli(s[9 + c]));
        }
    }
    C<R> w0[3], w1[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        w0[r] = cmul(u[r][0], h0[0]);
        w1[r] = cmul(u[r][0], h1[0]);
        w0[r] = cfma(w0[r], u[r][1], h0[1]);
        w1[r] = cfma(w1[r], u[r][1], h1[1]);
        w0[r] = cfma(w0[r], u[r][2], h0[2]);
        w1[r] = cfma(w1[r], u[r][2], h1[2]);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        acc[r] = cadd(acc[r], w0[r]);
        acc[3 + r] = cadd(acc[3 + r], w1[r]);
        if constexpr (MU == 0) {
            acc[6 + r] = cadd(acc[6 + r], w0[r]);
            acc[9 + r] = cadd(acc[9 + r], w1[r]);
        } else if constexpr (MU == 1) {
            acc[6 + r] = cadd(acc[6 + r], cmulmi(w1[r]));
            acc[9 + r] = cadd(acc[9 + r], cmulmi(w0[r]));
        } else if constexpr (MU == 2) {
            acc[6 + r] = csub(acc[6 + r], w1[r]);
            acc[9 + r] = cadd(acc[9 + r], w0[r]);
        } else {
            acc[6 + r] = cadd(acc[6 + r], cmulmi(w0[r]));
            acc[9 + r] = cadd(acc[9 + r], cmuli(w1[r]));
        }
    }
}

template <int MU, typename R>
__device__ __forceinline__ void hop_bwd(const C<R> s[12], const C<R> u[3][3], C<R> acc[12]) {
    C<R> g0[3], g1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if constexpr (MU == 0) {
            g0[c] = csub(s[c], s[6 + c]);
            g1[c] = csub(s[3 + c], s[9 + c]);
        } else if constexpr (MU == 1) {
            g0[c] = csub(s[c], cmuli(s[9 + c]));
            g1[c] = csub(s[3 + c], cmuli(s[6 + c]));
        } else if constexpr (MU == 2) {
            g0[c] = csub(s[c], s[9 + c]);
            g1[c] = cadd(s[3 + c], s[6 + c]);
        } else {
            g0[c] = csub(s[c], cmuli(s[6 + c]));
            g1[c] = cadd(s[3 + c], cmuli(s[9 + c]));
        }
    }
    // w = U^H g
    C<R> w0[3], w1[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        w0[r] = cmulc(u[0][r], g0[0]);
        w1[r] = cmulc(u[0][r], g1[0]);
        w0[r] = cfmac(w0[r], u[1][r], g0[1]);
        w1[r] = cfmac(w1[r], u[1][r], g1[1]);
        w0[r] = cfmac(w0[r], u[2][r], g0[2]);
        w1[r] = cfmac(w1[r], u[2][r], g1[2]);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        acc[r] = cadd(acc[r], w0[r]);
        acc[3 + r] = cadd(acc[3 + r], w1[r]);
        if constexpr (MU == 0) {
            acc[6 + r] = csub(acc[6 + r], w0[r]);
            acc[9 + r] = csub(acc[9 + r], w1[r]);
        } else if constexpr (MU == 1) {
            acc[6 + r] = cadd(acc[6 + r], cmuli(w1[r]));
            acc[9 + r] = cadd(acc[9 + r], cmuli(w0[r]));
        } else if constexpr (MU == 2) {
            acc[6 + r] = cadd(acc[6 + r], w1[r]);
            acc[9 + r] = csub(acc[9 + r], w0[r]);
        } else {
            acc[6 + r] = cadd(acc[6 + r], cmuli(w0[r]));
            acc[9 + r] = cadd(acc[9 + r], cmulmi(w1[r]));
        }
    }
}

// PAIR64: FP64 also issues both hops' loads together (the direction split with
// 12- or 8-real links, where the registers this takes keep 3 wavefronts per SIMD).
template <int SP, int LP, int RECON, int MU, bool NT, bool PAIR64 = false>
__device__ __forceinline__ void hop_pair(const WilsonArgs& a, int p, int32_t i, const int32_t nb[8],
                                         const SpinorView& vin, C<typename SpinorIO<SP>::R> acc[12]) {
    using R = typename SpinorIO<SP>::R;
    using F = LinkFmt<LP, RECON>;
    C<R> sf[12], sb[12];
    uint32_t wf[F::kWords], wb[F::kWords];
    C<typename LinkReal<LP>::R> u[3][3];
    if constexpr (SP != P64 || PAIR64) {
        // all loads of both hops first: one memory round trip instead of two
        // (FP64 otherwise keeps the two trips: its registers would cut the occupancy)
        SpinorIO<SP>::load(vin, (int64_t)vin.site0 + nb[MU], sf);
        link_load_words<LP, RECON, NT>(a.links, a.g.vh, p * 4 + MU, i, wf);
        SpinorIO<SP>::load(vin, (int64_t)vin.site0 + nb[4 + MU], sb);
        link_load_words<LP, RECON, NT>(a.links, a.g.vh, (1 - p) * 4 + MU, nb[4 + MU], wb);
        __builtin_amdgcn_sched_barrier(0);   // keep the arithmetic below every load
        link_decode<LP, RECON>(wf, u);
        hop_fwd<MU>(sf, u, acc);
        link_decode<LP, RECON>(wb, u);
        hop_bwd<MU>(sb, u, acc);
    } else {
        SpinorIO<SP>::load(vin, (int64_t)vin.site0 + nb[MU], sf);
        link_load_words<LP, RECON, NT>(a.links, a.g.vh, p * 4 + MU, i, wf);
        link_decode<LP, RECON>(wf, u);
        hop_fwd<MU>(sf, u, acc);
        SpinorIO<SP>::load(vin, (int64_t)vin.site0 + nb[4 + MU], sb);
        link_load_words<LP, RECON, NT>(a.links, a.g.vh, (1 - p) * 4 + MU, nb[4 + MU], wb);
        link_decode<LP, RECON>(wb, u);
        hop_bwd<MU>(sb, u, acc);
    }
}

__device__ __forceinline__ double coef(const Coef& c) { return c.d ? c.f * (*c.d) : c.f; }

// Tile order for cache reuse of the neighbour spinors.  In index order the
// tiles holding the x0 neighbours of a tile lie a whole x0 slice (S tiles)
// away, too far back for that slice's spinors to still be in L2.  With chunk c
// (c divides S) the position p of a launch is mapped to the tile
//   x0 = (p mod c N0) / c,  j = (p / c N0) c + p mod c,  tile = x0 S + j,
// i.e. c consecutive tiles of every x0 slice in turn: x0 neighbours are then c
// positions apart and x1 neighbours (s1 / tile sites apart) mostly inside the
// same chunk.  A permutation of the tiles: the arithmetic is unchanged.
__device__ __forceinline__ int32_t order_tile(int32_t p, int32_t nbx, int n0, int c) {
    if (c <= 0) return p;
    const int32_t S = nbx / n0;
    const int32_t cn = c * n0;
    const int32_t k = p / cn;
    const int32_t rem = p - k * cn;
    const int32_t x0 = rem / c;
    return x0 * S + k * c + (rem - x0 * c);
}

// Block index remap that gives each of the 8 XCDs (workgroups dispatched
// round-robin, linear id mod 8) one contiguous range of tiles, so that
// neighbour re-reads stay in that XCD's L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned lin, unsigned total) {
    const unsigned x = lin & 7u;
    const unsigned q = total >> 3, r = total & 7u;
    const unsigned start = x * q + (x < r ? x : r);
    return start + (lin >> 3);
}

// Launch position -> (parity slot y, position within that parity).  With both
// parities in one launch (the full Q) the two parities of a tile take adjacent
// positions, so after the XCD remap they run on the same XCD at about the same
// time: the links one parity reads as forward links the other reads as backward
// links, and the second read finds them in that XCD's L2.  The position is then
// mapped to a tile by order_tile.
__device__ __forceinline__ int32_t parity_slot(unsigned lin, int& y) {
    if (gridDim.y == 2) {
        y = (int)(lin & 1u);
        return (int32_t)(lin >> 1);
    }
    y = (int)(lin / gridDim.x);
    return (int32_t)(lin - (unsigned)y * gridDim.x);
}

template <int SP, int LP, int RECON, int BLOCK, bool NT>
__global__ void __launch_bounds__(BLOCK) k_wilson(WilsonArgs a) {
    using R = typename SpinorIO<SP>::R;
    __shared__ double red_lds[BLOCK / 64];
    unsigned lin = blockIdx.y * gridDim.x + blockIdx.x;
    if (a.xcd_remap) lin = xcd_remap(lin, gridDim.x * gridDim.y);
    int y;
    const int32_t pos = parity_slot(lin, y);
    const int32_t i = order_tile(pos, (int32_t)gridDim.x, a.g.n0, a.order_c) * BLOCK + threadIdx.x;
    const int p = a.p0 + y;
    double red = 0.0;
    if (i < a.g.vh) {
        const SiteCoord x = eo_coords(a.g, p, i);
        int32_t nb[8];
        eo_neighbours(a.g, i, x, nb);
        C<R> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
        const SpinorView& vin = a.in[y];
        hop_pair<SP, LP, RECON, 0, NT>(a, p, i, nb, vin, acc);
        hop_pair<SP, LP, RECON, 1, NT>(a, p, i, nb, vin, acc);
        hop_pair<SP, LP, RECON, 2, NT>(a, p, i, nb, vin, acc);
        hop_pair<SP, LP, RECON, 3, NT>(a, p, i, nb, vin, acc);

        const R b = (R)a.b_hop;
        if (a.has_self) {
            C<R> sf[12];
            SpinorIO<SP>::load(a.self[y], (int64_t)a.self[y].site0 + i, sf);
            const R as = (R)a.a_self;
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = {as * sf[k].r + b * acc[k].r, as * sf[k].i + b * acc[k].i};
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = cscale(b, acc[k]);
        }
        if (a.gamma5) {
#pragma unroll
            for (int k = 6; k < 12; ++k) acc[k] = cneg(acc[k]);
        }
        const R c0 = (R)coef(a.c0);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = cscale(c0, acc[k]);
        for (int j = 0; j < a.nv; ++j) {
            C<R> vv[12];
            SpinorIO<SP>::load(a.v[j][y], (int64_t)a.v[j][y].site0 + i, vv);
            const R cj = (R)coef(a.cv[j]);
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = {acc[k].r + cj * vv[k].r, acc[k].i + cj * vv[k].i};
        }
        SpinorIO<SP>::store(a.out[y], (int64_t)a.out[y].site0 + i, acc);
        if (a.partials) {
            if constexpr (SP == P16) {
                // norm of what was stored (after F16 rounding)
                SpinorIO<SP>::load(a.out[y], (int64_t)a.out[y].site0 + i, acc);
            }
#pragma unroll
            for (int k = 0; k < 12; ++k) red += (double)acc[k].r * acc[k].r + (double)acc[k].i * acc[k].i;
        }
    }
    if (a.partials) {
        const double s = block_sum(red, red_lds);
        if (threadIdx.x == 0) a.partials[lin] = s;
    }
}

// Direction-split variant for small lattices, where one lane per site leaves
// most SIMDs with a single wavefront: a workgroup of 4 wavefronts covers 64
// sites and wavefront w computes the two hops +-mu with mu = w (the direction is
// uniform per wavefront, so there is no divergence).  The four partial sums
// meet in LDS and are added in a fixed order; wavefront w then finishes spin
// component w of the 64 outputs.  For F16 outputs wavefront 0 finishes the
// whole spinor, because the per-site scale needs all 24 reals.
template <int SP, int LP, int RECON, bool NT>
__global__ void __launch_bounds__(256) k_wilson_dirsplit(WilsonArgs a) {
    using R = typename SpinorIO<SP>::R;
    __shared__ C<R> part[4][12][64];
    __shared__ double red_lds[4];
    unsigned lin = blockIdx.y * gridDim.x + blockIdx.x;
    if (a.xcd_remap) lin = xcd_remap(lin, gridDim.x * gridDim.y);
    int y;
    const int32_t pos = parity_slot(lin, y);
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int32_t i = order_tile(pos, (int32_t)gridDim.x, a.g.n0, a.order_c) * 64 + lane;
    const int p = a.p0 + y;
    const bool active = i < a.g.vh;
    if (active) {
        const SiteCoord x = eo_coords(a.g, p, i);
        int32_t nb[8];
        eo_neighbours(a.g, i, x, nb);
        C<R> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
        const SpinorView& vin = a.in[y];
        switch (w) {
            case 0: hop_pair<SP, LP, RECON, 0, NT, RECON != 18>(a, p, i, nb, vin, acc); break;
            case 1: hop_pair<SP, LP, RECON, 1, NT, RECON != 18>(a, p, i, nb, vin, acc); break;
            case 2: hop_pair<SP, LP, RECON, 2, NT, RECON != 18>(a, p, i, nb, vin, acc); break;
            default: hop_pair<SP, LP, RECON, 3, NT, RECON != 18>(a, p, i, nb, vin, acc); break;
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) part[w][k][lane] = acc[k];
    }
    __syncthreads();
    double red = 0.0;
    if (active) {
        const R b = (R)a.b_hop;
        const R as = (R)a.a_self;
        const R c0 = (R)coef(a.c0);
        if constexpr (SP == P16) {
            if (w == 0) {
                C<R> t[12];
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    t[k] = cadd(cadd(part[0][k][lane], part[1][k][lane]), cadd(part[2][k][lane], part[3][k][lane]));
                if (a.has_self) {
                    C<R> sf[12];
                    SpinorIO<SP>::load(a.self[y], (int64_t)a.self[y].site0 + i, sf);
#pragma unroll
                    for (int k = 0; k < 12; ++k) t[k] = {as * sf[k].r + b * t[k].r, as * sf[k].i + b * t[k].i};
                } else {
#pragma unroll
                    for (int k = 0; k < 12; ++k) t[k] = cscale(b, t[k]);
                }
                if (a.gamma5) {
#pragma unroll
                    for (int k = 6; k < 12; ++k) t[k] = cneg(t[k]);
                }
#pragma unroll
                for (int k = 0; k < 12; ++k) t[k] = cscale(c0, t[k]);
                for (int j = 0; j < a.nv; ++j) {
                    C<R> vv[12];
                    SpinorIO<SP>::load(a.v[j][y], (int64_t)a.v[j][y].site0 + i, vv);
                    const R cj = (R)coef(a.cv[j]);
#pragma unroll
                    for (int k = 0; k < 12; ++k) t[k] = {t[k].r + cj * vv[k].r, t[k].i + cj * vv[k].i};
                }
                SpinorIO<SP>::store(a.out[y], (int64_t)a.out[y].site0 + i, t);
                if (a.partials) {
                    SpinorIO<SP>::load(a.out[y], (int64_t)a.out[y].site0 + i, t);
#pragma unroll
                    for (int k = 0; k < 12; ++k) red += (double)t[k].r * t[k].r + (double)t[k].i * t[k].i;
                }
            }
        } else {
            const int64_t so = (int64_t)a.out[y].site0 + i;
            if constexpr (SP == P32) {
                // wavefronts 0..2 finish the two 16-byte planes 2w, 2w+1 each
                // (components 4w..4w+3), so that every store is a full word
                if (w < 3) {
                    C<R> t4[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int c = 4 * w + k;
                        C<R> t = cadd(cadd(part[0][c][lane], part[1][c][lane]),
                                      cadd(part[2][c][lane], part[3][c][lane]));
                        if (a.has_self) {
                            const C<R> sf = SpinorIO<SP>::load_comp(a.self[y], (int64_t)a.self[y].site0 + i, c);
                            t = {as * sf.r + b * t.r, as * sf.i + b * t.i};
                        } else {
                            t = cscale(b, t);
                        }
                        if (a.gamma5 && c >= 6) t = cneg(t);
                        t = cscale(c0, t);
                        for (int j = 0; j < a.nv; ++j) {
                            const C<R> vv = SpinorIO<SP>::load_comp(a.v[j][y], (int64_t)a.v[j][y].site0 + i, c);
                            const R cj = (R)coef(a.cv[j]);
                            t = {t.r + cj * vv.r, t.i + cj * vv.i};
                        }
                        t4[k] = t;
                        red += (double)t.r * t.r + (double)t.i * t.i;
                    }
                    SpinorIO<SP>::store_plane(a.out[y], so, 2 * w, t4[0], t4[1]);
                    SpinorIO<SP>::store_plane(a.out[y], so, 2 * w + 1, t4[2], t4[3]);
                }
            } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int c = 3 * w + k;
                C<R> t = cadd(cadd(part[0][c][lane], part[1][c][lane]), cadd(part[2][c][lane], part[3][c][lane]));
                if (a.has_self) {
                    const C<R> sf = SpinorIO<SP>::load_comp(a.self[y], (int64_t)a.self[y].site0 + i, c);
                    t = {as * sf.r + b * t.r, as * sf.i + b * t.i};
                } else {
                    t = cscale(b, t);
                }
                if (a.gamma5 && w >= 2) t = cneg(t);
                t = cscale(c0, t);
                for (int j = 0; j < a.nv; ++j) {
                    const C<R> vv = SpinorIO<SP>::load_comp(a.v[j][y], (int64_t)a.v[j][y].site0 + i, c);
                    const R cj = (R)coef(a.cv[j]);
                    t = {t.r + cj * vv.r, t.i + cj * vv.i};
                }
                SpinorIO<SP>::store_comp(a.out[y], so, c, t);
                red += (double)t.r * t.r + (double)t.i * t.i;
            }
            }
        }
    }
    if (a.partials) {
        const double s = block_sum(red, red_lds);
        if (threadIdx.x == 0) a.partials[lin] = s;
    }
}

// Links of a multi-right-hand-side tile in LDS, per direction a block of
// planes of 64 sites (lane l touches consecutive words).  F32/F16 links are
// decoded to 18 reals once per tile (the 12- and 8-real reconstructions then
// run once per link, not once per right-hand side); FP64 links stay in their
// stored words and are decoded per right-hand side, which keeps the LDS of a
// 12-real FP64 tile at 48 KiB.
template <int LP, int RECON>
struct StagedLinks {
    using LR = typename LinkReal<LP>::R;
    static constexpr bool kDecoded = LP != P64;
    static constexpr int kWords = kDecoded ? 18 : LinkFmt<LP, RECON>::kWords;
    __device__ static __forceinline__ void put(uint32_t* lw, int dir, int lane, const uint32_t words[]) {
        if constexpr (kDecoded) {
            C<LR> u[3][3];
            link_decode<LP, RECON>(words, u);
            float* d = reinterpret_cast<float*>(lw) + dir * 18 * 64 + lane;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    d[(2 * (3 * r + c)) * 64] = u[r][c].r;
                    d[(2 * (3 * r + c) + 1) * 64] = u[r][c].i;
                }
        } else {
#pragma unroll
            for (int k = 0; k < kWords; ++k) lw[(dir * kWords + k) * 64 + lane] = words[k];
        }
    }
    __device__ static __forceinline__ void get(const uint32_t* lw, int dir, int lane, C<LR> u[3][3]) {
        if constexpr (kDecoded) {
            const float* d = reinterpret_cast<const float*>(lw) + dir * 18 * 64 + lane;
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) u[r][c] = {d[(2 * (3 * r + c)) * 64], d[(2 * (3 * r + c) + 1) * 64]};
        } else {
            uint32_t words[kWords];
#pragma unroll
            for (int k = 0; k < kWords; ++k) words[k] = lw[(dir * kWords + k) * 64 + lane];
            link_decode<LP, RECON>(words, u);
        }
    }
};

// Many right-hand sides on one gauge field: a workgroup of 4 wavefronts owns
// 64 output sites; it first stages the 8 links of each site into LDS (forward
// links at the tile's own sites, backward links at the neighbours; see
// StagedLinks), then wavefront q computes right-hand sides q, q+4, q+8, ... for
// the 64 sites, reading the links from LDS.  Links leave HBM once per apply
// instead of once per right-hand side; every spinor load of a
// wavefront is one right-hand side's 64 consecutive sites.  The per-site
// arithmetic is that of k_wilson (same hop order and epilogue), so results
// match the one-lane-per-site kernel bit for bit.
//
// One tile: output parity p, sites 64*tile .. 64*tile+63 of that parity, and
// right-hand sides r0 .. r1-1.  The views address right-hand side 0;
// right-hand side r sits r * rhs_bytes further.  `self` may be null (no
// same-site term).  Must be reached by all 256 threads of the workgroup (it
// synchronises once).
template <int SP, int LP, int RECON, bool NT>
__device__ __forceinline__ void mrhs_tile(const GeomK& g, const char* links, int p, int32_t tile,
                                          const SpinorView& in, const SpinorView* self, const SpinorView& out,
                                          double a_self, double b_hop, int gamma5, double c0d, int r0, int r1,
                                          uint32_t* lw, int nv = 0, const SpinorView* v = nullptr, int vstride = 1,
                                          const Coef* cv = nullptr) {
    using R = typename SpinorIO<SP>::R;
    using LR = typename LinkReal<LP>::R;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int32_t i = tile * 64 + lane;
    const bool active = i < g.vh;
    int32_t nb[8];
    using SL = StagedLinks<LP, RECON>;
    if (active) {
        const SiteCoord x = eo_coords(g, p, i);
        eo_neighbours(g, i, x, nb);
        // wavefront w stages the forward link mu = w and the backward link mu = w
        uint32_t words[LinkFmt<LP, RECON>::kWords];
        link_load_words<LP, RECON, NT>(links, g.vh, p * 4 + w, i, words);
        SL::put(lw, w, lane, words);
        link_load_words<LP, RECON, NT>(links, g.vh, (1 - p) * 4 + w, nb[4 + w], words);
        SL::put(lw, 4 + w, lane, words);
    }
    __syncthreads();
    if (!active) return;
#pragma unroll 1
    for (int r = r0 + w; r < r1; r += 4) {
        // re-read links from LDS for every right-hand side instead of letting
        // them be hoisted into registers (which would cost occupancy)
        int lo = lane;
        asm volatile("" : "+v"(lo));
        SpinorView vin = in;
        vin.base += (int64_t)r * vin.rhs_bytes;
        C<R> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = {R(0), R(0)};
        // spinor loads of both hops of a direction first (one memory round
        // trip per direction; FP64: one per hop, for its registers); the
        // arithmetic order stays fwd 0, bwd 0, fwd 1, ...
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            C<R> sf[12], sb[12];
            C<LR> u[3][3];
            SpinorIO<SP>::load(vin, (int64_t)vin.site0 + nb[mu], sf);
            if constexpr (SP != P64) {
                SpinorIO<SP>::load(vin, (int64_t)vin.site0 + nb[4 + mu], sb);
                __builtin_amdgcn_sched_barrier(0);
            }
            SL::get(lw, mu, lo, u);
            if (mu == 0) hop_fwd<0>(sf, u, acc);
            if (mu == 1) hop_fwd<1>(sf, u, acc);
            if (mu == 2) hop_fwd<2>(sf, u, acc);
            if (mu == 3) hop_fwd<3>(sf, u, acc);
            if constexpr (SP == P64) SpinorIO<SP>::load(vin, (int64_t)vin.site0 + nb[4 + mu], sb);
            SL::get(lw, 4 + mu, lo, u);
            if (mu == 0) hop_bwd<0>(sb, u, acc);
            if (mu == 1) hop_bwd<1>(sb, u, acc);
            if (mu == 2) hop_bwd<2>(sb, u, acc);
            if (mu == 3) hop_bwd<3>(sb, u, acc);
        }
        const R b = (R)b_hop;
        if (self) {
            SpinorView vs = *self;
            vs.base += (int64_t)r * vs.rhs_bytes;
            C<R> sf[12];
            SpinorIO<SP>::load(vs, (int64_t)vs.site0 + i, sf);
            const R as = (R)a_self;
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = {as * sf[k].r + b * acc[k].r, as * sf[k].i + b * acc[k].i};
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = cscale(b, acc[k]);
        }
        if (gamma5) {
#pragma unroll
            for (int k = 6; k < 12; ++k) acc[k] = cneg(acc[k]);
        }
        const R c0 = (R)c0d;
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = cscale(c0, acc[k]);
        for (int j = 0; j < nv; ++j) {
            SpinorView vj = v[j * vstride];
            vj.base += (int64_t)r * vj.rhs_bytes;
            C<R> vv[12];
            SpinorIO<SP>::load(vj, (int64_t)vj.site0 + i, vv);
            const R cj = (R)coef(cv[j]);
#pragma unroll
            for (int k = 0; k < 12; ++k) acc[k] = {acc[k].r + cj * vv[k].r, acc[k].i + cj * vv[k].i};
        }
        SpinorView vo = out;
        vo.base += (int64_t)r * vo.rhs_bytes;
        SpinorIO<SP>::store(vo, (int64_t)vo.site0 + i, acc);
    }
}

// Work order of the multi-right-hand-side launch: a 1-D grid of tiles x ny
// output parities x ngroups groups of `rg` right-hand sides.  Group-major
// order runs every tile for one group before the next group (the spinors
// re-read by neighbouring tiles are then those of rg fields only, so they stay
// in L2; links are read once per group); tile-major order runs the groups of a
// tile next to each other (they share the tile's links in L2).
// XCD-group order (group_major = 2, ngroups dividing 8): workgroup b runs on
// XCD b mod 8 (the dispatcher's round robin); XCD x takes group x mod ngroups
// and part x / ngroups of the tile list, in order.  The XCDs holding the same
// part walk the same tiles at about the same time, so each tile's links come
// from HBM once and from the shared last-level cache for the other groups,
// while each XCD's L2 holds the neighbour spinors of its own rg fields only.
struct MrhsGrid {
    int32_t tiles;       // tiles of 64 sites per parity
    int ny;              // output parities (1 or 2)
    int rg;              // right-hand sides per workgroup
    int ngroups;
    int group_major;     // 0 tile-major, 1 group-major, 2 XCD groups
    int nrhs;
    int32_t per_part;    // XCD groups: tile positions per part
};

template <int SP, int LP, int RECON, bool NT>
__global__ void __launch_bounds__(256) k_wilson_mrhs(WilsonArgs a, MrhsGrid m) {
    extern __shared__ uint32_t lw[];   // [8 dirs][StagedLinks words][64 sites]
    const unsigned per_group = (unsigned)(m.ny * m.tiles);
    unsigned grp, rem;
    if (m.group_major == 2) {
        const unsigned x = blockIdx.x & 7u, k = blockIdx.x >> 3;
        grp = x % (unsigned)m.ngroups;
        rem = (x / (unsigned)m.ngroups) * (unsigned)m.per_part + k;
        if (rem >= per_group) return;   // the whole workgroup: before any barrier
    } else {
        unsigned lin = blockIdx.x;
        if (a.xcd_remap) lin = xcd_remap(lin, gridDim.x);
        if (m.group_major) {
            grp = lin / per_group;
            rem = lin - grp * per_group;
        } else {
            rem = lin / (unsigned)m.ngroups;
            grp = lin - rem * (unsigned)m.ngroups;
        }
    }
    int y = 0;
    int32_t pos = (int32_t)rem;
    if (m.ny == 2) {
        y = (int)(rem & 1u);
        pos = (int32_t)(rem >> 1);
    }
    const int32_t tile = order_tile(pos, m.tiles, a.g.n0, a.order_c);
    const int r0 = (int)grp * m.rg;
    const int r1 = min(m.nrhs, r0 + m.rg);
    mrhs_tile<SP, LP, RECON, NT>(a.g, a.links, a.p0 + y, tile, a.in[y], a.has_self ? &a.self[y] : nullptr, a.out[y],
                                 a.a_self, a.b_hop, a.gamma5, coef(a.c0), r0, r1, lw, a.nv, &a.v[0][y], 2, a.cv);
}

template <int SP, int LP, int RECON>
size_t mrhs_lds_bytes() {
    return (size_t)8 * StagedLinks<LP, RECON>::kWords * 64 * sizeof(uint32_t);
}

// FP64 18-real links need 72 KiB of LDS per workgroup (of the 160 KiB per CU):
// opt in above the default 64 KiB limit.
template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

template <int SP, int LP, int RECON, bool NT>
hipError_t launch_mrhs_nt(const WilsonArgs& a, const MrhsGrid& m, hipStream_t st) {
    const dim3 grid(m.group_major == 2 ? (unsigned)(8 * (int64_t)m.per_part)
                                       : (unsigned)((int64_t)m.tiles * m.ny * m.ngroups));
    const size_t lds = mrhs_lds_bytes<SP, LP, RECON>();
    const hipError_t e = allow_lds(&k_wilson_mrhs<SP, LP, RECON, NT>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_wilson_mrhs<SP, LP, RECON, NT>), grid, dim3(256), lds, st, a, m);
    return hipGetLastError();
}

// non-temporal link loads (automatic: when every link is read once, i.e. one
// output parity (ny = 1) and one group of right-hand sides)
template <int SP, int LP, int RECON>
hipError_t launch_mrhs_fmt(const WilsonArgs& a, const MrhsGrid& m, int link_nt, hipStream_t st) {
    const bool nt = link_nt < 0 ? (m.ny == 1 && m.ngroups == 1) : link_nt != 0;
    return nt ? launch_mrhs_nt<SP, LP, RECON, true>(a, m, st) : launch_mrhs_nt<SP, LP, RECON, false>(a, m, st);
}

// Q on several lattices (each with its own links and right-hand sides) in one
// persistent launch: the tiles of all lattices (both output parities) form one
// list; a grid of a fixed number of workgroups (a small multiple of what the
// device holds at once, independent of the lattices) walks it, workgroup b
// taking one contiguous chunk of tiles (chunks adjacent in the list go to
// workgroups on the same XCD), and each tile runs mrhs_tile with the epilogue
// of Q.
template <int SP, int LP, int RECON>
__global__ void __launch_bounds__(256) k_wilson_multi(MultiArgs a) {
    extern __shared__ uint32_t lw[];
    const unsigned lin = xcd_remap(blockIdx.x, gridDim.x);
    const int chunk = (a.total + (int)gridDim.x - 1) / (int)gridDim.x;
    const int t0 = (int)lin * chunk;
    const int t1 = min(a.total, t0 + chunk);
    for (int t = t0; t < t1; ++t) {
        int j = 0;
        while (j + 1 < a.njobs && t >= a.job[j + 1].tile0) ++j;
        const QJob& J = a.job[j];
        const int local = t - J.tile0;
        const int y = local / J.tiles;
        const int32_t tile = local - y * J.tiles;
        mrhs_tile<SP, LP, RECON, false>(J.g, J.links, y, tile, J.in[y], &J.self[y], J.out[y], J.a_self, -0.5, 1, 1.0,
                                        0, J.nrhs, lw);
        __syncthreads();   // the next tile overwrites the staged links
    }
}

std::atomic<int> g_multi_grid{4};

template <int SP, int LP, int RECON>
hipError_t launch_multi_fmt(const MultiArgs& a, hipStream_t st) {
    const size_t lds = mrhs_lds_bytes<SP, LP, RECON>();
    auto kernel = &k_wilson_multi<SP, LP, RECON>;
    hipError_t e = allow_lds(kernel, lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), 256, lds)) !=
        hipSuccess)
        return e;
    // a multiple (default 4) of the workgroups the device holds at once: one
    // resident set walking long chunks leaves each workgroup a serial chain of
    // memory round trips; a larger grid overlaps them and still bounds the grid
    const int grid = std::max(1, std::min(a.total, multi_grid_factor() * std::max(1, per_cu) * cus));
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(256), lds, st, a);
    return hipGetLastError();
}

template <int SP, int LP, int RECON, bool NT>
hipError_t launch_nt(const WilsonArgs& a, int ny, int block, hipStream_t st) {
    if (block == 0) {
        // direction split: 64 sites per workgroup of 4 wavefronts
        const dim3 grid((unsigned)((a.g.vh + 63) / 64), ny);
        hipLaunchKernelGGL((k_wilson_dirsplit<SP, LP, RECON, NT>), grid, dim3(256), 0, st, a);
        return hipGetLastError();
    }
    const unsigned nbx = (unsigned)((a.g.vh + block - 1) / block);
    const dim3 grid(nbx, ny);
    switch (block) {
        case 64: hipLaunchKernelGGL((k_wilson<SP, LP, RECON, 64, NT>), grid, dim3(64), 0, st, a); break;
        case 128: hipLaunchKernelGGL((k_wilson<SP, LP, RECON, 128, NT>), grid, dim3(128), 0, st, a); break;
        default: hipLaunchKernelGGL((k_wilson<SP, LP, RECON, 256, NT>), grid, dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

// one output parity (ny = 1) reads every link once: non-temporal link loads
template <int SP, int LP, int RECON>
hipError_t launch_fmt(const WilsonArgs& a, int ny, int block, hipStream_t st) {
    return ny == 1 ? launch_nt<SP, LP, RECON, true>(a, ny, block, st)
                   : launch_nt<SP, LP, RECON, false>(a, ny, block, st);
}

}  // namespace

namespace ndq {

int wilson_blocks(const ndq_geom* g, int block, int ny) {
    const int per = block == 0 ? 64 : block;
    return ((g->vh + per - 1) / per) * ny;
}

hipError_t launch_wilson(int sprec, int lprec, int recon, const WilsonArgs& args, int ny, int block,
                         hipStream_t st) {
    // Single-right-hand-side kernels keep the index order, except the FP64
    // full Q, whose larger per-site footprint gains from the slice-chunked
    // order (measured on 24^3 x 48; the F32 and F16 forms gain nothing).
    WilsonArgs a = args;
    if (block < 0) {
        const Tuning t = launch_tuning(a.g, sprec, lprec, recon, ny);
        block = t.block;
        a.xcd_remap = t.xcd_remap;
        if (t.order && a.order_c == 0) a.order_c = tile_order(a.g, block == 0 ? 64 : block);
    }
    if (ny == 2 && sprec == P64 && a.order_c == 0) a.order_c = tile_order(a.g, block == 0 ? 64 : block);
    const int key = sprec * 1000 + lprec * 100 + recon;
    switch (key) {
        case P64 * 1000 + P64 * 100 + 18: return launch_fmt<P64, P64, 18>(a, ny, block, st);
        case P64 * 1000 + P64 * 100 + 12: return launch_fmt<P64, P64, 12>(a, ny, block, st);
        case P64 * 1000 + P64 * 100 + 8: return launch_fmt<P64, P64, 8>(a, ny, block, st);
        case P32 * 1000 + P32 * 100 + 18: return launch_fmt<P32, P32, 18>(a, ny, block, st);
        case P32 * 1000 + P32 * 100 + 12: return launch_fmt<P32, P32, 12>(a, ny, block, st);
        case P32 * 1000 + P32 * 100 + 8: return launch_fmt<P32, P32, 8>(a, ny, block, st);
        case P32 * 1000 + P16 * 100 + 18: return launch_fmt<P32, P16, 18>(a, ny, block, st);
        case P32 * 1000 + P16 * 100 + 12: return launch_fmt<P32, P16, 12>(a, ny, block, st);
        case P16 * 1000 + P32 * 100 + 18: return launch_fmt<P16, P32, 18>(a, ny, block, st);
        case P16 * 1000 + P32 * 100 + 12: return launch_fmt<P16, P32, 12>(a, ny, block, st);
        case P16 * 1000 + P32 * 100 + 8: return launch_fmt<P16, P32, 8>(a, ny, block, st);
        case P16 * 1000 + P16 * 100 + 18: return launch_fmt<P16, P16, 18>(a, ny, block, st);
        case P16 * 1000 + P16 * 100 + 12: return launch_fmt<P16, P16, 12>(a, ny, block, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_wilson_mrhs(int sprec, int lprec, int recon, const WilsonArgs& args, int ny, int nrhs,
                              hipStream_t st) {
    WilsonArgs a = args;
    const MrhsShape sh = mrhs_shape(args.g, sprec, lprec, recon, nrhs, ny);
    a.order_c = sh.chunk < 0 ? tile_order(a.g, 64) : sh.chunk;
    a.xcd_remap = sh.xcd_remap;
    MrhsGrid m;
    m.tiles = (a.g.vh + 63) / 64;
    m.ny = ny;
    m.rg = std::max(1, std::min(sh.rg > 0 ? sh.rg : nrhs, nrhs));
    m.ngroups = (nrhs + m.rg - 1) / m.rg;
    m.group_major = sh.group_major;
    m.nrhs = nrhs;
    m.per_part = 0;
    if (m.group_major == 2) {
        if (8 % m.ngroups != 0) {
            m.group_major = 1;   // XCD groups need a number of groups dividing 8
        } else {
            const int parts = 8 / m.ngroups;
            m.per_part = (int32_t)((m.tiles * (int64_t)ny + parts - 1) / parts);
        }
    }
    const int key = sprec * 1000 + lprec * 100 + recon;
    switch (key) {
        case P64 * 1000 + P64 * 100 + 18: return launch_mrhs_fmt<P64, P64, 18>(a, m, sh.link_nt, st);
        case P64 * 1000 + P64 * 100 + 12: return launch_mrhs_fmt<P64, P64, 12>(a, m, sh.link_nt, st);
        case P64 * 1000 + P64 * 100 + 8: return launch_mrhs_fmt<P64, P64, 8>(a, m, sh.link_nt, st);
        case P32 * 1000 + P32 * 100 + 18: return launch_mrhs_fmt<P32, P32, 18>(a, m, sh.link_nt, st);
        case P32 * 1000 + P32 * 100 + 12: return launch_mrhs_fmt<P32, P32, 12>(a, m, sh.link_nt, st);
        case P32 * 1000 + P32 * 100 + 8: return launch_mrhs_fmt<P32, P32, 8>(a, m, sh.link_nt, st);
        case P32 * 1000 + P16 * 100 + 18: return launch_mrhs_fmt<P32, P16, 18>(a, m, sh.link_nt, st);
        case P32 * 1000 + P16 * 100 + 12: return launch_mrhs_fmt<P32, P16, 12>(a, m, sh.link_nt, st);
        case P16 * 1000 + P32 * 100 + 18: return launch_mrhs_fmt<P16, P32, 18>(a, m, sh.link_nt, st);
        case P16 * 1000 + P32 * 100 + 12: return launch_mrhs_fmt<P16, P32, 12>(a, m, sh.link_nt, st);
        case P16 * 1000 + P32 * 100 + 8: return launch_mrhs_fmt<P16, P32, 8>(a, m, sh.link_nt, st);
        case P16 * 1000 + P16 * 100 + 18: return launch_mrhs_fmt<P16, P16, 18>(a, m, sh.link_nt, st);
        case P16 * 1000 + P16 * 100 + 12: return launch_mrhs_fmt<P16, P16, 12>(a, m, sh.link_nt, st);
        default: return hipErrorInvalidValue;
    }
}

int multi_grid_factor() { return g_multi_grid.load(std::memory_order_relaxed); }
void set_multi_grid_factor(int f) { g_multi_grid.store(f, std::memory_order_relaxed); }

hipError_t launch_wilson_multi(int sprec, int lprec, int recon, const MultiArgs& a, hipStream_t st) {
    const int key = sprec * 1000 + lprec * 100 + recon;
    switch (key) {
        case P64 * 1000 + P64 * 100 + 18: return launch_multi_fmt<P64, P64, 18>(a, st);
        case P64 * 1000 + P64 * 100 + 12: return launch_multi_fmt<P64, P64, 12>(a, st);
        case P64 * 1000 + P64 * 100 + 8: return launch_multi_fmt<P64, P64, 8>(a, st);
        case P32 * 1000 + P32 * 100 + 18: return launch_multi_fmt<P32, P32, 18>(a, st);
        case P32 * 1000 + P32 * 100 + 12: return launch_multi_fmt<P32, P32, 12>(a, st);
        case P32 * 1000 + P32 * 100 + 8: return launch_multi_fmt<P32, P32, 8>(a, st);
        case P32 * 1000 + P16 * 100 + 18: return launch_multi_fmt<P32, P16, 18>(a, st);
        case P32 * 1000 + P16 * 100 + 12: return launch_multi_fmt<P32, P16, 12>(a, st);
        case P16 * 1000 + P32 * 100 + 18: return launch_multi_fmt<P16, P32, 18>(a, st);
        case P16 * 1000 + P32 * 100 + 12: return launch_multi_fmt<P16, P32, 12>(a, st);
        case P16 * 1000 + P32 * 100 + 8: return launch_multi_fmt<P16, P32, 8>(a, st);
        case P16 * 1000 + P16 * 100 + 18: return launch_multi_fmt<P16, P16, 18>(a, st);
        case P16 * 1000 + P16 * 100 + 12: return launch_multi_fmt<P16, P16, 12>(a, st);
        default: return hipErrorInvalidValue;
    }
}

int tile_order(const GeomK& g, int block) {
    const int64_t per_slice = g.vh / g.n0;
    if (g.n0 < 4 || per_slice * g.n0 != g.vh || per_slice % block) return 0;
    const int64_t S = per_slice / block;
    const int64_t s1t = (g.s1 + block - 1) / block;   // x1 neighbours, in tiles
    for (int64_t c = std::max<int64_t>(2, 4 * s1t); c < S; ++c)
        if (S % c == 0) return (int)c;
    return 0;
}

WilsonArgs wilson_args(const ndq_geom* g, const ndq_gauge* U, int sprec) {
    WilsonArgs a;
    memset(&a, 0, sizeof(a));
    a.g = g->k;
    a.links = static_cast<const char*>(U->data);
    a.c0 = {1.0, nullptr};
    a.xcd_remap = tuning(sprec, U->prec, U->recon).xcd_remap;
    return a;
}

}  // namespace ndq

extern "C" {

int ndq_apply_Q(const ndq_geom* g, const ndq_gauge* U, double m, const ndq_spinor* in, const ndq_spinor* out,
                void* stream) {
    if (!g) return fail(NDQ_EINVAL, "ndq_apply_Q: NULL geometry");
    int rc = check_gauge(U);
    if (!rc) rc = check_spinor(g, in, NDQ_FULL, "ndq_apply_Q in");
    if (!rc) rc = check_spinor(g, out, NDQ_FULL, "ndq_apply_Q out");
    if (!rc) rc = check_pair(U, in);
    if (rc) return rc;
    if (in->prec != out->prec || in->nrhs != out->nrhs)
        return fail(NDQ_EINVAL, "ndq_apply_Q: in and out must share precision and nrhs");
    if (in->data == out->data) return fail(NDQ_EINVAL, "ndq_apply_Q: in and out must not alias");
    hipStream_t st = as_stream(stream);
    const bool batched = in->nrhs > 1;
    for (int r = 0; r < (batched ? 1 : in->nrhs); ++r) {
        WilsonArgs a = wilson_args(g, U, in->prec);
        a.p0 = 0;
        for (int p = 0; p < 2; ++p) {
            a.in[p] = view_of(g, in, 1 - p, r);
            a.self[p] = view_of(g, in, p, r);
            a.out[p] = view_of(g, out, p, r);
        }
        a.has_self = 1;
        a.a_self = 4.0 + m;
        a.b_hop = -0.5;
        a.gamma5 = 1;
        if (batched) NDQ_HIP(launch_wilson_mrhs(in->prec, U->prec, U->recon, a, 2, in->nrhs, st));
        else NDQ_HIP(launch_wilson(in->prec, U->prec, U->recon, a, 2, -1, st));
    }
    return NDQ_OK;
}

int ndq_apply_Q_multi(const ndq_q_job* jobs, int32_t njobs, void* stream) {
    if (!jobs || njobs < 1 || njobs > kMaxJobs)
        return fail(NDQ_EINVAL, "ndq_apply_Q_multi: need 1..%d jobs (got %d)", kMaxJobs, njobs);
    MultiArgs a;
    memset(&a, 0, sizeof(a));
    a.njobs = njobs;
    int64_t total = 0;
    int sprec = -1, lprec = -1, recon = -1;
    for (int j = 0; j < njobs; ++j) {
        const ndq_q_job& J = jobs[j];
        if (!J.g) return fail(NDQ_EINVAL, "ndq_apply_Q_multi: job %d: NULL geometry", j);
        int rc = check_gauge(J.U);
        if (!rc) rc = check_spinor(J.g, J.in, NDQ_FULL, "ndq_apply_Q_multi in");
        if (!rc) rc = check_spinor(J.g, J.out, NDQ_FULL, "ndq_apply_Q_multi out");
        if (!rc) rc = check_pair(J.U, J.in);
        if (rc) return rc;
        if (J.in->prec != J.out->prec || J.in->nrhs != J.out->nrhs)
            return fail(NDQ_EINVAL, "ndq_apply_Q_multi: job %d: in and out must share precision and nrhs", j);
        if (J.in->data == J.out->data) return fail(NDQ_EINVAL, "ndq_apply_Q_multi: job %d: in and out alias", j);
        if (j == 0) {
            sprec = J.in->prec;
            lprec = J.U->prec;
            recon = J.U->recon;
        } else if (J.in->prec != sprec || J.U->prec != lprec || J.U->recon != recon) {
            return fail(NDQ_EINVAL, "ndq_apply_Q_multi: job %d: all jobs must share spinor precision and link format", j);
        }
        QJob& q = a.job[j];
        q.g = J.g->k;
        q.links = static_cast<const char*>(J.U->data);
        for (int p = 0; p < 2; ++p) {
            q.in[p] = view_of(J.g, J.in, 1 - p, 0);
            q.self[p] = view_of(J.g, J.in, p, 0);
            q.out[p] = view_of(J.g, J.out, p, 0);
        }
        q.a_self = 4.0 + J.m;
        q.nrhs = J.in->nrhs;
        q.tiles = (J.g->vh + 63) / 64;
        q.tile0 = (int)total;
        total += 2 * (int64_t)q.tiles;
    }
    if (total > INT32_MAX) return fail(NDQ_EINVAL, "ndq_apply_Q_multi: too many sites");
    a.total = (int)total;
    NDQ_HIP(launch_wilson_multi(sprec, lprec, recon, a, as_stream(stream)));
    return NDQ_OK;
}

int ndq_apply_dslash(const ndq_geom* g, const ndq_gauge* U, const ndq_spinor* in, const ndq_spinor* out,
                     void* stream) {
    if (!g) return fail(NDQ_EINVAL, "ndq_apply_dslash: NULL geometry");
    int rc = check_gauge(U);
    if (!rc) rc = check_spinor(g, in, -1, "ndq_apply_dslash in");
    if (!rc) rc = check_spinor(g, out, -1, "ndq_apply_dslash out");
    if (!rc) rc = check_pair(U, in);
    if (rc) return rc;
    if (in->parity == NDQ_FULL || out->parity == NDQ_FULL || in->parity == out->parity)
        return fail(NDQ_EINVAL, "ndq_apply_dslash: in and out must be opposite parity fields");
    if (in->prec != out->prec || in->nrhs != out->nrhs)
        return fail(NDQ_EINVAL, "ndq_apply_dslash: in and out must share precision and nrhs");
    hipStream_t st = as_stream(stream);
    const int p = out->parity;
    const bool batched = in->nrhs > 1;
    for (int r = 0; r < (batched ? 1 : in->nrhs); ++r) {
        WilsonArgs a = wilson_args(g, U, in->prec);
        a.p0 = p;
        a.in[0] = view_of(g, in, 1 - p, r);
        a.out[0] = view_of(g, out, p, r);
        a.has_self = 0;
        a.b_hop = 1.0;
        a.gamma5 = 0;
        if (batched) NDQ_HIP(launch_wilson_mrhs(in->prec, U->prec, U->recon, a, 1, in->nrhs, st));
        else NDQ_HIP(launch_wilson(in->prec, U->prec, U->recon, a, 1, -1, st));
    }
    return NDQ_OK;
}

int ndq_apply_Qhat_ee(const ndq_geom* g, const ndq_gauge* U, double m, const ndq_spinor* in, const ndq_spinor* out,
                      const ndq_spinor* tmp, void* stream) {
    if (!g) return fail(NDQ_EINVAL, "ndq_apply_Qhat_ee: NULL geometry");
    int rc = check_gauge(U);
    if (!rc) rc = check_spinor(g, in, NDQ_EVEN, "ndq_apply_Qhat_ee in");
    if (!rc) rc = check_spinor(g, out, NDQ_EVEN, "ndq_apply_Qhat_ee out");
    if (!rc) rc = check_spinor(g, tmp, NDQ_ODD, "ndq_apply_Qhat_ee tmp");
    if (!rc) rc = check_pair(U, in);
    if (rc) return rc;
    if (in->prec != out->prec || in->prec != tmp->prec || in->nrhs != out->nrhs || tmp->nrhs < in->nrhs)
        return fail(NDQ_EINVAL, "ndq_apply_Qhat_ee: fields must share precision and nrhs");
    if (in->data == out->data) return fail(NDQ_EINVAL, "ndq_apply_Qhat_ee: in and out must not alias");
    if (4.0 + m == 0.0) return fail(NDQ_ESINGULAR, "ndq_apply_Qhat_ee: 4 + m = 0");
    hipStream_t st = as_stream(stream);
    for (int r = 0; r < in->nrhs; ++r) {
        WilsonArgs a = wilson_args(g, U, in->prec);
        a.p0 = 1;
        a.in[0] = view_of(g, in, 0, r);
        a.out[0] = view_of(g, tmp, 1, r);
        a.b_hop = 1.0;
        NDQ_HIP(launch_wilson(in->prec, U->prec, U->recon, a, 1, -1, st));
        WilsonArgs b = wilson_args(g, U, in->prec);
        b.p0 = 0;
        b.in[0] = view_of(g, tmp, 1, r);
        b.self[0] = view_of(g, in, 0, r);
        b.out[0] = view_of(g, out, 0, r);
        b.has_self = 1;
        b.a_self = 4.0 + m;
        b.b_hop = -1.0 / (4.0 * (4.0 + m));
        b.gamma5 = 1;
        NDQ_HIP(launch_wilson(in->prec, U->prec, U->recon, b, 1, -1, st));
    }
    return NDQ_OK;
}

}  // extern "C"
