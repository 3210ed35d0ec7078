// Device-side building blocks shared by the ndq HIP kernels (gfx950):
// complex arithmetic, exact division by lattice extents, even/odd site
// indexing, and loaders/storers for the packed spinor and link layouts.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace ndq {

enum { P64 = 0, P32 = 1, P16 = 2 };

// ---------------------------------------------------------------------------
// complex numbers
// ---------------------------------------------------------------------------
template <typename R>
struct C {
    R r, i;
};

template <typename R> __device__ __forceinline__ C<R> cadd(C<R> a, C<R> b) { return {a.r + b.r, a.i + b.i}; }
template <typename R> __device__ __forceinline__ C<R> csub(C<R> a, C<R> b) { return {a.r - b.r, a.i - b.i}; }
template <typename R> __device__ __forceinline__ C<R> cneg(C<R> a) { return {-a.r, -a.i}; }
template <typename R> __device__ __forceinline__ C<R> cconj(C<R> a) { return {a.r, -a.i}; }
// i*a and -i*a
template <typename R> __device__ __forceinline__ C<R> cmuli(C<R> a) { return {-a.i, a.r}; }
template <typename R> __device__ __forceinline__ C<R> cmulmi(C<R> a) { return {a.i, -a.r}; }
template <typename R> __device__ __forceinline__ C<R> cmul(C<R> a, C<R> b) {
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
// conj(a) * b
template <typename R> __device__ __forceinline__ C<R> cmulc(C<R> a, C<R> b) {
    return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
template <typename R> __device__ __forceinline__ C<R> cscale(R s, C<R> a) { return {s * a.r, s * a.i}; }
// a + b*c
template <typename R> __device__ __forceinline__ C<R> cfma(C<R> a, C<R> b, C<R> c) {
    return {a.r + b.r * c.r - b.i * c.i, a.i + b.r * c.i + b.i * c.r};
}
// a + conj(b)*c
template <typename R> __device__ __forceinline__ C<R> cfmac(C<R> a, C<R> b, C<R> c) {
    return {a.r + b.r * c.r + b.i * c.i, a.i + b.r * c.i - b.i * c.r};
}

// ---------------------------------------------------------------------------
// exact division n / d for 0 <= n < 2^31 by a fixed d >= 1:
// q = (n * m) >> s with l = ceil(log2 d), m = ceil(2^(31+l) / d) < 2^32, s = 31 + l
// (Granlund & Montgomery, "Division by invariant integers using multiplication").
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t m;
    uint32_t s;
};

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv d) {
    return (uint32_t)(((uint64_t)n * d.m) >> d.s);
}

// ---------------------------------------------------------------------------
// geometry passed to kernels by value
// ---------------------------------------------------------------------------
struct GeomK {
    int32_t n0, n1, n2, n3;
    int32_t nh3;   // N3 / 2
    int32_t s1;    // eo stride of x1: N2 * N3 / 2
    int32_t s0;    // eo stride of x0: N1 * N2 * N3 / 2
    int32_t vh;    // V / 2
    FastDiv d_nh3, d_n2, d_n1;
};

struct SiteCoord {
    int32_t x0, x1, x2, x3;
};

// Coordinates of the site with parity p and even/odd index i.
__device__ __forceinline__ SiteCoord eo_coords(const GeomK& g, int p, int32_t i) {
    const uint32_t q = fdiv((uint32_t)i, g.d_nh3);
    const int32_t x3h = i - (int32_t)q * g.nh3;
    const uint32_t r = fdiv(q, g.d_n2);
    const int32_t x2 = (int32_t)q - (int32_t)r * g.n2;
    const uint32_t x0 = fdiv(r, g.d_n1);
    const int32_t x1 = (int32_t)r - (int32_t)x0 * g.n1;
    const int32_t bit = (p + (int32_t)x0 + x1 + x2) & 1;
    return {(int32_t)x0, x1, x2, 2 * x3h + bit};
}

// Even/odd indices (within parity 1-p) of the 8 neighbours of site (p, i):
// nb[mu] = x + mu-hat, nb[4+mu] = x - mu-hat, periodic.
__device__ __forceinline__ void eo_neighbours(const GeomK& g, int32_t i, const SiteCoord& x, int32_t nb[8]) {
    const int32_t row = i - (x.x3 >> 1);   // eo index of (x0, x1, x2, 0..1)
    const int32_t x3p = (x.x3 + 1 == g.n3) ? 0 : x.x3 + 1;
    const int32_t x3m = (x.x3 == 0) ? g.n3 - 1 : x.x3 - 1;
    nb[3] = row + (x3p >> 1);
    nb[7] = row + (x3m >> 1);
    nb[2] = (x.x2 == g.n2 - 1) ? i - (g.n2 - 1) * g.nh3 : i + g.nh3;
    nb[6] = (x.x2 == 0) ? i + (g.n2 - 1) * g.nh3 : i - g.nh3;
    nb[1] = (x.x1 == g.n1 - 1) ? i - (g.n1 - 1) * g.s1 : i + g.s1;
    nb[5] = (x.x1 == 0) ? i + (g.n1 - 1) * g.s1 : i - g.s1;
    nb[0] = (x.x0 == g.n0 - 1) ? i - (g.n0 - 1) * g.s0 : i + g.s0;
    nb[4] = (x.x0 == 0) ? i + (g.n0 - 1) * g.s0 : i - g.s0;
}

// ---------------------------------------------------------------------------
// packed spinor fields
//
// A spinor "view" addresses one right-hand side of one site subset.  Sites
// are planes of 16-byte words with a plane stride of `stride` sites:
//   F64: 12 planes of double2 (one complex component each, c = 3*spin + colour)
//   F32:  6 planes of float4  (components 2j, 2j+1)
//   F16:  3 planes of 8 halves (components 4j..4j+3) scaled by a per-site F32
//         factor stored in a float plane right after the three half planes.
// ---------------------------------------------------------------------------
struct SpinorView {
    char* base;        // first plane of right-hand side 0
    int32_t stride;    // plane stride in sites
    int32_t site0;     // offset of this subset inside the planes (p*V/2 for a full field)
    int64_t rhs_bytes; // distance between right-hand sides
};

template <int P> struct SpinorIO;

template <> struct SpinorIO<P64> {
    using R = double;
    static constexpr int kBytesPerSite = 192;
    __device__ static __forceinline__ void load(const SpinorView& v, int64_t s, C<R> out[12]) {
        const double2* p = reinterpret_cast<const double2*>(v.base) + s;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double2 w = p[(int64_t)c * v.stride];
            out[c] = {w.x, w.y};
        }
    }
    __device__ static __forceinline__ void store(const SpinorView& v, int64_t s, const C<R> in[12]) {
        double2* p = reinterpret_cast<double2*>(v.base) + s;
#pragma unroll
        for (int c = 0; c < 12; ++c) p[(int64_t)c * v.stride] = make_double2(in[c].r, in[c].i);
    }
    // single complex component c (plane c)
    __device__ static __forceinline__ C<R> load_comp(const SpinorView& v, int64_t s, int c) {
        const double2 w = reinterpret_cast<const double2*>(v.base)[(int64_t)c * v.stride + s];
        return {w.x, w.y};
    }
    __device__ static __forceinline__ void store_comp(const SpinorView& v, int64_t s, int c, C<R> x) {
        reinterpret_cast<double2*>(v.base)[(int64_t)c * v.stride + s] = make_double2(x.r, x.i);
    }
};

template <> struct SpinorIO<P32> {
    using R = float;
    static constexpr int kBytesPerSite = 96;
    __device__ static __forceinline__ void load(const SpinorView& v, int64_t s, C<R> out[12]) {
        const float4* p = reinterpret_cast<const float4*>(v.base) + s;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const float4 w = p[(int64_t)j * v.stride];
            out[2 * j] = {w.x, w.y};
            out[2 * j + 1] = {w.z, w.w};
        }
    }
    __device__ static __forceinline__ void store(const SpinorView& v, int64_t s, const C<R> in[12]) {
        float4* p = reinterpret_cast<float4*>(v.base) + s;
#pragma unroll
        for (int j = 0; j < 6; ++j)
            p[(int64_t)j * v.stride] = make_float4(in[2 * j].r, in[2 * j].i, in[2 * j + 1].r, in[2 * j + 1].i);
    }
    // single complex component c: half (c & 1) of float4 plane c >> 1
    __device__ static __forceinline__ C<R> load_comp(const SpinorView& v, int64_t s, int c) {
        const float2 w = reinterpret_cast<const float2*>(v.base)[2 * ((int64_t)(c >> 1) * v.stride + s) + (c & 1)];
        return {w.x, w.y};
    }
    __device__ static __forceinline__ void store_comp(const SpinorView& v, int64_t s, int c, C<R> x) {
        reinterpret_cast<float2*>(v.base)[2 * ((int64_t)(c >> 1) * v.stride + s) + (c & 1)] = make_float2(x.r, x.i);
    }
    // components 2j and 2j+1 (the whole 16-byte word of plane j)
    __device__ static __forceinline__ void store_plane(const SpinorView& v, int64_t s, int j, C<R> x, C<R> y) {
        reinterpret_cast<float4*>(v.base)[(int64_t)j * v.stride + s] = make_float4(x.r, x.i, y.r, y.i);
    }
};

template <> struct SpinorIO<P16> {
    using R = float;
    static constexpr int kBytesPerSite = 52;
    __device__ static __forceinline__ void load(const SpinorView& v, int64_t s, C<R> out[12]) {
        const uint4* p = reinterpret_cast<const uint4*>(v.base) + s;
        const float scale = reinterpret_cast<const float*>(v.base + (int64_t)48 * v.stride)[s];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const uint4 w = p[(int64_t)j * v.stride];
            const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                __half2 h = *reinterpret_cast<const __half2*>(&words[k]);
                float2 f = __half22float2(h);
                out[4 * j + k] = {f.x * scale, f.y * scale};
            }
        }
    }
    __device__ static __forceinline__ void store(const SpinorView& v, int64_t s, const C<R> in[12]) {
        float amax = 0.f;
#pragma unroll
        for (int c = 0; c < 12; ++c) amax = fmaxf(amax, fmaxf(fabsf(in[c].r), fabsf(in[c].i)));
        const float inv = amax > 0.f ? 1.0f / amax : 0.f;
        uint4* p = reinterpret_cast<uint4*>(v.base) + s;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            uint32_t words[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                __half2 h = __floats2half2_rn(in[4 * j + k].r * inv, in[4 * j + k].i * inv);
                words[k] = *reinterpret_cast<uint32_t*>(&h);
            }
            p[(int64_t)j * v.stride] = make_uint4(words[0], words[1], words[2], words[3]);
        }
        reinterpret_cast<float*>(v.base + (int64_t)48 * v.stride)[s] = amax;
    }
    // single complex component c: half2 (c & 3) of plane c >> 2, times the site's scale
    __device__ static __forceinline__ C<R> load_comp(const SpinorView& v, int64_t s, int c) {
        const uint32_t w = reinterpret_cast<const uint32_t*>(v.base)[4 * ((int64_t)(c >> 2) * v.stride + s) + (c & 3)];
        const float scale = reinterpret_cast<const float*>(v.base + (int64_t)48 * v.stride)[s];
        const float2 f = __half22float2(*reinterpret_cast<const __half2*>(&w));
        return {f.x * scale, f.y * scale};
    }
};

// ---------------------------------------------------------------------------
// packed links
//
// All 4V links: block (p, mu) at index p*4 + mu holds the links U_mu(x) of the
// V/2 sites x of parity p, in even/odd index order.  Inside a block, a link of
// B bytes is split into B/16 planes of 16-byte words followed by one plane of
// the remaining B%16 bytes (4 or 8), each plane with a stride of V/2 sites.
// Real order in a link record:
//   18: U[row][col] row-major, (re, im) pairs
//   12: columns a = U[.][0] and b = U[.][1]: a1 a2 a3 b1 b2 b3 as (re, im)
//    8: a2, a3, b1 as (re, im), then arg a1, arg c1
// ---------------------------------------------------------------------------
template <int P> struct LinkReal;
template <> struct LinkReal<P64> { using S = double; using R = double; };
template <> struct LinkReal<P32> { using S = float; using R = float; };
template <> struct LinkReal<P16> { using S = __half; using R = float; };

template <int P, int RECON>
struct LinkFmt {
    static constexpr int kBytes = RECON * (P == P64 ? 8 : P == P32 ? 4 : 2);
    static constexpr int kN16 = kBytes / 16;
    static constexpr int kTail = kBytes % 16;
    static constexpr int kWords = kBytes / 4;
};

// NT = true loads with the non-temporal hint.  An even/odd dslash reads every
// link exactly once, so there the hint keeps links from displacing the spinor
// words that neighbouring sites re-read from the caches; a full Q apply reads
// each link twice (as forward link of its site and backward link of the
// neighbour), and there the second read should find it cached (NT = false).
typedef unsigned int u32x4_v __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_v __attribute__((ext_vector_type(2)));

template <bool NT, typename T>
__device__ __forceinline__ T load_hinted(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int P, int RECON, bool NT = false>
__device__ __forceinline__ void link_load_words(const char* base, int32_t vh, int blk, int32_t i, uint32_t w[]) {
    using F = LinkFmt<P, RECON>;
    const char* b = base + (int64_t)blk * F::kBytes * vh;
#pragma unroll
    for (int j = 0; j < F::kN16; ++j) {
        const u32x4_v x = load_hinted<NT>(reinterpret_cast<const u32x4_v*>(b + (int64_t)j * 16 * vh) + i);
        w[4 * j + 0] = x.x;
        w[4 * j + 1] = x.y;
        w[4 * j + 2] = x.z;
        w[4 * j + 3] = x.w;
    }
    if constexpr (F::kTail == 8) {
        const u32x2_v x = load_hinted<NT>(reinterpret_cast<const u32x2_v*>(b + (int64_t)F::kN16 * 16 * vh) + i);
        w[4 * F::kN16 + 0] = x.x;
        w[4 * F::kN16 + 1] = x.y;
    } else if constexpr (F::kTail == 4) {
        w[4 * F::kN16] = load_hinted<NT>(reinterpret_cast<const uint32_t*>(b + (int64_t)F::kN16 * 16 * vh) + i);
    }
}

template <int P, int RECON>
__device__ __forceinline__ void link_store_words(char* base, int32_t vh, int blk, int32_t i, const uint32_t w[]) {
    using F = LinkFmt<P, RECON>;
    char* b = base + (int64_t)blk * F::kBytes * vh;
#pragma unroll
    for (int j = 0; j < F::kN16; ++j)
        reinterpret_cast<uint4*>(b + (int64_t)j * 16 * vh)[i] = make_uint4(w[4 * j], w[4 * j + 1], w[4 * j + 2], w[4 * j + 3]);
    if constexpr (F::kTail == 8) {
        reinterpret_cast<uint2*>(b + (int64_t)F::kN16 * 16 * vh)[i] = make_uint2(w[4 * F::kN16], w[4 * F::kN16 + 1]);
    } else if constexpr (F::kTail == 4) {
        reinterpret_cast<uint32_t*>(b + (int64_t)F::kN16 * 16 * vh)[i] = w[4 * F::kN16];
    }
}

// Real number k of a link record held in 32-bit words.
template <int P>
__device__ __forceinline__ typename LinkReal<P>::R link_real(const uint32_t w[], int k) {
    if constexpr (P == P64) {
        const uint64_t bits = (uint64_t)w[2 * k] | ((uint64_t)w[2 * k + 1] << 32);
        return __longlong_as_double((long long)bits);
    } else if constexpr (P == P32) {
        return __uint_as_float(w[k]);
    } else {
        const uint32_t word = w[k >> 1];
        const unsigned short hb = (k & 1) ? (unsigned short)(word >> 16) : (unsigned short)(word & 0xffffu);
        return __half2float(__ushort_as_half(hb));
    }
}

template <int P>
__device__ __forceinline__ void link_set_real(uint32_t w[], int k, double x) {
    if constexpr (P == P64) {
        const uint64_t bits = (uint64_t)__double_as_longlong(x);
        w[2 * k] = (uint32_t)bits;
        w[2 * k + 1] = (uint32_t)(bits >> 32);
    } else if constexpr (P == P32) {
        w[k] = __float_as_uint((float)x);
    } else {
        const uint32_t hb = (uint32_t)__half_as_ushort(__float2half_rn((float)x));
        if (k & 1) w[k >> 1] = (w[k >> 1] & 0xffffu) | (hb << 16);
        else w[k >> 1] = (w[k >> 1] & 0xffff0000u) | hb;
    }
}

// sin and cos of a stored phase |x| <= pi (plus rounding).  Cody-Waite
// reduction by pi/2 to |r| <= pi/4, then the Taylor series of sin and cos in
// Horner form, truncated where the next term is below the type's rounding
// ((pi/4)^19/19! ~ 1e-18 in double, (pi/4)^11/11! ~ 2e-9 in float).  Avoids the
// large-argument reduction of the general library routine, which the
// register-bound stencil cannot afford.
__device__ __forceinline__ void sincos_pm_pi(double x, double& s, double& c) {
    const double q = rint(x * 0.63661977236758134308);  // 2/pi
    const double r = (x - q * 1.5707963267948966192) - q * 6.123233995736766036e-17;
    const double r2 = r * r;
    double ps = 1.0 / 121645100408832000.0;                // 1/19!
    ps = ps * -r2 + 1.0 / 355687428096000.0;               // 1/17!
    ps = ps * -r2 + 1.0 / 1307674368000.0;                 // 1/15!
    ps = ps * -r2 + 1.0 / 6227020800.0;                    // 1/13!
    ps = ps * -r2 + 1.0 / 39916800.0;                      // 1/11!
    ps = ps * -r2 + 1.0 / 362880.0;                        // 1/9!
    ps = ps * -r2 + 1.0 / 5040.0;                          // 1/7!
    ps = ps * -r2 + 1.0 / 120.0;                           // 1/5!
    ps = ps * -r2 + 1.0 / 6.0;                             // 1/3!
    const double sr = r - r * r2 * ps;
    double pc = 1.0 / 6402373705728000.0;                  // 1/18!
    pc = pc * -r2 + 1.0 / 20922789888000.0;                // 1/16!
    pc = pc * -r2 + 1.0 / 87178291200.0;                   // 1/14!
    pc = pc * -r2 + 1.0 / 479001600.0;                     // 1/12!
    pc = pc * -r2 + 1.0 / 3628800.0;                       // 1/10!
    pc = pc * -r2 + 1.0 / 40320.0;                         // 1/8!
    pc = pc * -r2 + 1.0 / 720.0;                           // 1/6!
    pc = pc * -r2 + 1.0 / 24.0;                            // 1/4!
    pc = pc * -r2 + 0.5;                                   // 1/2!
    const double cr = 1.0 - r2 * pc;
    const int k = ((int)q) & 3;
    s = (k == 0) ? sr : (k == 1) ? cr : (k == 2) ? -sr : -cr;
    c = (k == 0) ? cr : (k == 1) ? -sr : (k == 2) ? -cr : sr;
}

__device__ __forceinline__ void sincos_pm_pi(float x, float& s, float& c) {
    const float q = rintf(x * 0.636619772f);
    const float r = (x - q * 1.57079637f) + q * 4.37113883e-8f;  // pi/2 = 1.57079637 - 4.37e-8
    const float r2 = r * r;
    float ps = 1.0f / 362880.0f;
    ps = ps * -r2 + 1.0f / 5040.0f;
    ps = ps * -r2 + 1.0f / 120.0f;
    ps = ps * -r2 + 1.0f / 6.0f;
    const float sr = r - r * r2 * ps;
    float pc = 1.0f / 3628800.0f;
    pc = pc * -r2 + 1.0f / 40320.0f;
    pc = pc * -r2 + 1.0f / 720.0f;
    pc = pc * -r2 + 1.0f / 24.0f;
    pc = pc * -r2 + 0.5f;
    const float cr = 1.0f - r2 * pc;
    const int k = ((int)q) & 3;
    s = (k == 0) ? sr : (k == 1) ? cr : (k == 2) ? -sr : -cr;
    c = (k == 0) ? cr : (k == 1) ? -sr : (k == 2) ? -cr : sr;
}

// Decode a link record into the full 3x3 matrix u[row][col].
template <int P, int RECON>
__device__ __forceinline__ void link_decode(const uint32_t w[], C<typename LinkReal<P>::R> u[3][3]) {
    using R = typename LinkReal<P>::R;
    if constexpr (RECON == 18) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) u[r][c] = {link_real<P>(w, 2 * (3 * r + c)), link_real<P>(w, 2 * (3 * r + c) + 1)};
    } else if constexpr (RECON == 12) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            u[r][0] = {link_real<P>(w, 2 * r), link_real<P>(w, 2 * r + 1)};
            u[r][1] = {link_real<P>(w, 6 + 2 * r), link_real<P>(w, 6 + 2 * r + 1)};
        }
        // c = conj(a x b)  (Sec. 2.1, Eq. 3)
        u[0][2] = cconj(csub(cmul(u[1][0], u[2][1]), cmul(u[2][0], u[1][1])));
        u[1][2] = cconj(csub(cmul(u[2][0], u[0][1]), cmul(u[0][0], u[2][1])));
        u[2][2] = cconj(csub(cmul(u[0][0], u[1][1]), cmul(u[1][0], u[0][1])));
    } else {
        static_assert(RECON == 8, "recon must be 18, 12 or 8");
        const C<R> a2 = {link_real<P>(w, 0), link_real<P>(w, 1)};
        const C<R> a3 = {link_real<P>(w, 2), link_real<P>(w, 3)};
        const C<R> b1 = {link_real<P>(w, 4), link_real<P>(w, 5)};
        const R th_a = link_real<P>(w, 6);
        const R th_c = link_real<P>(w, 7);
        const R n = a2.r * a2.r + a2.i * a2.i + a3.r * a3.r + a3.i * a3.i;
        const R b1sq = b1.r * b1.r + b1.i * b1.i;
        const R ma1 = sqrt(fmax(R(1) - n, R(0)));
        const R mc1 = sqrt(fmax(n - b1sq, R(0)));
        R sa, ca, sc, cc;
        sincos_pm_pi(th_a, sa, ca);
        sincos_pm_pi(th_c, sc, cc);
        const C<R> a1 = {ma1 * ca, ma1 * sa};
        const C<R> c1 = {mc1 * cc, mc1 * sc};
        const R inv = R(1) / n;
        // unitarity of the columns together with c = conj(a x b):
        // b2 = -(a1* a2 b1 + a3* c1*)/n     b3 = (-a1* a3 b1 + a2* c1*)/n
        // c2 = (-a1* a2 c1 + a3* b1*)/n     c3 = -(a1* a3 c1 + a2* b1*)/n
        const C<R> a1c_a2 = cmulc(a1, a2);
        const C<R> a1c_a3 = cmulc(a1, a3);
        const C<R> b2 = cscale(-inv, cadd(cmul(a1c_a2, b1), cmulc(a3, cconj(c1))));
        const C<R> b3 = cscale(inv, csub(cmulc(a2, cconj(c1)), cmul(a1c_a3, b1)));
        const C<R> c2 = cscale(inv, csub(cmulc(a3, cconj(b1)), cmul(a1c_a2, c1)));
        const C<R> c3 = cscale(-inv, cadd(cmul(a1c_a3, c1), cmulc(a2, cconj(b1))));
        u[0][0] = a1; u[0][1] = b1; u[0][2] = c1;
        u[1][0] = a2; u[1][1] = b2; u[1][2] = c2;
        u[2][0] = a3; u[2][1] = b3; u[2][2] = c3;
    }
}

template <int P, int RECON>
__device__ __forceinline__ void link_load(const char* base, int32_t vh, int blk, int32_t i,
                                          C<typename LinkReal<P>::R> u[3][3]) {
    uint32_t w[LinkFmt<P, RECON>::kWords];
    link_load_words<P, RECON>(base, vh, blk, i, w);
    link_decode<P, RECON>(w, u);
}

// ---------------------------------------------------------------------------
// wavefront / block reductions in FP64
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Sum over the block; valid in thread 0.  `lds` needs blockDim.x/64 doubles.
__device__ __forceinline__ double block_sum(double x, double* lds) {
    x = wave_sum(x);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = x;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < nw; ++k) s += lds[k];
    }
    return s;
}

}  // namespace ndq
