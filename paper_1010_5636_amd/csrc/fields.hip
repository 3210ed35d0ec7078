// Conversion between canonical complex128 fields and the packed layouts.
#include "ndq_internal.h"

using namespace ndq;

namespace {

// One lane per (lexicographic site, mu): encode link U_mu(x).
template <int LP, int RECON>
__global__ void k_gauge_pack(GeomK g, const double2* __restrict__ canon, char* __restrict__ links,
                             int* __restrict__ singular) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t v = 2 * (int64_t)g.vh;
    if (t >= 4 * v) return;
    const int64_t lex = t >> 2;
    const int mu = (int)(t & 3);
    // parity of a lexicographic site from its coordinates
    const int64_t x3 = lex % g.n3;
    const int64_t q = lex / g.n3;
    const int64_t x2 = q % g.n2;
    const int64_t r = q / g.n2;
    const int64_t x1 = r % g.n1;
    const int64_t x0 = r / g.n1;
    const int p = (int)((x0 + x1 + x2 + x3) & 1);
    const int32_t i = (int32_t)(lex >> 1);
    const double2* u = canon + (lex * 4 + mu) * 9;   // [3][3] row-major
    uint32_t w[LinkFmt<LP, RECON>::kWords];
#pragma unroll
    for (int k = 0; k < LinkFmt<LP, RECON>::kWords; ++k) w[k] = 0;
    if constexpr (RECON == 18) {
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            link_set_real<LP>(w, 2 * e, u[e].x);
            link_set_real<LP>(w, 2 * e + 1, u[e].y);
        }
    } else if constexpr (RECON == 12) {
#pragma unroll
        for (int row = 0; row < 3; ++row) {
            link_set_real<LP>(w, 2 * row, u[3 * row].x);
            link_set_real<LP>(w, 2 * row + 1, u[3 * row].y);
            link_set_real<LP>(w, 6 + 2 * row, u[3 * row + 1].x);
            link_set_real<LP>(w, 6 + 2 * row + 1, u[3 * row + 1].y);
        }
    } else {
        const double2 a1 = u[0], a2 = u[3], a3 = u[6], b1 = u[1], c1 = u[2];
        const double n = a2.x * a2.x + a2.y * a2.y + a3.x * a3.x + a3.y * a3.y;
        if (!(n >= 1e-12)) *reinterpret_cast<volatile int*>(singular) = 1;
        link_set_real<LP>(w, 0, a2.x);
        link_set_real<LP>(w, 1, a2.y);
        link_set_real<LP>(w, 2, a3.x);
        link_set_real<LP>(w, 3, a3.y);
        link_set_real<LP>(w, 4, b1.x);
        link_set_real<LP>(w, 5, b1.y);
        link_set_real<LP>(w, 6, atan2(a1.y, a1.x));
        link_set_real<LP>(w, 7, atan2(c1.y, c1.x));
    }
    link_store_words<LP, RECON>(links, g.vh, p * 4 + mu, i, w);
}

// One lane per (parity, eo site, mu): decode link into canonical order.
template <int LP, int RECON>
__global__ void k_gauge_unpack(GeomK g, const char* __restrict__ links, double2* __restrict__ canon) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = blockIdx.y >> 2;
    const int mu = blockIdx.y & 3;
    if (i >= g.vh) return;
    const SiteCoord x = eo_coords(g, p, i);
    const int64_t lex = 2 * (int64_t)i + (x.x3 & 1);
    C<typename LinkReal<LP>::R> u[3][3];
    link_load<LP, RECON>(links, g.vh, p * 4 + mu, i, u);
    double2* dst = canon + (lex * 4 + mu) * 9;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) dst[3 * r + c] = make_double2((double)u[r][c].r, (double)u[r][c].i);
}

// One lane per (rhs, canonical site).  Full fields: canonical lexicographic
// site -> packed site p*V/2 + lex/2.  Parity fields: eo order on both sides.
template <int SP>
__global__ void k_spinor_pack(GeomK g, int full, int64_t nsites, int nrhs, const double2* __restrict__ canon,
                              SpinorView dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsites * nrhs) return;
    const int64_t rhs = t / nsites;
    const int64_t s = t - rhs * nsites;
    int64_t site = s;
    if (full) {
        const int64_t x3 = s % g.n3;
        const int64_t q = s / g.n3;
        const int64_t x2 = q % g.n2;
        const int64_t r = q / g.n2;
        const int64_t x1 = r % g.n1;
        const int64_t x0 = r / g.n1;
        const int p = (int)((x0 + x1 + x2 + x3) & 1);
        site = (int64_t)p * g.vh + (s >> 1);
    }
    using R = typename SpinorIO<SP>::R;
    C<R> c[12];
    const double2* src = canon + t * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = {(R)src[k].x, (R)src[k].y};
    SpinorView v = dst;
    v.base += rhs * dst.rhs_bytes;
    SpinorIO<SP>::store(v, site, c);
}

template <int SP>
__global__ void k_spinor_unpack(GeomK g, int full, int64_t nsites, int nrhs, SpinorView src,
                                double2* __restrict__ canon) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsites * nrhs) return;
    const int64_t rhs = t / nsites;
    const int64_t s = t - rhs * nsites;
    int64_t site = s;
    if (full) {
        const int64_t x3 = s % g.n3;
        const int64_t q = s / g.n3;
        const int64_t x2 = q % g.n2;
        const int64_t r = q / g.n2;
        const int64_t x1 = r % g.n1;
        const int64_t x0 = r / g.n1;
        const int p = (int)((x0 + x1 + x2 + x3) & 1);
        site = (int64_t)p * g.vh + (s >> 1);
    }
    using R = typename SpinorIO<SP>::R;
    C<R> c[12];
    SpinorView v = src;
    v.base += rhs * src.rhs_bytes;
    SpinorIO<SP>::load(v, site, c);
    double2* dst = canon + t * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) dst[k] = make_double2((double)c[k].r, (double)c[k].i);
}

template <int LP, int RECON>
int launch_gauge_pack(const ndq_geom* g, const void* canon, char* links, int* flag, hipStream_t st) {
    const int64_t n = 4 * g->volume;
    const int block = 256;
    hipLaunchKernelGGL((k_gauge_pack<LP, RECON>), dim3((unsigned)((n + block - 1) / block)), dim3(block), 0, st,
                       g->k, static_cast<const double2*>(canon), links, flag);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

template <int LP, int RECON>
int launch_gauge_unpack(const ndq_geom* g, const char* links, void* canon, hipStream_t st) {
    const int block = 256;
    hipLaunchKernelGGL((k_gauge_unpack<LP, RECON>), dim3((g->vh + block - 1) / block, 8), dim3(block), 0, st, g->k,
                       links, static_cast<double2*>(canon));
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

}  // namespace

extern "C" {

int ndq_gauge_pack(const ndq_geom* g, const void* d_canon, const ndq_gauge* dst, void* stream) {
    if (!g || !d_canon) return fail(NDQ_EINVAL, "ndq_gauge_pack: NULL argument");
    int rc = check_gauge(dst);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    char* links = static_cast<char*>(dst->data);
    // recon 8: the status word after the links (inside the caller's buffer,
    // see ndq_gauge_bytes) collects the singularity flag; lanes only store 1
    int* flag = nullptr;
    if (dst->recon == 8) {
        flag = reinterpret_cast<int*>(links + gauge_status_offset(g, dst->prec, dst->recon));
        NDQ_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
    }
    switch (dst->prec * 100 + dst->recon) {
        case NDQ_F64 * 100 + 18: rc = launch_gauge_pack<P64, 18>(g, d_canon, links, flag, st); break;
        case NDQ_F64 * 100 + 12: rc = launch_gauge_pack<P64, 12>(g, d_canon, links, flag, st); break;
        case NDQ_F64 * 100 + 8: rc = launch_gauge_pack<P64, 8>(g, d_canon, links, flag, st); break;
        case NDQ_F32 * 100 + 18: rc = launch_gauge_pack<P32, 18>(g, d_canon, links, flag, st); break;
        case NDQ_F32 * 100 + 12: rc = launch_gauge_pack<P32, 12>(g, d_canon, links, flag, st); break;
        case NDQ_F32 * 100 + 8: rc = launch_gauge_pack<P32, 8>(g, d_canon, links, flag, st); break;
        case NDQ_F16 * 100 + 18: rc = launch_gauge_pack<P16, 18>(g, d_canon, links, flag, st); break;
        case NDQ_F16 * 100 + 12: rc = launch_gauge_pack<P16, 12>(g, d_canon, links, flag, st); break;
        default: rc = fail(NDQ_EPREC, "ndq_gauge_pack: unsupported format");
    }
    if (flag && rc == NDQ_OK) {
        int h = 0;
        NDQ_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
        NDQ_HIP(hipStreamSynchronize(st));
        if (h) rc = fail(NDQ_ESINGULAR, "8-real links are singular where |a2|^2 + |a3|^2 < 1e-12 (e.g. U = 1)");
    }
    return rc;
}

int ndq_gauge_unpack(const ndq_geom* g, const ndq_gauge* src, void* d_canon, void* stream) {
    if (!g || !d_canon) return fail(NDQ_EINVAL, "ndq_gauge_unpack: NULL argument");
    int rc = check_gauge(src);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    const char* links = static_cast<const char*>(src->data);
    switch (src->prec * 100 + src->recon) {
        case NDQ_F64 * 100 + 18: return launch_gauge_unpack<P64, 18>(g, links, d_canon, st);
        case NDQ_F64 * 100 + 12: return launch_gauge_unpack<P64, 12>(g, links, d_canon, st);
        case NDQ_F64 * 100 + 8: return launch_gauge_unpack<P64, 8>(g, links, d_canon, st);
        case NDQ_F32 * 100 + 18: return launch_gauge_unpack<P32, 18>(g, links, d_canon, st);
        case NDQ_F32 * 100 + 12: return launch_gauge_unpack<P32, 12>(g, links, d_canon, st);
        case NDQ_F32 * 100 + 8: return launch_gauge_unpack<P32, 8>(g, links, d_canon, st);
        case NDQ_F16 * 100 + 18: return launch_gauge_unpack<P16, 18>(g, links, d_canon, st);
        case NDQ_F16 * 100 + 12: return launch_gauge_unpack<P16, 12>(g, links, d_canon, st);
        default: return fail(NDQ_EPREC, "ndq_gauge_unpack: unsupported format");
    }
}

int ndq_spinor_pack(const ndq_geom* g, const void* d_canon, const ndq_spinor* dst, void* stream) {
    if (!g || !d_canon) return fail(NDQ_EINVAL, "ndq_spinor_pack: NULL argument");
    int rc = check_spinor(g, dst, -1, "ndq_spinor_pack dst");
    if (rc) return rc;
    const int full = dst->parity == NDQ_FULL;
    const int64_t nsites = spinor_sites(g, dst->parity);
    const int64_t n = nsites * dst->nrhs;
    const int block = 256;
    const dim3 grid((unsigned)((n + block - 1) / block));
    const SpinorView v = view_of(g, dst, 0, 0);
    const double2* c = static_cast<const double2*>(d_canon);
    hipStream_t st = as_stream(stream);
    switch (dst->prec) {
        case NDQ_F64: hipLaunchKernelGGL(k_spinor_pack<P64>, grid, dim3(block), 0, st, g->k, full, nsites, dst->nrhs, c, v); break;
        case NDQ_F32: hipLaunchKernelGGL(k_spinor_pack<P32>, grid, dim3(block), 0, st, g->k, full, nsites, dst->nrhs, c, v); break;
        default: hipLaunchKernelGGL(k_spinor_pack<P16>, grid, dim3(block), 0, st, g->k, full, nsites, dst->nrhs, c, v); break;
    }
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

int ndq_spinor_unpack(const ndq_geom* g, const ndq_spinor* src, void* d_canon, void* stream) {
    if (!g || !d_canon) return fail(NDQ_EINVAL, "ndq_spinor_unpack: NULL argument");
    int rc = check_spinor(g, src, -1, "ndq_spinor_unpack src");
    if (rc) return rc;
    const int full = src->parity == NDQ_FULL;
    const int64_t nsites = spinor_sites(g, src->parity);
    const int64_t n = nsites * src->nrhs;
    const int block = 256;
    const dim3 grid((unsigned)((n + block - 1) / block));
    const SpinorView v = view_of(g, src, 0, 0);
    double2* c = static_cast<double2*>(d_canon);
    hipStream_t st = as_stream(stream);
    switch (src->prec) {
        case NDQ_F64: hipLaunchKernelGGL(k_spinor_unpack<P64>, grid, dim3(block), 0, st, g->k, full, nsites, src->nrhs, v, c); break;
        case NDQ_F32: hipLaunchKernelGGL(k_spinor_unpack<P32>, grid, dim3(block), 0, st, g->k, full, nsites, src->nrhs, v, c); break;
        default: hipLaunchKernelGGL(k_spinor_unpack<P16>, grid, dim3(block), 0, st, g->k, full, nsites, src->nrhs, v, c); break;
    }
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

}  // extern "C"
