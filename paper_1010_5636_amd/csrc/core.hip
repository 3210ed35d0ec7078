// Error reporting, geometry handles and index tables.
#include <stdio.h>
#include <string.h>

#include <new>

#include "ndq_internal.h"

namespace {
thread_local char g_last_error[512] = "";

ndq::FastDiv make_fastdiv(uint32_t d) {
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    const uint64_t num = 1ull << (31 + l);
    ndq::FastDiv f;
    f.m = (uint32_t)((num + d - 1) / d);
    f.s = 31 + l;
    return f;
}

// The multiply-shift identity holds for every n < 2^31; check it on the
// values the kernels can produce (all n below the lattice volume).
bool fastdiv_ok(ndq::FastDiv f, uint32_t d, uint32_t nmax) {
    const uint32_t probes[] = {0u, 1u, d - 1, d, d + 1, nmax / 2, nmax - 1, nmax};
    for (uint32_t n : probes)
        if (ndq::fdiv(n, f) != n / d) return false;
    for (uint32_t n = 0; n < nmax && n < (1u << 16); ++n)
        if (ndq::fdiv(n, f) != n / d) return false;
    return true;
}

// Index tables from the stencil's own index functions (one lane per eo site).
__global__ void k_geom_tables(ndq::GeomK g, int32_t* nb, int32_t* lex_of_eo, int32_t* nb_eo) {
    const int p = blockIdx.y;
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.vh) return;
    const ndq::SiteCoord x = ndq::eo_coords(g, p, i);
    int32_t n[8];
    ndq::eo_neighbours(g, i, x, n);
    const int32_t lex = 2 * i + (x.x3 & 1);
    if (lex_of_eo) lex_of_eo[(int64_t)p * g.vh + i] = lex;
    if (nb_eo) {
        for (int d = 0; d < 8; ++d) nb_eo[((int64_t)p * g.vh + i) * 8 + d] = n[d];
    }
    if (nb) {
        const int32_t x3p = (x.x3 + 1 == g.n3) ? 0 : x.x3 + 1;
        const int32_t x3m = (x.x3 == 0) ? g.n3 - 1 : x.x3 - 1;
        for (int d = 0; d < 8; ++d) {
            int32_t bit = x.x3 & 1;
            if (d == 3) bit = x3p & 1;
            if (d == 7) bit = x3m & 1;
            nb[(int64_t)lex * 8 + d] = 2 * n[d] + bit;
        }
    }
}
}  // namespace

namespace ndq {

int fail(int status, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return status;
}

int check_gauge(const ndq_gauge* u) {
    if (!u || !u->data) return fail(NDQ_EINVAL, "gauge field: NULL descriptor or data");
    if (u->prec < NDQ_F64 || u->prec > NDQ_F16) return fail(NDQ_EPREC, "gauge field: bad precision %d", u->prec);
    if (u->recon != 18 && u->recon != 12 && u->recon != 8)
        return fail(NDQ_EPREC, "gauge field: recon must be 18, 12 or 8 (got %d)", u->recon);
    if (u->prec == NDQ_F16 && u->recon == 8) return fail(NDQ_EPREC, "gauge field: F16 storage supports recon 18 and 12");
    return NDQ_OK;
}

int check_spinor(const ndq_geom* g, const ndq_spinor* s, int want_parity, const char* name) {
    if (!s || !s->data) return fail(NDQ_EINVAL, "%s: NULL descriptor or data", name);
    if (s->prec < NDQ_F64 || s->prec > NDQ_F16) return fail(NDQ_EPREC, "%s: bad precision %d", name, s->prec);
    if (s->parity < NDQ_EVEN || s->parity > NDQ_FULL) return fail(NDQ_EINVAL, "%s: bad parity %d", name, s->parity);
    if (want_parity >= 0 && s->parity != want_parity)
        return fail(NDQ_EINVAL, "%s: expected parity %d, got %d", name, want_parity, s->parity);
    if (s->nrhs < 1 || s->nrhs > 4096) return fail(NDQ_EINVAL, "%s: nrhs must be in [1, 4096] (got %d)", name, s->nrhs);
    (void)g;
    return NDQ_OK;
}

int check_pair(const ndq_gauge* u, const ndq_spinor* s) {
    const bool l64 = u->prec == NDQ_F64, s64 = s->prec == NDQ_F64;
    if (l64 != s64) return fail(NDQ_EPREC, "F64 links need F64 spinors and vice versa");
    return NDQ_OK;
}

}  // namespace ndq

extern "C" {

const char* ndq_last_error(void) { return g_last_error; }

const char* ndq_status_string(int status) {
    switch (status) {
        case NDQ_OK: return "ok";
        case NDQ_EINVAL: return "invalid argument";
        case NDQ_EDIMS: return "invalid lattice dimensions";
        case NDQ_EPREC: return "unsupported precision or reconstruction";
        case NDQ_ENOMEM: return "workspace too small";
        case NDQ_ESINGULAR: return "singular input";
        case NDQ_ENOCONV: return "no convergence";
        case NDQ_ENAN: return "NaN or Inf encountered";
        case NDQ_EHIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char* ndq_version(void) { return "ndq 0.1 gfx950"; }

int ndq_geom_create(const int32_t dims[4], ndq_geom** out) {
    if (!dims || !out) return ndq::fail(NDQ_EINVAL, "ndq_geom_create: NULL argument");
    int64_t v = 1;
    for (int d = 0; d < 4; ++d) {
        if (dims[d] < 2 || (dims[d] & 1) || dims[d] > (1 << 20))
            return ndq::fail(NDQ_EDIMS, "extent %d of dimension %d must be even and in [2, 2^20]", dims[d], d);
        v *= dims[d];
    }
    if (v >= (int64_t(1) << 30)) return ndq::fail(NDQ_EDIMS, "volume %lld must be below 2^30", (long long)v);
    ndq_geom* g = new (std::nothrow) ndq_geom;
    if (!g) return ndq::fail(NDQ_EINVAL, "out of host memory");
    memcpy(g->dims, dims, sizeof(g->dims));
    g->volume = v;
    g->vh = (int32_t)(v / 2);
    ndq::GeomK& k = g->k;
    k.n0 = dims[0];
    k.n1 = dims[1];
    k.n2 = dims[2];
    k.n3 = dims[3];
    k.nh3 = dims[3] / 2;
    k.s1 = dims[2] * k.nh3;
    k.s0 = dims[1] * k.s1;
    k.vh = g->vh;
    k.d_nh3 = make_fastdiv((uint32_t)k.nh3);
    k.d_n2 = make_fastdiv((uint32_t)k.n2);
    k.d_n1 = make_fastdiv((uint32_t)k.n1);
    if (!fastdiv_ok(k.d_nh3, k.nh3, (uint32_t)g->vh) || !fastdiv_ok(k.d_n2, k.n2, (uint32_t)g->vh) ||
        !fastdiv_ok(k.d_n1, k.n1, (uint32_t)g->vh)) {
        delete g;
        return ndq::fail(NDQ_EDIMS, "internal: division constants failed their self-check");
    }
    *out = g;
    return NDQ_OK;
}

void ndq_geom_destroy(ndq_geom* g) { delete g; }

int64_t ndq_geom_volume(const ndq_geom* g) { return g ? g->volume : 0; }

int ndq_geom_tables(const ndq_geom* g, int32_t* d_nb, int32_t* d_lex_of_eo, int32_t* d_nb_eo, void* stream) {
    if (!g) return ndq::fail(NDQ_EINVAL, "ndq_geom_tables: NULL geometry");
    const int block = 256;
    dim3 grid((g->vh + block - 1) / block, 2);
    hipLaunchKernelGGL(k_geom_tables, grid, dim3(block), 0, ndq::as_stream(stream), g->k, d_nb, d_lex_of_eo, d_nb_eo);
    NDQ_HIP(hipGetLastError());
    return NDQ_OK;
}

size_t ndq_gauge_bytes(const ndq_geom* g, int prec, int recon) {
    if (!g || prec < NDQ_F64 || prec > NDQ_F16 || (recon != 18 && recon != 12 && recon != 8)) return 0;
    if (recon == 8) return ndq::gauge_status_offset(g, prec, recon) + 256;
    return (size_t)g->volume * 4 * ndq::link_bytes(prec, recon);
}

size_t ndq_spinor_bytes(const ndq_geom* g, int prec, int parity, int nrhs) {
    if (!g || prec < NDQ_F64 || prec > NDQ_F16 || parity < NDQ_EVEN || parity > NDQ_FULL || nrhs < 1) return 0;
    return (size_t)ndq::spinor_rhs_bytes(g, prec, parity) * (size_t)nrhs;
}

}  // extern "C"

#include "wilson.h"

#include <map>
#include <mutex>
#include <tuple>

namespace ndq {
namespace {
Tuning g_tuning[3][3][3];

using MrhsKey = std::tuple<int, int, int, int, int, int, int, int, int, int>;
std::mutex g_mrhs_mu;
std::map<MrhsKey, MrhsShape> g_mrhs;

MrhsKey mrhs_key(const GeomK& g, int sprec, int lprec, int recon, int nrhs, int ny) {
    return MrhsKey{g.n0, g.n1, g.n2, g.n3, sprec, lprec, recon, nrhs, ny, 0};
}
}  // namespace

Tuning& tuning(int sprec, int lprec, int recon) { return g_tuning[sprec][lprec][recon_index(recon)]; }

namespace {
using LaunchKey = std::tuple<int, int, int, int, int, int, int, int>;
std::mutex g_launch_mu;
std::map<LaunchKey, Tuning> g_launch;
LaunchKey launch_key(const GeomK& g, int sprec, int lprec, int recon, int ny) {
    return LaunchKey{g.n0, g.n1, g.n2, g.n3, sprec, lprec, recon, ny};
}
}  // namespace

Tuning launch_tuning(const GeomK& g, int sprec, int lprec, int recon, int ny) {
    std::lock_guard<std::mutex> lock(g_launch_mu);
    const auto it = g_launch.find(launch_key(g, sprec, lprec, recon, ny));
    if (it != g_launch.end()) return it->second;
    return tuning(sprec, lprec, recon);
}

void set_launch_tuning(const GeomK& g, int sprec, int lprec, int recon, int ny, const Tuning& t) {
    std::lock_guard<std::mutex> lock(g_launch_mu);
    g_launch[launch_key(g, sprec, lprec, recon, ny)] = t;
}

void clear_launch_tuning(int sprec, int lprec, int recon) {
    std::lock_guard<std::mutex> lock(g_launch_mu);
    for (auto it = g_launch.begin(); it != g_launch.end();) {
        const LaunchKey& k = it->first;
        if (std::get<4>(k) == sprec && std::get<5>(k) == lprec && std::get<6>(k) == recon) it = g_launch.erase(it);
        else ++it;
    }
}

// Defaults from a sweep of the work order on 24^3x48 and 32^3x64 (12 and 60
// fields): blocks of 8 or more F32/F64 fields run in group-major order with 6
// fields per workgroup, and the tiles in chunks spanning two x1 rows of the
// slice (the smallest divisor c of the slice's tiles with 64 c >= 2 s1), so
// that the neighbour spinors of nearby tiles are still in L2 when re-read.
// F16 fields (half the bytes per field) keep one group in tile order.
MrhsShape default_mrhs_shape(const GeomK& g, int sprec, int lprec, int recon, int nrhs, int ny) {
    (void)lprec; (void)recon; (void)ny;
    MrhsShape s;
    if (nrhs >= 8 && sprec != P16) {
        s.rg = 6;
        s.group_major = 1;
        const int64_t per_slice = g.vh / g.n0;
        if (g.n0 >= 4 && per_slice * g.n0 == g.vh && per_slice % 64 == 0) {
            const int64_t S = per_slice / 64;
            for (int64_t c = 1; c <= S; ++c) {
                if (S % c == 0 && 64 * c >= 2 * (int64_t)g.s1) {
                    s.chunk = (int)c;
                    break;
                }
            }
        }
    }
    return s;
}

MrhsShape mrhs_shape(const GeomK& g, int sprec, int lprec, int recon, int nrhs, int ny) {
    std::lock_guard<std::mutex> lock(g_mrhs_mu);
    const auto it = g_mrhs.find(mrhs_key(g, sprec, lprec, recon, nrhs, ny));
    if (it != g_mrhs.end()) return it->second;
    return default_mrhs_shape(g, sprec, lprec, recon, nrhs, ny);
}

void set_mrhs_shape(const GeomK& g, int sprec, int lprec, int recon, int nrhs, int ny, const MrhsShape& s) {
    std::lock_guard<std::mutex> lock(g_mrhs_mu);
    g_mrhs[mrhs_key(g, sprec, lprec, recon, nrhs, ny)] = s;
}
}  // namespace ndq

extern "C" int ndq_set_mrhs_launch(const ndq_geom* g, int sprec, int lprec, int recon, int nrhs, int ny, int rg,
                                   int group_major, int chunk, int xcd_remap, int link_nt) {
    if (!g || sprec < NDQ_F64 || sprec > NDQ_F16 || lprec < NDQ_F64 || lprec > NDQ_F16 ||
        (recon != 18 && recon != 12 && recon != 8) || nrhs < 1 || (ny != 1 && ny != 2) || rg < 0 || chunk < -1)
        return ndq::fail(NDQ_EINVAL, "ndq_set_mrhs_launch: bad argument");
    if (chunk > 0) {
        const int64_t per_slice = g->k.vh / g->k.n0;
        if (g->k.n0 < 2 || per_slice * g->k.n0 != g->k.vh || per_slice % 64 || (per_slice / 64) % chunk)
            return ndq::fail(NDQ_EINVAL, "ndq_set_mrhs_launch: chunk %d does not divide the 64-site tiles of a time slice",
                             chunk);
    }
    ndq::MrhsShape s;
    s.rg = rg;
    s.group_major = group_major == 2 ? 2 : group_major ? 1 : 0;
    s.chunk = chunk;
    s.xcd_remap = xcd_remap ? 1 : 0;
    s.link_nt = link_nt < 0 ? -1 : (link_nt ? 1 : 0);
    ndq::set_mrhs_shape(g->k, sprec, lprec, recon, nrhs, ny, s);
    return NDQ_OK;
}

extern "C" int ndq_get_mrhs_launch(const ndq_geom* g, int sprec, int lprec, int recon, int nrhs, int ny, int* rg,
                                   int* group_major, int* chunk, int* xcd_remap, int* link_nt) {
    if (!g || !rg || !group_major || !chunk || !xcd_remap || !link_nt)
        return ndq::fail(NDQ_EINVAL, "ndq_get_mrhs_launch: NULL argument");
    const ndq::MrhsShape s = ndq::mrhs_shape(g->k, sprec, lprec, recon, nrhs, ny);
    *rg = s.rg;
    *group_major = s.group_major;
    *chunk = s.chunk;
    *xcd_remap = s.xcd_remap;
    *link_nt = s.link_nt;
    return NDQ_OK;
}

extern "C" int ndq_set_launch_for(int sprec, int lprec, int recon, int block, int xcd_remap) {
    if (sprec < NDQ_F64 || sprec > NDQ_F16 || lprec < NDQ_F64 || lprec > NDQ_F16 ||
        (recon != 18 && recon != 12 && recon != 8))
        return ndq::fail(NDQ_EINVAL, "ndq_set_launch_for: bad format (%d, %d, %d)", sprec, lprec, recon);
    if (block != 0 && block != 64 && block != 128 && block != 256)
        return ndq::fail(NDQ_EINVAL, "ndq_set_launch_for: block must be 0, 64, 128 or 256 (got %d)", block);
    ndq::Tuning& t = ndq::tuning(sprec, lprec, recon);
    t.block = block;
    t.xcd_remap = xcd_remap ? 1 : 0;
    ndq::clear_launch_tuning(sprec, lprec, recon);   // an explicit shape replaces tuned ones
    return NDQ_OK;
}

extern "C" int ndq_get_launch_for(int sprec, int lprec, int recon, int* block, int* xcd_remap) {
    if (sprec < NDQ_F64 || sprec > NDQ_F16 || lprec < NDQ_F64 || lprec > NDQ_F16 ||
        (recon != 18 && recon != 12 && recon != 8) || !block || !xcd_remap)
        return ndq::fail(NDQ_EINVAL, "ndq_get_launch_for: bad format (%d, %d, %d) or NULL output", sprec, lprec, recon);
    const ndq::Tuning& t = ndq::tuning(sprec, lprec, recon);
    *block = t.block;
    *xcd_remap = t.xcd_remap;
    return NDQ_OK;
}

extern "C" int ndq_set_launch(int block, int xcd_remap) {
    if (block != 0 && block != 64 && block != 128 && block != 256)
        return ndq::fail(NDQ_EINVAL, "ndq_set_launch: block must be 0, 64, 128 or 256 (got %d)", block);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int r : {18, 12, 8}) ndq_set_launch_for(a, b, r, block, xcd_remap);
    return NDQ_OK;
}

extern "C" int ndq_get_launch_lattice(const ndq_geom* g, int sprec, int lprec, int recon, int ny, int* block,
                                      int* xcd_remap) {
    if (!g || sprec < NDQ_F64 || sprec > NDQ_F16 || lprec < NDQ_F64 || lprec > NDQ_F16 ||
        (recon != 18 && recon != 12 && recon != 8) || (ny != 1 && ny != 2) || !block || !xcd_remap)
        return ndq::fail(NDQ_EINVAL, "ndq_get_launch_lattice: bad argument");
    const ndq::Tuning t = ndq::launch_tuning(g->k, sprec, lprec, recon, ny);
    *block = t.block;
    *xcd_remap = t.xcd_remap;
    return NDQ_OK;
}
