// Host-side internals of libndq: the geometry handle, error reporting and
// helpers that turn ABI descriptors into kernel views.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>

#include "ndq.h"
#include "ndq_device.h"

struct ndq_geom {
    int32_t dims[4];
    int64_t volume;
    int32_t vh;
    ndq::GeomK k;
};

namespace ndq {

// Record a message for ndq_last_error() and return `status`.
int fail(int status, const char* fmt, ...);

#define NDQ_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::ndq::fail(NDQ_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                               __FILE__, __LINE__);                                          \
    } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int bytes_per_site(int prec) { return prec == NDQ_F64 ? 192 : prec == NDQ_F32 ? 96 : 52; }

inline int64_t spinor_sites(const ndq_geom* g, int parity) { return parity == NDQ_FULL ? g->volume : g->vh; }

inline int64_t spinor_rhs_bytes(const ndq_geom* g, int prec, int parity) {
    return spinor_sites(g, parity) * bytes_per_site(prec);
}

inline int link_bytes(int prec, int recon) { return recon * (prec == NDQ_F64 ? 8 : prec == NDQ_F32 ? 4 : 2); }

// Packed links: all 4V links, then (8-real links only) a 256-byte status area
// whose first int is the singularity flag of the last ndq_gauge_pack.
inline size_t gauge_status_offset(const ndq_geom* g, int prec, int recon) {
    return ((size_t)g->volume * 4 * link_bytes(prec, recon) + 255) & ~size_t(255);
}

// Validate a spinor descriptor; `want_parity` < 0 accepts any subset.
int check_spinor(const ndq_geom* g, const ndq_spinor* s, int want_parity, const char* name);
int check_gauge(const ndq_gauge* u);
// Spinor and link precisions must pair up: F64 with F64, F32/F16 with F32/F16.
int check_pair(const ndq_gauge* u, const ndq_spinor* s);

// View of right-hand side `rhs` of the parity-`p` half of a spinor field.
// For a parity field, p must equal its own parity.
inline SpinorView view_of(const ndq_geom* g, const ndq_spinor* s, int p, int rhs) {
    SpinorView v;
    const int64_t rb = spinor_rhs_bytes(g, s->prec, s->parity);
    v.base = static_cast<char*>(s->data) + rb * rhs;
    v.rhs_bytes = rb;
    if (s->parity == NDQ_FULL) {
        v.stride = (int32_t)g->volume;
        v.site0 = p * g->vh;
    } else {
        v.stride = g->vh;
        v.site0 = 0;
    }
    return v;
}

// Device scalar coefficient: value = f * (*d) if d != nullptr, else f.
struct Coef {
    double f;
    const double* d;
};

}  // namespace ndq
