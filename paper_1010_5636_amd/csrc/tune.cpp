// Launch autotuners of the stencil.
//
// ndq_autotune / ndq_autotune_q: the even/odd dslash (or the full Q) of one
// storage format on one lattice for every launch shape (one lane per site with
// 64/128/256-lane workgroups, or the direction split) with and without the XCD
// remap; records the fastest for that lattice, format and launch kind (other
// lattices keep the format's shape).
//
// ndq_autotune_mrhs: the work order of the multi-right-hand-side stencil
// (fields per workgroup, group order, tile chunk) for one lattice, format,
// number of fields and output parities; records the fastest for that key
// (ndq_set_mrhs_launch).  With NDQ_TUNE_CACHE naming a file, a key found
// there is applied without timing, and new results are appended to it.
//
// ndq_autotune_multi: the grid factor of the persistent multi-lattice launch
// for one set of jobs.
//
// All time back-to-back launches between two events on the caller's stream,
// on fields in the caller's workspace (the multi-lattice tuner: on the jobs'
// own fields).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "ndq_internal.h"
#include "wilson.h"

using namespace ndq;

namespace {

const int kBlocks[4] = {0, 64, 128, 256};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// One rotating set: links and the input and output spinors of a dslash (ny =
// 1: two half fields) or of Q (ny = 2: two full fields).
size_t set_spinor_bytes(const ndq_geom* g, int sprec, int ny) {
    return (size_t)spinor_rhs_bytes(g, sprec, ny == 2 ? NDQ_FULL : NDQ_EVEN);
}

int dslash_sets(const ndq_geom* g, const ndq_gauge* U, int sprec, int64_t rotate_bytes, int ny) {
    const size_t set_bytes = ndq_gauge_bytes(g, U->prec, U->recon) + 2 * set_spinor_bytes(g, sprec, ny);
    int nsets = rotate_bytes > 0 ? (int)((rotate_bytes + (int64_t)set_bytes - 1) / (int64_t)set_bytes) : 1;
    return std::max(1, std::min(nsets, 256));
}

size_t dslash_ws(const ndq_geom* g, const ndq_gauge* U, int sprec, int nsets, int ny) {
    const size_t lb = align256(ndq_gauge_bytes(g, U->prec, U->recon));
    const size_t sb = align256(set_spinor_bytes(g, sprec, ny));
    return (size_t)(nsets - 1) * lb + (size_t)nsets * 2 * sb + 256;
}

// Average microseconds of `reps` calls of launch(k) after `warm` untimed ones.
template <typename F>
int time_launches(F&& launch, int warm, int reps, hipStream_t st, hipEvent_t e0, hipEvent_t e1, double* us) {
    int rc;
    for (int k = 0; k < warm; ++k)
        if ((rc = launch(k))) return rc;
    NDQ_HIP(hipEventRecord(e0, st));
    for (int k = 0; k < reps; ++k)
        if ((rc = launch(k))) return rc;
    NDQ_HIP(hipEventRecord(e1, st));
    NDQ_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    NDQ_HIP(hipEventElapsedTime(&ms, e0, e1));
    *us = 1e3 * ms / reps;
    return NDQ_OK;
}

struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// ---- the on-disk cache of multi-RHS work orders ----------------------------
std::mutex g_cache_mu;

const char* cache_path() {
    const char* p = getenv("NDQ_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

bool cache_lookup(const ndq_geom* g, int sprec, int lprec, int recon, int nrhs, int ny, MrhsShape* s, double* us) {
    const char* path = cache_path();
    if (!path) return false;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        int d[4], sp, lp, rc, nr, y, rg, gm, ch, xcd, nt;
        double t;
        if (sscanf(line, "mrhs %d %d %d %d %d %d %d %d %d %d %d %d %d %d %lf", &d[0], &d[1], &d[2], &d[3], &sp, &lp,
                   &rc, &nr, &y, &rg, &gm, &ch, &xcd, &nt, &t) != 15)
            continue;
        if (d[0] == g->dims[0] && d[1] == g->dims[1] && d[2] == g->dims[2] && d[3] == g->dims[3] && sp == sprec &&
            lp == lprec && rc == recon && nr == nrhs && y == ny) {
            s->rg = rg;
            s->group_major = gm;
            s->chunk = ch;
            s->xcd_remap = xcd;
            s->link_nt = nt;
            *us = t;
            found = true;   // the last entry of a key wins
        }
    }
    fclose(f);
    return found;
}

void cache_store(const ndq_geom* g, int sprec, int lprec, int recon, int nrhs, int ny, const MrhsShape& s, double us) {
    const char* path = cache_path();
    if (!path) return;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "mrhs %d %d %d %d %d %d %d %d %d %d %d %d %d %d %.4f\n", g->dims[0], g->dims[1], g->dims[2], g->dims[3],
            sprec, lprec, recon, nrhs, ny, s.rg, s.group_major, s.chunk, s.xcd_remap, s.link_nt, us);
    fclose(f);
}

int check_format(const ndq_gauge* U, int sprec, const char* who) {
    int rc = check_gauge(U);
    if (rc) return rc;
    if (sprec < NDQ_F64 || sprec > NDQ_F16) return fail(NDQ_EPREC, "%s: bad spinor precision %d", who, sprec);
    if ((sprec == NDQ_F64) != (U->prec == NDQ_F64))
        return fail(NDQ_EPREC, "%s: F64 spinors go with F64 links, F32/F16 with F32/F16", who);
    return NDQ_OK;
}

}  // namespace

namespace {

int autotune_single(const ndq_geom* g, const ndq_gauge* U, int sprec, int reps, int64_t rotate_bytes, void* ws,
                    size_t ws_bytes, ndq_tune_result* out, void* stream, int ny) {
    const char* who = ny == 2 ? "ndq_autotune_q" : "ndq_autotune";
    if (!g || !out) return fail(NDQ_EINVAL, "%s: NULL argument", who);
    int rc = check_format(U, sprec, who);
    if (rc) return rc;
    if (reps < 1) return fail(NDQ_EINVAL, "%s: reps must be >= 1", who);
    hipStream_t st = as_stream(stream);
    const int nsets = dslash_sets(g, U, sprec, rotate_bytes, ny);
    const size_t need = dslash_ws(g, U, sprec, nsets, ny);
    if (!ws || ws_bytes < need) return fail(NDQ_ENOMEM, "%s: workspace too small (need %zu bytes)", who, need);
    const size_t lb = align256(ndq_gauge_bytes(g, U->prec, U->recon));
    const size_t sb = align256(set_spinor_bytes(g, sprec, ny));
    // set k: links (set 0 uses the caller's), two spinor fields
    std::vector<void*> links(nsets), fa(nsets), fb(nsets);
    char* p = static_cast<char*>(ws);
    for (int k = 0; k < nsets; ++k) {
        if (k == 0) {
            links[k] = U->data;
        } else {
            links[k] = p;
            p += lb;
            NDQ_HIP(hipMemcpyAsync(links[k], U->data, ndq_gauge_bytes(g, U->prec, U->recon), hipMemcpyDeviceToDevice, st));
        }
        fa[k] = p;
        p += sb;
        fb[k] = p;
        p += sb;
        // any finite pattern: 0x3c00 halves (1.0 in F16), a small number in F32/F64
        NDQ_HIP(hipMemsetD32Async(fa[k], 0x3c003c00u, sb / 4, st));
        NDQ_HIP(hipMemsetD32Async(fb[k], 0x3c003c00u, sb / 4, st));
    }
    Events ev;
    NDQ_HIP(hipEventCreate(&ev.e0));
    NDQ_HIP(hipEventCreate(&ev.e1));
    auto launch = [&](int k) -> int {
        const int s = k % nsets;
        const int par = (k / nsets) & 1;   // alternate the direction of the hop
        ndq_gauge u = *U;
        u.data = links[s];
        if (ny == 2) {
            ndq_spinor in{par ? fb[s] : fa[s], sprec, NDQ_FULL, 1};
            ndq_spinor o{par ? fa[s] : fb[s], sprec, NDQ_FULL, 1};
            return ndq_apply_Q(g, &u, -1.0, &in, &o, stream);
        }
        ndq_spinor in{par ? fb[s] : fa[s], sprec, par ? NDQ_ODD : NDQ_EVEN, 1};
        ndq_spinor o{par ? fa[s] : fb[s], sprec, par ? NDQ_EVEN : NDQ_ODD, 1};
        return ndq_apply_dslash(g, &u, &in, &o, stream);
    };
    const Tuning saved = launch_tuning(g->k, sprec, U->prec, U->recon, ny);
    memset(out, 0, sizeof(*out));
    double best = 1e300;
    int best_b = 0, best_x = 1;
    int best_o = 0;
    for (int o = 0; o < 2; ++o) {
        for (int b = 0; b < 4; ++b) {
            for (int x = 0; x < 2; ++x) {
                Tuning t;
                t.block = kBlocks[b];
                t.xcd_remap = x;
                t.order = o;
                set_launch_tuning(g->k, sprec, U->prec, U->recon, ny, t);
                double us = 0.0;
                if ((rc = time_launches(launch, std::min(8, 2 * nsets), reps, st, ev.e0, ev.e1, &us))) {
                    set_launch_tuning(g->k, sprec, U->prec, U->recon, ny, saved);
                    return rc;
                }
                (o ? out->us_order : out->us)[2 * b + x] = us;
                if (us < best) {
                    best = us;
                    best_b = kBlocks[b];
                    best_x = x;
                    best_o = o;
                }
            }
        }
    }
    // keep the shape in use unless another is more than 3% faster: shapes
    // within timing noise of each other should not flip from run to run
    int cur = 0;
    for (int b = 0; b < 4; ++b)
        if (kBlocks[b] == saved.block) cur = 2 * b + saved.xcd_remap;
    const double cur_us = (saved.order ? out->us_order : out->us)[cur];
    if (cur_us <= 1.03 * best) {
        best_b = saved.block;
        best_x = saved.xcd_remap;
        best_o = saved.order;
        best = cur_us;
    }
    Tuning t;
    t.block = best_b;
    t.xcd_remap = best_x;
    t.order = best_o;
    set_launch_tuning(g->k, sprec, U->prec, U->recon, ny, t);
    out->block = best_b;
    out->xcd_remap = best_x;
    out->order = best_o;
    out->us_best = best;
    out->nsets = nsets;
    return NDQ_OK;
}

}  // namespace

extern "C" size_t ndq_autotune_workspace_bytes(const ndq_geom* g, const ndq_gauge* U, int sprec, int64_t rotate_bytes) {
    if (!g || !U || check_gauge(U) || sprec < NDQ_F64 || sprec > NDQ_F16) return 0;
    return dslash_ws(g, U, sprec, dslash_sets(g, U, sprec, rotate_bytes, 1), 1);
}

extern "C" size_t ndq_autotune_q_workspace_bytes(const ndq_geom* g, const ndq_gauge* U, int sprec,
                                                 int64_t rotate_bytes) {
    if (!g || !U || check_gauge(U) || sprec < NDQ_F64 || sprec > NDQ_F16) return 0;
    return dslash_ws(g, U, sprec, dslash_sets(g, U, sprec, rotate_bytes, 2), 2);
}

extern "C" int ndq_autotune(const ndq_geom* g, const ndq_gauge* U, int sprec, int reps, int64_t rotate_bytes, void* ws,
                            size_t ws_bytes, ndq_tune_result* out, void* stream) {
    return autotune_single(g, U, sprec, reps, rotate_bytes, ws, ws_bytes, out, stream, 1);
}

extern "C" int ndq_autotune_q(const ndq_geom* g, const ndq_gauge* U, int sprec, int reps, int64_t rotate_bytes,
                              void* ws, size_t ws_bytes, ndq_tune_result* out, void* stream) {
    return autotune_single(g, U, sprec, reps, rotate_bytes, ws, ws_bytes, out, stream, 2);
}

extern "C" size_t ndq_autotune_mrhs_workspace_bytes(const ndq_geom* g, int sprec, int nrhs, int ny) {
    if (!g || sprec < NDQ_F64 || sprec > NDQ_F16 || nrhs < 2 || (ny != 1 && ny != 2)) return 0;
    const int par = ny == 2 ? NDQ_FULL : NDQ_EVEN;
    return 2 * align256((size_t)spinor_rhs_bytes(g, sprec, par) * nrhs) + 256;
}

extern "C" int ndq_autotune_mrhs(const ndq_geom* g, const ndq_gauge* U, int sprec, int nrhs, int ny, int reps, void* ws,
                                 size_t ws_bytes, ndq_mrhs_tune_result* out, void* stream) {
    if (!g || !out) return fail(NDQ_EINVAL, "ndq_autotune_mrhs: NULL argument");
    int rc = check_format(U, sprec, "ndq_autotune_mrhs");
    if (rc) return rc;
    if (nrhs < 2 || (ny != 1 && ny != 2) || reps < 1)
        return fail(NDQ_EINVAL, "ndq_autotune_mrhs: need nrhs >= 2, ny 1 or 2, reps >= 1");
    memset(out, 0, sizeof(*out));
    MrhsShape cached;
    double cached_us = 0.0;
    if (cache_lookup(g, sprec, U->prec, U->recon, nrhs, ny, &cached, &cached_us)) {
        set_mrhs_shape(g->k, sprec, U->prec, U->recon, nrhs, ny, cached);
        out->rg = cached.rg;
        out->group_major = cached.group_major;
        out->chunk = cached.chunk;
        out->xcd_remap = cached.xcd_remap;
        out->link_nt = cached.link_nt;
        out->us_best = cached_us;
        out->cached = 1;
        return NDQ_OK;
    }
    const size_t need = ndq_autotune_mrhs_workspace_bytes(g, sprec, nrhs, ny);
    if (!ws || ws_bytes < need) return fail(NDQ_ENOMEM, "ndq_autotune_mrhs: workspace too small (need %zu bytes)", need);
    hipStream_t st = as_stream(stream);
    const int par_in = ny == 2 ? NDQ_FULL : NDQ_ODD;
    const int par_out = ny == 2 ? NDQ_FULL : NDQ_EVEN;
    const size_t bb = align256((size_t)spinor_rhs_bytes(g, sprec, ny == 2 ? NDQ_FULL : NDQ_EVEN) * nrhs);
    char* p = static_cast<char*>(ws);
    ndq_spinor in{p, sprec, par_in, nrhs}, o{p + bb, sprec, par_out, nrhs};
    NDQ_HIP(hipMemsetD32Async(p, 0x3c003c00u, bb / 4, st));
    auto launch = [&](int) -> int {
        return ny == 2 ? ndq_apply_Q(g, U, -1.0, &in, &o, stream) : ndq_apply_dslash(g, U, &in, &o, stream);
    };
    // candidate orders: fields per workgroup, group order, tile chunk
    std::vector<int> rgs = {nrhs, (nrhs + 1) / 2, (nrhs + 2) / 3, 6, 4, 2};
    std::sort(rgs.begin(), rgs.end());
    rgs.erase(std::unique(rgs.begin(), rgs.end()), rgs.end());
    std::vector<int> chunks = {-1, 0};
    const MrhsShape dflt = default_mrhs_shape(g->k, sprec, U->prec, U->recon, nrhs, ny);
    if (dflt.chunk > 0) chunks.push_back(dflt.chunk);
    const MrhsShape saved = mrhs_shape(g->k, sprec, U->prec, U->recon, nrhs, ny);
    Events ev;
    NDQ_HIP(hipEventCreate(&ev.e0));
    NDQ_HIP(hipEventCreate(&ev.e1));
    double best = 1e300, saved_us = 1e300;
    MrhsShape bs = saved;
    int n = 0;
    auto trial = [&](const MrhsShape& s, double* us) -> int {
        set_mrhs_shape(g->k, sprec, U->prec, U->recon, nrhs, ny, s);
        return time_launches(launch, 2, reps, st, ev.e0, ev.e1, us);
    };
    if ((rc = trial(saved, &saved_us))) {
        set_mrhs_shape(g->k, sprec, U->prec, U->recon, nrhs, ny, saved);
        return rc;
    }
    best = saved_us;
    for (int rg : rgs) {
        if (rg > nrhs || rg < 1) continue;
        for (int gm = 0; gm < 2; ++gm) {
            if (rg == nrhs && gm) continue;
            for (int ch : chunks) {
                MrhsShape s;
                s.rg = rg;
                s.group_major = gm;
                s.chunk = ch;
                double us = 0.0;
                if ((rc = trial(s, &us))) {
                    set_mrhs_shape(g->k, sprec, U->prec, U->recon, nrhs, ny, saved);
                    return rc;
                }
                ++n;
                // a new order must beat the one in use by more than 3%
                if (us < best && us < saved_us / 1.03) {
                    best = us;
                    bs = s;
                }
            }
        }
    }
    set_mrhs_shape(g->k, sprec, U->prec, U->recon, nrhs, ny, bs);
    cache_store(g, sprec, U->prec, U->recon, nrhs, ny, bs, best);
    out->rg = bs.rg;
    out->group_major = bs.group_major;
    out->chunk = bs.chunk;
    out->xcd_remap = bs.xcd_remap;
    out->link_nt = bs.link_nt;
    out->us_best = best;
    out->us_previous = saved_us;
    out->nshapes = n;
    return NDQ_OK;
}

// ---- grid of the persistent multi-lattice launch ---------------------------

extern "C" int ndq_set_multi_grid(int factor) {
    if (factor < 1 || factor > 16) return fail(NDQ_EINVAL, "ndq_set_multi_grid: factor %d outside 1..16", factor);
    set_multi_grid_factor(factor);
    return NDQ_OK;
}

extern "C" int ndq_get_multi_grid(void) { return multi_grid_factor(); }

extern "C" int ndq_autotune_multi(const ndq_q_job* jobs, int32_t njobs, int reps, ndq_multi_tune_result* out,
                                  void* stream) {
    if (!out) return fail(NDQ_EINVAL, "ndq_autotune_multi: NULL result");
    if (reps < 1) return fail(NDQ_EINVAL, "ndq_autotune_multi: reps must be >= 1");
    memset(out, 0, sizeof(*out));
    hipStream_t st = as_stream(stream);
    const int saved = multi_grid_factor();
    // one launch first: checks the jobs before any timing
    int rc = ndq_apply_Q_multi(jobs, njobs, stream);
    if (rc) return rc;
    Events ev;
    NDQ_HIP(hipEventCreate(&ev.e0));
    NDQ_HIP(hipEventCreate(&ev.e1));
    auto launch = [&](int) -> int { return ndq_apply_Q_multi(jobs, njobs, stream); };
    const int factors[7] = {1, 2, 3, 4, 6, 8, 12};
    double saved_us = 0.0;
    set_multi_grid_factor(saved);
    if ((rc = time_launches(launch, 2, reps, st, ev.e0, ev.e1, &saved_us))) return rc;
    int best_f = saved;
    double best = saved_us;
    for (int k = 0; k < 7; ++k) {
        set_multi_grid_factor(factors[k]);
        double us = 0.0;
        if ((rc = time_launches(launch, 2, reps, st, ev.e0, ev.e1, &us))) {
            set_multi_grid_factor(saved);
            return rc;
        }
        out->us[k] = us;
        // a new factor must beat the one in use by more than 3%
        if (us < best && us < saved_us / 1.03) {
            best = us;
            best_f = factors[k];
        }
    }
    set_multi_grid_factor(best_f);
    out->factor = best_f;
    out->nfactors = 7;
    out->us_best = best;
    out->us_previous = saved_us;
    return NDQ_OK;
}
