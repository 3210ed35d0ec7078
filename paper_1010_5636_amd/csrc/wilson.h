// Launch interface of the Wilson stencil kernel (see wilson.hip).
#pragma once

#include <string.h>

#include "ndq_internal.h"

namespace ndq {

struct WilsonArgs {
    GeomK g;
    int p0;                    // parity of the output sites of grid row y = 0
    const char* links;
    SpinorView in[2];          // stencil input (parity 1 - p) per grid row
    SpinorView out[2];
    SpinorView self[2];        // same-site term (parity p)
    int has_self;
    double a_self, b_hop;
    int gamma5;
    Coef c0;
    Coef cv[3];
    SpinorView v[3][2];
    int nv;
    double* partials;          // per-block |out|^2 partial sums (nullptr: none)
    int xcd_remap;
    int order_c;               // tile order chunk (0: tiles in index order), see tile_order()
};

// Chunk c of the L2-friendly tile order for tiles of `block` sites on lattice g,
// or 0 when the lattice does not split into whole tiles per x0 slice.
int tile_order(const GeomK& g, int block);

// One lattice of a persistent multi-lattice launch of Q (NDQ_FULL fields):
// views per output parity y address right-hand side 0.
constexpr int kMaxJobs = 8;
struct QJob {
    GeomK g;
    const char* links;
    SpinorView in[2];     // parity 1 - y
    SpinorView self[2];   // parity y
    SpinorView out[2];    // parity y
    double a_self;        // 4 + m
    int nrhs;
    int tile0;            // first tile of this lattice in the joint list
    int tiles;            // tiles of 64 sites per parity
};
struct MultiArgs {
    QJob job[kMaxJobs];
    int njobs;
    int total;            // tiles over all lattices and both parities
};

// Launch shape of the stencil: block = 64/128/256 lanes with one lane per
// site, or 0 for the direction-split form; xcd_remap as in ndq_set_launch.
struct Tuning {
    int block = 0;
    int xcd_remap = 1;
    int order = 0;    // 1: tiles in the slice-chunked order of tile_order (autotuner only)
};
// Per storage format (spinor precision, link precision, recon index 0/1/2 for
// 18/12/8); set by ndq_set_launch / ndq_set_launch_for (the autotuner).
Tuning& tuning(int sprec, int lprec, int recon);
// The shape of one lattice and number of output parities (1: dslash, 2: Q):
// the autotuner's choice for that lattice if it made one, else the format's.
Tuning launch_tuning(const GeomK& g, int sprec, int lprec, int recon, int ny);
void set_launch_tuning(const GeomK& g, int sprec, int lprec, int recon, int ny, const Tuning& t);
void clear_launch_tuning(int sprec, int lprec, int recon);
inline int recon_index(int recon) { return recon == 18 ? 0 : recon == 12 ? 1 : 2; }

// Work order of the multi-right-hand-side stencil (see k_wilson_mrhs): rg
// right-hand sides per workgroup (0: all), group-major or tile-major order of
// the groups, tile-order chunk (-1: tile_order's choice, 0: index order), XCD
// remap.  Looked up per (lattice, spinor precision, link precision, recon,
// nrhs, output parities); set by ndq_set_mrhs_launch or the autotuner, else
// the default below.
struct MrhsShape {
    int rg = 0;
    int group_major = 0;
    int chunk = -1;
    int xcd_remap = 1;
    int link_nt = -1;    // links loaded with the non-temporal hint: -1 automatic, 0 no, 1 yes
};
MrhsShape mrhs_shape(const GeomK& g, int sprec, int lprec, int recon, int nrhs, int ny);
void set_mrhs_shape(const GeomK& g, int sprec, int lprec, int recon, int nrhs, int ny, const MrhsShape& s);
MrhsShape default_mrhs_shape(const GeomK& g, int sprec, int lprec, int recon, int nrhs, int ny);

WilsonArgs wilson_args(const ndq_geom* g, const ndq_gauge* U, int sprec);
int wilson_blocks(const ndq_geom* g, int block, int ny);
// block < 0: the shape and XCD remap of launch_tuning for this lattice and ny.
hipError_t launch_wilson(int sprec, int lprec, int recon, const WilsonArgs& a, int ny, int block, hipStream_t st);
// nrhs right-hand sides (a.in/out/self/v views point at rhs 0; rhs r at + r * rhs_bytes),
// links staged once in LDS; epilogue with up to 3 extra vectors, no partial sums.
hipError_t launch_wilson_multi(int sprec, int lprec, int recon, const MultiArgs& a, hipStream_t st);
// Workgroups of the persistent multi-lattice launch as a multiple of what the
// device holds at once (1..16; 4 unless set by ndq_set_multi_grid or the
// autotuner).
int multi_grid_factor();
void set_multi_grid_factor(int f);
hipError_t launch_wilson_mrhs(int sprec, int lprec, int recon, const WilsonArgs& a, int ny, int nrhs, hipStream_t st);

}  // namespace ndq
