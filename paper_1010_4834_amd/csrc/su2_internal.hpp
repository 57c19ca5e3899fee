// su2_internal.hpp -- kernel argument block and launcher declarations shared
// by the kernels (su2_kernels.hip) and the C-ABI host code (su2_api.hip).
#pragma once

#include "su2_device.hpp"

namespace su2 {

// Arguments common to the lattice kernels (passed by value).
struct KArgs {
    const LatDesc *desc;                 // per-lattice descriptors
    const Tile *tiles;                   // (lattice, first index) work list
    int ntiles;
    int xcd_remap;
    void *links;                         // native link buffer
    DevState *st;                        // seed / sweep counter
    unsigned int *err;                   // sampler try-cap hits (&st->err)
    uint32_t *trace;                     // per-link try record or null
    unsigned long long *tries_part;      // per-tile try counts
    double *plaq_part;                   // per-sweep-slot tile plaquette sums
    int sampler;                         // 0 hybrid, 1 Creutz
    int advance;                         // heat bath: substeps of whole sweeps (advance the counter)
    int nslots;                          // series slots of the partial buffers (0: no series)
    int every;                           // series: one measured sweep per `every` sweeps (>= 1)
};

// Optional timing events stamped by the launch itself (both null: none).
struct Ev {
    hipEvent_t a = nullptr, b = nullptr;
};

void launch_heatbath(const KArgs &a, bool f32, int mu, int par, int nl, int block, int grid, hipStream_t s,
                     bool trace, bool plaq, const Ev &ev = Ev{});
// Workgroups of `block` threads the heat-bath substep kernels keep resident
// per compute unit (the smallest over the four directions), 0 if unknown.
int heatbath_blocks_per_cu(bool f32, int nl, int block);
void launch_overrelax(const KArgs &a, bool f32, int mu, int par, int block, int grid, hipStream_t s,
                      const Ev &ev = Ev{});
void launch_init(const KArgs &a, bool f32, int hot, int block, int grid, hipStream_t s);
void launch_from_canon(const KArgs &a, bool f32, const double *canon, int block, hipStream_t s);
void launch_to_canon(const KArgs &a, bool f32, const void *src, int ndir, double *canon, int block,
                     hipStream_t s);
void launch_unit_defect(const KArgs &a, bool f32, unsigned long long *out, int block, hipStream_t s);
void launch_plaquette(const KArgs &a, bool f32, double *part, int block, int grid, hipStream_t s);
// Polyakov partials: one (hi, lo) pair per spatial tile; with a.nslots > 0
// they go to series slot ((sweep - run_base) / every) % nslots (2 * ntiles
// doubles per slot).
void launch_polyakov(const KArgs &a, bool f32, double *part, int block, int grid, hipStream_t s);
// Final reduction of the standalone measurements: `chunks` workgroups per
// lattice, cnt[nlat] arrival tickets (zero between launches), chunk scratch
// of 6 doubles per workgroup.  pp: k_plaquette partials (4 per tile) ->
// outp[l * ostride + 0..2] = (avg, spatial, temporal); pl: Polyakov
// partials -> outl[l * ostride].
void launch_finalize(const LatDesc *desc, int nlat, int chunks, const double *pp, const double *pl,
                     unsigned *cnt, double *chunk, double *outp, double *outl, long long ostride, hipStream_t s);
// Series values of nsw consecutive measured sweeps, slots slot0 .. slot0 +
// nsw - 1 (mod nslots): plaquette from the heat-bath partials (12 doubles
// per heat-bath tile per slot: 3 planes x 4 wavefronts, unused entries zero;
// slot stride pp_stride doubles) and Polyakov loop from the Polyakov
// partials (slot stride pl_stride); either may be null.  Two launches: C
// chunk sums per (lattice, sweep) into `chunk` (6 doubles each, nlat * nsw *
// C of them), then one fixed-order sum per (lattice, sweep) written to
// outp / outl[l * ostride + out0 + j] for sweep j of the batch.
void launch_series(const LatDesc *desc, int nlat, const double *pp, long long pp_stride, const double *pl,
                   long long pl_stride, int slot0, int nslots, int nsw, int C, double *chunk, double *outp,
                   double *outl, long long ostride, int out0, hipStream_t s);
// Seed, sweep word (also the `next` word) and series base of the device
// state, set by a one-thread kernel so that no host synchronisation is
// needed before the work that reads them (the error word is left alone).
void launch_set_state(DevState *st, unsigned long long seed, unsigned sweep, unsigned run_base, hipStream_t s);
void launch_set_state_mapped(DevState *st, const unsigned *src, hipStream_t s);
// Zero the error word.
void launch_clear_err(DevState *st, hipStream_t s);
// Copy the error word to `out` (mapped host memory).
void launch_err_to_host(const DevState *st, unsigned *out, hipStream_t s);
void launch_ape(const KArgs &a, bool f32, const void *src, int src_raw, void *dst, double alpha, int block,
                int grid, hipStream_t s);
void launch_wlines(const KArgs &a, bool f32, const void *sp, int sp_raw, int Rmax, void *sl, int block,
                   hipStream_t s);
void launch_wtrace(const KArgs &a, bool f32, int Rmax, int Tmax, long long V, int Nt, const void *sl, double *part,
                   int block, hipStream_t s);
// Workgroups per R of the Wilson-loop trace launch (its partials per R).
int wtrace_groups(const KArgs &a);
void launch_wfinal(const LatDesc *desc, int nparts, int Rmax, int Tmax, const double *part, double *out,
                   hipStream_t s);

}  // namespace su2
