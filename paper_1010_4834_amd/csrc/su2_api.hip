// su2_api.hip -- C ABI of the SU(2) library (include/su2.h): handles,
// validation, device memory, tile tables, graph capture of whole runs and
// of sweep units, per-kernel event timing, launch-shape autotuning and
// checkpoints.
//
// A lattice is an ensemble of one: every kernel walks the (lattice, tile)
// list of its handle, so the batched and the single-lattice paths are the
// same kernels.
#include "su2_internal.hpp"

#include "../../include/su2.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include <sys/types.h>

using su2::DevState;
using su2::KArgs;
using su2::LatDesc;
using su2::Tile;

namespace {

// Sweeps per captured unit graph at most, for runs too long for one run
// graph (SU2_GRAPH_SWEEPS overrides; 0 or 1 replays single-sweep graphs
// only).  Each graph launch leaves the GPU idle for a few microseconds
// before its first kernel, so such a run replays as many graphs of this
// size as fit and then at most one graph of each smaller power of two
// (300 sweeps: eighteen of 16, then 8 + 4).
constexpr int GRAPH_SWEEPS_DEFAULT = 16;
int graph_sweeps() {
    static const int n = [] {
        const char *e = std::getenv("SU2_GRAPH_SWEEPS");
        return e ? std::max(0, std::min(4096, std::atoi(e))) : GRAPH_SWEEPS_DEFAULT;
    }();
    return n;
}
// Largest lattice per precision.  Kernels address a link inside its
// (mu, parity) block with a 32-bit byte offset: cb * 16 in binary32 (below
// 8 V bytes) and up to cb * 16 + 16 vh in binary64 (below 16 V bytes, the
// (a2,a3) plane), so V <= 2^29 (binary32) and V <= 2^28 (binary64) keep every
// offset below 2^32.
constexpr long long MAX_SITES_F32 = 1LL << 29;
constexpr long long MAX_SITES_F64 = 1LL << 28;

struct EventPair {
    int kind;
    hipEvent_t a, b;
};

}  // namespace

struct su2_ensemble_s {
    int n = 0;
    bool f32 = true;
    int sampler = 0;
    int device = 0;
    bool failed = false;

    std::vector<LatDesc> hdesc;
    LatDesc *ddesc = nullptr;
    long long total_links = 0;  // 4 * sum V
    long long total_sites = 0;

    int block = 256, grid = 0, remap = 1, nl = 1;
    std::vector<Tile> htiles, hstiles, hvtiles, hmtiles, hmtiles_z, hmtiles_b, hmtiles_b3;
    Tile *tiles = nullptr, *stiles = nullptr, *vtiles = nullptr, *mtiles = nullptr;
    Tile *mtiles_z = nullptr;  // the heat-bath tiles of each lattice in (z, t, y, x) order
    // tile mode 3: the heat-bath tiles in eight blocks per lattice, (z half,
    // t quarter) for mu < 3 and (z quarter, y half) for mu = 3
    Tile *mtiles_b = nullptr, *mtiles_b3 = nullptr;
    int ntiles = 0, nstiles = 0, nvtiles = 0, nmtiles = 0;

    void *links = nullptr;
    bool own_links = true;
    size_t link_bytes = 0;

    DevState *st = nullptr;
    DevState hst{};
    unsigned long long *tries_part = nullptr;
    unsigned long long tries_acc = 0;  // folded from tries_part on reshapes
    unsigned long long updates = 0;

    double *part_plaq = nullptr, *part_poly = nullptr, *part_hb = nullptr;
    int nslots = 1;                 // per-sweep slots of part_hb / part_poly (series batches)
    unsigned *fin_cnt = nullptr;    // per-lattice arrival tickets of the final reduction
    double *fin_chunk = nullptr;    // per-workgroup chunk sums of the final reduction
    int fin_chunks = 1;             // workgroups per lattice in the final reduction
    double *res = nullptr;   // device scratch for single results
    double *hres = nullptr;  // pinned host mirror of res

    int ser_C = 1;                  // chunks per (lattice, sweep) of the series reduction
    double *ser_chunk = nullptr;    // their (hi, lo) pairs
    // Series values and the error word are written by kernels straight into
    // mapped, coherent pinned host memory (device addresses dser, derr), so
    // a call ends with one synchronisation and no copy.
    double *hser = nullptr, *dser = nullptr;
    size_t hser_cap = 0;            // doubles
    double *run_plaq = nullptr, *run_poly = nullptr;  // device targets of the current run
    int run_nm = 0;
    // mapped host words: [0] the error word written by the device, [4..7]
    // the run state (seed low and high, sweep, run base) written by the host
    // for the first node of a captured run
    unsigned *herr = nullptr, *derr = nullptr;

    hipStream_t own = nullptr, user = nullptr;
    // captured sweep graphs by (measurement mask, sweeps per measurement,
    // measured units per graph)
    std::map<unsigned long long, hipGraphExec_t> graphs;
    // whole runs captured as one graph (sweeps, series reduction, error
    // word) by (measurement mask, sweeps per measurement, sweeps)
    std::map<unsigned long long, hipGraphExec_t> run_graphs;

    void *sm[2] = {nullptr, nullptr};
    int sm_cur = -1;  // index of the valid smeared buffer, -1 none

    void *wl_s = nullptr;  // spatial lines of the Wilson loops
    size_t wl_s_bytes = 0;
    double *wpart = nullptr;
    size_t wpart_bytes = 0;

    uint32_t *trace = nullptr;

    bool timing = false;
    std::vector<EventPair> pending;
    std::vector<hipEvent_t> evpool;
    double tms[SU2_K_COUNT] = {};
    long long tcount[SU2_K_COUNT] = {};

    hipStream_t stream() const { return user ? user : own; }
};

struct su2_lattice_s : su2_ensemble_s {};

namespace {

#define HIPCHK(expr)                                  \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) {                       \
            E->failed = true;                         \
            if (std::getenv("SU2_LOG"))               \
                std::fprintf(stderr, "su2: %s failed: %s (%s:%d)\n", #expr, \
                             hipGetErrorString(e_), __FILE__, __LINE__); \
            return SU2_EDEVICE;                       \
        }                                             \
    } while (0)

#define CHK(st_expr)                   \
    do {                               \
        su2_status s_ = (st_expr);     \
        if (s_ != SU2_OK) return s_;   \
    } while (0)

size_t link_size(bool f32) { return f32 ? 16 : 32; }

bool dims_ok(const int *d, bool f32) {
    for (int k = 0; k < 4; ++k)
        if (d[k] < 2 || (d[k] & 1)) return false;
    long long V = (long long)d[0] * d[1] * d[2] * d[3];
    // site decompositions multiply quotients and divisors back with 24-bit
    // products; the largest quotient is Ny Nz Nt, the largest divisor Nx
    if ((long long)d[1] * d[2] * d[3] >= (1LL << 24) || d[0] >= (1 << 24)) return false;
    return V <= (f32 ? MAX_SITES_F32 : MAX_SITES_F64);
}

// 1/d rounded up to the next binary64, the reciprocal the device division
// helper needs to truncate to floor(n/d) without a correction step.
double recip_up(int d) { return std::nextafter(1.0 / d, HUGE_VAL); }

// Host buffers sized by the caller or by the lattice: an allocation failure
// becomes ENOMEM instead of an exception crossing the C ABI.
template <class T> su2_status host_buf(std::vector<T> &v, size_t n) {
    try {
        v.resize(n);
    } catch (const std::bad_alloc &) {
        return SU2_ENOMEM;
    } catch (const std::length_error &) {
        return SU2_ENOMEM;
    }
    return SU2_OK;
}

su2_status enter(su2_ensemble_s *E) {
    if (!E) return SU2_EINVAL;
    if (E->failed) return SU2_ESTATE;
    if (hipSetDevice(E->device) != hipSuccess) {
        E->failed = true;
        return SU2_EDEVICE;
    }
    return SU2_OK;
}

template <class P>
su2_status dalloc(su2_ensemble_s *E, P **p, size_t bytes) {
    if (*p) {
        if (hipFree(*p) != hipSuccess) { E->failed = true; return SU2_EDEVICE; }
        *p = nullptr;
    }
    if (bytes == 0) return SU2_OK;
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        *p = nullptr;
        return SU2_ENOMEM;
    }
    if (e != hipSuccess) { E->failed = true; return SU2_EDEVICE; }
    return SU2_OK;
}

// Mapped, coherent pinned host memory of `bytes` and its device address.
su2_status host_mapped(su2_ensemble_s *E, void **host, void **dev, size_t bytes) {
    (void)E;
    *host = *dev = nullptr;
    if (hipHostMalloc(host, bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        *host = nullptr;
        return SU2_ENOMEM;
    }
    if (hipHostGetDevicePointer(dev, *host, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(*host);
        *host = nullptr;
        return SU2_ENOMEM;
    }
    return SU2_OK;
}

// A device buffer or event pair owned by one call, released on every return
// path (errors included).
template <class P> struct TmpDev {
    P *p = nullptr;
    TmpDev() = default;
    TmpDev(const TmpDev &) = delete;
    TmpDev &operator=(const TmpDev &) = delete;
    ~TmpDev() {
        if (p) (void)hipFree(p);
    }
};
struct TmpEvents {
    hipEvent_t a = nullptr, b = nullptr;
    TmpEvents() = default;
    TmpEvents(const TmpEvents &) = delete;
    TmpEvents &operator=(const TmpEvents &) = delete;
    ~TmpEvents() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

KArgs kargs(su2_ensemble_s *E, int which = 0) {
    KArgs a;
    a.desc = E->ddesc;
    a.tiles = which == 0 ? E->tiles : which == 1 ? E->stiles : which == 2 ? E->vtiles
            : which == 3 ? E->mtiles : which == 4 ? E->mtiles_z : which == 5 ? E->mtiles_b : E->mtiles_b3;
    a.ntiles = which == 0 ? E->ntiles : which == 1 ? E->nstiles : which == 2 ? E->nvtiles : E->nmtiles;
    a.xcd_remap = E->remap != 0;
    a.links = E->links;
    a.st = E->st;
    a.err = &E->st->err;
    a.trace = E->trace;
    a.tries_part = E->tries_part;
    a.plaq_part = E->part_hb;
    a.sampler = E->sampler;
    a.advance = 0;
    a.nslots = 0;
    a.every = 1;
    return a;
}

// Heat-bath tile list of direction mu in the handle's tile mode: modes 0
// and 1 lexicographic, with (z, t, y, x) order for mu = 3; mode 2 (z, t, y,
// x) for every mu; mode 3 the XCD blocks.  All lists hold the same tiles.
const Tile *hb_tiles(const su2_ensemble_s *E, int mu) {
    if (E->remap == 3) return mu == 3 ? E->mtiles_b3 : E->mtiles_b;
    return (mu == 3 || E->remap == 2) ? E->mtiles_z : E->mtiles;
}

void drop_run_graphs(su2_ensemble_s *E) {
    for (auto &g : E->run_graphs)
        if (g.second) (void)hipGraphExecDestroy(g.second);
    E->run_graphs.clear();
}

void drop_graphs(su2_ensemble_s *E) {
    for (auto &g : E->graphs)
        if (g.second) (void)hipGraphExecDestroy(g.second);
    E->graphs.clear();
    drop_run_graphs(E);
}

// ---- per-kernel event timing -------------------------------------------
hipEvent_t take_event(su2_ensemble_s *E) {
    if (!E->evpool.empty()) {
        hipEvent_t e = E->evpool.back();
        E->evpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Timed {
    su2_ensemble_s *E;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    bool stamped;
    // stamped: the launch itself stamps a and b with the kernel's start and
    // end (see ev()); otherwise a and b are recorded on the stream around it.
    Timed(su2_ensemble_s *e, int k, hipStream_t s, bool stamp = false) : E(e), kind(k), stamped(stamp) {
        if (E->timing) {
            a = take_event(E);
            b = take_event(E);
            if (a && !stamped) (void)hipEventRecord(a, s);
        }
    }
    su2::Ev ev() const {
        su2::Ev v;
        if (E->timing && a && b) v.a = a, v.b = b;
        return v;
    }
    void done(hipStream_t s) {
        if (E->timing && a && b) {
            if (!stamped) (void)hipEventRecord(b, s);
            E->pending.push_back(EventPair{kind, a, b});
        }
    }
};

su2_status collect_timing(su2_ensemble_s *E) {
    for (auto &p : E->pending) {
        HIPCHK(hipEventSynchronize(p.b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
        E->tms[p.kind] += ms;
        E->tcount[p.kind] += 1;
        E->evpool.push_back(p.a);
        E->evpool.push_back(p.b);
    }
    E->pending.clear();
    return SU2_OK;
}

// ---- tile tables ----------------------------------------------------------
su2_status upload_desc(su2_ensemble_s *E) {
    HIPCHK(hipMemcpyAsync(E->ddesc, E->hdesc.data(), sizeof(LatDesc) * E->n, hipMemcpyHostToDevice,
                          E->stream()));
    return SU2_OK;
}

su2_status fold_tries(su2_ensemble_s *E) {
    if (!E->tries_part || E->ntiles == 0) return SU2_OK;
    std::vector<unsigned long long> h(E->ntiles);
    HIPCHK(hipMemcpyAsync(h.data(), E->tries_part, sizeof(unsigned long long) * E->ntiles,
                          hipMemcpyDeviceToHost, E->stream()));
    HIPCHK(hipStreamSynchronize(E->stream()));
    for (auto v : h) E->tries_acc += v;
    HIPCHK(hipMemsetAsync(E->tries_part, 0, sizeof(unsigned long long) * E->ntiles, E->stream()));
    return SU2_OK;
}

su2_status build_tiles(su2_ensemble_s *E) {
    CHK(fold_tries(E));
    E->htiles.clear();
    E->hstiles.clear();
    E->hvtiles.clear();
    E->hmtiles.clear();
    E->hmtiles_z.clear();
    E->hmtiles_b.clear();
    E->hmtiles_b3.clear();
    const int B = E->block;
    for (int l = 0; l < E->n; ++l) {
        LatDesc &d = E->hdesc[l];
        d.tile0 = (int)E->htiles.size();
        for (int s = 0; s < d.vh; s += B) E->htiles.push_back(make_int2(l, s));
        d.ntile = (int)E->htiles.size() - d.tile0;
        d.stile0 = (int)E->hstiles.size();
        for (int s = 0; s < d.ns; s += B) E->hstiles.push_back(make_int2(l, s));
        d.nstile = (int)E->hstiles.size() - d.stile0;
        d.vtile0 = (int)E->hvtiles.size();
        for (int s = 0; s < 2 * d.vh; s += B) E->hvtiles.push_back(make_int2(l, s));
        d.nvtile = (int)E->hvtiles.size() - d.vtile0;
        d.mtile0 = (int)E->hmtiles.size();
        for (int s = 0; s < d.vh; s += B * E->nl) E->hmtiles.push_back(make_int2(l, s));
        d.nmtile = (int)E->hmtiles.size() - d.mtile0;
        // The same tiles ordered by the (z, t, y, x) of their first site: the
        // XCD-aware walk gives each XCD a contiguous share of the list, which
        // in this order is a range of z over every t, so the temporal
        // neighbours of the mu = 3 substeps stay in that XCD's L2.
        //
        // Tile mode 3 gives each XCD (an eighth of the list) a block of the
        // lattice that is thick in two directions other than the one being
        // updated, so fewer staple links lie on its boundary: a slab four
        // t-slices thick (32^4 in lexicographic order) reads a halo of four
        // link classes times one face, about 14% of its links, a (z half,
        // t quarter) block about 11%.  mu = 3 staples reach forward in t, so
        // its blocks split z and y instead.
        std::vector<std::pair<long long, Tile>> zt, bl, bl3;
        for (int i = d.mtile0; i < d.mtile0 + d.nmtile; ++i) {
            const long long cbs = E->hmtiles[i].y, row = cbs / d.hx;  // row = y + Ny (z + Nz t)
            const long long y = row % d.n[1], z = (row / d.n[1]) % d.n[2], t = row / ((long long)d.n[1] * d.n[2]);
            const long long ztyx = ((z * d.n[3] + t) * d.n[1] + y) * d.hx + cbs % d.hx;
            zt.push_back({ztyx, E->hmtiles[i]});
            const long long b0 = (z * 2 / d.n[2]) * 4 + t * 4 / d.n[3];
            const long long b3 = (z * 4 / d.n[2]) * 2 + y * 2 / d.n[1];
            bl.push_back({(b0 << 40) + cbs, E->hmtiles[i]});
            bl3.push_back({(b3 << 40) + ztyx, E->hmtiles[i]});
        }
        const auto by_key = [](const auto &u, const auto &v) { return u.first < v.first; };
        std::sort(zt.begin(), zt.end(), by_key);
        std::sort(bl.begin(), bl.end(), by_key);
        std::sort(bl3.begin(), bl3.end(), by_key);
        for (auto &e : zt) E->hmtiles_z.push_back(e.second);
        for (auto &e : bl) E->hmtiles_b.push_back(e.second);
        for (auto &e : bl3) E->hmtiles_b3.push_back(e.second);
    }
    E->ntiles = (int)E->htiles.size();
    E->nstiles = (int)E->hstiles.size();
    E->nvtiles = (int)E->hvtiles.size();
    E->nmtiles = (int)E->hmtiles.size();
    CHK(dalloc(E, &E->tiles, sizeof(Tile) * E->ntiles));
    CHK(dalloc(E, &E->stiles, sizeof(Tile) * E->nstiles));
    CHK(dalloc(E, &E->vtiles, sizeof(Tile) * E->nvtiles));
    CHK(dalloc(E, &E->mtiles, sizeof(Tile) * E->nmtiles));
    CHK(dalloc(E, &E->mtiles_z, sizeof(Tile) * E->nmtiles));
    CHK(dalloc(E, &E->mtiles_b, sizeof(Tile) * E->nmtiles));
    CHK(dalloc(E, &E->mtiles_b3, sizeof(Tile) * E->nmtiles));
    CHK(dalloc(E, &E->tries_part, sizeof(unsigned long long) * E->ntiles));
    CHK(dalloc(E, &E->part_plaq, sizeof(double) * 4 * E->ntiles));
    {   // series partials of up to nslots sweeps (about 64 MiB at most),
        // reduced once per batch of sweeps
        const size_t per_sweep = sizeof(double) * (12 * (size_t)E->nmtiles + 2 * (size_t)E->nstiles);
        E->nslots = (int)std::min<size_t>(512, std::max<size_t>(1, (size_t(64) << 20) / per_sweep));
    }
    CHK(dalloc(E, &E->part_poly, sizeof(double) * 2 * (size_t)E->nstiles * E->nslots));
    CHK(dalloc(E, &E->part_hb, sizeof(double) * 12 * (size_t)E->nmtiles * E->nslots));
    {   // series reduction: chunks of ~256 partial tiles per (lattice, sweep)
        int most = 1;
        for (const LatDesc &d : E->hdesc) most = std::max(most, std::max(d.nmtile, d.nstile));
        E->ser_C = std::min(64, std::max(1, (most + 255) / 256));
        CHK(dalloc(E, &E->ser_chunk, sizeof(double) * 6 * (size_t)E->n * E->nslots * E->ser_C));
    }
    {   // final-reduction workgroups per lattice: ~2048 partial tiles each
        int most = 1;
        for (const LatDesc &d : E->hdesc) most = std::max(most, std::max(d.nmtile, std::max(d.ntile, d.nstile)));
        E->fin_chunks = std::min(64, std::max(1, (most + 2047) / 2048));
    }
    CHK(dalloc(E, &E->fin_cnt, sizeof(unsigned) * E->n));
    CHK(dalloc(E, &E->fin_chunk, sizeof(double) * 6 * (size_t)E->n * E->fin_chunks));
    HIPCHK(hipMemsetAsync(E->fin_cnt, 0, sizeof(unsigned) * E->n, E->stream()));
    HIPCHK(hipMemsetAsync(E->part_hb, 0, sizeof(double) * 12 * (size_t)E->nmtiles * E->nslots, E->stream()));
    HIPCHK(hipMemsetAsync(E->tries_part, 0, sizeof(unsigned long long) * E->ntiles, E->stream()));
    HIPCHK(hipMemcpyAsync(E->tiles, E->htiles.data(), sizeof(Tile) * E->ntiles, hipMemcpyHostToDevice,
                          E->stream()));
    HIPCHK(hipMemcpyAsync(E->stiles, E->hstiles.data(), sizeof(Tile) * E->nstiles, hipMemcpyHostToDevice,
                          E->stream()));
    HIPCHK(hipMemcpyAsync(E->vtiles, E->hvtiles.data(), sizeof(Tile) * E->nvtiles, hipMemcpyHostToDevice,
                          E->stream()));
    HIPCHK(hipMemcpyAsync(E->mtiles, E->hmtiles.data(), sizeof(Tile) * E->nmtiles, hipMemcpyHostToDevice,
                          E->stream()));
    HIPCHK(hipMemcpyAsync(E->mtiles_b, E->hmtiles_b.data(), sizeof(Tile) * E->nmtiles, hipMemcpyHostToDevice,
                          E->stream()));
    HIPCHK(hipMemcpyAsync(E->mtiles_b3, E->hmtiles_b3.data(), sizeof(Tile) * E->nmtiles, hipMemcpyHostToDevice,
                          E->stream()));
    HIPCHK(hipMemcpyAsync(E->mtiles_z, E->hmtiles_z.data(), sizeof(Tile) * E->nmtiles, hipMemcpyHostToDevice,
                          E->stream()));
    CHK(upload_desc(E));
    HIPCHK(hipStreamSynchronize(E->stream()));
    drop_graphs(E);
    return SU2_OK;
}

// Seed / sweep / run_base of the device state from the host mirror (not the
// device-written error word), by a one-thread kernel in stream order: no
// host synchronisation.
su2_status upload_state(su2_ensemble_s *E) {
    E->hst.next = E->hst.sweep;
    su2::launch_set_state(E->st, E->hst.seed, E->hst.sweep, E->hst.run_base, E->stream());
    HIPCHK(hipGetLastError());
    return SU2_OK;
}

// End of a call that reports results: one synchronisation of the handle's
// stream, after which the error word (non-finite staples, sampler try-cap
// hits since the last report) is read.  A non-zero word is this call's
// ENUMERIC and is cleared, so the next call starts clean.
su2_status finish(su2_ensemble_s *E, bool err_enqueued = false) {
    if (!err_enqueued) su2::launch_err_to_host(E->st, E->derr, E->stream());
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(E->stream()));
    if (*E->herr == 0u) return SU2_OK;
    *E->herr = 0u;
    su2::launch_clear_err(E->st, E->stream());
    HIPCHK(hipGetLastError());
    return SU2_ENUMERIC;
}

void invalidate_measure_buffers(su2_ensemble_s *E) { E->sm_cur = -1; }

// Descriptor of lattice l with extents d, whose links start at link `off`
// of the buffer and whose sites at site `sites` of the ensemble.
void fill_desc(LatDesc &D, const int *d, int l, long long off, long long sites, double beta) {
    std::memset(&D, 0, sizeof(D));
    for (int k = 0; k < 4; ++k) D.n[k] = d[k];
    const long long V = (long long)d[0] * d[1] * d[2] * d[3];
    D.hx = d[0] / 2;
    D.vh = (int)(V / 2);
    D.ns = d[0] * d[1] * d[2];
    D.lat_id = l;
    D.off = off;
    D.soff = 3 * sites;
    D.toff = off;
    D.inv_hx = recip_up(D.hx);
    D.inv_nx = recip_up(d[0]);
    D.inv_ny = recip_up(d[1]);
    D.inv_nz = recip_up(d[2]);
    D.beta = beta;
    D.betaf = (float)beta;
}

// ---- creation ----------------------------------------------------------------
su2_status create_common(int n, const int *dims, const double *betas, su2_start start, uint64_t seed,
                         su2_prec prec, void *device_links, size_t device_bytes, su2_ensemble_s *E) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return SU2_ENODEV;
    }
    if (hipGetDevice(&E->device) != hipSuccess) return SU2_ENODEV;
    E->n = n;
    E->f32 = (prec == SU2_F32);
    E->hdesc.resize(n);
    long long off = 0, sites = 0;
    for (int l = 0; l < n; ++l) {
        const int *d = dims + 4 * l;
        fill_desc(E->hdesc[l], d, l, off, sites, betas ? betas[l] : 0.0);
        const long long V = (long long)d[0] * d[1] * d[2] * d[3];
        off += 4 * V;
        sites += V;
    }
    E->total_links = off;
    E->total_sites = sites;
    E->link_bytes = (size_t)off * link_size(E->f32);
    if (hipStreamCreateWithFlags(&E->own, hipStreamNonBlocking) != hipSuccess) return SU2_EDEVICE;
    if (device_links) {
        if (device_bytes < E->link_bytes) return SU2_EINVAL;
        E->links = device_links;
        E->own_links = false;
    } else {
        CHK(dalloc(E, &E->links, E->link_bytes));
    }
    CHK(dalloc(E, &E->ddesc, sizeof(LatDesc) * n));
    CHK(dalloc(E, &E->st, sizeof(DevState)));
    CHK(dalloc(E, &E->res, sizeof(double) * 4 * n));
    if (hipHostMalloc((void **)&E->hres, sizeof(double) * 4 * n, hipHostMallocDefault) != hipSuccess) {
        E->hres = nullptr;
        return SU2_ENOMEM;
    }
    if (host_mapped(E, (void **)&E->herr, (void **)&E->derr, sizeof(unsigned) * 16) != SU2_OK) return SU2_ENOMEM;
    E->hst.seed = seed;
    E->hst.sweep = 0;
    E->hst.run_base = 0;
    HIPCHK(hipMemsetAsync(E->st, 0, sizeof(DevState), E->stream()));
    CHK(upload_state(E));
    CHK(build_tiles(E));
    KArgs a = kargs(E);
    su2::launch_init(a, E->f32, start == SU2_HOT ? 1 : 0, E->block, E->grid, E->stream());
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(E->stream()));
    return SU2_OK;
}

void destroy_common(su2_ensemble_s *E) {
    if (!E) return;
    (void)hipSetDevice(E->device);
    if (E->own) (void)hipStreamSynchronize(E->own);
    if (E->user) (void)hipStreamSynchronize(E->user);
    drop_graphs(E);
    for (auto &p : E->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : E->evpool) (void)hipEventDestroy(e);
    void *bufs[] = {E->ddesc, E->tiles, E->stiles, E->vtiles, E->mtiles, E->mtiles_z, E->mtiles_b, E->mtiles_b3, E->st, E->tries_part, E->part_plaq,
                    E->part_poly, E->part_hb, E->fin_cnt, E->fin_chunk, E->res, E->ser_chunk,
                    E->sm[0], E->sm[1], E->wl_s, E->wpart, E->trace};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (E->own_links && E->links) (void)hipFree(E->links);
    if (E->hres) (void)hipHostFree(E->hres);
    if (E->hser) (void)hipHostFree(E->hser);
    if (E->herr) (void)hipHostFree(E->herr);
    if (E->own) (void)hipStreamDestroy(E->own);
}

// ---- one sweep --------------------------------------------------------------
// Eight substep launches that also advance the device sweep counter; with a
// plaquette series the odd substeps mu >= 1 sum the plaquettes of the
// sweep's final configuration into the partial slot of its measurement,
// with a Polyakov series k_polyakov does the same.  The slots are reduced
// per batch of measurements (series_batch), so a sweep holds no reduction
// launch.
su2_status enqueue_sweep(su2_ensemble_s *E, int meas, int every, hipStream_t s) {
    KArgs a = kargs(E, 3);
    a.advance = 1;
    a.nslots = E->nslots;
    a.every = every;
    for (int mu = 0; mu < 4; ++mu)
        for (int par = 0; par < 2; ++par) {
            const bool plaq = (meas & 1) && par == 1 && mu >= 1;
            a.tiles = hb_tiles(E, mu);
            Timed t(E, SU2_K_HEATBATH, s, true);
            su2::launch_heatbath(a, E->f32, mu, par, E->nl, E->block, E->grid, s, E->trace != nullptr, plaq,
                                 t.ev());
            t.done(s);
        }
    if (meas & 2) {
        KArgs p = kargs(E, 1);
        p.nslots = E->nslots;
        p.every = every;
        Timed t(E, SU2_K_POLYAKOV, s);
        su2::launch_polyakov(p, E->f32, E->part_poly, E->block, E->grid, s);
        t.done(s);
    }
    HIPCHK(hipGetLastError());
    return SU2_OK;
}

// One unit: `every` sweeps, the last of which measures (meas != 0).
su2_status enqueue_unit(su2_ensemble_s *E, int meas, int every, hipStream_t s) {
    for (int k = 0; k < every; ++k) CHK(enqueue_sweep(E, k == every - 1 ? meas : 0, every, s));
    return SU2_OK;
}

// Series values of the nmeas measurements of units u0 .. u0 + nmeas - 1 of
// the current run.
su2_status series_batch(su2_ensemble_s *E, int meas, int u0, int nmeas, hipStream_t s) {
    Timed r(E, SU2_K_REDUCE, s);
    su2::launch_series(E->ddesc, E->n, (meas & 1) ? E->part_hb : nullptr, 12 * (long long)E->nmtiles,
                       (meas & 2) ? E->part_poly : nullptr, 2 * (long long)E->nstiles, u0 % E->nslots,
                       E->nslots, nmeas, E->ser_C, E->ser_chunk, E->run_plaq, E->run_poly, E->run_nm, u0, s);
    r.done(s);
    HIPCHK(hipGetLastError());
    return SU2_OK;
}

// Capture `units` consecutive units into one executable graph.
su2_status capture_units(su2_ensemble_s *E, int meas, int every, int units, hipGraphExec_t *out) {
    HIPCHK(hipStreamBeginCapture(E->own, hipStreamCaptureModeRelaxed));
    su2_status st = SU2_OK;
    for (int k = 0; k < units && st == SU2_OK; ++k) st = enqueue_unit(E, meas, every, E->own);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(E->own, &g);
    if (st != SU2_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    HIPCHK(e);
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    return SU2_OK;
}

unsigned long long graph_key(int meas, int every, int units) {
    return ((unsigned long long)(unsigned)units << 34) | ((unsigned long long)(unsigned)every << 2) |
           (unsigned)meas;
}

// Units per graph: the largest graph holds G = max(1, graph_sweeps() / every)
// units; the others 2^k < G units.  All of them are captured together on
// the first run with this (meas, every), so later runs of any length only
// replay graphs.
int units_per_graph(int every) { return std::max(1, graph_sweeps() / every); }

su2_status ensure_graphs(su2_ensemble_s *E, int meas, int every) {
    const int G = units_per_graph(every);
    std::vector<int> sizes{G};
    for (int u = 1; u < G; u <<= 1) sizes.push_back(u);
    for (int u : sizes) {
        hipGraphExec_t &g = E->graphs[graph_key(meas, every, u)];
        if (!g) CHK(capture_units(E, meas, every, u, &g));
    }
    return SU2_OK;
}

// nunits units: graphs of G units, then the binary remainder (2^k < G).
su2_status run_units(su2_ensemble_s *E, int nunits, int meas, int every) {
    hipStream_t s = E->stream();
    const bool use_graph = !E->timing && (long long)nunits * every > 1 && !std::getenv("SU2_NO_GRAPH");
    if (!use_graph) {
        for (int u = 0; u < nunits; ++u) CHK(enqueue_unit(E, meas, every, s));
        return SU2_OK;
    }
    CHK(ensure_graphs(E, meas, every));
    const int G = units_per_graph(every);
    int left = nunits;
    for (; left >= G; left -= G) HIPCHK(hipGraphLaunch(E->graphs[graph_key(meas, every, G)], s));
    for (int u = 1 << 30; u >= 1; u >>= 1)
        if (left & u) HIPCHK(hipGraphLaunch(E->graphs[graph_key(meas, every, u)], s));
    return SU2_OK;
}

// A whole run as one graph: the device state from the run state in mapped
// host memory, its measured units with the series reduction behind each
// batch of them, the unmeasured remainder and the copy of the error word.  One launch
// instead of a state kernel and one launch per graph size (the GPU idled
// ~9 us between the state kernel and the first sweep, and ~8 us at each
// hand-over between graphs), and the series kernels right behind the last
// sweep; kept for runs of up to RUN_GRAPH_MAX_SWEEPS sweeps, at most
// RUN_GRAPH_MAX of them per handle.
constexpr int RUN_GRAPH_MAX_SWEEPS = 256;
constexpr size_t RUN_GRAPH_MAX = 8;

bool run_graph_ok(const su2_ensemble_s *E, int nsweeps) {
    return !E->timing && nsweeps > 1 && nsweeps <= RUN_GRAPH_MAX_SWEEPS && !std::getenv("SU2_NO_GRAPH");
}

su2_status capture_run(su2_ensemble_s *E, int meas, int every, int nsweeps, hipGraphExec_t *out) {
    const int nm = meas ? nsweeps / every : 0;
    HIPCHK(hipStreamBeginCapture(E->own, hipStreamCaptureModeRelaxed));
    su2_status st = SU2_OK;
    su2::launch_set_state_mapped(E->st, E->derr + 4, E->own);
    for (int done = 0; done < nm && st == SU2_OK; done += E->nslots) {
        const int b = std::min(E->nslots, nm - done);
        for (int k = 0; k < b && st == SU2_OK; ++k) st = enqueue_unit(E, meas, every, E->own);
        if (st == SU2_OK) st = series_batch(E, meas, done, b, E->own);
    }
    for (int k = nm * every; k < nsweeps && st == SU2_OK; ++k) st = enqueue_unit(E, 0, 1, E->own);
    if (st == SU2_OK) su2::launch_err_to_host(E->st, E->derr, E->own);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(E->own, &g);
    if (st != SU2_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    HIPCHK(e);
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    return SU2_OK;
}

// nsweeps sweeps; with meas, sweep k (0-based) of the run is measured when
// (k + 1) % every == 0 (nsweeps / every measurements, series batches of at
// most nslots of them) and the remaining nsweeps % every sweeps at the end
// measure nothing.  With err_enqueued the run may be one captured graph,
// which also sets the device state from the host mirror and copies the error
// word (then *err_enqueued is set and finish() skips the copy); otherwise,
// with upload, the state is set by upload_state first.
su2_status run_sweeps(su2_ensemble_s *E, int nsweeps, int meas, int every, bool *err_enqueued = nullptr,
                      bool upload = false) {
    const int nm = meas ? nsweeps / every : 0;
    if (err_enqueued) *err_enqueued = false;
    if (err_enqueued && run_graph_ok(E, nsweeps)) {
        // every call synchronises before it returns, so no replay of a run
        // graph is pending while these words are rewritten
        E->hst.next = E->hst.sweep;
        volatile unsigned *rs = E->herr + 4;
        rs[0] = (unsigned)E->hst.seed;
        rs[1] = (unsigned)(E->hst.seed >> 32);
        rs[2] = E->hst.sweep;
        rs[3] = E->hst.run_base;
        const unsigned long long key = graph_key(meas, every, nsweeps);
        auto it = E->run_graphs.find(key);
        if (it == E->run_graphs.end()) {
            if (E->run_graphs.size() >= RUN_GRAPH_MAX) drop_run_graphs(E);
            hipGraphExec_t g = nullptr;
            CHK(capture_run(E, meas, every, nsweeps, &g));
            it = E->run_graphs.emplace(key, g).first;
        }
        HIPCHK(hipGraphLaunch(it->second, E->stream()));
        *err_enqueued = true;
        E->hst.sweep += (unsigned)nsweeps;
        E->updates += (unsigned long long)nsweeps * (unsigned long long)E->total_links;
        invalidate_measure_buffers(E);
        return SU2_OK;
    }
    if (upload) CHK(upload_state(E));
    for (int done = 0; done < nm; done += E->nslots) {
        const int b = std::min(E->nslots, nm - done);
        CHK(run_units(E, b, meas, every));
        CHK(series_batch(E, meas, done, b, E->stream()));
    }
    const int rest = nsweeps - nm * every;
    if (rest > 0) CHK(run_units(E, rest, 0, 1));
    E->hst.sweep += (unsigned)nsweeps;
    E->updates += (unsigned long long)nsweeps * (unsigned long long)E->total_links;
    invalidate_measure_buffers(E);
    return SU2_OK;
}

// Host staging of the series of nm measurements per lattice and both
// observables (mapped pinned memory, written by the series kernels).
su2_status ensure_series(su2_ensemble_s *E, int nm) {
    const size_t need = 2 * (size_t)nm * E->n;
    if (need > E->hser_cap) {
        drop_run_graphs(E);  // they hold the old series pointers
        if (E->hser) (void)hipHostFree(E->hser);
        E->hser = E->dser = nullptr;
        E->hser_cap = 0;
        CHK(host_mapped(E, (void **)&E->hser, (void **)&E->dser, sizeof(double) * need));
        E->hser_cap = need;
    }
    return SU2_OK;
}

su2_status set_seed(su2_ensemble_s *E, uint64_t seed) {
    if (E->hst.seed != seed) {
        E->hst.seed = seed;
        CHK(upload_state(E));
    }
    return SU2_OK;
}

// ---- measurements -------------------------------------------------------------
su2_status measure_plaquette(su2_ensemble_s *E, int l, double *avg, double *sp, double *tp) {
    hipStream_t s = E->stream();
    const KArgs a = kargs(E);
    {
        Timed t(E, SU2_K_PLAQUETTE, s);
        su2::launch_plaquette(a, E->f32, E->part_plaq, E->block, E->grid, s);
        t.done(s);
    }
    {
        Timed t(E, SU2_K_REDUCE, s);
        su2::launch_finalize(E->ddesc, E->n, E->fin_chunks, E->part_plaq, nullptr, E->fin_cnt, E->fin_chunk,
                             E->res, nullptr, 4, s);
        t.done(s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(E->hres, E->res, sizeof(double) * 4 * E->n, hipMemcpyDeviceToHost, s));
    const su2_status st = finish(E);
    if (st == SU2_EDEVICE) return st;
    if (avg) *avg = E->hres[4 * l + 0];
    if (sp) *sp = E->hres[4 * l + 1];
    if (tp) *tp = E->hres[4 * l + 2];
    return st;
}

su2_status measure_polyakov(su2_ensemble_s *E, int l, double *out) {
    hipStream_t s = E->stream();
    const KArgs a = kargs(E, 1);
    {
        Timed t(E, SU2_K_POLYAKOV, s);
        su2::launch_polyakov(a, E->f32, E->part_poly, E->block, E->grid, s);
        t.done(s);
    }
    {
        Timed t(E, SU2_K_REDUCE, s);
        su2::launch_finalize(E->ddesc, E->n, E->fin_chunks, nullptr, E->part_poly, E->fin_cnt, E->fin_chunk,
                             nullptr, E->res, 4, s);
        t.done(s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(E->hres, E->res, sizeof(double) * 4 * E->n, hipMemcpyDeviceToHost, s));
    const su2_status st = finish(E);
    if (st == SU2_EDEVICE) return st;
    if (out) *out = E->hres[4 * l];
    return st;
}

bool finite_unit(const double *u, double tol) {
    double n2 = 0;
    for (int c = 0; c < 4; ++c) {
        if (!std::isfinite(u[c])) return false;
        n2 += u[c] * u[c];
    }
    return std::fabs(1.0 - n2) <= tol;
}

// canonical host <-> device for lattice l
su2_status set_links_l(su2_ensemble_s *E, int l, const double *host) {
    const LatDesc &d = E->hdesc[l];
    const long long V = 2LL * d.vh;
    for (long long i = 0; i < 4 * V; ++i)
        if (!finite_unit(host + 4 * i, 1e-6)) return SU2_EINVAL;
    TmpDev<double> stage;   // lattice l only
    CHK(dalloc(E, &stage.p, sizeof(double) * 16 * (size_t)V));
    hipStream_t s = E->stream();
    HIPCHK(hipMemcpyAsync(stage.p, host, sizeof(double) * 16 * V, hipMemcpyHostToDevice, s));
    // only the tiles of lattice l
    KArgs a = kargs(E);
    a.tiles = E->tiles + d.tile0;
    a.ntiles = d.ntile;
    su2::launch_from_canon(a, E->f32, stage.p, E->block, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    invalidate_measure_buffers(E);
    return SU2_OK;
}

su2_status get_links_l(su2_ensemble_s *E, int l, const void *src, int ndir, double *host) {
    const LatDesc &d = E->hdesc[l];
    const long long V = 2LL * d.vh;
    TmpDev<double> stage;   // lattice l only
    CHK(dalloc(E, &stage.p, sizeof(double) * 4 * ndir * (size_t)V));
    hipStream_t s = E->stream();
    KArgs a = kargs(E);
    a.tiles = E->tiles + d.tile0;
    a.ntiles = d.ntile;
    su2::launch_to_canon(a, E->f32, src, ndir, stage.p, E->block, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(host, stage.p, sizeof(double) * 4 * ndir * V, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return SU2_OK;
}

su2_status stats_common(su2_ensemble_s *E, uint64_t *tries, uint64_t *updates, double *defect) {
    if (tries) {
        std::vector<unsigned long long> h(E->ntiles);
        HIPCHK(hipMemcpyAsync(h.data(), E->tries_part, sizeof(unsigned long long) * E->ntiles,
                              hipMemcpyDeviceToHost, E->stream()));
        HIPCHK(hipStreamSynchronize(E->stream()));
        unsigned long long t = E->tries_acc;
        for (auto v : h) t += v;
        *tries = t;
    }
    if (updates) *updates = E->updates;
    if (defect) {
        TmpDev<unsigned long long> m;
        CHK(dalloc(E, &m.p, sizeof(unsigned long long)));
        HIPCHK(hipMemsetAsync(m.p, 0, sizeof(unsigned long long), E->stream()));
        su2::launch_unit_defect(kargs(E), E->f32, m.p, E->block, E->stream());
        HIPCHK(hipGetLastError());
        unsigned long long bits = 0;
        HIPCHK(hipMemcpyAsync(&bits, m.p, sizeof(bits), hipMemcpyDeviceToHost, E->stream()));
        HIPCHK(hipStreamSynchronize(E->stream()));
        std::memcpy(defect, &bits, sizeof(double));
    }
    return finish(E);
}

su2_status set_launch_common(su2_ensemble_s *E, int block, int grid, int remap, int nl) {
    if (block < 64 || block > 256 || (block & 63)) return SU2_EINVAL;
    if (grid < 0 || (grid & 7)) return SU2_EINVAL;
    if (remap < 0 || remap > 3) return SU2_EINVAL;
    if (nl != 1 && nl != 2 && nl != 4) return SU2_EINVAL;
    const bool reshape = block != E->block || nl != E->nl;
    E->grid = grid;
    E->remap = remap;
    if (reshape) {
        E->block = block;
        E->nl = nl;
        CHK(build_tiles(E));
    }
    drop_graphs(E);
    return SU2_OK;
}

// Time one sweep per candidate shape; links, sweep counter and tries are
// restored afterwards.
struct Shape { int block, grid, remap, nl; };
// Shapes found per size class; shared by all handles of the process.
std::map<std::string, Shape> g_tune_cache;
std::mutex g_tune_mutex;

bool tune_cache_get(const std::string &key, Shape &out) {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) return false;
    out = it->second;
    return true;
}

void tune_cache_put(const std::string &key, const Shape &v) {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[key] = v;
}

su2_status autotune_common(su2_ensemble_s *E) {
    char key[160];
    std::snprintf(key, sizeof key, "%s:n%d:sites%lld:t%lld", E->f32 ? "f32" : "f64", E->n, E->total_sites,
                  (long long)E->hdesc[0].n[3]);
    Shape cached;
    if (tune_cache_get(key, cached)) return set_launch_common(E, cached.block, cached.grid, cached.remap, cached.nl);

    hipStream_t s = E->stream();
    TmpDev<char> backup;
    CHK(dalloc(E, &backup.p, E->link_bytes));
    HIPCHK(hipMemcpyAsync(backup.p, E->links, E->link_bytes, hipMemcpyDeviceToDevice, s));
    CHK(fold_tries(E));
    const unsigned long long tries0 = E->tries_acc, upd0 = E->updates;
    const DevState st0 = E->hst;
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, E->device));
    const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    struct TimingOff {  // timing is off while tuning and restored on every return path
        su2_ensemble_s *E;
        bool saved;
        ~TimingOff() { E->timing = saved; }
    } timing_off{E, E->timing};
    E->timing = false;
    CHK(ensure_series(E, 4));

    const int blocks[] = {64, 128, 256};
    // persistent grids of 4, 8, 16 workgroups per CU, and -1: as many as the
    // heat-bath kernel keeps resident (its occupancy for the block size)
    const int gmul[] = {0, 4, 8, 16, -1};
    const int nls[] = {1, 2, 4};
    TmpEvents ev;
    HIPCHK(hipEventCreate(&ev.a));
    HIPCHK(hipEventCreate(&ev.b));
    hipEvent_t ea = ev.a, eb = ev.b;
    float best = 1e30f;
    Shape bestc{E->block, E->grid, E->remap, E->nl};
    for (int nl : nls)
        for (int b : blocks)
            for (int gm : gmul)
                for (int rm = 0; rm < 4; ++rm) {
                    const int per_cu = gm >= 0 ? gm : su2::heatbath_blocks_per_cu(E->f32, nl, b);
                    const int g = per_cu > 0 ? per_cu * cus / 8 * 8 : 0;
                    if (gm < 0 && per_cu <= 0) continue;
                    CHK(set_launch_common(E, b, g, rm, nl));
                    // series slots 0..3 of this candidate's four sweeps
                    E->hst = st0;
                    E->hst.run_base = st0.sweep;
                    CHK(upload_state(E));
                    CHK(enqueue_sweep(E, 1, 1, s));  // warm-up (with the plaquette series)
                    HIPCHK(hipEventRecord(ea, s));
                    for (int r = 0; r < 3; ++r) CHK(enqueue_sweep(E, 1, 1, s));
                    HIPCHK(hipEventRecord(eb, s));
                    HIPCHK(hipEventSynchronize(eb));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, ea, eb));
                    if (ms < best) {
                        best = ms;
                        bestc = Shape{b, g, rm, nl};
                    }
                }
    CHK(set_launch_common(E, bestc.block, bestc.grid, bestc.remap, bestc.nl));
    HIPCHK(hipMemcpyAsync(E->links, backup.p, E->link_bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemsetAsync(E->tries_part, 0, sizeof(unsigned long long) * E->ntiles, s));
    HIPCHK(hipStreamSynchronize(s));
    E->tries_acc = tries0;
    E->updates = upd0;
    E->hst = st0;
    CHK(upload_state(E));
    tune_cache_put(key, bestc);
    invalidate_measure_buffers(E);
    return SU2_OK;
}

su2_status get_timing_common(su2_ensemble_s *E, su2_kernel_kind kind, double *ms, int64_t *launches) {
    if ((int)kind < 0 || kind >= SU2_K_COUNT) return SU2_EINVAL;
    CHK(collect_timing(E));
    if (ms) *ms = E->tms[kind];
    if (launches) *launches = E->tcount[kind];
    return SU2_OK;
}

su2_status set_timing_common(su2_ensemble_s *E, int enable) {
    CHK(collect_timing(E));
    E->timing = enable != 0;
    for (int k = 0; k < SU2_K_COUNT; ++k) {
        E->tms[k] = 0;
        E->tcount[k] = 0;
    }
    return SU2_OK;
}

// ---- allocation-free heat bath ---------------------------------------------------
// The state, descriptor, tile list and per-tile try counters of
// su2_heatbath_noalloc live in one file-scope device array (each GPU holds
// its own copy): 512 header bytes (DevState at 0, LatDesc at 256), then
// NOALLOC_MAX_TILES tiles and as many try counters.  Tiles of 256 half-sites,
// so lattices up to 2^27 sites fit.
constexpr int NOALLOC_BLOCK = 256;
constexpr long long NOALLOC_MAX_SITES = 1LL << 27;
constexpr int NOALLOC_MAX_TILES = (int)(NOALLOC_MAX_SITES / 2 / NOALLOC_BLOCK);
constexpr size_t NOALLOC_HDR = 512;
constexpr size_t NOALLOC_BYTES =
    NOALLOC_HDR + (size_t)NOALLOC_MAX_TILES * (sizeof(Tile) + sizeof(unsigned long long));
static_assert(sizeof(DevState) <= 256 && sizeof(LatDesc) <= 256, "scratch header layout");

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
unsigned char *g_scratch[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on device `dev`, taken once per device with
// that device current (the caller's).  In host code the array's name is only
// a host-side stand-in; kernels get this address.
su2_status scratch_of(int dev, unsigned char **out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return SU2_ENODEV;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SU2_EDEVICE;
        }
        g_scratch[dev] = (unsigned char *)p;
    }
    *out = g_scratch[dev];
    return SU2_OK;
}

// Per call: descriptor and state into the header, tiles (0, 256 i), try
// counters zeroed; a kernel, so the call stays capturable.
__global__ void k_noalloc_setup(unsigned char *sc, LatDesc d, unsigned long long seed, unsigned sweep, int ntiles) {
    Tile *tiles = reinterpret_cast<Tile *>(sc + NOALLOC_HDR);
    unsigned long long *tries = reinterpret_cast<unsigned long long *>(tiles + NOALLOC_MAX_TILES);
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < ntiles) {
        tiles[i] = make_int2(0, i * NOALLOC_BLOCK);
        tries[i] = 0ull;
    }
    if (i == 0) {
        DevState *st = reinterpret_cast<DevState *>(sc);
        st->seed = seed;
        st->sweep = sweep;
        st->next = sweep;
        st->run_base = sweep;
        st->err = 0u;
        *reinterpret_cast<LatDesc *>(sc + 256) = d;
    }
}

__global__ void k_noalloc_err(const unsigned char *sc, uint32_t *out) {
    *out = reinterpret_cast<const DevState *>(sc)->err;
}

}  // namespace

// ============================================================================
extern "C" {

su2_status su2_heatbath_noalloc(void *device_links, int Nx, int Ny, int Nz, int Nt, su2_prec prec, double beta,
                                int nsweeps, uint64_t seed, uint32_t sweep, uint32_t *device_err,
                                void *hip_stream) {
    const int d[4] = {Nx, Ny, Nz, Nt};
    if (!device_links || (prec != SU2_F32 && prec != SU2_F64) || !dims_ok(d, prec == SU2_F32)) return SU2_EINVAL;
    if ((long long)Nx * Ny * Nz * Nt > NOALLOC_MAX_SITES) return SU2_EINVAL;
    if (!(beta >= 0.0) || !std::isfinite(beta) || nsweeps < 0) return SU2_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return SU2_ENODEV;
    }
    unsigned char *sc = nullptr;
    CHK(scratch_of(dev, &sc));
    LatDesc D;
    fill_desc(D, d, 0, 0, 0, beta);
    const int ntiles = (D.vh + NOALLOC_BLOCK - 1) / NOALLOC_BLOCK;
    D.tile0 = D.mtile0 = 0;
    D.ntile = D.nmtile = ntiles;
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_noalloc_setup, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, sc, D,
                       (unsigned long long)seed, (unsigned)sweep, ntiles);
    KArgs a{};
    a.desc = reinterpret_cast<const LatDesc *>(sc + 256);
    a.tiles = reinterpret_cast<const Tile *>(sc + NOALLOC_HDR);
    a.ntiles = ntiles;
    a.xcd_remap = 1;
    a.links = device_links;
    a.st = reinterpret_cast<DevState *>(sc);
    a.err = &a.st->err;
    a.trace = nullptr;
    a.tries_part = reinterpret_cast<unsigned long long *>(sc + NOALLOC_HDR + sizeof(Tile) * NOALLOC_MAX_TILES);
    a.plaq_part = nullptr;
    a.sampler = SU2_HYBRID;
    a.advance = 1;
    a.nslots = 0;
    a.every = 1;
    for (int k = 0; k < nsweeps; ++k)
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par)
                su2::launch_heatbath(a, prec == SU2_F32, mu, par, 1, NOALLOC_BLOCK, 0, s, false, false);
    if (device_err) hipLaunchKernelGGL(k_noalloc_err, dim3(1), dim3(1), 0, s, sc, device_err);
    return hipGetLastError() == hipSuccess ? SU2_OK : SU2_EDEVICE;
}


const char *su2_status_str(su2_status st) {
    switch (st) {
    case SU2_OK: return "ok";
    case SU2_EINVAL: return "invalid argument";
    case SU2_ENOMEM: return "out of memory";
    case SU2_ENODEV: return "no GPU device";
    case SU2_EDEVICE: return "GPU runtime error";
    case SU2_ESTATE: return "handle failed or call out of sequence";
    case SU2_EIO: return "I/O error";
    case SU2_ENUMERIC: return "non-finite value or sampler failure";
    }
    return "unknown status";
}

size_t su2_link_bytes(int Nx, int Ny, int Nz, int Nt, su2_prec prec) {
    const int d[4] = {Nx, Ny, Nz, Nt};
    if ((prec != SU2_F32 && prec != SU2_F64) || !dims_ok(d, prec == SU2_F32)) return 0;
    return (size_t)4 * Nx * Ny * Nz * (size_t)Nt * link_size(prec == SU2_F32);
}

// ---- ensembles -------------------------------------------------------------
su2_status su2_ensemble_create(int n, const int *dims, const double *betas, su2_start start, uint64_t seed,
                               su2_prec prec, void *device_links, size_t device_bytes, su2_ensemble *out) {
    if (!out || n <= 0 || !dims || !betas) return SU2_EINVAL;
    *out = nullptr;
    if ((start != SU2_COLD && start != SU2_HOT) || (prec != SU2_F32 && prec != SU2_F64)) return SU2_EINVAL;
    if (n > (1 << 23)) return SU2_EINVAL;
    long long sites = 0;
    for (int l = 0; l < n; ++l) {
        if (!dims_ok(dims + 4 * l, prec == SU2_F32)) return SU2_EINVAL;
        if (!(betas[l] >= 0.0) || !std::isfinite(betas[l])) return SU2_EINVAL;
        sites += (long long)dims[4 * l] * dims[4 * l + 1] * dims[4 * l + 2] * dims[4 * l + 3];
    }
    if (sites > (1LL << 31)) return SU2_EINVAL;
    auto *E = new (std::nothrow) su2_ensemble_s();
    if (!E) return SU2_ENOMEM;
    su2_status st = create_common(n, dims, betas, start, seed, prec, device_links, device_bytes, E);
    if (st != SU2_OK) {
        destroy_common(E);
        delete E;
        return st;
    }
    *out = E;
    return SU2_OK;
}

su2_status su2_ensemble_destroy(su2_ensemble ens) {
    if (!ens) return SU2_EINVAL;
    destroy_common(ens);
    delete ens;
    return SU2_OK;
}

su2_status su2_ensemble_set_stream(su2_ensemble E, void *stream) {
    CHK(enter(E));
    HIPCHK(hipStreamSynchronize(E->stream()));
    E->user = (hipStream_t)stream;
    return SU2_OK;
}

su2_status su2_ensemble_set_sampler(su2_ensemble E, su2_sampler sampler) {
    CHK(enter(E));
    if (sampler != SU2_HYBRID && sampler != SU2_CREUTZ) return SU2_EINVAL;
    if (E->sampler != (int)sampler) drop_graphs(E);
    E->sampler = (int)sampler;
    return SU2_OK;
}

su2_status su2_ensemble_run(su2_ensemble E, int nsweeps, int measure_every, uint64_t seed, double *plaq,
                            double *poly) {
    CHK(enter(E));
    if (nsweeps < 0 || measure_every < 1) return SU2_EINVAL;
    if (nsweeps == 0) return SU2_OK;
    const int meas = (plaq ? 1 : 0) | (poly ? 2 : 0);
    const int nm = meas ? nsweeps / measure_every : 0;
    if (nm > 0) CHK(ensure_series(E, nm));
    E->hst.seed = seed;
    E->hst.run_base = E->hst.sweep;
    // the series kernels write measurement k of lattice l to [l * nm + k]
    E->run_plaq = E->dser;
    E->run_poly = E->dser + (size_t)nm * E->n;
    E->run_nm = nm;
    bool err_enqueued = false;
    CHK(run_sweeps(E, nsweeps, nm > 0 ? meas : 0, measure_every, &err_enqueued, true));
    const su2_status st = finish(E, err_enqueued);
    if (st == SU2_EDEVICE) return st;
    for (int m = 0; m < 2 && nm > 0; ++m) {
        double *dst = m == 0 ? plaq : poly;
        if (dst) std::memcpy(dst, E->hser + (size_t)m * nm * E->n, sizeof(double) * nm * E->n);
    }
    return st;
}

static su2_status dims_of(const su2_ensemble_s *E, int i, int *dims) {
    if (!dims || i < 0 || i >= E->n) return SU2_EINVAL;
    for (int k = 0; k < 4; ++k) dims[k] = E->hdesc[i].n[k];
    return SU2_OK;
}

su2_status su2_ensemble_count(su2_ensemble E, int *n) {
    CHK(enter(E));
    if (!n) return SU2_EINVAL;
    *n = E->n;
    return SU2_OK;
}

su2_status su2_ensemble_get_dims(su2_ensemble E, int i, int *dims) {
    CHK(enter(E));
    return dims_of(E, i, dims);
}

su2_status su2_ensemble_get_links(su2_ensemble E, int i, double *host) {
    CHK(enter(E));
    if (i < 0 || i >= E->n || !host) return SU2_EINVAL;
    return get_links_l(E, i, E->links, 4, host);
}

su2_status su2_ensemble_set_links(su2_ensemble E, int i, const double *host) {
    CHK(enter(E));
    if (i < 0 || i >= E->n || !host) return SU2_EINVAL;
    return set_links_l(E, i, host);
}

static su2_status trace_common(su2_ensemble_s *E, int enable) {
    CHK(enter(E));
    HIPCHK(hipStreamSynchronize(E->stream()));
    if (enable) {
        if (!E->trace) {
            CHK(dalloc(E, &E->trace, sizeof(uint32_t) * 4 * (size_t)E->total_sites));
            HIPCHK(hipMemsetAsync(E->trace, 0, sizeof(uint32_t) * 4 * (size_t)E->total_sites, E->stream()));
        }
    } else if (E->trace) {
        HIPCHK(hipFree(E->trace));
        E->trace = nullptr;
    }
    drop_graphs(E);
    return SU2_OK;
}

su2_status su2_ensemble_trace_tries(su2_ensemble E, int enable) { return trace_common(E, enable); }

su2_status su2_ensemble_get_tries(su2_ensemble E, int i, uint32_t *host) {
    CHK(enter(E));
    if (i < 0 || i >= E->n || !host) return SU2_EINVAL;
    if (!E->trace) return SU2_ESTATE;
    const LatDesc &d = E->hdesc[i];
    HIPCHK(hipMemcpyAsync(host, E->trace + d.toff, sizeof(uint32_t) * 8 * (size_t)d.vh, hipMemcpyDeviceToHost,
                          E->stream()));
    HIPCHK(hipStreamSynchronize(E->stream()));
    return SU2_OK;
}

su2_status su2_ensemble_stats(su2_ensemble E, uint64_t *tries, uint64_t *updates) {
    CHK(enter(E));
    return stats_common(E, tries, updates, nullptr);
}

su2_status su2_ensemble_set_launch(su2_ensemble E, int block, int grid, int xcd_remap, int links_per_lane) {
    CHK(enter(E));
    return set_launch_common(E, block, grid, xcd_remap, links_per_lane);
}

su2_status su2_ensemble_get_launch(su2_ensemble E, int *block, int *grid, int *xcd_remap, int *links_per_lane) {
    CHK(enter(E));
    if (block) *block = E->block;
    if (grid) *grid = E->grid;
    if (xcd_remap) *xcd_remap = E->remap;
    if (links_per_lane) *links_per_lane = E->nl;
    return SU2_OK;
}

su2_status su2_ensemble_autotune(su2_ensemble E) {
    CHK(enter(E));
    return autotune_common(E);
}

su2_status su2_ensemble_set_timing(su2_ensemble E, int enable) {
    CHK(enter(E));
    return set_timing_common(E, enable);
}

su2_status su2_ensemble_get_timing(su2_ensemble E, su2_kernel_kind kind, double *ms, int64_t *launches) {
    CHK(enter(E));
    return get_timing_common(E, kind, ms, launches);
}

// ---- single lattice ----------------------------------------------------------
su2_status su2_create(int Nx, int Ny, int Nz, int Nt, su2_start start, uint64_t seed, su2_prec prec,
                      void *device_links, size_t device_bytes, su2_lattice *out) {
    if (!out) return SU2_EINVAL;
    *out = nullptr;
    const int d[4] = {Nx, Ny, Nz, Nt};
    if ((start != SU2_COLD && start != SU2_HOT) || (prec != SU2_F32 && prec != SU2_F64)) return SU2_EINVAL;
    if (!dims_ok(d, prec == SU2_F32)) return SU2_EINVAL;
    auto *E = new (std::nothrow) su2_lattice_s();
    if (!E) return SU2_ENOMEM;
    const double beta = 0.0;
    su2_status st = create_common(1, d, &beta, start, seed, prec, device_links, device_bytes, E);
    if (st != SU2_OK) {
        destroy_common(E);
        delete E;
        return st;
    }
    *out = E;
    return SU2_OK;
}

su2_status su2_destroy(su2_lattice E) {
    if (!E) return SU2_EINVAL;
    destroy_common(E);
    delete E;
    return SU2_OK;
}

su2_status su2_set_stream(su2_lattice E, void *stream) { return su2_ensemble_set_stream(E, stream); }
su2_status su2_set_sampler(su2_lattice E, su2_sampler s) { return su2_ensemble_set_sampler(E, s); }

static su2_status set_beta(su2_ensemble_s *E, double beta) {
    if (E->hdesc[0].beta != beta) {
        E->hdesc[0].beta = beta;
        E->hdesc[0].betaf = (float)beta;
        CHK(upload_desc(E));
    }
    return SU2_OK;
}

su2_status su2_heatbath(su2_lattice E, double beta, int nsweeps, uint64_t seed) {
    CHK(enter(E));
    if (!(beta >= 0.0) || !std::isfinite(beta) || nsweeps < 0) return SU2_EINVAL;
    if (nsweeps == 0) return SU2_OK;
    CHK(set_beta(E, beta));
    CHK(set_seed(E, seed));
    bool err_enqueued = false;
    CHK(run_sweeps(E, nsweeps, 0, 1, &err_enqueued));
    return finish(E, err_enqueued);
}

su2_status su2_heatbath_substep(su2_lattice E, double beta, uint64_t seed, int mu, int parity) {
    CHK(enter(E));
    if (!(beta >= 0.0) || !std::isfinite(beta) || mu < 0 || mu > 3 || (parity != 0 && parity != 1))
        return SU2_EINVAL;
    CHK(set_beta(E, beta));
    CHK(set_seed(E, seed));
    hipStream_t s = E->stream();
    {
        Timed t(E, SU2_K_HEATBATH, s, true);
        KArgs a = kargs(E, 3);
        a.tiles = hb_tiles(E, mu);
        su2::launch_heatbath(a, E->f32, mu, parity, E->nl, E->block, E->grid, s,
                             E->trace != nullptr, false, t.ev());
        t.done(s);
    }
    HIPCHK(hipGetLastError());
    E->updates += (unsigned long long)E->total_links / 8;
    invalidate_measure_buffers(E);
    return SU2_OK;
}

su2_status su2_overrelax(su2_lattice E, int nsweeps) {
    CHK(enter(E));
    if (nsweeps < 0) return SU2_EINVAL;
    hipStream_t s = E->stream();
    const KArgs a = kargs(E);
    for (int k = 0; k < nsweeps; ++k)
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par) {
                Timed t(E, SU2_K_OVERRELAX, s, true);
                su2::launch_overrelax(a, E->f32, mu, par, E->block, E->grid, s, t.ev());
                t.done(s);
            }
    HIPCHK(hipGetLastError());
    if (nsweeps == 0) return SU2_OK;
    invalidate_measure_buffers(E);
    return finish(E);
}

su2_status su2_plaquette(su2_lattice E, double *avg, double *sp, double *tp) {
    CHK(enter(E));
    return measure_plaquette(E, 0, avg, sp, tp);
}

su2_status su2_polyakov(su2_lattice E, double *avg) {
    CHK(enter(E));
    return measure_polyakov(E, 0, avg);
}

su2_status su2_ape_smear(su2_lattice E, double alpha, int nsteps) {
    CHK(enter(E));
    if (!(alpha >= 0.0 && alpha <= 1.0) || nsteps < 0) return SU2_EINVAL;
    const size_t bytes = (size_t)3 * E->total_sites * link_size(E->f32);
    for (int b = 0; b < 2; ++b)
        if (!E->sm[b]) CHK(dalloc(E, &E->sm[b], bytes));
    hipStream_t s = E->stream();
    const KArgs a = kargs(E);
    const void *src = E->links;
    int raw = 1, cur = 0;
    if (nsteps == 0) {  // smeared copy = raw spatial links
        su2::launch_ape(a, E->f32, E->links, 1, E->sm[0], 0.0, E->block, E->grid, s);
        cur = 0;
    }
    for (int k = 0; k < nsteps; ++k) {
        cur = k & 1;
        Timed t(E, SU2_K_APE, s);
        su2::launch_ape(a, E->f32, src, raw, E->sm[cur], alpha, E->block, E->grid, s);
        t.done(s);
        src = E->sm[cur];
        raw = 0;
    }
    HIPCHK(hipGetLastError());
    E->sm_cur = cur;
    return SU2_OK;
}

su2_status su2_get_smeared(su2_lattice E, double *host) {
    CHK(enter(E));
    if (!host) return SU2_EINVAL;
    if (E->sm_cur < 0) return SU2_ESTATE;
    return get_links_l(E, 0, E->sm[E->sm_cur], 3, host);
}

su2_status su2_wilson_loops(su2_lattice E, int Rmax, int Tmax, double *out) {
    CHK(enter(E));
    const LatDesc &d = E->hdesc[0];
    const int smin = std::min(d.n[0], std::min(d.n[1], d.n[2]));
    if (!out || Rmax < 1 || Tmax < 1 || Rmax > smin || Tmax > d.n[3] || Tmax > 32) return SU2_EINVAL;
    const size_t qb = link_size(E->f32);
    const long long V = E->total_sites;
    const size_t sb = qb * (size_t)3 * Rmax * V;
    if (sb > E->wl_s_bytes) {
        CHK(dalloc(E, &E->wl_s, sb));
        E->wl_s_bytes = sb;
    }
    const KArgs va = kargs(E, 2);
    const int nparts = su2::wtrace_groups(va);
    // partials, then the Rmax * Tmax results
    const size_t pb = sizeof(double) * (2 * (size_t)Rmax * nparts * Tmax + (size_t)Rmax * Tmax);
    if (pb > E->wpart_bytes) {
        CHK(dalloc(E, &E->wpart, pb));
        E->wpart_bytes = pb;
    }
    hipStream_t s = E->stream();
    const bool sm = E->sm_cur >= 0;
    Timed t(E, SU2_K_WILSON, s);
    su2::launch_wlines(va, E->f32, sm ? E->sm[E->sm_cur] : E->links, sm ? 0 : 1, Rmax, E->wl_s, E->block, s);
    su2::launch_wtrace(va, E->f32, Rmax, Tmax, V, d.n[3], E->wl_s, E->wpart, E->block, s);
    double *dout = E->wpart + 2 * (size_t)Rmax * nparts * Tmax;
    su2::launch_wfinal(E->ddesc, nparts, Rmax, Tmax, E->wpart, dout, s);
    t.done(s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, dout, sizeof(double) * Rmax * Tmax, hipMemcpyDeviceToHost, s));
    return finish(E);
}

su2_status su2_release_buffers(su2_lattice E) {
    CHK(enter(E));
    HIPCHK(hipStreamSynchronize(E->stream()));
    for (void **b : {&E->sm[0], &E->sm[1], &E->wl_s}) {
        if (*b) HIPCHK(hipFree(*b));
        *b = nullptr;
    }
    if (E->wpart) HIPCHK(hipFree(E->wpart));
    E->wpart = nullptr;
    E->wl_s_bytes = E->wpart_bytes = 0;
    E->sm_cur = -1;
    return SU2_OK;
}

su2_status su2_get_links(su2_lattice E, double *host) {
    CHK(enter(E));
    if (!host) return SU2_EINVAL;
    return get_links_l(E, 0, E->links, 4, host);
}

su2_status su2_set_links(su2_lattice E, const double *host) {
    CHK(enter(E));
    if (!host) return SU2_EINVAL;
    return set_links_l(E, 0, host);
}

su2_status su2_device_links(su2_lattice E, void **ptr, size_t *bytes) {
    CHK(enter(E));
    if (ptr) *ptr = E->links;
    if (bytes) *bytes = E->link_bytes;
    return SU2_OK;
}

su2_status su2_get_dims(su2_lattice E, int *dims) {
    CHK(enter(E));
    return dims_of(E, 0, dims);
}

su2_status su2_get_sweep(su2_lattice E, uint32_t *sweep) {
    CHK(enter(E));
    if (!sweep) return SU2_EINVAL;
    *sweep = E->hst.sweep;
    return SU2_OK;
}

su2_status su2_set_sweep(su2_lattice E, uint32_t sweep) {
    CHK(enter(E));
    E->hst.sweep = sweep;
    return upload_state(E);
}

su2_status su2_stats(su2_lattice E, uint64_t *tries, uint64_t *updates, double *defect) {
    CHK(enter(E));
    return stats_common(E, tries, updates, defect);
}

su2_status su2_trace_tries(su2_lattice E, int enable) { return trace_common(E, enable); }

su2_status su2_get_tries(su2_lattice E, uint32_t *host) {
    CHK(enter(E));
    if (!host) return SU2_EINVAL;
    if (!E->trace) return SU2_ESTATE;
    HIPCHK(hipMemcpyAsync(host, E->trace, sizeof(uint32_t) * 4 * (size_t)E->total_sites, hipMemcpyDeviceToHost,
                          E->stream()));
    HIPCHK(hipStreamSynchronize(E->stream()));
    return SU2_OK;
}

// Checkpoint: "SU2CKPT1", u32 version, i32 Nx Ny Nz Nt, i32 prec, u32 sweep,
// u64 seed, then 16 V float64 in the canonical layout (little-endian).
su2_status su2_save(su2_lattice E, const char *path) {
    CHK(enter(E));
    if (!path) return SU2_EINVAL;
    const LatDesc &d = E->hdesc[0];
    const long long V = 2LL * d.vh;
    std::vector<double> h;
    CHK(host_buf(h, (size_t)16 * V));
    CHK(get_links_l(E, 0, E->links, 4, h.data()));
    FILE *f = std::fopen(path, "wb");
    if (!f) return SU2_EIO;
    const char magic[8] = {'S', 'U', '2', 'C', 'K', 'P', 'T', '1'};
    const uint32_t version = 1;
    const int32_t hdr[5] = {d.n[0], d.n[1], d.n[2], d.n[3], E->f32 ? (int32_t)SU2_F32 : (int32_t)SU2_F64};
    const uint32_t sweep = E->hst.sweep;
    const uint64_t seed = E->hst.seed;
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&version, 4, 1, f) == 1 &&
              std::fwrite(hdr, 4, 5, f) == 5 && std::fwrite(&sweep, 4, 1, f) == 1 &&
              std::fwrite(&seed, 8, 1, f) == 1 && std::fwrite(h.data(), 8, h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SU2_OK : SU2_EIO;
}

// Standalone configuration file: "SU2CONF1", i32 Nx Ny Nz Nt, then 16 V
// float64 in the canonical layout (little-endian); no precision, seed or
// sweep counter.
su2_status su2_save_config(su2_lattice E, const char *path) {
    CHK(enter(E));
    if (!path) return SU2_EINVAL;
    const LatDesc &d = E->hdesc[0];
    const long long V = 2LL * d.vh;
    std::vector<double> h;
    CHK(host_buf(h, (size_t)16 * V));
    CHK(get_links_l(E, 0, E->links, 4, h.data()));
    FILE *f = std::fopen(path, "wb");
    if (!f) return SU2_EIO;
    const char magic[8] = {'S', 'U', '2', 'C', 'O', 'N', 'F', '1'};
    const int32_t ext[4] = {d.n[0], d.n[1], d.n[2], d.n[3]};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(ext, 4, 4, f) == 4 &&
              std::fwrite(h.data(), 8, h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SU2_OK : SU2_EIO;
}

namespace {
// The rest of the file must be exactly the 16 V float64 the header
// announces, checked before anything is allocated for it; then read.
su2_status read_payload(FILE *f, long long V, std::vector<double> &h) {
    const long long payload = 16 * V * (long long)sizeof(double);
    const off_t here = ftello(f);
    off_t end = -1;
    if (here >= 0 && fseeko(f, 0, SEEK_END) == 0) end = ftello(f);
    if (end < here || (long long)(end - here) != payload || fseeko(f, here, SEEK_SET) != 0) return SU2_EIO;
    CHK(host_buf(h, (size_t)16 * V));
    return std::fread(h.data(), 8, h.size(), f) == h.size() ? SU2_OK : SU2_EIO;
}
}  // namespace

su2_status su2_load(const char *path, su2_lattice *out) {
    if (!path || !out) return SU2_EINVAL;
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return SU2_EIO;
    char magic[8];
    uint32_t version = 0, sweep = 0;
    int32_t hdr[5] = {0, 0, 0, 0, (int32_t)SU2_F64};
    uint64_t seed = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8;
    const bool ckpt = ok && std::memcmp(magic, "SU2CKPT1", 8) == 0;
    const bool conf = ok && std::memcmp(magic, "SU2CONF1", 8) == 0;
    if (ckpt)
        ok = std::fread(&version, 4, 1, f) == 1 && version == 1 && std::fread(hdr, 4, 5, f) == 5 &&
             std::fread(&sweep, 4, 1, f) == 1 && std::fread(&seed, 8, 1, f) == 1;
    else if (conf)
        ok = std::fread(hdr, 4, 4, f) == 4;   // binary64, seed 0, sweep 0
    else
        ok = false;
    if (!ok || (hdr[4] != SU2_F32 && hdr[4] != SU2_F64) || !dims_ok(hdr, hdr[4] == SU2_F32)) {
        std::fclose(f);
        return SU2_EIO;
    }
    const long long V = (long long)hdr[0] * hdr[1] * hdr[2] * hdr[3];
    std::vector<double> h;
    const su2_status rs = read_payload(f, V, h);
    std::fclose(f);
    if (rs != SU2_OK) return rs;
    su2_lattice E = nullptr;
    CHK(su2_create(hdr[0], hdr[1], hdr[2], hdr[3], SU2_COLD, seed, (su2_prec)hdr[4], nullptr, 0, &E));
    su2_status st = set_links_l(E, 0, h.data());
    if (st == SU2_OK) {
        E->hst.sweep = sweep;
        E->hst.seed = seed;
        st = upload_state(E);
    }
    if (st == SU2_OK) st = finish(E);
    if (st != SU2_OK) {
        su2_destroy(E);
        return st == SU2_EINVAL ? SU2_EIO : st;
    }
    *out = E;
    return SU2_OK;
}

su2_status su2_set_launch(su2_lattice E, int block, int grid, int remap, int links_per_lane) {
    return su2_ensemble_set_launch(E, block, grid, remap, links_per_lane);
}

su2_status su2_get_launch(su2_lattice E, int *block, int *grid, int *remap, int *links_per_lane) {
    return su2_ensemble_get_launch(E, block, grid, remap, links_per_lane);
}

su2_status su2_autotune(su2_lattice E, double beta) {
    CHK(enter(E));
    if (!(beta >= 0.0) || !std::isfinite(beta)) return SU2_EINVAL;
    CHK(set_beta(E, beta));
    return autotune_common(E);
}

su2_status su2_set_timing(su2_lattice E, int enable) { return su2_ensemble_set_timing(E, enable); }

su2_status su2_get_timing(su2_lattice E, su2_kernel_kind kind, double *ms, int64_t *launches) {
    return su2_ensemble_get_timing(E, kind, ms, launches);
}

}  // extern "C"
