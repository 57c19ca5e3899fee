/*
 * su2.h -- C ABI of the MI355X (gfx950) SU(2) lattice gauge Monte Carlo
 * library: checkerboard heat-bath sweeps of the Wilson action and the
 * measurements they feed.
 *
 * Method: N. Cardoso, P. Bicudo, "SU(2) Lattice Gauge Theory Simulations on
 * Fermi GPUs", arXiv:1010.4834.  Each call below names the section or
 * equation of the paper that defines what it computes.
 *
 * Conventions shared by every call
 *  - Every call returns su2_status (SU2_OK = 0); nothing aborts or throws
 *    across the ABI.  After SU2_EDEVICE the handle is failed and every later
 *    call on it returns SU2_ESTATE (su2_destroy excepted).
 *  - Lattice extents Nx, Ny, Nz, Nt are even and >= 2 (the even/odd
 *    checkerboard of a periodic lattice needs even extents).  mu = 0,1,2 are
 *    x,y,z and mu = 3 is time (the paper's U_4).
 *  - Host link arrays use the canonical layout: site s = x + Nx*(y + Ny*(z +
 *    Nz*t)), element [(s*4 + mu)*4 + c] with c = 0..3 the components
 *    (a0, a1, a2, a3) of U = a0 1 + i a.sigma (paper Sec. 2), in float64.
 *    Host pointers are borrowed for the duration of the call only; host
 *    arrays are sized by the caller (su2_get_dims, su2_ensemble_count and
 *    su2_ensemble_get_dims return the extents).
 *  - Device memory (the link buffer, smeared links, Wilson lines, reduction
 *    partials) is owned by the handle unless the caller passes its own link
 *    buffer to su2_create / su2_ensemble_create, which must then outlive the
 *    handle.  Calls run on the handle's stream.  Calls that return host
 *    results synchronise it, and so do the heat-bath and over-relaxation
 *    sweep calls, which report their own numeric failures (below);
 *    su2_heatbath_substep does not.
 *  - SU2_ENUMERIC: a link whose staple is not finite (a non-finite
 *    neighbour link) is not sampled; it becomes NaN and is counted, as is a
 *    sampler that reaches its try cap.  The call that ran the update returns
 *    SU2_ENUMERIC (a non-synchronising call: the next synchronising call),
 *    and the count is cleared once reported.
 *  - A handle is not thread-safe; separate handles are independent.
 *  - Precision SU2_F32 keeps links in binary32 and does every global
 *    reduction and the reunitarisation norm in binary64 (compensated
 *    two-sum accumulation); SU2_F64 is binary64 throughout.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *    counter = (site, sweep, lattice_id<<8 | purpose<<4 | mu<<1 | parity,
 *    try).  A link update uses one call per try of its a0 draw and the
 *    call with try word 0xFFFFFFFF for the direction of its vector part.
 *    One heat-bath sweep consumes the counters of one sweep index;
 *    each lattice keeps a sweep counter so successive calls continue the
 *    stream.  Link updates do not depend on launch shapes (bit for bit);
 *    reductions agree up to the rounding of their summation order.
 */
#ifndef SU2_H
#define SU2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct su2_lattice_s *su2_lattice;   /* one lattice */
typedef struct su2_ensemble_s *su2_ensemble; /* independent lattices, one launch */

typedef enum {
    SU2_OK = 0,
    SU2_EINVAL = -1,   /* invalid argument                                  */
    SU2_ENOMEM = -2,   /* device or host allocation failed                  */
    SU2_ENODEV = -3,   /* no usable GPU                                     */
    SU2_EDEVICE = -4,  /* a HIP call failed; the handle is now failed       */
    SU2_ESTATE = -5,   /* handle previously failed, or call out of sequence */
    SU2_EIO = -6,      /* file I/O or format error                          */
    SU2_ENUMERIC = -7  /* non-finite value or sampler failure detected      */
} su2_status;

typedef enum { SU2_COLD = 0, SU2_HOT = 1 } su2_start;
typedef enum { SU2_F64 = 0, SU2_F32 = 1 } su2_prec;
/* SU2_HYBRID: Kennedy-Pendleton for alpha = beta*k >= 2, Creutz below it;
 * SU2_CREUTZ: Creutz for every alpha.  Both are exact samplers of the a0
 * law of paper Sec. 2. */
typedef enum { SU2_HYBRID = 0, SU2_CREUTZ = 1 } su2_sampler;

/* Kernel classes for su2_get_timing. */
typedef enum {
    SU2_K_HEATBATH = 0, /* one (mu, parity) heat-bath substep        */
    SU2_K_OVERRELAX = 1,
    SU2_K_PLAQUETTE = 2,
    SU2_K_POLYAKOV = 3,
    SU2_K_REDUCE = 4,   /* final reductions (measurements, series) */
    SU2_K_APE = 5,
    SU2_K_WILSON = 6,
    SU2_K_COUNT = 7
} su2_kernel_kind;

/* Human-readable name of a status code (static storage). */
const char *su2_status_str(su2_status st);

/* Bytes of the native device link buffer of one lattice: 4*V links of 16 B
 * (F32) or 32 B (F64).  Returns 0 for invalid extents (see su2_create). */
size_t su2_link_bytes(int Nx, int Ny, int Nz, int Nt, su2_prec prec);

/* ---- one lattice ------------------------------------------------------ */

/* Allocate a lattice and initialise it (paper Sec. 4 kernel list: cold start
 * U = 1, hot start a Haar-random SU(2) element per link, Haar measure of
 * Sec. 2).  The hot start draws Philox purpose 1 with `seed`.
 * device_links: optional caller-owned device buffer of su2_link_bytes()
 * bytes (NULL: the library allocates).  EINVAL on odd or < 2 extents, a
 * volume above 2^29 sites (SU2_F32) or 2^28 sites (SU2_F64) -- kernels address
 * a link inside its (mu, parity) block with a 32-bit byte offset --,
 * Ny*Nz*Nt >= 2^24 or Nx >= 2^24, or a bad enum; ENODEV without a GPU. */
su2_status su2_create(int Nx, int Ny, int Nz, int Nt, su2_start start, uint64_t seed,
                      su2_prec prec, void *device_links, size_t device_bytes,
                      su2_lattice *out);
/* Waits for the handle's streams, then frees its device and pinned host
 * memory and captured graphs; a caller-owned link buffer is left to the
 * caller.  EINVAL for NULL. */
su2_status su2_destroy(su2_lattice lat);

/* Run later work on this HIP stream (a hipStream_t; NULL = the library's
 * own stream). */
su2_status su2_set_stream(su2_lattice lat, void *hip_stream);
/* Sampler of a0 for later heat-bath calls (SU2_HYBRID by default); EINVAL
 * for other values.  It changes the draws, so a run that switches samplers
 * is a different Markov chain. */
su2_status su2_set_sampler(su2_lattice lat, su2_sampler sampler);

/* nsweeps heat-bath sweeps (paper Sec. 2: each link drawn from
 * exp(beta/2 Tr(U V)), V the staple, via a0 ~ sqrt(1-a0^2) exp(beta k a0)
 * and a random direction; paper Sec. 4: chessboard order, separately by
 * direction and parity).  A sweep is mu = 0..3, even then odd.  The updated
 * link is renormalised with a binary64 norm.  beta >= 0 and finite,
 * nsweeps >= 0, else EINVAL.  Synchronises; ENUMERIC if a staple was not
 * finite or a sampler hit its try cap in these sweeps (the affected links
 * are NaN). */
su2_status su2_heatbath(su2_lattice lat, double beta, int nsweeps, uint64_t seed);

/* A single (mu, parity) heat-bath substep with sweep index = the current
 * counter; the counter is not advanced (custom schedules, parity tests).
 * Does not synchronise: a numeric failure is reported by the next
 * synchronising call. */
su2_status su2_heatbath_substep(su2_lattice lat, double beta, uint64_t seed, int mu,
                                int parity);

/* nsweeps over-relaxation sweeps (paper Sec. 2, over-relaxation equation):
 * U -> W^dag U^dag W^dag with W = V/sqrt(det V), which keeps Tr(U V); same
 * chessboard order; no random numbers; the sweep counter is not advanced.
 * Synchronises; ENUMERIC for a non-finite staple (that link becomes NaN). */
su2_status su2_overrelax(su2_lattice lat, int nsweeps);

/* Mean plaquette (paper Sec. 2, eq. for <P>): 1/2 Re Tr of the oriented
 * plaquette, averaged over the 6V plaquettes (cold start: exactly 1).
 * spatial / temporal: the averages over the 3V planes with nu < 3 / nu = 3.
 * Pointers may be NULL.  Synchronises. */
su2_status su2_plaquette(su2_lattice lat, double *avg, double *spatial, double *temporal);

/* Polyakov loop (paper Sec. 2): (1/N_sigma) sum over spatial sites of
 * 1/2 Tr prod_{t=0}^{Nt-1} U_4(x,t).  Signed, per configuration.
 * Synchronises. */
su2_status su2_polyakov(su2_lattice lat, double *avg);

/* APE smearing of the spatial links (paper Sec. 2, APE equation): nsteps
 * Jacobi steps U' = P_SU(2)[(1-alpha) U + (alpha/4) sum of the four spatial
 * staples], into a separate smeared-link buffer; the Markov chain is not
 * touched.  0 <= alpha <= 1, nsteps >= 0.  The buffer is dropped by the next
 * update of the links. */
su2_status su2_ape_smear(su2_lattice lat, double alpha, int nsteps);

/* On-axis Wilson loops (paper Sec. 2, W(R,T)): out[(R-1)*Tmax + (T-1)] for
 * 1 <= R <= Rmax, 1 <= T <= Tmax, half trace averaged over all sites and the
 * three spatial directions.  Spatial lines use the smeared links when
 * su2_ape_smear produced them since the last update, else the raw links;
 * the temporal sides always use the raw links.  The handle keeps a device
 * buffer of 3*Rmax*V spatial-line quaternions (grown on demand and kept, so
 * that repeated measurements allocate nothing; freed with the handle).  Rmax <= min(Nx,Ny,Nz), Tmax <= min(Nt, 32), else EINVAL.
 * Synchronises. */
su2_status su2_wilson_loops(su2_lattice lat, int Rmax, int Tmax, double *out);

/* Free the measurement buffers the handle keeps between calls: the smeared
 * links (2 x 3V links), the Wilson-line buffer (3 Rmax V quaternions: 382 MB
 * for Rmax = 12 at 24^3 x 48 in binary32) and the Wilson-loop partials.  The
 * next su2_ape_smear / su2_wilson_loops allocates them again; the smeared
 * links are gone (su2_get_smeared: ESTATE).  Synchronises. */
su2_status su2_release_buffers(su2_lattice lat);

/* Copy links to / from a host array in the canonical layout (V*16 float64).
 * set rounds to binary32 for SU2_F32 lattices and rejects non-finite values
 * or links with |1 - |U|^2| > 1e-6 (EINVAL). */
su2_status su2_get_links(su2_lattice lat, double *host);
su2_status su2_set_links(su2_lattice lat, const double *host);
/* Smeared spatial links [s][mu<3][4] float64 (ESTATE if none). */
su2_status su2_get_smeared(su2_lattice lat, double *host);

/* Native device link buffer: [mu][parity][site/2] per lattice; F32 links are
 * float4, F64 links two float64x2 planes (a0,a1) and (a2,a3) per
 * (mu, parity) block. */
su2_status su2_device_links(su2_lattice lat, void **device_ptr, size_t *bytes);

/* Extents Nx, Ny, Nz, Nt of the lattice into dims[0..3], from which a caller
 * sizes the host arrays above (V = Nx Ny Nz Nt).  EINVAL if dims is NULL. */
su2_status su2_get_dims(su2_lattice lat, int *dims);

/* Sweep counter (the Philox sweep word of the next sweep). */
su2_status su2_get_sweep(su2_lattice lat, uint32_t *sweep);
su2_status su2_set_sweep(su2_lattice lat, uint32_t sweep);

/* Cumulative heat-bath tries and updates, and the largest |1 - |U|^2| over
 * the current links.  Any pointer may be NULL.  Synchronises. */
su2_status su2_stats(su2_lattice lat, uint64_t *tries, uint64_t *updates,
                     double *max_unit_defect);

/* Per-link record of later heat-bath calls: tries | creutz << 31, in
 * canonical [s][mu] order (V*4 uint32).  enable = 0 frees it. */
su2_status su2_trace_tries(su2_lattice lat, int enable);
su2_status su2_get_tries(su2_lattice lat, uint32_t *host);

/* Configuration files (paper Sec. 4 kernel list: a configuration read from
 * an input file as the third way to initialise the lattice).  All values
 * little-endian.
 * Checkpoint (su2_save): "SU2CKPT1", u32 version 1, i32 Nx Ny Nz Nt, i32
 * precision, u32 sweep counter, u64 seed, then 16 V float64 links in the
 * canonical layout.  A resumed run is bitwise identical to an uninterrupted
 * one (the random stream is counter based).
 * Configuration (su2_save_config): "SU2CONF1", i32 Nx Ny Nz Nt, then the
 * 16 V float64 links in the canonical layout; no precision, seed or sweep
 * counter, so any writer that knows the layout can produce one. */
su2_status su2_save(su2_lattice lat, const char *path);
su2_status su2_save_config(su2_lattice lat, const char *path);
/* Reads either file.  A checkpoint restores precision, seed and sweep
 * counter; a configuration gives a binary64 lattice with seed 0 and sweep
 * counter 0.  EIO for anything else: wrong magic or version, invalid
 * extents or precision, a payload other than exactly 16 V float64 (checked
 * before it is read), or links that are not unit quaternions; ENOMEM if the
 * host copy of the links cannot be allocated.  *out is NULL on failure. */
su2_status su2_load(const char *path, su2_lattice *out);

/* Launch shape: threads per workgroup (64, 128, 192 or 256), resident
 * workgroups of the persistent grid (0 = one workgroup per tile; else a
 * multiple of 8), the tile mode (0: tiles round-robin over the XCDs; 1: each
 * XCD takes a contiguous share of the tile list; 2: as 1, with the heat-bath
 * tiles of every direction in (z, t, y, x) order, which modes 0 and 1 use for
 * the temporal direction only; 3: as 1, with each lattice's heat-bath tiles
 * in eight blocks -- (z half, t quarter) for mu < 3, (z quarter, y half) for
 * mu = 3 -- so that an XCD's share reads fewer halo links), and heat-bath
 * links per lane (1, 2 or 4: a
 * lane draws its links in one rejection loop).  Link updates do not depend
 * on it; reductions only in rounding.  EINVAL for other values. */
su2_status su2_set_launch(su2_lattice lat, int block, int grid, int xcd_remap, int links_per_lane);
su2_status su2_get_launch(su2_lattice lat, int *block, int *grid, int *xcd_remap, int *links_per_lane);
/* Time the candidate launch shapes on this lattice and keep the fastest
 * (the links are saved and restored around the trial sweeps). */
su2_status su2_autotune(su2_lattice lat, double beta);

/* Per-kernel timing with HIP events on the handle's stream (enable = 1
 * also disables graph replay so every kernel is timed).  Heat-bath and
 * over-relaxation launches have their events stamped by the launch itself
 * with the kernel's start and end; the other kernels are bracketed by event
 * records (which adds the dispatch latency).  get_timing
 * returns the summed milliseconds and launch count since enabling. */
su2_status su2_set_timing(su2_lattice lat, int enable);
su2_status su2_get_timing(su2_lattice lat, su2_kernel_kind kind, double *ms, int64_t *launches);

/* ---- allocation-free heat bath ---------------------------------------- */

/* For callers that cannot allocate device memory or synchronise: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * nsweeps heat-bath sweeps, exactly those of su2_heatbath (bit for bit the
 * same links for the same links, beta, seed and sweep counter; hybrid
 * sampler), of ONE lattice held by the caller in device memory in the
 * native layout of su2_device_links (device_links, su2_link_bytes bytes,
 * updated in place), enqueued on hip_stream (NULL: the null stream) of the
 * current device.  `sweep` is the Philox sweep word of the first sweep (the
 * caller keeps the counter: the next call continues with sweep + nsweeps).
 * Allocates nothing and does not synchronise: the state, descriptor, tile
 * list and try counters live in a fixed device array of 4 MiB + 512 B per
 * GPU, held until the process ends, so lattices are limited to 2^27 sites
 * (EINVAL beyond; also EINVAL for the arguments su2_create / su2_heatbath
 * refuse or a NULL device_links).  Every call on a GPU uses that GPU's one
 * array: calls that overlap on one GPU (other streams, other threads) race
 * and must be ordered by the caller.  device_err (nullable, device memory)
 * receives the count of non-finite staples and try-cap hits of this call
 * (the affected links are NaN).  ENODEV without a current device, EDEVICE
 * if a launch fails. */
su2_status su2_heatbath_noalloc(void *device_links, int Nx, int Ny, int Nz, int Nt, su2_prec prec,
                                double beta, int nsweeps, uint64_t seed, uint32_t sweep,
                                uint32_t *device_err, void *hip_stream);

/* ---- ensembles of independent lattices -------------------------------- */

/* n independent lattices of uneven sizes and couplings that advance in the
 * same kernel launches (paper Sec. 2 heat bath and Sec. 4 chessboard on each
 * lattice; one workgroup walks a (lattice, tile) list).  dims: n*4 extents
 * (host, read during the call); betas: n couplings; lattice i uses
 * lattice_id i in the Philox counter; hot starts draw with `seed`.  The
 * lattices lie back to back in one link buffer: device_links, if not NULL,
 * is a caller-owned device buffer of at least the sum of su2_link_bytes()
 * over the lattices (device_bytes, else EINVAL), which the library uses
 * but never frees.  EINVAL for n < 1 or n > 2^23, a NULL array, any
 * lattice su2_create would refuse, more than 2^31 sites in all, or a beta
 * < 0 or not finite; ENODEV without a GPU;
 * EDEVICE or ENOMEM if device or pinned memory cannot be had. */
su2_status su2_ensemble_create(int n, const int *dims, const double *betas, su2_start start,
                               uint64_t seed, su2_prec prec, void *device_links,
                               size_t device_bytes, su2_ensemble *out);
su2_status su2_ensemble_destroy(su2_ensemble ens);
su2_status su2_ensemble_set_stream(su2_ensemble ens, void *hip_stream);
su2_status su2_ensemble_set_sampler(su2_ensemble ens, su2_sampler sampler);

/* nsweeps heat-bath sweeps of every lattice at its own beta (paper Sec. 2
 * heat bath, Sec. 4 chessboard), with the mean plaquette and Polyakov loop
 * (paper Sec. 2) of every lattice measured after every measure_every-th
 * sweep: with M = nsweeps / measure_every, measurement k (after sweep
 * (k+1)*measure_every of the run) of lattice i goes to plaq[i*M + k] and
 * poly[i*M + k]; the last nsweeps % measure_every sweeps measure nothing.
 * Either pointer may be NULL to skip that measurement.  The sweeps (eight
 * substep launches each; the plaquette is summed inside the odd substeps of
 * measured sweeps) are replayed from captured HIP graphs: a run of 2 to 256
 * sweeps is one graph (run state, sweeps, series reduction and error word),
 * captured on the first run of that length, measure_every and measurement
 * choice; longer runs replay graphs of up to 16 sweeps (environment
 * SU2_GRAPH_SWEEPS) and of the smaller powers of two.  Partial sums are
 * reduced once per batch of measurements and the series stay on the device
 * until the end.  Measuring does not change the Markov chain.
 * Synchronises once; ENUMERIC as for su2_heatbath.  measure_every >= 1,
 * nsweeps >= 0, else EINVAL.  Environment SU2_NO_GRAPH launches every
 * kernel directly. */
su2_status su2_ensemble_run(su2_ensemble ens, int nsweeps, int measure_every, uint64_t seed,
                            double *plaq, double *poly);
/* Number of lattices, and the extents Nx, Ny, Nz, Nt of lattice i into
 * dims[0..3]: the series of su2_ensemble_run hold count*(nsweeps /
 * measure_every) values and the link arrays of lattice i V_i*16.  EINVAL for
 * a NULL pointer or i out of range.  The calls below act as their su2_*
 * counterparts on lattice i (links in the canonical host layout, V_i*16
 * float64; set rounds to binary32 for SU2_F32 and refuses non-unit links)
 * or on the whole ensemble (statistics summed over the lattices; one launch
 * shape, timing and try record for all of them). */
su2_status su2_ensemble_count(su2_ensemble ens, int *n);
su2_status su2_ensemble_get_dims(su2_ensemble ens, int i, int *dims);
su2_status su2_ensemble_get_links(su2_ensemble ens, int i, double *host);
su2_status su2_ensemble_set_links(su2_ensemble ens, int i, const double *host);
su2_status su2_ensemble_stats(su2_ensemble ens, uint64_t *tries, uint64_t *updates);
/* Per-link try record of later sweeps of every lattice (as su2_trace_tries);
 * lattice i's record, V_i*4 uint32 in canonical [s][mu] order. */
su2_status su2_ensemble_trace_tries(su2_ensemble ens, int enable);
su2_status su2_ensemble_get_tries(su2_ensemble ens, int i, uint32_t *host);
su2_status su2_ensemble_set_launch(su2_ensemble ens, int block, int grid, int xcd_remap,
                                   int links_per_lane);
su2_status su2_ensemble_get_launch(su2_ensemble ens, int *block, int *grid, int *xcd_remap,
                                   int *links_per_lane);
su2_status su2_ensemble_autotune(su2_ensemble ens);
su2_status su2_ensemble_set_timing(su2_ensemble ens, int enable);
su2_status su2_ensemble_get_timing(su2_ensemble ens, su2_kernel_kind kind, double *ms,
                                   int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* SU2_H */
