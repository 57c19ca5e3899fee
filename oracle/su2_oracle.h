/*
 * su2_oracle.h -- serial FP64 CPU oracle for checkerboard SU(2) heat-bath
 * lattice gauge Monte Carlo (Cardoso & Bicudo, "SU(2) Lattice Gauge Theory
 * Simulations on Fermi GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  It
 * is plain, slow and written to be read against the paper; it shares no code
 * with the GPU path (no headers, helpers or tables).  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Canonical layout used throughout the oracle (and by the library's host
 * interchange calls): site index s = x + Nx*(y + Ny*(z + Nz*t)), link array
 * U[(s*4 + mu)*4 + c], c = 0..3 the quaternion components (a0, a1, a2, a3)
 * of U = a0*1 + i a.sigma  (paper Sec. 2, SU(2) parametrisation).
 * mu = 0,1,2 are x,y,z; mu = 3 is the temporal direction (the paper's U_4).
 *
 * Parity unpinned: the Philox counter layout, the uniform conversion, the
 * hybrid sampler switch and the sweep order are conventions of this code
 * (the paper uses an LCG / CURAND and prints no sampler code); they are
 * pinned only by agreement of independent implementations and statistics.
 */
#ifndef SU2_ORACLE_H
#define SU2_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* sampler selection (paper Sec. 2, a0 distribution; Creutz cited there) */
#define OR_SAMPLER_HYBRID 0 /* Kennedy-Pendleton for alpha >= 2, Creutz below */
#define OR_SAMPLER_CREUTZ 1 /* Creutz for every alpha                         */
#define OR_SAMPLER_KP     2 /* Kennedy-Pendleton for every alpha (tests only) */

/* Philox random-number purposes (third counter word) */
#define OR_PURPOSE_HEATBATH 0
#define OR_PURPOSE_HOT      1
#define OR_PURPOSE_GAUGE    2

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 4). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* one 32-bit word -> uniform in (0,1); bits = 32 (FP64 lattices) or 23
 * (FP32 lattices).  Both are exact in binary64. */
double or_uniform(uint32_t w, int bits);

/* quaternion product c = a*b for U = a0 + i a.sigma (paper Sec. 2) */
void or_qmul(const double a[4], const double b[4], double c[4]);

/* 0 if every extent is even and >= 2, else -1 */
int or_check_dims(const int n[4]);
int64_t or_volume(const int n[4]);
int or_parity(const int n[4], int64_t s);
int64_t or_neighbor(const int n[4], int64_t s, int mu, int step);

/* initial configurations (paper Sec. 4 kernel list: cold / hot start) */
void or_cold(const int n[4], double *U);
void or_hot(const int n[4], double *U, uint64_t seed, uint32_t lat_id);

/* staple V of link (s, mu): the weight of the link is exp(beta/2 Tr(U V)) */
void or_staple(const int n[4], const double *U, int64_t s, int mu, double V[4]);

/* one heat-bath draw of delta = 1 - a0 at coupling alpha = beta*k; returns
 * the number of tries.  ctr3 = the first three Philox counter words; the try
 * index is the fourth. *used_creutz (nullable) reports the sampler branch. */
uint32_t or_sample_delta(double alpha, int sampler, uint64_t seed,
                         const uint32_t ctr3[3], int ubits, double *delta,
                         int *used_creutz);

/* the full draw X = (a0, a), a isotropic of norm sqrt(1 - a0^2) from its
 * own Philox call (try word 0xFFFFFFFF); returns the tries */
uint32_t or_sample_link(double alpha, int sampler, uint64_t seed, const uint32_t ctr3[3],
                        int ubits, double X[4], int *used_creutz);

/* n draws with counters (i, 0, 0, try), i = 0..n-1 (sampler statistics) */
void or_sample_many(double alpha, int sampler, uint64_t seed, int64_t nsamp,
                    int ubits, double *delta, uint32_t *tries);

/* heat-bath update of the single link (s, mu); returns the trace word */
uint32_t or_heatbath_link(const int n[4], double *U, int64_t s, int mu,
                          double beta, uint64_t seed, uint32_t sweep,
                          uint32_t lat_id, int sampler, int ubits);

/* heat-bath update of one substep (mu, parity) / one full sweep.
 * trace (nullable, [V][4] uint32): per link, tries | (creutz << 31).
 * order (nullable): permutation of 0..V-1 giving the visiting order inside
 * each (mu, parity) class (used to show the class members are independent).
 * Returns the total number of tries. */
uint64_t or_heatbath_substep(const int n[4], double *U, double beta,
                             uint64_t seed, uint32_t sweep, uint32_t lat_id,
                             int sampler, int ubits, int mu, int parity,
                             uint32_t *trace, const int64_t *order);
uint64_t or_heatbath_sweep(const int n[4], double *U, double beta,
                           uint64_t seed, uint32_t sweep, uint32_t lat_id,
                           int sampler, int ubits, uint32_t *trace,
                           const int64_t *order);

/* over-relaxation sweep: U -> W^dag U^dag W^dag, W = V/|V| */
void or_overrelax_sweep(const int n[4], double *U);

/* mean plaquette: tot = (1/6V) sum 1/2 Tr U_P, sp / tp = spatial / temporal
 * planes, each normalised by 3V (any pointer nullable) */
void or_plaquette(const int n[4], const double *U, double *tot, double *sp,
                  double *tp);

/* Polyakov loop (1/N_sigma) sum_x 1/2 Tr prod_t U_3(x,t) */
double or_polyakov(const int n[4], const double *U);

/* APE smearing of the spatial links; S = [V][3][4] smeared spatial links */
void or_ape(const int n[4], const double *U, double alpha, int nsteps, double *S);

/* on-axis Wilson loops W[(R-1)*Tmax + (T-1)], R = 1..Rmax, T = 1..Tmax.
 * Spatial lines use S ([V][3][4]) when given, else the links in U. */
void or_wilson(const int n[4], const double *U, const double *S, int Rmax,
               int Tmax, double *W);

/* the single loop W(R,T) of or_wilson (sampled checks at large sizes) */
double or_wilson_rt(const int n[4], const double *U, const double *S, int R, int T);

/* random gauge transformation U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag */
void or_gauge_transform(const int n[4], double *U, uint64_t seed);

/* largest |1 - |U|^2| over all links */
double or_max_unit_defect(const int n[4], const double *U);

#ifdef __cplusplus
}
#endif
#endif
