/*
 * su2_oracle.c -- serial FP64 oracle for the SU(2) checkerboard heat bath.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU baseline to check the GPU library.  Never part of the
 * product path.  Shares no code with the GPU library.
 *
 * Paper: N. Cardoso, P. Bicudo, "SU(2) Lattice Gauge Theory Simulations on
 * Fermi GPUs" (arXiv:1010.4834).  Citations below name its sections and
 * equations.  Built with -O2 -ffp-contract=off, no fast-math.
 */
#include "su2_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon et al., SC'11,
 * Sec. 4.2): each round multiplies counter words 0 and 2 by two fixed odd
 * constants, swaps/xors the halves with the key, and the key is advanced by
 * the Weyl constants (golden ratio, sqrt(3)-1) between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double or_uniform(uint32_t w, int bits)
{
    if (bits == 23) /* (2m+1) 2^-24 with m the top 23 bits */
        return (2.0 * (double)(w >> 9) + 1.0) * 0x1p-24;
    return (2.0 * (double)w + 1.0) * 0x1p-33; /* (2w+1) 2^-33 */
}

/* counter word 2: lattice id, purpose, direction and parity */
static uint32_t or_tag(uint32_t lat_id, int purpose, int mu, int parity)
{
    return (lat_id << 8) | ((uint32_t)purpose << 4) | ((uint32_t)mu << 1) | (uint32_t)parity;
}

static void or_draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                    uint32_t c3, uint32_t w[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, w);
}

/* ------------------------------------------------------------------------ */
/* SU(2) elements as four reals, U = a0 + i a.sigma (paper Sec. 2).
 * Product: (a0 b0 - a.b,  a0 b + b0 a - a x b). */
void or_qmul(const double a[4], const double b[4], double c[4])
{
    double r0 = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double r1 = a[0] * b[1] + b[0] * a[1] - (a[2] * b[3] - a[3] * b[2]);
    double r2 = a[0] * b[2] + b[0] * a[2] - (a[3] * b[1] - a[1] * b[3]);
    double r3 = a[0] * b[3] + b[0] * a[3] - (a[1] * b[2] - a[2] * b[1]);
    c[0] = r0; c[1] = r1; c[2] = r2; c[3] = r3;
}

static void or_dag(const double a[4], double c[4])
{
    c[0] = a[0]; c[1] = -a[1]; c[2] = -a[2]; c[3] = -a[3];
}

static void or_set(double c[4], const double a[4]) { memcpy(c, a, 4 * sizeof(double)); }

/* ------------------------------------------------------------------------ */
/* Periodic hypercubic lattice (paper Sec. 2: periodic in time and space). */
int or_check_dims(const int n[4])
{
    for (int d = 0; d < 4; ++d)
        if (n[d] < 2 || (n[d] & 1)) return -1;
    return 0;
}

int64_t or_volume(const int n[4]) { return (int64_t)n[0] * n[1] * n[2] * n[3]; }

static void or_coords(const int n[4], int64_t s, int c[4])
{
    for (int d = 0; d < 4; ++d) {
        c[d] = (int)(s % n[d]);
        s /= n[d];
    }
}

static int64_t or_index(const int n[4], const int c[4])
{
    return (int64_t)c[0] + (int64_t)n[0] * (c[1] + (int64_t)n[1] * (c[2] + (int64_t)n[2] * c[3]));
}

int or_parity(const int n[4], int64_t s)
{
    int c[4];
    or_coords(n, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

int64_t or_neighbor(const int n[4], int64_t s, int mu, int step)
{
    int c[4];
    or_coords(n, s, c);
    c[mu] = ((c[mu] + step) % n[mu] + n[mu]) % n[mu];
    return or_index(n, c);
}

static double *or_link(double *U, int64_t s, int mu) { return U + (s * 4 + mu) * 4; }
static const double *or_clink(const double *U, int64_t s, int mu) { return U + (s * 4 + mu) * 4; }

/* ------------------------------------------------------------------------ */
/* Initial configurations (paper Sec. 4, "Cold start" / "Hot start").
 * Hot start: a Haar-random element (measure of paper Sec. 2) from four
 * Box-Muller normals of one Philox call, normalised. */
void or_cold(const int n[4], double *U)
{
    int64_t V = or_volume(n);
    for (int64_t i = 0; i < 4 * V; ++i) {
        double *u = U + 4 * i;
        u[0] = 1.0; u[1] = 0.0; u[2] = 0.0; u[3] = 0.0;
    }
}

static void or_haar_from_words(const uint32_t w[4], double u[4])
{
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = or_uniform(w[0], 32), u1 = or_uniform(w[1], 32);
    double u2 = or_uniform(w[2], 32), u3 = or_uniform(w[3], 32);
    double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
    double z[4] = {r01 * cos(two_pi * u1), r01 * sin(two_pi * u1),
                   r23 * cos(two_pi * u3), r23 * sin(two_pi * u3)};
    double nrm = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2] + z[3] * z[3]);
    for (int c = 0; c < 4; ++c) u[c] = z[c] / nrm;
}

void or_hot(const int n[4], double *U, uint64_t seed, uint32_t lat_id)
{
    int64_t V = or_volume(n);
    for (int64_t s = 0; s < V; ++s) {
        int p = or_parity(n, s);
        for (int mu = 0; mu < 4; ++mu) {
            uint32_t w[4];
            or_draw(seed, (uint32_t)s, 0u, or_tag(lat_id, OR_PURPOSE_HOT, mu, p), 0u, w);
            or_haar_from_words(w, or_link(U, s, mu));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Staple (paper Sec. 2, the six plaquettes containing a link, and the
 * over-relaxation equation for Sigma).  Sigma is the sum of the six
 * transporters x -> x+mu; the heat-bath weight exp(beta/2 Tr(U V)) needs
 * V = Sigma^dag, so that Tr(U_mu(x) V) is the sum of the six plaquette
 * traces containing U_mu(x).  Summed nu ascending, upper then lower:
 *   upper: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
 *   lower: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)                     */
void or_staple(const int n[4], const double *U, int64_t s, int mu, double V[4])
{
    V[0] = V[1] = V[2] = V[3] = 0.0;
    int64_t xp = or_neighbor(n, s, mu, +1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int64_t xpn = or_neighbor(n, s, nu, +1);
        int64_t xmn = or_neighbor(n, s, nu, -1);
        int64_t xpmn = or_neighbor(n, xp, nu, -1);
        double a[4], b[4], t[4], up[4], dn[4];

        or_dag(or_clink(U, xpn, mu), b);
        or_qmul(or_clink(U, xp, nu), b, t);
        or_dag(or_clink(U, s, nu), a);
        or_qmul(t, a, up);

        or_dag(or_clink(U, xpmn, nu), a);
        or_dag(or_clink(U, xmn, mu), b);
        or_qmul(a, b, t);
        or_qmul(t, or_clink(U, xmn, nu), dn);

        for (int c = 0; c < 4; ++c) V[c] += up[c];
        for (int c = 0; c < 4; ++c) V[c] += dn[c];
    }
}

/* ------------------------------------------------------------------------ */
/* a0 sampler (paper Sec. 2): a0 in [-1,1] with density proportional to
 * sqrt(1 - a0^2) exp(alpha a0), alpha = beta k.  We draw delta = 1 - a0.
 *
 * Kennedy-Pendleton (Phys. Lett. B 156 (1985) 393): with uniforms r1..r4,
 *   lambda^2 = -(ln r1 + cos^2(2 pi r2) ln r3) / (2 alpha),
 *   accept iff r4^2 <= 1 - lambda^2, then delta = 2 lambda^2.
 * Creutz (Phys. Rev. D 21 (1980) 2308, cited in paper Sec. 2): draw
 *   a0 from exp(alpha a0) on [-1,1] by inversion, accept with probability
 *   sqrt(1 - a0^2).  In delta form, with c = 1 - exp(-2 alpha):
 *   delta = -log1p(-(1-u1) c) / alpha, accept iff u2^2 <= delta (2 - delta);
 *   for alpha < 1e-20 the exp(alpha a0) factor is below binary64 resolution
 *   and delta = 2 (1 - u1).
 * One Philox call per try; counter word 3 is the try index.              */
uint32_t or_sample_delta(double alpha, int sampler, uint64_t seed,
                         const uint32_t ctr3[3], int ubits, double *delta,
                         int *used_creutz)
{
    const double two_pi = 6.283185307179586476925286766559;
    int creutz = (sampler == OR_SAMPLER_CREUTZ) ||
                 (sampler == OR_SAMPLER_HYBRID && !(alpha >= 2.0));
    if (used_creutz) *used_creutz = creutz;
    double c = creutz ? -expm1(-2.0 * alpha) : 0.0;
    for (uint32_t j = 0;; ++j) {
        uint32_t w[4];
        or_draw(seed, ctr3[0], ctr3[1], ctr3[2], j, w);
        if (creutz) {
            double u1 = or_uniform(w[0], ubits), u2 = or_uniform(w[1], ubits);
            double d = (alpha >= 1e-20) ? -log1p(-(1.0 - u1) * c) / alpha
                                        : 2.0 * (1.0 - u1);
            if (u2 * u2 <= d * (2.0 - d)) {
                *delta = d;
                return j + 1;
            }
        } else {
            double r1 = or_uniform(w[0], ubits), r2 = or_uniform(w[1], ubits);
            double r3 = or_uniform(w[2], ubits), r4 = or_uniform(w[3], ubits);
            double cs = cos(two_pi * r2);
            double lam2 = -(log(r1) + cs * cs * log(r3)) / (2.0 * alpha);
            if (r4 * r4 <= 1.0 - lam2) {
                *delta = 2.0 * lam2;
                return j + 1;
            }
        }
    }
}

/* Draw X = (x0, x): x0 = a0 from the law of paper Sec. 2 by
 * or_sample_delta's loop, and x uniformly on the 2-sphere of radius
 * sqrt(1 - x0^2) from its own Philox call (try word 0xFFFFFFFF):
 * cos(theta) = 1 - 2 u1, phi = 2 pi u2, |x| = sqrt(delta (2 - delta)).
 * The direction thus does not depend on the number of tries or on alpha.
 * Returns the tries; *used_creutz (nullable) reports the branch. */
uint32_t or_sample_link(double alpha, int sampler, uint64_t seed, const uint32_t ctr3[3],
                        int ubits, double X[4], int *used_creutz)
{
    const double two_pi = 6.283185307179586476925286766559;
    double d;
    uint32_t tries = or_sample_delta(alpha, sampler, seed, ctr3, ubits, &d, used_creutz);
    uint32_t w[4];
    or_draw(seed, ctr3[0], ctr3[1], ctr3[2], 0xFFFFFFFFu, w);
    double u1 = or_uniform(w[0], ubits), u2 = or_uniform(w[1], ubits);
    double cth = 1.0 - 2.0 * u1;
    double sth = 2.0 * sqrt(u1 * (1.0 - u1));
    double ra = sqrt(d * (2.0 - d));
    X[0] = 1.0 - d;
    X[1] = ra * sth * cos(two_pi * u2);
    X[2] = ra * sth * sin(two_pi * u2);
    X[3] = ra * cth;
    return tries;
}

/* Heat-bath update of link (s, mu) (paper Sec. 2): X from or_sample_link
 * with coupling alpha = beta k, k = sqrt(det V); U' = X W^dag with W = V/k
 * (the identity if V = 0), renormalised. */
static uint32_t or_update_link(const int n[4], double *U, int64_t s, int mu,
                               double beta, uint64_t seed, uint32_t sweep,
                               uint32_t lat_id, int sampler, int ubits)
{
    int p = or_parity(n, s);
    double V[4];
    or_staple(n, U, s, mu, V);
    double k2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2] + V[3] * V[3];
    double k = sqrt(k2);
    double alpha = beta * k;

    uint32_t ctr3[3] = {(uint32_t)s, sweep, or_tag(lat_id, OR_PURPOSE_HEATBATH, mu, p)};
    double X[4];
    int creutz;
    uint32_t tries = or_sample_link(alpha, sampler, seed, ctr3, ubits, X, &creutz);

    double Wd[4];
    if (k2 > 0.0) {
        Wd[0] = V[0] / k; Wd[1] = -V[1] / k; Wd[2] = -V[2] / k; Wd[3] = -V[3] / k;
    } else {
        Wd[0] = 1.0; Wd[1] = Wd[2] = Wd[3] = 0.0;
    }
    double Un[4];
    or_qmul(X, Wd, Un);
    double nrm = sqrt(Un[0] * Un[0] + Un[1] * Un[1] + Un[2] * Un[2] + Un[3] * Un[3]);
    double *u = or_link(U, s, mu);
    for (int c = 0; c < 4; ++c) u[c] = Un[c] / nrm;
    return tries | ((uint32_t)creutz << 31);
}

uint32_t or_heatbath_link(const int n[4], double *U, int64_t s, int mu,
                          double beta, uint64_t seed, uint32_t sweep,
                          uint32_t lat_id, int sampler, int ubits)
{
    return or_update_link(n, U, s, mu, beta, seed, sweep, lat_id, sampler, ubits);
}

void or_sample_many(double alpha, int sampler, uint64_t seed, int64_t nsamp,
                    int ubits, double *delta, uint32_t *tries)
{
    for (int64_t i = 0; i < nsamp; ++i) {
        uint32_t ctr3[3] = {(uint32_t)i, 0u, 0u};
        uint32_t t = or_sample_delta(alpha, sampler, seed, ctr3, ubits, delta + i, NULL);
        if (tries) tries[i] = t;
    }
}

/* Chessboard update (paper Sec. 4): links are updated separately by
 * direction and by even/odd sites.  Order: mu = 0..3, even then odd. */
uint64_t or_heatbath_substep(const int n[4], double *U, double beta,
                             uint64_t seed, uint32_t sweep, uint32_t lat_id,
                             int sampler, int ubits, int mu, int parity,
                             uint32_t *trace, const int64_t *order)
{
    int64_t V = or_volume(n);
    uint64_t total = 0;
    for (int64_t i = 0; i < V; ++i) {
        int64_t s = order ? order[i] : i;
        if (or_parity(n, s) != parity) continue;
        uint32_t t = or_update_link(n, U, s, mu, beta, seed, sweep, lat_id, sampler, ubits);
        total += t & 0x7FFFFFFFu;
        if (trace) trace[s * 4 + mu] = t;
    }
    return total;
}

uint64_t or_heatbath_sweep(const int n[4], double *U, double beta,
                           uint64_t seed, uint32_t sweep, uint32_t lat_id,
                           int sampler, int ubits, uint32_t *trace,
                           const int64_t *order)
{
    uint64_t total = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p)
            total += or_heatbath_substep(n, U, beta, seed, sweep, lat_id, sampler,
                                         ubits, mu, p, trace, order);
    return total;
}

/* Over-relaxation (paper Sec. 2).  The printed form uses Sigma^dag on both
 * sides; the action-preserving reflection is U' = W^dag U^dag W^dag with
 * W = V/|V| (V = Sigma^dag), for which Tr(U' V) = Tr(U V). */
void or_overrelax_sweep(const int n[4], double *U)
{
    int64_t V = or_volume(n);
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p)
            for (int64_t s = 0; s < V; ++s) {
                if (or_parity(n, s) != p) continue;
                double St[4];
                or_staple(n, U, s, mu, St);
                double k2 = St[0] * St[0] + St[1] * St[1] + St[2] * St[2] + St[3] * St[3];
                if (!(k2 > 0.0)) continue;
                double k = sqrt(k2);
                double Wd[4] = {St[0] / k, -St[1] / k, -St[2] / k, -St[3] / k};
                double Ud[4], t[4], r[4];
                or_dag(or_clink(U, s, mu), Ud);
                or_qmul(Wd, Ud, t);
                or_qmul(t, Wd, r);
                double nrm = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
                double *u = or_link(U, s, mu);
                for (int c = 0; c < 4; ++c) u[c] = r[c] / nrm;
            }
}

/* ------------------------------------------------------------------------ */
/* Neumaier compensated summation */
typedef struct { double sum, comp; } or_acc;

static void or_acc_add(or_acc *a, double v)
{
    double t = a->sum + v;
    if (fabs(a->sum) >= fabs(v))
        a->comp += (a->sum - t) + v;
    else
        a->comp += (v - t) + a->sum;
    a->sum = t;
}

static double or_acc_get(const or_acc *a) { return a->sum + a->comp; }

/* Mean plaquette (paper Sec. 2, eq. for <P>): 1/2 Re Tr of
 * U_mu(s) U_nu(s+mu) U_mu(s+nu)^dag U_nu(s)^dag, averaged over the 6 V
 * plaquettes (so a cold start gives exactly 1). */
void or_plaquette(const int n[4], const double *U, double *tot, double *sp, double *tp)
{
    int64_t V = or_volume(n);
    or_acc a_sp = {0, 0}, a_tp = {0, 0}, a_all = {0, 0};
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                int64_t smu = or_neighbor(n, s, mu, +1), snu = or_neighbor(n, s, nu, +1);
                double a[4], b[4], t1[4], t2[4], t3[4];
                or_qmul(or_clink(U, s, mu), or_clink(U, smu, nu), t1);
                or_dag(or_clink(U, snu, mu), a);
                or_qmul(t1, a, t2);
                or_dag(or_clink(U, s, nu), b);
                or_qmul(t2, b, t3);
                or_acc_add(&a_all, t3[0]);
                if (nu == 3) or_acc_add(&a_tp, t3[0]);
                else         or_acc_add(&a_sp, t3[0]);
            }
    if (tot) *tot = or_acc_get(&a_all) / (6.0 * (double)V);
    if (sp) *sp = or_acc_get(&a_sp) / (3.0 * (double)V);
    if (tp) *tp = or_acc_get(&a_tp) / (3.0 * (double)V);
}

/* Polyakov loop (paper Sec. 2): product of the temporal links from t = 0 to
 * Nt-1 in ascending t, half trace, averaged over the spatial sites. */
double or_polyakov(const int n[4], const double *U)
{
    int64_t Ns = (int64_t)n[0] * n[1] * n[2];
    or_acc acc = {0, 0};
    for (int64_t xs = 0; xs < Ns; ++xs) {
        double P[4] = {1, 0, 0, 0}, t[4];
        for (int tt = 0; tt < n[3]; ++tt) {
            or_qmul(P, or_clink(U, xs + Ns * tt, 3), t);
            or_set(P, t);
        }
        or_acc_add(&acc, P[0]);
    }
    return or_acc_get(&acc) / (double)Ns;
}

/* APE smearing (paper Sec. 2, the APE equation) of the spatial links only,
 * with the four spatial staples (both orientations of the two other spatial
 * directions), each a transporter x -> x+mu:
 *   U' = P_SU(2)[(1-alpha) U + (alpha/4) sum of staples].
 * For SU(2) the projection of a nonzero multiple of an element is its
 * normalisation.  All links of a step are smeared from the previous step. */
void or_ape(const int n[4], const double *U, double alpha, int nsteps, double *S)
{
    int64_t V = or_volume(n);
    double *A = (double *)malloc(sizeof(double) * 12 * V);
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 3; ++mu) or_set(S + (s * 3 + mu) * 4, or_clink(U, s, mu));
    for (int step = 0; step < nsteps; ++step) {
        memcpy(A, S, sizeof(double) * 12 * V);
        for (int64_t s = 0; s < V; ++s)
            for (int mu = 0; mu < 3; ++mu) {
                double sum[4] = {0, 0, 0, 0};
                int64_t xp = or_neighbor(n, s, mu, +1);
                for (int nu = 0; nu < 3; ++nu) {
                    if (nu == mu) continue;
                    int64_t xpn = or_neighbor(n, s, nu, +1), xmn = or_neighbor(n, s, nu, -1);
                    int64_t xmnp = or_neighbor(n, xmn, mu, +1);
                    double a[4], b[4], t[4], st[4];
                    /* forward: U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag */
                    or_qmul(A + (s * 3 + nu) * 4, A + (xpn * 3 + mu) * 4, t);
                    or_dag(A + (xp * 3 + nu) * 4, b);
                    or_qmul(t, b, st);
                    for (int c = 0; c < 4; ++c) sum[c] += st[c];
                    /* backward: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) */
                    or_dag(A + (xmn * 3 + nu) * 4, a);
                    or_qmul(a, A + (xmn * 3 + mu) * 4, t);
                    or_qmul(t, A + (xmnp * 3 + nu) * 4, st);
                    for (int c = 0; c < 4; ++c) sum[c] += st[c];
                }
                const double *u = A + (s * 3 + mu) * 4;
                double w[4];
                for (int c = 0; c < 4; ++c) w[c] = (1.0 - alpha) * u[c] + 0.25 * alpha * sum[c];
                double nrm = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
                double *o = S + (s * 3 + mu) * 4;
                if (nrm > 0.0)
                    for (int c = 0; c < 4; ++c) o[c] = w[c] / nrm;
                else
                    or_set(o, u);
            }
    }
    free(A);
}

/* On-axis Wilson loop (paper Sec. 2, W(R,T)): spatial line of R links along
 * mu from x, temporal line of T links from x + R mu, the spatial line back
 * from x + T t, the temporal line back to x.  Half trace, averaged over all
 * sites and the three spatial directions (W(1,1) is then the mean
 * spatial-temporal plaquette). */
double or_wilson_rt(const int n[4], const double *U, const double *S, int R, int T)
{
    int64_t V = or_volume(n);
    or_acc acc = {0, 0};
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 3; ++mu) {
            double L[4] = {1, 0, 0, 0}, t[4], d[4];
            int64_t y = s;
            for (int i = 0; i < R; ++i) { /* S_mu(x; R) */
                const double *u = S ? S + (y * 3 + mu) * 4 : or_clink(U, y, mu);
                or_qmul(L, u, t); or_set(L, t);
                y = or_neighbor(n, y, mu, +1);
            }
            for (int j = 0; j < T; ++j) { /* T(x + R mu; T) */
                or_qmul(L, or_clink(U, y, 3), t); or_set(L, t);
                y = or_neighbor(n, y, 3, +1);
            }
            for (int i = 0; i < R; ++i) { /* back along -mu */
                y = or_neighbor(n, y, mu, -1);
                const double *u = S ? S + (y * 3 + mu) * 4 : or_clink(U, y, mu);
                or_dag(u, d); or_qmul(L, d, t); or_set(L, t);
            }
            for (int j = 0; j < T; ++j) { /* back along -t */
                y = or_neighbor(n, y, 3, -1);
                or_dag(or_clink(U, y, 3), d); or_qmul(L, d, t); or_set(L, t);
            }
            or_acc_add(&acc, L[0]);
        }
    return or_acc_get(&acc) / (3.0 * (double)V);
}

void or_wilson(const int n[4], const double *U, const double *S, int Rmax,
               int Tmax, double *W)
{
    for (int R = 1; R <= Rmax; ++R)
        for (int T = 1; T <= Tmax; ++T)
            W[(R - 1) * Tmax + (T - 1)] = or_wilson_rt(n, U, S, R, T);
}

/* Gauge transformation with a Haar-random g(x) per site (purpose 2). */
void or_gauge_transform(const int n[4], double *U, uint64_t seed)
{
    int64_t V = or_volume(n);
    double *g = (double *)malloc(sizeof(double) * 4 * V);
    for (int64_t s = 0; s < V; ++s) {
        uint32_t w[4];
        or_draw(seed, (uint32_t)s, 0u, or_tag(0, OR_PURPOSE_GAUGE, 0, or_parity(n, s)), 0u, w);
        or_haar_from_words(w, g + 4 * s);
    }
    for (int64_t s = 0; s < V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            double gd[4], t[4];
            or_dag(g + 4 * or_neighbor(n, s, mu, +1), gd);
            or_qmul(g + 4 * s, or_clink(U, s, mu), t);
            or_qmul(t, gd, or_link(U, s, mu));
        }
    free(g);
}

double or_max_unit_defect(const int n[4], const double *U)
{
    int64_t V = or_volume(n);
    double m = 0.0;
    for (int64_t i = 0; i < 4 * V; ++i) {
        const double *u = U + 4 * i;
        double d = fabs(1.0 - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + u[3] * u[3]));
        if (d > m) m = d;
    }
    return m;
}
