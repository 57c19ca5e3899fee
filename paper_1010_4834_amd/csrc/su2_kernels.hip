// su2_kernels.hip -- gfx950 kernels of the SU(2) library and their launchers.
//
// Method: Cardoso & Bicudo, "SU(2) Lattice Gauge Theory Simulations on Fermi
// GPUs" (arXiv:1010.4834); each kernel names the passage it implements.
// All kernels walk a (lattice, tile) list so one launch advances a whole
// batch of independent lattices; per-tile lattice data live in scalar
// registers and every link load is one global load from a scalar block base
// plus a 32-bit lane offset.  Nothing here is a dense contraction (at most
// 4x4 real products per quaternion): no MFMA, vector-ALU code fed by
// coalesced float4 / float64x2 loads of the parity-split layout.
#include <hip/hip_ext.h>

#include "su2_internal.hpp"

namespace su2 {

// ---------------------------------------------------------------------------
// Site coordinates of half-site `cb` of parity `par`.
struct Site {
    int c[4];  // x, y, z, t
    int s;     // full-site index
};

__device__ __forceinline__ Site site_of(const LatDesc &d, int cb, int par) {
    Site S;
    int row, j, r2, y, z, t;
    udiv(cb, d.hx, d.inv_hx, row, j);
    udiv(row, d.n[1], d.inv_ny, r2, y);
    udiv(r2, d.n[2], d.inv_nz, t, z);
    const int x = 2 * j + ((par + y + z + t) & 1);
    S.c[0] = x; S.c[1] = y; S.c[2] = z; S.c[3] = t;
    S.s = x + (int)__umul24((unsigned)d.n[0], (unsigned)row);  // row < Ny Nz Nt < 2^24
    return S;
}

// Periodic forward / backward steps of the full-site index along mu.
__device__ __forceinline__ int stride_of(const LatDesc &d, int mu) {
    return mu == 0 ? 1 : mu == 1 ? d.n[0] : mu == 2 ? d.n[0] * d.n[1] : d.ns;
}
// Both candidate steps are uniform; they are pinned as scalars so that the
// select picks one of them rather than a multiplier of the stride (which
// would put a 32-bit vector multiply on every neighbour).
__device__ __forceinline__ int step_fwd(const LatDesc &d, const Site &S, int mu) {
    const int st = stride_of(d, mu);
    const int in = uni(st), wrap = uni(-(d.n[mu] - 1) * st);
    return S.c[mu] == d.n[mu] - 1 ? wrap : in;
}
__device__ __forceinline__ int step_bwd(const LatDesc &d, const Site &S, int mu) {
    const int st = stride_of(d, mu);
    const int in = uni(-st), wrap = uni((d.n[mu] - 1) * st);
    return S.c[mu] == 0 ? wrap : in;
}

// Uniform bases of the (direction, parity) blocks of one lattice in a link
// buffer whose lattice starts at link `first` ([mu][parity][cb]).
template <class T, int NDIR> struct Blocks {
    char *b[NDIR][2];
    uint32_t hoff;
};
template <class T, int NDIR>
__device__ __forceinline__ Blocks<T, NDIR> blocks(const void *buf, long long first, int vh) {
    Blocks<T, NDIR> B;
#pragma unroll
    for (int mu = 0; mu < NDIR; ++mu)
#pragma unroll
        for (int p = 0; p < 2; ++p)
            B.b[mu][p] = (char *)buf + (first + (long long)(2 * mu + p) * vh) * Links<T>::BYTES;
    B.hoff = (uint32_t)vh << 4;
    return B;
}

// Block base of (mu, p); an unrolled select so the bases stay in scalar
// registers (indexing the array with run-time values would spill it to
// private memory and turn every link load into a flat load).
template <class T, int NDIR>
__device__ __forceinline__ char *bsel(const Blocks<T, NDIR> &B, int mu, int p) {
    char *r = B.b[0][0];
#pragma unroll
    for (int m = 0; m < NDIR; ++m) {
        r = (mu == m && p == 0) ? B.b[m][0] : r;
        r = (mu == m && p == 1) ? B.b[m][1] : r;
    }
    return r;
}

template <class T, int NDIR>
__device__ __forceinline__ Q<T> lds_(const Blocks<T, NDIR> &B, int mu, int p, uint32_t cb) {
    return Links<T>::ld(bsel(B, mu, p), B.hoff, cb);
}
template <class T, int NDIR>
__device__ __forceinline__ void sts_(const Blocks<T, NDIR> &B, int mu, int p, uint32_t cb, const Q<T> &q) {
    Links<T>::st(bsel(B, mu, p), B.hoff, cb, q);
}

// Staple V of link (x, MU), x of parity `par` (paper Sec. 2: the six
// plaquettes containing the link; V is the adjoint of the sum of the
// transporters x -> x+mu of the over-relaxation equation, so that the link
// weight is exp(beta/2 Tr(U V))).  nu ascending, upper then lower:
//   upper U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag,
//   lower U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu).
// 18 link loads (gather); 7 distinct per update once shared with
// neighbouring lanes.  combine() does the arithmetic on the gathered links.
template <class T, int MU>
__device__ __forceinline__ void gather(const LatDesc &d, const Blocks<T, 4> &B, const Site &S, int par,
                                       Q<T> (&L)[18]) {
    const int op = par ^ 1;
    const int s_mu = S.s + step_fwd(d, S, MU);
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU) continue;
        const int q = 6 * (nu < MU ? nu : nu - 1);
        const int fn = step_fwd(d, S, nu), bn = step_bwd(d, S, nu);
        L[q + 0] = lds_(B, nu, op, (uint32_t)s_mu >> 1);            // U_nu(x+mu)
        L[q + 1] = lds_(B, MU, op, (uint32_t)(S.s + fn) >> 1);      // U_mu(x+nu)
        L[q + 2] = lds_(B, nu, par, (uint32_t)S.s >> 1);            // U_nu(x)
        L[q + 3] = lds_(B, nu, par, (uint32_t)(s_mu + bn) >> 1);    // U_nu(x+mu-nu)
        L[q + 4] = lds_(B, MU, op, (uint32_t)(S.s + bn) >> 1);      // U_mu(x-nu)
        L[q + 5] = lds_(B, nu, op, (uint32_t)(S.s + bn) >> 1);      // U_nu(x-nu)
    }
}

// V accumulates nu ascending, upper then lower staple, in one chain of
// fused multiply-adds.  The planes nu < MU come first, so Vlow (the fused
// plaquette) is V as it stands after plane MU - 1: the substep updates its
// links bit for bit the same with and without the plaquette.
template <class T, int MU>
__device__ __forceinline__ Q<T> combine(const Q<T> (&L)[18], Q<T> *Vlow = nullptr) {
    Q<T> V{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU) continue;
        const int q = 6 * (nu < MU ? nu : nu - 1);
        const Q<T> &A = L[q + 0], &Bm = L[q + 1], &C = L[q + 2], &D = L[q + 3], &E = L[q + 4], &F = L[q + 5];
        qmul_acc(V, A, qdag(qmul(C, Bm)));
        qmul_acc(V, qdag(qmul(E, D)), F);
        if (Vlow && nu == MU - 1) *Vlow = V;
    }
    return V;
}

template <class T, int MU>
__device__ __forceinline__ Q<T> staple(const LatDesc &d, const Blocks<T, 4> &B, const Site &S, int par,
                                       Q<T> *Vlow = nullptr) {
    Q<T> L[18];
    gather<T, MU>(d, B, S, par, L);
    return combine<T, MU>(L, Vlow);
}

template <class T, int N> __device__ __forceinline__ T pick(const T (&a)[N], int m) {
    T r = a[0];
#pragma unroll
    for (int k = 1; k < N; ++k) r = (m == k) ? a[k] : r;
    return r;
}
template <class T, int N> __device__ __forceinline__ void put(T (&a)[N], int m, T v) {
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (m == k) a[k] = v;
}


// ---------------------------------------------------------------------------
// Heat-bath substep (paper Sec. 2 heat bath; Sec. 4 chessboard): every link
// (x, MU) with parity(x) = par is redrawn from exp(beta/2 Tr(U V)).
// a0 from Kennedy-Pendleton (alpha >= 2) or Creutz (alpha < 2, or always
// with the Creutz sampler); one Philox call per try, counter (s, sweep,
// tag, try); the direction of the vector part from the call with try word
// 0xFFFFFFFF.  New link X W^dag with W = V/k, renormalised with a binary64
// norm.  The samplers multiply by 1/alpha, formed once per link (binary32:
// the hardware reciprocal, within 1 ulp; binary64: a division), instead of
// dividing on every try.
//
// Each lane owns NL links of the class (one per block-sized slice of its
// tile).  Staples first; then a single rejection loop in which a lane moves
// on to its next link as soon as one is accepted, so a wavefront waits for
// the lane with the most tries over NL links rather than NL times for the
// slowest lane; then the new links are composed and stored.
//
// PLAQ (odd substeps, MU >= 1): every plaquette of a plane (nu, MU) with
// nu < MU holds exactly one MU-link at an odd site, updated here after all
// its other links are final; 1/2 Tr(U' (upper + lower staple of plane nu))
// over nu < MU and over the three odd substeps MU = 1, 2, 3 is therefore the
// plaquette sum (paper Sec. 2, eq. for <P>) of the configuration at the end
// of the sweep; by linearity only the summed staple of those planes is
// kept.  Each wavefront writes its binary64 sum to slot MU-1 of its tile.
template <class T, int MU, bool TRACE, int NL, bool PLAQ>
__global__ __launch_bounds__(256) void k_heatbath(KArgs a, int par) {
    using M = Mth<T>;
    // the first substep of a sweep takes the sweep word from `next`, and so
    // does a lone substep (no advance: part of the next sweep to run)
    const bool first = a.advance && MU == 0 && par == 0;
    const uint32_t sweep = uni((first || !a.advance) ? a.st->next : a.st->sweep);
    const uint32_t k0 = uni((unsigned)a.st->seed), k1 = uni((unsigned)(a.st->seed >> 32));
    if (a.advance && blockIdx.x == 0 && threadIdx.x == 0) {
        if (first) a.st->sweep = sweep;
        if (MU == 3 && par == 1) a.st->next = sweep + 1u;
    }
    double *plaq_part = a.plaq_part;
    if (PLAQ && a.nslots > 0)
        plaq_part += (long long)(((sweep - uni(a.st->run_base)) / (uint32_t)a.every) % (uint32_t)a.nslots) * 12 *
                     a.ntiles;
    TileWalk w(a.ntiles, a.xcd_remap);
    if (!w.ok()) return;
    int tile = w.tile();
    Tile tl = load_tile(a.tiles, tile);
    LatDesc d = load_desc(a.desc + tl.x);
    while (true) {
        const Blocks<T, 4> B = blocks<T, 4>(a.links, d.off, d.vh);
        const uint32_t c2 = tag(d.lat_id, PURPOSE_HEATBATH, MU, par);
        const T beta = (sizeof(T) == 4) ? (T)d.betaf : (T)d.beta;

        int sidx[NL];
        T alpha[NL], ial[NL];  // alpha = beta k and its reciprocal (0 when alpha = 0)
        Q<T> Wd[NL];
        Q<T> Vl[NL];  // summed staples of the planes nu < MU (PLAQ only)
        uint32_t pend = 0, nonfinite = 0;
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int cb = tl.y + m * (int)blockDim.x + (int)threadIdx.x;
            sidx[m] = 0;
            alpha[m] = T(0);
            ial[m] = T(0);
            Wd[m] = qone<T>();
            if (cb < d.vh) {
                Vl[m] = Q<T>{T(0), T(0), T(0), T(0)};
                const Site S = site_of(d, cb, par);
                const Q<T> V = staple<T, MU>(d, B, S, par, PLAQ ? &Vl[m] : nullptr);
                const T k2 = V.a * V.a + V.b * V.b + V.c * V.c + V.d * V.d;
                // a non-finite staple (a non-finite neighbour link) is not
                // sampled: the link becomes NaN and the error word counts it
                if (k2 <= M::MAXV) pend |= 1u << m;
                else nonfinite |= 1u << m;
                T k, ik;
                if (sizeof(T) == 4) {
                    ik = M::rsqrt_(k2);
                    k = k2 > T(0) ? k2 * ik : T(0);
                } else {
                    k = M::sqrt_(k2);
                    ik = T(1) / k;
                }
                sidx[m] = S.s;
                alpha[m] = beta * k;
                if (alpha[m] > T(0)) ial[m] = M::rcp_(alpha[m]);
                if (k2 > T(0)) Wd[m] = Q<T>{V.a * ik, -V.b * ik, -V.c * ik, -V.d * ik};
            }
        }

        // Creutz factor -expm1(-2 alpha) per link, formed only when a lane of
        // the wavefront samples with Creutz (as a loop invariant it would
        // otherwise be hoisted and evaluated for every link).
        T cfv[NL];
        bool creutz_any = false;
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            cfv[m] = T(0);
            creutz_any |= ((pend >> m) & 1u) && ((a.sampler == 1) || !(alpha[m] >= T(2)));
        }
        if (__ballot(creutz_any)) {
#pragma unroll
            for (int m = 0; m < NL; ++m)
                if (((pend >> m) & 1u) && alpha[m] >= T(1e-20)) cfv[m] = -M::expm1_(T(-2) * alpha[m]);
        }

        // Rejection loop: a lane moves to its next link when one is accepted.
        T delta[NL];
        uint32_t rec[NL];
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            delta[m] = ((nonfinite >> m) & 1u) ? M::nan_() : T(0);
            rec[m] = 0;
        }
        if (__ballot(nonfinite != 0u)) {
            if (nonfinite) atomicAdd(a.err, (unsigned)__popc(nonfinite));
        }
        // The loop runs while any lane of the wavefront has a link pending;
        // each pass is one try of every active lane, so the wavefront's try
        // count is the sum of the active-lane counts (scalar work).
        uint32_t j = 0, wtries = 0;
        while (true) {
            const unsigned long long act = __ballot(pend != 0u);
            if (act == 0ull) break;
            wtries += (uint32_t)__popcll(act);
            if (!pend) continue;
            const int m = __builtin_ctz(pend);
            const int s = pick(sidx, m);
            const T al = pick(alpha, m), ia = pick(ial, m);
            const bool creutz = (a.sampler == 1) || !(al >= T(2));
            const uint4 wd = philox10((uint32_t)s, sweep, c2, j, k0, k1);
            bool acc;
            T dl;
            if (creutz) {
                const T u1 = M::u(wd.x), u2 = M::u(wd.y);
                if (al >= T(1e-20)) {
                    const T cf = pick(cfv, m);
                    dl = -M::log1p_(-(T(1) - u1) * cf) * ia;
                } else {
                    dl = T(2) * (T(1) - u1);
                }
                acc = u2 * u2 <= dl * (T(2) - dl);
            } else {
                const T r1 = M::u(wd.x), r2 = M::u(wd.y), r3 = M::u(wd.z), r4 = M::u(wd.w);
                const T cs = M::cos2pi(r2);
                const T lam2 = -(M::lg(r1) + cs * cs * M::lg(r3)) * (ia * (T(0.5) * M::LN_LG));
                acc = r4 * r4 <= T(1) - lam2;
                dl = T(2) * lam2;
            }
            ++j;
            if (acc || j >= MAX_TRIES) {
                if (!acc) {
                    atomicAdd(a.err, 1u);
                    dl = M::nan_();
                }
                put(delta, m, dl);
                put(rec, m, j | ((uint32_t)creutz << 31));
                pend &= pend - 1;
                j = 0;
            }
        }

        // Direction from its own Philox call (try word 0xFFFFFFFF), then
        // U' = X W^dag, renormalised.
        double pq = 0.0;
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int cb = tl.y + m * (int)blockDim.x + (int)threadIdx.x;
            if (cb < d.vh) {
                const uint4 wd = philox10((uint32_t)sidx[m], sweep, c2, 0xFFFFFFFFu, k0, k1);
                const T u1 = M::u(wd.x), u2 = M::u(wd.y);
                const T dl = delta[m];
                const T cth = T(1) - T(2) * u1;
                const T sth = T(2) * M::sqrt_(u1 * (T(1) - u1));
                const T ra = M::sqrt_(dl * (T(2) - dl));
                const T rs = ra * sth;
                const Q<T> X{T(1) - dl, rs * M::cos2pi(u2), rs * M::sin2pi(u2), ra * cth};
                const Q<T> Un = qnormalize(qmul(X, Wd[m]));
                sts_(B, MU, par, (uint32_t)cb, Un);
                if (TRACE) a.trace[d.toff + (long long)sidx[m] * 4 + MU] = rec[m];
                if (PLAQ)  // 1/2 Re Tr(U' V_low)
                    pq += (double)(Un.a * Vl[m].a - Un.b * Vl[m].b - Un.c * Vl[m].c - Un.d * Vl[m].d);
            }
        }
        if (PLAQ) {
            pq = wave_sum_f64(pq);
            if ((threadIdx.x & 63) == 0)
                plaq_part[(3 * (long long)tile + (MU - 1)) * 4 + (threadIdx.x >> 6)] = pq;
        }
        if ((threadIdx.x & 63) == 0 && wtries) atomicAdd(&a.tries_part[tile], (unsigned long long)wtries);
        if (!w.next()) break;
        tile = w.tile();
        tl = load_tile(a.tiles, tile);
        d = load_desc(a.desc + tl.x);
    }
}

// Over-relaxation substep (paper Sec. 2, over-relaxation equation, in its
// action-preserving form U' = W^dag U^dag W^dag, W = V/k).
template <class T, int MU>
__global__ __launch_bounds__(256) void k_overrelax(KArgs a, int par) {
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = load_tile(a.tiles, tile);
        const LatDesc d = load_desc(a.desc + tl.x);
        const Blocks<T, 4> B = blocks<T, 4>(a.links, d.off, d.vh);
        const int cb = tl.y + (int)threadIdx.x;
        if (cb >= d.vh) return;
        const Site S = site_of(d, cb, par);
        const Q<T> V = staple<T, MU>(d, B, S, par);
        const T k2 = V.a * V.a + V.b * V.b + V.c * V.c + V.d * V.d;
        if (!(k2 <= Mth<T>::MAXV)) {  // non-finite staple: NaN link, counted
            atomicAdd(a.err, 1u);
            const T nan = Mth<T>::nan_();
            sts_(B, MU, par, (uint32_t)cb, Q<T>{nan, nan, nan, nan});
            return;
        }
        if (!(k2 > T(0))) return;
        const T ik = T(1) / Mth<T>::sqrt_(k2);
        const Q<T> Wd{V.a * ik, -V.b * ik, -V.c * ik, -V.d * ik};
        const Q<T> U = lds_(B, MU, par, (uint32_t)cb);
        sts_(B, MU, par, (uint32_t)cb, qnormalize(qmul(qmul(Wd, qdag(U)), Wd)));
    });
}

// ---------------------------------------------------------------------------
// Initial configurations (paper Sec. 4: cold start U = 1; hot start a
// Haar-random element per link, Haar measure of Sec. 2): one Philox call
// (purpose 1, sweep 0, try 0) -> four Box-Muller normals in binary64 ->
// normalised, rounded to the link precision.
template <class T>
__global__ __launch_bounds__(256) void k_init(KArgs a, int hot) {
    const unsigned long long seed = a.st->seed;
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = load_tile(a.tiles, tile);
        const LatDesc d = load_desc(a.desc + tl.x);
        const Blocks<T, 4> B = blocks<T, 4>(a.links, d.off, d.vh);
        const int cb = tl.y + (int)threadIdx.x;
        if (cb >= d.vh) return;
        for (int par = 0; par < 2; ++par) {
            const Site S = site_of(d, cb, par);
            for (int mu = 0; mu < 4; ++mu) {
                Q<double> z = qone<double>();
                if (hot) {
                    const uint4 w = philox10((uint32_t)S.s, 0u, tag(d.lat_id, PURPOSE_HOT, mu, par),
                                             0u, (uint32_t)seed, (uint32_t)(seed >> 32));
                    const double u0 = Mth<double>::u(w.x), u1 = Mth<double>::u(w.y);
                    const double u2 = Mth<double>::u(w.z), u3 = Mth<double>::u(w.w);
                    const double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
                    const double tp = 6.283185307179586476925286766559;
                    z = Q<double>{r01 * cos(tp * u1), r01 * sin(tp * u1), r23 * cos(tp * u3),
                                  r23 * sin(tp * u3)};
                    const double nrm = sqrt(z.a * z.a + z.b * z.b + z.c * z.c + z.d * z.d);
                    z = Q<double>{z.a / nrm, z.b / nrm, z.c / nrm, z.d / nrm};
                }
                sts_(B, mu, par, (uint32_t)cb, Q<T>{(T)z.a, (T)z.b, (T)z.c, (T)z.d});
            }
        }
    });
}

// Canonical float64 [s][mu][4] <-> native layout (ndir = 4: links,
// ndir = 3: smeared spatial links).  One lattice per launch (the tile list
// holds only its tiles); `canon` is that lattice's canonical array.
template <class T>
__global__ __launch_bounds__(256) void k_from_canon(KArgs a, const double *canon) {
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = load_tile(a.tiles, tile);
        const LatDesc d = load_desc(a.desc + tl.x);
        const Blocks<T, 4> B = blocks<T, 4>(a.links, d.off, d.vh);
        const int cb = tl.y + (int)threadIdx.x;
        if (cb >= d.vh) return;
        const double *c = canon;
        for (int par = 0; par < 2; ++par) {
            const Site S = site_of(d, cb, par);
            for (int mu = 0; mu < 4; ++mu) {
                const double *u = c + ((long long)S.s * 4 + mu) * 4;
                sts_(B, mu, par, (uint32_t)cb, Q<T>{(T)u[0], (T)u[1], (T)u[2], (T)u[3]});
            }
        }
    });
}

template <class T>
__global__ __launch_bounds__(256) void k_to_canon(KArgs a, const void *src, int ndir, double *canon) {
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = load_tile(a.tiles, tile);
        const LatDesc d = load_desc(a.desc + tl.x);
        const long long base = ndir == 4 ? d.off : d.soff;
        const Blocks<T, 4> B = blocks<T, 4>(src, base, d.vh);
        const int cb = tl.y + (int)threadIdx.x;
        if (cb >= d.vh) return;
        double *c = canon;
        for (int par = 0; par < 2; ++par) {
            const Site S = site_of(d, cb, par);
            for (int mu = 0; mu < ndir; ++mu) {
                const Q<T> q = lds_(B, mu, par, (uint32_t)cb);
                double *u = c + ((long long)S.s * ndir + mu) * 4;
                u[0] = q.a; u[1] = q.b; u[2] = q.c; u[3] = q.d;
            }
        }
    });
}

// Largest |1 - |U|^2| (bit pattern of a non-negative double is monotone).
template <class T>
__global__ __launch_bounds__(256) void k_unit_defect(KArgs a, unsigned long long *out) {
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = load_tile(a.tiles, tile);
        const LatDesc d = load_desc(a.desc + tl.x);
        const Blocks<T, 4> B = blocks<T, 4>(a.links, d.off, d.vh);
        const int cb = tl.y + (int)threadIdx.x;
        double m = 0.0;
        if (cb < d.vh)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const Q<T> u = lds_(B, q >> 1, q & 1, (uint32_t)cb);
                const double n2 = (double)u.a * u.a + (double)u.b * u.b + (double)u.c * u.c +
                                  (double)u.d * u.d;
                const double e = fabs(1.0 - n2);
                m = (e > m || e != e) ? e : m;
            }
#pragma unroll
        for (int k = 32; k >= 1; k >>= 1) {
            const double o = __shfl_xor(m, k, 64);
            m = (o > m || o != o) ? o : m;
        }
        if ((threadIdx.x & 63) == 0) {
            const unsigned long long bits = (m != m) ? 0x7FF8000000000000ull : __double_as_longlong(m);
            atomicMax(out, bits);
        }
    });
}

// ---------------------------------------------------------------------------
// Plaquette partial sums (paper Sec. 2, eq. for <P>): per site, the six
// planes mu < nu of 1/2 Tr[U_mu(s) U_nu(s+mu) U_mu(s+nu)^dag U_nu(s)^dag]
// = 1/2 Tr[(U_mu(s) U_nu(s+mu)) (U_nu(s) U_mu(s+nu))^dag], traced in link
// precision, accumulated in binary64 per lane, then a compensated block sum
// per tile (spatial, temporal planes).
template <class T>
__global__ __launch_bounds__(256) void k_plaquette(KArgs a, double *part) {
    __shared__ DD lds[2 * 4];
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = load_tile(a.tiles, tile);
        const LatDesc d = load_desc(a.desc + tl.x);
        const Blocks<T, 4> B = blocks<T, 4>(a.links, d.off, d.vh);
        const int cb = tl.y + (int)threadIdx.x;
        DD acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
        if (cb < d.vh) {
            double sp = 0.0, tp = 0.0;
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                const Site S = site_of(d, cb, par);
                const int op = par ^ 1;
                Q<T> U[4];
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) U[mu] = lds_(B, mu, par, (uint32_t)cb);
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    const uint32_t smu = (uint32_t)(S.s + step_fwd(d, S, mu)) >> 1;
#pragma unroll
                    for (int nu = mu + 1; nu < 4; ++nu) {
                        const uint32_t snu = (uint32_t)(S.s + step_fwd(d, S, nu)) >> 1;
                        const Q<T> Unu_smu = lds_(B, nu, op, smu);
                        const Q<T> Umu_snu = lds_(B, mu, op, snu);
                        const T tr = half_tr_xyd(qmul(U[mu], Unu_smu), qmul(U[nu], Umu_snu));
                        if (nu == 3) tp += (double)tr;
                        else sp += (double)tr;
                    }
                }
            }
            acc[0] = DD{sp, 0.0};
            acc[1] = DD{tp, 0.0};
        }
        dd_block_sum<2>(acc, lds);
        if (threadIdx.x == 0) {
            part[4 * tile + 0] = acc[0].hi; part[4 * tile + 1] = acc[0].lo;
            part[4 * tile + 2] = acc[1].hi; part[4 * tile + 3] = acc[1].lo;
        }
    });
}

// Polyakov loop partial sums (paper Sec. 2): per spatial site, the product
// of the temporal links t = 0 .. Nt-1 in ascending t, half trace.
template <class T>
__global__ __launch_bounds__(256) void k_polyakov(KArgs a, double *part) {
    __shared__ DD lds[4];
    if (a.nslots > 0)
        part += (long long)(((uni(a.st->sweep) - uni(a.st->run_base)) / (uint32_t)a.every) % (uint32_t)a.nslots) *
                2 * a.ntiles;
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = load_tile(a.tiles, tile);
        const LatDesc d = load_desc(a.desc + tl.x);
        const Blocks<T, 4> B = blocks<T, 4>(a.links, d.off, d.vh);
        const int xs = tl.y + (int)threadIdx.x;
        DD acc[1] = {{0.0, 0.0}};
        if (xs < d.ns) {
            int row, x, z, y;
            udiv(xs, d.n[0], d.inv_nx, row, x);
            udiv(row, d.n[1], d.inv_ny, z, y);
            Q<T> P = qone<T>();
            const int p0 = (x + y + z) & 1;
            // unrolled so that the loads of several t issue together ahead
            // of the (ordered) product chain
#pragma unroll 4
            for (int t = 0; t < d.n[3]; ++t) {
                const uint32_t cb = (uint32_t)(xs + d.ns * t) >> 1;
                P = qmul(P, lds_(B, 3, (p0 + t) & 1, cb));
            }
            acc[0] = DD{(double)P.a, 0.0};
        }
        dd_block_sum<1>(acc, lds);
        if (threadIdx.x == 0) {
            part[2 * tile + 0] = acc[0].hi;
            part[2 * tile + 1] = acc[0].lo;
        }
    });
}

// Final per-lattice reduction of the standalone measurements' tile
// partials in a fixed order.  Workgroup b handles chunk b % C of lattice
// b / C: it sums its share of the lattice's partials, writes a (hi, lo) pair
// per quantity to `chunk`, and the last chunk of the lattice to arrive
// (ticket in cnt[l]) combines the C pairs in chunk order and writes the
// plaquette (avg, spatial, temporal) and / or the Polyakov loop.
__device__ __forceinline__ void chunk_range(int n, int C, int c, int &lo, int &hi) {
    lo = (int)(((long long)n * c) / C);
    hi = (int)(((long long)n * (c + 1)) / C);
}

__global__ __launch_bounds__(256) void k_finalize(const LatDesc *desc, const double *pp, const double *pl,
                                                  unsigned *cnt, double *chunk, int C, double *outp, double *outl,
                                                  long long ostride) {
    __shared__ DD lds[3 * 4];
    __shared__ int last;
    last = 1;
    const int l = blockIdx.x / C, c = blockIdx.x % C;
    const LatDesc d = load_desc(desc + l);
    // four independent compensated accumulators per quantity (the sums are
    // latency bound), combined in a fixed order
    DD a4[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 3; ++k) a4[u][k] = DD{0.0, 0.0};
    if (pp) {
        int lo, hi;
        chunk_range(d.ntile, C, c, lo, hi);
        for (int t0 = lo + (int)threadIdx.x; t0 < hi; t0 += 4 * blockDim.x) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u * (int)blockDim.x;
                if (t < hi) {
                    const double4 q = reinterpret_cast<const double4 *>(pp)[d.tile0 + (long long)t];
                    a4[u][0] = dd_add(a4[u][0], DD{q.x, q.y});
                    a4[u][1] = dd_add(a4[u][1], DD{q.z, q.w});
                }
            }
        }
    }
    if (pl) {
        int lo, hi;
        chunk_range(d.nstile, C, c, lo, hi);
        for (int t0 = lo + (int)threadIdx.x; t0 < hi; t0 += 4 * blockDim.x) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u * (int)blockDim.x;
                if (t < hi) {
                    const double2 q = reinterpret_cast<const double2 *>(pl)[d.stile0 + (long long)t];
                    a4[u][2] = dd_add(a4[u][2], DD{q.x, q.y});
                }
            }
        }
    }
    DD acc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k] = dd_add(dd_add(a4[0][k], a4[1][k]), dd_add(a4[2][k], a4[3][k]));
    dd_block_sum<3>(acc, lds);
    if (C > 1) {  // chunk sums meet in the last chunk of the lattice to arrive
        if (threadIdx.x == 0) {
            double *ch = chunk + 6 * (long long)blockIdx.x;
            for (int k = 0; k < 3; ++k) {
                ch[2 * k] = acc[k].hi;
                ch[2 * k + 1] = acc[k].lo;
            }
            __threadfence();
            last = atomicAdd(&cnt[l], 1u) == (unsigned)(C - 1);
        }
        __syncthreads();
        if (!last) return;
    }
    if (threadIdx.x == 0) {
        DD tot[3] = {acc[0], acc[1], acc[2]};
        if (C > 1) {
            __threadfence();
            const volatile double *ch = chunk + 6 * (long long)l * C;
            for (int k = 0; k < 3; ++k) tot[k] = DD{0.0, 0.0};
            for (int cc = 0; cc < C; ++cc)
                for (int k = 0; k < 3; ++k)
                    tot[k] = dd_add(tot[k], DD{ch[6 * cc + 2 * k], ch[6 * cc + 2 * k + 1]});
            cnt[l] = 0u;
        }
        const double V = 2.0 * (double)d.vh;
        const double sp = tot[0].hi + tot[0].lo, tp = tot[1].hi + tot[1].lo;
        if (pp) {
            double *o = outp + l * ostride;
            o[0] = (sp + tp) / (6.0 * V);
            o[1] = sp / (3.0 * V);
            o[2] = tp / (3.0 * V);
        }
        if (pl) outl[l * ostride] = (tot[2].hi + tot[2].lo) / (double)d.ns;
    }
}

// Series values of a batch of measured sweeps, in two fixed-order passes.
// k_series_part: workgroup (l C + c, j) sums chunk c of C of lattice l's
// partials of slot (slot0 + j) % nslots -- the heat-bath plaquette partials
// [tile][plane slot 0, 1 spatial, 2 temporal][wavefront] and the Polyakov
// (hi, lo) pairs -- into three (hi, lo) pairs (spatial planes, temporal
// planes, Polyakov).  k_series_final: workgroup (l, j) adds the C chunk pairs
// in chunk order and writes the mean plaquette and Polyakov loop of sweep
// out0 + j.  Many workgroups per sweep keep the partial reads (0.8 MB per
// sweep at 32^4) off a single compute unit.
__global__ __launch_bounds__(256) void k_series_part(const LatDesc *desc, const double *pp, long long pp_stride,
                                                     const double *pl, long long pl_stride, int slot0, int nslots,
                                                     int Cn, double *chunk) {
    __shared__ DD lds[3 * 4];
    // x: lattice-major (lattice, chunk) pairs (lattice counts beyond the
    // y / z grid limits fit in x); y: measured sweep of the batch
    const int C = Cn, c = blockIdx.x % Cn, l = blockIdx.x / Cn, j = blockIdx.y, nsw = gridDim.y;
    const long long slot = (slot0 + j) % nslots;
    const LatDesc d = load_desc(desc + l);
    DD a4[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 3; ++k) a4[u][k] = DD{0.0, 0.0};
    if (pp) {
        int lo, hi;
        chunk_range(d.nmtile, C, c, lo, hi);
        const double4 *q4 = reinterpret_cast<const double4 *>(pp + slot * pp_stride) + 3 * (long long)d.mtile0;
        for (int t0 = lo + (int)threadIdx.x; t0 < hi; t0 += 4 * blockDim.x) {
            double4 v[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u * (int)blockDim.x;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    v[u][k] = t < hi ? q4[3 * (long long)t + k] : make_double4(0.0, 0.0, 0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    DD &x = a4[u][k == 2 ? 1 : 0];
                    x = dd_add(x, DD{(v[u][k].x + v[u][k].y), 0.0});
                    x = dd_add(x, DD{(v[u][k].z + v[u][k].w), 0.0});
                }
        }
    }
    if (pl) {
        int lo, hi;
        chunk_range(d.nstile, C, c, lo, hi);
        const double2 *q2 = reinterpret_cast<const double2 *>(pl + slot * pl_stride) + d.stile0;
        for (int t0 = lo + (int)threadIdx.x; t0 < hi; t0 += 4 * blockDim.x) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u * (int)blockDim.x;
                if (t < hi) a4[u][2] = dd_add(a4[u][2], DD{q2[t].x, q2[t].y});
            }
        }
    }
    DD acc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k] = dd_add(dd_add(a4[0][k], a4[1][k]), dd_add(a4[2][k], a4[3][k]));
    dd_block_sum<3>(acc, lds);
    if (threadIdx.x == 0) {
        double *o = chunk + 6 * (((long long)l * nsw + j) * C + c);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            o[2 * k] = acc[k].hi;
            o[2 * k + 1] = acc[k].lo;
        }
    }
}

__global__ __launch_bounds__(64) void k_series_final(const LatDesc *desc, const double *chunk, int C, bool plaq,
                                                     bool poly, double *outp, double *outl, long long ostride,
                                                     int out0) {
    const int l = blockIdx.x, j = blockIdx.y, nsw = gridDim.y;
    if (threadIdx.x != 0) return;
    const double *ch = chunk + 6 * ((long long)l * nsw + j) * C;
    DD tot[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int c = 0; c < C; ++c)
        for (int k = 0; k < 3; ++k) tot[k] = dd_add(tot[k], DD{ch[6 * c + 2 * k], ch[6 * c + 2 * k + 1]});
    const LatDesc d = load_desc(desc + l);
    const long long o = l * ostride + out0 + j;
    if (plaq) outp[o] = ((tot[0].hi + tot[0].lo) + (tot[1].hi + tot[1].lo)) / (12.0 * (double)d.vh);
    if (poly) outl[o] = (tot[2].hi + tot[2].lo) / (double)d.ns;
}

// Device state words set from the host values without a host copy.
__global__ void k_set_state(DevState *st, unsigned long long seed, unsigned sweep, unsigned run_base) {
    st->seed = seed;
    st->sweep = sweep;
    st->next = sweep;
    st->run_base = run_base;
}

// The same from the run state the host wrote into mapped host memory before
// launching a captured run (words: seed low, seed high, sweep, run base), so
// that the run's first node needs no kernel arguments of its own.
// Run state from mapped host memory: src[0] the seed, src[1] the sweep word
// (low half) and the run base (high half).  Two relaxed system-scope loads
// are in flight together, one round trip to host memory (four dependent
// volatile reads took four, ~8 us).
__global__ void k_set_state_mapped(DevState *st, const unsigned long long *src) {
    const unsigned long long seed = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const unsigned long long sr = __hip_atomic_load(src + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    st->seed = seed;
    st->sweep = (unsigned)sr;
    st->next = (unsigned)sr;
    st->run_base = (unsigned)(sr >> 32);
}

__global__ void k_clear_err(DevState *st) { st->err = 0u; }

__global__ void k_err_to_host(const DevState *st, unsigned *out) { *out = st->err; }

// ---------------------------------------------------------------------------
// APE smearing step (paper Sec. 2, APE equation) of the spatial links, all
// at once from the previous step: U' = normalise[(1-alpha) U + (alpha/4)
// sum over the two other spatial nu of the forward staple
// U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag and the backward staple
// U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)] with a binary64 norm.
// src_raw: read the lattice links (first step) or the smeared buffer.
// Work item v = 2 tile + parity: the two parities of a tile are neighbours
// in the walk, so an XCD updates both halves of its share of the lattice
// while the links they share are in its L2 (with the parities in separate
// passes every link was fetched twice).  A lane updates the three spatial
// links of its site.

// APE step of the three spatial links of one site (paper Sec. 2, APE
// equation).  Their twelve staples touch 24 distinct links: the three own
// links O[m] = U_m(x) and the backward links K[n] = U_n(x-n), used by every
// plane, and per spatial plane {m, n} (m < n) six links used by it alone,
// each loaded once: F_mn = U_m(x+n), F_nm = U_n(x+m), M_mn = U_m(x-n),
// M_nm = U_n(x-m), D_nm = U_n(x+m-n), D_mn = U_m(x+n-m).  Plane {m, n} adds
// to the sum of direction m its forward staple U_n(x) U_m(x+n) U_n(x+m)^dag
// and its backward staple U_n(x-n)^dag U_m(x-n) U_n(x-n+m), and the same
// with m and n exchanged to the sum of direction n.  The planes run {0,1},
// {0,2}, {1,2}, so every direction accumulates its two other directions in
// ascending order, forward then backward.  Then U' = normalise[(1-alpha) U
// + (alpha/4) sum], the norm in binary64: the hardware 1/sqrt estimate and
// two Newton steps (each squares the relative error; after the second it is
// below binary64 rounding).  A smeared sum is in general far from unit
// norm, so there is no near-group shortcut.
template <class T>
__device__ __forceinline__ void ape_site(const LatDesc &d, const Blocks<T, 3> &Bs, const Blocks<T, 3> &Bd, int cb,
                                         int par, T alpha) {
    const Site S = site_of(d, cb, par);
    const int op = par ^ 1;
    int f[3], b[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        f[m] = step_fwd(d, S, m);
        b[m] = step_bwd(d, S, m);
    }
    Q<T> O[3], K[3], sum[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        O[m] = lds_(Bs, m, par, (uint32_t)cb);
        K[m] = lds_(Bs, m, op, (uint32_t)(S.s + b[m]) >> 1);
        sum[m] = Q<T>{T(0), T(0), T(0), T(0)};
    }
#pragma unroll
    for (int pl = 0; pl < 3; ++pl) {
        const int m = pl == 2 ? 1 : 0, n = pl == 0 ? 1 : 2;
        const Q<T> Fmn = lds_(Bs, m, op, (uint32_t)(S.s + f[n]) >> 1);
        const Q<T> Fnm = lds_(Bs, n, op, (uint32_t)(S.s + f[m]) >> 1);
        const Q<T> Mmn = lds_(Bs, m, op, (uint32_t)(S.s + b[n]) >> 1);
        const Q<T> Mnm = lds_(Bs, n, op, (uint32_t)(S.s + b[m]) >> 1);
        const Q<T> Dnm = lds_(Bs, n, par, (uint32_t)(S.s + f[m] + b[n]) >> 1);
        const Q<T> Dmn = lds_(Bs, m, par, (uint32_t)(S.s + f[n] + b[m]) >> 1);
        qmul_acc(sum[m], qmul(O[n], Fmn), qdag(Fnm));
        qmul_acc(sum[m], qmul(qdag(K[n]), Mmn), Dnm);
        qmul_acc(sum[n], qmul(O[m], Fnm), qdag(Fmn));
        qmul_acc(sum[n], qmul(qdag(K[m]), Mnm), Dmn);
    }
    const T w0 = T(1) - alpha, w1 = T(0.25) * alpha;
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
        const Q<T> &u = O[mu], &sm = sum[mu];
        const Q<T> w{w0 * u.a + w1 * sm.a, w0 * u.b + w1 * sm.b, w0 * u.c + w1 * sm.c, w0 * u.d + w1 * sm.d};
        const double wa = w.a, wb = w.b, wc = w.c, wd = w.d;
        const double n2 = wa * wa + wb * wb + wc * wc + wd * wd;
        Q<T> un = u;
        if (n2 > 0.0) {
            double y = __builtin_amdgcn_rsq(n2);
            const double h = 0.5 * n2;
            y = y * (1.5 - h * y * y);
            y = y * (1.5 - h * y * y);
            un = Q<T>{(T)(wa * y), (T)(wb * y), (T)(wc * y), (T)(wd * y)};
        }
        sts_(Bd, mu, par, (uint32_t)cb, un);
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_ape(KArgs a, const void *src, int src_raw, void *dst, T alpha) {
    for_each_tile(2 * a.ntiles, a.xcd_remap, [&](int v) {
        const Tile tl = load_tile(a.tiles, v >> 1);
        const int par = v & 1;
        const LatDesc d = load_desc(a.desc + tl.x);
        const Blocks<T, 3> Bs = blocks<T, 3>(src, src_raw ? d.off : d.soff, d.vh);
        const Blocks<T, 3> Bd = blocks<T, 3>(dst, d.soff, d.vh);
        const int cb = tl.y + (int)threadIdx.x;
        if (cb >= d.vh) return;
        ape_site<T>(d, Bs, Bd, cb, par, alpha);
    });
}

// ---------------------------------------------------------------------------
// Wilson loops (paper Sec. 2, W(R,T)).  Spatial lines first: S_mu(x;R) =
// U_mu(x) .. U_mu(x+(R-1)mu), stored per site as Q<T> arrays
// sl[(mu*Rmax + R-1)*V + s].  `sp` / `sp_raw`: the spatial links (smeared
// buffer or raw links).  Temporal lines are not stored: the trace kernel
// builds them by transport from the raw temporal links.
template <class T>
__global__ __launch_bounds__(256) void k_wlines(KArgs a, const void *sp, int sp_raw, int Rmax, Q<T> *sl) {
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tv = load_tile(a.tiles, tile);
        const LatDesc d = load_desc(a.desc + tv.x);
        const Blocks<T, 3> Bs = blocks<T, 3>(sp, sp_raw ? d.off : d.soff, d.vh);
        const int s = tv.y + (int)threadIdx.x;
        const long long V = 2LL * d.vh;
        if (s >= V) return;
        int c[4], r = s;
        udiv(r, d.n[0], d.inv_nx, r, c[0]);
        udiv(r, d.n[1], d.inv_ny, r, c[1]);
        udiv(r, d.n[2], d.inv_nz, c[3], c[2]);
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            const int st = mu == 0 ? 1 : mu == 1 ? d.n[0] : d.n[0] * d.n[1];
            Q<T> P = qone<T>();
            int cm = c[mu];
            for (int R = 1; R <= Rmax; ++R) {
                const int y = s + (cm - c[mu]) * st;
                const int par = (c[0] + c[1] + c[2] + c[3] - c[mu] + cm) & 1;
                P = qmul(P, lds_(Bs, mu, par, (uint32_t)y >> 1));
                sl[((long long)mu * Rmax + R - 1) * V + s] = P;
                cm = (cm + 1 == d.n[mu]) ? 0 : cm + 1;
            }
        }
    });
}

// W(R,T) partials: blockIdx.y = R-1; per site x and spatial mu the loop
// 1/2 Tr[S(x;R) T(x+R mu;T) S(x+T t;R)^dag T(x;T)^dag] = 1/2 Tr[A_T S(x+T t;R)^dag]
// with A_T = T(x;T)^dag S(x;R) T(x+R mu;T), built by transport up the two
// temporal sides: A_0 = S(x;R), A_T = U_t(x+(T-1)t)^dag A_{T-1} U_t(x+R mu+(T-1)t).
// Temporal links come from the raw link buffer, the spatial lines from sl.
//
// A lane owns a column of NC sites x_j = x_0 + j t (j < NC; NC divides Nt)
// of lattice 0 and takes the three directions mu one after another: at
// temporal offset m from x_0 every column site with step k = m - j < Tmax
// applies the same two temporal links and meets the same spatial line at
// x_0 + (m+1) t, so each is loaded once per column instead of once per site
// (NC + Tmax - 1 offsets of three loads per mu).  Column q = (spatial site
// q % Ns, t block q / Ns); column tile i is columns [i B, (i+1) B) for block
// size B.  A workgroup walks its share of the column tiles (a fixed
// assignment), each lane summing in binary64, then one compensated block sum
// per (R, workgroup, T).
template <class T, int TMAX, int NC>
__device__ __forceinline__ void wtrace_body(const KArgs &a, int Rmax, int Tmax, int ncols, int nctiles,
                                            const Q<T> *sl, double *part) {
    __shared__ DD lds[TMAX * 4];
    const int R = blockIdx.y + 1;
    double sum[TMAX];
#pragma unroll
    for (int k = 0; k < TMAX; ++k) sum[k] = 0.0;
    const LatDesc d = load_desc(a.desc);
    const Blocks<T, 4> B = blocks<T, 4>(a.links, d.off, d.vh);
    const long long V = 2LL * d.vh;
    const Q<T> *slR = sl + (long long)(R - 1) * V;
    const long long mstride = (long long)Rmax * V;
    for (TileWalk w(nctiles, a.xcd_remap); w.ok(); w.next()) {
        const int q = w.tile() * (int)blockDim.x + (int)threadIdx.x;
        if (q >= ncols) continue;
        // q = sp + Ns tb: spatial site sp = x + Nx (y + Ny z), t0 = NC tb
        int c[3], r, tb, sp;
        udiv(q, d.n[0], d.inv_nx, r, c[0]);
        udiv(r, d.n[1], d.inv_ny, r, c[1]);
        udiv(r, d.n[2], d.inv_nz, tb, c[2]);
        sp = q - tb * d.ns;
        const int t0 = NC * tb;
        const int s0 = sp + t0 * d.ns;  // site of x_0
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            const int st = mu == 0 ? 1 : mu == 1 ? d.n[0] : d.n[0] * d.n[1];
            int cm = c[mu] + R;
            if (cm >= d.n[mu]) cm -= d.n[mu];
            const int sR = s0 + (cm - c[mu]) * st;  // x_0 + R mu
            Q<T> A[NC];
#pragma unroll
            for (int j = 0; j < NC; ++j) A[j] = slR[mu * mstride + s0 + j * d.ns];
            // parity of x_0 + m t and of x_0 + R mu + m t (R flips it when odd)
            const int p0 = (c[0] + c[1] + c[2] + t0) & 1, pR = p0 ^ (R & 1);
            int tm = t0;  // t of x_0 + m t
#pragma unroll
            for (int m = 0; m < NC + TMAX - 1; ++m) {
                if (m < NC + Tmax - 1) {
                    const int dt = (tm - t0) * d.ns;  // x_0 + m t = s0 + dt
                    const int pm = (p0 + m) & 1, pRm = (pR + m) & 1;
                    const Q<T> ua = qdag(lds_(B, 3, pm, (uint32_t)(s0 + dt) >> 1));
                    const Q<T> ub = lds_(B, 3, pRm, (uint32_t)(sR + dt) >> 1);
                    tm = (tm + 1 == d.n[3]) ? 0 : tm + 1;
                    const Q<T> top = slR[mu * mstride + s0 + (tm - t0) * d.ns];  // S(x_0 + (m+1) t; R)
#pragma unroll
                    for (int j = 0; j < NC; ++j) {
                        const int k = m - j;
                        if (k >= 0 && k < TMAX && k < Tmax) {
                            A[j] = qmul(qmul(ua, A[j]), ub);
                            sum[k] += (double)half_tr_xyd(A[j], top);
                        }
                    }
                }
            }
        }
    }
    // Wavefront sums by binary64 butterflies in a fixed order (each lane holds
    // a plain binary64 sum; a compensated butterfly cost as much as a tenth of
    // the kernel's instructions), then the workgroup's wavefronts combined by
    // compensated sums in thread 0.
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6, nw = (int)blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < TMAX; ++k) {
        const double ws = wave_sum_f64(sum[k]);
        if (lane == 0) lds[wave * TMAX + k] = DD{ws, 0.0};
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < TMAX; ++k)
            if (k < Tmax) {
                DD acc = lds[k];
                for (int w = 1; w < nw; ++w) acc = dd_add(acc, lds[w * TMAX + k]);
                double *p = part + 2 * (((long long)(R - 1) * gridDim.x + blockIdx.x) * Tmax + k);
                p[0] = acc.hi;
                p[1] = acc.lo;
            }
}

// Binary32 traces are held to 128 registers (4 waves per SIMD): under that
// bound the compiler also schedules the unrolled offsets without copying the
// binary64 sums around their run-time bounds, 10% faster at 24^3 x 48 than
// the same code unbounded (122 registers, also 4 waves).  Binary64 traces
// need more registers and run unbounded (the bound would spill).
template <int TMAX, int NC>
__global__ __launch_bounds__(256, 4) void k_wtrace(KArgs a, int Rmax, int Tmax, int ncols, int nctiles,
                                                   const Q<float> *sl, double *part) {
    wtrace_body<float, TMAX, NC>(a, Rmax, Tmax, ncols, nctiles, sl, part);
}
template <int TMAX, int NC>
__global__ __launch_bounds__(256) void k_wtrace64(KArgs a, int Rmax, int Tmax, int ncols, int nctiles,
                                                  const Q<double> *sl, double *part) {
    wtrace_body<double, TMAX, NC>(a, Rmax, Tmax, ncols, nctiles, sl, part);
}

// One block per (R, T): fixed-order sum over the k_wtrace workgroups'
// partials (nparts per R) of lattice 0.
__global__ __launch_bounds__(256) void k_wfinal(const LatDesc *desc, int ntiles, int Tmax, const double *part,
                                                double *out) {
    __shared__ DD lds[4];
    const int R = blockIdx.x / Tmax + 1, k = blockIdx.x % Tmax;
    DD acc[1] = {{0.0, 0.0}};
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
        const double *p = part + 2 * (((long long)(R - 1) * ntiles + t) * Tmax + k);
        acc[0] = dd_add(acc[0], DD{p[0], p[1]});
    }
    dd_block_sum<1>(acc, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = (acc[0].hi + acc[0].lo) / (6.0 * (double)desc[0].vh);
}

// ---------------------------------------------------------------------------
// Launchers
static inline dim3 grid_of(const KArgs &a, int grid) {
    int g = grid > 0 ? grid : ((a.ntiles + 7) / 8) * 8;
    if (g < 8) g = 8;
    return dim3((unsigned)g);
}

// With timing events the launch itself stamps them with the kernel's own
// start and end (the dispatch's timestamps), so nothing is queued between
// the events and the kernel.
template <class K>
static void launch_ev(K kern, dim3 g, dim3 b, hipStream_t s, const Ev &ev, const KArgs &a, int par) {
    if (ev.a && ev.b) hipExtLaunchKernelGGL(kern, g, b, 0, s, ev.a, ev.b, 0, a, par);
    else hipLaunchKernelGGL(kern, g, b, 0, s, a, par);
}

template <class T, int MU, int NL>
static void launch_hb_nl(const KArgs &a, int par, int block, int grid, hipStream_t s, bool trace, bool plaq,
                         const Ev &ev) {
    const dim3 g = grid_of(a, grid), b(block);
    if (plaq) {
        if constexpr (MU >= 1) {
            if (trace) launch_ev(k_heatbath<T, MU, true, NL, true>, g, b, s, ev, a, par);
            else launch_ev(k_heatbath<T, MU, false, NL, true>, g, b, s, ev, a, par);
        }
    } else {
        if (trace) launch_ev(k_heatbath<T, MU, true, NL, false>, g, b, s, ev, a, par);
        else launch_ev(k_heatbath<T, MU, false, NL, false>, g, b, s, ev, a, par);
    }
}

template <class T, int MU>
static void launch_hb_mu(const KArgs &a, int par, int nl, int block, int grid, hipStream_t s, bool trace,
                         bool plaq, const Ev &ev) {
    switch (nl) {
    case 1: launch_hb_nl<T, MU, 1>(a, par, block, grid, s, trace, plaq, ev); break;
    case 2: launch_hb_nl<T, MU, 2>(a, par, block, grid, s, trace, plaq, ev); break;
    default: launch_hb_nl<T, MU, 4>(a, par, block, grid, s, trace, plaq, ev); break;
    }
}

template <class T>
static void launch_hb_t(const KArgs &a, int mu, int par, int nl, int block, int grid, hipStream_t s,
                        bool trace, bool plaq, const Ev &ev) {
    switch (mu) {
    case 0: launch_hb_mu<T, 0>(a, par, nl, block, grid, s, trace, false, ev); break;
    case 1: launch_hb_mu<T, 1>(a, par, nl, block, grid, s, trace, plaq, ev); break;
    case 2: launch_hb_mu<T, 2>(a, par, nl, block, grid, s, trace, plaq, ev); break;
    default: launch_hb_mu<T, 3>(a, par, nl, block, grid, s, trace, plaq, ev); break;
    }
}

void launch_heatbath(const KArgs &a, bool f32, int mu, int par, int nl, int block, int grid, hipStream_t s,
                     bool trace, bool plaq, const Ev &ev) {
    if (f32) launch_hb_t<float>(a, mu, par, nl, block, grid, s, trace, plaq, ev);
    else launch_hb_t<double>(a, mu, par, nl, block, grid, s, trace, plaq, ev);
}

template <class T, int NL> static int hb_occ(int block) {
    int best = 1 << 30;
    const void *k[4] = {(const void *)k_heatbath<T, 0, false, NL, false>, (const void *)k_heatbath<T, 1, false, NL, false>,
                        (const void *)k_heatbath<T, 2, false, NL, false>, (const void *)k_heatbath<T, 3, false, NL, false>};
    for (const void *f : k) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, block, 0) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        best = n < best ? n : best;
    }
    return best;
}

int heatbath_blocks_per_cu(bool f32, int nl, int block) {
    if (f32) return nl == 1 ? hb_occ<float, 1>(block) : nl == 2 ? hb_occ<float, 2>(block) : hb_occ<float, 4>(block);
    return nl == 1 ? hb_occ<double, 1>(block) : nl == 2 ? hb_occ<double, 2>(block) : hb_occ<double, 4>(block);
}

template <class T>
static void launch_or_t(const KArgs &a, int mu, int par, int block, int grid, hipStream_t s, const Ev &ev) {
    const dim3 g = grid_of(a, grid), b((unsigned)block);
    switch (mu) {
    case 0: launch_ev(k_overrelax<T, 0>, g, b, s, ev, a, par); break;
    case 1: launch_ev(k_overrelax<T, 1>, g, b, s, ev, a, par); break;
    case 2: launch_ev(k_overrelax<T, 2>, g, b, s, ev, a, par); break;
    default: launch_ev(k_overrelax<T, 3>, g, b, s, ev, a, par); break;
    }
}

void launch_overrelax(const KArgs &a, bool f32, int mu, int par, int block, int grid, hipStream_t s, const Ev &ev) {
    if (f32) launch_or_t<float>(a, mu, par, block, grid, s, ev);
    else launch_or_t<double>(a, mu, par, block, grid, s, ev);
}

void launch_init(const KArgs &a, bool f32, int hot, int block, int grid, hipStream_t s) {
    if (f32) hipLaunchKernelGGL((k_init<float>), grid_of(a, grid), dim3(block), 0, s, a, hot);
    else hipLaunchKernelGGL((k_init<double>), grid_of(a, grid), dim3(block), 0, s, a, hot);
}

void launch_from_canon(const KArgs &a, bool f32, const double *canon, int block, hipStream_t s) {
    if (f32) hipLaunchKernelGGL((k_from_canon<float>), grid_of(a, 0), dim3(block), 0, s, a, canon);
    else hipLaunchKernelGGL((k_from_canon<double>), grid_of(a, 0), dim3(block), 0, s, a, canon);
}

void launch_to_canon(const KArgs &a, bool f32, const void *src, int ndir, double *canon, int block,
                     hipStream_t s) {
    if (f32) hipLaunchKernelGGL((k_to_canon<float>), grid_of(a, 0), dim3(block), 0, s, a, src, ndir, canon);
    else hipLaunchKernelGGL((k_to_canon<double>), grid_of(a, 0), dim3(block), 0, s, a, src, ndir, canon);
}

void launch_unit_defect(const KArgs &a, bool f32, unsigned long long *out, int block, hipStream_t s) {
    if (f32) hipLaunchKernelGGL((k_unit_defect<float>), grid_of(a, 0), dim3(block), 0, s, a, out);
    else hipLaunchKernelGGL((k_unit_defect<double>), grid_of(a, 0), dim3(block), 0, s, a, out);
}

void launch_plaquette(const KArgs &a, bool f32, double *part, int block, int grid, hipStream_t s) {
    if (f32) hipLaunchKernelGGL((k_plaquette<float>), grid_of(a, grid), dim3(block), 0, s, a, part);
    else hipLaunchKernelGGL((k_plaquette<double>), grid_of(a, grid), dim3(block), 0, s, a, part);
}

void launch_polyakov(const KArgs &a, bool f32, double *part, int block, int grid, hipStream_t s) {
    if (f32) hipLaunchKernelGGL((k_polyakov<float>), grid_of(a, grid), dim3(block), 0, s, a, part);
    else hipLaunchKernelGGL((k_polyakov<double>), grid_of(a, grid), dim3(block), 0, s, a, part);
}

void launch_finalize(const LatDesc *desc, int nlat, int chunks, const double *pp, const double *pl,
                     unsigned *cnt, double *chunk, double *outp, double *outl, long long ostride, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)(nlat * chunks)), dim3(256), 0, s, desc, pp, pl, cnt, chunk,
                       chunks, outp, outl, ostride);
}

void launch_series(const LatDesc *desc, int nlat, const double *pp, long long pp_stride, const double *pl,
                   long long pl_stride, int slot0, int nslots, int nsw, int C, double *chunk, double *outp,
                   double *outl, long long ostride, int out0, hipStream_t s) {
    hipLaunchKernelGGL(k_series_part, dim3((unsigned)(C * nlat), (unsigned)nsw), dim3(256), 0, s, desc, pp,
                       pp_stride, pl, pl_stride, slot0, nslots, C, chunk);
    hipLaunchKernelGGL(k_series_final, dim3((unsigned)nlat, (unsigned)nsw), dim3(64), 0, s, desc, chunk, C,
                       pp != nullptr, pl != nullptr, outp, outl, ostride, out0);
}

void launch_set_state(DevState *st, unsigned long long seed, unsigned sweep, unsigned run_base, hipStream_t s) {
    hipLaunchKernelGGL(k_set_state, dim3(1), dim3(1), 0, s, st, seed, sweep, run_base);
}

void launch_set_state_mapped(DevState *st, const unsigned *src, hipStream_t s) {
    hipLaunchKernelGGL(k_set_state_mapped, dim3(1), dim3(1), 0, s, st, (const unsigned long long *)src);
}

void launch_clear_err(DevState *st, hipStream_t s) { hipLaunchKernelGGL(k_clear_err, dim3(1), dim3(1), 0, s, st); }

void launch_err_to_host(const DevState *st, unsigned *out, hipStream_t s) {
    hipLaunchKernelGGL(k_err_to_host, dim3(1), dim3(1), 0, s, st, out);
}


void launch_ape(const KArgs &a, bool f32, const void *src, int src_raw, void *dst, double alpha, int block,
                int grid, hipStream_t s) {
    KArgs w = a;
    w.ntiles = 2 * a.ntiles;  // work items (tile, parity)
    const dim3 g = grid_of(w, grid);
    if (f32) hipLaunchKernelGGL((k_ape<float>), g, dim3(block), 0, s, a, src, src_raw, dst, (float)alpha);
    else hipLaunchKernelGGL((k_ape<double>), g, dim3(block), 0, s, a, src, src_raw, dst, alpha);
}

void launch_wlines(const KArgs &a, bool f32, const void *sp, int sp_raw, int Rmax, void *sl, int block,
                   hipStream_t s) {
    if (f32)
        hipLaunchKernelGGL((k_wlines<float>), grid_of(a, 0), dim3(block), 0, s, a, sp, sp_raw, Rmax,
                           (Q<float> *)sl);
    else
        hipLaunchKernelGGL((k_wlines<double>), grid_of(a, 0), dim3(block), 0, s, a, sp, sp_raw, Rmax,
                           (Q<double> *)sl);
}

// Workgroups per R of the Wilson trace: enough to fill the chip a few times
// over, each taking several column tiles (a multiple of 8, one share per XCD).
int wtrace_groups(const KArgs &a) {
    const int g = ((a.ntiles + 7) / 8) * 8;
    return g < 1024 ? (g < 8 ? 8 : g) : 1024;
}

// Column height of the Wilson trace: in binary32 with up to 16 time steps,
// 6 or else 4 when it divides Nt (the same four waves per SIMD; 8 would
// spill registers); otherwise 2 (extents are even).
template <class T> static int wtrace_nc(int Nt, int Tmax) {
    if (sizeof(T) == 4 && Tmax <= 16) return Nt % 6 == 0 ? 6 : Nt % 4 == 0 ? 4 : 2;
    return 2;
}

template <class T, int NC>
static void launch_wtrace_nc(const KArgs &a, int Rmax, int Tmax, long long V, const void *sl, double *part,
                             int block, hipStream_t s) {
    const dim3 g(wtrace_groups(a), (unsigned)Rmax), b((unsigned)block);
    const int ncols = (int)(V / NC), nct = (ncols + block - 1) / block;
    const Q<T> *l = (const Q<T> *)sl;
    if constexpr (sizeof(T) == 4) {
        if (Tmax <= 4) hipLaunchKernelGGL((k_wtrace<4, NC>), g, b, 0, s, a, Rmax, Tmax, ncols, nct, l, part);
        else if (Tmax <= 8) hipLaunchKernelGGL((k_wtrace<8, NC>), g, b, 0, s, a, Rmax, Tmax, ncols, nct, l, part);
        else if (Tmax <= 16) hipLaunchKernelGGL((k_wtrace<16, NC>), g, b, 0, s, a, Rmax, Tmax, ncols, nct, l, part);
        else if constexpr (NC == 2) hipLaunchKernelGGL((k_wtrace<32, NC>), g, b, 0, s, a, Rmax, Tmax, ncols, nct, l, part);
    } else {
        if (Tmax <= 4) hipLaunchKernelGGL((k_wtrace64<4, NC>), g, b, 0, s, a, Rmax, Tmax, ncols, nct, l, part);
        else if (Tmax <= 8) hipLaunchKernelGGL((k_wtrace64<8, NC>), g, b, 0, s, a, Rmax, Tmax, ncols, nct, l, part);
        else if (Tmax <= 16) hipLaunchKernelGGL((k_wtrace64<16, NC>), g, b, 0, s, a, Rmax, Tmax, ncols, nct, l, part);
        else if constexpr (NC == 2) hipLaunchKernelGGL((k_wtrace64<32, NC>), g, b, 0, s, a, Rmax, Tmax, ncols, nct, l, part);
    }
}

template <class T>
static void launch_wtrace_t(const KArgs &a, int Rmax, int Tmax, long long V, int Nt, const void *sl, double *part,
                            int block, hipStream_t s) {
    const int nc = wtrace_nc<T>(Nt, Tmax);
    if constexpr (sizeof(T) == 4) {
        if (nc == 6) return launch_wtrace_nc<T, 6>(a, Rmax, Tmax, V, sl, part, block, s);
        if (nc == 4) return launch_wtrace_nc<T, 4>(a, Rmax, Tmax, V, sl, part, block, s);
    }
    launch_wtrace_nc<T, 2>(a, Rmax, Tmax, V, sl, part, block, s);
}

void launch_wtrace(const KArgs &a, bool f32, int Rmax, int Tmax, long long V, int Nt, const void *sl, double *part,
                   int block, hipStream_t s) {
    if (f32) launch_wtrace_t<float>(a, Rmax, Tmax, V, Nt, sl, part, block, s);
    else launch_wtrace_t<double>(a, Rmax, Tmax, V, Nt, sl, part, block, s);
}

void launch_wfinal(const LatDesc *desc, int nparts, int Rmax, int Tmax, const double *part, double *out,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_wfinal, dim3((unsigned)(Rmax * Tmax)), dim3(256), 0, s, desc, nparts, Tmax, part, out);
}

}  // namespace su2
