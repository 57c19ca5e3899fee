// su2_kernels.hip -- gfx950 kernels of the SU(2) library and their launchers.
//
// Method: Cardoso & Bicudo, "SU(2) Lattice Gauge Theory Simulations on Fermi
// GPUs" (arXiv:1010.4834); each kernel names the passage it implements.
// All kernels walk a (lattice, tile) list so one launch advances a whole
// batch of independent lattices; the per-lattice descriptor is read with
// scalar loads.  Nothing here is a dense contraction (at most 4x4 real
// products per quaternion), so the kernels are vector-ALU code bound by HBM
// traffic: coalesced float4 / float64x2 loads of the parity-split layout.
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
    S.s = x + d.n[0] * row;
    return S;
}

// Periodic forward / backward steps of the full-site index along mu.
__device__ __forceinline__ int stride_of(const LatDesc &d, int mu) {
    return mu == 0 ? 1 : mu == 1 ? d.n[0] : mu == 2 ? d.n[0] * d.n[1] : d.ns;
}
__device__ __forceinline__ int step_fwd(const LatDesc &d, const Site &S, int mu) {
    const int st = stride_of(d, mu);
    return S.c[mu] == d.n[mu] - 1 ? -(d.n[mu] - 1) * st : st;
}
__device__ __forceinline__ int step_bwd(const LatDesc &d, const Site &S, int mu) {
    const int st = stride_of(d, mu);
    return S.c[mu] == 0 ? (d.n[mu] - 1) * st : -st;
}

__device__ __forceinline__ long long blk(const LatDesc &d, int mu, int par) {
    return d.off + (long long)(2 * mu + par) * d.vh;
}

// Staple V of link (x, MU), x of parity `par` (paper Sec. 2: the six
// plaquettes containing the link; V is the adjoint of the sum of the
// transporters x -> x+mu of the over-relaxation equation, so that the link
// weight is exp(beta/2 Tr(U V))).  nu ascending, upper then lower:
//   upper U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag,
//   lower U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu).
// 18 link loads; 7 distinct per update once shared with neighbouring lanes.
template <class T, int MU>
__device__ __forceinline__ Q<T> staple(const LatDesc &d, const void *L, const Site &S, int par) {
    using IO = Links<T>;
    const int op = par ^ 1;
    const int s_mu = S.s + step_fwd(d, S, MU);
    Q<T> V{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU) continue;
        const int fn = step_fwd(d, S, nu), bn = step_bwd(d, S, nu);
        const Q<T> A = IO::ld(L, blk(d, nu, op), d.vh, s_mu >> 1);
        const Q<T> B = IO::ld(L, blk(d, MU, op), d.vh, (S.s + fn) >> 1);
        const Q<T> C = IO::ld(L, blk(d, nu, par), d.vh, S.s >> 1);
        const Q<T> D = IO::ld(L, blk(d, nu, par), d.vh, (s_mu + bn) >> 1);
        const Q<T> E = IO::ld(L, blk(d, MU, op), d.vh, (S.s + bn) >> 1);
        const Q<T> F = IO::ld(L, blk(d, nu, op), d.vh, (S.s + bn) >> 1);
        qacc(V, qmul(A, qdag(qmul(C, B))));
        qacc(V, qmul(qdag(qmul(E, D)), F));
    }
    return V;
}

// ---------------------------------------------------------------------------
// Heat-bath substep (paper Sec. 2 heat bath; Sec. 4 chessboard): every link
// (x, MU) with parity(x) = par is redrawn from exp(beta/2 Tr(U V)).
// delta = 1 - a0 from Kennedy-Pendleton (alpha >= 2) or Creutz (alpha < 2,
// or always with SU2_CREUTZ); one Philox call per try, counter (s, sweep,
// tag, try).  Direction from the call with try word 0xFFFFFFFF.  New link
// X W^dag with W = V/k, renormalised in binary64.
template <class T, int MU, bool TRACE>
__global__ __launch_bounds__(256) void k_heatbath(KArgs a, int par) {
    using M = Mth<T>;
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = a.tiles[tile];
        const LatDesc &d = a.desc[tl.x];
        const int cb = tl.y + (int)threadIdx.x;
        uint32_t tries = 0;
        if (cb < d.vh) {
            const Site S = site_of(d, cb, par);
            const Q<T> V = staple<T, MU>(d, a.links, S, par);
            const T k2 = V.a * V.a + V.b * V.b + V.c * V.c + V.d * V.d;
            const T beta = (sizeof(T) == 4) ? (T)d.betaf : (T)d.beta;
            T k, ik;
            if (sizeof(T) == 4) {
                ik = M::rsqrt_(k2);
                k = k2 > T(0) ? k2 * ik : T(0);
            } else {
                k = M::sqrt_(k2);
                ik = T(1) / k;
            }
            const T alpha = beta * k;
            const uint32_t c0 = (uint32_t)S.s, c1 = a.st->sweep, c2 = tag(d.lat_id, PURPOSE_HEATBATH, MU, par);
            const unsigned long long seed = a.st->seed;
            const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
            const bool creutz = (a.sampler == 1) || !(alpha >= T(2));
            const T cfac = creutz ? -M::expm1_(T(-2) * alpha) : T(0);
            const T hia = T(0.5) / alpha;
            const T ia = T(1) / alpha;
            T delta = T(0);
            bool done = false;
            for (uint32_t j = 0; j < MAX_TRIES; ++j) {
                const uint4 w = philox10(c0, c1, c2, j, k0, k1);
                bool acc;
                T dl;
                if (creutz) {
                    const T u1 = M::u(w.x), u2 = M::u(w.y);
                    dl = (alpha >= T(1e-20)) ? -M::log1p_(-(T(1) - u1) * cfac) * ia
                                             : T(2) * (T(1) - u1);
                    acc = u2 * u2 <= dl * (T(2) - dl);
                } else {
                    const T r1 = M::u(w.x), r2 = M::u(w.y), r3 = M::u(w.z), r4 = M::u(w.w);
                    const T cs = M::cos2pi(r2);
                    const T lam2 = -(M::ln(r1) + cs * cs * M::ln(r3)) * hia;
                    acc = r4 * r4 <= T(1) - lam2;
                    dl = T(2) * lam2;
                }
                if (acc) {
                    delta = dl;
                    tries = j + 1;
                    done = true;
                    break;
                }
            }
            if (!done) {
                atomicAdd(&a.st->err, 1u);
                delta = M::nan_();
                tries = MAX_TRIES;
            }
            const uint4 w = philox10(c0, c1, c2, 0xFFFFFFFFu, k0, k1);
            const T u1 = M::u(w.x), u2 = M::u(w.y);
            const T cth = T(1) - T(2) * u1;
            const T sth = T(2) * M::sqrt_(u1 * (T(1) - u1));
            const T ra = M::sqrt_(delta * (T(2) - delta));
            const T rs = ra * sth;
            const Q<T> X{T(1) - delta, rs * M::cos2pi(u2), rs * M::sin2pi(u2), ra * cth};
            Q<T> Wd;
            if (k2 > T(0)) Wd = Q<T>{V.a * ik, -V.b * ik, -V.c * ik, -V.d * ik};
            else Wd = qone<T>();
            const Q<T> Un = qnormalize(qmul(X, Wd));
            Links<T>::st(a.links, blk(d, MU, par), d.vh, cb, Un);
            if (TRACE)
                a.trace[d.toff + (long long)S.s * 4 + MU] = tries | ((uint32_t)creutz << 31);
        }
        // tries of this tile: one atomic per wavefront, spread over tiles
        uint32_t t = tries;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m, 64);
        if ((threadIdx.x & 63) == 0 && t) atomicAdd(&a.tries_part[tile], (unsigned long long)t);
    });
}

// Over-relaxation substep (paper Sec. 2, over-relaxation equation, in its
// action-preserving form U' = W^dag U^dag W^dag, W = V/k).
template <class T, int MU>
__global__ __launch_bounds__(256) void k_overrelax(KArgs a, int par) {
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = a.tiles[tile];
        const LatDesc &d = a.desc[tl.x];
        const int cb = tl.y + (int)threadIdx.x;
        if (cb >= d.vh) return;
        const Site S = site_of(d, cb, par);
        const Q<T> V = staple<T, MU>(d, a.links, S, par);
        const T k2 = V.a * V.a + V.b * V.b + V.c * V.c + V.d * V.d;
        if (!(k2 > T(0))) return;
        const T ik = T(1) / Mth<T>::sqrt_(k2);
        const Q<T> Wd{V.a * ik, -V.b * ik, -V.c * ik, -V.d * ik};
        const Q<T> U = Links<T>::ld(a.links, blk(d, MU, par), d.vh, cb);
        const Q<T> Un = qnormalize(qmul(qmul(Wd, qdag(U)), Wd));
        Links<T>::st(a.links, blk(d, MU, par), d.vh, cb, Un);
    });
}

// ---------------------------------------------------------------------------
// Initial configurations (paper Sec. 4: cold start U = 1; hot start a
// Haar-random element per link, Haar measure of Sec. 2): one Philox call
// (purpose 1, sweep 0, try 0) -> four Box-Muller normals in binary64 ->
// normalised, rounded to the link precision.
template <class T>
__global__ __launch_bounds__(256) void k_init(KArgs a, int hot) {
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = a.tiles[tile];
        const LatDesc &d = a.desc[tl.x];
        const int cb = tl.y + (int)threadIdx.x;
        if (cb >= d.vh) return;
        const unsigned long long seed = a.st->seed;
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
                Links<T>::st(a.links, blk(d, mu, par), d.vh, cb,
                             Q<T>{(T)z.a, (T)z.b, (T)z.c, (T)z.d});
            }
        }
    });
}

// Canonical float64 [s][mu][4] <-> native layout.
template <class T>
__global__ __launch_bounds__(256) void k_from_canon(KArgs a, const double *canon) {
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = a.tiles[tile];
        const LatDesc &d = a.desc[tl.x];
        const int cb = tl.y + (int)threadIdx.x;
        if (cb >= d.vh) return;
        const double *c = canon + 16 * (d.off / 4);
        for (int par = 0; par < 2; ++par) {
            const Site S = site_of(d, cb, par);
            for (int mu = 0; mu < 4; ++mu) {
                const double *u = c + ((long long)S.s * 4 + mu) * 4;
                Links<T>::st(a.links, blk(d, mu, par), d.vh, cb, Q<T>{(T)u[0], (T)u[1], (T)u[2], (T)u[3]});
            }
        }
    });
}

template <class T>
__global__ __launch_bounds__(256) void k_to_canon(KArgs a, const void *src, long long src_stride_dirs,
                                                   int ndir, double *canon) {
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = a.tiles[tile];
        const LatDesc &d = a.desc[tl.x];
        const int cb = tl.y + (int)threadIdx.x;
        if (cb >= d.vh) return;
        const long long base = ndir == 4 ? d.off : d.soff;
        double *c = canon + (long long)ndir * 4 * (base / ndir);
        (void)src_stride_dirs;
        for (int par = 0; par < 2; ++par) {
            const Site S = site_of(d, cb, par);
            for (int mu = 0; mu < ndir; ++mu) {
                const Q<T> q = Links<T>::ld(src, base + (long long)(2 * mu + par) * d.vh, d.vh, cb);
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
        const Tile tl = a.tiles[tile];
        const LatDesc &d = a.desc[tl.x];
        const int cb = tl.y + (int)threadIdx.x;
        double m = 0.0;
        if (cb < d.vh)
            for (int q = 0; q < 8; ++q) {
                const Q<T> u = Links<T>::ld(a.links, d.off + (long long)q * d.vh, d.vh, cb);
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
            unsigned long long bits = (m != m) ? 0x7FF8000000000000ull : __double_as_longlong(m);
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
    __shared__ DD lds[2 * 16];
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = a.tiles[tile];
        const LatDesc &d = a.desc[tl.x];
        const int cb = tl.y + (int)threadIdx.x;
        DD acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
        if (cb < d.vh) {
            double sp = 0.0, tp = 0.0;
            for (int par = 0; par < 2; ++par) {
                const Site S = site_of(d, cb, par);
                const int op = par ^ 1;
                Q<T> U[4];
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) U[mu] = Links<T>::ld(a.links, blk(d, mu, par), d.vh, cb);
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    const int smu = (S.s + step_fwd(d, S, mu)) >> 1;
#pragma unroll
                    for (int nu = mu + 1; nu < 4; ++nu) {
                        const int snu = (S.s + step_fwd(d, S, nu)) >> 1;
                        const Q<T> Unu_smu = Links<T>::ld(a.links, blk(d, nu, op), d.vh, smu);
                        const Q<T> Umu_snu = Links<T>::ld(a.links, blk(d, mu, op), d.vh, snu);
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
    __shared__ DD lds[16];
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = a.tiles[tile];
        const LatDesc &d = a.desc[tl.x];
        const int xs = tl.y + (int)threadIdx.x;
        DD acc[1] = {{0.0, 0.0}};
        if (xs < d.ns) {
            int row, x, z, y;
            udiv(xs, d.n[0], d.inv_nx, row, x);
            udiv(row, d.n[1], d.inv_ny, z, y);
            Q<T> P = qone<T>();
            for (int t = 0; t < d.n[3]; ++t) {
                const int s = xs + d.ns * t;
                const int par = (x + y + z + t) & 1;
                P = qmul(P, Links<T>::ld(a.links, blk(d, 3, par), d.vh, s >> 1));
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

// Final per-lattice reduction of tile partials in a fixed order.
// kind 0: plaquette (K = 2: spatial, temporal) -> (avg, spatial, temporal)
// kind 1: Polyakov (K = 1) -> value / N_sigma
// Output slot: out[l * ostride + idx * width], idx = sweep - run_base when
// `series`, else 0.
template <int K>
__global__ __launch_bounds__(256) void k_finalize(const LatDesc *desc, const double *part, int kind,
                                                  const DevState *st, int series, double *out,
                                                  long long ostride) {
    __shared__ DD lds[K * 4];
    const LatDesc &d = desc[blockIdx.x];
    const int t0 = kind == 0 ? d.tile0 : d.stile0;
    const int nt = kind == 0 ? d.ntile : d.nstile;
    DD acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = DD{0.0, 0.0};
    for (int t = threadIdx.x; t < nt; t += blockDim.x)
#pragma unroll
        for (int k = 0; k < K; ++k)
            acc[k] = dd_add(acc[k], DD{part[2 * K * (t0 + t) + 2 * k], part[2 * K * (t0 + t) + 2 * k + 1]});
    dd_block_sum<K>(acc, lds);
    if (threadIdx.x == 0) {
        const long long idx = series ? (long long)(st->sweep - st->run_base) : 0;
        const double V = 2.0 * (double)d.vh;
        if constexpr (K == 2) {
            const double sp = acc[0].hi + acc[0].lo, tp = acc[1].hi + acc[1].lo;
            double *o = out + blockIdx.x * ostride + idx * (series ? 1 : 3);
            o[0] = (sp + tp) / (6.0 * V);
            if (!series) {
                o[1] = sp / (3.0 * V);
                o[2] = tp / (3.0 * V);
            }
        } else {
            double *o = out + blockIdx.x * ostride + idx;
            o[0] = (acc[0].hi + acc[0].lo) / (double)d.ns;
        }
    }
}

__global__ void k_bump(DevState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st->sweep = st->sweep + 1u;
}

// ---------------------------------------------------------------------------
// APE smearing step (paper Sec. 2, APE equation) of the spatial links, all
// at once from the previous step: U' = normalise[(1-alpha) U + (alpha/4)
// sum over the two other spatial nu of the forward staple
// U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag and the backward staple
// U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)] with a binary64 norm.
// src_raw: read the lattice links (first step) or the smeared buffer.
template <class T>
__global__ __launch_bounds__(256) void k_ape(KArgs a, const void *src, int src_raw, void *dst, T alpha) {
    using IO = Links<T>;
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tl = a.tiles[tile];
        const LatDesc &d = a.desc[tl.x];
        const int cb = tl.y + (int)threadIdx.x;
        if (cb >= d.vh) return;
        const long long sb = src_raw ? d.off : d.soff;
        for (int par = 0; par < 2; ++par) {
            const Site S = site_of(d, cb, par);
            const int op = par ^ 1;
            for (int mu = 0; mu < 3; ++mu) {
                const int s_mu = S.s + step_fwd(d, S, mu);
                Q<T> sum{T(0), T(0), T(0), T(0)};
                for (int nu = 0; nu < 3; ++nu) {
                    if (nu == mu) continue;
                    const int fn = step_fwd(d, S, nu), bn = step_bwd(d, S, nu);
                    const Q<T> a1 = IO::ld(src, sb + (2 * nu + par) * (long long)d.vh, d.vh, S.s >> 1);
                    const Q<T> a2 = IO::ld(src, sb + (2 * mu + op) * (long long)d.vh, d.vh, (S.s + fn) >> 1);
                    const Q<T> a3 = IO::ld(src, sb + (2 * nu + op) * (long long)d.vh, d.vh, s_mu >> 1);
                    qacc(sum, qmul(qmul(a1, a2), qdag(a3)));
                    const Q<T> b1 = IO::ld(src, sb + (2 * nu + op) * (long long)d.vh, d.vh, (S.s + bn) >> 1);
                    const Q<T> b2 = IO::ld(src, sb + (2 * mu + op) * (long long)d.vh, d.vh, (S.s + bn) >> 1);
                    const Q<T> b3 = IO::ld(src, sb + (2 * nu + par) * (long long)d.vh, d.vh, (s_mu + bn) >> 1);
                    qacc(sum, qmul(qmul(qdag(b1), b2), b3));
                }
                const Q<T> u = IO::ld(src, sb + (2 * mu + par) * (long long)d.vh, d.vh, cb);
                const T w0 = T(1) - alpha, w1 = T(0.25) * alpha;
                const Q<T> w{w0 * u.a + w1 * sum.a, w0 * u.b + w1 * sum.b, w0 * u.c + w1 * sum.c,
                             w0 * u.d + w1 * sum.d};
                const double n2 = (double)w.a * w.a + (double)w.b * w.b + (double)w.c * w.c +
                                  (double)w.d * w.d;
                const Q<T> o = n2 > 0.0 ? qnormalize(w) : u;
                IO::st(dst, d.soff + (2 * mu + par) * (long long)d.vh, d.vh, cb, o);
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Wilson loops (paper Sec. 2, W(R,T)).  Lines first: temporal lines
// T(x;T) = U_4(x) .. U_4(x+(T-1)t) and spatial lines S_mu(x;R) =
// U_mu(x) .. U_mu(x+(R-1)mu), stored per site as Q<T> arrays
//   tl[(T-1)*V + s], sl[(mu*Rmax + R-1)*V + s].
// `sp` / `sp_raw`: the spatial links (smeared buffer or raw links).
template <class T>
__global__ __launch_bounds__(256) void k_wlines(KArgs a, const void *sp, int sp_raw, int Rmax,
                                                 int Tmax, Q<T> *tl, Q<T> *sl) {
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tv = a.tiles[tile];
        const LatDesc &d = a.desc[tv.x];
        const int s = tv.y + (int)threadIdx.x;
        const long long V = 2LL * d.vh;
        if (s >= V) return;
        int c[4], r = s;
        udiv(r, d.n[0], d.inv_nx, r, c[0]);
        udiv(r, d.n[1], d.inv_ny, r, c[1]);
        udiv(r, d.n[2], d.inv_nz, c[3], c[2]);
        {   // temporal lines
            Q<T> P = qone<T>();
            int t = c[3];
            for (int TT = 1; TT <= Tmax; ++TT) {
                const int y = s + (t - c[3]) * d.ns;
                const int par = (c[0] + c[1] + c[2] + t) & 1;
                P = qmul(P, Links<T>::ld(a.links, blk(d, 3, par), d.vh, y >> 1));
                tl[(long long)(TT - 1) * V + s] = P;
                t = (t + 1 == d.n[3]) ? 0 : t + 1;
            }
        }
        const long long sb = sp_raw ? d.off : d.soff;
        for (int mu = 0; mu < 3; ++mu) {
            const int st = mu == 0 ? 1 : mu == 1 ? d.n[0] : d.n[0] * d.n[1];
            Q<T> P = qone<T>();
            int cm = c[mu];
            for (int R = 1; R <= Rmax; ++R) {
                const int y = s + (cm - c[mu]) * st;
                const int par = (c[0] + c[1] + c[2] + c[3] - c[mu] + cm) & 1;
                P = qmul(P, Links<T>::ld(sp, sb + (2 * mu + par) * (long long)d.vh, d.vh, y >> 1));
                sl[((long long)mu * Rmax + R - 1) * V + s] = P;
                cm = (cm + 1 == d.n[mu]) ? 0 : cm + 1;
            }
        }
    });
}

// W(R,T) partials: blockIdx.y = R-1; per site and spatial mu,
// 1/2 Tr[S(x;R) T(x+R mu;T) S(x+T t;R)^dag T(x;T)^dag]
// = 1/2 Tr[(S(x;R) T(x+R mu;T)) (T(x;T) S(x+T t;R))^dag], summed over mu in
// binary64 per lane, then a compensated block sum per (R, tile, T).
template <class T, int TMAX>
__global__ __launch_bounds__(256) void k_wtrace(KArgs a, int Rmax, int Tmax, const Q<T> *tl,
                                                const Q<T> *sl, double *part) {
    __shared__ DD lds[TMAX * 4];
    const int R = blockIdx.y + 1;
    for_each_tile(a.ntiles, a.xcd_remap, [&](int tile) {
        const Tile tv = a.tiles[tile];
        const LatDesc &d = a.desc[tv.x];
        const int s = tv.y + (int)threadIdx.x;
        const long long V = 2LL * d.vh;
        DD acc[TMAX];
#pragma unroll
        for (int k = 0; k < TMAX; ++k) acc[k] = DD{0.0, 0.0};
        if (s < V) {
            int c[4], r = s;
            udiv(r, d.n[0], d.inv_nx, r, c[0]);
            udiv(r, d.n[1], d.inv_ny, r, c[1]);
            udiv(r, d.n[2], d.inv_nz, c[3], c[2]);
            int sR[3];
            Q<T> S0[3];
#pragma unroll
            for (int mu = 0; mu < 3; ++mu) {
                const int st = mu == 0 ? 1 : mu == 1 ? d.n[0] : d.n[0] * d.n[1];
                int cm = c[mu] + R;
                if (cm >= d.n[mu]) cm -= d.n[mu];
                sR[mu] = s + (cm - c[mu]) * st;
                S0[mu] = sl[((long long)mu * Rmax + R - 1) * V + s];
            }
#pragma unroll
            for (int k = 0; k < TMAX; ++k) {
                if (k < Tmax) {
                    const int TT = k + 1;
                    int ct = c[3] + TT;
                    while (ct >= d.n[3]) ct -= d.n[3];
                    const int sT = s + (ct - c[3]) * d.ns;
                    const Q<T> t0 = tl[(long long)k * V + s];
                    double v = 0.0;
#pragma unroll
                    for (int mu = 0; mu < 3; ++mu) {
                        const Q<T> t1 = tl[(long long)k * V + sR[mu]];
                        const Q<T> s2 = sl[((long long)mu * Rmax + R - 1) * V + sT];
                        v += (double)half_tr_xyd(qmul(S0[mu], t1), qmul(t0, s2));
                    }
                    acc[k] = DD{v, 0.0};
                }
            }
        }
        dd_block_sum<TMAX>(acc, lds);
        if (threadIdx.x == 0)
            for (int k = 0; k < Tmax; ++k) {
                double *p = part + 2 * (((long long)(R - 1) * a.ntiles + tile) * Tmax + k);
                p[0] = acc[k].hi;
                p[1] = acc[k].lo;
            }
    });
}

// One block per (R, T): fixed-order sum over the tiles of lattice 0.
__global__ __launch_bounds__(256) void k_wfinal(const LatDesc *desc, int ntiles, int Tmax,
                                                const double *part, double *out) {
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

template <class T, int MU>
static void launch_hb_mu(const KArgs &a, int par, int block, int grid, hipStream_t s, bool trace) {
    if (trace) hipLaunchKernelGGL((k_heatbath<T, MU, true>), grid_of(a, grid), dim3(block), 0, s, a, par);
    else hipLaunchKernelGGL((k_heatbath<T, MU, false>), grid_of(a, grid), dim3(block), 0, s, a, par);
}

template <class T>
static void launch_hb_t(const KArgs &a, int mu, int par, int block, int grid, hipStream_t s, bool trace) {
    switch (mu) {
    case 0: launch_hb_mu<T, 0>(a, par, block, grid, s, trace); break;
    case 1: launch_hb_mu<T, 1>(a, par, block, grid, s, trace); break;
    case 2: launch_hb_mu<T, 2>(a, par, block, grid, s, trace); break;
    default: launch_hb_mu<T, 3>(a, par, block, grid, s, trace); break;
    }
}

void launch_heatbath(const KArgs &a, bool f32, int mu, int par, int block, int grid, hipStream_t s,
                     bool trace) {
    if (f32) launch_hb_t<float>(a, mu, par, block, grid, s, trace);
    else launch_hb_t<double>(a, mu, par, block, grid, s, trace);
}

template <class T>
static void launch_or_t(const KArgs &a, int mu, int par, int block, int grid, hipStream_t s) {
    switch (mu) {
    case 0: hipLaunchKernelGGL((k_overrelax<T, 0>), grid_of(a, grid), dim3(block), 0, s, a, par); break;
    case 1: hipLaunchKernelGGL((k_overrelax<T, 1>), grid_of(a, grid), dim3(block), 0, s, a, par); break;
    case 2: hipLaunchKernelGGL((k_overrelax<T, 2>), grid_of(a, grid), dim3(block), 0, s, a, par); break;
    default: hipLaunchKernelGGL((k_overrelax<T, 3>), grid_of(a, grid), dim3(block), 0, s, a, par); break;
    }
}

void launch_overrelax(const KArgs &a, bool f32, int mu, int par, int block, int grid, hipStream_t s) {
    if (f32) launch_or_t<float>(a, mu, par, block, grid, s);
    else launch_or_t<double>(a, mu, par, block, grid, s);
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
    if (f32) hipLaunchKernelGGL((k_to_canon<float>), grid_of(a, 0), dim3(block), 0, s, a, src, 0LL, ndir, canon);
    else hipLaunchKernelGGL((k_to_canon<double>), grid_of(a, 0), dim3(block), 0, s, a, src, 0LL, ndir, canon);
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

void launch_finalize(const LatDesc *desc, int nlat, const double *part, int kind, const DevState *st,
                     int series, double *out, long long ostride, hipStream_t s) {
    if (kind == 0)
        hipLaunchKernelGGL((k_finalize<2>), dim3(nlat), dim3(256), 0, s, desc, part, kind, st, series, out, ostride);
    else
        hipLaunchKernelGGL((k_finalize<1>), dim3(nlat), dim3(256), 0, s, desc, part, kind, st, series, out, ostride);
}

void launch_bump(DevState *st, hipStream_t s) { hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, s, st); }

void launch_ape(const KArgs &a, bool f32, const void *src, int src_raw, void *dst, double alpha, int block,
                int grid, hipStream_t s) {
    if (f32) hipLaunchKernelGGL((k_ape<float>), grid_of(a, grid), dim3(block), 0, s, a, src, src_raw, dst, (float)alpha);
    else hipLaunchKernelGGL((k_ape<double>), grid_of(a, grid), dim3(block), 0, s, a, src, src_raw, dst, alpha);
}

void launch_wlines(const KArgs &a, bool f32, const void *sp, int sp_raw, int Rmax, int Tmax, void *tl,
                   void *sl, int block, hipStream_t s) {
    if (f32)
        hipLaunchKernelGGL((k_wlines<float>), grid_of(a, 0), dim3(block), 0, s, a, sp, sp_raw, Rmax, Tmax,
                           (Q<float> *)tl, (Q<float> *)sl);
    else
        hipLaunchKernelGGL((k_wlines<double>), grid_of(a, 0), dim3(block), 0, s, a, sp, sp_raw, Rmax, Tmax,
                           (Q<double> *)tl, (Q<double> *)sl);
}

template <class T>
static void launch_wtrace_t(const KArgs &a, int Rmax, int Tmax, const void *tl, const void *sl, double *part,
                            hipStream_t s) {
    dim3 g(grid_of(a, 0).x, (unsigned)Rmax);
    const Q<T> *t = (const Q<T> *)tl;
    const Q<T> *l = (const Q<T> *)sl;
    if (Tmax <= 4) hipLaunchKernelGGL((k_wtrace<T, 4>), g, dim3(256), 0, s, a, Rmax, Tmax, t, l, part);
    else if (Tmax <= 8) hipLaunchKernelGGL((k_wtrace<T, 8>), g, dim3(256), 0, s, a, Rmax, Tmax, t, l, part);
    else if (Tmax <= 16) hipLaunchKernelGGL((k_wtrace<T, 16>), g, dim3(256), 0, s, a, Rmax, Tmax, t, l, part);
    else hipLaunchKernelGGL((k_wtrace<T, 32>), g, dim3(256), 0, s, a, Rmax, Tmax, t, l, part);
}

void launch_wtrace(const KArgs &a, bool f32, int Rmax, int Tmax, const void *tl, const void *sl, double *part,
                   hipStream_t s) {
    if (f32) launch_wtrace_t<float>(a, Rmax, Tmax, tl, sl, part, s);
    else launch_wtrace_t<double>(a, Rmax, Tmax, tl, sl, part, s);
}

void launch_wfinal(const LatDesc *desc, int ntiles, int Rmax, int Tmax, const double *part, double *out,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_wfinal, dim3((unsigned)(Rmax * Tmax)), dim3(256), 0, s, desc, ntiles, Tmax, part, out);
}

}  // namespace su2
