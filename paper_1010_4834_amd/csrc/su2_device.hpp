// su2_device.hpp -- device-side building blocks of the gfx950 SU(2) library:
// lattice descriptors, SU(2) quaternion algebra, the Philox4x32-10 stream,
// per-precision math and compensated binary64 reductions.
//
// Method: Cardoso & Bicudo, "SU(2) Lattice Gauge Theory Simulations on Fermi
// GPUs" (arXiv:1010.4834).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace su2 {

// ---------------------------------------------------------------------------
// Lattice descriptor, one per lattice of a batch (read with scalar loads).
// Link storage of lattice l: links [off, off + 4V) ordered [mu][parity][cb],
// cb = s >> 1 with s = x + Nx*(y + Ny*(z + Nz*t)) (Nx even, so the sites of
// one parity in an x-row are contiguous).  A float link is one float4; a
// double link lives in two float64x2 planes: within the (mu, parity) block
// starting at link b, components (a0,a1) at double2 index 2b + cb and
// (a2,a3) at 2b + vh + cb.  Every wavefront load is one contiguous 1 KiB.
struct LatDesc {
    int n[4];        // extents Nx, Ny, Nz, Nt (even, >= 2)
    int hx;          // Nx / 2
    int vh;          // V / 2
    int ns;          // Nx * Ny * Nz
    int lat_id;      // lattice id in the Philox counter
    long long off;   // first link of this lattice in the link buffer
    long long soff;  // first link in the smeared-link buffers (3V links)
    long long toff;  // first entry of the per-link try record ([s][mu])
    double inv_hx, inv_ny, inv_nz, inv_nx;  // 1/d for the division helper
    double beta;
    float betaf;
    int tile0, ntile;    // range in the half-site tile table
    int stile0, nstile;  // range in the spatial-site tile table
    int vtile0, nvtile;  // range in the full-site tile table
    int mtile0, nmtile;  // range in the heat-bath (links-per-lane) tile table
};

// Mutable state read by the kernels; lives in device memory so that one
// captured graph serves every sweep.
// The sweep counter advances without a kernel of its own: within a sweep the
// first substep (mu = 0, even) reads `next` and publishes it as `sweep`, the
// other substeps read `sweep`, and the last (mu = 3, odd) writes
// `next = sweep + 1`.  Every workgroup writes the same value and no launch
// reads a word that it writes, so one captured sweep serves every sweep.
struct DevState {
    unsigned long long seed;
    unsigned int sweep;     // Philox sweep word of the sweep in progress
    unsigned int next;      // sweep word of the following sweep
    unsigned int run_base;  // sweep index of the first sweep of a series
    unsigned int err;       // non-finite staples and sampler try-cap hits
};

// A tile: lattice index and first index (half-site, spatial site or site).
typedef int2 Tile;

// Random-number purposes (third Philox counter word).
constexpr uint32_t PURPOSE_HEATBATH = 0;
constexpr uint32_t PURPOSE_HOT = 1;
constexpr uint32_t MAX_TRIES = 4096;  // never reached for finite links

__device__ __forceinline__ uint32_t tag(int lat_id, uint32_t purpose, int mu, int parity) {
    return ((uint32_t)lat_id << 8) | (purpose << 4) | ((uint32_t)mu << 1) | (uint32_t)parity;
}

// q = n / d, r = n % d for 0 <= n < 2^31, 0 < d < 2^24 and n / d < 2^24,
// with no correction step.  inv is 1/d rounded up to the next binary64
// (the host stores it so), at most (1 + 3 2^-53)/d.  The rounded product
// n inv is then at least n/d (rounding is monotone and n/d <= n inv) and
// exceeds it by less than 2^-27, below the distance 1/d > 2^-24 from a
// non-integer n/d to the next integer; truncating it gives floor(n/d).
// q d <= n < 2^31, so the 24-bit multiply is exact.  The extent checks at
// creation guarantee the bounds (every quotient is at most Ny Nz Nt < 2^24,
// every divisor at most Nx < 2^24).
__device__ __forceinline__ void udiv(int n, int d, double inv, int &q, int &r) {
    q = (int)((double)n * inv);
    r = n - (int)__umul24((unsigned)q, (unsigned)d);
}

// ---------------------------------------------------------------------------
// SU(2) as four reals, U = a0 + i a.sigma (paper Sec. 2).
template <class T> struct Q { T a, b, c, d; };

template <class T>
__device__ __forceinline__ Q<T> qmul(const Q<T> &x, const Q<T> &y) {
    // (x0 y0 - x.y,  x0 y + y0 x - x cross y), each component one chain of
    // a product and three fused multiply-adds
    Q<T> r;
    r.a = x.a * y.a - x.b * y.b - x.c * y.c - x.d * y.d;
    r.b = x.a * y.b + x.b * y.a - x.c * y.d + x.d * y.c;
    r.c = x.a * y.c + x.c * y.a - x.d * y.b + x.b * y.d;
    r.d = x.a * y.d + x.d * y.a - x.b * y.c + x.c * y.b;
    return r;
}
// s += x y (four fused multiply-adds per component)
template <class T>
__device__ __forceinline__ void qmul_acc(Q<T> &s, const Q<T> &x, const Q<T> &y) {
    s.a = s.a + x.a * y.a - x.b * y.b - x.c * y.c - x.d * y.d;
    s.b = s.b + x.a * y.b + x.b * y.a - x.c * y.d + x.d * y.c;
    s.c = s.c + x.a * y.c + x.c * y.a - x.d * y.b + x.b * y.d;
    s.d = s.d + x.a * y.d + x.d * y.a - x.b * y.c + x.c * y.b;
}
template <class T> __device__ __forceinline__ Q<T> qdag(const Q<T> &x) {
    return Q<T>{x.a, -x.b, -x.c, -x.d};
}
// 1/2 Re Tr(x y^dag) = x0 y0 + x.y
template <class T> __device__ __forceinline__ T half_tr_xyd(const Q<T> &x, const Q<T> &y) {
    return x.a * y.a + x.b * y.b + x.c * y.c + x.d * y.d;
}
template <class T> __device__ __forceinline__ Q<T> qone() { return Q<T>{T(1), T(0), T(0), T(0)}; }

// Scale to unit norm with the squared norm and the scale factor evaluated
// in binary64 (the reunitarisation that keeps binary32 links on the group).
// Updated links have |1 - n2| ~ 1e-7, where 1 - e/2 + 3e^2/8 (e = n2 - 1)
// equals 1/sqrt(n2) to O(e^3); farther from the group the exact form is used.
// The exact form sits behind a wavefront-uniform branch: as a plain per-lane
// branch it is if-converted, and every lane then pays for a binary64 square
// root and division whose result it discards.  The empty volatile asm (no
// instruction) keeps the compiler from speculating the rare block back onto
// the common path.
template <class T> __device__ __forceinline__ Q<T> qnormalize(const Q<T> &x) {
    const double a = x.a, b = x.b, c = x.c, d = x.d;
    const double n2 = a * a + b * b + c * c + d * d;
    const double e = n2 - 1.0;
    const bool near = fabs(e) < 1e-4;
    double f = 1.0 - e * (0.5 - 0.375 * e);
    if (__ballot(!near)) {
        double g = 1.0 / sqrt(n2);
        __asm__ volatile("" : "+v"(g));
        if (!near) f = g;
    }
    return Q<T>{(T)(a * f), (T)(b * f), (T)(c * f), (T)(d * f)};
}

// ---------------------------------------------------------------------------
// Link access through the uniform base `p` of one (lattice, mu, parity)
// block (scalar registers) plus a 32-bit per-lane byte offset, so each
// wavefront load is one global load with a scalar base and no 64-bit
// address math.  `hoff` (binary64 only) = 16 vh bytes, the distance from the
// (a0,a1) plane to the (a2,a3) plane of a block.
template <class T> struct Links;

template <> struct Links<float> {
    static constexpr int BYTES = 16;
    static __device__ __forceinline__ Q<float> ld(const char *p, uint32_t hoff, uint32_t cb) {
        (void)hoff;
        const float4 v = *reinterpret_cast<const float4 *>(p + (cb << 4));
        return Q<float>{v.x, v.y, v.z, v.w};
    }
    static __device__ __forceinline__ void st(char *p, uint32_t hoff, uint32_t cb, const Q<float> &q) {
        (void)hoff;
        *reinterpret_cast<float4 *>(p + (cb << 4)) = make_float4(q.a, q.b, q.c, q.d);
    }
};

template <> struct Links<double> {
    static constexpr int BYTES = 32;
    static __device__ __forceinline__ Q<double> ld(const char *p, uint32_t hoff, uint32_t cb) {
        const uint32_t o = cb << 4;
        const double2 l = *reinterpret_cast<const double2 *>(p + o);
        const double2 h = *reinterpret_cast<const double2 *>(p + (o + hoff));
        return Q<double>{l.x, l.y, h.x, h.y};
    }
    static __device__ __forceinline__ void st(char *p, uint32_t hoff, uint32_t cb, const Q<double> &q) {
        const uint32_t o = cb << 4;
        *reinterpret_cast<double2 *>(p + o) = make_double2(q.a, q.b);
        *reinterpret_cast<double2 *>(p + (o + hoff)) = make_double2(q.c, q.d);
    }
};

// ---------------------------------------------------------------------------
// a ^ b ^ c in one gfx950 three-input bit operation (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return (uint32_t)__builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products on counter words 0 and 2 with a Weyl-advanced key.
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return make_uint4(c0, c1, c2, c3);
}

// ---------------------------------------------------------------------------
// Per-precision math.  binary32 uses the hardware transcendental units
// (v_log_f32 is log2, v_sin/v_cos take revolutions); binary64 uses the
// correctly rounded library routines.
template <class T> struct Mth;

template <> struct Mth<float> {
    // (2m+1) 2^-24, m = the top 23 bits: exact, in (0,1).  Formed as
    // (1 + m 2^-23) - (1 - 2^-24), an exact (Sterbenz) difference.
    static __device__ __forceinline__ float u(uint32_t w) {
        return __uint_as_float((w >> 9) | 0x3F800000u) - 0x1.fffffep-1f;
    }
    static __device__ __forceinline__ float ln(float x) {
        return __builtin_amdgcn_logf(x) * 0.693147180559945309f;
    }
    // lg: the cheapest logarithm (log2 here); ln(x) = LN_LG * lg(x)
    static __device__ __forceinline__ float lg(float x) { return __builtin_amdgcn_logf(x); }
    static constexpr float LN_LG = 0.693147180559945309f;
    static __device__ __forceinline__ float cos2pi(float r) { return __builtin_amdgcn_cosf(r); }
    static __device__ __forceinline__ float sin2pi(float r) { return __builtin_amdgcn_sinf(r); }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float log1p_(float x) { return log1pf(x); }
    static __device__ __forceinline__ float expm1_(float x) { return expm1f(x); }
    static __device__ __forceinline__ float nan_() { return __builtin_nanf(""); }
    static constexpr float MAXV = __FLT_MAX__;  // largest finite value
};

template <> struct Mth<double> {
    // (2w+1) 2^-33 = w 2^-32 + 2^-33, exact
    static __device__ __forceinline__ double u(uint32_t w) { return fma((double)w, 0x1p-32, 0x1p-33); }
    static __device__ __forceinline__ double ln(double x) { return log(x); }
    static __device__ __forceinline__ double lg(double x) { return log(x); }
    static constexpr double LN_LG = 1.0;
    static __device__ __forceinline__ double cos2pi(double r) {
        return cos(6.283185307179586476925286766559 * r);
    }
    static __device__ __forceinline__ double sin2pi(double r) {
        return sin(6.283185307179586476925286766559 * r);
    }
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
    static __device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
    static __device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double log1p_(double x) { return log1p(x); }
    static __device__ __forceinline__ double expm1_(double x) { return expm1(x); }
    static __device__ __forceinline__ double nan_() { return __builtin_nan(""); }
    static constexpr double MAXV = __DBL_MAX__;
};

// ---------------------------------------------------------------------------
// Compensated binary64 sums: (hi, lo) pairs combined with two-sum, in a
// fixed order so that results are reproducible run to run.
struct DD { double hi, lo; };

__device__ __forceinline__ DD dd_add(DD a, DD b) {
    double s = a.hi + b.hi;
    double bb = s - a.hi;
    double e = (a.hi - (s - bb)) + (b.hi - bb);
    e += a.lo + b.lo;
    double h = s + e;
    return DD{h, e - (h - s)};
}

// Wavefront sums that need no lane-index registers: XOR butterflies within
// each 32-lane half by ds_swizzle in bit-mask mode (lane j reads lane j ^ X),
// then the two half sums read back as uniform values.  All 64 lanes must be
// active; every lane receives the total.
template <int X> __device__ __forceinline__ uint32_t swz_xor(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (X << 10));
}
template <int X> __device__ __forceinline__ double swz_xor(double v) {
    const unsigned long long b = __double_as_longlong(v);
    const uint32_t lo = swz_xor<X>((uint32_t)b), hi = swz_xor<X>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const unsigned long long b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += swz_xor<1>(v);
    v += swz_xor<2>(v);
    v += swz_xor<4>(v);
    v += swz_xor<8>(v);
    v += swz_xor<16>(v);
    return readlane_f64(v, 0) + readlane_f64(v, 32);
}

__device__ __forceinline__ DD dd_wave_sum(DD v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        DD o{__shfl_xor(v.hi, m, 64), __shfl_xor(v.lo, m, 64)};
        v = dd_add(v, o);
    }
    return v;
}

// Block-wide sum of K pairs per thread; thread 0 receives the totals.
// `lds` holds K * (blockDim.x / 64) pairs.  Every thread must call it.
template <int K>
__device__ __forceinline__ void dd_block_sum(DD (&v)[K], DD *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = dd_wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) lds[wave * K + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            DD t = lds[k];
            for (int w = 1; w < nw; ++w) t = dd_add(t, lds[w * K + k]);
            v[k] = t;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Values every lane of a wavefront agrees on, moved to scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned uni(unsigned v) {
    return (unsigned)__builtin_amdgcn_readfirstlane((int)v);
}

// Descriptor and tile tables are read-only while a kernel runs and are
// indexed uniformly, so they are read through the constant address space:
// scalar loads into scalar registers, no vector load and read-back.
template <class T> using cptr = const __attribute__((address_space(4))) T *;

// Descriptor of one lattice in scalar registers.
__device__ __forceinline__ LatDesc load_desc(const LatDesc *p) {
    static_assert(sizeof(LatDesc) % 4 == 0, "descriptor is a whole number of dwords");
    LatDesc d;
    const cptr<int> src = (cptr<int>)p;
    int *dst = reinterpret_cast<int *>(&d);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(LatDesc) / 4); ++i) dst[i] = uni(src[i]);
    return d;
}

__device__ __forceinline__ Tile load_tile(const Tile *t, int i) {
    const cptr<int> p = (cptr<int>)(t + i);
    return make_int2(uni(p[0]), uni(p[1]));
}

// ---------------------------------------------------------------------------
// Tile walk of a persistent grid.  With xcd_remap, workgroup b runs on XCD
// b % 8 (round-robin dispatch) and is given tiles from that XCD's
// contiguous eighth of the tile list, so neighbouring tiles (which share
// staple links) meet in the same L2.
struct TileWalk {
    int base, i, step, lim;
    __device__ __forceinline__ TileWalk(int ntiles, int xcd_remap) {
        const int G = gridDim.x, b = blockIdx.x;
        base = 0, i = b, step = G, lim = ntiles;
        if (xcd_remap && (G & 7) == 0) {
            const int tx = (ntiles + 7) >> 3;  // tiles per XCD
            base = (b & 7) * tx;
            i = b >> 3;
            step = G >> 3;
            lim = min(tx, ntiles - base);
        }
    }
    __device__ __forceinline__ bool ok() const { return i < lim; }
    __device__ __forceinline__ int tile() const { return base + i; }
    __device__ __forceinline__ bool next() {
        i += step;
        return i < lim;
    }
};

template <class F>
__device__ __forceinline__ void for_each_tile(int ntiles, int xcd_remap, F &&body) {
    for (TileWalk w(ntiles, xcd_remap); w.ok(); w.next()) body(w.tile());
}

}  // namespace su2
