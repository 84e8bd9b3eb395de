// croft_kernels.hip -- HIP kernels for gfx950: one axis pass of the 3D FFT.
//
// A pass runs batched 1D FFTs of length n along one axis of the grid (steps
// 1, 5 and 9 of the paper's algorithm, Section 4.1).  The paper's pack,
// all-to-all and unpack steps between them (steps 2-4, 6-8) are the layout
// change that makes the next axis contiguous; on one GPU no data is moved for
// it: a strided pass reads a tile of `L` neighbouring lines of the next axis
// directly (each row of the tile is one contiguous L-element segment), runs
// the FFT through LDS, and writes the results back in place, so the grid stays
// in its natural layout and the closing transposes of Section 4.2 are free.
//
// Inside a block the 1D FFT is a Stockham autosort FFT (mixed radix 2, 3, 4,
// 5, 8, 16): stage s with radix R, span Ns (the product of the earlier
// radices) and k = j mod Ns maps
//     v[q] = a[j + q N/R] * w_{Ns R}^{q k}       q = 0 .. R-1
//     V    = DFT_R(v)
//     b[(j / Ns) Ns R + k + q Ns] = V[q]
// for every butterfly j < N/R.  The first stage reads global memory and the
// last writes it (both with consecutive j on consecutive threads); the stages
// between exchange through LDS.  Twiddles come from a per-length table of
// w_N^m = exp(-2 pi i m / N) computed on the host in FP64.  The inverse
// direction conjugates on load and on store.
//
// Half storage: a line is loaded as FP16/BF16 pairs scaled by 2^e of the line
// that stored each element, computed in FP32, and stored with one new
// exponent per line chosen from the line's largest |re|, |im|.

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "croft_internal.h"

namespace croft {
namespace {

// ------------------------------------------------------------------ complex
template <typename R>
struct cx {
    R x, y;
};
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cx<R> scale(cx<R> a, R s) { return {a.x * s, a.y * s}; }
// a * (-i)
template <typename R>
__device__ __forceinline__ cx<R> mul_mi(cx<R> a) { return {a.y, -a.x}; }

template <typename R>
struct Kc {
    static constexpr R rs2 = R(0.70710678118654752440);   // cos(pi/4)
    static constexpr R c8 = R(0.92387953251128675613);    // cos(pi/8)
    static constexpr R s8 = R(0.38268343236508977173);    // sin(pi/8)
    static constexpr R s3 = R(0.86602540378443864676);    // sin(pi/3)
    static constexpr R c51 = R(0.30901699437494742410);   // cos(2pi/5)
    static constexpr R c52 = R(-0.80901699437494742410);  // cos(4pi/5)
    static constexpr R s51 = R(0.95105651629515357212);   // sin(2pi/5)
    static constexpr R s52 = R(0.58778525229247312917);   // sin(4pi/5)
};

// ------------------------------------------------- forward DFT codelets
// In place on v[0..R-1]: V[k] = sum_j v[j] exp(-2 pi i j k / R).
template <typename R>
__device__ __forceinline__ void dft4(cx<R> &a0, cx<R> &a1, cx<R> &a2, cx<R> &a3) {
    const cx<R> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_mi(a1 - a3);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
}

template <int RAD, typename R>
struct Dft;

template <typename R>
struct Dft<2, R> {
    static __device__ __forceinline__ void run(cx<R> *v) {
        const cx<R> a = v[0];
        v[0] = a + v[1];
        v[1] = a - v[1];
    }
};

template <typename R>
struct Dft<3, R> {
    static __device__ __forceinline__ void run(cx<R> *v) {
        const cx<R> t = v[1] + v[2], d = v[1] - v[2];
        const cx<R> m = {v[0].x - R(0.5) * t.x, v[0].y - R(0.5) * t.y};
        const R s = Kc<R>::s3;
        v[0] = v[0] + t;
        v[1] = {m.x + s * d.y, m.y - s * d.x};
        v[2] = {m.x - s * d.y, m.y + s * d.x};
    }
};

template <typename R>
struct Dft<4, R> {
    static __device__ __forceinline__ void run(cx<R> *v) { dft4(v[0], v[1], v[2], v[3]); }
};

template <typename R>
struct Dft<5, R> {
    static __device__ __forceinline__ void run(cx<R> *v) {
        using K = Kc<R>;
        const cx<R> t1 = v[1] + v[4], t2 = v[2] + v[3], d1 = v[1] - v[4], d2 = v[2] - v[3];
        const cx<R> m1 = {v[0].x + K::c51 * t1.x + K::c52 * t2.x, v[0].y + K::c51 * t1.y + K::c52 * t2.y};
        const cx<R> m2 = {v[0].x + K::c52 * t1.x + K::c51 * t2.x, v[0].y + K::c52 * t1.y + K::c51 * t2.y};
        const cx<R> n1 = {K::s51 * d1.x + K::s52 * d2.x, K::s51 * d1.y + K::s52 * d2.y};
        const cx<R> n2 = {K::s52 * d1.x - K::s51 * d2.x, K::s52 * d1.y - K::s51 * d2.y};
        v[0] = v[0] + t1 + t2;
        v[1] = {m1.x + n1.y, m1.y - n1.x};
        v[4] = {m1.x - n1.y, m1.y + n1.x};
        v[2] = {m2.x + n2.y, m2.y - n2.x};
        v[3] = {m2.x - n2.y, m2.y + n2.x};
    }
};

template <typename R>
struct Dft<8, R> {
    static __device__ __forceinline__ void run(cx<R> *v) {
        const R h = Kc<R>::rs2;
        dft4(v[0], v[2], v[4], v[6]);  // even half -> E0..E3
        dft4(v[1], v[3], v[5], v[7]);  // odd half  -> O0..O3
        const cx<R> o1 = {(v[3].x + v[3].y) * h, (v[3].y - v[3].x) * h};   // O1 w8
        const cx<R> o2 = mul_mi(v[5]);                                      // O2 w8^2
        const cx<R> o3 = {(v[7].y - v[7].x) * h, -(v[7].x + v[7].y) * h};  // O3 w8^3
        const cx<R> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1];
        v[0] = e0 + o0;
        v[4] = e0 - o0;
        v[1] = e1 + o1;
        v[5] = e1 - o1;
        v[2] = e2 + o2;
        v[6] = e2 - o2;
        v[3] = e3 + o3;
        v[7] = e3 - o3;
    }
};

template <typename R>
struct Dft<16, R> {
    // 16 = 4 x 4: DFT4 down the columns n2 (inputs 4 n1 + n2), twiddle by
    // w16^(n2 k1), DFT4 along the rows; output k1 + 4 k2.
    static __device__ __forceinline__ void run(cx<R> *v) {
        using K = Kc<R>;
        for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
        // now v[4 k1 + n2] = A[n2][k1]
        const cx<R> w1 = {K::c8, -K::s8}, w2 = {K::rs2, -K::rs2}, w3 = {K::s8, -K::c8};
        const cx<R> w6 = {-K::rs2, -K::rs2}, w9 = {-K::c8, K::s8};
        v[5] = cmul(v[5], w1);    // (k1 1, n2 1): w^1
        v[6] = cmul(v[6], w2);    // (1, 2): w^2
        v[7] = cmul(v[7], w3);    // (1, 3): w^3
        v[9] = cmul(v[9], w2);    // (2, 1): w^2
        v[10] = mul_mi(v[10]);    // (2, 2): w^4
        v[11] = cmul(v[11], w6);  // (2, 3): w^6
        v[13] = cmul(v[13], w3);  // (3, 1): w^3
        v[14] = cmul(v[14], w6);  // (3, 2): w^6
        v[15] = cmul(v[15], w9);  // (3, 3): w^9
        for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
        // v[4 k1 + k2] = X[k1 + 4 k2]: transpose the 4 x 4 block
        cx<R> t;
        t = v[1]; v[1] = v[4]; v[4] = t;
        t = v[2]; v[2] = v[8]; v[8] = t;
        t = v[3]; v[3] = v[12]; v[12] = t;
        t = v[6]; v[6] = v[9]; v[9] = t;
        t = v[7]; v[7] = v[13]; v[13] = t;
        t = v[11]; v[11] = v[14]; v[14] = t;
    }
};

// ------------------------------------------------------- storage policies
struct StC64 {
    using R = float;
    static constexpr bool kHalf = false;
    static __device__ __forceinline__ cx<R> load(const void *p, long long i, int) {
        const float2 v = reinterpret_cast<const float2 *>(p)[i];
        return {v.x, v.y};
    }
    static __device__ __forceinline__ void store(void *p, long long i, cx<R> v, int) {
        reinterpret_cast<float2 *>(p)[i] = make_float2(v.x, v.y);
    }
};

struct StC128 {
    using R = double;
    static constexpr bool kHalf = false;
    static __device__ __forceinline__ cx<R> load(const void *p, long long i, int) {
        const double2 v = reinterpret_cast<const double2 *>(p)[i];
        return {v.x, v.y};
    }
    static __device__ __forceinline__ void store(void *p, long long i, cx<R> v, int) {
        reinterpret_cast<double2 *>(p)[i] = make_double2(v.x, v.y);
    }
};

__device__ __forceinline__ float f16_bits_to_float(unsigned short b) {
    return __half2float(__ushort_as_half(b));
}
__device__ __forceinline__ unsigned short float_to_f16_bits(float f) {
    return __half_as_ushort(__float2half_rn(f));
}
__device__ __forceinline__ float bf16_bits_to_float(unsigned short b) {
    return __uint_as_float(static_cast<unsigned>(b) << 16);
}
// Round to nearest, ties to even, on the upper 16 bits of the binary32 value.
__device__ __forceinline__ unsigned short float_to_bf16_bits(float f) {
    const unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<unsigned short>((u >> 16) | 0x40u);
    return static_cast<unsigned short>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <bool BF>
struct StHalf {
    using R = float;
    static constexpr bool kHalf = true;
    // value = stored * 2^e
    static __device__ __forceinline__ cx<R> load(const void *p, long long i, int e) {
        const unsigned u = reinterpret_cast<const unsigned *>(p)[i];
        const unsigned short lo = static_cast<unsigned short>(u & 0xffffu);
        const unsigned short hi = static_cast<unsigned short>(u >> 16);
        const float re = BF ? bf16_bits_to_float(lo) : f16_bits_to_float(lo);
        const float im = BF ? bf16_bits_to_float(hi) : f16_bits_to_float(hi);
        return {ldexpf(re, e), ldexpf(im, e)};
    }
    // stores v * 2^-e, rounded to nearest even
    static __device__ __forceinline__ void store(void *p, long long i, cx<R> v, int e) {
        const float re = ldexpf(v.x, -e), im = ldexpf(v.y, -e);
        const unsigned lo = BF ? float_to_bf16_bits(re) : float_to_f16_bits(re);
        const unsigned hi = BF ? float_to_bf16_bits(im) : float_to_f16_bits(im);
        reinterpret_cast<unsigned *>(p)[i] = lo | (hi << 16);
    }
};

// Exponent for a line whose largest |re|, |im| is mx: the e with
// mx * 2^-e in [2^14, 2^15); 0 for an all-zero line.
__device__ __forceinline__ int line_exponent(float mx) {
    if (!(mx > 0.0f)) return 0;
    if (!(mx <= 3.402823466e38f)) return 127;
    int E;
    frexpf(mx, &E);  // mx = f 2^E, f in [0.5, 1)
    int e = E - 15;
    return e < -128 ? -128 : (e > 127 ? 127 : e);
}

// --------------------------------------------------------- launch arguments
struct PassArgs {
    const void *in;
    void *out;
    const void *tw;
    const int8_t *in_exp;
    int8_t *out_exp;
    long long nlines;  // contiguous: lines; strided: p range (== es)
    long long es;      // element stride
    long long nw;      // strided: w count
    long long ntiles;  // strided: tiles of L lines per w
    ExpMap em;
    int inverse;
    // runtime-radix kernel only
    int n, T, L, S;
    int radix[kMaxStages];
};

// ------------------------------------------------------ radix plans
struct RPlan {
    int n = 1, S = 0, rmax = 1;
    int r[kMaxStages] = {};
};

// Factor n into radices: the 5s, then the 3s, then the power of two as
// radix-8 stages with one radix-4 or radix-16 stage for the remainder
// (2 and 4 stand alone for n = 2, 4).
constexpr RPlan make_rplan(int n) {
    RPlan p;
    p.n = n;
    int m = n, c5 = 0, c3 = 0, a2 = 0;
    while (m % 5 == 0) { m /= 5; ++c5; }
    while (m % 3 == 0) { m /= 3; ++c3; }
    while (m % 2 == 0) { m /= 2; ++a2; }
    if (m != 1) { p.S = -1; return p; }
    for (int i = 0; i < c5; ++i) p.r[p.S++] = 5;
    for (int i = 0; i < c3; ++i) p.r[p.S++] = 3;
    int k = a2 / 3, rem = a2 % 3;
    if (rem == 1 && k >= 1) {
        for (int i = 0; i < k - 1; ++i) p.r[p.S++] = 8;
        p.r[p.S++] = 16;
    } else {
        for (int i = 0; i < k; ++i) p.r[p.S++] = 8;
        if (rem == 1) p.r[p.S++] = 2;
        if (rem == 2) p.r[p.S++] = 4;
    }
    for (int i = 0; i < p.S; ++i) p.rmax = p.r[i] > p.rmax ? p.r[i] : p.rmax;
    return p;
}

constexpr int ns_before(const RPlan &p, int s) {
    int v = 1;
    for (int i = 0; i < s; ++i) v *= p.r[i];
    return v;
}

constexpr int floor_pow2(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}
constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

constexpr int kLdsLimit = 65536;

// Compile-time launch shape of the static kernel for length N.
// T = N / rmax threads per line (one butterfly per thread on the largest-radix
// stages).  Contiguous passes take about 256 threads per block.  Strided
// passes take L neighbouring lines so that each row of the tile is a
// 128-byte segment (16 x 8-byte, 8 x 16-byte or 32 x 4-byte elements), or
// more lines when T is small, within 1024 threads and the LDS limit.
template <int N, int KIND, int STORE_BYTES, int COMPUTE_BYTES>
struct SCfg {
    static constexpr RPlan plan = make_rplan(N);
    static constexpr int S = plan.S;
    static constexpr int T = N / plan.rmax;
    static constexpr int kLdsLines = cmax(1, kLdsLimit / (N * COMPUTE_BYTES));
    static constexpr int L = KIND == kContiguous
                                 ? floor_pow2(cmax(1, cmin(cmin(256 / T, 256), kLdsLines)))
                                 : floor_pow2(cmax(1, cmin(cmin(cmax(128 / STORE_BYTES, 256 / T), 1024 / T), kLdsLines)));
    static constexpr int kBlock = T * L;
    static constexpr size_t kLds = (size_t)L * N * COMPUTE_BYTES + 4 * (size_t)L;
};

// ------------------------------------------------------------ block context
template <typename R>
struct Ctx {
    cx<R> *lds;
    unsigned *red;     // per-line max (half storage)
    long long base;    // element index of the line's first element
    long long es;
    int t, l, L, n;
    bool valid;        // the line exists
    int ebase;         // input exponent index without the j term
    long long ea3;     // input exponent stride along the line
    int kind;
};

template <int KIND>
__device__ __forceinline__ int lds_index(int l, int e, int n, int L) {
    return KIND == kContiguous ? l * n + e : e * L + l;
}

template <class St>
__device__ __forceinline__ cx<typename St::R> load_elem(const PassArgs &a, long long base, long long es,
                                                        int e, int ebase, long long ea3) {
    int ex = 0;
    if (St::kHalf && a.in_exp) ex = a.in_exp[ebase + ea3 * e];
    cx<typename St::R> v = St::load(a.in, base + es * e, ex);
    if (a.inverse) v.y = -v.y;
    return v;
}

// ------------------------------------------------------------ static kernel
template <class Cfg, class St, int KIND, int S>
__device__ __forceinline__ void static_stage(const PassArgs &a, Ctx<typename St::R> &c) {
    using R = typename St::R;
    constexpr int N = Cfg::plan.n;
    constexpr int T = Cfg::T;
    constexpr int L = Cfg::L;
    constexpr int RAD = Cfg::plan.r[S];
    constexpr int Ns = ns_before(Cfg::plan, S);
    constexpr int NB = N / RAD;
    constexpr int B = (NB + T - 1) / T;
    constexpr bool kGuard = (NB % T) != 0;
    constexpr int kTwStride = N / (Ns * RAD);
    constexpr bool kLast = (S == Cfg::S - 1);
    const cx<R> *tw = reinterpret_cast<const cx<R> *>(a.tw);

    cx<R> v[B][RAD];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = c.t + b * T;
        if (!kGuard || j < NB) {
#pragma unroll
            for (int q = 0; q < RAD; ++q) {
                const int e = j + q * NB;
                if constexpr (S == 0) {
                    v[b][q] = c.valid ? load_elem<St>(a, c.base, c.es, e, c.ebase, c.ea3) : cx<R>{R(0), R(0)};
                } else {
                    v[b][q] = c.lds[lds_index<KIND>(c.l, e, N, L)];
                }
            }
            if constexpr (Ns > 1) {
                const int k = j % Ns;
#pragma unroll
                for (int q = 1; q < RAD; ++q) v[b][q] = cmul(v[b][q], tw[q * k * kTwStride]);
            }
            Dft<RAD, R>::run(v[b]);
        }
    }

    if constexpr (kLast) {
        // outputs of the last stage: index j + q * NB (Ns * RAD == N)
        int ex = 0;
        if constexpr (St::kHalf) {
            float mx = 0.0f;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int j = c.t + b * T;
                if (!kGuard || j < NB) {
#pragma unroll
                    for (int q = 0; q < RAD; ++q)
                        mx = fmaxf(mx, fmaxf(fabsf(v[b][q].x), fabsf(v[b][q].y)));
                }
            }
            atomicMax(&c.red[c.l], __float_as_uint(mx));
            __syncthreads();
            ex = line_exponent(__uint_as_float(c.red[c.l]));
        }
        if (c.valid) {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int j = c.t + b * T;
                if (!kGuard || j < NB) {
#pragma unroll
                    for (int q = 0; q < RAD; ++q) {
                        cx<R> o = v[b][q];
                        if (a.inverse) o.y = -o.y;
                        St::store(a.out, c.base + c.es * (j + q * NB), o, ex);
                    }
                }
            }
        }
        if constexpr (St::kHalf) c.ebase = ex;  // hand the exponent back to the caller
    } else {
        if constexpr (S > 0) __syncthreads();
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = c.t + b * T;
            if (!kGuard || j < NB) {
                const int k = j % Ns;
                const int o0 = (j / Ns) * Ns * RAD + k;
#pragma unroll
                for (int q = 0; q < RAD; ++q) c.lds[lds_index<KIND>(c.l, o0 + q * Ns, N, L)] = v[b][q];
            }
        }
        __syncthreads();
        static_stage<Cfg, St, KIND, S + 1>(a, c);
    }
}

// Line coordinates of this thread: contiguous q = line; strided q = p, w.
template <int KIND>
__device__ __forceinline__ void line_coords(const PassArgs &a, int l, int L, long long &q, long long &w,
                                            bool &valid) {
    if (KIND == kContiguous) {
        q = (long long)blockIdx.x * L + l;
        w = 0;
        valid = q < a.nlines;
    } else {
        const long long tile = (long long)blockIdx.x % a.ntiles;
        w = (long long)blockIdx.x / a.ntiles;
        q = tile * L + l;
        valid = q < a.es;
    }
}

template <class Cfg, class St, int KIND>
__global__ void __launch_bounds__(Cfg::kBlock) fft_static(const PassArgs a) {
    using R = typename St::R;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int N = Cfg::plan.n;
    constexpr int T = Cfg::T;
    constexpr int L = Cfg::L;
    Ctx<R> c;
    c.lds = reinterpret_cast<cx<R> *>(smem);
    c.red = reinterpret_cast<unsigned *>(smem + (size_t)L * N * sizeof(cx<R>));
    const int tid = threadIdx.x;
    if (KIND == kContiguous) {
        c.l = tid / T;
        c.t = tid % T;
    } else {
        c.l = tid % L;
        c.t = tid / L;
    }
    long long q, w;
    line_coords<KIND>(a, c.l, L, q, w, c.valid);
    c.es = KIND == kContiguous ? 1 : a.es;
    c.base = KIND == kContiguous ? q * N : q + w * a.es * N;
    c.L = L;
    c.n = N;
    c.kind = KIND;
    c.ebase = 0;
    c.ea3 = 0;
    if constexpr (St::kHalf) {
        const ExpMap &m = a.em;
        c.ebase = (int)((q % m.qmod) * m.a0 + (q / m.qmod) * m.a1 + w * m.a2);
        c.ea3 = m.a3;
        if (c.t == 0) c.red[c.l] = 0u;
        __syncthreads();
    }
    static_stage<Cfg, St, KIND, 0>(a, c);
    if constexpr (St::kHalf) {
        if (c.valid && c.t == 0 && a.out_exp) {
            const ExpMap &m = a.em;
            a.out_exp[(q % m.qmod) * m.b0 + (q / m.qmod) * m.b1 + w * m.b2] = (int8_t)c.ebase;
        }
    }
}

// ------------------------------------------------------- runtime-radix kernel
// Any supported length.  Stages ping-pong between two LDS buffers, the last
// stage included; a final sweep stores the line from LDS.
template <int RAD, typename R, int KIND>
__device__ __forceinline__ void generic_stage(const cx<R> *src, cx<R> *dst, const cx<R> *tw, int n, int L,
                                              int l, int t, int T, int Ns) {
    const int NB = n / RAD;
    const int tws = n / (Ns * RAD);
    for (int j = t; j < NB; j += T) {
        cx<R> v[RAD];
#pragma unroll
        for (int q = 0; q < RAD; ++q) v[q] = src[lds_index<KIND>(l, j + q * NB, n, L)];
        const int k = j % Ns;
        if (Ns > 1) {
#pragma unroll
            for (int q = 1; q < RAD; ++q) v[q] = cmul(v[q], tw[q * k * tws]);
        }
        Dft<RAD, R>::run(v);
        const int o0 = (j / Ns) * Ns * RAD + k;
#pragma unroll
        for (int q = 0; q < RAD; ++q) dst[lds_index<KIND>(l, o0 + q * Ns, n, L)] = v[q];
    }
}

template <class St, int KIND>
__global__ void __launch_bounds__(256) fft_generic(const PassArgs a) {
    using R = typename St::R;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = a.n, T = a.T, L = a.L;
    cx<R> *buf0 = reinterpret_cast<cx<R> *>(smem);
    cx<R> *buf1 = buf0 + (size_t)L * n;
    unsigned *red = reinterpret_cast<unsigned *>(buf1 + (size_t)L * n);
    const cx<R> *tw = reinterpret_cast<const cx<R> *>(a.tw);
    const int tid = threadIdx.x;
    int l, t;
    if (KIND == kContiguous) {
        l = tid / T;
        t = tid % T;
    } else {
        l = tid % L;
        t = tid / L;
    }
    const bool active = tid < T * L;
    long long q, w;
    bool valid;
    line_coords<KIND>(a, l, L, q, w, valid);
    valid = valid && active;
    const long long es = KIND == kContiguous ? 1 : a.es;
    const long long base = KIND == kContiguous ? q * n : q + w * a.es * n;
    int ebase = 0;
    if constexpr (St::kHalf) {
        const ExpMap &m = a.em;
        ebase = (int)((q % m.qmod) * m.a0 + (q / m.qmod) * m.a1 + w * m.a2);
        if (active && t == 0) red[l] = 0u;
    }
    // load the line into buf0 (coalesced: consecutive t, consecutive e)
    if (active) {
        for (int e = t; e < n; e += T)
            buf0[lds_index<KIND>(l, e, n, L)] =
                valid ? load_elem<St>(a, base, es, e, ebase, St::kHalf ? a.em.a3 : 0) : cx<R>{R(0), R(0)};
    }
    __syncthreads();
    cx<R> *src = buf0, *dst = buf1;
    int Ns = 1;
    for (int s = 0; s < a.S; ++s) {
        const int rad = a.radix[s];
        if (active) {
            switch (rad) {
                case 2: generic_stage<2, R, KIND>(src, dst, tw, n, L, l, t, T, Ns); break;
                case 3: generic_stage<3, R, KIND>(src, dst, tw, n, L, l, t, T, Ns); break;
                case 4: generic_stage<4, R, KIND>(src, dst, tw, n, L, l, t, T, Ns); break;
                case 5: generic_stage<5, R, KIND>(src, dst, tw, n, L, l, t, T, Ns); break;
                case 8: generic_stage<8, R, KIND>(src, dst, tw, n, L, l, t, T, Ns); break;
                default: generic_stage<16, R, KIND>(src, dst, tw, n, L, l, t, T, Ns); break;
            }
        }
        Ns *= rad;
        cx<R> *tmp = src;
        src = dst;
        dst = tmp;
        __syncthreads();
    }
    int ex = 0;
    if constexpr (St::kHalf) {
        float mx = 0.0f;
        if (active)
            for (int e = t; e < n; e += T) {
                const cx<R> v = src[lds_index<KIND>(l, e, n, L)];
                mx = fmaxf(mx, fmaxf(fabsf((float)v.x), fabsf((float)v.y)));
            }
        if (active) atomicMax(&red[l], __float_as_uint(mx));
        __syncthreads();
        if (active) ex = line_exponent(__uint_as_float(red[l]));
        if (valid && t == 0 && a.out_exp) {
            const ExpMap &m = a.em;
            a.out_exp[(q % m.qmod) * m.b0 + (q / m.qmod) * m.b1 + w * m.b2] = (int8_t)ex;
        }
    }
    if (valid) {
        for (int e = t; e < n; e += T) {
            cx<R> o = src[lds_index<KIND>(l, e, n, L)];
            if (a.inverse) o.y = -o.y;
            St::store(a.out, base + es * e, o, ex);
        }
    }
}

// ------------------------------------------------------------ kernel table
struct Entry {
    int n, kind, dtype;
    const void *func;
    int T, L, block;
    size_t lds;
    RPlan plan;
};

template <int N, int KIND, class St, int SB, int DT>
Entry make_entry() {
    using Cfg = SCfg<N, KIND, SB, (int)sizeof(cx<typename St::R>)>;
    Entry e;
    e.n = N;
    e.kind = KIND;
    e.dtype = DT;
    e.func = reinterpret_cast<const void *>(&fft_static<Cfg, St, KIND>);
    e.T = Cfg::T;
    e.L = Cfg::L;
    e.block = Cfg::kBlock;
    e.lds = Cfg::kLds;
    e.plan = Cfg::plan;
    return e;
}

#define CROFT_ENTRIES_FOR(N)                                          \
    make_entry<N, kContiguous, StC64, 8, kC64>(),                     \
        make_entry<N, kStrided, StC64, 8, kC64>(),                    \
        make_entry<N, kContiguous, StC128, 16, kC128>(),              \
        make_entry<N, kStrided, StC128, 16, kC128>(),                 \
        make_entry<N, kContiguous, StHalf<false>, 4, kC16F>(),        \
        make_entry<N, kStrided, StHalf<false>, 4, kC16F>(),           \
        make_entry<N, kContiguous, StHalf<true>, 4, kC16B>(),         \
        make_entry<N, kStrided, StHalf<true>, 4, kC16B>()

const std::vector<Entry> &table() {
    static const std::vector<Entry> t = {
        CROFT_ENTRIES_FOR(2),   CROFT_ENTRIES_FOR(4),   CROFT_ENTRIES_FOR(8),
        CROFT_ENTRIES_FOR(16),  CROFT_ENTRIES_FOR(32),  CROFT_ENTRIES_FOR(64),
        CROFT_ENTRIES_FOR(128), CROFT_ENTRIES_FOR(256), CROFT_ENTRIES_FOR(512),
        CROFT_ENTRIES_FOR(1024), CROFT_ENTRIES_FOR(2048), CROFT_ENTRIES_FOR(4096),
        CROFT_ENTRIES_FOR(48),  CROFT_ENTRIES_FOR(60),  CROFT_ENTRIES_FOR(72),
        CROFT_ENTRIES_FOR(80),  CROFT_ENTRIES_FOR(96),  CROFT_ENTRIES_FOR(100),
        CROFT_ENTRIES_FOR(384),
    };
    return t;
}

const void *generic_func(int kind, int dtype) {
    if (kind == kContiguous) {
        switch (dtype) {
            case kC64: return reinterpret_cast<const void *>(&fft_generic<StC64, kContiguous>);
            case kC128: return reinterpret_cast<const void *>(&fft_generic<StC128, kContiguous>);
            case kC16F: return reinterpret_cast<const void *>(&fft_generic<StHalf<false>, kContiguous>);
            default: return reinterpret_cast<const void *>(&fft_generic<StHalf<true>, kContiguous>);
        }
    }
    switch (dtype) {
        case kC64: return reinterpret_cast<const void *>(&fft_generic<StC64, kStrided>);
        case kC128: return reinterpret_cast<const void *>(&fft_generic<StC128, kStrided>);
        case kC16F: return reinterpret_cast<const void *>(&fft_generic<StHalf<false>, kStrided>);
        default: return reinterpret_cast<const void *>(&fft_generic<StHalf<true>, kStrided>);
    }
}

}  // namespace

bool select_kernel(int n, int kind, int dtype, bool force_generic, KernelConfig *cfg) {
    if (n < 1 || n > kMaxLength) return false;
    if (!force_generic) {
        for (const Entry &e : table()) {
            if (e.n == n && e.kind == kind && e.dtype == dtype) {
                cfg->func = e.func;
                cfg->generic = false;
                cfg->threads_per_line = e.T;
                cfg->lines = e.L;
                cfg->block = e.block;
                cfg->lds = e.lds;
                cfg->nstages = e.plan.S;
                for (int s = 0; s < e.plan.S; ++s) cfg->radix[s] = e.plan.r[s];
                return true;
            }
        }
    }
    const RPlan p = make_rplan(n);
    if (p.S < 0) return false;
    const int cb = dtype == kC128 ? 16 : 8;                      // compute bytes
    const int sb = (int)element_bytes(dtype);                    // storage bytes
    int T = n / p.rmax;
    if (T < 1) T = 1;
    if (T > 256) T = 256;
    const size_t per_line = 2 * (size_t)n * cb + 4;
    int lds_lines = (int)((160 * 1024) / per_line);
    if (lds_lines < 1) return false;
    int L;
    if (kind == kContiguous) {
        L = 256 / T;
    } else {
        L = 128 / sb;
        if (L * T > 256) L = 256 / T;
        if (L < 1) L = 1;
    }
    if (L > lds_lines) L = lds_lines;
    if (L < 1) L = 1;
    // round down to a power of two
    int p2 = 1;
    while (p2 * 2 <= L) p2 *= 2;
    L = p2;
    cfg->func = generic_func(kind, dtype);
    cfg->generic = true;
    cfg->threads_per_line = T;
    cfg->lines = L;
    cfg->block = ((T * L + 63) / 64) * 64;
    cfg->lds = (size_t)L * per_line;
    cfg->nstages = p.S;
    for (int s = 0; s < p.S; ++s) cfg->radix[s] = p.r[s];
    return true;
}

hipError_t launch_pass(const PassLaunch &pl, int dtype, const void *in, void *out, const int8_t *in_exp,
                       int8_t *out_exp, int inverse, hipStream_t stream) {
    PassArgs a;
    a.in = in;
    a.out = out;
    a.tw = pl.tw;
    a.in_exp = in_exp;
    a.out_exp = out_exp;
    a.es = pl.es;
    a.nw = pl.nw;
    a.em = pl.em;
    a.inverse = inverse;
    a.n = pl.n;
    a.T = pl.cfg.threads_per_line;
    a.L = pl.cfg.lines;
    a.S = pl.cfg.nstages;
    for (int s = 0; s < kMaxStages; ++s) a.radix[s] = pl.cfg.radix[s];
    long long blocks;
    if (pl.kind == kContiguous) {
        a.nlines = pl.nlines;
        a.ntiles = 1;
        blocks = (pl.nlines + a.L - 1) / a.L;
    } else {
        a.nlines = pl.es;
        a.ntiles = (pl.es + a.L - 1) / a.L;
        blocks = a.ntiles * pl.nw;
    }
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    void *args[] = {&a};
    return hipLaunchKernel(pl.cfg.func, dim3((unsigned)blocks), dim3(pl.cfg.block), args, pl.cfg.lds,
                           stream);
}

}  // namespace croft
