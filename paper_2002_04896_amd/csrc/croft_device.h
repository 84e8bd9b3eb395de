// croft_device.h -- device code of the HIP kernels for gfx950: one axis pass
// of the 3D FFT (included by the kernel translation units only).
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
// direction swaps real and imaginary parts on load and on store:
// swap(DFT(swap(x))) is the unnormalised inverse DFT.
//
// Half storage: a line is loaded as FP16/BF16 pairs scaled by 2^e of the line
// that stored each element, computed in FP32, and stored with one new
// exponent per line chosen from the line's largest |re|, |im|.

#pragma once

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "croft_internal.h"

namespace croft {
namespace dev {

// ------------------------------------------------------------------ complex
template <typename R>
struct cx {
    R x, y;
};
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
// Floating-point contraction is off for this file (-ffp-contract=off): every
// fused multiply-add below is written out, so the rounding of each operation
// is fixed by the source and does not depend on how a configuration is
// scheduled -- all tile shapes of a length give bit-identical results.
template <typename R>
__device__ __forceinline__ R fmaR(R a, R b, R c) {
    return __builtin_fma(a, b, c);
}
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {fmaR(a.x, b.x, -(a.y * b.y)), fmaR(a.x, b.y, a.y * b.x)};
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
        const cx<R> m = {fmaR(R(-0.5), t.x, v[0].x), fmaR(R(-0.5), t.y, v[0].y)};
        const R s = Kc<R>::s3;
        v[0] = v[0] + t;
        v[1] = {fmaR(s, d.y, m.x), fmaR(-s, d.x, m.y)};
        v[2] = {fmaR(-s, d.y, m.x), fmaR(s, d.x, m.y)};
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
        const cx<R> m1 = {fmaR(K::c52, t2.x, fmaR(K::c51, t1.x, v[0].x)),
                          fmaR(K::c52, t2.y, fmaR(K::c51, t1.y, v[0].y))};
        const cx<R> m2 = {fmaR(K::c51, t2.x, fmaR(K::c52, t1.x, v[0].x)),
                          fmaR(K::c51, t2.y, fmaR(K::c52, t1.y, v[0].y))};
        const cx<R> n1 = {fmaR(K::s52, d2.x, K::s51 * d1.x), fmaR(K::s52, d2.y, K::s51 * d1.y)};
        const cx<R> n2 = {fmaR(-K::s51, d2.x, K::s52 * d1.x), fmaR(-K::s51, d2.y, K::s52 * d1.y)};
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
// fetch() issues the global load and returns the stored bits untouched, so a
// prefetched tile costs no arithmetic until decode() runs on it.
typedef float vf2 __attribute__((ext_vector_type(2)));
typedef double vd2 __attribute__((ext_vector_type(2)));

struct StC64 {
    using R = float;
    using Raw = vf2;
    static constexpr bool kHalf = false;
    static __device__ __forceinline__ Raw fetch(const void *p, long long i) {
        return reinterpret_cast<const vf2 *>(p)[i];
    }
    static __device__ __forceinline__ cx<R> decode(Raw r, int) { return {r.x, r.y}; }
    static __device__ __forceinline__ void store(void *p, long long i, cx<R> v, int) {
        reinterpret_cast<float2 *>(p)[i] = make_float2(v.x, v.y);
    }
    static __device__ __forceinline__ Raw pack(cx<R> v, int) {
        vf2 w;
        w.x = v.x;
        w.y = v.y;
        return w;
    }
    static __device__ __forceinline__ void store_g(__attribute__((address_space(1))) char *p, cx<R> v, int) {
        *(__attribute__((address_space(1))) vf2 *)p = pack(v, 0);
    }
};

struct StC128 {
    using R = double;
    using Raw = vd2;
    static constexpr bool kHalf = false;
    static __device__ __forceinline__ Raw fetch(const void *p, long long i) {
        return reinterpret_cast<const vd2 *>(p)[i];
    }
    static __device__ __forceinline__ cx<R> decode(Raw r, int) { return {r.x, r.y}; }
    static __device__ __forceinline__ void store(void *p, long long i, cx<R> v, int) {
        reinterpret_cast<double2 *>(p)[i] = make_double2(v.x, v.y);
    }
    static __device__ __forceinline__ Raw pack(cx<R> v, int) {
        vd2 w;
        w.x = v.x;
        w.y = v.y;
        return w;
    }
    static __device__ __forceinline__ void store_g(__attribute__((address_space(1))) char *p, cx<R> v, int) {
        *(__attribute__((address_space(1))) vd2 *)p = pack(v, 0);
    }
};

__device__ __forceinline__ float f16_bits_to_float(unsigned short b) {
    return __half2float(__ushort_as_half(b));
}
__device__ __forceinline__ float bf16_bits_to_float(unsigned short b) {
    return __uint_as_float(static_cast<unsigned>(b) << 16);
}
// Two binary32 values to two bfloat16 (first in the low half), rounded to
// nearest, ties to even: one v_cvt_pk_bf16_f32 on gfx950.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned floats_to_bf16x2_bits(float lo, float hi) {
    const f32x2 w = {lo, hi};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(w, bf16x2));
}
// The same to two binary16, rounded to nearest, ties to even: one
// v_cvt_pk_f16_f32 on gfx950.
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned floats_to_f16x2_bits(float lo, float hi) {
    const f32x2 w = {lo, hi};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(w, f16x2));
}

template <bool BF>
struct StHalf {
    using R = float;
    using Raw = unsigned;
    static constexpr bool kHalf = true;
    static __device__ __forceinline__ Raw fetch(const void *p, long long i) {
        return reinterpret_cast<const unsigned *>(p)[i];
    }
    // the stored value itself, unscaled
    static __device__ __forceinline__ cx<R> decode_raw(Raw u) {
        const unsigned short lo = static_cast<unsigned short>(u & 0xffffu);
        const unsigned short hi = static_cast<unsigned short>(u >> 16);
        return {BF ? bf16_bits_to_float(lo) : f16_bits_to_float(lo), BF ? bf16_bits_to_float(hi) : f16_bits_to_float(hi)};
    }
    // value = stored * 2^e
    static __device__ __forceinline__ cx<R> decode(Raw u, int e) {
        const unsigned short lo = static_cast<unsigned short>(u & 0xffffu);
        const unsigned short hi = static_cast<unsigned short>(u >> 16);
        const float re = BF ? bf16_bits_to_float(lo) : f16_bits_to_float(lo);
        const float im = BF ? bf16_bits_to_float(hi) : f16_bits_to_float(hi);
        return {ldexpf(re, e), ldexpf(im, e)};
    }
    // stores v * 2^-e, rounded to nearest even
    static __device__ __forceinline__ unsigned encode(cx<R> v, int e) {
        const float re = ldexpf(v.x, -e), im = ldexpf(v.y, -e);
        if constexpr (BF) return floats_to_bf16x2_bits(re, im);
        return floats_to_f16x2_bits(re, im);
    }
    static __device__ __forceinline__ void store(void *p, long long i, cx<R> v, int e) {
        reinterpret_cast<unsigned *>(p)[i] = encode(v, e);
    }
    static __device__ __forceinline__ Raw pack(cx<R> v, int e) { return encode(v, e); }
    static __device__ __forceinline__ void store_g(__attribute__((address_space(1))) char *p, cx<R> v, int e) {
        *(__attribute__((address_space(1))) unsigned *)p = encode(v, e);
    }
};

// Exponent for a line whose largest |re|, |im| is mx: the e with
// mx * 2^-e in [2^14, 2^15); 0 for an all-zero line.
__device__ __forceinline__ int line_exponent(float mx) {
    if (!(mx > 0.0f)) return 0;
    if (!(mx <= 3.402823466e38f)) return 127;
    int E;
    frexpf(mx, &E);  // mx = f 2^E, f in [0.5, 1)
    const int e = E - 15;
    return e < -128 ? -128 : (e > 127 ? 127 : e);
}

// The same exponent for a line whose values carry a common factor 2^ein not
// yet applied: mx is the largest |re|, |im| before the factor.  Scaling by a
// power of two is exact, so this is line_exponent(mx 2^ein) wherever that
// product is a normal FP32 value, without forming it.
__device__ __forceinline__ int line_exponent_scaled(float mx, int ein) {
    if (!(mx > 0.0f)) return 0;
    if (!(mx <= 3.402823466e38f)) return 127;
    int E;
    frexpf(mx, &E);
    const int e = E + ein - 15;
    return e < -128 ? -128 : (e > 127 ? 127 : e);
}

// Largest of v over each aligned group of T lanes (T a power of two up to 64)
// by a butterfly of cross-lane moves: DPP quad permutations for lane
// distances 1 and 2, ds_swizzle for 4, 8 and 16 (within 32-lane halves),
// ds_bpermute for 32.  Unsigned order, as for the bits of non-negative floats.
template <int T>
__device__ __forceinline__ unsigned lanes_max_u32(unsigned v) {
    if constexpr (T >= 2) v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false));
    if constexpr (T >= 4) v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false));
    if constexpr (T >= 8) v = max(v, (unsigned)__builtin_amdgcn_ds_swizzle((int)v, 0x101F));
    if constexpr (T >= 16) v = max(v, (unsigned)__builtin_amdgcn_ds_swizzle((int)v, 0x201F));
    if constexpr (T >= 32) v = max(v, (unsigned)__builtin_amdgcn_ds_swizzle((int)v, 0x401F));
    if constexpr (T >= 64) {
        const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        v = max(v, (unsigned)__builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, (int)v));
    }
    return v;
}

// (q % qmod) c0 + (q / qmod) c1 + w c2 for a line q < 2^31, in 32 bits
// (exponent arrays hold fewer than 2^31 entries): the division is the
// multiply and shift the exponent map carries.
__device__ __forceinline__ unsigned exp_line_index(const ExpMap &m, long long q, long long w, long long c0,
                                                   long long c1, long long c2) {
    const unsigned uq = (unsigned)q;
    const unsigned d = (unsigned)(((unsigned long long)uq * m.qmul) >> m.qshift);
    const unsigned r = uq - d * (unsigned)m.qmod;
    return r * (unsigned)c0 + d * (unsigned)c1 + (unsigned)w * (unsigned)c2;
}

// The inverse transform is swap(DFT(swap(x))) with swap(a + ib) = b + ia.
template <bool INV, typename R>
__device__ __forceinline__ cx<R> maybe_swap(cx<R> v) {
    if constexpr (INV) return {v.y, v.x};
    return v;
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
    long long total;   // tiles in the launch
    ExpMap em;
    const void *tw2;   // real x pass: w_N^k, N = 2 n (the real line length)
    // fused multiply pass: the real multiplier (data layout), per-block
    // energy partials, and the spectrum elements per x-line (nx/2 + 1)
    const void *mul;
    double *partial;
    long long hx;
    // Bluestein's algorithm (runtime kernel): chirp (n), kernel DFT (m), m
    const void *chirp;
    const void *bhat;
    int m;
    int inverse;       // runtime-radix kernel only (static kernels take it as a template argument)
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
// LDS twiddle table: stage s >= 1 holds (r_s - 1) * Ns_s entries,
// entry (q, k) = w_N^(q k N / (Ns R)) at offset (q - 1) Ns + k.
constexpr int tw_offset(const RPlan &p, int s) {
    int o = 0;
    for (int i = 1; i < s; ++i) o += (p.r[i] - 1) * ns_before(p, i);
    return o;
}

constexpr int floor_pow2(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}
constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// LDS budget used to size default tiles: two blocks fit in a CU's 160 KiB.
constexpr int kLdsLimit = 80 * 1024;

// Compile-time launch shape of a static kernel for length N.
//   EPT: elements per thread (T = N / EPT threads per line); 0 = the largest
//        radix, so the largest-radix stages take one butterfly per thread.
//   LREQ: lines per block; 0 = the default: about 256 threads for contiguous
//        lines; for strided lines enough neighbouring lines that each row of
//        the tile is a 128-byte segment, more when T is small, within 1024
//        threads and the LDS budget.
//   PAD: contiguous lines only: one padding element per 32 in LDS.
//   PF: prefetch the next tile's loads while transforming the current one.
//   NT: global loads and stores carry the non-temporal (streaming) hint.
//   XO: with one block per tile, each XCD takes a contiguous run of tiles.
template <int N, int KIND, int STORE_BYTES, int COMPUTE_BYTES, int EPT = 0, int LREQ = 0, int PAD = 0,
          int PF = 1, int NT = 0, int XO = 0>
struct SCfg {
    static constexpr bool kPrefetch = PF != 0;
    static constexpr bool kNT = NT != 0;
    static constexpr bool kXO = XO != 0;
    static constexpr RPlan plan = make_rplan(N);
    static constexpr int S = plan.S;
    static constexpr int kEpt = EPT > 0 ? EPT : plan.rmax;
    static constexpr int T = cmax(1, N / kEpt);
    static constexpr int kLineStride = (KIND == kContiguous && PAD) ? N + (N + 31) / 32 : N;
    static constexpr int kTwN = tw_offset(plan, S);
    static constexpr int kLdsLines = cmax(1, (kLdsLimit - kTwN * COMPUTE_BYTES) / (kLineStride * COMPUTE_BYTES));
    static constexpr int L = LREQ > 0 ? LREQ
                             : KIND == kContiguous
                                 ? floor_pow2(cmax(1, cmin(cmin(256 / T, 256), kLdsLines)))
                                 : floor_pow2(cmax(1, cmin(cmin(cmax(128 / STORE_BYTES, 256 / T), 1024 / T), kLdsLines)));
    static constexpr int kBlock = T * L;
    // lines never straddle a wavefront: stages sync per wave, not per block
    static constexpr bool kWaveSync = KIND == kContiguous && T <= 64 && (64 % T) == 0;
    static constexpr size_t kLdsData = (size_t)L * kLineStride * COMPUTE_BYTES;
    static constexpr size_t kLds = kLdsData + (size_t)kTwN * COMPUTE_BYTES + 4 * (size_t)L;
};

template <int KIND, int LS, int PAD>
__device__ __forceinline__ int lds_index(int l, int e, int L) {
    if constexpr (KIND == kContiguous) return l * LS + e + (PAD ? (e >> 5) : 0);
    return e * L + l;
}

template <bool WAVE>
__device__ __forceinline__ void stage_sync() {
    if constexpr (WAVE) {
        // all lanes of a line are in this wavefront: order its LDS accesses
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// ------------------------------------------------------------ static kernel
// A block holds a tile of L lines and loops over tiles with a stride of the
// grid size; while one tile is transformed the global loads of the next are
// in flight (they are only decoded when that tile starts).
template <class Cfg, class St>
struct Tile {
    static constexpr int R0 = Cfg::plan.r[0];
    static constexpr int NB0 = Cfg::plan.n / R0;
    static constexpr int B0 = (NB0 + Cfg::T - 1) / Cfg::T;
    // with prefetch: the stored bits (and exponents), decoded when the tile
    // starts; without: the decoded values
    static constexpr bool kRaw = Cfg::kPrefetch;
    using Elem = typename std::conditional<kRaw, typename St::Raw, cx<typename St::R>>::type;
    Elem e[B0][R0];
    int ex[(kRaw && St::kHalf) ? B0 : 1][(kRaw && St::kHalf) ? R0 : 1];
    int lex = 0;  // line-scaled contiguous passes: the line's input exponent
};

// 16-bit storage, contiguous lines: every element of a line carries the
// line's one input exponent (the first pass reads x-lines, exponents per
// x-line; the planner sends contiguous passes with per-element exponents to
// the runtime-radix kernel).  The FFT is linear, so the pass transforms the
// stored values unscaled and folds 2^ein into the output scaling: the
// element-wise scaling and the per-element exponent loads disappear, and the
// results are the same bits (scaling by a power of two commutes with every
// rounding, as long as no value leaves FP32's normal range).
template <class St, int KIND>
constexpr bool kLineScaled = St::kHalf && KIND == kContiguous;

struct TileCoord {
    long long q;      // line coordinate of this thread (contiguous: line; strided: p)
    long long w;      // strided: line block
    long long tbase;  // element index of the tile's first element (uniform in the block)
    bool valid;
};

// Element index = tbase + lane + (b T + q NB) es: the tile origin and the
// stage offsets are uniform across the block, the lane part is fixed per
// thread, so each access costs one address add.
template <class Cfg, int KIND>
__device__ __forceinline__ TileCoord tile_coord(const PassArgs &a, long long tx, long long w, int l) {
    TileCoord c;
    c.q = tx * Cfg::L + l;
    c.w = w;
    c.tbase = KIND == kContiguous ? tx * Cfg::L * Cfg::plan.n : tx * Cfg::L + w * a.es * Cfg::plan.n;
    c.valid = c.q < (KIND == kContiguous ? a.nlines : a.es);
    return c;
}

// Byte offset of the thread's first element from the tile origin; it fits in
// 32 bits (the planner sends larger strides to the runtime-radix kernel), so
// an access is a uniform 64-bit base plus this one per-thread register.
template <class Cfg, class St, int KIND>
__device__ __forceinline__ unsigned lane_offset(int l, int t, long long es) {
    const long long e = (KIND == kContiguous ? (long long)l * Cfg::plan.n : (long long)l) + (long long)t * es;
    return (unsigned)(e * (long long)sizeof(typename St::Raw));
}

// The tile base is the same in every lane; saying so (readfirstlane) keeps it
// in scalar registers, so each access is a scalar base plus one 32-bit lane
// offset register (global address space kept explicit).
typedef __attribute__((address_space(1))) char gchar;

__device__ __forceinline__ gchar *uniform_gptr(const void *p, long long byte_off) {
    const unsigned long long v = reinterpret_cast<unsigned long long>(p) + (unsigned long long)byte_off;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (gchar *)(((unsigned long long)hi << 32) | lo);
}

// The 32-bit lane offset, re-materialised at each access: left to itself the
// compiler hoists one 64-bit zero-extended copy out of the tile loop and adds
// it in 64 bits, so each access would hold a 64-bit address in vector
// registers instead of a scalar base plus this one offset register.
__device__ __forceinline__ unsigned lane_reg(unsigned v) {
    unsigned r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// base: the tile's origin, made uniform once per tile (uniform_gptr); the
// uniform element offset is then added in scalar registers.  REMAT: the lane
// offset re-materialised here (the one-line-per-lane kernels, where the copy
// is the load's own destination register); otherwise the caller passes one
// copy made in the same block as a group of accesses, which all fold it.
template <class St, bool NT = false, bool REMAT = true>
__device__ __forceinline__ typename St::Raw fetch_at(gchar *base, long long uniform_elem, unsigned lane_bytes) {
    using Raw = typename St::Raw;
    if constexpr (REMAT) lane_bytes = lane_reg(lane_bytes);
    gchar *b = base + uniform_elem * (long long)sizeof(Raw);
    const __attribute__((address_space(1))) Raw *q = (const __attribute__((address_space(1))) Raw *)(b + lane_bytes);
    if constexpr (NT) return __builtin_nontemporal_load(q);
    return *q;
}

template <class St, bool NT = false, bool REMAT = true>
__device__ __forceinline__ void store_at(gchar *base, long long uniform_elem, unsigned lane_bytes,
                                         cx<typename St::R> v, int ex) {
    if constexpr (REMAT) lane_bytes = lane_reg(lane_bytes);
    gchar *b = base + uniform_elem * (long long)sizeof(typename St::Raw);
    if constexpr (NT) {
        __builtin_nontemporal_store(St::pack(v, ex), (__attribute__((address_space(1))) typename St::Raw *)(b + lane_bytes));
    } else {
        St::store_g(b + lane_bytes, v, ex);
    }
}

// The input exponent of every element when a pass is given none.
static __device__ const int8_t kZeroExponent = 0;

template <class Cfg, class St, int KIND, bool INV>
__device__ __forceinline__ void fetch_tile(const PassArgs &a, const TileCoord &c, int t, unsigned lane,
                                           long long es, Tile<Cfg, St> &tl) {
    using TL = Tile<Cfg, St>;
    if (!c.valid) return;
    // exponent of element (line q, position j) at ebase(q) + a3 j: the lane
    // part ebase + a3 t as one 32-bit offset (exponent arrays hold fewer than
    // 2^31 entries), the rest uniform, as for the data
    // (no input exponents: every load reads the one zero byte)
    unsigned elane = 0;
    long long ea3 = 0;
    const int8_t *ep = &kZeroExponent;
    if constexpr (St::kHalf) {
        if (a.in_exp) {
            const ExpMap &m = a.em;
            ep = a.in_exp;
            ea3 = m.a3;
            elane = exp_line_index(m, c.q, c.w, m.a0, m.a1, m.a2) + (unsigned)ea3 * (unsigned)t;
        }
    }
    // contiguous tiles: the tile origin made uniform once per tile (left in
    // each access, the compiler computes it in vector registers there)
    const long long ut = KIND == kContiguous ? 0 : c.tbase;
    gchar *const ib = uniform_gptr(a.in, (c.tbase - ut) * (long long)sizeof(typename St::Raw));
    gchar *const eb = uniform_gptr(ep, 0);
    if constexpr (kLineScaled<St, KIND>) tl.lex = *(const __attribute__((address_space(1))) int8_t *)(eb + lane_reg(elane));
#pragma unroll
    for (int b = 0; b < TL::B0; ++b) {
        const int j = t + b * Cfg::T;
        if ((TL::NB0 % Cfg::T) == 0 || j < TL::NB0) {
            const unsigned lr = lane_reg(lane);  // one copy for the group's loads
#pragma unroll
            for (int q = 0; q < TL::R0; ++q) {
                const long long u = ut + (long long)(b * Cfg::T + q * TL::NB0) * es;
                const typename St::Raw r = fetch_at<St, Cfg::kNT, false>(ib, u, lr);
                int ex = 0;
                if constexpr (St::kHalf && !kLineScaled<St, KIND>)
                    ex = *(const __attribute__((address_space(1))) int8_t *)(eb + ea3 * (b * Cfg::T + q * TL::NB0) +
                                                                              lane_reg(elane));
                if constexpr (TL::kRaw) {
                    tl.e[b][q] = r;
                    if constexpr (St::kHalf) tl.ex[b][q] = ex;
                } else if constexpr (kLineScaled<St, KIND>) {
                    tl.e[b][q] = maybe_swap<INV>(St::decode_raw(r));
                } else {
                    tl.e[b][q] = maybe_swap<INV>(St::decode(r, ex));
                }
            }
        }
    }
}

template <typename R>
__device__ __forceinline__ R uniform_r(R v) {
    if constexpr (sizeof(R) == 4) {
        return __builtin_bit_cast(R, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
    } else {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
        const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
        return __builtin_bit_cast(R, ((unsigned long long)hi << 32) | lo);
    }
}
template <typename R>
__device__ __forceinline__ cx<R> uniform_cx(cx<R> v) { return {uniform_r(v.x), uniform_r(v.y)}; }

// IO bit 0: the first stage reads its inputs from LDS (natural order)
// instead of the tile; bit 1: the last stage writes its outputs to LDS
// (natural order) instead of global memory.
constexpr int kFromLds = 1, kToLds = 2;

template <class Cfg, class St, int KIND, bool INV, int S, int IO = 0>
__device__ __forceinline__ void static_stage(const PassArgs &a, cx<typename St::R> *lds,
                                             const cx<typename St::R> *tws, unsigned *red, int t, int l,
                                             const TileCoord &c, unsigned lane, long long es,
                                             const Tile<Cfg, St> &tl, int &ex_out) {
    using R = typename St::R;
    constexpr int N = Cfg::plan.n;
    constexpr int T = Cfg::T;
    constexpr int L = Cfg::L;
    constexpr int LS = Cfg::kLineStride;
    constexpr int PAD = LS != N;
    constexpr int RAD = Cfg::plan.r[S];
    constexpr int Ns = ns_before(Cfg::plan, S);
    constexpr int NB = N / RAD;
    constexpr int B = (NB + T - 1) / T;
    constexpr bool kGuard = (NB % T) != 0;
    constexpr bool kLast = (S == Cfg::S - 1);
    constexpr int kTw = tw_offset(Cfg::plan, S);

    cx<R> v[B][RAD];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + b * T;
        if (!kGuard || j < NB) {
#pragma unroll
            for (int q = 0; q < RAD; ++q) {
                if constexpr (S == 0 && (IO & kFromLds)) {
                    v[b][q] = maybe_swap<INV>(lds[lds_index<KIND, LS, PAD>(l, j + q * NB, L)]);
                } else if constexpr (S == 0) {
                    if constexpr (Tile<Cfg, St>::kRaw && kLineScaled<St, KIND>)
                        v[b][q] = maybe_swap<INV>(St::decode_raw(tl.e[b][q]));
                    else if constexpr (Tile<Cfg, St>::kRaw)
                        v[b][q] = maybe_swap<INV>(St::decode(tl.e[b][q], St::kHalf ? tl.ex[b][q] : 0));
                    else
                        v[b][q] = tl.e[b][q];
                } else {
                    v[b][q] = lds[lds_index<KIND, LS, PAD>(l, j + q * NB, L)];
                }
            }
            if constexpr (Ns > 1) {
                const int k = j % Ns;
#pragma unroll
                for (int q = 1; q < RAD; ++q) {
                    cx<R> w = tws[kTw + (q - 1) * Ns + k];
                    // a wavefront of one tile position: the twiddle is the
                    // same in every lane and lives in scalar registers
                    if constexpr (KIND != kContiguous && L % 64 == 0) w = uniform_cx(w);
                    v[b][q] = cmul(v[b][q], w);
                }
            }
            Dft<RAD, R>::run(v[b]);
        }
        // keep the scheduler from hoisting the next butterfly's LDS loads
        // above this one: bounds the registers live in wide tiles
        if constexpr (B > 1) __builtin_amdgcn_sched_barrier(0);
    }

    if constexpr (kLast && (IO & kToLds)) {
        // outputs of the last stage in natural order (index j + q * NB) into LDS
        if constexpr (S > 0 || (IO & kFromLds)) stage_sync<Cfg::kWaveSync>();
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = t + b * T;
            if (!kGuard || j < NB) {
#pragma unroll
                for (int q = 0; q < RAD; ++q)
                    lds[lds_index<KIND, LS, PAD>(l, j + q * NB, L)] = maybe_swap<INV>(v[b][q]);
            }
        }
    } else if constexpr (kLast) {
        // outputs of the last stage: index j + q * NB (Ns * RAD == N)
        int ex = 0;
        if constexpr (St::kHalf) {
            float mx = 0.0f;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int j = t + b * T;
                if (!kGuard || j < NB) {
#pragma unroll
                    for (int q = 0; q < RAD; ++q) mx = fmaxf(mx, fmaxf(fabsf(v[b][q].x), fabsf(v[b][q].y)));
                }
            }
            float lmx;
            if constexpr (Cfg::kWaveSync) {
                // the line's T lanes are one aligned group of its wavefront
                lmx = __uint_as_float(lanes_max_u32<T>(__float_as_uint(mx)));
            } else {
                atomicMax(&red[l], __float_as_uint(mx));
                stage_sync<Cfg::kWaveSync>();
                lmx = __uint_as_float(red[l]);
            }
            ex = kLineScaled<St, KIND> ? line_exponent_scaled(lmx, tl.lex) : line_exponent(lmx);
            ex_out = ex;
            // unscaled values: store v 2^(lex - ex)
            if constexpr (kLineScaled<St, KIND>) ex -= tl.lex;
        }
        if (c.valid) {
            const long long ut = KIND == kContiguous ? 0 : c.tbase;
            gchar *const ob = uniform_gptr(a.out, (c.tbase - ut) * (long long)sizeof(typename St::Raw));
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int j = t + b * T;
                if (!kGuard || j < NB) {
                    const unsigned lr = lane_reg(lane);  // one copy for the group's stores
#pragma unroll
                    for (int q = 0; q < RAD; ++q) {
                        const long long u = ut + (long long)(b * T + q * NB) * es;
                        store_at<St, Cfg::kNT, false>(ob, u, lr, maybe_swap<INV>(v[b][q]), ex);
                    }
                }
            }
        }
    } else {
        if constexpr (S > 0 || (IO & kFromLds)) stage_sync<Cfg::kWaveSync>();
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = t + b * T;
            if (!kGuard || j < NB) {
                const int k = j % Ns;
                const int o0 = (j / Ns) * Ns * RAD + k;
#pragma unroll
                for (int q = 0; q < RAD; ++q) lds[lds_index<KIND, LS, PAD>(l, o0 + q * Ns, L)] = v[b][q];
            }
        }
        stage_sync<Cfg::kWaveSync>();
        static_stage<Cfg, St, KIND, INV, S + 1, IO>(a, lds, tws, red, t, l, c, lane, es, tl, ex_out);
    }
}

template <class Cfg>
__device__ __forceinline__ int tw_source(int i) {
    // entry i of the LDS twiddle table -> index into the length-N table
    constexpr RPlan p = Cfg::plan;
    int src = 0;
#pragma unroll
    for (int s = 1; s < kMaxStages; ++s) {
        if (s < p.S) {
            const int o = tw_offset(p, s), ns = ns_before(p, s), r = p.r[s];
            if (i >= o && i < o + (r - 1) * ns) {
                const int q = (i - o) / ns + 1, k = (i - o) % ns;
                src = q * k * (p.n / (ns * r));
            }
        }
    }
    return src;
}

// With one block per tile, workgroup b runs on XCD b mod 8 (the dispatcher
// deals workgroups to the 8 XCDs in turn); this order gives each XCD one
// contiguous run of tiles, so its L2 serves neighbouring row segments (a
// gain for the 4 KiB stride of a 512 y pass, a loss for the z pass).
__device__ __forceinline__ long long xcd_tile(long long b, long long n) {
    constexpr long long kXcds = 8;
    const long long per = n / kXcds, rem = n % kXcds, x = b % kXcds, i = b / kXcds;
    return x * per + (x < rem ? x : rem) + i;
}

template <class Cfg, class St, int KIND, bool INV>
__global__ void __launch_bounds__(Cfg::kBlock) fft_static(const PassArgs a) {
    using R = typename St::R;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int T = Cfg::T;
    constexpr int L = Cfg::L;
    cx<R> *lds = reinterpret_cast<cx<R> *>(smem);
    cx<R> *tws = reinterpret_cast<cx<R> *>(smem + Cfg::kLdsData);
    unsigned *red = reinterpret_cast<unsigned *>(smem + Cfg::kLdsData + (size_t)Cfg::kTwN * sizeof(cx<R>));
    const int tid = threadIdx.x;
    const int l = KIND == kContiguous ? tid / T : tid % L;
    // with whole wavefronts of lines, t is the wavefront's index: uniform
    const int t = KIND == kContiguous ? tid % T
                  : (L % 64 == 0 ? (int)__builtin_amdgcn_readfirstlane((unsigned)(tid / L)) : tid / L);

    if constexpr (Cfg::kTwN > 0) {
        const cx<R> *W = reinterpret_cast<const cx<R> *>(a.tw);
        for (int i = tid; i < Cfg::kTwN; i += Cfg::kBlock) tws[i] = W[tw_source<Cfg>(i)];
        __syncthreads();
    }

    long long tile = blockIdx.x;
    if (tile >= a.total) return;
    const long long G = gridDim.x;
    if constexpr (Cfg::kXO) {
        if (G == a.total) tile = xcd_tile(tile, a.total);
    }
    const long long es = KIND == kContiguous ? 1 : a.es;
    // tile -> (tx, w), advanced incrementally by G tiles per iteration
    long long tx, w, gx = G, gw = 0;
    if constexpr (KIND == kContiguous) {
        tx = tile;
        w = 0;
    } else {
        tx = tile % a.ntiles;
        w = tile / a.ntiles;
        gx = G % a.ntiles;
        gw = G / a.ntiles;
    }
    Tile<Cfg, St> cur;
    TileCoord c = tile_coord<Cfg, KIND>(a, tx, w, l);
    const unsigned lane = lane_offset<Cfg, St, KIND>(l, t, es);
    if constexpr (Cfg::kPrefetch) fetch_tile<Cfg, St, KIND, INV>(a, c, t, lane, es, cur);
    for (;;) {
        const long long nt = tile + G;
        const bool more = nt < a.total;
        long long ntx = tx + gx, nw = w + gw;
        if (KIND != kContiguous && ntx >= a.ntiles) {
            ntx -= a.ntiles;
            nw += 1;
        }
        const TileCoord nc = tile_coord<Cfg, KIND>(a, ntx, nw, l);
        Tile<Cfg, St> nxt;
        if constexpr (Cfg::kPrefetch) {
            if (more) fetch_tile<Cfg, St, KIND, INV>(a, nc, t, lane, es, nxt);
        } else {
            fetch_tile<Cfg, St, KIND, INV>(a, c, t, lane, es, cur);
        }

        int ex = 0;
        if constexpr (St::kHalf && !Cfg::kWaveSync) {
            if (t == 0) red[l] = 0u;
            stage_sync<Cfg::kWaveSync>();
        }
        static_stage<Cfg, St, KIND, INV, 0>(a, lds, tws, red, t, l, c, lane, es, cur, ex);
        if constexpr (St::kHalf) {
            if (c.valid && t == 0 && a.out_exp) {
                const ExpMap &m = a.em;
                a.out_exp[exp_line_index(m, c.q, c.w, m.b0, m.b1, m.b2)] = (int8_t)ex;
            }
        }
        if (!more) break;
        // the next tile overwrites LDS that this one read last
        stage_sync<Cfg::kWaveSync>();
        if constexpr (Cfg::kPrefetch) cur = nxt;
        c = nc;
        tile = nt;
        tx = ntx;
        w = nw;
    }
}

// ------------------------------------------------- lane-per-line strided pass
// A strided pass of length N = 64 TPL (radices 8, 8, TPL: 512 and 1024) with
// one line per lane: a tile of L = BLOCK / TPL neighbouring lines (BLOCK =
// 512 threads, or 256 at 512; each tile position an L-element row segment:
// 256 bytes for 4-byte storage at 512 and for 8-byte storage at 1024 or in
// 256-thread blocks), thread t (of TPL per line) holding positions
// t + TPL m, m < 64, of its line.  It runs the three Stockham stages of the
// other kernels butterfly for butterfly, with the same twiddles and the same
// operations, so its results are bit-identical to theirs; but the first two
// stages stay in registers.  Stage-0 butterflies j = t + TPL a (a < 8) read
// positions j + (N/8) q, all the thread's own, and write outputs 8j + p;
// stage-1 butterfly 8t + r reads outputs 8t + r + (N/8) q of stage 0, i.e.
// output r of butterfly t + TPL q: the same thread again.  Stage-1 butterfly
// 8t + r writes 64t + r + 8p; stage 2 (butterflies j < 64, reading j + 64q,
// q < TPL) needs one element from every thread of the line, so there is one
// exchange through LDS, made as real parts then imaginary parts through an
// area of N L floats (128 KiB in 512-thread blocks); thread t takes
// butterflies (64/TPL) t + u.  With 64-line tiles a wavefront is one t:
// positions, twiddle indices and the tile origin are uniform, so addresses
// are a scalar base plus the lane's offset; with 32-line tiles the two
// halves of a wavefront are t and t + 1.  A 256-thread block at 512
// (32-line tiles, 256-byte rows of complex64, a 64 KiB exchange area) lets
// two blocks share a CU, each overlapping its loads with the other's stages.
constexpr int kLanesBlock = 512;

// A zero the compiler cannot see through, made once per tile.  Added to the
// twiddle indices and to the strides, it keeps the twiddle reads and the
// 64-bit offsets of the tile's 128 accesses in the tile loop: hoisted out
// of it as loop invariants, they would stay live across the whole loop,
// more than the scalar registers hold, and spill.
__device__ __forceinline__ int opaque_zero() {
    int z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}
template <int N, class St, int BLOCK = kLanesBlock>
struct LanesCfg {
    using R = typename St::R;
    static constexpr int TPL = N / 64;              // threads per line
    static constexpr int L = BLOCK / TPL;           // lines per tile
    static constexpr int NB2 = 64 / TPL;            // stage-2 butterflies per thread
    static constexpr size_t kX = (size_t)N * L * sizeof(R);              // one component of the tile
    static constexpr size_t kTw = kX;                                    // w_N^m, m < N
    static constexpr size_t kRed = kTw + (size_t)N * sizeof(cx<R>);      // [TPL][L] line maxima
    static constexpr size_t kBytes = kRed + (size_t)TPL * L * sizeof(unsigned);
    static constexpr RPlan plan = make_rplan(N);
    static_assert(plan.S == 3 && plan.r[0] == 8 && plan.r[1] == 8 && plan.r[2] == TPL, "radices 8, 8, N/64");
    static_assert(L == 32 || L == 64, "a tile is one or two lines per wavefront lane group");
};


// NTM: the non-temporal hint on the loads (bit 0) and on the stores (bit 1).
// REV: with one block per tile, the tiles in reverse order (the pass starts
// where the previous pass, run forward, stopped writing).
// PF (persistent grids of whole tiles, es a multiple of L): the stored rows
// of positions 0 .. N/2 - 1 of the block's next tile are copied into the
// exchange area (global_load_lds, 16 bytes a lane, no registers held) as
// soon as the current tile's exchange is done, before its stores; they
// arrive during the last stage and the stores, and the next tile loads
// only its other half from global memory.  Issued before the stores, they
// complete before them (vector memory counts in order), so waiting for
// them leaves the stores in flight: 64 stores per lane follow them, and a
// wait for at most 62 outstanding operations covers the copy.
// RP (16-bit storage): the block loads its next tile into registers (64
// registers of 16-bit pairs) during the current one: the first half as soon
// as the current tile is decoded, the second after the exchange (a wave
// holds at most 63 vector memory operations, and after the decode the
// previous tile's stores still hold many of them), so they are in flight
// during the butterflies, the exchange and the stores.  No address the
// tile loop could hoist stays live across it (the exchange and line-maximum
// addresses are made each tile): with the prefetched registers it would
// spill, and each reload would wait for every load in flight.  The input
// exponents sit packed four to a register; they are
// loaded once per block where every tile of the block reads the same ones
// (whole tiles, the exponent index independent of the plane, and the
// block's line stride a multiple of the index period: the 512^3 z pass),
// else once per tile.
template <int N, class St, bool INV, int NTM, int BLOCK = kLanesBlock, bool XO = false, bool REV = false,
          bool PF = false, bool RP = false>
__global__ void __launch_bounds__(BLOCK) fft_lanes(const PassArgs a) {
    using R = typename St::R;
    using C = LanesCfg<N, St, BLOCK>;
    static_assert(sizeof(R) == 4, "FP32 compute: 64 elements per thread in registers");
    static_assert(!RP || (St::kHalf && !PF), "register prefetch: 16-bit storage, no LDS copy");
    constexpr int TPL = C::TPL, L = C::L, NB2 = C::NB2;
    constexpr bool kUniform = L == 64;  // a wavefront is one t
    extern __shared__ __align__(16) unsigned char smem[];
    R *xl = reinterpret_cast<R *>(smem);
    cx<R> *tws = reinterpret_cast<cx<R> *>(smem + C::kTw);
    unsigned *red = reinterpret_cast<unsigned *>(smem + C::kRed);
    const int tid = threadIdx.x;
    const int l = tid % L;
    // t = t0 + h: t0 uniform in the wavefront, h the half (0 when L = 64)
    const int t0 = (int)__builtin_amdgcn_readfirstlane((unsigned)((tid >> 6) * (64 / L)));
    const int h = kUniform ? 0 : (tid >> 5) & 1;
    const int t = t0 + h;
    {
        const cx<R> *W = reinterpret_cast<const cx<R> *>(a.tw);
        for (int i = tid; i < N; i += BLOCK) tws[i] = W[i];
        __syncthreads();
    }
    long long tile = blockIdx.x;
    if (tile >= a.total) return;
    const long long G = gridDim.x;
    if (XO && G == a.total) tile = xcd_tile(tile, a.total);
    if (REV && G == a.total) tile = a.total - 1 - tile;
    const long long es = a.es;
    long long tx = tile % a.ntiles, w = tile / a.ntiles;
    const long long gx = G % a.ntiles, gw = G / a.ntiles;
    // the lane's part of an element offset: its line, and its half's share of
    // the position (h for the loads, NB2 h for the stores)
    const unsigned lane_b = (unsigned)(((long long)l + h * es) * (long long)sizeof(typename St::Raw));
    const unsigned lane_s = (unsigned)(((long long)l + (long long)NB2 * h * es) * (long long)sizeof(typename St::Raw));
    using Raw = typename St::Raw;
    constexpr int kS = (int)sizeof(Raw);
    // rows 0 .. N/2 - 1 of tile (ctx, cw) into the exchange area: row p at
    // byte (p L + line) kS; a wave instruction moves 1 KiB (16 bytes a lane)
    auto copy_half = [&](long long ctx, long long cw) {
        constexpr int kRowB = L * kS;
        static_assert(kRowB >= 16 && 1024 % kRowB == 0, "whole rows per 1 KiB copy");
        constexpr int kRowsPerI = 1024 / kRowB, kLanesPerRow = 64 / kRowsPerI, kInstr = (N / 2) / kRowsPerI;
        const int lane = tid & 63;
        const int wave = (int)__builtin_amdgcn_readfirstlane((unsigned)(tid >> 6));
        const char *gb = reinterpret_cast<const char *>(a.in) + (ctx * L + cw * es * N) * (long long)kS;
        const long long rowb = es * (long long)kS;
        const int rr = lane / kLanesPerRow, cb = (lane % kLanesPerRow) * 16;
        for (int k = wave; k < kInstr; k += BLOCK / 64) {
            const char *src = gb + (long long)(k * kRowsPerI + rr) * rowb + cb;
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                             (__attribute__((address_space(3))) void *)(smem + (size_t)k * 1024), 16,
                                             0, 0);
        }
    };
    static_assert(!PF || (size_t)(N / 2) * L * kS <= C::kX, "the copied half fits the exchange area");
    // RP: the raw values of the next tile, and the packed input exponents
    Raw rawn[RP ? 64 : 1];
    unsigned epk[RP ? 16 : 1];
    // positions t + TPL m, m0 <= m < m1, of tile (ctx, cw)
    auto issue_loads = [&](long long ctx, long long cw, int tzz, int m0, int m1) {
        if (ctx * L + l < es) {
            gchar *const nb = uniform_gptr(a.in, (ctx * L + cw * es * N) * (long long)kS);
            const long long est = es + tzz;
#pragma unroll
            for (int m = 0; m < 64; ++m)
                if (m >= m0 && m < m1)
                    rawn[m] = fetch_at<St, (NTM & 1) != 0>(nb, (t0 + tzz + (long long)TPL * m) * est, lane_b);
        }
    };
    auto load_exponents = [&](long long ctx, long long cw, int tzz) {
#pragma unroll
        for (int k = 0; k < (RP ? 16 : 1); ++k) epk[k] = 0;
        const long long cq = ctx * L + l;
        if (a.in_exp && cq < es) {
            const ExpMap &m = a.em;
            const unsigned el = exp_line_index(m, cq, cw, m.a0, m.a1, m.a2) + (unsigned)m.a3 * (unsigned)h;
            gchar *const eb = uniform_gptr(a.in_exp, 0);
            const long long ea3t = m.a3 + tzz;
            // every byte load in flight before the first is packed
            unsigned bt[RP ? 64 : 1];
#pragma unroll
            for (int mm = 0; mm < (RP ? 64 : 0); ++mm)
                bt[mm] = *(const __attribute__((address_space(1))) uint8_t *)(
                    eb + ea3t * (t0 + tzz + (long long)TPL * mm) + lane_reg(el));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int mm = 0; mm < (RP ? 64 : 0); ++mm) epk[mm >> 2] |= bt[mm] << (8 * (mm & 3));
        }
    };
    bool ehoist = true;  // RP: every tile of the block reads the same exponents
    if constexpr (RP) {
        const ExpMap &m = a.em;
        const bool qinv = m.a0 == 0 || ((gx * L) % m.qmod == 0 && (a.ntiles * L) % m.qmod == 0);
        ehoist = G >= a.total || !a.in_exp ||
                 (es % L == 0 && m.a1 == 0 && qinv && (m.a2 == 0 || a.total == a.ntiles));
        issue_loads(tx, w, opaque_zero(), 0, 64);
        load_exponents(tx, w, opaque_zero());
    }
    bool first = true;
    if constexpr (PF) copy_half(tx, w);
    for (;;) {
        const int tz = opaque_zero();
        const long long q = tx * L + l;  // this lane's line
        const bool valid = q < es;
        const long long tbase = tx * L + w * es * N;
        // the block's next tile
        const long long nt = tile + G;
        long long ntx = tx + gx, nw = w + gw;
        if (ntx >= a.ntiles) {
            ntx -= a.ntiles;
            nw += 1;
        }
        if constexpr (PF) {
            // this wave's copy of the tile's first half is done (the first
            // tile: nothing else in flight; later: the previous tile's 64
            // stores per lane followed it), then every wave's
            if (first) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
            else __builtin_amdgcn_s_waitcnt(0xCF7E);        // vmcnt(62)
            first = false;
            __syncthreads();
        }
        cx<R> v[64];
        if constexpr (RP) {
            if (valid) {
#pragma unroll
                for (int m = 0; m < 64; ++m)
                    v[m] = maybe_swap<INV>(St::decode(rawn[m], (int)(int8_t)(epk[m >> 2] >> (8 * (m & 3)))));
            } else {
#pragma unroll
                for (int m = 0; m < 64; ++m) v[m] = {R(0), R(0)};
            }
            // the next tile's first half now, its second half after the
            // exchange: a wave holds at most 63 vector memory operations,
            // and the previous tile's stores are still in flight here
            if (nt < a.total) issue_loads(ntx, nw, tz, 0, 32);
            __builtin_amdgcn_sched_barrier(0);
        } else if (valid) {
            unsigned elane = 0;
            long long ea3 = 0;
            const int8_t *ep = &kZeroExponent;
            if constexpr (St::kHalf) {
                if (a.in_exp) {
                    const ExpMap &m = a.em;
                    ep = a.in_exp;
                    ea3 = m.a3;
                    elane = exp_line_index(m, q, w, m.a0, m.a1, m.a2) + (unsigned)ea3 * (unsigned)h;
                }
            }
            // every load in flight before the first decode
            typename St::Raw raw[64];
            int ex[St::kHalf ? 64 : 1];
            gchar *const ib = uniform_gptr(a.in, tbase * (long long)sizeof(typename St::Raw));
            gchar *const eb = uniform_gptr(ep, 0);
            const long long est = es + tz, ea3t = ea3 + tz;
#pragma unroll
            for (int m = 0; m < 64; ++m) {
                const long long pos0 = t0 + tz + TPL * m;  // uniform part of the position
                if (!PF || m >= 32)
                    raw[m] = fetch_at<St, (NTM & 1) != 0>(ib, pos0 * est, lane_b);
                if constexpr (St::kHalf)
                    ex[m] = *(const __attribute__((address_space(1))) int8_t *)(eb + ea3t * pos0 + lane_reg(elane));
            }
            if constexpr (PF) {
                // positions t + TPL m, m < 32, from the copy in the exchange area
                const Raw *xr = reinterpret_cast<const Raw *>(smem);
#pragma unroll
                for (int m = 0; m < 32; ++m) raw[m] = xr[(t + TPL * m) * L + l];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < 64; ++m) v[m] = maybe_swap<INV>(St::decode(raw[m], St::kHalf ? ex[m] : 0));
        } else {
#pragma unroll
            for (int m = 0; m < 64; ++m) v[m] = {R(0), R(0)};
        }
        // stage 0: butterfly t + TPL a on v[a + 8p] (positions t + TPL (a + 8p)); output p to v[a + 8p]
#pragma unroll
        for (int aa = 0; aa < 8; ++aa) {
            cx<R> u8[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) u8[p] = v[aa + 8 * p];
            Dft<8, R>::run(u8);
#pragma unroll
            for (int p = 0; p < 8; ++p) v[aa + 8 * p] = u8[p];
        }
        // stage 1: butterfly 8t + r on v[8r + p] (output r of stage-0
        // butterfly t + TPL p), twiddles w_N^(p r N / 64)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            cx<R> u8[8];
            u8[0] = v[8 * r];
#pragma unroll
            for (int p = 1; p < 8; ++p) u8[p] = cmul(v[8 * r + p], tws[p * r * (N / 64) + tz]);
            Dft<8, R>::run(u8);
#pragma unroll
            for (int p = 0; p < 8; ++p) v[8 * r + p] = u8[p];
        }
        // exchange: v[8r + p] is element 64t + r + 8p; stage-2 butterfly
        // NB2 t + u reads elements NB2 t + u + 64p into y[TPL u + p]
        cx<R> y[64];
#pragma unroll
        for (int part = 0; part < 2; ++part) {
            __syncthreads();  // the previous readers of the area are done
            // RP: the exchange addresses are made here, each tile, rather
            // than hoisted out of the tile loop, where with the prefetched
            // registers they would spill
            const int tzx = (RP || N == 1024) ? opaque_zero() : 0;
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int p = 0; p < 8; ++p)
                    xl[(64 * t + r + 8 * p) * L + l + tzx] = part ? v[8 * r + p].y : v[8 * r + p].x;
            __syncthreads();
#pragma unroll
            for (int u = 0; u < NB2; ++u)
#pragma unroll
                for (int p = 0; p < TPL; ++p) {
                    const R e = xl[(NB2 * t + u + 64 * p) * L + l + tzx];
                    if (part) y[TPL * u + p].y = e;
                    else y[TPL * u + p].x = e;
                }
        }
        if constexpr (RP) {
            if (nt < a.total) {
                __builtin_amdgcn_sched_barrier(0);
                issue_loads(ntx, nw, opaque_zero(), 32, 64);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if constexpr (PF) {
            if (nt < a.total) {
                __syncthreads();  // every wave has read its exchange values
                __builtin_amdgcn_sched_barrier(0);
                copy_half(ntx, nw);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // stage 2: butterfly j = NB2 t + u, twiddles w_N^(p j); outputs j + 64p
        float mx = 0.0f;
#pragma unroll
        for (int u = 0; u < NB2; ++u) {
            const int j = NB2 * t + u;
            cx<R> uu[TPL];
            uu[0] = y[TPL * u];
#pragma unroll
            for (int p = 1; p < TPL; ++p) {
                uu[p] = cmul(y[TPL * u + p], tws[p * j + tz]);
            }
            Dft<TPL, R>::run(uu);
#pragma unroll
            for (int p = 0; p < TPL; ++p) {
                y[TPL * u + p] = uu[p];
                if constexpr (St::kHalf) mx = fmaxf(mx, fmaxf(fabsf(uu[p].x), fabsf(uu[p].y)));
            }
        }
        int ex = 0;
        if constexpr (St::kHalf) {
            // the line's maximum over its TPL threads (RP: addresses made
            // each tile, as for the exchange)
            const int tzr = RP ? opaque_zero() : 0;
            red[t * L + l + tzr] = __float_as_uint(mx);
            __syncthreads();
            unsigned mb = red[l + tzr];
#pragma unroll
            for (int k = 1; k < TPL; ++k) mb = max(mb, red[k * L + l + tzr]);
            ex = line_exponent(__uint_as_float(mb));
        }
        if (valid) {
            gchar *const ob = uniform_gptr(a.out, tbase * (long long)sizeof(typename St::Raw));
            const long long est = es + tz;
            // one copy of the lane offset for the tile's stores, where the
            // kernel has a register to spare for it (not at 256 VGPRs: the
            // register prefetch and length 1024 copy it at each store)
            constexpr bool kShare = N == 512 && !RP;
            const unsigned ls = kShare ? lane_reg(lane_s) : lane_s;
#pragma unroll
            for (int u = 0; u < NB2; ++u)
#pragma unroll
                for (int p = 0; p < TPL; ++p) {
                    // position NB2 t + u + 64 p: NB2 t0 + u + 64 p uniform, NB2 h in lane_s
                    const long long pos = (long long)NB2 * (t0 + tz) + u + 64 * p;
                    store_at<St, (NTM & 2) != 0, !kShare>(ob, pos * est, ls, maybe_swap<INV>(y[TPL * u + p]), ex);
                }
            if constexpr (St::kHalf) {
                if (t == 0 && a.out_exp) {
                    const ExpMap &m = a.em;
                    a.out_exp[exp_line_index(m, q, w, m.b0, m.b1, m.b2)] = (int8_t)ex;
                }
            }
        }
        if constexpr (RP) {
            if (!ehoist && nt < a.total) load_exponents(ntx, nw, tz);
        }
        tile = nt;
        if (tile >= a.total) break;
        tx = ntx;
        w = nw;
    }
}

// ------------------------------------------------------------ real transforms
// The x pass of a real-to-complex (forward) or complex-to-real (backward)
// transform of real lines of even length N = 2M.  A real line is read (or
// written) as the complex line z[n] = x[2n] + i x[2n+1] of length M, whose
// M-point FFT runs through LDS as in the complex passes.  Forward, the
// half spectrum follows from Z = DFT_M(z) as
//   X[k] = (A + B)/2 - i w^k (A - B)/2,  A = Z[k mod M], B = conj Z[(M-k) mod M],
// for k = 0..M, w = exp(-2 pi i/N).  Backward, the unnormalised inverse of the
// half spectrum X[0..M] starts from
//   Z'[k] = (A + B) + i conj(w^k) (A - B),  A = X[k], B = conj X[M-k],  k < M,
// whose unnormalised M-point inverse is N (x[2n] + i x[2n+1]).  The imaginary
// parts of X[0] and X[M] are dropped (they vanish for the spectrum of a real
// line), which makes the backward result the real inverse of the Hermitian
// extension of any half spectrum.
// Lines: l = y + ny z; real lines are M complex apart, spectra M + 1.
// A tile's L lines are consecutive, so its spectra form one contiguous range
// of L (M + 1) elements: the split (forward) and the merge (backward) walk
// that range with the whole block, giving coalesced global accesses whatever
// M + 1 is.  LDS: the tile's lines (M per line; the kx = M terms of the
// backward input in a side column), the stage twiddles, and w_N^k, k <= M.
// (Lengths whose table would not fit read w_N^k from global memory.)
template <class Cfg, class CB>
struct RealLds {
    static constexpr int M = Cfg::plan.n;
    static constexpr size_t kW2 = Cfg::kLdsData + (size_t)Cfg::kTwN * CB::value;
    static constexpr bool kW2InLds =
        kW2 + (size_t)(M + 1 + Cfg::L) * CB::value <= (size_t)160 * 1024;
    static constexpr size_t kNyq = kW2 + (kW2InLds ? (size_t)(M + 1) * CB::value : 0);
    static constexpr size_t kBytes = kNyq + (size_t)Cfg::L * CB::value;
};

template <class Cfg, class St, bool INV>
__global__ void __launch_bounds__(Cfg::kBlock) fft_real_x(const PassArgs a) {
    using R = typename St::R;
    using Lay = RealLds<Cfg, std::integral_constant<int, (int)sizeof(cx<R>)>>;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int M = Cfg::plan.n;
    constexpr int H = M + 1;
    constexpr int T = Cfg::T;
    constexpr int L = Cfg::L;
    constexpr int LS = Cfg::kLineStride;
    constexpr int PAD = LS != M;
    cx<R> *lds = reinterpret_cast<cx<R> *>(smem);
    cx<R> *tws = reinterpret_cast<cx<R> *>(smem + Cfg::kLdsData);
    cx<R> *w2s = reinterpret_cast<cx<R> *>(smem + Lay::kW2);
    cx<R> *nyq = reinterpret_cast<cx<R> *>(smem + Lay::kNyq);
    const cx<R> *W2 = reinterpret_cast<const cx<R> *>(a.tw2);
    auto w2 = [&](int k) -> cx<R> {
        if constexpr (Lay::kW2InLds) return w2s[k];
        else return W2[k];
    };
    unsigned *red = nullptr;
    const int tid = threadIdx.x;
    const int l = tid / T;
    const int t = tid % T;
    {
        const cx<R> *W = reinterpret_cast<const cx<R> *>(a.tw);
        for (int i = tid; i < Cfg::kTwN; i += Cfg::kBlock) tws[i] = W[tw_source<Cfg>(i)];
        if constexpr (Lay::kW2InLds)
            for (int i = tid; i <= M; i += Cfg::kBlock) w2s[i] = W2[i];
        __syncthreads();
    }
    auto at = [&](int line, int k) -> cx<R> & { return lds[lds_index<kContiguous, LS, PAD>(line, k, L)]; };
    const unsigned lane = lane_offset<Cfg, St, kContiguous>(l, t, 1);
    for (long long tile = blockIdx.x; tile < a.total; tile += gridDim.x) {
        const TileCoord c = tile_coord<Cfg, kContiguous>(a, tile, 0, l);
        const long long q0 = tile * L;
        const int nl = (int)(a.nlines - q0 < L ? a.nlines - q0 : L);  // lines in this tile
        int ex = 0;
        if constexpr (!INV) {
            Tile<Cfg, St> cur;
            fetch_tile<Cfg, St, kContiguous, false>(a, c, t, lane, 1, cur);
            static_stage<Cfg, St, kContiguous, false, 0, kToLds>(a, lds, tws, red, t, l, c, lane, 1, cur, ex);
            __syncthreads();
            cx<R> *out = reinterpret_cast<cx<R> *>(a.out) + q0 * H;
#pragma unroll 1
            for (int i = tid; i < nl * H; i += Cfg::kBlock) {
                const int ln = i / H, k = i - ln * H;
                const cx<R> A = at(ln, k == M ? 0 : k);
                const cx<R> Bc = at(ln, k == 0 ? 0 : M - k);
                const cx<R> B = {Bc.x, -Bc.y};
                const cx<R> s = {(A.x + B.x) * R(0.5), (A.y + B.y) * R(0.5)};
                const cx<R> d = {(A.x - B.x) * R(0.5), (A.y - B.y) * R(0.5)};
                const cx<R> wd = cmul(w2(k), d);                         // w^k (A - B)/2
                const cx<R> z = {s.x + wd.y, s.y - wd.x};                // s - i wd
                if constexpr (Cfg::kNT)
                    __builtin_nontemporal_store(St::pack(z, 0), reinterpret_cast<typename St::Raw *>(out) + i);
                else
                    St::store(out, i, z, 0);
            }
        } else {
            const cx<R> *X = reinterpret_cast<const cx<R> *>(a.in) + q0 * H;
            auto load_x = [&](int i) -> cx<R> {
                if constexpr (Cfg::kNT)
                    return St::decode(__builtin_nontemporal_load(reinterpret_cast<const typename St::Raw *>(X) + i), 0);
                else
                    return X[i];
            };
            // the tile's spectra into LDS, every load of a thread in flight
            // before its first LDS store where that takes at most 16 values
            constexpr int kIter = (L * H + Cfg::kBlock - 1) / Cfg::kBlock;
            if constexpr (kIter <= 16) {
                cx<R> v[kIter];
#pragma unroll
                for (int it = 0; it < kIter; ++it) {
                    const int i = tid + it * Cfg::kBlock;
                    if (i < nl * H) v[it] = load_x(i);
                }
#pragma unroll
                for (int it = 0; it < kIter; ++it) {
                    const int i = tid + it * Cfg::kBlock;
                    if (i < nl * H) {
                        const int ln = i / H, k = i - ln * H;
                        if (k < M) at(ln, k) = v[it];
                        else nyq[ln] = v[it];
                    }
                }
            } else {
#pragma unroll 1
                for (int i = tid; i < nl * H; i += Cfg::kBlock) {
                    const int ln = i / H, k = i - ln * H;
                    const cx<R> v = load_x(i);
                    if (k < M) at(ln, k) = v;
                    else nyq[ln] = v;
                }
            }
            __syncthreads();
            // pairs (k, M - k), 0 <= k <= M/2, merged in place; k = 0 pairs with X[M]
            constexpr int P = M / 2 + 1;
#pragma unroll 1
            for (int i = tid; i < nl * P; i += Cfg::kBlock) {
                const int ln = i / P, k = i - ln * P;
                const int r = M - k;
                const cx<R> xk = at(ln, k);
                const cx<R> xr = k == 0 ? nyq[ln] : at(ln, r);
                // Z'[k] = (A + B) + i conj(w^k) (A - B), A = X[k], B = conj X[M-k];
                // only the real parts of X[0] and X[M] enter
                cx<R> A = xk, B = {xr.x, -xr.y};
                if (k == 0) A.y = B.y = R(0);
                const cx<R> wk = w2(k);
                const cx<R> dk = cmul(cx<R>{A.x - B.x, A.y - B.y}, cx<R>{wk.x, -wk.y});
                at(ln, k) = cx<R>{A.x + B.x - dk.y, A.y + B.y + dk.x};
                if (k != 0 && r != k) {
                    // the partner: A = X[M-k], B = conj X[k]
                    const cx<R> A2 = xr, B2 = {xk.x, -xk.y};
                    const cx<R> wr = w2(r);
                    const cx<R> dr = cmul(cx<R>{A2.x - B2.x, A2.y - B2.y}, cx<R>{wr.x, -wr.y});
                    at(ln, r) = cx<R>{A2.x + B2.x - dr.y, A2.y + B2.y + dr.x};
                }
            }
            __syncthreads();
            Tile<Cfg, St> none;
            static_stage<Cfg, St, kContiguous, true, 0, kFromLds>(a, lds, tws, red, t, l, c, lane, 1, none, ex);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ fused multiply
// The reciprocal-space step of a PME-style convolution on the half spectrum,
// in one pass along z (strided lines, in place): forward FFT of each z-line,
// multiplication of every element by the real multiplier G (same layout as
// the spectrum), inverse FFT, store.  The tile stays in LDS between the two
// transforms.  Each block also sums w(kx) G |Q|^2 over the elements it
// multiplied (Q the full 3D spectrum at that point; w = 1 for kx = 0 and
// kx = nx/2, else 2, which counts the mirrored half) in FP64 and writes one
// partial per block.
template <class Cfg, class St>
__global__ void __launch_bounds__(Cfg::kBlock) fft_conv_z(const PassArgs a) {
    using R = typename St::R;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int N = Cfg::plan.n;
    constexpr int L = Cfg::L;
    constexpr int B = Cfg::kBlock;
    static_assert(B % L == 0, "a thread keeps its line across the multiply loop");
    cx<R> *lds = reinterpret_cast<cx<R> *>(smem);
    cx<R> *tws = reinterpret_cast<cx<R> *>(smem + Cfg::kLdsData);
    double *sum = reinterpret_cast<double *>(smem);  // reuses the tile area after the last tile
    unsigned *red = nullptr;
    const int tid = threadIdx.x;
    const int l = tid % L;
    const int t = tid / L;
    if constexpr (Cfg::kTwN > 0) {
        const cx<R> *W = reinterpret_cast<const cx<R> *>(a.tw);
        for (int i = tid; i < Cfg::kTwN; i += B) tws[i] = W[tw_source<Cfg>(i)];
        __syncthreads();
    }
    const R *G = reinterpret_cast<const R *>(a.mul);
    const long long es = a.es;
    const unsigned lane = lane_offset<Cfg, St, kStrided>(l, t, es);
    double acc = 0.0;
    for (long long tile = blockIdx.x; tile < a.total; tile += gridDim.x) {
        const long long tx = tile % a.ntiles, w = tile / a.ntiles;
        const TileCoord c = tile_coord<Cfg, kStrided>(a, tx, w, l);
        int ex = 0;
        Tile<Cfg, St> cur;
        fetch_tile<Cfg, St, kStrided, false>(a, c, t, lane, es, cur);
        // the multiplier of this thread's elements (e = t + k T); with few
        // elements per thread it is loaded now, so that the loads are in
        // flight during the forward stages (wide tiles load it afterwards, as
        // holding it across the stages would spill)
        constexpr int T = B / L;
        constexpr int E = (N + T - 1) / T;
        constexpr bool kEarly = E <= 8;
        const R *g = G + c.tbase + l;
        R gv[E];
        if (kEarly && c.valid) {
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int e = t + k * T;
                gv[k] = e < N ? g[(long long)e * es] : R(0);
            }
        }
        static_stage<Cfg, St, kStrided, false, 0, kToLds>(a, lds, tws, red, t, l, c, lane, es, cur, ex);
        __syncthreads();
        if (c.valid) {
            // element (line l, position e) sits at LDS index e L + l
            const long long kx = c.q % a.hx;
            const double wgt = (kx == 0 || kx == a.hx - 1) ? 1.0 : 2.0;
            if (!kEarly) {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int e = t + k * T;
                    gv[k] = e < N ? g[(long long)e * es] : R(0);
                }
            }
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int e = t + k * T;
                if (e < N) {
                    cx<R> &v = lds[e * L + l];
                    const double m2 = (double)v.x * v.x + (double)v.y * v.y;
                    acc = fma(wgt * (double)gv[k], m2, acc);
                    v = cx<R>{v.x * gv[k], v.y * gv[k]};
                }
            }
        }
        __syncthreads();
        Tile<Cfg, St> none;
        static_stage<Cfg, St, kStrided, true, 0, kFromLds>(a, lds, tws, red, t, l, c, lane, es, none, ex);
        __syncthreads();
    }
    // block sum in a fixed order: thread i's value, then a tree over the block
    sum[tid] = acc;
    __syncthreads();
    for (int h = 1; h < B; h *= 2) {
        if ((tid & (2 * h - 1)) == 0 && tid + h < B) sum[tid] += sum[tid + h];
        __syncthreads();
    }
    if (tid == 0) a.partial[blockIdx.x] = sum[0];
}

// ------------------------------------------------------------ batched form
// One launch runs one pass of many grids of uneven sizes (or, cooperatively,
// all passes): a block takes one tile of one (grid, pass) segment, found by
// binary search over the segments' first tiles.  Every length uses 256 threads per block (T = 4 or 8 threads
// per line, 256 / T lines per tile), so one kernel serves all of them; the
// arithmetic per butterfly is the same as in the single-grid kernels.
struct BatchItem {
    long long offset;      // element offset of the grid in the packed buffers
    long long tile_begin;  // first tile of this segment within the launch
    long long es, nlines, nw, ntiles, total;
    const void *tw;        // twiddle table of the segment's length
    int code;              // compiled (length, kind, shape), see batch_code
    int from_in;           // 1: the segment reads the `in` buffer (the grid's first pass)
};

struct BatchArgs {
    const BatchItem *items;
    int nitems;
    const void *in;
    void *out;
};

// One launch over all passes of all grids: the blocks loop over the tiles of
// pass 0 (block b takes tiles b, b + G, ...), meet at a grid-wide barrier,
// loop over the tiles of pass 1, meet again, then pass 2.  The launch is
// cooperative (every block resident), and every block reaches both
// barriers, so the barrier cannot wait on a block that is not running.
// Measured on an MI355X (768 resident blocks): a cooperative launch costs
// about 20 us against a few for a plain one, and a grid-wide barrier 60 to
// 100 us (the runtime's) or about 80 us (an arrival counter polled by each
// block), against a few us between two launches replayed from a graph; so
// the per-pass launches in a graph stay the faster form.  Handing tiles out
// from a counter instead of striding was slower still (one contended atomic
// per tile).  The thread index reaches the tile code through a per-tile
// opaque zero: seen as loop invariant, the lane and LDS offsets of every
// compiled (length, kind, shape) case were hoisted out of the tile loop and
// held across it (200 to 330 vector registers for complex64, against about
// 120 without the loop).  More blocks per CU only add to the barriers' cost
// (0.74, 0.75, 0.87 ms for the 64-grid batch with 1, 2, 3 blocks per CU), so
// the grid is one block per CU.
struct BatchCoopArgs {
    const BatchItem *items;     // all segments, pass by pass
    int item_begin[4];          // segments of pass p: [item_begin[p], item_begin[p + 1])
    long long tiles[3];         // tiles of pass p, numbered from 0 within the pass
    const void *in;
    void *out;
};

constexpr int kBatchLengths[8] = {48, 60, 64, 72, 80, 96, 100, 128};
// Two tile shapes per length for complex64 (one for complex128), all of 256
// threads: shape 0 (the default) has 8 threads per line for 64 and 128 and
// 4 for the others; shape 1 swaps them (4 threads and 64-line tiles for 64
// and 128, 8 threads and 32-line tiles for the others).  The autotuner picks
// per (length, kind).  complex128 keeps shape 0 only: shape 1 of 64 and 128
// holds twice the elements per thread, which took the kernel past 256
// vector registers and halved its occupancy for every length.
constexpr int kBatchShapes = 2;
template <class St>
constexpr int batch_shapes() { return sizeof(typename St::R) == 4 ? 2 : 1; }
constexpr int batch_threads(int n, int shape = 0) {
    return ((n == 64 || n == 128) != (shape == 1)) ? 8 : 4;
}

template <int N, int KIND, class St, int SH = 0>
using BCfg = SCfg<N, KIND, (int)sizeof(typename St::Raw), (int)sizeof(cx<typename St::R>),
                  N / batch_threads(N, SH), 256 / batch_threads(N, SH), 0, 0>;

template <class Cfg, class St, int KIND, bool INV>
__device__ __forceinline__ void batch_tile(const PassArgs &a, long long tile, unsigned char *smem, int tid) {
    using R = typename St::R;
    static_assert(Cfg::kBlock == 256, "batched configurations use 256 threads");
    constexpr int T = Cfg::T;
    constexpr int L = Cfg::L;
    cx<R> *lds = reinterpret_cast<cx<R> *>(smem);
    cx<R> *tws = reinterpret_cast<cx<R> *>(smem + Cfg::kLdsData);
    unsigned *red = nullptr;
    const int l = KIND == kContiguous ? tid / T : tid % L;
    // with whole wavefronts of lines, t is the wavefront's index: uniform
    const int t = KIND == kContiguous ? tid % T
                  : (L % 64 == 0 ? (int)__builtin_amdgcn_readfirstlane((unsigned)(tid / L)) : tid / L);
    if constexpr (Cfg::kTwN > 0) {
        const cx<R> *W = reinterpret_cast<const cx<R> *>(a.tw);
        for (int i = tid; i < Cfg::kTwN; i += Cfg::kBlock) tws[i] = W[tw_source<Cfg>(i)];
        __syncthreads();
    }
    const long long es = KIND == kContiguous ? 1 : a.es;
    const long long tx = KIND == kContiguous ? tile : tile % a.ntiles;
    const long long w = KIND == kContiguous ? 0 : tile / a.ntiles;
    const TileCoord c = tile_coord<Cfg, KIND>(a, tx, w, l);
    const unsigned lane = lane_offset<Cfg, St, KIND>(l, t, es);
    Tile<Cfg, St> cur;
    fetch_tile<Cfg, St, KIND, INV>(a, c, t, lane, es, cur);
    int ex = 0;
    static_stage<Cfg, St, KIND, INV, 0>(a, lds, tws, red, t, l, c, lane, es, cur, ex);
}

// tid: threadIdx.x
template <class St, bool INV>
__device__ __forceinline__ void batch_dispatch(const BatchItem &it, long long lt, const void *in, void *out,
                                               unsigned char *smem, int tid) {
    const size_t eb = sizeof(typename St::Raw);
    PassArgs a;
    a.in = reinterpret_cast<const char *>(it.from_in ? in : out) + it.offset * eb;
    a.out = reinterpret_cast<char *>(out) + it.offset * eb;
    a.tw = it.tw;
    a.in_exp = nullptr;
    a.out_exp = nullptr;
    a.nlines = it.nlines;
    a.es = it.es;
    a.nw = it.nw;
    a.ntiles = it.ntiles;
    a.total = it.total;
    a.inverse = INV;
    switch (it.code) {
#define CROFT_BATCH_CASE(I, SH)                                                                               \
    case 2 * I + 16 * SH:                                                                                     \
        if constexpr (SH < batch_shapes<St>())                                                                \
            batch_tile<BCfg<kBatchLengths[I], kContiguous, St, SH>, St, kContiguous, INV>(a, lt, smem, tid); \
        break;                                                                                                \
    case 2 * I + 1 + 16 * SH:                                                                                 \
        if constexpr (SH < batch_shapes<St>())                                                                \
            batch_tile<BCfg<kBatchLengths[I], kStrided, St, SH>, St, kStrided, INV>(a, lt, smem, tid);       \
        break;
        CROFT_BATCH_CASE(0, 0)
        CROFT_BATCH_CASE(1, 0)
        CROFT_BATCH_CASE(2, 0)
        CROFT_BATCH_CASE(3, 0)
        CROFT_BATCH_CASE(4, 0)
        CROFT_BATCH_CASE(5, 0)
        CROFT_BATCH_CASE(6, 0)
        CROFT_BATCH_CASE(7, 0)
        CROFT_BATCH_CASE(0, 1)
        CROFT_BATCH_CASE(1, 1)
        CROFT_BATCH_CASE(2, 1)
        CROFT_BATCH_CASE(3, 1)
        CROFT_BATCH_CASE(4, 1)
        CROFT_BATCH_CASE(5, 1)
        CROFT_BATCH_CASE(6, 1)
        CROFT_BATCH_CASE(7, 1)
#undef CROFT_BATCH_CASE
        default: break;
    }
}

__device__ __forceinline__ int find_segment(const BatchItem *items, int lo, int hi, long long tile) {
    // last segment in [lo, hi] whose first tile is <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (items[mid].tile_begin <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class St, bool INV>
__global__ void __launch_bounds__(256) fft_batch_coop(const BatchCoopArgs b) {
    extern __shared__ __align__(16) unsigned char smem[];
#pragma unroll 1
    for (int p = 0; p < 3; ++p) {
        for (long long tile = blockIdx.x; tile < b.tiles[p]; tile += gridDim.x) {
            const int si = find_segment(b.items, b.item_begin[p], b.item_begin[p + 1] - 1, tile);
            const BatchItem it = b.items[si];
            batch_dispatch<St, INV>(it, tile - it.tile_begin, b.in, b.out, smem, (int)threadIdx.x + opaque_zero());
            __syncthreads();  // the next tile reuses the LDS
        }
        if (p < 2) {
            __threadfence();  // this pass's stores, before any block reads them
            cooperative_groups::this_grid().sync();
        }
    }
}

template <class St, bool INV>
__global__ void __launch_bounds__(256) fft_batch(const BatchArgs b) {
    extern __shared__ __align__(16) unsigned char smem[];
    const long long tile = blockIdx.x;
    const BatchItem it = b.items[find_segment(b.items, 0, b.nitems - 1, tile)];
    batch_dispatch<St, INV>(it, tile - it.tile_begin, b.in, b.out, smem, (int)threadIdx.x);
}

// ------------------------------------------------------------ kernel table
struct Entry {
    int n, kind, dtype, cand;
    const void *func[2];  // forward, inverse
    int T, L, block;
    size_t lds;
    RPlan plan;
    int plain = -1;  // non-temporal candidates: the candidate without the hint
    bool whole_tiles = false;  // runs only where every tile is whole (es a multiple of L)
};

// An entry whose kernel uses the non-temporal hint, with the candidate index
// of its plain twin, taken where a pass's rows are not whole 128-byte lines:
// the same kernel without the hint, or, where another plain kernel is the
// faster one there, that one.
inline Entry with_plain(Entry e, int plain) {
    e.plain = plain;
    return e;
}

template <int N, int KIND, class St, int SB, int DT, int EPT = 0, int LREQ = 0, int PAD = 0, int PF = 1,
          int NT = 0, int XO = 0>
Entry make_entry(int cand) {
    using Cfg = SCfg<N, KIND, SB, (int)sizeof(cx<typename St::R>), EPT, LREQ, PAD, PF, NT, XO>;
    static_assert(Cfg::kBlock <= 1024, "block too large");
    static_assert(Cfg::kLds <= 160 * 1024, "LDS beyond the 160 KiB of a gfx950 workgroup");
    static_assert(Cfg::S >= 1, "length must have a radix plan");
    Entry e;
    e.n = N;
    e.kind = KIND;
    e.dtype = DT;
    e.cand = cand;
    e.func[0] = reinterpret_cast<const void *>(&fft_static<Cfg, St, KIND, false>);
    e.func[1] = reinterpret_cast<const void *>(&fft_static<Cfg, St, KIND, true>);
    e.T = Cfg::T;
    e.L = Cfg::L;
    e.block = Cfg::kBlock;
    e.lds = Cfg::kLds;
    e.plan = Cfg::plan;
    return e;
}

// The lane-per-line strided configuration of length N (512 or 1024).
template <int N, class St, int DT, int NTM, int BLOCK = kLanesBlock, bool XO = false, bool REV = false,
          bool PF = false, bool RP = false>
Entry make_lanes_entry(int cand) {
    using C = LanesCfg<N, St, BLOCK>;
    static_assert(C::kBytes <= 160 * 1024, "LDS beyond the 160 KiB of a gfx950 workgroup");
    Entry e;
    e.n = N;
    e.kind = kStrided;
    e.dtype = DT;
    e.cand = cand;
    e.func[0] = reinterpret_cast<const void *>(&fft_lanes<N, St, false, NTM, BLOCK, XO, REV, PF, RP>);
    e.func[1] = reinterpret_cast<const void *>(&fft_lanes<N, St, true, NTM, BLOCK, XO, REV, PF, RP>);
    e.whole_tiles = PF;
    e.T = C::TPL;
    e.L = C::L;
    e.block = BLOCK;
    e.lds = C::kBytes;
    e.plan = C::plan;
    return e;
}

// The real x pass of length 2N on the contiguous configuration of length N.
// NT: the non-temporal hint on the pass's global loads and stores (candidate 1)
template <int N, class St, int SB, int DT, int NT = 0>
Entry make_real_entry() {
    using Cfg = SCfg<N, kContiguous, SB, (int)sizeof(cx<typename St::R>), 0, 0, 0, 1, NT>;
    using Lay = RealLds<Cfg, std::integral_constant<int, (int)sizeof(cx<typename St::R>)>>;
    static_assert(Lay::kBytes <= 160 * 1024, "LDS beyond the 160 KiB of a gfx950 workgroup");
    Entry e;
    e.n = N;
    e.kind = kRealX;
    e.dtype = DT;
    e.cand = NT;
    e.func[0] = reinterpret_cast<const void *>(&fft_real_x<Cfg, St, false>);
    e.func[1] = reinterpret_cast<const void *>(&fft_real_x<Cfg, St, true>);
    e.T = Cfg::T;
    e.L = Cfg::L;
    e.block = Cfg::kBlock;
    e.lds = Lay::kBytes;
    e.plan = Cfg::plan;
    return e;
}

// The fused multiply pass of length N on a strided configuration (EW elements
// per thread and LW lines per tile; 0 = the default shape).
template <int N, class St, int SB, int DT, int EW = 0, int LW = 0>
Entry make_conv_entry(int cand) {
    using Cfg = SCfg<N, kStrided, SB, (int)sizeof(cx<typename St::R>), EW, LW, 0, 0>;
    static_assert(Cfg::kLds <= 160 * 1024, "LDS beyond the 160 KiB of a gfx950 workgroup");
    static_assert((size_t)Cfg::kBlock * sizeof(double) <= Cfg::kLdsData, "block sum fits the tile area");
    Entry e;
    e.n = N;
    e.kind = kConvZ;
    e.dtype = DT;
    e.cand = cand;
    e.func[0] = e.func[1] = reinterpret_cast<const void *>(&fft_conv_z<Cfg, St>);
    e.T = Cfg::T;
    e.L = Cfg::L;
    e.block = Cfg::kBlock;
    e.lds = Cfg::kLds;
    e.plan = Cfg::plan;
    return e;
}

}  // namespace dev
}  // namespace croft
