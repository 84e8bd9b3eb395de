// croft_bluestein.hip -- lengths with a prime factor above 5 (Bluestein 1970).
// With c[j] = exp(-pi i j^2 / n),
//   X[k] = c[k] sum_j (x[j] c[j]) conj(c[k - j]),
// a circular convolution of length m (a power of two >= 2n - 1) done as
// m-point FFTs in LDS: forward FFT of the chirped, zero-padded line, product
// with the kernel's DFT (precomputed, divided by m), then the inverse FFT as
// swap(DFT(swap(.))) and the final chirp.  The kernel is compiled for every
// m a plan can need, so that its Stockham stages have their radix, span and
// stride as constants (a power-of-two span makes the butterfly index
// arithmetic shifts and masks).  a.tw is the m-point twiddle table; the line
// geometry, exponents and inverse-by-swap are those of the runtime-radix
// kernel.
#include <hip/hip_runtime.h>

#include "croft_device.h"
#include "croft_internal.h"

namespace croft {
using namespace dev;
namespace {

// The launch shape of the kernel for convolution length M: T threads per
// line (one per butterfly of the widest stage, at most 256), L lines per
// block (as many as 256 threads and the LDS allow, and for strided passes
// rows of at most 128 bytes, rounded down to a power of two), the m-point
// twiddle table in LDS where it takes at most 16 KiB.
template <class St, int KIND, int M>
struct BlueCfg {
    using R = typename St::R;
    static constexpr RPlan P = make_rplan(M);
    static constexpr int T = M / P.rmax > 256 ? 256 : M / P.rmax;
    static constexpr int CB = (int)sizeof(cx<R>);
    static constexpr bool kTwLds = (long long)M * CB <= 16384;
    static constexpr long long lds_of(int lines) {
        return (kTwLds ? (long long)M * CB : 0) + 2LL * lines * M * CB + 4LL * lines;
    }
    static constexpr int max_lines() {
        int k = 0;
        while (lds_of(k + 1) <= 160 * 1024) ++k;
        return k;
    }
    static constexpr int lines() {
        int want = 256 / T;
        if (KIND != kContiguous) {
            const int row = 128 / (int)sizeof(typename St::Raw);
            want = want < row ? want : row;
        }
        if (want < 1) want = 1;
        if (want > max_lines()) want = max_lines();
        int p2 = 1;
        while (p2 * 2 <= want) p2 *= 2;
        return p2;
    }
    static constexpr int L = lines();
    static constexpr long long kLds = lds_of(L);
};

// LDS position of element e of line l: contiguous lines one after another,
// strided tiles element-major (the L lines of a tile side by side)
template <int KIND, int M, int L>
__device__ __forceinline__ int lds_at(int l, int e) {
    return KIND == kContiguous ? l * M + e : e * L + l;
}

// One Stockham stage of the m-point FFT: butterfly j (of M / RAD) reads
// positions j + q M/RAD, twiddles them by w_{NS RAD}^{q (j mod NS)}, and
// writes positions (j div NS) NS RAD + (j mod NS) + q NS.
template <int RAD, int NS, int M, int T, int L, typename R, int KIND>
__device__ __forceinline__ void stage(const cx<R> *src, cx<R> *dst, const cx<R> *tw, int l, int t) {
    constexpr int NB = M / RAD;
    constexpr int TWS = M / (NS * RAD);
#pragma unroll
    for (int jj = 0; jj < (NB + T - 1) / T; ++jj) {
        const int j = t + jj * T;
        if (NB % T != 0 && j >= NB) break;
        cx<R> v[RAD];
#pragma unroll
        for (int q = 0; q < RAD; ++q) v[q] = src[lds_at<KIND, M, L>(l, j + q * NB)];
        const int k = j % NS;
        if constexpr (NS > 1) {
#pragma unroll
            for (int q = 1; q < RAD; ++q) v[q] = cmul(v[q], tw[q * k * TWS]);
        }
        Dft<RAD, R>::run(v);
        const int o0 = (j / NS) * NS * RAD + k;
#pragma unroll
        for (int q = 0; q < RAD; ++q) dst[lds_at<KIND, M, L>(l, o0 + q * NS)] = v[q];
    }
}

// Stages S.. of the m-point FFT, ping-ponging between src and dst; returns
// the buffer that holds the result
template <int S, int NS, int M, int T, int L, typename R, int KIND>
__device__ __forceinline__ cx<R> *stages(cx<R> *src, cx<R> *dst, const cx<R> *tw, int l, int t, bool active) {
    constexpr RPlan P = make_rplan(M);
    if constexpr (S == P.S) {
        return src;
    } else {
        constexpr int RAD = P.r[S];
        if (active) stage<RAD, NS, M, T, L, R, KIND>(src, dst, tw, l, t);
        __syncthreads();
        return stages<S + 1, NS * RAD, M, T, L, R, KIND>(dst, src, tw, l, t, active);
    }
}

template <class St, int KIND, int M>
__global__ void __launch_bounds__(256) fft_bluestein(const PassArgs a) {
    using R = typename St::R;
    static_assert((M & (M - 1)) == 0, "power-of-two convolution length");
    extern __shared__ __align__(16) unsigned char smem[];
    using C = BlueCfg<St, KIND, M>;
    constexpr int T = C::T, L = C::L;
    constexpr int EPT = M / T;  // convolution elements per thread
    const int n = a.n;
    // the m-point twiddle table first, where it fits (one global read per
    // block instead of one per twiddled butterfly and stage), then the two
    // line buffers and the line maxima
    constexpr bool kTwLds = C::kTwLds;
    cx<R> *buf0 = reinterpret_cast<cx<R> *>(smem) + (kTwLds ? M : 0);
    cx<R> *buf1 = buf0 + L * M;
    unsigned *red = reinterpret_cast<unsigned *>(buf1 + L * M);
    const cx<R> *tw = reinterpret_cast<const cx<R> *>(a.tw);
    if constexpr (kTwLds) {
        cx<R> *twl = reinterpret_cast<cx<R> *>(smem);
        for (int i = threadIdx.x; i < M; i += blockDim.x) twl[i] = tw[i];
        tw = twl;  // made visible by the barrier after the chirped line
    }
    const cx<R> *ch = reinterpret_cast<const cx<R> *>(a.chirp);
    const cx<R> *bh = reinterpret_cast<const cx<R> *>(a.bhat);
    const int tid = threadIdx.x;
    const int l = KIND == kContiguous ? tid / T : tid % L;
    const int t = KIND == kContiguous ? tid % T : tid / L;
    const bool active = tid < T * L;
    long long q, w;
    if (KIND == kContiguous) {
        q = (long long)blockIdx.x * L + l;
        w = 0;
    } else {
        // each XCD takes a contiguous run of tiles: the 32-byte rows of
        // neighbouring tiles share 128-byte lines, which then meet in one L2
        const long long b = xcd_tile(blockIdx.x, gridDim.x);
        q = (b % a.ntiles) * L + l;
        w = b / a.ntiles;
    }
    const bool valid = active && q < (KIND == kContiguous ? a.nlines : a.es);
    const long long es = KIND == kContiguous ? 1 : a.es;
    const long long base = KIND == kContiguous ? q * n : q + w * a.es * n;
    const bool inv = a.inverse != 0;
    int ebase = 0;
    if constexpr (St::kHalf) {
        const ExpMap &mp = a.em;
        ebase = (int)exp_line_index(mp, q, w, mp.a0, mp.a1, mp.a2);
        if (active && t == 0) red[l] = 0u;
    }
    // chirped line, zero-padded to m (every load of the thread in flight at once)
    if (active) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = t + i * T;
            cx<R> v = {R(0), R(0)};
            if (valid && e < n) {
                int ex = 0;
                if constexpr (St::kHalf) ex = a.in_exp ? (int)a.in_exp[ebase + a.em.a3 * e] : 0;
                v = St::decode(St::fetch(a.in, base + es * e), ex);
                if (inv) v = {v.y, v.x};
                v = cmul(v, ch[e]);
            }
            buf0[lds_at<KIND, M, L>(l, e)] = v;
        }
    }
    __syncthreads();
    cx<R> *r = stages<0, 1, M, T, L, R, KIND>(buf0, buf1, tw, l, t, active);
    // product with the kernel's DFT, swapped: the next forward FFT then gives
    // the unnormalised inverse once swapped back
    if (active) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = t + i * T;
            cx<R> &v = r[lds_at<KIND, M, L>(l, e)];
            const cx<R> p = cmul(v, bh[e]);
            v = {p.y, p.x};
        }
    }
    __syncthreads();
    cx<R> *o = stages<0, 1, M, T, L, R, KIND>(r, r == buf0 ? buf1 : buf0, tw, l, t, active);
    // X[k] = c[k] swap(o[k]); every thread rewrites only the entries it reads later
    if (active) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = t + i * T;
            if (e < n) {
                cx<R> &v = o[lds_at<KIND, M, L>(l, e)];
                v = cmul(cx<R>{v.y, v.x}, ch[e]);
            }
        }
    }
    int ex = 0;
    if constexpr (St::kHalf) {
        float mx = 0.0f;
        if (active) {
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                const int e = t + i * T;
                if (e < n) {
                    const cx<R> v = o[lds_at<KIND, M, L>(l, e)];
                    mx = fmaxf(mx, fmaxf(fabsf((float)v.x), fabsf((float)v.y)));
                }
            }
        }
        if (active) atomicMax(&red[l], __float_as_uint(mx));
        __syncthreads();
        if (active) ex = line_exponent(__uint_as_float(red[l]));
        if (valid && t == 0 && a.out_exp) {
            const ExpMap &mp = a.em;
            a.out_exp[exp_line_index(mp, q, w, mp.b0, mp.b1, mp.b2)] = (int8_t)ex;
        }
    }
    if (valid) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = t + i * T;
            if (e < n) {
                cx<R> v = o[lds_at<KIND, M, L>(l, e)];
                if (inv) v = {v.y, v.x};
                St::store(a.out, base + es * e, v, ex);
            }
        }
    }
}

template <class St, int KIND, int M>
BluesteinLaunch launch_of() {
    using C = BlueCfg<St, KIND, M>;
    BluesteinLaunch b;
    if constexpr (C::max_lines() >= 1) {
        b.func = reinterpret_cast<const void *>(&fft_bluestein<St, KIND, M>);
        b.T = C::T;
        b.L = C::L;
        b.lds = (size_t)C::kLds;
    }
    return b;
}

template <class St, int KIND>
BluesteinLaunch for_length(int m) {
    switch (m) {
        case 16: return launch_of<St, KIND, 16>();
        case 32: return launch_of<St, KIND, 32>();
        case 64: return launch_of<St, KIND, 64>();
        case 128: return launch_of<St, KIND, 128>();
        case 256: return launch_of<St, KIND, 256>();
        case 512: return launch_of<St, KIND, 512>();
        case 1024: return launch_of<St, KIND, 1024>();
        case 2048: return launch_of<St, KIND, 2048>();
        case 4096: return launch_of<St, KIND, 4096>();
        case 8192: return launch_of<St, KIND, 8192>();
        default: return BluesteinLaunch{};
    }
}

template <int KIND>
BluesteinLaunch for_dtype(int dtype, int m) {
    switch (dtype) {
        case kC64: return for_length<StC64, KIND>(m);
        case kC128: return for_length<StC128, KIND>(m);
        case kC16F: return for_length<StHalf<false>, KIND>(m);
        default: return for_length<StHalf<true>, KIND>(m);
    }
}

}  // namespace

BluesteinLaunch bluestein_kernel(int kind, int dtype, int m) {
    return kind == kContiguous ? for_dtype<kContiguous>(dtype, m) : for_dtype<kStrided>(dtype, m);
}

}  // namespace croft
