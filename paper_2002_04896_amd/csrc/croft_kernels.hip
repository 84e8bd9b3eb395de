// croft_kernels.hip -- kernel selection and launch, and the runtime-radix
// kernel that runs lengths without a compiled static configuration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "croft_device.h"
#include "croft_internal.h"

namespace croft {
namespace dev {
// compiled static configurations, one translation unit per dtype
std::vector<Entry> entries_c64();
std::vector<Entry> entries_c128();
std::vector<Entry> entries_c16f();
std::vector<Entry> entries_c16b();
}  // namespace dev
using namespace dev;
namespace {

// ------------------------------------------------------- runtime-radix kernel
// Any supported length.  Stages ping-pong between two LDS buffers, the last
// stage included; a final sweep stores the line from LDS.
template <int KIND>
__device__ __forceinline__ int glds(int l, int e, int n, int L) {
    return KIND == kContiguous ? l * n + e : e * L + l;
}

template <int RAD, typename R, int KIND>
__device__ __forceinline__ void generic_stage(const cx<R> *src, cx<R> *dst, const cx<R> *tw, int n, int L,
                                              int l, int t, int T, int Ns) {
    const int NB = n / RAD;
    const int tws = n / (Ns * RAD);
    for (int j = t; j < NB; j += T) {
        cx<R> v[RAD];
#pragma unroll
        for (int q = 0; q < RAD; ++q) v[q] = src[glds<KIND>(l, j + q * NB, n, L)];
        const int k = j % Ns;
        if (Ns > 1) {
#pragma unroll
            for (int q = 1; q < RAD; ++q) v[q] = cmul(v[q], tw[q * k * tws]);
        }
        Dft<RAD, R>::run(v);
        const int o0 = (j / Ns) * Ns * RAD + k;
#pragma unroll
        for (int q = 0; q < RAD; ++q) dst[glds<KIND>(l, o0 + q * Ns, n, L)] = v[q];
    }
}

// TWL: the length-n twiddle table is copied into LDS ahead of the line
// buffers (one global read per block instead of one per twiddled butterfly
// and stage), where the planner found room for it.
template <class St, int KIND, bool TWL>
__global__ void __launch_bounds__(256) fft_generic(const PassArgs a) {
    using R = typename St::R;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = a.n, T = a.T, L = a.L;
    cx<R> *buf0 = reinterpret_cast<cx<R> *>(smem) + (TWL ? n : 0);
    cx<R> *buf1 = buf0 + (size_t)L * n;
    unsigned *red = reinterpret_cast<unsigned *>(buf1 + (size_t)L * n);
    const cx<R> *tw = reinterpret_cast<const cx<R> *>(a.tw);
    if constexpr (TWL) {
        cx<R> *twl = reinterpret_cast<cx<R> *>(smem);
        for (int i = threadIdx.x; i < n; i += blockDim.x) twl[i] = tw[i];
        tw = twl;  // made visible by the barrier after the line loads
    }
    const int tid = threadIdx.x;
    const int l = KIND == kContiguous ? tid / T : tid % L;
    const int t = KIND == kContiguous ? tid % T : tid / L;
    const bool active = tid < T * L;
    long long q, w;
    if (KIND == kContiguous) {
        q = (long long)blockIdx.x * L + l;
        w = 0;
    } else {
        // each XCD takes a contiguous run of tiles: the narrow rows of
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
        const ExpMap &m = a.em;
        ebase = (int)exp_line_index(m, q, w, m.a0, m.a1, m.a2);
        if (active && t == 0) red[l] = 0u;
    }
    // load the line into buf0 (consecutive t read consecutive e), up to 8
    // loads of a thread in flight before their LDS stores
    if (active) {
        constexpr int kChunk = 8;
        for (int e0 = t; e0 < n; e0 += kChunk * T) {
            cx<R> v[kChunk];
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                const int e = e0 + c * T;
                v[c] = {R(0), R(0)};
                if (valid && e < n) {
                    int ex = 0;
                    if constexpr (St::kHalf) ex = a.in_exp ? (int)a.in_exp[ebase + a.em.a3 * e] : 0;
                    v[c] = St::decode(St::fetch(a.in, base + es * e), ex);
                    if (inv) v[c] = {v[c].y, v[c].x};
                }
            }
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                const int e = e0 + c * T;
                if (e < n) buf0[glds<KIND>(l, e, n, L)] = v[c];
            }
        }
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
                const cx<R> v = src[glds<KIND>(l, e, n, L)];
                mx = fmaxf(mx, fmaxf(fabsf((float)v.x), fabsf((float)v.y)));
            }
        if (active) atomicMax(&red[l], __float_as_uint(mx));
        __syncthreads();
        if (active) ex = line_exponent(__uint_as_float(red[l]));
        if (valid && t == 0 && a.out_exp) {
            const ExpMap &m = a.em;
            a.out_exp[exp_line_index(m, q, w, m.b0, m.b1, m.b2)] = (int8_t)ex;
        }
    }
    if (valid) {
        for (int e = t; e < n; e += T) {
            cx<R> o = src[glds<KIND>(l, e, n, L)];
            if (inv) o = {o.y, o.x};
            St::store(a.out, base + es * e, o, ex);
        }
    }
}

// Stages of the plan in a.radix over LDS lines of length len, ping-ponging
// between two buffers; returns the buffer that holds the result.
template <typename R, int KIND>
__device__ cx<R> *run_stages(const PassArgs &a, cx<R> *src, cx<R> *dst, const cx<R> *tw, int len, int L, int l,
                             int t, int T, bool active) {
    int Ns = 1;
    for (int s = 0; s < a.S; ++s) {
        const int rad = a.radix[s];
        if (active) {
            switch (rad) {
                case 2: generic_stage<2, R, KIND>(src, dst, tw, len, L, l, t, T, Ns); break;
                case 3: generic_stage<3, R, KIND>(src, dst, tw, len, L, l, t, T, Ns); break;
                case 4: generic_stage<4, R, KIND>(src, dst, tw, len, L, l, t, T, Ns); break;
                case 5: generic_stage<5, R, KIND>(src, dst, tw, len, L, l, t, T, Ns); break;
                case 8: generic_stage<8, R, KIND>(src, dst, tw, len, L, l, t, T, Ns); break;
                default: generic_stage<16, R, KIND>(src, dst, tw, len, L, l, t, T, Ns); break;
            }
        }
        Ns *= rad;
        cx<R> *tmp = src;
        src = dst;
        dst = tmp;
        __syncthreads();
    }
    return src;
}

// ------------------------------------------------------ fused multiply (any length)
// The fused forward FFT / multiply / inverse FFT pass of a convolution plan for
// 2^a 3^b 5^c lengths without a compiled fused kernel: strided lines, one tile
// per block, the runtime-radix stages twice, the product (and the energy
// terms, as in the compiled kernel) in between.
template <class St>
__global__ void __launch_bounds__(256) fft_generic_conv(const PassArgs a) {
    using R = typename St::R;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = a.n, T = a.T, L = a.L;
    cx<R> *buf0 = reinterpret_cast<cx<R> *>(smem);
    cx<R> *buf1 = buf0 + (size_t)L * n;
    const cx<R> *tw = reinterpret_cast<const cx<R> *>(a.tw);
    const R *G = reinterpret_cast<const R *>(a.mul);
    const int tid = threadIdx.x;
    const int l = tid % L;
    const int t = tid / L;
    const bool active = tid < T * L;
    const long long q = ((long long)blockIdx.x % a.ntiles) * L + l;
    const long long w = (long long)blockIdx.x / a.ntiles;
    const bool valid = active && q < a.es;
    const long long es = a.es;
    const long long base = q + w * es * n;
    if (active) {
        for (int e = t; e < n; e += T) {
            cx<R> v = {R(0), R(0)};
            if (valid) v = St::decode(St::fetch(a.in, base + es * e), 0);
            buf0[glds<kStrided>(l, e, n, L)] = v;
        }
    }
    __syncthreads();
    cx<R> *r = run_stages<R, kStrided>(a, buf0, buf1, tw, n, L, l, t, T, active);
    double acc = 0.0;
    if (valid) {
        const long long kx = q % a.hx;
        const double wgt = (kx == 0 || kx == a.hx - 1) ? 1.0 : 2.0;
        for (int e = t; e < n; e += T) {
            cx<R> &v = r[glds<kStrided>(l, e, n, L)];
            const R gv = G[base + es * e];
            const double m2 = (double)v.x * v.x + (double)v.y * v.y;
            acc = fma(wgt * (double)gv, m2, acc);
            v = cx<R>{v.y * gv, v.x * gv};  // the product, swapped for the inverse
        }
    }
    __syncthreads();
    cx<R> *o = run_stages<R, kStrided>(a, r, r == buf0 ? buf1 : buf0, tw, n, L, l, t, T, active);
    if (valid) {
        for (int e = t; e < n; e += T) {
            const cx<R> v = o[glds<kStrided>(l, e, n, L)];
            St::store(a.out, base + es * e, cx<R>{v.y, v.x}, 0);
        }
    }
    __syncthreads();
    double *sum = reinterpret_cast<double *>(smem);  // the line buffers are free now
    const int B = blockDim.x;
    sum[tid] = acc;
    __syncthreads();
    for (int h = 1; h < B; h *= 2) {
        if ((tid & (2 * h - 1)) == 0 && tid + h < B) sum[tid] += sum[tid + h];
        __syncthreads();
    }
    if (tid == 0) a.partial[blockIdx.x] = sum[0];
}

const std::vector<Entry> &table() {
    static const std::vector<Entry> t = [] {
        std::vector<Entry> v;
        for (auto f : {entries_c64, entries_c128, entries_c16f, entries_c16b}) {
            std::vector<Entry> e = f();
            v.insert(v.end(), e.begin(), e.end());
        }
        return v;
    }();
    return t;
}

template <bool TWL>
const void *generic_func_t(int kind, int dtype) {
    if (kind == kContiguous) {
        switch (dtype) {
            case kC64: return reinterpret_cast<const void *>(&fft_generic<StC64, kContiguous, TWL>);
            case kC128: return reinterpret_cast<const void *>(&fft_generic<StC128, kContiguous, TWL>);
            case kC16F: return reinterpret_cast<const void *>(&fft_generic<StHalf<false>, kContiguous, TWL>);
            default: return reinterpret_cast<const void *>(&fft_generic<StHalf<true>, kContiguous, TWL>);
        }
    }
    switch (dtype) {
        case kC64: return reinterpret_cast<const void *>(&fft_generic<StC64, kStrided, TWL>);
        case kC128: return reinterpret_cast<const void *>(&fft_generic<StC128, kStrided, TWL>);
        case kC16F: return reinterpret_cast<const void *>(&fft_generic<StHalf<false>, kStrided, TWL>);
        default: return reinterpret_cast<const void *>(&fft_generic<StHalf<true>, kStrided, TWL>);
    }
}

const void *generic_func(int kind, int dtype, bool twl) {
    return twl ? generic_func_t<true>(kind, dtype) : generic_func_t<false>(kind, dtype);
}

// One block of 256 threads: thread i sums partial[i], partial[i + 256], ...
// in order, then a fixed tree over the block.
__global__ void __launch_bounds__(256) sum_partials(const double *partial, int n, double *energy) {
    __shared__ double s[256];
    const int tid = threadIdx.x;
    double v = 0.0;
    for (int i = tid; i < n; i += 256) v += partial[i];
    s[tid] = v;
    __syncthreads();
    for (int h = 128; h > 0; h /= 2) {
        if (tid < h) s[tid] += s[tid + h];
        __syncthreads();
    }
    if (tid == 0) energy[0] = s[0];
}

}  // namespace

int kernel_candidates(int n, int kind, int dtype) {
    int c = 0;
    for (const Entry &e : table())
        if (e.n == n && e.kind == kind && e.dtype == dtype) ++c;
    return c;
}

bool select_kernel(int n, int kind, int dtype, bool force_generic, int cand, KernelConfig *cfg) {
    if (n < 1 || n > kMaxLength) return false;
    if (!force_generic || kind == kRealX || kind == kConvZ) {
        const Entry *pick = nullptr;
        for (const Entry &e : table()) {
            if (e.n == n && e.kind == kind && e.dtype == dtype) {
                if (e.cand == 0 && !pick) pick = &e;
                if (e.cand == cand) pick = &e;
            }
        }
        if (pick) {
            cfg->func = pick->func[0];
            cfg->func_inv = pick->func[1];
            cfg->generic = false;
            cfg->bluestein = 0;
            cfg->candidate = pick->cand;
            cfg->plain = pick->plain;
            cfg->whole_tiles = pick->whole_tiles;
            cfg->threads_per_line = pick->T;
            cfg->lines = pick->L;
            cfg->block = pick->block;
            cfg->lds = pick->lds;
            cfg->nstages = pick->plan.S;
            for (int s = 0; s < pick->plan.S; ++s) cfg->radix[s] = pick->plan.r[s];
            return true;
        }
    }
    if (kind == kRealX || kind == kConvZ) return false;  // compiled configurations only
    const int cb = dtype == kC128 ? 16 : 8;                      // compute bytes
    if (make_rplan(n).S < 0) {
        // Bluestein: the kernel compiled for the convolution length m
        const int m = bluestein_length(n);
        const RPlan pm = make_rplan(m);
        const BluesteinLaunch bl = bluestein_kernel(kind, dtype, m);
        if (!bl.func || pm.S < 0) return false;
        const int T = bl.T, L = bl.L;
        cfg->func = cfg->func_inv = bl.func;
        cfg->generic = true;
        cfg->bluestein = m;
        cfg->candidate = 0;
        cfg->plain = -1;
        cfg->whole_tiles = false;
        cfg->threads_per_line = T;
        cfg->lines = L;
        cfg->block = ((T * L + 63) / 64) * 64;
        cfg->lds = bl.lds;
        cfg->nstages = pm.S;
        for (int s = 0; s < pm.S; ++s) cfg->radix[s] = pm.r[s];
        return true;
    }
    const RPlan p = make_rplan(n);
    const int sb = (int)element_bytes(dtype);                    // storage bytes
    int T = n / p.rmax;
    if (T < 1) T = 1;
    if (T > 256) T = 256;
    const size_t per_line = 2 * (size_t)n * cb + 4;
    int lds_lines = (int)((160 * 1024) / per_line);
    if (lds_lines < 1) return false;
    // the twiddle table in LDS where it leaves room for the lines below
    const size_t table = (size_t)n * cb;
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
    int p2 = 1;  // round down to a power of two
    while (p2 * 2 <= L) p2 *= 2;
    L = p2;
    // Twiddles are read from the second stage on; a plan of at most one
    // stage reads none, and a length-1 pass has no table at all.
    const bool twl = p.S >= 2 && table + (size_t)L * per_line <= 160 * 1024;
    cfg->func = cfg->func_inv = generic_func(kind, dtype, twl);
    cfg->generic = true;
    cfg->bluestein = 0;
    cfg->candidate = 0;
    cfg->plain = -1;
    cfg->whole_tiles = false;
    cfg->threads_per_line = T;
    cfg->lines = L;
    cfg->block = ((T * L + 63) / 64) * 64;
    cfg->lds = (twl ? table : 0) + (size_t)L * per_line;
    cfg->nstages = p.S;
    for (int s = 0; s < p.S; ++s) cfg->radix[s] = p.r[s];
    return true;
}

long long pass_tiles(const PassLaunch &pl) {
    const int L = pl.cfg.lines;
    if (!strided_kind(pl.kind)) return (pl.nlines + L - 1) / L;
    return ((pl.es + L - 1) / L) * pl.nw;
}

long long pass_blocks(const PassLaunch &pl) {
    long long blocks = pass_tiles(pl);
    if (!pl.cfg.generic && pl.cfg.resident > 0 && pl.cfg.grid_waves > 0)
        blocks = std::min<long long>(blocks, (long long)pl.cfg.resident * pl.cfg.grid_waves);
    return blocks;
}

hipError_t launch_pass(const PassLaunch &pl, int dtype, const void *in, void *out, const int8_t *in_exp,
                       int8_t *out_exp, int inverse, hipStream_t stream, const void *mul, double *partial) {
    (void)dtype;
    PassArgs a;
    a.in = in;
    a.out = out;
    a.tw = pl.tw;
    a.tw2 = pl.tw2;
    a.chirp = pl.chirp;
    a.bhat = pl.bhat;
    a.m = pl.cfg.bluestein;
    a.mul = mul;
    a.partial = partial;
    a.hx = pl.hx;
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
    a.nlines = !strided_kind(pl.kind) ? pl.nlines : pl.es;
    a.ntiles = !strided_kind(pl.kind) ? 1 : (pl.es + a.L - 1) / a.L;
    a.total = pass_tiles(pl);
    if (a.total <= 0) return hipSuccess;
    const long long blocks = pass_blocks(pl);
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    void *args[] = {&a};
    const void *f = inverse ? pl.cfg.func_inv : pl.cfg.func;
    return hipLaunchKernel(f, dim3((unsigned)blocks), dim3(pl.cfg.block), args, pl.cfg.lds, stream);
}

hipError_t launch_sum_partials(const double *partial, int n, double *energy, hipStream_t stream) {
    void *args[] = {&partial, &n, &energy};
    return hipLaunchKernel(reinterpret_cast<const void *>(&sum_partials), dim3(1), dim3(256), args, 0, stream);
}

bool select_generic_conv(int n, int dtype, KernelConfig *cfg) {
    if ((dtype != kC64 && dtype != kC128) || make_rplan(n).S < 0) return false;
    if (!select_kernel(n, kStrided, dtype, true, 0, cfg) || cfg->bluestein) return false;
    cfg->func = cfg->func_inv = dtype == kC64 ? reinterpret_cast<const void *>(&fft_generic_conv<StC64>)
                                              : reinterpret_cast<const void *>(&fft_generic_conv<StC128>);
    // two line buffers, no twiddle table; the block sum reuses the line buffers
    const size_t lines = (size_t)cfg->lines * 2 * n * (dtype == kC128 ? 16 : 8);
    cfg->lds = std::max(lines, (size_t)cfg->block * sizeof(double));
    return true;
}

}  // namespace croft
