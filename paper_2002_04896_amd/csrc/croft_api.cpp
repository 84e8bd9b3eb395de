// croft_api.cpp -- the C ABI of include/croft.h: plan construction, pass
// schedules, execution, errors and introspection.
#include "croft.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "croft_internal.h"

using namespace croft;

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_last_error;
thread_local int g_last_status = CROFT_SUCCESS;

void clear_error() {
    g_last_error.clear();
    g_last_status = CROFT_SUCCESS;
}

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    g_last_status = code;
    return code;
}

int fail_hip(hipError_t e, const char *what) {
    return fail(CROFT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}
}  // namespace

// -------------------------------------------------------------------- plan
struct croft_plan {
    int dtype = 0, dir = -1, flags = 0, slabs = 1;
    int device = 0;
    // grids (one for a plain plan)
    std::vector<Geometry> grids;
    std::vector<size_t> offsets;  // element offsets, grids.size() + 1 entries
    // per grid: the pass list of the plain schedule
    std::vector<std::vector<PassLaunch>> passes;
    std::map<int, void *> twiddles;  // length -> device table
    std::map<int, std::pair<void *, void *>> bluestein;  // length -> (chirp, kernel DFT)
    int8_t *e1 = nullptr, *e2 = nullptr;  // half storage: exponents after x and y passes
    int8_t *scratch = nullptr;            // half storage: this device's static scratch array
    size_t work_bytes = 0;
    // real transforms: grids[0] holds the real dimensions; the backward
    // direction runs its complex passes in `rwork` (the input is kept)
    bool real = false;
    void *rwork = nullptr;
    // convolution plans (real, with the fused multiply pass): energy partials
    bool conv = false;
    double *partial = nullptr;
    long long partial_count = 0;  // doubles in `partial`
    // unfused schedule (the paper's Option 2): FFT passes on contiguous lines
    // with standalone transposes between them, through a work grid
    bool unfused = false;
    void *uwork = nullptr;
    // slab schedule; slab_auto: K was left to the plan (K = 0 at create)
    bool slab_auto = false;
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
    // batched form: one launch per pass over the grids the batched kernel
    // compiles (device segment tables), the others grid by grid
    bool batched = false;
    void *bitems = nullptr;            // all segments, pass by pass (device)
    int bbegin[4] = {0, 0, 0, 0};      // segments of pass p: [bbegin[p], bbegin[p + 1])
    long long btiles[3] = {0, 0, 0};   // tiles of pass p
    size_t blds[3] = {0, 0, 0};
    int bresident = 0;                 // cooperative launch: blocks the device holds at once
    bool coop_direct = false;          // CROFT_GRAPH: the cooperative launch could not be captured
    std::vector<size_t> loose;  // grids run with their own launches
    std::vector<size_t> bgrids;  // grids the batched kernel runs
    std::map<std::pair<int, int>, int> bshape;  // (length, kind) -> tile shape of the batched kernel
    // batched form: graph cache
    hipGraphExec_t graph = nullptr;
    const void *graph_in = nullptr;
    void *graph_out = nullptr;
    hipStream_t graph_stream = nullptr;
    // CROFT_TEST_FAIL_ALLOC=k: the k-th plan allocation of this create fails
    int fail_alloc_at = 0;
    int alloc_count = 0;
    // profiling
    bool profiling = false;
    std::vector<std::vector<std::pair<hipEvent_t, hipEvent_t>>> prof;  // per execute, per pass
    std::vector<hipEvent_t> event_pool;
};

namespace {

bool is_half(int dtype) { return dtype == CROFT_C16F || dtype == CROFT_C16B; }

size_t compute_bytes(int dtype) { return dtype == CROFT_C128 ? 16 : 8; }

int check_dims(int nx, int ny, int nz) {
    const int d[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        if (d[a] < 1) return fail(CROFT_ERR_INVALID_VALUE, "axis %d length %d < 1", a, d[a]);
        if (d[a] > kMaxLength)
            return fail(CROFT_ERR_UNSUPPORTED_SIZE, "axis %d length %d unsupported (need 1..%d)", a, d[a],
                        kMaxLength);
    }
    if ((long long)nx * ny * nz > 0x7fffffffLL)
        return fail(CROFT_ERR_UNSUPPORTED_SIZE, "grid of %lld elements exceeds 2^31 - 1",
                    (long long)nx * ny * nz);
    return CROFT_SUCCESS;
}

int check_dtype_dir(int dtype, int dir) {
    if (dtype < CROFT_C64 || dtype > CROFT_C16B) return fail(CROFT_ERR_UNSUPPORTED_DTYPE, "unknown dtype %d", dtype);
    if (dir != CROFT_FORWARD && dir != CROFT_BACKWARD)
        return fail(CROFT_ERR_INVALID_VALUE, "direction %d is neither CROFT_FORWARD (-1) nor CROFT_BACKWARD (+1)",
                    dir);
    return CROFT_SUCCESS;
}

int no_kernel(int n, int dtype) {
    if (!smooth_length(n))
        return fail(CROFT_ERR_UNSUPPORTED_SIZE,
                    "length %d needs Bluestein's algorithm, whose %d-point convolution does not fit in LDS for "
                    "dtype %d (complex128: lengths up to 2048 only)",
                    n, bluestein_length(n), dtype);
    return fail(CROFT_ERR_UNSUPPORTED_SIZE, "no kernel for length %d", n);
}

// Non-temporal stores of part of a 128-byte line cost a read-modify-write,
// and partial non-temporal loads fetch their lines again: where the rows of
// a strided pass are not whole lines (a real grid's half-spectrum y pass,
// 257 complex64 per row: 0.34-0.41 ms with the hint on loads or stores,
// 0.20 without), a candidate with the hint gives way to its plain twin.
// Likewise a candidate that runs whole tiles only (the half-tile copy into
// LDS) gives way to its twin where the last tile of a row is partial.
void plain_on_partial_lines(const PassLaunch &p, int dtype, KernelConfig *cfg) {
    if (p.kind != kStrided || cfg->generic || cfg->plain < 0) return;
    const bool partial_lines = (p.es * (long long)element_bytes(dtype)) % 128 != 0;
    const bool partial_tiles = cfg->whole_tiles && p.es % cfg->lines != 0;
    if (!partial_lines && !partial_tiles) return;
    KernelConfig c;
    if (select_kernel(p.n, p.kind, dtype, false, cfg->plain, &c) && c.candidate == cfg->plain) *cfg = c;
}

// Static kernels address a thread's first element as a uniform 64-bit tile
// base plus a 32-bit per-thread byte offset; true when that offset fits.
bool lane_offset_fits(const PassLaunch &p, int dtype) {
    if (p.cfg.generic) return true;
    const long long L = p.cfg.lines, T = p.cfg.threads_per_line;
    const long long e = strided_kind(p.kind) ? (L - 1) + (T - 1) * p.es : (L - 1) * p.n + (T - 1);
    return (e + 1) * (long long)element_bytes(dtype) <= 0xffffffffLL;
}

// Most blocks a fused multiply pass can launch, over every compiled
// configuration of its length (the autotuner launches each of them, and the
// wisdom may pick any) and the runtime-radix one: one energy partial per
// block.  A persistent grid launches at most its tile count.
long long conv_partials_needed(const PassLaunch &pl, int dtype) {
    long long most = pass_tiles(pl);
    PassLaunch t = pl;
    const int ncand = kernel_candidates(pl.n, kConvZ, dtype);
    for (int c = 0; c < ncand; ++c)
        if (select_kernel(pl.n, kConvZ, dtype, false, c, &t.cfg)) most = std::max(most, pass_tiles(t));
    if (select_generic_conv(pl.n, dtype, &t.cfg)) most = std::max(most, pass_tiles(t));
    return std::max(1LL, most);
}

// The pass list of one grid, without device resources (twiddle pointers are
// filled in later).  Half storage always runs all three axes, so that every
// pass re-scales its lines and the output exponents are per z-line.
int build_passes(const Geometry &g, int dtype, int dir, int flags, std::vector<PassLaunch> *out) {
    const int dims[3] = {g.nx, g.ny, g.nz};
    const long long N = (long long)g.nx * g.ny * g.nz;
    const bool half = is_half(dtype);
    out->clear();
    for (int axis = 0; axis < 3; ++axis) {
        const int n = dims[axis];
        if (n == 1 && !half) continue;
        PassLaunch p;
        p.axis = axis;
        p.n = n;
        p.es = axis == 0 ? 1 : (axis == 1 ? (long long)g.nx : (long long)g.nx * g.ny);
        p.kind = p.es == 1 ? kContiguous : kStrided;
        if (p.kind == kContiguous) {
            p.nlines = N / n;
            p.nw = 1;
        } else {
            p.nlines = p.es;
            p.nw = N / (p.es * n);
        }
        int cand = 0, waves = 1;
        wisdom_lookup(n, p.kind, dtype, dir, wisdom_axis(p.kind, axis), &cand, &waves);
        if (!select_kernel(n, p.kind, dtype, (flags & CROFT_FORCE_GENERIC) != 0, cand, &p.cfg))
            return no_kernel(n, dtype);
        if (!lane_offset_fits(p, dtype) && !select_kernel(n, p.kind, dtype, true, 0, &p.cfg))
            return no_kernel(n, dtype);
        plain_on_partial_lines(p, dtype, &p.cfg);
        p.cfg.grid_waves = waves;
        if (half) {
            ExpMap &m = p.em;
            const long long big = 1LL << 31;  // no wrap
            if (axis == 0) {
                // lines l = y + ny z; input exponents per x-line; output per x-line
                set_exp_qmod(m, big); m.a0 = 1; m.b0 = 1;
            } else if (axis == 1) {
                if (p.kind == kStrided) {  // q = x, w = z, j = y
                    set_exp_qmod(m, big); m.a2 = g.ny; m.a3 = 1; m.b0 = 1; m.b2 = g.nx;
                } else {                   // nx == 1: q = z, j = y
                    set_exp_qmod(m, big); m.a0 = g.ny; m.a3 = 1; m.b0 = 1;
                }
            } else {
                if (p.kind == kStrided) {  // q = x + nx y, j = z
                    set_exp_qmod(m, g.nx); m.a0 = 1; m.a3 = g.nx; m.b0 = 1; m.b1 = g.nx;
                } else {                   // nx == ny == 1: one line, j = z
                    set_exp_qmod(m, big); m.a3 = 1; m.b0 = 1;
                }
            }
        }
        // 16-bit storage: the static contiguous kernels take one input
        // exponent per line; a contiguous pass whose elements come from
        // different lines (y with nx = 1, z with nx = ny = 1) runs the
        // runtime-radix kernel
        if (half && p.kind == kContiguous && p.em.a3 != 0 && !p.cfg.generic &&
            !select_kernel(n, p.kind, dtype, true, 0, &p.cfg))
            return no_kernel(n, dtype);
        out->push_back(p);
    }
    if (out->empty()) {  // 1 x 1 x 1 grid: one length-1 pass copies in to out
        PassLaunch p;
        p.axis = 0;
        p.n = 1;
        p.es = 1;
        p.kind = kContiguous;
        p.nlines = 1;
        if (!select_kernel(1, kContiguous, dtype, true, 0, &p.cfg))
            return fail(CROFT_ERR_INTERNAL, "no kernel for a 1-point grid");
        out->push_back(p);
    }
    return CROFT_SUCCESS;
}

// The pass list of the unfused schedule: along x, y and z in turn, each
// axis's FFT over contiguous lines of the grid as the preceding transposes
// leave it (x fastest, then y fastest, then z fastest).  Length-1 axes keep
// a pass entry that runs nothing.
int build_unfused_passes(const Geometry &g, int dtype, int dir, int flags, std::vector<PassLaunch> *out) {
    const int dims[3] = {g.nx, g.ny, g.nz};
    const long long N = (long long)g.nx * g.ny * g.nz;
    out->clear();
    for (int axis = 0; axis < 3; ++axis) {
        PassLaunch p;
        p.axis = axis;
        p.n = dims[axis];
        p.kind = kContiguous;
        p.es = 1;
        p.nlines = N / p.n;
        p.nw = 1;
        int cand = 0, waves = 1;
        wisdom_lookup(p.n, kContiguous, dtype, dir, -1, &cand, &waves);
        const bool generic = (flags & CROFT_FORCE_GENERIC) != 0 || p.n == 1;
        if (!select_kernel(p.n, kContiguous, dtype, generic, cand, &p.cfg)) return no_kernel(p.n, dtype);
        if (!lane_offset_fits(p, dtype) && !select_kernel(p.n, kContiguous, dtype, true, 0, &p.cfg))
            return no_kernel(p.n, dtype);
        p.cfg.grid_waves = waves;
        out->push_back(p);
    }
    return CROFT_SUCCESS;
}

// The pass list of a real transform of an nx x ny x nz real grid (nx even):
// the real x pass on the half-length complex view, and the complex y and z
// passes on the (nx/2 + 1) x ny x nz half spectrum.  Forward runs x, y, z;
// backward z, y, x.
// tune_dir: the direction the wisdom lookup assumes (0 when the passes run
// in both directions, as in a convolution plan).
int build_real_passes(const Geometry &g, int dtype, int dir, int flags, std::vector<PassLaunch> *out,
                      int tune_dir = 2) {
    if (tune_dir == 2) tune_dir = dir;
    out->clear();
    const int m = g.nx / 2;
    const long long h = (long long)m + 1;  // spectrum elements per x-line
    PassLaunch xp;
    xp.axis = 0;
    xp.n = m;
    xp.kind = kRealX;
    xp.es = 1;
    xp.nlines = (long long)g.ny * g.nz;
    int cand = 0, waves = 1;
    wisdom_lookup(m, kRealX, dtype, tune_dir, -1, &cand, &waves);
    if (!select_kernel(m, kRealX, dtype, false, cand, &xp.cfg))
        return fail(CROFT_ERR_UNSUPPORTED_SIZE, "no real x kernel for nx = %d (half length %d)", g.nx, m);
    xp.cfg.grid_waves = waves;
    std::vector<PassLaunch> yz;
    for (int axis = 1; axis < 3; ++axis) {
        const int n = axis == 1 ? g.ny : g.nz;
        if (n == 1) continue;
        PassLaunch p;
        p.axis = axis;
        p.n = n;
        p.kind = kStrided;
        p.es = axis == 1 ? h : h * g.ny;
        p.nlines = p.es;
        p.nw = axis == 1 ? g.nz : 1;
        wisdom_lookup(n, kStrided, dtype, tune_dir, axis, &cand, &waves);
        if (!select_kernel(n, kStrided, dtype, (flags & CROFT_FORCE_GENERIC) != 0, cand, &p.cfg))
            return no_kernel(n, dtype);
        if (!lane_offset_fits(p, dtype) && !select_kernel(n, kStrided, dtype, true, 0, &p.cfg))
            return no_kernel(n, dtype);
        plain_on_partial_lines(p, dtype, &p.cfg);
        p.cfg.grid_waves = waves;
        yz.push_back(p);
    }
    if (dir == CROFT_FORWARD) {
        out->push_back(xp);
        out->insert(out->end(), yz.begin(), yz.end());
    } else {
        out->insert(out->end(), yz.rbegin(), yz.rend());
        out->push_back(xp);
    }
    return CROFT_SUCCESS;
}

// The pass list of a convolution plan: the forward real passes up to the
// last axis of length > 1 (z, else y), that axis as the fused forward /
// multiply / inverse pass, then the backward passes in reverse order.
int build_conv_passes(const Geometry &g, int dtype, int flags, std::vector<PassLaunch> *out) {
    std::vector<PassLaunch> fwd;
    int rc = build_real_passes(g, dtype, CROFT_FORWARD, flags, &fwd, 0);
    if (rc != CROFT_SUCCESS) return rc;
    if (fwd.size() < 2)
        return fail(CROFT_ERR_UNSUPPORTED_SIZE, "convolution plans need ny > 1 or nz > 1");
    PassLaunch c = fwd.back();  // the last complex pass becomes the fused one
    fwd.pop_back();
    c.kind = kConvZ;
    c.hx = (long long)g.nx / 2 + 1;
    int cand = 0, waves = 1;
    wisdom_lookup(c.n, kConvZ, dtype, 0, -1, &cand, &waves);
    const bool compiled = select_kernel(c.n, kConvZ, dtype, false, cand, &c.cfg);
    if ((!compiled || !lane_offset_fits(c, dtype)) && !select_generic_conv(c.n, dtype, &c.cfg))
        return fail(CROFT_ERR_UNSUPPORTED_SIZE,
                    "no fused multiply kernel for length %d (the fused axis needs a 2^a 3^b 5^c length)", c.n);
    c.cfg.grid_waves = waves;
    out->clear();
    for (PassLaunch pl : fwd) {
        pl.dir = CROFT_FORWARD;
        out->push_back(pl);
    }
    c.dir = CROFT_FORWARD;
    out->push_back(c);
    for (auto it = fwd.rbegin(); it != fwd.rend(); ++it) {
        PassLaunch pl = *it;
        pl.dir = CROFT_BACKWARD;
        out->push_back(pl);
    }
    return CROFT_SUCCESS;
}

int check_real_dims(int nx, int ny, int nz, int dtype) {
    if (dtype != CROFT_C64 && dtype != CROFT_C128)
        return fail(CROFT_ERR_UNSUPPORTED_DTYPE, "real transforms take CROFT_C64 or CROFT_C128");
    if (nx < 4 || nx % 2 != 0 || nx / 2 > kMaxLength)
        return fail(CROFT_ERR_UNSUPPORTED_SIZE, "real transforms need an even nx in 4..%d (got %d)",
                    2 * kMaxLength, nx);
    const int rc = check_dims(nx / 2, ny, nz);
    if (rc != CROFT_SUCCESS) return rc;
    if (((long long)nx / 2 + 1) * ny * nz > 0x7fffffffLL)
        return fail(CROFT_ERR_UNSUPPORTED_SIZE, "half spectrum exceeds 2^31 - 1 elements");
    return CROFT_SUCCESS;
}

// Largest exponent index a pass touches (host-side bound check of ExpMap).
void exp_extent(const PassLaunch &p, long long *in_max, long long *out_max) {
    const ExpMap &m = p.em;
    const long long qmax = p.kind == kContiguous ? p.nlines - 1 : p.es - 1;
    const long long wmax = p.kind == kContiguous ? 0 : p.nw - 1;
    long long imax = 0, omax = 0;
    // the maps are sums of non-negative terms; the maximum over q of
    // (q % qmod) a0 + (q / qmod) a1 is reached at q = qmax or at the largest
    // q with q % qmod == qmod - 1
    const long long cands[2] = {qmax, m.qmod <= qmax ? ((qmax + 1) / m.qmod) * m.qmod - 1 : qmax};
    for (long long q : cands) {
        if (q < 0) continue;
        const long long iq = (q % m.qmod) * m.a0 + (q / m.qmod) * m.a1 + wmax * m.a2 + (p.n - 1) * m.a3;
        const long long oq = (q % m.qmod) * m.b0 + (q / m.qmod) * m.b1 + wmax * m.b2;
        imax = std::max(imax, iq);
        omax = std::max(omax, oq);
    }
    *in_max = imax;
    *out_max = omax;
}

int check_exp_maps(const Geometry &g, const std::vector<PassLaunch> &ps) {
    const long long sizes[4] = {(long long)g.ny * g.nz, (long long)g.ny * g.nz, (long long)g.nx * g.nz,
                                (long long)g.nx * g.ny};
    for (size_t i = 0; i < ps.size(); ++i) {
        // the kernels divide q by qmod with the map's multiply and shift,
        // exact for q < 2^31
        const long long qmax = ps[i].kind == kContiguous ? ps[i].nlines - 1 : ps[i].es - 1;
        if (qmax >= (1LL << 31))
            return fail(CROFT_ERR_INTERNAL, "line index of pass %zu exceeds 2^31 - 1", i);
        long long imax, omax;
        exp_extent(ps[i], &imax, &omax);
        if (imax >= sizes[i] || omax >= sizes[i + 1])
            return fail(CROFT_ERR_INTERNAL, "exponent map of pass %zu out of range", i);
    }
    return CROFT_SUCCESS;
}

// Device memory owned by a plan.  With CROFT_TEST_FAIL_ALLOC=k in the
// environment (k >= 1) the k-th such allocation of a plan creation reports
// hipErrorOutOfMemory without allocating, so tests can drive every
// out-of-memory path of plan creation and its cleanup from the host.
hipError_t plan_alloc(croft_plan *p, void **ptr, size_t bytes) {
    if (p->fail_alloc_at > 0 && ++p->alloc_count == p->fail_alloc_at) {
        *ptr = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(ptr, bytes);
}

void destroy_plan(croft_plan *p) {
    if (!p) return;
    for (auto &kv : p->twiddles) (void)hipFree(kv.second);
    for (auto &kv : p->bluestein) {
        (void)hipFree(kv.second.first);
        (void)hipFree(kv.second.second);
    }
    if (p->e1) (void)hipFree(p->e1);
    if (p->e2) (void)hipFree(p->e2);
    if (p->rwork) (void)hipFree(p->rwork);
    if (p->uwork) (void)hipFree(p->uwork);
    if (p->partial) (void)hipFree(p->partial);
    for (int i = 0; i < 2; ++i) {
        if (p->side[i]) (void)hipStreamDestroy(p->side[i]);
        if (p->join[i]) (void)hipEventDestroy(p->join[i]);
    }
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->graph) (void)hipGraphExecDestroy(p->graph);
    if (p->bitems) (void)hipFree(p->bitems);
    for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
    for (auto &v : p->prof)
        for (auto &pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    delete p;
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

// Kernel attributes (LDS above 64 KiB) and the number of blocks the device
// holds at once, which sizes the persistent grid.
int prepare_kernel(KernelConfig *cfg) {
    hipError_t e;
    const void *fs[2] = {cfg->func, cfg->func_inv};
    for (int i = 0; i < 2; ++i) {
        if (cfg->lds > 65536) {
            e = hipFuncSetAttribute(fs[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)cfg->lds);
            if (e != hipSuccess) return fail_hip(e, "LDS attribute");
        }
    }
    cfg->resident = 0;
    if (!cfg->generic) {
        int nb = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cfg->func, cfg->block, cfg->lds);
        if (e != hipSuccess) return fail_hip(e, "occupancy query");
        if (nb < 1) return fail(CROFT_ERR_INTERNAL, "kernel cannot be resident (block %d, LDS %zu)", cfg->block,
                                cfg->lds);
        cfg->resident = nb * device_cus();
    }
    return CROFT_SUCCESS;
}

// Device resources for the passes of every grid: twiddle tables (one per
// distinct length), exponent scratch, kernel attributes.
int attach_resources(croft_plan *p) {
    hipError_t e;
    const bool dbl = p->dtype == CROFT_C128;
    // the table w_n^m, m < n, of a length, uploaded once per plan
    auto table = [&](int n, const void **out) -> int {
        if (!p->twiddles.count(n)) {
            std::vector<double> w(2 * (size_t)n);
            twiddles_fp64(n, w.data());
            void *d = nullptr;
            const size_t bytes = (size_t)n * compute_bytes(p->dtype);
            if ((e = plan_alloc(p, &d, bytes)) != hipSuccess) {
                (void)hipGetLastError();
                return fail(CROFT_ERR_OUT_OF_MEMORY, "twiddle table: %s", hipGetErrorString(e));
            }
            p->twiddles[n] = d;
            p->work_bytes += bytes;
            if (dbl) {
                e = hipMemcpy(d, w.data(), bytes, hipMemcpyHostToDevice);
            } else {
                std::vector<float> f(w.size());
                round_to_fp32(w.data(), w.size(), f.data());
                e = hipMemcpy(d, f.data(), bytes, hipMemcpyHostToDevice);
            }
            if (e != hipSuccess) return fail_hip(e, "twiddle upload");
        }
        *out = p->twiddles[n];
        return CROFT_SUCCESS;
    };
    // Bluestein's chirp and kernel DFT of a length (convolution length m)
    auto upload = [&](const std::vector<double> &v, void **out) -> int {
        const size_t count = v.size() / 2;
        const size_t bytes = count * compute_bytes(p->dtype);
        if ((e = plan_alloc(p, out, bytes)) != hipSuccess) {
            (void)hipGetLastError();
            *out = nullptr;
            return fail(CROFT_ERR_OUT_OF_MEMORY, "Bluestein table: %s", hipGetErrorString(e));
        }
        p->work_bytes += bytes;
        if (dbl) {
            e = hipMemcpy(*out, v.data(), bytes, hipMemcpyHostToDevice);
        } else {
            std::vector<float> f(v.size());
            round_to_fp32(v.data(), v.size(), f.data());
            e = hipMemcpy(*out, f.data(), bytes, hipMemcpyHostToDevice);
        }
        return e == hipSuccess ? CROFT_SUCCESS : fail_hip(e, "Bluestein table upload");
    };
    auto blue = [&](int n, int m, PassLaunch *pl) -> int {
        if (!p->bluestein.count(n)) {
            std::vector<double> c(2 * (size_t)n), b(2 * (size_t)m);
            bluestein_tables_fp64(n, m, c.data(), b.data());
            std::pair<void *, void *> t{nullptr, nullptr};
            int rc = upload(c, &t.first);
            if (rc == CROFT_SUCCESS) rc = upload(b, &t.second);
            if (rc != CROFT_SUCCESS) {
                if (t.first) (void)hipFree(t.first);
                return rc;
            }
            p->bluestein[n] = t;
        }
        pl->chirp = p->bluestein[n].first;
        pl->bhat = p->bluestein[n].second;
        return CROFT_SUCCESS;
    };
    for (auto &ps : p->passes) {
        for (PassLaunch &pl : ps) {
            int rc;
            pl.tw = nullptr;
            if (pl.cfg.bluestein) {
                if ((rc = table(pl.cfg.bluestein, &pl.tw)) != CROFT_SUCCESS) return rc;
                if ((rc = blue(pl.n, pl.cfg.bluestein, &pl)) != CROFT_SUCCESS) return rc;
            } else if (pl.n > 1 && (rc = table(pl.n, &pl.tw)) != CROFT_SUCCESS) {
                return rc;
            }
            if (pl.kind == kRealX && (rc = table(2 * pl.n, &pl.tw2)) != CROFT_SUCCESS) return rc;
            if ((rc = prepare_kernel(&pl.cfg)) != CROFT_SUCCESS) return rc;
        }
    }
    if (p->conv) {
        long long count = 1;
        for (const PassLaunch &pl : p->passes[0])
            if (pl.kind == kConvZ) count = std::max(count, conv_partials_needed(pl, p->dtype));
        if ((e = plan_alloc(p, (void **)&p->partial, sizeof(double) * (size_t)count)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CROFT_ERR_OUT_OF_MEMORY, "energy partials: %s", hipGetErrorString(e));
        }
        p->partial_count = count;
        p->work_bytes += sizeof(double) * (size_t)count;
    }
    if (p->real && (p->dir == CROFT_BACKWARD || p->conv) && p->passes[0].size() > 1) {
        const Geometry &g = p->grids[0];
        const size_t bytes = ((size_t)g.nx / 2 + 1) * g.ny * g.nz * compute_bytes(p->dtype);
        if ((e = plan_alloc(p, &p->rwork, bytes)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CROFT_ERR_OUT_OF_MEMORY, "real backward work buffer: %s", hipGetErrorString(e));
        }
        p->work_bytes += bytes;
    }
    if (p->unfused) {
        const Geometry &g = p->grids[0];
        const size_t bytes = (size_t)g.nx * g.ny * g.nz * element_bytes(p->dtype);
        if ((e = plan_alloc(p, &p->uwork, bytes)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CROFT_ERR_OUT_OF_MEMORY, "unfused work grid: %s", hipGetErrorString(e));
        }
        p->work_bytes += bytes;
    }
    if (is_half(p->dtype)) {
        const Geometry &g = p->grids[0];
        const size_t b1 = (size_t)g.ny * g.nz, b2 = (size_t)g.nx * g.nz;
        if ((e = plan_alloc(p, (void **)&p->e1, b1)) != hipSuccess || (e = plan_alloc(p, (void **)&p->e2, b2)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CROFT_ERR_OUT_OF_MEMORY, "exponent scratch: %s", hipGetErrorString(e));
        }
        p->work_bytes += b1 + b2;
        // the allocation-free execute's exponents: the device's static array
        if ((e = noalloc_scratch(p->device, &p->scratch)) != hipSuccess)
            return fail_hip(e, "static scratch address");
    }
    if (p->slabs > 1 || (p->slab_auto && (p->flags & CROFT_MEASURE))) {
        for (int i = 0; i < 2; ++i) {
            if ((e = hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking)) != hipSuccess)
                return fail_hip(e, "stream create");
            if ((e = hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming)) != hipSuccess)
                return fail_hip(e, "event create");
        }
        if ((e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming)) != hipSuccess)
            return fail_hip(e, "event create");
    }
    return CROFT_SUCCESS;
}

// CROFT_MEASURE: time every compiled configuration of each distinct pass
// (candidate x persistent grid size, forward and inverse) on scratch buffers,
// keep the fastest and record it as wisdom.
int measure_passes(croft_plan *p) {
    size_t maxN = 0, maxE = 1;
    for (const Geometry &g : p->grids) {
        maxN = std::max(maxN, (size_t)g.nx * g.ny * g.nz);
        maxE = std::max({maxE, (size_t)g.ny * g.nz, (size_t)g.nx * g.nz, (size_t)g.nx * g.ny});
    }
    const size_t bytes = maxN * element_bytes(p->dtype);
    void *a = nullptr, *b = nullptr;
    int8_t *ei = nullptr, *eo = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int rc = CROFT_SUCCESS;
    auto cleanup = [&]() {
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        if (ei) (void)hipFree(ei);
        if (eo) (void)hipFree(eo);
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
    };
    if (plan_alloc(p, &a, bytes) != hipSuccess || plan_alloc(p, &b, bytes) != hipSuccess ||
        plan_alloc(p, (void **)&ei, maxE) != hipSuccess || plan_alloc(p, (void **)&eo, maxE) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(CROFT_ERR_OUT_OF_MEMORY, "autotune scratch of %zu bytes", 2 * bytes);
    }
    hipError_t e;
    if ((e = hipMemset(a, 0, bytes)) != hipSuccess || (e = hipMemset(ei, 0, maxE)) != hipSuccess ||
        (e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) {
        cleanup();
        return fail_hip(e, "autotune setup");
    }
    const bool persist = !(p->flags & CROFT_NO_WISDOM);
    const bool inv = p->dir == CROFT_BACKWARD;
    // (n, kind, wisdom axis) -> configuration: strided passes are tuned per
    // axis, as their strides differ
    std::map<std::tuple<int, int, int>, KernelConfig> best;
    for (auto &ps : p->passes) {
        for (PassLaunch &pl : ps) {
            const int wax = wisdom_axis(pl.kind, pl.axis);
            if (pl.cfg.generic || best.count({pl.n, pl.kind, wax})) continue;
            const int ncand = kernel_candidates(pl.n, pl.kind, p->dtype);
            float best_ms = 1e30f;
            KernelConfig pick = pl.cfg;
            // every pass of the plan with this (length, kind, axis): a choice
            // is timed on all the geometries it will run (e.g. the z passes of
            // every grid of a batched plan)
            std::vector<const PassLaunch *> same;
            for (auto &ps2 : p->passes)
                for (const PassLaunch &q : ps2)
                    if (q.n == pl.n && q.kind == pl.kind && wisdom_axis(q.kind, q.axis) == wax) same.push_back(&q);
            for (int c = 0; c < ncand && rc == CROFT_SUCCESS; ++c) {
                KernelConfig cfg;
                if (!select_kernel(pl.n, pl.kind, p->dtype, false, c, &cfg) || cfg.candidate != c) continue;
                bool fits = true;
                for (const PassLaunch *q : same) {
                    PassLaunch t = *q;
                    t.cfg = cfg;
                    fits = fits && lane_offset_fits(t, p->dtype);
                    // a candidate some pass would swap for its plain twin is not timed
                    KernelConfig tw = cfg;
                    plain_on_partial_lines(t, p->dtype, &tw);
                    fits = fits && tw.candidate == cfg.candidate;
                }
                if (!fits) continue;
                if ((rc = prepare_kernel(&cfg)) != CROFT_SUCCESS) break;
                // a choice serves both directions (the wisdom key has none), and
                // the two instantiations of a configuration can differ in speed
                // (e.g. one spills registers), so both are timed
                const int ndir = cfg.func_inv != cfg.func ? 2 : 1;
                for (int waves : {1, 2, 4, 0}) {
                    float total = 0.f;
                    for (const PassLaunch *q : same) {
                        PassLaunch t = *q;
                        t.cfg = cfg;
                        t.cfg.grid_waves = waves;
                        if (t.kind == kConvZ && pass_blocks(t) > p->partial_count) {
                            rc = fail(CROFT_ERR_INTERNAL, "fused pass of %lld blocks exceeds %lld energy partials",
                                      pass_blocks(t), p->partial_count);
                            break;
                        }
                        for (int d = 0; d < ndir && e == hipSuccess; ++d) {
                            const int iv = ndir == 2 ? d : (int)inv;
                            float best_rep = 1e30f;
                            e = launch_pass(t, p->dtype, a, b, ei, eo, iv, 0, a, p->partial);  // warm-up
                            for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
                                float ms = 0.f;
                                e = hipEventRecord(t0, 0);
                                if (e == hipSuccess) e = launch_pass(t, p->dtype, a, b, ei, eo, iv, 0, a, p->partial);
                                if (e == hipSuccess) e = hipEventRecord(t1, 0);
                                if (e == hipSuccess) e = hipEventSynchronize(t1);
                                if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
                                best_rep = std::min(best_rep, ms);
                            }
                            total += best_rep;
                        }
                        if (e != hipSuccess) break;
                    }
                    if (rc != CROFT_SUCCESS) break;
                    if (e != hipSuccess) {
                        rc = fail_hip(e, "autotune launch");
                        break;
                    }
                    if (total < best_ms) {
                        best_ms = total;
                        pick = cfg;
                        pick.grid_waves = waves;
                    }
                }
            }
            if (rc != CROFT_SUCCESS) break;
            best[{pl.n, pl.kind, wax}] = pick;
            wisdom_record(pl.n, pl.kind, p->dtype, wax, pick.candidate, pick.grid_waves, persist);
        }
    }
    cleanup();
    if (rc != CROFT_SUCCESS) return rc;
    for (auto &ps : p->passes)
        for (PassLaunch &pl : ps) {
            if (pl.cfg.generic) continue;  // a pass the planner sent to the runtime-radix kernel keeps it
            auto it = best.find({pl.n, pl.kind, wisdom_axis(pl.kind, pl.axis)});
            if (it != best.end()) pl.cfg = it->second;
        }
    return CROFT_SUCCESS;
}

int run_grid(croft_plan *p, size_t gi, const char *in, char *out, const int8_t *in_exp, int8_t *out_exp,
             hipStream_t s, std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof, int8_t *e1 = nullptr,
             int8_t *e2 = nullptr);
int run_slabs(croft_plan *p, const char *in, char *out, const int8_t *in_exp, int8_t *out_exp, hipStream_t s,
              std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof, int8_t *e1 = nullptr, int8_t *e2 = nullptr);

// The slab counts a grid can take: 1, 2, 4, 8, 16 where they divide nz.
std::vector<int> slab_candidates(int nz) {
    std::vector<int> ks;
    for (int k : {1, 2, 4, 8, 16})
        if (nz % k == 0) ks.push_back(k);
    return ks;
}

// CROFT_MEASURE with K = 0: time the whole transform (the plan's direction,
// its chosen pass configurations) under each slab count on scratch buffers,
// keep the fastest (best of five runs each) and record it as wisdom.
int measure_slabs(croft_plan *p) {
    const Geometry &g = p->grids[0];
    const std::vector<int> ks = slab_candidates(g.nz);
    const size_t bytes = (size_t)g.nx * g.ny * g.nz * element_bytes(p->dtype);
    const size_t ebytes = std::max((size_t)g.ny * g.nz, (size_t)g.nx * g.ny);
    void *a = nullptr, *b = nullptr;
    int8_t *ei = nullptr, *eo = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    auto cleanup = [&]() {
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        if (ei) (void)hipFree(ei);
        if (eo) (void)hipFree(eo);
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
    };
    if (ks.size() > 1) {
        if (plan_alloc(p, &a, bytes) != hipSuccess || plan_alloc(p, &b, bytes) != hipSuccess ||
            plan_alloc(p, (void **)&ei, ebytes) != hipSuccess || plan_alloc(p, (void **)&eo, ebytes) != hipSuccess) {
            (void)hipGetLastError();
            cleanup();
            return fail(CROFT_ERR_OUT_OF_MEMORY, "slab autotune scratch of %zu bytes", 2 * bytes);
        }
        hipError_t e;
        if ((e = hipMemset(a, 0, bytes)) != hipSuccess || (e = hipMemset(ei, 0, ebytes)) != hipSuccess ||
            (e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) {
            cleanup();
            return fail_hip(e, "slab autotune setup");
        }
    }
    int best_k = 1;
    float best_ms = 1e30f;
    int rc = CROFT_SUCCESS;
    for (size_t i = 0; i < ks.size() && ks.size() > 1 && rc == CROFT_SUCCESS; ++i) {
        p->slabs = ks[i];
        auto once = [&]() {
            return ks[i] > 1 ? run_slabs(p, (const char *)a, (char *)b, ei, eo, nullptr, nullptr)
                             : run_grid(p, 0, (const char *)a, (char *)b, ei, eo, nullptr, nullptr);
        };
        if ((rc = once()) != CROFT_SUCCESS) break;  // warm-up
        float best_rep = 1e30f;
        for (int rep = 0; rep < 5 && rc == CROFT_SUCCESS; ++rep) {
            float ms = 0.f;
            hipError_t e = hipEventRecord(t0, nullptr);
            if (e == hipSuccess && (rc = once()) != CROFT_SUCCESS) break;
            if (e == hipSuccess) e = hipEventRecord(t1, nullptr);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e != hipSuccess) rc = fail_hip(e, "slab autotune timing");
            best_rep = std::min(best_rep, ms);
        }
        if (best_rep < best_ms) {
            best_ms = best_rep;
            best_k = ks[i];
        }
    }
    cleanup();
    if (rc != CROFT_SUCCESS) return rc;
    p->slabs = best_k;
    slab_wisdom_record(g.nx, g.ny, g.nz, p->dtype, best_k, !(p->flags & CROFT_NO_WISDOM));
    return CROFT_SUCCESS;
}

// Batched plans: the segment table of the batched kernels (one segment per
// grid and pass, pass by pass) for the plan's tile shapes, uploaded; the
// launch LDS of each pass and the cooperative launch's grid size.
int upload_batch_tables(croft_plan *p) {
    const size_t ib = batch_item_bytes();
    std::vector<char> host;
    int nseg = 0;
    for (int i = 0; i < 3; ++i) {
        p->btiles[i] = 0;
        p->blds[i] = 0;
    }
    for (int i = 0; i < 3; ++i) {
        p->bbegin[i] = nseg;
        for (size_t g : p->bgrids) {
            const std::vector<PassLaunch> &ps = p->passes[g];
            if ((size_t)i >= ps.size()) continue;
            const PassLaunch &pl = ps[i];
            BatchConfig bc;
            const int code = batch_code(pl.n, pl.kind, p->bshape[{pl.n, pl.kind}]);
            if (!batch_config(code, p->dtype, &bc)) return fail(CROFT_ERR_INTERNAL, "batch configuration %d", code);
            long long ntiles, total;
            if (pl.kind == kContiguous) {
                ntiles = 1;
                total = (pl.nlines + bc.lines - 1) / bc.lines;
            } else {
                ntiles = (pl.es + bc.lines - 1) / bc.lines;
                total = ntiles * pl.nw;
            }
            host.resize(host.size() + ib);
            batch_item_fill(host.data() + host.size() - ib, (long long)p->offsets[g], p->btiles[i], pl.es,
                            pl.kind == kContiguous ? pl.nlines : pl.es, pl.nw, ntiles, total, pl.tw, code, i == 0);
            ++nseg;
            p->btiles[i] += total;
            p->blds[i] = std::max(p->blds[i], bc.lds);
        }
    }
    p->bbegin[3] = nseg;
    if (!nseg) return CROFT_SUCCESS;
    hipError_t e;
    if (!p->bitems) {
        // every shape choice gives the same number of segments
        if ((e = plan_alloc(p, &p->bitems, host.size())) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CROFT_ERR_OUT_OF_MEMORY, "batch tables: %s", hipGetErrorString(e));
        }
        p->work_bytes += host.size();
    }
    if ((e = hipMemcpy(p->bitems, host.data(), host.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return fail_hip(e, "batch table upload");
    const size_t lds = std::max({p->blds[0], p->blds[1], p->blds[2]});
    int nb = 1 << 30;
    for (int inv = 0; inv < 2; ++inv) {
        const void *fs[2] = {batch_kernel(p->dtype, inv), batch_coop_kernel(p->dtype, inv)};
        for (const void *f : fs) {
            if (lds > 65536 &&
                (e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
                return fail_hip(e, "LDS attribute");
        }
        // the cooperative grid must fit at once: the smaller occupancy of the
        // two directions, at the largest LDS any pass needs
        int n = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fs[1], 256, lds)) != hipSuccess)
            return fail_hip(e, "occupancy query");
        nb = std::min(nb, n);
    }
    if (nb < 1) return fail(CROFT_ERR_INTERNAL, "the cooperative batched kernel cannot be resident");
    p->bresident = nb * std::max(1, device_cus());
    return CROFT_SUCCESS;
}

int run_batch(croft_plan *p, const void *in, void *out, hipStream_t s,
              std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof);

// CROFT_MEASURE on a batched plan: for each (length, kind) of the batched
// kernel in the batch, time the whole batch (its own launch form) with each
// compiled tile shape of that pair, the others at their current choice; keep
// the fastest (best of five) and record it as wisdom (kind 4 + kind).
int measure_batch_shapes(croft_plan *p) {
    const size_t bytes = p->offsets.back() * element_bytes(p->dtype);
    void *a = nullptr, *b = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    auto cleanup = [&]() {
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
    };
    hipError_t e;
    if (plan_alloc(p, &a, bytes) != hipSuccess || plan_alloc(p, &b, bytes) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(CROFT_ERR_OUT_OF_MEMORY, "batch autotune scratch of %zu bytes", 2 * bytes);
    }
    if ((e = hipMemset(a, 0, bytes)) != hipSuccess || (e = hipEventCreate(&t0)) != hipSuccess ||
        (e = hipEventCreate(&t1)) != hipSuccess) {
        cleanup();
        return fail_hip(e, "batch autotune setup");
    }
    int rc = CROFT_SUCCESS;
    const bool persist = !(p->flags & CROFT_NO_WISDOM);
    for (auto &kv : p->bshape) {
        float best = 1e30f;
        int pick = kv.second;
        for (int shape = 0; shape < batch_shape_count(p->dtype) && rc == CROFT_SUCCESS; ++shape) {
            kv.second = shape;
            if ((rc = upload_batch_tables(p)) != CROFT_SUCCESS) break;
            if ((rc = run_batch(p, a, b, nullptr, nullptr)) != CROFT_SUCCESS) break;  // warm-up
            float best_rep = 1e30f;
            for (int rep = 0; rep < 5 && rc == CROFT_SUCCESS; ++rep) {
                float ms = 0.f;
                e = hipEventRecord(t0, nullptr);
                if (e == hipSuccess && (rc = run_batch(p, a, b, nullptr, nullptr)) != CROFT_SUCCESS) break;
                if (e == hipSuccess) e = hipEventRecord(t1, nullptr);
                if (e == hipSuccess) e = hipEventSynchronize(t1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
                if (e != hipSuccess) rc = fail_hip(e, "batch autotune timing");
                best_rep = std::min(best_rep, ms);
            }
            if (best_rep < best) {
                best = best_rep;
                pick = shape;
            }
        }
        if (rc != CROFT_SUCCESS) break;
        kv.second = pick;
        wisdom_record(kv.first.first, kBatchWisdomKind + kv.first.second, p->dtype, -1, pick, 0, persist);
    }
    cleanup();
    if (rc != CROFT_SUCCESS) return rc;
    return upload_batch_tables(p);
}

// Batched plans: which grids the batched kernel runs (the others run with
// launches of their own), each (length, kind)'s tile shape (wisdom, else
// shape 0; CROFT_MEASURE times them), and the uploaded tables.
int build_batch_tables(croft_plan *p) {
    const bool usable = (p->dtype == CROFT_C64 || p->dtype == CROFT_C128) && !(p->flags & CROFT_FORCE_GENERIC);
    for (size_t g = 0; g < p->grids.size(); ++g) {
        const std::vector<PassLaunch> &ps = p->passes[g];
        bool ok = usable && ps.size() <= 3;
        for (const PassLaunch &pl : ps) ok = ok && batch_code(pl.n, pl.kind) >= 0;
        (ok ? p->bgrids : p->loose).push_back(g);
    }
    for (size_t g : p->bgrids)
        for (const PassLaunch &pl : p->passes[g]) {
            int shape = 0, waves = 0;
            if (!wisdom_lookup(pl.n, kBatchWisdomKind + pl.kind, p->dtype, p->dir, -1, &shape, &waves) || shape < 0 ||
                shape >= batch_shape_count(p->dtype))
                shape = 0;
            p->bshape[{pl.n, pl.kind}] = shape;
        }
    int rc = upload_batch_tables(p);
    if (rc == CROFT_SUCCESS && (p->flags & CROFT_MEASURE) && p->bbegin[3] > 0) rc = measure_batch_shapes(p);
    return rc;
}

croft_plan *new_plan(const std::vector<Geometry> &grids, int dtype, int dir, int flags, int slabs,
                     bool batched = false, bool real = false, bool conv = false) {
    croft_plan *p = new (std::nothrow) croft_plan;
    if (!p) {
        fail(CROFT_ERR_OUT_OF_MEMORY, "host allocation failed");
        return nullptr;
    }
    p->dtype = dtype;
    p->dir = dir;
    p->flags = flags;
    p->slabs = slabs;
    p->grids = grids;
    p->offsets.assign(1, 0);
    for (const Geometry &g : grids) p->offsets.push_back(p->offsets.back() + (size_t)g.nx * g.ny * g.nz);
    p->passes.resize(grids.size());
    p->real = real || conv;
    p->conv = conv;
    p->unfused = (flags & CROFT_UNFUSED) != 0;
    for (size_t i = 0; i < grids.size(); ++i) {
        const int rc = conv                         ? build_conv_passes(grids[i], dtype, flags, &p->passes[i])
                       : real                       ? build_real_passes(grids[i], dtype, dir, flags, &p->passes[i])
                       : (flags & CROFT_UNFUSED) != 0 ? build_unfused_passes(grids[i], dtype, dir, flags, &p->passes[i])
                                                      : build_passes(grids[i], dtype, dir, flags, &p->passes[i]);
        if (rc != CROFT_SUCCESS) {
            delete p;
            return nullptr;
        }
        if (is_half(dtype) && check_exp_maps(grids[i], p->passes[i]) != CROFT_SUCCESS) {
            delete p;
            return nullptr;
        }
    }
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        fail_hip(e, "hipGetDevice");
        delete p;
        return nullptr;
    }
    p->batched = batched;
    if (const char *fa = std::getenv("CROFT_TEST_FAIL_ALLOC")) p->fail_alloc_at = std::atoi(fa);
    if (slabs == 0) {
        // K left to the plan: a recorded choice for this grid, else 1;
        // CROFT_MEASURE times every K below
        p->slab_auto = true;
        int k = 1;
        p->slabs = slab_wisdom_lookup(grids[0].nx, grids[0].ny, grids[0].nz, dtype, &k) ? k : 1;
    }
    if (attach_resources(p) != CROFT_SUCCESS || ((flags & CROFT_MEASURE) && measure_passes(p) != CROFT_SUCCESS) ||
        (p->slab_auto && (flags & CROFT_MEASURE) && measure_slabs(p) != CROFT_SUCCESS) ||
        (p->batched && build_batch_tables(p) != CROFT_SUCCESS)) {
        const std::string msg = g_last_error;
        const int status = g_last_status;
        destroy_plan(p);
        g_last_error = msg;
        g_last_status = status;
        return nullptr;
    }
    return p;
}

// ---------------------------------------------------------------- execute
hipEvent_t pool_event(croft_plan *p) {
    hipEvent_t e = nullptr;
    if (!p->event_pool.empty()) {
        e = p->event_pool.back();
        p->event_pool.pop_back();
        return e;
    }
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch one pass over elements [off, off + ...) of a grid.
int run_pass(croft_plan *p, const PassLaunch &pl, const void *in, void *out, const int8_t *ie, int8_t *oe,
             hipStream_t s, std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof, const void *mul = nullptr) {
    hipEvent_t a = nullptr, b = nullptr;
    if (prof) {
        a = pool_event(p);
        b = pool_event(p);
        if (!a || !b) return fail(CROFT_ERR_HIP, "profiling event creation failed");
        (void)hipEventRecord(a, s);
    }
    if (pl.kind == kConvZ && pass_blocks(pl) > p->partial_count)
        return fail(CROFT_ERR_INTERNAL, "fused pass of %lld blocks exceeds %lld energy partials", pass_blocks(pl),
                    p->partial_count);
    const int dir = pl.dir ? pl.dir : p->dir;
    const hipError_t e = launch_pass(pl, p->dtype, in, out, ie, oe, dir == CROFT_BACKWARD, s, mul, p->partial);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    const hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return fail_hip(e2, "kernel launch");
    if (prof) {
        (void)hipEventRecord(b, s);
        prof->push_back({a, b});
    }
    return CROFT_SUCCESS;
}

// Plain schedule of one grid: each pass over the whole grid, the first
// reading `in`, the rest working in place on `out`.  Half storage: the
// intermediate exponents go to e1 (after x) and e2 (after y); NULL takes the
// plan's own arrays.
int run_grid(croft_plan *p, size_t gi, const char *in, char *out, const int8_t *in_exp, int8_t *out_exp,
             hipStream_t s, std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof, int8_t *e1, int8_t *e2) {
    const std::vector<PassLaunch> &ps = p->passes[gi];
    const bool half = is_half(p->dtype);
    if (!e1) e1 = p->e1;
    if (!e2) e2 = p->e2;
    if (p->real && p->dir == CROFT_BACKWARD) {
        // complex passes from `in` into the work buffer, the real x pass from
        // there into `out`
        for (size_t i = 0; i < ps.size(); ++i) {
            const bool last = i + 1 == ps.size();
            const void *src = i == 0 ? (const void *)in : (const void *)p->rwork;
            void *dst = last ? (void *)out : p->rwork;
            const int rc = run_pass(p, ps[i], src, dst, nullptr, nullptr, s, prof);
            if (rc != CROFT_SUCCESS) return rc;
        }
        return CROFT_SUCCESS;
    }
    for (size_t i = 0; i < ps.size(); ++i) {
        const void *src = i == 0 ? (const void *)in : (const void *)out;
        const int8_t *ie = nullptr;
        int8_t *oe = nullptr;
        if (half) {
            ie = i == 0 ? in_exp : (i == 1 ? e1 : e2);
            oe = i == 0 ? e1 : (i == 1 ? e2 : out_exp);
        }
        const int rc = run_pass(p, ps[i], src, out, ie, oe, s, prof);
        if (rc != CROFT_SUCCESS) return rc;
    }
    return CROFT_SUCCESS;
}

// Convolution plan: `in` -> work buffer (forward x pass), complex passes and
// the fused pass in place there, work buffer -> `out` (backward x pass), then
// the energy sum.
int run_conv(croft_plan *p, const void *in, const void *mul, void *out, double *energy, hipStream_t s,
             std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof) {
    const std::vector<PassLaunch> &ps = p->passes[0];
    for (size_t i = 0; i < ps.size(); ++i) {
        const void *src = i == 0 ? in : (const void *)p->rwork;
        void *dst = i + 1 == ps.size() ? out : p->rwork;
        const int rc = run_pass(p, ps[i], src, dst, nullptr, nullptr, s, prof, mul);
        if (rc != CROFT_SUCCESS) return rc;
        if (ps[i].kind == kConvZ && energy) {
            const hipError_t e = launch_sum_partials(p->partial, (int)pass_blocks(ps[i]), energy, s);
            if (e != hipSuccess) return fail_hip(e, "energy sum launch");
        }
    }
    return CROFT_SUCCESS;
}

// Slab schedule (K = p->slabs): the x and y passes slab by slab along z on two
// side streams, then the z pass over the whole grid on the caller's stream.
// e1, e2 as for run_grid.
int run_slabs(croft_plan *p, const char *in, char *out, const int8_t *in_exp, int8_t *out_exp, hipStream_t s,
              std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof, int8_t *e1, int8_t *e2) {
    const Geometry &g = p->grids[0];
    if (!e1) e1 = p->e1;
    if (!e2) e2 = p->e2;
    const std::vector<PassLaunch> &ps = p->passes[0];
    const bool half = is_half(p->dtype);
    const size_t eb = element_bytes(p->dtype);
    const int K = p->slabs;
    const int dz = g.nz / K;
    // passes along x and y (those with axis < 2), and the z pass if present
    std::vector<const PassLaunch *> xy;
    const PassLaunch *zp = nullptr;
    for (const PassLaunch &pl : ps) (pl.axis < 2 ? xy.push_back(&pl) : (void)(zp = &pl));
    hipError_t e;
    if ((e = hipEventRecord(p->fork, s)) != hipSuccess) return fail_hip(e, "event record");
    for (int i = 0; i < 2; ++i)
        if ((e = hipStreamWaitEvent(p->side[i], p->fork, 0)) != hipSuccess) return fail_hip(e, "stream wait");
    for (int k = 0; k < K; ++k) {
        hipStream_t ss = p->side[k & 1];
        const long long z0 = (long long)k * dz;
        const size_t off = (size_t)z0 * g.nx * g.ny * eb;
        for (size_t i = 0; i < xy.size(); ++i) {
            PassLaunch pl = *xy[i];
            if (pl.kind == kContiguous) pl.nlines = pl.nlines / K;
            else pl.nw = pl.nw / K;
            const void *src = i == 0 ? (const void *)(in + off) : (const void *)(out + off);
            const int8_t *ie = nullptr;
            int8_t *oe = nullptr;
            if (half) {
                // x pass: exponents per x-line (y + ny z); y pass: per y-line (x + nx z)
                if (pl.axis == 0) {
                    ie = in_exp ? in_exp + z0 * g.ny : nullptr;
                    oe = e1 + z0 * g.ny;
                } else {
                    ie = e1 + z0 * g.ny;
                    oe = e2 + z0 * g.nx;
                }
            }
            const int rc = run_pass(p, pl, src, out + off, ie, oe, ss, prof);
            if (rc != CROFT_SUCCESS) return rc;
        }
    }
    for (int i = 0; i < 2; ++i) {
        if ((e = hipEventRecord(p->join[i], p->side[i])) != hipSuccess) return fail_hip(e, "event record");
        if ((e = hipStreamWaitEvent(s, p->join[i], 0)) != hipSuccess) return fail_hip(e, "stream wait");
    }
    if (zp) {
        const void *src = xy.empty() ? (const void *)in : (const void *)out;
        const int rc = run_pass(p, *zp, src, out, half ? e2 : nullptr, half ? out_exp : nullptr, s, prof);
        if (rc != CROFT_SUCCESS) return rc;
    }
    return CROFT_SUCCESS;
}

// One standalone transpose (profiled like a pass).
int run_permute(croft_plan *p, const void *in, void *out, const long long d[3], const long long so[3], int b,
                hipStream_t s, std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof) {
    hipEvent_t a = nullptr, e2 = nullptr;
    if (prof) {
        a = pool_event(p);
        e2 = pool_event(p);
        if (!a || !e2) return fail(CROFT_ERR_HIP, "profiling event creation failed");
        (void)hipEventRecord(a, s);
    }
    hipError_t e = launch_permute(p->dtype, in, out, d, so, b, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "transpose launch");
    if (prof) {
        (void)hipEventRecord(e2, s);
        prof->push_back({a, e2});
    }
    return CROFT_SUCCESS;
}

// Unfused schedule (the paper's Option 2, Section 5.1): six sweeps.
//   FFT along x (contiguous)        in   -> work    (x, y, z), x fastest
//   transpose to y fastest          work -> out     (y, x, z)
//   FFT along y (contiguous)        out, in place
//   transpose to z fastest          out  -> work    (z, x, y)
//   FFT along z (contiguous)        work, in place
//   transpose back to x fastest     work -> out     (x, y, z)
// A length-1 axis skips its FFT (the first transpose then reads `in`).
int run_unfused(croft_plan *p, const char *in, char *out, hipStream_t s,
                std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof) {
    const Geometry &g = p->grids[0];
    const std::vector<PassLaunch> &ps = p->passes[0];
    const long long nx = g.nx, ny = g.ny, nz = g.nz;
    char *w = static_cast<char *>(p->uwork);
    int rc;
    const char *cur = in;
    if (ps[0].n > 1) {
        if ((rc = run_pass(p, ps[0], in, w, nullptr, nullptr, s, prof)) != CROFT_SUCCESS) return rc;
        cur = w;
    }
    {   // (x, y, z) -> (y, x, z): offset y + ny (x + nx z)
        const long long d[3] = {nx, ny, nz}, so[3] = {ny, 1, ny * nx};
        if ((rc = run_permute(p, cur, out, d, so, 1, s, prof)) != CROFT_SUCCESS) return rc;
    }
    if (ps[1].n > 1 && (rc = run_pass(p, ps[1], out, out, nullptr, nullptr, s, prof)) != CROFT_SUCCESS) return rc;
    {   // (y, x, z) -> (z, x, y): offset z + nz (x + nx y)
        const long long d[3] = {ny, nx, nz}, so[3] = {nz * nx, nz, 1};
        if ((rc = run_permute(p, out, w, d, so, 2, s, prof)) != CROFT_SUCCESS) return rc;
    }
    if (ps[2].n > 1 && (rc = run_pass(p, ps[2], w, w, nullptr, nullptr, s, prof)) != CROFT_SUCCESS) return rc;
    {   // (z, x, y) -> (x, y, z): offset x + nx (y + ny z)
        const long long d[3] = {nz, nx, ny}, so[3] = {nx * ny, 1, nx};
        if ((rc = run_permute(p, w, out, d, so, 1, s, prof)) != CROFT_SUCCESS) return rc;
    }
    return CROFT_SUCCESS;
}

// All transforms of a batched plan: one launch per pass for the grids the
// batched kernel compiles, then the remaining grids with their own launches.
int run_batch(croft_plan *p, const void *in, void *out, hipStream_t s,
              std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof) {
    const size_t eb = element_bytes(p->dtype);
    const int inv = p->dir == CROFT_BACKWARD;
    const size_t ib = batch_item_bytes();
    const int nlaunch = (p->flags & CROFT_PERSISTENT) ? (p->bbegin[3] > 0 ? 1 : 0) : 3;
    for (int i = 0; i < nlaunch; ++i) {
        const int n = p->bbegin[i + 1] - p->bbegin[i];
        if (!(p->flags & CROFT_PERSISTENT) && n == 0) continue;
        hipEvent_t a = nullptr, b = nullptr;
        if (prof) {
            a = pool_event(p);
            b = pool_event(p);
            if (!a || !b) return fail(CROFT_ERR_HIP, "profiling event creation failed");
            (void)hipEventRecord(a, s);
        }
        hipError_t e;
        if (p->flags & CROFT_PERSISTENT) {
            const size_t lds = std::max({p->blds[0], p->blds[1], p->blds[2]});
            const long long most = std::max({p->btiles[0], p->btiles[1], p->btiles[2]});
            // one block per CU: the grid-wide barriers cost more with more blocks
            const int blocks = (int)std::min<long long>({(long long)p->bresident, (long long)std::max(1, device_cus()), most});
            e = launch_batch_coop(p->bitems, p->bbegin, p->btiles, blocks, lds, p->dtype, inv, in, out, s);
        } else {
            e = launch_batch((const char *)p->bitems + (size_t)p->bbegin[i] * ib, n, p->btiles[i], p->blds[i],
                             p->dtype, inv, in, out, s);
        }
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return fail_hip(e, "batched kernel launch");
        if (prof) {
            (void)hipEventRecord(b, s);
            prof->push_back({a, b});
        }
    }
    for (size_t g : p->loose) {
        const int rc = run_grid(p, g, (const char *)in + p->offsets[g] * eb, (char *)out + p->offsets[g] * eb,
                                nullptr, nullptr, s, prof);
        if (rc != CROFT_SUCCESS) return rc;
    }
    return CROFT_SUCCESS;
}

// Bytes of the real grid and of its half spectrum (real plans).
void real_bytes(const croft_plan *p, size_t *real_b, size_t *spec_b) {
    const Geometry &g = p->grids[0];
    const size_t cb = element_bytes(p->dtype);
    *real_b = (size_t)g.nx * g.ny * g.nz * (cb / 2);
    *spec_b = ((size_t)g.nx / 2 + 1) * g.ny * g.nz * cb;
}

// The real x pass reads (writes) the real grid and writes (reads) the half
// spectrum; each complex pass reads and writes the half spectrum; the fused
// multiply pass also reads the multiplier (half the bytes of the spectrum).
double real_algorithmic_bytes(const std::vector<PassLaunch> &ps, size_t real_b, size_t spec_b) {
    double b = 0;
    for (const PassLaunch &pl : ps)
        b += pl.kind == kRealX ? (double)real_b + spec_b : (pl.kind == kConvZ ? 2.5 : 2.0) * spec_b;
    return b;
}

int check_buffers(croft_plan *p, const void *in, const void *out) {
    if (!in || !out) return fail(CROFT_ERR_INVALID_VALUE, "NULL data pointer");
    const char *a = (const char *)in, *b = (const char *)out;
    if (p->real) {
        size_t rb, sb;
        real_bytes(p, &rb, &sb);
        const size_t ib = p->dir == CROFT_FORWARD ? rb : sb, ob = p->dir == CROFT_FORWARD ? sb : rb;
        if (a < b + ob && b < a + ib)
            return fail(CROFT_ERR_INVALID_VALUE, "real transforms run out of place: in and out overlap");
    } else {
        const size_t bytes = p->offsets.back() * element_bytes(p->dtype);
        if (a != b && a < b + bytes && b < a + bytes)
            return fail(CROFT_ERR_INVALID_VALUE, "in and out overlap without being equal");
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(CROFT_ERR_INVALID_VALUE, "the current device (%d) is not the plan's device (%d)", dev,
                    p->device);
    return CROFT_SUCCESS;
}

int execute_any(croft_plan *p, const void *in, const int8_t *in_exp, void *out, int8_t *out_exp,
                hipStream_t s, int8_t *e1 = nullptr, int8_t *e2 = nullptr) {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> rec;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof = p->profiling ? &rec : nullptr;
    int rc;
    if (p->unfused)
        rc = run_unfused(p, (const char *)in, (char *)out, s, prof);
    else if (p->slabs > 1)
        rc = run_slabs(p, (const char *)in, (char *)out, in_exp, out_exp, s, prof, e1, e2);
    else
        rc = run_grid(p, 0, (const char *)in, (char *)out, in_exp, out_exp, s, prof, e1, e2);
    if (prof) p->prof.push_back(std::move(rec));
    return rc;
}

// Dry-run description shared by the complex and real forms.
// mode 0: complex plan, 1: real plan, 2: convolution plan
int describe_impl(int nx, int ny, int nz, int dtype, int dir, int mode, char *buf, size_t len) {
    const bool real = mode != 0;
    clear_error();
    int rc = check_dtype_dir(dtype, dir);
    if (rc != CROFT_SUCCESS) return rc;
    rc = real ? check_real_dims(nx, ny, nz, dtype) : check_dims(nx, ny, nz);
    if (rc != CROFT_SUCCESS) return rc;
    if (!buf && len) return fail(CROFT_ERR_INVALID_VALUE, "NULL buffer");
    const Geometry g{nx, ny, nz};
    std::vector<PassLaunch> ps;
    rc = mode == 2 ? build_conv_passes(g, dtype, 0, &ps)
         : real    ? build_real_passes(g, dtype, dir, 0, &ps)
                   : build_passes(g, dtype, dir, 0, &ps);
    if (rc != CROFT_SUCCESS) return rc;
    if (is_half(dtype) && (rc = check_exp_maps(g, ps)) != CROFT_SUCCESS) return rc;
    static const char *names[] = {"c64", "c128", "c16f", "c16b"};
    static const char *kind_names[] = {"contiguous", "strided", "real", "fused"};
    std::string s;
    char line[512];
    const size_t N = (size_t)nx * ny * nz;
    const size_t eb = element_bytes(dtype);
    const size_t spec_b = ((size_t)nx / 2 + 1) * ny * nz * eb;
    const double alg = real ? real_algorithmic_bytes(ps, N * (eb / 2), spec_b) : 6.0 * N * eb;
    snprintf(line, sizeof line, "grid %dx%dx%d %s%s %s elements=%zu bytes=%zu algorithmic_bytes=%.0f\n", nx, ny,
             nz, names[dtype], mode == 2 ? " convolution" : (real ? " real" : ""),
             dir == CROFT_FORWARD ? "forward" : "backward", N, real ? spec_b : N * eb, alg);
    s += line;
    for (size_t i = 0; i < ps.size(); ++i) {
        const PassLaunch &pl = ps[i];
        std::string rad;
        for (int k = 0; k < pl.cfg.nstages; ++k) rad += (k ? "x" : "") + std::to_string(pl.cfg.radix[k]);
        if (rad.empty()) rad = "copy";
        const long long blocks = pass_tiles(pl);
        snprintf(line, sizeof line,
                 "pass %zu axis=%c n=%d kind=%s kernel=%s radices=%s stride=%lld lines=%lld T=%d L=%d block=%d "
                 "blocks=%lld lds=%zu candidate=%d waves=%d bluestein=%d\n",
                 i, "xyz"[pl.axis], pl.n, kind_names[pl.kind],
                 pl.cfg.bluestein ? "bluestein" : (pl.cfg.generic ? "generic" : "static"), rad.c_str(), pl.es,
                 !strided_kind(pl.kind) ? pl.nlines : pl.es * pl.nw, pl.cfg.threads_per_line, pl.cfg.lines,
                 pl.cfg.block, blocks, pl.cfg.lds, pl.cfg.candidate, pl.cfg.grid_waves, pl.cfg.bluestein);
        s += line;
    }
    if (mode == 2) {
        long long count = 1;
        for (const PassLaunch &pl : ps)
            if (pl.kind == kConvZ) count = std::max(count, conv_partials_needed(pl, dtype));
        snprintf(line, sizeof line, "energy_partials=%lld\n", count);
        s += line;
    }
    if (len) {
        const size_t n = std::min(len - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = '\0';
    }
    return CROFT_SUCCESS;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char *croft_last_error(void) { return g_last_error.c_str(); }

int croft_last_status(void) { return g_last_status; }

croft_plan_t croft_plan_create_ex(int nx, int ny, int nz, int dtype, int dir, int flags, int slabs) {
    clear_error();
    if (check_dtype_dir(dtype, dir) != CROFT_SUCCESS) return nullptr;
    if (check_dims(nx, ny, nz) != CROFT_SUCCESS) return nullptr;
    if (flags & ~(CROFT_MEASURE | CROFT_FORCE_GENERIC | CROFT_NO_WISDOM | CROFT_UNFUSED)) {
        fail(CROFT_ERR_INVALID_VALUE, "unknown flags 0x%x", flags);
        return nullptr;
    }
    if ((flags & CROFT_UNFUSED) && (is_half(dtype) || slabs > 1)) {
        fail(is_half(dtype) ? CROFT_ERR_UNSUPPORTED_DTYPE : CROFT_ERR_INVALID_VALUE,
             "CROFT_UNFUSED takes CROFT_C64 or CROFT_C128 and the plain schedule (slabs 0 or 1)");
        return nullptr;
    }
    if ((flags & CROFT_UNFUSED) && slabs == 0) slabs = 1;
    if (slabs < 0 || (slabs > 1 && nz % slabs != 0)) {
        fail(CROFT_ERR_INVALID_VALUE, "slab count %d must be 0, 1 or a divisor of nz = %d", slabs, nz);
        return nullptr;
    }
    return new_plan({Geometry{nx, ny, nz}}, dtype, dir, flags, slabs);
}

croft_plan_t croft_plan_create(int nx, int ny, int nz, int dtype, int dir) {
    return croft_plan_create_ex(nx, ny, nz, dtype, dir, CROFT_ESTIMATE, 1);
}

int croft_plan_destroy(croft_plan_t plan) {
    destroy_plan(plan);
    return CROFT_SUCCESS;
}

int croft_execute(croft_plan_t p, const void *in, void *out, hipStream_t stream) {
    if (!p) return fail(CROFT_ERR_INVALID_VALUE, "NULL plan");
    if (p->batched) return fail(CROFT_ERR_INVALID_VALUE, "batched plan: use croft_execute_batched");
    if (is_half(p->dtype))
        return fail(CROFT_ERR_UNSUPPORTED_DTYPE, "half-storage plan: use croft_execute_scaled");
    if (p->conv) return fail(CROFT_ERR_INVALID_VALUE, "convolution plan: use croft_execute_convolution");
    const int rc = check_buffers(p, in, out);
    if (rc != CROFT_SUCCESS) return rc;
    return execute_any(p, in, nullptr, out, nullptr, stream);
}

croft_plan_t croft_plan_create_convolution(int nx, int ny, int nz, int dtype, int flags) {
    clear_error();
    if (check_dtype_dir(dtype, CROFT_FORWARD) != CROFT_SUCCESS) return nullptr;
    if (check_real_dims(nx, ny, nz, dtype) != CROFT_SUCCESS) return nullptr;
    if (flags & ~(CROFT_MEASURE | CROFT_FORCE_GENERIC | CROFT_NO_WISDOM)) {
        fail(CROFT_ERR_INVALID_VALUE, "unknown flags 0x%x", flags);
        return nullptr;
    }
    return new_plan({Geometry{nx, ny, nz}}, dtype, CROFT_FORWARD, flags, 1, false, true, true);
}

int croft_execute_convolution(croft_plan_t p, const void *in, const void *mul, void *out, double *energy,
                              hipStream_t stream) {
    if (!p) return fail(CROFT_ERR_INVALID_VALUE, "NULL plan");
    if (!p->conv) return fail(CROFT_ERR_INVALID_VALUE, "not a convolution plan");
    if (!in || !mul || !out) return fail(CROFT_ERR_INVALID_VALUE, "NULL data pointer");
    size_t rb, sb;
    real_bytes(p, &rb, &sb);
    const size_t mb = sb / 2;  // one real per spectrum element
    const char *a = (const char *)in, *b = (const char *)out, *m = (const char *)mul;
    if (a != b && a < b + rb && b < a + rb)
        return fail(CROFT_ERR_INVALID_VALUE, "in and out overlap without being equal");
    if (m < b + rb && b < m + mb) return fail(CROFT_ERR_INVALID_VALUE, "mul overlaps out");
    if (energy && (const char *)energy < b + rb && b < (const char *)energy + sizeof(double))
        return fail(CROFT_ERR_INVALID_VALUE, "energy overlaps out");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(CROFT_ERR_INVALID_VALUE, "the current device (%d) is not the plan's device (%d)", dev,
                    p->device);
    std::vector<std::pair<hipEvent_t, hipEvent_t>> rec;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> *prof = p->profiling ? &rec : nullptr;
    const int rc = run_conv(p, in, mul, out, energy, stream, prof);
    if (prof) p->prof.push_back(std::move(rec));
    return rc;
}

int croft_execute_scaled(croft_plan_t p, const void *in, const int8_t *in_exp, void *out, int8_t *out_exp,
                         hipStream_t stream) {
    if (!p) return fail(CROFT_ERR_INVALID_VALUE, "NULL plan");
    if (p->batched) return fail(CROFT_ERR_INVALID_VALUE, "batched plan: use croft_execute_batched");
    if (!is_half(p->dtype))
        return fail(CROFT_ERR_UNSUPPORTED_DTYPE, "croft_execute_scaled needs a CROFT_C16F/CROFT_C16B plan");
    if (!out_exp) return fail(CROFT_ERR_INVALID_VALUE, "NULL out_exp");
    const int rc = check_buffers(p, in, out);
    if (rc != CROFT_SUCCESS) return rc;
    return execute_any(p, in, in_exp, out, out_exp, stream);
}

int croft_execute_scaled_noalloc(croft_plan_t p, const void *in, const int8_t *in_exp, void *out, int8_t *out_exp,
                                 hipStream_t stream) {
    if (!p) return fail(CROFT_ERR_INVALID_VALUE, "NULL plan");
    if (p->batched) return fail(CROFT_ERR_INVALID_VALUE, "batched plan: use croft_execute_batched");
    if (!is_half(p->dtype))
        return fail(CROFT_ERR_UNSUPPORTED_DTYPE, "croft_execute_scaled_noalloc needs a CROFT_C16F/CROFT_C16B plan");
    if (!out_exp) return fail(CROFT_ERR_INVALID_VALUE, "NULL out_exp");
    if (p->profiling)
        return fail(CROFT_ERR_INVALID_VALUE, "per-pass profiling creates events: disable it for the "
                                             "allocation-free execute");
    const Geometry &g = p->grids[0];
    const size_t b1 = (size_t)g.ny * g.nz, b2 = (size_t)g.nx * g.nz;
    const size_t off2 = (b1 + 255) / 256 * 256;
    if (off2 + b2 > kNoAllocScratchBytes)
        return fail(CROFT_ERR_UNSUPPORTED_SIZE,
                    "grid %dx%dx%d needs %zu bytes of exponent scratch (ny*nz + nx*nz, the first rounded up to "
                    "256); the static array holds %zu",
                    g.nx, g.ny, g.nz, off2 + b2, kNoAllocScratchBytes);
    if (!p->scratch) return fail(CROFT_ERR_INTERNAL, "no static scratch address for the plan's device");
    const int rc = check_buffers(p, in, out);
    if (rc != CROFT_SUCCESS) return rc;
    return execute_any(p, in, in_exp, out, out_exp, stream, p->scratch, p->scratch + off2);
}

croft_plan_t croft_plan_create_batched(int count, const int *dims, int dtype, int dir, int flags) {
    clear_error();
    if (count < 1 || !dims) {
        fail(CROFT_ERR_INVALID_VALUE, "batched plan needs count >= 1 and dims");
        return nullptr;
    }
    if (check_dtype_dir(dtype, dir) != CROFT_SUCCESS) return nullptr;
    if (is_half(dtype)) {
        fail(CROFT_ERR_UNSUPPORTED_DTYPE, "batched plans take CROFT_C64 or CROFT_C128");
        return nullptr;
    }
    if (flags & ~(CROFT_MEASURE | CROFT_FORCE_GENERIC | CROFT_NO_WISDOM | CROFT_PERSISTENT | CROFT_GRAPH)) {
        fail(CROFT_ERR_INVALID_VALUE, "unknown flags 0x%x", flags);
        return nullptr;
    }

    std::vector<Geometry> grids;
    long long total = 0;
    for (int i = 0; i < count; ++i) {
        if (check_dims(dims[3 * i], dims[3 * i + 1], dims[3 * i + 2]) != CROFT_SUCCESS) {
            g_last_error = "grid " + std::to_string(i) + ": " + g_last_error;
            return nullptr;
        }
        grids.push_back({dims[3 * i], dims[3 * i + 1], dims[3 * i + 2]});
        total += (long long)dims[3 * i] * dims[3 * i + 1] * dims[3 * i + 2];
    }
    if (total > 0x7fffffffLL) {
        fail(CROFT_ERR_UNSUPPORTED_SIZE, "batch of %lld elements exceeds 2^31 - 1", total);
        return nullptr;
    }
    return new_plan(grids, dtype, dir, flags, 1, true);
}

croft_plan_t croft_plan_create_real(int nx, int ny, int nz, int dtype, int dir, int flags) {
    clear_error();
    if (check_dtype_dir(dtype, dir) != CROFT_SUCCESS) return nullptr;
    if (check_real_dims(nx, ny, nz, dtype) != CROFT_SUCCESS) return nullptr;
    if (flags & ~(CROFT_MEASURE | CROFT_FORCE_GENERIC | CROFT_NO_WISDOM)) {
        fail(CROFT_ERR_INVALID_VALUE, "unknown flags 0x%x", flags);
        return nullptr;
    }
    return new_plan({Geometry{nx, ny, nz}}, dtype, dir, flags, 1, false, true);
}

int croft_plan_batched_offsets(croft_plan_t p, size_t *elem_offsets) {
    if (!p || !elem_offsets) return fail(CROFT_ERR_INVALID_VALUE, "NULL argument");
    std::copy(p->offsets.begin(), p->offsets.end(), elem_offsets);
    return CROFT_SUCCESS;
}

int croft_execute_batched(croft_plan_t p, const void *in, void *out, hipStream_t stream) {
    if (!p) return fail(CROFT_ERR_INVALID_VALUE, "NULL plan");
    if (!p->batched) return fail(CROFT_ERR_INVALID_VALUE, "not a batched plan: use croft_execute");
    int rc = check_buffers(p, in, out);
    if (rc != CROFT_SUCCESS) return rc;
    if (p->profiling) {
        std::vector<std::pair<hipEvent_t, hipEvent_t>> rec;
        rc = run_batch(p, in, out, stream, &rec);
        p->prof.push_back(std::move(rec));
        return rc;
    }
    // Launches go straight to the stream unless the plan asked for graph
    // replay: on MI355X a replayed graph of these one to three launches took
    // about 15 us longer than the same launches issued directly for one 32^3
    // grid and was no faster for 64 grids.  A cooperative launch the runtime
    // refuses to capture is issued directly.
    if (!(p->flags & CROFT_GRAPH) || p->coop_direct) return run_batch(p, in, out, stream, nullptr);
    if (!p->graph || p->graph_in != in || p->graph_out != out || p->graph_stream != stream) {
        if (p->graph) {
            (void)hipGraphExecDestroy(p->graph);
            p->graph = nullptr;
        }
        hipStream_t cap;
        hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e != hipSuccess) return fail_hip(e, "stream create");
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cap);
            return fail_hip(e, "begin capture");
        }
        rc = run_batch(p, in, out, cap, nullptr);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cap, &graph);
        (void)hipStreamDestroy(cap);
        if ((rc != CROFT_SUCCESS || e != hipSuccess) && (p->flags & CROFT_PERSISTENT)) {
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            p->coop_direct = true;
            return run_batch(p, in, out, stream, nullptr);
        }
        if (rc != CROFT_SUCCESS) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail_hip(e, "end capture");
        e = hipGraphInstantiate(&p->graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            p->graph = nullptr;
            return fail_hip(e, "graph instantiate");
        }
        p->graph_in = in;
        p->graph_out = out;
        p->graph_stream = stream;
    }
    const hipError_t e = hipGraphLaunch(p->graph, stream);
    if (e != hipSuccess) return fail_hip(e, "graph launch");
    return CROFT_SUCCESS;
}

int croft_plan_info(croft_plan_t p, struct croft_plan_info *info) {
    if (!p || !info) return fail(CROFT_ERR_INVALID_VALUE, "NULL argument");
    std::memset(info, 0, sizeof *info);
    const Geometry &g = p->grids[0];
    info->nx = g.nx;
    info->ny = g.ny;
    info->nz = g.nz;
    info->dtype = p->dtype;
    info->dir = p->dir;
    info->batched_count = p->batched ? (int)p->grids.size() : 0;
    info->real = p->real ? 1 : 0;
    info->convolution = p->conv ? 1 : 0;
    info->slabs = p->slabs;
    const std::vector<PassLaunch> &ps = p->passes[0];
    info->npasses = (int)std::min<size_t>(ps.size(), CROFT_MAX_PASSES);
    for (int i = 0; i < info->npasses; ++i) {
        const PassLaunch &pl = ps[i];
        croft_pass_info &pi = info->pass[i];
        pi.axis = pl.axis;
        pi.n = pl.n;
        pi.kind = pl.kind;
        pi.generic = pl.cfg.generic ? 1 : 0;
        pi.nstages = pl.cfg.nstages;
        for (int s = 0; s < pl.cfg.nstages; ++s) pi.radices[s] = pl.cfg.radix[s];
        pi.threads_per_line = pl.cfg.threads_per_line;
        pi.lines_per_block = pl.cfg.lines;
        pi.block_threads = pl.cfg.block;
        pi.blocks = pass_tiles(pl);
        pi.lds_bytes = pl.cfg.lds;
        pi.bluestein = pl.cfg.bluestein;
    }
    info->elements = p->offsets.back();
    info->element_bytes = element_bytes(p->dtype);
    info->work_bytes = p->work_bytes;
    info->algorithmic_bytes = 6.0 * (double)info->elements * (double)info->element_bytes;
    double fl = 0;
    for (const Geometry &gg : p->grids) {
        const double n = (double)gg.nx * gg.ny * gg.nz;
        if (n > 1) fl += 5.0 * n * std::log2(n);
    }
    info->flops = fl;
    info->graph_replay = !p->batched                                 ? -1
                         : !(p->flags & CROFT_GRAPH) || p->coop_direct ? 0
                         : p->graph                                    ? 1
                                                                       : -1;
    if (p->real) {
        size_t rb, sb;
        real_bytes(p, &rb, &sb);
        info->algorithmic_bytes = real_algorithmic_bytes(p->passes[0], rb, sb);
        info->flops = p->conv ? fl : fl / 2;
    }
    return CROFT_SUCCESS;
}

int croft_plan_describe(int nx, int ny, int nz, int dtype, int dir, char *buf, size_t len) {
    return describe_impl(nx, ny, nz, dtype, dir, 0, buf, len);
}

int croft_plan_describe_real(int nx, int ny, int nz, int dtype, int dir, char *buf, size_t len) {
    return describe_impl(nx, ny, nz, dtype, dir, 1, buf, len);
}

int croft_plan_describe_convolution(int nx, int ny, int nz, int dtype, char *buf, size_t len) {
    return describe_impl(nx, ny, nz, dtype, CROFT_FORWARD, 2, buf, len);
}

int croft_plan_profile(croft_plan_t p, int enable) {
    if (!p) return fail(CROFT_ERR_INVALID_VALUE, "NULL plan");
    p->profiling = enable != 0;
    return CROFT_SUCCESS;
}

int croft_plan_profile_read(croft_plan_t p, double *pass_ms, int max_passes, int *executes) {
    if (!p || (!pass_ms && max_passes > 0) || max_passes < 0) return fail(CROFT_ERR_INVALID_VALUE, "bad argument");
    for (int i = 0; i < max_passes; ++i) pass_ms[i] = 0.0;
    int rc = CROFT_SUCCESS;
    for (auto &rec : p->prof) {
        for (size_t i = 0; i < rec.size(); ++i) {
            hipError_t e = hipEventSynchronize(rec[i].second);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, rec[i].first, rec[i].second);
            if (e != hipSuccess && rc == CROFT_SUCCESS) rc = fail_hip(e, "profiling event");
            if ((int)i < max_passes) pass_ms[i] += ms;
            p->event_pool.push_back(rec[i].first);
            p->event_pool.push_back(rec[i].second);
        }
    }
    if (executes) *executes = (int)p->prof.size();
    p->prof.clear();
    return rc;
}

}  // extern "C"
