/*
 * croft.h -- C ABI of the MI355X (gfx950) complex-to-complex 3D FFT library.
 *
 * The operation is the 3D discrete Fourier transform of the paper, Section 2.1:
 *   forward  (Eq. 1):  Y(k) = sum_j X(j) exp(-2 pi i (kx jx/Nx + ky jy/Ny + kz jz/Nz))
 *   backward (Eq. 2):  the same sum with exp(+2 pi i ...).  The library does
 *                      NOT apply Eq. (2)'s factor 1/(Nx Ny Nz): backward after
 *                      forward returns Nx*Ny*Nz times the input (the paper's
 *                      Section 5.3 round trip, with the caller normalising).
 * It is computed as the paper's algorithm (Section 4.1): batched 1D FFTs along
 * x, then y, then z, with the transposes between the stages folded into the
 * passes so the output comes back in the input's layout (Section 4.2).
 *
 * Layout (all entry points): a grid is one array ("1D input array", Section
 * 5.2) holding element (x, y, z) at index x + nx*(y + ny*z).  A torch tensor of
 * shape (nz, ny, nx), contiguous, has exactly this layout.
 *   CROFT_C64   complex float  (re, im interleaved), 8 bytes per element
 *   CROFT_C128  complex double (re, im interleaved), 16 bytes per element
 *   CROFT_C16F  two IEEE binary16 (re, im), 4 bytes per element, plus int8
 *               power-of-two exponents: value = stored * 2^exp
 *   CROFT_C16B  as CROFT_C16F with bfloat16 halves
 * Half-storage plans compute in FP32 and must be run through
 * croft_execute_scaled, which carries the exponents.
 *
 * Sizes: every axis length n satisfies 1 <= n <= 4096; the grid holds at
 * most 2^31 - 1 elements.  Lengths of the form 2^a 3^b 5^c run mixed-radix
 * Stockham kernels; any other length runs Bluestein's algorithm (a chirp
 * convolution of power-of-two length m >= 2n - 1 held in LDS), which for
 * CROFT_C128 limits such lengths to n <= 2048.  Others give
 * CROFT_ERR_UNSUPPORTED_SIZE.  Grids need not be cubic.
 *
 * Ownership: the caller owns `in`, `out` (device memory) and the exponent
 * arrays.  A plan owns its device tables (twiddles, exponent scratch,
 * batch descriptors), allocated at create and freed at destroy; a plan is
 * bound to the device that was current when it was created.
 *
 * Streams and concurrency: execute calls are asynchronous and ordered on the
 * given stream (NULL = the null stream); they do not synchronise the host,
 * allocate, or copy, except where an entry point says otherwise, so a caller
 * may capture croft_execute, croft_execute_convolution and (for plans made
 * without CROFT_GRAPH) croft_execute_batched into a HIP graph (not while
 * per-pass profiling is enabled).  One execute
 * may be in flight per plan at a time (plans hold per-call scratch): use one
 * plan per concurrently used stream.  Destroy a plan only after its work has
 * completed.
 *
 * Errors: every call returns a croft_status (create functions return NULL
 * and leave it in croft_last_status()); croft_last_error() then holds a
 * message for the calling thread.  HIP launch errors are reported as
 * CROFT_ERR_HIP with HIP's own message.  No C++ exception crosses this
 * boundary.  A failed create frees whatever it had allocated.  For tests, the
 * environment variable CROFT_TEST_FAIL_ALLOC=k (k >= 1) makes the k-th device
 * allocation of each plan creation fail as CROFT_ERR_OUT_OF_MEMORY.
 */
#ifndef CROFT_H
#define CROFT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct croft_plan *croft_plan_t;

enum croft_dtype {
    CROFT_C64 = 0,  /* complex float storage, FP32 compute */
    CROFT_C128 = 1, /* complex double storage, FP64 compute (the paper's type, Section 5) */
    CROFT_C16F = 2, /* complex FP16 storage with per-line exponents, FP32 compute */
    CROFT_C16B = 3  /* complex BF16 storage with per-line exponents, FP32 compute */
};

enum croft_direction {
    CROFT_FORWARD = -1, /* Eq. (1): exponent sign -1 */
    CROFT_BACKWARD = 1  /* Eq. (2) without its 1/N factor: exponent sign +1 */
};

enum croft_status {
    CROFT_SUCCESS = 0,
    CROFT_ERR_INVALID_VALUE = 1,    /* NULL or bad argument, overlapping buffers */
    CROFT_ERR_UNSUPPORTED_SIZE = 2, /* axis length outside 1..4096, or a length no kernel covers */
    CROFT_ERR_UNSUPPORTED_DTYPE = 3,/* unknown dtype, or a call that does not fit it */
    CROFT_ERR_OUT_OF_MEMORY = 4,    /* a plan allocation failed */
    CROFT_ERR_HIP = 5,              /* a HIP runtime call or kernel launch failed */
    CROFT_ERR_INTERNAL = 6
};

/* Flags for croft_plan_create_ex / croft_plan_create_batched. */
enum croft_flags {
    CROFT_ESTIMATE = 0,       /* default heuristics, no device timing at create */
    CROFT_MEASURE = 1,        /* time candidate configurations at create (autotune) */
    CROFT_FORCE_GENERIC = 2,  /* use the runtime-radix kernels for every pass */
    CROFT_NO_WISDOM = 4,      /* MEASURE: neither read nor write the wisdom file */
    CROFT_UNFUSED = 16,       /* croft_plan_create_ex, C64/C128: the paper's Option 2 (Section 5.1,
                                 no overlap), kept as the measured baseline of the fused passes:
                                 the three FFTs run on contiguous lines with three standalone
                                 LDS-tiled transposes of the whole grid between and after them
                                 (six sweeps instead of three) through a plan-owned work grid;
                                 same results.  Profiled launches: FFT x, transpose, FFT y,
                                 transpose, FFT z, transpose (length-1 axes skip their FFT). */
    CROFT_PERSISTENT = 8,     /* batched plans: one cooperative launch for every pass of every
                                 grid (all blocks resident, looping over the tiles of pass 0, a
                                 grid-wide barrier, pass 1, a barrier, pass 2) instead
                                 of one launch per pass; same results bit for bit. */
    CROFT_GRAPH = 32          /* batched plans: replay the launches of croft_execute_batched from
                                 a HIP graph captured on first use for the given (in, out,
                                 stream) and captured again when they change; such a capture
                                 creates a stream and instantiates a graph inside that execute
                                 (host and driver allocations), later replays allocate
                                 nothing, and the call cannot itself be captured by the
                                 caller.  Without it the
                                 launches are issued directly, which measured faster: the
                                 replayed graph took about 15 us longer for one 32^3 grid and
                                 was no faster for 64 grids.  A cooperative launch
                                 (CROFT_PERSISTENT) the runtime refuses to capture is issued
                                 directly: croft_plan_info.graph_replay. */
};

/* Create a plan for one nx x ny x nz transform (the paper's problem statement,
 * Section 2.1, Eq. 1-2; its API runs one forward transform of the local grid,
 * Section 5.2).  dtype: croft_dtype; dir: croft_direction.  Returns NULL on
 * failure (see croft_last_error).  Allocates device memory on the current
 * device. */
croft_plan_t croft_plan_create(int nx, int ny, int nz, int dtype, int dir);

/* As croft_plan_create, with croft_flags and the slab count K of the pipelined
 * schedule: K > 1 splits the grid into K slabs along z and runs the x and y
 * passes slab by slab on two internal streams, so that a slab written by the
 * x pass is read back by the y pass while still cache resident; the z pass
 * then runs over the whole grid.  This is the one-GPU form of the paper's
 * overlap of chunked communication with computation and its iteration
 * parameter K (Section 5.1, where K = 2).  K must divide nz; K = 1 is the
 * plain three-pass schedule.  K = 0 lets the plan choose: with CROFT_MEASURE
 * it times the whole transform for every K in {1, 2, 4, 8, 16} dividing nz,
 * keeps the fastest and records it in the wisdom (the CROFT_WISDOM file as
 * "slabs nx ny nz dtype K", and this process); without CROFT_MEASURE it
 * takes a recorded K for the same grid and dtype, else 1.  The chosen K is
 * croft_plan_info.slabs.  The result does not depend on K (bit for bit). */
croft_plan_t croft_plan_create_ex(int nx, int ny, int nz, int dtype, int dir, int flags, int slabs);

/* Run the transform of a C64/C128 plan.  in == out runs in place; otherwise
 * the buffers must not overlap and `in` is left unchanged.  Each buffer holds
 * nx*ny*nz elements of the plan's dtype (real plans: the layouts given at
 * croft_plan_create_real).  Asynchronous on `stream`. */
int croft_execute(croft_plan_t plan, const void *in, void *out, hipStream_t stream);

/* Run the transform of a C16F/C16B plan.  Values are stored * 2^exp.
 *   in_exp:  ny*nz int8, one per x-line, index y + ny*z (NULL: all zero)
 *   out_exp: nx*ny int8, one per z-line, index x + nx*y (required)
 * Every output z-line is scaled so that its largest |re| or |im| lies in
 * [2^14, 2^15) before rounding to nearest even (an all-zero line gets 0).
 * in == out runs in place.  out_exp may be the same array as in_exp (the
 * input exponents are consumed by the first pass, the output exponents
 * written by the last).  Asynchronous on `stream`. */
int croft_execute_scaled(croft_plan_t plan, const void *in, const int8_t *in_exp, void *out,
                         int8_t *out_exp, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * transform as croft_execute_scaled, with the same arguments and results bit
 * for bit, but the intermediate per-line exponents (ny*nz bytes after the x
 * pass, nx*nz after the y pass) live in a static array of
 * CROFT_NOALLOC_SCRATCH_BYTES on each GPU instead of the plan's own, and the
 * call allocates nothing (no device or host allocation, no event or stream
 * creation).  Every call on a GPU shares that GPU's array, which keeps the
 * last call's contents (each pass writes all the exponents the next one
 * reads, so nothing needs clearing): calls that overlap on one GPU, from any
 * plans or streams, race -- order them on one stream.  The array is
 * allocated when the library is loaded and held by each GPU until the
 * process ends.
 * Errors: CROFT_ERR_UNSUPPORTED_SIZE when ny*nz (rounded up to 256) plus
 * nx*nz exceeds CROFT_NOALLOC_SCRATCH_BYTES; CROFT_ERR_INVALID_VALUE while
 * per-pass profiling is enabled on the plan (it creates events); otherwise
 * as croft_execute_scaled. */
#define CROFT_NOALLOC_SCRATCH_BYTES (4u << 20)
int croft_execute_scaled_noalloc(croft_plan_t plan, const void *in, const int8_t *in_exp, void *out,
                                 int8_t *out_exp, hipStream_t stream);

/* Free a plan and its device tables.  NULL is a no-op returning CROFT_SUCCESS. */
int croft_plan_destroy(croft_plan_t plan);

/* Message describing the last failed call on this thread ("" if none). */
const char *croft_last_error(void);

/* The croft_status of the last failed call on this thread (CROFT_SUCCESS if
 * none).  Create functions, which return NULL on failure, report their status
 * here; like the message, it is reset when a create function starts. */
int croft_last_status(void);

/* Batched form: `count` independent transforms of uneven sizes,
 * dims[3*i + 0..2] = (nx, ny, nz) of grid i.  Grids are packed back to back in
 * one buffer, grid i starting at element offset offsets[i] (see
 * croft_plan_batched_offsets).  dtype CROFT_C64 or CROFT_C128.  flags:
 * croft_flags (CROFT_MEASURE autotunes the kernel configuration per length
 * and records it in the wisdom file). */
croft_plan_t croft_plan_create_batched(int count, const int *dims, int dtype, int dir, int flags);

/* Element offsets of the grids of a batched plan: count + 1 values, the last
 * being the total element count.  `elem_offsets` is host memory. */
int croft_plan_batched_offsets(croft_plan_t plan, size_t *elem_offsets);

/* Run every transform of a batched plan (one from croft_plan_create_batched;
 * others give CROFT_ERR_INVALID_VALUE): one launch per axis pass covering
 * all grids -- or, with CROFT_PERSISTENT, one cooperative launch -- issued on
 * `stream`, or with CROFT_GRAPH replayed from a HIP graph.  Grids whose lengths
 * the batched kernels do not compile (any outside 48, 60, 64, 72, 80, 96, 100,
 * 128) run with launches of their own (inside the same graph with CROFT_GRAPH).
 * Same in/out rules as croft_execute. */
int croft_execute_batched(croft_plan_t plan, const void *in, void *out, hipStream_t stream);

/* Real transforms (Section 1: PME transforms a real charge grid forward and
 * brings the reciprocal-space result back to a real grid; the spectrum of a
 * real grid is Hermitian, Y(-k) = conj Y(k), so the kx = 0..nx/2 half of
 * Eq. (1)'s output determines the rest).  dtype CROFT_C64 (float reals,
 * complex float spectrum, FP32 compute) or CROFT_C128 (double, FP64).
 * nx even, 4 <= nx <= 8192, with nx/2 among the lengths the library compiles
 * (powers of two 2..4096 and 48, 60, 72, 80, 96, 100, 384); ny and nz as for
 * croft_plan_create.  flags: CROFT_MEASURE, CROFT_FORCE_GENERIC (y and z
 * passes only), CROFT_NO_WISDOM.  Returns NULL on failure.
 * Layouts, run with croft_execute (out of place only: overlapping in and out
 * give CROFT_ERR_INVALID_VALUE; `in` is left unchanged):
 *   real grid:     nx*ny*nz reals, element (x, y, z) at x + nx*(y + ny*z)
 *   half spectrum: (nx/2+1)*ny*nz complex, (kx, ky, kz) at
 *                  kx + (nx/2+1)*(ky + ny*kz), kx = 0..nx/2
 *   CROFT_FORWARD:  real grid -> Y(kx, ky, kz) of Eq. (1), kx <= nx/2.
 *   CROFT_BACKWARD: half spectrum -> real grid: the unnormalised inverse of
 *                   Eq. (2) over z and y, then along x the real inverse of
 *                   the Hermitian extension in kx, which uses only the real
 *                   parts of the kx = 0 and kx = nx/2 terms
 *                   x(n) = Re H(0) + (-1)^n Re H(nx/2)
 *                          + 2 Re sum_{0<k<nx/2} H(k) exp(2 pi i k n / nx).
 *                   For the spectrum of a real grid this is nx*ny*nz times
 *                   that grid (no 1/N factor, as for complex plans).
 * A backward plan with ny*nz > 1 owns a work buffer of one half spectrum
 * (counted in croft_plan_info.work_bytes). */
croft_plan_t croft_plan_create_real(int nx, int ny, int nz, int dtype, int dir, int flags);

/* Convolution plans: the reciprocal-space step of particle-mesh Ewald
 * (Section 1: a forward FFT of the charge grid, a product in reciprocal
 * space, a reverse FFT back to the grid), on a real grid, in one call:
 *   Q   = the forward real transform of `in` (Eq. 1, half spectrum),
 *   out = the backward real transform (as croft_plan_create_real, without
 *         1/N) of G * Q, G the real multiplier `mul` given on the half
 *         spectrum,
 *   *energy = sum over the full spectrum of G(k) |Q(k)|^2, G extended to
 *         kx > nx/2 by G(-k) = G(k) (so the kx = 1..nx/2-1 terms count twice).
 * Passes: the forward x (real) and y passes, then ONE pass along z that
 * transforms forward, multiplies by G and transforms back while each tile
 * stays in LDS, then the backward y and x passes: five sweeps instead of the
 * six of two separate transforms, and G is read once.  With nz = 1 the fused
 * pass runs along y.
 * dtype CROFT_C64 (float reals and multiplier, FP32 compute) or CROFT_C128
 * (double, FP64).  Sizes as for croft_plan_create_real, plus ny*nz > 1, and
 * the fused axis length must be a compiled length (powers of two 2..4096,
 * 48, 60, 72, 80, 96, 100, 384).  flags: CROFT_MEASURE, CROFT_FORCE_GENERIC
 * (y pass only), CROFT_NO_WISDOM.  The plan owns a half-spectrum work buffer
 * and the per-block energy partials.  Returns NULL on failure. */
croft_plan_t croft_plan_create_convolution(int nx, int ny, int nz, int dtype, int flags);

/* Run a convolution plan (asynchronous on `stream`).
 *   in:     nx*ny*nz reals (x + nx*(y + ny*z)); left unchanged unless in == out
 *   mul:    (nx/2+1)*ny*nz reals, element (kx, ky, kz) at kx + (nx/2+1)*(ky + ny*kz)
 *   out:    nx*ny*nz reals; may equal `in`, must not otherwise overlap it or `mul`
 *   energy: one double in device memory, or NULL to skip the sum; computed
 *           in FP64 from per-block partials in a fixed order (the same
 *           inputs give the same bits). */
int croft_execute_convolution(croft_plan_t plan, const void *in, const void *mul, void *out, double *energy,
                              hipStream_t stream);

/* Dry run of croft_plan_create_convolution (no GPU). */
int croft_plan_describe_convolution(int nx, int ny, int nz, int dtype, char *buf, size_t len);

/* Description of a plan, filled by croft_plan_info. */
#define CROFT_MAX_PASSES 8
#define CROFT_MAX_STAGES 12
struct croft_pass_info {
    int axis;            /* 0 = x, 1 = y, 2 = z */
    int n;               /* transform length */
    int kind;            /* 0: contiguous lines, 1: strided lines, 2: real x pass (n = nx/2),
                            3: fused forward / multiply / inverse pass (strided lines) */
    int generic;         /* 1 if the runtime-radix kernel runs this pass */
    int nstages;
    int radices[CROFT_MAX_STAGES];
    int threads_per_line;
    int lines_per_block;
    int block_threads;
    long long blocks;    /* grid size of one launch over the whole grid */
    size_t lds_bytes;
    int bluestein;       /* > 0: Bluestein's algorithm runs this pass with a convolution
                            of this power-of-two length (radices describe that FFT) */
};
struct croft_plan_info {
    int nx, ny, nz, dtype, dir;
    int batched_count;   /* 0 for a single-grid plan */
    int slabs;           /* K of the slab schedule (1 = plain) */
    int npasses;
    struct croft_pass_info pass[CROFT_MAX_PASSES];
    size_t elements;          /* total elements (all grids for a batched plan) */
    size_t element_bytes;     /* bytes per stored element */
    size_t work_bytes;        /* device scratch owned by the plan */
    double algorithmic_bytes; /* 3 sweeps x (read + write) x elements x element_bytes; real
                                 plans: real grid + half spectrum for the x pass, twice the
                                 half spectrum for each of the others */
    double flops;             /* sum over grids of 5 N log2 N (real plans: 2.5 N log2 N) */
    int real;                 /* 1 for a plan of croft_plan_create_real or _convolution */
    int convolution;          /* 1 for a plan of croft_plan_create_convolution */
    int graph_replay;         /* batched plans: 1 once croft_execute_batched replays a captured
                                 graph (CROFT_GRAPH), 0 if it issues its launches directly
                                 (no CROFT_GRAPH, or a cooperative launch that could not be
                                 captured), -1 before the first execute with CROFT_GRAPH and
                                 for plans that are not batched */
};
int croft_plan_info(croft_plan_t plan, struct croft_plan_info *info);

/* Dry run: write a text description of the plan that croft_plan_create would
 * build (passes, radices, launch shapes, bytes) into buf (len bytes, always
 * NUL-terminated when len > 0).  Uses no GPU.  Returns a croft_status. */
int croft_plan_describe(int nx, int ny, int nz, int dtype, int dir, char *buf, size_t len);

/* The same dry run for the plan croft_plan_create_real would build. */
int croft_plan_describe_real(int nx, int ny, int nz, int dtype, int dir, char *buf, size_t len);

/* Per-kernel timing: while enabled, every execute on the plan records HIP
 * events around each pass launch on the stream it is launched on.
 * croft_plan_profile_read waits for the recorded events, then writes for each
 * pass p (p < max_passes) the total milliseconds over the recorded executes
 * into pass_ms[p] and the execute count into *executes, and clears the record.
 * Enabling allocates events; not for use under stream capture. */
int croft_plan_profile(croft_plan_t plan, int enable);
int croft_plan_profile_read(croft_plan_t plan, double *pass_ms, int max_passes, int *executes);

#ifdef __cplusplus
}
#endif
#endif /* CROFT_H */
