"""Benchmark: forward C2C 3D FFT at 512^3 complex64 on one MI355X.

Prints ONE JSON line.  A step is one forward 3D FFT of the whole grid (the
three axis passes with their in-LDS transposes) on a PME-style charge grid
already resident in HBM; `value` is GFLOP/s by the 5 N log2 N convention.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--size 512] [--slabs K]
                  [--no-cpu-baseline] [--no-forms] [--calibrate-copy] [--only-form half]

The dominant kernel's roofline uses HIP events recorded by the library around
each pass launch on the stream the pass runs on, over the timed region.
After all GPU timing, the CPU leg times the FP64 oracle on a bounded sample
(`cpu_baseline`) and compares exact oracle output lines with the GPU's
results (`oracle_check`: the complex64 headline, complex128, both 16-bit
storage forms, the 64-grid batch and the 1024^3 grid).  `--no-coop` leaves
out the batched form's cooperative launch (profiled runs: rocprofv3 has
ended in a segmentation fault at exit in runs that included it).
`--calibrate-copy` instead times a plain device copy of the same bytes (used
to scale the HBM byte counters).  The line also carries the half-storage
(FP16, BF16 at 512^3) and batched (64 uneven grids) forms, each timed next to
the plain complex64 form on the same GPU with its error against it, and the
smaller cubes (32^3 latency; 256^3 and 384^3 forward and inverse, warm and
with the Infinity Cache flushed) under "configs" (`--no-forms` skips both).
The effective rate is also given as a fraction of a measured device copy.
`--only-form half` runs only the FP16 and BF16 storage forms (each beside a
complex64 transform of the same values) and prints them, for counter runs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3D FFT GFLOP/s (5N·log2N) + achieved HBM GB/s at 512³ c64, 1 MI355X"
HBM_PEAK_GBPS = 8000.0
KERNEL_SOURCES = ["paper_2002_04896_amd/csrc/croft_device.h",
                  "paper_2002_04896_amd/csrc/croft_entries_c64.hip",
                  "paper_2002_04896_amd/csrc/croft_kernels.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_512cube_c64.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def flops_5nlogn(n: int) -> float:
    return 5.0 * n * math.log2(n) if n > 1 else 0.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--slabs", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--only-form", choices=["half"], default=None,
                    help="time one form alone (for profiling) and print it")
    ap.add_argument("--no-coop", action="store_true",
                    help="skip the batched form's cooperative single launch")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_c64, n):
    """Time the FP64 oracle (naive O(n^2) DFT per line, Eq. 1) on a bounded
    sample of the 512^3 transform: half of the lines of every axis, in place.
    The rate is that of the sample: 5 N log2 N times the fraction of the work
    done, over the measured seconds."""
    import numpy as np
    import oracle

    a = x_c64.astype(np.complex128)
    lines = n * n
    sample = lines // 2
    t0 = time.perf_counter()
    for axis in range(3):
        oracle.dft_axis_lines(a, axis, 0, sample, -1)
    dt = time.perf_counter() - t0
    frac = sample / lines
    N = n ** 3
    work = flops_5nlogn(N) * frac
    true_flops = 8.0 * N * 3 * n * frac            # one complex multiply-add per term: 8 flops
    return {"value": work / dt / 1e9, "unit": "GFLOP/s", "cores": oracle.max_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "measured_s": dt, "true_GFLOPs": true_flops / dt / 1e9,
            "sample": f"naive FP64 DFT of {sample} of the {lines} lines of each axis ({frac:g} of the work) "
                      f"of the {n}^3 PME grid, in place, {dt:.1f} s on {oracle.max_threads()} threads; "
                      f"value = 5 N log2 N x {frac:g} / {dt:.1f} s (a rate, not extrapolated)"}


def sample_pairs(ny, nz, count, seed):
    """(ky, kz) output lines to check: the corners plus seeded random ones."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = [(0, 0), (ny - 1, nz - 1), (ny // 2, nz // 3)]
    pts += [(int(a), int(b)) for a, b in zip(rng.integers(0, ny, count - 3), rng.integers(0, nz, count - 3))]
    return pts


def device_lines(t, kyz):
    """Lines Y(., ky, kz) of a (nz, ny, nx[, 2]) device tensor, to the host."""
    import torch
    kz = torch.tensor([b for _, b in kyz], device=t.device)
    ky = torch.tensor([a for a, _ in kyz], device=t.device)
    return t[kz, ky].cpu().numpy()


def oracle_checks(checks):
    """Compare every collected GPU result with exact FP64 oracle lines (the
    CPU leg: runs after all GPU timing).  Each check is a dict with a
    `compute` callable returning (GPU lines, oracle lines) and a tolerance."""
    import oracle
    out = {}
    for c in checks:
        t0 = time.perf_counter()
        got, ref = c["compute"](oracle)
        err = oracle.rel_l2(got, ref)
        out[c["name"]] = {"rel_l2": err, "tol": c["tol"], "ok": bool(err <= c["tol"]), "lines": c["lines"],
                          "what": c["what"], "oracle_s": time.perf_counter() - t0}
    return out


def calibrate_copy(torch, steps, warmup):
    """A plain device-to-device copy of 1 GiB, for scaling HBM counters."""
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    nbytes = 2 * src.numel() * 4
    print(json.dumps({"calibrate_copy_bytes": nbytes, "ms": ms, "GBps": nbytes / ms / 1e6}))


SETTLE_MS = 100.0


def settle(torch, fn, ms=SETTLE_MS):
    """Run `fn` untimed until `ms` of wall time has passed (four calls at
    least) and return the number of calls.  After the GPU has idled (the
    host generating or checking inputs), its first 10-20 transforms of a
    512^3 grid run 5-30% slower than the steady state while the clocks
    settle; this comes before the warm-up steps, which still run as asked."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    while True:
        for _ in range(4):
            fn()
            k += 1
        torch.cuda.synchronize()
        if (time.perf_counter() - t0) * 1e3 >= ms:
            return k


def time_plan(torch, croft, plan, fn, steps, warmup, npasses, settle_ms=SETTLE_MS):
    """Settle, warm up, then time exactly `steps` calls between two
    synchronisations, with per-pass HIP events recorded by the library."""
    if settle_ms > 0:
        settle(torch, fn, settle_ms)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    croft.croft_plan_profile(plan, True)
    stream = torch.cuda.current_stream()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    croft.croft_plan_profile(plan, False)
    pass_ms, n = croft.croft_plan_profile_read(plan, max(npasses, 1))
    ms = start.elapsed_time(end) / steps
    return ms, [m / max(n, 1) for m in pass_ms[:npasses]], wall


def rel_l2_dev(torch, a, b) -> float:
    """||a - b|| / ||b|| over complex128 views, on the device."""
    a = a.to(torch.complex128)
    b = b.to(torch.complex128)
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def measure_real(torch, np, croft, pme, steps):
    """Real forward (real grid -> half spectrum) and backward transforms of the
    PME grid, timed next to the complex64 transform of the same grid, with the
    error of the half spectrum against that transform's first half and the
    round-trip error."""
    n = pme.shape[0]
    N = n ** 3
    d_c = torch.from_numpy(pme).cuda()
    d_cy = torch.empty_like(d_c)
    cplan = croft.croft_plan_create(n, n, n, croft.CROFT_C64, croft.CROFT_FORWARD)
    ms_c64, _, _ = time_plan(torch, croft, cplan, lambda: croft.croft_execute(cplan, d_c, d_cy), steps, 3, 3)
    croft.croft_plan_destroy(cplan)
    d_x = d_c.real.contiguous()
    del d_c
    d_h = torch.empty((n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    d_back = torch.empty_like(d_x)
    out = {}
    for name, direction, src, dst in (("real_forward", croft.CROFT_FORWARD, d_x, d_h),
                                      ("real_backward", croft.CROFT_BACKWARD, d_h, d_back)):
        plan = croft.croft_plan_create_real(n, n, n, croft.CROFT_C64, direction, 0)
        info = croft.croft_plan_info(plan)
        ms, pm, _ = time_plan(torch, croft, plan, lambda: croft.croft_execute(plan, src, dst), steps, 3,
                              info["npasses"])
        croft.croft_plan_destroy(plan)
        out[name] = {"ms": ms, "GFLOPs_2.5NlogN": info["flops"] / ms / 1e6,
                     "effective_GBps": info["algorithmic_bytes"] / ms / 1e6,
                     "algorithmic_bytes": info["algorithmic_bytes"], "pass_ms": pm,
                     "c2c_c64_ms": ms_c64, "speedup_vs_c2c": ms_c64 / ms}
    out["real_forward"]["rel_l2_vs_c2c_half"] = rel_l2_dev(torch, d_h, d_cy[:, :, : n // 2 + 1])
    out["real_backward"]["round_trip_rel_l2"] = rel_l2_dev(torch, (d_back / N).to(torch.complex64),
                                                           d_x.to(torch.complex64))
    del d_x, d_h, d_back, d_cy
    torch.cuda.empty_cache()
    return out


def measure_conv(torch, np, croft, synth, pme, steps):
    """The fused convolution plan (forward real transform, product with the
    PME influence function, backward real transform, energy) on the PME grid,
    timed next to the same steps run as separate plans, with the bitwise
    comparison of the two."""
    n = pme.shape[0]
    d_x = torch.from_numpy(np.ascontiguousarray(pme.real)).cuda()
    d_g = torch.from_numpy(synth.pme_influence(n, n, n).astype(np.float32)).cuda()
    out = torch.empty_like(d_x)
    d_e = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan = croft.croft_plan_create_convolution(n, n, n, croft.CROFT_C64, 0)
    info = croft.croft_plan_info(plan)
    ms, pm, _ = time_plan(torch, croft, plan,
                          lambda: croft.croft_execute_convolution(plan, d_x, d_g, out, d_e), steps, 3,
                          info["npasses"])
    croft.croft_plan_destroy(plan)
    # unfused: real forward plan, elementwise product (torch), real backward plan
    h = torch.empty((n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    ref = torch.empty_like(d_x)
    f = croft.croft_plan_create_real(n, n, n, croft.CROFT_C64, croft.CROFT_FORWARD, 0)
    b = croft.croft_plan_create_real(n, n, n, croft.CROFT_C64, croft.CROFT_BACKWARD, 0)
    hr = torch.view_as_real(h)
    g3 = d_g[..., None]

    def unfused():
        croft.croft_execute(f, d_x, h)
        hr.mul_(g3)
        croft.croft_execute(b, h, ref)
    settle(torch, unfused)
    for _ in range(3):
        unfused()
    torch.cuda.synchronize()
    a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a_.record()
    for _ in range(steps):
        unfused()
    b_.record()
    torch.cuda.synchronize()
    ms_unfused = a_.elapsed_time(b_) / steps
    croft.croft_plan_destroy(f)
    croft.croft_plan_destroy(b)
    res = {"ms": ms, "effective_GBps": info["algorithmic_bytes"] / ms / 1e6,
           "algorithmic_bytes": info["algorithmic_bytes"], "pass_ms": pm, "energy": float(d_e.item()),
           "unfused_ms": ms_unfused, "speedup_vs_unfused": ms_unfused / ms,
           "bitwise_equal_to_unfused": bool(torch.equal(out, ref))}
    del d_x, d_g, out, h, ref
    torch.cuda.empty_cache()
    return res


def measure_large(torch, np, croft, pme, steps, checks):
    """A 1024^3 complex64 PME grid (8 GiB), forward, out of place: the 512^3
    PME grid repeated 2 x 2 x 2 on the device (a periodic charge grid of the
    same density; generating a fresh 1024^3 grid on the host takes a minute).
    Its exact lines follow from the 512^3 grid's: the repeated grid's
    transform is 8 Y512(k/2) where every component of k is even, else 0."""
    n = 1024
    half = torch.from_numpy(pme).cuda()
    d_in = half.repeat(2, 2, 2)
    qtot = 8.0 * float(half.real.to(torch.float64).sum())
    del half
    d_out = torch.empty_like(d_in)
    plan = croft.croft_plan_create(n, n, n, croft.CROFT_C64, croft.CROFT_FORWARD)
    info = croft.croft_plan_info(plan)
    ms, pm, _ = time_plan(torch, croft, plan, lambda: croft.croft_execute(plan, d_in, d_out), steps, 2, 3)
    croft.croft_plan_destroy(plan)
    dc = d_out[0, 0, 0].item()
    half_pairs = sample_pairs(n // 2, n // 2, 8, seed=12)
    kyz = [(2 * a, 2 * b) for a, b in half_pairs] + [(1, 0), (n - 2, 3)]
    got = device_lines(d_out, kyz)
    del d_in, d_out
    torch.cuda.empty_cache()

    def compute(o):
        y512 = o.dft3d_lines(pme, half_pairs, -1)
        ref = np.zeros((len(kyz), n), np.complex128)
        ref[: len(half_pairs), 0::2] = 8.0 * y512
        return got, ref
    checks.append({"name": "c64_1024cube", "compute": compute, "tol": 1e-5, "lines": len(kyz),
                   "what": "8 lines with even (ky, kz) from 8 x the oracle lines of the 512^3 grid at "
                           "half the frequencies, 2 lines with an odd component (exactly zero)"})
    return {"ms": ms, "GFLOPs": flops_5nlogn(n ** 3) / ms / 1e6,
            "effective_GBps": info["algorithmic_bytes"] / ms / 1e6,
            "effective_frac_of_8TBps": info["algorithmic_bytes"] / ms / 1e6 / HBM_PEAK_GBPS, "pass_ms": pm,
            "dc_minus_total_charge": dc.real - qtot}


def measure_c128(torch, np, croft, pme, steps, checks):
    """The paper's own precision (double complex, Section 5): forward 512^3
    complex128 on the same PME grid, FP64 compute, with the roofline of its
    dominant pass (2 N 16 bytes per launch against 8 TB/s)."""
    n = pme.shape[0]
    N = n ** 3
    d_in = torch.from_numpy(pme.astype(np.complex128)).cuda()
    d_out = torch.empty_like(d_in)
    plan = croft.croft_plan_create(n, n, n, croft.CROFT_C128, croft.CROFT_FORWARD)
    info = croft.croft_plan_info(plan)
    ms, pm, _ = time_plan(torch, croft, plan, lambda: croft.croft_execute(plan, d_in, d_out), steps, 3, 3)
    croft.croft_plan_destroy(plan)
    kyz = sample_pairs(n, n, 8, seed=13)
    got = device_lines(d_out, kyz)
    del d_in, d_out
    torch.cuda.empty_cache()
    checks.append({"name": "c128_512cube", "compute": lambda o: (got, o.dft3d_lines(pme, kyz, -1)),
                   "tol": 1e-12, "lines": len(kyz), "what": "exact oracle lines of the complex128 transform"})
    dom = max(range(3), key=lambda i: pm[i])
    per_launch = 2.0 * N * 16
    achieved = per_launch / pm[dom] / 1e6
    return {"ms": ms, "GFLOPs": flops_5nlogn(N) / ms / 1e6,
            "effective_GBps": info["algorithmic_bytes"] / ms / 1e6,
            "effective_frac_of_8TBps": info["algorithmic_bytes"] / ms / 1e6 / HBM_PEAK_GBPS, "pass_ms": pm,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBPS, "traffic": None,
                         "kernel": f"pass {'xyz'[dom]}", "bytes_per_launch": per_launch,
                         "avg_launch_ms": pm[dom]}}


def measure_bluestein(torch, np, croft, synth, steps, checks, smooth_ms):
    """Lengths with a large prime factor (Bluestein's algorithm): a forward
    509^3 complex64 transform (509 is prime; every axis runs as a chirp-
    multiplied convolution of length 1024 held in LDS), N(0,1) input, next to
    the 512^3 transform of nearly the same size."""
    n = 509
    N = n ** 3
    x = synth.normal_c((n, n, n), seed=6).astype(np.complex64)
    d_in = torch.from_numpy(x).cuda()
    d_out = torch.empty_like(d_in)
    plan = croft.croft_plan_create(n, n, n, croft.CROFT_C64, croft.CROFT_FORWARD)
    info = croft.croft_plan_info(plan)
    ms, pm, _ = time_plan(torch, croft, plan, lambda: croft.croft_execute(plan, d_in, d_out), steps, 3, 3)
    croft.croft_plan_destroy(plan)
    kyz = sample_pairs(n, n, 8, seed=16)
    got = device_lines(d_out, kyz)
    del d_in, d_out
    torch.cuda.empty_cache()
    checks.append({"name": "bluestein_509cube", "compute": lambda o: (got, o.dft3d_lines(x, kyz, -1)),
                   "tol": 1e-5, "lines": len(kyz), "what": "exact oracle lines of the 509^3 transform"})
    return {"ms": ms, "GFLOPs": flops_5nlogn(N) / ms / 1e6,
            "effective_GBps": info["algorithmic_bytes"] / ms / 1e6,
            "effective_frac_of_8TBps": info["algorithmic_bytes"] / ms / 1e6 / HBM_PEAK_GBPS, "pass_ms": pm,
            "bluestein_length": info["passes"][0]["bluestein"],
            "c64_512cube_ms": smooth_ms, "time_vs_512cube": ms / smooth_ms}


def measure_unfused(torch, np, croft, pme, steps, fused_ms):
    """The paper's Option 2 (no overlap; pack / all-to-all / unpack as
    separate sweeps, Section 5.1) on one GPU: the unfused plan, whose three
    FFTs run on contiguous lines with three standalone LDS-tiled transposes
    of the whole grid, on the same 512^3 PME grid, beside the fused plan."""
    n = pme.shape[0]
    N = n ** 3
    d_in = torch.from_numpy(pme).cuda()
    d_out = torch.empty_like(d_in)
    plan = croft.croft_plan_create_ex(n, n, n, croft.CROFT_C64, croft.CROFT_FORWARD, croft.CROFT_UNFUSED, 0)
    ms, pm, _ = time_plan(torch, croft, plan, lambda: croft.croft_execute(plan, d_in, d_out), steps, 3, 6)
    croft.croft_plan_destroy(plan)
    del d_in, d_out
    torch.cuda.empty_cache()
    sweep = 2.0 * N * 8
    return {"ms": ms, "fused_ms": fused_ms, "fusion_speedup": ms / fused_ms,
            "fft_pass_ms": [pm[0], pm[2], pm[4]], "transpose_ms": [pm[1], pm[3], pm[5]],
            "transpose_GBps": [sweep / t / 1e6 for t in (pm[1], pm[3], pm[5])],
            "bytes_moved": 12.0 * N * 8, "effective_GBps_of_moved": 12.0 * N * 8 / ms / 1e6}


def copy_bandwidth(torch, nbytes=1 << 31, reps=10):
    """GB/s of a plain device-to-device copy of nbytes (read + write counted)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / ms / 1e6


def measure_configs(torch, np, croft, synth):
    """The smaller cubes: 32^3 (U[-1,1), latency-bound: median of 200
    individually timed calls, and the round trip), and 256^3 and 384^3
    (N(0,1)) forward and inverse, warm (back to back) and with the 256 MB
    Infinity Cache flushed before each call by writing a 512 MiB buffer."""
    out = {}
    a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def one(fn, flush=None):
        if flush is not None:
            flush.fill_(0.0)
        a_.record()
        fn()
        b_.record()
        torch.cuda.synchronize()
        return a_.elapsed_time(b_)

    # 32^3
    n = 32
    x = torch.from_numpy(synth.uniform_c((n, n, n), seed=1).astype(np.complex64)).cuda()
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    f = croft.croft_plan_create(n, n, n, croft.CROFT_C64, croft.CROFT_FORWARD)
    bk = croft.croft_plan_create(n, n, n, croft.CROFT_C64, croft.CROFT_BACKWARD)
    for _ in range(20):
        croft.croft_execute(f, x, y)
    t_f = [one(lambda: croft.croft_execute(f, x, y)) for _ in range(200)]
    t_b = [one(lambda: croft.croft_execute(bk, y, z)) for _ in range(200)]
    croft.croft_plan_destroy(f)
    croft.croft_plan_destroy(bk)
    # the same transform as one cooperative launch (a batched plan of one grid)
    c = croft.croft_plan_create_batched([(n, n, n)], croft.CROFT_C64, croft.CROFT_FORWARD, croft.CROFT_PERSISTENT)
    yc = torch.empty_like(x)
    for _ in range(20):
        croft.croft_execute_batched(c, x, yc)
    t_c = [one(lambda: croft.croft_execute_batched(c, x, yc)) for _ in range(200)]
    croft.croft_plan_destroy(c)
    # and replayed from a captured graph
    c = croft.croft_plan_create_batched([(n, n, n)], croft.CROFT_C64, croft.CROFT_FORWARD,
                                        croft.CROFT_PERSISTENT | croft.CROFT_GRAPH)
    yg = torch.empty_like(x)
    for _ in range(20):
        croft.croft_execute_batched(c, x, yg)
    t_g = [one(lambda: croft.croft_execute_batched(c, x, yg)) for _ in range(200)]
    croft.croft_plan_destroy(c)
    out["c64_32cube"] = {"forward_median_us": 1e3 * float(np.median(t_f)),
                         "inverse_median_us": 1e3 * float(np.median(t_b)),
                         "forward_one_launch_median_us": 1e3 * float(np.median(t_c)),
                         "one_launch_bitwise_equal": bool(torch.equal(yc, y)),
                         "forward_one_launch_graph_median_us": 1e3 * float(np.median(t_g)),
                         "one_launch_graph_bitwise_equal": bool(torch.equal(yg, y)),
                         "round_trip_rel_l2": rel_l2_dev(torch, z / n ** 3, x)}
    flush = torch.empty(1 << 27, dtype=torch.float32, device="cuda")  # 512 MiB
    for n in (256, 384):
        x = torch.from_numpy(synth.normal_c((n, n, n), seed=2).astype(np.complex64)).cuda()
        y = torch.empty_like(x)
        z = torch.empty_like(x)
        f = croft.croft_plan_create(n, n, n, croft.CROFT_C64, croft.CROFT_FORWARD)
        bk = croft.croft_plan_create(n, n, n, croft.CROFT_C64, croft.CROFT_BACKWARD)
        info = croft.croft_plan_info(f)
        r = {}
        for name, fn in (("forward", lambda: croft.croft_execute(f, x, y)),
                         ("inverse", lambda: croft.croft_execute(bk, y, z))):
            settle(torch, fn)
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            a_.record()
            for _ in range(50):
                fn()
            b_.record()
            torch.cuda.synchronize()
            warm = a_.elapsed_time(b_) / 50
            flushed = float(np.median([one(fn, flush) for _ in range(20)]))
            r[name + "_warm_ms"] = warm
            r[name + "_flushed_ms"] = flushed
        r["GFLOPs_warm"] = flops_5nlogn(n ** 3) / r["forward_warm_ms"] / 1e6
        r["effective_GBps_flushed"] = info["algorithmic_bytes"] / r["forward_flushed_ms"] / 1e6
        r["round_trip_rel_l2"] = rel_l2_dev(torch, z / n ** 3, x)
        croft.croft_plan_destroy(f)
        croft.croft_plan_destroy(bk)
        out[f"c64_{n}cube"] = r
        del x, y, z
    del flush
    torch.cuda.empty_cache()
    return out


def measure_shard_share(torch, np, croft, steps):
    """One GPU's share of a 1024^3 complex64 transform split over 8 GPUs by
    z-slabs (design only: no second GPU here): the x and y passes of a
    1024 x 1024 x 128 slab, and the z pass of the 1024 x 128 x 1024 y-slab it
    holds after the all-to-all, each timed from the library's per-pass
    events; the exchange itself is modeled (each GPU sends 1/8 of its 1 GiB
    to each of 7 peers over its own xGMI link at about 153 GB/s)."""
    out = {}
    for name, dims, keep in (("xy_slab_1024x1024x128", (1024, 1024, 128), (0, 1)),
                             ("z_slab_1024x128x1024", (1024, 128, 1024), (2,))):
        nx, ny, nz = dims
        d_in = torch.zeros((nz, ny, nx), dtype=torch.complex64, device="cuda")
        d_in.real.normal_()
        d_out = torch.empty_like(d_in)
        plan = croft.croft_plan_create(nx, ny, nz, croft.CROFT_C64, croft.CROFT_FORWARD)
        info = croft.croft_plan_info(plan)
        _, pm, _ = time_plan(torch, croft, plan, lambda: croft.croft_execute(plan, d_in, d_out), steps, 2,
                             info["npasses"])
        croft.croft_plan_destroy(plan)
        axes = [p["axis"] for p in info["passes"]]
        out[name] = {"pass_ms": {"xyz"[a]: pm[i] for i, a in enumerate(axes) if a in keep}}
        del d_in, d_out
        torch.cuda.empty_cache()
    local = sum(out["xy_slab_1024x1024x128"]["pass_ms"].values()) + out["z_slab_1024x128x1024"]["pass_ms"]["z"]
    exchange = (2 ** 30 / 8) / 153e9 * 1e3
    out["local_ms"] = local
    out["modeled_exchange_ms_each"] = exchange
    out["modeled_8gpu_ms"] = local + 2 * exchange
    out["modeled_8gpu_ms_transposed_output"] = local + exchange
    return out


def measure_forms(torch, np, croft, synth, steps, checks, only=None, coop=True):
    """Half-storage (512^3) and batched (64 uneven grids) forms, each timed
    next to the plain complex64 form on the same input and GPU, with its error
    against that form (only="half": the half-storage forms alone)."""
    out = {}
    n = 512
    N = n ** 3
    v = synth.normal_c((n, n, n), seed=5)
    # the complex64 transform of the input before quantisation, for the
    # information of the error it carries into the 16-bit forms
    d_orig = torch.from_numpy(v.astype(np.complex64)).cuda()
    orig_out = torch.empty_like(d_orig)
    oplan = croft.croft_plan_create(n, n, n, croft.CROFT_C64, croft.CROFT_FORWARD)
    croft.croft_execute(oplan, d_orig, orig_out)
    torch.cuda.synchronize()
    croft.croft_plan_destroy(oplan)
    del d_orig
    for name, dt, kind in (("c16f", croft.CROFT_C16F, "f16"), ("c16b", croft.CROFT_C16B, "bf16")):
        data, e = synth.quantize_half(v, kind)
        tdt = torch.float16 if kind == "f16" else torch.bfloat16
        d_in = torch.from_numpy(data.view(np.int16)).cuda().view(tdt)
        d_out = torch.empty_like(d_in)
        e_in = torch.from_numpy(e).cuda()
        e_out = torch.empty((n, n), dtype=torch.int8, device="cuda")
        plan = croft.croft_plan_create(n, n, n, dt, croft.CROFT_FORWARD)
        ms, pm, _ = time_plan(torch, croft, plan,
                              lambda: croft.croft_execute_scaled(plan, d_in, e_in, d_out, e_out),
                              steps, 3, 3)
        info = croft.croft_plan_info(plan)
        croft.croft_plan_destroy(plan)
        # the plain complex64 form on the stored input's exact values
        vals = (d_in.float()[..., 0] + 1j * d_in.float()[..., 1]).to(torch.complex64)
        vals = vals * torch.pow(2.0, e_in.float())[:, :, None]
        c_out = torch.empty_like(vals)
        cplan = croft.croft_plan_create(n, n, n, croft.CROFT_C64, croft.CROFT_FORWARD)
        ms_c64, _, _ = time_plan(torch, croft, cplan, lambda: croft.croft_execute(cplan, vals, c_out),
                                 steps, 3, 3)
        croft.croft_plan_destroy(cplan)
        got = (d_out.float()[..., 0] + 1j * d_out.float()[..., 1]) * torch.pow(2.0, e_out.float())[None, :, :]
        err = rel_l2_dev(torch, got, c_out)
        kyz = sample_pairs(n, n, 8, seed=14)
        bits = device_lines(d_out.view(torch.int16), kyz).view(np.uint16)      # (8, nx, 2)
        oe = e_out.cpu().numpy()
        line_exp = np.stack([oe[ky] for ky, _ in kyz])                       # z-line exponents (x)

        def compute(o, data=data, e=e, kind=kind, kyz=kyz, bits=bits, line_exp=line_exp):
            # sampled line i holds the z-lines (x, ky_i): exponents oe[ky_i, :]
            gl = o.decode_half(bits[:, None], line_exp, kind, 1)[:, 0]
            return gl, o.dft3d_lines(o.decode_half(data, e, kind, 0), kyz, -1)
        checks.append({"name": name, "compute": compute, "tol": 5e-3, "lines": len(kyz),
                       "what": "exact oracle lines of the decoded stored input"})
        err_orig = rel_l2_dev(torch, got, orig_out)
        out[name] = {"ms": ms, "GFLOPs": flops_5nlogn(N) / ms / 1e6,
                     "effective_GBps": info["algorithmic_bytes"] / ms / 1e6, "pass_ms": pm,
                     "c64_ms": ms_c64, "speedup_vs_c64": ms_c64 / ms, "rel_l2_vs_c64": err,
                     "rel_l2_vs_c64_of_unquantised_input": err_orig}
        del d_in, d_out, vals, c_out, got
        torch.cuda.empty_cache()
    del orig_out
    torch.cuda.empty_cache()
    if only == "half":
        return out
    # batched: 64 uneven PME grids
    dims = synth.batch_dims(4)
    grids = [synth.pme_grid(int(a), int(b), int(c), seed=400 + i)[0] for i, (a, b, c) in enumerate(dims)]
    flat = np.concatenate([g.ravel() for g in grids]).astype(np.complex64)
    d_in = torch.from_numpy(flat).cuda()
    d_out = torch.empty_like(d_in)
    fl = sum(flops_5nlogn(int(a) * int(b) * int(c)) for a, b, c in dims)
    a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_batched(flags, dst):
        plan = croft.croft_plan_create_batched([tuple(int(t) for t in d) for d in dims], croft.CROFT_C64,
                                               croft.CROFT_FORWARD, flags)
        settle(torch, lambda: croft.croft_execute_batched(plan, d_in, dst))
        for _ in range(3):
            croft.croft_execute_batched(plan, d_in, dst)
        torch.cuda.synchronize()
        a_.record()
        for _ in range(steps):
            croft.croft_execute_batched(plan, d_in, dst)
        b_.record()
        torch.cuda.synchronize()
        info = croft.croft_plan_info(plan)
        croft.croft_plan_destroy(plan)
        return a_.elapsed_time(b_) / steps, info
    ms, info = time_batched(0, d_out)
    # tile shapes chosen by the autotuner on this GPU (nothing read or written to a wisdom file)
    d_meas = torch.empty_like(d_in)
    ms_meas, _ = time_batched(croft.CROFT_MEASURE | croft.CROFT_NO_WISDOM, d_meas)
    # the same launches replayed from a captured graph
    d_graph = torch.empty_like(d_in)
    ms_graph, _ = time_batched(croft.CROFT_GRAPH, d_graph)
    if coop:
        d_coop = torch.empty_like(d_in)
        ms_coop, _ = time_batched(croft.CROFT_PERSISTENT, d_coop)
    # the same grids as separate plain plans on one stream
    plans = [croft.croft_plan_create(int(a), int(b), int(c), croft.CROFT_C64, croft.CROFT_FORWARD)
             for a, b, c in dims]
    offs = np.concatenate([[0], np.cumsum([g.size for g in grids])])
    ref = torch.empty_like(d_in)
    views = [(d_in[offs[i]:offs[i + 1]], ref[offs[i]:offs[i + 1]]) for i in range(len(grids))]

    def plain_all():
        for p, (i_, o_) in zip(plans, views):
            croft.croft_execute(p, i_, o_)
    settle(torch, plain_all)
    for _ in range(3):
        plain_all()
    torch.cuda.synchronize()
    a_.record()
    for _ in range(steps):
        plain_all()
    b_.record()
    torch.cuda.synchronize()
    ms_plain = a_.elapsed_time(b_) / steps
    for p in plans:
        croft.croft_plan_destroy(p)
    out["batched_64"] = {"ms": ms, "GFLOPs": fl / ms / 1e6, "elements": int(flat.size),
                         "effective_GBps": info["algorithmic_bytes"] / ms / 1e6,
                         "plain_calls_ms": ms_plain, "speedup_vs_plain_calls": ms_plain / ms,
                         "bitwise_equal_to_plain_calls": bool(torch.equal(d_out, ref)),
                         "measured_shapes_ms": ms_meas,
                         "measured_shapes_bitwise_equal": bool(torch.equal(d_meas, d_out)),
                         "graph_replay_ms": ms_graph,
                         "graph_replay_bitwise_equal": bool(torch.equal(d_graph, d_out))}
    if coop:
        out["batched_64"]["cooperative_ms"] = ms_coop
        out["batched_64"]["cooperative_bitwise_equal"] = bool(torch.equal(d_coop, d_out))
    # two exact lines per grid
    host_out = d_out.cpu().numpy()
    per = []
    for i, (a, b, c) in enumerate(dims):
        nx, ny, nz = int(a), int(b), int(c)
        kyz = sample_pairs(ny, nz, 3, seed=500 + i)[:2]
        g = host_out[offs[i]:offs[i + 1]].reshape(nz, ny, nx)
        per.append((flat[offs[i]:offs[i + 1]].reshape(nz, ny, nx), kyz, np.stack([g[kz, ky] for ky, kz in kyz])))

    def compute(o):
        got = np.concatenate([gl.ravel() for _, _, gl in per])
        ref = np.concatenate([o.dft3d_lines(x, kyz, -1).ravel() for x, kyz, _ in per])
        return got, ref
    checks.append({"name": "batched_64", "compute": compute, "tol": 1e-5, "lines": 2 * len(dims),
                   "what": "2 exact oracle lines of each of the 64 grids"})
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2002_04896_amd as croft
    from paper_2002_04896_amd import synth

    if args.calibrate_copy:
        calibrate_copy(torch, args.steps, args.warmup)
        return
    checks = []
    if args.only_form == "half":
        print(json.dumps({"forms": measure_forms(torch, np, croft, synth, args.steps, checks, only="half")}))
        return

    n = args.size
    N = n ** 3
    grid, qtot = synth.pme_grid(n, n, n, seed=3)
    x = grid.astype(np.complex64)                      # imag = 0, real part rounded to FP32
    del grid
    d_in = torch.from_numpy(x).cuda()
    d_out = torch.empty_like(d_in)
    plan = croft.croft_plan_create_ex(n, n, n, croft.CROFT_C64, croft.CROFT_FORWARD, 0, args.slabs)
    info = croft.croft_plan_info(plan)
    npasses = info["npasses"]
    head = lambda: croft.croft_execute(plan, d_in, d_out)
    settle_steps = settle(torch, head)
    ms, pass_ms, _ = time_plan(torch, croft, plan, head, args.steps, args.warmup, npasses, settle_ms=0)
    # sanity: DC bin equals the total charge
    dc = d_out[0, 0, 0].item()
    croft.croft_plan_destroy(plan)
    kyz = sample_pairs(n, n, 8, seed=11)
    head_lines = device_lines(d_out, kyz)
    checks.append({"name": f"c64_{n}cube", "compute": lambda o: (head_lines, o.dft3d_lines(x, kyz, -1)),
                   "tol": 1e-5, "lines": len(kyz), "what": "exact oracle lines of the headline transform"})
    copy_gbps = copy_bandwidth(torch)

    gflops = flops_5nlogn(N) / ms / 1e6
    alg_bytes = info["algorithmic_bytes"]
    dom = max(range(npasses), key=lambda i: pass_ms[i])
    pinfo = info["passes"][dom]
    per_launch = 2.0 * N * info["element_bytes"]       # one sweep: read + write every element
    achieved = per_launch / pass_ms[dom] / 1e6         # GB/s
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        if t.get("kernel_hash") == kernel_hash() and t.get("pass") == dom and t.get("size") == n:
            traffic = t.get("bytes_per_launch")
    line = {
        "metric": METRIC, "value": gflops, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "settle": {"ms": SETTLE_MS, "steps": settle_steps,
                   "what": "untimed transforms before the warm-up steps, until the GPU clocks settle after "
                           "the host-side input generation (every form is timed the same way)"},
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"forward C2C 3D FFT {n}^3 complex64, PME charge grid "
                               f"(one +-1 charge per cell, order-4 B-spline), out of place",
                   "nx": n, "ny": n, "nz": n, "slabs": args.slabs, "parallelism": "single GPU"},
        "effective_hbm_GBps": alg_bytes / ms / 1e6,
        "effective_frac_of_8TBps": alg_bytes / ms / 1e6 / HBM_PEAK_GBPS,
        "copy_GBps": copy_gbps,
        "effective_frac_of_copy": alg_bytes / ms / 1e6 / copy_gbps,
        "pass_ms": pass_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": f"pass {'xyz'[pinfo['axis']]} "
                               f"({'contiguous' if pinfo['kind'] == 0 else 'strided'}, "
                               f"radices {'x'.join(map(str, pinfo['radices']))})",
                     "bytes_per_launch": per_launch, "avg_launch_ms": pass_ms[dom]},
        "check": {"dc": [dc.real, dc.imag], "total_charge": qtot},
    }
    if not args.no_forms:
        del d_in, d_out
        torch.cuda.empty_cache()
        line["forms"] = measure_real(torch, np, croft, x, max(10, args.steps // 2))
        line["forms"]["convolution"] = measure_conv(torch, np, croft, synth, x, max(10, args.steps // 2))
        line["forms"]["c128_512cube"] = measure_c128(torch, np, croft, x, max(10, args.steps // 2), checks)
        line["forms"]["option2_unfused_512cube"] = measure_unfused(torch, np, croft, x, max(10, args.steps // 2), ms)
        line["forms"]["bluestein_509cube"] = measure_bluestein(torch, np, croft, synth, max(10, args.steps // 2),
                                                               checks, ms)
        line["forms"]["c64_1024cube"] = measure_large(torch, np, croft, x, max(5, args.steps // 5), checks)
        line["forms"].update(measure_forms(torch, np, croft, synth, max(10, args.steps // 2), checks,
                                           coop=not args.no_coop))
        line["configs"] = measure_configs(torch, np, croft, synth)
        line["forms"]["shard_share_1024cube_8gpu"] = measure_shard_share(torch, np, croft, max(5, args.steps // 5))
    if not args.no_cpu_baseline:
        # the CPU leg, after every GPU measurement: the oracle's own rate on
        # a bounded sample, and exact oracle lines against each GPU result
        line["oracle_check"] = oracle_checks(checks)
        line["cpu_baseline"] = cpu_baseline(x, n)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
