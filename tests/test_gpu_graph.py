"""croft_execute, croft_execute_convolution and croft_execute_batched under
HIP graph capture.

The execute calls launch kernels only (no allocation, copy or host
synchronisation), so a caller may capture them.  Each test captures one call
with torch.cuda.graph, then replays the graph several times with eager work of
its own and synchronisations in between, and checks every replay bit for bit
against the eager result.
"""
import numpy as np
import pytest
import torch

import paper_2002_04896_amd as croft
from paper_2002_04896_amd import synth

pytestmark = pytest.mark.gpu

C64 = croft.CROFT_C64
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD


def replay_and_check(graph, out, ref, noise):
    for rep in range(3):
        out.fill_(float("nan"))
        noise()                              # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep}"


def noise_fn():
    a = torch.randn(1 << 20, device="cuda")
    return lambda: a.mul_(1.0001).sum()


@pytest.mark.parametrize("slabs", [1, 4])
def test_complex_plan_capture(slabs):
    nx, ny, nz = 64, 48, 40
    x = torch.from_numpy(synth.normal_c((nz, ny, nx), seed=71).astype(np.complex64)).cuda()
    ref = torch.empty_like(x)
    out = torch.empty_like(x)
    plan = croft.croft_plan_create_ex(nx, ny, nz, C64, FWD, 0, slabs)
    try:
        croft.croft_execute(plan, x, ref)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            croft.croft_execute(plan, x, out)          # warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            croft.croft_execute(plan, x, out)
        replay_and_check(g, out, ref, noise_fn())
    finally:
        torch.cuda.synchronize()
        croft.croft_plan_destroy(plan)


@pytest.mark.parametrize("direction", [FWD, BWD], ids=["r2c", "c2r"])
def test_real_plan_capture(direction):
    nx, ny, nz = 64, 40, 24
    if direction == FWD:
        x = torch.from_numpy(synth.normal_c((nz, ny, nx), seed=72).real.astype(np.float32)).cuda()
        out_shape, out_dtype = (nz, ny, nx // 2 + 1), torch.complex64
    else:
        x = torch.from_numpy(synth.normal_c((nz, ny, nx // 2 + 1), seed=72).astype(np.complex64)).cuda()
        out_shape, out_dtype = (nz, ny, nx), torch.float32
    ref = torch.empty(out_shape, dtype=out_dtype, device="cuda")
    out = torch.empty_like(ref)
    plan = croft.croft_plan_create_real(nx, ny, nz, C64, direction, 0)
    try:
        croft.croft_execute(plan, x, ref)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            croft.croft_execute(plan, x, out)
        replay_and_check(g, out if out_dtype == torch.float32 else torch.view_as_real(out),
                         ref if out_dtype == torch.float32 else torch.view_as_real(ref), noise_fn())
    finally:
        torch.cuda.synchronize()
        croft.croft_plan_destroy(plan)


def test_convolution_capture_with_energy():
    nx, ny, nz = 64, 48, 32
    x = torch.from_numpy(synth.normal_c((nz, ny, nx), seed=73).real.astype(np.float32)).cuda()
    g_mul = torch.from_numpy(synth.pme_influence(nx, ny, nz).astype(np.float32)).cuda()
    ref = torch.empty_like(x)
    ref_e = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = torch.empty_like(x)
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan = croft.croft_plan_create_convolution(nx, ny, nz, C64, 0)
    try:
        croft.croft_execute_convolution(plan, x, g_mul, ref, ref_e)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            croft.croft_execute_convolution(plan, x, g_mul, out, e)
        noise = noise_fn()
        for rep in range(3):
            out.fill_(float("nan"))
            e.fill_(float("nan"))
            noise()
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, ref) and torch.equal(e, ref_e), f"replay {rep}"
    finally:
        torch.cuda.synchronize()
        croft.croft_plan_destroy(plan)


@pytest.mark.parametrize("flags", [0, croft.CROFT_PERSISTENT], ids=["per-pass", "cooperative"])
def test_batched_plan_capture(flags):
    """Without CROFT_GRAPH a batched plan issues its launches directly (one
    per pass, or one cooperative launch, plus the own launches of a grid the
    batched kernels do not compile), so a caller may capture the call."""
    dims = [(48, 60, 64), (64, 64, 64), (45, 27, 2)]
    total = sum(a * b * c for a, b, c in dims)
    rng = np.random.Generator(np.random.PCG64(74))
    x = torch.from_numpy((rng.standard_normal(total) + 1j * rng.standard_normal(total)).astype(np.complex64)).cuda()
    ref = torch.empty_like(x)
    out = torch.empty_like(x)
    plan = croft.croft_plan_create_batched(dims, C64, FWD, flags)
    try:
        croft.croft_execute_batched(plan, x, ref)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            croft.croft_execute_batched(plan, x, out)  # warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            croft.croft_execute_batched(plan, x, out)
        replay_and_check(g, out, ref, noise_fn())
        assert croft.croft_plan_info(plan)["graph_replay"] == 0
    finally:
        torch.cuda.synchronize()
        croft.croft_plan_destroy(plan)
