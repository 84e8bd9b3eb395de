"""The cooperative single launch of batched plans (CROFT_PERSISTENT): every
pass of every grid in one launch, passes separated by grid-wide barriers.
It runs the same butterflies as the one-launch-per-pass form, so the tests
compare bit for bit against that form (itself checked against single-grid
plans and the oracle in test_gpu_parity.py)."""
import sys

import numpy as np
import pytest
import torch

import paper_2002_04896_amd as croft

pytestmark = pytest.mark.gpu

C64, C128 = croft.CROFT_C64, croft.CROFT_C128
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD

SMALL = [(48, 60, 64), (64, 64, 64)]
UNEVEN = [(48, 60, 64), (128, 72, 80), (100, 96, 48), (64, 64, 64), (80, 100, 72), (96, 128, 60),
          (8, 1, 3), (45, 27, 2), (1, 64, 1), (60, 1, 100)]


def batch_input(dims, dtype, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    total = sum(a * b * c for a, b, c in dims)
    npdt = np.complex64 if dtype == C64 else np.complex128
    return torch.from_numpy((rng.standard_normal(total) + 1j * rng.standard_normal(total)).astype(npdt)).cuda()


def run(dims, dtype, direction, flags, d_in, in_place=False):
    print(f"batched {len(dims)} grids dtype={dtype} dir={direction} flags={flags} in_place={in_place}",
          flush=True)
    sys.stdout.flush()
    plan = croft.croft_plan_create_batched(dims, dtype, direction, flags)
    try:
        out = d_in.clone() if in_place else torch.full_like(d_in, complex(float("nan"), 0))
        src = out if in_place else d_in
        croft.croft_execute_batched(plan, src, out)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    return out


def same_bits(a, b):
    return torch.equal(torch.view_as_real(a), torch.view_as_real(b))


@pytest.mark.parametrize("dtype,direction", [(C64, FWD), (C128, BWD)], ids=["c64-fwd", "c128-bwd"])
@pytest.mark.parametrize("dims", [SMALL, UNEVEN], ids=["two-grids", "ten-uneven"])
def test_cooperative_launch_equals_per_pass_launches(dims, dtype, direction):
    d_in = batch_input(dims, dtype, 81)
    ref = run(dims, dtype, direction, 0, d_in)
    for rep in range(3):
        got = run(dims, dtype, direction, croft.CROFT_PERSISTENT, d_in)
        assert same_bits(got, ref), rep


def test_cooperative_launch_in_place():
    d_in = batch_input(UNEVEN, C64, 82)
    ref = run(UNEVEN, C64, FWD, 0, d_in)
    got = run(UNEVEN, C64, FWD, croft.CROFT_PERSISTENT, d_in, in_place=True)
    assert same_bits(got, ref)


def test_cooperative_launch_against_the_oracle_and_replays():
    """The one-launch form on its own against the FP64 oracle, replayed from
    the plan's graph (CROFT_GRAPH): every replay, and a re-capture for new
    buffers, gives the same bits."""
    import oracle
    from paper_2002_04896_amd import synth
    dims = [tuple(int(v) for v in d) for d in synth.batch_dims(7, count=12)]
    grids = [synth.pme_grid(nx, ny, nz, seed=700 + i)[0] for i, (nx, ny, nz) in enumerate(dims)]
    flat = np.concatenate([g.ravel() for g in grids]).astype(np.complex64)
    d_in = torch.from_numpy(flat).cuda()
    plan = croft.croft_plan_create_batched(dims, C64, FWD, croft.CROFT_PERSISTENT | croft.CROFT_GRAPH)
    try:
        offs = croft.croft_plan_batched_offsets(plan, len(dims))
        outs = []
        for rep in range(4):
            out = torch.full_like(d_in, complex(float("nan"), 0))
            croft.croft_execute_batched(plan, d_in, out)
            torch.cuda.synchronize()
            outs.append(out)
        captured = croft.croft_plan_info(plan)["graph_replay"]
        print(f"cooperative launch captured in the plan's graph: {captured}", flush=True)
        assert captured == 1
        # new buffers: a new capture, counters still at zero
        d_in2 = d_in.clone()
        out2 = torch.full_like(d_in, complex(float("nan"), 0))
        croft.croft_execute_batched(plan, d_in2, out2)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    for o in outs[1:] + [out2]:
        assert same_bits(o, outs[0])
    got = outs[0].cpu().numpy()
    for i, (nx, ny, nz) in enumerate(dims):
        seen = flat[offs[i]:offs[i + 1]].reshape(nz, ny, nx).astype(np.complex128)
        err = oracle.rel_l2(got[offs[i]:offs[i + 1]].reshape(nz, ny, nx), oracle.dft3d(seen, FWD))
        assert err <= 1e-5, (i, dims[i], err)
