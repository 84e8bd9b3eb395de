"""Injected allocation failures: with CROFT_TEST_FAIL_ALLOC=k the k-th device
allocation of a plan creation fails.  Every such failure must come back as
CROFT_ERR_OUT_OF_MEMORY with a message, free what the creation had already
allocated, and leave the library usable.  The failure is forced on the host;
no kernel runs in a failing state."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_04896_amd as croft

pytestmark = pytest.mark.gpu

C64, C128, C16F = croft.CROFT_C64, croft.CROFT_C128, croft.CROFT_C16F
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD
MEASURE = croft.CROFT_MEASURE | croft.CROFT_NO_WISDOM

# (name, create): one of each kind of plan-owned memory -- twiddle tables,
# Bluestein tables, half-storage exponents, the real backward work buffer,
# the energy partials, the unfused work grid, batch tables, and the
# autotuners' scratch (passes, slab count, batched tile shapes)
CASES = [
    ("plain", lambda: croft.croft_plan_create(48, 60, 64, C64, FWD)),
    ("bluestein", lambda: croft.croft_plan_create(97, 8, 6, C128, BWD)),
    ("half", lambda: croft.croft_plan_create(64, 32, 16, C16F, FWD)),
    ("real-backward", lambda: croft.croft_plan_create_real(64, 40, 48, C64, BWD)),
    ("convolution", lambda: croft.croft_plan_create_convolution(64, 40, 48, C64)),
    ("unfused", lambda: croft.croft_plan_create_ex(64, 40, 48, C64, FWD, croft.CROFT_UNFUSED, 1)),
    ("batched", lambda: croft.croft_plan_create_batched([(48, 60, 64), (8, 1, 3)], C64, FWD)),
    ("measure", lambda: croft.croft_plan_create_ex(128, 128, 64, C64, FWD, MEASURE, 1)),
    ("measure-slabs", lambda: croft.croft_plan_create_ex(128, 64, 32, C64, FWD, MEASURE, 0)),
    ("measure-batched", lambda: croft.croft_plan_create_batched([(48, 60, 64), (64, 64, 64)], C64, FWD,
                                                                MEASURE)),
]


@pytest.fixture
def fail_at(monkeypatch):
    def set_k(k):
        if k:
            monkeypatch.setenv("CROFT_TEST_FAIL_ALLOC", str(k))
        else:
            monkeypatch.delenv("CROFT_TEST_FAIL_ALLOC", raising=False)
    yield set_k
    monkeypatch.delenv("CROFT_TEST_FAIL_ALLOC", raising=False)


@pytest.mark.parametrize("name,create", CASES, ids=[c[0] for c in CASES])
def test_every_allocation_failure_is_reported_and_cleaned_up(name, create, fail_at):
    print(f"injected allocation failures: {name}", flush=True)
    fail_at(0)
    croft.croft_plan_destroy(create())   # loads the code objects the creation needs
    torch.cuda.synchronize()
    free_before = torch.cuda.mem_get_info()[0]
    failures = 0
    for k in range(1, 64):
        fail_at(k)
        try:
            plan = create()
        except croft.CroftError as e:
            assert f"status {croft.CROFT_ERR_OUT_OF_MEMORY}" in str(e), (k, str(e))
            assert croft.croft_last_status() == croft.CROFT_ERR_OUT_OF_MEMORY
            failures += 1
            continue
        croft.croft_plan_destroy(plan)   # k is past the creation's last allocation
        break
    else:
        pytest.fail(f"{name}: still failing after 63 allocations")
    assert failures >= 1, name
    fail_at(0)
    torch.cuda.synchronize()
    # every failed creation freed what it had allocated (these plans own at
    # most a few MiB each, and 1..k-1 creations failed part way)
    assert torch.cuda.mem_get_info()[0] >= free_before - (8 << 20), name


def test_library_works_after_injected_failures(fail_at):
    fail_at(1)
    with pytest.raises(croft.CroftError, match="out of memory"):
        croft.croft_plan_create(32, 32, 32, C64, FWD)
    fail_at(0)
    rng = np.random.Generator(np.random.PCG64(90))
    x = (rng.standard_normal((32, 32, 32)) + 1j * rng.standard_normal((32, 32, 32))).astype(np.complex64)
    d = torch.from_numpy(x).cuda()
    out = torch.empty_like(d)
    plan = croft.croft_plan_create(32, 32, 32, C64, FWD)
    try:
        croft.croft_execute(plan, d, out)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    assert oracle.rel_l2(out.cpu().numpy(), oracle.dft3d(x.astype(np.complex128), FWD)) <= 1e-5
    assert croft.croft_last_status() == croft.CROFT_SUCCESS
