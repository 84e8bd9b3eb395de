"""Helpers shared by the GPU tests: run the library through its C ABI on
torch device memory and bring results back for the oracle."""
import numpy as np
import torch

import paper_2002_04896_amd as croft

TOL = {croft.CROFT_C64: 1e-5, croft.CROFT_C128: 1e-12, croft.CROFT_C16F: 5e-3, croft.CROFT_C16B: 5e-3}
NP_DTYPE = {croft.CROFT_C64: np.complex64, croft.CROFT_C128: np.complex128}


def to_device(x: np.ndarray, dtype: int) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x.astype(NP_DTYPE[dtype]))).cuda()


def run_fft(x: np.ndarray, dtype=croft.CROFT_C64, direction=croft.CROFT_FORWARD, inplace=False,
            flags=0, slabs=1, poison=True):
    """Transform x (numpy, shape (nz, ny, nx)) on the GPU; returns (input as
    the GPU saw it, as complex128; output as complex128; input after the call)."""
    nz, ny, nx = x.shape
    d_in = to_device(x, dtype)
    seen = d_in.cpu().numpy().astype(np.complex128)
    if inplace:
        d_out = d_in
    else:
        d_out = torch.empty_like(d_in)
        if poison:
            d_out.fill_(complex(float("nan"), float("nan")))
    plan = croft.croft_plan_create_ex(nx, ny, nz, dtype, direction, flags, slabs)
    try:
        croft.croft_execute(plan, d_in, d_out)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    return seen, d_out.cpu().numpy().astype(np.complex128), d_in.cpu().numpy().astype(np.complex128)


HALF_TORCH = {croft.CROFT_C16F: torch.float16, croft.CROFT_C16B: torch.bfloat16}
HALF_KIND = {croft.CROFT_C16F: "f16", croft.CROFT_C16B: "bf16"}


def run_half(data_u16: np.ndarray, exp_in: np.ndarray, dtype, direction=croft.CROFT_FORWARD,
             inplace=False, slabs=1, in_exp_null=False):
    """Half-storage transform.  data_u16: (nz, ny, nx, 2) bit patterns; exp_in:
    (nz, ny) int8.  Returns (out bits (nz, ny, nx, 2) uint16, out_exp (ny, nx))."""
    nz, ny, nx, _ = data_u16.shape
    d_in = torch.from_numpy(np.ascontiguousarray(data_u16.view(np.int16))).cuda().view(HALF_TORCH[dtype])
    d_out = d_in if inplace else torch.full_like(d_in, float("nan"))
    e_in = None if in_exp_null else torch.from_numpy(np.ascontiguousarray(exp_in)).cuda()
    e_out = torch.full((ny, nx), 99, dtype=torch.int8, device="cuda")
    plan = croft.croft_plan_create_ex(nx, ny, nz, dtype, direction, 0, slabs)
    try:
        croft.croft_execute_scaled(plan, d_in, e_in, d_out, e_out)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    out = d_out.view(torch.int16).cpu().numpy().view(np.uint16)
    return out, e_out.cpu().numpy()
