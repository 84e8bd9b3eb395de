"""Bit-exact check of the half-storage rounding on the GPU.

On grids whose axis lengths are 1 and 2, each output of a pass is one FP32
addition or subtraction of two decoded inputs (the radix-2 butterfly; the
inverse is the same with real and imaginary parts swapped on the way in and
out), so the stored output is fixed completely by IEEE binary32 arithmetic
and the documented storage rule: after each pass every line is scaled by
2^-e, with e chosen so that its largest |re| or |im| lies in [2^14, 2^15),
and rounded to nearest, ties to even.  The test replays exactly that in
numpy float32 (numpy's own round-to-nearest-even conversions) and compares
every stored bit and every exponent.
"""
import numpy as np
import pytest

import paper_2002_04896_amd as croft
from paper_2002_04896_amd import synth
from gpu_helpers import HALF_KIND, run_half

pytestmark = pytest.mark.gpu

F16, BF16 = croft.CROFT_C16F, croft.CROFT_C16B
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD


def to_bits(v32, kind):
    """float32 values -> 16-bit patterns, rounded to nearest even."""
    if kind == "f16":
        return v32.astype(np.float16).view(np.uint16)
    u = v32.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def from_bits(bits, kind):
    if kind == "f16":
        return bits.view(np.float16).astype(np.float32)
    return (bits.astype(np.uint32) << 16).view(np.float32)


def decode(bits, e, axis, kind):
    scale = np.ldexp(np.float32(1), np.expand_dims(e.astype(np.int32), axis)).astype(np.float32)
    return from_bits(bits[..., 0], kind) * scale, from_bits(bits[..., 1], kind) * scale


def encode(re, im, axis, kind):
    m = np.maximum(np.abs(re), np.abs(im)).max(axis=axis)
    e = np.where(m > 0, np.frexp(m)[1] - 15, 0).astype(np.int32)
    scale = np.ldexp(np.float32(1), -np.expand_dims(e, axis)).astype(np.float32)
    return np.stack([to_bits(re * scale, kind), to_bits(im * scale, kind)], axis=-1), e.astype(np.int8)


def butterfly(re, im, axis, inverse):
    """Length-2 DFT along `axis` (a length-1 axis is left alone), in float32."""
    if re.shape[axis] == 1:
        return re, im
    if inverse:
        re, im = im, re
    a_re, b_re = np.take(re, 0, axis), np.take(re, 1, axis)
    a_im, b_im = np.take(im, 0, axis), np.take(im, 1, axis)
    re = np.stack([a_re + b_re, a_re - b_re], axis=axis)
    im = np.stack([a_im + b_im, a_im - b_im], axis=axis)
    if inverse:
        re, im = im, re
    return re, im


@pytest.mark.parametrize("direction", [FWD, BWD], ids=["fwd", "bwd"])
@pytest.mark.parametrize("dtype", [F16, BF16], ids=["f16", "bf16"])
@pytest.mark.parametrize("nzyx", [(2, 2, 2), (1, 2, 2), (2, 1, 2), (2, 2, 1)], ids=str)
def test_stored_bits_follow_the_rounding_rule(nzyx, dtype, direction):
    kind = HALF_KIND[dtype]
    for seed in range(8):
        data, e_in = synth.quantize_half(synth.normal_c(nzyx, seed=60 + seed), kind)
        out, oe = run_half(data, e_in, dtype, direction)
        # replay: x pass (numpy axis 2, exponents per x-line), then y (axis 1), then z (axis 0)
        bits, e = data.view(np.uint16), e_in
        prev_axis = 2
        for axis in (2, 1, 0):
            re, im = decode(bits, e, prev_axis, kind)
            re, im = butterfly(re, im, axis, direction == BWD)
            bits, e = encode(re, im, axis, kind)
            prev_axis = axis
        np.testing.assert_array_equal(oe, e, err_msg=f"seed {seed}")
        np.testing.assert_array_equal(out, bits, err_msg=f"seed {seed}")
