"""Plant plausible mistakes in copies of the oracle's C source and check that
the pins catch every one of them (a dropped term, a wrong sign, a wrong index,
a transposed operand, a skipped axis, a wrong table).  The mutants are built
and run on the CPU only; the real oracle is untouched."""
import os

import numpy as np
import pytest

import oracle

MUTANTS = {
    "dropped_term": ("acc_re += x[0] * wr - x[1] * wi;", "acc_re += x[0] * wr;"),
    "wrong_sign": ("const double wr = c[m], wi = sign * s[m];",
                   "const double wr = c[m], wi = -sign * s[m];"),
    "wrong_index": ("            m += k;\n", "            m += k + 1;\n"),
    # plane stride taken from the wrong pair of axes (in bounds while nz <= ny)
    "transposed_plane_stride": ("base = (l % nx) + (l / nx) * (long)nx * ny;",
                                "base = (l % nx) + (l / nx) * (long)nx * nz;"),
    "skipped_z_axis": ("data, 2, 0, (long)nx * ny, sign)) return -1;\n    return 0;",
                       "data, 2, 0, 0, sign)) return -1;\n    return 0;"),
    "half_angle_table": ("c[m] = cos(kTwoPi * (double)m / (double)n);",
                         "c[m] = cos(0.5 * kTwoPi * (double)m / (double)n);"),
    "brute_mixed_axes": ("(double)((ky * jy) % ny) / ny", "(double)((ky * jx) % ny) / ny"),
    "lines_wrong_step": ("my += ky[i];", "my += kz[i];"),
    "lines_dropped_conj_sign": ("const double wr = tz[mz], wi = sign * tz[nz + mz];",
                                "const double wr = tz[mz], wi = tz[nz + mz];"),
}


def battery(o: oracle.Oracle) -> list:
    """The pins, condensed: returns the names of the checks that failed."""
    rng = np.random.Generator(np.random.PCG64(7))
    nz, ny, nx = 6, 10, 12
    x = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    failed = []
    ref = np.fft.fftn(x)
    if oracle.rel_l2(o.dft3d(x, -1), ref) > 1e-12:
        failed.append("dft3d_vs_pocketfft")
    if oracle.rel_l2(o.dft3d(x, +1), np.fft.ifftn(x) * x.size) > 1e-12:
        failed.append("backward_vs_pocketfft")
    if oracle.rel_l2(o.dft3d_brute(x, -1), ref) > 1e-12:
        failed.append("brute_vs_pocketfft")
    kyz = [(3, 5), (7, 2)]
    lines = o.dft3d_lines(x, kyz, -1)
    if max(oracle.rel_l2(lines[i], ref[kz, ky]) for i, (ky, kz) in enumerate(kyz)) > 1e-12:
        failed.append("lines_vs_pocketfft")
    return failed


def test_real_oracle_passes_battery():
    assert battery(oracle.Oracle()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    path = os.path.join(tmp_path, f"mut_{name}.c")
    with open(path, "w") as f:
        f.write(mutated)
    lib = oracle.compile_oracle(path, os.path.join(tmp_path, f"libmut_{name}.so"))
    assert battery(oracle.Oracle(oracle.bind(lib))) != []
