"""The C ABI without a GPU: symbols, argument validation, dry-run plans."""
import ctypes
import os
import re

import pytest

import paper_2002_04896_amd as croft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "croft.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(croft_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(croft.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), f"{name} declared in croft.h but not exported"
    assert sorted(croft.EXPORTED) == names


def test_binding_constants_match_the_header():
    """Every enumerator and integer #define of croft.h has the same value in
    the Python binding."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    consts = {}
    for body in re.findall(r"enum\s+\w+\s*\{(.*?)\}", text, flags=re.S):
        for name, val in re.findall(r"(CROFT_\w+)\s*=\s*(\d+)", body):
            consts[name] = int(val)
    for m in re.finditer(r"#define\s+(CROFT_\w+)\s+\(?(\d+)u?(?:\s*<<\s*(\d+))?\)?\s*$", text, flags=re.M):
        consts[m.group(1)] = int(m.group(2)) << int(m.group(3) or 0)
    assert {"CROFT_GRAPH", "CROFT_PERSISTENT", "CROFT_UNFUSED", "CROFT_C16B", "CROFT_MAX_PASSES",
            "CROFT_NOALLOC_SCRATCH_BYTES"} <= set(consts)
    for name, val in consts.items():
        assert getattr(croft, name) == val, name
    flags = [consts[k] for k in ("CROFT_MEASURE", "CROFT_FORCE_GENERIC", "CROFT_NO_WISDOM",
                                 "CROFT_PERSISTENT", "CROFT_UNFUSED", "CROFT_GRAPH")]
    assert all(f & (f - 1) == 0 for f in flags) and len(set(flags)) == len(flags)


def test_graph_flag_is_for_batched_plans_only():
    with pytest.raises(ValueError, match="flags"):
        croft.croft_plan_create_ex(8, 8, 8, croft.CROFT_C64, -1, croft.CROFT_GRAPH, 1)
    with pytest.raises(ValueError, match="flags"):
        croft.croft_plan_create_real(8, 8, 8, croft.CROFT_C64, -1, croft.CROFT_GRAPH)


@pytest.mark.parametrize("dims,msg", [
    ((0, 4, 4), "< 1"), ((4, -2, 4), "< 1"), ((4097, 4, 4), "unsupported"),
    ((4, 4, 4097), "unsupported"), ((4, 4, 8192), "unsupported"), ((4, 5000, 4), "unsupported"),
])
def test_create_rejects_bad_sizes(dims, msg):
    with pytest.raises(ValueError, match=msg):
        croft.croft_plan_create(*dims)


# one prime for every convolution length the Bluestein kernel is compiled
# for (16 .. 8192), and 13, 14 (a prime factor times a power of two)
@pytest.mark.parametrize("n", [7, 11, 13, 14, 17, 41, 97, 131, 509, 1009, 2039, 4093])
def test_lengths_with_large_prime_factors_use_bluestein(n):
    _, passes = parse_describe(croft.croft_plan_describe(n, 6, 5))
    p = passes[0]
    m = int(p["bluestein"])
    assert p["kernel"] == "bluestein" and m >= 2 * n - 1 and m & (m - 1) == 0 and m < 4 * n
    assert int(p["lds"]) <= 160 * 1024 and int(p["block"]) <= 256
    # every geometry and dtype has a compiled kernel for m, and its launch fits
    for dt in (croft.CROFT_C64, croft.CROFT_C128, croft.CROFT_C16F, croft.CROFT_C16B):
        if dt == croft.CROFT_C128 and m > 4096:
            continue
        _, contiguous = parse_describe(croft.croft_plan_describe(n, 3, 2, dt))
        _, strided = parse_describe(croft.croft_plan_describe(2, n, 3, dt))
        for q in (contiguous[0], strided[1]):
            assert q["kernel"] == "bluestein" and int(q["bluestein"]) == m, (dt, q)
            T, L = int(q["T"]), int(q["L"])
            assert T * L <= int(q["block"]) <= 256 and int(q["lds"]) <= 160 * 1024, (dt, q)


def test_bluestein_complex128_limit():
    _, passes = parse_describe(croft.croft_plan_describe(2039, 2, 1, croft.CROFT_C128))
    assert passes[0]["kernel"] == "bluestein" and passes[0]["bluestein"] == "4096"
    with pytest.raises(ValueError, match="Bluestein"):
        croft.croft_plan_describe(2053, 2, 1, croft.CROFT_C128)


def test_create_rejects_bad_dtype_and_direction():
    with pytest.raises(ValueError, match="dtype"):
        croft.croft_plan_create(8, 8, 8, 7, croft.CROFT_FORWARD)
    with pytest.raises(ValueError, match="direction"):
        croft.croft_plan_create(8, 8, 8, croft.CROFT_C64, 0)
    with pytest.raises(ValueError, match="flags"):
        croft.croft_plan_create_ex(8, 8, 8, croft.CROFT_C64, -1, 64, 1)
    with pytest.raises(ValueError, match="slab"):
        croft.croft_plan_create_ex(8, 8, 12, croft.CROFT_C64, -1, 0, 5)
    with pytest.raises(ValueError, match="2\\^31"):
        croft.croft_plan_create(4096, 4096, 256)


def test_batched_create_rejects_bad_grids():
    with pytest.raises(ValueError, match="grid 1"):
        croft.croft_plan_create_batched([(8, 8, 8), (8, 4097, 8)])
    with pytest.raises(ValueError, match="C64 or"):
        croft.croft_plan_create_batched([(8, 8, 8)], croft.CROFT_C16F)
    with pytest.raises(ValueError, match="count"):
        croft.croft_plan_create_batched([])


def test_null_plan_calls():
    lib = croft.load()
    assert lib.croft_execute(None, None, None, None) == croft.CROFT_ERR_INVALID_VALUE
    assert "NULL plan" in croft.croft_last_error()
    assert lib.croft_execute_scaled(None, None, None, None, None, None) == croft.CROFT_ERR_INVALID_VALUE
    assert lib.croft_execute_batched(None, None, None, None) == croft.CROFT_ERR_INVALID_VALUE
    assert lib.croft_plan_destroy(None) == croft.CROFT_SUCCESS
    assert lib.croft_plan_info(None, None) == croft.CROFT_ERR_INVALID_VALUE
    assert lib.croft_plan_profile(None, 1) == croft.CROFT_ERR_INVALID_VALUE


def parse_describe(text):
    lines = text.strip().split("\n")
    head = lines[0]
    passes = []
    for ln in lines[1:]:
        if not ln.startswith("pass "):
            continue
        kv = dict(tok.split("=", 1) for tok in ln.split()[2:])
        passes.append(kv)
    return head, passes


def describe_extra(text, key):
    """The value of a `key=value` line of a dry-run description."""
    for ln in text.strip().split("\n"):
        if ln.startswith(key + "="):
            return ln.split("=", 1)[1]
    raise KeyError(key)


def test_describe_512_cube():
    head, passes = parse_describe(croft.croft_plan_describe(512, 512, 512))
    assert "elements=134217728" in head and "bytes=1073741824" in head
    assert "algorithmic_bytes=6442450944" in head
    assert [p["axis"] for p in passes] == ["x", "y", "z"]
    assert [p["kind"] for p in passes] == ["contiguous", "strided", "strided"]
    assert [p["stride"] for p in passes] == ["1", "512", "262144"]
    for p in passes:
        assert p["kernel"] == "static" and p["radices"] == "8x8x8"
        assert int(p["lines"]) == 512 * 512


@pytest.mark.parametrize("n,rad", [(384, "3x8x16"), (48, "3x16"), (60, "5x3x4"), (72, "3x3x8"),
                                   (80, "5x16"), (96, "3x8x4"), (100, "5x5x4"), (128, "8x16"),
                                   (1024, "8x8x16"), (32, "8x4"), (2, "2"), (4096, "8x8x8x8"),
                                   (120, "5x3x8"), (160, "5x8x4"), (192, "3x8x8"), (240, "5x3x16"),
                                   (320, "5x8x8"), (480, "5x3x8x4"), (200, None), (288, None), (360, None),
                                   (400, None), (576, None), (640, None), (720, None), (768, None), (960, None)])
def test_describe_factorisations(n, rad):
    _, passes = parse_describe(croft.croft_plan_describe(n, 2, 3))
    assert passes[0]["kernel"] == "static"
    if rad is not None:
        assert passes[0]["radices"] == rad
    prod = 1
    for r in passes[0]["radices"].split("x"):
        prod *= int(r)
    assert prod == n


def test_describe_generic_fallback_and_skipped_axes():
    _, passes = parse_describe(croft.croft_plan_describe(45, 1, 27))
    assert [p["axis"] for p in passes] == ["x", "z"]          # length-1 axis skipped
    assert passes[0]["kernel"] == "generic" and passes[0]["radices"] == "5x3x3"
    assert passes[1]["kind"] == "strided" and passes[1]["stride"] == "45"
    _, passes = parse_describe(croft.croft_plan_describe(1, 1, 1))
    assert len(passes) == 1 and passes[0]["radices"] == "copy"
    _, passes = parse_describe(croft.croft_plan_describe(1, 30, 8))
    assert passes[0]["axis"] == "y" and passes[0]["kind"] == "contiguous"


@pytest.mark.parametrize("args", [(1, 1, 1), (1, 1, 1, croft.CROFT_C16F), (1, 16, 1, croft.CROFT_C16B),
                                  (480, 2, 3), (2, 480, 3, croft.CROFT_C128), (45, 1, 27), (2, 3, 2000),
                                  (4000, 2, 1, croft.CROFT_C128), (6, 2, 5)])
def test_runtime_radix_twiddles_in_lds_only_where_stages_read_them(args):
    """The runtime-radix kernel copies the length-n twiddle table into LDS
    only for plans of two or more stages (the first stage reads no twiddle,
    and a length-1 pass has no table to copy), and only where it fits beside
    the line buffers; its LDS is two line buffers plus one line maximum each."""
    dt = args[3] if len(args) > 3 else croft.CROFT_C64
    cb = 16 if dt == croft.CROFT_C128 else 8
    _, passes = parse_describe(croft.croft_plan_describe(*args))
    seen = 0
    for p in passes:
        if p["kernel"] != "generic" or p["bluestein"] != "0":
            continue
        seen += 1
        n, L = int(p["n"]), int(p["L"])
        lines = L * (2 * n * cb + 4)
        stages = 0 if p["radices"] == "copy" else len(p["radices"].split("x"))
        table = n * cb if stages >= 2 and n * cb + lines <= 160 * 1024 else 0
        assert int(p["lds"]) == table + lines, (args, p)
    assert seen


def test_describe_half_runs_every_axis():
    _, passes = parse_describe(croft.croft_plan_describe(1, 16, 1, croft.CROFT_C16F))
    assert [p["axis"] for p in passes] == ["x", "y", "z"]
    assert [p["n"] for p in passes] == ["1", "16", "1"]


def test_describe_launch_shapes_fit_the_device():
    for n in [2, 3, 5, 8, 16, 45, 48, 60, 100, 384, 512, 1000, 1024, 3000, 4096]:
        for dt in range(4):
            _, passes = parse_describe(croft.croft_plan_describe(n, 8, 16, dt))
            for p in passes:
                assert int(p["block"]) <= 1024 and int(p["block"]) % 1 == 0
                assert int(p["lds"]) <= 160 * 1024
                assert int(p["T"]) * int(p["L"]) <= int(p["block"])


def _describe_with_wisdom(tmp_path, monkeypatch, text, *args):
    w = tmp_path / "wisdom.txt"
    w.write_text(text)
    monkeypatch.setenv("CROFT_WISDOM", str(w))
    return parse_describe(croft.croft_plan_describe(*args))[1]


def test_builtin_wisdom_picks_one_line_per_lane_at_512(tmp_path, monkeypatch):
    # complex64 strided passes of length 512, both directions: one line per
    # lane (8 threads per line) in 32-line tiles (256-byte rows, 256-thread
    # blocks) on both axes, the y pass one block per tile with non-temporal
    # loads and the tiles in reverse order, the z pass with non-temporal
    # loads and stores, one block per tile, the tile's first half copied
    # into LDS
    for direction in (croft.CROFT_FORWARD, croft.CROFT_BACKWARD):
        passes = _describe_with_wisdom(tmp_path, monkeypatch, "", 512, 512, 512, croft.CROFT_C64, direction)
        assert [p["candidate"] for p in passes][1:] == ["15", "18"]
        for p in passes[1:]:
            assert (p["T"], p["L"], p["block"]) == ("8", "32", "256")
        assert [p["waves"] for p in passes][1:] == ["0", "0"]
    # a wisdom line for any axis comes before the built-in per-axis choices
    passes = _describe_with_wisdom(tmp_path, monkeypatch, "512 1 0 2 1\n", 512, 512, 512)
    assert [p["candidate"] for p in passes][1:] == ["2", "2"]
    assert passes[1]["L"] == "32" and passes[1]["T"] == "32"


def test_wisdom_file_overrides_choice(tmp_path, monkeypatch):
    passes = _describe_with_wisdom(tmp_path, monkeypatch, "512 1 0 0 1\n512 0 0 2 3\n", 512, 512, 512)
    assert passes[0]["candidate"] == "2" and passes[0]["waves"] == "3"
    assert passes[1]["candidate"] == "0" and passes[1]["L"] == "16" and passes[1]["waves"] == "1"
    # the last matching line wins
    passes = _describe_with_wisdom(tmp_path, monkeypatch, "512 1 0 0 1\n512 1 0 4 2\n", 512, 512, 512)
    assert passes[2]["candidate"] == "4" and passes[2]["block"] == "512"


def test_non_temporal_candidates_give_way_on_partial_lines(tmp_path, monkeypatch):
    # a real grid's half-spectrum y pass has 257 complex64 per row, not whole
    # 128-byte lines: the complex grid's y choice (candidate 15, non-temporal
    # loads) gives way to its plain twin (10); the z rows (257 * 512
    # elements) are whole lines and whole 32-line tiles and keep candidate 18
    monkeypatch.setenv("CROFT_WISDOM", str(tmp_path / "none.txt"))
    passes = parse_describe(croft.croft_plan_describe_real(512, 512, 512))[1]
    assert [p["candidate"] for p in passes][1:] == ["10", "18"]
    # the same twin for any non-temporal candidate named in a wisdom file
    for cand, plain in ((7, 6), (9, 8), (11, 10), (12, 8), (13, 8), (14, 10), (15, 10)):
        w = tmp_path / "w.txt"
        w.write_text(f"512 1 0 {cand} 0 1\n")
        monkeypatch.setenv("CROFT_WISDOM", str(w))
        passes = parse_describe(croft.croft_plan_describe_real(512, 512, 512))[1]
        assert passes[1]["candidate"] == str(plain)
        passes = parse_describe(croft.croft_plan_describe(512, 512, 512))[1]
        assert passes[1]["candidate"] == str(cand)


def test_wisdom_per_axis_choices(tmp_path, monkeypatch):
    # complex64 at 512: the built-in choices differ between the y pass (one
    # line per lane, XCD-contiguous tile order) and the z pass (dispatch
    # order)
    passes = _describe_with_wisdom(tmp_path, monkeypatch, "", 512, 512, 512, croft.CROFT_C64)
    assert [p["candidate"] for p in passes][1:] == ["15", "18"]
    # a file line for any axis comes before the built-in per-axis choices ...
    passes = _describe_with_wisdom(tmp_path, monkeypatch, "512 1 0 4 1\n", 512, 512, 512, croft.CROFT_C64)
    assert [p["candidate"] for p in passes][1:] == ["4", "4"]
    # ... and a line for the pass's own axis before one for any axis
    passes = _describe_with_wisdom(tmp_path, monkeypatch, "512 1 0 4 1\n512 1 0 2 2 2\n", 512, 512, 512,
                                   croft.CROFT_C64)
    assert [p["candidate"] for p in passes][1:] == ["4", "2"] and passes[2]["waves"] == "2"


def test_builtin_half_storage_one_line_per_lane_at_512(tmp_path, monkeypatch):
    # 16-bit storage at 512: x the non-temporal contiguous tile on a
    # persistent grid of four waves; one line per lane on both strided axes,
    # y in 32-line tiles (256-thread blocks, XCD-contiguous order,
    # non-temporal loads), z in 64-line tiles (the next tile loaded into
    # registers; FP16 with the non-temporal hint on those loads)
    for dt, z in ((croft.CROFT_C16F, "23"), (croft.CROFT_C16B, "20")):
        passes = _describe_with_wisdom(tmp_path, monkeypatch, "", 512, 512, 512, dt)
        assert [p["candidate"] for p in passes] == ["3", "14", z]
        assert passes[0]["waves"] == "4"
        assert (passes[1]["T"], passes[1]["L"], passes[1]["block"]) == ("8", "32", "256")
        assert (passes[2]["T"], passes[2]["L"], passes[2]["block"]) == ("8", "64", "512")


def test_builtin_complex128_choices_at_512(tmp_path, monkeypatch):
    # complex128 at 512, both directions: x the non-temporal contiguous tile,
    # y and z the wide tile with fewer threads (16-line tiles, 512-thread
    # blocks), y one block per tile, z on two waves of resident blocks (the
    # XCD-ordered y tile is the faster y pass alone but slows the z pass)
    for direction in (croft.CROFT_FORWARD, croft.CROFT_BACKWARD):
        passes = _describe_with_wisdom(tmp_path, monkeypatch, "", 512, 512, 512, croft.CROFT_C128, direction)
        assert [p["candidate"] for p in passes] == ["3", "4", "4"]
        assert [p["waves"] for p in passes] == ["0", "0", "2"]
        for p in passes[1:]:
            assert (p["L"], p["block"]) == ("16", "512")


def test_builtin_one_line_per_lane_at_1024(tmp_path, monkeypatch):
    # complex64 strided passes of length 1024: 16 threads per line, 32-line
    # tiles (256-byte rows) in 512-thread blocks, one block per tile, both
    # directions; y in the XCD-contiguous order, z non-temporal
    for direction in (croft.CROFT_FORWARD, croft.CROFT_BACKWARD):
        passes = _describe_with_wisdom(tmp_path, monkeypatch, "", 1024, 1024, 1024, croft.CROFT_C64, direction)
        assert [p["candidate"] for p in passes][1:] == ["8", "7"]
        for p in passes[1:]:
            assert (p["T"], p["L"], p["block"], p["waves"]) == ("16", "32", "512", "0")
            assert int(p["lds"]) <= 160 * 1024


def test_wisdom_unknown_candidate_falls_back_to_default(tmp_path, monkeypatch):
    passes = _describe_with_wisdom(tmp_path, monkeypatch, "512 1 0 99 1\n", 512, 512, 512)
    assert passes[1]["candidate"] == "0"


def test_wisdom_does_not_affect_generic_lengths(tmp_path, monkeypatch):
    passes = _describe_with_wisdom(tmp_path, monkeypatch, "45 0 0 2 2\n", 45, 8, 8)
    assert passes[0]["kernel"] == "generic"


def test_every_candidate_fits_the_device(tmp_path, monkeypatch):
    for n in (128, 256, 512, 1024):
        for dt in range(4):
            for kind in (0, 1):
                for cand in range(5):
                    passes = _describe_with_wisdom(tmp_path, monkeypatch, f"{n} {kind} {dt} {cand} 1\n",
                                                   n, n if kind else 2, 4, dt)
                    for p in passes:
                        assert int(p["block"]) <= 1024 and int(p["lds"]) <= 160 * 1024


# ------------------------------------------------------------ real plans
def test_describe_real_512_cube_forward_and_backward():
    head, passes = parse_describe(croft.croft_plan_describe_real(512, 512, 512))
    spec = 257 * 512 * 512
    assert "real forward" in head and f"bytes={spec * 8}" in head
    # x pass: real grid (4 B per value) + half spectrum; y, z: twice the half spectrum
    assert f"algorithmic_bytes={512 ** 3 * 4 + spec * 8 + 4 * spec * 8}" in head
    assert [p["axis"] for p in passes] == ["x", "y", "z"]
    assert [p["kind"] for p in passes] == ["real", "strided", "strided"]
    assert [p["n"] for p in passes] == ["256", "512", "512"]
    assert [p["stride"] for p in passes] == ["1", "257", str(257 * 512)]
    assert passes[0]["lines"] == str(512 * 512)
    assert passes[0]["kernel"] == "static"
    _, back = parse_describe(croft.croft_plan_describe_real(512, 512, 512, croft.CROFT_C64, croft.CROFT_BACKWARD))
    assert [p["axis"] for p in back] == ["z", "y", "x"]
    assert [p["kind"] for p in back] == ["strided", "strided", "real"]


@pytest.mark.parametrize("dims,skipped", [((64, 1, 8), "y"), ((64, 8, 1), "z"), ((16, 1, 1), "yz")])
def test_describe_real_skips_unit_axes(dims, skipped):
    _, passes = parse_describe(croft.croft_plan_describe_real(*dims))
    axes = [p["axis"] for p in passes]
    assert axes[0] == "x" and not any(a in axes for a in skipped)


@pytest.mark.parametrize("nx", [4, 8, 96, 120, 144, 160, 192, 200, 768, 1024, 8192])
@pytest.mark.parametrize("dt", [croft.CROFT_C64, croft.CROFT_C128])
def test_describe_real_supported_lengths_fit_the_device(nx, dt):
    _, passes = parse_describe(croft.croft_plan_describe_real(nx, 6, 5, dt))
    assert passes[0]["kind"] == "real" and int(passes[0]["n"]) == nx // 2
    for p in passes:
        assert int(p["block"]) <= 1024 and int(p["lds"]) <= 160 * 1024


@pytest.mark.parametrize("dims,dt,msg", [
    ((7, 4, 4), croft.CROFT_C64, "even nx"), ((2, 4, 4), croft.CROFT_C64, "even nx"),
    ((8194, 4, 4), croft.CROFT_C64, "even nx"), ((162, 4, 4), croft.CROFT_C64, "no real x kernel"),
    ((16, 4097, 4), croft.CROFT_C64, "unsupported"), ((16, 4, 4), croft.CROFT_C16F, "CROFT_C64 or CROFT_C128"),
])
def test_real_plans_reject_bad_arguments(dims, dt, msg):
    with pytest.raises(ValueError, match=msg):
        croft.croft_plan_describe_real(*dims, dt)
    with pytest.raises(ValueError, match=msg):
        croft.croft_plan_create_real(*dims, dt)


# ------------------------------------------------------ convolution plans
def test_describe_convolution_512_cube():
    head, passes = parse_describe(croft.croft_plan_describe_convolution(512, 512, 512))
    spec = 257 * 512 * 512
    assert "convolution" in head
    # x fwd (real + spectrum), y fwd, fused z (2 + multiplier), y bwd, x bwd
    assert f"algorithmic_bytes={2 * (512 ** 3 * 4 + spec * 8) + 4 * spec * 8 + 2.5 * spec * 8:.0f}" in head
    assert [p["axis"] for p in passes] == ["x", "y", "z", "y", "x"]
    assert [p["kind"] for p in passes] == ["real", "strided", "fused", "strided", "real"]
    assert passes[2]["stride"] == str(257 * 512) and passes[2]["kernel"] == "static"


def test_describe_convolution_fuses_y_when_nz_is_one():
    _, passes = parse_describe(croft.croft_plan_describe_convolution(64, 48, 1))
    assert [p["axis"] for p in passes] == ["x", "y", "x"]
    assert passes[1]["kind"] == "fused" and passes[1]["stride"] == "33"


@pytest.mark.parametrize("dims,dt,msg", [
    ((16, 1, 1), croft.CROFT_C64, "ny > 1 or nz > 1"), ((16, 4, 7), croft.CROFT_C64, "no fused"),
    ((15, 4, 4), croft.CROFT_C64, "even nx"), ((16, 4, 4), croft.CROFT_C16B, "CROFT_C64 or CROFT_C128"),
])
def test_convolution_plans_reject_bad_arguments(dims, dt, msg):
    with pytest.raises(ValueError, match=msg):
        croft.croft_plan_describe_convolution(*dims, dt)
    with pytest.raises(ValueError, match=msg):
        croft.croft_plan_create_convolution(*dims, dt)


def test_static_kernels_are_only_used_where_lane_offsets_fit_32_bits():
    # 4096 x 4096 x 100 complex128: a z-line tile spans (T-1) * 2^24 elements
    # of 16 B beyond 4 GiB, so the z pass must take the 64-bit runtime-radix kernel
    _, passes = parse_describe(croft.croft_plan_describe(4096, 4096, 100, croft.CROFT_C128))
    assert passes[2]["kernel"] == "generic"
    for p in passes:
        T, L, es = int(p["T"]), int(p["L"]), int(p["stride"])
        span = (L - 1) + (T - 1) * es if p["kind"] == "strided" else (L - 1) * int(p["n"]) + T - 1
        assert p["kernel"] == "generic" or (span + 1) * 16 <= 0xFFFFFFFF
    _, passes = parse_describe(croft.croft_plan_describe(4096, 4096, 100, croft.CROFT_C64))
    assert passes[2]["kernel"] == "static"


def test_describe_convolution_uncompiled_fused_length_runs_the_runtime_kernel():
    _, passes = parse_describe(croft.croft_plan_describe_convolution(32, 20, 24))
    assert passes[2]["kind"] == "fused" and passes[2]["kernel"] == "generic"
    _, passes = parse_describe(croft.croft_plan_describe_convolution(32, 20, 64))
    assert passes[2]["kind"] == "fused" and passes[2]["kernel"] == "static"


@pytest.mark.parametrize("dims,dt,n", [((512, 512, 256), croft.CROFT_C64, 256),
                                       ((512, 64, 512), croft.CROFT_C64, 512),
                                       ((64, 64, 128), croft.CROFT_C128, 128)])
def test_energy_partials_cover_every_fused_candidate(dims, dt, n, tmp_path, monkeypatch):
    """The convolution plan holds one energy partial per block of its fused
    pass; the autotuner launches every compiled candidate of the fused length
    (they differ in lines per tile, so in block count), and the wisdom may
    start the plan on any of them.  Whatever candidate the plan starts on,
    the partials it sizes must cover the largest block count among them."""
    w = tmp_path / "w.txt"
    monkeypatch.setenv("CROFT_WISDOM", str(w))
    counts, blocks = set(), []
    for cand in range(4):
        for waves in (0, 1, 2):
            w.write_text(f"{n} 3 {dt} {cand} {waves}\n")
            text = croft.croft_plan_describe_convolution(*dims, dt)
            fused = [p for p in parse_describe(text)[1] if p["kind"] == "fused"]
            assert len(fused) == 1
            blocks.append(int(fused[0]["blocks"]))
            counts.add(int(describe_extra(text, "energy_partials")))
    assert len(counts) == 1, counts                       # independent of the starting candidate
    assert len(set(blocks)) > 1                            # the candidates do differ in block count
    assert counts.pop() >= max(blocks)


def test_unfused_schedule_rejects_half_storage_and_slabs():
    with pytest.raises(ValueError, match="CROFT_UNFUSED"):
        croft.croft_plan_create_ex(8, 8, 8, croft.CROFT_C16F, croft.CROFT_FORWARD, croft.CROFT_UNFUSED, 1)
    with pytest.raises(ValueError, match="CROFT_UNFUSED"):
        croft.croft_plan_create_ex(8, 8, 8, croft.CROFT_C64, croft.CROFT_FORWARD, croft.CROFT_UNFUSED, 4)


def test_half_tile_copy_candidates_need_whole_tiles(tmp_path, monkeypatch):
    # candidates that copy the next tile's first half into LDS run whole
    # tiles only: with es not a multiple of the tile's lines the planner runs
    # their twin (complex64 at 512: 17, 18 -> 8; at 1024: 10-12 -> 6)
    for n, cand, twin, nx in ((512, 17, 8, 40), (512, 18, 8, 48), (1024, 10, 6, 40), (1024, 12, 6, 48)):
        # es = nx * 21: 840 and 1008, not multiples of 32
        passes = _describe_with_wisdom(tmp_path, monkeypatch, f"{n} 1 0 {cand} 1 2\n", nx, 21, n)
        assert passes[2]["candidate"] == str(twin), (n, cand)
        passes = _describe_with_wisdom(tmp_path, monkeypatch, f"{n} 1 0 {cand} 1 2\n", 64, 20, n)
        assert passes[2]["candidate"] == str(cand), (n, cand)
