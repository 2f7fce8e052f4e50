"""C-ABI checks that need no GPU: the built library exports every function
include/pauli.h declares, and invalid requests fail with the documented status
before any device call (so these run in a container without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pauli.h")

OK, EINVAL, EUNSUPPORTED, EHIP, ENOMEM = 0, 1, 2, 3, 4


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\*?\s+\*?(pauli_[a-z_]+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2401_16378_amd as p
    if not os.path.exists(p.LIB_PATH):
        pytest.fail("libpauli.so is not built (python -m paper_2401_16378_amd.build)")
    return p.load_library()


@pytest.fixture(scope="module")
def pauli():
    import paper_2401_16378_amd as p
    return p


def test_header_declarations_exported(lib, pauli):
    names = declared_functions()
    assert len(names) >= 15, names
    raw = ctypes.CDLL(pauli.LIB_PATH)
    for name in names:
        assert hasattr(raw, name), "libpauli.so does not export %s" % name
    assert sorted(pauli.EXPORTS) == names


def test_version_and_defaults(lib, pauli):
    assert lib.pauli_version() == 1
    o = pauli._Opts()
    lib.pauli_opts_default(ctypes.byref(o))
    assert (o.algo, o.in_dtype, o.out_dtype, o.tile) == (2, 0, 0, 0)
    assert o.stream is None and o.workspace is None and o.workspace_bytes == 0


def opts(pauli, algo="split_bf16", in_dt=0, out_dt=0, tile=0, ws=None, ws_bytes=0):
    o = pauli._opts(algo, in_dt, out_dt, tile, None)
    if ws is not None:
        o.workspace = ws
        o.workspace_bytes = ws_bytes
    return o


FAKE_IN = 0x10000000      # never dereferenced: every call below fails validation first
FAKE_OUT = 0x20000000


@pytest.mark.parametrize("fn", ["pauli_decompose", "pauli_reconstruct", "pauli_decompose_backward",
                                "pauli_decompose_hermitian"])
def test_validation_errors(lib, pauli, fn):
    f = getattr(lib, fn)
    o = opts(pauli)
    cases = [
        (FAKE_IN, -1, 1, FAKE_OUT, o, EINVAL),            # N < 0
        (FAKE_IN, 17, 1, FAKE_OUT, o, EINVAL),            # N > 16
        (FAKE_IN, 4, 0, FAKE_OUT, o, EINVAL),             # batch < 1
        (None, 4, 1, FAKE_OUT, o, EINVAL),                # NULL input
        (FAKE_IN, 4, 1, None, o, EINVAL),                 # NULL output
        (FAKE_IN + 8, 4, 1, FAKE_OUT, o, EINVAL),         # input not 16-byte aligned
        (FAKE_IN, 4, 1, FAKE_OUT + 8, o, EINVAL),         # output not 16-byte aligned
        (FAKE_IN, 4, 1, FAKE_IN + 256, o, EINVAL),        # overlap
        (FAKE_IN, 4, 1, FAKE_OUT, opts(pauli, in_dt=7), EINVAL),
        (FAKE_IN, 4, 1, FAKE_OUT, opts(pauli, tile=99), EINVAL),
        (FAKE_IN, 4, 1, FAKE_OUT, opts(pauli, tile=1), EINVAL),    # 512-row tile at N = 4
        (FAKE_IN, 12, 1, FAKE_OUT, opts(pauli, algo="fp32", tile=1), EINVAL),   # not offered for binary32
        (FAKE_IN, 10, 1, FAKE_OUT, opts(pauli, ws=0x30000008, ws_bytes=1 << 30), EINVAL),  # misaligned ws
        (FAKE_IN, 10, 1, FAKE_OUT, opts(pauli, ws=0x30000000, ws_bytes=1024), ENOMEM),
    ]
    for a, N, b, out, oo, want in cases:
        st = f(a, N, b, out, ctypes.byref(oo))
        assert st == want, (fn, N, b, st, want, pauli.last_error())
        assert pauli.last_error() != ""
    o.algo = 9
    assert f(FAKE_IN, 4, 1, FAKE_OUT, ctypes.byref(o)) == EINVAL


def test_workspace_sizes(lib):
    # split-bf16: 12 bytes per element, fp32: 8, binary64 Gray: none; N < 5 padded to 32 x 32
    assert lib.pauli_workspace_bytes(2, 10, 1) == 12 * 4 ** 10
    assert lib.pauli_workspace_bytes(1, 10, 3) == 3 * 8 * 4 ** 10
    assert lib.pauli_workspace_bytes(0, 10, 1) == 0
    assert lib.pauli_workspace_bytes(2, 3, 1) == 12 * 32 * 32
    assert lib.pauli_workspace_bytes(2, 17, 1) == 0
    assert lib.pauli_workspace_bytes(5, 4, 1) == 0


def test_tiles(lib):
    n = lib.pauli_tile_count(2)
    assert n >= 6 and lib.pauli_tile_count(1) == n and lib.pauli_tile_count(0) == 1
    assert lib.pauli_tile_count(7) == 0
    for algo in (1, 2):
        for N in range(0, 17):
            t = lib.pauli_tile_selected(algo, N)
            assert 1 <= t <= n and lib.pauli_tile_valid(algo, t, N) == 1, (algo, N, t)
    # 512-row tiles need N >= 9; binary32 has no 4 x 32-row register-ring tiles
    assert lib.pauli_tile_valid(2, 1, 9) == 1 and lib.pauli_tile_valid(2, 1, 8) == 0
    for t in (1, 2, 7, 10, 11):
        assert lib.pauli_tile_valid(1, t, 12) == 0
    for t in (3, 4, 5, 6, 8, 9, 12, 13, 14, 15):
        assert lib.pauli_tile_valid(1, t, 12) == 1
    assert lib.pauli_tile_valid(0, 1, 10) == 1 and lib.pauli_tile_valid(0, 2, 10) == 0
    assert lib.pauli_tile_valid(2, 0, 10) == 0 and lib.pauli_tile_valid(2, n + 1, 10) == 0
    assert lib.pauli_batched_tile_count() >= 1
    nb = lib.pauli_batched_tile_count()
    assert nb == 9
    # every shape runs split-fp16; the 512-row fused shape (7) only it
    assert all(lib.pauli_batched_tile_valid(4, t) == 1 for t in range(1, nb + 1))
    assert all(lib.pauli_batched_tile_valid(a, t) == (t != 7) for a in (1, 2) for t in range(1, nb + 1))
    assert lib.pauli_batched_tile_valid(2, nb + 1) == 0 and lib.pauli_batched_tile_valid(1, 0) == 0
    assert lib.pauli_batched_tile_valid(0, 1) == 0 and lib.pauli_batched_tile_valid(3, 1) == 0
    assert lib.pauli_batched_tile_valid(1, 1) == 1 and lib.pauli_batched_tile_valid(0, 1) == 0


def test_batched_validation(lib, pauli):
    vp = ctypes.c_void_p
    G = (vp * 2)(FAKE_IN, FAKE_IN + (1 << 20))
    O = (vp * 2)(FAKE_OUT, FAKE_OUT + (1 << 20))
    Ns = (ctypes.c_int * 2)(3, 5)
    o = opts(pauli)
    assert lib.pauli_decompose_batched(0, G, Ns, O, ctypes.byref(o)) == EINVAL
    assert lib.pauli_decompose_batched(2, None, Ns, O, ctypes.byref(o)) == EINVAL
    bad = (ctypes.c_int * 2)(3, 13)
    assert lib.pauli_decompose_batched(2, G, bad, O, ctypes.byref(o)) == EINVAL
    assert lib.pauli_decompose_batched(2, G, Ns, O, ctypes.byref(opts(pauli, algo="fp64_gray"))) == EUNSUPPORTED
    assert lib.pauli_decompose_batched(2, G, Ns, O, ctypes.byref(opts(pauli, in_dt=1))) == EUNSUPPORTED
    # no workspace
    assert lib.pauli_decompose_batched(2, G, Ns, O, ctypes.byref(o)) == ENOMEM
    need = lib.pauli_batched_workspace_bytes(2, Ns, 2)
    assert need > 12 * (32 * 32 + 32 * 32)
    small = opts(pauli, ws=0x40000000, ws_bytes=need - 1)
    assert lib.pauli_decompose_batched(2, G, Ns, O, ctypes.byref(small)) == ENOMEM
    assert lib.pauli_batched_workspace_bytes(2, bad, 2) == 0
    assert lib.pauli_batched_tile_selected(2, Ns, 2) >= 1
    ws = opts(pauli, algo="fp32", tile=lib.pauli_batched_tile_count() + 1, ws=0x40000000, ws_bytes=need)
    assert lib.pauli_decompose_batched(2, G, Ns, O, ctypes.byref(ws)) == EINVAL


def test_pass_entry_points_validation(lib, pauli):
    o = opts(pauli)
    assert lib.pauli_pack(FAKE_IN, 10, 1, 0, ctypes.byref(o)) == ENOMEM
    assert lib.pauli_contract(10, 1, 0, FAKE_OUT, ctypes.byref(o)) == ENOMEM
    assert lib.pauli_pack(FAKE_IN, 10, 1, 5, ctypes.byref(o)) == EINVAL
    g = opts(pauli, algo="fp64_gray")
    assert lib.pauli_pack(FAKE_IN, 10, 1, 0, ctypes.byref(g)) == EUNSUPPORTED
    ws = opts(pauli, ws=0x30000000, ws_bytes=12 * 4 ** 10)
    assert lib.pauli_pack(None, 10, 1, 0, ctypes.byref(ws)) == EINVAL
    assert lib.pauli_contract(10, 1, 0, 0x30000000 + 4096, ctypes.byref(ws)) == EINVAL   # overlaps workspace
    # mode 3 (Hermitian decomposition) takes the register-ring tiles only
    lds_tile = opts(pauli, tile=13, ws=0x30000000, ws_bytes=12 * 4 ** 10)
    assert lib.pauli_contract(10, 1, 3, FAKE_OUT, ctypes.byref(lds_tile)) == EINVAL
    assert lib.pauli_pack(FAKE_IN, 10, 1, 4, ctypes.byref(ws)) == EINVAL


def test_autotune_validation(lib, pauli):
    o = opts(pauli)
    assert lib.pauli_autotune(5, 3, ctypes.byref(o)) == EINVAL
    assert lib.pauli_autotune(0, 3, ctypes.byref(o)) == EINVAL
    assert lib.pauli_autotune(3, 5, ctypes.byref(opts(pauli, algo="fp64_gray"))) == EUNSUPPORTED


def test_coeffs_at_validation(lib, pauli):
    u32 = ctypes.c_uint
    ns = (u32 * 3)(0, 5, 15)
    o = opts(pauli)
    f = lib.pauli_coeffs_at
    cases = [
        (FAKE_IN, -1, ns, 3, FAKE_OUT, EINVAL),
        (FAKE_IN, 17, ns, 3, FAKE_OUT, EINVAL),
        (FAKE_IN, 2, ns, 0, FAKE_OUT, EINVAL),
        (None, 2, ns, 3, FAKE_OUT, EINVAL),
        (FAKE_IN, 2, None, 3, FAKE_OUT, EINVAL),
        (FAKE_IN, 2, ns, 3, None, EINVAL),
        (FAKE_IN + 8, 2, ns, 3, FAKE_OUT, EINVAL),
        (FAKE_IN, 1, ns, 3, FAKE_OUT, EINVAL),        # 5 and 15 are not below 4^1
        (FAKE_IN, 2, ns, 3, FAKE_IN + 64, EINVAL),    # output inside G
    ]
    for G, N, s, c, out, want in cases:
        assert f(G, N, s, c, out, ctypes.byref(o)) == want, (N, c, pauli.last_error())
        assert pauli.last_error() != ""
    small = opts(pauli, ws=0x30000000, ws_bytes=64)
    assert f(FAKE_IN, 2, ns, 3, FAKE_OUT, ctypes.byref(small)) == ENOMEM
    mis = opts(pauli, ws=0x30000010, ws_bytes=1 << 20)
    assert f(FAKE_IN, 2, ns, 3, FAKE_OUT, ctypes.byref(mis)) == EINVAL
    assert lib.pauli_coeffs_at_workspace_bytes(2, 0) == 0
    assert lib.pauli_coeffs_at_workspace_bytes(17, 5) == 0
    assert lib.pauli_coeffs_at_workspace_bytes(2, 1) == 768          # chunk + entry + one partial
    assert lib.pauli_coeffs_at_workspace_bytes(14, 1) >= 16 * 128     # a single string split 128 ways
    big = lib.pauli_coeffs_at_workspace_bytes(14, 1 << 20)
    assert 24 * (1 << 20) <= big <= 24 * (1 << 20) + 16 * (2048 * 256 + (1 << 20)) + 1024


def test_fwht_algo_queries(lib, pauli):
    assert pauli.ALGOS["fwht"] == 3
    assert lib.pauli_workspace_bytes(3, 14, 1) == 16 * 4 ** 14
    assert lib.pauli_workspace_bytes(3, 14, 2) == 2 * 16 * 4 ** 14
    assert lib.pauli_workspace_bytes(3, 8, 1) == 0                 # one kernel in LDS up to N = 8
    assert lib.pauli_workspace_bytes(3, 16, 1) == 16 * 4 ** 16
    assert lib.pauli_tile_count(3) == 1
    assert all(lib.pauli_tile_valid(3, 1, N) == 1 for N in range(0, 17))
    assert lib.pauli_tile_valid(3, 1, 17) == 0 and lib.pauli_tile_valid(3, 2, 10) == 0
    o = opts(pauli, algo="fwht")
    assert lib.pauli_decompose(FAKE_IN, 17, 1, FAKE_OUT, ctypes.byref(o)) == EINVAL
    small = opts(pauli, algo="fwht", ws=0x30000000, ws_bytes=1024)
    assert lib.pauli_decompose(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(small)) == ENOMEM
    assert lib.pauli_pack(FAKE_IN, 10, 1, 0, ctypes.byref(o)) == EUNSUPPORTED
    assert lib.pauli_autotune(9, 10, ctypes.byref(o)) == EUNSUPPORTED


def test_fwht_f32_algo_queries(lib, pauli):
    """The binary32-intermediate FWHT: half the workspace, the same range,
    tile and refusals as the binary64 one."""
    assert pauli.ALGOS["fwht_f32"] == 5
    assert lib.pauli_workspace_bytes(5, 14, 1) == 8 * 4 ** 14
    assert lib.pauli_workspace_bytes(5, 9, 3) == 3 * 8 * 4 ** 9
    assert lib.pauli_workspace_bytes(5, 8, 1) == 0
    assert lib.pauli_tile_count(5) == 1
    assert all(lib.pauli_tile_valid(5, 1, N) == 1 for N in range(0, 17))
    assert lib.pauli_tile_valid(5, 1, 17) == 0
    o = opts(pauli, algo="fwht_f32")
    assert lib.pauli_decompose(FAKE_IN, 17, 1, FAKE_OUT, ctypes.byref(o)) == EINVAL
    small = opts(pauli, algo="fwht_f32", ws=0x30000000, ws_bytes=8 * 4 ** 10 - 1)
    assert lib.pauli_decompose(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(small)) == ENOMEM
    assert lib.pauli_pack(FAKE_IN, 10, 1, 0, ctypes.byref(o)) == EUNSUPPORTED
    assert lib.pauli_autotune(9, 10, ctypes.byref(o)) == EUNSUPPORTED
    assert lib.pauli_decompose_hermitian(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(o)) == EUNSUPPORTED
    assert lib.pauli_workspace_bytes(7, 10, 1) == 0            # no algo 7


def test_split_i8_algo_queries(lib, pauli):
    """The fixed-point int8 path: six one-byte planes of workspace plus its
    scale record and partial maxima, one tile shape; every single-matrix entry
    point takes it (a short workspace fails before any device call), the
    batched and tuning ones refuse it."""
    assert pauli.ALGOS["split_i8"] == 6
    for N, batch in ((14, 1), (10, 3), (3, 2)):
        Dp = max(1 << N, 32)
        need = lib.pauli_workspace_bytes(6, N, batch)
        packed = (Dp * Dp * 6 * batch + 255) // 256 * 256
        assert packed < need <= packed + 256 + 32 * batch + 8 * 1024 * batch
    assert lib.pauli_tile_count(6) == 1
    assert all(lib.pauli_tile_valid(6, 1, N) == 1 for N in range(0, 17))
    assert lib.pauli_tile_valid(6, 2, 10) == 0 and lib.pauli_tile_valid(6, 1, 17) == 0
    assert lib.pauli_tile_selected(6, 14) == 0
    assert lib.pauli_tile_valid_hermitian(6, 1, 10) == 1 and lib.pauli_tile_valid_hermitian(6, 2, 10) == 0
    o = opts(pauli, algo="split_i8")
    assert lib.pauli_decompose(FAKE_IN, 17, 1, FAKE_OUT, ctypes.byref(o)) == EINVAL
    forced = opts(pauli, algo="split_i8", tile=2)
    assert lib.pauli_decompose(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(forced)) == EINVAL
    small = opts(pauli, algo="split_i8", ws=0x30000000, ws_bytes=6 * 4 ** 10)
    assert lib.pauli_decompose(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(small)) == ENOMEM
    assert lib.pauli_reconstruct(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(small)) == ENOMEM
    assert lib.pauli_decompose_backward(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(small)) == ENOMEM
    assert lib.pauli_decompose_hermitian(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(forced)) == EINVAL
    for mode in (0, 1, 2, 3):   # every mode; the workspace is required
        assert lib.pauli_pack(FAKE_IN, 10, 1, mode, ctypes.byref(o)) == ENOMEM
        assert lib.pauli_contract(10, 1, mode, FAKE_OUT, ctypes.byref(small)) == ENOMEM
    assert lib.pauli_autotune(9, 10, ctypes.byref(o)) == EUNSUPPORTED
    assert lib.pauli_batched_workspace_bytes(1, (ctypes.c_int * 1)(5), 6) == 0


def test_hermitian_queries_and_validation(lib, pauli):
    """The Hermitian variant runs on the matrix-core algorithms' register-ring
    tiles only; the other algorithms and the LDS-staged tiles are refused
    before any device call."""
    f = lib.pauli_decompose_hermitian
    for algo in ("fp64_gray", "fwht"):
        assert f(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(opts(pauli, algo=algo))) == EUNSUPPORTED
    for t in range(1, 13):
        assert lib.pauli_tile_valid_hermitian(2, t, 10) == lib.pauli_tile_valid(2, t, 10) == 1
    for t in (13, 14, 15):
        assert lib.pauli_tile_valid(2, t, 10) == 1 and lib.pauli_tile_valid_hermitian(2, t, 10) == 0
        assert f(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(opts(pauli, tile=t))) == EINVAL
        assert f(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(opts(pauli, algo="fp32", tile=t))) == EINVAL
    for t in (1, 2, 7, 10, 11):
        assert lib.pauli_tile_valid_hermitian(1, t, 12) == 0
    for t in (3, 4, 5, 6, 8, 9, 12):
        assert lib.pauli_tile_valid_hermitian(1, t, 12) == 1
    assert lib.pauli_tile_valid_hermitian(0, 1, 10) == 0 and lib.pauli_tile_valid_hermitian(3, 1, 10) == 0
    assert lib.pauli_tile_valid_hermitian(2, 1, 8) == 0 and lib.pauli_tile_valid_hermitian(2, 1, 17) == 0
    # the Hermitian defaults: one wave of 4 x 32 rows for the split paths from N = 12
    for algo in (2, 4):
        assert lib.pauli_tile_selected_hermitian(algo, 14) == lib.pauli_tile_selected_hermitian(algo, 12) == 7
        assert lib.pauli_tile_valid_hermitian(algo, 7, 12) == 1
        assert lib.pauli_tile_selected_hermitian(algo, 11) == lib.pauli_tile_selected(algo, 11)
    assert lib.pauli_tile_selected_hermitian(1, 14) == 3
    assert lib.pauli_tile_selected_hermitian(0, 14) == lib.pauli_tile_selected_hermitian(3, 14) == 0
    assert lib.pauli_tile_selected_hermitian(2, 17) == 0
    assert f(FAKE_IN, 10, 1, FAKE_OUT, ctypes.byref(opts(pauli, tile=-1))) == EINVAL


def test_coeffs_at_backward_validation(lib, pauli):
    u32 = ctypes.c_uint
    ns = (u32 * 3)(0, 5, 15)
    o = opts(pauli)
    f = lib.pauli_coeffs_at_backward
    assert f(FAKE_IN, 2, ns, 0, FAKE_OUT, ctypes.byref(o)) == EINVAL
    assert f(FAKE_IN, 1, ns, 3, FAKE_OUT, ctypes.byref(o)) == EINVAL      # 5 and 15 are not below 4^1
    assert f(FAKE_IN, 2, None, 3, FAKE_OUT, ctypes.byref(o)) == EINVAL
    assert f(FAKE_IN, 2, ns, 3, FAKE_IN + 16, ctypes.byref(o)) == EINVAL   # overlap
    small = opts(pauli, ws=0x30000000, ws_bytes=64)
    assert f(FAKE_IN, 2, ns, 3, FAKE_OUT, ctypes.byref(small)) == ENOMEM
    # the workspace bound covers the adjoint's plan (entries + 2^N + 1 offsets)
    assert lib.pauli_coeffs_at_workspace_bytes(14, 1) >= 4 * (2 ** 14 + 1)


def test_missing_library_fails_loudly(tmp_path):
    """No CPU fallback, checked in a fresh interpreter whose library path
    points at nothing: loading the library raises, and a decomposition of a
    host tensor raises too (the binding has no CPU path to fall back on)."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2401_16378_amd as p\n"
        "p.LIB_PATH = %r\n"
        "import torch\n"
        "G = torch.zeros(4, 4, dtype=torch.complex64)\n"
        "for f in (lambda: p.load_library(p.LIB_PATH), lambda: p.decompose(G)):\n"
        "    try:\n"
        "        f()\n"
        "    except Exception as e:\n"
        "        print('raised', type(e).__name__)\n"
        "    else:\n"
        "        print('computed')\n"
    ) % (ROOT, str(tmp_path / "absent" / "libpauli.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    lines = [l for l in r.stdout.splitlines() if l.startswith(("raised", "computed"))]
    assert lines and all(l.startswith("raised") for l in lines), (r.stdout, r.stderr)


def test_tune_cache_file_is_read(tmp_path):
    """The PAULI_TUNE_CACHE file feeds the tile choice of a fresh process:
    single-matrix lines "algo N tile" and batch lines "B planes tile
    c_1 .. c_12" (c_n matrices of order n); malformed lines are ignored."""
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    cache.write_text("2 10 3\n"
                     "B 3 4 0 0 1 1 2 1 0 0 0 0 0 0\n"      # one N=3, one N=4, two N=5, one N=6
                     "not a line\n")
    code = (
        "import sys, ctypes; sys.path.insert(0, %r)\n"
        "import paper_2401_16378_amd as p\n"
        "lib = p.load_library()\n"
        "Na = (ctypes.c_int * 5)(5, 3, 6, 4, 5)\n"
        "print(lib.pauli_tile_selected(2, 10), lib.pauli_batched_tile_selected(5, Na, 2),"
        " lib.pauli_batched_tile_selected(5, Na, 1))\n"
    ) % ROOT
    env = dict(os.environ, PAULI_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    tile, btile, btile_fp32 = map(int, r.stdout.split())
    assert (tile, btile) == (3, 4)
    assert btile_fp32 == 8                       # binary32 has no entry: the default shape


def test_tune_cache_invalid_tiles_fall_back(tmp_path):
    """A tune file naming a tile that does not exist, or one that the algo
    does not build (binary32 has no 4 x 32-row register-ring tiles), is not
    used: the lookups return the default shapes instead."""
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    cache.write_text("2 10 99\n"
                     "1 10 1\n"                                  # fp32 register ring RB=4: not built
                     "B 3 9 0 0 1 1 2 1 0 0 0 0 0 0\n"           # shape 9 does not exist
                     "B 1 -2 0 0 1 1 2 1 0 0 0 0 0 0\n"          # negative shape
                     "B 3 0 0 0 0 1 0 0 0 0 0 0 0 0\n")          # shape 0 for one N=5
    code = (
        "import sys, ctypes; sys.path.insert(0, %r)\n"
        "import paper_2401_16378_amd as p\n"
        "lib = p.load_library()\n"
        "Na = (ctypes.c_int * 5)(5, 3, 6, 4, 5)\n"
        "Nb = (ctypes.c_int * 1)(5)\n"
        "print(lib.pauli_tile_selected(2, 10), lib.pauli_tile_selected(1, 10),"
        " lib.pauli_batched_tile_selected(5, Na, 2), lib.pauli_batched_tile_selected(5, Na, 1),"
        " lib.pauli_batched_tile_selected(1, Nb, 2))\n"
    ) % ROOT
    env = dict(os.environ, PAULI_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    t_bf16, t_fp32, b_bf16, b_fp32, b_one = map(int, r.stdout.split())
    assert t_bf16 == 1 and t_fp32 == 15          # the defaults at N=10
    assert (b_bf16, b_fp32, b_one) == (9, 8, 9)   # the default shapes


def test_noalloc_validation(lib, pauli):
    """The no-allocation entry point checks its arguments like
    pauli_decompose and refuses, before any HIP call, a request whose scratch
    exceeds the fixed array."""
    assert lib.pauli_noalloc_scratch_bytes() == 64 << 20
    o = opts(pauli)
    f = lib.pauli_decompose_noalloc
    assert f(FAKE_IN, -1, 1, FAKE_OUT, ctypes.byref(o)) == EINVAL
    assert f(None, 4, 1, FAKE_OUT, ctypes.byref(o)) == EINVAL
    assert f(FAKE_IN, 4, 0, FAKE_OUT, ctypes.byref(o)) == EINVAL
    assert f(FAKE_IN, 12, 1, FAKE_OUT, ctypes.byref(o)) == ENOMEM            # 192 MiB packed operand
    assert "fixed scratch" in pauli.last_error()
    assert f(FAKE_IN, 11, 2, FAKE_OUT, ctypes.byref(o)) == ENOMEM            # 2 x 48 MiB
    assert f(FAKE_IN, 12, 1, FAKE_OUT, ctypes.byref(opts(pauli, algo="fwht"))) == ENOMEM
    assert f(FAKE_IN, 17, 1, FAKE_OUT, ctypes.byref(opts(pauli, algo="fwht"))) == EINVAL
    # a workspace in the options is ignored, not checked against the buffers
    ws = opts(pauli, ws=FAKE_IN, ws_bytes=1 << 30)
    assert f(FAKE_IN, 12, 1, FAKE_OUT, ctypes.byref(ws)) == ENOMEM


def test_entry_points_compile():
    """The driver-facing scripts at the repository root parse and define
    their entry points (nothing is built or run here)."""
    import importlib
    import py_compile
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for name in ("__graft_entry__.py", "bench.py"):
        py_compile.compile(os.path.join(root, name), doraise=True)
    g = importlib.import_module("__graft_entry__")
    assert callable(g.build) and callable(g.smoke)
