"""Input range of the matrix-core paths, and the single-matrix autotuner.

* Scaling: the decomposition is linear, and multiplying G by 2^k changes no
  rounding in any path while every intermediate stays a normal number, so
  c(2^k G) = 2^k c(G) bit for bit.  The binary32-accumulating paths
  (SPLIT_BF16, FP32) accumulate unscaled partial sums of up to 2^N terms and
  hold for components below 2^(126 - N); SPLIT_FP16 rescales every input to
  just below 2^15 first, so it holds for every finite complex64 input whose
  components are normal numbers.
* Mixed magnitudes: rows of G scaled by 2^40, 1 and 2^-40 against the oracle
  at each path's tolerance (of max|c|).
* pauli_autotune on one matrix: the chosen tiles are valid, written to the
  tune file and read back by a fresh process.
"""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = {"fp32": 1e-5, "split_bf16": 1e-6, "split_fp16": 1e-6}
N = 8


def lib():
    import paper_2401_16378_amd as p
    p.load_library()
    return p


def largest_k(algo, G):
    """The largest k of the documented range for this input."""
    e = int(np.ceil(np.log2(max(np.abs(G.real).max(), np.abs(G.imag).max()))))
    return (127 - e) if algo == "split_fp16" else (126 - N - e)


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
def test_scaling_is_exact(algo):
    p = lib()
    G = workloads.iid_complex(N, 8100, np.complex64)
    c0 = p.decompose(torch.from_numpy(G).cuda(), algo=algo, out_dtype=torch.complex128)
    kmax = largest_k(algo, G)
    assert kmax >= 60
    # SPLIT_FP16 also far down (its prescale is exact for any normal input);
    # the others keep every split part and partial sum normal at -60
    for k in (-60, 60, kmax) + ((-100,) if algo == "split_fp16" else ()):
        Gk = torch.from_numpy(G).cuda() * (2.0 ** k)
        assert torch.isfinite(torch.view_as_real(Gk)).all()
        ck = p.decompose(Gk, algo=algo, out_dtype=torch.complex128)
        assert torch.equal(ck, c0 * (2.0 ** k)), (algo, k)


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
def test_mixed_magnitudes(algo):
    p = lib()
    Nm = 9
    G = workloads.iid_complex(Nm, 8200, np.complex64)
    s = np.random.default_rng(8201).integers(-1, 2, 1 << Nm)
    G = (G * np.ldexp(1.0, 40 * s)[:, None]).astype(np.complex64)
    c = p.decompose(torch.from_numpy(G).cuda(), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    ref = oracle.decompose(G.astype(np.complex128), threads=16)
    err = np.abs(c - ref).max() / np.abs(ref).max()
    assert err <= TOL[algo], err
    # the small rows still count where they dominate: a coefficient whose
    # flip mask pairs small rows only is checked on a matrix of small rows
    Gs = (workloads.iid_complex(Nm, 8202, np.complex64) * np.float32(2.0 ** -40)).astype(np.complex64)
    cs = p.decompose(torch.from_numpy(Gs).cuda(), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    refs = oracle.decompose(Gs.astype(np.complex128), threads=16)
    assert np.abs(cs - refs).max() / np.abs(refs).max() <= TOL[algo]


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16"])
def test_autotune_single_matrix(tmp_path, algo):
    """pauli_autotune(9, 10) in a fresh process with PAULI_TUNE_CACHE set:
    every chosen tile is valid, the file holds one line per N, a second fresh
    process selects the same tiles, and a decomposition with the tuned tile
    equals the one with that tile forced."""
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, PAULI_TUNE_CACHE=str(cache))
    code = (
        "import sys, ctypes; sys.path.insert(0, %r)\n"
        "import paper_2401_16378_amd as p\n"
        "L = p.load_library()\n"
        "o = p._opts(%r, 0, 0)\n"
        "st = L.pauli_autotune(9, 10, ctypes.byref(o))\n"
        "print('status', st, p.last_error())\n"
        "print('tiles', L.pauli_tile_selected(o.algo, 9), L.pauli_tile_selected(o.algo, 10))\n"
    ) % (ROOT, algo)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    out = dict(l.split(" ", 1) for l in r.stdout.splitlines() if l.startswith(("status", "tiles")))
    assert out["status"].split()[0] == "0", out
    t9, t10 = map(int, out["tiles"].split())
    p = lib()
    assert p.tile_valid(t9, 9, algo) and p.tile_valid(t10, 10, algo)
    lines = sorted(l.split() for l in cache.read_text().splitlines() if not l.startswith("B"))
    a = str(p.ALGOS[algo])
    assert [a, "9", str(t9)] in lines and [a, "10", str(t10)] in lines
    code2 = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2401_16378_amd as p\n"
        "L = p.load_library()\n"
        "print(L.pauli_tile_selected(%d, 9), L.pauli_tile_selected(%d, 10))\n"
    ) % (ROOT, p.ALGOS[algo], p.ALGOS[algo])
    r2 = subprocess.run([sys.executable, "-c", code2], env=env, capture_output=True, text=True, timeout=300)
    assert r2.returncode == 0, r2.stderr
    assert tuple(map(int, r2.stdout.split())) == (t9, t10)
    G = torch.from_numpy(workloads.iid_complex(10, 8300, np.complex64)).cuda()
    assert torch.equal(p.decompose(G, algo=algo, tile=t10), p.decompose(G, algo=algo, tile=1))
