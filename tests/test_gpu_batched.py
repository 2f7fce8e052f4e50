"""Uneven batch through the C ABI: 512 complex64 matrices with N uniform on
3..9 (102 Hermitian), one batched pack and one persistent contraction launch
replayed from a captured HIP graph.

Every output tile sums its K slices in the same order whatever the tile
shape, so the batch must reproduce the single-matrix path bit for bit; the
single-matrix path is checked against the oracle elsewhere, and here every
matrix is also checked against the oracle directly (all coefficients for
N <= 8, a seeded sample for N = 9).
"""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


def lib():
    import paper_2401_16378_amd as p
    p.load_library()
    return p


def threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def batch():
    Ns, mats, herm = workloads.batch_spec()
    dev = [torch.from_numpy(m).to("cuda") for m in mats]
    return Ns, mats, herm, dev


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16"])
def test_batch_vs_oracle(batch, algo):
    p = lib()
    Ns, mats, herm, dev = batch
    outs = p.decompose_batched(dev, algo=algo)
    torch.cuda.synchronize()
    worst = 0.0
    for k, (N, G) in enumerate(zip(Ns, mats)):
        c = outs[k].cpu().numpy().astype(np.complex128)
        if N <= 8:
            ref = oracle.decompose(G, threads=threads())
            got = c
        else:
            ns = workloads.sample_indices(4 ** N, 2048, seed=k)
            ref = oracle.coeffs_at(G, ns, threads=threads())
            got = c[ns.astype(np.int64)]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        assert err <= 1e-6, (k, N, err)
        if herm[k]:
            assert np.abs(c.imag).max() <= 1e-6 * np.abs(c).max()
    assert worst > 0.0


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16"])
def test_batch_bitexact_vs_single(batch, algo):
    p = lib()
    Ns, mats, herm, dev = batch
    outs = p.decompose_batched(dev, algo=algo)
    for k in range(0, len(dev), 7):
        single = p.decompose(dev[k], algo=algo)
        assert torch.equal(outs[k], single), k


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_every_tile_shape(batch, tile, algo):
    p = lib()
    if not p.batched_tile_valid(tile, algo):
        assert tile == 7 and algo == "split_bf16"
        return
    Ns, mats, herm, dev = batch
    ref = p.decompose_batched(dev, algo=algo, tile=1)
    got = p.decompose_batched(dev, algo=algo, tile=tile)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)


def test_graph_replays_and_new_buffers(batch):
    """Replay the captured graph several times with eager work and
    synchronisations in between, and with fresh output buffers; every replay
    must equal the first result."""
    p = lib()
    Ns, mats, herm, dev = batch
    first = [o.clone() for o in p.decompose_batched(dev)]
    for r in range(3):
        # unrelated eager work on the same stream between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        outs = [torch.full_like(o, float("nan")) for o in first]
        p.decompose_batched(dev, outs=outs)
        torch.cuda.synchronize()
        for a, b in zip(first, outs):
            assert torch.equal(a, b), r
        del junk
    # new input buffers (same sizes): the descriptor table is refreshed per call
    dev2 = [d.clone() for d in dev]
    outs2 = p.decompose_batched(dev2)
    for a, b in zip(first, outs2):
        assert torch.equal(a, b)


def test_batch_plan_replays(batch):
    """BatchPlan marshals the arguments once; every run() replays the graph
    on the current contents of the same buffers."""
    p = lib()
    Ns, mats, herm, dev = batch
    ref = [o.clone() for o in p.decompose_batched(dev)]
    src = [d.clone() for d in dev]
    plan = p.BatchPlan(src)
    for r in range(3):
        outs = plan.run()
        torch.cuda.synchronize()
        for a, b in zip(ref, outs):
            assert torch.equal(a, b), r
    # doubling every input doubles every coefficient exactly (the split grids
    # are powers of two), so a stale read would show
    for d in src:
        d.mul_(2)
    outs = plan.run()
    torch.cuda.synchronize()
    for a, b in zip(ref, outs):
        assert torch.equal(2 * a, b)


def test_autotune_batched(batch):
    p = lib()
    Ns, mats, herm, dev = batch
    t = p.autotune_batched(dev)
    assert 1 <= t <= p.load_library().pauli_batched_tile_count()
    ref = p.decompose_batched(dev, tile=1)
    got = p.decompose_batched(dev)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)


def test_small_mixed_batch_fp32():
    p = lib()
    Ns = [1, 2, 5, 3, 7, 4, 6, 9]
    mats = [workloads.iid_complex(n, 40 + n, np.complex64) for n in Ns]
    dev_m = [torch.from_numpy(m).to("cuda") for m in mats]
    tiles = [t for t in range(1, p.load_library().pauli_batched_tile_count() + 1) if p.batched_tile_valid(t, "fp32")]
    assert len(tiles) == p.load_library().pauli_batched_tile_count() - 1   # all but the 512-row fused shape
    for tile in tiles:
        outs = p.decompose_batched(dev_m, algo="fp32", tile=tile)
        for m, o in zip(mats, outs):
            ref = oracle.decompose(m)
            assert np.abs(o.cpu().numpy() - ref).max() / np.abs(ref).max() <= 1e-5, tile
    assert 1 <= p.autotune_batched(dev_m, algo="fp32") in tiles


def test_batched_arguments_refused():
    """Outputs of the wrong count, size, dtype or layout, and a matrix with a
    batch dimension, are refused before any launch (the kernels write 4^N
    values through each output pointer); correct outputs are filled."""
    p = lib()
    mats = [torch.from_numpy(workloads.iid_complex(n, 4400 + n, np.complex64)).cuda() for n in (3, 4)]
    good = [torch.empty(4 ** n, dtype=torch.complex64, device="cuda") for n in (3, 4)]
    bad_sets = [
        good[:1],                                                                    # one output for two matrices
        [good[0], torch.empty(4 ** 4 - 1, dtype=torch.complex64, device="cuda")],    # one value short
        [good[0], torch.empty(4 ** 4, dtype=torch.complex128, device="cuda")],       # wrong dtype
        [good[0], torch.empty(2 * 4 ** 4, dtype=torch.complex64, device="cuda")[::2]],   # not contiguous
    ]
    for outs in bad_sets:
        with pytest.raises(ValueError):
            p.decompose_batched(mats, outs=outs)
        with pytest.raises(ValueError):
            p.BatchPlan(mats, outs=outs)
    with pytest.raises(ValueError):
        p.decompose_batched([mats[0], torch.stack([mats[1], mats[1]])])
    outs = p.decompose_batched(mats, outs=good)
    torch.cuda.synchronize()
    for m, o, g in zip(mats, outs, good):
        assert o is g
        assert torch.equal(o, p.decompose(m))


def test_graph_cache_bounded_by_eviction():
    """More distinct batches (N lists) than the graph cache keeps: the least
    recently used captures are released and rebuilt on demand, and every
    call still returns the single-matrix result."""
    p = lib()
    rng = np.random.default_rng(4242)
    mats = [torch.from_numpy(workloads.iid_complex(int(n), 4300 + k, np.complex64)).cuda()
            for k, n in enumerate(rng.integers(3, 7, 80))]
    singles = [p.decompose(m) for m in mats]
    for k in range(1, 81):                      # 80 distinct N lists: prefixes of the list
        outs = p.decompose_batched(mats[:k])
        torch.cuda.synchronize()
        for a, b in zip(outs, singles[:k]):
            assert torch.equal(a, b), k
    outs = p.decompose_batched(mats[:1])        # the first capture was evicted long ago
    torch.cuda.synchronize()
    assert torch.equal(outs[0], singles[0])


def test_autotune_batched_writes_tune_cache(tmp_path):
    """pauli_autotune_batched records its choice in the PAULI_TUNE_CACHE file
    (a "B planes tile c_1 .. c_12" line), which a later process reads back."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, PAULI_TUNE_CACHE=str(cache))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import numpy as np, torch, workloads, paper_2401_16378_amd as p\n"
        "mats = [torch.from_numpy(workloads.iid_complex(n, 5200 + k, np.complex64)).cuda()\n"
        "        for k, n in enumerate([3, 4, 5, 6, 6, 5])]\n"
        "print('tuned', p.autotune_batched(mats), flush=True)\n"
    ) % root
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    tuned = int([l for l in r.stdout.splitlines() if l.startswith("tuned")][0].split()[1])
    lines = cache.read_text().splitlines()
    assert "B 3 %d 0 0 1 1 2 2 0 0 0 0 0 0" % tuned in lines, lines


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
def test_large_members(algo):
    """Members up to the batched limit N = 12 next to small ones: every
    member equals its single-matrix decomposition bit for bit, for every
    tile shape, and a seeded sample of each large member matches the
    oracle."""
    p = lib()
    Ns = [12, 3, 10, 11, 5, 12, 9]
    mats = [workloads.iid_complex(n, 8400 + k, np.complex64) for k, n in enumerate(Ns)]
    dev = [torch.from_numpy(m).cuda() for m in mats]
    singles = [p.decompose(d, algo=algo) for d in dev]
    nb = p.load_library().pauli_batched_tile_count()
    for tile in range(1, nb + 1):
        if not p.batched_tile_valid(tile, algo):
            continue
        outs = p.decompose_batched(dev, algo=algo, tile=tile)
        for k in range(len(Ns)):
            assert torch.equal(outs[k], singles[k]), (tile, k, Ns[k])
    tol = 1e-5 if algo == "fp32" else 1e-6
    for k, (n, G) in enumerate(zip(Ns, mats)):
        if n < 10:
            continue
        ns = workloads.sample_indices(4 ** n, 4096, seed=8500 + k)
        ref = oracle.coeffs_at(G.astype(np.complex128), ns, threads=threads())
        got = singles[k].cpu().numpy()[ns.astype(np.int64)].astype(np.complex128)
        assert np.abs(got - ref).max() / np.abs(ref).max() <= tol, (k, n)
