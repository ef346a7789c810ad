"""Batched solves of many uneven single-block plans in one captured graph."""
import numpy as np
import pytest

import workloads as W
from oracle import separable

pytestmark = pytest.mark.gpu


def _blocks(nblocks, lo, hi, zlo, zhi, seed):
    """Uneven blocks in the style of the batched workload, at test sizes: the
    first half uniform, the second half with stretched ends; one block with
    power-of-two n+1 so the sine-FFT path is in the batch too."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(nblocks):
        nx, ny = int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))
        nz = int(rng.integers(zlo, zhi + 1))
        if b == 0:
            nx, ny = 31, 63
        k2 = W.draw_k2(rng, 4)
        if b < nblocks // 2:
            hx, hy = W.uniform_steps(nx), W.uniform_steps(ny)
        else:
            hx, hy = W.stretched_ends_steps(nx, max(1, nx // 8)), W.stretched_ends_steps(ny, max(1, ny // 8))
        out.append(W.Problem(hx, hy, np.ones(nz + 1), W.layer_map(nz, 4), k2))
    return out


def _rel(u, ref):
    return np.linalg.norm((u - ref).ravel()) / np.linalg.norm(ref.ravel())


@pytest.mark.parametrize("prec,tol", [("c128", 1e-10), ("mixed", 1e-8)])
def test_batch_matches_oracle_and_single_plans(hs, prec, tol):
    import torch
    probs = _blocks(7, 12, 48, 8, 40, seed=5)
    nrhs = [1, 3, 2, 1, 2, 3, 1]
    rng = np.random.default_rng(6)
    plans = [hs.Plan(p, prec, max_rhs=r) for p, r in zip(probs, nrhs)]
    fs_np = [W.complex_normal(rng, (r,) + p.shape) for p, r in zip(probs, nrhs)]
    fs = [hs.to_device(f) for f in fs_np]
    batch = hs.Batch(plans, nrhs)
    us = batch.solve(fs)
    torch.cuda.synchronize()
    for p, plan, f_np, f, u in zip(probs, plans, fs_np, fs, us):
        got = u.cpu().numpy()
        ref = separable.solve(p, f_np)
        for r in range(f_np.shape[0]):
            assert _rel(got[r], ref[r]) < tol
        single = plan.solve(f).cpu().numpy()
        assert np.array_equal(got, single)


def test_batch_graph_replay_and_recapture(hs):
    import torch
    probs = _blocks(4, 10, 30, 6, 20, seed=9)
    nrhs = [2, 1, 2, 1]
    rng = np.random.default_rng(10)
    plans = [hs.Plan(p, "c128", max_rhs=r) for p, r in zip(probs, nrhs)]
    fs = [hs.to_device(W.complex_normal(rng, (r,) + p.shape)) for p, r in zip(probs, nrhs)]
    batch = hs.Batch(plans, nrhs)
    us = [torch.empty_like(f) for f in fs]
    results = []
    for _ in range(3):
        for u in us:
            u.zero_()
        batch.solve(fs, us)
        torch.cuda.synchronize()
        results.append([u.cpu().numpy() for u in us])
    for rep in results[1:]:
        for a, b in zip(results[0], rep):
            assert np.array_equal(a, b)
    # new output arrays force a new capture; same answer
    us2 = batch.solve(fs)
    torch.cuda.synchronize()
    for a, u in zip(results[0], us2):
        assert np.array_equal(a, u.cpu().numpy())


def test_batch_rejects_decomposed_plans(hs):
    p, _ = W.c2_decomposed(core_cells=16, pml_cells=3, nz=8, nlayers=2)
    plan = hs.Plan(p, "c128")
    with pytest.raises(hs.HSError):
        hs.Batch([plan], [1])


@pytest.mark.parametrize("prec,tol", [("c128", 1e-10), ("mixed", 1e-8)])
def test_batch_tuner_keeps_parity_and_caches(hs, prec, tol, tmp_path):
    """The batch's own autotuner times its launch shapes on the whole graph;
    the tuned batch still matches the oracle, and a second batch of the same
    shapes takes the shapes from the cache file."""
    import torch
    probs = _blocks(6, 16, 40, 12, 48, seed=21)
    nrhs = [2, 1, 1, 2, 1, 2]
    rng = np.random.default_rng(22)
    plans = [hs.Plan(p, prec, max_rhs=r, refine_steps=1 if prec == "mixed" else 0) for p, r in zip(probs, nrhs)]
    fs_np = [W.complex_normal(rng, (r,) + p.shape) for p, r in zip(probs, nrhs)]
    fs = [hs.to_device(f) for f in fs_np]
    us = [torch.empty_like(f) for f in fs]
    cache = str(tmp_path / "batch_tune.jsonl")
    batch = hs.Batch(plans, nrhs)
    batch.tune(fs, us, cache=cache)
    us = batch.solve(fs, us)
    torch.cuda.synchronize()
    for p, f_np, u in zip(probs, fs_np, us):
        ref = separable.solve(p, f_np)
        got = u.cpu().numpy()
        for r in range(f_np.shape[0]):
            assert _rel(got[r], ref[r]) < tol
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"fixed_rows"' in lines[0]
    batch2 = hs.Batch(plans, nrhs)
    batch2.tune(fs, [torch.empty_like(f) for f in fs], cache=cache)
    assert len(open(cache).read().strip().splitlines()) == 1


def test_batch_new_pointers_back_to_back(hs):
    """Solves with new array pointers issued back to back, with no
    synchronization between them: each capture waits for the previous graph
    before its descriptors are rewritten, so every result is right."""
    import torch
    probs = _blocks(5, 12, 36, 8, 30, seed=31)
    nrhs = [1, 2, 1, 1, 2]
    rng = np.random.default_rng(32)
    plans = [hs.Plan(p, "mixed", max_rhs=r, refine_steps=1) for p, r in zip(probs, nrhs)]
    batch = hs.Batch(plans, nrhs)
    sets = []
    for _ in range(3):
        fs_np = [W.complex_normal(rng, (r,) + p.shape) for p, r in zip(probs, nrhs)]
        fs = [hs.to_device(f) for f in fs_np]
        sets.append((fs_np, fs, batch.solve(fs)))
    torch.cuda.synchronize()
    for fs_np, fs, us in sets:
        for p, f_np, u in zip(probs, fs_np, us):
            ref = separable.solve(p, f_np)
            got = u.cpu().numpy()
            for r in range(f_np.shape[0]):
                assert _rel(got[r], ref[r]) < 1e-8
