"""Fused-form layouts (cells per wave) and the autotuner: every feasible layout must give
the oracle's result to the same tolerance as the default one."""
import sys

import numpy as np
import pytest

import npfem_inputs as I
from _runners import cell_errors, lib_types, oracle_types, run_oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mixed(seed=111):
    tids = np.array([I.RBC] * 6 + [I.PLT] * 19, dtype=np.int32)
    tids = tids[np.random.default_rng(seed).permutation(len(tids))]
    return I.make_batch(tids, seed=seed)


def _run(batch, b, forces, K):
    import torch
    x = torch.tensor(b.x0, dtype=torch.float32, device="cuda")
    v = torch.tensor(b.v0, dtype=torch.float32, device="cuda")
    for f in forces:
        batch.step(x, v, torch.tensor(f, dtype=torch.float32, device="cuda"), I.DT, K)
    batch.check()
    return x.double().cpu().numpy()


@pytest.mark.parametrize("rbc_gw,plt_gw", [(1, 4), (2, 4), (2, 2), (1, 1)])
def test_layout_parity(rbc_gw, plt_gw):
    from paper_1911_03062_amd import npfem as N
    types = lib_types()
    b = _mixed()
    forces = list(I.force_stream(b, seed=112, sigma=20.0, n_steps=4))
    batch = N.Batch([types[int(t)] for t in b.types], 32, "fused")
    batch.set_cells_per_wave(types[I.RBC], rbc_gw)
    batch.set_cells_per_wave(types[I.PLT], plt_gw)
    assert batch.cells_per_wave(types[I.RBC]) == rbc_gw
    assert batch.cells_per_wave(types[I.PLT]) == plt_gw
    _say(f"case: layouts RBC {rbc_gw} / PLT {plt_gw} cells per wave, 4 steps")
    xg = _run(batch, b, forces, 10)
    xo, _ = run_oracle(oracle_types(), b.types, b.offsets, b.x0, b.v0, forces, 10)
    err = cell_errors(b.types, b.offsets, xg, xo)
    _say(f"layouts {rbc_gw}/{plt_gw}: max err/diam {err.max():.3e}")
    assert err.max() <= 1e-5


def test_layout_errors():
    from paper_1911_03062_amd import npfem as N
    types = lib_types()
    batch = N.Batch([types[I.RBC]], 32, "fused")
    with pytest.raises(N.NpfemError) as ei:
        batch.set_cells_per_wave(types[I.RBC], 4)           # not feasible for 258 vertices
    assert ei.value.name == "NPFEM_E_UNSUPPORTED"
    with pytest.raises(N.NpfemError) as ei:
        batch.set_cells_per_wave(types[I.PLT], 4)           # type not in the batch
    assert ei.value.name == "NPFEM_E_INVALID"
    mixed = N.Batch([types[I.PLT], types[I.RBC]], 32, "fused")
    with pytest.raises(N.NpfemError) as ei:
        mixed.set_cells_per_wave(types[I.PLT], 8)           # 32 platelets exceed the LDS budget
    assert ei.value.name == "NPFEM_E_UNSUPPORTED"
    plain = N.Batch([types[I.RBC]], 32, "plain")
    with pytest.raises(N.NpfemError) as ei:
        plain.autotune(10)
    assert ei.value.name == "NPFEM_E_UNSUPPORTED"


def test_autotune_picks_a_feasible_layout_and_keeps_parity():
    from paper_1911_03062_amd import npfem as N
    types = lib_types()
    b = _mixed(seed=121)
    forces = list(I.force_stream(b, seed=122, sigma=20.0, n_steps=3))
    batch = N.Batch([types[int(t)] for t in b.types], 32, "fused")
    _say("case: autotune K=10, 2 reps")
    chosen = batch.autotune(10, reps=2)
    _say(f"autotune chose {chosen}")
    assert batch.cells_per_wave(types[I.RBC]) in types[I.RBC].cells_per_wave()
    assert batch.cells_per_wave(types[I.PLT]) in types[I.PLT].cells_per_wave()
    xg = _run(batch, b, forces, 10)
    xo, _ = run_oracle(oracle_types(), b.types, b.offsets, b.x0, b.v0, forces, 10)
    err = cell_errors(b.types, b.offsets, xg, xo)
    _say(f"after autotune: max err/diam {err.max():.3e}")
    assert err.max() <= 1e-5


def test_cell_order_does_not_change_results():
    """The fused work list sends the types with the most vertices per cell first, whatever
    order the batch lists its cells in; that order only decides when a cell's group runs, so
    every cell's step is bitwise the same when the batch lists its cells in another order
    (platelets first here, red cells first in the other batch)."""
    import torch
    from paper_1911_03062_amd import npfem as N
    types = lib_types()
    b = _mixed(seed=121)
    forces = list(I.force_stream(b, seed=122, sigma=20.0, n_steps=3))
    order = np.concatenate([np.where(b.types == I.PLT)[0], np.where(b.types == I.RBC)[0]])
    idx = np.concatenate([np.arange(b.offsets[c], b.offsets[c + 1]) for c in order])
    _say(f"case: {len(order)} cells listed platelets first vs the original order, 3 steps x K = 10")
    results = []
    for cells, cols in ((np.arange(len(b.types)), np.arange(b.x0.shape[1])), (order, idx)):
        batch = N.Batch([types[int(b.types[c])] for c in cells], 32, "fused")
        x = torch.tensor(np.ascontiguousarray(b.x0[:, cols]), dtype=torch.float32, device="cuda")
        v = torch.tensor(np.ascontiguousarray(b.v0[:, cols]), dtype=torch.float32, device="cuda")
        for f in forces:
            ft = torch.tensor(np.ascontiguousarray(np.asarray(f)[:, cols]), dtype=torch.float32,
                              device="cuda")
            batch.step(x, v, ft, I.DT, 10)
        batch.check()
        xo = np.empty_like(b.x0, dtype=np.float32)
        vo = np.empty_like(b.v0, dtype=np.float32)
        xo[:, cols] = x.cpu().numpy()
        vo[:, cols] = v.cpu().numpy()
        results.append((xo, vo))
    assert np.array_equal(results[0][0], results[1][0])
    assert np.array_equal(results[0][1], results[1][1])
