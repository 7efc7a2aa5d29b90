"""HIP-graph replays of recorded steps (npfem_graph_create) against eager steps on the same
inputs: the fused kernel is deterministic, so replays must agree bitwise. Each replay is
separated from the next by eager work and a synchronisation, and every replay is checked."""
import sys

import numpy as np
import pytest

import npfem_inputs as I
from _runners import lib_types

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _setup(form="fused", n_rbc=7, n_plt=20, seed=81, n_steps=3):
    import torch
    from paper_1911_03062_amd import npfem as N
    types = lib_types()
    tids = np.array([I.RBC] * n_rbc + [I.PLT] * n_plt, dtype=np.int32)
    tids = tids[np.random.default_rng(seed).permutation(len(tids))]
    b = I.make_batch(tids, seed=seed)
    batch = N.Batch([types[int(t)] for t in tids], 32, form)
    forces = [torch.tensor(f, dtype=torch.float32, device="cuda")
              for f in I.force_stream(b, seed=seed + 1, sigma=30.0, n_steps=n_steps)]
    x0 = torch.tensor(b.x0, dtype=torch.float32, device="cuda")
    v0 = torch.tensor(np.random.default_rng(seed + 2).normal(0, 0.05, b.x0.shape),
                      dtype=torch.float32, device="cuda")
    return batch, forces, x0, v0, tids


def _eager(batch, forces, x0, v0, K):
    x, v = x0.clone(), v0.clone()
    for f in forces:
        batch.step(x, v, f, I.DT, K)
    batch.check()
    return x, v


@pytest.mark.parametrize("form", ["fused", "plain"])
def test_graph_replays_match_eager_steps(form):
    import torch
    n = (7, 20) if form == "fused" else (1, 2)
    batch, forces, x0, v0, _ = _setup(form, *n)
    K = 10
    xe, ve = _eager(batch, forces, x0, v0, K)
    xg, vg = x0.clone(), v0.clone()
    g = batch.graph(xg, vg, forces, I.DT, K)
    scratch_x, scratch_v = x0.clone(), v0.clone()
    for rep in range(3):
        _say(f"case: {form} graph of {len(forces)} steps, replay {rep}")
        xg.copy_(x0)
        vg.copy_(v0)
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(xg, xe) and torch.equal(vg, ve), rep
        # eager work between replays
        batch.step(scratch_x, scratch_v, forces[0], I.DT, K)
        torch.cuda.synchronize()
    batch.check()


def test_graph_keeps_the_active_list_of_its_creation():
    import torch
    batch, forces, x0, v0, tids = _setup("fused", 5, 11, seed=91, n_steps=1)
    sub = np.array([0, 3, 4, 9, 15], dtype=np.int32)
    K = 10
    # reference: the subset stepped eagerly
    batch.set_active(sub)
    xe, ve = _eager(batch, forces, x0, v0, K)
    xg, vg = x0.clone(), v0.clone()
    g = batch.graph(xg, vg, forces, I.DT, K)
    batch.set_active(None)       # later changes of the list must not reach the graph
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(xg, xe) and torch.equal(vg, ve)
    off = batch.offsets
    untouched = [c for c in range(len(tids)) if c not in set(sub.tolist())]
    for c in untouched:
        s = slice(int(off[c]), int(off[c + 1]))
        assert torch.equal(xg[:, s], x0[:, s])


def test_graph_argument_errors():
    import torch
    from paper_1911_03062_amd import npfem as N
    batch, forces, x0, v0, _ = _setup("fused", 1, 1, seed=95, n_steps=1)
    with pytest.raises(N.NpfemError) as ei:
        batch.graph(x0.clone(), v0.clone(), [], I.DT, 10)
    assert ei.value.name == "NPFEM_E_INVALID"
    with pytest.raises(N.NpfemError) as ei:
        batch.graph(x0.clone(), v0.clone(), forces, 2 * I.DT, 10)
    assert ei.value.name == "NPFEM_E_DT"
    with pytest.raises(ValueError):
        batch.graph(x0.clone(), v0.clone(), [forces[0].double()], I.DT, 10)


def test_graph_replays_of_the_viscoelastic_kernel_variant():
    """Types with position-based and Rayleigh damping and a velocity cap run the kernel variant
    with those paths (and the extra m M~^-1 product); its replays also equal eager steps."""
    import torch
    from paper_1911_03062_amd import npfem as N
    inp = I.cell_type_inputs()
    types = {k: N.CellType(x, t, m.with_rayleigh(0.0, 0.01).with_kappa(0.8).with_v_max(0.08), I.DT)
             for k, (x, t, m) in inp.items()}
    tids = np.array([I.RBC] * 5 + [I.PLT] * 11, dtype=np.int32)
    b = I.make_batch(tids, seed=86)
    batch = N.Batch([types[int(t)] for t in tids], 32, "fused")
    forces = [torch.tensor(f, dtype=torch.float32, device="cuda")
              for f in I.force_stream(b, seed=87, sigma=30.0, n_steps=3)]
    x0 = torch.tensor(b.x0, dtype=torch.float32, device="cuda")
    v0 = torch.tensor(np.random.default_rng(88).normal(0, 0.05, b.x0.shape), dtype=torch.float32,
                      device="cuda")
    xe, ve = _eager(batch, forces, x0, v0, 10)
    xg, vg = x0.clone(), v0.clone()
    g = batch.graph(xg, vg, forces, I.DT, 10)
    for rep in range(3):
        _say(f"case: viscoelastic graph of 3 steps, replay {rep}")
        xg.copy_(x0)
        vg.copy_(v0)
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(xg, xe) and torch.equal(vg, ve), rep
        _eager(batch, forces[:1], x0, v0, 2)   # eager work between replays
