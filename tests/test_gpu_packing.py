"""Particle-in-kernel contact detection and the cell-packing step on the GPU against the FP64
oracle: the contact decisions (which vertices collide, with which neighbour) bit for bit in the
batch precision, the projection points to rounding, and packing steps one by one."""
import sys

import numpy as np
import pytest

import npfem_inputs as I
import oracle as O
from _runners import cell_errors

pytestmark = pytest.mark.gpu

P = I.PACKING


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _types():
    from paper_1911_03062_amd import npfem as N
    inp = I.cell_type_inputs()
    return ({k: N.CellType(x, t, m, I.DT) for k, (x, t, m) in inp.items()},
            {k: O.CellType(x, t, m, I.DT) for k, (x, t, m) in inp.items()})


def _detect(batch, x_np, precision, radius=P["radius"], sep=P["separation"], weight=P["weight"]):
    import torch
    dt = torch.float64 if precision == 64 else torch.float32
    x = torch.tensor(x_np, dtype=dt, device="cuda").contiguous()
    cp = torch.full_like(x, float("nan"))
    cw = torch.full((x.shape[1],), float("nan"), dtype=dt, device="cuda")
    batch.detect_contacts(x, radius, sep, weight, cp, cw)
    torch.cuda.synchronize()
    return cp.double().cpu().numpy(), cw.double().cpu().numpy()


def _compare(pg, wg, po, wo, x, precision):
    assert np.array_equal(wg, wo)                                   # same contacts, same weight
    off = wo == 0
    assert np.array_equal(pg[:, off], x[:, off])                    # p = x without contact
    tol = 1e-12 if precision == 64 else 2e-5
    err = np.abs(pg[:, ~off] - po[:, ~off]).max() if (~off).any() else 0.0
    assert err <= tol * max(1.0, np.abs(x).max() / 10.0), err       # same neighbour, rounding
    return err


@pytest.mark.parametrize("precision,form,spread", [(32, "fused", 0.0), (64, "plain", 0.0),
                                                   (32, "plain", 3000.0)])
def test_detection_matches_oracle(precision, form, spread):
    """6 RBC + 10 platelets placed at random at hematocrit 0.4 (many contacts); with `spread`,
    four more cells thousands of radii away (distant grid cells sharing hash buckets)."""
    from paper_1911_03062_amd import npfem as N
    lt, ot = _types()
    tids = np.array([I.RBC] * 6 + [I.PLT] * 10, dtype=np.int32)
    tids = tids[np.random.default_rng(301).permutation(len(tids))]
    b = I.packing_batch(tids, seed=302)
    x = b.x0
    types, offsets = b.types, b.offsets
    if spread:
        far = I.make_batch(np.array([I.PLT, I.RBC, I.PLT, I.PLT], dtype=np.int32), seed=303,
                           translate=spread)
        types = np.concatenate([types, far.types])
        offsets = np.concatenate([offsets, offsets[-1] + far.offsets[1:]])
        x = np.concatenate([x, far.x0], axis=1)
    batch = N.Batch([lt[int(t)] for t in types], precision=precision, form=form)
    _say(f"case: contact detection FP{precision} {form}, {len(types)} cells, spread {spread}")
    pg, wg = _detect(batch, x, precision)
    dtype = np.float64 if precision == 64 else np.float32
    po, wo, j = O.pik_contacts(ot, types, offsets, x, P["radius"], P["separation"], P["weight"], dtype)
    err = _compare(pg, wg, po, wo, x, precision)
    _say(f"contacts {np.mean(wo > 0):.3f} of the vertices, max |p - p_oracle| {err:.3e} um")
    assert np.mean(wo > 0) > 0.2


def test_detection_single_cell_empty_batch_and_errors():
    import torch
    from paper_1911_03062_amd import npfem as N
    lt, _ = _types()
    b = I.make_batch(np.array([I.RBC], dtype=np.int32), seed=5)
    one = N.Batch([lt[I.RBC]], precision=32, form="fused")
    pg, wg = _detect(one, b.x0, 32)
    assert np.all(wg == 0.0) and np.array_equal(pg, b.x0)          # no foreign vertex at all
    empty = N.Batch([], precision=32, form="fused")
    e = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    empty.detect_contacts(e, 1.0, 1.0, 1.0, e, torch.zeros((0,), device="cuda"))
    x = torch.tensor(b.x0, dtype=torch.float32, device="cuda")
    cw = torch.empty((x.shape[1],), dtype=torch.float32, device="cuda")
    for r, s, w in ((0.0, 1.0, 1.0), (-1.0, 1.0, 1.0), (float("nan"), 1.0, 1.0),
                    (float("inf"), 1.0, 1.0), (1.0, -0.1, 1.0), (1.0, 1.0, -1.0),
                    (1.0, float("nan"), 1.0)):
        with pytest.raises(N.NpfemError) as ei:
            one.detect_contacts(x, r, s, w, torch.empty_like(x), cw)
        assert ei.value.name == "NPFEM_E_INVALID"
    with pytest.raises(N.NpfemError) as ei:
        N._check(N.lib().npfem_detect_contacts(one._h, None, 1.0, 1.0, 1.0, None, None, None))
    assert ei.value.name == "NPFEM_E_INVALID"


@pytest.mark.parametrize("precision,form", [(32, "fused"), (64, "plain")])
def test_packing_steps_match_oracle_stepwise(precision, form):
    """Packing steps (contacts from the current positions, no external force): each GPU step
    against the oracle's packing step from the same (GPU) state, so that a contact decision
    never flips between the two sides."""
    import torch
    from paper_1911_03062_amd import npfem as N
    lt, ot = _types()
    tids = np.array([I.RBC] * 4 + [I.PLT] * 8, dtype=np.int32)
    tids = tids[np.random.default_rng(311).permutation(len(tids))]
    b = I.packing_batch(tids, seed=312)
    batch = N.Batch([lt[int(t)] for t in b.types], precision=precision, form=form)
    dt = torch.float64 if precision == 64 else torch.float32
    dtype = np.float64 if precision == 64 else np.float32
    x = torch.tensor(b.x0, dtype=dt, device="cuda")
    v = torch.zeros_like(x)
    f = torch.zeros_like(x)
    K = P["n_pd_iters"]
    _say(f"case: packing steps FP{precision} {form}, 4 RBC + 8 PLT, 5 steps x K = {K}")
    worst = 0.0
    for s in range(5):
        x0 = x.double().cpu().numpy()
        v0 = v.double().cpu().numpy()
        cp, cw = batch.detect_contacts(x, P["radius"], P["separation"], P["weight"])
        batch.step(x, v, f, I.DT, K, contacts=(cp, cw))
        batch.check()
        xo, vo, wo = O.packing_step(ot, b.types, b.offsets, x0, v0, K, P["radius"],
                                    P["separation"], P["weight"], dtype)
        assert np.array_equal(cw.double().cpu().numpy(), wo)
        err = cell_errors(b.types, b.offsets, x.double().cpu().numpy(), xo)
        worst = max(worst, err.max())
        _say(f"step {s}: contacts {np.mean(wo > 0):.3f}, max err/diam {err.max():.3e}")
    assert worst <= (1e-10 if precision == 64 else 1e-5)


def test_full_size_detection_sampled():
    """The packing workload at full size (20 000 RBC + 4 000 platelets at hematocrit 0.4,
    5.42 M vertices) in one detection pass; the oracle searches sampled vertices by brute
    force over every vertex of the batch."""
    from paper_1911_03062_amd import npfem as N
    lt, ot = _types()
    w = I.WORKLOADS["large_24000"]
    b = I.packing_batch(w.types(), seed=w.seed)
    batch = N.Batch([lt[int(t)] for t in b.types], precision=32, form="fused")
    _say(f"case: contact detection, packing {b.n_cells} cells ({b.v_total} vertices), sampled")
    pg, wg = _detect(batch, b.x0, 32)
    rng = np.random.default_rng(321)
    rows = np.unique(np.concatenate([rng.choice(b.v_total, 200, replace=False),
                                     np.nonzero(wg > 0)[0][:20], [0, b.v_total - 1]]))
    po, wo, _ = O.pik_contacts(ot, b.types, b.offsets, b.x0, P["radius"], P["separation"],
                               P["weight"], np.float32, rows=rows)
    _compare(pg[:, rows], wg[rows], po, wo, b.x0[:, rows], 32)
    _say(f"full size: {np.mean(wg > 0):.3f} of the vertices in contact; {len(rows)} sampled")
    assert 0.1 < np.mean(wg > 0) < 0.9


def test_full_size_packing_step_sampled():
    """One packing step of the full-size placement (24 000 cells, the bench's layout and K):
    the oracle finds the contacts of 2 RBC and 2 platelets by brute force over all 5.42 M
    vertices and steps those cells; positions within the fused form's tolerance and the
    contact decisions bit for bit."""
    import torch
    from paper_1911_03062_amd import npfem as N
    lt, ot = _types()
    w = I.WORKLOADS["large_24000"]
    b = I.packing_batch(w.types(), seed=w.seed)
    batch = N.Batch([lt[int(t)] for t in b.types], precision=32, form="fused")
    batch.set_cells_per_wave(lt[I.RBC], 2)
    batch.set_cells_per_wave(lt[I.PLT], 4)
    K = P["n_pd_iters"]
    _say(f"case: packing step at full size ({b.n_cells} cells), K = {K}, 4 sampled cells")
    x = torch.tensor(b.x0, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(x)
    cp, cw = batch.detect_contacts(x, P["radius"], P["separation"], P["weight"])
    batch.step(x, v, torch.zeros_like(x), I.DT, K, contacts=(cp, cw))
    batch.check()
    xg = x.double().cpu().numpy()
    wg = cw.double().cpu().numpy()
    rng = np.random.default_rng(331)
    cells = np.concatenate([rng.choice(np.nonzero(b.types == I.RBC)[0], 2, replace=False),
                            rng.choice(np.nonzero(b.types == I.PLT)[0], 2, replace=False)])
    rows = np.concatenate([np.arange(b.offsets[c], b.offsets[c + 1]) for c in cells])
    po, wo, _ = O.pik_contacts(ot, b.types, b.offsets, b.x0, P["radius"], P["separation"],
                               P["weight"], np.float32, rows=rows)
    assert np.array_equal(wg[rows], wo)
    p_full = b.x0.copy()
    w_full = np.zeros(b.v_total)
    p_full[:, rows] = po
    w_full[rows] = wo
    xo, _ = O.step_batch(ot, b.types, b.offsets, b.x0, np.zeros_like(b.x0), np.zeros_like(b.x0),
                         K, cells=cells, contact_p=p_full, contact_w=w_full)
    err = cell_errors(b.types, b.offsets, xg, xo, cells)
    _say(f"full-size packing step: {np.mean(wo > 0):.3f} of the sampled vertices in contact, "
         f"max err/diam {err.max():.3e}")
    assert np.mean(wo > 0) > 0.1
    assert err.max() <= 1e-5


def test_detection_ignores_the_active_subset():
    """npfem_batch_set_active restricts steps, not detection: every cell takes part."""
    import torch
    from paper_1911_03062_amd import npfem as N
    lt, _ = _types()
    tids = np.array([I.RBC] * 3 + [I.PLT] * 6, dtype=np.int32)
    b = I.packing_batch(tids, seed=341)
    batch = N.Batch([lt[int(t)] for t in b.types], precision=32, form="fused")
    _say("case: contact detection with an active subset of 2 of 9 cells")
    p_all, w_all = _detect(batch, b.x0, 32)
    batch.set_active([1, 7])
    p_sub, w_sub = _detect(batch, b.x0, 32)
    assert (w_all > 0).any()
    assert np.array_equal(w_all, w_sub) and np.array_equal(p_all, p_sub)
