"""Collision energies (particle-in-kernel technique) on the GPU against the FP64 oracle, both
forms: contacting vertices are pulled toward their projection points by w (x - p) in grad g."""
import sys

import numpy as np
import pytest

import npfem_inputs as I
import oracle as O
from _runners import cell_errors, lib_types, oracle_types

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(seed, frac=0.1, w=400.0, gap=0.1):
    tids = np.array([I.RBC] * 3 + [I.PLT] * 5, dtype=np.int32)
    tids = tids[np.random.default_rng(seed).permutation(len(tids))]
    b = I.make_batch(tids, seed=seed)
    rng = np.random.default_rng(seed + 1)
    v0 = rng.normal(0, 0.05, size=b.x0.shape).astype(np.float32).astype(np.float64)
    cw = np.where(rng.random(b.v_total) < frac, w, 0.0).astype(np.float32).astype(np.float64)
    cp = (b.x0 + gap * rng.normal(size=b.x0.shape)).astype(np.float32).astype(np.float64)
    forces = [np.where(cw > 0, 0.0, f) for f in I.force_stream(b, seed=seed + 2, sigma=10.0, n_steps=3)]
    return b, v0, cp, cw, forces


def _run_gpu(types, b, v0, forces, K, form, precision, contacts):
    import torch
    from paper_1911_03062_amd import npfem as N
    batch = N.Batch([types[int(t)] for t in b.types], precision=precision, form=form)
    dt = torch.float64 if precision == 64 else torch.float32
    x = torch.tensor(b.x0, dtype=dt, device="cuda")
    v = torch.tensor(v0, dtype=dt, device="cuda")
    con = None
    if contacts is not None:
        con = tuple(torch.tensor(a, dtype=dt, device="cuda").contiguous() for a in contacts)
    for f in forces:
        batch.step(x, v, torch.tensor(f, dtype=dt, device="cuda"), I.DT, K, contacts=con)
    batch.check()
    return x.double().cpu().numpy(), v.double().cpu().numpy()


def _run_oracle(b, v0, forces, K, contacts):
    ot = oracle_types()
    x, v = b.x0.copy(), v0.copy()
    for f in forces:
        if contacts is None:
            x, v = O.step_batch(ot, b.types, b.offsets, x, v, f, K)
        else:
            x, v = O.step_batch(ot, b.types, b.offsets, x, v, f, K, contact_p=contacts[0],
                                contact_w=contacts[1])
    return x, v


@pytest.mark.parametrize("form,precision", [("fused", 32), ("plain", 64), ("plain", 32)])
def test_contacts_mixed_batch(form, precision):
    b, v0, cp, cw, forces = _case(180)
    _say(f"case: contacts {form} FP{precision}, 3 RBC + 5 PLT, {int((cw > 0).sum())} contacting "
         f"vertices of {b.v_total}, 3 steps x K = 10")
    xo, vo = _run_oracle(b, v0, forces, 10, (cp, cw))
    xg, vg = _run_gpu(lib_types(), b, v0, forces, 10, form, precision, (cp, cw))
    err = cell_errors(b.types, b.offsets, xg, xo)
    xf, _ = _run_oracle(b, v0, forces, 10, None)
    sep = cell_errors(b.types, b.offsets, xf, xo)
    _say(f"contacts {form}/{precision}: max err/diam {err.max():.3e}, contacts vs none {sep.min():.3e}")
    if precision == 64:
        assert err.max() <= 1e-10
    else:
        assert err.max() <= 1e-5
    assert sep.min() > 100 * err.max()


def test_zero_weights_and_argument_errors():
    import torch
    from paper_1911_03062_amd import npfem as N
    b, v0, cp, _, forces = _case(181)
    cw0 = np.zeros(b.v_total)
    _say("case: contacts with zero weights, fused FP32")
    xa, _ = _run_gpu(lib_types(), b, v0, forces, 10, "fused", 32, None)
    xb, _ = _run_gpu(lib_types(), b, v0, forces, 10, "fused", 32, (cp, cw0))
    d = cell_errors(b.types, b.offsets, xa, xb)
    _say(f"zero weights vs no contacts: {d.max():.3e}")
    assert d.max() <= 1e-7
    batch = N.Batch([lib_types()[int(t)] for t in b.types], precision=32, form="fused")
    x = torch.tensor(b.x0, dtype=torch.float32, device="cuda")
    with pytest.raises(N.NpfemError) as ei:
        N._check(N.lib().npfem_step_contacts(batch._h, x.data_ptr(), x.data_ptr(), x.data_ptr(),
                                             I.DT, 1, None, None, x.data_ptr(), None))
    assert ei.value.name == "NPFEM_E_INVALID"


def test_contacts_full_size_sampled():
    """The benchmark's contacts leg at full size: 5 % of the 5.4 M vertices in contact
    (w = 400 pN/um within 0.1 um, their forces zeroed), 2 steps of K = 20, sampled cells."""
    import torch
    from paper_1911_03062_amd import npfem as N
    w = I.WORKLOADS["large_24000"]
    b = w.batch()
    rng = np.random.default_rng(13)
    cw = np.where(rng.random(b.v_total) < 0.05, 400.0, 0.0).astype(np.float32).astype(np.float64)
    cp = (b.x0 + 0.1 * rng.normal(size=b.x0.shape)).astype(np.float32).astype(np.float64)
    forces = [np.where(cw > 0, 0.0, f) for f in w.forces(b, n_steps=2)]
    _say(f"case: contacts fused, {w.name} ({b.n_cells} cells), 2 steps x K = {w.n_pd_iters}")
    xg, _ = _run_gpu(lib_types(), b, b.v0, forces, w.n_pd_iters, "fused", 32, (cp, cw))
    srng = np.random.default_rng(10)
    cells = np.unique(np.concatenate([srng.choice(b.n_cells, 20, replace=False),
                                      [0, b.n_cells - 1]])).astype(np.int64)
    ot = oracle_types()
    x, v = b.x0.copy(), b.v0.copy()
    for f in forces:
        x, v = O.step_batch(ot, b.types, b.offsets, x, v, f, w.n_pd_iters, cells=cells,
                            contact_p=cp, contact_w=cw)
    err = cell_errors(b.types, b.offsets, xg, x, cells)
    _say(f"contacts full size: sampled {len(cells)} cells, max err/diam {err.max():.3e}")
    assert err.max() <= 1e-5
