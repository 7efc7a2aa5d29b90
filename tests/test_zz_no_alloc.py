"""The allocation-free contact detection (npfem_detect_contacts_noalloc, a static per-GPU
workspace) against npfem_detect_contacts on the same batches: bitwise the same outputs, on two
calls in a row with the second batch smaller (the shared workspace keeps the first call's
contents), in both precisions, and against the FP64 oracle's contact decisions."""
import sys

import numpy as np
import pytest

import npfem_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

P = I.PACKING


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(batch, x_np, precision, noalloc):
    import torch
    dt = torch.float64 if precision == 64 else torch.float32
    x = torch.tensor(x_np, dtype=dt, device="cuda").contiguous()
    cp = torch.full_like(x, float("nan"))
    cw = torch.full((x.shape[1],), float("nan"), dtype=dt, device="cuda")
    if noalloc:
        batch.detect_contacts_noalloc(x, P["radius"], P["separation"], P["weight"], cp, cw)
    else:
        batch.detect_contacts(x, P["radius"], P["separation"], P["weight"], cp, cw)
    torch.cuda.synchronize()
    return cp.cpu().numpy(), cw.cpu().numpy()


@pytest.mark.parametrize("precision,form", [(32, "fused"), (64, "plain")])
def test_noalloc_detection_matches_allocating_entry_point(precision, form):
    from paper_1911_03062_amd import npfem as N
    inp = I.cell_type_inputs()
    lt = {k: N.CellType(x, t, m, I.DT) for k, (x, t, m) in inp.items()}
    ot = {k: O.CellType(x, t, m, I.DT) for k, (x, t, m) in inp.items()}
    dtype = np.float64 if precision == 64 else np.float32
    # the second call's batch is smaller than the first's
    for n_rbc, n_plt, seed in ((7, 12, 401), (2, 3, 402)):
        tids = np.array([I.RBC] * n_rbc + [I.PLT] * n_plt, dtype=np.int32)
        tids = tids[np.random.default_rng(seed).permutation(len(tids))]
        b = I.packing_batch(tids, seed=seed + 10)
        batch = N.Batch([lt[int(t)] for t in tids], precision=precision, form=form)
        _say(f"case: noalloc detection FP{precision} {form}, {n_rbc} RBC + {n_plt} PLT, "
             f"{b.v_total} vertices")
        pn, wn = _run(batch, b.x0, precision, noalloc=True)
        pa, wa = _run(batch, b.x0, precision, noalloc=False)
        assert np.array_equal(wn, wa)
        assert np.array_equal(pn, pa)
        po, wo, _ = O.pik_contacts(ot, tids, b.offsets, b.x0, P["radius"], P["separation"],
                                   P["weight"], dtype)
        assert np.array_equal(wn.astype(np.float64), wo)
        frac = float(np.mean(wo > 0))
        _say(f"  bitwise equal to npfem_detect_contacts; {frac:.3f} of the vertices in contact")
        assert frac > 0.1


def test_noalloc_detection_rejects_batches_above_its_workspace():
    import torch
    from paper_1911_03062_amd import npfem as N
    inp = I.cell_type_inputs()
    x, t, m = inp[I.RBC]
    rbc = N.CellType(x, t, m, I.DT)
    n = (1 << 19) // len(x) + 1          # one red cell more than 2^19 vertices hold
    batch = N.Batch([rbc] * n, precision=32, form="fused")
    V = batch.vertex_count
    assert V > (1 << 19)
    xs = torch.zeros((3, V), dtype=torch.float32, device="cuda")
    cp = torch.empty_like(xs)
    cw = torch.empty((V,), dtype=torch.float32, device="cuda")
    with pytest.raises(N.NpfemError) as e:
        batch.detect_contacts_noalloc(xs, P["radius"], P["separation"], P["weight"], cp, cw)
    assert e.value.name == "NPFEM_E_UNSUPPORTED"
    assert "524288" in str(e.value)
