"""The Skalak membrane with its line-searched quasi-Newton step (plain form) on the GPU against
the FP64 oracle: loads where the full step is accepted, and an inflated cell where the line
search halves the step."""
import sys

import numpy as np
import pytest

import npfem_inputs as I
import oracle as O
from _runners import cell_errors, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _types():
    from paper_1911_03062_amd import npfem as N
    inp = I.cell_type_inputs()
    lt = {k: N.CellType(x, t, m.with_membrane("skalak"), I.DT) for k, (x, t, m) in inp.items()}
    ot = {k: O.CellType(x, t, m.with_membrane("skalak"), I.DT) for k, (x, t, m) in inp.items()}
    return lt, ot


@pytest.mark.parametrize("precision", [64, 32])
def test_skalak_plain_mixed_batch(precision):
    lt, ot = _types()
    tids = np.array([I.RBC] * 2 + [I.PLT] * 3, dtype=np.int32)
    b = I.make_batch(tids, seed=190)
    rng = np.random.default_rng(191)
    v0 = rng.normal(0, 0.05, size=b.x0.shape).astype(np.float32).astype(np.float64)
    forces = list(I.force_stream(b, seed=192, sigma=20.0, n_steps=3))
    _say(f"case: Skalak plain FP{precision}, 2 RBC + 3 PLT, 3 steps x K = 10")
    xo, vo = run_oracle(ot, b.types, b.offsets, b.x0, v0, forces, 10)
    xg, vg = run_gpu(lt, b.types, b.x0, v0, forces, 10, form="plain", precision=precision)
    err = cell_errors(b.types, b.offsets, xg, xo)
    xp, _ = run_oracle({k: O.CellType(x, t, m, I.DT) for k, (x, t, m) in I.cell_type_inputs().items()},
                       b.types, b.offsets, b.x0, v0, forces, 10)
    sep = cell_errors(b.types, b.offsets, xp, xo)
    _say(f"Skalak plain FP{precision}: max err/diam {err.max():.3e}, Skalak vs PD {sep.min():.3e}")
    assert err.max() <= (1e-10 if precision == 64 else 1e-5)
    assert sep.min() > 100 * err.max()


@pytest.mark.parametrize("precision", [64, 32])
def test_skalak_inflated_cell_halves_the_step(precision):
    """Cells inflated by 40 % (area strain ~ 1.8): the full quasi-Newton step overshoots and the
    line search halves it (step lengths 1/2 to 1/8); K = 4 iterates against the oracle's."""
    lt, ot = _types()
    b = I.make_batch([I.RBC, I.PLT], seed=193, identity=True)
    x0 = b.x0.copy()
    for c in range(b.n_cells):
        s = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
        x0[:, s] = 1.4 * x0[:, s]
    x0 = x0.astype(np.float32).astype(np.float64)
    v0 = np.zeros_like(x0)
    forces = [np.zeros_like(x0)]
    _say(f"case: Skalak plain FP{precision}, RBC + PLT inflated by 40 %, 1 step x K = 4")
    xo, _ = run_oracle(ot, b.types, b.offsets, x0, v0, forces, 4)
    xg, _ = run_gpu(lt, b.types, x0, v0, forces, 4, form="plain", precision=precision)
    err = cell_errors(b.types, b.offsets, xg, xo)
    # step lengths the oracle's line search takes, per cell and iteration, read off its
    # updates: each is a multiple of the full quasi-Newton step -L^-1 grad g
    steps = []
    for c in range(b.n_cells):
        ct = ot[int(b.types[c])]
        sl_ = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
        xk = x0[:, sl_].T[None].copy()
        y = xk.copy()
        for _ in range(4):
            d = -O.solve(ct, O.gradient(xk, y, ct))
            xn = O.line_search_update(ct, xk, y)
            steps.append(float(np.sum((xn - xk) * d) / np.sum(d * d)))
            xk = xn
    halved = min(steps) < 1.0
    _say(f"Skalak inflated FP{precision}: max err/diam {err.max():.3e}; step lengths {steps}")
    assert halved
    assert err.max() <= (1e-10 if precision == 64 else 1e-5)


def test_skalak_fused_is_unsupported():
    from paper_1911_03062_amd import npfem as N
    lt, _ = _types()
    with pytest.raises(N.NpfemError) as ei:
        N.Batch([lt[I.RBC]], precision=32, form="fused")
    assert ei.value.name == "NPFEM_E_UNSUPPORTED"
