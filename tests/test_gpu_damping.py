"""Position-based velocity damping on the GPU (both forms) against the FP64 oracle."""
import sys

import numpy as np
import pytest

import npfem_inputs as I
import oracle as O
from _runners import cell_errors, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

KAPPA = {I.RBC: 0.8, I.PLT: 0.5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _types():
    from paper_1911_03062_amd import npfem as N
    inp = I.cell_type_inputs()
    lt = {k: N.CellType(x, t, m.with_kappa(KAPPA[k]), I.DT) for k, (x, t, m) in inp.items()}
    ot = {k: O.CellType(x, t, m.with_kappa(KAPPA[k]), I.DT) for k, (x, t, m) in inp.items()}
    return lt, ot


@pytest.mark.parametrize("form", ["fused", "plain"])
def test_damped_mixed_batch(form):
    lt, ot = _types()
    tids = np.array([I.RBC] * 5 + [I.PLT] * 9, dtype=np.int32)
    tids = tids[np.random.default_rng(131).permutation(len(tids))]
    b = I.make_batch(tids, seed=131)
    rng = np.random.default_rng(132)
    v0 = rng.normal(0, 0.05, size=b.x0.shape).astype(np.float32).astype(np.float64)
    forces = list(I.force_stream(b, seed=133, sigma=20.0, n_steps=6))
    _say(f"case: {form} damped batch 5 RBC (kappa 0.8) + 9 PLT (0.5), 6 steps")
    xo, vo = run_oracle(ot, b.types, b.offsets, b.x0, v0, forces, 10)
    xg, vg = run_gpu(lt, b.types, b.x0, v0, forces, 10, form=form)
    err = cell_errors(b.types, b.offsets, xg, xo)
    # the damping must matter at this scale: compare with the undamped oracle
    xu, _ = run_oracle({k: O.CellType(x, t, m, I.DT) for k, (x, t, m) in I.cell_type_inputs().items()},
                       b.types, b.offsets, b.x0, v0, forces, 10)
    sep = cell_errors(b.types, b.offsets, xu, xo)
    _say(f"{form} damped: max err/diam {err.max():.3e}; damped vs undamped {sep.min():.3e}")
    assert err.max() <= 1e-5
    assert sep.min() > 100 * err.max()


def test_damped_kicked_step_fused():
    lt, ot = _types()
    b = I.make_batch([I.RBC], seed=141, identity=True)
    rng = np.random.default_rng(142)
    v0 = rng.normal(0, 0.2, size=b.x0.shape).astype(np.float32).astype(np.float64)
    f = [rng.normal(0, 200.0, size=b.x0.shape).astype(np.float32).astype(np.float64)]
    xo, _ = run_oracle(ot, b.types, b.offsets, b.x0, v0, f, 10)
    xg, _ = run_gpu(lt, b.types, b.x0, v0, f, 10)
    err = cell_errors(b.types, b.offsets, xg, xo)[0]
    _say(f"fused damped kicked step: err/diam {err:.3e}")
    assert err <= 1e-7


def _rayleigh_types(alpha, beta, kappa=None):
    from paper_1911_03062_amd import npfem as N
    inp = I.cell_type_inputs()
    def mat(k, m):
        m = m.with_rayleigh(alpha, beta)
        return m.with_kappa(kappa[k]) if kappa else m
    lt = {k: N.CellType(x, t, mat(k, m), I.DT) for k, (x, t, m) in inp.items()}
    ot = {k: O.CellType(x, t, mat(k, m), I.DT) for k, (x, t, m) in inp.items()}
    return lt, ot


@pytest.mark.parametrize("precision,alpha,beta,kappa", [(64, 0.3, 0.05, None), (32, 0.3, 0.05, None),
                                                         (64, 0.0, 0.02, KAPPA)])
def test_rayleigh_plain_mixed_batch(precision, alpha, beta, kappa):
    """Rayleigh damping (M~ solve in the prediction, (beta/h) K e in every gradient) in the
    plain form, alone and with position-based damping, against the oracle."""
    lt, ot = _rayleigh_types(alpha, beta, kappa)
    tids = np.array([I.RBC] * 3 + [I.PLT] * 4, dtype=np.int32)
    tids = tids[np.random.default_rng(170).permutation(len(tids))]
    b = I.make_batch(tids, seed=170)
    rng = np.random.default_rng(171)
    v0 = rng.normal(0, 0.05, size=b.x0.shape).astype(np.float32).astype(np.float64)
    forces = list(I.force_stream(b, seed=172, sigma=20.0, n_steps=4))
    _say(f"case: Rayleigh plain FP{precision}, alpha {alpha}, beta {beta}, kappa {kappa}, "
         f"3 RBC + 4 PLT, 4 steps")
    xo, vo = run_oracle(ot, b.types, b.offsets, b.x0, v0, forces, 10)
    xg, vg = run_gpu(lt, b.types, b.x0, v0, forces, 10, form="plain", precision=precision)
    err = cell_errors(b.types, b.offsets, xg, xo)
    xu, _ = run_oracle({k: O.CellType(x, t, m, I.DT) for k, (x, t, m) in I.cell_type_inputs().items()},
                       b.types, b.offsets, b.x0, v0, forces, 10)
    sep = cell_errors(b.types, b.offsets, xu, xo)
    verr = np.abs(vg - vo).max() / np.abs(vo).max()
    _say(f"Rayleigh plain FP{precision}: max err/diam {err.max():.3e}, v err {verr:.3e}, "
         f"damped vs undamped {sep.min():.3e}")
    if precision == 64:
        assert err.max() <= 1e-10 and verr <= 1e-8
    else:
        assert err.max() <= 1e-5
    assert sep.min() > 100 * err.max()


@pytest.mark.parametrize("alpha,beta,kappa", [(0.5, 0.0, None), (0.3, 0.05, None), (0.0, 0.01, KAPPA)])
def test_rayleigh_fused_mixed_batch(alpha, beta, kappa):
    """The fused form: alpha alone scales the prediction and the mass term; beta adds the
    m M~^-1 product for the prediction and the (beta/h) K e term through the L^-1 product
    (grad_mass and - c e); also with position-based damping (the paper's beta_D = 0.01)."""
    lt, ot = _rayleigh_types(alpha, beta, kappa)
    tids = np.array([I.RBC] * 5 + [I.PLT] * 9, dtype=np.int32)
    tids = tids[np.random.default_rng(176).permutation(len(tids))]
    b = I.make_batch(tids, seed=173)
    rng = np.random.default_rng(174)
    v0 = rng.normal(0, 0.05, size=b.x0.shape).astype(np.float32).astype(np.float64)
    forces = list(I.force_stream(b, seed=175, sigma=20.0, n_steps=4))
    _say(f"case: Rayleigh fused FP32, alpha {alpha}, beta {beta}, kappa {kappa}, 5 RBC + 9 PLT, 4 steps")
    xo, vo = run_oracle(ot, b.types, b.offsets, b.x0, v0, forces, 10)
    xg, vg = run_gpu(lt, b.types, b.x0, v0, forces, 10)
    err = cell_errors(b.types, b.offsets, xg, xo)
    xu, _ = run_oracle({k: O.CellType(x, t, m, I.DT) for k, (x, t, m) in I.cell_type_inputs().items()},
                       b.types, b.offsets, b.x0, v0, forces, 10)
    sep = cell_errors(b.types, b.offsets, xu, xo)
    verr = np.abs(vg - vo).max() / np.abs(vo).max()
    _say(f"Rayleigh fused: max err/diam {err.max():.3e}, v err {verr:.3e}, damped vs undamped {sep.min():.3e}")
    assert err.max() <= 1e-5
    assert sep.min() > 100 * err.max()


def test_viscoelastic_full_size_sampled():
    """The benchmark's viscoelastic leg at full size: 20 000 RBC + 4 000 PLT with Rayleigh
    beta_D = 0.01 and kappa = 0.8 on every cell, autotuned layouts, 2 steps of K = 20; the
    oracle steps sampled cells (including strongly forced ones)."""
    w = I.WORKLOADS["large_24000"]
    b = w.batch()
    forces = list(w.forces(b, n_steps=2))
    lt, ot = _rayleigh_types(0.0, 0.01, {I.RBC: 0.8, I.PLT: 0.8})
    _say(f"case: viscoelastic fused, {w.name} ({b.n_cells} cells), 2 steps x K = {w.n_pd_iters}")
    xg, _ = run_gpu(lt, b.types, b.x0, b.v0, forces, w.n_pd_iters)
    rng = np.random.default_rng(9)
    strong = I.strong_cells(b, w.seed, w.strong_fraction)
    cells = np.unique(np.concatenate([rng.choice(b.n_cells, 20, replace=False), strong[:6],
                                      [0, b.n_cells - 1]])).astype(np.int64)
    xo, _ = run_oracle(ot, b.types, b.offsets, b.x0, b.v0, forces, w.n_pd_iters, cells=cells)
    err = cell_errors(b.types, b.offsets, xg, xo, cells)
    _say(f"viscoelastic full size: sampled {len(cells)} cells, max err/diam {err.max():.3e}")
    assert err.max() <= 1e-5
