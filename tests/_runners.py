"""Runners shared by the parity tests: the same seeded inputs through the GPU library and
through the FP64 oracle."""
from __future__ import annotations

import numpy as np

import npfem_inputs as I
import oracle as O


def oracle_types(dt=I.DT):
    return {k: O.CellType(x, t, m, dt) for k, (x, t, m) in I.cell_type_inputs().items()}


def lib_types(dt=I.DT):
    from paper_1911_03062_amd import npfem as N
    return {k: N.CellType(x, t, m, dt) for k, (x, t, m) in I.cell_type_inputs().items()}


def run_gpu(types, type_ids, x0, v0, forces, K, form="fused", precision=32, vol_area=False):
    """Run len(forces) steps on cuda:0; returns (x, v[, vol_area]) as float64 numpy."""
    import torch
    from paper_1911_03062_amd import npfem as N
    b = N.Batch([types[int(t)] for t in type_ids], precision=precision, form=form)
    dt = torch.float64 if precision == 64 else torch.float32
    x = torch.tensor(x0, dtype=dt, device="cuda").contiguous()
    v = torch.tensor(v0, dtype=dt, device="cuda").contiguous()
    va = torch.zeros((len(type_ids), 2), dtype=torch.float64, device="cuda") if vol_area else None
    for f in forces:
        ft = torch.tensor(f, dtype=dt, device="cuda").contiguous()
        b.step(x, v, ft, I.DT, K, vol_area=va)
    b.check()
    out = (x.double().cpu().numpy(), v.double().cpu().numpy())
    if vol_area:
        out = out + (va.cpu().numpy(),)
    return out


def run_oracle(otypes, type_ids, offsets, x0, v0, forces, K, cells=None):
    x, v = x0.copy(), v0.copy()
    for f in forces:
        x, v = O.step_batch(otypes, type_ids, offsets, x, v, f, K, cells=cells)
    return x, v


def cell_errors(type_ids, offsets, xa, xb, cells=None):
    """max over vertices of |xa - xb| / diameter, per listed cell."""
    cells = np.arange(len(type_ids)) if cells is None else np.asarray(cells)
    out = np.empty(len(cells))
    for i, c in enumerate(cells):
        s = slice(int(offsets[c]), int(offsets[c + 1]))
        d = np.linalg.norm(xa[:, s] - xb[:, s], axis=0).max()
        out[i] = d / I.DIAMETER[int(type_ids[c])]
    return out


def cell_displacement(type_ids, offsets, x0, x1, cells):
    out = np.empty(len(cells))
    for i, c in enumerate(cells):
        s = slice(int(offsets[c]), int(offsets[c + 1]))
        out[i] = np.linalg.norm(x1[:, s] - x0[:, s], axis=0).max()
    return out
