"""Serving loop on the GPU: continuous batching over the fused kernel. Every tracked
session's state after its requests were served in the mix equals the same requests run
alone, within 1e-6 of the cell diameter; all requests complete; latencies are recorded."""
import sys

import numpy as np
import pytest

import npfem_inputs as I

pytestmark = pytest.mark.gpu


def test_serving_results_equal_alone_runs():
    import torch
    from paper_1911_03062_amd import npfem as N
    from paper_1911_03062_amd import serving as S
    types = {k: N.CellType(x, t, m, I.DT) for k, (x, t, m) in I.cell_type_inputs().items()}
    rest = {k: x for k, (x, t, m) in I.cell_type_inputs().items()}
    reqs, sessions = S.poisson_workload(duration_s=1.0, rate=200.0, seed=5, n_min=20, n_max=400)
    print(f"case: serving {len(reqs)} requests, {len(sessions)} sessions", flush=True)
    pool = S.SlotPool(types, rest, hbm_budget_bytes=32 << 20)
    srv = S.StepServer(pool, n_pd_iters=10, sigma=1.0)
    rng = np.random.default_rng(0)
    tracked = [int(s) for s in rng.choice(len(sessions), size=min(6, len(sessions)), replace=False)]
    srv.track = set(tracked)
    stats = srv.run(reqs, sessions)
    assert all(r.done >= 0 for r in reqs)
    summ = S.latency_summary(reqs)
    print(f"serving: {summ}, ticks {len(stats['ticks'])}", flush=True)
    shared = sum(1 for tk in stats["ticks"] if len(tk.requests) > 1)
    for sid in tracked:
        rids = [r.rid for r in reqs if r.session == sid]
        xa, va = S.replay_alone(types, rest, sessions[sid], rids, 10, 1.0)
        xm, vm = srv.finals[sid]
        s = sessions[sid]
        diam = np.concatenate([np.full(s.n_rbc * 258, I.RBC_DIAMETER),
                               np.full(s.n_plt * 66, I.PLT_DIAMETER)])
        err = (np.linalg.norm(xa - xm, axis=0) / diam).max()
        print(f"session {sid}: {len(rids)} requests, {s.n_rbc}+{s.n_plt} cells, "
              f"mix vs alone max diff/diam {err:.3e}", flush=True)
        assert err <= 1e-6
    print(f"ticks shared by more than one request: {shared}", flush=True)
