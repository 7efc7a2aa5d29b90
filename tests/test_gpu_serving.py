"""Serving loop on the GPU: continuous batching over the fused kernel. Requests arrive in a
burst (4 000/s for 60 ms, sessions of 20-400 cells) so that many are waiting while earlier
ticks run and are admitted together: every compared session must have run in at least one
tick shared with other sessions, and its state (positions and velocities) after its requests
were served in the mix must equal the same requests run alone, within 1e-6 of the cell
diameter (velocities: 1e-6 of the diameter per time step). All requests complete."""
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
    reqs, sessions = S.poisson_workload(duration_s=0.06, rate=4000.0, seed=5, n_min=20, n_max=400)
    print(f"case: serving burst of {len(reqs)} requests, {len(sessions)} sessions", flush=True)
    pool = S.SlotPool(types, rest, hbm_budget_bytes=32 << 20)
    srv = S.StepServer(pool, n_pd_iters=10, sigma=1.0)
    srv.track = set(sessions)
    stats = srv.run(reqs, sessions)
    assert all(r.done >= 0 for r in reqs)
    ticks = stats["ticks"]
    summ = S.latency_summary(reqs)
    shared = [len(tk.requests) > 1 for tk in ticks]
    print(f"serving: {summ}, ticks {len(ticks)}, shared by more than one request "
          f"{sum(shared)}, largest tick {max(len(tk.requests) for tk in ticks)} requests",
          flush=True)
    assert sum(shared) > 0
    # sessions that ran in a shared tick: compare six of them (seeded choice)
    mixed = sorted({r.session for r in reqs if shared[r.tick]})
    assert len(mixed) >= 6, mixed
    rng = np.random.default_rng(0)
    picked = [int(s) for s in rng.choice(mixed, size=6, replace=False)]
    n_bitwise = 0
    for sid in picked:
        rids = [r.rid for r in reqs if r.session == sid]
        assert any(shared[r.tick] for r in reqs if r.session == sid)
        xa, va = S.replay_alone(types, rest, sessions[sid], rids, 10, 1.0)
        xm, vm = srv.finals[sid]
        s = sessions[sid]
        diam = np.concatenate([np.full(s.n_rbc * 258, I.RBC_DIAMETER),
                               np.full(s.n_plt * 66, I.PLT_DIAMETER)])
        err = (np.linalg.norm(xa - xm, axis=0) / diam).max()
        verr = (np.linalg.norm(va - vm, axis=0) * I.DT / diam).max()
        n_bitwise += int(np.array_equal(xa, xm) and np.array_equal(va, vm))
        print(f"session {sid}: {len(rids)} requests, {s.n_rbc}+{s.n_plt} cells, mix vs alone "
              f"max diff/diam x {err:.3e}, v dt {verr:.3e}", flush=True)
        assert err <= 1e-6 and verr <= 1e-6
    print(f"bitwise identical alone and in the mix: {n_bitwise} of {len(picked)} sessions",
          flush=True)


def test_sessions_moved_out_to_host_memory_keep_their_results():
    """A slot pool far smaller than the sessions' cells (4 MiB: about 530 cells, sessions of
    20-200): idle sessions are moved out to pinned host memory and back; sessions that were
    moved must end as the same requests run alone (within 1e-6 of the diameter)."""
    from paper_1911_03062_amd import npfem as N
    from paper_1911_03062_amd import serving as S
    types = {k: N.CellType(x, t, m, I.DT) for k, (x, t, m) in I.cell_type_inputs().items()}
    rest = {k: x for k, (x, t, m) in I.cell_type_inputs().items()}
    reqs, sessions = S.poisson_workload(duration_s=0.08, rate=3000.0, seed=9, n_min=20, n_max=200)
    print(f"case: serving with moves to host memory, {len(reqs)} requests, "
          f"{len(sessions)} sessions", flush=True)
    pool = S.SlotPool(types, rest, hbm_budget_bytes=4 << 20)
    srv = S.StepServer(pool, n_pd_iters=10, sigma=1.0)
    srv.track = set(sessions)
    stats = srv.run(reqs, sessions)
    assert all(r.done >= 0 for r in reqs)
    moved = sorted(sid for sid, s in sessions.items() if s.moved > 0)
    print(f"moved out {stats['evictions']} times, back {stats['restores']} times; "
          f"{len(moved)} sessions moved", flush=True)
    assert stats["evictions"] > 0 and stats["restores"] > 0 and len(moved) >= 4
    rng = np.random.default_rng(1)
    for sid in [int(s) for s in rng.choice(moved, size=4, replace=False)]:
        rids = [r.rid for r in reqs if r.session == sid]
        xa, va = S.replay_alone(types, rest, sessions[sid], rids, 10, 1.0)
        xm, vm = srv.finals[sid]
        s = sessions[sid]
        diam = np.concatenate([np.full(s.n_rbc * 258, I.RBC_DIAMETER),
                               np.full(s.n_plt * 66, I.PLT_DIAMETER)])
        err = (np.linalg.norm(xa - xm, axis=0) / diam).max()
        verr = (np.linalg.norm(va - vm, axis=0) * I.DT / diam).max()
        print(f"session {sid}: moved {s.moved} times, {len(rids)} requests, mix vs alone "
              f"x {err:.3e}, v dt {verr:.3e}", flush=True)
        assert err <= 1e-6 and verr <= 1e-6
