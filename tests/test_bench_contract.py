"""Host checks of the benchmark's contract: the one-GPU guard, the committed counter summary
that its roofline reads (it must describe the current kernel sources), and the packing
placement its packing leg uses."""
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np

import npfem_inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_contract", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_reported_only_for_the_kernel_sources_it_was_measured_on():
    """The roofline's measured traffic comes from the committed counter summary only when that
    summary was taken on the current fused-kernel sources; after a kernel edit it is null until
    new counters are committed."""
    b = _bench_module()
    with open(b.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    assert t["bytes_per_launch"] > t["algorithmic_bytes_per_launch"] > 0
    if t["source_hash"] == b.kernel_source_hash():
        assert b.measured_traffic() == t["bytes_per_launch"]
    else:
        assert b.measured_traffic() is None


def test_packing_placement_box_and_overlaps():
    """Centres uniform in a cube of (sum of nominal volumes / hematocrit)^(1/3); the cells
    interpenetrate (no overlap avoidance): many vertices lie within 1 um of another cell."""
    tids = np.array([I.RBC] * 10 + [I.PLT] * 5, dtype=np.int32)
    b = I.packing_batch(tids, seed=11)
    edge = ((10 * I.NOMINAL_VOLUME[I.RBC] + 5 * I.NOMINAL_VOLUME[I.PLT]) / I.PACKING["hematocrit"]) ** (1 / 3)
    centres = np.array([b.x0[:, b.offsets[c]:b.offsets[c + 1]].mean(axis=1) for c in range(b.n_cells)])
    assert centres.min() > -0.5 and centres.max() < edge + 0.5
    assert centres.max() > 0.6 * edge                       # spread over the box
    again = I.packing_batch(tids, seed=11)
    assert np.array_equal(again.x0, b.x0)                   # seeded
    cell_of = np.repeat(np.arange(b.n_cells), np.diff(b.offsets))
    close = 0
    for c in range(b.n_cells):
        mine = b.x0[:, cell_of == c].T
        other = b.x0[:, cell_of != c].T
        d2 = ((mine[:, None, :] - other[None, :, :]) ** 2).sum(-1)
        close += int((d2.min(axis=1) < 1.0).sum())
    assert close > 0.2 * b.v_total
