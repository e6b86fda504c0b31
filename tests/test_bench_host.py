"""Host logic of bench.py and the sweep driver (no GPU): the multi-GPU refusal, the guard on
recorded traffic (kernel sources must hash to the profiled ones; other options get none),
the sweep judgement (shape-sensitive cases, fastest path within |dD| <= 0.01), and the
per-case steady test over consecutive windows."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def test_recorded_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    rec = {"kernel": "k", "workload": "droplet_shear_8x8x8", "sources": ["k.hip"],
           "sha256": hashlib.sha256(b"kernel v1\n").hexdigest(), "bytes_per_step": 123}
    (tmp_path / "profiles" / "k_fused3_droplet_8x8x8.md").write_text("# x\n\ntraffic-record " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    got = bench.recorded_traffic("droplet_shear_8x8x8", 3)
    assert got is not None and got["bytes_per_step"] == 123
    assert bench.recorded_traffic("droplet_shear_8x8x8", 3, default_options=False) is None
    assert bench.recorded_traffic("droplet_shear_8x8x8", 1) is None      # no record for that path
    assert bench.recorded_traffic("droplet_shear_16x8x8", 3) is None     # other workload
    src.write_text("kernel v2\n")
    assert bench.recorded_traffic("droplet_shear_8x8x8", 3) is None      # the kernel changed


def test_sweep_judgement():
    plain = {"D": np.array([0.10, 0.20, 0.30, 0.40, 0.05]), "steady_step": np.array([900, 800, -1, 700, 600]),
             "wall_s": 70.0}
    # case 3 is shape-sensitive (the chained body takes the other branch); case 2 never
    # became steady in the plain sweep
    cold = {"D": np.array([0.10, 0.2005, 0.9, 0.47, 0.05]), "wall_s": 27.0}
    surrogate = np.array([0.105, 0.23, 0.3, 0.4, 0.05])
    J = bench.sweep_judgement(plain, cold, {"surrogate_with_fallback": (20.0, surrogate),
                                            "batched_cold": (cold["wall_s"], cold["D"])})
    assert J["shape_sensitive"].tolist() == [False, False, False, True, False]
    assert J["valid"].tolist() == [True, True, False, False, True]
    assert J["within"]["batched_cold"] == 1.0
    assert abs(J["within"]["surrogate_with_fallback"] - 2 / 3) < 1e-12   # case 1 is off by 0.03
    assert J["best"] == (27.0, "batched_cold")                           # fastest path within 0.01
    assert abs(J["within_all_steady"]["batched_cold"] - 0.75) < 1e-12
    # nothing faster qualifies: the plain sweep answers itself
    J2 = bench.sweep_judgement(plain, cold, {"batched_cold": (27.0, cold["D"] + 0.02)})
    assert J2["best"] == (70.0, "plain")


class _StubLattice:
    """Stands in for a lattice in the per-case sweep loop: D(t) follows a prescribed
    sequence, sampled once per `every` steps."""

    def __init__(self, seq):
        self.seq, self.k = seq, 0

    def autotune(self, reps=1):
        return {}

    def step_status(self, n):
        self.k += 1
        return 0

    def diagnostics(self):
        return {"D": self.seq[min(self.k, len(self.seq)) - 1]}

    def close(self):
        pass


class _StubLb:
    def __init__(self, seqs):
        self.seqs = list(seqs)

    def from_workload(self, wl):
        return _StubLattice(self.seqs.pop(0))


def test_per_case_steady_test_over_consecutive_windows(monkeypatch):
    """D(t) with a plateau (a slow extremum of the transient) before it moves on: one window
    of two samples is met on the plateau, two consecutive windows are not, and both are met
    once D has settled."""
    import types

    from paper_1406_2686_amd import surrogate as sg

    torch_stub = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    monkeypatch.setitem(sys.modules, "torch", torch_stub)
    plateau = [0.10, 0.12, 0.13, 0.13, 0.13, 0.15, 0.18, 0.20, 0.20, 0.20, 0.20, 0.20, 0.20]
    one = sg.solve_plain(_StubLb([plateau]), [None], every=100, window=200, tol=1e-3, max_steps=5000,
                         autotune=False, windows=1)
    two = sg.solve_plain(_StubLb([plateau]), [None], every=100, window=200, tol=1e-3, max_steps=5000,
                         autotune=False, windows=2)
    # one window: samples 3 and 5 (t = 300, 500) agree -> steady at t = 500, D = 0.13
    assert one["steady_step"][0] == 500 and one["D"][0] == 0.13
    # two windows: samples t - 400, t - 200, t all agree only from t = 1200 on
    assert two["steady_step"][0] == 1200 and two["D"][0] == 0.20
    # never settling: not steady (-1) after max_steps
    ramp = [0.01 * k for k in range(1, 80)]
    r = sg.solve_plain(_StubLb([ramp]), [None], every=100, window=200, tol=1e-3, max_steps=3000,
                       autotune=False, windows=2)
    assert r["steady_step"][0] == -1
