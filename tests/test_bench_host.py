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
    """Every path is judged on every case the plain sweep brought to steady D, and gated on
    that; shape sensitivity comes from the two plain sweeps alone and is only reported."""
    plain = {"D": np.array([0.10, 0.20, 0.30, 0.40, 0.05]), "steady_step": np.array([900, 800, -1, 700, 600]),
             "wall_s": 70.0}
    # the autotuned plain sweep takes the other branch on case 3; case 2 never became steady
    alt = {"D": np.array([0.10, 0.2001, 0.31, 0.47, 0.05]), "wall_s": 60.0}
    cold = {"D": plain["D"].copy(), "wall_s": 27.0}          # the batch equals the chained plain sweep
    surrogate = np.array([0.105, 0.23, 0.3, 0.4, 0.05])
    J = bench.sweep_judgement(plain, alt, {"surrogate_with_fallback": (20.0, surrogate),
                                           "batched_cold": (cold["wall_s"], cold["D"])})
    assert J["shape_sensitive"].tolist() == [False, False, False, True, False]
    assert J["steady"].tolist() == [True, True, False, True, True]
    assert J["within_all_steady"]["batched_cold"] == 1.0
    assert J["within_all_steady"]["plain_tuned"] == 0.75           # off by 0.07 on case 3: counted
    assert J["within_all_steady"]["surrogate_with_fallback"] == 0.75  # off by 0.03 on case 1
    assert J["within_shape_insensitive"]["plain_tuned"] == 1.0
    assert J["best"] == (27.0, "batched_cold")
    # a batched answer off on the shape-sensitive case does not qualify
    off = cold["D"].copy()
    off[3] = 0.47
    J2 = bench.sweep_judgement(plain, alt, {"batched_cold": (27.0, off)})
    assert J2["within_all_steady"]["batched_cold"] == 0.75 and J2["best"] == (70.0, "plain")
    # with agreeing plain sweeps, the tuned one is the faster qualifying path
    J3 = bench.sweep_judgement(plain, dict(alt, D=plain["D"] + 0.001), {"batched_cold": (80.0, cold["D"])})
    assert J3["best"] == (60.0, "plain_tuned")


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
                         tune="chained", windows=1)
    two = sg.solve_plain(_StubLb([plateau]), [None], every=100, window=200, tol=1e-3, max_steps=5000,
                         tune="chained", windows=2)
    # one window: samples 3 and 5 (t = 300, 500) agree -> steady at t = 500, D = 0.13
    assert one["steady_step"][0] == 500 and one["D"][0] == 0.13
    # two windows: samples t - 400, t - 200, t all agree only from t = 1200 on
    assert two["steady_step"][0] == 1200 and two["D"][0] == 0.20
    # never settling: not steady (-1) after max_steps
    ramp = [0.01 * k for k in range(1, 80)]
    r = sg.solve_plain(_StubLb([ramp]), [None], every=100, window=200, tol=1e-3, max_steps=3000,
                       tune="chained", windows=2)
    assert r["steady_step"][0] == -1
