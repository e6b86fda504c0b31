"""FP64 oracle reference for the long runs of the 128 x 64 x 128 viscoelastic droplet in
shear (2R/H = 0.5, G at the mean-field binodal, polymer in the droplet, Ca = 0.2) at one
Deborah number: 20,000 steps, the length the FP32 path is held to 1e-5 relative L2 over.

Writes droplet_long_De<De>.npz next to this file:
  * the fields rho (2), u (3) and C - I (6) after 20,000 steps on every 8th node in x and z
    and every 4th in y (16 x 16 x 16 nodes), stored in FP32 (6e-8 relative, far below the
    1e-5 they are compared at);
  * the diagnostics record (FP64) after 1,000, 2,000, 5,000, 10,000 and 20,000 steps, as
    a JSON string.
Calls only the oracle and the seeded input generator.  Usage:
    python tests/golden/droplet_long_reference.py <De> [steps]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

MARKS = (1000, 2000, 5000, 10000, 20000)


def sample_mask(nx=128, ny=64, nz=128):
    sel = np.zeros((nz, ny, nx), bool)
    sel[::8, ::4, ::8] = True
    return sel.ravel()


def main():
    De = float(sys.argv[1])
    last = int(sys.argv[2]) if len(sys.argv) > 2 else MARKS[-1]
    wl = workloads.droplet_cfg1(De=De, variant="physics")
    o = oracle.from_workload(wl)
    sel = sample_mask()
    diags, s, t0 = {}, 0, time.time()
    for m in MARKS:
        if m > last:
            break
        st = o.step(m - s)
        if st != 0:
            raise SystemExit(f"oracle fault flags {st} at step {m}")
        s = m
        diags[str(m)] = o.diagnostics()
        print(f"De {De:g}: step {m} ({time.time() - t0:.0f} s)", flush=True)
    rho, u, C = o.get_fields()
    cmi = C[:, sel] - np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])[:, None]
    out = os.path.join(HERE, f"droplet_long_De{De:g}.npz")
    np.savez_compressed(out, step=np.int64(s), rho=rho[:, sel].astype(np.float32), u=u[:, sel].astype(np.float32),
                        CmI=cmi.astype(np.float32), diags=json.dumps(diags))
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
