"""Writes traj_grad_plummer16384.npz: the FP64 oracle's gradient of the
differentiation workload at its full size, for the GPU parity test.

Workload: Plummer sphere N = 16384 (seed 1003), eps 0.01, 200 KDK steps
dt = 1e-3, loss L = sum |x_T - y|^2 with y the seeded perturbed snapshot
(seed 1005).  The oracle integrates the exact FP32 values the GPU starts
from (positions, masses, velocities and y rounded to FP32, widened to FP64)
in FP64 and differentiates by reverse mode, storing every state.

Stored: L, the indices of 1024 sampled bodies, and dL/dx0, dL/dv0 (3
components each) and dL/dm at those bodies, in FP64; SHA-256 digests of the
FP32 inputs so the test can refuse a fixture made from other inputs.
Calls only oracle/ and the seeded generators in ics/ (about 4 minutes on
8 cores).

    python tests/golden/make_traj_grad_plummer16384.py
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import ics  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "traj_grad_plummer16384.npz")


def inputs():
    w = ics.WORKLOADS["adjoint16384"]
    pm, v = ics.plummer(w["n"], w["seed"])
    y = ics.perturbed_snapshot(pm, w["seed"] + 2)
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    return w, f32(pm), f32(v), f32(y)


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    w, pm, v, y = inputs()
    oracle.build(force=False)
    t0 = time.time()
    L, gx, gv, gm = oracle.traj_grad(pm.astype(np.float64), v.astype(np.float64), y.astype(np.float64),
                                     w["eps"], w["dt"], w["steps"])
    idx = ics.sample_targets(w["n"], 1024, w["seed"] + 7)
    np.savez_compressed(OUT, L=np.float64(L), idx=idx, gx=gx[idx], gv=gv[idx], gm=gm[idx],
                        gx_norm=np.linalg.norm(gx), gv_norm=np.linalg.norm(gv), gm_norm=np.linalg.norm(gm),
                        inputs_sha256=np.array(digest(pm, v, y)))
    print(f"wrote {OUT}: L = {L:.12e}, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
