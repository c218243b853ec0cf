"""Write the oracle's reference for the adaptive swirl workload run to 40
coarse steps (levels 3-7, 32x32 patches, regrid every 2 coarse steps with
tau_refine = 0.05, tau_coarsen = 0.025).

Calls only the CPU oracle (oracle/) and the seeded input recipes
(workloads/).  Output: swirl_amr_40.npz with the final leaf set (exact), the
final time, the largest |q| and the total mass (cell sums weighted by the
cell area), and a seeded sample of interior values given as (level, ix, iy,
i, j, value).  Takes a few minutes on eight cores.

    python tests/golden/make_swirl_amr_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from workloads import synth as S  # noqa: E402

NCOARSE, EVERY, TAU_R, TAU_C, NSAMPLE = 40, 2, 0.05, 0.025, 40000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "swirl_amr_40.npz")


def main():
    O.build()
    O.set_threads(os.cpu_count() or 1)
    w = S.workload("swirl_amr")
    o = O.from_workload(w)
    dt = w["dt_coarse"]
    t = 0.0
    t0 = time.time()
    for k in range(NCOARSE):
        if k % EVERY == 0 and k > 0:
            o.ghost_fill()
            tags, _ = o.tag(TAU_R, TAU_C)
            o.regrid(o.adapt(tags))
        o.coarse_step(t, dt)
        t = t + dt
        print(f"coarse step {k + 1}/{NCOARSE}: {o.n} leaves, {time.time() - t0:.0f} s", flush=True)
    leaves = o.leaves()
    q = o.interior()[:, 0]
    mx = w["mx"]
    rng = np.random.default_rng(40)
    k = rng.integers(0, len(leaves), NSAMPLE)
    i = rng.integers(0, mx, NSAMPLE)
    j = rng.integers(0, mx, NSAMPLE)
    area = 4.0 ** -leaves[:, 0].astype(np.float64) / (mx * mx)
    np.savez_compressed(OUT, leaves=leaves, t=t, qmax=np.abs(q).max(), mass=(q.sum(axis=(1, 2)) * area).sum(),
                        sample_leaf=leaves[k], sample_i=i.astype(np.int32), sample_j=j.astype(np.int32),
                        sample_value=q[k, j, i])
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
