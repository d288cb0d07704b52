"""Write oracle values of the three-level colliding-ring problem at quarter size.

Workload: two rings (R = 1, sigma = 0.1 R) with centres 3R apart on the z
axis, each tilted 15 degrees toward the other, radius perturbations seeds 5
and 6; levels at dx = R/8, R/16, R/32 with 8^3 blocks (finest within 4
sigma, level 1 = parents of the finest dilated by a block, level 0 = 8 sigma
tube plus the parents of level 1 dilated by a block).  Same geometry as the
full-size three-level workload (R/32, R/64, R/128 with 16^3 blocks) at a
quarter of its resolution, so the oracle stays affordable.  For components
omega_x and omega_z, 500 cells of each Omega_k are drawn (PCG64 seed 41)
and phi_k there is evaluated by the composite oracle.  Only oracle/ is
called.

    python tests/golden/make_colliding_rings_quarter.py     # a few minutes on 8 cores
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import composite as C          # noqa: E402
from paper_2010_13213_amd import inputs    # noqa: E402

N_SAMPLE = 500


def main():
    t0 = time.time()
    p = inputs.colliding_rings(nb=8, dx0=1.0 / 8, components=(0, 2))
    blocks = [lv.blocks for lv in p.levels]
    orc = C.CompositeOracle(p.nb, p.dx0, blocks)
    rng = np.random.Generator(np.random.PCG64(41))
    sample = [rng.choice(np.nonzero(orc.mask[k])[0], N_SAMPLE, replace=False) for k in range(3)]
    out = {"n_blocks": np.array([len(b) for b in blocks])}
    for k in range(3):
        out["sample%d" % k] = sample[k]
    for c in range(2):
        f = [lv.values[c].reshape(-1) for lv in p.levels]
        phi = orc.solve(f, sample=sample)
        for k in range(3):
            out["phi%d_c%d" % (k, c)] = phi[k][sample[k]]
        print("component %d done at %.0f s" % (c, time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(HERE, "colliding_rings_quarter_samples.npz"), **out)
    print("wrote colliding_rings_quarter_samples.npz in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
