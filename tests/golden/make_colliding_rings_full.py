"""Write oracle values of the full-size three-level colliding-ring problem on sampled cells.

Workload: two rings (R = 1, sigma = 0.1 R) with centres 3R apart on the z
axis, each tilted 15 degrees toward the other, radius perturbations seeds 5
and 6; levels at dx = R/32, R/64, R/128 with 16^3 blocks (finest within 4
sigma: 4776 blocks; level 1 = parents of the finest dilated by a block:
2137; level 0 = 8 sigma tube plus the parents of level 1 dilated by a
block: 992).  For components omega_x and omega_z, 2000 cells of each
Omega_k are drawn (PCG64 seed 51) and phi_k there is evaluated by the
composite oracle in the paper's order (Sec. 3.4): the full psi_0 and psi_1
fields by the oracle's zero-padded FFT over their bounding boxes, the
sampled phi_k by direct sums over every source cell.  Only oracle/ and the
input generator are called.

    python tests/golden/make_colliding_rings_full.py     # about 30 min, ~25 GB of memory
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import composite as C          # noqa: E402
from paper_2010_13213_amd import inputs    # noqa: E402

N_SAMPLE = 2000
COMPONENTS = (0, 2)


def main():
    t0 = time.time()
    p = inputs.colliding_rings(components=COMPONENTS)
    blocks = [lv.blocks for lv in p.levels]
    print("blocks per level", [len(b) for b in blocks], "%.0f s" % (time.time() - t0), flush=True)
    orc = C.CompositeOracle(p.nb, p.dx0, blocks, fft_min_targets=100000)
    print("oracle set up at %.0f s" % (time.time() - t0), flush=True)
    rng = np.random.Generator(np.random.PCG64(51))
    sample = [np.sort(rng.choice(np.nonzero(orc.mask[k])[0], N_SAMPLE, replace=False)) for k in range(3)]
    out = {"n_blocks": np.array([len(b) for b in blocks]), "components": np.array(COMPONENTS)}
    for k in range(3):
        out["sample%d" % k] = sample[k]
    for c in range(len(COMPONENTS)):
        f = [lv.values[c].reshape(-1) for lv in p.levels]
        phi = orc.solve(f, sample=sample)
        for k in range(3):
            out["phi%d_c%d" % (k, c)] = phi[k][sample[k]]
        print("component %d done at %.0f s" % (COMPONENTS[c], time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(HERE, "colliding_rings_full_samples.npz"), **out)
    print("wrote colliding_rings_full_samples.npz in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
