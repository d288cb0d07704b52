"""Write oracle values of the full-size two-level perturbed ring on sampled cells.

Workload: coarse dx = R/32 ring support (8 sigma, 208 blocks of 16^3), fine
dx = R/64 blocks within 3 sigma of the core perturbed by 32 random modes
(seed 3, max |dR| = 0.01 R), components omega_x and omega_y.  For each level
and component, 600 cells of Omega_k are drawn (PCG64 seed 31) and phi_k is
evaluated there by the composite oracle (every psi and convolution a direct
sum, Sec. 3.4 of the paper).  Only oracle/ is called.

    python tests/golden/make_two_level_ring.py      # about 10 min on 8 cores
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import composite as C          # noqa: E402
from paper_2010_13213_amd import inputs    # noqa: E402

N_SAMPLE = 600


def main():
    t0 = time.time()
    p = inputs.two_level_ring(components=(0, 1))
    blocks = [lv.blocks for lv in p.levels]
    orc = C.CompositeOracle(p.nb, p.dx0, blocks)
    rng = np.random.Generator(np.random.PCG64(31))
    sample = [rng.choice(np.nonzero(orc.mask[k])[0], N_SAMPLE, replace=False) for k in range(2)]
    out = {"sample0": sample[0], "sample1": sample[1],
           "n_blocks0": len(blocks[0]), "n_blocks1": len(blocks[1])}
    for c in range(2):
        f = [lv.values[c].reshape(-1) for lv in p.levels]
        phi = orc.solve(f, sample=sample)
        out["phi0_c%d" % c] = phi[0][sample[0]]
        out["phi1_c%d" % c] = phi[1][sample[1]]
        print("component %d done at %.0f s" % (c, time.time() - t0), flush=True)
    np.savez_compressed(os.path.join(HERE, "two_level_ring_samples.npz"), **out)
    print("wrote two_level_ring_samples.npz in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
