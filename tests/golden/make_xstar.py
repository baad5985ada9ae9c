"""Write the converged PWLS reference x* for a seeded scan, using only the CPU oracle.

x* is the minimiser of 1/2 ||y - A x||_W^2 + R(x) over x >= 0 (the paper's reference reconstruction,
obtained there by thousands of FGM iterations with adaptive restart; Section IV-A). The oracle runs
preconditioned projected FGM with gradient restart until both the RMS change over 100 iterations
(< 2e-7 mm^-1, 0.01 HU) and the KKT residual (< 1e-8 relative) are small, or maxit is reached.

Usage: python tests/golden/make_xstar.py {cfg1|cfg2} SEED [MAXIT]
Writes tests/golden/xstar_<cfg>_seed<SEED>.npz (float32 image plus run metadata).
"""
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))

import oracle  # noqa: E402
from paper_1512_04564_amd import synth  # noqa: E402


def main():
    cfg, seed = sys.argv[1], int(sys.argv[2])
    maxit = int(sys.argv[3]) if len(sys.argv) > 3 else 8000
    g = {"cfg1": synth.CFG1, "cfg2": synth.CFG2}[cfg]
    scan = synth.noisy_scan(g, seed, truth=False)
    t0 = time.time()
    x, its, kkt = oracle.xstar(g, scan.y, scan.w, np.zeros((g.ny, g.nx)), maxit=maxit)
    dt = time.time() - t0
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"xstar_{cfg}_seed{seed}.npz")
    np.savez_compressed(out, x=x.astype(np.float32), iterations=its, kkt=kkt, seconds=dt,
                        threads=oracle.num_threads(), potential="hyperbola", delta=1e-4, beta=1024.0)
    print(f"{out}: {its} iterations, kkt {kkt:.3e}, {dt:.0f} s on {oracle.num_threads()} threads")


if __name__ == "__main__":
    main()
