"""Write the oracle's full-length trace of the finite-molecule workload
(64^3, h 0.2, 8 atoms with s+p projectors, 32 states, LDA exchange, kick
0.01 along z, dt 0.005, 500 ETRS steps) to c2_etrs_500_trace.txt.

The values come from the CPU oracle alone (oracle/), run on the seeded
inputs of paper_1912_07921_amd.workloads (which holds no arithmetic of the
method).  The GPU parity test compares the library's own 500-step run,
in FP64 and in the mixed form, with this trace.

Usage: python tests/golden/make_c2_etrs_trace.py   (about 15 minutes on 8
cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_1912_07921_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "c2_etrs_500_trace.txt")


def main():
    w = W.c2(nsteps=500)
    o = oracle.Oracle(w.spec)
    t = time.perf_counter()
    psi = o.kick(w.psi0, w.kick)
    psi, dip, nrm = o.propagate_etrs(psi, w.vion, w.nsteps, w.dt)
    sec = time.perf_counter() - t
    rho = o.density(psi)
    E = o.energy(psi, w.vion, w.nsteps * w.dt)
    with open(OUT, "w") as f:
        f.write("# Oracle trace of the 64^3 finite-molecule workload "
                "(c2_molecule_64): kick 0.01 z, dt 0.005, 500 ETRS steps.\n")
        f.write("# Written by make_c2_etrs_trace.py from oracle/ only "
                f"({oracle.num_threads()} threads, {sec:.0f} s).\n")
        f.write(f"# energy_end {E:.17e}\n")
        f.write(f"# density_sum_end {rho.sum():.17e}\n")
        f.write("# norms_end " + " ".join(f"{v:.17e}" for v in nrm[-1])
                + "\n")
        f.write("# columns: step  d_x  d_y  d_z  (atomic units, "
                "d = h^3 sum r n)\n")
        for i, d in enumerate(dip):
            f.write(f"{i} {d[0]:.17e} {d[1]:.17e} {d[2]:.17e}\n")
    print(f"wrote {OUT} in {sec:.0f} s")


if __name__ == "__main__":
    main()
