"""Writes tgv128_oracle_samples.txt: the oracle's state after 10 CFL-0.5
S2O4 steps of the 128^3 Taylor-Green vortex (Ma 0.1, Re 1600, Pr 0.72) at
512 seeded sample cells, with the step count, final time and per-component
max |Q|.  Calls only the oracle and the seeded input generators; runs in a
few minutes on 8 cores.  Regenerate after any change to the oracle's
arithmetic."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2207_01173_amd import workloads as W  # noqa: E402

N, STEPS, SAMPLES, SEED = 128, 10, 512, 128


def main():
    p = W.tgv_params(N, ma=0.1, re=1600.0, pr=0.72, cfl=0.5)
    q0 = W.tgv_initial(p)
    q, dt_last = O.step(p, q0, STEPS, 0.0)
    st = O.stats(p, q)
    rng = np.random.Generator(np.random.PCG64(SEED))
    idx = rng.integers(0, N, size=(SAMPLES, 3))
    maxabs = np.abs(q).max(axis=(1, 2, 3))
    out = os.path.join(HERE, "tgv128_oracle_samples.txt")
    with open(out, "w") as f:
        f.write("# Oracle state after %d CFL-0.5 S2O4 steps of the %d^3 TGV (Ma 0.1, Re 1600, Pr 0.72),\n"
                "# written by make_tgv128_samples.py (oracle only).\n" % (STEPS, N))
        f.write("# steps %d\n# dt_last %.17e\n# Ek %.17e\n# eps_com %.17e\n" % (STEPS, dt_last, st["Ek"], st["eps_com"]))
        f.write("# maxabs " + " ".join("%.17e" % v for v in maxabs) + "\n")
        f.write("# columns: iz iy ix rho rhoU rhoV rhoW rhoE\n")
        for iz, iy, ix in idx:
            f.write("%d %d %d " % (iz, iy, ix) + " ".join("%.17e" % v for v in q[:, iz, iy, ix]) + "\n")
    print(out)


if __name__ == "__main__":
    main()
