"""Write the oracle reference of the zonal-jet serial SDC workload.

T127 on the 192 x 384 Gaussian grid, SDC with 5 Lobatto nodes and 8 sweeps
per step (the paper's reference SDC(5,8), Sec. 6.1), 20 steps of dt = 60 s,
nu = 1e5 m^2/s, initial condition from tests/_ics.py with seed 2.  Calls only
the oracle and the seeded input generator; the output is
tests/golden/jet_t127_sdc5x8_20x60s.npz with the state after the first step
and the final state (complex128 [3, K]); the initial state is rebuilt by
tests/_ics.py wherever it is needed.

Run from the repository root:  python tests/golden/make_jet_sdc.py
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import sdc, swe  # noqa: E402
from tests._ics import jet_state  # noqa: E402

T, NLAT, NLON, NN, NSWEEP, NSTEP, DT, SEED = 127, 192, 384, 5, 8, 20, 60.0, 2
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "jet_t127_sdc5x8_20x60s.npz")


def main():
    t0 = time.time()
    lv = swe.Level(T, NLAT, NLON)
    sd = sdc.SDC(NN)
    x0 = jet_state(T, NLAT, NLON, SEED)
    x = x0.copy()
    first = None
    for step in range(NSTEP):
        x = sdc.serial_sdc(lv, sd, DT, x, 1, NSWEEP)
        if step == 0:
            first = x.copy()
        print(f"step {step + 1}/{NSTEP} {time.time() - t0:.1f}s", flush=True)
    np.savez_compressed(OUT, first=first, final=x,
                        meta=np.array([T, NLAT, NLON, NN, NSWEEP, NSTEP, DT, SEED]))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
