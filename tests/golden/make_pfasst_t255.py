"""Write the oracle reference of the full-size PFASST block.

Two-level PFASST(16, 5, 3, 8, 1/2) of Sec. 5.2 (Algorithm 1) at its full size:
fine T255 on the 384 x 768 Gaussian grid with 5 Lobatto nodes, coarse T127 on
192 x 384 with 3 nodes, 16 time steps of dt = 60 s solved as one block, 8
iterations (the last stopping after its fine sweep), nu = 1e5 m^2/s, initial
state paper_1904_05988_amd.inputs.seeded_state(255, 3) (n^-2 spectra, mean
geopotential, balanced 20 m/s solid body).

Calls only the oracle and the seeded input generator.  The full arrays do not
fit a small fixture, so the file keeps a fixed sample of spectral slots (every
137th slot of the m-major layout plus the zonal modes m = 0, n <= 15) of:
  pred    [16, 3, S]      fine last-node values after the predictor
  last    [7, 16, 3, S]   fine last-node values after step D of iterations 1..7
  first   [3, 16, 3, S]   fine node-0 values (the new initial conditions) after
                          step D of iterations 1, 4 and 7 (index 0, 3, 6)
  final   [16, 3, S]      fine last-node values after the fine sweep of the
                          eighth (last) iteration
  slots   [S]             the sampled slots
  meta    T_f, nlat_f, nlon_f, n_f, T_c, nlat_c, nlon_c, n_c, n_ts, n_iter, dt, seed
The output is tests/golden/pfasst_t255_t127_16x8.npz (about 2.5 MB).

Run from the repository root:  python tests/golden/make_pfasst_t255.py
(about 15 minutes on 8 cores).
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import pfasst, sdc, swe  # noqa: E402
from paper_1904_05988_amd import inputs  # noqa: E402

FINE = (255, 384, 768, 5)
COARSE = (127, 192, 384, 3)
N_TS, N_ITER, DT, SEED = 16, 8, 60.0, 3
FIRST_ITERS = (0, 3, 6)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pfasst_t255_t127_16x8.npz")


def sample_slots(T):
    K = (T + 1) * (T + 2) // 2
    return np.unique(np.concatenate([np.arange(0, K, 137), np.arange(16)]))


def main():
    t0 = time.time()
    lf = swe.Level(*FINE[:3])
    lc = swe.Level(*COARSE[:3])
    th0 = inputs.seeded_state(FINE[0], SEED)
    print(f"levels ready {time.time() - t0:.1f}s", flush=True)
    res = pfasst.run(lf, lc, sdc.SDC(FINE[3]), sdc.SDC(COARSE[3]), DT, th0, N_TS, N_ITER)
    print(f"pfasst done {time.time() - t0:.1f}s", flush=True)
    s = sample_slots(FINE[0])
    last = np.array([a[:, -1][..., s] for a in res.after_iter])
    first = np.array([res.after_iter[k][:, 0][..., s] for k in FIRST_ITERS])
    meta = np.array(list(FINE[:4]) + list(COARSE[:4]) + [N_TS, N_ITER, DT, SEED], dtype=np.float64)
    np.savez_compressed(OUT, pred=res.pred_end[..., s], last=last, first=first,
                        final=res.end_values[-1][..., s], slots=s, meta=meta)
    print("wrote", OUT, f"{time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
