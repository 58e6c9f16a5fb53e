"""Write the oracle's config-1 spectrum used by the GPU parity test.

    python tests/golden/make_oracle_reference.py

Calls only the CPU oracle (package ``oracle``) and the seeded workload
generator; re-run it whenever the oracle's arithmetic changes.  Output:
tests/golden/oracle_config1_cl.npy, C_ell[3][2501] (TT, TE, EE) for the
fiducial cosmology of the 400-mode, 2000-output-time, l <= 2500 workload.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import cmb_workloads as W  # noqa: E402
import oracle as O  # noqa: E402


def main():
    wl = W.config1()
    t0 = time.time()
    r = O.solve(wl.cosmo, wl.prec, wl.k, wl.n_tau, wl.ell_max, True)
    assert np.all(r["status"] == 0)
    np.save(os.path.join(HERE, "oracle_config1_cl.npy"), r["Cl"])
    print(f"wrote oracle_config1_cl.npy in {time.time() - t0:.1f} s; mean steps {r['nsteps'].mean():.1f}")


if __name__ == "__main__":
    main()
