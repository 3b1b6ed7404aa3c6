"""Write tests/golden/plate128x96_kn0.1_steady.npz: the oracle's FP64 steady
state of the flat-plate workload (128x96 cells clustered at the plate, 40x40
trapezoid velocities on [-5, 5]^2, air, Ma 0.1, Kn 0.1, 4 levels), converged
to an RMS residual of 1e-8.  Calls only the oracle; about an hour on one
host core.

    python tests/golden/make_plate128x96_steady.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle.solver import Oracle  # noqa: E402


def main(tol=1e-8, max_cycles=150):
    case = wl.config3(precision="fp64")
    o = Oracle(case)
    t0 = time.time()
    for n in range(max_cycles):
        norms = o.step1()
        o.history.append(norms)
        print(n, norms, f"{time.time() - t0:.0f}s", flush=True)
        if np.max(norms) < tol:
            break
        o.advance()
    rho, U, V, T = o.primitive()
    hist = np.array(o.history)
    first_1e6 = int(np.argmax(hist.max(axis=1) < 1e-6))
    out = os.path.join(HERE, "plate128x96_kn0.1_steady.npz")
    np.savez_compressed(out, rho=rho.reshape(case.ny, case.nx), U=U.reshape(case.ny, case.nx),
                        V=V.reshape(case.ny, case.nx), T=T.reshape(case.ny, case.nx), history=hist,
                        cycles_to_1e6=first_1e6, tol=tol)
    print("wrote", out, "cycles to 1e-6:", first_1e6)


if __name__ == "__main__":
    main()
