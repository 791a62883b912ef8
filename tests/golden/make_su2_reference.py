"""Write tests/golden/su2_landau_oracle.json: the FP64 oracle's Landau-gauge
fix of the 32^4 smooth SU(2) configuration (eps = 0.5, seed 2001),
overrelaxation omega = 1.7, stop at theta < 1e-12 checked every 20 sweeps.
Calls only the oracle and the input generator.

    python tests/golden/make_su2_reference.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1212_5221_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "su2_landau_oracle.json")
DIMS = (32, 32, 32, 32)


def main():
    seed = 2001
    U = I.su2_smooth(DIMS, 0.5, seed)
    F0, th0 = O.su2_measure(U, DIMS, "landau")
    plaq = O.su2_plaquette(U, DIMS)
    t = time.time()
    st, done = O.su2_run(U, DIMS, "landau", "or", omega=1.7, max_sweeps=20000, tol=1e-12, check_every=20)
    el = time.time() - t
    F, th = O.su2_measure(U, DIMS, "landau")
    data = {str(seed): {"seed": seed, "dims": list(DIMS), "eps": 0.5, "omega": 1.7, "tol": 1e-12,
                        "check_every": 20, "status": st, "sweeps": int(done[0]), "F_input": F0,
                        "theta_input": th0, "plaquette": plaq, "F": F, "theta": th,
                        "oracle_seconds": el, "threads": os.environ.get("OMP_NUM_THREADS")}}
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
    print(json.dumps(data[str(seed)]))


if __name__ == "__main__":
    main()
