"""Write the oracle's regression record for the 32^3 small box.

Calls only the oracle (and the seeded input generator).  The paper prints no
worked example for the projection, so the stored values are the oracle's own
solution of the 32^3 stratified box (periodic x,y, walls in z, H=0.3, 1%
density noise, S = sin(2 pi x) sin(2 pi y) cos(pi z), seed 0), kept to catch
any later change of the solution, the cycle count or the residual history.
Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1910_12979_amd import inputs as I  # noqa: E402


def record():
    p = I.SMALL_BOX(0)
    alg = O.mac_project(p)
    ref = O.mac_project(p, mode="definition")
    idx = [(0, 0, 0), (5, 17, 3), (31, 31, 31), (16, 8, 24)]
    return {
        "workload": "32^3 box, H=0.3, rho noise 0.01, S=sin sin cos, seed 0, V(2,2), rtol 1e-10",
        "algorithm_cycles": alg["cycles"],
        "algorithm_hist": [float(x) for x in alg["hist"]],
        "definition_phi_l2": float(np.linalg.norm(ref["phi"])),
        "definition_phi_samples": {str(k): float(ref["phi"][k]) for k in idx},
        "definition_u_l2": float(np.linalg.norm(ref["u"])),
        "definition_w_l2": float(np.linalg.norm(ref["w"])),
        "sum_abs_f": float(alg["sum_abs_f"]),
    }


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_box_oracle.json")
    with open(out, "w") as fh:
        json.dump(record(), fh, indent=1)
    print("wrote", out)
