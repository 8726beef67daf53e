"""Regression record of the oracle on the 32^3 small box (tests/golden)."""
import json
import os

import numpy as np

from oracle import oracle as O
from paper_1910_12979_amd import inputs as I

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "small_box_oracle.json")


def test_small_box_record_unchanged():
    g = json.load(open(GOLD))
    p = I.SMALL_BOX(0)
    alg = O.mac_project(p)
    ref = O.mac_project(p, mode="definition")
    assert alg["cycles"] == g["algorithm_cycles"]
    np.testing.assert_allclose(alg["hist"], g["algorithm_hist"], rtol=1e-6, atol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(ref["phi"]), g["definition_phi_l2"], rtol=1e-12)
    for k, v in g["definition_phi_samples"].items():
        np.testing.assert_allclose(ref["phi"][tuple(int(x) for x in k.strip("()").split(","))], v, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(ref["u"]), g["definition_u_l2"], rtol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(ref["w"]), g["definition_w_l2"], rtol=1e-12)
