"""The oracle reproduces its committed fixture (regression guard), and the
fixture itself satisfies what the paper fixes for Y+Y (ranks halve, the
discarded singular values are at rounding level)."""
import json
import math
import os

import numpy as np

import oracle as O
import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_yy_small_fixture():
    g = json.load(open(os.path.join(HERE, "yy_small_round.json")))
    assert g["input_ranks"] == [1, 10, 10, 10, 1]
    d = synth.yy_small()
    X = O.add(1.0, d["Y"], 1.0, d["Y"])
    for direction in ("RLR", "LRL"):
        Xt, info = O.round_tt(X, d["tol"], direction, return_info=True)
        assert O.ranks(Xt) == g[direction]["ranks"] == [1, 5, 5, 5, 1]
        assert math.isclose(info["norm"], g[direction]["norm"], rel_tol=1e-13)
        for s, sg in zip(info["sigmas"], g[direction]["sigmas"]):
            s, sg = np.asarray(s), np.asarray(sg)
            assert np.allclose(s[:5], sg[:5], rtol=1e-12)
            assert np.all(sg[5:] < 1e-13 * sg[0])   # duplicated directions carry no content
