"""Writes the stored expected values under tests/golden/ by calling only the oracle.

The paper prints no worked numerical example (its figures read data files that
are not part of the text), so no stored value here is the paper's own; every
value below comes from the FP64 oracle on the seeded small workload
"Y+Y, N=4, I=64, Y ranks 5, tol 1e-10" (rounding, Alg. 2).

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import synth  # noqa: E402


def main():
    d = synth.yy_small()
    Y = d["Y"]
    X = O.add(1.0, Y, 1.0, Y)
    out = {}
    for direction in ("RLR", "LRL"):
        Xt, info = O.round_tt(X, d["tol"], direction, return_info=True)
        out[direction] = {
            "ranks": O.ranks(Xt),
            "norm": info["norm"],
            "delta": info["delta"],
            "sigmas": [[float(v) for v in s] for s in info["sigmas"]],
        }
    out["input_ranks"] = O.ranks(X)
    out["norm_gram"] = O.norm_gram(X)
    out["workload"] = synth.WORKLOADS[0]
    with open(os.path.join(HERE, "yy_small_round.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
