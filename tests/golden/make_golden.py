"""Writes the stored expected values under tests/golden/ by running the CPU
oracle (and nothing else) on the seeded workloads. The paper prints no worked
numbers for these networks; these files record the oracle's results so that
GPU tests can compare against them without re-running the slow cases.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path[:0] = [os.path.dirname(os.path.dirname(HERE)), os.path.dirname(HERE)]

import oracle  # noqa: E402
from checks import digest  # noqa: E402
from paper_2306_07212_amd import workloads as wl  # noqa: E402

CASES = {
    "plain_small": (wl.plain_small, False),
    "differentiable_small": (wl.differentiable_small, True),
    "differentiable": (wl.differentiable, True),
}


def main(names):
    for name in names:
        maker, incl = CASES[name]
        net = maker()
        box = wl.cube(net.D)
        r = oracle.extract(net, box.lo, box.hi, include_output=incl)
        out = {
            "workload": net.name, "widths": net.widths, "include_output": incl,
            "box": [box.lo.tolist(), box.hi.tolist()],
            "V": int(r.V), "E": int(r.E), "M": int(r.M),
            "splits": int(r.steps[:, 2].sum()), "keys": int(r.steps[:, 3].sum()),
            "steps": r.steps.tolist(), "min_margin": r.min_margin,
            "digest": digest(r.S, r.edges),
            "source": "oracle/pcx_oracle.c via tests/golden/make_golden.py",
        }
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(out, f)
        print(name, r.V, r.E, out["digest"][:16])


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
