"""Writes small_imag_oracle.json: the CPU FP64 oracle's physical quantities
after the smallest imaginary-time workload (32^3 grid, dx 0.25, dt 0.1 dx^2,
trap (1, 1.4, 2), g 10, normalised Gaussian start, 200 steps).

The paper prints no numeric results for this case, so these values are the
oracle's own (a regression record, pinned only through the oracle's
mathematical checks); they are produced by calling nothing but the oracle.

    python tests/golden/make_small_imag.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1206_1361_amd import inputs  # noqa: E402


def compute():
    w = inputs.SMALL_IMAG
    psi = inputs.initial_state(w)
    oracle.step(psi, w.dx, w.dt, w.omega, w.g, oracle.IMAG, w.steps)
    return oracle.observables(psi, w.dx, w.omega, w.g)


def main():
    w = inputs.SMALL_IMAG
    obs = compute()
    out = {
        "workload": w.description,
        "steps": w.steps,
        "source": "oracle (gpo_step + gpo_observables), FP64",
        "observables": obs,
    }
    with open(os.path.join(HERE, "small_imag_oracle.json"), "w") as f:
        json.dump(out, f, indent=2)
        f.write("\n")


if __name__ == "__main__":
    main()
