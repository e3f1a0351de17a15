"""Write the FP64 oracle's energies at d=2, D=6, chi=144 (seed 0) after one
and two CTM iterations of the reduced method to config3_oracle.json.

Calls only oracle/ and synth/; run from the repository root:
    python tests/golden/make_config3.py
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import site_tensors  # noqa: E402


def main():
    A, B = site_tensors(2, 6, 0)
    out = {"d": 2, "D": 6, "chi": 144, "seed": 0, "method": "reduced", "iterations": {}}
    env = O.init_env(A, B)
    t0 = time.time()
    for it in range(1, 3):
        env = O.ctm_iteration(env, A, B, 144, O.REDUCED)
        e, eb = O.energy(env, A, B)
        out["iterations"][str(it)] = {"e_site": e, "e_bond": eb}
        print(f"iteration {it}: e_site {e:.15f} ({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "config3_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
