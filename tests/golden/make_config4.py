"""Write the FP64 oracle's results at d=2, D=8, chi=256 (seed 0):

* config4_oracle.json: per-site and per-bond energies after the first CTM
  iteration (the bootstrap; its left and up moves use standard isometries
  by the shape rule) and after one more left move of the reduced method;
* spectra_D8_chi256.txt: the singular values of the two large truncation
  inputs of the first reduced insertion after that iteration, for anchor a:
  the side product L = C1 T1 reshaped (chi D) x (D chi) and the row M' =
  C'1 T'2 C'2 reshaped the same way (both 2048 x 2048, truncated to 256).
  GPU kernel tests build matrices with these spectra.

Calls only oracle/ and synth/; run from the repository root (tens of
minutes on 8 cores; the oracle at this size needs about 20 GB of memory):
    python tests/golden/make_config4.py [D chi]
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import oracle.ctm as OC  # noqa: E402
from synth import site_tensors  # noqa: E402


def main(D=8, chi=256):
    A, B = site_tensors(2, D, 0)
    t0 = time.time()
    out = {"d": 2, "D": D, "chi": chi, "seed": 0, "method": "reduced", "results": {}}
    env = O.init_env(A, B)
    env = O.ctm_iteration(env, A, B, chi, O.REDUCED)
    e, eb = O.energy(env, A, B)
    out["results"]["iteration1"] = {"e_site": e, "e_bond": eb}
    print(f"iteration 1: e_site {e:.15f} ({time.time() - t0:.0f} s)", flush=True)
    # truncation inputs of the next (reduced) left insertion, anchor a
    fenv = OC.frame_env(env, 0)
    sites = {"a": OC.rotate_site(A, 0), "b": OC.rotate_site(B, 0)}
    assert not OC.insertion_is_standard(fenv, sites, "a", O.REDUCED, chi)
    _, _, parts = OC.anchor_reduced(fenv, sites, "a", chi, return_parts=True)
    L = parts["L"]
    Mp = parts["Mp"]
    sL = np.linalg.svd(L.reshape(L.shape[0] * D, D * L.shape[3]), compute_uv=False)
    sM = np.linalg.svd(Mp.reshape(Mp.shape[0] * D, D * Mp.shape[3]), compute_uv=False)
    with open(os.path.join(HERE, f"spectra_D{D}_chi{chi}.txt"), "w") as f:
        f.write(f"# singular values (descending) of the truncation inputs L and M' of anchor a,\n"
                f"# first reduced left insertion after one CTM iteration, d=2 D={D} chi={chi} seed 0\n"
                f"# written by tests/golden/make_config4.py from the oracle; columns: L M'\n")
        for a, b in zip(sL, sM):
            f.write(f"{a:.6e} {b:.6e}\n")
    print(f"spectra written ({time.time() - t0:.0f} s)", flush=True)
    env = O.move(env, A, B, 0, chi, O.REDUCED)
    e, eb = O.energy(env, A, B)
    out["results"]["iteration1_left"] = {"e_site": e, "e_bond": eb}
    print(f"iteration 1 + left move: e_site {e:.15f} ({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, f"config_D{D}_chi{chi}_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    if len(sys.argv) == 3:
        main(int(sys.argv[1]), int(sys.argv[2]))
    else:
        main()
