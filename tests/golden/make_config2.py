"""Write the FP64 oracle's results at d=2, D=4, chi=64 (seed 0) for the
three isometry methods, each run once with LAPACK's gesdd and once with
gesvd as the truncation SVD, to config_D4_chi64_oracle.json:

* standard move, 4 iterations: energies, <S^z> on both sublattices and the
  row correlation S_zz(x), x = 1..4;
* sequential-order (reduced) and reduced-env moves, 2 iterations: energies.

A third run ("noise") uses gesdd after adding seeded Gaussian noise of
Frobenius norm eps ||M|| (one ulp of backward error) to every matrix the
oracle truncates.  The differences between the runs are how far rounding
alone moves the oracle's own answer at this size; the GPU parity tests hold
the library to the larger of ten times the driver spread and a hundred
times the one-ulp spread (a backward-error budget of 100 ulps for the GPU's
truncations), never less than 1e-10 relative.

Calls only oracle/ and synth/; run from the repository root (a few minutes):
    python tests/golden/make_config2.py
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

SZ = np.array([[0.5, 0.0], [0.0, -0.5]])
RUNS = {"standard": (O.STANDARD, 4), "reduced": (O.REDUCED, 2), "reduced_env": (O.REDUCED_ENV, 2)}


def _noisy_truncate(plain, seed=1000):
    rng = np.random.default_rng(seed)

    def noisy(M, k, tau=None):
        Mp = M + rng.standard_normal(M.shape) * (2.220446049250313e-16 * np.linalg.norm(M)
                                                 / np.sqrt(M.size))
        return plain(Mp, k) if tau is None else plain(Mp, k, tau)
    return noisy


def main():
    A, B = site_tensors(2, 4, 0)
    out = {"d": 2, "D": 4, "chi": 64, "seed": 0, "results": {}}
    t0 = time.time()
    plain = OC.truncate
    for driver in ("gesdd", "gesvd", "noise"):
        if driver == "noise":
            OC.SVD_DRIVER = "gesdd"
            OC.truncate = _noisy_truncate(plain)
        else:
            OC.SVD_DRIVER = driver
        res = {}
        for name, (method, iters) in RUNS.items():
            r = O.solve(A, B, 64, method, max_iters=iters)
            rec = {"iterations": iters, "e_site": r["e_site"], "e_bond": r["e_bond"]}
            if name == "standard":
                rec["sz"] = O.expect1(r["env"], A, B, SZ)
                rec["szz"] = O.row_correlation(r["env"], A, B, SZ, 4)
            res[name] = rec
            print(f"{driver} {name}: e_site {r['e_site']:.15f} ({time.time() - t0:.0f} s)", flush=True)
        out["results"][driver] = res
    OC.SVD_DRIVER = "gesdd"
    OC.truncate = plain
    with open(os.path.join(HERE, "config_D4_chi64_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
