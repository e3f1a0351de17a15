"""Write the FP64 oracle's results at d=2, D=8, chi=256 (seed 0):

* config4_oracle.json: per-site and per-bond energies after the first CTM
  iteration (the bootstrap; its left and up moves use standard isometries
  by the shape rule) and after one more left move of the reduced method;
* spectra_D8_chi256.txt: the singular values of the two large truncation
  inputs of the first reduced insertion after that iteration, for anchor a:
  the side product L = C1 T1 reshaped (chi D) x (D chi) and the row M' =
  C'1 T'2 C'2 reshaped the same way (both 2048 x 2048, truncated to 256).
  GPU kernel tests build matrices with these spectra.

With a third argument "gesvd" the oracle's truncations use LAPACK's
gesvd instead of gesdd (an equally valid SVD) and only the energies are
written, to config_D<D>_chi<chi>_oracle_gesvd.json; with "noise" every
matrix the oracle truncates first gets seeded Gaussian noise of Frobenius
norm eps ||M|| (a backward error of one ulp, the class of error any stable
SVD makes), written to ..._oracle_noise.json.  The difference between a
variant and the plain run is how far rounding alone moves the oracle's
results, from which the GPU parity bar at this size is derived (gesvd is
used where it finishes in reasonable time; at D=8 its 16384 x 4096
bootstrap SVDs take hours, so the noise variant stands in).

Calls only oracle/ and synth/; run from the repository root (about 20
minutes on 6 cores at D=8; the oracle at this size needs about 20 GB of
memory):
    python tests/golden/make_config4.py [D chi [gesvd]]
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


def _noisy_truncate(seed=1000):
    rng = np.random.default_rng(seed)
    plain = OC.truncate

    def noisy(M, k, tau=None):
        Mp = M + rng.standard_normal(M.shape) * (2.220446049250313e-16 * np.linalg.norm(M)
                                                 / np.sqrt(M.size))
        return plain(Mp, k) if tau is None else plain(Mp, k, tau)
    return noisy


def main(D=8, chi=256, driver="gesdd"):
    if driver == "noise":
        OC.truncate = _noisy_truncate()
    else:
        OC.SVD_DRIVER = driver
    A, B = site_tensors(2, D, 0)
    t0 = time.time()
    out = {"d": 2, "D": D, "chi": chi, "seed": 0, "method": "reduced", "svd_driver": driver,
           "results": {}}
    env = O.init_env(A, B)
    env = O.ctm_iteration(env, A, B, chi, O.REDUCED)
    e, eb = O.energy(env, A, B)
    out["results"]["iteration1"] = {"e_site": e, "e_bond": eb}
    print(f"iteration 1: e_site {e:.15f} ({time.time() - t0:.0f} s)", flush=True)
    # truncation inputs of the next (reduced) left insertion, anchor a
    fenv = OC.frame_env(env, 0)
    sites = {"a": OC.rotate_site(A, 0), "b": OC.rotate_site(B, 0)}
    assert not OC.insertion_is_standard(fenv, sites, "a", O.REDUCED, chi)
    if driver == "gesdd":
        write_spectra(fenv, sites, D, chi)
        print(f"spectra written ({time.time() - t0:.0f} s)", flush=True)
    env = O.move(env, A, B, 0, chi, O.REDUCED)
    e, eb = O.energy(env, A, B)
    out["results"]["iteration1_left"] = {"e_site": e, "e_bond": eb}
    print(f"iteration 1 + left move: e_site {e:.15f} ({time.time() - t0:.0f} s)", flush=True)
    suffix = "" if driver == "gesdd" else "_" + driver
    with open(os.path.join(HERE, f"config_D{D}_chi{chi}_oracle{suffix}.json"), "w") as f:
        json.dump(out, f, indent=1)


def write_spectra(fenv, sites, D, chi):
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


if __name__ == "__main__":
    if len(sys.argv) >= 3:
        main(int(sys.argv[1]), int(sys.argv[2]), *(sys.argv[3:4]))
    else:
        main()
