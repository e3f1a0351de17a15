"""CPU checks of the C-ABI: the library loads, exports every symbol the
headers declare, and its host-side logic (argument validation, workspace
sizing, error codes) behaves; no call here reaches a GPU."""

import ctypes
import os
import re
import subprocess
import sys

import pytest

import paper_2306_08212_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names.update(re.findall(r"\b(ctm_\w+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        from paper_2306_08212_amd import build
        build.build()
    return P.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(P.EXPORTS) <= names


def test_workspace_size_validation(lib):
    good = P.Config(d=2, D=2, chi=8)
    assert P.workspace_size(good) > 0
    bad = [P.Config(d=1), P.Config(D=0), P.Config(chi=0), P.Config(method=7),
           P.Config(precision=3), P.Config(boot_iters=-1), P.Config(svd_cutoff=-1.0),
           P.Config(svd_cutoff=1.0),
           # chi below D^2: the initial traced-boundary bonds would not fit
           P.Config(D=3, chi=8), P.Config(D=2, chi=3), P.Config(D=8, chi=63),
           # chi' and chi'' below chi (0 means chi)
           P.Config(chi=8, chi_p=4), P.Config(chi=8, chi_pp=7), P.Config(chi_p=-1)]
    for cfg in bad:
        c = cfg.to_c()
        assert lib.ctm_workspace_size(ctypes.byref(c)) == 0, cfg
    assert lib.ctm_workspace_size(None) == 0


def test_workspace_size_grows_with_sizes(lib):
    sizes = [P.workspace_size(P.Config(d=2, D=D, chi=chi)) for D, chi in
             [(2, 4), (2, 8), (2, 16), (3, 9), (3, 36), (4, 64)]]
    assert sizes[0] < sizes[1] < sizes[2]
    assert sizes[3] < sizes[4] < sizes[5]
    # a larger chi' or chi'' needs more workspace
    assert P.workspace_size(P.Config(D=3, chi=18, chi_p=36)) > P.workspace_size(P.Config(D=3, chi=18))
    assert P.workspace_size(P.Config(D=3, chi=18, chi_pp=36)) > P.workspace_size(P.Config(D=3, chi=18))
    # FP32 / BF16 chains never need more than FP64
    for prec in (P.FP32, P.BF16):
        assert P.workspace_size(P.Config(D=4, chi=64, precision=prec)) <= \
            P.workspace_size(P.Config(D=4, chi=64, precision=P.FP64))
    # the headline size fits comfortably in one MI355X (288 GB)
    assert P.workspace_size(P.Config(D=8, chi=256, precision=P.FP32)) < 40e9


def test_init_rejects_bad_arguments_before_any_device_work(lib):
    A = (ctypes.c_double * (2 * 16))()
    h = ctypes.c_void_p()
    cfg = P.Config(d=2, D=2, chi=8)
    need = P.workspace_size(cfg)
    fake = 0x10000   # never dereferenced: the size check comes first
    c = cfg.to_c(0, fake, need - 1)
    assert lib.ctm_init(ctypes.byref(c), A, A, 0, ctypes.byref(h)) == P.CTM_ENOMEM
    c = cfg.to_c(0, 0, need)
    assert lib.ctm_init(ctypes.byref(c), A, A, 0, ctypes.byref(h)) == P.CTM_EINVAL
    c = cfg.to_c(0, fake, need)
    assert lib.ctm_init(ctypes.byref(c), None, A, 0, ctypes.byref(h)) == P.CTM_EINVAL
    assert lib.ctm_init(ctypes.byref(c), A, A, 0, None) == P.CTM_EINVAL
    bad = P.Config(d=2, D=2, chi=0).to_c(0, fake, need)
    assert lib.ctm_init(ctypes.byref(bad), A, A, 0, ctypes.byref(h)) == P.CTM_EINVAL
    # chi < D^2 is refused before any device work
    bad = P.Config(d=2, D=2, chi=3).to_c(0, fake, need)
    assert lib.ctm_init(ctypes.byref(bad), A, A, 0, ctypes.byref(h)) == P.CTM_EINVAL
    assert P.workspace_size(P.Config(d=2, D=2, chi=4)) > 0


def test_null_solver_calls(lib):
    for f, args in [(lib.ctm_move, (None, 0)), (lib.ctm_iterate, (None, 1)),
                    (lib.ctm_converge, (None, 1, 1e-6, None, None)),
                    (lib.ctm_energy, (None, None, None, None)),
                    (lib.ctm_get_env, (None, 0, None, 0, None, None)),
                    (lib.ctm_set_env, (None, 0, None, 1, 1)),
                    (lib.ctm_set_precision, (None, 0)), (lib.ctm_set_graphs, (None, 1)),
                    (lib.ctm_profile, (None, 1)),
                    (lib.ctm_profile_read, (None, 0, None, None, None, None))]:
        assert f(*args) == P.CTM_EINVAL
    assert lib.ctm_moves_done(None) == -1
    lib.ctm_destroy(None)


def test_status_strings(lib):
    seen = set()
    for st in range(6):
        s = P.status_string(st)
        assert s and s not in seen
        seen.add(s)
    assert "unknown" in P.status_string(99)
    # a Jacobi SVD that did not converge is reported as a numeric failure
    assert "SVD" in P.status_string(P.CTM_ENUMERIC)


def test_kernel_entry_validation(lib):
    assert lib.ctm_kernel_tsvd_workspace(0, 4, 4) == 0
    assert lib.ctm_kernel_tsvd_workspace(64, 64, 8) > 0
    assert lib.ctm_kernel_tsvd_workspace(2048, 2048, 256) > lib.ctm_kernel_tsvd_workspace(256, 256, 64)
    assert lib.ctm_kernel_gemm(5, 1, 1, 1, 1.0, None, 1, 0, None, 1, 0, 0.0, None, 1, None) == P.CTM_EINVAL
    assert lib.ctm_kernel_gemm(0, -1, 1, 1, 1.0, 1, 1, 0, 1, 1, 0, 0.0, 1, 1, None) == P.CTM_EINVAL
    assert lib.ctm_kernel_tsvd(None, 4, 4, 2, 0.0, None, None, None, 0, None) == P.CTM_EINVAL
    dims = (ctypes.c_int64 * 2)(3, 4)
    perm = (ctypes.c_int * 2)(0, 0)      # not a permutation
    assert lib.ctm_kernel_permute(0, 1, 2, dims, perm, 0, 1, 1.0, None) == P.CTM_EINVAL


def test_env_index_layout():
    assert P.env_index("C1a") == 0 and P.env_index("C1b") == 1
    assert P.env_index("C4b") == 7 and P.env_index("T1a") == 8 and P.env_index("T4b") == 15
    assert [P.env_index(n) for n in P.ENV_NAMES] == sorted(P.env_index(n) for n in P.ENV_NAMES)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
