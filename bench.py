"""Benchmark: corner-transfer moves per second on one MI355X.

A step is one directional move (two column insertions) of the reduced
(sequential-order) method, at d = 2, D = 8, chi = 256 by default, with the
absorption chains in FP32 on the matrix cores and the truncation SVDs, norms
and energy in FP64.  The first iteration (the standard-move bootstrap that
grows the traced-boundary bonds to chi) and W warm-up moves run before the
timed region; inputs and environment are resident in HBM throughout.  Moves
are replayed from captured HIP graphs once warm (the library's default).

Prints one JSON line.  Run `python bench.py --help` for the knobs.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks (dense) for the kernel classes that are one kernel
# each; the Jacobi round runs on the FP64 vector ALUs (256 CUs x 4 SIMDs x 16
# lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s)
PEAK = {"gemm_f64": (78.6e12, "TFLOP/s", "mfma"), "gemm_f32": (157.3e12, "TFLOP/s", "mfma"),
        "gemm_bf16": (2.5e15, "TFLOP/s", "mfma"), "permute": (8.0e12, "GB/s", "hbm"),
        "svd_round": (78.6e12, "TFLOP/s", "alu"), "chol": (78.6e12, "TFLOP/s", "alu")}
KERNEL_OF = {"gemm_f64": "gemm_f64_kernel", "gemm_f32": "gemm_f32_kernel",
             "gemm_bf16": "gemm_bf16_kernel", "permute": "permute_ctile_kernel/permute_rows_kernel",
             "svd_round": "jac_round_kernel", "chol": "chol_apply_kernel"}
# HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE, for a
# kernel whose code is the one the counters were taken on; none is listed
# for the current kernels (the roofline's traffic is then null).
TRAFFIC = {}
MOVE_ORDER = (0, 2, 1, 3)     # left, right, up, down


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _roctx():
    """roctxProfilerResume / roctxProfilerPause of the ROCm profiler SDK:
    under `rocprofv3 --selected-regions` they bracket what is recorded (the
    profiled pass, so the trace holds the launches whose durations the HIP
    events measure); otherwise they do nothing.  None when the library is
    absent."""
    import ctypes
    for name in ("librocprofiler-sdk-roctx.so.1", "/opt/rocm/lib/librocprofiler-sdk-roctx.so.1"):
        try:
            lib = ctypes.CDLL(name)
            lib.roctxProfilerResume.argtypes = [ctypes.c_uint64]
            lib.roctxProfilerPause.argtypes = [ctypes.c_uint64]
            return lib
        except (OSError, AttributeError):
            continue
    return None


def f_move(d, D, chi):
    """Flop model of one reduced move (two insertions): per insertion four
    absorption chains (two inside the anchors, two edge updates) of
    2[(2+2d) chi^3 D^3 + 2 d chi^2 D^5] flop each, plus the chi^3 D^2 and
    chi^3 D terms of the anchors and corners (36 and 12 per insertion)."""
    ins = 8 * ((2 + 2 * d) * chi ** 3 * D ** 3 + 2 * d * chi ** 2 * D ** 5) \
        + 36 * chi ** 3 * D ** 2 + 12 * chi ** 3 * D
    return 2.0 * ins


def _oracle_quarter_move(d, D, chi, seed):
    """Seconds for one reduced anchor, one edge absorption chain and two
    corner absorptions of the FP64 oracle (a quarter of a move) from a seeded
    random environment at full bond dimension chi."""
    import numpy as np
    import oracle.ctm as OC
    from synth import site_tensors
    A, B = site_tensors(d, D, seed)
    rng = np.random.default_rng(seed + 1000)
    env = {}
    for k in OC.ENV_KEYS:
        shape = (chi, chi) if k[0] == "C" else (chi, D, D, chi)
        t = rng.standard_normal(shape)
        env[k] = t / np.linalg.norm(t)
    sites = {"a": A, "b": B}
    t0 = time.perf_counter()
    v1, v2 = OC.anchor_reduced(env, sites, "a", chi)
    T1n = OC.absorb_chain(env["T1a"], OC._site_in_T1(A), v1, v2, v1, v2)
    G = np.einsum("jm,mubq->jubq", env["C1a"], env["T2a"], optimize=True)
    G = np.einsum("jubq,jum->mbq", G, v1, optimize=True)
    np.einsum("mbq,mbn->nq", G, v2, optimize=True)
    G4 = np.einsum("mj,pkbm->jkbp", env["C4a"], env["T4a"], optimize=True)
    G4 = np.einsum("jkbp,jkm->mbp", G4, v1, optimize=True)
    np.einsum("mbp,mbn->pn", G4, v2, optimize=True)
    dt = time.perf_counter() - t0
    del T1n
    return dt


def cpu_baseline(d, D, chi, seed=0):
    """The FP64 oracle timed on a bounded sample of the same workload (a
    quarter of a move, see _oracle_quarter_move) with every host thread the
    BLAS uses, and the same sample on one thread; moves/s = 1 / (4 t)."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count() or 1
    dt = _oracle_quarter_move(d, D, chi, seed)
    dt1 = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            dt1 = _oracle_quarter_move(d, D, chi, seed)
    return {"value": 1.0 / (4.0 * dt), "unit": "moves/s", "cores": int(cores),
            "kind": "oracle",
            "value_1_thread": (1.0 / (4.0 * dt1)) if dt1 else None,
            "sample": f"one reduced anchor + one edge chain + two corner absorptions "
                      f"(1/4 move) at d={d}, D={D}, chi={chi} from a seeded random "
                      f"full-rank environment, FP64 NumPy: {dt:.1f} s on {cores} threads, "
                      f"{dt1:.1f} s on 1 thread; moves/s = 1/(4 t)" if dt1 else
                      f"one reduced anchor + one edge chain + two corner absorptions "
                      f"(1/4 move) at d={d}, D={D}, chi={chi}, FP64 NumPy, {dt:.1f} s"}


def method_comparison(d=2, D=4, chi=64, moves=8, oracle_moves=1, seed=0):
    """Time per move of the three isometry methods at one size, FP64 on the
    GPU (graph replay, after the bootstrap iteration and a warm-up
    iteration) and in the oracle (one move after the bootstrap, on the
    host's BLAS threads): the analogue of the paper's timing comparison of
    standard, reduced-env and sequential-order CTM (Sec. V, Fig. 7)."""
    import numpy as np
    import torch
    import oracle as O
    import paper_2306_08212_amd as P
    from synth import site_tensors
    A, B = site_tensors(d, D, seed)
    out = {"workload": f"d={d}, D={D}, chi={chi}, FP64, one directional move", "gpu_ms": {},
           "oracle_ms": {}}
    for name, pm, om in (("standard", P.STANDARD, O.STANDARD), ("reduced_env", P.REDUCED_ENV,
                          O.REDUCED_ENV), ("sequential", P.REDUCED, O.REDUCED)):
        s = P.Solver(P.Config(d=d, D=D, chi=chi, method=pm, precision=P.FP64), A, B)
        s.iterate(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(moves):
            s.move(MOVE_ORDER[s.moves_done % 4])
        torch.cuda.synchronize()
        out["gpu_ms"][name] = 1e3 * (time.perf_counter() - t0) / moves
        s.close()
        env = O.ctm_iteration(O.init_env(A, B), A, B, chi, om)
        t0 = time.perf_counter()
        for i in range(oracle_moves):
            env = O.move(env, A, B, MOVE_ORDER[i % 4], chi, om)
        out["oracle_ms"][name] = 1e3 * (time.perf_counter() - t0) / oracle_moves
        log(f"bench: method {name}: gpu {out['gpu_ms'][name]:.2f} ms/move, "
            f"oracle {out['oracle_ms'][name]:.0f} ms/move")
    return out


def _breakdown(results):
    """Per-(D, chi band) solve count, p50 latency and mean iterations."""
    import numpy as np
    groups = {}
    for r in results:
        if r.status != "ok":
            continue
        band = "chi<=64" if r.chi <= 64 else ("chi<=144" if r.chi <= 144 else "chi<=256")
        groups.setdefault(f"D={r.D},{band}", []).append(r)
    out = {}
    for k in sorted(groups):
        lat = sorted(x.latency for x in groups[k])
        out[k] = {"solves": len(lat), "p50_s": float(np.median(lat)),
                  "mean_iters": float(np.mean([x.iters for x in groups[k]]))}
    return out


def serve_stream(args):
    """Serving: the stream of independent solves of the serving workload --
    D uniform in {3..dmax}, chi uniform in [D^2, min(4 D^2, 256)], FP32
    chains, each until delta < tol or max_iters iterations.  First all
    requests at t = 0 (closed loop) for the saturated rate mu, then a seeded
    Poisson stream at 0.8 mu for the latency percentiles; admission by the
    HBM budget (0.8 of free memory) and up to 16 solves in flight."""
    from paper_2306_08212_amd.serve import GpuBackend, Request, Server, summarize
    from synth import serving_stream
    be = GpuBackend()

    def reqs(n, seed, rate):
        out = []
        for q in serving_stream(n, seed, rate, d=args.d, D_min=3, D_max=args.serve_dmax):
            out.append(Request(id=q["id"], d=q["d"], D=q["D"], chi=q["chi"], seed=q["seed"],
                               t_arrival=q["t_arrival"], max_iters=args.serve_iters,
                               tol=args.serve_tol, precision=1))
        return out

    n = args.serve_requests

    def progress(r):
        log(f"bench: served request {r.id} (D={r.D}, chi={r.chi}, {r.iters} iterations, "
            f"{r.latency:.2f} s)")

    res_closed = Server(be, max_slots=16, on_result=progress).run(reqs(n, 7, 0.0))
    closed = summarize(res_closed)
    mu = closed["solves_per_s"] or 1.0
    log(f"bench: serving closed loop {closed}")
    rate = 0.8 * mu
    res_open = Server(be, max_slots=16, on_result=progress).run(reqs(n, 8, rate))
    opened = summarize(res_open)
    log(f"bench: serving open loop at {rate:.2f}/s {opened}")
    return {"workload": f"{n} solves, D uniform in 3..{args.serve_dmax}, chi uniform in "
                        f"[D^2, min(4 D^2, 256)], d={args.d}, FP32 chains, until delta < "
                        f"{args.serve_tol:g} or {args.serve_iters} iterations",
            "closed_loop": closed, "open_loop_rate_per_s": rate, "open_loop": opened,
            "open_loop_by_D_chi": _breakdown(res_open)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8, help="timed moves")
    ap.add_argument("--warmup", type=int, default=8,
                    help="untimed moves after the bootstrap (a move is captured into a "
                         "HIP graph the second time its direction comes up, so 8 moves "
                         "leave all four directions captured)")
    ap.add_argument("--D", type=int, default=8)
    ap.add_argument("--chi", type=int, default=256)
    ap.add_argument("--d", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=4,
                    help="moves timed again with FP64 chains (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests in each serving stream (the full serving workload is "
                         "512; 0 = skip serving)")
    ap.add_argument("--serve-dmax", type=int, default=8,
                    help="largest D in the serving stream (D uniform in 3..dmax)")
    ap.add_argument("--serve-iters", type=int, default=10,
                    help="iteration cap per solve (the serving workload's own cap is 30; "
                         "10 keeps the default run to a few minutes)")
    ap.add_argument("--serve-tol", type=float, default=1e-6, help="delta that ends a solve")
    ap.add_argument("--no-methods", action="store_true",
                    help="skip the standard / reduced-env / sequential comparison")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--method-sweep", action="store_true",
                    help="only time the three isometry methods (FP64, GPU) at D = 4..8 with the "
                         "paper's chi = 10 (D + 1) and print one JSON line per D, then exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 20 plain device copies of MIB MiB through the library's "
                         "permute kernel (identity permutation) and exit: the reference for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only; --gpus {args.gpus} is not "
              f"supported (independent environment solves would shard across GPUs by request)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2306_08212_amd as P
    from synth import site_tensors

    lib = P.load()   # fails loudly if libctm.so is missing
    torch.cuda.set_device(0)
    if args.method_sweep:
        for Dm in range(4, 9):
            chim = 10 * (Dm + 1)
            row = {"D": Dm, "chi": chim, "gpu_ms_per_move": {}}
            Am, Bm = site_tensors(args.d, Dm, args.seed)
            for name, pm in (("standard", P.STANDARD), ("reduced_env", P.REDUCED_ENV),
                             ("sequential", P.REDUCED)):
                sm = P.Solver(P.Config(d=args.d, D=Dm, chi=chim, method=pm, precision=P.FP64),
                              Am, Bm)
                sm.iterate(1)
                for i in range(4):
                    sm.move(MOVE_ORDER[sm.moves_done % 4])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for i in range(4):
                    sm.move(MOVE_ORDER[sm.moves_done % 4])
                torch.cuda.synchronize()
                row["gpu_ms_per_move"][name] = 1e3 * (time.perf_counter() - t0) / 4
                sm.close()
                log(f"bench: D={Dm} chi={chim} {name}: {row['gpu_ms_per_move'][name]:.1f} ms/move")
            print(json.dumps(row), flush=True)
        # the headline size, mixed precision: the two reduced methods
        row = {"D": 8, "chi": 256, "precision": "fp32", "gpu_ms_per_move": {}}
        Am, Bm = site_tensors(args.d, 8, args.seed)
        for name, pm in (("reduced_env", P.REDUCED_ENV), ("sequential", P.REDUCED)):
            sm = P.Solver(P.Config(d=args.d, D=8, chi=256, method=pm, precision=P.FP32), Am, Bm)
            sm.iterate(1)
            for i in range(4):
                sm.move(MOVE_ORDER[sm.moves_done % 4])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(4):
                sm.move(MOVE_ORDER[sm.moves_done % 4])
            torch.cuda.synchronize()
            row["gpu_ms_per_move"][name] = 1e3 * (time.perf_counter() - t0) / 4
            sm.close()
            log(f"bench: D=8 chi=256 fp32 {name}: {row['gpu_ms_per_move'][name]:.1f} ms/move")
        print(json.dumps(row), flush=True)
        return
    if args.copy_probe > 0:
        import ctypes
        n = args.copy_probe * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        dims = (ctypes.c_int64 * 1)(n)
        perm = (ctypes.c_int * 1)(0)
        st = torch.cuda.current_stream().cuda_stream
        for _ in range(20):
            rc = lib.ctm_kernel_permute(0, x.data_ptr(), 1, dims, perm, 0, y.data_ptr(), 1.0, st)
            if rc != 0:
                raise RuntimeError(f"copy probe: status {rc}")
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                          "launches": 20}), flush=True)
        return
    d, D, chi = args.d, args.D, args.chi
    A, B = site_tensors(d, D, args.seed)
    cfg = P.Config(d=d, D=D, chi=chi, method=P.REDUCED, precision=P.PRECISIONS[args.precision])
    log(f"bench: workspace {P.workspace_size(cfg) / 1e9:.2f} GB")
    t0 = time.perf_counter()
    s = P.Solver(cfg, A, B)
    s.iterate(1)
    torch.cuda.synchronize()
    log(f"bench: init + bootstrap iteration {time.perf_counter() - t0:.1f} s")
    for i in range(args.warmup):
        s.move(MOVE_ORDER[s.moves_done % 4])
        torch.cuda.synchronize()
        log(f"bench: warmup move {i + 1}/{args.warmup}")

    def timed(nmoves, tag, profile=False):
        """Wall time of nmoves moves (torch events around the launches, the
        device synchronised on both sides).  With profile=True every kernel
        launch is also bracketed by HIP events on the stream it runs on, for
        the per-class durations, with a short gate kernel ahead of each start
        event (so the interval is the kernel's own duration, not the time
        the host takes to issue it); the moves then run eagerly, so the
        headline number comes from an unprofiled pass."""
        torch.cuda.synchronize()
        rt = _roctx() if profile else None
        if profile:
            s.profile(True)
            if rt is not None:
                rt.roctxProfilerResume(0)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for i in range(nmoves):
            s.move(MOVE_ORDER[s.moves_done % 4])
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        prof = None
        if profile:
            if rt is not None:
                rt.roctxProfilerPause(0)
            prof = s.profile_read()
            s.profile(False)
        log(f"bench: {tag}{' (profiled)' if profile else ''}: {nmoves} moves in {ms:.1f} ms")
        return ms, prof

    ms, _ = timed(args.steps, args.precision)
    moves_per_s = args.steps / (ms / 1e3)
    nprof = max(1, min(args.steps, 4))
    _, prof = timed(nprof, args.precision, profile=True)

    # dominant kernel by summed duration, among the classes that are one kernel
    dom = max((k for k in prof if k in PEAK), key=lambda k: prof[k][1])
    n, kms, kfl, kby = prof[dom]
    peak, unit, bound = PEAK[dom]
    if unit == "TFLOP/s":
        achieved = kfl / (kms / 1e3) / 1e12
        peak_u = peak / 1e12
    else:
        achieved = kby / (kms / 1e3) / 1e9
        peak_u = peak / 1e9
    fm = f_move(d, D, chi)
    # per-class kernel time summed over all streams; share = fraction of the
    # summed kernel time of the profiled moves (the profiled pass itself is
    # stretched by the gate kernels, so its wall time is not the reference)
    total_k = sum(v[1] for v in prof.values())
    breakdown = {k: {"launches": v[0] / nprof, "ms_per_move": v[1] / nprof,
                     "share": v[1] / total_k if total_k > 0 else 0.0}
                 for k, v in prof.items() if v[0]}
    # achieved rates of the classes with an algorithmic count: matrix-core
    # GEMMs in TFLOP/s (fraction of their dtype's dense peak), memory-bound
    # classes in GB/s (fraction of 8 TB/s)
    for k, rec in breakdown.items():
        _, c_ms, c_fl, c_by = prof[k]
        if c_ms <= 0:
            continue
        if k.startswith("gemm") and c_fl > 0:
            tf = c_fl / (c_ms / 1e3) / 1e12
            rec["tflops"] = tf
            rec["frac_of_peak"] = tf / (PEAK[k][0] / 1e12)
        elif k in ("permute", "copy", "reduce") and c_by > 0:
            gbs = c_by / (c_ms / 1e3) / 1e9
            rec["gb_per_s"] = gbs
            rec["frac_of_peak"] = gbs / 8000.0
    gemm_flops = sum(prof[k][2] for k in ("gemm_f64", "gemm_f32", "gemm_bf16")) / nprof
    # the truncation (FP64 SVDs, their QR steps and GEMMs, norms) against
    # the absorption chains (FP32 / BF16 GEMMs and permutes), as shares of
    # the summed kernel time of a move
    trunc_cls = ("gemm_f64", "svd_round", "svd_other", "chol", "reduce")
    trunc_share = sum(prof[k][1] for k in trunc_cls if k in prof) / total_k if total_k else None

    fp64_mps = None
    if args.fp64_steps > 0 and args.precision != "fp64":
        s.set_precision(P.FP64)
        for i in range(8):   # capture the FP64 moves of all four directions
            s.move(MOVE_ORDER[s.moves_done % 4])
        ms64, _ = timed(args.fp64_steps, "fp64")
        fp64_mps = args.fp64_steps / (ms64 / 1e3)
    s.close()

    methods = None
    if not args.no_methods:
        methods = method_comparison(d=d)

    serving = None
    if args.serve_requests > 0:
        serving = serve_stream(args)

    cpu = None
    if not args.no_cpu:
        log("bench: timing the CPU oracle sample")
        cpu = cpu_baseline(d, D, chi, args.seed)

    out = {
        "metric": "CTM moves/s at D=8,chi=256 (mixed vs FP64 plain); p50/p99 solve latency",
        "value": moves_per_s,
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"reduced (sequential-order) CTM move, d={d}, D={D}, chi={chi}, "
                               f"{args.precision} absorption chains, FP64 truncation",
                   "d": d, "D": D, "chi": chi, "method": "reduced",
                   "precision": args.precision},
        "roofline": {"bound": bound, "kernel": KERNEL_OF[dom], "achieved": achieved,
                     "peak": peak_u, "unit": unit, "frac": achieved / peak_u,
                     "traffic": TRAFFIC.get(KERNEL_OF[dom]),
                     "launches_per_move": n / nprof, "avg_launch_us": 1e3 * kms / max(n, 1)},
        "move_model": {"flop_per_move": fm, "move_tflops": fm * moves_per_s / 1e12,
                       "frac_of_fp32_mfma_peak": fm * moves_per_s / 157.3e12,
                       "gemm_flop_per_move_measured": gemm_flops},
        "fp64_moves_per_s": fp64_mps,
        "truncation_share": trunc_share,
        "method_comparison": methods,
        "serving": serving,
        "kernel_breakdown": breakdown,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
