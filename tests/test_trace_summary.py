"""The kernel-trace summariser that turns a rocprofv3 kernel trace of the
bench into the tables kept with the profiles (CPU only, synthetic traces)."""

import csv

from paper_2306_08212_amd import trace_summary as T


def _write(tmp_path, rows):
    path = tmp_path / "run_kernel_trace.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp",
                                          "Stream_Id"])
        w.writeheader()
        for name, s, e, sid in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": s, "End_Timestamp": e,
                        "Stream_Id": sid})
    return str(tmp_path)


def test_busy_time_is_the_union_of_intervals():
    ev = [(0, 10, "a", "1"), (5, 20, "b", "2"), (30, 40, "c", "1"), (35, 38, "d", "2")]
    # [0, 20) and [30, 40): 30 ns
    assert abs(T.busy_ms(ev) - 30e-6) < 1e-15
    assert T.busy_ms([]) == 0.0


def test_names_lose_namespaces_templates_and_arguments():
    assert T._name({"Kernel_Name": "void ctm::(anonymous namespace)::gemm_f64_kernel<4>(int, double)"}) \
        == "gemm_f64_kernel"


def test_windows_of_a_bench_trace(tmp_path, capsys):
    # two timed moves with one FP32 chain GEMM each (stream 1) beside a Jacobi
    # round (stream 2), then a profiled pass of one move between gate kernels
    rows = []
    t = 0
    for _ in range(2):
        rows += [("void ctm::gemm_f32_kernel(int)", t, t + 100, 1),
                 ("void ctm::jac_round_kernel(int)", t + 50, t + 300, 2)]
        t += 400
    rows += [("prof_gate_kernel", t, t + 10, 1), ("void ctm::gemm_f32_kernel(int)", t + 20, t + 120, 1),
             ("void ctm::jac_round_kernel(int)", t + 130, t + 180, 1), ("prof_gate_kernel", t + 190, t + 200, 1)]
    d = _write(tmp_path, rows)
    assert T.main([d, "--steps", "2", "--profiled", "1", "--kernel", "jac_round_kernel"]) == 0
    out = capsys.readouterr().out
    assert "2 moves before the profiled pass, 1 FP32 chain GEMMs per move" in out
    # the window runs from the first chain GEMM to the last round's end: 700 ns over 2 moves
    assert "Wall time per move 0.0 ms" in out
    assert "| 2 | 1 | 0.0 | 71 |" in out          # stream 2: 2 x 250 ns of 700 ns
    assert "`jac_round_kernel` in the profiled pass: 1 launches, average 0.05 us." in out
