"""Host tooling that turns rocprofv3 output into the committed summaries
(paper_2605_07612_amd.profiling): the comment-insensitive source hash, the
launch-window statistics of a kernel trace and the calibrated counter means.
CPU only, on small synthetic CSV files written here."""
import csv

import pytest

from paper_2605_07612_amd import profiling as pf


def test_code_text_drops_comments_keeps_literals():
    src = ("int a = b / c; // Heun's \"stage\"\n"
           "/* the paper's /* note */ const char *s = \"x // y /* z */\";\n"
           "char q = '\"', r = '/'; // it's\n"
           "d = *p;   e = 1;\n")
    assert pf.code_text(src) == ("int a = b / c; const char *s = \"x // y /* z */\"; "
                                 "char q = '\"', r = '/'; d = *p; e = 1;")


def test_source_hash_ignores_comments_not_code(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("__global__ void k(float *x) { x[0] = 1.0f; }  // one\n")
    b.write_text("// a different comment\n__global__ void k(float *x) {\n  x[0] = 1.0f;  /* same code */\n}\n")
    c.write_text("__global__ void k(float *x) { x[0] = 2.0f; }\n")
    assert pf.sources_sha256([a]) == pf.sources_sha256([b])
    assert pf.sources_sha256([a]) != pf.sources_sha256([c])
    # the file boundary counts: two files are not their concatenation
    d = tmp_path / "d.hip"
    d.write_text("x")
    e = tmp_path / "e.hip"
    e.write_text("y")
    f = tmp_path / "f.hip"
    f.write_text("x y")
    assert pf.sources_sha256([d, e]) != pf.sources_sha256([f])


def _trace_csv(path, launches):
    """launches: (name, start_ns, duration_ns)"""
    cols = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id", "Kernel_Name",
            "Correlation_Id", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
            "Accum_VGPR_Count", "SGPR_Count", "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z",
            "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, cols)
        w.writeheader()
        for d, (name, t0, ns) in enumerate(launches):
            w.writerow(dict(Kind="KERNEL_DISPATCH", Agent_Id=1, Queue_Id=1, Stream_Id=0, Thread_Id=1, Dispatch_Id=d,
                            Kernel_Id=0, Kernel_Name=name, Correlation_Id=d, Start_Timestamp=t0,
                            End_Timestamp=t0 + ns, LDS_Block_Size=0, Scratch_Size=0, VGPR_Count=0,
                            Accum_VGPR_Count=0, SGPR_Count=0, Workgroup_Size_X=256, Workgroup_Size_Y=1,
                            Workgroup_Size_Z=1, Grid_Size_X=1024, Grid_Size_Y=1, Grid_Size_Z=1))


def test_trace_window(tmp_path):
    # 3 untimed then 2 timed steps of (s1, s2); the CSV is not in start order
    launches = []
    t = 0
    for step in range(5):
        d1, d2 = (300, 400) if step < 3 else (100, 200)
        launches.append(("void f4::s1<float>(int)", t, d1))
        launches.append(("void f4::s2<float>(int)", t + 1000, d2))
        t += 2000
    path = tmp_path / "run_kernel_trace.csv"
    _trace_csv(path, launches[::-1])
    rows = pf.read_trace(path)
    assert [r[0] for r in rows[:2]] == ["f4::s1<float>", "f4::s2<float>"]  # sorted, short names
    stats, span = pf.window_table(rows, r"f4::s", 3, 2)
    assert {s["kernel"]: s["avg_us"] for s in stats} == {"f4::s1<float>": 0.1, "f4::s2<float>": 0.2}
    # from the start of s1 of step 3 (6000 ns) to the end of s2 of step 4 (9200 ns), per step
    assert span == pytest.approx((9200 - 6000) / 2 / 1e3)
    table = pf.trace_table(rows, match=None, top=16)
    assert {s["kernel"]: s["calls"] for s in table} == {"f4::s1<float>": 5, "f4::s2<float>": 5}


def _counter_csv(path, dispatches):
    """dispatches: (name, grid, {counter: value})"""
    cols = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
            "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
            "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, cols, extrasaction="ignore")
        w.writeheader()
        for d, (name, grid, counters) in enumerate(dispatches):
            for cname, v in counters.items():
                w.writerow(dict(Dispatch_Id=d, Grid_Size=grid, Kernel_Name=name, Counter_Name=cname,
                                Counter_Value=v))


def test_counter_summary_calibration(tmp_path):
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    gib = 1 << 30
    # the calibration copy reads 1 GiB, which FETCH_SIZE reports as half (KiB)
    _counter_csv(f, [("__amd_rocclr_copyBuffer", 512, {"FETCH_SIZE": gib / 1024 / 2}),
                     ("f4::k<float>", 4096, {"FETCH_SIZE": 1000.0}),
                     ("f4::k<float>", 4096, {"FETCH_SIZE": 3000.0}),
                     ("f4::other", 64, {"FETCH_SIZE": 7.0})])
    _counter_csv(w, [("__amd_rocclr_copyBuffer", 512, {"WRITE_SIZE": gib / 1024}),
                     ("f4::k<float>", 4096, {"WRITE_SIZE": 500.0}),
                     ("f4::k<float>", 4096, {"WRITE_SIZE": 700.0})])
    recs, scale = pf.counter_summary([(["FETCH_SIZE"], str(f)), (["WRITE_SIZE"], str(w))], r"f4::k<",
                                     ("copyBuffer", gib))
    assert scale["FETCH_SIZE"]["scale"] == pytest.approx(2.0)
    assert scale["WRITE_SIZE"]["scale"] == pytest.approx(1.0)
    assert len(recs) == 1
    r = recs[0]
    assert (r["kernel"], r["grid"], r["dispatches"]) == ("f4::k<float>", 4096, 2)
    assert r["FETCH_SIZE"] == 2000.0 and r["FETCH_SIZE_scaled"] == 4000.0
    assert r["WRITE_SIZE"] == 600.0 and r["WRITE_SIZE_scaled"] == 600.0
