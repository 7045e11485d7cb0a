"""Host logic of the rocprofv3 condenser: counter scaling by the copy probe,
choice of the finest grid per kernel class, and the kernel-time table."""
import csv
import json

from paper_1012_4307_amd import profile_summary as PS

NAMES = {
    "up": "k_up_rb<float, 8>",
    "down_p": "k_down_rb<float, 4, 1>",
    "down_s": "k_down_rb<float, 4, 2>",
    "down_f64": "k_down_rb<double, 4, 0>",
    "up_f64": "k_up_rb<double, 8>",
}


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, grid, value in rows:
            w.writerow(dict(Kernel_Name=f"void ecs::(anonymous namespace)::{name}(ecs::Grid<float>)",
                            Grid_Size=grid, Counter_Name=counter, Counter_Value=value))


def test_traffic_scales_by_copy_probe_and_takes_finest_grid(tmp_path):
    copy_kib = PS.COPY_BYTES / 1024
    fetch, write = [("k_copy16", 1 << 20, copy_kib / 2)], [("k_copy16", 1 << 20, copy_kib)]
    for q, (cls, name) in enumerate(NAMES.items()):
        # a coarse launch of the same kernel must be ignored
        fetch += [(name, 1000, 1.0), (name, 500000 + q, 100.0 * (q + 1)), (name, 500000 + q, 100.0 * (q + 1))]
        write += [(name, 1000, 1.0), (name, 500000 + q, 10.0 * (q + 1))]
    fe, wr = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fe, "FETCH_SIZE", fetch)
    _counter_csv(wr, "WRITE_SIZE", write)
    algo = {c: 1000 for c in NAMES}
    PS.traffic(str(fe), str(wr), str(tmp_path / "t.txt"), str(tmp_path / "t.json"), "cf", "cw", algo)
    rec = json.loads((tmp_path / "t.json").read_text())
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    assert rec["sources_digest"] == PS.sources_digest()
    assert rec["commands"] == {"fetch": "cf", "write": "cw"}
    for q, (cls, name) in enumerate(NAMES.items()):
        k = rec["kernels"][cls]
        assert k["kernel"] == name and k["grid_threads"] == 500000 + q
        assert k["hbm_bytes_per_launch"] == round((200.0 + 10.0) * (q + 1) * 1024)
    assert set(PS.ALGO_BYTES_PER_NODE) == set(NAMES)


def test_stats_table(tmp_path):
    trace = tmp_path / "k.csv"
    with open(trace, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z",
                                          "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for t0, dur in ((0, 3000), (5000, 5000)):
            w.writerow(dict(Kernel_Name="void ecs::(anonymous namespace)::k_tail<float>(ecs::TailArgs<float>)",
                            Grid_Size_X=1024, Grid_Size_Y=1, Grid_Size_Z=1, Start_Timestamp=t0,
                            End_Timestamp=t0 + dur))
    PS.stats(str(trace), str(tmp_path / "s.txt"), "cmd")
    text = (tmp_path / "s.txt").read_text()
    assert "k_tail<float>" in text and "2 dispatches" in text
    row = next(ln for ln in text.splitlines() if ln.startswith("k_tail"))
    assert row.split()[1:4] == ["1024", "2", "4.00"]


def test_trace_class_average_takes_the_finest_grid_of_the_class():
    """The bench's in-process trace cross-check: kernel events of the class
    (with or without the single right-hand-side template flag) on the largest
    grid are averaged; other grids, other kernels, runtime events and classes
    without a pattern are ignored."""
    def ev(name, grid, dur, cat="kernel", ph="X"):
        return {"ph": ph, "cat": cat, "name": f"void ecs::(anonymous namespace)::{name}(ecs::Grid<float>, int)",
                "dur": dur, "args": {"grid": [grid, 1, 1], "block": [256, 1, 1]}}
    events = [ev("k_up_rb<float, 8, false>", 4632, 25.0), ev("k_up_rb<float, 8, false>", 4632, 27.0),
              ev("k_up_rb<float, 8, false>", 1168, 10.0),          # the 1025^2 level
              ev("k_up_rb<float, 8>", 4632, 26.0),                 # the form without the flag
              ev("k_up_rb<double, 8, false>", 9999, 40.0),         # another class
              ev("k_up_rb<float, 8, false>", 9999, 99.0, cat="cuda_runtime"),
              ev("k_up_rb<float, 8, false>", 9999, 99.0, ph="i")]
    assert PS.trace_class_avg(events, "up") == 26.0
    assert PS.trace_class_avg(events, "up_f64") == 40.0
    assert PS.trace_class_avg(events, "down_p") is None
    assert PS.trace_class_avg(events, "mdot") is None
