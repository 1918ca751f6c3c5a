"""Host logic of the rocprofv3 summary tool: kernel names, per-dispatch averages
of trace durations and counters, the calibration of HBM bytes against the plain
copy, the SQ ratios, and the comment-blind kernel-source hash bench.py checks."""
import csv
import os

import pytest

from paper_2005_02704_amd import rocprof_summary as rs

GEOM = "void lidarseg::(anonymous namespace)::k_geom<512, 2048>(lidarseg::BatchHeader const*, lidarseg::Workspace)"
CC = "void lidarseg::(anonymous namespace)::k_cc<512, 2048>(lidarseg::BatchHeader const*, lidarseg::Workspace)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_kernel_names():
    assert rs.kname(GEOM) == "k_geom"
    assert rs.kname(CC) == "k_cc"
    assert rs.kname(COPY) == COPY


def test_trace_and_traffic(tmp_path):
    _write(str(tmp_path / "trace" / "x_kernel_trace.csv"),
           [{"Kernel_Name": GEOM, "Start_Timestamp": 0, "End_Timestamp": 100_000},
            {"Kernel_Name": GEOM, "Start_Timestamp": 0, "End_Timestamp": 120_000},
            {"Kernel_Name": CC, "Start_Timestamp": 5, "End_Timestamp": 90_005}])
    by = rs.trace_summary(str(tmp_path / "trace"))
    assert by["k_geom"] == [100_000, 120_000] and by["k_cc"] == [90_000]
    # a 512 MiB copy whose counter reads half the bytes: scale x2; smaller copies are staging
    _write(str(tmp_path / "fetch" / "x_counter_collection.csv"),
           [{"Kernel_Name": COPY, "Grid_Size": 1 << 20, "Counter_Value": 262144.0},
            {"Kernel_Name": COPY, "Grid_Size": 4096, "Counter_Value": 7.0},
            {"Kernel_Name": GEOM, "Grid_Size": 1, "Counter_Value": 1000.0},
            {"Kernel_Name": GEOM, "Grid_Size": 1, "Counter_Value": 3000.0}])
    fb, fcopy = rs.counter_summary(str(tmp_path / "fetch"))
    assert fcopy == [262144.0]
    assert fb["k_geom"] == [1000.0, 3000.0]


def test_sq_summary_and_ratios(tmp_path):
    rows_a, rows_b = [], []
    for rep in (1, 3):   # two dispatches: averages are 2x the base values
        for k in (GEOM, CC):
            rows_a += [{"Kernel_Name": k, "Counter_Name": "SQ_WAVES", "Counter_Value": 100 * rep},
                       {"Kernel_Name": k, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 5000 * rep}]
            rows_b += [{"Kernel_Name": k, "Counter_Name": "SQ_ACTIVE_INST_VALU",
                        "Counter_Value": (76 if k == GEOM else 50) * rep},
                       {"Kernel_Name": k, "Counter_Name": "SQ_BUSY_CU_CYCLES", "Counter_Value": 100 * rep}]
        rows_b.append({"Kernel_Name": COPY, "Counter_Name": "SQ_WAVES", "Counter_Value": 9})
    _write(str(tmp_path / "a" / "x_counter_collection.csv"), rows_a)
    _write(str(tmp_path / "b" / "x_counter_collection.csv"), rows_b)
    by = rs.sq_summary([str(tmp_path / "a"), str(tmp_path / "b")])
    assert set(by) == {"k_geom", "k_cc"}
    assert by["k_geom"]["SQ_WAVES"] == 200 and by["k_geom"]["SQ_INSTS_VALU"] == 10000
    lines = rs.sq_lines(by)
    valu = next(line for line in lines if line.startswith("VALU busy"))
    assert "0.76" in valu and "0.5" in valu and "[SQ_ACTIVE_INST_VALU / SQ_BUSY_CU_CYCLES]" in valu
    per_wave = next(line for line in lines if line.startswith("VALU instructions per wave"))
    assert per_wave.split()[4] == "50" and per_wave.split()[5] == "50"
    # ratios whose counters were not collected are left out
    assert not any(line.startswith("LDS busy") for line in lines)


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2005_02704_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "lidarseg_internal.h").write_text("int x;\n")
    (csrc / "lidarseg_kernels.hip").write_text("int f() { return 1; }  // one\n/* block */\n")
    monkeypatch.setattr(rs, "ROOT", str(tmp_path))
    h0 = rs.kernel_source_hash()
    (csrc / "lidarseg_kernels.hip").write_text("int  f() {\n  return 1;  // another comment\n}\n")
    assert rs.kernel_source_hash() == h0
    (csrc / "lidarseg_kernels.hip").write_text("int f() { return 2; }\n")
    assert rs.kernel_source_hash() != h0


@pytest.mark.parametrize("name", ["k_geom_batch64_street.txt", "k_geom_batch64_street_sq.txt"])
def test_committed_summaries_name_their_command(name):
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles", name)
    text = open(path).read()
    assert "command: rocprofv3" in text and "bench.py" in text and "_work" not in text
