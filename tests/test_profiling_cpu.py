"""Host-side checks of the rocprofv3 summaries: launch selection, copy-kernel
calibration and the source digest that ties a traffic report to the kernels
it measured. Synthetic counter files, no GPU."""
import csv
import json
import os

from paper_1804_01830_amd import profiling as P

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]

LINE = {"metric": "m", "config": {"grid": [128, 128, 32], "workload": "disk-mixed-128x128x32", "batch": 8},
        "plan_info": {"padded": [256, 256, 64], "tile_z": 8, "ez": 4, "z_groups": 1},
        "roofline": {"kernel": "k_z_serial", "algorithmic_bytes_per_launch": 1000000}}
BLOCK = 8 * 16                                    # tk * Pz / E threads
GRID = (128 // 8 * 256 + (128 + 8) // 8 * 8) * BLOCK   # kx tiles x ky rows, Nyquist strip groups x batch


def _write(directory, counter, rows):
    os.makedirs(directory)
    with open(os.path.join(directory, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, wg, grid, val) in enumerate(rows):
            w.writerow({k: 0 for k in FIELDS} | {"Dispatch_Id": i, "Kernel_Name": name, "Workgroup_Size": wg,
                                                  "Grid_Size": grid, "Counter_Name": counter,
                                                  "Counter_Value": val})


def test_traffic_uses_matching_launches_and_copy_scale(tmp_path):
    z = "void dds::k_z_serial<float, 64, 4, 3>(dds::cplx<float> const*)"
    # tuning launches of another shape, three timed launches, the 512 MiB copy
    _write(tmp_path / "f", "FETCH_SIZE", [(z, 256, GRID * 2, 9e9), (z, BLOCK, GRID, 400.0), (z, BLOCK, GRID, 410.0),
                                          (z, BLOCK, GRID, 405.0), ("elementwise_kernel", 256, 1 << 20, 262144.0)])
    _write(tmp_path / "w", "WRITE_SIZE", [(z, BLOCK, GRID, 600.0), ("elementwise_kernel", 256, 1 << 20, 524288.0)])
    t = P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), LINE, 512)
    assert t["FETCH_SIZE"]["launches"] == 3 and abs(t["FETCH_SIZE"]["factor"] - 2.0) < 1e-12
    assert t["FETCH_SIZE"]["bytes"] == 405.0 * 1024 * 2.0
    assert t["WRITE_SIZE"]["bytes"] == 600.0 * 1024 * 1.0


def test_stored_traffic_requires_current_sources(tmp_path):
    _write(tmp_path / "f", "FETCH_SIZE", [("void dds::k_z_serial<float>", BLOCK, GRID, 100.0),
                                          ("copy", 64, 64, 1024.0)])
    _write(tmp_path / "w", "WRITE_SIZE", [("void dds::k_z_serial<float>", BLOCK, GRID, 50.0),
                                          ("copy", 64, 64, 1024.0)])
    line_file = tmp_path / "bench.log"
    line_file.write_text("[bench] noise\n" + json.dumps(LINE) + "\n")
    report = P.traffic_report(str(tmp_path / "f"), str(tmp_path / "w"), str(line_file), 1, "t",
                              "rocprofv3 --pmc {COUNTER} -- python3 bench.py")
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "z.md").write_text(report)
    got = P.stored_traffic(str(prof), "disk-mixed-128x128x32", 8, "k_z_serial")
    assert got == (100.0 + 50.0) * 1024
    assert P.stored_traffic(str(prof), "disk-mixed-128x128x32", 1, "k_z_serial") is None
    (prof / "z.md").write_text(report.replace(P.source_digest(), "0" * 64))
    assert P.stored_traffic(str(prof), "disk-mixed-128x128x32", 8, "k_z_serial") is None


def test_relax_traffic_report_selects_the_fp32_step_and_tracks_its_sources(tmp_path):
    k32 = "void dds::(anonymous namespace)::k_relax_march<float, 64, 16>(float const*, float*)"
    k64 = "void dds::(anonymous namespace)::k_relax_march<double, 64, 16>(double const*, double*)"
    _write(tmp_path / "f", "FETCH_SIZE", [(k32, 1024, 1 << 20, 100.0), (k32, 1024, 1 << 20, 110.0),
                                          (k32, 1024, 1 << 20, 105.0), (k64, 1024, 1 << 20, 9e9),
                                          ("elementwise_kernel", 256, 1 << 20, 262144.0)])
    _write(tmp_path / "w", "WRITE_SIZE", [(k32, 1024, 1 << 20, 50.0), (k64, 1024, 1 << 20, 9e9),
                                          ("elementwise_kernel", 256, 1 << 20, 524288.0)])
    line = {"metric": "m", "config": {"workload": "relax-layer"},
            "roofline": {"algorithmic_bytes_per_launch": 300000}}
    (tmp_path / "bench.json").write_text(json.dumps(line) + "\n")
    report = P.relax_traffic_report(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "bench.json"), 512,
                                     "t", "rocprofv3 --pmc {COUNTER} -- python3 bench.py --relax")
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "relax.md").write_text(report)
    got = P.stored_traffic(str(prof), "relax-layer", 1, "k_relax_march", sources=P.RELAX_SOURCES)
    assert got == 105.0 * 1024 * 2.0 + 50.0 * 1024
    # the digest of the passes' sources does not stand in for the relaxation's
    assert P.stored_traffic(str(prof), "relax-layer", 1, "k_relax_march") is None


def test_kernels_report_scales_every_library_kernel(tmp_path):
    ka = "void dds::k_yx_inv<256, 128>(float const*)"
    kb = "void dds::k_xy_fwd<256, 128>(float const*)"
    _write(tmp_path / "f", "FETCH_SIZE", [(ka, 1024, 4096, 10.0)] * 5 + [(kb, 1024, 4096, 3.0)] * 5 +
           [("elementwise_kernel", 256, 1 << 20, 262144.0)])
    _write(tmp_path / "w", "WRITE_SIZE", [(ka, 1024, 4096, 7.0)] * 5 + [(kb, 1024, 4096, 2.0)] * 5 +
           [("elementwise_kernel", 256, 1 << 20, 524288.0)])
    rep = P.kernels_report(str(tmp_path / "f"), str(tmp_path / "w"), 512, "t", "cmd {COUNTER}")
    rows = [l for l in rep.splitlines() if l.startswith("| `")]
    assert rows[0].startswith("| `dds::k_yx_inv") and rows[1].startswith("| `dds::k_xy_fwd")
    assert f"| {10.0 * 1024 * 2.0 / 1e6:.1f} | {7.0 * 1024 / 1e6:.1f} |" in rows[0]


def test_counters_report_takes_medians_per_kernel_shape(tmp_path):
    z = "void dds::k_z_serial<float, 64, 4, 3, 8>(dds::cplx<float> const*)"
    y = "void dds::(anonymous namespace)::k_yx_inv<256, 128>(dds::cplx<float> const*)"
    # two counter runs; the copy kernel and a shape launched too few times are left out
    _write(tmp_path / "a", "VALUBusy", [(z, BLOCK, GRID, 40.0), (z, BLOCK, GRID, 44.0), (z, BLOCK, GRID, 42.0),
                                        (z, BLOCK, GRID, 90.0), (z, 256, GRID, 5.0), (y, 1024, 262144, 30.0),
                                        (y, 1024, 262144, 31.0), (y, 1024, 262144, 29.0), (y, 1024, 262144, 33.0),
                                        ("elementwise_kernel", 256, 1 << 20, 1.0)])
    _write(tmp_path / "b", "SQ_WAVES", [(z, BLOCK, GRID, 8704.0)] * 4 + [(y, 1024, 262144, 4096.0)] * 4)
    rep = P.counters_report([str(tmp_path / "a"), str(tmp_path / "b")], "t", ["cmd a", "cmd b"], min_launches=4)
    lines = [l for l in rep.splitlines() if l.startswith("| `")]
    assert len(lines) == 2 and "| VALUBusy | SQ_WAVES |" in rep
    zl = [l for l in lines if "k_z_serial" in l][0]
    assert "| 128 |" in zl and "| 44 | 8704 |" in zl                  # median of 40, 42, 44, 90
    yl = [l for l in lines if "k_yx_inv" in l][0]
    assert "`dds::k_yx_inv<256, 128>`" in yl and "| 31 | 4096 |" in yl
