"""The profile summary tool on small synthetic rocprofv3 outputs: counter
calibration by the copy kernel, per-kernel bytes, the staleness hash that
ignores comments but not code, and the benchmark's per-stage bytes."""
import json
import os
import sys

import pytest

from paper_2112_13169_amd import prof_summary as ps

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        fh.write(",".join(f'"{h}"' for h in header) + "\n")
        for r in rows:
            fh.write(",".join(f'"{v}"' for v in r) + "\n")


def test_summary_calibrates_counters_by_the_copy(tmp_path):
    kt = tmp_path / "kt"
    _write(str(kt / "kt_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
            "StdDev"],
           [["void vg::(anonymous namespace)::k_rays<false>(vg::RayParams)", 10, 300000, 30000,
             90.0, 29000, 31000, 1.0],
            ["__amd_rocclr_copyBuffer", 1, 20000, 20000, 10.0, 20000, 20000, 0.0]])
    hdr = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
           "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
           "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
           "Counter_Value", "Start_Timestamp", "End_Timestamp"]

    def pmc(name, counter, rays_kib, copy_kib):
        rows = [[i, i, "Agent 1", 1, 1, 1, 256, 1,
                 "void vg::(anonymous namespace)::k_rays<false>(vg::RayParams)", 256, 0, 0, 64, 0,
                 40, counter, rays_kib, 0, 1] for i in range(1, 4)]
        rows.append([9, 9, "Agent 1", 1, 1, 1, 131072, 2, "__amd_rocclr_copyBuffer", 256, 0, 0,
                     8, 0, 16, counter, copy_kib, 0, 1])
        # a later, smaller copy (a frame upload) must not be taken for the calibration
        rows.append([10, 10, "Agent 1", 1, 1, 1, 4096, 2, "__amd_rocclr_copyBuffer", 256, 0, 0,
                     8, 0, 16, counter, copy_kib / 50, 0, 1])
        _write(str(tmp_path / name / "pmc_counter_collection.csv"), hdr, rows)

    # a 1 MiB copy reads as 512 KiB fetched (factor 2) and 1024 KiB written
    pmc("fetch", "FETCH_SIZE", 100.0, 512.0)
    pmc("write", "WRITE_SIZE", 300.0, 1024.0)
    md, js = tmp_path / "out.md", tmp_path / "out.json"
    ps.main(["--kt", str(kt), "--fetch", str(tmp_path / "fetch"), "--write",
             str(tmp_path / "write"), "--workload", "w", "--cal-bytes", str(1 << 20),
             "--command", "cmd", "--md", str(md), "--json", str(js)])
    t = json.loads(js.read_text())
    assert t["fetch_factor"] == 2.0 and t["write_factor"] == 1.0
    assert t["kernels"]["k_rays<false>"]["hbm_bytes_per_launch"] == 1024 * (100 * 2 + 300)
    # 512 000 bytes in the kernel's 30 us average: 17.07 GB/s
    assert t["kernels"]["k_rays<false>"]["gb_per_s"] == round(512000 / 30000, 1)
    assert t["hbm_peak_gbs"] == 8000.0
    assert t["source_hash"] == ps.kernel_source_hash()
    text = md.read_text()
    assert "`k_rays<false>`" in text and "cmd" in text


def test_hash_ignores_comments_but_not_code():
    base = "int f(int a) { return a + 1; }\n"
    assert ps.code_only(base) == ps.code_only("// note\n" + base + "/* more\n lines */\n")
    assert ps.code_only(base) != ps.code_only(base.replace("+ 1", "+ 2"))
    files = {rel: base for rel in ps.KERNEL_SOURCES}
    h0 = ps.kernel_source_hash(lambda rel: files[rel])
    files[ps.KERNEL_SOURCES[0]] = "/* c */ " + base
    assert ps.kernel_source_hash(lambda rel: files[rel]) == h0
    files[ps.KERNEL_SOURCES[1]] = base + "int g;"
    assert ps.kernel_source_hash(lambda rel: files[rel]) != h0


def test_stage_traffic_is_the_launch_weighted_mean_of_its_kernels(tmp_path, monkeypatch):
    """A stage whose launches use one of several kernel forms reports the
    bytes of an average launch, not the sum over the forms."""
    import bench
    from paper_2112_13169_amd.prof_summary import kernel_source_hash
    path = tmp_path / "traffic.json"
    kernels = {"k_rays<false, false, true>": dict(hbm_bytes_per_launch=8000, launches=90),
               "k_rays<false, false, false>": dict(hbm_bytes_per_launch=9000, launches=10)}
    path.write_text(json.dumps(dict(workload="w", source_hash=kernel_source_hash(),
                                    kernels=kernels)))
    assert bench.measured_traffic("k_rays", str(path), "w") == pytest.approx(8100.0)
    assert bench.measured_traffic("k_rays", str(path), "other") is None
    assert bench.measured_traffic("k_seed", str(path), "w") is None
