"""Host logic of the rocprofv3 summaries (no GPU): counter means per kernel,
copy calibration, and the staleness check on the kernel sources' hash."""
import json

from paper_cs_0605069_amd import profiling

HEAD = ("Correlation_Id,Dispatch_Id,Agent_Id,Queue_Id,Process_Id,Thread_Id,Grid_Size,Kernel_Id,Kernel_Name,"
        "Workgroup_Size,LDS_Block_Size,Scratch_Size,VGPR_Count,Accum_VGPR_Count,SGPR_Count,Counter_Name,"
        "Counter_Value,Start_Timestamp,End_Timestamp\n")


def _csv(path, counter, rows):
    with open(path, "w") as f:
        f.write(HEAD)
        for i, (name, v) in enumerate(rows):
            f.write(f'{i},{i},"Agent 1",1,1,1,64,1,"{name}",64,0,0,8,0,8,"{counter}",{v},0,1\n')


def test_traffic_summary_scales_by_the_copy(tmp_path):
    k = "void (anonymous namespace)::tiled::k_sus_level<4, 2, 6, 4>(DevCode, DevState)"
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(k, 100.0), (k, 300.0), ("__amd_rocclr_copyBuffer", 512.0),
                                            ("__amd_rocclr_copyBuffer", 4.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(k, 10.0), (k, 30.0), ("__amd_rocclr_copyBuffer", 1024.0)])
    text = profiling.traffic_markdown(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 1 << 20, "sus=4", "cmd")
    (tmp_path / "t.txt").write_text(text)
    block = profiling.read_traffic(str(tmp_path / "t.txt"))
    assert block is not None and block["shapes"] == {"sus": "4"}
    assert abs(block["fetch_scale"] - 2.0) < 1e-12 and abs(block["write_scale"] - 1.0) < 1e-12
    # mean fetch 200 KiB x 2, mean write 20 KiB x 1
    assert abs(block["kernels"]["sus_level"]["bytes_per_dispatch"] - (400 + 20) * 1024) < 1e-6
    assert block["kernels"]["sus_level"]["dispatches"] == 2


def test_stale_traffic_is_ignored(tmp_path):
    block = {"source_sha256": "0" * 64, "shapes": {}, "kernels": {}}
    (tmp_path / "t.txt").write_text("x\n```json\n" + json.dumps(block) + "\n```\n")
    assert profiling.read_traffic(str(tmp_path / "t.txt")) is None
    assert profiling.read_traffic(str(tmp_path / "missing.txt")) is None


def test_kernel_names():
    assert profiling.short_name("void ns::tiled::k_check<4, 1, 6>(DevCode, DevState, x)") == "k_check<4, 1, 6>"
    assert profiling.kind_of("k_variable<4, 1, 4>") == "variable"
    assert profiling.kind_of("__amd_rocclr_copyBuffer") is None
