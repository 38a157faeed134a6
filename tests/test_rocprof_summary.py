"""The rocprofv3 summary helper (host logic): counter calibration on the copy kernel, the
matching of a kernel's last launches to the bench step, and the stored ratio."""
import json

from paper_2607_14025_amd import rocprof_summary as R


def _csv(path, counter, rows):
    with open(path, "w") as fh:
        fh.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for d, n, v in rows:
            fh.write(f'{d},"{n}","{counter}",{v}\n')


def test_traffic_ratio(tmp_path):
    copy = "void at::native::elementwise_kernel<MulFunctor<double>>(int)"
    kern = "void stern::(anonymous namespace)::k_plane_hw<72, float, 4, 7, false>(stern::Z<float>*, int)"
    # copy: FETCH 2^19 KiB (half the 1 GiB it reads), WRITE 2^20 KiB; kernel: 3 dispatches, the bench step has 2
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(1, copy, 2 ** 19), (2, kern, 999.0), (3, kern, 1000.0), (4, kern, 3000.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(1, copy, 2 ** 20), (2, kern, 5.0), (3, kern, 4000.0), (4, kern, 2000.0)])
    algo = 2.0 * 1024 * 2000.0 + 1024 * 3000.0  # calibrated fetch of the last two (2x) + write (1x)
    line = dict(metric="m", steps=20, kernels_steps=1, config=dict(workload="wl"),
                kernels=dict(plane_h32=dict(launches=2, bytes_per_launch=algo / 1.25)))
    (tmp_path / "b.log").write_text("bench: noise\n" + json.dumps(line) + "\n")
    tj = tmp_path / "t.json"
    md = R.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "b.log"), "plane_h32",
                   "k_plane_hw<72, float, 4, 7, false>", "t", "cf", "cw", str(tj))
    t = json.loads(tj.read_text())["wl:plane_h32"]
    assert abs(t["measured_over_algorithmic"] - 1.25) < 1e-12
    assert t["launches_matched"] == 2 and t["source_sha1"] == R.source_hash("plane_h32")
    assert abs(t["read_bytes_per_launch"] - 2.0 * 1024 * 2000.0) < 1e-6
    assert "1.250" in md


def test_mfma_summary_takes_the_final_apply(tmp_path):
    """Only the dispatches after the last but one Delta n launch count; FLOPs are MOPS x 512
    and the busy fraction is busy / (active x SIMDs)."""
    dn = "void stern::(anonymous namespace)::k_plane_dn<72>(stern::Z<double> const*)"
    red = "void stern::(anonymous namespace)::k_reduce_bf16w(__bf16 const*)"
    rows = []
    for d, n, mops, busy, act in ((1, red, 7.0, 1.0, 1.0), (2, dn, 0, 0, 1.0), (3, red, 1e6, 2048.0, 8.0),
                                  (4, red, 3e6, 6144.0, 8.0), (5, dn, 0, 0, 1.0), (6, red, 5.0, 1.0, 1.0)):
        for c, v in (("SQ_INSTS_VALU_MFMA_MOPS_BF16", mops), ("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0),
                     ("SQ_VALU_MFMA_BUSY_CYCLES", busy), ("GRBM_GUI_ACTIVE", act)):
            rows.append((d, n, c, v))
    with open(tmp_path / "m.csv", "w") as fh:
        fh.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for d, n, c, v in rows:
            fh.write(f'{d},"{n}","{c}",{v}\n')
    md = R.mfma(str(tmp_path / "m.csv"), "t", "cmd", simds=1024, xcds=1)
    line = [l for l in md.splitlines() if l.startswith("| `k_reduce_bf16w")][0].split("|")
    assert line[2].strip() == "2"                                    # dispatches 3 and 4 only
    assert float(line[3]) == round(2e6 * 512 / 1e9, 2)               # mean BF16 GFLOP per dispatch
    assert line[5].strip() == "50.0%"                                # 8192 / (16 x 1024)
    # a run's agent file gives the SIMDs and XCDs: GRBM_GUI_ACTIVE is summed over 2 XCDs here
    (tmp_path / "run_counter_collection.csv").write_text((tmp_path / "m.csv").read_text())
    (tmp_path / "run_agent_info.csv").write_text(
        '"Agent_Type","Simd_Count","Num_Xcc","Max_Engine_Clk_Fcompute"\n"CPU",0,1,0\n"GPU",2048,2,2400\n')
    md = R.mfma(str(tmp_path / "run_counter_collection.csv"), "t", "cmd")
    line = [l for l in md.splitlines() if l.startswith("| `k_reduce_bf16w")][0].split("|")
    assert line[5].strip() == "50.0%"                                # 8192 / (16 / 2 x 2048)
