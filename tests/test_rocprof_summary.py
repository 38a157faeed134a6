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
    line = dict(metric="m", steps=1, kernels=dict(plane_h32=dict(launches=2, bytes_per_launch=algo / 1.25)))
    (tmp_path / "b.log").write_text("bench: noise\n" + json.dumps(line) + "\n")
    tj = tmp_path / "t.json"
    md = R.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "b.log"), "plane_h32",
                   "k_plane_hw<72, float, 4, 7, false>", "t", "cf", "cw", str(tj))
    t = json.loads(tj.read_text())["plane_h32"]
    assert abs(t["measured_over_algorithmic"] - 1.25) < 1e-12
    assert t["launches_matched"] == 2 and t["source_sha1"] == R.source_hash("plane_h32")
    assert abs(t["read_bytes_per_launch"] - 2.0 * 1024 * 2000.0) < 1e-6
    assert "1.250" in md
