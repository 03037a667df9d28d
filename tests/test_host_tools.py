"""Host-side helpers: rocprofv3 CSV summaries and the counter calibration."""
import json

from paper_2507_04192_amd import rocprof_summary as R


def test_short_names():
    assert R.short_name("void mpm::k_p2g<float, 3, 1>(mpm::Geo, mpm::Phys<float>, int const*)") == \
        "k_p2g<float, 3, 1>"
    assert R.short_name("__amd_rocclr_copyBuffer(char*, char*)") == "__amd_rocclr_copyBuffer"


def _pmc_csv(path, counter, rows):
    hdr = "Correlation_Id,Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    with open(path, "w") as f:
        f.write(hdr)
        for i, (name, v) in enumerate(rows):
            f.write(f'{i},{i},"{name}",{counter},{v}\n')


def test_traffic_scales_by_the_copy(tmp_path):
    fd, wd = tmp_path / "f", tmp_path / "w"
    fd.mkdir()
    wd.mkdir()
    k = "void mpm::k_g2p<float, 3, 1>(mpm::Geo)"
    # the copy of 1 MiB reads 512 fetch units and 1024 write units
    _pmc_csv(fd / "x_counter_collection.csv", "FETCH_SIZE",
             [("__amd_rocclr_copyBuffer(char*)", 512.0), (k, 100.0), (k, 300.0)])
    _pmc_csv(wd / "x_counter_collection.csv", "WRITE_SIZE",
             [("__amd_rocclr_copyBuffer(char*)", 1024.0), (k, 50.0)])
    t = R.traffic(str(fd), str(wd), 1 << 20)
    g = t["kernels"]["k_g2p<float, 3, 1>"]
    assert g["fetch_bytes"] == 200.0 * 2048 and g["write_bytes"] == 50.0 * 1024
    json.dumps(t)
    assert len(t["csrc_sha256"]) == 64


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_measured_traffic_sums_kernels_and_checks_the_sources(tmp_path, monkeypatch):
    import bench
    t = {"csrc_sha256": R.kernel_sources_hash(),
         "kernels": {"a": {"fetch_bytes": 10.0, "write_bytes": 5.0},
                     "b": {"fetch_bytes": 1.0, "write_bytes": 2.0}}}
    f = tmp_path / "traffic.txt"
    f.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("a") == 15.0
    assert bench.measured_traffic(["a", "b"]) == 18.0
    assert bench.measured_traffic(["a", "missing"]) is None
    t["csrc_sha256"] = "0" * 64            # counters taken on other sources
    f.write_text(json.dumps(t))
    assert bench.measured_traffic("a") is None


def test_paper_timing_cases_match_the_table():
    """The paper's granular timing cases (Table tab:simulation_params): the
    column's particle count is the table's exactly, the cylinder's within
    0.03%; grid, spacing and the App. A material as the paper states."""
    from paper_2507_04192_amd import workloads as W
    col, xc = W.granular_column_paper()
    assert col.n == (400, 32, 200) and xc.shape[1] == 2408448
    cyl, xy = W.cylinder_paper_grid()
    assert cyl.n == (400, 400, 100) and abs(xy.shape[1] - 2712960) <= 0.0003 * 2712960
    for cfg in (col, cyl):
        assert cfg.dx == 1 / 400 and cfg.dt == 1e-5 and cfg.material == W.DP_JAUMANN
        assert cfg.rho0 == 2650.0 and cfg.poisson == 0.3 and cfg.psi_deg == 0.0 and cfg.cohesion == 0.0
        assert abs(cfg.youngs / (3 * (1 - 2 * cfg.poisson)) - 0.7e6) < 1e-6
        assert cfg.wall_mode[4] == W.STICK
    assert col.phi_deg == 19.8 and cyl.phi_deg == 20.0
