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
