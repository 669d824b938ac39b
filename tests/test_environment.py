"""Environment capture helpers (no GPU): sysfs parsing on a fake tree."""
import os

from paper_2608_15764_amd import environment


def _w(path, text):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write(text)


def test_sysfs_metrics_on_a_fake_device(tmp_path):
    d = tmp_path / "card0" / "device"
    _w(str(d / "vendor"), "0x1002\n")
    _w(str(d / "pp_dpm_sclk"), "S: 112Mhz\n0: 500Mhz\n1: 2400Mhz *\n")
    _w(str(d / "pp_dpm_mclk"), "0: 2000Mhz *\n")
    _w(str(d / "power_dpm_force_performance_level"), "auto\n")
    _w(str(d / "hwmon" / "hwmon3" / "power1_input"), "264000000\n")
    _w(str(d / "hwmon" / "hwmon3" / "power1_cap"), "1400000000\n")
    _w(str(d / "hwmon" / "hwmon3" / "temp2_input"), "46000\n")
    _w(str(d / "hwmon" / "hwmon3" / "temp2_label"), "hotspot\n")
    assert environment.gpu_devices(str(tmp_path)) == [str(d)]
    m = environment.sysfs_metrics(str(d))
    assert m["sclk"] == "2400Mhz" and m["mclk"] == "2000Mhz"
    assert m["power_w"] == 264.0 and m["power_cap_w"] == 1400.0
    assert m["temp_hotspot_c"] == 46.0 and m["perf_level"] == "auto"


def test_no_gpu_is_reported_not_raised(tmp_path):
    assert environment.sysfs_metrics.__call__ is not None
    assert environment.gpu_devices(str(tmp_path)) == []
    info = environment.static_info()
    assert info["cpu_count"] and "python" in info
