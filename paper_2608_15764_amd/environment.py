"""Environment capture around a measurement session.

The method records driver, runtime, clocks, power limit and throttle state
for every session and checks that no throttling happened during collection
(Section 3, "Environment").  This module collects the same facts on the
MI355X host: runtime versions, the host CPU, and the GPU's current shader
memory, fabric and SoC clock levels, power, power cap, temperatures and performance
level from sysfs, taken before and after a session so that a clock change
is visible beside the numbers.  Everything is read from files; no helper
program is started from the measuring process.
"""
import os
import platform

def _read(path):
    try:
        with open(path) as f:
            return f.read().strip()
    except OSError:
        return None


def _current_level(text):
    """The level marked current ('*') in a pp_dpm_* table, e.g. '2400Mhz'."""
    if not text:
        return None
    for line in text.splitlines():
        if line.rstrip().endswith("*"):
            return line.split(":", 1)[-1].replace("*", "").strip()
    return None


def gpu_devices(root="/sys/class/drm"):
    """sysfs device directories of AMD GPUs (PCI vendor 0x1002)."""
    out = []
    try:
        names = sorted(os.listdir(root))
    except OSError:
        return out
    for n in names:
        if not n.startswith("card") or "-" in n:
            continue
        d = os.path.join(root, n, "device")
        if _read(os.path.join(d, "vendor")) == "0x1002":
            out.append(d)
    return out


def sysfs_metrics(device_dir=None):
    """Clocks, power, temperatures and performance level read from sysfs
    (plain file reads: no helper program is started)."""
    devs = [device_dir] if device_dir else gpu_devices()
    if not devs:
        return {"error": "no AMD GPU in sysfs"}
    d = devs[0]
    m = {"device": d,
         "sclk": _current_level(_read(os.path.join(d, "pp_dpm_sclk"))),
         "mclk": _current_level(_read(os.path.join(d, "pp_dpm_mclk"))),
         "fclk": _current_level(_read(os.path.join(d, "pp_dpm_fclk"))),
         "socclk": _current_level(_read(os.path.join(d, "pp_dpm_socclk"))),
         "perf_level": _read(os.path.join(d, "power_dpm_force_performance_level")),
         "link": _read(os.path.join(d, "current_link_speed"))}
    hw = os.path.join(d, "hwmon")
    try:
        hws = sorted(os.listdir(hw))
    except OSError:
        hws = []
    for h in hws:
        base = os.path.join(hw, h)
        for f, key, scale in (("power1_input", "power_w", 1e-6),
                              ("power1_average", "power_avg_w", 1e-6),
                              ("power1_cap", "power_cap_w", 1e-6)):
            v = _read(os.path.join(base, f))
            if v is not None and v.lstrip("-").isdigit():
                m[key] = int(v) * scale
        for i in range(1, 6):
            v = _read(os.path.join(base, f"temp{i}_input"))
            if v is not None and v.lstrip("-").isdigit():
                label = _read(os.path.join(base, f"temp{i}_label")) or f"temp{i}"
                m[f"temp_{label}_c"] = int(v) / 1000.0
    return m


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def static_info():
    info = {"host": platform.node(), "python": platform.python_version(),
            "cpu_model": cpu_model(), "cpu_count": os.cpu_count()}
    try:
        import torch
        info["torch"] = torch.__version__
        info["hip_runtime"] = getattr(torch.version, "hip", None)
    except ImportError:
        pass
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    try:
        with open(os.path.join(rocm, ".info", "version")) as f:
            info["rocm"] = f.read().strip()
    except OSError:
        pass
    return info
