"""Environment capture around a measurement session.

The method records driver, runtime, clocks, power limit and throttle state
for every session and checks that no throttling happened during collection
(Section 3, "Environment").  This module collects the same facts on the
MI355X host: runtime versions, the host CPU, and a flattened subset of
``amd-smi metric`` (clocks, power, temperature, throttle / violation
counters), taken before and after a session so a changing clock or a
throttle event is visible beside the numbers.
"""
import json
import os
import platform
import shutil
import subprocess

KEEP = ("clk", "clock", "power", "temp", "throttle", "violation", "socket_power",
        "gfx_activity", "umc_activity", "ecc")


def _flatten(obj, prefix="", out=None):
    out = {} if out is None else out
    if isinstance(obj, dict):
        for k, v in obj.items():
            _flatten(v, f"{prefix}.{k}" if prefix else str(k), out)
    elif isinstance(obj, list):
        for i, v in enumerate(obj):
            _flatten(v, f"{prefix}[{i}]", out)
    else:
        out[prefix] = obj
    return out


def amd_smi_metrics(timeout=30, limit=80):
    """Selected flattened ``amd-smi metric --json`` fields, or an error."""
    exe = shutil.which("amd-smi") or "/opt/rocm/bin/amd-smi"
    if not os.path.exists(exe):
        return {"error": "amd-smi not found"}
    try:
        r = subprocess.run([exe, "metric", "--json"], capture_output=True, text=True,
                           timeout=timeout)
    except (OSError, subprocess.TimeoutExpired) as e:
        return {"error": f"amd-smi failed: {e}"}
    try:
        flat = _flatten(json.loads(r.stdout))
    except ValueError:
        return {"error": "amd-smi output is not JSON", "rc": r.returncode}
    keep = {k: v for k, v in flat.items()
            if any(t in k.lower() for t in KEEP) and v not in (None, "N/A", "")}
    return dict(list(keep.items())[:limit])


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
