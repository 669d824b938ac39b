"""Environment capture helpers (no GPU)."""
from paper_2608_15764_amd import environment


def test_flatten_and_static_info():
    assert environment._flatten({"a": {"b": [1, {"c": 2}]}}) == {"a.b[0]": 1, "a.b[1].c": 2}
    info = environment.static_info()
    assert info["cpu_count"] and "python" in info


def test_metrics_degrade_gracefully():
    m = environment.amd_smi_metrics(timeout=20)
    assert isinstance(m, dict)       # either selected fields or an "error" entry
