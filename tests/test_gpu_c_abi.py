"""The C ABI used from plain C (gcc, HIP runtime only), checked against the
oracle."""
import os
import subprocess

import pytest

from conftest import ROOT

pytestmark = pytest.mark.gpu


def _gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except ImportError:
        return False


@pytest.mark.skipif(not _gpu(), reason="needs a GPU")
def test_plain_c_program(tmp_path):
    from oracle import checksums, plan as oplan, splitmix
    lib_dir = os.path.join(ROOT, "paper_2608_15764_amd")
    exe = str(tmp_path / "c_abi_check")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    subprocess.run(["gcc", "-O2", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm, "include"),
                    os.path.join(ROOT, "tests", "c_abi_check.c"), "-o", exe,
                    "-L", lib_dir, "-lilpsweep", "-L", os.path.join(rocm, "lib"),
                    "-lamdhip64", f"-Wl,-rpath,{lib_dir}",
                    f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"], check=True)
    nbytes, seed = 64 << 20, 7
    out = subprocess.run([exe, str(nbytes), str(seed)], check=True, capture_output=True,
                         text=True, timeout=120).stdout
    res = {l.split()[0]: tuple(int(v) for v in l.split()[1:]) for l in out.strip().splitlines()}
    words = splitmix.buffer_words(seed, nbytes)
    whole = checksums.whole_buffer(words)
    L = nbytes // 16
    for name, K in (("plain", 4), ("lds_async", 8), ("batched_K2", 2), ("noalloc", 4)):
        assert res[name][:2] == whole and res[name][2] == L, name
    from paper_2608_15764_amd import ilpsweep as isw
    # K = 3 does not divide the pass: every order reads the same prefix
    nw8 = isw.sweep_device_info()["num_cus"] * 8
    p3 = oplan.wave_group(L, 3, nw8)
    for name, order in (("blocked_K3", oplan.BLOCKED), ("strided_K3", oplan.STRIDED)):
        want = checksums.combine(*checksums.per_wave(words, 16, 3, p3["Q"], nw8,
                                                     order=order))
        assert res[name] == (*want, p3["issued"]), name
    n_waves = isw.sweep_device_info()["num_cus"] * 32
    p = oplan.wave_group(L, 3, n_waves)
    want = checksums.combine(*checksums.per_wave(words, 16, 3, p["Q"], n_waves))
    assert res["batched_K3"] == (*want, p["issued"])
    # a captured graph replays against the buffer's current contents
    assert res["graph_K3_rep0"] == res["batched_K3"]
    assert res["graph_K2_rep0"][:2] == whole
    words1 = splitmix.buffer_words(seed + 1, nbytes)
    assert res["graph_K2_rep1"] == (*checksums.whole_buffer(words1), L)
    want1 = checksums.combine(*checksums.per_wave(words1, 16, 3, p["Q"], n_waves))
    assert res["graph_K3_rep1"] == (*want1, p["issued"])
    # the fused graph ran after the refill: both points equal the unfused cell
    assert res["fused_0"] == res["fused_1"] == res["graph_K3_rep1"]
    # split two-stream launch over the refilled buffer: each stream reads
    # its whole half exactly once
    (a0, an), (b0, bn) = checksums.two_stream_regions(L)
    assert res["split_a"] == (*checksums.whole_buffer(words1[a0 * 4:(a0 + an) * 4]), an)
    assert res["split_b"] == (*checksums.whole_buffer(words1[b0 * 4:(b0 + bn) * 4]), bn)
