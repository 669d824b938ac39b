"""Audit of our own gfx950 assembly (the counterpart of the paper's SASS
audit, Section 3 "Instruments"): every plain-load kernel issues exactly K
vector loads per loop iteration, all of them before the first wait on the
vector-memory counter, with no register spills; the LDS-direct loop issues
loads without a destination register."""
import os
import re

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_2608_15764_amd", "csrc")
ASM_DIR = os.path.join(ROOT, "_build", "asm")


def _asm(name):
    src = os.path.join(CSRC, name + ".hip")
    out = os.path.join(ASM_DIR, name + ".s")
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    if not os.path.exists(out) or os.path.getmtime(out) < max(map(os.path.getmtime, deps)):
        from paper_2608_15764_amd import build
        os.makedirs(ASM_DIR, exist_ok=True)
        build.asm_one(name + ".hip")
    with open(out) as f:
        return f.read()


def _functions(text):
    """{mangled name: list of instruction lines} for every kernel body."""
    out = {}
    name, body = None, []
    for line in text.splitlines():
        m = re.match(r"^(_Z\w+):", line)
        if m:
            name, body = m.group(1), []
            continue
        if name is None:
            continue
        body.append(line.strip())
        if body[-1].startswith("s_endpgm"):
            out[name] = body
            name = None
    return out


def _meta(text, name):
    """.vgpr_count / spill counts from the kernel's metadata block."""
    i = text.find(f".name:           {name}")
    if i < 0:
        i = text.find(f".symbol:         {name}.kd")
    blk = text[max(0, i - 3000): i + 3000]
    g = lambda k: int(re.search(rf"\.{k}:\s+(\d+)", blk).group(1))
    return {k: g(k) for k in ("vgpr_count", "vgpr_spill_count", "sgpr_spill_count",
                              "private_segment_fixed_size")}


def _loop(lines):
    """Instructions of the innermost loop (header label to back-branch)."""
    for i, l in enumerate(lines):
        if "Loop Header" in l:
            label = l.split(":")[0]
            body = []
            for l2 in lines[i + 1:]:
                body.append(l2)
                if re.match(r"s_cbranch_\w+\s+" + re.escape(label) + r"\b", l2) or \
                        re.match(r"s_branch\s+" + re.escape(label) + r"\b", l2):
                    return body
    return None


LOAD = re.compile(r"^(global|buffer)_load_(dword|dwordx2|dwordx4|b32|b64|b128)\b")


@pytest.fixture(scope="module")
def plain():
    t = _asm("kernels_plain")
    return t, _functions(t)


def _plain_name(K, V, P):
    return f"_ZN3ilp11plain_kloadILi{K}ELi{V}ELi{P}EEEvNS_9PlainArgsE"


@pytest.mark.parametrize("P", [0, 1, 2, 3])
@pytest.mark.parametrize("V", [4, 8, 16])
@pytest.mark.parametrize("K", range(1, 17))
def test_plain_loop_issues_exactly_K_loads_before_consuming(plain, K, V, P):
    text, funcs = plain
    name = _plain_name(K, V, P)
    body = _loop(funcs[name])
    assert body is not None, name
    loads = [i for i, l in enumerate(body) if LOAD.match(l)]
    assert len(loads) == K, (name, len(loads))
    waits = [i for i, l in enumerate(body) if l.startswith("s_waitcnt") and "vmcnt" in l]
    assert waits and waits[0] > loads[-1], "a load is consumed before all K are issued"
    assert not any(l.startswith(("scratch_", "buffer_store")) for l in body)
    m = _meta(text, name)
    assert m["vgpr_spill_count"] == 0 and m["sgpr_spill_count"] == 0
    assert m["private_segment_fixed_size"] == 0


@pytest.fixture(scope="module")
def lds():
    t = _asm("kernels_lds")
    return t, _functions(t)


@pytest.mark.parametrize("D", [1, 2, 4, 8, 16])
def test_lds_async_loop_has_no_register_destination_loads(lds, D):
    text, funcs = lds
    name = f"_ZN3ilp12lds_kernel_tILi1ELi{D}ELi0EEEvNS_7LdsArgsE"
    body = _loop(funcs[name])
    assert body is not None
    assert sum(l.startswith("global_load_lds_dwordx4") for l in body) == D
    assert not any(LOAD.match(l) for l in body)
    assert sum(l.startswith("ds_read_b128") for l in body) == D
    m = _meta(text, name)
    assert m["vgpr_spill_count"] == 0 and m["private_segment_fixed_size"] == 0


@pytest.mark.parametrize("D", [1, 2, 4, 8, 16])
def test_lds_matched_loop_goes_through_registers(lds, D):
    text, funcs = lds
    name = f"_ZN3ilp12lds_kernel_tILi2ELi{D}ELi0EEEvNS_7LdsArgsE"
    body = _loop(funcs[name])
    assert body is not None
    assert sum(bool(LOAD.match(l)) for l in body) == D
    assert sum(l.startswith("ds_write_b128") for l in body) == D
    assert sum(l.startswith("ds_read_b128") for l in body) == D
    assert not any(l.startswith("global_load_lds") for l in body)


def _kernel_names(text):
    return re.findall(r"^\s+\.name:\s+(\S+)\s*$", text, re.M)


@pytest.mark.parametrize("src", ["kernels_plain", "kernels_fused", "kernels_lds", "kernels_misc",
                                 "kernels_chase", "kernels_xcd"])
def test_no_kernel_spills_or_uses_scratch(src):
    text = _asm(src)
    names = [n for n in _kernel_names(text) if n.startswith("_Z")]
    assert names, src
    for n in names:
        m = _meta(text, n)
        assert m["vgpr_spill_count"] == 0 and m["sgpr_spill_count"] == 0, n
        assert m["private_segment_fixed_size"] == 0, n


@pytest.fixture(scope="module")
def misc():
    t = _asm("kernels_misc")
    return t, _functions(t)


@pytest.mark.parametrize("DT", [0, 1, 2])
@pytest.mark.parametrize("NL", [4, 8])
def test_reduce_loop_keeps_all_its_loads_in_flight(misc, DT, NL):
    """The streaming sum issues all NL 16-byte loads of a wave-group before
    the first wait, so NL x 1 KiB per wave is in flight."""
    text, funcs = misc
    name = f"_ZN3ilp9reduce_fpILi{DT}ELi{NL}EEEvNS_10ReduceArgsE"
    body = _loop(funcs[name])
    assert body is not None, name
    loads = [i for i, l in enumerate(body) if LOAD.match(l)]
    assert len(loads) == NL, (name, len(loads))
    waits = [i for i, l in enumerate(body) if l.startswith("s_waitcnt") and "vmcnt" in l]
    assert waits and waits[0] > loads[-1]
    m = _meta(text, name)
    assert m["vgpr_spill_count"] == 0 and m["private_segment_fixed_size"] == 0


@pytest.fixture(scope="module")
def fused():
    t = _asm("kernels_fused")
    return t, _functions(t)


@pytest.mark.parametrize("P", [0, 1, 2, 3])
@pytest.mark.parametrize("V", [4, 8, 16])
@pytest.mark.parametrize("K", range(1, 17))
def test_fused_batch_keeps_the_K_load_loop(fused, K, V, P):
    """The fused batch kernel issues its K loads of a group back to back and
    waits only after the last (the point list is read with scalar loads,
    which the vector-memory counter does not count), and never has more than
    K vector loads outstanding."""
    text, funcs = fused
    name = f"_ZN3ilp11fused_kloadILi{K}ELi{V}ELi{P}EEEvNS_9FusedArgsE"
    lines = funcs[name]
    runs, cur = [], 0
    for l in lines:
        if l.startswith("s_waitcnt") and "vmcnt" in l:
            runs.append(cur)
            cur = 0
        elif LOAD.match(l):
            cur += 1
    runs.append(cur)
    assert max(runs) == K and runs.count(K) >= 1, (name, runs)
    assert sum(bool(LOAD.match(l)) for l in lines) == K, name
    assert not any(l.startswith(("scratch_", "flat_")) for l in lines), name
    m = _meta(text, name)
    assert m["vgpr_spill_count"] == 0 and m["sgpr_spill_count"] == 0
    assert m["private_segment_fixed_size"] == 0


def _loops(lines):
    """Every loop (header label to back-branch), in program order."""
    out = []
    for i, l in enumerate(lines):
        if "Loop Header" in l:
            label = l.split(":")[0]
            body = []
            for l2 in lines[i + 1:]:
                body.append(l2)
                if re.match(r"s_cbranch_\w+\s+" + re.escape(label) + r"\b", l2):
                    out.append(body)
                    break
    return out


@pytest.mark.parametrize("P", [0, 1, 2, 3])
@pytest.mark.parametrize("kernel", ["chase", "chase_walkers"])
def test_chase_loops_keep_one_dependent_load_in_flight(kernel, P):
    """Every hop loop of the latency probes issues exactly one load and
    waits for the previous one before it (the address depends on it), and
    stores nothing: one dependent load in flight, so the time per hop is the
    load-to-use latency."""
    t = _asm("kernels_chase")
    fns = _functions(t)
    args = "ChaseArgs" if kernel == "chase" else "WalkArgs"
    name = f"_ZN3ilp{len(kernel)}{kernel}ILi{P}EEEvNS_{len(args)}{args}E"
    assert name in fns, sorted(fns)
    # the hop loops (the sampled probe also has a loop copying its samples
    # out of LDS, which loads nothing from memory)
    loops = [b for b in _loops(fns[name]) if any(LOAD.match(l) for l in b)]
    assert len(loops) == (3 if kernel == "chase" else 2), len(loops)
    for body in loops:
        loads = [i for i, l in enumerate(body) if LOAD.match(l)]
        assert len(loads) == 1, body
        waits = [i for i, l in enumerate(body) if re.match(r"s_waitcnt\s+vmcnt\(0\)", l)]
        assert waits and waits[0] < loads[0], body
        assert not any(l.startswith(("global_store", "buffer_store", "flat_store"))
                       for l in body), body


@pytest.mark.parametrize("P", [0, 1, 2, 3])
@pytest.mark.parametrize("kernel", ["xcd_subset", "xcd_split"])
def test_xcd_subset_loop_is_the_plain_K8_loop(P, kernel):
    """The XCD reads issue the plain loop's eight 16-byte loads per
    iteration, all before the first wait, and store nothing in the loop."""
    text = _asm("kernels_xcd")
    funcs = _functions(text)
    args = "XcdArgs" if kernel == "xcd_subset" else "XcdSplitArgs"
    name = f"_ZN3ilp{len(kernel)}{kernel}ILi{P}EEEvNS_{len(args)}{args}E"
    assert name in funcs, sorted(funcs)
    body = _loop(funcs[name])
    assert body is not None
    loads = [i for i, l in enumerate(body) if LOAD.match(l)]
    assert len(loads) == 8 and all(re.search(r"dwordx4|b128", body[i]) for i in loads)
    waits = [i for i, l in enumerate(body) if l.startswith("s_waitcnt") and "vmcnt" in l]
    assert waits and waits[0] > loads[-1]
    assert not any(l.startswith(("global_store", "buffer_store", "scratch_")) for l in body)
