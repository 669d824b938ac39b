"""The committed profile summaries (no GPU): each names the commands that
made it, those commands run committed files only (the profiler on
``bench.py``, the summariser of this package), every bench mode they name
exists, and every PMC pass stays within one run's counter limits."""
import os
import re
import shlex

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
FILES = sorted(f for f in os.listdir(PROFILES) if f.endswith((".txt", ".md")))

# counters per hardware block that one rocprofv3 --pmc run can hold, and
# how many of a block's slots a derived counter takes
LIMITS = {"SQ": 8, "TCC": 4, "TCP": 4, "TA": 2, "TD": 2, "GRBM": 2}
DERIVED = {"FETCH_SIZE": {"TCC": 3}, "WRITE_SIZE": {"TCC": 2},
           "MemUnitStalled": {"TA": 1, "GRBM": 1}}


def _commands(path):
    with open(path) as f:
        return [ln[len("# command: "):].strip() for ln in f if ln.startswith("# command: ")]


def _bench_modes():
    with open(os.path.join(ROOT, "bench.py")) as f:
        text = f.read()
    m = re.search(r'"--only".*?choices=\[(.*?)\]', text, re.S)
    return set(re.findall(r'"(\w+)"', m.group(1)))


@pytest.mark.parametrize("name", FILES)
def test_profile_names_its_commands(name):
    cmds = _commands(os.path.join(PROFILES, name))
    assert cmds, f"{name}: no '# command:' line"
    modes = _bench_modes()
    for c in cmds:
        assert "_work" not in c and "/root/reference" not in c, c
        if c.startswith("rocprofv3"):
            prog = c.split(" -- ", 1)[1].split()
            assert prog[:2] == ["python3", "bench.py"], c
            if "--only" in prog:
                assert prog[prog.index("--only") + 1] in modes, c
        else:
            assert c.startswith("python -m paper_2608_15764_amd.rocprof "), c
            toks = shlex.split(c)
            # no placeholder to fill in (a kernel's template name aside)
            rest = [t for i, t in enumerate(toks) if i == 0 or toks[i - 1] != "--kernel"]
            assert not any("<" in t for t in rest), c


def _pmc_sets():
    for name in FILES:
        for c in _commands(os.path.join(PROFILES, name)):
            if c.startswith("rocprofv3 --pmc"):
                toks = shlex.split(c.split(" -- ", 1)[0])[2:]
                yield name, [t for t in toks[:toks.index("-f")]]


@pytest.mark.parametrize("name,counters", list(_pmc_sets()))
def test_pmc_pass_fits_one_run(name, counters):
    use = {}
    for c in counters:
        base = re.sub(r"_(sum|avr|min|max)$", "", c)
        blocks = DERIVED.get(base) or {base.split("_")[0]: 1}
        for b, n in blocks.items():
            use[b] = use.get(b, 0) + n
    for b, n in use.items():
        assert b in LIMITS and n <= LIMITS[b], (name, counters, use)
