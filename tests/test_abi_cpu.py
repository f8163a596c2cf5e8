"""C-ABI checks that need no GPU: the library loads, exports every entry
point the header declares, its host-only plan generator agrees with the
oracle's, and device calls fail loudly where there is no GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2410_04349_amd as hb
from oracle import epg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hb.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return set(re.findall(r"\b(hb_[a-z_]+)\s*\(", txt))


def test_header_symbols_exported():
    names = _declared()
    assert names, "no declarations found"
    lib = ctypes.CDLL(hb.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(hb.EXPORTED)


def test_version():
    assert "gfx950" in hb.hb_version()


SP = [1.0, 0.3, 0.4, 0.4, 0.2, 0.3]
COST = [0.1, 0.2, 0.1, 0.6, 1.0, 0.6]
RULES = [[0, 1, 2, 3], [2, 4], [5, 4]]


def test_epg_path_paper_examples():
    got = hb.hb_epg_path(SP, COST, RULES)
    assert [r for r, _ in got] == [1, 0, 2]            # Example 5: phi2, phi1, phi3
    assert got[1][1] == [2, 1, 3, 0]                  # sname, price, pname, color
    seq, _, _ = epg.sequential_path(RULES, SP, COST)
    assert got == [(r, p) for r, p in seq]


@pytest.mark.parametrize("seed", range(20))
def test_epg_path_matches_oracle_random(seed):
    r = np.random.default_rng(seed)
    n_p = int(r.integers(1, 12))
    rules = [list(map(int, r.choice(n_p, size=int(r.integers(1, min(n_p, 6) + 1)), replace=False)))
             for _ in range(int(r.integers(1, 10)))]
    sp = [float(x) for x in r.choice([0.0, 0.1, 0.25, 0.5, 1.0], size=n_p)] if seed % 2 else list(r.random(n_p))
    cost = [float(x) for x in r.choice([0.1, 0.5, 1.0], size=n_p)] if seed % 3 else list(r.random(n_p) + 0.05)
    seq, _, _ = epg.sequential_path(rules, sp, cost)
    assert hb.hb_epg_path(sp, cost, rules) == [(a, b) for a, b in seq]


def test_epg_path_rejects_bad_estimates():
    with pytest.raises(hb.HbError):
        hb.hb_epg_path([0.5], [0.0], [[0]])
    with pytest.raises(hb.HbError):
        hb.hb_epg_path([1.5], [1.0], [[0]])
    with pytest.raises(hb.HbError):
        hb.hb_epg_path([0.5], [1.0], [[3]])


def test_no_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(hb.HbError) as e:
        hb.hb_create(0, allocator="hip")
    assert e.value.status == hb.HB_ERR_HIP


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structs have the header's field offsets and
    sizes (compiled against include/hb.h with the host C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"hb_pred": hb.HbPred, "hb_rule": hb.HbRule, "hb_column": hb.HbColumn, "hb_job": hb.HbJob,
               "hb_batch_info": hb.HbBatchInfo, "hb_match_stats": hb.HbMatchStats,
               "hb_work_stats": hb.HbWorkStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hb.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)
