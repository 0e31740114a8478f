"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad factor tables before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "thck.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b([a-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_symbols_exported():
    from paper_2409_12708_amd import thck
    lib = thck.load_library()
    syms = _header_symbols()
    assert len(syms) >= 15, syms
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(syms) == sorted(thck.EXPORTS)


def test_capacity_matches_profile():
    from paper_2409_12708_amd import thck
    import synth
    for n, D in [(8, 16), (24, 128), (40, 256), (16, 256)]:
        b = synth.bond_profile(n, D)
        assert thck.capacity(n, D) == sum(b[j] * 2 * b[j + 1] for j in range(n))


def _load(t, chi, zeta):
    from paper_2409_12708_amd import thck
    lib = thck.load_library()
    h = C.c_void_p()
    st = lib.thc_load_factors(C.byref(h), chi.shape[0], chi.shape[1], thck._dptr(t), thck._dptr(chi),
                              thck._dptr(zeta), 0, None)
    return st, lib.thc_last_error().decode()


def test_load_factors_rejects_bad_input():
    rng = np.random.default_rng(0)
    L, N = 3, 4
    t = rng.standard_normal((L, L)); t = t + t.T
    chi = rng.standard_normal((L, N))
    z = rng.standard_normal((N, N)); z = z + z.T
    bad = z.copy(); bad[0, 1] += 1.0
    st, msg = _load(t, chi, bad)
    assert st == -1 and "zeta" in msg
    st, msg = _load(t + np.triu(np.ones((L, L)), 1), chi, z)
    assert st == -1 and "t " in msg + " "
    chi2 = chi.copy(); chi2[1, 2] = np.nan
    st, msg = _load(t, chi2, z)
    assert st == -4
    t2 = t.copy(); t2[0, 0] = np.inf
    st, msg = _load(t2, chi, z)
    assert st == -4


def test_default_opts():
    from paper_2409_12708_amd import thck
    o = thck.make_opts(64)
    assert o.D_max == 64 and o.rel_cutoff == 1e-14 and o.include_T == 1 and o.include_V == 1 and o.prec == 0


def test_struct_layouts_match_header(tmp_path):
    # the ctypes structures must have the C sizes and field offsets of thck.h
    import ctypes as C
    import shutil
    import subprocess
    from paper_2409_12708_amd import thck as T
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    fields = {
        "thc_mps": [f for f, _ in T.ThcMps._fields_],
        "thc_opts": [f for f, _ in T.ThcOpts._fields_],
        "thc_stats": [f for f, _ in T.ThcStats._fields_],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "thck.h"', "int main(void) {"]
    for s, fs in fields.items():
        lines.append(f'  printf("{s} %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'  printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.split("\n") if l)
    for s, cls in (("thc_mps", T.ThcMps), ("thc_opts", T.ThcOpts), ("thc_stats", T.ThcStats)):
        assert int(out[s]) == C.sizeof(cls), s
        for f, _ in cls._fields_:
            assert int(out[f"{s}.{f}"]) == getattr(cls, f).offset, (s, f)


def test_flag_constants_match_header():
    # every THC_FLAG_* of the header has the binding's FLAG_* of the same
    # value, and the binding defines no flag the header lacks
    from paper_2409_12708_amd import thck
    src = open(os.path.join(ROOT, "include", "thck.h")).read()
    header = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define THC_FLAG_([A-Z0-9_]+)\s+(\d+)ull", src)}
    binding = {k[len("FLAG_"):]: v for k, v in vars(thck).items() if k.startswith("FLAG_") and isinstance(v, int)}
    assert header and header == binding
    assert len(set(header.values())) == len(header)  # distinct bits
    assert all(v & (v - 1) == 0 for v in header.values())
