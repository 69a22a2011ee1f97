"""The C-ABI library loads and exports every entry point the header declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dfrsw.h")
LIB = os.path.join(ROOT, "paper_2101_05617_amd", "libdfrsw.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("dfr_rhs", "dfr_jvp_complex_step", "kiops_phi_apply", "epi_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert missing == []


def test_binding_names_match_header():
    from paper_2101_05617_amd import dfrsw
    for n in dfrsw.exported_symbols():
        assert n in declared()


def test_constants_match_header():
    # the precision codes and the FP32 forms' eps bound as the binding has them
    from paper_2101_05617_amd import dfrsw
    src = open(HEADER).read()
    m = re.search(r"#define\s+DFR_FP32_EPS_MIN\s+([0-9.eE+-]+)", src)
    assert m and float(m.group(1)) == dfrsw.DFR_FP32_EPS_MIN
    for name in ("DFR_FP64", "DFR_FP32_JV", "DFR_FP32_JV_BASIS32"):
        v = re.search(name + r"\s*=\s*(\d+)", src)
        assert v and int(v.group(1)) == getattr(dfrsw, name)
    for name, key in (("DFR_ROUNDS_HOST", "host"), ("DFR_ROUNDS_DEVICE", "device")):
        v = re.search(name + r"\s*=\s*(\d+)", src)
        assert v and int(v.group(1)) == dfrsw.ROUNDS[key]


def test_struct_layouts_match_header(tmp_path):
    # the structs passed by pointer through the boundary: every field's offset
    # and each struct's size as the C compiler lays them out from the header,
    # against the binding's ctypes declarations
    import shutil
    import subprocess
    from paper_2101_05617_amd import dfrsw
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"dfr_grid_desc": dfrsw._GridDesc, "kiops_opts": dfrsw.KiopsOpts,
               "kiops_stats": dfrsw.KiopsStats, "kiops_decision": dfrsw.KiopsDecision,
               "kiops_replay": dfrsw._KiopsReplay}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-o", str(exe), str(src)], check=True, capture_output=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_decision_replay_marshalling():
    # the binding's kiops_replay: the replay list as the library reads it,
    # the record as the library writes it, and the pointer in kiops_opts
    from paper_2101_05617_amd import dfrsw
    play = [(0.25, 12, True), (0.125, 16, False), (0.125, 20, True)]
    r = dfrsw.DecisionReplay(play=play, rec_cap=4)
    st = r.struct
    assert st.n_play == 3 and st.pos == 0 and st.n_rec == 0 and st.rec_cap == 4
    assert [(st.play[i].tau, st.play[i].m, st.play[i].accept) for i in range(3)] == \
        [(0.25, 12, 1), (0.125, 16, 0), (0.125, 20, 1)]
    # what the library does after two attempts
    st.rec[0] = dfrsw.KiopsDecision(0.25, 12, 1)
    st.rec[1] = dfrsw.KiopsDecision(0.125, 16, 0)
    st.n_rec, st.pos = 2, 2
    assert r.recorded() == [(0.25, 12, True), (0.125, 16, False)] and r.pos == 2
    st.n_rec = 5      # more attempts than the record holds
    with pytest.raises(ValueError):
        r.recorded()
    o = dfrsw.kiops_opts(tol=1e-8, replay=r)
    assert ctypes.addressof(o.replay.contents) == ctypes.addressof(st)
    assert not dfrsw.kiops_opts(tol=1e-8).replay


def test_header_is_self_contained_c99(tmp_path):
    # a C caller includes the header alone
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "only_header.c"
    src.write_text(f'#include "{HEADER}"\nint main(void) {{ return DFR_OK; }}\n')
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-pedantic", "-c", str(src), "-o", str(tmp_path / "o.o")],
                   check=True, capture_output=True)
