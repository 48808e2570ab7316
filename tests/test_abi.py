"""The C ABI library loads and exports every function include/sos.h declares (CPU only)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sos.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sos_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sos_setup", "sos_step", "sos_solve", "sos_batch_setup", "sos_batch_solve"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1708_04174_amd import binding as B
    lib = B.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(B.EXPORTED) == declared_functions()


def test_default_settings_without_gpu():
    from paper_1708_04174_amd import binding as B
    s = B.sos_default_settings()
    assert s.tol == 1e-4 and s.max_iters == 2000 and s.check_every == 10 and s.alpha == 1.0
    assert s.precision == B.SOS_FP64 and s.partition == B.SOS_PART_PAPER


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1708_04174_amd import binding as B
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "libsos.so"))
    with pytest.raises(ImportError):
        B.load()


def test_settings_defaults_cover_every_field():
    from paper_1708_04174_amd import binding as B
    s = B.sos_default_settings()
    assert s.polish_iters == 1 and s.block_threads == 0 and s.eig_form == 0 and s.warm_budget == 0


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes mirrors of sos_settings and sos_info against the C compiler's layout of
    # include/sos.h (sizes and every field offset)
    import ctypes as C
    import shutil
    import subprocess
    from paper_1708_04174_amd import binding as B
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sos.h"', 'int main(void) {']
    for st in (B.sos_settings, B.sos_info):
        lines.append(f'printf("{st.__name__} size %zu\\n", sizeof({st.__name__}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{st.__name__} {f} %zu\\n", offsetof({st.__name__}, {f}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c_layout = {(l.split()[0], l.split()[1]): int(l.split()[2]) for l in out if l.strip()}
    for st in (B.sos_settings, B.sos_info):
        assert c_layout[(st.__name__, "size")] == C.sizeof(st)
        for f, _ in st._fields_:
            assert c_layout[(st.__name__, f)] == getattr(st, f).offset, (st.__name__, f)


def test_bench_refuses_more_than_one_gpu():
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["n_gpus"] == 2 and "one GPU" in rec["error"]
