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
