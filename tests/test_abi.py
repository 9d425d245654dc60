"""CPU-side checks of the boundary: the built library loads and exports every
entry point include/mp_weno.h declares (no compute calls, no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mp_weno.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mp_weno_\w+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("mp_weno_init", "mp_weno_rhs", "mp_weno_step", "mp_weno_dt"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2608_00746_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libmpweno.so not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) == set(binding.EXPORTED)
    lib.mp_weno_abi_version.restype = ctypes.c_int32
    assert lib.mp_weno_abi_version() == 3
    lib.mp_weno_max_phases.restype = ctypes.c_int32
    assert lib.mp_weno_max_phases() >= 5


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2608_00746_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(ImportError):
        binding.lib()


def test_product_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2608_00746_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", txt).split("\"\"\"")[0] or \
                    "import oracle" not in txt, f
                assert "from oracle" not in txt and "import oracle" not in txt, f
                assert "mpo_" not in txt, f
