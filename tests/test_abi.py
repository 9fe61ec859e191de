"""The C-ABI library loads and exports every entry point its header declares.

Runs without a GPU: only dlopen and symbol lookup, no compute calls.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cryosplat.h")
LIB = os.path.join(ROOT, "paper_2508_04929_amd", "libcryosplat.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("cs_create", "cs_destroy", "cs_last_error", "cs_render",
                     "cs_render_backward", "cs_loss_and_grad", "cs_adam_step", "cs_pair_count"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcryosplat.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcryosplat.so not built")
def test_binding_loads_and_declares_signatures():
    from paper_2508_04929_amd import binding
    lib = binding.load_library()
    for name in binding.EXPORTS:
        assert hasattr(lib, name)
    assert set(binding.EXPORTS) == set(declared_functions())


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2508_04929_amd import binding
    with pytest.raises(binding.CryoSplatError):
        binding.load_library(str(tmp_path / "missing.so"))


PROBE = os.path.join(ROOT, "paper_2508_04929_amd", "libcsprobe.so")


@pytest.mark.skipif(not os.path.exists(PROBE), reason="libcsprobe.so not built")
def test_probe_library_loads_and_exports_its_probes():
    from paper_2508_04929_amd import probe
    lib = probe.load()
    for name in ("csp_fma", "csp_exp", "csp_lds", "csp_mfma", "csp_copy", "csp_wall_clock_khz"):
        assert hasattr(lib, name)
