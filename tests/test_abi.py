"""The C-ABI library loads on the CPU host and exports every entry point that
include/pr.h declares (no compute call: that needs a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pr.h")).read()
    return sorted(set(re.findall(r"^\s*(?:pr_status|const char\*)\s+(pr_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("pr_create_problem", "pr_fine_propagate", "pr_coarse_sweep",
                     "pr_parareal_iterate", "pr_adjoint"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2502_08370_amd import _binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libpr.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(B.exported_symbols()) == set(declared_symbols())


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2502_08370_amd import _binding as B
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "libpr.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(ImportError):
        B.lib()


def test_null_handle_is_rejected_without_a_gpu():
    """Entry points validate their handle before any device call: a NULL handle gives
    PR_EINVAL and a message (host-only, so it runs here)."""
    from paper_2502_08370_amd import _binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libpr.so is not built (run __graft_entry__.build())")
    lib = B.lib()
    assert lib.pr_profile_control(None, 3) == 1
    assert b"NULL" in lib.pr_last_error()
