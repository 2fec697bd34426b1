"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, and host-only calls behave."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "mulment.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ["mm_layout", "mm_khop_build", "mm_repulsion", "mm_sweep", "mm_coarsen",
              "mm_prolong", "mm_objective", "mm_full_stress"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    import paper_1506_04383_amd as mm

    L = mm.lib()
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert set(declared_symbols()) == set(mm.EXPORTS)


def test_params_default_is_paper_configuration():
    import paper_1506_04383_amd as mm

    p = mm.default_params()
    assert (p.k, p.alpha0, p.alpha_decay, p.alpha_min, p.iters_per_round) == (1, 1.0, 0.3, 0.008, 2)
    assert (p.b, p.f, p.eps_final) == (2.0, 20.0, 1e-4)
    assert p == mm.Params()


def test_null_arguments_are_rejected_without_device():
    import paper_1506_04383_amd as mm

    L = mm.lib()
    assert L.mm_params_default(None) == 1
    assert b"NULL" in L.mm_last_error()
    assert L.mm_sync(None) == 1
    assert L.mm_khop_info(None, None, None, None) == 1
