"""Host-side checks of the C ABI (no GPU compute)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "nmg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nmg_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2603_01064_amd import nmg
    try:
        lib = nmg.load_library()
    except ImportError as e:
        pytest.fail(str(e))
    names = _declared()
    assert "nmg_solve" in names and "nmg_train_step" in names
    missing = [n for n in names if getattr(lib, n, None) is None]
    assert not missing, missing


def test_binding_names_match_abi():
    from paper_2603_01064_amd import nmg
    for n in ("setup_hierarchy", "load_smoother_weights", "vcycle", "solve", "train_step"):
        assert callable(getattr(nmg, n))


def test_setup_rejects_bad_shapes_on_host():
    """Argument checks run before any device work (n not 2^k-1, levels)."""
    from paper_2603_01064_amd import nmg
    nmg.load_library()
    for kw in (dict(n=100, s=0.01, levels=3), dict(n=15, s=0.01, levels=5), dict(n=15, s=-1.0, levels=2)):
        with pytest.raises(nmg.NMGError) as ei:
            nmg.setup_hierarchy(nmg.Problem(**kw))
        assert ei.value.code == -2
