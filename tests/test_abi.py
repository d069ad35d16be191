"""The C-ABI library loads and exports every function include/empp.h
declares; host-only entry points validate their arguments.  No compute
calls (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "empp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(empp_[a-z_]+)\s*\(", src)))


def test_header_matches_binding_list():
    from paper_2605_05543_amd import _lib

    assert _declared() == sorted(_lib.EXPORTS)


def test_every_declared_symbol_is_exported():
    from paper_2605_05543_amd import _lib

    for name in _declared():
        assert hasattr(_lib.lib, name), name
    # and nothing from the oracle leaks into the product library
    syms = os.popen(f"nm -D --defined-only {_lib.LIB_PATH}").read()
    assert "oracle_" not in syms


def test_workspace_size_and_validation():
    from paper_2605_05543_amd import _lib

    cfg = _lib.Config(n=65536, depth=512, q=-1.602176634e-19, m=9.1093837015e-31, dt=1e-13)
    nbytes = _lib.empp_workspace_size(cfg)
    # the two rings (positions, velocities) and the pass's light-cone
    # records, 32 bytes per (particle, slot) each, plus the per-chunk
    # partials (at most 128 chunks x 12 doubles per target) and small
    # per-particle arrays
    ring = 65536 * 512 * 32 * 3
    partials = 128 * 12 * 65536 * 8
    assert ring + partials <= nbytes < ring + partials + 64 * 2**20
    # the warm-start cache adds N*N uint16 brackets
    cfg.guess = _lib.EMPP_GUESS_PREVIOUS
    warm = _lib.empp_workspace_size(cfg)
    assert ring + 65536 * 65536 * 2 <= warm < nbytes + 65536 * 65536 * 2
    for bad in (dict(n=1), dict(depth=1), dict(depth=4065), dict(dt=0.0), dict(dt=float("nan")), dict(m=-1.0),
                dict(ext_field=3), dict(precision=7), dict(guess=9), dict(guess_group_log2=5),
                dict(guess_group_log2=17), dict(recon=2), dict(guess=1, depth=4), dict(guess=3, depth=2)):
        c = _lib.Config(n=64, depth=32, q=-1.0, m=1.0, dt=1e-13)
        for k, v in bad.items():
            setattr(c, k, v)
        with pytest.raises(_lib.EmppError) as ei:
            _lib.empp_workspace_size(c)
        assert ei.value.status in (_lib.EMPP_EINVAL, _lib.EMPP_EUNSUPPORTED), bad


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2605_05543_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "empp_oracle" not in text, f
