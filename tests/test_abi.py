"""The C-ABI library loads (no GPU needed) and exports every function that
include/halign.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "halign.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(halign_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_named_calls():
    names = declared()
    for must in ("halign_sw_batch", "halign_merge", "halign_msa", "halign_center_exact",
                 "halign_featurize", "halign_mlp_forward", "halign_mlp_backward", "halign_adam_step",
                 "halign_topk_center", "halign_train_proposer", "halign_center_learned"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1704_00878_amd import _build
    if not os.path.exists(_build.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(_build.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_raises_without_library(monkeypatch, tmp_path):
    import paper_1704_00878_amd as H
    monkeypatch.setattr(H, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(H, "_lib", None)
    with pytest.raises(RuntimeError):
        H.lib()
