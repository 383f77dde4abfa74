"""The C-ABI library loads and exports every function include/crop.h
declares (no compute calls: this runs without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crop.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(crop_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_calls():
    names = declared_functions()
    for need in ("crop_create", "crop_destroy", "crop_set_partitions", "crop_set_seed",
                 "crop_load_transactions", "crop_load_outer", "crop_run_exact",
                 "crop_result_sizes", "crop_read_partition"):
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_1210_0461_amd as crop
    out = subprocess.run(["nm", "-D", "--defined-only", crop.LIB_PATH], check=True,
                         capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (crop_[a-z0-9_]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_binding_names_match_c_functions():
    import paper_1210_0461_amd as crop
    for n in declared_functions():
        assert hasattr(crop, n), n


def test_static_calls_without_gpu():
    import paper_1210_0461_amd as crop
    assert crop.crop_abi_version() == 4
    assert crop.crop_status_string(0) == "ok"
    assert crop.crop_status_string(-4) == "output buffer too small"


def test_no_oracle_in_product_sources():
    pkg = os.path.join(ROOT, "paper_1210_0461_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liborc" not in text and "crop_oracle" not in text, f
