"""Host-only checks of the C ABI library (no GPU calls)."""
import os
import re
import subprocess

import pytest

import paper_2604_12241_amd as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "amlm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(amlm_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    declared = _header_functions()
    assert declared == sorted(A.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (amlm_[a-z_]+)\b", out))
    missing = [f for f in declared if f not in exported]
    assert not missing, missing


def test_library_loads_and_reports_columns():
    L = A.lib()
    for name in A.EXPORTS:
        assert getattr(L, name) is not None
    assert A.amlm_num_columns(A.params(L=6)) == 9
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_FAN_OUT | A.AMLM_CYCLES, L=3)) == 3
    # the unordered scatter-gather modifier adds no column and needs AMLM_SG
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_ALL | A.AMLM_SG_UNORDERED, L=4)) == 7
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_FAN_OUT | A.AMLM_SG_UNORDERED, L=4)) == 0
    # the distinct-counterparty columns come after the cycle columns
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_ALL | A.AMLM_DEG_OUT | A.AMLM_DEG_IN, L=4)) == 9
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_DEG_IN, L=4)) == 1
    # participation columns: one per requested SG / GS, last; need SG or GS, not the phase order
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_ALL | A.AMLM_DEG_IN | A.AMLM_PART, L=4)) == 10
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_GS | A.AMLM_PART, L=4)) == 2
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_FAN_IN | A.AMLM_CYCLES | A.AMLM_PART, L=4)) == 0
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_SG | A.AMLM_SG_PHASE | A.AMLM_PART, L=4)) == 0
    # four size bins of SG, last; need SG, not the phase order
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_ALL | A.AMLM_PART | A.AMLM_SG_SIZES, L=4)) == 13
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_GS | A.AMLM_SG_SIZES, L=4)) == 0
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_SG | A.AMLM_SG_PHASE | A.AMLM_SG_SIZES, L=4)) == 0
    assert A.amlm_num_columns(A.params(L=9)) == 0          # invalid L
    assert A.amlm_num_columns(A.params(k=0)) == 0          # invalid k
    assert A.amlm_num_columns(A.params(delta=-1)) == 0     # invalid window
    assert A.amlm_num_columns(A.params(patterns=1 << 12)) == 0  # unknown pattern bit
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_ALL | (1 << 12), L=4)) == 0
    assert A.amlm_num_columns(A.params(patterns=A.AMLM_ALL | (1 << 13), L=4)) == 0
    assert A.amlm_num_columns(A.params(schedule=4)) == 0   # unknown schedule


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle and fails loudly without its
    library (no CPU fallback)."""
    pkg = os.path.join(ROOT, "paper_2604_12241_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "liboracle" not in src, f
