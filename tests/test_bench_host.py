"""Host logic of bench.py: the algorithmic byte count of the product and the
code hash that ties a counter summary to the sources it was taken on."""
from __future__ import annotations

import os
import shutil

import bench


def test_spmm_bytes_formula():
    # 128^3 Helmholtz at p = 32, complex128: values 16 B and int32 column
    # indices per stored entry, int32 row pointers, Z read once, Y written once
    n, nnz, p = 2097152, 14581760, 32
    assert bench.spmm_bytes(n, nnz, p, 16) == nnz * 20 + 4 * (n + 1) + 2 * n * p * 16
    # the grid-stencil product reads no column indices
    assert bench.spmm_bytes(n, nnz, p, 16, colind=False) == 2389180420
    assert bench.spmm_bytes(n, nnz, p, 8, colind=False) == nnz * 8 + 4 * (n + 1) + 2 * n * p * 8


def _copy_sources(tmp_path):
    for item in bench.SPMM_SOURCES:
        rel = item[0] if isinstance(item, tuple) else item
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, rel), dst)


def test_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    base = bench.source_hash(bench.SPMM_SOURCES)
    _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.source_hash(bench.SPMM_SOURCES) == base
    grid = tmp_path / "paper_1601_05362_amd/csrc/grid.hpp"
    text = grid.read_text()
    grid.write_text("// an added comment\n" + text.replace("namespace blk {", "namespace blk {  /* note */", 1))
    assert bench.source_hash(bench.SPMM_SOURCES) == base
    grid.write_text(text.replace("constexpr int GRID_WG_PER_CU = 2;", "constexpr int GRID_WG_PER_CU = 3;", 1))
    assert bench.source_hash(bench.SPMM_SOURCES) != base

