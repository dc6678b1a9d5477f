"""Host-side logic of bench.py (CPU only): the engine-code hash that decides
whether the committed chain traffic counters apply to the sources, and the
per-site algorithmic flop count the roofline line divides by."""
import os
import shutil

import bench

SOURCES = bench.ENGINE_SOURCES


def _copy_sources(tmp_path):
    dst = tmp_path / "paper_2507_18700_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in SOURCES:
        shutil.copy(os.path.join(bench.ROOT, "paper_2507_18700_amd", "csrc", f), dst / f)
    return dst


def _hash_at(root, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(root))
    return bench.engine_source_hash()


def test_hash_ignores_comments_and_whitespace(tmp_path, monkeypatch):
    ref = bench.engine_source_hash()
    dst = _copy_sources(tmp_path)
    p = dst / "engine_impl.h"
    src = p.read_text()
    p.write_text("// a new leading comment\n/* and a block\n   comment */\n" + src.replace("\n", "\n  ", 5) + "\n\n")
    assert _hash_at(tmp_path, monkeypatch) == ref


def test_hash_follows_code_changes(tmp_path, monkeypatch):
    ref = bench.engine_source_hash()
    dst = _copy_sources(tmp_path)
    p = dst / "kernels.h"
    p.write_text(p.read_text() + "\nstatic const int hash_probe = 1;\n")
    assert _hash_at(tmp_path, monkeypatch) != ref


def test_site_flops_of_the_2d_glu_cell():
    # 2D cell [2 d_h -> 3 d_h], GLU [d_h -> 2 d_h], amplitude head [d_h -> 2], 2 flops per MAC
    assert bench.site_flops(128) == 2 * 256 * 384 + 2 * 128 * 256 + 2 * 128 * 2 == 262656
