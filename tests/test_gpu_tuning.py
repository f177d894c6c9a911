"""The autotune table with a device: a timed choice lands in the process-wide
table under the batch's size class, and an imported entry is used in place of
timing.  Tiles only regroup atoms across workgroups, so every tile size gives
bit-identical results."""

import pytest
import torch

from paper_2501_11592_amd import clomp as C
from paper_2501_11592_amd import workloads as W
from tests.gpu_helpers import dev

pytestmark = pytest.mark.gpu


def _items(sigs):
    return [dict(At=dev(s.At), m=s.m, y=dev(s.y), k=s.k) for s in sigs]


def test_autotune_table_written_then_used(tmp_path):
    C.tuning_table_clear()
    sigs = [W.single_small(300 + i, n=3000, m=200, k=20) for i in range(3)]
    items = _items(sigs)
    fl = C.FLAG_CORR_FLOW
    tuned = C.Solver(0, method="clomp", flags=fl | C.FLAG_AUTOTUNE)
    a = tuned.solve_batch(items)
    torch.cuda.synchronize()
    lines = C.tuning_table_export().splitlines()
    assert lines[0] == "clomp-tuning 1" and len(lines) == 2, lines
    key, kb = lines[1].split(" ")
    arch, dt, meth, sched, mo, no, co = key.split("/")
    print(f"autotuned {key} -> {kb} KB")
    # m = 200 (octave 7), n = 3000 (octave 11), three iterated signals (octave 1)
    assert arch.startswith("gfx") and (dt, meth, sched) == ("f32", "clomp", "corr")
    assert (mo, no, co) == ("m7", "n11", "c1")
    assert int(kb) == tuned.get_tuning()["pass_tile_kb"] in (128, 256, 512, 1024, 2048)

    # a saved table from "an earlier process": 384 KB is not a timing
    # candidate, so a fresh handle that reports it took it from the table
    f = tmp_path / "tuning.txt"
    f.write_text(f"clomp-tuning 1\n{key} 384\n")
    C.tuning_table_clear()
    assert C.load_tuning_table(f) == 1
    fresh = C.Solver(0, method="clomp", flags=fl | C.FLAG_AUTOTUNE)
    plain = C.Solver(0, method="clomp", flags=fl)
    b = fresh.solve_batch(items)
    c = plain.solve_batch(items)
    torch.cuda.synchronize()
    assert fresh.get_tuning()["pass_tile_kb"] == 384
    assert plain.get_tuning()["pass_tile_kb"] == 256
    for i in range(len(sigs)):
        for out in (a, b):
            assert torch.equal(out.support[i], c.support[i])
            assert torch.equal(out.x[i], c.x[i])
    # the table still holds the imported entry, untouched by the solve
    assert C.tuning_table_export() == f"clomp-tuning 1\n{key} 384\n"
    for s in (tuned, fresh, plain):
        s.close()
    C.tuning_table_clear()
