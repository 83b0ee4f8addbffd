"""Host logic of the autotuner table (no GPU)."""
from paper_1512_02548_amd import tune
from paper_1512_02548_amd import workloads as wl


def test_classes_and_table_roundtrip(tmp_path):
    specs = wl.batch_tank_specs(count=20, seed=5)
    cl = tune.classes(specs)
    assert sum(len(v) for v in cl.values()) == 20
    assert all(P in (4, 6, 8) and nz in (2, 4, 8) for (P, nz) in cl)
    table = {k: 1 + (i % 4) for i, k in enumerate(sorted(cl))}
    path = tmp_path / "tiles.json"
    tune.save(table, path)
    assert tune.load(path) == table
    s = specs[0]
    assert tune.tiles_for(table, s) == table[(s.P, s.nz)]
    assert tune.tiles_for(None, s) == 0
