"""Host logic of the GEMM autotuner: which shapes a run times, and how an existing table is read."""
from paper_2205_05175_amd.autotune import load_entries, shapes_to_tune

SHAPES = {
    (20, 76, 115520, True, False, 0, 0): 5,   # 2 M N K = 3.5e8
    (400, 1520, 1520, True, True, 0, 0): 3,   # 1.85e9
    (250, 1000, 1000, True, True, 0, 1): 1,   # exactly 5e8
    (20, 8000, 76, True, False, 0, 0): 1,     # 2.4e7
}


def test_all_shapes_without_a_bound_in_a_fixed_order():
    got = shapes_to_tune(SHAPES)
    assert [s for s, _ in got] == sorted(SHAPES)
    assert dict(got) == SHAPES


def test_max_flops_keeps_only_the_products_below_it():
    got = dict(shapes_to_tune(SHAPES, 5e8))
    assert set(got) == {(20, 76, 115520, True, False, 0, 0), (20, 8000, 76, True, False, 0, 0)}
    assert got[(20, 76, 115520, True, False, 0, 0)] == 5
    assert shapes_to_tune(SHAPES, 1e7) == []


def test_load_entries_reads_keys_and_keeps_lines(tmp_path):
    p = tmp_path / "t.txt"
    p.write_text("# header\n"
                 "2 20 76 30400 1 0 0 0 1 32032 64 256  # (20,76), 5 per call\n"
                 "1 400 5776 400 1 0 0 0 1 64032 32 1\n"
                 "1 2 3\n")
    e = load_entries(str(p))
    assert set(e) == {(2, 20, 76, 30400, 1, 0, 0, 0), (1, 400, 5776, 400, 1, 0, 0, 0)}
    assert e[(2, 20, 76, 30400, 1, 0, 0, 0)].endswith("5 per call")
    assert load_entries(str(tmp_path / "missing.txt")) == {}


def test_committed_table_is_well_formed():
    # every line parses; the split-BF16 context keeps tile choices only for its products below the
    # split threshold (a split-BF16 entry, or one for a product that goes out grouped, would take the
    # product off its grouped launch)
    import os
    from paper_2205_05175_amd import TUNING_PATH
    lines = [l for l in open(TUNING_PATH) if l.split("#")[0].strip()]
    e = load_entries(TUNING_PATH)
    assert len(e) == len(lines) and os.path.getsize(TUNING_PATH) > 0
    for key, line in e.items():
        f = [int(x) for x in line.split("#")[0].split()]
        prec, M, N, K = key[:4]
        assert prec in (0, 1, 2) and f[8] in (1, 2)
        if prec == 2:
            assert f[8] == 1 and 2.0 * M * N * K < 5e8
