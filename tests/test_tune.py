"""Host logic of the Jacobi tile autotuner (no GPU)."""
import pytest

from paper_2008_08825_amd import tune


def test_candidates_respect_kernel_constraints():
    assert tune.candidates(64) == [(1, 64), (2, 64), (4, 64)]
    for np_ in range(64, 2049, 64):
        for kc, rr in tune.candidates(np_):
            assert np_ % (16 * kc) == 0 and kc & (kc - 1) == 0
            assert rr % 64 == 0 and np_ % rr == 0
    assert (1, 256) in tune.candidates(256) and (16, 256) in tune.candidates(1024)
    with pytest.raises(ValueError):
        tune.candidates(100)


def test_table_validation_and_round_trip(tmp_path):
    table = [(64, 1, 64), (512, 4, 256), (1024, 8, 256)]
    p = tmp_path / "tiles.json"
    tune.save(table, str(p), {"note": "test"})
    assert tune.load(str(p)) == table
    for bad in ([(64, 3, 64)], [(64, 1, 96)], [(128, 1, 64), (64, 1, 64)], [(0, 1, 64)]):
        with pytest.raises(ValueError):
            tune.validate(bad)


def test_packaged_table_is_valid():
    """Rows for the padded orders of the 256-problem batch (128..1024), each a valid candidate."""
    table = tune.packaged()
    assert [r[0] for r in table] == list(range(128, 1025, 64))
    for np_, kc, rr in table:
        assert (kc, rr) in tune.candidates(np_) and kc <= tune.default_kc(np_)


def test_builtin_batch_choice_is_a_candidate():
    for np_ in range(64, 4097, 64):
        kc, rr = tune.builtin_batch_tiles(np_)
        assert (kc, rr) in tune.candidates(np_) and kc <= tune.default_kc(np_)
