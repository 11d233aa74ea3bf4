"""Host-side logic of the checkpointed autograd function (no GPU): the automatic
checkpoint interval from a memory budget."""
from types import SimpleNamespace

from paper_2002_08377_amd import rt
from paper_2002_08377_amd.autograd import auto_checkpoint_interval, record_bytes


def _system(N, K, dtype):
    return SimpleNamespace(mesh=SimpleNamespace(n_cells=N), angles=SimpleNamespace(K=K),
                           params=SimpleNamespace(dtype=dtype))


def test_record_bytes():
    assert record_bytes(_system(1000, 80, rt.F32)) == 1000 * (80 * 4 + rt.SRC_TAPE * 8)
    assert record_bytes(_system(1000, 80, rt.F64)) == 1000 * (80 * 8 + rt.SRC_TAPE * 8)


def test_auto_interval_tapes_everything_when_it_fits():
    s = _system(884736, 80, rt.F32)
    rec = record_bytes(s)
    assert auto_checkpoint_interval(s, 40, 40 * rec) == 40
    assert auto_checkpoint_interval(s, 40, 10 ** 15) == 40


def test_auto_interval_is_the_longest_segment_that_fits():
    s = _system(884736, 80, rt.F32)
    rec = record_bytes(s)
    ckpt = rec + 40 * 884736
    for budget_records in (1, 2, 7, 8, 13, 39):
        L = auto_checkpoint_interval(s, 40, budget_records * rec)
        n_ckpt = lambda L: (40 + L - 1) // L - 1
        assert L * rec + n_ckpt(L) * ckpt <= budget_records * rec or L == 1
        # one step longer would not fit
        if L < 40:
            assert (L + 1) * rec + n_ckpt(L + 1) * ckpt > budget_records * rec


def test_auto_interval_degenerate_cases():
    s = _system(10, 8, rt.F64)
    assert auto_checkpoint_interval(s, 0, 0) == 1
    assert auto_checkpoint_interval(s, 5, 0) == 1   # nothing fits: one step per segment
