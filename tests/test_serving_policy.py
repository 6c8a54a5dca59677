"""CPU tests of the serving admission policy (no GPU)."""
from paper_1511_05578_amd.serving import plan_admission


def fp(L, b):
    return {64: 1, 128: 4, 256: 16, 512: 64}[L] * b


def test_groups_same_L_in_arrival_order():
    g = plan_admission([64, 128, 64, 64, 256], 0, 1000, free_slots=2, max_batch=4, footprint=fp)
    assert g == [[0, 2, 3], [1]]


def test_budget_shrinks_group_then_blocks_head():
    # head L=512 needs 64 per request: budget 100 admits one of them, then stops
    g = plan_admission([512, 512, 64], 0, 100, free_slots=3, max_batch=4, footprint=fp)
    assert g == [[0]]
    # nothing fits: head of line waits, younger small requests do not overtake it
    g = plan_admission([512, 64], 50, 100, free_slots=2, max_batch=4, footprint=fp)
    assert g == []


def test_max_batch_and_slots():
    g = plan_admission([64] * 10, 0, 1000, free_slots=2, max_batch=3, footprint=fp)
    assert g == [[0, 1, 2], [3, 4, 5]]
    assert plan_admission([], 0, 1000, 4, 4, fp) == []
    assert plan_admission([64], 0, 1000, 0, 4, fp) == []


def test_batch_cap():
    from paper_1511_05578_amd.serving import batch_cap
    assert [batch_cap(L) for L in (64, 128, 256, 512, 1024)] == [4, 4, 2, 1, 1]
    assert batch_cap(64, max_batch=8) == 8
    g = plan_admission([512, 512, 64, 64], 0, 1000, free_slots=3, max_batch=batch_cap, footprint=fp)
    assert g == [[0], [1], [2, 3]]
