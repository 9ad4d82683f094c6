"""Host-side tuning logic: the batched schedule planner and the LDS layout
estimate, with synthetic inputs (no GPU)."""
from paper_1804_05028_amd import autotune as at
from paper_1804_05028_amd import decompose as dc


def test_schedule_sizes_include_remainders():
    assert at.schedule_sizes(36, (4, 8, 12, 16)) == [4, 8, 12, 16]   # 36 % 8 = 36 % 16 = 4
    assert at.schedule_sizes(16, (4, 6, 16)) == [4, 6, 16]           # 16 % 6 = 4
    assert at.schedule_sizes(3, (4, 8)) == [3]
    assert at.schedule_sizes(20, (6,)) == [2, 6]


def test_plan_schedule_picks_the_cheapest_tiling():
    # per-launch times of the 36-site triangular momentum sectors (ms, lanes)
    best_of = {4: (508.0, 2), 8: (655.0, 2), 12: (826.0, 4), 16: (906.0, 4)}
    plan = at.plan_schedule(36, (4, 8, 12, 16), best_of)
    assert plan["batch"] == 16
    assert plan["groups"] == [(0, 16, 4), (16, 16, 4), (32, 4, 2)]
    assert plan["est_ms"] == 2 * 906.0 + 508.0
    # make the 12-sector launch cheap enough and the tiling changes
    best_of[12] = (700.0, 4)
    plan = at.plan_schedule(36, (4, 8, 12, 16), best_of)
    assert plan["batch"] == 12 and plan["groups"] == [(0, 12, 4), (12, 12, 4), (24, 12, 4)]


def test_plan_schedule_ties_and_small_sets():
    assert at.plan_schedule(8, (4, 8), {4: (1.0, 1), 8: (2.0, 2)})["batch"] == 4   # equal cost: smaller batch
    plan = at.plan_schedule(3, (4, 8), {3: (5.0, 2)})
    assert plan["groups"] == [(0, 3, 2)] and plan["est_ms"] == 5.0


def test_table_layout_counts_the_position1_table():
    args = dict(n_sub=4, sub_bits=9, n_perms=400, sym_entries=5000, n_elems=864, n_bonds=108)
    one = dc.table_layout(**args)
    two = dc.table_layout(**args, two_stage=True)
    assert one is not None and two is not None
    assert two[0] == one[0] and two[1] - one[1] == (2 * 400 + 15) // 16 * 16
