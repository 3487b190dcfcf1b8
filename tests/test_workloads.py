"""Host logic of the seeded workloads and the benchmark's helpers (CPU only):
the served request stream, re-plan thresholds, the day's anatomy and the
tile order used to cut row shares."""
import numpy as np

from workloads import (BLADDER, NORMAL, PAPER_SCALE, PTV, RECTUM, SMALL, day_geometry, penalty_table,
                       replan_penalty_table, served_requests)


def test_served_requests_deterministic_and_shaped():
    a = served_requests(10.0, 400, seed=5)
    b = served_requests(10.0, 400, seed=5)
    assert [(r.arrival_s, r.patient, r.replan) for r in a] == [(r.arrival_s, r.patient, r.replan) for r in b]
    t = np.array([r.arrival_s for r in a])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 0.1) < 0.02           # Poisson at 10 per second
    frac = np.mean([r.replan for r in a[1:]])
    assert 0.22 < frac < 0.38                               # 30 % re-plans
    first = {}
    for i, r in enumerate(a):
        if not r.replan:
            assert r.patient == i and r.spec.seed == 1000 + i
            assert np.array_equal(r.table, penalty_table(r.spec))
            first[r.patient] = r.spec
        else:
            assert r.patient in first and r.spec == first[r.patient]   # an earlier patient


def test_replan_thresholds_within_their_ranges():
    rng = np.random.default_rng(0)
    base = penalty_table(SMALL)
    for _ in range(200):
        t = replan_penalty_table(SMALL, rng)
        # rows are structure ids: the target's two thresholds are redrawn
        assert 66.0 <= t[PTV, 0] < 74.0 and t[PTV, 0] == t[PTV, 1]
        others = [NORMAL, RECTUM, BLADDER]
        assert np.array_equal(t[others, 0], base[others, 0])
        ratio = t[others, 1] / base[others, 1]
        assert np.all((ratio >= 0.9) & (ratio < 1.1))
        assert np.array_equal(t[:, 2:], base[:, 2:])          # weights unchanged


def test_day_geometry_scales():
    d = day_geometry(PAPER_SCALE)
    assert (d.nx, d.ny, d.nz, d.h, d.n_beams, d.beamlet, d.sigma, d.tau) == \
        (PAPER_SCALE.nx, PAPER_SCALE.ny, PAPER_SCALE.nz, PAPER_SCALE.h, PAPER_SCALE.n_beams,
         PAPER_SCALE.beamlet, PAPER_SCALE.sigma, PAPER_SCALE.tau)
    assert d.r_ptv == PAPER_SCALE.r_ptv * 0.95 and d.r_bladder == PAPER_SCALE.r_bladder * 1.2
    assert d.r_rectum == PAPER_SCALE.r_rectum * 0.9


def test_tile_order_matches_nested_tiles():
    import bench
    for nx, ny, nz in ((9, 7, 5), (8, 8, 4), (1, 1, 1), (5, 13, 3)):
        want = []
        for z0 in range(0, nz, 2):
            for y0 in range(0, ny, 4):
                for x0 in range(0, nx, 4):
                    for z in range(z0, min(z0 + 2, nz)):
                        for y in range(y0, min(y0 + 4, ny)):
                            for x in range(x0, min(x0 + 4, nx)):
                                want.append(x + nx * (y + ny * z))
        assert bench.tile_order(nx, ny, nz).tolist() == want


def test_shared_live_time_by_hand():
    import bench
    # patient 0: [0, 10) and [5, 20) overlap for 5 ms each way; patient 1 alone;
    # a third plan of patient 0 inside [12, 14) overlaps the second only
    live = [(0.0, 10.0), (5.0, 20.0), (0.0, 30.0), (12.0, 14.0)]
    patients = [0, 0, 1, 0]
    shared, total, partners = bench.shared_live_time(live, patients)
    assert total == 10 + 15 + 30 + 2
    assert shared == 5 + (5 + 2) + 0 + 2      # overlaps of [5,20) with [0,10) and [12,14) are disjoint
    assert partners == 3
    assert bench.shared_live_time([(0.0, 1.0)], [7]) == (0.0, 1.0, 0)
