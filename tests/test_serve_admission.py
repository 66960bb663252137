"""Host logic of the serving loop: first-come-first-served admission under slot and
HBM limits, request footprints, and the separable initial field (no GPU)."""
from collections import deque

import numpy as np

from paper_1604_03570_amd import boxtile as bt
from paper_1604_03570_amd import inputs as I
from paper_1604_03570_amd.serve import Admission, _Shapes, offered_load


def _reqs(sizes):
    return deque(I.Request(i, 0.0, 32, 32, 10, "f64", (0.5, 0.5, 0.5)) for i in range(len(sizes))), list(sizes)


def test_admission_is_fifo_and_respects_the_budget():
    q, sizes = _reqs([40, 30, 50, 10])
    fp = lambda r: sizes[r.rid]
    adm = Admission(budget=100, max_slots=8)
    got = adm.admit(q, fp)
    assert [(r.rid, n) for r, n in got] == [(0, 40), (1, 30)]  # 50 does not fit; 10 waits behind it
    assert adm.used == 70 and adm.active == 2 and [r.rid for r in q] == [2, 3]
    adm.release(40)
    got = adm.admit(q, fp)
    assert [(r.rid, n) for r, n in got] == [(2, 50), (3, 10)]
    assert adm.used == 90 and adm.active == 3 and not q


def test_admission_slot_limit_and_oversize_rejection():
    q, sizes = _reqs([5, 500, 5, 5, 5])
    fp = lambda r: sizes[r.rid]
    adm = Admission(budget=100, max_slots=2)
    got = adm.admit(q, fp)
    assert [(r.rid, n) for r, n in got] == [(0, 5), (1, None), (2, 5)]  # 500 can never fit: rejected
    assert adm.active == 2 and [r.rid for r in q] == [3, 4]
    assert adm.admit(q, fp) == []  # slots full
    adm.release(5)
    assert [(r.rid, n) for r, n in adm.admit(q, fp)] == [(3, 5)]


def test_footprint_is_two_multifabs_of_the_request_shape():
    sh = _Shapes()
    for n, be, dt in [(96, 64, "f64"), (32, 64, "f32"), (256, 32, "f64")]:
        r = I.Request(0, 0.0, n, be, 10, dt, (0.5, 0.5, 0.5))
        ba = bt.BoxArray.chop(I.domain_box(n), min(be, n))
        assert sh.footprint(r) == 2 * ba.multifab_bytes(1, 1, bt.F64 if dt == "f64" else bt.F32)
        assert sh.footprint(r) >= 2 * n ** 3 * (8 if dt == "f64" else 4)


def test_separable_gaussian_matches_the_plain_one():
    for c in [(0.5, 0.5, 0.5), (0.3, 0.6, 0.7)]:
        a = I.gaussian(32, c)
        b = I.gaussian_separable(32, c)
        assert np.abs(a - b).max() <= 4e-16 * np.abs(a).max()


def test_request_stream_shape():
    rs = I.request_stream(2000, 200.0, seed=0)
    assert len(rs) == 2000
    assert all(32 <= r.n <= 256 and r.n % 32 == 0 and r.box_edge in (32, 64) and 10 <= r.steps <= 200 for r in rs)
    span = rs[-1].arrival - rs[0].arrival
    assert 8.0 < span < 12.0  # 2000 Poisson arrivals at 200/s
    assert 0.4 < sum(r.dtype == "f32" for r in rs) / len(rs) < 0.6
    assert 0.5e11 < offered_load(rs) < 2e11
