"""Host logic of the serving loop (no GPU): which waiting requests share one
block problem, and the request trace generator."""
from paper_1508_02897_amd.serving import Request, coalesce_group, make_requests


def _req(rid, N, medium, ns, arrival=0.0):
    return Request(rid=rid, N=N, medium_seed=medium, n_sources=ns, source_seed=rid,
                   arrival=arrival)


def test_group_takes_arrived_requests_on_the_same_factor_in_arrival_order():
    pending = [_req(0, 4096, 3, 4), _req(1, 4096, 2, 5), _req(2, 4096, 3, 6),
               _req(3, 2048, 3, 2), _req(4, 4096, 3, 5), _req(5, 4096, 3, 1)]
    g = coalesce_group(pending, 0, 0.0, set(), 16)
    # same N and medium only; 4 + 6 + 5 = 15, then 1 more fits exactly 16
    assert [r.rid for r in g] == [0, 2, 4, 5]
    assert sum(r.n_sources for r in g) == 16


def test_group_respects_the_source_limit_and_skips_what_does_not_fit():
    pending = [_req(0, 1024, 1, 8), _req(1, 1024, 1, 8), _req(2, 1024, 1, 1),
               _req(3, 1024, 1, 2)]
    g = coalesce_group(pending, 0, 0.0, set(), 16)
    assert [r.rid for r in g] == [0, 1]
    g = coalesce_group(pending, 0, 0.0, set(), 12)
    assert [r.rid for r in g] == [0, 2, 3]


def test_group_ignores_taken_and_not_yet_arrived_requests():
    pending = [_req(0, 512, 0, 2, 0.0), _req(1, 512, 0, 2, 0.5), _req(2, 512, 0, 2, 1.0),
               _req(3, 512, 0, 2, 3.0)]
    assert [r.rid for r in coalesce_group(pending, 0, 2.0, {1}, 16)] == [0, 2]
    # arrivals are sorted: the scan stops at the first request still to come
    assert [r.rid for r in coalesce_group(pending, 0, 0.7, set(), 16)] == [0, 1]
    # a lead later in the list takes only requests after it
    assert [r.rid for r in coalesce_group(pending, 2, 5.0, set(), 16)] == [2, 3]


def test_lone_request_is_its_own_group():
    pending = [_req(0, 2048, 5, 3), _req(1, 2048, 6, 3), _req(2, 4096, 5, 3)]
    assert [r.rid for r in coalesce_group(pending, 0, 0.0, set(), 16)] == [0]


def test_request_trace_is_the_same_closed_and_open_loop():
    closed = make_requests(40, [512, 1024, 2048, 4096], seed=5)
    opened = make_requests(40, [512, 1024, 2048, 4096], seed=5, rate=0.5)
    assert [(r.N, r.medium_seed, r.n_sources, r.source_seed) for r in closed] == \
        [(r.N, r.medium_seed, r.n_sources, r.source_seed) for r in opened]
    assert all(r.arrival == 0.0 for r in closed)
    arr = [r.arrival for r in opened]
    assert arr == sorted(arr) and arr[0] > 0
    assert all(1 <= r.n_sources <= 8 and 0 <= r.medium_seed < 8 for r in closed)
