"""Host logic of the solve server: admission by device footprint, FIFO order
with bounded backfill, batching of requests on the same operator."""
import numpy as np

from paper_2112_02211_amd import problems as P
from paper_2112_02211_amd.serve import Scheduler, operator_key


class Req:
    def __init__(self, rid, key, size, prob=None):
        self.rid, self.key, self.size, self.prob = rid, key, size, prob


def size_fn(key, prob, nrhs, resident):
    return (0 if resident else 100) + 10 * nrhs


def test_fifo_and_batching_by_operator():
    s = Scheduler(budget=10_000, size_fn=size_fn, max_batch=3)
    for rid, key in enumerate(["a", "b", "a", "a", "c", "a"]):
        s.submit(Req(rid, key, 1), now=0.0)
    j = s.next_job(set(), set(), 0, 0.0)
    assert j.key == "a" and [r.rid for r in j.requests] == [0, 2, 3] and j.needs_setup
    j = s.next_job(set(), {"a"}, 0, 0.0)
    assert j.key == "b"
    j = s.next_job(set(), {"a"}, 0, 0.0)
    assert j.key == "c"
    j = s.next_job(set(), {"a"}, 0, 0.0)
    assert j.key == "a" and [r.rid for r in j.requests] == [5] and not j.needs_setup
    assert s.next_job(set(), set(), 0, 0.0) is None


def test_busy_operator_waits_and_others_proceed():
    s = Scheduler(budget=10_000, size_fn=size_fn)
    s.submit(Req(0, "a", 1), 0.0)
    s.submit(Req(1, "b", 1), 0.0)
    j = s.next_job({"a"}, set(), 0, 0.0)
    assert j.key == "b"
    assert s.next_job({"a"}, set(), 0, 0.0) is None


def test_admission_by_footprint_with_backfill_and_starvation_guard():
    def sz(key, prob, nrhs, resident):
        return {"big": 900, "small": 50}[key]
    s = Scheduler(budget=1000, size_fn=sz, starve_s=1.0)
    s.submit(Req(0, "big", 1), 0.0)
    s.submit(Req(1, "small", 1), 0.0)
    # 200 bytes in use: the big job does not fit, the small one is backfilled
    j = s.next_job(set(), set(), 200, 0.5)
    assert j.key == "small"
    s.submit(Req(2, "small", 1), 0.6)
    # once the oldest request has waited past the guard, nothing jumps it
    assert s.next_job(set(), set(), 200, 2.0) is None
    # evictable cached bytes count as available
    j = s.next_job(set(), set(), 200, 2.0, evictable_bytes=150)
    assert j.key == "big"


def test_operator_key_identifies_the_discrete_operator():
    reqs = P.request_stream(40, rate=10.0, seed=9, meshes=(2, 3), orders=(6,), share=0.5)
    keys = [operator_key(r.prob) for r in reqs]
    assert len(set(keys)) < len(keys)            # shared scatterers occur
    for r, k in zip(reqs, keys):
        for r2, k2 in zip(reqs, keys):
            same = (r.prob.n_elem == r2.prob.n_elem and r.prob.p == r2.prob.p and
                    r.prob.kappa == r2.prob.kappa and
                    np.array_equal(r.prob.bump_centres, r2.prob.bump_centres) and
                    np.array_equal(r.prob.bump_amps, r2.prob.bump_amps))
            assert same == (k == k2)


def test_request_stream_is_seeded_and_poisson():
    a = P.request_stream(200, rate=50.0, seed=5)
    b = P.request_stream(200, rate=50.0, seed=5)
    assert [r.arrival for r in a] == [r.arrival for r in b]
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert 0.7 / 50 < gaps.mean() < 1.3 / 50
    for r in a:
        e1, p = r.prob.n_elem[0], r.prob.p
        ppw = 2 * np.pi * e1 * p / r.prob.kappa
        assert 8.0 <= ppw <= 12.0 and e1 in (4, 8, 12, 16) and p in (8, 10)
        assert 5 <= len(r.prob.bump_centres) <= 20


def test_take_pulls_the_oldest_requests_of_one_operator():
    s = Scheduler(budget=10_000, size_fn=size_fn)
    for rid, key in enumerate(["a", "b", "a", "c", "a"]):
        s.submit(Req(rid, key, 1), now=0.0)
    got = s.take("a", 2)
    assert [r.rid for r in got] == [0, 2]
    assert [r.rid for r in s.pending] == [1, 3, 4]
    assert s.take("a", 0) == [] and [r.rid for r in s.take("a", 5)] == [4]
    assert s.take("zzz", 3) == []


def test_operator_groups_collect_lone_requests_on_one_mesh():
    # requests alone on their operator and on the same mesh form one group job
    # (oldest first, up to group_ops); operators with several requests, running
    # or cached operators, and other meshes are left alone
    m8 = P.bump_problem("m", (2, 2, 2), 8, 10.0, 3, 1, 1, 30, 1e-8)
    m6 = P.bump_problem("m", (2, 2, 2), 6, 10.0, 3, 1, 1, 30, 1e-8)
    s = Scheduler(budget=10_000, size_fn=size_fn, group_ops=3)
    for rid, (key, prob) in enumerate([("a", m8), ("b", m6), ("c", m8), ("d", m8), ("d", m8),
                                       ("e", m8), ("f", m8), ("g", m8)]):
        s.submit(Req(rid, key, 1, prob), 0.0)
    j = s.next_job({"f"}, {"e"}, 0, 0.0)
    assert j.group and [r.rid for r in j.requests] == [0, 2, 7]     # a, c, g (d has two, e cached, f busy)
    assert j.need_bytes == 3 * size_fn(None, None, 1, False) and j.needs_setup
    j = s.next_job({"f"}, {"e"}, 0, 0.0)
    assert not j.group and j.key == "b"                              # no partner on the p = 6 mesh
    j = s.next_job({"f"}, {"e"}, 0, 0.0)
    assert not j.group and j.key == "d" and len(j.requests) == 2
    j = s.next_job({"f"}, {"e"}, 0, 0.0)
    assert not j.group and j.key == "e" and not j.needs_setup
    assert s.next_job({"f"}, {"e"}, 0, 0.0) is None                  # f still busy
    # off by default
    s = Scheduler(budget=10_000, size_fn=size_fn)
    for rid, key in enumerate("xyz"):
        s.submit(Req(rid, key, 1, m8), 0.0)
    assert not s.next_job(set(), set(), 0, 0.0).group
