"""The solve server on the GPU: every request's solution is the same when it is
served alone and when it is served in a mix with others (concurrent slots,
shared cached operators, lock-step batches), within 1e-8 relative (the solves
run to 1e-10), and matches the oracle's direct solve.
"""
import dataclasses

import numpy as np
import pytest

from oracle import hps_oracle as O
from paper_2112_02211_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _fresh(reqs):
    return [P.Request(r.rid, r.arrival, dataclasses.replace(r.prob)) for r in reqs]


def test_same_result_alone_and_in_the_mix():
    from paper_2112_02211_amd.serve import Server, ServeConfig, latency_stats
    reqs = P.request_stream(14, rate=60.0, seed=11, meshes=(2, 3), orders=(6, 8), share=0.5)
    cfg = ServeConfig(slots=4, tol=1e-10, restart=30)
    # all requests queued at once: requests on a shared operator are batched
    # deterministically and the slots run concurrently
    srv = Server(cfg)
    mix = srv.run(_fresh(reqs), closed_loop=True)
    srv.close()
    # and the same stream replayed in real time (batching then depends on timing)
    srv = Server(cfg)
    live = srv.run(_fresh(reqs))
    srv.close()
    st = latency_stats(mix)
    assert st["all_converged"] and st["requests"] == len(reqs)
    assert st["p50_ms"] <= st["p99_ms"]
    assert max(r.batch for r in mix) > 1                      # batching happened
    spans = sorted((r.start, r.finish) for r in mix)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))  # overlap happened
    for r in reqs:
        srv1 = Server(ServeConfig(slots=1, tol=1e-10, restart=30))
        alone = srv1.run(_fresh([r]), closed_loop=True)[0]
        srv1.close()
        for res in (mix, live):
            got = next(x for x in res if x.rid == r.rid)
            err = np.linalg.norm(got.u - alone.u) / np.linalg.norm(alone.u)
            assert err < 1e-8, (r.rid, err, got.batch)
    # spot checks against the oracle's direct solve
    for r in reqs[:3]:
        op = O.build(r.prob)
        ud = O.solve_direct(op)
        got = next(x for x in mix if x.rid == r.rid)
        assert np.linalg.norm(got.u - ud) / np.linalg.norm(ud) < 1e-8


def test_admission_respects_a_small_budget():
    from paper_2112_02211_amd.serve import Server, ServeConfig
    reqs = P.request_stream(6, rate=100.0, seed=12, meshes=(3,), orders=(8,), share=0.0)
    srv = Server(ServeConfig(slots=3, tol=1e-8, restart=20))
    one = srv._size("x", reqs[0].prob, 1, False)
    srv.budget = int(1.5 * one)          # room for one job at a time
    srv.sched.budget = srv.budget
    res = srv.run(_fresh(reqs), closed_loop=True)
    srv.close()
    assert all(r.converged for r in res)
    spans = sorted((r.start, r.finish) for r in res)
    assert all(spans[i + 1][0] >= spans[i][1] - 1e-3 for i in range(len(spans) - 1))


def test_late_request_joins_the_running_job():
    # two requests on one operator, the second arriving 2 ms after the first,
    # while the first job is still building the operator (setup takes far
    # longer): it waits while the operator is busy, then joins the running job
    # at its first tick boundary, and gets the same answer as alone
    from paper_2112_02211_amd.serve import Server, ServeConfig
    base = P.bump_problem("j", (3, 3, 3), 8, 24.0, 6, 2, 41, 8, 1e-10)
    reqs = []
    for i in range(2):
        pr = dataclasses.replace(base, source_points=base.source_points[i:i + 1].copy())
        reqs.append(P.Request(i, 0.0 if i == 0 else 0.002, pr))
    cfg = ServeConfig(slots=2, tol=1e-10, restart=8)
    srv = Server(cfg)
    res = srv.run(_fresh(reqs))
    srv.close()
    a, b = sorted(res, key=lambda r: r.rid)
    assert a.converged and b.converged
    assert a.ticks > 2
    assert b.job == a.job and b.batch == 2 and b.start > a.start
    for r in (a, b):
        srv1 = Server(ServeConfig(slots=1, tol=1e-10, restart=8))
        alone = srv1.run(_fresh([reqs[r.rid]]), closed_loop=True)[0]
        srv1.close()
        assert np.linalg.norm(r.u - alone.u) / np.linalg.norm(alone.u) < 1e-8


def test_per_rhs_residuals_are_reported():
    from paper_2112_02211_amd import hps
    prob = P.bump_problem("r", (2, 2, 2), 8, 14.0, 4, 5, 42, 20, 1e-10)
    ctx = hps.Context.from_problem(prob)
    xyz = ctx.nodes()
    S = np.concatenate([P.rhs_data(prob, xyz, r)[0] for r in range(5)])
    s = torch.from_numpy(S).cuda()
    t = torch.zeros_like(s)
    u, st, ok = ctx.gmres(s, t, tol=1e-10, restart=20, solver="batched")
    assert ok and len(st["rhs_rel_res"]) == 5
    assert max(st["rhs_rel_res"]) <= 1e-10 and max(st["rhs_rel_res"]) == st["true_rel_res"]
    # one cycle at a time from the current iterate reaches the same solution
    u2 = torch.zeros_like(s)
    for _ in range(50):
        _, st2, ok2 = ctx.gmres(s, t, tol=1e-10, restart=20, u=u2, solver="batched", max_iters=20,
                                use_x0=True)
        if ok2:
            break
    assert ok2
    assert (torch.linalg.norm(u2 - u) / torch.linalg.norm(u)).item() < 1e-8


@pytest.mark.parametrize("solver", ["gmres", "fgmres"])
def test_per_rhs_residual_single_solvers(solver):
    from paper_2112_02211_amd import hps
    prob = P.bump_problem("r1", (2, 2, 2), 8, 14.0, 4, 2, 43, 20, 1e-10)
    ctx = hps.Context.from_problem(prob)
    xyz = ctx.nodes()
    S = np.concatenate([P.rhs_data(prob, xyz, r)[0] for r in range(2)])
    s = torch.from_numpy(S).cuda()
    t = torch.zeros_like(s)
    u, st, ok = ctx.gmres(s, t, tol=1e-10, restart=20, solver=solver)
    assert ok and len(st["rhs_rel_res"]) == 2
    assert 0.0 < max(st["rhs_rel_res"]) <= 1e-10
    assert max(st["rhs_rel_res"]) == st["true_rel_res"]


def test_lambda_bucketed_operators_serve_the_same_solutions():
    # operators whose blocks are shared on a lambda grid change the
    # preconditioner, not the system: every served solution matches the
    # unbucketed server's and the oracle's direct solve
    from paper_2112_02211_amd.serve import Server, ServeConfig, latency_stats
    reqs = P.request_stream(8, rate=60.0, seed=13, meshes=(2, 3), orders=(6, 8), share=0.5)
    srv = Server(ServeConfig(slots=3, tol=1e-10, restart=30, lambda_bucket=1e-2))
    res = srv.run(_fresh(reqs), closed_loop=True)
    shared = [(ctx.n_blocks, ctx.nl) for ctx in srv.cache.values()]
    srv.close()
    assert latency_stats(res)["all_converged"]
    srv = Server(ServeConfig(slots=3, tol=1e-10, restart=30))
    ref = srv.run(_fresh(reqs), closed_loop=True)
    srv.close()
    for r in reqs:
        got = next(x for x in res if x.rid == r.rid)
        want = next(x for x in ref if x.rid == r.rid)
        assert np.linalg.norm(got.u - want.u) / np.linalg.norm(want.u) < 1e-8, r.rid
    for r in reqs[:2]:
        ud = O.solve_direct(O.build(r.prob))
        got = next(x for x in res if x.rid == r.rid)
        assert np.linalg.norm(got.u - ud) / np.linalg.norm(ud) < 1e-8
    assert shared and all(b <= n for b, n in shared) and any(b < n for b, n in shared)


def test_operator_groups_serve_the_same_solutions():
    # requests alone on their operator and sharing a mesh are solved in operator
    # groups (one launch for all); each solution equals the one served alone
    from paper_2112_02211_amd.serve import Server, ServeConfig, latency_stats
    reqs = P.request_stream(10, rate=60.0, seed=14, meshes=(2,), orders=(6,), share=0.0)
    srv = Server(ServeConfig(slots=2, tol=1e-10, restart=30, group_ops=4))
    res = srv.run(_fresh(reqs), closed_loop=True)
    srv.close()
    st = latency_stats(res)
    assert st["all_converged"] and st["requests"] == len(reqs)
    assert max(r.batch for r in res) > 1                         # groups were formed
    for r in reqs:
        srv1 = Server(ServeConfig(slots=1, tol=1e-10, restart=30))
        alone = srv1.run(_fresh([r]), closed_loop=True)[0]
        srv1.close()
        got = next(x for x in res if x.rid == r.rid)
        assert np.linalg.norm(got.u - alone.u) / np.linalg.norm(alone.u) < 1e-8, r.rid
    op = O.build(reqs[0].prob)
    got = next(x for x in res if x.rid == reqs[0].rid)
    ud = O.solve_direct(op)
    assert np.linalg.norm(got.u - ud) / np.linalg.norm(ud) < 1e-8


@pytest.mark.parametrize("group_ops", [0, 4])
def test_separable_operators_serve_the_same_solutions(group_ops):
    # operators with the separable J^-1 (no stored blocks): the same
    # preconditioner, so every served solution matches the stored-block server's
    # and the oracle's direct solve; also in operator groups
    from paper_2112_02211_amd.serve import Server, ServeConfig, latency_stats
    reqs = P.request_stream(8, rate=60.0, seed=15, meshes=(2, 3), orders=(6, 8), share=0.5)
    srv = Server(ServeConfig(slots=3, tol=1e-10, restart=30, block_prec="separable",
                             group_ops=group_ops))
    res = srv.run(_fresh(reqs), closed_loop=True)
    srv.close()
    assert latency_stats(res)["all_converged"]
    srv = Server(ServeConfig(slots=3, tol=1e-10, restart=30))
    ref = srv.run(_fresh(reqs), closed_loop=True)
    srv.close()
    for r in reqs:
        got = next(x for x in res if x.rid == r.rid)
        want = next(x for x in ref if x.rid == r.rid)
        assert np.linalg.norm(got.u - want.u) / np.linalg.norm(want.u) < 1e-8, r.rid
    for r in reqs[:2]:
        ud = O.solve_direct(O.build(r.prob))
        got = next(x for x in res if x.rid == r.rid)
        assert np.linalg.norm(got.u - ud) / np.linalg.norm(ud) < 1e-8
