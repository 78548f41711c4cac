"""Full-size requests of the serving stream (the mixed stream of problems.
request_stream, seed 5: meshes 4^3 ... 16^3, p in {8, 10}) served by the solve
server and compared with the oracle's converged solutions of the same four
requests (tests/golden/request_stream_r<rid>_oracle.npz, written by
make_golden.py --request: oracle MGS-GMRES to a preconditioned residual of
1e-13) at the golden's sampled nodes:

    request 24: 12^3 leaves, p = 8,  kappa = 57.9
    request  4: 12^3 leaves, p = 10, kappa = 75.9
    request  6: 16^3 leaves, p = 8,  kappa = 75.7
    request 39: 16^3 leaves, p = 10, kappa = 123.3

All four are queued at once and served on four slots, once with FP64 flexible
GMRES and the separable J^-1 and once with iterative refinement (FP32-stored
inner vectors), each to a true residual of 1e-11 so that the solution error
stays below the 1e-8 bar (the ratio of error to residual reaches about 260 on
request 39, so 1e-10 is not enough there).
"""
import dataclasses
import os

import numpy as np
import pytest

from paper_2112_02211_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))
RIDS = (24, 4, 6, 39)
SHAPES = {24: ((12, 12, 12), 8), 4: ((12, 12, 12), 10), 6: ((16, 16, 16), 8), 39: ((16, 16, 16), 10)}


def _requests():
    stream = P.request_stream(max(RIDS) + 1, rate=1.0, seed=5)
    out = []
    for rid in RIDS:
        r = stream[rid]
        assert (tuple(r.prob.n_elem), r.prob.p) == SHAPES[rid]
        out.append(P.Request(r.rid, 0.0, dataclasses.replace(r.prob)))
    return out


@pytest.mark.parametrize("solver", ["fgmres", "ir"])
def test_full_size_served_requests_match_the_oracle(solver):
    from paper_2112_02211_amd.serve import Server, ServeConfig
    cfg = ServeConfig(slots=4, block_prec="separable", precond_prec="fp64", solver=solver, restart=10,
                      tol=1e-11)
    srv = Server(cfg)
    res = srv.run(_requests(), closed_loop=True)
    srv.close()
    assert len(res) == len(RIDS)
    for r in res:
        g = np.load(os.path.join(HERE, "golden", f"request_stream_r{r.rid}_oracle.npz"))
        assert float(g["pcrr"]) <= 1e-13
        assert r.converged and r.true_rel_res <= 1e-11, (r.rid, r.true_rel_res)
        assert r.u.shape[0] == int(g["N"])
        want = g["u"]
        err = np.linalg.norm(r.u[g["idx"]] - want) / np.linalg.norm(want)
        assert err < 1e-8, (solver, r.rid, err)
