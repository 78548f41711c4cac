"""hps_apply_noalloc: the operator apply with its face buffer in the library's
static device array (for callers that cannot allocate), through the C-ABI.

Checked against hps_apply (the same kernels with a context workspace) bit for
bit on two calls in a row, the second on a smaller input, in two orders of
contexts; a face buffer beyond the static limit is refused before any launch.
"""
import numpy as np
import pytest

from paper_2112_02211_amd import problems as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _vec(N, k, seed):
    rng = np.random.default_rng(seed)
    return torch.from_numpy((rng.standard_normal(k * N) + 1j * rng.standard_normal(k * N))).cuda()


def test_noalloc_apply_matches_apply_on_two_calls():
    from paper_2112_02211_amd import hps
    big = hps.Context.from_problem(P.workload("bumps_8x8x8_p10"), block_precs=("separable",))
    small = hps.Context.from_problem(P.bump_problem("s", (3, 2, 2), 7, 9.0, 3, 1, 5, 30, 1e-10),
                                     block_precs=("separable",))
    # first call: 3 right-hand sides on 8^3 leaves; second: 1 on 3 x 2 x 2 leaves
    for ctx, k, seed in ((big, 3, 1), (small, 1, 2), (big, 2, 3)):
        x = _vec(ctx.N, k, seed)
        want = ctx.apply(x)
        got = torch.full_like(x, complex(np.nan, np.nan))
        ctx.apply_noalloc(x, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
    big.free()
    small.free()


def test_noalloc_apply_refuses_a_face_buffer_beyond_the_scratch():
    from paper_2112_02211_amd import hps
    ctx = hps.Context.from_problem(P.workload("bumps_8x8x8_p10"), block_precs=("separable",))
    limit = 64 << 20
    per_rhs = ctx.nl * ctx.nb * 16
    k = limit // per_rhs + 1          # the smallest count that does not fit
    x = torch.zeros(k * ctx.N, dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(hps.HPSError, match="static scratch"):
        ctx.apply_noalloc(x, y)
    # the largest count that fits still matches hps_apply
    k -= 1
    x = _vec(ctx.N, k, 4)
    y = torch.empty_like(x)
    ctx.apply_noalloc(x, y)
    assert torch.equal(y, ctx.apply(x))
    ctx.free()
