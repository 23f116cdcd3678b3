"""apd_dual_objective_grad_noalloc (the evaluation with its scratch in the
library's static device array) against apd_dual_objective_grad, through the
C ABI: identical objective, gradient, counts, centroids and maximum relative
error, on two calls in a row with the second problem smaller than the first,
in 2D and 3D and for every precision tier; and a problem too large for the
static array is refused before any device work."""
import numpy as np
import pytest

import apd_synth as S

pytestmark = pytest.mark.gpu


def _prob(inst):
    import paper_2403_03571_amd as apd
    return apd.Problem.from_instance(inst, "cuda:0")


def _w(inst, seed):
    rng = np.random.default_rng(seed)
    import torch
    return torch.as_tensor(rng.uniform(-0.3, 0.3, inst.n) * inst.n ** (-2.0 / inst.dim), device="cuda:0")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp64"])
@pytest.mark.parametrize("dim", [2, 3])
def test_noalloc_matches_the_allocating_call(prec, dim):
    import paper_2403_03571_amd as apd
    ctx = apd.Context(0)
    if dim == 2:
        first = S.custom(2, 400, (700, 650), seed=61, sigma=0.3)
        second = S.custom(2, 60, (130, 171), seed=62, sigma=0.3)
    else:
        first = S.custom(3, 300, (70, 64, 66), seed=63, sigma=0.3)
        second = S.custom(3, 40, (23, 30, 19), seed=64, sigma=0.3)
    for inst in (first, second):  # the second call on a smaller problem
        prob = _prob(inst)
        w = _w(inst, 7)
        print(f"[noalloc] dim {dim} {prec} n={inst.n} grid={inst.grid}", flush=True)
        ref = ctx.apd_dual_objective_grad(prob, w, prec=prec, counts=True, centroids=True)
        got = ctx.apd_dual_objective_grad(prob, w, prec=prec, counts=True, centroids=True, noalloc=True)
        assert got["g"] == ref["g"]
        assert got["maxrel"] == ref["maxrel"]
        for k in ("grad", "counts", "centroids"):
            assert np.array_equal(got[k].cpu().numpy(), ref[k].cpu().numpy()), k
    ctx.close()


def test_noalloc_refuses_problems_beyond_the_static_array():
    import paper_2403_03571_amd as apd
    ctx = apd.Context(0)
    inst = S.custom(3, 20, (8, 8, 8), seed=65)
    small = _prob(inst)
    big = apd.Problem(3, (512, 512, 512), inst.lo, inst.hi, small.x, small.A, small.v)
    with pytest.raises(apd.ApdError) as e:
        ctx.apd_dual_objective_grad(big, _w(inst, 1), noalloc=True)
    assert e.value.status == 7 and "static array" in e.value.message
    # the context still works afterwards
    out = ctx.apd_dual_objective_grad(small, _w(inst, 1), noalloc=True, counts=True)
    assert int(out["counts"].sum()) == 512
    ctx.close()


def test_noalloc_with_the_norm_cost():
    """A cost other than the squared norm (p = 1, FP64 tier, its per-block
    cost sums also in the static array): identical to the allocating call,
    twice, the second problem smaller."""
    import dataclasses
    import paper_2403_03571_amd as apd
    ctx = apd.Context(0)
    for inst in (S.custom(2, 150, (300, 260), seed=66, sigma=0.3), S.custom(2, 30, (90, 70), seed=67)):
        inst = dataclasses.replace(inst, power=1)
        prob = _prob(inst)
        w = _w(inst, 8)
        ref = ctx.apd_dual_objective_grad(prob, w, prec="fp64", counts=True)
        got = ctx.apd_dual_objective_grad(prob, w, prec="fp64", counts=True, noalloc=True)
        assert got["g"] == ref["g"]
        assert np.array_equal(got["grad"].cpu().numpy(), ref["grad"].cpu().numpy())
        assert np.array_equal(got["counts"].cpu().numpy(), ref["counts"].cpu().numpy())
    ctx.close()
