"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Labels are compared element by element (bit-exact: the re-check tier makes
every label that of an exact double argmin), counts exactly, gradients to
the last bit, the objective to a relative 1e-12 (the two sum in different
orders), centroids to 1e-13.
"""
import numpy as np
import pytest

import apd_synth as S
import oracle as O

pytestmark = pytest.mark.gpu

# "fp32" runs the matrix-core kernel, "fp32-valu" the vector one with the
# per-tile candidate lists (the library's default), "fp32-full" the vector
# one over every seed, "bf16" the bf16 matrix-core tier with the candidate
# lists, "bf16-full" that tier over every seed, "fp32-hyb" the hybrid
# kernel over every seed (matrix cores form the quadratic in u0, the vector
# ALU evaluates it)
PRECS = ["fp64", "fp32", "fp32-valu", "fp32-full", "fp32-hyb", "bf16", "bf16-full"]
SINGLE = ["fp32", "fp32-valu", "fp32-full", "fp32-hyb", "bf16", "bf16-full"]


def _tier(ctx, prec):
    ctx.apd_set_variant(3 if prec == "fp32-hyb" else 1 if prec in ("fp32-valu", "fp32-full") else 0)
    ctx.apd_set_culling(not (prec.endswith("-full") or prec == "fp32-hyb"))
    return prec.split("-")[0]


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2403_03571_amd as apd
    assert torch.cuda.is_available()
    return apd.Context(0)


def _prob(inst):
    import paper_2403_03571_amd as apd
    return apd.Problem.from_instance(inst, "cuda:0")


def _dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0",
                           dtype=dtype or torch.float64)


def _random_w(inst, seed, scale=None):
    # weights of the size of the squared cell radius, so that cells move
    rng = np.random.default_rng(seed)
    scale = scale if scale is not None else 0.3 * inst.n ** (-2.0 / inst.dim)
    return rng.uniform(-scale, scale, inst.n)


CASES = [
    # several tiles in each direction and a ragged tail
    ("2d-ragged", lambda: S.custom(2, 37, (70, 150), seed=1, sigma=0.3)),
    ("2d-box", lambda: S.custom(2, 90, (131, 67), seed=2, sigma=0.2, lo=(-1.0, 0.5), hi=(2.0, 1.25))),
    ("3d-ragged", lambda: S.custom(3, 29, (20, 21, 19), seed=3, sigma=0.3)),
    ("3d-aniso", lambda: S.custom(3, 70, (33, 18, 25), seed=4, amax=4.0)),
    ("c1", S.make_c1),
    # scans of at least 96 seeds (group minima), over more than one staged
    # chunk (512 seeds in the FP32 3D tile, 256 in the bf16 3D tile, 1024
    # in the 2D ones) with a ragged last chunk
    ("2d-long", lambda: S.custom(2, 700, (97, 130), seed=5, sigma=0.3)),
    ("3d-long", lambda: S.custom(3, 530, (23, 20, 26), seed=6, amax=3.0)),
    ("2d-many", lambda: S.custom(2, 1500, (150, 140), seed=7, sigma=0.3)),
    # strongly anisotropic matrices (condition number up to 144), where the
    # single-precision coefficients must not lose the cancellation in e^T A e
    ("2d-aniso12", lambda: S.custom(2, 120, (90, 110), seed=9, amax=12.0)),
    ("3d-aniso8", lambda: S.custom(3, 90, (24, 30, 22), seed=10, amax=8.0)),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_assign_matches_oracle(ctx, name, make, prec):
    inst = make()
    w = _random_w(inst, 11)
    print(f"[assign] {name} {prec} n={inst.n} grid={inst.grid}", flush=True)
    lab = ctx.apd_assign(_prob(inst), _dev(w), prec=_tier(ctx, prec)).cpu().numpy()
    ref, best, second = O.assign(inst, w)
    assert np.array_equal(lab, ref), int(np.sum(lab != ref))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_dual_objective_grad_matches_oracle(ctx, name, make, prec):
    inst = make()
    w = _random_w(inst, 12)
    print(f"[eval] {name} {prec}", flush=True)
    out = ctx.apd_dual_objective_grad(_prob(inst), _dev(w), prec=_tier(ctx, prec), counts=True,
                                      centroids=True)
    ev = O.evaluate(inst, w)
    assert np.array_equal(out["counts"].cpu().numpy(), ev.counts)
    assert np.array_equal(out["grad"].cpu().numpy(), ev.grad)
    assert out["maxrel"] == ev.maxrel
    assert abs(out["g"] - ev.g) <= 1e-12 * max(1e-3, abs(ev.g))
    np.testing.assert_allclose(out["centroids"].cpu().numpy(), ev.centroids, rtol=0, atol=1e-13)


def test_volumes_sum_to_the_domain(ctx):
    inst = S.custom(2, 64, (100, 90), seed=5, sigma=0.4)
    out = ctx.apd_dual_objective_grad(_prob(inst), _dev(_random_w(inst, 3)), counts=True)
    assert int(out["counts"].sum()) == inst.J
    assert abs(float(out["grad"].sum())) < 1e-14


def test_c2_full_size_counts_equal_the_oracle(ctx):
    """1024^2 pixels, N = 1000 (the C2 workload) at weights with realistic
    boundaries: every cell's pixel count, the gradient and the objective
    equal the oracle's (every label: test_gpu_fullsize)."""
    inst = S.make_c2()
    w = _random_w(inst, 21)
    ev = O.evaluate(inst, w)
    for prec in SINGLE:
        print(f"[c2] full size {prec}", flush=True)
        out = ctx.apd_dual_objective_grad(_prob(inst), _dev(w), prec=_tier(ctx, prec), counts=True)
        assert np.array_equal(out["counts"].cpu().numpy(), ev.counts)
        assert np.array_equal(out["grad"].cpu().numpy(), ev.grad)
        assert abs(out["g"] - ev.g) <= 1e-12 * abs(ev.g)
    ctx.apd_set_variant(1)
    ctx.apd_set_culling(True)


def test_c3_full_size_sampled(ctx):
    """256^3 voxels, N = 10^4 (the C3 workload): labels at 3000 sampled voxels
    equal the oracle's; counts sum to J."""
    import torch
    inst = S.make_c3()
    w = _random_w(inst, 22)
    print("[c3] full size", flush=True)
    prob = _prob(inst)
    idx = np.random.default_rng(1).choice(inst.J, 3000, replace=False)
    ref, _, _ = O.assign_pixels(inst, w, idx)
    labs = []
    for prec in SINGLE:
        lab = ctx.apd_assign(prob, _dev(w), prec=_tier(ctx, prec))
        assert np.array_equal(lab.cpu().numpy()[idx], ref), prec
        out = ctx.apd_dual_objective_grad(prob, _dev(w), prec=_tier(ctx, prec), counts=True)
        cnt = out["counts"]
        assert int(cnt.sum()) == inst.J
        # the counts are those of the labels
        bc = torch.bincount(lab.long(), minlength=inst.n)
        assert torch.equal(bc.cpu(), cnt.cpu())
        labs.append(lab)
    # every single-precision kernel gives the same labels everywhere
    assert all(torch.equal(labs[0], lb) for lb in labs[1:])
    ctx.apd_set_variant(1)
    ctx.apd_set_culling(True)


# -------------------------------------------------------- relative gap

def _oracle_gap(inst, w):
    """(labels, relative top-two gap) of the oracle in the gauge w - max w:
    (C_(2) - C_(1)) / (C_(2) + max w), 1 for a single seed."""
    ref, best, second = O.assign(inst, w)
    wmax = float(np.max(w))
    with np.errstate(invalid="ignore", divide="ignore"):
        gap = (second - best) / (second + wmax)
    gap = np.where(np.isinf(second), 1.0, gap)
    return ref, np.maximum(gap, 0.0)


def _round_down32(g):
    f = g.astype(np.float32)
    up = f.astype(np.float64) > g
    f[up] = np.nextafter(f[up], np.float32(-np.inf))
    return f


GAP_CASES = [CASES[0], CASES[1], CASES[2], CASES[5], CASES[6], CASES[8]]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name,make", GAP_CASES, ids=[c[0] for c in GAP_CASES])
def test_rel_gap_is_a_lower_bound_of_the_oracle_gap(ctx, name, make, prec):
    """apd_assign's rel_gap never exceeds the oracle's relative top-two gap;
    it equals it (rounded down to FP32) wherever the pass decided in double:
    every pixel of the FP64 tier, and every near-tie pixel (oracle gap below
    1e-6, which no single-precision certificate settles); elsewhere the bound
    is close to the gap."""
    inst = make()
    w = _random_w(inst, 31)
    print(f"[gap] {name} {prec}", flush=True)
    lab, gap = ctx.apd_assign(_prob(inst), _dev(w), prec=_tier(ctx, prec), rel_gap=True)
    lab, gap = lab.cpu().numpy(), gap.cpu().numpy()
    ref, go = _oracle_gap(inst, w)
    assert np.array_equal(lab, ref)
    assert (gap >= 0).all() and (gap <= 1).all()
    assert (gap.astype(np.float64) <= go).all(), float(np.max(gap - go))
    exact = _round_down32(go)
    if prec == "fp64":
        assert np.array_equal(gap, exact)
    else:
        near = go < 1e-6
        assert np.array_equal(gap[near], exact[near])
        if prec.endswith("-full") or prec == "fp32":
            # over every seed the bound follows the gap closely (with the
            # candidate lists a runner-up outside the list is bounded by the
            # list's U only)
            far = go > 1e-2
            assert np.median(gap[far] / go[far]) > 0.99
    ctx.apd_set_variant(1)
    ctx.apd_set_culling(True)


@pytest.mark.parametrize("prec", PRECS)
def test_rel_gap_at_exact_ties_and_one_seed(ctx, prec):
    """Exact ties give a gap of 0 and the double path's value everywhere near
    them; a single seed has gap 1 everywhere."""
    x = np.array([[0.25, 0.5], [0.75, 0.5], [0.5, 0.25], [0.5, 0.75], [0.25, 0.5]])
    A = np.broadcast_to(np.eye(2), (5, 2, 2)).copy()
    inst = S.Instance(2, (64, 64), (0.0, 0.0), (1.0, 1.0), x, A, np.full(5, 0.2))
    w = np.zeros(5)
    lab, gap = ctx.apd_assign(_prob(inst), _dev(w), prec=_tier(ctx, prec), rel_gap=True)
    ref, go = _oracle_gap(inst, w)
    gap = gap.cpu().numpy()
    assert np.array_equal(lab.cpu().numpy(), ref)
    assert (gap[go == 0] == 0).all() and (go == 0).sum() > 100
    assert (gap.astype(np.float64) <= go).all()
    one = S.custom(2, 1, (9, 7), seed=0)
    _, g1 = ctx.apd_assign(_prob(one), _dev(np.zeros(1)), prec=_tier(ctx, prec), rel_gap=True)
    assert bool((g1 == 1).all())
    ctx.apd_set_variant(1)
    ctx.apd_set_culling(True)


# ------------------------------------- boundary-aware refinement (adaptive)

ADAPT_CASES = [
    # cells of 60-70 pixels across: most tiles lie inside one cell
    ("2d-fine", lambda: S.custom(2, 60, (512, 480), seed=41, sigma=0.3)),
    ("2d-fine-box", lambda: S.custom(2, 40, (390, 517), seed=42, sigma=0.2, lo=(-1.0, 0.5),
                                     hi=(2.0, 1.25))),
    ("3d-fine", lambda: S.custom(3, 30, (80, 72, 90), seed=43, sigma=0.3)),
]


@pytest.mark.parametrize("prec", ["fp32-valu", "bf16"])
@pytest.mark.parametrize("name,make", ADAPT_CASES, ids=[c[0] for c in ADAPT_CASES])
def test_adaptive_refinement_is_exact(ctx, name, make, prec):
    """Tiles whose candidate list holds one seed are credited whole (closed-
    form moments): counts, gradient, objective, centroids and labels equal
    the oracle's and those of the pixel-by-pixel pass, and tiles were in
    fact credited."""
    inst = make()
    w = _random_w(inst, 51)
    ev = O.evaluate(inst, w)
    ref, _, _ = O.assign(inst, w)
    print(f"[adaptive] {name} {prec}", flush=True)
    credited = {}
    for on in (True, False):
        ctx.apd_set_adaptive(on)
        out = ctx.apd_dual_objective_grad(_prob(inst), _dev(w), prec=_tier(ctx, prec), counts=True,
                                          centroids=True)
        credited[on] = ctx.apd_last_pass_stats()["tiles_credited"]
        assert np.array_equal(out["counts"].cpu().numpy(), ev.counts), on
        assert np.array_equal(out["grad"].cpu().numpy(), ev.grad), on
        assert abs(out["g"] - ev.g) <= 1e-12 * max(1e-3, abs(ev.g)), on
        np.testing.assert_allclose(out["centroids"].cpu().numpy(), ev.centroids, rtol=0, atol=1e-13)
        lab = ctx.apd_assign(_prob(inst), _dev(w), prec=_tier(ctx, prec)).cpu().numpy()
        assert np.array_equal(lab, ref), on
    assert credited[True] > 0 and credited[False] == 0, credited
    ctx.apd_set_adaptive(True)
    ctx.apd_set_variant(1)
    ctx.apd_set_culling(True)


# ------------------------------------- costs beyond |.|^2_A (power p)

POWER_CASES = [
    ("2d-ragged", lambda: S.custom(2, 37, (70, 150), seed=1, sigma=0.3)),
    ("2d-box", lambda: S.custom(2, 90, (131, 67), seed=2, sigma=0.2, lo=(-1.0, 0.5), hi=(2.0, 1.25))),
    ("3d-ragged", lambda: S.custom(3, 29, (20, 21, 19), seed=3, sigma=0.3)),
]


@pytest.mark.parametrize("p", [1, 3, 4])
@pytest.mark.parametrize("name,make", POWER_CASES, ids=[c[0] for c in POWER_CASES])
def test_power_cost_matches_oracle(ctx, name, make, p):
    """C_ij = |y_j - x_i|_{A_i}^p - w_i in the FP64 tier: labels and the
    relative gap bit for bit, counts and gradient exactly, the objective
    (summed pixel by pixel) to 1e-12, centroids to 1e-13."""
    import dataclasses
    inst = dataclasses.replace(make(), power=p)
    w = _random_w(inst, 41) * (inst.n ** (1.0 / inst.dim)) ** (2 - p)
    print(f"[power {p}] {name}", flush=True)
    lab, gap = ctx.apd_assign(_prob(inst), _dev(w), prec="fp64", rel_gap=True)
    ref, go = _oracle_gap(inst, w)
    assert np.array_equal(lab.cpu().numpy(), ref)
    assert np.array_equal(gap.cpu().numpy(), _round_down32(go))
    out = ctx.apd_dual_objective_grad(_prob(inst), _dev(w), prec="fp64", counts=True, centroids=True)
    ev = O.evaluate(inst, w)
    assert np.array_equal(out["counts"].cpu().numpy(), ev.counts)
    assert np.array_equal(out["grad"].cpu().numpy(), ev.grad)
    assert out["maxrel"] == ev.maxrel
    assert abs(out["g"] - ev.g) <= 1e-12 * max(1e-3, abs(ev.g))
    np.testing.assert_allclose(out["centroids"].cpu().numpy(), ev.centroids, rtol=0, atol=1e-13)


def test_power_cost_fit_is_certified_and_other_tiers_refused(ctx):
    """Algorithm 2 with the norm cost (p = 1) in the FP64 tier: certified by
    the oracle's recount, evaluation count within a band of the oracle
    solver's; the single-precision tiers refuse such costs."""
    import dataclasses
    import paper_2403_03571_amd as apd
    inst = dataclasses.replace(S.custom(2, 20, 128, seed=9, sigma=0.3), power=1)
    w, rep = ctx.apd_fit_weights(_prob(inst), eps=0.01, prec="fp64")
    assert rep.converged, rep
    ev = O.evaluate(inst, w.cpu().numpy())
    assert ev.maxrel < 0.01 and abs(ev.maxrel - rep.max_rel_err) < 1e-12
    _, orep = O.fit_weights(inst, eps=0.01)
    assert orep.converged and abs(rep.evals - orep.evals) <= max(10, 0.5 * orep.evals)
    for prec in ("fp32", "bf16"):
        with pytest.raises(apd.ApdError) as e:
            ctx.apd_dual_objective_grad(_prob(inst), _dev(np.zeros(inst.n)), prec=prec)
        assert e.value.status == 1


# -------------------------------------------------------------- edge cases

def test_single_seed_takes_every_pixel(ctx):
    inst = S.custom(2, 1, (5, 3), seed=0)
    for prec in PRECS:
        lab = ctx.apd_assign(_prob(inst), _dev(np.zeros(1)), prec=_tier(ctx, prec)).cpu().numpy()
        assert (lab == 0).all()


def test_one_pixel_and_thin_grids(ctx):
    for grid in [(1, 1), (1, 200), (200, 1), (1, 1, 1), (1, 9, 70), (70, 1, 3)]:
        inst = S.custom(len(grid), 13, grid, seed=6)
        w = _random_w(inst, 7)
        ref, _, _ = O.assign(inst, w)
        for prec in PRECS:
            lab = ctx.apd_assign(_prob(inst), _dev(w), prec=_tier(ctx, prec)).cpu().numpy()
            assert np.array_equal(lab, ref), (grid, prec)


def test_exact_ties_go_to_the_lowest_index(ctx):
    """Seeds placed symmetrically so that many pixel centres are exactly
    equidistant; duplicated seeds tie everywhere."""
    x = np.array([[0.25, 0.5], [0.75, 0.5], [0.5, 0.25], [0.5, 0.75], [0.25, 0.5]])
    A = np.broadcast_to(np.eye(2), (5, 2, 2)).copy()
    inst = S.Instance(2, (64, 64), (0.0, 0.0), (1.0, 1.0), x, A, np.full(5, 0.2))
    ref, best, second = O.assign(inst, np.zeros(5))
    assert np.sum(best == second) > 100
    for prec in PRECS:
        lab = ctx.apd_assign(_prob(inst), _dev(np.zeros(5)), prec=_tier(ctx, prec)).cpu().numpy()
        assert np.array_equal(lab, ref), prec
        assert not (lab == 4).any()


def test_large_weight_offsets(ctx):
    """A common offset of w changes nothing; a wide spread of w makes many
    cells empty and others large."""
    inst = S.custom(2, 50, (90, 110), seed=8)
    for w in (_random_w(inst, 1) + 123.0, _random_w(inst, 2, scale=0.5)):
        ref, _, _ = O.assign(inst, w)
        for prec in PRECS:
            lab = ctx.apd_assign(_prob(inst), _dev(w), prec=_tier(ctx, prec)).cpu().numpy()
            assert np.array_equal(lab, ref)


def test_deterministic(ctx):
    inst = S.custom(3, 200, (30, 30, 30), seed=9)
    w = _dev(_random_w(inst, 4))
    a = ctx.apd_dual_objective_grad(_prob(inst), w, counts=True)
    b = ctx.apd_dual_objective_grad(_prob(inst), w, counts=True)
    assert a["g"] == b["g"]
    assert bool((a["counts"] == b["counts"]).all())


def test_invalid_inputs_raise(ctx):
    import paper_2403_03571_amd as apd
    inst = S.custom(2, 10, (20, 20), seed=3)
    prob = _prob(inst)
    w = _dev(np.zeros(10))
    bad = inst.A.copy()
    bad[3] = [[1.0, 2.0], [2.0, 1.0]]
    with pytest.raises(apd.ApdError) as e:
        ctx.apd_assign(apd.Problem(2, inst.grid, inst.lo, inst.hi, prob.x, _dev(bad), prob.v), w)
    assert e.value.status == 2
    wn = np.zeros(10)
    wn[2] = np.nan
    with pytest.raises(apd.ApdError) as e:
        ctx.apd_dual_objective_grad(prob, _dev(wn))
    assert e.value.status == 8
    with pytest.raises(apd.ApdError) as e:
        ctx.apd_dual_objective_grad(apd.Problem(2, inst.grid, inst.lo, inst.hi, prob.x, prob.A,
                                                prob.v * 1.01), w)
    assert e.value.status == 3
    with pytest.raises(apd.ApdError) as e:
        ctx.apd_assign(apd.Problem(2, (0, 5), inst.lo, inst.hi, prob.x, prob.A, prob.v), w)
    assert e.value.status == 1


# ------------------------------------------------------------- the solver

@pytest.mark.parametrize("prec", PRECS)
def test_fit_c1_certified_by_the_oracle(ctx, prec):
    inst = S.make_c1()
    w, rep = ctx.apd_fit_weights(_prob(inst), eps=0.01, prec=_tier(ctx, prec))
    assert rep.converged, rep
    ev = O.evaluate(inst, w.cpu().numpy())
    assert ev.maxrel < 0.01
    assert ev.maxrel == rep.max_rel_err
    wo, ro = O.fit_weights(inst, eps=0.01)
    print(f"[fit c1] gpu iters={rep.iters} evals={rep.evals}  oracle iters={ro.iters} evals={ro.evals}")
    assert abs(rep.evals - ro.evals) <= max(3, 0.2 * ro.evals)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp64"])
def test_graph_replayed_fit_equals_the_eager_fit(ctx, prec):
    """A fit replays its captured evaluation graph every pass; the same fit
    with eager passes (profiling on) takes the identical path: the same
    weights to the last bit and the same number of passes -- every replay
    gave the eager result."""
    inst = S.custom(2, 120, (200, 160), seed=71, sigma=0.3)
    w_g, r_g = ctx.apd_fit_weights(_prob(inst), prec=prec)
    ctx.apd_set_profiling(True)
    w_e, r_e = ctx.apd_fit_weights(_prob(inst), prec=prec)
    ctx.apd_set_profiling(False)
    assert r_g.converged and r_e.converged
    assert r_g.evals == r_e.evals and r_g.iters == r_e.iters
    np.testing.assert_array_equal(w_g.cpu().numpy(), w_e.cpu().numpy())
    # a second graph-replayed fit on the same context agrees too
    w_2, r_2 = ctx.apd_fit_weights(_prob(inst), prec=prec)
    np.testing.assert_array_equal(w_2.cpu().numpy(), w_g.cpu().numpy())


def test_fit_multiphase_2d_and_3d(ctx):
    for inst in (S.custom(2, 120, (256, 256), seed=3, sigma=0.35, amax=4.0),
                 S.custom(3, 60, (48, 48, 48), seed=4, sigma=0.3)):
        w, rep = ctx.apd_fit_weights(_prob(inst), eps=0.01, prec="fp32")
        assert rep.converged, rep
        ev = O.evaluate(inst, w.cpu().numpy())
        assert ev.maxrel < 0.01 and ev.maxrel == rep.max_rel_err


def test_coarse_to_fine_start_certified(ctx):
    """A fit started on the grid halved along every axis (odd sizes rounded
    up) to a looser tolerance, then run on the problem's grid: it converges
    there, the oracle's count at the returned weights meets the 1 % rule of
    Algorithm 2 on the problem's grid and equals the library's, and the
    coarse passes are reported inside the total.  Without the option the
    report carries no coarse passes."""
    for inst in (S.custom(2, 120, (257, 255), seed=3, sigma=0.35, amax=4.0),
                 S.custom(3, 60, (49, 48, 47), seed=4, sigma=0.3)):
        w, rep = ctx.apd_fit_weights(_prob(inst), eps=0.01, prec="fp32", coarse_eps=0.03)
        assert rep.converged, rep
        assert 0 < rep.coarse_evals < rep.evals, rep
        assert tuple(rep.grid[:inst.dim]) == inst.grid
        ev = O.evaluate(inst, w.cpu().numpy())
        assert ev.maxrel < 0.01 and ev.maxrel == rep.max_rel_err
        _, rep0 = ctx.apd_fit_weights(_prob(inst), eps=0.01, prec="fp32")
        assert rep0.coarse_evals == 0 and rep0.converged


def test_fit_lattice_needs_no_iteration(ctx):
    x = np.array([[0.25, 0.25], [0.75, 0.25], [0.25, 0.75], [0.75, 0.75]])
    inst = S.Instance(2, (64, 64), (0.0, 0.0), (1.0, 1.0), x,
                      np.broadcast_to(np.eye(2), (4, 2, 2)).copy(), np.full(4, 0.25))
    w, rep = ctx.apd_fit_weights(_prob(inst))
    assert rep.converged and rep.iters == 0 and rep.evals == 1


def test_not_converged_reports_the_resolution_rule(ctx):
    inst = S.custom(2, 80, (16, 16), seed=1, sigma=0.5)   # far below (2.9)
    w, rep = ctx.apd_fit_weights(_prob(inst), max_evals=30)
    assert not rep.converged and rep.status == "APD_ERR_NOT_CONVERGED"


def test_lloyd_step_matches_oracle(ctx):
    import torch
    inst = S.custom(2, 30, (120, 120), seed=13, sigma=0.2)
    prob = _prob(inst)
    x = prob.x.clone()
    w = torch.zeros(inst.n, dtype=torch.float64, device="cuda:0")
    x1, w1, rep = ctx.apd_lloyd_step(prob, x, w)
    assert rep.converged
    # the new seeds are the centroids of the cells at the fitted weights
    ev = O.evaluate(inst, w1.cpu().numpy())
    np.testing.assert_allclose(x1.cpu().numpy(), ev.centroids, rtol=0, atol=1e-13)


def test_algorithm3_on_a_polycrystal_like_instance(ctx):
    """Algorithm 3 from uniform seeds on a small polycrystal-like instance
    (areas spanning a factor ~196, elongated small grains), grid from (2.10)
    at 2 %: every Lloyd step moves the seeds to the oracle's centroids of
    the cells at the fitted weights, and the final fit is certified by the
    oracle."""
    import torch
    import paper_2403_03571_amd as apd
    probe = S.make_microstructure(61, M=64, n=150)
    M = apd.apd_choose_resolution(2, 0.02, float(probe.v.min()), 1.0)
    assert M == O.choose_resolution(2, 0.02, float(probe.v.min()), 1.0)
    inst = S.make_microstructure(61, M=M, n=150)
    prob = _prob(inst)
    w, rep = ctx.apd_fit_weights(prob, eps=0.02)
    assert rep.converged
    x = prob.x.clone()
    for _ in range(2):
        xin = x.cpu().numpy().copy()
        x, w, rep = ctx.apd_lloyd_step(prob, x, w, eps=0.02)
        assert rep.converged
        ev = O.evaluate(inst, w.cpu().numpy(), x=xin)
        np.testing.assert_allclose(x.cpu().numpy(), ev.centroids, rtol=0, atol=1e-13)
    final = apd.Problem(prob.dim, prob.grid, prob.lo, prob.hi, x, prob.A, prob.v)
    w, rep = ctx.apd_fit_weights(final, w=w, eps=0.02)
    assert rep.converged
    assert O.evaluate(inst, w.cpu().numpy(), x=x.cpu().numpy()).maxrel < 0.02


def test_bf16_tier_rechecks_more_but_agrees(ctx):
    """The bf16 tier's looser rounding bound sends more pixels to the double
    re-check than the fp32 tier, and the labels still agree everywhere."""
    import torch
    inst = S.make_c2()
    w = _dev(_random_w(inst, 31))
    prob = _prob(inst)
    a = ctx.apd_assign(prob, w, prec="fp32")
    n32 = ctx.apd_last_pass_stats()["rechecked"]
    b = ctx.apd_assign(prob, w, prec="bf16")
    n16 = ctx.apd_last_pass_stats()["rechecked"]
    print(f"[bf16] rechecked fp32 {n32} bf16 {n16} of {inst.J}")
    assert torch.equal(a, b)
    assert n16 >= n32
    assert n16 < 0.2 * inst.J


def test_culling_with_extreme_weights_and_anisotropy(ctx):
    """Candidate lists under stress: very anisotropic matrices (aspect 12),
    weights spread over several cell radii (cells far from their seeds,
    empty cells), and seeds outside the box."""
    for dim, grid in ((2, (150, 170)), (3, (30, 26, 34))):
        inst = S.custom(dim, 80, grid, seed=40 + dim, amax=12.0, lo=[0.0] * dim, hi=[1.0] * dim)
        inst.x = inst.x * 1.4 - 0.2
        for scale in (0.3, 3.0):
            w = _random_w(inst, 5, scale=scale * inst.n ** (-2.0 / dim))
            ref, _, _ = O.assign(inst, w)
            for prec in ("fp32-valu", "fp32-full", "fp32-hyb", "bf16", "bf16-full"):
                lab = ctx.apd_assign(_prob(inst), _dev(w), prec=_tier(ctx, prec)).cpu().numpy()
                assert np.array_equal(lab, ref), (dim, scale, prec)
    ctx.apd_set_culling(True)


@pytest.mark.parametrize("dim", [2, 3])
def test_exact_box_bounds_with_needle_cells(ctx, dim):
    """The candidate lists take exact bounds of each quadratic form over a
    box (2D: its range at every level; 3D: its maximum in the per-wave
    lists): matrices of condition
    number up to 1600 in 2D and about 70 in 3D (needle-shaped cells crossing many
    tiles), seeds on and outside the box's faces, weights spread over
    several cell radii; labels equal the oracle's with and without the
    lists, on both single-precision tiers."""
    if dim == 2:
        inst = S.custom(2, 90, (203, 161), seed=61, amax=40.0, lo=[0.0, 0.0], hi=[1.0, 1.0])
    else:
        inst = S.custom(3, 70, (41, 36, 45), seed=64, amax=20.0, lo=[0.0] * 3, hi=[1.0] * 3)
    inst.x = inst.x * 1.3 - 0.15
    inst.x[:10, 0] = 0.0          # seeds on the box's faces
    inst.x[10:20, 1] = 1.0
    for scale in (0.3, 2.0):
        w = _random_w(inst, 63, scale=scale * inst.n ** (-2.0 / dim))
        ref, _, _ = O.assign(inst, w)
        for prec in ("fp32-valu", "fp32-full", "fp32-hyb", "bf16", "bf16-full"):
            lab = ctx.apd_assign(_prob(inst), _dev(w), prec=_tier(ctx, prec)).cpu().numpy()
            assert np.array_equal(lab, ref), (scale, prec)
    ctx.apd_set_culling(True)


@pytest.mark.parametrize("n,grid", [(3000, (70, 90)), (600, (70, 90)), (3000, (600, 500)),
                                    (600, (400, 300))])
def test_culling_overflow_falls_back_to_every_seed(ctx, n, grid):
    """A tight cluster of seeds far outside the box: every seed is a
    candidate of every tile and super-tile -- 600 fit a list (a long list
    scan), 3000 do not (the kernel and the re-check scan all seeds); the
    larger grids go through super-tiles.  Near-ties are everywhere."""
    rng = np.random.default_rng(77)
    x = np.array([6.0, -4.0]) + 1e-3 * rng.standard_normal((n, 2))
    A = np.broadcast_to(np.eye(2), (n, 2, 2)).copy()
    inst = S.Instance(2, grid, (0.0, 0.0), (1.0, 1.0), x, A, np.full(n, 1.0 / n))
    # weights that cancel the distance to the box centre, so that many cells
    # cross the box
    c = np.array([0.5, 0.5])
    w = (x * x).sum(1) - 2.0 * x @ c + 2e-4 * rng.standard_normal(n)
    ref, _, _ = O.assign(inst, w)
    assert np.unique(ref).size > 10
    for prec in ("fp32-valu", "fp32-full", "bf16", "bf16-full"):
        lab = ctx.apd_assign(_prob(inst), _dev(w), prec=_tier(ctx, prec)).cpu().numpy()
        assert np.array_equal(lab, ref), prec
    ctx.apd_set_culling(True)


def test_autotune_picks_an_exact_kernel(ctx, tmp_path):
    """The autotuner times the exact kernels of the fp32 tier and keeps the
    fastest; the cache reproduces the choice; results are unchanged."""
    from paper_2403_03571_amd import tune
    inst = S.custom(2, 200, (256, 256), seed=21, sigma=0.3)
    prob = _prob(inst)
    w = _dev(_random_w(inst, 9))
    ref, _, _ = O.assign(inst, w.cpu().numpy())
    choice = tune.tuned(ctx, prob, "fp32", cache=str(tmp_path / "t.json"), reps=2)
    assert not choice["cached"] and len(choice["pass_ms"]) == 6
    assert choice["pixels_per_lane"] in (0, 4, 8)
    assert min(choice["pass_ms"]) > 0.0
    assert choice["variant"] in (0, 1, 3)
    lab = ctx.apd_assign(prob, w, prec="fp32").cpu().numpy()
    assert np.array_equal(lab, ref)
    again = tune.tuned(ctx, prob, "fp32", cache=str(tmp_path / "t.json"))
    assert again["cached"] and again["variant"] == choice["variant"]
    # in 3D every candidate, the hybrid kernel included, is timed
    inst3 = S.custom(3, 300, (48, 40, 44), seed=22, sigma=0.3)
    prob3 = _prob(inst3)
    w3 = _dev(_random_w(inst3, 9))
    ref3, _, _ = O.assign(inst3, w3.cpu().numpy())
    c3 = ctx.apd_autotune(prob3, w3, reps=2)
    print(f"[autotune 3d] {c3}", flush=True)
    assert min(c3["pass_ms"]) > 0.0
    assert np.array_equal(ctx.apd_assign(prob3, w3, prec="fp32").cpu().numpy(), ref3)
    ctx.apd_set_variant(2)
    ctx.apd_set_culling(True)
    ctx.apd_set_pixels_per_lane(0)


def test_default_kernel_by_seed_count(ctx):
    """Over every seed the default (variant 2) runs the hybrid kernel from
    1536 seeds on grids of at least 128 hybrid tiles (16 x 16 x 8 in 3D,
    32 x 32 in 2D) and the vector kernel otherwise, in 2D and 3D; the labels
    equal the oracle's either way."""
    import bench
    ctx.apd_set_variant(2)
    ctx.apd_set_culling(False)
    cases = ((S.custom(3, 300, (40, 36, 44), seed=71, sigma=0.3), "fp32-vector"),
             (S.custom(3, 9000, (48, 40, 44), seed=72, sigma=0.3), "fp32-vector"),    # 54 tiles
             (S.custom(3, 1536, (130, 129, 65), seed=75, sigma=0.3), "fp32-hybrid"),  # 729 tiles
             (S.custom(3, 1535, (130, 129, 65), seed=76, sigma=0.3), "fp32-vector"),
             (S.custom(3, 2000, (64, 66, 62), seed=78, sigma=0.3), "fp32-hybrid"),    # 160 tiles
             (S.custom(2, 500, (150, 170), seed=73, sigma=0.3), "fp32-vector"),
             (S.custom(2, 8192, (300, 280), seed=74, sigma=0.3), "fp32-vector"),      # 90 tiles
             (S.custom(2, 3100, (1030, 520), seed=77, sigma=0.3), "fp32-hybrid"))     # 561 tiles
    for inst, kernel in cases:
        assert bench.hyb_by_default(inst) == (kernel == "fp32-hybrid"), inst.grid
        w = _random_w(inst, 5)
        lab = ctx.apd_assign(_prob(inst), _dev(w), prec="fp32").cpu().numpy()
        assert ctx.apd_last_pass_stats()["kernel"] == kernel, (inst.n, inst.dim)
        ref, _, _ = O.assign(inst, w)
        assert np.array_equal(lab, ref), (inst.n, inst.dim, int(np.sum(lab != ref)))
    ctx.apd_set_culling(True)


@pytest.mark.parametrize("pp", [4, 8])
def test_tile_shapes_give_the_same_labels(ctx, pp):
    """Both tile shapes of the vector kernel (4 or 8 pixels per lane) and of
    the bf16 kernel (2 or 4 rows per lane), with and without candidate
    lists, on 2D and 3D cases with ragged edges."""
    ctx.apd_set_variant(1)
    for inst in (S.custom(2, 300, (130, 200), seed=61, sigma=0.3),
                 S.custom(3, 200, (45, 20, 27), seed=62, sigma=0.2)):
        w = _random_w(inst, 3)
        ref, _, _ = O.assign(inst, w)
        evr = O.evaluate(inst, w)
        ctx.apd_set_pixels_per_lane(pp)
        for prec in ("fp32", "bf16"):
            for cull in (True, False):
                ctx.apd_set_culling(cull)
                lab = ctx.apd_assign(_prob(inst), _dev(w), prec=prec).cpu().numpy()
                assert np.array_equal(lab, ref), (inst.dim, pp, prec, cull)
                out = ctx.apd_dual_objective_grad(_prob(inst), _dev(w), prec=prec, counts=True)
                np.testing.assert_array_equal(out["counts"].cpu().numpy(), evr.counts)
    ctx.apd_set_pixels_per_lane(0)
    ctx.apd_set_culling(True)
    import paper_2403_03571_amd as apd
    with pytest.raises(apd.ApdError, match="INVALID_ARG"):
        ctx.apd_set_pixels_per_lane(6)


# ------------------------------------------- pixel weights and refinement

MASKED = [
    ("2d-disk", lambda: S.custom(2, 60, (150, 131), seed=51, sigma=0.3), (0.5, 0.45), 0.41),
    ("3d-ball", lambda: S.custom(3, 40, (30, 26, 33), seed=52, sigma=0.2), (0.5, 0.5, 0.5), 0.45),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name,make,centre,radius", MASKED, ids=[m[0] for m in MASKED])
def test_pixel_weights_match_oracle(ctx, name, make, centre, radius, prec):
    """A disk / ball domain with fractional boundary pixels: weighted counts
    exactly, gradient to the last bits, objective to 1e-12, centroids to
    1e-13; the labels do not depend on the weights."""
    inst = make()
    q = S.disk_weights(inst.grid, inst.lo, inst.hi, centre, radius)
    mi = S.masked(inst, q)
    w = _random_w(mi, 21)
    ref = O.evaluate(mi, w)
    out = ctx.apd_dual_objective_grad(_prob(mi), _dev(w), prec=_tier(ctx, prec), counts=True,
                                      centroids=True)
    np.testing.assert_array_equal(out["counts"].cpu().numpy(), ref.counts)
    np.testing.assert_allclose(out["grad"].cpu().numpy(), ref.grad, rtol=0, atol=1e-15)
    assert out["g"] == pytest.approx(ref.g, rel=1e-12, abs=1e-15)
    np.testing.assert_allclose(out["centroids"].cpu().numpy(), ref.centroids, rtol=0, atol=1e-13)
    lab = ctx.apd_assign(_prob(mi), _dev(w), prec=_tier(ctx, prec)).cpu().numpy()
    np.testing.assert_array_equal(lab, O.assign(inst, w)[0])
    ctx.apd_set_variant(1)
    ctx.apd_set_culling(True)


def test_fit_on_a_disk_domain_certified_by_the_oracle(ctx):
    import paper_2403_03571_amd as apd
    inst = S.custom(2, 80, (300, 300), seed=53, sigma=0.25)
    inst.x = 0.5 + 0.35 * (inst.x - 0.5)          # seeds inside the disk
    mi = S.masked(inst, S.disk_weights(inst.grid, inst.lo, inst.hi, (0.5, 0.5), 0.45))
    w, rep = ctx.apd_fit_weights(_prob(mi), eps=0.01)
    assert rep.converged
    assert O.evaluate(mi, w.cpu().numpy()).maxrel < 0.01
    # the volumes must sum to the weighted domain measure
    bad = S.Instance(2, mi.grid, mi.lo, mi.hi, mi.x, mi.A, inst.v, mass=mi.mass)
    with pytest.raises(apd.ApdError, match="VOLUMES"):
        ctx.apd_dual_objective_grad(_prob(bad), _dev(np.zeros(inst.n)))
    with pytest.raises(apd.ApdError, match="INVALID_ARG"):
        ctx.apd_fit_weights_batched([_prob(mi)])


def test_refinement_matches_the_oracle(ctx):
    """On a grid too coarse for 1 % the fit refines the grid as the oracle
    does (the same grid) and converges; the result is certified by the
    oracle on that grid."""
    inst = S.custom(2, 40, (20, 20), seed=34, sigma=0.3)
    w, rep = ctx.apd_fit_weights(_prob(inst), eps=0.01, max_evals=300)
    assert not rep.converged and rep.refinements == 0
    w, rep = ctx.apd_fit_weights(_prob(inst), eps=0.01, max_evals=300, refine=4)
    _, rep_o, grid_o = O.fit_weights_refine(inst, eps=0.01, max_refine=4, max_evals=300)
    assert rep.converged and rep.refinements >= 1
    assert tuple(rep.grid[:2]) == grid_o
    fine = S.Instance(2, grid_o, inst.lo, inst.hi, inst.x, inst.A, inst.v)
    assert O.evaluate(fine, w.cpu().numpy()).maxrel < 0.01
