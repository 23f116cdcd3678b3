"""Rounding bounds behind the single-precision certificates, checked by
replaying the kernels' arithmetic on the CPU in exact rational arithmetic.

The FP32 vector tier evaluates the cost of seed i at pixel k in tile-local
coordinates u = y - anchor as fl(fl(a00 u0 + beta) u0 + alpha), with beta and
alpha formed by fused multiply-adds from FP32 coefficients that are computed
in double about the anchor (eq. (2.1) expanded; Algorithm 1 at pixel
centres, eq. (2.6)).  The bf16 tier forms the same cost as a dot product of
hi/lo-split bf16 coefficients and integer features, accumulated in FP32.
Both tiers settle a pixel only when its top-two gap exceeds the sum of the
two costs' rounding bounds plus slack, which is sound when, for every seed of
true cost C <= B at a pixel at offset u from the tile anchor (r^2 =
lambda_G |u|^2, lambda_G the Gershgorin bound),
  FP32: |C_hat - C| <= 2^-20 (B + 4 r sqrt(B) + 4 r^2)      (e32)
  bf16: |C_hat - C| <= 2^-15 (3 r^2 + 2 r sqrt(B)) + 2^-18 B  (e16).

Here every FP32 operation of the kernels (fused multiply-adds included) is
rounded once from its exact rational value, and the costs are compared with
the exact rational cost, on adversarial seeds: condition numbers up to 10^3
(and 10^6), seeds outside the box, weights spread over several cell radii,
boxes away from the origin.  The test also checks the intermediate claims of
the derivation (the rounding count, the sum of the monomials against its
bound) and
the slack added for the double-precision evaluation of the definition.  The
bf16 matrix-core sum is replayed in two orders (one rounding, and a rounding
after every product in slot order); the hardware's order lies within the
derivation's bound for any order.
"""
from __future__ import annotations

from fractions import Fraction as F

import numpy as np
import pytest


def e32(B: float, r2: float) -> float:
    r = np.sqrt(r2)
    return 2.0 ** -20 * (B + 4.0 * r * np.sqrt(B) + 4.0 * r2)


def e16(B: float, r2: float) -> float:
    r = np.sqrt(r2)
    return 2.0 ** -15 * (3.0 * r2 + 2.0 * r * np.sqrt(B)) + 2.0 ** -18 * B


# ------------------------------------------------------------ exact rounding

def rnd32(x: F) -> float:
    """x rounded to the nearest float32 (ties to even), as a Python float."""
    if x == 0:
        return 0.0
    neg = x < 0
    m = -x if neg else x
    e = m.numerator.bit_length() - m.denominator.bit_length()
    if m < F(2) ** e:
        e -= 1
    assert e >= -126, "subnormal result"
    ulp = F(2) ** (e - 23)
    q = m / ulp
    n = q.numerator // q.denominator
    rem = q - n
    if rem > F(1, 2) or (rem == F(1, 2) and n % 2 == 1):
        n += 1
    v = n * ulp
    assert v < F(2) ** 128, "overflow"
    out = float(v)
    return -out if neg else out


def f32(d: float) -> float:
    return rnd32(F(d))


def fma32(a: float, b: float, c: float) -> float:
    return rnd32(F(a) * F(b) + F(c))


def mul32(a: float, b: float) -> float:
    return rnd32(F(a) * F(b))


def add32(a: float, b: float) -> float:
    return rnd32(F(a) + F(b))


def bf16_bits(f: float) -> int:
    """The kernel's round-to-nearest-even to bf16 on the float32 bits."""
    u = int(np.array(f, dtype=np.float32).view(np.uint32))
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFFFFFF
    return u >> 16


def bf16_value(h: int) -> float:
    return float(np.array(h << 16, dtype=np.uint32).view(np.float32))


# ------------------------------------------------------------ instances

def rot2(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s], [s, c]])


def rot3(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a + b*b - c*c - d*d, 2*(b*c - a*d), 2*(b*d + a*c)],
                     [2*(b*c + a*d), a*a - b*b + c*c - d*d, 2*(c*d - a*b)],
                     [2*(b*d - a*c), 2*(c*d + a*b), a*a - b*b - c*c + d*d]])


def adversarial_seeds(rng, dim, n, kappa_max, lo, hi, N_cells):
    """Seeds in and around the box, SPD matrices with condition numbers up to
    kappa_max, weights spread over several cell radii."""
    span = np.asarray(hi) - np.asarray(lo)
    x = np.asarray(lo) - 0.5 * span + 2.0 * span * rng.random((n, dim))
    A = np.empty((n, dim, dim))
    for i in range(n):
        kap = np.exp(rng.uniform(0.0, np.log(kappa_max)))
        ev = np.exp(rng.uniform(-1.0, 1.0)) * np.array([1.0, kap] if dim == 2 else
                                                         [1.0, np.sqrt(kap), kap])
        R = rot2(rng.uniform(0, np.pi)) if dim == 2 else rot3(rng)
        M = R @ np.diag(ev) @ R.T
        A[i] = 0.5 * (M + M.T)
    cell_r2 = (np.prod(span) / N_cells) ** (2.0 / dim)
    lam = np.array([np.linalg.eigvalsh(A[i]).max() for i in range(n)])
    w = rng.uniform(-6.0, 6.0, n) * cell_r2 * lam
    return x, A, w


def upper(A_i, r, c):
    return A_i[r, c] if r <= c else A_i[c, r]


def gershgorin(A_i, dim):
    return max(sum(abs(upper(A_i, r, c)) for c in range(dim)) for r in range(dim))


# ------------------------------------------------------------ the kernels' arithmetic

def seed_terms(x_i, A_i, w_i, anc, wmax, dim):
    """seed_terms in double, in the kernel's order (no contraction)."""
    e = [x_i[d] - anc[d] for d in range(dim)]
    wp = w_i - wmax
    ee = 0.0
    l = [0.0] * dim
    for r in range(dim):
        ae = 0.0
        for k in range(dim):
            ae += upper(A_i, r, k) * e[k]
        l[r] = -2.0 * ae
        ee += e[r] * ae
    c = ee - wp
    q = [(1.0 if r == k else 2.0) * upper(A_i, r, k) for r in range(dim) for k in range(r, dim)]
    return q, l, c, wp


def tile_anchor(g, tile_idx, ext, dim):
    anc_i = [tile_idx[d] * ext[d] + ext[d] // 2 for d in range(dim)]
    anc = [g["lo"][d] + float(anc_i[d]) * g["s"][d] for d in range(dim)]
    return anc_i, anc


def vec_cost(q, l, c, u, dim):
    """The vector tile's FP32 cost: lane_coef then the Horner step."""
    qf = [f32(t) for t in q]
    lf = [f32(t) for t in l]
    cf = f32(c)
    if dim == 2:
        a00, q01, q11 = qf
        beta = fma32(q01, u[1], lf[0])
        alpha = fma32(fma32(q11, u[1], lf[1]), u[1], cf)
    else:
        a00, q01, q02, q11, q12, q22 = qf
        beta = fma32(q01, u[1], fma32(q02, u[2], lf[0]))
        alpha = fma32(fma32(q11, u[1], fma32(q12, u[2], lf[1])), u[1],
                      fma32(fma32(q22, u[2], lf[2]), u[2], cf))
    return fma32(fma32(a00, u[0], beta), u[0], alpha)


def bf16_cost(q, l, c, v, h, dim, sequential):
    """The bf16 tile's cost: hi/lo slots, exact products, FP32 sum."""
    if dim == 2:
        cq = [f32(q[0] * h[0] * h[0]), f32(q[1] * h[0] * h[1]), f32(q[2] * h[1] * h[1])]
        fq = [v[0] * v[0], v[0] * v[1], v[1] * v[1]]
    else:
        pairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
        cq = [f32(q[t] * h[a] * h[b]) for t, (a, b) in enumerate(pairs)]
        fq = [v[a] * v[b] for a, b in pairs]
    cl = [f32(l[d] * h[d]) for d in range(dim)]
    fl = [v[d] for d in range(dim)]
    coefs = cq + cl + [f32(c)]
    feats = fq + fl + [1.0]
    nq = len(cq)
    prods = []
    for k, (cc, ff) in enumerate(zip(coefs, feats)):
        hi = bf16_bits(cc)
        rest = add32(cc, -bf16_value(hi))
        lo = bf16_bits(rest)
        assert F(cc) - F(bf16_value(hi)) == F(rest)  # exact difference
        assert abs(F(cc) - F(bf16_value(hi)) - F(bf16_value(lo))) <= F(2) ** -16 * abs(F(cc))
        fh = bf16_bits(ff)
        if k == len(coefs) - 1:
            # the constant in three parts (24 significant bits)
            third = bf16_bits(add32(rest, -bf16_value(lo)))
            assert F(rest) - F(bf16_value(lo)) == F(add32(rest, -bf16_value(lo)))
            parts = F(bf16_value(hi)) + F(bf16_value(lo)) + F(bf16_value(third))
            assert abs(F(cc) - parts) <= F(2) ** -24 * abs(F(cc))
            prods += [F(bf16_value(hi)), F(bf16_value(lo)), F(bf16_value(third))]
            continue
        if k < nq:
            flo = bf16_bits(ff - bf16_value(fh))
            assert bf16_value(fh) + bf16_value(flo) == ff  # integer features split exactly
            prods += [F(bf16_value(hi)) * F(bf16_value(fh)), F(bf16_value(hi)) * F(bf16_value(flo)),
                      F(bf16_value(lo)) * F(bf16_value(fh))]
        else:
            assert bf16_value(fh) == ff
            prods += [F(bf16_value(hi)) * F(ff), F(bf16_value(lo)) * F(ff)]
    for p in prods:  # products of two bf16 numbers are exact in FP32
        assert F(rnd32(p)) == p
    if not sequential:
        return rnd32(sum(prods, F(0)))
    acc = 0.0
    for p in prods:
        acc = rnd32(F(acc) + p)
    return acc


# ------------------------------------------------------------ the check

CASES = [
    # dim, grid, P (pixels per lane along axis 0), box, kappa_max
    (2, (256, 256), 4, ((0.0, 0.0), (1.0, 1.0)), 1e3),
    (2, (256, 256), 8, ((0.0, 0.0), (1.0, 1.0)), 1e3),
    (2, (200, 300), 4, ((3.5, -2.25), (4.5, 0.75)), 1e3),
    (2, (256, 256), 4, ((0.0, 0.0), (1.0, 1.0)), 1e6),
    (3, (64, 64, 64), 8, ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0)), 1e3),
    (3, (48, 40, 56), 4, ((-1.0, 2.0, 0.5), (1.0, 3.0, 1.5)), 1e3),
]


def tile_ext(dim, p):
    return (8 * p, 32) if dim == 2 else (4 * p, 8, 8)


def worst_ratios(case):
    """Largest error / bound over the sampled (seed, pixel) pairs of a case:
    (FP32 error / (9 2^-24 S), FP32 error / e32, bf16 error / e16)."""
    dim, grid, P, (lo, hi), kmax = CASES[case]
    rng = np.random.default_rng(700 + case)
    s = [(hi[d] - lo[d]) / grid[d] for d in range(dim)]
    g = {"lo": list(lo), "s": s}
    x, A, w = adversarial_seeds(rng, dim, 24, kmax, lo, hi, N_cells=200)
    wmax = float(np.max(w))
    ext = tile_ext(dim, P)
    # the kernels' bound of every Gershgorin bound, in FP32
    lam = f32(max(gershgorin(A[i], dim) for i in range(len(x))) * 1.0001)
    worst32 = worst16 = worst_gamma = 0.0
    ntiles = [max(1, grid[d] // ext[d]) for d in range(dim)]
    for _ in range(6):
        tile = [int(rng.integers(0, ntiles[d])) for d in range(dim)]
        anc_i, anc = tile_anchor(g, tile, ext, dim)
        for i in range(len(x)):
            q, l, c, wp = seed_terms(x[i], A[i], w[i], anc, wmax, dim)
            for _ in range(3):
                k = [tile[d] * ext[d] + int(rng.integers(0, ext[d])) for d in range(dim)]
                # FP32 local coordinates of the pixel, as the kernel forms them
                u = [mul32(float(k[d] - anc_i[d]) + 0.5, f32(s[d])) for d in range(dim)]
                # exact cost in the shifted gauge at the exact pixel centre
                y = [F(lo[d]) + (F(k[d]) + F(1, 2)) * F(s[d]) for d in range(dim)]
                dd = [y[d] - F(x[i][d]) for d in range(dim)]
                quad = sum(F(upper(A[i], r, cc)) * dd[r] * dd[cc] for r in range(dim) for cc in range(dim))
                C = quad - (F(w[i]) - F(wmax))
                assert C >= 0
                # the monomials of the expansion about the exact anchor
                ua = [(F(k[d] - anc_i[d]) + F(1, 2)) * F(s[d]) for d in range(dim)]
                ea = [F(x[i][d]) - (F(lo[d]) + F(anc_i[d]) * F(s[d])) for d in range(dim)]
                Ae = [sum(F(upper(A[i], r, cc)) * ea[cc] for cc in range(dim)) for r in range(dim)]
                S = (sum(abs(F(upper(A[i], r, cc)) * ua[r] * ua[cc]) for r in range(dim) for cc in range(dim))
                     + sum(abs(2 * Ae[d] * ua[d]) for d in range(dim))
                     + sum(ea[d] * Ae[d] for d in range(dim)) + abs(F(w[i]) - F(wmax)))
                Cf = float(C)
                # the pixel's r^2 = lambda_G |u|^2 (1.01), as the kernels form it
                r2 = mul32(mul32(lam, fma32(u[0], u[0], fma32(u[1], u[1], mul32(u[2], u[2]) if dim == 3
                                                               else 0.0))), f32(1.01))
                r = float(np.sqrt(r2))
                # the monomials' sum against its bound for a cost C
                assert float(S) <= Cf + 4.0 * r * np.sqrt(Cf) + 4.0 * r2
                c32 = vec_cost(q, l, c, u, dim)
                err32 = abs(F(c32) - C)
                # the rounding count: at most 9 roundings of 2^-24 per monomial
                worst_gamma = max(worst_gamma, float(err32 / S) / (9 * 2.0 ** -24))
                worst32 = max(worst32, float(err32) / e32(Cf, r2))
                h = [0.5 * s[d] for d in range(dim)]
                v = [float(2 * (k[d] - anc_i[d]) + 1) for d in range(dim)]
                for seq in (False, True):
                    c16 = bf16_cost(q, l, c, v, h, dim, seq)
                    worst16 = max(worst16, float(abs(F(c16) - C)) / e16(Cf, r2))
    return worst_gamma, worst32, worst16


def _split3(x: float):
    """An FP32 value as the exact sum of three bf16 parts, as the kernel
    splits it (round to nearest even, then the exact remainders)."""
    hi = bf16_bits(x)
    r = add32(x, -bf16_value(hi))
    assert F(x) - F(bf16_value(hi)) == F(r)
    mid = bf16_bits(r)
    lo_v = add32(r, -bf16_value(mid))
    assert F(r) - F(bf16_value(mid)) == F(lo_v)
    lo = bf16_bits(lo_v)
    assert bf16_value(lo) == lo_v  # the last remainder is a bf16 value
    return [bf16_value(hi), bf16_value(mid), bf16_value(lo)]


def _mfma16(start: float, prods, order):
    """One bf16 matrix-core product of K = 16 slots (exact products) added to
    the accumulator start: "fused" (one rounding), "left"/"right" (every
    addition rounded, slots first-to-last or last-to-first)."""
    for p in prods:
        assert F(rnd32(p)) == p  # products of two bf16 numbers are exact in FP32
    if order == "fused":
        return rnd32(F(start) + sum(prods, F(0)))
    acc = start
    for p in (prods if order == "left" else prods[::-1]):
        acc = rnd32(F(acc) + p)
    return acc


def hyb2_cost(q, l, c, o1, j, sgn, s, order):
    """The 2D hybrid tile's cost: as hyb3_cost with beta = (2a01 h1) o1 + l0
    and alpha = (a11 h1^2) o1^2 + (l1 h1) o1 + c, the feature o1^2 (up to
    961) as the exact sum of two bf16 values, each against a11's three
    parts."""
    h1 = 0.5 * s[1]
    cb = [f32(q[1] * h1), f32(l[0])]
    ca11, ca1 = f32(q[2] * h1 * h1), f32(l[1] * h1)
    cc = f32(c)
    f2 = float(o1 * o1)
    f2h = bf16_value(bf16_bits(f2))
    f2l = f2 - f2h
    for f in (float(o1), f2h, f2l):
        assert bf16_value(bf16_bits(f)) == f
    pb = [F(part) * F(f) for cf, f in zip(cb, [float(o1), 1.0]) for part in _split3(cf)]
    pa = ([F(part) * F(f2h) for part in _split3(ca11)] + [F(part) * F(f2l) for part in _split3(ca11)]
          + [F(part) * F(float(o1)) for part in _split3(ca1)])
    chi = bf16_value(bf16_bits(cc))
    pa.append(F(chi))
    crest = add32(cc, -chi)
    assert F(cc) - F(chi) == F(crest)
    beta = _mfma16(0.0, pb, order)
    alpha = _mfma16(crest, pa, order)
    uj = mul32(float(j) + 0.5, f32(s[0]))
    qq = fma32(f32(q[0]), mul32(uj, uj), alpha)
    return fma32(-beta if sgn else beta, uj, qq)


def hyb3_cost(q, l, c, o1, o2, j, sgn, s, order):
    """The 3D hybrid tile's cost: beta and alpha from bf16 matrix-core
    products (coefficients in half-pixel units, rounded to FP32 once and
    split exactly into three bf16 parts; exact integer features), alpha's
    accumulator starting at c - c_hi; then q = fl(a00 u_j^2 + alpha) and
    C = fl(q +- beta u_j) on the ALU."""
    h1, h2 = 0.5 * s[1], 0.5 * s[2]
    cb = [f32(q[1] * h1), f32(q[2] * h2), f32(l[0])]
    ca = [f32(q[3] * h1 * h1), f32(q[4] * h1 * h2), f32(q[5] * h2 * h2), f32(l[1] * h1), f32(l[2] * h2)]
    cc = f32(c)
    fb = [float(o1), float(o2), 1.0]
    fa = [float(o1 * o1), float(o1 * o2), float(o2 * o2), float(o1), float(o2)]
    for f in fb + fa:
        assert bf16_value(bf16_bits(f)) == f  # the features are bf16 values
    pb = [F(part) * F(f) for cf, f in zip(cb, fb) for part in _split3(cf)]
    pa = [F(part) * F(f) for cf, f in zip(ca, fa) for part in _split3(cf)]
    chi = bf16_value(bf16_bits(cc))
    pa.append(F(chi))
    crest = add32(cc, -chi)
    assert F(cc) - F(chi) == F(crest)
    beta = _mfma16(0.0, pb, order)
    alpha = _mfma16(crest, pa, order)
    uj = mul32(float(j) + 0.5, f32(s[0]))
    qq = fma32(f32(q[0]), mul32(uj, uj), alpha)
    return fma32(-beta if sgn else beta, uj, qq)


HYB_CASES = [
    # grid, box, kappa_max
    ((64, 64, 64), ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0)), 1e3),
    ((48, 40, 56), ((-1.0, 2.0, 0.5), (1.0, 3.0, 1.5)), 1e3),
    ((64, 48, 40), ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0)), 1e6),
    ((256, 256), ((0.0, 0.0), (1.0, 1.0)), 1e3),
    ((200, 300), ((3.5, -2.25), (4.5, 0.75)), 1e3),
    ((256, 256), ((0.0, 0.0), (1.0, 1.0)), 1e6),
]


@pytest.mark.parametrize("case", range(len(HYB_CASES)))
def test_hybrid_costs_within_bounds(case):
    """The hybrid tile (3D 16 x 16 x 8 pixels, 2D 32 x 32; rows +-(j + 1/2) s0
    about the anchor; beta and alpha from bf16 matrix-core products): its
    FP32 cost, under every rounding model of the matrix-core sums, is within
    19 (3D) or 13 (2D) roundings of 2^-24 of the monomials' sum S, and within
    the tile's bound of the exact cost (3D 1.3125 e32, 2D e32)."""
    grid, (lo, hi), kmax = HYB_CASES[case]
    dim = len(grid)
    rng = np.random.default_rng(900 + case)
    s = [(hi[d] - lo[d]) / grid[d] for d in range(dim)]
    g = {"lo": list(lo), "s": s}
    x, A, w = adversarial_seeds(rng, dim, 20, kmax, lo, hi, N_cells=200)
    wmax = float(np.max(w))
    ext = (16, 16, 8) if dim == 3 else (32, 32)
    half_rows = ext[0] // 2
    lam = f32(max(gershgorin(A[i], dim) for i in range(len(x))) * 1.0001)
    worst_gamma = worst32 = 0.0
    ntiles = [max(1, grid[d] // ext[d]) for d in range(dim)]
    for _ in range(4):
        tile = [int(rng.integers(0, ntiles[d])) for d in range(dim)]
        anc_i, anc = tile_anchor(g, tile, ext, dim)
        for i in range(len(x)):
            q, l, c, wp = seed_terms(x[i], A[i], w[i], anc, wmax, dim)
            for _ in range(3):
                j, sgn = int(rng.integers(0, half_rows)), int(rng.integers(0, 2))
                k = [anc_i[0] + (-1 - j if sgn else j)] + \
                    [tile[d] * ext[d] + int(rng.integers(0, ext[d])) for d in range(1, dim)]
                u1 = mul32(float(k[1] - anc_i[1]) + 0.5, f32(s[1]))
                u2 = mul32(float(k[2] - anc_i[2]) + 0.5, f32(s[2])) if dim == 3 else 0.0
                u0 = mul32(float(j) + 0.5, f32(s[0])) * (-1.0 if sgn else 1.0)
                assert u0 == mul32(float(k[0] - anc_i[0]) + 0.5, f32(s[0]))
                y = [F(lo[d]) + (F(k[d]) + F(1, 2)) * F(s[d]) for d in range(dim)]
                dd = [y[d] - F(x[i][d]) for d in range(dim)]
                C = sum(F(upper(A[i], r, cc)) * dd[r] * dd[cc] for r in range(dim) for cc in range(dim)) \
                    - (F(w[i]) - F(wmax))
                assert C >= 0
                ua = [(F(k[d] - anc_i[d]) + F(1, 2)) * F(s[d]) for d in range(dim)]
                ea = [F(x[i][d]) - (F(lo[d]) + F(anc_i[d]) * F(s[d])) for d in range(dim)]
                Ae = [sum(F(upper(A[i], r, cc)) * ea[cc] for cc in range(dim)) for r in range(dim)]
                S = (sum(abs(F(upper(A[i], r, cc)) * ua[r] * ua[cc]) for r in range(dim) for cc in range(dim))
                     + sum(abs(2 * Ae[d] * ua[d]) for d in range(dim))
                     + sum(ea[d] * Ae[d] for d in range(dim)) + abs(F(w[i]) - F(wmax)))
                Cf = float(C)
                r2 = mul32(mul32(lam, fma32(u0, u0, fma32(u1, u1, mul32(u2, u2)))), f32(1.01))
                assert float(S) <= Cf + 4.0 * np.sqrt(r2) * np.sqrt(Cf) + 4.0 * r2
                for order in ("fused", "left", "right"):
                    if dim == 3:
                        o1, o2 = 2 * (k[1] - anc_i[1]) + 1, 2 * (k[2] - anc_i[2]) + 1
                        cost = hyb3_cost(q, l, c, o1, o2, j, sgn, s, order)
                        nround, bound = 19, 1.3125 * e32(Cf, r2)
                    else:
                        o1 = 2 * (k[1] - anc_i[1]) + 1
                        cost = hyb2_cost(q, l, c, o1, j, sgn, s, order)
                        nround, bound = 13, e32(Cf, r2)
                    err = abs(F(cost) - C)
                    worst_gamma = max(worst_gamma, float(err / S) / (nround * 2.0 ** -24))
                    worst32 = max(worst32, float(err) / bound)
    assert worst_gamma <= 1.0, worst_gamma
    assert worst32 <= 1.0, worst32


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fp32_and_bf16_costs_within_bounds(case):
    worst_gamma, worst32, worst16 = worst_ratios(case)
    assert worst_gamma <= 1.0, worst_gamma
    assert worst32 <= 1.0, worst32
    assert worst16 <= 1.0, worst16


def test_double_cost_slack():
    """The double-precision evaluation of the definition (d = y - x, each row
    of A d, d^T (A d), minus w) is within 2^-48 ((kappa + 1) C + |w_max| +
    lambda_G sum_d Y_d^2) of the exact cost, C the cost in the shifted gauge:
    the slack the certificates add (with 2^-44) covers twice that."""
    rng = np.random.default_rng(711)
    worst = 0.0
    for dim, lo, hi, kmax in [(2, (1e4, -3e3), (1e4 + 1.0, -3e3 + 1.0), 1e6),
                              (3, (-50.0, 20.0, 7.0), (-49.0, 21.0, 8.0), 1e4),
                              (2, (0.0, 0.0), (1.0, 1.0), 1e8)]:
        grid = (97,) * dim
        s = [(hi[d] - lo[d]) / grid[d] for d in range(dim)]
        x, A, w = adversarial_seeds(rng, dim, 16, kmax, lo, hi, N_cells=50)
        w = w + 1e3  # a large common offset of the weights
        wmax = float(np.max(w))
        lamG = max(gershgorin(A[i], dim) for i in range(len(x)))
        Y2 = sum((abs(lo[d]) + grid[d] * s[d]) ** 2 for d in range(dim))
        for i in range(len(x)):
            ev = np.linalg.eigvalsh(A[i])
            kap = gershgorin(A[i], dim) / ev.min()
            for _ in range(20):
                k = [int(rng.integers(0, grid[d])) for d in range(dim)]
                y = [lo[d] + (k[d] + 0.5) * s[d] for d in range(dim)]
                d_ = [y[r] - x[i][r] for r in range(dim)]
                qd = 0.0
                for r in range(dim):
                    row = 0.0
                    for cc in range(dim):
                        t = upper(A[i], r, cc) * d_[cc]
                        row = t if cc == 0 else row + t
                    t = d_[r] * row
                    qd = t if r == 0 else qd + t
                Cd = qd - w[i]
                ye = [F(lo[d]) + (F(k[d]) + F(1, 2)) * F(s[d]) for d in range(dim)]
                de = [ye[r] - F(x[i][r]) for r in range(dim)]
                Ce = sum(F(upper(A[i], r, cc)) * de[r] * de[cc] for r in range(dim) for cc in range(dim)) - F(w[i])
                Cs = float(Ce + F(wmax))
                bound = 2.0 ** -48 * ((kap + 1.0) * Cs + abs(wmax) + lamG * Y2)
                worst = max(worst, float(abs(F(Cd) - Ce)) / bound)
    assert worst <= 1.0, worst
