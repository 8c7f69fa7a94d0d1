"""Pair-by-pair check of the precision form's screen bound (Section 4).

The matrix-core screens evaluate the inner-product form of eq. (ip2) in
bf16 / fp16 / fp32 with fp32 accumulation and only reject a pair when that
value proves it to be outside the radius.  Their start values rest on a
rounding bound: operand representation, operands below the normal range,
and the accumulation inside the matrix instruction, whose order and rounding
are not specified (the bound allows twice the sequential-sum error).  Here
the library's test entry point (include/snn_testing.h) hands back every
pair's screen value D, the candidates' H, the start values C and both
operand row sets for small adversarial inputs, and the test checks, in
float64 / exact arithmetic of its own:

1. the operands are the round-to-nearest-even bf16 / fp16 values of the
   centred rows (computed here by frexp and rint, not bit tricks);
2. the accumulation model: |D - (sum_k A_k B_k + C)| <= 2 gamma32_{K+1}
   (sum_k |A_k B_k| + |C|), plus the products of operands below the normal
   range in case the matrix core reads those as zero;
3. the whole screen error against the derived per-pair bound E:
   |D - (s^2 y_q . y_j + C)| <= E, with y = fl32(p - mu) and s the fp16
   scale (1 otherwise);
4. every pair the normative rule accepts passes (D >= H), and the CSR equals
   the brute-force oracle's.

Inputs: coordinates at bf16 and fp16 rounding ties, hi/lo splits whose lo
term is subnormal and fp16 operands below 2^-14, every K padding (d = 1, 15,
17, 33, 42), near-duplicates far from the mean, and scaled lattices with
pairs exactly at S = fl(R*R).
"""

import math
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0**-24


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_07679_amd import binding

    return binding


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


# ---- rounding to bf16 / fp16 by the definition: nearest value of the format,
# ties to the even significand; spacing 2^(e - p) at exponent e, fixed below
# the normal range
def round_to_format(x, p, emin):
    """x (float32 array) rounded to a binary format with p significand bits
    (the implicit one included) and smallest normal exponent emin (values
    2^emin <= |v|), returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)  # x = m 2^e, 0.5 <= |m| < 1: the leading bit is 2^(e-1)
    e = np.maximum(e - 1, emin)  # exponent of the leading bit, clamped below the normal range
    ulp = np.ldexp(1.0, e - (p - 1))
    return np.rint(x / ulp) * ulp  # rint: ties to even


def bf16_value(x):
    return round_to_format(x, 8, -126)


def f16_value(x):
    return round_to_format(x, 11, -14)


def decode_bf16(bits):
    u = bits.astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def decode_f16(bits):
    return bits.astype(np.uint16).view(np.float16).astype(np.float64)


def gamma32(k):
    return k * U32 / (1.0 - k * U32)


def c_rep(kind):
    ub, uh = 2.0**-8, 2.0**-11
    return {"bf16": ub * (2 + ub), "bf16x3": ub * ub * (3 + 3 * ub), "fp16": uh * (2 + uh), "fp32": 0.0}[kind]


def screen_kind(lay):
    prec = {1: "mixed", 3: "fp32", 4: "fp16"}[lay["precision"]]
    if prec == "mixed":
        return "bf16x3" if lay["terms"] == 3 else "bf16"
    return prec


def check_screen(B, P, Q, R, precision, terms=0, label=""):
    """All four checks for one input set and one screen.  Returns the
    observed statistics."""
    idx = B.Index(to_dev(P))
    out = idx.screen_values(to_dev(Q), R, precision=precision, terms=terms)
    lay = out["layout"]
    kind = screen_kind(lay)
    D = out["D"].cpu().numpy().astype(np.float64)
    H = out["H"].cpu().numpy().astype(np.float64)
    C = out["C"].cpu().numpy().astype(np.float64)
    A = out["A"].cpu().numpy()
    Bo = out["B"].cpu().numpy()
    view = idx.view()
    mu = view["mu"].cpu().numpy()
    perm = view["perm"].cpu().numpy()
    d = P.shape[1]
    m, n = Q.shape[0], P.shape[0]
    e = lay["scale_exp"]
    s2 = 2.0 ** (2 * e)
    # centred rows as the index forms them: fl32(p - mu), p promoted exactly
    yq = (Q.astype(np.float64) - mu).astype(np.float32)
    yj = (P[perm].astype(np.float64) - mu).astype(np.float32)

    # 1. operands
    K = lay["chain"]
    if kind == "fp32":
        Av = A.astype(np.float64)
        assert np.array_equal(A[:, :d], yq), f"{label}: fp32 query rows"
        assert np.array_equal(Bo, yj), f"{label}: fp32 candidate rows"
        assert np.array_equal(A[:, d], C.astype(np.float32)), f"{label}: start values"
        Aeff = np.zeros((m, K))
        Aeff[:, :d] = yq
        Beff = np.zeros((n, K))
        Beff[:, :d] = yj
        Cv = C
    else:
        dec = decode_f16 if kind == "fp16" else decode_bf16
        Av, Bv = dec(A), dec(Bo)
        if kind == "fp16":
            wq = np.zeros((m, K))
            wq[:, :d] = f16_value(np.ldexp(yq.astype(np.float64), e))
            wj = np.zeros((n, K))
            wj[:, :d] = f16_value(np.ldexp(yj.astype(np.float64), e))
        elif kind == "bf16":
            wq = np.zeros((m, K))
            wq[:, :d] = bf16_value(yq)
            wj = np.zeros((n, K))
            wj[:, :d] = bf16_value(yj)
        else:
            hq, hj = bf16_value(yq), bf16_value(yj)
            lq = bf16_value((yq.astype(np.float64) - hq).astype(np.float32))
            lj = bf16_value((yj.astype(np.float64) - hj).astype(np.float32))
            wq = np.zeros((m, K))
            wq[:, :3 * d] = np.concatenate([hq, hq, lq], axis=1)
            wj = np.zeros((n, lay["kb"]))
            seg = [hj, lj, hj] if lay["kb"] >= 3 * d else [hj, lj]
            wj[:, :len(seg) * d] = np.concatenate(seg, axis=1)
        assert np.array_equal(Av, wq), f"{label}: query operands are not the rounded rows"
        assert np.array_equal(Bv, wj), f"{label}: candidate operands are not the rounded rows"
        Aeff = Av
        # the product chain reuses the first candidate slices past the stored row
        Beff = Bv if lay["kb"] == K else np.concatenate([Bv, Bv[:, :K - lay["kb"]]], axis=1)
        Cv = C

    # 2. accumulation: exact products (they fit float64), long-double sums
    Al, Bl = Aeff.astype(np.longdouble), Beff.astype(np.longdouble)
    X = (Al @ Bl.T) + Cv[:, None].astype(np.longdouble)
    absum = (np.abs(Al) @ np.abs(Bl).T) + np.abs(Cv)[:, None].astype(np.longdouble)
    tiny = 2.0**-14 if kind == "fp16" else 2.0**-126
    sub_a = (np.abs(Aeff) < tiny) & (Aeff != 0)
    sub_b = (np.abs(Beff) < tiny) & (Beff != 0)
    flush = (np.abs(Al) * sub_a) @ np.abs(Bl).T + np.abs(Al) @ (np.abs(Bl) * sub_b).T
    err_acc = np.abs(D.astype(np.longdouble) - X)
    ulp_slack = absum * np.longdouble(2.0**-52)
    g = gamma32(K + 1)
    assert np.all(err_acc <= 2 * g * absum + flush + ulp_slack), f"{label}: accumulation beyond the model"
    acc_ratio = float(np.max(err_acc / np.maximum(g * absum, np.longdouble(1e-300))))

    # 3. the screen error against the derived per-pair bound
    ydot = yq.astype(np.longdouble) @ yj.astype(np.longdouble).T
    nq = np.sqrt(np.sum(yq.astype(np.float64) ** 2, axis=1))
    nj = np.sqrt(np.sum(yj.astype(np.float64) ** 2, axis=1))
    t = 3.0 if kind == "bf16x3" else 1.0
    delta = 2.0 ** (-14 - e) if kind == "fp16" else 2.0**-126
    sub = 1.01 * (1 + 2.0**-8) * t * math.sqrt(K) * delta
    e_sub = sub * (nq[:, None] + nj[None, :]) + 1.01 * t * K * delta * delta
    nn = nq[:, None] * nj[None, :]
    E_rep = c_rep(kind) * nn + e_sub
    E_acc = 2 * g * (1.02 * nn + e_sub + np.abs(Cv)[:, None] / s2) * 1.01
    E = s2 * (E_rep + E_acc) * (1 + 1e-12)
    err = np.abs(D - (s2 * ydot + Cv[:, None]).astype(np.float64))
    assert np.all(err <= E), f"{label}: screen error beyond the derived bound (max ratio {np.max(err / E):.3g})"
    ratio = float(np.max(err / E))

    # 4. every accepted pair passes; the CSR equals the oracle's
    ref = oracle.brute_radius(P, Q, R)
    acc_mask = np.zeros((m, n), dtype=bool)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    for q in range(m):
        acc_mask[q, inv[ref.col[ref.row_ptr[q]:ref.row_ptr[q + 1]]]] = True
    passes = D >= H[None, :]
    assert np.all(passes[acc_mask]), f"{label}: an accepted pair fails the screen"
    rp, col, dist = (x.cpu().numpy() for x in idx.query(to_dev(Q), R, precision=precision, terms=terms)[:3])
    assert np.array_equal(rp, ref.row_ptr) and np.array_equal(col, ref.col), f"{label}: CSR differs from the oracle"
    margin = float(np.min((D - H[None, :])[acc_mask]) / s2) if acc_mask.any() else float("nan")
    st = {"kind": kind, "accepted": int(acc_mask.sum()), "passed": int(passes.sum()), "acc_ratio": acc_ratio,
          "bound_ratio": ratio, "min_margin": margin}
    say(f"  {label} {kind}: accepted {st['accepted']} passed {st['passed']} of {m * n}, "
        f"accumulation error / gamma_(K+1) sum {acc_ratio:.3f}, screen error / bound {ratio:.3f}")
    idx.close()
    return st


def screens_for(d):
    out = [("mixed", 1), ("fp16", 0)]
    if 3 * d <= 128:
        out.append(("mixed", 3))
    if d <= 16:
        out.append(("fp32", 0))
    return out


def rng(*tag):
    return np.random.default_rng([2212, 7679, 77, *tag])


def symmetric(X):
    """[X; -X]: column sums are exactly zero when the float64 sums are exact,
    so the centre is 0 and the centred rows are the coordinates themselves."""
    return np.concatenate([X, -X]).astype(X.dtype)


def tie_set(d=16, n=1500, m=160):
    """Coordinates halfway between neighbouring bf16 values, or neighbouring
    fp16 values after the screen's power-of-two scale, or plain."""
    g = rng(1, d)
    e = g.integers(-3, 3, size=(n, d)).astype(np.float64)
    odd = 2 * g.integers(0, 64, size=(n, d)) + 1
    bf_tie = (128 + odd / 2.0) / 128.0 * 2.0**e  # (1 + k/128) + 2^-8: halfway between bf16 values
    f16_tie = (1.0 + (2 * g.integers(0, 512, size=(n, d)) + 1) * 2.0**-11) * 2.0**e
    plain = np.round(g.standard_normal((n, d)) * 1024.0) / 1024.0  # dyadic: the centre stays exactly 0
    pick = g.integers(0, 3, size=(n, d))
    X = np.where(pick == 0, bf_tie, np.where(pick == 1, f16_tie, plain)).astype(np.float32)
    X *= np.where(g.random((n, d)) < 0.5, -1.0, 1.0).astype(np.float32)
    P = symmetric(X)
    Q = np.concatenate([P[g.choice(P.shape[0], m // 2, replace=False)],
                        P[g.choice(P.shape[0], m - m // 2, replace=False)] * np.float32(1.0 + 2.0**-9)])
    return P, Q.astype(np.float32)


def radius_for(P, Q, k):
    """A radius with about k neighbours per query (from a sample of squared distances)."""
    S = np.sort(oracle.normative_sqdist(P, Q[0]))
    return float(np.sqrt(S[min(k, S.size - 1)]))


@pytest.mark.parametrize("precision,terms", [("mixed", 1), ("mixed", 3), ("fp16", 0), ("fp32", 0)])
def test_rounding_ties(B, precision, terms):
    P, Q = tie_set()
    R = radius_for(P, Q, 40)
    say(f"ties d=16 n={P.shape[0]} m={Q.shape[0]} R={R:.4f}")
    st = check_screen(B, P, Q, R, precision, terms, "ties")
    assert st["accepted"] > Q.shape[0]


def subnormal_set(d=16, n=1200, m=128):
    """Rows mixing coordinates near 1 with ones whose bf16 lo term is
    subnormal (|y| ~ 2^-120), fp32-subnormal coordinates, and ones that fall
    below fp16's normal range after the screen's scale."""
    g = rng(2, d)
    X = g.standard_normal((n, d))
    kind = g.integers(0, 4, size=(n, d))
    X = np.where(kind == 1, X * 2.0**-120, X)
    X = np.where(kind == 2, X * 2.0**-130, X)
    X = np.where(kind == 3, X * 2.0**-30, X)  # fp16 subnormal after the scale 2^12
    X = X.astype(np.float32)
    P = symmetric(X)
    Q = P[g.choice(P.shape[0], m, replace=False)] * np.float32(1 - 2.0**-12)
    return P, Q.astype(np.float32)


@pytest.mark.parametrize("precision,terms", [("mixed", 1), ("mixed", 3), ("fp16", 0), ("fp32", 0)])
def test_subnormal_operands(B, precision, terms):
    P, Q = subnormal_set()
    R = radius_for(P, Q, 30)
    say(f"subnormal terms d=16 R={R:.4g}")
    check_screen(B, P, Q, R, precision, terms, "subnormal")


@pytest.mark.parametrize("d", [1, 15, 17, 33, 42])
def test_k_padding(B, d):
    g = rng(3, d)
    P = g.standard_normal((2500, d)).astype(np.float32)
    Q = np.concatenate([P[:60] + np.float32(0.01), g.standard_normal((60, d)).astype(np.float32)])
    R = radius_for(P, Q, 25)
    say(f"K padding d={d} R={R:.4f}")
    for precision, terms in screens_for(d):
        check_screen(B, P, Q, R, precision, terms, f"d={d}")


def test_near_duplicates_far_from_the_mean(B):
    g = rng(4)
    d = 16
    centre = np.full(d, 1000.0)
    A = centre + 1e-3 * g.standard_normal((800, d))
    P = np.concatenate([A, -A]).astype(np.float32)  # mean 0, |y| ~ 4000
    Q = P[g.choice(P.shape[0], 96, replace=False)] + np.float32(2e-4)
    R = 0.004
    say(f"near-duplicates far from the mean R={R}")
    for precision, terms in screens_for(d):
        st = check_screen(B, P, Q, R, precision, terms, "far")
        assert st["accepted"] > 0


@pytest.mark.parametrize("offset", [0.0, 1000.0])
def test_scaled_lattice_ties(B, offset):
    """Lattice points of spacing 1/8 in d = 3: squared distances are k/64, so
    pairs with S exactly fl(R*R) = 25/64 exist for R = 5/8 (inclusive)."""
    ax = np.arange(-6, 7) / 8.0
    L = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3) + offset
    P = L.astype(np.float64)
    Q = (np.stack(np.meshgrid(ax[4:9], ax[4:9], ax[4:9], indexing="ij"), axis=-1).reshape(-1, 3) + offset)
    R = 5.0 / 8.0
    say(f"scaled lattice offset={offset} n={P.shape[0]} m={Q.shape[0]}")
    for precision, terms in screens_for(3):
        st = check_screen(B, P, Q, R, precision, terms, f"lattice+{offset}")
        assert st["accepted"] > 0
    # ties at the boundary are counted
    S = oracle.normative_sqdist(P, Q[0])
    assert np.any(S == R * R)
