"""Pins of the FP64 oracle against things other than itself: hand-worked
fixtures, exact-rational brute force, eID set counting, closed forms, the
PID-mean identity of Sec. 4.1 and the invariants of Sec. 3.3 / 3.4.  CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import erfc

import oracle
import synth
from tests import golden


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _dyadic(n, m, seed, denom=16, zero_rows=()):
    rng = _rng(seed)
    U = rng.integers(0, denom + 1, size=(n, m)) / denom
    for r in zero_rows:
        U[r] = 0.0
    return U


# ---------------------------------------------------------------- fixtures
def test_golden_handworked_weighted():
    g = golden.load("handworked_weighted_3x4.txt")
    U = np.array([[float(v) for v in g[k]] for k in ("u1", "u2", "u3")])
    w = np.array([float(v) for v in g["w"]])
    r = oracle.pid(U, w)
    np.testing.assert_allclose(r["mass"], [float(v) for v in g["mass"]], rtol=0, atol=1e-15)
    P = np.array([[float(v) for v in g[f"inclusion_row{i}"]] for i in (1, 2, 3)])
    np.testing.assert_allclose(r["inclusion"], P, rtol=0, atol=1e-15)
    for key in ("in_in", "in_out", "depth"):
        np.testing.assert_allclose(r[key], [float(v) for v in g[key]], rtol=0, atol=1e-15)
    rank, _ = oracle.rank_order(r["depth"])
    assert rank.tolist() == [int(v) for v in g["rank"]]
    pm = oracle.pid_mean(U, w)
    assert abs(pm["mbar"] - float(g["mean_mbar"][0])) < 1e-15
    for key in ("in_in", "in_out", "depth"):
        np.testing.assert_allclose(pm[key], [float(v) for v in g["mean_" + key]], rtol=0, atol=1e-15)


def test_golden_nested_chain_binary_exact():
    g = golden.load("nested_binary_chain.txt")
    B = np.array([[int(v) for v in g[k]] for k in ("a1", "a2", "a3")], dtype=np.uint8)
    rb = oracle.binary_pid(B)
    # IN_in is one correctly rounded division of exact integers: bit-exact
    assert rb["in_in"].tolist() == [float(v) for v in g["in_in"]]
    np.testing.assert_allclose(rb["in_out"], [float(v) for v in g["in_out"]], rtol=4e-16, atol=0)
    rank, _ = oracle.rank_order(rb["depth"])
    assert rank.tolist() == [int(v) for v in g["rank"]]
    rm = oracle.binary_pid_mean(B)
    assert rm["in_in"].tolist() == [float(v) for v in g["mean_in_in"]]
    assert rm["in_out"].tolist() == [float(v) for v in g["mean_in_out"]]
    assert rm["depth"].tolist() == [float(v) for v in g["mean_depth"]]
    # the soft path on the same 0/1 values agrees
    rs = oracle.pid(B)
    np.testing.assert_allclose(rs["depth"], [float(v) for v in g["depth"]], rtol=0, atol=1e-15)


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed,n,m,weighted,zero_rows", [
    (1, 1, 7, False, ()), (2, 3, 11, True, ()), (3, 5, 16, True, (2,)),
    (4, 6, 23, False, ()), (5, 4, 9, True, (0, 3)), (6, 6, 17, True, ()),
])
def test_exact_rational_bruteforce(seed, n, m, weighted, zero_rows):
    U = _dyadic(n, m, seed, zero_rows=zero_rows)
    w = _rng(seed + 100).integers(1, 5, size=m).astype(np.float64) if weighted else None
    ex = oracle.exact_pid(U, w)
    r = oracle.pid(U, w)
    np.testing.assert_allclose(r["inclusion"], np.array([[float(v) for v in row] for row in ex["inclusion"]]), atol=1e-15, rtol=0)
    for key in ("in_in", "in_out", "depth"):
        np.testing.assert_allclose(r[key], [float(v) for v in ex[key]], atol=1e-15, rtol=0)
    exm = oracle.exact_pid_mean(U, w)
    rm = oracle.pid_mean(U, w)
    for key in ("in_in", "in_out", "depth"):
        np.testing.assert_allclose(rm[key], [float(v) for v in exm[key]], atol=1e-15, rtol=0)
    for zr in zero_rows:   # zero-mass member: every inclusion it starts is 0 -> depth 0
        assert r["depth"][zr] == 0.0 and rm["depth"][zr] == 0.0


# ---------------------------------------------------------------- binary / eID
@pytest.mark.parametrize("seed", [11, 12, 13])
def test_binary_reduces_to_eid(seed):
    B = synth.random_binary(7, 60, seed).numpy()
    assert (B.sum(1) > 0).all()
    ein, eout, edep = oracle.eid_sets(B)
    rs = oracle.pid(B)
    rb = oracle.binary_pid(B)
    for r in (rs, rb):
        np.testing.assert_allclose(r["in_in"], [float(v) for v in ein], atol=1e-15, rtol=0)
        np.testing.assert_allclose(r["in_out"], [float(v) for v in eout], atol=1e-15, rtol=0)
        np.testing.assert_allclose(r["depth"], [float(v) for v in edep], atol=1e-15, rtol=0)
    # IN_in of the canonical binary path is the correctly rounded exact value
    assert rb["in_in"].tolist() == [float(v) for v in ein]
    # IN_out: a few ulps of the exact rational
    for a, b in zip(rb["in_out"], eout):
        assert abs(Fraction(a) - b) <= 8 * Fraction(2) ** -53 * max(b, Fraction(1, 2 ** 10))


def test_empty_member_conventions_differ():
    """An empty mask: eID's operator gives 1 (Eq. 1), the PID operator gives 0
    (Sec. 3.2); the oracle follows PID."""
    B = np.array([[1, 1, 0, 0], [0, 0, 0, 0], [1, 1, 1, 0]], dtype=np.uint8)
    _, _, edep = oracle.eid_sets(B)
    r = oracle.binary_pid(B)
    assert r["in_in"][1] == 0.0 and r["in_out"][1] == 0.0
    assert edep[1] > 0      # eID counts the empty set as included everywhere
    assert oracle.incl(B[1], B[0]) == 0.0


def test_nested_chain_closed_form():
    rng = _rng(21)
    counts = np.sort(rng.choice(np.arange(1, 400), size=9, replace=False))
    n, M = counts.size, int(counts[-1])
    B = np.zeros((n, M), dtype=np.uint8)
    for i, a in enumerate(counts):
        B[i, :a] = 1
    r = oracle.binary_pid(B)
    for i in range(n):      # 0-based closed form of the nested chain
        a = [Fraction(int(c)) for c in counts]
        cin = (Fraction(n - i) + sum(a[j] / a[i] for j in range(i))) / n
        cout = (Fraction(i + 1) + sum(a[i] / a[j] for j in range(i + 1, n))) / n
        assert r["in_in"][i] == float(cin)
        assert abs(r["in_out"][i] - float(cout)) <= 4e-16
    # the middle of the chain is the deepest
    assert int(np.argmax(r["depth"])) in (n // 2 - 1, n // 2, n // 2 + 1)


# ---------------------------------------------------------------- orderings
def test_concentric_soft_disks_unimodal():
    radii = np.linspace(0.08, 0.42, 25)
    U = synth.concentric_disks(radii, 96, 40.0).numpy()
    for r in (oracle.pid(U), oracle.pid_mean(U)):
        assert np.all(np.diff(r["in_in"]) < 0), "IN_in must fall with the radius"
        assert np.all(np.diff(r["in_out"]) > 0), "IN_out must rise with the radius"
        d = r["depth"]
        k = int(np.argmax(d))
        assert np.all(np.diff(d[: k + 1]) > 0) and np.all(np.diff(d[k:]) < 0)
        assert 0 < k < len(radii) - 1


def test_fig3_fuzzy_disks_centred_deeper():
    """Three soft disks with radii 3, 2, 4 pixels and a Gaussian fall-off of
    variance 0.8 outside the radius (the setting of Fig. 3): u1 centred between
    the others is deeper than u1 shifted away."""
    res = 40
    yy, xx = np.meshgrid(np.arange(res) + 0.5, np.arange(res) + 0.5, indexing="ij")

    def disk(cx, cy, r):
        d = np.hypot(xx - cx, yy - cy)
        return np.where(d <= r, 1.0, np.exp(-((d - r) ** 2) / (2 * 0.8))).ravel()

    u2, u3 = disk(20, 20, 2), disk(20, 20, 4)
    centred = oracle.pid(np.stack([disk(20, 20, 3), u2, u3]))["depth"][0]
    shifted = oracle.pid(np.stack([disk(27, 20, 3), u2, u3]))["depth"][0]
    assert centred > shifted


# ---------------------------------------------------------------- Sec. 4.1
@pytest.mark.parametrize("seed", [31, 32])
def test_pidmean_recall_identity(seed):
    """``u_i <_p ubar == (1/N) sum_j u_i <_p u_j`` (Sec. 4.1, Eq. PIDmean)."""
    U = synth.random_soft(9, 300, seed).numpy()
    w = _rng(seed).uniform(0.5, 1.5, size=300)
    a, b = oracle.pid(U, w), oracle.pid_mean(U, w)
    np.testing.assert_allclose(a["in_in"], b["in_in"], atol=1e-15, rtol=0)
    lit = oracle.pid_mean_literal(U, w)
    for key in ("in_in", "in_out", "depth"):
        np.testing.assert_allclose(lit[key], b[key], atol=1e-15, rtol=0)


@pytest.mark.parametrize("seed", [33, 34])
def test_pidmean_numerators_are_gram_row_sums(seed):
    """``A_i = sum_x w u_i s(x) = sum_j G_ij`` with ``s = sum_j u_j``: PID-mean's
    IN_out is the Gram row sum over the total mass (Sec. 4.1 against Sec. 3.2);
    the all-pairs and PID-mean depths of one ensemble share these sums."""
    U = synth.random_soft(11, 350, seed).numpy()
    w = _rng(seed).uniform(0.5, 1.5, size=350)
    G, m = oracle.gram(U, w), oracle.mass(U, w)
    b = oracle.pid_mean(U, w)
    np.testing.assert_allclose(b["in_out"], G.sum(axis=1) / m.sum(), rtol=1e-14, atol=0)
    np.testing.assert_allclose(b["in_in"], G.sum(axis=1) / (len(U) * m), rtol=1e-14, atol=0)


def test_equal_masses_pidmean_equals_pid():
    """Integer translations of one pattern inside the grid have equal masses;
    then the mass-weighted and unweighted means of IN_out coincide."""
    rng = _rng(41)
    pat = rng.integers(0, 17, size=(7, 7)) / 16.0   # dyadic: every mass sum is exact
    res = 24
    U = []
    for k in range(8):
        img = np.zeros((res, res))
        ox, oy = rng.integers(0, res - 7, size=2)
        img[oy:oy + 7, ox:ox + 7] = pat
        U.append(img.ravel())
    U = np.array(U)
    a, b = oracle.pid(U), oracle.pid_mean(U)
    np.testing.assert_allclose(a["mass"], a["mass"][0], rtol=0, atol=0)
    np.testing.assert_allclose(a["depth"], b["depth"], atol=2e-16, rtol=0)


@pytest.mark.parametrize("seed", [51, 52, 53])
def test_cv_error_bound(seed):
    """|PID - PID-mean| <= (1/N) sum_j |m_j - mbar| / mbar <= CV of the masses.
    (The paper bounds the error by the CV of the masses, Sec. 4.1; this is the
    bound derived for these definitions.)"""
    U = synth.random_soft(10, 400, seed).numpy()
    U *= _rng(seed).uniform(0.2, 1.0, size=(10, 1))   # spread the masses
    a, b = oracle.pid(U), oracle.pid_mean(U)
    m = a["mass"]
    mbar = m.mean()
    bound = np.abs(m - mbar).mean() / mbar
    cv = m.std() / mbar
    assert np.max(np.abs(a["in_out"] - b["in_out"])) <= bound + 1e-15
    assert np.max(np.abs(a["depth"] - b["depth"])) <= bound + 1e-15
    assert bound <= cv + 1e-15


# ---------------------------------------------------------------- Sec. 3.5
def test_phi_extraction():
    f = np.linspace(-1, 2, 1001)
    iso = dict(kind="gaussian", c=0.5, sigma=0.05, side=1)
    p = oracle.extract(f, iso)
    np.testing.assert_allclose(p, 0.5 * erfc(-(f - 0.5) / (0.05 * math.sqrt(2))), rtol=1e-12, atol=1e-17)
    assert oracle.extract(np.array([0.5]), iso)[0] == 0.5
    # textbook value Phi(1) = 0.8413447460685429...
    assert abs(oracle.extract(np.array([0.55]), iso)[0] - 0.8413447460685429) < 1e-15
    # side = -1 is the sublevel set: p(f) = 1 - p_{+}(f)
    pm = oracle.extract(f, dict(iso, side=-1))
    np.testing.assert_allclose(pm, 1 - p, atol=1e-15)
    # sigma -> 0 gives the step (away from the isovalue)
    step = oracle.extract(f, dict(kind="step", c=0.5, side=1))
    sharp = oracle.extract(f, dict(iso, sigma=1e-9))
    far = np.abs(f - 0.5) > 1e-6
    np.testing.assert_array_equal(sharp[far], step[far])
    assert oracle.extract(np.array([0.5]), dict(kind="step", c=0.5, side=1))[0] == 0.0


# ---------------------------------------------------------------- Sec. 3.3 / 3.4
def test_operator_properties():
    rng = _rng(61)
    u, v1, v2 = rng.uniform(0, 1, size=(3, 200))
    w = rng.uniform(0.5, 1.5, size=200)
    a, b = 0.3, 0.6
    # linear in v
    assert abs(oracle.incl(u, a * v1 + b * v2, w) - (a * oracle.incl(u, v1, w) + b * oracle.incl(u, v2, w))) < 1e-15
    # monotone in v
    assert oracle.incl(u, np.maximum(v1, v2), w) >= oracle.incl(u, v1, w)
    # scale invariant in u
    assert abs(oracle.incl(2.5 * u, v1, w) - oracle.incl(u, v1, w)) < 1e-15
    # limiting cases
    assert abs(oracle.incl(u, np.ones_like(u), w) - 1.0) < 1e-15
    assert oracle.incl(u, np.zeros_like(u), w) == 0.0
    # directional
    assert oracle.incl(u, v1, w) != oracle.incl(v1, u, w)


def test_pid_invariants():
    rng = _rng(71)
    U = synth.random_soft(8, 250, 72).numpy()
    w = rng.uniform(0.5, 1.5, size=250)
    base = oracle.pid(U, w)
    basem = oracle.pid_mean(U, w)
    # member permutation: depths permute with the members
    perm = rng.permutation(8)
    r = oracle.pid(U[perm], w)
    np.testing.assert_allclose(r["depth"], base["depth"][perm], atol=1e-15)
    np.testing.assert_allclose(oracle.pid_mean(U[perm], w)["depth"], basem["depth"][perm], atol=1e-15)
    # grid-point permutation (a bijection of the domain, Sec. 3.3)
    gp = rng.permutation(250)
    np.testing.assert_allclose(oracle.pid(U[:, gp], w[gp])["depth"], base["depth"], atol=1e-15)
    # w -> alpha w
    np.testing.assert_allclose(oracle.pid(U, 3.0 * w)["depth"], base["depth"], atol=1e-15)
    np.testing.assert_allclose(oracle.pid_mean(U, 3.0 * w)["depth"], basem["depth"], atol=1e-15)
    # splitting a cell in two halves of the same value
    U2 = np.concatenate([U, U[:, :1]], axis=1)
    w2 = np.concatenate([w, w[:1] / 2])
    w2[0] = w[0] / 2
    np.testing.assert_allclose(oracle.pid(U2, w2)["depth"], base["depth"], atol=1e-15)
    # range
    for r in (base, basem):
        assert np.all(r["depth"] >= 0) and np.all(r["depth"] <= 1)
    assert np.all(base["inclusion"] >= 0) and np.all(base["inclusion"] <= 1 + 1e-15)


def test_degenerate_ensembles():
    rng = _rng(81)
    u = rng.uniform(0, 1, size=120)
    w = rng.uniform(0.5, 1.5, size=120)
    self_incl = float((w * u * u).sum() / (w * u).sum())
    r1 = oracle.pid(u[None, :], w)            # N = 1
    assert abs(r1["depth"][0] - self_incl) < 1e-15
    rid = oracle.pid(np.stack([u] * 5), w)    # identical members
    np.testing.assert_allclose(rid["depth"], self_incl, atol=1e-15)
    rm = oracle.pid_mean(np.stack([u] * 5), w)
    np.testing.assert_allclose(rm["depth"], self_incl, atol=1e-15)
    B = (u > 0.5).astype(np.uint8)
    rb = oracle.binary_pid(np.stack([B] * 4))  # identical binary members: depth 1
    assert rb["depth"].tolist() == [1.0] * 4


# ---------------------------------------------------------------- second evaluations
@pytest.mark.parametrize("seed", [91, 92])
def test_linear_form_matches_matrix_form(seed):
    U = synth.random_soft(12, 500, seed).numpy()
    U[3] = 0.0     # a zero-mass member
    w = _rng(seed).uniform(0.5, 1.5, size=500)
    a, b = oracle.pid(U, w), oracle.pid_linear(U, w)
    for key in ("in_in", "in_out", "depth"):
        np.testing.assert_allclose(a[key], b[key], atol=1e-15, rtol=0)


def test_chunked_large_forms_match():
    F = synth.bump_fields_3d(5, 12, 7)
    iso = dict(kind="gaussian", c=0.5, sigma=0.05, side=1)
    U = oracle.extract(F.numpy(), iso)
    w = synth.volume_weights(12 ** 3, 3).numpy()
    a, b = oracle.pid(U, w), oracle.pid_large(F.numpy(), w, iso, chunk=100)
    for key in ("mass", "in_in", "in_out", "depth"):
        np.testing.assert_allclose(a[key], b[key], atol=1e-14, rtol=1e-13)
    a, b = oracle.pid_mean(U, w), oracle.pid_mean_large(F.numpy(), w, iso, chunk=100)
    for key in ("mass", "in_in", "in_out", "depth"):
        np.testing.assert_allclose(a[key], b[key], atol=1e-14, rtol=1e-13)


def test_rank_order_brute_force():
    d = np.array([0.5, 0.7, 0.5, 0.9, 0.1, 0.7])
    rank, order = oracle.rank_order(d)
    assert order.tolist() == [3, 1, 5, 0, 2, 4]
    for i in range(d.size):
        assert rank[i] == sum(1 for j in range(d.size) if d[j] > d[i] or (d[j] == d[i] and j < i))


# ---------------------------------------------------------------- planted mistakes
def _pins_pass(pid_fn):
    """A compact set of pins evaluated on an arbitrary pid implementation."""
    g = golden.load("handworked_weighted_3x4.txt")
    U = np.array([[float(v) for v in g[k]] for k in ("u1", "u2", "u3")])
    w = np.array([float(v) for v in g["w"]])
    ok = True
    r = pid_fn(U, w)
    ok &= np.allclose(r["depth"], [float(v) for v in g["depth"]], atol=1e-15, rtol=0)
    ok &= np.allclose(r["in_out"], [float(v) for v in g["in_out"]], atol=1e-15, rtol=0)
    Ud = _dyadic(4, 13, 5)
    ex = oracle.exact_pid(Ud)
    ok &= np.allclose(pid_fn(Ud, None)["in_in"], [float(v) for v in ex["in_in"]], atol=1e-15, rtol=0)
    return bool(ok)


def test_planted_mistakes_are_caught():
    """Plausible oracle mistakes -- a transposed matrix, dropped weights in the
    numerator, division by N-1, max instead of min -- each fail a pin."""
    assert _pins_pass(oracle.pid)

    def transposed(U, w):
        r = oracle.pid(U, w)
        P = r["inclusion"].T
        n = P.shape[0]
        return dict(in_in=P.sum(1) / n, in_out=P.sum(0) / n, depth=np.minimum(P.sum(1), P.sum(0)) / n)

    def no_w_numerator(U, w):
        G = oracle.gram(U, None)
        m = oracle.mass(U, w)
        P = G / m[:, None]
        n = P.shape[0]
        return dict(in_in=P.sum(1) / n, in_out=P.sum(0) / n, depth=np.minimum(P.sum(1), P.sum(0)) / n)

    def n_minus_one(U, w):
        r = oracle.pid(U, w)
        n = r["inclusion"].shape[0]
        return {k: (v * n / (n - 1) if k != "inclusion" else v) for k, v in r.items()}

    def use_max(U, w):
        r = oracle.pid(U, w)
        r = dict(r)
        r["depth"] = np.maximum(r["in_in"], r["in_out"])
        return r

    for bad in (transposed, no_w_numerator, n_minus_one, use_max):
        assert not _pins_pass(bad), bad.__name__


# ---------------------------------------------------------------- generators
def test_generators_deterministic():
    a, ia = synth.config0(res=32, n=10)
    b, ib = synth.config0(res=32, n=10)
    assert ia == ib and ia and bool((a == b).all())
    assert a.dtype.is_floating_point and float(a.min()) >= 0 and float(a.max()) <= 1
    c, _ = synth.config1(res=32, n=20)
    assert c.shape == (20, 1024)
    U, w = synth.config3(res=8, n=4)
    assert U.shape == (4, 512) and w.shape == (512,) and float(w.min()) >= 0.5
    reqs = synth.serving_requests(50)
    assert all(r.arrival_s > 0 for r in reqs) and reqs == synth.serving_requests(50)


def test_binary_float_product_is_the_integer_product():
    B = synth.random_binary(9, 3000, 17).numpy()
    a, b = oracle.binary_pid(B), oracle.binary_pid(B, float_product=True)
    assert (a["gram"] == b["gram"]).all()
    for key in ("in_in", "in_out", "depth", "inclusion"):
        assert (a[key] == b[key]).all()


# ------------------------------------------------ contour-boxplot bands
def test_boxplot_bands_handworked():
    """Three members, six points, ranked deepest first as 2, 0, 1; inside
    where u >= 0.5 (0.5 itself is inside).  Binarised rows:
    b0 = 110010, b1 = 010011, b2 = 110001.  Median = b2; the two deepest
    (2, 0): union 110011, intersection 110000; all three: union 110011,
    intersection 010000."""
    U = np.array([[0.9, 0.5, 0.1, 0.0, 0.6, 0.49],
                  [0.2, 0.7, 0.3, 0.0, 0.8, 1.0],
                  [1.0, 0.5, 0.0, 0.0, 0.4, 0.51]])
    r = oracle.boxplot_bands(U, [2, 0, 1], 2, 3, 0.5)
    assert r["median"].tolist() == [1, 1, 0, 0, 0, 1]
    assert r["union_inner"].tolist() == [1, 1, 0, 0, 1, 1]
    assert r["inter_inner"].tolist() == [1, 1, 0, 0, 0, 0]
    assert r["union_outer"].tolist() == [1, 1, 0, 0, 1, 1]
    assert r["inter_outer"].tolist() == [0, 1, 0, 0, 0, 0]
    # bits: median 1, inner union 2, inner intersection 4, outer union 8, outer intersection 16
    assert r["code"].tolist() == [15, 31, 0, 0, 10, 11]


def test_boxplot_bands_nesting_and_special_cases():
    rng = _rng(77)
    n, m = 9, 400
    U = rng.random((n, m))
    order = rng.permutation(n)
    r = oracle.boxplot_bands(U, order, 4, 7, 0.5)
    # intersections shrink and unions grow with the group; the median lies between
    assert np.all(r["inter_outer"] <= r["inter_inner"])
    assert np.all(r["inter_inner"] <= r["median"])
    assert np.all(r["median"] <= r["union_inner"])
    assert np.all(r["union_inner"] <= r["union_outer"])
    # a group of one is the median itself
    r1 = oracle.boxplot_bands(U, order, 1, 1, 0.5)
    for k in ("union_inner", "inter_inner", "union_outer", "inter_outer"):
        assert np.array_equal(r1[k], r1["median"])
    assert np.array_equal(r1["median"], U[order[0]] >= 0.5)
    # the whole ensemble does not depend on the order
    rn = oracle.boxplot_bands(U, rng.permutation(n), n, n, 0.5)
    assert np.array_equal(rn["union_outer"], (U >= 0.5).any(axis=0))
    assert np.array_equal(rn["inter_outer"], (U >= 0.5).all(axis=0))


def test_boxplot_bands_de_morgan():
    """On binary masks the union of the complements is the complement of the
    intersection (and vice versa)."""
    B = synth.random_binary(7, 300, 5).numpy().astype(np.float64)
    order = [3, 1, 6, 0, 2, 5, 4]
    a = oracle.boxplot_bands(B, order, 3, 7, 0.5)
    c = oracle.boxplot_bands(1.0 - B, order, 3, 7, 0.5)
    assert np.array_equal(c["union_inner"], ~a["inter_inner"])
    assert np.array_equal(c["inter_outer"], ~a["union_outer"])
    assert np.array_equal(c["median"], ~a["median"])


# ------------------------------------------ Sec. 3.5, 3.6, 6.3: further models
def test_golden_probability_models():
    g = golden.load("weighted_mean_and_models.txt")
    f = np.array([float(v) for v in g["f"]])
    cases = {"ramp_up": dict(kind="ramp", c=0.5, width=0.125, side=1),
             "ramp_down": dict(kind="ramp", c=0.5, width=0.125, side=-1),
             "tent": dict(kind="tent", c=0.5, width=0.125),
             "density": dict(kind="density", c=0.5)}
    for key, iso in cases.items():
        assert oracle.extract(f, iso).tolist() == [float(v) for v in g[key]], key


def test_models_reduce_to_library_distributions():
    """The ramp is the CDF of the uniform isovalue distribution, the tent the
    width-scaled density of the symmetric triangular distribution."""
    from scipy import stats
    rng = _rng(77)
    for c, h in ((0.5, 0.05), (-2.0, 1.5), (10.0, 1e-3)):
        f = c + h * rng.uniform(-3, 3, size=2000)
        up = oracle.extract(f, dict(kind="ramp", c=c, width=h, side=1))
        np.testing.assert_allclose(up, stats.uniform(loc=c - h, scale=2 * h).cdf(f), atol=1e-12, rtol=0)
        down = oracle.extract(f, dict(kind="ramp", c=c, width=h, side=-1))
        np.testing.assert_allclose(down, stats.uniform(loc=c - h, scale=2 * h).sf(f), atol=1e-12, rtol=0)
        tent = oracle.extract(f, dict(kind="tent", c=c, width=h))
        np.testing.assert_allclose(tent, h * stats.triang(0.5, loc=c - h, scale=2 * h).pdf(f), atol=1e-9, rtol=0)
        # the tent is twice the distance of the ramp to the nearer of 0 and 1
        np.testing.assert_allclose(tent, 2 * np.minimum(up, 1 - up), atol=1e-12, rtol=0)
        dens = oracle.extract(f, dict(kind="density", c=abs(c) + h))
        assert dens.min() >= 0.0 and dens.max() <= 1.0
        inside = (f > 0) & (f < abs(c) + h)
        np.testing.assert_allclose(dens[inside] * (abs(c) + h), f[inside], rtol=1e-15)
    # a vanishing width gives the sharp isovalue away from the level itself
    f = rng.uniform(0, 1, size=5000)
    f = f[np.abs(f - 0.5) > 1e-6]
    for side in (1, -1):
        ramp = oracle.extract(f, dict(kind="ramp", c=0.5, width=1e-9, side=side))
        assert (ramp == oracle.extract(f, dict(kind="step", c=0.5, side=side))).all()


# ------------------------------------------ Sec. 4.1: reliability-weighted mean
def test_golden_weighted_mean():
    g = golden.load("weighted_mean_and_models.txt")
    U = np.array([[float(v) for v in g[k]] for k in ("wu1", "wu2", "wu3")])
    r = np.array([float(v) for v in g["wr"]])
    res = oracle.pid_mean_weighted(U, r)
    assert abs(res["mbar"] - float(g["w_mbar"][0])) < 1e-15
    for key in ("in_in", "in_out", "depth"):
        np.testing.assert_allclose(res[key], [float(v) for v in g["w_" + key]], rtol=0, atol=1e-15)
    assert oracle.rank_order(res["depth"])[0].tolist() == [int(v) for v in g["w_rank"]]


@pytest.mark.parametrize("seed,weighted", [(1, False), (2, True), (3, True)])
def test_weighted_mean_pins(seed, weighted):
    rng = _rng(seed)
    n, m = 7, 40
    U = _dyadic(n, m, seed + 50, zero_rows=(4,))
    w = rng.integers(1, 4, size=m).astype(np.float64) if weighted else None
    # unit weights: the plain PID-mean
    a, b = oracle.pid_mean_weighted(U, np.ones(n), w), oracle.pid_mean(U, w)
    for key in ("in_in", "in_out", "depth"):
        np.testing.assert_allclose(a[key], b[key], rtol=0, atol=1e-15)
    # integer weights: the plain PID-mean of the ensemble with member j
    # repeated r_j times (members of weight 0 compared against that mean too)
    r = rng.integers(0, 4, size=n)
    r[0] = 2
    rep = np.repeat(U, r, axis=0)
    plain = oracle.pid_mean(rep, w)
    wm = oracle.pid_mean_weighted(U, r.astype(np.float64), w)
    first = np.concatenate([[0], np.cumsum(r)[:-1]])
    for j in range(n):
        if r[j] > 0:
            for key in ("in_in", "in_out"):
                assert abs(wm[key][j] - plain[key][first[j]]) < 1e-14, (key, j)
    # one-hot weights: the mean contour is that member
    for k in (0, 3):
        e = np.zeros(n)
        e[k] = 5.0
        res = oracle.pid_mean_weighted(U, e, w)
        for i in range(n):
            assert abs(res["in_in"][i] - oracle.incl(U[i], U[k], w)) < 1e-15
            assert abs(res["in_out"][i] - oracle.incl(U[k], U[i], w)) < 1e-15
    # scale invariance in r; weighted recall identity through the Gram numerators
    rr = rng.uniform(0.1, 2.0, size=n)
    x, y = oracle.pid_mean_weighted(U, rr, w), oracle.pid_mean_weighted(U, 3.7 * rr, w)
    np.testing.assert_allclose(x["depth"], y["depth"], rtol=0, atol=1e-15)
    G, mm = oracle.gram(U, w), oracle.mass(U, w)
    for i in range(n):
        exp = (G[i] @ rr) / (rr.sum() * mm[i]) if mm[i] > 0 else 0.0
        assert abs(x["in_in"][i] - exp) < 1e-14
    # a planted mistake (ubar normalised by N instead of sum r) fails the pin
    bad_ubar = (rr[:, None] * U).sum(axis=0) / n
    assert abs(oracle.incl(U[0], bad_ubar, w) - x["in_in"][0]) > 1e-3
