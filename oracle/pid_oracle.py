"""FP64 CPU oracle for Probabilistic Inclusion Depth (PID) and PID-mean.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
statement of what the GPU path computes.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product path never
does, and it shares no code, table or helper with the HIP kernels.

Everything is evaluated in float64 on exactly the stored input values (F16,
BF16 and F32 inputs widen to F64 exactly).  Binary masks are handled with exact
integers.  Each function names the passage of the paper it follows:

* mass ``m(u) = sum_x w_x u(x)``                           -- Sec. 3.2 (mass), Sec. 3.4 (non-uniform grids)
* inclusion ``u <_p v = sum w u v / sum w u``, 0 if m(u)=0 -- Sec. 3.2, Eqs. expectation_form / prob_contain
* PID: IN_in, IN_out = means over j of the inclusions; min  -- Sec. 3.2, Eq. pid
* PID-mean against the mean contour ``ubar``               -- Sec. 4.1
* fuzzy extraction ``p = P(inside | isovalue ~ N(c, s^2))`` -- Sec. 3.5 (isovalue distribution)
* further probability models: a uniform isovalue distribution (Sec. 3.5),
  the level-centred map with linear fall-off (Sec. 3.6, weather example) and
  the normalised density (Sec. 6.3)
* PID-mean against a reliability-weighted mean contour   -- Sec. 4.1 (properties of PID-mean)
* binary reduction to the eID subset operator              -- Sec. 3.1 Eq. 1 and Sec. 3.2 Eq. binary_reduction
* ranking: deepest first                                   -- Sec. 5.1
* contour-boxplot bands: median, unions and intersections
  of the binarised deepest members                         -- Sec. 1 (pipeline), Sec. 6 and 6.1

Readings taken where the paper is silent or inconsistent (all listed in the
design notes of the repository):

* zero mass: ``u <_p v = 0`` when ``m(u) = 0`` (the PID convention of Sec. 3.2,
  not the eID convention of Eq. 1); PID-mean uses 0 when ``m(ubar) = 0``;
* the self term ``j = i`` is included and the means divide by N;
* inside side: ``side = +1`` means ``f > c`` is inside (``p = Phi((f-c)/s)``),
  ``side = -1`` is the sublevel set ``f < c`` of Sec. 3.1 Eq. 2;
* binary threshold is strict: ``side*(f - c) > 0`` is inside;
* ranks: rank 0 is the deepest member, ties broken by the lower index;
* boxplot binarisation: a point is inside a member when ``u >= threshold``;
* uniform isovalue distribution: the isovalue is uniform on ``[c - h, c + h]``
  (``h`` = ``width``), so ``p = P(q < f)`` rises linearly from 0 to 1 there;
* level-centred map: ``p = max(0, 1 - |f - c| / h)``, 1 at the target level and
  0 from a distance ``h`` (``width``) on (the paper gives no fall-off width);
* normalised density: ``p = clip(f / c, 0, 1)`` with ``c`` the normalising
  density, e.g. the ensemble's largest density (the paper does not say which);
* reliability weights ``r_j >= 0`` (sum > 0): ``ubar = sum_j r_j u_j / sum_j r_j``.

Pinned by ``tests/test_oracle_pins.py`` against exact-rational brute force,
eID set counting, closed forms for nested chains, a hand-worked fixture, the
PID-mean identity of Sec. 4.1 and the invariants of Sec. 3.3.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
from scipy.special import ndtr

__all__ = [
    "extract", "mass", "incl", "gram", "inclusion_matrix", "pid", "pid_mean",
    "pid_mean_literal", "pid_linear", "rank_order", "eid_sets",
    "binary_pid", "binary_pid_mean", "pid_large", "pid_mean_large",
    "exact_pid", "exact_pid_mean", "boxplot_bands", "pid_mean_weighted",
]


def _f64(a):
    return np.asarray(a).astype(np.float64, copy=False)


# ---------------------------------------------------------------- Sec. 3.5
def extract(data, iso=None):
    """Membership probabilities from stored values.

    ``iso`` is None / ``{"kind": "none"}`` (the values already are soft masks,
    Sec. 3.5 explicit soft masks), ``{"kind": "gaussian", "c", "sigma", "side"}``
    (isovalue ~ N(c, sigma^2): inside probability
    ``Phi(side*(f - c)/sigma)``), ``{"kind": "step", "c", "side"}`` (a sharp
    isovalue: inside iff ``side*(f - c) > 0``, compared exactly in float64),
    ``{"kind": "ramp", "c", "width", "side"}`` (isovalue uniform on
    ``[c - width, c + width]``: inside probability ``P(q < f)`` for side +1,
    ``P(q > f)`` for side -1), ``{"kind": "tent", "c", "width"}`` (the
    level-centred map of Sec. 3.6: 1 at ``f = c``, falling linearly to 0 at
    ``|f - c| = width``) or ``{"kind": "density", "c"}`` (the normalised
    density of Sec. 6.3: ``f / c`` clipped to [0, 1])."""
    f = _f64(data)
    if iso is None or iso.get("kind", "none") == "none":
        return f
    side = float(iso.get("side", 1))
    c = float(iso["c"])
    kind = iso["kind"]
    if kind == "gaussian":
        return ndtr(side * (f - c) / float(iso["sigma"]))
    if kind == "step":
        return (side * (f - c) > 0).astype(np.float64)
    if kind == "ramp":
        h = float(iso["width"])
        lo = c - h                          # support of the isovalue: [c - h, c + h]
        below = np.clip((f - lo) / (2.0 * h), 0.0, 1.0)   # P(q < f)
        return below if side > 0 else 1.0 - below
    if kind == "tent":
        h = float(iso["width"])
        return np.maximum(0.0, 1.0 - np.abs(f - c) / h)
    if kind == "density":
        return np.clip(f / c, 0.0, 1.0)
    raise ValueError(iso)


# ---------------------------------------------------------------- Sec. 3.2 / 3.4
def mass(U, w=None):
    """``m(u_i) = sum_x w_x u_i(x)`` for every row of U (w = 1 on a uniform grid)."""
    U = _f64(U)
    if w is None:
        return U.sum(axis=-1)
    return (U * _f64(w)).sum(axis=-1)


def incl(u, v, w=None):
    """``u <_p v``: the expectation of v under the measure induced by u,
    ``sum w u v / sum w u``; 0 when the mass of u is 0."""
    u, v = _f64(u), _f64(v)
    ww = np.ones_like(u) if w is None else _f64(w)
    m = float((ww * u).sum())
    if m == 0.0:
        return 0.0
    return float((ww * u * v).sum()) / m


def gram(U, w=None):
    """``G_ij = sum_x w_x u_i(x) u_j(x)`` (the numerators of every inclusion)."""
    U = _f64(U)
    Uw = U if w is None else U * _f64(w)
    return Uw @ U.T


def inclusion_matrix(U, w=None):
    """``P_ij = u_i <_p u_j = G_ij / m_i`` with the zero-mass convention."""
    G = gram(U, w)
    m = mass(U, w)
    P = np.zeros_like(G)
    nz = m > 0
    P[nz] = G[nz] / m[nz, None]
    return P, m


def _depths(P):
    n = P.shape[0]
    in_in = P.sum(axis=1) / n      # (1/N) sum_j u_i <_p u_j
    in_out = P.sum(axis=0) / n     # (1/N) sum_j u_j <_p u_i
    return in_in, in_out, np.minimum(in_in, in_out)


def pid(U, w=None):
    """All-pairs PID (Sec. 3.2 Eq. pid, weighted sums of Sec. 3.4)."""
    P, m = inclusion_matrix(U, w)
    in_in, in_out, depth = _depths(P)
    return dict(inclusion=P, mass=m, in_in=in_in, in_out=in_out, depth=depth)


# ---------------------------------------------------------------- Sec. 4.1
def pid_mean(U, w=None):
    """PID-mean: each member against the mean contour ``ubar = mean_i u_i``:
    ``IN_in = u_i <_p ubar``, ``IN_out = ubar <_p u_i``, depth = min."""
    U = _f64(U)
    ubar = U.mean(axis=0)
    m = mass(U, w)
    mbar = float(mass(ubar, w))
    Uw = U if w is None else U * _f64(w)
    A = Uw @ ubar                        # sum_x w u_i ubar
    in_in = np.where(m > 0, A / np.where(m > 0, m, 1.0), 0.0)
    in_out = A / mbar if mbar > 0 else np.zeros_like(A)
    return dict(mass=m, mbar=mbar, in_in=in_in, in_out=in_out,
                depth=np.minimum(in_in, in_out))


def pid_mean_literal(U, w=None):
    """PID-mean evaluated as 2N explicit calls of the inclusion operator on a
    materialised ``ubar`` (a second evaluation of ``pid_mean``)."""
    U = _f64(U)
    ubar = U.mean(axis=0)
    in_in = np.array([incl(u, ubar, w) for u in U])
    in_out = np.array([incl(ubar, u, w) for u in U])
    return dict(in_in=in_in, in_out=in_out, depth=np.minimum(in_in, in_out))


def pid_mean_weighted(U, r, w=None):
    """PID-mean against a reliability-weighted mean contour (Sec. 4.1, the
    optional weighting of the point-wise mean): ``ubar = sum_j r_j u_j /
    sum_j r_j`` with member weights ``r_j >= 0`` (not all 0); then
    ``IN_in = u_i <_p ubar``, ``IN_out = ubar <_p u_i``, depth = min, each
    evaluated by the inclusion operator on the materialised ``ubar``."""
    U = _f64(U)
    r = _f64(r)
    ubar = (r[:, None] * U).sum(axis=0) / r.sum()
    in_in = np.array([incl(u, ubar, w) for u in U])
    in_out = np.array([incl(ubar, u, w) for u in U])
    return dict(mass=mass(U, w), mbar=float(mass(ubar, w)), in_in=in_in, in_out=in_out,
                depth=np.minimum(in_in, in_out))


def pid_linear(U, w=None):
    """All-pairs PID depths without the N x N matrix.  Because ``u <_p v`` is
    linear in v (Sec. 3.3): ``IN_in(i) = <u_i, ubar>_w / m_i`` and
    ``IN_out(i) = <u_i, utilde>_w`` with ``utilde = (1/N) sum_j u_j / m_j``
    over members with ``m_j > 0``."""
    U = _f64(U)
    n = U.shape[0]
    m = mass(U, w)
    Uw = U if w is None else U * _f64(w)
    ubar = U.mean(axis=0)
    inv = np.where(m > 0, 1.0 / np.where(m > 0, m, 1.0), 0.0)
    utilde = (U * inv[:, None]).sum(axis=0) / n
    in_in = np.where(m > 0, (Uw @ ubar) * inv, 0.0)
    in_out = Uw @ utilde
    return dict(mass=m, in_in=in_in, in_out=in_out, depth=np.minimum(in_in, in_out))


# ---------------------------------------------------------------- Sec. 5.1
def rank_order(depth):
    """``order[k]`` = the member at position k when sorted deepest first (ties
    by lower index); ``rank[i]`` = position of member i (0 = deepest)."""
    depth = np.asarray(depth, dtype=np.float64)
    order = np.lexsort((np.arange(depth.size), -depth)).astype(np.int32)
    rank = np.empty_like(order)
    rank[order] = np.arange(depth.size, dtype=np.int32)
    return rank, order


# ---------------------------------------------------------------- Sec. 3.1 Eq. 1
def eid_sets(masks):
    """Epsilon Inclusion Depth by set counting on binary masks: ``A <_eps B =
    1 - |A \\ B| / |A|`` (1 when A is empty, Eq. 1), the means over j of Eq. 3
    and the min of Eq. 4.  Exact rationals."""
    sets = [set(np.flatnonzero(np.asarray(b)).tolist()) for b in masks]
    n = len(sets)

    def sub(a, b):
        if len(a) == 0:
            return Fraction(1)
        return 1 - Fraction(len(a - b), len(a))

    in_in = [sum(sub(sets[i], sets[j]) for j in range(n)) / n for i in range(n)]
    in_out = [sum(sub(sets[j], sets[i]) for j in range(n)) / n for i in range(n)]
    return in_in, in_out, [min(a, b) for a, b in zip(in_in, in_out)]


# ---------------------------------------------------------------- binary, exact
def binary_pid(B, float_product=False):
    """PID of binary masks with integer sums and one fixed FP64 finishing order.

    ``float_product=True`` forms the integer products ``G = B B^T`` with a
    float64 matrix product, which is exact while every count is below 2^53
    (0/1 entries, so every partial sum is an integer of at most M); it is the
    same integer matrix, computed faster for large M.

    ``G`` and ``m`` are exact int64.  ``P_ij = fl(G_ij / m_i)``;
    ``IN_in(i) = fl(S_i / (N m_i))`` with ``S_i = sum_j G_ij`` (one rounding of
    the exact mean of row i); ``IN_out(i) = fl(sum_j fl(G_ij / m_j)) / N`` with
    the sum taken in ascending j, one rounding per addition.  Zero-mass rows are
    0 (Sec. 3.2 convention)."""
    if float_product:
        Bf = np.asarray(B).astype(np.float64)
        assert Bf.shape[1] < 2 ** 53
        G = (Bf @ Bf.T).astype(np.int64)
        m = Bf.sum(axis=1).astype(np.int64)
    else:
        Bi = np.asarray(B).astype(np.int64)
        G = Bi @ Bi.T
        m = Bi.sum(axis=1)
    n = G.shape[0]
    S = G.sum(axis=1)
    P = np.zeros((n, n), dtype=np.float64)
    in_in = np.zeros(n)
    in_out = np.zeros(n)
    for i in range(n):
        if m[i] > 0:
            for j in range(n):
                P[i, j] = float(G[i, j]) / float(m[i])
            in_in[i] = float(S[i]) / (float(n) * float(m[i]))
        acc = 0.0
        for j in range(n):
            if m[j] > 0:
                acc = acc + float(G[j, i]) / float(m[j])
        in_out[i] = acc / float(n)
    return dict(gram=G, mass_int=m, rowsum=S, inclusion=P, mass=m.astype(np.float64),
                in_in=in_in, in_out=in_out, depth=np.minimum(in_in, in_out))


def binary_pid_mean(B):
    """PID-mean of binary masks, exact up to one rounding per result:
    ``IN_in = S_i / (N m_i)`` and ``IN_out = S_i / sum_k m_k`` where
    ``S_i = sum_x u_i(x) s(x)`` and ``s(x) = sum_j u_j(x)`` (so that
    ``A_i = S_i / N`` and ``m(ubar) = sum_k m_k / N``)."""
    Bi = np.asarray(B).astype(np.int64)
    n = Bi.shape[0]
    s = Bi.sum(axis=0)
    S = Bi @ s
    m = Bi.sum(axis=1)
    tot = int(m.sum())
    in_in = np.array([float(S[i]) / (float(n) * float(m[i])) if m[i] > 0 else 0.0 for i in range(n)])
    in_out = np.array([float(S[i]) / float(tot) if tot > 0 else 0.0 for i in range(n)])
    return dict(rowsum=S, mass_int=m, mass=m.astype(np.float64), in_in=in_in,
                in_out=in_out, depth=np.minimum(in_in, in_out))


# ---------------------------------------------------------------- exact rationals
def exact_pid(U, w=None):
    """All-pairs PID in exact rational arithmetic, by loops over (i, j, x),
    using the complement form ``1 - sum w u (1 - v) / sum w u`` of Sec. 3.4.
    For tiny inputs only."""
    Uq = [[Fraction(float(v)) for v in row] for row in np.asarray(U, dtype=np.float64)]
    M = len(Uq[0])
    wq = [Fraction(1)] * M if w is None else [Fraction(float(v)) for v in np.asarray(w, dtype=np.float64)]
    n = len(Uq)

    def inc(u, v):
        den = sum(wq[x] * u[x] for x in range(M))
        if den == 0:
            return Fraction(0)
        return 1 - sum(wq[x] * u[x] * (1 - v[x]) for x in range(M)) / den

    P = [[inc(Uq[i], Uq[j]) for j in range(n)] for i in range(n)]
    in_in = [sum(P[i]) / n for i in range(n)]
    in_out = [sum(P[j][i] for j in range(n)) / n for i in range(n)]
    return dict(inclusion=P, in_in=in_in, in_out=in_out,
                depth=[min(a, b) for a, b in zip(in_in, in_out)])


def exact_pid_mean(U, w=None):
    """PID-mean in exact rationals (tiny inputs only)."""
    Uq = [[Fraction(float(v)) for v in row] for row in np.asarray(U, dtype=np.float64)]
    n, M = len(Uq), len(Uq[0])
    wq = [Fraction(1)] * M if w is None else [Fraction(float(v)) for v in np.asarray(w, dtype=np.float64)]
    ubar = [sum(Uq[i][x] for i in range(n)) / n for x in range(M)]

    def inc(u, v):
        den = sum(wq[x] * u[x] for x in range(M))
        return Fraction(0) if den == 0 else sum(wq[x] * u[x] * v[x] for x in range(M)) / den

    in_in = [inc(Uq[i], ubar) for i in range(n)]
    in_out = [inc(ubar, Uq[i]) for i in range(n)]
    return dict(in_in=in_in, in_out=in_out, depth=[min(a, b) for a, b in zip(in_in, in_out)])


# ---------------------------------------------------------------- large inputs
def _chunks(M, chunk):
    for s in range(0, M, chunk):
        yield slice(s, min(M, s + chunk))


def pid_large(data, w=None, iso=None, chunk=1 << 18):
    """``pid`` for ensembles too large to widen to float64 at once: the same
    sums over x (Gram numerators and masses), accumulated over point chunks in
    float64, then the same ratios and means."""
    data = np.asarray(data)
    n, M = data.shape
    G = np.zeros((n, n))
    m = np.zeros(n)
    for sl in _chunks(M, chunk):
        U = extract(data[:, sl], iso)
        Uw = U if w is None else U * _f64(np.asarray(w)[sl])
        G += Uw @ U.T
        m += Uw.sum(axis=1)
    P = np.zeros_like(G)
    nz = m > 0
    P[nz] = G[nz] / m[nz, None]
    in_in, in_out, depth = _depths(P)
    return dict(inclusion=P, mass=m, in_in=in_in, in_out=in_out, depth=depth)


def pid_mean_large(data, w=None, iso=None, chunk=1 << 18):
    """``pid_mean`` over point chunks (the sums over x accumulated in float64)."""
    data = np.asarray(data)
    n, M = data.shape
    A = np.zeros(n)
    m = np.zeros(n)
    mbar = 0.0
    for sl in _chunks(M, chunk):
        U = extract(data[:, sl], iso)
        ubar = U.mean(axis=0)
        ww = None if w is None else _f64(np.asarray(w)[sl])
        Uw = U if ww is None else U * ww
        A += Uw @ ubar
        m += Uw.sum(axis=1)
        mbar += float(ubar.sum() if ww is None else (ubar * ww).sum())
    in_in = np.where(m > 0, A / np.where(m > 0, m, 1.0), 0.0)
    in_out = A / mbar if mbar > 0 else np.zeros_like(A)
    return dict(mass=m, mbar=mbar, in_in=in_in, in_out=in_out,
                depth=np.minimum(in_in, in_out))


# ------------------------------------------------------- Sec. 1, Sec. 6 / 6.1
BAND_MEDIAN, BAND_UNION_INNER, BAND_INTER_INNER, BAND_UNION_OUTER, BAND_INTER_OUTER = 1, 2, 4, 8, 16


def boxplot_bands(U, order, k_inner, k_outer, threshold):
    """Contour-boxplot bands of an ensemble ranked by depth.

    The members are binarised (inside where ``u >= threshold``: 0.5 for soft
    masks, 0.02 for normalised densities in the examples of Sec. 6); the
    median is the deepest member ``order[0]``; a band of the ``k`` deepest
    members ``order[:k]`` is bounded by the per-point union and intersection
    of their binarised masks (Sec. 1 and Sec. 6: envelopes of the 50 % and
    100 % groups).  ``k_inner`` and ``k_outer`` are the group sizes.  Returns
    boolean arrays of length M and ``code``, one byte per point with the
    bits BAND_MEDIAN, BAND_UNION_INNER, BAND_INTER_INNER, BAND_UNION_OUTER,
    BAND_INTER_OUTER."""
    U = _f64(U)
    order = [int(i) for i in order]
    B = U >= float(threshold)
    def union(k):
        return np.any(B[order[:k]], axis=0)
    def inter(k):
        return np.all(B[order[:k]], axis=0)
    out = dict(median=B[order[0]].copy(), union_inner=union(k_inner), inter_inner=inter(k_inner),
               union_outer=union(k_outer), inter_outer=inter(k_outer))
    code = (out["median"] * BAND_MEDIAN + out["union_inner"] * BAND_UNION_INNER
            + out["inter_inner"] * BAND_INTER_INNER + out["union_outer"] * BAND_UNION_OUTER
            + out["inter_outer"] * BAND_INTER_OUTER)
    out["code"] = code.astype(np.uint8)
    return out
