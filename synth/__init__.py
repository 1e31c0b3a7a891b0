"""Seeded synthetic ensembles for PID (Probabilistic Inclusion Depth).

This module only *makes inputs*: scalar fields and soft masks on uniform grids,
the per-point volume weights that stand in for a non-uniform grid, and the
request mix of the serving workload.  It holds none of the depth arithmetic and
is shared by the CPU oracle (``oracle/``) and the GPU path alike.

Conventions (the same for every generator):

* Random parameters are drawn with ``numpy.random.Generator(PCG64(seed))``; the
  per-point noise of the scalar-field ensemble is drawn with a torch generator
  seeded from the same seed, on the device the fields are built on.
* Grid points sit at cell centres ``(i + 1/2) / res`` of the unit square/cube and
  are flattened with x fastest (``index = (z*res + y)*res + x``).
* Every ensemble is returned member-major, ``N x M``, in the stored dtype.  Both
  sides of a parity test consume exactly those stored bits.

The shapes follow the workloads of the paper: 2D closed curves with Fourier
perturbations turned into soft masks (the synthetic contour ensembles of the
ranking-consistency study, Sec. 5.1), scalar-field ensembles whose fuzzy
contours come from an isovalue distribution (Sec. 3.5), large 3D
perturbed-sphere ensembles, and binary 3D ellipsoid ensembles with 20 %
outliers (the scalability study, Sec. 5.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

BASE_SEED = 20251215


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def grid_coords(res: int, dim: int, device="cpu", dtype=torch.float64):
    """Cell-centre coordinates of a ``res**dim`` grid, x fastest.  Returns a
    tuple of flat tensors (x, y[, z])."""
    t = (torch.arange(res, device=device, dtype=dtype) + 0.5) / res
    if dim == 2:
        yy, xx = torch.meshgrid(t, t, indexing="ij")
        return xx.reshape(-1), yy.reshape(-1)
    zz, yy, xx = torch.meshgrid(t, t, t, indexing="ij")
    return xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)


# --------------------------------------------------------------------------
# 2D: soft masks from perturbed closed curves
# --------------------------------------------------------------------------
@dataclass
class Curve2D:
    amp: np.ndarray      # a_m, m = 1..modes
    phase: np.ndarray    # phi_m
    k: float             # sigmoid steepness
    cx: float = 0.5
    cy: float = 0.5


def curve_params_2d(n, modes, n_out, outlier, seed, r0=0.3, amp_sd=0.05,
                    k_lo=20.0, k_hi=80.0, shift=0.15, rot_lo=30.0, rot_hi=90.0):
    """Draw the curve parameters of an N-member 2D ensemble.

    Draw order: a permutation that picks the outlier members, then for every
    member (in index order) the amplitudes, the phases, k and one outlier
    parameter (drawn for every member so the streams stay aligned; used only by
    outliers).  ``outlier`` is ``"shift"`` (centre moved by ``shift`` along a
    random direction) or ``"rotate"`` (shape rotated about the centre by an
    angle in [rot_lo, rot_hi] degrees, i.e. phi_m -> phi_m - m*alpha)."""
    rng = _rng(seed)
    out_idx = set(rng.permutation(n)[:n_out].tolist())
    curves = []
    m = np.arange(1, modes + 1)
    for i in range(n):
        amp = rng.normal(0.0, amp_sd, size=modes)
        phase = rng.uniform(0.0, 2 * np.pi, size=modes)
        k = rng.uniform(k_lo, k_hi)
        extra = rng.uniform(0.0, 1.0)
        c = Curve2D(amp, phase, float(k))
        if i in out_idx:
            if outlier == "shift":
                beta = 2 * np.pi * extra
                c.cx += shift * math.cos(beta)
                c.cy += shift * math.sin(beta)
            elif outlier == "rotate":
                alpha = np.deg2rad(rot_lo + (rot_hi - rot_lo) * extra)
                c.phase = np.mod(phase - m * alpha, 2 * np.pi)
            else:
                raise ValueError(outlier)
        curves.append(c)
    return curves, sorted(out_idx), r0


def soft_masks_2d(curves, r0, res, device="cpu", dtype=torch.float32):
    """``u = sigmoid(k * d)`` with ``d`` the first-order signed distance to the
    polar curve ``r(theta) = r0 (1 + sum a_m cos(m theta + phi_m))``:
    ``d = (r(theta) - rho) / sqrt(1 + (r'(theta)/r(theta))**2)``, positive
    inside.  Evaluated in float64, stored as ``dtype``."""
    x, y = grid_coords(res, 2, device)
    out = torch.empty((len(curves), res * res), dtype=dtype, device=device)
    for i, c in enumerate(curves):
        dx, dy = x - c.cx, y - c.cy
        rho = torch.sqrt(dx * dx + dy * dy)
        th = torch.atan2(dy, dx)
        r = torch.ones_like(th)
        dr = torch.zeros_like(th)
        for mm, (a, ph) in enumerate(zip(c.amp, c.phase), start=1):
            arg = mm * th + float(ph)
            r = r + float(a) * torch.cos(arg)
            dr = dr - float(a) * mm * torch.sin(arg)
        r = r0 * r
        dr = r0 * dr
        d = (r - rho) / torch.sqrt(1.0 + (dr / r) ** 2)
        out[i] = torch.sigmoid(c.k * d).to(dtype)
    return out


def config0(device="cpu", res=128, n=50):
    """2D plain PID in FP64: N=50, 128x128, modes 1..4, 3 outliers shifted by
    0.15.  Returns (U float64 N x M, outlier indices)."""
    curves, out_idx, r0 = curve_params_2d(n, 4, 3, "shift", BASE_SEED + 0)
    return soft_masks_2d(curves, r0, res, device, torch.float64), out_idx


def config1(device="cpu", res=512, n=256):
    """2D soft masks in FP32: N=256, 512x512, modes 1..8, 5% outliers
    (round-half-up, 13 of 256) rotated by U(30, 90) degrees."""
    n_out = int(math.floor(0.05 * n + 0.5))
    curves, out_idx, r0 = curve_params_2d(n, 8, n_out, "rotate", BASE_SEED + 1)
    return soft_masks_2d(curves, r0, res, device, torch.float32), out_idx


# --------------------------------------------------------------------------
# 3D scalar fields: sums of Gaussian bumps plus noise
# --------------------------------------------------------------------------
def bump_fields_3d(n, res, seed, n_bumps=16, noise_sd=0.02, device="cpu",
                   dtype=torch.float32):
    """Each member: ``sum_b A_b exp(-|x - c_b|^2 / (2 s_b^2))`` with
    ``c_b ~ U[0,1]^3``, ``s_b ~ U(0.05, 0.15)``, ``A_b ~ N(1, 0.2^2)``, plus
    i.i.d. ``N(0, noise_sd^2)`` noise per point.  Bumps are evaluated
    separably (outer product of three 1D Gaussians)."""
    rng = _rng(seed)
    t = (torch.arange(res, device=device, dtype=torch.float64) + 0.5) / res
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    out = torch.empty((n, res ** 3), dtype=dtype, device=device)
    for i in range(n):
        cen = rng.uniform(0.0, 1.0, size=(n_bumps, 3))
        sig = rng.uniform(0.05, 0.15, size=n_bumps)
        amp = rng.normal(1.0, 0.2, size=n_bumps)
        f = torch.zeros((res, res, res), dtype=torch.float64, device=device)
        for b in range(n_bumps):
            g = [torch.exp(-((t - float(cen[b, d])) ** 2) / (2 * sig[b] ** 2)) for d in range(3)]
            f += float(amp[b]) * g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]
        noise = torch.randn((res ** 3,), generator=gen, device=device, dtype=torch.float32)
        out[i] = (f.reshape(-1) + noise_sd * noise.to(torch.float64)).to(dtype)
    return out


def config2(device="cpu", res=128, n=128):
    """Scalar-field ensemble: N=128 fields on 128^3 (FP32).  The isovalue
    follows N(c=0.5, sigma=0.05); the binary variant thresholds at c."""
    return bump_fields_3d(n, res, BASE_SEED + 2, device=device), dict(c=0.5, sigma=0.05, side=1)


# --------------------------------------------------------------------------
# 3D perturbed spheres (real spherical harmonics up to degree 6)
# --------------------------------------------------------------------------
def real_sh_basis(lmax, cos_t, phi):
    """Orthonormal real spherical harmonics Y_lm, l = 1..lmax, m = -l..l, as a
    list of tensors in (l, m) order.  Associated Legendre functions by the
    standard three-term recurrence (no Condon-Shortley phase)."""
    sin_t = torch.sqrt(torch.clamp(1.0 - cos_t * cos_t, min=0.0))
    P = {}
    for m in range(lmax + 1):
        pmm = torch.ones_like(cos_t)
        dfact = 1.0
        for k in range(1, m + 1):
            dfact *= (2 * k - 1)
        if m > 0:
            pmm = dfact * sin_t ** m
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = cos_t * (2 * m + 1) * pmm
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * cos_t * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    out = []
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                out.append(K * P[(l, 0)])
            elif m > 0:
                out.append(math.sqrt(2) * K * torch.cos(m * phi) * P[(l, am)])
            else:
                out.append(math.sqrt(2) * K * torch.sin(am * phi) * P[(l, am)])
    return out


def sphere_params(n, seed, lmax=6, coef_sd=0.03, k_lo=30.0, k_hi=90.0):
    rng = _rng(seed)
    nb = (lmax + 1) ** 2 - 1
    coef = np.empty((n, nb))
    ks = np.empty(n)
    for i in range(n):
        coef[i] = rng.normal(0.0, coef_sd, size=nb)
        ks[i] = rng.uniform(k_lo, k_hi)
    w_seed = int(rng.integers(0, 2 ** 62))
    return coef, ks, w_seed


def perturbed_spheres_3d(n, res, seed, r0=0.3, lmax=6, device="cpu",
                         dtype=torch.float16, chunk=1 << 20):
    """``u = sigmoid(k (r(dir) - rho))`` with ``rho = |x - (1/2,1/2,1/2)|`` and
    ``r(dir) = r0 (1 + sum_{l<=lmax} sum_m c_lm Y_lm(dir))``, ``c_lm ~
    N(0, 0.03^2)``, ``k ~ U(30, 90)``.  Evaluated in float64 chunk by chunk,
    stored as ``dtype``.  Returns (U, w_seed)."""
    coef, ks, w_seed = sphere_params(n, seed, lmax)
    C = torch.tensor(coef, dtype=torch.float64, device=device)
    K = torch.tensor(ks, dtype=torch.float64, device=device)[:, None]
    M = res ** 3
    out = torch.empty((n, M), dtype=dtype, device=device)
    t = (torch.arange(res, device=device, dtype=torch.float64) + 0.5) / res
    for s in range(0, M, chunk):
        idx = torch.arange(s, min(M, s + chunk), device=device)
        x = t[idx % res] - 0.5
        y = t[(idx // res) % res] - 0.5
        z = t[idx // (res * res)] - 0.5
        rho = torch.sqrt(x * x + y * y + z * z)
        cos_t = z / rho
        phi = torch.atan2(y, x)
        B = torch.stack(real_sh_basis(lmax, cos_t, phi))  # nb x chunk
        r = r0 * (1.0 + C @ B)                              # n x chunk
        out[:, s:s + idx.numel()] = torch.sigmoid(K * (r - rho[None, :])).to(dtype)
    return out, w_seed


def ellipsoid_params(n, seed, frac_out=0.2):
    """Per-member ellipsoid centre (3), semi-axes (3) and a rotation angle about
    z for the scalability ensembles of Sec. 5.2 (80 % normal members, 20 %
    outliers).  Normal members: centre N(1/2, 0.01^2) per axis, semi-axes
    (0.30, 0.22, 0.15) x (1 + N(0, 0.04^2)), angle N(0, 0.05^2).  Outliers
    (the last round(frac_out * n) members): centre N(1/2, 0.05^2), semi-axes
    x U(0.6, 1.3) each, angle U(0.5, 1.5) rad."""
    rng = _rng(seed)
    n_out = int(math.floor(frac_out * n + 0.5))
    base = np.array([0.30, 0.22, 0.15])
    cen = rng.normal(0.5, 0.01, size=(n, 3))
    ax = base * (1.0 + rng.normal(0.0, 0.04, size=(n, 3)))
    ang = rng.normal(0.0, 0.05, size=n)
    if n_out:
        cen[n - n_out:] = rng.normal(0.5, 0.05, size=(n_out, 3))
        ax[n - n_out:] = base * rng.uniform(0.6, 1.3, size=(n_out, 3))
        ang[n - n_out:] = rng.uniform(0.5, 1.5, size=n_out)
    return cen, ax, ang


def ellipsoids_3d(n, res, seed, frac_out=0.2, device="cpu", members_per_chunk=None):
    """Binary 3D ellipsoid masks (uint8 0/1, N x res^3) with controlled
    contamination, the shape of the scalability study (Sec. 5.2): inside where
    ``sum_k ((R (x - c))_k / a_k)^2 <= 1`` on cell centres, evaluated in
    float32 a chunk of members at a time (on ``device``)."""
    cen, ax, ang = ellipsoid_params(n, seed, frac_out)
    M = res ** 3
    if members_per_chunk is None:          # about 2^26 float temporaries per chunk
        members_per_chunk = max(1, min(256, (1 << 26) // M))
    out = torch.empty((n, M), dtype=torch.uint8, device=device)
    t = (torch.arange(res, device=device, dtype=torch.float32) + 0.5) / res
    z = t.view(res, 1, 1).expand(res, res, res).reshape(-1)
    y = t.view(1, res, 1).expand(res, res, res).reshape(-1)
    x = t.view(1, 1, res).expand(res, res, res).reshape(-1)
    for s in range(0, n, members_per_chunk):
        e = min(n, s + members_per_chunk)
        c = torch.tensor(cen[s:e], dtype=torch.float32, device=device)
        a = torch.tensor(ax[s:e], dtype=torch.float32, device=device)
        th = torch.tensor(ang[s:e], dtype=torch.float32, device=device)[:, None]
        dx, dy, dz = x[None] - c[:, 0:1], y[None] - c[:, 1:2], z[None] - c[:, 2:3]
        rx = torch.cos(th) * dx - torch.sin(th) * dy
        ry = torch.sin(th) * dx + torch.cos(th) * dy
        q = (rx / a[:, 0:1]) ** 2 + (ry / a[:, 1:2]) ** 2 + (dz / a[:, 2:3]) ** 2
        out[s:e] = (q <= 1.0).to(torch.uint8)
    return out


def volume_weights(m, seed, device="cpu", lo=0.5, hi=1.5):
    """Per-point weights ``U(lo, hi)`` in FP32 standing in for the cell volumes
    of a non-uniform grid (Sec. 3.4)."""
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    w = torch.rand((m,), generator=gen, device=device, dtype=torch.float32)
    return (lo + (hi - lo) * w).to(torch.float32)


def config3(device="cpu", res=256, n=64, weights=True):
    """Large 3D PID-mean: N=64 FP16 perturbed-sphere masks on 256^3 with
    optional U(0.5, 1.5) FP32 per-point weights.  Returns (U, w or None)."""
    U, w_seed = perturbed_spheres_3d(n, res, BASE_SEED + 3, device=device)
    w = volume_weights(res ** 3, w_seed, device) if weights else None
    return U, w


# --------------------------------------------------------------------------
# Constructions with known depth structure
# --------------------------------------------------------------------------
def concentric_disks(radii, res, k, device="cpu", dtype=torch.float64):
    """Soft disks ``sigmoid(k (r - |x - c|))`` centred in the unit square."""
    x, y = grid_coords(res, 2, device)
    rho = torch.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2)
    return torch.stack([torch.sigmoid(k * (float(r) - rho)) for r in radii]).to(dtype)


def binary_disks(radii, res, device="cpu"):
    """Binary disks ``|x - c| < r`` as uint8 0/1 (a nested chain when the radii
    are increasing)."""
    x, y = grid_coords(res, 2, device)
    rho = torch.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2)
    return torch.stack([(rho < float(r)).to(torch.uint8) for r in radii])


def random_binary(n, m, seed, p_lo=0.2, p_hi=0.8, device="cpu"):
    """Independent Bernoulli masks with a per-member density ``U(p_lo, p_hi)``,
    uint8 0/1."""
    rng = _rng(seed)
    p = rng.uniform(p_lo, p_hi, size=(n, 1))
    return torch.from_numpy((rng.uniform(size=(n, m)) < p).astype(np.uint8)).to(device)


def random_soft(n, m, seed, device="cpu", dtype=torch.float32):
    """Smooth-ish random soft masks: a per-member random threshold of a shared
    random field plus member noise, passed through a sigmoid (values in (0,1))."""
    rng = _rng(seed)
    base = rng.normal(size=m)
    out = np.empty((n, m))
    for i in range(n):
        out[i] = 1.0 / (1.0 + np.exp(-(rng.uniform(2, 6)) * (base + rng.normal(0, 0.5, size=m) - rng.normal(0, 0.5))))
    return torch.from_numpy(out).to(dtype).to(device)


# --------------------------------------------------------------------------
# Serving workload: request mix
# --------------------------------------------------------------------------
SIDES_2D = tuple(range(128, 1025, 64))
SIDES_3D = tuple(range(64, 193, 16))


@dataclass
class Request:
    rid: int
    arrival_s: float
    kind: str        # "2d" | "3d"
    n: int
    side: int
    variant: str     # "pairs" | "mean"

    @property
    def m(self):
        return self.side ** (2 if self.kind == "2d" else 3)


def serving_requests(count, rate_hz=200.0, seed=BASE_SEED + 4, frac_2d=0.6,
                     frac_pairs=0.5):
    """Poisson arrivals at ``rate_hz``.  60% 2D requests (N ~ U{32..512},
    side from 128..1024 in steps of 64), 40% 3D (N ~ U{16..128}, side from
    64..192 in steps of 16); each tagged all-pairs or PID-mean 50/50."""
    rng = _rng(seed)
    t = 0.0
    reqs = []
    for r in range(count):
        t += rng.exponential(1.0 / rate_hz)
        if rng.uniform() < frac_2d:
            kind, n, side = "2d", int(rng.integers(32, 513)), int(rng.choice(SIDES_2D))
        else:
            kind, n, side = "3d", int(rng.integers(16, 129)), int(rng.choice(SIDES_3D))
        variant = "pairs" if rng.uniform() < frac_pairs else "mean"
        reqs.append(Request(r, t, kind, n, side, variant))
    return reqs


def serving_pool(kind, side, n_max, device="cpu"):
    """Base ensemble for one (kind, side) of the serving pool: FP16 masks as in
    the 2D soft-mask workload (modes 1..8, 5% rotated outliers) or the 3D
    perturbed-sphere workload.  Requests take the first N members."""
    seed = BASE_SEED + 100 + side + (0 if kind == "2d" else 10000)
    if kind == "2d":
        curves, _, r0 = curve_params_2d(n_max, 8, max(1, n_max // 20), "rotate", seed)
        return soft_masks_2d(curves, r0, side, device, torch.float16)
    U, _ = perturbed_spheres_3d(n_max, side, seed, device=device)
    return U
