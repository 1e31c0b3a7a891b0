"""Comparison helpers for the GPU parity tests (no GPU work in here)."""
import numpy as np

# Tolerances (absolute, on every depth, IN_in, IN_out and inclusion entry)
TOL_MIXED = 1e-4     # 16-bit MFMA inputs with FP32 accumulation
TOL_F32 = 2e-6       # FP32 vector FMA
TOL_F64 = 1e-12      # FP64 vector FMA


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def max_err(res, ref, keys=("in_in", "in_out", "depth")):
    out = {}
    for k in keys:
        if k in res and k in ref:
            out[k] = float(np.max(np.abs(np64(res[k]) - np.asarray(ref[k], dtype=np.float64))))
    return out


def assert_close(res, ref, tol, keys=("mass_rel", "in_in", "in_out", "depth", "inclusion"), label=""):
    for k in keys:
        if k == "mass_rel":
            if "mass" in res and "mass" in ref:
                a, b = np64(res["mass"]), np.asarray(ref["mass"], dtype=np.float64)
                rel = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
                assert np.all(rel <= max(tol, 1e-12) * 10), f"{label} mass rel err {rel.max()}"
            continue
        if k not in res or k not in ref:
            continue
        a, b = np64(res[k]), np.asarray(ref[k], dtype=np.float64)
        err = np.max(np.abs(a - b)) if a.size else 0.0
        assert err <= tol, f"{label} {k}: max abs err {err:.3e} > {tol:.1e}"


def assert_bitwise(res, ref, keys=("in_in", "in_out", "depth", "inclusion", "mass"), label=""):
    for k in keys:
        if k not in res or k not in ref:
            continue
        a, b = np64(res[k]), np.asarray(ref[k], dtype=np.float64)
        bad = np.flatnonzero(a.ravel() != b.ravel())
        assert bad.size == 0, f"{label} {k}: {bad.size} entries differ, first {bad[:5]} " \
                              f"gpu {a.ravel()[bad[:3]]} ref {b.ravel()[bad[:3]]}"


def tie_groups(depth_ref, tol):
    """Members whose reference depths are within 2*tol (transitive closure)."""
    d = np.asarray(depth_ref, dtype=np.float64)
    order = np.argsort(-d, kind="stable")
    groups, cur = [], [order[0]]
    for a, b in zip(order[:-1], order[1:]):
        if abs(d[a] - d[b]) <= 2 * tol:
            cur.append(b)
        else:
            groups.append(cur)
            cur = [b]
    groups.append(cur)
    return groups


def assert_ranks(rank_gpu, depth_ref, tol, label=""):
    """Ranks equal outside tie groups: inside a group the GPU may permute."""
    from oracle import rank_order
    rg = rank_gpu.detach().cpu().numpy().astype(np.int64)
    rr, _ = rank_order(depth_ref)
    if tol == 0:
        assert (rg == rr).all(), f"{label} ranks differ"
        return
    for g in tie_groups(depth_ref, tol):
        assert sorted(rg[g].tolist()) == sorted(rr[g].tolist()), f"{label} ranks differ in group {g}"
