"""Python binding of ``libpid.so``, the MI355X (gfx950) PID library.

Argument marshalling only: every step of the depth computation runs in the
HIP kernels behind the C ABI declared in ``include/pid.h``.  PyTorch provides
device memory (tensors) and streams.  The functions carry the names of the C
entry points; each checks its tensors, fills the C structs, allocates the
outputs and the workspace as torch tensors, and calls the library on the
current torch stream (or the stream given).

The library must have been built (``python -m paper_2512_15187_amd.build``);
there is no fallback: a missing library or device raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpid.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pid.h")

# ---- enums (mirror include/pid.h) ----
PID_OK, PID_ERR_INVALID_ARG, PID_ERR_UNSUPPORTED, PID_ERR_WORKSPACE_TOO_SMALL = 0, 1, 2, 3
PID_ERR_DEVICE, PID_ERR_VALUE_RANGE, PID_ERR_OVER_BUDGET, PID_ERR_CANCELLED, PID_ERR_INTERNAL = 4, 5, 6, 7, 8
PID_F64, PID_F32, PID_F16, PID_BF16, PID_U8, PID_B1 = 0, 1, 2, 3, 4, 5
PID_ISO_NONE, PID_ISO_GAUSSIAN, PID_ISO_STEP, PID_ISO_RAMP, PID_ISO_TENT, PID_ISO_DENSITY = 0, 1, 2, 3, 4, 5
GEMM = {"auto": 0, "f64": 1, "f32": 2, "f16": 3, "bf16": 4, "bf16_split": 5, "i8": 6}
PID_FLAG_VALIDATE = 1

_DTYPES = {torch.float64: PID_F64, torch.float32: PID_F32, torch.float16: PID_F16,
           torch.bfloat16: PID_BF16, torch.uint8: PID_U8}


class PidError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_STATUS = {0: "PID_OK", 1: "PID_ERR_INVALID_ARG", 2: "PID_ERR_UNSUPPORTED",
           3: "PID_ERR_WORKSPACE_TOO_SMALL", 4: "PID_ERR_DEVICE", 5: "PID_ERR_VALUE_RANGE",
           6: "PID_ERR_OVER_BUDGET", 7: "PID_ERR_CANCELLED", 8: "PID_ERR_INTERNAL"}


class pid_ensemble(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("data", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


class pid_iso(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("side", ctypes.c_int32),
                ("c", ctypes.c_double), ("sigma", ctypes.c_double)]


class pid_out(ctypes.Structure):
    _fields_ = [("inclusion", ctypes.c_void_p), ("mass", ctypes.c_void_p),
                ("in_in", ctypes.c_void_p), ("in_out", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("rank", ctypes.c_void_p), ("order", ctypes.c_void_p)]


class pid_request(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("gemm", ctypes.c_int32), ("ens", pid_ensemble),
                ("iso", pid_iso), ("out", pid_out), ("ready", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpid.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2512_15187_amd.build`")
    lib = ctypes.CDLL(path)
    V, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "pid_workspace_size": ([P(pid_ensemble), P(pid_iso), I32, I32, P(ctypes.c_size_t)], I32),
        "pid_all_pairs": ([P(pid_ensemble), P(pid_iso), I32, P(pid_out), V, ctypes.c_size_t, V], I32),
        "pid_mean": ([P(pid_ensemble), P(pid_iso), P(pid_out), V, ctypes.c_size_t, V], I32),
        "pid_pairs_depths": ([P(pid_ensemble), P(pid_iso), P(pid_out), V, ctypes.c_size_t, V], I32),
        "pid_mean_weighted": ([P(pid_ensemble), P(pid_iso), V, P(pid_out), V, ctypes.c_size_t, V], I32),
        "pid_field_max": ([P(pid_ensemble), V, V], I32),
        "pid_pack_bits": ([P(pid_ensemble), V, I64, V], I32),
        "pid_both_static": ([P(pid_ensemble), P(pid_iso), I32, P(pid_out), P(pid_out), V], I32),
        "pid_both": ([P(pid_ensemble), P(pid_iso), I32, P(pid_out), P(pid_out), V, ctypes.c_size_t, V], I32),
        "pid_extract": ([P(pid_ensemble), P(pid_iso), V, I32, V], I32),
        "pid_rank": ([V, I64, V, V, V], I32),
        "pid_bands": ([P(pid_ensemble), P(pid_iso), V, I64, I64, ctypes.c_double, V, V], I32),
        "pid_server_create": ([I32, V, ctypes.c_size_t, I32, P(V)], I32),
        "pid_submit": ([V, P(pid_request), P(ctypes.c_uint64)], I32),
        "pid_poll": ([V, ctypes.c_uint64, P(I32), P(I32)], I32),
        "pid_wait": ([V, ctypes.c_uint64, P(I32)], I32),
        "pid_request_times": ([V, ctypes.c_uint64, P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double)], I32),
        "pid_server_destroy": ([V], I32),
        "pid_server_set_budget": ([V, ctypes.c_size_t], I32),
        "pid_server_clock": ([V, P(ctypes.c_double)], I32),
        "pid_request_device_times": ([V, ctypes.c_uint64, P(ctypes.c_double), P(ctypes.c_double)], I32),
        "pid_release": ([V, ctypes.c_uint64], I32),
        "pid_timing_enable": ([I32], I32),
        "pid_timing_get": ([ctypes.c_char_p, P(ctypes.c_double), P(I64)], I32),
        "pid_timing_select": ([ctypes.c_char_p], I32),
        "pid_timing_sample": ([I32], I32),
        "pid_status_string": ([I32], ctypes.c_char_p),
        "pid_last_error": ([], ctypes.c_char_p),
        "pid_abi_version": ([], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def declared_symbols(header: str = HEADER):
    """Names of the functions declared in include/pid.h."""
    text = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\*\s]+?\b(pid_\w+)\s*\(", text, re.M)))


def _check(status):
    if status != PID_OK:
        msg = load_library().pid_last_error().decode(errors="replace")
        raise PidError(status, msg)


def _require_gpu(t: torch.Tensor, what: str):
    if not torch.cuda.is_available():
        raise RuntimeError("the PID library needs a GPU; none is available")
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")


class PackedMasks:
    """Bit-packed binary masks (PID_B1): ``words`` is an N x ldw int32 device
    tensor (unit stride along a row) whose row i holds the bits of member i,
    point x in bit x mod 32 of word x / 32; ``m`` is the number of points."""

    def __init__(self, words: torch.Tensor, m: int):
        if words.dtype != torch.int32 or words.dim() != 2 or words.stride(1) != 1:
            raise ValueError("words must be a 2-D int32 tensor with unit stride along a row")
        if not 1 <= m <= 32 * words.shape[1]:
            raise ValueError("m must be between 1 and 32 * words.shape[1]")
        self.words, self.m = words, int(m)
        self.shape = (words.shape[0], self.m)
        self.device = words.device


def make_ensemble(U, weights: torch.Tensor | None = None, validate: bool = False):
    """Fill pid_ensemble from an N x M (row-strided) device tensor or from
    PackedMasks."""
    if isinstance(U, PackedMasks):
        _require_gpu(U.words, "words")
        if weights is not None:
            raise ValueError("bit-packed masks take no point weights")
        return pid_ensemble(U.words.shape[0], U.m, 32 * U.words.stride(0), PID_B1, 0, U.words.data_ptr(), None)
    _require_gpu(U, "U")
    if U.dim() != 2 or U.stride(1) != 1:
        raise ValueError("U must be 2-D with unit stride along the points")
    if U.dtype == torch.bool:
        raise ValueError("pass binary masks as uint8 0/1")
    if U.dtype not in _DTYPES:
        raise ValueError(f"unsupported dtype {U.dtype}")
    e = pid_ensemble(U.shape[0], U.shape[1], U.stride(0), _DTYPES[U.dtype],
                     PID_FLAG_VALIDATE if validate else 0, U.data_ptr(), None)
    if weights is not None:
        _require_gpu(weights, "weights")
        if weights.dtype != torch.float32 or weights.dim() != 1 or weights.numel() != U.shape[1] \
                or not weights.is_contiguous():
            raise ValueError("weights must be a contiguous float32 vector of length M")
        e.weights = weights.data_ptr()
    return e


def make_iso(iso: dict | None):
    """``None`` / {"kind": "none"}; {"kind": "gaussian", "c", "sigma", "side"};
    {"kind": "step", "c", "side"}; {"kind": "ramp", "c", "width", "side"};
    {"kind": "tent", "c", "width"}; {"kind": "density", "c"} (the width goes
    into the C struct's ``sigma``)."""
    if iso is None or iso.get("kind", "none") == "none":
        return pid_iso(PID_ISO_NONE, 1, 0.0, 0.0)
    kind = {"gaussian": PID_ISO_GAUSSIAN, "step": PID_ISO_STEP, "ramp": PID_ISO_RAMP, "tent": PID_ISO_TENT,
            "density": PID_ISO_DENSITY}[iso["kind"]]
    width = iso.get("width", iso.get("sigma", 0.0))
    return pid_iso(kind, int(iso.get("side", 1)), float(iso["c"]), float(width))


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def pid_workspace_size(U, weights=None, iso=None, variant=0, gemm="auto") -> int:
    lib = load_library()
    e, i = make_ensemble(U, weights), make_iso(iso)
    out = ctypes.c_size_t(0)
    _check(lib.pid_workspace_size(ctypes.byref(e), ctypes.byref(i), int(variant), GEMM[gemm], ctypes.byref(out)))
    return int(out.value)


def _outputs(n, device, inclusion):
    d = dict(mass=torch.empty(n, dtype=torch.float64, device=device),
             in_in=torch.empty(n, dtype=torch.float64, device=device),
             in_out=torch.empty(n, dtype=torch.float64, device=device),
             depth=torch.empty(n, dtype=torch.float64, device=device),
             rank=torch.empty(n, dtype=torch.int32, device=device),
             order=torch.empty(n, dtype=torch.int32, device=device))
    if inclusion:
        d["inclusion"] = torch.empty((n, n), dtype=torch.float64, device=device)
    o = pid_out(d["inclusion"].data_ptr() if inclusion else None, d["mass"].data_ptr(),
                d["in_in"].data_ptr(), d["in_out"].data_ptr(), d["depth"].data_ptr(),
                d["rank"].data_ptr(), d["order"].data_ptr())
    return d, o


def _workspace(nbytes, device, workspace):
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError("workspace too small")
        return workspace
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def pid_all_pairs(U, weights=None, iso=None, gemm="auto", inclusion=True, workspace=None,
                  stream=None, validate=False):
    """All-pairs PID.  Returns a dict of device tensors: inclusion (N x N, if
    asked), mass, in_in, in_out, depth (float64), rank, order (int32)."""
    lib = load_library()
    e, i = make_ensemble(U, weights, validate), make_iso(iso)
    ws_n = ctypes.c_size_t(0)
    _check(lib.pid_workspace_size(ctypes.byref(e), ctypes.byref(i), 0, GEMM[gemm], ctypes.byref(ws_n)))
    ws = _workspace(ws_n.value, U.device, workspace)
    d, o = _outputs(U.shape[0], U.device, inclusion)
    _check(lib.pid_all_pairs(ctypes.byref(e), ctypes.byref(i), GEMM[gemm], ctypes.byref(o),
                             ctypes.c_void_p(ws.data_ptr()), ws_n.value, _stream_ptr(stream)))
    d["_workspace"] = ws
    return d


def pid_mean(U, weights=None, iso=None, workspace=None, stream=None, validate=False):
    """PID-mean.  Returns mass, in_in, in_out, depth (float64), rank, order."""
    lib = load_library()
    e, i = make_ensemble(U, weights, validate), make_iso(iso)
    ws_n = ctypes.c_size_t(0)
    _check(lib.pid_workspace_size(ctypes.byref(e), ctypes.byref(i), 1, 0, ctypes.byref(ws_n)))
    ws = _workspace(ws_n.value, U.device, workspace)
    d, o = _outputs(U.shape[0], U.device, False)
    _check(lib.pid_mean(ctypes.byref(e), ctypes.byref(i), ctypes.byref(o),
                        ctypes.c_void_p(ws.data_ptr()), ws_n.value, _stream_ptr(stream)))
    d["_workspace"] = ws
    return d


def pid_pairs_depths(U, weights=None, iso=None, workspace=None, stream=None, validate=False):
    """All-pairs PID depths without the inclusion matrix (three streaming
    passes, O(N M)).  Returns mass, in_in, in_out, depth (float64), rank, order."""
    lib = load_library()
    e, i = make_ensemble(U, weights, validate), make_iso(iso)
    ws_n = ctypes.c_size_t(0)
    _check(lib.pid_workspace_size(ctypes.byref(e), ctypes.byref(i), 3, 0, ctypes.byref(ws_n)))
    ws = _workspace(ws_n.value, U.device, workspace)
    d, o = _outputs(U.shape[0], U.device, False)
    _check(lib.pid_pairs_depths(ctypes.byref(e), ctypes.byref(i), ctypes.byref(o),
                                ctypes.c_void_p(ws.data_ptr()), ws_n.value, _stream_ptr(stream)))
    d["_workspace"] = ws
    return d


def pid_mean_weighted(U, member_weights, weights=None, iso=None, workspace=None, stream=None, validate=False):
    """PID-mean against the mean contour weighted by ``member_weights`` (a
    float64 device vector of N reliabilities).  Returns mass, in_in, in_out,
    depth (float64), rank, order."""
    lib = load_library()
    e, i = make_ensemble(U, weights, validate), make_iso(iso)
    _require_gpu(member_weights, "member_weights")
    if member_weights.dtype != torch.float64 or member_weights.numel() != U.shape[0] \
            or not member_weights.is_contiguous():
        raise ValueError("member_weights must be a contiguous float64 vector of length N")
    ws_n = ctypes.c_size_t(0)
    _check(lib.pid_workspace_size(ctypes.byref(e), ctypes.byref(i), 4, 0, ctypes.byref(ws_n)))
    ws = _workspace(ws_n.value, U.device, workspace)
    d, o = _outputs(U.shape[0], U.device, False)
    _check(lib.pid_mean_weighted(ctypes.byref(e), ctypes.byref(i), ctypes.c_void_p(member_weights.data_ptr()),
                                 ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), ws_n.value, _stream_ptr(stream)))
    d["_workspace"] = ws
    return d


def pid_pack_bits(U, out=None, stream=None) -> PackedMasks:
    """Pack N x M uint8 0/1 device masks into PackedMasks (on the device).
    ``out``: an N x ldw int32 device tensor to fill (unit stride along a row,
    32 * ldw >= M; its words past the last one that holds points are left as
    they are), else a new one whose rows are padded to a multiple of four
    words (16-byte rows, which the PID-mean kernels read as vectors)."""
    lib = load_library()
    e = make_ensemble(U)
    if U.dtype != torch.uint8:
        raise ValueError("pid_pack_bits packs uint8 0/1 masks")
    m = U.shape[1]
    if out is None:
        words = torch.zeros((U.shape[0], (m + 127) // 128 * 4), dtype=torch.int32, device=U.device)
    else:
        words = out
        _require_gpu(words, "out")
        if words.dtype != torch.int32 or words.dim() != 2 or words.stride(1) != 1 or words.shape[0] != U.shape[0] \
                or 32 * words.shape[1] < m:
            raise ValueError("out must be an N x ldw int32 tensor with unit row stride and 32 * ldw >= M")
    ld = 32 * words.stride(0)
    _check(lib.pid_pack_bits(ctypes.byref(e), ctypes.c_void_p(words.data_ptr()), ld, _stream_ptr(stream)))
    return PackedMasks(words, m)


def pid_field_max(U, stream=None):
    """Largest stored value of the ensemble as a one-element float64 device
    tensor (NaN values skipped)."""
    lib = load_library()
    e = make_ensemble(U)
    out = torch.empty(1, dtype=torch.float64, device=U.device)
    _check(lib.pid_field_max(ctypes.byref(e), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def pid_both(U, weights=None, iso=None, gemm="auto", inclusion=True, workspace=None, stream=None,
             validate=False):
    """All-pairs PID and PID-mean in one call, from one all-pairs pass (the
    PID-mean numerators are the Gram row sums).  Returns (pairs dict, mean
    dict)."""
    lib = load_library()
    e, i = make_ensemble(U, weights, validate), make_iso(iso)
    ws_n = ctypes.c_size_t(0)
    _check(lib.pid_workspace_size(ctypes.byref(e), ctypes.byref(i), 2, GEMM[gemm], ctypes.byref(ws_n)))
    ws = _workspace(ws_n.value, U.device, workspace)
    dp, op = _outputs(U.shape[0], U.device, inclusion)
    dm, om = _outputs(U.shape[0], U.device, False)
    _check(lib.pid_both(ctypes.byref(e), ctypes.byref(i), GEMM[gemm], ctypes.byref(op), ctypes.byref(om),
                        ctypes.c_void_p(ws.data_ptr()), ws_n.value, _stream_ptr(stream)))
    dp["_workspace"] = ws
    return dp, dm


def pid_extract(U, iso, out_dtype=torch.float32, stream=None):
    """Membership probabilities (N x M dense) from stored values."""
    lib = load_library()
    e, i = make_ensemble(U), make_iso(iso)
    out = torch.empty((U.shape[0], U.shape[1]), dtype=out_dtype, device=U.device)
    odt = {torch.float32: PID_F32, torch.float64: PID_F64}[out_dtype]
    _check(lib.pid_extract(ctypes.byref(e), ctypes.byref(i), ctypes.c_void_p(out.data_ptr()), odt,
                           _stream_ptr(stream)))
    return out


BAND_MEDIAN, BAND_UNION_INNER, BAND_INTER_INNER, BAND_UNION_OUTER, BAND_INTER_OUTER = 1, 2, 4, 8, 16
BAND_BAD_ORDER = 128


def pid_bands(U, order, k_inner, k_outer, threshold=0.5, iso=None, stream=None):
    """Contour-boxplot bands (one uint8 code per point, bits BAND_*) of the
    ensemble U ranked by ``order`` (int32 device tensor, deepest first)."""
    lib = load_library()
    _require_gpu(order, "order")
    if order.dtype != torch.int32 or order.dim() != 1 or not order.is_contiguous():
        raise ValueError("order must be a contiguous 1-D int32 tensor")
    if order.numel() < k_outer:
        raise ValueError("order has fewer than k_outer entries")
    e, i = make_ensemble(U), make_iso(iso)
    out = torch.empty(U.shape[1], dtype=torch.uint8, device=U.device)
    _check(lib.pid_bands(ctypes.byref(e), ctypes.byref(i), ctypes.c_void_p(order.data_ptr()), int(k_inner),
                         int(k_outer), float(threshold), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def pid_rank(depth, stream=None):
    """(rank, order) int32 device tensors from a float64 depth vector."""
    lib = load_library()
    _require_gpu(depth, "depth")
    depth = depth.contiguous()
    if depth.dtype != torch.float64:
        raise ValueError("depth must be float64")
    n = depth.numel()
    rank = torch.empty(n, dtype=torch.int32, device=depth.device)
    order = torch.empty(n, dtype=torch.int32, device=depth.device)
    _check(lib.pid_rank(ctypes.c_void_p(depth.data_ptr()), n, ctypes.c_void_p(rank.data_ptr()),
                        ctypes.c_void_p(order.data_ptr()), _stream_ptr(stream)))
    return rank, order


class PreparedCall:
    """One depth call with its structs, outputs and workspace allocated once,
    so that repeated ``run()`` calls allocate nothing (benchmark loops,
    serving drivers).  variant: "pairs", "mean", "both" (then ``out`` holds
    the all-pairs results and ``out_mean`` the PID-mean ones) or "depths"
    (all-pairs depths without the inclusion matrix)."""

    def __init__(self, variant, U, weights=None, iso=None, gemm="auto", inclusion=False, member_weights=None):
        lib = load_library()
        self.variant = {"pairs": 0, "mean": 1, "both": 2, "depths": 3, "weighted": 4}[variant]
        if self.variant == 4 and (member_weights is None or member_weights.dtype != torch.float64):
            raise ValueError("variant 'weighted' needs float64 member_weights")
        self.member_weights = member_weights
        self.gemm = GEMM[gemm]
        self.e, self.i = make_ensemble(U, weights), make_iso(iso)
        n = ctypes.c_size_t(0)
        _check(lib.pid_workspace_size(ctypes.byref(self.e), ctypes.byref(self.i), self.variant, self.gemm,
                                      ctypes.byref(n)))
        self.ws_bytes = n.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=U.device)
        self.out, self.o = _outputs(U.shape[0], U.device, inclusion and self.variant in (0, 2))
        if self.variant == 2:
            self.out_mean, self.om = _outputs(U.shape[0], U.device, False)
        self._keep = (U, weights)

    def run(self, stream=None):
        lib = load_library()
        st = _stream_ptr(stream)
        ws = ctypes.c_void_p(self.ws.data_ptr())
        if self.variant == 0:
            _check(lib.pid_all_pairs(ctypes.byref(self.e), ctypes.byref(self.i), self.gemm, ctypes.byref(self.o),
                                     ws, self.ws_bytes, st))
        elif self.variant == 1:
            _check(lib.pid_mean(ctypes.byref(self.e), ctypes.byref(self.i), ctypes.byref(self.o), ws,
                                self.ws_bytes, st))
        elif self.variant == 3:
            _check(lib.pid_pairs_depths(ctypes.byref(self.e), ctypes.byref(self.i), ctypes.byref(self.o), ws,
                                        self.ws_bytes, st))
        elif self.variant == 4:
            _check(lib.pid_mean_weighted(ctypes.byref(self.e), ctypes.byref(self.i),
                                         ctypes.c_void_p(self.member_weights.data_ptr()), ctypes.byref(self.o), ws,
                                         self.ws_bytes, st))
        else:
            _check(lib.pid_both(ctypes.byref(self.e), ctypes.byref(self.i), self.gemm, ctypes.byref(self.o),
                                ctypes.byref(self.om), ws, self.ws_bytes, st))
        return self.out


def pid_timing_enable(on: bool = True):
    """Turn per-kernel event timing on/off (clears the totals)."""
    _check(load_library().pid_timing_enable(1 if on else 0))


def pid_timing_select(names=None):
    """Time only the listed kernels (a comma-separated string or a list);
    None times all of them."""
    if names is not None and not isinstance(names, str):
        names = ",".join(names)
    _check(load_library().pid_timing_select(None if names is None else names.encode()))


def pid_timing_sample(every: int = 1):
    """Bracket only every `every`-th launch of each timed kernel."""
    _check(load_library().pid_timing_sample(int(every)))


def pid_timing_get(kernel: str):
    """(total milliseconds, launches) of one library kernel since enabling."""
    ms, n = ctypes.c_double(0), ctypes.c_int64(0)
    _check(load_library().pid_timing_get(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


_VARIANT = {"pairs": 0, "mean": 1, "depths": 3}


class PidServer:
    """Continuous-batching server over ``pid_server_*``.  The arena is a
    device buffer owned by this object."""

    def __init__(self, arena_bytes: int, max_slots: int = 4, device: int = 0, budget: int = 0):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the PID server needs a GPU")
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        h = ctypes.c_void_p()
        _check(lib.pid_server_create(device, ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                     int(max_slots), ctypes.byref(h)))
        self.h = h
        self._keep = {}
        if budget:
            self.pid_server_set_budget(budget)

    def pid_server_set_budget(self, footprint_bytes: int):
        """Footprint budget in bytes (0 = none)."""
        _check(load_library().pid_server_set_budget(self.h, int(footprint_bytes)))

    def pid_server_clock(self) -> float:
        """Seconds on the server's clock."""
        t = ctypes.c_double()
        _check(load_library().pid_server_clock(self.h, ctypes.byref(t)))
        return t.value

    def pid_submit(self, U, variant="pairs", weights=None, iso=None, gemm="auto", inclusion=False,
                   validate=False):
        """Queue a request (variant "pairs", "mean" or "depths"); returns
        (ticket, outputs dict filled on completion)."""
        lib = load_library()
        e, i = make_ensemble(U, weights, validate), make_iso(iso)
        d, o = _outputs(U.shape[0], U.device, inclusion and variant == "pairs")
        # the server's streams wait for the work queued so far on the current
        # stream (the inputs and the output allocations)
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(U.device))
        req = pid_request(_VARIANT[variant], GEMM[gemm], e, i, o, ctypes.c_void_p(ev.cuda_event))
        t = ctypes.c_uint64(0)
        _check(lib.pid_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (U, weights, d, ev)
        return t.value, d

    def pid_poll(self, ticket):
        done, res = ctypes.c_int(0), ctypes.c_int(0)
        _check(load_library().pid_poll(self.h, ticket, ctypes.byref(done), ctypes.byref(res)))
        return bool(done.value), res.value

    def pid_wait(self, ticket):
        res = ctypes.c_int(0)
        _check(load_library().pid_wait(self.h, ticket, ctypes.byref(res)))
        return res.value

    def last_error(self) -> str:
        """Error text of the last failed request waited for or polled on
        this thread."""
        return load_library().pid_last_error().decode(errors="replace")

    def pid_request_times(self, ticket):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(load_library().pid_request_times(self.h, ticket, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def pid_request_device_times(self, ticket):
        """(start, end) of the request on the device, ms after server creation."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(load_library().pid_request_device_times(self.h, ticket, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def release(self, ticket):
        """Forget a finished request (server record and the tensors kept for it)."""
        _check(load_library().pid_release(self.h, ticket))
        self._keep.pop(ticket, None)

    def pid_server_destroy(self):
        if self.h:
            _check(load_library().pid_server_destroy(self.h))
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.pid_server_destroy()
        except Exception:
            pass
