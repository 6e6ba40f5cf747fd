"""Python binding of ``libgfnc.so`` (the C ABI in ``include/gfnc.h``).

GF(2^n) random linear network coding on MI355X: region multiply-add,
encoding (a coefficient matrix times a generation of source packets) and
Gauss-Jordan decoding, after Guenther, Appel and Carle, arXiv 1909.02871
(Sec. II defines the operations; Sec. IV the table-lookup and
bit-decomposition kernels they are computed with on CPUs).

This module only marshals arguments: torch CUDA tensors supply device
pointers and streams, every computation runs in the library's HIP kernels.
If the library is missing or no GPU is present the calls raise; there is no
CPU fallback.

Names match the C entry points: ``gf_init``, ``gf_region_madd``,
``gf_region_mul``, ``gf_region_madd_batched``, ``gf_encode``, ``gf_decode``,
``gf_decode_noalloc``, ``gf_invert``, ``gf_encode_batched`` (device descriptors, with a
plan from ``gf_plan_encode``), ``gf_decode_batched`` (device descriptors and a
workspace, no plan), ``gf_plan_decode``/``gf_plan_recode`` with
``gf_plan_launch``/``gf_plan_launch_graph``, ``gf_encode_each`` and the serving
runtime ``Server``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GFNC_LIB") or os.path.join(_HERE, "libgfnc.so")

GF_2, GF_4, GF_16, GF_256 = 1, 2, 4, 8
FIELDS = (GF_2, GF_4, GF_16, GF_256)
GF_OK, GF_EINVAL, GF_ENOTINIT, GF_EDEVICE, GF_ESINGULAR, GF_ENOMEM, GF_ERANGE = 0, -1, -2, -3, -4, -5, -6
GF_ECANCELED = -7
GF_MAX_N = 256
GF_MAX_K = 65535

_lib = None


class GFError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, strerror(code) if _lib else "error", code))


class gf_region(C.Structure):
    _fields_ = [("y", C.c_void_p), ("x", C.c_void_p), ("len", C.c_uint64), ("c", C.c_uint32),
                ("reserved", C.c_uint32)]


class gf_gen(C.Structure):
    _fields_ = [("C", C.c_void_p), ("S", C.c_void_p), ("Y", C.c_void_p), ("K", C.c_uint32), ("N", C.c_uint32),
                ("len", C.c_uint64), ("ld_s", C.c_uint64), ("ld_y", C.c_uint64)]


class gf_sys(C.Structure):
    _fields_ = [("C", C.c_void_p), ("B", C.c_void_p), ("S", C.c_void_p), ("N", C.c_uint32),
                ("reserved", C.c_uint32), ("len", C.c_uint64), ("ld_b", C.c_uint64), ("ld_s", C.c_uint64)]


class gf_recode_desc(C.Structure):
    _fields_ = [("R", C.c_void_p), ("Cin", C.c_void_p), ("Bin", C.c_void_p), ("Cout", C.c_void_p),
                ("Yout", C.c_void_p), ("Kout", C.c_uint32), ("M", C.c_uint32), ("N", C.c_uint32),
                ("reserved", C.c_uint32), ("len", C.c_uint64), ("ld_cin", C.c_uint64), ("ld_b", C.c_uint64),
                ("ld_cout", C.c_uint64), ("ld_y", C.c_uint64)]


class gf_tuning(C.Structure):
    _fields_ = [("form", C.c_int), ("bytes_per_lane", C.c_int), ("grid_blocks", C.c_int),
                ("reserved", C.c_int)]


_SIGS = {
    "gf_init": (C.c_int, []),
    "gf_strerror": (C.c_char_p, [C.c_int]),
    "gf_region_madd": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_size_t, C.c_void_p]),
    "gf_region_mul": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_size_t, C.c_void_p]),
    "gf_region_madd_batched": (C.c_int, [C.c_int, C.c_void_p, C.c_int, C.c_size_t, C.c_void_p]),
    "gf_encode": (C.c_int, [C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p,
                            C.c_size_t, C.c_size_t, C.c_void_p]),
    "gf_decode_workspace": (C.c_size_t, [C.c_int, C.c_int, C.c_int]),
    "gf_decode": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p, C.c_size_t,
                            C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "gf_decode_noalloc": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p, C.c_size_t,
                                    C.c_size_t, C.c_void_p, C.c_void_p]),
    "gf_invert": (C.c_int, [C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gf_plan_encode": (C.c_int, [C.c_int, C.POINTER(gf_gen), C.c_int, C.POINTER(gf_tuning),
                                 C.POINTER(C.c_void_p)]),
    "gf_plan_decode": (C.c_int, [C.c_int, C.POINTER(gf_sys), C.c_int, C.POINTER(gf_tuning),
                                 C.POINTER(C.c_void_p)]),
    "gf_encode_batched": (C.c_int, [C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "gf_plan_errors": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "gf_decode_batched": (C.c_int, [C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.c_void_p]),
    "gf_plan_launch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gf_plan_launch_graph": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gf_plan_tuning": (C.c_int, [C.c_void_p, C.POINTER(gf_tuning)]),
    "gf_ceiling": (C.c_int, [C.c_int, C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_void_p]),
    "gf_plan_destroy": (None, [C.c_void_p]),
    "gf_encode_each": (C.c_int, [C.c_int, C.POINTER(gf_gen), C.c_int, C.POINTER(gf_tuning), C.c_void_p]),
    "gf_recode": (C.c_int, [C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p,
                            C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_size_t, C.c_void_p]),
    "gf_plan_recode": (C.c_int, [C.c_int, C.POINTER(gf_recode_desc), C.c_int, C.POINTER(gf_tuning),
                                 C.POINTER(C.c_void_p)]),
}

#: every symbol the header declares
EXPORTS = tuple(_SIGS)


def lib():
    """Load ``libgfnc.so`` (building it first only if it does not exist)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().gf_strerror(code).decode()


def _check(rc: int, what: str):
    if rc != GF_OK:
        raise GFError(rc, what)


# ------------------------------------------------------------------ helpers

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("gfnc needs a ROCm GPU; torch.cuda.is_available() is False")
    return torch


def _stream(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev_u8(t, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.uint8:
        raise TypeError("%s must be a CUDA uint8 tensor" % name)
    return t


def _rank_ptr(d_rank, count: int, name: str = "d_rank"):
    """Device pointer of an int32 CUDA tensor with at least `count` entries, or None."""
    if d_rank is None:
        return None
    torch = _torch()
    if not isinstance(d_rank, torch.Tensor) or d_rank.device.type != "cuda" or d_rank.dtype != torch.int32:
        raise TypeError("%s must be a CUDA int32 tensor" % name)
    if not d_rank.is_contiguous() or d_rank.numel() < count:
        raise ValueError("%s must be contiguous with at least %d entries" % (name, count))
    return d_rank.data_ptr()


def _rows(t, name: str) -> Tuple[int, int, int]:
    """(rows, row length, leading dimension in bytes) of a 2-D uint8 tensor with unit inner stride."""
    _dev_u8(t, name)
    if t.dim() != 2 or (t.stride(1) != 1 and t.shape[1] > 1):
        raise ValueError("%s must be 2-D with contiguous rows" % name)
    return t.shape[0], t.shape[1], max(t.stride(0), t.shape[1])


# ------------------------------------------------------------------ API

def gf_init():
    _torch()
    _check(lib().gf_init(), "gf_init")


def gf_region_madd(field: int, y, x, c: int, length: Optional[int] = None, stream=None):
    """y += c * x over ``length`` bytes (default: all of x). In place on y."""
    _dev_u8(y, "y"); _dev_u8(x, "x")
    n = x.numel() if length is None else length
    if n > x.numel() or n > y.numel():
        raise ValueError("length exceeds a buffer")
    _check(lib().gf_region_madd(field, y.data_ptr(), x.data_ptr(), c, n, _stream(stream)), "gf_region_madd")


def gf_region_mul(field: int, y, x, c: int, length: Optional[int] = None, stream=None):
    """y = c * x over ``length`` bytes (default: all of x)."""
    _dev_u8(y, "y"); _dev_u8(x, "x")
    n = x.numel() if length is None else length
    if n > x.numel() or n > y.numel():
        raise ValueError("length exceeds a buffer")
    _check(lib().gf_region_mul(field, y.data_ptr(), x.data_ptr(), c, n, _stream(stream)), "gf_region_mul")


def make_regions(regions: Sequence[Tuple[int, int, int, int]]):
    """Device descriptor array for gf_region_madd_batched from (y_ptr, x_ptr, len, c) tuples."""
    torch = _torch()
    arr = (gf_region * len(regions))()
    for i, (yp, xp, n, c) in enumerate(regions):
        arr[i] = gf_region(yp, xp, n, c, 0)
    host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
    return host.to("cuda")


def gf_region_madd_batched(field: int, d_regions, count: int, max_len: int, stream=None):
    _dev_u8(d_regions, "d_regions")
    if d_regions.numel() < count * C.sizeof(gf_region):
        raise ValueError("descriptor buffer too small")
    _check(lib().gf_region_madd_batched(field, d_regions.data_ptr(), count, max_len, _stream(stream)),
           "gf_region_madd_batched")


def gf_encode(field: int, Cm, S, Y, length: Optional[int] = None, stream=None):
    """Y[:K, :length] = Cm (K x N) * S (N rows) over GF(2^field)."""
    K, N, _ = _rows(Cm, "C")
    if not Cm.is_contiguous():
        raise ValueError("C must be contiguous")
    nS, lS, ld_s = _rows(S, "S")
    nY, lY, ld_y = _rows(Y, "Y")
    L = min(lS, lY) if length is None else length
    if nS < N or nY < K or L > lS or L > lY:
        raise ValueError("shape mismatch")
    _check(lib().gf_encode(field, Cm.data_ptr(), K, N, S.data_ptr(), ld_s, Y.data_ptr(), ld_y, L,
                           _stream(stream)), "gf_encode")


def gf_decode_workspace(field: int, max_N: int, count: int = 1) -> int:
    return int(lib().gf_decode_workspace(field, max_N, count))


def gf_decode(field: int, Cm, B, S, ws=None, d_rank=None, length: Optional[int] = None, stream=None):
    """S = Cm^-1 B (enqueued; S untouched if Cm is singular). d_rank: CUDA int32 tensor of 1 or None."""
    torch = _torch()
    N, N2, _ = _rows(Cm, "C")
    if N != N2 or not Cm.is_contiguous():
        raise ValueError("C must be a contiguous N x N matrix")
    nB, lB, ld_b = _rows(B, "B")
    nS, lS, ld_s = _rows(S, "S")
    L = min(lB, lS) if length is None else length
    if nB < N or nS < N or L > lB or L > lS:
        raise ValueError("shape mismatch")
    if ws is None:
        ws = torch.empty(gf_decode_workspace(field, N), dtype=torch.uint8, device=Cm.device)
    _dev_u8(ws, "ws")
    if not ws.is_contiguous():
        raise ValueError("ws must be contiguous")
    rp = _rank_ptr(d_rank, 1)
    _check(lib().gf_decode(field, Cm.data_ptr(), B.data_ptr(), ld_b, N, S.data_ptr(), ld_s, L, ws.data_ptr(),
                           ws.numel(), rp, _stream(stream)), "gf_decode")
    return ws


def gf_decode_noalloc(field: int, Cm, B, S, d_rank=None, length: Optional[int] = None, stream=None):
    """gf_decode with the library's fixed device scratch instead of a workspace (allocates nothing)."""
    N, N2, _ = _rows(Cm, "C")
    if N != N2 or not Cm.is_contiguous():
        raise ValueError("C must be a contiguous N x N matrix")
    nB, lB, ld_b = _rows(B, "B")
    nS, lS, ld_s = _rows(S, "S")
    L = min(lB, lS) if length is None else length
    if nB < N or nS < N or L > lB or L > lS:
        raise ValueError("shape mismatch")
    rp = _rank_ptr(d_rank, 1)
    _check(lib().gf_decode_noalloc(field, Cm.data_ptr(), B.data_ptr(), ld_b, N, S.data_ptr(), ld_s, L, rp,
                                   _stream(stream)), "gf_decode_noalloc")


def gf_invert(field: int, Cm, Cinv, d_rank=None, stream=None):
    N, N2, _ = _rows(Cm, "C")
    _dev_u8(Cinv, "Cinv")
    if N != N2 or not Cm.is_contiguous() or not Cinv.is_contiguous() or tuple(Cinv.shape) != (N, N):
        raise ValueError("C and Cinv must be contiguous N x N matrices")
    rp = _rank_ptr(d_rank, 1)
    _check(lib().gf_invert(field, Cm.data_ptr(), N, Cinv.data_ptr(), rp, _stream(stream)), "gf_invert")


def _tuning(t: Optional[dict]):
    if t is None:
        return None
    return C.byref(gf_tuning(t.get("form", 0), t.get("bytes_per_lane", 0), t.get("grid_blocks", 0), 0))


class Plan:
    """A batched plan (encode, recode or decode) over many uneven generations."""

    def __init__(self, handle: int, kind: str, count: int, keep, field: int = 0):
        self._h = C.c_void_p(handle)
        self.kind = kind
        self.count = count
        self.field = field
        self._keep = keep   # tensors the plan points into

    def errors(self) -> int:
        """Descriptors gf_encode_batched skipped since the last call (synchronises)."""
        v = C.c_uint64()
        _check(lib().gf_plan_errors(self._h, C.byref(v)), "gf_plan_errors")
        return int(v.value)

    def tuning(self) -> dict:
        t = gf_tuning()
        _check(lib().gf_plan_tuning(self._h, C.byref(t)), "gf_plan_tuning")
        return {"form": t.form, "bytes_per_lane": t.bytes_per_lane, "grid_blocks": t.grid_blocks}

    def destroy(self):
        if self._h:
            lib().gf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _gen_desc(Cm, S, Y, length=None) -> gf_gen:
    K, N, _ = _rows(Cm, "C")
    nS, lS, ld_s = _rows(S, "S")
    nY, lY, ld_y = _rows(Y, "Y")
    L = min(lS, lY) if length is None else length
    if nS < N or nY < K or L > lS or L > lY or not Cm.is_contiguous():
        raise ValueError("shape mismatch")
    return gf_gen(Cm.data_ptr(), S.data_ptr(), Y.data_ptr(), K, N, L, ld_s, ld_y)


def gf_plan_encode(field: int, gens: Sequence[tuple], tune: Optional[dict] = None) -> Plan:
    """gens: (C, S, Y) or (C, S, Y, length) tensors per generation."""
    arr = (gf_gen * len(gens))(*[_gen_desc(*g) for g in gens])
    h = C.c_void_p()
    _check(lib().gf_plan_encode(field, arr, len(gens), _tuning(tune), C.byref(h)), "gf_plan_encode")
    return Plan(h.value, "encode", len(gens), list(gens), field)


def gf_plan_encode_desc(field: int, arr, count: int, tune: Optional[dict] = None, keep=None) -> Plan:
    """Plan from a ctypes array of gf_gen built by the caller."""
    h = C.c_void_p()
    _check(lib().gf_plan_encode(field, arr, count, _tuning(tune), C.byref(h)), "gf_plan_encode")
    return Plan(h.value, "encode", count, keep, field)


def gf_plan_decode(field: int, systems: Sequence[tuple], tune: Optional[dict] = None) -> Plan:
    """systems: (C, B, S) or (C, B, S, length) tensors per system."""
    descs = []
    for s in systems:
        Cm, B, S = s[:3]
        length = s[3] if len(s) > 3 else None
        N, N2, _ = _rows(Cm, "C")
        nB, lB, ld_b = _rows(B, "B")
        nS, lS, ld_s = _rows(S, "S")
        L = min(lB, lS) if length is None else length
        if N != N2 or nB < N or nS < N or L > lB or L > lS or not Cm.is_contiguous():
            raise ValueError("shape mismatch")
        descs.append(gf_sys(Cm.data_ptr(), B.data_ptr(), S.data_ptr(), N, 0, L, ld_b, ld_s))
    return gf_plan_decode_desc(field, (gf_sys * len(descs))(*descs), len(descs), tune, list(systems))


def gf_plan_decode_desc(field: int, arr, count: int, tune: Optional[dict] = None, keep=None) -> Plan:
    h = C.c_void_p()
    _check(lib().gf_plan_decode(field, arr, count, _tuning(tune), C.byref(h)), "gf_plan_decode")
    return Plan(h.value, "decode", count, keep, field)


def _device_array(arr, name: str):
    """A ctypes array of descriptors copied into a CUDA uint8 tensor."""
    torch = _torch()
    return torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to("cuda")


def make_gens(arr):
    """Device copy of a ctypes array of gf_gen (for gf_encode_batched)."""
    return _device_array(arr, "gens")


def make_systems(arr):
    """Device copy of a ctypes array of gf_sys (for gf_decode_batched)."""
    return _device_array(arr, "systems")


def gf_encode_batched(field: int, d_gens, count: int, plan: Plan, stream=None):
    """Encode the generations of the device descriptor array d_gens (a CUDA uint8 tensor of
    ``count`` gf_gen, e.g. from make_gens; None: the plan's own) with the plan's schedule."""
    if d_gens is not None:
        _dev_u8(d_gens, "d_gens")
        if not d_gens.is_contiguous() or d_gens.numel() < count * C.sizeof(gf_gen):
            raise ValueError("d_gens must be contiguous with %d descriptors" % count)
    _check(lib().gf_encode_batched(field, None if d_gens is None else d_gens.data_ptr(), count, plan._h,
                                   _stream(stream)), "gf_encode_batched")


def gf_decode_batched(field: int, d_sys, count: int, d_rank=None, ws=None, max_N: int = GF_MAX_N, stream=None):
    """Decode the systems of the device descriptor array d_sys (a CUDA uint8 tensor of ``count``
    gf_sys, e.g. from make_systems), no plan; ws: CUDA uint8 workspace (allocated for max_N if None).
    Returns the workspace."""
    torch = _torch()
    _dev_u8(d_sys, "d_sys")
    if not d_sys.is_contiguous() or d_sys.numel() < count * C.sizeof(gf_sys):
        raise ValueError("d_sys must be contiguous with %d descriptors" % count)
    if ws is None:
        ws = torch.empty(max(1, gf_decode_workspace(field, max_N, max(count, 1))), dtype=torch.uint8,
                         device=d_sys.device)
    _dev_u8(ws, "ws")
    if not ws.is_contiguous():
        raise ValueError("ws must be contiguous")
    rp = _rank_ptr(d_rank, count)
    _check(lib().gf_decode_batched(field, d_sys.data_ptr(), count, rp, ws.data_ptr(), ws.numel(),
                                   _stream(stream)), "gf_decode_batched")
    return ws


def gf_plan_launch(plan: Plan, d_rank=None, stream=None):
    """Run a plan on the descriptors it was made with (d_rank: decode plans)."""
    rp = _rank_ptr(d_rank, plan.count) if plan.kind == "decode" else None
    _check(lib().gf_plan_launch(plan._h, rp, _stream(stream)), "gf_plan_launch")


def gf_plan_launch_graph(plan: Plan, d_rank=None, stream=None):
    rp = _rank_ptr(d_rank, plan.count) if plan.kind == "decode" else None
    _check(lib().gf_plan_launch_graph(plan._h, rp, _stream(stream)), "gf_plan_launch_graph")


def gf_ceiling(what: int, buf, blocks: int, iters: int, stream=None):
    """Diagnostic microbenchmark (0 copy, 1 table step, 2 FP4 MFMA, 3 bit-plane step, 4 copy by
    16 KiB chunks) on the CUDA uint8 tensor ``buf`` (enqueued; time it with events)."""
    _dev_u8(buf, "buf")
    _check(lib().gf_ceiling(what, buf.data_ptr(), buf.numel(), blocks, iters, _stream(stream)), "gf_ceiling")


def gf_encode_each(field: int, gens, count: Optional[int] = None, tune: Optional[dict] = None, stream=None):
    """Per-generation launches (unbatched baseline). gens: ctypes gf_gen array or tensor tuples."""
    if not isinstance(gens, C.Array):
        gens = (gf_gen * len(gens))(*[_gen_desc(*g) for g in gens])
    n = len(gens) if count is None else count
    _check(lib().gf_encode_each(field, gens, n, _tuning(tune), _stream(stream)), "gf_encode_each")


# ------------------------------------------------------------------ serving

def _recode_desc(R, Cin, Bin, Cout, Yout, length=None) -> gf_recode_desc:
    """Rows may be views into larger buffers (e.g. packets stored as [coefficients | payload] rows)."""
    Kout, M, _ = _rows(R, "R")
    M2, N, ld_cin = _rows(Cin, "Cin")
    K2, N2, ld_cout = _rows(Cout, "Cout")
    nB, lB, ld_b = _rows(Bin, "Bin")
    nY, lY, ld_y = _rows(Yout, "Yout")
    L = min(lB, lY) if length is None else length
    if not R.is_contiguous():
        raise ValueError("R must be contiguous")
    if M2 < M or K2 < Kout or N2 != N or nB < M or nY < Kout or L > lB or L > lY:
        raise ValueError("shape mismatch")
    return gf_recode_desc(R.data_ptr(), Cin.data_ptr(), Bin.data_ptr(), Cout.data_ptr(), Yout.data_ptr(), Kout, M,
                          N, 0, L, ld_cin, ld_b, ld_cout, ld_y)


def gf_recode(field: int, R, Cin, Bin, Cout, Yout, length: Optional[int] = None, stream=None):
    """Cout = R * Cin and Yout[:, :length] = R * Bin over GF(2^field) (recoding received packets)."""
    d = _recode_desc(R, Cin, Bin, Cout, Yout, length)
    _check(lib().gf_recode(field, d.R, d.Kout, d.M, d.N, d.Cin, d.ld_cin, d.Bin, d.ld_b, d.Cout, d.ld_cout, d.Yout,
                           d.ld_y, d.len, _stream(stream)), "gf_recode")


def gf_plan_recode(field: int, items: Sequence[tuple], tune: Optional[dict] = None) -> Plan:
    """items: (R, Cin, Bin, Cout, Yout) or (..., length) tensors per recoding; run with
    gf_encode_batched or gf_plan_launch_graph."""
    arr = (gf_recode_desc * len(items))(*[_recode_desc(*it) for it in items])
    h = C.c_void_p()
    _check(lib().gf_plan_recode(field, arr, len(items), _tuning(tune), C.byref(h)), "gf_plan_recode")
    return Plan(h.value, "recode", len(items), list(items))


def gf_plan_recode_desc(field: int, arr, count: int, tune: Optional[dict] = None, keep=None) -> Plan:
    """Recode plan from a ctypes array of gf_recode_desc built by the caller."""
    h = C.c_void_p()
    _check(lib().gf_plan_recode(field, arr, count, _tuning(tune), C.byref(h)), "gf_plan_recode")
    return Plan(h.value, "recode", count, keep)


class gf_serve_config(C.Structure):
    _fields_ = [("field", C.c_int), ("max_slots", C.c_int), ("burst", C.c_int), ("dry_run", C.c_int),
                ("budget_bytes", C.c_uint64)]


class gf_serve_done(C.Structure):
    _fields_ = [("id", C.c_uint64), ("kind", C.c_int), ("status", C.c_int), ("rank", C.c_int),
                ("packets_seen", C.c_int), ("packets_dropped", C.c_int), ("out", C.c_void_p),
                ("ld_out", C.c_uint64), ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class gf_serve_status(C.Structure):
    _fields_ = [("state", C.c_int), ("rank", C.c_int), ("packets_pending", C.c_int), ("packets_seen", C.c_int),
                ("packets_dropped", C.c_int)]


class gf_serve_counters(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("steps", "submitted", "admitted", "completed", "queued", "active",
                                           "inflight_steps", "arena_bytes", "arena_used", "arena_peak",
                                           "packets_pushed", "packets_absorbed", "encode_tiles", "absorb_items")]


_SERVE_SIGS = {
    "gf_serve_create": (C.c_int, [C.POINTER(gf_serve_config), C.POINTER(C.c_void_p)]),
    "gf_serve_destroy": (None, [C.c_void_p]),
    "gf_serve_submit_encode": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_int, C.c_int, C.c_void_p,
                                         C.c_size_t, C.c_size_t, C.c_double]),
    "gf_serve_submit_decode": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int, C.c_size_t, C.c_double]),
    "gf_serve_push_packet": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_double]),
    "gf_serve_push_packets": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gf_serve_step": (C.c_int, [C.c_void_p, C.c_double]),
    "gf_serve_poll": (C.c_int, [C.c_void_p, C.POINTER(gf_serve_done), C.c_int]),
    "gf_serve_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "gf_serve_copy_out": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_size_t, C.c_void_p]),
    "gf_serve_cancel": (C.c_int, [C.c_void_p, C.c_uint64, C.c_double]),
    "gf_serve_query": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(gf_serve_status)]),
    "gf_serve_drain": (C.c_int, [C.c_void_p, C.c_double]),
    "gf_serve_stats": (C.c_int, [C.c_void_p, C.POINTER(gf_serve_counters)]),
}
_SIGS.update(_SERVE_SIGS)
EXPORTS = tuple(_SIGS)


class Server:
    """The serving runtime (``gf_serve_*``): continuous batching of encode and
    progressive-decode requests in one device arena.

    Inputs are device pointers (ints) or CUDA uint8 tensors; outputs are
    device pointers into the server's arena, valid until ``release``.
    ``dry_run=True`` runs the scheduler only (no GPU needed)."""

    def __init__(self, field: int = GF_256, budget_bytes: int = 1 << 30, max_slots: int = 0, burst: int = 0,
                 dry_run: bool = False):
        if not dry_run:
            _torch()
        cfg = gf_serve_config(field, max_slots, burst, 1 if dry_run else 0, budget_bytes)
        h = C.c_void_p()
        _check(lib().gf_serve_create(C.byref(cfg), C.byref(h)), "gf_serve_create")
        self._h = h
        self.field = field
        self._buf = (gf_serve_done * 1024)()
        self._shape = {}   # request id -> (output rows, bytes per row)

    @staticmethod
    def _ptr(x):
        if hasattr(x, "data_ptr"):
            if getattr(x, "device", None) is None or x.device.type != "cuda":
                raise TypeError("server inputs must be CUDA tensors or device pointers")
            return x.data_ptr()
        return int(x)

    def submit_encode(self, rid: int, Cm, S, K: int, N: int, ld_s: int, length: int, now: float):
        _check(lib().gf_serve_submit_encode(self._h, rid, self._ptr(Cm), K, N, self._ptr(S), ld_s, length, now),
               "gf_serve_submit_encode")
        self._shape[rid] = (K, length)

    def submit_decode(self, rid: int, N: int, length: int, now: float):
        _check(lib().gf_serve_submit_decode(self._h, rid, N, length, now), "gf_serve_submit_decode")
        self._shape[rid] = (N, length)

    def push_packet(self, rid: int, coef, payload, release: float):
        _check(lib().gf_serve_push_packet(self._h, rid, self._ptr(coef), self._ptr(payload), release),
               "gf_serve_push_packet")

    def push_packets(self, rid: int, coefs, payloads, releases):
        """Push many packets: sequences of device pointers and release times."""
        import numpy as np
        c = np.ascontiguousarray(np.asarray(coefs, dtype=np.uint64))
        p = np.ascontiguousarray(np.asarray(payloads, dtype=np.uint64))
        r = np.ascontiguousarray(np.asarray(releases, dtype=np.float64))
        if not (c.size == p.size == r.size):
            raise ValueError("length mismatch")
        _check(lib().gf_serve_push_packets(self._h, rid, int(c.size), c.ctypes.data, p.ctypes.data, r.ctypes.data),
               "gf_serve_push_packets")

    def step(self, now: float) -> int:
        rc = lib().gf_serve_step(self._h, now)
        if rc < 0:
            raise GFError(rc, "gf_serve_step")
        return rc

    def poll(self) -> List[dict]:
        out = []
        while True:
            n = lib().gf_serve_poll(self._h, self._buf, len(self._buf))
            if n < 0:
                raise GFError(n, "gf_serve_poll")
            for i in range(n):
                d = self._buf[i]
                out.append({"id": d.id, "kind": "encode" if d.kind == 0 else "decode", "status": d.status,
                            "rank": d.rank, "packets_seen": d.packets_seen, "packets_dropped": d.packets_dropped,
                            "out": d.out, "ld_out": d.ld_out, "t_submit": d.t_submit, "t_admit": d.t_admit,
                            "t_done": d.t_done})
            if n < len(self._buf):
                return out

    def release(self, rid: int):
        _check(lib().gf_serve_release(self._h, rid), "gf_serve_release")
        self._shape.pop(rid, None)

    def query(self, rid: int) -> dict:
        """State (0 queued, 1 admitted, 2 completed), rank so far and packet counts of a request."""
        st = gf_serve_status()
        _check(lib().gf_serve_query(self._h, rid, C.byref(st)), "gf_serve_query")
        return {"state": st.state, "rank": st.rank, "packets_pending": st.packets_pending,
                "packets_seen": st.packets_seen, "packets_dropped": st.packets_dropped}

    def cancel(self, rid: int, now: float):
        """Give up on a request that has not completed (polled later with status GF_ECANCELED)."""
        _check(lib().gf_serve_cancel(self._h, rid, now), "gf_serve_cancel")

    def copy_out(self, rid: int, dst, stream=None):
        """Copy a completed request's output rows into the 2-D CUDA uint8 tensor `dst`
        (enqueued on `stream`, default torch's current stream)."""
        _dev_u8(dst, "dst")
        rows, length = self._shape.get(rid, (0, 0))
        if dst.dim() != 2 or (dst.stride(1) != 1 and dst.shape[1] > 1) or dst.shape[0] < rows or dst.shape[1] < length:
            raise ValueError("dst must be 2-D with contiguous rows, at least %d x %d" % (rows, length))
        _check(lib().gf_serve_copy_out(self._h, rid, dst.data_ptr(), max(dst.stride(0), dst.shape[1]),
                                       _stream(stream)), "gf_serve_copy_out")

    def drain(self, now: float):
        _check(lib().gf_serve_drain(self._h, now), "gf_serve_drain")

    def stats(self) -> dict:
        c = gf_serve_counters()
        _check(lib().gf_serve_stats(self._h, C.byref(c)), "gf_serve_stats")
        return {n: getattr(c, n) for n, _ in gf_serve_counters._fields_}

    def close(self):
        if self._h:
            lib().gf_serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
