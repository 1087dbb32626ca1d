"""Thin ctypes binding of ``libhntt.so`` (the C ABI in include/hntt.h).

Argument marshalling only: every step of a transform runs in the library's
HIP kernels.  PyTorch provides device memory (tensors on ``cuda``, i.e. HIP on
ROCm) and streams.  Tensors hold unsigned words: ``torch.uint32``/``int32``
for 32-bit words, ``torch.uint64``/``int64`` for 64-bit words (the bits are
read as unsigned).

If the library has not been built, loading raises ``HnttNotBuilt``; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# HNTT_LIB: another build of the library (e.g. one with sanitized host code)
LIB_PATH = os.environ.get("HNTT_LIB") or os.path.join(_HERE, "libhntt.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE, EBUSY = 0, -1, -2, -3, -4, -5
PLAIN = 0x1
NO_NORMALIZE = 0x2
NO_GRAPH = 0x4
MONT = 0x8
VALIDATE = 0x10
STATIC_SCRATCH_BYTES = 32 << 20  # HNTT_STATIC_SCRATCH_BYTES
POLICY_FLAGS = {"lazy": 0, "plain": PLAIN, "mont": MONT}

_c_u64 = ctypes.c_uint64
_c_u32 = ctypes.c_uint32
_c_vp = ctypes.c_void_p


class HnttNotBuilt(RuntimeError):
    pass


class HnttError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"hntt error {status}: {message}")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("p", _c_u64), ("omega", _c_u64), ("data", _c_vp), ("log2_len", _c_u32), ("word_bits", _c_u32)]


class PwDesc(ctypes.Structure):
    _fields_ = [("p", _c_u64), ("a", _c_vp), ("b", _c_vp), ("c", _c_vp), ("len", _c_u64), ("word_bits", _c_u32),
                ("reserved", _c_u32)]


class Tuning(ctypes.Structure):
    _fields_ = [("log2_len", _c_u32), ("word_bits", _c_u32), ("g_cols", _c_u32), ("g_rows", _c_u32),
                ("batch_chunk", _c_u32), ("row_log2", _c_u32), ("g_rows_inv", _c_u32)]


class PolyDesc(ctypes.Structure):
    _fields_ = [("a", _c_vp), ("b", _c_vp), ("out", _c_vp), ("na", _c_u32), ("nb", _c_u32)]


class BigmulDesc(ctypes.Structure):
    _fields_ = [("a", _c_vp), ("b", _c_vp), ("out", _c_vp), ("na", _c_u32), ("nb", _c_u32)]


#: every function include/hntt.h declares, with its ctypes signature
SIGNATURES = {
    "hntt_create": (ctypes.c_int, [ctypes.POINTER(_c_vp), ctypes.c_int, ctypes.c_size_t]),
    "hntt_destroy": (None, [_c_vp]),
    "hntt_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "hntt_last_error": (ctypes.c_char_p, [_c_vp]),
    "hntt_ntt_forward": (ctypes.c_int, [_c_vp, ctypes.POINTER(Desc), ctypes.c_size_t, _c_u32, _c_vp]),
    "hntt_ntt_inverse": (ctypes.c_int, [_c_vp, ctypes.POINTER(Desc), ctypes.c_size_t, _c_u32, _c_vp]),
    "hntt_pointwise_mul": (ctypes.c_int, [_c_vp, ctypes.POINTER(PwDesc), ctypes.c_size_t, _c_u32, _c_vp]),
    "hntt_polymul_crt": (ctypes.c_int, [_c_vp, ctypes.POINTER(PolyDesc), ctypes.c_size_t, _c_u32, _c_vp]),
    "hntt_polymul_crt_static": (ctypes.c_int, [_c_vp, ctypes.POINTER(PolyDesc), ctypes.c_size_t, _c_u32, _c_vp]),
    "hntt_polymul_plan_create": (ctypes.c_int, [_c_vp, ctypes.POINTER(PolyDesc), ctypes.c_size_t, _c_u32, _c_vp,
                                                ctypes.c_size_t, _c_vp, ctypes.POINTER(_c_vp)]),
    "hntt_polymul_plan_workspace_bytes": (ctypes.c_size_t, [_c_vp]),
    "hntt_polymul_plan_exec_mode": (ctypes.c_int, [_c_vp, ctypes.POINTER(ctypes.c_char_p)]),
    "hntt_polymul_plan_execute": (ctypes.c_int, [_c_vp, _c_vp, _c_vp]),
    "hntt_polymul_workspace_size": (ctypes.c_int, [ctypes.POINTER(PolyDesc), ctypes.c_size_t,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "hntt_polymul_plan_destroy": (None, [_c_vp]),
    "hntt_bigmul": (ctypes.c_int, [_c_vp, ctypes.POINTER(BigmulDesc), ctypes.c_size_t, _c_u32, _c_vp]),
    "hntt_bigmul_plan_create": (ctypes.c_int, [_c_vp, ctypes.POINTER(BigmulDesc), ctypes.c_size_t, _c_u32, _c_vp,
                                               ctypes.c_size_t, _c_vp, ctypes.POINTER(_c_vp)]),
    "hntt_bigmul_workspace_size": (ctypes.c_int, [ctypes.POINTER(BigmulDesc), ctypes.c_size_t,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "hntt_is_prime": (ctypes.c_int, [_c_u64]),
    "hntt_primitive_root": (_c_u64, [_c_u64]),
    "hntt_root_of_unity": (ctypes.c_int, [_c_u64, _c_u32, ctypes.POINTER(_c_u64)]),
    "hntt_find_prime": (_c_u64, [_c_u32, _c_u32]),
    "hntt_shoup_constant": (ctypes.c_int, [_c_u64, _c_u64, _c_u32, ctypes.POINTER(_c_u64)]),
    "hntt_validate": (ctypes.c_int, [_c_vp, ctypes.POINTER(Desc), ctypes.c_size_t, _c_u32]),
    "hntt_set_tuning": (ctypes.c_int, [_c_vp, ctypes.POINTER(Tuning)]),
    "hntt_get_plan": (ctypes.c_int, [_c_vp, _c_u32, _c_u32, ctypes.POINTER(Tuning)]),
    "hntt_trace_enable": (ctypes.c_int, [_c_vp, ctypes.c_int]),
    "hntt_trace_read": (ctypes.c_int, [_c_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_size_t)]),
    "hntt_trace_reset": (ctypes.c_int, [_c_vp]),
    "hntt_debug_butterfly": (ctypes.c_int, [_c_vp, ctypes.c_int, _c_u32, _c_u64, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                            _c_vp, ctypes.c_size_t, _c_vp]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the built library (once).  Raises HnttNotBuilt when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HnttNotBuilt(f"{path} is missing: build it with `python -m paper_1205_2926_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


# ------------------------------------------------------------------------------------------------
# host number theory (no GPU needed)
def is_prime(n: int) -> bool:
    return bool(load().hntt_is_prime(n))


def primitive_root(p: int) -> int:
    return int(load().hntt_primitive_root(p))


def root_of_unity(p: int, log2_len: int) -> int:
    out = _c_u64()
    rc = load().hntt_root_of_unity(p, log2_len, ctypes.byref(out))
    if rc:
        raise HnttError(rc, f"no 2^{log2_len}-th root of unity mod {p}")
    return int(out.value)


def find_prime(bits: int, v: int) -> int:
    return int(load().hntt_find_prime(bits, v))


def shoup_constant(w: int, p: int, word_bits: int) -> int:
    out = _c_u64()
    rc = load().hntt_shoup_constant(w, p, word_bits, ctypes.byref(out))
    if rc:
        raise HnttError(rc, "bad Shoup constant arguments")
    return int(out.value)


def bigmul_workspace_size(lengths: Sequence[tuple[int, int]]) -> int:
    """Workspace bytes of a large-integer product plan for (na, nb) limb counts (host only)."""
    arr = (BigmulDesc * len(lengths))()
    for i, (na, nb) in enumerate(lengths):
        arr[i] = BigmulDesc(None, None, None, na, nb)
    out = ctypes.c_size_t(0)
    rc = load().hntt_bigmul_workspace_size(arr, len(lengths), ctypes.byref(out))
    if rc:
        raise HnttError(rc, "bad bigmul lengths")
    return int(out.value)


def polymul_workspace_size(lengths: Sequence[tuple[int, int]]) -> int:
    """Workspace bytes of a polymul plan for products of (na, nb) coefficients (host only)."""
    arr = (PolyDesc * len(lengths))()
    for i, (na, nb) in enumerate(lengths):
        arr[i] = PolyDesc(None, None, None, na, nb)
    out = ctypes.c_size_t(0)
    rc = load().hntt_polymul_workspace_size(arr, len(lengths), ctypes.byref(out))
    if rc:
        raise HnttError(rc, "bad polymul lengths")
    return int(out.value)


def strerror(status: int) -> str:
    return load().hntt_strerror(status).decode()


# ------------------------------------------------------------------------------------------------
def _word_bits(t: torch.Tensor) -> int:
    es = t.element_size()
    if es not in (4, 8) or t.dtype.is_floating_point or t.dtype.is_complex:
        raise TypeError(f"expected a 32- or 64-bit integer tensor, got {t.dtype}")
    return es * 8


def _stream_handle(stream, device) -> int:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


class PolymulPlan:
    """A planned batch of products (hntt_polymul_plan_*); execute() enqueues it, destroy() frees it."""

    def __init__(self, ctx, pairs, outs, plain, graph, workspace, stream, big=False):
        self.ctx = ctx
        self.arr = ctx.bigmul_descs(pairs, outs) if big else ctx.poly_descs(pairs, outs)
        self.keep = (list(pairs), list(outs), workspace)
        flags = (PLAIN if plain else 0) | (0 if graph else NO_GRAPH)
        h = _c_vp()
        dev = outs[0].device if outs else torch.device("cuda", ctx.device)
        ws_ptr = workspace.data_ptr() if workspace is not None else None
        ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
        create = ctx.lib.hntt_bigmul_plan_create if big else ctx.lib.hntt_polymul_plan_create
        ctx._check(create(ctx.handle, self.arr, len(pairs), flags, ws_ptr, ws_bytes, _stream_handle(stream, dev),
                          ctypes.byref(h)))
        self.handle = h
        self.device = dev

    @property
    def workspace_bytes(self) -> int:
        return int(self.ctx.lib.hntt_polymul_plan_workspace_bytes(self.handle))

    def execute(self, stream=None):
        self.ctx._check(self.ctx.lib.hntt_polymul_plan_execute(self.ctx.handle, self.handle,
                                                               _stream_handle(stream, self.device)))

    EXEC_MODES = {0: "not executed", 1: "graph", 2: "direct", 3: "direct (graph capture failed)"}

    @property
    def exec_mode(self) -> str:
        """How the last execution was enqueued: graph, direct, or direct after a failed capture (with
        the reason)."""
        msg = ctypes.c_char_p()
        mode = int(self.ctx.lib.hntt_polymul_plan_exec_mode(self.handle, ctypes.byref(msg)))
        text = self.EXEC_MODES.get(mode, str(mode))
        if mode == 3 and msg.value:
            text += ": " + msg.value.decode()
        return text

    def destroy(self):
        if getattr(self, "handle", None):
            self.ctx.lib.hntt_polymul_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Context:
    """A library context bound to one HIP device (twiddle tables and workspaces live here)."""

    def __init__(self, device: int = 0, mem_budget: int = 0):
        self.lib = load()
        self.device = device
        h = _c_vp()
        rc = self.lib.hntt_create(ctypes.byref(h), device, mem_budget)
        if rc:
            raise HnttError(rc, "hntt_create failed")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.hntt_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self.lib.hntt_last_error(self.handle).decode()

    def _check(self, rc: int):
        if rc:
            raise HnttError(rc, self.last_error() or strerror(rc))

    # -- descriptor helpers ----------------------------------------------------------------------
    @staticmethod
    def descs(rows: Iterable[torch.Tensor], p: int, omega: int, log2_len: int | None = None):
        rows = list(rows)
        arr = (Desc * len(rows))()
        for i, t in enumerate(rows):
            wb = _word_bits(t)
            l = log2_len if log2_len is not None else (t.numel().bit_length() - 1)
            arr[i] = Desc(p, omega, t.data_ptr(), l, wb)
        return arr

    @staticmethod
    def rows_of(x: torch.Tensor) -> list[torch.Tensor]:
        """Rows of a [batch, L] (or [L]) contiguous tensor as separate transforms."""
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return [x] if x.dim() == 1 else list(x.reshape(-1, x.shape[-1]).unbind(0))

    # -- transforms --------------------------------------------------------------------------------
    def ntt_forward(self, x, p: int, omega: int, plain: bool = False, normalize: bool = True, stream=None,
                    mont: bool = False, validate: bool = False):
        """In-place forward NTT of every row of x (natural in, bit-reversed out).  plain selects
        Algorithm 2, mont Algorithm 5; the default is Algorithm 3.  validate checks on the
        device that every input word is below p first (HNTT_VALIDATE)."""
        self._transform(self.lib.hntt_ntt_forward, x, p, omega, plain, normalize, stream, mont, validate)
        return x

    def ntt_inverse(self, x, p: int, omega: int, plain: bool = False, normalize: bool = True, stream=None,
                    mont: bool = False, validate: bool = False):
        """In-place inverse NTT of every row of x (bit-reversed in, natural out, times L^-1)."""
        self._transform(self.lib.hntt_ntt_inverse, x, p, omega, plain, normalize, stream, mont, validate)
        return x

    def _transform(self, fn, x, p, omega, plain, normalize, stream, mont=False, validate=False):
        rows = self.rows_of(x) if isinstance(x, torch.Tensor) else list(x)
        arr = self.descs(rows, p, omega)
        flags = ((PLAIN if plain else 0) | (MONT if mont else 0) | (0 if normalize else NO_NORMALIZE) |
                 (VALIDATE if validate else 0))
        dev = rows[0].device if rows else torch.device("cuda", self.device)
        self._check(fn(self.handle, arr, len(rows), flags, _stream_handle(stream, dev)))

    def ntt_descs(self, fn_name: str, arr, flags: int = 0, stream=None):
        """Call hntt_ntt_forward/inverse with a prebuilt descriptor array."""
        fn = getattr(self.lib, fn_name)
        self._check(fn(self.handle, arr, len(arr), flags, _stream_handle(stream, torch.device("cuda", self.device))))

    def validate(self, arr, flags: int = 0) -> int:
        return int(self.lib.hntt_validate(self.handle, arr, len(arr), flags))

    def pointwise_mul(self, a: torch.Tensor, b: torch.Tensor, c: torch.Tensor, p: int, stream=None,
                      validate: bool = False):
        wb = _word_bits(a)
        d = (PwDesc * 1)(PwDesc(p, a.data_ptr(), b.data_ptr(), c.data_ptr(), a.numel(), wb, 0))
        self._check(self.lib.hntt_pointwise_mul(self.handle, d, 1, VALIDATE if validate else 0,
                                                _stream_handle(stream, a.device)))
        return c

    @staticmethod
    def poly_descs(pairs: Sequence[tuple[torch.Tensor, torch.Tensor]], outs: Sequence[torch.Tensor]):
        arr = (PolyDesc * len(pairs))()
        for i, ((a, b), o) in enumerate(zip(pairs, outs)):
            if a.element_size() != 4 or b.element_size() != 4 or o.element_size() != 8:
                raise TypeError("operands must be 32-bit and outputs 64-bit integer tensors")
            if o.numel() < a.numel() + b.numel() - 1:
                raise ValueError("output shorter than na + nb - 1")
            arr[i] = PolyDesc(a.data_ptr(), b.data_ptr(), o.data_ptr(), a.numel(), b.numel())
        return arr

    def polymul_crt(self, pairs: Sequence[tuple[torch.Tensor, torch.Tensor]], outs: Sequence[torch.Tensor],
                    plain: bool = False, graph: bool = True, stream=None):
        """Exact products out[i] = a_i * b_i (three primes + CRT), one call for the whole batch."""
        arr = self.poly_descs(pairs, outs)
        dev = outs[0].device if outs else torch.device("cuda", self.device)
        flags = (PLAIN if plain else 0) | (0 if graph else NO_GRAPH)
        self._check(self.lib.hntt_polymul_crt(self.handle, arr, len(pairs), flags, _stream_handle(stream, dev)))
        return outs

    def polymul_crt_static(self, pairs: Sequence[tuple[torch.Tensor, torch.Tensor]], outs: Sequence[torch.Tensor],
                           plain: bool = False, stream=None):
        """hntt_polymul_crt_static: the same products in the library's static device workspace
        (no device allocation; the twiddle tables of every length must already be resident)."""
        arr = self.poly_descs(pairs, outs)
        dev = outs[0].device if outs else torch.device("cuda", self.device)
        flags = PLAIN if plain else 0
        self._check(self.lib.hntt_polymul_crt_static(self.handle, arr, len(pairs), flags,
                                                     _stream_handle(stream, dev)))
        return outs

    def polymul_plan(self, pairs, outs, plain: bool = False, graph: bool = True, workspace: torch.Tensor = None,
                     stream=None) -> "PolymulPlan":
        return PolymulPlan(self, pairs, outs, plain, graph, workspace, stream)

    # -- large-integer products --------------------------------------------------------------------
    @staticmethod
    def bigmul_descs(pairs: Sequence[tuple[torch.Tensor, torch.Tensor]], outs: Sequence[torch.Tensor]):
        arr = (BigmulDesc * len(pairs))()
        for i, ((a, b), o) in enumerate(zip(pairs, outs)):
            if a.element_size() != 4 or b.element_size() != 4 or o.element_size() != 4:
                raise TypeError("limbs must be 32-bit integer tensors")
            if o.numel() < a.numel() + b.numel():
                raise ValueError("output shorter than na + nb limbs")
            arr[i] = BigmulDesc(a.data_ptr(), b.data_ptr(), o.data_ptr(), a.numel(), b.numel())
        return arr

    def bigmul(self, pairs: Sequence[tuple[torch.Tensor, torch.Tensor]], outs: Sequence[torch.Tensor],
               plain: bool = False, graph: bool = True, stream=None):
        """out[i] = a_i * b_i for integers given as little-endian base-2^32 limbs (int32 tensors)."""
        arr = self.bigmul_descs(pairs, outs)
        dev = outs[0].device if outs else torch.device("cuda", self.device)
        flags = (PLAIN if plain else 0) | (0 if graph else NO_GRAPH)
        self._check(self.lib.hntt_bigmul(self.handle, arr, len(pairs), flags, _stream_handle(stream, dev)))
        return outs

    def bigmul_plan(self, pairs, outs, plain: bool = False, graph: bool = True, workspace: torch.Tensor = None,
                    stream=None) -> "PolymulPlan":
        return PolymulPlan(self, pairs, outs, plain, graph, workspace, stream, big=True)

    # -- schedule tuning ---------------------------------------------------------------------------
    def set_tuning(self, log2_len: int, word_bits: int, g_cols: int = 0, g_rows: int = 0, batch_chunk: int = 0,
                   row_log2: int = 0, g_rows_inv: int = 0):
        t = Tuning(log2_len, word_bits, g_cols, g_rows, batch_chunk, row_log2, g_rows_inv)
        self._check(self.lib.hntt_set_tuning(self.handle, ctypes.byref(t)))

    def get_plan(self, log2_len: int, word_bits: int) -> dict:
        t = Tuning()
        self._check(self.lib.hntt_get_plan(self.handle, log2_len, word_bits, ctypes.byref(t)))
        return {k: getattr(t, k) for k in ("g_cols", "g_rows", "batch_chunk", "row_log2", "g_rows_inv")}

    # -- kernel timing -----------------------------------------------------------------------------
    def trace(self, enable: bool = True):
        self._check(self.lib.hntt_trace_enable(self.handle, int(enable)))

    def trace_reset(self):
        self._check(self.lib.hntt_trace_reset(self.handle))

    def trace_read(self) -> dict:
        """Per-kernel launch counts and total milliseconds since the last reset."""
        import json
        n = ctypes.c_size_t(0)
        self.lib.hntt_trace_read(self.handle, None, ctypes.byref(n))
        buf = ctypes.create_string_buffer(n.value + 64)
        n2 = ctypes.c_size_t(len(buf))
        self._check(self.lib.hntt_trace_read(self.handle, buf, ctypes.byref(n2)))
        return json.loads(buf.value.decode())

    def debug_butterfly(self, kind: int, p: int, x, y, w, wp, xo, yo, stream=None):
        wb = _word_bits(x)
        self._check(self.lib.hntt_debug_butterfly(self.handle, kind, wb, p, x.data_ptr(), y.data_ptr(), w.data_ptr(),
                                                  wp.data_ptr(), xo.data_ptr(), yo.data_ptr(), x.numel(),
                                                  _stream_handle(stream, x.device)))
