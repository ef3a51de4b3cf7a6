"""Python binding of libhipmr.so (ctypes): argument marshalling only.

Every step of the elementwise / map-reduce path runs in the library's
run-time generated HIP kernels; this module turns torch tensors and Python
scalars into the C ABI's ``void *args[]`` and maps status codes to
exceptions (the paper raises exceptions instead of requiring explicit error
checks, section "The Basics of GPU programming").  If the shared library is
missing, importing the binding's entry points raises: there is no fallback.

Calls of the C ABI keep their names: ``compile``, ``elementwise``,
``reduce``, ... .  On top sit the paper's two classes,
``ElementwiseKernel(arguments, operation, name)`` and
``ReductionKernel(dtype_out, arguments, map_expr, reduce_expr, neutral)``
(section "Efficient Evaluation of Element-wise Expressions" and section
"Map-Reduce").
"""

from __future__ import annotations

import ctypes
import os
import struct
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
# HIPMR_LIBRARY names another build of the same library (the sanitizer build
# the CPU tests can run against); by default the in-tree libhipmr.so
LIB_PATH = os.environ.get("HIPMR_LIBRARY") or os.path.join(_HERE, "libhipmr.so")

OK = 0
F32, F64, I8, U8, I16, U16, I32, U32, I64, BF16, F16, FP8, C64 = range(1, 14)
DTYPE_NAMES = {F32: "float", F64: "double", I8: "int8_t", U8: "uint8_t", I16: "int16_t",
               U16: "uint16_t", I32: "int", U32: "unsigned", I64: "int64_t",
               BF16: "bfloat16", F16: "half", FP8: "fp8_e4m3", C64: "complex64"}

CFG_NONTEMPORAL, CFG_FORCE_SCALAR, CFG_TEMPORAL = 1, 2, 4
CFG_TEMPORAL_LOADS, CFG_TEMPORAL_STORES, CFG_SEG_GLOBAL, CFG_TUNED = 8, 16, 32, 64
ACCESS_INDEX, ACCESS_SHIFTED, ACCESS_FIXED, ACCESS_OTHER = 1, 2, 4, 8


class HipmrError(RuntimeError):
    code = None

    def __init__(self, message, code=None):
        super().__init__(message)
        if code is not None:
            self.code = code


class InvalidError(HipmrError, ValueError):
    code = -1


class ParseError(HipmrError, ValueError):
    code = -2


class CompileError(HipmrError):
    code = -3


class HipError(HipmrError):
    code = -4


class MismatchError(HipmrError, ValueError):
    code = -5


class UnsupportedError(HipmrError):
    code = -6


class BudgetError(HipmrError):
    code = -7


class WorkspaceError(HipmrError, ValueError):
    code = -8


_ERRORS = {c.code: c for c in (InvalidError, ParseError, CompileError, HipError, MismatchError,
                               UnsupportedError, BudgetError, WorkspaceError)}


class LaunchConfig(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("items_per_thread", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("vec", ctypes.c_int32), ("flags", ctypes.c_int32)]


class HandleInfo(ctypes.Structure):
    _fields_ = [("is_reduce", ctypes.c_int32), ("result_dtype", ctypes.c_int32),
                ("nargs", ctypes.c_int32), ("vectorizable", ctypes.c_int32),
                ("vec", ctypes.c_int32), ("hash", ctypes.c_uint32)]


class CacheStats(ctypes.Structure):
    _fields_ = [("memory_hits", ctypes.c_uint64), ("disk_hits", ctypes.c_uint64),
                ("compiles", ctypes.c_uint64), ("disk_rejects", ctypes.c_uint64),
                ("compile_ms", ctypes.c_double)]


_lib = None
_lib_lock = threading.Lock()

_VP, _SZ, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_CP = ctypes.c_char_p
_SIGS = {
    "hipmr_compile": (_I32, [_CP, _CP, ctypes.POINTER(_VP)]),
    "hipmr_compile_named": (_I32, [_CP, _CP, _CP, ctypes.POINTER(_VP)]),
    "hipmr_elementwise": (_I32, [_VP, _I64, _VP, _VP]),
    "hipmr_elementwise_ex": (_I32, [_VP, _I64, _VP, ctypes.POINTER(LaunchConfig), _VP]),
    "hipmr_reduce_workspace_bytes": (_SZ, [_VP, _I64]),
    "hipmr_reduce": (_I32, [_VP, _CP, _CP, _CP, _I64, _VP, _VP, _VP, _SZ, _VP]),
    "hipmr_reduce_ex": (_I32, [_VP, _CP, _CP, _CP, _I64, _VP, _VP, _VP, _SZ,
                               ctypes.POINTER(LaunchConfig), _VP]),
    "hipmr_prepare_reduce": (_I32, [_VP, _CP, _CP]),
    "hipmr_prepare_reduce_ex": (_I32, [_VP, _CP, _CP, ctypes.POINTER(LaunchConfig)]),
    "hipmr_scan_workspace_bytes": (_SZ, [_VP, _I64]),
    "hipmr_scan": (_I32, [_VP, _CP, _CP, _I64, _VP, _VP, _I32, _VP, _SZ,
                          ctypes.POINTER(LaunchConfig), _VP]),
    "hipmr_segmented_workspace_bytes": (_SZ, [_VP, _I32, _I64]),
    "hipmr_reduce_segmented": (_I32, [_VP, _CP, _CP, _I32, _VP, _I64, _VP, _VP, _VP, _SZ,
                                      ctypes.POINTER(LaunchConfig), _VP]),
    "hipmr_noalloc_scratch_bytes": (_SZ, []),
    "hipmr_reduce_segmented_noalloc": (_I32, [_VP, _CP, _CP, _I32, _VP, _I64, _VP, _VP,
                                              ctypes.POINTER(LaunchConfig), _VP]),
    "hipmr_autotune_segmented": (_I32, [_VP, _CP, _CP, _I32, _VP, _I64, _VP, _VP, _VP, _SZ, _I32,
                                        ctypes.POINTER(LaunchConfig), _VP]),
    "hipmr_autotune_reduce": (_I32, [_VP, _CP, _CP, _I64, _VP, _VP, _VP, _SZ, _I32,
                                     ctypes.POINTER(LaunchConfig), _VP]),
    "hipmr_server_workspace_bytes": (_SZ, [_VP]),
    "hipmr_server_create": (_I32, [_VP, _VP, _SZ, ctypes.POINTER(_VP)]),
    "hipmr_server_submit": (_I32, [_VP, _VP, ctypes.POINTER(ctypes.c_uint64)]),
    "hipmr_server_poll": (_I32, [_VP, _VP, _I32, ctypes.POINTER(_I32)]),
    "hipmr_server_wait_idle": (_I32, [_VP]),
    "hipmr_server_run_schedule": (_I32, [_VP, _VP, _I32, _VP]),
    "hipmr_server_destroy": (None, [_VP]),
    "hipmr_server_now_ns": (_I64, []),
    "hipmr_graph_begin_capture": (_I32, [_VP]),
    "hipmr_graph_end_capture": (_I32, [_VP, ctypes.POINTER(_VP)]),
    "hipmr_graph_launch": (_I32, [_VP, _VP]),
    "hipmr_graph_destroy": (None, [_VP]),
    "hipmr_reduce_compensated": (_I32, [_VP, _I64, _VP, _D, _VP, _VP, _SZ,
                                        ctypes.POINTER(LaunchConfig), _VP]),
    "hipmr_norm2": (_I32, [_VP, _I64, _VP, _D, _I32, _VP, _VP, _SZ,
                           ctypes.POINTER(LaunchConfig), _VP]),
    "hipmr_last_error": (_CP, []),
    "hipmr_release": (None, [_VP]),
    "hipmr_get_handle_info": (_I32, [_VP, ctypes.POINTER(HandleInfo)]),
    "hipmr_get_arg_info": (_I32, [_VP, _I32] + [ctypes.POINTER(_I32)] * 5),
    "hipmr_get_arg_access": (_I32, [_VP, _I32, ctypes.POINTER(_I32)]),
    "hipmr_get_kernel_source": (_I32, [_VP, _I32, _CP, _CP, _CP, _SZ, ctypes.POINTER(_SZ)]),
    "hipmr_get_last_symbols": (_I32, [_VP, _CP, _SZ, ctypes.POINTER(_SZ)]),
    "hipmr_get_cache_stats": (_I32, [ctypes.POINTER(CacheStats)]),
    "hipmr_cache_drop_memory": (None, []),
    "hipmr_sha256_hex": (_I32, [_VP, _SZ, _CP]),
    "hipmr_dtype_size": (_I32, [_I32]),
    "hipmr_selftest_compile": (_I32, [ctypes.POINTER(_I32)]),
}


def lib():
    """The loaded shared library; raises if it has not been built."""
    global _lib
    if _lib is None:
        with _lib_lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(
                        f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                        "(make -C paper_1304_5553_amd/csrc); there is no fallback path")
                handle = ctypes.CDLL(LIB_PATH)
                for name, (res, args) in _SIGS.items():
                    fn = getattr(handle, name)
                    fn.restype = res
                    fn.argtypes = args
                _lib = handle
    return _lib


def _check(status):
    if status != OK:
        msg = lib().hipmr_last_error().decode(errors="replace")
        raise _ERRORS.get(status, HipmrError)(msg, status)


def _stream_ptr(stream):
    if stream is None:
        import torch
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:      # the current stream's handle without a Stream object
            return raw(torch.cuda.current_device())
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _config(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, LaunchConfig):
        return ctypes.byref(cfg)
    c = LaunchConfig()
    for k, v in dict(cfg).items():
        setattr(c, k, int(v))
    return ctypes.byref(c)


_PACK = {F32: "<f", F64: "<d"}
_INT_MASK = {I8: 0xFF, U8: 0xFF, I16: 0xFFFF, U16: 0xFFFF, I32: 0xFFFFFFFF, U32: 0xFFFFFFFF,
             I64: 0xFFFFFFFFFFFFFFFF}
_CTYPE_F32 = ctypes.c_float

_CTYPE = {F32: ctypes.c_float, F64: ctypes.c_double, I8: ctypes.c_int8, U8: ctypes.c_uint8,
          I16: ctypes.c_int16, U16: ctypes.c_uint16, I32: ctypes.c_int32, U32: ctypes.c_uint32,
          I64: ctypes.c_int64, BF16: ctypes.c_uint16, F16: ctypes.c_uint16, FP8: ctypes.c_uint8,
          C64: ctypes.c_float * 2}


def torch_dtype(code):
    import torch
    return {F32: torch.float32, F64: torch.float64, I8: torch.int8, U8: torch.uint8,
            I16: torch.int16, U16: torch.uint16, I32: torch.int32, U32: torch.uint32,
            I64: torch.int64, BF16: torch.bfloat16, F16: torch.float16,
            FP8: torch.float8_e4m3fn, C64: torch.complex64}[code]


def _lowp_bits(code, value):
    """Bit pattern of a Python number rounded to bfloat16 / half / fp8."""
    import torch
    t = torch.tensor([float(value)], dtype=torch.float32)
    if code == FP8:
        return int(t.clamp(-448, 448).to(torch.float8_e4m3fn).view(torch.uint8).item())
    return int(t.to(torch_dtype(code)).view(torch.int16).item()) & 0xFFFF


class Arg:
    __slots__ = ("name", "dtype", "pointer", "const", "read", "written", "access")


_META = {}                # (expr, dtypes, name) -> the handle's metadata (a function of the text)
_META_LOCK = threading.Lock()


class Kernel:
    """A compiled handle (the C ABI's hipmr_handle).  compile() of text seen
    before returns the library's cached handle with one more reference; its
    metadata (argument types and access kinds) is a function of the text
    and is kept here too, so a repeated compile costs one C call."""

    def __init__(self, expr, dtypes, name=None):
        self.expr = expr
        self.dtypes = dtypes
        key = (expr, dtypes, name)
        meta = _META.get(key)
        h = _VP()
        if meta is not None:
            fn, text = meta[-1]
            st = fn(*text, ctypes.byref(h))
            if st != OK:
                _check(st)
        else:
            L = lib()
            if name is None:
                fn, text = L.hipmr_compile, (expr.encode(), dtypes.encode())
            else:
                fn, text = L.hipmr_compile_named, (expr.encode(), dtypes.encode(), name.encode())
            _check(fn(*text, ctypes.byref(h)))
            meta = self._metadata(h, dtypes) + ((fn, text),)
            with _META_LOCK:
                _META[key] = meta
        self._h = h
        (self.is_reduce, self.result_dtype, self.vectorizable, self.vec, self.args,
         self._sized, _) = meta
        self._tls = None                  # per-thread argument buffers, made by the first marshal

    @staticmethod
    def _metadata(h, dtypes):
        info = HandleInfo()
        _check(lib().hipmr_get_handle_info(h, ctypes.byref(info)))
        args = []
        for k in range(info.nargs):
            vals = [_I32() for _ in range(5)]
            _check(lib().hipmr_get_arg_info(h, k, *[ctypes.byref(v) for v in vals]))
            a = Arg()
            a.dtype, a.pointer, a.const, a.read, a.written = (v.value for v in vals)
            acc = _I32()
            _check(lib().hipmr_get_arg_access(h, k, ctypes.byref(acc)))
            a.access = acc.value
            args.append(a)
        names = [d.strip().replace("*", " ").split()[-1]
                 for d in dtypes.split(":", 1)[-1].split(",") if d.strip()]
        for a, nm in zip(args, names):
            a.name = nm
        # arrays that must hold n elements (accessed at i or i +/- E)
        sized = [k for k, a in enumerate(args)
                 if a.pointer and a.access & (ACCESS_INDEX | ACCESS_SHIFTED)]
        return (bool(info.is_reduce), info.result_dtype, bool(info.vectorizable), info.vec,
                tuple(args), sized)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hipmr_release(h)
            self._h = None

    def check_lengths(self, n, args):
        """Arrays the kernels read or write at i or i +/- E must hold at least
        n elements (section "Efficient Evaluation of Element-wise
        Expressions": the operands of one call share a length); arrays read
        only at fixed indices may be shorter."""
        for k in self._sized:
            val = args[k] if k < len(args) else None
            if hasattr(val, "numel") and val.numel() < n:
                raise InvalidError(f"array '{self.args[k].name}' has {val.numel()} elements, "
                                   f"fewer than n = {n}")

    def marshal(self, args):
        """(storage, ctypes array of pointers) for the C ABI's args: every
        value sits in its own 8-byte slot of one buffer (a device pointer, or
        the scalar's bytes in its C type), and args[k] points at slot k.  The
        library copies the values during the call, so each thread reuses one
        pair of buffers per handle, rewritten by its next call."""
        if len(args) != len(self.args):
            raise InvalidError(f"expected {len(self.args)} arguments, got {len(args)}")
        tls = self._tls
        if tls is None:
            with _META_LOCK:
                if self._tls is None:
                    self._tls = threading.local()
            tls = self._tls
        bufs = getattr(tls, "bufs", None)
        if bufs is None:
            nargs = max(1, len(args))
            store = (ctypes.c_uint64 * nargs)()
            base = ctypes.addressof(store)
            bufs = tls.bufs = (store, (ctypes.c_void_p * nargs)(*range(base, base + 8 * nargs, 8)))
        store, ptrs = bufs
        for k, (decl, val) in enumerate(zip(self.args, args)):
            if decl.pointer:
                store[k] = val if isinstance(val, int) else (0 if val is None else val.data_ptr())
            elif decl.dtype in (BF16, F16, FP8):
                store[k] = _lowp_bits(decl.dtype, val)
            elif decl.dtype == C64:
                z = complex(val)
                struct.pack_into("<ff", store, 8 * k, _CTYPE_F32(z.real).value, _CTYPE_F32(z.imag).value)
            elif decl.dtype in _INT_MASK:              # C conversion: wrap to the width
                store[k] = int(val) & _INT_MASK[decl.dtype]
            else:                                      # float / double, as C converts them
                struct.pack_into(_PACK[decl.dtype], store, 8 * k, _CTYPE[decl.dtype](val).value)
        return store, ptrs

    def last_symbols(self):
        """Symbols of the kernels the last call on this handle launched."""
        buf = ctypes.create_string_buffer(4096)
        ln = ctypes.c_size_t()
        _check(lib().hipmr_get_last_symbols(self._h, buf, len(buf), ctypes.byref(ln)))
        return [s for s in buf.value.decode().split(",") if s]

    def source(self, kind, combine_op=None, neutral=None):
        ln = ctypes.c_size_t()
        _check(lib().hipmr_get_kernel_source(self._h, kind, _enc(combine_op), _enc(neutral),
                                             None, 0, ctypes.byref(ln)))
        buf = ctypes.create_string_buffer(ln.value + 1)
        _check(lib().hipmr_get_kernel_source(self._h, kind, _enc(combine_op), _enc(neutral),
                                             buf, len(buf), ctypes.byref(ln)))
        return buf.value.decode()


def _enc(s):
    return None if s is None else s.encode()


def _check_out(out, dtype_code, count, what):
    """The output tensor the library will write `count` values of the
    result type into: device memory of that dtype, contiguous, large
    enough (the C ABI takes a bare pointer and cannot check any of it)."""
    import torch
    if not isinstance(out, torch.Tensor):
        raise InvalidError(f"{what}: out must be a device tensor")
    if not dtype_code:
        raise MismatchError(f"{what}: the handle is an elementwise handle (it has no result type)")
    want = torch_dtype(dtype_code)
    if out.dtype != want:
        raise MismatchError(f"{what}: out has dtype {out.dtype}, the result type is {want}")
    if not out.is_contiguous():
        raise InvalidError(f"{what}: out must be contiguous")
    if out.numel() < count:
        raise InvalidError(f"{what}: out holds {out.numel()} elements, {count} are written")


def _nbytes(t):
    return t.numel() * t.element_size()


def _check_offsets(offsets):
    import torch
    if not isinstance(offsets, torch.Tensor) or offsets.dtype != torch.int64:
        raise MismatchError("offsets must be a device tensor of int64")
    if not offsets.is_contiguous() or offsets.dim() != 1 or offsets.numel() < 1:
        raise InvalidError("offsets must be a contiguous 1-d tensor of nseg + 1 values")


# --------------------------------------------------------------- C ABI names
def compile(expr, dtypes, name=None) -> Kernel:   # noqa: A001 - the C ABI's name
    return Kernel(expr, dtypes, name)


def elementwise(handle: Kernel, n, args, stream=None, config=None):
    handle.check_lengths(int(n), args)
    keep, ptrs = handle.marshal(args)
    _check(lib().hipmr_elementwise_ex(handle.handle, int(n), ptrs, _config(config),
                                      _stream_ptr(stream)))
    return keep


_ws_cache = {}
_ws_lock = threading.Lock()


def workspace(nbytes, device, stream_ptr):
    """A device workspace of at least nbytes, cached per (device, stream)."""
    import torch
    key = (str(device), stream_ptr)
    with _ws_lock:
        buf = _ws_cache.get(key)
        if buf is None or buf.numel() < nbytes:
            buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
            _ws_cache[key] = buf
        return buf


def reduce_workspace_bytes(handle: Kernel, n):
    return lib().hipmr_reduce_workspace_bytes(handle.handle, int(n))


def reduce(handle: Kernel, map_expr, combine_op, neutral, n, args, out, workspace_buf=None,
           stream=None, config=None):   # noqa: A001 - the C ABI's name
    _check_out(out, handle.result_dtype, 1, "reduce")
    s = _stream_ptr(stream)
    need = reduce_workspace_bytes(handle, n)
    if workspace_buf is None:
        workspace_buf = workspace(need, out.device, s)
    handle.check_lengths(int(n), args)
    keep, ptrs = handle.marshal(args)
    _check(lib().hipmr_reduce_ex(handle.handle, _enc(map_expr), _enc(combine_op), _enc(neutral),
                                 int(n), ptrs, ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(workspace_buf.data_ptr()),
                                 _nbytes(workspace_buf),
                                 _config(config), s))
    return out


def _f64_out(out, args):
    import torch
    if out is not None:
        _check_out(out, F64, 1, "compensated sum / norm")
        return out
    device = next((a.device for a in args if isinstance(a, torch.Tensor)), torch.device("cuda"))
    return torch.empty((), dtype=torch.float64, device=device)


def reduce_compensated(handle: Kernel, n, args, post_scale=1.0, out=None, workspace_buf=None,
                       stream=None, config=None):
    """Compensated float sum (FP64 result) = post_scale * sum map(i)."""
    out = _f64_out(out, args)
    s = _stream_ptr(stream)
    if workspace_buf is None:
        workspace_buf = workspace(reduce_workspace_bytes(handle, n), out.device, s)
    handle.check_lengths(int(n), args)
    keep, ptrs = handle.marshal(args)
    _check(lib().hipmr_reduce_compensated(handle.handle, int(n), ptrs, float(post_scale),
                                          ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(workspace_buf.data_ptr()),
                                          _nbytes(workspace_buf), _config(config), s))
    return out


def norm2(handle: Kernel, n, args, post_scale=1.0, passes=2, out=None, workspace_buf=None,
          stream=None, config=None):
    """L2 norm (FP64 result) = post_scale * sqrt(sum map(i)^2); scaled two-pass by default."""
    out = _f64_out(out, args)
    s = _stream_ptr(stream)
    if workspace_buf is None:
        workspace_buf = workspace(reduce_workspace_bytes(handle, n), out.device, s)
    handle.check_lengths(int(n), args)
    keep, ptrs = handle.marshal(args)
    _check(lib().hipmr_norm2(handle.handle, int(n), ptrs, float(post_scale), int(passes),
                             ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(workspace_buf.data_ptr()), _nbytes(workspace_buf),
                             _config(config), s))
    return out


def scan_workspace_bytes(handle: Kernel, n):
    return lib().hipmr_scan_workspace_bytes(handle.handle, int(n))


def scan(handle: Kernel, combine_op, neutral, n, args, out, exclusive=False, workspace_buf=None,
         stream=None, config=None):
    """out[i] = neutral (+) map(0) (+) ... (+) map(i) (inclusive) or up to
    map(i - 1) (exclusive); `out` is a device tensor of n result values."""
    _check_out(out, handle.result_dtype, int(n), "scan")
    s = _stream_ptr(stream)
    if workspace_buf is None:
        workspace_buf = workspace(scan_workspace_bytes(handle, n), out.device, s)
    handle.check_lengths(int(n), args)
    keep, ptrs = handle.marshal(args)
    _check(lib().hipmr_scan(handle.handle, combine_op.encode(), neutral.encode(), int(n), ptrs,
                            ctypes.c_void_p(out.data_ptr()), 1 if exclusive else 0,
                            ctypes.c_void_p(workspace_buf.data_ptr()), _nbytes(workspace_buf),
                            _config(config), s))
    return out


def segmented_workspace_bytes(handle: Kernel, nseg, total_n):
    return lib().hipmr_segmented_workspace_bytes(handle.handle, int(nseg), int(total_n))


def reduce_segmented(handle: Kernel, combine_op, neutral, offsets, total_n, args, out,
                     workspace_buf=None, stream=None, config=None):
    """out[s] = fold of map(i) over i in [offsets[s], offsets[s+1]) (device
    int64 offsets, nseg + 1 of them)."""
    _check_offsets(offsets)
    nseg = offsets.numel() - 1
    _check_out(out, handle.result_dtype, nseg, "reduce_segmented")
    s = _stream_ptr(stream)
    if workspace_buf is None:
        workspace_buf = workspace(segmented_workspace_bytes(handle, nseg, total_n), out.device, s)
    handle.check_lengths(int(total_n), args)
    keep, ptrs = handle.marshal(args)
    _check(lib().hipmr_reduce_segmented(handle.handle, combine_op.encode(), neutral.encode(), nseg,
                                        ctypes.c_void_p(offsets.data_ptr()), int(total_n), ptrs,
                                        ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(workspace_buf.data_ptr()),
                                        _nbytes(workspace_buf), _config(config), s))
    return out


def noalloc_scratch_bytes():
    """Bytes of the library's static scratch array (per device)."""
    return lib().hipmr_noalloc_scratch_bytes()


def reduce_segmented_noalloc(handle: Kernel, combine_op, neutral, offsets, total_n, args, out,
                             stream=None, config=None):
    """reduce_segmented without a workspace and without any allocation: the
    tile table and partials live in the library's static scratch array.  Run
    reduce_segmented once on the device with the same arguments first."""
    _check_offsets(offsets)
    nseg = offsets.numel() - 1
    _check_out(out, handle.result_dtype, nseg, "reduce_segmented_noalloc")
    handle.check_lengths(int(total_n), args)
    keep, ptrs = handle.marshal(args)
    _check(lib().hipmr_reduce_segmented_noalloc(handle.handle, combine_op.encode(), neutral.encode(),
                                                nseg, ctypes.c_void_p(offsets.data_ptr()),
                                                int(total_n), ptrs, ctypes.c_void_p(out.data_ptr()),
                                                _config(config), _stream_ptr(stream)))
    return out


def autotune_segmented(handle: Kernel, combine_op, neutral, offsets, total_n, args, out,
                       reps=10, workspace_buf=None, stream=None):
    """Times the candidate geometries on this data and stores the fastest;
    returns it as a dict."""
    _check_offsets(offsets)
    nseg = offsets.numel() - 1
    _check_out(out, handle.result_dtype, nseg, "autotune_segmented")
    s = _stream_ptr(stream)
    if workspace_buf is None:
        workspace_buf = workspace(segmented_workspace_bytes(handle, nseg, total_n), out.device, s)
    handle.check_lengths(int(total_n), args)
    keep, ptrs = handle.marshal(args)
    best = LaunchConfig()
    _check(lib().hipmr_autotune_segmented(handle.handle, combine_op.encode(), neutral.encode(), nseg,
                                          ctypes.c_void_p(offsets.data_ptr()), int(total_n), ptrs,
                                          ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(workspace_buf.data_ptr()),
                                          _nbytes(workspace_buf), int(reps), ctypes.byref(best), s))
    return {f: getattr(best, f) for f, _ in LaunchConfig._fields_}


def autotune_reduce(handle: Kernel, combine_op, neutral, n, args, out, reps=10,
                    workspace_buf=None, stream=None):
    _check_out(out, handle.result_dtype, 1, "autotune_reduce")
    s = _stream_ptr(stream)
    if workspace_buf is None:
        workspace_buf = workspace(reduce_workspace_bytes(handle, n), out.device, s)
    handle.check_lengths(int(n), args)
    keep, ptrs = handle.marshal(args)
    best = LaunchConfig()
    _check(lib().hipmr_autotune_reduce(handle.handle, combine_op.encode(), neutral.encode(), int(n),
                                       ptrs, ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(workspace_buf.data_ptr()),
                                       _nbytes(workspace_buf), int(reps), ctypes.byref(best), s))
    return {f: getattr(best, f) for f, _ in LaunchConfig._fields_}


class Graph:
    """Captures the hipmr calls issued inside ``with graph.capture(stream):``
    into a HIP graph; ``graph.launch(stream)`` replays them."""

    def __init__(self):
        self._g = _VP()

    def capture(self, stream):
        graph = self

        class _Ctx:
            def __enter__(self_inner):
                graph._stream = _stream_ptr(stream)
                _check(lib().hipmr_graph_begin_capture(graph._stream))
                return graph

            def __exit__(self_inner, exc_type, exc, tb):
                st = lib().hipmr_graph_end_capture(graph._stream, ctypes.byref(graph._g))
                if exc_type is None:
                    _check(st)
                return False
        return _Ctx()

    def launch(self, stream=None):
        _check(lib().hipmr_graph_launch(self._g, _stream_ptr(stream)))

    def __del__(self):
        if getattr(self, "_g", None) is not None and self._g.value and _lib is not None:
            _lib.hipmr_graph_destroy(self._g)
            self._g = None


def prepare_reduce(handle: Kernel, combine_op, neutral):
    _check(lib().hipmr_prepare_reduce(handle.handle, combine_op.encode(), neutral.encode()))


def cache_stats():
    s = CacheStats()
    _check(lib().hipmr_get_cache_stats(ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in CacheStats._fields_}


def cache_drop_memory():
    lib().hipmr_cache_drop_memory()


def sha256_hex(data: bytes) -> str:
    out = ctypes.create_string_buffer(65)
    _check(lib().hipmr_sha256_hex(data, len(data), out))
    return out.value.decode()


def selftest_compile() -> int:
    n = _I32()
    _check(lib().hipmr_selftest_compile(ctypes.byref(n)))
    return n.value


# --------------------------------------------------------------- paper classes
def _tensor_args(kernel, args):
    import torch
    n = None
    for decl, a in zip(kernel.args, args):
        if decl.pointer:
            if not isinstance(a, torch.Tensor):
                raise InvalidError(f"argument {decl.name} must be a tensor")
            if not a.is_contiguous():
                raise InvalidError(f"argument {decl.name} must be contiguous (flat arrays)")
            if a.dtype != torch_dtype(decl.dtype):
                raise MismatchError(f"argument {decl.name}: expected {torch_dtype(decl.dtype)}, "
                                    f"got {a.dtype}")
            if n is None:
                n = a.numel()
            elif a.numel() != n:
                # all arrays of one elementwise / map-reduce call share a length
                raise MismatchError("all array arguments must have the same length")
    return n if n is not None else 0


class ElementwiseKernel:
    """ElementwiseKernel(arguments, operation, name): run ``operation`` for
    every index i of the (same-length) array arguments."""

    def __init__(self, arguments, operation, name="kernel"):
        self.kernel = Kernel(operation, arguments, name)

    def __call__(self, *args, stream=None, config=None):
        n = _tensor_args(self.kernel, args)
        elementwise(self.kernel, n, args, stream=stream, config=config)


_C_NAMES = {"float32": "float", "float64": "double", "int32": "int", "int64": "int64_t",
            "uint32": "unsigned"}


def _c_type_name(dtype_out):
    if isinstance(dtype_out, str):
        return dtype_out
    name = str(dtype_out).replace("torch.", "").replace("<class 'numpy.", "").rstrip("'>")
    if name in _C_NAMES:
        return _C_NAMES[name]
    import numpy as np
    return _C_NAMES[np.dtype(dtype_out).name]


class ReductionKernel:
    """ReductionKernel(dtype_out, arguments, map_expr, reduce_expr, neutral):
    calling it returns a 0-d device tensor holding
    neutral (+) map(0) (+) ... (+) map(n-1)."""

    def __init__(self, dtype_out, arguments, map_expr, reduce_expr, neutral, name="reduce"):
        self.map_expr = map_expr
        self.reduce_expr = reduce_expr
        self.neutral = str(neutral)
        self.kernel = Kernel(map_expr, f"{_c_type_name(dtype_out)}: {arguments}", name)
        prepare_reduce(self.kernel, reduce_expr, self.neutral)

    def __call__(self, *args, stream=None, out=None, config=None):
        import torch
        n = _tensor_args(self.kernel, args)
        device = next((a.device for a in args if isinstance(a, torch.Tensor)), torch.device("cuda"))
        if out is None:
            out = torch.empty((), dtype=torch_dtype(self.kernel.result_dtype), device=device)
        return reduce(self.kernel, self.map_expr, self.reduce_expr, self.neutral, n, args, out,
                      stream=stream, config=config)


# --------------------------------------------------------------- serving
JOB_SUM, JOB_DOT, JOB_NORM2, JOB_MAX, JOB_AXPBY_SUM, JOB_COUNT_POS, JOB_SUMSQ, JOB_WMEAN = range(8)
JOB_NAMES = ["sum", "dot", "norm2", "max", "axpby_sum", "count_pos", "sumsq", "wmean"]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("nstreams", ctypes.c_int32),
                ("max_batch_jobs", ctypes.c_int32), ("max_batch_tiles", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("max_batch_bytes", ctypes.c_uint64),
                ("solo_bytes", ctypes.c_uint64), ("batch_backlog", ctypes.c_int32),
                ("resident", ctypes.c_int32)]


def _sjob_dtype():
    import numpy as np
    dt = np.dtype([("x", np.uint64), ("y", np.uint64), ("w", np.uint64), ("n", np.int64),
                   ("tmpl", np.int32), ("dtype", np.int32), ("arrival_ns", np.int64),
                   ("out", np.uint64), ("a", np.float32), ("b", np.float32)])
    assert dt.itemsize == 64
    return dt


def _completion_dtype():
    import numpy as np
    dt = np.dtype([("ticket", np.uint64), ("status", np.int32), ("batch_jobs", np.int32),
                   ("arrival_ns", np.int64), ("launch_ns", np.int64), ("done_ns", np.int64)])
    assert dt.itemsize == 40
    return dt


class Server:
    """The serving request loop (hipmr_server_*): jobs are numpy records of
    ``Server.JOB`` (device pointers as integers)."""

    def __init__(self, hbm_budget_bytes=0, nstreams=0, max_batch_jobs=0, max_batch_tiles=0,
                 blocks_per_cu=0, max_batch_bytes=0, solo_bytes=0, batch_backlog=0, resident=0,
                 device=None):
        import torch
        self.JOB = _sjob_dtype()
        self.COMPLETION = _completion_dtype()
        self.cfg = ServerConfig(hbm_budget_bytes, nstreams, max_batch_jobs, max_batch_tiles,
                                blocks_per_cu, max_batch_bytes, solo_bytes, batch_backlog,
                                int(resident))
        nbytes = lib().hipmr_server_workspace_bytes(ctypes.byref(self.cfg))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8,
                                     device=device or torch.device("cuda"))
        h = _VP()
        _check(lib().hipmr_server_create(ctypes.byref(self.cfg),
                                         ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                         ctypes.byref(h)))
        self._s = h

    def jobs(self, count):
        import numpy as np
        return np.zeros(count, dtype=self.JOB)

    def submit(self, job):
        import numpy as np
        rec = np.ascontiguousarray(np.asarray(job, dtype=self.JOB).reshape(1))
        t = ctypes.c_uint64()
        _check(lib().hipmr_server_submit(self._s, rec.ctypes.data, ctypes.byref(t)))
        return t.value

    def poll(self, cap=4096):
        import numpy as np
        out = np.zeros(cap, dtype=self.COMPLETION)
        nd = _I32()
        _check(lib().hipmr_server_poll(self._s, out.ctypes.data, cap, ctypes.byref(nd)))
        return out[:nd.value]

    def wait_idle(self):
        _check(lib().hipmr_server_wait_idle(self._s))

    def run_schedule(self, jobs):
        import numpy as np
        jobs = np.ascontiguousarray(jobs, dtype=self.JOB)
        done = np.zeros(len(jobs), dtype=self.COMPLETION)
        _check(lib().hipmr_server_run_schedule(self._s, jobs.ctypes.data, len(jobs),
                                               done.ctypes.data))
        return done

    def close(self):
        if getattr(self, "_s", None) is not None and self._s.value and _lib is not None:
            _lib.hipmr_server_destroy(self._s)
        self._s = None

    def __del__(self):
        self.close()


def server_now_ns():
    return lib().hipmr_server_now_ns()
