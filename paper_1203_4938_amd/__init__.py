"""dpfft: batched complex-to-complex FFTs on an AMD MI355X (gfx950).

Thin ctypes binding of ``libdpfft.so`` (see ``include/dpfft.h``).  The
functions ``fft_plan``, ``fft_exec``, ``fft_destroy``, ``fft_workspace_bytes``,
``fft_status_str``, ``fft_last_error`` and ``fft_plan_describe`` mirror the C
entry points one to one and only marshal arguments; :class:`Plan` wraps them
for torch tensors (device memory and the current stream come from torch).
Every transform runs in the library's HIP kernels; there is no fallback: if
the library is missing or fails to load, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch  # loaded first so the library binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpfft.so")

FFT_OK, FFT_E_INVALID, FFT_E_UNSUPPORTED, FFT_E_NOMEM, FFT_E_DEVICE, FFT_E_INTERNAL = range(6)
FFT_FORWARD, FFT_INVERSE = -1, +1
FFT_F_INPLACE, FFT_F_NO_AUTOTUNE, FFT_F_GRAPH, FFT_F_PER_SIZE, FFT_F_REAL, FFT_F_CONV = \
    1, 2, 4, 8, 16, 32
PRECISIONS = {"fp32": 0, "fp16": 1, "bf16": 2, "fp16_split": 3, "bf16_split": 4, "bf16_split3": 5}

#: names of every C entry point declared in include/dpfft.h
EXPORTS = ("fft_plan", "fft_exec", "fft_destroy", "fft_workspace_bytes", "fft_status_str",
           "fft_last_error", "fft_plan_describe", "fft_plan_num_steps", "fft_exec_steps",
           "fft_plan_dry", "fft_autotune", "fft_conv_exec", "fft_exec_noalloc",
           "img_workspace_bytes", "img_compress", "img_encode")


class FftError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        super().__init__(f"{where}: {_status_name(status)}: {msg}")


class FftDesc(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("n", ctypes.c_int64 * 2), ("batch", ctypes.c_int64),
                ("dist", ctypes.c_int64), ("ragged_sizes", ctypes.POINTER(ctypes.c_int64)),
                ("ragged_offsets", ctypes.POINTER(ctypes.c_int64)),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


IMG_F_GRAPH = 1


class ImgDesc(ctypes.Structure):
    """img_desc_t: images height x width (multiples of 4), batch, codewords k,
    Lloyd iterations, activity threshold tau."""
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("k", ctypes.c_int32), ("iters", ctypes.c_int32), ("tau", ctypes.c_float),
                ("flags", ctypes.c_uint32)]


class ImgOut(ctypes.Structure):
    _fields_ = [("y", ctypes.c_void_p), ("cb", ctypes.c_void_p), ("cr", ctypes.c_void_p),
                ("mean", ctypes.c_void_p), ("act", ctypes.c_void_p), ("dev", ctypes.c_void_p),
                ("codebook", ctypes.c_void_p), ("code", ctypes.c_void_p)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1203_4938_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.fft_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(FftDesc), vp]
    lib.fft_plan.restype = ctypes.c_int
    lib.fft_exec.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp]
    lib.fft_exec.restype = ctypes.c_int
    lib.fft_destroy.argtypes = [vp]
    lib.fft_destroy.restype = ctypes.c_int
    lib.fft_workspace_bytes.argtypes = [vp]
    lib.fft_workspace_bytes.restype = ctypes.c_size_t
    lib.fft_status_str.argtypes = [ctypes.c_int]
    lib.fft_status_str.restype = ctypes.c_char_p
    lib.fft_last_error.argtypes = []
    lib.fft_last_error.restype = ctypes.c_char_p
    lib.fft_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.fft_plan_describe.restype = ctypes.c_size_t
    lib.fft_plan_num_steps.argtypes = [vp]
    lib.fft_plan_num_steps.restype = ctypes.c_int
    lib.fft_exec_steps.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int]
    lib.fft_exec_steps.restype = ctypes.c_int
    lib.fft_plan_dry.argtypes = [ctypes.POINTER(FftDesc), ctypes.c_char_p, ctypes.c_size_t]
    lib.fft_plan_dry.restype = ctypes.c_int
    lib.fft_autotune.argtypes = [ctypes.POINTER(FftDesc), vp, ctypes.c_int, ctypes.c_char_p,
                                 ctypes.c_size_t]
    lib.fft_autotune.restype = ctypes.c_int
    lib.fft_conv_exec.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, vp]
    lib.fft_conv_exec.restype = ctypes.c_int
    lib.fft_exec_noalloc.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.fft_exec_noalloc.restype = ctypes.c_int
    lib.img_workspace_bytes.argtypes = [ctypes.POINTER(ImgDesc)]
    lib.img_workspace_bytes.restype = ctypes.c_size_t
    lib.img_compress.argtypes = [ctypes.POINTER(ImgDesc), vp, ctypes.POINTER(ImgOut), vp, vp]
    lib.img_compress.restype = ctypes.c_int
    lib.img_encode.argtypes = [ctypes.POINTER(ImgDesc), vp, vp, vp, vp, vp]
    lib.img_encode.restype = ctypes.c_int
    return lib


_lib = _load()


def _status_name(s: int) -> str:
    return _lib.fft_status_str(s).decode()


# ---------------------------------------------------------------------------
# one-to-one wrappers of the C entry points
# ---------------------------------------------------------------------------
def fft_status_str(status: int) -> str:
    return _status_name(status)


def fft_last_error() -> str:
    return _lib.fft_last_error().decode()


def fft_plan(desc: FftDesc, stream: int = 0) -> tuple[int, Optional[int]]:
    """Returns (status, handle or None)."""
    h = ctypes.c_void_p()
    st = _lib.fft_plan(ctypes.byref(h), ctypes.byref(desc), ctypes.c_void_p(stream))
    return st, (h.value if st == FFT_OK else None)


def fft_exec(handle: int, in_ptr: int, out_ptr: int, direction: int, workspace: int = 0,
             stream: int = 0) -> int:
    return _lib.fft_exec(ctypes.c_void_p(handle), ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                         direction, ctypes.c_void_p(workspace), ctypes.c_void_p(stream))


def fft_conv_exec(handle: int, in_ptr: int, filter_ptr: int, filter_dist: int, out_ptr: int,
                  workspace: int = 0, stream: int = 0) -> int:
    return _lib.fft_conv_exec(ctypes.c_void_p(handle), ctypes.c_void_p(in_ptr),
                              ctypes.c_void_p(filter_ptr), int(filter_dist),
                              ctypes.c_void_p(out_ptr), ctypes.c_void_p(workspace),
                              ctypes.c_void_p(stream))


def fft_exec_noalloc(handle: int, in_ptr: int, out_ptr: int, direction: int,
                     stream: int = 0) -> int:
    return _lib.fft_exec_noalloc(ctypes.c_void_p(handle), ctypes.c_void_p(in_ptr),
                                 ctypes.c_void_p(out_ptr), direction, ctypes.c_void_p(stream))


def img_workspace_bytes(desc: ImgDesc) -> int:
    return _lib.img_workspace_bytes(ctypes.byref(desc))


def img_compress(rgb: torch.Tensor, k: int, iters: int, tau: float, stream=None,
                 graph: bool = False) -> dict:
    """Image block compression of a batch of RGB images (uint8 CUDA tensor of
    shape (batch, height, width, 3) or (height, width, 3)): returns the
    outputs of img_compress as tensors y, cb, cr, mean, act, dev, codebook,
    code.  graph=True sets IMG_F_GRAPH (pays off only for repeated calls on
    the same buffers; this function allocates new outputs per call)."""
    if rgb.dim() == 3:
        rgb = rgb.unsqueeze(0)
    if rgb.dtype != torch.uint8 or rgb.device.type != "cuda" or not rgb.is_contiguous() or \
            rgb.dim() != 4 or rgb.shape[-1] != 3:
        raise ValueError("rgb must be a contiguous uint8 CUDA tensor (batch, height, width, 3)")
    B, h, w = (int(v) for v in rgb.shape[:3])
    d = ImgDesc(height=h, width=w, batch=B, k=int(k), iters=int(iters), tau=float(tau),
                flags=IMG_F_GRAPH if graph else 0)
    dev = rgb.device
    f32 = dict(dtype=torch.float32, device=dev)
    nb = (h // 4) * (w // 4)
    res = {"y": torch.empty((B, h, w), **f32), "cb": torch.empty((B, h // 2, w // 2), **f32),
           "cr": torch.empty((B, h // 2, w // 2), **f32),
           "mean": torch.empty((B, h // 4, w // 4), **f32),
           "act": torch.empty((B, h // 4, w // 4), **f32), "dev": torch.empty((B, nb, 16), **f32),
           "codebook": torch.empty((B, int(k), 16), **f32),
           "code": torch.empty((B, nb), dtype=torch.int32, device=dev)}
    o = ImgOut(*(res[n].data_ptr() for n in ("y", "cb", "cr", "mean", "act", "dev", "codebook",
                                             "code")))
    wsb = _lib.img_workspace_bytes(ctypes.byref(d))
    ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=dev)
    st = _lib.img_compress(ctypes.byref(d), ctypes.c_void_p(rgb.data_ptr()), ctypes.byref(o),
                           ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(_stream_handle(stream)))
    if st != FFT_OK:
        raise FftError(st, "img_compress", fft_last_error())
    res["_workspace"] = ws
    return res


def img_encode(dev: torch.Tensor, act: torch.Tensor, codebook: torch.Tensor, height: int,
               width: int, tau: float, stream=None) -> torch.Tensor:
    """Step (e) alone: codes (int32, (batch, blocks)) of deviation vectors
    (batch, blocks, 16), activities (batch, blocks) and codebooks (batch, k, 16)."""
    B, k = int(codebook.shape[0]), int(codebook.shape[1])
    for t in (dev, act, codebook):
        if t.dtype != torch.float32 or t.device.type != "cuda" or not t.is_contiguous():
            raise ValueError("dev, act and codebook must be contiguous float32 CUDA tensors")
    d = ImgDesc(height=int(height), width=int(width), batch=B, k=k, iters=0, tau=float(tau))
    code = torch.empty((B, (height // 4) * (width // 4)), dtype=torch.int32, device=dev.device)
    st = _lib.img_encode(ctypes.byref(d), ctypes.c_void_p(dev.data_ptr()),
                         ctypes.c_void_p(act.data_ptr()), ctypes.c_void_p(codebook.data_ptr()),
                         ctypes.c_void_p(code.data_ptr()), ctypes.c_void_p(_stream_handle(stream)))
    if st != FFT_OK:
        raise FftError(st, "img_encode", fft_last_error())
    return code


def fft_plan_num_steps(handle: Optional[int]) -> int:
    return _lib.fft_plan_num_steps(ctypes.c_void_p(handle))


def fft_exec_steps(handle: int, in_ptr: int, out_ptr: int, direction: int, workspace: int,
                   stream: int, first: int, count: int) -> int:
    return _lib.fft_exec_steps(ctypes.c_void_p(handle), ctypes.c_void_p(in_ptr),
                               ctypes.c_void_p(out_ptr), direction, ctypes.c_void_p(workspace),
                               ctypes.c_void_p(stream), first, count)


def fft_plan_dry(desc: FftDesc) -> tuple[int, str]:
    """Plan on the host only; returns (status, description or error message)."""
    buf = ctypes.create_string_buffer(1 << 16)
    st = _lib.fft_plan_dry(ctypes.byref(desc), buf, len(buf))
    return st, (buf.value.decode() if st == FFT_OK else fft_last_error())


def fft_autotune(desc: FftDesc, stream: int = 0, reps: int = 10) -> tuple[int, str]:
    """Time the candidate kernel variants for desc; returns (status, report)."""
    buf = ctypes.create_string_buffer(1 << 16)
    st = _lib.fft_autotune(ctypes.byref(desc), ctypes.c_void_p(stream), reps, buf, len(buf))
    return st, (buf.value.decode() if st == FFT_OK else fft_last_error())


def fft_destroy(handle: Optional[int]) -> int:
    return _lib.fft_destroy(ctypes.c_void_p(handle))


def fft_workspace_bytes(handle: Optional[int]) -> int:
    return _lib.fft_workspace_bytes(ctypes.c_void_p(handle))


def fft_plan_describe(handle: Optional[int]) -> str:
    need = _lib.fft_plan_describe(ctypes.c_void_p(handle), None, 0)
    buf = ctypes.create_string_buffer(need + 1)
    _lib.fft_plan_describe(ctypes.c_void_p(handle), buf, need + 1)
    return buf.value.decode()


def make_desc(n=None, batch: int = 1, *, rank: int = 1, shape=None, dist: int = 0,
              ragged_sizes: Optional[Sequence[int]] = None,
              ragged_offsets: Optional[Sequence[int]] = None,
              precision: str = "fp32", flags: int = 0):
    """Builds an FftDesc; returns (desc, keepalive) -- keep the second alive
    while the desc is in use (it owns the ragged arrays)."""
    d = FftDesc()
    d.rank = rank
    if rank == 2:
        d.n[0], d.n[1] = int(shape[0]), int(shape[1])
    else:
        d.n[0] = int(n) if n is not None else 0
    d.batch = int(batch)
    d.dist = int(dist)
    keep = []
    if ragged_sizes is not None:
        arr = (ctypes.c_int64 * len(ragged_sizes))(*[int(v) for v in ragged_sizes])
        keep.append(arr)
        d.ragged_sizes = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int64))
        d.batch = len(ragged_sizes)
    if ragged_offsets is not None:
        arr = (ctypes.c_int64 * len(ragged_offsets))(*[int(v) for v in ragged_offsets])
        keep.append(arr)
        d.ragged_offsets = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int64))
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d.flags = flags
    return d, keep


# ---------------------------------------------------------------------------
# torch-facing plan object
# ---------------------------------------------------------------------------
class Plan:
    """A dpfft plan for torch complex64 CUDA tensors.

    ``Plan(n, batch)`` -- batch of length-n signals (last axis);
    ``Plan(shape=(ny, nx), batch=b, rank=2)`` -- batch of images;
    ``Plan(ragged_sizes=[...])`` -- ragged batch packed back to back;
    ``real=True`` -- real samples: the forward transform takes float32
    samples and returns the n//2 + 1 bins (rank 2: ny x (nx//2 + 1)) as
    complex64, the inverse takes those bins and returns float32 samples;
    ``conv=True`` -- the plan also runs :meth:`conv` (fused circular
    convolution with filter spectra).
    """

    def __init__(self, n: Optional[int] = None, batch: int = 1, *, rank: int = 1, shape=None,
                 dist: int = 0, ragged_sizes=None, ragged_offsets=None, precision: str = "fp32",
                 inplace: bool = False, graph: bool = False, per_size: bool = False,
                 autotune: bool = True, real: bool = False, conv: bool = False, stream=None):
        flags = (FFT_F_INPLACE if inplace else 0) | (FFT_F_GRAPH if graph else 0) | \
                (FFT_F_PER_SIZE if per_size else 0) | (0 if autotune else FFT_F_NO_AUTOTUNE) | \
                (FFT_F_REAL if real else 0) | (FFT_F_CONV if conv else 0)
        self.real = bool(real)
        self.desc, self._keep = make_desc(n, batch, rank=rank, shape=shape, dist=dist,
                                          ragged_sizes=ragged_sizes, ragged_offsets=ragged_offsets,
                                          precision=precision, flags=flags)
        self.rank = rank
        self.batch = int(self.desc.batch)
        self.ragged = ragged_sizes is not None
        if self.ragged:
            sizes = [int(v) for v in ragged_sizes]
            if ragged_offsets is None:
                offs, acc = [], 0
                for v in sizes:
                    offs.append(acc)
                    acc += v
            else:
                offs = [int(v) for v in ragged_offsets]
            self.sizes, self.offsets = sizes, offs
            self.numel = max((o + s for o, s in zip(offs, sizes)), default=0)
        elif self.real:
            rows = int(self.desc.n[0]) if rank == 2 else 1
            nr = int(self.desc.n[1]) if rank == 2 else int(self.desc.n[0])
            #: float32 samples of the real side, complex64 bins of the spectrum side
            self.real_numel = self.batch * rows * nr
            self.cplx_numel = self.batch * rows * (nr // 2 + 1)
            self.real_shape = (rows, nr) if rank == 2 else (nr,)
            self.cplx_shape = (rows, nr // 2 + 1) if rank == 2 else (nr // 2 + 1,)
            self.numel = self.cplx_numel
        else:
            per = int(self.desc.n[0]) * (int(self.desc.n[1]) if rank == 2 else 1)
            d = int(dist) if dist else per
            self.numel = (self.batch - 1) * d + per if self.batch else 0
        s = _stream_handle(stream)
        st, h = fft_plan(self.desc, s)
        if st != FFT_OK:
            raise FftError(st, "fft_plan", fft_last_error())
        self.handle = h
        self.workspace_bytes = fft_workspace_bytes(h)
        self._ws = None

    def describe(self) -> str:
        return fft_plan_describe(self.handle)

    def workspace(self, device) -> Optional[torch.Tensor]:
        if self.workspace_bytes == 0:
            return None
        if self._ws is None or self._ws.device != device:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)
        return self._ws

    def exec(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, inverse: bool = False,
             stream=None) -> torch.Tensor:
        if self.real:
            return self._exec_real(x, out, inverse, stream)
        _check_tensor(x, self.numel, "x")
        if out is None:
            out = torch.empty_like(x)
        else:
            _check_tensor(out, self.numel, "out")
        ws = self.workspace(x.device)
        st = fft_exec(self.handle, x.data_ptr(), out.data_ptr(),
                      FFT_INVERSE if inverse else FFT_FORWARD,
                      ws.data_ptr() if ws is not None else 0, _stream_handle(stream))
        if st != FFT_OK:
            raise FftError(st, "fft_exec", fft_last_error())
        return out

    def conv(self, x: torch.Tensor, spec: torch.Tensor, out: Optional[torch.Tensor] = None,
             stream=None) -> torch.Tensor:
        """Circular convolution of every signal of x with the filter whose
        spectrum (the forward transform of the filter, natural order) is
        ``spec``: one spectrum (n elements) shared by every signal, or one per
        signal laid out like x."""
        _check_tensor(x, self.numel, "x")
        n = int(self.desc.n[0])
        if spec.numel() == n:
            _check_tensor(spec, n, "spec")
            fdist = 0
        else:
            _check_tensor(spec, self.numel, "spec")
            fdist = int(self.desc.dist) if self.desc.dist else n
        if out is None:
            out = torch.empty_like(x)
        else:
            _check_tensor(out, self.numel, "out")
        ws = self.workspace(x.device)
        st = fft_conv_exec(self.handle, x.data_ptr(), spec.data_ptr(), fdist, out.data_ptr(),
                           ws.data_ptr() if ws is not None else 0, _stream_handle(stream))
        if st != FFT_OK:
            raise FftError(st, "fft_conv_exec", fft_last_error())
        return out

    def _exec_real(self, x, out, inverse, stream):
        if not inverse:
            _check_tensor(x, self.real_numel, "x", torch.float32)
            if out is None:
                out = torch.empty((self.batch, *self.cplx_shape), dtype=torch.complex64,
                                  device=x.device)
            _check_tensor(out, self.cplx_numel, "out")
        else:
            _check_tensor(x, self.cplx_numel, "x")
            if out is None:
                out = torch.empty((self.batch, *self.real_shape), dtype=torch.float32,
                                  device=x.device)
            _check_tensor(out, self.real_numel, "out", torch.float32)
        ws = self.workspace(x.device)
        st = fft_exec(self.handle, x.data_ptr(), out.data_ptr(),
                      FFT_INVERSE if inverse else FFT_FORWARD,
                      ws.data_ptr() if ws is not None else 0, _stream_handle(stream))
        if st != FFT_OK:
            raise FftError(st, "fft_exec", fft_last_error())
        return out

    def num_steps(self) -> int:
        return fft_plan_num_steps(self.handle)

    def exec_steps(self, x: torch.Tensor, out: torch.Tensor, first: int, count: int,
                   inverse: bool = False, stream=None) -> torch.Tensor:
        """Enqueue launches [first, first+count) only (timing one kernel)."""
        ws = self.workspace(x.device)
        st = fft_exec_steps(self.handle, x.data_ptr(), out.data_ptr(),
                            FFT_INVERSE if inverse else FFT_FORWARD,
                            ws.data_ptr() if ws is not None else 0, _stream_handle(stream),
                            first, count)
        if st != FFT_OK:
            raise FftError(st, "fft_exec_steps", fft_last_error())
        return out

    def close(self):
        if getattr(self, "handle", None):
            fft_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_handle(stream) -> int:
    if stream is None:
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return 0
    return int(getattr(stream, "cuda_stream", stream))


def _check_tensor(t: torch.Tensor, numel: int, name: str, dtype=torch.complex64):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, the plan needs {numel}")


_cache: dict = {}


def fft(x: torch.Tensor, inverse: bool = False) -> torch.Tensor:
    """Batched FFT over the last axis of a contiguous complex64 CUDA tensor."""
    n = x.shape[-1]
    b = x.numel() // n if n else 0
    key = (n, b)
    p = _cache.get(key)
    if p is None:
        p = _cache[key] = Plan(n, b)
    return p.exec(x, inverse=inverse)


def ifft(x: torch.Tensor) -> torch.Tensor:
    return fft(x, inverse=True)
