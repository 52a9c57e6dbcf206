"""Thin ctypes binding of the C ABI in include/phasemask.h.

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory (tensors) and the stream (the current torch
stream of the tensors' device is handed to the library before each call).
If the library has not been built, importing this module raises ImportError:
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # must load before the library: the process then has one HIP runtime

# PHASEMASK_LIBRARY names another build of the same library (for instance the
# timeline build, libphasemask_timeline.so) to load instead.
_LIB_PATH = os.environ.get("PHASEMASK_LIBRARY") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libphasemask.so")

# Every function the header declares, with (restype, argtypes).
_c_handle = ctypes.c_void_p
_SIGNATURES = {
    "phasemask_create": (ctypes.c_int, [ctypes.POINTER(_c_handle), ctypes.c_int, ctypes.c_int,
                                        ctypes.c_uint, ctypes.c_void_p]),
    "phasemask_destroy": (ctypes.c_int, [_c_handle]),
    "phasemask_set_stream": (ctypes.c_int, [_c_handle, ctypes.c_void_p]),
    "phasemask_set_illumination": (ctypes.c_int, [_c_handle, ctypes.c_void_p]),
    "phasemask_solve": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "phasemask_solve_field": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "phasemask_solve_noalloc": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "phasemask_solve_many": (ctypes.c_int, [_c_handle, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "phasemask_workspace_size": (ctypes.c_size_t, [_c_handle, ctypes.c_int]),
    "phasemask_set_workspace": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_size_t]),
    "phasemask_solve_raar": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    "phasemask_error": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "phasemask_fft2": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "phasemask_create_batched": (ctypes.c_int, [ctypes.POINTER(_c_handle), ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                                ctypes.c_uint, ctypes.c_void_p]),
    "phasemask_solve_batched": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "phasemask_intensity_loss_fwd": (ctypes.c_int, [_c_handle, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_void_p]),
    "phasemask_intensity_loss_bwd": (ctypes.c_int, [_c_handle, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_void_p]),
    "phasemask_batch_schedule": (ctypes.c_int, [_c_handle]),
    "phasemask_batch_config": (ctypes.c_int, [_c_handle, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "phasemask_solve_adam": (ctypes.c_int, [_c_handle, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    "phasemask_initial_phase": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]),
    "phasemask_physical_error": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_void_p]),
    "phasemask_time_passes": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_float),
                                             ctypes.POINTER(ctypes.c_float)]),
    "phasemask_probe_exchange": (ctypes.c_int, [_c_handle, ctypes.c_void_p, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_float)]),
    "phasemask_workspace_bytes": (ctypes.c_size_t, [_c_handle]),
    "phasemask_probe_dft16": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.c_int, ctypes.POINTER(ctypes.c_float)]),
    "phasemask_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "phasemask_last_error": (ctypes.c_char_p, []),
}

PM_FLAG_NO_GRAPH = 0x1
PM_FLAG_NO_TUNE = 0x2
PM_FLAG_VALIDATE = 0x4

STATUS = {0: "PM_OK", -1: "PM_EINVAL", -2: "PM_EUNSUPPORTED", -3: "PM_ENOMEM",
          -4: "PM_EDEVICE", -5: "PM_ESTATE"}


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is not built; run `python -m paper_1302_0120_amd.build` (HIP, gfx950)")
    lib = ctypes.CDLL(_LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class PhaseMaskError(RuntimeError):
    """A non-PM_OK status from the library."""

    def __init__(self, status: int, call: str):
        self.status = status
        why = lib.phasemask_last_error().decode(errors="replace")
        super().__init__(f"{call}: {STATUS.get(status, status)}: {why}")


def _check(status: int, call: str):
    if status != 0:
        raise PhaseMaskError(status, call)


def _dev_ptr(t: torch.Tensor, dtype, shape, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


class PhaseMask:
    """One plan for height x width masks on one device (see include/phasemask.h)."""

    def __init__(self, height: int, width: int, flags: int = 0, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.height, self.width = int(height), int(width)
        self.shape = (self.height, self.width)
        h = _c_handle()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _check(lib.phasemask_create(ctypes.byref(h), self.height, self.width, flags, stream),
                   "phasemask_create")
        self._h = h

    def _stream(self):
        if self._h is None:
            raise PhaseMaskError(-5, "use after close")
        _check(lib.phasemask_set_stream(self._h, torch.cuda.current_stream(self.device).cuda_stream),
               "phasemask_set_stream")

    def set_illumination(self, p: torch.Tensor | None):
        """Illumination amplitude p of Eq. 1 for the later solves and error
        evaluations (float32 [height, width], p >= 0), or None for p = 1."""
        pp = None if p is None else _dev_ptr(p, torch.float32, self.shape, "illumination")
        self._stream()
        _check(lib.phasemask_set_illumination(self._h, pp), "phasemask_set_illumination")
        self._illum = p  # the copy is stream-ordered; keep the source alive meanwhile

    def solve(self, target: torch.Tensor, init_phase: torch.Tensor, n_iter: int,
              out: torch.Tensor | None = None, history: bool | torch.Tensor = True):
        """Run n_iter GS iterations; returns (phase, history or None)."""
        tp = _dev_ptr(target, torch.float32, self.shape, "target")
        pp = _dev_ptr(init_phase, torch.float32, self.shape, "init_phase")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        op = _dev_ptr(out, torch.float32, self.shape, "out")
        hist = None
        if isinstance(history, torch.Tensor):
            hist = history
        elif history:
            hist = torch.empty(2 * int(n_iter) + 1, dtype=torch.float64, device=self.device)
        hp = 0 if hist is None else _dev_ptr(hist, torch.float64, (2 * int(n_iter) + 1,), "history")
        self._stream()
        _check(lib.phasemask_solve(self._h, tp, pp, int(n_iter), op, hp or None), "phasemask_solve")
        return out, hist

    def solve_many(self, targets: torch.Tensor, init_phases: torch.Tensor, n_iter: int,
                   out: torch.Tensor | None = None, history: bool | torch.Tensor = True):
        """n_iter GS iterations on a uniform batch: float32 [batch, height,
        width] targets and initial phases; returns (phases [batch, height,
        width], histories [batch, 2 n_iter + 1] or None)."""
        if targets.dim() != 3:
            raise ValueError("targets must be [batch, height, width]")
        b = int(targets.shape[0])
        shape = (b,) + self.shape
        tp = _dev_ptr(targets, torch.float32, shape, "targets")
        pp = _dev_ptr(init_phases, torch.float32, shape, "init_phases")
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        op = _dev_ptr(out, torch.float32, shape, "out")
        hist = None
        if isinstance(history, torch.Tensor):
            hist = history
        elif history:
            hist = torch.empty((b, 2 * int(n_iter) + 1), dtype=torch.float64, device=self.device)
        hp = 0 if hist is None else _dev_ptr(hist, torch.float64, (b, 2 * int(n_iter) + 1), "history")
        self._stream()
        _check(lib.phasemask_solve_many(self._h, b, tp, pp, int(n_iter), op, hp or None), "phasemask_solve_many")
        return out, hist

    def solve_noalloc(self, target: torch.Tensor, init_phase: torch.Tensor, n_iter: int,
                      out: torch.Tensor, history: torch.Tensor | None = None):
        """phasemask_solve in the library's per-GPU scratch array: the library
        allocates nothing, so the caller passes the output (and history)
        buffers.  Returns (out, history)."""
        tp = _dev_ptr(target, torch.float32, self.shape, "target")
        pp = _dev_ptr(init_phase, torch.float32, self.shape, "init_phase")
        op = _dev_ptr(out, torch.float32, self.shape, "out")
        hp = 0 if history is None else _dev_ptr(history, torch.float64, (2 * int(n_iter) + 1,), "history")
        self._stream()
        _check(lib.phasemask_solve_noalloc(self._h, tp, pp, int(n_iter), op, hp or None), "phasemask_solve_noalloc")
        return out, history

    def solve_field(self, target: torch.Tensor, init_field: torch.Tensor, n_iter: int,
                    out: torch.Tensor | None = None, history: bool | torch.Tensor = True):
        """n_iter GS iterations from the complex field init_field (complex64
        [height, width]); returns (u^n as complex64, history or None)."""
        tp = _dev_ptr(target, torch.float32, self.shape, "target")
        fp = _dev_ptr(init_field, torch.complex64, self.shape, "init_field")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.complex64, device=self.device)
        op = _dev_ptr(out, torch.complex64, self.shape, "out")
        hist = None
        if isinstance(history, torch.Tensor):
            hist = history
        elif history:
            hist = torch.empty(2 * int(n_iter) + 1, dtype=torch.float64, device=self.device)
        hp = 0 if hist is None else _dev_ptr(hist, torch.float64, (2 * int(n_iter) + 1,), "history")
        self._stream()
        _check(lib.phasemask_solve_field(self._h, tp, fp, int(n_iter), op, hp or None), "phasemask_solve_field")
        return out, hist

    def workspace_size(self, n_iter: int) -> int:
        """Bytes a caller-owned workspace needs for solves of up to n_iter iterations."""
        if self._h is None:
            raise PhaseMaskError(-5, "use after close")
        return int(lib.phasemask_workspace_size(self._h, int(n_iter)))

    def set_workspace(self, buf: torch.Tensor | None):
        """Work in the caller's device buffer `buf` (a contiguous uint8 tensor,
        256-byte aligned, at least workspace_size(n) bytes) from now on, or in
        plan-owned buffers again with None.  The tensor is kept referenced here
        while the plan uses it."""
        if self._h is None:
            raise PhaseMaskError(-5, "use after close")
        self._stream()
        if buf is None:
            _check(lib.phasemask_set_workspace(self._h, None, 0), "phasemask_set_workspace")
        else:
            if not (buf.is_cuda and buf.dtype == torch.uint8 and buf.is_contiguous()):
                raise ValueError("workspace must be a contiguous uint8 device tensor")
            _check(lib.phasemask_set_workspace(self._h, buf.data_ptr(), buf.numel()), "phasemask_set_workspace")
        self._ws = buf

    def solve_raar(self, target: torch.Tensor, init_phase: torch.Tensor, n_iter: int, beta: float,
                   out: torch.Tensor | None = None, history: bool = True):
        """RAAR (relaxed averaged alternating reflections); returns (phase of
        the shadow P_S x^n, history [E_F(x^0) .. E_F(x^{n-1}), E_F(P_S x^n)])."""
        tp = _dev_ptr(target, torch.float32, self.shape, "target")
        pp = _dev_ptr(init_phase, torch.float32, self.shape, "init_phase")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        op = _dev_ptr(out, torch.float32, self.shape, "out")
        hist = torch.empty(int(n_iter) + 1, dtype=torch.float64, device=self.device) if history else None
        self._stream()
        _check(lib.phasemask_solve_raar(self._h, tp, pp, int(n_iter), float(beta), op,
                                        hist.data_ptr() if hist is not None else None),
               "phasemask_solve_raar")
        return out, hist

    def error(self, target: torch.Tensor, phase: torch.Tensor, out: torch.Tensor | None = None):
        """(E_F, G) of exp(i phase) as a float64 device tensor of 2 entries."""
        tp = _dev_ptr(target, torch.float32, self.shape, "target")
        pp = _dev_ptr(phase, torch.float32, self.shape, "phase")
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=self.device)
        ep = _dev_ptr(out, torch.float64, (2,), "errors")
        self._stream()
        _check(lib.phasemask_error(self._h, tp, pp, ep), "phasemask_error")
        return out

    def initial_phase(self, target: torch.Tensor, t_dark: float = 3e-4, out: torch.Tensor | None = None):
        """The paper's initial mask: phase of the back-propagated 1-bit target."""
        tp = _dev_ptr(target, torch.float32, self.shape, "target")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        op = _dev_ptr(out, torch.float32, self.shape, "out")
        self._stream()
        _check(lib.phasemask_initial_phase(self._h, tp, float(t_dark), op), "phasemask_initial_phase")
        return out

    def physical_error(self, target: torch.Tensor, phase: torch.Tensor, t_lit: float = 0.1,
                       t_dark: float = 3e-4, out: torch.Tensor | None = None):
        """(E_lit, E_dark) of Eq. 8 as a float64 device tensor of 2 entries."""
        tp = _dev_ptr(target, torch.float32, self.shape, "target")
        pp = _dev_ptr(phase, torch.float32, self.shape, "phase")
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=self.device)
        ep = _dev_ptr(out, torch.float64, (2,), "errors")
        self._stream()
        _check(lib.phasemask_physical_error(self._h, tp, pp, float(t_lit), float(t_dark), ep),
               "phasemask_physical_error")
        return out

    def fft2(self, x: torch.Tensor, inverse: bool = False, out: torch.Tensor | None = None):
        """Unnormalised complex64 2-D DFT (inverse without 1/N)."""
        xp = _dev_ptr(x, torch.complex64, self.shape, "x")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.complex64, device=self.device)
        op = _dev_ptr(out, torch.complex64, self.shape, "out")
        self._stream()
        _check(lib.phasemask_fft2(self._h, xp, op, 1 if inverse else 0), "phasemask_fft2")
        return out

    def intensity_loss_fwd(self, phase: torch.Tensor, target_intensity: torch.Tensor):
        """Per-sample loss (float64 [batch]) and the saved buffer for backward."""
        b = phase.shape[0] if phase.dim() == 3 else 1
        shp = (b, *self.shape) if phase.dim() == 3 else self.shape
        pp = _dev_ptr(phase, torch.float32, shp, "phase")
        ip = _dev_ptr(target_intensity, torch.float32, shp, "target_intensity")
        loss = torch.empty(b, dtype=torch.float64, device=self.device)
        saved = torch.empty((b, *self.shape), dtype=torch.complex64, device=self.device)
        self._stream()
        _check(lib.phasemask_intensity_loss_fwd(self._h, b, pp, ip, loss.data_ptr(), saved.data_ptr()),
               "phasemask_intensity_loss_fwd")
        return loss, saved

    def intensity_loss_bwd(self, phase: torch.Tensor, saved: torch.Tensor, grad_loss: torch.Tensor):
        b = saved.shape[0]
        shp = (b, *self.shape) if phase.dim() == 3 else self.shape
        pp = _dev_ptr(phase, torch.float32, shp, "phase")
        sp = _dev_ptr(saved, torch.complex64, (b, *self.shape), "saved")
        gl = _dev_ptr(grad_loss, torch.float64, (b,), "grad_loss")
        grad = torch.empty_like(phase)
        self._stream()
        _check(lib.phasemask_intensity_loss_bwd(self._h, b, pp, sp, gl, grad.data_ptr()),
               "phasemask_intensity_loss_bwd")
        return grad

    def solve_adam(self, target_intensity: torch.Tensor, init_phase: torch.Tensor, n_steps: int, lr: float,
                   betas=(0.9, 0.999), eps: float = 1e-8, out: torch.Tensor | None = None,
                   history: bool = True):
        """n_steps of Adam on the intensity loss for phases [B][H][W] (or
        [H][W]); returns (phase, losses [n_steps + 1][B] float64 or None)."""
        b = init_phase.shape[0] if init_phase.dim() == 3 else 1
        shp = (b, *self.shape) if init_phase.dim() == 3 else self.shape
        ip = _dev_ptr(target_intensity, torch.float32, shp, "target_intensity")
        pp = _dev_ptr(init_phase, torch.float32, shp, "init_phase")
        if out is None:
            out = torch.empty(shp, dtype=torch.float32, device=self.device)
        op = _dev_ptr(out, torch.float32, shp, "out")
        hist = torch.empty((int(n_steps) + 1, b), dtype=torch.float64, device=self.device) if history else None
        self._stream()
        _check(lib.phasemask_solve_adam(self._h, b, ip, pp, int(n_steps), float(lr), float(betas[0]),
                                        float(betas[1]), float(eps), op, 0 if hist is None else hist.data_ptr()),
               "phasemask_solve_adam")
        return out, hist

    def time_passes(self, target: torch.Tensor, phase: torch.Tensor, reps: int = 100):
        """(column-pass ms, row-pass ms): average kernel durations over `reps`
        iterations, from events recorded by the launches themselves."""
        tp = _dev_ptr(target, torch.float32, self.shape, "target")
        pp = _dev_ptr(phase, torch.float32, self.shape, "phase")
        c, r = ctypes.c_float(), ctypes.c_float()
        self._stream()
        _check(lib.phasemask_time_passes(self._h, tp, pp, int(reps), ctypes.byref(c), ctypes.byref(r)),
               "phasemask_time_passes")
        return float(c.value), float(r.value)

    def probe_exchange(self, buffer: torch.Tensor, reps: int = 100) -> float:
        """ms for `reps` pairs of this plan's column and row passes in copy
        mode (the iterate exchange without its arithmetic) on `buffer`, a
        complex64 [height, width] device tensor that is copied in place and
        comes back unchanged."""
        bp = _dev_ptr(buffer, torch.complex64, self.shape, "buffer")
        ms = ctypes.c_float()
        self._stream()
        _check(lib.phasemask_probe_exchange(self._h, bp, int(reps), ctypes.byref(ms)), "phasemask_probe_exchange")
        return float(ms.value)

    @property
    def workspace_bytes(self) -> int:
        return int(lib.phasemask_workspace_bytes(self._h)) if self._h is not None else 0

    def close(self):
        if getattr(self, "_h", None) is not None:
            _check(lib.phasemask_destroy(self._h), "phasemask_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedPhaseMask:
    """One plan for a batch of masks of uneven sizes (powers of two in
    [64, 1024] per side), solved together (see include/phasemask.h)."""

    def __init__(self, shapes, flags: int = 0, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self.shapes = [(int(h), int(w)) for h, w in shapes]
        n = len(self.shapes)
        hs = (ctypes.c_int * n)(*[h for h, _ in self.shapes])
        ws = (ctypes.c_int * n)(*[w for _, w in self.shapes])
        h = _c_handle()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _check(lib.phasemask_create_batched(ctypes.byref(h), n, hs, ws, flags, stream),
                   "phasemask_create_batched")
        self._h = h
        self._ptr_cache: dict = {}

    def _ptr_array(self, tensors, dtype, name):
        ptrs = tuple(_dev_ptr(t, dtype, shp, f"{name}[{i}]")
                     for i, (t, shp) in enumerate(zip(tensors, self.shapes)))
        arr = self._ptr_cache.get(ptrs)
        if arr is None:
            if len(self._ptr_cache) > 64:
                self._ptr_cache.clear()
            arr = torch.tensor(ptrs, dtype=torch.int64).to(self.device)
            self._ptr_cache[ptrs] = arr
        return arr

    def solve(self, targets, init_phases, n_iter: int, outs=None, final_err: bool | torch.Tensor = True):
        """n_iter GS iterations for every mask; returns (list of phases,
        final E_F per mask as a float64 device tensor, or None)."""
        if len(targets) != len(self.shapes) or len(init_phases) != len(self.shapes):
            raise ValueError(f"expected {len(self.shapes)} targets and phases")
        if outs is None:
            outs = [torch.empty(shp, dtype=torch.float32, device=self.device) for shp in self.shapes]
        tp = self._ptr_array(targets, torch.float32, "targets")
        pp = self._ptr_array(init_phases, torch.float32, "init_phases")
        op = self._ptr_array(outs, torch.float32, "outs")
        err = None
        if isinstance(final_err, torch.Tensor):
            err = final_err
        elif final_err:
            err = torch.empty(len(self.shapes), dtype=torch.float64, device=self.device)
        ep = 0 if err is None else _dev_ptr(err, torch.float64, (len(self.shapes),), "final_err")
        if self._h is None:
            raise PhaseMaskError(-5, "use after close")
        _check(lib.phasemask_set_stream(self._h, torch.cuda.current_stream(self.device).cuda_stream),
               "phasemask_set_stream")
        _check(lib.phasemask_solve_batched(self._h, tp.data_ptr(), pp.data_ptr(), int(n_iter),
                                           op.data_ptr(), ep or None), "phasemask_solve_batched")
        return outs, err

    @property
    def schedule(self) -> int:
        return int(lib.phasemask_batch_schedule(self._h))

    @property
    def config(self):
        """(FFT schedule, concurrent chains, group budget in bytes) the tuner chose."""
        sc, ch, gb = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(lib.phasemask_batch_config(self._h, ctypes.byref(sc), ctypes.byref(ch), ctypes.byref(gb)),
               "phasemask_batch_config")
        return int(sc.value), int(ch.value), int(gb.value)

    @property
    def workspace_bytes(self) -> int:
        return int(lib.phasemask_workspace_bytes(self._h)) if self._h is not None else 0

    def close(self):
        if getattr(self, "_h", None) is not None:
            _check(lib.phasemask_destroy(self._h), "phasemask_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_PLANS: dict = {}


def plan_for(height: int, width: int, device=None) -> PhaseMask:
    """A cached plan per (device, height, width)."""
    dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    key = (dev, int(height), int(width))
    if key not in _PLANS:
        _PLANS[key] = PhaseMask(height, width, device=torch.device("cuda", dev))
    return _PLANS[key]


class IntensityLoss(torch.autograd.Function):
    """loss_b = sum_k (|F exp(i phase_b)|_k^2 - I_{b,k})^2 with unitary F, for
    phase [H][W] or [B][H][W] (float32, device).  Returns float64 losses
    (scalar for a 2-D phase, [B] otherwise); backward runs the hand-written
    adjoint kernel."""

    @staticmethod
    def forward(ctx, phase, target_intensity):
        phase = phase.contiguous()
        h, w = phase.shape[-2], phase.shape[-1]
        plan = plan_for(h, w, phase.device)
        loss, saved = plan.intensity_loss_fwd(phase, target_intensity.contiguous())
        ctx.save_for_backward(phase, saved)
        ctx.plan = plan
        return loss if phase.dim() == 3 else loss[0]

    @staticmethod
    def backward(ctx, grad_loss):
        phase, saved = ctx.saved_tensors
        g = grad_loss.reshape(-1).to(torch.float64).contiguous()
        if g.numel() == 1 and saved.shape[0] > 1:
            g = g.expand(saved.shape[0]).contiguous()
        return ctx.plan.intensity_loss_bwd(phase, saved, g), None


def intensity_loss(phase: torch.Tensor, target_intensity: torch.Tensor) -> torch.Tensor:
    return IntensityLoss.apply(phase, target_intensity)


class AdamIntensityStep:
    """Gradient-based phase optimisation on the intensity loss: one step is
    the per-sample losses loss_b = intensity_loss(phase_b, I_b), the
    gradient of sum_b loss_b (the adjoint kernel with unit upstream
    gradients, as autograd would pass them) and a fused Adam update of
    `phase` (a leaf float32 tensor with requires_grad, [B][H][W] or [H][W]).

    The step runs on a plan of its own, so nothing else can regrow the
    buffers it uses.  `warmup` eager steps first size the plan's partial
    sums and create the optimizer state; they are then undone (phase and
    optimizer state restored).  With capture=True they run on the step's own
    stream (so nothing inside the graph allocates through the library or
    switches streams), and the whole step (loss, gradient, Adam) is then
    recorded once into a graph on that stream: every step() replays it, so a
    step costs device time only.  Step k of a captured run equals step k of
    an eager one, bitwise.  step() returns the step's per-sample losses (a tensor the
    graph rewrites on each replay); phase.grad holds the step's gradient."""

    def __init__(self, phase: torch.Tensor, target_intensity: torch.Tensor, lr: float,
                 betas=(0.9, 0.999), eps: float = 1e-8, capture: bool = True, warmup: int = 2):
        if not (phase.is_leaf and phase.requires_grad and phase.is_cuda and phase.dtype == torch.float32):
            raise ValueError("phase must be a float32 device leaf tensor with requires_grad")
        if not phase.is_contiguous():
            raise ValueError("phase must be contiguous")
        self.phase = phase
        self.target = target_intensity.contiguous()
        batch = phase.shape[0] if phase.dim() == 3 else 1
        self.plan = PhaseMask(phase.shape[-2], phase.shape[-1], device=phase.device)
        self.ones = torch.ones(batch, dtype=torch.float64, device=phase.device)
        self.opt = torch.optim.Adam([phase], lr=lr, betas=betas, eps=eps, fused=True, capturable=True)
        self.graph = None
        self.loss = None
        cur = torch.cuda.current_stream(phase.device)
        self.stream = torch.cuda.Stream(device=phase.device) if capture else cur
        start = phase.detach().clone()
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            for _ in range(warmup):
                self._eager()
            with torch.no_grad():
                phase.copy_(start)
            for st in self.opt.state.values():
                for v in st.values():
                    if isinstance(v, torch.Tensor):
                        v.zero_()
        cur.wait_stream(self.stream)
        if capture:
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph, stream=self.stream):
                self.loss = self._eager()

    def _eager(self):
        with torch.no_grad():
            p = self.phase.detach()
            loss, saved = self.plan.intensity_loss_fwd(p, self.target)
            self.phase.grad = self.plan.intensity_loss_bwd(p, saved, self.ones)
        self.opt.step()
        return loss

    def step(self) -> torch.Tensor:
        if self.graph is None:
            return self._eager()
        self.graph.replay()
        return self.loss


def probe_dft16(matrix_units: bool, x: torch.Tensor, reps: int):
    """One 16-point DFT stage over x (complex64, waves * 1024 points) on the
    vector ALUs or as FP32 matrix products, reps times; returns (out, ms)."""
    if not (x.is_cuda and x.dtype == torch.complex64 and x.is_contiguous() and x.dim() == 1):
        raise ValueError("x must be a contiguous 1-D complex64 device tensor")
    if x.numel() % 4096 != 0:
        raise ValueError("x must hold a multiple of 4096 points")
    out = torch.empty_like(x)
    ms = ctypes.c_float()
    torch.cuda.synchronize(x.device)
    _check(lib.phasemask_probe_dft16(int(bool(matrix_units)), x.data_ptr(), out.data_ptr(), x.numel() // 1024,
                                     int(reps), ctypes.byref(ms)), "phasemask_probe_dft16")
    return out, float(ms.value)


def solve(target: torch.Tensor, init_phase: torch.Tensor, n_iter: int, history: bool = True):
    """GS phase mask for `target` from `init_phase` (device float32 [H][W])."""
    p = plan_for(target.shape[0], target.shape[1], target.device)
    return p.solve(target, init_phase, n_iter, history=history)
