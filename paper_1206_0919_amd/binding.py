"""ctypes binding of libshasta.so (the C ABI of include/shasta.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Functions keep the C names.  PyTorch provides device
memory (the caller-owned workspace and the FP64 field arrays) and the stream.

The library must have been built (``python -m paper_1206_0919_amd.build``);
importing this module without it raises immediately, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SHASTA_LIB") or os.path.join(HERE, "lib", "libshasta.so")

OK, EINVAL, ESTATE, EWORKSPACE, EHIP, ENONFINITE, ENOCONVERGE = range(7)
FP64, FP32_MIXED = 0, 1
BC_OUTFLOW = 0
EOS_IDEAL, EOS_BAG, EOS_TABLE, EOS_BARYON = 0, 1, 2, 3
FIELDS = ("E", "Mx", "My", "Mz", "R", "e", "p", "vx", "vy", "vz", "n")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_1206_0919_amd.build` (no CPU fallback exists)")

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_h = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)

_SIGS = {
    "shasta_create": ([ctypes.POINTER(_h), ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                       ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp], ctypes.c_int),
    "shasta_workspace_bytes": ([_h, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "shasta_bind_workspace": ([_h, _vp, ctypes.c_size_t], ctypes.c_int),
    "shasta_set_eos": ([_h, ctypes.c_int, _dp, ctypes.c_int], ctypes.c_int),
    "shasta_write_primitive": ([_h, ctypes.c_int] + [_vp] * 5, ctypes.c_int),
    "shasta_write_conserved": ([_h, ctypes.c_int] + [_vp] * 5, ctypes.c_int),
    "shasta_set_step_index": ([_h, ctypes.c_int64], ctypes.c_int),
    "shasta_get_step_index": ([_h, _i64p], ctypes.c_int),
    "shasta_step": ([_h, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "shasta_step_noalloc": ([_h, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "shasta_read_field": ([_h, ctypes.c_int, ctypes.c_int, _vp], ctypes.c_int),
    "shasta_reduce": ([_h, ctypes.c_int, _dp, _i64p], ctypes.c_int),
    "shasta_destroy": ([_h], ctypes.c_int),
    "shasta_last_error": ([_h], ctypes.c_char_p),
    "shasta_status_str": ([ctypes.c_int], ctypes.c_char_p),
    "shasta_set_tiles": ([_h, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "shasta_set_persistent": ([_h, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "shasta_get_tiles": ([_h, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                          ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "shasta_get_persistent": ([_h, ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "shasta_autotune": ([_h, ctypes.c_double, ctypes.c_int], ctypes.c_int),
    "shasta_forget_tuning": ([], ctypes.c_int),
    "shasta_set_antidiffusion": ([_h, ctypes.c_double], ctypes.c_int),
    "shasta_set_graph": ([_h, ctypes.c_int], ctypes.c_int),
    "shasta_set_profiling": ([_h, ctypes.c_int], ctypes.c_int),
    "shasta_read_profile": ([_h, _dp, _i64p], ctypes.c_int),
    "shasta_stream_copy": ([_vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "shasta_march_copy": ([_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                           ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp], ctypes.c_int),
    "shasta_selftest_math": ([_vp, _vp, ctypes.c_int, ctypes.c_int, _vp], ctypes.c_int),
    "shasta_selftest_recover": ([_h, _vp, _vp, ctypes.c_int], ctypes.c_int),
}
EXPORTS = tuple(_SIGS)

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    globals()[_name] = _f


class ShastaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"[{status}] {msg}")
        self.status = status


def _check(h, status):
    if status != OK:
        msg = shasta_last_error(h) if h else shasta_status_str(status)
        raise ShastaError(status, (msg or b"").decode())
    return status


class Shasta:
    """Convenience wrapper: a handle plus a torch-owned device workspace.

    dims: list of (nx, ny, nz) per event.  All field arrays handed in or out
    are torch float64 CUDA tensors of shape (nz, ny, nx).
    """

    def __init__(self, dims, dx, precision=FP64, stream=None, eos=None, device=None):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda", torch.cuda.current_device()) \
            if device is None else torch.device(device)
        if isinstance(dims[0], int):
            dims = [tuple(dims)]
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.dx = float(dx)
        self.precision = precision
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        arr = (ctypes.c_int32 * (3 * len(self.dims)))(*[v for d in self.dims for v in d])
        h = _h()
        _check(None, shasta_create(ctypes.byref(h), len(self.dims), arr, self.dx,
                                   precision, BC_OUTFLOW, _vp(self.stream.cuda_stream)))
        self.h = h
        nbytes = ctypes.c_size_t()
        _check(self.h, shasta_workspace_bytes(self.h, ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self.ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        _check(self.h, shasta_bind_workspace(self.h, _vp(self.ws.data_ptr()),
                                             self.workspace_bytes))
        if eos is not None:
            self.set_eos(*eos)

    # -- lifecycle
    def close(self):
        if getattr(self, "h", None):
            shasta_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls
    def set_eos(self, kind, params=()):
        params = [float(x) for x in params]
        arr = (ctypes.c_double * max(1, len(params)))(*params)
        _check(self.h, shasta_set_eos(self.h, int(kind), arr, len(params)))

    def set_eos_table(self, e_nodes, p_nodes):
        """Tabled EOS: node energy densities (from 0, increasing) and pressures."""
        self.set_eos(EOS_TABLE, list(e_nodes) + list(p_nodes))

    def _dev(self, a, ev):
        t = self.torch
        nx, ny, nz = self.dims[ev]
        if not isinstance(a, t.Tensor):
            a = t.as_tensor(a)
        a = a.to(device=self.device, dtype=t.float64).contiguous()
        assert a.numel() == nx * ny * nz
        return a

    def write_primitive(self, ev, e, vx, vy, vz, n):
        arrs = [self._dev(a, ev) for a in (e, vx, vy, vz, n)]
        self.torch.cuda.synchronize(self.device)
        _check(self.h, shasta_write_primitive(self.h, ev, *[_vp(a.data_ptr()) for a in arrs]))

    def write_conserved(self, ev, E, Mx, My, Mz, R):
        arrs = [self._dev(a, ev) for a in (E, Mx, My, Mz, R)]
        self.torch.cuda.synchronize(self.device)
        _check(self.h, shasta_write_conserved(self.h, ev, *[_vp(a.data_ptr()) for a in arrs]))

    def step(self, dt, nsteps=1):
        _check(self.h, shasta_step(self.h, float(dt), int(nsteps)))

    def step_noalloc(self, dt, nsteps=1):
        _check(self.h, shasta_step_noalloc(self.h, float(dt), int(nsteps)))

    def set_step_index(self, k):
        _check(self.h, shasta_set_step_index(self.h, int(k)))

    def step_index(self):
        k = ctypes.c_int64()
        _check(self.h, shasta_get_step_index(self.h, ctypes.byref(k)))
        return k.value

    def read_field(self, ev, field):
        f = FIELDS.index(field) if isinstance(field, str) else int(field)
        nx, ny, nz = self.dims[ev]
        out = self.torch.empty((nz, ny, nx), dtype=self.torch.float64, device=self.device)
        _check(self.h, shasta_read_field(self.h, ev, f, _vp(out.data_ptr())))
        return out

    def read_conserved(self, ev=0):
        return [self.read_field(ev, q) for q in range(5)]

    def reduce(self, ev=0):
        out = (ctypes.c_double * 12)()
        cnt = (ctypes.c_int64 * 4)()
        st = shasta_reduce(self.h, ev, out, cnt)
        res = dict(sums=list(out[0:5]), outflow=list(out[5:10]), max_eps=out[10],
                   t=out[11], clamp=cnt[0], floor=cnt[1], noconv=cnt[2],
                   nonfinite=cnt[3], status=st)
        if st not in (OK, ENONFINITE, ENOCONVERGE):
            _check(self.h, st)
        return res

    def set_tiles(self, axis, p0, p1=0):
        _check(self.h, shasta_set_tiles(self.h, axis, p0, p1))

    def set_persistent(self, axis, enable):
        _check(self.h, shasta_set_persistent(self.h, axis, int(bool(enable))))

    def get_tiles(self, axis):
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(self.h, shasta_get_tiles(self.h, axis, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def get_persistent(self, axis):
        e = ctypes.c_int()
        _check(self.h, shasta_get_persistent(self.h, axis, ctypes.byref(e)))
        return bool(e.value)

    def decomposition(self):
        """Per axis (p0, p1, persistent): what shasta_autotune chose."""
        return [(*self.get_tiles(a), int(self.get_persistent(a))) for a in range(3)]

    def set_decomposition(self, dec):
        for a, (p0, p1, pers) in enumerate(dec):
            self.set_tiles(a, p0, p1)
            self.set_persistent(a, pers)

    def autotune(self, dt, reps=3):
        _check(self.h, shasta_autotune(self.h, float(dt), int(reps)))

    def set_antidiffusion(self, diff):
        _check(self.h, shasta_set_antidiffusion(self.h, float(diff)))

    def selftest_recover(self, cells):
        """cells: (n, 5) float64 tensor of (E, Mx, My, Mz, R) -> (n, 4) tensor of
        (e, p, |v|, clamped + 2 floored) from the device recovery."""
        t = self.torch
        c = cells.to(device=self.device, dtype=t.float64).contiguous()
        out = t.empty((c.shape[0], 4), dtype=t.float64, device=self.device)
        _check(self.h, shasta_selftest_recover(self.h, _vp(c.data_ptr()), _vp(out.data_ptr()),
                                               c.shape[0]))
        return out

    def set_graph(self, enable):
        _check(self.h, shasta_set_graph(self.h, int(bool(enable))))

    def set_profiling(self, enable):
        _check(self.h, shasta_set_profiling(self.h, int(bool(enable))))

    def read_profile(self):
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int64 * 4)()
        _check(self.h, shasta_read_profile(self.h, ms, n))
        return list(ms), list(n)


def forget_tuning():
    _check(None, shasta_forget_tuning())


def _check_device_buffers(nbytes, *tensors):
    for t in tensors:
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("device buffers must be contiguous GPU tensors")
        if t.numel() * t.element_size() < nbytes:
            raise ValueError(f"buffer of {t.numel() * t.element_size()} bytes, "
                             f"the copy needs {nbytes}")


def stream_copy(src, dst, nbytes, stream):
    _check_device_buffers(int(nbytes), src, dst)
    st = shasta_stream_copy(_vp(src.data_ptr()), _vp(dst.data_ptr()), int(nbytes),
                            _vp(stream.cuda_stream))
    if st != OK:
        raise ShastaError(st, "stream copy failed")


def march_copy(src, dst, dims, pitch, axis, seg_len, precision, stream):
    """Copy src to dst (five fields of dims = (nx, ny, nz), field q at
    element q * pitch) with the memory pattern of the y (axis 1) or z
    (axis 2) sweep and no arithmetic."""
    nx, ny, nz = (int(d) for d in dims)
    if src.dtype != dst.dtype or (precision == FP64) != (src.element_size() == 8):
        raise ValueError("march copy: float64 buffers for FP64, float32 for FP32_MIXED")
    _check_device_buffers((4 * int(pitch) + nx * ny * nz) * src.element_size(), src, dst)
    st = shasta_march_copy(_vp(src.data_ptr()), _vp(dst.data_ptr()), nx, ny, nz, int(pitch),
                           int(axis), int(seg_len), int(precision), _vp(stream.cuda_stream))
    if st != OK:
        raise ShastaError(st, "march copy failed")


def selftest_math(inp, out, which, stream):
    st = shasta_selftest_math(_vp(inp.data_ptr()), _vp(out.data_ptr()), inp.numel(),
                              int(which), _vp(stream.cuda_stream))
    if st != OK:
        raise ShastaError(st, "selftest failed")
