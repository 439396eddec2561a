"""ctypes binding of liblmfmm.so (argument marshalling only).

Every numerical step runs in the HIP library; this module passes device
pointers of torch tensors and the current HIP stream through the C ABI of
``include/lmfmm.h``.  If the library is missing the first call raises: there
is no CPU fallback.

Layouts (identical to the C ABI):
  * coordinates: float64 tensors of shape (2, n) on the GPU (row 0 x, row 1 y);
  * densities: complex128 (FP64 path) or complex64 (mixed path) tensors of
    shape (nrhs, n) on the GPU.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblmfmm.so")

OK, EINVAL, EDOMAIN, ENOMEM, EHIP, ETOL, ENODEV = 0, -1, -2, -3, -4, -5, -6
C128, C64_MIXED = 0, 1

_lib = None


class LMFMMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lmfmm status {status}: {msg}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("order", ctypes.c_int * 32), ("root_x_lo", ctypes.c_double),
                ("root_width", ctypes.c_double), ("m2l_pairs", ctypes.c_int64),
                ("leaves_src", ctypes.c_int64), ("leaves_tgt", ctypes.c_int64), ("near_nodes_mid", ctypes.c_int),
                ("near_nodes_ray", ctypes.c_int), ("m2l_classes", ctypes.c_int), ("m2l_nodes", ctypes.c_int64),
                ("table_seconds", ctypes.c_double), ("kernel_flops", ctypes.c_double * 8),
                ("kernel_ms", ctypes.c_double * 8), ("kernel_launches", ctypes.c_int64 * 8),
                ("timed_applies", ctypes.c_int64), ("graph_applies", ctypes.c_int64)]


# kernel indices of Stats.kernel_* (LMFMM_K_* in lmfmm.h)
KERNELS = ["tree", "p2m", "m2m", "m2l", "near_sweep", "l2p_near", "l2l", "other"]


class BatchStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int), ("instances", ctypes.c_int), ("tuned_from_cache", ctypes.c_int),
                ("prepare_seconds", ctypes.c_double), ("kernel_flops", ctypes.c_double * 8),
                ("kernel_ms", ctypes.c_double * 8), ("kernel_launches", ctypes.c_int64 * 8),
                ("timed_applies", ctypes.c_int64), ("graph_applies", ctypes.c_int64)]


class Instance(ctypes.Structure):
    _fields_ = [("n_src", ctypes.c_int64), ("src_xy", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("n_tgt", ctypes.c_int64), ("tgt_xy", ctypes.c_void_p), ("u", ctypes.c_void_p)]


EXPORTS = ["lmfmm_create", "lmfmm_destroy", "lmfmm_set_option", "lmfmm_apply", "lmfmm_apply_noalloc",
           "lmfmm_apply_adjoint",
           "lmfmm_grad_coords", "lmfmm_direct", "lmfmm_get_stats", "lmfmm_sync_status", "lmfmm_batch_create",
           "lmfmm_batch_destroy", "lmfmm_batch_set_option", "lmfmm_batch_apply", "lmfmm_batch_get_choice",
           "lmfmm_batch_sync_status", "lmfmm_batch_get_stats",
           "lmfmm_status_string", "lmfmm_last_error"]


def lib():
    """Load liblmfmm.so (raises if it has not been built).

    torch is imported first: torch ships its own HIP runtime with the same
    soname (libamdhip64.so.7) as the system one the library links, and the
    first one loaded serves the whole process.  Loading torch's first keeps the
    runtime torch was built against, which both sides then share."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (see above)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1902_08250_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    I = ctypes.c_int
    D = ctypes.c_double
    L.lmfmm_create.argtypes = [ctypes.POINTER(D), D, I, D, ctypes.POINTER(P)]
    L.lmfmm_destroy.argtypes = [P]
    L.lmfmm_set_option.argtypes = [P, ctypes.c_char_p, ctypes.c_char_p]
    L.lmfmm_apply.argtypes = [P, I64, P, P, I64, P, P, I, I, P]
    L.lmfmm_direct.argtypes = [P, I64, P, P, I64, P, P, I, I, P]
    L.lmfmm_apply_noalloc.argtypes = [P, I64, P, P, I64, P, P, I, I, P]
    L.lmfmm_apply_adjoint.argtypes = [P, I64, P, I64, P, P, P, I, I, P]
    L.lmfmm_grad_coords.argtypes = [P, I64, P, P, I64, P, P, P, P, I, I, P]
    L.lmfmm_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    L.lmfmm_sync_status.argtypes = [P, P]
    L.lmfmm_batch_create.argtypes = [I, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I), I, D,
                                     ctypes.POINTER(P)]
    L.lmfmm_batch_destroy.argtypes = [P]
    L.lmfmm_batch_set_option.argtypes = [P, ctypes.c_char_p, ctypes.c_char_p]
    L.lmfmm_batch_apply.argtypes = [P, ctypes.POINTER(Instance), I, I, P]
    L.lmfmm_batch_get_choice.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(D),
                                         ctypes.POINTER(I)]
    L.lmfmm_batch_sync_status.argtypes = [P, P]
    L.lmfmm_batch_get_stats.argtypes = [P, ctypes.POINTER(BatchStats)]
    L.lmfmm_status_string.argtypes = [I]
    L.lmfmm_status_string.restype = ctypes.c_char_p
    L.lmfmm_last_error.argtypes = []
    L.lmfmm_last_error.restype = ctypes.c_char_p
    for name in EXPORTS[:-2]:
        getattr(L, name).restype = I
    _lib = L
    return L


def _check(rc):
    if rc != OK:
        L = lib()
        raise LMFMMError(rc, L.lmfmm_last_error().decode() or L.lmfmm_status_string(rc).decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _xy(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.dim() == 2
            and t.shape[0] == 2 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape (2, n)")
    return t


def _dens(t, n, name):
    import torch
    if t.dim() == 1:
        t = t.unsqueeze(0)
    if not (t.dim() == 2 and t.is_cuda and t.dtype in (torch.complex128, torch.complex64) and t.shape[1] == n):
        raise ValueError(f"{name} must be a complex64/complex128 CUDA tensor of shape (nrhs, {n})")
    return t.contiguous()


def _prec(dtype):
    import torch
    return C128 if dtype == torch.complex128 else C64_MIXED


def _out(t, nrhs, n, dtype, device, name):
    """A caller-supplied output: CUDA, contiguous, shape (nrhs, n), dtype of the densities
    (the C side cannot know buffer sizes, so a wrong buffer would be written out of bounds)."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous() and t.dtype == dtype
            and tuple(t.shape) == (nrhs, n) and t.device == device):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape ({nrhs}, {n}) on {device}")
    return t


class Plan:
    """A plan for one three-layer medium: k = (k1, k2, k3) complex, d > 0.

    component: the part of the scattered field applied (Section 3): "2t"
    (default, g_2^t: targets in the middle layer), "2b" (g_2^b, middle layer),
    "1s" (g_1^s, top layer), "3s" (g_3^s, bottom layer) or "impedance" (the
    impedance half-space of wave number k[0] with impedance alpha; targets
    above y = 0)."""

    def __init__(self, k, d, order=16, tol=1e-6, levels=None, fixed_order=False, domain=None, component=None,
                 alpha=None):
        L = lib()
        kk = [complex(v) for v in k]
        arr = (ctypes.c_double * 6)(kk[0].real, kk[0].imag, kk[1].real, kk[1].imag, kk[2].real, kk[2].imag)
        h = ctypes.c_void_p()
        _check(L.lmfmm_create(arr, float(d), int(order), float(tol), ctypes.byref(h)))
        self._h = h
        self.k, self.d, self.order, self.tol = tuple(kk), float(d), int(order), float(tol)
        if levels is not None:
            self.set_option("levels", str(levels))
        if fixed_order:
            self.set_option("fixed_order", "1")
        if domain is not None:
            self.set_option("domain", ",".join(repr(float(v)) for v in domain))
        if alpha is not None:
            self.set_option("alpha", repr(float(alpha)))
        if component is not None:
            self.set_option("component", component)

    def set_option(self, key, value):
        _check(lib().lmfmm_set_option(self._h, key.encode(), str(value).encode()))

    def close(self):
        if getattr(self, "_h", None):
            lib().lmfmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, src, q, tgt, out=None, stream=None):
        """u[r, i] = sum_j g_2^t(tgt_i, src_j) q[r, j]."""
        import torch
        src, tgt = _xy(src, "src"), _xy(tgt, "tgt")
        q = _dens(q, src.shape[1], "q")
        if out is not None:
            u = _out(out, q.shape[0], tgt.shape[1], q.dtype, q.device, "out")
        else:
            u = torch.empty((q.shape[0], tgt.shape[1]), dtype=q.dtype, device=q.device)
        _check(lib().lmfmm_apply(self._h, src.shape[1], src.data_ptr(), q.data_ptr(), tgt.shape[1], tgt.data_ptr(),
                                 u.data_ptr(), q.shape[0], _prec(q.dtype), _stream(stream)))
        return u

    def apply_noalloc(self, src, q, tgt, out, stream=None):
        """lmfmm_apply_noalloc: the apply without device allocation, into the given
        output (the plan's tables for this geometry must exist)."""
        src, tgt = _xy(src, "src"), _xy(tgt, "tgt")
        q = _dens(q, src.shape[1], "q")
        u = _out(out, q.shape[0], tgt.shape[1], q.dtype, q.device, "out")
        _check(lib().lmfmm_apply_noalloc(self._h, src.shape[1], src.data_ptr(), q.data_ptr(), tgt.shape[1],
                                         tgt.data_ptr(), u.data_ptr(), q.shape[0], _prec(q.dtype), _stream(stream)))
        return u

    def direct(self, src, q, tgt, stream=None):
        """Brute-force GPU direct sum (every pair by quadrature)."""
        import torch
        src, tgt = _xy(src, "src"), _xy(tgt, "tgt")
        q = _dens(q, src.shape[1], "q")
        u = torch.empty((q.shape[0], tgt.shape[1]), dtype=q.dtype, device=q.device)
        _check(lib().lmfmm_direct(self._h, src.shape[1], src.data_ptr(), q.data_ptr(), tgt.shape[1], tgt.data_ptr(),
                                  u.data_ptr(), q.shape[0], _prec(q.dtype), _stream(stream)))
        return u

    def apply_adjoint(self, src, tgt, w, stream=None):
        """v[r, j] = sum_i g_2^t(tgt_i, src_j) w[r, i] (transpose, no conjugation)."""
        import torch
        src, tgt = _xy(src, "src"), _xy(tgt, "tgt")
        w = _dens(w, tgt.shape[1], "w")
        v = torch.empty((w.shape[0], src.shape[1]), dtype=w.dtype, device=w.device)
        _check(lib().lmfmm_apply_adjoint(self._h, src.shape[1], src.data_ptr(), tgt.shape[1], tgt.data_ptr(),
                                         w.data_ptr(), v.data_ptr(), w.shape[0], _prec(w.dtype), _stream(stream)))
        return v

    def grad_coords(self, src, q, tgt, w, stream=None):
        """Gradients of L = Re sum w*u with respect to the coordinates: (dsrc, dtgt)."""
        import torch
        src, tgt = _xy(src, "src"), _xy(tgt, "tgt")
        q = _dens(q, src.shape[1], "q")
        w = _dens(w, tgt.shape[1], "w")
        dsrc = torch.empty_like(src)
        dtgt = torch.empty_like(tgt)
        _check(lib().lmfmm_grad_coords(self._h, src.shape[1], src.data_ptr(), q.data_ptr(), tgt.shape[1],
                                       tgt.data_ptr(), w.data_ptr(), dsrc.data_ptr(), dtgt.data_ptr(), q.shape[0],
                                       _prec(q.dtype), _stream(stream)))
        return dsrc, dtgt

    def sync_status(self, stream=None):
        _check(lib().lmfmm_sync_status(self._h, _stream(stream)))

    def stats(self):
        s = Stats()
        _check(lib().lmfmm_get_stats(self._h, ctypes.byref(s)))
        d = {f: getattr(s, f) for f, _ in Stats._fields_}
        d["order"] = list(s.order)[: s.levels + 1]
        for f in ("kernel_flops", "kernel_ms", "kernel_launches"):
            d[f] = dict(zip(KERNELS, list(getattr(s, f))))
        return d


class Batch:
    """Many independent problems applied in one graph launch (lmfmm_batch_*).

    media: list of (k, d); order_set: candidate order floors for the autotuner."""

    def __init__(self, media, order_set=(12, 16, 20), tol=1e-6, tune=True, graph=True, tune_cache=None):
        L = lib()
        n = len(media)
        karr = (ctypes.c_double * (6 * n))()
        darr = (ctypes.c_double * n)()
        for i, (k, d) in enumerate(media):
            kk = [complex(v) for v in k]
            for j in range(3):
                karr[6 * i + 2 * j] = kk[j].real
                karr[6 * i + 2 * j + 1] = kk[j].imag
            darr[i] = float(d)
        oarr = (ctypes.c_int * len(order_set))(*order_set)
        h = ctypes.c_void_p()
        _check(L.lmfmm_batch_create(n, karr, darr, oarr, len(order_set), float(tol), ctypes.byref(h)))
        self._h = h
        self.n = n
        self._keep = None
        if not tune:
            self.set_option("tune", "0")
        if not graph:
            self.set_option("graph", "0")
        if tune_cache is not None:
            self.set_option("tune_cache", tune_cache)

    def set_option(self, key, value):
        _check(lib().lmfmm_batch_set_option(self._h, key.encode(), str(value).encode()))

    def apply(self, items, outs=None, stream=None):
        """items: list of (src, q, tgt); returns the list of outputs u (reuses outs if given,
        which keeps the descriptors fixed so that later calls replay the prepared launches).
        Every instance must have the same number of right-hand sides and the same dtype."""
        import torch
        if len(items) != self.n:
            raise ValueError("one (src, q, tgt) per instance")
        if outs is not None and len(outs) != self.n:
            raise ValueError("one output per instance")
        checked = []
        nrhs = dtype = None
        for i, (src, q, tgt) in enumerate(items):
            src, tgt = _xy(src, f"src[{i}]"), _xy(tgt, f"tgt[{i}]")
            q = _dens(q, src.shape[1], f"q[{i}]")
            if nrhs is None:
                nrhs, dtype = q.shape[0], q.dtype
            elif q.shape[0] != nrhs or q.dtype != dtype:
                raise ValueError(f"instance {i}: densities of shape {tuple(q.shape)} and dtype {q.dtype}; every "
                                 f"instance must have {nrhs} right-hand sides of dtype {dtype}")
            checked.append((src, q, tgt))
        if outs is None:
            outs = [torch.empty((nrhs, tgt.shape[1]), dtype=dtype, device=q.device) for (_, q, tgt) in checked]
        else:
            outs = [_out(u, nrhs, tgt.shape[1], dtype, q.device, f"outs[{i}]")
                    for i, (u, (_, q, tgt)) in enumerate(zip(outs, checked))]
        arr = (Instance * self.n)()
        keep = []
        for i, ((src, q, tgt), u) in enumerate(zip(checked, outs)):
            keep += [src, q, tgt, u]
            arr[i] = Instance(src.shape[1], src.data_ptr(), q.data_ptr(), tgt.shape[1], tgt.data_ptr(), u.data_ptr())
        _check(lib().lmfmm_batch_apply(self._h, arr, nrhs, _prec(dtype), _stream(stream)))
        self._keep = keep
        return outs

    def sync_status(self, stream=None):
        """Synchronise and raise if any instance's points left the bounding box the
        batch was prepared for (or their layer); the next apply then prepares again."""
        _check(lib().lmfmm_batch_sync_status(self._h, _stream(stream)))

    def stats(self):
        s = BatchStats()
        _check(lib().lmfmm_batch_get_stats(self._h, ctypes.byref(s)))
        d = {f: getattr(s, f) for f, _ in BatchStats._fields_}
        for f in ("kernel_flops", "kernel_ms", "kernel_launches"):
            d[f] = dict(zip(KERNELS, list(getattr(s, f))))
        return d

    def choices(self):
        out = []
        for i in range(self.n):
            o, L_, us, sw = ctypes.c_int(), ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
            _check(lib().lmfmm_batch_get_choice(self._h, i, ctypes.byref(o), ctypes.byref(L_), ctypes.byref(us),
                                                ctypes.byref(sw)))
            out.append(dict(order=o.value, levels=L_.value, us=us.value, near_sweep=sw.value))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().lmfmm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
