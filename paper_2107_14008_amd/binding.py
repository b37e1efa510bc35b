"""ctypes binding of libpmfmm.so (argument marshalling only).

Every call maps one-to-one onto an ``extern "C"`` entry point declared in
include/pmfmm.h.  Device arrays are passed as raw pointers of torch CUDA
tensors and streams as torch's raw stream handles; no computation happens
here.  If the library has not been built the import fails loudly: there is
no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmfmm.so")

PMFMM_FP64, PMFMM_FP32 = 0, 1
TRUNC_EXACT, TRUNC_TABLE, TRUNC_R2 = 0, 1, 2
ROUND_NEAREST, ROUND_FLOOR = 0, 1
M2L_INSIDE, M2L_CENTRE = 0, 1
ACCUM_FP64, ACCUM_FP32_TWOSUM = 0, 1

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE",
          -5: "EUNSUPPORTED"}


class PmfmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("box", C.c_double), ("r_s", C.c_double), ("r_cut", C.c_double),
        ("G", C.c_double), ("theta", C.c_double),
        ("max_leaf", C.c_int32), ("order", C.c_int32),
        ("m2l_cut", C.c_int32), ("precision", C.c_int32), ("trunc", C.c_int32),
        ("table_size", C.c_int32), ("table_level", C.c_int32),
        ("table_round", C.c_int32), ("chunk", C.c_int32),
        ("wg_waves", C.c_int32), ("grid_wgs", C.c_int32),
        ("timing", C.c_int32), ("threads", C.c_int32),
        ("planner", C.c_int32), ("accum", C.c_int32),
    ]


class Lists(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("n_boxes", C.c_int64), ("n_leaves", C.c_int64),
        ("n_cells", C.c_int64), ("n_p2p", C.c_int64), ("n_m2l", C.c_int64),
        ("n_items", C.c_int64), ("candidate_pairs", C.c_int64),
        ("perm", C.POINTER(C.c_int32)),
        ("box_first_leaf", C.POINTER(C.c_int32)),
        ("box_first_cell", C.POINTER(C.c_int32)),
        ("leaf_first", C.POINTER(C.c_int32)),
        ("leaf_count", C.POINTER(C.c_int32)),
        ("leaf_cell", C.POINTER(C.c_int32)),
        ("cell_first", C.POINTER(C.c_int32)),
        ("cell_count", C.POINTER(C.c_int32)),
        ("cell_child", C.POINTER(C.c_int32)),
        ("cell_lo", C.POINTER(C.c_double)),
        ("cell_hi", C.POINTER(C.c_double)),
        ("p2p_row", C.POINTER(C.c_int32)),
        ("p2p_j", C.POINTER(C.c_int32)),
        ("p2p_shift", C.POINTER(C.c_int32)),
        ("m2l_row", C.POINTER(C.c_int32)),
        ("m2l_src", C.POINTER(C.c_int32)),
        ("m2l_shift", C.POINTER(C.c_int32)),
    ]


class Timings(C.Structure):
    _fields_ = [("far_ms", C.c_double), ("p2p_ms", C.c_double),
                ("reduce_ms", C.c_double), ("total_ms", C.c_double),
                ("adjoint_ms", C.c_double)]


class Schedule(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("wg_waves", C.c_int32),
                ("grid_wgs", C.c_int32), ("pad", C.c_int32), ("p2p_ms", C.c_double)]


# name -> (restype, argtypes); the exports of include/pmfmm.h
SIGNATURES = {
    "pmfmm_params_init": (None, [C.POINTER(Params)]),
    "pmfmm_create": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_void_p)]),
    "pmfmm_destroy": (None, [C.c_void_p]),
    "pmfmm_last_error": (C.c_char_p, []),
    "pmfmm_plan": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "pmfmm_plan_batch": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Params),
                                   C.POINTER(C.c_int64), C.c_void_p,
                                   C.c_void_p]),
    "pmfmm_build": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                              C.c_int32, C.c_void_p]),
    "pmfmm_build_batch": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Params),
                                    C.POINTER(C.c_int64), C.c_void_p,
                                    C.c_void_p, C.c_int32, C.c_void_p]),
    "pmfmm_set_eval": (C.c_int, [C.c_void_p, C.POINTER(Params)]),
    "pmfmm_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pmfmm_forward_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pmfmm_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p]),
    "pmfmm_long_range": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p]),
    "pmfmm_kick": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "pmfmm_drift": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                              C.c_void_p]),
    "pmfmm_get_lists": (C.c_int, [C.c_void_p, C.POINTER(Lists)]),
    "pmfmm_get_timings": (C.c_int, [C.c_void_p, C.POINTER(Timings)]),
    "pmfmm_version": (C.c_char_p, []),
    "pmfmm_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Schedule), C.c_int32,
                                 C.c_int32, C.c_char_p, C.POINTER(Schedule),
                                 C.POINTER(Schedule), C.c_void_p]),
    # include/pmfmm_peak.h
    "pmfmm_peak_fma": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double)]),
    "pmfmm_peak_last_error": (C.c_char_p, []),
}

_lib = None


def library():
    """Load libpmfmm.so once; raise if it has not been built.

    torch is imported first when it is installed: torch carries its own HIP
    runtime, and the library must bind to that same runtime (its dependency
    is resolved by soname to the copy already in the process).  Two HIP
    runtimes in one process do not share devices or memory.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2107_14008_amd.build` (there is no fallback)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc):
    if rc != 0:
        raise PmfmmError(rc, library().pmfmm_last_error().decode())


def make_params(**kw) -> Params:
    p = Params()
    library().pmfmm_params_init(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _ptr(x):
    """Raw pointer of a torch tensor or numpy array (no copy)."""
    if isinstance(x, np.ndarray):
        return C.c_void_p(x.ctypes.data)
    return C.c_void_p(x.data_ptr())


def _stream(stream):
    if stream is None:
        return C.c_void_p(0)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev(x, name, shape, device=None):
    """Check that x is a contiguous float64 torch CUDA tensor of `shape`
    (None entries are free) on `device`; raise ValueError before any kernel
    can read or write past it."""
    if isinstance(x, np.ndarray) or not hasattr(x, "data_ptr"):
        raise ValueError(f"{name} must be a float64 torch CUDA tensor, got {type(x).__name__}")
    if getattr(x.device, "type", None) != "cuda":
        raise ValueError(f"{name} must be on a CUDA device, got {x.device}")
    if device is not None and x.device != device:
        raise ValueError(f"{name} is on {x.device}, expected {device}")
    if str(x.dtype) != "torch.float64":
        raise ValueError(f"{name} must be float64, got {x.dtype}")
    if x.dim() != len(shape) or any(s is not None and x.shape[k] != s for k, s in enumerate(shape)):
        raise ValueError(f"{name} must have shape {tuple('n' if s is None else s for s in shape)}"
                         f", got {tuple(x.shape)}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x


def _host(a, name, shape):
    """float64 C-contiguous copy (or view) of a host array of `shape`."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != len(shape) or any(s is not None and a.shape[k] != s for k, s in enumerate(shape)):
        raise ValueError(f"{name} must have shape {tuple('n' if s is None else s for s in shape)}"
                         f", got {a.shape}")
    return a


def _particles(pos, mass):
    """Validated (pos (n, 3), mass (n), on_device) of one build call."""
    if isinstance(pos, np.ndarray) != isinstance(mass, np.ndarray):
        raise ValueError("pos and mass must both be numpy arrays or both torch CUDA tensors")
    if isinstance(pos, np.ndarray):
        pos = _host(pos, "pos", (None, 3))
        mass = _host(mass, "mass", (pos.shape[0],))
        return pos, mass, False
    _dev(pos, "pos", (None, 3))
    _dev(mass, "mass", (pos.shape[0],), pos.device)
    return pos, mass, True


def kick(vel, acc, dt, stream=None):
    """vel += acc dt (device (n, 3) float64)."""
    _dev(vel, "vel", (None, 3))
    _dev(acc, "acc", (vel.shape[0], 3), vel.device)
    _check(library().pmfmm_kick(int(vel.shape[0]), _ptr(vel), _ptr(acc), float(dt), _stream(stream)))


def drift(pos, vel, dt, box, stream=None):
    """pos += vel dt, wrapped into [0, box) (device (n, 3) float64)."""
    _dev(pos, "pos", (None, 3))
    _dev(vel, "vel", (pos.shape[0], 3), pos.device)
    _check(library().pmfmm_drift(int(pos.shape[0]), _ptr(pos), _ptr(vel), float(dt), float(box),
                                 _stream(stream)))


def peak_fma(precision: int, iters: int = 20000):
    """Measured vector FMA rate (TFLOP/s, kernel ms) of the current device:
    precision PMFMM_FP64 or PMFMM_FP32 (unpacked)."""
    tf, ms = C.c_double(), C.c_double()
    rc = library().pmfmm_peak_fma(int(precision), int(iters), C.byref(tf), C.byref(ms))
    if rc != 0:
        raise PmfmmError(rc, library().pmfmm_peak_last_error().decode())
    return tf.value, ms.value


class Context:
    """One library context (pmfmm_ctx)."""

    def __init__(self, **params):
        self.params = make_params(**params)
        h = C.c_void_p()
        _check(library().pmfmm_create(C.byref(self.params), C.byref(h)))
        self._h = h
        self.n = 0

    def close(self):
        if getattr(self, "_h", None):
            library().pmfmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- planning / build
    def plan(self, pos, mass):
        pos = _host(pos, "pos", (None, 3))
        mass = _host(mass, "mass", (pos.shape[0],))
        _check(library().pmfmm_plan(self._h, len(mass), _ptr(pos), _ptr(mass)))
        self.n = len(mass)

    def plan_batch(self, per_box, counts, pos, mass):
        arr = (Params * len(per_box))(*per_box)
        cnt = (C.c_int64 * len(counts))(*counts)
        if len(counts) != len(per_box):
            raise ValueError("one count per box is needed")
        pos = _host(pos, "pos", (int(sum(counts)), 3))
        mass = _host(mass, "mass", (int(sum(counts)),))
        _check(library().pmfmm_plan_batch(self._h, len(per_box), arr, cnt,
                                          _ptr(pos), _ptr(mass)))
        self.n = int(sum(counts))

    def build(self, pos, mass, stream=None):
        """pos (n, 3), mass (n): float64 torch CUDA tensors (contiguous) or
        numpy arrays (copied to float64 if needed)."""
        pos, mass, on_dev = _particles(pos, mass)
        _check(library().pmfmm_build(self._h, int(mass.shape[0]), _ptr(pos),
                                     _ptr(mass), int(on_dev), _stream(stream)))
        self.n = int(mass.shape[0])

    def build_batch(self, per_box, counts, pos, mass, stream=None):
        arr = (Params * len(per_box))(*per_box)
        cnt = (C.c_int64 * len(counts))(*counts)
        if len(counts) != len(per_box):
            raise ValueError("one count per box is needed")
        pos, mass, on_dev = _particles(pos, mass)
        if pos.shape[0] != int(sum(counts)):
            raise ValueError(f"pos holds {pos.shape[0]} particles, the counts {int(sum(counts))}")
        _check(library().pmfmm_build_batch(self._h, len(per_box), arr, cnt,
                                           _ptr(pos), _ptr(mass), int(on_dev),
                                           _stream(stream)))
        self.n = int(sum(counts))

    def set_eval(self, **kw):
        """Apply the changes to a copy; keep them only once the library has
        accepted them (a rejected call leaves params as they were)."""
        p = Params()
        C.pointer(p)[0] = self.params
        for k, v in kw.items():
            if not hasattr(p, k):
                raise KeyError(k)
            setattr(p, k, v)
        _check(library().pmfmm_set_eval(self._h, C.byref(p)))
        self.params = p

    def _built(self):
        if self.n <= 0:
            raise PmfmmError(-4, "forward / adjoint before build")

    # ---- compute
    def forward(self, out, stream=None):
        """out: float64 CUDA tensor (n, 3), written in caller order."""
        self._built()
        _dev(out, "out", (self.n, 3))
        _check(library().pmfmm_forward(self._h, _ptr(out), _stream(stream)))
        return out

    def forward_static(self, out, stream=None):
        """As forward, through pmfmm_forward_static (no device allocation:
        the library's static scratch array instead of the context's
        buffers)."""
        self._built()
        _dev(out, "out", (self.n, 3))
        _check(library().pmfmm_forward_static(self._h, _ptr(out), _stream(stream)))
        return out

    def adjoint(self, w, grad_pos, grad_mass, stream=None):
        """w, grad_pos: float64 CUDA (n, 3); grad_mass: float64 CUDA (n)."""
        self._built()
        _dev(w, "w", (self.n, 3))
        _dev(grad_pos, "grad_pos", (self.n, 3), w.device)
        _dev(grad_mass, "grad_mass", (self.n,), w.device)
        _check(library().pmfmm_adjoint(self._h, _ptr(w), _ptr(grad_pos),
                                       _ptr(grad_mass), _stream(stream)))
        return grad_pos, grad_mass

    def autotune(self, out, stream=None, cands=None, repeats=3, cache_path=None):
        """pmfmm_autotune: time candidate schedules (chunk, wg_waves,
        grid_wgs) of the P2P launch on the built context and apply the
        fastest.  out: float64 CUDA (n, 3), written.  Returns (best
        schedule dict, [per-candidate dicts]) (the list is empty on a cache
        hit)."""
        self._built()
        _dev(out, "out", (self.n, 3))
        n = len(cands) if cands else 24
        carr = (Schedule * n)(*[Schedule(int(c), int(w), int(g), 0, -1.0) for c, w, g in cands]) \
            if cands else None
        res = (Schedule * n)(*[Schedule(0, 0, 0, 0, -2.0) for _ in range(n)])
        best = Schedule()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(library().pmfmm_autotune(self._h, _ptr(out), carr, n if cands else 0,
                                        int(repeats), path, res, C.byref(best),
                                        _stream(stream)))
        # the library applied the schedule: keep the Python copy in step
        self.params.chunk, self.params.wg_waves, self.params.grid_wgs = (
            best.chunk, best.wg_waves, best.grid_wgs)

        def d(sc):
            return dict(chunk=sc.chunk, wg_waves=sc.wg_waves, grid_wgs=sc.grid_wgs,
                        p2p_ms=sc.p2p_ms)
        timed = [d(r) for r in res if r.p2p_ms != -2.0]
        return d(best), timed

    def long_range(self, n_pm, pos, mass, out, stream=None):
        """Long-range (mesh) accelerations into out (n, 3), caller order."""
        _dev(pos, "pos", (None, 3))
        _dev(mass, "mass", (pos.shape[0],), pos.device)
        _dev(out, "out", (pos.shape[0], 3), pos.device)
        _check(library().pmfmm_long_range(self._h, int(n_pm), int(pos.shape[0]), _ptr(pos),
                                          _ptr(mass), _ptr(out), _stream(stream)))
        return out

    # ---- introspection
    def lists(self) -> dict:
        L = Lists()
        _check(library().pmfmm_get_lists(self._h, C.byref(L)))

        def arr(ptr, n, dt=np.int32):
            if n == 0:
                return np.zeros(0, dt)
            return np.ctypeslib.as_array(ptr, shape=(n,)).copy()
        nl, nc = L.n_leaves, L.n_cells
        return dict(
            n=L.n, n_boxes=L.n_boxes, n_leaves=nl, n_cells=nc, n_p2p=L.n_p2p,
            n_m2l=L.n_m2l, n_items=L.n_items,
            candidate_pairs=L.candidate_pairs,
            perm=arr(L.perm, L.n),
            box_first_leaf=arr(L.box_first_leaf, L.n_boxes + 1),
            box_first_cell=arr(L.box_first_cell, L.n_boxes + 1),
            leaf_first=arr(L.leaf_first, nl), leaf_count=arr(L.leaf_count, nl),
            leaf_cell=arr(L.leaf_cell, nl),
            cell_first=arr(L.cell_first, nc), cell_count=arr(L.cell_count, nc),
            cell_child=arr(L.cell_child, 2 * nc).reshape(nc, 2),
            cell_lo=arr(L.cell_lo, 3 * nc, np.float64).reshape(nc, 3),
            cell_hi=arr(L.cell_hi, 3 * nc, np.float64).reshape(nc, 3),
            p2p_row=arr(L.p2p_row, nl + 1), p2p_j=arr(L.p2p_j, L.n_p2p),
            p2p_shift=arr(L.p2p_shift, L.n_p2p),
            m2l_row=arr(L.m2l_row, nc + 1), m2l_src=arr(L.m2l_src, L.n_m2l),
            m2l_shift=arr(L.m2l_shift, L.n_m2l),
        )

    def timings(self) -> dict:
        t = Timings()
        _check(library().pmfmm_get_timings(self._h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in Timings._fields_}
