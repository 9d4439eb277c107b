"""Python binding of libfr3d (include/fr3d.h): argument marshalling only.

Every computation runs in the HIP library; torch provides device memory and
the stream.  Importing this module loads the in-tree libfr3d.so and fails
loudly if it has not been built.

    from paper_1703_01216_amd import fr3d
    ctx = fr3d.Context()                       # current torch device and stream
    ctx.load_kernel(nx=128, ny=128, nz=128, precision=32)
    ctx.set_data(F, delta)                     # F: (nz, ny, nx) float32 cuda tensor
    rep = ctx.solve_discrepancy(zeta)          # zeta: output tensor of the same shape
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfr3d.so")

OK, E_INVALID, E_STATE, E_NOMEM, E_DEVICE = 0, 1, 2, 3, 4
CG_LIMIT = 32
UNFINISHED = 64
NOROOT_HIGH, NOROOT_LOW, MAXITER, NAN_INPUT, PRED_FALLBACK = 1, 2, 4, 8, 16

EXPORTED = [
    "fr3d_dp_opts_default", "fr3d_create", "fr3d_destroy", "fr3d_set_stream", "fr3d_load_kernel",
    "fr3d_set_data", "fr3d_solve_alpha", "fr3d_solve_discrepancy", "fr3d_recover_c",
    "fr3d_source_potential", "fr3d_apply_operator", "fr3d_add_noise", "fr3d_get_octant",
    "fr3d_get_data_spectrum", "fr3d_get_features", "fr3d_get_smax", "fr3d_set_timing",
    "fr3d_get_timing", "fr3d_status_string", "fr3d_last_error", "fr3d_set_lanes", "fr3d_solve_batch", "fr3d_solve_group", "fr3d_set_graphs", "fr3d_set_filter", "fr3d_load_layered", "fr3d_solve_exact", "fr3d_solve_exact_discrepancy",
    "fr3d_solve_per_frequency", "fr3d_load_kernel_samples", "fr3d_set_diagnostics", "fr3d_get_singular_values",
    "fr3d_predictor_set_calibration", "fr3d_solve_alpha_dev", "fr3d_solve_discrepancy_dev",
    "fr3d_predictor_set", "fr3d_predictor_get", "fr3d_predictor_forward", "fr3d_predictor_train_step",
    "fr3d_predictor_save", "fr3d_predictor_load", "fr3d_set_tile", "fr3d_recover_c_noalloc",
]
PASS_NAMES = ["fwd_x", "fwd_y", "fwd_z", "inv_z", "inv_y", "inv_x"]
TUNING_PATH = os.path.join(HERE, "data", "tuning.json")
N_PARAMS = 25089
N_NORM = 132


class Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double), ("D", ctypes.c_double), ("kind", ctypes.c_int32),
                ("q", ctypes.c_int32), ("precision", ctypes.c_int32), ("alpha_relative", ctypes.c_int32),
                ("hz", ctypes.c_double)]


class DpOpts(ctypes.Structure):
    _fields_ = [("log10_alpha_lo", ctypes.c_double), ("log10_alpha_hi", ctypes.c_double),
                ("max_steps", ctypes.c_int32), ("tol", ctypes.c_double),
                ("accept_lo", ctypes.c_double), ("accept_hi", ctypes.c_double),
                ("tau", ctypes.c_double), ("h_op", ctypes.c_double), ("mu", ctypes.c_double),
                ("use_predictor", ctypes.c_int32), ("seed_walk", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("seed_slope", ctypes.c_double),
                ("seed_slope_x", ctypes.c_double), ("seed_snap_lo", ctypes.c_double),
                ("seed_slope_ratio", ctypes.c_double)]


class Report(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("residual", ctypes.c_double),
                ("zeta_norm", ctypes.c_double), ("delta", ctypes.c_double),
                ("target", ctypes.c_double), ("n_evals", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("n_clamped", ctypes.c_int64), ("residual_full_box", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}

    @classmethod
    def from_device(cls, rep_dev):
        """Decode a report written to device memory by a _dev solve (a uint8
        tensor of ctypes.sizeof(Report) bytes; copied to the host here)."""
        raw = bytes(rep_dev.cpu().numpy().tobytes())
        return cls.from_buffer_copy(raw[:ctypes.sizeof(cls)]).as_dict()


class Fr3dError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fr3d status {status}: {msg}")
        self.status = status


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1703_01216_amd.build.build()")
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "fr3d_dp_opts_default": (None, [ctypes.POINTER(DpOpts)]),
        "fr3d_create": (I32, [ctypes.POINTER(P), I32, P]),
        "fr3d_destroy": (I32, [P]),
        "fr3d_set_stream": (I32, [P, P]),
        "fr3d_load_kernel": (I32, [P, ctypes.POINTER(Geom)]),
        "fr3d_set_data": (I32, [P, P, D]),
        "fr3d_solve_alpha": (I32, [P, D, P, ctypes.POINTER(Report)]),
        "fr3d_solve_discrepancy": (I32, [P, ctypes.POINTER(DpOpts), P, ctypes.POINTER(Report)]),
        "fr3d_solve_alpha_dev": (I32, [P, D, P, P]),
        "fr3d_solve_discrepancy_dev": (I32, [P, ctypes.POINTER(DpOpts), P, P]),
        "fr3d_recover_c": (I32, [P, P, P, D, P, ctypes.POINTER(I64)]),
        "fr3d_recover_c_noalloc": (I32, [I32, I64, P, P, D, P, P, P]),
        "fr3d_source_potential": (I32, [P, D, P]),
        "fr3d_apply_operator": (I32, [P, P, P]),
        "fr3d_add_noise": (I32, [P, P, P, D, ctypes.POINTER(D)]),
        "fr3d_get_octant": (I32, [P, P, I64]),
        "fr3d_get_data_spectrum": (I32, [P, P, I64]),
        "fr3d_get_features": (I32, [P, P, P]),
        "fr3d_get_smax": (I32, [P, ctypes.POINTER(D)]),
        "fr3d_set_timing": (I32, [P, I32]),
        "fr3d_get_timing": (I32, [P, I32, ctypes.POINTER(D), ctypes.POINTER(I64)]),
        "fr3d_status_string": (ctypes.c_char_p, [I32]),
        "fr3d_last_error": (ctypes.c_char_p, [P]),
        "fr3d_set_lanes": (I32, [P, I32]),
        "fr3d_set_graphs": (I32, [P, I32]),
        "fr3d_set_filter": (I32, [P, I32, I32]),
        "fr3d_load_layered": (I32, [P, ctypes.POINTER(Geom)]),
        "fr3d_solve_exact": (I32, [P, P, D, P, I32, D, ctypes.POINTER(Report)]),
        "fr3d_solve_per_frequency": (I32, [P, ctypes.POINTER(DpOpts), P, P, P, ctypes.POINTER(Report)]),
        "fr3d_load_kernel_samples": (I32, [P, ctypes.POINTER(Geom), P]),
        "fr3d_set_diagnostics": (I32, [P, I32]),
        "fr3d_get_singular_values": (I32, [P, P, I64]),
        "fr3d_predictor_set_calibration": (I32, [P, ctypes.POINTER(ctypes.c_double), I64]),
        "fr3d_solve_exact_discrepancy": (I32, [P, P, D, ctypes.POINTER(DpOpts), P, I32, D, ctypes.POINTER(Report)]),
        "fr3d_solve_batch": (I32, [P, I32, ctypes.POINTER(P), ctypes.POINTER(D), ctypes.POINTER(P),
                                   ctypes.POINTER(DpOpts), P, D, ctypes.POINTER(P), P, ctypes.POINTER(Report)]),
        "fr3d_solve_group": (I32, [I32, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(D), ctypes.POINTER(P),
                                   ctypes.POINTER(DpOpts), ctypes.POINTER(P), D, ctypes.POINTER(P),
                                   ctypes.POINTER(Report)]),
        "fr3d_predictor_set": (I32, [P, ctypes.POINTER(ctypes.c_float), I64, ctypes.POINTER(ctypes.c_float)]),
        "fr3d_predictor_get": (I32, [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
        "fr3d_predictor_forward": (I32, [P, P, I32, P]),
        "fr3d_predictor_train_step": (I32, [P, P, P, I32, D, P, P]),
        "fr3d_predictor_save": (I32, [P, ctypes.c_char_p]),
        "fr3d_predictor_load": (I32, [P, ctypes.c_char_p]),
        "fr3d_set_tile": (I32, [P, I32, I32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def default_opts(**kw) -> DpOpts:
    o = DpOpts()
    lib().fr3d_dp_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """One solver context on a device, enqueuing on a torch stream."""

    def __init__(self, device: int | None = None, stream=None):
        import torch
        self.torch = torch
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        self._lib = lib()
        self._ctx = ctypes.c_void_p()
        st = stream if stream is not None else torch.cuda.current_stream(device)
        self._stream = st
        s = self._lib.fr3d_create(ctypes.byref(self._ctx), int(device), ctypes.c_void_p(st.cuda_stream))
        if s != OK:
            raise Fr3dError(s, self._lib.fr3d_status_string(s).decode())
        self.geom = None

    # ------------------------------------------------------------ plumbing
    def _chk(self, s):
        if s != OK:
            raise Fr3dError(s, self._lib.fr3d_last_error(self._ctx).decode())

    def close(self):
        if self._ctx:
            self._lib.fr3d_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dtype(self):
        return self.torch.float64 if self.geom.precision == 64 else self.torch.float32

    @property
    def shape(self):
        return (self.geom.nz, self.geom.ny, self.geom.nx)

    def _arr(self, t, name):
        if t is None:
            raise ValueError(f"{name} is None")
        if self.geom is None:
            raise ValueError("no kernel loaded on this context")
        if not t.is_cuda or t.dtype != self.dtype or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} cuda tensor of shape {self.shape}")
        return ctypes.c_void_p(t.data_ptr())

    def set_stream(self, stream):
        self._stream = stream
        self._chk(self._lib.fr3d_set_stream(self._ctx, ctypes.c_void_p(stream.cuda_stream)))

    # ------------------------------------------------------------ calls of include/fr3d.h
    def load_kernel(self, nx, ny, nz, h=1.0, D=0.0, kind=0, q=-1, precision=32, alpha_relative=0, hz=0.0):
        g = Geom(nx, ny, nz, h, D, kind, q, precision, alpha_relative, hz)
        self._chk(self._lib.fr3d_load_kernel(self._ctx, ctypes.byref(g)))
        self.geom = g

    def load_kernel_samples(self, k, nx, ny, nz, h=1.0, D=0.0, q=-1, precision=32, alpha_relative=0, hz=0.0):
        """The caller's wrapped kernel table k (float64 cuda tensor [2nz][2ny][2nx])."""
        if not (k.is_cuda and k.dtype == self.torch.float64 and k.is_contiguous()
                and tuple(k.shape) == (2 * nz, 2 * ny, 2 * nx)):
            raise ValueError("k must be a contiguous float64 cuda tensor of shape (2nz, 2ny, 2nx)")
        g = Geom(nx, ny, nz, h, D, 0, q, precision, alpha_relative, hz)
        self._chk(self._lib.fr3d_load_kernel_samples(self._ctx, ctypes.byref(g), _ptr(k)))
        self.geom = g

    def load_layered(self, nx, ny, nz, h=1.0, D=0.0, kind=0, q=-1, precision=32, alpha_relative=0, hz=0.0):
        """Per-frequency z-systems (Algorithm 1 as run in Sec. 5) instead of the 3D embedding."""
        g = Geom(nx, ny, nz, h, D, kind, q, precision, alpha_relative, hz)
        self._chk(self._lib.fr3d_load_layered(self._ctx, ctypes.byref(g)))
        self.geom = g

    def set_data(self, F, delta):
        self._chk(self._lib.fr3d_set_data(self._ctx, self._arr(F, "F"), float(delta)))

    def solve_alpha(self, alpha, zeta):
        rep = Report()
        self._chk(self._lib.fr3d_solve_alpha(self._ctx, float(alpha), self._arr(zeta, "zeta"), ctypes.byref(rep)))
        return rep.as_dict()

    def solve_discrepancy(self, zeta, opts: DpOpts | None = None, **kw):
        o = opts if opts is not None else default_opts(**kw)
        rep = Report()
        self._chk(self._lib.fr3d_solve_discrepancy(self._ctx, ctypes.byref(o), self._arr(zeta, "zeta"),
                                                   ctypes.byref(rep)))
        return rep.as_dict()

    def _rep_dev(self, rep_dev):
        if rep_dev is None or not rep_dev.is_cuda or rep_dev.dtype != self.torch.uint8 or \
                rep_dev.numel() < ctypes.sizeof(Report) or not rep_dev.is_contiguous():
            raise ValueError(f"rep_dev must be a contiguous uint8 cuda tensor of >= {ctypes.sizeof(Report)} bytes")
        return ctypes.c_void_p(rep_dev.data_ptr())

    def solve_alpha_dev(self, alpha, zeta, rep_dev):
        """fr3d_solve_alpha_dev: enqueued without a host synchronisation; the
        report goes to rep_dev (decode with Report.from_device)."""
        self._chk(self._lib.fr3d_solve_alpha_dev(self._ctx, float(alpha), self._arr(zeta, "zeta"),
                                                 self._rep_dev(rep_dev)))

    def solve_discrepancy_dev(self, zeta, rep_dev, opts: DpOpts | None = None, **kw):
        """fr3d_solve_discrepancy_dev: the whole search enqueued without a host
        synchronisation; the report goes to rep_dev."""
        o = opts if opts is not None else default_opts(**kw)
        self._chk(self._lib.fr3d_solve_discrepancy_dev(self._ctx, ctypes.byref(o), self._arr(zeta, "zeta"),
                                                       self._rep_dev(rep_dev)))

    def solve_per_frequency(self, zeta, alphas=None, flags=None, opts: DpOpts | None = None, **kw):
        """One alpha per lateral frequency (fr3d_solve_per_frequency); alphas
        (float64) and flags (int32), if given, are cuda tensors of Kx x Py."""
        o = opts if opts is not None else default_opts(**kw)
        rep = Report()
        self._chk(self._lib.fr3d_solve_per_frequency(self._ctx, ctypes.byref(o), self._arr(zeta, "zeta"),
                                                     _ptr(alphas), _ptr(flags), ctypes.byref(rep)))
        return rep.as_dict()

    def solve_exact(self, F, alpha, zeta, max_iter=2000, tol=1e-6):
        """Tikhonov for the exact operator by CG (fr3d_solve_exact)."""
        rep = Report()
        self._chk(self._lib.fr3d_solve_exact(self._ctx, self._arr(F, "F"), float(alpha), self._arr(zeta, "zeta"),
                                             int(max_iter), float(tol), ctypes.byref(rep)))
        return rep.as_dict()

    def solve_exact_discrepancy(self, F, delta, zeta, max_iter=2000, tol=1e-6, opts: DpOpts | None = None, **kw):
        o = opts if opts is not None else default_opts(**kw)
        rep = Report()
        self._chk(self._lib.fr3d_solve_exact_discrepancy(self._ctx, self._arr(F, "F"), float(delta), ctypes.byref(o),
                                                         self._arr(zeta, "zeta"), int(max_iter), float(tol),
                                                         ctypes.byref(rep)))
        return rep.as_dict()

    def recover_c(self, zeta, V0, c0, c_out):
        n = ctypes.c_int64()
        self._chk(self._lib.fr3d_recover_c(self._ctx, self._arr(zeta, "zeta"), self._arr(V0, "V0"), float(c0),
                                           self._arr(c_out, "c"), ctypes.byref(n)))
        return int(n.value)

    def source_potential(self, V0, A0=1.0):
        self._chk(self._lib.fr3d_source_potential(self._ctx, float(A0), self._arr(V0, "V0")))

    def apply_operator(self, zeta, F_out):
        self._chk(self._lib.fr3d_apply_operator(self._ctx, self._arr(zeta, "zeta"), self._arr(F_out, "F")))

    def add_noise(self, F, e, delta_rel):
        d = ctypes.c_double()
        self._chk(self._lib.fr3d_add_noise(self._ctx, self._arr(F, "F"), self._arr(e, "e"), float(delta_rel),
                                           ctypes.byref(d)))
        return d.value

    def get_octant(self):
        g = self.geom
        out = self.torch.empty((g.nx + 1, g.nz + 1, g.ny + 1, 2), dtype=self.torch.float64, device="cuda")
        self._chk(self._lib.fr3d_get_octant(self._ctx, _ptr(out), out.numel() * 8))
        return out

    def get_data_spectrum(self):
        g = self.geom
        out = self.torch.empty((g.nx + 1, 2 * g.nz, 2 * g.ny, 2), dtype=self.dtype, device="cuda")
        self._chk(self._lib.fr3d_get_data_spectrum(self._ctx, _ptr(out), out.numel() * out.element_size()))
        return out

    def get_singular_values(self):
        """Per-frequency systems' singular values, descending: [Px/2+1][Py/2+1][nz] float64."""
        g = self.geom
        out = self.torch.empty((g.nx + 1, g.ny + 1, g.nz), dtype=self.torch.float64, device="cuda")
        self._chk(self._lib.fr3d_get_singular_values(self._ctx, _ptr(out), out.numel() * 8))
        return out

    def get_features(self):
        feat = self.torch.empty(65, dtype=self.torch.float32, device="cuda")
        en = self.torch.empty(64, dtype=self.torch.float64, device="cuda")
        self._chk(self._lib.fr3d_get_features(self._ctx, _ptr(feat), _ptr(en)))
        return feat, en

    def get_smax(self):
        d = ctypes.c_double()
        self._chk(self._lib.fr3d_get_smax(self._ctx, ctypes.byref(d)))
        return d.value

    def set_filter(self, kind: int, order: int = 1):
        """0 Tikhonov, 1 iterated Tikhonov of the given order, 2 truncated SVD."""
        self._chk(self._lib.fr3d_set_filter(self._ctx, int(kind), int(order)))

    def set_diagnostics(self, on: bool):
        """Full-box residual in every report (residual_full_box)."""
        self._chk(self._lib.fr3d_set_diagnostics(self._ctx, 1 if on else 0))

    def set_graphs(self, on: bool):
        self._chk(self._lib.fr3d_set_graphs(self._ctx, 1 if on else 0))

    def set_lanes(self, lanes: int):
        self._chk(self._lib.fr3d_set_lanes(self._ctx, int(lanes)))

    def solve_batch(self, F_list, deltas, zetas, opts: DpOpts | None = None, V0=None, c0=1.0, c_list=None,
                    feat=None, **kw):
        n = len(F_list)
        if len(deltas) != n or len(zetas) != n or (c_list is not None and len(c_list) != n):
            raise ValueError("batch lists must have equal lengths")
        o = opts if opts is not None else default_opts(**kw)
        PA = ctypes.c_void_p * max(n, 1)
        Fa = PA(*[self._arr(f, "F").value for f in F_list])
        Za = PA(*[self._arr(z, "zeta").value for z in zetas])
        Da = (ctypes.c_double * max(n, 1))(*[float(d) for d in deltas])
        reps = (Report * max(n, 1))()
        Ca = PA(*[self._arr(cc, "c").value for cc in c_list]) if c_list is not None else None
        v0 = self._arr(V0, "V0") if c_list is not None else None
        if feat is not None and (feat.dtype != self.torch.float32 or feat.numel() < 65 * n or not feat.is_cuda):
            raise ValueError("feat must be a float32 cuda tensor with room for n x 65 values")
        self._chk(self._lib.fr3d_solve_batch(self._ctx, n, Fa, Da, Za, ctypes.byref(o), v0, float(c0), Ca,
                                             _ptr(feat), reps))
        return [reps[i].as_dict() for i in range(n)]

    # ------------------------------------------------------------ predictor
    def predictor_set(self, params, norm):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        nm = np.ascontiguousarray(norm, dtype=np.float32).ravel()
        if p.size != N_PARAMS or nm.size != N_NORM:
            raise ValueError(f"need {N_PARAMS} parameters and {N_NORM} normalisation values")
        fp = ctypes.POINTER(ctypes.c_float)
        self._chk(self._lib.fr3d_predictor_set(self._ctx, p.ctypes.data_as(fp), p.size, nm.ctypes.data_as(fp)))

    def predictor_get(self):
        import numpy as np
        p = np.empty(N_PARAMS, dtype=np.float32)
        nm = np.empty(N_NORM, dtype=np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        self._chk(self._lib.fr3d_predictor_get(self._ctx, p.ctypes.data_as(fp), nm.ctypes.data_as(fp)))
        return p, nm

    def predictor_forward(self, X, y):
        self._chk(self._lib.fr3d_predictor_forward(self._ctx, _ptr(X), int(X.shape[0]), _ptr(y)))

    def predictor_train_step(self, X, t, lr, loss=None, grad=None):
        self._chk(self._lib.fr3d_predictor_train_step(self._ctx, _ptr(X), _ptr(t), int(X.shape[0]), float(lr),
                                                      _ptr(loss), _ptr(grad)))

    def predictor_set_calibration(self, coef=None):
        """Seed calibration (66 coefficients: intercept, then one per raw feature); None clears it."""
        import numpy as np
        if coef is None:
            self._chk(self._lib.fr3d_predictor_set_calibration(self._ctx, None, 0))
            return
        c = np.ascontiguousarray(coef, dtype=np.float64).ravel()
        self._chk(self._lib.fr3d_predictor_set_calibration(
            self._ctx, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), c.size))

    def predictor_save(self, path):
        self._chk(self._lib.fr3d_predictor_save(self._ctx, os.fsencode(path)))

    def predictor_load(self, path):
        self._chk(self._lib.fr3d_predictor_load(self._ctx, os.fsencode(path)))

    def set_tile(self, pass_id: int, shift: int):
        self._chk(self._lib.fr3d_set_tile(self._ctx, int(pass_id), int(shift)))

    def tuning_key(self):
        g = self.geom
        return f"{2 * g.nx}x{2 * g.ny}x{2 * g.nz}/fp{g.precision}"

    def apply_tuning(self, path: str = TUNING_PATH, batched: bool = False):
        """Tile variants from an autotuner cache (JSON {key: {pass name: shift}});
        returns the applied entry or None when the cache has nothing for this
        geometry.  batched: prefer the entry tuned for solves of several lanes
        at once (key + "/batch", autotune --batched) when there is one.
        Without an entry for this exact padded box, each pass takes its
        variant from the cube whose side is that pass's transform length (the
        pass kernels are compiled per length)."""
        import json
        if not os.path.exists(path):
            return None
        cache = json.load(open(path))
        entry = (cache.get(self.tuning_key() + "/batch") if batched else None) or cache.get(self.tuning_key())
        if not entry:
            g = self.geom
            axis = {"fwd_x": 2 * g.nx, "inv_x": 2 * g.nx, "fwd_y": 2 * g.ny, "inv_y": 2 * g.ny,
                    "fwd_z": 2 * g.nz, "inv_z": 2 * g.nz}
            entry = {}
            for name, P in axis.items():
                cube = (cache.get(f"{P}x{P}x{P}/fp{g.precision}/batch") if batched else None) or \
                    cache.get(f"{P}x{P}x{P}/fp{g.precision}")
                if cube and name in cube:
                    entry[name] = cube[name]
        for k, v in entry.items():
            self.set_tile(PASS_NAMES.index(k), int(v))
        return entry or None

    def set_timing(self, on: bool):
        self._chk(self._lib.fr3d_set_timing(self._ctx, 1 if on else 0))

    def get_timing(self, pass_id: int):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._chk(self._lib.fr3d_get_timing(self._ctx, int(pass_id), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def recover_c_noalloc(zeta, V0, c0, c_out, n_clamped=None, stream=None):
    """fr3d_recover_c_noalloc: the recovery of c with no context, no device
    allocation and no host synchronisation.  zeta, V0, c_out: contiguous cuda
    tensors of one dtype (float32 or float64) and size; n_clamped: a one-element
    int64 cuda tensor that receives the clamped-cell count, or None.  Enqueued
    on `stream` (default: torch's current stream)."""
    import torch
    ts = (zeta, V0, c_out)
    if any(t is None or not t.is_cuda or not t.is_contiguous() for t in ts) or \
            len({t.dtype for t in ts}) != 1 or len({t.numel() for t in ts}) != 1 or \
            zeta.dtype not in (torch.float32, torch.float64):
        raise ValueError("zeta, V0, c_out must be contiguous cuda tensors of one float dtype and size")
    if n_clamped is not None and (not n_clamped.is_cuda or n_clamped.dtype != torch.int64 or n_clamped.numel() < 1):
        raise ValueError("n_clamped must be an int64 cuda tensor")
    st = stream if stream is not None else torch.cuda.current_stream()
    prec = 64 if zeta.dtype == torch.float64 else 32
    s = lib().fr3d_recover_c_noalloc(prec, zeta.numel(), _ptr(zeta), _ptr(V0), float(c0), _ptr(c_out),
                                     _ptr(n_clamped), ctypes.c_void_p(st.cuda_stream))
    if s != OK:
        raise Fr3dError(s, lib().fr3d_status_string(s).decode())


def solve_group(ctxs, F_list, deltas, zetas, opts: DpOpts | None = None, V0_list=None, c0=1.0, c_list=None, **kw):
    """Discrepancy solves of items of different geometries: item i on ctxs[i]
    (fr3d_solve_group).  Returns one report dict per item."""
    n = len(F_list)
    if len(ctxs) != n or len(deltas) != n or len(zetas) != n:
        raise ValueError("group lists must have equal lengths")
    if c_list is not None and (V0_list is None or len(c_list) != n or len(V0_list) != n):
        raise ValueError("recovery needs V0_list and c_list of the group's length")
    if n == 0:
        return []
    o = opts if opts is not None else default_opts(**kw)
    PA = ctypes.c_void_p * n
    Ca_ = PA(*[c._ctx.value for c in ctxs])
    Fa = PA(*[c._arr(f, "F").value for c, f in zip(ctxs, F_list)])
    Za = PA(*[c._arr(z, "zeta").value for c, z in zip(ctxs, zetas)])
    Da = (ctypes.c_double * n)(*[float(d) for d in deltas])
    reps = (Report * n)()
    Va = PA(*[c._arr(v, "V0").value for c, v in zip(ctxs, V0_list)]) if c_list is not None else None
    Oa = PA(*[c._arr(x, "c").value for c, x in zip(ctxs, c_list)]) if c_list is not None else None
    L = lib()
    s = L.fr3d_solve_group(n, Ca_, Fa, Da, Za, ctypes.byref(o), Va, float(c0), Oa, reps)
    if s != OK:
        raise Fr3dError(s, L.fr3d_last_error(ctxs[0]._ctx).decode())
    return [reps[i].as_dict() for i in range(n)]
