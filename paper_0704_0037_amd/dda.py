"""Python binding of the DDA C-ABI (include/dda.h): argument marshalling only.

Every computation runs in the HIP library libdda_mi355x.so built next to this file.  Vectors are
torch tensors on the GPU in the library's component-major layout ([3][N], or [n_rhs][3][N]);
PyTorch supplies device memory and the stream, nothing else.  Importing this module on a
machine where the library is missing raises immediately: there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdda_mi355x.so")

OK, EINVAL, ENOMEM, EHIP, ENOTCONV, EBREAKDOWN, ESYMMETRY, ENOTSUP = 0, -1, -2, -3, -4, -5, -6, -7
POL_LDR, POL_CM, POL_RR, POL_CLDR = 0, 1, 2, 3
QMR, BICGSTAB, BICG, CGNR = 0, 1, 2, 3
FP64, FP32_REFINE, FP32_PRODUCT, FP32_RELAXED = 0, 1, 2, 3
BREAKDOWN_REPORT, BREAKDOWN_RECOVER = 0, 1


class Beam(ct.Structure):
    _fields_ = [("prop", ct.c_double * 3), ("pol_re", ct.c_double * 3), ("pol_im", ct.c_double * 3),
                ("w0", ct.c_double), ("center", ct.c_double * 3)]


class SetupOpts(ct.Structure):
    _fields_ = [("pad", ct.c_int32 * 3), ("lines_per_block", ct.c_int32), ("fp32", ct.c_int32)]


class SolveOpts(ct.Structure):
    _fields_ = [("solver", ct.c_int32), ("precision", ct.c_int32), ("maxit", ct.c_int32),
                ("check_every", ct.c_int32), ("inner_tol", ct.c_double), ("x0", ct.c_void_p),
                ("graph", ct.c_int32), ("x0_check", ct.c_int32), ("on_breakdown", ct.c_int32),
                ("resume", ct.c_int32), ("relax_at", ct.c_double), ("pack", ct.c_int32)]


class SolveInfo(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("iters", ct.c_int32), ("matvecs", ct.c_int32), ("outer", ct.c_int32),
                ("res_rec", ct.c_double), ("res_true", ct.c_double), ("t_solve_s", ct.c_double),
                ("res_hist", ct.POINTER(ct.c_double)), ("res_hist_cap", ct.c_int32),
                ("res_hist_len", ct.c_int32)]


class DDAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None

# every symbol include/dda.h declares, with its ctypes signature
_SIGS = {
    "dda_setup": (ct.c_int, [ct.POINTER(ct.c_void_p), ct.POINTER(ct.c_int32), ct.c_void_p,
                             ct.POINTER(ct.c_double), ct.c_double, ct.c_int32, ct.POINTER(SetupOpts), ct.c_void_p]),
    "dda_free": (ct.c_int, [ct.c_void_p]),
    "dda_num_dipoles": (ct.c_int64, [ct.c_void_p]),
    "dda_padded_grid": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int32)]),
    "dda_polarizability": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.POINTER(ct.c_double)]),
    "dda_asymmetry": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_void_p, ct.c_int32, ct.c_int32,
                                 ct.POINTER(ct.c_double)]),
    "dda_checkpoint_save": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_char_p]),
    "dda_checkpoint_load": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_char_p]),
    "dda_orientation_average": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_double, ct.c_void_p,
                                           ct.POINTER(ct.c_double)]),
    "dda_setup_materials": (ct.c_int, [ct.POINTER(ct.c_void_p), ct.POINTER(ct.c_int32), ct.c_void_p, ct.c_int32,
                                       ct.POINTER(ct.c_double), ct.c_double, ct.c_int32, ct.POINTER(SetupOpts),
                                       ct.c_void_p]),
    "dda_orientation_average_mueller": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_double,
                                                   ct.c_void_p, ct.POINTER(ct.c_double), ct.c_int32,
                                                   ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]),
    "dda_orientation_average_adaptive": (ct.c_int, [ct.c_void_p, ct.c_double, ct.c_int32, ct.c_int32, ct.c_int32,
                                                    ct.c_double, ct.c_void_p, ct.POINTER(ct.c_double),
                                                    ct.POINTER(ct.c_int32)]),
    "dda_rhs": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_void_p]),
    "dda_matvec": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_void_p, ct.c_void_p]),
    "dda_tune_padding": (ct.c_int, [ct.POINTER(ct.c_int32), ct.POINTER(ct.c_uint8), ct.POINTER(ct.c_double),
                                     ct.c_double, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32,
                                     ct.POINTER(ct.c_int32), ct.POINTER(ct.c_float)]),
    "dda_matvec_noalloc": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_void_p, ct.c_void_p]),
    "dda_matvec_f32": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_void_p, ct.c_void_p]),
    "dda_matvec_batch": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_int32, ct.c_void_p, ct.c_void_p]),
    "dda_solve": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_int32, ct.c_double, ct.POINTER(SolveOpts),
                             ct.c_void_p, ct.POINTER(SolveInfo)]),
    "dda_solve_many": (ct.c_int, [ct.POINTER(ct.c_void_p), ct.c_int32, ct.POINTER(Beam), ct.c_double,
                                  ct.POINTER(SolveOpts), ct.POINTER(ct.c_void_p), ct.POINTER(SolveInfo)]),
    "dda_cross_sections": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_void_p, ct.POINTER(ct.c_double)]),
    "dda_farfield": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_double),
                                ct.POINTER(ct.c_double)]),
    "dda_mueller": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_void_p, ct.c_void_p, ct.c_double,
                               ct.POINTER(ct.c_double), ct.c_int32, ct.POINTER(ct.c_double)]),
    "dda_matvec_timed": (ct.c_int, [ct.c_void_p, ct.POINTER(Beam), ct.c_int32, ct.c_int32, ct.c_void_p,
                                    ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_float), ct.POINTER(ct.c_float)]),
    "dda_tune": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_int32)]),
    "dda_get_tiles": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_int32)]),
    "dda_set_tiles": (ct.c_int, [ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_int32)]),
    "dda_net_num_params": (ct.c_int64, []),
    "dda_net_create": (ct.c_int, [ct.POINTER(ct.c_void_p), ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p]),
    "dda_net_free": (ct.c_int, [ct.c_void_p]),
    "dda_net_set_params": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "dda_net_get_params": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "dda_net_features": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.POINTER(Beam), ct.c_void_p]),
    "dda_net_target": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.POINTER(Beam), ct.c_void_p, ct.c_void_p]),
    "dda_net_forward": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p]),
    "dda_net_grad": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_double),
                                ct.c_void_p]),
    "dda_net_train_step": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_double,
                                      ct.POINTER(ct.c_double)]),
    "dda_guess": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.POINTER(Beam), ct.c_int32, ct.c_void_p, ct.c_void_p]),
    "dda_strerror": (ct.c_char_p, [ct.c_int]),
    "dda_last_error": (ct.c_char_p, []),
}


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"HIP library not built: {_LIB_PATH} (run __graft_entry__.build())")
        L = ct.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, what):
    if status != OK:
        L = lib()
        msg = L.dda_last_error().decode() or L.dda_strerror(status).decode()
        raise DDAError(status, f"{what}: {msg}")


def make_beam(prop=(0.0, 0.0, 1.0), pol=(1.0, 0.0, 0.0), w0=0.0, center=(0.0, 0.0, 0.0)):
    """dda_beam: a plane wave (w0 = 0) or a focused beam of waist radius w0 at center."""
    b = Beam()
    pol = [complex(p) for p in pol]
    for i in range(3):
        b.prop[i] = float(prop[i])
        b.pol_re[i] = pol[i].real
        b.pol_im[i] = pol[i].imag
        b.center[i] = float(center[i])
    b.w0 = float(w0)
    return b


def _beam(obj):
    if isinstance(obj, Beam):
        return obj
    if hasattr(obj, "prop") and hasattr(obj, "pol"):
        return make_beam(obj.prop, obj.pol, getattr(obj, "w0", 0.0), getattr(obj, "center", (0.0, 0.0, 0.0)))
    prop, pol = obj
    return make_beam(prop, pol)


def _beams(objs):
    arr = (Beam * len(objs))()
    for i, o in enumerate(objs):
        arr[i] = _beam(o)
    return arr


def _ptr(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ct.c_void_p(t.data_ptr())


class Context:
    """One particle on the current GPU (wraps dda_setup / dda_free)."""

    def __init__(self, mask, m, kd, polarizability=POL_LDR, pad=None, fp32=False, lines_per_block=0,
                 stream=None):
        L = lib()
        mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        if mask.ndim != 3:
            raise ValueError("mask must be a 3-D array [nz][ny][nx]")
        nz, ny, nx = mask.shape
        self.grid = (nx, ny, nz)
        grid = (ct.c_int32 * 3)(nx, ny, nz)
        ms = [complex(v) for v in m] if isinstance(m, (list, tuple, np.ndarray)) else [complex(m)]
        mm = (ct.c_double * (2 * len(ms)))(*[p for v in ms for p in (v.real, v.imag)])
        opts = SetupOpts()
        if pad is not None:
            for i in range(3):
                opts.pad[i] = int(pad[i])
        opts.lines_per_block = int(lines_per_block)
        opts.fp32 = 1 if fp32 else 0
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ct.c_void_p()
        if len(ms) == 1:
            _check(L.dda_setup(ct.byref(h), grid, mask.ctypes.data_as(ct.c_void_p), mm, float(kd),
                               int(polarizability), ct.byref(opts), ct.c_void_p(stream.cuda_stream)), "dda_setup")
        else:  # an inhomogeneous particle: mask values 1..len(m) name the materials
            _check(L.dda_setup_materials(ct.byref(h), grid, mask.ctypes.data_as(ct.c_void_p), len(ms), mm, float(kd),
                                         int(polarizability), ct.byref(opts), ct.c_void_p(stream.cuda_stream)),
                   "dda_setup_materials")
        self._h = h
        self.n = int(L.dda_num_dipoles(h))
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "_h", None):
            lib().dda_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------ queries
    def padded_grid(self):
        out = (ct.c_int32 * 3)()
        _check(lib().dda_padded_grid(self._h, out), "dda_padded_grid")
        return tuple(out)

    def polarizability(self, beam):
        out = (ct.c_double * 2)()
        _check(lib().dda_polarizability(self._h, ct.byref(_beam(beam)), out), "dda_polarizability")
        return complex(out[0], out[1])

    def vector(self, n_rhs=None, dtype=torch.complex128):
        shape = (3, self.n) if n_rhs is None else (n_rhs, 3, self.n)
        return torch.empty(shape, dtype=dtype, device=self.device)

    # ------------------------------------------------------------------ compute
    def rhs(self, beam):
        b = self.vector()
        _check(lib().dda_rhs(self._h, ct.byref(_beam(beam)), ct.c_void_p(b.data_ptr())), "dda_rhs")
        return b

    def matvec(self, beam, x, y=None):
        y = self.vector() if y is None else y
        _check(lib().dda_matvec(self._h, ct.byref(_beam(beam)), _ptr(x, torch.complex128, (3, self.n), "x"),
                                _ptr(y, torch.complex128, (3, self.n), "y")), "dda_matvec")
        return y

    def matvec_noalloc(self, beam, x, y):
        """dda_matvec_noalloc: the product with the library's fixed work array (y given by the caller)."""
        _check(lib().dda_matvec_noalloc(self._h, ct.byref(_beam(beam)), _ptr(x, torch.complex128, (3, self.n), "x"),
                                        _ptr(y, torch.complex128, (3, self.n), "y")), "dda_matvec_noalloc")
        return y

    def matvec_f32(self, beam, x, y=None):
        y = self.vector(dtype=torch.complex64) if y is None else y
        _check(lib().dda_matvec_f32(self._h, ct.byref(_beam(beam)), _ptr(x, torch.complex64, (3, self.n), "x"),
                                    _ptr(y, torch.complex64, (3, self.n), "y")), "dda_matvec_f32")
        return y

    def matvec_batch(self, beams, x, y=None):
        n = len(beams)
        y = self.vector(n) if y is None else y
        _check(lib().dda_matvec_batch(self._h, _beams(beams), n, _ptr(x, torch.complex128, (n, 3, self.n), "x"),
                                      _ptr(y, torch.complex128, (n, 3, self.n), "y")), "dda_matvec_batch")
        return y

    def matvec_timed(self, beams, x, y, reps, precision=FP64):
        """Mean per-kernel and whole-product durations (ms) of `reps` back-to-back products of the
        [n][3][N] batch x (one beam per vector; complex64 for FP32_REFINE)."""
        if isinstance(beams, Beam) or hasattr(beams, "prop"):
            beams = [beams]
        n = len(beams)
        dt = torch.complex128 if precision == FP64 else torch.complex64
        k = (ct.c_float * 5)()
        tot = ct.c_float()
        _check(lib().dda_matvec_timed(self._h, _beams(beams), n, int(precision), _ptr(x, dt, (n, 3, self.n), "x"),
                                      _ptr(y, dt, (n, 3, self.n), "y"), int(reps), k, ct.byref(tot)),
               "dda_matvec_timed")
        return list(k), tot.value

    def tiles(self, precision=FP64):
        t = (ct.c_int32 * 2)()
        _check(lib().dda_get_tiles(self._h, int(precision), t), "dda_get_tiles")
        return [t[0], t[1]]

    def set_tiles(self, tiles, precision=FP64):
        t = (ct.c_int32 * 2)(*[int(v) for v in tiles])
        _check(lib().dda_set_tiles(self._h, int(precision), t), "dda_set_tiles")

    def tune(self, precision=FP64, reps=3, cache=None, n_rhs=1):
        """Autotune the x/y tile schedule (dda_tune).  With a cache file (JSON; default: the
        DDA_TUNE_CACHE environment variable, if set) a schedule found earlier for the same grid,
        padded grid and precision is reused instead of timed again."""
        import json
        cache = cache if cache is not None else os.environ.get("DDA_TUNE_CACHE")
        key = f"{self.grid}|{tuple(self.padded_grid())}|{int(precision)}|{int(n_rhs)}"
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                self.set_tiles(table[key], precision)
                return list(table[key])
        t = (ct.c_int32 * 2)()
        _check(lib().dda_tune(self._h, int(precision), int(n_rhs), int(reps), t), "dda_tune")
        res = [t[0], t[1]]
        if cache:
            table[key] = res
            with open(cache, "w") as f:
                json.dump(table, f)
        return res

    def solve(self, beams, tol=1e-5, solver=QMR, precision=FP64, maxit=0, check_every=0, inner_tol=0.0, x0=None,
              x_out=None, history=0, raise_on_fail=True, graph=0, x0_check=False, on_breakdown=BREAKDOWN_REPORT,
              resume=False, relax_at=0.0):
        n = len(beams)
        x_out = self.vector(n) if x_out is None else x_out
        opts = SolveOpts(solver, precision, maxit, check_every, inner_tol,
                         None if x0 is None else _ptr(x0, torch.complex128, (n, 3, self.n), "x0").value, graph,
                         1 if x0_check else 0, on_breakdown, 1 if resume else 0, float(relax_at))
        infos = (SolveInfo * n)()
        hists = []
        for i in range(n):
            if history:
                h = (ct.c_double * history)()
                hists.append(h)
                infos[i].res_hist = ct.cast(h, ct.POINTER(ct.c_double))
                infos[i].res_hist_cap = history
        st = lib().dda_solve(self._h, _beams(beams), n, float(tol), ct.byref(opts),
                             _ptr(x_out, torch.complex128, (n, 3, self.n), "x_out"), infos)
        out = []
        for i in range(n):
            d = {f: getattr(infos[i], f) for f, _ in SolveInfo._fields_ if f != "res_hist"}
            if history:
                d["res_hist"] = list(hists[i][: infos[i].res_hist_len])
            out.append(d)
        if raise_on_fail and st not in (OK,):
            _check(st, "dda_solve")
        return x_out, out, st

    def cross_sections(self, beam, x):
        out = (ct.c_double * 3)()
        _check(lib().dda_cross_sections(self._h, ct.byref(_beam(beam)), _ptr(x, torch.complex128, (3, self.n), "x"),
                                        out), "dda_cross_sections")
        return tuple(out)

    def farfield(self, beam, x, dirs):
        dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        F = np.zeros((len(dirs), 3), dtype=np.complex128)
        _check(lib().dda_farfield(self._h, ct.byref(_beam(beam)), _ptr(x, torch.complex128, (3, self.n), "x"),
                                  len(dirs), dirs.ctypes.data_as(ct.POINTER(ct.c_double)),
                                  F.ctypes.data_as(ct.POINTER(ct.c_double))), "dda_farfield")
        return F

    def checkpoint_save(self, path, x):
        """Write the last stopped double-precision solve (iterate x [n][3][N]) to `path`."""
        _check(lib().dda_checkpoint_save(self._h, ct.c_void_p(x.data_ptr()) if x.is_cuda else None,
                                         os.fsencode(path)), "dda_checkpoint_save")

    def checkpoint_load(self, path, x):
        """Read a checkpoint into the context and the iterate buffer x [n][3][N] (then solve with
        resume=True)."""
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex128 and x.is_contiguous()):
            raise TypeError("x must be a contiguous complex128 CUDA/HIP tensor")
        _check(lib().dda_checkpoint_load(self._h, ct.c_void_p(x.data_ptr()), os.fsencode(path)),
               "dda_checkpoint_load")

    def orientation_average(self, n_beta=3, n_gamma=3, tol=1e-5, solver=QMR, precision=FP64, maxit=0):
        """Orientation-averaged (Cext, Cabs, Csca) and the Romberg error of <Cext>
        (dda_orientation_average)."""
        opts = SolveOpts(solver, precision, maxit, 0, 0.0, None, 0, 0, BREAKDOWN_REPORT)
        out = (ct.c_double * 4)()
        _check(lib().dda_orientation_average(self._h, int(n_beta), int(n_gamma), float(tol), ct.byref(opts), out),
               "dda_orientation_average")
        return {"Cext": out[0], "Cabs": out[1], "Csca": out[2], "err": out[3]}

    def orientation_average_adaptive(self, eps=1e-3, n_beta_min=2, n_beta_max=8, n_gamma=3, tol=1e-5, solver=QMR,
                                     precision=FP64, maxit=0):
        """Orientation average with the cos(beta) grid doubled until Romberg's error estimates are
        at most eps <Cext> (dda_orientation_average_adaptive): averages, error estimates and the
        level n used (2^n + 1 beta values)."""
        opts = SolveOpts(solver, precision, maxit, 0, 0.0, None, 0, 0, BREAKDOWN_REPORT)
        out = (ct.c_double * 5)()
        n = ct.c_int32(0)
        _check(lib().dda_orientation_average_adaptive(self._h, float(eps), int(n_beta_min), int(n_beta_max),
                                                      int(n_gamma), float(tol), ct.byref(opts), out, ct.byref(n)),
               "dda_orientation_average_adaptive")
        return {"Cext": out[0], "Cabs": out[1], "Csca": out[2], "err": out[3], "err_abs": out[4], "n_beta": n.value}

    def orientation_average_mueller(self, theta, n_beta=3, n_gamma=3, n_alpha=8, tol=1e-5, solver=QMR,
                                    precision=FP64, maxit=0):
        """Orientation-averaged Mueller matrix [n_theta][4][4] (alpha through n_alpha scattering
        planes) and the Romberg error estimate of S11 per angle (dda_orientation_average_mueller)."""
        theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        M = np.zeros((len(theta), 4, 4), dtype=np.float64)
        err = np.zeros(len(theta), dtype=np.float64)
        opts = SolveOpts(solver, precision, maxit, 0, 0.0, None, 0, 0, BREAKDOWN_REPORT)
        dp = ct.POINTER(ct.c_double)
        _check(lib().dda_orientation_average_mueller(self._h, int(n_beta), int(n_gamma), int(n_alpha), float(tol),
                                                     ct.byref(opts), theta.ctypes.data_as(dp), len(theta),
                                                     M.ctypes.data_as(dp), err.ctypes.data_as(dp)),
               "dda_orientation_average_mueller")
        return M, err

    def asymmetry(self, beam, x, n_theta=0, n_phi=0):
        """(Csca, g) by integrating the far field over the sphere (dda_asymmetry; grid sizes 0:
        chosen from the particle's size)."""
        out = (ct.c_double * 2)()
        _check(lib().dda_asymmetry(self._h, ct.byref(_beam(beam)), _ptr(x, torch.complex128, (3, self.n), "x"),
                                   int(n_theta), int(n_phi), out), "dda_asymmetry")
        return out[0], out[1]

    def mueller(self, beam, x1, x2, phi, theta):
        theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        M = np.zeros((len(theta), 4, 4), dtype=np.float64)
        p2 = ct.c_void_p(0) if x2 is None else _ptr(x2, torch.complex128, (3, self.n), "x2")
        _check(lib().dda_mueller(self._h, ct.byref(_beam(beam)), _ptr(x1, torch.complex128, (3, self.n), "x1"), p2,
                                 float(phi), theta.ctypes.data_as(ct.POINTER(ct.c_double)), len(theta),
                                 M.ctypes.data_as(ct.POINTER(ct.c_double))), "dda_mueller")
        return M


def _info_dict(inf):
    return {f: getattr(inf, f) for f, _ in SolveInfo._fields_ if f != "res_hist"}


def tune_padding(mask, m, kd, polarizability=POL_LDR, n_rhs=1, reps=5, n_cand=3):
    """dda_tune_padding: the fastest padded grid (Lx, Ly, Lz) for this particle, and its product
    time in milliseconds; pass the grid as Context(..., pad=...)."""
    mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
    nz, ny, nx = mask.shape
    grid = (ct.c_int32 * 3)(nx, ny, nz)
    mm = (ct.c_double * 2)(complex(m).real, complex(m).imag)
    out = (ct.c_int32 * 3)()
    ms = ct.c_float()
    _check(lib().dda_tune_padding(grid, mask.ctypes.data_as(ct.POINTER(ct.c_uint8)), mm, float(kd), int(polarizability),
                                  int(n_rhs), int(reps), int(n_cand), out, ct.byref(ms)), "dda_tune_padding")
    return tuple(out), ms.value


def solve_many(contexts, beams, tol=1e-5, solver=QMR, maxit=0, check_every=0, graph=0, x_out=None,
               raise_on_fail=True, precision=FP64, pack=False):
    """One right-hand side per context, all solved together (dda_solve_many), each on its own stream;
    pack=True batches the particles that share a padded grid into one launch per pass."""
    n = len(contexts)
    if len(beams) != n:
        raise ValueError("one beam per context")
    xs = [c.vector() for c in contexts] if x_out is None else list(x_out)
    hs = (ct.c_void_p * n)(*[c._h.value for c in contexts])
    ps = (ct.c_void_p * n)(*[_ptr(x, torch.complex128, (3, c.n), "x_out").value for x, c in zip(xs, contexts)])
    opts = SolveOpts(solver, precision, maxit, check_every, 0.0, None, graph, 0)
    opts.pack = 1 if pack else 0
    infos = (SolveInfo * n)()
    st = lib().dda_solve_many(hs, n, _beams(beams), float(tol), ct.byref(opts), ps, infos)
    if raise_on_fail and st != OK:
        _check(st, "dda_solve_many")
    return xs, [_info_dict(infos[i]) for i in range(n)], st


class Net:
    """The learned-initial-guess network on a G^3 box (wraps dda_net_*)."""

    def __init__(self, grid, params, max_batch=8, device="cuda"):
        params = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if params.size != num_params():
            raise ValueError(f"expected {num_params()} parameters, got {params.size}")
        self.grid = int(grid)
        self.max_batch = int(max_batch)
        self.device = torch.device(device)
        h = ct.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().dda_net_create(ct.byref(h), self.grid, self.max_batch, params.ctypes.data, ct.c_void_p(stream)),
               "dda_net_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dda_net_free(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def cells(self):
        return self.grid ** 3

    def params(self):
        out = np.empty(num_params(), dtype=np.float32)
        _check(lib().dda_net_get_params(self._h, out.ctypes.data), "dda_net_get_params")
        return out

    def set_params(self, params):
        params = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        _check(lib().dda_net_set_params(self._h, params.ctypes.data), "dda_net_set_params")

    def features(self, ctx, beam, out=None):
        out = torch.empty((self.cells, 16), dtype=torch.bfloat16, device=self.device) if out is None else out
        _check(lib().dda_net_features(self._h, ctx._h, ct.byref(_beam(beam)),
                                      _ptr(out, torch.bfloat16, (self.cells, 16), "feat")), "dda_net_features")
        return out

    def target(self, ctx, beam, x, out=None):
        out = torch.empty((self.cells, 6), dtype=torch.float32, device=self.device) if out is None else out
        _check(lib().dda_net_target(self._h, ctx._h, ct.byref(_beam(beam)), _ptr(x, torch.complex128, (3, ctx.n), "x"),
                                    _ptr(out, torch.float32, (self.cells, 6), "tgt")), "dda_net_target")
        return out

    def forward(self, feat):
        b = feat.shape[0]
        out = torch.empty((b, self.cells, 6), dtype=torch.float32, device=self.device)
        _check(lib().dda_net_forward(self._h, _ptr(feat, torch.bfloat16, (b, self.cells, 16), "feat"), b,
                                     _ptr(out, torch.float32, (b, self.cells, 6), "out")), "dda_net_forward")
        return out

    def grad(self, feat, tgt):
        b = feat.shape[0]
        loss = ct.c_double()
        g = np.empty(num_params(), dtype=np.float32)
        _check(lib().dda_net_grad(self._h, _ptr(feat, torch.bfloat16, (b, self.cells, 16), "feat"),
                                  _ptr(tgt, torch.float32, (b, self.cells, 6), "tgt"), b, ct.byref(loss),
                                  g.ctypes.data), "dda_net_grad")
        return loss.value, g

    def train_step(self, feat, tgt, lr):
        b = feat.shape[0]
        loss = ct.c_double()
        _check(lib().dda_net_train_step(self._h, _ptr(feat, torch.bfloat16, (b, self.cells, 16), "feat"),
                                        _ptr(tgt, torch.float32, (b, self.cells, 6), "tgt"), b, float(lr),
                                        ct.byref(loss)), "dda_net_train_step")
        return loss.value

    def guess(self, ctx, beams, feat=None):
        """Initial guesses [n][3][N] for the beams on ctx's particle."""
        n = len(beams)
        if feat is None:
            feat = torch.empty((n, self.cells, 16), dtype=torch.bfloat16, device=self.device)
            for i, b in enumerate(beams):
                self.features(ctx, b, feat[i])
        x0 = ctx.vector(n)
        _check(lib().dda_guess(ctx._h, self._h, _beams(beams), n, _ptr(feat, torch.bfloat16, (n, self.cells, 16), "feat"),
                               _ptr(x0, torch.complex128, (n, 3, ctx.n), "x0")), "dda_guess")
        return x0


def num_params():
    return int(lib().dda_net_num_params())
