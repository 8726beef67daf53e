"""Python binding of libmacproj.so (ctypes): argument marshalling only.

Every step of the projection runs in the HIP library; this module turns torch
tensors into device pointers (``data_ptr()``) and torch's current stream into
a ``hipStream_t``.  Function names follow the C ABI in include/macproj.h.
The library must be built (``python -m paper_1910_12979_amd.build``); there is
no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os
from types import SimpleNamespace

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmacproj.so")

MG_OK, MG_PENDING = 0, 1
STATUS = {0: "OK", 1: "PENDING", -1: "INVALID_ARG", -2: "BAD_SIZE", -3: "INCOMPATIBLE_RHS",
          -4: "NOT_CONVERGED", -5: "NONFINITE", -6: "OOM", -7: "HIP", -8: "BUDGET", -9: "BUSY"}
MG_BC_PERIODIC, MG_BC_WALL, MG_BC_OUTFLOW, MG_BC_WALL_OUTFLOW, MG_BC_OUTFLOW_WALL = 0, 1, 2, 3, 4
MG_FP64, MG_MIXED = 0, 1
STEP = {"smooth": 0, "resid_restrict": 1, "prolong": 2, "coarse": 3, "down": 4, "up": 5}
ARRAY = {"phi": 0, "f": 1, "bx": 2, "by": 3, "bz": 4}
HIST_MAX = 128


class MGError(RuntimeError):
    def __init__(self, code, detail=""):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__(f"{self.name} ({code}): {detail}")


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double), ("bc", ctypes.c_int32 * 3),
                ("pre_sweeps", ctypes.c_int32), ("post_sweeps", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("max_cycles", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("inner_cycles", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("cycles", ctypes.c_int32), ("nlevels", ctypes.c_int32),
                ("hist_len", ctypes.c_int32), ("rel_resid0", ctypes.c_double), ("rel_resid", ctypes.c_double),
                ("mean_removed", ctypes.c_double), ("sum_f", ctypes.c_double),
                ("sum_abs_f", ctypes.c_double), ("norm_f", ctypes.c_double),
                ("phi_mean", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_smooth", ctypes.c_double), ("ms_other", ctypes.c_double),
                ("bytes_model", ctypes.c_double), ("resid_hist", ctypes.c_double * HIST_MAX)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "resid_hist"}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        d["hist"] = list(self.resid_hist[: max(self.hist_len, 0)])
        return d


MG_KIND_MAC, MG_KIND_NODAL = 0, 1


class Problem(ctypes.Structure):
    _fields_ = [("p", Params), ("rho", ctypes.c_void_p), ("beta0_cc", ctypes.c_void_p),
                ("beta0_edge", ctypes.c_void_p), ("S", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("w", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("kind", ctypes.c_int32), ("box", ctypes.c_int32 * 3)]


_lib = None


def lib():
    """Load libmacproj.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the library binds to)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1910_12979_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        P, S = ctypes.POINTER(Params), ctypes.POINTER(Stats)
        L.mg_default_params.argtypes = [P, i32, i32, i32, d]
        L.mg_default_params.restype = None
        L.mg_num_levels_for.argtypes = [P]
        L.mg_num_levels_for.restype = i32
        L.mg_workspace_bytes.argtypes = [P]
        L.mg_workspace_bytes.restype = ctypes.c_size_t
        L.mg_setup.argtypes = [P, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.mg_destroy.argtypes = [vp]
        L.mg_set_params.argtypes = [vp, P]
        L.mg_set_coefficients.argtypes = [vp, vp, vp, vp, vp]
        L.mac_project.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, S, vp]
        L.mg_vcycle.argtypes = [vp, vp, vp, ctypes.POINTER(d), vp]
        L.mg_level_info.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(d)]
        L.mg_level_copy.argtypes = [vp, i32, i32, vp, i32, vp]
        L.mg_level_step.argtypes = [vp, i32, i32, i32, vp]
        L.project_batch.argtypes = [i32, ctypes.POINTER(Problem), S, vp]
        L.serve_create.argtypes = [ctypes.c_size_t, i32, ctypes.POINTER(vp)]
        L.serve_submit.argtypes = [vp, ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_uint64)]
        L.serve_poll.argtypes = [vp, ctypes.c_uint64, S]
        L.serve_wait.argtypes = [vp, ctypes.c_uint64, S]
        L.serve_counters.argtypes = [vp, ctypes.POINTER(d)]
        L.serve_destroy.argtypes = [vp]
        L.mg_tune_sweep.argtypes = [i32]
        L.mg_autotune.argtypes = [vp, i32, vp]
        L.mg_sweep_config.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.mg_set_graphs.argtypes = [vp, i32]
        L.mg_set_bottom.argtypes = [vp, i32]
        L.mg_set_boxes.argtypes = [vp, ctypes.POINTER(i32)]
        L.mg_beta0_from_p0.argtypes = [i32, d, vp, vp, vp, vp, vp, vp]
        L.mac_project_full.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, S, vp]
        d3 = ctypes.POINTER(d)
        L.mac_project_radial.argtypes = [vp, vp, i32, d, vp, d3, vp, vp, vp, vp, vp, S, vp]
        L.mg_map_radial.argtypes = [i32, i32, i32, d, i32, d, vp, d3, vp, vp]
        L.nodal_num_levels_for.argtypes = [P]
        L.nodal_num_levels_for.restype = i32
        L.nodal_setup.argtypes = [P, ctypes.POINTER(vp)]
        L.nodal_destroy.argtypes = [vp]
        L.nodal_project.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, S, vp]
        L.nodal_set_coefficients.argtypes = [vp, vp, vp, vp]
        L.nodal_level_info.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(d)]
        L.nodal_level_copy.argtypes = [vp, i32, i32, vp, i32, vp]
        L.nodal_level_step.argtypes = [vp, i32, i32, i32, vp]
        L.nodal_set_graphs.argtypes = [vp, i32]
        L.nodal_set_bottom.argtypes = [vp, i32]
        L.nodal_tune_sweep.argtypes = [i32]
        L.mac_project_static.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, S, vp]
        cp, i3 = ctypes.c_char_p, ctypes.POINTER(i32)
        L.mg_tune_cache_save.argtypes = [cp]
        L.mg_tune_cache_load.argtypes = [cp]
        L.mg_tune_cache_clear.argtypes = []
        L.mg_tune_record.argtypes = [cp, i3, i32, i32, i32, i32]
        L.mg_tune_lookup.argtypes = [cp, i3, i32, i32, i32]
        L.mg_strerror.argtypes = [ctypes.c_int]
        L.mg_strerror.restype = ctypes.c_char_p
        L.mg_last_error.argtypes = []
        L.mg_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def mg_tune_sweep(cfg: int):
    """Force a fused-sweep tile configuration (-1: per-shape default)."""
    _check(lib().mg_tune_sweep(int(cfg)))


def _cstr(x):
    return None if x is None else str(x).encode()


def tune_cache_save(path=None) -> int:
    """Write the tuning table (None: to MACPROJ_TUNE_CACHE); entries written."""
    return _check_count(lib().mg_tune_cache_save(_cstr(path)))


def tune_cache_load(path=None) -> int:
    """Merge a tuning cache file into the table; entries taken."""
    return _check_count(lib().mg_tune_cache_load(_cstr(path)))


def tune_cache_clear():
    _check(lib().mg_tune_cache_clear())


def tune_record(n, cfg, rho=True, fp64=True, coarse=False, arch=None):
    t = (ctypes.c_int32 * 3)(*[int(a) for a in n])
    _check(lib().mg_tune_record(_cstr(arch), t, int(rho), int(fp64), int(coarse), int(cfg)))


def tune_lookup(n, rho=True, fp64=True, coarse=False, arch=None) -> int:
    t = (ctypes.c_int32 * 3)(*[int(a) for a in n])
    return lib().mg_tune_lookup(_cstr(arch), t, int(rho), int(fp64), int(coarse))


def _check_count(code):
    if code < 0:
        raise MGError(code, last_error())
    return code


def last_error() -> str:
    return lib().mg_last_error().decode()


def _check(code, allow=(MG_OK,)):
    if code not in allow:
        raise MGError(code, last_error())
    return code


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, dtype=None, shape=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def bc_code(periodic_d, out_lo, out_hi):
    """mg_bc of one direction from its periodic flag and outflow flags."""
    if periodic_d:
        return MG_BC_PERIODIC
    return {(False, False): MG_BC_WALL, (True, True): MG_BC_OUTFLOW,
            (False, True): MG_BC_WALL_OUTFLOW, (True, False): MG_BC_OUTFLOW_WALL}[(bool(out_lo), bool(out_hi))]


def make_params(n, dx, periodic=(True, True, False), pre_sweeps=2, post_sweeps=2, rtol=1e-10,
                max_cycles=100, precision="fp64", outflow=None, inner_cycles=0) -> Params:
    """``outflow``: None or six booleans (x low, x high, ..., z high) marking
    sides of non-periodic directions as outflow sides (phi = 0).
    ``inner_cycles``: FP32 V-cycles per refinement step in mixed precision
    (0: one)."""
    p = Params()
    nx, ny, nz = n
    lib().mg_default_params(ctypes.byref(p), nx, ny, nz, float(dx))
    outflow = (False,) * 6 if outflow is None else tuple(outflow)
    for d in range(3):
        p.bc[d] = bc_code(periodic[d], outflow[2 * d], outflow[2 * d + 1])
    p.pre_sweeps, p.post_sweeps = pre_sweeps, post_sweeps
    p.rtol, p.max_cycles = float(rtol), int(max_cycles)
    p.precision = MG_MIXED if precision in ("mixed", MG_MIXED) else MG_FP64
    p.inner_cycles = int(inner_cycles)
    return p


def mg_num_levels_for(params: Params) -> int:
    return lib().mg_num_levels_for(ctypes.byref(params))


def mg_workspace_bytes(params: Params) -> int:
    return lib().mg_workspace_bytes(ctypes.byref(params))


def field_shapes(n):
    nx, ny, nz = n
    return {"rho": (nz, ny, nx), "S": (nz, ny, nx), "phi": (nz, ny, nx), "u": (nz, ny, nx + 1),
            "v": (nz, ny + 1, nx), "w": (nz + 1, ny, nx), "beta0_cc": (nz,), "beta0_edge": (nz + 1,)}


class Hierarchy:
    """An mg_setup handle: one box shape on the current device."""

    def __init__(self, params: Params, workspace=None):
        self.params = params
        self.n = tuple(params.n)
        self._h = ctypes.c_void_p()
        ws = _ptr(workspace, name="workspace") if workspace is not None else None
        nbytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
        _check(lib().mg_setup(ctypes.byref(params), ws, nbytes, ctypes.byref(self._h)))
        self.nlevels = lib().mg_num_levels_for(ctypes.byref(params))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().mg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: Params):
        _check(lib().mg_set_params(self._h, ctypes.byref(params)))
        self.params = params

    def set_coefficients(self, rho, beta0_cc, beta0_edge, stream=None):
        import torch
        sh = field_shapes(self.n)
        _check(lib().mg_set_coefficients(self._h, _ptr(rho, torch.float64, sh["rho"], "rho"),
                                         _ptr(beta0_cc, torch.float64, sh["beta0_cc"], "beta0_cc"),
                                         _ptr(beta0_edge, torch.float64, sh["beta0_edge"], "beta0_edge"),
                                         _stream(stream)))

    def mac_project(self, rho, beta0_cc, beta0_edge, S, u, v, w, phi=None, stream=None,
                    allow=(MG_OK,)):
        """Project in place; returns the stats dict.  Raises MGError unless the
        status is in ``allow``."""
        import torch
        sh = field_shapes(self.n)
        f64 = torch.float64
        st = Stats()
        code = lib().mac_project(self._h, _ptr(rho, f64, sh["rho"], "rho"),
                                 _ptr(beta0_cc, f64, sh["beta0_cc"], "beta0_cc"),
                                 _ptr(beta0_edge, f64, sh["beta0_edge"], "beta0_edge"),
                                 _ptr(S, f64, sh["S"], "S"), _ptr(u, f64, sh["u"], "u"),
                                 _ptr(v, f64, sh["v"], "v"), _ptr(w, f64, sh["w"], "w"),
                                 _ptr(phi, f64, sh["phi"], "phi"), ctypes.byref(st), _stream(stream))
        _check(code, allow)
        out = st.as_dict()
        out["code"] = code
        return out

    def mac_project_full(self, rho, beta0_cc, beta0_edge, S, p0_cc, gamma1_cc, dp0dt_cc, u, v, w, phi=None,
                         stream=None, allow=(MG_OK,)):
        """mac_project with the dp0/dt term of the constraint given per layer
        (p0, Gamma1 and dp0/dt at the layer centres)."""
        import torch
        sh = field_shapes(self.n)
        f64 = torch.float64
        nz = self.n[2]
        st = Stats()
        code = lib().mac_project_full(self._h, _ptr(rho, f64, sh["rho"], "rho"),
                                      _ptr(beta0_cc, f64, sh["beta0_cc"], "beta0_cc"),
                                      _ptr(beta0_edge, f64, sh["beta0_edge"], "beta0_edge"),
                                      _ptr(S, f64, sh["S"], "S"), _ptr(p0_cc, f64, (nz,), "p0_cc"),
                                      _ptr(gamma1_cc, f64, (nz,), "gamma1_cc"),
                                      _ptr(dp0dt_cc, f64, (nz,), "dp0dt_cc"), _ptr(u, f64, sh["u"], "u"),
                                      _ptr(v, f64, sh["v"], "v"), _ptr(w, f64, sh["w"], "w"),
                                      _ptr(phi, f64, sh["phi"], "phi"), ctypes.byref(st), _stream(stream))
        _check(code, allow)
        out = st.as_dict()
        out["code"] = code
        return out

    def mac_project_radial(self, rho, beta0_r, dr, centre, S, u, v, w, phi=None, stream=None, allow=(MG_OK,)):
        """mac_project with beta0 given as a radial profile beta0_r (device,
        values at r = (m + 1/2) dr) about ``centre`` (3 floats)."""
        import torch
        sh = field_shapes(self.n)
        f64 = torch.float64
        st = Stats()
        nr = int(beta0_r.shape[0])
        c = (ctypes.c_double * 3)(*[float(x) for x in centre])
        code = lib().mac_project_radial(self._h, _ptr(rho, f64, sh["rho"], "rho"), nr, float(dr),
                                        _ptr(beta0_r, f64, (nr,), "beta0_r"), c, _ptr(S, f64, sh["S"], "S"),
                                        _ptr(u, f64, sh["u"], "u"), _ptr(v, f64, sh["v"], "v"),
                                        _ptr(w, f64, sh["w"], "w"), _ptr(phi, f64, sh["phi"], "phi"),
                                        ctypes.byref(st), _stream(stream))
        _check(code, allow)
        out = st.as_dict()
        out["code"] = code
        return out

    def mg_vcycle(self, phi, rhs, stream=None):
        import torch
        sh = field_shapes(self.n)["phi"]
        rel = ctypes.c_double()
        _check(lib().mg_vcycle(self._h, _ptr(phi, torch.float64, sh, "phi"), _ptr(rhs, torch.float64, sh, "rhs"),
                               ctypes.byref(rel), _stream(stream)))
        return rel.value

    def mg_autotune(self, reps=10, stream=None):
        """Pick the fastest sweep tile configuration per level shape."""
        _check(lib().mg_autotune(self._h, int(reps), _stream(stream)))

    def set_graphs(self, enable: bool):
        """Replay captured V-cycles (default on) or launch every cycle eagerly."""
        _check(lib().mg_set_graphs(self._h, 1 if enable else 0))

    def set_bottom(self, enable: bool):
        """Coarse levels in one workgroup launch (default on) or per-level launches."""
        _check(lib().mg_set_bottom(self._h, 1 if enable else 0))

    def set_boxes(self, box):
        """Split the finest level into boxes of box = (bx, by, bz) cells with a
        halo exchange between them; None or (0, 0, 0) for a single box."""
        if box is None:
            _check(lib().mg_set_boxes(self._h, None))
            return
        t = (ctypes.c_int32 * 3)(*[int(b) for b in box])
        _check(lib().mg_set_boxes(self._h, t))

    def sweep_config(self, level):
        """Fused-sweep tile (tx, ty, tz, index) of a level, or None if unfused."""
        t = (ctypes.c_int32 * 4)()
        _check(lib().mg_sweep_config(self._h, level, t))
        return None if t[3] < 0 else (t[0], t[1], t[2], t[3])

    def level_info(self, level):
        dims = (ctypes.c_int32 * 3)()
        dx = ctypes.c_double()
        _check(lib().mg_level_info(self._h, level, dims, ctypes.byref(dx)))
        return (dims[0], dims[1], dims[2]), dx.value

    def level_copy(self, level, array, tensor, to_hierarchy, stream=None):
        import torch
        (nx, ny, nz), _ = self.level_info(level)
        _check(lib().mg_level_copy(self._h, level, ARRAY[array],
                                   _ptr(tensor, torch.float64, (nz, ny, nx), array),
                                   1 if to_hierarchy else 0, _stream(stream)))

    def level_step(self, level, step, arg=0, stream=None):
        _check(lib().mg_level_step(self._h, level, STEP[step], arg, _stream(stream)))


STATIC_SCRATCH_BYTES = 32 << 20


def mac_project_static(params: Params, rho, beta0_cc, beta0_edge, S, u, v, w, phi=None, stream=None,
                       allow=(MG_OK,)):
    """The allocation-free projection (no hierarchy handle: the library's
    fixed per-device scratch array holds the levels).  Returns the stats dict."""
    import torch
    sh = field_shapes(tuple(params.n))
    f64 = torch.float64
    st = Stats()
    code = lib().mac_project_static(ctypes.byref(params), _ptr(rho, f64, sh["rho"], "rho"),
                                    _ptr(beta0_cc, f64, sh["beta0_cc"], "beta0_cc"),
                                    _ptr(beta0_edge, f64, sh["beta0_edge"], "beta0_edge"),
                                    _ptr(S, f64, sh["S"], "S"), _ptr(u, f64, sh["u"], "u"),
                                    _ptr(v, f64, sh["v"], "v"), _ptr(w, f64, sh["w"], "w"),
                                    _ptr(phi, f64, sh["phi"], "phi"), ctypes.byref(st), _stream(stream))
    _check(code, allow)
    out = st.as_dict()
    out["code"] = code
    return out


def mg_setup(params: Params, workspace=None) -> Hierarchy:
    return Hierarchy(params, workspace)


def mac_project(h: Hierarchy, *args, **kw):
    return h.mac_project(*args, **kw)


def mg_vcycle(h: Hierarchy, phi, rhs, stream=None):
    return h.mg_vcycle(phi, rhs, stream)


def mg_destroy(h: Hierarchy):
    h.close()


# ---------------------------------------------------------------- problems
def mg_beta0_from_p0(rho0_base, p0_edge, p0_cc, gamma1_cc, stream=None):
    """beta0 at layer centres and z faces from p0 and the layer Gamma1, on the
    device of p0_cc (new tensors, filled on the stream)."""
    import torch
    nz = p0_cc.shape[0]
    f64 = torch.float64
    b0c = torch.empty(nz, dtype=f64, device=p0_cc.device)
    b0e = torch.empty(nz + 1, dtype=f64, device=p0_cc.device)
    _check(lib().mg_beta0_from_p0(nz, float(rho0_base), _ptr(p0_edge, f64, (nz + 1,), "p0_edge"),
                                  _ptr(p0_cc, f64, (nz,), "p0_cc"), _ptr(gamma1_cc, f64, (nz,), "gamma1_cc"),
                                  _ptr(b0c, f64, (nz,), "beta0_cc"), _ptr(b0e, f64, (nz + 1,), "beta0_edge"),
                                  _stream(stream)))
    return b0c, b0e


def mg_map_radial(n, dx, beta0_r, dr, centre, stream=None):
    """beta0 of a radial profile at the cell centres of an n box (a new
    device tensor (nz, ny, nx), filled on the stream)."""
    import torch
    nx, ny, nz = n
    f64 = torch.float64
    nr = int(beta0_r.shape[0])
    out = torch.empty((nz, ny, nx), dtype=f64, device=beta0_r.device)
    c = (ctypes.c_double * 3)(*[float(x) for x in centre])
    _check(lib().mg_map_radial(nx, ny, nz, float(dx), nr, float(dr), _ptr(beta0_r, f64, (nr,), "beta0_r"), c,
                               _ptr(out, f64, (nz, ny, nx), "beta0_out"), _stream(stream)))
    return out


def to_device(prob, device="cuda", phi=True):
    """Copy an inputs.Problem's host arrays to device tensors (base-state
    arrays that the problem does not carry stay None)."""
    import torch
    names = ("rho", "beta0_cc", "beta0_edge", "S", "u", "v", "w", "p0_cc", "p0_edge", "gamma1_cc", "dp0dt_cc",
             "beta0_r")
    t = {name: (torch.from_numpy(np.ascontiguousarray(getattr(prob, name))).to(device)
                if getattr(prob, name, None) is not None else None)
         for name in names}
    nx, ny, nz = prob.n
    t["phi"] = torch.zeros((nz, ny, nx), dtype=torch.float64, device=device) if phi else None
    return SimpleNamespace(**t)


def params_of(prob, precision="fp64", rtol=None, max_cycles=None, inner_cycles=0) -> Params:
    return make_params(prob.n, prob.dx, prob.periodic, prob.pre_sweeps, prob.post_sweeps,
                       prob.rtol if rtol is None else rtol,
                       prob.max_cycles if max_cycles is None else max_cycles, precision,
                       outflow=getattr(prob, "outflow", None), inner_cycles=inner_cycles)


def problem_struct(params: Params, d, box=None) -> Problem:
    """mg_problem for device tensors d (a namespace from to_device); box:
    cells per box of a multi-box finest level (None: one box)."""
    import torch
    sh = field_shapes(tuple(params.n))
    f64 = torch.float64
    pr = Problem()
    pr.p = params
    pr.rho = _ptr(d.rho, f64, sh["rho"], "rho")
    pr.beta0_cc = _ptr(d.beta0_cc, f64, sh["beta0_cc"], "beta0_cc")
    pr.beta0_edge = _ptr(d.beta0_edge, f64, sh["beta0_edge"], "beta0_edge")
    pr.S = _ptr(d.S, f64, sh["S"], "S")
    pr.u = _ptr(d.u, f64, sh["u"], "u")
    pr.v = _ptr(d.v, f64, sh["v"], "v")
    pr.w = _ptr(d.w, f64, sh["w"], "w")
    pr.phi = _ptr(d.phi, f64, sh["phi"], "phi") if d.phi is not None else None
    pr.kind = MG_KIND_MAC
    if box is not None:
        for k in range(3):
            pr.box[k] = int(box[k])
    return pr


def nodal_problem_struct(params: Params, d) -> Problem:
    """mg_problem of kind MG_KIND_NODAL for device tensors d (a namespace
    from nodal_to_device): u, v, w are the cell-centred velocities, phi the
    node values."""
    import torch
    nx, ny, nz = tuple(params.n)
    cell = (nz, ny, nx)
    per = tuple(params.bc[k] == MG_BC_PERIODIC for k in range(3))
    f64 = torch.float64
    pr = Problem()
    pr.p = params
    pr.rho = _ptr(d.rho, f64, cell, "rho")
    pr.beta0_cc = _ptr(d.beta0_cc, f64, (nz,), "beta0_cc")
    pr.beta0_edge = None
    pr.S = _ptr(d.S, f64, cell, "S")
    pr.u = _ptr(d.uc, f64, cell, "uc")
    pr.v = _ptr(d.vc, f64, cell, "vc")
    pr.w = _ptr(d.wc, f64, cell, "wc")
    pr.phi = _ptr(d.phi, f64, node_dims((nx, ny, nz), per)[::-1], "phi") if d.phi is not None else None
    pr.kind = MG_KIND_NODAL
    return pr


def project_batch_problems(problems, stream=None):
    """project_batch over mg_problem structs (any kinds); returns (code, [stats dicts])."""
    n = len(problems)
    arr = (Problem * max(n, 1))()
    for i, pr in enumerate(problems):
        arr[i] = pr
    stats = (Stats * max(n, 1))()
    code = lib().project_batch(n, arr, stats, _stream(stream))
    return code, [stats[i].as_dict() for i in range(n)]


def project_batch(params_list, tensors_list, stream=None, boxes=None):
    """Solve many MAC problems with shared launches; returns (code, [stats dicts])."""
    boxes = boxes or [None] * len(params_list)
    return project_batch_problems([problem_struct(p, d, b) for p, d, b in zip(params_list, tensors_list, boxes)],
                                  stream)


class Server:
    """serve_create / serve_submit / serve_poll / serve_wait / serve_destroy."""

    def __init__(self, hbm_budget_bytes, max_inflight=64):
        self._s = ctypes.c_void_p()
        _check(lib().serve_create(int(hbm_budget_bytes), int(max_inflight), ctypes.byref(self._s)))
        self._keep = {}

    def submit(self, params: Params, d, box=None) -> int:
        """Queue a MAC projection of the tensors in d (box: multi-box finest
        level); they must stay alive (this object keeps a reference) until
        the ticket completes."""
        return self.submit_problem(problem_struct(params, d, box), d)

    def submit_nodal(self, params: Params, d) -> int:
        """Queue a nodal projection of the tensors in d (from nodal_to_device)."""
        return self.submit_problem(nodal_problem_struct(params, d), d)

    def submit_problem(self, pr: Problem, d) -> int:
        import torch
        torch.cuda.current_stream().synchronize()      # inputs ready for the server's stream
        t = ctypes.c_uint64()
        _check(lib().serve_submit(self._s, ctypes.byref(pr), ctypes.byref(t)))
        self._keep[t.value] = d            # keep the buffers alive until done
        return t.value

    def poll(self, ticket):
        st = Stats()
        code = lib().serve_poll(self._s, ticket, ctypes.byref(st))
        if code == MG_PENDING:
            return None
        self._keep.pop(ticket, None)
        out = st.as_dict()
        out["code"] = code
        return out

    def wait(self, ticket):
        st = Stats()
        code = lib().serve_wait(self._s, ticket, ctypes.byref(st))
        self._keep.pop(ticket, None)
        out = st.as_dict()
        out["code"] = code
        return out

    def counters(self):
        c = (ctypes.c_double * 6)()
        _check(lib().serve_counters(self._s, c))
        return {"submitted": c[0], "completed": c[1], "queued": c[2], "inflight": c[3],
                "resident_bytes": c[4], "peak_inflight": c[5]}

    def close(self):
        if self._s.value:
            lib().serve_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


serve_create = Server


# ---------------------------------------------------------------- nodal projection
NODAL_ARRAY = {"phi": 0, "f": 1, "sigma": 2}


def node_dims(n, periodic):
    """Node counts (Nx, Ny, Nz): n in a periodic direction, n + 1 at walls."""
    return tuple(int(n[d]) + (0 if periodic[d] else 1) for d in range(3))


class NodalHierarchy:
    """A nodal_setup handle (nodal projection of cell-centred velocities)."""

    def __init__(self, params: Params):
        self.params = params
        self.n = tuple(params.n)
        self.periodic = tuple(params.bc[d] == MG_BC_PERIODIC for d in range(3))
        self._h = ctypes.c_void_p()
        _check(lib().nodal_setup(ctypes.byref(params), ctypes.byref(self._h)))
        self.nlevels = lib().nodal_num_levels_for(ctypes.byref(params))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().nodal_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def project(self, rho, beta0_cc, S, uc, vc, wc, phi=None, stream=None, allow=(MG_OK,)):
        import torch
        nx, ny, nz = self.n
        cell = (nz, ny, nx)
        f64 = torch.float64
        st = Stats()
        code = lib().nodal_project(self._h, _ptr(rho, f64, cell, "rho"), _ptr(beta0_cc, f64, (nz,), "beta0_cc"),
                                   _ptr(S, f64, cell, "S"), _ptr(uc, f64, cell, "uc"), _ptr(vc, f64, cell, "vc"),
                                   _ptr(wc, f64, cell, "wc"),
                                   _ptr(phi, f64, node_dims(self.n, self.periodic)[::-1], "phi"),
                                   ctypes.byref(st), _stream(stream))
        _check(code, allow)
        out = st.as_dict()
        out["code"] = code
        return out

    def set_graphs(self, enable: bool):
        _check(lib().nodal_set_graphs(self._h, 1 if enable else 0))

    def set_bottom(self, enable: bool):
        _check(lib().nodal_set_bottom(self._h, 1 if enable else 0))

    def set_coefficients(self, rho, beta0_cc, stream=None):
        import torch
        nx, ny, nz = self.n
        _check(lib().nodal_set_coefficients(self._h, _ptr(rho, torch.float64, (nz, ny, nx), "rho"),
                                            _ptr(beta0_cc, torch.float64, (nz,), "beta0_cc"), _stream(stream)))

    def level_info(self, level):
        dims = (ctypes.c_int32 * 6)()
        dx = ctypes.c_double()
        _check(lib().nodal_level_info(self._h, level, dims, ctypes.byref(dx)))
        return (dims[0], dims[1], dims[2]), (dims[3], dims[4], dims[5]), dx.value

    def level_copy(self, level, array, tensor, to_hierarchy, stream=None):
        _check(lib().nodal_level_copy(self._h, level, NODAL_ARRAY[array], _ptr(tensor, name=array),
                                      1 if to_hierarchy else 0, _stream(stream)))

    def level_step(self, level, step, arg=0, stream=None):
        _check(lib().nodal_level_step(self._h, level, STEP[step], arg, _stream(stream)))


def nodal_tune_sweep(cfg: int):
    """Force a fused nodal sweep tile configuration (-1: per-level default)."""
    _check(lib().nodal_tune_sweep(int(cfg)))


def nodal_to_device(prob, device="cuda", phi=True):
    """Device tensors of an inputs.NodalProblem."""
    import torch
    t = {name: torch.from_numpy(np.ascontiguousarray(getattr(prob, name))).to(device)
         for name in ("rho", "beta0_cc", "S", "uc", "vc", "wc")}
    Nx, Ny, Nz = node_dims(prob.n, prob.periodic)
    t["phi"] = torch.zeros((Nz, Ny, Nx), dtype=torch.float64, device=device) if phi else None
    return SimpleNamespace(**t)
