"""ctypes binding of libcmhd.so (include/cmhd.h), argument marshalling only.

Device memory and streams come from PyTorch: the state is a float64 CUDA
(ROCm) tensor of shape [8, nz+6, ny, nx], the workspace a uint8 tensor, and
every call runs on torch's current stream.  All arithmetic of the step runs
in the library's kernels; if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libcmhd.so")

CMHD_OK, CMHD_EINVAL, CMHD_EDEVICE, CMHD_ENONFINITE, CMHD_EDT = 0, -1, -2, -3, -4
CMHD_ESTATE, CMHD_EWORKSPACE = -5, -6
CMHD_FP64, CMHD_FP32_SPLIT = 0, 1
CMHD_ZBC_PERIODIC, CMHD_ZBC_SOLAR = 0, 1
MAX_RAD = 16


class CmhdGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
                ("z0", ctypes.c_double), ("z1", ctypes.c_double),
                ("zbc", ctypes.c_int), ("prec", ctypes.c_int)]


class CmhdParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("gamma", "R", "mu0", "eta", "nu", "D_rho", "kappa0", "g_z")] + [
        ("Bext", ctypes.c_double * 3), ("B_floor", ctypes.c_double)] + [
        (n, ctypes.c_double) for n in
        ("eta_s", "chi_s", "chi_rho", "z_s", "z_t", "tau_u", "tau_A", "t_ramp", "f_bot")] + [
        ("n_rad", ctypes.c_int), ("rad_lnT", ctypes.c_double * MAX_RAD),
        ("rad_lnL", ctypes.c_double * MAX_RAD)] + [
        (n, ctypes.c_double) for n in ("T_rad_lo", "T_rad_hi", "c_adv", "c_diff", "c_nudge")] + [
        (n, ctypes.c_double) for n in
        ("nc_tau", "nc_lnrho_magn", "nc_lnrho_width", "nc_z_max", "nc_z_width")]


class CmhdGranParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int)] + [
        (n, ctypes.c_double) for n in
        ("Lx", "Ly", "r_gran", "r_lane", "r_excl", "t_gran", "v0", "vmin_frac", "life_var",
         "amp_var", "f_rot")]


class CmhdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cmhd error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load the library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is missing: build it with "
                          "`python -m paper_1908_08557_amd.build`")
    lib = ctypes.CDLL(LIBPATH)
    P, D, I, U, S = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_uint, ctypes.c_size_t
    sig = {
        "cmhd_init_grid": (I, [ctypes.POINTER(CmhdGrid), ctypes.POINTER(CmhdParams),
                               ctypes.POINTER(D), ctypes.POINTER(D), P, ctypes.POINTER(P)]),
        "cmhd_init_grid_z": (I, [ctypes.POINTER(CmhdGrid), ctypes.POINTER(CmhdParams),
                                 ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D), P,
                                 ctypes.POINTER(P)]),
        "cmhd_state_elems": (S, [P]),
        "cmhd_workspace_bytes": (S, [P]),
        "cmhd_bind_workspace": (I, [P, P, S]),
        "cmhd_set_stream": (I, [P, P]),
        "cmhd_set_driver": (I, [P, P, P, P]),
        "cmhd_set_driver_snapshots": (I, [P, P, D, P, D]),
        "cmhd_fill_ghosts": (I, [P, P, D]),
        "cmhd_rk3_step": (I, [P, P, ctypes.POINTER(D), D, ctypes.POINTER(D)]),
        "cmhd_cfl_dt": (I, [P, P, ctypes.POINTER(D)]),
        "cmhd_cfl_dt_noalloc": (I, [P, P, ctypes.POINTER(D)]),
        "cmhd_eval_rhs": (I, [P, P, D, P]),
        "cmhd_get_fields": (I, [P, P, U, P, I, I]),
        "cmhd_set_fields": (I, [P, P, U, P, I, I]),
        "cmhd_bz_plane": (I, [P, P, D, P]),
        "cmhd_check_finite": (I, [P, P]),
        "cmhd_adjoint_workspace_bytes": (S, [P]),
        "cmhd_bind_adjoint_workspace": (I, [P, P, S]),
        "cmhd_rk3_step_jvp": (I, [P, P, D, D, P, P, P]),
        "cmhd_rk3_step_vjp": (I, [P, P, D, D, P, P, P]),
        "cmhd_bz_plane_vjp": (I, [P, D, P, P]),
        "cmhd_profile_enable": (I, [P, I]),
        "cmhd_profile_read": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(I)]),
        "cmhd_last_error": (ctypes.c_char_p, [P]),
        "cmhd_destroy": (None, [P]),
        "cmhd_gran_create": (I, [ctypes.POINTER(CmhdGranParams), P, ctypes.POINTER(P)]),
        "cmhd_gran_workspace_bytes": (S, [P]),
        "cmhd_gran_bind_workspace": (I, [P, P, S]),
        "cmhd_gran_update": (I, [P, D, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D),
                                 ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)]),
        "cmhd_gran_velocity": (I, [P, D, P]),
        "cmhd_gran_list": (I, [P, ctypes.POINTER(D), I, ctypes.POINTER(I)]),
        "cmhd_gran_last_error": (ctypes.c_char_p, [P]),
        "cmhd_gran_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names the binding expects the library to export."""
    return ["cmhd_init_grid", "cmhd_init_grid_z", "cmhd_state_elems", "cmhd_workspace_bytes", "cmhd_bind_workspace",
            "cmhd_set_stream", "cmhd_set_driver", "cmhd_set_driver_snapshots",
            "cmhd_fill_ghosts", "cmhd_rk3_step",
            "cmhd_cfl_dt", "cmhd_cfl_dt_noalloc", "cmhd_eval_rhs", "cmhd_get_fields", "cmhd_set_fields", "cmhd_bz_plane", "cmhd_check_finite",
            "cmhd_adjoint_workspace_bytes", "cmhd_bind_adjoint_workspace", "cmhd_rk3_step_jvp",
            "cmhd_rk3_step_vjp", "cmhd_bz_plane_vjp",
            "cmhd_profile_enable", "cmhd_profile_read", "cmhd_last_error", "cmhd_destroy",
            "cmhd_gran_create", "cmhd_gran_workspace_bytes", "cmhd_gran_bind_workspace",
            "cmhd_gran_update", "cmhd_gran_velocity", "cmhd_gran_list", "cmhd_gran_last_error",
            "cmhd_gran_destroy"]


def make_grid(grid: dict, precision: str = "fp64") -> CmhdGrid:
    g = CmhdGrid()
    g.nx, g.ny, g.nz = grid["nx"], grid["ny"], grid["nz"]
    g.Lx, g.Ly, g.z0, g.z1 = grid["Lx"], grid["Ly"], grid["z0"], grid["z1"]
    g.zbc = CMHD_ZBC_SOLAR if grid["zbc"] == "solar" else CMHD_ZBC_PERIODIC
    g.prec = {"fp64": CMHD_FP64, "fp32_split": CMHD_FP32_SPLIT}[precision]
    return g


def make_params(par: dict) -> CmhdParams:
    p = CmhdParams()
    for name in ("gamma", "R", "mu0", "eta", "nu", "D_rho", "kappa0", "g_z", "B_floor",
                 "eta_s", "chi_s", "chi_rho", "z_s", "z_t", "tau_u", "tau_A", "t_ramp", "f_bot",
                 "T_rad_lo", "T_rad_hi", "c_adv", "c_diff", "c_nudge"):
        setattr(p, name, float(par[name]))
    for name, default in (("nc_tau", 0.0), ("nc_lnrho_magn", 8.0), ("nc_lnrho_width", 2.0),
                          ("nc_z_max", 3.0), ("nc_z_width", 0.3)):
        setattr(p, name, float(par.get(name, default)))
    for i in range(3):
        p.Bext[i] = float(par["Bext"][i])
    lnT = np.asarray(par["rad_lnT"], dtype=np.float64)
    lnL = np.asarray(par["rad_lnL"], dtype=np.float64)
    if len(lnT) > MAX_RAD:
        raise ValueError("radiation table too long")
    p.n_rad = len(lnT)
    for i in range(len(lnT)):
        p.rad_lnT[i] = lnT[i]
        p.rad_lnL[i] = lnL[i]
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Solver:
    """One library context: grid, parameters, bound workspace."""

    def __init__(self, grid: dict, params: dict, lnrho0_z, precision: str = "fp64",
                 device: str = "cuda", lnT0_z=None):
        self.lib = load()
        self.grid = dict(grid)
        self.params = dict(params)
        self.precision = precision
        self.device = torch.device(device)
        self._g = make_grid(grid, precision)
        self._p = make_params(params)
        lr = np.ascontiguousarray(np.asarray(lnrho0_z, dtype=np.float64))
        self._lr = lr
        if lnT0_z is None and "nc_lnT0_z" in params:
            lnT0_z = params["nc_lnT0_z"]
        lt = None if lnT0_z is None else np.ascontiguousarray(np.asarray(lnT0_z, np.float64))
        self._lt = lt
        dptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        ctx = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        zz = None
        if "z" in grid:
            zz = np.ascontiguousarray(np.asarray(grid["z"], dtype=np.float64))
        self._z = zz
        rc = self.lib.cmhd_init_grid_z(ctypes.byref(self._g), ctypes.byref(self._p), dptr(zz),
                                       dptr(lr), dptr(lt), ctypes.c_void_p(stream),
                                       ctypes.byref(ctx))
        if rc != CMHD_OK:
            raise CmhdError(rc, "cmhd_init_grid failed (see stderr)")
        self.ctx = ctx
        nbytes = self.lib.cmhd_workspace_bytes(ctx)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._check(self.lib.cmhd_bind_workspace(ctx, ctypes.c_void_p(base + off), nbytes))
        g = grid
        self.state_shape = (8, g["nz"] + 6, g["ny"], g["nx"])

    # -- helpers ---------------------------------------------------------------
    def _check(self, rc):
        if rc != CMHD_OK:
            msg = self.lib.cmhd_last_error(self.ctx).decode()
            raise CmhdError(rc, msg)

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self._check(self.lib.cmhd_set_stream(self.ctx, ctypes.c_void_p(s)))

    def _state(self, state):
        if (state.dtype != torch.float64 or not state.is_cuda or not state.is_contiguous()
                or tuple(state.shape) != self.state_shape):
            raise ValueError(f"state must be a contiguous float64 device tensor {self.state_shape}")
        return ctypes.c_void_p(state.data_ptr())

    def new_state(self, host_state=None):
        if host_state is None:
            return torch.zeros(self.state_shape, dtype=torch.float64, device=self.device)
        return torch.as_tensor(np.ascontiguousarray(host_state), dtype=torch.float64,
                               device=self.device).contiguous()

    # -- API ---------------------------------------------------------------------
    def set_driver(self, uh, bz=None, ah=None):
        self._stream()
        dev = lambda a: None if a is None else torch.as_tensor(
            np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a,
            dtype=torch.float64, device=self.device).contiguous()
        self._drv = (dev(uh), dev(bz), dev(ah))   # kept alive until the stream passes
        self._check(self.lib.cmhd_set_driver(self.ctx, _ptr(self._drv[0]), _ptr(self._drv[1]),
                                             _ptr(self._drv[2])))

    def set_driver_snapshots(self, uh0, t0, uh1, t1):
        """Nudging target interpolated linearly in time between u*_0 at t0 and
        u*_1 at t1 (device or host arrays [2, ny, nx])."""
        self._stream()
        dev = lambda a: torch.as_tensor(
            np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a,
            dtype=torch.float64, device=self.device).contiguous()
        self._drv = (dev(uh0), dev(uh1))
        self._check(self.lib.cmhd_set_driver_snapshots(self.ctx, _ptr(self._drv[0]), float(t0),
                                                       _ptr(self._drv[1]), float(t1)))

    def fill_ghosts(self, state, t=0.0):
        self._stream()
        self._check(self.lib.cmhd_fill_ghosts(self.ctx, self._state(state), float(t)))

    def rk3_step(self, state, t, dt):
        self._stream()
        tt = ctypes.c_double(t)
        used = ctypes.c_double(0.0)
        self._check(self.lib.cmhd_rk3_step(self.ctx, self._state(state), ctypes.byref(tt),
                                           float(dt), ctypes.byref(used)))
        return tt.value, used.value

    def eval_rhs(self, state, t=0.0):
        """Right-hand side dF/dt as a new device tensor in the state layout
        (entries outside the interior and the u_h ghost rows are zero)."""
        self._stream()
        out = torch.zeros(self.state_shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.cmhd_eval_rhs(self.ctx, self._state(state), float(t), _ptr(out)))
        return out

    def cfl_dt(self, state):
        self._stream()
        dt = ctypes.c_double(0.0)
        self._check(self.lib.cmhd_cfl_dt(self.ctx, self._state(state), ctypes.byref(dt)))
        return dt.value

    def cfl_dt_noalloc(self, state):
        """cmhd_cfl_dt_noalloc: the time step of a state whose ghost planes are
        filled, with the library's fixed device scratch (allocates nothing)."""
        self._stream()
        dt = ctypes.c_double(0.0)
        self._check(self.lib.cmhd_cfl_dt_noalloc(self.ctx, self._state(state), ctypes.byref(dt)))
        return dt.value

    def get_fields(self, state, mask=0xFF, with_ghosts=False):
        """Selected fields copied to a new host float64 array."""
        self._stream()
        nsel = bin(mask & 0xFF).count("1")
        g = self.grid
        nzc = g["nz"] + 6 if with_ghosts else g["nz"]
        out = np.empty((nsel, nzc, g["ny"], g["nx"]))
        self._check(self.lib.cmhd_get_fields(self.ctx, self._state(state), mask,
                                             ctypes.c_void_p(out.ctypes.data), 1,
                                             1 if with_ghosts else 0))
        return out

    def set_fields(self, state, src, mask=0xFF, with_ghosts=False):
        """Copy host fields [nsel, nz(+6), ny, nx] (the layout of get_fields)
        into the device state."""
        self._stream()
        nsel = bin(mask & 0xFF).count("1")
        g = self.grid
        nzc = g["nz"] + 6 if with_ghosts else g["nz"]
        a = np.ascontiguousarray(src, dtype=np.float64)
        if a.shape != (nsel, nzc, g["ny"], g["nx"]):
            raise ValueError(f"src must have shape {(nsel, nzc, g['ny'], g['nx'])}")
        self._check(self.lib.cmhd_set_fields(self.ctx, self._state(state), mask,
                                             ctypes.c_void_p(a.ctypes.data), 1,
                                             1 if with_ghosts else 0))
        return state

    def bz_plane(self, state, z, out=None):
        self._stream()
        if out is None:
            out = torch.empty((self.grid["ny"], self.grid["nx"]), dtype=torch.float64,
                              device=self.device)
        self._check(self.lib.cmhd_bz_plane(self.ctx, self._state(state), float(z), _ptr(out)))
        return out

    def check_finite(self, state):
        self._stream()
        rc = self.lib.cmhd_check_finite(self.ctx, self._state(state))
        if rc == CMHD_ENONFINITE:
            return False
        self._check(rc)
        return True

    # -- differentiation ---------------------------------------------------------
    def bind_adjoint(self):
        if getattr(self, "adj_workspace", None) is not None:
            return
        nbytes = self.lib.cmhd_adjoint_workspace_bytes(self.ctx)
        self.adj_workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.adj_workspace.data_ptr()
        off = (-base) % 256
        self._check(self.lib.cmhd_bind_adjoint_workspace(self.ctx, ctypes.c_void_p(base + off),
                                                         nbytes))

    def _plane2(self, a):
        if a is None:
            return None
        if (a.dtype != torch.float64 or not a.is_cuda or not a.is_contiguous()
                or tuple(a.shape) != (2, self.grid["ny"], self.grid["nx"])):
            raise ValueError("driver arrays must be contiguous float64 device tensors [2, ny, nx]")
        return a

    def rk3_step_jvp(self, x, t, dt, dx, duh=None):
        """Tangent of one step at x (x's derived ghosts are refreshed)."""
        self.bind_adjoint()
        self._stream()
        dy = torch.zeros_like(x)
        self._check(self.lib.cmhd_rk3_step_jvp(self.ctx, self._state(x), float(t), float(dt),
                                               self._state(dx), _ptr(self._plane2(duh)),
                                               self._state(dy)))
        return dy

    def rk3_step_vjp(self, x, t, dt, ybar, uhbar=None):
        """(d step/dx)^T ybar; (d step/du*)^T ybar is added into uhbar."""
        self.bind_adjoint()
        self._stream()
        xbar = torch.zeros_like(x)
        self._check(self.lib.cmhd_rk3_step_vjp(self.ctx, self._state(x), float(t), float(dt),
                                               self._state(ybar), self._state(xbar),
                                               _ptr(self._plane2(uhbar))))
        return xbar

    def bz_plane_vjp(self, z, bzbar, xbar):
        self._stream()
        self._check(self.lib.cmhd_bz_plane_vjp(self.ctx, float(z), _ptr(bzbar.contiguous()),
                                               self._state(xbar)))
        return xbar

    def profile(self, enable=True):
        self._check(self.lib.cmhd_profile_enable(self.ctx, 1 if enable else 0))

    def profile_read(self, which="substage"):
        """(total ms, launches) since the last read of the fused substage
        kernel ("substage") or of the boundary work before it ("ghosts")."""
        sel = {"substage": 0, "ghosts": 1}[which]
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int(0)
        self._check(self.lib.cmhd_profile_read(self.ctx, sel, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.cmhd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Granulation:
    """One granulation-driver object of the library (photospheric plane)."""

    FIELDS = ("r_gran", "r_lane", "r_excl", "t_gran", "v0", "vmin_frac", "life_var", "amp_var",
              "f_rot")

    def __init__(self, params: dict, device: str = "cuda", workspace: bool = True):
        """workspace=False: the granule bookkeeping only (update, granules),
        host work that runs without a GPU; velocity() then raises."""
        self.lib = load()
        self.device = torch.device(device)
        q = CmhdGranParams()
        q.nx, q.ny = int(params["nx"]), int(params["ny"])
        q.Lx, q.Ly = float(params["Lx"]), float(params["Ly"])
        for n in self.FIELDS:
            setattr(q, n, float(params[n]))
        self._q = q
        self.shape = (2, q.ny, q.nx)
        obj = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream if workspace else None
        rc = self.lib.cmhd_gran_create(ctypes.byref(q), ctypes.c_void_p(stream), ctypes.byref(obj))
        if rc != CMHD_OK:
            raise CmhdError(rc, "cmhd_gran_create: invalid parameters")
        self.obj = obj
        self.workspace = None
        if not workspace:
            return
        nbytes = self.lib.cmhd_gran_workspace_bytes(obj)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._check(self.lib.cmhd_gran_bind_workspace(obj, ctypes.c_void_p(base + (-base) % 256),
                                                      nbytes))

    def _check(self, rc):
        if rc != CMHD_OK:
            raise CmhdError(rc, self.lib.cmhd_gran_last_error(self.obj).decode())

    def update(self, t, unif, xi, vext=None):
        """Advance the population to t; returns the number of births (the
        draws consumed from the front of unif and, two each, of xi)."""
        dp = ctypes.POINTER(ctypes.c_double)
        u = np.ascontiguousarray(unif, dtype=np.float64)
        x = np.ascontiguousarray(xi, dtype=np.float64)
        n_pool = min(u.size, x.size // 2)
        v = None if vext is None else np.ascontiguousarray(vext, dtype=np.float64)
        if v is not None and v.shape != self.shape:
            raise ValueError(f"vext must have shape {self.shape}")
        births = ctypes.c_longlong(0)
        self._check(self.lib.cmhd_gran_update(
            self.obj, float(t), None if v is None else v.ctypes.data_as(dp), u.ctypes.data_as(dp),
            x.ctypes.data_as(dp), n_pool, ctypes.byref(births)))
        return births.value

    def velocity(self, t, out=None):
        """Driver snapshot at time t (runs on the stream current at creation)."""
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        if tuple(out.shape) != self.shape or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float64 tensor {self.shape}")
        self._check(self.lib.cmhd_gran_velocity(self.obj, float(t), _ptr(out)))
        return out

    def granules(self):
        """Living granules as rows (x, y, t0, T, v_max, t_max)."""
        n = ctypes.c_int(0)
        self._check(self.lib.cmhd_gran_list(self.obj, None, 0, ctypes.byref(n)))
        out = np.zeros((max(n.value, 1), 6))
        self._check(self.lib.cmhd_gran_list(
            self.obj, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n.value,
            ctypes.byref(n)))
        return out[:n.value]

    def close(self):
        if getattr(self, "obj", None):
            self.lib.cmhd_gran_destroy(self.obj)
            self.obj = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solver_for(workload, precision="fp64", device="cuda"):
    """Solver for a workloads.Workload, with its driver already set."""
    s = Solver(workload.grid, workload.params, workload.lnrho0_z, precision, device,
               lnT0_z=workload.lnT0_z)
    if workload.grid["zbc"] == "solar" and workload.uh_target is not None:
        s.set_driver(workload.uh_target, ah=workload.ah_target)
    return s
