"""ctypes binding of the hybrid-step C ABI (include/hk.h).

Argument marshalling only: every step of the method runs in the gfx950
kernels of libhk_f32.so / libhk_f64.so.  PyTorch supplies the HIP stream and,
through allocator callbacks, the device memory (its caching allocator).
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import lib_path

MAX_SPECIES = 6
MAX_LEVELS = 8
KIND = {"electron": 0, "ion": 1, "positron": 2, "photon": 3}
PROFILE = {"none": 0, "uniform": 1, "ramp": 2, "foil": 3}
SWITCH = {"all_pic": 0, "threshold": 1, "cnn": 2, "all_fluid": 3, "fixed": 4}
BC = {"periodic": 0, "open": 1}
COMP = {"ex": 0, "ey": 1, "ez": 2, "bx": 3, "by": 4, "bz": 5, "jx": 6, "jy": 7, "jz": 8}
NTIMERS = 12
TIMER_NAMES = ["switch_ms", "particles_ms", "fluid_ms", "conversion_ms", "fields_ms", "merge_ms",
               "push_kernel_ms", "rebins", "push_launches", "particles_pushed", "tiles_pushed",
               "unused"]
STATUS = {0: "HK_OK", -1: "HK_EINVAL", -2: "HK_ENOMEM", -3: "HK_EDEVICE", -4: "HK_ENUMERIC",
          -5: "HK_EOVERFLOW", -6: "HK_ESTATE", -7: "HK_EIO", -8: "HK_ENOTSUP"}


class HKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc_x", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double)]


class SpeciesDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ppc", C.c_int32), ("profile", C.c_int32),
                ("mobile", C.c_int32), ("fluid", C.c_int32), ("ionizable", C.c_int32),
                ("z_max", C.c_int32), ("target", C.c_int32), ("qed", C.c_int32),
                ("pad", C.c_int32), ("charge", C.c_double), ("mass", C.c_double),
                ("n0", C.c_double), ("x0", C.c_double), ("length", C.c_double),
                ("u_th", C.c_double), ("ip_ev", C.c_double * MAX_LEVELS), ("gamma_ad", C.c_double)]


class LaserDesc(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("polarization", C.c_int32), ("i_antenna", C.c_int32),
                ("pad", C.c_int32), ("a0", C.c_double), ("waist", C.c_double),
                ("duration", C.c_double), ("t_center", C.c_double), ("lambda_um", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class RunDesc(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("switch_mode", C.c_int32), ("switch_every", C.c_int32),
                ("dilation", C.c_int32), ("hysteresis", C.c_int32),
                ("enable_ionization", C.c_int32), ("enable_qed", C.c_int32),
                ("thr_a", C.c_double), ("thr_grad", C.c_double), ("thr_sigma_u", C.c_double),
                ("thr_ion", C.c_double), ("thr_chi", C.c_double), ("n_floor", C.c_double),
                ("spawn_frac", C.c_double), ("thr_hot", C.c_double), ("stream", C.c_void_p),
                ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_ctx", C.c_void_p)]


class Diag(C.Structure):
    _fields_ = [("t", C.c_double), ("step", C.c_int64), ("u_e", C.c_double), ("u_b", C.c_double),
                ("kin", C.c_double * MAX_SPECIES), ("fluid_kin", C.c_double * MAX_SPECIES),
                ("count", C.c_double * MAX_SPECIES), ("fluid_mass", C.c_double * MAX_SPECIES),
                ("charge_total", C.c_double), ("gauss_max", C.c_double), ("gauss_l2", C.c_double),
                ("conv_loss", C.c_double), ("ion_energy", C.c_double),
                ("photon_energy", C.c_double), ("kinetic_fraction", C.c_double),
                ("fallback_fraction", C.c_double), ("fluid_th", C.c_double * MAX_SPECIES)]


class Particles(C.Structure):
    _fields_ = [("n", C.c_size_t), ("x", C.c_void_p), ("u", C.c_void_p), ("w", C.c_void_p),
                ("id", C.c_void_p), ("z", C.c_void_p), ("tau", C.c_void_p)]


class CnnDesc(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", C.c_void_p)]


class CnnTrainDesc(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("weight_decay", C.c_double), ("lambda_e", C.c_double), ("dropout", C.c_int32),
                ("pad", C.c_int32)]


class SpTrainDesc(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("weight_decay", C.c_double), ("delta", C.c_double), ("lambda_e", C.c_double),
                ("dropout", C.c_int32), ("pad", C.c_int32)]


ABI_SYMBOLS = ["hk_create", "hk_destroy", "hk_step", "hk_switch_map", "hk_set_switch_map",
               "hk_set_switch_mode", "hk_diagnostics", "hk_get_field", "hk_set_field",
               "hk_get_rho", "hk_get_divE", "hk_particle_count", "hk_get_particles",
               "hk_set_particles", "hk_get_fluid", "hk_set_fluid", "hk_get_fluid_p", "hk_set_fluid_p", "hk_enable_timing",
               "hk_timers", "hk_qed_tables", "hk_cnn_nparams", "hk_cnn_create", "hk_cnn_destroy",
               "hk_cnn_set_params", "hk_cnn_get_params", "hk_cnn_set_norm", "hk_cnn_forward",
               "hk_cnn_loss_grad", "hk_cnn_train_step", "hk_cnn_last_error", "hk_cnn_forward_noalloc", "hk_set_cnn",
               "hk_dataset_create", "hk_dataset_destroy", "hk_dataset_size", "hk_dataset_get", "hk_dataset_stats",
               "hk_dump_training", "hk_train", "hk_dataset_predict", "hk_dataset_last_error", "hk_node_inputs", "hk_node_state",
               "hk_sp_nparams", "hk_sp_create", "hk_sp_destroy", "hk_sp_set_params", "hk_sp_get_params",
               "hk_sp_set_norm", "hk_sp_forward", "hk_sp_loss_grad", "hk_sp_train_step", "hk_sp_last_error",
               "hk_swn_nparams", "hk_swn_create", "hk_swn_destroy", "hk_swn_set_params", "hk_swn_get_params",
               "hk_swn_forward", "hk_swn_loss_grad", "hk_swn_train_step", "hk_swn_last_error",
               "hk_real_size", "hk_strerror", "hk_last_error", "hk_save", "hk_load"]

_libs: dict = {}


def load(prec: str = "f32"):
    """Load (once) the C-ABI library of the given precision ('f32' or 'f64')."""
    if prec in _libs:
        return _libs[prec]
    path = lib_path(prec)
    if not os.path.exists(path):
        raise RuntimeError("HIP library %s is not built (run __graft_entry__.build())" % path)
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so memory and streams from torch's allocator are valid in both
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    P = C.POINTER
    vp = C.c_void_p
    L.hk_create.argtypes = [P(GridDesc), P(SpeciesDesc), C.c_int, P(LaserDesc), P(RunDesc), P(vp)]
    L.hk_destroy.argtypes = [vp]
    L.hk_destroy.restype = None
    L.hk_step.argtypes = [vp, C.c_int]
    L.hk_save.argtypes = [vp, C.c_char_p]
    L.hk_load.argtypes = [vp, C.c_char_p]
    L.hk_switch_map.argtypes = [vp, vp, C.c_size_t]
    L.hk_set_switch_map.argtypes = [vp, vp, C.c_size_t]
    L.hk_set_switch_mode.argtypes = [vp, C.c_int]
    L.hk_diagnostics.argtypes = [vp, P(Diag)]
    L.hk_get_field.argtypes = [vp, C.c_int, vp, C.c_size_t]
    L.hk_set_field.argtypes = [vp, C.c_int, vp, C.c_size_t]
    L.hk_get_rho.argtypes = [vp, vp, C.c_size_t]
    L.hk_get_divE.argtypes = [vp, vp, C.c_size_t]
    L.hk_particle_count.argtypes = [vp, C.c_int, P(C.c_size_t)]
    L.hk_get_particles.argtypes = [vp, C.c_int, P(Particles)]
    L.hk_set_particles.argtypes = [vp, C.c_int, P(Particles)]
    L.hk_get_fluid.argtypes = [vp, C.c_int, vp, vp, C.c_size_t]
    L.hk_set_fluid.argtypes = [vp, C.c_int, vp, vp, C.c_size_t]
    L.hk_get_fluid_p.argtypes = [vp, C.c_int, vp, C.c_size_t]
    L.hk_set_fluid_p.argtypes = [vp, C.c_int, vp, C.c_size_t]
    L.hk_enable_timing.argtypes = [vp, C.c_int]
    L.hk_timers.argtypes = [vp, vp, C.c_int]
    L.hk_qed_tables.argtypes = [vp, vp, vp, vp]
    L.hk_cnn_nparams.restype = C.c_int
    L.hk_cnn_create.argtypes = [P(CnnDesc), P(vp)]
    L.hk_cnn_destroy.argtypes = [vp]
    L.hk_cnn_set_params.argtypes = [vp, vp, C.c_size_t]
    L.hk_cnn_get_params.argtypes = [vp, vp, C.c_size_t]
    L.hk_cnn_set_norm.argtypes = [vp, vp, vp]
    L.hk_cnn_forward.argtypes = [vp, vp] + [C.c_int] * 4 + [vp]
    L.hk_cnn_forward_noalloc.argtypes = [vp, vp] + [C.c_int] * 4 + [vp]
    L.hk_cnn_loss_grad.argtypes = [vp, vp, vp, vp] + [C.c_int] * 4 + [C.c_float, C.c_int, vp,
                                                                      P(C.c_double)]
    L.hk_cnn_train_step.argtypes = [vp, vp, vp, vp] + [C.c_int] * 4 + [P(CnnTrainDesc), P(C.c_double)]
    L.hk_cnn_last_error.restype = C.c_char_p
    L.hk_cnn_last_error.argtypes = [vp]
    L.hk_dataset_create.argtypes = [P(CnnDesc), P(vp)]
    L.hk_dataset_destroy.argtypes = [vp]
    L.hk_dataset_size.argtypes = [vp]
    L.hk_dataset_get.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, C.c_size_t]
    L.hk_dataset_stats.argtypes = [vp, vp, vp]
    L.hk_dump_training.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int]
    L.hk_train.argtypes = [vp, vp, C.c_int, C.c_int, P(CnnTrainDesc), C.c_uint64, vp]
    L.hk_dataset_predict.argtypes = [vp, vp, C.c_int, vp]
    L.hk_dataset_last_error.restype = C.c_char_p
    L.hk_dataset_last_error.argtypes = [vp]
    L.hk_set_cnn.argtypes = [vp, vp]
    L.hk_sp_nparams.restype = C.c_int
    L.hk_sp_create.argtypes = [P(CnnDesc), P(vp)]
    L.hk_sp_destroy.argtypes = [vp]
    L.hk_sp_destroy.restype = None
    L.hk_sp_set_params.argtypes = [vp, vp, C.c_size_t]
    L.hk_sp_get_params.argtypes = [vp, vp, C.c_size_t]
    L.hk_sp_set_norm.argtypes = [vp, vp, vp]
    L.hk_sp_forward.argtypes = [vp, vp] + [C.c_int] * 5 + [vp]
    L.hk_sp_loss_grad.argtypes = [vp, vp, vp] + [C.c_int] * 4 + [C.c_double, C.c_double, C.c_int, vp,
                                                                 P(C.c_double)]
    L.hk_sp_train_step.argtypes = [vp, vp, vp] + [C.c_int] * 4 + [P(SpTrainDesc), P(C.c_double)]
    L.hk_sp_last_error.restype = C.c_char_p
    L.hk_sp_last_error.argtypes = [vp]
    L.hk_swn_nparams.restype = C.c_int
    L.hk_swn_create.argtypes = [P(CnnDesc), P(vp)]
    L.hk_swn_destroy.argtypes = [vp]
    L.hk_swn_destroy.restype = None
    L.hk_swn_set_params.argtypes = [vp, vp, C.c_size_t]
    L.hk_swn_get_params.argtypes = [vp, vp, C.c_size_t]
    L.hk_swn_forward.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, vp]
    L.hk_swn_loss_grad.argtypes = [vp, vp, vp, vp, C.c_int, C.c_double, C.c_int, vp, P(C.c_double)]
    L.hk_swn_train_step.argtypes = [vp, vp, vp, vp, C.c_int, P(CnnTrainDesc), P(C.c_double)]
    L.hk_swn_last_error.restype = C.c_char_p
    L.hk_swn_last_error.argtypes = [vp]
    L.hk_node_inputs.argtypes = [vp, vp, vp, vp, C.c_size_t]
    L.hk_node_state.argtypes = [vp, vp, C.c_size_t]
    L.hk_real_size.restype = C.c_int
    L.hk_strerror.restype = C.c_char_p
    L.hk_strerror.argtypes = [C.c_int]
    L.hk_last_error.restype = C.c_char_p
    L.hk_last_error.argtypes = [vp]
    _libs[prec] = L
    return L


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def descriptors(cfg: dict):
    """Marshal a config dictionary (see configs.py) into the ABI descriptors."""
    g = cfg["grid"]
    grid = GridDesc(nx=g["nx"], ny=g["ny"], nz=g["nz"], bc_x=BC[g.get("bc_x", "open")],
                    dx=g["dx"], dy=g["dy"], dz=g["dz"], dt=g["dt"])
    sps = (SpeciesDesc * MAX_SPECIES)()
    for i, s in enumerate(cfg["species"]):
        sp = sps[i]
        sp.kind = KIND[s["kind"]]
        sp.ppc = s.get("ppc", 0)
        sp.profile = PROFILE[s.get("profile", "none")]
        sp.mobile = int(s.get("mobile", True))
        sp.fluid = int(s.get("fluid", False))
        sp.ionizable = int(s.get("ionizable", False))
        sp.z_max = s.get("z_max", 0)
        sp.target = s.get("target", 0)
        sp.qed = int(s.get("qed", False))
        sp.charge = s["charge"]
        sp.mass = s["mass"]
        sp.n0 = s.get("n0", 0.0)
        sp.x0 = s.get("x0", 0.0)
        sp.length = s.get("length", 1.0)
        sp.u_th = s.get("u_th", 0.0)
        sp.gamma_ad = s.get("gamma_ad", 0.0)
        for k, v in enumerate(s.get("ip_ev", [])):
            sp.ip_ev[k] = v
    las = cfg.get("laser", {})
    laser = LaserDesc(enabled=int(las.get("enabled", False)),
                      polarization=1 if las.get("polarization", "linear") == "circular" else 0,
                      i_antenna=las.get("i_antenna", 2), a0=las.get("a0", 0.0),
                      waist=las.get("waist", 1.0), duration=las.get("duration", 1.0),
                      t_center=las.get("t_center", 0.0), lambda_um=las.get("lambda_um", 0.8))
    r = cfg["run"]
    run = RunDesc(seed=r["seed"], switch_mode=SWITCH[r.get("switch_mode", "all_pic")],
                  switch_every=r.get("switch_every", 1), dilation=r.get("dilation", 1),
                  hysteresis=r.get("hysteresis", 2),
                  enable_ionization=int(r.get("enable_ionization", False)),
                  enable_qed=int(r.get("enable_qed", False)), thr_a=r.get("thr_a", 0.5),
                  thr_grad=r.get("thr_grad", 0.2), thr_sigma_u=r.get("thr_sigma_u", 0.05),
                  thr_ion=r.get("thr_ion", 1e-6), thr_chi=r.get("thr_chi", 1e-3),
                  n_floor=r.get("n_floor", 1e-10), spawn_frac=r.get("spawn_frac", 0.5),
                  thr_hot=r.get("thr_hot", 0.0))
    return grid, sps, len(cfg["species"]), laser, run


class _TorchMemory:
    """Device memory and stream from PyTorch's caching allocator."""

    def __init__(self):
        import torch
        self.torch = torch
        torch.cuda.init()   # the caching allocator needs an initialized context
        self.device = torch.cuda.current_device()
        self.stream = torch.cuda.current_stream()

        def _alloc(nbytes, ctx):
            # a ctypes callback that raises returns an undefined value to C:
            # every failure (out of memory above all) must come back as NULL
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream))
            except Exception:
                return 0

        def _free(ptr, ctx):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:      # interpreter shutdown: torch already torn down
                pass

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


class Sim:
    """One simulation context on the current GPU."""

    def __init__(self, cfg: dict, precision: str = "f32", torch_memory: bool = True):
        self.lib = load(precision)
        self.cfg = cfg
        self.precision = precision
        self.real = np.float32 if self.lib.hk_real_size() == 4 else np.float64
        grid, sps, ns, laser, run = descriptors(cfg)
        self._mem = None
        if torch_memory:
            self._mem = _TorchMemory()
            run.stream = self._mem.stream.cuda_stream
            run.alloc = self._mem.alloc
            run.free = self._mem.free
        self._keep = (grid, sps, laser, run)
        h = C.c_void_p()
        rc = self.lib.hk_create(C.byref(grid), sps, ns, C.byref(laser), C.byref(run), C.byref(h))
        if rc != 0:
            raise HKError(rc, self.lib.hk_strerror(rc).decode())
        self.h = h
        self.nx, self.ny, self.nz = grid.nx, grid.ny, grid.nz
        self.nspecies = ns

    # -- helpers
    def _check(self, rc):
        if rc != 0:
            raise HKError(rc, self.lib.hk_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.hk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx + 1)

    @property
    def nodes(self):
        return (self.nx + 1) * self.ny * self.nz

    # -- ABI calls
    def step(self, n: int = 1):
        self._check(self.lib.hk_step(self.h, n))

    def get_field(self, comp) -> np.ndarray:
        c = COMP[comp] if isinstance(comp, str) else comp
        out = np.empty(self.shape, self.real)
        self._check(self.lib.hk_get_field(self.h, c, _ptr(out), out.nbytes))
        return out

    def set_field(self, comp, arr):
        c = COMP[comp] if isinstance(comp, str) else comp
        a = np.ascontiguousarray(arr, self.real).reshape(self.shape)
        self._check(self.lib.hk_set_field(self.h, c, _ptr(a), a.nbytes))

    def count(self, sp: int) -> int:
        n = C.c_size_t()
        self._check(self.lib.hk_particle_count(self.h, sp, C.byref(n)))
        return n.value

    def get_particles(self, sp: int) -> dict:
        n = self.count(sp)
        x = np.empty((n, 3)); u = np.empty((n, 3)); w = np.empty(n)
        idv = np.empty(n, np.uint64); z = np.empty(n, np.int32); tau = np.empty(n)
        p = Particles(n=n, x=_ptr(x), u=_ptr(u), w=_ptr(w), id=_ptr(idv), z=_ptr(z), tau=_ptr(tau))
        self._check(self.lib.hk_get_particles(self.h, sp, C.byref(p)))
        return {"x": x, "u": u, "w": w, "id": idv, "z": z, "tau": tau}

    def set_particles(self, sp: int, x, u, w, ids=None, z=None, tau=None):
        x = np.ascontiguousarray(x, np.float64); u = np.ascontiguousarray(u, np.float64)
        w = np.ascontiguousarray(w, np.float64)
        n = len(w)
        ids = np.ascontiguousarray(ids if ids is not None else np.arange(n), np.uint64)
        z = None if z is None else np.ascontiguousarray(z, np.int32)
        tau = None if tau is None else np.ascontiguousarray(tau, np.float64)
        p = Particles(n=n, x=_ptr(x), u=_ptr(u), w=_ptr(w), id=_ptr(ids), z=_ptr(z), tau=_ptr(tau))
        self._check(self.lib.hk_set_particles(self.h, sp, C.byref(p)))

    def save(self, path: str):
        self._check(self.lib.hk_save(self.h, str(path).encode()))

    def load(self, path: str):
        self._check(self.lib.hk_load(self.h, str(path).encode()))

    def get_fluid(self, sp: int):
        n = np.empty(self.shape); u = np.empty(self.shape + (3,))
        self._check(self.lib.hk_get_fluid(self.h, sp, _ptr(n), _ptr(u), self.nodes))
        return n, u

    def set_fluid(self, sp: int, n, u):
        n = np.ascontiguousarray(n, np.float64).reshape(self.shape)
        u = np.ascontiguousarray(u, np.float64).reshape(self.shape + (3,))
        self._check(self.lib.hk_set_fluid(self.h, sp, _ptr(n), _ptr(u), self.nodes))

    def get_pressure(self, sp: int) -> np.ndarray:
        p = np.empty(self.shape)
        self._check(self.lib.hk_get_fluid_p(self.h, sp, _ptr(p), self.nodes))
        return p

    def set_pressure(self, sp: int, p):
        p = np.ascontiguousarray(p, np.float64).reshape(self.shape)
        self._check(self.lib.hk_set_fluid_p(self.h, sp, _ptr(p), self.nodes))

    def get_switch(self) -> np.ndarray:
        out = np.empty(self.shape, np.uint8)
        self._check(self.lib.hk_switch_map(self.h, _ptr(out), out.size))
        return out

    def set_switch(self, m):
        m = np.ascontiguousarray(m, np.uint8).reshape(self.shape)
        self._check(self.lib.hk_set_switch_map(self.h, _ptr(m), m.size))

    def set_switch_mode(self, mode: str):
        self._check(self.lib.hk_set_switch_mode(self.h, SWITCH[mode]))

    def diagnostics(self) -> dict:
        d = Diag()
        self._check(self.lib.hk_diagnostics(self.h, C.byref(d)))
        out = {}
        for name, _ in Diag._fields_:
            v = getattr(d, name)
            out[name] = list(v)[: self.nspecies] if hasattr(v, "__len__") else v
        return out

    def rho(self) -> np.ndarray:
        out = np.empty(self.shape)
        self._check(self.lib.hk_get_rho(self.h, _ptr(out), out.size))
        return out

    def divE(self) -> np.ndarray:
        out = np.empty(self.shape)
        self._check(self.lib.hk_get_divE(self.h, _ptr(out), out.size))
        return out

    def node_inputs(self):
        """(raw[n, 8], e[n], hot[n]) over the node grid [nz][ny][NX] (x fastest)."""
        g = self.cfg["grid"]
        nx = g["nx"] if g.get("bc_x", "open") == "periodic" else g["nx"] + 1
        n = nx * self.ny * self.nz
        raw = np.empty((n, 8)); e = np.empty(n); hot = np.empty(n, np.uint8)
        self._check(self.lib.hk_node_inputs(self.h, _ptr(raw), _ptr(e), _ptr(hot), n))
        return raw, e, hot

    def node_state(self, out=None):
        """States for the next-state surrogate: a torch float32 tensor
        [nz, ny, NX, 10] on the GPU (E, B, J averaged to the nodes, rho)."""
        import torch
        g = self.cfg["grid"]
        nx = g["nx"] if g.get("bc_x", "open") == "periodic" else g["nx"] + 1
        if out is None:
            out = torch.empty((self.nz, self.ny, nx, 10), device="cuda", dtype=torch.float32)
        assert out.is_contiguous() and out.dtype == torch.float32 and out.numel() == nx * self.ny * self.nz * 10
        self._check(self.lib.hk_node_state(self.h, out.data_ptr(), nx * self.ny * self.nz))
        return out

    def set_cnn(self, cnn):
        """Use `cnn` (a CNN, kept alive by this object) in switch mode "cnn"; None detaches."""
        self._cnn = cnn
        self._check(self.lib.hk_set_cnn(self.h, cnn.h if cnn is not None else None))

    def enable_timing(self, on=True):
        self._check(self.lib.hk_enable_timing(self.h, int(on)))

    def timers(self) -> dict:
        out = np.zeros(NTIMERS)
        self._check(self.lib.hk_timers(self.h, _ptr(out), NTIMERS))
        return dict(zip(TIMER_NAMES, out.tolist()))


def qed_tables(precision: str = "f32"):
    """(W_e[256], W_b[256], X_e[256, 128], X_b[256, 128]) as the library built them."""
    L = load(precision)
    We = np.empty(256); Wb = np.empty(256)
    Xe = np.empty((256, 128)); Xb = np.empty((256, 128))
    rc = L.hk_qed_tables(_ptr(We), _ptr(Wb), _ptr(Xe), _ptr(Xb))
    if rc:
        raise HKError(rc, "hk_qed_tables failed")
    return We, Wb, Xe, Xb


class CNN:
    """The switch network on the GPU (device memory from torch's allocator).
    Crops are torch tensors on cuda:0: x [B, D, H, W, 8] float32 (normalized),
    y and e [B, D-8, H-8, W-8] float32."""

    def __init__(self, seed: int = 0, precision: str = "f32"):
        import torch
        self.lib = load(precision)
        self._mem = _TorchMemory()
        d = CnnDesc(seed=seed, stream=self._mem.stream.cuda_stream, alloc=self._mem.alloc,
                    free=self._mem.free, alloc_ctx=None)
        h = C.c_void_p()
        rc = self.lib.hk_cnn_create(C.byref(d), C.byref(h))
        if rc:
            raise HKError(rc, "hk_cnn_create failed")
        self.h = h
        self.nparams = self.lib.hk_cnn_nparams()

    def _check(self, rc):
        if rc:
            raise HKError(rc, self.lib.hk_cnn_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.hk_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        a = np.ascontiguousarray(p, np.float32)
        assert a.size == self.nparams
        self._check(self.lib.hk_cnn_set_params(self.h, _ptr(a), a.size))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.nparams, np.float32)
        self._check(self.lib.hk_cnn_get_params(self.h, _ptr(a), a.size))
        return a

    def set_norm(self, mean, std):
        m = np.ascontiguousarray(mean, np.float32); s = np.ascontiguousarray(std, np.float32)
        self._check(self.lib.hk_cnn_set_norm(self.h, _ptr(m), _ptr(s)))

    def forward(self, x):
        import torch
        x = x.contiguous()
        B, D, H, W, _ = x.shape
        out = torch.empty((B, D - 8, H - 8, W - 8), device=x.device, dtype=torch.float32)
        self._check(self.lib.hk_cnn_forward(self.h, x.data_ptr(), B, D, H, W, out.data_ptr()))
        return out

    def forward_noalloc(self, x, out=None):
        """hk_cnn_forward_noalloc: the same logits from the library's static
        scratch array; only enqueued on the network's stream."""
        x = x.contiguous()
        B, D, H, W, _ = x.shape
        if out is None:
            import torch
            out = torch.empty((B, D - 8, H - 8, W - 8), device=x.device, dtype=torch.float32)
        self._check(self.lib.hk_cnn_forward_noalloc(self.h, x.data_ptr(), B, D, H, W, out.data_ptr()))
        return out

    def loss_grad(self, x, y, e, lam=0.1, mask_step=-1):
        x = x.contiguous(); y = y.contiguous(); e = e.contiguous()
        B, D, H, W, _ = x.shape
        g = np.empty(self.nparams, np.float32)
        loss = C.c_double()
        self._check(self.lib.hk_cnn_loss_grad(self.h, x.data_ptr(), y.data_ptr(), e.data_ptr(), B, D, H, W,
                                              float(lam), int(mask_step), _ptr(g), C.byref(loss)))
        return loss.value, g

    def train_step(self, x, y, e, lr=1e-3, lam=0.1, dropout=True, weight_decay=0.01):
        x = x.contiguous(); y = y.contiguous(); e = e.contiguous()
        B, D, H, W, _ = x.shape
        t = CnnTrainDesc(lr=lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=weight_decay,
                         lambda_e=lam, dropout=int(dropout))
        loss = C.c_double()
        self._check(self.lib.hk_cnn_train_step(self.h, x.data_ptr(), y.data_ptr(), e.data_ptr(), B, D, H,
                                               W, C.byref(t), C.byref(loss)))
        return loss.value


class Dataset:
    """Training set of the learned switch in device memory (hk_dataset_*):
    snapshots of all-PIC runs with their labels, filled by hk_dump_training
    and sampled on the device by hk_train."""

    def __init__(self, precision: str = "f32"):
        self.lib = load(precision)
        self._mem = _TorchMemory()
        d = CnnDesc(seed=0, stream=self._mem.stream.cuda_stream, alloc=self._mem.alloc,
                    free=self._mem.free, alloc_ctx=None)
        h = C.c_void_p()
        rc = self.lib.hk_dataset_create(C.byref(d), C.byref(h))
        if rc:
            raise HKError(rc, "hk_dataset_create failed")
        self.h = h

    def _check(self, rc):
        if rc:
            raise HKError(rc, self.lib.hk_dataset_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.hk_dataset_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return self.lib.hk_dataset_size(self.h)

    def dump(self, sim, steps: int, every: int, window: int = 10):
        """Append snapshots of the all-PIC simulation `sim` (hk_dump_training)."""
        if sim.lib is not self.lib:
            raise ValueError("the simulation and the training set come from different precisions")
        rc = self.lib.hk_dump_training(sim.h, self.h, int(steps), int(every), int(window))
        if rc:
            raise HKError(rc, self.lib.hk_last_error(sim.h).decode())

    def dims(self, k: int):
        d = np.zeros(3, np.int32)
        self._check(self.lib.hk_dataset_get(self.h, k, _ptr(d), None, None, None, None, 0))
        return tuple(int(v) for v in d)

    def get(self, k: int):
        """(raw [D, H, W, 8], ehat [D, H, W], y [D, H, W], thr [D, H, W]) of
        snapshot k: inputs, conversion energy, label, threshold flags."""
        dims = self.dims(k)
        n = int(np.prod(dims))
        raw = np.empty(dims + (8,), np.float32); e = np.empty(dims, np.float32)
        y = np.empty(dims, np.uint8); thr = np.empty(dims, np.uint8)
        self._check(self.lib.hk_dataset_get(self.h, k, None, _ptr(raw), _ptr(e), _ptr(y), _ptr(thr), n))
        return raw, e, y, thr

    def stats(self):
        m = np.empty(8, np.float32); s = np.empty(8, np.float32)
        self._check(self.lib.hk_dataset_stats(self.h, _ptr(m), _ptr(s)))
        return m, s

    def train(self, cnn, iters: int, B: int = 64, lr=1e-3, lam=0.1, seed=0, dropout=True, weight_decay=0.01):
        """hk_train: iters AdamW steps on device-sampled crops; the batch losses."""
        t = CnnTrainDesc(lr=lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=weight_decay,
                         lambda_e=lam, dropout=int(dropout))
        losses = np.zeros(max(int(iters), 1))
        self._check(self.lib.hk_train(cnn.h, self.h, int(iters), int(B), C.byref(t), int(seed), _ptr(losses)))
        return losses[:iters]

    def predict(self, cnn, k: int):
        """Logits (torch, device, [D, H, W]) of snapshot k, no dropout."""
        import torch
        out = torch.empty(self.dims(k), device="cuda", dtype=torch.float32)
        self._check(self.lib.hk_dataset_predict(cnn.h, self.h, int(k), out.data_ptr()))
        return out


class StatePredictor:
    """The next-state surrogate on the GPU (device memory from torch's
    allocator).  Patches are torch tensors on cuda:0: x and y [B, D, H, W, 10]
    float32, normalized."""

    def __init__(self, seed: int = 0, precision: str = "f32"):
        self.lib = load(precision)
        self._mem = _TorchMemory()
        d = CnnDesc(seed=seed, stream=self._mem.stream.cuda_stream, alloc=self._mem.alloc,
                    free=self._mem.free, alloc_ctx=None)
        h = C.c_void_p()
        rc = self.lib.hk_sp_create(C.byref(d), C.byref(h))
        if rc:
            raise HKError(rc, "hk_sp_create failed")
        self.h = h
        self.nparams = self.lib.hk_sp_nparams()

    @property
    def stream(self):
        return self._mem.stream

    def _check(self, rc):
        if rc:
            raise HKError(rc, self.lib.hk_sp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.hk_sp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        a = np.ascontiguousarray(p, np.float32)
        assert a.size == self.nparams
        self._check(self.lib.hk_sp_set_params(self.h, _ptr(a), a.size))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.nparams, np.float32)
        self._check(self.lib.hk_sp_get_params(self.h, _ptr(a), a.size))
        return a

    def set_norm(self, mean, std):
        m = np.ascontiguousarray(mean, np.float32); s = np.ascontiguousarray(std, np.float32)
        assert m.size == 10 and s.size == 10
        self._check(self.lib.hk_sp_set_norm(self.h, _ptr(m), _ptr(s)))

    def forward(self, x, mask_step=-1, out=None):
        import torch
        x = x.contiguous()
        B, D, H, W, C_ = x.shape
        assert C_ == 10 and x.dtype == torch.float32
        if out is None:
            out = torch.empty_like(x)
        self._check(self.lib.hk_sp_forward(self.h, x.data_ptr(), B, D, H, W, int(mask_step), out.data_ptr()))
        return out

    def loss_grad(self, x, y, delta=0.01, lam=0.1, mask_step=-1, grad=True):
        x = x.contiguous(); y = y.contiguous()
        B, D, H, W, _ = x.shape
        assert y.shape == x.shape
        g = np.empty(self.nparams, np.float32) if grad else None
        loss = C.c_double()
        self._check(self.lib.hk_sp_loss_grad(self.h, x.data_ptr(), y.data_ptr(), B, D, H, W, float(delta),
                                             float(lam), int(mask_step), None if g is None else _ptr(g),
                                             C.byref(loss)))
        return loss.value, g

    def train_step(self, x, y, lr=1e-3, delta=0.01, lam=0.1, dropout=True, weight_decay=0.01):
        x = x.contiguous(); y = y.contiguous()
        B, D, H, W, _ = x.shape
        t = SpTrainDesc(lr=lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=weight_decay, delta=delta,
                        lambda_e=lam, dropout=int(dropout))
        loss = C.c_double()
        self._check(self.lib.hk_sp_train_step(self.h, x.data_ptr(), y.data_ptr(), B, D, H, W, C.byref(t),
                                              C.byref(loss)))
        return loss.value


class SwitchNet:
    """The paper's per-node switch classifier on the GPU (device memory from
    torch's allocator).  x: torch [n, 10] float32 on cuda:0 (normalized node
    features); y, e: [n] float32."""

    def __init__(self, seed: int = 0, precision: str = "f32"):
        self.lib = load(precision)
        self._mem = _TorchMemory()
        d = CnnDesc(seed=seed, stream=self._mem.stream.cuda_stream, alloc=self._mem.alloc,
                    free=self._mem.free, alloc_ctx=None)
        h = C.c_void_p()
        rc = self.lib.hk_swn_create(C.byref(d), C.byref(h))
        if rc:
            raise HKError(rc, "hk_swn_create failed")
        self.h = h
        self.nparams = self.lib.hk_swn_nparams()

    def _check(self, rc):
        if rc:
            raise HKError(rc, self.lib.hk_swn_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.hk_swn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        a = np.ascontiguousarray(p, np.float32)
        assert a.size == self.nparams
        self._check(self.lib.hk_swn_set_params(self.h, _ptr(a), a.size))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.nparams, np.float32)
        self._check(self.lib.hk_swn_get_params(self.h, _ptr(a), a.size))
        return a

    def forward(self, x, mask_step=-1, sample=0, out=None):
        import torch
        x = x.contiguous()
        n, c_ = x.shape
        assert c_ == 10 and x.dtype == torch.float32
        if out is None:
            out = torch.empty(n, device=x.device, dtype=torch.float32)
        self._check(self.lib.hk_swn_forward(self.h, x.data_ptr(), n, int(mask_step), int(sample), out.data_ptr()))
        return out

    def loss_grad(self, x, y, e, lam=0.1, mask_step=-1, grad=True):
        x = x.contiguous(); y = y.contiguous(); e = e.contiguous()
        g = np.empty(self.nparams, np.float32) if grad else None
        loss = C.c_double()
        self._check(self.lib.hk_swn_loss_grad(self.h, x.data_ptr(), y.data_ptr(), e.data_ptr(), x.shape[0],
                                              float(lam), int(mask_step), None if g is None else _ptr(g),
                                              C.byref(loss)))
        return loss.value, g

    def train_step(self, x, y, e, lr=1e-3, lam=0.1, dropout=True, weight_decay=0.01):
        x = x.contiguous(); y = y.contiguous(); e = e.contiguous()
        t = CnnTrainDesc(lr=lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=weight_decay,
                         lambda_e=lam, dropout=int(dropout))
        loss = C.c_double()
        self._check(self.lib.hk_swn_train_step(self.h, x.data_ptr(), y.data_ptr(), e.data_ptr(), x.shape[0],
                                               C.byref(t), C.byref(loss)))
        return loss.value
