"""Python binding of libhp2sph (HP2SPH spherical-harmonic analysis on MI355X).

Argument marshalling only: every stage runs in the HIP kernels of
libhp2sph.so (built in-tree by paper_1904_10514_amd.build).  PyTorch supplies
device memory and the current stream.  There is no CPU fallback: importing
this package fails if the library has not been built, and every call that
needs a GPU fails if none is visible.

    plan = Plan(nside=1024, lmax=2048, batch=64, mode="f32_refine")
    alm = plan.analyze(maps)            # (sum of alm sizes,) complex128
    cl = plan.power_spectrum(alm)       # (sum of lmax+1,) float64
    maps2 = plan.synthesize(alm)        # (sum of npix,) float64

Conventions (see include/hp2sph.h): maps are float64 in HEALPix RING order,
maps of a batch back to back; a_lm are complex128 packed m-major for m >= 0,
index m (2 lmax + 1 - m)/2 + l, maps back to back.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhp2sph.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libhp2sph.so is not built; run `python paper_1904_10514_amd/build.py` "
        "(hipcc, gfx950) before importing paper_1904_10514_amd")

# PyTorch ships its own HIP runtime (libamdhip64.so.7, the soname of the
# system one the library links against).  Whichever is loaded first serves the
# whole process, and the library must share the runtime instance that owns the
# tensors and streams it is given: so torch, and with it its runtime, is
# loaded before the library.
try:
    import torch as _torch_rt   # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIB_PATH)

HP2SPH_F64, HP2SPH_F32_REFINE, HP2SPH_F32, HP2SPH_EQUAL_WEIGHT = 0, 1, 2, 3
MODES = {"f64": HP2SPH_F64, "f32_refine": HP2SPH_F32_REFINE, "f32": HP2SPH_F32,
         "equal_weight": HP2SPH_EQUAL_WEIGHT}
MAX_JACOBI = 1000
ERRORS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EWORKSPACE", -5: "ESTATE"}
TABLE_RINGS, TABLE_POLE, TABLE_ANALYSIS, TABLE_SYNTHESIS, TABLE_GIVENS = 0, 1, 2, 3, 4
MAX_NSIDE = 2048

EXPORTED = [
    "hp2sph_plan_create", "hp2sph_workspace_size", "hp2sph_analyze", "hp2sph_synthesize",
    "hp2sph_power_spectrum", "hp2sph_plan_destroy", "hp2sph_last_error", "hp2sph_host_table",
    "hp2sph_profile", "hp2sph_profile_read", "hp2sph_plan_create_ex", "hp2sph_plan_strategy",
    "hp2sph_analyze_iterative", "hp2sph_set_schedule", "hp2sph_autotune", "hp2sph_schedules",
    "hp2sph_schedule_map", "hp2sph_gemm_check", "hp2sph_analyze_noalloc", "hp2sph_set_option",
    "hp2sph_get_option",
]
STRATEGIES = {"auto": 0, "staged": 1, "tables": 2}
SCHEDULES = ["xcd_round_robin", "xcd_balanced", "linear", "linear_rows"]
OPTIONS = ["fold_grid", "pack_maps", "ring_order", "ring_threads"]
MAX_TUNE_REPS = 100
NSTAGES = 13
STAGES = ["ring_forward", "pole", "gemm_analysis", "sweep_analysis", "pack", "unpack",
          "sweep_synthesis", "gemm_synthesis", "ring_inverse", "cl", "residual_fold",
          "ring_adjoint", "gemm_adjoint"]

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_lib.hp2sph_plan_create.argtypes = [ctypes.POINTER(_i32), ctypes.POINTER(_i32), _i32, _i32, ctypes.POINTER(_vp)]
_lib.hp2sph_workspace_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
_sz = ctypes.c_size_t
_lib.hp2sph_analyze.argtypes = [_vp, _vp, _vp, _vp, _sz, _vp]
_lib.hp2sph_synthesize.argtypes = [_vp, _vp, _vp, _vp, _sz, _vp]
_lib.hp2sph_analyze_iterative.argtypes = [_vp, _vp, _vp, _i32, _vp, _sz, _vp]
_lib.hp2sph_power_spectrum.argtypes = [_vp, _vp, _vp, _vp]
_lib.hp2sph_plan_destroy.argtypes = [_vp]
_lib.hp2sph_last_error.restype = ctypes.c_char_p
_lib.hp2sph_plan_create_ex.argtypes = [ctypes.POINTER(_i32), ctypes.POINTER(_i32), _i32, _i32, _i32,
                                        ctypes.POINTER(_vp)]
_lib.hp2sph_plan_strategy.argtypes = [_vp, ctypes.POINTER(_i32)]
_lib.hp2sph_profile.argtypes = [_vp, _i32]
_lib.hp2sph_profile_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32), _i32]
_lib.hp2sph_set_schedule.argtypes = [_vp, _i32]
_lib.hp2sph_autotune.argtypes = [_vp, _vp, _vp, _vp, _sz, _vp, _i32, ctypes.POINTER(ctypes.c_double)]
_lib.hp2sph_schedules.argtypes = [_vp, ctypes.POINTER(_i32), _i32, ctypes.POINTER(_i32)]
_lib.hp2sph_schedule_map.argtypes = [_i32, _vp, _vp, _vp, _i32, _vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
_lib.hp2sph_host_table.argtypes = [_i32, _i32, _i32, _vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
_lib.hp2sph_gemm_check.argtypes = [_i32, _i32, _i32, _i32] + [ctypes.POINTER(ctypes.c_int64)] * 3
_lib.hp2sph_analyze_noalloc.argtypes = [_vp, _vp, _vp, _vp]
_lib.hp2sph_set_option.argtypes = [_vp, _i32, _i32]
_lib.hp2sph_get_option.argtypes = [_vp, _i32, ctypes.POINTER(_i32)]
NOALLOC_WORKSPACE = 256 << 20
for _f in EXPORTED:
    if _f not in ("hp2sph_last_error",):
        getattr(_lib, _f).restype = ctypes.c_int


class HP2SPHError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = _lib.hp2sph_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {msg}")


def _check(code, where):
    if code != 0:
        raise HP2SPHError(code, where)


def lib():
    """The loaded ctypes library (for tests of the raw C ABI)."""
    return _lib


def npix(nside):
    return 12 * int(nside) * int(nside)


def alm_size(lmax):
    return (int(lmax) + 1) * (int(lmax) + 2) // 2


def host_table(nside, table, block=0):
    """A set-up table computed on the host (no GPU), as float64 numpy."""
    cnt = ctypes.c_int64(0)
    _check(_lib.hp2sph_host_table(int(nside), int(table), int(block), None, 0, ctypes.byref(cnt)), "host_table")
    out = np.empty(cnt.value, dtype=np.float64)
    _check(_lib.hp2sph_host_table(int(nside), int(table), int(block), out.ctypes.data, cnt.value,
                                  ctypes.byref(cnt)), "host_table")
    return out


def schedule_map(sched, M, N, K):
    """Host-only: the workgroup -> (problem, tile) map of schedule `sched` (a
    name of SCHEDULES) for GEMM problems of sizes M x N, extent K, in launch
    order, as an (workgroups, 2) int32 array ((-1, -1): no tile)."""
    M, N, K = (np.ascontiguousarray(x, dtype=np.int32) for x in (M, N, K))
    if not (len(M) == len(N) == len(K)):
        raise ValueError("M, N, K must have the same length")
    cnt = ctypes.c_int64(0)
    sid = SCHEDULES.index(sched)
    _check(_lib.hp2sph_schedule_map(sid, M.ctypes.data, N.ctypes.data, K.ctypes.data, len(M), None, 0,
                                    ctypes.byref(cnt)), "schedule_map")
    out = np.empty(cnt.value, dtype=np.int32)
    _check(_lib.hp2sph_schedule_map(sid, M.ctypes.data, N.ctypes.data, K.ctypes.data, len(M), out.ctypes.data,
                                    cnt.value, ctypes.byref(cnt)), "schedule_map")
    return out.reshape(-1, 2)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: libhp2sph runs on MI355X only (no CPU fallback)")
    return torch


def _check_tensor(t, name, dtype, numel, device):
    """The C ABI takes raw pointers, so every buffer is checked here before a
    call: its dtype, element count, contiguity and device (the plan's)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda or t.device != device:
        raise ValueError(f"{name} must live on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, the plan expects {numel}")


class Plan:
    """A plan for a batch of maps (uniform or uneven nside)."""

    def __init__(self, nside, lmax=None, batch=None, mode="f64", strategy="auto"):
        torch = _torch()
        if np.isscalar(nside):
            if batch is None:
                batch = 1
            nside = [int(nside)] * int(batch)
        nside = [int(v) for v in nside]
        batch = len(nside)
        if lmax is None:
            lmax = [2 * v for v in nside]
        elif np.isscalar(lmax):
            lmax = [int(lmax)] * batch
        lmax = [int(v) for v in lmax]
        if len(lmax) != batch:
            raise ValueError("lmax must match nside")
        self.nside, self.lmax, self.batch = nside, lmax, batch
        self.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        arr_n = (_i32 * batch)(*nside)
        arr_l = (_i32 * batch)(*lmax)
        h = _vp()
        strat = STRATEGIES[strategy] if isinstance(strategy, str) else int(strategy)
        _check(_lib.hp2sph_plan_create_ex(arr_n, arr_l, batch, self.mode, strat, ctypes.byref(h)), "plan_create")
        self._h = h
        s = _i32(0)
        _check(_lib.hp2sph_plan_strategy(self._h, ctypes.byref(s)), "plan_strategy")
        self.strategy = {v: k for k, v in STRATEGIES.items()}[s.value]
        ws = ctypes.c_size_t(0)
        _check(_lib.hp2sph_workspace_size(self._h, ctypes.byref(ws)), "workspace_size")
        self.workspace_bytes = ws.value
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._ws = torch.empty(max(ws.value, 1) + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.npix_total = sum(npix(v) for v in nside)
        self.alm_total = sum(alm_size(v) for v in lmax)
        self.cl_total = sum(v + 1 for v in lmax)
        self.map_offsets = np.concatenate([[0], np.cumsum([npix(v) for v in nside])])
        self.alm_offsets = np.concatenate([[0], np.cumsum([alm_size(v) for v in lmax])])
        self.cl_offsets = np.concatenate([[0], np.cumsum([v + 1 for v in lmax])])

    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _maps(self, maps):
        import torch
        _check_tensor(maps, "maps", torch.float64, self.npix_total, self.device)

    def _alm(self, alm, name="alm"):
        import torch
        _check_tensor(alm, name, torch.complex128, self.alm_total, self.device)

    def _alm_out(self, out):
        import torch
        if out is None:
            return torch.empty(self.alm_total, dtype=torch.complex128, device=self.device)
        self._alm(out, "out")
        return out

    def analyze(self, maps, out=None):
        _torch()
        self._maps(maps)
        out = self._alm_out(out)
        _check(_lib.hp2sph_analyze(self._h, maps.data_ptr(), out.data_ptr(), self._ws_ptr, self.workspace_bytes,
                                   self._stream()), "analyze")
        return out

    def analyze_noalloc(self, maps, out):
        """hp2sph_analyze_noalloc: the analysis with the library's static device
        workspace (no workspace argument, nothing allocated); `out` must be
        given.  Calls that overlap in time on one device race on that workspace."""
        _torch()
        self._maps(maps)
        self._alm(out, "out")
        _check(_lib.hp2sph_analyze_noalloc(self._h, maps.data_ptr(), out.data_ptr(), self._stream()),
               "analyze_noalloc")
        return out

    def analyze_iterative(self, maps, niter, out=None):
        """Equal-weight analysis with `niter` Jacobi iterations (mode="equal_weight")."""
        _torch()
        self._maps(maps)
        out = self._alm_out(out)
        _check(_lib.hp2sph_analyze_iterative(self._h, maps.data_ptr(), out.data_ptr(), int(niter), self._ws_ptr,
                                             self.workspace_bytes, self._stream()), "analyze_iterative")
        return out

    def synthesize(self, alm, out=None):
        torch = _torch()
        self._alm(alm)
        if out is None:
            out = torch.empty(self.npix_total, dtype=torch.float64, device=self.device)
        else:
            _check_tensor(out, "out", torch.float64, self.npix_total, self.device)
        _check(_lib.hp2sph_synthesize(self._h, alm.data_ptr(), out.data_ptr(), self._ws_ptr, self.workspace_bytes,
                                      self._stream()), "synthesize")
        return out

    def power_spectrum(self, alm, out=None):
        torch = _torch()
        self._alm(alm)
        if out is None:
            out = torch.empty(self.cl_total, dtype=torch.float64, device=self.device)
        else:
            _check_tensor(out, "out", torch.float64, self.cl_total, self.device)
        _check(_lib.hp2sph_power_spectrum(self._h, alm.data_ptr(), out.data_ptr(), self._stream()),
               "power_spectrum")
        return out

    def set_schedule(self, name):
        """Workgroup schedule (one of SCHEDULES) for every GEMM of the plan."""
        if name not in SCHEDULES:
            raise ValueError(f"schedule must be one of {SCHEDULES}")
        _check(_lib.hp2sph_set_schedule(self._h, SCHEDULES.index(name)), "set_schedule")

    def autotune(self, maps, reps=3, out=None):
        """Time the analysis of `maps` under each candidate GEMM schedule and
        launch option and keep the fastest (synchronous).  Returns (ms per
        analysis, alm)."""
        _torch()
        self._maps(maps)
        out = self._alm_out(out)
        ms = ctypes.c_double(0.0)
        _check(_lib.hp2sph_autotune(self._h, maps.data_ptr(), out.data_ptr(), self._ws_ptr, self.workspace_bytes,
                                    self._stream(), int(reps), ctypes.byref(ms)), "autotune")
        return ms.value, out

    @property
    def schedules(self):
        """Schedule names of the GEMMs analyze launches, in launch order."""
        n = _i32(0)
        _check(_lib.hp2sph_schedules(self._h, None, 0, ctypes.byref(n)), "schedules")
        buf = (_i32 * max(n.value, 1))()
        _check(_lib.hp2sph_schedules(self._h, buf, n.value, ctypes.byref(n)), "schedules")
        return [SCHEDULES[buf[i]] for i in range(n.value)]

    def set_option(self, name, value):
        """Launch option of a work-list stage (one of OPTIONS): 'fold_grid'
        (0, or a persistent grid of that many workgroups), 'pack_maps' (maps
        per pack tile: 16, 32 or 64), 'ring_order' (item order of the ring
        transform: 0, 1 or 2) or 'ring_threads' (workgroup size of the ring
        transform up to nside 1024: 256 or 512)."""
        if name not in OPTIONS:
            raise ValueError(f"option must be one of {OPTIONS}")
        _check(_lib.hp2sph_set_option(self._h, OPTIONS.index(name), int(value)), "set_option")

    def option(self, name):
        """Value of a launch option in use."""
        if name not in OPTIONS:
            raise ValueError(f"option must be one of {OPTIONS}")
        v = _i32(0)
        _check(_lib.hp2sph_get_option(self._h, OPTIONS.index(name), ctypes.byref(v)), "get_option")
        return v.value

    def profile(self, enable):
        """Start (True, clears the accumulators) or stop per-stage event timing."""
        _check(_lib.hp2sph_profile(self._h, 1 if enable else 0), "profile")

    def profile_read(self):
        """{stage: (total ms, launches)} accumulated since profile(True)."""
        ms = (ctypes.c_double * NSTAGES)()
        n = (_i32 * NSTAGES)()
        _check(_lib.hp2sph_profile_read(self._h, ms, n, NSTAGES), "profile_read")
        return {STAGES[i]: (ms[i], n[i]) for i in range(NSTAGES)}

    def close(self):
        if getattr(self, "_h", None):
            _lib.hp2sph_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
