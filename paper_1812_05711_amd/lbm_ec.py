"""Python binding of the C ABI in include/lbm_ec.h (ctypes).

Argument marshalling only: every step of the time loop runs in the HIP
library.  PyTorch supplies the device workspace and the stream.  If the
native library is missing, every call raises; there is no fallback.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_ec.so")

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, EBUSY = 0, 1, 2, 3, 4, 5
FP64, FP32_DEV, FP32_DEV_F64MATH = 0, 1, 2
INIT_NOISE, INIT_EQ29, INIT_REST = 0, 1, 2
Y_TRIDIAGONAL, Y_SPECTRAL = 0, 1
RATES_ANTISYMMETRIC, RATES_SYMMETRIC = 0, 1
# columns of a batch history row: step, rms u_y, max |u|, sum of rho_c,
# amplitude of the first x mode of u_y (lattice units), unhealthy nodes,
# collector current (lattice units)
HIST_COLS = 7
HIST_CURRENT = 6

_PRECISION = {"fp64": FP64, "fp32": FP32_DEV, "fp32_dev": FP32_DEV, "fp32_f64math": FP32_DEV_F64MATH}
_INIT = {"noise": INIT_NOISE, "eq29": INIT_EQ29, "rest": INIT_REST}
_RATES = {"antisymmetric": RATES_ANTISYMMETRIC, "symmetric": RATES_SYMMETRIC}


class LbmEcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm_ec error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("T", ctypes.c_double),
        ("C", ctypes.c_double),
        ("M", ctypes.c_double),
        ("Fe", ctypes.c_double),
        ("tau_plus", ctypes.c_double),
        ("Lambda", ctypes.c_double),
        ("Lambda_g", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("init_mode", ctypes.c_int32),
        ("noise_amp", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("instance_id", ctypes.c_int32),
        ("charge_rates", ctypes.c_int32),
        ("body_force_x", ctypes.c_double),
    ]


_lib = None


def lib():
    """The loaded native library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"native library {LIB_PATH} is missing; build it with "
                           "python -m paper_1812_05711_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Params)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.lbm_ec_params_default.argtypes = [P]
    L.lbm_ec_params_default.restype = ctypes.c_int
    L.lbm_ec_validate.argtypes = [P]
    L.lbm_ec_validate.restype = ctypes.c_int
    L.lbm_ec_workspace_bytes.argtypes = [P]
    L.lbm_ec_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_ec_create.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.lbm_ec_create.restype = ctypes.c_int
    L.lbm_ec_step.argtypes = [vp, ctypes.c_int64]
    L.lbm_ec_step.restype = ctypes.c_int
    L.lbm_ec_steps_done.argtypes = [vp]
    L.lbm_ec_steps_done.restype = ctypes.c_int64
    L.lbm_ec_fields.argtypes = [vp, vp, vp, vp, vp, vp]
    L.lbm_ec_fields.restype = ctypes.c_int
    L.lbm_ec_fields_rho_m1.argtypes = [vp, vp]
    L.lbm_ec_fields_rho_m1.restype = ctypes.c_int
    L.lbm_ec_poisson.argtypes = [vp, vp, vp]
    L.lbm_ec_poisson.restype = ctypes.c_int
    L.lbm_ec_poisson_static.argtypes = [P, vp, vp, vp]
    L.lbm_ec_poisson_static.restype = ctypes.c_int
    L.lbm_ec_poisson_static_bytes.argtypes = [P]
    L.lbm_ec_poisson_static_bytes.restype = ctypes.c_size_t
    L.lbm_ec_stats.argtypes = [vp, dp]
    L.lbm_ec_stats.restype = ctypes.c_int
    L.lbm_ec_profile_begin.argtypes = [vp, ctypes.c_uint32]
    L.lbm_ec_profile_begin.restype = ctypes.c_int
    L.lbm_ec_profile_end.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
    L.lbm_ec_profile_end.restype = ctypes.c_int
    L.lbm_ec_checkpoint_bytes.argtypes = [vp]
    L.lbm_ec_checkpoint_bytes.restype = ctypes.c_size_t
    L.lbm_ec_save.argtypes = [vp, vp, ctypes.c_size_t]
    L.lbm_ec_save.restype = ctypes.c_int
    L.lbm_ec_load.argtypes = [vp, vp, ctypes.c_size_t]
    L.lbm_ec_load.restype = ctypes.c_int
    i32 = ctypes.c_int32
    L.lbm_ec_batch_workspace_bytes.argtypes = [P, i32, i32, i32]
    L.lbm_ec_batch_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_ec_batch_create.argtypes = [i32, i32, i32, i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.lbm_ec_batch_create.restype = ctypes.c_int
    L.lbm_ec_batch_admit.argtypes = [vp, P, ctypes.c_int64, ctypes.POINTER(i32)]
    L.lbm_ec_batch_admit.restype = ctypes.c_int
    L.lbm_ec_batch_step.argtypes = [vp, ctypes.c_int64]
    L.lbm_ec_batch_step.restype = ctypes.c_int
    L.lbm_ec_batch_poll.argtypes = [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
    L.lbm_ec_batch_poll.restype = ctypes.c_int
    L.lbm_ec_batch_steps_done.argtypes = [vp, i32]
    L.lbm_ec_batch_steps_done.restype = ctypes.c_int64
    L.lbm_ec_batch_fields.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.lbm_ec_batch_fields.restype = ctypes.c_int
    L.lbm_ec_batch_fields_rho_m1.argtypes = [vp, i32, vp]
    L.lbm_ec_batch_fields_rho_m1.restype = ctypes.c_int
    L.lbm_ec_batch_history.argtypes = [vp, i32, dp, i32]
    L.lbm_ec_batch_history.restype = ctypes.c_int
    L.lbm_ec_batch_release.argtypes = [vp, i32]
    L.lbm_ec_batch_release.restype = ctypes.c_int
    L.lbm_ec_batch_free_bytes.argtypes = [vp]
    L.lbm_ec_batch_free_bytes.restype = ctypes.c_size_t
    L.lbm_ec_batch_destroy.argtypes = [vp]
    L.lbm_ec_batch_destroy.restype = None
    L.lbm_ec_set_tuning.argtypes = [vp, i32, i32, i32, i32]
    L.lbm_ec_set_tuning.restype = ctypes.c_int
    L.lbm_ec_batch_set_tuning.argtypes = [vp, i32, i32, i32, i32]
    L.lbm_ec_batch_set_tuning.restype = ctypes.c_int
    L.lbm_ec_debug_poison.argtypes = [vp]
    L.lbm_ec_debug_poison.restype = ctypes.c_int
    L.lbm_ec_batch_debug_poison.argtypes = [vp, i32]
    L.lbm_ec_batch_debug_poison.restype = ctypes.c_int
    L.lbm_ec_set_y_solver.argtypes = [vp, i32]
    L.lbm_ec_set_y_solver.restype = ctypes.c_int
    L.lbm_ec_set_T.argtypes = [vp, ctypes.c_double]
    L.lbm_ec_set_T.restype = ctypes.c_int
    L.lbm_ec_batch_set_T.argtypes = [vp, i32, ctypes.c_double]
    L.lbm_ec_batch_set_T.restype = ctypes.c_int
    L.lbm_ec_destroy.argtypes = [vp]
    L.lbm_ec_destroy.restype = None
    L.lbm_ec_last_error.argtypes = []
    L.lbm_ec_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(code):
    if code != OK:
        raise LbmEcError(code, lib().lbm_ec_last_error().decode())


def make_params(nx, ny, T=200.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25,
                Lambda_g=1e-6, precision="fp64", init_mode="noise", noise_amp=1e-3,
                seed=181205711, instance_id=0, charge_rates="antisymmetric", body_force_x=0.0):
    p = Params()
    _check(lib().lbm_ec_params_default(ctypes.byref(p)))
    p.nx, p.ny = int(nx), int(ny)
    p.T, p.C, p.M, p.Fe = float(T), float(C), float(M), float(Fe)
    p.tau_plus, p.Lambda, p.Lambda_g = float(tau_plus), float(Lambda), float(Lambda_g)
    p.precision = _PRECISION[precision] if isinstance(precision, str) else int(precision)
    p.init_mode = _INIT[init_mode] if isinstance(init_mode, str) else int(init_mode)
    p.noise_amp = float(noise_amp)
    p.seed = int(seed) % (1 << 64)
    p.instance_id = int(instance_id)
    p.charge_rates = _RATES[charge_rates] if isinstance(charge_rates, str) else int(charge_rates)
    p.body_force_x = float(body_force_x)
    return p


def workspace_bytes(p: Params) -> int:
    n = lib().lbm_ec_workspace_bytes(ctypes.byref(p))
    if n == 0:
        _check(lib().lbm_ec_validate(ctypes.byref(p)))
    return n


STATIC_SCRATCH_BYTES = 64 << 20  # LBM_EC_STATIC_SCRATCH_BYTES


def poisson_static_bytes(**kw) -> int:
    """Scratch bytes lbm_ec_poisson_static needs for these parameters."""
    return int(lib().lbm_ec_poisson_static_bytes(ctypes.byref(make_params(**kw))))


def poisson_static(rho_c: torch.Tensor, out: torch.Tensor = None, stream=None, **kw) -> torch.Tensor:
    """phi for a nondimensional charge density (ny, nx) through
    lbm_ec_poisson_static, which allocates no device memory: its scratch is a
    static array of the library.  `out` (a float64 (ny, nx) device tensor)
    receives phi; allocate it beforehand to keep the whole call free of
    allocations.  kw: the parameters of make_params (nx, ny, T, M, tau_plus,
    init_mode, precision ...)."""
    p = make_params(**kw)
    assert rho_c.is_cuda and rho_c.dtype == torch.float64 and rho_c.is_contiguous()
    assert tuple(rho_c.shape) == (p.ny, p.nx)
    if out is None:
        out = torch.empty_like(rho_c)
    assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.shape == rho_c.shape
    if stream is None:
        stream = torch.cuda.current_stream(rho_c.device)
    with torch.cuda.device(rho_c.device):
        _check(lib().lbm_ec_poisson_static(ctypes.byref(p), ctypes.c_void_p(rho_c.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream)))
    return out


class Simulation:
    """One simulation on a GPU: its workspace is a torch uint8 tensor."""

    def __init__(self, device="cuda:0", stream=None, **kw):
        self.device = torch.device(device)
        self.params = make_params(**kw)
        nbytes = workspace_bytes(self.params)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            h = ctypes.c_void_p()
            _check(lib().lbm_ec_create(ctypes.byref(self.params), ctypes.c_void_p(self.workspace.data_ptr()),
                                       nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    @property
    def nx(self):
        return self.params.nx

    @property
    def ny(self):
        return self.params.ny

    def step(self, n=1):
        _check(lib().lbm_ec_step(self._h, int(n)))
        return self

    def steps_done(self):
        return int(lib().lbm_ec_steps_done(self._h))

    def fields(self):
        """Dict of nondimensional FP64 device tensors (ny, nx): rho, ux, uy,
        rho_c, phi, and rho_m1 = rho - 1 (lbm_ec_fields_rho_m1)."""
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "rho_c", "phi", "rho_m1")}
        _check(lib().lbm_ec_fields(self._h, *[ctypes.c_void_p(out[k].data_ptr())
                                              for k in ("rho", "ux", "uy", "rho_c", "phi")]))
        _check(lib().lbm_ec_fields_rho_m1(self._h, ctypes.c_void_p(out["rho_m1"].data_ptr())))
        return out

    def poisson(self, rho_c: torch.Tensor) -> torch.Tensor:
        """phi for a nondimensional charge density (testing entry point)."""
        rho_c = rho_c.to(device=self.device, dtype=torch.float64).contiguous()
        assert tuple(rho_c.shape) == (self.ny, self.nx)
        phi = torch.empty_like(rho_c)
        _check(lib().lbm_ec_poisson(self._h, ctypes.c_void_p(rho_c.data_ptr()), ctypes.c_void_p(phi.data_ptr())))
        return phi

    def stats(self):
        buf = (ctypes.c_double * 10)()
        code = lib().lbm_ec_stats(self._h, buf)
        if code not in (OK, EUNSTABLE):
            _check(code)
        names = ["steps", "mass_dev", "charge", "rms_uy", "max_u", "min_rho_c", "bad", "max_ex", "q_injector",
                 "q_collector"]
        return dict(zip(names, list(buf))), code == OK

    def set_tuning(self, fft_threads=256, collide_bx=256, collide_by=1, collide_tw=0):
        _check(lib().lbm_ec_set_tuning(self._h, int(fft_threads), int(collide_bx), int(collide_by),
                                       int(collide_tw)))

    def set_y_solver(self, solver):
        """'tridiagonal' (default) or 'spectral' (lbm_ec_set_y_solver)."""
        code = {"tridiagonal": Y_TRIDIAGONAL, "spectral": Y_SPECTRAL}.get(solver, solver)
        _check(lib().lbm_ec_set_y_solver(self._h, int(code)))

    def set_T(self, T):
        """Continue the run at electric Rayleigh number T (lbm_ec_set_T)."""
        _check(lib().lbm_ec_set_T(self._h, float(T)))
        self.params.T = float(T)

    def debug_poison(self):
        """Test hook: a NaN into one population of the current state."""
        _check(lib().lbm_ec_debug_poison(self._h))

    def save(self) -> torch.Tensor:
        """Checkpoint of the current state in a new device uint8 tensor."""
        n = lib().lbm_ec_checkpoint_bytes(self._h)
        buf = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().lbm_ec_save(self._h, ctypes.c_void_p(buf.data_ptr()), n))
        return buf

    def load(self, buf: torch.Tensor):
        """Replaces the state with a checkpoint taken by save() on an
        instance with the same grid and parameters."""
        assert buf.is_cuda and buf.dtype == torch.uint8 and buf.is_contiguous()
        _check(lib().lbm_ec_load(self._h, ctypes.c_void_p(buf.data_ptr()), buf.numel()))

    KERNEL_CLASSES = ("forward", "tridiag", "inverse", "collide")

    def profile_begin(self, classes=None):
        """Times the kernel classes named in `classes` (default: all of
        self.KERNEL_CLASSES) until profile_end."""
        names = self.KERNEL_CLASSES if classes is None else classes
        mask = 0
        for c in names:
            mask |= 1 << self.KERNEL_CLASSES.index(c)
        _check(lib().lbm_ec_profile_begin(self._h, mask))

    def profile_end(self):
        """{class: (total_ms, launches)} since profile_begin (waits for the stream)."""
        n = len(self.KERNEL_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(lib().lbm_ec_profile_end(self._h, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNEL_CLASSES)}

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_ec_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_workspace_bytes(params_list, max_slots, hist_rows):
    n = len(params_list)
    arr = (Params * max(n, 1))(*params_list) if n else None
    return int(lib().lbm_ec_batch_workspace_bytes(arr, n, int(max_slots), int(hist_rows)))


class Batch:
    """Many simulations advanced together (C ABI lbm_ec_batch_*).

    The workspace is one torch uint8 tensor of `workspace_bytes`; the batch
    runs on its own torch stream unless one is given.
    """

    def __init__(self, max_slots, workspace_bytes, precision="fp32_f64math", emit_every=100, hist_rows=256,
                 device="cuda:0", stream=None):
        self.device = torch.device(device)
        self.precision = _PRECISION[precision] if isinstance(precision, str) else int(precision)
        self.hist_rows = int(hist_rows)
        self.emit_every = int(emit_every)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=self.device)
            h = ctypes.c_void_p()
            _check(lib().lbm_ec_batch_create(int(max_slots), self.precision, self.emit_every, self.hist_rows,
                                             ctypes.c_void_p(self.workspace.data_ptr()), int(workspace_bytes),
                                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._shape = {}

    def admit(self, n_steps, **kw):
        """Slot index, or None when no slot or workspace is free (EBUSY)."""
        kw.setdefault("precision", self.precision)
        p = make_params(**kw)
        slot = ctypes.c_int32(-1)
        code = lib().lbm_ec_batch_admit(self._h, ctypes.byref(p), int(n_steps), ctypes.byref(slot))
        if code == EBUSY:
            return None
        _check(code)
        self._shape[slot.value] = (p.ny, p.nx)
        return slot.value

    def step(self, n=1):
        _check(lib().lbm_ec_batch_step(self._h, int(n)))
        return self

    def poll(self):
        cap = 4096
        buf = (ctypes.c_int32 * cap)()
        nd = ctypes.c_int32(0)
        _check(lib().lbm_ec_batch_poll(self._h, buf, cap, ctypes.byref(nd)))
        return [buf[i] for i in range(nd.value)]

    def steps_done(self, slot):
        return int(lib().lbm_ec_batch_steps_done(self._h, int(slot)))

    def fields(self, slot):
        ny, nx = self._shape[slot]
        out = {k: torch.empty((ny, nx), dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "rho_c", "phi", "rho_m1")}
        _check(lib().lbm_ec_batch_fields(self._h, int(slot), *[ctypes.c_void_p(out[k].data_ptr())
                                                               for k in ("rho", "ux", "uy", "rho_c", "phi")]))
        _check(lib().lbm_ec_batch_fields_rho_m1(self._h, int(slot), ctypes.c_void_p(out["rho_m1"].data_ptr())))
        self.stream.synchronize()
        return out

    def history(self, slot):
        """The slot's history rows, shape (hist_rows, HIST_COLS); unused rows are zero."""
        import numpy as np

        buf = (ctypes.c_double * (HIST_COLS * self.hist_rows))()
        _check(lib().lbm_ec_batch_history(self._h, int(slot), buf, self.hist_rows))
        return np.frombuffer(buf, dtype=np.float64).reshape(self.hist_rows, HIST_COLS).copy()

    def set_tuning(self, fft_threads=256, collide_bx=256, collide_by=1, collide_tw=0):
        _check(lib().lbm_ec_batch_set_tuning(self._h, int(fft_threads), int(collide_bx), int(collide_by),
                                             int(collide_tw)))

    def set_T(self, slot, T):
        """Continue the slot at electric Rayleigh number T (lbm_ec_batch_set_T)."""
        _check(lib().lbm_ec_batch_set_T(self._h, int(slot), float(T)))

    def debug_poison(self, slot):
        """Test hook: a NaN into one population of the slot's current state."""
        _check(lib().lbm_ec_batch_debug_poison(self._h, int(slot)))

    def release(self, slot):
        _check(lib().lbm_ec_batch_release(self._h, int(slot)))
        self._shape.pop(slot, None)

    def free_bytes(self):
        return int(lib().lbm_ec_batch_free_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_ec_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
