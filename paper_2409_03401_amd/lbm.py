"""Python binding of liblbm.so (include/lbm.h): argument marshalling only.

Every step of the method runs in the HIP kernels of the library; this module
allocates device memory with torch, passes pointers and the current HIP stream,
and turns return codes into exceptions.  It fails loudly when the library has
not been built or no GPU is present: there is no CPU fallback.
"""

import ctypes
import math
import os
from dataclasses import dataclass, field, replace
from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

# ---- constants of include/lbm.h ------------------------------------------------------
LBM_OK, LBM_EINVAL, LBM_ESIZE, LBM_EUNSTABLE, LBM_EUNSUPPORTED, LBM_EHIP = 0, -1, -2, -3, -4, -5
LBM_NONE, LBM_D2Q9, LBM_D3Q19, LBM_D2Q5, LBM_D3Q7 = 0, 9, 19, 5, 7
LBM_PERIODIC, LBM_WALLS = 0, 1
LBM_FP64, LBM_FP32, LBM_FP32_FP16STORE, LBM_FP32_BF16STORE = 0, 1, 2, 3
LBM_OUT_F64, LBM_OUT_F32 = 0, 1
LBM_BGK, LBM_TRT, LBM_MRT = 0, 1, 2
_COLLISION = {"BGK": LBM_BGK, "TRT": LBM_TRT, "MRT": LBM_MRT}
# moments in the order of the LBM_M_* bits; cC, muC exist with a third composition
MOMENTS = ("phi", "cA", "cB", "muA", "muB", "p", "ux", "uy", "uz", "cC", "muC")
TERNARY_MOMENTS = MOMENTS[:9]
# diagnostics in the order of the LBM_D_* indices; sum_cC exists with a third composition
DIAGNOSTICS = ("sum_cA", "sum_cB", "sum_phi", "kinetic_energy", "max_u", "interface_measure",
               "free_energy", "nan_count", "droplets", "mean_radius", "sum_cC")
PRECISIONS = {"fp64": LBM_FP64, "fp32": LBM_FP32, "fp16": LBM_FP32_FP16STORE, "bf16": LBM_FP32_BF16STORE}
_FLUID = {None: LBM_NONE, "none": LBM_NONE, "D2Q9": LBM_D2Q9, "D3Q19": LBM_D3Q19}
# D2Q5 / D3Q7: reduced scalar lattices; D2Q9 / D3Q19: the paper's
_SCALAR = {"D2Q5": LBM_D2Q5, "D3Q7": LBM_D3Q7, "D2Q9": LBM_D2Q9, "D3Q19": LBM_D3Q19}
_BC = {"periodic": LBM_PERIODIC, "walls": LBM_WALLS}
_ERRNAMES = {LBM_EINVAL: "LBM_EINVAL", LBM_ESIZE: "LBM_ESIZE", LBM_EUNSTABLE: "LBM_EUNSTABLE",
             LBM_EUNSUPPORTED: "LBM_EUNSUPPORTED", LBM_EHIP: "LBM_EHIP"}


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class _Config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("fluid", ctypes.c_int32), ("scalar", ctypes.c_int32), ("bc", ctypes.c_int32 * 3),
        ("precision", ctypes.c_int32), ("gravity_mean_subtract", ctypes.c_int32),
        ("W", ctypes.c_double), ("lambda_", ctypes.c_double), ("M_phi", ctypes.c_double),
        ("M_A", ctypes.c_double * 2), ("M_B", ctypes.c_double * 2),
        ("c_eq", (ctypes.c_double * 2) * 2),
        ("rho0", ctypes.c_double), ("drho", ctypes.c_double), ("g", ctypes.c_double * 3),
        ("sigma", ctypes.c_double), ("nu", ctypes.c_double * 2),
        ("store_ref", ctypes.c_double * 4), ("store_shift", ctypes.c_int32 * 4),
        ("collision", ctypes.c_int32), ("variable_density", ctypes.c_int32), ("trt_magic", ctypes.c_double * 2),
        ("general_kappa", ctypes.c_int32), ("ncomp", ctypes.c_int32), ("kappa", (ctypes.c_double * 3) * 2),
        ("mrt_rates", (ctypes.c_double * 3) * 2),
        ("c_eq_C", ctypes.c_double * 2), ("M_C", ctypes.c_double * 2),
        ("store_shift_C", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


_LIB = None

# exported entry points and their ctypes signatures
_SIGS = {
    "lbm_state_bytes": (ctypes.c_int, [ctypes.POINTER(_Config), ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_checkpoint_bytes": (ctypes.c_int, [ctypes.POINTER(_Config), ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_init": (ctypes.c_int, [ctypes.POINTER(_Config), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.POINTER(ctypes.c_void_p)]),
    "lbm_init_composition": (ctypes.c_int, [ctypes.POINTER(_Config), ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "lbm_init_multi": (ctypes.c_int, [ctypes.POINTER(_Config), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "lbm_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "lbm_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p),
                                   ctypes.c_int32, ctypes.c_void_p]),
    "lbm_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "lbm_run_series": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "lbm_get_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_set_populations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_restore": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_step_external": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "lbm_phase_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_adjoint_bytes": (ctypes.c_int, [ctypes.POINTER(_Config), ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_adjoint_seed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "lbm_adjoint_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "lbm_adjoint_step_phi": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "lbm_init_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "lbm_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_adjoint_step_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p]),
    "lbm_adjoint_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_adjoint_theta": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_adjoint_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_adjoint_set": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbm_step_count": (ctypes.c_int64, [ctypes.c_void_p]),
    "lbm_probe_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_void_p]),
    "lbm_destroy": (None, [ctypes.c_void_p]),
    "lbm_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load liblbm.so once; raise if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2409_03401_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(code):
    if code != LBM_OK:
        raise LBMError(code, lib().lbm_last_error().decode())


@dataclass
class LBMConfig:
    """Parameters in lattice units; mirrors ``lbm_config`` of include/lbm.h."""
    nx: int
    ny: int
    nz: int = 1
    fluid: Optional[str] = None
    scalar: str = "D2Q5"
    bc: Tuple[str, str, str] = ("periodic", "periodic", "periodic")
    W: float = 4.0
    lam: float = 1.0
    M_phi: float = 0.1
    M_A: Tuple[float, float] = (0.1, 0.1)
    M_B: Tuple[float, float] = (0.1, 0.1)
    # c_eq[phase] = (c^A, c^B) for the paper's ternary fluid, or (c^A, c^B, c^C) with a
    # third independent composition C (N components; needs M_C)
    c_eq: Tuple[Tuple[float, ...], Tuple[float, ...]] = ((0.2, 0.1), (0.6, 0.3))
    M_C: Optional[Tuple[float, float]] = None
    store_shift_C: int = 6
    rho0: float = 1.0
    drho: float = 0.0
    g: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    sigma: float = 0.0
    nu: Tuple[float, float] = (0.1, 0.1)
    gravity_mean_subtract: bool = False
    precision: str = "fp32"
    # 16-bit storage: moving population k of field F (f, g, hA, hB) is stored as
    # (x - w_k store_ref[F]) * 2^store_shift[F] in FP16, as x - w_k store_ref[F] in BF16
    store_ref: Tuple[float, float, float, float] = (0.0, 0.5, 0.0, 0.0)
    store_shift: Tuple[int, int, int, int] = (8, 0, 6, 6)
    # "BGK" (the paper's), "TRT" or "MRT"; TRT magic parameters of (f, the scalar lattices)
    collision: str = "BGK"
    trt_magic: Tuple[float, float] = (3.0 / 16.0, 0.25)
    # MRT free rates: f (bulk, third, fourth order), scalars (second, third, fourth order)
    mrt_rates: Tuple[Tuple[float, float, float], Tuple[float, float, float]] = ((1.2, 1.1, 1.2), (1.1, 1.0, 1.2))
    # False: Boussinesq (the paper's); True: rho(phi) model with pressure and viscous forces
    variable_density: bool = False
    # general curvatures ((k_AA, k_AB, k_BB) of phase 0, of phase 1) = K (K_pi)^-1; None: identity
    kappa: Optional[Tuple[Tuple[float, float, float], Tuple[float, float, float]]] = None

    @property
    def nodes(self):
        return self.nx * self.ny * self.nz

    @property
    def ncomp(self):
        """Independent compositions: 2 (A, B) or 3 (A, B, C)."""
        return len(self.c_eq[0])

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def qf(self):
        return _FLUID[self.fluid]

    @property
    def qs(self):
        return _SCALAR[self.scalar]

    def to_c(self) -> _Config:
        c = _Config()
        c.dim = 2 if self.scalar in ("D2Q5", "D2Q9") else 3
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.fluid = _FLUID[self.fluid]
        c.scalar = _SCALAR[self.scalar]
        for a in range(3):
            c.bc[a] = _BC[self.bc[a]]
        c.precision = PRECISIONS[self.precision]
        c.gravity_mean_subtract = int(bool(self.gravity_mean_subtract))
        c.W, c.lambda_, c.M_phi = self.W, self.lam, self.M_phi
        for i in range(2):
            c.M_A[i], c.M_B[i], c.nu[i] = self.M_A[i], self.M_B[i], self.nu[i]
            for a in range(2):
                c.c_eq[i][a] = self.c_eq[i][a]
        if len(self.c_eq[0]) != len(self.c_eq[1]) or self.ncomp not in (2, 3):
            raise ValueError("c_eq needs 2 or 3 compositions per phase, the same for both phases")
        if (self.M_C is not None) != (self.ncomp == 3):
            raise ValueError("a third composition takes c_eq entries and M_C together")
        c.ncomp = self.ncomp
        if self.ncomp == 3:
            for i in range(2):
                c.c_eq_C[i] = self.c_eq[i][2]
                c.M_C[i] = self.M_C[i]
            c.store_shift_C = int(self.store_shift_C)
        c.rho0, c.drho, c.sigma = self.rho0, self.drho, self.sigma
        for a in range(3):
            c.g[a] = self.g[a]
        for i in range(4):
            c.store_ref[i] = self.store_ref[i]
            c.store_shift[i] = int(self.store_shift[i])
        c.collision = _COLLISION[self.collision]
        c.variable_density = int(bool(self.variable_density))
        for i in range(2):
            for j in range(3):
                c.mrt_rates[i][j] = float(self.mrt_rates[i][j])
        c.general_kappa = int(self.kappa is not None)
        if self.kappa is not None:
            for pi in range(2):
                for i in range(3):
                    c.kappa[pi][i] = float(self.kappa[pi][i])
        c.trt_magic[0], c.trt_magic[1] = float(self.trt_magic[0]), float(self.trt_magic[1])
        return c


def state_bytes(cfg: LBMConfig) -> int:
    n = ctypes.c_size_t()
    _check(lib().lbm_state_bytes(ctypes.byref(cfg.to_c()), ctypes.byref(n)))
    return n.value


def checkpoint_bytes(cfg: LBMConfig) -> int:
    n = ctypes.c_size_t()
    _check(lib().lbm_checkpoint_bytes(ctypes.byref(cfg.to_c()), ctypes.byref(n)))
    return n.value


def adjoint_bytes(cfg: LBMConfig) -> int:
    n = ctypes.c_size_t()
    _check(lib().lbm_adjoint_bytes(ctypes.byref(cfg.to_c()), ctypes.byref(n)))
    return n.value


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _on(stream, *temps):
    """Prepare a launch on `stream` (None: the current stream) that reads tensors made
    on the current stream: the launch stream first waits for the current one, and the
    caching allocator is told that `temps` are in use on the launch stream."""
    cur = torch.cuda.current_stream()
    if stream is not None and stream != cur:
        stream.wait_stream(cur)
        for t in temps:
            t.record_stream(stream)
    return _stream_ptr(stream)


def _dev_f64(a, n, device):
    t = torch.as_tensor(a, dtype=torch.float64, device=device).reshape(-1).contiguous()
    if t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    return t


class Simulation:
    """One domain on one GPU: state buffer (torch uint8 tensor) plus the library handle."""

    def __init__(self, cfg: LBMConfig, phi0, muA0, muB0, device="cuda", stream=None, c0=None, mu_x0=()):
        """c0 = (cA0, cB0) gives the compositions instead of the closure
        (lbm_init_composition: the initial condition of Section 4.2.1).  With a third
        composition, mu_x0 = (muC0,) and c0 = (cA0, cB0, cC0) (lbm_init_multi)."""
        if not torch.cuda.is_available():
            raise RuntimeError("liblbm needs a GPU; none is visible")
        L = lib()
        self.cfg = cfg
        self.device = torch.device(device)
        self._c = cfg.to_c()
        nbytes = state_bytes(cfg)
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        n = cfg.nodes
        if len(mu_x0) != cfg.ncomp - 2:
            raise ValueError(f"{cfg.ncomp} compositions need {cfg.ncomp - 2} entries in mu_x0")
        self._inputs = [_dev_f64(a, n, self.device) for a in (phi0, muA0, muB0) + tuple(mu_x0)]
        ptrs = [ctypes.c_void_p(t.data_ptr()) for t in self._inputs]
        h = ctypes.c_void_p()
        if cfg.ncomp != 2:
            mu = (ctypes.c_void_p * cfg.ncomp)(*[p.value for p in ptrs[1:]])
            cp = None
            self._c_inputs = []
            if c0 is not None:
                if len(c0) != cfg.ncomp:
                    raise ValueError(f"c0 needs {cfg.ncomp} compositions")
                self._c_inputs = [_dev_f64(a, n, self.device) for a in c0]
                cp = (ctypes.c_void_p * cfg.ncomp)(*[t.data_ptr() for t in self._c_inputs])
            _check(L.lbm_init_multi(ctypes.byref(self._c), ctypes.c_void_p(self.state.data_ptr()), nbytes, ptrs[0],
                                    mu, cp, _on(stream, self.state, *self._inputs, *self._c_inputs),
                                    ctypes.byref(h)))
        elif c0 is None:
            _check(L.lbm_init(ctypes.byref(self._c), ctypes.c_void_p(self.state.data_ptr()), nbytes,
                              *ptrs, _on(stream, self.state, *self._inputs), ctypes.byref(h)))
        else:
            self._c_inputs = [_dev_f64(a, n, self.device) for a in c0]
            cp = [ctypes.c_void_p(t.data_ptr()) for t in self._c_inputs]
            _check(L.lbm_init_composition(ctypes.byref(self._c), ctypes.c_void_p(self.state.data_ptr()), nbytes,
                                          ptrs[0], cp[0], cp[1], ptrs[1], ptrs[2],
                                          _on(stream, self.state, *self._inputs, *self._c_inputs), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nslots(self):
        return self.cfg.qf + (1 + self.cfg.ncomp) * self.cfg.qs

    def step(self, n=1, stream=None):
        _check(lib().lbm_step(self._h, int(n), _stream_ptr(stream)))

    @property
    def step_count(self):
        return lib().lbm_step_count(self._h)

    @property
    def moment_names(self):
        return MOMENTS if self.cfg.ncomp == 3 else TERNARY_MOMENTS

    def moments(self, names: Optional[Sequence[str]] = None, dtype=torch.float64,
                stream=None) -> Dict[str, torch.Tensor]:
        """Fields named in `names` (default: every moment of this run)."""
        if names is None:
            names = self.moment_names
        out_dtype = LBM_OUT_F64 if dtype == torch.float64 else LBM_OUT_F32
        outs = {}
        ptrs = (ctypes.c_void_p * len(MOMENTS))()
        mask = 0
        for i, name in enumerate(MOMENTS):
            if name in names:
                t = torch.empty(self.cfg.shape, dtype=dtype, device=self.device)
                outs[name] = t
                ptrs[i] = t.data_ptr()
                mask |= 1 << i
        _check(lib().lbm_moments(self._h, mask, ptrs, out_dtype, _stream_ptr(stream)))
        return outs

    def diagnostics(self, stream=None) -> Dict[str, float]:
        out = (ctypes.c_double * len(DIAGNOSTICS))()
        _check(lib().lbm_diagnostics(self._h, out, _stream_ptr(stream)))
        d = dict(zip(self.diagnostic_names, list(out)))
        for k in ("nan_count", "droplets"):  # integer counts (exact in FP64)
            d[k] = int(d[k])
        return d

    @property
    def diagnostic_names(self):
        return DIAGNOSTICS if self.cfg.ncomp == 3 else DIAGNOSTICS[:-1]

    def run_series(self, steps: int, every: int, stream=None) -> Dict[str, np.ndarray]:
        """Advance `steps` steps recording the diagnostics every `every` steps (and of
        the starting state): arrays of length steps // every + 1 per diagnostic, plus
        "step" (time steps since init)."""
        if every < 1 or steps < 0 or steps % every:
            raise ValueError("steps must be a non-negative multiple of every >= 1")
        rows = steps // every + 1
        out = (ctypes.c_double * (rows * len(DIAGNOSTICS)))()
        start = self.step_count
        _check(lib().lbm_run_series(self._h, int(steps), int(every), out, _stream_ptr(stream)))
        a = np.frombuffer(out, dtype=np.float64).reshape(rows, len(DIAGNOSTICS)).copy()
        d = {k: a[:, i] for i, k in enumerate(self.diagnostic_names)}
        for k in ("nan_count", "droplets"):
            d[k] = d[k].astype(np.int64)
        d["step"] = start + every * np.arange(rows, dtype=np.int64)
        return d

    def populations(self, stream=None) -> torch.Tensor:
        """[slot][z][y][x] FP64 decoded populations: f_0.., g_0.., hA_0.., hB_0.."""
        t = torch.empty((self.nslots,) + self.cfg.shape, dtype=torch.float64, device=self.device)
        _check(lib().lbm_get_populations(self._h, ctypes.c_void_p(t.data_ptr()), _stream_ptr(stream)))
        return t

    def set_populations(self, pops, stream=None):
        t = torch.as_tensor(pops, dtype=torch.float64, device=self.device).contiguous()
        if t.numel() != self.nslots * self.cfg.nodes:
            raise ValueError("wrong population count")
        _check(lib().lbm_set_populations(self._h, ctypes.c_void_p(t.data_ptr()), _on(stream, t)))

    def save(self, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(checkpoint_bytes(self.cfg), dtype=torch.uint8, device=self.device)
        _check(lib().lbm_save(self._h, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def restore(self, ckpt: torch.Tensor, stream=None):
        _check(lib().lbm_restore(self._h, ctypes.c_void_p(ckpt.data_ptr()), _stream_ptr(stream)))

    def set_state(self, ckpt: torch.Tensor, stream=None):
        """Restore the checkpoint `ckpt` (lbm_save layout) as the current state."""
        _check(lib().lbm_set_state(self._h, ctypes.c_void_p(ckpt.data_ptr()), _stream_ptr(stream)))

    # ---- discrete adjoint (reverse mode) ----------------------------------------------
    @property
    def phi_dtype(self):
        """Type of the phi fields of step_external / phase_field (the compute type)."""
        return torch.float64 if self.cfg.precision == "fp64" else torch.float32

    def step_external(self, src: torch.Tensor, dst: torch.Tensor, phi_src: Optional[torch.Tensor] = None,
                      stream=None):
        """One step from checkpoint `src` into checkpoint `dst` (lbm_save layout);
        phi_src, when given, receives phi of `src`."""
        _check(lib().lbm_step_external(self._h, _ptr(src), _ptr(dst),
                                       _ptr(phi_src) if phi_src is not None else None, _stream_ptr(stream)))

    def phase_field(self, state: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """phi of the checkpoint `state` in the compute type ([node])."""
        if out is None:
            out = torch.empty(self.cfg.nodes, dtype=self.phi_dtype, device=self.device)
        _check(lib().lbm_phase_field(self._h, _ptr(state), _ptr(out), _stream_ptr(stream)))
        return out

    def adjoint_workspace(self) -> torch.Tensor:
        return torch.zeros(adjoint_bytes(self.cfg), dtype=torch.uint8, device=self.device)

    def adjoint_seed(self, state: torch.Tensor, dL_dphi: torch.Tensor, work: torch.Tensor, stream=None):
        """Start the adjoint from dL/dphi_T at the checkpoint `state`; clears the theta partials."""
        d = _dev_f64(dL_dphi, self.cfg.nodes, self.device)
        _check(lib().lbm_adjoint_seed(self._h, _ptr(state), _ptr(d), _ptr(work), _on(stream, d)))

    def adjoint_step_phi(self, state: torch.Tensor, phi: torch.Tensor, work: torch.Tensor, stream=None):
        """Adjoint of the step taken from checkpoint `state` whose phi is `phi`; the
        parameter gradient stays in the workspace (adjoint_theta)."""
        _check(lib().lbm_adjoint_step_phi(self._h, _ptr(state), _ptr(phi), _ptr(work), _stream_ptr(stream)))

    def adjoint_step(self, state: torch.Tensor, work: torch.Tensor, grad_params: torch.Tensor, stream=None):
        """lbm_adjoint_step: adjoint of the step taken from checkpoint `state`; the
        parameter gradient collected so far is added to grad_params (6 FP64, device)."""
        _check(lib().lbm_adjoint_step(self._h, _ptr(state), _ptr(work), _ptr(grad_params), _stream_ptr(stream)))

    def adjoint_step_noalloc(self, state: torch.Tensor, adj_state: torch.Tensor, grad_params: torch.Tensor,
                             stream=None):
        """lbm_adjoint_step_noalloc: the adjoint step with its scratch inside the library
        (adj_state: the adjoint state part of a workspace, adjoint_state_bytes)."""
        _check(lib().lbm_adjoint_step_noalloc(self._h, _ptr(state), _ptr(adj_state), _ptr(grad_params),
                                              _stream_ptr(stream)))

    @property
    def adjoint_state_bytes(self):
        """Bytes of the adjoint state (two copies of the adjoint slots, three c_F rows)."""
        row = (4 * self.cfg.nodes + 255) // 256 * 256
        return (2 * self.nslots + 3) * row

    def init_adjoint(self, work: torch.Tensor, grad_phi0: torch.Tensor, grad_params: torch.Tensor, stream=None):
        """lbm_init_adjoint: dL/dphi_0 into grad_phi0 through lbm_init (mu_0 fixed), the
        remaining parameter gradient added to grad_params."""
        _check(lib().lbm_init_adjoint(self._h, _ptr(work), _ptr(grad_phi0), _ptr(grad_params),
                                      _on(stream, *self._inputs)))

    def adjoint_init(self, work: torch.Tensor, grad_phi0: torch.Tensor, stream=None):
        """dL/dphi_0 (written into grad_phi0) through lbm_init, mu_0 held fixed."""
        phi0, muA0, muB0 = self._inputs
        _check(lib().lbm_adjoint_init(self._h, _ptr(phi0), _ptr(muA0), _ptr(muB0), _ptr(work), _ptr(grad_phi0),
                                      _on(stream, phi0, muA0, muB0)))

    def adjoint_theta(self, work: torch.Tensor, stream=None) -> torch.Tensor:
        """dL/dtheta (THETA_NAMES order) accumulated since the last seed or set."""
        out = torch.empty(6, dtype=torch.float64, device=self.device)
        _check(lib().lbm_adjoint_theta(self._h, _ptr(work), _ptr(out), _stream_ptr(stream)))
        return out

    def adjoint_get(self, work: torch.Tensor, stream=None) -> torch.Tensor:
        t = torch.empty((self.nslots,) + self.cfg.shape, dtype=torch.float64, device=self.device)
        _check(lib().lbm_adjoint_get(self._h, _ptr(work), _ptr(t), _stream_ptr(stream)))
        return t

    def adjoint_set(self, work: torch.Tensor, lam, stream=None):
        t = torch.as_tensor(lam, dtype=torch.float64, device=self.device).contiguous()
        if t.numel() != self.nslots * self.cfg.nodes:
            raise ValueError("wrong adjoint population count")
        _check(lib().lbm_adjoint_set(self._h, _ptr(work), _ptr(t), _on(stream, t)))


# parameters the adjoint differentiates, in the order of grad_theta
THETA_NAMES = ("M_phi", "M_A0", "M_A1", "M_B0", "M_B1", "W")


def theta_of(cfg: LBMConfig):
    return (cfg.M_phi, cfg.M_A[0], cfg.M_A[1], cfg.M_B[0], cfg.M_B[1], cfg.W)


def with_theta(cfg: LBMConfig, theta) -> LBMConfig:
    t = [float(v) for v in theta]
    return replace(cfg, M_phi=t[0], M_A=(t[1], t[2]), M_B=(t[3], t[4]), W=t[5])


class PhaseFieldRun(torch.autograd.Function):
    """phi_T = run(phi_0, theta) for `steps` steps on the GPU, differentiable in
    phi_0 and theta = (M_phi, M^A_0, M^A_1, M^B_0, M^B_1, W) (THETA_NAMES).

    Forward keeps a checkpoint every `segment` steps (default ceil(sqrt(steps)));
    backward recomputes each segment from its checkpoint into `segment` state
    buffers (keeping phi of each state, which the step computes anyway) and runs
    the adjoint steps through it in reverse, then the adjoint of the
    initialisation.  The recompute of a segment runs on a second stream, overlapped with
    the adjoint steps of the segment after it (two sets of segment buffers).  Peak
    memory: about (steps / segment + 2 segment) checkpoints.  mu_0 enters as a
    constant."""

    @staticmethod
    def forward(ctx, phi0, theta, cfg, steps, muA0, muB0, segment=None):
        if cfg.precision not in ("fp32", "fp64") or cfg.gravity_mean_subtract:
            raise ValueError("the adjoint runs on fp32 or fp64 storage without gravity_mean_subtract")
        if cfg.collision != "BGK" or cfg.variable_density or cfg.kappa is not None or cfg.ncomp != 2:
            raise ValueError("the adjoint covers the paper's BGK Boussinesq model of the ternary fluid")
        steps = int(steps)
        seg = int(segment) if segment else max(1, math.isqrt(max(steps - 1, 0)) + 1)
        c = with_theta(cfg, theta.detach().double().cpu().tolist())
        sim = Simulation(c, phi0.detach(), muA0, muB0, device=phi0.device)
        ckpts = []
        n = 0
        while n < steps:
            ckpts.append(sim.save())
            k = min(seg, steps - n)
            sim.step(k)
            n += k
        phiT = sim.moments(["phi"])["phi"].reshape(phi0.shape).to(phi0.dtype)
        ctx.sim, ctx.ckpts, ctx.final = sim, ckpts, sim.save()
        ctx.seg, ctx.steps = seg, steps
        ctx.phi_shape, ctx.phi_dtype = phi0.shape, phi0.dtype
        ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
        return phiT

    @staticmethod
    def backward(ctx, grad_phiT):
        sim = ctx.sim
        dev = sim.device
        main = torch.cuda.current_stream(dev)
        side = torch.cuda.Stream(device=dev)        # default priority
        work = sim.adjoint_workspace()
        sim.adjoint_seed(ctx.final, grad_phiT.detach().to(torch.float64).contiguous(), work)
        nbytes = ctx.final.numel()
        width = min(ctx.seg, ctx.steps)
        nseg = len(ctx.ckpts)
        # two sets of segment buffers: the side stream recomputes segment s - 1 into one
        # while the adjoint steps of segment s run on the main stream from the other
        nbuf = 2 if nseg > 1 else 1
        seg_states = [[None] + [torch.empty(nbytes, dtype=torch.uint8, device=dev) for _ in range(width - 1)]
                      for _ in range(nbuf)]
        seg_phi = [[torch.empty(sim.cfg.nodes, dtype=sim.phi_dtype, device=dev) for _ in range(width)]
                   for _ in range(nbuf)]
        ready = [torch.cuda.Event() for _ in range(nbuf)]
        free = [torch.cuda.Event() for _ in range(nbuf)]
        side.wait_stream(main)                      # checkpoints and the seed are done

        def recompute(s, b):
            n0 = s * ctx.seg
            length = min(ctx.seg, ctx.steps - n0)
            states = [ctx.ckpts[s]] + seg_states[b][1:length]
            side.wait_event(free[b])                # the adjoint that read buffer b is done
            for j in range(1, length):
                sim.step_external(states[j - 1], states[j], seg_phi[b][j - 1], stream=side)
            sim.phase_field(states[length - 1], seg_phi[b][length - 1], stream=side)
            ready[b].record(side)
            return states

        pending = recompute(nseg - 1, 0)
        for i, s in enumerate(reversed(range(nseg))):
            b = i % nbuf
            states = pending
            if s > 0:
                pending = recompute(s - 1, (i + 1) % nbuf)
            main.wait_event(ready[b])
            for j in reversed(range(len(states))):
                sim.adjoint_step_phi(states[j], seg_phi[b][j], work)
            free[b].record(main)
        gphi0 = torch.empty(sim.cfg.shape, dtype=torch.float64, device=dev)
        sim.adjoint_init(work, gphi0)
        gth = sim.adjoint_theta(work)
        main.wait_stream(side)
        for t in ctx.ckpts + [x for buf in seg_states for x in buf[1:]] + [x for buf in seg_phi for x in buf]:
            t.record_stream(side)                   # used on the side stream as well
        ctx.sim = ctx.ckpts = ctx.final = None
        return (gphi0.reshape(ctx.phi_shape).to(ctx.phi_dtype), gth.to(ctx.theta_device, ctx.theta_dtype),
                None, None, None, None, None)


def phase_field_run(phi0, theta, cfg: LBMConfig, steps: int, muA0, muB0, segment=None):
    """Differentiable final phase field; see PhaseFieldRun."""
    return PhaseFieldRun.apply(phi0, theta, cfg, steps, muA0, muB0, segment)
