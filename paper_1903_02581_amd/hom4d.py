"""Python binding of libhom4d.so (ctypes): argument marshalling only.

Every step of the propagation runs in the HIP library; torch supplies device
memory (the state, adjoint and checkpoint buffers) and the stream.  The
binding fails loudly when the library has not been built.

C ABI: include/hom4d.h.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhom4d.so")

FP64 = 0
MIXED = 1
COULOMB_TABLE = 0
COULOMB_DIRECT = 1

STATUS = {0: "HOM4D_OK", -1: "HOM4D_EINVAL", -2: "HOM4D_EUNBOUND", -3: "HOM4D_ESTATE",
          -4: "HOM4D_ENOMEM", -5: "HOM4D_EHIP", -6: "HOM4D_ENONFINITE", -7: "HOM4D_ENORMDRIFT",
          -8: "HOM4D_ECONFIG", -9: "HOM4D_ECORRUPT"}

EXPORTS = ["hom4d_create", "hom4d_destroy", "hom4d_validate_cfg", "hom4d_state_bytes",
           "hom4d_bind_state", "hom4d_set_potential", "hom4d_set_field", "hom4d_init_state",
           "hom4d_load_state", "hom4d_store_state", "hom4d_checkpoint_bytes",
           "hom4d_save_checkpoint", "hom4d_load_checkpoint", "hom4d_step", "hom4d_observables",
           "hom4d_set_norm_tol", "hom4d_entanglement", "hom4d_gather_slice", "hom4d_marginal",
           "hom4d_conditional", "hom4d_edge_packet", "hom4d_grad_begin",
           "hom4d_grad_backward", "hom4d_grad_backward_noalloc", "hom4d_grad_end", "hom4d_run_pass", "hom4d_set_pass_plan",
           "hom4d_pass_plan", "hom4d_pass_timing", "hom4d_pass_times", "hom4d_strerror",
           "hom4d_last_error"]


class HomCfg(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("precision", c_int32),
                ("coulomb_mode", c_int32), ("lx_nm", c_double), ("ly_nm", c_double),
                ("mstar_rel", c_double), ("eps_r", c_double), ("b_tesla", c_double),
                ("dt_fs", c_double), ("soft_nm", c_double), ("coulomb_c", c_double),
                ("screen_nm", c_double)]


class HomObs(ctypes.Structure):
    _fields_ = [("norm", c_double), ("p_tt", c_double), ("p_tb", c_double), ("p_bt", c_double),
                ("p_bb", c_double), ("p_b", c_double), ("p_ab", c_double), ("step", c_int64)]


class Hom4dError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} ({detail})")
        self.status = status


_LIB = None


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load libhom4d.so; raise if it has not been built (no fallback path exists)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_1903_02581_amd.build` "
                           "or __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    vp, dp, i32p = c_void_p, POINTER(c_double), POINTER(c_int32)
    sig = {
        "hom4d_create": ([POINTER(HomCfg), vp, POINTER(vp)], c_int),
        "hom4d_destroy": ([vp], c_int),
        "hom4d_validate_cfg": ([POINTER(HomCfg)], c_int),
        "hom4d_state_bytes": ([POINTER(HomCfg)], c_size_t),
        "hom4d_bind_state": ([vp, vp], c_int),
        "hom4d_set_potential": ([vp, dp], c_int),
        "hom4d_set_field": ([vp, c_double], c_int),
        "hom4d_init_state": ([vp, dp, dp, c_int32], c_int),
        "hom4d_load_state": ([vp, dp], c_int),
        "hom4d_store_state": ([vp, dp], c_int),
        "hom4d_checkpoint_bytes": ([vp], c_size_t),
        "hom4d_save_checkpoint": ([vp, vp, c_size_t], c_int),
        "hom4d_load_checkpoint": ([vp, vp, c_size_t], c_int),
        "hom4d_step": ([vp, c_int64], c_int),
        "hom4d_observables": ([vp, dp, POINTER(HomObs)], c_int),
        "hom4d_set_norm_tol": ([vp, c_double], c_int),
        "hom4d_entanglement": ([vp, i32p, c_int32, c_int32, i32p, c_int32, c_int32, dp], c_int),
        "hom4d_gather_slice": ([vp, i32p, c_int32, c_int32, i32p, c_int32, c_int32, dp], c_int),
        "hom4d_marginal": ([vp, dp], c_int),
        "hom4d_conditional": ([vp, c_int32, c_int32, dp], c_int),
        "hom4d_edge_packet": ([vp, dp, c_double, c_double, c_int32, c_double, dp, dp], c_int),
        "hom4d_grad_begin": ([vp, c_int32, vp, c_size_t], c_int),
        "hom4d_grad_backward": ([vp, dp, dp, vp, dp, dp, dp], c_int),
        "hom4d_grad_backward_noalloc": ([vp, dp, dp, vp, dp, dp, dp], c_int),
        "hom4d_grad_end": ([vp], c_int),
        "hom4d_run_pass": ([vp, c_int32, c_int32], c_int),
        "hom4d_set_pass_plan": ([vp, c_int32], c_int),
        "hom4d_pass_plan": ([vp], c_int),
        "hom4d_pass_timing": ([vp, c_int32], c_int),
        "hom4d_pass_times": ([vp, dp, POINTER(c_int64)], c_int),
        "hom4d_strerror": ([c_int], ctypes.c_char_p),
        "hom4d_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if path is None:
        _LIB = lib
    return lib


def make_cfg(nx, ny, lx, ly, *, dt_fs, b_tesla, mstar_rel=0.067, eps_r=12.9, soft_nm=2.0,
             coulomb_c=1.0, screen_nm=0.0, precision="fp64", coulomb_mode="table") -> HomCfg:
    prec = {"fp64": FP64, "mixed": MIXED}[precision]
    mode = {"table": COULOMB_TABLE, "direct": COULOMB_DIRECT}[coulomb_mode]
    return HomCfg(int(nx), int(ny), prec, mode, float(lx), float(ly), float(mstar_rel),
                  float(eps_r), float(b_tesla), float(dt_fs), float(soft_nm), float(coulomb_c),
                  float(screen_nm))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def _c128(a, shape) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).reshape(shape)
    return a


class Propagator:
    """One two-electron state on one GPU, advanced by the HIP library.

    The state is a torch tensor of (nx*ny)^2 complex values (complex128 for
    precision='fp64', complex64 for 'mixed') in the canonical [x1][y1][x2][y2]
    order; the library holds its pointer.
    """

    def __init__(self, nx, ny, lx, ly, *, dt_fs, b_tesla, mstar_rel=0.067, eps_r=12.9,
                 soft_nm=2.0, coulomb_c=1.0, screen_nm=0.0, precision="fp64",
                 coulomb_mode="table", device="cuda:0"):
        import torch
        self.lib = load_library()
        self.cfg = make_cfg(nx, ny, lx, ly, dt_fs=dt_fs, b_tesla=b_tesla, mstar_rel=mstar_rel,
                            eps_r=eps_r, soft_nm=soft_nm, coulomb_c=coulomb_c,
                            screen_nm=screen_nm, precision=precision, coulomb_mode=coulomb_mode)
        self.nx, self.ny = int(nx), int(ny)
        self.precision = precision
        self.device = torch.device(device)
        self._check(self.lib.hom4d_validate_cfg(byref(self.cfg)), "validate_cfg")
        self.state_bytes = int(self.lib.hom4d_state_bytes(byref(self.cfg)))
        dtype = torch.complex128 if precision == "fp64" else torch.complex64
        n = (self.nx * self.ny) ** 2
        self.psi = torch.empty(n, dtype=dtype, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.h = c_void_p()
        self._check(self.lib.hom4d_create(byref(self.cfg), c_void_p(self.stream.cuda_stream),
                                          byref(self.h)), "create")
        self._check(self.lib.hom4d_bind_state(self.h, c_void_p(self.psi.data_ptr())), "bind_state")
        self._pool = None
        self._lam = None

    @classmethod
    def from_workload(cls, w, precision="fp64", coulomb_mode="table", device="cuda:0",
                      **overrides):
        kw = dict(dt_fs=w.dt_fs, b_tesla=w.b_tesla, mstar_rel=w.mstar_rel, eps_r=w.eps_r,
                  soft_nm=w.soft_nm, coulomb_c=w.coulomb_c, precision=precision,
                  coulomb_mode=coulomb_mode, device=device)
        kw.update(overrides)
        p = cls(w.nx, w.ny, w.lx, w.ly, **kw)
        p.set_potential(w.v_table)
        p.init_state(w.psi_a, w.psi_b, w.sym)
        return p

    # ------------------------------------------------------------------ plumbing
    def _check(self, rc: int, where: str):
        if rc != 0:
            detail = self.lib.hom4d_last_error().decode(errors="replace")
            raise Hom4dError(rc, where, detail)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.hom4d_destroy(self.h)
            self.h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------- state
    def set_potential(self, v_mev):
        v = np.ascontiguousarray(np.asarray(v_mev, dtype=np.float64)).reshape(self.nx, self.ny)
        self._check(self.lib.hom4d_set_potential(self.h, _dptr(v)), "set_potential")

    def set_field(self, b_tesla: float):
        self._check(self.lib.hom4d_set_field(self.h, float(b_tesla)), "set_field")

    def init_state(self, psi_a, psi_b, sym: int = -1):
        a = _c128(psi_a, (self.nx, self.ny))
        b = _c128(psi_b, (self.nx, self.ny))
        self._check(self.lib.hom4d_init_state(self.h, _dptr(a.view(np.float64)),
                                              _dptr(b.view(np.float64)), int(sym)), "init_state")

    def load_state(self, psi4d):
        n = self.nx * self.ny
        a = _c128(psi4d, (n * n,))
        self._check(self.lib.hom4d_load_state(self.h, _dptr(a.view(np.float64))), "load_state")

    def store_state(self) -> np.ndarray:
        n = self.nx * self.ny
        out = np.empty(n * n, dtype=np.complex128)
        self._check(self.lib.hom4d_store_state(self.h, _dptr(out.view(np.float64))), "store_state")
        return out.reshape(self.nx, self.ny, self.nx, self.ny)

    def save_checkpoint(self) -> np.ndarray:
        """Checkpoint image of the state (header + state bits) as a uint8 array."""
        nb = int(self.lib.hom4d_checkpoint_bytes(self.h))
        buf = np.empty(nb, dtype=np.uint8)
        self._check(self.lib.hom4d_save_checkpoint(self.h, c_void_p(buf.ctypes.data), nb),
                    "save_checkpoint")
        return buf

    def load_checkpoint(self, image):
        """Restore a checkpoint image (state and step count); the library checks it."""
        buf = np.ascontiguousarray(np.asarray(image, dtype=np.uint8)).ravel()
        self._check(self.lib.hom4d_load_checkpoint(self.h, c_void_p(buf.ctypes.data), buf.size),
                    "load_checkpoint")

    def step(self, n: int = 1):
        self._check(self.lib.hom4d_step(self.h, int(n)), "step")

    def synchronize(self):
        self.stream.synchronize()

    # ------------------------------------------------------------- observables
    def observables(self, w_top, check: bool = False) -> dict:
        w = np.ascontiguousarray(np.asarray(w_top, dtype=np.float64)).reshape(self.nx, self.ny)
        o = HomObs()
        rc = self.lib.hom4d_observables(self.h, _dptr(w), byref(o))
        if rc != 0 and (check or rc not in (-6, -7)):
            self._check(rc, "observables")
        return dict(norm=o.norm, p_tt=o.p_tt, p_tb=o.p_tb, p_bt=o.p_bt, p_bb=o.p_bb, p_b=o.p_b,
                    p_ab=o.p_ab, step=int(o.step), status=int(rc))

    def set_norm_tol(self, tol: float):
        self._check(self.lib.hom4d_set_norm_tol(self.h, float(tol)), "set_norm_tol")

    def _slice_args(self, ix1, ix2):
        a = np.ascontiguousarray(np.asarray(ix1, dtype=np.int32))
        b = np.ascontiguousarray(np.asarray(ix2, dtype=np.int32))
        return a, b

    def entanglement(self, ix1, jy1: int, ix2, jy2: int) -> float:
        a, b = self._slice_args(ix1, ix2)
        s = c_double()
        self._check(self.lib.hom4d_entanglement(self.h, a.ctypes.data_as(POINTER(c_int32)),
                                                len(a), int(jy1),
                                                b.ctypes.data_as(POINTER(c_int32)), len(b),
                                                int(jy2), byref(s)), "entanglement")
        return float(s.value)

    def gather_slice(self, ix1, jy1: int, ix2, jy2: int) -> np.ndarray:
        a, b = self._slice_args(ix1, ix2)
        out = np.empty((len(a), len(b)), dtype=np.complex128)
        self._check(self.lib.hom4d_gather_slice(self.h, a.ctypes.data_as(POINTER(c_int32)),
                                                len(a), int(jy1),
                                                b.ctypes.data_as(POINTER(c_int32)), len(b),
                                                int(jy2), _dptr(out.view(np.float64))),
                    "gather_slice")
        return out

    def marginal(self) -> np.ndarray:
        """P(x1, y1) = sum over (x2, y2) of |Psi|^2, shape [nx, ny]."""
        out = np.empty((self.nx, self.ny), dtype=np.float64)
        self._check(self.lib.hom4d_marginal(self.h, _dptr(out)), "marginal")
        return out

    def conditional(self, ix2: int, jy2: int) -> np.ndarray:
        """|Psi(x1, y1, ix2, jy2)|^2 over (x1, y1), shape [nx, ny]."""
        out = np.empty((self.nx, self.ny), dtype=np.float64)
        self._check(self.lib.hom4d_conditional(self.h, int(ix2), int(jy2), _dptr(out)),
                    "conditional")
        return out

    def edge_packet(self, v_col, sigma_x: float, xc: float, top: bool, e_above_lll: float):
        """One electron's Gaussian edge-state packet on this grid, built on the GPU
        (Eq. (H_effective), Eq. (singlepwp)): shape [nx, ny] complex128, and
        dict(k0, e1_k0, target)."""
        v = np.ascontiguousarray(v_col, dtype=np.float64)
        if v.shape != (self.ny,):
            raise ValueError(f"v_col must have shape ({self.ny},)")
        out = np.empty((self.nx, self.ny), dtype=np.complex128)
        info = np.zeros(3, dtype=np.float64)
        self._check(self.lib.hom4d_edge_packet(self.h, _dptr(v), float(sigma_x), float(xc),
                                               1 if top else 0, float(e_above_lll),
                                               _dptr(out.view(np.float64)), _dptr(info)),
                    "edge_packet")
        return out, dict(k0=float(info[0]), e1_k0=float(info[1]), target=float(info[2]))

    # ---------------------------------------------------------------- adjoint
    def grad_begin(self, ckpt_every: int, steps: int):
        """Open a recording for `steps` forward steps with a checkpoint every ckpt_every."""
        import torch
        slots = int(steps) // int(ckpt_every) + 1
        nb = slots * self.state_bytes
        if self._pool is None or self._pool.numel() < nb:
            self._pool = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self._check(self.lib.hom4d_grad_begin(self.h, int(ckpt_every),
                                              c_void_p(self._pool.data_ptr()), nb), "grad_begin")

    def grad_backward(self, w_top, coeffs=(1.0, 0.0, 0.0, 1.0), noalloc: bool = False):
        """Reverse sweep: returns (L, dL/dV [nx, ny], dL/dB).  noalloc: through
        hom4d_grad_backward_noalloc (fixed device scratch, no allocation in the call)."""
        import torch
        w = np.ascontiguousarray(np.asarray(w_top, dtype=np.float64)).reshape(self.nx, self.ny)
        cf = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
        if self._lam is None:
            self._lam = torch.empty_like(self.psi)
        loss = c_double()
        dldb = c_double()
        dldv = np.empty((self.nx, self.ny), dtype=np.float64)
        fn = self.lib.hom4d_grad_backward_noalloc if noalloc else self.lib.hom4d_grad_backward
        self._check(fn(self.h, _dptr(w), _dptr(cf), c_void_p(self._lam.data_ptr()), byref(loss),
                       _dptr(dldv), byref(dldb)),
                    "grad_backward_noalloc" if noalloc else "grad_backward")
        return float(loss.value), dldv, float(dldb.value)

    def set_pass_plan(self, plan: int):
        """0: fused three-pass steps where built (default); 1: four per-axis passes."""
        self._check(self.lib.hom4d_set_pass_plan(self.h, int(plan)), "set_pass_plan")

    @property
    def passes_per_step(self) -> int:
        rc = self.lib.hom4d_pass_plan(self.h)
        if rc < 0:
            self._check(rc, "pass_plan")
        return int(rc)

    PASS_KINDS = ("x1", "y1", "x2", "y2", "plane")

    def pass_timing(self, enable: bool):
        """Bracket every pass kernel launched from now on by a HIP event pair (measurement)."""
        self._check(self.lib.hom4d_pass_timing(self.h, 1 if enable else 0), "pass_timing")

    def pass_times(self) -> dict:
        """{kind: (summed seconds, launches)} of the launches recorded since pass_timing(True)."""
        ms = np.zeros(5, dtype=np.float64)
        cnt = np.zeros(5, dtype=np.int64)
        self._check(self.lib.hom4d_pass_times(self.h, _dptr(ms), cnt.ctypes.data_as(POINTER(c_int64))),
                    "pass_times")
        return {k: (float(ms[i]) * 1e-3, int(cnt[i])) for i, k in enumerate(self.PASS_KINDS) if cnt[i]}

    def run_pass(self, axis: int, reps: int = 1):
        """Launch one of the four fused pass kernels reps times (measurement only)."""
        self._check(self.lib.hom4d_run_pass(self.h, int(axis), int(reps)), "run_pass")

    def grad_end(self):
        self._check(self.lib.hom4d_grad_end(self.h), "grad_end")
