"""Thin ctypes binding of libdgweno.so (include/dgweno.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Device buffers are torch tensors (float64, contiguous, on the GPU);
work is queued on the current torch stream.  If the library is missing the
import fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgweno.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EDEVICE, DG_ENONFINITE, DG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
DG_FLUX_EULER = 3
FLUX_LINADV, FLUX_BURGERS = 0, 1
MODE_DG, MODE_LO, MODE_WENO = 0, 1, 2


class DGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dgweno error {code}: {msg}")
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double),
        ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
        ("p", ctypes.c_int32), ("flux", ctypes.c_int32),
        ("vel_x", ctypes.c_double), ("vel_y", ctypes.c_double),
        ("omega", ctypes.c_double), ("rot_cx", ctypes.c_double), ("rot_cy", ctypes.c_double),
        ("bc_value", ctypes.c_double),
        ("mode", ctypes.c_int32),
        ("q", ctypes.c_double), ("b", ctypes.c_double), ("w_nb", ctypes.c_double),
        ("weno_eps", ctypes.c_double), ("weno_pow", ctypes.c_double),
        ("lambda_override", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("zhao_theta", ctypes.c_double),
        ("rk_order", ctypes.c_int32),
        ("bc_kind", ctypes.c_int32),
        ("quad_vol", ctypes.c_int32), ("quad_face", ctypes.c_int32), ("quad_proj", ctypes.c_int32),
        ("cfl_mode", ctypes.c_int32),
        ("check_finite", ctypes.c_int32),
        ("device", ctypes.c_int32),
    ]


EXPORTS = {
    # name: (restype, argtypes)
    "dg_default_desc": (None, [ctypes.POINTER(MeshDesc)]),
    "dg_init_mesh": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "dg_destroy": (None, [ctypes.c_void_p]),
    "dg_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "dg_proj_nodes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "dg_project_ic": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "dg_rhs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "dg_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]),
    "dg_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32]),
    "dg_stable_dt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_double)]),
    "dg_check_finite": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "dg_set_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "dg_set_fused": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "dg_get_fused": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "dg_set_step_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "dg_get_step_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "dg_get_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32)]),
    "dg_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "dg_set_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "dg_get_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "dg_stream_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "dg_last_error": (ctypes.c_char_p, []),
    "dg_validate_desc": (ctypes.c_int, [ctypes.POINTER(MeshDesc)]),
    "dg_rhs_vjp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "dg_step_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "dg_adjoint_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "dg_adjoint_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "dg_revolve_stats": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "dg_batch_create": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "dg_batch_destroy": (None, [ctypes.c_void_p]),
    "dg_batch_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "dg_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "dg_batch_run_sequential": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "dg_batch_num_classes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "dg_batch_set_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32]),
    "dg_batch_get_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "dg_batch_set_branches": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "dg_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_char_p, ctypes.c_int32]),
    "dg_step_static": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.c_void_p, ctypes.c_double,
                                      ctypes.c_double]),
    "dg_run_signature": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                                        ctypes.c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the library (after torch, so one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2309_12019_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != DG_OK:
        raise DGError(rc, _lib.dg_last_error().decode())


def _ptr(t: Optional[torch.Tensor], n: int, name: str):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 GPU tensor")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def desc_from_fields(f: dict) -> MeshDesc:
    lib = load()
    d = MeshDesc()
    lib.dg_default_desc(ctypes.byref(d))
    d.dim, d.nx, d.ny = f["dim"], f["nx"], f.get("ny", 1)
    d.x0, d.x1, d.y0, d.y1 = f["x0"], f["x1"], f["y0"], f["y1"]
    d.periodic_x, d.periodic_y = int(f["periodic_x"]), int(f["periodic_y"])
    d.p, d.flux = f["p"], f["flux"]
    d.vel_x, d.vel_y = f["vx"], f["vy"]
    d.omega, d.rot_cx, d.rot_cy = f["omega"], f["cx"], f["cy"]
    d.bc_value = f["bc_value"]
    d.mode = f["mode"]
    d.q, d.b, d.w_nb = f["q"], f["b"], f["w_nb"]
    d.weno_eps, d.weno_pow = f["eps"], f["r"]
    d.lambda_override = f["lambda_override"]
    d.zhao_theta = f.get("theta", 1.0)
    d.rk_order = f.get("rk_order", 3)
    d.bc_kind = f.get("bc_kind", 0)
    d.quad_vol, d.quad_face, d.quad_proj = f.get("quad_vol", 0), f.get("quad_face", 0), f.get("quad_proj", 0)
    d.cfl_mode = f.get("cfl_mode", 0)
    d.check_finite = int(f.get("check_finite", 0))
    return d


class DG:
    """One discretised problem on the current GPU (owns a dg_ctx)."""

    def __init__(self, desc: MeshDesc, stream: Optional[torch.cuda.Stream] = None):
        lib = load()
        self.lib = lib
        st = stream if stream is not None else torch.cuda.current_stream()
        desc.stream = ctypes.c_void_p(st.cuda_stream)
        self.desc = desc
        h = ctypes.c_void_p()
        _check(lib.dg_init_mesh(ctypes.byref(desc), ctypes.byref(h)))
        self.h = h
        nc, nl, nq = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.dg_sizes(h, ctypes.byref(nc), ctypes.byref(nl), ctypes.byref(nq)))
        self.ncells, self.nloc, self.nproj = nc.value, nl.value, nq.value
        self.ncomp = 3 if desc.flux == DG_FLUX_EULER else 1   # values per projection node
        self.device = torch.device("cuda", desc.device if desc.device >= 0 else torch.cuda.current_device())

    @classmethod
    def from_workload(cls, w, stream=None) -> "DG":
        return cls(desc_from_fields(w.fields()), stream)

    def close(self):
        if getattr(self, "h", None):
            self.lib.dg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self) -> Tuple[int, int]:
        return (self.ncells, self.nloc)

    def empty(self) -> torch.Tensor:
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    def proj_nodes(self) -> np.ndarray:
        dim = self.desc.dim
        out = np.empty((self.ncells, self.nproj, dim), dtype=np.float64)
        _check(self.lib.dg_proj_nodes(self.h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def project_ic(self, u_at_nodes: torch.Tensor, U: Optional[torch.Tensor] = None) -> torch.Tensor:
        U = self.empty() if U is None else U
        nvals = self.ncells * self.nproj * self.ncomp
        _check(self.lib.dg_project_ic(self.h, _ptr(u_at_nodes, nvals, "u_at_nodes"),
                                      _ptr(U, self.ncells * self.nloc, "U")))
        return U

    def rhs(self, U: torch.Tensor, out: Optional[torch.Tensor] = None, with_gamma: bool = False):
        out = self.empty() if out is None else out
        gam = torch.empty(self.ncells, dtype=torch.float64, device=self.device) if with_gamma else None
        n = self.ncells * self.nloc
        _check(self.lib.dg_rhs(self.h, _ptr(U, n, "U"), _ptr(out, n, "dUdt"), _ptr(gam, self.ncells, "gamma")))
        return (out, gam) if with_gamma else out

    def step(self, U: torch.Tensor, dt: float) -> torch.Tensor:
        _check(self.lib.dg_step(self.h, _ptr(U, self.ncells * self.nloc, "U"), float(dt)))
        return U

    def run(self, U: torch.Tensor, dt: float, nsteps: int) -> torch.Tensor:
        _check(self.lib.dg_run(self.h, _ptr(U, self.ncells * self.nloc, "U"), float(dt), int(nsteps)))
        return U

    def run_signature(self, U: torch.Tensor, dt: float, nsteps: int,
                      sig: Optional[torch.Tensor] = None) -> torch.Tensor:
        """dg_run_signature: nsteps SSP-RK3 steps of U in place (as run) and
        the branch records, an int32 tensor [3, n_cells] (sensor, lambda_e,
        LLF hashes) holding the uint32 bits."""
        if sig is None:
            sig = torch.empty((3, self.ncells), dtype=torch.int32, device=self.device)
        if not (sig.is_cuda and sig.dtype == torch.int32 and sig.is_contiguous() and sig.numel() == 3 * self.ncells):
            raise ValueError("sig must be a contiguous int32 GPU tensor of 3 * n_cells entries")
        _check(self.lib.dg_run_signature(self.h, _ptr(U, self.ncells * self.nloc, "U"), float(dt), int(nsteps),
                                         ctypes.c_void_p(sig.data_ptr())))
        return sig

    def set_time(self, t: float) -> None:
        """Set the context's clock (dg_set_time): the time of the state the
        next dg_step / dg_run / dg_rhs sees."""
        _check(self.lib.dg_set_time(self.h, float(t)))

    def time(self) -> float:
        t = ctypes.c_double()
        _check(self.lib.dg_get_time(self.h, ctypes.byref(t)))
        return t.value

    def stable_dt(self, U: torch.Tensor, cfl: float) -> float:
        out = ctypes.c_double()
        _check(self.lib.dg_stable_dt(self.h, _ptr(U, self.ncells * self.nloc, "U"), float(cfl),
                                     ctypes.byref(out)))
        return out.value

    def count_nonfinite(self, U: torch.Tensor) -> int:
        cnt = ctypes.c_int64()
        rc = self.lib.dg_check_finite(self.h, _ptr(U, self.ncells * self.nloc, "U"), ctypes.byref(cnt))
        if rc not in (DG_OK, DG_ENONFINITE):
            _check(rc)
        return cnt.value

    def rhs_vjp(self, U: torch.Tensor, v: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.empty() if out is None else out
        n = self.ncells * self.nloc
        _check(self.lib.dg_rhs_vjp(self.h, _ptr(U, n, "U"), _ptr(v, n, "v"), _ptr(out, n, "out")))
        return out

    def step_adjoint(self, Un: torch.Tensor, dt: float, lam_out: torch.Tensor,
                     lam_in: Optional[torch.Tensor] = None) -> torch.Tensor:
        lam_in = self.empty() if lam_in is None else lam_in
        n = self.ncells * self.nloc
        _check(self.lib.dg_step_adjoint(self.h, _ptr(Un, n, "Un"), float(dt), _ptr(lam_out, n, "lam_out"),
                                        _ptr(lam_in, n, "lam_in")))
        return lam_in

    def checkpoints(self, nsnaps: int) -> torch.Tensor:
        return torch.empty((nsnaps + 2) * self.ncells * self.nloc, dtype=torch.float64, device=self.device)

    def stage_checkpoints(self, nsteps: int) -> torch.Tensor:
        return torch.empty(2 * nsteps * self.ncells * self.nloc, dtype=torch.float64, device=self.device)

    def adjoint_forward(self, U0, dt, nsteps, nsnaps, ckpt, UT=None, stages=None) -> torch.Tensor:
        UT = self.empty() if UT is None else UT
        n = self.ncells * self.nloc
        _check(self.lib.dg_adjoint_forward(self.h, _ptr(U0, n, "U0"), _ptr(UT, n, "UT"), float(dt), int(nsteps),
                                           int(nsnaps), _ptr(ckpt, (nsnaps + 2) * n, "ckpt"),
                                           _ptr(stages, 2 * nsteps * n, "stages")))
        return UT

    def adjoint_backward(self, dt, nsteps, nsnaps, ckpt, lam, stages=None) -> torch.Tensor:
        n = self.ncells * self.nloc
        _check(self.lib.dg_adjoint_backward(self.h, float(dt), int(nsteps), int(nsnaps),
                                            _ptr(ckpt, (nsnaps + 2) * n, "ckpt"),
                                            _ptr(stages, 2 * nsteps * n, "stages"), _ptr(lam, n, "lam")))
        return lam

    def set_tile(self, tx: int, ty: int = 1) -> None:
        _check(self.lib.dg_set_tile(self.h, int(tx), int(ty)))

    def set_fused(self, mode: int) -> None:
        """Fused step kernel: -1 automatic, 0 off, 1 on (dg_set_fused); 0 also
        gives the adjoint separate launches for its two passes."""
        _check(self.lib.dg_set_fused(self.h, int(mode)))

    def fused(self) -> bool:
        a = ctypes.c_int32()
        _check(self.lib.dg_get_fused(self.h, ctypes.byref(a)))
        return bool(a.value)

    def tile(self) -> Tuple[int, int]:
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.dg_get_tile(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_step_tile(self, tx: int, ty: int = 1) -> None:
        """Fused step kernel's tile (dg_set_step_tile): 2D 16x16 or 16x8."""
        _check(self.lib.dg_set_step_tile(self.h, int(tx), int(ty)))

    def step_tile(self) -> Tuple[int, int]:
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.dg_get_step_tile(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def initial_state(self, w, on_device: bool = False) -> torch.Tensor:
        """Project the workload's initial data with the library's projection.
        The data are evaluated at the projection nodes on the host (numpy), or
        with on_device on the GPU (torch; the same formulas, other rounding of
        cos and sqrt), which large meshes need to start in seconds."""
        pts = self.proj_nodes()
        if on_device:
            vals = w.eval_ic(torch.from_numpy(pts).to(self.device))
        else:
            vals = torch.from_numpy(np.ascontiguousarray(w.eval_ic(pts))).to(self.device)
        return self.project_ic(vals.reshape(-1).contiguous())


class Batch:
    """Many independent problems advanced together (dg_batch_*).

    The states live in one arena tensor; `views()` returns per-problem views
    of shape (n_cells, n_loc)."""

    def __init__(self, descs, stream: Optional[torch.cuda.Stream] = None):
        lib = load()
        self.lib = lib
        st = stream if stream is not None else torch.cuda.current_stream()
        arr = (MeshDesc * len(descs))(*descs)
        for d in arr:
            d.stream = ctypes.c_void_p(st.cuda_stream)
        self._descs = arr
        h = ctypes.c_void_p()
        _check(lib.dg_batch_create(arr, len(descs), ctypes.byref(h)))
        self.h = h
        self.count = len(descs)
        offs = np.zeros(self.count + 1, dtype=np.int64)
        tot = ctypes.c_int64()
        _check(lib.dg_batch_layout(h, offs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(tot)))
        self.offsets = offs
        self.total = tot.value
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.nloc = [(d.p + 1) ** d.dim for d in descs]

    @classmethod
    def from_workloads(cls, ws, stream=None) -> "Batch":
        return cls([desc_from_fields(w.fields()) for w in ws], stream)

    def close(self):
        if getattr(self, "h", None):
            self.lib.dg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self) -> torch.Tensor:
        return torch.empty(self.total, dtype=torch.float64, device=self.device)

    def views(self, arena: torch.Tensor):
        return [arena[self.offsets[i]:self.offsets[i + 1]].view(-1, self.nloc[i]) for i in range(self.count)]

    def _dts(self, dts) -> np.ndarray:
        a = np.ascontiguousarray(np.asarray(dts, dtype=np.float64))
        if a.shape != (self.count,):
            raise ValueError(f"need {self.count} time steps")
        return a

    def run(self, arena: torch.Tensor, dts, nsteps: int) -> torch.Tensor:
        a = self._dts(dts)
        _check(self.lib.dg_batch_run(self.h, _ptr(arena, self.total, "arena"),
                                     a.ctypes.data_as(ctypes.c_void_p), int(nsteps)))
        return arena

    def run_sequential(self, arena: torch.Tensor, dts, nsteps: int) -> torch.Tensor:
        a = self._dts(dts)
        _check(self.lib.dg_batch_run_sequential(self.h, _ptr(arena, self.total, "arena"),
                                                a.ctypes.data_as(ctypes.c_void_p), int(nsteps)))
        return arena

    def tune(self, arena: torch.Tensor, dts, reps: int = 5) -> str:
        a = self._dts(dts)
        buf = ctypes.create_string_buffer(16384)
        _check(self.lib.dg_batch_tune(self.h, _ptr(arena, self.total, "arena"),
                                      a.ctypes.data_as(ctypes.c_void_p), int(reps), buf, len(buf)))
        return buf.value.decode()

    def num_classes(self) -> int:
        n = ctypes.c_int32()
        _check(self.lib.dg_batch_num_classes(self.h, ctypes.byref(n)))
        return n.value

    def schedule(self, cls: int):
        info = np.zeros(10, dtype=np.int32)
        _check(self.lib.dg_batch_get_schedule(self.h, int(cls), info.ctypes.data_as(ctypes.c_void_p)))
        keys = ("dim", "p", "flux", "mode", "problems", "tx", "ty", "grid_per_cu", "order", "branch")
        return dict(zip(keys, info.tolist()))

    def set_schedule(self, cls: int, tx: int, ty: int, grid_per_cu: int, order: int) -> None:
        _check(self.lib.dg_batch_set_schedule(self.h, int(cls), int(tx), int(ty), int(grid_per_cu), int(order)))

    def set_branches(self, n: int) -> None:
        _check(self.lib.dg_batch_set_branches(self.h, int(n)))


# coefficients one dg_step_static call can hold (its static stage buffers)
STATIC_STAGE_DOUBLES = 1 << 20


def step_static(desc: "MeshDesc", U: torch.Tensor, dt: float, t: float = 0.0,
                stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """dg_step_static: one SSP step of U (contiguous float64, [n_cells, n_loc])
    in place, with no context and no allocation (stage states in the
    library's static device array), queued on `stream` (default: torch's
    current stream).  The descriptor's own stream field is overwritten."""
    lib = load()
    st = stream if stream is not None else torch.cuda.current_stream()
    d = MeshDesc.from_buffer_copy(desc)
    d.stream = ctypes.c_void_p(st.cuda_stream)
    if not (U.is_cuda and U.dtype == torch.float64 and U.is_contiguous()):
        raise ValueError("U must be a contiguous float64 GPU tensor")
    _check(lib.dg_step_static(ctypes.byref(d), ctypes.c_void_p(U.data_ptr()), float(dt), float(t)))
    return U


def stream_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """dst = src by the library's streaming copy kernel (dg_stream_copy) on
    the current stream: the measured bandwidth ceiling."""
    lib = load()
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in size")
    n = src.numel()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(lib.dg_stream_copy(_ptr(src, n, "src"), _ptr(dst, n, "dst"), n, stream))


def revolve_stats(nsteps: int, nsnaps: int) -> dict:
    """Host-only statistics of the checkpoint schedule (no GPU needed)."""
    lib = load()
    st = np.zeros(6, dtype=np.int64)
    _check(lib.dg_revolve_stats(int(nsteps), int(nsnaps), st.ctypes.data_as(ctypes.c_void_p)))
    keys = ("forward_steps", "recomputed_steps", "stores", "adjoint_steps", "max_slot", "actions")
    return dict(zip(keys, st.tolist()))


class DGRunFunction(torch.autograd.Function):
    """U^N = run(U^0) as a differentiable op: the forward stores checkpoints,
    the backward runs the hand-written discrete adjoint over them."""

    @staticmethod
    def forward(ctx, U0, dg: "DG", dt: float, nsteps: int, nsnaps: int, keep_stages: bool):
        ckpt = dg.checkpoints(nsnaps)
        stages = dg.stage_checkpoints(nsteps) if keep_stages else None
        UT = dg.adjoint_forward(U0.detach().contiguous(), dt, nsteps, nsnaps, ckpt, stages=stages)
        ctx.dg, ctx.dt, ctx.nsteps, ctx.nsnaps, ctx.ckpt, ctx.stages = dg, dt, nsteps, nsnaps, ckpt, stages
        return UT

    @staticmethod
    def backward(ctx, gUT):
        lam = gUT.detach().clone().contiguous()
        ctx.dg.adjoint_backward(ctx.dt, ctx.nsteps, ctx.nsnaps, ctx.ckpt, lam, stages=ctx.stages)
        ctx.ckpt = ctx.stages = None
        return lam, None, None, None, None, None


def run_differentiable(dg: "DG", U0: torch.Tensor, dt: float, nsteps: int, nsnaps: Optional[int] = None,
                       keep_stages: bool = False):
    """nsteps SSP-RK3 steps of U0 with gradients through torch.autograd
    (binomial checkpointing with nsnaps stored states; keep_stages also stores
    the RK stage states of every step the forward sweep advances)."""
    return DGRunFunction.apply(U0, dg, dt, nsteps, nsteps if nsnaps is None else nsnaps, keep_stages)
