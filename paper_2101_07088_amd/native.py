"""ctypes binding of libdpse.so; names follow include/dpse.h."""
from __future__ import annotations

import ctypes
import enum
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdpse.so")

DPSE_FP64 = 0
DPSE_MIXED = 1
DPSE_GAUGE_NONE = 1
DPSE_KMAX_GT = 2
DPSE_UNIFORM_FAST = 4
DPSE_ONE_JUMP = 8
DPSE_TRIPLY = 16
DPSE_DETERMINISTIC = 32

_STATUS = {
    0: "DPSE_OK", 1: "DPSE_EINVAL", 2: "DPSE_ENOMEM", 3: "DPSE_EHIP", 4: "DPSE_ENONNEUTRAL",
    5: "DPSE_EOUTSIDE", 6: "DPSE_ECONSTRAINT", 7: "DPSE_ETOOMANY", 8: "DPSE_ESCRATCH",
}
DPSE_ESCRATCH = 8
STATIC_SCRATCH_BYTES = 64 << 20   # the static workspace array of dpse_solve_static, per device


class Stage(enum.IntEnum):
    F_I = 0
    F_O = 1
    FH_I = 2
    PSI = 3
    PSIZ = 4
    GRIDS = 5
    FAR = 6
    NEAR = 7
    SCALARS = 8
    WALL_HAT = 9
    WALL_PHI = 10
    WALL_SCALARS = 11
    FH_O = 12


class DpseError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_STATUS.get(status, status)} ({_lib().dpse_status_string(status).decode()})")


class _Params(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_double), ("Ly", ctypes.c_double), ("H", ctypes.c_double),
                ("eps", ctypes.c_double), ("eps_bottom", ctypes.c_double), ("eps_top", ctypes.c_double),
                ("xi", ctypes.c_double), ("g_w", ctypes.c_double),
                ("Nx", ctypes.c_int32), ("Ny", ctypes.c_int32), ("Nz", ctypes.c_int32),
                ("support", ctypes.c_int32), ("r_cut", ctypes.c_double), ("delta", ctypes.c_double),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("g_t", ctypes.c_double), ("H_E", ctypes.c_double),
                ("n_sigma", ctypes.c_double), ("z_lo", ctypes.c_double), ("z_hi", ctypes.c_double),
                ("r_cut", ctypes.c_double), ("xi_e", ctypes.c_double), ("support", ctypes.c_int32),
                ("n_modes", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64),
                ("max_n", ctypes.c_int64), ("table_bytes", ctypes.c_int64)]


_LIB = None


def library_path() -> str:
    return _LIB_PATH


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2101_07088_amd.build` "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(_LIB_PATH)
        vp, i64, i32, pd = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        L.dpse_status_string.restype = ctypes.c_char_p
        L.dpse_status_string.argtypes = [ctypes.c_int]
        L.dpse_derive.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Info)]
        L.dpse_plan_create.argtypes = [ctypes.POINTER(_Params), i64, vp, ctypes.POINTER(vp)]
        L.dpse_plan_info.argtypes = [vp, ctypes.POINTER(_Info)]
        L.dpse_solve.argtypes = [vp, i64, pd, pd, pd, pd, pd]
        L.dpse_solve_batch.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                       ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       ctypes.POINTER(vp), ctypes.POINTER(vp)]
        L.dpse_workspace_size.argtypes = [ctypes.POINTER(_Params), i64, ctypes.POINTER(i64)]
        L.dpse_plan_create_unbound.argtypes = [ctypes.POINTER(_Params), i64, ctypes.POINTER(vp)]
        L.dpse_plan_bind.argtypes = [vp, vp, i64, vp]
        L.dpse_solve_graph.argtypes = [vp, i64, pd, pd, pd, pd, pd]
        L.dpse_solve_static.argtypes = [vp, vp, i64, pd, pd, pd, pd, pd]
        L.dpse_batch_graph_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                              ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                              ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i32),
                                              ctypes.c_int, ctypes.POINTER(vp)]
        L.dpse_graph_launch.argtypes = [vp, vp]
        L.dpse_graph_destroy.argtypes = [vp]
        L.dpse_plan_autotune.argtypes = [vp, i64, pd, pd, ctypes.c_int, ctypes.POINTER(i32),
                                         ctypes.POINTER(ctypes.c_double)]
        L.dpse_plan_set_tiles.argtypes = [vp, ctypes.POINTER(i32)]
        L.dpse_plan_set_walls.argtypes = [vp, pd, pd]
        L.dpse_solve_near.argtypes = [vp, i64, pd, pd, pd, pd, pd]
        L.dpse_bd_step.argtypes = [vp, i64, pd, pd, pd, pd, ctypes.c_double, ctypes.c_double, pd, pd]
        L.dpse_sync.argtypes = [vp]
        L.dpse_plan_destroy.argtypes = [vp]
        L.dpse_debug_copy.argtypes = [vp, ctypes.c_int, vp, i64, ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.dpse_set_timing.argtypes = [vp, ctypes.c_int]
        L.dpse_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int)]
        L.dpse_stage_name.restype = ctypes.c_char_p
        L.dpse_stage_name.argtypes = [ctypes.c_int]
        for name in ("dpse_derive", "dpse_plan_create", "dpse_plan_info", "dpse_solve", "dpse_solve_batch",
                     "dpse_sync", "dpse_plan_destroy", "dpse_debug_copy", "dpse_set_timing",
                     "dpse_stage_times", "dpse_workspace_size", "dpse_plan_create_unbound", "dpse_plan_bind",
                     "dpse_solve_graph", "dpse_batch_graph_create", "dpse_graph_launch", "dpse_graph_destroy",
                     "dpse_plan_autotune", "dpse_plan_set_tiles", "dpse_plan_set_walls", "dpse_solve_near",
                     "dpse_bd_step", "dpse_solve_static"):
            getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(status: int, where: str):
    if status != 0:
        raise DpseError(status, where)


def _params(p, precision: int = DPSE_FP64, delta: float = 0.0) -> _Params:
    """Accepts any object with the SlabParams attribute names."""
    flags = 0
    if not getattr(p, "gauge", True):
        flags |= DPSE_GAUGE_NONE
    if getattr(p, "kmax_gt", False):
        flags |= DPSE_KMAX_GT
    if getattr(p, "uniform_fast", False):
        flags |= DPSE_UNIFORM_FAST
    if getattr(p, "one_jump", False):
        flags |= DPSE_ONE_JUMP
    if getattr(p, "triply", False):
        flags |= DPSE_TRIPLY
    if getattr(p, "deterministic", False):
        flags |= DPSE_DETERMINISTIC
    return _Params(Lx=p.Lx, Ly=p.Ly, H=p.H, eps=p.eps, eps_bottom=p.eps_b, eps_top=p.eps_t, xi=p.xi,
                   g_w=getattr(p, "g_w", 0.0), Nx=p.Nx, Ny=p.Ny, Nz=p.Nz, support=getattr(p, "n_g", 0),
                   r_cut=p.r_cut, delta=delta, precision=precision, flags=flags)


def _info_dict(info: _Info) -> dict:
    return {name: getattr(info, name) for name, _ in _Info._fields_}


def derive(params, precision: int = DPSE_FP64) -> dict:
    """Host-only parameter derivation and validation (no GPU needed)."""
    prm = _params(params, precision)
    info = _Info()
    _check(_lib().dpse_derive(ctypes.byref(prm), ctypes.byref(info)), "dpse_derive")
    return _info_dict(info)


def workspace_size(params, max_n: int, precision: int = DPSE_FP64) -> int:
    """Device bytes of the workspace of a solve of up to max_n charges (host only)."""
    prm = _params(params, precision)
    b = ctypes.c_int64()
    _check(_lib().dpse_workspace_size(ctypes.byref(prm), int(max_n), ctypes.byref(b)), "dpse_workspace_size")
    return b.value


def check_charges(torch, pos, q, device=None):
    """Validates the inputs of a solve before any pointer reaches the library:
    pos float64 [n, 3] and q float64 [n], contiguous HIP tensors on one device
    (the plan's, when given). Raises ValueError (TypeError for a wrong type);
    returns n."""
    for name, t in (("pos", pos), ("q", q)):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.dtype != torch.float64:
            raise ValueError(f"{name} must be float64, got {t.dtype}")
        if not t.is_cuda:
            raise ValueError(f"{name} must be a HIP device tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    if q.dim() != 1 or q.shape[0] < 1:
        raise ValueError(f"q must have shape (n,) with n >= 1, got {tuple(q.shape)}")
    n = int(q.shape[0])
    if tuple(pos.shape) != (n, 3):
        raise ValueError(f"pos must have shape ({n}, 3), got {tuple(pos.shape)}")
    if pos.device != q.device:
        raise ValueError("pos and q are on different devices")
    if device is not None and pos.device.index != device:
        raise ValueError(f"inputs are on cuda:{pos.device.index}, the plan on cuda:{device}")
    return n


def check_outputs(torch, n, device, energy, phi, force):
    """Validates caller-given outputs (None entries are skipped): energy
    float64 with at least one element, phi float64 [n], force float64 [n, 3],
    contiguous, on `device`."""
    for name, t, shape in (("energy", energy, None), ("phi", phi, (n,)), ("force", force, (n, 3))):
        if t is None:
            continue
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 HIP tensor")
        if t.device.index != device:
            raise ValueError(f"{name} is on cuda:{t.device.index}, the plan on cuda:{device}")
        if shape is None and t.numel() < 1:
            raise ValueError("energy needs one element")
        if shape is not None and tuple(t.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")


class Plan:
    """A plan for one slab system on the current HIP device and stream.

    With own_workspace=False the plan holds only its tables; attach device
    memory with bind() before solving (several plans may share one arena if
    they run on one stream)."""

    def __init__(self, params, max_n: int, precision: int = DPSE_FP64, stream=None, own_workspace: bool = True):
        import torch
        self._torch = torch
        self.params = params
        self.precision = precision
        self.max_n = int(max_n)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.workspace = None
        self.device = torch.cuda.current_device()
        prm = _params(params, precision)
        h = ctypes.c_void_p()
        if own_workspace:
            _check(_lib().dpse_plan_create(ctypes.byref(prm), self.max_n, ctypes.c_void_p(stream.cuda_stream),
                                           ctypes.byref(h)), "dpse_plan_create")
        else:
            _check(_lib().dpse_plan_create_unbound(ctypes.byref(prm), self.max_n, ctypes.byref(h)),
                   "dpse_plan_create_unbound")
        self._h = h
        info = _Info()
        _check(_lib().dpse_plan_info(h, ctypes.byref(info)), "dpse_plan_info")
        self.info = _info_dict(info)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def _io(self, pos, q, energy, phi, force):
        torch = self._torch
        n = check_charges(torch, pos, q, self.device)
        check_outputs(torch, n, self.device, energy, phi, force)
        dev = pos.device
        if energy is None:
            energy = torch.empty(1, dtype=torch.float64, device=dev)
        if phi is None:
            phi = torch.empty(n, dtype=torch.float64, device=dev)
        if force is None:
            force = torch.empty((n, 3), dtype=torch.float64, device=dev)
        return n, energy, phi, force

    def solve(self, pos, q, energy=None, phi=None, force=None):
        """Enqueues a solve. pos: float64 [n,3], q: float64 [n] HIP tensors.
        Returns (energy[1], phi[n], force[n,3]) device tensors (allocated if
        not given)."""
        n, energy, phi, force = self._io(pos, q, energy, phi, force)
        _check(_lib().dpse_solve(self._h, n, pos.data_ptr(), q.data_ptr(), energy.data_ptr(), phi.data_ptr(),
                                 force.data_ptr()), "dpse_solve")
        return energy, phi, force

    def solve_near(self, pos, q, energy=None, phi=None, force=None):
        """dpse_solve_near: the near field at pos with the far field and gauge
        constant of the plan's last full solve of these charges held fixed."""
        n, energy, phi, force = self._io(pos, q, energy, phi, force)
        _check(_lib().dpse_solve_near(self._h, n, pos.data_ptr(), q.data_ptr(), energy.data_ptr(), phi.data_ptr(),
                                      force.data_ptr()), "dpse_solve_near")
        return energy, phi, force

    def bd_step(self, pos, force, w_prev, w_next, mu_dt: float, noise: float, pos_out, escaped):
        """dpse_bd_step: pos_out = pos + mu_dt force + noise (w_prev + w_next);
        escaped (int32 device tensor [1]) counts charges leaving the slab."""
        torch = self._torch
        for name, t in (("pos", pos), ("force", force), ("w_prev", w_prev), ("w_next", w_next),
                        ("pos_out", pos_out)):
            if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
                    and t.dim() == 2 and t.shape[1] == 3 and t.shape == pos.shape
                    and t.device.index == self.device):
                raise ValueError(f"{name} must be a contiguous float64 [n, 3] tensor on cuda:{self.device}")
        if not (isinstance(escaped, torch.Tensor) and escaped.dtype == torch.int32 and escaped.is_cuda
                and escaped.numel() >= 1 and escaped.device.index == self.device):
            raise ValueError(f"escaped must be an int32 tensor on cuda:{self.device}")
        _check(_lib().dpse_bd_step(self._h, int(pos.shape[0]), pos.data_ptr(), force.data_ptr(), w_prev.data_ptr(),
                                   w_next.data_ptr(), float(mu_dt), float(noise), pos_out.data_ptr(),
                                   escaped.data_ptr()), "dpse_bd_step")

    def bind(self, workspace, stream=None):
        """Attaches a caller-owned uint8 device tensor (kept referenced here)
        and a stream to a plan made with own_workspace=False."""
        if stream is None:
            stream = self._torch.cuda.current_stream()
        _check(_lib().dpse_plan_bind(self._h, workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                     ctypes.c_void_p(stream.cuda_stream)), "dpse_plan_bind")
        self.workspace = workspace
        self.stream = stream

    def solve_graph(self, pos, q, energy, phi, force):
        """dpse_solve_graph: the solve as one graph launch (re-captured when
        the sizes, buffers or stream change). Outputs must be given."""
        torch = self._torch
        n = check_charges(torch, pos, q, self.device)
        if energy is None or phi is None or force is None:
            raise ValueError("solve_graph needs all three outputs (the graph records their addresses)")
        check_outputs(torch, n, self.device, energy, phi, force)
        _check(_lib().dpse_solve_graph(self._h, n, pos.data_ptr(), q.data_ptr(), energy.data_ptr(),
                                       phi.data_ptr(), force.data_ptr()), "dpse_solve_graph")
        return energy, phi, force

    def solve_static(self, pos, q, energy, phi, force, stream=None):
        """dpse_solve_static: the solve with its workspace in the library's
        static device array (no allocation in the call). The plan must have
        been made with own_workspace=False; it stays bound to that array and
        to `stream` (default: the current stream). Outputs must be given."""
        torch = self._torch
        n = check_charges(torch, pos, q, self.device)
        if energy is None or phi is None or force is None:
            raise ValueError("solve_static needs all three outputs (it allocates nothing)")
        check_outputs(torch, n, self.device, energy, phi, force)
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(_lib().dpse_solve_static(self._h, ctypes.c_void_p(stream.cuda_stream), n, pos.data_ptr(),
                                        q.data_ptr(), energy.data_ptr(), phi.data_ptr(), force.data_ptr()),
               "dpse_solve_static")
        self.workspace = None
        self.stream = stream
        return energy, phi, force

    def autotune(self, pos, q, reps: int = 3):
        """dpse_plan_autotune: times the launch-shape candidates of spreading,
        interpolation and the column kernel on these charges and keeps the
        fastest. Returns (choice[3], {(stage, index): ms})."""
        check_charges(self._torch, pos, q, self.device)
        ch = (ctypes.c_int32 * 3)()
        ms = (ctypes.c_double * (3 * 16))()
        _check(_lib().dpse_plan_autotune(self._h, int(q.shape[0]), pos.data_ptr(), q.data_ptr(), int(reps), ch, ms),
               "dpse_plan_autotune")
        times = {(s, i): ms[16 * s + i] for s in range(3) for i in range(16) if ms[16 * s + i] > 0}
        return tuple(ch), times

    def set_tiles(self, choice):
        ch = (ctypes.c_int32 * 3)(*[int(c) for c in choice])
        _check(_lib().dpse_plan_set_tiles(self._h, ch), "dpse_plan_set_tiles")

    def set_walls(self, sigma_b=None, sigma_t=None):
        """dpse_plan_set_walls: fixed charge densities on the bottom and top
        walls, float64 [Ny, Nx] HIP tensors of their values at the x,y grid
        points (None: no charge on that wall; both None removes them)."""
        torch = self._torch
        ptrs = []
        for sg in (sigma_b, sigma_t):
            if sg is None:
                ptrs.append(None)
                continue
            assert sg.dtype == torch.float64 and sg.is_cuda and sg.is_contiguous()
            assert tuple(sg.shape) == (self.params.Ny, self.params.Nx)
            ptrs.append(sg.data_ptr())
        _check(_lib().dpse_plan_set_walls(self._h, ptrs[0], ptrs[1]), "dpse_plan_set_walls")
        self._walls = (sigma_b, sigma_t)  # kept alive until the stream has copied them

    def sync(self) -> int:
        """Waits for the stream; raises DpseError for a device-detected error."""
        st = _lib().dpse_sync(self._h)
        _check(st, "dpse_sync")
        return st

    def sync_status(self) -> int:
        return _lib().dpse_sync(self._h)

    def debug(self, stage: Stage) -> np.ndarray:
        """Copies a stage output of the last solve (layouts in include/dpse.h)."""
        p = self.params
        nkx = p.Nx // 2 + 1
        G = p.Nz * p.Ny * p.Nx
        sizes = {Stage.F_I: G, Stage.F_O: G, Stage.FH_I: 2 * p.Nz * p.Ny * nkx, Stage.FH_O: 2 * p.Nz * p.Ny * nkx, Stage.PSI: 2 * p.Nz * p.Ny * nkx,
                 Stage.PSIZ: 2 * p.Nz * p.Ny * nkx, Stage.GRIDS: 4 * G, Stage.FAR: 4 * self.max_n,
                 Stage.NEAR: 4 * self.max_n, Stage.SCALARS: 8, Stage.WALL_HAT: 4 * p.Ny * nkx,
                 Stage.WALL_PHI: G, Stage.WALL_SCALARS: 4}
        buf = np.empty(sizes[stage] * 8, dtype=np.uint8)
        eb = ctypes.c_int32()
        cnt = ctypes.c_int64()
        _check(_lib().dpse_debug_copy(self._h, int(stage), buf.ctypes.data, buf.nbytes, ctypes.byref(eb),
                                      ctypes.byref(cnt)), "dpse_debug_copy")
        dt = np.float64 if eb.value == 8 else np.float32
        a = buf[: cnt.value * eb.value].view(dt).astype(np.float64)
        if stage in (Stage.F_I, Stage.F_O, Stage.WALL_PHI):
            return a.reshape(p.Nz, p.Ny, p.Nx)
        if stage == Stage.WALL_HAT:
            c = a.reshape(2, p.Ny, nkx, 2)
            return c[..., 0] + 1j * c[..., 1]
        if stage in (Stage.FH_I, Stage.FH_O, Stage.PSI, Stage.PSIZ):
            c = a.reshape(p.Nz, p.Ny, nkx, 2)
            return c[..., 0] + 1j * c[..., 1]
        if stage == Stage.GRIDS:
            return np.moveaxis(a.reshape(p.Nz, p.Ny, p.Nx, 4), -1, 0)
        if stage in (Stage.FAR, Stage.NEAR):
            return a.reshape(-1, 4)
        return a

    def set_timing(self, enable: bool = True):
        _check(_lib().dpse_set_timing(self._h, int(bool(enable))), "dpse_set_timing")

    def stage_times(self) -> tuple:
        """Mean per-stage milliseconds over the solves recorded since the last
        call: (dict name -> ms, number of solves)."""
        ns = 10
        ms = (ctypes.c_double * ns)()
        cnt = ctypes.c_int()
        _check(_lib().dpse_stage_times(self._h, ms, ns, ctypes.byref(cnt)), "dpse_stage_times")
        return {_lib().dpse_stage_name(i).decode(): ms[i] for i in range(ns)}, cnt.value

    def close(self):
        if getattr(self, "_h", None):
            _lib().dpse_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(plans: Sequence[Plan], pos: Sequence, q: Sequence, energy: Optional[Sequence] = None,
                phi: Optional[Sequence] = None, force: Optional[Sequence] = None):
    """Enqueues one solve per plan through dpse_solve_batch; outputs are
    allocated when not given. Returns lists (energy, phi, force)."""
    import torch
    k = len(plans)
    if not (len(pos) == len(q) == k) or k < 1:
        raise ValueError("one position and one charge tensor per plan")
    for i in range(k):
        check_charges(torch, pos[i], q[i], plans[i].device)
    if energy is None:
        energy = [torch.empty(1, dtype=torch.float64, device=p_.device) for p_ in pos]
    if phi is None:
        phi = [torch.empty(q_.shape[0], dtype=torch.float64, device=q_.device) for q_ in q]
    if force is None:
        force = [torch.empty((q_.shape[0], 3), dtype=torch.float64, device=q_.device) for q_ in q]
    VP = ctypes.c_void_p * k
    hs = VP(*[p_.handle.value for p_ in plans])
    ns = (ctypes.c_int64 * k)(*[int(q_.shape[0]) for q_ in q])
    for i in range(k):
        check_outputs(torch, int(q[i].shape[0]), plans[i].device, energy[i], phi[i], force[i])
    ptr = lambda ts: VP(*[t.data_ptr() for t in ts])
    _check(_lib().dpse_solve_batch(k, hs, ns, ptr(pos), ptr(q), ptr(energy), ptr(phi), ptr(force)),
           "dpse_solve_batch")
    return energy, phi, force


class BatchGraph:
    """dpse_batch_graph_create: a batch of solves captured into one graph.
    The tensors passed here are kept referenced; launch() re-runs the batch on
    whatever they hold."""

    def __init__(self, plans: Sequence[Plan], pos: Sequence, q: Sequence, energy: Sequence, phi: Sequence,
                 force: Sequence, branch: Optional[Sequence[int]] = None, n_branches: int = 1):
        import torch
        k = len(plans)
        if not (len(pos) == len(q) == len(energy) == len(phi) == len(force) == k) or k < 1:
            raise ValueError("one tensor of each kind per plan")
        for i in range(k):
            n = check_charges(torch, pos[i], q[i], plans[i].device)
            check_outputs(torch, n, plans[i].device, energy[i], phi[i], force[i])
        VP = ctypes.c_void_p * k
        hs = VP(*[p_.handle.value for p_ in plans])
        ns = (ctypes.c_int64 * k)(*[int(q_.shape[0]) for q_ in q])
        ptr = lambda ts: VP(*[t.data_ptr() for t in ts])
        br = None if branch is None else (ctypes.c_int32 * k)(*[int(b) for b in branch])
        h = ctypes.c_void_p()
        _check(_lib().dpse_batch_graph_create(k, hs, ns, ptr(pos), ptr(q), ptr(energy), ptr(phi), ptr(force), br,
                                              int(n_branches), ctypes.byref(h)), "dpse_batch_graph_create")
        self._h = h
        self._keep = (list(plans), list(pos), list(q), list(energy), list(phi), list(force))

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(_lib().dpse_graph_launch(self._h, ctypes.c_void_p(stream.cuda_stream)), "dpse_graph_launch")

    def close(self):
        if getattr(self, "_h", None):
            _lib().dpse_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
