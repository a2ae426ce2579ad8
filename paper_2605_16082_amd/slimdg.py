"""ctypes binding of libslimdg (slimdg.h): argument marshalling only.

Every step of the operator runs in the HIP library; this module builds the
C mesh description from NumPy arrays, allocates device buffers with torch,
passes raw device pointers and torch's current HIP stream, and maps status
codes to exceptions.  It raises if the library is not built: there is no
fallback path.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# SLIMDG_LIB selects another build of the same library (the host-sanitizer
# build of the ABI tests); by default the in-tree libslimdg.so.
LIB_PATH = os.environ.get("SLIMDG_LIB") or os.path.join(_PKG, "libslimdg.so")

SDG_FP64, SDG_FP32, SDG_FP32_STATE_FP64_SOLVE = 0, 1, 2
SDG_DV_VU, SDG_DV_VD = 0, 1
SDG_SCHEME_SSPRK3_LIE, SDG_SCHEME_SPLIT_IMEX = 0, 1
SDG_DV_MAX_COMP = 4
SDG_PROBE_READ, SDG_PROBE_WRITE, SDG_PROBE_COPY = 0, 1, 2
STATUS_NAMES = {0: "SDG_OK", -1: "SDG_E_ARG", -2: "SDG_E_MESH", -3: "SDG_E_HIP", -4: "SDG_E_STATE",
                -5: "SDG_E_UNSUPPORTED", -6: "SDG_E_NUMERIC", -7: "SDG_E_WORKSPACE"}

EXPORTED = (
    "sdg_abi_version", "sdg_last_error", "sdg_query_layout", "sdg_prism_slots", "sdg_create",
    "sdg_destroy", "sdg_mesh_upload", "sdg_set_params", "sdg_set_velocity", "sdg_set_diffusivity",
    "sdg_set_fields", "sdg_rhs_3d", "sdg_rk_stage", "sdg_vertical_implicit_solve", "sdg_step",
    "sdg_mass", "sdg_sync", "sdg_get_tuning", "sdg_set_tuning", "sdg_autotune",
    "sdg_graph_capture_step", "sdg_graph_launch", "sdg_apply_mass", "sdg_m_dot", "sdg_step_adjoint",
    "sdg_column_dv_solve", "sdg_step_adjoint_imex", "sdg_mass_noalloc", "sdg_stream_probe",
    "sdg_step_keep_half", "sdg_step_adjoint_imex_half",
)


class SlimDGError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("n_members", ctypes.c_int32),
        ("n_tri", ctypes.c_int32),
        ("n_vert", ctypes.c_int32),
        ("member_tri_off", ctypes.c_void_p),
        ("vxy", ctypes.c_void_p),
        ("tri", ctypes.c_void_p),
        ("nbr", ctypes.c_void_p),
        ("nlayers", ctypes.c_void_p),
        ("zlev", ctypes.c_void_p),
        ("n_fields", ctypes.c_int32),
        ("precision", ctypes.c_int32),
    ]


class Layout(ctypes.Structure):
    _fields_ = [
        ("n_prisms", ctypes.c_int64),
        ("n_slots", ctypes.c_int64),
        ("n_cells", ctypes.c_int32),
        ("max_layers", ctypes.c_int32),
        ("n_fields", ctypes.c_int32),
        ("state_elem_bytes", ctypes.c_int32),
        ("state_bytes", ctypes.c_size_t),
        ("velocity_bytes", ctypes.c_size_t),
        ("workspace_bytes", ctypes.c_size_t),
    ]


SDG_DEPTH_BUCKETS = 6


class Tuning(ctypes.Structure):
    _fields_ = [("tile_layers", ctypes.c_int32), ("xcd_remap", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("walk_layers", ctypes.c_int32 * SDG_DEPTH_BUCKETS)]


class Params(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double),
        ("penalty_eta", ctypes.c_double),
        ("t_ext", ctypes.c_void_p),
        ("w_is_zero", ctypes.c_int32),
        ("check_finite", ctypes.c_int32),
        ("time_scheme", ctypes.c_int32),
        ("okubo_scale", ctypes.c_double),
    ]


_lib = None


def load_library(path: str | None = None):
    """Load libslimdg.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built; run `python -m paper_2605_16082_amd.build`")
    lib = ctypes.CDLL(p)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    sig = {
        "sdg_abi_version": ([], i32),
        "sdg_last_error": ([], ctypes.c_char_p),
        "sdg_query_layout": ([ctypes.POINTER(MeshDesc), ctypes.POINTER(Layout)], i32),
        "sdg_prism_slots": ([ctypes.POINTER(MeshDesc), vp], i32),
        "sdg_create": ([ctypes.POINTER(vp), i32, vp], i32),
        "sdg_destroy": ([vp], i32),
        "sdg_mesh_upload": ([vp, ctypes.POINTER(MeshDesc), vp, sz], i32),
        "sdg_set_params": ([vp, ctypes.POINTER(Params)], i32),
        "sdg_set_velocity": ([vp, vp], i32),
        "sdg_set_diffusivity": ([vp, vp], i32),
        "sdg_set_fields": ([vp, vp], i32),
        "sdg_rhs_3d": ([vp, vp, vp], i32),
        "sdg_rk_stage": ([vp, i32, vp, vp, vp], i32),
        "sdg_vertical_implicit_solve": ([vp, vp, vp], i32),
        "sdg_step": ([vp, i32], i32),
        "sdg_mass": ([vp, vp, vp], i32),
        "sdg_sync": ([vp], i32),
        "sdg_get_tuning": ([vp, ctypes.POINTER(Tuning)], i32),
        "sdg_set_tuning": ([vp, ctypes.POINTER(Tuning)], i32),
        "sdg_autotune": ([vp, i32, ctypes.POINTER(Tuning)], i32),
        "sdg_graph_capture_step": ([vp], i32),
        "sdg_graph_launch": ([vp, i32], i32),
        "sdg_apply_mass": ([vp, vp, vp, i32], i32),
        "sdg_m_dot": ([vp, vp, vp, vp], i32),
        "sdg_step_adjoint": ([vp, vp, vp, vp, vp], i32),
        "sdg_column_dv_solve": ([vp, i32, i32, vp, vp], i32),
        "sdg_step_adjoint_imex": ([vp, vp, vp, vp, vp], i32),
        "sdg_step_keep_half": ([vp, vp], i32),
        "sdg_step_adjoint_imex_half": ([vp, vp, vp, vp, vp], i32),
        "sdg_mass_noalloc": ([vp, vp, vp], i32),
        "sdg_stream_probe": ([i32, vp, vp, sz, i32, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if path is None:
        _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = load_library().sdg_last_error()
        raise SlimDGError(status, msg.decode() if msg else "")


class Mesh:
    """Host-side mesh description (keeps the NumPy arrays it points to alive)."""

    def __init__(self, vxy, tri, nbr, nlayers, zlev, n_fields: int, precision: int = SDG_FP64,
                 member_tri_off=None):
        self.vxy = np.ascontiguousarray(vxy, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        self.nlayers = np.ascontiguousarray(nlayers, dtype=np.int32)
        self.zlev = np.ascontiguousarray(zlev, dtype=np.float64)
        self.n_fields = int(n_fields)
        self.precision = int(precision)
        self.member_tri_off = (None if member_tri_off is None
                               else np.ascontiguousarray(member_tri_off, dtype=np.int32))
        n_members = 1 if self.member_tri_off is None else len(self.member_tri_off) - 1
        self._desc = MeshDesc(
            n_members, self.tri.shape[0], self.vxy.shape[0],
            None if self.member_tri_off is None else self.member_tri_off.ctypes.data,
            self.vxy.ctypes.data, self.tri.ctypes.data, self.nbr.ctypes.data,
            self.nlayers.ctypes.data, self.zlev.ctypes.data, self.n_fields, self.precision)

    @classmethod
    def from_workload(cls, w, precision: int = SDG_FP64, n_fields: int | None = None):
        return cls(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev,
                   w.n_fields if n_fields is None else n_fields, precision, w.member_tri_off)

    @property
    def desc(self) -> MeshDesc:
        return self._desc

    @property
    def n_members(self) -> int:
        return int(self._desc.n_members)

    def layout(self) -> Layout:
        lib = load_library()
        out = Layout()
        _check(lib.sdg_query_layout(ctypes.byref(self._desc), ctypes.byref(out)))
        return out

    def prism_slots(self) -> np.ndarray:
        lib = load_library()
        n = int(self.nlayers.sum())
        out = np.empty(n, dtype=np.int64)
        _check(lib.sdg_prism_slots(ctypes.byref(self._desc), out.ctypes.data))
        return out


def _ptr(t) -> int:
    return int(t.data_ptr())


class SlimDG:
    """One uploaded mesh on one GPU.  Device buffers are torch tensors; every
    call enqueues on torch's current stream of ``device`` at construction."""

    def __init__(self, mesh: Mesh, device: int = 0):
        import torch

        self.torch = torch
        self.mesh = mesh
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        self.layout = mesh.layout()
        self.slots_np = mesh.prism_slots()
        self.n_slots = int(self.layout.n_slots)
        self.n_fields = int(self.layout.n_fields)
        self.dtype = torch.float64 if mesh.precision == SDG_FP64 else torch.float32
        self.stream = torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        _check(self.lib.sdg_create(ctypes.byref(ctx), device, ctypes.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx
        self.workspace = torch.empty(int(self.layout.workspace_bytes), dtype=torch.uint8, device=self.device)
        _check(self.lib.sdg_mesh_upload(self.ctx, ctypes.byref(mesh.desc), _ptr(self.workspace),
                                        int(self.layout.workspace_bytes)))
        self.slots = torch.from_numpy(self.slots_np).to(self.device)
        self._keep = {}

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.sdg_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # -- buffers -------------------------------------------------------------
    def zeros(self, rows: int):
        return self.torch.zeros((rows, 6, self.n_slots), dtype=self.dtype, device=self.device)

    def new_state(self):
        return self.zeros(self.n_fields)

    def scatter(self, natural, out=None):
        """(K, 6, P) natural-order values -> device (K, 6, n_slots) in cell layout."""
        torch = self.torch
        src = torch.as_tensor(np.ascontiguousarray(natural), dtype=self.dtype).to(self.device)
        if out is None:
            out = self.zeros(src.shape[0])
        out[:, :, self.slots] = src
        return out

    def gather(self, dev) -> np.ndarray:
        """Device (K, 6, n_slots) -> (K, 6, P) float64 NumPy in natural order."""
        return dev[:, :, self.slots].double().cpu().numpy()

    def _check_nodal(self, t, rows):
        if (t.dtype != self.dtype or t.device != self.device or not t.is_contiguous()
                or tuple(t.shape) != (rows, 6, self.n_slots)):
            raise ValueError(f"expected a contiguous {self.dtype} tensor of shape ({rows}, 6, {self.n_slots}) "
                             f"on {self.device}, got {t.dtype} {tuple(t.shape)} on {t.device}")

    # -- state ---------------------------------------------------------------
    def set_params(self, dt: float, t_ext=None, penalty_eta: float = 4.0, w_is_zero: bool = False,
                   check_finite: bool = False, time_scheme: int = SDG_SCHEME_SSPRK3_LIE,
                   okubo_scale: float = 0.0):
        text = np.zeros(self.n_fields) if t_ext is None else np.ascontiguousarray(t_ext, dtype=np.float64)
        self._keep["t_ext"] = text
        p = Params(float(dt), float(penalty_eta), text.ctypes.data, int(bool(w_is_zero)), int(bool(check_finite)),
                   int(time_scheme), float(okubo_scale))
        _check(self.lib.sdg_set_params(self.ctx, ctypes.byref(p)))
        self.time_scheme = int(time_scheme)

    def set_velocity(self, U):
        self._check_nodal(U, 3)
        self._keep["U"] = U
        _check(self.lib.sdg_set_velocity(self.ctx, _ptr(U)))

    def set_diffusivity(self, kappa):
        if kappa.dtype != self.torch.float64 or kappa.numel() < int(self.layout.max_layers) or not kappa.is_contiguous():
            raise ValueError(f"kappa must be a contiguous float64 device tensor with >= {self.layout.max_layers} entries")
        self._keep["kappa"] = kappa
        _check(self.lib.sdg_set_diffusivity(self.ctx, _ptr(kappa)))

    def set_fields(self, state):
        self._check_nodal(state, self.n_fields)
        self._keep["state"] = state
        _check(self.lib.sdg_set_fields(self.ctx, _ptr(state)))

    # -- operator ------------------------------------------------------------
    def rhs_3d(self, T, out=None):
        out = self.new_state() if out is None else out
        self._check_nodal(T, self.n_fields)
        self._check_nodal(out, self.n_fields)
        _check(self.lib.sdg_rhs_3d(self.ctx, _ptr(T), _ptr(out)))
        return out

    def rk_stage(self, stage: int, Tn, Ts, out=None):
        out = self.new_state() if out is None else out
        for t in (Ts, out) if Tn is None else (Tn, Ts, out):
            self._check_nodal(t, self.n_fields)
        _check(self.lib.sdg_rk_stage(self.ctx, int(stage), None if Tn is None else _ptr(Tn), _ptr(Ts), _ptr(out)))
        return out

    def vertical_implicit_solve(self, Tstar, out=None):
        out = self.new_state() if out is None else out
        self._check_nodal(Tstar, self.n_fields)
        self._check_nodal(out, self.n_fields)
        _check(self.lib.sdg_vertical_implicit_solve(self.ctx, _ptr(Tstar), _ptr(out)))
        return out

    def step(self, n_steps: int = 1):
        _check(self.lib.sdg_step(self.ctx, int(n_steps)))

    def mass(self, T) -> np.ndarray:
        self._check_nodal(T, self.n_fields)
        out = np.zeros(self.mesh.n_members * self.n_fields, dtype=np.float64)
        _check(self.lib.sdg_mass(self.ctx, _ptr(T), out.ctypes.data))
        return out.reshape(self.mesh.n_members, self.n_fields)

    def mass_noalloc(self, T) -> np.ndarray:
        """``mass`` through the entry point that keeps its partial sums in the
        library's static device scratch (no workspace, no allocation)."""
        self._check_nodal(T, self.n_fields)
        out = np.zeros(self.mesh.n_members * self.n_fields, dtype=np.float64)
        _check(self.lib.sdg_mass_noalloc(self.ctx, _ptr(T), out.ctypes.data))
        return out.reshape(self.mesh.n_members, self.n_fields)

    def sync(self):
        _check(self.lib.sdg_sync(self.ctx))

    # -- launch shape, autotuning, graph replay -------------------------------
    def get_tuning(self) -> tuple[int, int, int]:
        """(tile_layers, xcd_remap, persistent) of the stage kernel; tile_layers
        0 means walks segmented per depth bucket (``walk_layers``)."""
        t = Tuning()
        _check(self.lib.sdg_get_tuning(self.ctx, ctypes.byref(t)))
        return int(t.tile_layers), int(t.xcd_remap), int(t.persistent)

    def walk_layers(self) -> list[int]:
        """Per depth bucket walk segmentation (zeros unless tile_layers is 0)."""
        t = Tuning()
        _check(self.lib.sdg_get_tuning(self.ctx, ctypes.byref(t)))
        return [int(v) for v in t.walk_layers]

    def set_tuning(self, tile_layers: int, xcd_remap: int = 1, persistent: int = 0, walk_layers=None):
        wl = (ctypes.c_int32 * SDG_DEPTH_BUCKETS)(*([0] * SDG_DEPTH_BUCKETS if walk_layers is None
                                                     else [int(v) for v in walk_layers]))
        t = Tuning(int(tile_layers), int(xcd_remap), int(persistent), wl)
        _check(self.lib.sdg_set_tuning(self.ctx, ctypes.byref(t)))

    def autotune(self, reps: int = 5) -> tuple[int, int, int]:
        """Measure and keep the fastest launch shape; returns get_tuning()."""
        t = Tuning()
        _check(self.lib.sdg_autotune(self.ctx, int(reps), ctypes.byref(t)))
        return int(t.tile_layers), int(t.xcd_remap), int(t.persistent)

    def graph_capture_step(self):
        _check(self.lib.sdg_graph_capture_step(self.ctx))

    def graph_launch(self, n_steps: int = 1):
        _check(self.lib.sdg_graph_launch(self.ctx, int(n_steps)))

    # -- mass operator and adjoint ---------------------------------------------
    def apply_mass(self, X, out=None, inverse: bool = False):
        out = self.new_state() if out is None else out
        self._check_nodal(X, self.n_fields)
        self._check_nodal(out, self.n_fields)
        _check(self.lib.sdg_apply_mass(self.ctx, _ptr(X), _ptr(out), int(bool(inverse))))
        return out

    def m_dot(self, X, Y) -> np.ndarray:
        """(n_members, n_fields) array of X_f^T M Y_f."""
        self._check_nodal(X, self.n_fields)
        self._check_nodal(Y, self.n_fields)
        out = np.zeros(self.mesh.n_members * self.n_fields, dtype=np.float64)
        _check(self.lib.sdg_m_dot(self.ctx, _ptr(X), _ptr(Y), out.ctypes.data))
        return out.reshape(self.mesh.n_members, self.n_fields)

    def step_adjoint_imex(self, z_next, z_out, x_prev=None, dkappa=None):
        """Reverse of one split-IMEX step; x_prev is the state before that step."""
        self._check_nodal(z_next, self.n_fields)
        self._check_nodal(z_out, self.n_fields)
        if x_prev is not None:
            self._check_nodal(x_prev, self.n_fields)
        if dkappa is not None and (dkappa.dtype != self.torch.float64 or dkappa.numel() < int(self.layout.max_layers)):
            raise ValueError("dkappa must be a float64 device tensor with >= max_layers entries")
        _check(self.lib.sdg_step_adjoint_imex(self.ctx, _ptr(z_next), _ptr(z_out),
                                              None if x_prev is None else _ptr(x_prev),
                                              None if dkappa is None else _ptr(dkappa)))

    def step_keep_half(self, x_half):
        """One split-IMEX step of the set fields that leaves its half-step
        state x_h in x_half (what step_adjoint_imex_half takes)."""
        self._check_nodal(x_half, self.n_fields)
        _check(self.lib.sdg_step_keep_half(self.ctx, _ptr(x_half)))

    def step_adjoint_imex_half(self, z_next, z_out, x_half=None, dkappa=None):
        """Reverse of one split-IMEX step given that step's x_h."""
        self._check_nodal(z_next, self.n_fields)
        self._check_nodal(z_out, self.n_fields)
        if x_half is not None:
            self._check_nodal(x_half, self.n_fields)
        if dkappa is not None and (dkappa.dtype != self.torch.float64 or dkappa.numel() < int(self.layout.max_layers)):
            raise ValueError("dkappa must be a float64 device tensor with >= max_layers entries")
        _check(self.lib.sdg_step_adjoint_imex_half(self.ctx, _ptr(z_next), _ptr(z_out),
                                                   None if x_half is None else _ptr(x_half),
                                                   None if dkappa is None else _ptr(dkappa)))

    def step_adjoint(self, z_next, z_out, x_next=None, dkappa=None):
        self._check_nodal(z_next, self.n_fields)
        self._check_nodal(z_out, self.n_fields)
        if x_next is not None:
            self._check_nodal(x_next, self.n_fields)
        if dkappa is not None and (dkappa.dtype != self.torch.float64 or dkappa.numel() < int(self.layout.max_layers)):
            raise ValueError("dkappa must be a float64 device tensor with >= max_layers entries")
        _check(self.lib.sdg_step_adjoint(self.ctx, _ptr(z_next), _ptr(z_out),
                                         None if x_next is None else _ptr(x_next),
                                         None if dkappa is None else _ptr(dkappa)))

    # -- matrix-free column solves -------------------------------------------------
    def column_dv_solve(self, kind: int, F, out=None):
        """x with D x = F per column (kind SDG_DV_VU or SDG_DV_VD); F (n_comp, 6, n_slots)."""
        n_comp = int(F.shape[0])
        out = self.zeros(n_comp) if out is None else out
        self._check_nodal(F, n_comp)
        self._check_nodal(out, n_comp)
        _check(self.lib.sdg_column_dv_solve(self.ctx, int(kind), n_comp, _ptr(F), _ptr(out)))
        return out


def stream_probe(kind: int, src, dst, nbytes: int, workgroups: int):
    """Enqueue one streaming probe (SDG_PROBE_READ / _WRITE / _COPY) on torch's
    current stream; src and dst are device tensors (src may be None for WRITE)."""
    import torch

    lib = load_library()
    stream = torch.cuda.current_stream(dst.device)
    _check(lib.sdg_stream_probe(int(kind), None if src is None else _ptr(src), _ptr(dst), int(nbytes),
                                int(workgroups), ctypes.c_void_p(stream.cuda_stream)))


def from_workload(w, precision: int = SDG_FP64, device: int = 0, time_scheme: int = SDG_SCHEME_SSPRK3_LIE,
                  okubo_scale: float = 0.0):
    """Upload a workload and set velocity, diffusivity, params and fields."""
    import torch

    mesh = Mesh.from_workload(w, precision)
    s = SlimDG(mesh, device)
    U = s.scatter(w.U)
    kappa = torch.as_tensor(np.ascontiguousarray(w.kappa, dtype=np.float64)).to(s.device)
    state = s.scatter(w.T0)
    s.set_params(w.dt, w.t_ext, w.penalty, w.w_is_zero, time_scheme=time_scheme, okubo_scale=okubo_scale)
    s.set_velocity(U)
    s.set_diffusivity(kappa)
    s.set_fields(state)
    return s, U, kappa, state
