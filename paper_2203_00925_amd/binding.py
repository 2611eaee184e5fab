"""Thin Python binding of libmifvm (ctypes over the C ABI in include/mifvm.h).

Argument marshalling only: host arrays are passed as NumPy buffers, device
buffers as torch CUDA (HIP) tensors' data pointers, streams as the raw
hipStream_t of a torch stream.  Every computation runs in the library.  If
the library has not been built, importing this module raises - there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libmifvm.so")

OK, NOT_CONVERGED, FELL_BACK = 0, 1, 2
ZERO_FLUX, NEUMANN, DIRICHLET = 0, 1, 2
VAR_SCALAR, VAR_POTENTIAL = 0, 1
FIELD_U, FIELD_VEL, FIELD_SOURCE, FIELD_P, FIELD_ION, FIELD_EFIELD = 0, 1, 2, 3, 4, 5
RENUMBER_NONE, RENUMBER_MORTON, RENUMBER_RCM = 0, 1, 2
SOLVE_PLAIN, SOLVE_IR_FP32, SOLVE_LEARNED, SOLVE_FGMRES, SOLVE_AMG = 0, 1, 2, 3, 4
CYCLE_V, CYCLE_W = 1, 2
FP64, FP32 = 0, 1
F64, F32 = 0, 1                           # element types of field arrays at the ABI
KERNELS = ("ghost_fill", "grad_limiter", "node_interp", "face_flux", "update", "cg_setup",
           "cg_spmv", "cg_axpy", "cg_dir", "rhs", "assemble", "nn_layer1", "nn_layer2", "nn_layer3",
           "fcg_vec", "nn_train", "mf_vertex", "mf_face", "mf_gather", "nn_fused", "cg_alpha", "fv_cell")
NN_PARAMS = 9537
LOSS_RESIDUAL, LOSS_ENERGY = 0, 1
NN_FORM_AUTO, NN_FORM_LAYERS, NN_FORM_FUSED = 0, 1, 2

EXPORTS = {  # id: (name, dtype, shape-fn(info))
    0: ("cell_perm", np.int32, lambda i: (i.nc,)),
    1: ("vert_perm", np.int32, lambda i: (i.nv,)),
    2: ("volume", np.float64, lambda i: (i.nc,)),
    3: ("centre", np.float64, lambda i: (3, i.nc + i.nb)),
    4: ("face_lr", np.int32, lambda i: (2, i.nf)),
    5: ("face_abc", np.int32, lambda i: (3, i.nf)),
    6: ("face_coef", np.float64, lambda i: (3, i.nf)),
    7: ("face_s", np.float64, lambda i: (3, i.nf)),
    8: ("stencil_ptr", np.int64, lambda i: (i.nc + 1,)),
    9: ("stencil_idx", np.int32, lambda i: (i.stencil_entries,)),
    10: ("node_ptr", np.int64, lambda i: (i.nv + 1,)),
    11: ("node_idx", np.int32, lambda i: (i.node_entries,)),
    12: ("node_alpha", np.float64, lambda i: (i.node_entries,)),
    13: ("ghost_owner", np.int32, lambda i: (i.nb,)),
    14: ("ghost_tag", np.int32, lambda i: (i.nb,)),
    15: ("minv", np.float64, lambda i: (6, i.nc)),
    16: ("edge_nbr_ptr", np.int64, lambda i: (i.nc + 1,)),
    17: ("edge_nbr_idx", np.int32, lambda i: (i.edge_nbr_entries,)),
}
EXPORT_IDS = {v[0]: k for k, v in EXPORTS.items()}


class MifvmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mifvm error {code}: {msg}")
        self.code = code


class _MeshOpts(C.Structure):
    _fields_ = [("renumber", C.c_int32), ("nmeshes", C.c_int32),
                ("mesh_cell_start", C.c_void_p), ("no_matrix", C.c_int32), ("pad_", C.c_int32)]


class MeshInfo(C.Structure):
    _fields_ = [("nc", C.c_int64), ("nv", C.c_int64), ("nf", C.c_int64),
                ("nf_interior", C.c_int64), ("nb", C.c_int64), ("nmeshes", C.c_int32),
                ("pad0_", C.c_int32),
                ("stencil_entries", C.c_int64), ("stencil_padded", C.c_int64),
                ("node_entries", C.c_int64), ("matrix_nnz", C.c_int64),
                ("matrix_padded", C.c_int64), ("stencil_max", C.c_int32),
                ("node_max", C.c_int32), ("row_max", C.c_int32), ("tile_rows", C.c_int32),
                ("halo_max", C.c_int32), ("tile_vertices_max", C.c_int32), ("halo_entries", C.c_int64),
                ("ws_bytes", C.c_size_t), ("edge_nbr_entries", C.c_int64),
                ("foreign_rows", C.c_int64), ("foreign_entries", C.c_int64)]


class _Params(C.Structure):
    _fields_ = [("diffusivity", C.c_double), ("precision", C.c_int32), ("pad_", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("chunk", C.c_int32),
                ("restart", C.c_int32), ("history_cap", C.c_int32),
                ("history", C.POINTER(C.c_double)), ("method", C.c_int32),
                ("graph", C.c_int32), ("inner_tol", C.c_double),
                ("stall_window", C.c_int32), ("learned_maxit", C.c_int32),
                ("matrix_free", C.c_int32), ("learned_smoother", C.c_int32)]


class TuneInfo(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("graph", C.c_int32), ("step_graph", C.c_int32),
                ("from_cache", C.c_int32), ("ms_per_iteration", C.c_double),
                ("ms_per_step_direct", C.c_double), ("ms_per_step_graph", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32),
                ("history_len", C.c_int32), ("outer", C.c_int32),
                ("rel_residual", C.c_double), ("ms", C.c_double),
                ("fell_back", C.c_int32), ("learned_iterations", C.c_int32)]


class BatchOpts(C.Structure):
    _fields_ = [("item_rows", C.c_int32), ("grid", C.c_int32), ("policy", C.c_int32),
                ("spin_limit", C.c_int32), ("vertex_batch", C.c_int32), ("chunk", C.c_int32)]


class BatchSolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("restart", C.c_int32),
                ("solve_every", C.c_int32), ("pad_", C.c_int32)]


class BatchInfo(C.Structure):
    _fields_ = [("solves", C.c_int32), ("pad_", C.c_int32), ("iterations_max", C.c_int64),
                ("iterations_sum", C.c_int64), ("iterations_mean", C.c_double),
                ("rel_residual_max", C.c_double), ("ms", C.c_double)]


class BatchTuneInfo(C.Structure):
    _fields_ = [("item_rows", C.c_int32), ("grid", C.c_int32), ("policy", C.c_int32),
                ("from_cache", C.c_int32), ("trials", C.c_int32), ("iterations", C.c_int32),
                ("ms_best", C.c_double), ("vertex_batch", C.c_int32), ("chunk", C.c_int32),
                ("ms_persistent", C.c_double), ("ms_launches", C.c_double),
                ("p_item_rows", C.c_int32), ("p_grid", C.c_int32), ("p_policy", C.c_int32),
                ("p_vertex_batch", C.c_int32)]


class AmgOpts(C.Structure):
    _fields_ = [("theta", C.c_double), ("omega", C.c_double), ("max_levels", C.c_int32),
                ("coarse_max", C.c_int32), ("cycle", C.c_int32), ("pad_", C.c_int32)]


class AmgInfo(C.Structure):
    _fields_ = [("levels", C.c_int32), ("pad_", C.c_int32), ("rows", C.c_int64 * 16),
                ("nnz", C.c_int64 * 16), ("setup_ms", C.c_double), ("ws_bytes", C.c_size_t)]


def _amg_info(info):
    return {"levels": info.levels, "rows": list(info.rows[:info.levels]), "nnz": list(info.nnz[:info.levels]),
            "setup_ms": info.setup_ms, "ws_bytes": int(info.ws_bytes)}


class AmgHost:
    """Host-only multigrid setup of a CSR matrix (mifvm_amg_host_*), no GPU."""

    def __init__(self, ptr, col, val, theta=0.0, omega=0.0, max_levels=0, coarse_max=0):
        ptr = np.ascontiguousarray(ptr, np.int64)
        col = np.ascontiguousarray(col, np.int32)
        val = np.ascontiguousarray(val, np.float64)
        h = C.c_void_p()
        opts = AmgOpts(float(theta), float(omega), int(max_levels), int(coarse_max), 0, 0)
        _check(_lib.mifvm_amg_host_build(C.c_int64(len(ptr) - 1), ptr.ctypes.data_as(C.c_void_p),
                                         col.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p),
                                         C.byref(opts), C.byref(h)))
        self._h = h
        info = AmgInfo()
        _check(_lib.mifvm_amg_host_info(self._h, C.byref(info)))
        self.info = _amg_info(info)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mifvm_amg_host_destroy(self._h)
            self._h = None

    def export(self, level, what):
        """what: 'agg', 'ptr', 'col', 'val', 'cinv'."""
        n, nnz = self.info["rows"][level], self.info["nnz"][level]
        dt, count = {"agg": (np.int32, n), "ptr": (np.int64, n + 1), "col": (np.int32, nnz),
                     "val": (np.float64, nnz), "cinv": (np.float64, n * n)}[what]
        out = np.empty(count, dt)
        _check(_lib.mifvm_amg_host_export(self._h, int(level), ["agg", "ptr", "col", "val", "cinv"].index(what),
                                          out.ctypes.data_as(C.c_void_p), C.c_size_t(out.nbytes)))
        return out


class StreamerOpts(C.Structure):
    _fields_ = [("mobility", C.c_double), ("charge_scale", C.c_double), ("alpha_a", C.c_double),
                ("alpha_b", C.c_double), ("cfl", C.c_double), ("tol", C.c_double),
                ("maxit", C.c_int32), ("restart", C.c_int32), ("matrix_free", C.c_int32),
                ("pad_", C.c_int32)]


class StreamerInfo(C.Structure):
    _fields_ = [("steps", C.c_int32), ("iterations_max", C.c_int32), ("iterations_sum", C.c_int64),
                ("time", C.c_double), ("last_dt", C.c_double)]


class _NnOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("init_scale", C.c_double)]


class _TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("loss", C.c_int32), ("seed", C.c_uint64),
                ("lr", C.c_double), ("lr_min", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double)]


class _TrainInfo(C.Structure):
    _fields_ = [("steps", C.c_int64), ("loss_first", C.c_double), ("loss_last", C.c_double),
                ("ms", C.c_double)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_2203_00925_amd.build` (no fallback exists)")
    lib = C.CDLL(_LIB_PATH)
    P, I32, I64, D, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    sig = {
        "mifvm_last_error": (C.c_char_p, []),
        "mifvm_version": (C.c_char_p, []),
        "mifvm_mesh_preprocess": (C.c_int, [P, I64, P, I64, P, P, I64, P, C.POINTER(P)]),
        "mifvm_mesh_get_info": (C.c_int, [P, C.POINTER(MeshInfo)]),
        "mifvm_mesh_destroy": (None, [P]),
        "mifvm_mesh_export": (C.c_int, [P, I32, P, SZ]),
        "mifvm_state_create": (C.c_int, [P, C.POINTER(_Params), P, SZ, P, C.POINTER(P)]),
        "mifvm_state_destroy": (None, [P]),
        "mifvm_set_bc": (C.c_int, [P, I32, I32, I32, D]),
        "mifvm_set_bc_values": (C.c_int, [P, I32, I32, P, P]),
        "mifvm_set_diffusivity": (C.c_int, [P, D]),
        "mifvm_set_mesh_diffusivity": (C.c_int, [P, P, I32]),
        "mifvm_mesh_values": (C.c_int, [P, I32, P, I32]),
        "mifvm_set_field": (C.c_int, [P, I32, P, I32, P]),
        "mifvm_get_field": (C.c_int, [P, I32, P, I32, P]),
        "mifvm_cfl_dt": (C.c_int, [P, D, C.POINTER(D), P]),
        "mifvm_step": (C.c_int, [P, I32, D, P]),
        "mifvm_residual": (C.c_int, [P, P, P, P, P, P, P]),
        "mifvm_conservation": (C.c_int, [P, C.POINTER(D), P]),
        "mifvm_poisson_assemble": (C.c_int, [P, P]),
        "mifvm_poisson_apply": (C.c_int, [P, P, P, P]),
        "mifvm_poisson_apply_free": (C.c_int, [P, P, P, P]),
        "mifvm_fgmres_bytes": (C.c_int, [P, I32, C.POINTER(SZ)]),
        "mifvm_fgmres_attach": (C.c_int, [P, I32, P, SZ]),
        "mifvm_poisson_rhs": (C.c_int, [P, P, P, P]),
        "mifvm_poisson_solve": (C.c_int, [P, P, C.POINTER(SolveOpts), C.POINTER(SolveInfo), P]),
        "mifvm_kernel_timing": (C.c_int, [P, I32]),
        "mifvm_kernel_timing_select": (C.c_int, [P, C.c_uint64]),
        "mifvm_step_graph": (C.c_int, [P, I32, D, P]),
        "mifvm_autotune": (C.c_int, [P, C.c_char_p, C.POINTER(TuneInfo), P]),
        "mifvm_batch_bytes": (C.c_int, [P, C.POINTER(SZ)]),
        "mifvm_batch_create": (C.c_int, [P, C.POINTER(BatchOpts), P, SZ, P, C.POINTER(P)]),
        "mifvm_batch_destroy": (None, [P]),
        "mifvm_batch_set_schedule": (C.c_int, [P, C.POINTER(BatchOpts), P]),
        "mifvm_batch_get_schedule": (C.c_int, [P, C.POINTER(BatchOpts)]),
        "mifvm_batch_solve": (C.c_int, [P, C.POINTER(BatchSolveOpts), C.POINTER(BatchInfo), P]),
        "mifvm_batch_run": (C.c_int, [P, I32, C.POINTER(BatchSolveOpts), C.POINTER(BatchInfo), P]),
        "mifvm_batch_autotune": (C.c_int, [P, C.c_char_p, I32, C.POINTER(BatchTuneInfo), P]),
        "mifvm_kernel_stats": (C.c_int, [P, I32, C.POINTER(D), C.POINTER(I64), P]),
        "mifvm_nn_workspace_bytes": (SZ, []),
        "mifvm_nn_create": (C.c_int, [C.POINTER(_NnOpts), P, SZ, P, C.POINTER(P)]),
        "mifvm_nn_destroy": (None, [P]),
        "mifvm_nn_get_params": (C.c_int, [P, P, I64, P]),
        "mifvm_nn_set_params": (C.c_int, [P, P, I64, P]),
        "mifvm_nn_save": (C.c_int, [P, P, C.POINTER(SZ), P]),
        "mifvm_nn_load": (C.c_int, [P, P, SZ, P]),
        "mifvm_nn_attach_bytes": (C.c_int, [P, I32, C.POINTER(SZ)]),
        "mifvm_nn_attach": (C.c_int, [P, P, I32, P, SZ, P]),
        "mifvm_nn_apply": (C.c_int, [P, P, P, P]),
        "mifvm_nn_apply_layers": (C.c_int, [P, P, P, P]),
        "mifvm_nn_form": (C.c_int, [P, I32, C.POINTER(I32), C.POINTER(C.c_float), C.POINTER(C.c_float)]),
        "mifvm_nn_sample": (C.c_int, [P, P, C.POINTER(D), P]),
        "mifvm_nn_loss_grad": (C.c_int, [P, P, I32, C.POINTER(D), P, P]),
        "mifvm_nn_train": (C.c_int, [P, P, I32, P, P, I32, C.POINTER(_TrainOpts),
                                     C.POINTER(_TrainInfo), P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc, allow=(OK,)):
    if rc not in allow:
        raise MifvmError(rc, _lib.mifvm_last_error().decode())
    return rc


def _ptr(a):
    """Device pointer of a torch tensor (or None)."""
    return None if a is None else C.c_void_p(a.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Mesh:
    """Host-side preprocessed mesh (mifvm_mesh_preprocess)."""

    def __init__(self, xyz, tets, btris, btags, renumber=RENUMBER_MORTON, mesh_cell_start=None,
                 no_matrix=False):
        xyz = np.ascontiguousarray(xyz, np.float64)
        tets = np.ascontiguousarray(tets, np.int32)
        btris = np.ascontiguousarray(btris, np.int32)
        btags = np.ascontiguousarray(btags, np.int32)
        h = C.c_void_p()
        if mesh_cell_start is not None:
            starts = np.ascontiguousarray(mesh_cell_start, np.int64)
            opts = _MeshOpts(renumber, len(starts) - 1, starts.ctypes.data, int(no_matrix), 0)
        else:
            starts = None
            opts = _MeshOpts(renumber, 1, None, int(no_matrix), 0)
        _check(_lib.mifvm_mesh_preprocess(
            xyz.ctypes.data, len(xyz), tets.ctypes.data, len(tets),
            btris.ctypes.data, btags.ctypes.data, len(btags), C.byref(opts), C.byref(h)))
        self._h = h
        self.info = MeshInfo()
        _check(_lib.mifvm_mesh_get_info(h, C.byref(self.info)))

    @classmethod
    def from_cube(cls, m, renumber=RENUMBER_MORTON, no_matrix=False):
        return cls(m.xyz, m.tets, m.btris, m.btags, renumber, no_matrix=no_matrix)

    @classmethod
    def from_batch(cls, meshes, renumber=RENUMBER_MORTON, no_matrix=False):
        """Independent meshes as one batch: vertex ids of mesh k are offset by
        the vertices of meshes 0..k-1; cells stay in mesh order."""
        voff = np.cumsum([0] + [m.nv for m in meshes])
        coff = np.cumsum([0] + [m.nc for m in meshes])
        xyz = np.concatenate([m.xyz for m in meshes])
        tets = np.concatenate([m.tets + voff[k] for k, m in enumerate(meshes)])
        btris = np.concatenate([m.btris + voff[k] for k, m in enumerate(meshes)])
        btags = np.concatenate([m.btags for m in meshes])
        return cls(xyz, tets, btris, btags, renumber, mesh_cell_start=coff, no_matrix=no_matrix)

    def export(self, name):
        what = EXPORT_IDS[name]
        _, dt, shape = EXPORTS[what]
        out = np.empty(shape(self.info), dt)
        _check(_lib.mifvm_mesh_export(self._h, what, out.ctypes.data, out.nbytes))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.mifvm_mesh_destroy(h)
            self._h = None


class State:
    """Device-resident mesh and fields (mifvm_state_create); the workspace is
    a torch uint8 tensor on the current device."""

    def __init__(self, mesh: Mesh, diffusivity=0.0, device="cuda", stream=None, precision=FP64):
        import torch
        self.mesh = mesh
        nbytes = int(mesh.info.ws_bytes)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self._off = (-base) % 256
        h = C.c_void_p()
        params = _Params(float(diffusivity), int(precision), 0)
        _check(_lib.mifvm_state_create(mesh._h, C.byref(params), C.c_void_p(base + self._off),
                                       nbytes, _stream(stream), C.byref(h)))
        self._h = h
        self.device = device

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.mifvm_state_destroy(h)
            self._h = None

    # -- boundary conditions and fields --------------------------------------
    def set_bc(self, var, tag, kind, value=0.0):
        _check(_lib.mifvm_set_bc(self._h, var, tag, kind, float(value)))

    def set_bcs(self, var, kinds, values=None):
        values = values if values is not None else [0.0] * len(kinds)
        for t, (k, v) in enumerate(zip(kinds, values)):
            self.set_bc(var, t, k, v)

    def set_bc_values(self, var, tag, vals, stream=None):
        """Per-face values of one tag: one float64 per boundary triangle of
        the mesh, in the order given to the mesh."""
        import torch
        t = torch.as_tensor(vals).to(device=self.device, dtype=torch.float64).contiguous()
        _check(_lib.mifvm_set_bc_values(self._h, var, tag, _ptr(t), _stream(stream)))
        (stream or torch.cuda.current_stream()).synchronize()   # t may be a temporary

    def set_diffusivity(self, D):
        _check(_lib.mifvm_set_diffusivity(self._h, float(D)))

    def set_mesh_diffusivity(self, Ds):
        a = np.ascontiguousarray(Ds, np.float64)
        _check(_lib.mifvm_set_mesh_diffusivity(self._h, a.ctypes.data, len(a)))

    def mesh_values(self, what):
        """Per-mesh results: 'dt', 'conservation', 'iterations', 'rel_residual'."""
        ids = {"dt": 0, "conservation": 1, "iterations": 2, "rel_residual": 3}
        out = np.empty(self.mesh.info.nmeshes, np.float64)
        _check(_lib.mifvm_mesh_values(self._h, ids[what], out.ctypes.data, len(out)))
        return out

    def set_field(self, field, t, stream=None):
        """A float32 tensor crosses the ABI as float32, anything else as float64."""
        import torch
        dt = torch.float32 if t.dtype == torch.float32 else torch.float64
        t = t.to(device=self.device, dtype=dt).contiguous()
        code = F32 if dt == torch.float32 else F64
        _check(_lib.mifvm_set_field(self._h, field, _ptr(t), code, _stream(stream)))
        (stream or torch.cuda.current_stream()).synchronize()   # t may be a temporary

    def get_field(self, field, stream=None, dtype=None):
        import torch
        dtype = dtype or torch.float64
        n = self.mesh.info.nc * (3 if field in (FIELD_VEL, FIELD_EFIELD) else 1)
        out = torch.empty(n, dtype=dtype, device=self.device)
        code = F32 if dtype == torch.float32 else F64
        _check(_lib.mifvm_get_field(self._h, field, _ptr(out), code, _stream(stream)))
        return out

    # -- step ------------------------------------------------------------------
    def cfl_dt(self, cfl, stream=None):
        dt = C.c_double()
        _check(_lib.mifvm_cfl_dt(self._h, float(cfl), C.byref(dt), _stream(stream)))
        return dt.value

    def step(self, n_steps, dt, stream=None):
        _check(_lib.mifvm_step(self._h, int(n_steps), float(dt), _stream(stream)))

    def step_graph(self, n_steps, dt, stream=None):
        _check(_lib.mifvm_step_graph(self._h, int(n_steps), float(dt), _stream(stream)))

    def norm_l2(self, field, exact=None, stream=None):
        """sqrt(sum mu_i (a_i - e_i)^2) of a field against `exact` (user order)."""
        import torch
        e = None if exact is None else exact.to(device=self.device, dtype=torch.float64).contiguous()
        out = C.c_double()
        _check(_lib.mifvm_norm_l2(self._h, int(field), _ptr(e), C.byref(out), _stream(stream)))
        return out.value

    def streamer_step(self, n_steps, mobility, charge_scale, alpha_a=0.0, alpha_b=0.0, cfl=0.4,
                      tol=1e-10, maxit=0, restart=0, matrix_free=False, stream=None):
        """Coupled loop (mifvm_streamer_step): n_e = FIELD_U, n_p = FIELD_ION,
        P = FIELD_P; returns the step count, CG iterations and simulated time."""
        opts = StreamerOpts(float(mobility), float(charge_scale), float(alpha_a), float(alpha_b),
                            float(cfl), float(tol), int(maxit), int(restart), 1 if matrix_free else 0, 0)
        info = StreamerInfo()
        _check(_lib.mifvm_streamer_step(self._h, int(n_steps), C.byref(opts), C.byref(info),
                                        _stream(stream)))
        return {"steps": info.steps, "iterations_max": info.iterations_max,
                "iterations_sum": info.iterations_sum, "time": info.time, "last_dt": info.last_dt}

    def autotune(self, cache_path=None, stream=None):
        info = TuneInfo()
        path = cache_path.encode() if cache_path else None
        _check(_lib.mifvm_autotune(self._h, path, C.byref(info), _stream(stream)))
        return {f: getattr(info, f) for f, _ in TuneInfo._fields_}

    def residual(self, stream=None):
        import torch
        i = self.mesh.info
        kw = dict(dtype=torch.float64, device=self.device)
        res = torch.empty(i.nc, **kw)
        grad = torch.empty(3 * i.nc, **kw)
        psi = torch.empty(i.nc, **kw)
        un = torch.empty(i.nv, **kw)
        flux = torch.empty(i.nf, **kw)
        _check(_lib.mifvm_residual(self._h, _ptr(res), _ptr(grad), _ptr(psi), _ptr(un),
                                   _ptr(flux), _stream(stream)))
        return dict(res=res, grad=grad.view(3, i.nc), psi=psi, u_node=un, flux=flux)

    def conservation(self, stream=None):
        t = C.c_double()
        _check(_lib.mifvm_conservation(self._h, C.byref(t), _stream(stream)))
        return t.value

    # -- Poisson -----------------------------------------------------------------
    def poisson_assemble(self, stream=None):
        _check(_lib.mifvm_poisson_assemble(self._h, _stream(stream)))

    def poisson_apply(self, x, stream=None):
        import torch
        x = x.to(device=self.device, dtype=torch.float64).contiguous()
        y = torch.empty_like(x)
        _check(_lib.mifvm_poisson_apply(self._h, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def fgmres_attach(self, m=30):
        """Workspace for method SOLVE_FGMRES with cycles of m steps."""
        import torch
        n = C.c_size_t()
        _check(_lib.mifvm_fgmres_bytes(self._h, int(m), C.byref(n)))
        ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        _check(_lib.mifvm_fgmres_attach(self._h, int(m), C.c_void_p(ws.data_ptr() + off), n.value))
        self._gm_ws = ws

    def amg_build(self, theta=0.0, omega=0.0, max_levels=0, coarse_max=0, cycle=0, stream=None):
        """Multigrid hierarchy of the assembled K, uploaded into a workspace
        this object keeps (mifvm_amg_build + mifvm_amg_attach); cycle: 0 or
        CYCLE_V, or CYCLE_W."""
        import torch
        opts = AmgOpts(float(theta), float(omega), int(max_levels), int(coarse_max), int(cycle), 0)
        info = AmgInfo()
        _check(_lib.mifvm_amg_build(self._h, C.byref(opts), C.byref(info), _stream(stream)))
        ws = torch.empty(int(info.ws_bytes) + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        _check(_lib.mifvm_amg_attach(self._h, C.c_void_p(ws.data_ptr() + off), C.c_size_t(info.ws_bytes),
                                     _stream(stream)))
        self._amg_ws = ws
        return _amg_info(info)

    def amg_apply(self, r, learned_smoother=False, stream=None):
        """z = V(r), one multigrid cycle (user cell order)."""
        import torch
        r = r.to(device=self.device, dtype=torch.float64).contiguous()
        z = torch.empty_like(r)
        _check(_lib.mifvm_amg_apply(self._h, 1 if learned_smoother else 0, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def poisson_apply_free(self, x, stream=None):
        """K x from the discretisation (no stored matrix)."""
        import torch
        x = x.to(device=self.device, dtype=torch.float64).contiguous()
        y = torch.empty_like(x)
        _check(_lib.mifvm_poisson_apply_free(self._h, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def poisson_rhs(self, f=None, stream=None):
        import torch
        y = torch.empty(self.mesh.info.nc, dtype=torch.float64, device=self.device)
        if f is not None:
            f = f.to(device=self.device, dtype=torch.float64).contiguous()
        _check(_lib.mifvm_poisson_rhs(self._h, _ptr(f), _ptr(y), _stream(stream)))
        return y

    def poisson_solve(self, f=None, tol=1e-10, maxit=20000, chunk=0, restart=500,
                      history=0, method=SOLVE_PLAIN, inner_tol=1e-4, graph=-1, stream=None,
                      allow_not_converged=False, stall_window=0, learned_maxit=0,
                      allow_fell_back=False, matrix_free=False, learned_smoother=False):
        """chunk 0 / graph -1: the autotuned schedule (32 iterations per host
        check, direct launches when not tuned)."""
        import torch
        if f is not None:
            f = f.to(device=self.device, dtype=torch.float64).contiguous()
        hist = (C.c_double * max(int(history), 1))()
        opts = SolveOpts(float(tol), int(maxit), int(chunk), int(restart), int(history), hist,
                         int(method), int(graph), float(inner_tol), int(stall_window),
                         int(learned_maxit), 1 if matrix_free else 0, 1 if learned_smoother else 0)
        info = SolveInfo()
        allow = (OK,) + ((NOT_CONVERGED,) if allow_not_converged else ()) + \
            ((FELL_BACK,) if allow_fell_back else ())
        rc = _check(_lib.mifvm_poisson_solve(self._h, _ptr(f), C.byref(opts), C.byref(info),
                                             _stream(stream)), allow)
        return dict(status=rc, iterations=info.iterations, restarts=info.restarts,
                    outer=info.outer, rel_residual=info.rel_residual, ms=info.ms,
                    history=list(hist[:info.history_len]), fell_back=info.fell_back,
                    learned_iterations=info.learned_iterations)

    # -- per-kernel timing ----------------------------------------------------------
    def kernel_timing(self, enable=True, only=None):
        """Per-kernel event timing on or off; `only`: the kernel names (from
        KERNELS) that get events, the others launch untimed."""
        if only is None:
            _check(_lib.mifvm_kernel_timing(self._h, 1 if enable else 0))
            return
        mask = 0
        for name in only:
            mask |= 1 << KERNELS.index(name)
        _check(_lib.mifvm_kernel_timing_select(self._h, C.c_uint64(mask if enable else 0)))

    def kernel_stats(self, stream=None):
        """{kernel: (total_ms, launches)} since timing was enabled (synchronises)."""
        out = {}
        for k, name in enumerate(KERNELS):
            ms, n = C.c_double(), C.c_int64()
            _check(_lib.mifvm_kernel_stats(self._h, k, C.byref(ms), C.byref(n), _stream(stream)))
            out[name] = (ms.value, n.value)
        return out


BQ_ROTATE, BQ_XCD, BQ_LARGEST, BQ_LAUNCHES = 0, 1, 2, 3


class Batch:
    """Persistent batched solve of every mesh of a multi-mesh state
    (mifvm_batch_*); the workspace is a torch uint8 tensor."""

    def __init__(self, state, item_rows=0, grid=0, policy=-1, spin_limit=0, vertex_batch=0, chunk=0,
                 stream=None):
        import torch
        self.state = state
        n = C.c_size_t()
        _check(_lib.mifvm_batch_bytes(state._h, C.byref(n)))
        self.ws = torch.empty(n.value + 256, dtype=torch.uint8, device=state.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        h = C.c_void_p()
        opts = BatchOpts(int(item_rows), int(grid), int(policy), int(spin_limit), int(vertex_batch), int(chunk))
        _check(_lib.mifvm_batch_create(state._h, C.byref(opts), C.c_void_p(base + off), n.value,
                                       _stream(stream), C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.mifvm_batch_destroy(h)
            self._h = None

    def schedule(self):
        o = BatchOpts()
        _check(_lib.mifvm_batch_get_schedule(self._h, C.byref(o)))
        return {"item_rows": o.item_rows, "grid": o.grid, "policy": o.policy, "spin_limit": o.spin_limit,
                "vertex_batch": o.vertex_batch, "chunk": o.chunk}

    def set_schedule(self, item_rows=0, grid=0, policy=-1, spin_limit=0, vertex_batch=0, chunk=0, stream=None):
        o = BatchOpts(int(item_rows), int(grid), int(policy), int(spin_limit), int(vertex_batch), int(chunk))
        _check(_lib.mifvm_batch_set_schedule(self._h, C.byref(o), _stream(stream)))

    @staticmethod
    def _info(rc, info):
        return dict(status=rc, solves=info.solves, iterations_max=info.iterations_max,
                    iterations_sum=info.iterations_sum, iterations_mean=info.iterations_mean,
                    rel_residual_max=info.rel_residual_max, ms=info.ms)

    def solve(self, tol=1e-10, maxit=20000, restart=500, stream=None, allow_not_converged=False):
        o = BatchSolveOpts(float(tol), int(maxit), int(restart), 1, 0)
        info = BatchInfo()
        allow = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        rc = _check(_lib.mifvm_batch_solve(self._h, C.byref(o), C.byref(info), _stream(stream)), allow)
        return self._info(rc, info)

    def run(self, n_steps, tol=1e-10, maxit=20000, restart=500, solve_every=1, stream=None):
        o = BatchSolveOpts(float(tol), int(maxit), int(restart), int(solve_every), 0)
        info = BatchInfo()
        rc = _check(_lib.mifvm_batch_run(self._h, int(n_steps), C.byref(o), C.byref(info), _stream(stream)))
        return self._info(rc, info)

    def autotune(self, cache_path=None, iterations=0, stream=None):
        info = BatchTuneInfo()
        path = cache_path.encode() if cache_path else None
        _check(_lib.mifvm_batch_autotune(self._h, path, int(iterations), C.byref(info), _stream(stream)))
        return {f: getattr(info, f) for f, _ in BatchTuneInfo._fields_}


class Network:
    """Learned preconditioner (mifvm_nn_*): parameters in a torch uint8
    workspace on the current device."""

    def __init__(self, seed=0, init_scale=1.0, device="cuda", stream=None):
        import torch
        nbytes = int(_lib.mifvm_nn_workspace_bytes())
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        h = C.c_void_p()
        _check(_lib.mifvm_nn_create(C.byref(_NnOpts(int(seed), float(init_scale))),
                                    C.c_void_p(base + off), nbytes, _stream(stream), C.byref(h)))
        self._h = h
        self.device = device
        self._attached = []

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            for st in getattr(self, "_attached", []):
                # only states still attached to this network
                if st._h and getattr(st, "_nn", None) is self:
                    _lib.mifvm_nn_attach(st._h, None, 0, None, 0, None)
            _lib.mifvm_nn_destroy(h)
            self._h = None

    def get_params(self, stream=None):
        out = np.empty(NN_PARAMS, np.float32)
        _check(_lib.mifvm_nn_get_params(self._h, out.ctypes.data, NN_PARAMS, _stream(stream)))
        return out

    def set_params(self, p, stream=None):
        p = np.ascontiguousarray(p, np.float32)
        _check(_lib.mifvm_nn_set_params(self._h, p.ctypes.data, len(p), _stream(stream)))

    def save(self, stream=None):
        n = C.c_size_t()
        _check(_lib.mifvm_nn_save(self._h, None, C.byref(n), _stream(stream)))
        buf = (C.c_char * n.value)()
        _check(_lib.mifvm_nn_save(self._h, buf, C.byref(n), _stream(stream)))
        return bytes(buf[:n.value])

    def load(self, blob, stream=None):
        buf = C.create_string_buffer(bytes(blob), len(blob))
        _check(_lib.mifvm_nn_load(self._h, buf, len(blob), _stream(stream)))

    def attach(self, state, training=False, stream=None):
        """Attach to a single-mesh state; the per-state buffers are kept on
        the state object."""
        import torch
        n = C.c_size_t()
        _check(_lib.mifvm_nn_attach_bytes(state._h, 1 if training else 0, C.byref(n)))
        ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        _check(_lib.mifvm_nn_attach(state._h, self._h, 1 if training else 0,
                                    C.c_void_p(ws.data_ptr() + off), n.value, _stream(stream)))
        state._nn_ws = ws
        state._nn = self
        self._attached.append(state)

    def train(self, states, samples, state_of_sample, epochs=1, lr=1e-3, lr_min=1e-4, seed=0,
              beta1=0.9, beta2=0.999, eps=1e-8, loss=LOSS_RESIDUAL, stream=None):
        """samples: list of FP32 device tensors from State.nn_sample."""
        states = list(states)
        hs = (C.c_void_p * len(states))(*[s._h for s in states])
        ptrs = (C.c_void_p * len(samples))(*[t.data_ptr() for t in samples])
        sos = np.ascontiguousarray(state_of_sample, np.int32)
        opts = _TrainOpts(int(epochs), int(loss), int(seed), float(lr), float(lr_min), float(beta1),
                          float(beta2), float(eps))
        info = _TrainInfo()
        ep = np.zeros(int(epochs), np.float64)
        _check(_lib.mifvm_nn_train(self._h, hs, len(states), ptrs, sos.ctypes.data, len(samples),
                                   C.byref(opts), C.byref(info), ep.ctypes.data, _stream(stream)))
        return dict(steps=info.steps, loss_first=info.loss_first, loss_last=info.loss_last,
                    ms=info.ms, epoch_loss=ep)


def _state_nn_apply(self, r, stream=None, layers=False):
    """z = network(r), FP64 user order (layers: the layer-by-layer form)."""
    import torch
    r = r.to(device=self.device, dtype=torch.float64).contiguous()
    z = torch.empty_like(r)
    fn = _lib.mifvm_nn_apply_layers if layers else _lib.mifvm_nn_apply
    _check(fn(self._h, _ptr(r), _ptr(z), _stream(stream)))
    return z


def _state_nn_sample(self, out=None, stream=None):
    """(FP32 internal-order sample of the current true residual, its RMS)."""
    import torch
    if out is None:
        out = torch.empty(self.mesh.info.nc, dtype=torch.float32, device=self.device)
    rms = C.c_double()
    _check(_lib.mifvm_nn_sample(self._h, _ptr(out), C.byref(rms), _stream(stream)))
    return out, rms.value


def _state_nn_loss_grad(self, sample, loss_kind=LOSS_RESIDUAL, stream=None):
    loss = C.c_double()
    grad = np.empty(NN_PARAMS, np.float32)
    _check(_lib.mifvm_nn_loss_grad(self._h, _ptr(sample), int(loss_kind), C.byref(loss),
                                   grad.ctypes.data, _stream(stream)))
    return loss.value, grad


def _state_nn_form(self, form=-1):
    """Select the network's forward form (NN_FORM_AUTO / _LAYERS / _FUSED;
    -1 leaves it) and return (form in use, ms layers, ms fused)."""
    chosen, ml, mf = C.c_int32(), C.c_float(), C.c_float()
    _check(_lib.mifvm_nn_form(self._h, int(form), C.byref(chosen), C.byref(ml), C.byref(mf)))
    return chosen.value, ml.value, mf.value


State.nn_apply = _state_nn_apply
State.nn_form = _state_nn_form
State.nn_sample = _state_nn_sample
State.nn_loss_grad = _state_nn_loss_grad
