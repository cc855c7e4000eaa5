"""ctypes binding of libnnms (include/nnms.h): argument marshalling only.

Every step of the solve runs inside the library's HIP kernels.  PyTorch is
used, when requested, only as the device allocator and for streams.  If the
built library is missing, importing this module raises: there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnnms.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2412_08981_amd.build.build() first")
# One HIP runtime per process.  PyTorch ships its own libamdhip64 and links it
# by a name that does not match the soname this library asks for, so loading
# this library first would bring in a second runtime, and whichever of the two
# opens the device last gets no device.  Loading PyTorch first makes this
# library bind to PyTorch's runtime (same soname).
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = C.CDLL(LIB_PATH)

MAX_LEVELS = 8
MAX_RESTART = 64
FP64, MIXED = 0, 1
BARYCENTRIC, MLS = 0, 1  # transfer between levels
LU, ILU = 0, 1  # subdomain solver of the smoother
SWEEPS, INVERSE = 0, 1  # how dense-LU subdomain solves are applied
DEVICE_PTRS, NO_GRAPH = 1, 2

STATUS = {
    0: "OK", 1: "INVALID_ARG", 2: "BAD_MESH", 3: "POINT_LOCATION", 4: "OUT_OF_MEMORY", 5: "BUDGET",
    6: "SINGULAR", 7: "NOT_CONVERGED", 8: "DEVICE", 9: "IN_USE",
}


class NNMSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class setup_opts(C.Structure):
    _fields_ = [("nparts", C.c_int32 * MAX_LEVELS), ("overlap", C.c_int32), ("its", C.c_int32),
                ("precision", C.c_int32), ("transfer", C.c_int32), ("mls_alpha", C.c_double),
                ("subsolver", C.c_int32), ("ilu_fill", C.c_int32 * MAX_LEVELS), ("mls_restrict", C.c_int32),
                ("ncomp", C.c_int32), ("mls_clip", C.c_int32), ("dense_apply", C.c_int32)]


class level_info(C.Structure):
    _fields_ = [("nv", C.c_int64), ("nt", C.c_int64), ("ninterior", C.c_int64), ("nnz", C.c_int64),
                ("nparts", C.c_int32), ("max_block", C.c_int32), ("min_block", C.c_int32), ("transfer", C.c_int32),
                ("s_total", C.c_int64), ("factor_elems", C.c_int64), ("p_nnz", C.c_int64),
                ("subsolver", C.c_int32), ("mls_restrict", C.c_int32), ("ilu_nnz", C.c_int64),
                ("r_nnz", C.c_int64), ("ncomp", C.c_int32), ("dense_apply", C.c_int32), ("ndof", C.c_int64)]


class kappa_t(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ncentres", C.c_int32), ("value", C.c_double),
                ("centres", C.POINTER(C.c_double)), ("mu", C.POINTER(C.c_double)), ("width", C.c_double),
                ("per_tet", C.POINTER(C.POINTER(C.c_double)))]


class rhs_t(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("value", C.c_double),
                ("values", C.POINTER(C.c_double)), ("vector", C.c_double * 3)]


class assemble_opts_t(C.Structure):
    _fields_ = [("kappa", C.POINTER(kappa_t)), ("rhs", C.POINTER(rhs_t)), ("restart_cap", C.c_int32),
                ("reserved", C.c_int32), ("max_device_bytes", C.c_int64), ("poisson_ratio", C.c_double)]


class solve_opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_it", C.c_int32), ("rtol", C.c_double), ("flags", C.c_int32),
                ("reserved", C.c_int32)]


class solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("cycles", C.c_int32), ("status", C.c_int32), ("running", C.c_int32),
                ("relres", C.c_double)]


class tuning_t(C.Structure):
    _fields_ = [("spmv_lanes", C.c_int32 * MAX_LEVELS), ("pt_lanes", C.c_int32 * MAX_LEVELS),
                ("ras_groups", C.c_int32 * MAX_LEVELS), ("ras_blocks", C.c_int32 * MAX_LEVELS),
                ("krylov_lanes", C.c_int32), ("tuned", C.c_int32)]

    def to_dict(self):
        return {"spmv_lanes": list(self.spmv_lanes), "pt_lanes": list(self.pt_lanes),
                "ras_groups": list(self.ras_groups), "ras_blocks": list(self.ras_blocks),
                "krylov_lanes": int(self.krylov_lanes), "tuned": int(self.tuned)}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        for k in ("spmv_lanes", "pt_lanes", "ras_groups", "ras_blocks"):
            for i, v in enumerate(d.get(k, [1] * MAX_LEVELS)):
                getattr(t, k)[i] = int(v)
        t.krylov_lanes, t.tuned = int(d["krylov_lanes"]), int(d.get("tuned", 1))
        return t


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class allocator_t(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


vp = C.c_void_p
_sig = {
    "nnms_last_error": (C.c_char_p, []),
    "nnms_device_bytes_in_use": (C.c_int64, []),
    "nnms_mesh_create": (C.c_int, [C.c_int64, vp, C.c_int64, vp, vp, C.POINTER(vp)]),
    "nnms_mesh_destroy": (None, [vp]),
    "nnms_mesh_coarsen": (C.c_int, [vp, C.c_int32, C.c_uint64, C.POINTER(vp), C.POINTER(C.c_int64)]),
    "nnms_mesh_read": (C.c_int, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp, vp, vp]),
    "nnms_setup_opts_default": (C.c_int, [C.POINTER(setup_opts)]),
    "nnms_hierarchy_setup": (C.c_int, [vp, C.c_int32, C.POINTER(setup_opts), C.POINTER(allocator_t), vp, C.POINTER(vp)]),
    "nnms_hierarchy_setup_host": (C.c_int, [vp, C.c_int32, C.POINTER(setup_opts), C.POINTER(vp)]),
    "nnms_hierarchy_destroy": (C.c_int, [vp]),
    "nnms_hierarchy_level_info": (C.c_int, [vp, C.c_int32, C.POINTER(level_info)]),
    "nnms_hierarchy_csr": (C.c_int, [vp, C.c_int32, vp, vp]),
    "nnms_hierarchy_partition": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
    "nnms_hierarchy_transfer": (C.c_int, [vp, C.c_int32, vp, vp]),
    "nnms_hierarchy_transfer_csr": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
    "nnms_hierarchy_ilu_pattern": (C.c_int, [vp, C.c_int32, vp, vp]),
    "nnms_hierarchy_restriction_csr": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
    "nnms_system_ilu_values": (C.c_int, [vp, C.c_int32, vp]),
    "nnms_hierarchy_system_bytes": (C.c_int64, [vp, C.c_int32]),
    "nnms_assemble": (C.c_int, [vp, C.POINTER(kappa_t), C.c_double, vp, C.POINTER(vp)]),
    "nnms_assemble_ex": (C.c_int, [vp, C.POINTER(assemble_opts_t), vp, C.POINTER(vp)]),
    "nnms_system_destroy": (C.c_int, [vp]),
    "nnms_system_device_bytes": (C.c_int64, [vp]),
    "nnms_system_rhs": (C.c_int, [vp, vp]),
    "nnms_system_matrix": (C.c_int, [vp, C.c_int32, vp]),
    "nnms_apply_operator": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
    "nnms_apply_smoother": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
    "nnms_apply_prolong": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
    "nnms_apply_restrict": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
    "nnms_apply_vcycle": (C.c_int, [vp, vp, vp, vp]),
    "nnms_apply_smoother_noalloc": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
    "nnms_solve_opts_default": (C.c_int, [C.POINTER(solve_opts)]),
    "nnms_solve": (C.c_int, [vp, vp, vp, C.POINTER(solve_opts), C.POINTER(solve_info), vp]),
    "nnms_solve_batch": (C.c_int, [vp, C.c_int32, vp, vp, C.POINTER(solve_opts), C.POINTER(solve_info), vp]),
    "nnms_batch_create": (C.c_int, [vp, C.c_int32, C.POINTER(solve_opts), vp, C.POINTER(vp)]),
    "nnms_batch_start": (C.c_int, [vp, C.c_int32, vp]),
    "nnms_batch_step": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_int32)]),
    "nnms_batch_result": (C.c_int, [vp, C.c_int32, vp, C.POINTER(solve_info)]),
    "nnms_batch_destroy": (C.c_int, [vp]),
    "nnms_time_kernel": (C.c_int, [vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double)]),
    "nnms_system_factor": (C.c_int, [vp, C.c_int32, C.c_int32, vp, vp, C.POINTER(C.c_int32)]),
    "nnms_system_factor_pairs": (C.c_int, [vp, C.c_int32, C.c_int32, vp, vp, C.POINTER(C.c_int32)]),
    "nnms_system_inverse_panels": (C.c_int, [vp, C.c_int32, C.c_int32, vp, C.POINTER(C.c_int32),
                                             C.POINTER(C.c_int32)]),
    "nnms_hierarchy_get_tuning": (C.c_int, [vp, C.POINTER(tuning_t)]),
    "nnms_hierarchy_set_tuning": (C.c_int, [vp, C.POINTER(tuning_t)]),
    "nnms_autotune": (C.c_int, [vp, C.c_int32, C.POINTER(tuning_t)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_sig)


def last_error() -> str:
    return _lib.nnms_last_error().decode()


def _check(code: int, ok=(0,)):
    if code not in ok:
        raise NNMSError(code, last_error())
    return code


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def device_bytes_in_use() -> int:
    return int(_lib.nnms_device_bytes_in_use())


# ---------------------------------------------------------------------------
class Mesh:
    """nnms_mesh_create / nnms_mesh_destroy."""

    def __init__(self, xyz: np.ndarray, tets: np.ndarray, dirichlet: Optional[np.ndarray] = None):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
        h = C.c_void_p()
        _check(_lib.nnms_mesh_create(xyz.shape[0], _ptr(xyz), tets.shape[0], _ptr(tets),
                                     None if d is None else _ptr(d), C.byref(h)))
        self.handle = h
        self.nv = xyz.shape[0]

    @classmethod
    def from_workload(cls, m) -> "Mesh":
        return cls(m.xyz, m.tets, m.dirichlet)

    def coarsen(self, rounds: int = 8, seed: int = 0):
        """Algorithm 1: (coarse Mesh, number of removed vertices)."""
        h = C.c_void_p()
        removed = C.c_int64()
        _check(_lib.nnms_mesh_coarsen(self.handle, rounds, C.c_uint64(seed & (2 ** 64 - 1)), C.byref(h),
                                      C.byref(removed)))
        m = Mesh.__new__(Mesh)
        m.handle = h
        nv = C.c_int64()
        _check(_lib.nnms_mesh_read(h, C.byref(nv), None, None, None, None))
        m.nv = nv.value
        return m, removed.value

    def read(self):
        """(xyz [nv,3], tets [nt,4], dirichlet [nv]) of the mesh."""
        nv, nt = C.c_int64(), C.c_int64()
        _check(_lib.nnms_mesh_read(self.handle, C.byref(nv), C.byref(nt), None, None, None))
        xyz = np.empty((nv.value, 3))
        tets = np.empty((nt.value, 4), dtype=np.int32)
        d = np.empty(nv.value, dtype=np.uint8)
        _check(_lib.nnms_mesh_read(self.handle, None, None, _ptr(xyz), _ptr(tets), _ptr(d)))
        return xyz, tets, d

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:  # _lib is None at interpreter exit
            _lib.nnms_mesh_destroy(self.handle)
            self.handle = None


def _torch_allocator():
    import torch

    def _alloc(n, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(n))
        except Exception:
            return None

    def _free(p, ctx):
        torch.cuda.caching_allocator_delete(p)

    fa, ff = ALLOC_FN(_alloc), FREE_FN(_free)
    return allocator_t(fa, ff, None), (fa, ff)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Hierarchy:
    """setup(hierarchy): nnms_hierarchy_setup (device) or _setup_host (host only)."""

    def __init__(self, meshes: Sequence[Mesh], nparts: Sequence[int] = (), overlap: int = 1, its: int = 3,
                 precision: int = FP64, device: bool = True, torch_alloc: bool = False, stream=None,
                 transfer: int = BARYCENTRIC, mls_alpha: float = 1.0, subsolver: int = LU,
                 ilu_fill: Sequence[int] = (), mls_restrict: bool = False, ncomp: int = 1, mls_clip: bool = False,
                 dense_apply: int = SWEEPS):
        o = setup_opts()
        _check(_lib.nnms_setup_opts_default(C.byref(o)))
        for l, p in enumerate(nparts):
            o.nparts[l] = int(p)
        o.overlap, o.its, o.precision = overlap, its, precision
        o.transfer, o.mls_alpha = transfer, mls_alpha
        o.subsolver = subsolver
        o.mls_restrict = 1 if mls_restrict else 0
        o.ncomp = int(ncomp)
        o.mls_clip = 1 if mls_clip else 0
        o.dense_apply = int(dense_apply)
        for l, k in enumerate(ilu_fill):
            o.ilu_fill[l] = int(k)
        self.meshes = list(meshes)
        arr = (C.c_void_p * len(meshes))(*[m.handle for m in meshes])
        h = C.c_void_p()
        self._keep = None
        if device:
            al = None
            if torch_alloc:
                al, self._keep = _torch_allocator()
            _check(_lib.nnms_hierarchy_setup(arr, len(meshes), C.byref(o), None if al is None else C.byref(al),
                                             _stream_ptr(stream), C.byref(h)))
        else:
            _check(_lib.nnms_hierarchy_setup_host(arr, len(meshes), C.byref(o), C.byref(h)))
        self.handle = h
        self.L = len(meshes)
        self.precision = precision

    def level_info(self, level: int) -> level_info:
        li = level_info()
        _check(_lib.nnms_hierarchy_level_info(self.handle, level, C.byref(li)))
        return li

    def csr(self, level: int):
        li = self.level_info(level)
        rp = np.empty(li.ndof + 1, dtype=np.int32)
        col = np.empty(li.nnz, dtype=np.int32)
        _check(_lib.nnms_hierarchy_csr(self.handle, level, _ptr(rp), _ptr(col)))
        return rp, col

    def partition(self, level: int):
        li = self.level_info(level)
        owner = np.empty(li.ndof, dtype=np.int32)
        s_ptr = np.empty(li.nparts + 1, dtype=np.int64)
        s_idx = np.empty(li.s_total, dtype=np.int32)
        _check(_lib.nnms_hierarchy_partition(self.handle, level, _ptr(owner), _ptr(s_ptr), _ptr(s_idx)))
        return owner, [s_idx[s_ptr[p]:s_ptr[p + 1]] for p in range(li.nparts)]

    def transfer(self, level: int):
        li = self.level_info(level)
        idx = np.empty(li.ndof * 4, dtype=np.int32)
        w = np.empty(li.ndof * 4, dtype=np.float64)
        _check(_lib.nnms_hierarchy_transfer(self.handle, level, _ptr(idx), _ptr(w)))
        return idx.reshape(-1, 4), w.reshape(-1, 4)

    def restriction_csr(self, level: int):
        """The restriction (P^T or the fine-to-coarse MLS operator) as CSR
        (row_ptr, col, w) over the coarse vertices."""
        li, lc = self.level_info(level), self.level_info(level + 1)
        rp = np.empty(lc.ndof + 1, dtype=np.int32)
        col = np.empty(li.r_nnz, dtype=np.int32)
        w = np.empty(li.r_nnz, dtype=np.float64)
        _check(_lib.nnms_hierarchy_restriction_csr(self.handle, level, _ptr(rp), _ptr(col), _ptr(w)))
        return rp, col, w

    def ilu_pattern(self, level: int):
        """(row_ptr, col) of the level's ILU patterns, subdomains concatenated."""
        li = self.level_info(level)
        rp = np.empty(li.s_total + 1, dtype=np.int32)
        col = np.empty(li.ilu_nnz, dtype=np.int32)
        _check(_lib.nnms_hierarchy_ilu_pattern(self.handle, level, _ptr(rp), _ptr(col)))
        return rp, col

    def transfer_csr(self, level: int):
        """P_level as CSR (row_ptr, col, w) over the fine unknowns."""
        li = self.level_info(level)
        rp = np.empty(li.ndof + 1, dtype=np.int32)
        col = np.empty(li.p_nnz, dtype=np.int32)
        w = np.empty(li.p_nnz, dtype=np.float64)
        _check(_lib.nnms_hierarchy_transfer_csr(self.handle, level, _ptr(rp), _ptr(col), _ptr(w)))
        return rp, col, w

    def get_tuning(self) -> dict:
        t = tuning_t()
        _check(_lib.nnms_hierarchy_get_tuning(self.handle, C.byref(t)))
        return t.to_dict()

    def set_tuning(self, d: dict):
        t = tuning_t.from_dict(d)
        _check(_lib.nnms_hierarchy_set_tuning(self.handle, C.byref(t)))

    def signature(self) -> str:
        """Identifies the hierarchy's shapes (sizes, subdomains, precision) for tuning caches."""
        parts = []
        for l in range(self.L):
            li = self.level_info(l)
            parts.append(f"{li.nv}-{li.nnz}-{li.nparts}" + (f"-c{li.ncomp}" if li.ncomp != 1 else "")
                         + (f"-mls{li.p_nnz}-{li.r_nnz}" if li.transfer == MLS else "")
                         + (f"-ilu{li.ilu_nnz}" if li.subsolver == ILU else "")
                         + ("-inv" if li.dense_apply == INVERSE else ""))
        return f"p{self.precision}_" + "_".join(parts)

    def system_bytes(self, restart: int = 30) -> int:
        return int(_lib.nnms_hierarchy_system_bytes(self.handle, restart))

    def destroy(self):
        if getattr(self, "handle", None):
            _check(_lib.nnms_hierarchy_destroy(self.handle))
            self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.nnms_hierarchy_destroy(self.handle)
            self.handle = None


def _kappa(kappa) -> tuple:
    """kappa_t of a coefficient: None or kind 'const' (value), 'loggauss'
    (centres, mu, width) or 'per_tet' (value = one array of per-tetrahedron
    values per level); the arrays it points to are returned to be kept alive."""
    k = kappa_t()
    keep = []
    kind = "const" if kappa is None else getattr(kappa, "kind", "const")
    if kind == "const":
        k.kind, k.value = 0, float(1.0 if kappa is None else kappa.value)
    elif kind == "per_tet":
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in kappa.value]
        ptrs = (C.POINTER(C.c_double) * len(arrs))(*[a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs])
        keep = [arrs, ptrs]
        k.kind, k.per_tet = 2, C.cast(ptrs, C.POINTER(C.POINTER(C.c_double)))
    else:
        c = np.ascontiguousarray(kappa.centres, dtype=np.float64).ravel()
        mu = np.ascontiguousarray(kappa.mu, dtype=np.float64)
        keep = [c, mu]
        k.kind, k.ncentres, k.width = 1, int(mu.shape[0]), float(kappa.width)
        k.centres = c.ctypes.data_as(C.POINTER(C.c_double))
        k.mu = mu.ctypes.data_as(C.POINTER(C.c_double))
    return k, keep


def _rhs(f) -> tuple:
    """rhs_t of a source term: a number (constant f) or an object with kind
    'per_tet' (one value per finest-level tetrahedron) or 'nodal' (P1 nodal
    values of the finest level) and `values`."""
    r = rhs_t()
    if isinstance(f, (int, float, np.floating)):
        r.kind, r.value = 0, float(f)
        r.vector[0] = r.vector[1] = r.vector[2] = float(f)
        return r, None
    if not hasattr(f, "kind"):  # a constant body force (three components)
        v = [float(x) for x in f]
        r.kind = 0
        r.vector[0], r.vector[1], r.vector[2] = v
        return r, None
    v = np.ascontiguousarray(f.values, dtype=np.float64)
    r.kind = {"per_tet": 1, "nodal": 2}[f.kind]
    r.values = v.ctypes.data_as(C.POINTER(C.c_double))
    return r, v


class System:
    """assemble(mesh, kappa): nnms_assemble_ex; operator applications; solve(b).

    f: a constant or a load field (see _rhs); restart_cap: Krylov columns kept
    (0 = the maximum); budget: device bytes the assembly may take (0 = no
    limit; NNMSError BUDGET beyond)."""

    def __init__(self, h: Hierarchy, kappa=None, f=1.0, stream=None, restart_cap: int = 0, budget: int = 0,
                 poisson_ratio: float = 0.3):
        k, keep = _kappa(kappa)
        r, keep_r = _rhs(f)
        o = assemble_opts_t()
        o.kappa, o.rhs = C.pointer(k), C.pointer(r)
        o.restart_cap, o.max_device_bytes = int(restart_cap), int(budget)
        o.poisson_ratio = float(poisson_ratio)
        s = C.c_void_p()
        _check(_lib.nnms_assemble_ex(h.handle, C.byref(o), _stream_ptr(stream), C.byref(s)))
        self.handle = s
        self.h = h
        self.n = [h.level_info(l).ndof for l in range(h.L)]

    def device_bytes(self) -> int:
        return int(_lib.nnms_system_device_bytes(self.handle))

    def rhs(self) -> np.ndarray:
        b = np.empty(self.n[0])
        _check(_lib.nnms_system_rhs(self.handle, _ptr(b)))
        return b

    def ilu_values(self, level: int) -> np.ndarray:
        v = np.empty(self.h.level_info(level).ilu_nnz)
        _check(_lib.nnms_system_ilu_values(self.handle, level, _ptr(v)))
        return v

    def matrix_values(self, level: int) -> np.ndarray:
        v = np.empty(self.h.level_info(level).nnz)
        _check(_lib.nnms_system_matrix(self.handle, level, _ptr(v)))
        return v

    def _apply(self, fn, level, x, nout):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(nout)
        if level is None:
            _check(fn(self.handle, _ptr(x), _ptr(y), None))
        else:
            _check(fn(self.handle, level, _ptr(x), _ptr(y), None))
        return y

    def apply_operator(self, level, x):
        return self._apply(_lib.nnms_apply_operator, level, x, self.n[level])

    def apply_smoother(self, level, r):
        return self._apply(_lib.nnms_apply_smoother, level, r, self.n[level])

    def apply_prolong(self, level, x):
        return self._apply(_lib.nnms_apply_prolong, level, x, self.n[level])

    def apply_restrict(self, level, x):
        return self._apply(_lib.nnms_apply_restrict, level, x, self.n[level + 1])

    def apply_vcycle(self, r):
        return self._apply(_lib.nnms_apply_vcycle, None, r, self.n[0])

    def apply_smoother_noalloc(self, level: int, r_ptr: int, z_ptr: int, stream=None):
        """nnms_apply_smoother_noalloc on device pointers (nv_level doubles each)."""
        _check(_lib.nnms_apply_smoother_noalloc(self.handle, level, C.c_void_p(r_ptr), C.c_void_p(z_ptr),
                                                _stream_ptr(stream)))

    def factor(self, level: int, part: int):
        """Stored factor tiles of one subdomain: (grid (N*64)^2, inv(L_ii) tiles [N,64,64])."""
        N = C.c_int32()
        _check(_lib.nnms_system_factor(self.handle, level, part, None, None, C.byref(N)))
        lu = np.empty((N.value * 64, N.value * 64))
        il = np.empty((N.value, 64, 64))
        _check(_lib.nnms_system_factor(self.handle, level, part, _ptr(lu), _ptr(il), C.byref(N)))
        return lu, il

    def inverse_panels(self, level: int, part: int) -> np.ndarray:
        """Inverse panels X_p = J_p^{-1} E_o of one subdomain: (N*64, No*64), local rows x owned columns."""
        N, No = C.c_int32(), C.c_int32()
        _check(_lib.nnms_system_inverse_panels(self.handle, level, part, None, C.byref(N), C.byref(No)))
        x = np.empty((N.value * 64, No.value * 64))
        _check(_lib.nnms_system_inverse_panels(self.handle, level, part, _ptr(x), C.byref(N), C.byref(No)))
        return x

    def factor_pairs(self, level: int, part: int):
        """Pair coupling tiles of one subdomain's factor: (X_L [NP,64,64], X_U [NP,64,64])."""
        NP = C.c_int32()
        _check(_lib.nnms_system_factor_pairs(self.handle, level, part, None, None, C.byref(NP)))
        xl = np.empty((NP.value, 64, 64))
        xu = np.empty((NP.value, 64, 64))
        if NP.value:
            _check(_lib.nnms_system_factor_pairs(self.handle, level, part, _ptr(xl), _ptr(xu), C.byref(NP)))
        return xl, xu

    def autotune(self, reps: int = 10) -> dict:
        """nnms_autotune: time the launch-shape candidates on this system and
        store the fastest in its hierarchy."""
        t = tuning_t()
        _check(_lib.nnms_autotune(self.handle, reps, C.byref(t)))
        return t.to_dict()

    def time_kernel(self, kind: int, level: int, reps: int = 10) -> float:
        """Mean milliseconds of one launch (HIP events on the launch stream)."""
        ms = C.c_double()
        _check(_lib.nnms_time_kernel(self.handle, kind, level, reps, C.byref(ms)))
        return ms.value

    def solve(self, b: np.ndarray, restart: int = 30, rtol: float = 1e-8, max_it: int = 1000, graph: bool = True,
              raise_on_fail: bool = True):
        """Host vectors; returns (x, info)."""
        o = solve_opts(restart, max_it, rtol, 0 if graph else NO_GRAPH, 0)
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty(self.n[0])
        info = solve_info()
        code = _lib.nnms_solve(self.handle, _ptr(b), _ptr(x), C.byref(o), C.byref(info), None)
        if raise_on_fail:
            _check(code)
        return x, info

    def solve_device(self, b_ptr: int, x_ptr: int, restart: int = 30, rtol: float = 1e-8, max_it: int = 1000,
                     stream=None, graph: bool = True):
        """Device pointers (e.g. torch tensors' data_ptr()); returns info."""
        o = solve_opts(restart, max_it, rtol, DEVICE_PTRS | (0 if graph else NO_GRAPH), 0)
        info = solve_info()
        _check(_lib.nnms_solve(self.handle, C.c_void_p(b_ptr), C.c_void_p(x_ptr), C.byref(o), C.byref(info),
                               _stream_ptr(stream)))
        return info

    def destroy(self):
        if getattr(self, "handle", None):
            _lib.nnms_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if _lib is not None:
            self.destroy()


def solve_batch(systems: Sequence[System], bs: Sequence[np.ndarray], restart: int = 30, rtol: float = 1e-8,
                max_it: int = 1000, graph: bool = True):
    """nnms_solve_batch with host vectors; returns (xs, infos)."""
    nb = len(systems)
    hs = (C.c_void_p * nb)(*[s.handle for s in systems])
    bs = [np.ascontiguousarray(b, dtype=np.float64) for b in bs]
    xs = [np.empty(s.n[0]) for s in systems]
    bp = (C.c_void_p * nb)(*[b.ctypes.data for b in bs])
    xp = (C.c_void_p * nb)(*[x.ctypes.data for x in xs])
    infos = (solve_info * nb)()
    o = solve_opts(restart, max_it, rtol, 0 if graph else NO_GRAPH, 0)
    _check(_lib.nnms_solve_batch(hs, nb, bp, xp, C.byref(o), infos, None))
    return xs, list(infos)


class Batch:
    """nnms_batch_*: slots advanced together, one Arnoldi step per launch sequence."""

    def __init__(self, systems: Sequence[System], restart: int = 30, rtol: float = 1e-8, max_it: int = 1000,
                 graph: bool = True, stream=None):
        nb = len(systems)
        self.systems = list(systems)
        hs = (C.c_void_p * nb)(*[s.handle for s in systems])
        o = solve_opts(restart, max_it, rtol, 0 if graph else NO_GRAPH, 0)
        h = C.c_void_p()
        _check(_lib.nnms_batch_create(hs, nb, C.byref(o), _stream_ptr(stream), C.byref(h)))
        self.handle = h

    def start(self, slot: int, b_ptr: int):
        _check(_lib.nnms_batch_start(self.handle, slot, C.c_void_p(b_ptr)))

    def step(self, iterations: int = 1) -> int:
        a = C.c_int32()
        _check(_lib.nnms_batch_step(self.handle, iterations, C.byref(a)))
        return a.value

    def result(self, slot: int, x_ptr: Optional[int]):
        info = solve_info()
        _check(_lib.nnms_batch_result(self.handle, slot, None if x_ptr is None else C.c_void_p(x_ptr),
                                      C.byref(info)))
        return info

    def destroy(self):
        if getattr(self, "handle", None):
            _lib.nnms_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if _lib is not None:
            self.destroy()
