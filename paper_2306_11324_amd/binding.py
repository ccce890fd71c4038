"""Thin ctypes binding of the igafmm C ABI (include/igafmm.h).

Argument marshalling only: every numerical step runs in the HIP library.
Device arrays are torch tensors (complex128, on the context's GPU); host arrays
are numpy arrays.  If the shared library is missing, importing this module
raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libigafmm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2306_11324_amd.build`")
# PyTorch ships its own HIP runtime under the same soname as the system one.
# Loading torch first makes the library bind to that runtime, so the process
# holds exactly one HIP runtime (two copies do not see the same devices).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

IGB_OK = 0
IGB_WARN_NOT_CONVERGED = 1
IGB_HOST_ONLY = -1
SOFT, HARD = 0, 1
FP64, MIX_FP32, MIX_BF16 = 0, 1, 2
CFIE, SINGLE_LAYER, OP_V, OP_KSTAR, OP_K, OP_W = 0, 1, 2, 3, 4, 5
PART_NEAR, PART_FAR, PART_ALL = 1, 2, 3
MV_LOWPREC = 4
MV_HOST = 8
CONTEXT_STREAM = "context"   # pass as stream=...: order the call on the context's own stream


class IgbPatch(C.Structure):
    _fields_ = [("deg_u", C.c_int), ("deg_v", C.c_int), ("ncp_u", C.c_int), ("ncp_v", C.c_int),
                ("knots_u", C.POINTER(C.c_double)), ("knots_v", C.POINTER(C.c_double)),
                ("cpw", C.POINTER(C.c_double))]


class IgbOpParams(C.Structure):
    _fields_ = [("kappa", C.c_double), ("bc", C.c_int), ("eta_c", C.c_double), ("q", C.c_int),
                ("eta_adm", C.c_double), ("kcap", C.c_double), ("leaf_depth", C.c_int),
                ("precision", C.c_int), ("far_on_the_fly", C.c_int), ("quad_extra", C.c_int),
                ("formulation", C.c_int), ("separate", C.c_int), ("far_recompress_tol", C.c_double)]


class IgbSolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("maxit", C.c_int), ("inner_tol", C.c_double),
                ("refine_max", C.c_int), ("verbose", C.c_int)]


class IgbSolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("relres", C.c_double),
                ("relres_true", C.c_double), ("matvecs", C.c_int64), ("refinements", C.c_int),
                ("escalated", C.c_int), ("seconds", C.c_double)]


class IgbOpInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nelem", C.c_int64), ("n2", C.c_int64), ("nclusters", C.c_int64),
                ("leaf_level", C.c_int), ("nq", C.c_int), ("far_pairs", C.c_int64),
                ("far_per_level", C.c_int64 * 16), ("near_elem_pairs", C.c_int64), ("nnz", C.c_int64),
                ("device_bytes", C.c_int64), ("estimated_bytes", C.c_int64), ("assembly_near_ms", C.c_double),
                ("assembly_far_ms", C.c_double), ("far_factor_entries", C.c_int64),
                ("near_col_entries", C.c_int64), ("near_tile_entries", C.c_int64),
                ("near_group_staged", C.c_int64)]


_P = C.c_void_p
_SIGS = {
    "igb_ctx_create": (C.c_int, [C.c_int, C.c_size_t, C.POINTER(_P)]),
    "igb_ctx_destroy": (None, [_P]),
    "igb_ctx_used_bytes": (C.c_size_t, [_P]),
    "build_geometry": (C.c_int, [_P, C.POINTER(IgbPatch), C.c_int, C.c_int, C.c_int, C.POINTER(_P)]),
    "igb_geom_destroy": (None, [_P]),
    "igb_geom_dims": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "igb_geom_s0_map": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "assemble_nearfield": (C.c_int, [_P, _P, C.POINTER(IgbOpParams), C.POINTER(_P)]),
    "igb_op_destroy": (None, [_P]),
    "igb_op_get_info": (C.c_int, [_P, C.POINTER(IgbOpInfo)]),
    "igb_op_ndof": (C.c_int64, [_P]),
    "igb_op_bytes": (C.c_int64, [_P]),
    "igb_op_solve_bytes": (C.c_int, [_P, C.c_int, C.c_int, C.POINTER(C.c_int64)]),
    "igb_op_near_csr": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "igb_op_far_blocks": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "igb_op_near_pairs": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "igb_op_potential_plan": (C.c_int, [_P, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int64),
                                        C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "h2_matvec": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, _P]),
    "h2_matvec_noalloc": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, _P]),
    "cfie_rhs": (C.c_int, [_P, C.POINTER(C.c_double), C.c_int, _P, _P]),
    "cfie_solve": (C.c_int, [_P, C.POINTER(C.c_double), C.c_int, C.POINTER(IgbSolveParams), _P,
                             C.POINTER(IgbSolveInfo)]),
    "farfield": (C.c_int, [_P, _P, C.c_int, C.POINTER(C.c_double), C.c_int, _P, _P]),
    "potential": (C.c_int, [_P, _P, C.c_int, C.POINTER(C.c_double), C.c_int, _P, _P]),
    "potential_h2": (C.c_int, [_P, _P, C.c_int, C.POINTER(C.c_double), C.c_int, _P, _P]),
    "igb_op_profile": (C.c_int, [_P, C.c_int]),
    "igb_op_use_graphs": (C.c_int, [_P, C.c_int]),
    "igb_op_set_tile_shape": (C.c_int, [_P, C.c_int, C.c_int]),
    "igb_op_kernel_time": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "igb_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class IgbError(RuntimeError):
    def __init__(self, fn, status):
        msg = _lib.igb_last_error().decode(errors="replace")
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


def _check(fn, st, allow_warn=False):
    if st < 0 or (st > 0 and not allow_warn):
        raise IgbError(fn, st)
    return st


def _dptr(t, n_complex=None):
    """Device address of a complex128 torch tensor on the GPU."""
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.complex128:
        raise TypeError("expected a complex128 torch tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if n_complex is not None and t.numel() < n_complex:
        raise ValueError(f"tensor has {t.numel()} elements, need {n_complex}")
    return C.c_void_p(t.data_ptr())


def _hptr(a, n_complex, writable):
    """Host address of a C-contiguous complex128 numpy array."""
    if not isinstance(a, np.ndarray) or a.dtype != np.complex128 or not a.flags.c_contiguous:
        raise TypeError("expected a C-contiguous complex128 numpy array")
    if writable and not a.flags.writeable:
        raise ValueError("output array is read-only")
    if a.size < n_complex:
        raise ValueError(f"array has {a.size} elements, need {n_complex}")
    return C.c_void_p(a.ctypes.data)


def _stream(stream):
    if stream == CONTEXT_STREAM:
        return C.c_void_p(2 ** 64 - 1)   # IGB_CONTEXT_STREAM
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


def _dbl(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


class Context:
    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = _P()
        _check("igb_ctx_create", _lib.igb_ctx_create(device, hbm_budget, C.byref(h)))
        self.h = h
        self.device = device

    def used_bytes(self) -> int:
        return _lib.igb_ctx_used_bytes(self.h)

    def __del__(self, _destroy=_lib.igb_ctx_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


class Geometry:
    def __init__(self, ctx: Context, patches, m: int, p: int):
        self.ctx = ctx
        keep = []
        arr = (IgbPatch * len(patches))()
        for i, pt in enumerate(patches):
            ku, pku = _dbl(pt.knots_u)
            kv, pkv = _dbl(pt.knots_v)
            cpw, pc = _dbl(pt.cpw)
            keep += [ku, kv, cpw]
            arr[i] = IgbPatch(pt.deg_u, pt.deg_v, cpw.shape[1], cpw.shape[0], pku, pkv, pc)
        h = _P()
        _check("build_geometry", _lib.build_geometry(ctx.h, arr, len(patches), m, p, C.byref(h)))
        self.h = h
        dims = (C.c_int64 * 3)()
        _check("igb_geom_dims", _lib.igb_geom_dims(h, dims))
        self.nelem, self.n2, self.n0 = dims[0], dims[1], dims[2]
        self.m, self.p = m, p

    def s0_map(self) -> np.ndarray:
        out = np.zeros(self.n2, dtype=np.int32)
        _check("igb_geom_s0_map", _lib.igb_geom_s0_map(self.h, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def __del__(self, _destroy=_lib.igb_geom_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


class Operator:
    def __init__(self, ctx: Context, geom: Geometry, kappa: float, bc: int = SOFT, eta_c: float = 0.0,
                 q: int = 6, eta_adm: float = 1.6, kcap: float = 0.0, leaf_depth: int = 2,
                 precision: int = FP64, far_on_the_fly: bool = False, quad_extra: int = 0,
                 formulation: int = CFIE, separate: bool = False, recompress_tol: float = 0.0):
        self.ctx, self.geom = ctx, geom
        self.params = IgbOpParams(kappa, bc, eta_c, q, eta_adm, kcap, leaf_depth, precision,
                                  1 if far_on_the_fly else 0, quad_extra, formulation, 1 if separate else 0,
                                  recompress_tol)
        h = _P()
        _check("assemble_nearfield", _lib.assemble_nearfield(ctx.h, geom.h, C.byref(self.params), C.byref(h)))
        self.h = h
        self.info = self.get_info()
        self.n = self.info.n

    def get_info(self) -> IgbOpInfo:
        info = IgbOpInfo()
        _check("igb_op_get_info", _lib.igb_op_get_info(self.h, C.byref(info)))
        return info

    def solve_bytes(self, ndir: int, restart: int = 30) -> int:
        """Device bytes the operator holds after a solve of ndir directions (size model)."""
        b = C.c_int64()
        _check("igb_op_solve_bytes", _lib.igb_op_solve_bytes(self.h, ndir, restart, C.byref(b)))
        return b.value

    def held_bytes(self) -> int:
        return int(_lib.igb_op_bytes(self.h))

    def near_csr(self):
        n, nnz = self.info.n, self.info.nnz
        rp = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(nnz, dtype=np.int32)
        val = np.zeros(2 * nnz, dtype=np.float64)
        _check("igb_op_near_csr", _lib.igb_op_near_csr(
            self.h, rp.ctypes.data_as(C.POINTER(C.c_int64)), col.ctypes.data_as(C.POINTER(C.c_int32)),
            val.ctypes.data_as(C.POINTER(C.c_double))))
        return rp, col, val.view(np.complex128)

    def far_blocks(self) -> np.ndarray:
        out = np.zeros((self.info.far_pairs, 4), dtype=np.int32)
        _check("igb_op_far_blocks", _lib.igb_op_far_blocks(self.h, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out[:, :3]

    def near_pairs(self):
        E, npairs = self.info.nelem, self.info.near_elem_pairs
        ptr = np.zeros(E + 1, dtype=np.int64)
        src = np.zeros(npairs, dtype=np.int32)
        kind = np.zeros(npairs, dtype=np.int32)
        _check("igb_op_near_pairs", _lib.igb_op_near_pairs(
            self.h, ptr.ctypes.data_as(C.POINTER(C.c_int64)), src.ctypes.data_as(C.POINTER(C.c_int32)),
            kind.ctypes.data_as(C.POINTER(C.c_int32))))
        return ptr, src, kind

    def potential_plan(self, points):
        """The H^2 potential's plan for host points [npts][3]: (counts, perm,
        box_ptr) with counts = boxes, box-node pairs, cluster-node pairs, direct
        pairs; box b holds the points perm[box_ptr[b]:box_ptr[b+1]]."""
        pt, pp = _dbl(np.atleast_2d(points))
        counts = np.zeros(4, dtype=np.int64)
        i32 = C.POINTER(C.c_int32)
        _check("igb_op_potential_plan", _lib.igb_op_potential_plan(
            self.h, pp, pt.shape[0], counts.ctypes.data_as(C.POINTER(C.c_int64)), None, None))
        perm = np.zeros(pt.shape[0], dtype=np.int32)
        box_ptr = np.zeros(int(counts[0]) + 1, dtype=np.int32)
        _check("igb_op_potential_plan", _lib.igb_op_potential_plan(
            self.h, pp, pt.shape[0], counts.ctypes.data_as(C.POINTER(C.c_int64)), perm.ctypes.data_as(i32),
            box_ptr.ctypes.data_as(i32)))
        return counts, perm, box_ptr

    def profile(self, enable: bool = True):
        _check("igb_op_profile", _lib.igb_op_profile(self.h, 1 if enable else 0))

    def use_graphs(self, enable: bool = True):
        """Capture the matvec into HIP graphs (single-threaded use; see the header)."""
        _check("igb_op_use_graphs", _lib.igb_op_use_graphs(self.h, 1 if enable else 0))

    def set_tile_shape(self, coupling_col_tiles: int = 0, near_col_tiles: int = 0):
        """Column tiles per workgroup of the fp64 block kernels (0: automatic)."""
        _check("igb_op_set_tile_shape", _lib.igb_op_set_tile_shape(self.h, int(coupling_col_tiles),
                                                                     int(near_col_tiles)))

    def kernel_time(self, name: str):
        """(launches, total ms) of the named kernel since the last query."""
        n = C.c_int64()
        ms = C.c_double()
        _check("igb_op_kernel_time", _lib.igb_op_kernel_time(self.h, name.encode(), C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def h2_matvec(self, x, y, nrhs: int = 1, parts: int = PART_ALL, stream=None):
        """y = A x for nrhs columns stored [nrhs][n] in x and y: complex128 torch
        tensors on the GPU, or (with MV_HOST in parts) numpy arrays on the host."""
        if parts & MV_HOST:
            xs, ys = _hptr(x, nrhs * self.n, False), _hptr(y, nrhs * self.n, True)
        else:
            xs, ys = _dptr(x, nrhs * self.n), _dptr(y, nrhs * self.n)
        _check("h2_matvec", _lib.h2_matvec(self.h, xs, ys, nrhs, parts, _stream(stream)))
        return y

    def h2_matvec_noalloc(self, x, y, nrhs: int = 1, parts: int = PART_ALL, stream=None):
        """h2_matvec with the work buffers in the library's per-GPU scratch array
        (allocates nothing; calls overlapping on one GPU race)."""
        _check("h2_matvec_noalloc", _lib.h2_matvec_noalloc(self.h, _dptr(x, nrhs * self.n),
                                                           _dptr(y, nrhs * self.n), nrhs, parts, _stream(stream)))
        return y

    def cfie_rhs(self, dirs, b, stream=None):
        d, pd = _dbl(np.atleast_2d(dirs))
        _check("cfie_rhs", _lib.cfie_rhs(self.h, pd, d.shape[0], _dptr(b, d.shape[0] * self.n), _stream(stream)))
        return b

    def cfie_solve(self, dirs, coeffs, tol=1e-8, restart=30, maxit=1000, inner_tol=0.0, refine_max=0,
                   verbose=False):
        d, pd = _dbl(np.atleast_2d(dirs))
        sp = IgbSolveParams(tol, restart, maxit, inner_tol, refine_max, 1 if verbose else 0)
        info = IgbSolveInfo()
        st = _check("cfie_solve", _lib.cfie_solve(self.h, pd, d.shape[0], C.byref(sp),
                                                  _dptr(coeffs, d.shape[0] * self.n), C.byref(info)),
                    allow_warn=True)
        return info, st

    def farfield(self, coeffs, obs, uinf, ndir: int = 1, stream=None):
        o, po = _dbl(np.atleast_2d(obs))
        _check("farfield", _lib.farfield(self.h, _dptr(coeffs, ndir * self.n), ndir, po, o.shape[0],
                                         _dptr(uinf, ndir * o.shape[0]), _stream(stream)))
        return uinf

    def potential(self, coeffs, points, u, ndir: int = 1, stream=None):
        """Scattered field u [ndir][npts] at host points [npts][3] off the boundary."""
        pt, pp = _dbl(np.atleast_2d(points))
        _check("potential", _lib.potential(self.h, _dptr(coeffs, ndir * self.n), ndir, pp, pt.shape[0],
                                           _dptr(u, ndir * pt.shape[0]), _stream(stream)))
        return u

    def potential_h2(self, coeffs, points, u, ndir: int = 1, stream=None):
        """potential() through the H^2 structure (octree boxes, interpolated far part)."""
        pt, pp = _dbl(np.atleast_2d(points))
        _check("potential_h2", _lib.potential_h2(self.h, _dptr(coeffs, ndir * self.n), ndir, pp, pt.shape[0],
                                                 _dptr(u, ndir * pt.shape[0]), _stream(stream)))
        return u

    def __del__(self, _destroy=_lib.igb_op_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None
