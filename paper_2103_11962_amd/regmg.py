"""Python binding of the regmg C ABI (argument marshalling only).

Every computation runs inside the HIP library ``_lib/libregmg.so``; this module
only converts torch tensors / numpy arrays to pointers and status codes to
exceptions.  Device vectors are torch tensors on the HIP device (float64,
contiguous).  The library must be built first (``__graft_entry__.build()``);
loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libregmg.so")

LAYOUT_COMPOSITE = 0
LAYOUT_REGIONAL = 1
PDE_LAPLACE, PDE_DIFFUSION, PDE_ELASTICITY = 0, 1, 2
PREC_FP64, PREC_FP32, PREC_FP32_BF16, PREC_FP32_BF16_AUTO = 0, 1, 2, 3
KERNEL_AUTO, KERNEL_NODE, KERNEL_TILED = 0, 1, 2

STATUS = {
    0: "RMG_OK", 1: "RMG_ERR_ARG", 2: "RMG_ERR_SHAPE", 3: "RMG_ERR_NUMERIC", 4: "RMG_ERR_DEVICE",
    5: "RMG_ERR_OOM", 6: "RMG_ERR_NOT_SETUP", 7: "RMG_ERR_BREAKDOWN", 8: "RMG_ERR_NOT_CONVERGED",
}

# every symbol the public header declares
SYMBOLS = (
    "rmg_options_default", "rmg_create", "rmg_destroy", "rmg_last_error", "rmg_build_regions",
    "rmg_set_region_stencil", "rmg_set_composite_stencil", "rmg_assemble_q1", "rmg_setup_hierarchy",
    "rmg_apply_vcycle", "rmg_solve", "rmg_to_regional", "rmg_to_composite", "rmg_regional_matvec",
    "rmg_interface_sum", "rmg_restrict", "rmg_prolongate_add", "rmg_smooth", "rmg_level_info",
    "rmg_get_level_stencil", "rmg_get_coarse_matrix", "rmg_profile", "rmg_profile_query",
    "rmg_tune_report", "rmg_set_prolongator_weights", "rmg_set_learned_prolongator", "rmg_prolongator_info",
    "rmg_get_prolongator_weights", "rmg_convergence_factor", "rmg_mlp_create", "rmg_mlp_destroy",
    "rmg_mlp_set_params", "rmg_mlp_get_params", "rmg_mlp_add_data", "rmg_mlp_add_samples", "rmg_mlp_clear_data",
    "rmg_mlp_num_data", "rmg_mlp_get_data", "rmg_mlp_forward", "rmg_mlp_loss_grad", "rmg_mlp_adam_step",
    "rmg_mlp_train", "rmg_mlp_init_params", "rmg_level_kernel", "rmg_set_composite_csr", "rmg_mg_solve",
    "rmg_mlp_set_loss", "rmg_set_region_kinds", "rmg_hybrid_level_info", "rmg_hybrid_aggregates",
    "rmg_hybrid_composite_ids", "rmg_hybrid_matrix", "rmg_amg_levels", "rmg_amg_level_info", "rmg_amg_matrix",
    "rmg_level_table_regions", "rmg_level_tiles", "rmg_level_transfer_tiles", "rmg_kernel_launches", "rmg_convergence_factor_noalloc",
    "rmg_level_precision",
)
SMOOTHER_CHEBYSHEV, SMOOTHER_JACOBI, SMOOTHER_GS, SMOOTHER_GS_FB, SMOOTHER_SYMGS = 0, 1, 2, 3, 4
TIMED_CHEB, TIMED_CG_MATVEC = 0, 1
P_GEOMETRIC, P_STORED, P_LEARNED = 0, 1, 2
PW_NONFINITE, PW_SUPPORT, PW_DIRICHLET, PW_COPIES, PW_SUM, PW_JUDGED_WORSE = 1, 2, 4, 8, 16, 32
MLP_NIN, MLP_NHIDDEN, MLP_NOUT, MLP_NPARAM = 27, 64, 208, 19472
MLP_LOSS_L2, MLP_LOSS_ENERGY = 0, 1


class Options(ctypes.Structure):
    _fields_ = [
        ("nlevels", ctypes.c_int),
        ("cheb_degree", ctypes.c_int),
        ("eig_ratio", ctypes.c_double),
        ("boost", ctypes.c_double),
        ("power_iters", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("precision", ctypes.c_int),
        ("stencil_kernel", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("autotune_cache", ctypes.c_char_p),
        ("smoother", ctypes.c_int),
        ("jacobi_omega", ctypes.c_double),
        ("symmetric", ctypes.c_int),
        ("batched", ctypes.c_int),
        ("judge_cycles", ctypes.c_int),
        ("hybrid", ctypes.c_int),
        ("cycle_gamma", ctypes.c_int),
        ("coarse_amg", ctypes.c_int),
        ("amg_coarse_size", ctypes.c_int),
        ("region_table", ctypes.c_int),
        ("tile_planes", ctypes.c_int),
        ("galerkin_generic", ctypes.c_int),
        ("bf16_tolerance", ctypes.c_double),
        ("bf16_cycles", ctypes.c_int),
        ("block_diag", ctypes.c_int),
        ("transfer_rows", ctypes.c_int),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("relres", ctypes.c_double),
        ("true_relres", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
        ("history", ctypes.POINTER(ctypes.c_double)),
        ("history_cap", ctypes.c_int),
        ("history_len", ctypes.c_int),
        ("setup_ms", ctypes.c_double),
        ("level_ms", ctypes.c_double * 12),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


def _torch_allocator(device, stream):
    """rmg_allocator backed by PyTorch's caching allocator on `stream` of `device`."""
    import torch

    def alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=device, stream=stream)
        except RuntimeError:
            return None

    def free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    return Allocator(ALLOC_FN(alloc), FREE_FN(free), None)


class RmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


_lib = None


def load():
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"regmg library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    H = ctypes.c_void_p
    sig = {
        "rmg_options_default": (None, [ctypes.POINTER(Options)]),
        "rmg_create": (I, [ctypes.POINTER(H), I, P, ctypes.POINTER(Allocator)]),
        "rmg_destroy": (I, [H]),
        "rmg_last_error": (ctypes.c_char_p, []),
        "rmg_build_regions": (I, [H, I, I, I, P, P, ctypes.c_uint32]),
        "rmg_set_region_stencil": (I, [H, I, I, P, I]),
        "rmg_set_composite_stencil": (I, [H, I, P, I]),
        "rmg_assemble_q1": (I, [H, I, D, P, P, D]),
        "rmg_setup_hierarchy": (I, [H, ctypes.POINTER(Options)]),
        "rmg_apply_vcycle": (I, [H, P, P, I]),
        "rmg_solve": (I, [H, P, P, I, D, I, ctypes.POINTER(SolveInfo)]),
        "rmg_to_regional": (I, [H, I, P, P]),
        "rmg_to_composite": (I, [H, I, P, P, I]),
        "rmg_regional_matvec": (I, [H, I, P, P]),
        "rmg_interface_sum": (I, [H, I, P, P]),
        "rmg_restrict": (I, [H, I, P, P]),
        "rmg_prolongate_add": (I, [H, I, P, P]),
        "rmg_smooth": (I, [H, I, P, P]),
        "rmg_level_info": (I, [H, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(I), ctypes.POINTER(D)]),
        "rmg_get_level_stencil": (I, [H, I, I, P]),
        "rmg_get_coarse_matrix": (I, [H, P]),
        "rmg_profile": (I, [H, I]),
        "rmg_tune_report": (I, [H, ctypes.c_char_p, I]),
        "rmg_profile_query": (I, [H, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(D)]),
        "rmg_set_prolongator_weights": (I, [H, P, I]),
        "rmg_set_learned_prolongator": (I, [H, P]),
        "rmg_prolongator_info": (I, [H, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(D),
                                     ctypes.POINTER(D)]),
        "rmg_get_prolongator_weights": (I, [H, P]),
        "rmg_convergence_factor": (I, [H, I, ctypes.POINTER(D)]),
        "rmg_convergence_factor_noalloc": (I, [H, I, ctypes.POINTER(D)]),
        "rmg_mlp_create": (I, [ctypes.POINTER(H), I, P]),
        "rmg_mlp_destroy": (I, [H]),
        "rmg_mlp_set_params": (I, [H, P]),
        "rmg_mlp_get_params": (I, [H, P]),
        "rmg_mlp_add_data": (I, [H, ctypes.c_int64, P, P, I]),
        "rmg_mlp_add_samples": (I, [H, H, I, ctypes.c_uint64, I]),
        "rmg_mlp_clear_data": (I, [H]),
        "rmg_mlp_num_data": (I, [H, ctypes.POINTER(ctypes.c_int64)]),
        "rmg_mlp_get_data": (I, [H, ctypes.c_int64, ctypes.c_int64, P, P]),
        "rmg_mlp_forward": (I, [H, ctypes.c_int64, P, P, I]),
        "rmg_mlp_loss_grad": (I, [H, ctypes.POINTER(D), P]),
        "rmg_mlp_adam_step": (I, [H, P, D]),
        "rmg_mlp_train": (I, [H, I, D, P]),
        "rmg_mlp_init_params": (I, [H, ctypes.c_uint64, D, P]),
        "rmg_level_kernel": (I, [H, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "rmg_level_precision": (I, [H, I, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
        "rmg_set_composite_csr": (I, [H, I, ctypes.c_int64, P, P, P, I]),
        "rmg_level_table_regions": (I, [H, I, ctypes.POINTER(I)]),
        "rmg_level_tiles": (I, [H, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "rmg_level_transfer_tiles": (I, [H, I, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "rmg_kernel_launches": (I, [ctypes.POINTER(ctypes.c_int64)]),
        "rmg_mg_solve": (I, [H, P, P, I, D, I, ctypes.POINTER(SolveInfo)]),
        "rmg_mlp_set_loss": (I, [H, I]),
        "rmg_set_region_kinds": (I, [H, P]),
        "rmg_hybrid_level_info": (I, [H, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64)]),
        "rmg_hybrid_aggregates": (I, [H, I, P]),
        "rmg_hybrid_composite_ids": (I, [H, I, P]),
        "rmg_hybrid_matrix": (I, [H, I, P, P, P]),
        "rmg_amg_levels": (I, [H, ctypes.POINTER(ctypes.c_int)]),
        "rmg_amg_level_info": (I, [H, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64)]),
        "rmg_amg_matrix": (I, [H, I, I, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code):
    if code != 0:
        raise RmgError(code, load().rmg_last_error().decode())


def _ptr(t):
    """Device pointer of a contiguous float64 torch tensor."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_contiguous() or t.dtype != torch.float64:
        raise ValueError("device vectors must be contiguous float64 tensors")
    return ctypes.c_void_p(t.data_ptr())


def kernel_launches() -> int:
    """Kernel launches the library has issued in this process so far."""
    n = ctypes.c_int64()
    _check(load().rmg_kernel_launches(ctypes.byref(n)))
    return n.value


def default_options(**kw) -> Options:
    o = Options()
    load().rmg_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k == "autotune_cache" and isinstance(v, str):
            v = v.encode()
        setattr(o, k, v)
    return o


class Handle:
    """One solver instance on one HIP device and stream."""

    def __init__(self, device: int = 0, stream=None, torch_allocator: bool = False, allocator=None):
        """torch_allocator: take every device buffer of the handle from PyTorch's caching
        allocator (on the handle's stream) instead of hipMalloc; allocator: any other
        ``Allocator`` (its callbacks must stay valid until close())."""
        import torch

        lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        # the callbacks must outlive every buffer they provided: kept on the handle
        self._alloc = allocator if allocator is not None else (_torch_allocator(device, stream) if torch_allocator
                                                               else None)
        h = ctypes.c_void_p()
        _check(lib.rmg_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream),
                              ctypes.byref(self._alloc) if self._alloc is not None else None))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load().rmg_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---------------------------------------------------------------- setup
    def build_regions(self, dim, ndof, extents, origins, dirichlet_mask):
        ext = np.ascontiguousarray(extents, dtype=np.int32).reshape(-1)
        org = np.ascontiguousarray(origins, dtype=np.int32).reshape(-1)
        nreg = ext.size // dim
        _check(load().rmg_build_regions(self._h, dim, ndof, nreg, ext.ctypes.data_as(ctypes.c_void_p),
                                        org.ctypes.data_as(ctypes.c_void_p), dirichlet_mask))

    def set_region_stencil(self, region, npts, coef):
        import torch

        if isinstance(coef, torch.Tensor):
            _check(load().rmg_set_region_stencil(self._h, region, npts, _ptr(coef), 1))
        else:
            c = np.ascontiguousarray(coef, dtype=np.float64)
            _check(load().rmg_set_region_stencil(self._h, region, npts, c.ctypes.data_as(ctypes.c_void_p), 0))

    def set_composite_stencil(self, npts, coef):
        import torch

        if isinstance(coef, torch.Tensor):
            _check(load().rmg_set_composite_stencil(self._h, npts, _ptr(coef), 1))
        else:
            c = np.ascontiguousarray(coef, dtype=np.float64)
            _check(load().rmg_set_composite_stencil(self._h, npts, c.ctypes.data_as(ctypes.c_void_p), 0))

    def set_composite_csr(self, npts, A):
        """Non-invasive split of an assembled composite matrix (scipy sparse, host)."""
        import scipy.sparse as sp

        A = sp.csr_matrix(A)
        rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
        ci = np.ascontiguousarray(A.indices, dtype=np.int32)
        v = np.ascontiguousarray(A.data, dtype=np.float64)
        _check(load().rmg_set_composite_csr(self._h, npts, int(v.size), rp.ctypes.data_as(ctypes.c_void_p),
                                            ci.ctypes.data_as(ctypes.c_void_p), v.ctypes.data_as(ctypes.c_void_p),
                                            0))

    def assemble_q1(self, pde, h, elem_coef=None, youngs=None, nu=0.3):
        y = None if youngs is None else np.ascontiguousarray(youngs, dtype=np.float64)
        _check(load().rmg_assemble_q1(self._h, pde, h, _ptr(elem_coef),
                                      None if y is None else y.ctypes.data_as(ctypes.c_void_p), nu))

    def setup_hierarchy(self, **kw):
        o = default_options(**kw)
        _check(load().rmg_setup_hierarchy(self._h, ctypes.byref(o)))

    # ---------------------------------------------------------------- solve
    def apply_vcycle(self, r, z, layout=LAYOUT_COMPOSITE):
        _check(load().rmg_apply_vcycle(self._h, _ptr(r), _ptr(z), layout))

    def solve(self, b, x, layout=LAYOUT_COMPOSITE, rtol=1e-8, maxit=200, history_cap=512, raise_on_fail=True,
              method="pcg"):
        """PCG (method "pcg") or multigrid as a solver (method "mg")."""
        info = SolveInfo()
        hist = (ctypes.c_double * history_cap)()
        info.history = hist
        info.history_cap = history_cap
        fn = load().rmg_solve if method == "pcg" else load().rmg_mg_solve
        code = fn(self._h, _ptr(b), _ptr(x), layout, rtol, maxit, ctypes.byref(info))
        if code != 0 and raise_on_fail:
            _check(code)
        out = {
            "status": STATUS.get(code, code), "iterations": info.iterations, "converged": bool(info.converged),
            "relres": info.relres, "true_relres": info.true_relres, "solve_ms": info.solve_ms,
            "setup_ms": info.setup_ms,
            "level_ms": list(info.level_ms),
            "history": [hist[i] for i in range(min(info.history_len, history_cap))],
        }
        return out

    # --------------------------------------------------------- step hooks
    def to_regional(self, level, comp, reg):
        _check(load().rmg_to_regional(self._h, level, _ptr(comp), _ptr(reg)))

    def to_composite(self, level, reg, comp, average=False):
        _check(load().rmg_to_composite(self._h, level, _ptr(reg), _ptr(comp), int(average)))

    def regional_matvec(self, level, v, z):
        _check(load().rmg_regional_matvec(self._h, level, _ptr(v), _ptr(z)))

    def interface_sum(self, level, v, w):
        _check(load().rmg_interface_sum(self._h, level, _ptr(v), _ptr(w)))

    def restrict(self, level, r, w):
        _check(load().rmg_restrict(self._h, level, _ptr(r), _ptr(w)))

    def prolongate_add(self, level, ubar, u):
        _check(load().rmg_prolongate_add(self._h, level, _ptr(ubar), _ptr(u)))

    def smooth(self, level, b, u):
        _check(load().rmg_smooth(self._h, level, _ptr(b), _ptr(u)))

    def level_info(self, level):
        nr, nc = ctypes.c_int64(), ctypes.c_int64()
        npts, lam = ctypes.c_int(), ctypes.c_double()
        _check(load().rmg_level_info(self._h, level, ctypes.byref(nr), ctypes.byref(nc), ctypes.byref(npts),
                                     ctypes.byref(lam)))
        return {"n_regional": nr.value, "n_composite": nc.value, "npts": npts.value, "lambda": lam.value}

    # ---- structured/unstructured hybrid hierarchy
    def set_region_kinds(self, kinds):
        """kinds[k] = 0 structured, 1 unstructured (used with setup_hierarchy(hybrid=1))."""
        k = np.ascontiguousarray(kinds, dtype=np.int32)
        _check(load().rmg_set_region_kinds(self._h, k.ctypes.data_as(ctypes.c_void_p)))

    def hybrid_level_info(self, level):
        n, c, z = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().rmg_hybrid_level_info(self._h, level, ctypes.byref(n), ctypes.byref(c), ctypes.byref(z)))
        return {"n_regional": n.value, "n_composite": c.value, "nnz": z.value}

    def hybrid_aggregates(self, level):
        out = np.zeros(self.hybrid_level_info(level)["n_regional"], dtype=np.int32)
        _check(load().rmg_hybrid_aggregates(self._h, level, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def hybrid_composite_ids(self, level):
        out = np.zeros(self.hybrid_level_info(level)["n_regional"], dtype=np.int64)
        _check(load().rmg_hybrid_composite_ids(self._h, level, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def hybrid_matrix(self, level):
        """The level's region matrices as one block-diagonal scipy CSR matrix over regional rows."""
        import scipy.sparse as sp

        info = self.hybrid_level_info(level)
        n, nnz = info["n_regional"], info["nnz"]
        rp = np.zeros(n + 1, dtype=np.int64)
        ci = np.zeros(max(nnz, 1), dtype=np.int32)
        v = np.zeros(max(nnz, 1))
        _check(load().rmg_hybrid_matrix(self._h, level, rp.ctypes.data_as(ctypes.c_void_p),
                                        ci.ctypes.data_as(ctypes.c_void_p), v.ctypes.data_as(ctypes.c_void_p)))
        return sp.csr_matrix((v[:nnz], ci[:nnz], rp), shape=(n, n))

    def amg_levels(self):
        """Levels of the AMG coarse solver (0 without one)."""
        n = ctypes.c_int()
        _check(load().rmg_amg_levels(self._h, ctypes.byref(n)))
        return n.value

    def amg_level_info(self, level):
        n, a, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().rmg_amg_level_info(self._h, level, ctypes.byref(n), ctypes.byref(a), ctypes.byref(p)))
        return {"n": n.value, "nnz_a": a.value, "nnz_p": p.value}

    def amg_matrix(self, level, which=0):
        """AMG level `level`'s matrix (which 0) or prolongator to the next level (which 1), scipy CSR."""
        import scipy.sparse as sp

        info = self.amg_level_info(level)
        n = info["n"]
        nnz = info["nnz_a"] if which == 0 else info["nnz_p"]
        ncols = n if which == 0 else self.amg_level_info(level + 1)["n"]
        rp = np.zeros(n + 1, dtype=np.int64)
        ci = np.zeros(max(nnz, 1), dtype=np.int32)
        v = np.zeros(max(nnz, 1))
        _check(load().rmg_amg_matrix(self._h, level, which, rp.ctypes.data_as(ctypes.c_void_p),
                                     ci.ctypes.data_as(ctypes.c_void_p), v.ctypes.data_as(ctypes.c_void_p)))
        return sp.csr_matrix((v[:nnz], ci[:nnz], rp), shape=(n, ncols))

    def level_kernel(self, level):
        k, c, cl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load().rmg_level_kernel(self._h, level, ctypes.byref(k), ctypes.byref(c), ctypes.byref(cl)))
        return {"kernel": k.value, "coefs": c.value, "coefs_lo": cl.value}

    def level_precision(self, level):
        t, r32, rbf = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(load().rmg_level_precision(self._h, level, ctypes.byref(t), ctypes.byref(r32), ctypes.byref(rbf)))
        return {"coef_type": t.value, "rho_fp32": r32.value, "rho_bf16": rbf.value}

    def level_tiles(self, level):
        n, t, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load().rmg_level_tiles(self._h, level, ctypes.byref(n), ctypes.byref(t), ctypes.byref(p)))
        return {"ntiles": n.value, "threads": t.value, "planes": p.value}

    def level_transfer_tiles(self, level):
        r, p = ctypes.c_int(), ctypes.c_int()
        _check(load().rmg_level_transfer_tiles(self._h, level, ctypes.byref(r), ctypes.byref(p)))
        return {"restriction": r.value, "prolongation": p.value}

    def level_table_regions(self, level):
        n = ctypes.c_int()
        _check(load().rmg_level_table_regions(self._h, level, ctypes.byref(n)))
        return n.value

    def level_stencil(self, level, region, npts, nnodes):
        out = np.zeros(npts * nnodes)
        _check(load().rmg_get_level_stencil(self._h, level, region, out.ctypes.data_as(ctypes.c_void_p)))
        return out.reshape(npts, nnodes)

    def coarse_matrix(self, n):
        out = np.zeros(n * n)
        _check(load().rmg_get_coarse_matrix(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out.reshape(n, n)

    # ---------------------------------------------------------- timing
    def profile(self, enable=True):
        _check(load().rmg_profile(self._h, int(enable)))

    def profile_query(self, kernel):
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check(load().rmg_profile_query(self._h, kernel, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def tune_report(self):
        buf = ctypes.create_string_buffer(8192)
        _check(load().rmg_tune_report(self._h, buf, 8192))
        return buf.value.decode()

    # ------------------------------------------------ stored / learned P
    def set_prolongator_weights(self, w):
        """Caller weights [n_regional][8] (numpy or device float64 tensor); None: geometric."""
        import torch

        if w is None:
            _check(load().rmg_set_prolongator_weights(self._h, None, 0))
        elif isinstance(w, torch.Tensor):
            _check(load().rmg_set_prolongator_weights(self._h, _ptr(w), 1))
        else:
            a = np.ascontiguousarray(w, dtype=np.float64)
            _check(load().rmg_set_prolongator_weights(self._h, a.ctypes.data_as(ctypes.c_void_p), 0))

    def set_learned_prolongator(self, theta):
        """MLP parameters (RMG_MLP_NPARAM floats) of the learned interpolation; None: geometric."""
        if theta is None:
            _check(load().rmg_set_learned_prolongator(self._h, None))
            return
        a = np.ascontiguousarray(theta, dtype=np.float32)
        if a.size != MLP_NPARAM:
            raise ValueError(f"expected {MLP_NPARAM} parameters")
        _check(load().rmg_set_learned_prolongator(self._h, a.ctypes.data_as(ctypes.c_void_p)))

    def prolongator_info(self):
        kind, flags, rl, rg = ctypes.c_int(), ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(load().rmg_prolongator_info(self._h, ctypes.byref(kind), ctypes.byref(flags), ctypes.byref(rl),
                                           ctypes.byref(rg)))
        return {"kind": kind.value, "flags": flags.value, "rho_learned": rl.value, "rho_geometric": rg.value}

    def prolongator_weights(self, n_regional):
        out = np.zeros((n_regional, 8))
        _check(load().rmg_get_prolongator_weights(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def convergence_factor(self, cycles=10):
        rho = ctypes.c_double()
        _check(load().rmg_convergence_factor(self._h, cycles, ctypes.byref(rho)))
        return rho.value

    def convergence_factor_noalloc(self, cycles=10):
        rho = ctypes.c_double()
        _check(load().rmg_convergence_factor_noalloc(self._h, cycles, ctypes.byref(rho)))
        return rho.value


def _fptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Mlp:
    """Trainer of the learned interpolation's MLP on one HIP device (rmg_mlp_*)."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        m = ctypes.c_void_p()
        _check(lib.rmg_mlp_create(ctypes.byref(m), device, ctypes.c_void_p(stream.cuda_stream)))
        self._m = m

    def close(self):
        if getattr(self, "_m", None) is not None and self._m.value:
            _check(load().rmg_mlp_destroy(self._m))
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_loss(self, kind):
        """MLP_LOSS_L2 or MLP_LOSS_ENERGY."""
        _check(load().rmg_mlp_set_loss(self._m, kind))

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        if a.size != MLP_NPARAM:
            raise ValueError(f"expected {MLP_NPARAM} parameters")
        _check(load().rmg_mlp_set_params(self._m, _fptr(a)))

    def init_params(self, seed=0, out_scale=0.01):
        out = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check(load().rmg_mlp_init_params(self._m, seed, out_scale, _fptr(out)))
        return out

    def params(self):
        out = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check(load().rmg_mlp_get_params(self._m, _fptr(out)))
        return out

    def add_data(self, X, E):
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, MLP_NIN)
        E = np.ascontiguousarray(E, dtype=np.float32).reshape(-1, 64)
        if X.shape[0] != E.shape[0]:
            raise ValueError("X and E need the same number of rows")
        _check(load().rmg_mlp_add_data(self._m, X.shape[0], _fptr(X), _fptr(E), 0))

    def add_samples(self, handle: Handle, nsamples, seed, sweeps=20):
        _check(load().rmg_mlp_add_samples(self._m, handle._h, nsamples, seed, sweeps))

    def clear_data(self):
        _check(load().rmg_mlp_clear_data(self._m))

    def num_data(self):
        n = ctypes.c_int64()
        _check(load().rmg_mlp_num_data(self._m, ctypes.byref(n)))
        return n.value

    def data(self, first, count):
        X = np.zeros((count, MLP_NIN), dtype=np.float32)
        E = np.zeros((count, 64), dtype=np.float32)
        _check(load().rmg_mlp_get_data(self._m, first, count, _fptr(X), _fptr(E)))
        return X, E

    def forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, MLP_NIN)
        Z = np.zeros((X.shape[0], MLP_NOUT), dtype=np.float32)
        _check(load().rmg_mlp_forward(self._m, X.shape[0], _fptr(X), _fptr(Z), 0))
        return Z

    def loss_grad(self):
        loss = ctypes.c_double()
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check(load().rmg_mlp_loss_grad(self._m, ctypes.byref(loss), _fptr(g)))
        return loss.value, g

    def adam_step(self, lr, grad=None):
        g = None if grad is None else np.ascontiguousarray(grad, dtype=np.float32)
        _check(load().rmg_mlp_adam_step(self._m, None if g is None else _fptr(g), lr))

    def train(self, steps, lr):
        hist = np.zeros(max(steps, 1))
        _check(load().rmg_mlp_train(self._m, steps, lr, _fptr(hist)))
        return hist[:steps]
