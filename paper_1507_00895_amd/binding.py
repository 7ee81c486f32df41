"""ctypes binding of libdf (the C ABI declared in include/df.h).

Argument marshalling only: torch tensors supply device pointers and the
stream; every step of the method runs in the HIP kernels of libdf.so.  If the
library has not been built, or no GPU is present, the calls raise; there is no
CPU fallback.

Same names as the ABI: df_workspace_size, df_dual_gf, df_bubble,
df_ladder_solve, df_sigma, df_iterate, df_strerror, df_version, the autotuner
calls, the warm-start network (df_mlp_*) and the lattice observables
(df_lattice_workspace_size, df_lattice).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdf.so")

DF_OK = 0
DF_E_INVAL = -1
DF_E_UNSUPPORTED = -2
DF_E_WORKSPACE = -3
DF_E_HIP = -4
DF_E_NONFINITE = -5
DF_E_NOT_CONVERGED = -6
DF_W_FALLBACK = 1

DF_FP64 = 0
DF_FP32_REFINE = 1
DF_FP32 = 2
DF_ADAPTIVE = 3

EXPORTED = ("df_workspace_size", "df_dual_gf", "df_bubble", "df_ladder_solve", "df_sigma",
            "df_iterate", "df_autotune", "df_ladder_variant", "df_ladder_set_variant",
            "df_autotune_reset", "df_strerror", "df_version", "df_bubble_noalloc")


class DfInst(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32), ("nk", ctypes.c_int32), ("n_nu", ctypes.c_int32),
        ("n_om", ctypes.c_int32), ("beta", ctypes.c_double),
        ("g", ctypes.c_void_p), ("delta", ctypes.c_void_p), ("eps", ctypes.c_void_p),
        ("gamma_uu", ctypes.c_void_p), ("gamma_ud", ctypes.c_void_p),
        ("sigma", ctypes.c_void_p), ("gd", ctypes.c_void_p), ("chi", ctypes.c_void_p),
        ("w", ctypes.c_void_p), ("logdet", ctypes.c_void_p), ("sigma_calc", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
    ]


class DfOpts(ctypes.Structure):
    _fields_ = [
        ("prec", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("mix", ctypes.c_double),
        ("tol", ctypes.c_double), ("switch_tol", ctypes.c_double), ("use_graph", ctypes.c_int32),
        ("accel", ctypes.c_int32), ("symmetry", ctypes.c_int32), ("graph_unroll", ctypes.c_int32),
    ]


class DfError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libdf.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1507_00895_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.df_workspace_size.argtypes = [P(DfInst), ctypes.c_int32, P(DfOpts), P(ctypes.c_size_t)]
    for name in ("df_dual_gf", "df_bubble", "df_sigma"):
        getattr(lib, name).argtypes = [P(DfInst), ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p]
    lib.df_ladder_solve.argtypes = [P(DfInst), ctypes.c_int32, P(DfOpts), ctypes.c_void_p,
                                    ctypes.c_size_t, ctypes.c_void_p]
    lib.df_bubble_noalloc.argtypes = [P(DfInst), ctypes.c_int32, ctypes.c_void_p]
    lib.df_iterate.argtypes = [P(DfInst), ctypes.c_int32, P(DfOpts), P(ctypes.c_int32),
                               P(ctypes.c_double), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    lib.df_autotune.argtypes = [P(DfInst), ctypes.c_int32, P(DfOpts), ctypes.c_void_p,
                                ctypes.c_size_t, ctypes.c_void_p]
    lib.df_ladder_variant.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t]
    lib.df_ladder_set_variant.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p]
    lib.df_autotune_reset.argtypes = []
    lib.df_strerror.argtypes = [ctypes.c_int]
    lib.df_strerror.restype = ctypes.c_char_p
    lib.df_version.argtypes = []
    for name in EXPORTED:
        if name not in ("df_strerror",):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def df_strerror(code: int) -> str:
    return load().df_strerror(int(code)).decode()


def df_version() -> int:
    return load().df_version()


def _check(fn: str, code: int, ok=(DF_OK,)) -> int:
    if code not in ok:
        raise DfError(fn, code, df_strerror(code))
    return code


# ---------------------------------------------------------------------------
# tensors <-> df_inst_t
# ---------------------------------------------------------------------------
def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


@dataclass
class Instance:
    """Device tensors of one problem instance (torch, on a HIP device).

    complex tensors are torch.complex128, eps is float64, status is int8.
    """
    D: int
    nk: int
    n_nu: int
    n_om: int
    beta: float
    g: object
    delta: object
    eps: object
    gamma_uu: object
    gamma_ud: object
    sigma: object = None
    gd: object = None
    chi: object = None
    w: object = None
    logdet: object = None
    sigma_calc: object = None
    status: object = None
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.nk ** self.D

    def to_c(self) -> DfInst:
        for name in ("g", "delta", "gamma_uu", "gamma_ud", "sigma", "gd", "chi", "w", "logdet",
                     "sigma_calc"):
            t = getattr(self, name)
            if t is not None:
                import torch
                if t.dtype != torch.complex128 or not t.is_contiguous() or not t.is_cuda:
                    raise TypeError(f"{name} must be a contiguous complex128 device tensor")
        return DfInst(self.D, self.nk, self.n_nu, self.n_om, float(self.beta),
                      _ptr(self.g), _ptr(self.delta), _ptr(self.eps), _ptr(self.gamma_uu),
                      _ptr(self.gamma_ud), _ptr(self.sigma), _ptr(self.gd), _ptr(self.chi),
                      _ptr(self.w), _ptr(self.logdet), _ptr(self.sigma_calc), _ptr(self.status))


def make_instance(problem, device="cuda", outputs: bool = True) -> Instance:
    """Upload a Problem (paper_1507_00895_amd.inputs) and allocate its outputs."""
    import torch
    c = dict(dtype=torch.complex128, device=device)
    N = problem.N
    inst = Instance(
        D=problem.D, nk=problem.nk, n_nu=problem.n_nu, n_om=problem.n_om, beta=problem.beta,
        g=torch.as_tensor(problem.g, **c).contiguous(),
        delta=torch.as_tensor(problem.delta, **c).contiguous(),
        eps=torch.as_tensor(problem.eps, dtype=torch.float64, device=device).contiguous(),
        gamma_uu=torch.as_tensor(problem.gamma_uu, **c).contiguous(),
        gamma_ud=torch.as_tensor(problem.gamma_ud, **c).contiguous(),
        sigma=torch.zeros((problem.n_nu, N), **c),
        meta=problem.summary(),
    )
    if outputs:
        inst.gd = torch.zeros((problem.n_nu, N), **c)
        inst.chi = torch.zeros((problem.n_om, problem.n_nu, N), **c)
        inst.w = torch.zeros((2, problem.n_om, problem.n_nu, N), **c)
        inst.logdet = torch.zeros((2, problem.n_om, N), **c)
        inst.status = torch.zeros((2, problem.n_om, N), dtype=torch.int8, device=device)
        inst.sigma_calc = torch.zeros((problem.n_nu, N), **c)
    return inst


def _arr(insts: Sequence[Instance]):
    arr = (DfInst * len(insts))()
    for i, x in enumerate(insts):
        arr[i] = x.to_c()
    return arr


def _opts(prec=DF_FP64, mix=0.5, tol=0.0, max_iter=10, use_graph=0, switch_tol=0.0,
          accel=0, symmetry=0, graph_unroll=0) -> DfOpts:
    return DfOpts(int(prec), int(max_iter), float(mix), float(tol), float(switch_tol),
                  int(use_graph), int(accel), int(symmetry), int(graph_unroll))


def make_opts(**kw) -> DfOpts:
    return _opts(**kw)


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream) or None
    return int(stream) or None


def df_workspace_size(insts: Sequence[Instance], opts: Optional[DfOpts] = None) -> int:
    lib = load()
    n = ctypes.c_size_t(0)
    _check("df_workspace_size", lib.df_workspace_size(_arr(insts), len(insts),
                                                      ctypes.byref(opts) if opts else None,
                                                      ctypes.byref(n)))
    return int(n.value)


def workspace(insts: Sequence[Instance], opts: Optional[DfOpts] = None, device="cuda"):
    """A torch uint8 device buffer of the size libdf asks for (256-B aligned)."""
    import torch
    nbytes = df_workspace_size(insts, opts)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-int(buf.data_ptr())) % 256
    return buf[off:off + nbytes]


def df_dual_gf(insts, ws, stream=None):
    return _check("df_dual_gf", load().df_dual_gf(_arr(insts), len(insts), _ptr(ws), ws.numel(),
                                                  _stream(stream)))


def df_bubble(insts, ws, stream=None):
    return _check("df_bubble", load().df_bubble(_arr(insts), len(insts), _ptr(ws), ws.numel(),
                                                _stream(stream)))


def df_bubble_noalloc(insts, stream=None):
    """df_bubble without a workspace (the library's own device scratch)."""
    return _check("df_bubble_noalloc", load().df_bubble_noalloc(_arr(insts), len(insts),
                                                                _stream(stream)))


def df_ladder_solve(insts, ws, opts: Optional[DfOpts] = None, stream=None):
    return _check("df_ladder_solve",
                  load().df_ladder_solve(_arr(insts), len(insts),
                                         ctypes.byref(opts) if opts else None, _ptr(ws), ws.numel(),
                                         _stream(stream)))


def df_sigma(insts, ws, stream=None):
    return _check("df_sigma", load().df_sigma(_arr(insts), len(insts), _ptr(ws), ws.numel(),
                                              _stream(stream)))


def df_iterate(insts, ws, opts: DfOpts, stream=None, allow=(DF_OK, DF_W_FALLBACK)):
    """Run the loop; returns (status code, iterations, [final diff per instance])."""
    iters = ctypes.c_int32(0)
    diffs = (ctypes.c_double * len(insts))()
    code = load().df_iterate(_arr(insts), len(insts), ctypes.byref(opts), ctypes.byref(iters),
                             diffs, _ptr(ws), ws.numel(), _stream(stream))
    _check("df_iterate", code, ok=allow)
    return code, int(iters.value), list(diffs)


def df_autotune(insts, ws, opts: Optional[DfOpts] = None, stream=None):
    """Time the ladder kernel variants on these instances; keep the fastest (synchronous)."""
    return _check("df_autotune", load().df_autotune(_arr(insts), len(insts),
                                                    ctypes.byref(opts) if opts else None,
                                                    _ptr(ws), ws.numel(), _stream(stream)))


def df_ladder_variant(n_nu: int, prec: int = DF_FP64) -> str:
    buf = ctypes.create_string_buffer(32)
    _check("df_ladder_variant", load().df_ladder_variant(int(n_nu), int(prec), buf, 32))
    return buf.value.decode()


def df_ladder_set_variant(n_nu: int, prec: int, name: str):
    return _check("df_ladder_set_variant", load().df_ladder_set_variant(int(n_nu), int(prec),
                                                                        name.encode()))


LADDER_KERNELS = ("gjb", "gjb_o3", "vector", "mfma", "mixed", "mixed_o3", "fp32", "fp32_o4", "fp32_o5",
                  "gjb_o4", "mixed_o4")
# every choice: a kernel build with one work-group per item, or (the FP64
# certified builds with an item loop) a persistent grid of 1x / 2x the
# resident work-groups
LADDER_VARIANTS = LADDER_KERNELS + tuple(f"{k}@p{p}" for p in (1, 2) for k in ("gjb", "gjb_o3"))


def df_autotune_reset():
    return _check("df_autotune_reset", load().df_autotune_reset())


# ---------------------------------------------------------------------------
# lattice observables (include/df_lattice.h)
# ---------------------------------------------------------------------------
LATTICE_EXPORTED = ("df_lattice_workspace_size", "df_lattice")


def _lattice_lib():
    lib = load()
    if getattr(lib, "_lattice_ready", False):
        return lib
    P = ctypes.POINTER
    lib.df_lattice_workspace_size.argtypes = [P(DfInst), P(ctypes.c_size_t)]
    lib.df_lattice.argtypes = [P(DfInst), ctypes.c_double] + [ctypes.c_void_p] * 4 + \
        [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    for name in LATTICE_EXPORTED:
        getattr(lib, name).restype = ctypes.c_int
    lib._lattice_ready = True
    return lib


def df_lattice_workspace_size(inst: Instance) -> int:
    n = ctypes.c_size_t(0)
    c = inst.to_c()
    _check("df_lattice_workspace_size",
           _lattice_lib().df_lattice_workspace_size(ctypes.byref(c), ctypes.byref(n)))
    return int(n.value)


def lattice_workspace(inst: Instance, device="cuda"):
    """A torch uint8 device buffer of the size df_lattice asks for (256-B aligned)."""
    import torch
    nbytes = df_lattice_workspace_size(inst)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-int(buf.data_ptr())) % 256
    return buf[off:off + nbytes]


def df_lattice(inst: Instance, mu: float, sigma_lat=None, g_lat=None, chi_ch=None, chi_sp=None,
               ws=None, stream=None):
    """Lattice observables of inst (its sigma = the dual self-energy): writes the given
    complex128 device tensors sigma_lat, g_lat [n_nu][N] and chi_ch, chi_sp [N]."""
    import torch
    for name, t in (("sigma_lat", sigma_lat), ("g_lat", g_lat), ("chi_ch", chi_ch),
                    ("chi_sp", chi_sp)):
        if t is not None and (t.dtype != torch.complex128 or not t.is_contiguous() or not t.is_cuda):
            raise TypeError(f"{name} must be a contiguous complex128 device tensor")
    if ws is None:
        ws = lattice_workspace(inst, device=inst.g.device)
    c = inst.to_c()
    return _check("df_lattice", _lattice_lib().df_lattice(
        ctypes.byref(c), float(mu), _ptr(sigma_lat), _ptr(g_lat), _ptr(chi_ch), _ptr(chi_sp),
        _ptr(ws), ws.numel(), _stream(stream)))


# ---------------------------------------------------------------------------
# learned warm start (include/df_mlp.h)
# ---------------------------------------------------------------------------
MLP_EXPORTED = ("df_mlp_param_count", "df_mlp_workspace_size", "df_mlp_forward",
                "df_mlp_loss_grad", "df_mlp_adam")


def _mlp_lib():
    lib = load()
    if getattr(lib, "_mlp_ready", False):
        return lib
    P = ctypes.POINTER
    lib.df_mlp_param_count.argtypes = [ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_size_t)]
    lib.df_mlp_workspace_size.argtypes = [ctypes.c_int32, P(ctypes.c_int32), ctypes.c_int32,
                                          P(ctypes.c_size_t)]
    lib.df_mlp_forward.argtypes = [ctypes.c_int32, P(ctypes.c_int32), ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p]
    lib.df_mlp_loss_grad.argtypes = [ctypes.c_int32, P(ctypes.c_int32), ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_void_p]
    lib.df_mlp_adam.argtypes = [ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p]
    for name in MLP_EXPORTED:
        getattr(lib, name).restype = ctypes.c_int
    lib._mlp_ready = True
    return lib


def _dims(dims):
    arr = (ctypes.c_int32 * len(dims))(*[int(x) for x in dims])
    return len(dims) - 1, arr


def df_mlp_param_count(dims) -> int:
    n, arr = _dims(dims)
    c = ctypes.c_size_t(0)
    _check("df_mlp_param_count", _mlp_lib().df_mlp_param_count(n, arr, ctypes.byref(c)))
    return int(c.value)


def mlp_workspace(dims, batch, device="cuda"):
    import torch
    n, arr = _dims(dims)
    c = ctypes.c_size_t(0)
    _check("df_mlp_workspace_size", _mlp_lib().df_mlp_workspace_size(n, arr, int(batch), ctypes.byref(c)))
    buf = torch.empty(int(c.value) + 256, dtype=torch.uint8, device=device)
    off = (-int(buf.data_ptr())) % 256
    return buf[off:off + int(c.value)]


def _f32(t, name):
    import torch
    if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
        raise TypeError(f"{name} must be a contiguous float32 device tensor")
    return int(t.data_ptr())


def df_mlp_forward(dims, params, X, Y, ws, stream=None):
    n, arr = _dims(dims)
    return _check("df_mlp_forward", _mlp_lib().df_mlp_forward(
        n, arr, _f32(params, "params"), _f32(X, "X"), int(X.shape[0]), _f32(Y, "Y"),
        _ptr(ws), ws.numel(), _stream(stream)))


def df_mlp_loss_grad(dims, params, X, T, grads, loss, ws, stream=None):
    n, arr = _dims(dims)
    return _check("df_mlp_loss_grad", _mlp_lib().df_mlp_loss_grad(
        n, arr, _f32(params, "params"), _f32(X, "X"), _f32(T, "T"), int(X.shape[0]),
        _f32(grads, "grads"), None if loss is None else _f32(loss, "loss"), _ptr(ws), ws.numel(),
        _stream(stream)))


def df_mlp_adam(params, grads, m, v, step, lr, stream=None):
    return _check("df_mlp_adam", _mlp_lib().df_mlp_adam(
        params.numel(), _f32(params, "params"), _f32(grads, "grads"), _f32(m, "m"), _f32(v, "v"),
        int(step), float(lr), _stream(stream)))
