"""ctypes binding of libelmfb.so: the C ABI of include/elmfb.h with the same names.

Argument marshalling only: every step of the computation runs in the library's HIP kernels.
Device buffers are torch CUDA (HIP) tensors; their data pointers are handed to the library and
the current torch stream is used unless a stream handle is given.  There is no fallback: if the
library is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libelmfb.so")

ABI_VERSION = 5
MAX_BC = 4
MAX_BC_PTS = 4096
MAX_LEVELS = 8

OK, E_INVALID, E_NOMEM, E_DEVICE, E_STATE, E_NUMERIC, E_UNSUPPORTED = range(7)
OP_D1, OP_NEG_LAPLACE, OP_IDENTITY, OP_OSCILLATOR, OP_HELMHOLTZ = 1, 2, 3, 4, 5
DOMAIN_BOX, DOMAIN_L = 0, 1
ANSATZ_NONE, ANSATZ_TANH_ORIGIN, ANSATZ_TANH_BOX = 0, 1, 2
FP64, FP32, BF16, FP16 = 0, 1, 2, 3
COPY_FOLDED = 0x100
LSQR, CGLS, MIXED_IR, NORMAL_CG, MIXED_IR_CG = 0, 1, 2, 3, 4

_OPS = {"d1": OP_D1, "neg_laplace": OP_NEG_LAPLACE, "identity": OP_IDENTITY,
        "oscillator": OP_OSCILLATOR, "helmholtz": OP_HELMHOLTZ}
_DOMAINS = {"box": DOMAIN_BOX, "l_shape": DOMAIN_L}
_ANSATZ = {"none": ANSATZ_NONE, "tanh_origin": ANSATZ_TANH_ORIGIN, "tanh_box": ANSATZ_TANH_BOX}
_PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp16": FP16}
_METHOD = {"lsqr": LSQR, "cgls": CGLS, "mixed_ir": MIXED_IR, "normal_cg": NORMAL_CG,
           "mixed_ir_cg": MIXED_IR_CG}


class ProblemDesc(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("op", ctypes.c_int32),
        ("ansatz", ctypes.c_int32),
        ("ansatz_omega", ctypes.c_double),
        ("lo", ctypes.c_double * 2),
        ("hi", ctypes.c_double * 2),
        ("n_points", ctypes.c_int32 * 2),
        ("n_levels", ctypes.c_int32),
        ("J", (ctypes.c_int32 * 2) * MAX_LEVELS),
        ("delta", ctypes.c_double),
        ("K", ctypes.c_int32),
        ("store_prec", ctypes.c_int32),
        ("W_host", ctypes.POINTER(ctypes.c_double)),
        ("b_host", ctypes.POINTER(ctypes.c_double)),
        ("op_coef", ctypes.c_double * 3),
        ("n_bc", ctypes.c_int32),
        ("bc_order", ctypes.c_int32 * MAX_BC),
        ("bc_x", ctypes.c_double * MAX_BC),
        ("bc_weight", ctypes.c_double * MAX_BC),
        ("bc_value", ctypes.c_double * MAX_BC),
        ("domain", ctypes.c_int32),
        ("n_bc_pts", ctypes.c_int32),
        ("bc_pts_host", ctypes.POINTER(ctypes.c_double)),
        ("bc_pts_val_host", ctypes.POINTER(ctypes.c_double)),
        ("bc_pts_weight", ctypes.c_double),
        ("input_norm", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("w_range", ctypes.c_double * 2),
        ("b_range", ctypes.c_double * 2),
    ]


class Sizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_rows", "n_phi", "nnz", "n_blocks", "n_block_points", "bytes_device",
                 "n_pairs", "n_bc", "n_interior")]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int32),
        ("iter_lim", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("inner_iters", ctypes.c_int32),
        ("outer_lim", ctypes.c_int32),
        ("atol", ctypes.c_double),
        ("btol", ctypes.c_double),
        ("x0_dev", ctypes.c_void_p),
        ("check_pts_dev", ctypes.c_void_p),
        ("check_ref_dev", ctypes.c_void_p),
        ("n_check", ctypes.c_int64),
        ("target_rel_l2", ctypes.c_double),
        ("n_rhs", ctypes.c_int32),
        ("estimate_cond", ctypes.c_int32),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("istop", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("outer_iters", ctypes.c_int32),
        ("rnorm", ctypes.c_double),
        ("arnorm", ctypes.c_double),
        ("anorm", ctypes.c_double),
        ("xnorm", ctypes.c_double),
        ("rel_l2", ctypes.c_double),
        ("ms_solve", ctypes.c_double),
        ("acond", ctypes.c_double),
        ("ms_assemble", ctypes.c_double),
    ]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class BatchShape(ctypes.Structure):
    _fields_ = [("rmvb_tile", ctypes.c_int32), ("mvb_ahead", ctypes.c_int32),
                ("gather_rows", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("ms_rmvb", ctypes.c_double * 3), ("ms_mvb", ctypes.c_double * 3),
                ("ms_gather", ctypes.c_double * 2)]

    def as_dict(self):
        return {"rmvb_tile": self.rmvb_tile, "mvb_ahead": self.mvb_ahead,
                "gather_rows": self.gather_rows, "from_cache": bool(self.from_cache),
                "ms_rmvb": {t: self.ms_rmvb[i] for i, t in enumerate((16, 32, 64))
                            if self.ms_rmvb[i] >= 0},
                "ms_mvb": {a: self.ms_mvb[i] for i, a in enumerate((4, 8, 16))
                           if self.ms_mvb[i] >= 0},
                "ms_gather": {r: self.ms_gather[i] for i, r in enumerate((1, 2))
                              if self.ms_gather[i] >= 0}}


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


class ElmfbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"elmfb error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: Optional[str] = None):
    """Load libelmfb.so (built in-tree by build.py) and declare the ABI signatures."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2409_01949_amd/build.py")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7); load it first
    # so that the library and torch's device allocations share one runtime in this process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "elmfb_define_problem": (i32, [ctypes.POINTER(ProblemDesc), ctypes.POINTER(P)]),
        "elmfb_draw_features": (i32, [ctypes.POINTER(ProblemDesc), ctypes.POINTER(dbl),
                                      ctypes.POINTER(dbl)]),
        "elmfb_query": (i32, [P, ctypes.POINTER(Sizes)]),
        "elmfb_points": (i32, [P, P, P]),
        "elmfb_assemble": (i32, [P, P, i32, P]),
        "elmfb_matvec": (i32, [P, P, P, P]),
        "elmfb_rmatvec": (i32, [P, P, P, P]),
        "elmfb_copy_rhs": (i32, [P, P, P]),
        "elmfb_copy_bc": (i32, [P, P, P]),
        "elmfb_copy_blocks": (i32, [P, i32, P, ctypes.POINTER(i64), P]),
        "elmfb_gram": (i32, [P, i32, i32, P]),
        "elmfb_copy_gram": (i32, [P, P, ctypes.POINTER(i64), ctypes.POINTER(i64), P]),
        "elmfb_precondition": (i32, [P, dbl, ctypes.POINTER(i32), P]),
        "elmfb_solve": (i32, [P, ctypes.POINTER(SolveOpts), P, ctypes.POINTER(SolveInfo), P]),
        "elmfb_evaluate": (i32, [P, P, i32, P, i64, P, P]),
        "elmfb_condition_estimate": (i32, [P, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                           ctypes.POINTER(i32)]),
        "elmfb_bidiag_sigma": (i32, [P, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
        "elmfb_time_kernels": (i32, [P, i32, i32, ctypes.POINTER(dbl), P]),
        "elmfb_time_gram_mv": (i32, [P, i32, ctypes.POINTER(dbl), P]),
        "elmfb_time_gram": (i32, [P, i32, i32, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl), P]),
        "elmfb_define_batch": (i32, [ctypes.POINTER(ProblemDesc), i32, i32, ctypes.POINTER(P)]),
        "elmfb_batch_query": (i32, [P, ctypes.POINTER(i64), ctypes.POINTER(Sizes)]),
        "elmfb_batch_query_instances": (i32, [P, ctypes.POINTER(Sizes)]),
        "elmfb_batch_assemble": (i32, [P, P, P]),
        "elmfb_batch_copy_blocks": (i32, [P, i32, P, ctypes.POINTER(i64), P]),
        "elmfb_batch_matvec": (i32, [P, P, P, P]),
        "elmfb_batch_rmatvec": (i32, [P, P, P, P]),
        "elmfb_batch_precondition": (i32, [P, ctypes.c_double, ctypes.POINTER(i32), P]),
        "elmfb_batch_precondition_patches": (i32, [P, ctypes.c_double, i32, ctypes.POINTER(i32),
                                                   P]),
        "elmfb_batch_patch_info": (i32, [P, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                         ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "elmfb_batch_autotune": (i32, [P, i32, i32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(i32), P]),
        "elmfb_batch_set_tile": (i32, [P, i32, i32]),
        "elmfb_batch_tune": (i32, [P, i32, i32, i32, ctypes.POINTER(BatchShape), P]),
        "elmfb_batch_set_shape": (i32, [P, i32, ctypes.POINTER(BatchShape)]),
        "elmfb_batch_time_kernels": (i32, [P, i32, i32, ctypes.POINTER(ctypes.c_double), P]),
        "elmfb_batch_set_coords": (i32, [P, i32]),
        "elmfb_batch_from_coords": (i32, [P, P, P, P]),
        "elmfb_batch_solve": (i32, [P, ctypes.POINTER(SolveOpts), P, ctypes.POINTER(SolveInfo), P]),
        "elmfb_batch_destroy": (None, [P]),
        "elmfb_batch_last_error": (ctypes.c_char_p, [P]),
        "elmfb_mlp_create": (i32, [i32, ctypes.POINTER(i32), i32, i32, ctypes.POINTER(P)]),
        "elmfb_mlp_query": (i32, [P, ctypes.POINTER(i64)]),
        "elmfb_mlp_set_params": (i32, [P, P]),
        "elmfb_mlp_get_params": (i32, [P, P]),
        "elmfb_mlp_get_grads": (i32, [P, P]),
        "elmfb_mlp_forward": (i32, [P, P, P, i32, P, P]),
        "elmfb_mlp_train_step": (i32, [P, P, P, P, i32, ctypes.POINTER(Adam), ctypes.POINTER(dbl),
                                       P]),
        "elmfb_mlp_destroy": (None, [P]),
        "elmfb_mlp_last_error": (ctypes.c_char_p, [P]),
        "elmfb_destroy": (None, [P]),
        "elmfb_last_error": (ctypes.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def bidiag_sigma(ab):
    """(sigma_max, sigma_min) of the lower bidiagonal given as (alpha_{i+1}, beta_{i+1}) pairs,
    i = 0..k, computed by the library on the host."""
    lib = load_library()
    a = np.ascontiguousarray(np.asarray(ab, dtype=np.float64).reshape(-1))
    k = a.size // 2 - 1
    smax, smin = ctypes.c_double(), ctypes.c_double()
    _check(lib.elmfb_bidiag_sigma(a.ctypes.data_as(ctypes.c_void_p), k, ctypes.byref(smax),
                                  ctypes.byref(smin)))
    return smax.value, smin.value


def _ptr(t) -> int:
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        if not t.is_cuda:
            raise ValueError("device tensor required")
        if not t.is_contiguous():
            raise ValueError("contiguous tensor required")
        return t.data_ptr()
    return int(t)


def _stream(stream):
    if stream is not None:
        return int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


def _check(code, handle=None):
    if code != OK:
        msg = _lib.elmfb_last_error(handle)
        raise ElmfbError(code, msg.decode() if msg else "")


def make_desc(dim, op, ansatz, ansatz_omega, lo, hi, n_points, levels, delta, K, W, b,
              store_prec="fp64", op_coef=(0.0, 0.0, 0.0), bc=(), domain="box", bc_pts=None,
              bc_vals=None, bc_weight=0.0, input_norm="local", seed=0, w_range=(-1.0, 1.0),
              b_range=(-1.0, 1.0)):
    """Descriptor from plain values.  W [n_phi, dim] and b [n_phi] are float64 host arrays
    (on an L-shaped domain: for every subdomain of each level's full grid), or both None for the
    library to draw them from seed over w_range and b_range; the returned tuple keeps them
    alive for the duration of the define call.  bc: 1D soft constraints as (x, derivative
    order, weight sqrt(lambda), value) tuples; bc_pts [n, 2], bc_vals [n], bc_weight: 2D
    Dirichlet rows at points; input_norm "local" or "global" feature inputs."""
    d = ProblemDesc()
    d.abi_version = ABI_VERSION
    d.dim = int(dim)
    d.op = _OPS[op] if isinstance(op, str) else int(op)
    d.ansatz = _ANSATZ[ansatz] if isinstance(ansatz, str) else int(ansatz)
    d.ansatz_omega = float(ansatz_omega)
    for a in range(2):
        d.lo[a] = float(lo[a]) if a < len(lo) else 0.0
        d.hi[a] = float(hi[a]) if a < len(hi) else 1.0
        d.n_points[a] = int(n_points[a]) if a < len(n_points) else 1
    d.n_levels = len(levels)
    for l, J in enumerate(levels[:MAX_LEVELS]):
        for a in range(2):
            d.J[l][a] = int(J[a]) if a < len(J) else 1
    d.delta = float(delta)
    d.K = int(K)
    d.store_prec = _PREC[store_prec] if isinstance(store_prec, str) else int(store_prec)
    for i, c in enumerate(op_coef):
        d.op_coef[i] = float(c)
    d.n_bc = len(bc)
    for i, (x, order, wgt, val) in enumerate(bc[:MAX_BC]):
        d.bc_x[i], d.bc_order[i], d.bc_weight[i], d.bc_value[i] = float(x), int(order), \
            float(wgt), float(val)
    keep = []
    if W is not None or b is not None:
        W = np.ascontiguousarray(W, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        d.W_host = W.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.b_host = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        keep = [W, b]
    d.domain = _DOMAINS[domain] if isinstance(domain, str) else int(domain)
    d.input_norm = {"local": 0, "global": 1}[input_norm] if isinstance(input_norm, str) \
        else int(input_norm)
    d.seed = int(seed) & ((1 << 64) - 1)
    for i in range(2):
        d.w_range[i] = float(w_range[i])
        d.b_range[i] = float(b_range[i])
    if bc_pts is not None:
        P = np.ascontiguousarray(bc_pts, dtype=np.float64).reshape(-1, 2)
        G = np.ascontiguousarray(bc_vals, dtype=np.float64).reshape(-1)
        d.n_bc_pts = P.shape[0]
        d.bc_pts_host = P.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.bc_pts_val_host = G.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.bc_pts_weight = float(bc_weight)
        keep += [P, G]
    return d, tuple(keep)


def desc_from_spec(spec, W, b, store_prec="fp64", bc_pts=None, bc_vals=None, bc_weight=0.0):
    """Descriptor from any object with the problem-specification attributes (Helmholtz: the
    operator's k^2 from meta["k"]; the Dirichlet points, values and weight from the caller)."""
    meta = getattr(spec, "meta", {}) or {}
    coef = meta.get("osc", (0.0, 0.0, 0.0))
    if spec.op == "helmholtz":
        coef = (float(meta["k"]) ** 2, 0.0, 0.0)
    return make_desc(spec.dim, spec.op, spec.ansatz, spec.ansatz_omega, spec.lo, spec.hi,
                     spec.n_points, spec.levels, spec.delta, spec.K, W, b, store_prec,
                     op_coef=coef, bc=tuple(meta.get("bc", ())),
                     domain=getattr(spec, "domain", "box"), bc_pts=bc_pts, bc_vals=bc_vals,
                     bc_weight=bc_weight, input_norm=getattr(spec, "input_norm", "local"),
                     seed=getattr(spec, "seed", 0), w_range=getattr(spec, "w_range", (-1.0, 1.0)),
                     b_range=getattr(spec, "b_range", (-1.0, 1.0)))


def draw_features(desc_and_keep):
    """The library's draw of W [n_params, dim] and b [n_params] for a descriptor (host code)."""
    lib = load_library()
    desc, _ = desc_and_keep
    n = desc.K * sum(int(np.prod([desc.J[l][a] for a in range(desc.dim)]))
                     for l in range(desc.n_levels))
    W = np.empty((n, desc.dim), dtype=np.float64)
    b = np.empty(n, dtype=np.float64)
    code = lib.elmfb_draw_features(ctypes.byref(desc),
                                   W.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if code != OK:
        msg = lib.elmfb_last_error(None)
        raise ElmfbError(code, msg.decode() if msg else "")
    return W, b


def define_problem(desc_and_keep) -> "Problem":
    lib = load_library()
    desc, keep = desc_and_keep
    h = ctypes.c_void_p()
    code = lib.elmfb_define_problem(ctypes.byref(desc), ctypes.byref(h))
    del keep
    if code != OK:
        msg = lib.elmfb_last_error(None)
        raise ElmfbError(code, msg.decode() if msg else "")
    return Problem(h)


class Problem:
    """Owns one elmfb_problem handle."""

    def __init__(self, handle):
        self.h = handle
        self.sizes = self.query()

    @classmethod
    def from_spec(cls, spec, W, b, store_prec="fp64", **bc):
        return define_problem(desc_from_spec(spec, W, b, store_prec, **bc))

    def query(self):
        s = Sizes()
        _check(_lib.elmfb_query(self.h, ctypes.byref(s)), self.h)
        return {n: getattr(s, n) for n, _ in Sizes._fields_}

    def points(self, xy, stream=None):
        _check(_lib.elmfb_points(self.h, _ptr(xy), _stream(stream)), self.h)

    def assemble(self, f, stream=None, n_rhs=None):
        """M and the right-hand sides of f [n_rhs, n_rows] (n_rhs from f's size by default)."""
        if n_rhs is None:
            n_rhs = max(1, int(f.numel()) // int(self.sizes["n_rows"]))
        _check(_lib.elmfb_assemble(self.h, _ptr(f), int(n_rhs), _stream(stream)), self.h)
        self.n_rhs = int(n_rhs)

    def matvec(self, v, y, stream=None):
        _check(_lib.elmfb_matvec(self.h, _ptr(v), _ptr(y), _stream(stream)), self.h)

    def rmatvec(self, u, x, stream=None):
        _check(_lib.elmfb_rmatvec(self.h, _ptr(u), _ptr(x), _stream(stream)), self.h)

    def copy_rhs(self, hvec, stream=None):
        _check(_lib.elmfb_copy_rhs(self.h, _ptr(hvec), _stream(stream)), self.h)

    def copy_bc(self, dst, stream=None):
        """The soft-constraint rows [n_bc, n_phi] into dst (FP64)."""
        _check(_lib.elmfb_copy_bc(self.h, _ptr(dst), _stream(stream)), self.h)

    def copy_blocks(self, dst=None, prec="fp64", folded=False, stream=None):
        """Returns the block table [n_blocks, 8] (int64); copies raw blocks into dst if given
        (folded: the block-Jacobi-folded M R^-1 instead of M)."""
        nb = self.sizes["n_blocks"]
        table = np.zeros((nb, 8), dtype=np.int64)
        pr = _PREC[prec] if isinstance(prec, str) else int(prec)
        if folded:
            pr |= COPY_FOLDED
        _check(_lib.elmfb_copy_blocks(self.h, pr, _ptr(dst) if dst is not None else None,
                                      table.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      _stream(stream)), self.h)
        return table

    def gram(self, prec="fp64", which="all", stream=None):
        pr = _PREC[prec] if isinstance(prec, str) else int(prec)
        w = {"diag": 0, "all": 1}[which] if isinstance(which, str) else int(which)
        _check(_lib.elmfb_gram(self.h, pr, w, _stream(stream)), self.h)

    def copy_gram(self, dst=None, stream=None):
        """Pair table [n_pairs, 3] (bi, bj, offset); copies the blocks into dst if given."""
        n = ctypes.c_int64()
        _check(_lib.elmfb_copy_gram(self.h, None, None, ctypes.byref(n), _stream(stream)), self.h)
        table = np.zeros((n.value, 3), dtype=np.int64)
        _check(_lib.elmfb_copy_gram(self.h, _ptr(dst) if dst is not None else None,
                                    table.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    ctypes.byref(n), _stream(stream)), self.h)
        return table

    def precondition(self, shift=1e-12, stream=None):
        """Block-Jacobi factors; returns the number of blocks that fell back to the identity."""
        nf = ctypes.c_int32()
        _check(_lib.elmfb_precondition(self.h, float(shift), ctypes.byref(nf), _stream(stream)),
               self.h)
        return nf.value

    def solve(self, coef, method="lsqr", iter_lim=15000, atol=1e-8, btol=1e-8, check_every=50,
              use_graph=True, x0=None, check_pts=None, check_ref=None, target_rel_l2=0.0,
              precond=False, inner_iters=100, outer_lim=10, stream=None, n_rhs=1,
              estimate_cond=False):
        """Solve for n_rhs assembled right-hand sides into coef [n_rhs, n_phi]; returns the
        info dict (a list of them when n_rhs > 1)."""
        o = SolveOpts()
        o.method = _METHOD[method] if isinstance(method, str) else int(method)
        o.iter_lim = int(iter_lim)
        o.check_every = int(check_every)
        o.use_graph = 1 if use_graph else 0
        o.precond = 1 if precond else 0
        o.inner_iters = int(inner_iters)
        o.outer_lim = int(outer_lim)
        o.atol = float(atol)
        o.btol = float(btol)
        o.x0_dev = _ptr(x0)
        o.check_pts_dev = _ptr(check_pts)
        o.check_ref_dev = _ptr(check_ref)
        o.n_check = int(check_pts.shape[0]) if check_ref is not None else 0
        o.target_rel_l2 = float(target_rel_l2)
        o.n_rhs = int(n_rhs)
        o.estimate_cond = 1 if estimate_cond else 0
        infos = (SolveInfo * max(1, int(n_rhs)))()
        _check(_lib.elmfb_solve(self.h, ctypes.byref(o), _ptr(coef), infos, _stream(stream)),
               self.h)
        out = [i.as_dict() for i in infos]
        return out[0] if n_rhs <= 1 else out

    def evaluate(self, coef, pts, u, stream=None, n_rhs=None):
        """u [n_rhs, n_pts] at pts [n_pts, dim] for coef [n_rhs, n_phi]."""
        n = pts.shape[0]
        if n_rhs is None:
            n_rhs = max(1, int(coef.numel()) // int(self.sizes["n_phi"]))
        _check(_lib.elmfb_evaluate(self.h, _ptr(coef), int(n_rhs), _ptr(pts), int(n), _ptr(u),
                                   _stream(stream)), self.h)

    def condition_estimate(self):
        """(sigma_max, sigma_min, k) of the bidiagonal B_k that the last solve's LSQR built."""
        smax, smin, k = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        _check(_lib.elmfb_condition_estimate(self.h, ctypes.byref(smax), ctypes.byref(smin),
                                             ctypes.byref(k)), self.h)
        return smax.value, smin.value, k.value

    def time_kernels(self, reps=20, prec="fp64", stream=None):
        """Average duration (ms) of one launch of the M v and M^T u streaming kernels, then of
        the row gather and the column pass that complete them."""
        out = (ctypes.c_double * 4)()
        pr = _PREC[prec] if isinstance(prec, str) else int(prec)
        _check(_lib.elmfb_time_kernels(self.h, pr, int(reps), out, _stream(stream)), self.h)
        return tuple(float(v) for v in out)

    def time_gram(self, prec="fp64", which="all", reps=5, stream=None):
        """(ms per Gram computation, useful flops) after computing the blocks as gram() does."""
        ms, fl = ctypes.c_double(), ctypes.c_double()
        pr = _PREC[prec] if isinstance(prec, str) else int(prec)
        w = {"diag": 0, "all": 1}[which] if isinstance(which, str) else int(which)
        _check(_lib.elmfb_time_gram(self.h, pr, w, int(reps), ctypes.byref(ms), ctypes.byref(fl),
                                    _stream(stream)), self.h)
        return ms.value, fl.value

    def time_gram_mv(self, reps=20, stream=None):
        """Average duration (ms) of the per-block pass of y = G p alone and of both passes."""
        out = (ctypes.c_double * 2)()
        _check(_lib.elmfb_time_gram_mv(self.h, int(reps), out, _stream(stream)), self.h)
        return float(out[0]), float(out[1])

    def destroy(self):
        if self.h is not None and _lib is not None:
            _lib.elmfb_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Batch:
    """Owns one elmfb_batch handle: many instances, n_rhs right-hand sides each."""

    def __init__(self, specs, Ws, bs, n_rhs, store_prec="fp64"):
        lib = load_library()
        keep = []
        arr = (ProblemDesc * len(specs))()
        for i, (sp, W, b) in enumerate(zip(specs, Ws, bs)):
            d, k = desc_from_spec(sp, W, b, store_prec)
            arr[i] = d
            keep.append(k)
        h = ctypes.c_void_p()
        code = lib.elmfb_define_batch(arr, len(specs), int(n_rhs), ctypes.byref(h))
        if code != OK:
            msg = lib.elmfb_last_error(None) or b""
            msg2 = lib.elmfb_batch_last_error(None) or b""
            raise ElmfbError(code, (msg2 or msg).decode())
        self.h = h
        self.n = len(specs)
        self.n_rhs = int(n_rhs)
        offs = np.zeros((self.n + 1, 2), dtype=np.int64)
        tot = Sizes()
        self._check(lib.elmfb_batch_query(self.h, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          ctypes.byref(tot)))
        self.offsets = offs
        self.sizes = {n: getattr(tot, n) for n, _ in Sizes._fields_}

    def _check(self, code):
        if code != OK:
            msg = _lib.elmfb_batch_last_error(self.h)
            raise ElmfbError(code, msg.decode() if msg else "")

    def query(self):
        """Totals over the batch as they stand (bytes_device changes as factors are formed);
        also refreshes self.sizes."""
        offs = np.zeros((self.n + 1, 2), dtype=np.int64)
        tot = Sizes()
        self._check(_lib.elmfb_batch_query(self.h, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           ctypes.byref(tot)))
        self.sizes = {n: getattr(tot, n) for n, _ in Sizes._fields_}
        return dict(self.sizes)

    def assemble(self, f, stream=None):
        self._check(_lib.elmfb_batch_assemble(self.h, _ptr(f), _stream(stream)))

    def query_instances(self):
        """Per-instance sizes: a list of dicts like Problem.query()."""
        arr = (Sizes * self.n)()
        self._check(_lib.elmfb_batch_query_instances(self.h, arr))
        return [{n: getattr(z, n) for n, _ in Sizes._fields_} for z in arr]

    def copy_blocks(self, dst=None, prec="fp64", folded=False, stream=None):
        """Block table [n_blocks, 8] (instance, level, ix0, nx, iy0, ny, K, element offset);
        copies the raw blocks of M (or, folded, of M R^-1: the patch blocks when the factors are
        of patches) in precision prec into dst if given."""
        nb = self.patch_info()["n_blocks"] if folded else self.sizes["n_blocks"]
        table = np.zeros((nb, 8), dtype=np.int64)
        pr = _PREC[prec] if isinstance(prec, str) else int(prec)
        if folded:
            pr |= COPY_FOLDED
        self._check(_lib.elmfb_batch_copy_blocks(
            self.h, pr, _ptr(dst) if dst is not None else None,
            table.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _stream(stream)))
        return table

    def matvec(self, v, y, stream=None):
        self._check(_lib.elmfb_batch_matvec(self.h, _ptr(v), _ptr(y), _stream(stream)))

    def rmatvec(self, u, x, stream=None):
        self._check(_lib.elmfb_batch_rmatvec(self.h, _ptr(u), _ptr(x), _stream(stream)))

    def precondition(self, shift=1e-12, patch=1, stream=None):
        """Block-Jacobi factors of every block (patch = 1) or of every patch of patch^d
        neighbouring subdomains; returns the number of identity fallbacks."""
        nf = ctypes.c_int32(0)
        if patch == 1:
            self._check(_lib.elmfb_batch_precondition(self.h, float(shift), ctypes.byref(nf),
                                                      _stream(stream)))
        else:
            self._check(_lib.elmfb_batch_precondition_patches(self.h, float(shift), int(patch),
                                                              ctypes.byref(nf), _stream(stream)))
        return int(nf.value)

    def patch_info(self, perm=False):
        """{'patch', 'n_blocks', 'n_entries'} of the factors held, and with perm=True the original
        column of every column of the preconditioned coefficients' order ('perm', int32)."""
        pt = ctypes.c_int32(0)
        nb = ctypes.c_int64(0)
        ne = ctypes.c_int64(0)
        pv = np.zeros(self.sizes["n_phi"], dtype=np.int32) if perm else None
        self._check(_lib.elmfb_batch_patch_info(
            self.h, ctypes.byref(pt), ctypes.byref(nb), ctypes.byref(ne),
            pv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if perm else None))
        out = {"patch": int(pt.value), "n_blocks": int(nb.value), "n_entries": int(ne.value)}
        if perm:
            out["perm"] = pv
        return out

    def autotune(self, prec="fp64", reps=5, stream=None):
        """Time the M^T U tile variants; returns ({tile: ms}, chosen tile)."""
        ms = (ctypes.c_double * 3)()
        ch = ctypes.c_int32(0)
        self._check(_lib.elmfb_batch_autotune(self.h, _PREC[prec], int(reps), ms, ctypes.byref(ch),
                                              _stream(stream)))
        return {t: ms[i] for i, t in enumerate((16, 32, 64)) if ms[i] >= 0}, int(ch.value)

    def set_coords(self, preconditioned):
        """Solve coefficients (x0 and result) as y = R x per block when True."""
        self._check(_lib.elmfb_batch_set_coords(self.h, 1 if preconditioned else 0))

    def from_coords(self, y, x, stream=None):
        """x = R^{-1} y per block (V layout)."""
        self._check(_lib.elmfb_batch_from_coords(self.h, _ptr(y), _ptr(x), _stream(stream)))

    def set_tile(self, prec, tile):
        self._check(_lib.elmfb_batch_set_tile(self.h, _PREC[prec], int(tile)))

    def tune(self, prec, reps=3, use_cache=True, stream=None):
        """Time the shapes of the M^T U, M V and gather passes and keep the fastest (or take
        them from the process's cache); returns the shapes and timings as a dict."""
        sh = BatchShape()
        self._check(_lib.elmfb_batch_tune(self.h, _PREC[prec], int(reps), 1 if use_cache else 0,
                                          ctypes.byref(sh), _stream(stream)))
        return sh.as_dict()

    def set_shape(self, prec, rmvb_tile=32, mvb_ahead=8, gather_rows=1):
        sh = BatchShape()
        sh.rmvb_tile, sh.mvb_ahead, sh.gather_rows = int(rmvb_tile), int(mvb_ahead), int(gather_rows)
        self._check(_lib.elmfb_batch_set_shape(self.h, _PREC[prec], ctypes.byref(sh)))

    def time_kernels(self, prec, reps=10, stream=None):
        """Average ms per launch of the batched M V pass, the row gather and the M^T U pass."""
        ms = (ctypes.c_double * 3)()
        self._check(_lib.elmfb_batch_time_kernels(self.h, _PREC[prec], int(reps), ms,
                                                  _stream(stream)))
        return tuple(float(v) for v in ms)

    def solve(self, coef, iter_lim=15000, atol=0.0, btol=1e-6, check_every=50, use_graph=True,
              method="lsqr", precond=False, inner_iters=500, outer_lim=20, x0=None, stream=None):
        o = SolveOpts()
        o.x0_dev = _ptr(x0)
        o.method = {"lsqr": LSQR, "mixed_ir": MIXED_IR}[method]
        o.iter_lim = int(iter_lim)
        o.check_every = int(check_every)
        o.use_graph = 1 if use_graph else 0
        o.precond = 1 if precond else 0
        o.inner_iters = int(inner_iters)
        o.outer_lim = int(outer_lim)
        o.atol = float(atol)
        o.btol = float(btol)
        infos = (SolveInfo * (self.n * self.n_rhs))()
        self._check(_lib.elmfb_batch_solve(self.h, ctypes.byref(o), _ptr(coef), infos,
                                           _stream(stream)))
        return [i.as_dict() for i in infos]

    def destroy(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.elmfb_batch_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class MLP:
    """Owns one elmfb_mlp handle (tanh network, bfloat16 products, FP32 master weights); with
    n_mod > 1 the output is modulated by per-sample weights f: y[k] = sum_i f_i z[i K + k]."""

    def __init__(self, dims, max_batch, n_mod=1):
        lib = load_library()
        d = (ctypes.c_int32 * len(dims))(*[int(v) for v in dims])
        h = ctypes.c_void_p()
        code = lib.elmfb_mlp_create(len(dims) - 1, d, int(n_mod), int(max_batch), ctypes.byref(h))
        if code != OK:
            raise ElmfbError(code, (lib.elmfb_mlp_last_error(None) or b"").decode())
        self.h = h
        self.dims = list(dims)
        self.n_mod = int(n_mod)
        self.n_out = self.dims[-1] // self.n_mod
        self.max_batch = int(max_batch)
        n = ctypes.c_int64(0)
        self._check(lib.elmfb_mlp_query(self.h, ctypes.byref(n)))
        self.n_params = int(n.value)

    def _check(self, code):
        if code != OK:
            msg = _lib.elmfb_mlp_last_error(self.h)
            raise ElmfbError(code, msg.decode() if msg else "")

    def set_params(self, vec):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        assert v.size == self.n_params
        self._check(_lib.elmfb_mlp_set_params(self.h, v.ctypes.data))

    def get_params(self):
        v = np.empty(self.n_params, dtype=np.float32)
        self._check(_lib.elmfb_mlp_get_params(self.h, v.ctypes.data))
        return v

    def get_grads(self):
        v = np.empty(self.n_params, dtype=np.float32)
        self._check(_lib.elmfb_mlp_get_grads(self.h, v.ctypes.data))
        return v

    def forward(self, x, f=None, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=x.device)
        self._check(_lib.elmfb_mlp_forward(self.h, _ptr(x), _ptr(f), int(x.shape[0]), _ptr(y),
                                           _stream(stream)))
        return y

    def train_step(self, x, t, f=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, update=True,
                   want_loss=True, stream=None):
        opt = Adam(lr, beta1, beta2, eps)
        loss = ctypes.c_double(0.0)
        self._check(_lib.elmfb_mlp_train_step(self.h, _ptr(x), _ptr(f), _ptr(t), int(x.shape[0]),
                                              ctypes.byref(opt) if update else None,
                                              ctypes.byref(loss) if want_loss else None,
                                              _stream(stream)))
        return float(loss.value) if want_loss else None

    def destroy(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.elmfb_mlp_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
