"""MI355X (gfx950) multi-level adaptive velocity-space DUGKS.

Thin Python binding of libmlvs.so (include/mlvs.h): argument marshalling only.
Every step of the scheme runs in the library's HIP kernels; PyTorch provides
device memory (through the library's allocator hooks) and the stream.  There
is no CPU fallback: if the library is not built, or no GPU is present, calls
raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlvs.so")

MLVS_BC_WALL, MLVS_BC_FARFIELD, MLVS_BC_OUTFLOW = 1, 2, 3

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int32_p = ctypes.POINTER(ctypes.c_int32)
_c_uint8_p = ctypes.POINTER(ctypes.c_uint8)


class mlvs_bc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rho", ctypes.c_double), ("u", ctypes.c_double),
                ("v", ctypes.c_double), ("T", ctypes.c_double)]


class mlvs_physics(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("K", ctypes.c_int), ("R", ctypes.c_double), ("Pr", ctypes.c_double),
                ("omega", ctypes.c_double), ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double),
                ("dt", ctypes.c_double), ("cfl", ctypes.c_double), ("precision", ctypes.c_int),
                ("compat", ctypes.c_int), ("face_compat", ctypes.c_int), ("map_moments", ctypes.c_int),
                ("positivity", ctypes.c_int)]


class mlvs_mesh(ctypes.Structure):
    _fields_ = [("ni", ctypes.c_int), ("nj", ctypes.c_int), ("node_x", _c_double_p), ("node_y", _c_double_p),
                ("periodic_i", ctypes.c_int), ("periodic_j", ctypes.c_int), ("bc_imin", _c_int32_p),
                ("bc_imax", _c_int32_p), ("bc_jmin", _c_int32_p), ("bc_jmax", _c_int32_p),
                ("n_bc", ctypes.c_int), ("bcs", ctypes.POINTER(mlvs_bc))]


class mlvs_umesh(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int), ("n_cells", ctypes.c_int), ("node_x", _c_double_p),
                ("node_y", _c_double_p), ("cell_ptr", _c_int32_p), ("cell_node", _c_int32_p),
                ("n_bedges", ctypes.c_int), ("bedge", _c_int32_p), ("n_bc", ctypes.c_int),
                ("bcs", ctypes.POINTER(mlvs_bc))]


class mlvs_vgrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("x", _c_double_p), ("wx", _c_double_p),
                ("y", _c_double_p), ("wy", _c_double_p)]


class mlvs_adapt_params(ctypes.Structure):
    _fields_ = [("C_split", ctypes.c_double), ("C_merge", ctypes.c_double), ("eps_merge", ctypes.c_double),
                ("tau_clust", ctypes.c_double), ("flux_test", ctypes.c_int), ("interval", ctypes.c_int)]


_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class mlvs_device(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("alloc", _ALLOC), ("free", _FREE), ("user", ctypes.c_void_p)]


class mlvs_adapt_report(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("n_unique", ctypes.c_int64), ("n_changed", ctypes.c_int64),
                ("n_cross", ctypes.c_int64), ("nbar", ctypes.c_double), ("neg_count", ctypes.c_int64),
                ("n_fallback", ctypes.c_int64), ("ms_criterion", ctypes.c_double), ("ms_dedupe", ctypes.c_double),
                ("ms_cluster", ctypes.c_double), ("ms_install", ctypes.c_double)]


class mlvs_train_cfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("val_frac", ctypes.c_double), ("seed", ctypes.c_uint64)]


class mlvs_train_report(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double), ("train_acc", ctypes.c_double),
                ("val_acc", ctypes.c_double), ("n_train", ctypes.c_int64), ("n_val", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("ms", ctypes.c_double)]


_c_float_p = ctypes.POINTER(ctypes.c_float)


# name -> (restype, argtypes)
_PROTOS = {
    "mlvs_vgrid_newton_cotes": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, _c_double_p, _c_double_p]),
    "mlvs_vgrid_gauss_hermite": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, _c_double_p,
                                                _c_double_p]),
    "mlvs_mu_ref_from_kn": (ctypes.c_int, [ctypes.c_double] * 6 + [_c_double_p]),
    "mlvs_create": (ctypes.c_int, [ctypes.POINTER(mlvs_physics), ctypes.POINTER(mlvs_mesh),
                                   ctypes.POINTER(mlvs_vgrid), ctypes.POINTER(mlvs_adapt_params),
                                   ctypes.POINTER(mlvs_device), ctypes.POINTER(ctypes.c_void_p)]),
    "mlvs_create_unstructured": (ctypes.c_int, [ctypes.POINTER(mlvs_physics), ctypes.POINTER(mlvs_umesh),
                                                ctypes.POINTER(mlvs_vgrid), ctypes.POINTER(mlvs_adapt_params),
                                                ctypes.POINTER(mlvs_device), ctypes.POINTER(ctypes.c_void_p)]),
    "mlvs_init_equilibrium": (ctypes.c_int, [ctypes.c_void_p, _c_double_p]),
    "mlvs_set_levels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_uint8_p, _c_int32_p]),
    "mlvs_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "mlvs_adapt": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(mlvs_adapt_report)]),
    "mlvs_criterion": (ctypes.c_int, [ctypes.c_void_p, _c_uint8_p]),
    "mlvs_moments": (ctypes.c_int, [ctypes.c_void_p, _c_double_p]),
    "mlvs_totals": (ctypes.c_int, [ctypes.c_void_p, _c_double_p]),
    "mlvs_level_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), _c_int32_p, _c_int32_p,
                                       ctypes.POINTER(ctypes.c_int64)]),
    "mlvs_level_kappa": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_uint8_p]),
    "mlvs_cell_levels": (ctypes.c_int, [ctypes.c_void_p, _c_int32_p]),
    "mlvs_get_f": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _c_double_p, _c_double_p, _c_int32_p]),
    "mlvs_set_f": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _c_double_p, _c_double_p]),
    "mlvs_get_state": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, _c_double_p]),
    "mlvs_set_state": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, _c_double_p]),
    "mlvs_info": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, ctypes.POINTER(ctypes.c_int64), _c_int32_p,
                                 _c_int32_p]),
    "mlvs_memory": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "mlvs_counters": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), _c_double_p, _c_double_p,
                                     ctypes.POINTER(ctypes.c_int64)]),
    "mlvs_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "mlvs_set_persistent": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "mlvs_set_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "mlvs_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "mlvs_graph_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int)]),
    "mlvs_variants": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "mlvs_set_variant": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "mlvs_time_stage": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_double_p]),
    "mlvs_stage_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                       _c_double_p]),
    "mlvs_step_stages": (ctypes.c_int, [ctypes.c_void_p, _c_int32_p, ctypes.POINTER(ctypes.c_int)]),
    "mlvs_stress": (ctypes.c_int, [ctypes.c_void_p, _c_double_p]),
    "mlvs_neg_count": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "mlvs_positivity_counts": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_int64)]),
    "mlvs_mlp_nparams": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    "mlvs_features": (ctypes.c_int, [ctypes.c_void_p, _c_float_p]),
    "mlvs_labels": (ctypes.c_int, [ctypes.c_void_p, _c_int32_p]),
    "mlvs_mlp_train": (ctypes.c_int, [_c_float_p, ctypes.c_int, _c_float_p, _c_int32_p, ctypes.c_int64,
                                      ctypes.POINTER(mlvs_train_cfg), ctypes.POINTER(mlvs_train_report)]),
    "mlvs_mlp_eval": (ctypes.c_int, [_c_float_p, ctypes.c_int, _c_float_p, _c_int32_p, ctypes.c_int, _c_float_p,
                                     _c_float_p, _c_double_p]),
    "mlvs_mlp_eval_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "mlvs_mlp_predict": (ctypes.c_int, [_c_float_p, ctypes.c_int, _c_float_p, ctypes.c_int, ctypes.c_int,
                                        _c_int32_p, _c_float_p]),
    "mlvs_selector_set": (ctypes.c_int, [ctypes.c_void_p, _c_float_p, ctypes.c_int]),
    "mlvs_selector_snapshot": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    "mlvs_selector_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(mlvs_train_cfg),
                                           ctypes.POINTER(mlvs_train_report)]),
    "mlvs_selector_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "mlvs_selector_params": (ctypes.c_int, [ctypes.c_void_p, _c_float_p, ctypes.POINTER(ctypes.c_int)]),
    "mlvs_selector_check": (ctypes.c_int, [ctypes.c_void_p, _c_int32_p, _c_int32_p]),
    "mlvs_set_strict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "mlvs_set_adapt": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(mlvs_adapt_params)]),
    "mlvs_destroy": (None, [ctypes.c_void_p]),
    "mlvs_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libmlvs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmlvs.so is not built (run paper_2609_35258_amd.build.build())")
        # Load torch first so that the library binds to the same HIP runtime
        # (libamdhip64.so.7) as torch: streams and memory are torch's.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MLVSError(RuntimeError):
    pass


def _check(status):
    if status != 0:
        msg = lib().mlvs_last_error().decode(errors="replace")
        raise MLVSError("mlvs error %d: %s" % (status, msg))


def _dp(a):
    return a.ctypes.data_as(_c_double_p)


def newton_cotes(n: int, a: float):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().mlvs_vgrid_newton_cotes(n, a, _dp(x), _dp(w)))
    return x, w


def gauss_hermite(n: int, R: float, T0: float):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().mlvs_vgrid_gauss_hermite(n, R, T0, _dp(x), _dp(w)))
    return x, w


def mu_ref_from_kn(Kn, rho, T, R, L, omega):
    out = ctypes.c_double()
    _check(lib().mlvs_mu_ref_from_kn(Kn, rho, T, R, L, omega, ctypes.byref(out)))
    return out.value


def _fp(a):
    return a.ctypes.data_as(_c_float_p)


def mlp_nparams(K: int) -> int:
    n = ctypes.c_int64()
    _check(lib().mlvs_mlp_nparams(K, ctypes.byref(n)))
    return n.value


def mlp_eval(params, K, X, y):
    """One device forward/backward pass: (probs [B][K], grad [n_params], mean loss)."""
    P = np.ascontiguousarray(params, np.float32)
    Xf = np.ascontiguousarray(X, np.float32)
    yy = np.ascontiguousarray(y, np.int32)
    B = len(yy)
    probs = np.zeros((B, K), np.float32)
    grad = np.zeros(len(P), np.float32)
    loss = ctypes.c_double()
    _check(lib().mlvs_mlp_eval(_fp(P), K, _fp(Xf), yy.ctypes.data_as(_c_int32_p), B, _fp(probs), _fp(grad),
                               ctypes.byref(loss)))
    return probs, grad, loss.value


def mlp_eval_noalloc(d_params, K, d_X, d_y, B, d_probs=None, d_grad=None, d_loss_sum=None, stream=None):
    """mlvs_mlp_eval_noalloc on device pointers (ints, e.g. torch tensors' data_ptr()); asynchronous."""
    _check(lib().mlvs_mlp_eval_noalloc(d_params, int(K), d_X, d_y, int(B), d_probs, d_grad, d_loss_sum, stream))


def mlp_predict(params, K, X, bf16=True):
    P = np.ascontiguousarray(params, np.float32)
    Xf = np.ascontiguousarray(X, np.float32)
    B = len(Xf)
    cls = np.zeros(B, np.int32)
    probs = np.zeros((B, K), np.float32)
    _check(lib().mlvs_mlp_predict(_fp(P), K, _fp(Xf), B, int(bf16), cls.ctypes.data_as(_c_int32_p), _fp(probs)))
    return cls, probs


def mlp_train(params, K, X, y, epochs=10, batch=4096, lr=1e-3, val_frac=0.2, seed=0):
    """Train on the device; returns (trained params, report dict)."""
    P = np.array(params, np.float32)
    Xf = np.ascontiguousarray(X, np.float32)
    yy = np.ascontiguousarray(y, np.int32)
    cfg = mlvs_train_cfg(int(epochs), int(batch), float(lr), 0.9, 0.999, 1e-8, float(val_frac), int(seed))
    rep = mlvs_train_report()
    _check(lib().mlvs_mlp_train(_fp(P), K, _fp(Xf), yy.ctypes.data_as(_c_int32_p), len(yy), ctypes.byref(cfg),
                                ctypes.byref(rep)))
    return P, {k: getattr(rep, k) for k, _ in mlvs_train_report._fields_}


class Solver:
    """One MLVS-DUGKS context on the current torch CUDA (HIP) device and stream."""

    def __init__(self, *, dim: int, bcs: Sequence, vx, vwx, vy, vwy, R: float, Pr: float, K: int,
                 omega: float, mu_ref: float, T_ref: float, cfl: float, node_x=None, node_y=None,
                 periodic_i: bool = False, periodic_j: bool = False, bc_imin=None, bc_imax=None, bc_jmin=None,
                 bc_jmax=None, umesh: Optional[dict] = None, dt: float = 0.0,
                 precision: int = 64, compat: int = 4, face_compat: bool = True, map_moments: int = 4,
                 adapt: Optional[dict] = None, device=None, graph: bool = False, positivity: str = "keep"):
        """Structured mesh: node_x, node_y ((nj+1, ni+1)), periodic flags and the
        bc_* id arrays.  Unstructured mesh: umesh = dict(nodes (n, 2), cell_ptr,
        cell_node, bedges (m, 3)) as in mlvs_umesh."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the MLVS library runs on the device only")
        L = lib()
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._keep = {}
        self.stream = torch.cuda.current_stream(self.device)
        if graph and self.stream.cuda_stream == 0:
            # graph capture needs a stream of its own (default priority)
            self.stream = torch.cuda.Stream(self.device)

        def _alloc(n, user):
            with torch.cuda.stream(self.stream):
                t = torch.empty(int(n), dtype=torch.uint8, device=self.device)
            p = t.data_ptr()
            self._keep[p] = t
            return p

        def _free(p, user):
            self._keep.pop(p, None)

        self._alloc_cb = _ALLOC(_alloc)
        self._free_cb = _FREE(_free)
        dev = mlvs_device(ctypes.c_void_p(self.stream.cuda_stream), self._alloc_cb, self._free_cb, None)
        self._arrays = []

        def keep(a, dt_=np.float64):
            a = np.ascontiguousarray(a, dtype=dt_)
            self._arrays.append(a)
            return a

        bc_arr = (mlvs_bc * max(len(bcs), 1))()
        for k, b in enumerate(bcs):
            bc_arr[k] = mlvs_bc(int(b.kind), float(b.rho), float(b.u), float(b.v), float(b.T))
        self._bc_arr = bc_arr
        i32 = lambda a: keep(a, np.int32).ctypes.data_as(_c_int32_p)
        if umesh is None:
            node_x = np.ascontiguousarray(node_x, dtype=np.float64)
            node_y = np.ascontiguousarray(node_y, dtype=np.float64)
            nj, ni = node_x.shape[0] - 1, node_x.shape[1] - 1
            mesh = mlvs_mesh(ni, nj, _dp(keep(node_x)), _dp(keep(node_y)), int(periodic_i), int(periodic_j),
                             i32(bc_imin), i32(bc_imax), i32(bc_jmin), i32(bc_jmax), len(bcs), bc_arr)
            n_cells = ni * nj
        else:
            nodes = np.asarray(umesh["nodes"], np.float64)
            ptr = np.asarray(umesh["cell_ptr"], np.int32)
            be = np.asarray(umesh["bedges"], np.int32).reshape(-1, 3)
            n_cells = len(ptr) - 1
            mesh = mlvs_umesh(len(nodes), n_cells, _dp(keep(nodes[:, 0])), _dp(keep(nodes[:, 1])), i32(ptr),
                              i32(umesh["cell_node"]), len(be), i32(be), len(bcs), bc_arr)
        vg = mlvs_vgrid(len(vx), len(vy), _dp(keep(vx)), _dp(keep(vwx)), _dp(keep(vy)), _dp(keep(vwy)))
        if positivity not in ("keep", "exp"):
            raise ValueError("positivity must be 'keep' or 'exp'")
        phys = mlvs_physics(dim, K, R, Pr, omega, mu_ref, T_ref, dt, cfl, precision, compat, int(face_compat),
                            map_moments, 1 if positivity == "exp" else 0)
        ap = None
        if adapt is not None:
            ap = mlvs_adapt_params(adapt["C_split"], adapt["C_merge"], adapt.get("eps_merge", 0.0),
                                   adapt["tau_clust"], int(adapt.get("flux_test", False)),
                                   int(adapt.get("interval", 0)))
        h = ctypes.c_void_p()
        create = L.mlvs_create if umesh is None else L.mlvs_create_unstructured
        _check(create(ctypes.byref(phys), ctypes.byref(mesh), ctypes.byref(vg),
                      ctypes.byref(ap) if ap is not None else None, ctypes.byref(dev), ctypes.byref(h)))
        self.h = h
        if graph:
            _check(L.mlvs_set_graph(self.h, 1))
        self.n_cells = n_cells
        self.dim = dim
        self.structured = umesh is None and dim == 2       # traversal tiles apply
        dt_ = ctypes.c_double()
        nc = ctypes.c_int64()
        nb = ctypes.c_int32()
        nbase = ctypes.c_int32()
        _check(L.mlvs_info(self.h, ctypes.byref(dt_), ctypes.byref(nc), ctypes.byref(nb), ctypes.byref(nbase)))
        self.dt = dt_.value
        self.n_blocks = nb.value
        self.n_base = nbase.value

    @classmethod
    def from_problem(cls, p, precision: int = 64, compat: int = 4, face_compat: bool = True,
                     map_moments: int = 4, adapt: Optional[dict] = None, dt: float = 0.0, graph: bool = False,
                     positivity: str = "keep"):
        """Build from a problem description (attributes as in the workload generators)."""
        if p.vel_kind == "gh":
            x, w = gauss_hermite(p.nv, p.R, p.gh_scale_T)
        else:
            x, w = newton_cotes(p.nv, p.vmax)
        if p.dim == 1:
            y, wy = np.zeros(1), np.ones(1)
        else:
            y, wy = x, w
        mu = mu_ref_from_kn(p.Kn, p.rho_ref, p.T_ref, p.R, p.L_ref, p.omega)
        if getattr(p, "unstructured", False):
            s = cls(dim=2, umesh=dict(nodes=p.nodes, cell_ptr=p.cell_ptr, cell_node=p.cell_node, bedges=p.bedges),
                    bcs=p.bcs, vx=x, vwx=w, vy=y, vwy=wy, R=p.R, Pr=p.Pr, K=p.K, omega=p.omega, mu_ref=mu,
                    T_ref=p.T_ref, cfl=p.cfl, dt=dt, precision=precision, compat=compat, face_compat=face_compat,
                    map_moments=map_moments, adapt=adapt, graph=graph, positivity=positivity)
            s.init_equilibrium(np.stack([p.rho0, p.u0, p.v0, p.T0], axis=1))
            return s
        s = cls(dim=p.dim, node_x=p.X, node_y=p.Y, periodic_i=p.periodic_i, periodic_j=p.periodic_j,
                bcs=p.bcs, bc_imin=p.bc_imin, bc_imax=p.bc_imax, bc_jmin=p.bc_jmin, bc_jmax=p.bc_jmax,
                vx=x, vwx=w, vy=y, vwy=wy, R=p.R, Pr=p.Pr, K=p.K, omega=p.omega, mu_ref=mu, T_ref=p.T_ref,
                cfl=p.cfl, dt=dt, precision=precision, compat=compat, face_compat=face_compat,
                map_moments=map_moments, adapt=adapt, graph=graph, positivity=positivity)
        s.init_equilibrium(np.stack([p.rho0.ravel(), p.u0.ravel(), p.v0.ravel(), p.T0.ravel()], axis=1))
        return s

    # -- calls -------------------------------------------------------------------
    def init_equilibrium(self, rho_u_v_T):
        a = np.ascontiguousarray(rho_u_v_T, dtype=np.float64)
        _check(lib().mlvs_init_equilibrium(self.h, _dp(a)))

    def step(self, n: int = 1):
        _check(lib().mlvs_step(self.h, int(n)))

    def moments(self):
        out = np.zeros((self.n_cells, 6))
        _check(lib().mlvs_moments(self.h, _dp(out)))
        return out

    def totals(self):
        out = np.zeros(4)
        _check(lib().mlvs_totals(self.h, _dp(out)))
        return out

    def level_info(self):
        n = ctypes.c_int()
        _check(lib().mlvs_level_info(self.h, ctypes.byref(n), None, None, None))
        npts = np.zeros(n.value, np.int32)
        ncell = np.zeros(n.value, np.int32)
        ncross = ctypes.c_int64()
        _check(lib().mlvs_level_info(self.h, ctypes.byref(n), npts.ctypes.data_as(_c_int32_p),
                                     ncell.ctypes.data_as(_c_int32_p), ctypes.byref(ncross)))
        return npts, ncell, ncross.value

    def level_kappa(self, level: int):
        out = np.zeros(self.n_blocks, np.uint8)
        _check(lib().mlvs_level_kappa(self.h, level, out.ctypes.data_as(_c_uint8_p)))
        return out

    def cell_levels(self):
        out = np.zeros(self.n_cells, np.int32)
        _check(lib().mlvs_cell_levels(self.h, out.ctypes.data_as(_c_int32_p)))
        return out

    def npts_per_cell(self):
        npts, _, _ = self.level_info()
        return npts[self.cell_levels()]

    def get_state(self):
        """List of (g, h) per cell, FP64 on the host."""
        n = self.npts_per_cell()
        tot = int(n.sum())
        g = np.zeros(tot)
        h = np.zeros(tot)
        _check(lib().mlvs_get_state(self.h, _dp(g), _dp(h)))
        off = np.concatenate([[0], np.cumsum(n)])
        return [(g[off[c]:off[c + 1]], h[off[c]:off[c + 1]]) for c in range(self.n_cells)]

    def stress(self):
        """Per-cell deviatoric stress (sigma_xx, sigma_xy, sigma_yy), shape (n_cells, 3)."""
        out = np.zeros((self.n_cells, 3))
        _check(lib().mlvs_stress(self.h, _dp(out)))
        return out

    def get_cell(self, cell: int):
        """(g, h) of one cell on its level, FP64 on the host (synchronises)."""
        n = ctypes.c_int32()
        _check(lib().mlvs_get_f(self.h, int(cell), None, None, ctypes.byref(n)))
        g = np.zeros(n.value)
        h = np.zeros(n.value)
        _check(lib().mlvs_get_f(self.h, int(cell), _dp(g), _dp(h), ctypes.byref(n)))
        return g, h

    def set_state(self, gs, hs):
        g = np.ascontiguousarray(np.concatenate(gs), dtype=np.float64)
        h = np.ascontiguousarray(np.concatenate(hs), dtype=np.float64)
        _check(lib().mlvs_set_state(self.h, _dp(g), _dp(h)))

    def set_levels(self, kappas, cell_level):
        k = np.ascontiguousarray(np.asarray(kappas, np.uint8).reshape(-1))
        cl = np.ascontiguousarray(cell_level, np.int32)
        n = len(k) // max(self.n_blocks, 1)
        _check(lib().mlvs_set_levels(self.h, n, k.ctypes.data_as(_c_uint8_p), cl.ctypes.data_as(_c_int32_p)))

    def set_adapt(self, adapt: dict):
        """Replace the adaptation parameters (dict as at creation)."""
        ap = mlvs_adapt_params(adapt["C_split"], adapt["C_merge"], adapt.get("eps_merge", 0.0), adapt["tau_clust"],
                               int(adapt.get("flux_test", False)), int(adapt.get("interval", 0)))
        _check(lib().mlvs_set_adapt(self.h, ctypes.byref(ap)))

    def adapt(self):
        rep = mlvs_adapt_report()
        _check(lib().mlvs_adapt(self.h, ctypes.byref(rep)))
        return {k: getattr(rep, k) for k, _ in mlvs_adapt_report._fields_}

    def criterion(self):
        out = np.zeros((self.n_cells, self.n_blocks), np.uint8)
        _check(lib().mlvs_criterion(self.h, out.ctypes.data_as(_c_uint8_p)))
        return out

    def features(self):
        out = np.zeros((self.n_cells, 10), np.float32)
        _check(lib().mlvs_features(self.h, _fp(out)))
        return out

    def labels(self):
        out = np.zeros(self.n_cells, np.int32)
        _check(lib().mlvs_labels(self.h, out.ctypes.data_as(_c_int32_p)))
        return out

    def selector_set(self, params, K):
        if params is None:
            _check(lib().mlvs_selector_set(self.h, None, 0))
            return
        self._sel = np.ascontiguousarray(params, np.float32)
        _check(lib().mlvs_selector_set(self.h, _fp(self._sel), int(K)))

    def selector_snapshot(self, reset: bool = False) -> int:
        """Record features and criterion labels of every cell; returns the stored sample count."""
        n = ctypes.c_int64()
        _check(lib().mlvs_selector_snapshot(self.h, int(reset), ctypes.byref(n)))
        return n.value

    def selector_train(self, epochs=10, batch=4096, lr=1e-3, val_frac=0.2, seed=0):
        """Train the context's selector on its recorded snapshots; returns the report dict."""
        cfg = mlvs_train_cfg(int(epochs), int(batch), float(lr), 0.9, 0.999, 1e-8, float(val_frac), int(seed))
        rep = mlvs_train_report()
        _check(lib().mlvs_selector_train(self.h, ctypes.byref(cfg), ctypes.byref(rep)))
        return {k: getattr(rep, k) for k, _ in mlvs_train_report._fields_}

    def selector_enable(self, on: bool = True):
        _check(lib().mlvs_selector_enable(self.h, int(on)))

    def selector_check(self, levels):
        """Tail-mass check of a proposed catalogue level per cell: bool array,
        True where no block the level merges has I_B > C_split."""
        lv = np.ascontiguousarray(levels, np.int32)
        if lv.shape != (self.n_cells,):
            raise ValueError("one level per cell")
        acc = np.zeros(self.n_cells, np.int32)
        _check(lib().mlvs_selector_check(self.h, lv.ctypes.data_as(_c_int32_p), acc.ctypes.data_as(_c_int32_p)))
        return acc.astype(bool)

    def selector_params(self):
        """(params as float32, K) of the installed network, or (None, 0)."""
        K = ctypes.c_int()
        _check(lib().mlvs_selector_params(self.h, None, ctypes.byref(K)))
        if K.value == 0:
            return None, 0
        out = np.zeros(mlp_nparams(K.value), np.float32)
        _check(lib().mlvs_selector_params(self.h, _fp(out), ctypes.byref(K)))
        return out, K.value

    def set_strict(self, flags: int):
        """Strict mode bits: 1 state checks after every step, 2 positivity violations are errors."""
        _check(lib().mlvs_set_strict(self.h, int(flags)))

    def memory(self):
        v = ctypes.c_size_t()
        _check(lib().mlvs_memory(self.h, ctypes.byref(v)))
        return v.value

    def counters(self):
        st, ad = ctypes.c_int64(), ctypes.c_int64()
        up, ip = ctypes.c_double(), ctypes.c_double()
        _check(lib().mlvs_counters(self.h, ctypes.byref(st), ctypes.byref(up), ctypes.byref(ip), ctypes.byref(ad)))
        return {"steps": st.value, "cell_updates": up.value, "iface_points": ip.value, "adaptations": ad.value}

    STAGES = {"cell": 0, "ghost": 1, "face_rec": 2, "face_target": 3, "xface": 4, "update": 5, "criterion": 6,
              "face": 7, "update_cell": 8, "persistent": 9}
    STAGE_NAMES = {v: k for k, v in STAGES.items()}

    def set_persistent(self, on: bool = True):
        _check(lib().mlvs_set_persistent(self.h, int(on)))

    def set_tiling(self, tw: int, th: int):
        """Traversal tiles (tw x th cells; 0, 0 row-major) of a structured mesh;
        reorders the state rows on the device, values unchanged."""
        _check(lib().mlvs_set_tiling(self.h, int(tw), int(th)))

    def tiling(self):
        tw, th = ctypes.c_int(), ctypes.c_int()
        _check(lib().mlvs_tiling(self.h, ctypes.byref(tw), ctypes.byref(th)))
        return tw.value, th.value

    def graph_info(self):
        """{persistent, captures, launches, grid, error} of the step launches."""
        pe, gr, er = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        ca, la = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().mlvs_graph_info(self.h, ctypes.byref(pe), ctypes.byref(ca), ctypes.byref(la), ctypes.byref(gr),
                                     ctypes.byref(er)))
        return {"persistent": pe.value, "captures": ca.value, "launches": la.value, "grid": gr.value,
                "error": er.value}

    def step_stages(self):
        """Names of the stages one step launches, in order."""
        n = ctypes.c_int()
        buf = (ctypes.c_int32 * 10)()
        _check(lib().mlvs_step_stages(self.h, buf, ctypes.byref(n)))
        return [self.STAGE_NAMES[buf[k]] for k in range(n.value)]

    def time_stage(self, stage, reps: int = 10):
        """Mean ms per launch of one stage, timed with HIP events on the context stream."""
        ms = ctypes.c_double()
        _check(lib().mlvs_time_stage(self.h, self.STAGES.get(stage, stage), int(reps), ctypes.byref(ms)))
        return ms.value

    def variants(self, stage):
        n = ctypes.c_int()
        _check(lib().mlvs_variants(self.STAGES.get(stage, stage), ctypes.byref(n)))
        return n.value

    def set_variant(self, stage, v: int):
        _check(lib().mlvs_set_variant(self.h, self.STAGES.get(stage, stage), int(v)))

    def stage_size(self, stage):
        it = ctypes.c_int64()
        pts = ctypes.c_double()
        _check(lib().mlvs_stage_size(self.h, self.STAGES.get(stage, stage), ctypes.byref(it), ctypes.byref(pts)))
        return it.value, pts.value

    def neg_count(self):
        v = ctypes.c_int64()
        _check(lib().mlvs_neg_count(self.h, ctypes.byref(v)))
        return v.value

    def positivity_counts(self):
        """(maps that took the exponential correction, maps whose Newton iteration failed)."""
        a, f = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().mlvs_positivity_counts(self.h, ctypes.byref(a), ctypes.byref(f)))
        return a.value, f.value

    def close(self):
        if getattr(self, "h", None):
            lib().mlvs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
