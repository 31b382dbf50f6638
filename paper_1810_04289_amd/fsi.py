"""Thin ctypes binding of the HIP library libfsi.so (include/fsi.h).

Argument marshalling only: every step of the solve runs in the library's HIP kernels.
torch supplies device memory (tensors' data pointers) and the HIP stream.  There is no
fallback: if libfsi.so is missing or cannot be loaded, construction raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsi.so")

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_MESH", 3: "ERR_OOM", 4: "ERR_HIP", 5: "ERR_INVERTED",
          6: "ERR_ZERO_PIVOT", 7: "ERR_DIVERGED"}

# C symbols declared in include/fsi.h, in declaration order
SYMBOLS = ["fsi_create", "fsi_destroy", "fsi_sizes", "fsi_last_error", "fsi_set_step",
           "fsi_impose_dirichlet", "fsi_residual", "fsi_jacobian", "fsi_jacobian_get", "fsi_jacobian_set",
           "fsi_spmv",
           "fsi_pc_setup", "fsi_pc_apply", "fsi_pc_apply_noalloc", "fsi_pc_tune", "fsi_pc_select", "fsi_set_graphs", "fsi_gmres", "fsi_newton_solve", "fsi_topology_get",
           "fsi_pc_sizes", "fsi_pc_get", "fsi_prof_enable", "fsi_prof_get", "fsi_set_newton_tol",
           "fsi_set_wait_limit"]
# include/fsi_guess.h
GUESS_SYMBOLS = ["fsi_mlp_create", "fsi_mlp_destroy", "fsi_mlp_last_error", "fsi_mlp_nparams", "fsi_mlp_set_params",
                 "fsi_mlp_get_params", "fsi_mlp_forward", "fsi_mlp_loss_grad", "fsi_mlp_train_step",
                 "fsi_mlp_set_scales", "fsi_guess_features", "fsi_guess_target", "fsi_guess_predict", "fsi_gemm_f32"]
GUESS_NIN = 18


class FsiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fsi {STATUS.get(code, code)}: {msg}")
        self.code = code


class MeshC(C.Structure):
    _fields_ = [("nverts", C.c_int32), ("ntets", C.c_int32), ("nbfaces", C.c_int32),
                ("X", C.c_void_p), ("tets", C.c_void_p), ("tet_domain", C.c_void_p),
                ("bfaces", C.c_void_p), ("bface_tag", C.c_void_p)]


class PhysicsC(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("rho_f", "mu_f", "rho_s", "E_s", "nu_s", "eta_s", "C_I")]


class OptsC(C.Structure):
    _fields_ = [("nsub", C.c_int32), ("overlap", C.c_int32), ("ilu_level", C.c_int32),
                ("ordering", C.c_int32), ("part", C.c_void_p), ("gmres_restart", C.c_int32),
                ("gmres_maxit", C.c_int32), ("gmres_rtol", C.c_double), ("newton_rtol", C.c_double),
                ("newton_atol", C.c_double), ("newton_maxit", C.c_int32), ("jac_lag", C.c_int32),
                ("ls_c", C.c_double), ("ls_max_halvings", C.c_int32), ("precision", C.c_int32)]


class LinStatsC(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("pad", C.c_int32), ("rnorm0", C.c_double), ("rnorm_est", C.c_double),
                ("rnorm_true", C.c_double)]


class StepStatsC(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("linear_iters", C.c_int32),
                ("line_search_cuts", C.c_int32), ("converged", C.c_int32),
                ("fnorm0", C.c_double), ("fnorm", C.c_double),
                ("t_funceval", C.c_double), ("t_jaceval", C.c_double), ("t_pcsetup", C.c_double),
                ("t_pcapply", C.c_double), ("t_kspsolve", C.c_double), ("t_kspsetup", C.c_double),
                ("fnorm_hist", C.c_double * 64), ("alpha_hist", C.c_double * 64),
                ("lin_hist", C.c_int32 * 64)]


def _todict(st) -> dict:
    out = {}
    for name, _ in st._fields_:
        v = getattr(st, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out


_lib = None


# precision of the Schwarz preconditioner (fsi_opts.precision): FP64; FP32 sweeps from rounded
# FP64 factors; BF16 factors with FP32 sweeps; FP32 factorization and sweeps
PREC_FP64, PREC_FP32, PREC_BF16, PREC_FP32_FACTOR = 0, 1, 2, 3


def load_library(path: str = LIB_PATH):
    """Load libfsi.so and declare its signatures.  Raises if the library is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with `python __graft_entry__.py` "
                                "or `python paper_1810_04289_amd/build.py`")
    L = C.CDLL(path)
    vp, i32, i64, dbl, flt = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float
    sig = {
        "fsi_create": [vp, vp, vp, vp, vp], "fsi_destroy": [vp], "fsi_sizes": [vp, vp, vp],
        "fsi_set_step": [vp, dbl, dbl, vp, vp, vp, vp], "fsi_impose_dirichlet": [vp, vp],
        "fsi_residual": [vp, vp, vp], "fsi_jacobian": [vp, vp], "fsi_jacobian_get": [vp, vp, vp, vp],
        "fsi_jacobian_set": [vp, vp],
        "fsi_spmv": [vp, vp, vp], "fsi_pc_setup": [vp], "fsi_pc_apply": [vp, vp, vp],
        "fsi_pc_apply_noalloc": [vp, vp, vp],
        "fsi_gmres": [vp, vp, vp, vp], "fsi_newton_solve": [vp, vp, vp],
        "fsi_topology_get": [vp, vp, vp, vp, vp], "fsi_pc_sizes": [vp, vp, vp, vp, vp],
        "fsi_pc_get": [vp] * 10, "fsi_prof_enable": [vp, i32], "fsi_prof_get": [vp, C.c_char_p, vp, vp],
        "fsi_set_newton_tol": [vp, dbl, dbl], "fsi_set_wait_limit": [vp, i32], "fsi_pc_tune": [vp, i32, vp, vp], "fsi_pc_select": [vp, i32], "fsi_set_graphs": [vp, i32],
        "fsi_mlp_create": [i32, i32, i32, i32, i64, vp, vp], "fsi_mlp_destroy": [vp],
        "fsi_mlp_set_params": [vp, vp], "fsi_mlp_get_params": [vp, vp, vp], "fsi_mlp_forward": [vp, vp, i64, vp],
        "fsi_mlp_loss_grad": [vp, vp, vp, i64, vp],
        "fsi_mlp_train_step": [vp, vp, vp, i64, flt, flt, flt, flt, vp], "fsi_mlp_set_scales": [vp, vp],
        "fsi_guess_features": [vp, vp, vp, i64, vp, vp], "fsi_guess_target": [vp, vp, vp, vp, i64, vp],
        "fsi_guess_predict": [vp, vp, vp, i64, vp, vp, vp],
        "fsi_gemm_f32": [i32, i32, i32, flt, vp, i64, i64, vp, i64, i64, flt, vp, i64, i32, vp, vp],
    }
    for k, a in sig.items():
        f = getattr(L, k)
        f.argtypes = a
        f.restype = C.c_int
    L.fsi_last_error.argtypes = [vp]
    L.fsi_last_error.restype = C.c_char_p
    L.fsi_mlp_last_error.argtypes = [vp]
    L.fsi_mlp_last_error.restype = C.c_char_p
    L.fsi_mlp_nparams.argtypes = [vp]
    L.fsi_mlp_nparams.restype = C.c_int64
    _lib = L
    return L


def default_opts(**kw) -> dict:
    o = dict(nsub=4, overlap=1, ilu_level=0, ordering=0, part=None, gmres_restart=30,
             gmres_maxit=1000, gmres_rtol=1e-3, newton_rtol=1e-6, newton_atol=0.0,
             newton_maxit=50, jac_lag=1, ls_c=1e-4, ls_max_halvings=10, precision=0)
    o.update(kw)
    return o


def _dptr(t):
    """Device pointer of a contiguous float64/uint8 torch tensor on a GPU."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


class Solver:
    """One solver instance (a mesh, physics, options) bound to a torch stream."""

    def __init__(self, mesh, phys: dict, opts: dict | None = None, stream=None):
        import torch
        L = load_library()
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        keep = [np.ascontiguousarray(mesh.X, dtype=np.float64),
                np.ascontiguousarray(mesh.tets, dtype=np.int32),
                np.ascontiguousarray(mesh.tet_domain, dtype=np.int8),
                np.ascontiguousarray(mesh.bfaces, dtype=np.int32),
                np.ascontiguousarray(mesh.bface_tag, dtype=np.int8)]
        m = MeshC(mesh.nverts, mesh.ntets, len(mesh.bfaces), *[k.ctypes.data for k in keep])
        ph = PhysicsC(**phys)
        o = default_opts(**(opts or {}))
        part = o.pop("part")
        if part is not None:
            part = np.ascontiguousarray(part, dtype=np.int32)
            keep.append(part)
        oc = OptsC(**o, part=None if part is None else part.ctypes.data)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = L.fsi_create(C.byref(m), C.byref(ph), C.byref(oc), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc:
            raise FsiError(rc, "create")
        self.h = h
        self.V = mesh.nverts
        n, nb = C.c_int64(), C.c_int64()
        L.fsi_sizes(h, C.byref(n), C.byref(nb))
        self.n, self.nnzb = n.value, nb.value

    def close(self):
        if getattr(self, "h", None):
            load_library().fsi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, what):
        if rc:
            raise FsiError(rc, f"{what}: {load_library().fsi_last_error(self.h).decode()}")

    def last_error(self) -> str:
        return load_library().fsi_last_error(self.h).decode()

    def vec(self, a=None):
        t = self.torch
        if a is None:
            return t.zeros(self.n, dtype=t.float64, device=self.device)
        return t.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)

    def set_step(self, t_n, dt, y_old, g, body_force=None, extra_mask=None):
        self._yold, self._g, self._bf = y_old, g, body_force
        em = None if extra_mask is None else np.ascontiguousarray(extra_mask, dtype=np.uint8)
        self._em = em
        self._chk(load_library().fsi_set_step(self.h, float(t_n), float(dt), _dptr(y_old), _dptr(g),
                                               _dptr(body_force), None if em is None else em.ctypes.data),
                  "set_step")

    def impose_dirichlet(self, y):
        self._chk(load_library().fsi_impose_dirichlet(self.h, _dptr(y)), "impose_dirichlet")

    def residual(self, y, F, check=True):
        rc = load_library().fsi_residual(self.h, _dptr(y), _dptr(F))
        if check:
            self._chk(rc, "residual")
        return rc

    def jacobian(self, y):
        self._chk(load_library().fsi_jacobian(self.h, _dptr(y)), "jacobian")

    def jacobian_get(self, values=True):
        rp = np.zeros(self.V + 1, dtype=np.int32)
        ci = np.zeros(self.nnzb, dtype=np.int32)
        vals = np.zeros((self.nnzb, 7, 7)) if values else None
        self._chk(load_library().fsi_jacobian_get(self.h, rp.ctypes.data, ci.ctypes.data,
                                                  None if vals is None else vals.ctypes.data), "jacobian_get")
        return rp, ci, vals

    def jacobian_set(self, vals):
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        assert vals.size == 49 * self.nnzb
        self._chk(load_library().fsi_jacobian_set(self.h, vals.ctypes.data), "jacobian_set")

    def spmv(self, x, y):
        self._chk(load_library().fsi_spmv(self.h, _dptr(x), _dptr(y)), "spmv")

    def pc_setup(self):
        self._chk(load_library().fsi_pc_setup(self.h), "pc_setup")

    def pc_apply(self, v, z):
        self._chk(load_library().fsi_pc_apply(self.h, _dptr(v), _dptr(z)), "pc_apply")

    def pc_apply_noalloc(self, v, z, check=True):
        """fsi_pc_apply_noalloc: the same operator, scratch in the library's static per-GPU array."""
        rc = load_library().fsi_pc_apply_noalloc(self.h, _dptr(v), _dptr(z))
        if check:
            self._chk(rc, "pc_apply_noalloc")
        return rc

    SWEEP_MB = (8, 16, 24, 32)

    def pc_tune(self, reps=3):
        """Times every sweep schedule on the current factors and keeps the fastest."""
        best = C.c_int32()
        us = (C.c_double * 4)()
        self._chk(load_library().fsi_pc_tune(self.h, int(reps), C.byref(best), us), "pc_tune")
        return best.value, dict(zip(self.SWEEP_MB, list(us)))

    def set_graphs(self, on=True):
        self._chk(load_library().fsi_set_graphs(self.h, int(bool(on))), "set_graphs")

    def pc_select(self, mb):
        self._chk(load_library().fsi_pc_select(self.h, int(mb)), "pc_select")

    def gmres(self, rhs, x):
        st = LinStatsC()
        self._chk(load_library().fsi_gmres(self.h, _dptr(rhs), _dptr(x), C.byref(st)), "gmres")
        return _todict(st)

    def set_newton_tol(self, rtol, atol):
        self._chk(load_library().fsi_set_newton_tol(self.h, rtol, atol), "set_newton_tol")

    def set_wait_limit(self, polls=-1):
        """Bound of the factorization's and sweeps' waits in polls (-1: the default)."""
        self._chk(load_library().fsi_set_wait_limit(self.h, int(polls)), "set_wait_limit")

    def newton_solve(self, y, check=True):
        st = StepStatsC()
        rc = load_library().fsi_newton_solve(self.h, _dptr(y), C.byref(st))
        if check:
            self._chk(rc, "newton_solve")
        return _todict(st), rc

    def topology(self):
        vk = np.zeros(self.V, dtype=np.int8)
        rk = np.zeros(self.n, dtype=np.uint8)
        nf = C.c_int32()
        L = load_library()
        L.fsi_topology_get(self.h, vk.ctypes.data, rk.ctypes.data, C.byref(nf), None)
        faces = np.zeros((nf.value, 3), dtype=np.int32)
        L.fsi_topology_get(self.h, None, None, C.byref(nf), faces.ctypes.data)
        return vk, rk, faces

    def pc_get(self, factors=True):
        L = load_library()
        ns, nr, nb, nl = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
        L.fsi_pc_sizes(self.h, C.byref(ns), C.byref(nr), C.byref(nb), C.byref(nl))
        ns, nr, nb = ns.value, nr.value, nb.value
        out = dict(part=np.zeros(self.V, dtype=np.int32), sub_ptr=np.zeros(ns + 1, dtype=np.int32),
                   sub_verts=np.zeros(nr, dtype=np.int32), sub_nowned=np.zeros(ns, dtype=np.int32),
                   blk_ptr=np.zeros(ns + 1, dtype=np.int64), lrowptr=np.zeros(nr + ns, dtype=np.int32),
                   lcolind=np.zeros(nb, dtype=np.int32),
                   factors=np.zeros((nb, 7, 7)) if factors else None,
                   udiag=np.zeros((nr, 7, 7)) if factors else None)
        ptr = lambda a: None if a is None else a.ctypes.data
        self._chk(L.fsi_pc_get(self.h, *[ptr(out[k]) for k in ("part", "sub_ptr", "sub_verts", "sub_nowned",
                                                                  "blk_ptr", "lrowptr", "lcolind", "factors",
                                                                  "udiag")]), "pc_get")
        out["nlevels_total"] = nl.value
        return out

    def prof_enable(self, on=True):
        self._chk(load_library().fsi_prof_enable(self.h, 1 if on else 0), "prof_enable")

    def prof_get(self, kernel: str):
        ms, cnt = C.c_double(), C.c_int64()
        self._chk(load_library().fsi_prof_get(self.h, kernel.encode(), C.byref(ms), C.byref(cnt)), "prof_get")
        return ms.value, cnt.value


def _fptr(t):
    """Device pointer of a contiguous float32/float64 torch tensor on a GPU."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


class MLP:
    """Node-wise perceptron of the learned Newton guess (include/fsi_guess.h)."""

    def __init__(self, nin: int = GUESS_NIN, hidden: int = 128, nlayers: int = 4, nout: int = 7, nmax: int = 1):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        L = load_library()
        h = C.c_void_p()
        rc = L.fsi_mlp_create(nin, hidden, nlayers, nout, nmax, None, C.byref(h))
        if rc:
            raise FsiError(rc, "fsi_mlp_create")
        self.h, self.nin, self.nout, self.nmax = h, nin, nout, nmax
        self.nparams = int(L.fsi_mlp_nparams(h))

    def close(self):
        if getattr(self, "h", None):
            load_library().fsi_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, what):
        if rc:
            raise FsiError(rc, f"{what}: {load_library().fsi_mlp_last_error(self.h).decode()}")

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparams
        self._chk(load_library().fsi_mlp_set_params(self.h, p.ctypes.data), "set_params")

    def get_params(self):
        p = np.zeros(self.nparams, dtype=np.float32)
        g = np.zeros(self.nparams, dtype=np.float32)
        self._chk(load_library().fsi_mlp_get_params(self.h, p.ctypes.data, g.ctypes.data), "get_params")
        return p, g

    def forward(self, X):
        n = X.shape[0]
        Y = self.torch.empty((n, self.nout), dtype=self.torch.float32, device=self.device)
        self._chk(load_library().fsi_mlp_forward(self.h, _fptr(X), n, _fptr(Y)), "forward")
        return Y

    def loss_grad(self, X, T):
        loss = C.c_double()
        self._chk(load_library().fsi_mlp_loss_grad(self.h, _fptr(X), _fptr(T), X.shape[0], C.byref(loss)),
                  "loss_grad")
        return loss.value

    def train_step(self, X, T, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        loss = C.c_double()
        self._chk(load_library().fsi_mlp_train_step(self.h, _fptr(X), _fptr(T), X.shape[0], lr, b1, b2, eps,
                                                    C.byref(loss)), "train_step")
        return loss.value

    def set_scales(self, sc):
        sc = np.ascontiguousarray(sc, dtype=np.float32)
        assert sc.size == 21
        self._chk(load_library().fsi_mlp_set_scales(self.h, sc.ctypes.data), "set_scales")

    def features(self, y1, y2, tfeat):
        V = y1.numel() // 7
        X = self.torch.empty((V, GUESS_NIN), dtype=self.torch.float32, device=self.device)
        tf = np.ascontiguousarray(tfeat, dtype=np.float32)
        self._chk(load_library().fsi_guess_features(self.h, _fptr(y1), _fptr(y2), V, tf.ctypes.data, _fptr(X)),
                  "features")
        return X

    def target(self, y, y1, y2):
        V = y.numel() // 7
        T = self.torch.empty((V, 7), dtype=self.torch.float32, device=self.device)
        self._chk(load_library().fsi_guess_target(self.h, _fptr(y), _fptr(y1), _fptr(y2), V, _fptr(T)), "target")
        return T

    def predict(self, y1, y2, tfeat=None, Xwork=None, out=None):
        """Guess for the next step: extrapolation corrected by the network (tfeat given),
        or the extrapolation alone."""
        V = y1.numel() // 7
        g = out if out is not None else self.torch.empty_like(y1)
        tf = None if tfeat is None else np.ascontiguousarray(tfeat, dtype=np.float32)
        if tf is not None and Xwork is None:
            Xwork = self.torch.empty((V, GUESS_NIN), dtype=self.torch.float32, device=self.device)
        self._chk(load_library().fsi_guess_predict(self.h, _fptr(y1), _fptr(y2), V,
                                                   None if tf is None else tf.ctypes.data,
                                                   _fptr(Xwork) if tf is not None else None, _fptr(g)), "predict")
        return g


def gemm_f32(A, B, C_=None, alpha=1.0, beta=0.0, transA=False, transB=False, nsplit=1):
    """C = alpha op(A) op(B) + beta C on the matrix cores (FP32 torch tensors on the GPU);
    nsplit > 1 splits K, with a workspace allocated here."""
    import torch
    M, K = (A.shape[1], A.shape[0]) if transA else A.shape
    K2, N = (B.shape[1], B.shape[0]) if transB else B.shape
    assert K == K2
    if C_ is None:
        C_ = torch.zeros((M, N), dtype=torch.float32, device=A.device)
    sam, sak = (1, A.shape[1]) if transA else (A.shape[1], 1)
    sbk, sbn = (1, B.shape[1]) if transB else (B.shape[1], 1)
    work = torch.empty(nsplit * M * N, dtype=torch.float32, device=C_.device) if nsplit > 1 else None
    rc = load_library().fsi_gemm_f32(M, N, K, alpha, _fptr(A), sam, sak, _fptr(B), sbk, sbn, beta, _fptr(C_),
                                      C_.shape[1], nsplit, _fptr(work), None)
    if rc:
        raise FsiError(rc, "fsi_gemm_f32")
    return C_
