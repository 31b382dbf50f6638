"""ctypes wrapper of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The oracle is a plain sequential restatement of the paper's
method (arXiv 1810.04289) and shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = ["topology.cpp", "physics.cpp", "schwarz.cpp", "krylov.cpp", "api.cpp"]

ERRORS = {0: "OK", 1: "ARG", 2: "MESH", 3: "OOM", 4: "HIP", 5: "INVERTED", 6: "ZERO_PIVOT", 7: "DIVERGED"}


def build(force: bool = False) -> str:
    """Compile the oracle with g++ -O2 -ffp-contract=off (plain IEEE FP64; the only fused
    operations are the explicit std::fma of the ILU block products)."""
    srcs = [os.path.join(_HERE, s) for s in _SRC]
    if not force and os.path.exists(_LIB):
        mt = os.path.getmtime(_LIB)
        if all(os.path.getmtime(s) <= mt for s in srcs + [os.path.join(_HERE, "core.hpp"),
                                                           os.path.join(_HERE, "fsio.h")]):
            return _LIB
    cmd = ["g++", "-O2", "-ffp-contract=off", "-std=c++17", "-fPIC", "-shared", "-o", _LIB + ".tmp"] + srcs
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Mesh_(C.Structure):
    _fields_ = [("nverts", C.c_int32), ("ntets", C.c_int32), ("nbfaces", C.c_int32),
                ("X", C.c_void_p), ("tets", C.c_void_p), ("tet_domain", C.c_void_p),
                ("bfaces", C.c_void_p), ("bface_tag", C.c_void_p)]


class Phys_(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("rho_f", "mu_f", "rho_s", "E_s", "nu_s", "eta_s", "C_I")]


class Opts_(C.Structure):
    _fields_ = [("nsub", C.c_int32), ("overlap", C.c_int32), ("ilu_level", C.c_int32),
                ("ordering", C.c_int32), ("part", C.c_void_p), ("gmres_restart", C.c_int32),
                ("gmres_maxit", C.c_int32), ("gmres_rtol", C.c_double), ("newton_rtol", C.c_double),
                ("newton_atol", C.c_double), ("newton_maxit", C.c_int32), ("jac_lag", C.c_int32),
                ("ls_c", C.c_double), ("ls_max_halvings", C.c_int32), ("precision", C.c_int32)]


class LinStats_(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("pad", C.c_int32), ("rnorm0", C.c_double), ("rnorm_est", C.c_double),
                ("rnorm_true", C.c_double)]


class StepStats_(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("linear_iters", C.c_int32),
                ("line_search_cuts", C.c_int32), ("converged", C.c_int32),
                ("fnorm0", C.c_double), ("fnorm", C.c_double),
                ("t_funceval", C.c_double), ("t_jaceval", C.c_double), ("t_pcsetup", C.c_double),
                ("t_pcapply", C.c_double), ("t_kspsolve", C.c_double), ("t_kspsetup", C.c_double),
                ("fnorm_hist", C.c_double * 64), ("alpha_hist", C.c_double * 64),
                ("lin_hist", C.c_int32 * 64)]


def stats_dict(st) -> dict:
    out = {}
    for name, _ in st._fields_:
        v = getattr(st, name)
        if hasattr(v, "__len__"):
            v = list(v)
        out[name] = v
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "fsio_create": [vp, vp, vp, vp], "fsio_destroy": [vp], "fsio_sizes": [vp, vp, vp],
            "fsio_set_step": [vp, dbl, dbl, vp, vp, vp, vp], "fsio_impose_dirichlet": [vp, vp],
            "fsio_residual": [vp, vp, vp], "fsio_residual_complex": [vp, vp, vp, vp, vp],
            "fsio_jacobian": [vp, vp], "fsio_jacobian_get": [vp, vp, vp, vp], "fsio_jacobian_set": [vp, vp],
            "fsio_spmv": [vp, vp, vp], "fsio_pc_setup": [vp], "fsio_pc_apply": [vp, vp, vp],
            "fsio_gmres": [vp, vp, vp, vp], "fsio_newton_solve": [vp, vp, vp],
            "fsio_topology_get": [vp, vp, vp, vp, vp], "fsio_pc_sizes": [vp, vp, vp, vp, vp],
            "fsio_pc_get": [vp] + [vp] * 9, "fsio_element": [vp, vp, i32, vp, vp],
            "fsio_element_ops": [vp, vp, i32, vp, vp],
        }
        for k, a in sig.items():
            f = getattr(L, k)
            f.argtypes = a
            f.restype = C.c_int
        L.fsio_last_error.argtypes = [vp]
        L.fsio_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle {ERRORS.get(code, code)}: {msg}")
        self.code = code


def default_opts(**kw) -> dict:
    o = dict(nsub=4, overlap=1, ilu_level=0, ordering=0, part=None, gmres_restart=30,
             gmres_maxit=1000, gmres_rtol=1e-3, newton_rtol=1e-6, newton_atol=0.0,
             newton_maxit=50, jac_lag=1, ls_c=1e-4, ls_max_halvings=10, precision=0)
    o.update(kw)
    return o


class Oracle:
    """One oracle solver instance on a mesh (host arrays, float64)."""

    def __init__(self, mesh, phys: dict, opts: dict | None = None):
        L = lib()
        self.mesh = mesh
        self._keep = [np.ascontiguousarray(mesh.X, dtype=np.float64),
                      np.ascontiguousarray(mesh.tets, dtype=np.int32),
                      np.ascontiguousarray(mesh.tet_domain, dtype=np.int8),
                      np.ascontiguousarray(mesh.bfaces, dtype=np.int32),
                      np.ascontiguousarray(mesh.bface_tag, dtype=np.int8)]
        m = Mesh_(mesh.nverts, mesh.ntets, len(mesh.bfaces), *[k.ctypes.data for k in self._keep])
        ph = Phys_(**phys)
        o = default_opts(**(opts or {}))
        part = o.pop("part")
        if part is not None:
            part = np.ascontiguousarray(part, dtype=np.int32)
            self._keep.append(part)
        oo = Opts_(**{k: v for k, v in o.items()}, part=_p(part))
        h = C.c_void_p()
        rc = L.fsio_create(C.byref(m), C.byref(ph), C.byref(oo), C.byref(h))
        if rc:
            raise OracleError(rc, "create")
        self.h = h
        self.V = mesh.nverts
        self.n = 7 * mesh.nverts
        nn, nb = C.c_int64(), C.c_int64()
        L.fsio_sizes(h, C.byref(nn), C.byref(nb))
        self.nnzb = nb.value

    def __del__(self):
        if getattr(self, "h", None):
            lib().fsio_destroy(self.h)
            self.h = None

    def _chk(self, rc, what):
        if rc:
            raise OracleError(rc, f"{what}: {lib().fsio_last_error(self.h).decode()}")

    def set_step(self, t, dt, y_old, g, body_force=None, extra_mask=None):
        self._yold = np.ascontiguousarray(y_old, dtype=np.float64)
        self._g = np.ascontiguousarray(g, dtype=np.float64)
        self._bf = None if body_force is None else np.ascontiguousarray(body_force, dtype=np.float64)
        self._em = None if extra_mask is None else np.ascontiguousarray(extra_mask, dtype=np.uint8)
        self._chk(lib().fsio_set_step(self.h, t, dt, _p(self._yold), _p(self._g), _p(self._bf),
                                      _p(self._em)), "set_step")

    def impose_dirichlet(self, y):
        y = np.array(y, dtype=np.float64)
        self._chk(lib().fsio_impose_dirichlet(self.h, _p(y)), "impose")
        return y

    def residual(self, y, check=True):
        y = np.ascontiguousarray(y, dtype=np.float64)
        F = np.zeros(self.n)
        rc = lib().fsio_residual(self.h, _p(y), _p(F))
        if check:
            self._chk(rc, "residual")
            return F
        return rc, F

    def residual_complex(self, y_re, y_im):
        yr = np.ascontiguousarray(y_re, dtype=np.float64)
        yi = np.ascontiguousarray(y_im, dtype=np.float64)
        Fr, Fi = np.zeros(self.n), np.zeros(self.n)
        self._chk(lib().fsio_residual_complex(self.h, _p(yr), _p(yi), _p(Fr), _p(Fi)), "residual_complex")
        return Fr, Fi

    def jacobian(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        self._chk(lib().fsio_jacobian(self.h, _p(y)), "jacobian")

    def jacobian_get(self):
        rp = np.zeros(self.V + 1, dtype=np.int32)
        ci = np.zeros(self.nnzb, dtype=np.int32)
        vals = np.zeros((self.nnzb, 7, 7))
        self._chk(lib().fsio_jacobian_get(self.h, _p(rp), _p(ci), _p(vals)), "jacobian_get")
        return rp, ci, vals

    def jacobian_set(self, vals):
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        assert vals.size == self.nnzb * 49
        self._chk(lib().fsio_jacobian_set(self.h, _p(vals)), "jacobian_set")

    def spmv(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.n)
        self._chk(lib().fsio_spmv(self.h, _p(x), _p(y)), "spmv")
        return y

    def pc_setup(self):
        self._chk(lib().fsio_pc_setup(self.h), "pc_setup")

    def pc_apply(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        z = np.zeros(self.n)
        self._chk(lib().fsio_pc_apply(self.h, _p(v), _p(z)), "pc_apply")
        return z

    def gmres(self, rhs, restart=None, maxit=None, rtol=None):
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        x = np.zeros(self.n)
        st = LinStats_()
        self._chk(lib().fsio_gmres(self.h, _p(rhs), _p(x), C.byref(st)), "gmres")
        return x, stats_dict(st)

    def newton_solve(self, y, check=True):
        y = np.array(y, dtype=np.float64)
        st = StepStats_()
        rc = lib().fsio_newton_solve(self.h, _p(y), C.byref(st))
        if check:
            self._chk(rc, "newton")
        return y, stats_dict(st), rc

    def topology(self):
        vk = np.zeros(self.V, dtype=np.int8)
        rk = np.zeros(self.n, dtype=np.uint8)
        nf = C.c_int32()
        lib().fsio_topology_get(self.h, _p(vk), _p(rk), C.byref(nf), None)
        faces = np.zeros((nf.value, 3), dtype=np.int32)
        lib().fsio_topology_get(self.h, None, None, C.byref(nf), _p(faces))
        return vk, rk, faces

    def pc_get(self, factors=True):
        ns, nr, nb, nl = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
        lib().fsio_pc_sizes(self.h, C.byref(ns), C.byref(nr), C.byref(nb), C.byref(nl))
        ns, nr, nb = ns.value, nr.value, nb.value
        out = dict(part=np.zeros(self.V, dtype=np.int32), sub_ptr=np.zeros(ns + 1, dtype=np.int32),
                   sub_verts=np.zeros(nr, dtype=np.int32), sub_nowned=np.zeros(ns, dtype=np.int32),
                   blk_ptr=np.zeros(ns + 1, dtype=np.int64), lrowptr=np.zeros(nr + ns, dtype=np.int32),
                   lcolind=np.zeros(nb, dtype=np.int32),
                   factors=np.zeros((nb, 7, 7)) if factors else None,
                   udiag=np.zeros((nr, 7, 7)) if factors else None)
        lib().fsio_pc_get(self.h, *[_p(out[k]) for k in ("part", "sub_ptr", "sub_verts", "sub_nowned",
                                                           "blk_ptr", "lrowptr", "lcolind", "factors",
                                                           "udiag")])
        out["nlevels_total"] = nl.value
        return out

    def element_ops(self, y, e):
        """(value operations, tangent operations per forward-mode direction) of element e."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        v, t = C.c_int64(), C.c_int64()
        self._chk(lib().fsio_element_ops(self.h, _p(y), int(e), C.byref(v), C.byref(t)), "element_ops")
        return v.value, t.value

    def element(self, y, e):
        y = np.ascontiguousarray(y, dtype=np.float64)
        Re = np.zeros(28)
        Je = np.zeros((28, 28))
        self._chk(lib().fsio_element(self.h, _p(y), int(e), _p(Re), _p(Je)), "element")
        return Re, Je


def jac_dense(rp, ci, vals, V):
    """Expand a block-sparse matrix into a dense array (small cases only)."""
    A = np.zeros((7 * V, 7 * V))
    for a in range(V):
        for k in range(rp[a], rp[a + 1]):
            b = ci[k]
            A[7 * a:7 * a + 7, 7 * b:7 * b + 7] = vals[k]
    return A


def jac_scipy(rp, ci, vals, V):
    import scipy.sparse as sp
    return sp.bsr_matrix((vals, ci, rp), shape=(7 * V, 7 * V)).tocsr()
