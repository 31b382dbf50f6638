"""Mixed-precision Schwarz preconditioner (FP32 or BF16 factor storage, FP32 sweeps) against
the FP64 oracle.

The factorization is FP64 in every mode; the sweeps use the FP64 factors rounded to FP32
(unit roundoff u = 2^-24) or BF16 (u = 2^-8) and accumulate in FP32.  A triangular solve
in precision u with factors rounded at u has a normwise relative error of order
c * u * cond(L) cond(U) for a modest c; the bounds below are stated per test from the
measured conditioning of the case.  What the outer FP64 solver needs is checked directly:
GMRES reaches its tolerance measured with the FP64 true residual, and Newton converges
to the same FP64 residual tolerance as the FP64 path.
"""
import numpy as np
import pytest

import oracle as O
from paper_1810_04289_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PH = W.physics_config1()
U32, U16 = 2.0 ** -24, 2.0 ** -8


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def fsi_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_04289_amd import fsi
    fsi.load_library()
    return fsi


def solvers(fsi, m, opts, y_old, g, mask=None):
    """Oracle (FP64) and GPU solvers in each precision, all set up for the same step."""
    o = O.Oracle(m, PH, opts)
    o.set_step(1e-3, 1e-3, y_old, g, extra_mask=mask)
    gs = {}
    for prec in (fsi.PREC_FP64, fsi.PREC_FP32, fsi.PREC_BF16):
        s = fsi.Solver(m, PH, dict(opts, precision=prec))
        s.set_step(1e-3, 1e-3, s.vec(y_old), s.vec(g), None, mask)
        gs[prec] = s
    return o, gs


def test_mixed_pc_apply_rigid_wall(fsi_mod):
    """Stable factorization (wall frozen): the rounded sweeps against the FP64 oracle."""
    fsi = fsi_mod
    m = W.tube_mesh()
    y0 = W.poiseuille_state(m, 30.0, PH["mu_f"], 5.0)
    g = W.dirichlet_values(m, 30.0)
    o, gs = solvers(fsi, m, dict(nsub=4, overlap=1, ilu_level=1), y0, g, mask=W.rigid_wall_mask(m))
    y = o.impose_dirichlet(W.perturbed_state(m, y0, seed=8))
    o.jacobian(y)
    o.pc_setup()
    _, _, Vr = o.jacobian_get()
    v = np.random.default_rng(3).standard_normal(m.n)
    zr = o.pc_apply(v)
    err = {}
    for prec, s in gs.items():
        s.jacobian_set(Vr)  # the oracle's matrix: only the sweep precision differs
        s.pc_setup()
        z = s.vec()
        s.pc_apply(s.vec(v), z)
        err[prec] = np.linalg.norm(z.cpu().numpy() - zr) / np.linalg.norm(zr)
    say(f"[mixed pc, rigid wall] rel. error vs FP64 oracle: FP64 {err[0]:.2e} FP32 {err[1]:.2e} BF16 {err[2]:.2e}")
    assert err[fsi.PREC_FP64] <= 1e-10
    # measured 1.5 u (FP32) and 0.5 u (BF16) on this case; bounds of 1e3 u
    assert err[fsi.PREC_FP32] <= 1e3 * U32
    assert err[fsi.PREC_BF16] <= 1e3 * U16 and err[fsi.PREC_BF16] > err[fsi.PREC_FP32]


def test_mixed_gmres_and_newton_on_the_tree(fsi_mod):
    """Compliant wall, bench-like Schwarz configuration (depth-1 tree, subdomains of the
    benchmark's size, ILU(3)): GMRES with rounded sweeps reaches rtol 1e-3 in the FP64
    true residual, and a Newton step reaches the FP64 residual tolerance."""
    fsi = fsi_mod
    m = W.tree_mesh(depth=1, h=W.TREE_H[1])
    y0 = np.zeros(m.n)
    g = W.dirichlet_values(m, 30.0)
    opts = dict(nsub=33, overlap=1, ilu_level=3, gmres_maxit=600)
    o, gs = solvers(fsi, m, opts, y0, g)
    y = o.impose_dirichlet(W.perturbed_state(m, y0, seed=3))
    rhs = -o.residual(y)
    its = {}
    for prec, s in gs.items():
        s.jacobian(s.vec(y))
        s.pc_setup()
        x = s.vec()
        st = s.gmres(s.vec(rhs), x)
        its[prec] = st["iters"]
        rel = st["rnorm_true"] / st["rnorm0"]
        say(f"[mixed gmres, tree1] precision {prec}: its {st['iters']} true rel {rel:.2e}")
        assert st["converged"] == 1 and rel <= 1e-3
    # the rounded preconditioner may cost iterations, not convergence
    assert its[fsi.PREC_FP32] <= 2 * its[fsi.PREC_FP64] + 10
    # one Newton step from rest (rigid-wall start, as the benchmark's first steps) with FP32
    # sweeps: the same FP64 tolerance as the FP64 path
    s = gs[fsi.PREC_FP32]
    mask = W.rigid_wall_mask(m)
    s.set_step(1e-3, 1e-3, s.vec(y0), s.vec(g), None, mask)
    o.set_step(1e-3, 1e-3, y0, g, extra_mask=mask)
    yd = s.vec(y0)
    st, rc = s.newton_solve(yd)
    say(f"[mixed newton, tree1] FP32 sweeps: rc {rc} NI {st['newton_iters']} LI {st['lin_hist'][:st['newton_iters']]}")
    assert rc == 0 and st["converged"] == 1
    F = o.residual(yd.cpu().numpy())
    assert np.linalg.norm(F) <= 1.01e-6 * st["fnorm0"]
    for s in gs.values():
        s.close()


def test_uneven_batched_schwarz_ilu0_fp32(fsi_mod):
    """Batched Schwarz on uneven subdomains at oracle-checkable size: the depth-1 tree in 9
    subdomains of lognormal size (sigma 0.5, mean about 2,900 vertices), overlap 2, ILU(0),
    FP32 sweeps under FP64 GMRES, wall held rigid (ILU(0) stalls GMRES on the compliant
    wall).  The GPU setup on the given partition equals the oracle's, the rounded sweeps
    stay within the FP32 bound of the FP64 oracle, and GMRES converges in the FP64 true
    residual under every sweep schedule the tuner can pick."""
    fsi = fsi_mod
    m = W.tree_mesh(depth=1, h=W.TREE_H[1])
    part = W.uneven_partition(m, 9, sigma=0.5, seed=0)
    g = W.dirichlet_values(m, 30.0)
    y0 = np.zeros(m.n)
    mask = W.rigid_wall_mask(m)
    opts = dict(nsub=9, overlap=2, ilu_level=0, part=part, gmres_maxit=600)
    o, gs = solvers(fsi, m, opts, y0, g, mask=mask)
    s = gs[fsi.PREC_FP32]
    y = o.impose_dirichlet(W.perturbed_state(m, y0, seed=2))
    o.jacobian(y)
    o.pc_setup()
    _, _, Vr = o.jacobian_get()
    a, b = s.pc_get(factors=False), o.pc_get(factors=False)
    for k in ("part", "sub_ptr", "sub_verts", "sub_nowned", "blk_ptr", "lrowptr", "lcolind"):
        assert np.array_equal(a[k], b[k]), k
    sizes = np.diff(a["sub_ptr"])
    say(f"[uneven] owned {np.bincount(part).tolist()} extended {sizes.tolist()}")
    s.jacobian_set(Vr)
    s.pc_setup()
    v = np.random.default_rng(7).standard_normal(m.n)
    zr = o.pc_apply(v)
    z = s.vec()
    s.pc_apply(s.vec(v), z)
    err = np.linalg.norm(z.cpu().numpy() - zr) / np.linalg.norm(zr)
    say(f"[uneven] FP32 sweeps vs FP64 oracle: {err:.2e}")
    assert err <= 1e3 * U32
    best, us = s.pc_tune(reps=2)
    say(f"[uneven] tuner: best {best}, us {us}")
    rhs = -o.residual(y)
    for mb in s.SWEEP_MB:
        s.pc_select(mb)
        x = s.vec()
        st = s.gmres(s.vec(rhs), x)
        rel = st["rnorm_true"] / st["rnorm0"]
        say(f"[uneven] schedule {mb}: gmres its {st['iters']} true rel {rel:.2e}")
        assert st["converged"] == 1 and rel <= 1e-3
    for t in gs.values():
        t.close()


def bf16_round(x64):
    """FP64 -> BF16 as the library rounds: to FP32 first, then to nearest even on the 16
    dropped bits (NaN stays NaN), returned as the FP32 value of the BF16 bits."""
    u = np.ascontiguousarray(x64, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = np.where(nan, u | 0x00400000, u + 0x7FFF + ((u >> 16) & 1))
    return ((r >> 16) << 16).astype(np.uint32).view(np.float32)


def test_rounded_factors_in_place(fsi_mod):
    """The rounded factors are written over the FP64 factors in chunked launches.  On the
    depth-1 tree (ILU(3), 33 subdomains: 1.3e8 factor entries, about 17 launches for FP32
    and 9 for BF16) every rounded entry equals the FP64 entry rounded, from the same
    matrix."""
    fsi = fsi_mod
    m = W.tree_mesh(depth=1, h=W.TREE_H[1])
    g = W.dirichlet_values(m, W.inflow_peak(1e-3))
    o, gs = solvers(fsi, m, dict(nsub=33, overlap=1, ilu_level=3), np.zeros(m.n), g, mask=W.rigid_wall_mask(m))
    del o
    f = {}
    for prec, s in gs.items():
        y = s.vec()
        s.impose_dirichlet(y)
        s.jacobian(y)  # bitwise the same Jacobian in every solver
        s.pc_setup()
        pc = s.pc_get()
        f[prec] = pc["factors"].reshape(-1)
        s.close()
    say(f"[rounded factors] {f[0].size} entries")
    assert np.array_equal(f[fsi.PREC_FP32], f[fsi.PREC_FP64].astype(np.float32).astype(np.float64))
    assert np.array_equal(f[fsi.PREC_BF16], bf16_round(f[fsi.PREC_FP64]).astype(np.float64))


def test_fp32_factorization(fsi_mod):
    """The factorization itself in FP32 (precision 3) on the compliant depth-1 tree, ILU(3),
    subdomains of the benchmark's size.  Its input is the FP64 Jacobian rounded to FP32.
    Checked: the backward error |LU - A32| / (|L||U|) on sampled rows of several
    subdomains (A32 that input); GMRES to rtol 1e-3 in the FP64 true residual; and a Newton
    step from rest to the FP64 tolerance.  The wall's elimination is forward-unstable (a
    change of one rounding in A moves the factors' leading digits), so FP32 factors differ
    from the FP64 ones and only the backward error is a property to compare."""
    import test_gpu_parity as TP
    fsi = fsi_mod
    m = W.tree_mesh(depth=1, h=W.TREE_H[1])
    y0 = np.zeros(m.n)
    g = W.dirichlet_values(m, 30.0)
    opts = dict(nsub=33, overlap=1, ilu_level=3, gmres_maxit=600)
    o = O.Oracle(m, PH, opts)
    o.set_step(1e-3, 1e-3, y0, g)
    y = o.impose_dirichlet(W.perturbed_state(m, y0, seed=3))
    rhs = -o.residual(y)
    its = {}
    for prec in (fsi.PREC_FP64, fsi.PREC_FP32_FACTOR):
        s = fsi.Solver(m, PH, dict(opts, precision=prec))
        s.set_step(1e-3, 1e-3, s.vec(y0), s.vec(g))
        s.jacobian(s.vec(y))
        s.pc_setup()
        if prec == fsi.PREC_FP32_FACTOR:
            rp, ci, Vg = s.jacobian_get()
            V32 = Vg.astype(np.float32).astype(np.float64)
            pc = s.pc_get()
            rng = np.random.default_rng(5)
            worst = max(TP.lu_identity_worst(pc, rp, ci, V32, sub, rng, 12) for sub in (0, 11, 32))
            say(f"[fp32 factorization, tree1] backward error |LU - A32| / (|L||U|): {worst:.3e}")
            # an entry of LU is a sum of at most 7 x 107 products (107 blocks in the longest
            # row), each added with one rounding at u = 2^-24: gamma_n = n u / (1 - n u) =
            # 4.5e-5 (measured 1.9e-7)
            assert worst <= 5e-5
        x = s.vec()
        st = s.gmres(s.vec(rhs), x)
        its[prec] = st["iters"]
        rel = st["rnorm_true"] / st["rnorm0"]
        say(f"[fp32 factorization, tree1] precision {prec}: GMRES its {st['iters']} true rel {rel:.2e}")
        assert st["converged"] == 1 and rel <= 1e-3
        if prec == fsi.PREC_FP32_FACTOR:
            mask = W.rigid_wall_mask(m)
            s.set_step(1e-3, 1e-3, s.vec(y0), s.vec(g), None, mask)
            o.set_step(1e-3, 1e-3, y0, g, extra_mask=mask)
            yd = s.vec(y0)
            st, rc = s.newton_solve(yd)
            say(f"[fp32 factorization newton, tree1] rc {rc} NI {st['newton_iters']} LI {st['lin_hist'][:st['newton_iters']]}")
            assert rc == 0 and st["converged"] == 1
            F = o.residual(yd.cpu().numpy())
            assert np.linalg.norm(F) <= 1.01e-6 * st["fnorm0"]
        s.close()
    assert its[fsi.PREC_FP32_FACTOR] <= 2 * its[fsi.PREC_FP64] + 10
