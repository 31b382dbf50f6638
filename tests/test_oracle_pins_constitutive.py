"""Pins of the oracle's constitutive and stabilization terms at finite strain and speed.

Each test fixes a part of the element residual by something the paper or the mathematics
determines, not by the oracle's own formula:
  * the wall (§2.1, St. Venant-Kirchhoff: F = I + grad d, E = (F^T F - I)/2,
    S = lambda tr(E) I + 2 mu E, Pi = F S): nodal forces of a homogeneous finite stretch
    and shear on a patch against the divergence theorem, objectivity under a superposed
    rotation, symmetry of the Cauchy stress sigma = Pi F^T / det F, and the order of a
    manufactured finite-strain solution;
  * the stabilization parameter tau_M of the SUPG/PSPG fluid (§2.2; the form is a
    reading, the paper defers it to its references): its closed form on an axis-aligned
    right tetrahedron, where the element metric is diagonal, its convective speed on a
    translating element, frame indifference of the whole fluid residual under a rigid
    rotation of the problem and its invariance under a Galilean boost;
  * dimensional homogeneity of every row under a change of units;
  * the harmonic mesh extension (§2.1 eq. (1)): second-order convergence to a harmonic
    field;
  * the fluid pressure: first-order (or better) convergence in a manufactured flow.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_1810_04289_amd import workload as W

PH = W.physics_config1()
LAM = PH["E_s"] * PH["nu_s"] / ((1 + PH["nu_s"]) * (1 - 2 * PH["nu_s"]))
MU = PH["E_s"] / (2 * (1 + PH["nu_s"]))


def one_tet_mesh(Xe, domain):
    tets = W._orient(Xe, np.array([[0, 1, 2, 3]])).astype(np.int32)
    bf, _ = W.boundary_faces(tets)
    return W.Mesh(X=np.asarray(Xe, float), tets=tets, tet_domain=np.array([domain], dtype=np.int8),
                  bfaces=bf, bface_tag=np.zeros(len(bf), dtype=np.int8))


def solid_cube(nc=3, seed=3, jitter=0.1):
    m = W.cube_mesh(nc, L=1.0, jitter=jitter, seed=seed)
    return W.Mesh(X=m.X, tets=m.tets, tet_domain=np.ones(m.ntets, dtype=np.int8), bfaces=m.bfaces,
                  bface_tag=np.zeros_like(m.bface_tag), info=m.info)


def rotation(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def first_piola(Fd):
    """Pi = F S of the St. Venant-Kirchhoff wall (§2.1)."""
    E = 0.5 * (Fd.T @ Fd - np.eye(3))
    S = LAM * np.trace(E) * np.eye(3) + 2 * MU * E
    return Fd @ S


GENERIC_TET = np.array([[0.02, -0.01, 0.03], [0.31, 0.04, -0.02], [0.07, 0.19, 0.05], [0.03, 0.06, 0.42]])

# homogeneous deformation gradients with finite strain: a triaxial stretch, a simple shear,
# and a general non-symmetric one
F_CASES = {
    "stretch": np.diag([1.3, 0.85, 1.1]),
    "shear": np.array([[1.0, 0.4, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]),
    "general": np.array([[1.12, 0.31, -0.08], [-0.05, 0.93, 0.22], [0.17, -0.11, 1.07]]),
}


# ------------------------------------------------------------------------------------------
# wall: homogeneous finite deformation of a patch against the divergence theorem
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("case", sorted(F_CASES))
def test_wall_nodal_forces_of_homogeneous_finite_strain(case):
    # A homogeneous deformation x = F X has a constant first Piola stress Pi, so the
    # P1 nodal force sum_K |K| Pi grad phi_a = Pi int grad phi_a vanishes at interior
    # vertices and equals Pi sum_f (A_f / 3) N_f (outward reference normals of the boundary
    # faces that hold a) at boundary vertices.
    Fh = F_CASES[case]
    m = solid_cube()
    dt = 1e-3
    y = np.zeros((m.nverts, 7))
    y[:, 4:7] = m.X @ (Fh - np.eye(3)).T
    o = O.Oracle(m, PH, dict(nsub=1, overlap=0))
    o.set_step(0.0, dt, np.zeros(m.n), np.zeros(m.n))
    F = o.residual(y.ravel()).reshape(-1, 7)
    P = m.X[m.bfaces]
    an = 0.5 * np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])   # A_f N_f
    wsum = np.zeros((m.nverts, 3))
    for j in range(3):
        np.add.at(wsum, m.bfaces[:, j], an / 3.0)
    expect = dt * wsum @ first_piola(Fh).T
    scale = np.abs(expect).max()
    assert scale > 0
    np.testing.assert_allclose(F[:, 0:3], expect, rtol=0, atol=1e-12 * scale)


@pytest.mark.parametrize("case", sorted(F_CASES))
def test_wall_forces_are_objective(case):
    # Superposing a rigid rotation Q on the deformed wall (x -> Q x) rotates the first
    # Piola stress (Pi -> Q Pi) and with it every nodal force.
    Fh = F_CASES[case]
    m = solid_cube(nc=2, seed=9)
    rng = np.random.default_rng(21)
    Q = rotation([0.3, -1.0, 0.7], 0.9)
    x = m.X @ Fh.T + 0.02 * rng.uniform(-1, 1, m.X.shape)          # a non-homogeneous state
    o = O.Oracle(m, PH, dict(nsub=1, overlap=0))
    o.set_step(0.0, 1e-3, np.zeros(m.n), np.zeros(m.n))
    y = np.zeros((m.nverts, 7))
    y[:, 4:7] = x - m.X
    F1 = o.residual(y.ravel()).reshape(-1, 7)
    y[:, 4:7] = x @ Q.T - m.X
    F2 = o.residual(y.ravel()).reshape(-1, 7)
    scale = np.abs(F1[:, 0:3]).max()
    np.testing.assert_allclose(F2[:, 0:3], F1[:, 0:3] @ Q.T, rtol=0, atol=1e-11 * scale)


@pytest.mark.parametrize("case", sorted(F_CASES))
def test_wall_cauchy_stress_is_symmetric(case):
    # The stress the oracle applies, recovered from one element's nodal forces
    # (R_a = dt |K| Pi grad phi_a, a = 1..3), gives a symmetric Cauchy stress
    # sigma = Pi F^T / det F (balance of angular momentum, §2.1).
    Fh = F_CASES[case]
    m = one_tet_mesh(GENERIC_TET, 1)
    dt = 1e-3
    y = np.zeros((4, 7))
    y[:, 4:7] = m.X @ (Fh - np.eye(3)).T
    o = O.Oracle(m, PH, dict(nsub=1, overlap=0))
    o.set_step(0.0, dt, np.zeros(m.n), np.zeros(m.n))
    Re, _ = o.element(y.ravel(), 0)
    Re = Re.reshape(4, 7)
    Xe = m.X[m.tets[0]]
    Jm = (Xe[1:] - Xe[0]).T
    vol = np.linalg.det(Jm) / 6.0
    G = np.linalg.inv(Jm)                  # row k: grad phi_{k+1}
    Rm = Re[1:, 0:3].T / (dt * vol)        # column k: Pi grad phi_{k+1}
    Pi = Rm @ np.linalg.inv(G.T)
    sigma = Pi @ Fh.T / np.linalg.det(Fh)
    assert np.abs(sigma - sigma.T).max() <= 1e-12 * np.abs(sigma).max()
    # and it is the stress of a finite strain: far from the linear-elastic one
    lin = LAM * np.trace(Fh - np.eye(3)) * np.eye(3) + MU * (Fh + Fh.T - 2 * np.eye(3))
    assert np.abs(Pi - lin).max() > 1e-3 * np.abs(Pi).max()


# ------------------------------------------------------------------------------------------
# stabilization parameter
# ------------------------------------------------------------------------------------------
def tau_from_pressure_block(o, y, m, dt, rho):
    """tau_M recovered from the PSPG pressure-pressure block dt (tau/rho) |K| grad phi_a . grad phi_b."""
    _, Je = o.element(y.ravel(), 0)
    Cpp = np.array([[Je[7 * a + 3, 7 * b + 3] for b in range(4)] for a in range(4)])
    Xe = m.X[m.tets[0]] + y.reshape(-1, 7)[m.tets[0], 4:7]
    Jm = (Xe[1:] - Xe[0]).T
    vol = np.linalg.det(Jm) / 6.0
    Gi = np.linalg.inv(Jm)
    g = np.vstack([-Gi.sum(0), Gi])
    L = vol * g @ g.T
    kappa = (Cpp * L).sum() / (L * L).sum()
    np.testing.assert_allclose(Cpp, kappa * L, rtol=1e-12, atol=1e-14 * np.abs(Cpp).max())
    return kappa * rho / dt


@pytest.mark.parametrize("hx,hy,hz,c,dt,mu", [
    (0.3, 0.1, 0.05, (20.0, -7.0, 3.0), 1e-2, 0.035),
    (0.2, 0.5, 0.1, (-1.0, 4.0, 9.0), 5e-2, 0.5),
    (0.05, 0.08, 0.02, (0.0, 0.0, 0.0), 1.0, 0.2),     # viscous limit
    (1.0, 2.0, 0.5, (3.0, 1.0, -2.0), 1e-3, 0.035),     # time-step limit
])
def test_tau_closed_form_on_axis_aligned_right_tet(hx, hy, hz, c, dt, mu):
    # With vertices 0, hx e1, hy e2, hz e3 the element map is diagonal, and the metric of the
    # unit reference element is diag(1/h_i^2): c.G.c = sum c_i^2 / h_i^2 and
    # G:G = sum 1/h_i^4.  With no mesh motion and a uniform velocity c, tau_M is
    # [(2/dt)^2 + c.G.c + C_I nu^2 G:G]^(-1/2) with C_I = 36.
    ph = dict(PH, mu_f=mu)
    Xe = np.array([[0, 0, 0], [hx, 0, 0], [0, hy, 0], [0, 0, hz]], float)
    m = one_tet_mesh(Xe, 0)
    assert np.array_equal(m.tets[0], [0, 1, 2, 3])
    y = np.zeros((4, 7))
    y[:, 0:3] = c
    o = O.Oracle(m, ph, dict(nsub=1, overlap=0))
    o.set_step(0.0, dt, y.ravel(), np.zeros(m.n))
    h = np.array([hx, hy, hz])
    nu = mu / ph["rho_f"]
    cGc = float(np.sum(np.square(c) / h ** 2))
    GG = float(np.sum(h ** -4.0))
    tau = (4.0 / dt ** 2 + cGc + 36.0 * nu ** 2 * GG) ** -0.5
    assert tau_from_pressure_block(o, y, m, dt, ph["rho_f"]) == pytest.approx(tau, rel=1e-12)


def test_tau_uses_velocity_relative_to_the_moving_mesh():
    # Translating the element rigidly (d = d_old + w dt at every vertex) leaves its metric
    # unchanged; the convective speed in tau_M is then the element mean of u - w.
    hx, hy, hz, dt, mu = 0.2, 0.07, 0.11, 4e-3, 0.05
    ph = dict(PH, mu_f=mu)
    Xe = np.array([[0, 0, 0], [hx, 0, 0], [0, hy, 0], [0, 0, hz]], float)
    m = one_tet_mesh(Xe, 0)
    u = np.array([12.0, -3.0, 5.0])
    w = np.array([-4.0, 6.0, 9.0])
    s0 = np.array([0.01, -0.02, 0.005])
    y = np.zeros((4, 7))
    yo = np.zeros((4, 7))
    y[:, 0:3] = u
    yo[:, 0:3] = u
    yo[:, 4:7] = s0
    y[:, 4:7] = s0 + w * dt
    o = O.Oracle(m, ph, dict(nsub=1, overlap=0))
    o.set_step(0.0, dt, yo.ravel(), np.zeros(m.n))
    h = np.array([hx, hy, hz])
    c = u - w
    tau = (4.0 / dt ** 2 + np.sum(c ** 2 / h ** 2) + 36.0 * (mu / ph["rho_f"]) ** 2 * np.sum(h ** -4.0)) ** -0.5
    assert tau_from_pressure_block(o, y, m, dt, ph["rho_f"]) == pytest.approx(tau, rel=1e-12)


def test_residual_is_dimensionally_homogeneous():
    # Changing the units of length, time and mass by factors a, b, c changes every row of
    # F = dt R by the factor its dimension implies: momentum rows (an impulse) a c / b,
    # continuity rows (a volume) a^3, mesh rows (|K| |grad phi|^2 d dt) a^2 b, kinematic rows a, Dirichlet rows and
    # dummy pressure rows the unit of their unknown.  A misplaced density, time step or
    # length scale anywhere in F breaks this.
    a, b, c = 0.37, 2.9, 5.3
    m = W.tube_mesh(n_sections=3, length=0.6, fluid_radii=(0.25, 0.5), wall_radii=(0.6,), nper=6)
    rng = np.random.default_rng(41)
    ph = dict(PH, eta_s=30.0, mu_f=0.2)
    dt = 2e-3
    y = np.zeros((m.nverts, 7))
    yo = np.zeros((m.nverts, 7))
    y[:, 0:3] = rng.uniform(-30, 30, (m.nverts, 3))
    y[:, 3] = rng.uniform(-100, 100, m.nverts)
    y[:, 4:7] = rng.uniform(-3e-3, 3e-3, (m.nverts, 3))
    yo[:, 0:3] = y[:, 0:3] + rng.uniform(-2, 2, (m.nverts, 3))
    yo[:, 4:7] = rng.uniform(-3e-3, 3e-3, (m.nverts, 3))
    g = rng.uniform(-1, 1, (m.nverts, 7))
    f = rng.uniform(-500, 500, (m.nverts, 3))
    unit = np.array([a / b] * 3 + [c / (a * b * b)] + [a] * 3)          # u, p, d

    def run(scaled):
        mesh, phx, dtx, yx, yox, gx, fx = m, ph, dt, y, yo, g, f
        if scaled:
            mesh = W.Mesh(X=m.X * a, tets=m.tets, tet_domain=m.tet_domain, bfaces=m.bfaces,
                          bface_tag=m.bface_tag)
            phx = dict(ph, rho_f=ph["rho_f"] * c / a ** 3, mu_f=ph["mu_f"] * c / (a * b),
                       rho_s=ph["rho_s"] * c / a ** 3, E_s=ph["E_s"] * c / (a * b * b),
                       eta_s=ph["eta_s"] * c / (a ** 3 * b))
            dtx, yx, yox, gx, fx = dt * b, y * unit, yo * unit, g * unit, f * a / (b * b)
        o = O.Oracle(mesh, phx, dict(nsub=1, overlap=0))
        o.set_step(0.0, dtx, yox.ravel(), gx.ravel(), body_force=fx.ravel())
        _, rk, _ = o.topology()
        return o.residual(yx.ravel()).reshape(-1, 7), rk.reshape(-1, 7)

    F1, rk = run(False)
    F2, _ = run(True)
    elem = np.array([a * c / b] * 3 + [a ** 3] + [a * a * b] * 3)
    scale = np.where(rk == 0, elem[None, :], np.where(rk == 2, a, unit[None, :]))
    for rows in (rk == 0, rk == 1, rk == 2, rk == 3):
        assert rows.any()
    for col in range(7):
        ref = F1[:, col] * scale[:, col]
        np.testing.assert_allclose(F2[:, col], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_fluid_residual_is_galilean_invariant():
    # A uniform velocity V added to the fluid (u and u_old) and to the mesh (d -> d + V dt,
    # so w -> w + V) leaves u - w, the velocity gradient, the mesh shape and the
    # acceleration unchanged: every row of F, the SUPG and PSPG terms included, is the same.
    rng = np.random.default_rng(33)
    m = W.cube_mesh(2, jitter=0.2, seed=6)
    m = W.Mesh(X=m.X, tets=m.tets, tet_domain=m.tet_domain, bfaces=m.bfaces,
               bface_tag=np.zeros_like(m.bface_tag), info=m.info)
    dt = 2e-3
    h = 0.5
    y = np.zeros((m.nverts, 7))
    yo = np.zeros((m.nverts, 7))
    y[:, 0:3] = rng.uniform(-40, 40, (m.nverts, 3))
    y[:, 3] = rng.uniform(-50, 50, m.nverts)
    y[:, 4:7] = 0.05 * h * rng.uniform(-1, 1, (m.nverts, 3))
    yo[:, 0:3] = y[:, 0:3] + rng.uniform(-3, 3, (m.nverts, 3))
    yo[:, 4:7] = 0.05 * h * rng.uniform(-1, 1, (m.nverts, 3))
    f = rng.uniform(-100, 100, (m.nverts, 3))
    V = np.array([17.0, -9.0, 23.0])
    ph = dict(PH, mu_f=0.3)

    def run(boost):
        yb, yob = y.copy(), yo.copy()
        if boost:
            yb[:, 0:3] += V
            yob[:, 0:3] += V
            yb[:, 4:7] += V * dt
        o = O.Oracle(m, ph, dict(nsub=1, overlap=0))
        o.set_step(0.0, dt, yob.ravel(), np.zeros(m.n), body_force=f.ravel())
        return o.residual(yb.ravel()).reshape(-1, 7)

    F1, F2 = run(False), run(True)
    for cols in ((0, 1, 2), (3,), (4, 5, 6)):
        scale = np.abs(F1[:, cols]).max()
        np.testing.assert_allclose(F2[:, cols], F1[:, cols], rtol=0, atol=1e-11 * scale)


def test_fluid_residual_is_frame_indifferent():
    # Rotating the whole problem (reference mesh, velocities, displacements, body force)
    # by Q rotates the momentum and mesh rows and leaves the continuity rows unchanged.
    # tau_M enters through c.G.c, which must be a scalar invariant.
    rng = np.random.default_rng(31)
    m = W.cube_mesh(2, jitter=0.2, seed=8)
    Xs = m.X * np.array([1.0, 0.35, 0.6])            # anisotropic elements
    m = W.Mesh(X=Xs, tets=m.tets, tet_domain=m.tet_domain, bfaces=m.bfaces,
               bface_tag=np.zeros_like(m.bface_tag), info=m.info)
    Q = rotation([0.2, 0.9, -0.4], 1.1)
    h = 0.15
    y = np.zeros((m.nverts, 7))
    yo = np.zeros((m.nverts, 7))
    y[:, 0:3] = rng.uniform(-40, 40, (m.nverts, 3))
    y[:, 3] = rng.uniform(-50, 50, m.nverts)
    y[:, 4:7] = 0.05 * h * rng.uniform(-1, 1, (m.nverts, 3))
    yo[:, 0:3] = y[:, 0:3] + rng.uniform(-1, 1, (m.nverts, 3))
    yo[:, 4:7] = 0.05 * h * rng.uniform(-1, 1, (m.nverts, 3))
    f = rng.uniform(-100, 100, (m.nverts, 3))
    ph = dict(PH, mu_f=0.3)
    dt = 2e-3

    def run(Xr, R):
        mr = W.Mesh(X=Xr, tets=m.tets, tet_domain=m.tet_domain, bfaces=m.bfaces, bface_tag=m.bface_tag)
        yr, yor = y.copy(), yo.copy()
        for a in (0, 4):
            yr[:, a:a + 3] = y[:, a:a + 3] @ R.T
            yor[:, a:a + 3] = yo[:, a:a + 3] @ R.T
        o = O.Oracle(mr, ph, dict(nsub=1, overlap=0))
        o.set_step(0.0, dt, yor.ravel(), np.zeros(m.n), body_force=(f @ R.T).ravel())
        return o.residual(yr.ravel()).reshape(-1, 7)

    F1 = run(m.X, np.eye(3))
    F2 = run(m.X @ Q.T, Q)
    for cols, rot in (((0, 1, 2), True), ((3,), False), ((4, 5, 6), True)):
        a = F1[:, cols] @ Q.T if rot else F1[:, cols]
        scale = np.abs(F1[:, cols]).max()
        np.testing.assert_allclose(F2[:, cols], a, rtol=0, atol=1e-11 * scale)
    # the stabilization is active here: dropping it would change the continuity rows
    assert np.abs(F1[:, 3]).max() > 0


# ------------------------------------------------------------------------------------------
# convergence orders (manufactured solutions)
# ------------------------------------------------------------------------------------------
def newton_sparse(o, m, y, iters=12, tol=1e-11):
    F0 = np.linalg.norm(o.residual(y))
    for _ in range(iters):
        F = o.residual(y)
        if np.linalg.norm(F) <= tol * F0:
            break
        o.jacobian(y)
        A = O.jac_scipy(*o.jacobian_get(), m.nverts).tocsc()
        y = y - spla.spsolve(A, F)
    return y


def _svk_field(X, A=0.02):
    """Manufactured wall displacement with strains of about 5% (larger amplitudes admit
    several discrete roots of the non-convex St. Venant-Kirchhoff energy)."""
    k = np.array([[1.1, 0.7, 0.4], [-0.5, 1.3, 0.8], [0.6, -0.9, 1.2]]) * (0.5 * math.pi)
    b = np.array([0.3, -0.2, 0.5])
    amp = A * np.array([1.0, 0.8, -0.9])
    ph = X @ k.T + b                    # phase of component i
    d = amp * np.sin(ph)
    gd = (amp * np.cos(ph))[..., :, None] * k[None] if X.ndim == 2 else None
    return d, gd


def _svk_piola_field(X):
    _, gd = _svk_field(X)
    Fd = np.eye(3)[None] + gd
    E = 0.5 * (np.einsum("nki,nkj->nij", Fd, Fd) - np.eye(3)[None])
    S = LAM * np.trace(E, axis1=1, axis2=2)[:, None, None] * np.eye(3)[None] + 2 * MU * E
    return np.einsum("nik,nkj->nij", Fd, S)


def svk_mms_error(nc):
    # steady wall: -div Pi = rho_s f in the reference configuration; the body force comes
    # from the exact field (divergence by fourth-order central differences of Pi)
    m = solid_cube(nc=nc, seed=1, jitter=0.1)
    d_ex, _ = _svk_field(m.X)
    hfd = 1e-3
    div = np.zeros((m.nverts, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = hfd
        dP = (8 * (_svk_piola_field(m.X + e) - _svk_piola_field(m.X - e))
              - (_svk_piola_field(m.X + 2 * e) - _svk_piola_field(m.X - 2 * e))) / (12 * hfd)
        div += dP[:, :, j]
    f = -div / PH["rho_s"]
    bnd = np.any((m.X < 1e-12) | (m.X > 1 - 1e-12), axis=1)
    g = np.zeros((m.nverts, 7))
    g[:, 4:7] = d_ex
    mask = np.zeros((m.nverts, 7), dtype=np.uint8)
    mask[bnd, 0:3] = 1
    mask[bnd, 4:7] = 1
    # a long step: the inertia left in the steady balance is rho_s d / dt^2 (1e-12 of the
    # stiffness here)
    o = O.Oracle(m, PH, dict(nsub=1, overlap=0))
    o.set_step(0.0, 100.0, np.zeros(m.n), g.ravel(), body_force=f.ravel(), extra_mask=mask.ravel())
    # Newton from the interpolated field (the discrete root does not depend on the start)
    y0 = np.zeros((m.nverts, 7))
    y0[:, 4:7] = d_ex
    y0[:, 0:3] = d_ex / 100.0
    y = newton_sparse(o, m, o.impose_dirichlet(y0.ravel())).reshape(-1, 7)
    err = np.sqrt(np.mean(np.sum((y[~bnd, 4:7] - d_ex[~bnd]) ** 2, 1)))
    return err / np.sqrt(np.mean(np.sum(d_ex ** 2, 1))), 1.0 / nc


def test_wall_manufactured_solution_second_order():
    errs = [svk_mms_error(nc) for nc in (4, 6, 8)]
    rates = [math.log(errs[i][0] / errs[i + 1][0]) / math.log(errs[i][1] / errs[i + 1][1]) for i in range(2)]
    # measured: 2.1e-2, 9.3e-3, 5.3e-3 (rates 1.97, 1.95)
    assert min(rates) > 1.8, (errs, rates)
    assert errs[-1][0] < 0.01, errs


def laplace_mms_error(nc):
    # harmonic mesh extension with the boundary values of a harmonic field; velocity and
    # pressure held at zero
    m = W.cube_mesh(nc, jitter=0.1, seed=4)
    x, yv, z = m.X[:, 0], m.X[:, 1], m.X[:, 2]
    A = 2e-3
    d_ex = A * np.stack([np.exp(0.5 * math.pi * x) * np.sin(0.5 * math.pi * yv),
                         np.sinh(0.5 * math.pi * z) * np.cos(0.5 * math.pi * x),
                         x * yv + yv ** 2 - z ** 2], 1)
    bnd = W.tag_vertices(m, [1])
    g = np.zeros((m.nverts, 7))
    g[:, 4:7] = d_ex
    mask = np.zeros((m.nverts, 7), dtype=np.uint8)
    mask[:, 0:4] = 1
    mask[bnd, 4:7] = 1
    o = O.Oracle(m, PH, dict(nsub=1, overlap=0))
    o.set_step(0.0, 1.0, g.ravel(), g.ravel(), extra_mask=mask.ravel())
    y = newton_sparse(o, m, o.impose_dirichlet(np.zeros(m.n))).reshape(-1, 7)
    err = np.sqrt(np.mean(np.sum((y[~bnd, 4:7] - d_ex[~bnd]) ** 2, 1)))
    return err / np.sqrt(np.mean(np.sum(d_ex ** 2, 1))), 1.0 / nc


def test_mesh_extension_second_order():
    # measured: 2.7e-3, 7.4e-4, 3.3e-4 (rates 1.84, 2.00)
    errs = [laplace_mms_error(nc) for nc in (4, 8, 12)]
    rates = [math.log(errs[i][0] / errs[i + 1][0]) / math.log(errs[i][1] / errs[i + 1][1]) for i in range(2)]
    assert rates[0] > 1.7 and rates[1] > 1.7, (errs, rates)


def ns_mms_pressure_error(nc, U=0.2):
    """Steady stabilized Navier-Stokes on the unit cube; L2 nodal pressure error."""
    rho, mu = PH["rho_f"], PH["mu_f"]
    nu = mu / rho
    m = W.cube_mesh(nc, jitter=0.1, seed=1)
    x, yv, z = m.X[:, 0], m.X[:, 1], m.X[:, 2]
    pi = math.pi
    s, c = np.sin, np.cos
    u = U * np.stack([s(pi * x) * c(pi * yv) * c(pi * z),
                      -0.5 * c(pi * x) * s(pi * yv) * c(pi * z),
                      -0.5 * c(pi * x) * c(pi * yv) * s(pi * z)], 1)
    du = np.zeros((m.nverts, 3, 3))
    du[:, 0, 0] = pi * c(pi * x) * c(pi * yv) * c(pi * z)
    du[:, 0, 1] = -pi * s(pi * x) * s(pi * yv) * c(pi * z)
    du[:, 0, 2] = -pi * s(pi * x) * c(pi * yv) * s(pi * z)
    du[:, 1, 0] = 0.5 * pi * s(pi * x) * s(pi * yv) * c(pi * z)
    du[:, 1, 1] = -0.5 * pi * c(pi * x) * c(pi * yv) * c(pi * z)
    du[:, 1, 2] = 0.5 * pi * c(pi * x) * s(pi * yv) * s(pi * z)
    du[:, 2, 0] = 0.5 * pi * s(pi * x) * c(pi * yv) * s(pi * z)
    du[:, 2, 1] = 0.5 * pi * c(pi * x) * s(pi * yv) * s(pi * z)
    du[:, 2, 2] = -0.5 * pi * c(pi * x) * c(pi * yv) * c(pi * z)
    du *= U
    lap = -3 * pi ** 2 * u
    p = U * c(pi * x) * s(pi * z)
    gp = U * np.stack([-pi * s(pi * x) * s(pi * z), 0 * x, pi * c(pi * x) * c(pi * z)], 1)
    f = np.einsum("aij,aj->ai", du, u) - nu * lap + gp / rho
    y = np.zeros((m.nverts, 7))
    y[:, 0:3] = u
    y[:, 3] = p
    bnd = W.tag_vertices(m, [1])
    mask = np.zeros((m.nverts, 7), dtype=np.uint8)
    mask[:, 4:7] = 1
    mask[bnd, 0:3] = 1
    pin = int(np.argmin(np.linalg.norm(m.X - 0.5, axis=1)))
    mask[pin, 3] = 1
    o = O.Oracle(m, PH, dict(nsub=1, overlap=0))
    o.set_step(0.0, 1e6, y.ravel(), y.ravel(), body_force=f.ravel(), extra_mask=mask.ravel())
    yh = newton_sparse(o, m, o.impose_dirichlet(y.ravel())).reshape(-1, 7)
    ep = yh[:, 3] - p
    ep -= ep.mean()
    return np.sqrt(np.mean(ep ** 2)) / np.sqrt(np.mean((p - p.mean()) ** 2)), 1.0 / nc


def test_manufactured_solution_pressure_converges():
    # the stabilized equal-order pair converges in pressure at first order or better; the
    # nodal error measured here: 1.9e-1, 8.8e-2, 4.1e-2 (rates 1.87, 1.89)
    errs = [ns_mms_pressure_error(nc) for nc in (4, 6, 9)]
    rates = [math.log(errs[i][0] / errs[i + 1][0]) / math.log(errs[i][1] / errs[i + 1][1]) for i in range(2)]
    assert min(rates) > 1.5, (errs, rates)
