// Oracle: element residuals, the nonlinear function F(y) and its exact Jacobian
// (test infrastructure only).
//
// Paper §2.1: ALE map x = X + d_m; harmonic mesh extension eq. (1); St. Venant-Kirchhoff
// wall eq. (2) with F = I + grad d, E = (F^T F - I)/2, S = lambda tr(E) I + 2 mu E,
// Pi = F S and the Lame constants from (E_s, nu_s); ALE Navier-Stokes eq. (3) with
// sigma_f = -p I + 2 mu eps(u).  §2.2: P1 elements for the wall and the mesh, a
// stabilized P1-P1 pair (SUPG + PSPG) for the fluid, strong interface coupling through
// shared unknowns (eqs. (6)-(7)), backward Euler eq. (9) and F(y) = 0 eq. (10).
//
// Readings where the paper is silent (all listed in the design notes):
//  * F = dt * R on every equation row (eq. (9) multiplied through), y - g on Dirichlet rows.
//  * SUPG/PSPG with tau_M = [(2/dt)^2 + cbar.G.cbar + C_I nu^2 G:G]^(-1/2), cbar the element
//    mean of u - w, G = Jxi^T Jxi, no LSIC term; the momentum residual r_q drops the
//    viscous term (it vanishes inside a P1 element).
//  * 4-point degree-2 quadrature for fluid terms and all masses; one point for the
//    constant stiffness integrands.
//  * wall in first-order form: solid momentum rows act on the velocity u, nodal kinematic
//    rows (d - d_old)/dt - u = 0 tie the displacement to it.
//  * body force: nodal field interpolated with the P1 basis.
#include <algorithm>
#include <cstring>

#include "core.hpp"

namespace fsio {

thread_local OpCount g_ops;

static const double kQa = (5.0 + 3.0 * std::sqrt(5.0)) / 20.0;  // barycentric weight of the own vertex
static const double kQb = (5.0 - std::sqrt(5.0)) / 20.0;        // weight of the other three

template <class T>
static T det3(const T m[3][3]) {
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
         m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
         m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

template <class T>
static void inv3(const T m[3][3], const T& det, T r[3][3]) {
  r[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) / det;
  r[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / det;
  r[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / det;
  r[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) / det;
  r[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / det;
  r[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / det;
  r[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) / det;
  r[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) / det;
  r[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / det;
}

// P1 shape-function gradients of the tet with vertex coordinates x[4][3]:
// with Jm = [x1-x0, x2-x0, x3-x0] and Jxi = Jm^{-1}, grad phi_a = row a-1 of Jxi (a>0),
// grad phi_0 = -(sum of the others).  Returns det Jm = 6|K|.
template <class T>
static T p1_gradients(const T x[4][3], T gr[4][3], T Jxi[3][3]) {
  T Jm[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Jm[i][j] = x[j + 1][i] - x[0][i];
  T det = det3(Jm);
  if (val(det) == 0.0) return det;
  inv3(Jm, det, Jxi);
  for (int k = 0; k < 3; ++k) {
    gr[1][k] = Jxi[0][k];
    gr[2][k] = Jxi[1][k];
    gr[3][k] = Jxi[2][k];
    gr[0][k] = -(gr[1][k] + gr[2][k] + gr[3][k]);
  }
  return det;
}

// Fluid element: rows [4][0..2] momentum, [4][3] continuity, [4][4..6] mesh Laplace.
// T: the unknowns' scalar; D: the data's (reference coordinates, old state, body force),
// double except when the operations are counted.
template <class T, class D>
static bool fluid_element(const Phys& ph, double dt, const D X[4][3], const T y[4][7],
                          const D yo[4][7], const D f[4][3], T R[4][7]) {
  const double rho = ph.rho_f, mu = ph.mu_f, nu = mu / rho;
  T x[4][3], w[4][3];
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) {
      x[a][i] = X[a][i] + y[a][4 + i];               // ALE map x = X + d_m
      w[a][i] = (y[a][4 + i] - yo[a][4 + i]) / dt;  // backward-Euler mesh velocity
    }
  T gr[4][3], Jxi[3][3];
  T det = p1_gradients(x, gr, Jxi);
  if (!(val(det) > 0.0)) return false;
  T vol = det / 6.0;

  T G[3][3];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) G[k][l] = Jxi[0][k] * Jxi[0][l] + Jxi[1][k] * Jxi[1][l] + Jxi[2][k] * Jxi[2][l];
  T gu[3][3], gp[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = 0.0;
      for (int a = 0; a < 4; ++a) s += y[a][i] * gr[a][j];
      gu[i][j] = s;  // d u_i / d x_j
    }
  for (int j = 0; j < 3; ++j) {
    T s = 0.0;
    for (int a = 0; a < 4; ++a) s += y[a][3] * gr[a][j];
    gp[j] = s;
  }
  T divu = gu[0][0] + gu[1][1] + gu[2][2];
  T cbar[3];
  for (int i = 0; i < 3; ++i) {
    T s = 0.0;
    for (int a = 0; a < 4; ++a) s += y[a][i] - w[a][i];
    cbar[i] = s / 4.0;
  }
  T GG = 0.0, cGc = 0.0;
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      GG += G[k][l] * G[k][l];
      cGc += cbar[k] * G[k][l] * cbar[l];
    }
  T tau = 1.0 / sqrt((2.0 / dt) * (2.0 / dt) + cGc + ph.C_I * nu * nu * GG);
  T pbar = (y[0][3] + y[1][3] + y[2][3] + y[3][3]) / 4.0;

  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 7; ++r) R[a][r] = 0.0;

  for (int q = 0; q < 4; ++q) {
    double lam[4];
    for (int a = 0; a < 4; ++a) lam[a] = (a == q) ? kQa : kQb;
    T uq[3], wq[3], cq[3];
    D uoq[3], fq[3];
    for (int i = 0; i < 3; ++i) {
      T su = 0.0, sw = 0.0;
      D so = 0.0, sf = 0.0;
      for (int a = 0; a < 4; ++a) {
        su += lam[a] * y[a][i];
        sw += lam[a] * w[a][i];
        so += lam[a] * yo[a][i];
        sf += lam[a] * f[a][i];
      }
      uq[i] = su; wq[i] = sw; uoq[i] = so; fq[i] = sf;
      cq[i] = uq[i] - wq[i];
    }
    T conv[3], rq[3], dudt[3];
    for (int i = 0; i < 3; ++i) {
      conv[i] = gu[i][0] * cq[0] + gu[i][1] * cq[1] + gu[i][2] * cq[2];
      dudt[i] = (uq[i] - uoq[i]) / dt;
      // strong momentum residual at the point (viscous term vanishes for P1)
      rq[i] = rho * dudt[i] + rho * conv[i] + gp[i] - rho * fq[i];
    }
    T wq4 = vol / 4.0;
    for (int a = 0; a < 4; ++a) {
      T cgrad = cq[0] * gr[a][0] + cq[1] * gr[a][1] + cq[2] * gr[a][2];
      for (int i = 0; i < 3; ++i)
        R[a][i] += wq4 * (rho * dudt[i] * lam[a] + rho * conv[i] * lam[a] - rho * fq[i] * lam[a] +
                          tau * cgrad * rq[i]);
      T gr_r = gr[a][0] * rq[0] + gr[a][1] * rq[1] + gr[a][2] * rq[2];
      R[a][3] += wq4 * (lam[a] * divu + (tau / rho) * gr_r);
    }
  }
  // viscous and pressure terms, exact for P1
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) {
      T s = 0.0;
      for (int j = 0; j < 3; ++j) s += (gu[i][j] + gu[j][i]) * gr[a][j];
      R[a][i] += vol * (mu * s - pbar * gr[a][i]);
    }

  // harmonic mesh extension on the reference configuration
  D X0[4][3], gr0[4][3], Jxi0[3][3];
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) X0[a][i] = X[a][i];
  D det0 = p1_gradients(X0, gr0, Jxi0);
  D vol0 = det0 / 6.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      D kab = vol0 * (gr0[a][0] * gr0[b][0] + gr0[a][1] * gr0[b][1] + gr0[a][2] * gr0[b][2]);
      for (int i = 0; i < 3; ++i) R[a][4 + i] += kab * y[b][4 + i];
    }

  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 7; ++r) R[a][r] = dt * R[a][r];
  return true;
}

// Solid element (total Lagrangian on the reference configuration): rows [4][0..2].
template <class T, class D>
static bool solid_element(const Phys& ph, double dt, const D X[4][3], const T y[4][7],
                          const D yo[4][7], const D f[4][3], T R[4][7]) {
  const double mus = ph.E_s / (2.0 * (1.0 + ph.nu_s));
  const double lams = ph.E_s * ph.nu_s / ((1.0 + ph.nu_s) * (1.0 - 2.0 * ph.nu_s));
  D gr0[4][3], Jxi0[3][3];
  D det0 = p1_gradients(X, gr0, Jxi0);
  D vol0 = det0 / 6.0;
  T F[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = (i == j) ? 1.0 : 0.0;
      for (int a = 0; a < 4; ++a) s += y[a][4 + i] * gr0[a][j];
      F[i][j] = s;
    }
  if (!(val(det3(F)) > 0.0)) return false;
  T E[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = 0.0;
      for (int k = 0; k < 3; ++k) s += F[k][i] * F[k][j];
      E[i][j] = 0.5 * (s - ((i == j) ? 1.0 : 0.0));
    }
  T trE = E[0][0] + E[1][1] + E[2][2];
  T S[3][3], P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) S[i][j] = 2.0 * mus * E[i][j] + ((i == j) ? lams * trE : T(0.0));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = 0.0;
      for (int k = 0; k < 3; ++k) s += F[i][k] * S[k][j];
      P[i][j] = s;
    }
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 7; ++r) R[a][r] = 0.0;
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i)
      R[a][i] = vol0 * (P[i][0] * gr0[a][0] + P[i][1] * gr0[a][1] + P[i][2] * gr0[a][2]);
  for (int q = 0; q < 4; ++q) {
    double lam[4];
    for (int a = 0; a < 4; ++a) lam[a] = (a == q) ? kQa : kQb;
    for (int i = 0; i < 3; ++i) {
      T uq = 0.0;
      D uoq = 0.0, fq = 0.0;
      for (int a = 0; a < 4; ++a) {
        uq += lam[a] * y[a][i];
        uoq += lam[a] * yo[a][i];
        fq += lam[a] * f[a][i];
      }
      T rq = ph.rho_s * (uq - uoq) / dt + ph.eta_s * uq - ph.rho_s * fq;
      for (int a = 0; a < 4; ++a) R[a][i] += (vol0 / 4.0) * lam[a] * rq;
    }
  }
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 7; ++r) R[a][r] = dt * R[a][r];
  return true;
}

template <class T>
static bool element_T(const fsio_solver& s, int e, const T* yv, T R[4][7]) {
  double X[4][3], yo[4][7], f[4][3];
  T y[4][7];
  for (int a = 0; a < 4; ++a) {
    int v = s.tets[4 * e + a];
    for (int i = 0; i < 3; ++i) {
      X[a][i] = s.X[3 * (size_t)v + i];
      f[a][i] = s.bforce.empty() ? 0.0 : s.bforce[3 * (size_t)v + i];
    }
    for (int r = 0; r < 7; ++r) {
      y[a][r] = yv[7 * (size_t)v + r];
      yo[a][r] = s.yold[7 * (size_t)v + r];
    }
  }
  return s.dom[e] == 0 ? fluid_element(s.ph, s.dt, X, y, yo, f, R)
                       : solid_element(s.ph, s.dt, X, y, yo, f, R);
}

// Nodal rows: Dirichlet y - g, dummy pressure p, kinematic (d - d_old) - dt u.
template <class T>
static void nodal_rows(const fsio_solver& s, const T* y, T* F) {
  const size_t n = 7 * (size_t)s.V;
  for (size_t i = 0; i < n; ++i) {
    switch (s.rowkind[i]) {
      case ROW_DIR: F[i] = y[i] - s.gval[i]; break;
      case ROW_DUMMY: F[i] = y[i]; break;
      case ROW_KIN: F[i] = y[i] - s.yold[i] - s.dt * y[i - 4]; break;
      default: break;
    }
  }
}

template <class T>
static int residual_T(fsio_solver& s, const T* y, T* F) {
  const size_t n = 7 * (size_t)s.V;
  for (size_t i = 0; i < n; ++i) F[i] = 0.0;
  T R[4][7];
  for (int e = 0; e < s.E; ++e) {
    if (!element_T(s, e, y, R)) {
      s.err = "inverted element " + std::to_string(e);
      return FSIO_ERR_INVERTED;
    }
    for (int a = 0; a < 4; ++a) {
      size_t v = s.tets[4 * e + a];
      for (int r = 0; r < 7; ++r)
        if (s.rowkind[7 * v + r] == ROW_ELEM) F[7 * v + r] += R[a][r];
    }
  }
  nodal_rows(s, y, F);
  return FSIO_OK;
}

int residual(fsio_solver& s, const double* y, double* F) { return residual_T(s, y, F); }
int residual_complex(fsio_solver& s, const Cplx* y, Cplx* F) { return residual_T(s, y, F); }

// Exact Jacobian (§3: analytically exact, no finite differences).  Each element
// residual is evaluated once with 28 forward-mode tangents, one per element unknown.
static bool element_jac(const fsio_solver& s, int e, const double* yv, double Re[28], double Je[28][28]) {
  double X[4][3], yo[4][7], f[4][3];
  D28 y[4][7], R[4][7];
  for (int a = 0; a < 4; ++a) {
    int v = s.tets[4 * e + a];
    for (int i = 0; i < 3; ++i) {
      X[a][i] = s.X[3 * (size_t)v + i];
      f[a][i] = s.bforce.empty() ? 0.0 : s.bforce[3 * (size_t)v + i];
    }
    for (int r = 0; r < 7; ++r) {
      y[a][r] = D28(yv[7 * (size_t)v + r]);
      y[a][r].d[7 * a + r] = 1.0;
      yo[a][r] = s.yold[7 * (size_t)v + r];
    }
  }
  bool ok = s.dom[e] == 0 ? fluid_element(s.ph, s.dt, X, y, yo, f, R)
                          : solid_element(s.ph, s.dt, X, y, yo, f, R);
  if (!ok) return false;
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 7; ++r) {
      Re[7 * a + r] = R[a][r].v;
      for (int c = 0; c < 28; ++c) Je[7 * a + r][c] = R[a][r].d[c];
    }
  return true;
}

int jacobian(fsio_solver& s, const double* y) {
  std::fill(s.J.vals.begin(), s.J.vals.end(), 0.0);
  double Re[28], Je[28][28];
  for (int e = 0; e < s.E; ++e) {
    if (!element_jac(s, e, y, Re, Je)) {
      s.err = "inverted element " + std::to_string(e);
      return FSIO_ERR_INVERTED;
    }
    for (int a = 0; a < 4; ++a) {
      int va = s.tets[4 * e + a];
      for (int b = 0; b < 4; ++b) {
        int vb = s.tets[4 * e + b];
        double* blk = &s.J.vals[49 * (size_t)s.J.find(va, vb)];
        for (int r = 0; r < 7; ++r) {
          if (s.rowkind[7 * (size_t)va + r] != ROW_ELEM) continue;
          for (int c = 0; c < 7; ++c) blk[7 * r + c] += Je[7 * a + r][7 * b + c];
        }
      }
    }
  }
  for (int v = 0; v < s.V; ++v) {
    double* blk = &s.J.vals[49 * (size_t)s.J.find(v, v)];
    for (int r = 0; r < 7; ++r) {
      switch (s.rowkind[7 * (size_t)v + r]) {
        case ROW_DIR:
        case ROW_DUMMY: blk[7 * r + r] = 1.0; break;
        case ROW_KIN:
          blk[7 * r + r] = 1.0;
          blk[7 * r + (r - 4)] = -s.dt;
          break;
        default: break;
      }
    }
  }
  s.jac_ready = true;
  return FSIO_OK;
}

// Operations of element e's residual at y, counted by the counting scalar: value
// operations (the residual's algorithmic flops) and tangent operations per forward-mode
// direction (what each of the 28 Jacobian columns adds on top of one value pass).
int element_ops(fsio_solver& s, const double* yv, int e, int64_t* value_ops, int64_t* tangent_ops) {
  Fl X[4][3], yo[4][7], f[4][3], y[4][7], R[4][7];
  for (int a = 0; a < 4; ++a) {
    int v = s.tets[4 * e + a];
    for (int i = 0; i < 3; ++i) {
      X[a][i] = Fl(s.X[3 * (size_t)v + i]);
      f[a][i] = Fl(s.bforce.empty() ? 0.0 : s.bforce[3 * (size_t)v + i]);
    }
    for (int r = 0; r < 7; ++r) {
      y[a][r] = Fl(yv[7 * (size_t)v + r], true);
      yo[a][r] = Fl(s.yold[7 * (size_t)v + r]);
    }
  }
  g_ops = OpCount{};
  bool ok = s.dom[e] == 0 ? fluid_element(s.ph, s.dt, X, y, yo, f, R) : solid_element(s.ph, s.dt, X, y, yo, f, R);
  *value_ops = g_ops.value;
  *tangent_ops = g_ops.tangent;
  return ok ? FSIO_OK : FSIO_ERR_INVERTED;
}

int element(fsio_solver& s, const double* y, int e, double* Re, double* Je) {
  double R[28], J[28][28];
  if (!element_jac(s, e, y, R, J)) return FSIO_ERR_INVERTED;
  std::memcpy(Re, R, sizeof(R));
  if (Je) std::memcpy(Je, J, sizeof(J));
  return FSIO_OK;
}

}  // namespace fsio
