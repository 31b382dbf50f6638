// Oracle: right-preconditioned restarted GMRES and the inexact Newton loop with
// backtracking (test infrastructure only).
//
// Paper §3: Newton update y <- y + alpha dy (eq. (11)) with a backtracking line search,
// dy from J dy = -F (eq. (12)), the Jacobian possibly from an earlier iterate; GMRES
// on the Schwarz-preconditioned system (eq. (13); the paper notes the preconditioner may
// be applied from the right, which is the reading taken here).  §4: Newton relative
// tolerance 1e-6, GMRES relative tolerance 1e-3.
//
// GMRES: x0 = 0, classical Gram-Schmidt applied twice, Givens rotations
// rho = hypot(a, b), c = a/rho, s = b/rho, happy breakdown when h_{j+1,j} <= 1e-14 ||h||,
// stop when |g_{j+1}| <= rtol ||b||; at the end of a cycle x += B^{-1}(V y) and the true
// residual restarts the next cycle.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "core.hpp"

namespace fsio {

static double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static double nrm2(const std::vector<double>& v) {
  double s = 0.0;
  for (double x : v) s += x * x;
  return std::sqrt(s);
}

int gmres(fsio_solver& s, const double* b, double* x, fsio_lin_stats* st, double* t_pcapply) {
  const size_t n = 7 * (size_t)s.V;
  const int m = s.opts.gmres_restart;
  const int maxit = s.opts.gmres_maxit;
  std::vector<double> bb(b, b + n);
  for (size_t i = 0; i < n; ++i) x[i] = 0.0;
  const double bnorm = nrm2(bb);
  fsio_lin_stats loc{};
  loc.rnorm0 = bnorm;
  if (bnorm == 0.0) {
    loc.converged = 1;
    if (st) *st = loc;
    return FSIO_OK;
  }
  const double target = s.opts.gmres_rtol * bnorm;
  std::vector<std::vector<double>> Vb(m + 1, std::vector<double>(n));
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), w(n), z(n), r = bb;
  auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  int its = 0;
  bool done = false;
  while (!done) {
    double beta = nrm2(r);
    for (size_t i = 0; i < n; ++i) Vb[0][i] = r[i] / beta;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = -1;
    for (int j = 0; j < m; ++j) {
      double t0 = now();
      pc_apply(s, Vb[j].data(), z.data());
      if (t_pcapply) *t_pcapply += now() - t0;
      spmv(s, z.data(), w.data());
      std::vector<double> h(j + 1, 0.0), h2(j + 1, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<double>& hp = pass == 0 ? h : h2;
        for (int i = 0; i <= j; ++i) {
          double d = 0.0;
          for (size_t k = 0; k < n; ++k) d += Vb[i][k] * w[k];
          hp[i] = d;
        }
        for (int i = 0; i <= j; ++i)
          for (size_t k = 0; k < n; ++k) w[k] -= hp[i] * Vb[i][k];
      }
      double hn2 = 0.0;
      for (int i = 0; i <= j; ++i) {
        h[i] += h2[i];
        hn2 += h[i] * h[i];
      }
      double hn = nrm2(w);
      for (int i = 0; i <= j; ++i) Hij(i, j) = h[i];
      Hij(j + 1, j) = hn;
      bool breakdown = hn <= 1e-14 * std::sqrt(hn2 + hn * hn);
      for (int i = 0; i < j; ++i) {
        double a = Hij(i, j), bq = Hij(i + 1, j);
        Hij(i, j) = cs[i] * a + sn[i] * bq;
        Hij(i + 1, j) = -sn[i] * a + cs[i] * bq;
      }
      double a = Hij(j, j), bq = Hij(j + 1, j);
      double rho = std::hypot(a, bq);
      cs[j] = a / rho;
      sn[j] = bq / rho;
      Hij(j, j) = rho;
      Hij(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      its++;
      if (!breakdown)
        for (size_t k = 0; k < n; ++k) Vb[j + 1][k] = w[k] / hn;
      loc.rnorm_est = std::fabs(g[j + 1]);
      jend = j;
      if (loc.rnorm_est <= target) { loc.converged = 1; done = true; break; }
      if (breakdown || its >= maxit) { done = true; break; }
    }
    // back substitution and the preconditioned update x += B^{-1} V y
    std::vector<double> yv(jend + 1);
    for (int i = jend; i >= 0; --i) {
      double sacc = g[i];
      for (int k = i + 1; k <= jend; ++k) sacc -= Hij(i, k) * yv[k];
      yv[i] = sacc / Hij(i, i);
    }
    std::fill(w.begin(), w.end(), 0.0);
    for (int i = 0; i <= jend; ++i)
      for (size_t k = 0; k < n; ++k) w[k] += yv[i] * Vb[i][k];
    double t0 = now();
    pc_apply(s, w.data(), z.data());
    if (t_pcapply) *t_pcapply += now() - t0;
    for (size_t k = 0; k < n; ++k) x[k] += z[k];
    if (!done) {
      loc.restarts++;
      spmv(s, x, w.data());
      for (size_t k = 0; k < n; ++k) r[k] = bb[k] - w[k];
    }
  }
  spmv(s, x, w.data());
  for (size_t k = 0; k < n; ++k) w[k] = bb[k] - w[k];
  loc.rnorm_true = nrm2(w);
  loc.iters = its;
  if (st) *st = loc;
  return FSIO_OK;
}

// Inexact Newton with backtracking (eqs. (11)-(12)); Armijo constant ls_c, halving,
// at most ls_max_halvings cuts; an inverted element rejects the trial step.
int newton(fsio_solver& s, double* y, fsio_step_stats* st) {
  const size_t n = 7 * (size_t)s.V;
  fsio_step_stats S;
  std::memset(&S, 0, sizeof(S));
  for (size_t i = 0; i < n; ++i) {  // step setup: Dirichlet values and dummy pressures
    if (s.rowkind[i] == ROW_DIR) y[i] = s.gval[i];
    if (s.rowkind[i] == ROW_DUMMY) y[i] = 0.0;
  }
  std::vector<double> F(n), Ft(n), yt(n), dy(n), rhs(n);
  double t0 = now();
  int rc = residual(s, y, F.data());
  S.t_funceval += now() - t0;
  if (rc) { if (st) *st = S; return rc; }
  double f0 = nrm2(F), fk = f0;
  S.fnorm0 = f0;
  S.fnorm_hist[0] = f0;
  int k = 0;
  int status = FSIO_OK;
  while (true) {
    if (fk <= std::max(s.opts.newton_rtol * f0, s.opts.newton_atol)) { S.converged = 1; break; }
    if (k >= s.opts.newton_maxit) { status = FSIO_ERR_DIVERGED; s.err = "newton maxit"; break; }
    if (k % std::max(1, s.opts.jac_lag) == 0) {
      t0 = now();
      rc = jacobian(s, y);
      S.t_jaceval += now() - t0;
      if (rc) { status = rc; break; }
      t0 = now();
      rc = pc_setup(s);
      S.t_pcsetup += now() - t0;
      if (rc) { status = rc; break; }
    }
    for (size_t i = 0; i < n; ++i) rhs[i] = -F[i];
    fsio_lin_stats ls{};
    t0 = now();
    double tpa = 0.0;
    gmres(s, rhs.data(), dy.data(), &ls, &tpa);
    S.t_kspsolve += now() - t0;
    S.t_pcapply += tpa;
    S.linear_iters += ls.iters;
    if (k < FSIO_MAX_NEWTON) S.lin_hist[k] = ls.iters;
    double alpha = 1.0;
    bool accepted = false;
    for (int h = 0; h <= s.opts.ls_max_halvings; ++h) {
      for (size_t i = 0; i < n; ++i) yt[i] = y[i] + alpha * dy[i];
      t0 = now();
      rc = residual(s, yt.data(), Ft.data());
      S.t_funceval += now() - t0;
      if (rc == FSIO_OK) {
        double ft = nrm2(Ft);
        if (ft <= (1.0 - s.opts.ls_c * alpha) * fk) {
          accepted = true;
          fk = ft;
          break;
        }
      }
      alpha *= 0.5;
      S.line_search_cuts++;
    }
    if (!accepted) { status = FSIO_ERR_DIVERGED; s.err = "line search failed"; break; }
    std::memcpy(y, yt.data(), n * sizeof(double));
    F.swap(Ft);
    k++;
    if (k < FSIO_MAX_NEWTON) { S.fnorm_hist[k] = fk; S.alpha_hist[k - 1] = alpha; }
  }
  S.newton_iters = k;
  S.fnorm = fk;
  if (st) *st = S;
  return status;
}

}  // namespace fsio
