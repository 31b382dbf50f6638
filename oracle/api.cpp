// Oracle C entry points (test infrastructure only; see fsio.h).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>

#include "core.hpp"

using namespace fsio;

extern "C" {

int fsio_create(const fsio_mesh* m, const fsio_physics* ph, const fsio_opts* o, fsio_solver** out) {
  if (!m || !ph || !o || !out || m->nverts <= 0 || m->ntets <= 0 || !m->X || !m->tets || !m->tet_domain)
    return FSIO_ERR_ARG;
  if (o->nsub <= 0 || o->overlap < 0 || o->gmres_restart <= 0 || o->gmres_restart > 200) return FSIO_ERR_ARG;
  if (o->ilu_level < 0 || o->ilu_level > 8) return FSIO_ERR_ARG;
  if (o->ordering != 0 && o->ordering != 1) return FSIO_ERR_ARG;  // RCM, 1WD
  fsio_solver* s = new (std::nothrow) fsio_solver();
  if (!s) return FSIO_ERR_OOM;
  s->V = m->nverts;
  s->E = m->ntets;
  s->B = m->nbfaces;
  s->X.assign(m->X, m->X + 3 * (size_t)s->V);
  s->tets.assign(m->tets, m->tets + 4 * (size_t)s->E);
  s->dom.assign(m->tet_domain, m->tet_domain + s->E);
  if (s->B > 0) {
    s->bfaces.assign(m->bfaces, m->bfaces + 3 * (size_t)s->B);
    s->btag.assign(m->bface_tag, m->bface_tag + s->B);
  }
  for (int v : s->tets)
    if (v < 0 || v >= s->V) { delete s; return FSIO_ERR_MESH; }
  for (int v : s->bfaces)
    if (v < 0 || v >= s->V) { delete s; return FSIO_ERR_MESH; }
  s->ph = Phys{ph->rho_f, ph->mu_f, ph->rho_s, ph->E_s, ph->nu_s, ph->eta_s, ph->C_I};
  s->opts = *o;
  s->opts.part = nullptr;
  int rc = build_topology(*s);
  if (rc) { delete s; return rc; }
  if (o->part) {
    s->part.assign(o->part, o->part + s->V);
    for (int p : s->part)
      if (p < 0 || p >= o->nsub) { delete s; return FSIO_ERR_ARG; }
  } else {
    rcb_partition(*s, o->nsub, s->part);
  }
  rc = build_subdomains(*s);
  if (rc) { delete s; return rc; }
  s->yold.assign(7 * (size_t)s->V, 0.0);
  s->gval.assign(7 * (size_t)s->V, 0.0);
  s->rowkind = s->rowkind_base;
  *out = s;
  return FSIO_OK;
}

int fsio_destroy(fsio_solver* s) {
  delete s;
  return FSIO_OK;
}

int fsio_sizes(const fsio_solver* s, int64_t* n, int64_t* nnzb) {
  if (!s) return FSIO_ERR_ARG;
  if (n) *n = 7 * (int64_t)s->V;
  if (nnzb) *nnzb = (int64_t)s->J.colind.size();
  return FSIO_OK;
}

const char* fsio_last_error(const fsio_solver* s) { return s ? s->err.c_str() : "null solver"; }

int fsio_set_step(fsio_solver* s, double t_n, double dt, const double* y_old, const double* g,
                  const double* bf, const uint8_t* extra_mask) {
  if (!s || !y_old || !g || !(dt > 0.0)) return FSIO_ERR_ARG;
  const size_t n = 7 * (size_t)s->V;
  s->t = t_n;
  s->dt = dt;
  s->yold.assign(y_old, y_old + n);
  set_rowkinds(*s, extra_mask);
  s->gval.assign(n, 0.0);
  for (size_t i = 0; i < n; ++i) s->gval[i] = s->forced_zero[i] ? 0.0 : g[i];
  if (bf) s->bforce.assign(bf, bf + 3 * (size_t)s->V);
  else s->bforce.clear();
  s->has_step = true;
  s->jac_ready = false;
  s->pc_ready = false;
  return FSIO_OK;
}

int fsio_impose_dirichlet(fsio_solver* s, double* y) {
  if (!s || !y || !s->has_step) return FSIO_ERR_ARG;
  for (size_t i = 0; i < s->rowkind.size(); ++i) {
    if (s->rowkind[i] == ROW_DIR) y[i] = s->gval[i];
    if (s->rowkind[i] == ROW_DUMMY) y[i] = 0.0;
  }
  return FSIO_OK;
}

int fsio_residual(fsio_solver* s, const double* y, double* F) {
  if (!s || !y || !F || !s->has_step) return FSIO_ERR_ARG;
  return residual(*s, y, F);
}

int fsio_residual_complex(fsio_solver* s, const double* yr, const double* yi, double* Fr, double* Fi) {
  if (!s || !yr || !yi || !Fr || !Fi || !s->has_step) return FSIO_ERR_ARG;
  const size_t n = 7 * (size_t)s->V;
  std::vector<Cplx> y(n), F(n);
  for (size_t i = 0; i < n; ++i) y[i] = Cplx(yr[i], yi[i]);
  int rc = residual_complex(*s, y.data(), F.data());
  for (size_t i = 0; i < n; ++i) { Fr[i] = F[i].real(); Fi[i] = F[i].imag(); }
  return rc;
}

int fsio_jacobian(fsio_solver* s, const double* y) {
  if (!s || !y || !s->has_step) return FSIO_ERR_ARG;
  return jacobian(*s, y);
}

int fsio_jacobian_get(const fsio_solver* s, int32_t* rowptr, int32_t* colind, double* vals) {
  if (!s) return FSIO_ERR_ARG;
  if (rowptr) std::copy(s->J.rowptr.begin(), s->J.rowptr.end(), rowptr);
  if (colind) std::copy(s->J.colind.begin(), s->J.colind.end(), colind);
  if (vals) std::copy(s->J.vals.begin(), s->J.vals.end(), vals);
  return FSIO_OK;
}

int fsio_jacobian_set(fsio_solver* s, const double* vals) {
  if (!s || !vals) return FSIO_ERR_ARG;
  std::copy(vals, vals + s->J.vals.size(), s->J.vals.begin());
  s->jac_ready = true;
  return FSIO_OK;
}

int fsio_spmv(fsio_solver* s, const double* x, double* y) {
  if (!s || !x || !y || !s->jac_ready) return FSIO_ERR_ARG;
  spmv(*s, x, y);
  return FSIO_OK;
}

int fsio_pc_setup(fsio_solver* s) {
  if (!s) return FSIO_ERR_ARG;
  return pc_setup(*s);
}

int fsio_pc_apply(fsio_solver* s, const double* v, double* z) {
  if (!s || !v || !z || !s->pc_ready) return FSIO_ERR_ARG;
  pc_apply(*s, v, z);
  return FSIO_OK;
}

int fsio_gmres(fsio_solver* s, const double* rhs, double* x, fsio_lin_stats* st) {
  if (!s || !rhs || !x || !s->pc_ready) return FSIO_ERR_ARG;
  return gmres(*s, rhs, x, st, nullptr);
}

int fsio_newton_solve(fsio_solver* s, double* y, fsio_step_stats* st) {
  if (!s || !y || !s->has_step) return FSIO_ERR_ARG;
  return newton(*s, y, st);
}

int fsio_topology_get(const fsio_solver* s, int8_t* vkind, uint8_t* rowkind, int32_t* n_iface,
                      int32_t* iface_faces) {
  if (!s) return FSIO_ERR_ARG;
  if (vkind) std::copy(s->vkind.begin(), s->vkind.end(), vkind);
  if (rowkind) std::copy(s->rowkind.begin(), s->rowkind.end(), rowkind);
  if (n_iface) *n_iface = (int32_t)(s->iface_faces.size() / 3);
  if (iface_faces) std::copy(s->iface_faces.begin(), s->iface_faces.end(), iface_faces);
  return FSIO_OK;
}

int fsio_pc_sizes(const fsio_solver* s, int32_t* nsub, int64_t* nrows, int64_t* nblocks, int64_t* nlev) {
  if (!s) return FSIO_ERR_ARG;
  int64_t r = 0, b = 0, l = 0;
  for (const Sub& S : s->subs) { r += S.verts.size(); b += S.colind.size(); l += S.nlevels; }
  if (nsub) *nsub = (int32_t)s->subs.size();
  if (nrows) *nrows = r;
  if (nblocks) *nblocks = b;
  if (nlev) *nlev = l;
  return FSIO_OK;
}

int fsio_pc_get(const fsio_solver* s, int32_t* part, int32_t* sub_ptr, int32_t* sub_verts,
                int32_t* sub_nowned, int64_t* blk_ptr, int32_t* lrowptr, int32_t* lcolind,
                double* factors, double* udiag) {
  if (!s) return FSIO_ERR_ARG;
  if (part) std::copy(s->part.begin(), s->part.end(), part);
  int64_t vo = 0, bo = 0, ro = 0;
  for (size_t i = 0; i < s->subs.size(); ++i) {
    const Sub& S = s->subs[i];
    if (sub_ptr) { sub_ptr[i] = (int32_t)vo; sub_ptr[i + 1] = (int32_t)(vo + S.verts.size()); }
    if (blk_ptr) { blk_ptr[i] = bo; blk_ptr[i + 1] = bo + (int64_t)S.colind.size(); }
    if (sub_verts) std::copy(S.verts.begin(), S.verts.end(), sub_verts + vo);
    if (sub_nowned) sub_nowned[i] = S.nowned;
    if (lrowptr) std::copy(S.rowptr.begin(), S.rowptr.end(), lrowptr + ro);
    if (lcolind) std::copy(S.colind.begin(), S.colind.end(), lcolind + bo);
    if (factors && s->pc_ready) std::copy(S.f.begin(), S.f.end(), factors + 49 * bo);
    if (udiag && s->pc_ready) std::copy(S.udiag.begin(), S.udiag.end(), udiag + 49 * vo);
    vo += (int64_t)S.verts.size();
    bo += (int64_t)S.colind.size();
    ro += (int64_t)S.verts.size() + 1;
  }
  return FSIO_OK;
}

int fsio_element(fsio_solver* s, const double* y, int32_t e, double* Re, double* Je) {
  if (!s || !y || !Re || e < 0 || e >= s->E || !s->has_step) return FSIO_ERR_ARG;
  return element(*s, y, e, Re, Je);
}

int fsio_element_ops(fsio_solver* s, const double* y, int32_t e, int64_t* value_ops, int64_t* tangent_ops) {
  if (!s || !y || !value_ops || !tangent_ops || e < 0 || e >= s->E || !s->has_step) return FSIO_ERR_ARG;
  return element_ops(*s, y, e, value_ops, tangent_ops);
}

}  // extern "C"
