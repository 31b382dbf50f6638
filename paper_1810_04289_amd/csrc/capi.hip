// C ABI of the HIP FSI library (declared in include/fsi.h): solver lifetime, uploads,
// the host drivers of GMRES and Newton, introspection and kernel timing.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

#include "fsi_internal.hpp"

using namespace fsi;

// Scratch of the allocation-free Schwarz application (fsi_pc_apply_noalloc): a file-scope
// device array, one copy on every GPU the library runs on, held until the process ends.
// Its first 256 bytes hold the sweeps' four error flags, the rest the forward sweep's
// values (7 per local row, FP64 or FP32), up to kScratchYBytes.  Host code reaches a
// GPU's copy only through the address hipGetSymbolAddress returns on that GPU; the
// array's name in host code is a stand-in, not a device address.
constexpr size_t kScratchFlagBytes = 256;
constexpr size_t kScratchYBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kScratchFlagBytes + kScratchYBytes];

namespace {

struct ScratchAddr {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
constexpr int kMaxDevices = 64;
ScratchAddr g_scratch[kMaxDevices];

// With the solver's device current: the address of that device's scratch, looked up once
// per device.
void scratch_attach(fsi_solver* s) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    s->scratch_err = e != hipSuccess ? e : hipErrorInvalidDevice;
    return;
  }
  ScratchAddr& a = g_scratch[dev];
  std::call_once(a.once, [&a] { a.err = hipGetSymbolAddress(&a.ptr, HIP_SYMBOL(scratch)); });
  s->scratch_err = a.err;
  s->scratch = a.err == hipSuccess ? (char*)a.ptr : nullptr;
}

// clears n int32 (a kernel, not a memset, so that the call can be captured in a graph)
__global__ void k_zero_i32(int32_t* p, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = 0;
}

struct Fail {
  fsi_status st;
};

inline void hip_ok(fsi_solver* s, hipError_t e, const char* what) {
  if (e != hipSuccess) {
    s->err = std::string(what) + ": " + hipGetErrorString(e);
    throw Fail{e == hipErrorOutOfMemory ? FSI_ERR_OOM : FSI_ERR_HIP};
  }
}

template <class T>
T* dalloc(fsi_solver* s, size_t count) {
  if (count == 0) count = 1;
  void* p = nullptr;
  hip_ok(s, hipMalloc(&p, count * sizeof(T)), "hipMalloc");
  s->allocs.push_back(p);
  return (T*)p;
}

template <class T>
T* upload(fsi_solver* s, const std::vector<T>& v) {
  T* p = dalloc<T>(s, v.size());
  if (!v.empty()) hip_ok(s, hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "upload");
  return p;
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void sync(fsi_solver* s) { hip_ok(s, hipStreamSynchronize(s->stream), "stream sync"); }

// ||a||_2 (deterministic reduction), read back to the host
double norm2(fsi_solver* s, const double* a) {
  hip_ok(s, launch_dot_partial(s, a, a, s->n, s->hdev + 3 * (kMaxRestart + 8)), "dot");
  hip_ok(s, hipMemcpyAsync(s->pinned, s->hdev + 3 * (kMaxRestart + 8), sizeof(double), hipMemcpyDeviceToHost,
                           s->stream), "readback");
  sync(s);
  return std::sqrt(s->pinned[0]);
}

void clear_flags(fsi_solver* s) {
  hip_ok(s, hipMemsetAsync(s->flags, 0, kFlags * sizeof(int32_t), s->stream), "memset flags");
}

// the sweeps' flag alone, before the calls that report it (so that an earlier call's
// error does not carry over)
void clear_sweep_flag(fsi_solver* s) {
  hip_ok(s, hipMemsetAsync(s->flags + 3, 0, sizeof(int32_t), s->stream), "memset flag");
}

// the four device flags: [0] inverted element, [1] zero pivot, [2] factorization wait bound,
// [3] sweep wait bound
void read_flags(fsi_solver* s, int32_t out[kFlags]) {
  hip_ok(s, hipMemcpyAsync(&s->pinned[200], s->flags, kFlags * sizeof(int32_t), hipMemcpyDeviceToHost, s->stream),
         "flag readback");
  sync(s);
  std::memcpy(out, &s->pinned[200], kFlags * sizeof(int32_t));
}

int32_t read_flag(fsi_solver* s, int which) {
  int32_t v[kFlags];
  read_flags(s, v);
  return v[which];
}

fsi_status residual_impl(fsi_solver* s, const double* y, double* F) {
  clear_flags(s);
  hip_ok(s, launch_residual(s, y, F), "residual");
  if (read_flag(s, 0)) {
    s->err = "inverted element";
    return FSI_ERR_INVERTED;
  }
  return FSI_OK;
}

fsi_status jacobian_impl(fsi_solver* s, const double* y) {
  clear_flags(s);
  hip_ok(s, launch_jacobian(s, y), "jacobian");
  if (read_flag(s, 0)) {
    s->err = "inverted element";
    return FSI_ERR_INVERTED;
  }
  s->jac_ready = true;
  s->pc_ready = false;
  return FSI_OK;
}

fsi_status pc_setup_impl(fsi_solver* s) {
  if (!s->jac_ready) {
    s->err = "pc_setup before jacobian";
    return FSI_ERR_ARG;
  }
  s->pc_ready = false;  // until these factors are known good
  clear_flags(s);
  hip_ok(s, launch_pc_setup(s), "pc_setup");
  hip_ok(s, launch_fac_round(s), "factor rounding");
  int32_t f[kFlags];
  read_flags(s, f);
  if (f[2]) {
    s->err = "a subdomain factorization waited on a pivot row beyond its bound";
    return FSI_ERR_HIP;
  }
  if (f[1]) {
    // the first and the last local row whose pivot block was singular, and their number
    const auto& off = s->h.sub_row_off;
    auto where = [&](int64_t r) {
      const int64_t sd = (int64_t)(std::upper_bound(off.begin(), off.end(), (int32_t)r) - off.begin()) - 1;
      if (r < 0 || sd < 0 || r >= (int64_t)s->h.lglob.size()) return std::string("?");
      return "subdomain " + std::to_string(sd) + ", local row " + std::to_string(r - off[sd]) + " (vertex " +
             std::to_string(s->h.lglob[r]) + ")";
    };
    s->err = "zero pivot in a subdomain factorization: " + std::to_string(f[6]) + " singular pivot blocks, first at " +
             where(0x7fffffff - (int64_t)f[5]) + ", last at " + where((int64_t)f[4] - 1);
    return FSI_ERR_ZERO_PIVOT;
  }
  s->pc_ready = true;
  return FSI_OK;
}

// Right-preconditioned restarted GMRES (§3 eq. (13)); classical Gram-Schmidt applied twice,
// Givens rotations rho = hypot(a,b), c = a/rho, s = b/rho; happy breakdown when
// h_{j+1,j} <= 1e-14 ||h||; stop when |g_{j+1}| <= rtol ||b||.
// t_pc (may be null) accumulates the preconditioner's time, t_setup (may be null) the
// solve's set-up before its first Arnoldi step (the paper's KSPSetUp).
fsi_status gmres_impl(fsi_solver* s, const double* b, double* x, fsi_lin_stats* st, double* t_pc,
                      double* t_setup) {
  const double ts0 = now();
  const int64_t n = s->n;
  const int m = s->opts.gmres_restart, maxit = s->opts.gmres_maxit;
  fsi_lin_stats L{};
  clear_sweep_flag(s);
  hip_ok(s, hipMemsetAsync(x, 0, n * sizeof(double), s->stream), "memset x");
  const double bnorm = norm2(s, b);
  L.rnorm0 = bnorm;
  if (bnorm == 0.0) {
    L.converged = 1;
    if (st) *st = L;
    if (t_setup) *t_setup += now() - ts0;
    return FSI_OK;
  }
  const double target = s->opts.gmres_rtol * bnorm;
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), yv(m + 1);
  auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  double* hA = s->hdev;                      // first Gram-Schmidt pass
  double* hB = s->hdev + (kMaxRestart + 8);  // second pass
  double* hn2 = s->hdev + 2 * (kMaxRestart + 8);
  hip_ok(s, hipMemcpyAsync(s->r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s->stream), "copy b");
  int its = 0;
  bool done = false;
  hipEvent_t e0, e1;
  hip_ok(s, hipEventCreate(&e0), "event");
  hip_ok(s, hipEventCreate(&e1), "event");
  if (t_setup) *t_setup += now() - ts0;
  // the preconditioner is bracketed by events; its time is read after the iteration's
  // own synchronization (no extra host wait between the sweeps and the SpMV)
  bool pc_timed = false;
  auto timed_pc = [&](const double* v, double* zz) {
    hip_ok(s, hipEventRecord(e0, s->stream), "event");
    hip_ok(s, launch_pc_apply(s, v, zz), "pc_apply");
    hip_ok(s, hipEventRecord(e1, s->stream), "event");
    pc_timed = true;
  };
  auto add_pc_time = [&]() {
    if (!pc_timed) return;
    float ms = 0.f;
    hip_ok(s, hipEventSynchronize(e1), "event");
    hip_ok(s, hipEventElapsedTime(&ms, e0, e1), "event");
    if (t_pc) *t_pc += ms * 1e-3;
    pc_timed = false;
  };
  // One Arnoldi step: z = B^-1 V_j, w = J z, two classical Gram-Schmidt passes against
  // V_0..V_j (coefficients to hA, hB) and |w|^2 to hn2.  Eagerly, or as the graph captured
  // for this j on its first use (same kernels, same order: the same results).  The
  // preconditioner's own time is measured only when run eagerly.
  auto arnoldi_kernels = [&](int j) -> hipError_t {
    hipError_t e = launch_pc_apply(s, s->Vb + (size_t)j * n, s->z);
    if (e == hipSuccess) e = launch_spmv(s, s->z, s->w);
    if (e == hipSuccess) e = launch_mdot(s, s->Vb, j + 1, s->w, n, hA);
    if (e == hipSuccess) e = launch_vupdate_mdot(s, s->Vb, j + 1, hA, s->w, n, hB);
    if (e == hipSuccess) e = launch_vupdate_sqnorm(s, s->Vb, j + 1, hB, s->w, n, hn2);
    return e;
  };
  auto arnoldi_step = [&](int j) {
    if (!s->graphs || s->prof) {
      timed_pc(s->Vb + (size_t)j * n, s->z);
      hip_ok(s, launch_spmv(s, s->z, s->w), "spmv");
      hip_ok(s, launch_mdot(s, s->Vb, j + 1, s->w, n, hA), "mdot");
      hip_ok(s, launch_vupdate_mdot(s, s->Vb, j + 1, hA, s->w, n, hB), "vupdate+mdot");
      hip_ok(s, launch_vupdate_sqnorm(s, s->Vb, j + 1, hB, s->w, n, hn2), "vupdate+norm");
      return;
    }
    if (!s->arnoldi[j]) {
      // captured on a private stream (the solver's may be the legacy default stream, which
      // cannot capture); the graph is then launched on the solver's stream
      if (!s->cap_stream)
        hip_ok(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking), "capture stream");
      hipGraph_t g = nullptr;
      hipStream_t keep = s->stream;
      s->stream = s->cap_stream;
      const hipError_t eb = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
      const hipError_t e = eb == hipSuccess ? arnoldi_kernels(j) : hipSuccess;
      const hipError_t ec = eb == hipSuccess ? hipStreamEndCapture(s->stream, &g) : hipSuccess;
      s->stream = keep;
      hip_ok(s, eb, "begin capture");
      hip_ok(s, e, "captured Arnoldi step");
      hip_ok(s, ec, "end capture");
      const hipError_t ei = hipGraphInstantiate(&s->arnoldi[j], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) s->arnoldi[j] = nullptr;
      hip_ok(s, ei, "instantiate");
    }
    hip_ok(s, hipGraphLaunch(s->arnoldi[j], s->stream), "graph launch");
  };
  while (!done) {
    const double beta = norm2(s, s->r);
    hip_ok(s, launch_scale(s, 1.0 / beta, s->r, s->Vb, n), "scale");
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = -1;
    for (int j = 0; j < m; ++j) {
      arnoldi_step(j);
      hip_ok(s, hipMemcpyAsync(s->pinned, s->hdev, 3 * (kMaxRestart + 8) * sizeof(double), hipMemcpyDeviceToHost,
                               s->stream), "h readback");
      sync(s);
      add_pc_time();
      const double* ha = s->pinned;
      const double* hb = s->pinned + (kMaxRestart + 8);
      double hsum2 = 0.0;
      for (int i = 0; i <= j; ++i) {
        Hij(i, j) = ha[i] + hb[i];
        hsum2 += Hij(i, j) * Hij(i, j);
      }
      const double hn = std::sqrt(s->pinned[2 * (kMaxRestart + 8)]);
      Hij(j + 1, j) = hn;
      const bool breakdown = hn <= 1e-14 * std::sqrt(hsum2 + hn * hn);
      for (int i = 0; i < j; ++i) {
        const double a = Hij(i, j), bq = Hij(i + 1, j);
        Hij(i, j) = cs[i] * a + sn[i] * bq;
        Hij(i + 1, j) = -sn[i] * a + cs[i] * bq;
      }
      const double a = Hij(j, j), bq = Hij(j + 1, j);
      const double rho = std::hypot(a, bq);
      cs[j] = a / rho;
      sn[j] = bq / rho;
      Hij(j, j) = rho;
      Hij(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      if (!breakdown) hip_ok(s, launch_scale(s, 1.0 / hn, s->w, s->Vb + (size_t)(j + 1) * n, n), "scale");
      L.rnorm_est = std::fabs(g[j + 1]);
      jend = j;
      if (L.rnorm_est <= target) {
        L.converged = 1;
        done = true;
        break;
      }
      if (breakdown || its >= maxit) {
        done = true;
        break;
      }
    }
    for (int i = jend; i >= 0; --i) {
      double acc = g[i];
      for (int k = i + 1; k <= jend; ++k) acc -= Hij(i, k) * yv[k];
      yv[i] = acc / Hij(i, i);
    }
    std::memcpy(s->pinned, yv.data(), (jend + 1) * sizeof(double));
    hip_ok(s, hipMemcpyAsync(s->yvdev, s->pinned, (jend + 1) * sizeof(double), hipMemcpyHostToDevice, s->stream),
           "y upload");
    hip_ok(s, launch_vcombine(s, s->Vb, jend + 1, s->yvdev, s->tmp, n), "vcombine");
    timed_pc(s->tmp, s->z);
    hip_ok(s, launch_axpby(s, 1.0, x, 1.0, s->z, x, n), "axpby");
    if (!done) {
      ++L.restarts;
      hip_ok(s, launch_spmv(s, x, s->w), "spmv");
      hip_ok(s, launch_axpby(s, 1.0, b, -1.0, s->w, s->r, n), "axpby");
    }
    add_pc_time();
  }
  hip_ok(s, launch_spmv(s, x, s->w), "spmv");
  hip_ok(s, launch_axpby(s, 1.0, b, -1.0, s->w, s->w, n), "axpby");
  L.rnorm_true = norm2(s, s->w);
  L.iters = its;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) *st = L;
  if (read_flag(s, 3)) {
    s->err = "a Schwarz sweep waited on a row beyond its bound";
    return FSI_ERR_HIP;
  }
  return FSI_OK;
}

// Inexact Newton with backtracking (§3 eqs. (11)-(12)).
fsi_status newton_impl(fsi_solver* s, double* y, fsi_step_stats* st) {
  const int64_t n = s->n;
  fsi_step_stats S;
  std::memset(&S, 0, sizeof(S));
  hip_ok(s, launch_impose(s, y), "impose");
  double t0 = now();
  fsi_status rc = residual_impl(s, y, s->F);
  S.t_funceval += now() - t0;
  if (rc) {
    if (st) *st = S;
    return rc;
  }
  const double f0 = norm2(s, s->F);
  double fk = f0;
  S.fnorm0 = f0;
  S.fnorm_hist[0] = f0;
  int k = 0;
  fsi_status status = FSI_OK;
  for (;;) {
    if (fk <= std::max(s->opts.newton_rtol * f0, s->opts.newton_atol)) {
      S.converged = 1;
      break;
    }
    if (k >= s->opts.newton_maxit) {
      status = FSI_ERR_DIVERGED;
      s->err = "Newton iteration limit reached";
      break;
    }
    if (k % std::max(1, s->opts.jac_lag) == 0) {
      t0 = now();
      rc = jacobian_impl(s, y);
      S.t_jaceval += now() - t0;
      if (rc) {
        status = rc;
        break;
      }
      t0 = now();
      rc = pc_setup_impl(s);
      sync(s);
      S.t_pcsetup += now() - t0;
      if (rc) {
        status = rc;
        break;
      }
    }
    hip_ok(s, launch_scale(s, -1.0, s->F, s->rhs, n), "negate");
    fsi_lin_stats ls{};
    t0 = now();
    double tpc = 0.0;
    const fsi_status lrc = gmres_impl(s, s->rhs, s->dy, &ls, &tpc, &S.t_kspsetup);
    S.t_kspsolve += now() - t0;
    if (lrc != FSI_OK) {
      status = lrc;
      break;
    }
    S.t_pcapply += tpc;
    S.linear_iters += ls.iters;
    if (k < FSI_MAX_NEWTON) S.lin_hist[k] = ls.iters;
    double alpha = 1.0;
    bool accepted = false;
    for (int hcut = 0; hcut <= s->opts.ls_max_halvings; ++hcut) {
      hip_ok(s, launch_axpby(s, 1.0, y, alpha, s->dy, s->yt, n), "trial");
      t0 = now();
      rc = residual_impl(s, s->yt, s->Ft);
      if (rc == FSI_OK) {
        const double ft = norm2(s, s->Ft);
        S.t_funceval += now() - t0;
        if (ft <= (1.0 - s->opts.ls_c * alpha) * fk) {
          accepted = true;
          fk = ft;
          break;
        }
      } else {
        S.t_funceval += now() - t0;
      }
      alpha *= 0.5;
      S.line_search_cuts++;
    }
    if (!accepted) {
      status = FSI_ERR_DIVERGED;
      s->err = "line search failed";
      break;
    }
    hip_ok(s, hipMemcpyAsync(y, s->yt, n * sizeof(double), hipMemcpyDeviceToDevice, s->stream), "accept");
    std::swap(s->F, s->Ft);
    ++k;
    if (k < FSI_MAX_NEWTON) {
      S.fnorm_hist[k] = fk;
      S.alpha_hist[k - 1] = alpha;
    }
  }
  sync(s);
  S.newton_iters = k;
  S.fnorm = fk;
  if (st) *st = S;
  return status;
}

fsi_status create_impl(const fsi_mesh* m, const fsi_physics* ph, const fsi_opts* o, void* stream, fsi_solver* s) {
  HostSetup& h = s->h;
  h.V = m->nverts;
  h.E = m->ntets;
  h.B = m->nbfaces;
  h.X.assign(m->X, m->X + 3 * (size_t)h.V);
  h.tets.assign(m->tets, m->tets + 4 * (size_t)h.E);
  h.dom.assign(m->tet_domain, m->tet_domain + h.E);
  if (h.B > 0) {
    h.bfaces.assign(m->bfaces, m->bfaces + 3 * (size_t)h.B);
    h.btag.assign(m->bface_tag, m->bface_tag + h.B);
  }
  for (int32_t v : h.tets)
    if (v < 0 || v >= h.V) {
      s->err = "tet index out of range";
      return FSI_ERR_MESH;
    }
  for (int32_t v : h.bfaces)
    if (v < 0 || v >= h.V) {
      s->err = "boundary face index out of range";
      return FSI_ERR_MESH;
    }
  for (int8_t d : h.dom)
    if (d != 0 && d != 1) {
      s->err = "tet_domain must be 0 or 1";
      return FSI_ERR_MESH;
    }
  s->ph = *ph;
  s->opts = *o;
  s->opts.part = nullptr;
  s->stream = (hipStream_t)stream;
  std::string e = build_topology(h);
  if (!e.empty()) {
    s->err = e;
    return FSI_ERR_MESH;
  }
  e = build_subdomains(h, *o);
  if (!e.empty()) {
    s->err = e;
    return FSI_ERR_ARG;
  }
  s->n = 7 * (int64_t)h.V;
  s->nnzb = (int64_t)h.colind.size();
  s->R = (int64_t)h.lglob.size();
  s->NB = (int64_t)h.lcol.size();
  for (int64_t i = 0; i < s->R; ++i) {
    s->max_lblk = std::max(s->max_lblk, h.ldiag[i] - h.lrowptr[i]);
    s->max_ublk = std::max(s->max_ublk, h.lrowptr[i + 1] - h.ldiag[i] - 1);
    s->max_rowblk = std::max(s->max_rowblk, h.lrowptr[i + 1] - h.lrowptr[i]);
  }
  std::vector<int32_t> blkrow(s->nnzb);
  for (int v = 0; v < h.V; ++v)
    for (int k = h.rowptr[v]; k < h.rowptr[v + 1]; ++k) blkrow[k] = v;

  s->X = upload(s, h.X);
  s->tets = upload(s, h.tets);
  s->fluid_elems = upload(s, h.fluid_elems);
  s->solid_elems = upload(s, h.solid_elems);
  s->fluid_celems = upload(s, h.fluid_celems);
  s->solid_celems = upload(s, h.solid_celems);
  s->vinc_ptr = upload(s, h.vinc_ptr);
  s->vinc = upload(s, h.vinc);
  s->elem_blk = upload(s, h.elem_blk);
  s->rowptr = upload(s, h.rowptr);
  s->colind = upload(s, h.colind);
  s->blkrow = upload(s, blkrow);
  s->vals = dalloc<double>(s, (size_t)s->nnzb * 49);
  s->elemR = dalloc<double>(s, (size_t)h.E * 28);
  s->rowkind = dalloc<uint8_t>(s, s->n);
  s->gval = dalloc<double>(s, s->n);
  s->yold = dalloc<double>(s, s->n);
  s->bforce = dalloc<double>(s, 3 * (size_t)h.V);
  s->lglob = upload(s, h.lglob);
  s->lowned = upload(s, h.lowned);
  s->lrowptr = upload(s, h.lrowptr);
  s->lcol = upload(s, h.lcol);
  s->lsrc = upload(s, h.lsrc);
  s->ldiag = upload(s, h.ldiag);
  s->fwd_sub_lvl = upload(s, h.fwd_sub_lvl);
  s->fwd_lvl_ptr = upload(s, h.fwd_lvl_ptr);
  s->fwd_rows = upload(s, h.fwd_rows);
  s->bwd_sub_lvl = upload(s, h.bwd_sub_lvl);
  s->bwd_lvl_ptr = upload(s, h.bwd_lvl_ptr);
  s->bwd_rows = upload(s, h.bwd_rows);
  {
    // per-wavefront task lists of both sweeps (level order inside each wavefront)
    // every candidate schedule (tasks of at most mb blocks); the row-length rule picks the
    // one used until fsi_pc_tune or fsi_pc_select chooses another
    for (int c = 0; c < kSweepPlans; ++c) {
      SweepPlan& P = s->plans[c];
      P.mb = kSweepPlanMB[c];
      auto tasks = [&](bool bwd, const std::vector<int32_t>& sub_lvl, const std::vector<int32_t>& lvl_ptr,
                       const std::vector<int32_t>& rows, const std::vector<int32_t>& qslot, int32_t** wtask_d,
                       int4** task_d, int4** aux_d, int32_t** nphase_d) {
        SweepTasks st = build_sweep_tasks(h, bwd, sub_lvl, lvl_ptr, rows, qslot, P.mb);
        *wtask_d = upload(s, st.wtask);
        *task_d = upload(s, st.task);
        *aux_d = upload(s, st.aux);
        *nphase_d = upload(s, st.nphase);
      };
      tasks(false, h.fwd_sub_lvl, h.fwd_lvl_ptr, h.fwd_rows, h.fwd_qslot, &P.fwd_wtask, &P.fwd_task,
            &P.fwd_task_aux, &P.fwd_nphase);
      tasks(true, h.bwd_sub_lvl, h.bwd_lvl_ptr, h.bwd_rows, h.bwd_qslot, &P.bwd_wtask, &P.bwd_task,
            &P.bwd_task_aux, &P.bwd_nphase);
    }
    select_plan(s, sweep_task_blocks(std::max(s->max_lblk, s->max_ublk)));
    std::vector<int32_t> lbyte(h.lslot.size());
    // a slot holds 7 values of the sweep arithmetic type (FP64, or FP32 for rounded factors)
    const int slot_bytes = 7 * (s->opts.precision == FSI_PREC_FP64 ? 8 : 4);
    for (size_t p = 0; p < lbyte.size(); ++p) lbyte[p] = h.lslot[p] >= 0 ? slot_bytes * h.lslot[p] : 0;
    s->lslot = upload(s, lbyte);
  }
  {
    // factorization groups: per pivot, the blocks of U_k that have a match in row i (the
    // others would update nothing), in runs of up to 2*kFacHalf blocks, each with the
    // forward level of its pivot row.  A block's code is (t << 16) | pos: t its index in U_k,
    // pos its position in row i plus one; both fit 16 bits since no row reaches 65535 blocks.
    if (s->max_rowblk >= 65535) {
      s->err = "a local row of 65535 blocks or more";
      return FSI_ERR_ARG;
    }
    std::vector<int32_t> lvl_of(h.lglob.size(), 0);
    for (int sd = 0; sd < h.ns; ++sd)
      for (int L = h.fwd_sub_lvl[sd]; L < h.fwd_sub_lvl[sd + 1]; ++L)
        for (int q = h.fwd_lvl_ptr[L]; q < h.fwd_lvl_ptr[L + 1]; ++q) lvl_of[h.fwd_rows[q]] = L - h.fwd_sub_lvl[sd];
    std::vector<int32_t> gptr(1, 0), glvl, codes, pres;
    std::vector<int64_t> crow(1, 0);
    std::vector<int4> grp;
    for (size_t i = 0; i + 1 < h.kent_ptr.size(); ++i) {
      const int64_t ub = h.umap_row[i];
      for (int k = h.kent_ptr[i]; k < h.kent_ptr[i + 1]; ++k) {
        const int pik = h.piv[4 * k], dk = h.piv[4 * k + 1], nu = h.piv[4 * k + 2], mo = h.piv[4 * k + 3];
        pres.clear();
        for (int t = 0; t < nu; ++t) {
          const int32_t pos = h.umap[ub + mo + t];
          if (pos > 0) pres.push_back((t << 16) | pos);
        }
        const int run = 2 * kFacHalf, np = (int)pres.size();
        const int ngk = std::max(1, (np + run - 1) / run);
        const int plev = lvl_of[h.lcol[h.lrowptr[i] + pik]];
        const int64_t off = (int64_t)codes.size() - crow.back();  // within row i's codes
        for (int g = 0; g < ngk; ++g) {
          const int nb = std::min(run, np - run * g);
          grp.push_back(make_int4(dk + 1, dk, (int32_t)(off + run * g), (pik << 6) | (std::max(nb, 0) << 1) | (g == 0)));
          glvl.push_back(plev);
        }
        codes.insert(codes.end(), pres.begin(), pres.end());
      }
      gptr.push_back((int32_t)grp.size());
      crow.push_back((int64_t)codes.size());
    }
    s->fgrp_ptr = upload(s, gptr);
    s->fgrp = upload(s, grp);
    s->fgrp_lvl = upload(s, glvl);
    s->umap = upload(s, codes);
    s->umap_row = upload(s, crow);
    // rows round-robin over the factorization's wavefronts, in level order
    s->fac_nw = fac_layout(s->max_rowblk, s->opts.precision == FSI_PREC_FP32_FACTOR ? 4 : 8).waves;
    if (s->fac_nw < 1) {
      s->err = "a local row is too long to stage in LDS for the factorization";
      return FSI_ERR_ARG;
    }
    std::vector<int32_t> wptr(1, 0), wrow, wlvl;
    std::vector<std::vector<int32_t>> lr(s->fac_nw), ll(s->fac_nw);
    for (int sd = 0; sd < h.ns; ++sd) {
      for (auto& v : lr) v.clear();
      for (auto& v : ll) v.clear();
      int next = 0;
      for (int L = h.fwd_sub_lvl[sd]; L < h.fwd_sub_lvl[sd + 1]; ++L)
        for (int q = h.fwd_lvl_ptr[L]; q < h.fwd_lvl_ptr[L + 1]; ++q) {
          lr[next % s->fac_nw].push_back(h.fwd_rows[q]);
          ll[next % s->fac_nw].push_back(L - h.fwd_sub_lvl[sd]);
          ++next;
        }
      for (int w = 0; w < s->fac_nw; ++w) {
        wrow.insert(wrow.end(), lr[w].begin(), lr[w].end());
        wlvl.insert(wlvl.end(), ll[w].begin(), ll[w].end());
        wptr.push_back((int32_t)wrow.size());
      }
    }
    s->fw_ptr = upload(s, wptr);
    s->fw_row = upload(s, wrow);
    s->fw_lvl = upload(s, wlvl);
  }
  s->sub_row_off = upload(s, h.sub_row_off);
  if (s->opts.precision == FSI_PREC_FP32_FACTOR) {  // the factorization itself in FP32
    s->fac32 = dalloc<float>(s, (size_t)s->NB * 49);
    s->udiag32 = dalloc<float>(s, (size_t)s->R * 49);
  } else {
    s->fac = dalloc<double>(s, (size_t)s->NB * 49);
    // rounded factors (FP32 or BF16 sweeps) are written over the FP64 ones after each
    // factorization: they share its buffer
    if (s->opts.precision != FSI_PREC_FP64) s->facs = s->fac;
    s->udiag = dalloc<double>(s, (size_t)s->R * 49);
  }
  s->ylocal = dalloc<double>(s, (size_t)s->R * 7);
  const int mrs = s->opts.gmres_restart;
  s->Vb = dalloc<double>(s, (size_t)(mrs + 1) * s->n);
  s->w = dalloc<double>(s, s->n);
  s->z = dalloc<double>(s, s->n);
  s->r = dalloc<double>(s, s->n);
  s->tmp = dalloc<double>(s, s->n);
  s->partial = dalloc<double>(s, (size_t)kRedBlocks * 32);
  s->hdev = dalloc<double>(s, 4 * (kMaxRestart + 8));
  s->yvdev = dalloc<double>(s, kMaxRestart + 8);
  s->F = dalloc<double>(s, s->n);
  s->Ft = dalloc<double>(s, s->n);
  s->yt = dalloc<double>(s, s->n);
  s->dy = dalloc<double>(s, s->n);
  s->rhs = dalloc<double>(s, s->n);
  s->flags = dalloc<int32_t>(s, kFlags);
  hip_ok(s, hipHostMalloc((void**)&s->pinned, 4 * (kMaxRestart + 8) * sizeof(double), hipHostMallocDefault),
         "hipHostMalloc");
  hip_ok(s, hipMemset(s->flags, 0, kFlags * sizeof(int32_t)), "memset");
  hip_ok(s, hipMemset(s->hdev, 0, 4 * (kMaxRestart + 8) * sizeof(double)), "memset");
  hip_ok(s, hipDeviceSynchronize(), "sync");
  scratch_attach(s);
  return FSI_OK;
}

fsi_status guard(fsi_solver* s, fsi_status (*fn)(fsi_solver*, void*), void* arg) {
  try {
    return fn(s, arg);
  } catch (const Fail& f) {
    return f.st;
  } catch (const std::bad_alloc&) {
    s->err = "host allocation failed";
    return FSI_ERR_OOM;
  } catch (...) {
    s->err = "unexpected exception";
    return FSI_ERR_HIP;
  }
}

}  // namespace

namespace fsi {
void prof_begin(fsi_solver* s, const char* name, hipEvent_t* ev) {
  (void)name;
  hipEvent_t a;
  if (!s->event_pool.empty()) {
    a = s->event_pool.back();
    s->event_pool.pop_back();
  } else {
    (void)hipEventCreate(&a);
  }
  (void)hipEventRecord(a, s->stream);
  *ev = a;
}
void prof_end(fsi_solver* s, const char* name, hipEvent_t a) {
  hipEvent_t b;
  if (!s->event_pool.empty()) {
    b = s->event_pool.back();
    s->event_pool.pop_back();
  } else {
    (void)hipEventCreate(&b);
  }
  (void)hipEventRecord(b, s->stream);
  s->prof_events.push_back(ProfEntry{name, a, b});
}
}  // namespace fsi

namespace fsi {
// Makes the schedule with tasks of mb blocks the one the sweeps use; false if mb is not a
// candidate.
void drop_graphs(fsi_solver* s) {
  for (auto& g : s->arnoldi)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

bool select_plan(fsi_solver* s, int mb) {
  for (const SweepPlan& P : s->plans)
    if (P.mb == mb && P.fwd_task) {
      if (mb != s->sweep_mb) drop_graphs(s);  // captured sweeps use the old task lists
      s->sweep_mb = mb;
      s->fwd_wtask = P.fwd_wtask;
      s->fwd_task = P.fwd_task;
      s->fwd_task_aux = P.fwd_task_aux;
      s->fwd_nphase = P.fwd_nphase;
      s->bwd_wtask = P.bwd_wtask;
      s->bwd_task = P.bwd_task;
      s->bwd_task_aux = P.bwd_task_aux;
      s->bwd_nphase = P.bwd_nphase;
      return true;
    }
  return false;
}
}  // namespace fsi

extern "C" {

fsi_status fsi_create(const fsi_mesh* m, const fsi_physics* ph, const fsi_opts* o, void* stream, fsi_solver** out) {
  if (!m || !ph || !o || !out || m->nverts <= 0 || m->ntets <= 0 || !m->X || !m->tets || !m->tet_domain ||
      (m->nbfaces > 0 && (!m->bfaces || !m->bface_tag)) || m->nbfaces < 0)
    return FSI_ERR_ARG;
  if (o->nsub <= 0 || o->nsub > m->nverts || o->overlap < 0 || o->ilu_level < 0 || o->ilu_level > 8 ||
      o->gmres_restart <= 0 || o->gmres_restart > kMaxRestart || o->gmres_maxit <= 0 || (o->ordering != FSI_ORDER_RCM && o->ordering != FSI_ORDER_1WD) ||
      o->precision < FSI_PREC_FP64 || o->precision > FSI_PREC_FP32_FACTOR || (int64_t)m->ntets * 16 >= (int64_t)INT32_MAX)
    return FSI_ERR_ARG;
  fsi_solver* s = new (std::nothrow) fsi_solver();
  if (!s) return FSI_ERR_OOM;
  struct A {
    const fsi_mesh* m;
    const fsi_physics* ph;
    const fsi_opts* o;
    void* st;
  } a{m, ph, o, stream};
  fsi_status rc = guard(s, [](fsi_solver* s, void* p) {
    A* a = (A*)p;
    return create_impl(a->m, a->ph, a->o, a->st, s);
  }, &a);
  if (rc) {
    fsi_destroy(s);
    return rc;
  }
  *out = s;
  return FSI_OK;
}

fsi_status fsi_destroy(fsi_solver* s) {
  if (!s) return FSI_OK;
  (void)hipStreamSynchronize(s->stream);
  drop_graphs(s);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  for (void* p : s->allocs) (void)hipFree(p);
  if (s->pinned) (void)hipHostFree(s->pinned);
  for (auto& e : s->prof_events) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto e : s->event_pool) (void)hipEventDestroy(e);
  delete s;
  return FSI_OK;
}

fsi_status fsi_sizes(const fsi_solver* s, int64_t* n, int64_t* nnzb) {
  if (!s) return FSI_ERR_ARG;
  if (n) *n = s->n;
  if (nnzb) *nnzb = s->nnzb;
  return FSI_OK;
}

const char* fsi_last_error(const fsi_solver* s) { return s ? s->err.c_str() : "null solver"; }

fsi_status fsi_set_step(fsi_solver* s, double t_n, double dt, const double* y_old, const double* g,
                        const double* bf, const uint8_t* extra_mask) {
  if (!s || !y_old || !g || !(dt > 0.0) || !std::isfinite(dt)) return FSI_ERR_ARG;
  struct A {
    double t, dt;
    const double *yo, *g, *bf;
    const uint8_t* em;
  } a{t_n, dt, y_old, g, bf, extra_mask};
  return guard(s, [](fsi_solver* s, void* p) {
    A* a = (A*)p;
    const size_t n = s->n;
    s->t = a->t;
    s->dt = a->dt;
    s->rowkind_host = s->h.rowkind_base;
    if (a->em)
      for (size_t i = 0; i < n; ++i)
        if (a->em[i]) s->rowkind_host[i] = RK_DIR;
    hip_ok(s, hipMemcpyAsync(s->rowkind, s->rowkind_host.data(), n, hipMemcpyHostToDevice, s->stream), "rowkind");
    hip_ok(s, hipMemcpyAsync(s->yold, a->yo, n * sizeof(double), hipMemcpyDeviceToDevice, s->stream), "yold");
    hip_ok(s, hipMemcpyAsync(s->gval, a->g, n * sizeof(double), hipMemcpyDeviceToDevice, s->stream), "g");
    // clamped wall rings take the value zero whatever g holds there
    std::vector<double> fz;
    bool any = false;
    for (size_t i = 0; i < n && !any; ++i) any = s->h.forced_zero[i] && s->rowkind_host[i] == RK_DIR;
    if (any) {
      sync(s);
      fz.resize(n);
      hip_ok(s, hipMemcpy(fz.data(), s->gval, n * sizeof(double), hipMemcpyDeviceToHost), "g down");
      for (size_t i = 0; i < n; ++i)
        if (s->h.forced_zero[i]) fz[i] = 0.0;
      hip_ok(s, hipMemcpy(s->gval, fz.data(), n * sizeof(double), hipMemcpyHostToDevice), "g up");
    }
    s->has_bforce = a->bf != nullptr;
    if (a->bf)
      hip_ok(s, hipMemcpyAsync(s->bforce, a->bf, 3 * (size_t)s->h.V * sizeof(double), hipMemcpyDeviceToDevice,
                               s->stream), "bforce");
    sync(s);
    s->has_step = true;
    s->jac_ready = false;
    s->pc_ready = false;
    return FSI_OK;
  }, &a);
}

fsi_status fsi_impose_dirichlet(fsi_solver* s, double* y) {
  if (!s || !y || !s->has_step) return FSI_ERR_ARG;
  return guard(s, [](fsi_solver* s, void* p) {
    hip_ok(s, launch_impose(s, (double*)p), "impose");
    sync(s);
    return FSI_OK;
  }, y);
}

fsi_status fsi_residual(fsi_solver* s, const double* y, double* F) {
  if (!s || !y || !F || !s->has_step) return FSI_ERR_ARG;
  const double* a[2] = {y, F};
  return guard(s, [](fsi_solver* s, void* p) {
    const double** a = (const double**)p;
    return residual_impl(s, a[0], (double*)a[1]);
  }, a);
}

fsi_status fsi_jacobian(fsi_solver* s, const double* y) {
  if (!s || !y || !s->has_step) return FSI_ERR_ARG;
  return guard(s, [](fsi_solver* s, void* p) { return jacobian_impl(s, (const double*)p); }, (void*)y);
}

fsi_status fsi_jacobian_get(const fsi_solver* cs, int32_t* rowptr, int32_t* colind, double* vals) {
  if (!cs) return FSI_ERR_ARG;
  fsi_solver* s = const_cast<fsi_solver*>(cs);
  if (rowptr) std::copy(s->h.rowptr.begin(), s->h.rowptr.end(), rowptr);
  if (colind) std::copy(s->h.colind.begin(), s->h.colind.end(), colind);
  if (vals) {
    if (!s->jac_ready) return FSI_ERR_ARG;
    return guard(s, [](fsi_solver* s, void* p) {
      sync(s);
      hip_ok(s, hipMemcpy(p, s->vals, (size_t)s->nnzb * 49 * sizeof(double), hipMemcpyDeviceToHost), "vals down");
      return FSI_OK;
    }, vals);
  }
  return FSI_OK;
}

fsi_status fsi_jacobian_set(fsi_solver* s, const double* vals) {
  if (!s || !vals) return FSI_ERR_ARG;
  return guard(s, [](fsi_solver* s, void* p) {
    sync(s);
    hip_ok(s, hipMemcpy(s->vals, p, (size_t)s->nnzb * 49 * sizeof(double), hipMemcpyHostToDevice), "vals up");
    s->jac_ready = true;
    s->pc_ready = false;
    return FSI_OK;
  }, (void*)vals);
}

fsi_status fsi_spmv(fsi_solver* s, const double* x, double* y) {
  if (!s || !x || !y || !s->jac_ready) return FSI_ERR_ARG;
  const double* a[2] = {x, y};
  return guard(s, [](fsi_solver* s, void* p) {
    const double** a = (const double**)p;
    hip_ok(s, launch_spmv(s, a[0], (double*)a[1]), "spmv");
    sync(s);
    return FSI_OK;
  }, a);
}

fsi_status fsi_pc_setup(fsi_solver* s) {
  if (!s) return FSI_ERR_ARG;
  return guard(s, [](fsi_solver* s, void*) {
    fsi_status rc = pc_setup_impl(s);
    sync(s);
    return rc;
  }, nullptr);
}

fsi_status fsi_pc_apply(fsi_solver* s, const double* v, double* z) {
  if (!s || !v || !z || !s->pc_ready) return FSI_ERR_ARG;
  const double* a[2] = {v, z};
  return guard(s, [](fsi_solver* s, void* p) {
    const double** a = (const double**)p;
    clear_sweep_flag(s);
    hip_ok(s, launch_pc_apply(s, a[0], (double*)a[1]), "pc_apply");
    if (read_flag(s, 3)) {
      s->err = "a Schwarz sweep waited on a row beyond its bound";
      return FSI_ERR_HIP;
    }
    return FSI_OK;
  }, a);
}

fsi_status fsi_pc_apply_noalloc(fsi_solver* s, const double* v, double* z) {
  if (!s || !v || !z || !s->pc_ready) return FSI_ERR_ARG;
  const double* a[2] = {v, z};
  return guard(s, [](fsi_solver* s, void* p) {
    const double** a = (const double**)p;
    if (!s->scratch) {
      s->err = std::string("no scratch address on this device: ") + hipGetErrorString(s->scratch_err);
      return FSI_ERR_HIP;
    }
    const size_t need = pc_apply_ws_bytes(s);
    if (need > kScratchYBytes) {
      s->err = "fsi_pc_apply_noalloc: the sweeps need " + std::to_string(need) + " bytes of scratch (" +
               std::to_string(s->R) + " local rows), above its " + std::to_string(kScratchYBytes) + " bytes";
      return FSI_ERR_ARG;
    }
    int32_t* fl = (int32_t*)s->scratch;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s->stream, fl, 4);
    hip_ok(s, hipGetLastError(), "clear scratch flags");
    const bool prof = s->prof;  // kernel timing would create events: off for this call
    s->prof = false;
    const hipError_t e = launch_pc_apply_ws(s, a[0], (double*)a[1], s->scratch + kScratchFlagBytes, fl);
    s->prof = prof;
    hip_ok(s, e, "pc_apply_noalloc");
    hip_ok(s, hipMemcpyAsync(&s->pinned[200], fl + 3, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream),
           "flag readback");
    sync(s);
    int32_t f;
    std::memcpy(&f, &s->pinned[200], sizeof f);
    if (f) {
      s->err = "a Schwarz sweep waited on a row beyond its bound";
      return FSI_ERR_HIP;
    }
    return FSI_OK;
  }, a);
}

fsi_status fsi_set_graphs(fsi_solver* s, int32_t on) {
  if (!s) return FSI_ERR_ARG;
  (void)hipStreamSynchronize(s->stream);
  if (!on) drop_graphs(s);
  s->graphs = on != 0;
  return FSI_OK;
}

fsi_status fsi_pc_select(fsi_solver* s, int32_t mb) {
  if (!s) return FSI_ERR_ARG;
  if (!select_plan(s, mb)) {
    s->err = "no sweep schedule with " + std::to_string(mb) + " blocks per task";
    return FSI_ERR_ARG;
  }
  return FSI_OK;
}

fsi_status fsi_pc_tune(fsi_solver* s, int32_t reps, int32_t* best_mb, double* us) {
  if (!s || reps < 1 || !s->pc_ready) return FSI_ERR_ARG;
  struct A {
    int reps;
    int32_t* best;
    double* us;
  } a{reps, best_mb, us};
  return guard(s, [](fsi_solver* s, void* p) {
    A* a = (A*)p;
    hipEvent_t e0, e1;
    hip_ok(s, hipEventCreate(&e0), "event");
    hip_ok(s, hipEventCreate(&e1), "event");
    // probe input: the current residual vector (finite values); output to scratch
    double best_t = 0.0;
    int best = s->sweep_mb;
    clear_sweep_flag(s);
    for (int c = 0; c < kSweepPlans; ++c) {
      const int mb = s->plans[c].mb;
      select_plan(s, mb);
      hip_ok(s, launch_pc_apply(s, s->F, s->z), "tune warm-up");
      hip_ok(s, hipEventRecord(e0, s->stream), "event");
      for (int r = 0; r < a->reps; ++r) hip_ok(s, launch_pc_apply(s, s->F, s->z), "tune");
      hip_ok(s, hipEventRecord(e1, s->stream), "event");
      hip_ok(s, hipEventSynchronize(e1), "event");
      float ms = 0.f;
      hip_ok(s, hipEventElapsedTime(&ms, e0, e1), "event");
      const double t = 1e3 * ms / a->reps;
      if (a->us) a->us[c] = t;
      if (c == 0 || t < best_t) best_t = t, best = mb;
    }
    select_plan(s, best);
    if (a->best) *a->best = best;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (read_flag(s, 3)) {
      s->err = "a Schwarz sweep waited on a row beyond its bound";
      return FSI_ERR_HIP;
    }
    return FSI_OK;
  }, &a);
}

fsi_status fsi_gmres(fsi_solver* s, const double* rhs, double* x, fsi_lin_stats* st) {
  if (!s || !rhs || !x || !s->pc_ready) return FSI_ERR_ARG;
  struct A {
    const double* b;
    double* x;
    fsi_lin_stats* st;
  } a{rhs, x, st};
  return guard(s, [](fsi_solver* s, void* p) {
    A* a = (A*)p;
    fsi_status rc = gmres_impl(s, a->b, a->x, a->st, nullptr, nullptr);
    sync(s);
    return rc;
  }, &a);
}

fsi_status fsi_set_wait_limit(fsi_solver* s, int32_t polls) {
  if (!s) return FSI_ERR_ARG;
  if (polls < -1) {
    s->err = "wait limit below -1";
    return FSI_ERR_ARG;
  }
  (void)hipStreamSynchronize(s->stream);
  drop_graphs(s);  // captured launches hold the old limit
  s->wait_limit = polls < 0 ? fsi::kWaitLimit : polls;
  return FSI_OK;
}

fsi_status fsi_set_newton_tol(fsi_solver* s, double rtol, double atol) {
  if (!s || !(rtol >= 0.0) || !(atol >= 0.0) || (rtol == 0.0 && atol == 0.0)) return FSI_ERR_ARG;
  s->opts.newton_rtol = rtol;
  s->opts.newton_atol = atol;
  return FSI_OK;
}

fsi_status fsi_newton_solve(fsi_solver* s, double* y, fsi_step_stats* st) {
  if (!s || !y || !s->has_step) return FSI_ERR_ARG;
  struct A {
    double* y;
    fsi_step_stats* st;
  } a{y, st};
  return guard(s, [](fsi_solver* s, void* p) {
    A* a = (A*)p;
    return newton_impl(s, a->y, a->st);
  }, &a);
}

fsi_status fsi_topology_get(const fsi_solver* s, int8_t* vkind, uint8_t* rowkind, int32_t* n_iface,
                            int32_t* iface_faces) {
  if (!s) return FSI_ERR_ARG;
  if (vkind) std::copy(s->h.vkind.begin(), s->h.vkind.end(), vkind);
  if (rowkind) {
    const std::vector<uint8_t>& rk = s->has_step ? s->rowkind_host : s->h.rowkind_base;
    std::copy(rk.begin(), rk.end(), rowkind);
  }
  if (n_iface) *n_iface = (int32_t)(s->h.iface.size() / 3);
  if (iface_faces) std::copy(s->h.iface.begin(), s->h.iface.end(), iface_faces);
  return FSI_OK;
}

fsi_status fsi_pc_sizes(const fsi_solver* s, int32_t* nsub, int64_t* nrows, int64_t* nblocks, int64_t* nlev) {
  if (!s) return FSI_ERR_ARG;
  if (nsub) *nsub = s->h.ns;
  if (nrows) *nrows = s->R;
  if (nblocks) *nblocks = s->NB;
  if (nlev) *nlev = (int64_t)s->h.fwd_lvl_ptr.size() - 1;
  return FSI_OK;
}

fsi_status fsi_pc_get(const fsi_solver* cs, int32_t* part, int32_t* sub_ptr, int32_t* sub_verts,
                      int32_t* sub_nowned, int64_t* blk_ptr, int32_t* lrowptr, int32_t* lcolind, double* factors,
                      double* udiag) {
  if (!cs) return FSI_ERR_ARG;
  fsi_solver* s = const_cast<fsi_solver*>(cs);
  const HostSetup& h = s->h;
  if (part) std::copy(h.part.begin(), h.part.end(), part);
  if (sub_ptr) std::copy(h.sub_row_off.begin(), h.sub_row_off.end(), sub_ptr);
  if (sub_verts) std::copy(h.lglob.begin(), h.lglob.end(), sub_verts);
  if (sub_nowned) std::copy(h.sub_nowned.begin(), h.sub_nowned.end(), sub_nowned);
  for (int i = 0; i < h.ns; ++i) {
    const int r0 = h.sub_row_off[i], r1 = h.sub_row_off[i + 1];
    const int b0 = h.lrowptr[r0];
    if (blk_ptr) {
      blk_ptr[i] = b0;
      blk_ptr[i + 1] = h.lrowptr[r1];
    }
    if (lrowptr)  // per-subdomain local row pointers, concatenated (size R + ns)
      for (int r = r0; r <= r1; ++r) lrowptr[r + i] = h.lrowptr[r] - b0;
    if (lcolind)
      for (int p = b0; p < h.lrowptr[r1]; ++p) lcolind[p] = h.lcol[p] - r0;
  }
  if ((factors || udiag) && !s->pc_ready) return FSI_ERR_ARG;
  const double* a[2] = {factors, udiag};
  if (factors || udiag)
    return guard(s, [](fsi_solver* s, void* p) {
      double** a = (double**)p;
      sync(s);
      const size_t nf = (size_t)s->NB * 49;
      if (s->opts.precision == FSI_PREC_FP32_FACTOR) {  // FP32 factorization: widened
        auto widen = [&](double* out, const float* dev, size_t cnt, const char* what) {
          std::vector<float> tmp(cnt);
          hip_ok(s, hipMemcpy(tmp.data(), dev, cnt * sizeof(float), hipMemcpyDeviceToHost), what);
          for (size_t i = 0; i < cnt; ++i) out[i] = (double)tmp[i];
        };
        if (a[0]) widen(a[0], s->fac32, nf, "fac");
        if (a[1]) widen(a[1], s->udiag32, (size_t)s->R * 49, "ud");
        return FSI_OK;
      }
      if (a[0] && s->opts.precision == FSI_PREC_FP64) {
        hip_ok(s, hipMemcpy(a[0], s->fac, nf * sizeof(double), hipMemcpyDeviceToHost), "fac");
      } else if (a[0]) {
        // the rounded factors the sweeps use, widened to FP64 from the last entry down (the
        // rounded entries fill the front of the same host buffer)
        const size_t w = s->opts.precision == FSI_PREC_FP32 ? 4 : 2;
        hip_ok(s, hipMemcpy(a[0], s->fac, nf * w, hipMemcpyDeviceToHost), "fac");
        unsigned char* b = (unsigned char*)a[0];
        for (size_t i = nf; i-- > 0;) {
          float f;
          if (w == 4) {
            std::memcpy(&f, b + 4 * i, 4);
          } else {
            uint16_t hbits;
            std::memcpy(&hbits, b + 2 * i, 2);
            const uint32_t u = (uint32_t)hbits << 16;
            std::memcpy(&f, &u, 4);
          }
          a[0][i] = (double)f;
        }
      }
      if (a[1]) hip_ok(s, hipMemcpy(a[1], s->udiag, (size_t)s->R * 49 * sizeof(double), hipMemcpyDeviceToHost), "ud");
      return FSI_OK;
    }, (void*)a);
  return FSI_OK;
}

fsi_status fsi_prof_enable(fsi_solver* s, int32_t on) {
  if (!s) return FSI_ERR_ARG;
  (void)hipStreamSynchronize(s->stream);
  for (auto& e : s->prof_events) {  // a new enable starts a fresh record
    s->event_pool.push_back(e.a);
    s->event_pool.push_back(e.b);
  }
  s->prof_events.clear();
  s->prof = on != 0;
  return FSI_OK;
}

fsi_status fsi_prof_get(fsi_solver* s, const char* kernel, double* total_ms, int64_t* count) {
  if (!s || !kernel) return FSI_ERR_ARG;
  struct A {
    const char* name;
    double* tot;
    int64_t* cnt;
  } a{kernel, total_ms, count};
  return guard(s, [](fsi_solver* s, void* p) {
    A* a = (A*)p;
    sync(s);
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto& e : s->prof_events) {
      if (e.name != a->name) continue;
      float ms = 0.f;
      hip_ok(s, hipEventElapsedTime(&ms, e.a, e.b), "event time");
      tot += ms;
      ++cnt;
    }
    if (a->tot) *a->tot = tot;
    if (a->cnt) *a->cnt = cnt;
    return FSI_OK;
  }, &a);
}

}  // extern "C"
