// Residual and exact-Jacobian assembly kernels (FuncEval / JacEval).
//
// Physics (paper §2.1-§2.2): ALE incompressible Navier-Stokes with SUPG/PSPG
// stabilization on the current configuration x = X + d, a St. Venant-Kirchhoff wall on
// the reference configuration, a harmonic mesh extension, backward Euler (eq. (9)); every
// equation row carries F = dt * R.  Stabilization parameter (the paper defers its form to
// its references): tau = [(2/dt)^2 + cbar.G.cbar + C_I nu^2 G:G]^(-1/2) with cbar the
// element mean of u - w and G = Jxi^T Jxi; no LSIC term; the viscous term of the strong
// residual vanishes for linear elements.  Quadrature: 4-point degree-2 rule for the fluid
// terms and all mass terms, exact single-point integration for constant integrands.
//
// Residual scatter: each element writes its 28-row residual to a staging buffer; a gather
// kernel then sums, per degree of freedom, the contributions of the incident elements in
// ascending element order.
//
// Jacobian: exact (§3, no finite differences).  Lane j of a 32-lane team evaluates the
// element residual in dual numbers seeded with the j-th element unknown, so one team
// produces the 28 columns of the element matrix at once, in registers, and adds column j
// straight into the 16 blocks of J the element touches.  Elements are coloured so that no
// two of one colour share a vertex; one launch per colour then updates disjoint entries of
// J, without atomics.  The sums follow the colour order, fixed at set-up, so the result is
// bitwise reproducible from run to run.
#include "fsi_internal.hpp"

namespace fsi {

struct PhysDev {
  double rho_f, mu_f, rho_s, mu_s, lam_s, eta_s, C_I, dt;
};

static PhysDev phys_dev(const fsi_solver* s) {
  PhysDev P;
  P.rho_f = s->ph.rho_f;
  P.mu_f = s->ph.mu_f;
  P.rho_s = s->ph.rho_s;
  P.mu_s = s->ph.E_s / (2.0 * (1.0 + s->ph.nu_s));                                 // Lame (§2.1)
  P.lam_s = s->ph.E_s * s->ph.nu_s / ((1.0 + s->ph.nu_s) * (1.0 - 2.0 * s->ph.nu_s));
  P.eta_s = s->ph.eta_s;
  P.C_I = s->ph.C_I;
  P.dt = s->dt;
  return P;
}

// ---- forward-mode dual number: value and one tangent -------------------------------------
struct DN {
  double v, t;
};
__device__ __forceinline__ DN mk(double v) { return DN{v, 0.0}; }
__device__ __forceinline__ DN operator+(DN a, DN b) { return DN{a.v + b.v, a.t + b.t}; }
__device__ __forceinline__ DN operator-(DN a, DN b) { return DN{a.v - b.v, a.t - b.t}; }
__device__ __forceinline__ DN operator-(DN a) { return DN{-a.v, -a.t}; }
__device__ __forceinline__ DN operator*(DN a, DN b) { return DN{a.v * b.v, a.t * b.v + a.v * b.t}; }
__device__ __forceinline__ DN operator/(DN a, DN b) {
  double q = a.v / b.v;
  return DN{q, (a.t - q * b.t) / b.v};
}
__device__ __forceinline__ DN operator+(DN a, double b) { return DN{a.v + b, a.t}; }
__device__ __forceinline__ DN operator+(double a, DN b) { return DN{a + b.v, b.t}; }
__device__ __forceinline__ DN operator-(DN a, double b) { return DN{a.v - b, a.t}; }
__device__ __forceinline__ DN operator-(double a, DN b) { return DN{a - b.v, -b.t}; }
__device__ __forceinline__ DN operator*(DN a, double b) { return DN{a.v * b, a.t * b}; }
__device__ __forceinline__ DN operator*(double a, DN b) { return DN{a * b.v, a * b.t}; }
__device__ __forceinline__ DN operator/(DN a, double b) { return DN{a.v / b, a.t / b}; }
__device__ __forceinline__ DN& operator+=(DN& a, DN b) { a = a + b; return a; }
__device__ __forceinline__ DN rsqrt_dn(DN a) {
  double r = 1.0 / sqrt(a.v);
  return DN{r, -0.5 * r * a.t / a.v};
}
__device__ __forceinline__ double rsqrt_dn(double a) { return 1.0 / sqrt(a); }
__device__ __forceinline__ double value(double a) { return a; }
__device__ __forceinline__ double value(DN a) { return a.v; }
template <class T> __device__ __forceinline__ T zero();
template <> __device__ __forceinline__ double zero<double>() { return 0.0; }
template <> __device__ __forceinline__ DN zero<DN>() { return DN{0.0, 0.0}; }

// barycentric weights of the symmetric 4-point degree-2 rule: (5 + 3 sqrt 5)/20, (5 - sqrt 5)/20
#define QW_A 0.58541019662496845446
#define QW_B 0.13819660112501051518

template <class T>
__device__ __forceinline__ void cross3(const T a[3], const T b[3], T c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Shape-function gradients of a tet from its edge vectors e1,e2,e3 (columns of dx/dxi):
// grad phi_1..3 are the rows of (dx/dxi)^{-1} = [e2 x e3; e3 x e1; e1 x e2] / det.
template <class T>
__device__ __forceinline__ T tet_grads(const T e1[3], const T e2[3], const T e3[3], T g[4][3]) {
  cross3(e2, e3, g[1]);
  cross3(e3, e1, g[2]);
  cross3(e1, e2, g[3]);
  T det = e1[0] * g[1][0] + e1[1] * g[1][1] + e1[2] * g[1][2];
  for (int k = 0; k < 3; ++k) {
    g[1][k] = g[1][k] / det;
    g[2][k] = g[2][k] / det;
    g[3][k] = g[3][k] / det;
    g[0][k] = -(g[1][k] + g[2][k] + g[3][k]);
  }
  return det;
}

// Fluid element residual rows: [a][0..2] momentum, [a][3] continuity, [a][4..6] mesh Laplace.
template <class T>
__device__ __forceinline__ bool fluid_elem(const PhysDev& P, const double X[4][3], const T y[4][7],
                                           const double yo[4][7], const double f[4][3], T R[4][7]) {
  const double rho = P.rho_f, mu = P.mu_f, dt = P.dt, nu = mu / rho;
  T e[3][3];
  for (int b = 0; b < 3; ++b)
    for (int i = 0; i < 3; ++i) e[b][i] = (X[b + 1][i] + y[b + 1][4 + i]) - (X[0][i] + y[0][4 + i]);
  T g[4][3];
  T det = tet_grads(e[0], e[1], e[2], g);
  bool ok = value(det) > 0.0;
  T vol = det / 6.0;
  T G[3][3];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) G[k][l] = g[1][k] * g[1][l] + g[2][k] * g[2][l] + g[3][k] * g[3][l];
  T gu[3][3], gp[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      gu[i][j] = y[0][i] * g[0][j] + y[1][i] * g[1][j] + y[2][i] * g[2][j] + y[3][i] * g[3][j];
  for (int j = 0; j < 3; ++j) gp[j] = y[0][3] * g[0][j] + y[1][3] * g[1][j] + y[2][3] * g[2][j] + y[3][3] * g[3][j];
  T divu = gu[0][0] + gu[1][1] + gu[2][2];
  // mesh velocity w_a = (d_a - d_a^old)/dt and element mean of u - w
  T w[4][3], cbar[3];
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) w[a][i] = (y[a][4 + i] - yo[a][4 + i]) / dt;
  for (int i = 0; i < 3; ++i)
    cbar[i] = ((y[0][i] - w[0][i]) + (y[1][i] - w[1][i]) + (y[2][i] - w[2][i]) + (y[3][i] - w[3][i])) / 4.0;
  T GG = zero<T>(), cGc = zero<T>();
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      GG += G[k][l] * G[k][l];
      cGc += cbar[k] * (G[k][l] * cbar[l]);
    }
  T tau = rsqrt_dn((2.0 / dt) * (2.0 / dt) + cGc + (P.C_I * nu * nu) * GG);
  T pbar = (y[0][3] + y[1][3] + y[2][3] + y[3][3]) / 4.0;
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 7; ++r) R[a][r] = zero<T>();
  T wq = vol / 4.0;
  for (int q = 0; q < 4; ++q) {
    T uq[3], cq[3], rq[3], mq[3], cv[3];
    for (int i = 0; i < 3; ++i) {
      T su = zero<T>(), sw = zero<T>();
      double so = 0.0, sf = 0.0;
      for (int a = 0; a < 4; ++a) {
        const double la = (a == q) ? QW_A : QW_B;
        su += la * y[a][i];
        sw += la * w[a][i];
        so += la * yo[a][i];
        sf += la * f[a][i];
      }
      uq[i] = su;
      cq[i] = su - sw;
      mq[i] = (su - so) / dt;
      rq[i] = rho * mq[i] - rho * sf;  // completed below with convection and pressure gradient
      mq[i] = rho * mq[i] - rho * sf;  // Galerkin part that multiplies phi_a
    }
    for (int i = 0; i < 3; ++i) {
      cv[i] = gu[i][0] * cq[0] + gu[i][1] * cq[1] + gu[i][2] * cq[2];
      rq[i] = rq[i] + rho * cv[i] + gp[i];
      mq[i] = mq[i] + rho * cv[i];
    }
    (void)uq;
    for (int a = 0; a < 4; ++a) {
      const double la = (a == q) ? QW_A : QW_B;
      T cg = cq[0] * g[a][0] + cq[1] * g[a][1] + cq[2] * g[a][2];
      T tcg = tau * cg;
      for (int i = 0; i < 3; ++i) R[a][i] += wq * (la * mq[i] + tcg * rq[i]);
      T gr = g[a][0] * rq[0] + g[a][1] * rq[1] + g[a][2] * rq[2];
      R[a][3] += wq * (la * divu + (tau / rho) * gr);
    }
  }
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) {
      T sv = (gu[i][0] + gu[0][i]) * g[a][0] + (gu[i][1] + gu[1][i]) * g[a][1] + (gu[i][2] + gu[2][i]) * g[a][2];
      R[a][i] += vol * (mu * sv - pbar * g[a][i]);
    }
  // harmonic extension of the mesh displacement on the reference configuration (eq. (1))
  {
    double e0[3][3], g0[4][3];
    for (int b = 0; b < 3; ++b)
      for (int i = 0; i < 3; ++i) e0[b][i] = X[b + 1][i] - X[0][i];
    double det0 = tet_grads(e0[0], e0[1], e0[2], g0);
    double vol0 = det0 / 6.0;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        double kab = vol0 * (g0[a][0] * g0[b][0] + g0[a][1] * g0[b][1] + g0[a][2] * g0[b][2]);
        for (int i = 0; i < 3; ++i) R[a][4 + i] += kab * y[b][4 + i];
      }
  }
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 7; ++r) R[a][r] = dt * R[a][r];
  return ok;
}

// Wall element residual rows [a][0..2] (total Lagrangian, reference configuration):
// |K0| Pi grad_X phi_a + consistent-mass inertia and damping of the velocity.
template <class T>
__device__ __forceinline__ bool solid_elem(const PhysDev& P, const double X[4][3], const T y[4][7],
                                           const double yo[4][7], const double f[4][3], T R[4][7]) {
  const double dt = P.dt;
  double e0[3][3], g0[4][3];
  for (int b = 0; b < 3; ++b)
    for (int i = 0; i < 3; ++i) e0[b][i] = X[b + 1][i] - X[0][i];
  double det0 = tet_grads(e0[0], e0[1], e0[2], g0);
  double vol0 = det0 / 6.0;
  T Fd[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = (y[0][4 + i] * g0[0][j] + y[1][4 + i] * g0[1][j]) + (y[2][4 + i] * g0[2][j] + y[3][4 + i] * g0[3][j]);
      Fd[i][j] = (i == j) ? s + 1.0 : s;
    }
  T detF = Fd[0][0] * (Fd[1][1] * Fd[2][2] - Fd[1][2] * Fd[2][1]) -
           Fd[0][1] * (Fd[1][0] * Fd[2][2] - Fd[1][2] * Fd[2][0]) +
           Fd[0][2] * (Fd[1][0] * Fd[2][1] - Fd[1][1] * Fd[2][0]);
  bool ok = value(detF) > 0.0;
  T Eg[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      T c = Fd[0][i] * Fd[0][j] + Fd[1][i] * Fd[1][j] + Fd[2][i] * Fd[2][j];
      Eg[i][j] = 0.5 * ((i == j) ? c - 1.0 : c);
      Eg[j][i] = Eg[i][j];
    }
  T trE = Eg[0][0] + Eg[1][1] + Eg[2][2];
  T S[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) S[i][j] = (i == j) ? (2.0 * P.mu_s) * Eg[i][j] + P.lam_s * trE : (2.0 * P.mu_s) * Eg[i][j];
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 7; ++r) R[a][r] = zero<T>();
  for (int i = 0; i < 3; ++i) {
    T Pi[3];
    for (int j = 0; j < 3; ++j) Pi[j] = Fd[i][0] * S[0][j] + Fd[i][1] * S[1][j] + Fd[i][2] * S[2][j];
    for (int a = 0; a < 4; ++a) R[a][i] = vol0 * (Pi[0] * g0[a][0] + Pi[1] * g0[a][1] + Pi[2] * g0[a][2]);
  }
  for (int q = 0; q < 4; ++q)
    for (int i = 0; i < 3; ++i) {
      T uq = zero<T>();
      double uo = 0.0, fq = 0.0;
      for (int a = 0; a < 4; ++a) {
        const double la = (a == q) ? QW_A : QW_B;
        uq += la * y[a][i];
        uo += la * yo[a][i];
        fq += la * f[a][i];
      }
      T rq = P.rho_s * ((uq - uo) / dt) + P.eta_s * uq - P.rho_s * fq;
      for (int a = 0; a < 4; ++a) {
        const double la = (a == q) ? QW_A : QW_B;
        R[a][i] += (vol0 / 4.0) * (la * rq);
      }
    }
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) R[a][i] = dt * R[a][i];
  return ok;
}

template <int KIND>
__device__ __forceinline__ void load_elem(int e, const int32_t* __restrict__ tets, const double* __restrict__ X,
                                          const double* __restrict__ yold, const double* __restrict__ bf,
                                          double Xe[4][3], double yo[4][7], double fe[4][3], int vid[4]) {
  for (int a = 0; a < 4; ++a) {
    int v = tets[4 * (size_t)e + a];
    vid[a] = v;
    for (int i = 0; i < 3; ++i) {
      Xe[a][i] = X[3 * (size_t)v + i];
      fe[a][i] = bf ? bf[3 * (size_t)v + i] : 0.0;
    }
    for (int r = 0; r < 7; ++r) yo[a][r] = (KIND == 1 && r >= 3) ? 0.0 : yold[7 * (size_t)v + r];
  }
}

// ---- FuncEval: one lane per element ---------------------------------------------------------
template <int KIND>  // 0 fluid, 1 wall
__global__ void __launch_bounds__(256) k_elem_res(PhysDev P, int nel, const int32_t* __restrict__ elems,
                                                  const int32_t* __restrict__ tets, const double* __restrict__ X,
                                                  const double* __restrict__ y, const double* __restrict__ yold,
                                                  const double* __restrict__ bf, double* __restrict__ elemR,
                                                  int32_t* __restrict__ flags) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nel) return;
  int e = elems[t];
  double Xe[4][3], yo[4][7], fe[4][3], ye[4][7], R[4][7];
  int vid[4];
  load_elem<KIND>(e, tets, X, yold, bf, Xe, yo, fe, vid);
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 7; ++r) ye[a][r] = y[7 * (size_t)vid[a] + r];
  bool ok = KIND == 0 ? fluid_elem<double>(P, Xe, ye, yo, fe, R) : solid_elem<double>(P, Xe, ye, yo, fe, R);
  if (!ok) atomicOr(&flags[0], 1);
  double* out = elemR + 28 * (size_t)e;
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 7; ++r) out[7 * a + r] = R[a][r];
}

// ---- JacEval: a 32-lane team per element, lane j = column j of the element matrix ----------
// elems: the elements of one colour (no two share a vertex).  A wavefront holds two
// elements.  For each local row vertex a in turn, the two teams write block row a of their
// element matrices (columns j = 7 b + c of rows 7 a + r) to the wavefront's LDS stage, and
// the wavefront then adds the stage to the blocks (a, b) of J on equation rows, 49
// consecutive entries per block, so that consecutive lanes update consecutive doubles.
template <int KIND>
__global__ void __launch_bounds__(256) k_elem_jac(PhysDev P, int nel, const int32_t* __restrict__ elems,
                                                  const int32_t* __restrict__ tets, const double* __restrict__ X,
                                                  const double* __restrict__ y, const double* __restrict__ yold,
                                                  const double* __restrict__ bf, const int32_t* __restrict__ elem_blk,
                                                  const uint8_t* __restrict__ rowkind, double* __restrict__ vals,
                                                  int32_t* __restrict__ flags) {
  __shared__ double stage[4][2 * 4 * 49];  // per wavefront: [element of the pair][b][7 r + c]
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = gt >> 5;
  const int j = gt & 31;
  const int lane = threadIdx.x & 63, half = lane >> 5, wv = threadIdx.x >> 6;
  const bool live = t < nel;
  const int e = live ? elems[t] : 0;
  double Xe[4][3], yo[4][7], fe[4][3];
  int vid[4];
  DN R[4][7];
  if (live) {
    load_elem<KIND>(e, tets, X, yold, bf, Xe, yo, fe, vid);
    DN ye[4][7];
    for (int a = 0; a < 4; ++a)
      for (int r = 0; r < 7; ++r) ye[a][r] = DN{y[7 * (size_t)vid[a] + r], (7 * a + r == j) ? 1.0 : 0.0};
    bool ok = KIND == 0 ? fluid_elem<DN>(P, Xe, ye, yo, fe, R) : solid_elem<DN>(P, Xe, ye, yo, fe, R);
    if (!ok && j == 0) atomicOr(&flags[0], 1);
  }
  // scatter metadata of the wavefront's two elements: their 16 blocks of J and, per local
  // row vertex a and row r, whether that row is an equation row
  __shared__ int mblk[4][2][16];
  __shared__ int mrow[4][2][4][8];
  const int t0 = (gt >> 6) << 1;  // first element of this wavefront
  {
    const int el = lane >> 5, k = lane & 31;
    const int tt = t0 + el;
    if (tt < nel) {
      const int ee = elems[tt];
      if (k < 16) mblk[wv][el][k] = elem_blk[16 * (size_t)ee + k];
      if (k < 28) {
        const int a = k / 7, r = k - 7 * a;
        mrow[wv][el][a][r] = rowkind[7 * (size_t)tets[4 * (size_t)ee + a] + r] == RK_ELEM;
      }
    } else {
      if (k < 28) mrow[wv][el][k / 7][k % 7] = 0;
      if (k < 16) mblk[wv][el][k] = 0;
    }
  }
  double* st = stage[wv];
  for (int a = 0; a < 4; ++a) {
    if (live && j < 28) {
      const int b = j / 7, c = j - 7 * b;
#pragma unroll
      for (int r = 0; r < 7; ++r) st[half * 196 + b * 49 + 7 * r + c] = R[a][r].t;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // 392 entries (two elements x four blocks x 49) over the 64 lanes: all loads first
    size_t off[7];
    bool use[7];
    double v[7];
#pragma unroll
    for (int it = 0; it < 7; ++it) {
      const int idx = lane + 64 * it < 392 ? lane + 64 * it : 0;  // past the end: entry 0, unused
      const int el = idx >= 196, rem = idx - 196 * el, b = rem / 49, ent = rem - 49 * b, r = ent / 7;
      use[it] = lane + 64 * it < 392 && mrow[wv][el][a][r];
      off[it] = 49 * (size_t)mblk[wv][el][4 * a + b] + ent;
      v[it] = use[it] ? vals[off[it]] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < 7; ++it)
      if (use[it]) vals[off[it]] = v[it] + st[lane + 64 * it];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ---- gathers ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_res_gather(int64_t n, const uint8_t* __restrict__ rowkind,
                                                    const int32_t* __restrict__ vinc_ptr,
                                                    const int32_t* __restrict__ vinc,
                                                    const double* __restrict__ elemR, const double* __restrict__ y,
                                                    const double* __restrict__ gval, const double* __restrict__ yold,
                                                    double dt, double* __restrict__ F) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = (int)(i / 7), r = (int)(i % 7);
  double out;
  switch (rowkind[i]) {
    case RK_DIR: out = y[i] - gval[i]; break;
    case RK_DUMMY: out = y[i]; break;
    case RK_KIN: out = (y[i] - yold[i]) - dt * y[i - 4]; break;
    default: {
      double acc = 0.0;
      for (int p = vinc_ptr[a]; p < vinc_ptr[a + 1]; ++p) {
        int code = vinc[p];
        acc += elemR[28 * (size_t)(code >> 2) + 7 * (code & 3) + r];
      }
      out = acc;
    }
  }
  F[i] = out;
}

// Before the element launches: 0 on equation rows, the nodal rows' entries elsewhere
// (identity on Dirichlet and dummy rows; d - dt u on kinematic rows, scaled as F).
__global__ void __launch_bounds__(256) k_jac_init(int64_t nnzb, const int32_t* __restrict__ blkrow,
                                                  const int32_t* __restrict__ colind,
                                                  const uint8_t* __restrict__ rowkind, double dt,
                                                  double* __restrict__ vals) {
  const int64_t n = nnzb * 49, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < n; gid += stride) {
    const int64_t k = gid / 49;
    const int ent = (int)(gid - 49 * k), r = ent / 7, c = ent % 7;
    const int a = blkrow[k];
    const uint8_t kind = rowkind[7 * (size_t)a + r];
    double out = 0.0;
    if (kind != RK_ELEM && colind[k] == a) {
      if (kind == RK_KIN) out = (c == r) ? 1.0 : (c == r - 4 ? -dt : 0.0);
      else out = (c == r) ? 1.0 : 0.0;
    }
    vals[gid] = out;
  }
}

__global__ void k_impose(int64_t n, const uint8_t* __restrict__ rowkind, const double* __restrict__ gval,
                         double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint8_t k = rowkind[i];
  if (k == RK_DIR) y[i] = gval[i];
  else if (k == RK_DUMMY) y[i] = 0.0;
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
// Per-entry launches (49 per block) stride over a capped grid: a dispatch packet holds the
// grid size as a 32-bit count of work-items.
static inline unsigned nblk_stride(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < (int64_t(1) << 20) ? (b > 0 ? b : 1) : (int64_t(1) << 20));
}

hipError_t launch_impose(fsi_solver* s, double* y) {
  if (s->n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_impose, dim3(nblk(s->n, 256)), dim3(256), 0, s->stream, s->n, s->rowkind, s->gval, y);
  return hipGetLastError();
}

hipError_t launch_residual(fsi_solver* s, const double* y, double* F) {
  const PhysDev P = phys_dev(s);
  const int nf = (int)s->h.fluid_elems.size(), nsd = (int)s->h.solid_elems.size();
  const double* bf = s->has_bforce ? s->bforce : nullptr;
  if (nf > 0)
    FSI_PROF_LAUNCH(s, "elem_res_fluid",
                    hipLaunchKernelGGL(k_elem_res<0>, dim3(nblk(nf, 256)), dim3(256), 0, s->stream, P, nf,
                                       s->fluid_elems, s->tets, s->X, y, s->yold, bf, s->elemR, s->flags));
  if (nsd > 0)
    FSI_PROF_LAUNCH(s, "elem_res_solid",
                    hipLaunchKernelGGL(k_elem_res<1>, dim3(nblk(nsd, 256)), dim3(256), 0, s->stream, P, nsd,
                                       s->solid_elems, s->tets, s->X, y, s->yold, bf, s->elemR, s->flags));
  FSI_PROF_LAUNCH(s, "res_gather",
                  hipLaunchKernelGGL(k_res_gather, dim3(nblk(s->n, 256)), dim3(256), 0, s->stream, s->n,
                                     s->rowkind, s->vinc_ptr, s->vinc, s->elemR, y, s->gval, s->yold, s->dt, F));
  return hipGetLastError();
}

hipError_t launch_jacobian(fsi_solver* s, const double* y) {
  const PhysDev P = phys_dev(s);
  const double* bf = s->has_bforce ? s->bforce : nullptr;
  FSI_PROF_LAUNCH(s, "jac_init",
                  hipLaunchKernelGGL(k_jac_init, dim3(nblk_stride(s->nnzb * 49)), dim3(256), 0, s->stream, s->nnzb,
                                     s->blkrow, s->colind, s->rowkind, s->dt, s->vals));
  // one launch per colour, fluid colours then wall colours
  const std::vector<int32_t>& fc = s->h.fluid_col;
  for (size_t c = 0; c + 1 < fc.size(); ++c) {
    const int n = fc[c + 1] - fc[c];
    if (n > 0)
      FSI_PROF_LAUNCH(s, "elem_jac_fluid",
                      hipLaunchKernelGGL(k_elem_jac<0>, dim3(nblk((int64_t)n * 32, 256)), dim3(256), 0, s->stream, P,
                                         n, s->fluid_celems + fc[c], s->tets, s->X, y, s->yold, bf, s->elem_blk,
                                         s->rowkind, s->vals, s->flags));
  }
  const std::vector<int32_t>& sc = s->h.solid_col;
  for (size_t c = 0; c + 1 < sc.size(); ++c) {
    const int n = sc[c + 1] - sc[c];
    if (n > 0)
      FSI_PROF_LAUNCH(s, "elem_jac_solid",
                      hipLaunchKernelGGL(k_elem_jac<1>, dim3(nblk((int64_t)n * 32, 256)), dim3(256), 0, s->stream, P,
                                         n, s->solid_celems + sc[c], s->tets, s->X, y, s->yold, bf, s->elem_blk,
                                         s->rowkind, s->vals, s->flags));
  }
  return hipGetLastError();
}

}  // namespace fsi
