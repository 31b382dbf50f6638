// Internal declarations of the FP64 oracle (test infrastructure only; see fsio.h).
#pragma once
#include <cmath>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "fsio.h"

namespace fsio {

// ---------------------------------------------------------------------------------------
// Scalars.  The residual is written once, templated on the scalar type:
//   double            -> F(y)
//   Dual<N>           -> F(y) and N directional derivatives (forward mode), giving the
//                        exact Jacobian of the element residual (paper §3: the Jacobian
//                        is exact, not a finite-difference approximation)
//   std::complex      -> complex-step derivative checks
// ---------------------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
};
template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r; }
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> inline Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> inline Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { a = a - b; return a; }
template <int N> inline Dual<N> sqrt(const Dual<N>& a) {
  Dual<N> r; r.v = std::sqrt(a.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / (2.0 * r.v); return r; }

// Counting scalar (measurement only): a value that counts the arithmetic done on it and
// knows whether it depends on the element's unknowns.  value: operations of one plain
// evaluation; tangent: operations each forward-mode direction adds (a + b and a * c with
// one dependent operand: 1 and 1; a * b with both dependent: 3; a / b: 1 if only a
// depends, 2 if only b, 3 if both; sqrt: 1 per direction).  Unary minus is not counted.
struct OpCount {
  int64_t value = 0, tangent = 0;
};
extern thread_local OpCount g_ops;
struct Fl {
  double v;
  bool dep;
  Fl() : v(0.0), dep(false) {}
  Fl(double x, bool d = false) : v(x), dep(d) {}
};
inline Fl fl_add(const Fl& a, const Fl& b, double v) {
  g_ops.value++;
  if (a.dep && b.dep) g_ops.tangent++;
  return Fl(v, a.dep || b.dep);
}
inline Fl operator+(const Fl& a, const Fl& b) { return fl_add(a, b, a.v + b.v); }
inline Fl operator-(const Fl& a, const Fl& b) { return fl_add(a, b, a.v - b.v); }
inline Fl operator-(const Fl& a) { return Fl(-a.v, a.dep); }
inline Fl operator*(const Fl& a, const Fl& b) {
  g_ops.value++;
  g_ops.tangent += (a.dep && b.dep) ? 3 : (a.dep || b.dep) ? 1 : 0;
  return Fl(a.v * b.v, a.dep || b.dep);
}
inline Fl operator/(const Fl& a, const Fl& b) {
  g_ops.value++;
  g_ops.tangent += (a.dep && b.dep) ? 3 : b.dep ? 2 : a.dep ? 1 : 0;
  return Fl(a.v / b.v, a.dep || b.dep);
}
inline Fl operator+(const Fl& a, double b) { return a + Fl(b); }
inline Fl operator+(double a, const Fl& b) { return Fl(a) + b; }
inline Fl operator-(const Fl& a, double b) { return a - Fl(b); }
inline Fl operator-(double a, const Fl& b) { return Fl(a) - b; }
inline Fl operator*(const Fl& a, double b) { return a * Fl(b); }
inline Fl operator*(double a, const Fl& b) { return Fl(a) * b; }
inline Fl operator/(const Fl& a, double b) { return a / Fl(b); }
inline Fl operator/(double a, const Fl& b) { return Fl(a) / b; }
inline Fl& operator+=(Fl& a, const Fl& b) { a = a + b; return a; }
inline Fl& operator-=(Fl& a, const Fl& b) { a = a - b; return a; }
inline Fl sqrt(const Fl& a) {
  g_ops.value++;
  if (a.dep) g_ops.tangent++;
  return Fl(std::sqrt(a.v), a.dep);
}
inline double val(const Fl& x) { return x.v; }

inline double val(double x) { return x; }
inline double val(const std::complex<double>& x) { return x.real(); }
template <int N> inline double val(const Dual<N>& x) { return x.v; }
using std::sqrt;

typedef Dual<28> D28;
typedef std::complex<double> Cplx;

// ---------------------------------------------------------------------------------------
// Data
// ---------------------------------------------------------------------------------------
enum VKind : int8_t { V_FLUID = 0, V_IFACE = 1, V_SOLID = 2 };
enum RowKind : uint8_t { ROW_ELEM = 0, ROW_DIR = 1, ROW_KIN = 2, ROW_DUMMY = 3 };

struct Bsr {
  int nb = 0;                 // block rows
  std::vector<int> rowptr, colind;
  std::vector<double> vals;   // [nnzb][7][7] row-major
  int find(int a, int b) const;  // block index of (a,b) or -1
};

struct Sub {
  std::vector<int> verts;     // local -> global vertex, reverse Cuthill-McKee order
  std::vector<char> owned;    // local vertex is in the non-overlapping part
  int nowned = 0;
  std::vector<int> rowptr, colind, src, diag;
  std::vector<double> f;      // factors: strict L (unit), strict U, inverse diagonal blocks
  std::vector<double> udiag;  // U_ii before inversion (kept for the LU = A pin)
  int nlevels = 0;
};

struct Phys { double rho_f, mu_f, rho_s, E_s, nu_s, eta_s, C_I; };

}  // namespace fsio

struct fsio_solver {
  int V = 0, E = 0, B = 0;
  std::vector<double> X;
  std::vector<int> tets;
  std::vector<int8_t> dom;
  std::vector<int> bfaces;
  std::vector<int8_t> btag;
  fsio::Phys ph{};
  fsio_opts opts{};
  std::vector<int> part;

  // topology
  std::vector<int8_t> vkind;
  std::vector<uint8_t> rowkind_base, forced_zero;
  std::vector<int> iface_faces;
  fsio::Bsr J;

  // step
  bool has_step = false;
  double t = 0.0, dt = 0.0;
  std::vector<double> yold, gval, bforce;
  std::vector<uint8_t> rowkind;

  // preconditioner
  std::vector<fsio::Sub> subs;
  bool pc_ready = false;
  bool jac_ready = false;

  std::string err;
};

namespace fsio {
int build_topology(fsio_solver& s);
void set_rowkinds(fsio_solver& s, const uint8_t* extra_mask);

int residual(fsio_solver& s, const double* y, double* F);
int residual_complex(fsio_solver& s, const Cplx* y, Cplx* F);
int jacobian(fsio_solver& s, const double* y);
int element(fsio_solver& s, const double* y, int e, double* Re, double* Je);
int element_ops(fsio_solver& s, const double* y, int e, int64_t* value_ops, int64_t* tangent_ops);

void rcb_partition(const fsio_solver& s, int nsub, std::vector<int>& part);
int build_subdomains(fsio_solver& s);
int pc_setup(fsio_solver& s);
void pc_apply(const fsio_solver& s, const double* v, double* z);
void spmv(const fsio_solver& s, const double* x, double* y);
int invert7(const double* A, double* Ainv);

int gmres(fsio_solver& s, const double* b, double* x, fsio_lin_stats* st, double* t_pcapply);
int newton(fsio_solver& s, double* y, fsio_step_stats* st);
}  // namespace fsio
