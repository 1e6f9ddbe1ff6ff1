// MQCT reference oracle: a plain, slow, FP64 CPU implementation of batched
// Ehrenfest mean-field trajectory propagation.  TEST INFRASTRUCTURE ONLY: it is
// used by the test-suite, by the smoke check and by the benchmark's CPU
// baseline, never by the product path, and it shares no code with the GPU
// library.
//
// What it computes (paper Section II):
//   * interaction-picture amplitudes a_n (Eq. 4) obeying
//       da_n/dt = -i sum_m M_nm(R) exp(i (E_n - E_m) t) a_m  - i Phidot (J_x a)_n     (Eq. 5)
//     where M is the coupling matrix (Eq. 6), tabulated on an R grid and
//     interpolated with a cubic spline (Section III), and J_x is the Coriolis
//     operator whose matrix elements are the square-root factors of Eq. 5.  The
//     printed Coriolis term carries no factor i; the unitary, energy-conserving
//     reading -i Phidot J_x is used (the sign is fixed by energy conservation,
//     stated at the end of Section II);
//   * classical R, Theta, Phi, P_R, P_Theta, P_Phi (Eqs. 7-10), restricted to
//     the plane Theta = pi/2 (end of Section II):
//       dR/dt = P_R/mu, dPhi/dt = P_Phi/(mu R^2)                                  (Eqs. 7, 8)
//       dP_R/dt = -sum_nm exp(i(E_n-E_m)t) M'_nm a_n^* a_m + P_Phi^2/(mu R^3)     (Eq. 9)
//       dP_Phi/dt = -i <[J_x, V]>                                                 (Eq. 10)
//   * fixed-step classical RK4 and adaptive Dormand-Prince 5(4) (published
//     tableau, Dormand & Prince 1980) as the time steppers;
//   * final probabilities |a_n|^2 and Monte-Carlo cross sections (end of
//     Section II: summed over final, averaged over initial degenerate states).
//
// Everything is templated on the scalar so that the same code, run on a dual
// number, yields the exact forward-mode derivative of the discrete RK4 map
// (used to check the adjoint).
//
// Pins (tests/test_oracle_*.py): natural-spline values against scipy, the Rabi
// closed form, the frozen-trajectory matrix exponential, free straight-line
// motion with Wigner-d Coriolis populations, norm / energy / angular-momentum
// invariants, RK4 convergence order, an independent DOP853 integration,
// scipy's RK45 (the same Dormand-Prince pair and controller) step for step, the
// h^5 scaling of the embedded error estimate, m-reflection symmetry, the literal-phase form, and the dual-number derivative
// against finite differences.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

namespace {

// ---------------------------------------------------------------- scalars
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual sin(Dual a) { return Dual(std::sin(a.v), std::cos(a.v) * a.d); }
inline Dual cos(Dual a) { return Dual(std::cos(a.v), -std::sin(a.v) * a.d); }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, 0.5 * a.d / s); }
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
using std::sin; using std::cos; using std::sqrt;

template <class T> struct Cx { T re, im; };
template <class T> inline Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> inline Cx<T> conjmul(Cx<T> a, Cx<T> b) {   // conj(a) * b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <class T> inline Cx<T> expi(T phi) { return {cos(phi), sin(phi)}; }

}  // namespace

// ---------------------------------------------------------------- system
extern "C" {

typedef struct {
  int32_t N, K;
  const double* R;        // [K] bohr, strictly increasing
  const double* E;        // [N] hartree
  const double* M;        // [K][N][N][2] coupling tables, complex interleaved (hartree)
  const double* M2;       // [K][N][N][2] natural-spline second derivatives of M
  const double* dM;       // optional tangent tables (same layout) for forward mode, or NULL
  const double* dM2;      // their second derivatives
  int32_t jx_nnz;
  const int32_t* jx_row;
  const int32_t* jx_col;
  const double* jx_val;   // J_x coordinate list (real symmetric)
  double mu;              // reduced mass, m_e
  int32_t literal_phase;  // 1: form exp(i(E_n - E_m)t) per element instead of factorising
  int32_t plant_coriolis_flip;  // tests only: 1 plants the wrong sign +i Phidot J_x in Eq. 5
  // Decoupled (AT) dynamics (Section III: the quantum equations, Eq. 5, are
  // propagated along a classical trajectory whose Eqs. 7-10 no longer feel the
  // quantum state).  The trajectory is driven by the tabulated potential U(R):
  //   dP_R/dt = -U'(R) + P_Phi^2/(mu R^3),   dP_Phi/dt = 0.
  int32_t decoupled;      // 1: AT dynamics (needs drv, drv2)
  const double* drv;      // [K] U(R_k), hartree
  const double* drv2;     // [K] its natural-spline second derivatives
} oracle_system;

enum { OR_EXITED = 1, OR_MAX_STEPS = 2, OR_STEP_UNDERFLOW = 4, OR_BELOW_GRID = 8,
       OR_NONFINITE = 16 };

// Natural cubic spline second derivatives for ncol independent columns of
// y[K][ncol] on knots x[K] (textbook tridiagonal system with zero end
// curvature, solved by forward elimination and back substitution).
void oracle_spline_prepare(int32_t K, const double* x, int64_t ncol, const double* y,
                           double* y2) {
  std::vector<double> diag(K), rhs(K), cprime(K);
  for (int64_t col = 0; col < ncol; ++col) {
    for (int k = 0; k < K; ++k) y2[(int64_t)k * ncol + col] = 0.0;
    if (K < 3) continue;
    // unknowns y2[1..K-2]
    for (int k = 1; k <= K - 2; ++k) {
      double hl = x[k] - x[k - 1], hr = x[k + 1] - x[k];
      double yl = y[(int64_t)(k - 1) * ncol + col], yc = y[(int64_t)k * ncol + col],
             yr = y[(int64_t)(k + 1) * ncol + col];
      diag[k] = (hl + hr) / 3.0;
      rhs[k] = (yr - yc) / hr - (yc - yl) / hl;
    }
    // forward elimination: sub-diagonal h_{k-1}/6, super-diagonal h_k/6
    for (int k = 1; k <= K - 2; ++k) {
      double sub = (x[k] - x[k - 1]) / 6.0;
      double sup = (x[k + 1] - x[k]) / 6.0;
      double den = diag[k];
      double r = rhs[k];
      if (k > 1) {
        den -= sub * cprime[k - 1];
        r -= sub * rhs[k - 1];
      }
      cprime[k] = sup / den;
      rhs[k] = r / den;
    }
    double nxt = 0.0;
    for (int k = K - 2; k >= 1; --k) {
      double v = rhs[k] - cprime[k] * nxt;
      y2[(int64_t)k * ncol + col] = v;
      nxt = v;
    }
  }
}

}  // extern "C"

namespace {

// Interval and weights of the spline at R: value = wa y_k + wb y_{k+1} + wc y2_k + wd y2_{k+1},
// derivative likewise with the d-weights.  Off-grid rule: above the last knot the
// value is held and the slope is zero; below the first knot the spline is
// continued linearly and the caller is told.
template <class T> struct SplineW {
  int k;
  T wa, wb, wc, wd;     // value weights
  T da, db, dc, dd;     // derivative weights
  bool below;
};

template <class T> SplineW<T> spline_weights(int K, const double* x, T R) {
  SplineW<T> w;
  double r = val(R);
  w.below = r < x[0];
  if (r > x[K - 1]) {
    w.k = K - 2;
    w.wa = T(0.0); w.wb = T(1.0); w.wc = T(0.0); w.wd = T(0.0);
    w.da = T(0.0); w.db = T(0.0); w.dc = T(0.0); w.dd = T(0.0);
    return w;
  }
  int k;
  if (w.below) {
    k = 0;
  } else {
    k = int(std::upper_bound(x, x + K, r) - x) - 1;
    if (k > K - 2) k = K - 2;
    if (k < 0) k = 0;
  }
  w.k = k;
  double h = x[k + 1] - x[k];
  if (w.below) {
    // value and slope at x[0] (A = 1, B = 0), continued linearly
    T s = R - T(x[0]);
    w.da = T(-1.0 / h); w.db = T(1.0 / h);
    w.dc = T(-(3.0 * 1.0 - 1.0) * h / 6.0); w.dd = T((3.0 * 0.0 - 1.0) * h / 6.0);
    w.wa = T(1.0) + s * w.da; w.wb = s * w.db; w.wc = s * w.dc; w.wd = s * w.dd;
    return w;
  }
  T A = (T(x[k + 1]) - R) / T(h);
  T B = T(1.0) - A;
  w.wa = A; w.wb = B;
  w.wc = (A * A * A - A) * T(h * h / 6.0);
  w.wd = (B * B * B - B) * T(h * h / 6.0);
  w.da = T(-1.0 / h); w.db = T(1.0 / h);
  w.dc = -(T(3.0) * A * A - T(1.0)) * T(h / 6.0);
  w.dd = (T(3.0) * B * B - T(1.0)) * T(h / 6.0);
  return w;
}

// One table element (complex) of a tabulated quantity at the weights.
template <class T> struct Elem { Cx<T> val, der; };

template <class T>
inline Elem<T> table_elem(const oracle_system* s, const SplineW<T>& w, int64_t n, int64_t m);

template <>
inline Elem<double> table_elem<double>(const oracle_system* s, const SplineW<double>& w,
                                       int64_t n, int64_t m) {
  const int64_t NN = (int64_t)s->N * s->N;
  const int64_t o0 = ((int64_t)w.k * NN + n * s->N + m) * 2;
  const int64_t o1 = o0 + NN * 2;
  Elem<double> e;
  e.val.re = w.wa * s->M[o0] + w.wb * s->M[o1] + w.wc * s->M2[o0] + w.wd * s->M2[o1];
  e.val.im = w.wa * s->M[o0 + 1] + w.wb * s->M[o1 + 1] + w.wc * s->M2[o0 + 1] + w.wd * s->M2[o1 + 1];
  e.der.re = w.da * s->M[o0] + w.db * s->M[o1] + w.dc * s->M2[o0] + w.dd * s->M2[o1];
  e.der.im = w.da * s->M[o0 + 1] + w.db * s->M[o1 + 1] + w.dc * s->M2[o0 + 1] + w.dd * s->M2[o1 + 1];
  return e;
}

template <>
inline Elem<Dual> table_elem<Dual>(const oracle_system* s, const SplineW<Dual>& w, int64_t n,
                                   int64_t m) {
  const int64_t NN = (int64_t)s->N * s->N;
  const int64_t o0 = ((int64_t)w.k * NN + n * s->N + m) * 2;
  const int64_t o1 = o0 + NN * 2;
  auto g = [&](const double* Y, const double* Y2, const double* dY, const double* dY2,
               int64_t off) {
    Dual y0(Y[off], dY ? dY[off] : 0.0), y1(Y[off + NN * 2], dY ? dY[off + NN * 2] : 0.0);
    Dual z0(Y2[off], dY2 ? dY2[off] : 0.0), z1(Y2[off + NN * 2], dY2 ? dY2[off + NN * 2] : 0.0);
    Dual v = w.wa * y0 + w.wb * y1 + w.wc * z0 + w.wd * z1;
    Dual d = w.da * y0 + w.db * y1 + w.dc * z0 + w.dd * z1;
    return std::pair<Dual, Dual>(v, d);
  };
  (void)o1;
  Elem<Dual> e;
  auto re = g(s->M, s->M2, s->dM, s->dM2, o0);
  auto im = g(s->M, s->M2, s->dM, s->dM2, o0 + 1);
  e.val.re = re.first; e.der.re = re.second;
  e.val.im = im.first; e.der.im = im.second;
  return e;
}

// State layout y[2N + 6]: a_n as (re, im) pairs, then R, Theta, Phi, P_R, P_Theta, P_Phi.
// Eq: the quantum energy <H_rot + V>; U: the driving potential (AT dynamics).
template <class T> struct Diag { T Eq; T U; bool below; };

// Right-hand side of Eqs. 5 and 7-10.
template <class T>
Diag<T> rhs(const oracle_system* s, T t, const T* y, T* f) {
  const int N = s->N;
  const T* a = y;
  T R = y[2 * N + 0], PR = y[2 * N + 3], PPh = y[2 * N + 5];
  T mu = T(s->mu);
  SplineW<T> w = spline_weights<T>(s->K, s->R, R);
  T Phidot = PPh / (mu * R * R);

  std::vector<Cx<T>> amp(N), xv(N), yv(N);
  for (int n = 0; n < N; ++n) amp[n] = {a[2 * n], a[2 * n + 1]};
  // x = J_x a
  for (int n = 0; n < N; ++n) xv[n] = {T(0.0), T(0.0)};
  for (int q = 0; q < s->jx_nnz; ++q) {
    int r = s->jx_row[q], c = s->jx_col[q];
    xv[r].re += T(s->jx_val[q]) * amp[c].re;
    xv[r].im += T(s->jx_val[q]) * amp[c].im;
  }
  // y_n = sum_m M_nm e^{i(E_n - E_m)t} a_m ;  force = sum_nm e^{i(E_n-E_m)t} M'_nm a_n^* a_m
  std::vector<Cx<T>> c(N), em(N);
  for (int m = 0; m < N; ++m) {
    em[m] = expi<T>(T(-s->E[m]) * t);       // e^{-i E_m t}
    c[m] = cmul(em[m], amp[m]);
  }
  Cx<T> force = {T(0.0), T(0.0)};
  Cx<T> Vexp = {T(0.0), T(0.0)};
  for (int n = 0; n < N; ++n) {
    Cx<T> u = {T(0.0), T(0.0)}, v = {T(0.0), T(0.0)};
    for (int m = 0; m < N; ++m) {
      Elem<T> e = table_elem<T>(s, w, n, m);
      if (s->literal_phase) {
        Cx<T> ph = expi<T>(T(s->E[n] - s->E[m]) * t);
        Cx<T> t1 = cmul(cmul(e.val, ph), amp[m]);
        Cx<T> t2 = cmul(cmul(e.der, ph), amp[m]);
        u.re += t1.re; u.im += t1.im;
        v.re += t2.re; v.im += t2.im;
      } else {
        Cx<T> t1 = cmul(e.val, c[m]);
        Cx<T> t2 = cmul(e.der, c[m]);
        u.re += t1.re; u.im += t1.im;
        v.re += t2.re; v.im += t2.im;
      }
    }
    if (s->literal_phase) {
      yv[n] = u;
      Cx<T> fz = conjmul(amp[n], v);
      force.re += fz.re; force.im += fz.im;
      Cx<T> vz = conjmul(amp[n], u);
      Vexp.re += vz.re; Vexp.im += vz.im;
    } else {
      Cx<T> ep = {em[n].re, -em[n].im};   // e^{+i E_n t}
      yv[n] = cmul(ep, u);
      Cx<T> fz = conjmul(c[n], v);
      force.re += fz.re; force.im += fz.im;
      Cx<T> vz = conjmul(c[n], u);
      Vexp.re += vz.re; Vexp.im += vz.im;
    }
  }
  // da/dt = -i y - i Phidot x
  T cor = s->plant_coriolis_flip ? -Phidot : Phidot;
  for (int n = 0; n < N; ++n) {
    T gr = yv[n].re + cor * xv[n].re;
    T gi = yv[n].im + cor * xv[n].im;
    f[2 * n] = gi;          // -i (gr + i gi) = gi - i gr
    f[2 * n + 1] = -gr;
  }
  // torque: -i <[J_x, V]> = -i (x^H y - y^H x) = 2 Im(x^H y)
  Cx<T> xy = {T(0.0), T(0.0)};
  for (int n = 0; n < N; ++n) {
    Cx<T> z = conjmul(xv[n], yv[n]);
    xy.re += z.re; xy.im += z.im;
  }
  f[2 * N + 0] = PR / mu;
  f[2 * N + 1] = T(0.0);
  f[2 * N + 2] = Phidot;
  f[2 * N + 3] = -force.re + PPh * PPh / (mu * R * R * R);
  f[2 * N + 4] = T(0.0);
  f[2 * N + 5] = T(2.0) * xy.im;
  Diag<T> d;
  d.U = T(0.0);
  if (s->decoupled) {
    // AT: the trajectory feels only the driving potential; no torque
    const int k = w.k;
    T U = w.wa * T(s->drv[k]) + w.wb * T(s->drv[k + 1]) + w.wc * T(s->drv2[k]) +
          w.wd * T(s->drv2[k + 1]);
    T dU = w.da * T(s->drv[k]) + w.db * T(s->drv[k + 1]) + w.dc * T(s->drv2[k]) +
           w.dd * T(s->drv2[k + 1]);
    f[2 * N + 3] = -dU + PPh * PPh / (mu * R * R * R);
    f[2 * N + 5] = T(0.0);
    d.U = U;
  }
  T Erot = T(0.0);
  for (int n = 0; n < N; ++n) Erot += T(s->E[n]) * (amp[n].re * amp[n].re + amp[n].im * amp[n].im);
  d.Eq = Erot + Vexp.re;
  d.below = w.below;
  return d;
}

// Conserved energy: classical kinetic + quantum <H_rot + V> (Ehrenfest), or
// classical kinetic + U(R) (AT: the trajectory's own energy).
template <class T> T total_energy(const oracle_system* s, T t, const T* y) {
  int N = s->N;
  std::vector<T> f(2 * N + 6);
  Diag<T> d = rhs<T>(s, t, y, f.data());
  T R = y[2 * N], PR = y[2 * N + 3], PPh = y[2 * N + 5], mu = T(s->mu);
  return PR * PR / (T(2.0) * mu) + PPh * PPh / (T(2.0) * mu * R * R) +
         (s->decoupled ? d.U : d.Eq);
}

// Conserved angular momentum: P_Phi - Re(a^H J_x a) (Ehrenfest), or P_Phi (AT).
template <class T> T angular_invariant(const oracle_system* s, const T* y) {
  int N = s->N;
  if (s->decoupled) return y[2 * N + 5];
  T jx = T(0.0);
  for (int q = 0; q < s->jx_nnz; ++q) {
    int r = s->jx_row[q], c = s->jx_col[q];
    jx += T(s->jx_val[q]) * (y[2 * r] * y[2 * c] + y[2 * r + 1] * y[2 * c + 1]);
  }
  return y[2 * N + 5] - jx;
}

template <class T> bool finite_state(const T* y, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(val(y[i]))) return false;
  return true;
}

// Classical fourth-order Runge-Kutta, exactly n_steps steps of size h; t_j = t0 + j h.
template <class T>
int32_t rk4(const oracle_system* s, T* y, double t0, double h, int64_t n_steps) {
  const int n = 2 * s->N + 6;
  std::vector<T> k1(n), k2(n), k3(n), k4(n), tmp(n);
  int32_t status = 0;
  T hh = T(h);
  for (int64_t j = 0; j < n_steps; ++j) {
    T t = T(t0 + double(j) * h);
    Diag<T> d1 = rhs<T>(s, t, y, k1.data());
    for (int i = 0; i < n; ++i) tmp[i] = y[i] + T(0.5) * hh * k1[i];
    Diag<T> d2 = rhs<T>(s, t + T(0.5) * hh, tmp.data(), k2.data());
    for (int i = 0; i < n; ++i) tmp[i] = y[i] + T(0.5) * hh * k2[i];
    Diag<T> d3 = rhs<T>(s, t + T(0.5) * hh, tmp.data(), k3.data());
    for (int i = 0; i < n; ++i) tmp[i] = y[i] + hh * k3[i];
    Diag<T> d4 = rhs<T>(s, t + hh, tmp.data(), k4.data());
    for (int i = 0; i < n; ++i)
      y[i] = y[i] + hh / T(6.0) * (k1[i] + T(2.0) * k2[i] + T(2.0) * k3[i] + k4[i]);
    if (d1.below || d2.below || d3.below || d4.below) status |= OR_BELOW_GRID;
    if (!finite_state(y, n)) { status |= OR_NONFINITE; break; }
  }
  return status;
}

// Dormand-Prince 5(4) coefficients (Dormand & Prince 1980).
const double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
// fifth-order weights minus embedded fourth-order weights
const double DP_E[7] = {71.0 / 57600, 0.0, -71.0 / 16695, 71.0 / 1920, -17253.0 / 339200,
                        22.0 / 525, -1.0 / 40};

double rms_scaled(const std::vector<double>& e, const std::vector<double>& sc) {
  double acc = 0.0;
  for (size_t i = 0; i < e.size(); ++i) { double r = e[i] / sc[i]; acc += r * r; }
  return std::sqrt(acc / double(e.size()));
}

struct Dp5Result { int32_t status; int64_t steps, rejects; double t; };

// One Dormand-Prince 5(4) attempt of size h from (t, y), with k[0] = f(t, y)
// given: the stages k[1..6] (k[6] = f(t + h, ynew), first same as last), the
// fifth-order solution ynew, and the returned scaled RMS norm of the embedded
// error estimate h sum_q DP_E[q] k[q] with sc_i = atol + rtol max(|y_i|, |ynew_i|).
double dp5_attempt(const oracle_system* s, double t, const double* y, double h, double rtol,
                   double atol, std::vector<std::vector<double>>& k, std::vector<double>& ynew,
                   int32_t& status) {
  const int n = 2 * s->N + 6;
  std::vector<double> tmp(n), err(n), sc(n);
  for (int st = 1; st < 7; ++st) {
    for (int i = 0; i < n; ++i) {
      double acc = y[i];
      for (int q = 0; q < st; ++q) acc += h * DP_A[st][q] * k[q][i];
      tmp[i] = acc;
    }
    Diag<double> d = rhs<double>(s, t + DP_C[st] * h, tmp.data(), k[st].data());
    if (d.below) status |= OR_BELOW_GRID;
    if (st == 6) ynew = tmp;
  }
  for (int i = 0; i < n; ++i) {
    double e = 0.0;
    for (int q = 0; q < 7; ++q) e += DP_E[q] * k[q][i];
    err[i] = h * e;
    sc[i] = atol + rtol * std::max(std::fabs(y[i]), std::fabs(ynew[i]));
  }
  return rms_scaled(err, sc);
}

// Adaptive Dormand-Prince 5(4) with first-same-as-last, scaled RMS error norm
// sc_i = atol + rtol max(|y_i|, |y_new,i|), step factor min(5, max(0.2, 0.9 err^-1/5))
// (no growth right after a rejection), starting step from the Hairer-Norsett-Wanner
// heuristic.  Stops after the first accepted step with R >= R_exit and P_R > 0.
Dp5Result dp5(const oracle_system* s, double* y, double t0, double rtol, double atol,
              int64_t max_steps, double h_min, double R_exit) {
  const int n = 2 * s->N + 6;
  std::vector<std::vector<double>> k(7, std::vector<double>(n));
  std::vector<double> tmp(n), ynew(n), err(n), sc(n);
  Dp5Result res{0, 0, 0, t0};
  double t = t0;
  int32_t status = 0;
  Diag<double> dg = rhs<double>(s, t, y, k[0].data());
  if (dg.below) status |= OR_BELOW_GRID;
  // starting step
  for (int i = 0; i < n; ++i) sc[i] = atol + rtol * std::fabs(y[i]);
  double d0 = rms_scaled(std::vector<double>(y, y + n), sc);
  double d1 = rms_scaled(k[0], sc);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
  for (int i = 0; i < n; ++i) tmp[i] = y[i] + h0 * k[0][i];
  rhs<double>(s, t + h0, tmp.data(), k[1].data());
  for (int i = 0; i < n; ++i) err[i] = (k[1][i] - k[0][i]);
  double d2 = rms_scaled(err, sc) / h0;
  double dm = std::max(d1, d2);
  double h1 = dm <= 1e-15 ? std::max(1e-6, h0 * 1e-3) : std::pow(0.01 / dm, 1.0 / 5.0);
  double h = std::min(100.0 * h0, h1);
  bool last_rejected = false;
  for (;;) {
    if (res.steps >= max_steps) { status |= OR_MAX_STEPS; break; }
    double en = dp5_attempt(s, t, y, h, rtol, atol, k, ynew, status);
    if (!std::isfinite(en)) { status |= OR_NONFINITE; break; }
    if (en <= 1.0) {
      t += h;
      for (int i = 0; i < n; ++i) y[i] = ynew[i];
      k[0] = k[6];
      res.steps++;
      double fac = en == 0.0 ? 5.0 : std::min(5.0, std::max(0.2, 0.9 * std::pow(en, -0.2)));
      if (last_rejected) fac = std::min(1.0, fac);
      last_rejected = false;
      if (y[2 * s->N] >= R_exit && y[2 * s->N + 3] > 0.0) { status |= OR_EXITED; break; }
      h *= fac;
    } else {
      res.rejects++;
      h *= std::max(0.2, 0.9 * std::pow(en, -0.2));
      last_rejected = true;
    }
    if (h < h_min) { status |= OR_STEP_UNDERFLOW; break; }
  }
  res.status = status;
  res.t = t;
  return res;
}

// Initial classical state (end of Section II / Section III: impact parameter b,
// collision energy U at the starting separation R0, planar motion):
// P_Phi = b sqrt(2 mu U), P_R = -sqrt(2 mu U - P_Phi^2 / R0^2), Theta = pi/2, Phi = 0.
void initial_classical(double mu, double E_coll, double b, double R0, double* c6) {
  double k = std::sqrt(2.0 * mu * E_coll);
  double PPh = b * k;
  c6[0] = R0;
  c6[1] = 0.5 * M_PI;
  c6[2] = 0.0;
  c6[3] = -std::sqrt(2.0 * mu * E_coll - PPh * PPh / (R0 * R0));
  c6[4] = 0.0;
  c6[5] = PPh;
}

}  // namespace

#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

// Number of OpenMP threads a parallel region of the oracle uses.
int32_t oracle_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Evaluate the spline of ncol columns at r: value and derivative.  Returns 1 when
// r lies below the first knot (linear continuation), else 0.
int32_t oracle_spline_eval(int32_t K, const double* x, int64_t ncol, const double* y,
                           const double* y2, double r, double* value, double* deriv) {
  SplineW<double> w = spline_weights<double>(K, x, r);
  for (int64_t c = 0; c < ncol; ++c) {
    const int64_t o0 = (int64_t)w.k * ncol + c, o1 = o0 + ncol;
    value[c] = w.wa * y[o0] + w.wb * y[o1] + w.wc * y2[o0] + w.wd * y2[o1];
    deriv[c] = w.da * y[o0] + w.db * y[o1] + w.dc * y2[o0] + w.dd * y2[o1];
  }
  return w.below ? 1 : 0;
}

// Right-hand side at (t, y); also returns the quantum energy <H_rot + V>.
double oracle_rhs(const oracle_system* s, double t, const double* y, double* f) {
  return rhs<double>(s, t, y, f).Eq;
}

// Scaled RMS norm of the embedded error estimate of one Dormand-Prince 5(4)
// attempt of size h from (t, y); ynew (may be NULL) receives the fifth-order
// solution.
double oracle_dp5_error(const oracle_system* s, double t, const double* y, double h, double rtol,
                        double atol, double* ynew) {
  const int n = 2 * s->N + 6;
  std::vector<std::vector<double>> k(7, std::vector<double>(n));
  std::vector<double> yn(n);
  int32_t status = 0;
  rhs<double>(s, t, y, k[0].data());
  double en = dp5_attempt(s, t, y, h, rtol, atol, k, yn, status);
  if (ynew) for (int i = 0; i < n; ++i) ynew[i] = yn[i];
  return en;
}

double oracle_total_energy(const oracle_system* s, double t, const double* y) {
  return total_energy<double>(s, t, y);
}

// Batch propagation.  Per trajectory b:
//   initial state: a0 [B][N][2] if given else a = e_{init_channel[b]};
//                  classical0 [B][6] if given else built from (E_coll, bparam, R0);
//   t0 [B] or NULL (0);
//   method 0 = RK4 with dt[b], n_steps[b]; 1 = DP5 (rtol, atol, max_steps, h_min),
//   exiting at R >= R0 with P_R > 0.
// Outputs (NULL allowed except P): P [B][N], a_final [B][N][2], classical [B][6],
// t_final, steps, rejects, status, norm_err, energy_err (relative), angmom_err.
// OpenMP parallel over trajectories.
int32_t oracle_propagate(const oracle_system* s, int64_t B, const int32_t* init_channel,
                         const double* a0, const double* classical0, const double* E_coll,
                         const double* bparam, const double* R0, const double* t0,
                         int32_t method, const double* dt, const int64_t* n_steps,
                         double rtol, double atol, int64_t max_steps, double h_min,
                         double* P, double* a_final, double* classical, double* t_final,
                         int64_t* steps, int64_t* rejects, int32_t* status, double* norm_err,
                         double* energy_err, double* angmom_err) {
  const int N = s->N;
  const int n = 2 * N + 6;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < B; ++b) {
    std::vector<double> y(n, 0.0);
    if (a0) {
      for (int i = 0; i < 2 * N; ++i) y[i] = a0[b * 2 * N + i];
    } else {
      y[2 * init_channel[b]] = 1.0;
    }
    double c6[6];
    if (classical0) {
      for (int i = 0; i < 6; ++i) c6[i] = classical0[b * 6 + i];
    } else {
      initial_classical(s->mu, E_coll[b], bparam[b], R0 ? R0[b] : s->R[s->K - 1], c6);
    }
    for (int i = 0; i < 6; ++i) y[2 * N + i] = c6[i];
    double tstart = t0 ? t0[b] : 0.0;
    double E0 = total_energy<double>(s, tstart, y.data());
    double J0 = angular_invariant<double>(s, y.data());
    int32_t st;
    int64_t nst = 0, nrej = 0;
    double tend;
    if (method == 0) {
      st = rk4<double>(s, y.data(), tstart, dt[b], n_steps[b]);
      nst = n_steps[b];
      tend = tstart + double(n_steps[b]) * dt[b];
    } else {
      Dp5Result r = dp5(s, y.data(), tstart, rtol, atol, max_steps, h_min, c6[0]);
      st = r.status; nst = r.steps; nrej = r.rejects; tend = r.t;
    }
    double nrm = 0.0;
    for (int i = 0; i < N; ++i) {
      double p = y[2 * i] * y[2 * i] + y[2 * i + 1] * y[2 * i + 1];
      P[b * N + i] = p;
      nrm += p;
    }
    if (a_final) for (int i = 0; i < 2 * N; ++i) a_final[b * 2 * N + i] = y[i];
    if (classical) for (int i = 0; i < 6; ++i) classical[b * 6 + i] = y[2 * N + i];
    if (t_final) t_final[b] = tend;
    if (steps) steps[b] = nst;
    if (rejects) rejects[b] = nrej;
    if (status) status[b] = st;
    if (norm_err) norm_err[b] = nrm - 1.0;
    if (energy_err) energy_err[b] = (total_energy<double>(s, tend, y.data()) - E0) / std::fabs(E0);
    if (angmom_err) angmom_err[b] = angular_invariant<double>(s, y.data()) - J0;
  }
  return 0;
}

// Forward-mode derivative of the discrete RK4 map along one tangent direction of
// the tables (s->dM, s->dM2 hold dM/d(direction) at the knots and its spline
// second derivatives).  Returns P [B][N] and dP [B][N].
int32_t oracle_tangent_rk4(const oracle_system* s, int64_t B, const int32_t* init_channel,
                           const double* E_coll, const double* bparam, const double* R0,
                           const double* dt, const int64_t* n_steps, double* P, double* dP) {
  const int N = s->N;
  const int n = 2 * N + 6;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < B; ++b) {
    std::vector<Dual> y(n, Dual(0.0));
    y[2 * init_channel[b]] = Dual(1.0);
    double c6[6];
    initial_classical(s->mu, E_coll[b], bparam[b], R0 ? R0[b] : s->R[s->K - 1], c6);
    for (int i = 0; i < 6; ++i) y[2 * N + i] = Dual(c6[i]);
    rk4<Dual>(s, y.data(), 0.0, dt[b], n_steps[b]);
    for (int i = 0; i < N; ++i) {
      Dual p = y[2 * i] * y[2 * i] + y[2 * i + 1] * y[2 * i + 1];
      P[b * N + i] = p.v;
      dP[b * N + i] = p.d;
    }
  }
  return 0;
}

// Monte-Carlo cross sections (bohr^2):
//   sigma[L'][L''] = (2 pi b_max / N_L') sum_{i : level(i) = L'} b_i sum_{n in L''} P_i(n)
// with N_L' the number of trajectories started in level L'.  Trajectories share
// one channel-to-level map of length N.
int32_t oracle_cross_sections(int64_t B, int32_t N, const int32_t* init_level,
                              const double* bparam, const double* P,
                              const int32_t* level_of_channel, int32_t n_levels, double b_max,
                              double* sigma) {
  std::vector<double> count(n_levels, 0.0);
  for (int64_t i = 0; i < (int64_t)n_levels * n_levels; ++i) sigma[i] = 0.0;
  for (int64_t b = 0; b < B; ++b) {
    count[init_level[b]] += 1.0;
    for (int nn = 0; nn < N; ++nn)
      sigma[(int64_t)init_level[b] * n_levels + level_of_channel[nn]] += bparam[b] * P[b * N + nn];
  }
  for (int L = 0; L < n_levels; ++L)
    for (int L2 = 0; L2 < n_levels; ++L2)
      sigma[(int64_t)L * n_levels + L2] =
          count[L] > 0 ? 2.0 * M_PI * b_max / count[L] * sigma[(int64_t)L * n_levels + L2] : 0.0;
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Coupling matrix of an asymmetric-top rotor + linear rotor (Section II, Eq. 17)
//
// With the potential expanded as V = sum_t v_t(R) tau_t (Eqs. 12-13), the matrix
// (Eq. 6) is linear in the coefficients: M(R) = sum_t v_t(R) G_t.  G_t is Eq. 17
// with v_t = 1: the sums over m1', m1'', k1'', k1' and eta are taken as they are
// written there, the only rearrangement being that the k-sum (which does not
// depend on m1', m1'' or eta) is evaluated once per element.  Eq. 18 is not used:
// as printed, its summation index m1' stands for the projection of j1' in one
// factor and of j1'' in another.  Elements between different m vanish (Eq. 5
// couples n' -> n'' within one m).
//
// Clebsch-Gordan coefficients come from Racah's closed form, summed in long
// double.

static long double fact_ld(int n) {
  long double f = 1.0L;
  for (int i = 2; i <= n; ++i) f *= (long double)i;
  return f;
}

// <j1 m1 j2 m2 | J M> (Condon-Shortley phase), integer arguments
static double cg_racah(int j1, int m1, int j2, int m2, int J, int M) {
  if (m1 + m2 != M) return 0.0;
  if (J < std::abs(j1 - j2) || J > j1 + j2) return 0.0;
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return 0.0;
  const long double pre =
      (2 * J + 1) * fact_ld(J + j1 - j2) * fact_ld(J - j1 + j2) * fact_ld(j1 + j2 - J) /
      fact_ld(j1 + j2 + J + 1) * fact_ld(J + M) * fact_ld(J - M) * fact_ld(j1 - m1) *
      fact_ld(j1 + m1) * fact_ld(j2 - m2) * fact_ld(j2 + m2);
  long double s = 0.0L;
  const int kmin = std::max(0, std::max(j2 - J - m1, j1 - J + m2));
  const int kmax = std::min(j1 + j2 - J, std::min(j1 - m1, j2 + m2));
  for (int k = kmin; k <= kmax; ++k) {
    const long double den = fact_ld(k) * fact_ld(j1 + j2 - J - k) * fact_ld(j1 - m1 - k) *
                            fact_ld(j2 + m2 - k) * fact_ld(J - j2 + m1 + k) *
                            fact_ld(J - j1 - m2 + k);
    s += ((k & 1) ? -1.0L : 1.0L) / den;
  }
  return (double)(sqrtl(pre) * s);
}

extern "C" {

double oracle_cg(int j1, int m1, int j2, int m2, int J, int M) {
  return cg_racah(j1, m1, j2, m2, J, M);
}

// G[t][q][n'] for every term t, the final states n'' = rows[q] (q < nrows; all
// N in order when rows is null) and every initial state n'.  Channels: total j,
// projection m, rotor-1 state rot1 and linear-rotor j2; rotor-1 state r has
// angular momentum rot1_j[r] and coefficients b[r * b_stride + k + j1] (Eq. 1).
// Terms: (lam1, mu1, lam2, lam) of Eq. 13.  Returns 0, or -1 for an index out of
// range.
int oracle_coupling_angular(int N, const int* jt, const int* mt, const int* rot1,
                            const int* j2t, int n1, const int* rot1_j, const double* b,
                            int b_stride, int T, const int* lam1, const int* mu1,
                            const int* lam2, const int* lam, int nrows, const int* rows,
                            double* G) {
  for (int n = 0; n < N; ++n)
    if (rot1[n] < 0 || rot1[n] >= n1 || 2 * rot1_j[rot1[n]] + 1 > b_stride) return -1;
  if (!rows) nrows = N;
  for (int q = 0; q < nrows; ++q)
    if (rows && (rows[q] < 0 || rows[q] >= N)) return -1;
  const double pi = M_PI;
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int t = 0; t < T; ++t)
    for (int q = 0; q < nrows; ++q) {
      const int f = rows ? rows[q] : q;          // final state n''
      const int l1 = lam1[t], u1 = mu1[t], l2 = lam2[t], l = lam[t];
      const int sgn = ((l1 + u1 + l2 + l) & 1) ? -1 : 1;
      for (int i = 0; i < N; ++i) {              // initial state n'
        double* out = G + ((int64_t)t * nrows + q) * N + i;
        *out = 0.0;
        if (mt[f] != mt[i]) continue;
        const int m = mt[i];
        const int ja = jt[i], j1a = rot1_j[rot1[i]], j2a = j2t[i];   // n'
        const int jb = jt[f], j1b = rot1_j[rot1[f]], j2b = j2t[f];   // n''
        const double* ba = b + (int64_t)rot1[i] * b_stride;
        const double* bb = b + (int64_t)rot1[f] * b_stride;
        // sum over k1'', k1' of b b [C(j1' k1' l1 mu1 | j1'' k1'') + s C(j1' k1' l1 -mu1 | j1'' k1'')]
        double ksum = 0.0;
        for (int kb = -j1b; kb <= j1b; ++kb)
          for (int ka = -j1a; ka <= j1a; ++ka)
            ksum += bb[kb + j1b] * ba[ka + j1a] *
                    (cg_racah(j1a, ka, l1, u1, j1b, kb) + sgn * cg_racah(j1a, ka, l1, -u1, j1b, kb));
        if (ksum == 0.0) continue;
        const double pre = std::sqrt((2 * j1b + 1) / (8 * pi * pi)) *
                           std::sqrt((2 * j1a + 1) / (8 * pi * pi)) *
                           std::sqrt((2 * l1 + 1) / (4 * pi));
        const double y2 = std::sqrt((2 * j2a + 1) * (2 * l2 + 1) / (4 * pi * (2 * j2b + 1))) *
                          cg_racah(j2a, 0, l2, 0, j2b, 0);
        const double d1 = 8 * pi * pi / (2 * j1b + 1);
        double s = 0.0;
        for (int m1a = -j1a; m1a <= j1a; ++m1a) {
          const double ca = cg_racah(j1a, m1a, j2a, m - m1a, ja, m);
          if (ca == 0.0) continue;
          for (int m1b = -j1b; m1b <= j1b; ++m1b) {
            const double cb = cg_racah(j1b, m1b, j2b, m - m1b, jb, m);
            if (cb == 0.0) continue;
            const int emax = std::min(l1, l2);
            for (int eta = -emax; eta <= emax; ++eta)
              s += ca * cb * ksum * cg_racah(l1, eta, l2, -eta, l, 0) * y2 *
                   cg_racah(j2a, m - m1a, l2, -eta, j2b, m - m1b) * d1 *
                   cg_racah(j1a, m1a, l1, eta, j1b, m1b);
          }
        }
        *out = pre * s;
      }
    }
  return 0;
}

}  // extern "C"
