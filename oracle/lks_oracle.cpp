// lks_oracle.cpp -- TEST INFRASTRUCTURE ONLY (see lks_oracle.h).
//
// Plain double-precision reference of the paper's forward LKS march with a
// rigidly moving Brinkman body and of its exact discrete adjoint.  Every loop
// is written the obvious way: no tiling, no fusion, no reordering beyond what
// the formulas state.  The scalar type T is double, or std::complex<double>
// for complex-step derivatives (comparisons and integer decisions always use
// the real part, so both instantiations take identical branches).
//
// Readings where the paper is silent (each is also listed in the design notes):
//   * lattice units dx = dt = 1; kappa is the lattice product dx*kappa;
//   * the velocity gradient in the equilibrium (Sec. 2.2) uses 2-point central
//     differences, and a second-order one-sided difference on the wall axis
//     at wall nodes;
//   * wall nodes are grid nodes that are not updated by the gather: their
//     velocity is imposed and their pressure copies the nearest interior node
//     along the inward normal (Sec. 2.2, "p and u are directly imposed");
//   * the body enters step n at the new time level n (Algorithm 1);
//   * u^G = dx^G/dt and omega = dtheta/dt use central differences in time,
//     one-sided at the first and last step;
//   * the temporal filter (Eq. chi_filtered) is a discrete sum over steps
//     1..nt, truncated at the ends and normalised by the sum of its weights;
//   * design spacing equals dx; the design centre xi^G is the geometric
//     centre of the design grid including its margin; margin gamma = 0;
//   * J1 (Eq. objective1) sums n.u over the target box after every step.
#include "lks_oracle.h"

#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

namespace {

using cplx = std::complex<double>;

inline double re(double v) { return v; }
inline double re(const cplx& v) { return v.real(); }

// Standard lattice velocity sets (Sec. 2.2 cites the textbook sets; the
// figure with the vectors is not part of the text).
struct Lattice {
  int Q;
  int c[15][3];
  double w[15];
};

Lattice make_lattice(int d) {
  Lattice L{};
  if (d == 2) {
    const int c[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                         {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    L.Q = 9;
    for (int i = 0; i < 9; ++i) {
      L.c[i][0] = c[i][0];
      L.c[i][1] = c[i][1];
      L.c[i][2] = 0;
      L.w[i] = (i == 0) ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
  } else {
    L.Q = 15;
    int k = 0;
    L.c[k][0] = L.c[k][1] = L.c[k][2] = 0;
    L.w[k++] = 2.0 / 9.0;
    for (int a = 0; a < 3; ++a)
      for (int s = 1; s >= -1; s -= 2) {
        L.c[k][0] = L.c[k][1] = L.c[k][2] = 0;
        L.c[k][a] = s;
        L.w[k++] = 1.0 / 9.0;
      }
    for (int sz = 1; sz >= -1; sz -= 2)
      for (int sy = 1; sy >= -1; sy -= 2)
        for (int sx = 1; sx >= -1; sx -= 2) {
          L.c[k][0] = sx;
          L.c[k][1] = sy;
          L.c[k][2] = sz;
          L.w[k++] = 1.0 / 72.0;
        }
  }
  return L;
}

const double kPi = 3.14159265358979323846;

// Cosine kernel of the grid transfer (Sec. 2.3), r in units of dx.
template <class T>
T wker(const T& r) {
  if (std::fabs(re(r)) > 2.0) return T(0.0);
  return (1.0 + std::cos(kPi * r / 2.0)) / 4.0;
}
template <class T>
T wker_d(const T& r) {
  if (std::fabs(re(r)) > 2.0) return T(0.0);
  return -(kPi / 8.0) * std::sin(kPi * r / 2.0);
}

template <class T>
struct Oracle {
  const orc_problem& P;
  int d;
  int n[3];
  long N;
  Lattice L;
  double A;
  int D[3];      // design grid extents incl. margin
  long Mtot;     // design points incl. margin
  long Min;      // inner design points
  double xiG[3];
  int MW;        // motion row width: 8 (rotation about z) or 12 (three angles)

  explicit Oracle(const orc_problem& p) : P(p) {
    d = p.d;
    for (int a = 0; a < 3; ++a) n[a] = (a < d) ? p.n[a] : 1;
    N = (long)n[0] * n[1] * n[2];
    L = make_lattice(d);
    A = 0.75 - 4.5 * p.nu;  // A = 3/4 - (9/2) nu / dx
    for (int a = 0; a < 3; ++a) D[a] = (a < d) ? p.m[a] + 2 * p.margin : 1;
    Mtot = (long)D[0] * D[1] * D[2];
    Min = 1;
    for (int a = 0; a < d; ++a) Min *= p.m[a];
    for (int a = 0; a < 3; ++a) xiG[a] = 0.5 * (D[a] - 1);
    MW = p.rot == 1 ? 12 : 8;
  }

  long idx(const int x[3]) const { return x[0] + (long)n[0] * (x[1] + (long)n[1] * x[2]); }
  void coords(long i, int x[3]) const {
    x[0] = (int)(i % n[0]);
    x[1] = (int)((i / n[0]) % n[1]);
    x[2] = (int)(i / ((long)n[0] * n[1]));
  }
  bool wall_axis(int a) const { return a < d && P.bc[a] == 1; }
  bool is_wall(const int x[3]) const {
    for (int a = 0; a < d; ++a)
      if (wall_axis(a) && (x[a] == 0 || x[a] == n[a] - 1)) return true;
    return false;
  }
  // Interior node whose pressure a wall node copies: every coordinate that
  // sits on a wall moves one node inward.
  long wall_source(const int x[3]) const {
    int s[3] = {x[0], x[1], x[2]};
    for (int a = 0; a < d; ++a) {
      if (!wall_axis(a)) continue;
      if (x[a] == 0) s[a] = 1;
      if (x[a] == n[a] - 1) s[a] = n[a] - 2;
    }
    return idx(s);
  }
  // Imposed velocity at a wall node: the face of the highest axis wins.
  const double* wall_velocity(const int x[3]) const {
    const double* uw = nullptr;
    for (int a = 0; a < d; ++a) {
      if (!wall_axis(a)) continue;
      if (x[a] == 0) uw = P.u_wall[a][0];
      if (x[a] == n[a] - 1) uw = P.u_wall[a][1];
    }
    return uw;
  }
  // Periodic wrap; returns false if the coordinate leaves a wall axis.
  bool wrap(int a, int& v) const {
    if (v >= 0 && v < n[a]) return true;
    if (a < d && !wall_axis(a)) {
      v %= n[a];
      if (v < 0) v += n[a];
      return true;
    }
    return false;
  }

  // Derivative stencil of axis a at node x: up to 3 (node, coefficient) pairs.
  int deriv_stencil(int a, const int x[3], long* nodes, double* coef) const {
    int y[3] = {x[0], x[1], x[2]};
    if (wall_axis(a) && x[a] == 0) {
      const double c3[3] = {-1.5, 2.0, -0.5};
      for (int k = 0; k < 3; ++k) {
        y[a] = k;
        nodes[k] = idx(y);
        coef[k] = c3[k];
      }
      return 3;
    }
    if (wall_axis(a) && x[a] == n[a] - 1) {
      const double c3[3] = {1.5, -2.0, 0.5};
      for (int k = 0; k < 3; ++k) {
        y[a] = n[a] - 1 - k;
        nodes[k] = idx(y);
        coef[k] = c3[k];
      }
      return 3;
    }
    int yp = x[a] + 1, ym = x[a] - 1;
    wrap(a, yp);
    wrap(a, ym);
    y[a] = yp;
    nodes[0] = idx(y);
    coef[0] = 0.5;
    y[a] = ym;
    nodes[1] = idx(y);
    coef[1] = -0.5;
    return 2;
  }

  // ---------------------------------------------------------------- motion
  // Temporal filter (Eq. chi_filtered with triangular weights w_t).
  void filter(const T* in, int stride, int R, T* out) const {
    const int nt = P.nt;
    for (int t = 0; t < nt; ++t) {
      T num = 0.0;
      double den = 0.0;
      for (int tau = 0; tau < nt; ++tau) {
        int dt = std::abs(t - tau);
        if (dt > R) continue;
        double w = (double)(R - dt) / (double)R;
        num += w * in[(long)tau * stride];
        den += w;
      }
      out[t] = num / den;
    }
  }
  // Time derivative used for u^G and omega (Eqs. u_g, omega).
  void time_derivative(const T* x, T* v) const {
    const int nt = P.nt;
    if (nt == 1) {
      v[0] = 0.0;
      return;
    }
    v[0] = x[1] - x[0];
    v[nt - 1] = x[nt - 1] - x[nt - 2];
    for (int t = 1; t < nt - 1; ++t) v[t] = 0.5 * (x[t + 1] - x[t - 1]);
  }
  void motion(const T* chi, const T* psi, T* mot) const {
    const int nt = P.nt;
    std::vector<T> f(nt), x(nt), v(nt);
    for (int a = 0; a < 3; ++a) {
      if (a < d) {
        filter(chi + a, 3, P.r_t, f.data());
        for (int t = 0; t < nt; ++t) x[t] = (P.xg_max[a] - P.xg_min[a]) * f[t] + P.xg_min[a];
        time_derivative(x.data(), v.data());
      } else {
        for (int t = 0; t < nt; ++t) x[t] = v[t] = 0.0;
      }
      for (int t = 0; t < nt; ++t) {
        mot[t * MW + a] = x[t];
        mot[t * MW + 3 + a] = v[t];
      }
    }
    if (P.rot == 1) {
      // three angle series, each through the same filter, bounds and rate
      for (int k = 0; k < 3; ++k) {
        filter(psi + k, 3, P.r_w, f.data());
        const double lo = k < 2 ? P.tilt_min[k] : P.th_min;
        const double hi = k < 2 ? P.tilt_max[k] : P.th_max;
        for (int t = 0; t < nt; ++t) x[t] = (hi - lo) * f[t] + lo;
        time_derivative(x.data(), v.data());
        for (int t = 0; t < nt; ++t) {
          mot[t * MW + 6 + k] = x[t];
          mot[t * MW + 9 + k] = v[t];
        }
      }
      return;
    }
    filter(psi, 1, P.r_w, f.data());
    for (int t = 0; t < nt; ++t) x[t] = (P.th_max - P.th_min) * f[t] + P.th_min;
    time_derivative(x.data(), v.data());
    for (int t = 0; t < nt; ++t) {
      mot[t * MW + 6] = x[t];
      mot[t * MW + 7] = v[t];
    }
  }

  // Rotation about coordinate axis `ax` by angle a, differentiated `order`
  // times with respect to a: the 2 x 2 block [[c, -s], [s, c]] sits on the
  // two other axes in cyclic order (y, z for x; z, x for y; x, y for z).
  void axis_rot(int ax, const T& a, int order, T M[3][3]) const {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M[i][j] = 0.0;
    // n-th derivatives of cos and sin
    const T c = std::cos(a), s = std::sin(a);
    T cn = c, sn = s;
    if (order == 1) {
      cn = -s;
      sn = c;
    } else if (order == 2) {
      cn = -c;
      sn = -s;
    }
    const int i = (ax + 1) % 3, j = (ax + 2) % 3;
    M[ax][ax] = order == 0 ? 1.0 : 0.0;
    M[i][i] = cn;
    M[i][j] = -sn;
    M[j][i] = sn;
    M[j][j] = cn;
  }
  void matmul(const T A_[3][3], const T B[3][3], T C[3][3]) const {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T v = 0.0;
        for (int k = 0; k < 3; ++k) v += A_[i][k] * B[k][j];
        C[i][j] = v;
      }
  }
  // R = Rz(th3) Ry(th2) Rx(th1) differentiated o[k] times in th_k.
  void euler_rot(const T* th, const int o[3], T R[3][3]) const {
    T X[3][3], Y[3][3], Z[3][3], ZY[3][3];
    axis_rot(0, th[0], o[0], X);
    axis_rot(1, th[1], o[1], Y);
    axis_rot(2, th[2], o[2], Z);
    matmul(Z, Y, ZY);
    matmul(ZY, X, R);
  }
  // M r for a 3 x 3 matrix and an offset r.
  void apply(const T M[3][3], const double r[3], T out[3]) const {
    for (int i = 0; i < 3; ++i) out[i] = M[i][0] * r[0] + M[i][1] * r[1] + M[i][2] * r[2];
  }

  // -------------------------------------------------------------- design
  bool inner(const int xi[3]) const {
    for (int a = 0; a < d; ++a)
      if (xi[a] < P.margin || xi[a] >= P.margin + P.m[a]) return false;
    return true;
  }
  long inner_index(const int xi[3]) const {
    int j[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) j[a] = xi[a] - P.margin;
    return j[0] + (long)P.m[0] * (j[1] + (long)P.m[1] * j[2]);
  }
  void design_coords(long k, int xi[3]) const {
    xi[0] = (int)(k % D[0]);
    xi[1] = (int)((k / D[0]) % D[1]);
    xi[2] = (int)(k / ((long)D[0] * D[1]));
  }
  // Eq. kappa_ref.
  void kappa_ref(const T* gamma, T* kref) const {
    for (long k = 0; k < Mtot; ++k) {
      int xi[3];
      design_coords(k, xi);
      if (!inner(xi)) {
        kref[k] = 0.0;
        continue;
      }
      T g = gamma[inner_index(xi)];
      kref[k] = P.kappa_max * P.q * g / ((1.0 - g) + P.q);
    }
  }

  // Rigid position and velocity of design point xi (Eqs. rigid_body_position,
  // rigid_body_velocity); rotation about z.
  void rigid(const int xi[3], const T* mot, T X[3], T U[3]) const {
    if (P.rot == 1) {
      // x_ref = R(th) r + x^G and its time derivative sum_k om_k (dR/dth_k) r + u^G
      const double r[3] = {xi[0] - xiG[0], xi[1] - xiG[1], xi[2] - xiG[2]};
      T R[3][3], v[3];
      const int o0[3] = {0, 0, 0};
      euler_rot(mot + 6, o0, R);
      apply(R, r, v);
      for (int a = 0; a < 3; ++a) {
        X[a] = v[a] + mot[a];
        U[a] = mot[3 + a];
      }
      for (int k = 0; k < 3; ++k) {
        int o[3] = {0, 0, 0};
        o[k] = 1;
        T dR[3][3], dv[3];
        euler_rot(mot + 6, o, dR);
        apply(dR, r, dv);
        for (int a = 0; a < 3; ++a) U[a] += mot[9 + k] * dv[a];
      }
      return;
    }
    T th = mot[6], om = mot[7];
    T c = std::cos(th), s = std::sin(th);
    double r1 = xi[0] - xiG[0], r2 = xi[1] - xiG[1];
    X[0] = c * r1 - s * r2 + mot[0];
    X[1] = s * r1 + c * r2 + mot[1];
    U[0] = om * (-s * r1 - c * r2) + mot[3];
    U[1] = om * (c * r1 - s * r2) + mot[4];
    if (d == 3) {
      X[2] = (xi[2] - xiG[2]) + mot[2];
      U[2] = mot[5];
    } else {
      X[2] = 0.0;
      U[2] = 0.0;
    }
  }

  // Visit the analysis nodes within the kernel support of position X:
  // fn(node, r[3]) with r = x - X per axis.  Wall nodes are skipped.
  template <class F>
  void support(const T X[3], F fn) const {
    int lo[3], cnt[3];
    for (int a = 0; a < 3; ++a) {
      if (a < d) {
        lo[a] = (int)std::floor(re(X[a])) - 1;
        cnt[a] = 4;
      } else {
        lo[a] = 0;
        cnt[a] = 1;
      }
    }
    for (int kz = 0; kz < cnt[2]; ++kz)
      for (int ky = 0; ky < cnt[1]; ++ky)
        for (int kx = 0; kx < cnt[0]; ++kx) {
          int x[3] = {lo[0] + kx, lo[1] + ky, lo[2] + kz};
          T r[3];
          for (int a = 0; a < 3; ++a) r[a] = (a < d) ? T((double)x[a]) - X[a] : T(0.0);
          bool ok = true;
          for (int a = 0; a < d; ++a) ok = ok && wrap(a, x[a]);
          if (!ok || is_wall(x)) continue;
          fn(idx(x), r);
        }
  }

  // Eqs. kappa and u_s: kappa(x) = sum_xi W kappa_ref, u_s(x) = sum_xi W u_s_ref.
  void map(const T* kref, const T* mot, T* kappa, T* us) const {
    for (long i = 0; i < N; ++i) kappa[i] = 0.0;
    for (long i = 0; i < (long)d * N; ++i) us[i] = 0.0;
    for (long k = 0; k < Mtot; ++k) {
      int xi[3];
      design_coords(k, xi);
      T X[3], U[3];
      rigid(xi, mot, X, U);
      support(X, [&](long node, const T r[3]) {
        T W = 1.0;
        for (int a = 0; a < d; ++a) W *= wker(r[a]);
        kappa[node] += W * kref[k];
        for (int a = 0; a < d; ++a) us[a * N + node] += W * U[a];
      });
    }
  }

  // Transpose of map for one step (sensitivity terms of Eqs. dJdgamma,
  // dJdchi, dJdpsi and the multipliers u~^G, omega~ of Sec. 2.5).
  void map_adjoint(const T* kref, const T* mot, const T* kbar, const T* usbar, T* kref_bar,
                   T* mbar) const {
    for (int j = 0; j < MW; ++j) mbar[j] = 0.0;
    T th = mot[6], om = mot[7];
    T c = std::cos(th), s = std::sin(th);
    for (long k = 0; k < Mtot; ++k) {
      int xi[3];
      design_coords(k, xi);
      T X[3], U[3];
      rigid(xi, mot, X, U);
      T kb = 0.0, Ub[3] = {0.0, 0.0, 0.0}, Xb[3] = {0.0, 0.0, 0.0};
      support(X, [&](long node, const T r[3]) {
        T wv[3], dv[3];
        for (int a = 0; a < d; ++a) {
          wv[a] = wker(r[a]);
          dv[a] = wker_d(r[a]);
        }
        T W = 1.0;
        for (int a = 0; a < d; ++a) W *= wv[a];
        T g = kref[k] * kbar[node];
        for (int a = 0; a < d; ++a) g += U[a] * usbar[a * N + node];
        kb += W * kbar[node];
        for (int a = 0; a < d; ++a) Ub[a] += W * usbar[a * N + node];
        for (int a = 0; a < d; ++a) {
          // dW/dX_a = -w'(r_a) * prod_{b != a} w(r_b)
          T dW = -dv[a];
          for (int b = 0; b < d; ++b)
            if (b != a) dW *= wv[b];
          Xb[a] += dW * g;
        }
      });
      kref_bar[k] += kb;
      if (P.rot == 1) {
        // through x_ref = R r + x^G and u_ref = sum_j om_j (dR/dth_j) r + u^G:
        // th_k gets Xb . (dR/dth_k) r + Ub . sum_j om_j (d2R/dth_k dth_j) r,
        // om_k gets Ub . (dR/dth_k) r
        const double r[3] = {xi[0] - xiG[0], xi[1] - xiG[1], xi[2] - xiG[2]};
        for (int a = 0; a < 3; ++a) {
          mbar[a] += Xb[a];
          mbar[3 + a] += Ub[a];
        }
        for (int kk = 0; kk < 3; ++kk) {
          int o[3] = {0, 0, 0};
          o[kk] = 1;
          T dR[3][3], dv[3];
          euler_rot(mot + 6, o, dR);
          apply(dR, r, dv);
          T thb = Xb[0] * dv[0] + Xb[1] * dv[1] + Xb[2] * dv[2];
          for (int j = 0; j < 3; ++j) {
            int o2[3] = {0, 0, 0};
            o2[kk] += 1;
            o2[j] += 1;
            T d2R[3][3], d2v[3];
            euler_rot(mot + 6, o2, d2R);
            apply(d2R, r, d2v);
            thb += mot[9 + j] * (Ub[0] * d2v[0] + Ub[1] * d2v[1] + Ub[2] * d2v[2]);
          }
          mbar[6 + kk] += thb;
          mbar[9 + kk] += Ub[0] * dv[0] + Ub[1] * dv[1] + Ub[2] * dv[2];
        }
        continue;
      }
      double r1 = xi[0] - xiG[0], r2 = xi[1] - xiG[1];
      T dX1 = -s * r1 - c * r2, dX2 = c * r1 - s * r2;       // R'(theta) r
      T dU1 = om * (-c * r1 + s * r2), dU2 = om * (-s * r1 - c * r2);  // omega R''(theta) r
      for (int a = 0; a < d; ++a) {
        mbar[a] += Xb[a];
        mbar[3 + a] += Ub[a];
      }
      mbar[6] += Xb[0] * dX1 + Xb[1] * dX2 + Ub[0] * dU1 + Ub[1] * dU2;
      mbar[7] += Ub[0] * dX1 + Ub[1] * dX2;
    }
  }

  // ------------------------------------------------------------ LKS step
  // Equilibrium of Sec. 2.2 at every node for every direction: feq[i*N + y].
  void equilibria(const T* st, std::vector<T>& feq) const {
    const T* p = st;
    const T* u = st + N;
    feq.assign((size_t)L.Q * N, T(0.0));
    for (long y = 0; y < N; ++y) {
      int x[3];
      coords(y, x);
      // Du[a][b] = D_a u_b at y
      T Du[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Du[a][b] = 0.0;
      for (int a = 0; a < d; ++a) {
        long nodes[3];
        double coef[3];
        int k = deriv_stencil(a, x, nodes, coef);
        for (int b = 0; b < d; ++b)
          for (int j = 0; j < k; ++j) Du[a][b] += coef[j] * u[b * N + nodes[j]];
      }
      T uu = 0.0;
      for (int b = 0; b < d; ++b) uu += u[b * N + y] * u[b * N + y];
      for (int i = 0; i < L.Q; ++i) {
        T cu = 0.0, cSc = 0.0;
        for (int a = 0; a < d; ++a) cu += (double)L.c[i][a] * u[a * N + y];
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b)
            cSc += (double)(L.c[i][a] * L.c[i][b]) * (Du[a][b] + Du[b][a]);
        feq[(size_t)i * N + y] =
            L.w[i] * (3.0 * p[y] + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu + A * cSc);
      }
    }
  }

  // Eqs. p_tmp, u_tmp, p, u plus the wall rule.
  void step(const T* st, const T* kappa, const T* us, T* out) const {
    std::vector<T> feq;
    equilibria(st, feq);
    T* po = out;
    T* uo = out + N;
    for (long xn = 0; xn < N; ++xn) {
      int x[3];
      coords(xn, x);
      if (is_wall(x)) continue;
      T ps = 0.0, ust[3] = {0.0, 0.0, 0.0};
      for (int i = 0; i < L.Q; ++i) {
        int y[3] = {x[0] - L.c[i][0], x[1] - L.c[i][1], x[2] - L.c[i][2]};
        T f = 0.0;
        for (int a = 0; a < d; ++a) {
          // pressure drop across a periodic seam (test mode only)
          if (P.dp_seam[a] != 0.0 && !wall_axis(a)) {
            if (y[a] < 0) f += 3.0 * L.w[i] * P.dp_seam[a];
            if (y[a] >= n[a]) f -= 3.0 * L.w[i] * P.dp_seam[a];
          }
          wrap(a, y[a]);
        }
        f += feq[(size_t)i * N + idx(y)];
        ps += f / 3.0;
        for (int a = 0; a < d; ++a) ust[a] += (double)L.c[i][a] * f;
      }
      po[xn] = ps;
      for (int a = 0; a < d; ++a)
        uo[a * N + xn] = (ust[a] + kappa[xn] * us[a * N + xn]) / (1.0 + kappa[xn]);
    }
    for (long xn = 0; xn < N; ++xn) {
      int x[3];
      coords(xn, x);
      if (!is_wall(x)) continue;
      const double* uw = wall_velocity(x);
      for (int a = 0; a < d; ++a) uo[a * N + xn] = uw[a];
      po[xn] = po[wall_source(x)];
    }
  }

  // Exact transpose of step().
  void step_adjoint(const T* st_in, const T* st_out, const T* kappa, const T* us, const T* lam,
                    T* lam_prev, T* kbar, T* usbar) const {
    std::vector<T> pb(lam, lam + N), ub(lam + N, lam + (long)(d + 1) * N);
    const T* uin = st_in + N;
    const T* uout = st_out + N;
    // wall rule transposed: the copied pressure flows back to its source
    for (long xn = 0; xn < N; ++xn) {
      int x[3];
      coords(xn, x);
      if (!is_wall(x)) continue;
      pb[wall_source(x)] += pb[xn];
    }
    for (long xn = 0; xn < N; ++xn) {
      int x[3];
      coords(xn, x);
      if (!is_wall(x)) continue;
      pb[xn] = 0.0;
      for (int a = 0; a < d; ++a) ub[a * N + xn] = 0.0;
    }
    // Brinkman correction transposed (Eq. u)
    std::vector<T> psb(N), usb((size_t)d * N);
    for (long xn = 0; xn < N; ++xn) {
      T k = kappa[xn];
      psb[xn] = pb[xn];
      T kb = 0.0;
      for (int a = 0; a < d; ++a) {
        T uba = ub[a * N + xn];
        usb[a * N + xn] = uba / (1.0 + k);
        kb += uba * (us[a * N + xn] - uout[a * N + xn]) / (1.0 + k);
        usbar[a * N + xn] = k * uba / (1.0 + k);
      }
      kbar[xn] = kb;
    }
    // gather transposed: F_i(y) = dJ/dfeq_i(y)
    std::vector<T> F((size_t)L.Q * N, T(0.0));
    for (long yn = 0; yn < N; ++yn) {
      int y[3];
      coords(yn, y);
      for (int i = 0; i < L.Q; ++i) {
        int x[3] = {y[0] + L.c[i][0], y[1] + L.c[i][1], y[2] + L.c[i][2]};
        bool ok = true;
        for (int a = 0; a < d; ++a) ok = ok && wrap(a, x[a]);
        if (!ok || is_wall(x)) continue;
        long xn = idx(x);
        T f = psb[xn] / 3.0;
        for (int a = 0; a < d; ++a) f += (double)L.c[i][a] * usb[a * N + xn];
        F[(size_t)i * N + yn] = f;
      }
    }
    // equilibrium transposed
    for (long i = 0; i < (long)(d + 1) * N; ++i) lam_prev[i] = 0.0;
    T* pp = lam_prev;
    T* up = lam_prev + N;
    std::vector<T> Sb((size_t)9 * N, T(0.0));  // Sbar[a][b] at each node
    for (long yn = 0; yn < N; ++yn) {
      for (int i = 0; i < L.Q; ++i) {
        T g = L.w[i] * F[(size_t)i * N + yn];
        T cu = 0.0;
        for (int a = 0; a < d; ++a) cu += (double)L.c[i][a] * uin[a * N + yn];
        pp[yn] += 3.0 * g;
        for (int a = 0; a < d; ++a)
          up[a * N + yn] += g * (3.0 * L.c[i][a] + 9.0 * cu * (double)L.c[i][a] - 3.0 * uin[a * N + yn]);
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b)
            Sb[(size_t)(a * 3 + b) * N + yn] += A * g * (double)(L.c[i][a] * L.c[i][b]);
      }
    }
    // velocity gradient transposed: S_ab = D_a u_b + D_b u_a
    for (long xn = 0; xn < N; ++xn) {
      int x[3];
      coords(xn, x);
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          T g = Sb[(size_t)(a * 3 + b) * N + xn];
          long nodes[3];
          double coef[3];
          int k = deriv_stencil(a, x, nodes, coef);  // D_a u_b
          for (int j = 0; j < k; ++j) up[b * N + nodes[j]] += coef[j] * g;
          k = deriv_stencil(b, x, nodes, coef);      // D_b u_a
          for (int j = 0; j < k; ++j) up[a * N + nodes[j]] += coef[j] * g;
        }
    }
  }

  // ------------------------------------------------- objective J2 (Sec. 2.6)
  // Eq. objective2 per step: the force density f(xi) = kappa_ref (u_ref -
  // u_S_ref) on the design points, u_ref the fluid velocity taken to the
  // design point by the transfer kernel W, u_S_ref the rigid velocity.  Step
  // sums: sum f_1 (F_L), u^G_2 sum f_2 (F_D) and omega sum e3 (x_ref - x^G) x f
  // (T); the normalisations are applied at the end.
  void j2_sums(const T* kref, const T* mot, const T* u, T& jl, T& jd, T& jt) const {
    for (long k = 0; k < Mtot; ++k) {
      int xi[3];
      design_coords(k, xi);
      T X[3], U[3];
      rigid(xi, mot, X, U);
      T ur[2] = {0.0, 0.0};
      support(X, [&](long node, const T r[3]) {
        const T W = wker(r[0]) * wker(r[1]);
        for (int a = 0; a < 2; ++a) ur[a] += W * u[a * N + node];
      });
      const T f0 = kref[k] * (ur[0] - U[0]), f1 = kref[k] * (ur[1] - U[1]);
      const T v0 = X[0] - mot[0], v1 = X[1] - mot[1];
      jl += f0;
      jd += mot[4] * f1;
      jt += mot[7] * (v0 * f1 - v1 * f0);
    }
  }
  double j2_scale_l() const { return 1.0 / ((double)P.nt * (double)Min); }
  double j2_scale_d() const { return 1.0 / ((P.xg_max[1] - P.xg_min[1]) * (double)Min); }
  double j2_scale_t() const { return 1.0 / (2.0 * M_PI * P.l_m * (double)Min); }
  // dJ2/d(everything the step-t sums depend on), scaled by dJ: the seed on
  // the fluid velocity (added into ubar [d][N], times `useed`), and the
  // direct terms into kref_bar and the step's motion partials mbar[8].
  void j2_adjoint(const T* kref, const T* mot, const T* u, double dJ, T* ubar, double useed,
                  T* kref_bar, T* mbar) const {
    const T th = mot[6], om = mot[7];
    const T c = std::cos(th), s = std::sin(th);
    const T a0 = j2_scale_l(), a1 = P.w_d * mot[4] * j2_scale_d();
    const T b = P.w_t * om * j2_scale_t();
    T sf1 = 0.0, svf = 0.0;
    for (long k = 0; k < Mtot; ++k) {
      int xi[3];
      design_coords(k, xi);
      T X[3], U[3];
      rigid(xi, mot, X, U);
      T ur[2] = {0.0, 0.0}, dur[2][2] = {{0.0, 0.0}, {0.0, 0.0}};  // dur[a][b] = d u_ref_b / dX_a
      support(X, [&](long node, const T r[3]) {
        const T w0 = wker(r[0]), w1 = wker(r[1]);
        const T d0 = -wker_d(r[0]) * w1, d1 = -w0 * wker_d(r[1]);
        for (int q = 0; q < 2; ++q) {
          const T uq = u[q * N + node];
          ur[q] += w0 * w1 * uq;
          dur[0][q] += d0 * uq;
          dur[1][q] += d1 * uq;
        }
      });
      const T f0 = kref[k] * (ur[0] - U[0]), f1 = kref[k] * (ur[1] - U[1]);
      const T v0 = X[0] - mot[0], v1 = X[1] - mot[1];
      // dJ_t/df
      const T g0 = a0 - b * v1, g1 = a1 + b * v0;
      // seed on the fluid velocity: sum_xi W kappa_ref g
      support(X, [&](long node, const T r[3]) {
        const T W = wker(r[0]) * wker(r[1]);
        ubar[node] += useed * dJ * W * kref[k] * g0;
        ubar[N + node] += useed * dJ * W * kref[k] * g1;
      });
      kref_bar[k] += dJ * (g0 * (ur[0] - U[0]) + g1 * (ur[1] - U[1]));
      const double r1 = xi[0] - xiG[0], r2 = xi[1] - xiG[1];
      const T dX0 = -s * r1 - c * r2, dX1 = c * r1 - s * r2;            // R' r
      const T dU0 = om * (-c * r1 + s * r2), dU1 = om * (-s * r1 - c * r2);  // omega R'' r
      const T Xb0 = dJ * kref[k] * (g0 * dur[0][0] + g1 * dur[0][1]);
      const T Xb1 = dJ * kref[k] * (g0 * dur[1][0] + g1 * dur[1][1]);
      const T Ub0 = -dJ * kref[k] * g0, Ub1 = -dJ * kref[k] * g1;
      mbar[0] += Xb0;
      mbar[1] += Xb1;
      mbar[3] += Ub0;
      mbar[4] += Ub1;
      // theta: through X (kernel position), U (rigid velocity) and v = R r
      mbar[6] += Xb0 * dX0 + Xb1 * dX1 + Ub0 * dU0 + Ub1 * dU1 +
                 dJ * b * (dX0 * f1 - dX1 * f0);
      mbar[7] += Ub0 * dX0 + Ub1 * dX1;
      sf1 += f1;
      svf += v0 * f1 - v1 * f0;
    }
    // explicit factors u^G_2 (F_D) and omega (T)
    mbar[4] += dJ * P.w_d * j2_scale_d() * sf1;
    mbar[7] += dJ * P.w_t * j2_scale_t() * svf;
  }

  // ------------------------------------------------------------ objective
  long target_count() const {
    long c = 1;
    for (int a = 0; a < 3; ++a) {
      int lo = (a < d) ? P.tgt_lo[a] : 0, hi = (a < d) ? P.tgt_hi[a] : 1;
      if (hi <= lo) return 0;
      c *= (hi - lo);
    }
    return c;
  }
  bool in_target(const int x[3]) const {
    for (int a = 0; a < d; ++a)
      if (x[a] < P.tgt_lo[a] || x[a] >= P.tgt_hi[a]) return false;
    return true;
  }

  void initial_state(const T* state0, T* st) const {
    if (state0) {
      for (long i = 0; i < (long)(d + 1) * N; ++i) st[i] = state0[i];
    } else {
      for (long i = 0; i < N; ++i) st[i] = 1.0 / 3.0;
      for (long i = N; i < (long)(d + 1) * N; ++i) st[i] = 0.0;
    }
  }

  // Forward march with J1 (Eq. objective1).  traj nullable.
  void forward(const T* gamma, const T* chi, const T* psi, const T* state0, T* state_final,
               T* J3, T* traj) const {
    const long S = (long)(d + 1) * N;
    std::vector<T> mot((size_t)P.nt * MW), kref(Mtot), kappa(N), us((size_t)d * N);
    std::vector<T> a(S), b(S);
    motion(chi, psi, mot.data());
    kappa_ref(gamma, kref.data());
    initial_state(state0, a.data());
    if (traj) std::copy(a.begin(), a.end(), traj);
    T s1 = 0.0, s2 = 0.0;
    T jl = 0.0, jd = 0.0, jt = 0.0;  // J2 step sums
    for (int t = 1; t <= P.nt; ++t) {
      map(kref.data(), &mot[(size_t)(t - 1) * MW], kappa.data(), us.data());
      step(a.data(), kappa.data(), us.data(), b.data());
      std::swap(a, b);
      if (traj) std::copy(a.begin(), a.end(), traj + (long)t * S);
      if (P.objective == 1) {
        j2_sums(kref.data(), &mot[(size_t)(t - 1) * MW], a.data() + N, jl, jd, jt);
        continue;
      }
      for (long xn = 0; xn < N; ++xn) {
        int x[3];
        coords(xn, x);
        if (!in_target(x)) continue;
        T un = 0.0;
        for (int k = 0; k < d; ++k) un += P.ndir[k] * a[(k + 1) * N + xn];
        s1 += un;
        s2 += un * un;
      }
    }
    long NT = (long)P.nt * target_count();
    T E = 0.0, V = 0.0;
    if (NT > 0) {
      E = s1 / (double)NT;
      V = s2 / (double)NT - E * E;
    }
    J3[0] = E - P.phi * V;
    J3[1] = E;
    J3[2] = V;
    if (P.objective == 1) {
      // Eq. objective2: J2 = F_L + w_D F_D + w_T T
      const T FL = jl * j2_scale_l(), FD = jd * j2_scale_d(), TT = jt * j2_scale_t();
      J3[0] = FL + P.w_d * FD + P.w_t * TT;
      J3[1] = FL;
      J3[2] = FD;
    }
    if (state_final) std::copy(a.begin(), a.end(), state_final);
  }

  // Sensitivity epilogue: chain rule through u^G = D_t x^G, the affine bound
  // maps, the temporal filter and kappa_ref(gamma).
  void sensitivities(const T* gamma, const T* kref_bar, const T* mbar, T* dg, T* dchi,
                     T* dpsi) const {
    const int nt = P.nt;
    for (long k = 0; k < Mtot; ++k) {
      int xi[3];
      design_coords(k, xi);
      if (!inner(xi)) continue;
      long j = inner_index(xi);
      T g = gamma[j];
      T den = (1.0 - g) + P.q;
      dg[j] = kref_bar[k] * P.kappa_max * P.q * (1.0 + P.q) / (den * den);
    }
    std::vector<T> xb(nt), vb(nt), fb(nt);
    auto chain = [&](int R, double scale, T* out, int stride) {
      // xb: direct position partials, vb: velocity partials
      std::vector<T> tot(xb);
      if (nt > 1) {
        // transpose of time_derivative
        tot[0] += -vb[0];
        tot[1] += vb[0];
        tot[nt - 1] += vb[nt - 1];
        tot[nt - 2] += -vb[nt - 1];
        for (int t = 1; t < nt - 1; ++t) {
          tot[t + 1] += 0.5 * vb[t];
          tot[t - 1] += -0.5 * vb[t];
        }
      }
      for (int t = 0; t < nt; ++t) fb[t] = scale * tot[t];
      // transpose of the temporal filter
      for (int tau = 0; tau < nt; ++tau) out[(long)tau * stride] = 0.0;
      for (int t = 0; t < nt; ++t) {
        double den = 0.0;
        for (int tau = 0; tau < nt; ++tau) {
          int dt = std::abs(t - tau);
          if (dt <= R) den += (double)(R - dt) / (double)R;
        }
        for (int tau = 0; tau < nt; ++tau) {
          int dt = std::abs(t - tau);
          if (dt > R) continue;
          out[(long)tau * stride] += ((double)(R - dt) / (double)R / den) * fb[t];
        }
      }
    };
    for (int a = 0; a < 3; ++a) {
      if (a >= d) {
        for (int t = 0; t < nt; ++t) dchi[t * 3 + a] = 0.0;
        continue;
      }
      for (int t = 0; t < nt; ++t) {
        xb[t] = mbar[t * MW + a];
        vb[t] = mbar[t * MW + 3 + a];
      }
      chain(P.r_t, P.xg_max[a] - P.xg_min[a], dchi + a, 3);
    }
    if (P.rot == 1) {
      for (int k = 0; k < 3; ++k) {
        for (int t = 0; t < nt; ++t) {
          xb[t] = mbar[t * MW + 6 + k];
          vb[t] = mbar[t * MW + 9 + k];
        }
        const double span = k < 2 ? P.tilt_max[k] - P.tilt_min[k] : P.th_max - P.th_min;
        chain(P.r_w, span, dpsi + k, 3);
      }
      return;
    }
    for (int t = 0; t < nt; ++t) {
      xb[t] = mbar[t * MW + 6];
      vb[t] = mbar[t * MW + 7];
    }
    chain(P.r_w, P.th_max - P.th_min, dpsi, 1);
  }

  void adjoint(const T* gamma, const T* chi, const T* psi, const T* state0, double dJ,
               const T* adj_terminal, T* adj_initial, T* dg, T* dchi, T* dpsi, T* kref_bar_out,
               T* mbar_out) const {
    const long S = (long)(d + 1) * N;
    const int nt = P.nt;
    std::vector<T> traj((size_t)(nt + 1) * S);
    T J3[3];
    forward(gamma, chi, psi, state0, nullptr, J3, traj.data());
    T E = J3[1];
    std::vector<T> mot((size_t)nt * MW), kref(Mtot), kappa(N), us((size_t)d * N);
    motion(chi, psi, mot.data());
    kappa_ref(gamma, kref.data());
    std::vector<T> lam(S, T(0.0)), lprev(S), kbar(N), usbar((size_t)d * N);
    std::vector<T> kref_bar(Mtot, T(0.0)), mbar((size_t)nt * MW, T(0.0));
    if (adj_terminal)
      for (long i = 0; i < S; ++i) lam[i] += adj_terminal[i];
    long NT = (long)nt * target_count();
    for (int t = nt; t >= 1; --t) {
      const T* st = &traj[(size_t)t * S];
      // J2: seed now, motion partials after the map transpose (which writes
      // the step's row)
      T j2m[12] = {};
      if (P.objective == 1)
        j2_adjoint(kref.data(), &mot[(size_t)(t - 1) * MW], st + N, dJ, lam.data() + N, 1.0,
                   kref_bar.data(), j2m);
      if (NT > 0 && P.objective != 1) {
        for (long xn = 0; xn < N; ++xn) {
          int x[3];
          coords(xn, x);
          if (!in_target(x)) continue;
          T un = 0.0;
          for (int k = 0; k < d; ++k) un += P.ndir[k] * st[(k + 1) * N + xn];
          T g = dJ * (1.0 - 2.0 * P.phi * (un - E)) / (double)NT;
          for (int k = 0; k < d; ++k) lam[(k + 1) * N + xn] += g * P.ndir[k];
        }
      }
      map(kref.data(), &mot[(size_t)(t - 1) * MW], kappa.data(), us.data());
      step_adjoint(&traj[(size_t)(t - 1) * S], st, kappa.data(), us.data(), lam.data(),
                   lprev.data(), kbar.data(), usbar.data());
      map_adjoint(kref.data(), &mot[(size_t)(t - 1) * MW], kbar.data(), usbar.data(),
                  kref_bar.data(), &mbar[(size_t)(t - 1) * MW]);
      for (int q = 0; q < 8; ++q) mbar[(size_t)(t - 1) * MW + q] += j2m[q];
      std::swap(lam, lprev);
    }
    if (adj_initial) std::copy(lam.begin(), lam.end(), adj_initial);
    if (kref_bar_out) std::copy(kref_bar.begin(), kref_bar.end(), kref_bar_out);
    if (mbar_out) std::copy(mbar.begin(), mbar.end(), mbar_out);
    sensitivities(gamma, kref_bar.data(), mbar.data(), dg, dchi, dpsi);
  }

  // ------------------------------------------ design prelude (Sec. 3.1, 2.6)
  // Eq. filtering on the inner design grid (gamma is [m2][m1][m0], design
  // spacing 1): cone weights (R - |x_i - x_j|) / R for |x_i - x_j| < R,
  // normalised by their sum at each point; points outside the grid are left
  // out of both sums.
  template <class F>
  void design_stencil(double R, const int i[3], F fn) const {
    const int r = (int)std::floor(R);
    const int rz = d == 3 ? r : 0;
    for (int dz = -rz; dz <= rz; ++dz)
      for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
          const int j[3] = {i[0] + dx, i[1] + dy, i[2] + dz};
          bool in = true;
          for (int a = 0; a < d; ++a) in = in && j[a] >= 0 && j[a] < P.m[a];
          if (!in) continue;
          const double w = (R - std::sqrt((double)(dx * dx + dy * dy + dz * dz))) / R;
          if (w <= 0.0) continue;
          fn(j[0] + (long)P.m[0] * (j[1] + (long)(d >= 2 ? P.m[1] : 1) * j[2]), w);
        }
  }
  void inner_coords(long k, int i[3]) const {
    i[0] = (int)(k % P.m[0]);
    i[1] = (int)((k / P.m[0]) % P.m[1]);
    i[2] = d == 3 ? (int)(k / ((long)P.m[0] * P.m[1])) : 0;
  }
  void design_filter(const T* g, double R, T* out) const {
    for (long k = 0; k < Min; ++k) {
      int i[3];
      inner_coords(k, i);
      T acc = 0.0;
      double W = 0.0;
      design_stencil(R, i, [&](long j, double w) {
        acc += w * g[j];
        W += w;
      });
      out[k] = acc / W;
    }
  }
  // Eq. projection (beta <= 0: the identity, its limit as beta -> 0).
  T project(const T& x, double beta, double eta) const {
    if (beta <= 0.0) return x;
    const double den = std::tanh(beta * eta) + std::tanh(beta * (1.0 - eta));
    return (std::tanh(beta * eta) + std::tanh(beta * (x - eta))) / den;
  }
  T project_d(const T& x, double beta, double eta) const {
    if (beta <= 0.0) return T(1.0);
    const double den = std::tanh(beta * eta) + std::tanh(beta * (1.0 - eta));
    const T c = std::cosh(beta * (x - eta));
    return beta / (c * c) / den;
  }
  void design_prelude(const T* g, double R, double beta, double eta, T* phys) const {
    std::vector<T> ft(Min);
    design_filter(g, R, ft.data());
    for (long k = 0; k < Min; ++k) phys[k] = project(ft[k], beta, eta);
  }
  // Chain rule back through the projection and the filter: the transposed
  // Jacobian, scattered from each filtered point to its stencil.
  void design_prelude_adjoint(const T* g, double R, double beta, double eta, const T* gbar,
                              T* out) const {
    std::vector<T> ft(Min);
    design_filter(g, R, ft.data());
    for (long k = 0; k < Min; ++k) out[k] = 0.0;
    for (long k = 0; k < Min; ++k) {
      int i[3];
      inner_coords(k, i);
      double W = 0.0;
      design_stencil(R, i, [&](long, double w) { W += w; });
      const T h = project_d(ft[k], beta, eta) * gbar[k];
      design_stencil(R, i, [&](long j, double w) { out[j] += (w / W) * h; });
    }
  }
  // Eqs. constraint1 .. constraint3.  G1, G2 on the projected density (the
  // field the flow sees), over the M inner design points; G3 from the motion
  // prelude's omega, summed over the steps 1..nt (dt = 1) with |omega|.
  void constraints(const T* phys, const T* chi, const T* psi, double vmax, double omax,
                   double pw, T* G, T* dG1, T* dG2, T* dG3_dpsi) const {
    T s = 0.0, sf = 0.0;
    for (long k = 0; k < Min; ++k) {
      s += phys[k];
      sf += 1.0 - phys[k];
    }
    G[0] = s / (vmax * (double)Min) - 1.0;
    G[1] = sf / (vmax * (double)Min) - 1.0;
    for (long k = 0; k < Min; ++k) {
      if (dG1) dG1[k] = 1.0 / (vmax * (double)Min);
      if (dG2) dG2[k] = -1.0 / (vmax * (double)Min);
    }
    const int nt = P.nt;
    std::vector<T> mot((size_t)nt * MW);
    motion(chi, psi, mot.data());
    // omega about z (with three angles: om_3, the rate of the angle about z)
    const int oc = P.rot == 1 ? 11 : 7;
    T S = 0.0;
    for (int t = 0; t < nt; ++t) S += std::pow(std::abs(mot[(size_t)t * MW + oc] / omax), pw);
    G[2] = std::pow(S, 1.0 / pw) - 1.0;
    if (dG3_dpsi) {
      // dG3/domega_n, then the motion prelude's chain rule (D_t^T, bounds,
      // filter^T) as for the adjoint's motion partials
      std::vector<T> mbar((size_t)nt * MW, T(0.0)), kb(Mtot, T(0.0)), dg(Min), dchi((size_t)nt * 3);
      // the p-norm is not differentiable where every omega is 0: take 0 there
      for (int t = 0; t < nt && re(S) > 0.0; ++t) {
        const T om = mot[(size_t)t * MW + oc];
        const T a = std::abs(om / omax);
        const double sg = re(om) < 0.0 ? -1.0 : 1.0;
        mbar[(size_t)t * MW + oc] = std::pow(S, 1.0 / pw - 1.0) * std::pow(a, pw - 1.0) * sg / omax;
      }
      sensitivities(phys, kb.data(), mbar.data(), dg.data(), dchi.data(), dG3_dpsi);
    }
  }

  // ------------------------------------------------ ALKS backward (Sec. 2.5)
  // The continuous-adjoint lattice kinetic scheme as the paper states it.
  // Multipliers of one time level: pt [N], ut [d][N], sl [3*3][N] (s~_ab in
  // plane a*3+b).  Sign and scale are the paper's: the source terms enter
  // with the signs of Eqs. ap, au, as and the sensitivities of Eqs. dJdgamma,
  // dJdchi, dJdpsi use u~ as it is.
  //
  // Vector multiplying c_i in the adjoint equilibrium at every node y:
  //   V_a = 3 (u~_a + 3 s~_ab u_b - p~ u_a) - A d_b (s~_ab + s~_ba),
  // where the divergence is read as minus the transpose of the forward's
  // difference operator (central inside, and the transposed one-sided
  // stencil next to walls).
  void alks_vector(const T* pt, const T* ut, const T* sl, const T* u, std::vector<T>& V) const {
    V.assign((size_t)d * N, T(0.0));
    for (long xn = 0; xn < N; ++xn) {
      int x[3];
      coords(xn, x);
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          T g = A * (sl[(size_t)(a * 3 + b) * N + xn] + sl[(size_t)(b * 3 + a) * N + xn]);
          long nodes[3];
          double coef[3];
          int k = deriv_stencil(b, x, nodes, coef);
          for (int j = 0; j < k; ++j) V[a * N + nodes[j]] += coef[j] * g;
        }
    }
    for (long y = 0; y < N; ++y)
      for (int a = 0; a < d; ++a) {
        T su = 0.0;
        for (int b = 0; b < d; ++b) su += sl[(size_t)(a * 3 + b) * N + y] * u[b * N + y];
        V[a * N + y] += 3.0 * (ut[a * N + y] + 3.0 * su - pt[y] * u[a * N + y]);
      }
  }

  // Adjoint equilibrium f~eq_i(y) = (p~ + pw) + c_i . V at every node of one
  // level; pw (nullable) is the pressure multiplier that wall nodes hand to
  // their interior source node.  It joins the pressure term only: the wall's
  // copy of p never multiplies the source node's velocity, so the coupling
  // in V keeps the node's own p~.  The forward never gathers into a wall
  // node, so no adjoint leaves one: f~eq is zero there.
  void alks_equilibria(const T* pt, const T* pw, const T* ut, const T* sl, const T* u,
                       std::vector<T>& ft) const {
    std::vector<T> V;
    alks_vector(pt, ut, sl, u, V);
    ft.assign((size_t)L.Q * N, T(0.0));
    for (long y = 0; y < N; ++y) {
      int x[3];
      coords(y, x);
      if (is_wall(x)) continue;
      for (int i = 0; i < L.Q; ++i) {
        T f = pt[y] + (pw ? pw[y] : T(0.0));
        for (int a = 0; a < d; ++a) f += (double)L.c[i][a] * V[a * N + y];
        ft[(size_t)i * N + y] = f;
      }
    }
  }

  // Eqs. ap_tmp .. as_tmp: moments of the adjoint equilibria one level
  // later, read at x + c_i (periodic wrap; nothing from outside the grid).
  void alks_gather(const std::vector<T>& ft, T* pt, T* ut, T* sl) const {
    for (long i = 0; i < N; ++i) pt[i] = 0.0;
    for (long i = 0; i < (long)d * N; ++i) ut[i] = 0.0;
    for (long i = 0; i < 9 * N; ++i) sl[i] = 0.0;
    for (long yn = 0; yn < N; ++yn) {
      int y[3];
      coords(yn, y);
      for (int i = 0; i < L.Q; ++i) {
        int x[3] = {y[0] + L.c[i][0], y[1] + L.c[i][1], y[2] + L.c[i][2]};
        bool ok = true;
        for (int a = 0; a < d; ++a) ok = ok && wrap(a, x[a]);
        if (!ok) continue;
        T f = L.w[i] * ft[(size_t)i * N + idx(x)];
        pt[yn] += f;
        for (int a = 0; a < d; ++a) ut[a * N + yn] += (double)L.c[i][a] * f;
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b)
            sl[(size_t)(a * 3 + b) * N + yn] += (double)(L.c[i][a] * L.c[i][b]) * f;
      }
    }
  }

  // Symmetric components of s~ in the carried state: (xx, yy, xy) in 2D,
  // (xx, yy, zz, xy, xz, yz) in 3D.
  int sym_count() const { return d * (d + 1) / 2; }
  void sym_pair(int k, int& a, int& b) const {
    if (k < d) {
      a = b = k;
      return;
    }
    const int off[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    a = off[k - d][0];
    b = off[k - d][1];
  }

  // Full ALKS backward.  adj_initial (nullable, [(d+1) + 1 + d + d(d+1)/2][N])
  // receives first (-3 p~, -V) of level 0, the scheme's estimate of
  // dJ/d(state0) in the forward's variables (the multipliers carry the
  // opposite sign), and then the ALKS state of level 0 itself: p~, u~ and
  // the symmetric components of s~.  adj_terminal (nullable, same layout)
  // carries an earlier run's state for the periodic approximation (Sec. 3.3,
  // Algorithm 1): its (p~, u~, s~) part becomes the moments of the last
  // level, t1, before that level's sources, exactly where a run without it
  // starts from zero; the adjoint equilibria of that level are then formed
  // like every other level's, with this run's velocity at t1.  Its first
  // d+1 planes are not read.
  void alks_adjoint(const T* gamma, const T* chi, const T* psi, const T* state0, double dJ,
                    const T* adj_terminal, T* adj_initial, T* dg, T* dchi, T* dpsi,
                    T* kref_bar_out, T* mbar_out) const {
    const long S = (long)(d + 1) * N;
    const int nt = P.nt;
    std::vector<T> traj((size_t)(nt + 1) * S);
    T J3[3];
    forward(gamma, chi, psi, state0, nullptr, J3, traj.data());
    T E = J3[1];
    std::vector<T> mot((size_t)nt * MW), kref(Mtot), kappa(N), us((size_t)d * N);
    motion(chi, psi, mot.data());
    kappa_ref(gamma, kref.data());
    std::vector<T> pt(N, T(0.0)), ut((size_t)d * N, T(0.0)), sl((size_t)9 * N, T(0.0));
    std::vector<T> pw(N, T(0.0));
    std::vector<T> ft, kbar(N), usbar((size_t)d * N);
    std::vector<T> kref_bar(Mtot, T(0.0)), mbar((size_t)nt * MW, T(0.0));
    if (adj_terminal) {
      const T* c = adj_terminal + S;
      for (long i = 0; i < N; ++i) pt[i] = c[i];
      for (long i = 0; i < (long)d * N; ++i) ut[i] = c[N + i];
      for (int k = 0; k < sym_count(); ++k) {
        int a, b;
        sym_pair(k, a, b);
        for (long i = 0; i < N; ++i) {
          const T v = c[(1 + d + k) * N + i];
          sl[(size_t)(a * 3 + b) * N + i] = v;
          sl[(size_t)(b * 3 + a) * N + i] = v;
        }
      }
    }
    long NT = (long)nt * target_count();
    for (int t = nt; t >= 1; --t) {
      const T* st = &traj[(size_t)t * S];
      // moments of level t from the adjoint equilibria of level t + 1 (zero
      // after the last step, or the carried terminal state)
      if (t < nt) {
        alks_equilibria(pt.data(), pw.data(), ut.data(), sl.data(),
                        &traj[(size_t)(t + 1) * S + N], ft);
        alks_gather(ft, pt.data(), ut.data(), sl.data());
      }
      map(kref.data(), &mot[(size_t)(t - 1) * MW], kappa.data(), us.data());
      // Eq. au: objective source -sum_i w_i c_i dJ/df_i = -(1/3) dJ/du, and
      // the Brinkman source -kappa u~ taken at the new value (implicit); the
      // kappa and objective terms of Eqs. ap and as are odd moments and vanish
      T j2m[12] = {};
      if (P.objective == 1)
        j2_adjoint(kref.data(), &mot[(size_t)(t - 1) * MW], st + N, dJ, ut.data(), -1.0 / 3.0,
                   kref_bar.data(), j2m);
      if (NT > 0 && P.objective != 1) {
        for (long xn = 0; xn < N; ++xn) {
          int x[3];
          coords(xn, x);
          if (!in_target(x)) continue;
          T un = 0.0;
          for (int k = 0; k < d; ++k) un += P.ndir[k] * st[(k + 1) * N + xn];
          T g = dJ * (1.0 - 2.0 * P.phi * (un - E)) / (double)NT;
          for (int k = 0; k < d; ++k) ut[k * N + xn] -= g * P.ndir[k] / 3.0;
        }
      }
      for (long xn = 0; xn < N; ++xn)
        for (int a = 0; a < d; ++a) ut[a * N + xn] /= (1.0 + kappa[xn]);
      // wall rule: a wall node's pressure is a copy of its interior source,
      // so its multiplier moves there (into pw); imposed velocities carry none
      for (long xn = 0; xn < N; ++xn) pw[xn] = 0.0;
      for (long xn = 0; xn < N; ++xn) {
        int x[3];
        coords(xn, x);
        if (!is_wall(x)) continue;
        pw[wall_source(x)] += pt[xn];
      }
      for (long xn = 0; xn < N; ++xn) {
        int x[3];
        coords(xn, x);
        if (!is_wall(x)) continue;
        pt[xn] = 0.0;
        for (int a = 0; a < d; ++a) ut[a * N + xn] = 0.0;
      }
      // Eqs. dJdgamma, dJdchi, dJdpsi: dJ/dkappa = 3 (u - u^S) . u~ and
      // dJ/du^S = -3 kappa u~, pulled back to the design grid by the
      // transfer's transpose
      for (long xn = 0; xn < N; ++xn) {
        T kb = 0.0;
        for (int a = 0; a < d; ++a) {
          kb += 3.0 * (st[(a + 1) * N + xn] - us[a * N + xn]) * ut[a * N + xn];
          usbar[a * N + xn] = -3.0 * kappa[xn] * ut[a * N + xn];
        }
        kbar[xn] = kb;
      }
      map_adjoint(kref.data(), &mot[(size_t)(t - 1) * MW], kbar.data(), usbar.data(),
                  kref_bar.data(), &mbar[(size_t)(t - 1) * MW]);
      for (int q = 0; q < 8; ++q) mbar[(size_t)(t - 1) * MW + q] += j2m[q];
    }
    if (adj_initial) {
      // level 0: moments gathered from level 1, no sources
      alks_equilibria(pt.data(), pw.data(), ut.data(), sl.data(), &traj[(size_t)1 * S + N], ft);
      alks_gather(ft, pt.data(), ut.data(), sl.data());
      std::vector<T> V;
      alks_vector(pt.data(), ut.data(), sl.data(), &traj[N], V);
      for (long i = 0; i < N; ++i) adj_initial[i] = -3.0 * pt[i];
      for (long i = 0; i < (long)d * N; ++i) adj_initial[N + i] = -V[i];
      T* c = adj_initial + S;
      for (long i = 0; i < N; ++i) c[i] = pt[i];
      for (long i = 0; i < (long)d * N; ++i) c[N + i] = ut[i];
      for (int k = 0; k < sym_count(); ++k) {
        int a, b;
        sym_pair(k, a, b);
        for (long i = 0; i < N; ++i) c[(1 + d + k) * N + i] = sl[(size_t)(a * 3 + b) * N + i];
      }
    }
    if (kref_bar_out) std::copy(kref_bar.begin(), kref_bar.end(), kref_bar_out);
    if (mbar_out) std::copy(mbar.begin(), mbar.end(), mbar_out);
    // the sign of the multipliers is folded into dJ/dkappa and dJ/du^S above,
    // so the chain rule is the one of the discrete adjoint
    sensitivities(gamma, kref_bar.data(), mbar.data(), dg, dchi, dpsi);
  }
};

int validate(const orc_problem* p) {
  if (!p) return -1;
  if (p->d != 2 && p->d != 3) return -2;
  for (int a = 0; a < p->d; ++a) {
    if (p->n[a] < 1) return -3;
    if (p->bc[a] == 1 && p->n[a] < 4) return -4;
    if (p->m[a] < 0) return -5;
  }
  if (p->margin < 0 || p->nt < 1 || p->r_t < 1 || p->r_w < 1) return -6;
  if (p->objective != 0 && p->objective != 1) return -7;
  if (p->objective == 1 && (p->d != 2 || !(p->l_m > 0.0) || !(p->xg_max[1] > p->xg_min[1])))
    return -8;
  if (p->rot != 0 && (p->rot != 1 || p->d != 3)) return -10;
  return 0;
}

template <class T>
std::vector<T> cjoin(const double* re_, const double* im, long n) {
  std::vector<T> v(n);
  for (long i = 0; i < n; ++i) v[i] = T(re_ ? re_[i] : 0.0, im ? im[i] : 0.0);
  return v;
}
void csplit(const std::vector<cplx>& v, double* re_, double* im) {
  for (size_t i = 0; i < v.size(); ++i) {
    if (re_) re_[i] = v[i].real();
    if (im) im[i] = v[i].imag();
  }
}

}  // namespace

extern "C" {

int orc_motion(const orc_problem* p, const double* chi, const double* psi, double* motion) {
  if (int e = validate(p)) return e;
  Oracle<double>(*p).motion(chi, psi, motion);
  return 0;
}

int orc_kappa_ref(const orc_problem* p, const double* gamma, double* kappa_ref) {
  if (int e = validate(p)) return e;
  Oracle<double>(*p).kappa_ref(gamma, kappa_ref);
  return 0;
}

int orc_map(const orc_problem* p, const double* kappa_ref, const double* motion8, double* kappa,
            double* us) {
  if (int e = validate(p)) return e;
  Oracle<double>(*p).map(kappa_ref, motion8, kappa, us);
  return 0;
}

int orc_map_adjoint(const orc_problem* p, const double* kappa_ref, const double* motion8,
                    const double* kbar, const double* usbar, double* kref_bar,
                    double* motion_bar8) {
  if (int e = validate(p)) return e;
  Oracle<double>(*p).map_adjoint(kappa_ref, motion8, kbar, usbar, kref_bar, motion_bar8);
  return 0;
}

int orc_step(const orc_problem* p, const double* state_in, const double* kappa,
             const double* us, double* state_out) {
  if (int e = validate(p)) return e;
  Oracle<double>(*p).step(state_in, kappa, us, state_out);
  return 0;
}

int orc_step_adjoint(const orc_problem* p, const double* state_in, const double* state_out,
                     const double* kappa, const double* us, const double* lam,
                     double* lam_prev, double* kbar, double* usbar) {
  if (int e = validate(p)) return e;
  Oracle<double>(*p).step_adjoint(state_in, state_out, kappa, us, lam, lam_prev, kbar, usbar);
  return 0;
}

int orc_forward(const orc_problem* p, const double* gamma, const double* chi, const double* psi,
                const double* state0, double* state_final, double* J_out, double* traj) {
  if (int e = validate(p)) return e;
  Oracle<double>(*p).forward(gamma, chi, psi, state0, state_final, J_out, traj);
  return 0;
}

int orc_adjoint(const orc_problem* p, const double* gamma, const double* chi, const double* psi,
                const double* state0, double dJ, const double* adj_terminal, double* adj_initial,
                double* dJ_dgamma, double* dJ_dchi, double* dJ_dpsi, double* kref_bar,
                double* motion_bar) {
  if (int e = validate(p)) return e;
  Oracle<double>(*p).adjoint(gamma, chi, psi, state0, dJ, adj_terminal, adj_initial, dJ_dgamma,
                             dJ_dchi, dJ_dpsi, kref_bar, motion_bar);
  return 0;
}

int orc_alks_adjoint(const orc_problem* p, const double* gamma, const double* chi,
                     const double* psi, const double* state0, double dJ,
                     const double* adj_terminal, double* adj_initial, double* dJ_dgamma,
                     double* dJ_dchi, double* dJ_dpsi, double* kref_bar, double* motion_bar) {
  if (int e = validate(p)) return e;
  Oracle<double>(*p).alks_adjoint(gamma, chi, psi, state0, dJ, adj_terminal, adj_initial,
                                  dJ_dgamma, dJ_dchi, dJ_dpsi, kref_bar, motion_bar);
  return 0;
}

int orc_alks_vector(const orc_problem* p, const double* carry, const double* u, double* V) {
  if (int e = validate(p)) return e;
  Oracle<double> o(*p);
  const long N = o.N;
  const int d = o.d;
  std::vector<double> sl((size_t)9 * N, 0.0), Vv;
  for (int k = 0; k < o.sym_count(); ++k) {
    int a, b;
    o.sym_pair(k, a, b);
    for (long i = 0; i < N; ++i) {
      sl[(size_t)(a * 3 + b) * N + i] = carry[(1 + d + k) * N + i];
      sl[(size_t)(b * 3 + a) * N + i] = carry[(1 + d + k) * N + i];
    }
  }
  o.alks_vector(carry, carry + N, sl.data(), u, Vv);
  std::copy(Vv.begin(), Vv.end(), V);
  return 0;
}

int orc_j2_sums(const orc_problem* p, const double* kappa_ref, const double* motion8,
                const double* u, double* sums3) {
  if (int e = validate(p)) return e;
  if (p->d != 2) return -9;
  double jl = 0.0, jd = 0.0, jt = 0.0;
  Oracle<double>(*p).j2_sums(kappa_ref, motion8, u, jl, jd, jt);
  sums3[0] = jl;
  sums3[1] = jd;
  sums3[2] = jt;
  return 0;
}

int orc_alks_gather(const orc_problem* p, const double* fields_next, const double* u_next,
                    double* fields_out) {
  if (int e = validate(p)) return e;
  Oracle<double> o(*p);
  const long N = o.N;
  const int d = o.d;
  std::vector<double> ft;
  o.alks_equilibria(fields_next, nullptr, fields_next + N, fields_next + (1 + d) * N, u_next, ft);
  o.alks_gather(ft, fields_out, fields_out + N, fields_out + (1 + d) * N);
  return 0;
}

int orc_design_prelude(const orc_problem* p, const double* gamma, double radius, double beta,
                       double eta, double* phys) {
  if (int e = validate(p)) return e;
  if (!(radius > 0.0)) return -1;
  Oracle<double>(*p).design_prelude(gamma, radius, beta, eta, phys);
  return 0;
}

int orc_design_prelude_adjoint(const orc_problem* p, const double* gamma, double radius,
                               double beta, double eta, const double* dJ_dphys,
                               double* dJ_dgamma) {
  if (int e = validate(p)) return e;
  if (!(radius > 0.0)) return -1;
  Oracle<double>(*p).design_prelude_adjoint(gamma, radius, beta, eta, dJ_dphys, dJ_dgamma);
  return 0;
}

int orc_constraints(const orc_problem* p, const double* phys, const double* chi,
                    const double* psi, double vmax, double omega_max, double p_omega,
                    double* G_out, double* dG1, double* dG2, double* dG3_dpsi) {
  if (int e = validate(p)) return e;
  if (!(vmax > 0.0) || !(omega_max > 0.0) || !(p_omega >= 1.0)) return -1;
  Oracle<double>(*p).constraints(phys, chi, psi, vmax, omega_max, p_omega, G_out, dG1, dG2,
                                 dG3_dpsi);
  return 0;
}

int orc_sensitivities(const orc_problem* p, const double* gamma, const double* kref_bar,
                      const double* motion_bar, const double* motion, double* dJ_dgamma,
                      double* dJ_dchi, double* dJ_dpsi) {
  (void)motion;  // the chain rule needs only the bounds and filter radii
  if (int e = validate(p)) return e;
  Oracle<double>(*p).sensitivities(gamma, kref_bar, motion_bar, dJ_dgamma, dJ_dchi, dJ_dpsi);
  return 0;
}

int orc_forward_cs(const orc_problem* p, const double* gamma_re, const double* gamma_im,
                   const double* chi_re, const double* chi_im, const double* psi_re,
                   const double* psi_im, const double* state0_re, const double* state0_im,
                   double* J_re, double* J_im) {
  if (int e = validate(p)) return e;
  Oracle<cplx> o(*p);
  auto g = cjoin<cplx>(gamma_re, gamma_im, o.Min);
  auto c = cjoin<cplx>(chi_re, chi_im, (long)p->nt * 3);
  auto s = cjoin<cplx>(psi_re, psi_im, (long)p->nt * (p->rot == 1 ? 3 : 1));
  std::vector<cplx> st;
  if (state0_re) st = cjoin<cplx>(state0_re, state0_im, (long)(o.d + 1) * o.N);
  std::vector<cplx> J(3);
  o.forward(g.data(), c.data(), s.data(), state0_re ? st.data() : nullptr, nullptr, J.data(),
            nullptr);
  csplit(J, J_re, J_im);
  return 0;
}

int orc_step_cs(const orc_problem* p, const double* s_re, const double* s_im, const double* k_re,
                const double* k_im, const double* us_re, const double* us_im, double* out_re,
                double* out_im) {
  if (int e = validate(p)) return e;
  Oracle<cplx> o(*p);
  long S = (long)(o.d + 1) * o.N;
  auto s = cjoin<cplx>(s_re, s_im, S);
  auto k = cjoin<cplx>(k_re, k_im, o.N);
  auto u = cjoin<cplx>(us_re, us_im, (long)o.d * o.N);
  // wall nodes and untouched entries stay at the input values' layout
  std::vector<cplx> out(S, cplx(0.0, 0.0));
  o.step(s.data(), k.data(), u.data(), out.data());
  csplit(out, out_re, out_im);
  return 0;
}

int orc_map_cs(const orc_problem* p, const double* kref_re, const double* kref_im,
               const double* mot_re, const double* mot_im, double* k_re, double* k_im,
               double* us_re, double* us_im) {
  if (int e = validate(p)) return e;
  Oracle<cplx> o(*p);
  auto kr = cjoin<cplx>(kref_re, kref_im, o.Mtot);
  auto m = cjoin<cplx>(mot_re, mot_im, o.MW);
  std::vector<cplx> k(o.N), u((size_t)o.d * o.N);
  o.map(kr.data(), m.data(), k.data(), u.data());
  csplit(k, k_re, k_im);
  csplit(u, us_re, us_im);
  return 0;
}

}  // extern "C"
