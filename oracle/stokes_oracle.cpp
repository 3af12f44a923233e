// FP64 CPU oracle for the divergence-conforming B-spline Stokes solver path.
//
// TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's CPU
// baseline may load this library.  It shares no code with the HIP path: it does
// its own spline evaluation, quadrature, assembly, incomplete Cholesky, PCG and
// MINRES, written as plainly as possible so that each step can be checked by eye
// against the paper (Cortes & Coutinho, "Performance Evaluation of Block Diagonal
// Preconditioners for Divergence-Conforming B-Spline Discretization of Stokes
// Equations").  Single-threaded, double precision throughout.
//
// Section / equation references below are to that paper:
//   Sec. 2.1        univariate B-splines, Cox-de Boor recursion, open knot vectors
//   Sec. 2.2        tensor-product (bivariate) B-splines; 3D is the same tensor product
//   Sec. 3.1        Stokes problem, eq. (stokes_weak): a(w,v) = (2 nu sym grad w, sym grad v),
//                   b(v,q) = -(div v, q)
//   Sec. 3.2        RT-type spaces V_h, Q_h; no-penetration constraint V_{0,h}; zero-mean Q_{0,h}
//   Sec. 4          Nitsche form eta_h (eq. nitsche_lhs), discrete system and its matrices
//   Sec. 5          MINRES, preconditioned MINRES in the M^{-1} norm (eq. linsys_precond),
//                   block-diagonal preconditioner (eq. general_precond_M)
//   Sec. 6.2        C_pen = 5(k'+1), manufactured square-domain solution
//   Sec. 6.4        zero-mean pressure filtering after the solve; IC(0) factorisation and
//                   IC(0)-PCG inner solves.
//
// Readings where the paper is silent (each is listed in the design notes):
//   * face length h_F = 1/N (element length normal to the face);
//   * pressure block M_Q = Diag(Q)/(2 nu)  (scaled mass matrix Q_nu = Q/(2 nu), Sec. 5.1);
//   * IC(0) in natural (component-major, x-fastest) order; on a non-positive pivot the
//     factorisation restarts on A + alpha*diag(A), alpha = 1e-3, 1e-2, 1e-1;
//   * inner PCG stops when ||r||_2 <= rtol ||b||_2 (x0 = 0, test after each update, <= 200 its);
//   * MINRES stops when |eta_j| <= tol * gamma_1 (relative M^{-1}-norm residual, x0 = 0);
//   * zero-mean pressure: p <- p - (w.p)/(w.1) with w_k = integral of phi_k;
//   * mapped geometry (Sec. 3.2, the 1/8 annulus of Sec. 6.3): polar map r = 1 + xi_0,
//     theta = (pi/4) xi_1 onto 1 < r < 2, 0 < theta < pi/4; k'+3 Gauss points per direction
//     for the matrices (k'+5 for loads and errors), the integrands being rational there;
//     h_F = 1/(N |DF^{-1} n|), the element length normal to the face (Bazilevs' definition,
//     equal to 1/N on the identity map).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Gauss-Legendre rule with n points on [0,1].  Nodes are the roots of the
// Legendre polynomial P_n found by Newton's method; weights 2/((1-x^2) P_n'(x)^2),
// then mapped from [-1,1] to [0,1].
// ---------------------------------------------------------------------------
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;  // P_0, P_1
      for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(t), p0 = P_{n-1}(t)
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = t;
      for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
    }
    x[i] = 0.5 * (1.0 - t);  // ascending order on [0,1]
    w[i] = 1.0 / ((1.0 - t * t) * dp * dp);  // = (2/((1-t^2)P'^2)) / 2
  }
}

// ---------------------------------------------------------------------------
// Univariate B-spline space (Sec. 2.1): degree d, N uniform elements, open knot
// vector with every interior breakpoint of multiplicity one (maximal continuity
// C^{d-1}), hence n = N + d basis functions.
// ---------------------------------------------------------------------------
struct Space1D {
  int deg = 0;
  int nel = 0;
  int nfun = 0;
  std::vector<double> knot;
};

Space1D make_space(int deg, int nel) {
  Space1D s;
  s.deg = deg;
  s.nel = nel;
  s.nfun = nel + deg;
  for (int i = 0; i <= deg; ++i) s.knot.push_back(0.0);
  for (int i = 1; i < nel; ++i) s.knot.push_back(double(i) / nel);
  for (int i = 0; i <= deg; ++i) s.knot.push_back(1.0);
  return s;
}

// Cox-de Boor recursion for basis function i of degree d, restricted to the
// knot span `span` (the polynomial piece living on that span, so it can be
// evaluated on the closed span, including its end points).  Quotients with a
// zero-length denominator are taken as zero.
double cdb_value(const std::vector<double>& t, int i, int d, int span, double x) {
  if (d == 0) return (i == span) ? 1.0 : 0.0;
  double a = 0.0, b = 0.0;
  double den1 = t[i + d] - t[i];
  double den2 = t[i + d + 1] - t[i + 1];
  if (den1 > 0.0) a = (x - t[i]) / den1 * cdb_value(t, i, d - 1, span, x);
  if (den2 > 0.0) b = (t[i + d + 1] - x) / den2 * cdb_value(t, i + 1, d - 1, span, x);
  return a + b;
}

// First derivative from the same recursion: d/dx N_{i,d} = d N_{i,d-1}/(t_{i+d}-t_i)
//                                                         - d N_{i+1,d-1}/(t_{i+d+1}-t_{i+1}).
double cdb_deriv(const std::vector<double>& t, int i, int d, int span, double x) {
  if (d == 0) return 0.0;
  double a = 0.0, b = 0.0;
  double den1 = t[i + d] - t[i];
  double den2 = t[i + d + 1] - t[i + 1];
  if (den1 > 0.0) a = d / den1 * cdb_value(t, i, d - 1, span, x);
  if (den2 > 0.0) b = d / den2 * cdb_value(t, i + 1, d - 1, span, x);
  return a - b;
}

// Values and derivatives of the deg+1 functions that are non-zero on element e,
// at the parameter points xs (all inside the closed element).
// out_v[q*(deg+1)+a] is function (e+a) at point q.
void eval_on_element(const Space1D& s, int e, const std::vector<double>& xs,
                     std::vector<double>& out_v, std::vector<double>& out_d) {
  int nloc = s.deg + 1;
  out_v.assign(xs.size() * nloc, 0.0);
  out_d.assign(xs.size() * nloc, 0.0);
  int span = s.deg + e;
  for (size_t q = 0; q < xs.size(); ++q)
    for (int a = 0; a < nloc; ++a) {
      out_v[q * nloc + a] = cdb_value(s.knot, e + a, s.deg, span, xs[q]);
      out_d[q * nloc + a] = cdb_deriv(s.knot, e + a, s.deg, span, xs[q]);
    }
}

// ---------------------------------------------------------------------------
// Discrete spaces (Sec. 3.2).  Velocity component c is the tensor product of
// degree p = k'+1 in direction c and degree k' in the other directions; the two
// functions of direction c that are non-zero on the boundary (first and last)
// are removed (no penetration, u.n = 0).  Pressure is degree k' in every
// direction with no constraint (the zero mean is imposed after the solve).
// Numbering: velocity component-major, x fastest; pressure after velocity.
// ---------------------------------------------------------------------------
struct Problem {
  int N = 0, kp = 0, dim = 0;
  int geom = 0;                       // 0: identity map (unit square/cube); 1: 1/8 annulus (2D)
  double nu = 1.0, cpen = 0.0, h = 0.0;
  int pdeg = 0;                       // velocity degree p = k'+1
  Space1D sp_hi, sp_lo;               // 1D spaces of degree p and k'
  int vcount[3][3];                   // vcount[c][dir]: retained 1D functions
  int64_t voff[4];                    // component offsets into the velocity numbering
  int64_t nu_dofs = 0, np_dofs = 0;

  // Assembled matrices (CSR, sorted columns).  A: n_u x n_u; B: n_p x n_u; Q: n_p x n_p.
  std::vector<int64_t> A_ptr, B_ptr, Q_ptr;
  std::vector<int32_t> A_col, B_col, Q_col;
  std::vector<double> A_val, B_val, Q_val;
  std::vector<double> diagQ, wvec;    // diag(Q) and w_k = integral of phi_k
  // Coefficients of the constant function 1 in the pressure space: all ones on the identity
  // map; on a mapped domain phi_k = phihat_k / J, and kappa = Q^{-1} w (the L2 projection of
  // the constant, which lies in the space).  The pressure is unique up to multiples of kappa.
  std::vector<double> kappa;

  // IC(0) factor of A: lower triangle of A's pattern, diagonal stored last in each row.
  bool have_L = false;
  int ic_shift_steps = 0;
  double ic_alpha = 0.0;
  std::vector<int64_t> L_ptr;
  std::vector<int32_t> L_col;
  std::vector<double> L_val;

  // IC(0) factor of Q, the same layout.
  bool have_LQ = false;
  std::vector<int64_t> LQ_ptr;
  std::vector<int32_t> LQ_col;
  std::vector<double> LQ_val;

  // Dense Cholesky factors for the "ideal" preconditioner blocks (small meshes only).
  bool have_dense_A = false, have_dense_Q = false;
  std::vector<double> cholA, cholQ;
};

// 1D function index range on element e for a space of degree d: [e, e+d].
// Velocity: translate a component-c multi-index of 1D functions to the global number.
int64_t vel_index(const Problem& P, int c, const int* i1d) {
  int64_t g = 0, stride = 1;
  for (int dir = 0; dir < P.dim; ++dir) {
    int i = i1d[dir];
    if (dir == c) {
      if (i == 0 || i == P.sp_hi.nfun - 1) return -1;  // removed (normal component on boundary)
      i -= 1;
    }
    g += i * stride;
    stride *= P.vcount[c][dir];
  }
  return P.voff[c] + g;
}

int64_t pre_index(const Problem& P, const int* i1d) {
  int64_t g = 0, stride = 1;
  for (int dir = 0; dir < P.dim; ++dir) {
    g += i1d[dir] * stride;
    stride *= P.sp_lo.nfun;
  }
  return g;
}

// Decode a velocity global index into (component, 1D indices in the full 1D spaces).
void vel_decode(const Problem& P, int64_t g, int* c_out, int* i1d) {
  int c = 0;
  while (c + 1 < P.dim && g >= P.voff[c + 1]) ++c;
  int64_t r = g - P.voff[c];
  for (int dir = 0; dir < P.dim; ++dir) {
    int i = int(r % P.vcount[c][dir]);
    r /= P.vcount[c][dir];
    if (dir == c) i += 1;
    i1d[dir] = i;
  }
  *c_out = c;
}

void pre_decode(const Problem& P, int64_t g, int* i1d) {
  for (int dir = 0; dir < P.dim; ++dir) {
    i1d[dir] = int(g % P.sp_lo.nfun);
    g /= P.sp_lo.nfun;
  }
}

int deg_of(const Problem& P, int c, int dir) { return (dir == c) ? P.pdeg : P.kp; }

// ---------------------------------------------------------------------------
// Sparsity pattern: (i,j) is stored when the supports of the two basis functions
// share at least one element.  Row-wise: the union of the functions living on
// the elements of supp(i).
// ---------------------------------------------------------------------------
struct ElemFun {
  std::vector<int64_t> vel;  // global velocity indices on the element (-1 entries skipped)
  std::vector<int64_t> pre;
};

void element_functions(const Problem& P, const int* e, ElemFun& out) {
  out.vel.clear();
  out.pre.clear();
  for (int c = 0; c < P.dim; ++c) {
    int n[3] = {1, 1, 1};
    for (int dir = 0; dir < P.dim; ++dir) n[dir] = deg_of(P, c, dir) + 1;
    for (int a2 = 0; a2 < n[2]; ++a2)
      for (int a1 = 0; a1 < n[1]; ++a1)
        for (int a0 = 0; a0 < n[0]; ++a0) {
          int a[3] = {a0, a1, a2};
          int i1d[3] = {0, 0, 0};
          for (int dir = 0; dir < P.dim; ++dir) i1d[dir] = e[dir] + a[dir];
          int64_t g = vel_index(P, c, i1d);
          if (g >= 0) out.vel.push_back(g);
        }
  }
  int m = P.kp + 1;
  int n2 = (P.dim == 3) ? m : 1;
  for (int a2 = 0; a2 < n2; ++a2)
    for (int a1 = 0; a1 < m; ++a1)
      for (int a0 = 0; a0 < m; ++a0) {
        int a[3] = {a0, a1, a2};
        int i1d[3] = {0, 0, 0};
        for (int dir = 0; dir < P.dim; ++dir) i1d[dir] = e[dir] + a[dir];
        out.pre.push_back(pre_index(P, i1d));
      }
}

// Elements in the support of 1D function i of degree d: [max(0,i-d), min(N-1,i)].
void support_range(const Problem& P, int i, int d, int* lo, int* hi) {
  *lo = std::max(0, i - d);
  *hi = std::min(P.N - 1, i);
}

void build_row(const Problem& P, const int* lo, const int* hi, bool want_vel, bool want_pre,
               std::vector<int32_t>& vcols, std::vector<int32_t>& pcols) {
  vcols.clear();
  pcols.clear();
  ElemFun ef;
  int e[3] = {0, 0, 0};
  int lo2 = (P.dim == 3) ? lo[2] : 0, hi2 = (P.dim == 3) ? hi[2] : 0;
  for (e[2] = lo2; e[2] <= hi2; ++e[2])
    for (e[1] = lo[1]; e[1] <= hi[1]; ++e[1])
      for (e[0] = lo[0]; e[0] <= hi[0]; ++e[0]) {
        element_functions(P, e, ef);
        if (want_vel)
          for (int64_t g : ef.vel) vcols.push_back(int32_t(g));
        if (want_pre)
          for (int64_t g : ef.pre) pcols.push_back(int32_t(g));
      }
  std::sort(vcols.begin(), vcols.end());
  vcols.erase(std::unique(vcols.begin(), vcols.end()), vcols.end());
  std::sort(pcols.begin(), pcols.end());
  pcols.erase(std::unique(pcols.begin(), pcols.end()), pcols.end());
}

void build_patterns(Problem& P) {
  std::vector<int32_t> vc, pc;
  P.A_ptr.assign(1, 0);
  P.A_col.clear();
  for (int64_t g = 0; g < P.nu_dofs; ++g) {
    int c, i1d[3] = {0, 0, 0};
    vel_decode(P, g, &c, i1d);
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int dir = 0; dir < P.dim; ++dir) support_range(P, i1d[dir], deg_of(P, c, dir), &lo[dir], &hi[dir]);
    build_row(P, lo, hi, true, false, vc, pc);
    P.A_col.insert(P.A_col.end(), vc.begin(), vc.end());
    P.A_ptr.push_back(int64_t(P.A_col.size()));
  }
  P.B_ptr.assign(1, 0);
  P.Q_ptr.assign(1, 0);
  P.B_col.clear();
  P.Q_col.clear();
  for (int64_t g = 0; g < P.np_dofs; ++g) {
    int i1d[3] = {0, 0, 0};
    pre_decode(P, g, i1d);
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int dir = 0; dir < P.dim; ++dir) support_range(P, i1d[dir], P.kp, &lo[dir], &hi[dir]);
    build_row(P, lo, hi, true, true, vc, pc);
    P.B_col.insert(P.B_col.end(), vc.begin(), vc.end());
    P.B_ptr.push_back(int64_t(P.B_col.size()));
    P.Q_col.insert(P.Q_col.end(), pc.begin(), pc.end());
    P.Q_ptr.push_back(int64_t(P.Q_col.size()));
  }
  P.A_val.assign(P.A_col.size(), 0.0);
  P.B_val.assign(P.B_col.size(), 0.0);
  P.Q_val.assign(P.Q_col.size(), 0.0);
}

double& csr_at(std::vector<int64_t>& ptr, std::vector<int32_t>& col, std::vector<double>& val,
               int64_t i, int64_t j) {
  auto b = col.begin() + ptr[i], e = col.begin() + ptr[i + 1];
  auto it = std::lower_bound(b, e, int32_t(j));
  return val[it - col.begin()];  // the pattern always contains (i,j) for supported pairs
}

// ---------------------------------------------------------------------------
// Per-point evaluation of a velocity basis function: vector value Phi (component c
// times the scalar tensor-product spline B) and its full gradient
// G[a][b] = d Phi_a / d x_b = delta_{a c} dB/dx_b.
// ---------------------------------------------------------------------------
struct VelEval {
  int64_t g;
  int c;
  double val[3];
  double grad[3][3];
};

struct PreEval {
  int64_t g;
  double val;
};

// Tables of the 1D functions of one element in each direction, at a set of points.
struct Tab1D {
  std::vector<double> v, d;  // [q*(deg+1)+a]
  int nloc;
};

void tensor_eval_velocity(const Problem& P, const int* e, const Tab1D tabs[3][2], const int* qidx,
                          std::vector<VelEval>& out) {
  // tabs[dir][0] = degree-k' table, tabs[dir][1] = degree-p table, for element e[dir].
  out.clear();
  for (int c = 0; c < P.dim; ++c) {
    int n[3] = {1, 1, 1};
    for (int dir = 0; dir < P.dim; ++dir) n[dir] = deg_of(P, c, dir) + 1;
    for (int a2 = 0; a2 < n[2]; ++a2)
      for (int a1 = 0; a1 < n[1]; ++a1)
        for (int a0 = 0; a0 < n[0]; ++a0) {
          int a[3] = {a0, a1, a2};
          int i1d[3] = {0, 0, 0};
          for (int dir = 0; dir < P.dim; ++dir) i1d[dir] = e[dir] + a[dir];
          int64_t g = vel_index(P, c, i1d);
          if (g < 0) continue;
          double fv[3], fd[3];
          for (int dir = 0; dir < P.dim; ++dir) {
            const Tab1D& t = tabs[dir][dir == c ? 1 : 0];
            fv[dir] = t.v[qidx[dir] * t.nloc + a[dir]];
            fd[dir] = t.d[qidx[dir] * t.nloc + a[dir]];
          }
          double B = 1.0;
          for (int dir = 0; dir < P.dim; ++dir) B *= fv[dir];
          double dB[3] = {0, 0, 0};
          for (int k = 0; k < P.dim; ++k) {
            double prod = 1.0;
            for (int dir = 0; dir < P.dim; ++dir) prod *= (dir == k) ? fd[dir] : fv[dir];
            dB[k] = prod;
          }
          VelEval ve;
          ve.g = g;
          ve.c = c;
          for (int r = 0; r < 3; ++r) {
            ve.val[r] = (r == c) ? B : 0.0;
            for (int s = 0; s < 3; ++s) ve.grad[r][s] = (r == c && s < P.dim) ? dB[s] : 0.0;
          }
          out.push_back(ve);
        }
  }
}

void tensor_eval_pressure(const Problem& P, const int* e, const Tab1D tabs[3][2], const int* qidx,
                          std::vector<PreEval>& out) {
  out.clear();
  int m = P.kp + 1;
  int n2 = (P.dim == 3) ? m : 1;
  for (int a2 = 0; a2 < n2; ++a2)
    for (int a1 = 0; a1 < m; ++a1)
      for (int a0 = 0; a0 < m; ++a0) {
        int a[3] = {a0, a1, a2};
        int i1d[3] = {0, 0, 0};
        double v = 1.0;
        for (int dir = 0; dir < P.dim; ++dir) {
          i1d[dir] = e[dir] + a[dir];
          const Tab1D& t = tabs[dir][0];
          v *= t.v[qidx[dir] * t.nloc + a[dir]];
        }
        out.push_back({pre_index(P, i1d), v});
      }
}

// sym grad: eps = (G + G^T)/2
void sym_grad(const VelEval& f, double eps[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) eps[a][b] = 0.5 * (f.grad[a][b] + f.grad[b][a]);
}

// ---------------------------------------------------------------------------
// Geometry map F (Sec. 3.2): the physical domain is the image of the parametric unit
// square/cube.  geom 0: the identity.  geom 1 (2D): one eighth of an annulus (Sec. 6.3),
// the polar map x = r cos(theta), y = r sin(theta) with r = 1 + xi_0, theta = (pi/4) xi_1.
// At a parametric point: x = F(xi), the Jacobian matrix DF[a][b] = dx_a/dxi_b, its
// inverse, J = det DF and the second derivatives dDF[k][a][b] = d(DF[a][b])/dxi_k.
// ---------------------------------------------------------------------------
struct GeoPoint {
  double x[3];
  double DF[3][3], Finv[3][3], J;
  double dDF[3][3][3];
};

void geometry(const Problem& P, const double* xi, GeoPoint& g) {
  for (int a = 0; a < 3; ++a) {
    g.x[a] = a < P.dim ? xi[a] : 0.0;
    for (int b = 0; b < 3; ++b) {
      g.DF[a][b] = g.Finv[a][b] = (a == b) ? 1.0 : 0.0;
      for (int k = 0; k < 3; ++k) g.dDF[k][a][b] = 0.0;
    }
  }
  g.J = 1.0;
  if (P.geom == 0) return;
  const double al = kPi / 4.0, r = 1.0 + xi[0], t = al * xi[1];
  const double c = std::cos(t), s = std::sin(t);
  g.x[0] = r * c;
  g.x[1] = r * s;
  g.DF[0][0] = c;
  g.DF[0][1] = -al * r * s;
  g.DF[1][0] = s;
  g.DF[1][1] = al * r * c;
  g.J = g.DF[0][0] * g.DF[1][1] - g.DF[0][1] * g.DF[1][0];
  g.Finv[0][0] = g.DF[1][1] / g.J;
  g.Finv[0][1] = -g.DF[0][1] / g.J;
  g.Finv[1][0] = -g.DF[1][0] / g.J;
  g.Finv[1][1] = g.DF[0][0] / g.J;
  // d/dxi_0 = d/dr
  g.dDF[0][0][1] = -al * s;
  g.dDF[0][1][1] = al * c;
  // d/dxi_1 = (pi/4) d/dtheta
  g.dDF[1][0][0] = -al * s;
  g.dDF[1][0][1] = -al * al * r * c;
  g.dDF[1][1][0] = al * c;
  g.dDF[1][1][1] = -al * al * r * s;
}

// Piola transform of a velocity basis function (the inverse of the pullback iota_u of
// Sec. 3.2): Phi = DF Phihat / J.  With M = DF / J, the parametric derivatives are
// dPhi_a/dxi_k = sum_b (dM_k[a][b] Phihat_b + M[a][b] dPhihat_b/dxi_k), where
// dM_k = dDF[k]/J - DF (dJ/dxi_k)/J^2 and dJ/dxi_k = J trace(Finv dDF[k]); the physical
// gradient is dPhi_a/dx_m = sum_k (dPhi_a/dxi_k) Finv[k][m].  On entry v holds Phihat and
// its parametric gradient; on exit the physical value and gradient.
void piola(const Problem& P, const GeoPoint& g, VelEval& v) {
  if (P.geom == 0) return;
  const int d = P.dim;
  double M[3][3] = {{0}}, dM[3][3][3] = {{{0}}};
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) M[a][b] = g.DF[a][b] / g.J;
  for (int k = 0; k < d; ++k) {
    double tr = 0.0;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) tr += g.Finv[a][b] * g.dDF[k][b][a];
    const double dJ = g.J * tr;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) dM[k][a][b] = g.dDF[k][a][b] / g.J - g.DF[a][b] * dJ / (g.J * g.J);
  }
  double val[3] = {0, 0, 0}, dxi[3][3] = {{0}};
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      val[a] += M[a][b] * v.val[b];
      for (int k = 0; k < d; ++k) dxi[a][k] += dM[k][a][b] * v.val[b] + M[a][b] * v.grad[b][k];
    }
  for (int a = 0; a < 3; ++a) {
    v.val[a] = val[a];
    for (int m = 0; m < 3; ++m) {
      double s = 0.0;
      if (a < d && m < d)
        for (int k = 0; k < d; ++k) s += dxi[a][k] * g.Finv[k][m];
      v.grad[a][m] = s;
    }
  }
}

// Gauss points per direction of the matrices: k'+2 is exact on the identity map; the
// mapped integrands are rational, one more point is taken there.
int matrix_points(const Problem& P) { return P.kp + 2 + (P.geom ? 1 : 0); }
// Loads and error norms: k'+4 points, k'+5 on the mapped domain.
int load_points(const Problem& P) { return P.kp + 4 + (P.geom ? 1 : 0); }

// ---------------------------------------------------------------------------
// Assembly (Sec. 4): for every element, Gauss quadrature with k'+2 points per
// direction (exact for these polynomial integrands on the identity map):
//   A_ij  += 2 nu (sym grad Phi_j : sym grad Phi_i)
//   B_kj  += -(div Phi_j) phi_k
//   Q_kl  += phi_k phi_l
// and for every boundary face F with outward normal n (Nitsche, eq. nitsche_lhs,
// a_h = a - eta_h):
//   A_ij  += -2 nu [ (sym grad Phi_i n).Phi_j + (sym grad Phi_j n).Phi_i ]
//            + 2 nu (C_pen/h_F) Phi_i.Phi_j
// ---------------------------------------------------------------------------
void build_tabs_for_element(const Problem& P, const int* e, const std::vector<double>& xq01,
                            Tab1D tabs[3][2]) {
  for (int dir = 0; dir < P.dim; ++dir) {
    std::vector<double> xs(xq01.size());
    for (size_t q = 0; q < xq01.size(); ++q) xs[q] = (e[dir] + xq01[q]) * P.h;
    eval_on_element(P.sp_lo, e[dir], xs, tabs[dir][0].v, tabs[dir][0].d);
    tabs[dir][0].nloc = P.sp_lo.deg + 1;
    eval_on_element(P.sp_hi, e[dir], xs, tabs[dir][1].v, tabs[dir][1].d);
    tabs[dir][1].nloc = P.sp_hi.deg + 1;
  }
}

void assemble(Problem& P) {
  int nq = matrix_points(P);
  std::vector<double> xq, wq;
  gauss_legendre01(nq, xq, wq);
  P.diagQ.assign(P.np_dofs, 0.0);
  P.wvec.assign(P.np_dofs, 0.0);
  double vol = 1.0;
  for (int d = 0; d < P.dim; ++d) vol *= P.h;  // element measure

  int nE[3] = {P.N, P.N, P.dim == 3 ? P.N : 1};
  Tab1D tabs[3][2];
  std::vector<VelEval> ve;
  std::vector<PreEval> pe;
  int e[3] = {0, 0, 0};
  for (e[2] = 0; e[2] < nE[2]; ++e[2])
    for (e[1] = 0; e[1] < nE[1]; ++e[1])
      for (e[0] = 0; e[0] < nE[0]; ++e[0]) {
        build_tabs_for_element(P, e, xq, tabs);
        int nq2 = (P.dim == 3) ? nq : 1;
        int q[3] = {0, 0, 0};
        for (q[2] = 0; q[2] < nq2; ++q[2])
          for (q[1] = 0; q[1] < nq; ++q[1])
            for (q[0] = 0; q[0] < nq; ++q[0]) {
              double wt = vol, xi[3] = {0, 0, 0};
              for (int dir = 0; dir < P.dim; ++dir) {
                wt *= wq[q[dir]];
                xi[dir] = (e[dir] + xq[q[dir]]) * P.h;
              }
              tensor_eval_velocity(P, e, tabs, q, ve);
              tensor_eval_pressure(P, e, tabs, q, pe);
              // physical quantities: dx = J dxi, Piola velocities, pressures phihat / J
              GeoPoint geo;
              geometry(P, xi, geo);
              wt *= geo.J;
              for (VelEval& v : ve) piola(P, geo, v);
              for (PreEval& pp : pe) pp.val /= geo.J;
              std::vector<std::array<std::array<double, 3>, 3>> eps(ve.size());
              for (size_t i = 0; i < ve.size(); ++i) {
                double t[3][3];
                sym_grad(ve[i], t);
                for (int a = 0; a < 3; ++a)
                  for (int b = 0; b < 3; ++b) eps[i][a][b] = t[a][b];
              }
              for (size_t i = 0; i < ve.size(); ++i)
                for (size_t j = 0; j < ve.size(); ++j) {
                  double s = 0.0;
                  for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) s += eps[j][a][b] * eps[i][a][b];
                  csr_at(P.A_ptr, P.A_col, P.A_val, ve[i].g, ve[j].g) += wt * 2.0 * P.nu * s;
                }
              for (size_t k = 0; k < pe.size(); ++k) {
                for (size_t j = 0; j < ve.size(); ++j) {
                  double div = 0.0;
                  for (int a = 0; a < P.dim; ++a) div += ve[j].grad[a][a];
                  csr_at(P.B_ptr, P.B_col, P.B_val, pe[k].g, ve[j].g) += -wt * div * pe[k].val;
                }
                for (size_t l = 0; l < pe.size(); ++l)
                  csr_at(P.Q_ptr, P.Q_col, P.Q_val, pe[k].g, pe[l].g) += wt * pe[k].val * pe[l].val;
                P.wvec[pe[k].g] += wt * pe[k].val;
              }
            }

        // Boundary faces of this element.
        for (int fdir = 0; fdir < P.dim; ++fdir)
          for (int side = 0; side < 2; ++side) {
            if (side == 0 && e[fdir] != 0) continue;
            if (side == 1 && e[fdir] != P.N - 1) continue;
            double nhat[3] = {0, 0, 0};  // parametric outward normal
            nhat[fdir] = side == 0 ? -1.0 : 1.0;
            // Face points: tensor Gauss rule in the tangential directions, fixed coordinate
            // 0 or 1 in direction fdir.
            Tab1D ftabs[3][2];
            for (int dir = 0; dir < P.dim; ++dir) {
              std::vector<double> xs;
              if (dir == fdir) {
                xs.push_back(side == 0 ? 0.0 : 1.0);
              } else {
                for (int qq = 0; qq < nq; ++qq) xs.push_back((e[dir] + xq[qq]) * P.h);
              }
              eval_on_element(P.sp_lo, e[dir], xs, ftabs[dir][0].v, ftabs[dir][0].d);
              ftabs[dir][0].nloc = P.sp_lo.deg + 1;
              eval_on_element(P.sp_hi, e[dir], xs, ftabs[dir][1].v, ftabs[dir][1].d);
              ftabs[dir][1].nloc = P.sp_hi.deg + 1;
            }
            double farea = 1.0;
            for (int dir = 0; dir < P.dim; ++dir)
              if (dir != fdir) farea *= P.h;
            int nqd[3] = {1, 1, 1};
            for (int dir = 0; dir < P.dim; ++dir) nqd[dir] = (dir == fdir) ? 1 : nq;
            int qf[3] = {0, 0, 0};
            for (qf[2] = 0; qf[2] < nqd[2]; ++qf[2])
              for (qf[1] = 0; qf[1] < nqd[1]; ++qf[1])
                for (qf[0] = 0; qf[0] < nqd[0]; ++qf[0]) {
                  double wt = farea, xi[3] = {0, 0, 0};
                  for (int dir = 0; dir < P.dim; ++dir) {
                    if (dir != fdir) wt *= wq[qf[dir]];
                    xi[dir] = dir == fdir ? (side == 0 ? 0.0 : 1.0) : (e[dir] + xq[qf[dir]]) * P.h;
                  }
                  tensor_eval_velocity(P, e, ftabs, qf, ve);
                  // physical outward normal n = Finv^T nhat / |Finv^T nhat|, surface measure
                  // dS = J |Finv^T nhat| dS_hat, and h_F = 1 / (N |Finv n|)
                  GeoPoint geo;
                  geometry(P, xi, geo);
                  double m[3] = {0, 0, 0}, mn = 0.0;
                  for (int a = 0; a < 3; ++a) {
                    for (int b = 0; b < 3; ++b) m[a] += geo.Finv[b][a] * nhat[b];
                    mn += m[a] * m[a];
                  }
                  mn = std::sqrt(mn);
                  double nrm[3], fn[3] = {0, 0, 0}, fnn = 0.0;
                  for (int a = 0; a < 3; ++a) nrm[a] = m[a] / mn;
                  for (int a = 0; a < 3; ++a) {
                    for (int b = 0; b < 3; ++b) fn[a] += geo.Finv[a][b] * nrm[b];
                    fnn += fn[a] * fn[a];
                  }
                  const double hF = 1.0 / (P.N * std::sqrt(fnn));
                  wt *= geo.J * mn;
                  for (VelEval& v : ve) piola(P, geo, v);
                  std::vector<std::array<double, 3>> tr(ve.size());  // (sym grad Phi) n
                  for (size_t i = 0; i < ve.size(); ++i) {
                    double t[3][3];
                    sym_grad(ve[i], t);
                    for (int a = 0; a < 3; ++a) {
                      double s = 0.0;
                      for (int b = 0; b < 3; ++b) s += t[a][b] * nrm[b];
                      tr[i][a] = s;
                    }
                  }
                  for (size_t i = 0; i < ve.size(); ++i)
                    for (size_t j = 0; j < ve.size(); ++j) {
                      double ti_vj = 0.0, tj_vi = 0.0, vi_vj = 0.0;
                      for (int a = 0; a < 3; ++a) {
                        ti_vj += tr[i][a] * ve[j].val[a];
                        tj_vi += tr[j][a] * ve[i].val[a];
                        vi_vj += ve[i].val[a] * ve[j].val[a];
                      }
                      double contrib = -2.0 * P.nu * (ti_vj + tj_vi) + 2.0 * P.nu * (P.cpen / hF) * vi_vj;
                      csr_at(P.A_ptr, P.A_col, P.A_val, ve[i].g, ve[j].g) += wt * contrib;
                    }
                }
          }
      }
  for (int64_t k = 0; k < P.np_dofs; ++k)
    P.diagQ[k] = csr_at(P.Q_ptr, P.Q_col, P.Q_val, k, k);
}

// ---------------------------------------------------------------------------
// Forcing functions.  Problem 1 (default): u = curl of psi with
// psi = x^2(1-x)^2 y^2(1-y)^2 (2D: u = (psi_y, -psi_x)), or u = curl(g,g,g) with
// g = phi(x)phi(y)phi(z), phi(t) = t^2(1-t)^2 (3D); p = prod cos(pi x_d); and
// f = -div(2 nu sym grad u) + grad p = -nu Lap u + grad p (u is divergence free).
// Problem 2: the paper's square-domain solution (Sec. 6.2) with the sign of the
// second velocity component chosen so that the field is divergence free.
// Problem 3: a pure gradient f = grad(phi), phi = sin(2 pi x) cos(pi y) [cos(pi z)].
// Problem 4 (1/8 annulus): see AnnulusPsi below.
// Optional sinusoid modes are added: f_d += a_{d,m} sin(pi k_m . x + ph_{d,m}).
// Every forcing is evaluated at the physical point x = F(xi).
// ---------------------------------------------------------------------------
struct Phi1 {  // phi(t) = t^2 (1-t)^2 and derivatives
  static double f0(double t) { return t * t * (1 - t) * (1 - t); }
  static double f1(double t) { return 2 * t - 6 * t * t + 4 * t * t * t; }
  static double f2(double t) { return 2 - 12 * t + 12 * t * t; }
  static double f3(double t) { return -12 + 24 * t; }
};

// Bivariate polynomials, sum c[i][j] x^i y^j (degree < 16), for the annulus solution.
struct Poly2 {
  double c[16][16] = {{0}};
};
Poly2 poly_mul(const Poly2& a, const Poly2& b) {
  Poly2 r;
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j)
      if (a.c[i][j] != 0.0)
        for (int k = 0; i + k < 16; ++k)
          for (int l = 0; j + l < 16; ++l) r.c[i + k][j + l] += a.c[i][j] * b.c[k][l];
  return r;
}
Poly2 poly_dx(const Poly2& a) {
  Poly2 r;
  for (int i = 1; i < 16; ++i)
    for (int j = 0; j < 16; ++j) r.c[i - 1][j] = i * a.c[i][j];
  return r;
}
Poly2 poly_dy(const Poly2& a) {
  Poly2 r;
  for (int i = 0; i < 16; ++i)
    for (int j = 1; j < 16; ++j) r.c[i][j - 1] = j * a.c[i][j];
  return r;
}
double poly_at(const Poly2& a, double x, double y) {
  double s = 0.0, xp = 1.0;
  for (int i = 0; i < 16; ++i, xp *= x) {
    double yp = 1.0;
    for (int j = 0; j < 16; ++j, yp *= y) s += a.c[i][j] * xp * yp;
  }
  return s;
}

// Problem 4, on the 1/8 annulus: u = curl psi = (psi_y, -psi_x) with psi = a^2 b^2,
// a = (x^2 + y^2 - 1)(x^2 + y^2 - 4) (zero on the arcs r = 1, 2), b = y (y - x) (zero on
// the sides theta = 0, pi/4): psi and grad psi vanish on the boundary, so u = 0 there and
// div u = 0; p = x y^2 (its mean is removed by the error routine).  The derivatives of psi
// up to third order are tabulated once.
struct AnnulusPsi {
  Poly2 d[4][4];  // d[i][j] = d^{i+j} psi / dx^i dy^j, i + j <= 3
  AnnulusPsi() {
    Poly2 r2m1, r2m4, b;
    r2m1.c[2][0] = 1; r2m1.c[0][2] = 1; r2m1.c[0][0] = -1;
    r2m4.c[2][0] = 1; r2m4.c[0][2] = 1; r2m4.c[0][0] = -4;
    b.c[0][2] = 1;    // y^2
    b.c[1][1] = -1;   // - x y
    const Poly2 a = poly_mul(r2m1, r2m4);
    const Poly2 ab = poly_mul(a, b);
    d[0][0] = poly_mul(ab, ab);
    for (int i = 0; i <= 3; ++i)
      for (int j = 0; i + j <= 3; ++j) {
        if (i == 0 && j == 0) continue;
        d[i][j] = j > 0 ? poly_dy(d[i][j - 1]) : poly_dx(d[i - 1][j]);
      }
  }
  double at(int i, int j, const double* x) const { return poly_at(d[i][j], x[0], x[1]); }
};
const AnnulusPsi& annulus_psi() {
  static const AnnulusPsi A;
  return A;
}

// Exact fields for error norms: velocity, velocity gradient, pressure.
void exact_solution(int problem, int dim, const double* x, double* u, double g[3][3], double* p) {
  for (int a = 0; a < 3; ++a) {
    u[a] = 0;
    for (int b = 0; b < 3; ++b) g[a][b] = 0;
  }
  *p = 0;
  if (problem == 1 && dim == 2) {
    double X0 = Phi1::f0(x[0]), X1 = Phi1::f1(x[0]), X2 = Phi1::f2(x[0]);
    double Y0 = Phi1::f0(x[1]), Y1 = Phi1::f1(x[1]), Y2 = Phi1::f2(x[1]);
    u[0] = X0 * Y1;
    u[1] = -X1 * Y0;
    g[0][0] = X1 * Y1;
    g[0][1] = X0 * Y2;
    g[1][0] = -X2 * Y0;
    g[1][1] = -X1 * Y1;
    *p = std::cos(kPi * x[0]) * std::cos(kPi * x[1]);
  } else if (problem == 1 && dim == 3) {
    double F0[3], F1[3], F2[3];
    for (int d = 0; d < 3; ++d) {
      F0[d] = Phi1::f0(x[d]);
      F1[d] = Phi1::f1(x[d]);
      F2[d] = Phi1::f2(x[d]);
    }
    // grad g and Hessian of g = F0[0] F0[1] F0[2]
    double dg[3], H[3][3];
    for (int a = 0; a < 3; ++a) {
      double v = 1;
      for (int d = 0; d < 3; ++d) v *= (d == a) ? F1[d] : F0[d];
      dg[a] = v;
      for (int b = 0; b < 3; ++b) {
        double w = 1;
        for (int d = 0; d < 3; ++d) {
          int order = (d == a) + (d == b);
          w *= order == 0 ? F0[d] : (order == 1 ? F1[d] : F2[d]);
        }
        H[a][b] = w;
      }
    }
    // u = curl(g,g,g) = (g_y - g_z, g_z - g_x, g_x - g_y)
    u[0] = dg[1] - dg[2];
    u[1] = dg[2] - dg[0];
    u[2] = dg[0] - dg[1];
    for (int b = 0; b < 3; ++b) {
      g[0][b] = H[1][b] - H[2][b];
      g[1][b] = H[2][b] - H[0][b];
      g[2][b] = H[0][b] - H[1][b];
    }
    *p = std::cos(kPi * x[0]) * std::cos(kPi * x[1]) * std::cos(kPi * x[2]);
  } else if (problem == 2) {
    // psi = X(x) Y(y), X = e^x x^2 (x-1)^2, Y = y^2 (y-1)^2; u = (psi_y, -psi_x).
    double ex = std::exp(x[0]), xx = x[0], y = x[1];
    double P0 = xx * xx * (xx - 1) * (xx - 1);
    double P1 = 4 * xx * xx * xx - 6 * xx * xx + 2 * xx;
    double P2 = 12 * xx * xx - 12 * xx + 2;
    double X0 = ex * P0, X1 = ex * (P0 + P1), X2 = ex * (P0 + 2 * P1 + P2);
    double Y0 = Phi1::f0(y), Y1 = Phi1::f1(y), Y2 = Phi1::f2(y);
    u[0] = X0 * Y1;
    u[1] = -X1 * Y0;
    g[0][0] = X1 * Y1;
    g[0][1] = X0 * Y2;
    g[1][0] = -X2 * Y0;
    g[1][1] = -X1 * Y1;
    double q = y * y - y;
    double G = 456 + xx * xx * (228 - 5 * q) + 2 * xx * (-228 + q) + 2 * xx * xx * xx * (-36 + q) +
               xx * xx * xx * xx * (12 + q);
    *p = -424 + 156 * std::exp(1.0) + q * (-456 + ex * G);
  } else if (problem == 4 && dim == 2) {
    const AnnulusPsi& A = annulus_psi();
    u[0] = A.at(0, 1, x);
    u[1] = -A.at(1, 0, x);
    g[0][0] = A.at(1, 1, x);
    g[0][1] = A.at(0, 2, x);
    g[1][0] = -A.at(2, 0, x);
    g[1][1] = -A.at(1, 1, x);
    *p = x[0] * x[1] * x[1];
  } else if (problem == 3) {
    // u = 0, p = phi (up to its mean)
    double v = std::sin(2 * kPi * x[0]) * std::cos(kPi * x[1]);
    if (dim == 3) v *= std::cos(kPi * x[2]);
    *p = v;
  }
}

void forcing(int problem, int dim, double nu, const double* x, double* f) {
  for (int a = 0; a < 3; ++a) f[a] = 0;
  if (problem == 1 && dim == 2) {
    double X0 = Phi1::f0(x[0]), X1 = Phi1::f1(x[0]), X2 = Phi1::f2(x[0]), X3 = Phi1::f3(x[0]);
    double Y0 = Phi1::f0(x[1]), Y1 = Phi1::f1(x[1]), Y2 = Phi1::f2(x[1]), Y3 = Phi1::f3(x[1]);
    // Lap u1 = X2 Y1 + X0 Y3 ; Lap u2 = -(X3 Y0 + X1 Y2)
    double lap0 = X2 * Y1 + X0 * Y3;
    double lap1 = -(X3 * Y0 + X1 * Y2);
    double px = -kPi * std::sin(kPi * x[0]) * std::cos(kPi * x[1]);
    double py = -kPi * std::cos(kPi * x[0]) * std::sin(kPi * x[1]);
    f[0] = -nu * lap0 + px;
    f[1] = -nu * lap1 + py;
  } else if (problem == 1 && dim == 3) {
    double F[4][3];
    for (int d = 0; d < 3; ++d) {
      F[0][d] = Phi1::f0(x[d]);
      F[1][d] = Phi1::f1(x[d]);
      F[2][d] = Phi1::f2(x[d]);
      F[3][d] = Phi1::f3(x[d]);
    }
    // Lap of dg/dx_a = sum_b d^3 g / (dx_a dx_b dx_b)
    double lapdg[3];
    for (int a = 0; a < 3; ++a) {
      double s = 0;
      for (int b = 0; b < 3; ++b) {
        double w = 1;
        for (int d = 0; d < 3; ++d) {
          int order = (d == a) + 2 * (d == b);
          w *= F[order][d];
        }
        s += w;
      }
      lapdg[a] = s;
    }
    double lap[3] = {lapdg[1] - lapdg[2], lapdg[2] - lapdg[0], lapdg[0] - lapdg[1]};
    double c0 = std::cos(kPi * x[0]), c1 = std::cos(kPi * x[1]), c2 = std::cos(kPi * x[2]);
    double s0 = std::sin(kPi * x[0]), s1 = std::sin(kPi * x[1]), s2 = std::sin(kPi * x[2]);
    double gp[3] = {-kPi * s0 * c1 * c2, -kPi * c0 * s1 * c2, -kPi * c0 * c1 * s2};
    for (int a = 0; a < 3; ++a) f[a] = -nu * lap[a] + gp[a];
  } else if (problem == 2) {
    double ex = std::exp(x[0]), xx = x[0], y = x[1];
    double P0 = xx * xx * (xx - 1) * (xx - 1);
    double P1 = 4 * xx * xx * xx - 6 * xx * xx + 2 * xx;
    double P2 = 12 * xx * xx - 12 * xx + 2;
    double P3 = 24 * xx - 12;
    double X0 = ex * P0, X1 = ex * (P0 + P1), X2 = ex * (P0 + 2 * P1 + P2),
           X3 = ex * (P0 + 3 * P1 + 3 * P2 + P3);
    double Y0 = Phi1::f0(y), Y1 = Phi1::f1(y), Y2 = Phi1::f2(y), Y3 = Phi1::f3(y);
    double lap0 = X2 * Y1 + X0 * Y3;
    double lap1 = -(X3 * Y0 + X1 * Y2);
    double q = y * y - y, dq = 2 * y - 1;
    double G = 456 + xx * xx * (228 - 5 * q) + 2 * xx * (-228 + q) + 2 * xx * xx * xx * (-36 + q) +
               xx * xx * xx * xx * (12 + q);
    double Gx = 2 * xx * (228 - 5 * q) + 2 * (-228 + q) + 6 * xx * xx * (-36 + q) + 4 * xx * xx * xx * (12 + q);
    double Gq = -5 * xx * xx + 2 * xx + 2 * xx * xx * xx + xx * xx * xx * xx;
    double px = q * ex * (G + Gx);
    double py = dq * (-456 + ex * G) + q * ex * Gq * dq;
    f[0] = -nu * lap0 + px;
    f[1] = -nu * lap1 + py;
  } else if (problem == 4 && dim == 2) {
    // f = -nu Lap u + grad p, Lap u = (psi_yxx + psi_yyy, -(psi_xxx + psi_xyy))
    const AnnulusPsi& A = annulus_psi();
    const double lap0 = A.at(2, 1, x) + A.at(0, 3, x);
    const double lap1 = -(A.at(3, 0, x) + A.at(1, 2, x));
    f[0] = -nu * lap0 + x[1] * x[1];
    f[1] = -nu * lap1 + 2.0 * x[0] * x[1];
  } else if (problem == 3) {
    double a = std::sin(2 * kPi * x[0]), da = 2 * kPi * std::cos(2 * kPi * x[0]);
    double b = std::cos(kPi * x[1]), db = -kPi * std::sin(kPi * x[1]);
    double c = 1, dc = 0;
    if (dim == 3) {
      c = std::cos(kPi * x[2]);
      dc = -kPi * std::sin(kPi * x[2]);
    }
    f[0] = da * b * c;
    f[1] = a * db * c;
    if (dim == 3) f[2] = a * b * dc;
  }
}

// Load vector [f]_i = integral of f . Phi_i with k'+4 Gauss points per direction.
void load_vector(const Problem& P, int problem, int nmodes, const double* amp, const int32_t* wave,
                 const double* phase, double* fout) {
  std::fill(fout, fout + P.nu_dofs, 0.0);
  int nq = load_points(P);
  std::vector<double> xq, wq;
  gauss_legendre01(nq, xq, wq);
  double vol = 1.0;
  for (int d = 0; d < P.dim; ++d) vol *= P.h;
  int nE[3] = {P.N, P.N, P.dim == 3 ? P.N : 1};
  Tab1D tabs[3][2];
  std::vector<VelEval> ve;
  int e[3] = {0, 0, 0};
  for (e[2] = 0; e[2] < nE[2]; ++e[2])
    for (e[1] = 0; e[1] < nE[1]; ++e[1])
      for (e[0] = 0; e[0] < nE[0]; ++e[0]) {
        build_tabs_for_element(P, e, xq, tabs);
        int nq2 = (P.dim == 3) ? nq : 1;
        int q[3] = {0, 0, 0};
        for (q[2] = 0; q[2] < nq2; ++q[2])
          for (q[1] = 0; q[1] < nq; ++q[1])
            for (q[0] = 0; q[0] < nq; ++q[0]) {
              double wt = vol, xi[3] = {0, 0, 0};
              for (int dir = 0; dir < P.dim; ++dir) {
                wt *= wq[q[dir]];
                xi[dir] = (e[dir] + xq[q[dir]]) * P.h;
              }
              GeoPoint geo;
              geometry(P, xi, geo);
              wt *= geo.J;
              const double* x = geo.x;  // forcing at the physical point
              double f[3];
              forcing(problem, P.dim, P.nu, x, f);
              for (int d = 0; d < P.dim; ++d)
                for (int m = 0; m < nmodes; ++m) {
                  double arg = phase[d * nmodes + m];
                  for (int k = 0; k < P.dim; ++k) arg += kPi * wave[m * P.dim + k] * x[k];
                  f[d] += amp[d * nmodes + m] * std::sin(arg);
                }
              tensor_eval_velocity(P, e, tabs, q, ve);
              for (VelEval& v : ve) {
                piola(P, geo, v);
                double s = 0;
                for (int a = 0; a < P.dim; ++a) s += f[a] * v.val[a];
                fout[v.g] += wt * s;
              }
            }
      }
}

// ---------------------------------------------------------------------------
// Load vector with non-homogeneous tangential boundary data (2D), Sec. 4: the
// Nitsche linear form of eq. nitsche_rhs added to the volume load,
//   f_i = (f, Phi_i) + sum_F int_F 2 nu ( -((sym grad Phi_i) n) . g + (C_pen/h_F) g . Phi_i ) dS.
//   kind 0: lid-driven cavity (Sec. 6.4): f = 0, g = (1, 0) on the side y = 1, g = 0 elsewhere.
//   kind 1: a verification flow with u = curl psi, psi = x(1-x)y(1-y), i.e.
//           u = (x(1-x)(1-2y), -(1-2x)y(1-y)), p = 0, f = -nu Lap u = (2nu(1-2y), -2nu(1-2x)),
//           g = u on every side (tangential there, u.n = 0).  u lies in the velocity space for
//           every k' >= 1, so a consistent discretisation returns it exactly.
// Volume and faces use k'+2 Gauss points per direction (exact: the integrands are polynomials
// of degree at most k'+3 per direction).
// ---------------------------------------------------------------------------
static void cavity_data(int kind, double nu, const double* x, int fdir, int side, double* f, double* g) {
  f[0] = f[1] = f[2] = 0.0;
  g[0] = g[1] = g[2] = 0.0;
  if (kind == 0) {
    if (fdir == 1 && side == 1) g[0] = 1.0;
    return;
  }
  f[0] = 2.0 * nu * (1.0 - 2.0 * x[1]);
  f[1] = -2.0 * nu * (1.0 - 2.0 * x[0]);
  g[0] = x[0] * (1.0 - x[0]) * (1.0 - 2.0 * x[1]);
  g[1] = -(1.0 - 2.0 * x[0]) * x[1] * (1.0 - x[1]);
}

void cavity_load(const Problem& P, int kind, double* fout) {
  std::fill(fout, fout + P.nu_dofs, 0.0);
  const int nq = P.kp + 2;
  std::vector<double> xq, wq;
  gauss_legendre01(nq, xq, wq);
  Tab1D tabs[3][2];
  std::vector<VelEval> ve;
  int e[3] = {0, 0, 0};
  for (e[1] = 0; e[1] < P.N; ++e[1])
    for (e[0] = 0; e[0] < P.N; ++e[0]) {
      // volume part (f, Phi_i)
      if (kind == 1) {
        build_tabs_for_element(P, e, xq, tabs);
        int q[3] = {0, 0, 0};
        for (q[1] = 0; q[1] < nq; ++q[1])
          for (q[0] = 0; q[0] < nq; ++q[0]) {
            double x[3] = {(e[0] + xq[q[0]]) * P.h, (e[1] + xq[q[1]]) * P.h, 0.0};
            const double wt = P.h * P.h * wq[q[0]] * wq[q[1]];
            double f[3], g[3];
            cavity_data(kind, P.nu, x, -1, -1, f, g);
            tensor_eval_velocity(P, e, tabs, q, ve);
            for (const VelEval& v : ve) fout[v.g] += wt * (f[0] * v.val[0] + f[1] * v.val[1]);
          }
      }
      // boundary sides of this element: l_h(Phi_i)
      for (int fdir = 0; fdir < 2; ++fdir)
        for (int side = 0; side < 2; ++side) {
          if ((side == 0 && e[fdir] != 0) || (side == 1 && e[fdir] != P.N - 1)) continue;
          double nrm[3] = {0, 0, 0};
          nrm[fdir] = side == 0 ? -1.0 : 1.0;
          const int t = 1 - fdir;  // tangential direction
          Tab1D ftabs[3][2];
          std::vector<double> xs_t(nq);
          for (int qq = 0; qq < nq; ++qq) xs_t[qq] = (e[t] + xq[qq]) * P.h;
          std::vector<double> xs_n(1, side == 0 ? 0.0 : 1.0);
          for (int dir = 0; dir < 2; ++dir) {
            const std::vector<double>& xs = dir == fdir ? xs_n : xs_t;
            eval_on_element(P.sp_lo, e[dir], xs, ftabs[dir][0].v, ftabs[dir][0].d);
            ftabs[dir][0].nloc = P.sp_lo.deg + 1;
            eval_on_element(P.sp_hi, e[dir], xs, ftabs[dir][1].v, ftabs[dir][1].d);
            ftabs[dir][1].nloc = P.sp_hi.deg + 1;
          }
          for (int qq = 0; qq < nq; ++qq) {
            int qf[3] = {0, 0, 0};
            qf[t] = qq;
            double x[3] = {0, 0, 0};
            x[t] = xs_t[qq];
            x[fdir] = xs_n[0];
            const double wt = P.h * wq[qq];
            double f[3], g[3];
            cavity_data(kind, P.nu, x, fdir, side, f, g);
            tensor_eval_velocity(P, e, ftabs, qf, ve);
            for (const VelEval& v : ve) {
              double eps[3][3];
              sym_grad(v, eps);
              double epsn_g = 0.0, g_v = 0.0;
              for (int a = 0; a < 3; ++a) {
                double en = 0.0;
                for (int b = 0; b < 3; ++b) en += eps[a][b] * nrm[b];
                epsn_g += en * g[a];
                g_v += g[a] * v.val[a];
              }
              fout[v.g] += wt * 2.0 * P.nu * (-epsn_g + (P.cpen / P.h) * g_v);
            }
          }
        }
    }
}

// ---------------------------------------------------------------------------
// Sparse kernels on the assembled matrices (plain loops).
// ---------------------------------------------------------------------------
// Saddle-point product [A B^T; B 0] [u; p].
void saddle_matvec(const Problem& P, const double* x, double* y) {
  const double* u = x;
  const double* p = x + P.nu_dofs;
  double* yu = y;
  double* yp = y + P.nu_dofs;
  for (int64_t i = 0; i < P.nu_dofs; ++i) {
    double s = 0;
    for (int64_t k = P.A_ptr[i]; k < P.A_ptr[i + 1]; ++k) s += P.A_val[k] * u[P.A_col[k]];
    yu[i] = s;
  }
  for (int64_t k = 0; k < P.np_dofs; ++k) {
    double s = 0;
    for (int64_t m = P.B_ptr[k]; m < P.B_ptr[k + 1]; ++m) {
      s += P.B_val[m] * u[P.B_col[m]];
      yu[P.B_col[m]] += P.B_val[m] * p[k];  // B^T p
    }
    yp[k] = s;
  }
}

void A_matvec(const Problem& P, const double* x, double* y) {
  for (int64_t i = 0; i < P.nu_dofs; ++i) {
    double s = 0;
    for (int64_t k = P.A_ptr[i]; k < P.A_ptr[i + 1]; ++k) s += P.A_val[k] * x[P.A_col[k]];
    y[i] = s;
  }
}

// Summation order of the inner products: forward (the default) or, for checks of the
// method's sensitivity to rounding, reversed.  The mathematical result is the same.
int g_sum_reverse = 0;

double dot(const double* a, const double* b, int64_t n) {
  double s = 0;
  if (g_sum_reverse) {
    for (int64_t i = n - 1; i >= 0; --i) s += a[i] * b[i];
    return s;
  }
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

// ---------------------------------------------------------------------------
// IC(0) (Sec. 6.4: incomplete Cholesky with zero fill-in of A, and of Q): L L^T ~ M with
// pattern(L) = pattern(tril M), computed row by row in natural order:
//   L_ij = (M_ij - sum_{k<j} L_ik L_jk) / L_jj      for j < i in the pattern
//   L_ii = sqrt(M_ii - sum_{k<i} L_ik^2)
// where the sums run over k present in both rows.  Returns false on a non-positive
// radicand.  alpha adds alpha * M_ii to the diagonal (the shift retry of A's factor).
// ---------------------------------------------------------------------------
bool ic0_factor_csr(const std::vector<int64_t>& M_ptr, const std::vector<int32_t>& M_col,
                    const std::vector<double>& M_val, int64_t n, double alpha, std::vector<int64_t>& L_ptr,
                    std::vector<int32_t>& L_col, std::vector<double>& L_val) {
  L_ptr.assign(1, 0);
  L_col.clear();
  L_val.clear();
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t k = M_ptr[i]; k < M_ptr[i + 1]; ++k) {
      if (M_col[k] > i) break;
      L_col.push_back(M_col[k]);
      double v = M_val[k];
      if (M_col[k] == i) v += alpha * M_val[k];
      L_val.push_back(v);
    }
    L_ptr.push_back(int64_t(L_col.size()));
  }
  for (int64_t i = 0; i < n; ++i) {
    int64_t rb = L_ptr[i], re = L_ptr[i + 1];  // row i, last entry is the diagonal
    for (int64_t m = rb; m < re - 1; ++m) {
      int64_t j = L_col[m];
      int64_t jb = L_ptr[j], je = L_ptr[j + 1];
      double s = L_val[m];
      // sum over k < j present in both rows i and j
      int64_t a = rb, b = jb;
      while (a < m && b < je - 1) {
        if (L_col[a] == L_col[b]) {
          s -= L_val[a] * L_val[b];
          ++a;
          ++b;
        } else if (L_col[a] < L_col[b]) {
          ++a;
        } else {
          ++b;
        }
      }
      L_val[m] = s / L_val[je - 1];
    }
    double d = L_val[re - 1];
    for (int64_t m = rb; m < re - 1; ++m) d -= L_val[m] * L_val[m];
    if (!(d > 0.0)) return false;
    L_val[re - 1] = std::sqrt(d);
  }
  return true;
}

bool ic0_try(Problem& P, double alpha) {
  return ic0_factor_csr(P.A_ptr, P.A_col, P.A_val, P.nu_dofs, alpha, P.L_ptr, P.L_col, P.L_val);
}

// IC(0) of A with the diagonal-shift retries alpha = 1e-3, 1e-2, 1e-1 on breakdown.
int ic0(Problem& P) {
  const double alphas[4] = {0.0, 1e-3, 1e-2, 1e-1};
  for (int s = 0; s < 4; ++s) {
    if (ic0_try(P, alphas[s])) {
      P.have_L = true;
      P.ic_shift_steps = s;
      P.ic_alpha = alphas[s];
      return 0;
    }
  }
  P.have_L = false;
  return -4;
}

// IC(0) of the pressure mass matrix Q (Sec. 6.4 factors both blocks).  Q is SPD; no shift.
int ic0_Q(Problem& P) {
  if (!ic0_factor_csr(P.Q_ptr, P.Q_col, P.Q_val, P.np_dofs, 0.0, P.LQ_ptr, P.LQ_col, P.LQ_val)) return -4;
  P.have_LQ = true;
  return 0;
}

// z = (L L^T)^{-1} r: forward substitution, then backward substitution with L^T done
// column-wise from the rows of L.
void ic0_solve_csr(const std::vector<int64_t>& L_ptr, const std::vector<int32_t>& L_col,
                   const std::vector<double>& L_val, int64_t n, const double* r, double* z) {
  std::vector<double> y(n);
  for (int64_t i = 0; i < n; ++i) {
    double s = r[i];
    int64_t re = L_ptr[i + 1];
    for (int64_t m = L_ptr[i]; m < re - 1; ++m) s -= L_val[m] * y[L_col[m]];
    y[i] = s / L_val[re - 1];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    int64_t re = L_ptr[i + 1];
    double zi = y[i] / L_val[re - 1];
    z[i] = zi;
    for (int64_t m = L_ptr[i]; m < re - 1; ++m) y[L_col[m]] -= L_val[m] * zi;
  }
}

void ic0_apply(const Problem& P, const double* r, double* z) {
  ic0_solve_csr(P.L_ptr, P.L_col, P.L_val, P.nu_dofs, r, z);
}

// Dense Cholesky (row-major, lower) for the ideal preconditioner blocks.
bool dense_cholesky(std::vector<double>& a, int64_t n) {
  for (int64_t j = 0; j < n; ++j) {
    double d = a[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= a[j * n + k] * a[j * n + k];
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    a[j * n + j] = d;
    for (int64_t i = j + 1; i < n; ++i) {
      double s = a[i * n + j];
      for (int64_t k = 0; k < j; ++k) s -= a[i * n + k] * a[j * n + k];
      a[i * n + j] = s / d;
    }
  }
  return true;
}

void dense_chol_solve(const std::vector<double>& l, int64_t n, const double* r, double* z) {
  std::vector<double> y(n);
  for (int64_t i = 0; i < n; ++i) {
    double s = r[i];
    for (int64_t k = 0; k < i; ++k) s -= l[i * n + k] * y[k];
    y[i] = s / l[i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int64_t k = i + 1; k < n; ++k) s -= l[k * n + i] * z[k];
    z[i] = s / l[i * n + i];
  }
}

enum { PCA_IC0 = 0, PCA_ICPCG = 1, PCA_JACOBI = 2, PCA_EXACT = 3, PCA_JPCG = 4 };
enum { PCQ_DIAG = 0, PCQ_EXACT = 1, PCQ_JPCG = 2, PCQ_IC0 = 3, PCQ_ICPCG = 4 };

// Inner PCG on A (Sec. 6.4): x0 = 0, stop when ||r||_2 <= rtol ||b||_2, tested after
// each update; preconditioner IC(0) (PCA_ICPCG) or Jacobi (PCA_JPCG).
int pcg_A(const Problem& P, int which, const double* b, double* x, double rtol, int maxit) {
  int64_t n = P.nu_dofs;
  std::vector<double> r(b, b + n), z(n), p(n), q(n);
  std::fill(x, x + n, 0.0);
  double bnorm = std::sqrt(dot(b, b, n));
  if (bnorm == 0.0) return 0;
  auto prec = [&](const double* in, double* out) {
    if (which == PCA_ICPCG) {
      ic0_apply(P, in, out);
    } else {
      for (int64_t i = 0; i < n; ++i) out[i] = in[i] / csr_at(const_cast<Problem&>(P).A_ptr,
                                                               const_cast<Problem&>(P).A_col,
                                                               const_cast<Problem&>(P).A_val, i, i);
    }
  };
  prec(r.data(), z.data());
  p = z;
  double rho = dot(r.data(), z.data(), n);
  int it = 0;
  while (it < maxit) {
    A_matvec(P, p.data(), q.data());
    double alpha = rho / dot(p.data(), q.data(), n);
    for (int64_t i = 0; i < n; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    ++it;
    if (std::sqrt(dot(r.data(), r.data(), n)) <= rtol * bnorm) break;
    prec(r.data(), z.data());
    double rho_new = dot(r.data(), z.data(), n);
    double beta = rho_new / rho;
    rho = rho_new;
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  return it;
}

// Inner PCG on the pressure mass matrix Q, preconditioned by Diag(Q) (PCQ_JPCG: the
// pressure half of the PCG(A,Q) variant, Sec. 5.1) or by IC(0) of Q (PCQ_ICPCG: the
// pressure half of IC(0)-PCG(A,Q), Sec. 6.4).  x0 = 0, stop when ||r||_2 <= rtol ||b||_2,
// tested after each update.
int pcg_Q(const Problem& P, int which, const double* b, double* x, double rtol, int maxit) {
  int64_t n = P.np_dofs;
  std::vector<double> r(b, b + n), z(n), p(n), q(n);
  std::fill(x, x + n, 0.0);
  double bnorm = std::sqrt(dot(b, b, n));
  if (bnorm == 0.0) return 0;
  auto prec = [&](const double* in, double* out) {
    if (which == PCQ_ICPCG) {
      ic0_solve_csr(P.LQ_ptr, P.LQ_col, P.LQ_val, n, in, out);
    } else {
      for (int64_t i = 0; i < n; ++i) out[i] = in[i] / P.diagQ[i];
    }
  };
  prec(r.data(), z.data());
  p = z;
  double rho = dot(r.data(), z.data(), n);
  int it = 0;
  while (it < maxit) {
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int64_t k = P.Q_ptr[i]; k < P.Q_ptr[i + 1]; ++k) acc += P.Q_val[k] * p[P.Q_col[k]];
      q[i] = acc;
    }
    double alpha = rho / dot(p.data(), q.data(), n);
    for (int64_t i = 0; i < n; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    ++it;
    if (std::sqrt(dot(r.data(), r.data(), n)) <= rtol * bnorm) break;
    prec(r.data(), z.data());
    double rho_new = dot(r.data(), z.data(), n);
    double beta = rho_new / rho;
    rho = rho_new;
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  return it;
}

// Block-diagonal preconditioner M = blkdiag(M_A, M_Q) applied to r: z = M^{-1} r (eq.
// general_precond_M).  M_Q = Diag(Q)/(2 nu), Q/(2 nu) (exact), L_Q L_Q^T/(2 nu) with
// L_Q the IC(0) factor of Q (PCQ_IC0), or Q/(2 nu) approximated by PCG on Q with the Jacobi
// (PCQ_JPCG) or IC(0) (PCQ_ICPCG) preconditioner; PCG iterations on Q are added to the
// inner count.
int apply_precond(const Problem& P, int pcA, int pcQ, double inner_tol, const double* r, double* z) {
  int64_t nu = P.nu_dofs, np = P.np_dofs;
  int inner = 0;
  switch (pcA) {
    case PCA_IC0:
      ic0_apply(P, r, z);
      break;
    case PCA_ICPCG:
    case PCA_JPCG:
      inner = pcg_A(P, pcA, r, z, inner_tol, 200);
      break;
    case PCA_JACOBI:
      for (int64_t i = 0; i < nu; ++i)
        z[i] = r[i] / csr_at(const_cast<Problem&>(P).A_ptr, const_cast<Problem&>(P).A_col,
                             const_cast<Problem&>(P).A_val, i, i);
      break;
    case PCA_EXACT:
      dense_chol_solve(P.cholA, nu, r, z);
      break;
  }
  if (pcQ == PCQ_DIAG) {
    for (int64_t k = 0; k < np; ++k) z[nu + k] = 2.0 * P.nu * r[nu + k] / P.diagQ[k];
  } else if (pcQ == PCQ_JPCG || pcQ == PCQ_ICPCG) {
    inner += pcg_Q(P, pcQ, r + nu, z + nu, inner_tol, 200);
    for (int64_t k = 0; k < np; ++k) z[nu + k] *= 2.0 * P.nu;
  } else if (pcQ == PCQ_IC0) {
    ic0_solve_csr(P.LQ_ptr, P.LQ_col, P.LQ_val, np, r + nu, z + nu);
    for (int64_t k = 0; k < np; ++k) z[nu + k] *= 2.0 * P.nu;
  } else {
    dense_chol_solve(P.cholQ, np, r + nu, z + nu);
    for (int64_t k = 0; k < np; ++k) z[nu + k] *= 2.0 * P.nu;
  }
  return inner;
}

// ---------------------------------------------------------------------------
// Preconditioned MINRES (Sec. 5; Paige-Saunders short recurrence with Givens QR,
// in the form of Elman, Silvester & Wathen).  x0 = 0.  Iteration j:
//   z_j <- z_j / gamma_j;  q = Acal z_j;  delta_j = q . z_j
//   v_{j+1} = q - (delta_j/gamma_j) v_j - (gamma_j/gamma_{j-1}) v_{j-1}
//   z_{j+1} = M^{-1} v_{j+1};  gamma_{j+1} = sqrt(v_{j+1} . z_{j+1})
//   a0 = c_j delta_j - c_{j-1} s_j gamma_j;  a1 = sqrt(a0^2 + gamma_{j+1}^2)
//   a2 = s_j delta_j + c_{j-1} c_j gamma_j;  a3 = s_{j-1} gamma_j
//   c_{j+1} = a0/a1;  s_{j+1} = gamma_{j+1}/a1
//   w_{j+1} = (z_j - a3 w_{j-1} - a2 w_j)/a1;  x_j = x_{j-1} + c_{j+1} eta w_{j+1}
//   eta <- -s_{j+1} eta;  stop when |eta| <= tol gamma_1   (|eta| = ||r_j||_{M^{-1}})
// ---------------------------------------------------------------------------
struct MinresOut {
  int iters = 0;
  int inner_total = 0;
  int status = 0;
};

MinresOut minres(const Problem& P, const double* b, double* x, double tol, int maxit, int pcA, int pcQ,
                 double inner_tol, bool fixed_iters, double* eta_hist, double* x_hist) {
  int64_t n = P.nu_dofs + P.np_dofs;
  MinresOut out;
  std::vector<double> v_prev(n, 0.0), v(b, b + n), v_next(n), z(n), z_next(n), q(n);
  std::vector<double> w_prev(n, 0.0), w(n, 0.0), w_next(n);
  std::fill(x, x + n, 0.0);
  out.inner_total += apply_precond(P, pcA, pcQ, inner_tol, v.data(), z.data());
  double g2 = dot(v.data(), z.data(), n);
  if (g2 < 0) {
    out.status = -4;
    return out;
  }
  double gamma = std::sqrt(g2), gamma_prev = 1.0, gamma1 = gamma;
  double eta = gamma;
  double c_prev = 1, c = 1, s_prev = 0, s = 0;
  if (eta_hist) eta_hist[0] = std::fabs(eta);
  if (gamma1 == 0.0) return out;
  int j = 0;
  while (j < maxit) {
    if (!fixed_iters && std::fabs(eta) <= tol * gamma1) break;
    ++j;
    for (int64_t i = 0; i < n; ++i) z[i] /= gamma;
    saddle_matvec(P, z.data(), q.data());
    double delta = dot(q.data(), z.data(), n);
    for (int64_t i = 0; i < n; ++i)
      v_next[i] = q[i] - (delta / gamma) * v[i] - (gamma / gamma_prev) * v_prev[i];
    out.inner_total += apply_precond(P, pcA, pcQ, inner_tol, v_next.data(), z_next.data());
    double gn2 = dot(v_next.data(), z_next.data(), n);
    if (gn2 < 0) {
      out.status = -4;
      out.iters = j;
      return out;
    }
    double gamma_next = std::sqrt(gn2);
    double a0 = c * delta - c_prev * s * gamma;
    double a1 = std::sqrt(a0 * a0 + gamma_next * gamma_next);
    double a2 = s * delta + c_prev * c * gamma;
    double a3 = s_prev * gamma;
    double c_next = a0 / a1, s_next = gamma_next / a1;
    for (int64_t i = 0; i < n; ++i) w_next[i] = (z[i] - a3 * w_prev[i] - a2 * w[i]) / a1;
    for (int64_t i = 0; i < n; ++i) x[i] += c_next * eta * w_next[i];
    eta = -s_next * eta;
    if (eta_hist) eta_hist[j] = std::fabs(eta);
    if (x_hist) std::memcpy(x_hist + (j - 1) * n, x, sizeof(double) * n);
    // shift the recurrences
    v_prev.swap(v);
    v.swap(v_next);
    z.swap(z_next);
    w_prev.swap(w);
    w.swap(w_next);
    gamma_prev = gamma;
    gamma = gamma_next;
    c_prev = c;
    c = c_next;
    s_prev = s;
    s = s_next;
    if (gamma == 0.0) break;  // exact invariant subspace: x is the exact solution
  }
  out.iters = j;
  if (!fixed_iters && std::fabs(eta) > tol * gamma1) out.status = 1;
  return out;
}

// Zero-mean pressure (Sec. 3.2; imposed by filtering after the solve, Sec. 6.4): p <- p - (w.p)/(w.1).
// Zero-mean pressure (the L2 mean, Sec. 3.2): p <- p - (w.p)/(w.kappa) kappa, kappa the
// coefficients of the constant function (all ones on the identity map).
void project_pressure(const Problem& P, double* p) {
  double wp = 0, w1 = 0;
  for (int64_t k = 0; k < P.np_dofs; ++k) {
    wp += P.wvec[k] * p[k];
    w1 += P.wvec[k] * P.kappa[k];
  }
  double m = wp / w1;
  for (int64_t k = 0; k < P.np_dofs; ++k) p[k] -= m * P.kappa[k];
}

// Residual norms of the original system: ||b - Acal x||_2 / ||b||_2 and the M^{-1}-norm
// ratio with the linear preconditioner that MINRES used (IC(0) when PCG was inner).
void true_residuals(const Problem& P, const double* b, const double* x, int pcA, int pcQ, double* rel2,
                    double* relM) {
  int64_t n = P.nu_dofs + P.np_dofs;
  std::vector<double> r(n), z(n), zb(n);
  saddle_matvec(P, x, r.data());
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
  int lin = (pcA == PCA_ICPCG) ? PCA_IC0 : (pcA == PCA_JPCG ? PCA_JACOBI : pcA);
  int linq = pcQ == PCQ_JPCG ? PCQ_DIAG : (pcQ == PCQ_ICPCG ? PCQ_IC0 : pcQ);
  apply_precond(P, lin, linq, 0.0, r.data(), z.data());
  apply_precond(P, lin, linq, 0.0, b, zb.data());
  double bb = dot(b, b, n), bm = dot(b, zb.data(), n);
  *rel2 = bb > 0 ? std::sqrt(dot(r.data(), r.data(), n) / bb) : 0.0;
  *relM = bm > 0 ? std::sqrt(std::max(0.0, dot(r.data(), z.data(), n)) / bm) : 0.0;
}

bool prepare_precond(Problem& P, int pcA, int pcQ) {
  if ((pcA == PCA_IC0 || pcA == PCA_ICPCG) && !P.have_L) {
    if (ic0(P) != 0) return false;
  }
  if ((pcQ == PCQ_IC0 || pcQ == PCQ_ICPCG) && !P.have_LQ) {
    if (ic0_Q(P) != 0) return false;
  }
  if (pcA == PCA_EXACT && !P.have_dense_A) {
    int64_t n = P.nu_dofs;
    P.cholA.assign(n * n, 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = P.A_ptr[i]; k < P.A_ptr[i + 1]; ++k) P.cholA[i * n + P.A_col[k]] = P.A_val[k];
    if (!dense_cholesky(P.cholA, n)) return false;
    P.have_dense_A = true;
  }
  if (pcQ == PCQ_EXACT && !P.have_dense_Q) {
    int64_t n = P.np_dofs;
    P.cholQ.assign(n * n, 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = P.Q_ptr[i]; k < P.Q_ptr[i + 1]; ++k) P.cholQ[i * n + P.Q_col[k]] = P.Q_val[k];
    if (!dense_cholesky(P.cholQ, n)) return false;
    P.have_dense_Q = true;
  }
  return true;
}

}  // namespace

// ===========================================================================
// C interface used by the Python test harness (ctypes).
// ===========================================================================
extern "C" {

// info layout for or_solve / or_minres
// [0] iters [1] inner_total [2] status [3] ic_shift_steps [4] relres_est (|eta|/gamma1)
// [5] relres_true_2 [6] relres_true_Minv
// flags bit 0: build the sparsity patterns only (no quadrature), for size checks.
// flags: bit 0 pattern only (no assembly); bit 1 the 1/8-annulus geometry (2D).
void* or_setup(int N, int kp, int dim, double nu, double cpen, int flags) {
  if (N < 1 || kp < 1 || (dim != 2 && dim != 3) || !(nu > 0)) return nullptr;
  if ((flags & 2) && dim != 2) return nullptr;
  Problem* P = new Problem();
  P->geom = (flags & 2) ? 1 : 0;
  P->N = N;
  P->kp = kp;
  P->dim = dim;
  P->nu = nu;
  P->pdeg = kp + 1;
  P->h = 1.0 / N;
  P->cpen = (cpen < 0) ? 5.0 * (kp + 1) : cpen;
  P->sp_hi = make_space(P->pdeg, N);
  P->sp_lo = make_space(kp, N);
  int64_t off = 0;
  for (int c = 0; c < dim; ++c) {
    int64_t cnt = 1;
    for (int dir = 0; dir < dim; ++dir) {
      P->vcount[c][dir] = (dir == c) ? P->sp_hi.nfun - 2 : P->sp_lo.nfun;
      cnt *= P->vcount[c][dir];
    }
    P->voff[c] = off;
    off += cnt;
  }
  P->voff[dim] = off;
  P->nu_dofs = off;
  P->np_dofs = 1;
  for (int dir = 0; dir < dim; ++dir) P->np_dofs *= P->sp_lo.nfun;
  build_patterns(*P);
  P->kappa.assign(P->np_dofs, 1.0);
  if (!(flags & 1)) {
    assemble(*P);
    // kappa = Q^{-1} w by CG preconditioned with IC(0) of Q (Q's Cholesky factor for the
    // polar map, where 1/J depends on xi_0 alone and Q keeps its Kronecker structure)
    if (P->geom != 0) {
      if (ic0_Q(*P) != 0) {
        delete P;
        return nullptr;
      }
      pcg_Q(*P, PCQ_ICPCG, P->wvec.data(), P->kappa.data(), 1e-15, 50);
    }
  }
  return P;
}

void or_free(void* h) { delete static_cast<Problem*>(h); }

void or_sizes(void* h, int64_t* n_u, int64_t* n_p) {
  Problem* P = static_cast<Problem*>(h);
  *n_u = P->nu_dofs;
  *n_p = P->np_dofs;
}

// which: 0 = A, 1 = B, 2 = Q, 3 = L (after or_ic0), 4 = L_Q (after or_ic0_q)
int64_t or_nnz(void* h, int which) {
  Problem* P = static_cast<Problem*>(h);
  switch (which) {
    case 0: return int64_t(P->A_col.size());
    case 1: return int64_t(P->B_col.size());
    case 2: return int64_t(P->Q_col.size());
    case 3: return int64_t(P->L_col.size());
    case 4: return int64_t(P->LQ_col.size());
  }
  return -1;
}

void or_get_csr(void* h, int which, int64_t* ptr, int32_t* col, double* val) {
  Problem* P = static_cast<Problem*>(h);
  const std::vector<int64_t>* pp = nullptr;
  const std::vector<int32_t>* cc = nullptr;
  const std::vector<double>* vv = nullptr;
  switch (which) {
    case 0: pp = &P->A_ptr; cc = &P->A_col; vv = &P->A_val; break;
    case 1: pp = &P->B_ptr; cc = &P->B_col; vv = &P->B_val; break;
    case 2: pp = &P->Q_ptr; cc = &P->Q_col; vv = &P->Q_val; break;
    case 3: pp = &P->L_ptr; cc = &P->L_col; vv = &P->L_val; break;
    case 4: pp = &P->LQ_ptr; cc = &P->LQ_col; vv = &P->LQ_val; break;
    default: return;
  }
  if (ptr) std::memcpy(ptr, pp->data(), pp->size() * sizeof(int64_t));
  if (col) std::memcpy(col, cc->data(), cc->size() * sizeof(int32_t));
  if (val) std::memcpy(val, vv->data(), vv->size() * sizeof(double));
}

void or_get_diagQ_w(void* h, double* diagQ, double* w) {
  Problem* P = static_cast<Problem*>(h);
  if (diagQ) std::memcpy(diagQ, P->diagQ.data(), P->np_dofs * sizeof(double));
  if (w) std::memcpy(w, P->wvec.data(), P->np_dofs * sizeof(double));
}

int or_ic0(void* h, int* shift_steps) {
  Problem* P = static_cast<Problem*>(h);
  int rc = P->have_L ? 0 : ic0(*P);
  if (shift_steps) *shift_steps = P->ic_shift_steps;
  return rc;
}

// IC(0) factor of Q (0, or -4 on a non-positive pivot).
int or_ic0_q(void* h) {
  Problem* P = static_cast<Problem*>(h);
  return P->have_LQ ? 0 : ic0_Q(*P);
}

// Inner products summed forward (0, the default) or in reverse order (1).
void or_set_sum_order(int reverse) { g_sum_reverse = reverse ? 1 : 0; }

// Load vector(s).  problem: 0 none, 1 manufactured (default), 2 paper square, 3 gradient.
// amp [nrhs][dim][nmodes], wave [nrhs][nmodes][dim], phase [nrhs][dim][nmodes]; f [nrhs][n_u].
void or_load(void* h, int problem, int nrhs, int nmodes, const double* amp, const int32_t* wave,
             const double* phase, double* f) {
  Problem* P = static_cast<Problem*>(h);
  for (int r = 0; r < nrhs; ++r) {
    const double* a = amp ? amp + int64_t(r) * P->dim * nmodes : nullptr;
    const int32_t* k = wave ? wave + int64_t(r) * nmodes * P->dim : nullptr;
    const double* ph = phase ? phase + int64_t(r) * P->dim * nmodes : nullptr;
    load_vector(*P, problem, a ? nmodes : 0, a, k, ph, f + int64_t(r) * P->nu_dofs);
  }
}

// Cavity-type load vector (2D; kind 0 lid, 1 verification flow).  Returns -1 for 3D or an
// unknown kind.
int or_load_cavity(void* h, int kind, double* f) {
  Problem* P = static_cast<Problem*>(h);
  if (P->dim != 2 || P->geom != 0 || kind < 0 || kind > 1) return -1;  // the cavity is the unit square
  cavity_load(*P, kind, f);
  return 0;
}

void or_matvec(void* h, const double* x, double* y) { saddle_matvec(*static_cast<Problem*>(h), x, y); }

int or_precond(void* h, int pcA, int pcQ, double inner_tol, const double* r, double* z, int* inner) {
  Problem* P = static_cast<Problem*>(h);
  if (!prepare_precond(*P, pcA, pcQ)) return -4;
  int it = apply_precond(*P, pcA, pcQ, inner_tol, r, z);
  if (inner) *inner = it;
  return 0;
}

// Plain MINRES on Acal x = b (no projection).  fixed != 0 runs exactly maxit iterations.
int or_minres(void* h, const double* b, double* x, double tol, int maxit, int pcA, int pcQ,
              double inner_tol, int fixed, double* info, double* eta_hist, double* x_hist) {
  Problem* P = static_cast<Problem*>(h);
  if (!prepare_precond(*P, pcA, pcQ)) {
    if (info) info[2] = -4;
    return -4;
  }
  int64_t n = P->nu_dofs + P->np_dofs;
  MinresOut o = minres(*P, b, x, tol, maxit, pcA, pcQ, inner_tol, fixed != 0, eta_hist, x_hist);
  if (info) {
    info[0] = o.iters;
    info[1] = o.inner_total;
    info[2] = o.status;
    info[3] = P->ic_shift_steps;
    double rel2 = 0, relM = 0;
    true_residuals(*P, b, x, pcA, pcQ, &rel2, &relM);
    info[4] = 0;
    info[5] = rel2;
    info[6] = relM;
    (void)n;
  }
  return o.status;
}

// Full solve as the product path defines it: b = [f; 0], MINRES, zero-mean pressure.
int or_solve(void* h, const double* f, double* u, double* p, double tol, int maxit, int pcA, int pcQ,
             double inner_tol, int fixed, double* info) {
  Problem* P = static_cast<Problem*>(h);
  int64_t nu = P->nu_dofs, np = P->np_dofs, n = nu + np;
  std::vector<double> b(n, 0.0), x(n);
  std::memcpy(b.data(), f, nu * sizeof(double));
  int rc = or_minres(h, b.data(), x.data(), tol, maxit, pcA, pcQ, inner_tol, fixed, info, nullptr, nullptr);
  project_pressure(*P, x.data() + nu);
  std::memcpy(u, x.data(), nu * sizeof(double));
  std::memcpy(p, x.data() + nu, np * sizeof(double));
  return rc;
}

void or_project(void* h, double* p) { project_pressure(*static_cast<Problem*>(h), p); }

// Adjoint solve for a loss L(u, p) with p the zero-mean pressure: the right-hand side
// is [g_u; P^T g_p] with P^T g_p = g_p - w (1.g_p)/(w.1); the system matrix is symmetric
// so the same MINRES and preconditioner are used.  lambda_p is returned zero-mean.
int or_adjoint(void* h, const double* g_u, const double* g_p, double* lam_u, double* lam_p, double tol,
               int maxit, int pcA, int pcQ, double inner_tol, double* info) {
  Problem* P = static_cast<Problem*>(h);
  int64_t nu = P->nu_dofs, np = P->np_dofs, n = nu + np;
  std::vector<double> b(n, 0.0), x(n);
  std::memcpy(b.data(), g_u, nu * sizeof(double));
  // P^T g_p for the projection P = I - kappa w^T / (w.kappa)
  double s1 = 0, w1 = 0;
  for (int64_t k = 0; k < np; ++k) {
    s1 += P->kappa[k] * g_p[k];
    w1 += P->wvec[k] * P->kappa[k];
  }
  for (int64_t k = 0; k < np; ++k) b[nu + k] = g_p[k] - P->wvec[k] * s1 / w1;
  int rc = or_minres(h, b.data(), x.data(), tol, maxit, pcA, pcQ, inner_tol, 0, info, nullptr, nullptr);
  project_pressure(*P, x.data() + nu);
  std::memcpy(lam_u, x.data(), nu * sizeof(double));
  std::memcpy(lam_p, x.data() + nu, np * sizeof(double));
  return rc;
}

// lambda_u^T A u / nu  (A is proportional to nu, so dA/dnu = A/nu).
double or_dnu_dot(void* h, const double* lam_u, const double* u) {
  Problem* P = static_cast<Problem*>(h);
  std::vector<double> au(P->nu_dofs);
  A_matvec(*P, u, au.data());
  return dot(lam_u, au.data(), P->nu_dofs) / P->nu;
}

// Discrete solution evaluation at parametric points (the physical points F(xi); on the
// identity map the two coincide): velocity, its divergence, pressure.
// pts [npts][dim]; out [npts][dim + 2] = (u_1..u_dim, div u, p).
void or_eval(void* h, const double* u, const double* p, int64_t npts, const double* pts, double* out) {
  Problem* P = static_cast<Problem*>(h);
  int dim = P->dim;
  for (int64_t t = 0; t < npts; ++t) {
    int e[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) e[d] = std::min(P->N - 1, std::max(0, int(pts[t * dim + d] * P->N)));
    Tab1D tabs[3][2];
    for (int dir = 0; dir < dim; ++dir) {
      std::vector<double> xs(1, pts[t * dim + dir]);
      eval_on_element(P->sp_lo, e[dir], xs, tabs[dir][0].v, tabs[dir][0].d);
      tabs[dir][0].nloc = P->sp_lo.deg + 1;
      eval_on_element(P->sp_hi, e[dir], xs, tabs[dir][1].v, tabs[dir][1].d);
      tabs[dir][1].nloc = P->sp_hi.deg + 1;
    }
    int q[3] = {0, 0, 0};
    std::vector<VelEval> ve;
    std::vector<PreEval> pe;
    tensor_eval_velocity(*P, e, tabs, q, ve);
    tensor_eval_pressure(*P, e, tabs, q, pe);
    GeoPoint geo;
    geometry(*P, pts + t * dim, geo);
    for (VelEval& v : ve) piola(*P, geo, v);
    for (PreEval& pp : pe) pp.val /= geo.J;
    double* o = out + t * (dim + 2);
    for (int k = 0; k < dim + 2; ++k) o[k] = 0;
    for (const VelEval& v : ve) {
      for (int a = 0; a < dim; ++a) o[a] += u[v.g] * v.val[a];
      for (int a = 0; a < dim; ++a) o[dim] += u[v.g] * v.grad[a][a];
    }
    for (const PreEval& pp : pe) o[dim + 1] += p[pp.g] * pp.val;
  }
}

// Error norms against the exact solution of `problem`: out = (|u-u_h|_H1, ||u-u_h||_L2, ||p-p_h||_L2)
// with k'+4 Gauss points per direction; the exact pressure's mean is removed first.
void or_errors(void* h, int problem, const double* u, const double* p, double* out) {
  Problem* P = static_cast<Problem*>(h);
  int dim = P->dim;
  int nq = load_points(*P);
  std::vector<double> xq, wq;
  gauss_legendre01(nq, xq, wq);
  double vol = 1.0;
  for (int d = 0; d < dim; ++d) vol *= P->h;
  // mean of the exact pressure
  double pmean = 0;
  int nE[3] = {P->N, P->N, dim == 3 ? P->N : 1};
  for (int pass = 0; pass < 2; ++pass) {
    double h1 = 0, l2u = 0, l2p = 0, pm = 0;
    int e[3] = {0, 0, 0};
    Tab1D tabs[3][2];
    std::vector<VelEval> ve;
    std::vector<PreEval> pe;
    for (e[2] = 0; e[2] < nE[2]; ++e[2])
      for (e[1] = 0; e[1] < nE[1]; ++e[1])
        for (e[0] = 0; e[0] < nE[0]; ++e[0]) {
          build_tabs_for_element(*P, e, xq, tabs);
          int nq2 = dim == 3 ? nq : 1;
          int q[3] = {0, 0, 0};
          for (q[2] = 0; q[2] < nq2; ++q[2])
            for (q[1] = 0; q[1] < nq; ++q[1])
              for (q[0] = 0; q[0] < nq; ++q[0]) {
                double wt = vol, xi[3] = {0, 0, 0};
                for (int dir = 0; dir < dim; ++dir) {
                  wt *= wq[q[dir]];
                  xi[dir] = (e[dir] + xq[q[dir]]) * P->h;
                }
                GeoPoint geo;
                geometry(*P, xi, geo);
                wt *= geo.J;
                const double* x = geo.x;
                double ue[3], ge[3][3], pex;
                exact_solution(problem, dim, x, ue, ge, &pex);
                if (pass == 0) {
                  pm += wt * pex;
                  continue;
                }
                tensor_eval_velocity(*P, e, tabs, q, ve);
                tensor_eval_pressure(*P, e, tabs, q, pe);
                for (VelEval& v : ve) piola(*P, geo, v);
                for (PreEval& pp : pe) pp.val /= geo.J;
                double uh[3] = {0, 0, 0}, gh[3][3] = {{0}}, ph = 0;
                for (const VelEval& v : ve)
                  for (int a = 0; a < 3; ++a) {
                    uh[a] += u[v.g] * v.val[a];
                    for (int b = 0; b < 3; ++b) gh[a][b] += u[v.g] * v.grad[a][b];
                  }
                for (const PreEval& pp : pe) ph += p[pp.g] * pp.val;
                for (int a = 0; a < dim; ++a) {
                  l2u += wt * (ue[a] - uh[a]) * (ue[a] - uh[a]);
                  for (int b = 0; b < dim; ++b) h1 += wt * (ge[a][b] - gh[a][b]) * (ge[a][b] - gh[a][b]);
                }
                l2p += wt * (pex - pmean - ph) * (pex - pmean - ph);
              }
        }
    if (pass == 0) {
      double area = 0.0;  // |Omega| = w . kappa, the integral of the constant function
      for (int64_t k = 0; k < P->np_dofs; ++k) area += P->wvec[k] * P->kappa[k];
      pmean = pm / area;
    } else {
      out[0] = std::sqrt(h1);
      out[1] = std::sqrt(l2u);
      out[2] = std::sqrt(l2p);
    }
  }
}

}  // extern "C"
