// Gauss-quadrature assembly of the discrete Stokes operators on the device (Sec. 4 of
// the paper) and of the load vector.
//
// Every CSR entry is computed by the workgroup lane that owns it, as a quadrature sum
// over the elements shared by the supports of its two basis functions: no scatter, no
// atomics, so the result is deterministic.  Basis functions are tensor products of 1D
// B-splines (Sec. 2.2); their values and derivatives at the Gauss points of every
// element come from a table built by k_tables_1d with the triangular Cox-de Boor
// recurrence.
//   A_ij = nu * int (delta_cd grad B_i . grad B_j + d_d B_i d_c B_j)          (2 nu eps:eps)
//        + sum over boundary faces of nu * int [ -(delta_cd d_n B_i + n_c d_d B_i) B_j
//                                                 -(delta_cd d_n B_j + n_d d_c B_j) B_i
//                                                 + 2 (C_pen/h_F) delta_cd B_i B_j ]
//   (Nitsche form eta_h, eq. nitsche_lhs, a_h = a - eta_h; component c of Phi_i, d of Phi_j)
//   B_kj = -int phi_k d_d B_j;  Q_kk = int phi_k^2;  w_k = int phi_k;  f_i = int f . Phi_i
#include "stokes_internal.h"

namespace stk {

constexpr double kPiD = 3.14159265358979323846;

// Gauss-Legendre node/weight i of the n-point rule on [0,1] (Newton on P_n).
__device__ void gl_node(int n, int i, double* x, double* w) {
  double t = cos(kPiD * (i + 0.75) / (n + 0.5));
  double dp = 1.0;
  for (int it = 0; it < 60; ++it) {
    double p0 = 1.0, p1 = t;
    for (int k = 1; k < n; ++k) {
      const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
      p0 = p1;
      p1 = p2;
    }
    dp = n * (t * p1 - p0) / (t * t - 1.0);
    const double dt = p1 / dp;
    t -= dt;
    if (fabs(dt) < 1e-16) break;
  }
  double p0 = 1.0, p1 = t;
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  dp = n * (t * p1 - p0) / (t * t - 1.0);
  *x = 0.5 * (1.0 - t);
  *w = 1.0 / ((1.0 - t * t) * dp * dp);
}

// Knot t_k of the open uniform knot vector of degree d on N elements.
__device__ __forceinline__ double knot(int k, int d, int N) {
  if (k <= d) return 0.0;
  if (k >= N + d) return 1.0;
  return double(k - d) / N;
}

// Values N[r] and derivatives D[r] (r = 0..d) of the functions e..e+d at x in element e,
// by the triangular recurrence on the knot differences (left/right arrays).
__device__ void basis_on_element(int d, int N, int e, double x, double* Nv, double* Dv) {
  const int span = d + e;
  double ndu[5][5];  // ndu[r][j]: value table (lower: knot differences)
  double left[5], right[5];
  ndu[0][0] = 1.0;
  for (int j = 1; j <= d; ++j) {
    left[j] = x - knot(span + 1 - j, d, N);
    right[j] = knot(span + j, d, N) - x;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      ndu[j][r] = right[r + 1] + left[j - r];
      const double tmp = ndu[r][j - 1] / ndu[j][r];
      ndu[r][j] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    ndu[j][j] = saved;
  }
  for (int r = 0; r <= d; ++r) Nv[r] = ndu[r][d];
  // first derivative from the degree d-1 values: N'_{e+r} = d (N_{e+r,d-1}/(t_{e+r+d}-t_{e+r})
  //                                                          - N_{e+r+1,d-1}/(t_{e+r+d+1}-t_{e+r+1}))
  for (int r = 0; r <= d; ++r) {
    double v = 0.0;
    if (d > 0) {
      const int i = e + r;
      // degree d-1 function i lives at position r-1 of the degree d-1 table (functions e+1..e+d)
      const double a = (r >= 1) ? ndu[r - 1][d - 1] : 0.0;
      const double b = (r <= d - 1) ? ndu[r][d - 1] : 0.0;
      const double den1 = knot(i + d, d, N) - knot(i, d, N);
      const double den2 = knot(i + d + 1, d, N) - knot(i + 1, d, N);
      if (den1 > 0.0) v += d * a / den1;
      if (den2 > 0.0) v -= d * b / den2;
    }
    Dv[r] = v;
  }
}

// Table layout for degree d: [(e * (nq + 2) + q) * (d + 1) + r], q = nq -> x = e/N (left end),
// q = nq + 1 -> x = (e+1)/N (right end).  Gauss weights (on [0,1]) in wq[0..nq).
__global__ void k_tables_1d(int d, int N, int nq, double* __restrict__ val, double* __restrict__ der,
                            double* __restrict__ wq) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int npts = nq + 2;
  if (tid >= N * npts) return;
  const int e = tid / npts, q = tid % npts;
  double x01, w;
  if (q < nq) {
    gl_node(nq, q, &x01, &w);
    if (e == 0) wq[q] = w;
  } else {
    x01 = (q == nq) ? 0.0 : 1.0;
  }
  const double x = (e + x01) / N;
  double Nv[5], Dv[5];
  basis_on_element(d, N, e, x, Nv, Dv);
  for (int r = 0; r <= d; ++r) {
    val[(size_t)tid * (d + 1) + r] = Nv[r];
    der[(size_t)tid * (d + 1) + r] = Dv[r];
  }
}

// Gauss points (physical coordinate) of element e: x = (e + xhat_q)/N.
__global__ void k_gauss_points(int nq, double* __restrict__ xq) {
  const int q = threadIdx.x;
  if (q < nq) {
    double x, w;
    gl_node(nq, q, &x, &w);
    xq[q] = x;
  }
}

struct AsmArgs {
  int N, kp, dim, nq;
  int geom;  // 0: identity map; 1: polar map of the 1/8 annulus (2D)
  double nu, cpen;
  int64_t n_u;
  int vcnt[3][3], vshift[3][3], vdeg[3][3];
  int64_t voff[4];
  int nlo;
  // 1D tables for degree k' (lo) and k'+1 (hi)
  const double* tv_lo;
  const double* td_lo;
  const double* tv_hi;
  const double* td_hi;
  const double* wq;
  const double* xq;  // Gauss points on [0,1] of the rule
};

struct Fun {
  int comp;     // velocity component, or -1 for a pressure function
  int i1[3];    // 1D function indices
  int deg[3];   // 1D degrees
  int elo[3], ehi[3];
};

__device__ __forceinline__ void decode_dof(const AsmArgs& a, int64_t g, Fun& f) {
  if (g < a.n_u) {
    int c = 0;
    while (c + 1 < a.dim && g >= a.voff[c + 1]) ++c;
    int64_t r = g - a.voff[c];
    for (int d = 0; d < a.dim; ++d) {
      const int i = int(r % a.vcnt[c][d]) + a.vshift[c][d];
      r /= a.vcnt[c][d];
      f.i1[d] = i;
      f.deg[d] = a.vdeg[c][d];
    }
    f.comp = c;
  } else {
    int64_t r = g - a.n_u;
    for (int d = 0; d < a.dim; ++d) {
      f.i1[d] = int(r % a.nlo);
      r /= a.nlo;
      f.deg[d] = a.kp;
    }
    f.comp = -1;
  }
  for (int d = 0; d < a.dim; ++d) {
    f.elo[d] = max(0, f.i1[d] - f.deg[d]);
    f.ehi[d] = min(a.N - 1, f.i1[d]);
  }
  for (int d = a.dim; d < 3; ++d) {
    f.i1[d] = 0;
    f.deg[d] = 0;
    f.elo[d] = f.ehi[d] = 0;
  }
}

// 1D value and derivative of function f in direction d at table point (e, q).
__device__ __forceinline__ void f1d(const AsmArgs& a, const Fun& f, int d, int e, int q, double* v, double* dv) {
  const int deg = f.deg[d];
  const int r = f.i1[d] - e;
  const size_t idx = ((size_t)e * (a.nq + 2) + q) * (deg + 1) + r;
  if (deg == a.kp) {
    *v = a.tv_lo[idx];
    *dv = a.td_lo[idx];
  } else {
    *v = a.tv_hi[idx];
    *dv = a.td_hi[idx];
  }
}

// Value B and gradient G of the scalar tensor-product spline of f at the point given by
// per-direction (element, table point).
__device__ __forceinline__ void eval_fun(const AsmArgs& a, const Fun& f, const int* e, const int* q, double* B,
                                         double* G) {
  double v[3] = {1, 1, 1}, dv[3] = {0, 0, 0};
  for (int d = 0; d < a.dim; ++d) f1d(a, f, d, e[d], q[d], &v[d], &dv[d]);
  double prod = 1.0;
  for (int d = 0; d < a.dim; ++d) prod *= v[d];
  *B = prod;
  for (int m = 0; m < a.dim; ++m) {
    double p = dv[m];
    for (int d = 0; d < a.dim; ++d)
      if (d != m) p *= v[d];
    G[m] = p;
  }
}

// ---------------------------------------------------------------------------
// Mapped geometry (Sec. 3.2), 2D: the polar map of one eighth of the annulus 1 < r < 2,
// 0 < theta < pi/4 (Sec. 6.3), x = r cos(theta), y = r sin(theta), r = 1 + xi_0,
// theta = (pi/4) xi_1.  Velocities are Piola transforms Phi = DF Phihat / J, pressures
// phihat / J.  Quadrature: k'+3 points per direction for the matrices, k'+5 for loads.
// ---------------------------------------------------------------------------
struct Geo {
  double x[2];
  double DF[2][2], Finv[2][2], J;
  double dDF[2][2][2];  // dDF[k][a][b] = d DF[a][b] / d xi_k
};

__device__ void polar_point(double xi0, double xi1, Geo& g) {
  const double al = 0.25 * kPiD, r = 1.0 + xi0, th = al * xi1;
  const double c = cos(th), s = sin(th);
  g.x[0] = r * c;
  g.x[1] = r * s;
  g.DF[0][0] = c;
  g.DF[0][1] = -al * r * s;
  g.DF[1][0] = s;
  g.DF[1][1] = al * r * c;
  g.J = al * r;
  g.Finv[0][0] = c;
  g.Finv[0][1] = s;
  g.Finv[1][0] = -s / (al * r);
  g.Finv[1][1] = c / (al * r);
  // radial derivatives
  g.dDF[0][0][0] = 0.0;
  g.dDF[0][0][1] = -al * s;
  g.dDF[0][1][0] = 0.0;
  g.dDF[0][1][1] = al * c;
  // angular derivatives (d/dxi_1 = (pi/4) d/dtheta)
  g.dDF[1][0][0] = -al * s;
  g.dDF[1][0][1] = -al * al * r * c;
  g.dDF[1][1][0] = al * c;
  g.dDF[1][1][1] = -al * al * r * s;
}

// Parametric coordinate of table point q of element e (Gauss point, or the element ends).
__device__ __forceinline__ double table_xi(const AsmArgs& a, int e, int q) {
  const double t = q < a.nq ? a.xq[q] : (q == a.nq ? 0.0 : 1.0);
  return (e + t) / a.N;
}

// Physical value and gradient of the Piola transform of Phihat = B e_c (parametric value B,
// parametric gradient G): Phi = B DF[:, c] / J; its parametric derivatives
// d_k Phi_a = G_k DF[a][c] / J + B d_k(DF[a][c] / J) with d_k J = J trace(Finv dDF[k]),
// then grad_x Phi_a = sum_k d_k Phi_a Finv[k][m].
__device__ void piola2(const Geo& g, int c, double B, const double* G, double* val, double grad[2][2]) {
  double dJ[2];
  for (int k = 0; k < 2; ++k) {
    double tr = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) tr += g.Finv[a][b] * g.dDF[k][b][a];
    dJ[k] = g.J * tr;
  }
  double dxi[2][2];
  for (int a = 0; a < 2; ++a) {
    val[a] = B * g.DF[a][c] / g.J;
    for (int k = 0; k < 2; ++k)
      dxi[a][k] = G[k] * g.DF[a][c] / g.J + B * (g.dDF[k][a][c] / g.J - g.DF[a][c] * dJ[k] / (g.J * g.J));
  }
  for (int a = 0; a < 2; ++a)
    for (int m = 0; m < 2; ++m) grad[a][m] = dxi[a][0] * g.Finv[0][m] + dxi[a][1] * g.Finv[1][m];
}

__device__ __forceinline__ void sym2(const double G[2][2], double E[2][2]) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) E[a][b] = 0.5 * (G[a][b] + G[b][a]);
}

__device__ double entry_value_mapped(const AsmArgs& a, int64_t gi, int64_t gj);

// Value of one saddle-matrix entry (row DOF gi, column DOF gj).
__device__ double entry_value(const AsmArgs& a, int64_t gi, int64_t gj) {
  if (a.geom != 0) return entry_value_mapped(a, gi, gj);
  Fun fi, fj;
  decode_dof(a, gi, fi);
  decode_dof(a, gj, fj);
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = max(fi.elo[d], fj.elo[d]);
    hi[d] = min(fi.ehi[d], fj.ehi[d]);
  }
  const double h = 1.0 / a.N;
  double vol = 1.0;
  for (int d = 0; d < a.dim; ++d) vol *= h;
  const int nq = a.nq;
  const int nq2 = a.dim == 3 ? nq : 1;
  double sum = 0.0;
  const bool vel_i = fi.comp >= 0, vel_j = fj.comp >= 0;
  int e[3], q[3];
  // volume terms
  for (e[2] = lo[2]; e[2] <= hi[2]; ++e[2])
    for (e[1] = lo[1]; e[1] <= hi[1]; ++e[1])
      for (e[0] = lo[0]; e[0] <= hi[0]; ++e[0])
        for (q[2] = 0; q[2] < nq2; ++q[2])
          for (q[1] = 0; q[1] < nq; ++q[1])
            for (q[0] = 0; q[0] < nq; ++q[0]) {
              double wt = vol;
              for (int d = 0; d < a.dim; ++d) wt *= a.wq[q[d]];
              double Bi, Gi[3] = {0, 0, 0}, Bj, Gj[3] = {0, 0, 0};
              eval_fun(a, fi, e, q, &Bi, Gi);
              eval_fun(a, fj, e, q, &Bj, Gj);
              if (vel_i && vel_j) {
                const int c = fi.comp, dd = fj.comp;
                double t = Gi[dd] * Gj[c];
                if (c == dd)
                  for (int m = 0; m < a.dim; ++m) t += Gi[m] * Gj[m];
                sum += wt * a.nu * t;
              } else if (vel_i && !vel_j) {  // B^T entry: B_{j,i} = -phi_j d_c B_i
                sum -= wt * Bj * Gi[fi.comp];
              } else if (!vel_i && vel_j) {  // B entry
                sum -= wt * Bi * Gj[fj.comp];
              }
            }
  // Nitsche boundary faces (velocity-velocity only)
  if (vel_i && vel_j) {
    const int c = fi.comp, dd = fj.comp;
    const double pen = 2.0 * a.cpen / h;  // 2 C_pen / h_F, h_F = 1/N
    for (int fd = 0; fd < a.dim; ++fd)
      for (int side = 0; side < 2; ++side) {
        const int eb = side == 0 ? 0 : a.N - 1;
        if (lo[fd] > eb || hi[fd] < eb) continue;
        const double s = side == 0 ? -1.0 : 1.0;
        double farea = 1.0;
        for (int d = 0; d < a.dim; ++d)
          if (d != fd) farea *= h;
        int flo[3], fhi[3], nqd[3];
        for (int d = 0; d < 3; ++d) {
          flo[d] = lo[d];
          fhi[d] = hi[d];
          nqd[d] = (d < a.dim) ? nq : 1;
        }
        flo[fd] = fhi[fd] = eb;
        nqd[fd] = 1;
        for (e[2] = flo[2]; e[2] <= fhi[2]; ++e[2])
          for (e[1] = flo[1]; e[1] <= fhi[1]; ++e[1])
            for (e[0] = flo[0]; e[0] <= fhi[0]; ++e[0])
              for (int q2 = 0; q2 < nqd[2]; ++q2)
                for (int q1 = 0; q1 < nqd[1]; ++q1)
                  for (int q0 = 0; q0 < nqd[0]; ++q0) {
                    q[0] = q0;
                    q[1] = q1;
                    q[2] = q2;
                    q[fd] = side == 0 ? nq : nq + 1;
                    double wt = farea;
                    for (int d = 0; d < a.dim; ++d)
                      if (d != fd) wt *= a.wq[q[d]];
                    double Bi, Gi[3] = {0, 0, 0}, Bj, Gj[3] = {0, 0, 0};
                    eval_fun(a, fi, e, q, &Bi, Gi);
                    eval_fun(a, fj, e, q, &Bj, Gj);
                    const double dn_i = s * Gi[fd], dn_j = s * Gj[fd];
                    const double nc = (c == fd) ? s : 0.0, nd = (dd == fd) ? s : 0.0;
                    double t = -(nc * Gi[dd] * Bj + nd * Gj[c] * Bi);
                    if (c == dd) t += -(dn_i * Bj + dn_j * Bi) + pen * Bi * Bj;
                    sum += wt * a.nu * t;
                  }
      }
  }
  return sum;
}

// The same on the mapped domain (2D): the volume integrands in physical form with dx =
// J dxi; B_kj = -int phi_k div Phi_j dx = -int phihat_k div Phi_j dxi (phi = phihat / J);
// boundary faces with the physical outward normal n = Finv^T nhat / |Finv^T nhat|, surface
// measure J |Finv^T nhat| dshat and h_F = 1 / (N |Finv n|).
__device__ double entry_value_mapped(const AsmArgs& a, int64_t gi, int64_t gj) {
  Fun fi, fj;
  decode_dof(a, gi, fi);
  decode_dof(a, gj, fj);
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = max(fi.elo[d], fj.elo[d]);
    hi[d] = min(fi.ehi[d], fj.ehi[d]);
  }
  const double h = 1.0 / a.N;
  const int nq = a.nq;
  const bool vel_i = fi.comp >= 0, vel_j = fj.comp >= 0;
  double sum = 0.0;
  int e[3] = {0, 0, 0}, q[3] = {0, 0, 0};
  for (e[1] = lo[1]; e[1] <= hi[1]; ++e[1])
    for (e[0] = lo[0]; e[0] <= hi[0]; ++e[0])
      for (q[1] = 0; q[1] < nq; ++q[1])
        for (q[0] = 0; q[0] < nq; ++q[0]) {
          const double wt = h * h * a.wq[q[0]] * a.wq[q[1]];
          Geo g;
          polar_point(table_xi(a, e[0], q[0]), table_xi(a, e[1], q[1]), g);
          double Bi, Gi[3] = {0, 0, 0}, Bj, Gj[3] = {0, 0, 0};
          eval_fun(a, fi, e, q, &Bi, Gi);
          eval_fun(a, fj, e, q, &Bj, Gj);
          double vi[2], vj[2], gri[2][2], grj[2][2];
          if (vel_i) piola2(g, fi.comp, Bi, Gi, vi, gri);
          if (vel_j) piola2(g, fj.comp, Bj, Gj, vj, grj);
          if (vel_i && vel_j) {
            double Ei[2][2], Ej[2][2];
            sym2(gri, Ei);
            sym2(grj, Ej);
            double t = 0.0;
            for (int x = 0; x < 2; ++x)
              for (int y = 0; y < 2; ++y) t += Ei[x][y] * Ej[x][y];
            sum += wt * g.J * 2.0 * a.nu * t;
          } else if (vel_i && !vel_j) {  // B^T entry
            sum -= wt * Bj * (gri[0][0] + gri[1][1]);
          } else if (!vel_i && vel_j) {  // B entry
            sum -= wt * Bi * (grj[0][0] + grj[1][1]);
          }
        }
  if (vel_i && vel_j) {
    for (int fd = 0; fd < 2; ++fd)
      for (int side = 0; side < 2; ++side) {
        const int eb = side == 0 ? 0 : a.N - 1;
        if (lo[fd] > eb || hi[fd] < eb) continue;
        const int t = 1 - fd;
        const double sgn = side == 0 ? -1.0 : 1.0;
        e[fd] = eb;
        q[fd] = side == 0 ? nq : nq + 1;
        for (e[t] = lo[t]; e[t] <= hi[t]; ++e[t])
          for (int qq = 0; qq < nq; ++qq) {
            q[t] = qq;
            Geo g;
            polar_point(table_xi(a, e[0], q[0]), table_xi(a, e[1], q[1]), g);
            // m = Finv^T nhat, nhat = sgn e_fd
            double m[2] = {sgn * g.Finv[fd][0], sgn * g.Finv[fd][1]};
            const double mn = sqrt(m[0] * m[0] + m[1] * m[1]);
            const double n[2] = {m[0] / mn, m[1] / mn};
            const double fn0 = g.Finv[0][0] * n[0] + g.Finv[0][1] * n[1];
            const double fn1 = g.Finv[1][0] * n[0] + g.Finv[1][1] * n[1];
            const double hF = 1.0 / (a.N * sqrt(fn0 * fn0 + fn1 * fn1));
            const double ws = h * a.wq[qq] * g.J * mn;
            double Bi, Gi[3] = {0, 0, 0}, Bj, Gj[3] = {0, 0, 0};
            eval_fun(a, fi, e, q, &Bi, Gi);
            eval_fun(a, fj, e, q, &Bj, Gj);
            double vi[2], vj[2], gri[2][2], grj[2][2], Ei[2][2], Ej[2][2];
            piola2(g, fi.comp, Bi, Gi, vi, gri);
            piola2(g, fj.comp, Bj, Gj, vj, grj);
            sym2(gri, Ei);
            sym2(grj, Ej);
            double ti_vj = 0.0, tj_vi = 0.0;
            for (int x = 0; x < 2; ++x) {
              ti_vj += (Ei[x][0] * n[0] + Ei[x][1] * n[1]) * vj[x];
              tj_vi += (Ej[x][0] * n[0] + Ej[x][1] * n[1]) * vi[x];
            }
            const double vv = vi[0] * vj[0] + vi[1] * vj[1];
            sum += ws * 2.0 * a.nu * (-(ti_vj + tj_vi) + (a.cpen / hF) * vv);
          }
      }
  }
  return sum;
}

// One wavefront per row; lanes over the row's entries.
__global__ void k_assemble_saddle(AsmArgs a, int64_t nrows, const int32_t* __restrict__ rowptr,
                                  const int32_t* __restrict__ col, double* __restrict__ val) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (row >= nrows) return;
  for (int32_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += 64) val[k] = entry_value(a, row, col[k]);
}

// diag(Q)_k = int phi_k^2 and w_k = int phi_k, one thread per pressure function.
__global__ void k_pressure_mass(AsmArgs a, double* __restrict__ diagQ, double* __restrict__ w) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t np = 1;
  for (int d = 0; d < a.dim; ++d) np *= a.nlo;
  if (k >= np) return;
  Fun f;
  decode_dof(a, a.n_u + k, f);
  const double h = 1.0 / a.N;
  double vol = 1.0;
  for (int d = 0; d < a.dim; ++d) vol *= h;
  const int nq2 = a.dim == 3 ? a.nq : 1;
  double s2 = 0.0, s1 = 0.0;
  int e[3], q[3];
  for (e[2] = f.elo[2]; e[2] <= f.ehi[2]; ++e[2])
    for (e[1] = f.elo[1]; e[1] <= f.ehi[1]; ++e[1])
      for (e[0] = f.elo[0]; e[0] <= f.ehi[0]; ++e[0])
        for (q[2] = 0; q[2] < nq2; ++q[2])
          for (q[1] = 0; q[1] < a.nq; ++q[1])
            for (q[0] = 0; q[0] < a.nq; ++q[0]) {
              double wt = vol;
              for (int d = 0; d < a.dim; ++d) wt *= a.wq[q[d]];
              double B, G[3];
              eval_fun(a, f, e, q, &B, G);
              // on the map phi = phihat / J and dx = J dxi: int phi^2 dx = int phihat^2 / J dxi,
              // int phi dx = int phihat dxi
              double ij = 1.0;
              if (a.geom != 0) {
                Geo g;
                polar_point(table_xi(a, e[0], q[0]), table_xi(a, e[1], q[1]), g);
                ij = 1.0 / g.J;
              }
              s2 += wt * B * B * ij;
              s1 += wt * B;
            }
  diagQ[k] = s2;
  w[k] = s1;
}

// Q_kl = int phi_k phi_l over the elements the two supports share; one wavefront per row,
// lanes over the row's entries (the pressure mass matrix, for the pressure-block CG).
__device__ double q_entry(const AsmArgs& a, int64_t k, int64_t l) {
  Fun fk, fl;
  decode_dof(a, a.n_u + k, fk);
  decode_dof(a, a.n_u + l, fl);
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    lo[d] = max(fk.elo[d], fl.elo[d]);
    hi[d] = min(fk.ehi[d], fl.ehi[d]);
    if (lo[d] > hi[d]) return 0.0;
  }
  const double h = 1.0 / a.N;
  double vol = 1.0;
  for (int d = 0; d < a.dim; ++d) vol *= h;
  const int nq2 = a.dim == 3 ? a.nq : 1;
  double s = 0.0;
  int e[3], q[3];
  for (e[2] = lo[2]; e[2] <= hi[2]; ++e[2])
    for (e[1] = lo[1]; e[1] <= hi[1]; ++e[1])
      for (e[0] = lo[0]; e[0] <= hi[0]; ++e[0])
        for (q[2] = 0; q[2] < nq2; ++q[2])
          for (q[1] = 0; q[1] < a.nq; ++q[1])
            for (q[0] = 0; q[0] < a.nq; ++q[0]) {
              double wt = vol;
              for (int d = 0; d < a.dim; ++d) wt *= a.wq[q[d]];
              double Bk, Bl, G[3];
              eval_fun(a, fk, e, q, &Bk, G);
              eval_fun(a, fl, e, q, &Bl, G);
              double ij = 1.0;
              if (a.geom != 0) {
                Geo g;
                polar_point(table_xi(a, e[0], q[0]), table_xi(a, e[1], q[1]), g);
                ij = 1.0 / g.J;
              }
              s += wt * Bk * Bl * ij;
            }
  return s;
}

__global__ void k_assemble_Q(AsmArgs a, int64_t nrows, const int32_t* __restrict__ rowptr,
                             const int32_t* __restrict__ col, double* __restrict__ val) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (row >= nrows) return;
  for (int32_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += 64) val[k] = q_entry(a, row, col[k]);
}

// ---------------------------------------------------------------------------
// Load vector.  Forcing: manufactured (curl of x^2(1-x)^2 y^2(1-y)^2 in 2D, curl of
// (g,g,g) with g = phi(x)phi(y)phi(z) in 3D, pressure prod cos(pi x_d), f = -nu Lap u +
// grad p) plus sinusoid modes.  Quadrature: the (k'+4)-point tables passed in `a`.
// ---------------------------------------------------------------------------
struct ModeArgs {
  int manufactured, nmodes, nrhs;
  const double* amp;    // [nrhs][dim][M]
  const int32_t* wave;  // [nrhs][M][dim]
  const double* phase;  // [nrhs][dim][M]
  const double* xq;     // Gauss points on [0,1] of the load rule
};

__device__ __forceinline__ void phi_derivs(double t, double* F) {
  F[0] = t * t * (1 - t) * (1 - t);
  F[1] = 2 * t - 6 * t * t + 4 * t * t * t;
  F[2] = 2 - 12 * t + 12 * t * t;
  F[3] = -12 + 24 * t;
}

__device__ void manufactured_force(int dim, double nu, const double* x, double* f) {
  if (dim == 2) {
    double X[4], Y[4];
    phi_derivs(x[0], X);
    phi_derivs(x[1], Y);
    // u = (X Y', -X' Y); Lap u = (X'' Y' + X Y''', -(X''' Y + X' Y''))
    const double l0 = X[2] * Y[1] + X[0] * Y[3];
    const double l1 = -(X[3] * Y[0] + X[1] * Y[2]);
    const double s0 = sin(kPiD * x[0]), c0 = cos(kPiD * x[0]);
    const double s1 = sin(kPiD * x[1]), c1 = cos(kPiD * x[1]);
    f[0] = -nu * l0 - kPiD * s0 * c1;
    f[1] = -nu * l1 - kPiD * c0 * s1;
  } else {
    double F[3][4];
    for (int d = 0; d < 3; ++d) phi_derivs(x[d], F[d]);
    // Lap(d g / d x_m) = sum_b d^3 g / (d x_m d x_b^2)
    double L[3];
    for (int m = 0; m < 3; ++m) {
      double s = 0.0;
      for (int b = 0; b < 3; ++b) {
        double prod = 1.0;
        for (int d = 0; d < 3; ++d) prod *= F[d][(d == m ? 1 : 0) + (d == b ? 2 : 0)];
        s += prod;
      }
      L[m] = s;
    }
    const double lap[3] = {L[1] - L[2], L[2] - L[0], L[0] - L[1]};
    double sn[3], cs[3];
    for (int d = 0; d < 3; ++d) {
      sn[d] = sin(kPiD * x[d]);
      cs[d] = cos(kPiD * x[d]);
    }
    const double gp[3] = {-kPiD * sn[0] * cs[1] * cs[2], -kPiD * cs[0] * sn[1] * cs[2], -kPiD * cs[0] * cs[1] * sn[2]};
    for (int m = 0; m < 3; ++m) f[m] = -nu * lap[m] + gp[m];
  }
}

// One thread per (velocity DOF, right-hand side); output f[r * n_u + i].
__global__ void k_load_vector(AsmArgs a, ModeArgs m, double* __restrict__ f) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_u * m.nrhs) return;
  const int64_t i = t % a.n_u;
  const int r = int(t / a.n_u);
  Fun fi;
  decode_dof(a, i, fi);
  const int c = fi.comp;
  const double h = 1.0 / a.N;
  double vol = 1.0;
  for (int d = 0; d < a.dim; ++d) vol *= h;
  const int nq = a.nq, nq2 = a.dim == 3 ? nq : 1;
  const int M = m.nmodes;
  double sum = 0.0;
  int e[3], q[3];
  for (e[2] = fi.elo[2]; e[2] <= fi.ehi[2]; ++e[2])
    for (e[1] = fi.elo[1]; e[1] <= fi.ehi[1]; ++e[1])
      for (e[0] = fi.elo[0]; e[0] <= fi.ehi[0]; ++e[0])
        for (q[2] = 0; q[2] < nq2; ++q[2])
          for (q[1] = 0; q[1] < nq; ++q[1])
            for (q[0] = 0; q[0] < nq; ++q[0]) {
              double wt = vol, x[3] = {0, 0, 0};
              for (int d = 0; d < a.dim; ++d) {
                wt *= a.wq[q[d]];
                x[d] = (e[d] + m.xq[q[d]]) * h;
              }
              double B, G[3];
              eval_fun(a, fi, e, q, &B, G);
              if (a.geom == 0) {
                double fv = 0.0;
                if (m.manufactured) {
                  double fm[3];
                  manufactured_force(a.dim, a.nu, x, fm);
                  fv = fm[c];
                }
                for (int k = 0; k < M; ++k) {
                  double arg = m.phase[((size_t)r * a.dim + c) * M + k];
                  for (int d = 0; d < a.dim; ++d) arg += kPiD * m.wave[((size_t)r * M + k) * a.dim + d] * x[d];
                  fv += m.amp[((size_t)r * a.dim + c) * M + k] * sin(arg);
                }
                sum += wt * fv * B;
              } else {
                // f at the physical point; f . Phi dx = B (DF[:, c] . f) dxi
                Geo g;
                polar_point(x[0], x[1], g);
                double fv[2] = {0.0, 0.0};
                if (m.manufactured) {
                  double fm[3];
                  manufactured_force(2, a.nu, g.x, fm);
                  fv[0] = fm[0];
                  fv[1] = fm[1];
                }
                for (int d = 0; d < 2; ++d)
                  for (int k = 0; k < M; ++k) {
                    double arg = m.phase[((size_t)r * 2 + d) * M + k];
                    for (int b = 0; b < 2; ++b) arg += kPiD * m.wave[((size_t)r * M + k) * 2 + b] * g.x[b];
                    fv[d] += m.amp[((size_t)r * 2 + d) * M + k] * sin(arg);
                  }
                sum += wt * B * (g.DF[0][c] * fv[0] + g.DF[1][c] * fv[1]);
              }
            }
  f[(size_t)r * a.n_u + i] = sum;
}

// Tangential boundary data of the 2D cavity-type problems: volume force f and boundary
// velocity g at x (on the side with normal direction fd, side 0: coordinate 0, 1:
// coordinate 1).  kind 0: lid-driven cavity (Sec. 6.4), f = 0, g = (1, 0) on y = 1.
// kind 1: u = curl(x(1-x)y(1-y)) = (x(1-x)(1-2y), -(1-2x)y(1-y)), p = 0, f = -nu Lap u,
// g = u, a flow that lies in the discrete velocity space for every k' >= 1.
__device__ void cavity_fg(int kind, double nu, const double* x, int fd, int side, double* f, double* g) {
  f[0] = f[1] = 0.0;
  g[0] = g[1] = 0.0;
  if (kind == 0) {
    if (fd == 1 && side == 1) g[0] = 1.0;
    return;
  }
  f[0] = 2.0 * nu * (1.0 - 2.0 * x[1]);
  f[1] = -2.0 * nu * (1.0 - 2.0 * x[0]);
  g[0] = x[0] * (1.0 - x[0]) * (1.0 - 2.0 * x[1]);
  g[1] = -(1.0 - 2.0 * x[0]) * x[1] * (1.0 - x[1]);
}

// f_i = (f, Phi_i) + l_h(Phi_i) with the Nitsche form of eq. nitsche_rhs,
//   l_h(v) = sum_F int_F 2 nu ( -((sym grad v) n) . g + (C_pen/h_F) g . v ) dS,
// for Phi_i = B e_c: ((sym grad Phi_i) n) . g = (g_c dB/dn + (n.g) dB/dx_c) / 2.
// One thread per velocity function (2D), quadrature over the elements and boundary sides
// of its support (k'+2 points per direction, table points nq / nq+1 at the element ends).
__global__ void k_load_cavity(AsmArgs a, int kind, const double* __restrict__ xq, double* __restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_u) return;
  Fun fi;
  decode_dof(a, i, fi);
  const int c = fi.comp;
  const double h = 1.0 / a.N;
  const int nq = a.nq;
  double sum = 0.0;
  int e[3] = {0, 0, 0}, q[3] = {0, 0, 0};
  if (kind == 1) {
    for (e[1] = fi.elo[1]; e[1] <= fi.ehi[1]; ++e[1])
      for (e[0] = fi.elo[0]; e[0] <= fi.ehi[0]; ++e[0])
        for (q[1] = 0; q[1] < nq; ++q[1])
          for (q[0] = 0; q[0] < nq; ++q[0]) {
            const double x[2] = {(e[0] + xq[q[0]]) * h, (e[1] + xq[q[1]]) * h};
            double fv[2], gv[2], B, G[3] = {0, 0, 0};
            cavity_fg(kind, a.nu, x, -1, -1, fv, gv);
            eval_fun(a, fi, e, q, &B, G);
            sum += h * h * a.wq[q[0]] * a.wq[q[1]] * fv[c] * B;
          }
  }
  const double pen = a.cpen / h;
  for (int fd = 0; fd < 2; ++fd)
    for (int side = 0; side < 2; ++side) {
      const int eb = side == 0 ? 0 : a.N - 1;
      if (fi.elo[fd] > eb || fi.ehi[fd] < eb) continue;
      const double sgn = side == 0 ? -1.0 : 1.0;
      const int t = 1 - fd;
      e[fd] = eb;
      q[fd] = side == 0 ? nq : nq + 1;
      for (e[t] = fi.elo[t]; e[t] <= fi.ehi[t]; ++e[t])
        for (int qq = 0; qq < nq; ++qq) {
          q[t] = qq;
          double x[2];
          x[t] = (e[t] + xq[qq]) * h;
          x[fd] = side == 0 ? 0.0 : 1.0;
          double fv[2], gv[2], B, G[3] = {0, 0, 0};
          cavity_fg(kind, a.nu, x, fd, side, fv, gv);
          eval_fun(a, fi, e, q, &B, G);
          const double epsn_g = 0.5 * (gv[c] * sgn * G[fd] + sgn * gv[fd] * G[c]);
          sum += h * a.wq[qq] * 2.0 * a.nu * (-epsn_g + pen * gv[c] * B);
        }
    }
  f[i] = sum;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
struct Tables {
  double *v_lo = nullptr, *d_lo = nullptr, *v_hi = nullptr, *d_hi = nullptr, *wq = nullptr, *xq = nullptr;
};

static AsmArgs make_args(const Spaces& S, double nu, double cpen, int nq, const Tables& T) {
  AsmArgs a;
  a.geom = S.geom;
  a.N = S.N;
  a.kp = S.kp;
  a.dim = S.dim;
  a.nq = nq;
  a.nu = nu;
  a.cpen = cpen;
  a.n_u = S.n_u;
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) {
      a.vcnt[c][d] = S.vcnt[c][d];
      a.vshift[c][d] = S.vshift[c][d];
      a.vdeg[c][d] = S.vdeg[c][d];
    }
  for (int c = 0; c < 4; ++c) a.voff[c] = S.voff[c];
  a.nlo = S.nlo;
  a.tv_lo = T.v_lo;
  a.td_lo = T.d_lo;
  a.tv_hi = T.v_hi;
  a.td_hi = T.d_hi;
  a.wq = T.wq;
  a.xq = T.xq;
  return a;
}

// Gauss points per direction: k'+2 (matrices) and k'+4 (loads) are exact on the identity
// map; the mapped integrands are rational, one more point is taken there.
static int matrix_points(const Spaces& S) { return S.kp + 2 + (S.geom ? 1 : 0); }
static int load_points(const Spaces& S) { return S.kp + 4 + (S.geom ? 1 : 0); }

static hipError_t build_tables(const Spaces& S, int nq, Tables& T, hipStream_t st) {
  const size_t npt = (size_t)S.N * (nq + 2);
  hipError_t e;
  if ((e = hipMalloc(&T.v_lo, npt * (S.kp + 1) * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc(&T.d_lo, npt * (S.kp + 1) * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc(&T.v_hi, npt * (S.kp + 2) * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc(&T.d_hi, npt * (S.kp + 2) * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc(&T.wq, 16 * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc(&T.xq, 16 * sizeof(double))) != hipSuccess) return e;
  const int nb = int((npt + 255) / 256);
  hipLaunchKernelGGL(k_tables_1d, dim3(nb), dim3(256), 0, st, S.kp, S.N, nq, T.v_lo, T.d_lo, T.wq);
  hipLaunchKernelGGL(k_tables_1d, dim3(nb), dim3(256), 0, st, S.kp + 1, S.N, nq, T.v_hi, T.d_hi, T.wq);
  hipLaunchKernelGGL(k_gauss_points, dim3(1), dim3(64), 0, st, nq, T.xq);
  return hipGetLastError();
}

static void free_tables(Tables& T) {
  hipFree(T.v_lo);
  hipFree(T.d_lo);
  hipFree(T.v_hi);
  hipFree(T.d_hi);
  hipFree(T.wq);
  hipFree(T.xq);
  T = Tables();
}

hipError_t assemble_saddle(const Spaces& S, double nu, double cpen, const int32_t* rowptr, const int32_t* col,
                           double* val, double* diagQ, double* w, hipStream_t st) {
  Tables T;
  const int nq = matrix_points(S);
  hipError_t e = build_tables(S, nq, T, st);
  if (e != hipSuccess) {
    free_tables(T);
    return e;
  }
  AsmArgs a = make_args(S, nu, cpen, nq, T);
  const int64_t n = S.n_u + S.n_p;
  const int rows_per_block = 4;
  hipLaunchKernelGGL(k_assemble_saddle, dim3(unsigned((n + rows_per_block - 1) / rows_per_block)), dim3(256), 0, st,
                     a, n, rowptr, col, val);
  hipLaunchKernelGGL(k_pressure_mass, dim3(unsigned((S.n_p + 255) / 256)), dim3(256), 0, st, a, diagQ, w);
  e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(st);
  free_tables(T);
  return e != hipSuccess ? e : e2;
}

hipError_t assemble_Q(const Spaces& S, const int32_t* rowptr, const int32_t* col, double* val, hipStream_t st) {
  Tables T;
  const int nq = matrix_points(S);
  hipError_t e = build_tables(S, nq, T, st);
  if (e != hipSuccess) {
    free_tables(T);
    return e;
  }
  AsmArgs a = make_args(S, 1.0, 0.0, nq, T);
  const int rows_per_block = 4;
  hipLaunchKernelGGL(k_assemble_Q, dim3(unsigned((S.n_p + rows_per_block - 1) / rows_per_block)), dim3(256), 0, st, a,
                     S.n_p, rowptr, col, val);
  e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(st);
  free_tables(T);
  return e != hipSuccess ? e : e2;
}

hipError_t assemble_load(const Spaces& S, double nu, int manufactured, int nmodes, int nrhs, const double* amp_d,
                         const int32_t* wave_d, const double* phase_d, double* f, hipStream_t st) {
  Tables T;
  const int nq = load_points(S);
  hipError_t e = build_tables(S, nq, T, st);
  if (e != hipSuccess) {
    free_tables(T);
    return e;
  }
  AsmArgs a = make_args(S, nu, 0.0, nq, T);
  ModeArgs m;
  m.manufactured = manufactured;
  m.nmodes = nmodes;
  m.nrhs = nrhs;
  m.amp = amp_d;
  m.wave = wave_d;
  m.phase = phase_d;
  m.xq = T.xq;
  const int64_t nt = S.n_u * nrhs;
  hipLaunchKernelGGL(k_load_vector, dim3(unsigned((nt + 127) / 128)), dim3(128), 0, st, a, m, f);
  e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(st);
  free_tables(T);
  return e != hipSuccess ? e : e2;
}

hipError_t assemble_load_cavity(const Spaces& S, double nu, double cpen, int kind, double* f, hipStream_t st) {
  if (S.geom != 0) return hipErrorInvalidValue;  // the cavity is the unit square
  Tables T;
  const int nq = S.kp + 2;
  hipError_t e = build_tables(S, nq, T, st);
  if (e != hipSuccess) {
    free_tables(T);
    return e;
  }
  AsmArgs a = make_args(S, nu, cpen, nq, T);
  hipLaunchKernelGGL(k_load_cavity, dim3(unsigned((S.n_u + 127) / 128)), dim3(128), 0, st, a, kind, T.xq, f);
  e = hipGetLastError();
  hipError_t e2 = hipStreamSynchronize(st);
  free_tables(T);
  return e != hipSuccess ? e : e2;
}

}  // namespace stk
