// Element kernels: stiffness of space-frame members and flat shells, and the element terms of
// the adjoint sensitivity.
//
// Sec. 2.2.1 of the paper defines the two element families by their inputs: the beam-column
// takes (E, G, Iy, Iz, J, A) and two end nodes; the quad shell (MITC-4, Dvorkin & Bathe) takes
// the 12 corner coordinates, t, E, nu and two stiffness-modification coefficients.  The
// formulation implemented here:
//  * member: Euler-Bernoulli space frame; e1 along the member, e2 = normalise(Z x e1) (Y for
//    vertical members), e3 = e1 x e2; K = T^T k T, T = diag(R, R, R, R).
//  * shell: flat facet on the mean plane of the corners (normal from the diagonals, e1 along
//    the xi mid-line); bilinear membrane; Reissner-Mindlin bending with beta = (theta_y,
//    -theta_x); MITC4 transverse shear tied at the edge mid-points; drilling penalty
//    1e-3 G t (theta_z - (v,x - u,y)/2)^2; corners offset rigidly to the mean plane;
//    2x2 Gauss quadrature; K = s (B W T)^T D (B W T) summed over Gauss points.
//
// Kernel layout.  Shell stiffness: one wavefront per element.  The 4 x 9 x 24 strain-
// displacement matrix G = B W T (global DOFs) and H = D G det J are staged in LDS, then each of
// the 64 lanes forms one 3 x 3 tile of K = sum G^T H.  Members: 12 threads per member, one row
// each.  Adjoint terms: one thread per (element, parameter); the element bilinear form
// lambda^T K(p) u is evaluated with forward-mode dual numbers seeded on that parameter, so
// every derivative is exact (no finite differences).
#include "sso_internal.h"

namespace sso {
namespace {

constexpr double ALPHA_DRILL = 1.0e-3;
constexpr double KAPPA_SHEAR = 5.0 / 6.0;
constexpr double VERTICAL_TOL = 1.0e-6;

// ---- forward-mode dual number -------------------------------------------------------------

struct Dual {
  double v, d;
  __device__ Dual() : v(0), d(0) {}
  __device__ Dual(double a) : v(a), d(0) {}
  __device__ Dual(double a, double b) : v(a), d(b) {}
};
__device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__device__ inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__device__ inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
__device__ inline Dual operator/(double a, Dual b) { return Dual(a) / b; }
__device__ inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
__device__ inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__device__ inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
__device__ inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
__device__ inline Dual sqrt_(Dual a) {
  double s = sqrt(a.v);
  return Dual(s, 0.5 * a.d / s);
}
__device__ inline double sqrt_(double a) { return sqrt(a); }
__device__ inline double val(double a) { return a; }
__device__ inline double val(Dual a) { return a.v; }

// ---- shell geometry -----------------------------------------------------------------------

template <class S>
struct QGeom {
  S R[3][3];      // rows e1, e2, e3
  S x[4], y[4], h[4];
  S area;
};

template <class S>
__device__ inline void cross3(const S a[3], const S b[3], S c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

template <class S>
__device__ inline S dot3(const S a[3], const S b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Mean-plane frame, local corner coordinates and offsets.  Returns false when degenerate.
template <class S>
__device__ bool quad_geom(const S X[4][3], QGeom<S>& g) {
  S c[3], d13[3], d24[3], nrm[3], a[3];
  for (int k = 0; k < 3; ++k) {
    c[k] = 0.25 * (X[0][k] + X[1][k] + X[2][k] + X[3][k]);
    d13[k] = X[2][k] - X[0][k];
    d24[k] = X[3][k] - X[1][k];
    a[k] = 0.5 * (X[1][k] + X[2][k] - X[0][k] - X[3][k]);
  }
  cross3(d13, d24, nrm);
  S nn = sqrt_(dot3(nrm, nrm));
  if (!(val(nn) > 0.0)) return false;
  S e1[3], e2[3], e3[3];
  for (int k = 0; k < 3; ++k) e3[k] = nrm[k] / nn;
  S ae = dot3(a, e3);
  S ap[3];
  for (int k = 0; k < 3; ++k) ap[k] = a[k] - ae * e3[k];
  S na = sqrt_(dot3(ap, ap));
  if (!(val(na) > 0.0)) return false;
  for (int k = 0; k < 3; ++k) e1[k] = ap[k] / na;
  cross3(e3, e1, e2);
  for (int k = 0; k < 3; ++k) {
    g.R[0][k] = e1[k];
    g.R[1][k] = e2[k];
    g.R[2][k] = e3[k];
  }
  for (int i = 0; i < 4; ++i) {
    S rel[3];
    for (int k = 0; k < 3; ++k) rel[k] = X[i][k] - c[k];
    g.x[i] = dot3(rel, e1);
    g.y[i] = dot3(rel, e2);
    g.h[i] = dot3(rel, e3);
  }
  g.area = 0.5 * nn;
  return true;
}

// Gauss-point data: shape functions, Cartesian derivatives, det J, J^{-1}, and the MITC4
// coefficients of the covariant shear strains gamma_xi, gamma_eta on (w, beta_x, beta_y) of
// each corner (tying points A (0,1), C (0,-1) for gamma_xi; B (-1,0), D (1,0) for gamma_eta).
template <class S>
struct QGP {
  S N[4], Nx[4], Ny[4];
  S det, Ji[2][2];
  S cw_xi[4], cbx_xi[4], cby_xi[4];
  S cw_eta[4], cbx_eta[4], cby_eta[4];
};

__device__ inline double gauss_xi(int gp) {
  const double g = 0.57735026918962576451;   // 1 / sqrt(3)
  return (gp == 0 || gp == 3) ? -g : g;
}
__device__ inline double gauss_eta(int gp) {
  const double g = 0.57735026918962576451;
  return (gp < 2) ? -g : g;
}

template <class S>
__device__ void quad_gp(const QGeom<S>& g, int gp, QGP<S>& q) {
  const double xi = gauss_xi(gp), eta = gauss_eta(gp);
  const double XI[4] = {-1.0, 1.0, 1.0, -1.0};
  const double ET[4] = {-1.0, -1.0, 1.0, 1.0};
  double dxi[4], deta[4];
  S J11 = 0.0, J12 = 0.0, J21 = 0.0, J22 = 0.0;
  for (int i = 0; i < 4; ++i) {
    q.N[i] = 0.25 * (1.0 + xi * XI[i]) * (1.0 + eta * ET[i]);
    dxi[i] = 0.25 * XI[i] * (1.0 + eta * ET[i]);
    deta[i] = 0.25 * ET[i] * (1.0 + xi * XI[i]);
    J11 += dxi[i] * g.x[i];
    J12 += dxi[i] * g.y[i];
    J21 += deta[i] * g.x[i];
    J22 += deta[i] * g.y[i];
  }
  q.det = J11 * J22 - J12 * J21;
  q.Ji[0][0] = J22 / q.det;
  q.Ji[0][1] = -J12 / q.det;
  q.Ji[1][0] = -J21 / q.det;
  q.Ji[1][1] = J11 / q.det;
  for (int i = 0; i < 4; ++i) {
    q.Nx[i] = q.Ji[0][0] * dxi[i] + q.Ji[0][1] * deta[i];
    q.Ny[i] = q.Ji[1][0] * dxi[i] + q.Ji[1][1] * deta[i];
  }
  // edge mid-point tangents: C on edge 0-1, A on edge 3-2 (d/dxi); B on edge 0-3, D on 1-2
  S xC = 0.5 * (g.x[1] - g.x[0]), yC = 0.5 * (g.y[1] - g.y[0]);
  S xA = 0.5 * (g.x[2] - g.x[3]), yA = 0.5 * (g.y[2] - g.y[3]);
  S xB = 0.5 * (g.x[3] - g.x[0]), yB = 0.5 * (g.y[3] - g.y[0]);
  S xD = 0.5 * (g.x[2] - g.x[1]), yD = 0.5 * (g.y[2] - g.y[1]);
  const double wA = 0.5 * (1.0 + eta), wC = 0.5 * (1.0 - eta);
  const double wB = 0.5 * (1.0 - xi), wD = 0.5 * (1.0 + xi);
  // gamma_xi: corners 0, 1 through C; corners 3, 2 through A
  q.cw_xi[0] = -0.5 * wC;  q.cbx_xi[0] = (0.5 * wC) * xC;  q.cby_xi[0] = (0.5 * wC) * yC;
  q.cw_xi[1] = 0.5 * wC;   q.cbx_xi[1] = (0.5 * wC) * xC;  q.cby_xi[1] = (0.5 * wC) * yC;
  q.cw_xi[2] = 0.5 * wA;   q.cbx_xi[2] = (0.5 * wA) * xA;  q.cby_xi[2] = (0.5 * wA) * yA;
  q.cw_xi[3] = -0.5 * wA;  q.cbx_xi[3] = (0.5 * wA) * xA;  q.cby_xi[3] = (0.5 * wA) * yA;
  // gamma_eta: corners 0, 3 through B; corners 1, 2 through D
  q.cw_eta[0] = -0.5 * wB; q.cbx_eta[0] = (0.5 * wB) * xB; q.cby_eta[0] = (0.5 * wB) * yB;
  q.cw_eta[3] = 0.5 * wB;  q.cbx_eta[3] = (0.5 * wB) * xB; q.cby_eta[3] = (0.5 * wB) * yB;
  q.cw_eta[1] = -0.5 * wD; q.cbx_eta[1] = (0.5 * wD) * xD; q.cby_eta[1] = (0.5 * wD) * yD;
  q.cw_eta[2] = 0.5 * wD;  q.cbx_eta[2] = (0.5 * wD) * xD; q.cby_eta[2] = (0.5 * wD) * yD;
}

// Local warped DOFs of corner i from its global displacement (ug) and rotation (rg):
// translations and rotations rotated into the frame, then u -= h theta_y, v += h theta_x.
template <class S, class T>
__device__ inline void to_local_warped(const QGeom<S>& g, int i, const T ug[3], const T rg[3],
                                       T d[6]) {
  T t[3], r[3];
  for (int k = 0; k < 3; ++k) {
    t[k] = g.R[k][0] * ug[0] + g.R[k][1] * ug[1] + g.R[k][2] * ug[2];
    r[k] = g.R[k][0] * rg[0] + g.R[k][1] * rg[1] + g.R[k][2] * rg[2];
  }
  d[0] = t[0] - g.h[i] * r[1];
  d[1] = t[1] + g.h[i] * r[0];
  d[2] = t[2];
  d[3] = r[0];
  d[4] = r[1];
  d[5] = r[2];
}

// Accumulate the 9 generalised strains (membrane 3, curvature 3, covariant shear 2 kept in
// gxi/geta, drilling 1) of corner i's local warped DOFs d at a Gauss point.
template <class S, class T>
__device__ inline void add_strains(const QGP<S>& q, int i, const T d[6], T eps[9], T& gxi,
                                   T& geta) {
  const T u = d[0], v = d[1], w = d[2], tx = d[3], ty = d[4], tz = d[5];
  eps[0] += q.Nx[i] * u;
  eps[1] += q.Ny[i] * v;
  eps[2] += q.Ny[i] * u + q.Nx[i] * v;
  eps[3] += q.Nx[i] * ty;                    // beta_x,x with beta_x = theta_y
  eps[4] += -(q.Ny[i] * tx);                 // beta_y,y with beta_y = -theta_x
  eps[5] += q.Ny[i] * ty - q.Nx[i] * tx;     // beta_x,y + beta_y,x
  gxi += q.cw_xi[i] * w + q.cbx_xi[i] * ty - q.cby_xi[i] * tx;
  geta += q.cw_eta[i] * w + q.cbx_eta[i] * ty - q.cby_eta[i] * tx;
  eps[8] += q.N[i] * tz - 0.5 * (q.Nx[i] * v) + 0.5 * (q.Ny[i] * u);
}

template <class S, class T>
__device__ inline void finish_shear(const QGP<S>& q, T gxi, T geta, T eps[9]) {
  eps[6] = q.Ji[0][0] * gxi + q.Ji[0][1] * geta;
  eps[7] = q.Ji[1][0] * gxi + q.Ji[1][1] * geta;
}

// Material moduli (per unit det J and scale): membrane Dm, bending Db (same pattern), shear
// kappa G t, drilling alpha G t.
template <class S>
struct QMat {
  S dm, db, ds, dd;
  double nu;
};

template <class S>
__device__ inline QMat<S> quad_mat(S t, double E, double nu) {
  QMat<S> m;
  double G = E / (2.0 * (1.0 + nu));
  m.dm = (E / (1.0 - nu * nu)) * t;
  m.db = (E / (12.0 * (1.0 - nu * nu))) * (t * t * t);
  m.ds = (KAPPA_SHEAR * G) * t;
  m.dd = (ALPHA_DRILL * G) * t;
  m.nu = nu;
  return m;
}

// H = D eps (generalised stresses per unit area).
template <class S, class T>
__device__ inline void apply_D(const QMat<S>& m, const T eps[9], T sig[9]) {
  const double nu = m.nu, hn = 0.5 * (1.0 - nu);
  sig[0] = m.dm * (eps[0] + nu * eps[1]);
  sig[1] = m.dm * (nu * eps[0] + eps[1]);
  sig[2] = m.dm * (hn * eps[2]);
  sig[3] = m.db * (eps[3] + nu * eps[4]);
  sig[4] = m.db * (nu * eps[3] + eps[4]);
  sig[5] = m.db * (hn * eps[5]);
  sig[6] = m.ds * eps[6];
  sig[7] = m.ds * eps[7];
  sig[8] = m.dd * eps[8];
}

__device__ inline bool quad_prop_ok(const double* pr, double scale) {
  const double t = pr[0], E = pr[1], nu = pr[2];
  return t > 0.0 && E > 0.0 && nu > -1.0 && nu < 0.5 && pr[3] == 1.0 && pr[4] == 1.0 &&
         scale >= 0.0 && isfinite(t) && isfinite(E) && isfinite(scale);
}

// ---- shell stiffness: one wavefront per element --------------------------------------------

constexpr int QW = 4;   // elements (wavefronts) per workgroup

__global__ void __launch_bounds__(64 * QW) k_quad_stiffness(Mesh m, double* coo, double* qarea,
                                                            unsigned* err) {
  __shared__ double Gs[QW][36][24];
  __shared__ double Hs[QW][36][24];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * QW + w;
  const bool active = e < m.n_quads;
  bool ok = true;
  if (active) {
    double X[4][3];
    for (int i = 0; i < 4; ++i) {
      int nd = m.quad_nodes[4 * e + i];
      for (int k = 0; k < 3; ++k) X[i][k] = m.xyz[3 * (int64_t)nd + k];
    }
    const double* pr = m.quad_prop + 5 * e;
    const double sc = m.quad_scale[e];
    QGeom<double> g;
    ok = quad_prop_ok(pr, sc) && quad_geom(X, g);
    if (ok) {
      QMat<double> mt = quad_mat<double>(pr[0], pr[1], pr[2]);
      for (int pass = 0; pass < 2; ++pass) {
        int pair = lane + 64 * pass;       // (gauss point, global column) pairs: 4 x 24
        if (pair < 96) {
          int gp = pair / 24, col = pair % 24;
          int i = col / 6, c = col % 6;
          QGP<double> q;
          quad_gp(g, gp, q);
          if (!(q.det > 0.0)) ok = false;
          double ug[3] = {0.0, 0.0, 0.0}, rg[3] = {0.0, 0.0, 0.0};
          if (c < 3) ug[c] = 1.0; else rg[c - 3] = 1.0;
          double d[6];
          to_local_warped(g, i, ug, rg, d);
          double eps[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gxi = 0.0, geta = 0.0;
          add_strains(q, i, d, eps, gxi, geta);
          finish_shear(q, gxi, geta, eps);
          double sig[9];
          apply_D(mt, eps, sig);
          double wgt = q.det * sc;
          for (int s = 0; s < 9; ++s) {
            Gs[w][gp * 9 + s][col] = eps[s];
            Hs[w][gp * 9 + s][col] = sig[s] * wgt;
          }
        }
      }
      if (lane == 0) qarea[e] = g.area;
    }
  }
  // a failed Jacobian on any lane marks the element
  ok = __all(ok) != 0;
  if (active && !ok && lane == 0) atomicOr(err, ERR_QUAD);
  __syncthreads();
  if (!active) return;
  const int a0 = 3 * (lane >> 3), b0 = 3 * (lane & 7);
  double acc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int r = 0; r < 36; ++r) {
    double ga[3], hb[3];
    for (int k = 0; k < 3; ++k) {
      ga[k] = Gs[w][r][a0 + k];
      hb[k] = Hs[w][r][b0 + k];
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) acc[i][j] += ga[i] * hb[j];
  }
  double* out = coo + 144 * (int64_t)m.n_beams + 576 * e;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out[24 * (a0 + i) + b0 + j] = acc[i][j];
}

// ---- members -------------------------------------------------------------------------------

template <class S>
struct BGeom {
  S L;
  S R[3][3];
};

template <class S>
__device__ bool beam_geom(const S Xi[3], const S Xj[3], BGeom<S>& g) {
  S d[3];
  for (int k = 0; k < 3; ++k) d[k] = Xj[k] - Xi[k];
  g.L = sqrt_(dot3(d, d));
  if (!(val(g.L) > 0.0)) return false;
  S e1[3], e2[3], e3[3];
  for (int k = 0; k < 3; ++k) e1[k] = d[k] / g.L;
  // Z x e1 = (-e1y, e1x, 0)
  S w[3] = {-e1[1], e1[0], S(0.0)};
  S nw = sqrt_(dot3(w, w));
  if (val(nw) < VERTICAL_TOL) {
    e2[0] = 0.0; e2[1] = 1.0; e2[2] = 0.0;
  } else {
    for (int k = 0; k < 3; ++k) e2[k] = w[k] / nw;
  }
  cross3(e1, e2, e3);
  for (int k = 0; k < 3; ++k) {
    g.R[0][k] = e1[k];
    g.R[1][k] = e2[k];
    g.R[2][k] = e3[k];
  }
  return true;
}

// out = k in, k the local Euler-Bernoulli space-frame matrix (DOFs u v w tx ty tz at i, j).
template <class S, class T>
__device__ inline void beam_apply_k(const double* pr, S L, const T in[12], T out[12]) {
  const double E = pr[0], G = pr[1], A = pr[2], Iy = pr[3], Iz = pr[4], J = pr[5];
  S L2 = L * L, L3 = L2 * L;
  S ea = (E * A) / L, gj = (G * J) / L;
  out[0] = ea * (in[0] - in[6]);
  out[6] = -out[0];
  out[3] = gj * (in[3] - in[9]);
  out[9] = -out[3];
  S z12 = (12.0 * E * Iz) / L3, z6 = (6.0 * E * Iz) / L2, z4 = (4.0 * E * Iz) / L,
    z2 = (2.0 * E * Iz) / L;
  T dv = in[1] - in[7], sz = in[5] + in[11];
  out[1] = z12 * dv + z6 * sz;
  out[7] = -out[1];
  out[5] = z6 * dv + z4 * in[5] + z2 * in[11];
  out[11] = z6 * dv + z2 * in[5] + z4 * in[11];
  S y12 = (12.0 * E * Iy) / L3, y6 = (6.0 * E * Iy) / L2, y4 = (4.0 * E * Iy) / L,
    y2 = (2.0 * E * Iy) / L;
  T dw = in[2] - in[8], sy = in[4] + in[10];
  out[2] = y12 * dw - y6 * sy;
  out[8] = -out[2];
  out[4] = -(y6 * dw) + y4 * in[4] + y2 * in[10];
  out[10] = -(y6 * dw) + y2 * in[4] + y4 * in[10];
}

__device__ inline bool beam_prop_ok(const double* pr) {
  for (int k = 0; k < 6; ++k)
    if (!(pr[k] > 0.0) || !isfinite(pr[k])) return false;
  return true;
}

// 12 threads per member: thread a forms column a of T^T k T (= row a by symmetry).
__global__ void k_beam_stiffness(Mesh m, double* coo, unsigned* err) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 12 * (int64_t)m.n_beams) return;
  int64_t e = t / 12;
  int a = (int)(t % 12);
  double Xi[3], Xj[3];
  int ni = m.beam_nodes[2 * e], nj = m.beam_nodes[2 * e + 1];
  for (int k = 0; k < 3; ++k) {
    Xi[k] = m.xyz[3 * (int64_t)ni + k];
    Xj[k] = m.xyz[3 * (int64_t)nj + k];
  }
  const double* pr = m.beam_prop + 6 * e;
  BGeom<double> g;
  if (!beam_prop_ok(pr) || !beam_geom(Xi, Xj, g)) {
    if (a == 0) atomicOr(err, ERR_BEAM);
    return;
  }
  double loc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, kl[12];
  const int blk = a / 3, comp = a % 3;
  for (int k = 0; k < 3; ++k) loc[3 * blk + k] = g.R[k][comp];   // T e_a
  beam_apply_k(pr, g.L, loc, kl);
  double* out = coo + 144 * e + 12 * a;
  for (int B = 0; B < 4; ++B)
    for (int j = 0; j < 3; ++j)
      out[3 * B + j] = g.R[0][j] * kl[3 * B] + g.R[1][j] * kl[3 * B + 1] + g.R[2][j] * kl[3 * B + 2];
}

// ---- adjoint element terms ------------------------------------------------------------------

// Members: thread (e, d), d in 0..5 = (node a = d / 3, coordinate d % 3).
// gbeam[6 e + d] = -c_lam d/dX (lambda_e^T K_e(X) u_e).
__global__ void __launch_bounds__(128) k_beam_adjoint(Mesh m, const double* u, const double* lam, double c_lam,
                               double* gbeam) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 6 * (int64_t)m.n_beams) return;
  int64_t e = t / 6;
  int d = (int)(t % 6);
  int nd[2] = {m.beam_nodes[2 * e], m.beam_nodes[2 * e + 1]};
  Dual X[2][3];
  for (int a = 0; a < 2; ++a)
    for (int k = 0; k < 3; ++k)
      X[a][k] = Dual(m.xyz[3 * (int64_t)nd[a] + k], (3 * a + k == d) ? 1.0 : 0.0);
  BGeom<Dual> g;
  beam_geom(X[0], X[1], g);
  Dual ul[12], ll[12];
  for (int a = 0; a < 2; ++a)
    for (int blk = 0; blk < 2; ++blk) {
      const double* us = u + 6 * (int64_t)nd[a] + 3 * blk;
      const double* ls = lam + 6 * (int64_t)nd[a] + 3 * blk;
      for (int k = 0; k < 3; ++k) {
        ul[6 * a + 3 * blk + k] = g.R[k][0] * us[0] + g.R[k][1] * us[1] + g.R[k][2] * us[2];
        ll[6 * a + 3 * blk + k] = g.R[k][0] * ls[0] + g.R[k][1] * ls[1] + g.R[k][2] * ls[2];
      }
    }
  Dual ku[12];
  beam_apply_k(m.beam_prop + 6 * e, g.L, ul, ku);
  Dual phi = 0.0;
  for (int k = 0; k < 12; ++k) phi += ll[k] * ku[k];
  gbeam[t] = -c_lam * phi.d;
}

// Quads: thread (e, d), d in 0..13 = 12 corner coordinates, thickness, stiffness scale.
// gquad[14 e + d] = c_lam (lam^T df/dp - lam^T dK/dp u) + c_u u^T df/dp, the last with u taken
// as 0 on constrained DOFs (the objectives weigh the load on the free DOFs; u there is the
// prescribed displacement, not a response to the load).
__global__ void __launch_bounds__(128) k_quad_adjoint(Mesh m, const double* u, const double* lam, double c_lam,
                               double c_u, double* gquad) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 14 * (int64_t)m.n_quads) return;
  int64_t e = t / 14;
  int d = (int)(t % 14);
  int nd[4];
  Dual X[4][3];
  for (int i = 0; i < 4; ++i) {
    nd[i] = m.quad_nodes[4 * e + i];
    for (int k = 0; k < 3; ++k)
      X[i][k] = Dual(m.xyz[3 * (int64_t)nd[i] + k], (3 * i + k == d) ? 1.0 : 0.0);
  }
  const double* pr = m.quad_prop + 5 * e;
  Dual tt(pr[0], d == 12 ? 1.0 : 0.0);
  Dual sc(m.quad_scale[e], d == 13 ? 1.0 : 0.0);
  QGeom<Dual> g;
  quad_geom(X, g);
  QMat<Dual> mt = quad_mat<Dual>(tt, pr[1], pr[2]);
  // corner DOFs in the local warped frame
  Dual dl[4][6], du[4][6];
  for (int i = 0; i < 4; ++i) {
    const double* us = u + 6 * (int64_t)nd[i];
    const double* ls = lam + 6 * (int64_t)nd[i];
    Dual ug[3] = {Dual(us[0]), Dual(us[1]), Dual(us[2])};
    Dual rg[3] = {Dual(us[3]), Dual(us[4]), Dual(us[5])};
    Dual lg[3] = {Dual(ls[0]), Dual(ls[1]), Dual(ls[2])};
    Dual lr[3] = {Dual(ls[3]), Dual(ls[4]), Dual(ls[5])};
    to_local_warped(g, i, ug, rg, du[i]);
    to_local_warped(g, i, lg, lr, dl[i]);
  }
  Dual phi = 0.0;
  for (int gp = 0; gp < 4; ++gp) {
    QGP<Dual> q;
    quad_gp(g, gp, q);
    Dual eu[9], el[9], gxu = 0.0, geu = 0.0, gxl = 0.0, gel = 0.0;
    for (int s = 0; s < 9; ++s) { eu[s] = 0.0; el[s] = 0.0; }
    for (int i = 0; i < 4; ++i) {
      add_strains(q, i, du[i], eu, gxu, geu);
      add_strains(q, i, dl[i], el, gxl, gel);
    }
    finish_shear(q, gxu, geu, eu);
    finish_shear(q, gxl, gel, el);
    Dual sig[9];
    apply_D(mt, eu, sig);
    Dual en = 0.0;
    for (int s = 0; s < 9; ++s) en += el[s] * sig[s];
    phi += en * q.det;
  }
  phi = phi * sc;
  // loads: -(gamma t + q) A / 4 on uz of each corner
  Dual fz = -((m.unit_weight * tt + m.surface_load) * g.area) / 4.0;
  double wz = 0.0;
  for (int i = 0; i < 4; ++i) {
    const int64_t z = 6 * (int64_t)nd[i] + 2;
    wz += c_lam * lam[z] + c_u * (m.fixed[z] ? 0.0 : u[z]);
  }
  gquad[t] = wz * fz.d - c_lam * phi.d;
}

// ---- penalised material volume of the size optimisation (Sec. 3.3) ------------------------
// Thread (e, d), d in 0..13 (the layout of the adjoint element terms): gw[14 e + d] =
// t_e dA_e/dX_d for the 12 corner coordinates, dW/dt_e = A_e - [t_e < t_min] / t_min for
// d = 12, 0 for d = 13; the d = 12 thread also writes the element's share of W,
// w[e] = A_e t_e + max(0, (t_min - t_e) / t_min), with A_e = |d13 x d24| / 2 (the load area).
__global__ void __launch_bounds__(128) k_volume_terms(Mesh m, double t_min, double* gw,
                                                      double* w) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 14 * (int64_t)m.n_quads) return;
  const int64_t e = t / 14;
  const int d = (int)(t % 14);
  Dual X[4][3];
  for (int i = 0; i < 4; ++i) {
    const int nd = m.quad_nodes[4 * e + i];
    for (int k = 0; k < 3; ++k)
      X[i][k] = Dual(m.xyz[3 * (int64_t)nd + k], (3 * i + k == d) ? 1.0 : 0.0);
  }
  QGeom<Dual> g;
  quad_geom(X, g);
  const double te = m.quad_prop[5 * e];
  const bool below = te < t_min;
  double v = 0.0;
  if (d < 12) {
    v = te * g.area.d;
  } else if (d == 12) {
    v = g.area.v - (below ? 1.0 / t_min : 0.0);
    w[e] = g.area.v * te + (below ? (t_min - te) / t_min : 0.0);
  }
  gw[t] = v;
}

// dg/dxyz of node I: sum over incident elements in ascending element order (the diagonal
// block slot of row I lists exactly the incident elements, sorted by contribution id).
__global__ void k_gather(Mesh m, const int32_t* bdiag, const int32_t* bseg, const int32_t* bperm,
                         const double* gbeam, const double* gquad, double* dg_dxyz) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 3 * (int64_t)m.n_nodes) return;
  int I = (int)(t / 3), c = (int)(t % 3);
  int s = bdiag[I];
  double acc = 0.0;
  for (int p = bseg[s]; p < bseg[s + 1]; ++p) {
    BlockRef r = decode_block(bperm[p], m.n_beams);
    acc += r.quad ? gquad[14 * (int64_t)r.e + 3 * r.la + c] : gbeam[6 * (int64_t)r.e + 3 * r.la + c];
  }
  dg_dxyz[t] = acc;
}

__global__ void k_quad_param_grads(int n_quads, const double* gquad, double* dg_dt,
                                   double* dg_dscale) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n_quads) return;
  if (dg_dt) dg_dt[e] = gquad[14 * e + 12];
  if (dg_dscale) dg_dscale[e] = gquad[14 * e + 13];
}

inline unsigned nblk(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

}  // namespace

hipError_t launch_element_stiffness(const Mesh& m, double* coo, double* qarea, unsigned* d_err,
                                    hipStream_t s) {
  if (m.n_beams)
    hipLaunchKernelGGL(k_beam_stiffness, dim3(nblk(12 * (int64_t)m.n_beams, 192)), dim3(192), 0,
                       s, m, coo, d_err);
  if (m.n_quads)
    hipLaunchKernelGGL(k_quad_stiffness, dim3(nblk(m.n_quads, QW)), dim3(64 * QW), 0, s, m, coo,
                       qarea, d_err);
  return hipGetLastError();
}

hipError_t launch_adjoint_terms(const Mesh& m, const Pattern& pat, const double* u,
                                const double* lam, double c_lam, double c_u, double* gbeam,
                                double* gquad, hipStream_t s) {
  (void)pat;
  if (m.n_beams)
    hipLaunchKernelGGL(k_beam_adjoint, dim3(nblk(6 * (int64_t)m.n_beams, 128)), dim3(128), 0, s,
                       m, u, lam, c_lam, gbeam);
  if (m.n_quads)
    hipLaunchKernelGGL(k_quad_adjoint, dim3(nblk(14 * (int64_t)m.n_quads, 128)), dim3(128), 0, s,
                       m, u, lam, c_lam, c_u, gquad);
  return hipGetLastError();
}

hipError_t launch_volume_terms(const Mesh& m, double t_min, double* gw, double* w,
                               hipStream_t s) {
  if (m.n_quads)
    hipLaunchKernelGGL(k_volume_terms, dim3(nblk(14 * (int64_t)m.n_quads, 128)), dim3(128), 0,
                       s, m, t_min, gw, w);
  return hipGetLastError();
}

hipError_t launch_gather(const Mesh& m, const Pattern& pat, const double* gbeam,
                         const double* gquad, double* dg_dxyz, double* dg_dt, double* dg_dscale,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(nblk(3 * (int64_t)m.n_nodes, 256)), dim3(256), 0, s, m,
                     pat.bdiag, pat.bseg, pat.bperm, gbeam, gquad, dg_dxyz);
  if (m.n_quads && (dg_dt || dg_dscale))
    hipLaunchKernelGGL(k_quad_param_grads, dim3(nblk(m.n_quads, 256)), dim3(256), 0, s,
                       m.n_quads, gquad, dg_dt, dg_dscale);
  return hipGetLastError();
}

}  // namespace sso
