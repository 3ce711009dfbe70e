// Oracle: plain, slow, FP64 CPU definition of the finite cell Stokes discretisation, the restricted
// additive smoother, the grid transfers and the geometric multigrid V-cycle of Saberi & Vogel,
// "A restricted additive smoother for finite cell flow problems" (arXiv 2403.11636).
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or load this file or the
// library built from it: only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
// use it. It shares no code, header or table with the HIP library.
//
// Every function states the passage it follows. Where the paper is silent, the reading taken is
// stated at the function (the full list of readings is kept in the design notes of the repository).
//
// Conventions
//   * Unit box [0,1]^d, d = 2 or 3, uniform background grid with n cells per axis; level l of the
//     hierarchy has n >> (nlev-1-l) cells per axis (level 0 = coarsest, nlev-1 = finest).
//   * Nodes are numbered lexicographically, x fastest. A vector holds d+1 fields in SoA order
//     [u_x | u_y | (u_z) | p], each field one value per node (Q1-Q1, Sec. 2 "we focus on Q1-Q1").
//   * The assembled operator of a level is kept as a node stencil: for every node, field f, neighbour
//     offset o in {-1,0,1}^d and field g, the entry L[(node,f),(node+o,g)].
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

enum { BC_NOSLIP = 0, BC_INFLOW = 1, BC_NEUMANN = 2 };
enum { ERR_OK = 0, ERR_ARG = -1, ERR_SINGULAR = -4, ERR_NOCONV = -5 };

struct Ball {
  double c[3];
  double r;
};

struct Level {
  int n = 0;        // cells per axis
  double h = 0;     // cell size
  int qd = 0;       // space-tree depth of its cut cells (the finest level's leaf size on every level)
  long N = 0;       // nodes (n+1)^d
  std::vector<double> st;       // node stencil, size N*(d+1)*3^d*(d+1)
  std::vector<signed char> kind;  // per cell: 0 physical, 1 fictitious, 2 cut
  std::vector<double> Z;        // cache_inverse rows, (d+1) x 5^d... (built on demand)
  std::vector<int> Zcount;      // |S_i| per node for Z
  std::vector<long> Zoff;       // offset of node i's rows in Z
  bool has_Z = false;
};

struct Prob {
  int d = 2, n = 8, nlev = 1, q = 3, force = 0;
  int immersed = 0;  // 1: the obstacle surfaces are Dirichlet boundaries (no-slip)
  double eta = 1, alpha_f = 1e-8, beta = 20, ubar = 0.3;
  int bc[6] = {0, 0, 0, 0, 0, 0};
  std::vector<Ball> balls;
  std::vector<Level> lev;
  // coarsest-level dense LU (Sec. 3: direct solver on the coarsest grid)
  std::vector<double> clu;
  std::vector<int> cpiv;
  int cdim = 0;
  bool bordered = false;
  bool coarse_ok = false;
};

int ipow(int b, int e) {
  int r = 1;
  while (e-- > 0) r *= b;
  return r;
}

// ---------------------------------------------------------------------------------------------
// Geometry: alpha of Eq. (7) with the small value alpha_f in the fictitious part. A point is in
// the fictitious part when it lies inside or on an obstacle ball (reading: phi = 0 is obstacle).
// ---------------------------------------------------------------------------------------------
double alpha_at(const Prob& P, const double* x) {
  for (const Ball& b : P.balls) {
    double s = 0;
    for (int k = 0; k < P.d; ++k) {
      double t = x[k] - b.c[k];
      s += t * t;
    }
    if (s <= b.r * b.r) return P.alpha_f;
  }
  return 1.0;
}

// Classify the box [lo, lo+s]^d: 1 if it lies inside (or on) some ball, 2 if some ball boundary
// passes through its interior, 0 otherwise (exact ball-box distance test).
int box_kind(const Prob& P, const double* lo, double s) {
  bool cut = false;
  for (const Ball& b : P.balls) {
    double dmin2 = 0, dmax2 = 0;
    for (int k = 0; k < P.d; ++k) {
      double a = lo[k] - b.c[k];
      double e = lo[k] + s - b.c[k];
      double m = 0;
      if (a > 0)
        m = a;
      else if (e < 0)
        m = -e;
      dmin2 += m * m;
      double M = std::max(std::fabs(a), std::fabs(e));
      dmax2 += M * M;
    }
    double r2 = b.r * b.r;
    if (dmax2 <= r2) return 1;
    if (dmin2 < r2) cut = true;
  }
  return cut ? 2 : 0;
}

// ---------------------------------------------------------------------------------------------
// Quadrature. The paper only asks for a "sufficiently accurate integration" of cut cells (Sec. 1).
// Reading: a space tree (quadtree/octree) splits a cell into 2^d children while the child is cut
// and its depth is below the level's depth; every leaf gets the 2^d-point tensor Gauss rule with
// alpha evaluated at each Gauss point. Uncut cells are leaves at depth 0. The depth is q on the
// finest level and one more per coarser level, so every level of the hierarchy of discretisations
// (Sec. 3) integrates its cut cells on leaves of the same size h_finest / 2^q: the coarse cell's
// tree descends through its fine cells and ends on their leaves. The alpha-weighted forms of a
// coarse level are then the Galerkin restrictions of the fine ones, and a physical sliver that the
// fine level resolves is not lost on a coarser one (with alpha_f = 1e-10 such a loss makes the
// coarse operator up to 1/alpha_f-fold softer there and the V-cycle diverge).
// ---------------------------------------------------------------------------------------------
struct QPt {
  double x[3];
  double w;
  double alpha;
};

const double kG0 = 0.5 - 0.5 / std::sqrt(3.0);
const double kG1 = 0.5 + 0.5 / std::sqrt(3.0);

void gauss_box(const Prob& P, const double* lo, double s, std::vector<QPt>& out) {
  int np = 1 << P.d;
  double w = std::pow(0.5 * s, P.d);
  for (int g = 0; g < np; ++g) {
    QPt q;
    q.x[0] = q.x[1] = q.x[2] = 0;
    for (int k = 0; k < P.d; ++k) q.x[k] = lo[k] + s * (((g >> k) & 1) ? kG1 : kG0);
    q.w = w;
    q.alpha = alpha_at(P, q.x);
    out.push_back(q);
  }
}

void tree_points(const Prob& P, const double* lo, double s, int depth, int maxdepth, std::vector<QPt>& out,
                 long* cut_leaves, double* cut_leaf_vol) {
  int kind = box_kind(P, lo, s);
  if (kind == 2 && depth < maxdepth) {
    int nc = 1 << P.d;
    for (int c = 0; c < nc; ++c) {
      double clo[3] = {0, 0, 0};
      for (int k = 0; k < P.d; ++k) clo[k] = lo[k] + (((c >> k) & 1) ? 0.5 * s : 0.0);
      tree_points(P, clo, 0.5 * s, depth + 1, maxdepth, out, cut_leaves, cut_leaf_vol);
    }
    return;
  }
  if (kind == 2) {
    if (cut_leaves) ++*cut_leaves;
    if (cut_leaf_vol) *cut_leaf_vol += std::pow(s, P.d);
  }
  gauss_box(P, lo, s, out);
}

// ---------------------------------------------------------------------------------------------
// Immersed Dirichlet boundary: the obstacle surfaces belong to Gamma_D of Eq. (5) (no-slip, w = 0),
// 2D. Quadrature on the arcs of the circles inside a cell. Reading (the paper fixes no rule): the
// circle is split at its crossings with the four lines of the cell box; a piece whose middle point
// lies in the closed box is cut into ceil(width / (pi/8)) equal angular parts, each integrated with
// the 6-point Gauss-Legendre rule in the angle, ds = r dtheta. n is the unit normal out of the
// physical domain, i.e. into the obstacle.
// ---------------------------------------------------------------------------------------------
struct APt {
  double x[3];
  double w;
  double n[3];
};

const double kGL6x[3] = {0.2386191860831969086305017, 0.6612093864662645136613996, 0.9324695142031520278123016};
const double kGL6w[3] = {0.4679139345726910473898703, 0.3607615730481386075698335, 0.1713244923791703450402961};

void arc_points(const Prob& P, const double* lo, double h, std::vector<APt>& out) {
  const double two_pi = 2.0 * M_PI;
  for (const Ball& b : P.balls) {
    std::vector<double> th = {0.0, two_pi};
    for (int k = 0; k < 2; ++k)
      for (int s = 0; s < 2; ++s) {
        const double dist = lo[k] + s * h - b.c[k];
        if (std::fabs(dist) >= b.r) continue;
        const double other = std::sqrt(b.r * b.r - dist * dist);
        for (int sg = -1; sg <= 1; sg += 2) {
          double t = k == 0 ? std::atan2(sg * other, dist) : std::atan2(dist, sg * other);
          if (t < 0) t += two_pi;
          th.push_back(t);
        }
      }
    std::sort(th.begin(), th.end());
    for (size_t i = 0; i + 1 < th.size(); ++i) {
      const double t0 = th[i], t1 = th[i + 1];
      if (!(t1 > t0)) continue;
      const double tm = 0.5 * (t0 + t1);
      const double pm[2] = {b.c[0] + b.r * std::cos(tm), b.c[1] + b.r * std::sin(tm)};
      bool inside = true;
      for (int k = 0; k < 2; ++k) inside = inside && pm[k] >= lo[k] && pm[k] <= lo[k] + h;
      if (!inside) continue;
      const int parts = (int)std::ceil((t1 - t0) / (M_PI / 8));
      for (int j = 0; j < parts; ++j) {
        const double a = t0 + (t1 - t0) * j / parts, e = t0 + (t1 - t0) * (j + 1) / parts;
        const double mid = 0.5 * (a + e), half = 0.5 * (e - a);
        for (int g = 0; g < 6; ++g) {
          const double xi = g < 3 ? -kGL6x[2 - g] : kGL6x[g - 3];
          const double wg = g < 3 ? kGL6w[2 - g] : kGL6w[g - 3];
          const double t = mid + half * xi;
          APt q;
          q.x[0] = b.c[0] + b.r * std::cos(t);
          q.x[1] = b.c[1] + b.r * std::sin(t);
          q.x[2] = 0;
          q.n[0] = -std::cos(t);
          q.n[1] = -std::sin(t);
          q.n[2] = 0;
          q.w = wg * half * b.r;
          out.push_back(q);
        }
      }
    }
  }
}

// Immersed Dirichlet boundary in 3D: quadrature on the parts of the sphere surfaces inside a cell
// box. Reading (the paper fixes no rule): a point of a sphere is c + r u with
// u = (sin theta cos phi, sin theta sin phi, cos theta), area element r^2 sin theta dtheta dphi.
// The part inside the box is where every u_k lies in [a_k, b_k] (the box bounds relative to the
// centre, divided by r). The theta-range is cut wherever the circle of radius rho = sin theta in the
// (u_0, u_1) plane starts or stops meeting one of the lines u_0 = a_0, b_0, u_1 = a_1, b_1 (rho equal
// to the line's distance) or passes a corner of their rectangle (rho^2 = x^2 + y^2). Between these
// cuts the ends of the admitted arcs move smoothly with theta up to square-root behaviour at the
// cuts, which the substitution theta = t0 + (t1 - t0)(3 s^2 - 2 s^3) removes; s in [0, 1] is split
// into ceil((t1 - t0) / (pi/8)) equal parts, each with the 6-point Gauss-Legendre rule. At each
// such theta the circle is split at its crossings with the four lines, and an arc whose middle
// point lies in the closed rectangle is split into ceil(width / (pi/8)) equal angular parts, each
// with the 6-point rule in phi. n = -u: out of the physical domain, into the obstacle.
// ---------------------------------------------------------------------------------------------
void sphere_points(const Prob& P, const double* lo, double h, std::vector<APt>& out) {
  const double two_pi = 2.0 * M_PI;
  auto gl6 = [](int g, double* xi, double* wg) {
    *xi = g < 3 ? -kGL6x[2 - g] : kGL6x[g - 3];
    *wg = g < 3 ? kGL6w[2 - g] : kGL6w[g - 3];
  };
  for (const Ball& B : P.balls) {
    double a[3], b[3];
    for (int k = 0; k < 3; ++k) {
      a[k] = (lo[k] - B.c[k]) / B.r;
      b[k] = (lo[k] + h - B.c[k]) / B.r;
    }
    // cos theta = u_2 in [a_2, b_2]
    if (!(std::min(b[2], 1.0) > std::max(a[2], -1.0))) continue;
    const double th_lo = b[2] >= 1.0 ? 0.0 : std::acos(b[2]);
    const double th_hi = a[2] <= -1.0 ? M_PI : std::acos(a[2]);
    if (!(th_hi > th_lo)) continue;
    std::vector<double> tcut = {th_lo, th_hi};
    auto cut_at_radius2 = [&](double rho2) {
      if (!(rho2 >= 0.0 && rho2 < 1.0)) return;
      const double q = std::asin(std::sqrt(rho2));  // sin theta = rho at q and pi - q
      if (q > th_lo && q < th_hi) tcut.push_back(q);
      if (M_PI - q > th_lo && M_PI - q < th_hi) tcut.push_back(M_PI - q);
    };
    const double xl[2] = {a[0], b[0]}, yl[2] = {a[1], b[1]};
    for (int i = 0; i < 2; ++i) cut_at_radius2(xl[i] * xl[i]);
    for (int j = 0; j < 2; ++j) cut_at_radius2(yl[j] * yl[j]);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) cut_at_radius2(xl[i] * xl[i] + yl[j] * yl[j]);
    std::sort(tcut.begin(), tcut.end());
    for (size_t i = 0; i + 1 < tcut.size(); ++i) {
      const double t0 = tcut[i], t1 = tcut[i + 1];
      if (!(t1 > t0)) continue;
      const int tparts = (int)std::ceil((t1 - t0) / (M_PI / 8));
      for (int pt = 0; pt < tparts; ++pt) {
        const double s0 = (double)pt / tparts, s1 = (double)(pt + 1) / tparts;
        for (int gt = 0; gt < 6; ++gt) {
          double xi, wg;
          gl6(gt, &xi, &wg);
          const double s = 0.5 * (s0 + s1) + 0.5 * (s1 - s0) * xi;
          const double th = t0 + (t1 - t0) * s * s * (3.0 - 2.0 * s);
          const double rho = std::sin(th), t = std::cos(th);
          const double wt = 0.5 * (s1 - s0) * wg * (t1 - t0) * 6.0 * s * (1.0 - s) * rho;
          if (!(rho > 0.0)) continue;
          // the circle of radius rho against the lines of the rectangle [a0, b0] x [a1, b1]
          std::vector<double> ph = {0.0, two_pi};
          for (int k = 0; k < 2; ++k) {
            const double v = xl[k] / rho;
            if (std::fabs(v) < 1.0) {
              const double q = std::acos(v);
              ph.push_back(q);
              ph.push_back(two_pi - q);
            }
          }
          for (int k = 0; k < 2; ++k) {
            const double v = yl[k] / rho;
            if (std::fabs(v) < 1.0) {
              const double q = std::asin(v);
              ph.push_back(q < 0 ? q + two_pi : q);
              ph.push_back(M_PI - q);
            }
          }
          std::sort(ph.begin(), ph.end());
          for (size_t j = 0; j + 1 < ph.size(); ++j) {
            const double f0 = ph[j], f1 = ph[j + 1];
            if (!(f1 > f0)) continue;
            const double fm = 0.5 * (f0 + f1);
            const double um = rho * std::cos(fm), vm = rho * std::sin(fm);
            if (!(um >= a[0] && um <= b[0] && vm >= a[1] && vm <= b[1])) continue;
            const int fparts = (int)std::ceil((f1 - f0) / (M_PI / 8));
            for (int pf = 0; pf < fparts; ++pf) {
              const double e0 = f0 + (f1 - f0) * pf / fparts, e1 = f0 + (f1 - f0) * (pf + 1) / fparts;
              for (int gf = 0; gf < 6; ++gf) {
                double xf, wf;
                gl6(gf, &xf, &wf);
                const double phi = 0.5 * (e0 + e1) + 0.5 * (e1 - e0) * xf;
                const double u[3] = {rho * std::cos(phi), rho * std::sin(phi), t};
                APt q;
                for (int k = 0; k < 3; ++k) {
                  q.x[k] = B.c[k] + B.r * u[k];
                  q.n[k] = -u[k];
                }
                q.w = B.r * B.r * wt * 0.5 * (e1 - e0) * wf;
                out.push_back(q);
              }
            }
          }
        }
      }
    }
  }
}

// Q1 basis of the cell with lower corner lo and size h, local node a has bit k of a as its
// k-th coordinate offset (tensor ordering). Returns values and physical gradients at x.
void q1_basis(int d, const double* lo, double h, const double* x, double* phi, double (*grad)[3]) {
  double xi[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) xi[k] = (x[k] - lo[k]) / h;
  int nn = 1 << d;
  for (int a = 0; a < nn; ++a) {
    double v = 1;
    for (int k = 0; k < d; ++k) v *= ((a >> k) & 1) ? xi[k] : 1.0 - xi[k];
    phi[a] = v;
    for (int j = 0; j < d; ++j) {
      double g = (((a >> j) & 1) ? 1.0 : -1.0) / h;
      for (int k = 0; k < d; ++k)
        if (k != j) g *= ((a >> k) & 1) ? xi[k] : 1.0 - xi[k];
      grad[a][j] = g;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Data of the problem: body force f (manufactured from a stream function) and Dirichlet data w.
// ---------------------------------------------------------------------------------------------
// g(t) = t^2 (1-t)^2 and its derivatives.
double g0(double t) { return t * t * (1 - t) * (1 - t); }
double g1(double t) { return 2 * t - 6 * t * t + 4 * t * t * t; }
double g2(double t) { return 2 - 12 * t + 12 * t * t; }
double g3(double t) { return -12 + 24 * t; }

// Manufactured body force f = -eta Lap u + grad p with u = curl psi.
//   2D: psi = g(x) g(y), u = (g(x) g'(y), -g'(x) g(y)), p = x^3 + y^3 - 1/2.
//   3D: u = (g(x) g'(y) g(z), -g'(x) g(y) g(z), 0), p = x^3 + y^3 + z^3 - 3/4.
void body_force(const Prob& P, const double* x, double* f) {
  f[0] = f[1] = f[2] = 0;
  if (P.force != 1) return;
  double X = x[0], Y = x[1];
  if (P.d == 2) {
    double lap_ux = g2(X) * g1(Y) + g0(X) * g3(Y);
    double lap_uy = -(g3(X) * g0(Y) + g1(X) * g2(Y));
    f[0] = -P.eta * lap_ux + 3 * X * X;
    f[1] = -P.eta * lap_uy + 3 * Y * Y;
  } else {
    double Z = x[2];
    double lap_ux = g2(X) * g1(Y) * g0(Z) + g0(X) * g3(Y) * g0(Z) + g0(X) * g1(Y) * g2(Z);
    double lap_uy = -(g3(X) * g0(Y) * g0(Z) + g1(X) * g2(Y) * g0(Z) + g1(X) * g0(Y) * g2(Z));
    f[0] = -P.eta * lap_ux + 3 * X * X;
    f[1] = -P.eta * lap_uy + 3 * Y * Y;
    f[2] = 3 * Z * Z;
  }
}

// Dirichlet data on face (axis k, side s): zero (no-slip) or a parabolic inflow of mean-like
// amplitude ubar through that face (Eq. 16 with H = 1; in 3D the product profile 16 y(1-y) z(1-z)).
void dirichlet_w(const Prob& P, int k, int s, const double* x, double* w) {
  w[0] = w[1] = w[2] = 0;
  if (P.bc[2 * k + s] != BC_INFLOW) return;
  double prof = P.ubar;
  for (int j = 0; j < P.d; ++j)
    if (j != k) prof *= 4.0 * x[j] * (1.0 - x[j]);
  double nk = s ? 1.0 : -1.0;
  w[k] = -nk * prof;  // points into the domain
}

// ---------------------------------------------------------------------------------------------
// Element matrix of cell `cell` on level `lv` (Eq. 9, 10 with the finite cell alpha of Eq. 5-7).
// Index of (local node a, field f) is f*2^d + a. Contains
//   a:  (eta grad v, alpha grad u) per velocity component, plus Nitsche terms on Dirichlet walls
//       -(v, n.eta grad u) - (n.eta grad v, u) + (v, lambda u), lambda = beta*eta/h (reading: the
//       paper does not fix lambda);
//   b:  -(div v, alpha p) + (v, n p) on Dirichlet walls, and the symmetric pressure-row entries;
//   c:  -(1/eta) (q - Pi0 q, p - Pi0 p) over the cell, Pi0 = cell mean (Eq. 10-11; reading: no alpha).
// Returns the volume quadrature points used (for the right-hand side).
// ---------------------------------------------------------------------------------------------
void cell_lo(const Prob& P, const Level& L, long cell, double* lo, int* ci) {
  long c = cell;
  for (int k = 0; k < P.d; ++k) {
    ci[k] = (int)(c % L.n);
    c /= L.n;
    lo[k] = ci[k] * L.h;
  }
  for (int k = P.d; k < 3; ++k) {
    ci[k] = 0;
    lo[k] = 0;
  }
}

void element_matrix(const Prob& P, const Level& L, long cell, std::vector<double>& Le,
                    std::vector<QPt>* pts_out) {
  const int d = P.d, nn = 1 << d, ne = nn * (d + 1);
  Le.assign((size_t)ne * ne, 0.0);
  double lo[3];
  int ci[3];
  cell_lo(P, L, cell, lo, ci);
  const double h = L.h;
  auto I = [&](int a, int f) { return f * nn + a; };

  std::vector<QPt> pts;
  tree_points(P, lo, h, 0, L.qd, pts, nullptr, nullptr);
  double phi[8], grad[8][3];
  for (const QPt& q : pts) {
    q1_basis(d, lo, h, q.x, phi, grad);
    double wa = q.w * q.alpha;
    for (int a = 0; a < nn; ++a)
      for (int b = 0; b < nn; ++b) {
        double gg = 0;
        for (int k = 0; k < d; ++k) gg += grad[a][k] * grad[b][k];
        double kv = wa * P.eta * gg;
        for (int c = 0; c < d; ++c) Le[(size_t)I(a, c) * ne + I(b, c)] += kv;
        for (int c = 0; c < d; ++c) {
          double bv = -wa * grad[a][c] * phi[b];
          Le[(size_t)I(a, c) * ne + I(b, d)] += bv;
          Le[(size_t)I(b, d) * ne + I(a, c)] += bv;
        }
      }
  }
  // Stabilisation: exact mass matrix with the 2^d Gauss rule (exact for Q1 x Q1), no alpha.
  {
    std::vector<QPt> cp;
    gauss_box(P, lo, h, cp);  // the alpha values it records are not used here
    std::vector<double> M((size_t)nn * nn, 0.0), m(nn, 0.0);
    for (const QPt& q : cp) {
      q1_basis(d, lo, h, q.x, phi, grad);
      for (int a = 0; a < nn; ++a) {
        m[a] += q.w * phi[a];
        for (int b = 0; b < nn; ++b) M[(size_t)a * nn + b] += q.w * phi[a] * phi[b];
      }
    }
    double vol = std::pow(h, d);
    for (int a = 0; a < nn; ++a)
      for (int b = 0; b < nn; ++b)
        Le[(size_t)I(a, d) * ne + I(b, d)] += -(1.0 / P.eta) * (M[(size_t)a * nn + b] - m[a] * m[b] / vol);
  }
  // Nitsche terms on the Dirichlet walls of the embedding box.
  const double lam = P.beta * P.eta / h;
  for (int k = 0; k < d; ++k)
    for (int s = 0; s < 2; ++s) {
      bool on_wall = s ? (ci[k] == L.n - 1) : (ci[k] == 0);
      if (!on_wall || P.bc[2 * k + s] == BC_NEUMANN) continue;
      double nk = s ? 1.0 : -1.0;
      int nt = 1 << (d - 1);
      double w = std::pow(0.5 * h, d - 1);
      for (int g = 0; g < nt; ++g) {
        double x[3] = {0, 0, 0};
        int t = 0;
        for (int j = 0; j < d; ++j) {
          if (j == k) {
            x[j] = lo[j] + (s ? h : 0.0);
          } else {
            x[j] = lo[j] + h * (((g >> t) & 1) ? kG1 : kG0);
            ++t;
          }
        }
        q1_basis(d, lo, h, x, phi, grad);
        for (int a = 0; a < nn; ++a)
          for (int b = 0; b < nn; ++b) {
            double kv = w * (-P.eta * phi[a] * nk * grad[b][k] - P.eta * nk * grad[a][k] * phi[b] +
                             lam * phi[a] * phi[b]);
            for (int c = 0; c < d; ++c) Le[(size_t)I(a, c) * ne + I(b, c)] += kv;
            double bv = w * phi[a] * nk * phi[b];
            Le[(size_t)I(a, k) * ne + I(b, d)] += bv;
            Le[(size_t)I(b, d) * ne + I(a, k)] += bv;
          }
      }
    }
  // Nitsche terms on the immersed obstacle surfaces (cut cells): the same forms as on the walls.
  if (P.immersed && box_kind(P, lo, h) == 2) {
    std::vector<APt> ap;
    if (d == 2)
      arc_points(P, lo, h, ap);
    else
      sphere_points(P, lo, h, ap);
    for (const APt& q : ap) {
      q1_basis(d, lo, h, q.x, phi, grad);
      for (int a = 0; a < nn; ++a)
        for (int b = 0; b < nn; ++b) {
          double dna = 0, dnb = 0;
          for (int k = 0; k < d; ++k) {
            dna += q.n[k] * grad[a][k];
            dnb += q.n[k] * grad[b][k];
          }
          double kv = q.w * (-P.eta * phi[a] * dnb - P.eta * dna * phi[b] + lam * phi[a] * phi[b]);
          for (int c = 0; c < d; ++c) Le[(size_t)I(a, c) * ne + I(b, c)] += kv;
          for (int c = 0; c < d; ++c) {
            double bv = q.w * phi[a] * q.n[c] * phi[b];
            Le[(size_t)I(a, c) * ne + I(b, d)] += bv;
            Le[(size_t)I(b, d) * ne + I(a, c)] += bv;
          }
        }
    }
  }
  if (pts_out) *pts_out = pts;
}

// Element right-hand side of Eq. (9): f(v) = (v, alpha f) - (n.eta grad v, w) + (v, lambda w) on
// Dirichlet walls (h = 0 on Neumann walls, "do-nothing"); g(q) = (n q, w) on Dirichlet walls.
void element_rhs(const Prob& P, const Level& L, long cell, const std::vector<QPt>& pts, double* Fe) {
  const int d = P.d, nn = 1 << d, ne = nn * (d + 1);
  for (int i = 0; i < ne; ++i) Fe[i] = 0;
  double lo[3];
  int ci[3];
  cell_lo(P, L, cell, lo, ci);
  const double h = L.h;
  double phi[8], grad[8][3], f[3], w3[3];
  for (const QPt& q : pts) {
    q1_basis(d, lo, h, q.x, phi, grad);
    body_force(P, q.x, f);
    for (int a = 0; a < nn; ++a)
      for (int c = 0; c < d; ++c) Fe[c * nn + a] += q.w * q.alpha * f[c] * phi[a];
  }
  const double lam = P.beta * P.eta / h;
  for (int k = 0; k < d; ++k)
    for (int s = 0; s < 2; ++s) {
      bool on_wall = s ? (ci[k] == L.n - 1) : (ci[k] == 0);
      if (!on_wall || P.bc[2 * k + s] == BC_NEUMANN) continue;
      double nk = s ? 1.0 : -1.0;
      int nt = 1 << (d - 1);
      double w = std::pow(0.5 * h, d - 1);
      for (int g = 0; g < nt; ++g) {
        double x[3] = {0, 0, 0};
        int t = 0;
        for (int j = 0; j < d; ++j) {
          if (j == k) {
            x[j] = lo[j] + (s ? h : 0.0);
          } else {
            x[j] = lo[j] + h * (((g >> t) & 1) ? kG1 : kG0);
            ++t;
          }
        }
        q1_basis(d, lo, h, x, phi, grad);
        dirichlet_w(P, k, s, x, w3);
        for (int a = 0; a < nn; ++a) {
          for (int c = 0; c < d; ++c)
            Fe[c * nn + a] += w * (-P.eta * nk * grad[a][k] * w3[c] + lam * phi[a] * w3[c]);
          Fe[d * nn + a] += w * phi[a] * nk * w3[k];
        }
      }
    }
}

// ---------------------------------------------------------------------------------------------
// Grid indexing helpers.
// ---------------------------------------------------------------------------------------------
void node_coords(int d, int n, long node, int* c) {
  long t = node;
  for (int k = 0; k < d; ++k) {
    c[k] = (int)(t % (n + 1));
    t /= (n + 1);
  }
  for (int k = d; k < 3; ++k) c[k] = 0;
}

long node_index(int d, int n, const int* c) {
  long idx = 0, m = 1;
  for (int k = 0; k < d; ++k) {
    idx += c[k] * m;
    m *= (n + 1);
  }
  return idx;
}

int nstencil(int d) { return ipow(3, d); }

size_t st_index(int d, long node, int f, int o, int g) {
  const int nf = d + 1, no = nstencil(d);
  return (((size_t)node * nf + f) * no + o) * nf + g;
}

// Cell node a (tensor bits) of cell ci.
long cell_node(int d, int n, const int* ci, int a) {
  int c[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) c[k] = ci[k] + ((a >> k) & 1);
  return node_index(d, n, c);
}

// Assemble the level operator L (Eq. 12) into the node stencil: sum of element matrices.
void assemble_level(Prob& P, int l) {
  Level& L = P.lev[l];
  const int d = P.d, nn = 1 << d, ne = nn * (d + 1), nf = d + 1;
  long ncell = 1;
  for (int k = 0; k < d; ++k) ncell *= L.n;
  L.kind.assign(ncell, 0);
  std::vector<double> all((size_t)ncell * ne * ne);
#pragma omp parallel for schedule(dynamic, 64)
  for (long c = 0; c < ncell; ++c) {
    double lo[3];
    int ci[3];
    cell_lo(P, L, c, lo, ci);
    L.kind[c] = (signed char)box_kind(P, lo, L.h);
    std::vector<double> Le;
    element_matrix(P, L, c, Le, nullptr);
    std::copy(Le.begin(), Le.end(), all.begin() + (size_t)c * ne * ne);
  }
  L.st.assign((size_t)L.N * nf * nstencil(d) * nf, 0.0);
  for (long c = 0; c < ncell; ++c) {
    double lo[3];
    int ci[3];
    cell_lo(P, L, c, lo, ci);
    const double* Le = &all[(size_t)c * ne * ne];
    for (int a = 0; a < nn; ++a)
      for (int b = 0; b < nn; ++b) {
        long na = cell_node(d, L.n, ci, a);
        int o = 0, m = 1;
        for (int k = 0; k < d; ++k) {
          o += (((b >> k) & 1) - ((a >> k) & 1) + 1) * m;
          m *= 3;
        }
        for (int f = 0; f < nf; ++f)
          for (int g = 0; g < nf; ++g) L.st[st_index(d, na, f, o, g)] += Le[(size_t)(f * nn + a) * ne + g * nn + b];
      }
  }
}

// y = L x on level l (plain stencil product); with absolute = true, y = |L| x (entrywise |L|).
void matvec(const Prob& P, int l, const double* x, double* y, bool absolute = false) {
  const Level& L = P.lev[l];
  const int d = P.d, nf = d + 1, no = nstencil(d);
  const long N = L.N;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    int c[3];
    node_coords(d, L.n, i, c);
    for (int f = 0; f < nf; ++f) {
      double s = 0;
      for (int o = 0; o < no; ++o) {
        int cc[3] = {0, 0, 0};
        bool in = true;
        int t = o;
        for (int k = 0; k < d; ++k) {
          cc[k] = c[k] + (t % 3) - 1;
          t /= 3;
          if (cc[k] < 0 || cc[k] > L.n) in = false;
        }
        if (!in) continue;
        long j = node_index(d, L.n, cc);
        for (int g = 0; g < nf; ++g) {
          const double a = L.st[st_index(d, i, f, o, g)];
          s += (absolute ? std::fabs(a) : a) * x[g * N + j];
        }
      }
      y[f * N + i] = s;
    }
  }
}

void residual(const Prob& P, int l, const double* x, const double* b, double* r) {
  const long n = (long)(P.d + 1) * P.lev[l].N;
  matvec(P, l, x, r);
  for (long i = 0; i < n; ++i) r[i] = b[i] - r[i];
}

// Entry L[(node_a, f), (node_b, g)] of the assembled level operator (zero outside the stencil).
double entry(const Prob& P, int l, long dof_a, long dof_b) {
  const Level& L = P.lev[l];
  const int d = P.d;
  long na = dof_a % L.N, nb = dof_b % L.N;
  int f = (int)(dof_a / L.N), g = (int)(dof_b / L.N);
  int ca[3], cb[3];
  node_coords(d, L.n, na, ca);
  node_coords(d, L.n, nb, cb);
  int o = 0, m = 1;
  for (int k = 0; k < d; ++k) {
    int dd = cb[k] - ca[k];
    if (dd < -1 || dd > 1) return 0.0;
    o += (dd + 1) * m;
    m *= 3;
  }
  return L.st[st_index(d, na, f, o, g)];
}

// ---------------------------------------------------------------------------------------------
// Subdomain S_i of pressure node i (Sec. 3.1, definition after Eq. 15): p_i, the pressures
// connected to it (reading: structural couplings of the pressure block, i.e. the 3^d nodes sharing a
// cell with i), and every velocity DoF connected to those pressures through a structural non-zero of
// B^T (the d components at the 5^d nodes within max-norm distance 2). Truncated at the box walls.
// The list is sorted by global DoF index, i.e. R_i is a set of rows of the identity in global order.
// ---------------------------------------------------------------------------------------------
void patch_dofs(const Prob& P, int l, long node, std::vector<long>& S) {
  const Level& L = P.lev[l];
  const int d = P.d;
  S.clear();
  int c[3];
  node_coords(d, L.n, node, c);
  auto window = [&](int rad, int field) {
    int w = 2 * rad + 1;
    int tot = ipow(w, d);
    for (int t = 0; t < tot; ++t) {
      int cc[3] = {0, 0, 0};
      int u = t;
      bool in = true;
      for (int k = 0; k < d; ++k) {
        cc[k] = c[k] + (u % w) - rad;
        u /= w;
        if (cc[k] < 0 || cc[k] > L.n) in = false;
      }
      if (in) S.push_back((long)field * L.N + node_index(d, L.n, cc));
    }
  };
  for (int f = 0; f < d; ++f) window(2, f);
  window(1, d);
}

// Dense LU with partial pivoting (the local direct solver of Sec. 3.1.2): A is n x n row-major,
// overwritten by its factors; piv receives the row interchanges. Ties in the pivot search go to the
// lowest row. Returns false if a pivot is exactly zero (singular block).
bool lu_factor(int n, double* A, int* piv) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = std::fabs(A[(size_t)i * n + k]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    piv[k] = p;
    if (best == 0.0) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
    double inv = 1.0 / A[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      double lik = A[(size_t)i * n + k] * inv;
      A[(size_t)i * n + k] = lik;
      if (lik != 0.0)
        for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= lik * A[(size_t)k * n + j];
    }
  }
  return true;
}

// Solve A y = rhs with the factors from lu_factor (rhs overwritten by y).
void lu_solve(int n, const double* A, const int* piv, double* y) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) std::swap(y[k], y[piv[k]]);
  for (int i = 0; i < n; ++i) {
    double s = y[i];
    for (int j = 0; j < i; ++j) s -= A[(size_t)i * n + j] * y[j];
    y[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int j = i + 1; j < n; ++j) s -= A[(size_t)i * n + j] * y[j];
    y[i] = s / A[(size_t)i * n + i];
  }
}

// Solve A^T y = rhs with the factors of A (P A = L U  =>  A^T = U^T L^T P).
void lu_solve_transpose(int n, const double* A, const int* piv, double* y) {
  for (int i = 0; i < n; ++i) {
    double s = y[i];
    for (int j = 0; j < i; ++j) s -= A[(size_t)j * n + i] * y[j];
    y[i] = s / A[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int j = i + 1; j < n; ++j) s -= A[(size_t)j * n + i] * y[j];
    y[i] = s;
  }
  for (int k = n - 1; k >= 0; --k)
    if (piv[k] != k) std::swap(y[k], y[piv[k]]);
}

// L_i = R_i L R_i^T as a dense |S_i| x |S_i| block (Eq. 15).
void patch_matrix(const Prob& P, int l, const std::vector<long>& S, std::vector<double>& Li) {
  const int m = (int)S.size();
  Li.assign((size_t)m * m, 0.0);
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) Li[(size_t)a * m + b] = entry(P, l, S[a], S[b]);
}

// Positions in S_i of the DoFs that the restricted prolongation R~_i^T keeps: the pressure p_i and
// the d velocity DoFs on the same node (Sec. 3.1, definition of R~_i).
void center_positions(const Prob& P, int l, long node, const std::vector<long>& S, int* pos) {
  const long N = P.lev[l].N;
  for (int f = 0; f <= P.d; ++f) {
    long dof = (long)f * N + node;
    pos[f] = (int)(std::lower_bound(S.begin(), S.end(), dof) - S.begin());
  }
}

// Local correction of subdomain i: y = L_i^{-1} R_i r, returning the d+1 kept entries (Eq. 15).
bool patch_correction(const Prob& P, int l, long node, const double* r, double* out) {
  std::vector<long> S;
  patch_dofs(P, l, node, S);
  std::vector<double> Li;
  patch_matrix(P, l, S, Li);
  const int m = (int)S.size();
  std::vector<int> piv(m);
  if (!lu_factor(m, Li.data(), piv.data())) return false;
  std::vector<double> y(m);
  for (int a = 0; a < m; ++a) y[a] = r[S[a]];
  lu_solve(m, Li.data(), piv.data(), y.data());
  int pos[4];
  center_positions(P, l, node, S, pos);
  for (int f = 0; f <= P.d; ++f) out[f] = y[pos[f]];
  return true;
}

// The d+1 kept rows of L_i^{-1} (cache_inverse, Sec. 3.1.2): row c of A^{-1} is the solution of
// A^T z = e_c. Stored as (d+1) x |S_i|.
bool inverse_rows(const Prob& P, int l, long node, std::vector<long>& S, std::vector<double>& Z) {
  patch_dofs(P, l, node, S);
  std::vector<double> Li;
  patch_matrix(P, l, S, Li);
  const int m = (int)S.size();
  std::vector<int> piv(m);
  if (!lu_factor(m, Li.data(), piv.data())) return false;
  int pos[4];
  center_positions(P, l, node, S, pos);
  Z.assign((size_t)(P.d + 1) * m, 0.0);
  for (int f = 0; f <= P.d; ++f) {
    std::vector<double> e(m, 0.0);
    e[pos[f]] = 1.0;
    lu_solve_transpose(m, Li.data(), piv.data(), e.data());
    std::copy(e.begin(), e.end(), Z.begin() + (size_t)f * m);
  }
  return true;
}

bool build_Z(Prob& P, int l) {
  Level& L = P.lev[l];
  if (L.has_Z) return true;
  const int nf = P.d + 1;
  L.Zcount.assign(L.N, 0);
  L.Zoff.assign(L.N + 1, 0);
  for (long i = 0; i < L.N; ++i) {
    std::vector<long> S;
    patch_dofs(P, l, i, S);
    L.Zcount[i] = (int)S.size();
    L.Zoff[i + 1] = L.Zoff[i] + (long)nf * S.size();
  }
  L.Z.assign(L.Zoff[L.N], 0.0);
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < L.N; ++i) {
    std::vector<long> S;
    std::vector<double> Z;
    if (!inverse_rows(P, l, i, S, Z)) {
#pragma omp atomic write
      ok = false;
      continue;
    }
    std::copy(Z.begin(), Z.end(), L.Z.begin() + L.Zoff[i]);
  }
  if (!ok) return false;
  L.has_Z = true;
  return true;
}

// One application of Eq. (14) with the smoother of Eq. (15):
//   x <- x + sum_i R~_i^T omega L_i^{-1} R_i (b - L x),  omega_i = omega * I.
// mode 0: every patch factorises L_i and solves (ground truth). mode 1: cache_inverse rows.
// Every patch reads the same residual; each DoF is written by exactly one patch.
int sweep(Prob& P, int l, double* x, const double* b, double omega, int mode) {
  const Level& L0 = P.lev[l];
  const int nf = P.d + 1;
  const long N = L0.N, nd = (long)nf * N;
  std::vector<double> r(nd);
  residual(P, l, x, b, r.data());
  if (mode == 1 && !build_Z(P, l)) return ERR_SINGULAR;
  const Level& L = P.lev[l];
  std::vector<double> upd(nd, 0.0);
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < N; ++i) {
    double y[4];
    if (mode == 0) {
      if (!patch_correction(P, l, i, r.data(), y)) {
#pragma omp atomic write
        ok = false;
        continue;
      }
    } else {
      std::vector<long> S;
      patch_dofs(P, l, i, S);
      const double* Z = &L.Z[L.Zoff[i]];
      const int m = L.Zcount[i];
      for (int f = 0; f < nf; ++f) {
        double s = 0;
        for (int a = 0; a < m; ++a) s += Z[(size_t)f * m + a] * r[S[a]];
        y[f] = s;
      }
    }
    for (int f = 0; f < nf; ++f) upd[f * N + i] = omega * y[f];
  }
  if (!ok) return ERR_SINGULAR;
  for (long k = 0; k < nd; ++k) x[k] += upd[k];
  return ERR_OK;
}

// ---------------------------------------------------------------------------------------------
// Grid transfers (Sec. 3, Eq. 13). On one process T is the identity and R = R~. The prolongation is
// the Q1 interpolation from the coarse grid of Algorithm 1 (uniform case: every cell coarsened) to
// the fine grid, applied to each field; restriction is its transpose, R = P^T.
// ---------------------------------------------------------------------------------------------
void prolong_add(const Prob& P, int lf, const double* xc, double* xf) {
  const Level& F = P.lev[lf];
  const Level& C = P.lev[lf - 1];
  const int d = P.d, nf = d + 1;
  for (long i = 0; i < F.N; ++i) {
    int c[3];
    node_coords(d, F.n, i, c);
    int ncomb = 1 << d;
    for (int t = 0; t < ncomb; ++t) {
      int cc[3] = {0, 0, 0};
      double w = 1;
      bool valid = true;
      for (int k = 0; k < d; ++k) {
        int bit = (t >> k) & 1;
        if (c[k] % 2 == 0) {
          if (bit) valid = false;
          cc[k] = c[k] / 2;
        } else {
          cc[k] = (c[k] - 1) / 2 + bit;
          w *= 0.5;
        }
      }
      if (!valid) continue;
      long j = node_index(d, C.n, cc);
      for (int f = 0; f < nf; ++f) xf[f * F.N + i] += w * xc[f * C.N + j];
    }
  }
}

void restrict_vec(const Prob& P, int lf, const double* rf, double* bc) {
  const Level& F = P.lev[lf];
  const Level& C = P.lev[lf - 1];
  const int d = P.d, nf = d + 1;
  for (long k = 0; k < (long)nf * C.N; ++k) bc[k] = 0;
  for (long i = 0; i < F.N; ++i) {
    int c[3];
    node_coords(d, F.n, i, c);
    int ncomb = 1 << d;
    for (int t = 0; t < ncomb; ++t) {
      int cc[3] = {0, 0, 0};
      double w = 1;
      bool valid = true;
      for (int k = 0; k < d; ++k) {
        int bit = (t >> k) & 1;
        if (c[k] % 2 == 0) {
          if (bit) valid = false;
          cc[k] = c[k] / 2;
        } else {
          cc[k] = (c[k] - 1) / 2 + bit;
          w *= 0.5;
        }
      }
      if (!valid) continue;
      long j = node_index(d, C.n, cc);
      for (int f = 0; f < nf; ++f) bc[f * C.N + j] += w * rf[f * F.N + i];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Coarsest grid: direct solve (Sec. 3). When the operator has the constant-pressure null space
// (alpha = 1 everywhere, or no obstacle, and every wall Dirichlet) the system is bordered with the
// constraint sum(p) = 0 (reading; the paper does not discuss the null space).
// ---------------------------------------------------------------------------------------------
bool pressure_nullspace(const Prob& P) {
  bool all_dir = true;
  for (int k = 0; k < 2 * P.d; ++k)
    if (P.bc[k] == BC_NEUMANN) all_dir = false;
  return all_dir && (P.balls.empty() || P.alpha_f == 1.0);
}

bool coarse_factor(Prob& P) {
  if (P.cdim) return P.coarse_ok;  // factorised once, on first use
  const Level& L = P.lev[0];
  const int nf = P.d + 1;
  const long nd = (long)nf * L.N;
  P.bordered = pressure_nullspace(P);
  const int m = (int)nd + (P.bordered ? 1 : 0);
  P.cdim = m;
  P.clu.assign((size_t)m * m, 0.0);
  for (long a = 0; a < nd; ++a)
    for (long b = 0; b < nd; ++b) P.clu[(size_t)a * m + b] = entry(P, 0, a, b);
  if (P.bordered)
    for (long a = P.d * L.N; a < nd; ++a) {
      P.clu[(size_t)a * m + nd] = 1.0;
      P.clu[(size_t)nd * m + a] = 1.0;
    }
  P.cpiv.assign(m, 0);
  P.coarse_ok = lu_factor(m, P.clu.data(), P.cpiv.data());
  return P.coarse_ok;
}

void coarse_solve(const Prob& P, const double* b, double* x) {
  const long nd = (long)(P.d + 1) * P.lev[0].N;
  std::vector<double> y(P.cdim, 0.0);
  for (long k = 0; k < nd; ++k) y[k] = b[k];
  lu_solve(P.cdim, P.clu.data(), P.cpiv.data(), y.data());
  for (long k = 0; k < nd; ++k) x[k] = y[k];
}

// V-cycle (Sec. 3 and the solver settings of Sec. 4): nu1 pre-smoothing sweeps, restriction of the
// residual, recursive coarse correction from a zero initial guess, prolongation, nu2 post sweeps.
int vcycle(Prob& P, int l, double* x, const double* b, int nu1, int nu2, double omega, int mode) {
  if (l == 0) {
    coarse_solve(P, b, x);
    return ERR_OK;
  }
  const int nf = P.d + 1;
  const long nd = (long)nf * P.lev[l].N, ndc = (long)nf * P.lev[l - 1].N;
  for (int s = 0; s < nu1; ++s) {
    int e = sweep(P, l, x, b, omega, mode);
    if (e) return e;
  }
  std::vector<double> r(nd), bc(ndc), xc(ndc, 0.0);
  residual(P, l, x, b, r.data());
  restrict_vec(P, l, r.data(), bc.data());
  int e = vcycle(P, l - 1, xc.data(), bc.data(), nu1, nu2, omega, mode);
  if (e) return e;
  prolong_add(P, l, xc.data(), x);
  for (int s = 0; s < nu2; ++s) {
    e = sweep(P, l, x, b, omega, mode);
    if (e) return e;
  }
  return ERR_OK;
}

double norm2(const double* v, long n) {
  double s = 0;
  for (long i = 0; i < n; ++i) s += v[i] * v[i];
  return std::sqrt(s);
}

}  // namespace

// =============================================================================================
// C interface used by the Python wrapper (ctypes).
// =============================================================================================
extern "C" {

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void* orc_create(int d, int n, int nlev, int q, double eta, double alpha_f, double beta, int nballs,
                 const double* balls, const int* bc, double ubar, int force, int immersed) {
  if (d < 2 || d > 3 || n < 1 || nlev < 1 || (n >> (nlev - 1)) < 1 || ((n >> (nlev - 1)) << (nlev - 1)) != n)
    return nullptr;
  if (immersed != 0 && immersed != 1) return nullptr;
  Prob* P = new Prob;
  P->immersed = immersed;
  P->d = d;
  P->n = n;
  P->nlev = nlev;
  P->q = q;
  P->eta = eta;
  P->alpha_f = alpha_f;
  P->beta = beta;
  P->ubar = ubar;
  P->force = force;
  for (int k = 0; k < 6; ++k) P->bc[k] = bc ? bc[k] : 0;
  for (int i = 0; i < nballs; ++i) {
    Ball b;
    b.c[0] = balls[4 * i + 0];
    b.c[1] = balls[4 * i + 1];
    b.c[2] = balls[4 * i + 2];
    b.r = balls[4 * i + 3];
    P->balls.push_back(b);
  }
  P->lev.resize(nlev);
  for (int l = 0; l < nlev; ++l) {
    Level& L = P->lev[l];
    L.n = n >> (nlev - 1 - l);
    L.h = 1.0 / L.n;
    L.qd = q + (nlev - 1 - l);
    L.N = 1;
    for (int k = 0; k < d; ++k) L.N *= (L.n + 1);
    assemble_level(*P, l);
  }
  P->bordered = pressure_nullspace(*P);
  return P;
}

void orc_destroy(void* h) { delete static_cast<Prob*>(h); }

long orc_nnodes(void* h, int l) { return static_cast<Prob*>(h)->lev[l].N; }
int orc_ncells_axis(void* h, int l) { return static_cast<Prob*>(h)->lev[l].n; }
int orc_coarse_ok(void* h) { return coarse_factor(*static_cast<Prob*>(h)) ? 1 : 0; }
int orc_bordered(void* h) { return static_cast<Prob*>(h)->bordered ? 1 : 0; }

void orc_cell_kinds(void* h, int l, signed char* out) {
  const Level& L = static_cast<Prob*>(h)->lev[l];
  std::copy(L.kind.begin(), L.kind.end(), out);
}

// Element matrix of one cell, (2^d (d+1))^2 row-major, index f*2^d + a.
void orc_element_matrix(void* h, int l, long cell, double* out) {
  Prob* P = static_cast<Prob*>(h);
  std::vector<double> Le;
  element_matrix(*P, P->lev[l], cell, Le, nullptr);
  std::copy(Le.begin(), Le.end(), out);
}

// Immersed-boundary quadrature of one cell: up to max points as [x (d), w, n (d)] (2D: arcs, 3D:
// sphere pieces); returns the number of points (which may exceed max; then only max are written).
long orc_arc_points(void* h, int l, long cell, double* out, long max) {
  Prob* P = static_cast<Prob*>(h);
  const Level& L = P->lev[l];
  const int d = P->d, stride = 2 * d + 1;
  double lo[3];
  int ci[3];
  cell_lo(*P, L, cell, lo, ci);
  std::vector<APt> ap;
  if (d == 2)
    arc_points(*P, lo, L.h, ap);
  else
    sphere_points(*P, lo, L.h, ap);
  for (long i = 0; i < (long)ap.size() && i < max; ++i) {
    for (int k = 0; k < d; ++k) out[stride * i + k] = ap[i].x[k];
    out[stride * i + d] = ap[i].w;
    for (int k = 0; k < d; ++k) out[stride * i + d + 1 + k] = ap[i].n[k];
  }
  return (long)ap.size();
}

// Quadrature statistics of one cell: [sum w*alpha, sum w*[alpha==1], number of points,
// number of leaves still cut at depth q, their total volume].
void orc_cell_quadrature(void* h, int l, long cell, double* out) {
  Prob* P = static_cast<Prob*>(h);
  const Level& L = P->lev[l];
  double lo[3];
  int ci[3];
  cell_lo(*P, L, cell, lo, ci);
  std::vector<QPt> pts;
  long cl = 0;
  double cv = 0;
  tree_points(*P, lo, L.h, 0, L.qd, pts, &cl, &cv);
  double sa = 0, sp = 0;
  for (const QPt& q : pts) {
    sa += q.w * q.alpha;
    if (q.alpha == 1.0) sp += q.w;
  }
  out[0] = sa;
  out[1] = sp;
  out[2] = (double)pts.size();
  out[3] = (double)cl;
  out[4] = cv;
}

// Global right-hand side b = (f, g) of Eq. (12) on level l.
void orc_rhs(void* h, int l, double* b) {
  Prob* P = static_cast<Prob*>(h);
  const Level& L = P->lev[l];
  const int d = P->d, nn = 1 << d, nf = d + 1;
  long ncell = 1;
  for (int k = 0; k < d; ++k) ncell *= L.n;
  std::vector<double> Fall((size_t)ncell * nn * nf);
#pragma omp parallel for schedule(dynamic, 64)
  for (long c = 0; c < ncell; ++c) {
    double lo[3];
    int ci[3];
    cell_lo(*P, L, c, lo, ci);
    std::vector<QPt> pts;
    tree_points(*P, lo, L.h, 0, L.qd, pts, nullptr, nullptr);
    element_rhs(*P, L, c, pts, &Fall[(size_t)c * nn * nf]);
  }
  for (long k = 0; k < (long)nf * L.N; ++k) b[k] = 0;
  for (long c = 0; c < ncell; ++c) {
    double lo[3];
    int ci[3];
    cell_lo(*P, L, c, lo, ci);
    for (int a = 0; a < nn; ++a) {
      long na = cell_node(d, L.n, ci, a);
      for (int f = 0; f < nf; ++f) b[f * L.N + na] += Fall[(size_t)c * nn * nf + f * nn + a];
    }
  }
}

void orc_matvec(void* h, int l, const double* x, double* y) { matvec(*static_cast<Prob*>(h), l, x, y); }

// y = |L| x (used by tests to bound rounding errors of residuals componentwise).
void orc_abs_matvec(void* h, int l, const double* x, double* y) { matvec(*static_cast<Prob*>(h), l, x, y, true); }

void orc_residual(void* h, int l, const double* x, const double* b, double* r) {
  residual(*static_cast<Prob*>(h), l, x, b, r);
}

// Level operator as COO triplets over the structural pattern (all in-grid stencil couplings,
// including numerical zeros). If rows == NULL only the count is returned.
long orc_coo(void* h, int l, long* rows, long* cols, double* vals) {
  Prob* P = static_cast<Prob*>(h);
  const Level& L = P->lev[l];
  const int d = P->d, nf = d + 1, no = nstencil(d);
  long cnt = 0;
  for (long i = 0; i < L.N; ++i) {
    int c[3];
    node_coords(d, L.n, i, c);
    for (int o = 0; o < no; ++o) {
      int cc[3] = {0, 0, 0};
      bool in = true;
      int t = o;
      for (int k = 0; k < d; ++k) {
        cc[k] = c[k] + (t % 3) - 1;
        t /= 3;
        if (cc[k] < 0 || cc[k] > L.n) in = false;
      }
      if (!in) continue;
      long j = node_index(d, L.n, cc);
      for (int f = 0; f < nf; ++f)
        for (int g = 0; g < nf; ++g) {
          if (rows) {
            rows[cnt] = (long)f * L.N + i;
            cols[cnt] = (long)g * L.N + j;
            vals[cnt] = L.st[st_index(d, i, f, o, g)];
          }
          ++cnt;
        }
    }
  }
  return cnt;
}

int orc_patch_dofs(void* h, int l, long node, long* out) {
  std::vector<long> S;
  patch_dofs(*static_cast<Prob*>(h), l, node, S);
  if (out) std::copy(S.begin(), S.end(), out);
  return (int)S.size();
}

int orc_patch_matrix(void* h, int l, long node, double* out) {
  Prob* P = static_cast<Prob*>(h);
  std::vector<long> S;
  patch_dofs(*P, l, node, S);
  std::vector<double> Li;
  patch_matrix(*P, l, S, Li);
  std::copy(Li.begin(), Li.end(), out);
  return (int)S.size();
}

int orc_inverse_rows(void* h, int l, long node, double* out) {
  Prob* P = static_cast<Prob*>(h);
  std::vector<long> S;
  std::vector<double> Z;
  if (!inverse_rows(*P, l, node, S, Z)) return ERR_SINGULAR;
  std::copy(Z.begin(), Z.end(), out);
  return (int)S.size();
}

int orc_smooth(void* h, int l, double* x, const double* b, int sweeps, double omega, int mode) {
  Prob* P = static_cast<Prob*>(h);
  for (int s = 0; s < sweeps; ++s) {
    int e = sweep(*P, l, x, b, omega, mode);
    if (e) return e;
  }
  return ERR_OK;
}

// One sweep evaluated only at the listed nodes: out[k*(d+1)+f] = x_new[f, nodes[k]].
int orc_smooth_nodes(void* h, int l, const double* x, const double* b, double omega, long cnt,
                     const long* nodes, double* out) {
  Prob* P = static_cast<Prob*>(h);
  const int nf = P->d + 1;
  const long N = P->lev[l].N;
  std::vector<double> r((size_t)nf * N);
  residual(*P, l, x, b, r.data());
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 16)
  for (long k = 0; k < cnt; ++k) {
    double y[4];
    if (!patch_correction(*P, l, nodes[k], r.data(), y)) {
#pragma omp atomic write
      ok = false;
      continue;
    }
    for (int f = 0; f < nf; ++f) out[k * nf + f] = x[f * N + nodes[k]] + omega * y[f];
  }
  return ok ? ERR_OK : ERR_SINGULAR;
}

// Patch corrections y (the d+1 kept entries of L_i^{-1} R_i r) for listed nodes and a given r.
int orc_patch_corrections(void* h, int l, const double* r, long cnt, const long* nodes, double* out) {
  Prob* P = static_cast<Prob*>(h);
  const int nf = P->d + 1;
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 16)
  for (long k = 0; k < cnt; ++k) {
    double y[4];
    if (!patch_correction(*P, l, nodes[k], r, y)) {
#pragma omp atomic write
      ok = false;
      continue;
    }
    for (int f = 0; f < nf; ++f) out[k * nf + f] = y[f];
  }
  return ok ? ERR_OK : ERR_SINGULAR;
}

void orc_restrict(void* h, int lf, const double* rf, double* bc) { restrict_vec(*static_cast<Prob*>(h), lf, rf, bc); }

void orc_prolong_add(void* h, int lf, const double* xc, double* xf) {
  prolong_add(*static_cast<Prob*>(h), lf, xc, xf);
}

int orc_coarse_solve(void* h, const double* b, double* x) {
  Prob* P = static_cast<Prob*>(h);
  if (!coarse_factor(*P)) return ERR_SINGULAR;
  coarse_solve(*P, b, x);
  return ERR_OK;
}

int orc_vcycle(void* h, double* x, const double* b, int nu1, int nu2, double omega, int mode) {
  Prob* P = static_cast<Prob*>(h);
  if (!coarse_factor(*P)) return ERR_SINGULAR;
  return vcycle(*P, P->nlev - 1, x, b, nu1, nu2, omega, mode);
}

// Standalone GMG (Sec. 4): V-cycles until ||b - L x||_2 <= rtol * ||b - L x0||_2 or max_iter cycles.
// hist (optional, max_iter+1 entries) receives the residual norms.
int orc_solve(void* h, double* x, const double* b, double rtol, int max_iter, int nu1, int nu2, double omega,
              int mode, int* iters, double* relres, double* hist) {
  Prob* P = static_cast<Prob*>(h);
  if (!coarse_factor(*P)) return ERR_SINGULAR;
  const int l = P->nlev - 1;
  const long nd = (long)(P->d + 1) * P->lev[l].N;
  std::vector<double> r(nd);
  residual(*P, l, x, b, r.data());
  const double r0 = norm2(r.data(), nd);
  if (hist) hist[0] = r0;
  *iters = 0;
  *relres = 0.0;
  if (r0 == 0.0) return ERR_OK;
  for (int it = 1; it <= max_iter; ++it) {
    int e = vcycle(*P, l, x, b, nu1, nu2, omega, mode);
    if (e) return e;
    residual(*P, l, x, b, r.data());
    double rn = norm2(r.data(), nd);
    if (hist) hist[it] = rn;
    *iters = it;
    *relres = rn / r0;
    if (rn <= rtol * r0) return ERR_OK;
  }
  return ERR_NOCONV;
}

}  // extern "C"
