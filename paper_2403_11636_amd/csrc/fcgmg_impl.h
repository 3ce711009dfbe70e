// Internal declarations of the fcgmg library: level data, operator constants, geometry and the
// element integrals of the finite cell Stokes operator (Saberi & Vogel, Eq. 5-12).
//
// The element routines are __host__ __device__: the host planner evaluates the uncut reference
// cells and the Nitsche face matrices once per level; the kernels integrate cut cells (setup, and
// on the fly in the immersed-boundary cache_none blocks) and the right-hand side.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "fcgmg.h"

namespace fcg {

// ------------------------------------------------------------------------------------------------
// Patch geometry per dimension. A vertex patch (subdomain S_i of Eq. 15) of node i holds the d
// velocity components of the 5^d nodes within max-norm distance 2 and the pressures of the 3^d
// nodes within distance 1; its block L_i is assembled from the 6^d cells around i.
// Column layout of a patch vector (and of the cache_inverse rows Z_i): component-major velocity
// [c][5^d window, x fastest] followed by the 3^d pressure window; out-of-grid entries are zero.
// ------------------------------------------------------------------------------------------------
template <int D>
struct PT {
  static constexpr int NN = 1 << D;                   // nodes per cell
  static constexpr int NV = D == 2 ? 25 : 125;        // velocity window nodes (5^d)
  static constexpr int NP = D == 2 ? 9 : 27;          // pressure window nodes (3^d)
  static constexpr int NW = D == 2 ? 36 : 216;        // window cells (6^d)
  static constexpr int BW = D == 2 ? 6 : 31;          // half bandwidth of K_i (lexicographic)
  static constexpr int NB = BW + 1;                   // band storage width
  static constexpr int ZS = D * NV + NP;              // |S_i| of an interior patch: 59 / 402
  static constexpr int ZSP = (ZS + 63) / 64 * 64;     // padded row length: 64 / 448
  static constexpr int NEL = (D + 1) * NN * NN;       // stored entries of one cut cell (K, B_c)
  static constexpr int THREADS = D == 2 ? 64 : 256;   // block size of the patch kernels
  static constexpr int NST = D == 2 ? 9 : 27;         // node stencil offsets (3^d)
  static constexpr int NSTEN = (2 * D + 2) * NST;     // stored stencil of one node (see node_op)
};

// Position of coefficient j (0 K, 1..D B_c, D+1..2D B_c^T, 2D+1 C) of stencil offset o in a stored
// node row (Level::nsten): 2D coefficient-major (j 9 + o), 3D offset-major (o 8 + j), so that a 3D
// offset's eight coefficients lie together in 64 bytes and load as wide vectors.
template <int D>
__host__ __device__ constexpr int sten_index(int j, int o) {
  return D == 2 ? j * PT<2>::NST + o : o * (2 * D + 2) + j;
}

// Layout of the level constants as the residual kernels stage them into LDS: the reference
// matrices of a physical uncut cell (a fictitious uncut cell is alpha_f times them), C, the Nitsche
// face matrices of the 2d faces and the node stencils of uniform neighbourhoods.
template <int D>
struct RefLayout {
  static constexpr int NN2 = (1 << D) * (1 << D);
  static constexpr int NS = D == 2 ? 9 : 27;             // stencil offsets
  static constexpr int oK = 0;                           // K            [NN2]
  static constexpr int oB = NN2;                         // B_c          [D][NN2]
  static constexpr int oC = NN2 * (1 + D);               // C            [NN2]
  static constexpr int oFK = NN2 * (2 + D);              // FK_face      [2D][NN2]
  static constexpr int oFB = NN2 * (2 + 3 * D);          // FB_face      [2D][NN2]
  static constexpr int oSK = NN2 * (2 + 5 * D);          // SK           [kind][NS]
  static constexpr int oSB = oSK + 2 * NS;               // SB           [kind][D][NS]
  static constexpr int oST = oSB + 2 * D * NS;           // ST           [kind][D][NS]
  static constexpr int oSC = oST + 2 * D * NS;           // SC           [NS]
  static constexpr int TOT = oSC + NS;
};

// Per-level operator constants (device resident, read through uniform loads).
struct OpConsts {
  double K[2][64];      // [0 physical, 1 fictitious] eta*alpha*int grad phi_a . grad phi_b
  double B[2][3][64];   // [kind][c]: -int alpha d_c phi_a phi_b  (a: velocity node, b: pressure)
  double C[64];         // -(1/eta) (M_ab - m_a m_b / |K|)
  double FK[6][64];     // Nitsche face matrix of face f (zero when the face is not Dirichlet)
  double FB[6][64];     // int_F phi_a n_k phi_b on face f (velocity component k = axis of f)
  int dirichlet[6];
  int n;                // cells per axis
  int immersed;         // 1: Nitsche terms on the obstacle arcs of cut cells (2D)
  double h, lam;
  // Assembled node stencils of a node whose 2^d cells are uncut, of one kind and away from the
  // walls, per kind, over the 3^d neighbour offsets: velocity-velocity (same component), velocity
  // row c / pressure column, pressure row / velocity column c, pressure-pressure.
  double SK[2][27];
  double SB[2][3][27];
  double ST[2][3][27];
  double SC[27];
  double pack[RefLayout<3>::TOT];  // the entries above in RefLayout<d> order
};

// Deepest space tree: quad_depth + n_levels - 1 may not exceed it.
constexpr int kMaxTreeDepth = 20;

struct Geom {
  const double* balls;  // nballs x 4 (centre, radius)
  int nballs;
  int q;                // space-tree depth of the level's cut cells
  double alpha_f;
};

struct Level {
  int n = 0;
  double h = 0;
  int qd = 0;                 // space-tree depth: quad_depth on the finest level, one more per coarser level
  int64_t N = 0, ncells = 0;
  int* cell_info = nullptr;   // -1 physical, -2 fictitious, >=0 index into cut_mats
  double* cut_mats = nullptr; // n_cut x NEL: K (NN x NN) then B_c (NN x NN) for c < d
  int64_t n_cut = 0, n_fict = 0;
  // 2D: the patch blocks are factorised by dense LU with partial pivoting instead of the block
  // Cholesky, because their velocity blocks may be indefinite (immersed Nitsche terms, or the
  // alpha-free Nitsche terms of a Dirichlet face that crosses an obstacle)
  bool dense_lu = false;
  int* node_class = nullptr;  // >=0 regular class id, <0: -(irregular index)-1
  // Operator row of each node: -1 / -2 when its 2^d cells are uncut, all physical / all fictitious
  // and it is at least 2 nodes from every wall (the level's reference stencil applies), otherwise
  // the index of its assembled stencil in nsten: NSTEN doubles over the 3^d neighbour offsets o and
  // the coefficients j = 0 velocity-velocity (every component), 1..d velocity c / pressure, d+1..2d
  // pressure / velocity c, 2d+1 pressure-pressure, at sten_index<D>(j, o).
  int* node_op = nullptr;
  double* nsten = nullptr;
  int64_t n_nsten = 0;
  int* fused_extra = nullptr;  // 2D cache_inverse: extra workgroups of heavy tiles (plan_fused2)
  int n_fused_extra = 0;
  int fused_extra_cap = 0;     // ints allocated for fused_extra
  double* rm = nullptr;        // fcgmg_vcycle_multi workspace: kMaxRhs residuals
  double* xm = nullptr;        //   kMaxRhs iterates (coarse levels)
  double* bm = nullptr;        //   kMaxRhs right-hand sides (coarse levels)
  int fshape = -1;             // fused-sweep tile shape chosen by fcgmg_autotune, -1: default by size
  int64_t n_classes = 0, n_irr = 0, irr_cols = 0;
  int64_t n_zrows = 0;        // streamed row blocks (n_irr, fewer where wall patches share rows)
  int* irr_nodes = nullptr;   // centre node of each streamed (irregular) patch
  int* irr_zrow = nullptr;    // its row block in Zirr / Mirr
  int* zrow_nodes = nullptr;  // node whose block gives row block k
  int* class_rep = nullptr;   // representative node of each class
  double* Zcls = nullptr;     // cache_inverse: n_classes x (d+1) x ZSP
  double* Zirr = nullptr;     // cache_inverse: n_zrows x (d+1) x ZSP
  double* Mcls = nullptr;     // cache_matrix: n_classes x n_pattern
  double* Mirr = nullptr;     // cache_matrix: n_irr x n_pattern
  OpConsts* consts = nullptr; // device copy
  OpConsts consts_h;          // host copy
  double* r = nullptr;        // residual scratch, (d+1) N
  double* x = nullptr;        // V-cycle iterate (levels below the finest)
  double* b = nullptr;        // V-cycle right-hand side (levels below the finest)
  double* xalt = nullptr;     // second iterate buffer of the fused 2D sweep
  size_t cached_bytes = 0;
  // FP32 copies for the mixed-precision V-cycle (cache_inverse, FCGMG_PREC_MIXED): inverse rows and
  // stored stencils rounded from the FP64 set-up, and the level vectors of the FP32 cycle
  float* Zcls32 = nullptr;
  float* Zirr32 = nullptr;
  float* nsten32 = nullptr;
  float* r32 = nullptr;
  float* x32 = nullptr;
  float* b32 = nullptr;
  float* xalt32 = nullptr;
};

// One fused 2D sweep over one level (the kernel's arguments; a batched launch takes an array).
template <class T>
struct Fused2Job {
  const OpConsts* oc;
  const int* node_op;
  const T* nsten;
  const int* extra;       // extra parts of split tiles (plan_fused2), or null
  int n_extra;            // their count: workgroups 0 .. n_extra-1
  const int* node_class;
  const T* Zcls;
  const T* Zirr;
  const T* x_in;
  const T* b;
  T* x_out;
  const T* xc;            // coarse vector of mode 2
  T omega;
  int ntx, nty, mode;
  int block0;             // first workgroup of the job in a batched launch
};

// One fused residual + restriction (2D), fine level F to F-1.
template <class T>
struct RR2Job {
  const OpConsts* oc;
  const int* node_op;
  const T* nsten;
  const T* x;
  const T* b;
  T* bc;
  int ntx, nty;
  int block0;
};

// One dense matvec x = A b of a coarsest level in a batched launch (4 rows per workgroup).
struct DenseJob {
  const double* A;
  const double* b;
  double* x;
  int n;
  int block0;
};

// ||b - L x||^2 of one 2D problem in a batched launch: workgroups block0 .. block0 + nblocks - 1.
struct NormJob {
  const OpConsts* oc;
  const int* node_op;
  const double* nsten;
  const double* x;
  const double* b;
  int ntx, nty;
  int block0, nblocks;
};

// The level data a kernel of value type T reads and writes.
template <class T>
struct LV;
template <>
struct LV<double> {
  static const double* Zcls(const Level& L) { return L.Zcls; }
  static const double* Zirr(const Level& L) { return L.Zirr; }
  static const double* nsten(const Level& L) { return L.nsten; }
  static double* r(const Level& L) { return L.r; }
  static double* x(const Level& L) { return L.x; }
  static double* b(const Level& L) { return L.b; }
  static double* xalt(const Level& L) { return L.xalt; }
};
template <>
struct LV<float> {
  static const float* Zcls(const Level& L) { return L.Zcls32; }
  static const float* Zirr(const Level& L) { return L.Zirr32; }
  static const float* nsten(const Level& L) { return L.nsten32; }
  static float* r(const Level& L) { return L.r32; }
  static float* x(const Level& L) { return L.x32; }
  static float* b(const Level& L) { return L.b32; }
  static float* xalt(const Level& L) { return L.xalt32; }
};

struct Ctx {
  fcgmg_params prm{};
  std::vector<double> balls_h;
  double* balls = nullptr;
  std::vector<Level> lev;
  double* coarse_inv = nullptr;  // dense inverse of the coarsest operator (ndof x ndof)
  float* coarse_inv32 = nullptr; // its FP32 rounding (mixed precision)
  // FGMRES (solver == FCGMG_SOLVER_FGMRES): basis V (m+1 vectors), preconditioned Z (m), work w,
  // zero vector, inner-product partials and coefficients; all finest-level FP64
  double* kv = nullptr;
  double* kz = nullptr;
  double* kw = nullptr;
  double* kzero = nullptr;
  double* kpart = nullptr;
  double* kh = nullptr;
  double* kh_host = nullptr;     // pinned host copy of kh (coefficients h, h2 and y)
  int coarse_n = 0;
  bool bordered = false;
  double* red = nullptr;         // reduction scratch
  double* red_host = nullptr;    // pinned host word
  double* red_host_dev = nullptr; // its device address (the reduction's finishing kernel writes it)
  int* err = nullptr;            // device error flag: first failing patch node, or INT_MAX
  int* pattern = nullptr;        // cache_matrix sparse pattern (encoded entries)
  int n_pattern = 0;
  bool none_integrate = false;  // cache_none: assemble from element integrals, cut cells integrated per sweep
  bool multi_ready = false;     // fcgmg_vcycle_multi workspace allocated
  // 3D cache_inverse: a second stream on which the shared-class apply of a sweep runs beside the
  // streamed-patch apply (the two write disjoint nodes), forked from and joined to the caller's
  // stream by the two events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  size_t bytes = 0;
  std::vector<void*> allocs;
  // event profiler
  struct ProfRec {
    int kind, level;
    hipEvent_t start, stop;
  };
  bool prof = false;
  mutable std::vector<ProfRec> prof_pending;
  mutable std::vector<hipEvent_t> prof_pool;
  mutable std::vector<double> prof_ms;      // [kind * nlev + level]
  mutable std::vector<int64_t> prof_count;
  Geom geom(const Level& L) const { return Geom{balls, (int)balls_h.size() / 4, L.qd, prm.alpha_fict}; }
  Geom geom_host() const { return Geom{balls_h.data(), (int)balls_h.size() / 4, prm.quad_depth, prm.alpha_fict}; }
};

// ------------------------------------------------------------------------------------------------
// Geometry (Eq. 7): alpha = 1 outside every ball, alpha_f inside or on a ball.
// ------------------------------------------------------------------------------------------------
template <int D>
__host__ __device__ inline double alpha_at(const Geom& g, const double* x) {
  for (int i = 0; i < g.nballs; ++i) {
    const double* b = g.balls + 4 * i;
    double s = 0;
    for (int k = 0; k < D; ++k) {
      double t = x[k] - b[k];
      s += t * t;
    }
    if (s <= b[3] * b[3]) return g.alpha_f;
  }
  return 1.0;
}

// Box [lo, lo+s]^D: 0 physical, 1 fictitious (inside a ball), 2 cut.
template <int D>
__host__ __device__ inline int box_kind(const Geom& g, const double* lo, double s) {
  bool cut = false;
  for (int i = 0; i < g.nballs; ++i) {
    const double* b = g.balls + 4 * i;
    double dmin2 = 0, dmax2 = 0;
    for (int k = 0; k < D; ++k) {
      double a = lo[k] - b[k], e = lo[k] + s - b[k];
      double m = a > 0 ? a : (e < 0 ? -e : 0.0);
      dmin2 += m * m;
      double M = fmax(fabs(a), fabs(e));
      dmax2 += M * M;
    }
    double r2 = b[3] * b[3];
    if (dmax2 <= r2) return 1;
    if (dmin2 < r2) cut = true;
  }
  return cut ? 2 : 0;
}

// Q1 basis of a cell (lower corner lo, size h) at x: values and physical gradients.
template <int D>
__host__ __device__ inline void q1(const double* lo, double h, const double* x, double* phi, double (*gr)[3]) {
  double t[3], u[3];
  const double ih = 1.0 / h;
  for (int k = 0; k < D; ++k) {
    t[k] = (x[k] - lo[k]) * ih;
    u[k] = 1.0 - t[k];
  }
  for (int a = 0; a < (1 << D); ++a) {
    double f[3];
    for (int k = 0; k < D; ++k) f[k] = ((a >> k) & 1) ? t[k] : u[k];
    double v = f[0] * f[1];
    if (D == 3) v *= f[2];
    phi[a] = v;
    for (int j = 0; j < D; ++j) {
      double gj = ((a >> j) & 1) ? ih : -ih;
      for (int k = 0; k < D; ++k)
        if (k != j) gj *= f[k];
      gr[a][j] = gj;
    }
  }
}

// Two-point Gauss abscissae on [0,1].
#define FCG_GA (0.21132486540518711775)
#define FCG_GB (0.78867513459481288225)

// Space-tree quadrature of one cell: visits every Gauss point (x, w, alpha) of the leaves. A box is
// split into its 2^D children while it is cut and shallower than q; every leaf gets the 2^D-point
// Gauss rule with alpha evaluated at each point. Iterative depth-first traversal (no recursion).
template <int D, class F>
__host__ __device__ inline void tree_quadrature(const Geom& g, const double* lo0, double h, F&& visit) {
  int child[kMaxTreeDepth + 1];
  double lo[kMaxTreeDepth + 1][3];
  for (int k = 0; k < 3; ++k) lo[0][k] = k < D ? lo0[k] : 0.0;
  int t = 0;
  child[0] = 0;
  for (;;) {
    const double s = h / (double)(1 << t);
    bool descend = false;
    if (t < g.q && t < kMaxTreeDepth) descend = box_kind<D>(g, lo[t], s) == 2;
    if (descend) {
      ++t;
      child[t] = 0;
      for (int k = 0; k < D; ++k) lo[t][k] = lo[t - 1][k];
      continue;
    }
    const double w = D == 2 ? 0.25 * s * s : 0.125 * s * s * s;
    for (int p = 0; p < (1 << D); ++p) {
      double x[3] = {0, 0, 0};
      for (int k = 0; k < D; ++k) x[k] = lo[t][k] + s * (((p >> k) & 1) ? FCG_GB : FCG_GA);
      visit(x, w, alpha_at<D>(g, x));
    }
    // advance to the next sibling, climbing while the current box was the last child
    while (t > 0 && child[t] == (1 << D) - 1) --t;
    if (t == 0) break;
    ++child[t];
    const double sp = h / (double)(1 << (t - 1));
    for (int k = 0; k < D; ++k) lo[t][k] = lo[t - 1][k] + (((child[t] >> k) & 1) ? 0.5 * sp : 0.0);
  }
}

// Immersed boundary (2D): Gauss points on the arcs of the obstacle circles inside the cell box
// [lo, lo + h]^2, the obstacle surfaces taken as part of Gamma_D in Eq. 5. Each circle is split at
// its crossings with the four lines of the box; a piece whose middle lies in the closed box is cut
// into ceil(width / (pi/8)) equal angular parts, each with the 6-point Gauss-Legendre rule in the
// angle. visit(x, w, nrm): point, weight (ds = r dtheta), unit normal pointing into the obstacle.
template <class F>
__host__ __device__ inline void arc_quadrature2(const Geom& g, const double* lo, double h, F&& visit) {
  const double gx[3] = {0.2386191860831969086305017, 0.6612093864662645136613996, 0.9324695142031520278123016};
  const double gw[3] = {0.4679139345726910473898703, 0.3607615730481386075698335, 0.1713244923791703450402961};
  const double two_pi = 6.283185307179586476925287;
  for (int i = 0; i < g.nballs; ++i) {
    const double* b = g.balls + 4 * i;
    const double r = b[3];
    double th[10];
    int nt = 0;
    th[nt++] = 0.0;
    th[nt++] = two_pi;
    for (int k = 0; k < 2; ++k)
      for (int s = 0; s < 2; ++s) {
        const double dist = lo[k] + s * h - b[k];
        if (fabs(dist) >= r) continue;
        const double other = sqrt(r * r - dist * dist);
        for (int sg = -1; sg <= 1; sg += 2) {
          double t = k == 0 ? atan2(sg * other, dist) : atan2(dist, sg * other);
          if (t < 0) t += two_pi;
          th[nt++] = t;
        }
      }
    for (int a = 1; a < nt; ++a)  // insertion sort of the break angles
      for (int c = a; c > 0 && th[c - 1] > th[c]; --c) {
        const double tmp = th[c];
        th[c] = th[c - 1];
        th[c - 1] = tmp;
      }
    for (int j = 0; j + 1 < nt; ++j) {
      const double t0 = th[j], t1 = th[j + 1];
      if (!(t1 > t0)) continue;
      const double tm = 0.5 * (t0 + t1);
      const double pm0 = b[0] + r * cos(tm), pm1 = b[1] + r * sin(tm);
      if (!(pm0 >= lo[0] && pm0 <= lo[0] + h && pm1 >= lo[1] && pm1 <= lo[1] + h)) continue;
      const int parts = (int)ceil((t1 - t0) / (0.125 * 3.141592653589793238462643));
      for (int p = 0; p < parts; ++p) {
        const double ta = t0 + (t1 - t0) * p / parts, te = t0 + (t1 - t0) * (p + 1) / parts;
        const double mid = 0.5 * (ta + te), half = 0.5 * (te - ta);
        for (int q = 0; q < 6; ++q) {
          const double xi = q < 3 ? -gx[2 - q] : gx[q - 3];
          const double wq = q < 3 ? gw[2 - q] : gw[q - 3];
          const double t = mid + half * xi;
          const double ct = cos(t), st = sin(t);
          const double x[3] = {b[0] + r * ct, b[1] + r * st, 0.0};
          const double nrm[2] = {-ct, -st};
          visit(x, wq * half * r, nrm);
        }
      }
    }
  }
}

// Immersed boundary (3D): Gauss points on the pieces of the obstacle spheres inside the cell box
// [lo, lo + h]^3, the obstacle surfaces taken as part of Gamma_D in Eq. 5. A sphere point is
// c + r (sin th cos ph, sin th sin ph, cos th), area element r^2 sin th dth dph. The polar range
// (cos th within the box's z-extent) is cut where the circle of latitude, radius sin th in the
// (x, y) plane, becomes tangent to one of the box's four x/y lines or passes one of their four
// corners; on each piece th = t0 + (t1 - t0)(3 s^2 - 2 s^3), which smooths the square-root ends, with
// s in ceil((t1 - t0) / (pi/8)) equal parts of 6 Gauss-Legendre points. At each th the circle is cut
// at its crossings with the four lines, and an arc whose middle lies in the closed rectangle is cut
// into ceil(width / (pi/8)) equal parts of 6 points in ph. visit(x, w, nrm): point, weight, unit
// normal pointing into the obstacle.
template <class F>
__host__ __device__ inline void sphere_quadrature3(const Geom& g, const double* lo, double h, F&& visit) {
  const double gx[3] = {0.2386191860831969086305017, 0.6612093864662645136613996, 0.9324695142031520278123016};
  const double gw[3] = {0.4679139345726910473898703, 0.3607615730481386075698335, 0.1713244923791703450402961};
  const double pi = 3.141592653589793238462643, two_pi = 6.283185307179586476925287, piece = 0.125 * pi;
  auto sort_small = [](double* v, int n) {
    for (int a = 1; a < n; ++a)
      for (int c = a; c > 0 && v[c - 1] > v[c]; --c) {
        const double tmp = v[c];
        v[c] = v[c - 1];
        v[c - 1] = tmp;
      }
  };
  for (int i = 0; i < g.nballs; ++i) {
    const double* bl = g.balls + 4 * i;
    const double r = bl[3];
    double lo_n[3], hi_n[3];  // box bounds relative to the centre, in radii
    for (int k = 0; k < 3; ++k) {
      lo_n[k] = (lo[k] - bl[k]) / r;
      hi_n[k] = (lo[k] + h - bl[k]) / r;
    }
    if (!(fmin(hi_n[2], 1.0) > fmax(lo_n[2], -1.0))) continue;
    const double th_a = hi_n[2] >= 1.0 ? 0.0 : acos(hi_n[2]);
    const double th_b = lo_n[2] <= -1.0 ? pi : acos(lo_n[2]);
    if (!(th_b > th_a)) continue;
    double cut[18];
    int nc = 0;
    cut[nc++] = th_a;
    cut[nc++] = th_b;
    // radius^2 of the circle of latitude at which it touches a line or passes a corner
    double rr[8];
    rr[0] = lo_n[0] * lo_n[0];
    rr[1] = hi_n[0] * hi_n[0];
    rr[2] = lo_n[1] * lo_n[1];
    rr[3] = hi_n[1] * hi_n[1];
    rr[4] = rr[0] + rr[2];
    rr[5] = rr[0] + rr[3];
    rr[6] = rr[1] + rr[2];
    rr[7] = rr[1] + rr[3];
    for (int k = 0; k < 8; ++k) {
      if (!(rr[k] >= 0.0 && rr[k] < 1.0)) continue;
      const double q = asin(sqrt(rr[k]));
      if (q > th_a && q < th_b) cut[nc++] = q;
      if (pi - q > th_a && pi - q < th_b) cut[nc++] = pi - q;
    }
    sort_small(cut, nc);
    for (int j = 0; j + 1 < nc; ++j) {
      const double t0 = cut[j], t1 = cut[j + 1];
      if (!(t1 > t0)) continue;
      const int tparts = (int)ceil((t1 - t0) / piece);
      for (int pt = 0; pt < tparts; ++pt) {
        const double s0 = (double)pt / tparts, s1 = (double)(pt + 1) / tparts;
        for (int qt = 0; qt < 6; ++qt) {
          const double xs = qt < 3 ? -gx[2 - qt] : gx[qt - 3];
          const double ws = qt < 3 ? gw[2 - qt] : gw[qt - 3];
          const double s = 0.5 * (s0 + s1) + 0.5 * (s1 - s0) * xs;
          const double th = t0 + (t1 - t0) * s * s * (3.0 - 2.0 * s);
          const double rho = sin(th), ct = cos(th);
          if (!(rho > 0.0)) continue;
          const double wth = 0.5 * (s1 - s0) * ws * (t1 - t0) * 6.0 * s * (1.0 - s) * rho;
          // the circle of radius rho against the lines x = lo_n[0], hi_n[0], y = lo_n[1], hi_n[1]
          double ph[10];
          int np = 0;
          ph[np++] = 0.0;
          ph[np++] = two_pi;
          for (int k = 0; k < 2; ++k) {
            const double v = (k ? hi_n[0] : lo_n[0]) / rho;
            if (fabs(v) < 1.0) {
              const double q = acos(v);
              ph[np++] = q;
              ph[np++] = two_pi - q;
            }
          }
          for (int k = 0; k < 2; ++k) {
            const double v = (k ? hi_n[1] : lo_n[1]) / rho;
            if (fabs(v) < 1.0) {
              const double q = asin(v);
              ph[np++] = q < 0.0 ? q + two_pi : q;
              ph[np++] = pi - q;
            }
          }
          sort_small(ph, np);
          for (int m = 0; m + 1 < np; ++m) {
            const double f0 = ph[m], f1 = ph[m + 1];
            if (!(f1 > f0)) continue;
            const double fm = 0.5 * (f0 + f1);
            const double xm = rho * cos(fm), ym = rho * sin(fm);
            if (!(xm >= lo_n[0] && xm <= hi_n[0] && ym >= lo_n[1] && ym <= hi_n[1])) continue;
            const int fparts = (int)ceil((f1 - f0) / piece);
            for (int pf = 0; pf < fparts; ++pf) {
              const double e0 = f0 + (f1 - f0) * pf / fparts, e1 = f0 + (f1 - f0) * (pf + 1) / fparts;
              for (int qf = 0; qf < 6; ++qf) {
                const double xf = qf < 3 ? -gx[2 - qf] : gx[qf - 3];
                const double wf = qf < 3 ? gw[2 - qf] : gw[qf - 3];
                const double phi = 0.5 * (e0 + e1) + 0.5 * (e1 - e0) * xf;
                const double u[3] = {rho * cos(phi), rho * sin(phi), ct};
                const double x[3] = {bl[0] + r * u[0], bl[1] + r * u[1], bl[2] + r * u[2]};
                const double nrm[3] = {-u[0], -u[1], -u[2]};
                visit(x, r * r * wth * 0.5 * (e1 - e0) * wf, nrm);
              }
            }
          }
        }
      }
    }
  }
}

// Entry e of a 3D cut cell's element data from the Nitsche forms at one boundary point (see
// nitsche_entry2): K[a][b] (e < 64) or B_c[a][b] (c = e / 64 - 1).
__host__ __device__ inline double nitsche_entry3(int e, double eta, double lam, double w, const double* nrm,
                                                 const double* phi, double (*gr)[3]) {
  const int blk = e / 64, ab = e % 64, a = ab / 8, b = ab % 8;
  if (blk == 0) {
    const double dna = nrm[0] * gr[a][0] + nrm[1] * gr[a][1] + nrm[2] * gr[a][2];
    const double dnb = nrm[0] * gr[b][0] + nrm[1] * gr[b][1] + nrm[2] * gr[b][2];
    return w * (-eta * phi[a] * dnb - eta * dna * phi[b] + lam * phi[a] * phi[b]);
  }
  return w * phi[a] * nrm[blk - 1] * phi[b];
}

// Entry e of a cell's element data from the Nitsche forms at one boundary point (weight w, normal
// nrm), the wall forms of Eq. 5 with w = 0: K[a][b] += -eta phi_a (n.grad phi_b) - eta (n.grad phi_a)
// phi_b + lambda phi_a phi_b; B_c[a][b] += phi_a n_c phi_b.
__host__ __device__ inline double nitsche_entry2(int e, double eta, double lam, double w, const double* nrm,
                                                 const double* phi, double (*gr)[3]) {
  const int blk = e / 16, ab = e % 16, a = ab / 4, b = ab % 4;
  if (blk == 0) {
    const double dna = nrm[0] * gr[a][0] + nrm[1] * gr[a][1], dnb = nrm[0] * gr[b][0] + nrm[1] * gr[b][1];
    return w * (-eta * phi[a] * dnb - eta * dna * phi[b] + lam * phi[a] * phi[b]);
  }
  return w * phi[a] * nrm[blk - 1] * phi[b];
}

// Entry e of a cell's alpha-weighted element data: e < NN*NN: K[a][b] = eta int alpha grad.grad;
// else B_c[a][b] = -int alpha d_c phi_a phi_b with c = e / (NN*NN) - 1.
template <int D>
__host__ __device__ inline double point_entry(int e, double eta, double wa, const double* phi, double (*gr)[3]) {
  constexpr int NN = 1 << D;
  const int blk = e / (NN * NN), ab = e % (NN * NN), a = ab / NN, b = ab % NN;
  if (blk == 0) {
    double s = 0;
    for (int k = 0; k < D; ++k) s += gr[a][k] * gr[b][k];
    return wa * eta * s;
  }
  return -wa * gr[a][blk - 1] * phi[b];
}

__host__ __device__ inline double gfun0(double t) { return t * t * (1 - t) * (1 - t); }
__host__ __device__ inline double gfun1(double t) { return 2 * t - 6 * t * t + 4 * t * t * t; }
__host__ __device__ inline double gfun2(double t) { return 2 - 12 * t + 12 * t * t; }
__host__ __device__ inline double gfun3(double t) { return -12 + 24 * t; }

// Body force of the manufactured solution u = curl psi (psi = prod g(x_k), g = t^2 (1-t)^2,
// 3D: u = (g g' g, -g' g g, 0)), p = sum x_k^3 - d/4:  f = -eta Lap u + grad p.
template <int D>
__host__ __device__ inline void body_force(int kind, double eta, const double* x, double* f) {
  f[0] = f[1] = f[2] = 0;
  if (kind != 1) return;
  const double X = x[0], Y = x[1];
  if (D == 2) {
    f[0] = -eta * (gfun2(X) * gfun1(Y) + gfun0(X) * gfun3(Y)) + 3 * X * X;
    f[1] = eta * (gfun3(X) * gfun0(Y) + gfun1(X) * gfun2(Y)) + 3 * Y * Y;
  } else {
    const double Z = x[2];
    f[0] = -eta * (gfun2(X) * gfun1(Y) * gfun0(Z) + gfun0(X) * gfun3(Y) * gfun0(Z) + gfun0(X) * gfun1(Y) * gfun2(Z)) +
           3 * X * X;
    f[1] = eta * (gfun3(X) * gfun0(Y) * gfun0(Z) + gfun1(X) * gfun2(Y) * gfun0(Z) + gfun1(X) * gfun0(Y) * gfun2(Z)) +
           3 * Y * Y;
    f[2] = 3 * Z * Z;
  }
}

// Dirichlet data on face (axis k, side s): zero, or the parabolic inflow of Eq. (16) (H = 1;
// product profile in 3D) pointing into the box.
template <int D>
__host__ __device__ inline void wall_data(int code, double ubar, int k, int s, const double* x, double* w) {
  w[0] = w[1] = w[2] = 0;
  if (code != FCGMG_BC_INFLOW) return;
  double prof = ubar;
  for (int j = 0; j < D; ++j)
    if (j != k) prof *= 4.0 * x[j] * (1.0 - x[j]);
  w[k] = s ? -prof : prof;
}

// ------------------------------------------------------------------------------------------------
// Kernel launchers (fcgmg_kernels.hip). All return hipError_t of the launch.
// ------------------------------------------------------------------------------------------------
template <int D> hipError_t k_classify_cells(const Ctx& c, Level& L, signed char* kinds, hipStream_t s);
template <int D> hipError_t k_cut_matrices(const Ctx& c, Level& L, const int* cut_cells, hipStream_t s);
template <int D> hipError_t k_node_stencils(const Ctx& c, const Level& L, const int* nodes, hipStream_t s);
template <int D> hipError_t k_rhs(const Ctx& c, const Level& L, double* b, hipStream_t s);
template <int D, class T>
hipError_t k_residual(const Ctx& c, const Level& L, const T* x, const T* b, T* r, hipStream_t s, int nrhs = 1,
                      int64_t sv = 0);
template <int D> hipError_t k_patch_inverse_rows(const Ctx& c, const Level& L, const int* nodes, int64_t count,
                                                 double* Z, hipStream_t s);
template <int D, class T>
hipError_t k_apply_regular(const Ctx& c, const Level& L, const T* r, T* x, hipStream_t s, int nrhs = 1,
                           int64_t sv = 0);
template <int D, class T>
hipError_t k_apply_irregular(const Ctx& c, const Level& L, const T* r, T* x, hipStream_t s);
constexpr int kMaxRhs = 8;  // right-hand sides of one stacked sweep (fcgmg_smooth_multi)
template <int D, class T>
hipError_t k_apply_irregular_multi(const Ctx& c, const Level& L, const T* r, T* x, int64_t nd, int nrhs,
                                   hipStream_t s);
template <class T>
hipError_t k_sweep_fused2(const Ctx& c, const Level& L, const T* x_in, const T* b, T* x_out, int mode, const T* xc,
                          hipStream_t s);
void plan_fused2(const Level& L, const std::vector<int>& node_class, std::vector<int>& extra);
int fused2_num_shapes();
void fused2_shape_dims(int k, int* tx, int* ty, int* nt, int* wpe);
// Batched launches over independent 2D problems (one tile shape for all jobs)
int batch_fused2_blocks(const Level& L);
Fused2Job<double> batch_fused2_job(const Ctx& c, const Level& L, const double* x_in, const double* b, double* x_out,
                                   int mode, const double* xc);
int batch_rr2_blocks(const Level& F);
RR2Job<double> batch_rr2_job(const Level& F, const double* x, const double* b, double* bc);
hipError_t k_batch_fused2(const Fused2Job<double>* jobs, const int* block_job, int nblocks, hipStream_t s);
// nrhs stacked vectors of one 2D level (x_in, b, x_out sv apart; xc sc apart), FP64
hipError_t k_sweep_fused2_multi(const Ctx& c, const Level& L, const double* x_in, const double* b, double* x_out,
                                int mode, const double* xc, int nrhs, int64_t sv, int64_t sc, hipStream_t s);
hipError_t k_residual_restrict2_multi(const Level& F, const double* x, const double* b, double* bc, int nrhs,
                                      int64_t sv, int64_t sc, hipStream_t s);
// x_k = A b_k for nrhs vectors (b, x n apart), one launch
hipError_t k_dense_matvec_multi(const double* A, int n, const double* b, double* x, int nrhs, hipStream_t s);
hipError_t k_batch_fused2_persistent(const Fused2Job<double>* jobs, const int* block_job, int nblocks, hipStream_t s);
hipError_t k_batch_rr2(const RR2Job<double>* jobs, const int* block_job, int nblocks, hipStream_t s);
hipError_t k_batch_dense(const DenseJob* jobs, const int* block_job, int nblocks, hipStream_t s);
int batch_norm_blocks(const Level& L);
NormJob batch_norm_job(const Level& L, const double* x, const double* b);
hipError_t k_batch_sumsq(const NormJob* jobs, int njobs, const int* block_job, int nblocks, double* part, double* out,
                         hipStream_t s);
// Set the calling thread's error message (fcgmg_last_error) and return `code`.
int set_error(int code, const std::string& msg);
template <class T>
hipError_t k_residual_restrict2(const Ctx& c, const Level& F, const T* x, const T* b, T* bc, hipStream_t s);
template <int D> hipError_t k_patch_solve(const Ctx& c, const Level& L, int policy, const double* r, double* x,
                                          hipStream_t s);
template <int D> hipError_t k_store_matrices(const Ctx& c, const Level& L, const int* nodes, int64_t count,
                                             double* M, hipStream_t s);
template <int D> hipError_t k_coarse_matrix(const Ctx& c, const Level& L, double* A, int lda, hipStream_t s);
template <int D, class T>
hipError_t k_restrict(const Ctx& c, int fine, const T* rf, T* bc, hipStream_t s, int nrhs = 1, int64_t sf = 0,
                      int64_t sc = 0);
template <int D, class T>
hipError_t k_prolong_add(const Ctx& c, int fine, const T* xc, T* xf, hipStream_t s, int nrhs = 1, int64_t sc = 0,
                         int64_t sf = 0);
template <class T>
hipError_t k_dense_matvec(const T* A, int n, const T* b, T* x, hipStream_t s);
hipError_t k_sumsq(const double* v, int64_t n, double* partial, int nblocks, hipStream_t s);
hipError_t k_finish_sumsq(const double* partial, int nblocks, double* out, hipStream_t s);
template <class T>
hipError_t k_zero(T* v, int64_t n, hipStream_t s);
// dst = (float) src / dst += (double) src, n values
hipError_t k_round_to_float(const double* src, float* dst, int64_t n, hipStream_t s);
hipError_t k_add_float(const float* src, double* dst, int64_t n, hipStream_t s);
// FGMRES vector kernels (FP64): h[i] = s * V_i . w for i < j (part: kKrylovPartials scratch);
// w = s * w - sum_i h[i] V_i; v = a * w. V_i = V + i * ld.
constexpr int kKrylovPartials = 256 * 64;
hipError_t k_multi_dot(const double* V, int64_t ld, int j, const double* w, int64_t n, double s, double* part,
                       double* h, hipStream_t st);
hipError_t k_multi_axpy(double* w, double s, const double* V, int64_t ld, int j, const double* h, int64_t n,
                        hipStream_t st);
hipError_t k_scale_copy(const double* w, double a, double* v, int64_t n, hipStream_t st);
template <int D> int pattern_size();
template <int D> void pattern_entries(std::vector<int>& enc);

// Batched standalone GMG steps for the solve server (fcgmg_batch.cpp): a batch whose set of problems
// changes from step to step. Every problem must be 2D, cache_inverse, FP64 with nu_pre = nu_post = 2.
bool batch_engine_accepts(const fcgmg_params& p);
int batch_engine_create(fcgmg_batch** out);
// norms[k] = ||b_k - L x_k||_2 of the finest level of hs[k]; with `cycle`, one V-cycle on every
// problem first. One synchronisation of s.
int batch_engine_step(fcgmg_batch* bt, const std::vector<fcgmg_ctx*>& hs, double* const* x, const double* const* b,
                      bool cycle, hipStream_t s, std::vector<double>& norms);
void batch_engine_destroy(fcgmg_batch* bt);

}  // namespace fcg

// The library handle (fcgmg_h) is the context of one hierarchy.
struct fcgmg_ctx : public fcg::Ctx {};
