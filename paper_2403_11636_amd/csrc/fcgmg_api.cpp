// Host planner and C-ABI of the fcgmg library (see include/fcgmg.h).
//
// Set-up follows Saberi & Vogel (arXiv 2403.11636): the level hierarchy of Algorithm 1 (uniform
// background grid: every cell coarsened at each step), cell classification and cut-cell
// integration, classification of the vertex patches of Eq. (15) into shared regular classes and
// individual patches, the cache policy of Sec. 3.1.2 and the coarsest-grid direct solver (Sec. 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "fcgmg_impl.h"

using namespace fcg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define FCG_HIP(call)                                                                            \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail(FCGMG_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// A value for a message, in scientific notation (std::to_string prints every digit of a large one).
std::string sci(double v) {
  char buf[32];
  std::snprintf(buf, sizeof buf, "%.3e", v);
  return buf;
}

int dev_alloc(Ctx& c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return FCGMG_OK;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(FCGMG_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  c.allocs.push_back(*p);
  c.bytes += bytes;
  return FCGMG_OK;
}

template <class T>
int alloc_n(Ctx& c, T** p, size_t n) {
  return dev_alloc(c, reinterpret_cast<void**>(p), n * sizeof(T));
}

// Launch a kernel through `f` (returning hipError_t); with the profiler on, bracket it by events.
template <class F>
int launch(const Ctx& c, int kind, int level, hipStream_t s, F&& f) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c.prof) {
    for (hipEvent_t* e : {&e0, &e1}) {
      if (!c.prof_pool.empty()) {
        *e = c.prof_pool.back();
        c.prof_pool.pop_back();
      } else {
        FCG_HIP(hipEventCreate(e));
      }
    }
    FCG_HIP(hipEventRecord(e0, s));
  }
  const hipError_t err = f();
  if (err != hipSuccess) return fail(FCGMG_E_HIP, std::string("kernel launch: ") + hipGetErrorString(err));
  if (c.prof) {
    FCG_HIP(hipEventRecord(e1, s));
    c.prof_pending.push_back(Ctx::ProfRec{kind, level, e0, e1});
  }
  return FCGMG_OK;
}

int prof_collect(const Ctx& c) {
  const int nl = (int)c.lev.size();
  if (c.prof_ms.empty()) {
    c.prof_ms.assign((size_t)FCGMG_K_COUNT * nl, 0.0);
    c.prof_count.assign((size_t)FCGMG_K_COUNT * nl, 0);
  }
  for (const Ctx::ProfRec& r : c.prof_pending) {
    FCG_HIP(hipEventSynchronize(r.stop));
    float ms = 0;
    FCG_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
    c.prof_ms[(size_t)r.kind * nl + r.level] += ms;
    c.prof_count[(size_t)r.kind * nl + r.level] += 1;
    c.prof_pool.push_back(r.start);
    c.prof_pool.push_back(r.stop);
  }
  c.prof_pending.clear();
  return FCGMG_OK;
}

// ---------------------------------------------------------------------------------------------
// Reference element data of uncut cells and Nitsche face matrices (host, once per level).
// ---------------------------------------------------------------------------------------------
template <int D>
void build_consts(const Ctx& c, Level& L) {
  constexpr int NN = 1 << D;
  OpConsts& oc = L.consts_h;
  std::memset(&oc, 0, sizeof(oc));
  oc.n = L.n;
  oc.immersed = c.prm.immersed_nitsche;
  oc.h = L.h;
  const double eta = c.prm.eta;
  oc.lam = c.prm.nitsche_beta * eta / L.h;
  const double lo[3] = {0, 0, 0};
  // kind 0: alpha = 1 (no obstacle); kind 1: alpha = alpha_f everywhere (one ball covering the cell)
  const double cover[4] = {0.5 * L.h, 0.5 * L.h, 0.5 * L.h, 4.0 * L.h};
  for (int kind = 0; kind < 2; ++kind) {
    Geom g{cover, kind, 0, c.prm.alpha_fict};
    double acc[PT<D>::NEL] = {0};
    tree_quadrature<D>(g, lo, L.h, [&](const double* x, double w, double alpha) {
      double phi[NN], gr[NN][3];
      q1<D>(lo, L.h, x, phi, gr);
      for (int e = 0; e < PT<D>::NEL; ++e) acc[e] += point_entry<D>(e, eta, w * alpha, phi, gr);
    });
    for (int ab = 0; ab < NN * NN; ++ab) {
      oc.K[kind][ab] = acc[ab];
      for (int cc = 0; cc < D; ++cc) oc.B[kind][cc][ab] = acc[(1 + cc) * NN * NN + ab];
    }
  }
  // stabilisation: -(1/eta)(M - m m^T / |K|), exact 2^d Gauss (no alpha)
  {
    Geom g{nullptr, 0, 0, 1.0};
    double M[NN * NN] = {0}, m[NN] = {0};
    tree_quadrature<D>(g, lo, L.h, [&](const double* x, double w, double) {
      double phi[NN], gr[NN][3];
      q1<D>(lo, L.h, x, phi, gr);
      for (int a = 0; a < NN; ++a) {
        m[a] += w * phi[a];
        for (int b = 0; b < NN; ++b) M[a * NN + b] += w * phi[a] * phi[b];
      }
    });
    const double vol = std::pow(L.h, D);
    for (int a = 0; a < NN; ++a)
      for (int b = 0; b < NN; ++b) oc.C[a * NN + b] = -(1.0 / eta) * (M[a * NN + b] - m[a] * m[b] / vol);
  }
  // node stencils of uniform uncut neighbourhoods: sum of the element rows of the 2^d cells
  for (int kind = 0; kind < 2; ++kind)
    for (int sc = 0; sc < NN; ++sc) {
      int a = 0;
      for (int k = 0; k < D; ++k) a |= (1 - ((sc >> k) & 1)) << k;
      for (int bn = 0; bn < NN; ++bn) {
        int o = 0, mul = 1;
        for (int k = 0; k < D; ++k) {
          o += (((sc >> k) & 1) + ((bn >> k) & 1)) * mul;  // offset -1 + s + b shifted by +1
          mul *= 3;
        }
        oc.SK[kind][o] += oc.K[kind][a * NN + bn];
        for (int cc = 0; cc < D; ++cc) {
          oc.SB[kind][cc][o] += oc.B[kind][cc][a * NN + bn];
          oc.ST[kind][cc][o] += oc.B[kind][cc][bn * NN + a];
        }
        if (kind == 0) oc.SC[o] += oc.C[a * NN + bn];
      }
    }
  // Nitsche face terms: -(v, n.eta grad u) - (n.eta grad v, u) + (v, lambda u) per component and
  // (v, n p) + (n q, u) on each Dirichlet wall (2-point Gauss per tangential direction).
  for (int k = 0; k < D; ++k)
    for (int sd = 0; sd < 2; ++sd) {
      const int face = 2 * k + sd;
      const int code = c.prm.bc[face];
      oc.dirichlet[face] = code != FCGMG_BC_NEUMANN;
      if (!oc.dirichlet[face]) continue;
      const double nk = sd ? 1.0 : -1.0;
      const double w = D == 2 ? 0.5 * L.h : 0.25 * L.h * L.h;
      for (int gp = 0; gp < (1 << (D - 1)); ++gp) {
        double x[3] = {0, 0, 0};
        int t = 0;
        for (int j = 0; j < D; ++j) {
          if (j == k) {
            x[j] = sd ? L.h : 0.0;
          } else {
            x[j] = L.h * (((gp >> t) & 1) ? FCG_GB : FCG_GA);
            ++t;
          }
        }
        double phi[NN], gr[NN][3];
        q1<D>(lo, L.h, x, phi, gr);
        for (int a = 0; a < NN; ++a)
          for (int b = 0; b < NN; ++b) {
            oc.FK[face][a * NN + b] += w * (-eta * phi[a] * nk * gr[b][k] - eta * nk * gr[a][k] * phi[b] +
                                            oc.lam * phi[a] * phi[b]);
            oc.FB[face][a * NN + b] += w * phi[a] * nk * phi[b];
          }
      }
    }
  using R = RefLayout<D>;
  for (int i = 0; i < R::NN2; ++i) {
    oc.pack[R::oK + i] = oc.K[0][i];
    for (int cc = 0; cc < D; ++cc) oc.pack[R::oB + cc * R::NN2 + i] = oc.B[0][cc][i];
    oc.pack[R::oC + i] = oc.C[i];
    for (int f = 0; f < 2 * D; ++f) {
      oc.pack[R::oFK + f * R::NN2 + i] = oc.FK[f][i];
      oc.pack[R::oFB + f * R::NN2 + i] = oc.FB[f][i];
    }
  }
  for (int o = 0; o < R::NS; ++o) {
    for (int kind = 0; kind < 2; ++kind) {
      oc.pack[R::oSK + kind * R::NS + o] = oc.SK[kind][o];
      for (int cc = 0; cc < D; ++cc) {
        oc.pack[R::oSB + (kind * D + cc) * R::NS + o] = oc.SB[kind][cc][o];
        oc.pack[R::oST + (kind * D + cc) * R::NS + o] = oc.ST[kind][cc][o];
      }
    }
    oc.pack[R::oSC + o] = oc.SC[o];
  }
}

// ---------------------------------------------------------------------------------------------
// Operator code of every node (Level::node_op): a node at least 2 nodes from every wall whose 2^d
// cells are uncut and of one kind uses that kind's reference stencil (-1 physical, -2 fictitious);
// every other node gets a stored stencil. The row of a node is fixed by its cells and the walls
// that reach it, so nodes nearer a wall whose cells are uncut and of one kind share the row of
// their kind and wall position (per axis: node 0 or 1 from the low wall, interior, 1 or 0 from the
// high wall), computed from the first of them. sten_nodes lists the node of each stored row.
// ---------------------------------------------------------------------------------------------
template <int D>
void node_operator_codes(const Level& L, const std::vector<signed char>& kinds, std::vector<int>& op,
                         std::vector<int>& sten_nodes) {
  const int n = L.n;
  const int64_t m = n + 1;
  sten_nodes.clear();
  std::map<int, int> wall2row;
  for (int64_t node = 0; node < L.N; ++node) {
    const int c[3] = {(int)(node % m), (int)((node / m) % m), D == 3 ? (int)(node / (m * m)) : 0};
    bool interior = true;
    int wkey = 0;
    for (int k = 0; k < D; ++k) {
      interior = interior && c[k] >= 2 && c[k] <= n - 2;
      // wall case per axis: 0, 1 low wall, 2 interior, 3, 4 distance 1, 0 from the high wall
      // (injective in c on a level, also where the ranges meet on small grids)
      wkey = wkey * 5 + (c[k] <= 1 ? c[k] : (c[k] >= n - 1 ? 3 + c[k] - (n - 1) : 2));
    }
    // the cells of the node that exist: uncut and of one kind?
    bool uni = true;
    int kind0 = -1;
    for (int sc = 0; sc < (1 << D) && uni; ++sc) {
      int64_t cell = 0, mul = 1;
      bool in = true;
      for (int k = 0; k < D; ++k) {
        const int cc = c[k] - 1 + ((sc >> k) & 1);
        in = in && cc >= 0 && cc < n;
        cell += cc * mul;
        mul *= n;
      }
      if (!in) continue;
      const int kd = kinds[cell];
      if (kind0 < 0) kind0 = kd;
      uni = kd != 2 && kd == kind0;
    }
    if (uni && interior) {
      op[node] = -1 - kind0;
    } else if (uni) {
      const int key = wkey * 2 + kind0;
      auto it = wall2row.find(key);
      if (it == wall2row.end()) {
        op[node] = (int)sten_nodes.size();
        wall2row[key] = op[node];
        sten_nodes.push_back((int)node);
      } else {
        op[node] = it->second;
      }
    } else {
      op[node] = (int)sten_nodes.size();
      sten_nodes.push_back((int)node);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Patch classification. The block L_i of a patch is fixed by the cells of its 6^d window (cells
// c-3 .. c+2 per axis, clipped to the grid) and by the walls among them.
// * A patch whose window lies inside the grid (at least 3 nodes from every wall) and holds no cut
//   cell and only one kind of uncut cell has the same block as every other such patch of that
//   kind: these share one class (at most two per level, physical and fictitious), applied with
//   scalar loads of its rows.
// * Every other patch is streamed: individual rows, listed in irr_nodes. With share_walls, a
//   streamed patch whose window holds no cut cell and one kind (a wall patch) shares its rows with
//   the patches of the same kind at the same position relative to the walls (per axis: distance
//   0, 1 or 2 from the low wall, interior, or distance 2, 1, 0 from the high wall), computed once
//   from the first of them.
// zrow_nodes lists the nodes whose inverse rows are computed (row k from zrow_nodes[k]); irr_zrow
// gives the row of every streamed patch; node_class is the class (>= 0) or -(row) - 1.
// ---------------------------------------------------------------------------------------------
template <int D>
void classify_patches(const Level& L, const std::vector<signed char>& kinds, bool share_walls,
                      std::vector<int>& node_class, std::vector<int>& class_rep, std::vector<int>& irr_nodes,
                      std::vector<int>& irr_zrow, std::vector<int>& zrow_nodes) {
  const int n = L.n;
  const int64_t m = n + 1;  // summed-area tables over cells, size (n+1)^D
  std::vector<int> sat_cut(D == 2 ? m * m : m * m * m, 0), sat_fic(sat_cut.size(), 0);
  auto sidx = [&](int x, int y, int z) { return (int64_t)x + m * ((int64_t)y + m * (int64_t)z); };
  for (int z = 0; z < (D == 3 ? n : 1); ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const int64_t cell = x + (int64_t)n * (y + (int64_t)n * z);
        const int kc = kinds[cell] == 2, kf = kinds[cell] == 1;
        const int zz = D == 3 ? z + 1 : 0;
        if (D == 2) {
          sat_cut[sidx(x + 1, y + 1, 0)] = kc + sat_cut[sidx(x, y + 1, 0)] + sat_cut[sidx(x + 1, y, 0)] - sat_cut[sidx(x, y, 0)];
          sat_fic[sidx(x + 1, y + 1, 0)] = kf + sat_fic[sidx(x, y + 1, 0)] + sat_fic[sidx(x + 1, y, 0)] - sat_fic[sidx(x, y, 0)];
        } else {
          auto upd = [&](std::vector<int>& S, int v) {
            S[sidx(x + 1, y + 1, zz)] = v + S[sidx(x, y + 1, zz)] + S[sidx(x + 1, y, zz)] + S[sidx(x + 1, y + 1, zz - 1)] -
                                        S[sidx(x, y, zz)] - S[sidx(x, y + 1, zz - 1)] - S[sidx(x + 1, y, zz - 1)] +
                                        S[sidx(x, y, zz - 1)];
          };
          upd(sat_cut, kc);
          upd(sat_fic, kf);
        }
      }
  auto box_sum = [&](const std::vector<int>& S, const int* lo, const int* hi) -> int64_t {
    // inclusive cell ranges lo..hi
    if (D == 2)
      return S[sidx(hi[0] + 1, hi[1] + 1, 0)] - S[sidx(lo[0], hi[1] + 1, 0)] - S[sidx(hi[0] + 1, lo[1], 0)] +
             S[sidx(lo[0], lo[1], 0)];
    return S[sidx(hi[0] + 1, hi[1] + 1, hi[2] + 1)] - S[sidx(lo[0], hi[1] + 1, hi[2] + 1)] -
           S[sidx(hi[0] + 1, lo[1], hi[2] + 1)] - S[sidx(hi[0] + 1, hi[1] + 1, lo[2])] + S[sidx(lo[0], lo[1], hi[2] + 1)] +
           S[sidx(lo[0], hi[1] + 1, lo[2])] + S[sidx(hi[0] + 1, lo[1], lo[2])] - S[sidx(lo[0], lo[1], lo[2])];
  };
  std::map<int, int> key2cls, wall2row;
  node_class.assign(L.N, 0);
  class_rep.clear();
  irr_nodes.clear();
  irr_zrow.clear();
  zrow_nodes.clear();
  for (int64_t node = 0; node < L.N; ++node) {
    int c[3] = {(int)(node % m), (int)((node / m) % m), D == 3 ? (int)(node / (m * m)) : 0};
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int64_t tot = 1;
    int key = 0, wkey = 0;
    bool interior = true;
    for (int k = 0; k < D; ++k) {
      lo[k] = std::max(c[k] - 3, 0);
      hi[k] = std::min(c[k] + 2, n - 1);
      tot *= (hi[k] - lo[k] + 1);
      interior = interior && c[k] >= 3 && n - c[k] >= 3;
      // wall case per axis: 0..2 low wall, 3 interior, 4..6 distance 2..0 from the high wall
      // (injective in c on a level, also where the ranges meet on small grids)
      wkey = wkey * 7 + (c[k] <= 2 ? c[k] : (c[k] >= n - 2 ? 4 + c[k] - (n - 2) : 3));
    }
    const int64_t ncut = box_sum(sat_cut, lo, hi);
    const int64_t nfic = box_sum(sat_fic, lo, hi);
    const bool uniform = ncut == 0 && (nfic == 0 || nfic == tot);
    if (!interior && uniform && share_walls) {
      wkey = wkey * 2 + (nfic ? 1 : 0);
      auto it = wall2row.find(wkey);
      int row;
      if (it == wall2row.end()) {
        row = (int)zrow_nodes.size();
        wall2row[wkey] = row;
        zrow_nodes.push_back((int)node);
      } else {
        row = it->second;
      }
      node_class[node] = -row - 1;
      irr_nodes.push_back((int)node);
      irr_zrow.push_back(row);
    } else if (interior && uniform) {
      key = key * 2 + (nfic ? 1 : 0);
      auto it = key2cls.find(key);
      int cls;
      if (it == key2cls.end()) {
        cls = (int)class_rep.size();
        key2cls[key] = cls;
        class_rep.push_back((int)node);
      } else {
        cls = it->second;
      }
      node_class[node] = cls;
    } else {
      const int row = (int)zrow_nodes.size();
      node_class[node] = -row - 1;
      irr_nodes.push_back((int)node);
      irr_zrow.push_back(row);
      zrow_nodes.push_back((int)node);
    }
  }
}

// Dense inverse by Gaussian elimination with partial pivoting (host; coarsest grid only).
bool dense_inverse(int n, std::vector<double>& A, std::vector<double>& Inv) {
  Inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Inv[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + k]) > best) {
        best = std::fabs(A[(size_t)i * n + k]);
        p = i;
      }
    if (!(best > 0.0)) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
        std::swap(Inv[(size_t)k * n + j], Inv[(size_t)p * n + j]);
      }
    const double piv = A[(size_t)k * n + k];
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double l = A[(size_t)i * n + k] / piv;
      if (l == 0.0) continue;
      for (int j = k; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
      for (int j = 0; j < n; ++j) Inv[(size_t)i * n + j] -= l * Inv[(size_t)k * n + j];
    }
    for (int j = k; j < n; ++j) A[(size_t)k * n + j] /= piv;
    for (int j = 0; j < n; ++j) Inv[(size_t)k * n + j] /= piv;
  }
  return true;
}

constexpr int kCoarseMaxDofs = 6000;
constexpr int kRedBlocks = 512;

// True when a cut or fictitious cell has a face on a Dirichlet wall of the box. The Nitsche wall terms
// carry no alpha, so inside an obstacle they can outweigh the alpha_f-weighted volume terms and leave
// the velocity block of a patch indefinite.
template <int D>
bool obstacle_on_dirichlet_face(const fcgmg_params& P, const Level& L, const std::vector<signed char>& kinds) {
  for (int64_t cell = 0; cell < L.ncells; ++cell) {
    if (kinds[cell] == 0) continue;
    const int64_t ci[3] = {cell % L.n, (cell / L.n) % L.n, D == 3 ? cell / ((int64_t)L.n * L.n) : 0};
    for (int k = 0; k < D; ++k) {
      if (ci[k] == 0 && P.bc[2 * k] != FCGMG_BC_NEUMANN) return true;
      if (ci[k] == L.n - 1 && P.bc[2 * k + 1] != FCGMG_BC_NEUMANN) return true;
    }
  }
  return false;
}

template <int D>
int setup_impl(Ctx& c, hipStream_t s) {
  const fcgmg_params& P = c.prm;
  const int nlev = P.n_levels;
  c.lev.resize(nlev);
  int rc;
  if ((rc = alloc_n(c, &c.err, 1))) return rc;
  const int imax = INT_MAX;
  FCG_HIP(hipMemcpyAsync(c.err, &imax, sizeof(int), hipMemcpyHostToDevice, s));
  if (!c.balls_h.empty()) {
    if ((rc = alloc_n(c, &c.balls, c.balls_h.size()))) return rc;
    FCG_HIP(hipMemcpyAsync(c.balls, c.balls_h.data(), c.balls_h.size() * sizeof(double), hipMemcpyHostToDevice, s));
  }
  if ((rc = alloc_n(c, &c.red, kRedBlocks + 1))) return rc;
  if (D == 3 && P.cache_policy == FCGMG_CACHE_INVERSE) {
    FCG_HIP(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
    FCG_HIP(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming));
    FCG_HIP(hipEventCreateWithFlags(&c.ev_join, hipEventDisableTiming));
  }
  FCG_HIP(hipHostMalloc((void**)&c.red_host, sizeof(double), hipHostMallocDefault));
  FCG_HIP(hipHostGetDevicePointer((void**)&c.red_host_dev, c.red_host, 0));
  if (P.cache_policy == FCGMG_CACHE_MATRIX) {
    std::vector<int> enc;
    pattern_entries<D>(enc);
    c.n_pattern = (int)enc.size();
    if ((rc = alloc_n(c, &c.pattern, enc.size()))) return rc;
    FCG_HIP(hipMemcpyAsync(c.pattern, enc.data(), enc.size() * sizeof(int), hipMemcpyHostToDevice, s));
    FCG_HIP(hipStreamSynchronize(s));  // enc must outlive the copy
  }
  signed char* kinds_d = nullptr;
  for (int l = 0; l < nlev; ++l) {
    Level& L = c.lev[l];
    L.n = P.n_cells >> (nlev - 1 - l);
    L.qd = P.quad_depth + (nlev - 1 - l);
    L.h = 1.0 / L.n;
    L.N = 1;
    L.ncells = 1;
    for (int k = 0; k < D; ++k) {
      L.N *= (L.n + 1);
      L.ncells *= L.n;
    }
    const int64_t nd = (D + 1) * L.N;
    if ((rc = alloc_n(c, &L.r, nd))) return rc;
    if (l < nlev - 1) {
      if ((rc = alloc_n(c, &L.x, nd))) return rc;
      if ((rc = alloc_n(c, &L.b, nd))) return rc;
    }
    if (D == 2 && P.cache_policy == FCGMG_CACHE_INVERSE)
      if ((rc = alloc_n(c, &L.xalt, nd))) return rc;
    // cells
    FCG_HIP(hipMallocAsync((void**)&kinds_d, L.ncells, s));
    FCG_HIP(k_classify_cells<D>(c, L, kinds_d, s));
    std::vector<signed char> kinds(L.ncells);
    FCG_HIP(hipMemcpyAsync(kinds.data(), kinds_d, L.ncells, hipMemcpyDeviceToHost, s));
    FCG_HIP(hipStreamSynchronize(s));
    FCG_HIP(hipFreeAsync(kinds_d, s));
    std::vector<int> info(L.ncells), cut_list;
    for (int64_t i = 0; i < L.ncells; ++i) {
      if (kinds[i] == 2) {
        info[i] = (int)cut_list.size();
        cut_list.push_back((int)i);
      } else {
        info[i] = kinds[i] == 1 ? -2 : -1;
        if (kinds[i] == 1) ++L.n_fict;
      }
    }
    L.n_cut = (int64_t)cut_list.size();
    // blocks that may be indefinite are factorised by a dense LU with pivoting: in 2D with immersed
    // Nitsche terms or an obstacle over a Dirichlet face of the box, in 3D with immersed Nitsche
    // terms (cache_inverse, at set-up)
    L.dense_lu = D == 2 ? (P.immersed_nitsche || obstacle_on_dirichlet_face<D>(P, L, kinds))
                        : (P.immersed_nitsche && P.cache_policy == FCGMG_CACHE_INVERSE);
    if ((rc = alloc_n(c, &L.cell_info, L.ncells))) return rc;
    FCG_HIP(hipMemcpyAsync(L.cell_info, info.data(), L.ncells * sizeof(int), hipMemcpyHostToDevice, s));
    int* cut_d = nullptr;
    if (L.n_cut) {
      if ((rc = alloc_n(c, &L.cut_mats, (size_t)L.n_cut * PT<D>::NEL))) return rc;
      FCG_HIP(hipMallocAsync((void**)&cut_d, L.n_cut * sizeof(int), s));
      FCG_HIP(hipMemcpyAsync(cut_d, cut_list.data(), L.n_cut * sizeof(int), hipMemcpyHostToDevice, s));
      FCG_HIP(k_cut_matrices<D>(c, L, cut_d, s));
      FCG_HIP(hipFreeAsync(cut_d, s));
    }
    build_consts<D>(c, L);
    if ((rc = alloc_n(c, &L.consts, 1))) return rc;
    FCG_HIP(hipMemcpyAsync(L.consts, &L.consts_h, sizeof(OpConsts), hipMemcpyHostToDevice, s));
    // operator rows: the reference stencil of a uniform neighbourhood, else an assembled one
    std::vector<int> op(L.N), sten_nodes;
    node_operator_codes<D>(L, kinds, op, sten_nodes);
    L.n_nsten = (int64_t)sten_nodes.size();
    if ((rc = alloc_n(c, &L.node_op, L.N))) return rc;
    FCG_HIP(hipMemcpyAsync(L.node_op, op.data(), L.N * sizeof(int), hipMemcpyHostToDevice, s));
    if (L.n_nsten) {
      if ((rc = alloc_n(c, &L.nsten, (size_t)L.n_nsten * PT<D>::NSTEN))) return rc;
      int* sn_d = nullptr;
      FCG_HIP(hipMallocAsync((void**)&sn_d, L.n_nsten * sizeof(int), s));
      FCG_HIP(hipMemcpyAsync(sn_d, sten_nodes.data(), L.n_nsten * sizeof(int), hipMemcpyHostToDevice, s));
      FCG_HIP(k_node_stencils<D>(c, L, sn_d, s));
      FCG_HIP(hipFreeAsync(sn_d, s));
    }
    FCG_HIP(hipStreamSynchronize(s));  // op and sten_nodes must outlive the copies
    // patches
    std::vector<int> ncls, reps, irr, zrow, znodes, extra;
    classify_patches<D>(L, kinds, P.cache_policy == FCGMG_CACHE_INVERSE, ncls, reps, irr, zrow, znodes);
    L.n_classes = (int64_t)reps.size();
    L.n_irr = (int64_t)irr.size();
    L.n_zrows = (int64_t)znodes.size();
    L.irr_cols = 0;
    for (int node : znodes) {
      int cc[3] = {(int)(node % (L.n + 1)), (int)((node / (L.n + 1)) % (L.n + 1)), D == 3 ? (int)(node / ((int64_t)(L.n + 1) * (L.n + 1))) : 0};
      int64_t nv = 1, np = 1;
      for (int k = 0; k < D; ++k) {
        nv *= std::min(cc[k] + 2, L.n) - std::max(cc[k] - 2, 0) + 1;
        np *= std::min(cc[k] + 1, L.n) - std::max(cc[k] - 1, 0) + 1;
      }
      L.irr_cols += D * nv + np;
    }
    if ((rc = alloc_n(c, &L.node_class, L.N))) return rc;
    FCG_HIP(hipMemcpyAsync(L.node_class, ncls.data(), L.N * sizeof(int), hipMemcpyHostToDevice, s));
    if (L.n_classes) {
      if ((rc = alloc_n(c, &L.class_rep, L.n_classes))) return rc;
      FCG_HIP(hipMemcpyAsync(L.class_rep, reps.data(), L.n_classes * sizeof(int), hipMemcpyHostToDevice, s));
    }
    if (L.n_irr) {
      if ((rc = alloc_n(c, &L.irr_nodes, L.n_irr))) return rc;
      FCG_HIP(hipMemcpyAsync(L.irr_nodes, irr.data(), L.n_irr * sizeof(int), hipMemcpyHostToDevice, s));
      if ((rc = alloc_n(c, &L.irr_zrow, L.n_irr))) return rc;
      FCG_HIP(hipMemcpyAsync(L.irr_zrow, zrow.data(), L.n_irr * sizeof(int), hipMemcpyHostToDevice, s));
    }
    if (L.n_zrows) {
      if ((rc = alloc_n(c, &L.zrow_nodes, L.n_zrows))) return rc;
      FCG_HIP(hipMemcpyAsync(L.zrow_nodes, znodes.data(), L.n_zrows * sizeof(int), hipMemcpyHostToDevice, s));
    }
    if (D == 2 && P.cache_policy == FCGMG_CACHE_INVERSE) {
      plan_fused2(L, ncls, extra);
      L.n_fused_extra = (int)extra.size();
      L.fused_extra_cap = L.n_fused_extra;
      if (L.n_fused_extra) {
        if ((rc = alloc_n(c, &L.fused_extra, extra.size()))) return rc;
        FCG_HIP(hipMemcpyAsync(L.fused_extra, extra.data(), extra.size() * sizeof(int), hipMemcpyHostToDevice, s));
      }
    }
    // the host vectors above must outlive the asynchronous copies
    FCG_HIP(hipStreamSynchronize(s));
    // cache policy (Sec. 3.1.2)
    if (P.cache_policy == FCGMG_CACHE_INVERSE) {
      const size_t row = (size_t)(D + 1) * PT<D>::ZSP;
      if ((rc = alloc_n(c, &L.Zcls, L.n_classes * row))) return rc;
      if ((rc = alloc_n(c, &L.Zirr, L.n_zrows * row))) return rc;
      L.cached_bytes = (L.n_classes + L.n_zrows) * row * sizeof(double);
      FCG_HIP(k_patch_inverse_rows<D>(c, L, L.class_rep, L.n_classes, L.Zcls, s));
      FCG_HIP(k_patch_inverse_rows<D>(c, L, L.zrow_nodes, L.n_zrows, L.Zirr, s));
      if (P.precision == FCGMG_PREC_MIXED) {
        // FP32 copies, rounded from the FP64 factorisations
        const int64_t nd32 = (D + 1) * L.N;
        if ((rc = alloc_n(c, &L.Zcls32, L.n_classes * row))) return rc;
        if ((rc = alloc_n(c, &L.Zirr32, L.n_zrows * row))) return rc;
        if ((rc = alloc_n(c, &L.nsten32, (size_t)L.n_nsten * PT<D>::NSTEN))) return rc;
        if ((rc = alloc_n(c, &L.r32, nd32))) return rc;
        if ((rc = alloc_n(c, &L.x32, nd32))) return rc;
        if ((rc = alloc_n(c, &L.b32, nd32))) return rc;
        if (D == 2)
          if ((rc = alloc_n(c, &L.xalt32, nd32))) return rc;
        FCG_HIP(k_round_to_float(L.Zcls, L.Zcls32, (int64_t)(L.n_classes * row), s));
        FCG_HIP(k_round_to_float(L.Zirr, L.Zirr32, (int64_t)(L.n_zrows * row), s));
        FCG_HIP(k_round_to_float(L.nsten, L.nsten32, L.n_nsten * PT<D>::NSTEN, s));
      }
    } else if (P.cache_policy == FCGMG_CACHE_MATRIX) {
      if ((rc = alloc_n(c, &L.Mcls, L.n_classes * (size_t)c.n_pattern))) return rc;
      if ((rc = alloc_n(c, &L.Mirr, L.n_irr * (size_t)c.n_pattern))) return rc;
      L.cached_bytes = (L.n_classes + L.n_irr) * (size_t)c.n_pattern * sizeof(double);
      FCG_HIP(k_store_matrices<D>(c, L, L.class_rep, L.n_classes, L.Mcls, s));
      FCG_HIP(k_store_matrices<D>(c, L, L.irr_nodes, L.n_irr, L.Mirr, s));
      if (l > 0) FCG_HIP(k_patch_solve<D>(c, L, P.cache_policy, nullptr, nullptr, s));  // validation pass
    } else {
      if (l > 0) FCG_HIP(k_patch_solve<D>(c, L, P.cache_policy, nullptr, nullptr, s));  // validation pass
    }
    int errv = INT_MAX;
    FCG_HIP(hipMemcpyAsync(&errv, c.err, sizeof(int), hipMemcpyDeviceToHost, s));
    FCG_HIP(hipStreamSynchronize(s));
    if (errv != INT_MAX)
      return fail(FCGMG_E_SINGULAR, "singular local block L_i of patch node " + std::to_string(errv) + " on level " +
                                        std::to_string(l));
  }
  // coarsest level: dense operator, bordered when the constant pressure lies in the kernel
  {
    Level& L = c.lev[0];
    const int nd = (int)((D + 1) * L.N);
    if (nd > kCoarseMaxDofs)
      return fail(FCGMG_E_ARG, "coarsest level has " + std::to_string(nd) + " DoFs; the direct solver accepts at most " +
                                   std::to_string(kCoarseMaxDofs) + " (use more levels)");
    bool all_dir = true;
    for (int k = 0; k < 2 * D; ++k)
      if (P.bc[k] == FCGMG_BC_NEUMANN) all_dir = false;
    c.bordered = all_dir && (c.balls_h.empty() || P.alpha_fict == 1.0);
    double* A_d = nullptr;
    FCG_HIP(hipMallocAsync((void**)&A_d, (size_t)nd * nd * sizeof(double), s));
    FCG_HIP(k_coarse_matrix<D>(c, L, A_d, nd, s));
    std::vector<double> A((size_t)nd * nd);
    FCG_HIP(hipMemcpyAsync(A.data(), A_d, A.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    FCG_HIP(hipStreamSynchronize(s));
    FCG_HIP(hipFreeAsync(A_d, s));
    const int m = nd + (c.bordered ? 1 : 0);
    std::vector<double> Ab((size_t)m * m, 0.0), Inv;
    for (int i = 0; i < nd; ++i)
      for (int j = 0; j < nd; ++j) Ab[(size_t)i * m + j] = A[(size_t)i * nd + j];
    if (c.bordered)
      for (int i = (int)(D * L.N); i < nd; ++i) {
        Ab[(size_t)i * m + nd] = 1.0;
        Ab[(size_t)nd * m + i] = 1.0;
      }
    if (!dense_inverse(m, Ab, Inv)) return fail(FCGMG_E_SINGULAR, "singular coarsest-grid operator");
    std::vector<double> Ic((size_t)nd * nd);
    for (int i = 0; i < nd; ++i)
      for (int j = 0; j < nd; ++j) Ic[(size_t)i * nd + j] = Inv[(size_t)i * m + j];
    c.coarse_n = nd;
    if ((rc = alloc_n(c, &c.coarse_inv, Ic.size()))) return rc;
    FCG_HIP(hipMemcpyAsync(c.coarse_inv, Ic.data(), Ic.size() * sizeof(double), hipMemcpyHostToDevice, s));
    if (P.precision == FCGMG_PREC_MIXED) {
      if ((rc = alloc_n(c, &c.coarse_inv32, Ic.size()))) return rc;
      FCG_HIP(k_round_to_float(c.coarse_inv, c.coarse_inv32, (int64_t)Ic.size(), s));
    }
    FCG_HIP(hipStreamSynchronize(s));  // Ic must outlive the copy
  }
  if (P.solver == FCGMG_SOLVER_FGMRES) {
    const size_t nd = (size_t)(D + 1) * c.lev[nlev - 1].N, m = P.krylov_restart;
    if ((rc = alloc_n(c, &c.kv, (m + 1) * nd))) return rc;
    if ((rc = alloc_n(c, &c.kz, m * nd))) return rc;
    if ((rc = alloc_n(c, &c.kw, nd))) return rc;
    if ((rc = alloc_n(c, &c.kzero, nd))) return rc;
    if ((rc = alloc_n(c, &c.kpart, (size_t)kKrylovPartials))) return rc;
    if ((rc = alloc_n(c, &c.kh, (size_t)192))) return rc;
    FCG_HIP(hipHostMalloc((void**)&c.kh_host, 192 * sizeof(double), hipHostMallocDefault));
    FCG_HIP(k_zero<double>(c.kzero, (int64_t)nd, s));
    FCG_HIP(hipStreamSynchronize(s));
  }
  return FCGMG_OK;
}

// ---------------------------------------------------------------------------------------------
// Operations (dimension-dispatched).
// ---------------------------------------------------------------------------------------------
// T is the value type of the vectors: double for the FP64 operations, float for the V-cycle of the
// mixed-precision solve (cache_inverse only).
template <int D, class T = double>
int residual_impl(const Ctx& c, int l, const T* x, const T* b, T* r, hipStream_t s) {
  return launch(c, FCGMG_K_RESIDUAL, l, s, [&] { return k_residual<D, T>(c, c.lev[l], x, b, r, s); });
}

template <int D, class T = double>
int prolong_impl(const Ctx& c, int l, const T* xc, T* xf, hipStream_t s) {
  return launch(c, FCGMG_K_PROLONG, l, s, [&] { return k_prolong_add<D, T>(c, l, xc, xf, s); });
}

template <int D, class T = double>
int sweep_impl(const Ctx& c, int l, T* x, const T* b, hipStream_t s, T* rbuf = nullptr) {
  const Level& L = c.lev[l];
  T* r = rbuf ? rbuf : LV<T>::r(L);
  int rc;
  if ((rc = residual_impl<D, T>(c, l, x, b, r, s))) return rc;
  if (c.prm.cache_policy == FCGMG_CACHE_INVERSE) {
    if (D == 3 && c.side && L.n_classes && L.n_irr) {
      // the shared-class patches on the second stream, concurrently with the streamed ones: each
      // node is written by one of the two applies, both read only r
      FCG_HIP(hipEventRecord(c.ev_fork, s));
      FCG_HIP(hipStreamWaitEvent(c.side, c.ev_fork, 0));
      if ((rc = launch(c, FCGMG_K_APPLY_REGULAR, l, c.side, [&] { return k_apply_regular<D, T>(c, L, r, x, c.side); })))
        return rc;
      FCG_HIP(hipEventRecord(c.ev_join, c.side));
      if ((rc = launch(c, FCGMG_K_APPLY_IRREGULAR, l, s, [&] { return k_apply_irregular<D, T>(c, L, r, x, s); })))
        return rc;
      FCG_HIP(hipStreamWaitEvent(s, c.ev_join, 0));
      return FCGMG_OK;
    }
    if (L.n_classes)
      if ((rc = launch(c, FCGMG_K_APPLY_REGULAR, l, s, [&] { return k_apply_regular<D, T>(c, L, r, x, s); })))
        return rc;
    if (L.n_irr)
      if ((rc = launch(c, FCGMG_K_APPLY_IRREGULAR, l, s, [&] { return k_apply_irregular<D, T>(c, L, r, x, s); })))
        return rc;
    return FCGMG_OK;
  }
  if constexpr (std::is_same<T, double>::value)
    return launch(c, FCGMG_K_PATCH_SOLVE, l, s, [&] { return k_patch_solve<D>(c, L, c.prm.cache_policy, r, x, s); });
  return fail(FCGMG_E_ARG, "the FP32 cycle needs the cache_inverse policy");
}

// `sweeps` sweeps on level l. 2D cache_inverse: pairs of fused sweeps ping-pong between x and the
// level's second buffer (an odd first sweep runs unfused, in place); the arithmetic is identical.
// `mode` describes x on entry: 0 as given; 1 zero (contents undefined, not read); 2 still to be
// corrected by the prolongation of the coarse vector xc. The fused pair applies modes 1 and 2 while
// loading; otherwise x is zeroed or corrected first.
// `rbuf` / `abuf` replace the level's residual and second-iterate buffers when given.
template <int D, class T = double>
int smooth_impl(const Ctx& c, int l, T* x, const T* b, int sweeps, hipStream_t s, int mode = 0,
                const T* xc = nullptr, T* rbuf = nullptr, T* abuf = nullptr) {
  const Level& L = c.lev[l];
  T* xalt = (abuf && LV<T>::xalt(L)) ? abuf : LV<T>::xalt(L);
  int rc;
  const bool fused = D == 2 && c.prm.cache_policy == FCGMG_CACHE_INVERSE && xalt;
  if (mode != 0 && (!fused || sweeps % 2 == 1 || sweeps == 0)) {
    if (mode == 1)
      rc = launch(c, FCGMG_K_ZERO, l, s, [&] { return k_zero<T>(x, (D + 1) * L.N, s); });
    else
      rc = prolong_impl<D, T>(c, l, xc, x, s);
    if (rc) return rc;
    mode = 0;
  }
  if (fused) {
    int k = 0;
    if (sweeps % 2 == 1) {
      if ((rc = sweep_impl<D, T>(c, l, x, b, s, rbuf))) return rc;
      k = 1;
    }
    for (; k < sweeps; k += 2) {
      const int md = k == 0 ? mode : 0;
      const T* xcm = md == 2 ? xc : nullptr;
      if ((rc = launch(c, FCGMG_K_SWEEP_FUSED, l, s, [&] { return k_sweep_fused2<T>(c, L, x, b, xalt, md, xcm, s); })))
        return rc;
      if ((rc = launch(c, FCGMG_K_SWEEP_FUSED, l, s,
                       [&] { return k_sweep_fused2<T>(c, L, xalt, b, x, 0, (const T*)nullptr, s); })))
        return rc;
    }
    return FCGMG_OK;
  }
  for (int i = 0; i < sweeps; ++i)
    if ((rc = sweep_impl<D, T>(c, l, x, b, s, rbuf))) return rc;
  return FCGMG_OK;
}

// ---------------------------------------------------------------------------------------------
// Scratch of fcgmg_smooth_noalloc: one file-scope device array per GPU, held until the process
// ends. Host code never passes the array's name to a kernel (on the host it only stands in for the
// symbol): the device address comes from hipGetSymbolAddress, once per device, with that device
// current.
// ---------------------------------------------------------------------------------------------
constexpr size_t kNoAllocScratchDoubles = (size_t)12 << 20;  // 96 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(double** out) {
  int dev = -1;
  FCG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FCGMG_E_ARG, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    FCG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(FCGMG_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return FCGMG_OK;
}

template <class T = double>
int coarse_impl(const Ctx& c, const T* b, T* x, hipStream_t s) {
  const T* inv;
  if constexpr (std::is_same<T, double>::value)
    inv = c.coarse_inv;
  else
    inv = c.coarse_inv32;
  return launch(c, FCGMG_K_COARSE, 0, s, [&] { return k_dense_matvec<T>(inv, c.coarse_n, b, x, s); });
}

template <int D, class T = double>
int restrict_impl(const Ctx& c, int l, const T* rf, T* bc, hipStream_t s) {
  return launch(c, FCGMG_K_RESTRICT, l, s, [&] { return k_restrict<D, T>(c, l, rf, bc, s); });
}

// One V-cycle on level l (Sec. 3): pre-smoothing, restriction of the residual, the cycle on level
// l-1 from a zero initial guess, prolongation of its result, post-smoothing. `x_zero`: x holds zero
// on entry (its contents are not read). The coarsest solve writes every entry of its x.
template <int D, class T = double>
int vcycle_impl(const Ctx& c, int l, T* x, const T* b, hipStream_t s, bool x_zero = false) {
  if (l == 0) return coarse_impl<T>(c, b, x, s);
  int rc;
  if ((rc = smooth_impl<D, T>(c, l, x, b, c.prm.nu_pre, s, x_zero ? 1 : 0))) return rc;
  const Level& L = c.lev[l];
  const Level& C = c.lev[l - 1];
  T* cx = LV<T>::x(C);
  T* cb = LV<T>::b(C);
  if (D == 2) {
    if ((rc = launch(c, FCGMG_K_RESIDUAL_RESTRICT, l, s, [&] { return k_residual_restrict2<T>(c, L, x, b, cb, s); })))
      return rc;
  } else {
    T* r = LV<T>::r(L);
    if ((rc = residual_impl<D, T>(c, l, x, b, r, s))) return rc;
    if ((rc = restrict_impl<D, T>(c, l, r, cb, s))) return rc;
  }
  if ((rc = vcycle_impl<D, T>(c, l - 1, cx, cb, s, true))) return rc;
  return smooth_impl<D, T>(c, l, x, b, c.prm.nu_post, s, 2, cx);
}

// The sweeps of one level for nrhs vectors of one geometry (vectors nd apart): per sweep the
// residual and the shared-class rows per vector, then one stacked launch that streams each individual
// patch's rows once for all vectors. Per vector the arithmetic is that of sweep_impl.
template <int D>
int sweeps_multi(const Ctx& c, int l, double* x, const double* b, double* r, int nrhs, int sweeps, hipStream_t s) {
  const Level& L = c.lev[l];
  const int64_t nd = (D + 1) * L.N;
  int rc;
  // 3D: the shared-class applies on the handle's second stream, beside the stacked streamed apply
  // (disjoint nodes, both read only r), as in sweep_impl
  const bool fork = D == 3 && c.side && L.n_classes && L.n_irr;
  const hipStream_t sr = fork ? c.side : s;
  for (int it = 0; it < sweeps; ++it) {
    // the residuals and the shared-class applies of all vectors, one launch each
    if ((rc = launch(c, FCGMG_K_RESIDUAL, l, s, [&] { return k_residual<D, double>(c, L, x, b, r, s, nrhs, nd); })))
      return rc;
    if (fork) {
      FCG_HIP(hipEventRecord(c.ev_fork, s));
      FCG_HIP(hipStreamWaitEvent(c.side, c.ev_fork, 0));
    }
    if (L.n_classes)
      if ((rc = launch(c, FCGMG_K_APPLY_REGULAR, l, sr,
                       [&] { return k_apply_regular<D, double>(c, L, r, x, sr, nrhs, nd); })))
        return rc;
    if (fork) FCG_HIP(hipEventRecord(c.ev_join, c.side));
    if (L.n_irr)
      if ((rc = launch(c, FCGMG_K_APPLY_IRREGULAR, l, s,
                       [&] { return k_apply_irregular_multi<D, double>(c, L, r, x, nd, nrhs, s); })))
        return rc;
    if (fork) FCG_HIP(hipStreamWaitEvent(s, c.ev_join, 0));
  }
  return FCGMG_OK;
}

// The coarsest solve of coarse_impl for nrhs vectors (b, x coarse_n apart), one launch.
int coarse_multi(const Ctx& c, const double* b, double* x, int nrhs, hipStream_t s) {
  return launch(c, FCGMG_K_COARSE, 0, s, [&] { return k_dense_matvec_multi(c.coarse_inv, c.coarse_n, b, x, nrhs, s); });
}

// The sweeps of smooth_impl (2D, FP64, cache_inverse) for nrhs vectors of one level, nd apart: the
// entry mode and an odd first sweep are taken as smooth_impl takes them, then pairs of stacked fused
// sweeps between x and alt (nrhs vectors of scratch). xc: the coarse vectors of mode 2, ndc apart.
// Per vector the result is that of smooth_impl.
int smooth_multi2(const Ctx& c, int l, double* x, const double* b, double* alt, int nrhs, int sweeps, hipStream_t s,
                  int mode = 0, const double* xc = nullptr, int64_t ndc = 0) {
  const Level& L = c.lev[l];
  const int64_t nd = 3 * L.N;
  int rc;
  if (mode != 0 && (sweeps % 2 == 1 || sweeps == 0)) {
    if (mode == 1)
      rc = launch(c, FCGMG_K_ZERO, l, s, [&] { return k_zero<double>(x, nrhs * nd, s); });
    else
      rc = launch(c, FCGMG_K_PROLONG, l, s, [&] { return k_prolong_add<2, double>(c, l, xc, x, s, nrhs, ndc, nd); });
    if (rc) return rc;
    mode = 0;
  }
  int i = 0;
  if (sweeps % 2 == 1) {
    for (int k = 0; k < nrhs; ++k)
      if ((rc = sweep_impl<2, double>(c, l, x + k * nd, b + k * nd, s))) return rc;
    i = 1;
  }
  for (; i < sweeps; i += 2) {
    const int md = i == 0 ? mode : 0;
    const double* xcm = md == 2 ? xc : nullptr;
    if ((rc = launch(c, FCGMG_K_SWEEP_FUSED, l, s,
                     [&] { return k_sweep_fused2_multi(c, L, x, b, alt, md, xcm, nrhs, nd, ndc, s); })))
      return rc;
    if ((rc = launch(c, FCGMG_K_SWEEP_FUSED, l, s,
                     [&] { return k_sweep_fused2_multi(c, L, alt, b, x, 0, nullptr, nrhs, nd, ndc, s); })))
      return rc;
  }
  return FCGMG_OK;
}

// The V-cycle of vcycle_impl (2D, fused sweeps) for nrhs vectors of one geometry: the smoothing of
// every level by stacked fused sweeps, the residual + restriction and the coarsest solve per vector.
// The coarse levels use the handle's multi-vector workspace. Per vector the result is that of
// vcycle_impl.
int vcycle_multi2(const Ctx& c, int l, double* x, const double* b, int nrhs, hipStream_t s, bool x_zero) {
  const Level& L = c.lev[l];
  const int64_t nd = 3 * L.N;
  int rc;
  if (l == 0) return coarse_multi(c, b, x, nrhs, s);
  if ((rc = smooth_multi2(c, l, x, b, L.rm, nrhs, c.prm.nu_pre, s, x_zero ? 1 : 0))) return rc;
  const Level& C = c.lev[l - 1];
  const int64_t ndc = 3 * C.N;
  if ((rc = launch(c, FCGMG_K_RESIDUAL_RESTRICT, l, s,
                   [&] { return k_residual_restrict2_multi(L, x, b, C.bm, nrhs, nd, ndc, s); })))
    return rc;
  if ((rc = vcycle_multi2(c, l - 1, C.xm, C.bm, nrhs, s, true))) return rc;
  return smooth_multi2(c, l, x, b, L.rm, nrhs, c.prm.nu_post, s, 2, C.xm, ndc);
}

// The V-cycle of vcycle_impl (3D, unfused sweeps) for nrhs vectors of one geometry: every step per
// vector, except the streamed patch rows, which each sweep reads once for all vectors. The coarse
// levels use the handle's multi-vector workspace. Per vector the result is that of vcycle_impl.
template <int D>
int vcycle_multi_impl(const Ctx& c, int l, double* x, const double* b, int nrhs, hipStream_t s, bool x_zero) {
  const Level& L = c.lev[l];
  const int64_t nd = (D + 1) * L.N;
  int rc;
  if (l == 0) return coarse_multi(c, b, x, nrhs, s);
  // the vectors lie one after another: zeroing, residuals and transfers take all of them in one launch
  if (x_zero)
    if ((rc = launch(c, FCGMG_K_ZERO, l, s, [&] { return k_zero<double>(x, nrhs * nd, s); }))) return rc;
  if ((rc = sweeps_multi<D>(c, l, x, b, L.rm, nrhs, c.prm.nu_pre, s))) return rc;
  const Level& C = c.lev[l - 1];
  const int64_t ndc = (D + 1) * C.N;
  if ((rc = launch(c, FCGMG_K_RESIDUAL, l, s, [&] { return k_residual<D, double>(c, L, x, b, L.rm, s, nrhs, nd); })))
    return rc;
  if ((rc = launch(c, FCGMG_K_RESTRICT, l, s,
                   [&] { return k_restrict<D, double>(c, l, L.rm, C.bm, s, nrhs, nd, ndc); })))
    return rc;
  if ((rc = vcycle_multi_impl<D>(c, l - 1, C.xm, C.bm, nrhs, s, true))) return rc;
  if ((rc = launch(c, FCGMG_K_PROLONG, l, s,
                   [&] { return k_prolong_add<D, double>(c, l, C.xm, x, s, nrhs, ndc, nd); })))
    return rc;
  return sweeps_multi<D>(c, l, x, b, L.rm, nrhs, c.prm.nu_post, s);
}

// Allocate the multi-vector workspace (kMaxRhs vectors of r on every level, of x and b on the coarse
// levels) on first use; it stays with the handle.
int multi_workspace(Ctx& c) {
  if (c.multi_ready) return FCGMG_OK;
  const int nlev = (int)c.lev.size();
  int rc;
  for (int l = 0; l < nlev; ++l) {
    Level& L = c.lev[l];
    const size_t nd = (size_t)(c.prm.dim + 1) * (size_t)L.N;
    if ((rc = alloc_n(c, &L.rm, (size_t)kMaxRhs * nd))) return rc;
    if (l < nlev - 1) {
      if ((rc = alloc_n(c, &L.xm, (size_t)kMaxRhs * nd))) return rc;
      if ((rc = alloc_n(c, &L.bm, (size_t)kMaxRhs * nd))) return rc;
    }
  }
  c.multi_ready = true;
  return FCGMG_OK;
}

// x += V32(0, r): the FP32 V-cycle on the residual equation of the finest level from a zero guess
// (mixed precision). r is rounded into the finest level's FP32 right-hand side, the correction
// widened and added to the FP64 x.
template <int D>
int correction_fp32_impl(const Ctx& c, const double* r, double* x, hipStream_t s) {
  const int top = (int)c.lev.size() - 1;
  const Level& L = c.lev[top];
  const int64_t nd = (D + 1) * L.N;
  FCG_HIP(k_round_to_float(r, L.b32, nd, s));
  int rc;
  if ((rc = vcycle_impl<D, float>(c, top, L.x32, L.b32, s, true))) return rc;
  FCG_HIP(k_add_float(L.x32, x, nd, s));
  return FCGMG_OK;
}

// Cell kinds of a level on the host, as box_kind gives them cell by cell (0 physical, 1 inside a
// ball, 2 cut), but visiting each ball's bounding box of cells only: a cell outside it is at least
// the radius away from the ball in one axis, so that ball neither contains nor cuts it.
template <int D>
void classify_cells_host(const Geom& g, const Level& L, std::vector<signed char>& kinds) {
  kinds.assign(L.ncells, 0);
  std::vector<unsigned char> inside(L.ncells, 0);
  for (int i = 0; i < g.nballs; ++i) {
    const double* b = g.balls + 4 * i;
    int lo_c[3] = {0, 0, 0}, hi_c[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) {
      lo_c[k] = std::max(0, (int)std::floor((b[k] - b[3]) / L.h) - 1);
      hi_c[k] = std::min(L.n - 1, (int)std::floor((b[k] + b[3]) / L.h) + 1);
    }
    for (int z = lo_c[2]; z <= hi_c[2]; ++z)
      for (int y = lo_c[1]; y <= hi_c[1]; ++y)
        for (int x = lo_c[0]; x <= hi_c[0]; ++x) {
          const int64_t cell = x + (int64_t)L.n * (y + (int64_t)L.n * z);
          const double lo[3] = {(double)x * L.h, (double)y * L.h, D == 3 ? (double)z * L.h : 0.0};
          const Geom one{b, 1, g.q, g.alpha_f};
          const int kd = box_kind<D>(one, lo, L.h);
          if (kd == 1) inside[cell] = 1;
          else if (kd == 2) kinds[cell] = 2;
        }
  }
  for (int64_t cell = 0; cell < L.ncells; ++cell)
    if (inside[cell]) kinds[cell] = 1;
}

// Device bytes that setup_impl would allocate, from the same host-side planning (cell kinds by the
// exact ball-box test on the host, operator codes, patch classes, fused-sweep plan). Temporaries
// freed during set-up are not counted.
template <int D>
size_t footprint_impl(const fcgmg_params& P, const std::vector<double>& balls) {
  const int nlev = P.n_levels;
  const bool inverse = P.cache_policy == FCGMG_CACHE_INVERSE;
  const bool mixed = P.precision == FCGMG_PREC_MIXED;
  size_t bytes = sizeof(int) + balls.size() * sizeof(double) + (kRedBlocks + 1) * sizeof(double);
  size_t n_pattern = 0;
  if (P.cache_policy == FCGMG_CACHE_MATRIX) {
    std::vector<int> enc;
    pattern_entries<D>(enc);
    n_pattern = enc.size();
    bytes += n_pattern * sizeof(int);
  }
  const Geom g{balls.data(), (int)balls.size() / 4, P.quad_depth, P.alpha_fict};
  int64_t nd0 = 0;
  for (int l = 0; l < nlev; ++l) {
    Level L;
    L.n = P.n_cells >> (nlev - 1 - l);
    L.h = 1.0 / L.n;
    L.N = 1;
    L.ncells = 1;
    for (int k = 0; k < D; ++k) {
      L.N *= (L.n + 1);
      L.ncells *= L.n;
    }
    const size_t nd = (size_t)(D + 1) * L.N;
    if (l == 0) nd0 = (int64_t)nd;
    bytes += nd * sizeof(double) * (l < nlev - 1 ? 3 : 1);
    if (D == 2 && inverse) bytes += nd * sizeof(double);
    std::vector<signed char> kinds;
    classify_cells_host<D>(g, L, kinds);
    const int64_t n_cut = std::count(kinds.begin(), kinds.end(), (signed char)2);
    bytes += L.ncells * sizeof(int) + (size_t)n_cut * PT<D>::NEL * sizeof(double) + sizeof(OpConsts);
    std::vector<int> op(L.N), sten, ncls, reps, irr, zrow, znodes, extra;
    node_operator_codes<D>(L, kinds, op, sten);
    bytes += L.N * sizeof(int) + sten.size() * PT<D>::NSTEN * sizeof(double);
    classify_patches<D>(L, kinds, inverse, ncls, reps, irr, zrow, znodes);
    bytes += (L.N + reps.size() + 2 * irr.size() + znodes.size()) * sizeof(int);
    const size_t npatch = reps.size() + znodes.size();  // blocks with stored data
    if (D == 2 && inverse) {
      plan_fused2(L, ncls, extra);
      bytes += extra.size() * sizeof(int);
    }
    if (inverse) {
      const size_t row = (size_t)(D + 1) * PT<D>::ZSP;
      bytes += npatch * row * sizeof(double);
      if (mixed)
        bytes += (npatch * row + sten.size() * PT<D>::NSTEN + nd * (D == 2 ? 4 : 3)) * sizeof(float);
    } else if (P.cache_policy == FCGMG_CACHE_MATRIX) {
      bytes += npatch * n_pattern * sizeof(double);
    }
  }
  bytes += (size_t)nd0 * nd0 * (sizeof(double) + (mixed ? sizeof(float) : 0));
  if (P.solver == FCGMG_SOLVER_FGMRES) {
    int64_t N = 1;
    for (int k = 0; k < D; ++k) N *= P.n_cells + 1;
    bytes += ((size_t)(2 * P.krylov_restart + 3) * (D + 1) * N + kKrylovPartials + 192) * sizeof(double);
  }
  return bytes;
}

int norm_impl(const Ctx& c, const double* v, int64_t n, double* out, hipStream_t s);

// z = M^{-1} v: one V-cycle on the residual equation from a zero guess, FP64 or (mixed) FP32.
template <int D>
int precond_impl(const Ctx& c, const double* v, double* z, hipStream_t s) {
  const int top = (int)c.lev.size() - 1;
  if (c.prm.precision == FCGMG_PREC_MIXED) {
    FCG_HIP(k_zero<double>(z, (D + 1) * c.lev[top].N, s));
    return correction_fp32_impl<D>(c, v, z, s);
  }
  return vcycle_impl<D>(c, top, z, v, s, true);
}

// Flexible GMRES(m) with right preconditioning (Saad's FGMRES): Arnoldi on A M^{-1} with the
// preconditioned directions z_j kept, classical Gram-Schmidt twice per step (one device
// reduction each), Givens rotations and the small least-squares problem on the host. Stops when
// the Arnoldi estimate of ||b - A x|| reaches rtol * r0; the true residual is recomputed at every
// restart and decides. hist[k] is the estimate after k preconditioner applications.
template <int D>
int fgmres_impl(const Ctx& c, double* x, const double* b, double rtol, int max_iter, int* iters, double* rel_res,
                double* hist, hipStream_t s) {
  const int top = (int)c.lev.size() - 1;
  const int64_t nd = (D + 1) * c.lev[top].N;
  const int m = c.prm.krylov_restart;
  int rc;
  auto Vv = [&](int i) { return c.kv + (int64_t)i * nd; };
  auto Zv = [&](int i) { return c.kz + (int64_t)i * nd; };
  double r0, beta;
  if ((rc = residual_impl<D>(c, top, x, b, Vv(0), s))) return rc;
  if ((rc = norm_impl(c, Vv(0), nd, &r0, s))) return rc;
  if (hist) hist[0] = r0;
  *iters = 0;
  *rel_res = 0;
  if (!std::isfinite(r0)) return fail(FCGMG_E_NAN, "non-finite initial residual");
  if (r0 == 0.0) return FCGMG_OK;
  beta = r0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h(m + 1), h2(m + 1);
  int its = 0;
  for (;;) {
    FCG_HIP(k_scale_copy(Vv(0), 1.0 / beta, Vv(0), nd, s));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    bool done = false;
    for (int j = 0; j < m && its < max_iter; ++j) {
      if ((rc = precond_impl<D>(c, Vv(j), Zv(j), s))) return rc;
      // w = A z_j = -(0 - A z_j)
      if ((rc = residual_impl<D>(c, top, Zv(j), c.kzero, c.kw, s))) return rc;
      // first pass: h = V^T (A z) = -V^T w; w <- A z - V h = -w - V h
      FCG_HIP(k_multi_dot(c.kv, nd, j + 1, c.kw, nd, -1.0, c.kpart, c.kh, s));
      FCG_HIP(k_multi_axpy(c.kw, -1.0, c.kv, nd, j + 1, c.kh, nd, s));
      FCG_HIP(hipMemcpyAsync(c.kh_host, c.kh, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
      // second pass: h2 = V^T w; w <- w - V h2
      FCG_HIP(k_multi_dot(c.kv, nd, j + 1, c.kw, nd, 1.0, c.kpart, c.kh + 64, s));
      FCG_HIP(k_multi_axpy(c.kw, 1.0, c.kv, nd, j + 1, c.kh + 64, nd, s));
      FCG_HIP(hipMemcpyAsync(c.kh_host + 64, c.kh + 64, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
      double hn;
      if ((rc = norm_impl(c, c.kw, nd, &hn, s))) return rc;  // synchronises: h, h2 are on the host
      std::copy(c.kh_host, c.kh_host + j + 1, h.begin());
      std::copy(c.kh_host + 64, c.kh_host + 64 + j + 1, h2.begin());
      ++its;
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i] + h2[i];
      H[(size_t)(j + 1) * m + j] = hn;
      if (!std::isfinite(hn)) return fail(FCGMG_E_NAN, "non-finite Arnoldi vector at cycle " + std::to_string(its));
      if (hn > 0) FCG_HIP(k_scale_copy(c.kw, 1.0 / hn, Vv(j + 1), nd, s));
      // apply the previous rotations to column j, then a new one that zeroes H[j+1][j]
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
      }
      const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
      const double rr = std::hypot(a, bb);
      cs[j] = rr > 0 ? a / rr : 1.0;
      sn[j] = rr > 0 ? bb / rr : 0.0;
      H[(size_t)j * m + j] = rr;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      const double est = std::fabs(g[j + 1]);
      if (hist) hist[its] = est;
      *iters = its;
      *rel_res = est / r0;
      if (est <= rtol * r0 || hn == 0.0) {
        done = true;
        break;
      }
    }
    // x += Z y with H(0:k, 0:k) y = g(0:k)
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= H[(size_t)i * m + l] * y[l];
      y[i] = acc / H[(size_t)i * m + i];
    }
    for (int i = 0; i < k; ++i) c.kh_host[128 + i] = -y[i];  // multi_axpy subtracts
    FCG_HIP(hipMemcpyAsync(c.kh, c.kh_host + 128, k * sizeof(double), hipMemcpyHostToDevice, s));
    FCG_HIP(k_multi_axpy(x, 1.0, c.kz, nd, k, c.kh, nd, s));
    if ((rc = residual_impl<D>(c, top, x, b, Vv(0), s))) return rc;
    if ((rc = norm_impl(c, Vv(0), nd, &beta, s))) return rc;  // synchronises: y may be reused
    *rel_res = beta / r0;
    if (hist) hist[its] = beta;
    if (!std::isfinite(beta)) return fail(FCGMG_E_NAN, "non-finite residual at cycle " + std::to_string(its));
    if (beta <= rtol * r0) return FCGMG_OK;
    if (its >= max_iter)
      return fail(FCGMG_E_NOCONV, "no convergence in " + std::to_string(max_iter) + " cycles (rel. residual " +
                                      sci(*rel_res) + ")");
    (void)done;  // the estimate converged but the true residual did not: restart
  }
}

int norm_impl(const Ctx& c, const double* v, int64_t n, double* out, hipStream_t s) {
  FCG_HIP(k_sumsq(v, n, c.red, kRedBlocks, s));
  // the single finishing block writes the total into the pinned host word (no copy launch)
  FCG_HIP(k_finish_sumsq(c.red, kRedBlocks, c.red_host_dev, s));
  FCG_HIP(hipStreamSynchronize(s));
  *out = std::sqrt(*static_cast<volatile double*>(c.red_host));
  return FCGMG_OK;
}

// Device buffers of the autotuner, freed on every exit path.
struct TuneBuffers {
  std::vector<void*> p;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~TuneBuffers() {
    for (void* q : p) (void)hipFree(q);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// Time `reps` pairs of fused sweeps on level l with the level's current shape and plan; returns
// microseconds per sweep.
int time_fused_pairs(const Ctx& c, const Level& L, double* x, const double* b, double* y, int reps, TuneBuffers& tb,
                     hipStream_t s, double* us) {
  for (int w = 0; w < 2; ++w) {
    FCG_HIP(k_sweep_fused2<double>(c, L, x, b, y, 0, nullptr, s));
    FCG_HIP(k_sweep_fused2<double>(c, L, y, b, x, 0, nullptr, s));
  }
  FCG_HIP(hipEventRecord(tb.e0, s));
  for (int r = 0; r < reps; ++r) {
    FCG_HIP(k_sweep_fused2<double>(c, L, x, b, y, 0, nullptr, s));
    FCG_HIP(k_sweep_fused2<double>(c, L, y, b, x, 0, nullptr, s));
  }
  FCG_HIP(hipEventRecord(tb.e1, s));
  FCG_HIP(hipEventSynchronize(tb.e1));
  float ms = 0.f;
  FCG_HIP(hipEventElapsedTime(&ms, tb.e0, tb.e1));
  *us = 1e3 * ms / (2.0 * reps);
  return FCGMG_OK;
}

// Upload the extra-workgroup plan of shape k for level L into its (grown if needed) plan buffer.
int install_fused_plan(Ctx& c, Level& L, int k, const std::vector<int>& extra, hipStream_t s) {
  if ((int)extra.size() > L.fused_extra_cap) {
    int* grown = nullptr;
    int rc;
    if ((rc = alloc_n(c, &grown, extra.size()))) return rc;
    if (L.fused_extra) {
      auto it = std::find(c.allocs.begin(), c.allocs.end(), (void*)L.fused_extra);
      if (it != c.allocs.end()) c.allocs.erase(it);
      FCG_HIP(hipStreamSynchronize(s));
      FCG_HIP(hipFree(L.fused_extra));
      c.bytes -= (size_t)L.fused_extra_cap * sizeof(int);
    }
    L.fused_extra = grown;
    L.fused_extra_cap = (int)extra.size();
  }
  L.fshape = k;
  L.n_fused_extra = (int)extra.size();
  if (!extra.empty()) {
    FCG_HIP(hipMemcpyAsync(L.fused_extra, extra.data(), extra.size() * sizeof(int), hipMemcpyHostToDevice, s));
    FCG_HIP(hipStreamSynchronize(s));  // `extra` is the caller's host vector
  }
  return FCGMG_OK;
}

// Per 2D cache_inverse level below the coarsest: time the fused sweep with every tile shape on a
// vector of the level's size (the sweep's cost depends on the patch layout, not on the values) and
// keep the fastest. All shapes compute the same numbers, so only the time changes.
int autotune_impl(Ctx& c, int reps, int* shape_out, double* us_out, hipStream_t s) {
  const int ns = fused2_num_shapes(), nlev = (int)c.lev.size();
  for (int l = 0; l < nlev; ++l) {
    shape_out[l] = c.lev[l].fshape;
    if (us_out)
      for (int k = 0; k < ns; ++k) us_out[(size_t)l * ns + k] = -1.0;
  }
  if (c.prm.dim != 2 || c.prm.cache_policy != FCGMG_CACHE_INVERSE) return FCGMG_OK;
  TuneBuffers tb;
  FCG_HIP(hipEventCreate(&tb.e0));
  FCG_HIP(hipEventCreate(&tb.e1));
  int rc;
  for (int l = 1; l < nlev; ++l) {
    Level& L = c.lev[l];
    if (!L.xalt) continue;
    const size_t nd = (size_t)3 * (size_t)L.N;
    double* v[3] = {nullptr, nullptr, nullptr};
    for (double*& q : v) {
      hipError_t e = hipMalloc((void**)&q, nd * sizeof(double));
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FCGMG_E_NOMEM, "autotune: hipMalloc of " + std::to_string(nd * sizeof(double)) + " bytes failed");
      }
      tb.p.push_back(q);
    }
    FCG_HIP(hipMemsetAsync(v[0], 0, nd * sizeof(double), s));
    FCG_HIP(hipMemsetAsync(v[1], 0x3f, nd * sizeof(double), s));  // every double 0x3f3f...: finite, positive
    std::vector<int> ncls((size_t)L.N);
    FCG_HIP(hipMemcpyAsync(ncls.data(), L.node_class, ncls.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    FCG_HIP(hipStreamSynchronize(s));
    int best = -1;
    double best_us = 0.0;
    std::vector<int> extra;
    for (int k = 0; k < ns; ++k) {
      L.fshape = k;
      plan_fused2(L, ncls, extra);
      if ((rc = install_fused_plan(c, L, k, extra, s))) return rc;
      double us = 0.0;
      if ((rc = time_fused_pairs(c, L, v[0], v[1], v[2], reps, tb, s, &us))) return rc;
      if (us_out) us_out[(size_t)l * ns + k] = us;
      if (best < 0 || us < best_us) {
        best = k;
        best_us = us;
      }
    }
    L.fshape = best;
    plan_fused2(L, ncls, extra);
    if ((rc = install_fused_plan(c, L, best, extra, s))) return rc;
    shape_out[l] = best;
    for (double* q : v) {
      tb.p.erase(std::find(tb.p.begin(), tb.p.end(), (void*)q));
      FCG_HIP(hipFree(q));
    }
  }
  return FCGMG_OK;
}

// Give level l fused-sweep shape k (-1: default by size) and rebuild its plan.
int set_fused_shape_impl(Ctx& c, int l, int k, hipStream_t s) {
  Level& L = c.lev[l];
  if (c.prm.dim != 2 || c.prm.cache_policy != FCGMG_CACHE_INVERSE || !L.xalt)
    return fail(FCGMG_E_ARG, "the fused sweep runs on 2D cache_inverse levels only");
  std::vector<int> ncls((size_t)L.N), extra;
  FCG_HIP(hipMemcpyAsync(ncls.data(), L.node_class, ncls.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  FCG_HIP(hipStreamSynchronize(s));
  L.fshape = k;
  plan_fused2(L, ncls, extra);
  return install_fused_plan(c, L, k, extra, s);
}

bool valid_level(const Ctx* c, int l) { return c && l >= 0 && l < (int)c->lev.size(); }

}  // namespace


int fcg::set_error(int code, const std::string& msg) { return fail(code, msg); }

// Argument checks shared by set-up and the footprint estimate.
static int validate_params(const fcgmg_params& prm, const double* balls, int n_balls) {
  const fcgmg_params& P = prm;
  if (P.dim != 2 && P.dim != 3) return fail(FCGMG_E_ARG, "dim must be 2 or 3");
  if (P.n_levels < 1 || P.n_levels > 20) return fail(FCGMG_E_ARG, "n_levels out of range");
  if (P.n_cells < 1 || ((P.n_cells >> (P.n_levels - 1)) << (P.n_levels - 1)) != P.n_cells)
    return fail(FCGMG_E_ARG, "n_cells must be a positive multiple of 2^(n_levels-1)");
  if ((int64_t)P.n_cells + 1 > (P.dim == 2 ? 46340 : 1290))
    return fail(FCGMG_E_ARG, "grid too large for 32-bit node indices");
  if (P.quad_depth < 0 || P.quad_depth > 7) return fail(FCGMG_E_ARG, "quad_depth must be in [0,7]");
  if (P.quad_depth + P.n_levels - 1 > fcg::kMaxTreeDepth)
    return fail(FCGMG_E_ARG, "quad_depth + n_levels - 1 exceeds the deepest space tree (20)");
  if (P.cache_policy < 0 || P.cache_policy > 2) return fail(FCGMG_E_ARG, "unknown cache policy");
  if (P.precision != FCGMG_PREC_FP64 && P.precision != FCGMG_PREC_MIXED)
    return fail(FCGMG_E_ARG, "unknown precision");
  if (P.precision == FCGMG_PREC_MIXED && P.cache_policy != FCGMG_CACHE_INVERSE)
    return fail(FCGMG_E_ARG, "mixed precision needs the cache_inverse policy");
  if (P.solver != FCGMG_SOLVER_GMG && P.solver != FCGMG_SOLVER_FGMRES) return fail(FCGMG_E_ARG, "unknown solver");
  if (P.solver == FCGMG_SOLVER_FGMRES && (P.krylov_restart < 1 || P.krylov_restart > 63))
    return fail(FCGMG_E_ARG, "krylov_restart must be in [1,63]");
  if (P.immersed_nitsche != 0 && P.immersed_nitsche != 1) return fail(FCGMG_E_ARG, "immersed_nitsche must be 0 or 1");
  if (P.immersed_nitsche && P.dim == 3 && P.cache_policy != FCGMG_CACHE_INVERSE)
    return fail(FCGMG_E_ARG, "immersed_nitsche in 3D needs the cache_inverse policy");
  if (!(P.eta > 0) || !(P.alpha_fict >= 0) || !(P.nitsche_beta > 0) || !std::isfinite(P.omega))
    return fail(FCGMG_E_ARG, "eta, nitsche_beta must be > 0, alpha_fict >= 0, omega finite");
  if (P.nu_pre < 0 || P.nu_post < 0) return fail(FCGMG_E_ARG, "negative smoothing steps");
  for (int k = 0; k < 6; ++k)
    if (P.bc[k] < 0 || P.bc[k] > 2) return fail(FCGMG_E_ARG, "unknown boundary code");
  if (n_balls < 0 || (n_balls > 0 && !balls)) return fail(FCGMG_E_ARG, "bad obstacle list");
  for (int i = 0; i < n_balls; ++i)
    if (!(balls[4 * i + 3] > 0)) return fail(FCGMG_E_ARG, "obstacle radius must be > 0");
  return FCGMG_OK;
}

extern "C" {

const char* fcgmg_last_error(void) { return g_err.c_str(); }

void fcgmg_destroy(fcgmg_h h) {
  if (!h) return;
  for (const Ctx::ProfRec& r : h->prof_pending) {
    (void)hipEventSynchronize(r.stop);
    h->prof_pool.push_back(r.start);
    h->prof_pool.push_back(r.stop);
  }
  for (hipEvent_t e : h->prof_pool) (void)hipEventDestroy(e);
  if (h->side) {
    (void)hipStreamSynchronize(h->side);
    (void)hipStreamDestroy(h->side);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->red_host) (void)hipHostFree(h->red_host);
  if (h->kh_host) (void)hipHostFree(h->kh_host);
  delete h;
}

int fcgmg_footprint_bytes(const fcgmg_params* prm, const double* balls, int n_balls, size_t* bytes) {
  g_err.clear();
  if (!prm || !bytes) return fail(FCGMG_E_ARG, "null argument");
  int rc;
  if ((rc = validate_params(*prm, balls, n_balls))) return rc;
  const std::vector<double> bh(balls, balls + 4 * (size_t)n_balls);
  *bytes = prm->dim == 2 ? footprint_impl<2>(*prm, bh) : footprint_impl<3>(*prm, bh);
  return FCGMG_OK;
}

int fcgmg_setup_hierarchy(const fcgmg_params* prm, const double* balls, int n_balls, void* stream, fcgmg_h* out) {
  g_err.clear();
  if (!prm || !out) return fail(FCGMG_E_ARG, "null argument");
  *out = nullptr;
  int rc0;
  if ((rc0 = validate_params(*prm, balls, n_balls))) return rc0;
  const fcgmg_params& P = *prm;
  fcgmg_ctx* c = new fcgmg_ctx();
  c->prm = P;
  c->balls_h.assign(balls, balls + 4 * (size_t)n_balls);
  hipStream_t s = (hipStream_t)stream;
  const int rc = P.dim == 2 ? setup_impl<2>(*c, s) : setup_impl<3>(*c, s);
  if (rc != FCGMG_OK) {
    std::string keep = g_err;
    (void)hipStreamSynchronize(s);
    fcgmg_destroy(c);
    g_err = keep;
    return rc;
  }
  *out = c;
  return FCGMG_OK;
}

int fcgmg_num_levels(fcgmg_h h, int* n) {
  if (!h || !n) return fail(FCGMG_E_ARG, "null argument");
  *n = (int)h->lev.size();
  return FCGMG_OK;
}

int fcgmg_num_dofs(fcgmg_h h, int level, int64_t* n) {
  if (!valid_level(h, level) || !n) return fail(FCGMG_E_ARG, "bad handle or level");
  *n = (h->prm.dim + 1) * h->lev[level].N;
  return FCGMG_OK;
}

int fcgmg_level_stats_get(fcgmg_h h, int level, fcgmg_level_stats* o) {
  if (!valid_level(h, level) || !o) return fail(FCGMG_E_ARG, "bad handle or level");
  const Level& L = h->lev[level];
  o->n_cells_axis = L.n;
  o->n_nodes = L.N;
  o->n_cut_cells = L.n_cut;
  o->n_fict_cells = L.n_fict;
  o->n_classes = L.n_classes;
  o->n_irregular = L.n_irr;
  o->irregular_cols = L.irr_cols;
  o->cached_bytes = (int64_t)L.cached_bytes;
  o->n_stencils = L.n_nsten;
  return FCGMG_OK;
}

int fcgmg_rhs(fcgmg_h h, int level, double* b, void* stream) {
  if (!valid_level(h, level) || !b) return fail(FCGMG_E_ARG, "bad handle, level or pointer");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = h->prm.dim == 2 ? k_rhs<2>(*h, h->lev[level], b, s) : k_rhs<3>(*h, h->lev[level], b, s);
  if (e != hipSuccess) return fail(FCGMG_E_HIP, std::string("rhs: ") + hipGetErrorString(e));
  return FCGMG_OK;
}

int fcgmg_residual(fcgmg_h h, int level, const double* x, const double* b, double* r, void* stream) {
  if (!valid_level(h, level) || !x || !b || !r) return fail(FCGMG_E_ARG, "bad handle, level or pointer");
  if (r == x || r == b) return fail(FCGMG_E_ARG, "r must not alias x or b");
  hipStream_t s = (hipStream_t)stream;
  return h->prm.dim == 2 ? residual_impl<2>(*h, level, x, b, r, s) : residual_impl<3>(*h, level, x, b, r, s);
}

int fcgmg_smooth(fcgmg_h h, int level, double* x, const double* b, int sweeps, void* stream) {
  if (!valid_level(h, level) || !x || !b || sweeps < 0) return fail(FCGMG_E_ARG, "bad handle, level or pointer");
  hipStream_t s = (hipStream_t)stream;
  return h->prm.dim == 2 ? smooth_impl<2>(*h, level, x, b, sweeps, s) : smooth_impl<3>(*h, level, x, b, sweeps, s);
}

int fcgmg_smooth_noalloc(fcgmg_h h, int level, double* x, const double* b, int sweeps, void* stream) {
  if (!valid_level(h, level) || !x || !b || sweeps < 0) return fail(FCGMG_E_ARG, "bad handle, level or pointer");
  const Level& L = h->lev[level];
  const size_t nd = (size_t)(h->prm.dim + 1) * (size_t)L.N;
  const size_t nd_pad = (nd + 31) / 32 * 32;  // second buffer on a 256-byte boundary
  const size_t need = nd_pad + (L.xalt ? nd : 0);
  if (need > kNoAllocScratchDoubles)
    return fail(FCGMG_E_ARG, "level needs " + std::to_string(need) + " doubles of scratch; the static scratch holds " +
                                 std::to_string(kNoAllocScratchDoubles));
  double* base = nullptr;
  int rc;
  if ((rc = scratch_for_current_device(&base))) return rc;
  double* rbuf = base;
  double* abuf = L.xalt ? base + nd_pad : nullptr;
  hipStream_t s = (hipStream_t)stream;
  return h->prm.dim == 2 ? smooth_impl<2, double>(*h, level, x, b, sweeps, s, 0, nullptr, rbuf, abuf)
                         : smooth_impl<3, double>(*h, level, x, b, sweeps, s, 0, nullptr, rbuf, abuf);
}

int fcgmg_smooth_multi(fcgmg_h h, int level, double* x, const double* b, double* r, int nrhs, int sweeps,
                       void* stream) {
  if (!valid_level(h, level) || !x || !b || !r || sweeps < 0) return fail(FCGMG_E_ARG, "bad handle, level or pointer");
  if (nrhs < 1 || nrhs > fcg::kMaxRhs) return fail(FCGMG_E_ARG, "nrhs must be in [1,8]");
  if (h->prm.cache_policy != FCGMG_CACHE_INVERSE) return fail(FCGMG_E_ARG, "smooth_multi needs the cache_inverse policy");
  hipStream_t s = (hipStream_t)stream;
  auto run = [&](auto dim) -> int {
    constexpr int D = decltype(dim)::value;
    const fcg::Ctx& c = *h;
    const fcg::Level& L = c.lev[level];
    const int64_t nd = (D + 1) * L.N;
    if constexpr (D == 2) {
      // 2D: stacked fused sweeps (r serves as the second iterate of each vector)
      (void)nd;
      return smooth_multi2(c, level, x, b, r, nrhs, sweeps, s);
    }
    return sweeps_multi<D>(c, level, x, b, r, nrhs, sweeps, s);
  };
  return h->prm.dim == 2 ? run(std::integral_constant<int, 2>{}) : run(std::integral_constant<int, 3>{});
}

int fcgmg_vcycle_multi(fcgmg_h h, double* x, const double* b, int nrhs, void* stream) {
  if (!h || !x || !b) return fail(FCGMG_E_ARG, "bad handle or pointer");
  if (nrhs < 1 || nrhs > fcg::kMaxRhs) return fail(FCGMG_E_ARG, "nrhs must be in [1,8]");
  if (h->prm.cache_policy != FCGMG_CACHE_INVERSE) return fail(FCGMG_E_ARG, "vcycle_multi needs the cache_inverse policy");
  hipStream_t s = (hipStream_t)stream;
  const int top = (int)h->lev.size() - 1;
  const int64_t nd = (int64_t)(h->prm.dim + 1) * h->lev[top].N;
  int rc;
  (void)nd;
  if ((rc = multi_workspace(*h))) return rc;
  if (h->prm.dim == 2) return vcycle_multi2(*h, top, x, b, nrhs, s, false);
  return vcycle_multi_impl<3>(*h, top, x, b, nrhs, s, false);
}

int fcgmg_restrict(fcgmg_h h, int fine_level, const double* rf, double* bc, void* stream) {
  if (!valid_level(h, fine_level) || fine_level < 1 || !rf || !bc) return fail(FCGMG_E_ARG, "bad level or pointer");
  hipStream_t s = (hipStream_t)stream;
  return h->prm.dim == 2 ? restrict_impl<2>(*h, fine_level, rf, bc, s) : restrict_impl<3>(*h, fine_level, rf, bc, s);
}

int fcgmg_prolongate_add(fcgmg_h h, int fine_level, const double* ec, double* xf, void* stream) {
  if (!valid_level(h, fine_level) || fine_level < 1 || !ec || !xf) return fail(FCGMG_E_ARG, "bad level or pointer");
  hipStream_t s = (hipStream_t)stream;
  return h->prm.dim == 2 ? prolong_impl<2>(*h, fine_level, ec, xf, s) : prolong_impl<3>(*h, fine_level, ec, xf, s);
}

int fcgmg_coarse_solve(fcgmg_h h, const double* b, double* x, void* stream) {
  if (!h || !b || !x) return fail(FCGMG_E_ARG, "null argument");
  return coarse_impl(*h, b, x, (hipStream_t)stream);
}

int fcgmg_vcycle(fcgmg_h h, double* x, const double* b, void* stream) {
  if (!h || !x || !b) return fail(FCGMG_E_ARG, "null argument");
  hipStream_t s = (hipStream_t)stream;
  const int top = (int)h->lev.size() - 1;
  return h->prm.dim == 2 ? vcycle_impl<2>(*h, top, x, b, s) : vcycle_impl<3>(*h, top, x, b, s);
}

int fcgmg_vcycle_fp32(fcgmg_h h, const double* r, double* e, void* stream) {
  if (!h || !r || !e) return fail(FCGMG_E_ARG, "null argument");
  if (h->prm.precision != FCGMG_PREC_MIXED) return fail(FCGMG_E_ARG, "hierarchy not set up for mixed precision");
  hipStream_t s = (hipStream_t)stream;
  const Level& L = h->lev.back();
  FCG_HIP(k_zero<double>(e, (h->prm.dim + 1) * L.N, s));
  return h->prm.dim == 2 ? correction_fp32_impl<2>(*h, r, e, s) : correction_fp32_impl<3>(*h, r, e, s);
}

int fcgmg_norm(fcgmg_h h, int level, const double* v, double* out, void* stream) {
  if (!valid_level(h, level) || !v || !out) return fail(FCGMG_E_ARG, "bad handle, level or pointer");
  return norm_impl(*h, v, (h->prm.dim + 1) * h->lev[level].N, out, (hipStream_t)stream);
}

int fcgmg_solve(fcgmg_h h, double* x, const double* b, double rtol, int max_iter, int* iters, double* rel_res,
                double* res_hist, void* stream) {
  if (!h || !x || !b || !iters || !rel_res || max_iter < 0 || !(rtol >= 0))
    return fail(FCGMG_E_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  if (h->prm.solver == FCGMG_SOLVER_FGMRES)
    return h->prm.dim == 2 ? fgmres_impl<2>(*h, x, b, rtol, max_iter, iters, rel_res, res_hist, s)
                           : fgmres_impl<3>(*h, x, b, rtol, max_iter, iters, rel_res, res_hist, s);
  const int top = (int)h->lev.size() - 1;
  const Level& L = h->lev[top];
  const int64_t nd = (h->prm.dim + 1) * L.N;
  int rc;
  *iters = 0;
  *rel_res = 0;
  double r0;
  if ((rc = h->prm.dim == 2 ? residual_impl<2>(*h, top, x, b, L.r, s) : residual_impl<3>(*h, top, x, b, L.r, s)))
    return rc;
  if ((rc = norm_impl(*h, L.r, nd, &r0, s))) return rc;
  if (res_hist) res_hist[0] = r0;
  if (!std::isfinite(r0)) return fail(FCGMG_E_NAN, "non-finite initial residual");
  if (r0 == 0.0) return FCGMG_OK;
  const bool mixed = h->prm.precision == FCGMG_PREC_MIXED;
  for (int it = 1; it <= max_iter; ++it) {
    if (mixed)  // FP64 iterative refinement: L.r holds b - L x of the current iterate
      rc = h->prm.dim == 2 ? correction_fp32_impl<2>(*h, L.r, x, s) : correction_fp32_impl<3>(*h, L.r, x, s);
    else
      rc = fcgmg_vcycle(h, x, b, stream);
    if (rc) return rc;
    if ((rc = h->prm.dim == 2 ? residual_impl<2>(*h, top, x, b, L.r, s) : residual_impl<3>(*h, top, x, b, L.r, s)))
      return rc;
    double rn;
    if ((rc = norm_impl(*h, L.r, nd, &rn, s))) return rc;
    if (res_hist) res_hist[it] = rn;
    *iters = it;
    *rel_res = rn / r0;
    if (!std::isfinite(rn)) return fail(FCGMG_E_NAN, "non-finite residual at cycle " + std::to_string(it));
    if (rn <= rtol * r0) return FCGMG_OK;
  }
  return fail(FCGMG_E_NOCONV, "no convergence in " + std::to_string(max_iter) + " cycles (rel. residual " +
                                  sci(*rel_res) + ")");
}

int fcgmg_autotune(fcgmg_h h, int reps, int* shape_out, double* us_out, void* stream) {
  if (!h || !shape_out || reps < 1 || reps > 1000) return fail(FCGMG_E_ARG, "bad handle, pointer or reps (1..1000)");
  return autotune_impl(*h, reps, shape_out, us_out, (hipStream_t)stream);
}

int fcgmg_set_fused_shape(fcgmg_h h, int level, int k, void* stream) {
  if (!valid_level(h, level) || k < -1 || k >= fused2_num_shapes())
    return fail(FCGMG_E_ARG, "bad handle, level or shape index");
  return set_fused_shape_impl(*h, level, k, (hipStream_t)stream);
}

int fcgmg_set_cache_none_assembly(fcgmg_h h, int integrate) {
  if (!h || (integrate != 0 && integrate != 1)) return fail(FCGMG_E_ARG, "bad handle or mode");
  if (h->prm.cache_policy != FCGMG_CACHE_NONE) return fail(FCGMG_E_ARG, "the hierarchy does not use cache_none");
  h->none_integrate = integrate != 0;
  return FCGMG_OK;
}

int fcgmg_fused_shape(int k, int* tile_x, int* tile_y, int* threads, int* waves_per_simd) {
  if (k < 0 || k >= fused2_num_shapes() || !tile_x || !tile_y || !threads || !waves_per_simd)
    return fail(FCGMG_E_ARG, "shape index out of range or null pointer");
  fused2_shape_dims(k, tile_x, tile_y, threads, waves_per_simd);
  return FCGMG_OK;
}

int fcgmg_profile_enable(fcgmg_h h, int on) {
  if (!h) return fail(FCGMG_E_ARG, "null handle");
  h->prof = on != 0;
  return FCGMG_OK;
}

int fcgmg_profile_reset(fcgmg_h h) {
  if (!h) return fail(FCGMG_E_ARG, "null handle");
  int rc = prof_collect(*h);
  if (rc) return rc;
  std::fill(h->prof_ms.begin(), h->prof_ms.end(), 0.0);
  std::fill(h->prof_count.begin(), h->prof_count.end(), 0);
  return FCGMG_OK;
}

int fcgmg_profile_read(fcgmg_h h, int kind, int level, double* total_ms, int64_t* launches) {
  if (!valid_level(h, level) || kind < 0 || kind >= FCGMG_K_COUNT || !total_ms || !launches)
    return fail(FCGMG_E_ARG, "bad handle, kind, level or pointer");
  int rc = prof_collect(*h);
  if (rc) return rc;
  const size_t i = (size_t)kind * h->lev.size() + level;
  *total_ms = h->prof_ms[i];
  *launches = h->prof_count[i];
  return FCGMG_OK;
}

int fcgmg_device_bytes(fcgmg_h h, size_t* bytes) {
  if (!h || !bytes) return fail(FCGMG_E_ARG, "null argument");
  *bytes = h->bytes;
  return FCGMG_OK;
}

}  // extern "C"
