// HIP kernels (gfx950) of the fcgmg library: finite cell Stokes operator, restricted additive
// smoother under the three cache policies, grid transfers and reductions.
// Method: Saberi & Vogel, arXiv 2403.11636 (equation numbers refer to the paper).
#include <hip/hip_runtime.h>

#include <atomic>
#include <climits>
#include <cstdint>

#include "fcgmg_impl.h"

namespace fcg {

// Value in the constant address space: loads with a wavefront-uniform address from it are issued
// as scalar loads into SGPRs.
template <class T>
using cconst = __attribute__((address_space(4))) const T;

// Device (global) memory. Pointers that a kernel reads from a table in memory (the job tables of
// the batched launches) carry no address space, and loads through them would be issued as flat
// instructions, which count against both the vector-memory and the LDS wait counters (a wait for an
// LDS read then also waits for every load in flight). Cast to this space, they give global loads.
template <class T>
using gmem = __attribute__((address_space(1))) T;

namespace {

constexpr int kMaxLocalBalls = 16;

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <int D>
__device__ __forceinline__ void node_coords(int64_t node, int n, int* c) {
  const int64_t m = n + 1;
  c[0] = (int)(node % m);
  c[1] = (int)((node / m) % m);
  c[2] = D == 3 ? (int)(node / (m * m)) : 0;
}

template <int D>
__device__ __forceinline__ int64_t node_index(const int* c, int n) {
  const int64_t m = n + 1;
  return D == 2 ? c[0] + m * c[1] : c[0] + m * (c[1] + m * (int64_t)c[2]);
}

template <int D>
__device__ __forceinline__ int64_t cell_index(const int* c, int n) {
  return D == 2 ? c[0] + (int64_t)n * c[1] : c[0] + (int64_t)n * (c[1] + (int64_t)n * c[2]);
}

// Collect the balls that touch the box [lo, lo+s]^D into `out` (block-cooperative). The order of
// the list does not matter: alpha_at and box_kind only ask whether some ball contains / cuts.
// Returns the count, or -1 if more than kMaxLocalBalls touch the box (callers keep the full list).
template <int D>
__device__ int cull_balls(const Geom& g, const double* lo, double s, double* out, int* cnt_sh) {
  if (threadIdx.x == 0) *cnt_sh = 0;
  __syncthreads();
  for (int i = (int)threadIdx.x; i < g.nballs; i += (int)blockDim.x) {
    const double* b = g.balls + 4 * i;
    double dmin2 = 0;
    for (int k = 0; k < D; ++k) {
      double a = lo[k] - b[k], e = lo[k] + s - b[k];
      double m = a > 0 ? a : (e < 0 ? -e : 0.0);
      dmin2 += m * m;
    }
    if (dmin2 <= b[3] * b[3]) {
      const int slot = atomicAdd(cnt_sh, 1);
      if (slot < kMaxLocalBalls)
        for (int k = 0; k < 4; ++k) out[4 * slot + k] = b[k];
    }
  }
  __syncthreads();
  const int c = *cnt_sh;
  __syncthreads();
  return c > kMaxLocalBalls ? -1 : c;
}

}  // namespace

// ================================================================================================
// Cell classification (Eq. 7 / cut test of the space tree): 0 physical, 1 fictitious, 2 cut.
// ================================================================================================
template <int D>
__global__ void classify_cells_kernel(Geom g, int n, double h, int64_t ncells, signed char* kinds) {
  const int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (cell >= ncells) return;
  double lo[3];
  lo[0] = (double)(cell % n) * h;
  lo[1] = (double)((cell / n) % n) * h;
  lo[2] = D == 3 ? (double)(cell / ((int64_t)n * n)) * h : 0.0;
  kinds[cell] = (signed char)box_kind<D>(g, lo, h);
}

template <int D>
hipError_t k_classify_cells(const Ctx& c, Level& L, signed char* kinds, hipStream_t s) {
  const int bs = 256;
  const int64_t nb = (L.ncells + bs - 1) / bs;
  classify_cells_kernel<D><<<dim3((unsigned)nb), dim3(bs), 0, s>>>(c.geom(L), L.n, L.h, L.ncells, kinds);
  return hipGetLastError();
}

// ================================================================================================
// Cut-cell element data (Eq. 9 volume terms with alpha, Sec. 1 "sufficiently accurate
// integration"): one block per cut cell, threads over the (d+1) NN^2 entries K[a][b], B_c[a][b].
// ================================================================================================
template <int D>
__device__ void integrate_cell_entries(const Geom& g, const double* lo, double h, double eta, double* acc,
                                       int nper) {
  // acc[k] accumulates entry e = threadIdx.x + k*blockDim.x, k < nper
  constexpr int NN = 1 << D;
  tree_quadrature<D>(g, lo, h, [&](const double* x, double w, double alpha) {
    double phi[NN], gr[NN][3];
    q1<D>(lo, h, x, phi, gr);
    const double wa = w * alpha;
    for (int k = 0; k < nper; ++k) {
      const int e = (int)threadIdx.x + k * (int)blockDim.x;
      if (e < PT<D>::NEL) acc[k] += point_entry<D>(e, eta, wa, phi, gr);
    }
  });
}

template <int D>
__global__ void __launch_bounds__(64) cut_matrices_kernel(Geom g, int n, double h, double eta, int immersed,
                                                          double lam, const int* cut_cells, int64_t ncut,
                                                          double* out) {
  __shared__ double lball[4 * kMaxLocalBalls];
  __shared__ int cnt;
  constexpr int NEL = PT<D>::NEL;
  constexpr int NPER = (NEL + 63) / 64;
  for (int64_t ic = blockIdx.x; ic < ncut; ic += gridDim.x) {
    const int64_t cell = cut_cells[ic];
    double lo[3] = {0, 0, 0};
    lo[0] = (double)(cell % n) * h;
    lo[1] = (double)((cell / n) % n) * h;
    if (D == 3) lo[2] = (double)(cell / ((int64_t)n * n)) * h;
    const int nb = cull_balls<D>(g, lo, h, lball, &cnt);
    Geom gl = g;
    if (nb >= 0) {
      gl.balls = lball;
      gl.nballs = nb;
    }
    double acc[NPER];
    for (int k = 0; k < NPER; ++k) acc[k] = 0;
    integrate_cell_entries<D>(gl, lo, h, eta, acc, NPER);
    if constexpr (D == 2) {
      if (immersed)
        arc_quadrature2(gl, lo, h, [&](const double* x, double w, const double* nrm) {
          double phi[4], gr[4][3];
          q1<2>(lo, h, x, phi, gr);
          for (int k = 0; k < NPER; ++k) {
            const int e = (int)threadIdx.x + 64 * k;
            if (e < NEL) acc[k] += nitsche_entry2(e, eta, lam, w, nrm, phi, gr);
          }
        });
    } else {
      if (immersed)
        sphere_quadrature3(gl, lo, h, [&](const double* x, double w, const double* nrm) {
          double phi[8], gr[8][3];
          q1<3>(lo, h, x, phi, gr);
          for (int k = 0; k < NPER; ++k) {
            const int e = (int)threadIdx.x + 64 * k;
            if (e < NEL) acc[k] += nitsche_entry3(e, eta, lam, w, nrm, phi, gr);
          }
        });
    }
    for (int k = 0; k < NPER; ++k) {
      const int e = (int)threadIdx.x + 64 * k;
      if (e < NEL) out[ic * NEL + e] = acc[k];
    }
    __syncthreads();
  }
}

// Split form of the cut-cell integration (3D): the coarse levels have few cut cells and deep trees
// (the tree depth grows by one per coarser level), so one workgroup per cell leaves the GPU nearly
// idle. Each cell's tree is cut at depth sd into work items, in the order of the depth-first
// traversal: a box at depth sd whose ancestors are all cut, or a shallower leaf. One workgroup
// integrates each item's subtree (the same boxes and points as the whole traversal), and the cell's
// entries are the items' sums added in traversal order.
//
// Candidate `cand` of a cell (digits of D bits from depth 1 down to sd: the child taken at each
// depth) stops at the first box that is not descended into; it stands for that box only if all its
// digits below that depth are 0. item_depth = that depth, or -1.
template <int D>
__device__ __forceinline__ int cut_item_box(const Geom& g, int n, double h, int cell, int cand, int sd, int stop,
                                            double* lo, double* size) {
  lo[0] = (double)(cell % n) * h;
  lo[1] = (double)((cell / n) % n) * h;
  lo[2] = D == 3 ? (double)(cell / ((int64_t)n * n)) * h : 0.0;
  *size = h;
  int t = 0;
  for (; t < sd; ++t) {
    if (stop >= 0 ? t == stop : !(t < g.q && box_kind<D>(g, lo, *size) == 2)) break;
    const int digit = (cand >> (D * (sd - 1 - t))) & ((1 << D) - 1);
    const double half = 0.5 * *size;
    for (int k = 0; k < D; ++k) lo[k] += ((digit >> k) & 1) ? half : 0.0;
    *size = half;
  }
  return t;
}

template <int D>
__global__ void cut_frontier_kernel(Geom g, int n, double h, const int* __restrict__ cut_cells, int64_t ncut, int sd,
                                    int* __restrict__ item_depth) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (ncut << (D * sd))) return;
  const int cand = (int)(gid & ((1 << (D * sd)) - 1));
  double lo[3], size;
  const int t = cut_item_box<D>(g, n, h, cut_cells[gid >> (D * sd)], cand, sd, -1, lo, &size);
  item_depth[gid] = (cand & ((1 << (D * (sd - t))) - 1)) == 0 ? t : -1;
}

// Volume entries of one work item: the tree below the item's box, Q1 functions of its cell.
template <int D>
__global__ void __launch_bounds__(64) cut_items_kernel(Geom g, int n, double h, double eta,
                                                       const int* __restrict__ cut_cells, int sd,
                                                       const int* __restrict__ item_cell,
                                                       const int* __restrict__ item_cand,
                                                       const int* __restrict__ item_stop, int64_t nitems,
                                                       double* __restrict__ part) {
  __shared__ double lball[4 * kMaxLocalBalls];
  __shared__ int cnt;
  constexpr int NN = 1 << D, NEL = PT<D>::NEL, NPER = (NEL + 63) / 64;
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int cell = cut_cells[item_cell[it]];
    double lo[3], size;
    const int t = cut_item_box<D>(g, n, h, cell, item_cand[it], sd, item_stop[it], lo, &size);
    double clo[3] = {(double)(cell % n) * h, (double)((cell / n) % n) * h,
                     D == 3 ? (double)(cell / ((int64_t)n * n)) * h : 0.0};
    const int nb = cull_balls<D>(g, lo, size, lball, &cnt);
    Geom gl = g;
    if (nb >= 0) {
      gl.balls = lball;
      gl.nballs = nb;
    }
    gl.q = g.q - t;
    double acc[NPER];
    for (int k = 0; k < NPER; ++k) acc[k] = 0;
    tree_quadrature<D>(gl, lo, size, [&](const double* x, double w, double alpha) {
      double phi[NN], gr[NN][3];
      q1<D>(clo, h, x, phi, gr);
      const double wa = w * alpha;
      for (int k = 0; k < NPER; ++k) {
        const int e = (int)threadIdx.x + 64 * k;
        if (e < NEL) acc[k] += point_entry<D>(e, eta, wa, phi, gr);
      }
    });
    for (int k = 0; k < NPER; ++k) {
      const int e = (int)threadIdx.x + 64 * k;
      if (e < NEL) part[it * NEL + e] = acc[k];
    }
    __syncthreads();
  }
}

// A cell's entries: its items' volume sums in traversal order, then the immersed surface terms.
template <int D>
__global__ void __launch_bounds__(64) cut_sum_kernel(Geom g, int n, double h, double eta, int immersed, double lam,
                                                     const int* __restrict__ cut_cells,
                                                     const int* __restrict__ item_start, int64_t ncut,
                                                     const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double lball[4 * kMaxLocalBalls];
  __shared__ int cnt;
  constexpr int NEL = PT<D>::NEL, NPER = (NEL + 63) / 64;
  for (int64_t ic = blockIdx.x; ic < ncut; ic += gridDim.x) {
    double acc[NPER];
    for (int k = 0; k < NPER; ++k) acc[k] = 0;
    for (int it = item_start[ic]; it < item_start[ic + 1]; ++it)
      for (int k = 0; k < NPER; ++k) {
        const int e = (int)threadIdx.x + 64 * k;
        if (e < NEL) acc[k] += part[(int64_t)it * NEL + e];
      }
    if (immersed) {
      const int64_t cell = cut_cells[ic];
      const double lo[3] = {(double)(cell % n) * h, (double)((cell / n) % n) * h,
                            D == 3 ? (double)(cell / ((int64_t)n * n)) * h : 0.0};
      const int nb = cull_balls<D>(g, lo, h, lball, &cnt);
      Geom gl = g;
      if (nb >= 0) {
        gl.balls = lball;
        gl.nballs = nb;
      }
      if constexpr (D == 2)
        arc_quadrature2(gl, lo, h, [&](const double* x, double w, const double* nrm) {
          double phi[4], gr[4][3];
          q1<2>(lo, h, x, phi, gr);
          for (int k = 0; k < NPER; ++k) {
            const int e = (int)threadIdx.x + 64 * k;
            if (e < NEL) acc[k] += nitsche_entry2(e, eta, lam, w, nrm, phi, gr);
          }
        });
      else
        sphere_quadrature3(gl, lo, h, [&](const double* x, double w, const double* nrm) {
          double phi[8], gr[8][3];
          q1<3>(lo, h, x, phi, gr);
          for (int k = 0; k < NPER; ++k) {
            const int e = (int)threadIdx.x + 64 * k;
            if (e < NEL) acc[k] += nitsche_entry3(e, eta, lam, w, nrm, phi, gr);
          }
        });
    }
    for (int k = 0; k < NPER; ++k) {
      const int e = (int)threadIdx.x + 64 * k;
      if (e < NEL) out[ic * NEL + e] = acc[k];
    }
    __syncthreads();
  }
}

// Cut cells whose work the split form spreads: the split depth is the smallest that gives at least
// this many work candidates (at most 3, and at most the tree depth).
constexpr int64_t kCutWorkItems = 12000;

template <int D>
hipError_t k_cut_matrices(const Ctx& c, Level& L, const int* cut_cells, hipStream_t s) {
  if (L.n_cut == 0) return hipSuccess;
  const Geom g = c.geom(L);
  const double lam = c.prm.nitsche_beta * c.prm.eta / L.h;
  int sd = 0;
  if constexpr (D == 3)
    while (sd < 3 && sd < g.q && (L.n_cut << (D * sd)) < kCutWorkItems) ++sd;
  if (sd == 0) {
    const int64_t nb = L.n_cut < 65536 ? L.n_cut : 65536;
    cut_matrices_kernel<D><<<dim3((unsigned)nb), dim3(64), 0, s>>>(g, L.n, L.h, c.prm.eta, c.prm.immersed_nitsche, lam,
                                                                 cut_cells, L.n_cut, L.cut_mats);
    return hipGetLastError();
  }
  // work items: candidates on the GPU (the same box tests as the traversal), listed on the host
  const int64_t ncand = L.n_cut << (D * sd);
  int* depth_d = nullptr;
  hipError_t e = hipMallocAsync((void**)&depth_d, (size_t)ncand * sizeof(int), s);
  if (e != hipSuccess) return e;
  cut_frontier_kernel<D><<<dim3((unsigned)((ncand + 255) / 256)), dim3(256), 0, s>>>(g, L.n, L.h, cut_cells, L.n_cut, sd,
                                                                                     depth_d);
  std::vector<int> depth(ncand);
  if ((e = hipGetLastError()) == hipSuccess)
    e = hipMemcpyAsync(depth.data(), depth_d, (size_t)ncand * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const hipError_t f = hipFreeAsync(depth_d, s);
  if (e != hipSuccess) return e;
  if (f != hipSuccess) return f;
  std::vector<int> items;  // per item: cell index, candidate, stop depth
  std::vector<int> start(L.n_cut + 1, 0);
  for (int64_t i = 0; i < L.n_cut; ++i) {
    start[i] = (int)(items.size() / 3);
    for (int64_t k = 0; k < ((int64_t)1 << (D * sd)); ++k) {
      const int t = depth[(i << (D * sd)) + k];
      if (t >= 0) {
        items.push_back((int)i);
        items.push_back((int)k);
        items.push_back(t);
      }
    }
  }
  const int64_t nitems = (int64_t)(items.size() / 3);
  start[L.n_cut] = (int)nitems;
  std::vector<int> cols(3 * nitems);  // item_cell | item_cand | item_stop
  for (int64_t k = 0; k < nitems; ++k)
    for (int j = 0; j < 3; ++j) cols[j * nitems + k] = items[3 * k + j];
  int* meta_d = nullptr;
  double* part_d = nullptr;
  if ((e = hipMallocAsync((void**)&meta_d, (cols.size() + start.size()) * sizeof(int), s)) != hipSuccess) return e;
  if ((e = hipMallocAsync((void**)&part_d, (size_t)nitems * PT<D>::NEL * sizeof(double), s)) != hipSuccess) {
    (void)hipFreeAsync(meta_d, s);
    return e;
  }
  e = hipMemcpyAsync(meta_d, cols.data(), cols.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(meta_d + cols.size(), start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    const int64_t nb = nitems < 262144 ? nitems : 262144;
    cut_items_kernel<D><<<dim3((unsigned)nb), dim3(64), 0, s>>>(g, L.n, L.h, c.prm.eta, cut_cells, sd, meta_d,
                                                                 meta_d + nitems, meta_d + 2 * nitems, nitems, part_d);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int64_t nb = L.n_cut < 65536 ? L.n_cut : 65536;
    cut_sum_kernel<D><<<dim3((unsigned)nb), dim3(64), 0, s>>>(g, L.n, L.h, c.prm.eta, c.prm.immersed_nitsche, lam,
                                                              cut_cells, meta_d + cols.size(), L.n_cut, part_d,
                                                              L.cut_mats);
    e = hipGetLastError();
  }
  // the host vectors must outlive the copies from them
  const hipError_t w = hipStreamSynchronize(s);
  const hipError_t f1 = hipFreeAsync(part_d, s), f2 = hipFreeAsync(meta_d, s);
  if (e != hipSuccess) return e;
  if (w != hipSuccess) return w;
  return f1 != hipSuccess ? f1 : f2;
}

// ================================================================================================
// Right-hand side of Eq. (9): f(v) = (v, alpha f) - (n.eta grad v, w)_D + (v, lambda w)_D,
// g(q) = (n q, w)_D; Neumann walls carry h = 0. One thread per node gathers its cells.
// ================================================================================================
template <int D>
__global__ void rhs_kernel(Geom g, const OpConsts* __restrict__ oc, int force, double eta, double ubar,
                           int bc0, int bc1, int bc2, int bc3, int bc4, int bc5, int64_t N, double* b) {
  const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (node >= N) return;
  constexpr int NN = 1 << D;
  const int n = oc->n;
  const double h = oc->h, lam = oc->lam;
  const int bcs[6] = {bc0, bc1, bc2, bc3, bc4, bc5};
  int c[3];
  node_coords<D>(node, n, c);
  double acc[D + 1];
  for (int f = 0; f <= D; ++f) acc[f] = 0;
  for (int sc = 0; sc < NN; ++sc) {
    int cc[3] = {0, 0, 0};
    bool in = true;
    int a = 0;
    for (int k = 0; k < D; ++k) {
      const int sk = (sc >> k) & 1;
      cc[k] = c[k] - 1 + sk;
      if (cc[k] < 0 || cc[k] > n - 1) in = false;
      a |= (1 - sk) << k;
    }
    if (!in) continue;
    double lo[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) lo[k] = cc[k] * h;
    // the volume term (v, alpha f); body_force is zero for every kind but 1, and then it adds only
    // zeros
    if (force == 1)
      tree_quadrature<D>(g, lo, h, [&](const double* x, double w, double alpha) {
        double phi[NN], gr[NN][3], fv[3];
        q1<D>(lo, h, x, phi, gr);
        body_force<D>(force, eta, x, fv);
        for (int f = 0; f < D; ++f) acc[f] += w * alpha * fv[f] * phi[a];
      });
    for (int k = 0; k < D; ++k)
      for (int sd = 0; sd < 2; ++sd) {
        const bool on = sd ? (cc[k] == n - 1) : (cc[k] == 0);
        const int code = bcs[2 * k + sd];
        if (!on || code == FCGMG_BC_NEUMANN) continue;
        const double nk = sd ? 1.0 : -1.0;
        const double w = D == 2 ? 0.5 * h : 0.25 * h * h;
        for (int gp = 0; gp < (1 << (D - 1)); ++gp) {
          double x[3] = {0, 0, 0};
          int t = 0;
          for (int j = 0; j < D; ++j) {
            if (j == k) {
              x[j] = lo[j] + (sd ? h : 0.0);
            } else {
              x[j] = lo[j] + h * (((gp >> t) & 1) ? FCG_GB : FCG_GA);
              ++t;
            }
          }
          double phi[NN], gr[NN][3], wv[3];
          q1<D>(lo, h, x, phi, gr);
          wall_data<D>(code, ubar, k, sd, x, wv);
          for (int f = 0; f < D; ++f) acc[f] += w * (-eta * nk * gr[a][k] * wv[f] + lam * phi[a] * wv[f]);
          acc[D] += w * phi[a] * nk * wv[k];
        }
      }
  }
  for (int f = 0; f <= D; ++f) b[f * N + node] = acc[f];
}

template <int D>
hipError_t k_rhs(const Ctx& c, const Level& L, double* b, hipStream_t s) {
  const int bs = 128;
  const int64_t nb = (L.N + bs - 1) / bs;
  const int* bc = c.prm.bc;
  rhs_kernel<D><<<dim3((unsigned)nb), dim3(bs), 0, s>>>(c.geom(L), L.consts, c.prm.force, c.prm.eta, c.prm.ubar, bc[0],
                                                        bc[1], bc[2], bc[3], bc[4], bc[5], L.N, b);
  return hipGetLastError();
}

// ================================================================================================
// Residual r = b - L x (Eq. 12, 14). Each node sums the element rows of the 2^d cells around it:
// uncut cells use the reference matrices (read through uniform scalar loads) times alpha of the
// cell, cut cells their stored integrals, Dirichlet walls the Nitsche face matrices; the
// stabilisation C carries no alpha (Eq. 10). x comes from an LDS tile with a one-node halo.
// ================================================================================================
template <int D>
struct TileShape;
template <>
struct TileShape<2> {
  static constexpr int TX = 32, TY = 8, TZ = 1;
};
template <>
struct TileShape<3> {
  static constexpr int TX = 8, TY = 8, TZ = 4;
};

// Tile of block `bid` in an nt[0] x nt[1] x nt[2] tile grid. Consecutive workgroups are dealt
// round-robin to the 8 XCDs (each with its own L2), and the remap chooses which tiles share one:
// * R = 0: every XCD takes a contiguous range of tiles (a band of the grid), so halo re-reads of
//   neighbouring tiles hit the same L2;
// * R > 0: every XCD takes runs of R consecutive tiles along x, and each window of 8 R tiles spreads
//   over all 8 XCDs. The obstacles' cut tiles, which take longest, are then shared out evenly over
//   the XCDs instead of piling up in the bands that cross them.
// Either way it is a bijection of the first blocks onto themselves (8*floor(nb/8) for bands,
// 8R*floor(nb/(8R)) for runs); the remaining blocks keep their own tile.
template <int D, int R = 0>
__device__ __forceinline__ void tile_coords(int bid, const int* nt, int* t) {
  const int nb = nt[0] * nt[1] * nt[2];
  int lin = bid;
  if constexpr (R == 0) {
    const int nb8 = nb - nb % 8;
    if (bid < nb8) lin = (bid % 8) * (nb8 / 8) + bid / 8;
  } else {
    constexpr int W = 8 * R;
    const int nbw = nb - nb % W;
    if (bid < nbw) lin = ((bid / 8) / R) * W + (bid % 8) * R + (bid / 8) % R;
  }
  t[0] = lin % nt[0];
  t[1] = (lin / nt[0]) % nt[1];
  t[2] = lin / (nt[0] * nt[1]);
}

// Reference element matrices of a level (uncut physical cell; fictitious cells scale K and B by
// alpha_f), the stabilisation block and the Nitsche face matrices, packed for one dimension. The
// kernels copy them into LDS once per workgroup: the node loops then read only LDS.
template <int D, class T = double>
struct RefMats : RefLayout<D> {
  T v[RefLayout<D>::TOT];
  int dir[2 * D];
};

// Cooperative copy of the level constants into LDS by a workgroup of NT threads, rounded to T:
// every load is issued before the first store (caller synchronises afterwards).
template <int D, int NT, class T>
__device__ __forceinline__ void stage_refmats(const OpConsts* __restrict__ oc, RefMats<D, T>& rm) {
  constexpr int TOT = RefLayout<D>::TOT, NK = (TOT + NT - 1) / NT;
  T v[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + NT * k;
    v[k] = i < TOT ? (T)oc->pack[i] : T(0);
  }
  const int dv = threadIdx.x < 2 * D ? oc->dirichlet[threadIdx.x] : 0;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int i = threadIdx.x + NT * k;
    if (i < TOT) rm.v[i] = v[k];
  }
  if (threadIdx.x < 2 * D) rm.dir[threadIdx.x] = dv;
}

// Accumulate L x at node c (coords) into acc[0..D] cell by cell from the element matrices (Eq. 9-11):
// xat(f, o) returns x_f at c + o (o in {-1,0,1}^D), ci(cc) the kind/cut index of the in-grid cell
// with lower corner cc, cutp(cc, info) the address of a cut cell's integrals. The residual kernels
// apply the node stencils this assembles (node_stencil_kernel); set-up code applies it directly.
// UNR = false keeps the loop over the cells rolled (same order of operations, fewer registers).
template <int D, bool UNR = true, class CI, class CP, class XA>
__device__ __forceinline__ void node_apply(const RefMats<D>& rm, CI&& ci, CP&& cutp, double alpha_f, int n,
                                           const int* c, XA&& xat, double* acc) {
  constexpr int NN = 1 << D, NN2 = NN * NN;
#pragma unroll(UNR ? NN : 1)
  for (int sc = 0; sc < NN; ++sc) {
    int cc[3] = {0, 0, 0};
    bool in = true;
    int a = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int sk = (sc >> k) & 1;
      cc[k] = c[k] - 1 + sk;
      in = in && cc[k] >= 0 && cc[k] <= n - 1;
      a |= (1 - sk) << k;
    }
    if (!in) continue;
    const int info = ci(cc);
    double u[D + 1][NN];
#pragma unroll
    for (int bn = 0; bn < NN; ++bn) {
      int o[3] = {0, 0, 0};
#pragma unroll
      for (int k = 0; k < D; ++k) o[k] = -1 + ((sc >> k) & 1) + ((bn >> k) & 1);
#pragma unroll
      for (int f = 0; f <= D; ++f) u[f][bn] = xat(f, o);
    }
    if (info >= 0) {
      const double* Kp = cutp(cc, info);
      const double* Bp = Kp + NN * NN;
#pragma unroll
      for (int bn = 0; bn < NN; ++bn) {
        const double kab = Kp[a * NN + bn];
#pragma unroll
        for (int f = 0; f < D; ++f) {
          acc[f] += kab * u[f][bn] + Bp[f * NN * NN + a * NN + bn] * u[D][bn];
          acc[D] += Bp[f * NN * NN + bn * NN + a] * u[f][bn];
        }
      }
    } else {
      const double al = info == -1 ? 1.0 : alpha_f;
      double sk[D + 1];
#pragma unroll
      for (int f = 0; f <= D; ++f) sk[f] = 0;
#pragma unroll
      for (int bn = 0; bn < NN; ++bn) {
        const double kab = rm.v[RefMats<D>::oK + a * NN + bn];
#pragma unroll
        for (int f = 0; f < D; ++f) {
          sk[f] += kab * u[f][bn] + rm.v[RefMats<D>::oB + f * NN2 + a * NN + bn] * u[D][bn];
          sk[D] += rm.v[RefMats<D>::oB + f * NN2 + bn * NN + a] * u[f][bn];
        }
      }
#pragma unroll
      for (int f = 0; f <= D; ++f) acc[f] += al * sk[f];
    }
#pragma unroll
    for (int bn = 0; bn < NN; ++bn) acc[D] += rm.v[RefMats<D>::oC + a * NN + bn] * u[D][bn];
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const int face = 2 * k + sd;
        if (!rm.dir[face] || cc[k] != (sd ? n - 1 : 0)) continue;
#pragma unroll
        for (int bn = 0; bn < NN; ++bn) {
          const double fk = rm.v[RefMats<D>::oFK + face * NN2 + a * NN + bn];
#pragma unroll
          for (int f = 0; f < D; ++f) acc[f] += fk * u[f][bn];
          acc[k] += rm.v[RefMats<D>::oFB + face * NN2 + a * NN + bn] * u[D][bn];
          acc[D] += rm.v[RefMats<D>::oFB + face * NN2 + bn * NN + a] * u[k][bn];
        }
      }
  }
}

// acc[f] += sum over the 3^d offsets o of the node stencil applied to x around the node; cf(j, o) is
// the coefficient of block j (layout of Level::nsten), xat(f, o) the value x_f at the node + o.
template <int D, bool UNR, class T, class CF, class XA>
__device__ __forceinline__ void stencil_apply(CF&& cf, XA&& xat, T* acc) {
  constexpr int NS = PT<D>::NST;
#pragma unroll(UNR ? NS : 3)
  for (int o = 0; o < NS; ++o) {
    const int oo[3] = {o % 3 - 1, (o / 3) % 3 - 1, D == 3 ? o / 9 - 1 : 0};
    T u[D + 1];
#pragma unroll
    for (int f = 0; f <= D; ++f) u[f] = xat(f, oo);
    const T sk = cf(0, o);
#pragma unroll
    for (int f = 0; f < D; ++f) {
      acc[f] += sk * u[f] + cf(1 + f, o) * u[D];
      acc[D] += cf(1 + D + f, o) * u[f];
    }
    acc[D] += cf(1 + 2 * D, o) * u[D];
  }
}

// Stored 2D stencil (layout of Level::nsten at p): the six coefficients of offset o, and the terms
//   t_f = SK_o u_f(o) + SB_f,o p(o) (f < 2),  t_2 = ST_0,o u_0(o) + ST_1,o u_1(o) + SC_o p(o)
// with u = x at the node + o. The fused multiply-adds are explicit, and contraction is off here
// and in the sums of the terms below, so that every form of the row sum rounds alike in every
// kernel.
template <class T, class P>
__device__ __forceinline__ void stored_coefs2(P __restrict__ p, int o, T* c) {
#pragma unroll
  for (int j = 0; j < 6; ++j) c[j] = p[j * 9 + o];
}

template <class T>
__device__ __forceinline__ void stored_terms2(const T* c, T u0, T u1, T u2, T* t) {
#pragma clang fp contract(off)
  t[0] = fma(c[0], u0, c[1] * u2);
  t[1] = fma(c[0], u1, c[2] * u2);
  t[2] = fma(c[5], u2, fma(c[4], u1, c[3] * u0));
}

// Marks the values as used here: loads issued before are all in flight together, since the
// scheduler cannot move them past this point to shorten register lifetimes.
template <class T, int K>
__device__ __forceinline__ void in_flight_together(T (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) asm volatile("" : "+v"(v[k]));
}

// Row of a stored 2D stencil at p, one lane: the offset terms summed in the order of a butterfly
// over 16 lanes (lane = offset, lanes 9..15 empty; partners at distance 8, 4, 2, 1):
//   R(l, 8) = t_l + t_(l+8),  R(l, s) = R(l, 2s) + R(l+s, 2s),  row = R(0, 1)
//   = (((t0 + t8) + t4) + (t2 + t6)) + ((t1 + t5) + (t3 + t7)),
// so that the 8-lane form (stored_rows_group2), which starts from R(l, 8), gives the same bits. The
// coefficients load in three batches of three offsets.
template <class T, class XA, class P>
__device__ __forceinline__ void stored_row2(P __restrict__ p, XA&& xat, T* row) {
#pragma clang fp contract(off)
  auto terms = [&](const T* c, int o, T* t) {
    const int oo[3] = {o % 3 - 1, o / 3 - 1, 0};
    stored_terms2<T>(c, xat(0, oo), xat(1, oo), xat(2, oo), t);
  };
  T c[18], ta[3], tb[3], tc[3], A[3], L[3], R[3];
  // offsets 0, 8, 4: A = (t0 + t8) + t4
  stored_coefs2<T>(p, 0, c);
  stored_coefs2<T>(p, 8, c + 6);
  stored_coefs2<T>(p, 4, c + 12);
  in_flight_together(c);
  terms(c, 0, ta);
  terms(c + 6, 8, tb);
  terms(c + 12, 4, tc);
#pragma unroll
  for (int f = 0; f < 3; ++f) A[f] = (ta[f] + tb[f]) + tc[f];
  // offsets 2, 6, 1: L = A + (t2 + t6); t1 kept
  stored_coefs2<T>(p, 2, c);
  stored_coefs2<T>(p, 6, c + 6);
  stored_coefs2<T>(p, 1, c + 12);
  in_flight_together(c);
  terms(c, 2, ta);
  terms(c + 6, 6, tb);
  terms(c + 12, 1, tc);
#pragma unroll
  for (int f = 0; f < 3; ++f) L[f] = A[f] + (ta[f] + tb[f]);
  // offsets 5, 3, 7: R = (t1 + t5) + (t3 + t7)
  stored_coefs2<T>(p, 5, c);
  stored_coefs2<T>(p, 3, c + 6);
  stored_coefs2<T>(p, 7, c + 12);
  in_flight_together(c);
  terms(c, 5, ta);
  terms(c + 6, 3, tb);
#pragma unroll
  for (int f = 0; f < 3; ++f) R[f] = tc[f] + ta[f];
  terms(c + 12, 7, ta);
#pragma unroll
  for (int f = 0; f < 3; ++f) row[f] = L[f] + (R[f] + (tb[f] + ta[f]));
}

// Reference-stencil part of a row of L at a node with operator code op (Level::node_op): lanes
// with op < 0 apply the level's reference stencil of their kind, read from the packed level
// constants (oc->pack, FP64, rounded to T) with scalar loads. The lanes are taken kind by kind (a
// waterfall over the at most two kinds present in the wavefront), so every coefficient address is
// wavefront-uniform. Lanes with op >= 0 are left to stored_row_apply.
template <int D, bool UNR = true, class T, class XA>
__device__ __forceinline__ void ref_row_apply(const double* __restrict__ pack, int op, XA&& xat, T* acc) {
  using R = RefLayout<D>;
  constexpr int NS = PT<D>::NST;
  bool todo = op < 0;
  while (__ballot(todo) != 0) {
    if (todo) {
      const int k0 = __builtin_amdgcn_readfirstlane(-op - 1);
      if (-op - 1 == k0) {
        // read the lane value again inside the branch, so that the compiler keeps a scalar kind
        const int ku = __builtin_amdgcn_readfirstlane(-op - 1);
        cconst<double>* P = (cconst<double>*)pack;
        stencil_apply<D, UNR, T>(
            [&](int j, int o) -> T {
              if (j == 0) return (T)P[R::oSK + ku * NS + o];
              if (j <= D) return (T)P[R::oSB + (ku * D + j - 1) * NS + o];
              if (j <= 2 * D) return (T)P[R::oST + (ku * D + j - 1 - D) * NS + o];
              return (T)P[R::oSC + o];
            },
            xat, acc);
        todo = false;
      }
    }
  }
}

// Stored-stencil row (op >= 0), one lane: 2D sums the offset terms in the butterfly order of
// stored_row2; 3D runs the offsets in sequence, partly rolled so that the loads of the row do not
// all occupy registers at once.
template <int D, class T, class XA, class PN>
__device__ __forceinline__ void stored_row_apply(int op, PN __restrict__ nsten, XA&& xat, T* acc) {
#pragma clang fp contract(off)
  const auto p = nsten + (int64_t)op * PT<D>::NSTEN;
  if constexpr (D == 2) {
    T t[3];
    stored_row2<T>(p, xat, t);
#pragma unroll
    for (int f = 0; f < 3; ++f) acc[f] += t[f];
  } else {
    stencil_apply<D, false, T>([&](int j, int o) { return p[sten_index<D>(j, o)]; }, xat, acc);
  }
}

// Row of L at a node with operator code op: the level's reference stencil of a uniform
// neighbourhood (op < 0), or the node's own assembled stencil in nsten (op >= 0).
template <int D, bool UNR = true, class T, class XA, class PN>
__device__ __forceinline__ void node_row_apply(const double* __restrict__ pack, int op, PN __restrict__ nsten,
                                               XA&& xat, T* acc) {
  ref_row_apply<D, UNR, T>(pack, op, xat, acc);
  if (op >= 0) stored_row_apply<D, T>(op, nsten, xat, acc);
}

// Stored-stencil nodes of a 2D residual region in LDS (tile kernels): each wavefront compacts, per
// round k of its residual nodes, the entries with op >= 0 into its own segment (k, wavefront) of the
// list, in node order; cnt holds the length of every segment.
template <int NT, int NRES>
struct StoredList2 {
  static constexpr int NW = NT / 64, NSEG = NRES * NW;
  short e[NSEG * 64];
  int op[NSEG * 64];
  int cnt[NSEG];
};

template <int NT, int NRES>
__device__ __forceinline__ void stored_list_add(StoredList2<NT, NRES>& sl, int k, int e, int op, unsigned tid) {
  constexpr int NW = NT / 64;
  const bool st = op >= 0;
  const unsigned long long msk = __ballot(st);
  const int pos = __builtin_amdgcn_mbcnt_hi((unsigned)(msk >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)msk, 0));
  const int seg = k * NW + (int)(tid >> 6);
  if (st) {
    sl.e[seg * 64 + pos] = (short)e;
    sl.op[seg * 64 + pos] = op;
  }
  if ((tid & 63) == 0) sl.cnt[seg] = __popcll(msk);
}

// Partial sum R(j + OFF, S) of the butterfly order of stored_row2, for S >= LPN (the offsets of one
// lane j < LPN: j, j + LPN, ...; lane 0 also offset 8); term(k, t) gives the terms of offset j + k LPN
// (k < 8 / LPN), term(8 / LPN, t) those of offset 8.
template <int OFF, int S, int LPN, class T, class TF>
__device__ __forceinline__ void lane_tree2(int j, TF&& term, T* out) {
#pragma clang fp contract(off)
  if constexpr (S == 8) {
    term(OFF / LPN, out);
    if constexpr (OFF == 0) {
      if (j == 0) {
        T t8[3];
        term(8 / LPN, t8);
#pragma unroll
        for (int f = 0; f < 3; ++f) out[f] = out[f] + t8[f];
      }
    }
  } else {
    T a[3], b[3];
    lane_tree2<OFF, 2 * S, LPN, T>(j, term, a);
    lane_tree2<OFF + S, 2 * S, LPN, T>(j, term, b);
#pragma unroll
    for (int f = 0; f < 3; ++f) out[f] = a[f] + b[f];
  }
}

// rs[f RP + e] = b_f - (L x)_f for every listed node, LPN lanes per node (LPN = 8, 4 or 2): lane j
// takes offsets j, j + LPN, ... below 8 and lane 0 also offset 8; each lane forms its partial sum
// R(j, LPN) of the butterfly order of stored_row2 (lane_tree2), then a butterfly over the LPN lanes
// completes it, so the bits equal those of the per-lane form. The six coefficients of offset 8 are
// loaded by lanes k mod LPN and gathered by shuffles. The loads of the first trip (one node per
// group of LPN lanes) are issued before `between` runs (the reference-stencil residuals of the
// tile) and used after it, so that their latency is hidden behind that work. With 8 lanes per node
// the loads of the next two trips are issued together after it; further trips follow one by one.
// Entry e of the region (row width RW) is grid node (ox + e % RW, oy + e / RW) of the level (m
// nodes per axis, field stride N); x comes from the LDS tile xs (row width XW, field stride XP) at
// index (e % RW + 1) + XW (e / RW + 1).
template <int NT, int NRES, int RW, int RP, int XW, int XP, int LPN, class T, class BF, class PN, class PB>
__device__ __forceinline__ void stored_rows_group2(const StoredList2<NT, NRES>& sl, PN __restrict__ nsten,
                                                   PB __restrict__ b, int64_t N, int m, int ox, int oy,
                                                   const T* xs, T* rs, BF&& between, unsigned tid) {
#pragma clang fp contract(off)
  static_assert(LPN == 8 || LPN == 4 || LPN == 2, "lanes per node");
  constexpr int NSEG = StoredList2<NT, NRES>::NSEG, NG = NT / LPN;
  constexpr int NO = 8 / LPN;                  // offsets below 8 per lane
  constexpr int N8 = (6 + LPN - 1) / LPN;      // coefficients of offset 8 per lane
  constexpr int NC = 6 * NO + N8;
  constexpr int NF = (3 + LPN - 1) / LPN;      // fields written per lane (j, j + LPN, ... < 3)
  int pre[NSEG + 1];
  pre[0] = 0;
#pragma unroll
  for (int s = 0; s < NSEG; ++s) pre[s + 1] = pre[s] + sl.cnt[s];
  const int cnt = pre[NSEG];
  const int j = tid & (LPN - 1), g = (int)(tid / LPN);
  auto slot = [&](int t) {
    int s = 0;
#pragma unroll
    for (int k = 1; k < NSEG; ++k) s += t >= pre[k] ? 1 : 0;
    return s * 64 + t - pre[s];
  };
  // loads of entry t: the six coefficients of offsets j + k LPN, coefficients j + i LPN of offset 8,
  // b of fields j + i LPN
  auto issue = [&](int t, T* c, T* bl, int& e) {
    const int sidx = slot(t);
    e = sl.e[sidx];
    const auto p = nsten + (int64_t)sl.op[sidx] * PT<2>::NSTEN;
    const int64_t g = (ox + e % RW) + (int64_t)m * (oy + e / RW);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int f = j + i * LPN;
      bl[i] = b[(f < 3 ? f : 0) * N + g];
    }
#pragma unroll
    for (int k = 0; k < NO; ++k) stored_coefs2<T>(p, j + k * LPN, c + 6 * k);
#pragma unroll
    for (int i = 0; i < N8; ++i) {
      const int q = j + i * LPN;
      c[6 * NO + i] = p[(q < 6 ? q : 5) * 9 + 8];
    }
  };
  auto finish = [&](const T* c, const T* bl, int e) {
    const int xb = (e % RW + 1) + XW * (e / RW + 1);
    T c8[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) c8[q] = __shfl(c[6 * NO + q / LPN], q % LPN, LPN);
    auto term = [&](int k, T* t) {
      const int o = k < NO ? j + k * LPN : 8;
      const int xo = xb + (o % 3 - 1) + XW * (o / 3 - 1);
      stored_terms2<T>(k < NO ? c + 6 * k : c8, xs[xo], xs[XP + xo], xs[2 * XP + xo], t);
    };
    T v[3];
    lane_tree2<0, LPN, LPN, T>(j, term, v);
#pragma unroll
    for (int msk = LPN / 2; msk >= 1; msk >>= 1)
#pragma unroll
      for (int f = 0; f < 3; ++f) v[f] = v[f] + __shfl_xor(v[f], msk, LPN);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int f = j + i * LPN;
      if (f < 3) rs[f * RP + e] = bl[i] - (f == 0 ? v[0] : (f == 1 ? v[1] : v[2]));
    }
  };
  T c[NC], bl[NF];
  int e = 0;
  const bool first = g < cnt;
  if (first) issue(g, c, bl, e);
  between();
  // the next trips' loads go out together, before the first trip is finished (8-lane groups, whose
  // trips hold the fewest registers)
  constexpr int NX = LPN == 8 ? 2 : 0;
  T cx[NX > 0 ? NX : 1][NC], blx[NX > 0 ? NX : 1][NF];
  int ex[NX > 0 ? NX : 1];
#pragma unroll
  for (int k = 0; k < NX; ++k)
    if (g + (k + 1) * NG < cnt) issue(g + (k + 1) * NG, cx[k], blx[k], ex[k]);
  if (first) finish(c, bl, e);
#pragma unroll
  for (int k = 0; k < NX; ++k)
    if (g + (k + 1) * NG < cnt) finish(cx[k], blx[k], ex[k]);
  for (int t = g + (NX + 1) * NG; t < cnt; t += NG) {
    issue(t, c, bl, e);
    finish(c, bl, e);
  }
}

// Set-up: assembled stencils of the listed nodes. One wavefront per node; lane (o, g) applies the
// element rows to the unit vector of field g at offset o, which yields column (o, g) of the row.
template <int D>
__global__ void __launch_bounds__(256) node_stencil_kernel(const OpConsts* __restrict__ oc,
                                                          const int* __restrict__ cell_info,
                                                          const double* __restrict__ cut, double alpha_f,
                                                          const int* __restrict__ nodes, int64_t count,
                                                          double* __restrict__ nsten) {
  constexpr int NS = PT<D>::NST;
  __shared__ RefMats<D> rm;
  stage_refmats<D, 256, double>(oc, rm);
  __syncthreads();
  const int64_t k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int n = oc->n;
  for (int col = lane; col < NS * (D + 1) && k < count; col += 64) {
    const int o = col % NS, g = col / NS;
    const int oo[3] = {o % 3 - 1, (o / 3) % 3 - 1, D == 3 ? o / 9 - 1 : 0};
    int c[3];
    node_coords<D>(nodes[k], n, c);
    double acc[D + 1];
#pragma unroll
    for (int f = 0; f <= D; ++f) acc[f] = 0;
    node_apply<D, false>(
        rm, [&](const int* cc) { return cell_info[D == 2 ? cc[0] + n * cc[1] : cc[0] + n * (cc[1] + n * cc[2])]; },
        [&](const int*, int info) -> const double* { return cut + (int64_t)info * PT<D>::NEL; }, alpha_f, n, c,
        [&](int f, const int* q) {
          bool hit = f == g;
#pragma unroll
          for (int a = 0; a < D; ++a) hit = hit && q[a] == oo[a];
          return hit ? 1.0 : 0.0;
        },
        acc);
    double* p = nsten + k * PT<D>::NSTEN;
    if (g < D) {
      if (g == 0) p[sten_index<D>(0, o)] = acc[0];
      p[sten_index<D>(1 + D + g, o)] = acc[D];
    } else {
#pragma unroll
      for (int f = 0; f < D; ++f) p[sten_index<D>(1 + f, o)] = acc[f];
      p[sten_index<D>(1 + 2 * D, o)] = acc[D];
    }
  }
}

template <int D>
hipError_t k_node_stencils(const Ctx& c, const Level& L, const int* nodes, hipStream_t s) {
  if (L.n_nsten == 0) return hipSuccess;
  node_stencil_kernel<D><<<dim3((unsigned)((L.n_nsten + 3) / 4)), dim3(256), 0, s>>>(
      L.consts, L.cell_info, L.cut_mats, c.prm.alpha_fict, nodes, L.n_nsten, L.nsten);
  return hipGetLastError();
}

template <int D, class T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) residual_tile_kernel(const OpConsts* __restrict__ oc,
                                                           const int* __restrict__ node_op,
                                                           const T* __restrict__ nsten, int ntx, int nty, int ntz,
                                                           const T* __restrict__ x, const T* __restrict__ b,
                                                           T* __restrict__ r, int64_t sv) {
  // stacked vectors (sv apart): blockIdx.y is the vector
  x += (int64_t)blockIdx.y * sv;
  b += (int64_t)blockIdx.y * sv;
  r += (int64_t)blockIdx.y * sv;
  constexpr int TX = TileShape<D>::TX, TY = TileShape<D>::TY, TZ = TileShape<D>::TZ;
  constexpr int XW = TX + 2, XH = TY + 2, XD = D == 3 ? TZ + 2 : 1, XP = XW * XH * XD;
  constexpr int NXL = ((D + 1) * XP + 255) / 256;
  __shared__ T xs[(D + 1) * XP];
  const int n = oc->n;
  const int m = n + 1;
  const int64_t N = D == 2 ? (int64_t)m * m : (int64_t)m * m * m;
  const int nt[3] = {ntx, nty, ntz};
  int t[3];
  tile_coords<D, D == 3 ? 4 : 0>(blockIdx.x, nt, t);
  const int o0 = t[0] * TX - 1, o1 = t[1] * TY - 1, o2 = D == 3 ? t[2] * TZ - 1 : 0;
  const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = D == 3 ? threadIdx.x / (TX * TY) : 0;
  const int c[3] = {t[0] * TX + tx, t[1] * TY + ty, D == 3 ? t[2] * TZ + tz : 0};
  const bool inside = c[0] < m && c[1] < m && (D == 2 || c[2] < m);
  const int64_t node = D == 2 ? c[0] + (int64_t)m * c[1] : c[0] + (int64_t)m * (c[1] + (int64_t)m * c[2]);
  // every global load of the tile is issued before the first LDS store
  T bv[D + 1];
#pragma unroll
  for (int f = 0; f <= D; ++f) bv[f] = inside ? b[f * N + node] : T(0);
  const int op = inside ? node_op[node] : -1;
  T xv[NXL];
#pragma unroll
  for (int k = 0; k < NXL; ++k) {
    const int e = threadIdx.x + 256 * k;
    const int f = e / XP, p = e % XP;
    const int gx = o0 + p % XW, gy = o1 + (p / XW) % XH, gz = D == 3 ? o2 + p / (XW * XH) : 0;
    const bool ok = e < (D + 1) * XP && gx >= 0 && gx < m && gy >= 0 && gy < m && (D == 2 || (gz >= 0 && gz < m));
    xv[k] = ok ? x[f * N + (D == 2 ? gx + (int64_t)m * gy : gx + (int64_t)m * (gy + (int64_t)m * gz))] : T(0);
  }
#pragma unroll
  for (int k = 0; k < NXL; ++k)
    if (threadIdx.x + 256 * k < (D + 1) * XP) xs[threadIdx.x + 256 * k] = xv[k];
  __syncthreads();
  if (!inside) return;
  const int base = (tx + 1) + XW * ((ty + 1) + XH * (tz + 1) * (D == 3 ? 1 : 0));
  T acc[D + 1];
#pragma unroll
  for (int f = 0; f <= D; ++f) acc[f] = 0;
  node_row_apply<D, true, T>(oc->pack, op, nsten,
                    [&](int f, const int* o) {
                      return xs[f * XP + base + o[0] + XW * (o[1] + (D == 3 ? XH * o[2] : 0))];
                    },
                    acc);
#pragma unroll
  for (int f = 0; f <= D; ++f) r[f * N + node] = bv[f] - acc[f];
}

// Batched ||b - L x||^2 over independent 2D problems: one 32 x 8 tile per workgroup (the residual
// arithmetic of residual_tile_kernel), its partial sum written to part[block]; then one workgroup
// per job adds its partials in a fixed order.
__global__ void __launch_bounds__(256) residual_sumsq2_batch_kernel(const NormJob* __restrict__ jobs,
                                                                    const int* __restrict__ block_job,
                                                                    double* __restrict__ part) {
  constexpr int TX = TileShape<2>::TX, TY = TileShape<2>::TY;
  constexpr int XW = TX + 2, XH = TY + 2, XP = XW * XH;
  constexpr int NXL = (3 * XP + 255) / 256;
  __shared__ double xs[3 * XP];
  __shared__ double sh[4];
  const NormJob J = jobs[block_job[blockIdx.x]];
  // every pointer of the job addresses device memory (see gmem)
  const gmem<const OpConsts>* __restrict__ oc = (const gmem<const OpConsts>*)J.oc;
  const gmem<const double>* __restrict__ jb = (const gmem<const double>*)J.b;
  const gmem<const double>* __restrict__ jx = (const gmem<const double>*)J.x;
  const gmem<const int>* __restrict__ jop = (const gmem<const int>*)J.node_op;
  const gmem<const double>* __restrict__ jst = (const gmem<const double>*)J.nsten;
  const int bid = (int)blockIdx.x - J.block0;
  const int n = oc->n;
  const int m = n + 1;
  const int64_t N = (int64_t)m * m;
  const int nt[3] = {J.ntx, J.nty, 1};
  int t[3];
  tile_coords<2>(bid, nt, t);
  const int o0 = t[0] * TX - 1, o1 = t[1] * TY - 1;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int c[3] = {t[0] * TX + tx, t[1] * TY + ty, 0};
  const bool inside = c[0] < m && c[1] < m;
  const int64_t node = c[0] + (int64_t)m * c[1];
  double bv[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) bv[f] = inside ? jb[f * N + node] : 0.0;
  const int op = inside ? jop[node] : -1;
  double xv[NXL];
#pragma unroll
  for (int k = 0; k < NXL; ++k) {
    const int e = threadIdx.x + 256 * k;
    const int f = e / XP, p = e % XP;
    const int gx = o0 + p % XW, gy = o1 + p / XW;
    const bool ok = e < 3 * XP && gx >= 0 && gx < m && gy >= 0 && gy < m;
    xv[k] = ok ? jx[f * N + gx + (int64_t)m * gy] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < NXL; ++k)
    if (threadIdx.x + 256 * k < 3 * XP) xs[threadIdx.x + 256 * k] = xv[k];
  __syncthreads();
  double ss = 0;
  if (inside) {
    const int base = (tx + 1) + XW * (ty + 1);
    double acc[3] = {0, 0, 0};
    node_row_apply<2, true, double>((const double*)oc->pack, op, jst,
                                    [&](int f, const int* o) { return xs[f * XP + base + o[0] + XW * o[1]]; }, acc);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const double r = bv[f] - acc[f];
      ss += r * r;
    }
  }
  ss = wave_sum(ss);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ss;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void finish_batch_sumsq_kernel(const NormJob* __restrict__ jobs, const double* __restrict__ part,
                                          double* __restrict__ out) {
  const NormJob J = jobs[blockIdx.x];
  __shared__ double sh[4];
  double s = 0;
  for (int i = threadIdx.x; i < J.nblocks; i += blockDim.x) s += part[J.block0 + i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

int batch_norm_blocks(const Level& L) {
  const int m = L.n + 1;
  return ((m + TileShape<2>::TX - 1) / TileShape<2>::TX) * ((m + TileShape<2>::TY - 1) / TileShape<2>::TY);
}

NormJob batch_norm_job(const Level& L, const double* x, const double* b) {
  const int m = L.n + 1;
  return NormJob{L.consts, L.node_op, L.nsten, x, b, (m + TileShape<2>::TX - 1) / TileShape<2>::TX,
                 (m + TileShape<2>::TY - 1) / TileShape<2>::TY, 0, 0};
}

hipError_t k_batch_sumsq(const NormJob* jobs, int njobs, const int* block_job, int nblocks, double* part, double* out,
                         hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  residual_sumsq2_batch_kernel<<<dim3((unsigned)nblocks), dim3(256), 0, s>>>(jobs, block_job, part);
  finish_batch_sumsq_kernel<<<dim3((unsigned)njobs), dim3(256), 0, s>>>(jobs, part, out);
  return hipGetLastError();
}

template <int D>
void tile_grid(int n, int* nt) {
  nt[0] = (n + 1 + TileShape<D>::TX - 1) / TileShape<D>::TX;
  nt[1] = (n + 1 + TileShape<D>::TY - 1) / TileShape<D>::TY;
  nt[2] = D == 3 ? (n + 1 + TileShape<D>::TZ - 1) / TileShape<D>::TZ : 1;
}

template <int D, class T>
hipError_t k_residual(const Ctx& c, const Level& L, const T* x, const T* b, T* r, hipStream_t s, int nrhs,
                      int64_t sv) {
  int nt[3];
  tile_grid<D>(L.n, nt);
  const int nb = nt[0] * nt[1] * nt[2];
  residual_tile_kernel<D, T><<<dim3((unsigned)nb, (unsigned)nrhs), dim3(256), 0, s>>>(
      L.consts, L.node_op, LV<T>::nsten(L), nt[0], nt[1], nt[2], x, b, r, sv);
  return hipGetLastError();
}

// ================================================================================================
// Grid transfers (Eq. 13, one GPU: T = identity). P is the Q1 interpolation from level l-1 to l
// (coarse node 2I coincides with fine node I); R = P^T. Gather form, one thread per output node.
// ================================================================================================
// b_c at coarse node `node` = sum of the fine residuals around fine node 2*node, weights 1/2 per
// offset axis (R = P^T).
template <int D, class T>
__device__ __forceinline__ void restrict_node(int nf, int64_t Nf, int nc, int64_t Nc, const T* __restrict__ rf,
                                              T* __restrict__ bc, int64_t node) {
  int c[3];
  node_coords<D>(node, nc, c);
  T acc[D + 1];
  for (int f = 0; f <= D; ++f) acc[f] = 0;
  constexpr int NO = D == 2 ? 9 : 27;
  for (int o = 0; o < NO; ++o) {
    int fc[3] = {0, 0, 0};
    T w = 1;
    bool in = true;
    int t = o;
    for (int k = 0; k < D; ++k) {
      const int off = t % 3 - 1;
      t /= 3;
      fc[k] = 2 * c[k] + off;
      if (fc[k] < 0 || fc[k] > nf) in = false;
      if (off != 0) w *= 0.5;
    }
    if (!in) continue;
    const int64_t j = node_index<D>(fc, nf);
    for (int f = 0; f <= D; ++f) acc[f] += w * rf[f * Nf + j];
  }
  for (int f = 0; f <= D; ++f) bc[f * Nc + node] = acc[f];
}

// Q1 interpolation at the fine node with coordinates c of the coarse values xat(cc) (cc: coarse
// node coordinates): the coarse nodes of the enclosing coarse cell face, edge or vertex, in a fixed
// order, weighted by 1/2 per odd coordinate.
template <int D, class T, class CA>
__device__ __forceinline__ T prolong_sum(const int* c, CA&& xat) {
  T acc = 0;
  for (int t = 0; t < (1 << D); ++t) {
    int cc[3] = {0, 0, 0};
    T w = 1;
    bool valid = true;
    for (int k = 0; k < D; ++k) {
      const int bit = (t >> k) & 1;
      if ((c[k] & 1) == 0) {
        if (bit) valid = false;
        cc[k] = c[k] >> 1;
      } else {
        cc[k] = (c[k] >> 1) + bit;
        w *= 0.5;
      }
    }
    if (!valid) continue;
    acc += w * xat(cc);
  }
  return acc;
}

// Q1 interpolation of field f of the coarse vector xc at the fine node with coordinates c.
template <int D, class T>
__device__ __forceinline__ T prolong_value(int nc, int64_t Nc, const T* __restrict__ xc, const int* c, int f) {
  return prolong_sum<D, T>(c, [&](const int* cc) { return xc[f * Nc + node_index<D>(cc, nc)]; });
}

// x_f at fine node `node` += Q1 interpolation of the coarse correction.
template <int D, class T>
__device__ __forceinline__ void prolong_node(int nf, int64_t Nf, int nc, int64_t Nc, const T* __restrict__ xc,
                                             T* __restrict__ xf, int64_t node) {
  int c[3];
  node_coords<D>(node, nf, c);
  for (int f = 0; f <= D; ++f) xf[f * Nf + node] += prolong_value<D, T>(nc, Nc, xc, c, f);
}

// Stacked vectors: blockIdx.y is the vector, fine vectors sf apart, coarse ones sc apart.
template <int D, class T>
__global__ void restrict_kernel(int nf, int64_t Nf, int nc, int64_t Nc, const T* __restrict__ rf,
                                T* __restrict__ bc, int64_t sf, int64_t sc) {
  rf += (int64_t)blockIdx.y * sf;
  bc += (int64_t)blockIdx.y * sc;
  const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (node < Nc) restrict_node<D, T>(nf, Nf, nc, Nc, rf, bc, node);
}

template <int D, class T>
__global__ void prolong_add_kernel(int nf, int64_t Nf, int nc, int64_t Nc, const T* __restrict__ xc,
                                   T* __restrict__ xf, int64_t sc, int64_t sf) {
  xc += (int64_t)blockIdx.y * sc;
  xf += (int64_t)blockIdx.y * sf;
  const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (node < Nf) prolong_node<D, T>(nf, Nf, nc, Nc, xc, xf, node);
}

template <int D, class T>
hipError_t k_restrict(const Ctx& c, int fine, const T* rf, T* bc, hipStream_t s, int nrhs, int64_t sf, int64_t sc) {
  const Level& F = c.lev[fine];
  const Level& C = c.lev[fine - 1];
  const int bs = 256;
  restrict_kernel<D, T><<<dim3((unsigned)((C.N + bs - 1) / bs), (unsigned)nrhs), dim3(bs), 0, s>>>(
      F.n, F.N, C.n, C.N, rf, bc, sf, sc);
  return hipGetLastError();
}

template <int D, class T>
hipError_t k_prolong_add(const Ctx& c, int fine, const T* xc, T* xf, hipStream_t s, int nrhs, int64_t sc,
                         int64_t sf) {
  const Level& F = c.lev[fine];
  const Level& C = c.lev[fine - 1];
  const int bs = 256;
  prolong_add_kernel<D, T><<<dim3((unsigned)((F.N + bs - 1) / bs), (unsigned)nrhs), dim3(bs), 0, s>>>(
      F.n, F.N, C.n, C.N, xc, xf, sc, sf);
  return hipGetLastError();
}

// ================================================================================================
// Entry of the assembled level operator between two nodes (sum over the cells containing both).
// Used to build the dense coarsest operator for the direct solver (Sec. 3).
// ================================================================================================
template <int D>
__device__ double op_entry(const OpConsts* oc, const int* cell_info, const double* cut, const int* ca, int f,
                           const int* cb, int g) {
  constexpr int NN = 1 << D;
  constexpr int NEL = PT<D>::NEL;
  const int n = oc->n;
  int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
  for (int k = 0; k < D; ++k) {
    const int dd = cb[k] - ca[k];
    if (dd < -1 || dd > 1) return 0.0;
    const int mx = ca[k] > cb[k] ? ca[k] : cb[k];
    const int mn = ca[k] < cb[k] ? ca[k] : cb[k];
    lo[k] = mx - 1;  // cells with lower corner in [mx-1, mn]
    cnt[k] = mn - (mx - 1) + 1;
  }
  double s = 0;
  for (int i2 = 0; i2 < cnt[2]; ++i2)
    for (int i1 = 0; i1 < cnt[1]; ++i1)
      for (int i0 = 0; i0 < cnt[0]; ++i0) {
        int cc[3] = {lo[0] + i0, lo[1] + i1, D == 3 ? lo[2] + i2 : 0};
        bool in = true;
        for (int k = 0; k < D; ++k)
          if (cc[k] < 0 || cc[k] > n - 1) in = false;
        if (!in) continue;
        int a = 0, bb = 0;
        for (int k = 0; k < D; ++k) {
          a |= (ca[k] - cc[k]) << k;
          bb |= (cb[k] - cc[k]) << k;
        }
        const int info = cell_info[cell_index<D>(cc, n)];
        const double* Kp;
        const double* Bp;
        int bstride;
        if (info >= 0) {
          Kp = cut + (int64_t)info * NEL;
          Bp = Kp + NN * NN;
          bstride = NN * NN;
        } else {
          const int kind = info == -1 ? 0 : 1;
          Kp = oc->K[kind];
          Bp = oc->B[kind][0];
          bstride = 64;
        }
        if (f < D && g < D) {
          if (f == g) s += Kp[a * NN + bb];
        } else if (f < D && g == D) {
          s += Bp[f * bstride + a * NN + bb];
        } else if (f == D && g < D) {
          s += Bp[g * bstride + bb * NN + a];
        } else {
          s += oc->C[a * NN + bb];
        }
        for (int k = 0; k < D; ++k)
          for (int sd = 0; sd < 2; ++sd) {
            const int face = 2 * k + sd;
            if (!oc->dirichlet[face] || cc[k] != (sd ? n - 1 : 0)) continue;
            if (f < D && g < D) {
              if (f == g) s += oc->FK[face][a * NN + bb];
            } else if (f < D && g == D) {
              if (f == k) s += oc->FB[face][a * NN + bb];
            } else if (f == D && g < D) {
              if (g == k) s += oc->FB[face][bb * NN + a];
            }
          }
      }
  return s;
}

template <int D>
__global__ void coarse_matrix_kernel(const OpConsts* __restrict__ oc, const int* __restrict__ cell_info,
                                     const double* __restrict__ cut, int64_t N, double* A, int lda) {
  const int64_t nd = (D + 1) * N;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nd * nd) return;
  const int64_t row = idx / nd, col = idx % nd;
  const int f = (int)(row / N), g = (int)(col / N);
  int ca[3], cb[3];
  node_coords<D>(row % N, oc->n, ca);
  node_coords<D>(col % N, oc->n, cb);
  A[row * lda + col] = op_entry<D>(oc, cell_info, cut, ca, f, cb, g);
}

template <int D>
hipError_t k_coarse_matrix(const Ctx& c, const Level& L, double* A, int lda, hipStream_t s) {
  const int64_t nd = (D + 1) * L.N;
  const int bs = 256;
  coarse_matrix_kernel<D><<<dim3((unsigned)((nd * nd + bs - 1) / bs)), dim3(bs), 0, s>>>(L.consts, L.cell_info,
                                                                                        L.cut_mats, L.N, A, lda);
  return hipGetLastError();
}

// x = A b with a dense row-major n x n matrix (coarsest-grid solve through the stored inverse):
// one wavefront per row.
template <class T, class PA, class PB, class PX>
__device__ __forceinline__ void dense_row(PA __restrict__ A, int n, PB __restrict__ b, PX __restrict__ x, int row,
                                          int lane) {
  T s = 0;
  for (int j = lane; j < n; j += 64) s += A[(int64_t)row * n + j] * b[j];
  s = wave_sum(s);
  if (lane == 0) x[row] = s;
}

template <class T>
__global__ void dense_matvec_kernel(const T* __restrict__ A, int n, const T* __restrict__ b, T* __restrict__ x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row < n) dense_row<T>(A, n, b, x, row, threadIdx.x & 63);
}

__global__ void dense_matvec_batch_kernel(const DenseJob* __restrict__ jobs, const int* __restrict__ block_job) {
  const DenseJob J = jobs[block_job[blockIdx.x]];
  const int row = ((int)blockIdx.x - J.block0) * 4 + (threadIdx.x >> 6);
  if (row < J.n)
    dense_row<double>((const gmem<const double>*)J.A, J.n, (const gmem<const double>*)J.b, (gmem<double>*)J.x, row,
                      threadIdx.x & 63);
}

hipError_t k_batch_dense(const DenseJob* jobs, const int* block_job, int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  dense_matvec_batch_kernel<<<dim3((unsigned)nblocks), dim3(256), 0, s>>>(jobs, block_job);
  return hipGetLastError();
}

// nrhs right-hand sides (b and x n apart), blockIdx.y the vector.
__global__ void dense_matvec_multi_kernel(const double* __restrict__ A, int n, const double* __restrict__ b,
                                          double* __restrict__ x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t k = blockIdx.y;
  if (row < n) dense_row<double>(A, n, b + k * n, x + k * n, row, threadIdx.x & 63);
}

hipError_t k_dense_matvec_multi(const double* A, int n, const double* b, double* x, int nrhs, hipStream_t s) {
  dense_matvec_multi_kernel<<<dim3((unsigned)((n + 3) / 4), (unsigned)nrhs), dim3(256), 0, s>>>(A, n, b, x);
  return hipGetLastError();
}

template <class T>
hipError_t k_dense_matvec(const T* A, int n, const T* b, T* x, hipStream_t s) {
  dense_matvec_kernel<T><<<dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s>>>(A, n, b, x);
  return hipGetLastError();
}

// Sum of squares: fixed grid, fixed per-block order, then one block combines (deterministic).
__global__ void sumsq_kernel(const double* __restrict__ v, int64_t n, double* __restrict__ partial) {
  __shared__ double sh[4];
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double t = v[i];
    s += t * t;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void finish_sumsq_kernel(const double* __restrict__ partial, int nb, double* out) {
  __shared__ double sh[4];
  double s = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = sh[0] + sh[1] + sh[2] + sh[3];
}

hipError_t k_sumsq(const double* v, int64_t n, double* partial, int nblocks, hipStream_t s) {
  sumsq_kernel<<<dim3(nblocks), dim3(256), 0, s>>>(v, n, partial);
  return hipGetLastError();
}

hipError_t k_finish_sumsq(const double* partial, int nblocks, double* out, hipStream_t s) {
  finish_sumsq_kernel<<<dim3(1), dim3(256), 0, s>>>(partial, nblocks, out);
  return hipGetLastError();
}

static unsigned stream_blocks(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  return (unsigned)nb;
}

// ================================================================================================
// Krylov (FGMRES) vector kernels, FP64: block inner products against j basis vectors at once and
// the matching combined update. Fixed grid and summation order (deterministic).
// ================================================================================================
constexpr int kKrylovBlocks = 256;

// part[blk * j + i] = s * sum over this block's slice of V_i . w, for i < j (V_i = V + i * ld):
// w is read once per chunk of up to 16 basis vectors, each thread keeping 16 running sums.
constexpr int kDotChunk = 16;
__global__ void __launch_bounds__(256) multi_dot_kernel(const double* __restrict__ V, int64_t ld, int j,
                                                        const double* __restrict__ w, int64_t n, double s,
                                                        double* __restrict__ part) {
  __shared__ double sh[4][kDotChunk];
  for (int i0 = 0; i0 < j; i0 += kDotChunk) {
    const int cnt = min(kDotChunk, j - i0);
    double acc[kDotChunk];
#pragma unroll
    for (int q = 0; q < kDotChunk; ++q) acc[q] = 0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
      const double wk = w[k];
#pragma unroll
      for (int q = 0; q < kDotChunk; ++q)
        if (q < cnt) acc[q] += V[(i0 + q) * ld + k] * wk;
    }
#pragma unroll
    for (int q = 0; q < kDotChunk; ++q) {
      const double v = wave_sum(acc[q]);
      if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < cnt)
      part[blockIdx.x * j + i0 + threadIdx.x] =
          s * (sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x]);
    __syncthreads();
  }
}

// h[i] = sum over blocks of part[blk * j + i]
__global__ void multi_dot_finish_kernel(const double* __restrict__ part, int nb, int j, double* __restrict__ h) {
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    double acc = 0;
    for (int blk = 0; blk < nb; ++blk) acc += part[blk * j + i];
    h[i] = acc;
  }
}

// w = s * w - sum_{i < j} h[i] V_i
__global__ void multi_axpy_kernel(double* __restrict__ w, double s, const double* __restrict__ V, int64_t ld, int j,
                                  const double* __restrict__ h, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double acc = s * w[k];
    for (int i = 0; i < j; ++i) acc -= h[i] * V[i * ld + k];
    w[k] = acc;
  }
}

__global__ void scale_copy_kernel(const double* __restrict__ w, double a, double* __restrict__ v, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    v[k] = a * w[k];
}

hipError_t k_multi_dot(const double* V, int64_t ld, int j, const double* w, int64_t n, double s, double* part,
                       double* h, hipStream_t st) {
  multi_dot_kernel<<<dim3(kKrylovBlocks), dim3(256), 0, st>>>(V, ld, j, w, n, s, part);
  multi_dot_finish_kernel<<<dim3(1), dim3(64), 0, st>>>(part, kKrylovBlocks, j, h);
  return hipGetLastError();
}

hipError_t k_multi_axpy(double* w, double s, const double* V, int64_t ld, int j, const double* h, int64_t n,
                        hipStream_t st) {
  multi_axpy_kernel<<<dim3(stream_blocks(n)), dim3(256), 0, st>>>(w, s, V, ld, j, h, n);
  return hipGetLastError();
}

hipError_t k_scale_copy(const double* w, double a, double* v, int64_t n, hipStream_t st) {
  scale_copy_kernel<<<dim3(stream_blocks(n)), dim3(256), 0, st>>>(w, a, v, n);
  return hipGetLastError();
}

template <class T>
__global__ void zero_kernel(T* v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = T(0);
}

template <class T>
hipError_t k_zero(T* v, int64_t n, hipStream_t s) {
  zero_kernel<T><<<dim3(stream_blocks(n)), dim3(256), 0, s>>>(v, n);
  return hipGetLastError();
}

// Precision conversions of the mixed-precision solve: the FP64 residual rounded to FP32 for the FP32
// V-cycle, and its FP32 correction added to the FP64 iterate.
__global__ void round_to_float_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

__global__ void add_float_kernel(const float* __restrict__ src, double* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] += (double)src[i];
}

hipError_t k_round_to_float(const double* src, float* dst, int64_t n, hipStream_t s) {
  round_to_float_kernel<<<dim3(stream_blocks(n)), dim3(256), 0, s>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t k_add_float(const float* src, double* dst, int64_t n, hipStream_t s) {
  add_float_kernel<<<dim3(stream_blocks(n)), dim3(256), 0, s>>>(src, dst, n);
  return hipGetLastError();
}

}  // namespace fcg

#include "fcgmg_patch.inl"

namespace fcg {
#define FCG_INST(D)                                                                                           \
  template hipError_t k_classify_cells<D>(const Ctx&, Level&, signed char*, hipStream_t);                     \
  template hipError_t k_cut_matrices<D>(const Ctx&, Level&, const int*, hipStream_t);                         \
  template hipError_t k_rhs<D>(const Ctx&, const Level&, double*, hipStream_t);                               \
  template hipError_t k_residual<D, double>(const Ctx&, const Level&, const double*, const double*, double*,   \
                                            hipStream_t, int, int64_t);                                       \
  template hipError_t k_residual<D, float>(const Ctx&, const Level&, const float*, const float*, float*,       \
                                           hipStream_t, int, int64_t);                                        \
  template hipError_t k_node_stencils<D>(const Ctx&, const Level&, const int*, hipStream_t);                  \
  template hipError_t k_restrict<D, double>(const Ctx&, int, const double*, double*, hipStream_t, int, int64_t, \
                                            int64_t);                                                         \
  template hipError_t k_restrict<D, float>(const Ctx&, int, const float*, float*, hipStream_t, int, int64_t,  \
                                           int64_t);                                                          \
  template hipError_t k_prolong_add<D, double>(const Ctx&, int, const double*, double*, hipStream_t, int,     \
                                               int64_t, int64_t);                                             \
  template hipError_t k_prolong_add<D, float>(const Ctx&, int, const float*, float*, hipStream_t, int,        \
                                              int64_t, int64_t);                                              \
  template hipError_t k_coarse_matrix<D>(const Ctx&, const Level&, double*, int, hipStream_t);                \
  template hipError_t k_patch_inverse_rows<D>(const Ctx&, const Level&, const int*, int64_t, double*,         \
                                              hipStream_t);                                                   \
  template hipError_t k_apply_regular<D, double>(const Ctx&, const Level&, const double*, double*, hipStream_t, \
                                                 int, int64_t);                                               \
  template hipError_t k_apply_regular<D, float>(const Ctx&, const Level&, const float*, float*, hipStream_t,  \
                                                int, int64_t);                                                \
  template hipError_t k_apply_irregular<D, double>(const Ctx&, const Level&, const double*, double*,          \
                                                   hipStream_t);                                              \
  template hipError_t k_apply_irregular<D, float>(const Ctx&, const Level&, const float*, float*, hipStream_t); \
  template hipError_t k_apply_irregular_multi<D, double>(const Ctx&, const Level&, const double*, double*,    \
                                                         int64_t, int, hipStream_t);                          \
  template hipError_t k_patch_solve<D>(const Ctx&, const Level&, int, const double*, double*, hipStream_t);  \
  template hipError_t k_store_matrices<D>(const Ctx&, const Level&, const int*, int64_t, double*,             \
                                          hipStream_t);                                                       \
  template int pattern_size<D>();                                                                             \
  template void pattern_entries<D>(std::vector<int>&);
FCG_INST(2)
FCG_INST(3)
#undef FCG_INST
#define FCG_INST_T(T)                                                                                         \
  template hipError_t k_sweep_fused2<T>(const Ctx&, const Level&, const T*, const T*, T*, int, const T*,       \
                                        hipStream_t);                                                         \
  template hipError_t k_residual_restrict2<T>(const Ctx&, const Level&, const T*, const T*, T*, hipStream_t);   \
  template hipError_t k_dense_matvec<T>(const T*, int, const T*, T*, hipStream_t);                            \
  template hipError_t k_zero<T>(T*, int64_t, hipStream_t);
FCG_INST_T(double)
FCG_INST_T(float)
#undef FCG_INST_T
}  // namespace fcg
