// HIP kernels (gfx950) of the fcgmg library: finite cell Stokes operator, restricted additive
// smoother under the three cache policies, grid transfers and reductions.
// Method: Saberi & Vogel, arXiv 2403.11636 (equation numbers refer to the paper).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "fcgmg_impl.h"

namespace fcg {

namespace {

constexpr int kMaxLocalBalls = 16;

__device__ __forceinline__ double wave_sum(double v) {
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
  classify_cells_kernel<D><<<dim3((unsigned)nb), dim3(bs), 0, s>>>(c.geom(), L.n, L.h, L.ncells, kinds);
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
__global__ void __launch_bounds__(64) cut_matrices_kernel(Geom g, int n, double h, double eta, const int* cut_cells,
                                                          int64_t ncut, double* out) {
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
    for (int k = 0; k < NPER; ++k) {
      const int e = (int)threadIdx.x + 64 * k;
      if (e < NEL) out[ic * NEL + e] = acc[k];
    }
    __syncthreads();
  }
}

template <int D>
hipError_t k_cut_matrices(const Ctx& c, Level& L, const int* cut_cells, hipStream_t s) {
  if (L.n_cut == 0) return hipSuccess;
  const int64_t nb = L.n_cut < 65536 ? L.n_cut : 65536;
  cut_matrices_kernel<D><<<dim3((unsigned)nb), dim3(64), 0, s>>>(c.geom(), L.n, L.h, c.prm.eta, cut_cells, L.n_cut,
                                                                 L.cut_mats);
  return hipGetLastError();
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
  rhs_kernel<D><<<dim3((unsigned)nb), dim3(bs), 0, s>>>(c.geom(), L.consts, c.prm.force, c.prm.eta, c.prm.ubar, bc[0],
                                                        bc[1], bc[2], bc[3], bc[4], bc[5], L.N, b);
  return hipGetLastError();
}

// ================================================================================================
// Residual r = b - L x (Eq. 12, 14): one thread per node, summing the element contributions of the
// 2^d cells around it (uncut cells: reference matrices times alpha; cut cells: stored integrals;
// Dirichlet walls: Nitsche face matrices). The stabilisation C has no alpha (Eq. 10).
// ================================================================================================
template <int D>
__global__ void __launch_bounds__(256) residual_kernel(const OpConsts* __restrict__ oc, const int* __restrict__ cell_info,
                                                      const double* __restrict__ cut, int64_t N,
                                                      const double* __restrict__ x, const double* __restrict__ b,
                                                      double* __restrict__ r) {
  constexpr int NN = 1 << D;
  constexpr int NEL = PT<D>::NEL;
  const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (node >= N) return;
  const int n = oc->n;
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
    double u[D + 1][NN];
    for (int bn = 0; bn < NN; ++bn) {
      int cb[3] = {cc[0] + (bn & 1), cc[1] + ((bn >> 1) & 1), D == 3 ? cc[2] + ((bn >> 2) & 1) : 0};
      const int64_t j = node_index<D>(cb, n);
      for (int f = 0; f <= D; ++f) u[f][bn] = x[f * N + j];
    }
    for (int bn = 0; bn < NN; ++bn) {
      const double kab = Kp[a * NN + bn];
      const double cab = oc->C[a * NN + bn];
      for (int f = 0; f < D; ++f) {
        acc[f] += kab * u[f][bn] + Bp[f * bstride + a * NN + bn] * u[D][bn];
        acc[D] += Bp[f * bstride + bn * NN + a] * u[f][bn];
      }
      acc[D] += cab * u[D][bn];
    }
    // Nitsche terms of Dirichlet walls touched by this cell
    for (int k = 0; k < D; ++k)
      for (int sd = 0; sd < 2; ++sd) {
        const int face = 2 * k + sd;
        if (!oc->dirichlet[face]) continue;
        if (cc[k] != (sd ? n - 1 : 0)) continue;
        const double* FK = oc->FK[face];
        const double* FB = oc->FB[face];
        for (int bn = 0; bn < NN; ++bn) {
          for (int f = 0; f < D; ++f) acc[f] += FK[a * NN + bn] * u[f][bn];
          acc[k] += FB[a * NN + bn] * u[D][bn];
          acc[D] += FB[bn * NN + a] * u[k][bn];
        }
      }
  }
  for (int f = 0; f <= D; ++f) r[f * N + node] = b[f * N + node] - acc[f];
}

template <int D>
hipError_t k_residual(const Ctx& c, const Level& L, const double* x, const double* b, double* r, hipStream_t s) {
  const int bs = 256;
  const int64_t nb = (L.N + bs - 1) / bs;
  residual_kernel<D><<<dim3((unsigned)nb), dim3(bs), 0, s>>>(L.consts, L.cell_info, L.cut_mats, L.N, x, b, r);
  return hipGetLastError();
}

// ================================================================================================
// Grid transfers (Eq. 13, one GPU: T = identity). P is the Q1 interpolation from level l-1 to l
// (coarse node 2I coincides with fine node I); R = P^T. Gather form, one thread per output node.
// ================================================================================================
template <int D>
__global__ void restrict_kernel(int nf, int64_t Nf, int nc, int64_t Nc, const double* __restrict__ rf,
                                double* __restrict__ bc) {
  const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (node >= Nc) return;
  int c[3];
  node_coords<D>(node, nc, c);
  double acc[D + 1];
  for (int f = 0; f <= D; ++f) acc[f] = 0;
  constexpr int NO = D == 2 ? 9 : 27;
  for (int o = 0; o < NO; ++o) {
    int fc[3] = {0, 0, 0};
    double w = 1;
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

template <int D>
__global__ void prolong_add_kernel(int nf, int64_t Nf, int nc, int64_t Nc, const double* __restrict__ xc,
                                   double* __restrict__ xf) {
  const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (node >= Nf) return;
  int c[3];
  node_coords<D>(node, nf, c);
  double acc[D + 1];
  for (int f = 0; f <= D; ++f) acc[f] = 0;
  for (int t = 0; t < (1 << D); ++t) {
    int cc[3] = {0, 0, 0};
    double w = 1;
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
    const int64_t j = node_index<D>(cc, nc);
    for (int f = 0; f <= D; ++f) acc[f] += w * xc[f * Nc + j];
  }
  for (int f = 0; f <= D; ++f) xf[f * Nf + node] += acc[f];
}

template <int D>
hipError_t k_restrict(const Ctx& c, int fine, const double* rf, double* bc, hipStream_t s) {
  const Level& F = c.lev[fine];
  const Level& C = c.lev[fine - 1];
  const int bs = 256;
  restrict_kernel<D><<<dim3((unsigned)((C.N + bs - 1) / bs)), dim3(bs), 0, s>>>(F.n, F.N, C.n, C.N, rf, bc);
  return hipGetLastError();
}

template <int D>
hipError_t k_prolong_add(const Ctx& c, int fine, const double* xc, double* xf, hipStream_t s) {
  const Level& F = c.lev[fine];
  const Level& C = c.lev[fine - 1];
  const int bs = 256;
  prolong_add_kernel<D><<<dim3((unsigned)((F.N + bs - 1) / bs)), dim3(bs), 0, s>>>(F.n, F.N, C.n, C.N, xc, xf);
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
__global__ void dense_matvec_kernel(const double* __restrict__ A, int n, const double* __restrict__ b,
                                    double* __restrict__ x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0;
  for (int j = lane; j < n; j += 64) s += A[(int64_t)row * n + j] * b[j];
  s = wave_sum(s);
  if (lane == 0) x[row] = s;
}

hipError_t k_dense_matvec(const double* A, int n, const double* b, double* x, hipStream_t s) {
  dense_matvec_kernel<<<dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s>>>(A, n, b, x);
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

__global__ void zero_kernel(double* v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = 0.0;
}

hipError_t k_zero(double* v, int64_t n, hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  zero_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(v, n);
  return hipGetLastError();
}

}  // namespace fcg

#include "fcgmg_patch.inl"

namespace fcg {
#define FCG_INST(D)                                                                                           \
  template hipError_t k_classify_cells<D>(const Ctx&, Level&, signed char*, hipStream_t);                     \
  template hipError_t k_cut_matrices<D>(const Ctx&, Level&, const int*, hipStream_t);                         \
  template hipError_t k_rhs<D>(const Ctx&, const Level&, double*, hipStream_t);                               \
  template hipError_t k_residual<D>(const Ctx&, const Level&, const double*, const double*, double*,           \
                                    hipStream_t);                                                             \
  template hipError_t k_restrict<D>(const Ctx&, int, const double*, double*, hipStream_t);                    \
  template hipError_t k_prolong_add<D>(const Ctx&, int, const double*, double*, hipStream_t);                 \
  template hipError_t k_coarse_matrix<D>(const Ctx&, const Level&, double*, int, hipStream_t);                \
  template hipError_t k_patch_inverse_rows<D>(const Ctx&, const Level&, const int*, int64_t, double*,         \
                                              hipStream_t);                                                   \
  template hipError_t k_apply_inverse<D>(const Ctx&, const Level&, const double*, double*, hipStream_t);      \
  template hipError_t k_patch_solve<D>(const Ctx&, const Level&, int, const double*, double*, hipStream_t);  \
  template hipError_t k_store_matrices<D>(const Ctx&, const Level&, const int*, int64_t, double*,             \
                                          hipStream_t);                                                       \
  template int pattern_size<D>();                                                                             \
  template void pattern_entries<D>(std::vector<int>&);
FCG_INST(2)
FCG_INST(3)
#undef FCG_INST
}  // namespace fcg
