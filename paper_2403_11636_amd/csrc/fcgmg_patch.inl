// Vertex-patch kernels of the restricted additive smoother (Saberi & Vogel, Eq. 15, Sec. 3.1.2).
//
// Local block of subdomain S_i:  L_i = [[I_d (x) K_i, B_i], [B_i^T, C_i]]
//   K_i : velocity block of the 5^d window (the viscous form and the Nitsche terms act on each
//         velocity component alike, so the d velocity blocks are one scalar SPD matrix), stored as
//         a lower band (lexicographic order, half bandwidth 6 / 31);
//   B_i : d blocks 5^d x 3^d;  C_i : 3^d x 3^d stabilisation block.
// The local direct solve ("LU ... down to machine accuracy", Sec. 3.1.2) is done as the block LU
// with the pressure Schur complement S = C - sum_c B_c^T K^{-1} B_c; K = L L^T by a banded
// Cholesky, -S by a dense Cholesky. Entries of the window that fall outside the grid are replaced
// by decoupled identity rows (velocity) / -1 diagonals (pressure), which leaves the in-grid
// solution unchanged.
//
// Included by fcgmg_kernels.hip (single translation unit for all device code).

namespace fcg {

namespace {

template <int D>
struct PatchLDS {
  static constexpr int NV = PT<D>::NV, NP = PT<D>::NP, NB = PT<D>::NB, NPX = PT<D>::NP + 2;
  double Kb[NV * NB];        // lower band of K_i: Kb[i*NB + (i-j)] = K[i][j]
  double X[D * NV * NPX];    // per component c: [B_c | g_c | e_m] -> [V_c | z_c | y] -> [W_c | . | q]
  double S[NP * NP];         // C - sum V^T V, then the Cholesky factor of -S (lower)
  double Sinv[NP * NP];      // S^{-1} (inverse rows only)
  double t[NP];              // reduced pressure right-hand side, then the pressure solution
  double w[D][NP];           // y^T V_c = row m of K^{-1} B_c
  double tc[D][NP];          // S^{-1} w_c (inverse rows only)
  double qg[D];              // y^T z_c
  double cellbuf[PT<D>::NEL];
  double lball[4 * kMaxLocalBalls];
  int cnt;
  int bad;
};

template <int D>
__device__ __forceinline__ int vel_center() {
  return D == 2 ? 12 : 62;
}
template <int D>
__device__ __forceinline__ int pres_center() {
  return D == 2 ? 4 : 13;
}

// Window index helpers: velocity window 5^d (offset -2), pressure window 3^d (offset -1),
// cell window 6^d (cell lower corner offset -3), all lexicographic with x fastest.
template <int D>
__device__ __forceinline__ bool vel_in_grid(const int* c, int n, int v) {
  const int o[3] = {v % 5 - 2, (v / 5) % 5 - 2, D == 3 ? v / 25 - 2 : 0};
  for (int k = 0; k < D; ++k)
    if (c[k] + o[k] < 0 || c[k] + o[k] > n) return false;
  return true;
}
template <int D>
__device__ __forceinline__ bool pres_in_grid(const int* c, int n, int q) {
  const int o[3] = {q % 3 - 1, (q / 3) % 3 - 1, D == 3 ? q / 9 - 1 : 0};
  for (int k = 0; k < D; ++k)
    if (c[k] + o[k] < 0 || c[k] + o[k] > n) return false;
  return true;
}

// Assemble K_i, B_i, C_i of the patch centred at node c from the 6^d cell window (Eq. 15:
// L_i = R_i L R_i^T). source 0: cut cells from the stored integrals; source 1: cut cells
// integrated on the fly (cache_none). One barrier per window cell; within a cell every (a, b)
// pair lands in a distinct entry.
template <int D>
__device__ void patch_assemble(PatchLDS<D>& sh, const OpConsts* __restrict__ oc, const int* __restrict__ cell_info,
                               const double* __restrict__ cut, const Geom& g, double eta, const int* c,
                               int source) {
  constexpr int NN = 1 << D, NV = PT<D>::NV, NP = PT<D>::NP, NB = PT<D>::NB, NPX = NP + 2, NW = PT<D>::NW;
  constexpr int NEL = PT<D>::NEL;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = oc->n;
  for (int i = tid; i < NV * NB; i += nt) sh.Kb[i] = 0;
  for (int i = tid; i < D * NV * NPX; i += nt) sh.X[i] = 0;
  for (int i = tid; i < NP * NP; i += nt) sh.S[i] = 0;
  __syncthreads();
  for (int w = 0; w < NW; ++w) {
    const int wk[3] = {w % 6, (w / 6) % 6, D == 3 ? w / 36 : 0};
    int cc[3] = {0, 0, 0};
    bool in = true;
    for (int k = 0; k < D; ++k) {
      cc[k] = c[k] + wk[k] - 3;
      if (cc[k] < 0 || cc[k] > n - 1) in = false;
    }
    if (!in) continue;
    const int64_t cell = D == 2 ? cc[0] + (int64_t)n * cc[1] : cc[0] + (int64_t)n * (cc[1] + (int64_t)n * cc[2]);
    const int info = cell_info[cell];
    const double* Kp;
    const double* Bp;
    int bstride;
    if (info >= 0) {
      if (source == 1) {
        double lo[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) lo[k] = cc[k] * oc->h;
        const int nb = cull_balls<D>(g, lo, oc->h, sh.lball, &sh.cnt);
        Geom gl = g;
        if (nb >= 0) {
          gl.balls = sh.lball;
          gl.nballs = nb;
        }
        constexpr int NPER = (NEL + PT<D>::THREADS - 1) / PT<D>::THREADS;
        double acc[NPER];
        for (int k = 0; k < NPER; ++k) acc[k] = 0;
        integrate_cell_entries<D>(gl, lo, oc->h, eta, acc, NPER);
        if constexpr (D == 2) {
          if (oc->immersed)
            arc_quadrature2(gl, lo, oc->h, [&](const double* xq, double w, const double* nrm) {
              double phi[4], gr[4][3];
              q1<2>(lo, oc->h, xq, phi, gr);
              for (int k = 0; k < NPER; ++k) {
                const int e = tid + k * nt;
                if (e < NEL) acc[k] += nitsche_entry2(e, eta, oc->lam, w, nrm, phi, gr);
              }
            });
        }
        for (int k = 0; k < NPER; ++k) {
          const int e = tid + k * nt;
          if (e < NEL) sh.cellbuf[e] = acc[k];
        }
        __syncthreads();
        Kp = sh.cellbuf;
      } else {
        Kp = cut + (int64_t)info * NEL;
      }
      Bp = Kp + NN * NN;
      bstride = NN * NN;
    } else {
      const int kind = info == -1 ? 0 : 1;
      Kp = oc->K[kind];
      Bp = oc->B[kind][0];
      bstride = 64;
    }
    int fmask = 0;
    for (int k = 0; k < D; ++k) {
      if (cc[k] == 0 && oc->dirichlet[2 * k]) fmask |= 1 << (2 * k);
      if (cc[k] == n - 1 && oc->dirichlet[2 * k + 1]) fmask |= 1 << (2 * k + 1);
    }
    for (int it = tid; it < NN * NN * (D + 2); it += nt) {
      const int blk = it / (NN * NN), ab = it % (NN * NN), a = ab / NN, b = ab % NN;
      int va = 0, vb = 0, qa = 0, qb = 0, mv = 1, mq = 1;
      bool va_ok = true, vb_ok = true, qa_ok = true, qb_ok = true;
      for (int k = 0; k < D; ++k) {
        const int ak = (a >> k) & 1, bk = (b >> k) & 1;
        const int xa = wk[k] + ak - 1, xb = wk[k] + bk - 1;  // velocity window coordinate
        const int pa = wk[k] + ak - 2, pb = wk[k] + bk - 2;  // pressure window coordinate
        va_ok = va_ok && xa >= 0 && xa <= 4;
        vb_ok = vb_ok && xb >= 0 && xb <= 4;
        qa_ok = qa_ok && pa >= 0 && pa <= 2;
        qb_ok = qb_ok && pb >= 0 && pb <= 2;
        va += xa * mv;
        vb += xb * mv;
        qa += pa * mq;
        qb += pb * mq;
        mv *= 5;
        mq *= 3;
      }
      if (blk == 0) {
        if (va_ok && vb_ok && va >= vb) {
          double v = Kp[a * NN + b];
          for (int f = 0; f < 2 * D; ++f)
            if (fmask & (1 << f)) v += oc->FK[f][a * NN + b];
          sh.Kb[va * NB + (va - vb)] += v;
        }
      } else if (blk <= D) {
        const int cmp = blk - 1;
        if (va_ok && qb_ok) {
          double v = Bp[cmp * bstride + a * NN + b];
          for (int sd = 0; sd < 2; ++sd)
            if (fmask & (1 << (2 * cmp + sd))) v += oc->FB[2 * cmp + sd][a * NN + b];
          sh.X[(cmp * NV + va) * NPX + qb] += v;
        }
      } else {
        if (qa_ok && qb_ok) sh.S[qa * NP + qb] += oc->C[a * NN + b];
      }
    }
    __syncthreads();
  }
}

// Decouple window positions that lie outside the grid (truncated patches at the walls).
template <int D, class LDS>
__device__ void patch_pad(LDS& sh, const int* c, int n) {
  constexpr int NV = PT<D>::NV, NP = PT<D>::NP, NB = PT<D>::NB;
  for (int v = threadIdx.x; v < NV; v += blockDim.x)
    if (!vel_in_grid<D>(c, n, v)) sh.Kb[v * NB] = 1.0;
  for (int q = threadIdx.x; q < NP; q += blockDim.x)
    if (!pres_in_grid<D>(c, n, q)) sh.S[q * NP + q] = -1.0;
  __syncthreads();
}

// Banded Cholesky K = L L^T in place (right-looking, one barrier pair per column).
template <int D, class LDS>
__device__ void band_cholesky(LDS& sh) {
  constexpr int NV = PT<D>::NV, NB = PT<D>::NB, BW = PT<D>::BW;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < NV; ++k) {
    const double dkk = sh.Kb[k * NB];
    if (tid == 0 && !(dkk > 0.0)) sh.bad = 1;
    const double l = sqrt(dkk);
    const int last = k + BW < NV - 1 ? k + BW : NV - 1;
    const int m = last - k;
    __syncthreads();
    for (int i = k + 1 + tid; i <= last; i += nt) sh.Kb[i * NB + (i - k)] /= l;
    if (tid == 0) sh.Kb[k * NB] = l;
    __syncthreads();
    for (int p = tid; p < m * m; p += nt) {
      const int ii = k + 1 + p / m, jj = k + 1 + p % m;
      if (jj <= ii) sh.Kb[ii * NB + (ii - jj)] -= sh.Kb[ii * NB + (ii - k)] * sh.Kb[jj * NB + (jj - k)];
    }
    __syncthreads();
  }
}

// Forward substitution L V = X for the columns [c][col], col < ncol (thread per column).
template <int D>
__device__ void band_forward(PatchLDS<D>& sh, int ncol) {
  constexpr int NV = PT<D>::NV, NB = PT<D>::NB, BW = PT<D>::BW, NPX = PT<D>::NP + 2;
  for (int t = threadIdx.x; t < D * ncol; t += blockDim.x) {
    const int cmp = t / ncol, col = t % ncol;
    double* Xc = sh.X + cmp * NV * NPX + col;
    for (int i = 0; i < NV; ++i) {
      double v = Xc[i * NPX];
      const int k0 = i - BW > 0 ? i - BW : 0;
      for (int k = k0; k < i; ++k) v -= sh.Kb[i * NB + (i - k)] * Xc[k * NPX];
      Xc[i * NPX] = v / sh.Kb[i * NB];
    }
  }
  __syncthreads();
}

// Back substitution L^T W = V for the columns [c][col], col < ncol, plus the e_m column of c = 0.
template <int D>
__device__ void band_backward(PatchLDS<D>& sh, int ncol) {
  constexpr int NV = PT<D>::NV, NB = PT<D>::NB, BW = PT<D>::BW, NP = PT<D>::NP, NPX = NP + 2;
  for (int t = threadIdx.x; t < D * ncol + 1; t += blockDim.x) {
    const int cmp = t < D * ncol ? t / ncol : 0;
    const int col = t < D * ncol ? t % ncol : NP + 1;
    double* Xc = sh.X + cmp * NV * NPX + col;
    for (int i = NV - 1; i >= 0; --i) {
      double v = Xc[i * NPX];
      const int k1 = i + BW < NV - 1 ? i + BW : NV - 1;
      for (int k = i + 1; k <= k1; ++k) v -= sh.Kb[k * NB + (k - i)] * Xc[k * NPX];
      Xc[i * NPX] = v / sh.Kb[i * NB];
    }
  }
  __syncthreads();
}

// S <- S - sum_c V_c^T V_c; with_rhs: t <- t - sum_c V_c^T z_c, qg_c = y^T z_c; w_c = y^T V_c.
template <int D>
__device__ void schur_update(PatchLDS<D>& sh, bool with_rhs) {
  constexpr int NV = PT<D>::NV, NP = PT<D>::NP, NPX = NP + 2;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int mc = vel_center<D>();
  for (int e = tid; e < NP * NP; e += nt) {
    const int i = e / NP, j = e % NP;
    double s = 0;
    for (int cmp = 0; cmp < D; ++cmp) {
      const double* Xc = sh.X + cmp * NV * NPX;
      for (int k = 0; k < NV; ++k) s += Xc[k * NPX + i] * Xc[k * NPX + j];
    }
    sh.S[e] -= s;
  }
  const double* y = sh.X + (NP + 1);  // e_m column of component 0 after the forward pass
  for (int e = tid; e < D * NP + (with_rhs ? NP + D : 0); e += nt) {
    if (e < D * NP) {
      const int cmp = e / NP, i = e % NP;
      const double* Xc = sh.X + cmp * NV * NPX;
      double s = 0;
      for (int k = mc; k < NV; ++k) s += y[k * NPX] * Xc[k * NPX + i];
      sh.w[cmp][i] = s;
    } else if (e < D * NP + NP) {
      const int i = e - D * NP;
      double s = 0;
      for (int cmp = 0; cmp < D; ++cmp) {
        const double* Xc = sh.X + cmp * NV * NPX;
        for (int k = 0; k < NV; ++k) s += Xc[k * NPX + i] * Xc[k * NPX + NP];
      }
      sh.t[i] -= s;
    } else {
      const int cmp = e - D * NP - NP;
      const double* Xc = sh.X + cmp * NV * NPX;
      double s = 0;
      for (int k = mc; k < NV; ++k) s += y[k * NPX] * Xc[k * NPX + NP];
      sh.qg[cmp] = s;
    }
  }
  __syncthreads();
}

// Dense Cholesky of F = -S (lower factor in sh.S).
template <int D, class LDS>
__device__ void schur_cholesky(LDS& sh) {
  constexpr int NP = PT<D>::NP;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < NP * NP; e += nt) sh.S[e] = -sh.S[e];
  __syncthreads();
  for (int k = 0; k < NP; ++k) {
    const double dkk = sh.S[k * NP + k];
    if (tid == 0 && !(dkk > 0.0)) sh.bad = 1;
    const double l = sqrt(dkk);
    __syncthreads();
    for (int i = k + 1 + tid; i < NP; i += nt) sh.S[i * NP + k] /= l;
    if (tid == 0) sh.S[k * NP + k] = l;
    __syncthreads();
    const int m = NP - 1 - k;
    for (int p = tid; p < m * m; p += nt) {
      const int ii = k + 1 + p / m, jj = k + 1 + p % m;
      if (jj <= ii) sh.S[ii * NP + jj] -= sh.S[ii * NP + k] * sh.S[jj * NP + k];
    }
    __syncthreads();
  }
}

// p = S^{-1} t = -F^{-1} t by forward/back substitution with the factor of F (first wavefront;
// each row's dot product is a wavefront reduction). Result overwrites sh.t.
template <int D, class LDS>
__device__ void schur_solve(LDS& sh) {
  constexpr int NP = PT<D>::NP;
  const int lane = threadIdx.x;
  if (lane < 64) {
    for (int i = 0; i < NP; ++i) {
      double s = lane < i ? sh.S[i * NP + lane] * sh.t[lane] : 0.0;
      s = wave_sum(s);
      if (lane == 0) sh.t[i] = (-sh.t[i] - s) / sh.S[i * NP + i];
    }
    for (int i = NP - 1; i >= 0; --i) {
      double s = (lane > i && lane < NP) ? sh.S[lane * NP + i] * sh.t[lane] : 0.0;
      s = wave_sum(s);
      if (lane == 0) sh.t[i] = (sh.t[i] - s) / sh.S[i * NP + i];
    }
  }
  __syncthreads();
}

// Place the stored sparse pattern values of a patch (cache_matrix) into the zeroed LDS blocks.
template <int D>
__device__ void patch_load_pattern(PatchLDS<D>& sh, const int* __restrict__ pattern, int npat,
                                   const double* __restrict__ vals) {
  constexpr int NV = PT<D>::NV, NP = PT<D>::NP, NB = PT<D>::NB, NPX = NP + 2;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < NV * NB; i += nt) sh.Kb[i] = 0;
  for (int i = tid; i < D * NV * NPX; i += nt) sh.X[i] = 0;
  for (int i = tid; i < NP * NP; i += nt) sh.S[i] = 0;
  __syncthreads();
  for (int e = tid; e < npat; e += nt) {
    const int code = pattern[e];
    const int type = code >> 24, i = (code >> 12) & 0xfff, j = code & 0xfff;
    const double v = vals[e];
    if (type == 0) {
      sh.Kb[i * NB + (i - j)] = v;
    } else if (type <= D) {
      sh.X[((type - 1) * NV + i) * NPX + j] = v;
    } else {
      sh.S[i * NP + j] = v;
      sh.S[j * NP + i] = v;
    }
  }
  __syncthreads();
}

}  // namespace

// Sparse pattern of L_i kept by cache_matrix: lower band entries of K between window nodes at
// max-norm distance <= 1, all structural entries of the d blocks B_c, lower triangle of C.
template <int D>
void pattern_entries(std::vector<int>& enc) {
  enc.clear();
  constexpr int NV = PT<D>::NV, NP = PT<D>::NP;
  auto vco = [](int v, int* o) {
    o[0] = v % 5;
    o[1] = (v / 5) % 5;
    o[2] = D == 3 ? v / 25 : 0;
  };
  auto qco = [](int q, int* o) {
    o[0] = q % 3 + 1;
    o[1] = (q / 3) % 3 + 1;
    o[2] = D == 3 ? q / 9 + 1 : 0;
  };
  auto near = [](const int* a, const int* b) {
    for (int k = 0; k < D; ++k)
      if (a[k] - b[k] > 1 || b[k] - a[k] > 1) return false;
    return true;
  };
  for (int i = 0; i < NV; ++i)
    for (int j = 0; j <= i; ++j) {
      int a[3], b[3];
      vco(i, a);
      vco(j, b);
      if (near(a, b)) enc.push_back((0 << 24) | (i << 12) | j);
    }
  for (int c = 0; c < D; ++c)
    for (int i = 0; i < NV; ++i)
      for (int q = 0; q < NP; ++q) {
        int a[3], b[3];
        vco(i, a);
        qco(q, b);
        if (near(a, b)) enc.push_back(((1 + c) << 24) | (i << 12) | q);
      }
  for (int i = 0; i < NP; ++i)
    for (int j = 0; j <= i; ++j) {
      int a[3], b[3];
      qco(i, a);
      qco(j, b);
      if (near(a, b)) enc.push_back(((D + 1) << 24) | (i << 12) | j);
    }
}

// Entries of one type (0: K, 1..3: B_c, 4: C) in the 3D pattern.
int pattern_count3(int type) {
  std::vector<int> e;
  pattern_entries<3>(e);
  int n = 0;
  for (int code : e) n += (code >> 24) == type ? 1 : 0;
  return n;
}

template <int D>
int pattern_size() {
  std::vector<int> e;
  pattern_entries<D>(e);
  return (int)e.size();
}

// ================================================================================================
// cache_inverse set-up (Sec. 3.1.2): the d+1 rows of L_i^{-1} that the restricted prolongation
// keeps (velocity components and pressure of the centre node), written as (d+1) x ZSP rows in the
// patch column layout. One block per patch.
// ================================================================================================
template <int D>
__global__ void __launch_bounds__(PT<D>::THREADS) patch_inverse_rows_kernel(
    const OpConsts* __restrict__ oc, const int* __restrict__ cell_info, const double* __restrict__ cut, Geom g,
    double eta, const int* __restrict__ nodes, int64_t count, double* __restrict__ Z, int* err) {
  constexpr int NV = PT<D>::NV, NP = PT<D>::NP, NPX = NP + 2, ZS = PT<D>::ZS, ZSP = PT<D>::ZSP;
  __shared__ PatchLDS<D> sh;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = oc->n;
  const int ip = pres_center<D>(), mc = vel_center<D>();
  for (int64_t pi = blockIdx.x; pi < count; pi += gridDim.x) {
    const int64_t node = nodes[pi];
    int c[3];
    node_coords<D>(node, n, c);
    if (tid == 0) sh.bad = 0;
    patch_assemble<D>(sh, oc, cell_info, cut, g, eta, c, 0);
    patch_pad<D>(sh, c, n);
    if (tid < NV) sh.X[tid * NPX + NP + 1] = tid == mc ? 1.0 : 0.0;  // e_m column (component 0)
    band_cholesky<D>(sh);
    // forward: columns 0..NP-1 of every component and the e_m column of component 0
    for (int t = tid; t < D * NP + 1; t += nt) {
      const int cmp = t < D * NP ? t / NP : 0;
      const int col = t < D * NP ? t % NP : NP + 1;
      double* Xc = sh.X + cmp * NV * NPX + col;
      constexpr int NB = PT<D>::NB, BW = PT<D>::BW;
      for (int i = 0; i < NV; ++i) {
        double v = Xc[i * NPX];
        const int k0 = i - BW > 0 ? i - BW : 0;
        for (int k = k0; k < i; ++k) v -= sh.Kb[i * NB + (i - k)] * Xc[k * NPX];
        Xc[i * NPX] = v / sh.Kb[i * NB];
      }
    }
    __syncthreads();
    schur_update<D>(sh, false);
    schur_cholesky<D>(sh);
    // S^{-1} = -F^{-1}, column j by forward/back substitution (thread per column)
    for (int j = tid; j < NP; j += nt) {
      double u[NP];
      for (int i = 0; i < NP; ++i) {
        double s = i == j ? 1.0 : 0.0;
        for (int k = 0; k < i; ++k) s -= sh.S[i * NP + k] * u[k];
        u[i] = s / sh.S[i * NP + i];
      }
      for (int i = NP - 1; i >= 0; --i) {
        double s = u[i];
        for (int k = i + 1; k < NP; ++k) s -= sh.S[k * NP + i] * u[k];
        u[i] = s / sh.S[i * NP + i];
      }
      for (int i = 0; i < NP; ++i) sh.Sinv[i * NP + j] = -u[i];
    }
    __syncthreads();
    band_backward<D>(sh, NP);  // W_c = K^{-1} B_c, q = K^{-1} e_m
    for (int e = tid; e < D * NP; e += nt) {
      const int cmp = e / NP, j = e % NP;
      double s = 0;
      for (int i = 0; i < NP; ++i) s += sh.Sinv[j * NP + i] * sh.w[cmp][i];
      sh.tc[cmp][j] = s;
    }
    __syncthreads();
    double* Zp = Z + pi * (int64_t)(D + 1) * ZSP;
    for (int e = tid; e < (D + 1) * ZSP; e += nt) {
      const int f = e / ZSP, col = e % ZSP;
      double val = 0;
      if (col < D * NV) {
        const int cp = col / NV, k = col % NV;
        if (vel_in_grid<D>(c, n, k)) {
          const double* Wr = sh.X + (cp * NV + k) * NPX;
          double s = 0;
          if (f < D) {
            for (int j = 0; j < NP; ++j) s += Wr[j] * sh.tc[f][j];
            if (f == cp) s += sh.X[k * NPX + NP + 1];
          } else {
            for (int j = 0; j < NP; ++j) s -= Wr[j] * sh.Sinv[j * NP + ip];
          }
          val = s;
        }
      } else if (col < ZS) {
        const int j = col - D * NV;
        if (pres_in_grid<D>(c, n, j)) val = f < D ? -sh.tc[f][j] : sh.Sinv[ip * NP + j];
      }
      Zp[e] = val;
    }
    if (tid == 0 && sh.bad) atomicMin(err, (int)node);
    __syncthreads();
  }
}

// Dense LU of a 2D patch block (immersed boundary terms). Symmetric Nitsche is not coercive on cells
// with a small physical part, so the velocity block of a cut-band patch may be indefinite and the
// block Cholesky above does not apply. The whole block L_i (59 x 59: u_x, u_y, p over the window,
// decoupled positions outside the grid) is factorised by LU with partial pivoting (largest
// magnitude, lowest row on ties; Sec. 3.1.2 names LU). One wavefront per patch, the block in LDS.
constexpr int kLU2 = PT<2>::ZS;

// A (row-major) = I_2 (x) K_i (from the lower band), B_c and B_c^T, C_i of the assembled patch.
__device__ void patch_dense2(const PatchLDS<2>& sh, double* A) {
  constexpr int NV = PT<2>::NV, NP = PT<2>::NP, NB = PT<2>::NB, NPX = NP + 2, ZS = kLU2;
  for (int e = threadIdx.x; e < ZS * ZS; e += 64) {
    const int i = e / ZS, j = e % ZS;
    double v = 0;
    if (i < 2 * NV && j < 2 * NV) {
      const int vi = i % NV, vj = j % NV;
      if (i / NV == j / NV) {
        const int hi = vi > vj ? vi : vj, lo = vi > vj ? vj : vi;
        if (hi - lo < NB) v = sh.Kb[hi * NB + (hi - lo)];
      }
    } else if (i < 2 * NV) {
      v = sh.X[((i / NV) * NV + i % NV) * NPX + (j - 2 * NV)];
    } else if (j < 2 * NV) {
      v = sh.X[((j / NV) * NV + j % NV) * NPX + (i - 2 * NV)];
    } else {
      v = sh.S[(i - 2 * NV) * NP + (j - 2 * NV)];
    }
    A[e] = v;
  }
  __syncthreads();
}

// P A = L U in place (unit L below the diagonal, U on and above), row swaps in piv; returns true
// when a pivot column is zero (singular block). Wavefront-uniform.
__device__ bool lu_factor2(double* A, int* piv) {
  constexpr int ZS = kLU2;
  const int tid = threadIdx.x;
  bool bad = false;
  for (int k = 0; k < ZS; ++k) {
    // pivot row: largest |A[i][k]|, i >= k, lowest index on ties (a butterfly over the wavefront)
    const int i0 = k + tid;
    double pv = i0 < ZS ? fabs(A[i0 * ZS + k]) : -1.0;
    int pr = i0 < ZS ? i0 : ZS;
    for (int m = 32; m >= 1; m >>= 1) {
      const double ov = __shfl_xor(pv, m, 64);
      const int orow = __shfl_xor(pr, m, 64);
      if (ov > pv || (ov == pv && orow < pr)) {
        pv = ov;
        pr = orow;
      }
    }
    if (tid == 0) piv[k] = pr;
    if (!(pv > 0)) bad = true;
    if (pr != k)
      for (int j = tid; j < ZS; j += 64) {
        const double t = A[k * ZS + j];
        A[k * ZS + j] = A[pr * ZS + j];
        A[pr * ZS + j] = t;
      }
    __syncthreads();
    if (!bad) {
      const double inv = 1.0 / A[k * ZS + k];
      for (int i = k + 1 + tid; i < ZS; i += 64) A[i * ZS + k] *= inv;
      __syncthreads();
      const int w = ZS - k - 1;
      for (int e = tid; e < w * w; e += 64) {
        const int i = k + 1 + e / w, j = k + 1 + e % w;
        A[i * ZS + j] -= A[i * ZS + k] * A[k * ZS + j];
      }
    }
    __syncthreads();
  }
  return bad;
}

// z = row `row` of A^{-1}: A^T z = e_row, i.e. U^T w = e_row, L^T v = w, z = P^T v (one thread).
__device__ void lu_inverse_row2(const double* A, const int* piv, int row, double* z) {
  constexpr int ZS = kLU2;
  for (int i = 0; i < ZS; ++i) {
    double sum = i == row ? 1.0 : 0.0;
    for (int j = 0; j < i; ++j) sum -= A[j * ZS + i] * z[j];
    z[i] = sum / A[i * ZS + i];
  }
  for (int i = ZS - 1; i >= 0; --i) {
    double sum = z[i];
    for (int j = i + 1; j < ZS; ++j) sum -= A[j * ZS + i] * z[j];
    z[i] = sum;
  }
  for (int k = ZS - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k) {
      const double t = z[k];
      z[k] = z[p];
      z[p] = t;
    }
  }
}

// y = A^{-1} g in place (g <- P g, L u = g, U y = u with the factors of lu_factor2) by the whole
// (single) wavefront of the workgroup: lane i keeps entry i, and each solved entry is broadcast to
// the lanes below (forward: columns in ascending order) or above it (backward: descending order).
// Every lane calls it.
__device__ void lu_solve2_wave(const double* A, const int* piv, double* g) {
  constexpr int ZS = kLU2;
  static_assert(ZS <= 64, "one lane per row");
  const int lane = (int)(threadIdx.x & 63);
  if (lane == 0)
    for (int k = 0; k < ZS; ++k) {
      const int p = piv[k];
      if (p != k) {
        const double t = g[k];
        g[k] = g[p];
        g[p] = t;
      }
    }
  __syncthreads();
  double v = lane < ZS ? g[lane] : 0.0;
  for (int j = 0; j < ZS; ++j) {
    const double gj = __shfl(v, j);
    if (lane > j && lane < ZS) v -= A[lane * ZS + j] * gj;
  }
  for (int j = ZS - 1; j >= 0; --j) {
    if (lane == j) v = v / A[j * ZS + j];
    const double xj = __shfl(v, j);
    if (lane < j) v -= A[lane * ZS + j] * xj;
  }
  __syncthreads();
  if (lane < ZS) g[lane] = v;
}

// cache_inverse set-up with the immersed boundary terms (2D): the centre rows of L_i^{-1} from the
// dense LU by transposed solves.
__global__ void __launch_bounds__(64) patch_inverse_rows_lu2_kernel(
    const OpConsts* __restrict__ oc, const int* __restrict__ cell_info, const double* __restrict__ cut, Geom g,
    double eta, const int* __restrict__ nodes, int64_t count, double* __restrict__ Z, int* err) {
  constexpr int D = 2, NV = PT<2>::NV, ZS = kLU2, ZSP = PT<2>::ZSP;
  static_assert(PT<2>::THREADS == 64, "one wavefront per patch");
  __shared__ PatchLDS<2> sh;
  __shared__ double A[ZS * ZS];
  __shared__ double rhs[D + 1][ZS];
  __shared__ int piv[ZS];
  const int tid = threadIdx.x;
  const int n = oc->n;
  const int centre[D + 1] = {vel_center<2>(), NV + vel_center<2>(), D * NV + pres_center<2>()};
  for (int64_t pi = blockIdx.x; pi < count; pi += gridDim.x) {
    const int64_t node = nodes[pi];
    int c[3];
    node_coords<D>(node, n, c);
    patch_assemble<D>(sh, oc, cell_info, cut, g, eta, c, 0);
    patch_pad<D>(sh, c, n);
    patch_dense2(sh, A);
    const bool bad = lu_factor2(A, piv);
    if (tid <= D && !bad) lu_inverse_row2(A, piv, centre[tid], rhs[tid]);
    __syncthreads();
    double* Zp = Z + pi * (int64_t)(D + 1) * ZSP;
    for (int e = tid; e < (D + 1) * ZSP; e += 64) {
      const int f = e / ZSP, col = e % ZSP;
      double val = 0;
      if (!bad && col < ZS) {
        const bool in = col < D * NV ? vel_in_grid<D>(c, n, col % NV) : pres_in_grid<D>(c, n, col - D * NV);
        if (in) val = rhs[f][col];
      }
      Zp[e] = val;
    }
    if (tid == 0 && bad) atomicMin(err, (int)node);
    __syncthreads();
  }
}

// Dense LU of a 3D patch block (immersed boundary terms; see the 2D form above): the whole block
// (402 x 402: u_x, u_y, u_z, p over the window) does not fit LDS, so each workgroup factorises it in
// its own slot of a device buffer, row operations spread over the lanes, then takes the d+1 centre
// rows of the inverse by transposed solves with the d+1 right-hand sides in LDS. Set-up only.
constexpr int kLU3 = PT<3>::ZS;
constexpr int64_t kLU3Slot = (int64_t)kLU3 * kLU3;  // doubles of one workgroup's slot
constexpr int kLU3Blocks = 512;                      // workgroups (slots) of one launch

struct LU3LDS {
  double z[4][kLU3];  // the four right-hand sides, then the inverse rows
  int piv[kLU3];
  double red_v[4];
  int red_i[4];
  int pk;
  int bad;
};

// A (row-major, device memory) = I_3 (x) K_i (from the lower band), B_c and B_c^T, C_i.
__device__ void patch_dense3(const PatchLDS<3>& sh, double* __restrict__ A) {
  constexpr int NV = PT<3>::NV, NP = PT<3>::NP, NB = PT<3>::NB, NPX = NP + 2, ZS = kLU3;
  for (int i = threadIdx.x >> 6; i < ZS; i += blockDim.x >> 6)
    for (int j = threadIdx.x & 63; j < ZS; j += 64) {
      double v = 0;
      if (i < 3 * NV && j < 3 * NV) {
        const int vi = i % NV, vj = j % NV;
        if (i / NV == j / NV) {
          const int hi = vi > vj ? vi : vj, lo = vi > vj ? vj : vi;
          if (hi - lo < NB) v = sh.Kb[hi * NB + (hi - lo)];
        }
      } else if (i < 3 * NV) {
        v = sh.X[((i / NV) * NV + i % NV) * NPX + (j - 3 * NV)];
      } else if (j < 3 * NV) {
        v = sh.X[((j / NV) * NV + j % NV) * NPX + (i - 3 * NV)];
      } else {
        v = sh.S[(i - 3 * NV) * NP + (j - 3 * NV)];
      }
      A[(int64_t)i * ZS + j] = v;
    }
  __syncthreads();
}

// P A = L U in place (unit L below the diagonal, U on and above), the row interchanges in lu.piv;
// pivot: largest |A[i][k]|, lowest row on ties. lu.bad is set when a pivot column is zero.
// Right-looking in panels of kLU3Panel columns: within a panel each column is pivoted, its rows
// swapped in full, scaled and applied to the rest of the panel; then the panel's block row of U is
// formed and the trailing block updated once by the panel's rank-kLU3Panel product, so the trailing
// block streams through memory once per panel instead of once per column.
constexpr int kLU3Panel = 16;

__device__ void lu_factor3(double* __restrict__ A, LU3LDS& lu) {
  constexpr int ZS = kLU3, NBP = kLU3Panel;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6, nt = blockDim.x;
  if (tid == 0) lu.bad = 0;
  __syncthreads();
  for (int k0 = 0; k0 < ZS; k0 += NBP) {
    const int ke = k0 + NBP < ZS ? k0 + NBP : ZS;
    for (int k = k0; k < ke; ++k) {
      double pv = -1.0;
      int pr = ZS;
      for (int i = k + tid; i < ZS; i += nt) {
        const double v = fabs(A[(int64_t)i * ZS + k]);
        if (v > pv) {  // rows ascend per thread: the first of equal values is kept
          pv = v;
          pr = i;
        }
      }
      for (int msk = 32; msk >= 1; msk >>= 1) {
        const double ov = __shfl_xor(pv, msk, 64);
        const int orow = __shfl_xor(pr, msk, 64);
        if (ov > pv || (ov == pv && orow < pr)) {
          pv = ov;
          pr = orow;
        }
      }
      if (lane == 0) {
        lu.red_v[wave] = pv;
        lu.red_i[wave] = pr;
      }
      __syncthreads();
      if (tid == 0) {
        double bv = lu.red_v[0];
        int br = lu.red_i[0];
        for (int w = 1; w < nw; ++w)
          if (lu.red_v[w] > bv || (lu.red_v[w] == bv && lu.red_i[w] < br)) {
            bv = lu.red_v[w];
            br = lu.red_i[w];
          }
        lu.pk = br;
        lu.piv[k] = br;
        if (!(bv > 0)) lu.bad = 1;
      }
      __syncthreads();
      if (lu.bad) return;
      const int p = lu.pk;
      if (p != k)
        for (int j = tid; j < ZS; j += nt) {
          const double t = A[(int64_t)k * ZS + j];
          A[(int64_t)k * ZS + j] = A[(int64_t)p * ZS + j];
          A[(int64_t)p * ZS + j] = t;
        }
      __syncthreads();
      const double inv = 1.0 / A[(int64_t)k * ZS + k];
      for (int i = k + 1 + tid; i < ZS; i += nt) A[(int64_t)i * ZS + k] *= inv;
      __syncthreads();
      // the rest of the panel: columns k+1 .. ke-1
      const int w = ke - k - 1;
      if (w > 0) {
        for (int e = tid; e < (ZS - k - 1) * w; e += nt) {
          const int i = k + 1 + e / w, jj = k + 1 + e % w;
          A[(int64_t)i * ZS + jj] -= A[(int64_t)i * ZS + k] * A[(int64_t)k * ZS + jj];
        }
        __syncthreads();
      }
    }
    if (ke == ZS) break;
    // block row of U: rows k0+1 .. ke-1, columns ke .. ZS-1, by the unit lower panel triangle (each
    // thread one column, rows in order)
    for (int j = ke + tid; j < ZS; j += nt)
      for (int i = k0 + 1; i < ke; ++i) {
        double s = A[(int64_t)i * ZS + j];
        for (int t = k0; t < i; ++t) s -= A[(int64_t)i * ZS + t] * A[(int64_t)t * ZS + j];
        A[(int64_t)i * ZS + j] = s;
      }
    __syncthreads();
    // trailing block: A[i][j] -= sum over the panel's columns t of L[i][t] U[t][j]
    for (int i = ke + wave; i < ZS; i += nw)
      for (int j = ke + lane; j < ZS; j += 64) {
        double s = A[(int64_t)i * ZS + j];
        for (int t = k0; t < ke; ++t) s -= A[(int64_t)i * ZS + t] * A[(int64_t)t * ZS + j];
        A[(int64_t)i * ZS + j] = s;
      }
    __syncthreads();
  }
}

// lu.z[r] <- row rows[r] of A^{-1} for r < 4: A^T z = e_row, i.e. U^T w = e_row, L^T v = w,
// z = P^T v, all four at once; thread (r, j) updates entry j of right-hand side r after each step.
__device__ void lu_inverse_rows3(const double* __restrict__ A, LU3LDS& lu, const int* rows) {
  constexpr int ZS = kLU3;
  const int tid = threadIdx.x;
  for (int e = tid; e < 4 * ZS; e += blockDim.x) lu.z[e / ZS][e % ZS] = (e % ZS) == rows[e / ZS] ? 1.0 : 0.0;
  __syncthreads();
  // U^T w = e: w_i = z_i / U_ii, then z_j -= U_ij w_i for j > i
  for (int i = 0; i < ZS; ++i) {
    const double uii = A[(int64_t)i * ZS + i];
    for (int e = tid; e < 4 * (ZS - i); e += blockDim.x) {
      const int r = e / (ZS - i), j = i + e % (ZS - i);
      const double wi = lu.z[r][i] / uii;
      if (j > i) lu.z[r][j] -= A[(int64_t)i * ZS + j] * wi;
    }
    __syncthreads();
    if (tid < 4) lu.z[tid][i] /= uii;
    __syncthreads();
  }
  // L^T v = w (unit diagonal): v_i = z_i, then z_j -= L_ij v_i for j < i
  for (int i = ZS - 1; i > 0; --i) {
    for (int e = tid; e < 4 * i; e += blockDim.x) {
      const int r = e / i, j = e % i;
      lu.z[r][j] -= A[(int64_t)i * ZS + j] * lu.z[r][i];
    }
    __syncthreads();
  }
  // z = P^T v: the interchanges undone in reverse order
  if (tid < 4)
    for (int k = ZS - 1; k >= 0; --k) {
      const int p = lu.piv[k];
      if (p != k) {
        const double t = lu.z[tid][k];
        lu.z[tid][k] = lu.z[tid][p];
        lu.z[tid][p] = t;
      }
    }
  __syncthreads();
}

__global__ void __launch_bounds__(256) patch_inverse_rows_lu3_kernel(
    const OpConsts* __restrict__ oc, const int* __restrict__ cell_info, const double* __restrict__ cut, Geom g,
    double eta, const int* __restrict__ nodes, int64_t count, double* __restrict__ Z, double* __restrict__ slots,
    int* err) {
  constexpr int D = 3, NV = PT<3>::NV, ZS = kLU3, ZSP = PT<3>::ZSP;
  __shared__ PatchLDS<3> sh;
  __shared__ LU3LDS lu;
  const int tid = threadIdx.x;
  const int n = oc->n;
  const int centre[D + 1] = {vel_center<3>(), NV + vel_center<3>(), 2 * NV + vel_center<3>(),
                             D * NV + pres_center<3>()};
  double* A = slots + (int64_t)blockIdx.x * kLU3Slot;
  for (int64_t pi = blockIdx.x; pi < count; pi += gridDim.x) {
    const int64_t node = nodes[pi];
    int c[3];
    node_coords<D>(node, n, c);
    patch_assemble<D>(sh, oc, cell_info, cut, g, eta, c, 0);
    patch_pad<D>(sh, c, n);
    patch_dense3(sh, A);
    lu_factor3(A, lu);
    const bool bad = lu.bad != 0;
    if (!bad) lu_inverse_rows3(A, lu, centre);
    double* Zp = Z + pi * (int64_t)(D + 1) * ZSP;
    for (int e = tid; e < (D + 1) * ZSP; e += blockDim.x) {
      const int f = e / ZSP, col = e % ZSP;
      double val = 0;
      if (!bad && col < ZS) {
        const bool in = col < D * NV ? vel_in_grid<D>(c, n, col % NV) : pres_in_grid<D>(c, n, col - D * NV);
        if (in) val = lu.z[f][col];
      }
      Zp[e] = val;
    }
    if (tid == 0 && bad) atomicMin(err, (int)node);
    __syncthreads();
  }
}

template <int D>
hipError_t k_patch_inverse_rows(const Ctx& c, const Level& L, const int* nodes, int64_t count, double* Z,
                                hipStream_t s) {
  if (count == 0) return hipSuccess;
  if constexpr (D == 3) {
    if (L.dense_lu) {
      const int64_t nb = count < kLU3Blocks ? count : kLU3Blocks;
      double* slots = nullptr;
      hipError_t e = hipMallocAsync((void**)&slots, (size_t)nb * kLU3Slot * sizeof(double), s);
      if (e != hipSuccess) return e;
      patch_inverse_rows_lu3_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(
          L.consts, L.cell_info, L.cut_mats, c.geom(L), c.prm.eta, nodes, count, Z, slots, c.err);
      e = hipGetLastError();
      const hipError_t f = hipFreeAsync(slots, s);
      return e != hipSuccess ? e : f;
    }
  }
  if constexpr (D == 2) {
    if (L.dense_lu) {
      const int64_t nb = count < 262144 ? count : 262144;
      patch_inverse_rows_lu2_kernel<<<dim3((unsigned)nb), dim3(64), 0, s>>>(
          L.consts, L.cell_info, L.cut_mats, c.geom(L), c.prm.eta, nodes, count, Z, c.err);
      return hipGetLastError();
    }
  }
  const int64_t nb = count < 262144 ? count : 262144;
  patch_inverse_rows_kernel<D><<<dim3((unsigned)nb), dim3(PT<D>::THREADS), 0, s>>>(
      L.consts, L.cell_info, L.cut_mats, c.geom(L), c.prm.eta, nodes, count, Z, c.err);
  return hipGetLastError();
}

// ================================================================================================
// cache_matrix set-up: store the sparse pattern values of L_i (Sec. 3.1.2, "stored using a sparse
// format"). One block per patch.
// ================================================================================================
template <int D>
__global__ void __launch_bounds__(PT<D>::THREADS) store_matrices_kernel(
    const OpConsts* __restrict__ oc, const int* __restrict__ cell_info, const double* __restrict__ cut, Geom g,
    double eta, const int* __restrict__ nodes, int64_t count, const int* __restrict__ pattern, int npat,
    double* __restrict__ M) {
  constexpr int NV = PT<D>::NV, NP = PT<D>::NP, NB = PT<D>::NB, NPX = NP + 2;
  __shared__ PatchLDS<D> sh;
  for (int64_t pi = blockIdx.x; pi < count; pi += gridDim.x) {
    int c[3];
    node_coords<D>(nodes[pi], oc->n, c);
    patch_assemble<D>(sh, oc, cell_info, cut, g, eta, c, 0);
    for (int e = threadIdx.x; e < npat; e += blockDim.x) {
      const int code = pattern[e];
      const int type = code >> 24, i = (code >> 12) & 0xfff, j = code & 0xfff;
      double v;
      if (type == 0)
        v = sh.Kb[i * NB + (i - j)];
      else if (type <= D)
        v = sh.X[((type - 1) * NV + i) * NPX + j];
      else
        v = sh.S[i * NP + j];
      M[pi * npat + e] = v;
    }
    __syncthreads();
  }
}

template <int D>
hipError_t k_store_matrices(const Ctx& c, const Level& L, const int* nodes, int64_t count, double* M, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const int64_t nb = count < 262144 ? count : 262144;
  store_matrices_kernel<D><<<dim3((unsigned)nb), dim3(PT<D>::THREADS), 0, s>>>(
      L.consts, L.cell_info, L.cut_mats, c.geom(L), c.prm.eta, nodes, count, c.pattern, c.n_pattern, M);
  return hipGetLastError();
}

// L_i = R_i L R_i^T (Eq. 15) of the 3D patch centred at node c, retrieved from the rows of L that the
// residual applies (cache_none): the block's threads take the velocity nodes of the 5^3 window in
// turn; each reads its node's operator code and row (the level's reference stencil of its kind, or
// its stored stencil) and writes the entries whose column lies in the patch: its row of the lower
// band of K, of B_x, B_y, B_z (columns of the 3^3 pressure window) and, for the 27 inner nodes, its
// pressure row of C. Every entry is written once, by the thread of its row.
__device__ void patch_retrieve3(PatchLDS<3>& sh, const OpConsts* __restrict__ oc, const int* __restrict__ node_op,
                                const double* __restrict__ nsten, const int* c) {
  constexpr int NV = PT<3>::NV, NP = PT<3>::NP, NB = PT<3>::NB, NPX = NP + 2, NS = PT<3>::NST;
  using RL = RefLayout<3>;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = oc->n;
  for (int i = tid; i < NV * NB; i += nt) sh.Kb[i] = 0;
  for (int i = tid; i < 3 * NV * NPX; i += nt) sh.X[i] = 0;
  for (int i = tid; i < NP * NP; i += nt) sh.S[i] = 0;
  __syncthreads();
  for (int row = tid; row < NV; row += nt) {
    const int v[3] = {row % 5, (row / 5) % 5, row / 25};
    const int g0[3] = {c[0] + v[0] - 2, c[1] + v[1] - 2, c[2] + v[2] - 2};
    bool in = true;
    for (int k = 0; k < 3; ++k) in = in && g0[k] >= 0 && g0[k] <= n;
    if (in) {
      const int op = node_op[node_index<3>(g0, n)];
      const bool inner = v[0] >= 1 && v[0] <= 3 && v[1] >= 1 && v[1] <= 3 && v[2] >= 1 && v[2] <= 3;
      const int qa = (v[0] - 1) + 3 * (v[1] - 1) + 9 * (v[2] - 1);
      const double* __restrict__ st = op >= 0 ? nsten + (int64_t)op * PT<3>::NSTEN : nullptr;
      const double* __restrict__ pk = oc->pack;
      const int ku = op >= 0 ? 0 : -op - 1;
      // coefficient j of offset o: 0 K, 1..3 B_x, B_y, B_z, 7 C (the layout of the stored stencils)
      auto coef = [&](int j, int o) -> double {
        if (st) return st[sten_index<3>(j, o)];
        if (j == 0) return pk[RL::oSK + ku * NS + o];
        if (j <= 3) return pk[RL::oSB + (ku * 3 + j - 1) * NS + o];
        return pk[RL::oSC + o];
      };
      for (int o = 0; o < NS; ++o) {
        const int oo[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
        bool ok = true, inwin = true, inpres = true;
        int xb[3];
        for (int k = 0; k < 3; ++k) {
          const int gk = g0[k] + oo[k];
          ok = ok && gk >= 0 && gk <= n;
          xb[k] = v[k] + oo[k];
          inwin = inwin && xb[k] >= 0 && xb[k] <= 4;
          inpres = inpres && xb[k] >= 1 && xb[k] <= 3;
        }
        if (!ok) continue;
        if (inwin) {
          const int vb = xb[0] + 5 * xb[1] + 25 * xb[2];
          if (vb <= row) sh.Kb[row * NB + (row - vb)] = coef(0, o);
        }
        if (inpres) {
          const int qb = (xb[0] - 1) + 3 * (xb[1] - 1) + 9 * (xb[2] - 1);
          for (int cmp = 0; cmp < 3; ++cmp) sh.X[(cmp * NV + row) * NPX + qb] = coef(1 + cmp, o);
          if (inner) sh.S[qa * NP + qb] = coef(7, o);
        }
      }
    }
  }
  __syncthreads();
}

// ================================================================================================
// cache_matrix / cache_none application: for every node i, retrieve L_i (stored values, or the
// operator rows), factorise,
// solve L_i y = R_i r and add omega * (kept entries of y) to x (Eq. 14-15). One block per patch.
// x == nullptr: factorise only and report singular blocks (set-up validation).
// ================================================================================================
template <int D>
__global__ void __launch_bounds__(PT<D>::THREADS) patch_solve_kernel(
    const OpConsts* __restrict__ oc, const int* __restrict__ cell_info, const double* __restrict__ cut, Geom g,
    double eta, int policy, const int* __restrict__ node_class, const double* __restrict__ Mcls,
    const double* __restrict__ Mirr, const int* __restrict__ pattern, int npat, int64_t N,
    const double* __restrict__ r, double* __restrict__ x, double omega, int* err, const int* __restrict__ node_op,
    const double* __restrict__ nsten, bool integrate) {
  constexpr int NV = PT<D>::NV, NP = PT<D>::NP, NPX = NP + 2;
  __shared__ PatchLDS<D> sh;
  const int tid = threadIdx.x;
  const int n = oc->n;
  const int mc = vel_center<D>(), ip = pres_center<D>();
  for (int64_t node = blockIdx.x; node < N; node += gridDim.x) {
    int c[3];
    node_coords<D>(node, n, c);
    if (tid == 0) sh.bad = 0;
    if (policy == FCGMG_CACHE_MATRIX) {
      const int cls = node_class[node];
      const double* vals = cls >= 0 ? Mcls + (int64_t)cls * npat : Mirr + (int64_t)(-cls - 1) * npat;
      patch_load_pattern<D>(sh, pattern, npat, vals);
    } else if (D == 3 && !integrate) {
      if constexpr (D == 3) patch_retrieve3(sh, oc, node_op, nsten, c);
    } else {
      patch_assemble<D>(sh, oc, cell_info, cut, g, eta, c, 1);
    }
    patch_pad<D>(sh, c, n);
    // right-hand side g = R_i r (zero outside the grid) and the e_m column
    for (int e = tid; e < D * NV + NP; e += blockDim.x) {
      if (e < D * NV) {
        const int cmp = e / NV, v = e % NV;
        double val = 0;
        if (vel_in_grid<D>(c, n, v)) {
          int cc[3] = {c[0] + v % 5 - 2, c[1] + (v / 5) % 5 - 2, D == 3 ? c[2] + v / 25 - 2 : 0};
          val = r ? r[cmp * N + node_index<D>(cc, n)] : 0.0;
        }
        sh.X[(cmp * NV + v) * NPX + NP] = val;
        if (cmp == 0) sh.X[v * NPX + NP + 1] = v == mc ? 1.0 : 0.0;
      } else {
        const int q = e - D * NV;
        double val = 0;
        if (pres_in_grid<D>(c, n, q)) {
          int cc[3] = {c[0] + q % 3 - 1, c[1] + (q / 3) % 3 - 1, D == 3 ? c[2] + q / 9 - 1 : 0};
          val = r ? r[D * N + node_index<D>(cc, n)] : 0.0;
        }
        sh.t[q] = val;
      }
    }
    __syncthreads();
    band_cholesky<D>(sh);
    band_forward<D>(sh, NPX);
    schur_update<D>(sh, true);
    schur_cholesky<D>(sh);
    schur_solve<D>(sh);
    if (x != nullptr && tid <= D) {
      double y;
      if (tid < D) {
        double s = sh.qg[tid];
        for (int j = 0; j < NP; ++j) s -= sh.w[tid][j] * sh.t[j];
        y = s;
      } else {
        y = sh.t[ip];
      }
      x[tid * N + node] += omega * y;
    }
    if (tid == 0 && sh.bad) atomicMin(err, (int)node);
    __syncthreads();
  }
}

// ---- 3D factorising policies, one velocity component's columns at a time -----------------------
// The velocity block of L_i is I_3 (x) K, so the forward substitutions of the three components'
// coupling columns share the factor of K and are independent: each component's 27 columns B_c and
// its right-hand side g_c are loaded, substituted and folded into the Schur complement in turn. The
// block then needs LDS for K's band, one component's columns and S (about 68 KB instead of 134 KB),
// so two patches run on a CU at once.
struct Patch3LDS {
  static constexpr int NV = 125, NP = 27, NB = PT<3>::NB, NX = NP + 2;  // columns: B_c, g_c, e_m
  double Kb[NV * NB];  // lower band of K, then its Cholesky factor
  double X[NV * NX];   // [B_c | g_c | e_m] of one component, then L^{-1} of it
  double y[NV];        // L^{-1} e_m (row m of K^{-1} after the back substitution implied by y^T V)
  double rd[NV];       // 1 / L_ii
  double S[NP * NP];   // C - sum_c V_c^T V_c, then the Cholesky factor of -S
  double t[NP];        // pressure right-hand side, then the pressures
  double w[3][NP];     // y^T V_c
  double qg[3];        // y^T z_c
  int bad;
};

// Entries of L_i for one pass: pass < 0 takes K (lower band) and C; pass c the columns B_c. From the
// stored pattern values (cache_matrix) or from the operator rows of the window's velocity nodes
// (cache_none). The buffers of the pass were zeroed before.
__device__ void patch3_load(Patch3LDS& sh, int pass, bool rows, const OpConsts* __restrict__ oc,
                            const int* __restrict__ node_op, const double* __restrict__ nsten,
                            const int* __restrict__ pattern, int npat, int nk, int nbc,
                            const double* __restrict__ vals, const int* c) {
  constexpr int NV = Patch3LDS::NV, NP = Patch3LDS::NP, NB = Patch3LDS::NB, NX = Patch3LDS::NX, NS = PT<3>::NST;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (!rows) {
    // the pattern lists K (nk entries), then B_x, B_y, B_z (nbc each), then C: a pass reads its parts
    const int lo0 = pass < 0 ? 0 : nk + pass * nbc, hi0 = pass < 0 ? nk : lo0 + nbc;
    const int lo1 = pass < 0 ? nk + 3 * nbc : 0, hi1 = pass < 0 ? npat : 0;
    const int cnt0 = hi0 - lo0;
    for (int t = tid; t < cnt0 + (hi1 - lo1); t += nt) {
      const int e = t < cnt0 ? lo0 + t : lo1 + (t - cnt0);
      const int code = pattern[e];
      const int type = code >> 24, i = (code >> 12) & 0xfff, j = code & 0xfff;
      if (type == 0) {
        sh.Kb[i * NB + (i - j)] = vals[e];
      } else if (type > 3) {
        sh.S[i * NP + j] = vals[e];
        sh.S[j * NP + i] = vals[e];
      } else {
        sh.X[i * NX + j] = vals[e];
      }
    }
    return;
  }
  using RL = RefLayout<3>;
  const int n = oc->n;
  const double* __restrict__ pk = oc->pack;
  for (int row = tid; row < NV; row += nt) {
    const int v[3] = {row % 5, (row / 5) % 5, row / 25};
    const int g0[3] = {c[0] + v[0] - 2, c[1] + v[1] - 2, c[2] + v[2] - 2};
    bool in = true;
    for (int k = 0; k < 3; ++k) in = in && g0[k] >= 0 && g0[k] <= n;
    if (!in) continue;
    const int op = node_op[node_index<3>(g0, n)];
    const bool inner = v[0] >= 1 && v[0] <= 3 && v[1] >= 1 && v[1] <= 3 && v[2] >= 1 && v[2] <= 3;
    const int qa = (v[0] - 1) + 3 * (v[1] - 1) + 9 * (v[2] - 1);
    const double* __restrict__ st = op >= 0 ? nsten + (int64_t)op * PT<3>::NSTEN : nullptr;
    const int ku = op >= 0 ? 0 : -op - 1;
    // coefficient j of offset o: 0 K, 1..3 B_x, B_y, B_z, 7 C (the layout of the stored stencils)
    auto coef = [&](int j, int o) -> double {
      if (st) return st[sten_index<3>(j, o)];
      if (j == 0) return pk[RL::oSK + ku * NS + o];
      if (j <= 3) return pk[RL::oSB + (ku * 3 + j - 1) * NS + o];
      return pk[RL::oSC + o];
    };
    for (int o = 0; o < NS; ++o) {
      const int oo[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
      bool ok = true, inwin = true, inpres = true;
      int xb[3];
      for (int k = 0; k < 3; ++k) {
        const int gk = g0[k] + oo[k];
        ok = ok && gk >= 0 && gk <= n;
        xb[k] = v[k] + oo[k];
        inwin = inwin && xb[k] >= 0 && xb[k] <= 4;
        inpres = inpres && xb[k] >= 1 && xb[k] <= 3;
      }
      if (!ok) continue;
      if (pass < 0) {
        if (inwin) {
          const int vb = xb[0] + 5 * xb[1] + 25 * xb[2];
          if (vb <= row) sh.Kb[row * NB + (row - vb)] = coef(0, o);
        }
        if (inpres && inner) sh.S[qa * NP + (xb[0] - 1) + 3 * (xb[1] - 1) + 9 * (xb[2] - 1)] = coef(7, o);
      } else if (inpres) {
        sh.X[row * NX + (xb[0] - 1) + 3 * (xb[1] - 1) + 9 * (xb[2] - 1)] = coef(1 + pass, o);
      }
    }
  }
}

// Orders one wavefront's LDS accesses (they execute in order; this only keeps the compiler from
// moving them across).
__device__ __forceinline__ void patch3_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward substitution L V = X for the first ncol columns of the component buffer: a group of 8
// lanes of one wavefront per column, rows in blocks of 4. For a block starting at row i0, lane j of
// the group takes the band terms k = i0 - 1 - j - 8 t (t < 4) of all four rows, whose loads are in
// flight together, and a butterfly over the group adds each row's partial sums; the group's first
// lane then solves the block's own 4 x 4 triangle in registers (multiplying by the stored reciprocal
// diagonal) and writes the four values, which the next block reads.
__device__ void patch3_forward(Patch3LDS& sh, int ncol) {
  constexpr int NV = Patch3LDS::NV, NB = Patch3LDS::NB, NX = Patch3LDS::NX, BW = PT<3>::BW, G = 8, RB = 4;
  static_assert(G * 4 >= BW && RB <= G * 4 - BW + 1 + RB, "four terms per lane cover the band");
  const int grp = (int)threadIdx.x / G, j = (int)threadIdx.x % G;
  const bool act = grp < ncol;
  double* Xc = sh.X + (act ? grp : 0);
  for (int i0 = 0; i0 < NV; i0 += RB) {
    double part[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) part[r] = 0;
    double rhs[RB], rdg[RB], lblk[RB][RB];
    if (act) {
      double xv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = i0 - 1 - j - G * t;
        xv[t] = k >= 0 ? Xc[k * NX] : 0.0;
      }
      double a[RB][4];
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int row = i0 + r, k = i0 - 1 - j - G * t;
          a[r][t] = (row < NV && k >= 0 && k >= row - BW) ? sh.Kb[row * NB + (row - k)] : 0.0;
        }
      if (j == 0)
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const int row = i0 + r;
          rhs[r] = row < NV ? Xc[row * NX] : 0.0;
          rdg[r] = row < NV ? sh.rd[row] : 1.0;
#pragma unroll
          for (int q = 0; q < r; ++q) lblk[r][q] = row < NV ? sh.Kb[row * NB + (r - q)] : 0.0;
        }
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t) part[r] += a[r][t] * xv[t];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int m = 1; m < G; m <<= 1) part[r] += __shfl_xor(part[r], m, G);
    if (act && j == 0) {
      double v[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        double s = rhs[r] - part[r];
#pragma unroll
        for (int q = 0; q < r; ++q) s -= lblk[r][q] * v[q];
        v[r] = s * rdg[r];
        if (i0 + r < NV) Xc[(i0 + r) * NX] = v[r];
      }
    }
    patch3_wave_sync();
  }
  __syncthreads();
}

// Banded Cholesky K = L L^T in place with one barrier per column: at step k every thread updates its
// entries (ii, jj), k < jj <= ii <= k + BW, of the trailing band by K_ii,k K_jj,k / K_kk from the still
// unscaled column k (its four entries' loads in flight together), and scales column k - 1, which no
// thread reads any more; the last column is scaled after the loop. Thread (a, b) of the 8 x 32 layout
// takes rows k + 1 + a + 8 s (s < 4) and column k + 1 + b.
__device__ void patch3_cholesky(Patch3LDS& sh) {
  constexpr int NV = Patch3LDS::NV, NB = Patch3LDS::NB, BW = PT<3>::BW;
  const int a = (int)threadIdx.x / 32, b = (int)threadIdx.x % 32;
  for (int k = 0; k < NV; ++k) {
    if (k > 0) {
      // scale column k - 1 below the diagonal by 1 / sqrt(its diagonal)
      const int kp = k - 1, i = kp + 1 + (int)threadIdx.x;
      const int lastp = kp + BW < NV - 1 ? kp + BW : NV - 1;
      if (i <= lastp) sh.Kb[i * NB + (i - kp)] *= 1.0 / sqrt(sh.Kb[kp * NB]);
    }
    const double dkk = sh.Kb[k * NB];
    if (threadIdx.x == 0 && !(dkk > 0.0)) sh.bad = 1;
    const int last = k + BW < NV - 1 ? k + BW : NV - 1;
    const int jj = k + 1 + b;
    if (jj <= last) {
      const double cj = sh.Kb[jj * NB + (jj - k)] / dkk;
      double li[4], kv[4];
      int idx[4];
      bool ok[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int ii = k + 1 + a + 8 * s;
        ok[s] = ii <= last && ii >= jj;
        idx[s] = ok[s] ? ii * NB + (ii - jj) : 0;
        li[s] = ok[s] ? sh.Kb[ii * NB + (ii - k)] : 0.0;
        kv[s] = ok[s] ? sh.Kb[idx[s]] : 0.0;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (ok[s]) sh.Kb[idx[s]] = kv[s] - li[s] * cj;
    }
    __syncthreads();
    if (k > 0 && threadIdx.x == 0) sh.Kb[(k - 1) * NB] = sqrt(sh.Kb[(k - 1) * NB]);
  }
  if (threadIdx.x == 0) sh.Kb[(NV - 1) * NB] = sqrt(sh.Kb[(NV - 1) * NB]);
  __syncthreads();
  for (int i = (int)threadIdx.x; i < NV; i += (int)blockDim.x) sh.rd[i] = 1.0 / sh.Kb[i * NB];
  __syncthreads();
}

// Dense Cholesky of F = -S (27 x 27, lower factor in sh.S) with one barrier per column, the same
// scheme as patch3_cholesky.
__device__ void patch3_schur_cholesky(Patch3LDS& sh) {
  constexpr int NP = Patch3LDS::NP;
  const int a = (int)threadIdx.x / 32, b = (int)threadIdx.x % 32;
  for (int e = (int)threadIdx.x; e < NP * NP; e += (int)blockDim.x) sh.S[e] = -sh.S[e];
  __syncthreads();
  for (int k = 0; k < NP; ++k) {
    if (k > 0) {
      const int kp = k - 1, i = kp + 1 + (int)threadIdx.x;
      if (i < NP) sh.S[i * NP + kp] *= 1.0 / sqrt(sh.S[kp * NP + kp]);
    }
    const double dkk = sh.S[k * NP + k];
    if (threadIdx.x == 0 && !(dkk > 0.0)) sh.bad = 1;
    const int jj = k + 1 + b;
    if (jj < NP) {
      const double cj = sh.S[jj * NP + k] / dkk;
      double li[4], kv[4];
      bool ok[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int ii = k + 1 + a + 8 * s;
        ok[s] = ii < NP && ii >= jj;
        li[s] = ok[s] ? sh.S[ii * NP + k] : 0.0;
        kv[s] = ok[s] ? sh.S[ii * NP + jj] : 0.0;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (ok[s]) sh.S[(k + 1 + a + 8 * s) * NP + jj] = kv[s] - li[s] * cj;
    }
    __syncthreads();
    if (k > 0 && threadIdx.x == 0) sh.S[(k - 1) * NP + (k - 1)] = sqrt(sh.S[(k - 1) * NP + (k - 1)]);
  }
  if (threadIdx.x == 0) sh.S[(NP - 1) * NP + (NP - 1)] = sqrt(sh.S[(NP - 1) * NP + (NP - 1)]);
  __syncthreads();
}

// Component cmp's part of the Schur complement and of the reduced right-hand side:
// S -= V^T V, t -= V^T z, w_cmp = y^T V, qg_cmp = y^T z.
__device__ void patch3_schur(Patch3LDS& sh, int cmp) {
  constexpr int NV = Patch3LDS::NV, NP = Patch3LDS::NP, NX = Patch3LDS::NX;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int mc = vel_center<3>();
  for (int e = tid; e < NP * NP + 2 * NP + 1; e += nt) {
    if (e < NP * NP) {
      const int i = e / NP, j = e % NP;
      double s = 0;
#pragma unroll 5
      for (int k = 0; k < NV; ++k) s += sh.X[k * NX + i] * sh.X[k * NX + j];
      sh.S[e] -= s;
    } else if (e < NP * NP + NP) {
      const int i = e - NP * NP;
      double s = 0;
#pragma unroll 5
      for (int k = 0; k < NV; ++k) s += sh.X[k * NX + i] * sh.X[k * NX + NP];
      sh.t[i] -= s;
    } else if (e < NP * NP + 2 * NP) {
      const int i = e - NP * NP - NP;
      double s = 0;
      for (int k = mc; k < NV; ++k) s += sh.y[k] * sh.X[k * NX + i];
      sh.w[cmp][i] = s;
    } else {
      double s = 0;
      for (int k = mc; k < NV; ++k) s += sh.y[k] * sh.X[k * NX + NP];
      sh.qg[cmp] = s;
    }
  }
  __syncthreads();
}

// cache_matrix / cache_none application in 3D (Eq. 14-15), one workgroup per patch: L_i from its
// stored values or from the operator rows, banded Cholesky of K, then per velocity component the
// forward substitution of [B_c | g_c (| e_m)] and its Schur contribution, the Cholesky of -S and the
// pressure solve; x[i] += omega times the centre entries. x == nullptr: factorise only and report
// singular blocks (set-up validation).
__global__ void __launch_bounds__(256) patch_solve3c_kernel(
    const OpConsts* __restrict__ oc, int policy, const int* __restrict__ node_class, const double* __restrict__ Mcls,
    const double* __restrict__ Mirr, const int* __restrict__ pattern, int npat, int64_t N,
    const double* __restrict__ r, double* __restrict__ x, double omega, int* err, const int* __restrict__ node_op,
    const double* __restrict__ nsten, int nk, int nbc) {
  constexpr int NV = Patch3LDS::NV, NP = Patch3LDS::NP, NB = Patch3LDS::NB, NX = Patch3LDS::NX;
  __shared__ Patch3LDS sh;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = oc->n;
  const int mc = vel_center<3>(), ip = pres_center<3>();
  const bool rows = policy != FCGMG_CACHE_MATRIX;
  for (int64_t node = blockIdx.x; node < N; node += gridDim.x) {
    int c[3];
    node_coords<3>(node, n, c);
    const double* vals = nullptr;
    if (!rows) {
      const int cls = node_class[node];
      vals = cls >= 0 ? Mcls + (int64_t)cls * npat : Mirr + (int64_t)(-cls - 1) * npat;
    }
    for (int i = tid; i < NV * NB; i += nt) sh.Kb[i] = 0;
    for (int i = tid; i < NP * NP; i += nt) sh.S[i] = 0;
    if (tid == 0) sh.bad = 0;
    // the pressure right-hand side
    for (int q = tid; q < NP; q += nt) {
      double val = 0;
      if (r && pres_in_grid<3>(c, n, q)) {
        const int cc[3] = {c[0] + q % 3 - 1, c[1] + (q / 3) % 3 - 1, c[2] + q / 9 - 1};
        val = r[3 * N + node_index<3>(cc, n)];
      }
      sh.t[q] = val;
    }
    __syncthreads();
    patch3_load(sh, -1, rows, oc, node_op, nsten, pattern, npat, nk, nbc, vals, c);
    __syncthreads();
    patch_pad<3>(sh, c, n);
    patch3_cholesky(sh);
    for (int cmp = 0; cmp < 3; ++cmp) {
      for (int i = tid; i < NV * NX; i += nt) sh.X[i] = 0;
      __syncthreads();
      patch3_load(sh, cmp, rows, oc, node_op, nsten, pattern, npat, nk, nbc, vals, c);
      // g_c = R_i r (zero outside the grid), and for the first component the unit column e_m
      for (int v = tid; v < NV; v += nt) {
        double val = 0;
        if (r && vel_in_grid<3>(c, n, v)) {
          const int cc[3] = {c[0] + v % 5 - 2, c[1] + (v / 5) % 5 - 2, c[2] + v / 25 - 2};
          val = r[cmp * N + node_index<3>(cc, n)];
        }
        sh.X[v * NX + NP] = val;
        if (cmp == 0) sh.X[v * NX + NP + 1] = v == mc ? 1.0 : 0.0;
      }
      __syncthreads();
      patch3_forward(sh, cmp == 0 ? NX : NX - 1);
      if (cmp == 0) {
        for (int v = tid; v < NV; v += nt) sh.y[v] = sh.X[v * NX + NP + 1];
        __syncthreads();
      }
      patch3_schur(sh, cmp);
    }
    patch3_schur_cholesky(sh);
    schur_solve<3>(sh);
    if (x != nullptr && tid <= 3) {
      double yv;
      if (tid < 3) {
        double s = sh.qg[tid];
        for (int j = 0; j < NP; ++j) s -= sh.w[tid][j] * sh.t[j];
        yv = s;
      } else {
        yv = sh.t[ip];
      }
      x[tid * N + node] += omega * yv;
    }
    if (tid == 0 && sh.bad) atomicMin(err, (int)node);
    __syncthreads();
  }
}

// cache_matrix / cache_none sweep with the immersed boundary terms (2D): every patch block, loaded
// from its stored pattern values or assembled on the fly, is factorised by the dense LU at each
// application and solved for its gathered residual; the centre DoFs take omega times the solution.
__global__ void __launch_bounds__(64) patch_solve_lu2_kernel(
    const OpConsts* __restrict__ oc, const int* __restrict__ cell_info, const double* __restrict__ cut, Geom g,
    double eta, int policy, const int* __restrict__ node_class, const double* __restrict__ Mcls,
    const double* __restrict__ Mirr, const int* __restrict__ pattern, int npat, int64_t N,
    const double* __restrict__ r, double* __restrict__ x, double omega, int* err, int integrate) {
  constexpr int D = 2, NV = PT<2>::NV, ZS = kLU2;
  __shared__ PatchLDS<2> sh;
  __shared__ double A[ZS * ZS];
  __shared__ double gv[ZS];
  __shared__ int piv[ZS];
  const int tid = threadIdx.x;
  const int n = oc->n;
  const int centre[D + 1] = {vel_center<2>(), NV + vel_center<2>(), D * NV + pres_center<2>()};
  for (int64_t node = blockIdx.x; node < N; node += gridDim.x) {
    int c[3];
    node_coords<D>(node, n, c);
    if (policy == FCGMG_CACHE_MATRIX) {
      const int cls = node_class[node];
      const double* vals = cls >= 0 ? Mcls + (int64_t)cls * npat : Mirr + (int64_t)(-cls - 1) * npat;
      patch_load_pattern<D>(sh, pattern, npat, vals);
    } else {
      // cache_none: the element matrices the residual applies (reference ones and the cut cells'
      // set-up integrals), or with `integrate` the cut cells integrated again here
      patch_assemble<D>(sh, oc, cell_info, cut, g, eta, c, integrate ? 1 : 0);
    }
    patch_pad<D>(sh, c, n);
    // g = R_i r, zero outside the grid
    for (int e = tid; e < ZS; e += 64) {
      double val = 0;
      if (e < D * NV) {
        const int cmp = e / NV, v = e % NV;
        if (r && vel_in_grid<D>(c, n, v)) {
          int cc[3] = {c[0] + v % 5 - 2, c[1] + v / 5 - 2, 0};
          val = r[cmp * N + node_index<D>(cc, n)];
        }
      } else {
        const int q = e - D * NV;
        if (r && pres_in_grid<D>(c, n, q)) {
          int cc[3] = {c[0] + q % 3 - 1, c[1] + q / 3 - 1, 0};
          val = r[D * N + node_index<D>(cc, n)];
        }
      }
      gv[e] = val;
    }
    patch_dense2(sh, A);
    const bool bad = lu_factor2(A, piv);
    if (!bad) lu_solve2_wave(A, piv, gv);
    __syncthreads();
    if (x != nullptr && tid <= D && !bad) x[tid * N + node] += omega * gv[centre[tid]];
    if (tid == 0 && bad) atomicMin(err, (int)node);
    __syncthreads();
  }
}

// ================================================================================================
// cache_matrix / cache_none application in 2D: two patches per wavefront, 32 lanes each, and no
// workgroup barrier. L_i = [[I_2 (x) K, B], [B^T, C]] (K: 25 x 25 of half bandwidth 6, B_c: 25 x 9,
// C: 9 x 9) is solved by the same block elimination as patch_solve_kernel, arranged so that every
// lane carries one right-hand-side column of the velocity solves: lanes 0-8 the columns of B_x,
// lane 9 g_x, lanes 10-18 B_y, lane 19 g_y, lane 20 the unit vector of the centre velocity node
// (lanes 21-31 shadow column 0). Row i of the Cholesky factor of K is formed in every lane (the same
// values; no exchange) from the previous rows kept in registers; each lane advances its column by
// one row of the forward substitution, the 21 new values are exchanged through LDS, and the
// products that build the pressure Schur complement S = C - sum_c V_c^T V_c, its right-hand side
// and the centre-row terms are accumulated as the rows complete, so V is never stored. The 9 x 9
// system in F = -S is factorised in every lane. A lane's accumulation order does not depend on its
// column, so the computed S is exactly symmetric.
// ================================================================================================
constexpr int kS2Cols = 21;

// f(std::integral_constant<int, I>) for I = B .. E-1, unrolled at compile time.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Largest stored pattern of a 2D patch block (288 entries), rounded up to whole lane rounds.
constexpr int kMaxPattern2 = 320;

// Modes of the 2D factorising kernel: the stored pattern values (cache_matrix), the operator rows
// (cache_none), or the element integrals of the window with its cut cells integrated on the fly
// (cache_none, fcgmg_set_cache_none_assembly).
enum { kSolveMatrix = 0, kSolveRows = 1, kSolveIntegrate = 2 };

template <int MODE>
struct Solve2LDS {
  double Kb[25 * 7];              // lower band of K: Kb[v * 7 + (v - j)] = K[v][j]
  double X[25 * kS2Cols];         // X[v * 21 + l]: right-hand-side column l at velocity window node v, then V
  double C[81];                   // C, then F = -S (column l written by lane l)
  double aux[32];                 // pressure right-hand side, then t (0-8); w_c (9-26); y^T z_c (27, 28)
  double cell[MODE == kSolveIntegrate ? 48 : 1];                  // one cut cell integrated on the fly
  double lball[MODE == kSolveIntegrate ? 4 * kMaxLocalBalls : 1];  // the balls that touch it
  int bad;
};

// Orders the LDS accesses of one wavefront (its LDS instructions execute in order; this only stops
// the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  asm volatile("" ::: "memory");
}

// The balls that touch the box [lo, lo + s]^2, collected by the 32 lanes of one half-wavefront (lane
// l, half h) into `out`; -1 if more than kMaxLocalBalls touch it (the caller keeps the full list).
__device__ int cull_balls_half(const Geom& g, const double* lo, double s, double* out, int l, int half) {
  int cnt = 0;
  for (int base = 0; base < g.nballs; base += 32) {
    const int i = base + l;
    bool touch = false;
    if (i < g.nballs) {
      const double* b = g.balls + 4 * i;
      double dmin2 = 0;
      for (int k = 0; k < 2; ++k) {
        const double a = lo[k] - b[k], e = lo[k] + s - b[k];
        const double m = a > 0 ? a : (e < 0 ? -e : 0.0);
        dmin2 += m * m;
      }
      touch = dmin2 <= b[3] * b[3];
    }
    const unsigned hm = (unsigned)(__ballot(touch) >> (32 * half));
    const int pos = cnt + __popc(hm & ((1u << l) - 1u));
    if (touch && pos < kMaxLocalBalls)
      for (int k = 0; k < 4; ++k) out[4 * pos + k] = g.balls[4 * i + k];
    cnt += __popc(hm);
  }
  wave_lds_sync();
  return cnt > kMaxLocalBalls ? -1 : cnt;
}

template <int MODE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MODE == kSolveIntegrate ? 1 : 3, 8)))
patch_solve_lanes2_kernel(
    const OpConsts* __restrict__ oc, const int* __restrict__ node_op, const double* __restrict__ nsten,
    const int* __restrict__ node_class, const double* __restrict__ Mcls, const double* __restrict__ Mirr,
    const int* __restrict__ pattern, int npat, int64_t N, const double* __restrict__ r, double* __restrict__ x,
    double omega, int* err, const int* __restrict__ cell_info, Geom g, double eta) {
  constexpr int NV = 25, NP = 9, NB = 7, NC = kS2Cols, MC = 12;
  constexpr bool NONE = MODE != kSolveMatrix;
  __shared__ Solve2LDS<MODE> shp[2];
  const int half = (int)threadIdx.x >> 5, l = (int)threadIdx.x & 31;
  const int n = oc->n;
  const int64_t npair = (N + 1) / 2;
  for (int64_t pair = blockIdx.x; pair < npair; pair += gridDim.x) {
    // the half's LDS block through an opaque index, so that the hundreds of addresses derived from
    // it are formed where they are used instead of being hoisted out of this loop into registers
    int hsel = half;
    asm volatile("" : "+v"(hsel));
    Solve2LDS<MODE>& sh = shp[hsel];
    const int64_t node_raw = 2 * pair + half;
    const bool live = node_raw < N;
    const int64_t node = live ? node_raw : N - 1;  // a spare half repeats the last patch, unwritten
    int c[3];
    node_coords<2>(node, n, c);
    // global loads first, all independent of each other except the stored values (which follow the
    // patch class): the residual gather g = R_i r and, for cache_matrix, the pattern codes and values
    double rv[2], rp = 0;
    for (int k = 0; k < 2; ++k) {
      const int e = l + 32 * k, cmp = e / NV, v = e % NV;
      rv[k] = 0;
      if (r && e < 2 * NV && vel_in_grid<2>(c, n, v)) {
        const int cc[3] = {c[0] + v % 5 - 2, c[1] + v / 5 - 2, 0};
        rv[k] = r[cmp * N + node_index<2>(cc, n)];
      }
    }
    if (r && l < NP && pres_in_grid<2>(c, n, l)) {
      const int cc[3] = {c[0] + l % 3 - 1, c[1] + l / 3 - 1, 0};
      rp = r[2 * N + node_index<2>(cc, n)];
    }
    constexpr int NPL = NONE ? 1 : kMaxPattern2 / 32;  // stored pattern entries per lane
    int pcode[NPL];
    double pval[NPL];
    if constexpr (!NONE) {
      const int cls = node_class[node];
      const double* vals = cls >= 0 ? Mcls + (int64_t)cls * npat : Mirr + (int64_t)(-cls - 1) * npat;
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        const int e = l + 32 * k;
        pcode[k] = e < npat ? pattern[e] : -1;
        pval[k] = e < npat ? vals[e] : 0.0;
      }
    }
    for (int i = l; i < NV * NC; i += 32) sh.X[i] = 0;
    for (int i = l; i < NV * NB; i += 32) sh.Kb[i] = 0;
    for (int i = l; i < NP * NP; i += 32) sh.C[i] = 0;
    if (l == 0) sh.bad = 0;
    wave_lds_sync();
    if constexpr (!NONE) {
      // the stored pattern values of L_i (one shared block per class, one per individual patch)
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        const int code = pcode[k];
        if (code < 0) continue;
        const int type = code >> 24, i = (code >> 12) & 0xfff, j = code & 0xfff;
        const double v = pval[k];
        if (type == 0) {
          sh.Kb[i * NB + (i - j)] = v;
        } else if (type <= 2) {
          sh.X[i * NC + (type - 1) * 10 + j] = v;
        } else {
          sh.C[i * NP + j] = v;
          sh.C[j * NP + i] = v;
        }
      }
      wave_lds_sync();
    } else if constexpr (MODE == kSolveRows) {
      // L_i = R_i L R_i^T (Eq. 15) retrieved from the rows of L that the residual applies: lane
      // v < 25 takes velocity node v of the 5 x 5 window, reads its operator code and row (the
      // level's reference stencil of its kind, or its stored stencil) and writes the entries whose
      // column lies in the patch: its row of the lower band of K, of B_x and B_y (columns of the
      // 3 x 3 pressure window) and, for the nine inner nodes, its pressure row of C. Every entry of
      // the block is written once, by the lane of its row.
      if (l < NV && vel_in_grid<2>(c, n, l)) {
        using RL = RefLayout<2>;
        const int vx = l % 5, vy = l / 5;
        const int gx0 = c[0] + vx - 2, gy0 = c[1] + vy - 2;
        const int op = node_op[gx0 + (int64_t)(n + 1) * gy0];
        const bool inner = vx >= 1 && vx <= 3 && vy >= 1 && vy <= 3;
        const int qa = (vx - 1) + 3 * (vy - 1);
        const double* __restrict__ st = op >= 0 ? nsten + (int64_t)op * PT<2>::NSTEN : nullptr;
        const double* __restrict__ pk = oc->pack;
        const int ku = op >= 0 ? 0 : -op - 1;
        // coefficient j of offset o: 0 K, 1 / 2 B_x / B_y, 5 C (the layout of the stored stencils)
        auto coef = [&](int j, int o) -> double {
          if (st) return st[j * 9 + o];
          if (j == 0) return pk[RL::oSK + ku * 9 + o];
          if (j <= 2) return pk[RL::oSB + (ku * 2 + j - 1) * 9 + o];
          return pk[RL::oSC + o];
        };
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          const int ox = o % 3 - 1, oy = o / 3 - 1;
          const int gx = gx0 + ox, gy = gy0 + oy;
          if (gx < 0 || gx > n || gy < 0 || gy > n) continue;
          const int xb = vx + ox, yb = vy + oy;
          if (xb >= 0 && xb <= 4 && yb >= 0 && yb <= 4) {
            const int vb = xb + 5 * yb;
            if (vb <= l) sh.Kb[l * NB + (l - vb)] = coef(0, o);
          }
          if (xb >= 1 && xb <= 3 && yb >= 1 && yb <= 3) {
            const int qb = (xb - 1) + 3 * (yb - 1);
            sh.X[l * NC + qb] = coef(1, o);
            sh.X[l * NC + 10 + qb] = coef(2, o);
            if (inner) sh.C[qa * NP + qb] = coef(5, o);
          }
        }
      }
      wave_lds_sync();
    } else {
      const double h = oc->h;
      // on-the-fly assembly from the 6 x 6 cell window (Eq. 15: L_i = R_i L R_i^T): first the uncut
      // cells from the reference matrices, in window order, then the cut cells, integrated on the
      // fly; in the second pass each half takes its k-th cut cell at step k, so that the two halves
      // of the wavefront integrate together. Lane l holds the codes of window cells l and l + 32
      // (-3: outside the grid).
      int info2[2];
      for (int k = 0; k < 2; ++k) {
        const int w = l + 32 * k;
        const int cx = c[0] + w % 6 - 3, cy = c[1] + w / 6 - 3;
        info2[k] = (w < 36 && cx >= 0 && cx < n && cy >= 0 && cy < n) ? cell_info[cx + (int64_t)n * cy] : -3;
      }
      auto scatter = [&](int w, const double* Kp, const double* Bp, int bstride) {
        const int wx = w % 6, wy = w / 6;
        const int cx = c[0] + wx - 3, cy = c[1] + wy - 3;
        int fmask = 0;
        if (cx == 0 && oc->dirichlet[0]) fmask |= 1;
        if (cx == n - 1 && oc->dirichlet[1]) fmask |= 2;
        if (cy == 0 && oc->dirichlet[2]) fmask |= 4;
        if (cy == n - 1 && oc->dirichlet[3]) fmask |= 8;
        for (int k = 0; k < 2; ++k) {
          const int it = l + 32 * k;  // (block, a, b): K, B_x, B_y, C, 16 pairs each
          const int blk = it >> 4, ab = it & 15, a = ab >> 2, b = ab & 3;
          const int xa = wx + (a & 1) - 1, ya = wy + (a >> 1) - 1, xb = wx + (b & 1) - 1, yb = wy + (b >> 1) - 1;
          const int pxa = xa - 1, pya = ya - 1, pxb = xb - 1, pyb = yb - 1;
          const bool va_ok = xa >= 0 && xa <= 4 && ya >= 0 && ya <= 4;
          const bool vb_ok = xb >= 0 && xb <= 4 && yb >= 0 && yb <= 4;
          const bool qa_ok = pxa >= 0 && pxa <= 2 && pya >= 0 && pya <= 2;
          const bool qb_ok = pxb >= 0 && pxb <= 2 && pyb >= 0 && pyb <= 2;
          const int va = xa + 5 * ya, vb = xb + 5 * yb, qa = pxa + 3 * pya, qb = pxb + 3 * pyb;
          if (blk == 0) {
            if (va_ok && vb_ok && va >= vb) {
              double v = Kp[a * 4 + b];
              for (int f = 0; f < 4; ++f)
                if (fmask & (1 << f)) v += oc->FK[f][a * 4 + b];
              sh.Kb[va * NB + (va - vb)] += v;
            }
          } else if (blk <= 2) {
            const int cmp = blk - 1;
            if (va_ok && qb_ok) {
              double v = Bp[cmp * bstride + a * 4 + b];
              for (int sd = 0; sd < 2; ++sd)
                if (fmask & (1 << (2 * cmp + sd))) v += oc->FB[2 * cmp + sd][a * 4 + b];
              sh.X[va * NC + cmp * 10 + qb] += v;
            }
          } else if (qa_ok && qb_ok) {
            sh.C[qa * NP + qb] += oc->C[a * 4 + b];
          }
        }
        wave_lds_sync();
      };
      for (int w = 0; w < 36; ++w) {
        const int info = __shfl(w < 32 ? info2[0] : info2[1], (half << 5) + (w & 31), 64);
        if (info == -3 || info >= 0) continue;
        const int kind = info == -1 ? 0 : 1;
        scatter(w, oc->K[kind], oc->B[kind][0], 64);
      }
      // the cut cells of this half's window as a bit mask over the 36 window positions
      const unsigned long long m0 = __ballot(info2[0] >= 0), m1 = __ballot(info2[1] >= 0);
      unsigned long long cutm = ((m0 >> (32 * half)) & 0xffffffffull) | (((m1 >> (32 * half)) & 0xfull) << 32);
      const int ncut_h = __popcll(cutm);
      const int ncut_o = __shfl(ncut_h, ((1 - half) << 5), 64);
      const int nsteps = ncut_h > ncut_o ? ncut_h : ncut_o;
      for (int k = 0; k < nsteps; ++k) {
        const int w = cutm ? __builtin_ctzll(cutm) : -1;
        cutm &= cutm ? cutm - 1 : 0ull;
        const int info = __shfl(w >= 0 && w < 32 ? info2[0] : info2[1], (half << 5) + (w & 31), 64);
        if (w < 0) continue;  // this half has no more cut cells
        (void)info;
        const int wx = w % 6, wy = w / 6;
        const double lo[3] = {(c[0] + wx - 3) * h, (c[1] + wy - 3) * h, 0.0};
        const int nb = cull_balls_half(g, lo, h, sh.lball, l, half);
        Geom gl = g;
        if (nb >= 0) {
          gl.balls = sh.lball;
          gl.nballs = nb;
        }
        if (gl.q >= 3) {
          // the cell's tree below depth 3: lane l integrates sub-boxes l and l + 32 of the 8 x 8
          // (side h / 8) to the level's depth, every entry at once; the 32 partial sums are then
          // added by a butterfly. (A box above depth 3 that is not cut becomes uncut sub-boxes here:
          // the 2 x 2 Gauss rule is exact on each, so the integral is the same up to rounding.)
          double acc[48];
#pragma unroll
          for (int e = 0; e < 48; ++e) acc[e] = 0;
          const double hs = 0.125 * h;
          Geom gs = gl;
          gs.q = gl.q - 3;
          for (int k2 = 0; k2 < 2; ++k2) {
            const int bidx = l + 32 * k2;
            const double los[3] = {lo[0] + (bidx & 7) * hs, lo[1] + (bidx >> 3) * hs, 0.0};
            tree_quadrature<2>(gs, los, hs, [&](const double* xq, double wq, double alpha) {
              double phi[4], gr[4][3];
              q1<2>(lo, h, xq, phi, gr);
              const double wa = wq * alpha;
#pragma unroll
              for (int e = 0; e < 48; ++e) acc[e] += point_entry<2>(e, eta, wa, phi, gr);
            });
          }
#pragma unroll
          for (int e = 0; e < 48; ++e) {
            double v = acc[e];
            for (int m = 1; m < 32; m <<= 1) v += __shfl_xor(v, m, 32);
            acc[e] = v;
          }
          if (l == 0)
#pragma unroll
            for (int e = 0; e < 48; ++e) sh.cell[e] = acc[e];
        } else {
          // trees of depth 0 to 2: every lane walks the whole tree for entries l and l + 32
          double a0 = 0, a1 = 0;
          tree_quadrature<2>(gl, lo, h, [&](const double* xq, double wq, double alpha) {
            double phi[4], gr[4][3];
            q1<2>(lo, h, xq, phi, gr);
            const double wa = wq * alpha;
            a0 += point_entry<2>(l, eta, wa, phi, gr);
            if (l < 16) a1 += point_entry<2>(l + 32, eta, wa, phi, gr);
          });
          sh.cell[l] = a0;
          if (l < 16) sh.cell[l + 32] = a1;
        }
        wave_lds_sync();
        scatter(w, sh.cell, sh.cell + 16, 16);
      }
    }
    // window positions outside the grid are decoupled; g = R_i r (zero outside the grid) into the
    // columns 9 and 19, its pressure part into aux; the unit column of the centre velocity node
    if (l < NV && !vel_in_grid<2>(c, n, l)) sh.Kb[l * NB] = 1.0;
    if (l < NP && !pres_in_grid<2>(c, n, l)) sh.C[l * NP + l] = -1.0;
    for (int k = 0; k < 2; ++k) {
      const int e = l + 32 * k, cmp = e / NV, v = e % NV;
      if (e < 2 * NV) sh.X[v * NC + cmp * 10 + 9] = rv[k];
    }
    if (l < NV) sh.X[l * NC + 20] = l == MC ? 1.0 : 0.0;
    if (l < NP) sh.aux[l] = rp;
    wave_lds_sync();
    // velocity phase: band Cholesky of K row by row (every lane forms the same row and keeps the last
    // six in registers, shifted by one row per step), forward substitution of this lane's column (its
    // last six values in registers too), the new row of V exchanged through LDS, and the Schur
    // products accumulated as each row completes. The windows start as zero rows (inverse diagonal
    // 0), so the first steps need no bounds tests.
    const int lc = l < NC ? l : 0;
    const int cb = lc < 10 ? 0 : 10;  // first column of this lane's component block
    double Lw[6][5];                  // Lw[s][k - 1] = L[i - 6 + s][i - 6 + s - k], k = 1..5 (rows i-6..i-1)
    double Dw[6];                     // Dw[s] = 1 / L[i - 6 + s][i - 6 + s]
    double vw[6];                     // vw[s] = V[i - 6 + s][column]
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      Dw[s] = 0.0;
      vw[s] = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k) Lw[s][k] = 0.0;
    }
    double sacc[9], wacc = 0;
    for (int a = 0; a < 9; ++a) sacc[a] = 0;
    bool bad = false;
#pragma unroll 1
    for (int i = 0; i < NV; ++i) {
      const int ko = i * NB, xo = i * NC;
      double li[6];  // li[t] = L[i][i - 6 + t]
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        double s = sh.Kb[ko + (6 - t)];
#pragma unroll
        for (int u = 0; u < t; ++u) s -= li[u] * Lw[t][t - u - 1];  // L[i-6+t][i-6+u]
        li[t] = s * Dw[t];
      }
      double d = sh.Kb[ko];
#pragma unroll
      for (int t = 0; t < 6; ++t) d -= li[t] * li[t];
      bad |= !(d > 0.0);
      const double inv = rsqrt(d);
      double v = sh.X[xo + lc];
#pragma unroll
      for (int t = 0; t < 6; ++t) v -= li[t] * vw[t];
      v *= inv;
      // shift the windows by one row: row i enters at s = 5 with L[i][i-k] = li[6-k]
#pragma unroll
      for (int s = 0; s < 5; ++s) {
        Dw[s] = Dw[s + 1];
        vw[s] = vw[s + 1];
#pragma unroll
        for (int k = 0; k < 5; ++k) Lw[s][k] = Lw[s + 1][k];
      }
      Dw[5] = inv;
      vw[5] = v;
#pragma unroll
      for (int k = 1; k <= 5; ++k) Lw[5][k - 1] = li[6 - k];
      wave_lds_sync();  // every lane has read row i of X
      if (l < NC) sh.X[xo + l] = v;
      wave_lds_sync();
#pragma unroll
      for (int a = 0; a < 9; ++a) sacc[a] += sh.X[xo + cb + a] * v;
      if (i >= MC) wacc += sh.X[xo + 20] * v;
    }
    // F = -S = sum_c V_c^T V_c - C, column a from lanes a (B_x) and 10 + a (B_y); t = g_p - sum_c V_c^T z_c
    // from lanes 9 and 19; w_c and y^T z_c from every column lane
    double* sy = sh.X;  // 10 x 9: the sums of lanes 10-19 (X is no longer read)
    if (l >= 10 && l < 20)
      for (int a = 0; a < 9; ++a) sy[(l - 10) * 9 + a] = sacc[a];
    if (l < 20) sh.aux[l % 10 == 9 ? 27 + l / 10 : 9 + (l / 10) * 9 + l % 10] = wacc;
    wave_lds_sync();
    if (l < 9) {
      for (int a = 0; a < 9; ++a) sh.C[a * NP + l] = sacc[a] + sy[l * 9 + a] - sh.C[a * NP + l];
    } else if (l == 9) {
      for (int a = 0; a < 9; ++a) sh.aux[a] = sh.aux[a] - (sacc[a] + sy[9 * 9 + a]);
    }
    wave_lds_sync();
    // F p = -t by Cholesky F = R R^T in every lane (R in registers; the barrier at each row keeps
    // the compiler from loading all of F at once), then the two triangular solves
    const double* F = sh.C;
    double R[45], rinv[9], p[9];
    static_for<0, NP>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      wave_lds_sync();
      static_for<0, i>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        double s = F[i * NP + j];
        static_for<0, j>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          s -= R[i * (i + 1) / 2 + k] * R[j * (j + 1) / 2 + k];
        });
        R[i * (i + 1) / 2 + j] = s * rinv[j];
      });
      double d = F[i * NP + i];
      static_for<0, i>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        d -= R[i * (i + 1) / 2 + k] * R[i * (i + 1) / 2 + k];
      });
      bad |= !(d > 0.0);
      rinv[i] = rsqrt(d);
    });
    static_for<0, NP>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      double s = -sh.aux[i];
      static_for<0, i>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        s -= R[i * (i + 1) / 2 + k] * p[k];
      });
      p[i] = s * rinv[i];
    });
    static_for<0, NP>([&](auto ic) {
      constexpr int i = NP - 1 - decltype(ic)::value;
      double s = p[i];
      static_for<i + 1, NP>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        s -= R[k * (k + 1) / 2 + i] * p[k];
      });
      p[i] = s * rinv[i];
    });
    if (live && l <= 2 && x != nullptr && !bad) {
      double y;
      if (l < 2) {
        y = sh.aux[27 + l];
#pragma unroll
        for (int a = 0; a < 9; ++a) y -= sh.aux[9 + l * 9 + a] * p[a];
      } else {
        y = p[4];
      }
      x[l * N + node] += omega * y;
    }
    if (live && bad && l == 0) atomicMin(err, (int)node);
    wave_lds_sync();
  }
}

template <int D>
hipError_t k_patch_solve(const Ctx& c, const Level& L, int policy, const double* r, double* x, hipStream_t s) {
  const int64_t nb = L.N < 131072 ? L.N : 131072;
  if constexpr (D == 2) {
    if (L.dense_lu) {
      patch_solve_lu2_kernel<<<dim3((unsigned)nb), dim3(64), 0, s>>>(
          L.consts, L.cell_info, L.cut_mats, c.geom(L), c.prm.eta, policy, L.node_class, L.Mcls, L.Mirr,
          c.pattern, c.n_pattern, L.N, r, x, c.prm.omega, c.err, c.none_integrate ? 1 : 0);
      return hipGetLastError();
    }
    if (c.n_pattern > kMaxPattern2) return hipErrorInvalidValue;
    const int64_t npair = (L.N + 1) / 2;
    const int64_t nb2 = npair < 65536 ? npair : 65536;
#define FCG_LANES2(MODE)                                                                                     \
  patch_solve_lanes2_kernel<MODE><<<dim3((unsigned)nb2), dim3(64), 0, s>>>(                                  \
      L.consts, L.node_op, L.nsten, L.node_class, L.Mcls, L.Mirr, c.pattern, c.n_pattern, L.N, r, x,           \
      c.prm.omega, c.err, L.cell_info, c.geom(L), c.prm.eta)
    if (policy == FCGMG_CACHE_MATRIX)
      FCG_LANES2(kSolveMatrix);
    else if (c.none_integrate)
      FCG_LANES2(kSolveIntegrate);
    else
      FCG_LANES2(kSolveRows);
#undef FCG_LANES2
    return hipGetLastError();
  }
  if (D == 3 && !(policy == FCGMG_CACHE_NONE && c.none_integrate)) {
    // sizes of the K and B_c parts of the stored pattern (pattern_entries lists K, B_x, B_y, B_z, C)
    static const int nk = pattern_count3(0), nbc = pattern_count3(1);
    patch_solve3c_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(L.consts, policy, L.node_class, L.Mcls, L.Mirr,
                                                                   c.pattern, c.n_pattern, L.N, r, x, c.prm.omega,
                                                                   c.err, L.node_op, L.nsten, nk, nbc);
    return hipGetLastError();
  }
  patch_solve_kernel<D><<<dim3((unsigned)nb), dim3(PT<D>::THREADS), 0, s>>>(
      L.consts, L.cell_info, L.cut_mats, c.geom(L), c.prm.eta, policy, L.node_class, L.Mcls, L.Mirr, c.pattern,
      c.n_pattern, L.N, r, x, c.prm.omega, c.err, L.node_op, L.nsten, c.none_integrate);
  return hipGetLastError();
}

// ================================================================================================
// cache_inverse application (Eq. 14-15 with the stored rows Z_i): y_f = Z_i[f,:] . R_i r,
// x[i, f] += omega y_f.
//   Regular patches: the class rows are wavefront-uniform and read with scalar loads; a
//   "waterfall" loops over the distinct classes present in a wavefront. The residual comes from an
//   LDS tile (two-node halo).
//   Irregular patches: one wavefront per patch, lanes over the patch columns, rows streamed
//   coalesced from HBM, reduction across the wavefront.
// The fused 2D sweep kernel computes the residual tile itself (x with a three-node halo) and writes
// the new iterate to a second buffer; it performs exactly the same arithmetic as the residual
// kernel followed by the two apply kernels.
// ================================================================================================

// y[f] += Z[f,:] . g for a regular patch; rt(f, o) = r_f at the centre node + o. P is a pointer to
// the rows in the constant address space (scalar loads) or the global one (per-lane loads).
template <int D, bool UNR, class T, class P, class RA>
__device__ __forceinline__ void regular_rows(P Z, RA&& rt, T* y) {
  constexpr int NV = PT<D>::NV, NP = PT<D>::NP, ZSP = PT<D>::ZSP;
#pragma unroll
  for (int cmp = 0; cmp < D; ++cmp) {
#pragma unroll(UNR ? NV : 5)
    for (int v = 0; v < NV; ++v) {
      const int o[3] = {v % 5 - 2, (v / 5) % 5 - 2, D == 3 ? v / 25 - 2 : 0};
      const T gv = rt(cmp, o);
#pragma unroll
      for (int f = 0; f <= D; ++f) y[f] += Z[f * ZSP + cmp * NV + v] * gv;
    }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int o[3] = {q % 3 - 1, (q / 3) % 3 - 1, D == 3 ? q / 9 - 1 : 0};
    const T gv = rt(D, o);
#pragma unroll
    for (int f = 0; f <= D; ++f) y[f] += Z[f * ZSP + D * NV + q] * gv;
  }
}

// Regular patches of a wavefront: a waterfall over the classes present (at most two per level:
// interior physical and interior fictitious), each applied with scalar loads of its rows. Lanes
// with cls < 0 take no part.
template <int D, bool UNR = true, class T, class RA>
__device__ __forceinline__ void regular_apply(const T* __restrict__ Zcls, int cls, RA&& rt, T* y) {
  constexpr int ZSP = PT<D>::ZSP;
  bool todo = cls >= 0;
  while (__ballot(todo) != 0) {
    if (todo) {
      const int c0 = __builtin_amdgcn_readfirstlane(cls);
      if (cls == c0) {
        // read the lane value again inside the branch: the compiler would otherwise substitute the
        // (equal, per-lane) cls for c0 and lose the scalar address
        const int cu = __builtin_amdgcn_readfirstlane(cls);
        regular_rows<D, UNR, T>((cconst<T>*)(Zcls + (int64_t)cu * (D + 1) * ZSP), rt, y);
        todo = false;
      }
    }
  }
}

// Column j of a patch: field and offset of the node.
template <int D>
__device__ __forceinline__ void patch_column(int col, int* field, int* o) {
  constexpr int NV = PT<D>::NV;
  if (col < D * NV) {
    *field = col / NV;
    const int v = col % NV;
    o[0] = v % 5 - 2;
    o[1] = (v / 5) % 5 - 2;
    o[2] = D == 3 ? v / 25 - 2 : 0;
  } else {
    *field = D;
    const int q = col - D * NV;
    o[0] = q % 3 - 1;
    o[1] = (q / 3) % 3 - 1;
    o[2] = D == 3 ? q / 9 - 1 : 0;
  }
}

// acc[f] = Z[f,:] . g for an irregular patch, computed by a group of 16 lanes (j16 = lane in the
// group); rg(field, o) = r at centre + o, or 0 outside the grid. Each lane takes the neighbouring
// columns 2 j16 and 2 j16 + 1 of every step of 32 (the rows start 16-byte aligned, so the pair loads
// as one vector; an odd last column stands alone), summing them in that order. Every lane of the
// group returns the full sums. A wavefront holds 4 groups and each group takes two patches at once
// (A, B), so the rows of 8 patches stream from memory per wavefront and loop trip. The arithmetic
// of each patch does not depend on which patch it is paired with.
template <class T>
struct Pair2 {
  using type = typename std::conditional<std::is_same<T, double>::value, double2, float2>::type;
};

template <int D, class T, class RGA, class RGB, class PZ>
__device__ __forceinline__ void irregular_pair(PZ __restrict__ ZA, PZ __restrict__ ZB,
                                               bool has_b, int j16, RGA&& rga, RGB&& rgb, T* acca,
                                               T* accb) {
  using V2 = typename Pair2<T>::type;
  constexpr int ZS = PT<D>::ZS, ZSP = PT<D>::ZSP;
  static_assert(ZSP % 2 == 0, "rows of an even length, for aligned pairs");
#pragma unroll
  for (int f = 0; f <= D; ++f) acca[f] = accb[f] = 0;
  const PZ ZBs = has_b ? ZB : ZA;
#pragma unroll 2
  for (int c0 = 2 * j16; c0 < ZS; c0 += 32) {
    const bool two = c0 + 1 < ZS;
    int fa, fb, oa[3], ob[3];
    patch_column<D>(c0, &fa, oa);
    patch_column<D>(two ? c0 + 1 : c0, &fb, ob);
    V2 za[D + 1], zb[D + 1];
#pragma unroll
    for (int f = 0; f <= D; ++f) {
      za[f] = *(const V2*)(ZA + f * ZSP + c0);
      zb[f] = *(const V2*)(ZBs + f * ZSP + c0);
    }
    const T ga0 = rga(fa, oa), gb0 = has_b ? rgb(fa, oa) : T(0);
#pragma unroll
    for (int f = 0; f <= D; ++f) {
      acca[f] += za[f].x * ga0;
      accb[f] += zb[f].x * gb0;
    }
    if (two) {
      const T ga1 = rga(fb, ob), gb1 = has_b ? rgb(fb, ob) : T(0);
#pragma unroll
      for (int f = 0; f <= D; ++f) {
        acca[f] += za[f].y * ga1;
        accb[f] += zb[f].y * gb1;
      }
    }
  }
#pragma unroll
  for (int f = 0; f <= D; ++f)
#pragma unroll
    for (int msk = 8; msk >= 1; msk >>= 1) {
      acca[f] += __shfl_xor(acca[f], msk, 16);
      accb[f] += __shfl_xor(accb[f], msk, 16);
    }
}

// UNR: the class rows' column loop fully unrolled (fewest instructions) or rolled by 5 (3D: 44
// instead of 173 VGPRs, so more wavefronts per SIMD); the arithmetic and its order are the same.
template <int D, bool UNR, class T>
__global__ void __launch_bounds__(256) apply_regular_kernel(int n, int ntx, int nty, int ntz,
                                                            const int* __restrict__ node_class,
                                                            const T* __restrict__ Zcls,
                                                            const T* __restrict__ r, T* __restrict__ x,
                                                            T omega, int64_t sv) {
  // stacked vectors (sv apart): blockIdx.y is the vector
  r += (int64_t)blockIdx.y * sv;
  x += (int64_t)blockIdx.y * sv;
  constexpr int TX = TileShape<D>::TX, TY = TileShape<D>::TY, TZ = TileShape<D>::TZ;
  constexpr int HX = TX + 4, HY = TY + 4, HZ = D == 3 ? TZ + 4 : 1;
  constexpr int PLANE = HX * HY * HZ;
  __shared__ T rt[(D + 1) * PLANE];
  const int m = n + 1;
  const int64_t N = D == 2 ? (int64_t)m * m : (int64_t)m * m * m;
  const int nt[3] = {ntx, nty, ntz};
  int t[3];
  tile_coords<D, D == 3 ? 4 : 0>(blockIdx.x, nt, t);
  const int ox = t[0] * TX - 2, oy = t[1] * TY - 2, oz = D == 3 ? t[2] * TZ - 2 : 0;
  for (int e = threadIdx.x; e < (D + 1) * PLANE; e += 256) {
    const int f = e / PLANE, p = e % PLANE;
    const int gx = ox + p % HX, gy = oy + (p / HX) % HY, gz = D == 3 ? oz + p / (HX * HY) : 0;
    T v = 0;
    if (gx >= 0 && gx < m && gy >= 0 && gy < m && (D == 2 || (gz >= 0 && gz < m)))
      v = r[f * N + (D == 2 ? gx + (int64_t)m * gy : gx + (int64_t)m * (gy + (int64_t)m * gz))];
    rt[e] = v;
  }
  __syncthreads();
  const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = D == 3 ? threadIdx.x / (TX * TY) : 0;
  const int gx = t[0] * TX + tx, gy = t[1] * TY + ty, gz = D == 3 ? t[2] * TZ + tz : 0;
  const bool inside = gx < m && gy < m && (D == 2 || gz < m);
  const int64_t node = D == 2 ? gx + (int64_t)m * gy : gx + (int64_t)m * (gy + (int64_t)m * gz);
  const int cls = inside ? node_class[node] : -1;
  const int base = tx + 2 + HX * (ty + 2 + (D == 3 ? HY * (tz + 2) : 0));
  T y[D + 1];
#pragma unroll
  for (int f = 0; f <= D; ++f) y[f] = 0;
  regular_apply<D, UNR, T>(Zcls, cls, [&](int f, const int* o) {
    return rt[f * PLANE + base + o[0] + HX * (o[1] + (D == 3 ? HY * o[2] : 0))];
  }, y);
  if (cls >= 0)
#pragma unroll
    for (int f = 0; f <= D; ++f) x[f * N + node] += omega * y[f];
}

template <int D, class T>
__global__ void __launch_bounds__(256) apply_irregular_kernel(int n, int64_t nirr, const int* __restrict__ irr_nodes,
                                                              const int* __restrict__ irr_zrow,
                                                              const T* __restrict__ Zirr,
                                                              const T* __restrict__ r, T* __restrict__ x,
                                                              T omega) {
  constexpr int ZSP = PT<D>::ZSP;
  const int j16 = threadIdx.x & 15;
  const int m = n + 1;
  const int64_t N = D == 2 ? (int64_t)m * m : (int64_t)m * m * m;
  const int64_t stride = (int64_t)gridDim.x * 32;
  for (int64_t pa = blockIdx.x * 32 + (threadIdx.x >> 4); pa < nirr; pa += stride) {
    const int64_t pb = pa + 16;
    const bool has_b = pb < nirr;
    const int na = irr_nodes[pa], nbn = has_b ? irr_nodes[pb] : na;
    const int ca[3] = {na % m, (na / m) % m, D == 3 ? na / (m * m) : 0};
    const int cb[3] = {nbn % m, (nbn / m) % m, D == 3 ? nbn / (m * m) : 0};
    auto gather = [&](const int* c, int field, const int* o) {
      int cc[3] = {c[0] + o[0], c[1] + o[1], c[2] + o[2]};
      bool in = true;
      for (int k = 0; k < D; ++k) in = in && cc[k] >= 0 && cc[k] < m;
      return in ? r[field * N + (D == 2 ? cc[0] + (int64_t)m * cc[1] : cc[0] + (int64_t)m * (cc[1] + (int64_t)m * cc[2]))]
                : T(0);
    };
    T acca[D + 1], accb[D + 1];
    const int64_t za = irr_zrow[pa], zb = has_b ? irr_zrow[pb] : za;
    irregular_pair<D, T>(Zirr + za * (D + 1) * ZSP, Zirr + zb * (D + 1) * ZSP, has_b,
                      j16, [&](int f, const int* o) { return gather(ca, f, o); },
                      [&](int f, const int* o) { return gather(cb, f, o); }, acca, accb);
    if (j16 <= D) {
      T va = acca[0], vb = accb[0];
#pragma unroll
      for (int f = 1; f <= D; ++f)
        if (j16 == f) {
          va = acca[f];
          vb = accb[f];
        }
      x[j16 * N + na] += omega * va;
      if (has_b) x[j16 * N + nbn] += omega * vb;
    }
  }
}

// Streamed patches for nrhs right-hand sides at once (vectors nd apart, at most kMaxRhs): each
// 16-lane group takes one patch per trip, loads its rows once and applies them to the gathers of
// every right-hand side. Per right-hand side the arithmetic is that of irregular_pair, so each
// result equals the single-vector apply.
template <int D, class T>
__global__ void __launch_bounds__(256) apply_irregular_multi_kernel(int n, int64_t nirr, const int* __restrict__ irr_nodes,
                                                                    const int* __restrict__ irr_zrow,
                                                                    const T* __restrict__ Zirr,
                                                                    const T* __restrict__ r, T* __restrict__ x,
                                                                    int64_t nd, int nrhs, T omega) {
  constexpr int ZS = PT<D>::ZS, ZSP = PT<D>::ZSP;
  const int j16 = threadIdx.x & 15;
  const int m = n + 1;
  const int64_t N = D == 2 ? (int64_t)m * m : (int64_t)m * m * m;
  const int64_t stride = (int64_t)gridDim.x * 16;
  for (int64_t pa = blockIdx.x * 16 + (threadIdx.x >> 4); pa < nirr; pa += stride) {
    const int na = irr_nodes[pa];
    const T* Z = Zirr + (int64_t)irr_zrow[pa] * (D + 1) * ZSP;
    const int ca[3] = {na % m, (na / m) % m, D == 3 ? na / (m * m) : 0};
    T acc[kMaxRhs][D + 1];
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k)
#pragma unroll
      for (int f = 0; f <= D; ++f) acc[k][f] = 0;
    auto node_of = [&](int col, bool* in) {
      int field, o[3];
      patch_column<D>(col, &field, o);
      const int cc[3] = {ca[0] + o[0], ca[1] + o[1], ca[2] + o[2]};
      *in = true;
      for (int k = 0; k < D; ++k) *in = *in && cc[k] >= 0 && cc[k] < m;
      return field * N + (D == 2 ? cc[0] + (int64_t)m * cc[1] : cc[0] + (int64_t)m * (cc[1] + (int64_t)m * cc[2]));
    };
    // the column pairs and the order of irregular_pair
    using V2 = typename Pair2<T>::type;
#pragma unroll 2
    for (int c0 = 2 * j16; c0 < ZS; c0 += 32) {
      const bool two = c0 + 1 < ZS;
      bool in0, in1;
      const int64_t g0i = node_of(c0, &in0), g1i = node_of(two ? c0 + 1 : c0, &in1);
      V2 z[D + 1];
#pragma unroll
      for (int f = 0; f <= D; ++f) z[f] = *(const V2*)(Z + f * ZSP + c0);
#pragma unroll
      for (int k = 0; k < kMaxRhs; ++k)
        if (k < nrhs) {
          const T g0 = in0 ? r[k * nd + g0i] : T(0);
#pragma unroll
          for (int f = 0; f <= D; ++f) acc[k][f] += z[f].x * g0;
          if (two) {
            const T g1 = in1 ? r[k * nd + g1i] : T(0);
#pragma unroll
            for (int f = 0; f <= D; ++f) acc[k][f] += z[f].y * g1;
          }
        }
    }
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k)
#pragma unroll
      for (int f = 0; f <= D; ++f)
#pragma unroll
        for (int msk = 8; msk >= 1; msk >>= 1) acc[k][f] += __shfl_xor(acc[k][f], msk, 16);
    if (j16 <= D)
#pragma unroll
      for (int k = 0; k < kMaxRhs; ++k)
        if (k < nrhs) {
          T v = acc[k][0];
#pragma unroll
          for (int f = 1; f <= D; ++f)
            if (j16 == f) v = acc[k][f];
          x[k * nd + j16 * N + na] += omega * v;
        }
  }
}

template <int D, class T>
hipError_t k_apply_irregular_multi(const Ctx& c, const Level& L, const T* r, T* x, int64_t nd, int nrhs,
                                   hipStream_t s) {
  if (L.n_irr == 0) return hipSuccess;
  int64_t nb = (L.n_irr + 15) / 16;
  if (nb > 65536) nb = 65536;
  apply_irregular_multi_kernel<D, T><<<dim3((unsigned)nb), dim3(256), 0, s>>>(
      L.n, L.n_irr, L.irr_nodes, L.irr_zrow, LV<T>::Zirr(L), r, x, nd, nrhs, (T)c.prm.omega);
  return hipGetLastError();
}

// Tile shapes of the fused 2D sweep by level size (nodes): 32 x 8 tiles by 256 threads from
// kFusedBigTileNodes on, 8 x 4 by 128 from kFusedMidTileNodes on, 4 x 4 by 128 below.
constexpr int64_t kFusedBigTileNodes = 200000;
constexpr int64_t kFusedMidTileNodes = 30000;
struct Fused2Shape {
  int tx, ty, nt;
  int wpe;  // minimum waves per SIMD the compiler must allow (bounds the registers per lane)
};
constexpr Fused2Shape kFusedBig{32, 8, 256, 5}, kFusedMid{8, 4, 128, 5}, kFusedSmall{4, 4, 128, 4};
Fused2Shape fused2_shape(int64_t N) {
  return N >= kFusedBigTileNodes ? kFusedBig : (N >= kFusedMidTileNodes ? kFusedMid : kFusedSmall);
}

// The shapes fcgmg_autotune chooses from (tile x, tile y, threads, waves per SIMD); every shape does the same
// arithmetic per node, so the choice changes the time, not the result.
constexpr Fused2Shape kFusedShapes[] = {{32, 8, 256, 5}, {32, 8, 256, 4}, {32, 8, 256, 6}, {16, 16, 256, 5},
                                        {16, 8, 256, 5},  {8, 8, 128, 5},  {8, 4, 128, 5},  {4, 4, 128, 4}};
constexpr int kNumFusedShapes = 8;

// The level's shape: its autotuned one, else the default by size.
Fused2Shape level_fused2_shape(const Level& L) { return L.fshape >= 0 ? kFusedShapes[L.fshape] : fused2_shape(L.N); }

int fused2_num_shapes() { return kNumFusedShapes; }
void fused2_shape_dims(int k, int* tx, int* ty, int* nt, int* wpe) {
  *tx = kFusedShapes[k].tx;
  *ty = kFusedShapes[k].ty;
  *nt = kFusedShapes[k].nt;
  *wpe = kFusedShapes[k].wpe;
}

// Individual patches per workgroup part of a tile: two trips of all 16-lane groups on 32 x 8 tiles,
// one on the smaller shapes (where a whole tile takes at most two trips and splitting the heavy ones
// shortens the launch's tail).
constexpr int fused2_part_cap(const Fused2Shape& sh) { return (sh.tx * sh.ty >= 256 ? 4 : 2) * (sh.nt / 16); }
// the part code (tile * 4 + part) allows four parts per tile
constexpr bool fused2_shapes_fit() {
  for (int k = 0; k < kNumFusedShapes; ++k)
    if (kFusedShapes[k].tx * kFusedShapes[k].ty > 4 * fused2_part_cap(kFusedShapes[k]) ||
        kFusedShapes[k].nt < kFusedShapes[k].tx * kFusedShapes[k].ty || kFusedShapes[k].nt % 64)
      return false;
  return true;
}
static_assert(kFusedBig.tx * kFusedBig.ty <= 4 * fused2_part_cap(kFusedBig) &&
                  kFusedMid.tx * kFusedMid.ty <= 4 * fused2_part_cap(kFusedMid) &&
                  kFusedSmall.tx * kFusedSmall.ty <= 4 * fused2_part_cap(kFusedSmall) && fused2_shapes_fit(),
              "at most four parts per tile, and one thread per tile node at least");

// Fused sweep (2D): x_out = x_in + omega S (b - L x_in) for one TX x TY tile of nodes by NT >= TX TY
// threads; thread t < TX TY owns node t of the tile. Large grids use 32 x 8 tiles with one thread per
// node (less halo work); small grids, whose sweep time is the latency of one workgroup, use small
// tiles with four times as many threads (shorter residual and individual-patch loops per thread).
// The arithmetic of every node is the same for all shapes.
// mode 0: x_in as given; mode 1: x_in is zero (not read; the first sweep on a coarse level);
// mode 2: x_in plus the Q1 interpolation of the coarse vector xc (the coarse-grid correction of a
// V-cycle applied as the x tile is loaded, as prolong_add would apply it).
template <int TX, int TY, int NT, int CAP, class T>
__device__ __forceinline__ void fused2_body(const Fused2Job<T>& J, int bid, unsigned tid) {
  static_assert(NT >= TX * TY && NT % 64 == 0, "one thread per tile node at least");
  // every pointer of the job addresses device memory (see gmem)
  const gmem<const OpConsts>* __restrict__ oc = (const gmem<const OpConsts>*)J.oc;
  const gmem<const int>* __restrict__ node_op = (const gmem<const int>*)J.node_op;
  const gmem<const T>* __restrict__ nsten = (const gmem<const T>*)J.nsten;
  const gmem<const int>* __restrict__ extra = (const gmem<const int>*)J.extra;
  const gmem<const int>* __restrict__ node_class = (const gmem<const int>*)J.node_class;
  const T* __restrict__ Zcls = J.Zcls;  // read through the constant space (regular_apply)
  const gmem<const T>* __restrict__ Zirr = (const gmem<const T>*)J.Zirr;
  const gmem<const T>* __restrict__ x_in = (const gmem<const T>*)J.x_in;
  const gmem<const T>* __restrict__ b = (const gmem<const T>*)J.b;
  gmem<T>* __restrict__ x_out = (gmem<T>*)J.x_out;
  const gmem<const T>* __restrict__ xc = (const gmem<const T>*)J.xc;
  const T omega = J.omega;
  const int ntx = J.ntx, nty = J.nty, mode = J.mode;
  constexpr int XW = TX + 6, XH = TY + 6, XP = XW * XH;  // x tile, halo 3
  constexpr int RW = TX + 4, RH = TY + 4, RP = RW * RH;  // residual tile, halo 2
  constexpr int ZSP = PT<2>::ZSP;
  constexpr int NRES = (RP + NT - 1) / NT;                // residual nodes per thread
  __shared__ T xs[3 * XP];
  __shared__ T rs[3 * RP];
  __shared__ StoredList2<NT, NRES> sl;                    // residual nodes with a stored stencil
  constexpr int NWO = (TX * TY + 63) / 64;               // wavefronts that own tile nodes
  constexpr int NG = NT / 16;                             // 16-lane groups of the workgroup
  __shared__ int irr_tid[NWO * 64], irr_pidx[NWO * 64];
  __shared__ int irr_wcnt[NWO];
  const int n = oc->n;
  const int m = n + 1;
  const int64_t N = (int64_t)m * m;
  // Workgroups 0 .. n_extra-1 are the extra parts of tiles with more than CAP individual patches
  // (code tile * 4 + part, set-up): the longest-running workgroups, dispatched first. The rest are
  // part 0 of every tile, in runs of 4 tiles per XCD.
  int tile_lin, part = 0;
  if (bid >= J.n_extra) {
    const int nt[3] = {ntx, nty, 1};
    int t[3];
    tile_coords<2, 4>(bid - J.n_extra, nt, t);
    tile_lin = t[0] + ntx * t[1];
  } else {
    const int code = extra[bid];
    tile_lin = code >> 2;
    part = code & 3;
  }
  const int bx = (tile_lin % ntx) * TX, by = (tile_lin / ntx) * TY;
  // every global load that depends on no other one is issued before the first LDS store: the own
  // patch class, the x tile, and the operator code and b of this thread's residual nodes
  const int tx0 = tid % TX, ty0 = tid / TX;
  const bool inside0 = tid < TX * TY && bx + tx0 < m && by + ty0 < m;
  const int cls = inside0 ? node_class[(bx + tx0) + (int64_t)m * (by + ty0)] : -1;
  constexpr int NXL = (3 * XP + NT - 1) / NT;
  T xv[NXL];
#pragma unroll
  for (int k = 0; k < NXL; ++k) {
    const int e = tid + NT * k;
    const int f = e / XP, p = e % XP;
    const int gx = bx - 3 + p % XW, gy = by - 3 + p / XW;
    const bool ok = e < 3 * XP && gx >= 0 && gx < m && gy >= 0 && gy < m;
    xv[k] = (ok && mode != 1) ? x_in[f * N + gx + (int64_t)m * gy] : T(0);
  }
  // mode 2: the coarse nodes the x tile interpolates from (CW x CH from coarse node (cx0, cy0)),
  // loaded with the x tile and staged in the residual buffer, which is free until the residual
  constexpr int CW = XW / 2 + 2, CH = XH / 2 + 2, CP = CW * CH;
  constexpr int NCL = (3 * CP + NT - 1) / NT;
  static_assert(CP <= RP, "the coarse tile fits in the residual buffer");
  const int nc = n >> 1, mc = nc + 1;
  const int64_t Nc = (int64_t)mc * mc;
  const int cx0 = (bx - 3) >> 1, cy0 = (by - 3) >> 1;
  T cv[NCL];
  if (mode == 2)
#pragma unroll
    for (int k = 0; k < NCL; ++k) {
      const int e = tid + NT * k;
      const int f = e / CP, p = e % CP;
      const int gx = cx0 + p % CW, gy = cy0 + p / CW;
      cv[k] = (e < 3 * CP && gx >= 0 && gx < mc && gy >= 0 && gy < mc) ? xc[f * Nc + gx + (int64_t)mc * gy] : T(0);
    }
  int opv[NRES];
  T bvv[NRES][3];
#pragma unroll
  for (int k = 0; k < NRES; ++k) {
    const int e = tid + NT * k;
    const int cx = bx - 2 + e % RW, cy = by - 2 + e / RW;
    const bool ok = e < RP && cx >= 0 && cx < m && cy >= 0 && cy < m;
    const int64_t g = cx + (int64_t)m * cy;
    opv[k] = ok ? node_op[g] : -1;
#pragma unroll
    for (int f = 0; f < 3; ++f) bvv[k][f] = ok ? b[f * N + g] : T(0);
  }
  if (mode == 2) {
#pragma unroll
    for (int k = 0; k < NCL; ++k)
      if (tid + NT * k < 3 * CP) rs[tid + NT * k] = cv[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NXL; ++k) {
      const int e = tid + NT * k;
      const int f = e / XP, p = e % XP;
      const int c[3] = {bx - 3 + p % XW, by - 3 + p / XW, 0};
      if (e < 3 * XP && c[0] >= 0 && c[0] < m && c[1] >= 0 && c[1] < m)
        xv[k] += prolong_sum<2, T>(c, [&](const int* cc) { return rs[f * CP + (cc[0] - cx0) + CW * (cc[1] - cy0)]; });
    }
  }
#pragma unroll
  for (int k = 0; k < NXL; ++k)
    if (tid + NT * k < 3 * XP) xs[tid + NT * k] = xv[k];
  // nodes with a stored stencil are listed; groups of lanes compute their residuals
#pragma unroll
  for (int k = 0; k < NRES; ++k) stored_list_add<NT, NRES>(sl, k, tid + NT * k, opv[k], tid);
  __syncthreads();
  // residuals: nodes with a reference stencil per thread, while the stored rows load
  constexpr int LPN = TX * TY >= 256 ? 8 : (TX * TY >= 32 ? 4 : 2);  // lanes per stored row
  stored_rows_group2<NT, NRES, RW, RP, XW, XP, LPN, T>(sl, nsten, b, N, m, bx - 2, by - 2, xs, rs, [&] {
#pragma unroll
    for (int k = 0; k < NRES; ++k) {
      const int e = tid + NT * k;
      if (e < RP && opv[k] < 0) {
        const int px = e % RW, py = e / RW;
        const int cx = bx - 2 + px, cy = by - 2 + py;
        T rv[3] = {0, 0, 0};
        if (cx >= 0 && cx < m && cy >= 0 && cy < m) {
          const T* bv = bvv[k];
          const int xb = (px + 1) + XW * (py + 1);
          T acc[3] = {0, 0, 0};
          ref_row_apply<2, true, T>((const double*)oc->pack, opv[k],
                                    [&](int f, const int* o) { return xs[f * XP + xb + o[0] + XW * o[1]]; }, acc);
#pragma unroll
          for (int f = 0; f < 3; ++f) rv[f] = bv[f] - acc[f];
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) rs[f * RP + e] = rv[f];
      }
    }
  }, tid);
  __syncthreads();
  const int tx = tx0, ty = ty0;
  const bool inside = inside0;
  const int64_t node = (bx + tx) + (int64_t)m * (by + ty);
  const int rbase = (tx + 2) + RW * (ty + 2);
  T y[3] = {0, 0, 0};
  const int cls_reg = part == 0 ? cls : -1;  // regular patches belong to part 0
  regular_apply<2, true, T>(Zcls, cls_reg, [&](int f, const int* o) { return rs[f * RP + rbase + o[0] + RW * o[1]]; }, y);
  if (cls_reg >= 0) {
    const int xb = (tx + 3) + XW * (ty + 3);
#pragma unroll
    for (int f = 0; f < 3; ++f) x_out[f * N + node] = xs[f * XP + xb] + omega * y[f];
  }
  // Individual patches of the tile, listed in LDS in node order (one segment per wavefront, so
  // every part of a tile sees the same list); part p takes entries [p CAP, (p + 1) CAP), which
  // 16-lane groups process two patches at a time.
  if (tid < NWO * 64) {
    const bool irr = inside && cls < 0;
    const unsigned long long mask = __ballot(irr);
    const int pos = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0));
    if (irr) {
      irr_tid[(tid & ~63) + pos] = tid;
      irr_pidx[(tid & ~63) + pos] = -cls - 1;
    }
    if ((tid & 63) == 0) irr_wcnt[tid >> 6] = __popcll(mask);
  }
  __syncthreads();
  int pre[NWO + 1];
  pre[0] = 0;
#pragma unroll
  for (int w = 0; w < NWO; ++w) pre[w + 1] = pre[w] + irr_wcnt[w];
  const int cnt = pre[NWO];
  auto slot = [&](int e) {
    int w = 0;
#pragma unroll
    for (int k = 1; k < NWO; ++k) w += e >= pre[k] ? 1 : 0;
    return w * 64 + e - pre[w];
  };
  const int lo = part * CAP, hi = min(cnt, lo + CAP);
  const int j16 = tid & 15;
  for (int ea = lo + (tid >> 4); ea < hi; ea += 2 * NG) {
    const int eb = ea + NG;
    const bool has_b = eb < hi;
    const int sa = slot(ea), sb = has_b ? slot(eb) : sa;
    const int ta = irr_tid[sa], tb = irr_tid[sb];
    const int rba = (ta % TX + 2) + RW * (ta / TX + 2), rbb = (tb % TX + 2) + RW * (tb / TX + 2);
    T acca[3], accb[3];
    irregular_pair<2, T>(Zirr + (int64_t)irr_pidx[sa] * 3 * ZSP, Zirr + (int64_t)irr_pidx[sb] * 3 * ZSP,
                      has_b, j16, [&](int field, const int* o) { return rs[field * RP + rba + o[0] + RW * o[1]]; },
                      [&](int field, const int* o) { return rs[field * RP + rbb + o[0] + RW * o[1]]; }, acca, accb);
    if (j16 < 3) {
      const T va = j16 == 0 ? acca[0] : (j16 == 1 ? acca[1] : acca[2]);
      const T vb = j16 == 0 ? accb[0] : (j16 == 1 ? accb[1] : accb[2]);
      x_out[j16 * N + (bx + ta % TX) + (int64_t)m * (by + ta / TX)] =
          xs[j16 * XP + (ta % TX + 3) + XW * (ta / TX + 3)] + omega * va;
      if (has_b)
        x_out[j16 * N + (bx + tb % TX) + (int64_t)m * (by + tb / TX)] =
            xs[j16 * XP + (tb % TX + 3) + XW * (tb / TX + 3)] + omega * vb;
    }
  }
}

template <int TX, int TY, int NT, int WPE, class T>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
sweep_fused2_kernel(Fused2Job<T> J) {
  fused2_body<TX, TY, NT, fused2_part_cap(Fused2Shape{TX, TY, NT}), T>(J, (int)blockIdx.x, threadIdx.x);
}

// Stacked form: nrhs vectors of one level (x_in, b and x_out sv elements apart, xc sc apart) in one
// launch, blockIdx.y the vector: the workgroups of all vectors fill the chip together instead of one
// launch after another. Per vector the arithmetic is that of sweep_fused2_kernel.
template <int TX, int TY, int NT, int WPE, class T>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
sweep_fused2_multi_kernel(Fused2Job<T> J, int64_t sv, int64_t sc) {
  const int64_t k = blockIdx.y;
  J.x_in += k * sv;
  J.b += k * sv;
  J.x_out += k * sv;
  if (J.xc) J.xc += k * sc;
  fused2_body<TX, TY, NT, fused2_part_cap(Fused2Shape{TX, TY, NT}), T>(J, (int)blockIdx.x, threadIdx.x);
}

// Batched form: the workgroups of several jobs (levels of independent problems) in one launch;
// block_job maps a workgroup to its job, whose workgroups start at job.block0. There are no extra
// parts: one part holds the whole tile.
template <int TX, int TY, int NT, int WPE, class T>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
sweep_fused2_batch_kernel(const Fused2Job<T>* __restrict__ jobs, const int* __restrict__ block_job) {
  const Fused2Job<T> J = jobs[block_job[blockIdx.x]];
  fused2_body<TX, TY, NT, TX * TY, T>(J, (int)blockIdx.x - J.block0, threadIdx.x);
}

// Persistent form of the batched launch: as many workgroups as the chip holds at once, workgroup w
// taking tiles w, w + G, w + 2G, ... (G workgroups) in turn. Consecutive tiles go to consecutive
// workgroups, and so to the XCDs in the same round-robin order as the one-tile-per-workgroup launch.
// Every tile is taken exactly once and its arithmetic is that of that launch. (Handing out tiles by
// an atomic ticket instead serialises on the one counter: about 11 ns per ticket, three times the
// batched cycle's time.)
template <int TX, int TY, int NT, int WPE, class T>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
sweep_fused2_batch_persistent_kernel(const Fused2Job<T>* __restrict__ jobs, const int* __restrict__ block_job,
                                     int nblocks) {
  for (int blk = (int)blockIdx.x; blk < nblocks; blk += (int)gridDim.x) {
    // the thread index, opaque to the compiler: nothing derived from it is hoisted out of the loop,
    // where it would stay live across every tile and spill
    unsigned tid;
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(threadIdx.x));
    const Fused2Job<T> J = jobs[block_job[blk]];
    fused2_body<TX, TY, NT, TX * TY, T>(J, blk - J.block0, tid);
    // every thread is done with this tile's LDS before the next tile's stores
    __syncthreads();
  }
}



// Extra workgroups of the fused 2D sweep: tiles whose individual patches exceed one part
// (fused2_part_cap) get parts 1, 2, 3 (code tile * 4 + part), dispatched before the part-0 workgroups
// of all tiles.
void plan_fused2(const Level& L, const std::vector<int>& node_class, std::vector<int>& extra) {
  const Fused2Shape sh = level_fused2_shape(L);
  const int m = L.n + 1;
  const int ntx = (m + sh.tx - 1) / sh.tx, nty = (m + sh.ty - 1) / sh.ty;
  const int cap = fused2_part_cap(sh);
  extra.clear();
  for (int ty = 0; ty < nty; ++ty)
    for (int tx = 0; tx < ntx; ++tx) {
      int cnt = 0;
      for (int j = 0; j < sh.ty; ++j)
        for (int i = 0; i < sh.tx; ++i) {
          const int x = tx * sh.tx + i, y = ty * sh.ty + j;
          if (x < m && y < m && node_class[x + (int64_t)m * y] < 0) ++cnt;
        }
      for (int p = 1; p * cap < cnt; ++p) extra.push_back((tx + ntx * ty) * 4 + p);
    }
}

constexpr int64_t kRolledRegularNodes = 100000;

template <int D, class T>
hipError_t k_apply_regular(const Ctx& c, const Level& L, const T* r, T* x, hipStream_t s, int nrhs, int64_t sv) {
  if (L.n_classes == 0) return hipSuccess;
  int nt[3];
  tile_grid<D>(L.n, nt);
  const dim3 grid((unsigned)(nt[0] * nt[1] * nt[2]), (unsigned)nrhs);
  // 3D grids from kRolledRegularNodes nodes on: the rolled loop (occupancy over instruction count);
  // smaller levels, one short chain per workgroup, keep the unrolled one
  if constexpr (D == 3) {
    if (L.N >= kRolledRegularNodes) {
      apply_regular_kernel<D, false, T><<<grid, dim3(256), 0, s>>>(L.n, nt[0], nt[1], nt[2], L.node_class,
                                                                   LV<T>::Zcls(L), r, x, (T)c.prm.omega, sv);
      return hipGetLastError();
    }
  }
  apply_regular_kernel<D, true, T><<<grid, dim3(256), 0, s>>>(L.n, nt[0], nt[1], nt[2], L.node_class, LV<T>::Zcls(L),
                                                              r, x, (T)c.prm.omega, sv);
  return hipGetLastError();
}

template <int D, class T>
hipError_t k_apply_irregular(const Ctx& c, const Level& L, const T* r, T* x, hipStream_t s) {
  if (L.n_irr == 0) return hipSuccess;
  int64_t nb = (L.n_irr + 31) / 32;
  if (nb > 65536) nb = 65536;
  apply_irregular_kernel<D, T><<<dim3((unsigned)nb), dim3(256), 0, s>>>(L.n, L.n_irr, L.irr_nodes, L.irr_zrow,
                                                                        LV<T>::Zirr(L),
                                                                        r, x, (T)c.prm.omega);
  return hipGetLastError();
}

template <int TX, int TY, int NT, int WPE, class T>
hipError_t launch_fused2(const Ctx& c, const Level& L, const T* x_in, const T* b, T* x_out,
                         int mode, const T* xc, hipStream_t s) {
  const int ntx = (L.n + 1 + TX - 1) / TX, nty = (L.n + 1 + TY - 1) / TY;
  const Fused2Job<T> J{L.consts, L.node_op,    LV<T>::nsten(L), L.fused_extra, (int)L.n_fused_extra,
                       L.node_class,   LV<T>::Zcls(L), LV<T>::Zirr(L), x_in,          b,
                       x_out,          xc,             (T)c.prm.omega,  ntx,           nty,
                       mode,           0};
  sweep_fused2_kernel<TX, TY, NT, WPE, T><<<dim3((unsigned)(ntx * nty + L.n_fused_extra)), dim3(NT), 0, s>>>(J);
  return hipGetLastError();
}

template <class T>
hipError_t k_sweep_fused2(const Ctx& c, const Level& L, const T* x_in, const T* b, T* x_out, int mode, const T* xc,
                          hipStream_t s) {
  constexpr Fused2Shape B = kFusedBig, M = kFusedMid, S = kFusedSmall;
  if (L.fshape >= 0) {
#define FCG_FUSED_CASE(k)                                                                                  \
  case k:                                                                                                  \
    return launch_fused2<kFusedShapes[k].tx, kFusedShapes[k].ty, kFusedShapes[k].nt, kFusedShapes[k].wpe, T>( \
        c, L, x_in, b, x_out, mode, xc, s);
    static_assert(kNumFusedShapes == 8, "one case per shape");
    switch (L.fshape) {
      FCG_FUSED_CASE(0)
      FCG_FUSED_CASE(1)
      FCG_FUSED_CASE(2)
      FCG_FUSED_CASE(3)
      FCG_FUSED_CASE(4)
      FCG_FUSED_CASE(5)
      FCG_FUSED_CASE(6)
      default: FCG_FUSED_CASE(7)
    }
#undef FCG_FUSED_CASE
  }
  if (L.N >= kFusedBigTileNodes) return launch_fused2<B.tx, B.ty, B.nt, B.wpe, T>(c, L, x_in, b, x_out, mode, xc, s);
  if (L.N >= kFusedMidTileNodes) return launch_fused2<M.tx, M.ty, M.nt, M.wpe, T>(c, L, x_in, b, x_out, mode, xc, s);
  return launch_fused2<S.tx, S.ty, S.nt, S.wpe, T>(c, L, x_in, b, x_out, mode, xc, s);
}

template <int TX, int TY, int NT, int WPE>
hipError_t launch_fused2_multi(const Ctx& c, const Level& L, const double* x_in, const double* b, double* x_out,
                               int mode, const double* xc, int nrhs, int64_t sv, int64_t sc, hipStream_t s) {
  const int ntx = (L.n + 1 + TX - 1) / TX, nty = (L.n + 1 + TY - 1) / TY;
  const Fused2Job<double> J{L.consts, L.node_op, L.nsten, L.fused_extra, (int)L.n_fused_extra,
                            L.node_class, L.Zcls, L.Zirr, x_in, b, x_out, xc, c.prm.omega, ntx, nty, mode, 0};
  sweep_fused2_multi_kernel<TX, TY, NT, WPE, double>
      <<<dim3((unsigned)(ntx * nty + L.n_fused_extra), (unsigned)nrhs), dim3(NT), 0, s>>>(J, sv, sc);
  return hipGetLastError();
}

// Levels from this many nodes on take one fused launch per stacked vector: one vector's workgroups
// already fill the chip many times over there (4096^2 sweep of 8 vectors 4.49 ms one by one, 4.67 ms
// stacked).
constexpr int64_t kFusedStackMaxNodes = int64_t(1) << 21;

// One fused sweep of nrhs stacked vectors (FP64): one launch of the level's default tile shape for
// all vectors; a level with an autotuned shape, or a very large one, takes one launch per vector.
hipError_t k_sweep_fused2_multi(const Ctx& c, const Level& L, const double* x_in, const double* b, double* x_out,
                                int mode, const double* xc, int nrhs, int64_t sv, int64_t sc, hipStream_t s) {
  if (L.fshape >= 0 || L.N >= kFusedStackMaxNodes) {
    for (int k = 0; k < nrhs; ++k) {
      const hipError_t e =
          k_sweep_fused2<double>(c, L, x_in + k * sv, b + k * sv, x_out + k * sv, mode, xc ? xc + k * sc : nullptr, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  constexpr Fused2Shape B = kFusedBig, M = kFusedMid, S = kFusedSmall;
  if (L.N >= kFusedBigTileNodes)
    return launch_fused2_multi<B.tx, B.ty, B.nt, B.wpe>(c, L, x_in, b, x_out, mode, xc, nrhs, sv, sc, s);
  if (L.N >= kFusedMidTileNodes)
    return launch_fused2_multi<M.tx, M.ty, M.nt, M.wpe>(c, L, x_in, b, x_out, mode, xc, nrhs, sv, sc, s);
  return launch_fused2_multi<S.tx, S.ty, S.nt, S.wpe>(c, L, x_in, b, x_out, mode, xc, nrhs, sv, sc, s);
}

// Residual and restriction in one pass (2D, V-cycle): b_c = P^T (b - L x) for a TXC x TYC tile of
// coarse nodes. The fine residual of the (2 TXC + 1) x (2 TYC + 1) nodes the tile gathers from is
// computed into LDS from an x tile with halo 1; arithmetic and summation order are those of the
// residual and restriction kernels.
template <int TXC, int TYC, int NT, class T>
__device__ __forceinline__ void residual_restrict2_body(const RR2Job<T>& J, int bid) {
  static_assert(NT >= TXC * TYC && NT % 64 == 0, "one thread per coarse node at least");
  // every pointer of the job addresses device memory (see gmem)
  const gmem<const OpConsts>* __restrict__ oc = (const gmem<const OpConsts>*)J.oc;
  const gmem<const int>* __restrict__ node_op = (const gmem<const int>*)J.node_op;
  const gmem<const T>* __restrict__ nsten = (const gmem<const T>*)J.nsten;
  const gmem<const T>* __restrict__ x = (const gmem<const T>*)J.x;
  const gmem<const T>* __restrict__ b = (const gmem<const T>*)J.b;
  gmem<T>* __restrict__ bc = (gmem<T>*)J.bc;
  const int ntx = J.ntx, nty = J.nty;
  constexpr int RW = 2 * TXC + 1, RH = 2 * TYC + 1, RP = RW * RH;  // fine residual region
  constexpr int XW = RW + 2, XH = RH + 2, XP = XW * XH;            // x region, halo 1
  constexpr int NRES = (RP + NT - 1) / NT, NXL = (3 * XP + NT - 1) / NT;
  __shared__ T xs[3 * XP];
  __shared__ T rs[3 * RP];
  __shared__ StoredList2<NT, NRES> sl;  // residual nodes with a stored stencil
  const int n = oc->n;
  const int m = n + 1;
  const int64_t N = (int64_t)m * m;
  const int mc = (n >> 1) + 1;
  const int64_t Nc = (int64_t)mc * mc;
  const int nt[3] = {ntx, nty, 1};
  int t[3];
  tile_coords<2>(bid, nt, t);
  const int cx0 = t[0] * TXC, cy0 = t[1] * TYC;
  const int fx0 = 2 * cx0 - 1, fy0 = 2 * cy0 - 1;  // fine coordinates of residual-region entry 0
  T xv[NXL];
#pragma unroll
  for (int k = 0; k < NXL; ++k) {
    const int e = threadIdx.x + NT * k;
    const int f = e / XP, p = e % XP;
    const int gx = fx0 - 1 + p % XW, gy = fy0 - 1 + p / XW;
    xv[k] = (e < 3 * XP && gx >= 0 && gx < m && gy >= 0 && gy < m) ? x[f * N + gx + (int64_t)m * gy] : T(0);
  }
  int opv[NRES];
  T bv[NRES][3];
#pragma unroll
  for (int k = 0; k < NRES; ++k) {
    const int e = threadIdx.x + NT * k;
    const int gx = fx0 + e % RW, gy = fy0 + e / RW;
    const bool ok = e < RP && gx >= 0 && gx < m && gy >= 0 && gy < m;
    const int64_t g = gx + (int64_t)m * gy;
    opv[k] = ok ? node_op[g] : -1;
#pragma unroll
    for (int f = 0; f < 3; ++f) bv[k][f] = ok ? b[f * N + g] : T(0);
  }
#pragma unroll
  for (int k = 0; k < NXL; ++k)
    if (threadIdx.x + NT * k < 3 * XP) xs[threadIdx.x + NT * k] = xv[k];
  // nodes with a stored stencil are listed; groups of lanes compute their residuals
#pragma unroll
  for (int k = 0; k < NRES; ++k) stored_list_add<NT, NRES>(sl, k, threadIdx.x + NT * k, opv[k], threadIdx.x);
  __syncthreads();
  // residuals: nodes with a reference stencil per thread, while the stored rows load
  constexpr int LPN = TXC * TYC >= 128 ? 8 : 2;  // lanes per stored row
  stored_rows_group2<NT, NRES, RW, RP, XW, XP, LPN, T>(sl, nsten, b, N, m, fx0, fy0, xs, rs, [&] {
#pragma unroll
    for (int k = 0; k < NRES; ++k) {
      const int e = threadIdx.x + NT * k;
      if (e < RP && opv[k] < 0) {
        const int px = e % RW, py = e / RW;
        const int gx = fx0 + px, gy = fy0 + py;
        T rv[3] = {0, 0, 0};
        if (gx >= 0 && gx < m && gy >= 0 && gy < m) {
          const int xb = (px + 1) + XW * (py + 1);
          T acc[3] = {0, 0, 0};
          ref_row_apply<2, true, T>((const double*)oc->pack, opv[k], [&](int f, const int* o) { return xs[f * XP + xb + o[0] + XW * o[1]]; },
                                    acc);
#pragma unroll
          for (int f = 0; f < 3; ++f) rv[f] = bv[k][f] - acc[f];
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) rs[f * RP + e] = rv[f];
      }
    }
  }, threadIdx.x);
  __syncthreads();
  if (threadIdx.x >= TXC * TYC) return;
  const int cx = cx0 + threadIdx.x % TXC, cy = cy0 + threadIdx.x / TXC;
  if (cx >= mc || cy >= mc) return;
  T acc[3] = {0, 0, 0};
  for (int o = 0; o < 9; ++o) {
    const int ox = o % 3 - 1, oy = o / 3 - 1;
    const int gx = 2 * cx + ox, gy = 2 * cy + oy;
    if (gx < 0 || gx > n || gy < 0 || gy > n) continue;
    T w = 1;
    if (ox != 0) w *= 0.5;
    if (oy != 0) w *= 0.5;
    const int e = (gx - fx0) + RW * (gy - fy0);
#pragma unroll
    for (int f = 0; f < 3; ++f) acc[f] += w * rs[f * RP + e];
  }
  const int64_t cn = cx + (int64_t)mc * cy;
#pragma unroll
  for (int f = 0; f < 3; ++f) bc[f * Nc + cn] = acc[f];
}

template <int TXC, int TYC, int NT, class T>
__global__ void __launch_bounds__(NT) residual_restrict2_kernel(RR2Job<T> J) {
  residual_restrict2_body<TXC, TYC, NT, T>(J, (int)blockIdx.x);
}

template <int TXC, int TYC, int NT, class T>
__global__ void __launch_bounds__(NT) residual_restrict2_batch_kernel(const RR2Job<T>* __restrict__ jobs,
                                                                      const int* __restrict__ block_job) {
  const RR2Job<T> J = jobs[block_job[blockIdx.x]];
  residual_restrict2_body<TXC, TYC, NT, T>(J, (int)blockIdx.x - J.block0);
}

// Stacked form: nrhs vectors (x and b sv apart, bc sc apart), blockIdx.y the vector.
template <int TXC, int TYC, int NT, class T>
__global__ void __launch_bounds__(NT) residual_restrict2_multi_kernel(RR2Job<T> J, int64_t sv, int64_t sc) {
  const int64_t k = blockIdx.y;
  J.x += k * sv;
  J.b += k * sv;
  J.bc += k * sc;
  residual_restrict2_body<TXC, TYC, NT, T>(J, (int)blockIdx.x);
}

template <int TXC, int TYC, int NT, class T>
hipError_t launch_residual_restrict2(const Level& F, const T* x, const T* b, T* bc, hipStream_t s, int nrhs = 1,
                                     int64_t sv = 0, int64_t sc = 0) {
  const int mc = (F.n >> 1) + 1;
  const int ntx = (mc + TXC - 1) / TXC, nty = (mc + TYC - 1) / TYC;
  const RR2Job<T> J{F.consts, F.node_op, LV<T>::nsten(F), x, b, bc, ntx, nty, 0};
  if (nrhs > 1)
    residual_restrict2_multi_kernel<TXC, TYC, NT, T>
        <<<dim3((unsigned)(ntx * nty), (unsigned)nrhs), dim3(NT), 0, s>>>(J, sv, sc);
  else
    residual_restrict2_kernel<TXC, TYC, NT, T><<<dim3((unsigned)(ntx * nty)), dim3(NT), 0, s>>>(J);
  return hipGetLastError();
}

template <class T>
hipError_t k_residual_restrict2(const Ctx&, const Level& F, const T* x, const T* b, T* bc, hipStream_t s) {
  if (F.N >= kFusedBigTileNodes) return launch_residual_restrict2<16, 8, 256, T>(F, x, b, bc, s);
  if (F.N >= kFusedMidTileNodes) return launch_residual_restrict2<8, 4, 128, T>(F, x, b, bc, s);
  return launch_residual_restrict2<4, 4, 128, T>(F, x, b, bc, s);
}

// The fused residual + restriction of nrhs stacked vectors (FP64; x, b sv apart, bc sc apart) in one
// launch.
hipError_t k_residual_restrict2_multi(const Level& F, const double* x, const double* b, double* bc, int nrhs,
                                      int64_t sv, int64_t sc, hipStream_t s) {
  if (F.N >= kFusedBigTileNodes) return launch_residual_restrict2<16, 8, 256, double>(F, x, b, bc, s, nrhs, sv, sc);
  if (F.N >= kFusedMidTileNodes) return launch_residual_restrict2<8, 4, 128, double>(F, x, b, bc, s, nrhs, sv, sc);
  return launch_residual_restrict2<4, 4, 128, double>(F, x, b, bc, s, nrhs, sv, sc);
}

// ---- batched launches (independent 2D problems, one launch per V-cycle step) -------------------
// One tile shape for every job of a batched launch: 8 x 4 tiles by 128 threads (the arithmetic of a
// node does not depend on the shape, so the results equal those of the single-problem launches).
constexpr int kBatchTX = 8, kBatchTY = 4, kBatchNT = 128;

int batch_fused2_blocks(const Level& L) {
  const int m = L.n + 1;
  return ((m + kBatchTX - 1) / kBatchTX) * ((m + kBatchTY - 1) / kBatchTY);
}

Fused2Job<double> batch_fused2_job(const Ctx& c, const Level& L, const double* x_in, const double* b, double* x_out,
                                   int mode, const double* xc) {
  const int m = L.n + 1;
  // no extra parts in a batched launch: one part holds the whole tile
  return Fused2Job<double>{L.consts, L.node_op, L.nsten, nullptr, 0, L.node_class, L.Zcls, L.Zirr, x_in, b, x_out, xc,
                           c.prm.omega, (m + kBatchTX - 1) / kBatchTX, (m + kBatchTY - 1) / kBatchTY, mode, 0};
}

int batch_rr2_blocks(const Level& F) {
  const int mc = (F.n >> 1) + 1;
  return ((mc + kBatchTX - 1) / kBatchTX) * ((mc + kBatchTY - 1) / kBatchTY);
}

RR2Job<double> batch_rr2_job(const Level& F, const double* x, const double* b, double* bc) {
  const int mc = (F.n >> 1) + 1;
  return RR2Job<double>{F.consts, F.node_op, F.nsten, x, b, bc, (mc + kBatchTX - 1) / kBatchTX,
                        (mc + kBatchTY - 1) / kBatchTY, 0};
}

hipError_t k_batch_fused2(const Fused2Job<double>* jobs, const int* block_job, int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  sweep_fused2_batch_kernel<kBatchTX, kBatchTY, kBatchNT, 5, double><<<dim3((unsigned)nblocks), dim3(kBatchNT), 0, s>>>(
      jobs, block_job);
  return hipGetLastError();
}

// Workgroups of the persistent batched sweep that the device holds at once (occupancy per CU times
// CUs), looked up once per device.
int batch_fused2_resident_blocks() {
  // several host threads may ask at once (the solve server's workers); each stores the same value
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  const int known = cache[dev].load(std::memory_order_relaxed);
  if (known > 0) return known;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, sweep_fused2_batch_persistent_kernel<kBatchTX, kBatchTY, kBatchNT, 5, double>, kBatchNT, 0) !=
          hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1 || cus < 1)
    return 0;
  cache[dev].store(per_cu * cus, std::memory_order_relaxed);
  return per_cu * cus;
}

hipError_t k_batch_fused2_persistent(const Fused2Job<double>* jobs, const int* block_job, int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  const int resident = batch_fused2_resident_blocks();
  if (resident < 1) return hipErrorInvalidValue;
  const int grid = nblocks < resident ? nblocks : resident;
  sweep_fused2_batch_persistent_kernel<kBatchTX, kBatchTY, kBatchNT, 5, double>
      <<<dim3((unsigned)grid), dim3(kBatchNT), 0, s>>>(jobs, block_job, nblocks);
  return hipGetLastError();
}

hipError_t k_batch_rr2(const RR2Job<double>* jobs, const int* block_job, int nblocks, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  residual_restrict2_batch_kernel<kBatchTX, kBatchTY, kBatchNT, double>
      <<<dim3((unsigned)nblocks), dim3(kBatchNT), 0, s>>>(jobs, block_job);
  return hipGetLastError();
}

}  // namespace fcg
