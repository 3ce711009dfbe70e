// The coarse end of the V-cycle in one kernel (Sec. 3 V-cycle; smoother of Eq. 14-15 in the
// cache_inverse form). Levels 0..top are small enough for one workgroup of 1024 threads whose LDS
// holds x, b and r of all of them: every sweep, residual, restriction, coarsest solve and
// prolongation of those levels runs back to back inside the workgroup, separated by workgroup
// barriers, with no kernel launch between the dependent steps. Only the read-only level data
// (cell kinds, cut-cell integrals, patch classes and rows, coarsest inverse) come from memory.
// The per-node arithmetic is the same code as in the per-level kernels, so the results are
// identical to running the levels one kernel at a time.
//
// Included by fcgmg_kernels.hip.

namespace fcg {

namespace {

constexpr int kTailThreads = 1024;
constexpr int kTailMaxLevels = 6;

template <int D>
__device__ __forceinline__ int64_t tail_nodes(int n) {
  const int64_t m = n + 1;
  return D == 2 ? m * m : m * m * m;
}

// r = b - L x on one level (thread per node); X, B, R point into LDS.
template <int D>
__device__ void tail_residual(const TailLevel& T, const RefMats<D>& rm, const double* X, const double* B, double* R,
                              double alpha_f) {
  constexpr int NEL = PT<D>::NEL;
  const int n = T.n, m = n + 1;
  const int N = (int)tail_nodes<D>(n);
  for (int node = threadIdx.x; node < N; node += kTailThreads) {
    const int c[3] = {node % m, (node / m) % m, D == 3 ? node / (m * m) : 0};
    double acc[D + 1];
#pragma unroll
    for (int f = 0; f <= D; ++f) acc[f] = 0;
    node_apply<D, false>(
        rm, [&](const int* cc) { return T.cell_info[D == 2 ? cc[0] + n * cc[1] : cc[0] + n * (cc[1] + n * cc[2])]; },
        [&](const int*, int info) -> const double* { return T.cut + (int64_t)info * NEL; }, alpha_f, n, c,
        [&](int f, const int* o) {
          const int j = D == 2 ? (c[0] + o[0]) + m * (c[1] + o[1]) : (c[0] + o[0]) + m * ((c[1] + o[1]) + m * (c[2] + o[2]));
          return X[f * N + j];
        },
        acc);
#pragma unroll
    for (int f = 0; f <= D; ++f) R[f * N + node] = B[f * N + node] - acc[f];
  }
}

// x += omega S r on one level (regular and irregular patches), r complete.
template <int D>
__device__ void tail_apply(const TailLevel& T, double* X, const double* R, double omega) {
  constexpr int ZSP = PT<D>::ZSP;
  const int n = T.n, m = n + 1;
  const int N = (int)tail_nodes<D>(n);
  auto rlds = [&](const int* c, int f, const int* o) {
    int cc[3] = {c[0] + o[0], c[1] + o[1], c[2] + o[2]};
    bool in = true;
    for (int k = 0; k < D; ++k) in = in && cc[k] >= 0 && cc[k] < m;
    return in ? R[f * N + (D == 2 ? cc[0] + m * cc[1] : cc[0] + m * (cc[1] + m * cc[2]))] : 0.0;
  };
  // regular patches: every lane of a wavefront runs the same number of rounds (ballots inside)
  const int Npad = (N + kTailThreads - 1) / kTailThreads * kTailThreads;
  for (int node = threadIdx.x; node < Npad; node += kTailThreads) {
    const bool inside = node < N;
    const int cls = inside ? T.node_class[node] : -1;
    const int c[3] = {node % m, (node / m) % m, D == 3 ? node / (m * m) : 0};
    double y[D + 1];
#pragma unroll
    for (int f = 0; f <= D; ++f) y[f] = 0;
    regular_apply<D, false>(T.Zcls, cls, [&](int f, const int* o) { return rlds(c, f, o); }, y);
    if (cls >= 0)
#pragma unroll
      for (int f = 0; f <= D; ++f) X[f * N + node] += omega * y[f];
  }
  // irregular patches: groups of 16 lanes, two patches per group and trip
  const int j16 = threadIdx.x & 15;
  constexpr int NG = kTailThreads / 16;
  for (int64_t pa = threadIdx.x >> 4; pa < T.n_irr; pa += 2 * NG) {
    const int64_t pb = pa + NG;
    const bool has_b = pb < T.n_irr;
    const int na = T.irr_nodes[pa], nbn = has_b ? T.irr_nodes[pb] : na;
    const int ca[3] = {na % m, (na / m) % m, D == 3 ? na / (m * m) : 0};
    const int cb[3] = {nbn % m, (nbn / m) % m, D == 3 ? nbn / (m * m) : 0};
    double acca[D + 1], accb[D + 1];
    irregular_pair<D>(T.Zirr + pa * (int64_t)(D + 1) * ZSP, T.Zirr + (has_b ? pb : pa) * (int64_t)(D + 1) * ZSP,
                      has_b, j16, [&](int f, const int* o) { return rlds(ca, f, o); },
                      [&](int f, const int* o) { return rlds(cb, f, o); }, acca, accb);
    if (j16 <= D) {
      double va = acca[0], vb = accb[0];
#pragma unroll
      for (int f = 1; f <= D; ++f)
        if (j16 == f) {
          va = acca[f];
          vb = accb[f];
        }
      X[j16 * N + na] += omega * va;
      if (has_b) X[j16 * N + nbn] += omega * vb;
    }
  }
}

template <int D>
__device__ void tail_smooth(const TailLevel& T, const RefMats<D>& rm, double* X, const double* B, double* R,
                            int sweeps, double omega, double alpha_f) {
  for (int s = 0; s < sweeps; ++s) {
    tail_residual<D>(T, rm, X, B, R, alpha_f);
    __syncthreads();
    tail_apply<D>(T, X, R, omega);
    __syncthreads();
  }
}

}  // namespace

// TL[l].lds: offset (in doubles) of level l's x, b, r in the dynamic LDS; each (D+1) N_l long.
template <int D>
__global__ void __launch_bounds__(kTailThreads) tail_vcycle_kernel(const TailLevel* __restrict__ TL, int top,
                                                                  const double* __restrict__ Cinv, int cn, int nu1,
                                                                  int nu2, double omega, double alpha_f) {
  extern __shared__ double smem[];
  __shared__ RefMats<D> rms[kTailMaxLevels];
  for (int l = 0; l <= top; ++l) stage_refmats<D>(TL[l].oc, rms[l]);
  auto Xl = [&](int l) { return smem + TL[l].lds; };
  auto Bl = [&](int l) { return smem + TL[l].lds + (D + 1) * tail_nodes<D>(TL[l].n); };
  auto Rl = [&](int l) { return smem + TL[l].lds + 2 * (D + 1) * tail_nodes<D>(TL[l].n); };
  {
    const int nd = (int)((D + 1) * tail_nodes<D>(TL[top].n));
    for (int i = threadIdx.x; i < nd; i += kTailThreads) {
      Xl(top)[i] = TL[top].x[i];
      Bl(top)[i] = TL[top].b[i];
    }
    __syncthreads();
  }
  for (int l = top; l >= 1; --l) {
    const TailLevel& T = TL[l];
    const TailLevel& C = TL[l - 1];
    tail_smooth<D>(T, rms[l], Xl(l), Bl(l), Rl(l), nu1, omega, alpha_f);
    tail_residual<D>(T, rms[l], Xl(l), Bl(l), Rl(l), alpha_f);
    __syncthreads();
    const int64_t Nf = tail_nodes<D>(T.n), Nc = tail_nodes<D>(C.n);
    double* xc = Xl(l - 1);
    for (int64_t node = threadIdx.x; node < Nc; node += kTailThreads) {
      restrict_node<D>(T.n, Nf, C.n, Nc, Rl(l), Bl(l - 1), node);
      for (int f = 0; f <= D; ++f) xc[f * Nc + node] = 0.0;
    }
    __syncthreads();
  }
  {
    const int lane = threadIdx.x & 63;
    for (int row = threadIdx.x >> 6; row < cn; row += kTailThreads / 64) dense_row(Cinv, cn, Bl(0), Xl(0), row, lane);
    __syncthreads();
  }
  for (int l = 1; l <= top; ++l) {
    const TailLevel& T = TL[l];
    const TailLevel& C = TL[l - 1];
    const int64_t Nf = tail_nodes<D>(T.n), Nc = tail_nodes<D>(C.n);
    for (int64_t node = threadIdx.x; node < Nf; node += kTailThreads)
      prolong_node<D>(T.n, Nf, C.n, Nc, Xl(l - 1), Xl(l), node);
    __syncthreads();
    tail_smooth<D>(T, rms[l], Xl(l), Bl(l), Rl(l), nu2, omega, alpha_f);
  }
  {
    const int nd = (int)((D + 1) * tail_nodes<D>(TL[top].n));
    for (int i = threadIdx.x; i < nd; i += kTailThreads) TL[top].x[i] = Xl(top)[i];
  }
}

template <int D>
hipError_t k_tail_vcycle(const Ctx& c, hipStream_t s) {
  tail_vcycle_kernel<D><<<dim3(1), dim3(kTailThreads), c.tail_lds_bytes, s>>>(
      c.tail, c.tail_top, c.coarse_inv, c.coarse_n, c.prm.nu_pre, c.prm.nu_post, c.prm.omega, c.prm.alpha_fict);
  return hipGetLastError();
}

}  // namespace fcg
