// Energy-network jets on the matrix cores: for every quadrature point,
// N(x) - N(0), grad_x N and the Hessian d2N/dx2 of the input-convex network
// (Sec. 4.2.1; the hidden->hidden products are the dense part of the path).
//
// Per block: one tile of 16 quadrature points; wave w owns neuron tile w in
// every layer, so per-layer quantities (logistic pairs and input Jacobians)
// stay in that wave's registers.  Blocks are small (H/16 waves), so several
// run on a compute unit and one block's matrix products overlap another's
// vector work.  The
// FP64 16x16x4 product returns row (l / 16 + 4 r) of column (l % 16) in
// accumulator r of lane l, so lane l owns neurons nt*16 + l/16 + 4 r.
//   forward : 4 columns per qp -- the activation increment dz = z(x) - z(0)
//             and the three input tangents dz/dx_i;
//   backward: 1 column -- zbar_k = dN/dz_k;
//   Hessian : sum_k J_k^T diag(zbar_k s''(a_k)) J_k, J_k = da_k/dx
// (5 matrix columns per layer instead of the 10 of a forward second-order
// jet).  Hidden weights are read as matrix-core operands straight from a
// lane-ordered copy (one coalesced, cache-resident load per step).
//
// Activations are carried as increments over the reference state x = 0, so
// N(x) - N(0) keeps relative precision (delta_softplus, reference constants
// a0 / s0 / sb0 precomputed per neuron).
#include "device_common.h"
#include "gedmg_internal.h"

namespace gedmg {

typedef double d4_t __attribute__((ext_vector_type(4)));

template <int H, int L>
struct JetCfg {
  static constexpr int NT = H / 16;        // neuron tiles = waves per block
  static constexpr int WAVES = NT;
  static constexpr int QB = 16;            // quadrature points per batch
  static constexpr int QP = QB;            // activation row (doubles)
  static constexpr int Z_DBL = 4 * H * QP;
  static constexpr int X_DBL = QB * 3;
  // backward-pass state of the middle layer (L = 3): the logistic pair of each
  // of a lane's 4 rows, lane-contiguous.  Its input Jacobian is recovered from
  // the tangent activations zeta = s J that are still in the activation buffer.
  static constexpr int ST_DBL = (L > 2 ? L - 2 : 0) * WAVES * 2 * 4 * 64;
  // per-neuron constants of every hidden layer k (a0, s0, sb0 and the three
  // input weights: W0 for k = 0, Wx for k >= 1), then the output weights wz;
  // staged once per block so the tiles read them from LDS instead of memory
  static constexpr int C_DBL = L * 6 * H + H;
  static constexpr int M_DBL = kMathTabDoubles;  // exp / log tables
  static constexpr int LDS_BYTES = 8 * (Z_DBL + X_DBL + ST_DBL + C_DBL + M_DBL);
  static_assert(NT * QB * 10 <= Z_DBL, "reduction buffer aliases the activation buffer");
  static_assert(L <= 3, "the middle-layer Jacobian is recovered from the last activation buffer");
};

// HESS = false: value and gradient only, in reverse mode (1 forward column,
// the activation increment, and 1 adjoint column per layer; the gradient is
// the input weights contracted with the adjoints), writing jet entries 0..3
// and leaving the Hessian entries as they are.
template <int H, int L, bool HESS>
__global__ __launch_bounds__(H * 4, 2) void jet_f64_kernel(JetArgs a) {
  using C = JetCfg<H, L>;
  constexpr int NT = C::NT, QB = C::QB, QP = C::QP, NS = H / 4;
  extern __shared__ double lds[];
  double* Zs = lds;
  double* xs = Zs + C::Z_DBL;
  double* st = xs + C::X_DBL;  // [layer-1][wave][field][row][lane]
  double* cst = st + C::ST_DBL;  // [layer][a0, s0, sb0, w0, w1, w2][neuron], then wz[neuron]
  double* mt = cst + C::C_DBL;   // exp table [64][2], then log table [64][4]
  const double* et = mt;
  const double* lt = mt + 128;
  double* red = Zs;  // reused after the backward pass
  const NetLayout lay = make_layout_hd(3, H, L, 3);
  const double* __restrict__ net = a.net;
  const double* __restrict__ wop = a.wop;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = wave;
  const int li = lane & 15, lg = lane >> 4;
  const int j = li;  // qp column in the batch
  const int nbatch = (a.nq + QB - 1) / QB;
  for (int idx = threadIdx.x; idx < C::C_DBL; idx += blockDim.x) {
    double v;
    if (idx < L * 6 * H) {
      const int k = idx / (6 * H), f = (idx / H) % 6, n = idx % H;
      v = f == 0 ? net[lay.a0 + k * H + n]
        : f == 1 ? net[lay.s0 + k * H + n]
        : f == 2 ? net[lay.sb0 + k * H + n]
        : net[(k == 0 ? lay.W0 : k == 1 ? lay.Wx[1] : lay.Wx[2]) + n * 3 + (f - 3)];
    } else {
      v = net[lay.wz + idx - L * 6 * H];
    }
    cst[idx] = v;
  }
  for (int idx = threadIdx.x; idx < C::M_DBL; idx += blockDim.x) mt[idx] = a.mtab[idx];
  static_assert(QB * 3 <= C::WAVES * 64, "one input value per thread");
  // The next tile's inputs travel in a register of the first QB * 3 threads:
  // requested at the start of a tile, stored to LDS at the start of the next.
  const int xi = threadIdx.x;
  double xnext = 0.0;
  if (xi < QB * 3 && (long)blockIdx.x * QB + xi / 3 < a.nq) xnext = a.x[(long)blockIdx.x * QB * 3 + xi];

  for (int batch = blockIdx.x; batch < nbatch; batch += gridDim.x) {
    const long q0 = (long)batch * QB;
    if (xi < QB * 3) xs[xi] = xnext;
    const long q1 = (long)(batch + gridDim.x) * QB;
    xnext = 0.0;
    if (xi < QB * 3 && q1 + xi / 3 < a.nq) xnext = a.x[q1 * 3 + xi];
    __syncthreads();
    const double x[3] = {xs[j * 3], xs[j * 3 + 1], xs[j * 3 + 2]};

    // Backward-pass state: layer 0's logistic pairs in registers (its input
    // Jacobian is W0), layers 1 .. L-2 in this wave's LDS slice; the last
    // hidden layer's adjoint is wz, known in the forward pass, so its Hessian
    // term is added there and nothing of it is kept.
    double s0r[4], sb0r[4];
    double dz[4], zt[4][3];
    double part[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) part[t] = 0.0;
    double abar[4];
    constexpr bool hess = HESS;

    // layer 1: a_1 = W0 x + b0 (vector ALU)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = nt * 16 + lg + 4 * r;
      const double* c0 = cst + n;
      const double w0 = c0[3 * H], w1 = c0[4 * H], w2 = c0[5 * H];
      const double da = w0 * x[0] + w1 * x[1] + w2 * x[2];
      dz[r] = delta_softplus_tab(da, c0[0], c0[H], c0[2 * H], s0r[r], sb0r[r], et, lt);
      if (HESS) {
        zt[r][0] = s0r[r] * w0;
        zt[r][1] = s0r[r] * w1;
        zt[r][2] = s0r[r] * w2;
      }
      if (L == 1) {
        const double wz = cst[L * 6 * H + n];
        part[0] += wz * dz[r];
        abar[r] = wz * s0r[r];
        if (HESS) {
#pragma unroll
          for (int i = 0; i < 3; ++i) part[1 + i] += wz * zt[r][i];
        } else {
          part[1] += abar[r] * w0;
          part[2] += abar[r] * w1;
          part[3] += abar[r] * w2;
        }
        if (hess) {
          const double c2 = abar[r] * sb0r[r];
          part[4] += c2 * w0 * w0;
          part[5] += c2 * w1 * w1;
          part[6] += c2 * w2 * w2;
          part[7] += c2 * w0 * w1;
          part[8] += c2 * w0 * w2;
          part[9] += c2 * w1 * w2;
        }
      }
    }

#pragma unroll
    for (int k = 1; k < L; ++k) {
      constexpr int NCOL = HESS ? 4 : 1;  // forward columns
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = nt * 16 + lg + 4 * r;
        Zs[n * QP + j] = dz[r];
        if (HESS) {
#pragma unroll
          for (int i = 0; i < 3; ++i) Zs[(1 + i) * H * QP + n * QP + j] = zt[r][i];
        }
      }
      __syncthreads();
      d4_t acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = d4_t{0.0, 0.0, 0.0, 0.0};
      const double* Wk = wop + ((size_t)((k - 1) * 2) * NT + nt) * NS * 64 + lane;
#pragma unroll 8
      for (int s = 0; s < NS; ++s) {
        const double av = Wk[s * 64];
        const int zb = (4 * s + lg) * QP + li;
#pragma unroll
        for (int c = 0; c < NCOL; ++c)
          acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Zs[c * H * QP + zb], acc[c], 0, 0, 0);
      }
      __syncthreads();
      double* stk = st + ((size_t)(k - 1) * NT + nt) * 2 * 4 * 64 + lane;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = nt * 16 + lg + 4 * r;
        const double* ck = cst + k * 6 * H + n;
        const double wx[3] = {ck[3 * H], ck[4 * H], ck[5 * H]};
        const double da = acc[0][r] + wx[0] * x[0] + wx[1] * x[1] + wx[2] * x[2];
        double jk[3];
        if (HESS) {
#pragma unroll
          for (int i = 0; i < 3; ++i) jk[i] = acc[1 + i][r] + wx[i];
        }
        double s_, sb_;
        dz[r] = delta_softplus_tab(da, ck[0], ck[H], ck[2 * H], s_, sb_, et, lt);
        if (HESS) {
#pragma unroll
          for (int i = 0; i < 3; ++i) zt[r][i] = s_ * jk[i];
        }
        if (k == L - 1) {
          const double wz = cst[L * 6 * H + n];
          part[0] += wz * dz[r];
          abar[r] = wz * s_;
          if (HESS) {
#pragma unroll
            for (int i = 0; i < 3; ++i) part[1 + i] += wz * zt[r][i];
          } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) part[1 + i] += abar[r] * wx[i];
          }
          if (hess) {
            const double c2 = abar[r] * sb_;
            part[4] += c2 * jk[0] * jk[0];
            part[5] += c2 * jk[1] * jk[1];
            part[6] += c2 * jk[2] * jk[2];
            part[7] += c2 * jk[0] * jk[1];
            part[8] += c2 * jk[0] * jk[2];
            part[9] += c2 * jk[1] * jk[2];
          }
        } else {
          stk[(0 * 4 + r) * 64] = s_;
          if (HESS) stk[(1 * 4 + r) * 64] = sb_;
        }
      }
    }

    if (!HESS) {
      // reverse sweep for the gradient: zbar_{k-1} = W_k^T abar_k,
      // abar_{k-1} = s_{k-1} zbar_{k-1}, grad += W_x,{k-1}^T abar_{k-1}
#pragma unroll
      for (int k = L - 1; k >= 1; --k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Zs[(nt * 16 + lg + 4 * r) * QP + j] = abar[r];
        __syncthreads();
        d4_t acc = d4_t{0.0, 0.0, 0.0, 0.0};
        const double* Wt = wop + ((size_t)((k - 1) * 2 + 1) * NT + nt) * NS * 64 + lane;
#pragma unroll 8
        for (int s = 0; s < NS; ++s)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Wt[s * 64], Zs[(4 * s + lg) * QP + li], acc, 0, 0, 0);
        __syncthreads();
        const double* stk = st + ((size_t)(k - 2) * NT + nt) * 2 * 4 * 64 + lane;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int n = nt * 16 + lg + 4 * r;
          const double sv = (k - 1 == 0) ? s0r[r] : stk[(0 * 4 + r) * 64];
          abar[r] = acc[r] * sv;
          const double* wcol = cst + (k - 1) * 6 * H + n;  // input weights of layer k-1
#pragma unroll
          for (int i = 0; i < 3; ++i) part[1 + i] += abar[r] * wcol[(3 + i) * H];
        }
      }
    }

    if (hess) {
      // zbar_{k-1} = W_k^T abar_k, then layer k-1's adjoint and Hessian term
#pragma unroll
      for (int k = L - 1; k >= 1; --k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Zs[(nt * 16 + lg + 4 * r) * QP + j] = abar[r];
        __syncthreads();
        d4_t acc = d4_t{0.0, 0.0, 0.0, 0.0};
        const double* Wt = wop + ((size_t)((k - 1) * 2 + 1) * NT + nt) * NS * 64 + lane;
#pragma unroll 8
        for (int s = 0; s < NS; ++s)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Wt[s * 64], Zs[(4 * s + lg) * QP + li], acc, 0, 0, 0);
        __syncthreads();
        const double* stk = st + ((size_t)(k - 2) * NT + nt) * 2 * 4 * 64 + lane;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double sv, sbv, Jr[3];
          const int n = nt * 16 + lg + 4 * r;
          if (k - 1 == 0) {
            sv = s0r[r];
            sbv = sb0r[r];
#pragma unroll
            for (int i = 0; i < 3; ++i) Jr[i] = cst[(3 + i) * H + n];
          } else {
            // J = zeta / s from the tangent activations of this layer, which
            // are still in columns 1..3 of the activation buffer (the backward
            // products only overwrite column 0); where s underflows the Hessian
            // term s (1 - s) J J vanishes and J is taken as 0
            sv = stk[(0 * 4 + r) * 64];
            sbv = stk[(1 * 4 + r) * 64];
            const double rs = (sv > 1e-290) ? rcp_d(sv) : 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) Jr[i] = Zs[(1 + i) * H * QP + n * QP + j] * rs;
          }
          abar[r] = acc[r] * sv;
          const double c2 = abar[r] * sbv;
          part[4] += c2 * Jr[0] * Jr[0];
          part[5] += c2 * Jr[1] * Jr[1];
          part[6] += c2 * Jr[2] * Jr[2];
          part[7] += c2 * Jr[0] * Jr[1];
          part[8] += c2 * Jr[0] * Jr[2];
          part[9] += c2 * Jr[1] * Jr[2];
        }
      }
    }

    // reduce over the 4 row groups of the wave, then over the neuron tiles
#pragma unroll
    for (int t = 0; t < 10; ++t) {
      part[t] += __shfl_xor(part[t], 16, 64);
      part[t] += __shfl_xor(part[t], 32, 64);
    }
    __syncthreads();
    if (lg == 0) {
#pragma unroll
      for (int t = 0; t < 10; ++t) red[(nt * QB + j) * 10 + t] = part[t];
    }
    __syncthreads();
    constexpr int NOUT = HESS ? 10 : 4;
    for (int idx = threadIdx.x; idx < QB * NOUT; idx += blockDim.x) {
      const int jj = idx / NOUT, t = idx % NOUT;
      double v = 0.0;
#pragma unroll
      for (int u = 0; u < NT; ++u) v += red[(u * QB + jj) * 10 + t];
      if (t == 0) v += net[lay.wx] * xs[jj * 3] + net[lay.wx + 1] * xs[jj * 3 + 1] + net[lay.wx + 2] * xs[jj * 3 + 2];
      if (t >= 1 && t <= 3) v += net[lay.wx + t - 1];
      if (q0 + jj < a.nq) a.jet[(q0 + jj) * 10 + t] = v;
    }
    __syncthreads();
  }
}

template <int H, int L, bool HESS>
static hipError_t launch_f64_mode(const JetArgs& a, hipStream_t s, int num_cu) {
  using C = JetCfg<H, L>;
  const int nbatch = (a.nq + C::QB - 1) / C::QB;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, jet_f64_kernel<H, L, HESS>,
                                                              C::WAVES * 64, C::LDS_BYTES);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  int grid = num_cu * per_cu;
  if (grid > nbatch) grid = nbatch;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((jet_f64_kernel<H, L, HESS>), dim3(grid), dim3(C::WAVES * 64), C::LDS_BYTES, s, a);
  return hipGetLastError();
}

template <int H, int L>
static hipError_t launch_f64(const JetArgs& a, hipStream_t s, int num_cu) {
  return a.with_hessian ? launch_f64_mode<H, L, true>(a, s, num_cu) : launch_f64_mode<H, L, false>(a, s, num_cu);
}

hipError_t launch_energy_jet_f64(int H, const JetArgs& a, hipStream_t s, int num_cu) {
  switch (H * 10 + a.L) {
    case 161: return launch_f64<16, 1>(a, s, num_cu);
    case 162: return launch_f64<16, 2>(a, s, num_cu);
    case 163: return launch_f64<16, 3>(a, s, num_cu);
    case 321: return launch_f64<32, 1>(a, s, num_cu);
    case 322: return launch_f64<32, 2>(a, s, num_cu);
    case 323: return launch_f64<32, 3>(a, s, num_cu);
    case 641: return launch_f64<64, 1>(a, s, num_cu);
    case 642: return launch_f64<64, 2>(a, s, num_cu);
    case 643: return launch_f64<64, 3>(a, s, num_cu);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gedmg
