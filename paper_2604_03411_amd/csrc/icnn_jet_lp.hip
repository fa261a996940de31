// Mixed-precision energy-network jets: the hidden->hidden products run on the
// 16x16x32 BF16 or FP16 matrix cores with FP32 accumulation; activations,
// Jacobians and the Hessian sum are FP32; the result is returned in FP64 for
// the FP64 element kernel.  Same algorithm as the FP64 kernel (increment form
// over x = 0, 4 forward columns, 1 adjoint column, Hessian from per-layer
// Jacobians).
//
// Layouts (16x16x32): lane l supplies A[l%16][8(l/16) .. +7] and
// B[8(l/16) .. +7][l%16]; it receives C rows 4(l/16) .. +3 of column l%16.
// A = weights (each wave keeps its 16-row slice, forward and transposed, in
// registers for the whole persistent block); B = activations staged in LDS as
// [qp][neuron] rows, so a lane's 8-element K slice is one 16-byte load.
// Blocks of 4 waves at 4 waves per SIMD: the backward-pass state of the middle
// layers lives in LDS and layer 0's Jacobian is re-read from the staged input
// weights, which keeps the kernel within 128 registers.
#include "device_common.h"
#include "gedmg_internal.h"

namespace gedmg {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct Lp;
template <>
struct Lp<__bf16> {
  using v8 = bf16x8_t;
  using v4 = bf16x4_t;
  static __device__ __forceinline__ f4_t mfma(v8 a, v8 b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Lp<_Float16> {
  using v8 = f16x8_t;
  using v4 = f16x4_t;
  static __device__ __forceinline__ f4_t mfma(v8 a, v8 b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <int H, int L, int WAVES>
struct LpCfg {
  static constexpr int NT = H / 16;
  static constexpr int NQT = WAVES / NT;
  static constexpr int QB = 16 * NQT;
  static constexpr int KP = H < 32 ? 32 : H;   // K padded to the instruction depth
  static constexpr int KS = KP / 32;            // K steps per product
  static constexpr int HP = KP + 8;             // LDS row (elements)
  static constexpr int WHP = H + 8;             // row of the packed low-precision weights
  static constexpr int Z_BYTES = 4 * QB * HP * 2;
  static constexpr int X_BYTES = QB * 3 * 4;
  static constexpr int RED_BYTES = NT * QB * 10 * 4;
  // per-neuron constants in FP32, staged once per block: for every layer k
  // (a0, s0, sb0) at fields 3k..3k+2, then W0 (3), Wx of layers 1..L-1 (3
  // each) and wz: 6L + 1 fields of H
  static constexpr int NF = 6 * L + 1;
  static constexpr int C_BYTES = NF * H * 4;
  // backward-pass state of the middle layers 1 .. L-2: per wave, the logistic
  // pair and the input Jacobian (5 fields) of each of a lane's 4 rows,
  // lane-contiguous
  static constexpr int ST_BYTES = (L > 2 ? L - 2 : 0) * WAVES * 5 * 4 * 64 * 4;
  static constexpr int LDS_BYTES = (Z_BYTES > RED_BYTES ? Z_BYTES : RED_BYTES) + X_BYTES + C_BYTES + ST_BYTES;
  static_assert(WAVES % NT == 0, "waves must cover the neuron tiles");
};

template <typename T>
__device__ __forceinline__ T from_bits(uint16_t b) {
  return __builtin_bit_cast(T, b);
}

template <typename T, int H, int L, int WAVES>
__global__ __launch_bounds__(WAVES * 64, 4) void jet_lp_kernel(JetArgs a) {
  using C = LpCfg<H, L, WAVES>;
  using V8 = typename Lp<T>::v8;
  using V4 = typename Lp<T>::v4;
  constexpr int NT = C::NT, QB = C::QB, HP = C::HP, KS = C::KS, WHP = C::WHP;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* Zs = reinterpret_cast<T*>(lds_raw);
  float* red = reinterpret_cast<float*>(lds_raw);
  float* xs = reinterpret_cast<float*>(lds_raw + (C::Z_BYTES > C::RED_BYTES ? C::Z_BYTES : C::RED_BYTES));
  float* cf = xs + QB * 3;  // [field][neuron]
  float* st = cf + C::NF * H;  // [layer-1][wave][field][row][lane]
  const NetLayout lay = make_layout_hd(3, H, L, 3);
  const double* __restrict__ net = a.net;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = wave % NT, qt = wave / NT;
  const int li = lane & 15, lg = lane >> 4;
  const int j = qt * 16 + li;

  // weights of this wave's neuron tile, forward (W rows) and transposed
  V8 Wf[L > 1 ? L - 1 : 1][KS], Wb[L > 1 ? L - 1 : 1][KS];
#pragma unroll
  for (int k = 1; k < L; ++k)
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int m = 32 * s + 8 * lg + t;
        const uint16_t* Wk = a.w16 + (size_t)(k - 1) * H * WHP;
        Wf[k - 1][s][t] = (m < H) ? from_bits<T>(Wk[(nt * 16 + li) * WHP + m]) : from_bits<T>(0);
        Wb[k - 1][s][t] = (m < H) ? from_bits<T>(Wk[m * WHP + nt * 16 + li]) : from_bits<T>(0);
      }
  for (int idx = threadIdx.x; idx < C::NF * H; idx += blockDim.x) {
    const int f = idx / H, n = idx % H;
    double v;
    if (f < 3 * L) {
      const int k = f / 3, g = f % 3;
      v = net[(g == 0 ? lay.a0 : g == 1 ? lay.s0 : lay.sb0) + k * H + n];
    } else if (f < 3 * L + 3) {
      v = net[lay.W0 + n * 3 + (f - 3 * L)];
    } else if (f < 6 * L) {
      const int k = 1 + (f - 3 * L - 3) / 3, i = (f - 3 * L - 3) % 3;
      v = net[(k == 1 ? lay.Wx[1] : lay.Wx[2]) + n * 3 + i];
    } else {
      v = net[lay.wz + n];
    }
    cf[idx] = (float)v;
  }
  // zero the K padding of the activation rows once (never written afterwards)
  if (C::KP > H)
    for (int idx = threadIdx.x; idx < 4 * QB * HP; idx += blockDim.x)
      if (idx % HP >= H) Zs[idx] = from_bits<T>(0);
  __syncthreads();

  const int nbatch = (a.nq + QB - 1) / QB;
  // the next tile's inputs travel in a register of the first QB * 3 threads
  static_assert(QB * 3 <= WAVES * 64, "one input value per thread");
  const int xi = threadIdx.x;
  float xnext = 0.0f;
  if (xi < QB * 3 && (long)blockIdx.x * QB + xi / 3 < a.nq) xnext = (float)a.x[(long)blockIdx.x * QB * 3 + xi];
  for (int batch = blockIdx.x; batch < nbatch; batch += gridDim.x) {
    const long q0 = (long)batch * QB;
    if (xi < QB * 3) xs[xi] = xnext;
    {
      const long q1 = (long)(batch + gridDim.x) * QB;
      xnext = 0.0f;
      if (xi < QB * 3 && q1 + xi / 3 < a.nq) xnext = (float)a.x[q1 * 3 + xi];
    }
    __syncthreads();
    const float x[3] = {xs[j * 3], xs[j * 3 + 1], xs[j * 3 + 2]};

    // State kept for the backward pass: layers 0 .. L-2 (the last hidden
    // layer's adjoint is wz, so its Hessian term is added in the forward pass).
    float s0r[4], sb0r[4], dz[4], zt[4][3];
    float part[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) part[t] = 0.f;
    float abar[4];
    const bool hess = a.with_hessian != 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = nt * 16 + 4 * lg + r;
      const float w0 = cf[(3 * L) * H + n], w1 = cf[(3 * L + 1) * H + n], w2 = cf[(3 * L + 2) * H + n];
      const float da = w0 * x[0] + w1 * x[1] + w2 * x[2];
      dz[r] = delta_softplus(da, cf[n], cf[H + n], cf[2 * H + n], s0r[r], sb0r[r]);
      zt[r][0] = s0r[r] * w0;
      zt[r][1] = s0r[r] * w1;
      zt[r][2] = s0r[r] * w2;
      if (L == 1) {
        const float wz = cf[6 * L * H + n];
        part[0] += wz * dz[r];
#pragma unroll
        for (int i = 0; i < 3; ++i) part[1 + i] += wz * zt[r][i];
        abar[r] = wz * s0r[r];
        if (hess) {
          const float c2 = abar[r] * sb0r[r];
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
      {
        V4 v0, v1, v2, v3;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          v0[r] = (T)dz[r];
          v1[r] = (T)zt[r][0];
          v2[r] = (T)zt[r][1];
          v3[r] = (T)zt[r][2];
        }
        const int o = j * HP + nt * 16 + 4 * lg;
        *reinterpret_cast<V4*>(&Zs[o]) = v0;
        *reinterpret_cast<V4*>(&Zs[QB * HP + o]) = v1;
        *reinterpret_cast<V4*>(&Zs[2 * QB * HP + o]) = v2;
        *reinterpret_cast<V4*>(&Zs[3 * QB * HP + o]) = v3;
      }
      __syncthreads();
      f4_t acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int o = (qt * 16 + li) * HP + 32 * s + 8 * lg;
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[c] = Lp<T>::mfma(Wf[k - 1][s], *reinterpret_cast<const V8*>(&Zs[c * QB * HP + o]), acc[c]);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = nt * 16 + 4 * lg + r;
        const float* wx = cf + (3 * L + 3 + 3 * (k - 1)) * H + n;
        const float wx0 = wx[0], wx1 = wx[H], wx2 = wx[2 * H];
        const float da = acc[0][r] + wx0 * x[0] + wx1 * x[1] + wx2 * x[2];
        const float jk[3] = {acc[1][r] + wx0, acc[2][r] + wx1, acc[3][r] + wx2};
        float s_, sb_;
        dz[r] = delta_softplus(da, cf[3 * k * H + n], cf[(3 * k + 1) * H + n], cf[(3 * k + 2) * H + n], s_, sb_);
#pragma unroll
        for (int i = 0; i < 3; ++i) zt[r][i] = s_ * jk[i];
        if (k == L - 1) {
          const float wz = cf[6 * L * H + n];
          part[0] += wz * dz[r];
#pragma unroll
          for (int i = 0; i < 3; ++i) part[1 + i] += wz * zt[r][i];
          abar[r] = wz * s_;
          if (hess) {
            const float c2 = abar[r] * sb_;
            part[4] += c2 * jk[0] * jk[0];
            part[5] += c2 * jk[1] * jk[1];
            part[6] += c2 * jk[2] * jk[2];
            part[7] += c2 * jk[0] * jk[1];
            part[8] += c2 * jk[0] * jk[2];
            part[9] += c2 * jk[1] * jk[2];
          }
        } else if (hess) {
          float* stk = st + ((size_t)(k - 1) * WAVES + wave) * 5 * 4 * 64 + lane;
          stk[(0 * 4 + r) * 64] = s_;
          stk[(1 * 4 + r) * 64] = sb_;
#pragma unroll
          for (int i = 0; i < 3; ++i) stk[((2 + i) * 4 + r) * 64] = jk[i];
        }
      }
    }

    if (hess) {
#pragma unroll
      for (int k = L - 1; k >= 1; --k) {
        V4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = (T)abar[r];
        *reinterpret_cast<V4*>(&Zs[j * HP + nt * 16 + 4 * lg]) = v;
        __syncthreads();
        f4_t acc = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; ++s)
          acc = Lp<T>::mfma(Wb[k - 1][s], *reinterpret_cast<const V8*>(&Zs[(qt * 16 + li) * HP + 32 * s + 8 * lg]),
                            acc);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float sv, sbv, Jr[3];
          if (k - 1 == 0) {
            const int n = nt * 16 + 4 * lg + r;
            sv = s0r[r];
            sbv = sb0r[r];
#pragma unroll
            for (int i = 0; i < 3; ++i) Jr[i] = cf[(3 * L + i) * H + n];
          } else {
            const float* stk = st + ((size_t)(k - 2) * WAVES + wave) * 5 * 4 * 64 + lane;
            sv = stk[(0 * 4 + r) * 64];
            sbv = stk[(1 * 4 + r) * 64];
#pragma unroll
            for (int i = 0; i < 3; ++i) Jr[i] = stk[((2 + i) * 4 + r) * 64];
          }
          abar[r] = acc[r] * sv;
          const float c2 = abar[r] * sbv;
          part[4] += c2 * Jr[0] * Jr[0];
          part[5] += c2 * Jr[1] * Jr[1];
          part[6] += c2 * Jr[2] * Jr[2];
          part[7] += c2 * Jr[0] * Jr[1];
          part[8] += c2 * Jr[0] * Jr[2];
          part[9] += c2 * Jr[1] * Jr[2];
        }
      }
    }
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
    for (int idx = threadIdx.x; idx < QB * 10; idx += blockDim.x) {
      const int jj = idx / 10, t = idx % 10;
      double v = 0.0;
#pragma unroll
      for (int u = 0; u < NT; ++u) v += (double)red[(u * QB + jj) * 10 + t];
      if (t == 0)
        v += net[lay.wx] * xs[jj * 3] + net[lay.wx + 1] * xs[jj * 3 + 1] + net[lay.wx + 2] * xs[jj * 3 + 2];
      if (t >= 1 && t <= 3) v += net[lay.wx + t - 1];
      if (q0 + jj < a.nq) a.jet[(q0 + jj) * 10 + t] = v;
    }
    __syncthreads();
  }
}

template <typename T, int H, int L, int WAVES>
static hipError_t launch_lp(const JetArgs& a, hipStream_t s, int num_cu) {
  using C = LpCfg<H, L, WAVES>;
  const int nbatch = (a.nq + C::QB - 1) / C::QB;
  hipError_t e = hipFuncSetAttribute((const void*)jet_lp_kernel<T, H, L, WAVES>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS_BYTES);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, jet_lp_kernel<T, H, L, WAVES>, WAVES * 64, C::LDS_BYTES);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  int grid = num_cu * per_cu;
  if (grid > nbatch) grid = nbatch;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((jet_lp_kernel<T, H, L, WAVES>), dim3(grid), dim3(WAVES * 64), C::LDS_BYTES, s, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t dispatch(int H, const JetArgs& a, hipStream_t s, int num_cu) {
  switch (H * 10 + a.L) {
    case 161: return launch_lp<T, 16, 1, 4>(a, s, num_cu);
    case 162: return launch_lp<T, 16, 2, 4>(a, s, num_cu);
    case 163: return launch_lp<T, 16, 3, 4>(a, s, num_cu);
    case 321: return launch_lp<T, 32, 1, 4>(a, s, num_cu);
    case 322: return launch_lp<T, 32, 2, 4>(a, s, num_cu);
    case 323: return launch_lp<T, 32, 3, 4>(a, s, num_cu);
    case 641: return launch_lp<T, 64, 1, 4>(a, s, num_cu);
    case 642: return launch_lp<T, 64, 2, 4>(a, s, num_cu);
    case 643: return launch_lp<T, 64, 3, 4>(a, s, num_cu);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_energy_jet_lp(int precision, int H, const JetArgs& a, hipStream_t s, int num_cu) {
  if (precision == GEDMG_BF16) return dispatch<__bf16>(H, a, s, num_cu);
  if (precision == GEDMG_FP16) return dispatch<_Float16>(H, a, s, num_cu);
  return hipErrorInvalidValue;
}

}  // namespace gedmg
