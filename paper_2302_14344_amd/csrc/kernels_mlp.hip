// HIP kernels (gfx950) of the warm-start network: a perceptron with ReLU hidden layers
// and a linear output, BF16 operands on the matrix cores with FP32 accumulation, FP32
// master weights and Adam.
//
// All products go through one tiled GEMM, C[M x N] = opA[M x K] opB[K x N], whose
// operands are addressed through strides (so X W^T, dZ W and dZ^T X are the same kernel)
// and converted to BF16 while they are staged into LDS.  A 256-thread workgroup owns a
// 64 x 64 tile of C; each of its four waves owns 32 x 32 = 2 x 2 tiles of gfx950's
// 16x16x32 BF16 MFMA (one instruction per tile per 32-deep block of K), fed from LDS by one
// 16-byte read per operand and lane (tile rows padded to 80 bytes, which keeps those reads
// 16-byte aligned and spreads the rows over the banks).  Epilogues fuse the bias, the ReLU and the BF16 store of the next
// layer's input, or the ReLU mask of the backward pass.
#include "mlp_internal.hpp"

namespace subadmm {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even on the bit pattern (NaN kept quiet).
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename X>
__device__ inline uint16_t as_bf16(X v);
template <>
__device__ inline uint16_t as_bf16<float>(float v) { return to_bf16(v); }
template <>
__device__ inline uint16_t as_bf16<uint16_t>(uint16_t v) { return v; }

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

template <typename TA, typename TB>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs<TA, TB> g) {
  __shared__ __align__(16) uint16_t As[kBM][kBK + kPad];
  __shared__ __align__(16) uint16_t Bt[kBN][kBK + kPad];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const long m0 = (long)blockIdx.y * kBM, n0 = (long)blockIdx.x * kBN;
  const long kb = (long)blockIdx.z * g.k_chunk;
  const long ke = kb + g.k_chunk < g.K ? kb + g.k_chunk : g.K;

  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4_t){0.f, 0.f, 0.f, 0.f};

  for (long k0 = kb; k0 < ke; k0 += kBK) {
    // stage opA(m0.., k0..) and opB(k0.., n0..) as BF16; the faster-varying index of each
    // thread is the operand's unit-stride one, so global reads coalesce
#pragma unroll
    for (int q = 0; q < (kBM * kBK) / 256; ++q) {
      const int e = tid + 256 * q;
      int m, k;
      if (g.a_m_fast) { m = e % kBM; k = e / kBM; } else { k = e % kBK; m = e / kBK; }
      const long gm = m0 + m, gk = k0 + k;
      uint16_t v = 0;
      if (gm < g.M && gk < ke) v = as_bf16<TA>(g.A[gm * g.sam + gk * g.sak]);
      As[m][k] = v;
    }
#pragma unroll
    for (int q = 0; q < (kBN * kBK) / 256; ++q) {
      const int e = tid + 256 * q;
      int n, k;
      if (g.b_n_fast) { n = e % kBN; k = e / kBN; } else { k = e % kBK; n = e / kBK; }
      const long gn = n0 + n, gk = k0 + k;
      uint16_t v = 0;
      if (gn < g.N && gk < ke) v = as_bf16<TB>(g.B[gk * g.sbk + gn * g.sbn]);
      Bt[n][k] = v;
    }
    __syncthreads();
    // lane l supplies row l % 16 of A's tile and column l % 16 of B's with the eight k of
    // group l / 16; A and B take the same k assignment, so each product is a 32-deep sum
    static_assert(kBK % 32 == 0 && ((kBK + kPad) * 2) % 16 == 0, "16-byte fragment reads");
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 32) {
      bf16x8_t af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const uint16_t* pa = &As[32 * wm + 16 * i + (lane & 15)][kk + 8 * (lane >> 4)];
        af[i] = *reinterpret_cast<const bf16x8_t*>(pa);
        const uint16_t* pb = &Bt[32 * wn + 16 * i + (lane & 15)][kk + 8 * (lane >> 4)];
        bfr[i] = *reinterpret_cast<const bf16x8_t*>(pb);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  // epilogue: lane holds rows 4*(lane/16) + r, column lane % 16 of each 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long m = m0 + 32 * wm + 16 * i + 4 * (lane >> 4) + r;
        const long n = n0 + 32 * wn + 16 * j + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][r];
        switch (g.epi) {
          case EPI_STORE:
            g.C[(long)blockIdx.z * g.c_split + m * g.ldc + n] = v;
            break;
          case EPI_BIAS_F32:
            g.C[m * g.ldc + n] = v + g.bias[n];
            break;
          case EPI_BIAS_RELU_BF16: {
            v += g.bias[n];
            g.out_bf16[m * g.ldo + n] = to_bf16(v > 0.f ? v : 0.f);
            break;
          }
          case EPI_RELU_MASK: {
            const uint16_t a = g.mask[m * g.ldm + n];  // the ReLU output of the forward pass
            g.C[m * g.ldc + n] = (a != 0 && (a & 0x8000u) == 0) ? v : 0.f;
            break;
          }
        }
      }
}

template <typename TA, typename TB>
hipError_t launch_gemm(const GemmArgs<TA, TB>& g, int splits, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((unsigned)((g.N + kBN - 1) / kBN), (unsigned)((g.M + kBM - 1) / kBM), (unsigned)splits);
  hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB>), grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// Inference of the whole network for 64 rows per workgroup (the learned start): the input's
// affine map and BF16 rounding, then per layer the product on the 16x16x32 BF16 MFMA with the
// 32-deep k blocks in the order gemm_bf16_kernel takes them, bias, ReLU and the BF16 rounding
// of the hidden activations, which stay in LDS; the last layer's FP32 output plus bias goes to
// y.  The same arithmetic as the per-layer launches, so the same output bit for bit.  Wave w
// owns the column tiles w, w + 4, ... (at most four of 16 columns each) of all four 16-row
// tiles, so every weight is read once per workgroup.
constexpr int kInferLd = kInferMaxWidth + 8;  // 528-byte rows: 16-byte aligned fragment reads

__global__ void __launch_bounds__(256) mlp_infer_kernel(MlpInferArgs a) {
  __shared__ __align__(16) uint16_t buf[2][64][kInferLd];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int g = lane >> 4, cl = lane & 15;
  const long r0 = (long)blockIdx.x * 64;
  {
    // input rows, zero beyond the width up to the next multiple of 32 and beyond the batch
    const int w0 = a.w[0], kp = (w0 + 31) / 32 * 32;
    for (int q = tid; q < 64 * kp; q += 256) {
      const int r = q / kp, c = q - r * kp;
      const long gr = r0 + r;
      uint16_t v = 0;
      if (gr < a.batch && c < w0) {
        const float xv = a.x[gr * w0 + c];
        v = a.scale ? to_bf16(xv * a.scale[c] + a.shift[c]) : to_bf16(xv);
      }
      buf[0][r][c] = v;
    }
  }
  __syncthreads();
  int cur = 0;
  for (int l = 0; l < a.L; ++l) {
    const int K = a.w[l], N = a.w[l + 1];
    const int nct = (N + 15) / 16;
    const uint16_t* W = a.Wbf + a.off_Wbf[l];
    const float* bias = a.P + a.off_b[l];
    f32x4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
      bf16x8_t af[4], bfr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = *reinterpret_cast<const bf16x8_t*>(&buf[cur][16 * i + cl][k0 + 8 * g]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 16 * (wv + 4 * j) + cl;
        const int kb = k0 + 8 * g;
        if (n < N && a.vec_w[l] && kb + 8 <= K) {
          bfr[j] = *reinterpret_cast<const bf16x8_t*>(W + (long)n * K + kb);
        } else {
          bf16x8_t v;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            v[e] = __builtin_bit_cast(__bf16, (n < N && kb + e < K) ? W[(long)n * K + kb + e] : (uint16_t)0);
          bfr[j] = v;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (wv + 4 * j >= nct) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
      }
    }
    const bool last = l + 1 == a.L;
    const int nxt = cur ^ 1;
    // lane holds rows 4 * g + r, column cl of each 16 x 16 tile
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = 16 * (wv + 4 * j) + cl;
      if (wv + 4 * j >= nct || n >= N) continue;
      const float bn = bias[n];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * i + 4 * g + r;
          float v = acc[i][j][r];
          if (last) {
            if (r0 + row < a.batch) a.y[(r0 + row) * N + n] = v + bn;
          } else {
            v += bn;
            buf[nxt][row][n] = to_bf16(v > 0.f ? v : 0.f);
          }
        }
    }
    if (!last) {
      // zero the next layer's padding columns (an earlier, wider layer may have left values)
      const int np = (N + 31) / 32 * 32;
      for (int q = tid; q < 64 * (np - N); q += 256) buf[nxt][q / (np - N)][N + q % (np - N)] = 0;
    }
    __syncthreads();
    cur = nxt;
  }
}

hipError_t launch_mlp_infer(const MlpInferArgs& a, hipStream_t s) {
  if (a.batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)((a.batch + 63) / 64)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Minibatch gather: dst row r = src row idx[r] (FP32 rows of `width` entries); a row whose
// index lies outside [0, n_rows) is filled with NaN.
__global__ void gather_rows_kernel(const float* src, long n_rows, int width, const int32_t* idx, int count,
                                   float* dst) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)count * width) return;
  const long r = k / width;
  const int c = (int)(k - r * width);
  const int32_t i = idx[r];
  dst[k] = (i >= 0 && i < n_rows) ? src[(long)i * width + c] : __builtin_nanf("");
}

hipError_t launch_gather_rows(const float* src, long n_rows, int width, const int32_t* idx, int count, float* dst,
                              hipStream_t s) {
  const long n = (long)count * width;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, n_rows, width, idx,
                     count, dst);
  return hipGetLastError();
}

template hipError_t launch_gemm<float, uint16_t>(const GemmArgs<float, uint16_t>&, int, hipStream_t);
template hipError_t launch_gemm<uint16_t, uint16_t>(const GemmArgs<uint16_t, uint16_t>&, int, hipStream_t);
template hipError_t launch_gemm<float, float>(const GemmArgs<float, float>&, int, hipStream_t);

// ------------------------------------------------------------------------------------
// Element-wise kernels
// ------------------------------------------------------------------------------------
__global__ void cast_bf16_kernel(const float* x, uint16_t* y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = to_bf16(x[i]);
}

// Input normalisation in FP32 before the BF16 rounding: y = bf16(x * scale + shift) per column.
__global__ void cast_affine_bf16_kernel(const float* x, const float* scale, const float* shift, int width,
                                        uint16_t* y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % width);
    y[i] = to_bf16(x[i] * scale[c] + shift[c]);
  }
}

// dY = wt * (y - target); per-block partial sums of 0.5 wt (y - target)^2 in FP64.
__global__ void __launch_bounds__(256) loss_grad_kernel(const float* y, const float* t, const float* wt, float* dy,
                                                         long n, double* partial) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float r = y[i] - t[i];
    const float w = wt ? wt[i] : 1.f;
    dy[i] = w * r;
    acc += 0.5 * (double)w * (double)r * (double)r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void loss_sum_kernel(const double* partial, int n, float* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *loss = (float)s;
  }
}

// Column sums of a rows x cols FP32 matrix in two fixed-order stages (bias gradients).
__global__ void __launch_bounds__(256) colsum_partial_kernel(const float* a, long rows, int cols, long rows_per,
                                                              float* partial) {
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;  // 4 row groups
  __shared__ float red[4][64];
  const long r0 = (long)blockIdx.y * rows_per;
  const long r1 = r0 + rows_per < rows ? r0 + rows_per : rows;
  float s = 0.f;
  if (c < cols)
    for (long r = r0 + g; r < r1; r += 4) s += a[r * cols + c];
  red[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && c < cols) {
    const float t = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    partial[(long)blockIdx.y * cols + c] = t;
  }
}

// out[i] = sum over s of partial[s * n + i] (fixed order)
__global__ void sum_partials_kernel(const float* partial, int splits, long n, float* out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int q = 0; q < splits; ++q) s += partial[(long)q * n + i];
    out[i] = s;
  }
}

// Adam on the FP32 master parameters; the weight ranges are then re-cast to BF16.
__global__ void adam_kernel(float* p, const float* gr, float* m, float* v, long n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

hipError_t launch_cast_bf16(const float* x, uint16_t* y, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(cast_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t launch_cast_affine_bf16(const float* x, const float* scale, const float* shift, int width, uint16_t* y,
                                  long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(cast_affine_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, scale, shift, width, y, n);
  return hipGetLastError();
}

hipError_t launch_loss_grad(const float* y, const float* t, const float* wt, float* dy, long n, double* partial,
                            int max_blocks, float* loss, hipStream_t s) {
  long blocks = (n + 255) / 256;
  if (blocks > max_blocks) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(loss_grad_kernel, dim3((unsigned)blocks), dim3(256), 0, s, y, t, wt, dy, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !loss) return e;
  hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(64), 0, s, partial, (int)blocks, loss);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* a, long rows, int cols, float* partial, int splits, float* out, hipStream_t s) {
  const long rows_per = (rows + splits - 1) / splits;
  hipLaunchKernelGGL(colsum_partial_kernel, dim3((unsigned)((cols + 63) / 64), (unsigned)splits), dim3(256), 0, s, a,
                     rows, cols, rows_per, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s, partial, splits,
                     (long)cols, out);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const float* partial, int splits, long n, float* out, hipStream_t s) {
  const long blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)blocks), dim3(256), 0, s, partial, splits, n, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  const long blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace subadmm
