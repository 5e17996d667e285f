// Internal declarations of the warm-start network kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace subadmm {

enum : int { EPI_STORE = 0, EPI_BIAS_F32 = 1, EPI_BIAS_RELU_BF16 = 2, EPI_RELU_MASK = 3 };

// C[M x N] = opA[M x K] opB[K x N]; opA(m, k) = A[m * sam + k * sak],
// opB(k, n) = B[k * sbk + n * sbn].  BF16 storage is passed as uint16_t bit patterns.
template <typename TA, typename TB>
struct GemmArgs {
  const TA* A;
  long sam, sak;
  const TB* B;
  long sbk, sbn;
  long M, N, K;
  long k_chunk;        // K range of one split (multiple of the K tile)
  int a_m_fast;        // 1 if sam == 1 (stage A with m as the fast index)
  int b_n_fast;        // 1 if sbn == 1
  int epi;             // EPI_*
  float* C;
  long ldc;
  long c_split;        // offset between the partial results of successive splits
  const float* bias;
  uint16_t* out_bf16;
  long ldo;
  const uint16_t* mask;
  long ldm;
};

template <typename TA, typename TB>
hipError_t launch_gemm(const GemmArgs<TA, TB>& g, int splits, hipStream_t s);
hipError_t launch_cast_bf16(const float* x, uint16_t* y, long n, hipStream_t s);
hipError_t launch_gather_rows(const float* src, long n_rows, int width, const int32_t* idx, int count, float* dst,
                              hipStream_t s);
hipError_t launch_cast_affine_bf16(const float* x, const float* scale, const float* shift, int width, uint16_t* y,
                                  long n, hipStream_t s);
hipError_t launch_loss_grad(const float* y, const float* t, const float* wt, float* dy, long n, double* partial,
                            int max_blocks, float* loss, hipStream_t s);
hipError_t launch_colsum(const float* a, long rows, int cols, float* partial, int splits, float* out, hipStream_t s);
hipError_t launch_sum_partials(const float* partial, int splits, long n, float* out, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);

// Whole-network inference in one launch (no activations kept for a backward pass).
constexpr int kInferMaxLayers = 8, kInferMaxWidth = 256;
struct MlpInferArgs {
  const float* x;        // batch x w[0] FP32
  float* y;              // batch x w[L] FP32
  const float* scale;    // input affine (nullptr: none)
  const float* shift;
  const uint16_t* Wbf;   // BF16 weights, layer k: w[k+1] x w[k] row-major at off_Wbf[k]
  const float* P;        // FP32 parameters; layer k's bias at off_b[k]
  long batch;
  int L;
  int w[kInferMaxLayers + 1];
  long off_Wbf[kInferMaxLayers];
  long off_b[kInferMaxLayers];
  int vec_w[kInferMaxLayers];  // 1: layer k's weight rows allow 16-byte loads (K % 8 == 0, aligned)
};
hipError_t launch_mlp_infer(const MlpInferArgs& a, hipStream_t s);

}  // namespace subadmm

struct subadmm_mlp;
int32_t mlp_input_width(const subadmm_mlp* m);
int32_t mlp_output_width(const subadmm_mlp* m);
int32_t mlp_max_batch(const subadmm_mlp* m);
hipStream_t mlp_stream(const subadmm_mlp* m);
// advances on every bind and input-affine change (what a captured forward pass depends on)
uint64_t mlp_generation(const subadmm_mlp* m);
// subadmm_mlp_forward with its launches on stream s (a capture stream or the bound one)
int mlp_forward_on(subadmm_mlp* m, hipStream_t s, int32_t batch, const float* x, float* y);
// subadmm_mlp_infer on stream s: the fused inference when the widths allow it, else the forward
int mlp_infer_on(subadmm_mlp* m, hipStream_t s, int32_t batch, const float* x, float* y);
