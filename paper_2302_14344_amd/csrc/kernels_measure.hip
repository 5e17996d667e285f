// Accuracy measure of a step (the constraint error of the paper's evaluation, Sec. IV): per
// interface j with c_j = sum_i J_i,j v_hat_i + e_j and w_j = sum_i 1/beta_i, the residual of
// its constraint law (equality |c|; hard rows and the contact normal Fischer-Burmeister
// FB(c, w lambda) = c + w lambda - sqrt(c^2 + (w lambda)^2); soft w |lambda + k (e + alpha (c - e))|;
// friction |w lambda_t - P(w lambda_t - c_t)| with P the projection onto the disc of radius
// mu w lambda_n), and per scene the square root of the sum of squares over the interfaces
// whose kind is in the mask.  One workgroup per
// scene; FP64 arithmetic on the step's outputs; the scene's interfaces are summed in a fixed
// order.
#include "internal.hpp"

namespace subadmm {

namespace {

__device__ inline double fbd(double a, double b) { return a + b - __builtin_sqrt(a * a + b * b); }

__device__ inline double wave_sum_fixed(double v) {
  // butterfly over the 64 lanes in a fixed pattern: every lane ends with the same total
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace

template <typename T>
__global__ void __launch_bounds__(256) constraint_error_kernel(ErrorArgs<T> a) {
  __shared__ double part[4];
  const int sc = blockIdx.x;
  const Topo& t = a.t;
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int j = t.sc_if[sc] + tid; j < t.sc_if[sc + 1]; j += blockDim.x) {
    const int dim = t.if_dim[j], kind = t.if_kind[j], nm = t.if_nsub[j];
    if (!((a.kinds >> kind) & 1)) continue;
    double c[kMaxIfDim], lm[kMaxIfDim];
    double w = 0.0;
    for (int k = 0; k < dim; ++k) {
      c[k] = (double)a.e[t.if_row[j] + k];
      lm[k] = (double)a.lambda[t.if_row[j] + k];
    }
    for (int m = 0; m < nm; ++m) {
      const int i = m == 0 ? t.if_sub0[j] : m == 1 ? t.if_sub1[j] : t.if_subx[2 * j + m - 2];
      const int g0 = m == 0 ? t.if_slot0[j] : m == 1 ? t.if_slot1[j] : t.if_slotx[2 * j + m - 2];
      const int n = t.sub_n[i];
      const T* v = a.v_hat + t.sub_dof[i];
      w += 1.0 / (double)a.beta[i];
      for (int k = 0; k < dim; ++k) {
        const int g = g0 + k;
        if (a.J) {
          const T* row = a.J + t.sub_J[i] + (long)(g - t.sub_slot[i]) * n;
          double s = 0.0;
          for (int q = 0; q < n; ++q) s += (double)row[q] * (double)v[q];
          c[k] += s;
        } else {
          c[k] += (double)a.slot_sgn[g] * (double)v[a.slot_dof[g]];
        }
      }
    }
    double r2 = 0.0;
    if (kind == KIND_EQUALITY) {
      for (int k = 0; k < dim; ++k) r2 += c[k] * c[k];
    } else if (kind == KIND_HARD_INEQ) {
      for (int k = 0; k < dim; ++k) {
        const double f = fbd(c[k], w * lm[k]);
        r2 += f * f;
      }
    } else if (kind == KIND_SOFT) {
      const double kk = (double)a.ksoft[j], al = (double)a.asoft[j];
      for (int k = 0; k < dim; ++k) {
        const double ev = (double)a.e[t.if_row[j] + k];
        const double r = w * (lm[k] + kk * (ev + al * (c[k] - ev)));
        r2 += r * r;
      }
    } else {
      const double rn = fbd(c[0], w * lm[0]);
      const double q1 = w * lm[1] - c[1], q2 = w * lm[2] - c[2];
      const double rad = (double)a.mu[j] * w * (lm[0] > 0.0 ? lm[0] : 0.0);
      const double nq = __builtin_sqrt(q1 * q1 + q2 * q2);
      const double s = nq <= rad ? 1.0 : (nq > 0.0 ? rad / nq : 1.0);
      const double r1 = w * lm[1] - s * q1, r2t = w * lm[2] - s * q2;
      r2 = rn * rn + r1 * r1 + r2t * r2t;
    }
    acc += r2;
  }
  acc = wave_sum_fixed(acc);
  if ((tid & 63) == 0) part[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) tot += part[q];
    a.out[sc] = __builtin_sqrt(tot);
  }
}

template <typename T>
hipError_t launch_constraint_error(const ErrorArgs<T>& a, hipStream_t s) {
  if (a.t.n_scene == 0) return hipSuccess;
  hipLaunchKernelGGL(constraint_error_kernel<T>, dim3(a.t.n_scene), dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_constraint_error<float>(const ErrorArgs<float>&, hipStream_t);
template hipError_t launch_constraint_error<double>(const ErrorArgs<double>&, hipStream_t);

}  // namespace subadmm
