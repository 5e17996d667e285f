// HIP kernels (gfx950) of the learned warm start: per-interface features at the start of
// a step and the initial (z^0, u^0) built from the network's output.
//
// Interfaces of two classes take part: contacts (dim 3, one member) and revolute joints
// (equality, dim 5, one or two members).  Quantities are expressed in velocity units:
// a constraint force lambda is divided by the interface's z-metric weight
// w_hat = 1 / sum_i beta_i^-1 (Eq. 18 gives beta z = y + lambda, so lambda / w_hat is a
// velocity).
//   contact row (12): e_n, c (3), lambda_prev / w_hat (3), z_prev (3), log w_hat, mu
//   joint row (27):   e (5), c (5), lambda_prev / w_hat (5), z_prev member 0 (5),
//                     z_prev member 1 (5, zero for one member), log w_hat, |S_j| - 1
// with e_j the constraint error, c = sum_i J_i,j v_i the constraint velocity at the
// start-of-step velocity, and (z_prev, u_prev = -lambda_prev) the previous step's final
// values.  The network predicts the change: contact (6) = (delta lambda / w_hat (3),
// delta z (3)); joint (15) = (delta lambda / w_hat (5), delta z member 0 (5), member 1 (5)).
#include "internal.hpp"

namespace subadmm {

// Velocity of every DOF of the rigid model (v world, omega body per body block).
template <typename T>
__global__ void dof_velocity_kernel(Topo t, RigidModel<T> m, const T* vel, const T* omega, T* v_dof) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m.nb) return;
  T* v = v_dof + t.sub_dof[m.body_sub[k]] + 6 * m.body_local[k];
  for (int c = 0; c < 3; ++c) {
    v[c] = vel[3 * k + c];
    v[3 + c] = omega[3 * k + c];
  }
}

template <typename T>
__device__ inline T slot_velocity(const Topo& t, const T* J, const T* v_dof, int i, int g) {
  const int n = t.sub_n[i];
  const int loc = g - t.sub_slot[i];
  const T* row = J + t.sub_J[i] + (long)loc * n;
  const T* v = v_dof + t.sub_dof[i];
  T s = (T)0;
  for (int c = 0; c < n; ++c) s += row[c] * v[c];
  return s;
}

template <typename T>
__global__ void features_kernel(WarmArgs<T> a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.t.n_if) return;
  const int cls = a.if_class[j];
  if (cls < 0) return;
  const Topo& t = a.t;
  const int dim = t.if_dim[j];
  const bool two = t.if_nsub[j] == 2;
  const int sa = t.if_sub0[j];
  const int sb = two ? t.if_sub1[j] : sa;
  const int g0 = t.if_slot0[j], g1 = two ? t.if_slot1[j] : -1;
  const double wsum = 1.0 / (double)a.beta[sa] + (two ? 1.0 / (double)a.beta[sb] : 0.0);
  const double what = 1.0 / wsum;
  const T* e = a.e + t.if_row[j];
  float* x = (cls == 0 ? a.xc + (long)a.if_krow[j] * kContactIn : a.xj + (long)a.if_krow[j] * kJointIn);
  if (cls == 0) {
    x[0] = (float)e[0];
    for (int k = 0; k < 3; ++k) {
      x[1 + k] = (float)slot_velocity(t, a.J, a.v_dof, sa, g0 + k);
      x[4 + k] = (float)(-(double)a.u_prev[g0 + k] / what);
      x[7 + k] = (float)a.z_prev[g0 + k];
    }
    x[10] = (float)log(what);
    x[11] = (float)a.mu[j];
  } else {
    for (int k = 0; k < 5; ++k) {
      x[k] = (float)e[k];
      T c = slot_velocity(t, a.J, a.v_dof, sa, g0 + k);
      if (two) c += slot_velocity(t, a.J, a.v_dof, sb, g1 + k);
      x[5 + k] = (float)c;
      x[10 + k] = (float)(-(double)a.u_prev[g0 + k] / what);
      x[15 + k] = (float)a.z_prev[g0 + k];
      x[20 + k] = two ? (float)a.z_prev[g1 + k] : 0.f;
    }
    x[25] = (float)log(what);
    x[26] = two ? 1.f : 0.f;
    (void)dim;
  }
}

// Initial (z^0, u^0) per slot row: learned for the two interface classes (unless the
// network's output is not finite), the previous step's values elsewhere.
template <typename T>
__global__ void warm_apply_kernel(WarmArgs<T> a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.t.n_if) return;
  const Topo& t = a.t;
  const int dim = t.if_dim[j];
  const bool two = t.if_nsub[j] == 2;
  const int g[2] = {t.if_slot0[j], two ? t.if_slot1[j] : -1};
  const int cls = a.if_class[j];
  bool use = cls >= 0 && ((cls == 0 && a.yc) || (cls == 1 && a.yj));
  const float* y = nullptr;
  if (use) {
    y = cls == 0 ? a.yc + (long)a.if_krow[j] * kContactOut : a.yj + (long)a.if_krow[j] * kJointOut;
    const int no = cls == 0 ? kContactOut : kJointOut;
    for (int q = 0; q < no; ++q)
      if (!__builtin_isfinite(y[q])) use = false;
  }
  const int sa = t.if_sub0[j];
  const int sb = two ? t.if_sub1[j] : sa;
  const double what = 1.0 / (1.0 / (double)a.beta[sa] + (two ? 1.0 / (double)a.beta[sb] : 0.0));
  for (int k = 0; k < dim; ++k) {
    T lam = -a.u_prev[g[0] + k];
    if (use) lam += (T)(what * (double)y[k]);
    for (int mm = 0; mm < (two ? 2 : 1); ++mm) {
      const int s = g[mm] + k;
      a.u0[s] = -lam;
      a.z0[s] = use ? a.z_prev[s] + (T)y[dim + mm * dim + k] : a.z_prev[s];
    }
  }
}

// Training targets: the change from the previous step's values to the converged ones,
// in the network's output layout, and the loss weights of the ADMM metric
// sum_i beta_i |z_i - z*_i|^2 + beta_i^-1 |u_i - u*_i|^2: w_hat for the lambda / w_hat
// entries (sum_i beta_i^-1 w_hat^2 = w_hat), beta_i for member i's z entries, zero for an
// absent member and for every interface of a scene that did not converge.
template <typename T>
__global__ void targets_kernel(WarmArgs<T> a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.t.n_if) return;
  const int cls = a.if_class[j];
  if (cls < 0) return;
  const Topo& t = a.t;
  const int dim = cls == 0 ? 3 : 5;
  const bool two = t.if_nsub[j] == 2;
  const int sa = t.if_sub0[j];
  const int sb = two ? t.if_sub1[j] : sa;
  const int g[2] = {t.if_slot0[j], two ? t.if_slot1[j] : -1};
  const double wsum = 1.0 / (double)a.beta[sa] + (two ? 1.0 / (double)a.beta[sb] : 0.0);
  const double what = 1.0 / wsum;
  const bool ok = a.conv[a.if_scene[j]] != 0;
  float* y = cls == 0 ? a.tc : a.tj;
  float* w = cls == 0 ? a.wc : a.wj;
  const int no = cls == 0 ? kContactOut : kJointOut;
  if (y) y += (long)a.if_krow[j] * no;
  if (w) w += (long)a.if_krow[j] * no;
  for (int k = 0; k < dim; ++k) {
    if (y) y[k] = (float)(((double)a.u_prev[g[0] + k] - (double)a.u_fin[g[0] + k]) / what);
    if (w) w[k] = ok ? (float)what : 0.f;
    for (int mm = 0; mm < 2; ++mm) {
      const bool has = mm == 0 || two;
      const int s = has ? g[mm] + k : -1;
      if (y) y[dim + mm * dim + k] = has ? (float)((double)a.z_fin[s] - (double)a.z_prev[s]) : 0.f;
      if (w) w[dim + mm * dim + k] = (has && ok) ? (float)a.beta[mm == 0 ? sa : sb] : 0.f;
      if (cls == 0) break;  // contacts have one member
    }
  }
}

template <typename T>
hipError_t launch_dof_velocity(const Topo& t, const RigidModel<T>& m, const T* vel, const T* omega, T* v_dof,
                               hipStream_t s) {
  if (m.nb == 0) return hipSuccess;
  hipLaunchKernelGGL(dof_velocity_kernel<T>, dim3((m.nb + 255) / 256), dim3(256), 0, s, t, m, vel, omega, v_dof);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_features(const WarmArgs<T>& a, hipStream_t s) {
  if (a.t.n_if == 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel<T>, dim3((a.t.n_if + 127) / 128), dim3(128), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_warm_apply(const WarmArgs<T>& a, hipStream_t s) {
  if (a.t.n_if == 0) return hipSuccess;
  hipLaunchKernelGGL(warm_apply_kernel<T>, dim3((a.t.n_if + 127) / 128), dim3(128), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_targets(const WarmArgs<T>& a, hipStream_t s) {
  if (a.t.n_if == 0) return hipSuccess;
  hipLaunchKernelGGL(targets_kernel<T>, dim3((a.t.n_if + 127) / 128), dim3(128), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_targets<float>(const WarmArgs<float>&, hipStream_t);
template hipError_t launch_targets<double>(const WarmArgs<double>&, hipStream_t);
template hipError_t launch_dof_velocity<float>(const Topo&, const RigidModel<float>&, const float*, const float*,
                                               float*, hipStream_t);
template hipError_t launch_dof_velocity<double>(const Topo&, const RigidModel<double>&, const double*, const double*,
                                                double*, hipStream_t);
template hipError_t launch_features<float>(const WarmArgs<float>&, hipStream_t);
template hipError_t launch_features<double>(const WarmArgs<double>&, hipStream_t);
template hipError_t launch_warm_apply<float>(const WarmArgs<float>&, hipStream_t);
template hipError_t launch_warm_apply<double>(const WarmArgs<double>&, hipStream_t);

}  // namespace subadmm
