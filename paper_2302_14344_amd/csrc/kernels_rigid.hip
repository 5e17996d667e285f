// HIP kernels (gfx950) for the rigid-box model in maximal coordinates: the
// construction steps of Algorithm 1 (Eq. (2)-(5)) and the state update of Eq. (2), one
// launch each per step (the device functions are in rigid_device.hpp).
#include "rigid_device.hpp"

namespace subadmm {

// One workgroup per subsystem.
template <typename T>
__global__ void __launch_bounds__(128) rigid_assemble_kernel(Topo t, RigidModel<T> m, const T* pos,
                                                              const T* rot, const T* vel,
                                                              const T* omega, T dt, T* A, T* b,
                                                              T* J, T* e) {
  rigid_assemble_sub<T>(t, m, blockIdx.x, pos, rot, vel, omega, dt, A, b, J, e);
}

// One workgroup per scene (scenes of a few subsystems): the same entries, the scene's
// bodies and slot rows spread over the threads at once.
template <typename T>
__global__ void __launch_bounds__(256) rigid_assemble_scene_kernel(Topo t, RigidModel<T> m, const T* pos,
                                                                    const T* rot, const T* vel, const T* omega,
                                                                    T dt, T* A, T* b, T* J, T* e) {
  const int sc = blockIdx.x;
  rigid_assemble_scene<T>(t, m, t.sc_sub[sc], t.sc_sub[sc + 1], pos, rot, vel, omega, dt, A, b, J, e);
}

// One thread per body.
template <typename T>
__global__ void __launch_bounds__(256) rigid_advance_kernel(Topo t, RigidModel<T> m, RigidState<T> st,
                                                             const T* v_hat, T dt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m.nb) rigid_advance_body<T>(t, m, st, v_hat, dt, k);
}

template <typename T>
hipError_t launch_rigid_assemble(const Topo& t, const RigidModel<T>& m, const T* pos, const T* rot,
                                 const T* vel, const T* omega, T dt, T* A, T* b, T* J, T* e, bool per_scene,
                                 hipStream_t s) {
  if (t.n_sub == 0) return hipSuccess;
  if (per_scene)
    hipLaunchKernelGGL(rigid_assemble_scene_kernel<T>, dim3(t.n_scene), dim3(256), 0, s, t, m, pos, rot, vel,
                       omega, dt, A, b, J, e);
  else
    hipLaunchKernelGGL(rigid_assemble_kernel<T>, dim3(t.n_sub), dim3(128), 0, s, t, m, pos, rot, vel, omega,
                       dt, A, b, J, e);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rigid_advance(const Topo& t, const RigidModel<T>& m, RigidState<T> st, const T* v_hat,
                                T dt, hipStream_t s) {
  if (m.nb == 0) return hipSuccess;
  hipLaunchKernelGGL(rigid_advance_kernel<T>, dim3((m.nb + 255) / 256), dim3(256), 0, s, t, m, st, v_hat, dt);
  return hipGetLastError();
}

template hipError_t launch_rigid_assemble<float>(const Topo&, const RigidModel<float>&, const float*, const float*,
                                                 const float*, const float*, float, float*, float*, float*, float*,
                                                 bool, hipStream_t);
template hipError_t launch_rigid_assemble<double>(const Topo&, const RigidModel<double>&, const double*,
                                                  const double*, const double*, const double*, double, double*,
                                                  double*, double*, double*, bool, hipStream_t);
template hipError_t launch_rigid_advance<float>(const Topo&, const RigidModel<float>&, RigidState<float>,
                                                const float*, float, hipStream_t);
template hipError_t launch_rigid_advance<double>(const Topo&, const RigidModel<double>&, RigidState<double>,
                                                 const double*, double, hipStream_t);

}  // namespace subadmm
