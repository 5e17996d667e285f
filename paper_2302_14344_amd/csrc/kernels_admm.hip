// HIP kernels (gfx950) for the per-step factorisation and the ADMM iteration of the
// subsystem-based ADMM method (arXiv 2302.14344, Algorithm 1).
//
// factor_kernel: one workgroup per subsystem.  Forms K_i = A_i + beta_i J_c,i^T J_c,i
//   (Eq. (15), beta_i of Eq. (23)), Jacobi-scales it, factorises it in LDS (Cholesky)
//   and precomputes the slot-space operators of the x-update:
//     H_i = J K^-1 J^T (nc x nc),  d_i = J K^-1 b,  G_i = K^-1 J^T,  c_i = K^-1 b,
//   so that, with w_i = beta_i z_i - u_i,
//     x_i = J v_hat_i = d_i + H_i w_i   and   v_hat_i = c_i + G_i w_i,
//   which is Eq. (15) followed by x = J v_hat, reassociated.  The per-iteration work is
//   then one small dense matrix-vector product per subsystem with no sequential chain.
// loop_kernel: one workgroup per scene runs the whole iteration in one launch, with the
//   slot state in LDS:
//     x-update (Eq. 15) -> y = beta x + u (Eq. 18) -> residual (Eq. 22, deterministic
//     block reduction) -> stopping test -> z-update (Eq. 16-21) -> dual update (Eq. 14).
//   After a z-update u_i,j = -lambda_j and w = beta z - u = y + 2 lambda, so the kernel
//   keeps (y, w, u) per slot row.
#include "internal.hpp"

namespace subadmm {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ inline T dev_sqrt(T x);
template <>
__device__ inline float dev_sqrt<float>(float x) { return __builtin_sqrtf(x); }
template <>
__device__ inline double dev_sqrt<double>(double x) { return __builtin_sqrt(x); }

// ------------------------------------------------------------------------------------
// Per-step factorisation and slot-space operators (Alg. 1 factorisation step)
// ------------------------------------------------------------------------------------
template <typename T, typename C>
__global__ void __launch_bounds__(128) factor_kernel(FactorArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* sm = reinterpret_cast<C*>(smem_raw);
  __shared__ double red[2][2];
  __shared__ int bad;

  const int i = a.order[a.first + blockIdx.x];
  const int tid = threadIdx.x;
  const int bd = blockDim.x;
  const int n = a.t.sub_n[i];
  const int nc = a.t.sub_nc[i];
  // LDS leading dimensions are odd so that strided accesses fall in distinct banks
  const int ld = n | 1;
  C* K = sm;                   // n x n, row-major with leading dimension ld, lower used
  C* Jl = K + n * ld;          // nc x n, row-major, leading dimension ld
  C* X = Jl + nc * ld;         // (nc + 1) columns of length n, column stride ld
  C* sc = X + (nc + 1) * ld;   // Jacobi scaling 1/sqrt(K_rr)

  const T* A = a.A + a.t.sub_A[i];
  const T* J = a.J + a.t.sub_J[i];
  const T* b = a.b + a.t.sub_dof[i];
  if (tid == 0) bad = 0;
  for (int t = tid; t < n * n; t += bd) {
    const int r = t / n, c = t - r * n;
    K[r * ld + c] = (C)A[t];
  }
  for (int t = tid; t < nc * n; t += bd) {
    const int r = t / n, c = t - r * n;
    Jl[r * ld + c] = (C)J[t];
  }
  __syncthreads();

  // Eq. (23): beta_i = Tr(A_i) / Tr(J^T J); Tr(J^T J) = |J|_F^2.
  double trA = 0.0, trJ = 0.0;
  for (int t = tid; t < n; t += bd) trA += (double)K[t * ld + t];
  for (int t = tid; t < nc * n; t += bd) {
    const C v = Jl[(t / n) * ld + t % n];
    trJ += (double)v * (double)v;
  }
  {
    const int lane = tid & 63, wv = tid >> 6;
    double s0 = wave_sum(trA), s1 = wave_sum(trJ);
    if (lane == 0) { red[0][wv] = s0; red[1][wv] = s1; }
    __syncthreads();
    trA = 0.0; trJ = 0.0;
    for (int w = 0; w < bd / 64; ++w) { trA += red[0][w]; trJ += red[1][w]; }
  }
  C beta;
  if (a.rho > 0.0) beta = (C)a.rho;
  else beta = trJ > 0.0 ? (C)(trA / trJ) : (C)1;

  // K += beta J^T J (lower triangle).
  for (int t = tid; t < n * n; t += bd) {
    const int r = t / n, c = t - r * n;
    if (c <= r) {
      C s = 0;
      for (int k = 0; k < nc; ++k) s += Jl[k * ld + r] * Jl[k * ld + c];
      K[r * ld + c] += beta * s;
    }
  }
  __syncthreads();
  for (int r = tid; r < n; r += bd) {
    C dgl = K[r * ld + r];
    if (!(dgl > (C)0)) { bad = 1; dgl = (C)1; }
    sc[r] = (C)1 / dev_sqrt<C>(dgl);
  }
  __syncthreads();
  // K_hat = S K S, J_hat = J S (S = diag(sc)).
  for (int t = tid; t < n * n; t += bd) {
    const int r = t / n, c = t - r * n;
    if (c <= r) K[r * ld + c] *= sc[r] * sc[c];
  }
  for (int t = tid; t < nc * n; t += bd) {
    const int r = t / n, c = t - r * n;
    Jl[r * ld + c] *= sc[c];
  }
  __syncthreads();

  // Right-looking Cholesky K_hat = L L^T in LDS.
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      C dg = K[j * ld + j];
      if (!(dg > (C)0)) { bad = 1; dg = (C)1; }
      K[j * ld + j] = dev_sqrt<C>(dg);
    }
    __syncthreads();
    const C inv = (C)1 / K[j * ld + j];
    for (int r = j + 1 + tid; r < n; r += bd) K[r * ld + j] *= inv;
    __syncthreads();
    const int m = n - j - 1;
    for (int t = tid; t < m * m; t += bd) {
      const int rr = j + 1 + t / m, cc = j + 1 + t % m;
      if (cc <= rr) K[rr * ld + cc] -= K[rr * ld + j] * K[cc * ld + j];
    }
    __syncthreads();
  }

  // Solve K_hat X = [J_hat^T | S b]: one right-hand side per thread.
  for (int c = tid; c <= nc; c += bd) {
    C* x = X + c * ld;
    if (c < nc) {
      for (int r = 0; r < n; ++r) x[r] = Jl[c * ld + r];
    } else {
      for (int r = 0; r < n; ++r) x[r] = (C)b[r] * sc[r];
    }
    for (int r = 0; r < n; ++r) {
      C s = x[r];
      for (int k = 0; k < r; ++k) s -= K[r * ld + k] * x[k];
      x[r] = s / K[r * ld + r];
    }
    for (int r = n - 1; r >= 0; --r) {
      C s = x[r];
      for (int k = r + 1; k < n; ++k) s -= K[k * ld + r] * x[k];
      x[r] = s / K[r * ld + r];
    }
  }
  __syncthreads();

  // H = J_hat X_J, d = J_hat X_b, G = S X_J, c = S X_b.
  T* H = a.H + a.t.sub_H[i];
  T* dd = a.d + a.t.sub_slot[i];
  for (int t = tid; t < nc * (nc + 1); t += bd) {
    const int c = t / nc, r = t - c * nc;
    C s = 0;
    for (int k = 0; k < n; ++k) s += Jl[r * ld + k] * X[c * ld + k];
    if (c < nc) H[c * nc + r] = (T)s;
    else dd[r] = (T)s;
  }
  T* G = a.G + a.t.sub_J[i];
  T* cv = a.cvec + a.t.sub_dof[i];
  for (int t = tid; t < (nc + 1) * n; t += bd) {
    const int c = t / n, r = t - c * n;
    const T v = (T)(sc[r] * X[c * ld + r]);
    if (c < nc) G[c * n + r] = v;
    else cv[r] = v;
  }
  if (tid == 0) {
    a.beta[i] = (T)beta;
    if (bad) atomicOr(a.flags, FLAG_NOT_SPD);
  }
}

// ------------------------------------------------------------------------------------
// Contact projection of Eq. (21) in the scalar metric of Eq. (18): exact Signorini-
// Coulomb solution lambda_n = max(0, p_n), lambda_t = p_t clipped to the disc of radius
// mu lambda_n along p_t.
// ------------------------------------------------------------------------------------
template <typename T>
__device__ inline void contact_project(const T* p, T mu, T* lam) {
  const T ln = p[0] > (T)0 ? p[0] : (T)0;
  const T tn = dev_sqrt<T>(p[1] * p[1] + p[2] * p[2]);
  const T cap = mu * ln;
  lam[0] = ln;
  if (tn <= cap) {
    lam[1] = p[1];
    lam[2] = p[2];
  } else {
    const T f = cap / tn;
    lam[1] = f * p[1];
    lam[2] = f * p[2];
  }
}

// ------------------------------------------------------------------------------------
// Wave-level sum with DPP cross-lane moves (fixed order, so deterministic).  After the
// four in-row steps every lane of a 16-lane row holds the row sum; the two broadcast
// steps fold rows 0+1 into row 1 and rows 0..3 into row 3; lane 63 holds the total.
// ------------------------------------------------------------------------------------
__device__ inline float dpp_f(float v, int ctrl_sel) {
  int x = __float_as_int(v);
  int y;
  switch (ctrl_sel) {
    case 0: y = __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); break;   // quad_perm [1,0,3,2]
    case 1: y = __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false); break;   // quad_perm [2,3,0,1]
    case 2: y = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false); break;  // row_half_mirror
    case 3: y = __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false); break;  // row_mirror
    case 4: y = __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false); break;  // row_bcast:15
    default: y = __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false); break; // row_bcast:31
  }
  return __int_as_float(y);
}

__device__ inline double dpp_d(double v, int ctrl_sel) {
  const long long b = __double_as_longlong(v);
  int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
  int l2, h2;
  switch (ctrl_sel) {
    case 0: l2 = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false); h2 = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false); break;
    case 1: l2 = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false); h2 = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false); break;
    case 2: l2 = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false); h2 = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false); break;
    case 3: l2 = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false); h2 = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false); break;
    case 4: l2 = __builtin_amdgcn_update_dpp(0, lo, 0x142, 0xA, 0xF, false); h2 = __builtin_amdgcn_update_dpp(0, hi, 0x142, 0xA, 0xF, false); break;
    default: l2 = __builtin_amdgcn_update_dpp(0, lo, 0x143, 0xC, 0xF, false); h2 = __builtin_amdgcn_update_dpp(0, hi, 0x143, 0xC, 0xF, false); break;
  }
  const long long r = ((long long)(unsigned)h2 << 32) | (long long)(unsigned)l2;
  return __longlong_as_double(r);
}

__device__ inline float dpp_sel(float v, int k) { return dpp_f(v, k); }
__device__ inline double dpp_sel(double v, int k) { return dpp_d(v, k); }

// Sum over the 64 lanes of a wave; the result is valid in lane 63.
template <typename A>
__device__ inline A wave_total_lane63(A v) {
  v += dpp_sel(v, 0);
  v += dpp_sel(v, 1);
  v += dpp_sel(v, 2);
  v += dpp_sel(v, 3);
  v += dpp_sel(v, 4);
  v += dpp_sel(v, 5);
  return v;
}

// ------------------------------------------------------------------------------------
// Whole ADMM iteration of one scene per workgroup.  The block has at least as many
// threads as the scene has slot rows and interfaces: thread r owns slot row r and
// interface i0 + r, whose constant data stay in registers for the whole iteration.
// LDS holds the scene's H blocks and the slot vectors y, w, u.
// ------------------------------------------------------------------------------------
template <typename T, bool kHInLds>
__global__ void __launch_bounds__(1024) loop_kernel(LoopArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ T red[2][16];
  const int sc = blockIdx.x;
  const int tid = threadIdx.x;
  const int nwave = blockDim.x >> 6;
  const int lane = tid & 63, wv = tid >> 6;
  const int s0 = a.t.sc_slot[sc], s1 = a.t.sc_slot[sc + 1];
  const int ns = s1 - s0;
  const int i0 = a.t.sc_if[sc], i1 = a.t.sc_if[sc + 1];
  const int sb = a.t.sc_sub[sc], se = a.t.sc_sub[sc + 1];
  const long long h0 = a.t.sub_H[sb], h1 = a.t.sub_H[se];
  const int nh = kHInLds ? (int)(h1 - h0) : 0;
  T* Hs = reinterpret_cast<T*>(smem_raw);
  T* y = Hs + nh;
  T* w = y + ns;
  T* u = w + ns;

  // stage the scene's H_i blocks (contiguous in global memory)
  for (int q = tid; q < nh; q += blockDim.x) Hs[q] = a.H[h0 + q];
  const T* Hbase = kHInLds ? Hs : a.H + h0;

  // slot row owned by this thread
  const bool has_slot = tid < ns;
  int nc = 0, so = 0, hoff = 0;
  T be = (T)0, dr = (T)0;
  if (has_slot) {
    const int g = s0 + tid;
    const int i = a.t.slot_sub[g];
    nc = a.t.sub_nc[i];
    so = a.t.sub_slot[i] - s0;
    hoff = (int)(a.t.sub_H[i] - h0) + a.t.slot_loc[g];
    be = a.beta[i];
    dr = a.d[g];
    // warm start: w^0 = beta z^0 - u^0, y^0 = beta z^0 + u^0
    const T z0 = a.z_in ? a.z_in[g] : (T)0;
    const T u0 = a.u_in ? a.u_in[g] : (T)0;
    w[tid] = be * z0 - u0;
    y[tid] = be * z0 + u0;
    u[tid] = u0;
  }
  // interface owned by this thread
  const int j = i0 + tid;
  const bool has_if = j < i1;
  int kind = 0, dim = 0, two = 0, p0 = 0, p1 = 0;
  T ib0 = (T)0, ib1 = (T)0, iws = (T)0, mu = (T)0;
  T ev[kMaxIfDim];
  if (has_if) {
    kind = a.t.if_kind[j];
    dim = a.t.if_dim[j];
    two = a.t.if_nsub[j] == 2;
    p0 = a.t.if_slot0[j] - s0;
    p1 = two ? a.t.if_slot1[j] - s0 : p0;
    ib0 = (T)1 / a.beta[a.t.if_sub0[j]];
    ib1 = two ? (T)1 / a.beta[a.t.if_sub1[j]] : (T)0;
    iws = (T)1 / (ib0 + ib1);
    mu = a.mu[j];
    for (int k = 0; k < kMaxIfDim; ++k) ev[k] = k < dim ? a.e[a.t.if_row[j] + k] : (T)0;
  }
  __syncthreads();

  int it = 0, conv = 0;
  double th = 0.0, rth = 0.0;
  for (int l = 0; l < a.max_iters; ++l) {
    it = l + 1;
    // x-update (Eq. 15 reassociated): x = d + H w; y = beta x + u (Eq. 18).
    T pth = (T)0, pyy = (T)0;
    if (has_slot) {
      const T* Hr = Hbase + hoff;
      const T* wr = w + so;
      T x0 = dr, x1 = (T)0, x2 = (T)0, x3 = (T)0;
      int c = 0;
      for (; c + 4 <= nc; c += 4) {
        x0 += Hr[(c + 0) * nc] * wr[c + 0];
        x1 += Hr[(c + 1) * nc] * wr[c + 1];
        x2 += Hr[(c + 2) * nc] * wr[c + 2];
        x3 += Hr[(c + 3) * nc] * wr[c + 3];
      }
      for (; c < nc; ++c) x0 += Hr[c * nc] * wr[c];
      const T x = (x0 + x1) + (x2 + x3);
      const T yn = be * x + u[tid];
      const T df = yn - y[tid];
      pth = df * df;
      pyy = yn * yn;
      y[tid] = yn;
    }
    // Residual of Eq. (22) and |y|^2, reduced in a fixed order.
    pth = wave_total_lane63(pth);
    pyy = wave_total_lane63(pyy);
    if (lane == 63) { red[0][wv] = pth; red[1][wv] = pyy; }
    __syncthreads();
    T tt = (T)0, ty = (T)0;
    for (int q = 0; q < nwave; ++q) { tt += red[0][q]; ty += red[1][q]; }
    th = (double)tt;
    const double yn2 = __builtin_sqrt((double)ty);
    rth = __builtin_sqrt(th) / (yn2 > 1e-12 ? yn2 : 1e-12);
    if (!__builtin_isfinite(rth)) {
      if (tid == 0) atomicOr(a.flags, FLAG_NONFINITE);
      break;
    }
    if (rth <= a.tol) { conv = 1; break; }
    if (l + 1 == a.max_iters) break;

    // z-update (Eq. 16-21) and dual update (Eq. 14): u = -lambda, w = y + 2 lambda.
    if (has_if) {
      T p[kMaxIfDim], lam[kMaxIfDim];
#pragma unroll
      for (int k = 0; k < kMaxIfDim; ++k) {
        if (k < dim) {
          T s = ev[k] + y[p0 + k] * ib0;
          if (two) s += y[p1 + k] * ib1;
          p[k] = -s * iws;
        }
      }
      if (kind == KIND_CONTACT) {
        contact_project<T>(p, mu, lam);
      } else if (kind == KIND_HARD_INEQ) {
#pragma unroll
        for (int k = 0; k < kMaxIfDim; ++k) lam[k] = p[k] > (T)0 ? p[k] : (T)0;
      } else {
#pragma unroll
        for (int k = 0; k < kMaxIfDim; ++k) lam[k] = p[k];
      }
#pragma unroll
      for (int k = 0; k < kMaxIfDim; ++k) {
        if (k < dim) {
          u[p0 + k] = -lam[k];
          w[p0 + k] = y[p0 + k] + (T)2 * lam[k];
          if (two) {
            u[p1 + k] = -lam[k];
            w[p1 + k] = y[p1 + k] + (T)2 * lam[k];
          }
        }
      }
    }
    __syncthreads();
  }
  __syncthreads();

  // v_hat = c + G w (from the last x-update's w).
  const int d0 = a.t.sc_dof[sc], d1 = a.t.sc_dof[sc + 1];
  for (int dg = d0 + tid; dg < d1; dg += blockDim.x) {
    int i = sb;
    while (i + 1 < se && a.t.sub_dof[i + 1] <= dg) ++i;
    const int n = a.t.sub_n[i];
    const int r = dg - a.t.sub_dof[i];
    const int nci = a.t.sub_nc[i];
    const int soi = a.t.sub_slot[i] - s0;
    const T* G = a.G + a.t.sub_J[i] + r;
    T v = a.cvec[dg];
    for (int c = 0; c < nci; ++c) v += G[c * n] * w[soi + c];
    if (a.v_hat) a.v_hat[dg] = v;
  }
  // final z^l, u^l and lambda = -u.
  if (has_slot) {
    a.z_out[s0 + tid] = (w[tid] + u[tid]) / be;
    a.u_out[s0 + tid] = u[tid];
  }
  if (a.lambda && has_if) {
    for (int k = 0; k < dim; ++k) a.lambda[a.t.if_row[j] + k] = -u[p0 + k];
  }
  if (tid == 0) {
    a.st_iters[sc] = it;
    a.st_total[sc] += it;
    if (!conv) a.st_unconv[sc] += 1;
    a.st_conv[sc] = conv;
    a.st_theta[sc] = th;
    a.st_rtheta[sc] = rth;
  }
}

template <typename T>
hipError_t launch_factor(const FactorArgs<T>& a, int count, int max_n, int max_nc, bool fp64, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const size_t ld = (size_t)(max_n | 1);
  const size_t cs = fp64 ? sizeof(double) : sizeof(T);
  const size_t lds = cs * (ld * max_n + ld * max_nc + ld * (max_nc + 1) + (size_t)max_n);
  if (lds > 160 * 1024 - 1024) return hipErrorInvalidValue;
  if (fp64)
    hipLaunchKernelGGL((factor_kernel<T, double>), dim3(count), dim3(128), lds, s, a);
  else
    hipLaunchKernelGGL((factor_kernel<T, T>), dim3(count), dim3(128), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_loop(const LoopArgs<T>& a, int max_slot_scene, int max_if_scene, long long max_h_scene,
                       hipStream_t s) {
  if (a.t.n_scene == 0) return hipSuccess;
  const int need = max_slot_scene > max_if_scene ? max_slot_scene : max_if_scene;
  const int threads = ((need > 0 ? need : 1) + 63) / 64 * 64;
  if (threads > 1024) return hipErrorInvalidValue;
  const size_t slots = sizeof(T) * 3 * (size_t)(max_slot_scene > 0 ? max_slot_scene : 1);
  const size_t with_h = slots + sizeof(T) * (size_t)max_h_scene;
  if (with_h <= 150 * 1024) {
    hipLaunchKernelGGL((loop_kernel<T, true>), dim3(a.t.n_scene), dim3(threads), with_h, s, a);
  } else {
    if (slots > 150 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL((loop_kernel<T, false>), dim3(a.t.n_scene), dim3(threads), slots, s, a);
  }
  return hipGetLastError();
}

template hipError_t launch_factor<float>(const FactorArgs<float>&, int, int, int, bool, hipStream_t);
template hipError_t launch_factor<double>(const FactorArgs<double>&, int, int, int, bool, hipStream_t);
template hipError_t launch_loop<float>(const LoopArgs<float>&, int, int, long long, hipStream_t);
template hipError_t launch_loop<double>(const LoopArgs<double>&, int, int, long long, hipStream_t);

}  // namespace subadmm
