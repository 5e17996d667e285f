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
#include "rigid_device.hpp"

namespace subadmm {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Orders the LDS accesses of one wave's lanes (a wave's LDS instructions complete in
// issue order; the fences keep the compiler from moving accesses across this point).
__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The threads that factorise one subsystem: the whole workgroup (workgroup barriers), or
// one wave (its 64 lanes, wave-level fences), so that the waves of a workgroup factorise
// different small subsystems at the same time.
struct GroupWg {
  static constexpr bool kWave = false;
  __device__ static int rank() { return threadIdx.x; }
  __device__ static int size() { return blockDim.x; }
  __device__ static void sync() { __syncthreads(); }
};
struct GroupWave {
  static constexpr bool kWave = true;
  __device__ static int rank() { return threadIdx.x & 63; }
  __device__ static int size() { return 64; }
  __device__ static void sync() { wave_lds_fence(); }
};

// Subsystems a single wave factorises: every column loop fits its 64 lanes (n <= 64, at
// most 64 right-hand sides) and the working arrays fit the wave's share of LDS.
__host__ __device__ inline bool wave_factor_fits(int n, int nc, size_t cs, size_t slice) {
  return n <= 64 && nc + 1 <= 64 && factor_bytes(n, nc, cs) <= slice;
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
// Factorisation of subsystem i by the thread group Grp (the workgroup or one wave), with its
// working arrays at sm (LDS, or a global scratch area of the same layout); red (workgroup
// form only) and bad are scratch shared by the group.  Every entry is formed by one thread
// with the same arithmetic in either form; only the trace sums of Eq. 23 are added in
// another grouping.
template <typename T, typename C, typename Grp = GroupWg>
__device__ __attribute__((always_inline)) inline void factor_body(const FactorArgs<T>& a, const int i, C* sm,
                                                                 double (*red)[8], int& bad) {
  const int tid = Grp::rank();
  const int bd = Grp::size();
  const int n = a.t.sub_n[i];
  const int nc = a.t.sub_nc[i];
  // LDS leading dimensions are odd so that strided accesses fall in distinct banks
  const int ld = n | 1;
  C* K = sm;                   // n x n, row-major with leading dimension ld, lower used
  C* X = K + n * ld;           // (nc + 1) columns of length n, column stride ld: J rows, then b,
                               // solved in place
  C* Jl = X;                   // the first nc columns: J (nc x n, row-major, leading dimension ld)
  C* sc = X + (nc + 1) * ld;   // Jacobi scaling 1/sqrt(K_rr)
  C* dinv = sc + n;            // 1 / L_kk

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
  for (int t = tid; t < n; t += bd) X[nc * ld + t] = (C)b[t];
  Grp::sync();

  // Eq. (23): beta_i = Tr(A_i) / Tr(J^T J); Tr(J^T J) = |J|_F^2.
  double trA = 0.0, trJ = 0.0;
  for (int t = tid; t < n; t += bd) trA += (double)K[t * ld + t];
  for (int t = tid; t < nc * n; t += bd) {
    const C v = Jl[(t / n) * ld + t % n];
    trJ += (double)v * (double)v;
  }
  if constexpr (Grp::kWave) {
    trA = wave_sum(trA);
    trJ = wave_sum(trJ);
  } else {
    const int lane = tid & 63, wv = tid >> 6;
    double s0 = wave_sum(trA), s1 = wave_sum(trJ);
    if (lane == 0) { red[0][wv] = s0; red[1][wv] = s1; }
    Grp::sync();
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
  Grp::sync();
  for (int r = tid; r < n; r += bd) {
    C dgl = K[r * ld + r];
    if (!(dgl > (C)0)) { bad = 1; dgl = (C)1; }
    sc[r] = (C)1 / dev_sqrt<C>(dgl);
  }
  Grp::sync();
  // K_hat = S K S, J_hat = J S (S = diag(sc)).
  for (int t = tid; t < n * n; t += bd) {
    const int r = t / n, c = t - r * n;
    if (c <= r) K[r * ld + c] *= sc[r] * sc[c];
  }
  for (int t = tid; t < (nc + 1) * n; t += bd) {
    const int r = t / n, c = t - r * n;
    X[r * ld + c] *= sc[c];  // J_hat rows, then S b
  }
  Grp::sync();

  // Right-looking Cholesky K_hat = L L^T in LDS, one barrier per column: step j updates the
  // trailing lower triangle with the unscaled column j and pivot d_j (K -= k_j k_j^T / d_j),
  // leaving column j as it is; a final pass scales column j by 1/sqrt(d_j).
  for (int j = 0; j + 1 < n; ++j) {
    const int m = n - j - 1;
    const int R = bd / m;  // row groups (m < 64 <= bd)
    const int cc = j + 1 + tid % m, rg = tid / m;
    if (rg < R) {
      const C dg = K[j * ld + j];
      const C invd = dg > (C)0 ? (C)1 / dg : (C)1;
      const C kc = K[cc * ld + j] * invd;
      for (int rr = j + 1 + rg; rr < n; rr += R)
        if (cc <= rr) K[rr * ld + cc] -= K[rr * ld + j] * kc;
    }
    Grp::sync();
  }
  for (int j = tid; j < n; j += bd) {
    C dg = K[j * ld + j];
    if (!(dg > (C)0)) { bad = 1; dg = (C)1; }
    dinv[j] = dev_sqrt<C>(dg);  // L_jj (dinv is reused for 1 / L_jj below)
  }
  Grp::sync();
  for (int t = tid; t < n * n; t += bd) {
    const int r = t / n, j = t - r * n;
    if (j <= r) K[r * ld + j] = r == j ? dinv[j] : K[r * ld + j] / dinv[j];
  }
  Grp::sync();

  // T = L^-1 [J_hat^T | S b] by forward substitution in place, then H = T_J^T T_J and
  // d = T_J^T T_b (= J_hat K_hat^-1 J_hat^T and J_hat K_hat^-1 S b), then back substitution
  // in place gives K_hat^-1 [J_hat^T | S b] for G and c.  With at most one right-hand side
  // per thread: each sweep by columns of L for all right-hand sides at once, each step k
  // parallel over (row, right-hand side) pairs with one barrier; X keeps the numerators,
  // which are multiplied by 1/L_kk where used and once at the end of each sweep.
  T* H = a.H + a.t.sub_H[i];
  T* dd = a.d + a.t.sub_slot[i];
  const int m = nc + 1;
  if (m <= bd) {
    const int R = bd / m;  // row groups
    const int c = tid % m, rg = tid / m;
    const bool act = rg < R;
    C* x = X + c * ld;
    for (int r = tid; r < n; r += bd) dinv[r] = (C)1 / K[r * ld + r];
    Grp::sync();
    // Four pivot rows per barrier: every thread of column c forms the block's pivots in the
    // unblocked order (so the result is the same), updates its trailing rows, and after the
    // barrier (when no thread reads them any more) the row group 0 thread stores the block's
    // completed numerators.
    constexpr int B = 4;
    for (int k = 0; k + 1 < n; k += B) {
      C num[B], piv[B];
      const int nb = n - k < B ? n - k : B;
      if (act) {
#pragma unroll
        for (int q = 0; q < B; ++q) {
          if (q < nb) {
            C v = x[k + q];
            for (int p = 0; p < q; ++p) v -= K[(k + q) * ld + k + p] * piv[p];
            num[q] = v;
            piv[q] = v * dinv[k + q];
          }
        }
        for (int r = k + B + rg; r < n; r += R) {
          C v = x[r];
#pragma unroll
          for (int p = 0; p < B; ++p) v -= K[r * ld + k + p] * piv[p];
          x[r] = v;
        }
      }
      Grp::sync();
      if (act && rg == 0) {
        for (int q = 1; q < nb; ++q) x[k + q] = num[q];
      }
    }
    Grp::sync();
    if (act) {
      for (int r = rg; r < n; r += R) x[r] *= dinv[r];
    }
    Grp::sync();
    for (int t = tid; t < nc * (nc + 1); t += bd) {
      const int cc = t / nc, r = t - cc * nc;
      C s = 0;
      for (int k = 0; k < n; ++k) s += X[r * ld + k] * X[cc * ld + k];
      if (cc < nc) H[cc * nc + r] = (T)s;
      else dd[r] = (T)s;
    }
    Grp::sync();
    for (int k = n - 1; k > 0; k -= B) {
      C num[B], piv[B];
      const int nb = k + 1 < B ? k + 1 : B;
      if (act) {
#pragma unroll
        for (int q = 0; q < B; ++q) {
          if (q < nb) {
            C v = x[k - q];
            for (int p = 0; p < q; ++p) v -= K[(k - p) * ld + k - q] * piv[p];
            num[q] = v;
            piv[q] = v * dinv[k - q];
          }
        }
        for (int r = rg; r + B <= k; r += R) {
          C v = x[r];
#pragma unroll
          for (int p = 0; p < B; ++p) v -= K[(k - p) * ld + r] * piv[p];
          x[r] = v;
        }
      }
      Grp::sync();
      if (act && rg == 0) {
        for (int q = 1; q < nb; ++q) x[k - q] = num[q];
      }
    }
    Grp::sync();
    if (act) {
      for (int r = rg; r < n; r += R) x[r] *= dinv[r];
    }
  } else {
    for (int c = tid; c <= nc; c += bd) {  // one right-hand side per thread
      C* x = X + c * ld;
      for (int r = 0; r < n; ++r) {
        C s = x[r];
        for (int k = 0; k < r; ++k) s -= K[r * ld + k] * x[k];
        x[r] = s / K[r * ld + r];
      }
    }
    Grp::sync();
    for (int t = tid; t < nc * (nc + 1); t += bd) {
      const int cc = t / nc, r = t - cc * nc;
      C s = 0;
      for (int k = 0; k < n; ++k) s += X[r * ld + k] * X[cc * ld + k];
      if (cc < nc) H[cc * nc + r] = (T)s;
      else dd[r] = (T)s;
    }
    Grp::sync();
    for (int c = tid; c <= nc; c += bd) {
      C* x = X + c * ld;
      for (int r = n - 1; r >= 0; --r) {
        C s = x[r];
        for (int k = r + 1; k < n; ++k) s -= K[k * ld + r] * x[k];
        x[r] = s / K[r * ld + r];
      }
    }
  }
  Grp::sync();

  // G = S X_J, c = S X_b.
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

template <typename T, typename C>
__global__ void __launch_bounds__(512) factor_kernel(FactorArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[2][8];
  __shared__ int bad;
  factor_body<T, C>(a, a.order[a.first + blockIdx.x], reinterpret_cast<C*>(smem_raw), red, bad);
}

// Subsystems whose working arrays exceed the LDS: the same factorisation with its working
// arrays in device memory (scr + off[i] bytes), one 512-thread workgroup each (a workgroup's
// barriers order its device-memory accesses as they do its LDS accesses).
template <typename T, typename C>
__global__ void __launch_bounds__(512) factor_global_kernel(FactorArgs<T> a, char* scr, const int64_t* off) {
  __shared__ double red[2][8];
  __shared__ int bad;
  const int i = a.order[a.first + blockIdx.x];
  factor_body<T, C>(a, i, reinterpret_cast<C*>(scr + off[i]), red, bad);
}

// Small subsystems: each wave of a 256-thread workgroup factorises one subsystem in its
// quarter of the LDS (slice bytes), with no workgroup barrier.
template <typename T, typename C>
__global__ void __launch_bounds__(256) factor_wave_kernel(FactorArgs<T> a, int count, int slice) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int bad[4];
  const int wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 4 + wv;
  if (k >= count) return;
  factor_body<T, C, GroupWave>(a, a.order[a.first + k], reinterpret_cast<C*>(smem_raw + (size_t)wv * slice), nullptr,
                               bad[wv]);
}

// ------------------------------------------------------------------------------------
// Contact projection of Eq. (21) in the scalar metric of Eq. (18): exact Signorini-
// Coulomb solution lambda_n = max(0, p_n), lambda_t = p_t clipped to the disc of radius
// mu lambda_n along p_t.
// ------------------------------------------------------------------------------------
template <typename T>
__device__ inline T disc_scale(T cap, T tn2);
template <>
__device__ inline float disc_scale<float>(float cap, float tn2) {
  // The hardware reciprocal square root reads a denormal input as zero: a tangential part
  // below ~1e-19 (tn2 under the smallest normal float, met on separating contacts at rest)
  // would give cap * inf, NaN for cap = 0.  Such inputs take the FP64 square root, where
  // every FP32 value is normal.
  if (!(cap > 0.0f)) return 0.0f;
  if (tn2 >= __FLT_MIN__) return cap * __builtin_amdgcn_rsqf(tn2);
  return (float)((double)cap / __builtin_sqrt((double)tn2));
}
template <>
__device__ inline double disc_scale<double>(double cap, double tn2) { return cap / __builtin_sqrt(tn2); }

// Tested on squares (|p_t|^2 > (mu lambda_n)^2); the disc scale mu lambda_n / |p_t| uses the
// hardware reciprocal square root in FP32 (1 ulp; FP64 for inputs below the normal range)
// and the correctly rounded forms in FP64.
template <typename T>
__device__ inline void contact_project(const T* p, T mu, T* lam, int model) {
  if (model == 1) {
    cone_project<T>(p, mu, lam);
    return;
  }
  const T ln = p[0] > (T)0 ? p[0] : (T)0;
  const T tn2 = p[1] * p[1] + p[2] * p[2];
  const T cap = mu * ln;
  lam[0] = ln;
  if (tn2 > cap * cap) {
    const T f = disc_scale<T>(cap, tn2);
    lam[1] = f * p[1];
    lam[2] = f * p[2];
  } else {
    lam[1] = p[1];
    lam[2] = p[2];
  }
}

// e + ya ib0 + yb ib1 (the bracket of Eq. 17-21) and the soft z-update of Eq. 20,
// lambda = -k (e + alpha sum y/beta) / (1 + w alpha k), with explicit fused multiply-adds,
// so that every form of the z-update rounds the same way.
__device__ inline float zfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double zfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T>
__device__ inline T zsum(T e, T ya, T ib0, T yb, T ib1) {
  return zfma(yb, ib1, zfma(ya, ib0, e));
}
template <typename T>
__device__ inline T zsoft(T e, T ya, T ib0, T yb, T ib1, T k, T alpha) {
  return -k * zfma(alpha, zfma(yb, ib1, ya * ib0), e) / zfma(alpha * k, ib0 + ib1, (T)1);
}

// z-update (Eq. 16-21) and dual update (Eq. 14) of one interface of a fixed class, with
// the loops over its rows at their real length.

// z-update (Eq. 16-21) and dual update (Eq. 14) of an interface with more than two members
// (|S_j| up to 4): the bracket of Eq. 17-21 sums e_j and y_i / beta_i over every member and
// the weight w = sum 1/beta_i; lambda then acts on every member alike.  Member slots are
// read from the topology tables: y, u at slot - s0 (scene-local), w at the member's w
// offset (padded per-subsystem blocks when kPadW).  Used for the rare interfaces of this
// kind only, so the per-thread state of the common ones stays as it is.
template <typename T, bool kPadW>
__device__ inline void z_update_multi(const LoopArgs<T>& a, const int j, const int s0, const T* ev, const T* y,
                                      T* u, T* w) {
  const int nm = a.t.if_nsub[j], dim = a.t.if_dim[j], kind = a.t.if_kind[j];
  int ps[kMaxMembers], qs[kMaxMembers];
  T ib[kMaxMembers];
  T wsum = (T)0;
  for (int m = 0; m < kMaxMembers; ++m) {
    ps[m] = qs[m] = 0;
    ib[m] = (T)0;
    if (m >= nm) continue;
    const int i = m == 0 ? a.t.if_sub0[j] : m == 1 ? a.t.if_sub1[j] : a.t.if_subx[2 * j + m - 2];
    const int g = m == 0 ? a.t.if_slot0[j] : m == 1 ? a.t.if_slot1[j] : a.t.if_slotx[2 * j + m - 2];
    ps[m] = g - s0;
    qs[m] = (kPadW ? a.t.sub_wq[i] : a.t.sub_slot[i] - s0) + (g - a.t.sub_slot[i]);
    ib[m] = (T)1 / a.beta[i];
    wsum += ib[m];
  }
  T p[kMaxIfDim], lam[kMaxIfDim];
  for (int k = 0; k < kMaxIfDim; ++k) {
    p[k] = (T)0;
    if (k >= dim) continue;
    T sy = (T)0;
    for (int m = 0; m < nm; ++m) sy += y[ps[m] + k] * ib[m];
    p[k] = kind == KIND_SOFT ? -a.ksoft[j] * (ev[k] + a.asoft[j] * sy) / ((T)1 + wsum * a.asoft[j] * a.ksoft[j])
                             : -(ev[k] + sy) / wsum;
  }
  T cl[3];
  contact_project<T>(p, a.mu[j], cl, a.contact_model);
  for (int k = 0; k < kMaxIfDim; ++k) {
    T v = p[k];
    if (kind == KIND_HARD_INEQ) v = v > (T)0 ? v : (T)0;
    if (kind == KIND_CONTACT && k < 3) v = cl[k];
    lam[k] = v;
  }
  for (int m = 0; m < nm; ++m)
    for (int k = 0; k < dim; ++k) {
      const T yk = y[ps[m] + k];
      u[ps[m] + k] = -lam[k];
      w[qs[m] + k] = yk + (T)2 * lam[k];
    }
}

template <typename T, int D, int KIND>
__device__ inline void z_update_fixed(const T* ev, T ib0, T ib1, T iws, T mu, int p0, int p1, int q0, int q1,
                                      const T* y, T* u, T* w, int model) {
  T ya[D], yb[D], lam[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    ya[k] = y[p0 + k];
    yb[k] = y[p1 + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) lam[k] = -zsum(ev[k], ya[k], ib0, yb[k], ib1) * iws;
  if (KIND == KIND_CONTACT) {
    const T p3[3] = {lam[0], lam[1], lam[2]};
    contact_project<T>(p3, mu, lam, model);
  } else if (KIND == KIND_HARD_INEQ) {
#pragma unroll
    for (int k = 0; k < D; ++k) lam[k] = lam[k] > (T)0 ? lam[k] : (T)0;
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    u[p0 + k] = -lam[k];
    w[q0 + k] = ya[k] + (T)2 * lam[k];
  }
  if (p1 != p0) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      u[p1 + k] = -lam[k];
      w[q1 + k] = yb[k] + (T)2 * lam[k];
    }
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
// Whole ADMM iteration of one scene per workgroup.
//
// Slot row r is owned by lane kLanes*r (kLanes = 1 or 2 lanes share its dot product,
// combined with a DPP swap); kLanes = 0: a host map gives each lane its row and part, a
// row taking 1, 2 or 4 aligned lanes (combined with quad DPP).  Interface i0 + t is owned
// by thread t.  Their constant data stay in registers for the whole iteration.
//
// Every form adds a lane's share of a row's 16-byte vector products in one order: in groups
// of four, the t-th vector of a group to partial sum t mod 4, the vectors after the last full
// group to partial 0, and the lane's sum is (p0 + p1) + (p2 + p3); the lanes of a split row
// then add their sums pairwise, then by quads.
//
// LDS (kHInLds): the scene's H_i in a blocked layout of 16-byte vectors, vector
// (cb, r) = H_i[r][V*cb .. V*cb + V-1] at sub_hq[i] + cb * nc_i + r (zero padded), so
// that consecutive lanes of one subsystem read consecutive vectors; w in per-subsystem
// blocks padded to a multiple of V (read as broadcast vectors); y and u per slot row.
// Without kHInLds H is read from global memory in its plain column-major layout.
// Every phase issues its loads before their first use.
// ------------------------------------------------------------------------------------
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int N = 4;
  __device__ static float dot(const float4& a, const float4& b) {
    return (a.x * b.x + a.y * b.y) + (a.z * b.z + a.w * b.w);
  }
  __device__ static float get(const float4& a, int q) { return q == 0 ? a.x : q == 1 ? a.y : q == 2 ? a.z : a.w; }
  __device__ static float4 make(const float* v) { return make_float4(v[0], v[1], v[2], v[3]); }
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int N = 2;
  __device__ static double dot(const double2& a, const double2& b) { return a.x * b.x + a.y * b.y; }
  __device__ static double get(const double2& a, int q) { return q == 0 ? a.x : a.y; }
  __device__ static double2 make(const double* v) { return make_double2(v[0], v[1]); }
};

// Where the iteration kernel reads H_i: global memory or LDS (blocked layout).
constexpr int kHGlobal = 0, kHLds = 1;

template <typename T>
__device__ inline T pair_sum(T v) {
  return v + dpp_sel(v, 0);  // quad_perm [1,0,3,2]: adds the neighbouring lane
}

// Partial sums of one lane's share of x_r = H_i[r] . w_i from the blocked LDS layout: the
// row's vectors part, part + kp, ... (count cnt), H vector stride hs, w vector stride kp.
template <typename T, typename VT>
__device__ inline T row_dot_share(const VT* Hv, const VT* Wv, int cnt, int hs, int kp) {
  T acc[4] = {(T)0, (T)0, (T)0, (T)0};
  int t = 0;
  for (; t + 3 < cnt; t += 4) {
    VT hv[4], wq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      hv[k] = Hv[(t + k) * hs];
      wq[k] = Wv[(t + k) * kp];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += Vec16<T>::dot(hv[k], wq[k]);
  }
  for (; t < cnt; ++t) acc[0] += Vec16<T>::dot(Hv[t * hs], Wv[t * kp]);
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// The whole iteration of scene sc by the workgroup; smem_raw is the dynamic LDS area, red a
// workgroup-shared scratch for the residual sums.
template <typename T, int kHMode, int kLanes>
__device__ __attribute__((always_inline)) inline void loop_body(const LoopArgs<T>& a, const int sc,
                                                               unsigned char* smem_raw, T (*red)[8]) {
  static_assert(kLanes > 0 || kHMode == 1, "split rows need the LDS layout");
  using VT = typename Vec16<T>::type;
  constexpr int V = Vec16<T>::N;
  constexpr bool kHInLds = kHMode == kHLds;
  constexpr bool kPadW = kHInLds;  // w in padded per-subsystem blocks
  const int tid = threadIdx.x;
  const int bd = blockDim.x;
  const int nwave = bd >> 6;
  const int lane = tid & 63, wv = tid >> 6;
  if (a.skip_converged && a.skip_converged[sc]) return;
  const int s0 = a.t.sc_slot[sc], s1 = a.t.sc_slot[sc + 1];
  const int ns = s1 - s0;
  const int i0 = a.t.sc_if[sc], i1 = a.t.sc_if[sc + 1];
  const int sb = a.t.sc_sub[sc], se = a.t.sc_sub[sc + 1];
  const long long h0 = a.t.sub_H[sb];
  const int nhq = kHInLds ? a.t.sc_hq[sc] : 0;
  const int nwq = kPadW ? a.t.sc_wq[sc] : ns;
  VT* Hq = reinterpret_cast<VT*>(smem_raw);
  T* w = reinterpret_cast<T*>(Hq + nhq);  // padded blocks (kPadW) or per slot row
  T* y = w + nwq;
  T* u = y + ns;

  if (kHInLds) {
    // stage H_i into the blocked layout and clear the padded w area
    for (int i = sb; i < se; ++i) {
      const int nci = a.t.sub_nc[i];
      const int nq = (nci + V - 1) / V;
      const T* Hg = a.H + a.t.sub_H[i];
      VT* dst = Hq + a.t.sub_hq[i];
      for (int q = tid; q < nq * nci; q += bd) {
        const int cb = q / nci, rr = q - cb * nci;
        T v[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const int c = cb * V + k;
          v[k] = c < nci ? Hg[c * nci + rr] : (T)0;
        }
        dst[q] = Vec16<T>::make(v);
      }
    }
    for (int q = tid; q < nwq; q += bd) w[q] = (T)0;
    __syncthreads();
  }

  // slot row handled by this lane (and the lane's share of its dot product)
  int r, part, kp;
  if constexpr (kLanes == 0) {
    const int code = a.t.rmap[(size_t)sc * bd + tid];
    r = code >= 0 ? code >> 5 : ns;
    kp = code >= 0 ? (code >> 2) & 7 : 1;
    part = code >= 0 ? code & 3 : 0;
  } else {
    r = tid / kLanes;
    part = tid - r * kLanes;
    kp = kLanes;
  }
  const bool in_slot = r < ns;
  const bool owner = in_slot && part == 0;
  int nc = 0, hoff = 0, wo = 0, loc = 0;
  T be = (T)0, dr = (T)0;
  if (in_slot) {
    const int g = s0 + r;
    const int i = a.t.slot_sub[g];
    nc = a.t.sub_nc[i];
    loc = a.t.slot_loc[g];
    if (kHInLds) {
      hoff = a.t.sub_hq[i] + loc;
      wo = a.t.sub_wq[i];
    } else {
      hoff = (int)(a.t.sub_H[i] - h0) + loc;
      wo = a.t.sub_slot[i] - s0;
    }
    be = a.beta[i];
    dr = a.d[g];
    if (owner) {
      // warm start: w^0 = beta z^0 - u^0, y^0 = beta z^0 + u^0
      const T z0 = a.z_in ? a.z_in[g] : (T)0;
      const T u0 = a.u_in ? a.u_in[g] : (T)0;
      w[wo + loc] = be * z0 - u0;
      y[r] = be * z0 + u0;
      u[r] = u0;
    }
  }
  // interface owned by this thread (waves hold one interface class when the map is given)
  const bool use_map = a.t.zmap && a.t.zmap_block == bd;
  const int code = use_map ? a.t.zmap[(long)sc * bd + tid] : i0 + tid;
  // a map entry is an interface, or one row of an interface whose rows are independent
  // (equality, hard and soft rows of one or two members): j | (row + 1) << kZRowShift
  const int j = code >= 0 ? (code & kZIfMask) : code;
  const int zrow = code >= 0 ? (code >> kZRowShift) - 1 : -1;
  const bool has_if = use_map ? j >= 0 : j < i1;
  int kind = 0, dim = 0, p0 = 0, p1 = 0, q0 = 0, q1 = 0, erow = 0;
  bool multi = false;
  T ib0 = (T)0, ib1 = (T)0, iws = (T)0, mu = (T)0, ksj = (T)0, asj = (T)0;
  // the scene's e rows are staged in LDS after u (read by the z-update with its y loads
  // rather than held in registers for the whole iteration)
  T* el = u + ns;
  const int row0 = a.t.if_row[i0];
  for (int q = tid; q < a.t.if_row[i1] - row0; q += bd) el[q] = a.e[row0 + q];
  const T* ev = el;
  if (has_if) {
    kind = a.t.if_kind[j];
    dim = a.t.if_dim[j];
    multi = a.t.if_nsub[j] > 2;
    const bool two = a.t.if_nsub[j] == 2;
    const int sa = a.t.if_sub0[j];
    const int sbb = two ? a.t.if_sub1[j] : sa;
    const int k0 = zrow >= 0 ? zrow : 0;  // first row of this lane's share
    if (zrow >= 0) dim = 1;
    p0 = a.t.if_slot0[j] - s0 + k0;
    p1 = two ? a.t.if_slot1[j] - s0 + k0 : p0;
    const int wa = kPadW ? a.t.sub_wq[sa] : a.t.sub_slot[sa] - s0;
    const int wb = kPadW ? a.t.sub_wq[sbb] : a.t.sub_slot[sbb] - s0;
    q0 = wa + (a.t.if_slot0[j] - a.t.sub_slot[sa]) + k0;
    q1 = two ? wb + (a.t.if_slot1[j] - a.t.sub_slot[sbb]) + k0 : q0;
    ib0 = (T)1 / a.beta[sa];
    ib1 = two ? (T)1 / a.beta[sbb] : (T)0;
    iws = (T)1 / (ib0 + ib1);
    mu = a.mu[j];
    ksj = a.ksoft[j];
    asj = a.asoft[j];
    erow = a.t.if_row[j] + k0;
    ev = el + (erow - row0);
  }
  const T tol2 = (T)(a.tol * a.tol);
  // partials of absent waves stay zero, so that all eight are read as vectors
  if (tid < 16) red[tid >> 3][tid & 7] = (T)0;
  __syncthreads();

  int it = 0, conv = 0;
  T th = (T)0, yy = (T)0;
  for (int l = 0; l < a.max_iters; ++l) {
    it = l + 1;
    // x-update (Eq. 15 reassociated): x = d + H w; y = beta x + u (Eq. 18).
    T x = (T)0;
    if (in_slot) {
      if (kHInLds) {
        const int nq = (nc + V - 1) / V;
        const int cnt = (nq - part + kp - 1) / kp;
        x = row_dot_share<T, VT>(Hq + hoff + part * nc, reinterpret_cast<const VT*>(w + wo) + part, cnt, kp * nc,
                                 kp);
      } else {
        const T* Hr = a.H + h0 + hoff;
        const T* wr = w + wo;
        T acc[4] = {(T)0, (T)0, (T)0, (T)0};
        int c = part;
        for (; c + 3 * kLanes < nc; c += 4 * kLanes) {
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[k] += Hr[(c + k * kLanes) * nc] * wr[c + k * kLanes];
        }
        for (; c < nc; c += kLanes) acc[0] += Hr[c * nc] * wr[c];
        x = (acc[0] + acc[1]) + (acc[2] + acc[3]);
      }
    }
    if (kLanes == 2) x = pair_sum(x);
    if (kLanes == 0) {
      const T s2 = x + dpp_sel(x, 0);   // quad_perm [1,0,3,2]: the pair's sum
      const T s4 = s2 + dpp_sel(s2, 1);  // quad_perm [2,3,0,1]: the quad's sum
      x = kp == 1 ? x : kp == 2 ? s2 : s4;
    }
    T pth = (T)0, pyy = (T)0;
    if (owner) {
      // u[r] addressed from y's row (u = y + ns, ns scene-uniform), so that no second
      // per-lane address is held across the iteration
      const T yn = be * (dr + x) + y[r + ns];
      const T df = yn - y[r];
      pth = df * df;
      pyy = yn * yn;
      y[r] = yn;
    }
    // Residual of Eq. (22) and |y|^2, reduced in a fixed order.
    pth = wave_total_lane63(pth);
    pyy = wave_total_lane63(pyy);
    if (lane == 63) {
      // the wave index as a wave-uniform (scalar) value: the slot's address is formed anew
      // instead of being held in a vector register across the iteration
      const int sw = __builtin_amdgcn_readfirstlane(tid) >> 6;
      red[0][sw] = pth;
      red[1][sw] = pyy;
    }
    __syncthreads();
    {
      // the partials as 16-byte vectors (a few LDS reads per wave instead of sixteen)
      T tp[8], yp[8];
#pragma unroll
      for (int q = 0; q < 8; q += V) {
        const VT t4 = *reinterpret_cast<const VT*>(&red[0][q]);
        const VT y4 = *reinterpret_cast<const VT*>(&red[1][q]);
#pragma unroll
        for (int k = 0; k < V; ++k) {
          tp[q + k] = Vec16<T>::get(t4, k);
          yp[q + k] = Vec16<T>::get(y4, k);
        }
      }
      th = (T)0;
      yy = (T)0;
#pragma unroll
      for (int q = 0; q < 8; ++q) { th += tp[q]; yy += yp[q]; }
    }
    // r_theta = sqrt(theta)/max(|y|, 1e-12) <= tol, tested on squares
    if (!__builtin_isfinite((double)th) || !__builtin_isfinite((double)yy)) {
      if (tid == 0) atomicOr(a.flags, FLAG_NONFINITE);
      break;
    }
    if ((double)th <= (double)tol2 * ((double)yy > 1e-24 ? (double)yy : 1e-24)) { conv = 1; break; }
    if (l + 1 == a.max_iters) break;

    // z-update (Eq. 16-21) and dual update (Eq. 14): u = -lambda, w = y + 2 lambda.
    if (has_if && multi) {
      z_update_multi<T, kPadW>(a, j, s0, ev, y, u, w);
    } else if (has_if && kind == KIND_CONTACT) {
      z_update_fixed<T, 3, KIND_CONTACT>(ev, ib0, ib1, iws, mu, p0, p1, q0, q1, y, u, w, a.contact_model);
    } else if (has_if && kind == KIND_EQUALITY && dim == 5) {
      z_update_fixed<T, 5, KIND_EQUALITY>(ev, ib0, ib1, iws, mu, p0, p1, q0, q1, y, u, w, 0);
    } else if (has_if && kind == KIND_EQUALITY && dim == 1) {
      z_update_fixed<T, 1, KIND_EQUALITY>(ev, ib0, ib1, iws, mu, p0, p1, q0, q1, y, u, w, 0);
    } else if (has_if && kind == KIND_HARD_INEQ && dim == 1) {
      z_update_fixed<T, 1, KIND_HARD_INEQ>(ev, ib0, ib1, iws, mu, p0, p1, q0, q1, y, u, w, 0);
    } else if (has_if) {
      T ya[kMaxIfDim], yb[kMaxIfDim], p[kMaxIfDim], lam[kMaxIfDim];
#pragma unroll
      for (int k = 0; k < kMaxIfDim; ++k) {
        const int kk = k < dim ? k : 0;  // in-bounds address for unused rows
        ya[k] = y[p0 + kk];
        yb[k] = y[p1 + kk];
      }
      // soft (Eq. 20) or the p of Eq. 17-21 (ev holds the interface's rows in LDS)
#pragma unroll
      for (int k = 0; k < kMaxIfDim; ++k) {
        const T ek = k < dim ? ev[k] : (T)0;
        p[k] = kind == KIND_SOFT ? zsoft(ek, ya[k], ib0, yb[k], ib1, ksj, asj)
                                 : -zsum(ek, ya[k], ib0, yb[k], ib1) * iws;
      }
      // equality and soft: lambda = p; hard inequality: max(0, p); contact: Eq. (21)
      T cl[3];
      contact_project<T>(p, mu, cl, a.contact_model);
#pragma unroll
      for (int k = 0; k < kMaxIfDim; ++k) {
        T v = p[k];
        if (kind == KIND_HARD_INEQ) v = v > (T)0 ? v : (T)0;
        if (kind == KIND_CONTACT && k < 3) v = cl[k];
        lam[k] = v;
      }
#pragma unroll
      for (int k = 0; k < kMaxIfDim; ++k) {
        if (k < dim) {
          u[p0 + k] = -lam[k];
          w[q0 + k] = ya[k] + (T)2 * lam[k];
          if (p1 != p0) {
            u[p1 + k] = -lam[k];
            w[q1 + k] = yb[k] + (T)2 * lam[k];
          }
        }
      }
    }
    __syncthreads();
  }
  __syncthreads();

  // v_hat = c + G w (from the last x-update's w).
  const int d0 = a.t.sc_dof[sc], d1 = a.t.sc_dof[sc + 1];
  for (int dg = d0 + tid; dg < d1; dg += bd) {
    int i = sb;
    while (i + 1 < se && a.t.sub_dof[i + 1] <= dg) ++i;
    const int n = a.t.sub_n[i];
    const int rr = dg - a.t.sub_dof[i];
    const int nci = a.t.sub_nc[i];
    const int woi = kPadW ? a.t.sub_wq[i] : a.t.sub_slot[i] - s0;
    const T* G = a.G + a.t.sub_J[i] + rr;
    T v = a.cvec[dg];
    for (int c = 0; c < nci; ++c) v += G[c * n] * w[woi + c];
    if (a.v_hat) a.v_hat[dg] = v;
  }
  // final z^l, u^l and lambda = -u.
  if (owner) {
    a.z_out[s0 + r] = (w[wo + loc] + u[r]) / be;
    a.u_out[s0 + r] = u[r];
  }
  if (a.lambda && has_if) {
    for (int k = 0; k < dim; ++k) a.lambda[erow + k] = -u[p0 + k];
  }
  if (tid == 0) {
    const double yn = __builtin_sqrt((double)yy);
    a.st_iters[sc] = it;
    a.st_total[sc] += it;
    if (!conv) a.st_unconv[sc] += 1;
    if (a.st_fallback) a.st_fallback[sc] += 1;
    a.st_conv[sc] = conv;
    a.st_theta[sc] = (double)th;
    a.st_rtheta[sc] = __builtin_sqrt((double)th) / (yn > 1e-12 ? yn : 1e-12);
  }
}

template <typename T, int kHMode, int kLanes>
__global__ void __launch_bounds__(512) loop_kernel(LoopArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ __align__(16) T red[2][8];
  loop_body<T, kHMode, kLanes>(a, blockIdx.x, smem_raw, red);
}

// ------------------------------------------------------------------------------------
// Team form of the iteration (used when a scene's blocked H fits in LDS).  Every
// interface j owns a team of |S_j| d_j consecutive lanes inside one wave, one lane per
// member slot row (member 0's rows, then member 1's).  A lane computes its row's x and
// y (Eq. 15, 18); the team exchanges y with cross-lane shuffles and every lane of the
// team evaluates the interface's z-update (Eq. 16-21) and keeps its own row's dual
// u = -lambda (Eq. 14) in a register.  Only w = beta z - u is shared through LDS; it is
// double buffered by iteration parity, so the z-update of iteration l proceeds while
// the residual of iteration l is still being reduced, and one barrier per iteration
// serves both.  When the residual test stops the iteration at l, the z-update of l is
// discarded: v_hat uses the w buffer of iteration l and the kept u.
// ------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(512) team_loop_kernel(LoopArgs<T> a) {
  using VT = typename Vec16<T>::type;
  constexpr int V = Vec16<T>::N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ T red[2][2][8];
  const int sc = blockIdx.x;
  const int tid = threadIdx.x;
  const int bd = blockDim.x;
  const int nwave = bd >> 6;
  const int lane = tid & 63, wv = tid >> 6;
  if (a.skip_converged && a.skip_converged[sc]) return;
  const int s0 = a.t.sc_slot[sc];
  const int sb = a.t.sc_sub[sc], se = a.t.sc_sub[sc + 1];
  const int nhq = a.t.sc_hq[sc];
  const int nwq = a.t.sc_wq[sc];
  VT* Hq = reinterpret_cast<VT*>(smem_raw);
  T* wbuf0 = reinterpret_cast<T*>(Hq + nhq);
  T* wbuf1 = wbuf0 + nwq;

  for (int i = sb; i < se; ++i) {
    const int nci = a.t.sub_nc[i];
    const int nq = (nci + V - 1) / V;
    const T* Hg = a.H + a.t.sub_H[i];
    VT* dst = Hq + a.t.sub_hq[i];
    for (int q = tid; q < nq * nci; q += bd) {
      const int cb = q / nci, rr = q - cb * nci;
      T v[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int c = cb * V + k;
        v[k] = c < nci ? Hg[c * nci + rr] : (T)0;
      }
      dst[q] = Vec16<T>::make(v);
    }
  }
  for (int q = tid; q < 2 * nwq; q += bd) wbuf0[q] = (T)0;
  __syncthreads();

  // lane role
  const int code = a.t.lane_code[(size_t)sc * bd + tid];
  const bool act = code >= 0;
  const int j = act ? (code >> 4) : a.t.sc_if[sc];
  const int pos = act ? (code & 15) : 0;
  int kind = 0, dim = 1, two = 0, mem = 0, k_me = 0, nc = 0, hoff = 0, wo = 0, loc = 0, g = 0;
  T ib0 = (T)0, ib1 = (T)0, iws = (T)0, mu = (T)0, be = (T)1, dr = (T)0, ksj = (T)0, asj = (T)0;
  T ev[kMaxIfDim];
#pragma unroll
  for (int k = 0; k < kMaxIfDim; ++k) ev[k] = (T)0;
  T u_cur = (T)0, y_cur = (T)0;
  if (act) {
    kind = a.t.if_kind[j];
    dim = a.t.if_dim[j];
    two = a.t.if_nsub[j] == 2;
    mem = pos / dim;
    k_me = pos - mem * dim;
    const int sa = a.t.if_sub0[j];
    const int sbb = two ? a.t.if_sub1[j] : sa;
    const int i = mem ? sbb : sa;
    g = (mem ? a.t.if_slot1[j] : a.t.if_slot0[j]) + k_me;
    nc = a.t.sub_nc[i];
    loc = g - a.t.sub_slot[i];
    hoff = a.t.sub_hq[i] + loc;
    wo = a.t.sub_wq[i];
    be = a.beta[i];
    dr = a.d[g];
    ib0 = (T)1 / a.beta[sa];
    ib1 = two ? (T)1 / a.beta[sbb] : (T)0;
    iws = (T)1 / (ib0 + ib1);
    mu = a.mu[j];
    ksj = a.ksoft[j];
    asj = a.asoft[j];
#pragma unroll
    for (int k = 0; k < kMaxIfDim; ++k)
      if (k < dim) ev[k] = a.e[a.t.if_row[j] + k];
    // warm start: w^0 = beta z^0 - u^0, y^0 = beta z^0 + u^0
    const T z0 = a.z_in ? a.z_in[g] : (T)0;
    const T u0 = a.u_in ? a.u_in[g] : (T)0;
    u_cur = u0;
    y_cur = be * z0 + u0;
    wbuf0[wo + loc] = be * z0 - u0;
  }
  const int base = lane - pos;               // first lane of the team in this wave
  const int off_b = two ? dim : 0;           // member 1's rows follow member 0's
  const int nq = (nc + V - 1) / V;
  const T tol2 = (T)(a.tol * a.tol);
  __syncthreads();

  int it = 0, conv = 0;
  T th = (T)0, yy = (T)0;
  for (int l = 0; l < a.max_iters; ++l) {
    it = l + 1;
    const T* wc = (l & 1) ? wbuf1 : wbuf0;
    T* wn = (l & 1) ? wbuf0 : wbuf1;
    // x-update (Eq. 15 reassociated): x = d + H w, then y = beta x + u (Eq. 18)
    const T xr = row_dot_share<T, VT>(Hq + hoff, reinterpret_cast<const VT*>(wc + wo), nq, nc, 1);
    const T yn = be * (dr + xr) + u_cur;
    const T df = yn - y_cur;
    T pth = act ? df * df : (T)0;
    T pyy = act ? yn * yn : (T)0;

    // z-update of the lane's interface from the team's y (Eq. 16-21); ib1 = 0 for a
    // one-member interface, whose second shuffle then reads the first member again
    T p[kMaxIfDim];
#pragma unroll
    for (int k = 0; k < kMaxIfDim; ++k) {
      const int kk = k < dim ? k : 0;
      const T ya = __shfl(yn, base + kk, 64);
      const T yb = __shfl(yn, base + off_b + kk, 64);
      p[k] = kind == KIND_SOFT ? zsoft(ev[k], ya, ib0, yb, ib1, ksj, asj) : -zsum(ev[k], ya, ib0, yb, ib1) * iws;
    }
    T cl[3];
    contact_project<T>(p, mu, cl, a.contact_model);
    T lam_me = (T)0;
#pragma unroll
    for (int k = 0; k < kMaxIfDim; ++k) {
      T v = p[k];
      if (kind == KIND_HARD_INEQ) v = v > (T)0 ? v : (T)0;
      if (kind == KIND_CONTACT && k < 3) v = cl[k];
      if (k == k_me) lam_me = v;
    }
    if (act) wn[wo + loc] = yn + (T)2 * lam_me;  // w = beta z - u with u = -lambda

    // residual of Eq. (22) and |y|^2 of this x-update, reduced in a fixed order
    pth = wave_total_lane63(pth);
    pyy = wave_total_lane63(pyy);
    if (lane == 63) { red[l & 1][0][wv] = pth; red[l & 1][1][wv] = pyy; }
    __syncthreads();
    {
      T tp[8], yp[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        tp[q] = q < nwave ? red[l & 1][0][q] : (T)0;
        yp[q] = q < nwave ? red[l & 1][1][q] : (T)0;
      }
      th = (T)0;
      yy = (T)0;
#pragma unroll
      for (int q = 0; q < 8; ++q) { th += tp[q]; yy += yp[q]; }
    }
    y_cur = yn;
    if (!__builtin_isfinite((double)th) || !__builtin_isfinite((double)yy)) {
      if (tid == 0) atomicOr(a.flags, FLAG_NONFINITE);
      break;
    }
    // r_theta = sqrt(theta)/max(|y|, 1e-12) <= tol, tested on squares
    if ((double)th <= (double)tol2 * ((double)yy > 1e-24 ? (double)yy : 1e-24)) { conv = 1; break; }
    if (l + 1 == a.max_iters) break;
    u_cur = -lam_me;
  }
  __syncthreads();

  // v_hat = c + G w with the w of the last x-update
  const T* wf = ((it - 1) & 1) ? wbuf1 : wbuf0;
  const int d0 = a.t.sc_dof[sc], d1 = a.t.sc_dof[sc + 1];
  for (int dg = d0 + tid; dg < d1; dg += bd) {
    int i = sb;
    while (i + 1 < se && a.t.sub_dof[i + 1] <= dg) ++i;
    const int n = a.t.sub_n[i];
    const int rr = dg - a.t.sub_dof[i];
    const int nci = a.t.sub_nc[i];
    const T* G = a.G + a.t.sub_J[i] + rr;
    const T* wi = wf + a.t.sub_wq[i];
    T v = a.cvec[dg];
    for (int c = 0; c < nci; ++c) v += G[c * n] * wi[c];
    if (a.v_hat) a.v_hat[dg] = v;
  }
  if (act) {
    a.z_out[g] = (wf[wo + loc] + u_cur) / be;
    a.u_out[g] = u_cur;
    if (a.lambda && mem == 0) a.lambda[a.t.if_row[j] + k_me] = -u_cur;
  }
  if (tid == 0) {
    const double yn2 = __builtin_sqrt((double)yy);
    a.st_iters[sc] = it;
    a.st_total[sc] += it;
    if (!conv) a.st_unconv[sc] += 1;
    if (a.st_fallback) a.st_fallback[sc] += 1;
    a.st_conv[sc] = conv;
    a.st_theta[sc] = (double)th;
    a.st_rtheta[sc] = __builtin_sqrt((double)th) / (yn2 > 1e-12 ? yn2 : 1e-12);
  }
  (void)s0;
}

// ------------------------------------------------------------------------------------
// Wave form of the iteration: one wave per scene and no workgroup barrier.  Lane l owns
// the slot rows l, l + 64, ... (at most kWaveRows of them) and the scene's interface l.
// The LDS layout is the blocked one of loop_kernel; a wave's LDS operations complete in
// the order it issues them, so fences that keep the compiler from moving LDS accesses
// across them order the x-update's y stores before the z-update's loads and the
// z-update's u, w stores before the next x-update.  The residual is one DPP wave sum,
// read by every lane from lane 63.  Per row and per interface the arithmetic is the one
// of loop_kernel with one lane per row.
// ------------------------------------------------------------------------------------
constexpr int kWaveRows = 4;

__device__ inline float bcast_lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ inline double bcast_lane63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned int)hi << 32) | (unsigned int)lo));
}

template <typename T>
__global__ void __launch_bounds__(64) wave_loop_kernel(LoopArgs<T> a) {
  using VT = typename Vec16<T>::type;
  constexpr int V = Vec16<T>::N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int sc = blockIdx.x;
  const int lane = threadIdx.x;
  if (a.skip_converged && a.skip_converged[sc]) return;
  const int s0 = a.t.sc_slot[sc], s1 = a.t.sc_slot[sc + 1];
  const int ns = s1 - s0;
  const int i0 = a.t.sc_if[sc], i1 = a.t.sc_if[sc + 1];
  const int sb = a.t.sc_sub[sc], se = a.t.sc_sub[sc + 1];
  const int nhq = a.t.sc_hq[sc];
  const int nwq = a.t.sc_wq[sc];
  VT* Hq = reinterpret_cast<VT*>(smem_raw);
  T* w = reinterpret_cast<T*>(Hq + nhq);  // padded per-subsystem blocks
  T* y = w + nwq;
  T* u = y + ns;

  // stage H_i into the blocked layout and clear the padded w area
  for (int i = sb; i < se; ++i) {
    const int nci = a.t.sub_nc[i];
    const int nq = (nci + V - 1) / V;
    const T* Hg = a.H + a.t.sub_H[i];
    VT* dst = Hq + a.t.sub_hq[i];
    for (int q = lane; q < nq * nci; q += 64) {
      const int cb = q / nci, rr = q - cb * nci;
      T v[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int c = cb * V + k;
        v[k] = c < nci ? Hg[c * nci + rr] : (T)0;
      }
      dst[q] = Vec16<T>::make(v);
    }
  }
  for (int q = lane; q < nwq; q += 64) w[q] = (T)0;
  wave_lds_fence();

  // the lane's slot rows
  int nc[kWaveRows], hoff[kWaveRows], wo[kWaveRows], loc[kWaveRows];
  T be[kWaveRows], dr[kWaveRows];
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    const int r = lane + 64 * q;
    nc[q] = 0;
    hoff[q] = 0;
    wo[q] = 0;
    loc[q] = 0;
    be[q] = (T)1;
    dr[q] = (T)0;
    if (r < ns) {
      const int g = s0 + r;
      const int i = a.t.slot_sub[g];
      nc[q] = a.t.sub_nc[i];
      loc[q] = a.t.slot_loc[g];
      hoff[q] = a.t.sub_hq[i] + loc[q];
      wo[q] = a.t.sub_wq[i];
      be[q] = a.beta[i];
      dr[q] = a.d[g];
      // warm start: w^0 = beta z^0 - u^0, y^0 = beta z^0 + u^0
      const T z0 = a.z_in ? a.z_in[g] : (T)0;
      const T u0 = a.u_in ? a.u_in[g] : (T)0;
      w[wo[q] + loc[q]] = be[q] * z0 - u0;
      y[r] = be[q] * z0 + u0;
      u[r] = u0;
    }
  }
  // the lane's interface
  const int j = i0 + lane;
  const bool has_if = j < i1;
  int kind = 0, dim = 0, p0 = 0, p1 = 0, q0 = 0, q1 = 0;
  T ib0 = (T)0, ib1 = (T)0, iws = (T)0, mu = (T)0, ksj = (T)0, asj = (T)0;
  T ev[kMaxIfDim];
#pragma unroll
  for (int k = 0; k < kMaxIfDim; ++k) ev[k] = (T)0;
  if (has_if) {
    kind = a.t.if_kind[j];
    dim = a.t.if_dim[j];
    const bool two = a.t.if_nsub[j] == 2;
    const int sa = a.t.if_sub0[j];
    const int sbb = two ? a.t.if_sub1[j] : sa;
    p0 = a.t.if_slot0[j] - s0;
    p1 = two ? a.t.if_slot1[j] - s0 : p0;
    q0 = a.t.sub_wq[sa] + (a.t.if_slot0[j] - a.t.sub_slot[sa]);
    q1 = two ? a.t.sub_wq[sbb] + (a.t.if_slot1[j] - a.t.sub_slot[sbb]) : q0;
    ib0 = (T)1 / a.beta[sa];
    ib1 = two ? (T)1 / a.beta[sbb] : (T)0;
    iws = (T)1 / (ib0 + ib1);
    mu = a.mu[j];
    ksj = a.ksoft[j];
    asj = a.asoft[j];
#pragma unroll
    for (int k = 0; k < kMaxIfDim; ++k)
      if (k < dim) ev[k] = a.e[a.t.if_row[j] + k];
  }
  const T tol2 = (T)(a.tol * a.tol);
  wave_lds_fence();

  int it = 0, conv = 0;
  T th = (T)0, yy = (T)0;
  for (int l = 0; l < a.max_iters; ++l) {
    it = l + 1;
    // x-update (Eq. 15 reassociated) and y = beta x + u (Eq. 18) for the lane's rows
    T pth = (T)0, pyy = (T)0;
#pragma unroll
    for (int q = 0; q < kWaveRows; ++q) {
      const int r = lane + 64 * q;
      if (r < ns) {
        const int nq = (nc[q] + V - 1) / V;
        const T x = row_dot_share<T, VT>(Hq + hoff[q], reinterpret_cast<const VT*>(w + wo[q]), nq, nc[q], 1);
        const T yn = be[q] * (dr[q] + x) + u[r];
        const T df = yn - y[r];
        pth += df * df;
        pyy += yn * yn;
        y[r] = yn;
      }
    }
    // residual of Eq. (22) and |y|^2: one wave sum, the same value in every lane
    th = bcast_lane63(wave_total_lane63(pth));
    yy = bcast_lane63(wave_total_lane63(pyy));
    if (!__builtin_isfinite((double)th) || !__builtin_isfinite((double)yy)) {
      if (lane == 0) atomicOr(a.flags, FLAG_NONFINITE);
      break;
    }
    if ((double)th <= (double)tol2 * ((double)yy > 1e-24 ? (double)yy : 1e-24)) { conv = 1; break; }
    if (l + 1 == a.max_iters) break;
    wave_lds_fence();

    // z-update (Eq. 16-21) and dual update (Eq. 14): u = -lambda, w = y + 2 lambda
    if (has_if) {
      T ya[kMaxIfDim], yb[kMaxIfDim], p[kMaxIfDim], lam[kMaxIfDim];
#pragma unroll
      for (int k = 0; k < kMaxIfDim; ++k) {
        const int kk = k < dim ? k : 0;  // in-bounds address for unused rows
        ya[k] = y[p0 + kk];
        yb[k] = y[p1 + kk];
      }
#pragma unroll
      for (int k = 0; k < kMaxIfDim; ++k)
        p[k] = kind == KIND_SOFT ? zsoft(ev[k], ya[k], ib0, yb[k], ib1, ksj, asj)
                                 : -zsum(ev[k], ya[k], ib0, yb[k], ib1) * iws;
      T cl[3];
      contact_project<T>(p, mu, cl, a.contact_model);
#pragma unroll
      for (int k = 0; k < kMaxIfDim; ++k) {
        T v = p[k];
        if (kind == KIND_HARD_INEQ) v = v > (T)0 ? v : (T)0;
        if (kind == KIND_CONTACT && k < 3) v = cl[k];
        lam[k] = v;
      }
#pragma unroll
      for (int k = 0; k < kMaxIfDim; ++k) {
        if (k < dim) {
          u[p0 + k] = -lam[k];
          w[q0 + k] = ya[k] + (T)2 * lam[k];
          if (p1 != p0) {
            u[p1 + k] = -lam[k];
            w[q1 + k] = yb[k] + (T)2 * lam[k];
          }
        }
      }
    }
    wave_lds_fence();
  }
  wave_lds_fence();

  // v_hat = c + G w (from the last x-update's w).
  const int d0 = a.t.sc_dof[sc], d1 = a.t.sc_dof[sc + 1];
  for (int dg = d0 + lane; dg < d1; dg += 64) {
    int i = sb;
    while (i + 1 < se && a.t.sub_dof[i + 1] <= dg) ++i;
    const int n = a.t.sub_n[i];
    const int rr = dg - a.t.sub_dof[i];
    const int nci = a.t.sub_nc[i];
    const int woi = a.t.sub_wq[i];
    const T* G = a.G + a.t.sub_J[i] + rr;
    T v = a.cvec[dg];
    for (int c = 0; c < nci; ++c) v += G[c * n] * w[woi + c];
    if (a.v_hat) a.v_hat[dg] = v;
  }
  // final z^l, u^l and lambda = -u.
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    const int r = lane + 64 * q;
    if (r < ns) {
      a.z_out[s0 + r] = (w[wo[q] + loc[q]] + u[r]) / be[q];
      a.u_out[s0 + r] = u[r];
    }
  }
  if (a.lambda && has_if) {
    for (int k = 0; k < dim; ++k) a.lambda[a.t.if_row[j] + k] = -u[p0 + k];
  }
  if (lane == 0) {
    const double yn = __builtin_sqrt((double)yy);
    a.st_iters[sc] = it;
    a.st_total[sc] += it;
    if (!conv) a.st_unconv[sc] += 1;
    if (a.st_fallback) a.st_fallback[sc] += 1;
    a.st_conv[sc] = conv;
    a.st_theta[sc] = (double)th;
    a.st_rtheta[sc] = __builtin_sqrt((double)th) / (yn > 1e-12 ? yn : 1e-12);
  }
}

template <typename T>
hipError_t launch_wave_loop(const LoopArgs<T>& a, int max_slot_scene, int max_if_scene, int max_hq_scene,
                            int max_wq_scene, hipStream_t s) {
  if (a.t.n_scene == 0) return hipSuccess;
  if (max_slot_scene > 64 * kWaveRows || max_if_scene > 64) return hipErrorInvalidValue;
  const int ns = max_slot_scene > 0 ? max_slot_scene : 1;
  const size_t lds = 16 * (size_t)max_hq_scene + sizeof(T) * ((size_t)max_wq_scene + 2 * (size_t)ns) + 64;
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wave_loop_kernel<T>, dim3(a.t.n_scene), dim3(64), lds, s, a);
  return hipGetLastError();
}
template hipError_t launch_wave_loop<float>(const LoopArgs<float>&, int, int, int, int, hipStream_t);
template hipError_t launch_wave_loop<double>(const LoopArgs<double>&, int, int, int, int, hipStream_t);

template <typename T>
hipError_t launch_team_loop(const LoopArgs<T>& a, int max_hq_scene, int max_wq_scene, hipStream_t s) {
  if (a.t.n_scene == 0) return hipSuccess;
  const int threads = a.t.team_block;
  if (threads < 64 || threads > 512 || threads % 64) return hipErrorInvalidValue;
  const size_t lds = 16 * (size_t)max_hq_scene + sizeof(T) * 2 * (size_t)max_wq_scene + 64;
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(team_loop_kernel<T>, dim3(a.t.n_scene), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template hipError_t launch_team_loop<float>(const LoopArgs<float>&, int, int, hipStream_t);
template hipError_t launch_team_loop<double>(const LoopArgs<double>&, int, int, hipStream_t);

template <typename T>
hipError_t launch_factor(const FactorArgs<T>& a, int count, int max_n, int max_nc, bool fp64, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const size_t cs = fp64 ? sizeof(double) : sizeof(T);
  const size_t lds = factor_bytes(max_n, max_nc, cs);
  if (lds > 160 * 1024 - 1024) return hipErrorInvalidValue;
  // a class of small subsystems: one wave each, four per workgroup
  const size_t slice = (lds + 15) / 16 * 16;
  if (wave_factor_fits(max_n, max_nc, cs, kWaveFactorSlice) && slice <= kWaveFactorSlice) {
    const int blocks = (count + 3) / 4;
    if (fp64)
      hipLaunchKernelGGL((factor_wave_kernel<T, double>), dim3(blocks), dim3(256), 4 * slice, s, a, count, (int)slice);
    else
      hipLaunchKernelGGL((factor_wave_kernel<T, T>), dim3(blocks), dim3(256), 4 * slice, s, a, count, (int)slice);
    return hipGetLastError();
  }
  // a class of few subsystems (the largest ones) is latency-bound: give each more threads;
  // at least one thread per trailing column of the Cholesky factor's first step (n - 1)
  int threads = count < 256 ? 512 : count < 2048 ? 256 : 128;
  if (max_n > kMaxFactorDof) return hipErrorInvalidValue;
  while (threads < max_n - 1) threads *= 2;
  if (fp64)
    hipLaunchKernelGGL((factor_kernel<T, double>), dim3(count), dim3(threads), lds, s, a);
  else
    hipLaunchKernelGGL((factor_kernel<T, T>), dim3(count), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_factor_global(const FactorArgs<T>& a, int count, int max_n, bool fp64, char* scr, const int64_t* off,
                                hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (max_n > kMaxFactorDof) return hipErrorInvalidValue;
  if (fp64)
    hipLaunchKernelGGL((factor_global_kernel<T, double>), dim3(count), dim3(512), 0, s, a, scr, off);
  else
    hipLaunchKernelGGL((factor_global_kernel<T, T>), dim3(count), dim3(512), 0, s, a, scr, off);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_loop(const LoopArgs<T>& a, int max_slot_scene, int max_if_scene, long long max_h_scene,
                       int max_hq_scene, int max_wq_scene, int max_nc, hipStream_t s) {
  (void)max_h_scene;
  if (a.t.n_scene == 0) return hipSuccess;
  const int ns = max_slot_scene > 0 ? max_slot_scene : 1;
  // two lanes per slot row while the block stays within 4 waves (so that four or more
  // scenes stay resident per CU), else one
  const bool two = 2 * ns <= kTwoLaneMax && max_if_scene <= kTwoLaneMax;
  const int need = two ? (2 * ns > max_if_scene ? 2 * ns : max_if_scene) : (ns > max_if_scene ? ns : max_if_scene);
  const int threads = (need + 63) / 64 * 64;
  if (threads > 512) return hipErrorInvalidValue;
  const size_t rows = (size_t)a.t.max_row_scene;  // the scene's e rows, staged after u
  const size_t slots = sizeof(T) * (3 * (size_t)ns + rows);
  const size_t with_h = 16 * (size_t)max_hq_scene + sizeof(T) * ((size_t)max_wq_scene + 2 * (size_t)ns + rows) + 64;
  const bool hl = with_h <= 150 * 1024;
  (void)max_nc;
  if (!hl && slots > 150 * 1024) return hipErrorInvalidValue;
  if (hl && a.t.rmap && a.t.rmap_block <= 512) {
    hipLaunchKernelGGL((loop_kernel<T, kHLds, 0>), dim3(a.t.n_scene), dim3(a.t.rmap_block), with_h, s, a);
  } else if (hl && two) {
    hipLaunchKernelGGL((loop_kernel<T, kHLds, 2>), dim3(a.t.n_scene), dim3(threads), with_h, s, a);
  } else if (hl) {
    hipLaunchKernelGGL((loop_kernel<T, kHLds, 1>), dim3(a.t.n_scene), dim3(threads), with_h, s, a);
  } else if (two) {
    hipLaunchKernelGGL((loop_kernel<T, kHGlobal, 2>), dim3(a.t.n_scene), dim3(threads), slots, s, a);
  } else {
    hipLaunchKernelGGL((loop_kernel<T, kHGlobal, 1>), dim3(a.t.n_scene), dim3(threads), slots, s, a);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Several whole time steps per launch (Alg. 1 repeated), one workgroup per scene: the
// construction of the scene's subsystems, their factorisations one after another, the
// iteration, and the state update of its bodies, then the next step.  A scene does not
// wait for the others between steps, so the launch lasts as long as the largest sum of
// iterations over the steps of one scene rather than the sum over steps of the largest
// per-step count.  Every phase is the per-step kernels' code; the barriers between phases
// order the global-memory writes and reads of the workgroup.
// ------------------------------------------------------------------------------------
// The phases read their arguments through the argument block in device memory, and the
// block's address passes through an empty asm statement at the start of each phase: the
// compiler cannot move a phase's argument loads into another phase, so no phase keeps the
// others' arguments live in registers (the whole kernel inlined, its LDS addressed
// directly).
template <typename T>
__device__ __attribute__((always_inline)) inline const StepsArgs<T>* phase_args(const StepsArgs<T>* p) {
  uint64_t v = reinterpret_cast<uint64_t>(p);
  asm volatile("" : "+s"(v));
  return reinterpret_cast<const StepsArgs<T>*>(v);
}

template <typename T, typename C, int kLanes>
__global__ void __launch_bounds__(256, 4) steps_kernel(const StepsArgs<T>* __restrict__ ap) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double fred[2][8];
  __shared__ int fbad;
  __shared__ int wbad[4];
  __shared__ __align__(16) T lred[2][8];
  // workgroups are dispatched round-robin over the XCDs and their CUs in block order, so the
  // order decides which scenes share a CU
  const int sc = ap->sc_order[blockIdx.x];
  const int n_steps = ap->n_steps;
  const int tid = threadIdx.x, bd = blockDim.x;
  for (int step = 0; step < n_steps; ++step) {
    {
      // construction (Eq. 2-5) of the scene's subsystems at once: disjoint blocks of A, b, J
      // and rows of e
      const StepsArgs<T>& a = *phase_args(ap);
      const int sb = a.l.t.sc_sub[sc], se = a.l.t.sc_sub[sc + 1];
      rigid_assemble_scene<T, true>(a.l.t, a.m, sb, se, a.st.pos, a.st.rot, a.st.vel, a.st.omega, a.dt, a.A, a.b,
                                    a.J, a.e);
    }
    __syncthreads();
    {
      // penalty (Eq. 23) and factorisation per subsystem: the small subsystems one per wave,
      // the waves taking them in turn, each in its share of the LDS; then the others with the
      // whole workgroup, in LDS when they fit
      const StepsArgs<T>& a = *phase_args(ap);
      const int sb = a.l.t.sc_sub[sc], se = a.l.t.sc_sub[sc + 1];
      const int nwave = bd >> 6, wv = tid >> 6;
      const size_t slice = (size_t)a.lds_factor / (size_t)nwave / 16 * 16;
      int k = 0;
      for (int i = sb; i < se; ++i) {
        if (!wave_factor_fits(a.l.t.sub_n[i], a.l.t.sub_nc[i], sizeof(C), slice)) continue;
        if (k++ % nwave == wv)
          factor_body<T, C, GroupWave>(a.f, i, reinterpret_cast<C*>(smem_raw + (size_t)wv * slice), nullptr,
                                       wbad[wv]);
      }
      __syncthreads();
      for (int i = sb; i < se; ++i) {
        if (wave_factor_fits(a.l.t.sub_n[i], a.l.t.sub_nc[i], sizeof(C), slice)) continue;
        if (factor_bytes(a.l.t.sub_n[i], a.l.t.sub_nc[i], sizeof(C)) <= (size_t)a.lds_factor)
          factor_body<T, C>(a.f, i, reinterpret_cast<C*>(smem_raw), fred, fbad);
        else
          factor_body<T, C>(a.f, i, reinterpret_cast<C*>(a.fscr + a.sc_fscr[sc]), fred, fbad);
        __syncthreads();
      }
    }
    // the iteration (Eq. 15-22, 14) from the previous step's values or cold
    loop_body<T, kHLds, kLanes>(phase_args(ap)->l, sc, smem_raw, lred);
    __syncthreads();
    {
      // state update (Eq. 2)
      const StepsArgs<T>& a = *phase_args(ap);
      const int sb = a.l.t.sc_sub[sc], se = a.l.t.sc_sub[sc + 1];
      for (int q = a.m.sub_body_off[sb] + tid; q < a.m.sub_body_off[se]; q += bd)
        rigid_advance_body<T>(a.l.t, a.m, a.st, a.l.v_hat, a.dt, a.m.sub_body[q]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------
// Scenes too large for one workgroup (Alg. 1 over the whole problem): one launch per phase
// of each iteration.  x-update (Eq. 15, 18) one thread per slot row with the operators in
// device memory; residual (Eq. 22) and stopping test one workgroup per scene, summing the
// slot rows of the scene in a fixed order; z-update (Eq. 16-21) and dual update (Eq. 14) one
// thread per interface.  A scene that stops keeps its values: the later launches skip it.
// Same iteration as the per-scene kernel (u = -lambda, w = y + 2 lambda kept per slot row).
// ------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) large_init_kernel(LargeArgs<T> a) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const LoopArgs<T>& l = a.l;
  if (g < l.t.n_scene) a.done[g] = 0;
  if (g >= a.n_slot) return;
  const T be = l.beta[l.t.slot_sub[g]];
  const T z0 = l.z_in ? l.z_in[g] : (T)0;
  const T u0 = l.u_in ? l.u_in[g] : (T)0;
  a.w[g] = be * z0 - u0;
  a.y[g] = be * z0 + u0;
  a.u[g] = u0;
}

// x-update of slot row g (Eq. 15 reassociated, y = beta x + u) with its residual terms
template <typename T>
__device__ inline void large_xupdate_row(const LargeArgs<T>& a, const long g) {
  const LoopArgs<T>& l = a.l;
  const int i = l.t.slot_sub[g];
  const int nc = l.t.sub_nc[i], loc = l.t.slot_loc[g];
  const T* H = l.H + l.t.sub_H[i] + loc;  // column-major: H_i[loc][c] at c * nc + loc
  const T* w = a.w + l.t.sub_slot[i];
  T acc[4] = {(T)0, (T)0, (T)0, (T)0};
  int c = 0;
  for (; c + 3 < nc; c += 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += H[(long)(c + k) * nc] * w[c + k];
  }
  for (; c < nc; ++c) acc[0] += H[(long)c * nc] * w[c];
  const T x = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  const T yn = l.beta[i] * (l.d[g] + x) + a.u[g];
  const double df = (double)yn - (double)a.y[g];
  a.dy2[g] = df * df;
  a.yy2[g] = (double)yn * (double)yn;
  a.y[g] = yn;
}

template <typename T>
__global__ void __launch_bounds__(256) large_xupdate_kernel(LargeArgs<T> a) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.n_slot) return;
  if (a.done[a.sub_scene[a.l.t.slot_sub[g]]]) return;
  large_xupdate_row<T>(a, g);
}

// The stopping test of scene sc from its wave partials (fixed order); writes the statistics
// and the scene's stop flag; returns whether the scene stopped.
template <typename T>
__device__ inline int large_decide(const LargeArgs<T>& a, const int sc, const int l_iter, double (*red)[4]) {
  const LoopArgs<T>& l = a.l;
  const double th = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
  const double yy = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  const int it = l_iter + 1;
  const bool bad = !__builtin_isfinite(th) || !__builtin_isfinite(yy);
  const bool cv = !bad && th <= l.tol * l.tol * (yy > 1e-24 ? yy : 1e-24);
  if (bad) atomicOr(l.flags, FLAG_NONFINITE);
  const bool stop = cv || bad || it == l.max_iters;
  if (stop) {
    a.done[sc] = 1;
    const double yn = __builtin_sqrt(yy);
    l.st_iters[sc] = it;
    l.st_total[sc] += it;
    if (!cv) l.st_unconv[sc] += 1;
    l.st_conv[sc] = cv ? 1 : 0;
    l.st_theta[sc] = th;
    l.st_rtheta[sc] = __builtin_sqrt(th) / (yn > 1e-12 ? yn : 1e-12);
  }
  return stop ? 1 : 0;
}

// Residual of Eq. 22 of scene sc by the first 256 threads of its workgroup (threads take
// rows tid, tid + 256, ...; waves summed in a fixed order, whatever the workgroup's size)
// and the stopping test; returns on every thread whether the scene stopped (statistics
// written by thread 0).
template <typename T>
__device__ inline bool large_residual_scene(const LargeArgs<T>& a, const int sc, const int l_iter,
                                            double (*red)[4], int* stop) {
  const LoopArgs<T>& l = a.l;
  const int s0 = l.t.sc_slot[sc], s1 = l.t.sc_slot[sc + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid < 256) {
    double th = 0.0, yy = 0.0;
    for (int g = s0 + tid; g < s1; g += 256) {
      th += a.dy2[g];
      yy += a.yy2[g];
    }
    th = wave_total_lane63(th);
    yy = wave_total_lane63(yy);
    if (lane == 63) {
      red[0][wv] = th;
      red[1][wv] = yy;
    }
  }
  __syncthreads();
  if (tid == 0) *stop = large_decide<T>(a, sc, l_iter, red);
  __syncthreads();
  return *stop != 0;
}

template <typename T>
__global__ void __launch_bounds__(256) large_residual_kernel(LargeArgs<T> a, int l_iter) {
  __shared__ double red[2][4];
  __shared__ int stop;
  const int sc = blockIdx.x;
  if (a.done[sc]) return;
  large_residual_scene<T>(a, sc, l_iter, red, &stop);
}

// z-update (Eq. 16-21) and dual update of interface j on the global slot arrays
template <typename T>
__device__ inline void large_zupdate_if(const LargeArgs<T>& a, const int j) {
  const LoopArgs<T>& l = a.l;
  const int sa = l.t.if_sub0[j];
  if (l.t.if_nsub[j] > 2) {
    // the multi-member form on the global slot arrays (scene offset 0, unpadded w)
    T ev[kMaxIfDim];
    for (int k = 0; k < kMaxIfDim; ++k) ev[k] = k < l.t.if_dim[j] ? l.e[l.t.if_row[j] + k] : (T)0;
    z_update_multi<T, false>(l, j, 0, ev, a.y, a.u, a.w);
    return;
  }
  const bool two = l.t.if_nsub[j] == 2;
  const int sb = two ? l.t.if_sub1[j] : sa;
  const int kind = l.t.if_kind[j], dim = l.t.if_dim[j];
  const int p0 = l.t.if_slot0[j], p1 = two ? l.t.if_slot1[j] : p0;
  const T ib0 = (T)1 / l.beta[sa], ib1 = two ? (T)1 / l.beta[sb] : (T)0;
  const T iws = (T)1 / (ib0 + ib1);
  T ya[kMaxIfDim], yb[kMaxIfDim], p[kMaxIfDim];
#pragma unroll
  for (int k = 0; k < kMaxIfDim; ++k) {
    const int kk = k < dim ? k : 0;
    const T ev = k < dim ? l.e[l.t.if_row[j] + k] : (T)0;
    ya[k] = a.y[p0 + kk];
    yb[k] = two ? a.y[p1 + kk] : (T)0;
    p[k] = kind == KIND_SOFT ? zsoft(ev, ya[k], ib0, yb[k], ib1, l.ksoft[j], l.asoft[j])
                             : -zsum(ev, ya[k], ib0, yb[k], ib1) * iws;
  }
  T cl[3];
  contact_project<T>(p, l.mu[j], cl, l.contact_model);
#pragma unroll
  for (int k = 0; k < kMaxIfDim; ++k) {
    if (k >= dim) continue;
    T v = p[k];
    if (kind == KIND_HARD_INEQ) v = v > (T)0 ? v : (T)0;
    if (kind == KIND_CONTACT && k < 3) v = cl[k];
    a.u[p0 + k] = -v;
    a.w[p0 + k] = ya[k] + (T)2 * v;
    if (two) {
      a.u[p1 + k] = -v;
      a.w[p1 + k] = yb[k] + (T)2 * v;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) large_zupdate_kernel(LargeArgs<T> a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.l.t.n_if) return;
  if (a.done[a.sub_scene[a.l.t.if_sub0[j]]]) return;
  large_zupdate_if<T>(a, j);
}

// Outputs after the iteration: v_hat of DOF g (c + G w of the last x-update's w), z and u
// of slot row g, lambda of interface g (= -u at its first member)
template <typename T>
__device__ inline void large_final_item(const LargeArgs<T>& a, const long g, const bool dof, const bool slot,
                                        const bool iface) {
  const LoopArgs<T>& l = a.l;
  if (dof && g < a.n_dof && l.v_hat) {
    // subsystem of DOF g: the last i with sub_dof[i] <= g
    int lo = 0, hi = l.t.n_sub - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (l.t.sub_dof[mid] <= g) lo = mid;
      else hi = mid - 1;
    }
    const int i = lo, n = l.t.sub_n[i], nc = l.t.sub_nc[i], rr = (int)(g - l.t.sub_dof[i]);
    const T* G = l.G + l.t.sub_J[i] + rr;
    const T* w = a.w + l.t.sub_slot[i];
    T v = l.cvec[g];
    for (int c = 0; c < nc; ++c) v += G[(long)c * n] * w[c];
    l.v_hat[g] = v;
  }
  if (slot && g < a.n_slot) {
    const T be = l.beta[l.t.slot_sub[g]];
    l.z_out[g] = (a.w[g] + a.u[g]) / be;
    l.u_out[g] = a.u[g];
  }
  if (iface && g < l.t.n_if && l.lambda) {
    const int dim = l.t.if_dim[g];
    for (int k = 0; k < dim; ++k) l.lambda[l.t.if_row[g] + k] = -a.u[l.t.if_slot0[g] + k];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) large_final_kernel(LargeArgs<T> a) {
  large_final_item<T>(a, (long)blockIdx.x * blockDim.x + threadIdx.x, true, true, true);
}

// The whole iteration of one scene by one workgroup of 256 to 1024 threads (for scenes
// beyond the per-scene kernel's LDS layout but whose iteration one workgroup carries well):
// the same per-row x-update, per-scene residual (same summation order) and per-interface
// z-update as the phase kernels, with workgroup barriers in place of kernel boundaries, on
// the same global slot arrays.  Bitwise equal to the phase kernels.
template <typename T>
__global__ void __launch_bounds__(1024) large_scene_kernel(LargeArgs<T> a) {
  __shared__ double red[2][4];
  __shared__ int stop;
  const int sc = blockIdx.x;
  const LoopArgs<T>& l = a.l;
  const int tid = threadIdx.x, bd = blockDim.x;
  const int s0 = l.t.sc_slot[sc], s1 = l.t.sc_slot[sc + 1];
  const int i0 = l.t.sc_if[sc], i1 = l.t.sc_if[sc + 1];
  const int d0 = l.t.sc_dof[sc], d1 = l.t.sc_dof[sc + 1];
  if (tid == 0) a.done[sc] = 0;
  for (int g = s0 + tid; g < s1; g += bd) {
    const T be = l.beta[l.t.slot_sub[g]];
    const T z0 = l.z_in ? l.z_in[g] : (T)0;
    const T u0 = l.u_in ? l.u_in[g] : (T)0;
    a.w[g] = be * z0 - u0;
    a.y[g] = be * z0 + u0;
    a.u[g] = u0;
  }
  __syncthreads();
  for (int it = 0; it < l.max_iters; ++it) {
    for (int g = s0 + tid; g < s1; g += bd) large_xupdate_row<T>(a, g);
    __syncthreads();
    if (large_residual_scene<T>(a, sc, it, red, &stop)) break;
    for (int j = i0 + tid; j < i1; j += bd) large_zupdate_if<T>(a, j);
    __syncthreads();
  }
  for (int g = d0 + tid; g < d1; g += bd) large_final_item<T>(a, g, true, false, false);
  for (int g = s0 + tid; g < s1; g += bd) large_final_item<T>(a, g, false, true, false);
  for (int j = i0 + tid; j < i1; j += bd) large_final_item<T>(a, j, false, false, true);
}

__global__ void __launch_bounds__(256) large_alldone_kernel(const int32_t* done, int n_scene, int32_t* all_done) {
  __shared__ int open;
  if (threadIdx.x == 0) open = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < n_scene; s += blockDim.x)
    if (!done[s]) open = 1;
  __syncthreads();
  if (threadIdx.x == 0) *all_done = open ? 0 : 1;
}

template <typename T>
hipError_t launch_large_scene(const LargeArgs<T>& a, int threads, hipStream_t s) {
  if (a.l.t.n_scene == 0) return hipSuccess;
  if (threads < 256 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(large_scene_kernel<T>, dim3(a.l.t.n_scene), dim3(threads), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_large_scene<float>(const LargeArgs<float>&, int, hipStream_t);
template hipError_t launch_large_scene<double>(const LargeArgs<double>&, int, hipStream_t);

// ADMM's standard primal and dual residuals (Boyd et al. 2011, Sec. 3.3) of the iterate a
// solve returns, one 256-thread workgroup per scene: from the returned (z, u) (z_in, u_in)
// one more x-update (Eq. 15) and the z- and dual update (Eq. 16-21, 14) that would follow
// it, on the large-scene slot arrays as scratch (nothing returned is changed).  The
// x-update gives the x of the iteration's last x-update, from which v_hat was formed.
//   r_prim = |x - z'| / max(|x|, |z'|),  r_dual = |beta (z' - z)| / |u'|,  floors 1e-12,
// sums in FP64 over the scene's slot rows (threads take rows tid, tid + 256, ...; waves
// added in a fixed order).
template <typename T>
__global__ void __launch_bounds__(256) boyd_residual_kernel(LargeArgs<T> a, double* r_prim, double* r_dual) {
  __shared__ double red[5][4];
  const int sc = blockIdx.x;
  const LoopArgs<T>& l = a.l;
  const int tid = threadIdx.x, bd = blockDim.x, lane = tid & 63, wv = tid >> 6;
  const int s0 = l.t.sc_slot[sc], s1 = l.t.sc_slot[sc + 1];
  const int i0 = l.t.sc_if[sc], i1 = l.t.sc_if[sc + 1];
  for (int g = s0 + tid; g < s1; g += bd) {
    const T be = l.beta[l.t.slot_sub[g]];
    a.w[g] = be * l.z_in[g] - l.u_in[g];
    a.u[g] = l.u_in[g];
    a.y[g] = (T)0;
  }
  __syncthreads();
  for (int g = s0 + tid; g < s1; g += bd) large_xupdate_row<T>(a, g);
  __syncthreads();
  for (int j = i0 + tid; j < i1; j += bd) large_zupdate_if<T>(a, j);
  __syncthreads();
  // after the z-update: u' = -lambda and w' = y + 2 lambda, so z' = (w' + u') / beta
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int g = s0 + tid; g < s1; g += bd) {
    const double be = (double)l.beta[l.t.slot_sub[g]];
    const double x = ((double)a.y[g] - (double)l.u_in[g]) / be;
    const double zn = ((double)a.w[g] + (double)a.u[g]) / be;
    const double dz = be * (zn - (double)l.z_in[g]);
    const double un = (double)a.u[g];
    v[0] += (x - zn) * (x - zn);
    v[1] += x * x;
    v[2] += zn * zn;
    v[3] += dz * dz;
    v[4] += un * un;
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double t = wave_total_lane63(v[k]);
    if (lane == 63) red[k][wv] = t;
  }
  __syncthreads();
  if (tid == 0) {
    double q[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) q[k] = (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
    const double nx = __builtin_sqrt(q[1] > q[2] ? q[1] : q[2]), nu = __builtin_sqrt(q[4]);
    r_prim[sc] = __builtin_sqrt(q[0]) / (nx > 1e-12 ? nx : 1e-12);
    r_dual[sc] = __builtin_sqrt(q[3]) / (nu > 1e-12 ? nu : 1e-12);
  }
}

template <typename T>
hipError_t launch_boyd_residuals(const LargeArgs<T>& a, double* r_prim, double* r_dual, hipStream_t s) {
  if (a.l.t.n_scene == 0) return hipSuccess;
  hipLaunchKernelGGL(boyd_residual_kernel<T>, dim3(a.l.t.n_scene), dim3(256), 0, s, a, r_prim, r_dual);
  return hipGetLastError();
}
template hipError_t launch_boyd_residuals<float>(const LargeArgs<float>&, double*, double*, hipStream_t);
template hipError_t launch_boyd_residuals<double>(const LargeArgs<double>&, double*, double*, hipStream_t);

template <typename T>
hipError_t launch_large_loop(const LargeArgs<T>& a, hipStream_t s, int poll_every, int32_t* host_flag) {
  const unsigned bs = 256;
  const long most = a.n_slot > a.n_dof ? a.n_slot : a.n_dof;
  const long fin = most > a.l.t.n_if ? most : a.l.t.n_if;
  const long first = a.n_slot > a.l.t.n_scene ? a.n_slot : a.l.t.n_scene;
  hipLaunchKernelGGL(large_init_kernel<T>, dim3((unsigned)((first + bs - 1) / bs)), dim3(bs), 0, s, a);
  hipError_t e = hipGetLastError();
  for (int it = 0; it < a.l.max_iters && e == hipSuccess; ++it) {
    if (a.n_slot > 0)
      hipLaunchKernelGGL(large_xupdate_kernel<T>, dim3((unsigned)((a.n_slot + bs - 1) / bs)), dim3(bs), 0, s, a);
    hipLaunchKernelGGL(large_residual_kernel<T>, dim3(a.l.t.n_scene), dim3(bs), 0, s, a, it);
    if (it + 1 < a.l.max_iters && a.l.t.n_if > 0)
      hipLaunchKernelGGL(large_zupdate_kernel<T>, dim3((unsigned)((a.l.t.n_if + bs - 1) / bs)), dim3(bs), 0, s, a);
    e = hipGetLastError();
    if (e == hipSuccess && poll_every > 0 && host_flag && (it + 1) % poll_every == 0 && it + 1 < a.l.max_iters) {
      // every scene stopped: the launches left would return at once, so none are issued
      hipLaunchKernelGGL(large_alldone_kernel, dim3(1), dim3(bs), 0, s, a.done, a.l.t.n_scene, a.all_done);
      e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpyAsync(host_flag, a.all_done, sizeof(int32_t), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess && *host_flag) break;
    }
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(large_final_kernel<T>, dim3((unsigned)((fin + bs - 1) / bs)), dim3(bs), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_large_loop<float>(const LargeArgs<float>&, hipStream_t, int, int32_t*);
template hipError_t launch_large_loop<double>(const LargeArgs<double>&, hipStream_t, int, int32_t*);

template <typename T>
hipError_t launch_steps(const StepsArgs<T>& a, const StepsArgs<T>* dev_args, int max_slot_scene, int max_if_scene,
                        int max_hq_scene, int max_wq_scene, bool fp64, size_t lds, hipStream_t s) {
  if (a.l.t.n_scene == 0 || a.n_steps == 0) return hipSuccess;
  const int ns = max_slot_scene > 0 ? max_slot_scene : 1;
  const bool two = 2 * ns <= kTwoLaneMax && max_if_scene <= kTwoLaneMax;
  const int need = two ? (2 * ns > max_if_scene ? 2 * ns : max_if_scene) : (ns > max_if_scene ? ns : max_if_scene);
  const int threads = (need + 63) / 64 * 64;
  (void)max_hq_scene;
  (void)max_wq_scene;
  // at most 256 threads, and at most 128 VGPRs (the launch bound of four waves per SIMD), so
  // that four scenes of the multi-step kernel share a CU
  if (threads > 256 || lds > 150 * 1024) return hipErrorInvalidValue;
  // split rows within the default block: its lane map is built for exactly this block
  const bool split = a.l.t.rmap && a.l.t.rmap_block == threads;
  if (fp64 && split)
    hipLaunchKernelGGL((steps_kernel<T, double, 0>), dim3(a.l.t.n_scene), dim3(threads), lds, s, dev_args);
  else if (split)
    hipLaunchKernelGGL((steps_kernel<T, T, 0>), dim3(a.l.t.n_scene), dim3(threads), lds, s, dev_args);
  else if (fp64 && two)
    hipLaunchKernelGGL((steps_kernel<T, double, 2>), dim3(a.l.t.n_scene), dim3(threads), lds, s, dev_args);
  else if (fp64)
    hipLaunchKernelGGL((steps_kernel<T, double, 1>), dim3(a.l.t.n_scene), dim3(threads), lds, s, dev_args);
  else if (two)
    hipLaunchKernelGGL((steps_kernel<T, T, 2>), dim3(a.l.t.n_scene), dim3(threads), lds, s, dev_args);
  else
    hipLaunchKernelGGL((steps_kernel<T, T, 1>), dim3(a.l.t.n_scene), dim3(threads), lds, s, dev_args);
  return hipGetLastError();
}

template hipError_t launch_steps<float>(const StepsArgs<float>&, const StepsArgs<float>*, int, int, int, int, bool,
                                        size_t, hipStream_t);
template hipError_t launch_steps<double>(const StepsArgs<double>&, const StepsArgs<double>*, int, int, int, int, bool,
                                         size_t, hipStream_t);
template hipError_t launch_factor<float>(const FactorArgs<float>&, int, int, int, bool, hipStream_t);
template hipError_t launch_factor<double>(const FactorArgs<double>&, int, int, int, bool, hipStream_t);
template hipError_t launch_factor_global<float>(const FactorArgs<float>&, int, int, bool, char*, const int64_t*,
                                                hipStream_t);
template hipError_t launch_factor_global<double>(const FactorArgs<double>&, int, int, bool, char*, const int64_t*,
                                                 hipStream_t);
template hipError_t launch_loop<float>(const LoopArgs<float>&, int, int, long long, int, int, int, hipStream_t);
template hipError_t launch_loop<double>(const LoopArgs<double>&, int, int, long long, int, int, int, hipStream_t);

}  // namespace subadmm
