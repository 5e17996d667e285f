// HIP kernels (gfx950) of the deformable-body path: co-rotated linear-tetrahedron blocks,
// one subsystem per block (arXiv 2302.14344, Sec. II soft constraints folded into A_i, b_i;
// Algorithm 1 with multi-block subsystems).
//
// fem_assemble_kernel: one workgroup per block.  Eq. (2) with the elastic potential psi
//   linearised about the start-of-step positions x:
//     A = (2/t) M + (t/2) K(x),   b = (2/t) M v - d psi(x)^T + M g,
//   with per-tetrahedron rotation R (orthogonal polar factor of F = sum_a x_a g_a^T, by
//   Newton's iteration R <- (R + R^-T)/2), rest stiffness blocks
//     K0_ab = V (lambda g_a g_b^T + mu g_b g_a^T + mu (g_a . g_b) I),
//   co-rotated K_ab = R K0_ab R^T and elastic forces f_a = -R (V sigma) g_a with
//   sigma = lambda tr(G) I + mu (G + G^T), G = sum_b (R^T x_b - X_b) g_b^T.  A is written
//   by node pair (gather over the tetrahedra sharing the pair, so each entry is formed
//   once, in a fixed order).
// fem_factor_kernel: one workgroup per block, FP64 (or an FP32 trial on every block, FP64 again
//   for blocks whose condition estimate exceeds a threshold).  beta (Eq. 23), K = A + beta J^T J
//   in a permuted order with the constrained DOFs last, Cholesky factor L (with y = L^-1 b),
//   the inverse of the trailing factor block T = L_DD^-1, and S = T^T T, which is K^-1
//   restricted to the constrained DOFs (the Schur-complement inverse).  Since every slot row
//   of a block selects one DOF with sign +-1, the x-update of Eq. (15) followed by
//   x = J v_hat is  x = J_D (c_D + S J_D^T w)  with c = K^-1 b: one dense m x m product per
//   block.  The O(n^3) parts are 16 x 16 tile products on the FP64 (FP32) matrix cores.
// fem_loop_kernel: one launch with every block resident, one workgroup per block.  Each
//   workgroup does the z-update (Eq. 16-21) of the interfaces that touch its block
//   (two-member interfaces are computed by both members from the same y, so both obtain
//   the same lambda), the dual update (Eq. 14), the x-update and its share of the residual
//   (Eq. 22), and tests the residual of its scene.  The values exchanged between workgroups
//   (y and the residual partials) sit in three buffers used in turn and are written and
//   polled with agent-scope atomics, which reach the point of coherence across the chip's
//   L2 caches: no grid barrier and no device-wide cache write-back per iteration.
// fem_vhat_kernel: v_hat = K^-1 (b + J^T w) after the iteration, from the factorisation's
//   y = L^-1 P b and T = L_DD^-1 (each block's factors in the precision it was factorised in): v_D = T^T (y_D + T e_D), v_O = L_OO^-T (y_O - L_DO^T v_D).
#include <type_traits>

#include "internal.hpp"

namespace subadmm {

namespace {

constexpr int kFemThreads = 256;
constexpr int kNb = 16;  // factorisation block size

__device__ inline void mat3_inv(const double* m, double* o, double& det) {
  det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) + m[2] * (m[3] * m[7] - m[4] * m[6]);
  const double id = 1.0 / det;
  o[0] = (m[4] * m[8] - m[5] * m[7]) * id;
  o[1] = (m[2] * m[7] - m[1] * m[8]) * id;
  o[2] = (m[1] * m[5] - m[2] * m[4]) * id;
  o[3] = (m[5] * m[6] - m[3] * m[8]) * id;
  o[4] = (m[0] * m[8] - m[2] * m[6]) * id;
  o[5] = (m[2] * m[3] - m[0] * m[5]) * id;
  o[6] = (m[3] * m[7] - m[4] * m[6]) * id;
  o[7] = (m[1] * m[6] - m[0] * m[7]) * id;
  o[8] = (m[0] * m[4] - m[1] * m[3]) * id;
}

// Orthogonal polar factor: Newton's iteration X <- (X + X^-T) / 2 from X = F (quadratic
// convergence for non-singular F); at most 60 steps.
__device__ inline bool polar_rotation(const double* F, double* R) {
  double X[9], Xi[9];
  for (int k = 0; k < 9; ++k) X[k] = F[k];
  for (int it = 0; it < 60; ++it) {
    double det;
    mat3_inv(X, Xi, det);
    if (!(det != 0.0) || !__builtin_isfinite(det)) return false;
    double diff = 0.0, nrm = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const double nv = 0.5 * (X[r * 3 + c] + Xi[c * 3 + r]);
        const double d = nv - X[r * 3 + c];
        diff += d * d;
        nrm += nv * nv;
        X[r * 3 + c] = nv;
      }
    if (diff <= 1e-30 * nrm) break;
  }
  for (int k = 0; k < 9; ++k) R[k] = X[k];
  return true;
}

}  // namespace

// ------------------------------------------------------------------------------------
// Assembly
// ------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kFemThreads)
    fem_assemble_kernel(Topo t, FemModel f, const T* pos, const T* vel, double dt, double* A, double* b, double* scr,
                        int32_t* flags) {
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int n = t.sub_n[i];
  const int node0 = f.node_off[i];
  const int t0 = f.tet_off[i], t1 = f.tet_off[i + 1];
  const double lam = f.lame_l[i], mu = f.lame_m[i];
  // per tetrahedron: R and R P with P = V sigma (9 + 9 doubles in scratch)
  for (int e = t0 + tid; e < t1; e += blockDim.x) {
    const int32_t* vn = f.tet_node + 4 * (long)e;
    const double* g = f.tet_g + 12 * (long)e;
    double x[4][3];
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) x[a][c] = (double)pos[3 * (long)vn[a] + c];
    double F[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int a = 0; a < 4; ++a) s += x[a][r] * g[3 * a + c];
        F[r * 3 + c] = s;
      }
    double R[9];
    if (!polar_rotation(F, R)) {
      atomicOr(flags, FLAG_NONFINITE);
      for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    }
    double G[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int bb = 0; bb < 4; ++bb) {
      double du[3];
      for (int c = 0; c < 3; ++c)
        du[c] = R[0 * 3 + c] * x[bb][0] + R[1 * 3 + c] * x[bb][1] + R[2 * 3 + c] * x[bb][2] -
                f.rest[3 * (long)vn[bb] + c];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) G[r * 3 + c] += du[r] * g[3 * bb + c];
    }
    const double V = f.tet_vol[e];
    const double tr = G[0] + G[4] + G[8];
    double P[9], RP[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) P[r * 3 + c] = V * ((r == c ? lam * tr : 0.0) + mu * (G[r * 3 + c] + G[c * 3 + r]));
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) RP[r * 3 + c] = R[r * 3 + 0] * P[0 * 3 + c] + R[r * 3 + 1] * P[1 * 3 + c] + R[r * 3 + 2] * P[2 * 3 + c];
    double* o = scr + 18 * (long)e;
    for (int k = 0; k < 9; ++k) {
      o[k] = R[k];
      o[9 + k] = RP[k];
    }
  }
  double* Ai = A + t.sub_A[i];
  const long nn = (long)n * n;
  for (long k = tid; k < nn; k += blockDim.x) Ai[k] = 0.0;
  __syncthreads();
  const double h = 0.5 * dt, m2 = 2.0 / dt;
  const int p0 = f.pair_off[i], p1 = f.pair_off[i + 1];
  for (int q = p0 + tid; q < p1; q += blockDim.x) {
    const int ab = f.pair_ab[q];
    const int na = ab & 0xffff, nb = ab >> 16;
    double K[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int en = f.pent_off[q]; en < f.pent_off[q + 1]; ++en) {
      const int code = f.pent[en];
      const int e = t0 + (code >> 4);
      const int va = (code >> 2) & 3, vb = code & 3;
      const double* R = scr + 18 * (long)e;
      const double* ga = f.tet_g + 12 * (long)e + 3 * va;
      const double* gb = f.tet_g + 12 * (long)e + 3 * vb;
      const double V = f.tet_vol[e];
      double ra[3], rb[3];
      for (int r = 0; r < 3; ++r) {
        ra[r] = R[r * 3 + 0] * ga[0] + R[r * 3 + 1] * ga[1] + R[r * 3 + 2] * ga[2];
        rb[r] = R[r * 3 + 0] * gb[0] + R[r * 3 + 1] * gb[1] + R[r * 3 + 2] * gb[2];
      }
      const double dot = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) K[r * 3 + c] += V * (lam * ra[r] * rb[c] + mu * rb[r] * ra[c] + (r == c ? mu * dot : 0.0));
    }
    const double md = na == nb ? m2 * f.mass[node0 + na] : 0.0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Ai[(long)(3 * na + r) * n + 3 * nb + c] = h * K[r * 3 + c] + (r == c ? md : 0.0);
  }
  // b = (2/t) M v + elastic forces + M g
  const int nnode = n / 3;
  for (int a = tid; a < nnode; a += blockDim.x) {
    const int gnode = node0 + a;
    const int q = f.node_diag[gnode];
    double fa[3] = {0.0, 0.0, 0.0};
    for (int en = f.pent_off[q]; en < f.pent_off[q + 1]; ++en) {
      const int code = f.pent[en];
      const int e = t0 + (code >> 4);
      const int va = (code >> 2) & 3;
      const double* RP = scr + 18 * (long)e + 9;
      const double* ga = f.tet_g + 12 * (long)e + 3 * va;
      for (int r = 0; r < 3; ++r) fa[r] -= RP[r * 3 + 0] * ga[0] + RP[r * 3 + 1] * ga[1] + RP[r * 3 + 2] * ga[2];
    }
    const double ma = f.mass[gnode];
    double* bo = b + t.sub_dof[i] + 3 * a;
    for (int c = 0; c < 3; ++c) bo[c] = m2 * ma * (double)vel[3 * (long)gnode + c] + fa[c] - (c == 2 ? ma * f.gravity : 0.0);
  }
}

// Interface errors: nodal equality e = gamma (x_p - x_q) / t, ground contact
// e = (z_p / t, 0, 0); position differences formed in FP64.
template <typename T>
__global__ void fem_rows_kernel(Topo t, FemModel f, const T* pos, double dt, T* e) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= t.n_if) return;
  T* ej = e + t.if_row[j];
  const long p = f.if_node0[j];
  if (t.if_kind[j] == KIND_CONTACT) {
    ej[0] = (T)((double)pos[3 * p + 2] / dt);
    ej[1] = (T)0;
    ej[2] = (T)0;
  } else {
    const long q = f.if_node1[j];
    for (int c = 0; c < 3; ++c) ej[c] = (T)(f.baumgarte * ((double)pos[3 * p + c] - (double)pos[3 * q + c]) / dt);
  }
}

// ------------------------------------------------------------------------------------
// Factorisation
// ------------------------------------------------------------------------------------
namespace {


// 16 x 16 tile products on the matrix cores, FP64 (v_mfma_f64_16x16x4f64) and FP32
// (v_mfma_f32_16x16x4f32).  A 16-deep product is four instructions s = 0..3; in each, lane l
// supplies A[l % 16][k] and B[k][l % 16] for one k of the four, and the result lane l,
// register r holds D[row][l % 16].  With g = l / 16:
//   FP64: row = 4 r + g;   FP32: row = 4 g + r.
// The products below take k = row(s, g) (Mfma<F>::k), so that a result serves as the B
// operand of a following product as it stands; any other one-to-one choice of k only
// reorders the sum of a tile product.
typedef double v4f64 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

template <typename F>
struct Mfma;

template <>
struct Mfma<double> {
  typedef v4f64 V;
  static __device__ inline int k(int s, int g) { return 4 * s + g; }
  static __device__ inline V mul(const double* a, const double* b, V c) {
#pragma unroll
    for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], c, 0, 0, 0);
    return c;
  }
};

template <>
struct Mfma<float> {
  typedef v4f32 V;
  static __device__ inline int k(int s, int g) { return 4 * g + s; }
  static __device__ inline V mul(const float* a, const float* b, V c) {
#pragma unroll
    for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], c, 0, 0, 0);
    return c;
  }
};

__device__ inline double fsqrt(double x) { return __builtin_sqrt(x); }
__device__ inline float fsqrt(float x) { return __builtin_sqrtf(x); }

}  // namespace

// Factor precision F.  F = float is a trial on every block: after its Cholesky factor it
// takes kappa_est = (max_r L_rr / min_r L_rr)^2, a lower bound on the condition number of K
// (every pivot L_rr^2 lies between K's extreme eigenvalues); when kappa_est > kmax or a pivot
// is not positive it records the block for FP64 (prec = 1) and stops before writing what the
// FP64 run reads again (b, and A, which later holds T), else it completes in FP32 (prec = 0),
// its L and T kept as FP32 in the same buffers.  F = double with gate = 1 runs only the
// blocks the trial recorded; with gate = 0 it runs every block and records prec = 1 and its
// own kappa_est.
template <typename T, typename F>
__global__ void __launch_bounds__(kFemThreads)
    fem_factor_kernel(Topo t, FemModel f, const double* A, double* b, double rho, T* beta, double* L, double* Tw,
                      T* S, T* cd, int32_t* flags, int32_t* prec, double* kest, double kmax, int gate) {
  typedef Mfma<F> M;
  typedef typename M::V V;
  constexpr bool kTrial = sizeof(F) == sizeof(float);
  __shared__ int s_bad;
  extern __shared__ __align__(16) double fsm_raw[];
  F* fsm = reinterpret_cast<F*>(fsm_raw);
  const int i = blockIdx.x;
  if (!kTrial && gate && prec[i] == 0) return;
  const int tid = threadIdx.x;
  const int bd = blockDim.x;
  const int n = t.sub_n[i];
  const int m = f.m[i];
  const int o = n - m;
  const int nc = t.sub_nc[i];
  const int dof0 = t.sub_dof[i];
  const double* Ai = A + t.sub_A[i];
  F* Li = reinterpret_cast<F*>(L + t.sub_A[i]);
  const int32_t* perm = f.perm + dof0;
  const int pn = n > 32 ? n : 32;   // panel rows (at least 32)
  F* red = fsm;                     // 256 -- the block-diagonal tile
  F* dinv = fsm + kFemThreads;      // 16 x 16: inverse of the block-diagonal factor tile
  F* panel = dinv + kNb * kNb;      // pn x kNb: one row panel of L
  F* vec = panel + (long)pn * kNb;  // n
  if (tid == 0) s_bad = 0;

  // Eq. (23): beta = Tr(A) / Tr(J^T J), Tr(J^T J) = slot rows (each selects one DOF); in
  // FP64 for either F (the first 256 doubles of LDS, before anything else uses them)
  double* redd = fsm_raw;
  double tr = 0.0;
  for (int r = tid; r < n; r += bd) tr += Ai[(long)r * n + r];
  redd[tid] = tr;
  __syncthreads();
  for (int s = bd / 2; s > 0; s >>= 1) {
    if (tid < s) redd[tid] += redd[tid + s];
    __syncthreads();
  }
  const double be = rho > 0.0 ? rho : (nc > 0 ? redd[0] / (double)nc : 1.0);
  __syncthreads();
  if (tid == 0) beta[i] = (T)be;

  // K = P (A + beta J^T J) P^T, lower triangle: a wave per row, lanes along it (the row
  // of A is gathered through the permutation, kept in LDS)
  {
    int* pl = reinterpret_cast<int*>(vec);
    for (int r = tid; r < n; r += bd) pl[r] = perm[r];
    __syncthreads();
    const int lane = tid & 63, nw = bd >> 6;
    for (int r = tid >> 6; r < n; r += nw) {
      const int pr = pl[r];
      const double* Ar = Ai + (long)pr * n;
      F* Lr = Li + (long)r * n;
      for (int c = lane; c <= r; c += 64) {
        double v = Ar[pl[c]];
        if (c == r) v += be * (double)f.jtj[dof0 + pr];
        Lr[c] = (F)v;
      }
    }
    __syncthreads();
  }

  // Left-looking blocked Cholesky on the matrix cores, 16-column panels J: every tile row
  // I >= J first forms U_IJ = K_IJ - sum_{K<J} L_IK L_JK^T (the row panel L_J,<J staged in
  // LDS, shared by the waves), then the diagonal tile is factorised (one wave) and
  // L_IJ = U_IJ L_JJ^-T for I > J.  b (permuted) is carried as one more row, below the
  // matrix, so its factor row is y = L^-1 b (forward substitution for free).  K is read
  // once and every L tile written once (the right-looking update read and wrote the whole
  // trailing matrix per panel).
  F* yrow = vec;  // LDS, n (the permutation list kept there is no longer needed)
  for (int c = tid; c < n; c += bd) yrow[c] = (F)b[dof0 + perm[c]];
  double* yout = b + dof0;
  const int nbn = (n + kNb - 1) / kNb;  // tile rows of K; tile row nbn holds b's row alone
  const int lane = tid & 63, wv = tid >> 6, nwv = bd >> 6;
  const int g = lane >> 4, cn = lane & 15;
  auto rowp = [&](int r) -> F* { return r < n ? Li + (long)r * n : yrow; };
  auto rows_of = [&](int I) -> int { return I < nbn ? min(kNb, n - I * kNb) : 1; };
  __syncthreads();
  for (int J = 0; J < nbn; ++J) {
    const int j0 = J * kNb, jb = min(kNb, n - j0);
    // stage L_J,<J (jb x j0) in LDS, row stride j0
    for (int q = tid; q < jb * j0; q += bd) {
      const int rr = q / j0, c = q - rr * j0;
      panel[q] = Li[(long)(j0 + rr) * n + c];
    }
    __syncthreads();
    // U_IJ for the tile rows I >= J (the lane holds U_IJ[cn][row(r, g)], r = 0..3, and
    // writes it over K_IJ; the same lane reads it back for L_IJ)
    for (int I = J + wv; I <= nbn; I += nwv) {
      const int i0 = I * kNb, ib = rows_of(I);
      F* Ri = cn < ib ? rowp(i0 + cn) : nullptr;
      V acc = {0, 0, 0, 0};
      for (int K = 0; K < J; ++K) {
        const int k0 = K * kNb;
        F av[4], bv[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int kk = k0 + 4 * g + s2;
          av[s2] = cn < jb ? panel[cn * j0 + kk] : (F)0;  // L_JK[cn][k]
          bv[s2] = Ri ? Ri[kk] : (F)0;                   // L_IK[cn][k]
        }
        acc = M::mul(av, bv, acc);  // lane register r: (L_IK L_JK^T)[cn][row(r, g)]
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = M::k(r, g);
        if (Ri && c < jb) {
          const F u = Ri[j0 + c] - acc[r];
          if (I == J)
            red[cn * kNb + c] = u;
          else
            Ri[j0 + c] = u;
        }
      }
    }
    __syncthreads();
    // diagonal tile: L_JJ (in place, lower) and L_JJ^-1 (dinv), one wave
    if (wv == 0) {
      F* dg = red;
      for (int jj = 0; jj < jb; ++jj) {
        if (lane == jj) {
          F d = dg[jj * kNb + jj];
          if (!(d > (F)0) || !__builtin_isfinite(d)) {
            if (kTrial)
              s_bad = 1;
            else
              atomicOr(flags, FLAG_NOT_SPD);
            d = 1;
          }
          dg[jj * kNb + jj] = fsqrt(d);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane > jj && lane < jb) dg[lane * kNb + jj] /= dg[jj * kNb + jj];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane > jj && lane < jb)
          for (int c = jj + 1; c <= lane; ++c) dg[lane * kNb + c] -= dg[lane * kNb + jj] * dg[c * kNb + jj];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      // inverse by forward substitution, a lane per column; zero outside the lower jb x jb
      if (lane < kNb) {
        const int c = lane;
        F xcol[kNb];
#pragma unroll
        for (int r = 0; r < kNb; ++r) {
          F v = 0;
          if (r < jb && c < jb && r >= c) {
            F sacc = r == c ? (F)1 : (F)0;
            for (int p = c; p < r; ++p) sacc -= dg[r * kNb + p] * xcol[p];
            v = sacc / dg[r * kNb + r];
          }
          xcol[r] = v;
        }
#pragma unroll
        for (int r = 0; r < kNb; ++r) dinv[r * kNb + c] = xcol[r];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int q = lane; q < jb * jb; q += 64) {
        const int rr = q / jb, c = q - rr * jb;
        if (c <= rr) Li[(long)(j0 + rr) * n + j0 + c] = dg[rr * kNb + c];
      }
    }
    __syncthreads();
    // L_IJ = U_IJ L_JJ^-T for I > J (and b's row: y_J)
    for (int I = J + wv; I <= nbn; I += nwv) {
      if (I == J) continue;
      const int i0 = I * kNb, ib = rows_of(I);
      const F* Ri = cn < ib ? rowp(i0 + cn) : nullptr;
      F av[4], bv[4];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int c = M::k(s2, g);
        av[s2] = (Ri && c < jb) ? Ri[j0 + c] : (F)0;  // U_IJ[cn][c]
        bv[s2] = dinv[cn * kNb + c];                    // (L_JJ^-T)[c][cn]
      }
      V out = {0, 0, 0, 0};
      out = M::mul(av, bv, out);  // lane register r: L_IJ[row(r, g)][cn]
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = M::k(r, g);
        if (rr < ib && cn < jb) rowp(i0 + rr)[j0 + cn] = out[r];
      }
    }
    __syncthreads();
  }

  // kappa_est from the factor's diagonal (each wave reduces its share, then every thread
  // combines the waves' values in the same order)
  {
    F dmx = 0, dmn = 0;
    bool any = false;
    for (int r = tid; r < n; r += bd) {
      const F d = Li[(long)r * n + r];
      dmx = any ? (d > dmx ? d : dmx) : d;
      dmn = any ? (d < dmn ? d : dmn) : d;
      any = true;
    }
    double mx = any ? (double)dmx : 0.0, mn = any ? (double)dmn : __builtin_inf();
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      mx = fmax(mx, __shfl_xor(mx, off));
      mn = fmin(mn, __shfl_xor(mn, off));
    }
    double* kr = reinterpret_cast<double*>(dinv);  // dinv is not needed after the factor
    if (lane == 0) {
      kr[2 * wv] = mx;
      kr[2 * wv + 1] = mn;
    }
    __syncthreads();
    mx = kr[0];
    mn = kr[1];
    for (int w = 1; w < nwv; ++w) {
      mx = fmax(mx, kr[2 * w]);
      mn = fmin(mn, kr[2 * w + 1]);
    }
    const double ratio = mx / mn;
    const double kap = ratio * ratio;
    const bool to64 = kTrial && (s_bad != 0 || !(kap <= kmax));
    if (tid == 0 && (kTrial || !gate)) {
      prec[i] = kTrial ? (to64 ? 1 : 0) : 1;
      kest[i] = s_bad != 0 ? __builtin_inf() : kap;
    }
    if (to64) return;  // uniform over the workgroup
  }

  // T = L_DD^-1 (m x m lower, in this block's A storage: m^2 <= n^2), by 16-row blocks:
  // T_II = L_II^-1 (forward substitution, a lane per column), then for I > J
  // T_IJ = -T_II sum_{K=J}^{I-1} L_IK T_KJ, row block by row block, the column blocks J of
  // a row block spread over the waves, every 16 x 16 product on the matrix cores.
  F* Ti = reinterpret_cast<F*>(Tw + t.sub_A[i]);
  for (long k = tid; k < (long)m * m; k += bd) Ti[k] = 0;
  __syncthreads();
  const int nbk = (m + kNb - 1) / kNb;
  const F* Ld = Li + (long)o * n + o;  // L_DD[r][c] = Ld[r * n + c]
  for (int I = wv; I < nbk; I += nwv) {
    const int i0 = I * kNb, ib = min(kNb, m - i0);
    if (lane < ib) {
      const int c = lane;
      F xcol[kNb];
#pragma unroll
      for (int r = 0; r < kNb; ++r) {
        if (r < ib) {
          F sacc = r == c ? (F)1 : (F)0;
          for (int p = c; p < r; ++p) sacc -= Ld[(long)(i0 + r) * n + i0 + p] * xcol[p];
          xcol[r] = r < c ? (F)0 : sacc / Ld[(long)(i0 + r) * n + i0 + r];
        }
      }
#pragma unroll
      for (int r = 0; r < kNb; ++r)
        if (r < ib && r >= c) Ti[(long)(i0 + r) * m + i0 + c] = xcol[r];
    }
  }
  __syncthreads();
  for (int I = 1; I < nbk; ++I) {
    const int i0 = I * kNb, ib = min(kNb, m - i0);
    for (int J = wv; J < I; J += nwv) {
      const int j0 = J * kNb;  // J < I: a full block
      V acc = {0, 0, 0, 0};
      for (int K = J; K < I; ++K) {
        const int k0 = K * kNb;  // K < I: a full block
        F av[4], bv[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int kk = M::k(s2, g);
          av[s2] = cn < ib ? Ld[(long)(i0 + cn) * n + k0 + kk] : (F)0;
          bv[s2] = Ti[(long)(k0 + kk) * m + j0 + cn];
        }
        acc = M::mul(av, bv, acc);
      }
      // T_IJ = -T_II acc: acc (lane: rows row(r, g) of column cn) is the B operand as it stands
      F av[4], bv[4];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int kk = M::k(s2, g);
        av[s2] = (cn < ib && kk < ib) ? Ti[(long)(i0 + cn) * m + i0 + kk] : (F)0;
        bv[s2] = acc[s2];
      }
      V out = {0, 0, 0, 0};
      out = M::mul(av, bv, out);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = M::k(r, g);
        if (row < ib) Ti[(long)(i0 + row) * m + j0 + cn] = -out[r];
      }
    }
    __syncthreads();
  }

  // S = T^T T, lower 16 x 16 tiles: S_IJ = sum_{K >= I} T_KI^T T_KJ, a wave per tile.  Tile
  // layout of the iteration: entry (R, C) at ((R >> 2) * 16 + C) * 4 + (R & 3), so lane l
  // holds rows 16 I + 4 (l / 16) + k of column 16 J + l % 16 as four consecutive entries.
  T* Si = S + f.sq_off[i];
  const int ntile = nbk * (nbk + 1) / 2;
  for (int tt = wv; tt < ntile; tt += nwv) {
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= tt) ++I;
    const int J = tt - I * (I + 1) / 2;
    const int a0 = I * kNb, b0 = J * kNb;
    V acc = {0, 0, 0, 0};
    for (int K = I; K < nbk; ++K) {
      const int k0 = K * kNb, kb = min(kNb, m - k0);
      F av[4], bv[4];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int kk = M::k(s2, g);
        const bool in = kk < kb;
        av[s2] = (in && a0 + cn < m) ? Ti[(long)(k0 + kk) * m + a0 + cn] : (F)0;
        bv[s2] = (in && b0 + cn < m) ? Ti[(long)(k0 + kk) * m + b0 + cn] : (F)0;
      }
      acc = M::mul(av, bv, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = M::k(r, g);  // entry (row, cn) of the tile
      Si[(long)tt * 256 + (((row >> 2) * 16 + cn) << 2) + (row & 3)] =
          (a0 + row < m && b0 + cn < m) ? (T)acc[r] : (T)0;
    }
  }
  __syncthreads();

  // y = L^-1 P b (permuted order) replaces b in its storage (b is not read again this step)
  for (int c = tid; c < n; c += bd) yout[c] = (double)yrow[c];
  // c = K^-1 b on the constrained DOFs (the last m of the permuted order): with y = L^-1 b,
  // c_D = L_DD^-T y_D = T^T y_D
  for (int j = tid; j < m; j += bd) {
    double v = 0.0;
    for (int k = j; k < m; ++k) v += (double)Ti[(long)k * m + j] * (double)yrow[o + k];
    cd[f.dkey_off[i] + j] = (T)v;
  }
}

// v_hat = K^-1 (b + J^T w), original DOF order, from what the factorisation kept: y = L^-1 P b
// (permuted order, in b's storage) and T = L_DD^-1 (in A's storage).  With e = P J^T w, which
// is non-zero on the constrained DOFs only, L^-1 (P b + e) = y + [0; T e_D], hence
//   v_D = L_DD^-T (y_D + T e_D) = T^T (y_D + T e_D),   v_O = L_OO^-T (y_O - L_DO^T v_D).
namespace {

// The v_hat solve of one block with its factors L, T stored in precision F (sums in FP64).
template <typename T, typename F>
__device__ inline void fem_vhat_block(const Topo& t, const FemModel& f, int i, const F* Li, const F* Ti,
                                      const double* yb, const T* w, T* v_hat, double* vsm) {
  const int tid = threadIdx.x;
  const int bd = blockDim.x;
  const int n = t.sub_n[i];
  const int m = f.m[i];
  const int o = n - m;
  const int dof0 = t.sub_dof[i];
  const int32_t* perm = f.perm + dof0;
  const double* yi = yb + dof0;
  double* v = vsm;       // n, permuted order
  double* ed = v + n;    // m: e_D
  double* zd = ed + m;   // m: y_D + T e_D
  for (int k = tid; k < m; k += bd) {
    const int g = f.dkey_off[i] + k;
    double s = 0.0;
    for (int q = f.dk_off[g]; q < f.dk_off[g + 1]; ++q) {
      const int sl = f.dk_slot[q];
      s += (double)f.slot_sgn[sl] * (double)w[sl];
    }
    ed[k] = s;
  }
  __syncthreads();
  for (int k = tid; k < m; k += bd) {
    const F* Tk = Ti + (long)k * m;
    double s = yi[o + k];
    for (int p = 0; p <= k; ++p) s += (double)Tk[p] * ed[p];
    zd[k] = s;
  }
  __syncthreads();
  for (int j = tid; j < m; j += bd) {
    double s = 0.0;
    for (int k = j; k < m; ++k) s += (double)Ti[(long)k * m + j] * zd[k];
    v[o + j] = s;
  }
  __syncthreads();
  for (int c = tid; c < o; c += bd) {
    double s = yi[c];
    for (int r = 0; r < m; ++r) s -= (double)Li[(long)(o + r) * n + c] * v[o + r];
    v[c] = s;
  }
  __syncthreads();
  // L_OO^T v_O = (y_O - L_DO^T v_D): back substitution by columns, one wave
  if (tid < 64) {
    for (int c = o - 1; c >= 0; --c) {
      if (tid == 0) v[c] /= (double)Li[(long)c * n + c];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const double vc = v[c];
      for (int r = tid; r < c; r += 64) v[r] -= (double)Li[(long)c * n + r] * vc;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  for (int r = tid; r < n; r += bd) v_hat[dof0 + perm[r]] = (T)v[r];
}

}  // namespace

// prec[i] (written by the factorisation): 1 = the block's L and T are FP64, 0 = FP32.
template <typename T>
__global__ void __launch_bounds__(kFemThreads)
    fem_vhat_kernel(Topo t, FemModel f, const double* L, const double* Tw, const double* yb, const int32_t* prec,
                    const T* w, T* v_hat) {
  extern __shared__ __align__(16) double vsm[];
  const int i = blockIdx.x;
  if (prec[i])
    fem_vhat_block<T, double>(t, f, i, L + t.sub_A[i], Tw + t.sub_A[i], yb, w, v_hat, vsm);
  else
    fem_vhat_block<T, float>(t, f, i, reinterpret_cast<const float*>(L + t.sub_A[i]),
                             reinterpret_cast<const float*>(Tw + t.sub_A[i]), yb, w, v_hat, vsm);
}

// ------------------------------------------------------------------------------------
// Iteration
// ------------------------------------------------------------------------------------
namespace {

template <typename T>
__device__ inline T ld_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ inline void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Values exchanged between the workgroups of the iteration (slot y, residual partials)
// live in three buffers used in turn.  A buffer entry holds the all-ones bit pattern
// ("not written"; no arithmetic result has it) until its writer stores the value, so a
// reader polls the entry itself: no barrier, no counters.  A workgroup resets its own
// entries of the buffer of iteration l + 2 once it has seen every partial of iteration l
// (by then every reader of that buffer's previous use is done with it), and it waits for
// its stores to be acknowledged before publishing the next iteration, so a reader that has
// seen iteration l + 1 finds either the reset or the iteration-l + 2 value.
template <typename T>
__device__ inline T unwritten();
template <>
__device__ inline float unwritten<float>() { return __uint_as_float(0xffffffffu); }
template <>
__device__ inline double unwritten<double>() { return __longlong_as_double(-1ll); }
__device__ inline bool is_unwritten(float v) { return __float_as_uint(v) == 0xffffffffu; }
__device__ inline bool is_unwritten(double v) { return __double_as_longlong(v) == -1ll; }
// polls per wait before a workgroup gives up (FLAG_BARRIER)
constexpr long kMaxPolls = 1l << 24;

template <typename T>
__device__ inline T fsqrt(T x);
template <>
__device__ inline float fsqrt<float>(float x) { return __builtin_sqrtf(x); }
template <>
__device__ inline double fsqrt<double>(double x) { return __builtin_sqrt(x); }

// Fixed-order sum of two doubles per thread over the workgroup (deterministic): wave
// butterflies, then the four wave totals in order.  Every thread gets the totals.
// One DPP step on a double (both 32-bit halves moved by the same control).
template <int kCtrl, int kRowMask>
__device__ inline double dpp_double(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), kCtrl, kRowMask, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, kRowMask, 0xF, false);
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes of a wave in a fixed order (DPP only): pairs, quads, half rows and
// rows of 16, then rows 0+1 into row 1 and rows 0..3 into row 3; lane 63 holds the total.
__device__ inline double wave_sum_lane63(double v) {
  v += dpp_double<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_double<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_double<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_double<0x140, 0xF>(v);  // row_mirror
  v += dpp_double<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_double<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Sums of two values over the workgroup, identical in every thread (fixed order).
__device__ inline void block_sum2(double& v0, double& v1, double* red) {
  const int tid = threadIdx.x;
  v0 = wave_sum_lane63(v0);
  v1 = wave_sum_lane63(v1);
  if ((tid & 63) == 63) {
    red[2 * (tid >> 6)] = v0;
    red[2 * (tid >> 6) + 1] = v1;
  }
  __syncthreads();
  const int nw = blockDim.x >> 6;
  double s0 = 0.0, s1 = 0.0;
  for (int w = 0; w < nw; ++w) {
    s0 += red[2 * w];
    s1 += red[2 * w + 1];
  }
  v0 = s0;
  v1 = s1;
  __syncthreads();
}

constexpr int kMaxFemSlots = 512;  // slot rows per block (two per thread)

// Sum over the 16 lanes of each row of the wave (every lane receives its row's sum).  The
// pairing (lanes 8 apart, then 4, 2, 1 apart within the row) is the same for both forms.
__device__ inline float row_sum16(float x) {
  // DPP row rotations by 8, 4, 2, 1 lanes (row_ror:n = 0x120 + n)
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x128, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x124, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x122, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x121, 0xf, 0xf, false));
  return x;
}
__device__ inline double row_sum16(double x) {
  x += __shfl_xor(x, 8, 64);
  x += __shfl_xor(x, 4, 64);
  x += __shfl_xor(x, 2, 64);
  x += __shfl_xor(x, 1, 64);
  return x;
}

// Four consecutive entries of a 16-byte-aligned row.
template <typename T>
struct Quad;
template <>
struct Quad<float> {
  float4 v;
  __device__ void load(const float* p) { v = *reinterpret_cast<const float4*>(p); }
  __device__ void fma(float r, float* acc) const {
    acc[0] += v.x * r;
    acc[1] += v.y * r;
    acc[2] += v.z * r;
    acc[3] += v.w * r;
  }
  __device__ void store(float* p) const { *reinterpret_cast<float4*>(p) = v; }
  __device__ void zero() { v = make_float4(0.f, 0.f, 0.f, 0.f); }
  __device__ void to(float* o) const {
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};
template <>
struct Quad<double> {
  double2 a, b;
  __device__ void load(const double* p) {
    a = *reinterpret_cast<const double2*>(p);
    b = *reinterpret_cast<const double2*>(p + 2);
  }
  __device__ void fma(double r, double* acc) const {
    acc[0] += a.x * r;
    acc[1] += a.y * r;
    acc[2] += b.x * r;
    acc[3] += b.y * r;
  }
  __device__ void zero() {
    a = make_double2(0.0, 0.0);
    b = a;
  }
  __device__ void store(double* p) const {
    *reinterpret_cast<double2*>(p) = a;
    *reinterpret_cast<double2*>(p + 2) = b;
  }
  __device__ void to(double* o) const {
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
  }
};

}  // namespace

// Operator-product schedules.  A block's S is stored as its lower 16 x 16 tiles in row
// order; the four waves of the workgroup split the tiles of a block with MT tile rows
// evenly in that order.  In the fixed-size forms (template MT > 0, blocks of at most MT tile
// rows, rows beyond the block's own skipped) every tile's row and column are compile-time
// constants, so a tile costs its eight FMAs and nothing else: the lane's rd entries of
// every tile column, its column sums and the tile operands sit in registers under fixed
// names.  Resident form (R > 0): each wave keeps its first R tiles in registers and the
// rest in LDS for the whole step; R = 0 reads them from device memory every iteration.
constexpr int kResTiles = 35;
constexpr int kMtClasses[] = {8, 12, 16, 19};

template <int... Is, typename F>
__device__ __forceinline__ void static_for_seq(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(std::make_integer_sequence<int, N>{}, f);
}

__host__ __device__ constexpr int tri_row(int t) {
  int I = 0;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  return I;
}
__host__ __device__ constexpr int wave_tile_beg(int mt, int w) { return (mt * (mt + 1) / 2) * w / 4; }
__host__ __device__ constexpr int wave_tile_count(int mt, int w) {
  return wave_tile_beg(mt, w + 1) - wave_tile_beg(mt, w);
}
// LDS tiles of the resident form kept by the waves before wave w
__host__ __device__ constexpr int lds_tiles_before(int mt, int R, int w) {
  int n = 0;
  for (int v = 0; v < w; ++v) n += wave_tile_count(mt, v) > R ? wave_tile_count(mt, v) - R : 0;
  return n;
}

// Tile arithmetic as chains of explicit fused multiply-adds (no separate multiplies or
// adds the compiler could fuse differently in different instantiations), so every form of
// the product rounds identically.
__device__ inline float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T>
__device__ inline T dot4_acc(const T* e, const T* r, T acc) {
  return fmat(e[3], r[3], fmat(e[2], r[2], fmat(e[1], r[1], fmat(e[0], r[0], acc))));
}

template <typename T>
struct MatvecArgs {
  const T* rd;   // LDS, 16 mt entries (zero beyond m)
  T* ow;         // LDS, this wave's 16 mt partial products
  const T* sg;   // block's tiles in device memory, + 4 lane
  const T* sl;   // this wave's LDS tiles, + 4 lane
  int mt, g4, cc;
};

// Loads wave W's tiles before the iteration (resident form).
template <typename T, int MT, int R, int W>
__device__ __forceinline__ void load_tiles(Quad<T>* sreg, const MatvecArgs<T>& c) {
  constexpr int beg = wave_tile_beg(MT, W), cnt = wave_tile_count(MT, W), RR = R < cnt ? R : cnt;
  static_for<cnt>([&](auto rc) {
    constexpr int r = decltype(rc)::value, t = beg + r, I = tri_row(t);
    if constexpr (r < RR) {
      if (I < c.mt) sreg[r].load(c.sg + (long)t * 256); else sreg[r].zero();
    } else {
      // rows beyond the block's own are stored as zero tiles
      Quad<T> v;
      if (I < c.mt) v.load(c.sg + (long)t * 256); else v.zero();
      v.store(const_cast<T*>(c.sl) + (r - RR) * 256);
    }
  });
}

// One wave's share of vd += S rd (fixed-size form): tile (I, J) adds T rd_J to rows I and,
// below the diagonal, T^T rd_I to rows J.  Row sums are reduced over the 16 lanes of a
// row when the tile row (or the wave's range) ends; column sums stay per lane and are
// added at the end, one row group after another.
template <typename T, int MT, int R, int W>
__device__ __forceinline__ void matvec_fixed(const Quad<T>* sreg, const MatvecArgs<T>& c) {
  constexpr int beg = wave_tile_beg(MT, W), cnt = wave_tile_count(MT, W), RR = R < cnt ? R : cnt;
  constexpr int end = beg + cnt;
  T rdl[MT], cacc[MT];
  static_for<MT>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    rdl[j] = j < c.mt ? c.rd[16 * j + c.cc] : (T)0;
    cacc[j] = (T)0;
  });
  T racc[4] = {(T)0, (T)0, (T)0, (T)0}, ri[4] = {(T)0, (T)0, (T)0, (T)0}, rin[4] = {(T)0, (T)0, (T)0, (T)0};
  if constexpr (cnt > 0) {
    constexpr int I0 = tri_row(beg);
    if (I0 < c.mt)
#pragma unroll
      for (int k = 0; k < 4; ++k) ri[k] = c.rd[16 * I0 + 4 * c.g4 + k];
  }
  // tiles not in registers (LDS, or device memory when R = 0) are read PD tiles ahead into
  // a ring of registers; scheduling barriers at the tile boundaries keep the compiler from
  // hoisting further loads (which would cost registers the resident tiles need)
  constexpr int PD = R > 0 ? 2 : 8;
  Quad<T> pf[PD];
  // the device-memory tile addresses are formed here, in the iteration, from an opaque
  // copy of the base (otherwise they are hoisted out of the iteration loop and held in
  // registers, one pointer per tile)
  const T* sgp = c.sg;
  asm volatile("" : "+v"(sgp));
  auto fetch = [&](auto qc) {
    constexpr int q = decltype(qc)::value, tq = beg + q;
    if constexpr (q >= RR && q < cnt) {
      if constexpr (R > 0)
        pf[q % PD].load(c.sl + (q - RR) * 256);  // zero tiles beyond the block's rows
      else if (tri_row(tq) < c.mt)
        pf[q % PD].load(sgp + (long)tq * 256);
    }
  };
  // tile q is fetched at position q - PD; the first PD positions are fetched here
  static_for<PD>([&](auto qc) { fetch(qc); });
  static_for<cnt>([&](auto rc) {
    constexpr int r = decltype(rc)::value, t = beg + r, I = tri_row(t), J = t - I * (I + 1) / 2;
    __builtin_amdgcn_sched_barrier(0);
    // tiles of rows beyond the block's own are skipped (a branch per tile keeps each tile
    // its own scheduling region, which keeps the register allocation of the resident form
    // within its budget)
    if (I < c.mt) {
      if constexpr (J == 0 || r == 0) {
        // next tile row's rd entries, read one row ahead (zero beyond the block)
        if (I + 1 < c.mt) {
#pragma unroll
          for (int k = 0; k < 4; ++k) rin[k] = c.rd[16 * (I + 1) + 4 * c.g4 + k];
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) rin[k] = (T)0;
        }
      }
      Quad<T> v;
      if constexpr (r < RR)
        v = sreg[r];
      else
        v = pf[r % PD];
      fetch(std::integral_constant<int, r + PD>{});
      T e4[4];
      v.to(e4);
#pragma unroll
      for (int k = 0; k < 4; ++k) racc[k] = fmat(e4[k], rdl[J], racc[k]);
      if constexpr (J < I) cacc[J] = dot4_acc(e4, ri, cacc[J]);
      if constexpr (J == I || t == end - 1) {
        // a wave's tiles of one row are consecutive, so each of its rows is flushed once,
        // into entries that hold zero until then: a plain store
        if (I < c.mt) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const T q = row_sum16(racc[k]);
            if (c.cc == 0) c.ow[16 * I + 4 * c.g4 + k] = q;
          }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) racc[k] = (T)0;
        if constexpr (J == I) {
#pragma unroll
          for (int k = 0; k < 4; ++k) ri[k] = rin[k];
        }
      }
    } else {
      fetch(std::integral_constant<int, r + PD>{});
    }
  });
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (cnt > 0) {
    // column sums: reduce over the four row groups of the lane's column (all columns'
    // exchanges issued together), then one add per column entry
    constexpr int ncol = tri_row(end - 1);  // columns J < the wave's last tile row
    static_for<ncol>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      cacc[j] += __shfl_xor(cacc[j], 16, 64);
    });
    static_for<ncol>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      cacc[j] += __shfl_xor(cacc[j], 32, 64);
    });
    if (c.g4 == 0) {
      static_for<ncol>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j < c.mt) c.ow[16 * j + c.cc] += cacc[j];
      });
    }
  }
}

// MT > 0: fixed-size operator product (blocks of at most MT tile rows); R > 0 resident
// (two workgroups per CU, so at most 256 VGPRs per lane), R = 0 read every iteration.
// MT = 0 (R = 0): any block size; tile coordinates at run time, column sums reduced over
// the lane groups and added to LDS per tile.
template <typename T, int R, int MT>
__global__ void __launch_bounds__(kFemThreads, MT > 0 ? 2 : 1) fem_loop_kernel(FemLoopArgs<T> a) {
  extern __shared__ __align__(16) double lsm[];
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int bd = blockDim.x;
  const Topo& t = a.t;
  const int n_slot = t.sc_slot[t.n_scene];
  const int s0 = t.sub_slot[i];
  const int nc = t.sub_nc[i];
  const int m = a.f.m[i];
  const int mt = (m + 15) >> 4;  // 16 x 16 tiles of S per side
  const int scene = [&] {
    int lo = 0, hi = t.n_scene - 1;  // sc_sub[scene] <= i < sc_sub[scene + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (t.sc_sub[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
  }();
  // LDS: reductions, scene flags, per-slot state, the constrained-DOF vectors, matvec
  // partials, per-key slot lists and the static data of this block's interface groups
  double* red = lsm;                                        // 16
  T* y = reinterpret_cast<T*>(lsm + 16);                    // nc
  T* u = y + a.max_nc;
  T* w = u + a.max_nc;
  T* z = w + a.max_nc;
  T* lam = z + a.max_nc;
  T* rd = lam + a.max_nc;                                   // 16 mt (zero beyond m)
  T* vd = rd + a.max_mt16;                                  // m
  T* outw = vd + a.max_mt16;                                // per wave 16 mt partial products
  T* cdl = outw + 4 * a.max_mt16;                           // m: c = K^-1 b on the constrained DOFs
  T* gT = cdl + a.max_mt16;                                 // 7 per group: ib0, ib1, iws, mu, e0..e2
  int* gI = reinterpret_cast<int*>(gT + 7 * a.max_ng);      // 4 per group: q0, ga, gb, kind | dim << 4
  int* kl = gI + 4 * a.max_ng;                              // m + 1 key offsets, then nc slots
  const T be = a.beta[i];
  const T* Si = a.S + a.f.sq_off[i];
  const int dk0 = a.f.dkey_off[i];

  // per-step static data
  const int kbase = a.f.dk_off[dk0];
  for (int k = tid; k <= m; k += bd) kl[k] = a.f.dk_off[dk0 + k] - kbase;
  // slot (relative to the block) << 1 | (sign < 0) of every slot row selecting each DOF
  for (int q = tid; q < nc; q += bd) {
    const int ql = a.f.dk_slot[kbase + q] - s0;
    kl[m + 1 + q] = (ql << 1) | (a.f.slot_sgn[s0 + ql] < 0 ? 1 : 0);
  }
  for (int k = tid; k < m; k += bd) cdl[k] = a.cd[dk0 + k];
  // own slots: two per thread at most, sign and key in registers
  T sg[2] = {(T)0, (T)0};
  int kd[2] = {0, 0};
  for (int r = 0; r < 2; ++r) {
    const int q = tid + r * bd;
    if (q < nc) {
      sg[r] = (T)a.f.slot_sgn[s0 + q];
      kd[r] = a.f.slot_dk[s0 + q];
    }
  }
  // interface groups that touch this block: the first slot row of each
  __shared__ int ngroup;
  if (tid == 0) ngroup = 0;
  __syncthreads();
  for (int q = tid; q < nc; q += bd) {
    const int sl = s0 + q;
    if ((t.slot_mk[sl] & 7) != 0) continue;
    const int g = atomicAdd(&ngroup, 1);
    const int j = t.slot_if[sl];
    const bool two = t.if_nsub[j] == 2;
    const T ib0 = (T)1 / a.beta[t.if_sub0[j]];
    const T ib1 = two ? (T)1 / a.beta[t.if_sub1[j]] : (T)0;
    gI[4 * g + 0] = q;
    gI[4 * g + 1] = t.if_slot0[j];
    gI[4 * g + 2] = two ? t.if_slot1[j] : -1;
    gI[4 * g + 3] = t.if_kind[j] | (t.if_dim[j] << 4);
    gT[7 * g + 0] = ib0;
    gT[7 * g + 1] = ib1;
    gT[7 * g + 2] = (T)1 / (ib0 + ib1);
    gT[7 * g + 3] = a.mu[j];
    for (int k = 0; k < 3; ++k) gT[7 * g + 4 + k] = k < t.if_dim[j] ? a.e[t.if_row[j] + k] : (T)0;
  }
  // initial values: y^0 := beta z^0 + u^0 (relation after every z/u-update), w = beta z - u
  for (int q = tid; q < nc; q += bd) {
    const int sl = s0 + q;
    const T z0 = a.z_in ? a.z_in[sl] : (T)0;
    const T u0 = a.u_in ? a.u_in[sl] : (T)0;
    z[q] = z0;
    u[q] = u0;
    w[q] = be * z0 - u0;
    y[q] = be * z0 + u0;
    lam[q] = -u0;
  }
  __syncthreads();
  const int ng = ngroup;
  for (int k = m + tid; k < 16 * mt; k += bd) rd[k] = (T)0;
  // operator product: the lower tiles in row order, split evenly over the four waves
  const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g4 = lane >> 4, cc = lane & 15;
  T* ow = outw + wv * 16 * mt;
  // resident operator: registers, then LDS (16-byte aligned after the other arrays)
  Quad<T> sreg[(MT > 0 && R > 0) ? R : 1];
  MatvecArgs<T> mv;
  mv.rd = rd;
  mv.ow = ow;
  mv.sg = Si + 4 * lane;
  mv.mt = mt;
  mv.g4 = g4;
  mv.cc = cc;
  {
    T* slds = reinterpret_cast<T*>(
        (reinterpret_cast<uintptr_t>(kl + a.max_m + 1 + a.max_nc) + 15) & ~static_cast<uintptr_t>(15));
    mv.sl = slds + (long)lds_tiles_before(MT, R, wv) * 256 + 4 * lane;
  }
  if constexpr (MT > 0 && R > 0) {
    switch (wv) {
      case 0: load_tiles<T, MT, R, 0>(sreg, mv); break;
      case 1: load_tiles<T, MT, R, 1>(sreg, mv); break;
      case 2: load_tiles<T, MT, R, 2>(sreg, mv); break;
      default: load_tiles<T, MT, R, 3>(sreg, mv); break;
    }
  }
  // run-time schedule (MT = 0): this wave's first tile
  const int n_tile = mt * (mt + 1) / 2;
  const int t_beg = (n_tile * wv) / 4, t_end = (n_tile * (wv + 1)) / 4;
  int I0 = 0;
  while ((I0 + 1) * (I0 + 2) / 2 <= t_beg) ++I0;
  const int J0 = t_beg - I0 * (I0 + 1) / 2;

  const int sub0 = t.sc_sub[scene], sub1 = t.sc_sub[scene + 1];
  int it = 0, conv = 0;
  double th_s = 0.0, rt_s = 0.0;
  for (int l = 0; l < a.max_iters; ++l) {
    T* ybuf = a.ybuf + (long)(l % 3) * n_slot;
    double* part = a.part + (long)(l % 3) * 2 * kPartCopies * t.n_sub;
    {
      // x-update (Eq. 15): rd = J_D^T w; vd = cd + S rd; x = J_D vd; y = beta x + u (Eq. 18)
      for (int k = tid; k < m; k += bd) {
        T s = (T)0;
        for (int q = kl[k]; q < kl[k + 1]; ++q) {
          const int e = kl[m + 1 + q];
          s += (e & 1) ? -w[e >> 1] : w[e >> 1];
        }
        rd[k] = s;
      }
      __syncthreads();
      // vd = cd + S rd with S symmetric and only its lower tiles stored: a tile (I, J)
      // adds T rd_J to rows I and, below the diagonal, T^T rd_I to rows J.  Row sums
      // are kept per lane until the tile row ends, column sums are reduced per tile.
      for (int k = tid; k < 4 * 16 * mt; k += bd) outw[k] = (T)0;
      __syncthreads();
      if constexpr (MT > 0) {
        switch (wv) {
          case 0: matvec_fixed<T, MT, R, 0>(sreg, mv); break;
          case 1: matvec_fixed<T, MT, R, 1>(sreg, mv); break;
          case 2: matvec_fixed<T, MT, R, 2>(sreg, mv); break;
          default: matvec_fixed<T, MT, R, 3>(sreg, mv); break;
        }
      } else {
        int I = I0, J = J0;
        T racc[4] = {(T)0, (T)0, (T)0, (T)0};
        bool pending = false;
        auto row_flush = [&]() {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const T q = row_sum16(racc[k]);
            if (cc == 0) ow[16 * I + 4 * g4 + k] += q;
            racc[k] = (T)0;
          }
        };
        const T* base = Si + 4 * lane;
        for (int t = t_beg; t < t_end; t += 8) {
          Quad<T> v[8];
#pragma unroll
          for (int r = 0; r < 8; ++r)
            if (t + r < t_end) v[r].load(base + (long)(t + r) * 256);
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            if (t + r >= t_end) break;
            T e4[4];
            v[r].to(e4);
            const T rj = rd[16 * J + cc];
#pragma unroll
            for (int k = 0; k < 4; ++k) racc[k] = fmat(e4[k], rj, racc[k]);
            pending = true;
            if (J < I) {
              T cp = dot4_acc(e4, rd + 16 * I + 4 * g4, (T)0);
              cp += __shfl_xor(cp, 16, 64);
              cp += __shfl_xor(cp, 32, 64);
              if (g4 == 0) ow[16 * J + cc] += cp;
              ++J;
            } else {
              row_flush();
              pending = false;
              ++I;
              J = 0;
            }
          }
        }
        if (pending) row_flush();
      }
      __syncthreads();
      for (int k = tid; k < m; k += bd) {
        T s = (T)0;
        for (int q = 0; q < 4; ++q) s += outw[q * 16 * mt + k];
        vd[k] = cdl[k] + s;
      }
      __syncthreads();
      double pth = 0.0, pyy = 0.0;
      // this workgroup's resets of two iterations ago are performed before it publishes
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int q = tid + r * bd;
        if (q < nc) {
          const T x = sg[r] * vd[kd[r]];
          const T yn = be * x + u[q];
          const T df = yn - y[q];
          pth += (double)df * (double)df;
          pyy += (double)yn * (double)yn;
          y[q] = yn;
          st_agent(ybuf + s0 + q, yn);
        }
      }
      block_sum2(pth, pyy, red);
      // every copy of the partials gets them (readers spread over the copies)
      if (tid < 2 * kPartCopies)
        st_agent(part + (long)(tid >> 1) * 2 * t.n_sub + 2 * i + (tid & 1), (tid & 1) ? pyy : pth);
    }
    // the z-update's inputs (this thread's first interface group), read now so that their
    // latency overlaps the residual's reads; entries not yet written are read again later
    T pya[3] = {(T)0, (T)0, (T)0}, pyb[3] = {(T)0, (T)0, (T)0};
    if (tid < ng) {
      const int ga = gI[4 * tid + 1], gb = gI[4 * tid + 2], dim = gI[4 * tid + 3] >> 4;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k < dim) pya[k] = ld_agent(ybuf + ga + k);
        if (k < dim && gb >= 0) pyb[k] = ld_agent(ybuf + gb + k);
      }
    }
    // residual of Eq. (22) over this block's scene: every partial of the iteration, summed
    // in the same order by every workgroup of the scene (so all take the same decision)
    double p0 = 0.0, p1 = 0.0;
    bool lost = false;
    const double* mine = part + (long)(i % kPartCopies) * 2 * t.n_sub;
    for (long polls = 0;; ++polls) {
      double s0p = 0.0, s1p = 0.0;
      bool ready = true;
      for (int q = sub0 + tid; q < sub1; q += bd) {
        const double v0 = ld_agent(mine + 2 * q), v1 = ld_agent(mine + 2 * q + 1);
        ready = ready && !is_unwritten(v0) && !is_unwritten(v1);
        s0p += v0;
        s1p += v1;
      }
      if (__syncthreads_and(ready)) {
        p0 = s0p;
        p1 = s1p;
        break;
      }
      if (polls > kMaxPolls) {
        lost = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lost) {
      if (tid == 0) atomicOr(a.flags, FLAG_BARRIER);
      it = l + 1;
      break;
    }
    block_sum2(p0, p1, red);
    it = l + 1;
    {
      const double tol2 = a.tol * a.tol;
      const bool bad = !__builtin_isfinite(p0) || !__builtin_isfinite(p1);
      const bool cv = !bad && p0 <= tol2 * (p1 > 1e-24 ? p1 : 1e-24);
      if (cv || bad || l + 1 == a.max_iters) {
        if (bad && i == sub0 && tid == 0) atomicOr(a.flags, FLAG_NONFINITE);
        conv = cv;
        th_s = p0;
        rt_s = __builtin_sqrt(p0) / __builtin_sqrt(p1 > 1e-24 ? p1 : 1e-24);
        break;
      }
    }
    // every reader of the buffer of iteration l - 1 (= l + 2) is done with it: reset ours
    {
      T* yn2 = a.ybuf + (long)((l + 2) % 3) * n_slot;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int q = tid + r * bd;
        if (q < nc) st_agent(yn2 + s0 + q, unwritten<T>());
      }
      if (tid < 2 * kPartCopies) {
        double* pn2 = a.part + (long)((l + 2) % 3) * 2 * kPartCopies * t.n_sub;
        st_agent(pn2 + (long)(tid >> 1) * 2 * t.n_sub + 2 * i + (tid & 1), unwritten<double>());
      }
    }
    // z-update (Eq. 16-21) and dual update (Eq. 14) of the interfaces touching this block
    for (int g = tid; g < ng; g += bd) {
      const int q0 = gI[4 * g + 0], ga = gI[4 * g + 1], gb = gI[4 * g + 2], kdim = gI[4 * g + 3];
      const int kind = kdim & 15, dim = kdim >> 4;
      const T ib0 = gT[7 * g + 0], ib1 = gT[7 * g + 1], iws = gT[7 * g + 2], mu = gT[7 * g + 3];
      T p[3], lv[3];
      for (int k = 0; k < 3; ++k) {
        T ya = (T)0, yb = (T)0;
        if (k < dim) {
          ya = g == tid ? pya[k] : ld_agent(ybuf + ga + k);
          // once one wait of this thread has expired the iteration is abandoned: no
          // further entry is polled, so a lost exchange costs one poll budget, not one per entry
          for (long polls = 0; !lost && is_unwritten(ya) && polls <= kMaxPolls; ++polls) {
            __builtin_amdgcn_s_sleep(1);
            ya = ld_agent(ybuf + ga + k);
          }
          lost = lost || is_unwritten(ya);
          if (gb >= 0) {
            yb = g == tid ? pyb[k] : ld_agent(ybuf + gb + k);
            for (long polls = 0; !lost && is_unwritten(yb) && polls <= kMaxPolls; ++polls) {
              __builtin_amdgcn_s_sleep(1);
              yb = ld_agent(ybuf + gb + k);
            }
            lost = lost || is_unwritten(yb);
          }
        }
        p[k] = -(gT[7 * g + 4 + k] + ya * ib0 + yb * ib1) * iws;
      }
      if (kind == KIND_CONTACT && a.contact_model == 1) {
        cone_project<T>(p, mu, lv);
      } else if (kind == KIND_CONTACT) {
        const T ln = p[0] > (T)0 ? p[0] : (T)0;
        const T tn = fsqrt<T>(p[1] * p[1] + p[2] * p[2]);
        const T cap = mu * ln;
        lv[0] = ln;
        if (tn <= cap) {
          lv[1] = p[1];
          lv[2] = p[2];
        } else {
          const T fct = cap / tn;
          lv[1] = fct * p[1];
          lv[2] = fct * p[2];
        }
      } else if (kind == KIND_HARD_INEQ) {
        for (int k = 0; k < 3; ++k) lv[k] = p[k] > (T)0 ? p[k] : (T)0;
      } else {
        for (int k = 0; k < 3; ++k) lv[k] = p[k];
      }
      for (int k = 0; k < dim; ++k) {
        const int qq = q0 + k;
        u[qq] = -lv[k];
        z[qq] = (y[qq] + lv[k]) / be;
        w[qq] = y[qq] + (T)2 * lv[k];
        lam[qq] = lv[k];
      }
    }
    if (__syncthreads_or(lost)) {
      if (tid == 0) atomicOr(a.flags, FLAG_BARRIER);
      break;
    }
  }
  __syncthreads();
  // outputs of this block: final (z, u), the w of the last x-update, lambda rows of the
  // interfaces whose member 0 is this block
  for (int q = tid; q < nc; q += bd) {
    const int sl = s0 + q;
    if (a.z_out) a.z_out[sl] = z[q];
    if (a.u_out) a.u_out[sl] = u[q];
    a.w_out[sl] = w[q];
    const int j = t.slot_if[sl];
    const int mk = t.slot_mk[sl];
    if (a.lambda && (mk >> 3) == 0) a.lambda[t.if_row[j] + (mk & 7)] = lam[q];
  }
  if (tid == 0 && i == t.sc_sub[scene]) {
    a.st_iters[scene] = it;
    a.st_conv[scene] = conv;
    a.st_theta[scene] = th_s;
    a.st_rtheta[scene] = rt_s;
    a.st_total[scene] += it;
    if (!conv) a.st_unconv[scene] += 1;
  }
}

template <typename T>
__global__ void fem_advance_kernel(int64_t n_dof, const T* v_hat, T dt, T* pos, T* vel) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_dof) return;
  const T vh = v_hat[k];
  pos[k] += dt * vh;
  vel[k] = (T)2 * vh - vel[k];
}

template <typename T>
__global__ void fem_export_kernel(Topo t, FemModel f, const double* A, const double* b, T* Ao, T* bo, T* Jo) {
  const int i = blockIdx.x;
  const int n = t.sub_n[i];
  const long nn = (long)n * n;
  for (long k = threadIdx.x; k < nn; k += blockDim.x) Ao[t.sub_A[i] + k] = (T)A[t.sub_A[i] + k];
  for (int r = threadIdx.x; r < n; r += blockDim.x) bo[t.sub_dof[i] + r] = (T)b[t.sub_dof[i] + r];
  const int nc = t.sub_nc[i];
  T* Ji = Jo + t.sub_J[i];
  for (long k = threadIdx.x; k < (long)nc * n; k += blockDim.x) Ji[k] = (T)0;
  __syncthreads();
  for (int q = threadIdx.x; q < nc; q += blockDim.x) {
    const int sl = t.sub_slot[i] + q;
    Ji[(long)q * n + f.slot_dof[sl]] = (T)f.slot_sgn[sl];
  }
}

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------
template <typename T>
hipError_t launch_fem_assemble(const Topo& t, const FemModel& f, const T* pos, const T* vel, double dt, double* A,
                               double* b, double* scr, int32_t* flags, hipStream_t s) {
  if (t.n_sub == 0) return hipSuccess;
  hipLaunchKernelGGL(fem_assemble_kernel<T>, dim3(t.n_sub), dim3(kFemThreads), 0, s, t, f, pos, vel, dt, A, b, scr,
                     flags);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_rows(const Topo& t, const FemModel& f, const T* pos, double dt, T* e, hipStream_t s) {
  if (t.n_if == 0) return hipSuccess;
  hipLaunchKernelGGL(fem_rows_kernel<T>, dim3((t.n_if + 255) / 256), dim3(256), 0, s, t, f, pos, dt, e);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_factor(const Topo& t, const FemModel& f, const double* A, double* b, double rho, T* beta,
                             double* L, double* tinv, T* S, T* cd, int32_t* flags, int32_t* prec, double* kest,
                             double kmax, int max_n, int max_m, hipStream_t s) {
  if (t.n_sub == 0) return hipSuccess;
  (void)max_m;
  const size_t pn = max_n > 32 ? (size_t)max_n : 32;
  const size_t words = (size_t)kFemThreads + kNb * kNb + pn * kNb + (size_t)max_n;
  auto go = [&](auto kern, size_t lds, double km, int gate) -> hipError_t {
    if (lds > 64 * 1024) {
      const hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (ea != hipSuccess) return ea;
    }
    hipLaunchKernelGGL(kern, dim3(t.n_sub), dim3(kFemThreads), lds, s, t, f, A, b, rho, beta, L, tinv, S, cd, flags,
                       prec, kest, km, gate);
    return hipGetLastError();
  };
  if constexpr (std::is_same<T, float>::value) {
    if (kmax > 0.0) {
      // FP32 trial on every block, then FP64 on the blocks it recorded
      const hipError_t e = go(&fem_factor_kernel<T, float>, sizeof(float) * words, kmax, 0);
      if (e != hipSuccess) return e;
      return go(&fem_factor_kernel<T, double>, sizeof(double) * words, 0.0, 1);
    }
  }
  return go(&fem_factor_kernel<T, double>, sizeof(double) * words, 0.0, 0);
}

// Marks every entry of the exchange buffers "not written" (all-ones bits).
template <typename T>
__global__ void fem_unwritten_kernel(T* y, long n_y, double* part, long n_part) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_y) y[k] = unwritten<T>();
  if (k < n_part) part[k] = unwritten<double>();
}

template <typename T, int R, int MT>
static hipError_t resident_fem_loop(const FemLoopArgs<T>& a, size_t lds, int cus, bool& fits, hipStream_t s) {
  int per_cu = 0;
  const void* fn = reinterpret_cast<const void*>(&fem_loop_kernel<T, R, MT>);
  if (lds > 64 * 1024) {
    const hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) {
      (void)hipGetLastError();
      fits = false;
      return hipSuccess;
    }
  }
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kFemThreads, lds);
  if (e != hipSuccess) return e;
  fits = (long)per_cu * cus >= a.t.n_sub;
  if (!fits) return hipSuccess;
  // An ordinary dispatch: the grid fits the device at this occupancy, so every workgroup is
  // resident once the work queued before it on the stream has drained.  The kernel needs
  // nothing else of a cooperative launch (no grid-wide sync object; workgroups exchange
  // through polled buffers whose waits are bounded and report FLAG_BARRIER on expiry), and
  // a cooperative launch would put the dispatch on the runtime's separate cooperative queue.
  hipLaunchKernelGGL((fem_loop_kernel<T, R, MT>), dim3(a.t.n_sub), dim3(kFemThreads), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_loop(const FemLoopArgs<T>& a, int* form, hipStream_t s) {
  *form = 0;
  if (a.t.n_sub == 0) return hipSuccess;
  if (a.max_nc > kMaxFemSlots) return hipErrorInvalidValue;
  {
    const long n_y = 3 * (long)a.n_slot, n_part = 6 * (long)kPartCopies * a.t.n_sub;
    const long n = n_y > n_part ? n_y : n_part;
    hipLaunchKernelGGL(fem_unwritten_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a.ybuf, n_y,
                       a.part, n_part);
    const hipError_t ze = hipGetLastError();
    if (ze != hipSuccess) return ze;
  }
  const size_t lds = sizeof(double) * 16 +
                     sizeof(T) * (5 * (size_t)a.max_nc + 7 * (size_t)a.max_mt16 + 7 * (size_t)a.max_ng) +
                     sizeof(int) * (4 * (size_t)a.max_ng + (size_t)a.max_m + 1 + (size_t)a.max_nc);
  int dev = 0, cus = 0, lds_max = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  const int mt = a.max_mt16 / 16;
  bool fits = false;
  if constexpr (std::is_same<T, float>::value) {
    // smallest fixed-size class that holds every block
    int MT = 0;
    for (int c : kMtClasses)
      if (mt <= c) {
        MT = c;
        break;
      }
    if (MT > 0) {
      auto run = [&](auto mtc) -> hipError_t {
        constexpr int M = decltype(mtc)::value;
        if (a.resident) {
          const size_t lds_r = lds + 16 + (size_t)lds_tiles_before(M, kResTiles, 4) * 256 * sizeof(T);
          if (lds_r <= (size_t)lds_max) {
            const hipError_t er = resident_fem_loop<T, kResTiles, M>(a, lds_r, cus, fits, s);
            if (fits) *form = kResTiles;
            if (er != hipSuccess || fits) return er;
          }
        }
        return resident_fem_loop<T, 0, M>(a, lds, cus, fits, s);
      };
      switch (MT) {
        case 8: e = run(std::integral_constant<int, 8>{}); break;
        case 12: e = run(std::integral_constant<int, 12>{}); break;
        case 16: e = run(std::integral_constant<int, 16>{}); break;
        default: e = run(std::integral_constant<int, 19>{}); break;
      }
      if (e != hipSuccess || fits) return e;
    }
  }
  e = resident_fem_loop<T, 0, 0>(a, lds, cus, fits, s);
  if (e != hipSuccess) return e;
  return fits ? hipSuccess : hipErrorCooperativeLaunchTooLarge;
}

template <typename T>
hipError_t launch_fem_vhat(const Topo& t, const FemModel& f, const double* L, const double* Tw, const double* y,
                           const int32_t* prec, const T* w, T* v_hat, int max_n, hipStream_t s) {
  if (t.n_sub == 0) return hipSuccess;
  const size_t lds = sizeof(double) * 3 * (size_t)max_n;
  hipLaunchKernelGGL(fem_vhat_kernel<T>, dim3(t.n_sub), dim3(kFemThreads), lds, s, t, f, L, Tw, y, prec, w, v_hat);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_advance(int64_t n_dof, const T* v_hat, T dt, T* pos, T* vel, hipStream_t s) {
  if (n_dof == 0) return hipSuccess;
  hipLaunchKernelGGL(fem_advance_kernel<T>, dim3((unsigned)((n_dof + 255) / 256)), dim3(256), 0, s, n_dof, v_hat, dt,
                     pos, vel);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fem_export(const Topo& t, const FemModel& f, const double* A, const double* b, T* Ao, T* bo, T* Jo,
                             hipStream_t s) {
  if (t.n_sub == 0) return hipSuccess;
  hipLaunchKernelGGL(fem_export_kernel<T>, dim3(t.n_sub), dim3(kFemThreads), 0, s, t, f, A, b, Ao, bo, Jo);
  return hipGetLastError();
}

#define SUBADMM_FEM_INST(T)                                                                                          \
  template hipError_t launch_fem_assemble<T>(const Topo&, const FemModel&, const T*, const T*, double, double*,    \
                                             double*, double*, int32_t*, hipStream_t);                              \
  template hipError_t launch_fem_rows<T>(const Topo&, const FemModel&, const T*, double, T*, hipStream_t);          \
  template hipError_t launch_fem_factor<T>(const Topo&, const FemModel&, const double*, double*, double, T*,       \
                                           double*, double*, T*, T*, int32_t*, int32_t*, double*, double, int, int, \
                                           hipStream_t);                                                            \
  template hipError_t launch_fem_loop<T>(const FemLoopArgs<T>&, int*, hipStream_t);                                  \
  template hipError_t launch_fem_vhat<T>(const Topo&, const FemModel&, const double*, const double*, const double*, \
                                         const int32_t*, const T*, T*, int, hipStream_t);                           \
  template hipError_t launch_fem_advance<T>(int64_t, const T*, T, T*, T*, hipStream_t);                             \
  template hipError_t launch_fem_export<T>(const Topo&, const FemModel&, const double*, const double*, T*, T*, T*,  \
                                           hipStream_t);
SUBADMM_FEM_INST(float)
SUBADMM_FEM_INST(double)
#undef SUBADMM_FEM_INST

}  // namespace subadmm
